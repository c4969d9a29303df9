// sns_qr_solve_noalloc: the QR solve of sns_qr_solve with its workspace in a
// static device array instead of caller memory, for callers that cannot
// allocate (code under graph capture, tight serving loops).  The array lives
// in the library's code object: every device the library runs on holds its
// own copy until the process ends.  Host code never passes the array's name
// to a kernel (on the host that name is only a stand-in): the device address
// is looked up once per device with hipGetSymbolAddress and kept.
#include <mutex>

#include "common.hpp"
#include "kernels.hpp"
#include "solve.hpp"

namespace sns {
namespace {

constexpr size_t kScratchBytes = 64ull << 20;  // 64 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up on the first call
// on each device, with that device current).
sns_status scratch_address(void** out) {
  int dev = 0;
  SNS_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return SNS_ERR_HIP;
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    SNS_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return SNS_ERR_HIP;
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return SNS_OK;
}

}  // namespace
}  // namespace sns

extern "C" sns_status sns_qr_solve_noalloc(int64_t d, int64_t n, sns_dtype dtype, const void* SA,
                                           int64_t ld_sa, const void* Sb, double* x0, double* R,
                                           sns_info* info, void* stream) {
  // the same argument rules as sns_qr_solve, checked before anything else
  if (!SA || !Sb || !x0) return SNS_ERR_INVALID_ARG;
  if (dtype != SNS_F32 && dtype != SNS_F64) return SNS_ERR_DTYPE;
  size_t need = 0;
  sns_status s = sns_qr_solve_workspace_size(d, n, &need);
  if (s != SNS_OK) return s;
  if (ld_sa < n) return SNS_ERR_SHAPE;
  if (need > sns::kScratchBytes) return SNS_ERR_OUT_OF_MEMORY;
  void* ws = nullptr;
  if ((s = sns::scratch_address(&ws)) != SNS_OK) return s;
  // every buffer the QR solve takes from the workspace is written by its
  // kernels before it is read (the flags by the first load tile), so the
  // contents a previous call left behind do not matter
  return sns_qr_solve(d, n, dtype, SA, ld_sa, Sb, x0, R, info, ws, sns::kScratchBytes, stream);
}
