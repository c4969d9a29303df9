// Dense Gaussian sketch (Gaussian operator, i.i.d. normal entries):
// SA = d^{-1/2} G bf16(A), Sb = d^{-1/2} G bf16(b), on the matrix cores.
//
// G[k, i] = T[q] with q the byte (i & 15) of Philox4x32-10 at counter
// (i >> 4 mod 2^32, i >> 36, k, 1) and the sketch seed as key; T[q] is the
// normal quantile at (q + 1/2) / 256 rounded to bfloat16.  The table is built
// here on the host from the complementary error function by bisection and
// rounded to bfloat16 directly from the double's bits (ties to even).
//
// The product is a split-K GEMM on the matrix cores: G is generated per
// K-step into LDS (one Philox call per generator thread), A is converted to
// bf16 into LDS, and each work-group accumulates its 128 x 512 tile of SA
// over a chunk of rows in fp32; a second kernel adds the chunks in a fixed
// order and applies d^{-1/2}.
#include <math.h>
#include <mutex>
#include <string.h>

#include <type_traits>

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

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

// Tile of one work-group: 128 sketch rows x 512 columns of SA, fed by K-steps
// of 32 rows of A.  Eight waves: wave (wr, wc) owns rows [64 wr, 64 wr + 64)
// and columns [128 wc, 128 wc + 128) as 2 x 4 tiles of 32 x 32 computed with
// v_mfma_f32_32x32x16_bf16 (two k-substeps of 16 per K-step).  Every thread
// streams its share of the next 32 x 512 tile of A while the products run;
// waves 0-3 also generate the next K-step's G tile (one Philox call per
// thread).  One G tile serves all 512 columns, so the generator work per flop
// is half that of a 256-column tile.
constexpr int kTM = 128, kTN = 512, kKS = 32, kThreads = 512;
// LDS stages: the tile of K-step st is staged during K-step st - 2, so a wave
// can read the next K-step's first fragments before the barrier that closes
// the current one.
constexpr int kStages = 3;
constexpr int kPad = 40;  // LDS row stride in bf16: 32 values + 8 (keeps 16-byte reads conflict free)

struct GaussTable {
  uint32_t w[128];  // T[2e] in the low half, T[2e + 1] in the high half
};

// A tile in LDS: one row of kPad bf16 per column of A, holding its 32 K-step
// values as four 16-byte chunks.  Chunk q of row r sits at slot q ^ aswz(r),
// so that the 16-byte stores of one wave (rows 4 l + c, l = lane) spread over
// all banks while the fragment reads (32 consecutive rows, one chunk) stay
// conflict free.
__device__ __forceinline__ int aswz(int r) { return ((r >> 4) & 1) | (((r >> 3) & 1) << 1); }

__device__ __forceinline__ __bf16 bits_to_bf16(unsigned short u) {
  return __builtin_bit_cast(__bf16, u);
}

// SA partials (split K): partA[kc][k][j] = sum over this chunk's rows i of
// G[k, i] bf16(A[i, j]) (fp32 accumulation on the matrix cores), and
// partB[kc][k] = sum G[k, i] bf16(b[i]) (fp32 on the vector units).
// G[k, i] = T[q], q = byte (i & 15) of Philox4x32-10 at counter
// (i >> 4, 0, k, 1) (high counter word: i >> 36), key = seed.
__global__ __launch_bounds__(kThreads, 1) void k_gauss_sketch(
    const float* __restrict__ A, int64_t ld, int64_t m, int n, const float* __restrict__ b,
    uint64_t seed, int d, GaussTable table, int64_t ksteps, int vec_ok, int mt, int nt,
    float* __restrict__ partA, float* __restrict__ partB) {
  __shared__ unsigned short tbl[256];
  __shared__ __attribute__((aligned(16))) unsigned short Gbuf[kStages][kTM * kPad];
  __shared__ __attribute__((aligned(16))) unsigned short Bbuf[kStages][kTN * kPad];
  __shared__ float sbred[2][kTM];
  __shared__ __attribute__((aligned(16))) float bsh[kStages][kKS];  // b of the staged K-steps (rounded to bf16 when read)

  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wr = wave >> 2, wc = wave & 3;
  // Work-groups are handed to the 8 XCDs in turn; renumber them so that the
  // mt sketch-row tiles that read the same rows and columns of A run on one
  // XCD and share its L2.
  const int nwg = gridDim.x;
  const int h = blockIdx.x;
  const int L = (nwg % 8 == 0) ? (h % 8) * (nwg / 8) + h / 8 : h;
  const int bx = L % mt, by = (L / mt) % nt, kc = L / (mt * nt), S = nwg / (mt * nt);
  const int k0 = bx * kTM, j0 = by * kTN;
  const int64_t s0 = ksteps * kc / S, s1 = ksteps * (kc + 1) / S;
  if (t < 128) {
    tbl[2 * t] = (unsigned short)(table.w[t] & 0xFFFFu);
    tbl[2 * t + 1] = (unsigned short)(table.w[t] >> 16);
  }
  const bool gen = t < 256;  // waves 0-3 also generate G
  // generator role: sketch row gr, half gh (16 consecutive rows of A)
  const int gr = t & 127, gh = (t >> 7) & 1;
  const int gk = k0 + gr;
  const bool do_b = b != nullptr && by == 0;
  float sb = 0.f;
  // A-loading role (every thread): 4 columns (4 ac .. 4 ac + 3), 8 rows (8 ar .. 8 ar + 7)
  const int ac = t & 127, ar = t >> 7;
  const int aj = j0 + 4 * ac;

  f32x16 acc[2][4];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[rt][ct][q] = 0.f;

  float av[8][4];
  float bq[4];  // threads 0-7: b[32 st + 4 t .. + 3] of the K-step being staged
  const bool b_loader = do_b && t < kKS / 4;
  // this thread's 4 columns are all inside A (vector loads) when vec_ok
  const bool cols_in = vec_ok && aj + 3 < n;
  auto load_A = [&](int64_t st) {
    const int64_t i0 = st * kKS + 8 * ar;
    const float* p = A + i0 * ld + aj;  // one 64-bit product per step; rows by pointer steps
    if (cols_in) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
        if (i0 + e < m) x = *reinterpret_cast<const float4*>(p);
        av[e][0] = x.x; av[e][1] = x.y; av[e][2] = x.z; av[e][3] = x.w;
        p += ld;
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
#pragma unroll
        for (int c = 0; c < 4; ++c) av[e][c] = (i0 + e < m && aj + c < n) ? p[c] : 0.f;
        p += ld;
      }
    }
  };
  auto load_b = [&](int64_t st) {
    const int64_t i0 = st * kKS + 4 * t;
#pragma unroll
    for (int c = 0; c < 4; ++c) bq[c] = i0 + c < m ? b[i0 + c] : 0.f;
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      bf16x8 v;
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = (__bf16)av[e][c];
      *reinterpret_cast<bf16x8*>(&Bbuf[buf][(4 * ac + c) * kPad + 8 * (ar ^ aswz(4 * ac + c))]) = v;
    }
  };  auto store_A = [&](int buf) {
    if (b_loader) {
#pragma unroll
      for (int c = 0; c < 4; ++c) bsh[buf][4 * t + c] = bq[c];
    }
    store_tile(buf);
  };

  // G[gk, 16 jb .. 16 jb + 15] for the K-step st: one Philox call, 16 table lookups
  auto make_G = [&](int64_t st, bf16x8& lo, bf16x8& hi) {
    const uint64_t jb = (uint64_t)(st * kKS) / 16 + gh;  // 16-row block of A
    const U4 w = philox4x32_10(U4{(uint32_t)jb, (uint32_t)(jb >> 32), (uint32_t)gk, 1u},
                               (uint32_t)seed, (uint32_t)(seed >> 32));
    const uint32_t wv[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const unsigned short g = tbl[(wv[e >> 2] >> (8 * (e & 3))) & 0xFFu];
      if (e < 8) lo[e] = bits_to_bf16(g);
      else hi[e - 8] = bits_to_bf16(g);
    }
  };
  auto gen_G = [&](int64_t st, int buf) {
    bf16x8 lo, hi;
    if (gk < d) {
      make_G(st, lo, hi);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) { lo[e] = (__bf16)0.f; hi[e] = (__bf16)0.f; }
    }
    *reinterpret_cast<bf16x8*>(&Gbuf[buf][gr * kPad + 16 * gh]) = lo;
    *reinterpret_cast<bf16x8*>(&Gbuf[buf][gr * kPad + 16 * gh + 8]) = hi;
  };
  // Sb partial of this K-step: generator row gr, its 16 rows of half gh, in order
  auto sketch_b = [&](int buf) {
    const bf16x8 lo = *reinterpret_cast<const bf16x8*>(&Gbuf[buf][gr * kPad + 16 * gh]);
    const bf16x8 hi = *reinterpret_cast<const bf16x8*>(&Gbuf[buf][gr * kPad + 16 * gh + 8]);
    const float4* bp = reinterpret_cast<const float4*>(&bsh[buf][16 * gh]);
    float bv[16];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const float4 x = bp[c];
      bv[4 * c] = x.x; bv[4 * c + 1] = x.y; bv[4 * c + 2] = x.z; bv[4 * c + 3] = x.w;
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) bv[e] = (float)(__bf16)bv[e];
#pragma unroll
    for (int e = 0; e < 16; ++e) sb = fmaf((float)(e < 8 ? lo[e] : hi[e - 8]), bv[e], sb);
  };
  auto mfma = [&](int buf) {
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const int kofs = 16 * ks + 8 * (lane >> 5);
      bf16x8 ao[2], bo[4];
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
        ao[rt] = *reinterpret_cast<const bf16x8*>(
            &Gbuf[buf][(wr * 64 + rt * 32 + (lane & 31)) * kPad + kofs]);
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        const int r = wc * 128 + ct * 32 + (lane & 31);
        bo[ct] = *reinterpret_cast<const bf16x8*>(
            &Bbuf[buf][r * kPad + 8 * ((2 * ks + (lane >> 5)) ^ aswz(r))]);
      }
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
          acc[rt][ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ao[rt], bo[ct], acc[rt][ct], 0, 0, 0);
    }
  };

  // fragments of one K-substep from stage slot sl: G rows (f < 2), A columns (f >= 2)
  auto frag = [&](int sl, int ks, int f, bf16x8* ao, bf16x8* bo) {
    if (f < 2) {
      ao[f] = *reinterpret_cast<const bf16x8*>(
          &Gbuf[sl][(wr * 64 + f * 32 + (lane & 31)) * kPad + 16 * ks + 8 * (lane >> 5)]);
    } else {
      const int r = wc * 128 + (f - 2) * 32 + (lane & 31);
      bo[f - 2] = *reinterpret_cast<const bf16x8*>(
          &Bbuf[sl][r * kPad + 8 * ((2 * ks + (lane >> 5)) ^ aswz(r))]);
    }
  };

  __syncthreads();  // table ready
  if (s0 < s1) {
    // prologue: stage the first two K-steps
    load_A(s0);
    if (b_loader) load_b(s0);
    if (gen) gen_G(s0, 0);
    store_A(0);
    if (s0 + 1 < s1) {
      load_A(s0 + 1);
      if (b_loader) load_b(s0 + 1);
      if (gen) gen_G(s0 + 1, 1);
      store_A(1);
    }
    __syncthreads();
    // Straight-line K-steps: the K-step staged two ahead lies wholly inside A
    // (all 32 rows, this tile's 512 columns by vector loads) and every
    // generator row is a sketch row.  Each wave role runs its own loop with no
    // branch in the body, so the products can be interleaved with the loads,
    // the generator and the LDS stores; both loops meet the same barriers.
    const bool wg_fast = vec_ok && j0 + kTN <= n && k0 + kTM <= d;
    const int64_t sfull = m / kKS;  // K-steps [0, sfull) are full
    int64_t sf_end = (s1 < sfull ? s1 : sfull) - 2;
    if (!wg_fast || sf_end < s0) sf_end = s0;
    int cur = 0;
    bf16x8 f0a[2], f0b[4];  // first-substep fragments of the current K-step
    auto fast_step = [&](auto genc, auto dobc, int64_t st) {
      constexpr bool GEN = decltype(genc)::value, DOB = decltype(dobc)::value;
      const int n1 = cur == kStages - 1 ? 0 : cur + 1, n2 = n1 == kStages - 1 ? 0 : n1 + 1;
      const int64_t sn = st + 2;  // the K-step staged now
      float bn[4];
      if constexpr (DOB) {  // product lanes stage 4 values of b each (8 distinct per wave)
        const float* bp = b + sn * kKS + 4 * (lane & 7);
#pragma unroll
        for (int c = 0; c < 4; ++c) bn[c] = bp[c];
      }
      const float* p = A + (sn * kKS + 8 * ar) * ld + aj;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float4 x = *reinterpret_cast<const float4*>(p);
        av[e][0] = x.x; av[e][1] = x.y; av[e][2] = x.z; av[e][3] = x.w;
        p += ld;
      }
      __builtin_amdgcn_sched_barrier(0);  // the global loads go out first
      bf16x8 f1a[2], f1b[4];
      if constexpr (!GEN) {
        // Product waves: the second substep's fragments and (with b) this
        // K-step's Sb terms in the shadow of the products, in a fixed order.
        bf16x8 glo, ghi;
        float bv[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int ks = q >> 3, rt = (q >> 2) & 1, ct = q & 3;
          acc[rt][ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ks ? f1a[rt] : f0a[rt],
                                                                ks ? f1b[ct] : f0b[ct],
                                                                acc[rt][ct], 0, 0, 0);
          __builtin_amdgcn_sched_barrier(0);
          if (q < 6) frag(cur, 1, q, f1a, f1b);
          if constexpr (DOB) {
            if (q == 6) {
              glo = *reinterpret_cast<const bf16x8*>(&Gbuf[cur][gr * kPad + 16 * gh]);
              ghi = *reinterpret_cast<const bf16x8*>(&Gbuf[cur][gr * kPad + 16 * gh + 8]);
              const float4* bp4 = reinterpret_cast<const float4*>(&bsh[cur][16 * gh]);
#pragma unroll
              for (int c = 0; c < 4; ++c) {
                const float4 x = bp4[c];
                bv[4 * c] = x.x; bv[4 * c + 1] = x.y; bv[4 * c + 2] = x.z; bv[4 * c + 3] = x.w;
              }
#pragma unroll
              for (int e = 0; e < 16; ++e) bv[e] = (float)(__bf16)bv[e];
            } else if (q == 10 || q == 11) {
#pragma unroll
              for (int e = 8 * (q - 10); e < 8 * (q - 9); ++e)
                sb = fmaf((float)(e < 8 ? glo[e] : ghi[e - 8]), bv[e], sb);
            } else if (q == 15) {
              *reinterpret_cast<float4*>(&bsh[n2][4 * (lane & 7)]) =
                  make_float4(bn[0], bn[1], bn[2], bn[3]);
            }
          }
          __builtin_amdgcn_sched_barrier(0);
        }
      } else {
        // The generator's work for the K-step staged now runs in the shadow
        // of the 16 products, one slice after each product (the order is fixed
        // with scheduling fences): the second substep's fragment reads, the
        // ten Philox rounds, the 16 table lookups, then the G row's stores.
        const uint64_t jb = (uint64_t)(sn * kKS) / 16 + gh;
        U4 c = U4{(uint32_t)jb, (uint32_t)(jb >> 32), (uint32_t)gk, 1u};
        bf16x8 lo, hi;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int ks = q >> 3, rt = (q >> 2) & 1, ct = q & 3;
          acc[rt][ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ks ? f1a[rt] : f0a[rt],
                                                                ks ? f1b[ct] : f0b[ct],
                                                                acc[rt][ct], 0, 0, 0);
          __builtin_amdgcn_sched_barrier(0);
          if (q < 6) frag(cur, 1, q, f1a, f1b);
          if (q < 10) {  // Philox4x32-10 round q (key bumped q times)
            const uint32_t k0 = (uint32_t)seed + (uint32_t)q * 0x9E3779B9u;
            const uint32_t k1 = (uint32_t)(seed >> 32) + (uint32_t)q * 0xBB67AE85u;
            const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
            c = U4{(uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1,
                   (uint32_t)p0};
          } else if (q == 10) {
            const uint32_t wv[2] = {c.x, c.y};
#pragma unroll
            for (int e = 0; e < 8; ++e) lo[e] = bits_to_bf16(tbl[(wv[e >> 2] >> (8 * (e & 3))) & 0xFFu]);
          } else if (q == 11) {
            const uint32_t wv[2] = {c.z, c.w};
#pragma unroll
            for (int e = 0; e < 8; ++e) hi[e] = bits_to_bf16(tbl[(wv[e >> 2] >> (8 * (e & 3))) & 0xFFu]);
          } else if (q == 13) {
            *reinterpret_cast<bf16x8*>(&Gbuf[n2][gr * kPad + 16 * gh]) = lo;
            *reinterpret_cast<bf16x8*>(&Gbuf[n2][gr * kPad + 16 * gh + 8]) = hi;
          }
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      store_tile(n2);
      // K-step st + 1 was staged before the last barrier: read its first
      // fragments now, so the products can start right after this barrier.
#pragma unroll
      for (int f = 0; f < 6; ++f) frag(n1, 0, f, f0a, f0b);
      __syncthreads();
      cur = n1;
    };
    using T_ = std::true_type;
    using F_ = std::false_type;
    int64_t st = s0;
    if (sf_end > s0) {
#pragma unroll
      for (int f = 0; f < 6; ++f) frag(cur, 0, f, f0a, f0b);
      if (gen) {
        for (; st < sf_end; ++st) fast_step(T_{}, F_{}, st);
      } else {
        if (do_b)
          for (; st < sf_end; ++st) fast_step(F_{}, T_{}, st);
        else
          for (; st < sf_end; ++st) fast_step(F_{}, F_{}, st);
      }
    }
    for (; st < s1; ++st) {
      const int n1 = cur == kStages - 1 ? 0 : cur + 1, n2 = n1 == kStages - 1 ? 0 : n1 + 1;
      const bool more = st + 2 < s1;
      if (more) {  // in flight during the products
        load_A(st + 2);
        if (b_loader) load_b(st + 2);
      }
      mfma(cur);
      if (do_b && !gen && gk < d) sketch_b(cur);
      if (more) {
        if (gen) gen_G(st + 2, n2);
        store_A(n2);
      }
      __syncthreads();
      cur = n1;
    }
  }
  // epilogue: accumulator element q of lane l in a 32 x 32 tile is
  // row 8 (q / 4) + 4 (l / 32) + q % 4, column l % 32
  float* P = partA + (size_t)kc * d * n;
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const int col = j0 + wc * 128 + ct * 32 + (lane & 31);
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int row = k0 + wr * 64 + rt * 32 + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
        if (row < d && col < n) P[(size_t)row * n + col] = acc[rt][ct][q];
      }
    }
  if (do_b) {
    if (!gen) sbred[gh][gr] = sb;
    __syncthreads();
    if (t < kTM && k0 + t < d) partB[(size_t)kc * d + k0 + t] = sbred[0][t] + sbred[1][t];
  }
}

// SA = scale * sum_kc partA[kc], Sb = scale * sum_kc partB[kc] (chunks in order).
__global__ void k_gauss_reduce(int64_t dn, int d, int S, float scale, const float* __restrict__ partA,
                               const float* __restrict__ partB, float* __restrict__ SA,
                               float* __restrict__ Sb) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < dn + d;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (e < dn) {
      float s = 0.f;
      for (int c = 0; c < S; ++c) s += partA[(size_t)c * dn + e];
      SA[e] = s * scale;
    } else if (Sb) {
      const int64_t k = e - dn;
      float s = 0.f;
      for (int c = 0; c < S; ++c) s += partB[(size_t)c * d + k];
      Sb[k] = s * scale;
    }
  }
}

struct GaussPlan {
  int mt, nt, S;
  int64_t ksteps;
};

GaussPlan make_gauss_plan(const sns_matrix& A, uint32_t d) {
  GaussPlan g;
  g.mt = (int)((d + kTM - 1) / kTM);
  g.nt = (int)((A.n + kTN - 1) / kTN);
  g.ksteps = (A.m + kKS - 1) / kKS;
  const int64_t tiles = (int64_t)g.mt * g.nt;
  int64_t S = (256 + tiles - 1) / tiles;        // one work-group per CU (LDS-limited)
  const int64_t maxS = g.ksteps / 8 > 0 ? g.ksteps / 8 : 1;  // >= 8 K-steps per chunk
  if (S > maxS) S = maxS;
  if (S > 256) S = 256;
  if (S < 1) S = 1;
  g.S = (int)S;
  return g;
}

}  // namespace

size_t gauss_workspace_bytes(const sns_matrix& A, uint32_t d) {
  const GaussPlan g = make_gauss_plan(A, d);
  return align_up((size_t)g.S * d * A.n * sizeof(float)) + align_up((size_t)g.S * d * sizeof(float));
}

sns_status launch_gauss_sketch(const sns_matrix& A, uint32_t d, uint64_t seed, const void* b,
                               void* SA, void* Sb, void* ws, hipStream_t st) {
  if (A.dtype != SNS_F32 || A.layout != SNS_DENSE_ROWMAJOR) return SNS_ERR_DTYPE;
  const GaussPlan g = make_gauss_plan(A, d);
  float* partA = static_cast<float*>(ws);
  float* partB = reinterpret_cast<float*>(static_cast<char*>(ws) +
                                          align_up((size_t)g.S * d * A.n * sizeof(float)));
  GaussTable tab;
  const uint16_t* T = gauss_table_host();
  for (int e = 0; e < 128; ++e) tab.w[e] = (uint32_t)T[2 * e] | ((uint32_t)T[2 * e + 1] << 16);
  const int vec_ok = ((uintptr_t)A.values % 16 == 0) && (A.ld % 4 == 0);
  SNS_LAUNCH("gauss_mfma", k_gauss_sketch, dim3(g.mt * g.nt * g.S), dim3(kThreads), 0, st,
             static_cast<const float*>(A.values), A.ld, A.m, (int)A.n,
             static_cast<const float*>(b), seed, (int)d, tab, g.ksteps, vec_ok, g.mt, g.nt, partA,
             partB);
  const int64_t dn = (int64_t)d * A.n;
  int64_t blocks = (dn + d + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  const float scale = (float)(1.0 / sqrt((double)d));
  SNS_LAUNCH("gauss_reduce", k_gauss_reduce, dim3((unsigned)blocks), dim3(256), 0, st, dn, (int)d,
             g.S, scale, partA, b ? partB : nullptr, static_cast<float*>(SA),
             b ? static_cast<float*>(Sb) : nullptr);
  SNS_HIP_TRY(hipGetLastError());
  return SNS_OK;
}

}  // namespace sns

extern "C" sns_status sns_gaussian_table(uint16_t* out) {
  if (!out) return SNS_ERR_INVALID_ARG;
  memcpy(out, sns::gauss_table_host(), 256 * sizeof(uint16_t));
  return SNS_OK;
}
