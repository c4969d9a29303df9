// Stable counting sort of rows by CountSketch bucket (deterministic, integer
// only).  The keys are the rows 0..m-1, or the m entries of an ascending row
// list; for the sparse sign embedding with zeta nonzeros per column, key t
// stands for hash t % zeta of row t / zeta (zeta m keys, the row id and its
// sign land in the permutation as for the CountSketch).  Keys are cut into
// wave-blocks of `rw` consecutive keys; each wave hashes its block once,
// histograms it in LDS and keeps every key's bucket and sign (2 bytes); a
// two-level exclusive scan in bucket-major order turns the per-block counts
// into start offsets, and each wave then places its rows in ascending order
// from the kept hashes, ranking equal buckets within a batch of 64 rows by
// lane order.  The resulting order inside a bucket is ascending row index,
// independent of the launch.
#include <mutex>

#include "common.hpp"
#include "kernels.hpp"

namespace sns {

namespace {

// Hash k of row i of the sparse sign embedding: the CountSketch rule with
// counter word 2 = k (k = 0 is cs_hash).
__device__ __forceinline__ Hash ss_hash(uint64_t seed, uint32_t d, uint64_t i, uint32_t k) {
  const uint64_t j = i >> 1;
  const U4 w = philox4x32_10(U4{(uint32_t)j, (uint32_t)(j >> 32), k, 0u}, (uint32_t)seed,
                             (uint32_t)(seed >> 32));
  const uint32_t wh = (i & 1) ? w.z : w.x;
  const uint32_t ws = (i & 1) ? w.w : w.y;
  return Hash{(uint32_t)(((uint64_t)wh * d) >> 32), (ws >> 31) != 0u};
}

// A key's bucket (< 2^15) and sign in 16 bits, as kept between the passes.
__device__ __forceinline__ uint16_t pack_hash(const Hash& e) {
  return (uint16_t)(e.h | (e.neg ? 0x8000u : 0u));
}

// Row hashes for the test entry point.
__global__ void k_hash(uint64_t seed, uint32_t d, int64_t i0, int64_t count, uint32_t* h,
                       int8_t* s) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < count;
       t += (int64_t)gridDim.x * blockDim.x) {
    const Hash r = cs_hash(seed, d, (uint64_t)(i0 + t));
    if (h) h[t] = r.h;
    if (s) s[t] = r.neg ? -1 : 1;
  }
}

// counts[wb * d + k] = number of keys of wave-block wb in bucket k.  Key t is
// row t, or row rows[t] when a row list is given.  A work item is `waves`
// consecutive wave-blocks of one problem.
__device__ __forceinline__ void sort_count_item(const SortArgs& a, uint32_t loc, int waves,
                                                uint32_t* lds) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint32_t d = a.d;
  const int64_t wb = (int64_t)loc * waves + wv;
  uint32_t* hist = lds + (size_t)wv * d;
  for (uint32_t k = lane; k < d; k += 64) hist[k] = 0u;
  __syncthreads();
  const int64_t m = a.mdev ? (int64_t)*a.mdev : a.m;  // key count known only on the device
  if (wb < a.nwb) {
    const int64_t r0 = wb * a.rw, r1 = min(m, r0 + a.rw);  // r0 is even
    uint16_t* __restrict__ hkey = a.hkey;
    if (a.zeta > 1) {  // key t: hash t % zeta of row t / zeta (keys < 2^31)
      for (int64_t t = r0 + lane; t < r1; t += 64) {
        const uint32_t row = (uint32_t)t / a.zeta, k = (uint32_t)t - row * a.zeta;
        const Hash e = ss_hash(a.seed, d, row, k);
        atomicAdd(&hist[e.h], 1u);
        hkey[t] = pack_hash(e);
      }
    } else if (a.rows) {
      for (int64_t t = r0 + lane; t < r1; t += 64) {
        const Hash e = cs_hash(a.seed, d, a.rows[t]);
        atomicAdd(&hist[e.h], 1u);
        hkey[t] = pack_hash(e);
      }
    } else {
      // one Philox block per pair of rows; r0 is even, so pairs stay inside
      // the wave-block and the pair's two entries share one 4-byte word
      for (int64_t j = (r0 >> 1) + lane; 2 * j < r1; j += 64) {
        Hash e, o;
        cs_hash_pair(a.seed, d, (uint64_t)j, e, o);
        atomicAdd(&hist[e.h], 1u);
        if (2 * j + 1 < r1) {
          atomicAdd(&hist[o.h], 1u);
          reinterpret_cast<uint32_t*>(hkey)[j] =
              (uint32_t)pack_hash(e) | ((uint32_t)pack_hash(o) << 16);
        } else {
          hkey[2 * j] = pack_hash(e);
        }
      }
    }
  }
  __syncthreads();
  if (wb < a.nwb)
    for (uint32_t k = lane; k < d; k += 64) a.counts[wb * d + k] = hist[k];
}

__global__ void k_sort_count(const SortArgs* __restrict__ P, Map mp, int waves) {
  extern __shared__ uint32_t lds[];
  const uint32_t it = blockIdx.x;
  if (it >= mp.off[mp.nprob]) return;
  const int pi = map_find(mp, it);
  sort_count_item(P[pi], it - mp.off[pi], waves, lds);
}

// Within each segment of `seg` wave-blocks, replace counts by their exclusive
// prefix (per bucket) and record the segment totals.  A work item is 64
// buckets of one segment.
__global__ void k_scan_segments(const SortArgs* __restrict__ P, Map mp) {
  const uint32_t it = blockIdx.x;
  if (it >= mp.off[mp.nprob]) return;
  const int pi = map_find(mp, it);
  const SortArgs& a = P[pi];
  const uint32_t loc = it - mp.off[pi];
  const uint32_t kb = (a.d + 63) / 64;
  const uint32_t k = (loc % kb) * 64 + threadIdx.x;
  const int64_t s = loc / kb;
  if (k >= a.d) return;
  const int64_t w0 = s * a.seg, w1 = min(a.nwb, w0 + a.seg);
  uint32_t run = 0;
  int64_t wb = w0;
  // 32 counts loaded before any is overwritten: one memory round trip per 32
  for (; wb + 32 <= w1; wb += 32) {
    uint32_t c[32];
#pragma unroll
    for (int u = 0; u < 32; ++u) c[u] = a.counts[(wb + u) * a.d + k];
#pragma unroll
    for (int u = 0; u < 32; ++u) {
      a.counts[(wb + u) * a.d + k] = run;
      run += c[u];
    }
  }
  for (; wb < w1; ++wb) {
    const uint32_t c = a.counts[wb * a.d + k];
    a.counts[wb * a.d + k] = run;
    run += c;
  }
  a.segtot[s * a.d + k] = run;
}

// Exclusive scan across segments per bucket (in place in segtot), then across
// buckets: bucket_ptr[k] = rows in buckets < k, bucket_ptr[d] = m.  One work
// item (1024 threads) per problem.
__device__ __forceinline__ void scan_buckets_item(const SortArgs& a, uint32_t* wsum) {
  const int t = threadIdx.x, nt = blockDim.x;
  const uint32_t d = a.d;
  const uint32_t per = (d + nt - 1) / nt;
  const uint32_t k0 = min(d, t * per), k1 = min(d, k0 + per);
  uint32_t local = 0;
  for (uint32_t k = k0; k < k1; ++k) {
    uint32_t run = 0;
    int64_t s = 0;
    for (; s + 32 <= a.nseg; s += 32) {  // 32 loads in flight before the stores
      uint32_t c[32];
#pragma unroll
      for (int u = 0; u < 32; ++u) c[u] = a.segtot[(s + u) * d + k];
#pragma unroll
      for (int u = 0; u < 32; ++u) {
        a.segtot[(s + u) * d + k] = run;
        run += c[u];
      }
    }
    for (; s < a.nseg; ++s) {
      const uint32_t c = a.segtot[s * d + k];
      a.segtot[s * d + k] = run;
      run += c;
    }
    a.bucket_ptr[k] = run;  // bucket total for now
    local += run;
  }
  // exclusive scan of `local` over threads
  const int lane = t & 63, wv = t >> 6;
  uint32_t incl = local;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(incl, off, 64);
    if (lane >= off) incl += y;
  }
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  uint32_t before = 0;
  for (int w = 0; w < wv; ++w) before += wsum[w];
  uint32_t run = before + incl - local;
  for (uint32_t k = k0; k < k1; ++k) {
    const uint32_t c = a.bucket_ptr[k];
    a.bucket_ptr[k] = run;
    run += c;
  }
  if (t == nt - 1) a.bucket_ptr[d] = run;
}

__global__ __launch_bounds__(1024) void k_scan_buckets(const SortArgs* __restrict__ P, Map mp) {
  __shared__ uint32_t wsum[16];
  const uint32_t it = blockIdx.x;
  if (it >= mp.off[mp.nprob]) return;
  scan_buckets_item(P[map_find(mp, it)], wsum);
}

// Row id of key t (the hash was kept by the counting pass).
__device__ __forceinline__ int64_t key_row(const SortArgs& a, int64_t t) {
  if (a.zeta > 1) return (int64_t)((uint32_t)t / a.zeta);
  return a.rows ? (int64_t)a.rows[t] : t;
}

template <typename BT>
__device__ __forceinline__ void sort_scatter_item(const SortArgs& a, uint32_t loc, int waves,
                                                  uint32_t* lds) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint32_t d = a.d;
  const int64_t wb = (int64_t)loc * waves + wv;
  uint32_t* next = lds + (size_t)wv * d;  // this wave's own cursor per bucket
  if (wb >= a.nwb) return;
  const int64_t m = a.mdev ? (int64_t)*a.mdev : a.m;
  const int64_t r0 = wb * a.rw, r1 = min(m, r0 + a.rw);
  if (r0 >= r1) return;  // wave-block past the device-side key count
  {
    const int64_t s = wb / a.seg;
    for (uint32_t k = lane; k < d; k += 64)
      next[k] = a.bucket_ptr[k] + a.segtot[s * d + k] + a.counts[wb * d + k];
  }
  __builtin_amdgcn_wave_barrier();
  const uint16_t* __restrict__ hkey = a.hkey;
  const BT* __restrict__ b = static_cast<const BT*>(a.b);
  BT* bperm = static_cast<BT*>(a.bperm);
  const int nbits = d > 1 ? 32 - __clz((int)(d - 1)) : 0;  // bits of the largest bucket
  // the next batch's hash, row and b value are loaded one batch ahead
  uint32_t hk_n = 0u;
  int64_t i_n = 0;
  BT b_n = BT(0);
  if (r0 + lane < r1) {
    hk_n = hkey[r0 + lane];
    i_n = key_row(a, r0 + lane);
    if (bperm) b_n = b[i_n];
  }
  for (int64_t r = r0; r < r1; r += 64) {
    const int64_t tk = r + lane;
    const bool valid = tk < r1;
    const uint32_t hk = hk_n;
    const int64_t i = i_n;
    const BT bv = b_n;
    if (tk + 64 < r1) {
      hk_n = hkey[tk + 64];
      i_n = key_row(a, tk + 64);
      if (bperm) b_n = b[i_n];
    }
    const uint32_t h = valid ? (hk & 0x7FFFu) : 0u;
    const bool neg = (hk >> 15) != 0u;
    // lanes of this batch with the same bucket: the lanes holding a key whose
    // bucket agrees with this lane's in every bit (one ballot per bit of d-1);
    // the rank is the number of such lanes below this one
    uint64_t peers = __ballot(valid);
    for (int bit = 0; bit < nbits; ++bit) {
      const bool on = (h >> bit) & 1u;
      const uint64_t bal = __ballot(on);
      peers &= on ? bal : ~bal;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & ((1ull << lane) - 1ull));
    const bool last = lane == 63 || (peers >> (lane + 1)) == 0ull;
    if (valid) {
      const uint32_t pos = next[h] + rank;
      a.perm[pos] = (uint32_t)i | (neg ? 0x80000000u : 0u);
      if (bperm) bperm[pos] = neg ? -bv : bv;
      if (last) next[h] = pos + 1;
    }
  }
}

template <typename BT>
__global__ void k_sort_scatter(const SortArgs* __restrict__ P, Map mp, int waves) {
  extern __shared__ uint32_t lds[];
  // neighbouring wave-blocks fill the same cache lines of perm and bperm
  // (one entry per bucket each): keep them on one XCD so its L2 merges them
  const uint32_t n = mp.off[mp.nprob];
  if (blockIdx.x >= n) return;
  const uint32_t it = xcd_order(blockIdx.x, n);
  const int pi = map_find(mp, it);
  sort_scatter_item<BT>(P[pi], it - mp.off[pi], waves, lds);
}

// Bytes of the cursors and deltas at the head of the staged placing's LDS
// (16-byte aligned, so the staged values that follow are aligned).
__host__ __device__ constexpr size_t place_head_bytes(int waves, uint32_t d) {
  return ((size_t)(waves + 1) * d * 4 + 15) / 16 * 16;
}

// Staged placing of the kPlaceWaves consecutive wave-blocks of one
// work-group (all of their keys fit in LDS).  The group's entries of bucket k
// are one contiguous range of the output (wave-block order, then key order),
// so the group sorts its keys into LDS in output order and then writes each
// bucket's run with consecutive threads on consecutive addresses: the stores
// coalesce, and the cache lines a group fills are completed within its
// write-out.  LDS: cursor[kPlaceWaves][d], delta[d] (output position minus
// LDS position per bucket), then `cap` staged entries: row | sign, s(i) b[i],
// bucket.
constexpr int kPlaceWaves = 4;
constexpr int kPlaceBatches = 16;  // batches of 64 keys per wave-block, at most

template <typename BT>
__device__ __forceinline__ void sort_place_item(const SortArgs& a, uint32_t loc, int cap,
                                                char* lds, uint32_t* wsum) {
  constexpr int W = kPlaceWaves;
  const int t = threadIdx.x, nt = W * 64;
  const int lane = t & 63, wv = t >> 6;
  const uint32_t d = a.d;
  const int64_t wb0 = (int64_t)loc * W;
  const int64_t m = a.mdev ? (int64_t)*a.mdev : a.m;
  const int64_t k0 = wb0 * a.rw;
  const int64_t k1 = min(m, (wb0 + W) * a.rw);
  if (k0 >= k1) return;  // uniform over the group: no key to place
  uint32_t* cur = reinterpret_cast<uint32_t*>(lds);
  int32_t* delta = reinterpret_cast<int32_t*>(cur + (size_t)W * d);
  uint32_t* sperm = reinterpret_cast<uint32_t*>(lds + place_head_bytes(W, d));
  BT* sval = reinterpret_cast<BT*>(sperm + cap);
  uint16_t* sbkt = reinterpret_cast<uint16_t*>(sval + cap);
  const bool with_b = a.bperm != nullptr;

  // this wave's keys, hashes and b values: every load issued before any is used
  const int64_t r0 = (wb0 + wv) * a.rw, r1 = min(m, r0 + a.rw);
  uint32_t hk[kPlaceBatches];
  uint32_t row[kPlaceBatches];
  BT bv[kPlaceBatches];
#pragma unroll
  for (int u = 0; u < kPlaceBatches; ++u) {
    const int64_t tk = r0 + 64 * u + lane;
    const bool v = tk < r1;
    hk[u] = v ? (uint32_t)a.hkey[tk] : 0u;
    row[u] = v ? (a.zeta > 1 ? (uint32_t)tk / a.zeta : (a.rows ? a.rows[tk] : (uint32_t)tk)) : 0u;
  }
  const BT* __restrict__ b = static_cast<const BT*>(a.b);
#pragma unroll
  for (int u = 0; u < kPlaceBatches; ++u)
    bv[u] = (with_b && r0 + 64 * u + lane < r1) ? b[row[u]] : BT(0);

  // per bucket k: the group's output range starts at G_0 = start of its first
  // wave-block; wave-block w's entries start G_w - G_0 into it.  Thread t owns
  // buckets [b0, b1) for the exclusive scan of the group's counts.
  const uint32_t per = (d + nt - 1) / nt;
  const uint32_t b0 = min(d, t * per), b1 = min(d, b0 + per);
  const bool tail = wb0 + W >= a.nwb;
  const uint32_t* segA = a.segtot + (wb0 / a.seg) * d;
  const uint32_t* segB = tail ? segA : a.segtot + ((wb0 + W) / a.seg) * d;
  uint32_t local = 0;
#pragma unroll 4
  for (uint32_t k = b0; k < b1; ++k) {
    uint32_t g[W + 1];
    const uint32_t base = a.bucket_ptr[k] + segA[k];
#pragma unroll
    for (int w = 0; w < W; ++w)
      g[w] = wb0 + w < a.nwb ? base + a.counts[(wb0 + w) * d + k] : a.bucket_ptr[k + 1];
    g[W] = tail ? a.bucket_ptr[k + 1] : a.bucket_ptr[k] + segB[k] + a.counts[(wb0 + W) * d + k];
#pragma unroll
    for (int w = 1; w < W; ++w) cur[(size_t)w * d + k] = g[w] - g[0];
    cur[k] = g[W] - g[0];  // the group's count, for now
    delta[k] = (int32_t)g[0];
    local += g[W] - g[0];
  }
  uint32_t incl = local;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(incl, off, 64);
    if (lane >= off) incl += y;
  }
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  uint32_t run = incl - local;  // LDS start of bucket b0
  for (int w = 0; w < wv; ++w) run += wsum[w];
  for (uint32_t k = b0; k < b1; ++k) {
    const uint32_t cnt = cur[k];
    cur[k] = run;
#pragma unroll
    for (int w = 1; w < W; ++w) cur[(size_t)w * d + k] += run;
    delta[k] -= (int32_t)run;
    run += cnt;
  }
  __syncthreads();

  // each wave ranks its keys (batches of 64 in key order) into the staging area
  uint32_t* next = cur + (size_t)wv * d;
  const int nbits = d > 1 ? 32 - __clz((int)(d - 1)) : 0;
#pragma unroll
  for (int u = 0; u < kPlaceBatches; ++u) {
    if (r0 + 64 * u >= r1) break;  // uniform over the wave
    const bool valid = r0 + 64 * u + lane < r1;
    const uint32_t h = valid ? (hk[u] & 0x7FFFu) : 0u;
    const bool neg = (hk[u] >> 15) != 0u;
    uint64_t peers = __ballot(valid);
    for (int bit = 0; bit < nbits; ++bit) {
      const bool on = (h >> bit) & 1u;
      const uint64_t bal = __ballot(on);
      peers &= on ? bal : ~bal;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & ((1ull << lane) - 1ull));
    const bool last = lane == 63 || (peers >> (lane + 1)) == 0ull;
    if (valid) {
      const uint32_t pos = next[h] + rank;
      sperm[pos] = row[u] | (neg ? 0x80000000u : 0u);
      if (with_b) sval[pos] = neg ? -bv[u] : bv[u];
      sbkt[pos] = (uint16_t)h;
      if (last) next[h] = pos + 1;
    }
  }
  __syncthreads();

  // write-out in output order: entry j of the staging area goes to
  // delta[bucket] + j
  const int nk = (int)(k1 - k0);
  BT* bperm = static_cast<BT*>(a.bperm);
  for (int j = t; j < nk; j += nt) {
    const uint32_t gpos = (uint32_t)(delta[sbkt[j]] + j);
    if (gpos >= (uint64_t)a.m) continue;  // holds for consistent counts; keeps stores in bounds
    a.perm[gpos] = sperm[j];
    if (with_b) bperm[gpos] = sval[j];
  }
}

template <typename BT>
__global__ __launch_bounds__(kPlaceWaves * 64) void k_sort_place(const SortArgs* __restrict__ P,
                                                                 Map mp, int cap) {
  extern __shared__ __attribute__((aligned(16))) char lds_place[];
  __shared__ uint32_t wsum[kPlaceWaves];
  const uint32_t n = mp.off[mp.nprob];
  if (blockIdx.x >= n) return;
  const uint32_t it = xcd_order(blockIdx.x, n);
  const int pi = map_find(mp, it);
  sort_place_item<BT>(P[pi], it - mp.off[pi], cap, lds_place, wsum);
}

// Staged placing: at most this many keys per group, buckets and LDS bytes.
constexpr int kPlaceMaxKeys = 4096;
constexpr uint32_t kPlaceMaxD = 4096;
constexpr size_t kPlaceMaxLds = 144 * 1024;

size_t place_lds_bytes(int waves, uint32_t d, int cap, size_t es) {
  return place_head_bytes(waves, d) + (size_t)cap * (4 + es + 2);
}

int sort_waves(uint32_t maxd) {
  const int w = (int)(16384 / maxd);
  return w < 1 ? 1 : (w > 4 ? 4 : w);
}

}  // namespace

SortPlan make_sort_plan(int64_t m, uint32_t d, uint32_t zeta) {
  SortPlan p;
  p.m = m;
  p.d = d;
  p.zeta = zeta < 1 ? 1 : zeta;
  // at most ~4096 wave-blocks, at least 512 keys each, and at least d / 2
  // keys each so the d x nwb count matrix stays within ~2 entries per key
  int64_t rw = (m + 4095) / 4096;
  const int64_t rd = (int64_t)d / 2;
  rw = rw < rd ? rd : rw;
  rw = (rw + 63) / 64 * 64;
  p.rw = rw < 512 ? 512 : rw;
  p.nwb = (m + p.rw - 1) / p.rw;
  p.seg = 64;
  p.nseg = (p.nwb + p.seg - 1) / p.seg;
  return p;
}

void carve_sort(Carve& c, const SortPlan& p, size_t b_elem_bytes, SortBufs& s) {
  s.hkey = c.take<uint16_t>((size_t)p.m + 1);
  s.perm = c.take<uint32_t>((size_t)p.m);
  s.bperm = b_elem_bytes ? (void*)c.take<char>((size_t)p.m * b_elem_bytes) : nullptr;
  s.bucket_ptr = c.take<uint32_t>((size_t)p.d + 1);
  s.counts = c.take<uint32_t>((size_t)p.d * p.nwb);
  s.segtot = c.take<uint32_t>((size_t)p.d * p.nseg);
}

SortArgs sort_args(const SortPlan& p, uint64_t seed, const void* b, const SortBufs& s,
                   const uint32_t* rows, const uint32_t* mdev) {
  SortArgs a;
  a.seed = seed;
  a.m = p.m;
  a.rw = p.rw;
  a.nwb = p.nwb;
  a.seg = p.seg;
  a.nseg = p.nseg;
  a.d = p.d;
  a.zeta = p.zeta;
  a.rows = rows;
  a.mdev = mdev;
  a.b = b;
  a.hkey = s.hkey;
  a.perm = s.perm;
  a.bperm = b ? s.bperm : nullptr;
  a.bucket_ptr = s.bucket_ptr;
  a.counts = s.counts;
  a.segtot = s.segtot;
  return a;
}

SortJob build_sort_job(ArgTable& t, const std::vector<SortArgs>& a, bool f64) {
  SortJob j;
  j.count = (int)a.size();
  j.f64 = f64;
  if (a.empty()) return j;
  for (const SortArgs& x : a) j.maxd = x.d > j.maxd ? x.d : j.maxd;
  const int waves = sort_waves(j.maxd);
  // staged placing when every group's keys fit in LDS
  int64_t maxrw = 0;
  for (const SortArgs& x : a) maxrw = x.rw > maxrw ? x.rw : maxrw;
  j.cap = (int)(waves * maxrw);
  j.place_lds = place_lds_bytes(waves, j.maxd, j.cap, f64 ? 8 : 4);
  j.staged = waves == kPlaceWaves && maxrw <= 64 * kPlaceBatches && j.maxd <= kPlaceMaxD &&
             j.cap <= kPlaceMaxKeys && j.place_lds <= kPlaceMaxLds;
  std::vector<uint32_t> cnt, seg, one;
  for (const SortArgs& x : a) {
    cnt.push_back((uint32_t)((x.nwb + waves - 1) / waves));
    seg.push_back((uint32_t)(((x.d + 63) / 64) * x.nseg));
    one.push_back(1u);
  }
  j.args = t.add(a.data(), a.size());
  j.mcount = t.map(cnt, &j.ncount);
  j.mseg = t.map(seg, &j.nseg);
  j.mscan = t.map(one, &j.nscan);
  return j;
}

sns_status launch_sort_job(const SortJob& j, hipStream_t st) {
  if (j.count == 0) return SNS_OK;
  const int waves = sort_waves(j.maxd);
  const int nthr = waves * 64;
  const size_t lds = (size_t)waves * j.maxd * sizeof(uint32_t);
  SNS_LAUNCH("sort_count", k_sort_count, dim3(grid_for(j.ncount)), dim3(nthr), lds, st, j.args,
             j.mcount, waves);
  SNS_LAUNCH("scan_segments", k_scan_segments, dim3(grid_for(j.nseg)), dim3(64), 0, st, j.args,
             j.mseg);
  SNS_LAUNCH("scan_buckets", k_scan_buckets, dim3(grid_for(j.nscan)), dim3(1024), 0, st, j.args,
             j.mscan);
  if (j.staged) {
    if (j.place_lds > 64 * 1024) {  // more than the default dynamic LDS of a work-group
      static std::once_flag once;
      std::call_once(once, [] {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sort_place<double>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)kPlaceMaxLds);
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sort_place<float>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)kPlaceMaxLds);
      });
    }
    if (j.f64)
      SNS_LAUNCH("sort_place", k_sort_place<double>, dim3(grid_for(j.ncount)), dim3(nthr),
                 j.place_lds, st, j.args, j.mcount, j.cap);
    else
      SNS_LAUNCH("sort_place", k_sort_place<float>, dim3(grid_for(j.ncount)), dim3(nthr),
                 j.place_lds, st, j.args, j.mcount, j.cap);
  } else if (j.f64) {
    SNS_LAUNCH("sort_scatter", k_sort_scatter<double>, dim3(grid_for(j.ncount)), dim3(nthr), lds,
               st, j.args, j.mcount, waves);
  } else {
    SNS_LAUNCH("sort_scatter", k_sort_scatter<float>, dim3(grid_for(j.ncount)), dim3(nthr), lds,
               st, j.args, j.mcount, waves);
  }
  SNS_HIP_TRY(hipGetLastError());
  return SNS_OK;
}

sns_status launch_hash(uint64_t seed, uint32_t d, int64_t i0, int64_t count, uint32_t* h,
                       int8_t* s, hipStream_t st) {
  if (count == 0) return SNS_OK;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  SNS_LAUNCH("hash", k_hash, dim3((unsigned)blocks), dim3(256), 0, st, seed, d, i0, count, h, s);
  SNS_HIP_TRY(hipGetLastError());
  return SNS_OK;
}

}  // namespace sns
