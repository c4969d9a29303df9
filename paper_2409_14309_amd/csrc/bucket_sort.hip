// Stable counting sort of rows by CountSketch bucket (deterministic, integer
// only).  The keys are the rows 0..m-1, or the m entries of an ascending row
// list; for the sparse sign embedding with zeta nonzeros per column, key t
// stands for hash t % zeta of row t / zeta (zeta m keys, the row id and its
// sign land in the permutation as for the CountSketch).  Keys are cut into wave-blocks of `rw` consecutive keys; each wave
// histograms its block in LDS, a two-level exclusive scan in bucket-major
// order turns the per-block counts into start offsets, and each wave then
// places its rows in ascending order, ranking equal buckets within a batch of
// 64 rows by lane order.  The resulting order inside a bucket is ascending row
// index, independent of the launch.
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
    if (a.zeta > 1) {  // key t: hash t % zeta of row t / zeta (keys < 2^31)
      for (int64_t t = r0 + lane; t < r1; t += 64) {
        const uint32_t row = (uint32_t)t / a.zeta, k = (uint32_t)t - row * a.zeta;
        atomicAdd(&hist[ss_hash(a.seed, d, row, k).h], 1u);
      }
    } else if (a.rows) {
      for (int64_t t = r0 + lane; t < r1; t += 64)
        atomicAdd(&hist[cs_hash(a.seed, d, a.rows[t]).h], 1u);
    } else {
      for (int64_t j = (r0 >> 1) + lane; 2 * j < r1; j += 64) {
        Hash e, o;
        cs_hash_pair(a.seed, d, (uint64_t)j, e, o);
        atomicAdd(&hist[e.h], 1u);
        if (2 * j + 1 < r1) atomicAdd(&hist[o.h], 1u);
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
  // 16 counts loaded before any is overwritten: one memory round trip per 16
  for (; wb + 16 <= w1; wb += 16) {
    uint32_t c[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) c[u] = a.counts[(wb + u) * a.d + k];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
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
    for (; s + 16 <= a.nseg; s += 16) {  // 16 loads in flight before the stores
      uint32_t c[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) c[u] = a.segtot[(s + u) * d + k];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
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
  const uint32_t* rows = a.rows;
  const BT* b = static_cast<const BT*>(a.b);
  BT* bperm = static_cast<BT*>(a.bperm);
  uint32_t nrow = rows && r0 + lane < r1 ? rows[r0 + lane] : 0u;
  const int nbits = d > 1 ? 32 - __clz((int)(d - 1)) : 0;  // bits of the largest bucket
  for (int64_t r = r0; r < r1; r += 64) {
    const int64_t tk = r + lane;
    const bool valid = tk < r1;
    int64_t i = rows ? (int64_t)nrow : tk;
    if (rows) nrow = tk + 64 < r1 ? rows[tk + 64] : 0u;  // next batch in flight
    Hash hs;
    if (a.zeta > 1) {
      const uint32_t row = (uint32_t)tk / a.zeta, k = (uint32_t)tk - row * a.zeta;
      i = row;
      hs = ss_hash(a.seed, d, row, k);
    } else {
      hs = cs_hash(a.seed, d, (uint64_t)i);
    }
    const uint32_t h = valid ? hs.h : 0u;
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
      a.perm[pos] = (uint32_t)i | (hs.neg ? 0x80000000u : 0u);
      if (bperm) {
        const BT v = b[i];
        bperm[pos] = hs.neg ? -v : v;
      }
      if (last) next[h] = pos + 1;
    }
  }
}

template <typename BT>
__global__ void k_sort_scatter(const SortArgs* __restrict__ P, Map mp, int waves) {
  extern __shared__ uint32_t lds[];
  const uint32_t it = blockIdx.x;
  if (it >= mp.off[mp.nprob]) return;
  const int pi = map_find(mp, it);
  sort_scatter_item<BT>(P[pi], it - mp.off[pi], waves, lds);
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
  if (j.f64)
    SNS_LAUNCH("sort_scatter", k_sort_scatter<double>, dim3(grid_for(j.ncount)), dim3(nthr), lds,
               st, j.args, j.mcount, waves);
  else
    SNS_LAUNCH("sort_scatter", k_sort_scatter<float>, dim3(grid_for(j.ncount)), dim3(nthr), lds,
               st, j.args, j.mcount, waves);
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
