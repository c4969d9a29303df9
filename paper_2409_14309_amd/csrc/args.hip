// Device argument tables of the batched launches: built on the host, copied
// to the workspace by kernel launches whose parameters carry the bytes (so a
// capture of the launch sequence holds its arguments, and no host buffer has
// to outlive the call).
#include <string.h>

#include "common.hpp"
#include "kernels.hpp"

namespace sns {

namespace {

constexpr int kPutWords = 384;  // 3 KiB of table per launch
struct PutBlob {
  uint64_t w[kPutWords];
};

__global__ void k_put(PutBlob b, int nwords, uint64_t* __restrict__ dst) {
  for (int i = threadIdx.x; i < nwords; i += blockDim.x) dst[i] = b.w[i];
}

}  // namespace

size_t ArgTable::reserve(size_t nbytes) {
  const size_t off = (host_.size() + kArgTableAlign - 1) / kArgTableAlign * kArgTableAlign;
  host_.resize(off + nbytes, 0);
  // keep the image a whole number of 16-byte units
  host_.resize((host_.size() + kArgTableAlign - 1) / kArgTableAlign * kArgTableAlign, 0);
  return off;
}

void ArgTable::memcpy_bytes(size_t off, const void* src, size_t nbytes) {
  memcpy(host_.data() + off, src, nbytes);
}

Map ArgTable::map(const std::vector<uint32_t>& counts, uint32_t* total) {
  std::vector<uint32_t> off(counts.size() + 1, 0u);
  for (size_t i = 0; i < counts.size(); ++i) off[i + 1] = off[i] + counts[i];
  if (total) *total = off.back();
  Map m;
  m.off = add(off.data(), off.size());
  m.nprob = (int)counts.size();
  return m;
}

sns_status ArgTable::upload(hipStream_t st) const {
  if (host_.empty()) return SNS_OK;
  if (!dev_) return SNS_ERR_INVALID_ARG;
  const size_t nwords = host_.size() / 8;
  uint64_t* dst = reinterpret_cast<uint64_t*>(dev_);
  for (size_t w0 = 0; w0 < nwords; w0 += kPutWords) {
    const size_t nw = nwords - w0 < (size_t)kPutWords ? nwords - w0 : (size_t)kPutWords;
    PutBlob b;
    memset(&b, 0, sizeof(b));
    memcpy(b.w, host_.data() + w0 * 8, nw * 8);
    SNS_LAUNCH("put_args", k_put, dim3(1), dim3(128), 0, st, b, (int)nw, dst + w0);
  }
  SNS_HIP_TRY(hipGetLastError());
  return SNS_OK;
}

}  // namespace sns
