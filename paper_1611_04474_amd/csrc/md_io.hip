// Copies between device memory and pinned host memory by kernel, for the serving loop:
// one launch moves every input or output segment of a batch, with coalesced 16-byte
// loads and stores through the device's mapping of the pinned host pages. No runtime copy
// engine or staging path is involved, so enqueueing the copies costs one kernel launch
// and never waits on earlier work.
#include "md_common.hpp"

namespace md {
namespace {

constexpr int kSegMax = 128;          // segments per launch (kernel arguments under 4 KB)
constexpr int kCopyThreads = 256;
constexpr size_t kChunk = 64 * 1024;  // bytes per workgroup

struct SegBatch {
  int n;
  int64_t cum[kSegMax + 1];           // first workgroup of each segment
  md_copy_segment seg[kSegMax];
};

__global__ __launch_bounds__(kCopyThreads) void k_copy_segments(SegBatch b) {
  int s = 0;
  while (s + 1 < b.n && b.cum[s + 1] <= (int64_t)blockIdx.x) ++s;
  const md_copy_segment g = b.seg[s];
  const size_t c0 = (size_t)(blockIdx.x - b.cum[s]) * kChunk;
  const size_t c1 = c0 + kChunk < g.bytes ? c0 + kChunk : g.bytes;
  const unsigned char* src = (const unsigned char*)g.src;
  unsigned char* dst = (unsigned char*)g.dst;
  // 16-byte words when both ends are 16-byte aligned, bytes otherwise
  if ((((uintptr_t)src | (uintptr_t)dst) & 15) == 0) {
    const size_t w0 = c0 / 16, w1 = c1 / 16;
    const uint4* s4 = (const uint4*)src;
    uint4* d4 = (uint4*)dst;
    for (size_t w = w0 + threadIdx.x; w < w1; w += kCopyThreads) d4[w] = s4[w];
    for (size_t i = w1 * 16 + threadIdx.x; i < c1; i += kCopyThreads) dst[i] = src[i];
  } else {
    for (size_t i = c0 + threadIdx.x; i < c1; i += kCopyThreads) dst[i] = src[i];
  }
}

}  // namespace
}  // namespace md

extern "C" md_status md_copy_segments(const md_copy_segment* segs, int32_t n_segs, void* stream) {
  if (n_segs < 0 || (n_segs > 0 && !segs)) return MD_ERR_INVALID_ARG;
  for (int32_t k = 0; k < n_segs; ++k)
    if (segs[k].bytes > 0 && (!segs[k].dst || !segs[k].src)) return MD_ERR_INVALID_ARG;
  for (int32_t k0 = 0; k0 < n_segs; k0 += md::kSegMax) {
    md::SegBatch b;
    b.n = 0;
    b.cum[0] = 0;
    for (int32_t k = k0; k < n_segs && k < k0 + md::kSegMax; ++k) {
      if (segs[k].bytes == 0) continue;
      b.seg[b.n] = segs[k];
      b.cum[b.n + 1] = b.cum[b.n] + (int64_t)((segs[k].bytes + md::kChunk - 1) / md::kChunk);
      ++b.n;
    }
    if (b.n == 0) continue;
    hipLaunchKernelGGL(md::k_copy_segments, dim3((unsigned)b.cum[b.n]), dim3(md::kCopyThreads), 0,
                       (hipStream_t)stream, b);
    if (hipGetLastError() != hipSuccess) return MD_ERR_HIP;
  }
  return MD_OK;
}
