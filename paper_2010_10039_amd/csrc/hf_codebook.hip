// hf_codebook.hip -- stages 2 and 3 (Sec. 4.2, Algorithm 1 of the paper):
// the codebook kernels and their launchers; the device code is in
// hf_codebook_dev.h.
#include "hf_codebook_dev.h"

namespace hf {

template <int NT>
__global__ __launch_bounds__(NT) void codebook_kernel(const uint32_t* __restrict__ hist, hf_codebook book,
                                                      char* ws, uint32_t* status) {
  __shared__ CbLds lds;
  codebook_block<NT>(hist, book, ws, status, lds);
}

// Batched stage 3: workgroup s builds stream s's book from its histogram
// (an empty stream's histogram is zeroed here and its one offset set).
constexpr int kBatchCbThreads = 256;

__global__ __launch_bounds__(kBatchCbThreads) void batch_codebook_kernel(const BatchStream* __restrict__ streams) {
  __shared__ CbLds lds;
  batch_codebook_item<kBatchCbThreads>(streams[blockIdx.x], lds);
}

hipError_t launch_batch_codebook(const BatchStream* d_streams, uint32_t nstreams, hipStream_t stream) {
  batch_codebook_kernel<<<nstreams, kBatchCbThreads, 0, stream>>>(d_streams);
  return hipGetLastError();
}

size_t codebook_workspace_bytes(uint32_t alphabet, uint32_t tree_cap) {
  return alphabet > tree_cap ? global_layout(alphabet).total : 0;
}

hipError_t launch_codebook(const uint32_t* hist, const hf_codebook& book, void* ws, size_t ws_bytes,
                           uint32_t* status, hipStream_t stream, const KernelTimer& timer) {
  (void)ws_bytes;
  timer.before(stream);
  codebook_kernel<1024><<<1, 1024, 0, stream>>>(hist, book, (char*)ws, status);
  hipError_t e = hipGetLastError();
  timer.after(stream);
  return e;
}

}  // namespace hf
