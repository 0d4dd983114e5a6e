// hf_histogram.hip -- stage 1, histogramming (Sec. 4.1 of the paper).
//
// The paper builds on Gomez-Luna et al.: every thread block keeps private
// replicated sub-histograms in shared memory, updates them with atomics, and
// the block results are merged into one global histogram.  On gfx950:
//  - each workgroup reads one contiguous slab of the input with 16-byte
//    vector loads (several in flight per lane), so HBM sees long streams;
//  - R replicas of the bin window live in LDS one after another, a stride
//    of 1 mod 32 words apart, lane l updating replica l % R, so lanes of
//    different replicas hitting the same bin land on different banks;
//  - at the end every non-zero bin is added to the global histogram with
//    one global atomic, so peaked data costs a few hundred atomics per
//    workgroup, not one per bin;
//  - a bin window [lo, lo + W) lets alphabets too large for LDS run in
//    several passes over the input.
#include <algorithm>

#include "hf_hist_dev.h"

namespace hf {

__global__ void fill_u32_kernel(uint32_t* __restrict__ p, uint64_t count, uint32_t value) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < count; i += (uint64_t)gridDim.x * blockDim.x) p[i] = value;
}

__global__ void fill_u64_kernel(uint64_t* __restrict__ p, uint64_t count, uint64_t value) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < count; i += (uint64_t)gridDim.x * blockDim.x) p[i] = value;
}

// One launch counts bins [lo, lo + W).  Workgroup w takes the contiguous
// slabs [w*S/G, (w+1)*S/G); with slab_hist it stores each slab's counts
// (differences of the running LDS totals, so the LDS is never cleared in
// between) and, at the end, adds its totals to the global histogram.
// With slab_hist the global histogram is left to hist_reduce_kernel (this
// launch only zeroes it, from workgroup 0); otherwise every workgroup adds
// its totals to it with one atomic per non-zero bin.
template <int SB>
__global__ __launch_bounds__(kHistThreads) void histogram_kernel(
    const void* __restrict__ sym, uint64_t n, uint32_t A, uint32_t lo, uint32_t W, uint32_t R,
    uint32_t nslabs, uint64_t nblocks, uint32_t* __restrict__ hist, uint32_t* __restrict__ slab_hist,
    uint32_t* __restrict__ status) {
  extern __shared__ uint32_t sub[];
  const uint32_t tid = threadIdx.x;
  const bool all = lo == 0 && W == A;
  for (uint32_t i = tid; i < hist_window_words(W, A, R); i += blockDim.x) sub[i] = 0;
  if (slab_hist && blockIdx.x == 0)
    for (uint32_t b = tid; b < A; b += blockDim.x) hist[b] = 0;
  __syncthreads();

  const uint32_t Wp = hist_stride(W, A);
  uint32_t* const subr = sub + (tid & (R - 1)) * Wp;
  bool bad = false;
  const uint64_t g0 = (uint64_t)blockIdx.x * nslabs / gridDim.x;
  const uint64_t g1 = (uint64_t)(blockIdx.x + 1) * nslabs / gridDim.x;
  uint32_t prev[kSlabHistMaxAlphabet / kHistThreads];
#pragma unroll
  for (int k = 0; k < (int)(kSlabHistMaxAlphabet / kHistThreads); ++k) prev[k] = 0;
  for (uint64_t g = g0; g < g1; ++g) {
    const uint64_t s_lo = slab_begin(g, nblocks, nslabs, n);
    const uint64_t s_hi = slab_begin(g + 1, nblocks, nslabs, n);
    if (all) hist_range<SB, true>(subr, sym, s_lo, s_hi, lo, W, A, bad);
    else hist_range<SB, false>(subr, sym, s_lo, s_hi, lo, W, A, bad);
    if (slab_hist) {
      __syncthreads();
#pragma unroll
      for (int k = 0; k < (int)(kSlabHistMaxAlphabet / kHistThreads); ++k) {
        const uint32_t b = tid + k * kHistThreads;
        if (b < W) {
          uint32_t c = 0;
          for (uint32_t r = 0; r < R; ++r) c += sub[r * Wp + b];
          slab_hist[g * A + lo + b] = c - prev[k];
          prev[k] = c;
        }
      }
      __syncthreads();
    }
  }
  if (!slab_hist) {
    __syncthreads();
    for (uint32_t b = tid; b < W; b += blockDim.x) {
      uint32_t c = 0;
      for (uint32_t r = 0; r < R; ++r) c += sub[r * Wp + b];
      if (c) atomicAdd(&hist[lo + b], c);
    }
  }
  if (all) {
    __syncthreads();
    if (tid < R && sub[tid * Wp + A]) bad = true;
  }
  if (bad) raise_status(status, HF_ERR_SYMBOL);
}

// hist[b] += sum of rows [r0, r0 + kReduceRows) of the per-slab counts:
// coalesced row reads, one atomic per non-zero bin and workgroup.
constexpr uint32_t kReduceRows = 16;

__global__ __launch_bounds__(kHistThreads) void hist_reduce_kernel(const uint32_t* __restrict__ part,
                                                                   uint32_t nrows, uint32_t A,
                                                                   uint32_t* __restrict__ hist) {
  const uint32_t r0 = blockIdx.x * kReduceRows;
  const uint32_t r1 = min(nrows, r0 + kReduceRows);
  for (uint32_t b = threadIdx.x; b < A; b += blockDim.x) {
    uint32_t c = 0;
#pragma unroll 8
    for (uint32_t r = r0; r < r1; ++r) c += part[(uint64_t)r * A + b];
    if (c) atomicAdd(&hist[b], c);
  }
}

hipError_t launch_slab_hist_reduce(const uint32_t* slab_hist, uint32_t nslabs, uint32_t A, uint32_t* hist,
                                   hipStream_t stream) {
  hist_reduce_kernel<<<(nslabs + kReduceRows - 1) / kReduceRows, kHistThreads, 0, stream>>>(slab_hist, nslabs, A,
                                                                                            hist);
  return hipGetLastError();
}

// Batched stage 1: workgroup i counts the slab of work item items[i].
__global__ __launch_bounds__(kHistThreads) void batch_histogram_kernel(const BatchStream* __restrict__ streams,
                                                                       const uint32_t* __restrict__ item_stream,
                                                                       const uint32_t* __restrict__ items,
                                                                       uint32_t lds_words) {
  extern __shared__ uint32_t sub[];
  const uint32_t item = items[blockIdx.x];
  const BatchStream& bs = streams[item_stream[item]];
  batch_hist_item(bs, item - bs.item0, sub, lds_words);
}

// Batched stage 2: workgroup i sums bin chunk (items[i] & 63) of stream
// items[i] >> 6.
__global__ __launch_bounds__(kBatchReduceBins) void batch_hist_reduce_kernel(const BatchStream* __restrict__ streams,
                                                                             const uint32_t* __restrict__ items) {
  const uint32_t item = items[blockIdx.x];
  batch_reduce_item(streams[item >> 6], item & 63);
}

hipError_t launch_batch_hist_reduce(const BatchStream* d_streams, const uint32_t* d_red_items, uint32_t nred,
                                    hipStream_t stream) {
  if (nred == 0) return hipSuccess;
  batch_hist_reduce_kernel<<<nred, kBatchReduceBins, 0, stream>>>(d_streams, d_red_items);
  return hipGetLastError();
}

// Two replicas of the largest alphabet (more for smaller ones): peaked
// streams put many lanes on one bin, and every replica splits them.
uint32_t batch_hist_lds_words(uint32_t max_alphabet) {
  return std::max<uint32_t>(4096u, 2 * max_alphabet) + 64u;
}

hipError_t launch_batch_histogram(const BatchStream* d_streams, const uint32_t* d_item_stream,
                                  const uint32_t* d_items, uint32_t nitems, uint32_t lds_words,
                                  hipStream_t stream) {
  if (nitems == 0) return hipSuccess;
  const size_t lds = (size_t)lds_words * 4;
  if (lds > (64u << 10))
    (void)hipFuncSetAttribute((const void*)batch_histogram_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  batch_histogram_kernel<<<nitems, kHistThreads, lds, stream>>>(d_streams, d_item_stream, d_items, lds_words);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint64_t count, uint32_t value, hipStream_t stream) {
  if (count == 0) return hipSuccess;
  uint32_t blocks = (uint32_t)std::min<uint64_t>(1024, (count + 255) / 256);
  fill_u32_kernel<<<blocks, 256, 0, stream>>>(p, count, value);
  return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t* p, uint64_t count, uint64_t value, hipStream_t stream) {
  if (count == 0) return hipSuccess;
  uint32_t blocks = (uint32_t)std::min<uint64_t>(1024, (count + 255) / 256);
  fill_u64_kernel<<<blocks, 256, 0, stream>>>(p, count, value);
  return hipGetLastError();
}

// LDS per workgroup: up to 32 KiB of replicated window (four 4-wave
// workgroups per CU, the default slab count's occupancy).  Eight replicas of
// a 1024-bin alphabet measured 128 -> 82 us on a stream of three popular
// symbols and the same (LDS atomic issue bound) on the Lorenzo codes.
// Alphabets whose single copy needs more use one copy of up to 32768 bins
// (128 KiB) and several passes for larger alphabets.
static void hist_plan(uint32_t A, uint32_t* W, uint32_t* R) {
  const uint32_t budget = (32u << 10) + 512u;  // 32 KiB plus the trash bins and stride padding
  if (hist_stride(A, A) * 4u <= budget) {
    uint32_t r = 1;
    while (r < 16 && hist_stride(A, A) * 4u * (r * 2) <= budget) r *= 2;
    *W = A;
    *R = r;
  } else {
    *W = A < 32768u ? A : 32768u;
    *R = 1;
  }
}

uint32_t histogram_internal_slabs(uint64_t n, uint32_t alphabet, int num_cus) {
  if (alphabet > kSlabHistMaxAlphabet) return 0;
  const uint64_t nblocks = (n + kSlabBlock - 1) / kSlabBlock;
  uint64_t s = std::min<uint64_t>((uint64_t)num_cus * 8, (nblocks + 3) / 4);
  if (s > kMaxInternalSlabs) s = kMaxInternalSlabs;
  return (uint32_t)(s > 0 ? s : 1);
}

hipError_t launch_histogram(const void* sym, uint64_t n, uint32_t sym_bytes, uint32_t A,
                            uint32_t* hist, uint32_t nslabs, uint32_t* slab_hist, uint32_t* ws,
                            size_t ws_bytes, uint32_t* status, int num_cus, hipStream_t stream,
                            const KernelTimer& timer) {
  uint32_t W, R;
  hist_plan(A, &W, &R);
  const size_t lds = (size_t)hist_window_words(W, A, R) * sizeof(uint32_t);
  const uint64_t nblocks = (n + kSlabBlock - 1) / kSlabBlock;
  hipError_t e;
  if (!slab_hist && A <= kSlabHistMaxAlphabet) {
    // per-slab counts into the workspace when it has room
    const uint32_t s = histogram_internal_slabs(n, A, num_cus);
    if (ws && (size_t)s * A * sizeof(uint32_t) <= ws_bytes) {
      slab_hist = ws;
      nslabs = s;
    }
  }
  uint64_t grid;
  if (slab_hist) {
    grid = nslabs;  // one slab per workgroup
  } else {
    e = launch_fill_u32(hist, A, 0u, stream);
    if (e != hipSuccess) return e;
    const uint64_t wgs_per_cu = std::max<uint64_t>(1, std::min<uint64_t>(8, (160u << 10) / lds));
    grid = std::min<uint64_t>((uint64_t)num_cus * wgs_per_cu, (nblocks + 3) / 4);
    if (grid < 1) grid = 1;
    nslabs = (uint32_t)grid;
  }
  if (lds > (64u << 10)) {
    (void)hipFuncSetAttribute((const void*)histogram_kernel<1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipFuncSetAttribute((const void*)histogram_kernel<2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  }
  timer.before(stream);
  for (uint32_t lo = 0; lo < A; lo += W) {
    const uint32_t w = std::min(W, A - lo);
    if (sym_bytes == 1)
      histogram_kernel<1><<<(uint32_t)grid, kHistThreads, lds, stream>>>(sym, n, A, lo, w, R, nslabs, nblocks, hist,
                                                                         slab_hist, status);
    else
      histogram_kernel<2><<<(uint32_t)grid, kHistThreads, lds, stream>>>(sym, n, A, lo, w, R, nslabs, nblocks, hist,
                                                                         slab_hist, status);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  timer.after(stream);
  if (slab_hist) {
    hist_reduce_kernel<<<(nslabs + kReduceRows - 1) / kReduceRows, kHistThreads, 0, stream>>>(slab_hist, nslabs, A,
                                                                                              hist);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace hf
