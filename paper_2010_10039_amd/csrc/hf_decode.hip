// hf_decode.hip -- checker: chunk-parallel treeless canonical decoding with
// the First / Entry / reverse-codebook tables (Sec. 4.2.2 of the paper;
// Table 1, "get reverse codebook"), compared symbol by symbol with the
// input.  One lane decodes one chunk from its recorded bit offset.
#include "hf_device.h"
#include "hf_kernels.h"

namespace hf {

namespace {

constexpr int kDecThreads = 256;

__device__ __forceinline__ uint32_t get_bit(const uint32_t* __restrict__ w, uint64_t p) {
  return (w[p >> 5] >> (31 - (p & 31))) & 1u;
}

template <int SB>
__global__ __launch_bounds__(kDecThreads) void decode_check_kernel(
    const uint32_t* __restrict__ words, const uint64_t* __restrict__ offsets, uint64_t n,
    uint32_t chunk_log2, uint64_t nchunks, const uint64_t* __restrict__ first,
    const uint32_t* __restrict__ entry, const uint32_t* __restrict__ rev,
    const uint64_t* __restrict__ info, const void* __restrict__ expected,
    unsigned long long* __restrict__ result, uint32_t* __restrict__ status) {
  __shared__ uint64_t s_first[HF_MAX_CODELEN + 2];
  __shared__ uint32_t s_entry[HF_MAX_CODELEN + 2];
  const uint32_t m = (uint32_t)info[0];
  const uint32_t lmax = (uint32_t)(info[1] < HF_MAX_CODELEN ? info[1] : HF_MAX_CODELEN);
  for (uint32_t l = threadIdx.x; l <= HF_MAX_CODELEN; l += blockDim.x) {
    s_first[l] = first[l];
    s_entry[l] = entry[l];
  }
  if (threadIdx.x == 0) s_entry[HF_MAX_CODELEN + 1] = m;
  __syncthreads();

  const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nchunks) return;
  const uint64_t total = offsets[nchunks];
  uint64_t p = offsets[k];
  const uint64_t stop = offsets[k + 1];
  const uint64_t i0 = k << chunk_log2;
  const uint64_t i1 = min(n, i0 + (1ull << chunk_log2));
  unsigned long long bad = 0;
  uint64_t first_bad = n;
  uint64_t i = i0;
  for (; i < i1; ++i) {
    const uint32_t want = SB == 1 ? (uint32_t)((const uint8_t*)expected)[i]
                                  : (uint32_t)((const uint16_t*)expected)[i];
    bool ok = p < total;
    uint32_t got = 0xFFFFFFFFu;
    if (ok) {
      uint64_t v = get_bit(words, p++);
      uint32_t l = 1;
      while (l <= lmax && v < s_first[l] && p < total) {
        v = 2 * v + get_bit(words, p++);
        ++l;
      }
      ok = l <= lmax && v >= s_first[l] && (v - s_first[l]) < (uint64_t)(s_entry[l + 1] - s_entry[l]);
      if (ok) got = rev[s_entry[l] + (uint32_t)(v - s_first[l])];
    }
    if (!ok || got != want) {
      ++bad;
      if (first_bad == n) first_bad = i;
      if (!ok) break;  // lost synchronisation: the rest of the chunk is not checked
    }
  }
  if (i < i1) {
    bad += (i1 - i) - 1;  // symbols after the break count as mismatches too
  }
  if (p != stop) {
    ++bad;
    if (first_bad == n) first_bad = i1 > 0 ? i1 - 1 : 0;
  }
  if (bad) {
    atomicAdd(&result[0], bad);
    atomicMin(&result[1], (unsigned long long)first_bad);
    raise_status(status, HF_ERR_MISMATCH);
  }
}

}  // namespace

hipError_t launch_decode_check(const uint32_t* words, const uint64_t* offsets, uint64_t n,
                               uint32_t sym_bytes, uint32_t chunk_log2, const hf_codebook& book,
                               const void* expected, uint64_t* result, uint32_t* status,
                               hipStream_t stream) {
  hipError_t e = launch_fill_u64(result, 1, 0, stream);
  if (e == hipSuccess) e = launch_fill_u64(result + 1, 1, n, stream);
  if (e != hipSuccess || n == 0) return e;
  const uint64_t nchunks = (n + (1ull << chunk_log2) - 1) >> chunk_log2;
  const uint32_t grid = (uint32_t)((nchunks + kDecThreads - 1) / kDecThreads);
  if (sym_bytes == 1)
    decode_check_kernel<1><<<grid, kDecThreads, 0, stream>>>(
        words, offsets, n, chunk_log2, nchunks, book.first, book.entry, book.rev, book.info, expected,
        (unsigned long long*)result, status);
  else
    decode_check_kernel<2><<<grid, kDecThreads, 0, stream>>>(
        words, offsets, n, chunk_log2, nchunks, book.first, book.entry, book.rev, book.info, expected,
        (unsigned long long*)result, status);
  return hipGetLastError();
}

}  // namespace hf
