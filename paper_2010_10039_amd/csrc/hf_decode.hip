// hf_decode.hip -- chunk-parallel treeless canonical decoding with the
// First / Entry / reverse-codebook tables (Sec. 4.2.2 of the paper; Table 1,
// "get reverse codebook").  One lane decodes one chunk from its recorded bit
// offset.  The checker compares the decoded symbols with the input; the
// decoder writes them out, resolving codes of up to kDecPeek bits with one
// lookup in an LDS table of every kDecPeek-bit prefix.
#include "hf_device.h"
#include "hf_kernels.h"

namespace hf {

namespace {

constexpr int kDecThreads = 256;
constexpr uint32_t kDecPeek = 12;  // bits resolved by one table lookup
constexpr int kDecLanes = 64;      // decoder workgroup: one wave, one chunk per lane

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

// Prefix table: entry p (a kDecPeek-bit window, MSB first) holds
// (code length << 16 | symbol) when a code of at most kDecPeek bits starts
// the window, else 0.  By the canonical rule a code of length l is the
// first l bits v with First[l] <= v < First[l] + (Entry[l + 1] - Entry[l]),
// found by lengthening l while v < First[l].
__global__ __launch_bounds__(256) void decode_table_kernel(const uint64_t* __restrict__ first,
                                                           const uint32_t* __restrict__ entry,
                                                           const uint32_t* __restrict__ rev,
                                                           const uint64_t* __restrict__ info,
                                                           uint32_t* __restrict__ tab) {
  const uint32_t p = blockIdx.x * 256u + threadIdx.x;
  if (p >= (1u << kDecPeek)) return;
  const uint32_t m = (uint32_t)info[0];
  const uint32_t lmax = (uint32_t)(info[1] < HF_MAX_CODELEN ? info[1] : HF_MAX_CODELEN);
  const uint32_t L = lmax < kDecPeek ? lmax : kDecPeek;
  uint32_t out = 0;
  if (m > 0 && L > 0) {
    uint32_t l = 1;
    uint64_t v = p >> (kDecPeek - 1);
    while (l < L && v < first[l]) {
      ++l;
      v = p >> (kDecPeek - l);
    }
    const uint64_t cnt = (uint64_t)((l < HF_MAX_CODELEN ? entry[l + 1] : m) - entry[l]);
    if (v >= first[l] && v - first[l] < cnt) out = (l << 16) | rev[entry[l] + (uint32_t)(v - first[l])];
  }
  tab[p] = out;
}

template <int SB>
__global__ __launch_bounds__(kDecLanes) void decode_kernel(
    const uint32_t* __restrict__ words, const uint64_t* __restrict__ offsets, uint64_t n,
    uint32_t chunk_log2, uint64_t nchunks, const uint32_t* __restrict__ gtab,
    const uint64_t* __restrict__ first, const uint32_t* __restrict__ entry,
    const uint32_t* __restrict__ rev, const uint64_t* __restrict__ info, void* __restrict__ out,
    uint32_t* __restrict__ status) {
  __shared__ uint4 tab4[(1u << kDecPeek) / 4];
  __shared__ uint64_t s_first[HF_MAX_CODELEN + 2];
  __shared__ uint32_t s_entry[HF_MAX_CODELEN + 2];
  const uint32_t tid = threadIdx.x;
  for (uint32_t i = tid; i < (1u << kDecPeek) / 4; i += kDecLanes) tab4[i] = ((const uint4*)gtab)[i];
  const uint32_t m = (uint32_t)info[0];
  const uint32_t lmax = (uint32_t)(info[1] < HF_MAX_CODELEN ? info[1] : HF_MAX_CODELEN);
  for (uint32_t l = tid; l <= HF_MAX_CODELEN; l += kDecLanes) {
    s_first[l] = first[l];
    s_entry[l] = entry[l];
  }
  if (tid == 0) s_entry[HF_MAX_CODELEN + 1] = m;
  __syncthreads();
  const uint32_t* tab = (const uint32_t*)tab4;

  const uint64_t k = (uint64_t)blockIdx.x * kDecLanes + tid;
  if (k >= nchunks) return;
  const uint64_t nwords = (offsets[nchunks] + 31) >> 5;
  const uint64_t stop = offsets[k + 1];
  const uint64_t i0 = k << chunk_log2;
  const uint64_t i1 = min(n, i0 + (1ull << chunk_log2));
  // 64-bit window: words wi and wi + 1, the next bit at offset sh in it
  uint64_t wi = offsets[k] >> 5;
  uint32_t sh = (uint32_t)(offsets[k] & 31);
  uint32_t w0 = wi < nwords ? words[wi] : 0u;
  uint32_t w1 = wi + 1 < nwords ? words[wi + 1] : 0u;
  bool bad = false;
  for (uint64_t i = i0; i < i1; ++i) {
    const uint64_t win = ((((uint64_t)w0) << 32) | w1) << sh;  // at least 33 valid bits on top
    const uint32_t t = tab[(uint32_t)(win >> (64 - kDecPeek))];
    uint32_t len = t >> 16, sym = t & 0xFFFFu;
    if (len == 0) {
      // a code over kDecPeek bits (or none): lengthen bit by bit from memory
      uint64_t q = wi * 32 + sh;
      uint64_t v = 0;
      uint32_t l = 0;
      do {
        v = 2 * v + (q < nwords * 32 ? (words[q >> 5] >> (31 - (q & 31))) & 1u : 0u);
        ++q;
        ++l;
      } while (l < lmax && v < s_first[l]);
      if (l == 0 || v < s_first[l] || v - s_first[l] >= (uint64_t)(s_entry[l + 1] - s_entry[l])) {
        bad = true;
        break;
      }
      sym = rev[s_entry[l] + (uint32_t)(v - s_first[l])];
      len = l;
    }
    if (SB == 1) ((uint8_t*)out)[i] = (uint8_t)sym;
    else ((uint16_t*)out)[i] = (uint16_t)sym;
    sh += len;
    while (sh >= 32) {
      w0 = w1;
      ++wi;
      w1 = wi + 1 < nwords ? words[wi + 1] : 0u;
      sh -= 32;
    }
  }
  if (bad || wi * 32 + sh != stop) raise_status(status, HF_ERR_STREAM);
}

}  // namespace

size_t decode_workspace_bytes() { return (size_t)4 << kDecPeek; }

hipError_t launch_decode(const uint32_t* words, const uint64_t* offsets, uint64_t n, uint32_t sym_bytes,
                         uint32_t chunk_log2, const hf_codebook& book, void* out, void* ws, uint32_t* status,
                         hipStream_t stream) {
  if (n == 0) return hipSuccess;
  uint32_t* tab = (uint32_t*)ws;
  decode_table_kernel<<<(1u << kDecPeek) / 256, 256, 0, stream>>>(book.first, book.entry, book.rev, book.info, tab);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const uint64_t nchunks = (n + (1ull << chunk_log2) - 1) >> chunk_log2;
  const uint32_t grid = (uint32_t)((nchunks + kDecLanes - 1) / kDecLanes);
  if (sym_bytes == 1)
    decode_kernel<1><<<grid, kDecLanes, 0, stream>>>(words, offsets, n, chunk_log2, nchunks, tab, book.first,
                                                     book.entry, book.rev, book.info, out, status);
  else
    decode_kernel<2><<<grid, kDecLanes, 0, stream>>>(words, offsets, n, chunk_log2, nchunks, tab, book.first,
                                                     book.entry, book.rev, book.info, out, status);
  return hipGetLastError();
}

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
