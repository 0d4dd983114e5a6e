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
  // Window: two 4-word blocks in registers, cur (words wb .. wb + 3) and nxt
  // (the next four, loaded when cur was entered, so a refill waits on a
  // load issued some twenty symbols earlier); the next bit is bit sh of
  // word wb + idx, idx < 4.
  auto load = [&](uint64_t j) -> uint32_t { return j < nwords ? words[j] : 0u; };
  uint64_t wb = (offsets[k] >> 5) & ~3ull;
  uint32_t idx = (uint32_t)((offsets[k] >> 5) & 3);
  uint32_t sh = (uint32_t)(offsets[k] & 31);
  uint32_t c0 = load(wb), c1 = load(wb + 1), c2 = load(wb + 2), c3 = load(wb + 3);
  uint32_t n0 = load(wb + 4), n1 = load(wb + 5), n2 = load(wb + 6), n3 = load(wb + 7);
  bool bad = false;
  // Symbols go out 16 bytes at a time (G per group; a chunk starts at a
  // multiple of 256 symbols) when the output is 16-byte aligned, the ragged
  // end of a chunk one by one.
  constexpr uint32_t G = 16 / SB;
  const bool vec = ((uintptr_t)out & 15) == 0;
  uint32_t packed[4];
  uint64_t i = i0;
  while (i < i1 && !bad) {
    const uint32_t cnt = i1 - i >= G ? G : (uint32_t)(i1 - i);
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) packed[q] = 0;
#pragma unroll
    for (uint32_t g = 0; g < G; ++g) {
      if (g < cnt && !bad) {
        const uint32_t w0 = idx == 0 ? c0 : idx == 1 ? c1 : idx == 2 ? c2 : c3;
        const uint32_t w1 = idx == 0 ? c1 : idx == 1 ? c2 : idx == 2 ? c3 : n0;
        const uint64_t win = ((((uint64_t)w0) << 32) | w1) << sh;  // at least 33 valid bits on top
        const uint32_t t = tab[(uint32_t)(win >> (64 - kDecPeek))];
        uint32_t len = t >> 16, sym = t & 0xFFFFu;
        if (len == 0) {
          // a code over kDecPeek bits (or none): lengthen over the next 64 bits
          const uint32_t w2 = idx == 0 ? c2 : idx == 1 ? c3 : idx == 2 ? n0 : n1;
          const uint64_t w64 = win | (sh ? (uint64_t)w2 >> (32 - sh) : 0ull);
          uint64_t v = 0;
          uint32_t l = 0;
          do {
            v = 2 * v + ((w64 >> (63 - l)) & 1u);
            ++l;
          } while (l < lmax && v < s_first[l]);
          if (v < s_first[l] || v - s_first[l] >= (uint64_t)(s_entry[l + 1] - s_entry[l])) {
            bad = true;
            len = 0;
          } else {
            sym = rev[s_entry[l] + (uint32_t)(v - s_first[l])];
            len = l;
          }
        }
        packed[(g * SB) / 4] |= sym << (8 * ((g * SB) % 4));
        sh += len;
        while (sh >= 32) {
          sh -= 32;
          if (++idx == 4) {
            idx = 0;
            c0 = n0;
            c1 = n1;
            c2 = n2;
            c3 = n3;
            wb += 4;
            n0 = load(wb + 4);
            n1 = load(wb + 5);
            n2 = load(wb + 6);
            n3 = load(wb + 7);
          }
        }
      }
    }
    if (vec && cnt == G && !bad) {
      *(uint4*)((char*)out + i * SB) = make_uint4(packed[0], packed[1], packed[2], packed[3]);
    } else {
      for (uint32_t g = 0; g < cnt; ++g) {
        const uint32_t sym = (packed[(g * SB) / 4] >> (8 * ((g * SB) % 4))) & (SB == 1 ? 0xFFu : 0xFFFFu);
        if (SB == 1) ((uint8_t*)out)[i + g] = (uint8_t)sym;
        else ((uint16_t*)out)[i + g] = (uint16_t)sym;
      }
    }
    i += cnt;
  }
  const uint64_t wi = wb + idx;
  if (bad || wi * 32 + sh != stop) raise_status(status, HF_ERR_STREAM);
}

}  // namespace

size_t decode_workspace_bytes() { return (size_t)4 << kDecPeek; }

hipError_t launch_decode(const uint32_t* words, const uint64_t* offsets, uint64_t n, uint32_t sym_bytes,
                         uint32_t chunk_log2, const hf_codebook& book, void* out, void* ws, uint32_t* status,
                         hipStream_t stream, const KernelTimer& timer) {
  if (n == 0) {
    timer.before(stream);
    timer.after(stream);
    return hipSuccess;
  }
  uint32_t* tab = (uint32_t*)ws;
  decode_table_kernel<<<(1u << kDecPeek) / 256, 256, 0, stream>>>(book.first, book.entry, book.rev, book.info, tab);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const uint64_t nchunks = (n + (1ull << chunk_log2) - 1) >> chunk_log2;
  const uint32_t grid = (uint32_t)((nchunks + kDecLanes - 1) / kDecLanes);
  timer.before(stream);
  if (sym_bytes == 1)
    decode_kernel<1><<<grid, kDecLanes, 0, stream>>>(words, offsets, n, chunk_log2, nchunks, tab, book.first,
                                                     book.entry, book.rev, book.info, out, status);
  else
    decode_kernel<2><<<grid, kDecLanes, 0, stream>>>(words, offsets, n, chunk_log2, nchunks, tab, book.first,
                                                     book.entry, book.rev, book.info, out, status);
  e = hipGetLastError();
  timer.after(stream);
  return e;
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
