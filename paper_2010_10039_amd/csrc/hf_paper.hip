// hf_paper.hip -- the paper's own encoding format, as an ablation beside the
// exact dense encoder (Sec. 4.3, Interface ReduceShuffleMerge<M, r>;
// Sec. 5.2.2 and Table 3).
//
// Chunks of C = 2^M symbols, groups of G = 2^r symbols.  A group's codes are
// merged into one 32-bit word (the r rounds of reduce-merge); a group whose
// codes need more than 32 bits is "breaking": it leaves the stream and goes
// to a sparse side channel (global group index and raw symbols, ascending).
// A chunk's non-breaking words are concatenated (shuffle-merge) and padded to
// a whole 32-bit word; chunks follow one another word-aligned.
//
// Three launches: per-chunk bit and breaking counts; one workgroup scanning
// them into word and side-channel offsets (and checking capacities); per
// chunk, a workgroup scan of its groups' lengths, the words ORed into an LDS
// image of the chunk, and whole words copied out.
#include <algorithm>

#include "hf_device.h"
#include "hf_kernels.h"

namespace hf {

namespace {

constexpr int kPfThreads = 256;
constexpr int kPfWaves = kPfThreads / kWave;
constexpr int kPfMaxPer = 8;  // groups per thread: 2^(12 - 1) groups / 256 threads
constexpr int kScanThreads = 1024;

// Merged word of the group [g0, g1): right-aligned code bits, valid while
// len <= 32; `bad` is set by a symbol outside the alphabet or without a code.
template <int SB>
__device__ __forceinline__ void group_word(const void* sym, uint64_t g0, uint64_t g1, const uint8_t* cl,
                                           const uint64_t* cw, uint32_t A, uint32_t& word, uint32_t& len,
                                           bool& bad) {
  uint64_t acc = 0;
  uint32_t L = 0;
  for (uint64_t i = g0; i < g1; ++i) {
    const uint32_t s = sym_at<SB>(sym, i);
    const uint32_t l = s < A ? cl[s] : 0u;
    bad |= l == 0;
    if (L + l <= 32) acc = (acc << l) | cw[s < A ? s : 0];
    L += l;
  }
  word = (uint32_t)acc;
  len = L;
}

struct PfArgs {
  const void* sym;
  uint64_t n;
  const uint8_t* cl;
  const uint64_t* cw;
  uint32_t A;
  uint32_t M;
  uint32_t r;
  uint64_t nch;
  uint32_t* chunk_bits;  // ws
  uint32_t* chunk_brk;   // ws
  uint64_t* brk_off;     // ws: [nch + 1]
  uint64_t* offsets;     // out: chunk word offsets [nch + 1]
  uint32_t* out;
  uint64_t cap_words;
  uint64_t* brk_groups;
  void* brk_syms;
  uint64_t brk_cap;
  uint64_t* nbreak;
  uint32_t* status;
};

template <int SB>
__global__ __launch_bounds__(kPfThreads) void pf_count_kernel(PfArgs a) {
  __shared__ uint32_t sbits, sbrk;
  if (threadIdx.x == 0) sbits = sbrk = 0;
  __syncthreads();
  const uint64_t k = blockIdx.x;
  const uint64_t lo = k << a.M;
  const uint64_t hi = std::min<uint64_t>(a.n, lo + (1ull << a.M));
  const uint32_t G = 1u << a.r;
  const uint32_t ng = (uint32_t)((hi - lo + G - 1) >> a.r);
  uint32_t bits = 0, brk = 0;
  bool bad = false;
  for (uint32_t g = threadIdx.x; g < ng; g += kPfThreads) {
    const uint64_t g0 = lo + ((uint64_t)g << a.r);
    uint32_t w, L;
    group_word<SB>(a.sym, g0, std::min<uint64_t>(hi, g0 + G), a.cl, a.cw, a.A, w, L, bad);
    if (L > 32) ++brk;
    else bits += L;
  }
  if (bad) raise_status(a.status, HF_ERR_SYMBOL);
  atomicAdd(&sbits, bits);
  atomicAdd(&sbrk, brk);
  __syncthreads();
  if (threadIdx.x == 0) {
    a.chunk_bits[k] = sbits;
    a.chunk_brk[k] = sbrk;
  }
}

// offsets[k] = sum over j < k of ceil(bits_j / 32); brk_off likewise for the
// breaking counts; totals at [nch].  One workgroup.
__global__ __launch_bounds__(kScanThreads) void pf_scan_kernel(PfArgs a) {
  __shared__ uint32_t wtot[kScanThreads / kWave];
  __shared__ uint64_t carry_w, carry_b;
  if (threadIdx.x == 0) carry_w = carry_b = 0;
  __syncthreads();
  for (uint64_t base = 0; base < a.nch; base += kScanThreads) {
    const uint64_t k = base + threadIdx.x;
    const uint32_t w = k < a.nch ? (a.chunk_bits[k] + 31) / 32 : 0u;
    const uint32_t b = k < a.nch ? a.chunk_brk[k] : 0u;
    uint32_t tw, tb;
    const uint32_t pw = block_exclusive_scan<kScanThreads / kWave>(w, wtot, &tw);
    __syncthreads();
    const uint32_t pb = block_exclusive_scan<kScanThreads / kWave>(b, wtot, &tb);
    if (k < a.nch) {
      a.offsets[k] = carry_w + pw;
      a.brk_off[k] = carry_b + pb;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      carry_w += tw;
      carry_b += tb;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    a.offsets[a.nch] = carry_w;
    a.brk_off[a.nch] = carry_b;
    a.nbreak[0] = carry_b;
    if (carry_w > a.cap_words || carry_b > a.brk_cap) raise_status(a.status, HF_ERR_CAPACITY);
  }
}

template <int SB>
__global__ __launch_bounds__(kPfThreads) void pf_write_kernel(PfArgs a) {
  __shared__ uint32_t img[1u << 12];  // the chunk's words, at most one per symbol
  __shared__ uint32_t wtot[kPfWaves];
  const uint64_t k = blockIdx.x;
  const uint64_t lo = k << a.M;
  const uint64_t hi = std::min<uint64_t>(a.n, lo + (1ull << a.M));
  const uint32_t G = 1u << a.r;
  const uint32_t ng = (uint32_t)((hi - lo + G - 1) >> a.r);
  const uint64_t w0 = a.offsets[k];
  const uint32_t nw = (uint32_t)(a.offsets[k + 1] - w0);
  for (uint32_t i = threadIdx.x; i < nw; i += kPfThreads) img[i] = 0;
  // contiguous groups per thread, so a workgroup scan gives every group's place
  const uint32_t per = (ng + kPfThreads - 1) / kPfThreads;
  const uint32_t ga = std::min(ng, threadIdx.x * per);
  const uint32_t gb = std::min(ng, ga + per);
  uint32_t word[kPfMaxPer], len[kPfMaxPer];
  uint32_t bits = 0, brk = 0;
  bool bad = false;
#pragma unroll
  for (int j = 0; j < kPfMaxPer; ++j) {
    len[j] = 0;
    word[j] = 0;
    const uint32_t g = ga + j;
    if (g < gb) {
      const uint64_t g0 = lo + ((uint64_t)g << a.r);
      group_word<SB>(a.sym, g0, std::min<uint64_t>(hi, g0 + G), a.cl, a.cw, a.A, word[j], len[j], bad);
      if (len[j] > 32) ++brk;
      else bits += len[j];
    }
  }
  uint32_t tot;
  // bits of a chunk < 2^18, breaking groups < 2^12: one packed scan
  const uint32_t pre = block_exclusive_scan<kPfWaves>((brk << 20) | bits, wtot, &tot);
  uint32_t pos = pre & 0xFFFFFu;
  uint64_t bpos = a.brk_off[k] + (pre >> 20);
  const uint64_t gbase = lo >> a.r;
  const bool fits = a.offsets[a.nch] <= a.cap_words;
#pragma unroll
  for (int j = 0; j < kPfMaxPer; ++j) {
    const uint32_t g = ga + j;
    if (g >= gb) break;
    const uint32_t L = len[j];
    if (L > 32) {
      if (bpos < a.brk_cap) {
        a.brk_groups[bpos] = gbase + g;
        const uint64_t g0 = lo + ((uint64_t)g << a.r);
        for (uint32_t i = 0; i < G; ++i) {
          const uint32_t s = g0 + i < hi ? sym_at<SB>(a.sym, g0 + i) : 0u;
          if (SB == 1) ((uint8_t*)a.brk_syms)[bpos * G + i] = (uint8_t)s;
          else ((uint16_t*)a.brk_syms)[bpos * G + i] = (uint16_t)s;
        }
      }
      ++bpos;
      continue;
    }
    const uint32_t left = L == 32 ? word[j] : word[j] << (32 - L);
    const uint32_t idx = pos >> 5, sh = pos & 31;
    atomicOr(&img[idx], left >> sh);
    if (sh + L > 32) atomicOr(&img[idx + 1], left << (32 - sh));
    pos += L;
  }
  if (bad) raise_status(a.status, HF_ERR_SYMBOL);
  __syncthreads();
  if (fits)
    for (uint32_t i = threadIdx.x; i < nw; i += kPfThreads) a.out[w0 + i] = img[i];
}

}  // namespace

size_t paper_workspace_bytes(uint64_t n, uint32_t chunk_log2) {
  const uint64_t nch = (n + (1ull << chunk_log2) - 1) >> chunk_log2;
  return (size_t)(nch * 8 + 255) / 256 * 256 + (size_t)((nch + 1) * 8 + 255) / 256 * 256;
}

hipError_t launch_encode_paper(const void* sym, uint64_t n, uint32_t sym_bytes, const hf_codebook& book,
                               uint32_t M, uint32_t r, uint32_t* out, uint64_t cap_words, uint64_t* offsets,
                               uint64_t* brk_groups, void* brk_syms, uint64_t brk_cap, uint64_t* nbreak, void* ws,
                               uint32_t* status, hipStream_t stream, const KernelTimer& timer) {
  const uint64_t nch = (n + (1ull << M) - 1) >> M;
  if (n == 0) {
    hipError_t e = launch_fill_u64(offsets, 1, 0, stream);
    if (e != hipSuccess) return e;
    return launch_fill_u64(nbreak, 1, 0, stream);
  }
  PfArgs a;
  a.sym = sym;
  a.n = n;
  a.cl = book.cl;
  a.cw = book.cw;
  a.A = book.alphabet;
  a.M = M;
  a.r = r;
  a.nch = nch;
  a.chunk_bits = (uint32_t*)ws;
  a.chunk_brk = a.chunk_bits + nch;
  a.brk_off = (uint64_t*)((char*)ws + (nch * 8 + 255) / 256 * 256);
  a.offsets = offsets;
  a.out = out;
  a.cap_words = cap_words;
  a.brk_groups = brk_groups;
  a.brk_syms = brk_syms;
  a.brk_cap = brk_cap;
  a.nbreak = nbreak;
  a.status = status;
  timer.before(stream);
  if (sym_bytes == 1) pf_count_kernel<1><<<(uint32_t)nch, kPfThreads, 0, stream>>>(a);
  else pf_count_kernel<2><<<(uint32_t)nch, kPfThreads, 0, stream>>>(a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  pf_scan_kernel<<<1, kScanThreads, 0, stream>>>(a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (sym_bytes == 1) pf_write_kernel<1><<<(uint32_t)nch, kPfThreads, 0, stream>>>(a);
  else pf_write_kernel<2><<<(uint32_t)nch, kPfThreads, 0, stream>>>(a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  timer.after(stream);
  return hipSuccess;
}

}  // namespace hf
