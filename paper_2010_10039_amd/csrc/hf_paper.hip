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
// them into word and side-channel offsets (and checking capacities); a
// workgroup scan of the groups' lengths, the words ORed into an LDS image of
// the chunk, and whole words copied out.  A workgroup takes a tile of 4096
// symbols (8192 at r = 5), one or more whole chunks.
#include <algorithm>

#include "hf_device.h"
#include "hf_kernels.h"

namespace hf {

namespace {

constexpr int kPfThreads = 256;
constexpr int kPfWaves = kPfThreads / kWave;
constexpr int kScanThreads = 1024;
constexpr int kScanPer = 8;    // chunks per scan thread
constexpr int kPfMaxChunks = 32;  // chunks per tile: 2^(13 - 8)
constexpr uint32_t kPfBlocksPerCu = 32;  // measured: 8 a CU 224 us, 16 200 us, 32 198 us (M = 10, r = 2)

// A workgroup takes a tile of 2^TL symbols, TL = max(12, 8 + R): every
// thread holds 16 (or, at R = 5, 32) consecutive symbols, pf_per groups,
// all in one chunk, and the tile holds 2^(TL - M) whole chunks.
template <int R>
constexpr uint32_t pf_tile_log2() {
  return R < 5 ? 12u : 13u;
}
template <int R>
constexpr int pf_per() {
  return 1 << (pf_tile_log2<R>() - 8 - R);
}

// Merged words of this thread's NS = PER G symbols starting at `first`, of
// which the first `rem` are its own (FULL: all of them): right-aligned code
// bits, valid while len <= 32; `bad` is set by a symbol outside the alphabet
// or without a code.  All symbol loads and table lookups are issued before
// any merge, so they are in flight together; a partial thread clamps its
// loads into the stream and masks what lies past `rem`.  A code that enters
// a word has at most 32 bits, so only the low half of its 64-bit codeword is
// read: cw32[2 s] from the book, or tab[s] from the workgroup's LDS copy
// (TAB); and while a word fits, its bits so far and the next code fit in 32
// bits (a 32-bit code comes only into an empty word).
template <int SB, int R, int PER, bool TAB, bool FULL>
__device__ __forceinline__ void words_body(const void* sym, uint64_t n, uint64_t first, uint32_t rem,
                                           const uint8_t* cl, const uint32_t* cw32, uint32_t A,
                                           uint32_t (&word)[PER], uint32_t (&len)[PER], uint32_t (&s)[PER << R],
                                           bool& bad) {
  constexpr int G = 1 << R, NS = PER * G;
  uint32_t l[NS], c[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) s[i] = FULL ? sym_at<SB>(sym, first + i) : sym_at<SB>(sym, std::min<uint64_t>(first + i, n - 1));
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const uint32_t t = s[i] < A ? s[i] : 0u;
    l[i] = s[i] < A ? (uint32_t)cl[t] : 0u;
    c[i] = cw32[TAB ? t : 2 * t];
  }
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    uint32_t acc = 0, L = 0;
#pragma unroll
    for (int i = j * G; i < (j + 1) * G; ++i) {
      const bool in = FULL || (uint32_t)i < rem;
      const uint32_t li = in ? l[i] : 0u;
      bad |= in && li == 0;
      acc = in && L + li <= 32 ? (acc << (li & 31)) | c[i] : acc;
      L += li;
    }
    word[j] = acc;
    len[j] = L;
  }
#pragma unroll
  for (int i = 0; i < NS; ++i) s[i] = FULL || (uint32_t)i < rem ? s[i] : 0u;
}

// This thread's groups [ga, gb) of the chunk whose symbols end at hi; the
// symbols are returned too (0 past the thread's own).
template <int SB, int R, int PER, bool TAB>
__device__ __forceinline__ void thread_words(const void* sym, uint64_t n, uint64_t lo, uint64_t hi, uint32_t ga,
                                             uint32_t gb, const uint8_t* cl, const uint32_t* cw32, uint32_t A,
                                             uint32_t (&word)[PER], uint32_t (&len)[PER], uint32_t (&syms)[PER << R],
                                             bool& bad) {
  constexpr uint32_t NS = PER << R;
  const uint64_t first = lo + ((uint64_t)ga << R);
  const uint64_t end = std::min<uint64_t>(hi, lo + ((uint64_t)gb << R));
  const uint32_t rem = end > first ? (uint32_t)std::min<uint64_t>(end - first, NS) : 0u;
  if (rem == NS) words_body<SB, R, PER, TAB, true>(sym, n, first, rem, cl, cw32, A, word, len, syms, bad);
  else words_body<SB, R, PER, TAB, false>(sym, n, first, rem, cl, cw32, A, word, len, syms, bad);
}

struct PfArgs {
  const void* sym;
  uint64_t n;
  const uint8_t* cl;
  const uint32_t* cw32;  // the book's 64-bit codewords, read as 32-bit halves
  uint32_t A;
  uint32_t M;
  uint64_t nch;
  uint32_t* chunk_bits;  // ws
  uint32_t* chunk_brk;   // ws
  uint32_t* tile_w;      // ws: per tile, its chunks' words
  uint32_t* tile_b;      // ws: per tile, its breaking groups
  uint64_t* tile_off_w;  // ws: [ntiles + 1], exclusive scan of tile_w
  uint64_t* tile_off_b;  // ws: [ntiles + 1], exclusive scan of tile_b
  uint64_t ntiles;
  uint64_t* offsets;     // out: chunk word offsets [nch + 1]
  uint32_t* out;
  uint64_t cap_words;
  uint64_t* brk_groups;
  void* brk_syms;
  uint64_t brk_cap;
  uint64_t* nbreak;
  uint32_t* status;
};

// This thread's chunk in the tile (c-th of the tile, k in all, nch or more
// for none) and its groups [ga, gb) of that chunk.
template <int R>
__device__ __forceinline__ void pf_thread_groups(const PfArgs& a, uint64_t tile, uint32_t& c, uint64_t& k,
                                                 uint64_t& lo, uint64_t& hi, uint32_t& ga, uint32_t& gb) {
  constexpr uint32_t TL = pf_tile_log2<R>();
  const uint32_t tid = threadIdx.x, tpc = a.M + 8 - TL;  // log2 threads per chunk
  c = tid >> tpc;
  k = (tile << (TL - a.M)) + c;
  ga = gb = 0;
  lo = hi = 0;
  if (k >= a.nch) return;
  lo = k << a.M;
  hi = std::min<uint64_t>(a.n, lo + (1ull << a.M));
  const uint32_t ng = (uint32_t)((hi - lo + (1u << R) - 1) >> R);
  ga = std::min(ng, (tid & ((1u << tpc) - 1)) * (uint32_t)pf_per<R>());
  gb = std::min(ng, ga + (uint32_t)pf_per<R>());
}

// The workgroup's copy of the book when the alphabet has at most
// kPfTabAlphabet symbols: the codewords' low halves, then the lengths.
constexpr uint32_t kPfTabAlphabet = 4096;
extern __shared__ uint32_t pf_tab[];

__host__ __device__ inline uint32_t pf_tab_bytes(uint32_t A) { return (A * 5 + 3) & ~3u; }

template <bool TAB>
__device__ __forceinline__ void pf_stage_book(const PfArgs& a, const uint8_t*& cl, const uint32_t*& cw) {
  cl = a.cl;
  cw = a.cw32;
  if (!TAB) return;
  uint8_t* tcl = (uint8_t*)(pf_tab + a.A);
#pragma unroll 4
  for (uint32_t i = threadIdx.x; i < a.A; i += kPfThreads) {
    pf_tab[i] = a.cw32[2 * i];
    tcl[i] = a.cl[i];
  }
  __syncthreads();
  cl = tcl;
  cw = pf_tab;
}

// Each workgroup stages the book once and loops over tiles.
template <int SB, int R, bool TAB>
__global__ __launch_bounds__(kPfThreads) void pf_count_kernel(PfArgs a) {
  const uint64_t ntiles = a.ntiles;
  constexpr uint32_t TL = pf_tile_log2<R>();
  constexpr int PER = pf_per<R>();
  __shared__ uint32_t sacc[kPfMaxChunks];  // per chunk: breaking groups << 20 | bits
  const uint8_t* cl;
  const uint32_t* cw;
  pf_stage_book<TAB>(a, cl, cw);
  const uint32_t cpw = 1u << (TL - a.M), tid = threadIdx.x;
  bool bad = false;
  for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    if (tid < cpw) sacc[tid] = 0;
    __syncthreads();
    uint32_t c, ga, gb;
    uint64_t k, lo, hi;
    pf_thread_groups<R>(a, tile, c, k, lo, hi, ga, gb);
    uint32_t word[PER], len[PER], syms[PER << R];
    thread_words<SB, R, PER, TAB>(a.sym, a.n, lo, hi, ga, gb, cl, cw, a.A, word, len, syms, bad);
    uint32_t bits = 0, brk = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      brk += len[j] > 32;
      bits += len[j] > 32 ? 0u : len[j];
    }
    // a chunk's bits <= 2^16 and breaking groups <= 2^11: one packed sum over
    // the lanes of the chunk (a power of two up to the whole wave)
    uint32_t v = (brk << 20) | bits;
    const uint32_t width = std::min(1u << (a.M + 8 - TL), (uint32_t)kWave);
    if (width == kWave) {  // the wave lies in one chunk: DPP sum, total in the last lane
      v = wave_inclusive_scan(v);
      if (lane_id() == kWave - 1 && k < a.nch) atomicAdd(&sacc[c], v);
    } else {
      for (uint32_t o = 1; o < width; o <<= 1) v += __shfl_xor(v, (int)o);
      if ((lane_id() & (width - 1)) == 0 && k < a.nch) atomicAdd(&sacc[c], v);
    }
    __syncthreads();
    const uint64_t kt = (tile << (TL - a.M)) + tid;
    if (tid < kWave) {  // wave 0: the chunks' counts and the tile's totals
      const uint32_t sv = tid < cpw && kt < a.nch ? sacc[tid] : 0u;
      if (tid < cpw && kt < a.nch) {
        a.chunk_bits[kt] = sv & 0xFFFFFu;
        a.chunk_brk[kt] = sv >> 20;
      }
      // a tile's words <= 2^11 + 32 and breaking groups <= 2^11: one packed DPP sum
      const uint32_t t = wave_inclusive_scan((sv >> 20) << 16 | (((sv & 0xFFFFFu) + 31) / 32));
      if (tid == kWave - 1) {
        a.tile_w[tile] = t & 0xFFFFu;
        a.tile_b[tile] = t >> 16;
      }
    }
  }
  if (bad) raise_status(a.status, HF_ERR_SYMBOL);
}

// tile_off_w[t] = sum over tiles j < t of their words (each chunk's
// ceil(bits / 32)), tile_off_b likewise for the breaking groups; totals at
// [ntiles], and the stream's total words also at offsets[nch].  One
// workgroup, kScanPer consecutive tiles a thread.  Loads and stores go
// through LDS so that both are coalesced: a tile's words (at most 2^11 plus
// one a chunk) and breaking groups (at most 2^11) are packed into one word,
// brk << 16 | words, and so are the in-thread exclusive prefixes (at most 7
// tiles, < 2^16 each).
__global__ __launch_bounds__(kScanThreads) void pf_scan_kernel(PfArgs a) {
  constexpr uint32_t T = kScanThreads * kScanPer;  // chunks an iteration
  __shared__ uint32_t pk[T];
  __shared__ uint32_t base_w[kScanThreads], base_b[kScanThreads];
  __shared__ uint32_t wtot[kScanThreads / kWave];
  __shared__ uint64_t carry_w, carry_b;
  const uint32_t tid = threadIdx.x;
  if (tid == 0) carry_w = carry_b = 0;
  for (uint64_t base = 0; base < a.ntiles; base += T) {
#pragma unroll
    for (uint32_t i = tid; i < T; i += kScanThreads) {
      const uint64_t k = base + i;
      pk[i] = k < a.ntiles ? (a.tile_b[k] << 16) | a.tile_w[k] : 0u;
    }
    __syncthreads();
    uint32_t v[kScanPer], sw = 0, sb = 0;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
      v[j] = pk[tid * kScanPer + j];
      sw += v[j] & 0xFFFFu;
      sb += v[j] >> 16;
    }
    uint32_t tw, tb;
    const uint32_t pw = block_exclusive_scan<kScanThreads / kWave>(sw, wtot, &tw);
    __syncthreads();
    const uint32_t pb = block_exclusive_scan<kScanThreads / kWave>(sb, wtot, &tb);
    base_w[tid] = pw;
    base_b[tid] = pb;
    uint32_t run = 0;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
      pk[tid * kScanPer + j] = run;
      run += v[j];
    }
    __syncthreads();
    const uint64_t cw = carry_w, cb = carry_b;
#pragma unroll
    for (uint32_t i = tid; i < T; i += kScanThreads) {
      const uint64_t k = base + i;
      if (k < a.ntiles) {
        const uint32_t o = i / kScanPer, p = pk[i];
        a.tile_off_w[k] = cw + base_w[o] + (p & 0xFFFFu);
        a.tile_off_b[k] = cb + base_b[o] + (p >> 16);
      }
    }
    __syncthreads();
    if (tid == 0) {
      carry_w += tw;
      carry_b += tb;
    }
  }
  __syncthreads();
  if (tid == 0) {
    a.offsets[a.nch] = carry_w;
    a.tile_off_w[a.ntiles] = carry_w;
    a.tile_off_b[a.ntiles] = carry_b;
    a.nbreak[0] = carry_b;
    if (carry_w > a.cap_words || carry_b > a.brk_cap) raise_status(a.status, HF_ERR_CAPACITY);
  }
}

// The workgroup's chunks are consecutive in the output, so their words form
// one LDS image: a group's word has at most 32 bits (and two symbols at
// least), so a tile holds at most 2^11 words plus one of padding a chunk.
template <int SB, int R, bool TAB>
__global__ __launch_bounds__(kPfThreads) void pf_write_kernel(PfArgs a) {
  const uint64_t ntiles = a.ntiles;
  constexpr int PER = pf_per<R>();
  constexpr uint32_t G = 1u << R, TL = pf_tile_log2<R>();
  __shared__ uint32_t img[(1u << 11) + kPfMaxChunks];
  __shared__ uint32_t wtot[kPfWaves];
  __shared__ uint32_t cstart[kPfMaxChunks];  // each chunk's first bit in the tile's packed scan
  __shared__ uint32_t coff[kPfMaxChunks];    // each chunk's first word in the tile
  const uint8_t* cl;
  const uint32_t* cw;
  pf_stage_book<TAB>(a, cl, cw);
  const uint32_t tid = threadIdx.x;
  const bool fits = a.offsets[a.nch] <= a.cap_words;
  bool bad = false;
  for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const uint64_t k0 = tile << (TL - a.M);
    const uint64_t w0 = a.tile_off_w[tile];
    const uint32_t nw = (uint32_t)(a.tile_off_w[tile + 1] - w0);
    for (uint32_t i = tid; i < nw; i += kPfThreads) img[i] = 0;
    if (tid < kWave) {  // wave 0: the chunks' word offsets (in the tile and in the stream) and first bits
      const uint64_t kk = k0 + tid;
      const bool own = tid < (1u << (TL - a.M)) && kk < a.nch;
      const uint32_t b = own ? a.chunk_bits[kk] : 0u;
      const uint32_t w = (b + 31) / 32;
      const uint32_t x = wave_inclusive_scan(w) - w;
      const uint32_t y = wave_inclusive_scan(b) - b;  // a tile's bits <= 2^16
      if (own) {
        coff[tid] = x;
        cstart[tid] = y;
        a.offsets[kk] = w0 + x;
      }
    }
    uint32_t c, ga, gb;
    uint64_t k, lo, hi;
    pf_thread_groups<R>(a, tile, c, k, lo, hi, ga, gb);
    uint32_t word[PER], len[PER], syms[PER << R];
    thread_words<SB, R, PER, TAB>(a.sym, a.n, lo, hi, ga, gb, cl, cw, a.A, word, len, syms, bad);
    uint32_t bits = 0, brk = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      brk += len[j] > 32;
      bits += len[j] > 32 ? 0u : len[j];
    }
    uint32_t tot;
    // a tile's bits <= 2^16, breaking groups <= 2^11: one packed scan
    // (its barrier also publishes wave 0's coff and cstart, and the cleared image)
    const uint32_t pre = block_exclusive_scan<kPfWaves>((brk << 20) | bits, wtot, &tot);
    uint32_t pos = 0;  // the chunk's bits before this thread's: the tile's, less the earlier chunks'
    if (k < a.nch) pos = coff[c] * 32 + ((pre & 0xFFFFFu) - cstart[c]);
    uint64_t bpos = a.tile_off_b[tile] + (pre >> 20);
    const uint64_t gbase = lo >> R;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const uint32_t g = ga + j;
      if (g >= gb) break;
      const uint32_t L = len[j];
      if (L > 32) {
        if (bpos < a.brk_cap) {
          a.brk_groups[bpos] = gbase + g;
#pragma unroll
          for (uint32_t i = 0; i < G; ++i) {  // the group's symbols, 0 past the stream's end
            const uint32_t s = syms[j * G + i];
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
    __syncthreads();
    if (fits)
      for (uint32_t i = tid; i < nw; i += kPfThreads) a.out[w0 + i] = img[i];
    __syncthreads();  // the image, cstart and coff are rewritten by the next tile
  }
  if (bad) raise_status(a.status, HF_ERR_SYMBOL);
}

template <int SB, int R>
void launch_pf_r(bool write, const PfArgs& a, uint32_t nblk, hipStream_t stream) {
  if (a.A <= kPfTabAlphabet) {
    const uint32_t lds = pf_tab_bytes(a.A);
    if (write) pf_write_kernel<SB, R, true><<<nblk, kPfThreads, lds, stream>>>(a);
    else pf_count_kernel<SB, R, true><<<nblk, kPfThreads, lds, stream>>>(a);
  } else {
    if (write) pf_write_kernel<SB, R, false><<<nblk, kPfThreads, 0, stream>>>(a);
    else pf_count_kernel<SB, R, false><<<nblk, kPfThreads, 0, stream>>>(a);
  }
}

template <int SB>
void launch_pf(bool write, const PfArgs& a, uint32_t r, uint32_t nblk, hipStream_t stream) {
  switch (r) {
    case 1: launch_pf_r<SB, 1>(write, a, nblk, stream); break;
    case 2: launch_pf_r<SB, 2>(write, a, nblk, stream); break;
    case 3: launch_pf_r<SB, 3>(write, a, nblk, stream); break;
    case 4: launch_pf_r<SB, 4>(write, a, nblk, stream); break;
    default: launch_pf_r<SB, 5>(write, a, nblk, stream); break;
  }
}

}  // namespace

// Chunk counts (bits, breaking groups), tile totals, and the tiles' two
// exclusive scans; a tile holds at least one chunk, so nch bounds the tiles.
size_t paper_workspace_bytes(uint64_t n, uint32_t chunk_log2) {
  const uint64_t nch = (n + (1ull << chunk_log2) - 1) >> chunk_log2;
  return 2 * ((size_t)(nch * 8 + 255) / 256 * 256) + 2 * ((size_t)((nch + 1) * 8 + 255) / 256 * 256);
}

hipError_t launch_encode_paper(const void* sym, uint64_t n, uint32_t sym_bytes, const hf_codebook& book,
                               uint32_t M, uint32_t r, uint32_t* out, uint64_t cap_words, uint64_t* offsets,
                               uint64_t* brk_groups, void* brk_syms, uint64_t brk_cap, uint64_t* nbreak, void* ws,
                               uint32_t* status, uint32_t cus, hipStream_t stream, const KernelTimer& timer) {
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
  a.cw32 = (const uint32_t*)book.cw;
  a.A = book.alphabet;
  a.M = M;
  a.nch = nch;
  a.chunk_bits = (uint32_t*)ws;
  a.chunk_brk = a.chunk_bits + nch;
  const size_t pair_bytes = (size_t)(nch * 8 + 255) / 256 * 256, scan_bytes = (size_t)((nch + 1) * 8 + 255) / 256 * 256;
  a.tile_w = (uint32_t*)((char*)ws + pair_bytes);
  a.tile_b = a.tile_w + nch;
  a.tile_off_w = (uint64_t*)((char*)ws + 2 * pair_bytes);
  a.tile_off_b = (uint64_t*)((char*)ws + 2 * pair_bytes + scan_bytes);
  a.offsets = offsets;
  a.out = out;
  a.cap_words = cap_words;
  a.brk_groups = brk_groups;
  a.brk_syms = brk_syms;
  a.brk_cap = brk_cap;
  a.nbreak = nbreak;
  a.status = status;
  const uint32_t cl2 = (r < 5 ? 12u : 13u) - M;  // chunks per tile, log2 (pf_tile_log2)
  const uint64_t ntiles = (nch + (1u << cl2) - 1) >> cl2;
  a.ntiles = ntiles;
  // workgroups loop over tiles, a few tiles each, so that the last of them end close together
  const uint32_t nblk = (uint32_t)std::min<uint64_t>(ntiles, (uint64_t)cus * kPfBlocksPerCu);
  timer.before(stream);
  if (sym_bytes == 1) launch_pf<1>(false, a, r, nblk, stream);
  else launch_pf<2>(false, a, r, nblk, stream);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  pf_scan_kernel<<<1, kScanThreads, 0, stream>>>(a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (sym_bytes == 1) launch_pf<1>(true, a, r, nblk, stream);
  else launch_pf<2>(true, a, r, nblk, stream);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  timer.after(stream);
  return hipSuccess;
}

}  // namespace hf
