// hf_codebook.hip -- stages 2 and 3 (Sec. 4.2, Algorithm 1 of the paper):
// the codebook kernels and their launchers; the device code shared with the
// batched and persistent launches is in hf_codebook_dev.h.
#include "hf_codebook_dev.h"

namespace hf {

// ---------------------------------------------------------------------------
// Books of alphabets above kMultiAlphabet: the data-parallel steps over the
// whole grid.
// ---------------------------------------------------------------------------
// A lone workgroup is bound by its own memory pipeline on the scattered
// stores of the radix sort, of the leaf lengths and of the codewords (with
// 65536 used symbols about 0.82 M, 0.27 M and 0.18 M of 2.2 M cycles).  Above
// kMultiAlphabet those steps run over many workgroups, while the GenerateCL
// rounds and the depths (the sequential part of Algorithm 1) stay in one:
//  1. digit counts of radix pass 0 per block of kMB symbols, which also give
//     m and the largest count;
//  2. stable LSD radix passes of 8 bits over the count, each a count and a
//     scatter kernel; keys are count << 16 | symbol in symbol order, so
//     equal counts keep symbol order (the order of the paper's sorted
//     histogram, ties by symbol); the passes the largest count does not need
//     return at once, and the last pass lands in the tree's key array;
//  3. the rounds and the depths, one workgroup, tree in the workspace;
//  4. leaf lengths, counts per length and total bits; the last workgroup to
//     finish derives First and Entry (Sec. 4.2.2);
//  5. codewords: counts per (block, length) with offsets from the last
//     workgroup, then ranks within each length in symbol order.
// Every step returns at once when at most kCbLdsMaxUsed symbols are used:
// the single-workgroup kernel, launched last, then builds the book alone.
constexpr uint32_t kMultiAlphabet = 8192;
constexpr uint32_t kMB = 1024;    // symbols (keys) of a block
constexpr int kMT = 256;          // lanes of a block: one per digit in the scans
constexpr uint32_t kMPasses = 4;  // 8-bit digits of a 32-bit count

struct MultiState {
  uint32_t m, wmax, dsel, lmax, lminc, done_len, done_cw, pad;  // lminc = kMaxLen + 1 - lmin
  unsigned long long total;
  uint32_t cnt[kMaxLen + 1];
};

struct MultiLayout {
  size_t x, dig, st, cntw, total;
};

__host__ __device__ inline uint32_t multi_blocks(uint32_t A) { return (A + kMB - 1) / kMB; }

// After the tree's own arrays: the sort's second key buffer, the digit
// counts (digit-major), the state and the per-block length counts.
__host__ __device__ inline MultiLayout multi_layout(uint32_t A) {
  MultiLayout L;
  size_t o = global_layout(A).total;
  L.x = o;    o += align256((size_t)A * 8);
  L.dig = o;  o += align256((size_t)256 * multi_blocks(A) * 4);
  L.st = o;   o += align256(sizeof(MultiState));
  L.cntw = o; o += align256((size_t)multi_blocks(A) * (kMaxLen + 1) * 4);
  L.total = o;
  return L;
}

__device__ __forceinline__ uint32_t multi_passes(uint32_t wmax) {
  uint32_t p = 1;
  while (p < kMPasses && (wmax >> (8 * p)) != 0) ++p;
  return p;
}

// Pass p of P writes the tree's key array when P - 1 - p is even, else the
// second buffer, so the last pass ends in the key array.
__device__ __forceinline__ uint64_t* multi_dst(char* ws, uint32_t A, uint32_t P, uint32_t p) {
  return (uint64_t*)(ws + (((P - 1 - p) & 1) ? multi_layout(A).x : global_layout(A).key));
}

// The lanes of this wave whose 9-bit value equals mine.
__device__ __forceinline__ uint64_t match9(uint32_t d) {
  uint64_t eq = ~0ull;
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const bool on = (d >> q) & 1u;
    const uint64_t B = __ballot(on);
    eq &= on ? B : ~B;
  }
  return eq;
}

__global__ __launch_bounds__(kMT) void cbm_count_kernel(const uint32_t* __restrict__ hist, hf_codebook book,
                                                        char* ws, uint32_t pass) {
  const uint32_t A = book.alphabet, NB = gridDim.x, b = blockIdx.x, tid = threadIdx.x;
  MultiState* st = (MultiState*)(ws + multi_layout(A).st);
  uint32_t* dig = (uint32_t*)(ws + multi_layout(A).dig);
  __shared__ uint32_t c[256];
  uint32_t P = 1;
  if (pass > 0) {
    P = multi_passes(st->wmax);
    if (st->m <= kCbLdsMaxUsed || pass >= P) return;
  }
  c[tid] = 0;
  __syncthreads();
  const uint32_t i0 = b * kMB, i1 = min(A, i0 + kMB);
  if (pass == 0) {
    uint8_t* clu = (uint8_t*)(ws + global_layout(A).clu);
    uint32_t used = 0, hm = 0;
    for (uint32_t s = i0 + tid; s < i1; s += kMT) {
      const uint32_t h = hist[s];
      atomicAdd(&c[h & 255u], 1u);
      used += h != 0;
      hm = max(hm, h);
      if (!h) {  // unused symbols: no code
        book.cl[s] = 0;
        book.cw[s] = 0;
        clu[s] = 0;
      }
    }
    used = (uint32_t)wave_sum_u64(used);
    hm = wave_max_u32(hm);
    if (lane_id() == 0) {
      atomicAdd(&st->m, used);
      atomicMax(&st->wmax, hm);
    }
  } else {
    const uint64_t* src = multi_dst(ws, A, P, pass - 1);
    const uint32_t shift = 16 + 8 * pass;
    for (uint32_t s = i0 + tid; s < i1; s += kMT) atomicAdd(&c[(uint32_t)(src[s] >> shift) & 255u], 1u);
  }
  __syncthreads();
  dig[tid * NB + b] = c[tid];
}

// Block b places its kMB keys: digit d starts at the keys of smaller digits
// in every block plus the keys of digit d in earlier blocks; inside the
// block wave w owns keys [256 w, 256 w + 256) in groups of 64, and a key goes
// after the equal-digit keys of earlier waves, earlier groups and earlier
// lanes (a stable sort).
__global__ __launch_bounds__(kMT) void cbm_scatter_kernel(const uint32_t* __restrict__ hist, hf_codebook book,
                                                          char* ws, uint32_t pass) {
  constexpr int NW = kMT / kWave;
  const uint32_t A = book.alphabet, NB = gridDim.x, b = blockIdx.x, tid = threadIdx.x;
  const uint32_t lane = tid & (kWave - 1), wave = tid / kWave;
  MultiState* st = (MultiState*)(ws + multi_layout(A).st);
  const uint32_t* dig = (const uint32_t*)(ws + multi_layout(A).dig);
  const uint32_t P = multi_passes(st->wmax);
  if (st->m <= kCbLdsMaxUsed || pass >= P) return;
  uint64_t* dst = multi_dst(ws, A, P, pass);
  const uint64_t* src = pass ? multi_dst(ws, A, P, pass - 1) : nullptr;
  __shared__ uint32_t wc[NW][256];
  __shared__ uint32_t wtot[NW];
  // thread d: the keys of digit d before this block, and in all blocks
  uint32_t before = 0, tot = 0;
  for (uint32_t bb = 0; bb < NB; ++bb) {
    const uint32_t v = dig[tid * NB + bb];
    tot += v;
    before += bb < b ? v : 0u;
  }
  uint32_t all;
  const uint32_t base = block_exclusive_scan<NW>(tot, wtot, &all) + before;
#pragma unroll
  for (int w = 0; w < NW; ++w) wc[w][tid] = 0;
  __syncthreads();
  const uint32_t shift = 16 + 8 * pass;
  const uint32_t g0 = b * kMB + wave * 256;
  uint64_t k[4], eq[4];
  uint32_t d[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const uint32_t i = g0 + v * kWave + lane;
    k[v] = i < A ? (pass ? src[i] : ((uint64_t)hist[i] << 16 | i)) : 0ull;
    d[v] = i < A ? (uint32_t)(k[v] >> shift) & 255u : 256u;  // 256: past the alphabet
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    eq[v] = match9(d[v]);
    if (d[v] < 256u && (eq[v] >> lane) == 1ull) wc[wave][d[v]] += (uint32_t)__popcll(eq[v]);
  }
  __syncthreads();
  {  // this digit's start in each wave
    uint32_t run = base;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      const uint32_t t = wc[w][tid];
      wc[w][tid] = run;
      run += t;
    }
  }
  __syncthreads();
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    if (d[v] < 256u) {
      const uint32_t slot = wc[wave][d[v]] + (uint32_t)__popcll(eq[v] & lanemask_lt());
      dst[slot] = k[v];
      if ((eq[v] >> lane) == 1ull) wc[wave][d[v]] = slot + 1;
    }
  }
}

// The GenerateCL rounds and the depths over the sorted used keys (the last
// m of the sorted array: unused symbols sort first).
__global__ __launch_bounds__(1024) void cbm_tree_kernel(hf_codebook book, char* ws, uint32_t* status) {
  const uint32_t A = book.alphabet;
  MultiState* st = (MultiState*)(ws + multi_layout(A).st);
  const uint32_t m = st->m;
  if (m <= kCbLdsMaxUsed) return;
  __shared__ Shared sh;
  const GlobalLayout G = global_layout(A);
  Tree<uint32_t> t;
  t.key = (uint64_t*)(ws + G.key) + (A - m);
  t.iw = (uint64_t*)(ws + G.iw);
  t.mw = (uint64_t*)(ws + G.mw);
  t.mid = (uint32_t*)(ws + G.mid);
  t.par = (uint32_t*)(ws + G.par);
  t.usym = (uint32_t*)(ws + G.usym);
  t.clu = (uint8_t*)(ws + G.clu);
  t.dA = (uint16_t*)(ws + G.dA);
  t.dB = (uint16_t*)(ws + G.dB);
  t.nA = (uint32_t*)(ws + G.nA);
  t.nB = (uint32_t*)(ws + G.nB);
  uint16_t* dc = build_book_tree<uint32_t, 1024>(t, sh, m, status);
  if (threadIdx.x == 0) st->dsel = dc == t.dA ? 0u : 1u;
}

// Leaf i (sorted order) has length depth(parent) + 1; block b takes leaves
// [b kMB, b kMB + kMB).  The last block to finish derives First (the
// canonical recurrence, ones-first) and Entry (codes of shorter lengths).
__global__ __launch_bounds__(kMT) void cbm_len_kernel(hf_codebook book, char* ws, uint32_t* status) {
  const uint32_t A = book.alphabet, b = blockIdx.x, tid = threadIdx.x, lane = tid & (kWave - 1);
  MultiState* st = (MultiState*)(ws + multi_layout(A).st);
  const uint32_t m = st->m;
  if (m <= kCbLdsMaxUsed) return;
  const GlobalLayout G = global_layout(A);
  const uint64_t* key = (const uint64_t*)(ws + G.key) + (A - m);
  const uint32_t* par = (const uint32_t*)(ws + G.par);
  const uint16_t* dc = (const uint16_t*)(ws + (st->dsel ? G.dB : G.dA));
  uint8_t* clu = (uint8_t*)(ws + G.clu);
  __shared__ uint32_t cnt[kMaxLen + 1];
  __shared__ uint32_t s_last;
  for (uint32_t l = tid; l <= kMaxLen; l += kMT) cnt[l] = 0;
  __syncthreads();
  uint64_t bits = 0;
  uint32_t my_max = 0, my_min = 0xFFFFFFFFu;
  const uint32_t i0 = b * kMB;
  uint64_t kk[4];
  uint32_t dd[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const uint32_t i = i0 + v * kMT + tid;
    kk[v] = i < m ? key[i] : 0ull;
    dd[v] = i < m ? (uint32_t)dc[par[i]] : 0u;
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const bool valid = i0 + v * kMT + tid < m;
    uint32_t l = 0;
    if (valid) {
      l = dd[v] + 1;
      bits += (kk[v] >> 16) * l;
      my_max = max(my_max, l);
      my_min = min(my_min, l);
      if (l > kMaxLen) l = kMaxLen;  // flagged below; keeps indexes in range
      const uint32_t s = (uint32_t)(kk[v] & 0xFFFFu);
      clu[s] = (uint8_t)l;
      book.cl[s] = (uint8_t)l;
    }
    count_lengths(l, valid, cnt);
  }
  bits = wave_sum_u64(bits);
  my_max = wave_max_u32(my_max);
#pragma unroll
  for (int dlt = kWave / 2; dlt > 0; dlt >>= 1) my_min = min(my_min, (uint32_t)__shfl_xor(my_min, dlt, kWave));
  if (lane == 0 && my_max) {
    atomicAdd(&st->total, (unsigned long long)bits);
    atomicMax(&st->lmax, my_max);
    atomicMax(&st->lminc, kMaxLen + 1 - min(my_min, kMaxLen));
  }
  __syncthreads();
  for (uint32_t l = tid; l <= kMaxLen; l += kMT)
    if (cnt[l]) atomicAdd(&st->cnt[l], cnt[l]);
  __threadfence();
  __syncthreads();
  if (tid == 0) s_last = atomicAdd(&st->done_len, 1u) == gridDim.x - 1;
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  if (tid < kWave) {  // wave 0: lane j holds length j + 1
    const uint32_t lmax = __hip_atomic_load(&st->lmax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t L = lmax > kMaxLen ? kMaxLen : lmax;
    const uint32_t c = __hip_atomic_load(&st->cnt[lane + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t below = wave_inclusive_scan(c) - c;  // codes shorter than lane + 1
    uint64_t f = 0, mine = 0;
    for (int l = (int)L - 1; l >= 1; --l) {
      f = (f + (uint32_t)__builtin_amdgcn_readlane((int)c, l) + 1) >> 1;  // cnt[l + 1]
      if ((int)lane == l - 1) mine = f;
    }
    book.first[lane + 1] = mine;
    book.entry[lane + 1] = below;
    if (lane == 0) {
      book.first[0] = 0;
      book.entry[0] = 0;
      if (lmax > kMaxLen) raise_status(status, HF_ERR_CODELEN);
      book.info[0] = m;
      book.info[1] = lmax;
      book.info[2] = __hip_atomic_load(&st->total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      book.info[3] = kMaxLen + 1 - __hip_atomic_load(&st->lminc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// Codewords, pass 1: used symbols per length in block b (symbols [b kMB,
// b kMB + kMB)); the last block turns the counts into each block's first
// rank per length: Entry[l] plus the codes of length l in earlier blocks.
__global__ __launch_bounds__(kMT) void cbm_cwcount_kernel(hf_codebook book, char* ws) {
  const uint32_t A = book.alphabet, NB = gridDim.x, b = blockIdx.x, tid = threadIdx.x;
  MultiState* st = (MultiState*)(ws + multi_layout(A).st);
  if (st->m <= kCbLdsMaxUsed) return;
  const uint8_t* clu = (const uint8_t*)(ws + global_layout(A).clu);
  uint32_t* cntw = (uint32_t*)(ws + multi_layout(A).cntw);
  __shared__ uint32_t cnt[kMaxLen + 1];
  __shared__ uint32_t s_last;
  for (uint32_t l = tid; l <= kMaxLen; l += kMT) cnt[l] = 0;
  __syncthreads();
  uint32_t lv[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const uint32_t s = b * kMB + v * kMT + tid;
    lv[v] = s < A ? (uint32_t)clu[s] : 0u;
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) count_lengths(lv[v], lv[v] != 0, cnt);
  __syncthreads();
  for (uint32_t l = tid; l <= kMaxLen; l += kMT) cntw[b * (kMaxLen + 1) + l] = cnt[l];
  __threadfence();
  __syncthreads();
  if (tid == 0) s_last = atomicAdd(&st->done_cw, 1u) == gridDim.x - 1;
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  if (tid >= 1 && tid <= kMaxLen) {
    uint32_t run = book.entry[tid];
    for (uint32_t bb = 0; bb < NB; ++bb) {
      uint32_t* q = &cntw[bb * (kMaxLen + 1) + tid];
      const uint32_t c = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      *q = run;
      run += c;
    }
  }
}

// Codewords, pass 2: wave w of block b takes symbols [b kMB + 256 w, +256)
// in groups of 64; a used symbol's rank within its length is the block's
// first rank, plus the same-length symbols of earlier waves, groups and
// lanes.  rev[rank] = symbol, cw = First[l] + rank - Entry[l].
__global__ __launch_bounds__(kMT) void cbm_cw_kernel(hf_codebook book, char* ws) {
  constexpr int NW = kMT / kWave;
  const uint32_t A = book.alphabet, b = blockIdx.x, tid = threadIdx.x;
  const uint32_t lane = tid & (kWave - 1), wave = tid / kWave;
  MultiState* st = (MultiState*)(ws + multi_layout(A).st);
  if (st->m <= kCbLdsMaxUsed) return;
  const uint8_t* clu = (const uint8_t*)(ws + global_layout(A).clu);
  const uint32_t* cntw = (const uint32_t*)(ws + multi_layout(A).cntw);
  __shared__ uint32_t wc[NW][kMaxLen + 1];
  __shared__ uint64_t s_first[kMaxLen + 1];
  __shared__ uint32_t s_entry[kMaxLen + 1];
  for (uint32_t l = tid; l <= kMaxLen; l += kMT) {
    s_first[l] = book.first[l];
    s_entry[l] = book.entry[l];
    for (int w = 0; w < NW; ++w) wc[w][l] = 0;
  }
  __syncthreads();
  const uint32_t g0 = b * kMB + wave * 256;
  uint32_t lv[4];
  uint64_t eq[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const uint32_t s = g0 + v * kWave + lane;
    lv[v] = s < A ? (uint32_t)clu[s] : 0u;
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    eq[v] = match9(lv[v]);
    if (lv[v] && (eq[v] >> lane) == 1ull) wc[wave][lv[v]] += (uint32_t)__popcll(eq[v]);
  }
  __syncthreads();
  if (tid >= 1 && tid <= kMaxLen) {
    uint32_t run = cntw[b * (kMaxLen + 1) + tid];
    for (int w = 0; w < NW; ++w) {
      const uint32_t t = wc[w][tid];
      wc[w][tid] = run;
      run += t;
    }
  }
  __syncthreads();
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const uint32_t l = lv[v];
    if (l) {
      const uint32_t s = g0 + v * kWave + lane;
      const uint32_t pos = wc[wave][l] + (uint32_t)__popcll(eq[v] & lanemask_lt());
      book.rev[pos] = s;
      book.cw[s] = s_first[l] + (pos - s_entry[l]);
      if ((eq[v] >> lane) == 1ull) wc[wave][l] = pos + 1;
    }
  }
}

// The single-workgroup build: every book of an alphabet up to
// kMultiAlphabet, and above it the books of at most kCbLdsMaxUsed used
// symbols (multi: the grid-wide steps' state, or null).
template <int NT>
__global__ __launch_bounds__(NT) void codebook_kernel(const uint32_t* __restrict__ hist, hf_codebook book,
                                                      char* ws, uint32_t* status, const MultiState* multi) {
  if (multi && multi->m > kCbLdsMaxUsed) return;  // built by the grid-wide steps
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
  if (alphabet <= tree_cap) return 0;
  return alphabet > kMultiAlphabet ? multi_layout(alphabet).total : global_layout(alphabet).total;
}

hipError_t launch_codebook(const uint32_t* hist, const hf_codebook& book, void* ws, size_t ws_bytes,
                           uint32_t* status, hipStream_t stream, const KernelTimer& timer) {
  (void)ws_bytes;
  const uint32_t A = book.alphabet;
  char* w = (char*)ws;
  hipError_t e = hipSuccess;
  timer.before(stream);
  if (A > kMultiAlphabet) {
    const MultiLayout M = multi_layout(A);
    const uint32_t NB = multi_blocks(A);
    e = launch_fill_u32((uint32_t*)(w + M.st), sizeof(MultiState) / 4, 0u, stream);
    for (uint32_t p = 0; p < kMPasses && e == hipSuccess; ++p) {
      cbm_count_kernel<<<NB, kMT, 0, stream>>>(hist, book, w, p);
      cbm_scatter_kernel<<<NB, kMT, 0, stream>>>(hist, book, w, p);
      e = hipGetLastError();
    }
    if (e == hipSuccess) {
      cbm_tree_kernel<<<1, 1024, 0, stream>>>(book, w, status);
      cbm_len_kernel<<<NB, kMT, 0, stream>>>(book, w, status);
      cbm_cwcount_kernel<<<NB, kMT, 0, stream>>>(book, w);
      cbm_cw_kernel<<<NB, kMT, 0, stream>>>(book, w);
      codebook_kernel<1024><<<1, 1024, 0, stream>>>(hist, book, w, status, (const MultiState*)(w + M.st));
      e = hipGetLastError();
    }
  } else {
    codebook_kernel<1024><<<1, 1024, 0, stream>>>(hist, book, w, status, nullptr);
    e = hipGetLastError();
  }
  timer.after(stream);
  return e;
}

}  // namespace hf
