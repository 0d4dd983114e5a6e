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
// kMultiAlphabet those steps run over up to 64 workgroups, while the
// GenerateCL rounds and the depths (the sequential part of Algorithm 1) stay
// in one.  Three kernels after a fill of the state:
//  1. the sort: digit counts per block of kMB symbols (the first pass also
//     gives m and the largest count), a grid barrier, the stable scatter, a
//     grid barrier, for each 8-bit digit of the count the largest count
//     needs.  Keys are count << 16 | symbol in symbol order, so equal counts
//     keep symbol order (the paper's sorted histogram, ties by symbol), and
//     the last pass lands in the tree's key array;
//  2. the rounds and the depths, one workgroup, tree in the workspace;
//  3. the tail: leaf lengths, counts per length and total bits, a grid
//     barrier, First and Entry (Sec. 4.2.2, every block derives them), the
//     codes per (block, length), a grid barrier, and the codewords ranked
//     within each length in symbol order.
// Every kernel returns at once when at most kCbLdsMaxUsed symbols are used:
// the single-workgroup kernel, launched last, then builds the book alone.
// The grid barriers count arrivals in the state; all blocks of a grid this
// small are resident together, and a wait that passes its limit records
// HF_ERR_INTERNAL and goes on, so no launch can hang.
constexpr uint32_t kMultiAlphabet = 8192;
constexpr uint32_t kMB = 1024;    // symbols (keys) of a block
constexpr int kMT = 256;          // lanes of a block: one per digit in the scans
constexpr uint32_t kMPasses = 4;  // 8-bit digits of a 32-bit count
constexpr uint32_t kMaxBlocks = 65536 / kMB;  // blocks of the largest alphabet (one wave's lanes)
constexpr uint32_t kBarrierSpinLimit = 1u << 18;  // polls (0.1 - 0.3 s); a barrier takes microseconds

// Per-block slots instead of shared counters: read-modify-writes of one
// address from blocks on every XCD serialise at the coherence point.
struct MultiState {
  uint32_t flag_sort[kMaxBlocks];  // grid barriers: the last barrier each block passed
  uint32_t flag_tail[kMaxBlocks];  // (only the flags are cleared before a build)
  uint32_t m, wmax, dsel, pad;     // written by block 0 of the sort and the tree kernel
  uint32_t pm[kMaxBlocks];         // used symbols per block
  uint32_t pw[kMaxBlocks];         // largest count per block
  uint32_t plmax[kMaxBlocks];      // longest and shortest code per block of leaves
  uint32_t plmin[kMaxBlocks];      // (0xFFFFFFFF: no leaves)
  uint64_t pbits[kMaxBlocks];      // coded bits per block of leaves
  uint32_t pcnt[kMaxLen + 1][kMaxBlocks];  // codes per length per block of leaves
};
constexpr uint32_t kMultiFlagWords = 2 * kMaxBlocks;

struct MultiLayout {
  size_t x, dig, st, cntw, total;
};

__host__ __device__ inline uint32_t multi_blocks(uint32_t A) { return (A + kMB - 1) / kMB; }
// row length of a digit's counts: the blocks, rounded up for 16-byte loads
__host__ __device__ inline uint32_t multi_row(uint32_t A) { return (multi_blocks(A) + 3) & ~3u; }

// After the tree's own arrays: the sort's second key buffer, the digit
// counts (digit-major), the state and the per-block length counts.
__host__ __device__ inline MultiLayout multi_layout(uint32_t A) {
  MultiLayout L;
  size_t o = global_layout(A).total;
  L.x = o;    o += align256((size_t)A * 8);
  L.dig = o;  o += align256((size_t)256 * multi_row(A) * 4);
  L.st = o;   o += align256(sizeof(MultiState));
  L.cntw = o; o += align256((size_t)(kMaxLen + 1) * kMaxBlocks * 4);  // [length][block]
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

// Grid barrier number k (1, 2, ...) over one flag per block (zero before
// the launch): a block stores k in its flag, then wave 0 reads every flag
// at once (lane j the flag of block j) until all reach k.  Every block's
// writes before the barrier are visible to every block after it.
// The workgroup barrier first drains every wave's stores to the L2, so one
// release (an L2 write-back) and one acquire (an invalidate) per block
// suffice: a fence in every wave would flush the XCD's L2 once per wave.
__device__ __forceinline__ void grid_barrier(uint32_t* flags, uint32_t k, uint32_t* status) {
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(&flags[blockIdx.x], k, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  if (threadIdx.x < kWave) {
    const uint32_t lane = threadIdx.x;
    uint32_t spins = 0;
    for (;;) {
      // relaxed polls: an acquire per poll would invalidate the XCD's L2 each
      // time; the one acquire fence below follows the last poll
      const bool ok = lane >= gridDim.x ||
                      __hip_atomic_load(&flags[lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= k;
      if (__ballot(!ok) == 0ull) break;
      if (++spins > kBarrierSpinLimit) {
        if (lane == 0) raise_status(status, HF_ERR_INTERNAL);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

// Sum and maximum over the blocks' slots (wave 0; lane j reads block j).
__device__ __forceinline__ uint32_t slots_sum(const uint32_t* v, uint32_t nb) {
  const uint32_t lane = lane_id();
  return (uint32_t)wave_sum_u64(lane < nb ? __hip_atomic_load(&v[lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u);
}
__device__ __forceinline__ uint32_t slots_max(const uint32_t* v, uint32_t nb) {
  const uint32_t lane = lane_id();
  return wave_max_u32(lane < nb ? __hip_atomic_load(&v[lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u);
}

// Digit counts of block b's keys for pass p (pass 0 builds the keys from the
// histogram and also adds up m and the largest count).
__device__ __forceinline__ void sort_count(const uint32_t* __restrict__ hist, const hf_codebook& book, char* ws,
                                           uint32_t P, uint32_t pass, uint32_t* c) {
  const uint32_t A = book.alphabet, NB = gridDim.x, b = blockIdx.x, tid = threadIdx.x;
  MultiState* st = (MultiState*)(ws + multi_layout(A).st);
  uint32_t* dig = (uint32_t*)(ws + multi_layout(A).dig);
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
    // one slot per block
    used = (uint32_t)wave_sum_u64(used);
    hm = wave_max_u32(hm);
    __shared__ uint32_t red[2][kMT / kWave];
    if (lane_id() == 0) {
      red[0][tid / kWave] = used;
      red[1][tid / kWave] = hm;
    }
    __syncthreads();
    if (tid == 0) {
      uint32_t u = 0, x = 0;
#pragma unroll
      for (int w = 0; w < kMT / kWave; ++w) {
        u += red[0][w];
        x = max(x, red[1][w]);
      }
      st->pm[b] = u;
      st->pw[b] = x;
    }
  } else {
    const uint64_t* src = multi_dst(ws, A, P, pass - 1);
    const uint32_t shift = 16 + 8 * pass;
    for (uint32_t s = i0 + tid; s < i1; s += kMT) atomicAdd(&c[(uint32_t)(src[s] >> shift) & 255u], 1u);
  }
  __syncthreads();
  dig[tid * multi_row(A) + b] = c[tid];
  (void)NB;
}

// Block b places its kMB keys: digit d starts at the keys of smaller digits
// in every block plus the keys of digit d in earlier blocks; inside the
// block wave w owns keys [256 w, 256 w + 256) in groups of 64, and a key goes
// after the equal-digit keys of earlier waves, earlier groups and earlier
// lanes (a stable sort).
__device__ __forceinline__ void sort_scatter(const uint32_t* __restrict__ hist, const hf_codebook& book, char* ws,
                                             uint32_t P, uint32_t pass, uint32_t (*wc)[256], uint32_t* wtot) {
  constexpr int NW = kMT / kWave;
  const uint32_t A = book.alphabet, NB = gridDim.x, b = blockIdx.x, tid = threadIdx.x;
  const uint32_t lane = tid & (kWave - 1), wave = tid / kWave;
  const uint32_t* dig = (const uint32_t*)(ws + multi_layout(A).dig);
  uint64_t* dst = multi_dst(ws, A, P, pass);
  const uint64_t* src = pass ? multi_dst(ws, A, P, pass - 1) : nullptr;
  // thread d: the keys of digit d before this block, and in all blocks; the
  // counts come from blocks on other XCDs, so the row is read with 16-byte
  // loads that are all in flight together (at most 64 blocks: 16 loads)
  uint32_t before = 0, tot = 0;
  {
    const uint4* row = (const uint4*)(dig + tid * multi_row(A));
    uint4 v[kMaxBlocks / 4];
#pragma unroll
    for (uint32_t q = 0; q < kMaxBlocks / 4; ++q) v[q] = 4 * q < NB ? row[q] : make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
    for (uint32_t q = 0; q < kMaxBlocks / 4; ++q) {
      const uint32_t e[4] = {v[q].x, v[q].y, v[q].z, v[q].w};
#pragma unroll
      for (uint32_t j = 0; j < 4; ++j) {
        const uint32_t bb = 4 * q + j;
        const uint32_t x = bb < NB ? e[j] : 0u;  // the row's padding is never written
        tot += x;
        before += bb < b ? x : 0u;
      }
    }
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

__global__ __launch_bounds__(kMT) void cbm_sort_kernel(const uint32_t* __restrict__ hist, hf_codebook book,
                                                       char* ws, uint32_t* status) {
  constexpr int NW = kMT / kWave;
  __shared__ uint32_t c[256];
  __shared__ uint32_t wc[NW][256];
  __shared__ uint32_t wtot[NW];
  const uint32_t A = book.alphabet;
  MultiState* st = (MultiState*)(ws + multi_layout(A).st);
  __shared__ uint32_t s_mw[2];
  uint32_t k = 0;
  sort_count(hist, book, ws, 1, 0, c);
  grid_barrier(st->flag_sort, ++k, status);
  if (threadIdx.x < kWave) {
    const uint32_t m = slots_sum(st->pm, gridDim.x), wmax = slots_max(st->pw, gridDim.x);
    if (threadIdx.x == 0) {
      s_mw[0] = m;
      s_mw[1] = wmax;
      if (blockIdx.x == 0) {  // for the later kernels
        st->m = m;
        st->wmax = wmax;
      }
    }
  }
  __syncthreads();
  if (s_mw[0] <= kCbLdsMaxUsed) return;
  const uint32_t P = multi_passes(s_mw[1]);
  for (uint32_t p = 0; p < P; ++p) {
    if (p > 0) {
      sort_count(hist, book, ws, P, p, c);
      grid_barrier(st->flag_sort, ++k, status);
    }
    sort_scatter(hist, book, ws, P, p, wc, wtot);
    if (p + 1 < P) grid_barrier(st->flag_sort, ++k, status);
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

// The tail of the book.  Leaf i (sorted order) has length depth(parent) + 1;
// block b takes leaves [b kMB, b kMB + kMB).  After a grid barrier every
// block derives First (the canonical recurrence, ones-first) and Entry
// (codes of shorter lengths), block 0 publishes them; block b then counts
// the codes of each length among symbols [b kMB, b kMB + kMB), and after a
// second barrier ranks them: wave w takes symbols [b kMB + 256 w, +256) in
// groups of 64, and a symbol's rank within its length is Entry plus the
// same-length symbols of earlier blocks, waves, groups and lanes.
// rev[rank] = symbol, cw = First[l] + rank - Entry[l].
__global__ __launch_bounds__(kMT) void cbm_tail_kernel(hf_codebook book, char* ws, uint32_t* status) {
  constexpr int NW = kMT / kWave;
  const uint32_t A = book.alphabet, b = blockIdx.x, tid = threadIdx.x;
  const uint32_t lane = tid & (kWave - 1), wave = tid / kWave;
  MultiState* st = (MultiState*)(ws + multi_layout(A).st);
  const uint32_t m = st->m;
  if (m <= kCbLdsMaxUsed) return;
  const GlobalLayout G = global_layout(A);
  uint8_t* clu = (uint8_t*)(ws + G.clu);
  uint32_t* cntw = (uint32_t*)(ws + multi_layout(A).cntw);
  __shared__ uint32_t cnt[kMaxLen + 1];
  __shared__ uint32_t wc[NW][kMaxLen + 1];
  __shared__ uint64_t s_first[kMaxLen + 1];
  __shared__ uint32_t s_entry[kMaxLen + 1];
  for (uint32_t l = tid; l <= kMaxLen; l += kMT) cnt[l] = 0;
  __syncthreads();
  {  // lengths
    const uint64_t* key = (const uint64_t*)(ws + G.key) + (A - m);
    const uint32_t* par = (const uint32_t*)(ws + G.par);
    const uint16_t* dc = (const uint16_t*)(ws + (st->dsel ? G.dB : G.dA));
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
    __shared__ uint64_t rb[NW];
    __shared__ uint32_t rx[NW], rn[NW];
    if (lane == 0) {
      rb[wave] = bits;
      rx[wave] = my_max;
      rn[wave] = my_min;
    }
    __syncthreads();
    if (tid == 0) {  // this block's slots
      uint64_t tb = 0;
      uint32_t tx = 0, tn = 0xFFFFFFFFu;
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        tb += rb[w];
        tx = max(tx, rx[w]);
        tn = min(tn, rn[w]);
      }
      st->pbits[b] = tb;
      st->plmax[b] = tx;
      st->plmin[b] = tn;
    }
    for (uint32_t l = tid; l <= kMaxLen; l += kMT) st->pcnt[l][b] = cnt[l];
  }
  grid_barrier(st->flag_tail, 1, status);
  if (tid < kWave) {  // First and Entry; wave 0, lane j holds length j + 1
    const uint32_t nb = gridDim.x;
    const uint32_t lmax = slots_max(st->plmax, nb);
    uint32_t c = 0;
    {  // codes of length lane + 1: the row of per-block counts, 16-byte loads in flight
      const uint4* row = (const uint4*)st->pcnt[lane + 1];
      uint4 v[kMaxBlocks / 4];
#pragma unroll
      for (uint32_t q = 0; q < kMaxBlocks / 4; ++q) v[q] = 4 * q < nb ? row[q] : make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
      for (uint32_t q = 0; q < kMaxBlocks / 4; ++q) {
        c += 4 * q + 0 < nb ? v[q].x : 0u;
        c += 4 * q + 1 < nb ? v[q].y : 0u;
        c += 4 * q + 2 < nb ? v[q].z : 0u;
        c += 4 * q + 3 < nb ? v[q].w : 0u;
      }
    }
    const uint32_t L = lmax > kMaxLen ? kMaxLen : lmax;
    const uint32_t below = wave_inclusive_scan(c) - c;  // codes shorter than lane + 1
    uint64_t f = 0, mine = 0;
    for (int l = (int)L - 1; l >= 1; --l) {
      f = (f + (uint32_t)__builtin_amdgcn_readlane((int)c, l) + 1) >> 1;  // cnt[l + 1]
      if ((int)lane == l - 1) mine = f;
    }
    s_first[lane + 1] = mine;
    s_entry[lane + 1] = below;
    if (lane == 0) {
      s_first[0] = 0;
      s_entry[0] = 0;
    }
    if (b == 0) {
      const uint64_t total = wave_sum_u64(lane < nb ? st->pbits[lane] : 0ull);
      uint32_t mn = lane < nb ? st->plmin[lane] : 0xFFFFFFFFu;
#pragma unroll
      for (int dlt = kWave / 2; dlt > 0; dlt >>= 1) mn = min(mn, (uint32_t)__shfl_xor(mn, dlt, kWave));
      book.first[lane + 1] = mine;
      book.entry[lane + 1] = below;
      if (lane == 0) {
        book.first[0] = 0;
        book.entry[0] = 0;
        if (lmax > kMaxLen) raise_status(status, HF_ERR_CODELEN);
        book.info[0] = m;
        book.info[1] = lmax;
        book.info[2] = total;
        book.info[3] = mn;
      }
    }
  }
  // codes per length among this block's symbols, by wave
  for (uint32_t l = tid; l <= kMaxLen; l += kMT)
    for (int w = 0; w < NW; ++w) wc[w][l] = 0;
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
    uint32_t t = 0;
    for (int w = 0; w < NW; ++w) t += wc[w][tid];
    cntw[tid * kMaxBlocks + b] = t;
  }
  grid_barrier(st->flag_tail, 2, status);
  if (tid >= 1 && tid <= kMaxLen) {  // this block's first rank of length tid, then each wave's
    uint32_t run = s_entry[tid];
    const uint4* row = (const uint4*)(cntw + tid * kMaxBlocks);  // earlier blocks' codes, loads in flight
    uint4 v[kMaxBlocks / 4];
#pragma unroll
    for (uint32_t q = 0; q < kMaxBlocks / 4; ++q) v[q] = 4 * q < b ? row[q] : make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
    for (uint32_t q = 0; q < kMaxBlocks / 4; ++q) {
      run += 4 * q + 0 < b ? v[q].x : 0u;
      run += 4 * q + 1 < b ? v[q].y : 0u;
      run += 4 * q + 2 < b ? v[q].z : 0u;
      run += 4 * q + 3 < b ? v[q].w : 0u;
    }
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
                                                      char* ws, uint32_t* status, const MultiState* multi,
                                                      uint64_t* stamps) {
  if (multi && multi->m > kCbLdsMaxUsed) return;  // built by the grid-wide steps
  __shared__ CbLds lds;
  HF_CB_STAMP(0);
  codebook_block<NT>(hist, book, ws, status, lds, stamps, multi != nullptr);  // (sort_count zeroed the unused)
  if (stamps) {
    __syncthreads();
    HF_CB_STAMP(8);
  }
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
                           uint32_t* status, hipStream_t stream, const KernelTimer& timer, uint64_t* stamps) {
  (void)ws_bytes;
  const uint32_t A = book.alphabet;
  char* w = (char*)ws;
  hipError_t e = hipSuccess;
  timer.before(stream);
  if (A > kMultiAlphabet) {
    const MultiLayout M = multi_layout(A);
    const uint32_t NB = multi_blocks(A);
    e = launch_fill_u32((uint32_t*)(w + M.st), kMultiFlagWords, 0u, stream);
    if (e == hipSuccess) {
      cbm_sort_kernel<<<NB, kMT, 0, stream>>>(hist, book, w, status);
      cbm_tree_kernel<<<1, 1024, 0, stream>>>(book, w, status);
      cbm_tail_kernel<<<NB, kMT, 0, stream>>>(book, w, status);
      codebook_kernel<1024><<<1, 1024, 0, stream>>>(hist, book, w, status, (const MultiState*)(w + M.st), stamps);
      e = hipGetLastError();
    }
  } else {
    codebook_kernel<1024><<<1, 1024, 0, stream>>>(hist, book, w, status, nullptr, stamps);
    e = hipGetLastError();
  }
  timer.after(stream);
  return e;
}

}  // namespace hf
