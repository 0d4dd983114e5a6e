// hf_codebook_dev.h -- device code of stages 2 and 3: parallel Huffman code
// lengths and canonical codewords (Sec. 4.2, Algorithm 1 of the paper).
// Internal to libhf; the kernels and launchers are in hf_codebook.hip.
//
// One workgroup of 1024 lanes builds the whole book (the batched path
// launches one 256-lane workgroup per stream).  The paper runs its
// construction as cooperative grid-wide kernels over global memory; a
// codebook of a few thousand used symbols fits one gfx950 workgroup's LDS
// (160 KiB), where a barrier costs ~100 cycles instead of a grid sync, so the
// tree lives in LDS whenever at most kCbLdsMaxUsed symbols are used and in
// the workspace otherwise (same code, instantiated for both).
//
// Books of at most 256 used symbols whose counts sum below 2^32 - 1 (the
// common case: byte streams, quantization codes) take a one-wave path
// (build_book_small, below): the histogram is read once into registers,
// the rounds run with both runs and the queue of internal nodes in one
// wave's registers, merged by a bitonic network.  Other books take the
// steps below.
//
// Steps:
//  1. compaction: used symbols in ascending symbol order get compact index u;
//     unused symbols receive cl = cw = 0 at once;
//  2. sort leaves by (count, u) -- u preserves symbol order -- on 48-bit keys
//     (count << 16 | u): rank sort up to 512 used symbols, a stable LSD radix
//     sort on the count above (8 bits a pass); the paper sorts with Thrust;
//  3. GenerateCL: rounds of the parallel two-queue construction.  t = sum of
//     the two lightest available nodes (leaf before internal on equal
//     weight); every unconsumed leaf with weight <= t and every queued
//     internal node are merged by key (Merge Path: each element's output
//     position is its own index plus a binary search in the other run);
//     consecutive pairs meld into new internal nodes; an odd last node waits
//     for the next round.  Every lane keeps the queue cursors and computes t
//     itself from broadcast LDS reads, so a round costs three barriers and
//     no single-lane section.  This consumes nodes in exactly the order of a heap
//     keyed (weight, leaf-first, rank), so the lengths equal that heap's.
//     The paper's strict "< t" threshold and its leader-pointer updates are
//     replaced by "<= t" and one parent link per node;
//  4. depths of internal nodes by pointer jumping over parent links
//     (log2 depth steps); cl(leaf) = depth(parent) + 1;
//  5. GenerateCW + canonization: counts per length; First and Entry; the
//     rank of each symbol among equal lengths in symbol order from wave
//     ballots (a stable counting sort by length), giving cw = first[l] + rank
//     and rev[entry[l] + rank] = symbol.
#pragma once

#include "hf_device.h"
#include "hf_kernels.h"

namespace hf {

// Phase stamps of a traced build (hf_build_codebook_traced): lane 0 of
// wave 0 stores the shader clock at the given index when `stamps` is set,
// at points where it has just passed a workgroup barrier or where wave 0
// alone carries on; untraced builds pass null and store nothing.
#define HF_CB_STAMP(i)                                                              \
  do {                                                                              \
    if (stamps && threadIdx.x == 0) stamps[i] = __builtin_amdgcn_s_memtime();    \
  } while (0)


namespace {

constexpr uint32_t kMaxLen = HF_MAX_CODELEN;

__host__ __device__ inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

__host__ __device__ inline uint32_t pow2_ceil(uint32_t x) {
  uint32_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

// Global-memory layout of the tree when more than kCbLdsMaxUsed symbols
// are used (ids need 32 bits there).
struct GlobalLayout {
  size_t key, iw, mw, mid, par, usym, clu, dA, dB, nA, nB, total;
};

__host__ __device__ inline GlobalLayout global_layout(uint32_t A) {
  GlobalLayout L;
  size_t o = 0;
  const uint32_t P = pow2_ceil(A);
  L.key = o;  o += align256((size_t)P * 8);
  L.iw = o;   o += align256((size_t)A * 8);
  L.mw = o;   o += align256((size_t)A * 8);
  L.mid = o;  o += align256((size_t)A * 4);
  L.par = o;  o += align256((size_t)A * 8);
  L.usym = o; o += align256((size_t)A * 4);
  L.clu = o;  o += align256((size_t)A);
  L.dA = o;   o += align256((size_t)A * 2);
  L.dB = o;   o += align256((size_t)A * 2);
  L.nA = o;   o += align256((size_t)A * 4);
  L.nB = o;   o += align256((size_t)A * 4);
  L.total = o;
  return L;
}

template <typename IdT>
struct Tree {
  uint64_t* key;   // [P] leaves, sorted by (count << 16 | u); padding ~0
  uint64_t* iw;    // [m-1] internal node weights, creation order
  uint64_t* mw;    // [m] merged sequence of the current round: weights
  IdT* mid;        // [m] merged sequence: node ids (leaf i -> i, internal k -> m+k)
  IdT* par;        // [2m-1] parent internal index of every node id
  IdT* usym;       // [m] compact index -> symbol
  uint8_t* clu;    // [m] compact index -> code length
  uint16_t* dA;    // [m-1] depth ping-pong
  uint16_t* dB;
  IdT* nA;         // [m-1] jump-pointer ping-pong
  IdT* nB;
};

constexpr int kCbMaxWaves = 16;

// Above this many used symbols a round's runs are long enough that the whole
// workgroup merges them (three barriers a round) instead of one wave.
constexpr uint32_t kOneWaveRoundsMax = 1024;

struct Shared {
  uint64_t wsum[kCbMaxWaves];
  uint32_t wmax[kCbMaxWaves];
  uint32_t wtot[kCbMaxWaves];
  uint32_t cnt[kMaxLen + 1];
  uint32_t cntw[kCbMaxWaves][kMaxLen + 1];
  uint64_t first[kMaxLen + 1];
  uint32_t entry[kMaxLen + 1];
  uint64_t total;
  uint32_t a;
  uint32_t lmax, lmin;
  uint32_t rend[256];  // workgroup rounds: internal nodes created up to the end of each round
};

constexpr uint32_t kRoundEndsMax = 256;

// Per-wave aggregation of equal lengths before one LDS atomic per distinct
// length: the lanes sharing my length are the AND over the length's 7 bits
// of that bit's ballot or its complement, and the last of them adds their
// number.
__device__ __forceinline__ void count_lengths(uint32_t l, bool valid, uint32_t* cnt) {
  const uint32_t lv = valid ? l : 0u;  // used symbols have lengths >= 1
  uint64_t eq = ~0ull;
#pragma unroll
  for (int bit = 0; bit < 7; ++bit) {
    const bool on = (lv >> bit) & 1u;
    const uint64_t B = __ballot(on);
    eq &= on ? B : ~B;
  }
  if (valid && (eq >> lane_id()) == 1ull) atomicAdd(&cnt[lv], (uint32_t)__popcll(eq));
}

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}

// Orders this wave's earlier memory writes before its later reads (the
// single-wave rounds need no workgroup barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// GenerateCL rounds run by one wave: the round's threshold, selection count,
// carry and queue cursors are wave-uniform values obtained with readlane and
// ballots, so a round needs no workgroup barrier.  Merge ranks for runs of
// at most 64 nodes come from counting over register-broadcast weights.
template <typename IdT>
__device__ __forceinline__ void rounds_one_wave(const Tree<IdT>& t, uint32_t m, uint32_t* status) {
  const uint32_t lane = lane_id();
  uint32_t lc = 0, ih = 0, it = 0;
  for (uint32_t round = 0; (m - lc) + (it - ih) > 1; ++round) {
    if (round >= m) {  // every round creates at least one node: m - 1 rounds suffice
      if (lane == 0) raise_status(status, HF_ERR_INTERNAL);
      break;
    }
    // the two lightest nodes: lanes 0-1 read the leaf queue head, 2-3 the internal one
    uint64_t hv = ~0ull;
    if (lane < 2) {
      if (lc + lane < m) hv = t.key[lc + lane] >> 16;
    } else if (lane < 4) {
      if (ih + lane - 2 < it) hv = t.iw[ih + lane - 2];
    }
    const uint64_t l0 = readlane64(hv, 0), l1 = readlane64(hv, 1);
    const uint64_t i0 = readlane64(hv, 2), i1 = readlane64(hv, 3);
    uint64_t w1, w2;  // leaf first on equal weight; ~0 marks an empty slot
    if (l0 <= i0) {
      w1 = l0;
      w2 = l1 <= i0 ? l1 : i0;
    } else {
      w1 = i0;
      w2 = l0 <= i1 ? l0 : i1;
    }
    const uint64_t tw = w1 + w2;
    // a = leaves in [lc, m) no heavier than tw (a prefix of the sorted run)
    uint32_t a = 0;
    for (uint32_t base = lc; base < m; base += kWave) {
      const uint32_t p = base + lane;
      const uint32_t c = (uint32_t)__popcll(__ballot(p < m && (t.key[p] >> 16) <= tw));
      a += c;
      if (c < (uint32_t)kWave) break;
    }
    const uint32_t b = it - ih, total = a + b, pairs = total >> 1;
    // merge by key: leaf j goes to j + #internals lighter than it, internal q
    // to q + #leaves no heavier than it
    if (a <= (uint32_t)kWave && b <= (uint32_t)kWave) {
      const uint64_t wl = lane < a ? (t.key[lc + lane] >> 16) : ~0ull;
      const uint64_t wi = lane < b ? t.iw[ih + lane] : ~0ull;
      uint32_t rl = 0, ri = 0;
      for (uint32_t q = 0; q < b; ++q) rl += readlane64(wi, (int)q) < wl;
      for (uint32_t j = 0; j < a; ++j) ri += readlane64(wl, (int)j) <= wi;
      if (lane < a) {
        t.mw[lane + rl] = wl;
        t.mid[lane + rl] = (IdT)(lc + lane);
      }
      if (lane < b) {
        t.mw[lane + ri] = wi;
        t.mid[lane + ri] = (IdT)(m + ih + lane);
      }
    } else {
      for (uint32_t j = lane; j < a; j += kWave) {
        const uint64_t w = t.key[lc + j] >> 16;
        uint32_t lo = ih, hi = it;
        while (lo < hi) {
          const uint32_t md = (lo + hi) >> 1;
          if (t.iw[md] < w) lo = md + 1;
          else hi = md;
        }
        t.mw[j + (lo - ih)] = w;
        t.mid[j + (lo - ih)] = (IdT)(lc + j);
      }
      for (uint32_t q = lane; q < b; q += kWave) {
        const uint64_t w = t.iw[ih + q];
        uint32_t lo = lc, hi = lc + a;
        while (lo < hi) {
          const uint32_t md = (lo + hi) >> 1;
          if ((t.key[md] >> 16) <= w) lo = md + 1;
          else hi = md;
        }
        t.mw[q + (lo - lc)] = w;
        t.mid[q + (lo - lc)] = (IdT)(m + ih + q);
      }
    }
    wave_sync();
    // meld consecutive pairs; an odd last node stays in its queue
    for (uint32_t p = lane; p < pairs; p += kWave) {
      const uint32_t k = it + p;
      t.iw[k] = t.mw[2 * p] + t.mw[2 * p + 1];
      t.par[t.mid[2 * p]] = (IdT)k;
      t.par[t.mid[2 * p + 1]] = (IdT)k;
    }
    const bool carry_leaf = (total & 1) && (uint32_t)t.mid[total - 1] < m;
    const bool carry_int = (total & 1) && !carry_leaf;
    lc += a - (carry_leaf ? 1u : 0u);
    ih += b - (carry_int ? 1u : 0u);
    it += pairs;
    wave_sync();
  }
}

// Compaction in symbol order, NT symbols at a time (coalesced reads): used
// symbol s gets compact index u (its rank among used symbols), key[u] =
// count << 16 | u and usym[u] = s.  (Unused symbols' cl = cw = 0 are
// written by the histogram pass of codebook_block, with lane-contiguous
// stores, or before it by the grid-wide count of a large alphabet.)
template <int NT, typename IdT>
__device__ __forceinline__ void compact(const uint32_t* __restrict__ hist, uint32_t A, uint64_t* key, IdT* usym,
                                        const hf_codebook& book, uint32_t* wtot) {
  constexpr uint32_t V = 4;  // consecutive symbols per lane and chunk
  uint32_t run = 0;
  for (uint32_t c0 = 0; c0 < A; c0 += V * NT) {
    const uint32_t s = c0 + V * threadIdx.x;
    uint32_t h[V];
    uint32_t c = 0;
#pragma unroll
    for (uint32_t v = 0; v < V; ++v) {
      h[v] = s + v < A ? hist[s + v] : 0u;
      c += h[v] != 0;
    }
    uint32_t tot;
    uint32_t u = run + block_exclusive_scan<NT / kWave>(c, wtot, &tot);
#pragma unroll
    for (uint32_t v = 0; v < V; ++v) {
      if (h[v]) {
        key[u] = ((uint64_t)h[v] << 16) | u;
        usym[u] = (IdT)(s + v);
        ++u;
      }
    }
    run += tot;
    __syncthreads();  // wtot is reused by the next chunk
  }
}

// Stable LSD radix sort of key[0, m) (count << 16 | u, in u order) by the
// 32-bit count, 8 bits a pass, as many passes as the largest count needs;
// tmp[0, m) is the other buffer and cnt an LDS area of NT / 64 * 256 words.
// Wave w owns the contiguous segment w of the keys: it counts its digits
// (LDS atomics), a workgroup scan turns the counts into offsets in (digit,
// wave) order, and the wave scatters its segment 64 keys at a time.  The
// lanes of a group sharing my digit are the AND over its 8 bits of that
// bit's ballot or its complement; a key goes to its digit's offset plus the
// equal-digit lanes before it (so equal counts keep their order), and the
// last of them advances the offset.  A wave's LDS operations take effect
// in order, so the next group sees the advanced offsets.  Keys are read
// four groups ahead (the workspace's latency, not the placing, bounds a
// lone workgroup's pass).
template <int NT>
__device__ __forceinline__ void radix_sort_keys(uint64_t* key, uint64_t* tmp, uint32_t m, uint32_t wmax,
                                                Shared& sh, uint32_t* cnt) {
  constexpr uint32_t NW = NT / kWave;
  constexpr uint32_t PER = NW * 256 / NT;  // counters per thread in the scan
  const uint32_t tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  uint32_t passes = 0;
  while (passes < 4 && (wmax >> (8 * passes)) != 0) ++passes;
  const uint32_t seg = (m + NW - 1) / NW;
  const uint32_t s0 = min(m, wave * seg), s1 = min(m, s0 + seg);
  uint32_t* wc = cnt + wave * 256;
  uint64_t* src = key;
  uint64_t* dst = tmp;
  for (uint32_t p = 0; p < passes; ++p) {
    const uint32_t shift = 16 + 8 * p;
    for (uint32_t i = tid; i < NW * 256; i += NT) cnt[i] = 0;
    __syncthreads();
    // four groups of 64 keys are counted while the next four load
    uint64_t k[4], kn[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint32_t i = s0 + u * kWave + lane;
      kn[u] = i < s1 ? src[i] : 0ull;
    }
    for (uint32_t i0 = s0; i0 < s1; i0 += 4 * kWave) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        k[u] = kn[u];
        const uint32_t i = i0 + (4 + u) * kWave + lane;
        kn[u] = i < s1 ? src[i] : 0ull;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (i0 + u * kWave + lane < s1) atomicAdd(&wc[(uint32_t)(k[u] >> shift) & 255], 1u);
    }
    __syncthreads();
    // offsets in (digit, wave) order: thread t takes entries [PER t, PER t + PER)
    // of that order, entry j being counter (wave j % NW, digit j / NW)
    uint32_t v[PER], c = 0;
#pragma unroll
    for (uint32_t q = 0; q < PER; ++q) {
      const uint32_t j = PER * tid + q;
      v[q] = cnt[(j % NW) * 256 + j / NW];
      c += v[q];
    }
    uint32_t tot;
    uint32_t pre = block_exclusive_scan<NW>(c, sh.wtot, &tot);
    __syncthreads();
#pragma unroll
    for (uint32_t q = 0; q < PER; ++q) {
      const uint32_t j = PER * tid + q;
      cnt[(j % NW) * 256 + j / NW] = pre;
      pre += v[q];
    }
    __syncthreads();
    // four groups are placed while the next four load
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint32_t i = s0 + u * kWave + lane;
      kn[u] = i < s1 ? src[i] : 0ull;
    }
    for (uint32_t b0 = s0; b0 < s1; b0 += 4 * kWave) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        k[u] = kn[u];
        const uint32_t i = b0 + (4 + u) * kWave + lane;
        kn[u] = i < s1 ? src[i] : 0ull;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint32_t b = b0 + u * kWave;
        const bool valid = b + lane < s1;
        const uint32_t d = valid ? (uint32_t)(k[u] >> shift) & 255 : 256u;  // 256: no used digit
        uint64_t match = ~0ull;
#pragma unroll
        for (int q = 0; q < 9; ++q) {
          const bool on = (d >> q) & 1u;
          const uint64_t B = __ballot(on);
          match &= on ? B : ~B;
        }
        if (valid) {
          const uint32_t slot = wc[d] + (uint32_t)__popcll(match & lanemask_lt());
          dst[slot] = k[u];
          if ((match >> lane) == 1ull) wc[d] = slot + 1;
        }
      }
    }
    __syncthreads();
    uint64_t* t2 = src;
    src = dst;
    dst = t2;
  }
  if (src != key) {
    for (uint32_t i = tid; i < m; i += NT) key[i] = src[i];
  }
}

// Steps 3 and 4 of a book: the GenerateCL rounds over the sorted leaves
// t.key[0, m) (m >= 2) and the depth of every internal node; returns the
// array that holds the depths (one of t.dA, t.dB).
template <typename IdT, int NT>
__device__ __forceinline__ uint16_t* build_book_tree(const Tree<IdT>& t, Shared& sh, uint32_t m, uint32_t* status,
                                                     uint64_t* stamps = nullptr) {
  const uint32_t tid = threadIdx.x;
  const uint32_t wave = tid / kWave;
  // ---- 3. GenerateCL rounds ------------------------------------------------
  uint32_t nrounds = kRoundEndsMax + 1;  // rounds run by the workgroup (recorded up to kRoundEndsMax)
  if (sizeof(IdT) == 2 && m <= kOneWaveRoundsMax) {
    // tree in LDS, short runs: one wave runs the rounds
    if (wave == 0) rounds_one_wave(t, m, status);
    __syncthreads();
  } else {
  // every lane tracks the queues: leaves [lc, m), internal nodes [ih, it)
  uint32_t lc = 0, ih = 0, it = 0;
  nrounds = 0;
  for (uint32_t round = 0; (m - lc) + (it - ih) > 1; ++round) {
    if (round >= m) {  // every round creates at least one node: m - 1 rounds suffice
      if (tid == 0) raise_status(status, HF_ERR_INTERNAL);
      break;
    }
    // t = the two lightest available nodes, leaf first on equal weight
    uint64_t wsum = 0;
    {
      uint32_t li = lc, ii = ih;
      for (int p = 0; p < 2; ++p) {
        const bool leaf = li < m && (ii >= it || (t.key[li] >> 16) <= t.iw[ii]);
        wsum += leaf ? (t.key[li++] >> 16) : t.iw[ii++];
      }
    }
    // a = leaves in [lc, m) with weight <= t (a prefix of the sorted rest):
    // the blocks of `step` leaves lying wholly below t, then the leaves below
    // t inside the next block, each counted in one barrier
    uint32_t a;
    {
      const uint32_t R = m - lc, step = (R + NT - 1) / NT;
      const bool whole = tid * step < R && (t.key[lc + min(R, (tid + 1) * step) - 1] >> 16) <= wsum;
      const uint32_t c1 = (uint32_t)__syncthreads_count(whole);
      const uint32_t base = lc + c1 * step;
      const bool part = tid < step && base + tid < m && (t.key[base + tid] >> 16) <= wsum;
      const uint32_t c2 = (uint32_t)__syncthreads_count(part);
      a = min(R, c1 * step + c2);
    }
    const uint32_t b = it - ih;
    const uint32_t total = a + b, pairs = total >> 1;
    // Merge Path: leaves precede internal nodes of equal weight.  A long
    // merge is cut into NT equal output ranges: one binary search along the
    // range's first diagonal, then a sequential merge of the range;
    // otherwise each element finds its position in the other run.
    if (total > 2 * NT) {
      const uint32_t per = (total + NT - 1) / NT;
      const uint32_t d0 = min(total, tid * per), d1 = min(total, d0 + per);
      uint32_t lo = d0 > b ? d0 - b : 0u, hi = min(d0, a);
      while (lo < hi) {  // leaves [0, i) and internal nodes [0, d0 - i) come first
        const uint32_t md = (lo + hi) >> 1;
        if ((t.key[lc + md] >> 16) <= t.iw[ih + d0 - md - 1]) lo = md + 1;
        else hi = md;
      }
      uint32_t i = lo, j = d0 - lo;
      uint64_t wl = i < a ? t.key[lc + i] >> 16 : ~0ull;
      uint64_t wi = j < b ? t.iw[ih + j] : ~0ull;
      for (uint32_t d = d0; d < d1; ++d) {
        if (i < a && (j >= b || wl <= wi)) {
          t.mw[d] = wl;
          t.mid[d] = (IdT)(lc + i);
          ++i;
          wl = i < a ? t.key[lc + i] >> 16 : ~0ull;
        } else {
          t.mw[d] = wi;
          t.mid[d] = (IdT)(m + ih + j);
          ++j;
          wi = j < b ? t.iw[ih + j] : ~0ull;
        }
      }
    } else {
    for (uint32_t j = tid; j < a; j += NT) {
      const uint64_t w = t.key[lc + j] >> 16;
      uint32_t lo = ih, hi = it;
      while (lo < hi) {
        const uint32_t md = (lo + hi) >> 1;
        if (t.iw[md] < w) lo = md + 1;
        else hi = md;
      }
      const uint32_t pos = j + (lo - ih);
      t.mw[pos] = w;
      t.mid[pos] = (IdT)(lc + j);
    }
    for (uint32_t q = tid; q < b; q += NT) {
      const uint64_t w = t.iw[ih + q];
      uint32_t lo = lc, hi = lc + a;
      while (lo < hi) {
        const uint32_t md = (lo + hi) >> 1;
        if ((t.key[md] >> 16) <= w) lo = md + 1;
        else hi = md;
      }
      const uint32_t pos = q + (lo - lc);
      t.mw[pos] = w;
      t.mid[pos] = (IdT)(m + ih + q);
    }
    }
    __syncthreads();
    // Meld consecutive pairs; an odd last node stays in its queue
    for (uint32_t p = tid; p < pairs; p += NT) {
      const uint32_t k = it + p;
      t.iw[k] = t.mw[2 * p] + t.mw[2 * p + 1];
      t.par[t.mid[2 * p]] = (IdT)k;
      t.par[t.mid[2 * p + 1]] = (IdT)k;
    }
    const bool carry_leaf = (total & 1) && (uint32_t)t.mid[total - 1] < m;
    const bool carry_int = (total & 1) && !carry_leaf;
    lc += a - (carry_leaf ? 1u : 0u);
    ih += b - (carry_int ? 1u : 0u);
    it += pairs;
    if (tid == 0 && round < kRoundEndsMax) sh.rend[round] = it;
    nrounds = round + 1;
    __syncthreads();
  }
  }

  HF_CB_STAMP(4);
  // ---- 4. depths of internal nodes ------------------------------------------
  // A node's parent is created in a later round, so with the round ends
  // recorded the depths follow round by round from the last (the root, at
  // depth 0); otherwise by pointer jumping over parent links.
  const uint32_t nint = m - 1, root = m - 2;
  uint16_t* dc = t.dA;
  if (nrounds <= kRoundEndsMax) {
    if (tid == 0) dc[root] = 0;
    __syncthreads();
    for (int r = (int)nrounds - 1; r >= 0; --r) {
      const uint32_t k0 = r > 0 ? sh.rend[r - 1] : 0u, k1 = sh.rend[r];
      for (uint32_t k = k0 + tid; k < k1; k += NT)
        if (k != root) {
          const uint32_t d = (uint32_t)dc[(uint32_t)t.par[m + k]] + 1;
          dc[k] = (uint16_t)(d < 0xFFFFu ? d : 0xFFFFu);
        }
      __syncthreads();
    }
  } else {
  for (uint32_t k = tid; k < nint; k += NT) {
    t.dA[k] = (k == root) ? 0 : 1;
    t.nA[k] = (IdT)((k == root) ? root : (uint32_t)t.par[m + k]);
  }
  __syncthreads();
  uint16_t* dn = t.dB;
  IdT* nc = t.nA;
  IdT* nn = t.nB;
  for (int step = 0;; ++step) {
    int active = 0;
    for (uint32_t k = tid; k < nint; k += NT) {
      const IdT x = nc[k];
      const uint32_t d = (uint32_t)dc[k] + dc[x];
      dn[k] = (uint16_t)(d < 0xFFFFu ? d : 0xFFFFu);
      const IdT y = nc[x];
      nn[k] = y;
      active |= ((uint32_t)y != root);
    }
    uint16_t* td = dc; dc = dn; dn = td;
    IdT* tn = nc; nc = nn; nn = tn;
    if (!__syncthreads_or(active)) break;
    if (step >= 32) {  // depth < 2^32 needs at most 32 doublings
      if (tid == 0) raise_status(status, HF_ERR_INTERNAL);
      break;
    }
  }
  }
  return dc;
}

// lds_scratch: NT / 64 * 256 words of LDS free until the rounds.
template <typename IdT, int NT>
__device__ __forceinline__ void build_book(const Tree<IdT>& t, Shared& sh, const uint32_t* __restrict__ hist,
                                           uint32_t A, uint32_t m, uint32_t wmax, const hf_codebook& book,
                                           uint32_t* status, uint32_t* lds_scratch, uint64_t* stamps = nullptr) {
  constexpr int NW = NT / kWave;
  const uint32_t tid = threadIdx.x;
  const uint32_t lane = tid & (kWave - 1);
  const uint32_t wave = tid / kWave;

  // ---- 1. compaction -----------------------------------------------------
  compact<NT>(hist, A, t.key, t.usym, book, sh.wtot);
  for (uint32_t l = tid; l <= kMaxLen; l += NT) sh.cnt[l] = 0;
  if (tid == 0) {
    sh.total = 0;
    sh.lmax = 0;
    sh.lmin = 0xFFFFFFFFu;
  }
  __syncthreads();

  if (m <= 1) {
    // no tree: an empty book, or one symbol with the 1-bit code 0
    for (uint32_t l = tid; l <= kMaxLen; l += NT) {
      book.first[l] = 0;
      book.entry[l] = (m == 1 && l >= 2) ? 1u : 0u;
    }
    if (tid == 0) {
      uint64_t h0 = 0;
      if (m == 1) {
        const uint32_t s = (uint32_t)t.usym[0];
        h0 = t.key[0] >> 16;
        book.cl[s] = 1;
        book.cw[s] = 0;
        book.rev[0] = s;
      }
      book.info[0] = m;
      book.info[1] = m;
      book.info[2] = h0;
      book.info[3] = m;
    }
    return;
  }

  HF_CB_STAMP(2);
  // ---- 2. sort leaves ascending by (count, u) --------------------------------
  if (m <= 512) {
    // rank sort: keys are distinct (u in the low bits); broadcast reads
    for (uint32_t i = tid; i < m; i += NT) {
      const uint64_t k = t.key[i];
      uint32_t r = 0;
      uint32_t j = 0;
      for (; j + 4 <= m; j += 4) {
        const uint64_t k0 = t.key[j], k1 = t.key[j + 1], k2 = t.key[j + 2], k3 = t.key[j + 3];
        r += (k0 < k) + (k1 < k) + (k2 < k) + (k3 < k);
      }
      for (; j < m; ++j) r += t.key[j] < k;
      t.mw[r] = k;
    }
    __syncthreads();
    for (uint32_t i = tid; i < m; i += NT) t.key[i] = t.mw[i];
  } else {
    radix_sort_keys<NT>(t.key, t.mw, m, wmax, sh, lds_scratch);
  }
  __syncthreads();

  HF_CB_STAMP(3);
  uint16_t* dc = build_book_tree<IdT, NT>(t, sh, m, status, stamps);

  HF_CB_STAMP(5);
  // ---- 5a. leaf lengths, counts per length, total bits ----------------------
  uint64_t bits = 0;
  uint32_t my_max = 0, my_min = 0xFFFFFFFFu;
  // four leaves a lane at a time, every load issued before the first store
  // (the stores may alias the loads as far as the compiler knows)
  for (uint32_t i0 = 0; i0 < m; i0 += 4 * NT) {
    uint64_t kk[4];
    uint32_t pr[4], dd[4], sy[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const uint32_t i = i0 + v * NT + tid;
      kk[v] = i < m ? t.key[i] : 0ull;
      pr[v] = i < m ? (uint32_t)t.par[i] : 0u;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const bool valid = i0 + v * NT + tid < m;
      dd[v] = valid ? (uint32_t)dc[pr[v]] : 0u;
      sy[v] = valid ? (uint32_t)t.usym[(uint32_t)(kk[v] & 0xFFFFu)] : 0u;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const bool valid = i0 + v * NT + tid < m;
      uint32_t l = 0;
      if (valid) {
        l = dd[v] + 1;
        bits += (kk[v] >> 16) * l;
        my_max = max(my_max, l);
        my_min = min(my_min, l);
        if (l > kMaxLen) l = kMaxLen;  // flagged below; keeps indexes in range
        t.clu[(uint32_t)(kk[v] & 0xFFFFu)] = (uint8_t)l;
        book.cl[sy[v]] = (uint8_t)l;
      }
      count_lengths(l, valid, sh.cnt);
    }
  }
  bits = wave_sum_u64(bits);
  my_max = wave_max_u32(my_max);
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) my_min = min(my_min, (uint32_t)__shfl_xor(my_min, d, kWave));
  if (lane == 0) {
    atomicAdd((unsigned long long*)&sh.total, (unsigned long long)bits);
    atomicMax(&sh.lmax, my_max);
    atomicMin(&sh.lmin, my_min);
  }
  __syncthreads();

  HF_CB_STAMP(6);
  // ---- 5b. First and Entry (wave 0; lane j holds length j + 1) ----------------
  if (wave == 0) {
    const uint32_t L = sh.lmax > kMaxLen ? kMaxLen : sh.lmax;
    const uint32_t c = sh.cnt[lane + 1];
    const uint32_t below = wave_inclusive_scan(c) - c;  // codes shorter than lane + 1
    uint64_t f = 0, mine = 0;
    for (int l = (int)L - 1; l >= 1; --l) {
      f = (f + (uint32_t)__builtin_amdgcn_readlane((int)c, l) + 1) >> 1;  // cnt[l + 1]
      if ((int)lane == l - 1) mine = f;
    }
    sh.first[lane + 1] = mine;
    sh.entry[lane + 1] = below;
    if (lane == 0) {
      sh.first[0] = 0;
      sh.entry[0] = 0;
      if (sh.lmax > kMaxLen) raise_status(status, HF_ERR_CODELEN);
      book.info[0] = m;
      book.info[1] = sh.lmax;
      book.info[2] = sh.total;
      book.info[3] = sh.lmin;
    }
  }
  __syncthreads();
  for (uint32_t l = tid; l <= kMaxLen; l += NT) {
    book.first[l] = sh.first[l];
    book.entry[l] = sh.entry[l];
  }

  HF_CB_STAMP(7);
  // ---- 5c. rank within each length in symbol order -------------------------
  // Wave w takes a contiguous segment of compact indices.  In each 64-symbol
  // group the lanes sharing my length are the AND over the length's 7 bits
  // of that bit's ballot or its complement (past the segment lanes carry
  // length 0, which no used symbol has); the group's last lane of each length
  // updates that length's count (pass 1) or next rev slot (pass 2).  A
  // wave's LDS operations take effect in order, so the next group sees it.
  const uint32_t seg = ((m + NT - 1) / NT) * kWave;
  const uint32_t sbeg = min(m, wave * seg), send = min(m, sbeg + seg);
  uint32_t* wc = sh.cntw[wave];  // [kMaxLen + 1] this wave's count, then next slot, per length
  for (uint32_t l = lane; l <= kMaxLen; l += kWave) wc[l] = 0;
  for (int pass = 0; pass < 2; ++pass) {
    // four groups are ranked while the next four load
    uint32_t lv[4], sv[4], ln[4], sn[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const uint32_t u = sbeg + v * kWave + lane;
      ln[v] = u < send ? (uint32_t)t.clu[u] : 0u;
      sn[v] = (pass == 1 && u < send) ? (uint32_t)t.usym[u] : 0u;
    }
    for (uint32_t u0 = sbeg; u0 < send; u0 += 4 * kWave) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        lv[v] = ln[v];
        sv[v] = sn[v];
        const uint32_t u = u0 + (4 + v) * kWave + lane;
        ln[v] = u < send ? (uint32_t)t.clu[u] : 0u;
        sn[v] = (pass == 1 && u < send) ? (uint32_t)t.usym[u] : 0u;
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const bool valid = u0 + v * kWave + lane < send;
        const uint32_t l = valid ? lv[v] : 0u;
        uint64_t eq = ~0ull;
#pragma unroll
        for (int bit = 0; bit < 7; ++bit) {
          const bool on = (l >> bit) & 1u;
          const uint64_t B = __ballot(on);
          eq &= on ? B : ~B;
        }
        const bool last = valid && (eq >> lane) == 1ull;
        if (pass == 0) {
          if (last) wc[l] += (uint32_t)__popcll(eq);
        } else if (valid) {
          const uint32_t pos = wc[l] + (uint32_t)__popcll(eq & lanemask_lt());
          const uint32_t s = sv[v];
          book.rev[pos] = s;
          book.cw[s] = sh.first[l] + (pos - sh.entry[l]);
          if (last) wc[l] = pos + 1;
        }
      }
    }
    if (pass == 0) {
      __syncthreads();
      // slots: codes shorter than l, then earlier waves' codes of length l
      if (tid >= 1 && tid <= kMaxLen) {
        uint32_t run = sh.entry[tid];
        for (int w = 0; w < NW; ++w) {
          const uint32_t c = sh.cntw[w][tid];
          sh.cntw[w][tid] = run;
          run += c;
        }
      }
      __syncthreads();
    }
  }
}

// The codebook's LDS: the tree of up to C used symbols (more go to the
// workspace), reused by the small-book path.
template <uint32_t C>
struct CbLdsT {
  static_assert(C >= 1024, "the small-book layout needs 1024 slots");
  static constexpr uint32_t kCap = C;
  Shared sh;
  uint64_t key[C];
  uint64_t iw[C];
  uint64_t mw[C];  // also holds the depth arrays after the rounds
  uint16_t mid[C];
  uint16_t par[2 * C];
  uint16_t usym[C];
  uint8_t clu[C];
};
using CbLds = CbLdsT<kCbLdsMaxUsed>;

// ---------------------------------------------------------------------------
// Books of at most kSmallUsed used symbols whose counts sum below 2^32 - 1:
// every weight fits 32 bits and one wave runs the rounds with both runs and
// the queue of internal nodes in registers.  A round is that wave's
// dependent chain of instructions (about 1200 cycles, a third of it the
// merge network), so every step keeps uniform values scalar and avoids
// LDS round trips and branches on lane masks.  The rank sort, depths and
// codewords use every wave or wave 0 as marked.
// ---------------------------------------------------------------------------
constexpr uint32_t kSmallUsed = 256;
constexpr uint32_t kInf32 = 0xFFFFFFFFu;

constexpr uint32_t kLeafSlots = kSmallUsed + 2 * 64;  // sorted leaf weights, kInf32 past m
constexpr uint32_t kSerialUsed = 40;  // up to this many used symbols the tree is built one node a step

__device__ __forceinline__ uint32_t readlane32(uint32_t v, uint32_t l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)l);
}

// v of lane (lane ^ D), D a power of two below 64: DPP quad permutes for 1
// and 2, row shifts left and right on alternate 4-lane banks for 4, a row
// rotation for 8, and the row-swap instructions for 16 and 32.
template <int D>
__device__ __forceinline__ uint32_t lane_xor(uint32_t v) {
  if constexpr (D == 1) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
  } else if constexpr (D == 2) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
  } else if constexpr (D == 4) {
    const int t = __builtin_amdgcn_update_dpp(0, (int)v, 0x104, 0xF, 0x5, false);    // row_shl:4, banks 0, 2
    return (uint32_t)__builtin_amdgcn_update_dpp(t, (int)v, 0x114, 0xF, 0xA, false);  // row_shr:4, banks 1, 3
  } else if constexpr (D == 8) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xF, 0xF, false);  // row_ror:8
  } else if constexpr (D == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return (lane_id() & 16) ? r[0] : r[1];
  } else {
    static_assert(D == 32, "lane distance");
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return (lane_id() & 32) ? r[0] : r[1];
  }
}

// One half-cleaner of an ascending bitonic merge of the wave's 64 keys: of
// lanes l and l ^ D, the one with bit D clear keeps the smaller key.
template <int D>
__device__ __forceinline__ uint64_t half_clean(uint64_t k) {
  const uint32_t lo = lane_xor<D>((uint32_t)k), hi = lane_xor<D>((uint32_t)(k >> 32));
  const uint64_t p = ((uint64_t)hi << 32) | lo;
  return ((p < k) != ((lane_id() & D) != 0)) ? p : k;
}

template <int D>
__device__ __forceinline__ uint32_t half_clean(uint32_t k) {
  const uint32_t p = lane_xor<D>(k);
  return (lane_id() & D) ? max(p, k) : min(p, k);
}

// A bitonic sequence of 64 keys, one per lane, sorted ascending.
template <typename K>
__device__ __forceinline__ K bitonic_merge(K k) {
  k = half_clean<32>(k);
  k = half_clean<16>(k);
  k = half_clean<8>(k);
  k = half_clean<4>(k);
  k = half_clean<2>(k);
  return half_clean<1>(k);
}
__device__ __forceinline__ uint64_t bitonic_merge64(uint64_t k) { return bitonic_merge<uint64_t>(k); }
__device__ __forceinline__ uint32_t bitonic_merge32(uint32_t k) { return bitonic_merge<uint32_t>(k); }

// Merged position p holds node ref r (r < 256: leaf lc + r; else internal
// node ih + r - 256) and, on even p, the pair sum s: the nodes at positions
// 2k and 2k + 1 get parent it + k, whose weight is recorded.  Lanes past the
// pairs write their sinks.
__device__ __forceinline__ void link_merged(uint32_t r, uint32_t s, uint32_t p, uint32_t pairs, uint32_t lc,
                                            uint32_t ih, uint32_t it, uint16_t* parl, uint16_t* pari,
                                            uint32_t* iw, uint16_t* par_sink, uint32_t* iw_sink) {
  const bool in_pair = p < 2 * pairs;
  uint16_t* dst = r < 256 ? parl + lc + r : pari + ih + (r - 256);
  *(in_pair ? dst : par_sink) = (uint16_t)(it + (p >> 1));
  *(in_pair && !(p & 1) ? iw + it + (p >> 1) : iw_sink) = s;
}

// A wave-uniform value kept in a scalar register.
__device__ __forceinline__ uint32_t uniform32(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }

// One round's merge of leaves [lc, lc + a) and internal nodes [ih, ih + b)
// through LDS, for runs longer than a register: each node's merged position
// is its index plus a binary search in the other run (leaves first on equal
// weight); positions 2k and 2k + 1 get parent it + k, whose weight is
// accumulated in iw[it + k] (zero beforehand).
__device__ __noinline__ void merge_through_lds(const uint32_t* lw, uint32_t* iw, uint16_t* parl, uint16_t* pari,
                                               uint32_t lc, uint32_t ih, uint32_t it, uint32_t a, uint32_t b,
                                               uint32_t pairs) {
  wave_sync();  // every queued weight is in LDS
  for (uint32_t j = lane_id(); j < a; j += kWave) {
    const uint32_t w = lw[lc + j];
    uint32_t lo = ih, hi = it;  // first internal node not lighter than w
    while (lo < hi) {
      const uint32_t md = (lo + hi) >> 1;
      if (iw[md] < w) lo = md + 1;
      else hi = md;
    }
    const uint32_t pos = j + (lo - ih);
    if (pos < 2 * pairs) {
      parl[lc + j] = (uint16_t)(it + (pos >> 1));
      atomicAdd(&iw[it + (pos >> 1)], w);
    }
  }
  for (uint32_t q = lane_id(); q < b; q += kWave) {
    const uint32_t w = iw[ih + q];
    uint32_t lo = lc, hi = lc + a;  // first leaf heavier than w
    while (lo < hi) {
      const uint32_t md = (lo + hi) >> 1;
      if (lw[md] <= w) lo = md + 1;
      else hi = md;
    }
    const uint32_t pos = q + (lo - lc);
    if (pos < 2 * pairs) {
      pari[ih + q] = (uint16_t)(it + (pos >> 1));
      atomicAdd(&iw[it + (pos >> 1)], w);
    }
  }
  wave_sync();
}

// 32-bit sort keys of a small book: the words after its 64-bit keys.
template <typename Lds>
__device__ __forceinline__ uint32_t* small_key32(Lds& L) { return (uint32_t*)(L.key + kSmallUsed); }

// Wave-wide running maximum with DPP lane moves, as wave_inclusive_scan:
// lane 63 ends with the wave's maximum.
__device__ __forceinline__ uint32_t wave_inclusive_max(uint32_t v) {
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, true));  // row_shr:1
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, true));  // row_shr:2
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, true));  // row_shr:4
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, true));  // row_shr:8
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));  // row_bcast:15
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));  // row_bcast:31
  return v;
}

// Books of at most kSerialUsed used symbols: the textbook two-queue build,
// one node a step (the rounds cost about 1 K cycles each whatever their
// size, and a book of a few dozen symbols can need as many rounds as
// symbols).  Leaves, queued weights and parents sit one node a lane in
// registers, so a step is four lane reads into scalar registers, a scalar
// choice of the two lightest (leaf first on equal weight: the rounds' tie
// rule, so the tree is the same) and lane selects, without branches; LDS is
// written once at the end.  Run by one wave; not inlined, so that the rounds' code is
// compiled as it is without it.
__device__ __noinline__ void serial_tree(const uint32_t* lw, uint32_t* iw, uint16_t* parl, uint16_t* pari,
                                         uint32_t m_arg) {
  const uint32_t lane = lane_id();
  // m is wave-uniform; read it into a scalar register so that the walk's
  // loop, its cursors and its choices stay scalar (arguments of a call come
  // in vector registers)
  const uint32_t m = (uint32_t)__builtin_amdgcn_readfirstlane((int)m_arg);
  const uint32_t RW = lw[lane];        // leaf weights (kInf32 past m)
  uint32_t IWr = kInf32;               // lane k: weight of internal node k
  uint32_t PL = 0, PI = 0;             // lane e / k: parent of leaf e / internal node k
  uint32_t lc = 0, ih = 0;
  for (uint32_t k = 0; k + 1 < m; ++k) {
    const uint32_t l0 = (uint32_t)__builtin_amdgcn_readlane((int)RW, (int)lc);
    const uint32_t l1 = (uint32_t)__builtin_amdgcn_readlane((int)RW, (int)(lc + 1));
    const uint32_t i0 = (uint32_t)__builtin_amdgcn_readlane((int)IWr, (int)ih);      // kInf32 once ih = k
    const uint32_t i1 = (uint32_t)__builtin_amdgcn_readlane((int)IWr, (int)(ih + 1));
    // branch-free: the two picks, then the parents they get and the cursors
    const bool p1 = l0 <= i0;                   // first pick is leaf lc, else internal ih
    const uint32_t nl = p1 ? l1 : l0, ni = p1 ? i0 : i1;
    const bool p2 = nl <= ni;                   // second pick is a leaf, else an internal node
    const uint32_t w = (p1 ? l0 : i0) + (p2 ? nl : ni);
    const uint32_t l2 = lc + (p1 ? 1u : 0u), i2 = ih + (p1 ? 0u : 1u);  // where the second pick sits
    const bool leaf_here = (p1 && lane == lc) || (p2 && lane == l2);
    const bool int_here = (!p1 && lane == ih) || (!p2 && lane == i2);
    PL = leaf_here ? k : PL;
    PI = int_here ? k : PI;
    IWr = (lane == k ? w : IWr);
    lc = l2 + (p2 ? 1u : 0u);
    ih = i2 + (p2 ? 0u : 1u);
  }
  if (lane < m) parl[lane] = (uint16_t)PL;
  if (lane + 1 < m) {
    pari[lane] = (uint16_t)PI;
    iw[lane] = IWr;
  }
  wave_sync();
}

template <int NT, typename Lds>
__device__ __forceinline__ void build_book_small(Lds& L, uint32_t m, uint32_t narrow, const hf_codebook& book,
                                                 uint32_t* status, uint64_t* stamps = nullptr) {
  const uint32_t tid = threadIdx.x;
  const uint32_t lane = tid & (kWave - 1);
  const uint32_t wave = tid / kWave;
  uint64_t* key = L.key;                    // [kSmallUsed] count << 16 | u, u = compact index
  uint32_t* key32 = small_key32(L);         // [kSmallUsed] count << 8 | u when every count < 2^24
  uint16_t* usym = L.usym;                  // [m] compact index -> symbol
  uint32_t* lw = (uint32_t*)L.iw;           // [kLeafSlots] leaf weights, sorted by (count, u)
  uint32_t* iw = lw + kLeafSlots;           // [m-1] internal weights, creation order
  uint16_t* lu = L.mid;                     // [m] compact index of each sorted leaf
  uint16_t* parl = L.par;                   // [m] parent of each sorted leaf
  uint16_t* pari = L.par + kSmallUsed;      // [m-1] parent of each internal node

  // ---- 1. the keys of the used symbols are in LDS (compact_small) -------------
  uint32_t* rk = (uint32_t*)L.mw + 1024;  // [kSmallUsed] rank of each key
  for (uint32_t i = tid; i < kSmallUsed; i += NT) {
    iw[i] = 0;
    rk[i] = 0;
    if (i >= m) {  // above every used key
      key[i] = ~0ull;
      key32[i] = ~0u;
    }
  }
  for (uint32_t i = m + tid; i < kLeafSlots; i += NT) lw[i] = kInf32;
  for (uint32_t l = tid; l <= kMaxLen; l += NT) L.sh.cnt[l] = 0;
  __syncthreads();
  HF_CB_STAMP(2);

  // ---- 2. rank sort: rank(e) = #{j : key_j < key_e} ---------------------------
  // The key is the count above the compact (symbol-order) index, so this is
  // the rank by (count, symbol).  Each (block of e, block of j) pair of
  // 64-key blocks is counted by one wave from broadcast LDS reads, up to the
  // last used key of the j block (the keys past m are above every used one);
  // the partial ranks meet in LDS.  Counts below 2^24 take 32-bit keys,
  // half the LDS traffic.
  {
    const uint32_t nb = (m + kWave - 1) / kWave;
    for (uint32_t p = wave; p < 16; p += NT / kWave) {
      const uint32_t eb = p & 3, jb = p >> 2;
      if (eb >= nb || jb >= nb) continue;
      const uint32_t e = eb * kWave + lane;
      const uint32_t jn = min((uint32_t)kWave, (m - jb * kWave + 15) & ~15u);
      uint32_t c[4] = {0, 0, 0, 0};
      if (narrow) {
        const uint32_t ke = key32[e];
        const uint32_t* kj = key32 + jb * kWave;
        for (uint32_t j0 = 0; j0 < jn; j0 += 16) {
#pragma unroll
          for (uint32_t j = 0; j < 16; ++j) c[j & 3] += kj[j0 + j] < ke ? 1u : 0u;
        }
      } else {
        const uint64_t ke = key[e];
        const uint64_t* kj = key + jb * kWave;
        for (uint32_t j0 = 0; j0 < jn; j0 += 16) {
#pragma unroll
          for (uint32_t j = 0; j < 16; ++j) c[j & 3] += kj[j0 + j] < ke ? 1u : 0u;
        }
      }
      if (e < m) atomicAdd(&rk[e], c[0] + c[1] + c[2] + c[3]);
    }
  }
  __syncthreads();
  if (tid < m) {
    const uint32_t r = rk[tid];
    lw[r] = narrow ? key32[tid] >> 8 : (uint32_t)(key[tid] >> 16);
    lu[r] = (uint16_t)tid;
  }
  __syncthreads();
  HF_CB_STAMP(3);
  if (wave != 0) return;

  // ---- 3. GenerateCL rounds, one wave -----------------------------------------
  // The merge order is that of keys (weight, tag): tag j for leaf j of the
  // round's run and 64 + q (or 256 + q) for queued internal node q, so equal
  // weights put leaves first and keep each run's order, as the merge rule
  // requires.  Keys are 32-bit (weight << 7 | tag) while the round's heaviest
  // weight fits 25 bits, else 64-bit (weight << 32 | tag).  While the runs
  // fit 64 lanes the merge is a bitonic network in registers: runs of at most
  // 32 share one register (leaves ascending in lanes 0-31, internal nodes
  // descending in lanes 32-63), longer ones take two (a lane-by-lane compare
  // of the registers, then a network on each).  Merged position p then sits
  // in lane p (of the second register from p = 64), so pair k = (2k, 2k+1)
  // is internal node it + k, its weight the sum of two neighbouring lanes.  A
  // round with one run only (leaves, or internal nodes) needs no network.
  // The queue of internal nodes stays in a register between rounds, reversed
  // (lane 63 - q holds node ih + q), the layout the merges read; the next
  // queue is gathered from the pair sums by a ds_bpermute.  Longer runs are
  // merged through LDS by binary searches.  A round is one wave's dependent
  // chain, so the cursors are kept scalar (readfirstlane) and stores a lane
  // does not need go to a per-lane sink instead of behind a branch.
  if (m <= kSerialUsed) {
    serial_tree(lw, iw, parl, pari, m);
  } else {
    constexpr uint64_t kPad64 = 0xFFFFFFFF0000FFFFull;  // above every real key
    constexpr uint32_t kPad32 = 0xFFFFFFFFu;
    constexpr uint32_t kKey32MaxW = (1u << 25) - 2;      // room for a 7-bit tag below kPad32
    uint16_t* par_sink = L.par + 4 * kSmallUsed + lane;  // one u16 per lane past the depth words
    uint32_t* iw_sink = iw + kSmallUsed + lane;          // one word per lane past iw
    uint32_t lc = 0, ih = 0, it = 0;
    uint32_t qrev = kInf32;  // lane 63 - q: weight of node ih + q; kInf32 past the queue
    uint32_t qreg = 1;       // qrev holds the queue (at most 64 nodes)
    uint32_t RL = lw[lane];  // leaves lc .. lc + 63 (kInf32 past m)
    for (uint32_t round = 0;; ++round) {
      const uint32_t b = uniform32(it - ih);
      if ((m - lc) + b <= 1) break;
      if (round >= m) {  // every round creates at least one node
        if (lane == 0) raise_status(status, HF_ERR_INTERNAL);
        break;
      }
      uint32_t i0, i1, last_int;
      if (__builtin_expect(qreg, 1)) {
        i0 = readlane32(qrev, 63);
        i1 = readlane32(qrev, 62);
        last_int = readlane32(qrev, (kWave - b) & 63);  // node ih + b - 1 when b > 0
      } else {  // more than 64 queued: the queue is in LDS
        const uint32_t v = iw[ih + (lane & 1)];
        i0 = readlane32(v, 0);
        i1 = readlane32(v, 1);
        last_int = readlane32(iw[it - 1], 0);
      }
      const uint32_t l0 = readlane32(RL, 0), l1 = readlane32(RL, 1);
      // the two lightest nodes, leaf first on equal weight
      const uint32_t w1 = min(l0, i0);
      const uint32_t w2 = l0 <= i0 ? min(l1, i0) : min(l0, i1);
      const uint32_t tw = w1 + w2;  // <= the sum of all counts < 2^32 - 1
      uint32_t a = (uint32_t)__popcll(__ballot(RL <= tw));
      uint32_t RL2 = kInf32;  // leaves lc + 64 .. lc + 127 when the run reaches them
      uint32_t last_leaf = readlane32(RL, (a - 1) & 63);
      if (__builtin_expect(a == (uint32_t)kWave, 0)) {
        RL2 = lw[lc + kWave + lane];
        uint32_t c = (uint32_t)__popcll(__ballot(RL2 <= tw));
        a += c;
        for (uint32_t p = lc + 2 * kWave; c == (uint32_t)kWave && p < m; p += kWave) {
          c = (uint32_t)__popcll(__ballot(lw[p + lane] <= tw));
          a += c;
        }
        a = uniform32(a);
        if (a > (uint32_t)kWave)
          last_leaf = a <= 2u * kWave ? readlane32(RL2, (a - 1) & 63) : readlane32(lw[lc + a - 1], 0);
      }
      const uint32_t total = a + b, pairs = total >> 1;
      // the heaviest node of the merge: the run's last leaf unless the last
      // internal node is heavier; an odd one out waits for the next round
      const uint32_t leaf_last = uniform32((a != 0) & ((b == 0) | (last_leaf > last_int)));
      const uint32_t carry_leaf = total & leaf_last & 1u;
      const uint32_t carry_int = total & (leaf_last ^ 1u) & 1u;
      const uint32_t maxw = leaf_last ? last_leaf : last_int;
      const uint32_t lc_next = uniform32(lc + a - carry_leaf);
      const uint32_t RL_next = lw[lc_next + lane];  // issued before the merge
      const uint32_t fast = qreg & (a <= (b == 0 ? 2u * kWave : (uint32_t)kWave));
      if (__builtin_expect(fast, 1)) {
        const int kk = (int)(63 - lane) - (int)carry_int;  // pair feeding queue slot 63 - lane
        uint32_t s0, s1 = kInf32;  // pair sums on the lanes named below
        int src;                   // lane of pair kk's sum
        if (__builtin_expect(a != 0 && b != 0, 1)) {
          const uint32_t qi = 63 - lane;
          uint32_t xw, yw = kInf32, xi, yi = 0;  // merged weights and node refs (256 + q: internal)
          if (__builtin_expect(maxw <= kKey32MaxW, 1)) {
            const uint32_t kl = lane < a ? (RL << 7 | lane) : kPad32;
            const uint32_t ki = qi < b ? (qrev << 7 | (64u + qi)) : kPad32;
            uint32_t X, Y = kPad32;
            if (__builtin_expect(a <= 32 && b <= 32, 1)) {
              X = bitonic_merge32(lane < 32 ? kl : ki);
            } else {
              X = bitonic_merge32(min(kl, ki));
              Y = bitonic_merge32(max(kl, ki));
            }
            xw = X >> 7;
            yw = Y >> 7;
            xi = (X & 63u) | ((X & 64u) << 2);
            yi = (Y & 63u) | ((Y & 64u) << 2);
          } else {
            const uint64_t kl = lane < a ? ((uint64_t)RL << 32 | lane) : kPad64;
            const uint64_t ki = qi < b ? ((uint64_t)qrev << 32 | (256u + qi)) : kPad64;
            uint64_t X, Y = kPad64;
            if (a <= 32 && b <= 32) {
              X = bitonic_merge64(lane < 32 ? kl : ki);
            } else {
              const bool sw = ki < kl;
              X = bitonic_merge64(sw ? ki : kl);
              Y = bitonic_merge64(sw ? kl : ki);
            }
            xw = (uint32_t)(X >> 32);
            yw = (uint32_t)(Y >> 32);
            xi = (uint32_t)X & 0x1FFu;
            yi = (uint32_t)Y & 0x1FFu;
          }
          s0 = xw + lane_xor<1>(xw);
          s1 = yw + lane_xor<1>(yw);
          link_merged(xi, s0, lane, pairs, lc, ih, it, parl, pari, iw, par_sink, iw_sink);
          if (total > (uint32_t)kWave) link_merged(yi, s1, kWave + lane, pairs, lc, ih, it, parl, pari, iw, par_sink, iw_sink);
          src = (2 * kk) & 63;
        } else if (b == 0) {
          // leaves only: merged position p is leaf p of the run
          s0 = RL + lane_xor<1>(RL);
          s1 = RL2 + lane_xor<1>(RL2);
          link_merged(lane, s0, lane, pairs, lc, ih, it, parl, pari, iw, par_sink, iw_sink);
          if (total > (uint32_t)kWave) link_merged(kWave + lane, s1, kWave + lane, pairs, lc, ih, it, parl, pari, iw, par_sink, iw_sink);
          src = (2 * kk) & 63;
        } else {
          // internal nodes only: node ih + q sits in lane 63 - q, pair k = nodes
          // 2k and 2k + 1, its sum on lane 63 - 2k
          const uint32_t q = 63 - lane;
          s0 = qrev + lane_xor<1>(qrev);
          const bool in_pair = q < 2 * pairs;
          *(in_pair ? pari + ih + q : par_sink) = (uint16_t)(it + (q >> 1));
          *(in_pair && !(q & 1) ? iw + it + (q >> 1) : iw_sink) = s0;
          src = (63 - 2 * kk) & 63;
        }
        uint32_t nq = (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)s0);
        if (a != 0 && total > (uint32_t)kWave) {
          const uint32_t f1 = (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)s1);
          if (kk >= 32) nq = f1;
        }
        if (kk < 0) nq = last_int;  // the carried internal node
        if (kk >= (int)pairs) nq = kInf32;
        qrev = nq;
      } else {
        merge_through_lds(lw, iw, parl, pari, lc, ih, it, a, b, pairs);
      }
      lc = lc_next;
      ih = uniform32(ih + b - carry_int);
      it = uniform32(it + pairs);
      RL = RL_next;
      if (__builtin_expect(!fast, 0)) {
        // after a merge through LDS: reload the queue when it fits a register
        const uint32_t nb = it - ih;
        qreg = nb <= (uint32_t)kWave;
        if (qreg) qrev = 63 - lane < nb ? iw[ih + 63 - lane] : kInf32;
      }
    }
    wave_sync();  // parent links complete
  }

  HF_CB_STAMP(4);
  // ---- 4. depths of internal nodes by pointer jumping ----------------------------
  // dn[k] = distance to the current jump target | target << 16, one word a node
  uint32_t* dn = (uint32_t*)(L.par + 2 * kSmallUsed);
  const uint32_t nint = m - 1, root = m - 2;
  constexpr uint32_t NR = kSmallUsed / kWave;
  uint32_t d[NR], nx[NR];
#pragma unroll
  for (uint32_t r = 0; r < NR; ++r) {
    const uint32_t k = r * kWave + lane;
    const bool valid = k < nint && k != root;
    d[r] = valid ? 1u : 0u;
    nx[r] = valid ? (uint32_t)pari[k] : root;
  }
  for (uint32_t step = 0;; ++step) {
#pragma unroll
    for (uint32_t r = 0; r < NR; ++r) {
      const uint32_t k = r * kWave + lane;
      if (k < nint) dn[k] = d[r] | nx[r] << 16;
    }
    wave_sync();
    bool active = false;
#pragma unroll
    for (uint32_t r = 0; r < NR; ++r) {
      const uint32_t v = dn[nx[r]];
      d[r] += v & 0xFFFFu;
      nx[r] = v >> 16;
      active |= nx[r] != root;
    }
    wave_sync();
    if (!__ballot(active)) break;
    if (step >= 32) {
      if (lane == 0) raise_status(status, HF_ERR_INTERNAL);
      break;
    }
  }
#pragma unroll
  for (uint32_t r = 0; r < NR; ++r) {
    const uint32_t k = r * kWave + lane;
    if (k < nint) dn[k] = d[r];
  }
  wave_sync();

  HF_CB_STAMP(5);
  // ---- 5a. leaf lengths, counts per length, total bits ---------------------------
  // Total bits in two limbs per lane (this lane's sum of count x length is
  // below 2^40), each summed exactly by a DPP scan.
  uint64_t acc = 0;
#pragma unroll
  for (uint32_t r = 0; r < NR; ++r) {
    const uint32_t e = r * kWave + lane;
    if (e < m) {
      uint32_t l = (dn[parl[e]] & 0xFFFFu) + 1;
      acc += (uint64_t)lw[e] * l;
      if (l > kMaxLen) l = kMaxLen;  // flagged below; keeps indexes in range
      const uint32_t u = lu[e];
      L.clu[u] = (uint8_t)l;
      book.cl[(uint32_t)usym[u]] = (uint8_t)l;
      atomicAdd(&L.sh.cnt[l], 1u);
    }
  }
  const uint32_t blo = wave_inclusive_scan((uint32_t)acc & 0xFFFFFFu);  // < 2^30
  const uint32_t bhi = wave_inclusive_scan((uint32_t)(acc >> 24));      // < 2^22
  const uint64_t bits = ((uint64_t)readlane32(bhi, 63) << 24) + readlane32(blo, 63);
  wave_sync();

  HF_CB_STAMP(6);
  // ---- 5b. First and Entry: lane j holds length j + 1 ---------------------------
  // The lengths present come from one ballot of the counts.  first[l] =
  // ceil((first[l+1] + cnt[l+1]) / 2) with first[Lc] = 0 unrolls to
  // ceil((2^Lc - P_l) / 2^(Lc-l)) = 2^l - floor(P_l / 2^(Lc-l)), where P_l =
  // sum over k <= l of cnt[k] 2^(Lc-k) and P_Lc = 2^Lc (the Kraft sum of a
  // full tree is 1).  With counts summing below 2^32 no code is longer than
  // 46 bits, so each term is at most 2^46 and P is summed exactly in two
  // DPP-scanned limbs.
  const uint32_t len = lane + 1;
  const uint32_t cnt = L.sh.cnt[len];
  const uint64_t present = __ballot(cnt != 0);
  const uint32_t lmax = 64 - (uint32_t)__clzll(present), lmin = (uint32_t)__builtin_ctzll(present) + 1;
  const uint32_t Lc = lmax > kMaxLen ? kMaxLen : lmax;
  const uint32_t below = wave_inclusive_scan(cnt) - cnt;  // codes shorter than len
  const uint64_t term = len <= Lc ? (uint64_t)cnt << (Lc - len) : 0ull;
  const uint32_t plo = wave_inclusive_scan((uint32_t)term & 0xFFFFFFu);  // < 2^30
  const uint32_t phi = wave_inclusive_scan((uint32_t)(term >> 24));      // < 2^28
  const uint64_t P = ((uint64_t)phi << 24) + plo;
  const uint64_t fst = len < Lc ? (1ull << len) - (P >> (Lc - len)) : 0ull;
  book.first[len] = fst;
  book.entry[len] = below;
  uint64_t* fl = (uint64_t*)L.mw;        // [65] first, by length
  uint32_t* el = (uint32_t*)(fl + 65);  // [65] entry, by length
  fl[len] = fst;
  el[len] = below;
  if (lane == 0) {
    book.first[0] = 0;
    book.entry[0] = 0;
    if (lmax > kMaxLen) raise_status(status, HF_ERR_CODELEN);
    book.info[0] = m;
    book.info[1] = lmax;
    book.info[2] = bits;
    book.info[3] = lmin;
  }
  wave_sync();

  HF_CB_STAMP(7);
  // ---- 5c. codewords: rank within each length in symbol order -------------------
  // The lanes of a 64-symbol chunk that share my length are the AND over
  // the length's 7 bits of that bit's ballot or its complement (unused
  // lanes carry length 0, which no used symbol has).  The last lane of each
  // length advances that length's next rev slot (a wave's LDS operations
  // take effect in order, so the next chunk sees it).
  uint32_t* ns = (uint32_t*)L.mw + 1536;  // [kMaxLen + 1] next rev slot per length
  ns[len] = below;
  for (uint32_t u0 = 0; u0 < m; u0 += kWave) {
    const uint32_t u = u0 + lane;
    const bool valid = u < m;
    const uint32_t l = valid ? L.clu[u] : 0u;
    uint64_t eq = ~0ull;
#pragma unroll
    for (int bit = 0; bit < 7; ++bit) {
      const bool on = (l >> bit) & 1u;
      const uint64_t B = __ballot(on);
      eq &= on ? B : ~B;
    }
    if (valid) {
      const uint32_t pos = ns[l] + (uint32_t)__popcll(eq & lanemask_lt());
      const uint32_t s = usym[u];
      book.rev[pos] = s;
      book.cw[s] = fl[l] + (pos - el[l]);
      if ((eq >> lane) == 1ull) ns[l] = pos + 1;
    }
  }
}

// cl = cw = 0 for each of symbols s0 .. s0 + 3 (below A) whose count is 0.
__device__ __forceinline__ void zero_unused(const uint32_t (&h)[4], uint32_t s0, uint32_t A, const hf_codebook& book) {
#pragma unroll
  for (uint32_t v = 0; v < 4; ++v) {
    if (h[v] == 0 && s0 + v < A) {
      book.cl[s0 + v] = 0;
      book.cw[s0 + v] = 0;
    }
  }
}

// The whole book from hist[A] by one workgroup of NT lanes.  Up to 4 NT
// symbols the histogram is read once: thread t holds the counts of symbols
// 4t .. 4t+3, wave scans (DPP) give each used symbol its compact index, the
// number of used symbols, the sum of the counts (two limbs of 24 and 10
// bits, exact) and the largest count, and a small book is compacted straight
// from those registers.
template <int NT, typename Lds>
__device__ __forceinline__ void codebook_block(const uint32_t* __restrict__ hist, const hf_codebook& book,
                                               char* ws, uint32_t* status, Lds& L, uint64_t* stamps = nullptr,
                                               bool zeroed = false) {
  constexpr uint32_t C = Lds::kCap;
  constexpr int NW = NT / kWave;
  const uint32_t A = book.alphabet;
  const uint32_t tid = threadIdx.x;
  const uint32_t lane = tid & (kWave - 1), wave = tid / kWave;
  uint32_t m = 0, wmax = 0;
  uint64_t total = 0;
  if (A <= 4u * NT) {
    uint32_t h[4], c = 0, hm = 0;
    uint64_t sum = 0;
#pragma unroll
    for (uint32_t v = 0; v < 4; ++v) {
      const uint32_t s = 4 * tid + v;
      h[v] = s < A ? hist[s] : 0u;
      c += h[v] != 0;
      sum += h[v];
      hm = max(hm, h[v]);
    }
    const uint32_t cin = wave_inclusive_scan(c);
    const uint32_t slo = wave_inclusive_scan((uint32_t)sum & 0xFFFFFFu);  // < 2^30 over a wave
    const uint32_t shi = wave_inclusive_scan((uint32_t)(sum >> 24));      // < 2^16 over a wave
    const uint32_t mx = wave_inclusive_max(hm);
    if (lane == kWave - 1) {
      L.sh.wtot[wave] = cin;
      L.sh.wsum[wave] = ((uint64_t)shi << 24) + slo;
      L.sh.wmax[wave] = mx;
    }
    __syncthreads();
    HF_CB_STAMP(1);
    uint32_t pre = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      const uint32_t t = L.sh.wtot[w];
      pre += w < (int)wave ? t : 0u;
      m += t;
      total += L.sh.wsum[w];
      wmax = max(wmax, L.sh.wmax[w]);
    }
    if (m >= 2 && m <= kSmallUsed && total < 0xFFFFFFFFull) {
      // compaction in symbol order; unused symbols get cl = cw = 0
      const uint32_t narrow = wmax < (1u << 24);
      uint32_t* key32 = small_key32(L);
      uint32_t u = pre + cin - c;
#pragma unroll
      for (uint32_t v = 0; v < 4; ++v) {
        if (h[v]) {
          if (narrow) key32[u] = h[v] << 8 | u;
          else L.key[u] = ((uint64_t)h[v] << 16) | u;
          L.usym[u] = (uint16_t)(4 * tid + v);
          ++u;
        }
      }
      build_book_small<NT>(L, m, narrow, book, status, stamps);
      // Unused symbols get cl = cw = 0 from the waves that sit out the
      // rounds (wave 1 also covers wave 0's symbols); the used ones are
      // written by wave 0, so the two never meet.
      if (wave != 0) {
        zero_unused(h, 4 * tid, A, book);
        if (wave == 1) {
          const uint32_t s0 = 4 * lane;
          uint32_t h0[4];
#pragma unroll
          for (uint32_t v = 0; v < 4; ++v) h0[v] = s0 + v < A ? hist[s0 + v] : 0u;
          zero_unused(h0, s0, A, book);
        }
      }
      return;
    }
    zero_unused(h, 4 * tid, A, book);
    __syncthreads();  // wtot is reused by the compaction
  } else {
    uint32_t c = 0, hm = 0;
    uint64_t wsum = 0;
    if (zeroed) {  // two loops: a possible store between the loads would keep them from being batched
#pragma unroll 8
      for (uint32_t s = tid; s < A; s += NT) {
        const uint32_t h = hist[s];
        c += (h != 0);
        wsum += h;
        hm = max(hm, h);
      }
    } else {
#pragma unroll 8
      for (uint32_t s = tid; s < A; s += NT) {
        const uint32_t h = hist[s];
        c += (h != 0);
        wsum += h;
        hm = max(hm, h);
        if (!h) {  // unused: no code (lane-contiguous stores)
          book.cl[s] = 0;
          book.cw[s] = 0;
        }
      }
    }
    wsum = wave_sum_u64(wsum);
    hm = wave_max_u32(hm);
    if (lane == 0) {
      L.sh.wsum[wave] = wsum;
      L.sh.wmax[wave] = hm;
    }
    (void)block_exclusive_scan<NW>(c, L.sh.wtot, &m);  // (its barrier covers wsum and wmax)
    HF_CB_STAMP(1);
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      total += L.sh.wsum[w];
      wmax = max(wmax, L.sh.wmax[w]);
    }
    __syncthreads();  // wtot is reused by the compaction
    if (m >= 2 && m <= kSmallUsed && total < 0xFFFFFFFFull) {
      compact<NT>(hist, A, L.key, L.usym, book, L.sh.wtot);  // 64-bit keys
      build_book_small<NT>(L, m, 0, book, status, stamps);
      return;
    }
  }

  if (m <= C) {
    Tree<uint16_t> t;
    t.key = L.key;
    t.iw = L.iw;
    t.mw = L.mw;
    t.mid = L.mid;
    t.par = L.par;
    t.usym = L.usym;
    t.clu = L.clu;
    t.dA = (uint16_t*)L.mw;
    t.dB = t.dA + C;
    t.nA = t.dB + C;
    t.nB = t.nA + C;
    build_book<uint16_t, NT>(t, L.sh, hist, A, m, wmax, book, status, (uint32_t*)L.iw, stamps);
  } else {
    const GlobalLayout G = global_layout(A);
    Tree<uint32_t> t;
    t.key = (uint64_t*)(ws + G.key);
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
    build_book<uint32_t, NT>(t, L.sh, hist, A, m, wmax, book, status, (uint32_t*)L.iw, stamps);
  }
}

// Batched stage 3 for one stream: its book from its histogram, by one
// workgroup of NT lanes (an empty stream's histogram is zeroed here and its
// one offset set).
template <int NT, typename Lds>
__device__ __forceinline__ void batch_codebook_item(const BatchStream& bs, Lds& L) {
  if (bs.n == 0) {
    for (uint32_t b = threadIdx.x; b < bs.A; b += NT) bs.hist[b] = 0;
    if (threadIdx.x == 0) bs.offsets[0] = 0;
    __threadfence_block();
    __syncthreads();
  }
  codebook_block<NT>(bs.hist, bs.book, bs.cb_ws, bs.status, L);
}

}  // namespace
}  // namespace hf
