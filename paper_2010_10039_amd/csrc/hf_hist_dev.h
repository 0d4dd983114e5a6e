// hf_hist_dev.h -- device code of stage 1, histogramming (Sec. 4.1 of the
// paper): LDS replicas of the bin window and the per-slab batched counts.
// Internal to libhf; the kernels and launchers are in hf_histogram.hip.
#pragma once

#include "hf_device.h"
#include "hf_kernels.h"

namespace hf {

template <int SB>
__device__ __forceinline__ uint32_t sym_load(const void* p, uint64_t i) {
  if (SB == 1) return ((const uint8_t*)p)[i];
  return ((const uint16_t*)p)[i];
}

// LDS words between replicas: the window (plus the trash bin when it holds
// the whole alphabet) rounded up to 1 mod 32, so bin b of replica r sits on
// bank (b + r) mod 32 and lanes of different replicas that hit a popular bin
// use different banks.
__host__ __device__ inline uint32_t hist_stride(uint32_t W, uint32_t A) {
  const uint32_t w = W == A ? W + 1 : W;
  return (w + 30) / 32 * 32 + 1;
}

// Count one symbol into the lane's replica of the LDS window.
__device__ __forceinline__ void hist_count(uint32_t* subr, uint32_t s, uint32_t lo, uint32_t W, uint32_t A,
                                           bool& bad) {
  uint32_t b = s - lo;  // wraps for s < lo
  if (b < W) atomicAdd(&subr[b], 1u);
  bad |= (s >= A);
}

template <int SB>
__device__ __forceinline__ void hist_count_vec(uint32_t* subr, uint4 v, uint32_t lo, uint32_t W, uint32_t A,
                                               bool& bad) {
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (SB == 1) {
#pragma unroll
      for (int j = 0; j < 4; ++j) hist_count(subr, (w[k] >> (8 * j)) & 0xFFu, lo, W, A, bad);
    } else {
      hist_count(subr, w[k] & 0xFFFFu, lo, W, A, bad);
      hist_count(subr, w[k] >> 16, lo, W, A, bad);
    }
  }
}

// Whole alphabet in LDS: a symbol outside it is counted in the trash bin A
// (no branch); a non-zero trash count flags it at the end.
__device__ __forceinline__ void hist_count_all(uint32_t* subr, uint32_t s, uint32_t A) {
  atomicAdd(&subr[min(s, A)], 1u);
}

template <int SB>
__device__ __forceinline__ void hist_count_vec_all(uint32_t* subr, uint4 v, uint32_t A) {
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (SB == 1) {
#pragma unroll
      for (int j = 0; j < 4; ++j) hist_count_all(subr, (w[k] >> (8 * j)) & 0xFFu, A);
    } else {
      hist_count_all(subr, w[k] & 0xFFFFu, A);
      hist_count_all(subr, w[k] >> 16, A);
    }
  }
}

// Counts symbols [s_lo, s_hi) into the lane's replica `subr` of the LDS
// window: scalar head up to the first 16-byte boundary, 16-byte vectors
// (four in flight per lane), scalar tail.  ALL: the window is the whole
// alphabet plus a trash bin (lo = 0, W = A); otherwise symbols outside
// [lo, lo + W) are skipped.
template <int SB, bool ALL>
__device__ __forceinline__ void hist_range(uint32_t* subr, const void* __restrict__ sym, uint64_t s_lo,
                                           uint64_t s_hi, uint32_t lo, uint32_t W, uint32_t A, bool& bad) {
  constexpr uint32_t kPerVec = 16 / SB;
  const uint32_t tid = threadIdx.x;
  const uintptr_t addr = (uintptr_t)sym + s_lo * SB;
  uint64_t head = ((16 - (addr & 15)) & 15) / SB;
  if (head > s_hi - s_lo) head = s_hi - s_lo;
  const uint64_t nvec = (s_hi - s_lo - head) / kPerVec;
  const uint4* body = (const uint4*)((const char*)sym + (s_lo + head) * SB);
  uint64_t v = tid;
  constexpr int kUnroll = 4;
  for (; v + (kUnroll - 1) * (uint64_t)blockDim.x < nvec; v += kUnroll * (uint64_t)blockDim.x) {
    uint4 q[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) q[u] = body[v + u * (uint64_t)blockDim.x];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if (ALL) hist_count_vec_all<SB>(subr, q[u], A);
      else hist_count_vec<SB>(subr, q[u], lo, W, A, bad);
    }
  }
  for (; v < nvec; v += blockDim.x) {
    if (ALL) hist_count_vec_all<SB>(subr, body[v], A);
    else hist_count_vec<SB>(subr, body[v], lo, W, A, bad);
  }
  for (uint64_t i = tid; i < head; i += blockDim.x) {
    if (ALL) hist_count_all(subr, sym_load<SB>(sym, s_lo + i), A);
    else hist_count(subr, sym_load<SB>(sym, s_lo + i), lo, W, A, bad);
  }
  for (uint64_t i = s_lo + head + nvec * kPerVec + tid; i < s_hi; i += blockDim.x) {
    if (ALL) hist_count_all(subr, sym_load<SB>(sym, i), A);
    else hist_count(subr, sym_load<SB>(sym, i), lo, W, A, bad);
  }
}

// Interleaved replicas (bin b of replica r at word b R + r, lane l using
// replica l mod R) over the whole alphabet plus the trash bin A: lanes of
// different replicas that hit one bin use R consecutive banks, and
// neighbouring bins are R banks apart (peaked data sits on neighbouring
// bins).  Loads as in hist_range.
__device__ __forceinline__ void hist_count_il(uint32_t* subr, uint32_t s, uint32_t A, uint32_t R) {
  atomicAdd(&subr[min(s, A) * R], 1u);
}

template <int SB>
__device__ __forceinline__ void hist_count_vec_il(uint32_t* subr, uint4 v, uint32_t A, uint32_t R) {
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (SB == 1) {
#pragma unroll
      for (int j = 0; j < 4; ++j) hist_count_il(subr, (w[k] >> (8 * j)) & 0xFFu, A, R);
    } else {
      hist_count_il(subr, w[k] & 0xFFFFu, A, R);
      hist_count_il(subr, w[k] >> 16, A, R);
    }
  }
}

template <int SB>
__device__ __forceinline__ void hist_range_il(uint32_t* sub, uint32_t R, const void* __restrict__ sym,
                                              uint64_t s_lo, uint64_t s_hi, uint32_t A) {
  constexpr uint32_t kPerVec = 16 / SB;
  const uint32_t tid = threadIdx.x;
  uint32_t* const subr = sub + (tid & (R - 1));
  const uintptr_t addr = (uintptr_t)sym + s_lo * SB;
  uint64_t head = ((16 - (addr & 15)) & 15) / SB;
  if (head > s_hi - s_lo) head = s_hi - s_lo;
  const uint64_t nvec = (s_hi - s_lo - head) / kPerVec;
  const uint4* body = (const uint4*)((const char*)sym + (s_lo + head) * SB);
  uint64_t v = tid;
  constexpr int kUnroll = 4;
  for (; v + (kUnroll - 1) * (uint64_t)blockDim.x < nvec; v += kUnroll * (uint64_t)blockDim.x) {
    uint4 q[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) q[u] = body[v + u * (uint64_t)blockDim.x];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) hist_count_vec_il<SB>(subr, q[u], A, R);
  }
  for (; v < nvec; v += blockDim.x) hist_count_vec_il<SB>(subr, body[v], A, R);
  for (uint64_t i = tid; i < head; i += blockDim.x) hist_count_il(subr, sym_load<SB>(sym, s_lo + i), A, R);
  for (uint64_t i = s_lo + head + nvec * kPerVec + tid; i < s_hi; i += blockDim.x)
    hist_count_il(subr, sym_load<SB>(sym, i), A, R);
}

// Words of LDS a window needs: R replicas, hist_stride words apart.
__host__ __device__ inline uint32_t hist_window_words(uint32_t W, uint32_t A, uint32_t R) {
  return hist_stride(W, A) * R;
}

// Batched stage 1 for work item (stream bs, slab g): the slab's counts into
// its row of bs.part.  The LDS holds lds_words words: as many replicas of
// the alphabet as fit.
__device__ __forceinline__ void batch_hist_item(const BatchStream& bs, uint32_t g, uint32_t* sub, uint32_t lds_words) {
  const uint32_t A = bs.A;
  const uint32_t Wp = hist_stride(A, A);
  uint32_t R = 1;
  while (R < 16 && Wp * R * 2 <= lds_words) R *= 2;
  const uint32_t tid = threadIdx.x;
  for (uint32_t i = tid; i < (A + 1) * R; i += blockDim.x) sub[i] = 0;
  __syncthreads();
  const uint64_t s_lo = slab_begin(g, bs.nblocks, bs.nslabs, bs.n);
  const uint64_t s_hi = slab_begin(g + 1, bs.nblocks, bs.nslabs, bs.n);
  bool bad = false;
  if (bs.sym_bytes == 1) hist_range_il<1>(sub, R, bs.sym, s_lo, s_hi, A);
  else hist_range_il<2>(sub, R, bs.sym, s_lo, s_hi, A);
  __syncthreads();
  uint32_t* row = bs.part + (uint64_t)g * A;
  for (uint32_t b = tid; b < A; b += blockDim.x) {
    uint32_t c = 0;
    for (uint32_t r = 0; r < R; ++r) c += sub[b * R + r];
    row[b] = c;
  }
  if (tid < R && sub[A * R + tid]) bad = true;
  if (bad) raise_status(bs.status, HF_ERR_SYMBOL);
}

// Batched stage 2 for stream bs and bins [256 c, 256 c + 256): the counts
// of every slab into its histogram (coalesced row segments, one store per
// bin), by kBatchReduceBins lanes.
__device__ __forceinline__ void batch_reduce_item(const BatchStream& bs, uint32_t c) {
  const uint32_t b = c * kBatchReduceBins + threadIdx.x;
  if (b >= bs.A) return;
  const uint32_t* p = bs.part + b;
  uint32_t n = 0;
#pragma unroll 8
  for (uint32_t g = 0; g < bs.nslabs; ++g) n += p[(uint64_t)g * bs.A];
  bs.hist[b] = n;
}

}  // namespace hf
