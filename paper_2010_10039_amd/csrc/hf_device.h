// hf_device.h -- device-side helpers shared by the libhf kernels (gfx950,
// wave64).  Internal to libhf.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hf.h"

namespace hf {

constexpr int kWave = 64;

// First error wins: only a zero status is replaced.
__device__ __forceinline__ void raise_status(uint32_t* status, uint32_t code) {
  atomicCAS(status, 0u, code);
}

// Relaxed agent-scope atomics: visible across all XCDs of the device without
// ordering any other memory.  Used for self-contained 64-bit records.
__device__ __forceinline__ uint64_t load_agent(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_agent(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Bits of lanes strictly below this one.
__device__ __forceinline__ uint64_t lanemask_lt() {
  int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Inclusive prefix sum over the wave with DPP lane moves (no LDS): shifts by
// 1, 2, 4, 8 within each 16-lane row, then row 0's total into row 1 and row
// 2's into row 3 (row_bcast:15), then rows 0-1's total into rows 2-3
// (row_bcast:31).  Lanes with no source read 0.
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, true);  // row_shr:1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, true);  // row_shr:2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, true);  // row_shr:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, true);  // row_shr:8
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return v;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v = max(v, (uint32_t)__shfl_xor(v, d, kWave));
  return v;
}

// Exclusive scan over the whole workgroup (blockDim.x = 64 * NW).  `wtot`
// is an LDS array of NW words; *total receives the workgroup sum.  Contains
// one barrier; the caller must not overwrite `wtot` until every thread has
// returned (i.e. until its next barrier).
template <int NW>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* wtot, uint32_t* total) {
  const int lane = lane_id();
  const int w = threadIdx.x / kWave;
  uint32_t inc = wave_inclusive_scan(v);
  if (lane == kWave - 1) wtot[w] = inc;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    uint32_t t = wtot[i];
    pre += (i < w) ? t : 0u;
    tot += t;
  }
  *total = tot;
  return pre + inc - v;
}

template <int SB>
__device__ __forceinline__ uint32_t sym_at(const void* p, uint64_t i) {
  return SB == 1 ? (uint32_t)((const uint8_t*)p)[i] : (uint32_t)((const uint16_t*)p)[i];
}

// Last 32 content bits of the symbols [s_lo, s_hi) (right aligned, fewer if
// the content is shorter), computed by wave 0: lane j codes symbol s_hi-1-j.
template <int SB>
__device__ __forceinline__ uint32_t range_tail(const void* sym, uint64_t s_lo, uint64_t s_hi, uint32_t A,
                                               const uint8_t* cl, const uint64_t* cw) {
  const uint32_t lane = lane_id();
  uint32_t l = 0;
  uint64_t c = 0;
  if (lane < 32 && s_hi - s_lo > lane) {
    const uint32_t s = sym_at<SB>(sym, s_hi - 1 - lane);
    if (s < A) {
      l = cl[s];
      c = cw[s];
    }
  }
  // bits already taken by lanes nearer the end
  const uint32_t off = wave_inclusive_scan(l) - l;
  uint32_t part = (off < 32) ? (uint32_t)(c << off) : 0u;
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) part |= (uint32_t)__shfl_xor(part, d, kWave);
  return part;
}

}  // namespace hf
