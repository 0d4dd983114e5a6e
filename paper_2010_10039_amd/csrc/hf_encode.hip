// hf_encode.hip -- stage 4: encoding and bit concatenation (Sec. 4.3 of the
// paper: reduce-merge, shuffle-merge, blockwise code-length prefix sum and
// the coalescing copy of Table 1).
//
// The paper encodes a chunk of 2^M symbols with M merge rounds: r rounds of
// reduce-merge inside a thread, then s = M - r rounds of shuffle-merge in
// which right groups of 32-bit words are appended to left groups; chunks are
// then stitched with a prefix sum of their lengths and an optional gathering
// copy.  Here one workgroup of 256 lanes encodes a tile of 256 * 2^r
// symbols:
//  - reduce-merge: each lane looks up 2^r consecutive symbols in an LDS
//    codebook (packed cw << 5 | cl when every code has <= 27 bits) and
//    concatenates them in a 64-bit register, so codes up to 64 bits need no
//    side channel (the paper filters merged words over 32 bits out);
//  - shuffle-merge: the s pairwise append rounds collapse into one
//    workgroup exclusive scan of the lane bit counts, after which every lane
//    ORs its words into an LDS tile buffer at its bit offset (no contention
//    beyond the one word shared with each neighbour);
//  - tile offsets: single-pass decoupled look-back (Merrill & Garland) over
//    per-tile records {flag, aggregate | inclusive prefix} instead of a
//    separate prefix-sum kernel;
//  - gathering: the tile buffer, assembled at bit alignment 0, is written to
//    its final bit position in HBM with a funnel shift and coalesced stores.
//    The word shared with the previous tile belongs to this tile, which
//    completes it from the previous tile's published last 32 bits, so every
//    output word is stored exactly once with a plain store.
// Chunk offsets (the paper's per-chunk metadata) are the bit positions of
// the lanes that start a chunk, so the stream does not depend on the chunk
// size or on r.  Tiles are handed out by an atomic ticket so a tile only
// waits on tiles already taken by running workgroups.
#include <algorithm>

#include "hf_device.h"
#include "hf_kernels.h"

namespace hf {

namespace {

constexpr uint64_t kFlagAgg = 1ull << 62;
constexpr uint64_t kFlagIncl = 2ull << 62;
constexpr uint64_t kValueMask = (1ull << 62) - 1;
constexpr uint64_t kTailValid = 1ull << 32;
// Upper bound on polls of another tile's record (~0.5 s of sleeping polls);
// reaching it means a bug, reported as HF_ERR_INTERNAL instead of a hang.
constexpr uint32_t kSpinLimit = 1u << 22;

struct EncShared {
  uint32_t wtot[kEncWaves];
  uint32_t tile[2];
  uint64_t G;
  uint32_t pred_tail;
};

template <int NS, int SB>
__device__ __forceinline__ void load_symbols(const void* __restrict__ sym, uint64_t s0, uint64_t n,
                                             bool vec_ok, uint32_t (&v)[NS], uint32_t& nvalid) {
  if (s0 + NS <= n) {
    nvalid = NS;
    constexpr int kBytes = NS * SB;
    const char* p = (const char*)sym + s0 * SB;
    if constexpr (kBytes >= 4) {
      if (vec_ok) {
        constexpr int kWords = kBytes / 4;
        uint32_t w[kWords];
        if constexpr (kBytes >= 16) {
#pragma unroll
          for (int k = 0; k < kBytes / 16; ++k) {
            const uint4 q = ((const uint4*)p)[k];
            w[4 * k + 0] = q.x;
            w[4 * k + 1] = q.y;
            w[4 * k + 2] = q.z;
            w[4 * k + 3] = q.w;
          }
        } else if constexpr (kBytes == 8) {
          const uint2 q = *(const uint2*)p;
          w[0] = q.x;
          w[1] = q.y;
        } else {
          w[0] = *(const uint32_t*)p;
        }
#pragma unroll
        for (int i = 0; i < NS; ++i) {
          if (SB == 1) v[i] = (w[i / 4] >> (8 * (i % 4))) & 0xFFu;
          else v[i] = (w[i / 2] >> (16 * (i % 2))) & 0xFFFFu;
        }
        return;
      }
    }
    {
#pragma unroll
      for (int i = 0; i < NS; ++i)
        v[i] = (SB == 1) ? (uint32_t)((const uint8_t*)sym)[s0 + i] : (uint32_t)((const uint16_t*)sym)[s0 + i];
    }
  } else {
    nvalid = s0 < n ? (uint32_t)(n - s0) : 0u;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      v[i] = 0;
      if ((uint32_t)i < nvalid)
        v[i] = (SB == 1) ? (uint32_t)((const uint8_t*)sym)[s0 + i] : (uint32_t)((const uint16_t*)sym)[s0 + i];
    }
  }
}

// Append `len` (<= 32) bits of `code` to the lane accumulator; full 32-bit
// words go to the tile buffer (the first and last may be shared with the
// neighbouring lanes, hence the OR).
__device__ __forceinline__ void push_bits(uint64_t& acc, uint32_t& nb, uint32_t& wi, uint32_t* buf,
                                          uint32_t code, uint32_t len) {
  acc = (len == 32) ? ((acc << 32) | code) : ((acc << len) | code);
  nb += len;
  if (nb >= 32) {
    nb -= 32;
    atomicOr(&buf[wi++], (uint32_t)(acc >> nb));
  }
}

template <int R, int SB>
__global__ __launch_bounds__(kEncThreads) void encode_kernel(
    const void* __restrict__ sym, uint64_t n, uint32_t A, const uint8_t* __restrict__ cl,
    const uint64_t* __restrict__ cw, const uint64_t* __restrict__ info, uint32_t* __restrict__ out,
    uint64_t cap_words, uint64_t* __restrict__ offsets, uint32_t chunk_log2, uint64_t nchunks,
    uint32_t* __restrict__ ticket, uint64_t* __restrict__ lookback, uint64_t* __restrict__ tails,
    uint32_t ntiles, uint32_t* __restrict__ status, uint32_t table_ok, uint32_t vec_ok) {
  constexpr uint32_t NS = 1u << R;
  constexpr uint32_t T = kEncThreads * NS;
  extern __shared__ uint32_t lds[];
  __shared__ EncShared sh;

  const uint32_t tid = threadIdx.x;
  const uint32_t lane = tid & (kWave - 1);
  const uint32_t wave = tid / kWave;
  const uint32_t lmax = (uint32_t)info[1];
  const bool packed = table_ok && lmax <= kPackedMaxLen;
  uint32_t* tab = lds;
  uint32_t* buf = lds + (packed ? A : 0u);
  const uint32_t buf_words = packed ? (T * kPackedMaxLen + 31) / 32 + 2 : 2 * T + 2;

  if (packed)
    for (uint32_t s = tid; s < A; s += kEncThreads) {
      const uint32_t l = cl[s];
      tab[s] = l ? (((uint32_t)cw[s]) << 5) | l : 0u;
    }
  for (uint32_t i = tid; i < buf_words; i += kEncThreads) buf[i] = 0;
  if (tid == 0) sh.tile[0] = atomicAdd(ticket, 1u);
  __syncthreads();

  for (uint32_t it = 0;; ++it) {
    const uint32_t tile = sh.tile[it & 1];
    if (tile >= ntiles) break;
    if (tid == 0) sh.tile[(it + 1) & 1] = atomicAdd(ticket, 1u);
    const bool last = tile == ntiles - 1;
    const uint64_t s0 = (uint64_t)tile * T + (uint64_t)tid * NS;

    // ---- lookup: lane bit count --------------------------------------------
    uint32_t e[NS];
    uint32_t nvalid;
    load_symbols<NS, SB>(sym, s0, n, vec_ok != 0, e, nvalid);
    uint32_t L = 0;
    bool bad = false;
    if (packed) {
#pragma unroll
      for (uint32_t i = 0; i < NS; ++i) {
        uint32_t ent = 0;
        if (i < nvalid) {
          ent = e[i] < A ? tab[e[i]] : 0u;
          bad |= ent == 0;
        }
        e[i] = ent;
        L += ent & 31;
      }
    } else {
#pragma unroll
      for (uint32_t i = 0; i < NS; ++i) {
        if (i < nvalid) {
          const uint32_t l = e[i] < A ? cl[e[i]] : 0u;
          bad |= l == 0;
          L += l;
        }
      }
    }
    if (bad) raise_status(status, HF_ERR_SYMBOL);

    // ---- shuffle-merge offsets: workgroup scan --------------------------------
    uint32_t B;
    const uint32_t P = block_exclusive_scan<kEncWaves>(L, sh.wtot, &B);
    if (tid == 0) store_agent(&lookback[tile], (tile == 0 ? kFlagIncl : kFlagAgg) | (uint64_t)B);

    // ---- reduce-merge into the tile buffer ------------------------------------
    {
      uint64_t acc = 0;
      uint32_t nb = P & 31;
      uint32_t wi = P >> 5;
      if (packed) {
#pragma unroll
        for (uint32_t i = 0; i < NS; ++i) push_bits(acc, nb, wi, buf, e[i] >> 5, e[i] & 31);
      } else {
#pragma unroll
        for (uint32_t i = 0; i < NS; ++i) {
          const uint32_t s = e[i];
          if (i >= nvalid || s >= A) continue;
          const uint32_t l = cl[s];
          const uint64_t c = cw[s];
          if (l > 32) {
            push_bits(acc, nb, wi, buf, (uint32_t)(c >> 32), l - 32);
            push_bits(acc, nb, wi, buf, (uint32_t)c, 32);
          } else if (l > 0) {
            push_bits(acc, nb, wi, buf, (uint32_t)c, l);
          }
        }
      }
      if (nb) atomicOr(&buf[wi], (uint32_t)(acc << (32 - nb)));
    }
    __syncthreads();

    // ---- tail record + decoupled look-back (wave 0) ----------------------------
    if (wave == 0) {
      if (lane == 0 && !last) {
        uint32_t tail;
        if (B >= 32) {
          const uint32_t o = B & 31, w = (B >> 5) - 1;
          tail = o ? ((buf[w] << o) | (buf[w + 1] >> (32 - o))) : buf[w];
        } else {
          tail = B ? (buf[0] >> (32 - B)) : 0u;
        }
        store_agent(&tails[tile], kTailValid | tail);
      }
      uint64_t G = 0;
      uint32_t spins = 0;
      if (tile > 0) {
        int64_t top = (int64_t)tile - 1;
        for (;;) {
          const int64_t idx = top - (int64_t)lane;
          const uint64_t v = idx >= 0 ? load_agent(&lookback[idx]) : kFlagIncl;
          const uint64_t flag = v >> 62;
          const uint64_t incl = __ballot(flag == 2);
          const uint64_t empty = __ballot(flag == 0);
          const int fi = incl ? __ffsll((unsigned long long)incl) - 1 : 64;
          const uint64_t need = fi >= 63 ? ~0ull : ((2ull << fi) - 1);
          if ((empty & need) && ++spins < kSpinLimit) {
            __builtin_amdgcn_s_sleep(1);
            continue;
          }
          if (spins >= kSpinLimit) {
            if (lane == 0) raise_status(status, HF_ERR_INTERNAL);
            break;
          }
          G += wave_sum_u64((int)lane <= fi ? (v & kValueMask) : 0ull);
          if (fi < 64) break;
          top -= kWave;
        }
      }
      if (lane == 0) {
        if (tile > 0) store_agent(&lookback[tile], kFlagIncl | (G + B));
        sh.G = G;
        uint32_t pred = 0;
        if (tile > 0 && (G & 31)) {
          uint64_t tv;
          for (uint32_t k = 0;; ++k) {
            tv = load_agent(&tails[tile - 1]);
            if (tv & kTailValid) break;
            if (k >= kSpinLimit) {
              raise_status(status, HF_ERR_INTERNAL);
              break;
            }
            __builtin_amdgcn_s_sleep(1);
          }
          pred = (uint32_t)tv;
        }
        sh.pred_tail = pred;
      }
    }
    __syncthreads();

    // ---- gathering: funnel-shifted coalesced stores ------------------------------
    const uint64_t G = sh.G;
    const uint32_t q = (uint32_t)(G & 31);
    const uint64_t w0 = G >> 5;
    const uint64_t end_bit = G + B;
    uint64_t wend = (end_bit + 31) >> 5;
    if (!last && (end_bit & 31)) wend -= 1;  // the next tile owns the shared word
    const uint32_t nw = (uint32_t)(wend - w0);
    const uint32_t pred = sh.pred_tail;
    for (uint32_t i = tid; i < nw; i += kEncThreads) {
      uint32_t v;
      if (q == 0) {
        v = buf[i];
      } else {
        const uint32_t hi = i == 0 ? pred : buf[i - 1];
        v = (hi << (32 - q)) | (buf[i] >> q);
      }
      const uint64_t wi = w0 + i;
      if (wi < cap_words) out[wi] = v;
    }
    if (s0 < n && (s0 & ((1ull << chunk_log2) - 1)) == 0) offsets[s0 >> chunk_log2] = G + P;
    if (last && tid == 0) {
      offsets[nchunks] = end_bit;
      if (end_bit > 32ull * cap_words) raise_status(status, HF_ERR_CAPACITY);
    }
    __syncthreads();
    // clear what this tile used (one word past the content is read above)
    const uint32_t used = (B + 31) / 32 + 1;
    for (uint32_t i = tid; i < used; i += kEncThreads) buf[i] = 0;
  }
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

inline uint64_t tiles_for(uint64_t n, uint32_t r) {
  const uint64_t T = (uint64_t)kEncThreads << r;
  return (n + T - 1) / T;
}

using EncodeFn = void (*)(const void*, uint64_t, uint32_t, const uint8_t*, const uint64_t*,
                          const uint64_t*, uint32_t*, uint64_t, uint64_t*, uint32_t, uint64_t,
                          uint32_t*, uint64_t*, uint64_t*, uint32_t, uint32_t*, uint32_t, uint32_t);

template <int R>
EncodeFn pick_sb(uint32_t sb) {
  return sb == 1 ? (EncodeFn)encode_kernel<R, 1> : (EncodeFn)encode_kernel<R, 2>;
}

EncodeFn pick(uint32_t r, uint32_t sb) {
  switch (r) {
    case 1: return pick_sb<1>(sb);
    case 2: return pick_sb<2>(sb);
    case 3: return pick_sb<3>(sb);
    case 4: return pick_sb<4>(sb);
    case 5: return pick_sb<5>(sb);
    default: return pick_sb<6>(sb);
  }
}

// Occupancy-sized persistent grid, cached per kernel and LDS size.
struct OccEntry {
  const void* fn;
  size_t lds;
  int blocks;
};
OccEntry g_occ[64];
int g_nocc = 0;

int blocks_per_cu(EncodeFn fn, size_t lds) {
  for (int i = 0; i < g_nocc; ++i)
    if (g_occ[i].fn == (const void*)fn && g_occ[i].lds == lds) return g_occ[i].blocks;
  if (lds > (64u << 10))
    (void)hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)fn, kEncThreads, lds) != hipSuccess || nb < 1)
    nb = 1;
  if (g_nocc < 64) g_occ[g_nocc++] = {(const void*)fn, lds, nb};
  return nb;
}

}  // namespace

size_t encode_workspace_bytes(uint64_t n, uint32_t r) {
  const uint64_t nt = tiles_for(n, r);
  return 256 + 2 * align256(nt * 8);
}

EncodeWorkspace encode_workspace_layout(void* ws, uint64_t n, uint32_t r) {
  const uint64_t nt = tiles_for(n, r);
  char* p = (char*)ws;
  EncodeWorkspace w;
  w.ticket = (uint32_t*)p;
  w.lookback = (uint64_t*)(p + 256);
  w.tails = (uint64_t*)(p + 256 + align256(nt * 8));
  return w;
}

hipError_t launch_encode(const void* sym, uint64_t n, uint32_t sym_bytes, const hf_codebook& book,
                         uint32_t chunk_log2, uint32_t r, uint32_t* out, uint64_t cap_words,
                         uint64_t* offsets, void* ws, uint32_t* status, int num_cus,
                         hipStream_t stream, const KernelTimer& timer) {
  const uint64_t nchunks = (n + (1ull << chunk_log2) - 1) >> chunk_log2;
  if (n == 0) {
    hipError_t e = launch_fill_u64(offsets, 1, 0, stream);
    timer.before(stream);
    timer.after(stream);
    return e;
  }
  const uint64_t ntiles = tiles_for(n, r);
  const EncodeWorkspace w = encode_workspace_layout(ws, n, r);
  // one fill clears the ticket and every look-back and tail record
  const uint64_t clear_words = (256 + 2 * align256(ntiles * 8)) / 8;
  hipError_t e = launch_fill_u64((uint64_t*)ws, clear_words, 0, stream);
  if (e != hipSuccess) return e;

  const uint32_t T = (uint32_t)kEncThreads << r;
  const uint32_t A = book.alphabet;
  const uint32_t table_ok = A <= kPackedMaxAlphabet ? 1u : 0u;
  const size_t packed_words = table_ok ? (size_t)A + (T * kPackedMaxLen + 31) / 32 + 2 : 0;
  const size_t wide_words = 2 * (size_t)T + 2;
  const size_t lds = 4 * (packed_words > wide_words ? packed_words : wide_words);
  const uint32_t vec_ok = ((uintptr_t)sym % 16) == 0 ? 1u : 0u;
  EncodeFn fn = pick(r, sym_bytes);
  const int nb = blocks_per_cu(fn, lds);
  const uint64_t grid = std::min<uint64_t>(ntiles, (uint64_t)num_cus * nb);
  timer.before(stream);
  hipLaunchKernelGGL(fn, dim3((uint32_t)grid), dim3(kEncThreads), lds, stream, sym, n, A, book.cl,
                     book.cw, book.info, out, cap_words, offsets, chunk_log2, nchunks, w.ticket,
                     w.lookback, w.tails, (uint32_t)ntiles, status, table_ok, vec_ok);
  e = hipGetLastError();
  timer.after(stream);
  return e;
}

}  // namespace hf
