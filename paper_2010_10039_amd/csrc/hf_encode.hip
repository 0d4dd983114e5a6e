// hf_encode.hip -- stage 4: encoding and bit concatenation (Sec. 4.3 of the
// paper: reduce-merge, shuffle-merge, blockwise code-length prefix sum and
// the coalescing copy of Table 1).
//
// The paper encodes each chunk of 2^M symbols with M merge rounds (r rounds
// of reduce-merge inside a thread, then s = M - r rounds of shuffle-merge
// that append right groups of 32-bit words to left groups), then needs a
// prefix sum of the chunk lengths and an optional gathering copy to make
// the stream dense.  Here the stream is cut into slabs (whole 4096-symbol
// blocks, one workgroup each), and:
//  - slab offsets: a slab's bit total is sum_s count_g[s] * cl[s], taken from
//    the per-slab counts the histogram pass already produced (or, without
//    them, from one counting pass); each workgroup adds its predecessors'
//    totals.  No flags, no waiting between workgroups, no cleared state;
//  - reduce-merge: each lane looks up 2^r consecutive symbols (packed
//    cw << 5 | cl table in LDS when codes fit 27 bits) and concatenates their
//    codes in a 64-bit register, so codes up to 64 bits need no side
//    channel (the paper filters merged words over 32 bits out);
//  - shuffle-merge: the s pairwise append rounds become one workgroup scan of
//    lane bit counts, after which each lane ORs its words into an LDS tile
//    buffer at its bit offset;
//  - gathering: the tile buffer (bit alignment 0) is stored to its final
//    position with a funnel shift and coalesced 32-bit stores.  A word shared
//    with the previous tile belongs to the later tile, which completes it
//    from the earlier tile's last 32 bits (kept in LDS inside a slab and
//    computed by the prepass across slabs), so every output word is stored
//    once with a plain store.
// Chunk offsets are the bit positions of the lanes that start a chunk, so
// the stream does not depend on the chunk size, on r or on the slabs.
#include <algorithm>
#include <mutex>

#include "hf_codebook_dev.h"
#include "hf_device.h"
#include "hf_hist_dev.h"
#include "hf_kernels.h"

namespace hf {

namespace {

// The LDS tile buffer holds codes of up to this many bits per symbol.
constexpr uint32_t kLdsBufMaxLen = 32;
constexpr uint32_t kTableMaxAlphabet = 8192;
constexpr int kPreThreads = 256;
constexpr int kPreWaves = kPreThreads / kWave;

// Encoding modes, chosen per launch from the codebook's longest code:
//   kModeTable : codes <= 27 bits, alphabet <= 8192: packed table (code
//                left-aligned, 32 - cl in the low 5 bits) and tile buffer
//                in LDS;
//   kModeSplit : codes of 28 .. 31 bits, alphabet <= 4096: left-aligned
//                codes and a byte table of 32 - cl in LDS;
//   kModeGTable: codes <= 27 bits, alphabet above 8192: the table mode's
//                packed entries in the workspace (read through L2), tile
//                buffer in LDS;
//   kModeGlobal: codes <= 32 bits: codebook read from global memory (L2),
//                tile buffer in LDS;
//   kModeWide  : longer codes: codebook from global memory and bits ORed
//                straight into the output words the tile owns.
constexpr int kModeTable = 0;
constexpr int kModeGlobal = 1;
constexpr int kModeWide = 2;
constexpr int kModeSplit = 3;
constexpr int kModeGTable = 4;
constexpr uint32_t kSplitMaxLen = 31;  // 32 - cl >= 1 keeps the word-completion test exact
constexpr uint32_t kSplitMaxAlphabet = 4096;

// LDS words of the table modes' tables for an alphabet: A + 1 entries, and
// A + 1 bytes for the split mode up to 4096 symbols (none above 8192).
__host__ __device__ inline uint32_t table_words(uint32_t A) {
  if (A > kTableMaxAlphabet) return 0u;
  return (A + 1) + (A <= kSplitMaxAlphabet ? (A + 4) / 4 : 0u);
}

struct SlabArgs {
  const void* sym;
  uint64_t n;
  uint64_t nblocks;
  uint32_t nslabs;
  uint32_t A;
  const uint8_t* cl;
  const uint64_t* cw;
  const uint32_t* slab_hist;  // [nslabs * A] or null
  uint64_t* bits;             // [nslabs] bit total per slab
  uint32_t* tails;            // [nslabs] last 32 content bits per slab
  uint32_t* status;
};

struct EncArgs {
  const void* sym;
  uint64_t n;
  uint64_t nblocks;
  uint32_t nslabs;
  uint32_t A;
  const uint8_t* cl;
  const uint64_t* cw;
  const uint64_t* info;
  const uint64_t* bits;
  const uint32_t* tails;
  uint32_t* out;
  uint64_t cap_words;
  uint64_t* offsets;
  uint32_t chunk_log2;
  uint64_t nchunks;
  uint32_t* status;
  uint32_t vec_ok;
  const uint32_t* gtab;  // alphabets above 8192: packed entries [A + 1] in the workspace
};

template <int NS, int SB>
struct Raw {
  static constexpr int kBytes = NS * SB;
  static constexpr int kWords = (kBytes + 3) / 4;
  uint32_t w[kWords];

  // Symbols [s0, s0 + NS) clipped to `end`.
  __device__ __forceinline__ void load(const void* sym, uint64_t s0, uint64_t end, bool vec_ok) {
    if (s0 + NS <= end && vec_ok && kBytes >= 4) {
      const char* p = (const char*)sym + s0 * SB;
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
      } else if constexpr (kBytes == 4) {
        w[0] = *(const uint32_t*)p;
      }
      return;
    }
#pragma unroll
    for (int k = 0; k < kWords; ++k) w[k] = 0;
#pragma unroll
    for (int i = 0; i < NS; ++i)
      if (s0 + i < end) w[(i * SB) / 4] |= sym_at<SB>(sym, s0 + i) << (8 * ((i * SB) % 4));
  }

  __device__ __forceinline__ uint32_t symbol(int i) const {
    if (SB == 1) return (w[i / 4] >> (8 * (i % 4))) & 0xFFu;
    return (w[i / 2] >> (16 * (i % 2))) & 0xFFFFu;
  }
};

// Append `len` (<= 32) bits of `code` to the lane accumulator; each full
// 32-bit word is ORed into dst (the first and last may be shared with the
// neighbouring lanes).  Words at index >= limit are dropped.
template <typename Dst>
__device__ __forceinline__ void push_bits(uint64_t& acc, uint32_t& nb, uint64_t& wi, Dst* dst,
                                          uint64_t limit, uint32_t code, uint32_t len) {
  acc = (len == 32) ? ((acc << 32) | code) : ((acc << len) | code);
  nb += len;
  if (nb >= 32) {
    nb -= 32;
    if (wi < limit) atomicOr(&dst[wi], (uint32_t)(acc >> nb));
    ++wi;
  }
}

// Bits of code (c, l), which occupies content bits [p, p + l), that fall in
// [max(B - 32, 0), B), placed as in a last-32-bits record (content bit B - 1
// at bit 0).
__device__ __forceinline__ uint32_t tail_part(uint64_t c, uint32_t l, uint32_t p, uint32_t B) {
  const uint32_t s = B > 32 ? B - 32 : 0u;
  if (p + l <= s || p >= B) return 0u;
  const uint32_t lo = p > s ? p : s;
  const uint32_t hi = p + l < B ? p + l : B;
  const uint32_t w = hi - lo;
  const uint64_t seg = (c >> (p + l - hi)) & ((w >= 64) ? ~0ull : ((1ull << w) - 1));
  return (uint32_t)(seg << (B - hi));
}

// ---------------------------------------------------------------------------
// Prepass: bit total and last 32 bits of every slab.
// ---------------------------------------------------------------------------
template <int SB>
__global__ __launch_bounds__(kPreThreads) void slab_bits_kernel(SlabArgs a) {
  __shared__ uint64_t part[kPreWaves];
  const uint32_t g = blockIdx.x;
  const uint32_t tid = threadIdx.x;
  const uint64_t s_lo = slab_begin(g, a.nblocks, a.nslabs, a.n);
  const uint64_t s_hi = slab_begin(g + 1, a.nblocks, a.nslabs, a.n);
  uint64_t bits = 0;
  bool bad = false;
  if (a.slab_hist) {
    const uint32_t* row = a.slab_hist + (uint64_t)g * a.A;
    for (uint32_t s = tid; s < a.A; s += kPreThreads) bits += (uint64_t)row[s] * a.cl[s];
  } else {
    for (uint64_t i = s_lo + tid; i < s_hi; i += kPreThreads) {
      const uint32_t s = sym_at<SB>(a.sym, i);
      const uint32_t l = s < a.A ? a.cl[s] : 0u;
      bad |= l == 0;
      bits += l;
    }
  }
  bits = wave_sum_u64(bits);
  if (lane_id() == 0) part[tid / kWave] = bits;
  uint32_t tail = 0;
  if (tid < kWave) tail = range_tail<SB>(a.sym, s_lo, s_hi, a.A, a.cl, a.cw);
  __syncthreads();
  if (tid == 0) {
    uint64_t t = 0;
    for (int w = 0; w < kPreWaves; ++w) t += part[w];
    a.bits[g] = t;
    a.tails[g] = tail;
  }
  if (bad) raise_status(a.status, HF_ERR_SYMBOL);
}

// ---------------------------------------------------------------------------
// Encoder: one workgroup per slab.
// ---------------------------------------------------------------------------
// Table entry of a code of length l <= 27: the code left-aligned in bits
// [32 - l, 32) and f = 32 - l in bits [0, 5) (bits 5 .. 31 - l are zero);
// 0 marks a symbol without code.
__device__ __forceinline__ uint32_t pack_entry(uint32_t code, uint32_t l) { return (code << (32 - l)) | (32 - l); }

struct EncShared {
  uint32_t wtot[kEncWaves];
  uint64_t red[kEncWaves];
  uint32_t tail[2];  // last 32 bits of the previous / current tile
  uint32_t tailw;    // wide mode: current tile's last 32 bits
};

// `expect` is the slab's bit total from the prepass (sum of count * cl): a
// slab whose tiles add up to anything else held a symbol without code or
// outside the alphabet, or came with per-slab counts of other symbols.
template <int R, int SB, int MODE>
__device__ __forceinline__ void encode_slab(const EncArgs& a, const uint32_t* tab, uint32_t* buf,
                                            uint32_t* dummy, EncShared& sh, uint32_t g, uint64_t G,
                                            uint64_t expect) {
  constexpr uint32_t NS = 1u << R;
  constexpr uint32_t T = kEncThreads * NS;
  constexpr bool kTabMode = MODE == kModeTable || MODE == kModeSplit || MODE == kModeGTable;
  const uint32_t tid = threadIdx.x;
  const uint64_t s_lo = slab_begin(g, a.nblocks, a.nslabs, a.n);
  const uint64_t s_hi = slab_begin(g + 1, a.nblocks, a.nslabs, a.n);
  const bool last_slab = g == a.nslabs - 1;
  const uint32_t ntiles = (uint32_t)((s_hi - s_lo + T - 1) / T);

  Raw<NS, SB> raw;
  raw.load(a.sym, s_lo + (uint64_t)tid * NS, s_hi, a.vec_ok != 0);
  uint64_t run = 0;  // bits of this slab before the current tile
  // buf word i is output word (tile's first bit) / 32 + i: the first word
  // starts with the last (first bit % 32) bits before the tile, seeded here
  // for the slab's first tile and carried over for the others
  if (MODE != kModeWide && tid == 0) {
    const uint32_t q0 = (uint32_t)(G & 31);
    buf[0] = q0 ? sh.tail[0] << (32 - q0) : 0u;
  }

  for (uint32_t t = 0; t < ntiles; ++t) {
    const uint64_t s0 = s_lo + (uint64_t)t * T + (uint64_t)tid * NS;
    const uint32_t nvalid = s0 >= s_hi ? 0u : (s_hi - s0 >= NS ? NS : (uint32_t)(s_hi - s0));
    const bool last_tile = t == ntiles - 1;
    const uint64_t Gt = G + run;            // the tile's first bit in the stream
    const uint32_t q = (uint32_t)(Gt & 31);  // ... and its offset in buf[0]

    // ---- lookup: table entries (table modes) or symbols; lane bit count ----
    // ent: the code left-aligned (table mode: with 32 - cl in its low 5
    // bits); fsh: the split mode's 32 - cl (0: no code)
    constexpr bool kTab = kTabMode;
    const uint8_t* tabf = (const uint8_t*)(tab + a.A + 1);
    uint32_t ent[NS];
    uint32_t fsh[MODE == kModeSplit ? NS : 1];
    uint32_t L = 0;
    bool bad = false;
    bool full_tile = false;
    if (kTab && s_lo + (uint64_t)(t + 1) * T <= s_hi) {
      // whole tile inside the slab: no per-symbol branches; entry A is empty
      // and catches symbols outside the alphabet, an empty entry marks a
      // symbol without code (it counts 32 bits here; the slab's total then
      // differs from the prepass's, which flags it at the end of the slab)
      uint32_t fsum = 0;
#pragma unroll
      for (uint32_t i = 0; i < NS; ++i) {
        const uint32_t k = min(raw.symbol(i), a.A);
        const uint32_t e = tab[k];
        ent[i] = e;
        if (MODE == kModeSplit) {
          fsh[i] = tabf[k];
          fsum += fsh[i];
        } else {
          fsum += e & 31;
        }
      }
      L = 32 * NS - fsum;
      full_tile = true;
    } else {
#pragma unroll
      for (uint32_t i = 0; i < NS; ++i) {
        const uint32_t sv = raw.symbol(i);
        if (MODE == kModeTable || MODE == kModeGTable) {
          ent[i] = 0;
          if (i < nvalid) {
            const uint32_t e = tab[min(sv, a.A)];
            bad |= e == 0;
            ent[i] = e;
            L += e ? 32 - (e & 31) : 0u;
          }
        } else if (MODE == kModeSplit) {
          ent[i] = 0;
          fsh[i] = 0;
          if (i < nvalid) {
            const uint32_t k = min(sv, a.A);
            const uint32_t f = tabf[k];
            bad |= f == 0;
            ent[i] = tab[k];
            fsh[i] = f;
            L += f ? 32 - f : 0u;
          }
        } else {
          ent[i] = 0xFFFFFFFFu;
          if (i < nvalid) {
            const uint32_t l = sv < a.A ? a.cl[sv] : 0u;
            bad |= l == 0;
            if (l) ent[i] = sv;
            L += l;
          }
        }
      }
    }
    if (bad) raise_status(a.status, HF_ERR_SYMBOL);

    // ---- shuffle-merge offsets: workgroup scan ---------------------------------
    uint32_t B;
    const uint32_t P = block_exclusive_scan<kEncWaves>(L, sh.wtot, &B);
    if (!last_tile) raw.load(a.sym, s0 + T, s_hi, a.vec_ok != 0);  // next tile, in flight meanwhile

    // ---- reduce-merge ---------------------------------------------------------
    if (kTab) {
      // pend's low nb bits are this lane's bits of word wp so far (zeros for
      // the bits of earlier lanes).  A code of len = 32 - f bits completes the
      // word when nb >= f: the word is then bits [nb, nb + 32) of (pend:e), and
      // what is left is bits [f, nb); otherwise all of it joins pend.  Either
      // way the new pend is (pend:e) >> f (the shift reads only e's low 5
      // bits, f) and the new count is (nb - f) mod 32, which is below nb
      // exactly when a word completes (5 <= f <= 31).  At most one word
      // completes per code (<= 27 bits on <= 31 pending); the OR always
      // issues, into this lane's dummy word when none does.  The split mode
      // reads f from its byte table (1 <= f, so the test stays exact) and its
      // codes have no low bits to shift out.
      uint32_t pend = 0;
      uint32_t nb = (P + q) & 31;
      uint32_t* wp = buf + ((P + q) >> 5);
      uint32_t* const sink = dummy + tid;
      if (full_tile) {
#pragma unroll
        for (uint32_t i = 0; i < NS; ++i) {
          const uint32_t e = ent[i];
          const uint32_t f = MODE == kModeSplit ? fsh[i] : e;  // shift: its low 5 bits
          const uint32_t word = __builtin_amdgcn_alignbit(pend, e, nb);
          const uint32_t nb2 = (nb - f) & 31;
          const bool full = nb2 < nb;
          pend = __builtin_amdgcn_alignbit(pend, e, f);
          nb = nb2;
          atomicOr(full ? wp : sink, word);
          wp += full ? 1 : 0;
        }
      } else {
#pragma unroll
        for (uint32_t i = 0; i < NS; ++i) {
          const uint32_t e = ent[i];
          const uint32_t f = MODE == kModeSplit ? fsh[i] : (e & 31);
          if (f == 0) continue;  // past the slab's end, or a symbol without code (flagged)
          const uint32_t word = __builtin_amdgcn_alignbit(pend, e, nb);
          const bool full = nb >= f;
          pend = __builtin_amdgcn_alignbit(pend, e, f);
          nb = (nb - f) & 31;
          if (full) atomicOr(wp++, word);
        }
      }
      if (nb) atomicOr(wp, pend << (32 - nb));
    } else if (MODE == kModeGlobal) {
      uint64_t acc = 0;
      uint32_t nb = (P + q) & 31;
      uint64_t wi = (P + q) >> 5;
#pragma unroll
      for (uint32_t i = 0; i < NS; ++i)
        if (ent[i] != 0xFFFFFFFFu) push_bits(acc, nb, wi, buf, ~0ull, (uint32_t)a.cw[ent[i]], a.cl[ent[i]]);
      if (nb) atomicOr(&buf[wi], (uint32_t)(acc << (32 - nb)));
    } else if (P + L > (B > 32 ? B - 32 : 0u)) {
      // lanes holding the tile's last 32 bits build its tail record
      uint32_t p = P;
#pragma unroll
      for (uint32_t i = 0; i < NS; ++i) {
        if (ent[i] == 0xFFFFFFFFu) continue;
        const uint32_t l = a.cl[ent[i]];
        const uint32_t part = tail_part(a.cw[ent[i]], l, p, B);
        if (part) atomicOr(&sh.tailw, part);
        p += l;
      }
    }
    __syncthreads();

    // ---- wide mode: this tile's last 32 bits, for the next tile of the slab ----------
    if (MODE == kModeWide && tid == 0) sh.tail[(t + 1) & 1] = sh.tailw;

    // ---- gathering ----------------------------------------------------------------
    const uint32_t q_end = q + B;  // bit after the tile's last, counted from buf[0]
    const uint64_t w0 = Gt >> 5;
    const uint64_t end_bit = Gt + B;
    const bool stream_end = last_slab && last_tile;
    uint64_t wend = (end_bit + 31) >> 5;
    if (!stream_end && (end_bit & 31)) wend -= 1;  // the next tile owns the shared word
    const uint32_t nw = (uint32_t)(wend - w0);
    uint32_t carry = 0;  // the shared word's bits so far, for the next tile's buf[0]
    if (MODE != kModeWide) {
      // buf holds the output words w0 .. w0 + nw - 1 as they are: copy them,
      // four per lane from one 16-byte LDS read
      const uint32_t nwc = w0 >= a.cap_words ? 0u : (uint32_t)min((uint64_t)nw, a.cap_words - w0);
      uint32_t* const dst = a.out + w0;
      for (uint32_t i = 4 * tid; i < nwc; i += 4 * kEncThreads) {
        const uint4 v = *(const uint4*)(buf + i);
        dst[i] = v.x;
        if (i + 1 < nwc) dst[i + 1] = v.y;
        if (i + 2 < nwc) dst[i + 2] = v.z;
        if (i + 3 < nwc) dst[i + 3] = v.w;
      }
      if (tid == 0 && (q_end & 31)) carry = buf[q_end >> 5];
    } else {
      const uint32_t pred = sh.tail[t & 1];
      for (uint32_t i = tid; i < nw; i += kEncThreads) {
        const uint64_t wi = w0 + i;
        if (wi < a.cap_words) a.out[wi] = (i == 0 && q) ? (pred << (32 - q)) : 0u;
      }
      __syncthreads();
      const uint64_t limit = wend < a.cap_words ? wend : a.cap_words;
      const uint64_t pos = Gt + P;
      uint64_t acc = 0;
      uint32_t nb = (uint32_t)(pos & 31);
      uint64_t wi = pos >> 5;
#pragma unroll
      for (uint32_t i = 0; i < NS; ++i) {
        if (ent[i] == 0xFFFFFFFFu) continue;
        const uint32_t l = a.cl[ent[i]];
        const uint64_t c = a.cw[ent[i]];
        if (l > 32) {
          push_bits(acc, nb, wi, a.out, limit, (uint32_t)(c >> 32), l - 32);
          push_bits(acc, nb, wi, a.out, limit, (uint32_t)c, 32);
        } else {
          push_bits(acc, nb, wi, a.out, limit, (uint32_t)c, l);
        }
      }
      if (nb && wi < limit) atomicOr(&a.out[wi], (uint32_t)(acc << (32 - nb)));
    }
    if (s0 < s_hi && (s0 & ((1ull << a.chunk_log2) - 1)) == 0) a.offsets[s0 >> a.chunk_log2] = Gt + P;
    if (stream_end && tid == 0) {
      a.offsets[a.nchunks] = end_bit;
      if (end_bit > 32ull * a.cap_words) raise_status(a.status, HF_ERR_CAPACITY);
    }
    run += B;
    __syncthreads();
    if (MODE != kModeWide) {
      // clear the words this tile used; the shared word's bits start the next
      const uint32_t used = (q_end >> 5) + 1;
      for (uint32_t i = 4 * tid; i < used; i += 4 * kEncThreads) *(uint4*)(buf + i) = make_uint4(0u, 0u, 0u, 0u);
      if (tid == 0) buf[0] = carry;
    } else if (tid == 0) {
      sh.tailw = 0;
    }
  }
  // every mode: the slab's bits must add up to the prepass's total (else a
  // symbol had no code, or the per-slab counts were not these symbols' and
  // later slabs were placed at wrong offsets)
  if (tid == 0 && run != expect) raise_status(a.status, HF_ERR_SYMBOL);
}

__device__ __forceinline__ int encode_mode(uint32_t A, uint32_t lmax) {
  if (A <= kTableMaxAlphabet && lmax <= kPackedMaxLen) return kModeTable;
  if (A > kTableMaxAlphabet && lmax <= kPackedMaxLen) return kModeGTable;
  if (A <= kSplitMaxAlphabet && lmax <= kSplitMaxLen) return kModeSplit;
  return lmax <= kLdsBufMaxLen ? kModeGlobal : kModeWide;
}

// The table modes' LDS tables: tab[s] is the packed entry (table mode) or the
// left-aligned code (split mode, with 32 - cl in the bytes after tab[A]);
// entry A and the entries of unused symbols are empty.
__device__ __forceinline__ void build_tables(const EncArgs& a, int mode, uint32_t* tab) {
  if (mode != kModeTable && mode != kModeSplit) return;
  uint8_t* tabf = (uint8_t*)(tab + a.A + 1);
  for (uint32_t s = threadIdx.x; s <= a.A; s += kEncThreads) {
    const uint32_t l = s < a.A ? a.cl[s] : 0u;
    if (mode == kModeTable) {
      tab[s] = l ? pack_entry((uint32_t)a.cw[s], l) : 0u;
    } else {
      tab[s] = l ? (uint32_t)a.cw[s] << (32 - l) : 0u;
      tabf[s] = (uint8_t)(l ? 32 - l : 0u);
    }
  }
}

template <int R, int SB>
__global__ __launch_bounds__(kEncThreads) void encode_kernel(EncArgs a) {
  constexpr uint32_t T = kEncThreads << R;
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ EncShared sh;
  const uint32_t tid = threadIdx.x;
  const uint32_t g = blockIdx.x;
  const uint32_t lmax = (uint32_t)a.info[1];
  const int mode = encode_mode(a.A, lmax);
  // LDS: [tile buffer: T + 8 words, 16-byte aligned][tables, if A <= 8192:
  // A + 1 words and A + 1 bytes][kEncThreads dummy words]
  uint32_t* buf = lds;
  uint32_t* tab = lds + T + 8;
  uint32_t* dummy = tab + table_words(a.A);
  build_tables(a, mode, tab);
  if (mode != kModeWide)
    for (uint32_t i = tid; i < T + 8; i += kEncThreads) buf[i] = 0;
  // this slab's first bit: the bit totals of all earlier slabs
  uint64_t G = 0;
  for (uint32_t k = tid; k < g; k += kEncThreads) G += a.bits[k];
  G = wave_sum_u64(G);
  if (lane_id() == 0) sh.red[tid / kWave] = G;
  if (tid == 0) {
    sh.tail[0] = g > 0 ? a.tails[g - 1] : 0u;
    sh.tailw = 0;
  }
  __syncthreads();
  G = 0;
#pragma unroll
  for (int w = 0; w < kEncWaves; ++w) G += sh.red[w];
  if (mode == kModeTable) encode_slab<R, SB, kModeTable>(a, tab, buf, dummy, sh, g, G, a.bits[g]);
  else if (mode == kModeSplit) encode_slab<R, SB, kModeSplit>(a, tab, buf, dummy, sh, g, G, a.bits[g]);
  else if (mode == kModeGTable) encode_slab<R, SB, kModeGTable>(a, a.gtab, buf, dummy, sh, g, G, a.bits[g]);
  else if (mode == kModeGlobal) encode_slab<R, SB, kModeGlobal>(a, tab, buf, dummy, sh, g, G, a.bits[g]);
  else encode_slab<R, SB, kModeWide>(a, tab, buf, dummy, sh, g, G, a.bits[g]);
}

// Batched stage 4 for work item (stream bs, slab g): the slab's bit total
// and last 32 content bits, from its counts (kPreThreads lanes; part: LDS
// words, one per wave).
__device__ __forceinline__ void batch_slab_bits_item(const BatchStream& bs, uint32_t g, uint64_t* part) {
  const uint32_t tid = threadIdx.x;
  const uint32_t A = bs.A;
  const uint32_t* row = bs.part + (uint64_t)g * A;
  uint64_t bits = 0;
  for (uint32_t s = tid; s < A; s += kPreThreads) bits += (uint64_t)row[s] * bs.book.cl[s];
  bits = wave_sum_u64(bits);
  if (lane_id() == 0) part[tid / kWave] = bits;
  uint32_t tail = 0;
  if (tid < kWave) {
    const uint64_t s_lo = slab_begin(g, bs.nblocks, bs.nslabs, bs.n);
    const uint64_t s_hi = slab_begin(g + 1, bs.nblocks, bs.nslabs, bs.n);
    tail = bs.sym_bytes == 1 ? range_tail<1>(bs.sym, s_lo, s_hi, A, bs.book.cl, bs.book.cw)
                             : range_tail<2>(bs.sym, s_lo, s_hi, A, bs.book.cl, bs.book.cw);
  }
  __syncthreads();
  if (tid == 0) {
    uint64_t t = 0;
    for (int w = 0; w < kPreWaves; ++w) t += part[w];
    bs.slab_bits[g] = t;
    bs.slab_tail[g] = tail;
  }
}

// LDS bytes the batched encoder needs for reduction factor r and alphabets
// up to A: [tile buffer: T + 8 words][tables][kEncThreads dummy words].
__host__ __device__ inline size_t batch_encode_lds_bytes(uint32_t r, uint32_t A) {
  return 4 * (((size_t)kEncThreads << r) + 8 + (size_t)table_words(A) + kEncThreads);
}

// Batched stage 5 for work item (stream bs, slab g): encodes the slab; its
// first bit is the sum of the bit totals of the stream's earlier slabs.
// Each stream has its own alphabet, symbol width and codebook.
template <int R>
__device__ __forceinline__ void batch_encode_item(const BatchStream& bs, uint32_t g, uint32_t* lds, EncShared& sh) {
  constexpr uint32_t T = kEncThreads << R;
  const uint32_t tid = threadIdx.x;
  EncArgs a;
  a.sym = bs.sym;
  a.n = bs.n;
  a.nblocks = bs.nblocks;
  a.nslabs = bs.nslabs;
  a.A = bs.A;
  a.cl = bs.book.cl;
  a.cw = bs.book.cw;
  a.info = bs.book.info;
  a.bits = nullptr;
  a.tails = nullptr;
  a.gtab = nullptr;  // batched alphabets are at most 8192
  a.out = bs.out;
  a.cap_words = bs.cap_words;
  a.offsets = bs.offsets;
  a.chunk_log2 = bs.chunk_log2;
  a.nchunks = bs.nchunks;
  a.status = bs.status;
  a.vec_ok = ((uintptr_t)bs.sym % 16) == 0 ? 1u : 0u;
  const uint32_t lmax = (uint32_t)a.info[1];
  const int mode = encode_mode(a.A, lmax);
  uint32_t* buf = lds;  // same layout as encode_kernel
  uint32_t* tab = lds + T + 8;
  uint32_t* dummy = tab + table_words(a.A);
  build_tables(a, mode, tab);
  if (mode != kModeWide)
    for (uint32_t i = tid; i < T + 8; i += kEncThreads) buf[i] = 0;
  uint64_t G = 0;
  for (uint32_t k = tid; k < g; k += kEncThreads) G += bs.slab_bits[k];
  G = wave_sum_u64(G);
  if (lane_id() == 0) sh.red[tid / kWave] = G;
  if (tid == 0) {
    sh.tail[0] = g > 0 ? bs.slab_tail[g - 1] : 0u;
    sh.tailw = 0;
  }
  __syncthreads();
  G = 0;
#pragma unroll
  for (int w = 0; w < kEncWaves; ++w) G += sh.red[w];
  if (bs.sym_bytes == 1) {
    if (mode == kModeTable) encode_slab<R, 1, kModeTable>(a, tab, buf, dummy, sh, g, G, bs.slab_bits[g]);
    else if (mode == kModeSplit) encode_slab<R, 1, kModeSplit>(a, tab, buf, dummy, sh, g, G, bs.slab_bits[g]);
    else if (mode == kModeGlobal) encode_slab<R, 1, kModeGlobal>(a, tab, buf, dummy, sh, g, G, bs.slab_bits[g]);
    else encode_slab<R, 1, kModeWide>(a, tab, buf, dummy, sh, g, G, bs.slab_bits[g]);
  } else {
    if (mode == kModeTable) encode_slab<R, 2, kModeTable>(a, tab, buf, dummy, sh, g, G, bs.slab_bits[g]);
    else if (mode == kModeSplit) encode_slab<R, 2, kModeSplit>(a, tab, buf, dummy, sh, g, G, bs.slab_bits[g]);
    else if (mode == kModeGlobal) encode_slab<R, 2, kModeGlobal>(a, tab, buf, dummy, sh, g, G, bs.slab_bits[g]);
    else encode_slab<R, 2, kModeWide>(a, tab, buf, dummy, sh, g, G, bs.slab_bits[g]);
  }
}

// Batched stage 4: workgroup i handles work item i.
__global__ __launch_bounds__(kPreThreads) void batch_slab_bits_kernel(const BatchStream* __restrict__ streams,
                                                                      const uint32_t* __restrict__ item_stream) {
  __shared__ uint64_t part[kPreWaves];
  const BatchStream& bs = streams[item_stream[blockIdx.x]];
  batch_slab_bits_item(bs, blockIdx.x - bs.item0, part);
}

// Batched stage 5: workgroup i encodes the slab of work item items[i].
template <int R>
__global__ __launch_bounds__(kEncThreads) void batch_encode_kernel(const BatchStream* __restrict__ streams,
                                                                   const uint32_t* __restrict__ item_stream,
                                                                   const uint32_t* __restrict__ items) {
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ EncShared sh;
  const uint32_t item = items[blockIdx.x];
  const BatchStream& bs = streams[item_stream[item]];
  batch_encode_item<R>(bs, item - bs.item0, lds, sh);
}

using EncodeFn = void (*)(EncArgs);

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

size_t encode_lds_bytes(uint32_t A, uint32_t r) {
  const size_t T = (size_t)kEncThreads << r;
  return 4 * (kEncThreads + (size_t)table_words(A) + T + 8);
}

// Resident workgroups per CU, cached per kernel and LDS size.
struct OccEntry {
  const void* fn;
  size_t lds;
  int blocks;
};
OccEntry g_occ[64];
int g_nocc = 0;
std::mutex g_occ_mu;

int blocks_per_cu(EncodeFn fn, size_t lds) {
  std::lock_guard<std::mutex> lock(g_occ_mu);
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

int encode_blocks_per_cu(uint32_t alphabet, uint32_t sym_bytes) {
  const uint32_t r = kEncDefaultR;
  return blocks_per_cu(pick(r, sym_bytes), encode_lds_bytes(alphabet, r));
}

size_t encode_workspace_bytes(uint32_t nslabs, uint32_t alphabet) {
  const size_t gtab = alphabet > kTableMaxAlphabet ? align256(((size_t)alphabet + 1) * 4) : 0;
  return align256((size_t)nslabs * 8) + align256((size_t)nslabs * 4) + gtab;
}

// Packed table-mode entries of an alphabet above 8192, for the L2 table
// mode (entries of codes over 27 bits stay 0; such books take another mode).
__global__ __launch_bounds__(256) void gtable_kernel(const uint8_t* __restrict__ cl, const uint64_t* __restrict__ cw,
                                                     uint32_t A, uint32_t* __restrict__ gtab) {
  const uint32_t s = blockIdx.x * 256u + threadIdx.x;
  if (s > A) return;
  const uint32_t l = s < A ? cl[s] : 0u;
  gtab[s] = (l && l <= kPackedMaxLen) ? pack_entry((uint32_t)cw[s], l) : 0u;
}

hipError_t launch_encode(const void* sym, uint64_t n, uint32_t sym_bytes, const hf_codebook& book,
                         uint32_t chunk_log2, uint32_t r, uint32_t nslabs, const uint32_t* slab_hist,
                         uint32_t* out, uint64_t cap_words, uint64_t* offsets, void* ws,
                         uint32_t* status, hipStream_t stream, const KernelTimer& timer) {
  const uint64_t nchunks = (n + (1ull << chunk_log2) - 1) >> chunk_log2;
  if (n == 0) {
    hipError_t e = launch_fill_u64(offsets, 1, 0, stream);
    timer.before(stream);
    timer.after(stream);
    return e;
  }
  const uint64_t nblocks = (n + kSlabBlock - 1) / kSlabBlock;
  uint64_t* bits = (uint64_t*)ws;
  uint32_t* tails = (uint32_t*)((char*)ws + align256((size_t)nslabs * 8));
  const uint32_t A = book.alphabet;

  SlabArgs s;
  s.sym = sym;
  s.n = n;
  s.nblocks = nblocks;
  s.nslabs = nslabs;
  s.A = A;
  s.cl = book.cl;
  s.cw = book.cw;
  s.slab_hist = slab_hist;
  s.bits = bits;
  s.tails = tails;
  s.status = status;
  if (sym_bytes == 1) slab_bits_kernel<1><<<nslabs, kPreThreads, 0, stream>>>(s);
  else slab_bits_kernel<2><<<nslabs, kPreThreads, 0, stream>>>(s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;

  EncArgs a;
  a.sym = sym;
  a.n = n;
  a.nblocks = nblocks;
  a.nslabs = nslabs;
  a.A = A;
  a.cl = book.cl;
  a.cw = book.cw;
  a.info = book.info;
  a.bits = bits;
  a.tails = tails;
  a.out = out;
  a.cap_words = cap_words;
  a.offsets = offsets;
  a.chunk_log2 = chunk_log2;
  a.nchunks = nchunks;
  a.status = status;
  a.vec_ok = ((uintptr_t)sym % 16) == 0 ? 1u : 0u;
  a.gtab = nullptr;
  if (A > kTableMaxAlphabet) {
    uint32_t* gtab = (uint32_t*)((char*)ws + align256((size_t)nslabs * 8) + align256((size_t)nslabs * 4));
    gtable_kernel<<<(A + 1 + 255) / 256, 256, 0, stream>>>(book.cl, book.cw, A, gtab);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    a.gtab = gtab;
  }
  EncodeFn fn = pick(r, sym_bytes);
  const size_t lds = encode_lds_bytes(A, r);
  (void)blocks_per_cu(fn, lds);  // sets the LDS attribute when above 64 KiB
  timer.before(stream);
  hipLaunchKernelGGL(fn, dim3(nslabs), dim3(kEncThreads), lds, stream, a);
  e = hipGetLastError();
  timer.after(stream);
  return e;
}

// ---------------------------------------------------------------------------
// Persistent batched launch: every stage of every stream in one kernel.
// ---------------------------------------------------------------------------
namespace {

using FusedCbLds = CbLdsT<kFusedTreeCap>;
constexpr uint32_t kFusedSpinLimit = 1u << 18;  // polls (0.1 - 0.3 s); real waits are below a millisecond
constexpr uint32_t kFusedQueueClosed = 0x7FFFFFFFu;

// Waits until *counter reaches target: lane 0 polls with acquire loads, then
// every lane acquires.  A counter only counts items that come earlier in the
// queue, and the earliest unfinished item always has its inputs and a
// running workgroup, so the wait ends.  The spin limit turns a broken
// invariant into an error instead of a hang: the stream's status records
// HF_ERR_INTERNAL and the queue is closed (its head moved past every
// item), so the grid drains after the items already taken.
__device__ __forceinline__ void fused_wait(const uint32_t* counter, uint32_t target, uint32_t* status,
                                           uint32_t* head) {
  if (threadIdx.x == 0) {
    uint32_t spins = 0;
    while (__hip_atomic_load(counter, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (++spins > kFusedSpinLimit) {
        raise_status(status, HF_ERR_INTERNAL);
        atomicMax(head, kFusedQueueClosed);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// Publishes a finished item: every lane's stores reach device scope, then
// one count.
__device__ __forceinline__ void fused_done(uint32_t* counter) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace

// The queue holds, in this order: the slab histograms (hist_items order),
// the bin-chunk sums (red_items), one codebook per stream, the slab bit
// totals (item order) and the slab encodings (enc_items order).  Stream s
// has four counters after sync[0] (the queue head): slabs counted, bin
// chunks summed, book built, slab totals known.  A reduce item waits for
// all its stream's slabs, a codebook for all its chunks, a slab total for
// the book, an encoding for all the stream's slab totals.
__global__ __launch_bounds__(kEncThreads) void batch_persistent_kernel(FusedArgs f) {
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ EncShared sh;
  __shared__ uint64_t part[kPreWaves];
  __shared__ uint32_t s_item;
  const uint32_t nh = f.nitems;
  const uint32_t c_red = nh, c_cb = c_red + f.nred, c_bits = c_cb + f.nstreams, c_enc = c_bits + nh;
  const uint32_t total = c_enc + nh;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(f.sync, 1u);
    __syncthreads();
    const uint32_t i = s_item;
    __syncthreads();
    if (i >= total) break;
    uint32_t* done = nullptr;
    if (i < c_red) {
      const uint32_t item = f.hist_items[i];
      const uint32_t s = f.item_stream[item];
      const BatchStream& bs = f.streams[s];
      batch_hist_item(bs, item - bs.item0, lds, f.lds_words);
      done = f.sync + 1 + 4 * s;
    } else if (i < c_cb) {
      const uint32_t r = f.red_items[i - c_red];
      const BatchStream& bs = f.streams[r >> 6];
      uint32_t* cnt = f.sync + 1 + 4 * (r >> 6);
      fused_wait(cnt, bs.nslabs, bs.status, f.sync);
      batch_reduce_item(bs, r & 63);
      done = cnt + 1;
    } else if (i < c_bits) {
      const uint32_t s = i - c_cb;
      const BatchStream& bs = f.streams[s];
      uint32_t* cnt = f.sync + 1 + 4 * s;
      fused_wait(cnt + 1, bs.n ? (bs.A + kBatchReduceBins - 1) / kBatchReduceBins : 0u, bs.status, f.sync);
      batch_codebook_item<kEncThreads>(bs, *reinterpret_cast<FusedCbLds*>(lds));
      done = cnt + 2;
    } else if (i < c_enc) {
      const uint32_t item = i - c_bits;
      const uint32_t s = f.item_stream[item];
      const BatchStream& bs = f.streams[s];
      uint32_t* cnt = f.sync + 1 + 4 * s;
      fused_wait(cnt + 2, 1u, bs.status, f.sync);
      batch_slab_bits_item(bs, item - bs.item0, part);
      done = cnt + 3;
    } else {
      const uint32_t item = f.enc_items[i - c_enc];
      const uint32_t s = f.item_stream[item];
      const BatchStream& bs = f.streams[s];
      fused_wait(f.sync + 1 + 4 * s + 3, bs.nslabs, bs.status, f.sync);
      const uint32_t g = item - bs.item0;
      if (bs.r == 3) batch_encode_item<3>(bs, g, lds, sh);
      else if (bs.r == 5) batch_encode_item<5>(bs, g, lds, sh);
      else batch_encode_item<4>(bs, g, lds, sh);
    }
    if (done) fused_done(done);
    else __syncthreads();  // the next item reuses the LDS
  }
}

size_t batch_persistent_lds_bytes(const BatchStream* streams, uint32_t nstreams) {
  size_t b = sizeof(FusedCbLds);
  for (uint32_t s = 0; s < nstreams; ++s) {
    b = std::max(b, batch_encode_lds_bytes(streams[s].r, streams[s].A));
    b = std::max(b, (size_t)4 * hist_stride(streams[s].A, streams[s].A));
  }
  return (b + 15) & ~(size_t)15;
}

hipError_t launch_batch_persistent(const FusedArgs& f, size_t lds_bytes, int num_cus, hipStream_t stream) {
  const void* fn = (const void*)batch_persistent_kernel;
  if (lds_bytes > (64u << 10)) {
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
  }
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kEncThreads, lds_bytes) != hipSuccess || per_cu < 1)
    per_cu = 1;
  const uint64_t total = 3ull * f.nitems + f.nred + f.nstreams;
  const uint64_t grid = std::min<uint64_t>((uint64_t)per_cu * (uint64_t)std::max(num_cus, 1), std::max<uint64_t>(total, 1));
  batch_persistent_kernel<<<(uint32_t)grid, kEncThreads, lds_bytes, stream>>>(f);
  return hipGetLastError();
}

hipError_t launch_batch_slab_bits(const BatchStream* d_streams, const uint32_t* d_item_stream, uint32_t nitems,
                                  hipStream_t stream) {
  if (nitems == 0) return hipSuccess;
  batch_slab_bits_kernel<<<nitems, kPreThreads, 0, stream>>>(d_streams, d_item_stream);
  return hipGetLastError();
}

hipError_t launch_batch_encode(const BatchStream* d_streams, const uint32_t* d_item_stream,
                               const uint32_t* d_items, uint32_t nitems, uint32_t r, uint32_t max_alphabet,
                               hipStream_t stream) {
  if (nitems == 0) return hipSuccess;
  const size_t T = (size_t)kEncThreads << r;
  const size_t lds = 4 * (T + 8 + (size_t)table_words(max_alphabet) + kEncThreads);
  using Fn = void (*)(const BatchStream*, const uint32_t*, const uint32_t*);
  Fn fn;
  switch (r) {
    case 3: fn = batch_encode_kernel<3>; break;
    case 5: fn = batch_encode_kernel<5>; break;
    default: fn = batch_encode_kernel<4>; break;
  }
  if (lds > (64u << 10)) (void)hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(fn, dim3(nitems), dim3(kEncThreads), lds, stream, d_streams, d_item_stream, d_items);
  return hipGetLastError();
}

}  // namespace hf
