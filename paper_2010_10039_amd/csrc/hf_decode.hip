// hf_decode.hip -- treeless canonical decoding with the First / Entry /
// reverse-codebook tables (Sec. 4.2.2 of the paper; Table 1, "get reverse
// codebook").  The checker decodes each chunk bit by bit in one lane and
// compares it with the input; the decoder gives each chunk a wave whose
// lanes start at fixed bit strides and resynchronise (below).
#include <mutex>

#include "hf_device.h"
#include "hf_kernels.h"

namespace hf {

namespace {

constexpr int kDecThreads = 256;

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

// ---------------------------------------------------------------------------
// Decoder: one wave per chunk, lanes at bit strides (self-synchronisation).
// ---------------------------------------------------------------------------
// A chunk's bits are decoded in segments of up to 64 * S bits.  Lane j of
// the wave takes the S-bit region [seg + j S, seg + (j + 1) S) and decodes
// the codes that start in it:
//  A. every lane decodes from its region's first bit (a guess, except for
//     lane 0, whose start is a true code boundary) and marks each code start
//     in a bitmap;
//  B. a lane whose start differs from its left neighbour's end decodes again
//     from that end, and stops as soon as it meets a start it marked in A:
//     from there A's decode is the true one, so the rest of its count is the
//     number of marks left in the region (Huffman codes resynchronise after a
//     few codes).  Repeated until no start changes (at most 64 times: lane t
//     is right after round t);
//  C. an exclusive scan of the counts gives each lane its output position;
//     the lanes decode once more from their true starts into an LDS tile,
//     which is copied out with 16-byte stores.
// Regions are multiples of the gcd of the code lengths, so a fixed-length
// code is never out of step.  The treeless canonical rule (Sec. 4.2.2): the
// first l bits v of the window form a code of length l when v >= First[l]
// and l is the smallest such length; its symbol is
// rev[Entry[l] + v - First[l]].  With the window W left-aligned in 64 bits,
// that is W >= LJ[l] = First[l] << (64 - l), and LJ is non-increasing in l,
// so a code's length is lo + #{l in [lo, hi) : W < LJ[l]} for any bounds
// lo <= l <= hi; a table of every kPeek-bit prefix gives those bounds (and
// the symbol itself for codes of at most kPeek bits).
// Sizing: two 1024-lane workgroups share a CU (8 waves per SIMD, which caps
// the kernel at 64 VGPRs), so the per-wave LDS is small: a 1024-symbol
// output tile, segments of about 7/8 of it, regions of at most 96 bits.
// The decoder is issue- and latency-bound (three decodes per code), so the
// extra waves in flight matter more than longer segments would.
constexpr uint32_t kPeek = 12;
constexpr int kDWG = 1024;                          // threads of a decoder workgroup
constexpr int kDWaves = kDWG / kWave;
constexpr uint32_t kTile = 1024;                    // symbols per output round of a wave
constexpr uint32_t kSegSyms = kTile * 7 / 8;        // symbols a segment aims at
constexpr uint32_t kMaxRegion = 96;                 // bits of one lane's region, at most
constexpr uint32_t kWinWords = 2 * kMaxRegion + 8;  // stream words staged per segment
constexpr uint32_t kMapWords = 2 * kMaxRegion + 4;  // code-start bitmap words
constexpr uint32_t kTabShort = 1u << 30;            // table entry: the symbol is in bits [0, 16)
// Books of at most kPairAlphabet symbols (a symbol in 10 bits) use the pair
// form of the table: an entry whose prefix fixes a first code of at most
// kPeek bits has bit 31 set and holds that code's symbol (bits [0, 10)) and
// length (bits [20, 24)), and, when the prefix's remaining bits also hold a
// whole second code, its symbol (bits [10, 20)) and length (bits [24, 28),
// else 0).  One lookup then decodes two codes where both fit the prefix
// (two 6-bit codes on the Lorenzo stream: 57% of lookups).
constexpr uint32_t kPairAlphabet = 1024;
constexpr uint32_t kTabPair = 1u << 31;

template <int SB>
constexpr uint32_t tile_words() {
  return (kTile * SB + 16) / 4;
}
template <int SB>
constexpr uint32_t wave_words() {
  return tile_words<SB>() + kWinWords + kMapWords;
}
template <int SB>
constexpr size_t decode_lds_bytes() {
  return ((size_t)(1u << kPeek) + (size_t)kDWaves * wave_words<SB>()) * 4;
}

// Prefix table: entry p describes the windows whose first kPeek bits are p.
// Bits [16, 23): lo, the shortest code length among them, bits [23, 30): hi,
// the longest.  When hi <= kPeek the prefix fixes the code (lo == hi): bit
// 30 is set and bits [0, 16) hold its symbol, or the entry is 0 if no code
// starts with p (an incomplete code).  `pair`: the pair form above.
__global__ __launch_bounds__(256) void decode_table_kernel(const uint64_t* __restrict__ first,
                                                           const uint32_t* __restrict__ entry,
                                                           const uint32_t* __restrict__ rev,
                                                           const uint64_t* __restrict__ info,
                                                           uint32_t* __restrict__ tab, uint32_t pair) {
  const uint32_t p = blockIdx.x * 256u + threadIdx.x;
  if (p >= (1u << kPeek)) return;
  const uint32_t m = (uint32_t)info[0];
  const uint32_t lmax = (uint32_t)(info[1] < HF_MAX_CODELEN ? info[1] : HF_MAX_CODELEN);
  uint32_t out = 0;
  if (m > 0 && lmax > 0) {
    // length of the code at the top of W: the smallest l with W >= LJ[l]
    // (First[lmax] = 0, so l = lmax always qualifies)
    auto len_of = [&](uint64_t W) -> uint32_t {
      for (uint32_t l = 1; l < lmax; ++l)
        if ((W >> (64 - l)) >= first[l]) return l;
      return lmax;
    };
    const uint64_t wmin = (uint64_t)p << (64 - kPeek);
    const uint64_t wmax = wmin | ((1ull << (64 - kPeek)) - 1);
    const uint32_t lo = len_of(wmax), hi = len_of(wmin);
    out = (lo << 16) | (hi << 23);
    auto count_of = [&](uint32_t l) -> uint32_t { return (l < HF_MAX_CODELEN ? entry[l + 1] : m) - entry[l]; };
    if (hi <= kPeek) {
      const uint64_t v = p >> (kPeek - lo);
      if (v >= first[lo] && v - first[lo] < count_of(lo)) {
        const uint32_t sym = rev[entry[lo] + (uint32_t)(v - first[lo])];
        if (!pair) {
          out |= kTabShort | sym;
        } else {
          out = kTabPair | sym | lo << 20;
          // a second code in the remaining R bits: its length is the smallest
          // l <= R whose first l bits reach First[l] (the canonical rule)
          const uint32_t R = kPeek - lo, q = p & ((1u << R) - 1u);
          for (uint32_t l = 1; l <= R && l <= lmax; ++l) {
            const uint64_t v2 = q >> (R - l);
            if (v2 >= first[l]) {
              if (v2 - first[l] < count_of(l)) out |= rev[entry[l] + (uint32_t)(v2 - first[l])] << 10 | l << 24;
              break;
            }
          }
        }
      } else {
        out = 0;
      }
    }
  }
  tab[p] = out;
}

struct DecArgs {
  const uint32_t* words;
  const uint64_t* offsets;
  uint64_t n;
  uint32_t chunk_log2;
  uint64_t nchunks;
  const uint32_t* gtab;
  const uint64_t* first;
  const uint32_t* entry;
  const uint32_t* rev;
  const uint64_t* info;
  void* out;
  uint32_t* status;
};

// Per-workgroup tables in LDS.
struct DecShared {
  uint64_t first[HF_MAX_CODELEN + 1];
  uint64_t lj[HF_MAX_CODELEN + 4];  // First[l] << (64 - l); 0 past the longest length
  uint32_t entry[HF_MAX_CODELEN + 1];
  uint32_t cnt[HF_MAX_CODELEN + 1];
  uint32_t gcd;
};

// Instruction-order fence between the lanes of one wave: LDS requests of a
// wave are served in order, so this only keeps the compiler from moving LDS
// accesses across it.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The 64 stream bits from relative bit p of the staged words, first bit at the top.
__device__ __forceinline__ uint64_t dec_window(const uint32_t* win, uint32_t p) {
  const uint32_t wi = p >> 5, sh = p & 31;
  const uint64_t x = ((uint64_t)win[wi] << 32) | win[wi + 1];
  return (x << sh) | (((uint64_t)win[wi + 2] << sh) >> 32);
}

// Length of the code at the top of W (0: no code starts there).
__device__ __forceinline__ uint32_t dec_len(uint32_t t, uint64_t W, const uint64_t* lj) {
  const uint32_t lo = (t >> 16) & 127u, hi = (t >> 23) & 127u;
  uint32_t len = lo;
  // four bounds per pass, so a long code waits on one LDS round trip per four
  // lengths: W >= LJ[l] for every l >= hi (LJ is non-increasing), so the terms
  // past hi add nothing
  for (uint32_t l = lo; l < hi; l += 4)
    len += (W < lj[l] ? 1u : 0u) + (W < lj[l + 1] ? 1u : 0u) + (W < lj[l + 2] ? 1u : 0u) + (W < lj[l + 3] ? 1u : 0u);
  return len;
}

// Marks in [p, e) of the code-start bitmap (bit b of word i is position 32 i + b).
__device__ __forceinline__ uint32_t count_marks(const uint32_t* map, uint32_t p, uint32_t e) {
  if (p >= e) return 0u;
  const uint32_t wa = p >> 5, wb = (e - 1) >> 5;
  uint32_t c = 0;
  for (uint32_t w = wa; w <= wb; ++w) {
    uint32_t v = map[w];
    if (w == wa) v &= ~0u << (p & 31);
    if (w == wb && (e & 31)) v &= (1u << (e & 31)) - 1u;
    c += __builtin_popcount(v);
  }
  return c;
}

template <int SB>
__device__ __forceinline__ void tile_put(uint32_t* tile, uint32_t i, uint32_t sym) {
  if (SB == 1) ((uint8_t*)tile)[i] = (uint8_t)sym;
  else ((uint16_t*)tile)[i] = (uint16_t)sym;
}

// Output symbols [D, D + cnt) from tile entries [h, h + cnt), h = D mod G
// (G symbols to 16 bytes), so whole groups are 16-byte aligned on both sides.
template <int SB>
__device__ __forceinline__ void tile_copy_out(const uint32_t* tile, uint32_t h, uint32_t cnt, void* out,
                                              uint64_t D, bool vec) {
  constexpr uint32_t G = 16 / SB;
  const uint32_t lane = lane_id();
  const uint32_t ng = (h + cnt + G - 1) / G;
  char* const base = (char*)out + (D - h) * SB;
  for (uint32_t q = lane; q < ng; q += kWave) {
    const uint32_t lo = q * G, hi = lo + G;
    if (vec && lo >= h && hi <= h + cnt) {
      ((uint4*)base)[q] = ((const uint4*)tile)[q];
    } else {
      const uint32_t a = lo > h ? lo : h, b = hi < h + cnt ? hi : h + cnt;
      for (uint32_t u = a; u < b; ++u) {
        if (SB == 1) ((uint8_t*)base)[u] = ((const uint8_t*)tile)[u];
        else ((uint16_t*)base)[u] = ((const uint16_t*)tile)[u];
      }
    }
  }
}

template <int SB, bool PAIR>
__global__ __launch_bounds__(kDWG) __attribute__((amdgpu_waves_per_eu(8, 8))) void decode_kernel(DecArgs a) {
  extern __shared__ __align__(16) uint32_t dlds[];
  __shared__ DecShared ds;
  const uint32_t tid = threadIdx.x, lane = lane_id(), wv = tid / kWave;
  uint32_t* const tab = dlds;
  uint32_t* const tile = dlds + (1u << kPeek) + wv * wave_words<SB>();
  uint32_t* const win = tile + tile_words<SB>();
  uint32_t* const map = win + kWinWords;

  const uint32_t m = (uint32_t)a.info[0];
  for (uint32_t i = tid; i < (1u << kPeek) / 4; i += kDWG) ((uint4*)tab)[i] = ((const uint4*)a.gtab)[i];
  for (uint32_t l = tid; l < HF_MAX_CODELEN + 4; l += kDWG)
    if (l > HF_MAX_CODELEN) ds.lj[l] = 0;
  for (uint32_t l = tid; l <= HF_MAX_CODELEN; l += kDWG) {
    const uint64_t f = a.first[l];
    ds.first[l] = f;
    ds.lj[l] = l == 0 ? ~0ull : (l == HF_MAX_CODELEN ? f : f << (64 - l));
    ds.entry[l] = a.entry[l];
    ds.cnt[l] = (l < HF_MAX_CODELEN ? a.entry[l + 1] : m) - a.entry[l];
  }
  __syncthreads();
  if (tid == 0) {
    uint32_t g = 0;
    for (uint32_t l = 1; l <= HF_MAX_CODELEN; ++l)
      if (ds.cnt[l]) {
        uint32_t x = l, y = g;
        while (y) {
          const uint32_t t = x % y;
          x = y;
          y = t;
        }
        g = x;
      }
    ds.gcd = g ? g : 1u;
  }
  __syncthreads();
  const uint32_t gcd = ds.gcd;
  const uint64_t total_bits = a.offsets[a.nchunks];
  const uint64_t nwords = (total_bits + 31) >> 5;
  const bool vec = ((uintptr_t)a.out & 15) == 0;
  constexpr uint32_t G = 16 / SB;

  for (uint64_t k = (uint64_t)blockIdx.x * kDWaves + wv; k < a.nchunks; k += (uint64_t)gridDim.x * kDWaves) {
    const uint64_t b0 = a.offsets[k], b1 = a.offsets[k + 1];
    const uint64_t i0 = k << a.chunk_log2;
    const uint32_t ns = (uint32_t)min(a.n - i0, 1ull << a.chunk_log2);
    bool bad = b1 < b0 || b1 > total_bits;
    // region size: about kSegSyms symbols per segment at this chunk's bits per symbol
    uint64_t S64 = bad ? 1 : (b1 - b0) * (kSegSyms / kWave) / ns;
    const uint32_t S = (uint32_t)max(1ull, min((uint64_t)kMaxRegion, S64));
    uint64_t seg = b0;  // a true code boundary
    uint32_t done = 0;  // symbols of the chunk written
    while (!bad && seg < b1) {
      // this segment: regions of Sg bits (all 64 lanes busy on the chunk's tail)
      uint32_t Sg = (uint32_t)min((uint64_t)S, max(1ull, (b1 - seg + kWave - 1) / kWave));
      Sg = Sg >= gcd ? Sg / gcd * gcd : gcd;
      const uint64_t wbase = seg >> 5;
      const uint32_t r0 = (uint32_t)(seg & 31);
      const uint32_t E = (uint32_t)min(b1 - seg, (uint64_t)kWave * Sg) + r0;  // segment end (relative)
      const uint32_t J = min((uint32_t)kWave, (E - r0 + Sg - 1) / Sg);          // lanes with a region
      for (uint32_t i = lane; i < kWinWords; i += kWave) win[i] = wbase + i < nwords ? a.words[wbase + i] : 0u;
      for (uint32_t i = lane; i < kMapWords; i += kWave) map[i] = 0u;
      wave_lds_sync();
      const uint32_t g = min(r0 + lane * Sg, E);
      const uint32_t rend = min(g + Sg, E);

      // A: decode from the region's first bit, marking code starts
      uint32_t s = g, p = g, c = 0;
      while (p < rend) {
        const uint64_t W = dec_window(win, p);
        const uint32_t t = tab[W >> (64 - kPeek)];
        atomicOr(&map[p >> 5], 1u << (p & 31));
        ++c;
        if (PAIR && (t & kTabPair)) {
          const uint32_t q = p + ((t >> 20) & 15u), l2 = (t >> 24) & 15u;
          if (l2 && q < rend) {  // the second code starts in this region too
            atomicOr(&map[q >> 5], 1u << (q & 31));
            ++c;
            p = q + l2;
          } else {
            p = q;
          }
        } else {
          const uint32_t len = dec_len(t, W, ds.lj);
          p += len ? len : 1u;
        }
      }
      const uint32_t eA = p;
      uint32_t e = p;
      wave_lds_sync();

      // B: restart from the left neighbour's end until every start agrees
      for (int it = 0; it < kWave; ++it) {
        uint32_t pe = (uint32_t)__shfl_up((int)e, 1, kWave);
        if (lane == 0) pe = s;
        const bool need = lane < J && pe != s;
        if (__ballot(need) == 0ull) break;
        if (need) {
          s = pe;
          p = s;
          uint32_t cn = 0;
          bool met = false;
          while (p < rend) {
            if ((map[p >> 5] >> (p & 31)) & 1u) {
              met = true;
              break;
            }
            const uint64_t W = dec_window(win, p);
            const uint32_t t = tab[W >> (64 - kPeek)];
            ++cn;
            if (PAIR && (t & kTabPair)) {
              const uint32_t q = p + ((t >> 20) & 15u), l2 = (t >> 24) & 15u;
              if (l2 && q < rend && !((map[q >> 5] >> (q & 31)) & 1u)) {  // (a mark at q ends the walk there)
                ++cn;
                p = q + l2;
              } else {
                p = q;
              }
            } else {
              const uint32_t len = dec_len(t, W, ds.lj);
              p += len ? len : 1u;
            }
          }
          if (met) {
            cn += count_marks(map, p, rend);
            p = eA;
          }
          e = p;
          c = cn;
        }
      }
      if (lane >= J) c = 0;

      // C: output positions, then decode into the tile
      const uint32_t inc = wave_inclusive_scan(c);
      const uint32_t o = inc - c;
      const uint32_t T = (uint32_t)__shfl((int)inc, kWave - 1, kWave);
      const uint32_t eEnd = (uint32_t)__shfl((int)e, (int)J - 1, kWave);
      if (done + T > ns) {
        bad = true;
        break;
      }
      p = s;
      uint32_t td = 0;
      bool lbad = false;
      for (uint32_t rb = 0; rb < T; rb += kTile) {
        const uint64_t D = i0 + done + rb;
        const uint32_t h = (uint32_t)(D & (G - 1));
        while (!lbad && td < c && o + td < rb + kTile) {
          const uint64_t W = dec_window(win, p);
          const uint32_t t = tab[W >> (64 - kPeek)];
          if (PAIR && (t & kTabPair)) {
            tile_put<SB>(tile, h + o + td - rb, t & 1023u);
            p += (t >> 20) & 15u;
            ++td;
            const uint32_t l2 = (t >> 24) & 15u;
            if (l2 && td < c && o + td < rb + kTile) {
              tile_put<SB>(tile, h + o + td - rb, (t >> 10) & 1023u);
              p += l2;
              ++td;
            }
            continue;
          }
          const uint32_t len = dec_len(t, W, ds.lj);
          uint32_t sym = t & 0xFFFFu;
          if (!(t & kTabShort)) {
            bool ok = len != 0;
            if (ok) {
              const uint64_t v = W >> (64 - len);
              const uint64_t f = ds.first[len];
              ok = v >= f && v - f < ds.cnt[len];
              if (ok) {
                const uint32_t idx = ds.entry[len] + (uint32_t)(v - f);
                sym = a.rev[idx];  // codes longer than the table's prefix are rare
              }
            }
            if (!ok) {
              lbad = true;
              break;
            }
          }
          tile_put<SB>(tile, h + o + td - rb, sym);
          p += len;
          ++td;
        }
        wave_lds_sync();
        tile_copy_out<SB>(tile, h, min(kTile, T - rb), a.out, D, vec);
        wave_lds_sync();
      }
      if (__ballot(lbad) != 0ull) bad = true;
      done += T;
      seg = wbase * 32 + eEnd;
    }
    if (bad || done != ns || seg != b1) {
      if (lane == 0) raise_status(a.status, HF_ERR_STREAM);
    }
  }
}

}  // namespace

size_t decode_workspace_bytes() { return (size_t)4 << kPeek; }

hipError_t launch_decode(const uint32_t* words, const uint64_t* offsets, uint64_t n, uint32_t sym_bytes,
                         uint32_t chunk_log2, const hf_codebook& book, void* out, void* ws, uint32_t* status,
                         int num_cus, hipStream_t stream, const KernelTimer& timer) {
  if (n == 0) {
    timer.before(stream);
    timer.after(stream);
    return hipSuccess;
  }
  uint32_t* tab = (uint32_t*)ws;
  const bool pair = book.alphabet <= kPairAlphabet;
  decode_table_kernel<<<(1u << kPeek) / 256, 256, 0, stream>>>(book.first, book.entry, book.rev, book.info, tab,
                                                                pair ? 1u : 0u);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  static std::once_flag once;
  static hipError_t attr_err = hipSuccess;
  std::call_once(once, [] {
    const void* fns[4] = {(const void*)decode_kernel<1, false>, (const void*)decode_kernel<1, true>,
                          (const void*)decode_kernel<2, false>, (const void*)decode_kernel<2, true>};
    for (int i = 0; i < 4 && attr_err == hipSuccess; ++i)
      attr_err = hipFuncSetAttribute(fns[i], hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)(i < 2 ? decode_lds_bytes<1>() : decode_lds_bytes<2>()));
  });
  if (attr_err != hipSuccess) return attr_err;
  const uint64_t nchunks = (n + (1ull << chunk_log2) - 1) >> chunk_log2;
  // persistent waves: two workgroups per CU fit the LDS; each wave takes chunks in turn
  const uint64_t want = (nchunks + kDWaves - 1) / kDWaves;
  const uint32_t grid = (uint32_t)min(want, (uint64_t)max(1, num_cus) * 2);
  DecArgs a{words, offsets, n, chunk_log2, nchunks, tab, book.first, book.entry, book.rev, book.info, out, status};
  timer.before(stream);
  if (sym_bytes == 1) {
    if (pair) decode_kernel<1, true><<<grid, kDWG, decode_lds_bytes<1>(), stream>>>(a);
    else decode_kernel<1, false><<<grid, kDWG, decode_lds_bytes<1>(), stream>>>(a);
  } else {
    if (pair) decode_kernel<2, true><<<grid, kDWG, decode_lds_bytes<2>(), stream>>>(a);
    else decode_kernel<2, false><<<grid, kDWG, decode_lds_bytes<2>(), stream>>>(a);
  }
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
