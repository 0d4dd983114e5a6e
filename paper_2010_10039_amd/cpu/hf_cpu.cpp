// hf_cpu.cpp -- multi-core CPU histogram, parallel codebook and encoder
// (OpenMP).  The paper's CPU counterparts of the GPU path: the codebook
// built with OpenMP (Sec. 5.2.1, Table 5) and the multi-thread histogram +
// encoder (Sec. 5.2.2, Table 6).  A baseline for measurement, tested
// against the oracle; it shares no code with the oracle or the GPU library.
#include "hf_cpu.h"

#include <omp.h>

#include <algorithm>
#include <cstring>
#include <vector>

namespace {

constexpr int kOk = 0, kErrArg = 1, kErrSymbol = 16, kErrCapacity = 17, kErrCodeLen = 18;
constexpr int kMaxLen = 64;
constexpr uint64_t kInf = ~0ull;
// A round's merge runs on all threads from this many nodes up; below it a
// parallel region costs more than the merge.
constexpr uint32_t kParallelMerge = 16384;

int team(int nthreads) { return nthreads > 0 ? nthreads : omp_get_max_threads(); }

// Part t of T of [0, n).
inline uint64_t part_lo(uint64_t n, int T, int t) { return n * (uint64_t)t / (uint64_t)T; }

template <typename S>
int histogram_impl(const S* x, uint64_t n, uint32_t A, uint32_t* hist, int T) {
  // Peaked data increments the same few bins back to back; four interleaved
  // copies per thread (small alphabets) break that store-to-load chain.
  const uint32_t copies = A <= 4096 ? 4u : 1u;
  const size_t row = (size_t)A * copies;
  std::vector<uint32_t> part((size_t)T * row);
  int used = T, bad = 0;
#pragma omp parallel num_threads(T) reduction(| : bad)
  {
    const int t = omp_get_thread_num(), nt = omp_get_num_threads();
#pragma omp single
    used = nt;
    uint32_t* h = part.data() + (size_t)t * row;
    std::memset(h, 0, row * sizeof(uint32_t));
    const uint64_t lo = part_lo(n, nt, t), hi = part_lo(n, nt, t + 1);
    uint64_t i = lo;
    if (copies == 4) {
      for (; i + 4 <= hi; i += 4) {
        const uint32_t s0 = x[i], s1 = x[i + 1], s2 = x[i + 2], s3 = x[i + 3];
        if ((s0 | s1 | s2 | s3) < A) {
          ++h[s0];
          ++h[A + s1];
          ++h[2 * A + s2];
          ++h[3 * A + s3];
        } else {
          bad = 1;
          if (s0 < A) ++h[s0];
          if (s1 < A) ++h[A + s1];
          if (s2 < A) ++h[2 * A + s2];
          if (s3 < A) ++h[3 * A + s3];
        }
      }
    }
    for (; i < hi; ++i) {
      const uint32_t s = x[i];
      if (s < A) ++h[s];
      else bad = 1;
    }
  }
#pragma omp parallel for num_threads(T) schedule(static)
  for (int64_t b = 0; b < (int64_t)A; ++b) {
    uint32_t c = 0;
    for (int t = 0; t < used; ++t)
      for (uint32_t k = 0; k < copies; ++k) c += part[(size_t)t * row + (size_t)k * A + (size_t)b];
    hist[b] = c;
  }
  return bad ? kErrSymbol : kOk;
}

// Ascending sort of distinct 64-bit keys: sorted parts, then rounds of
// pairwise merges, each round's merges in parallel.
void parallel_sort(std::vector<uint64_t>& key, int T) {
  const size_t m = key.size();
  if (T <= 1 || m < 8192) {
    std::sort(key.begin(), key.end());
    return;
  }
  std::vector<size_t> b(T + 1);
  for (int t = 0; t <= T; ++t) b[t] = (size_t)part_lo(m, T, t);
#pragma omp parallel for num_threads(T) schedule(static, 1)
  for (int t = 0; t < T; ++t) std::sort(key.begin() + b[t], key.begin() + b[t + 1]);
  std::vector<uint64_t> tmp(m);
  for (int w = 1; w < T; w *= 2) {
#pragma omp parallel for num_threads(T) schedule(static, 1)
    for (int i = 0; i < T; i += 2 * w) {
      const size_t lo = b[i], mid = b[std::min(i + w, T)], hi = b[std::min(i + 2 * w, T)];
      std::merge(key.begin() + lo, key.begin() + mid, key.begin() + mid, key.begin() + hi, tmp.begin() + lo);
    }
    key.swap(tmp);
  }
}

// One GenerateCL round's merged sequence: a leaves L[0, a) and b internal
// nodes I[0, b), both ascending, merged with a leaf first on equal weight.
struct RoundMerge {
  const uint64_t* L;
  const uint64_t* I;
  uint32_t a, b;
  uint32_t leaf0, int0;  // node ids of L[0] and I[0]
  uint64_t* mw;
  uint32_t* mid;

  // Number of leaves among the first d merged nodes.
  uint32_t corank(uint32_t d) const {
    uint32_t lo = d > b ? d - b : 0, hi = d < a ? d : a;
    while (lo < hi) {
      const uint32_t i = (lo + hi) / 2, j = d - i;
      if (j > 0 && L[i] <= I[j - 1]) lo = i + 1;  // leaf i precedes internal j - 1: more leaves
      else hi = i;
    }
    return lo;
  }

  // Merged positions [d0, d1).
  void run(uint32_t d0, uint32_t d1) const {
    uint32_t i = corank(d0), j = d0 - i;
    for (uint32_t d = d0; d < d1; ++d) {
      if (j >= b || (i < a && L[i] <= I[j])) {
        mw[d] = L[i];
        mid[d] = leaf0 + i++;
      } else {
        mw[d] = I[j];
        mid[d] = int0 + j++;
      }
    }
  }
};

int codebook_impl(const uint32_t* hist, uint32_t A, uint8_t* cl, uint64_t* cw, uint64_t* first, uint32_t* entry,
                  uint32_t* rev, uint64_t* info, int T) {
  // ---- compaction: used symbols in symbol order -----------------------------
  std::vector<uint32_t> used_before(T + 1, 0);
#pragma omp parallel num_threads(T)
  {
    const int t = omp_get_thread_num(), nt = omp_get_num_threads();
    uint32_t c = 0;
    for (uint64_t s = part_lo(A, nt, t); s < part_lo(A, nt, t + 1); ++s) c += hist[s] != 0;
    used_before[t + 1] = c;
  }
  for (int t = 0; t < T; ++t) used_before[t + 1] += used_before[t];
  const uint32_t m = used_before[T];
  std::vector<uint64_t> key(m);  // count << 32 | symbol: ascending = by (count, symbol)
#pragma omp parallel num_threads(T)
  {
    const int t = omp_get_thread_num(), nt = omp_get_num_threads();
    uint32_t u = used_before[t];
    for (uint64_t s = part_lo(A, nt, t); s < part_lo(A, nt, t + 1); ++s) {
      if (hist[s]) key[u++] = ((uint64_t)hist[s] << 32) | s;
      cl[s] = 0;
      cw[s] = 0;
    }
  }
  for (int l = 0; l <= kMaxLen; ++l) first[l] = 0;
  if (m <= 1) {
    for (int l = 0; l <= kMaxLen; ++l) entry[l] = (m == 1 && l >= 2) ? 1u : 0u;
    uint64_t h0 = 0;
    if (m == 1) {
      const uint32_t s = (uint32_t)key[0];
      h0 = key[0] >> 32;
      cl[s] = 1;
      rev[0] = s;
    }
    info[0] = m;
    info[1] = m;
    info[2] = h0;
    info[3] = m;
    return kOk;
  }

  // ---- sort leaves by (count, symbol) --------------------------------------
  parallel_sort(key, T);
  std::vector<uint64_t> lw(m), iw(m - 1), mw(m);
  std::vector<uint32_t> lsym(m), par(2 * (size_t)m - 1), mid(m);
#pragma omp parallel for num_threads(T) schedule(static) if (m >= 8192)
  for (int64_t i = 0; i < (int64_t)m; ++i) {
    lw[i] = key[i] >> 32;
    lsym[i] = (uint32_t)key[i];
  }

  // ---- GenerateCL rounds -----------------------------------------------------
  // Node ids: leaf of rank i -> i, internal node k (creation order) -> m + k.
  std::vector<uint32_t> rend;  // internal nodes created by the end of each round
  uint32_t lc = 0, ih = 0, it = 0;
  while ((m - lc) + (it - ih) > 1) {
    const uint64_t l0 = lc < m ? lw[lc] : kInf, l1 = lc + 1 < m ? lw[lc + 1] : kInf;
    const uint64_t i0 = ih < it ? iw[ih] : kInf, i1 = ih + 1 < it ? iw[ih + 1] : kInf;
    uint64_t w1, w2;  // the two lightest nodes, leaf first on equal weight
    if (l0 <= i0) {
      w1 = l0;
      w2 = l1 <= i0 ? l1 : i0;
    } else {
      w1 = i0;
      w2 = l0 <= i1 ? l0 : i1;
    }
    const uint64_t t = w1 + w2;
    const uint32_t a = (uint32_t)(std::upper_bound(lw.begin() + lc, lw.end(), t) - (lw.begin() + lc));
    const uint32_t b = it - ih, total = a + b, pairs = total / 2;
    const RoundMerge rm{lw.data() + lc, iw.data() + ih, a, b, lc, m + ih, mw.data(), mid.data()};
    if (T > 1 && total >= kParallelMerge) {
#pragma omp parallel num_threads(T)
      {
        const int th = omp_get_thread_num(), nt = omp_get_num_threads();
        rm.run((uint32_t)part_lo(total, nt, th), (uint32_t)part_lo(total, nt, th + 1));
#pragma omp barrier
#pragma omp for schedule(static)
        for (int64_t p = 0; p < (int64_t)pairs; ++p) {
          iw[it + p] = mw[2 * p] + mw[2 * p + 1];
          par[mid[2 * p]] = m + it + (uint32_t)p;
          par[mid[2 * p + 1]] = m + it + (uint32_t)p;
        }
      }
    } else {
      rm.run(0, total);
      for (uint32_t p = 0; p < pairs; ++p) {
        iw[it + p] = mw[2 * p] + mw[2 * p + 1];
        par[mid[2 * p]] = m + it + p;
        par[mid[2 * p + 1]] = m + it + p;
      }
    }
    // an odd node out is the heaviest merged node; it waits for the next round
    const bool carry_leaf = (total & 1) && mid[total - 1] < m;
    const bool carry_int = (total & 1) && !carry_leaf;
    lc += a - (carry_leaf ? 1u : 0u);
    ih += b - (carry_int ? 1u : 0u);
    it += pairs;
    rend.push_back(it);
  }

  // ---- depths, round by round from the root -----------------------------------
  // A node's parent is created in a later round, so every node of a round
  // can take its depth at once when the later rounds are done.
  std::vector<uint32_t> dep(m - 1);
  const uint32_t root = m - 2;
  for (size_t r = rend.size(); r-- > 0;) {
    const uint32_t k0 = r ? rend[r - 1] : 0, k1 = rend[r];
#pragma omp parallel for num_threads(T) schedule(static) if (k1 - k0 >= kParallelMerge)
    for (int64_t k = k0; k < (int64_t)k1; ++k)
      dep[k] = (uint32_t)k == root ? 0u : dep[par[m + k] - m] + 1;
  }
  int too_long = 0;
#pragma omp parallel for num_threads(T) schedule(static) reduction(| : too_long) if (m >= 8192)
  for (int64_t i = 0; i < (int64_t)m; ++i) {
    const uint32_t l = dep[par[i] - m] + 1;
    if (l > (uint32_t)kMaxLen) too_long = 1;
    cl[lsym[i]] = (uint8_t)std::min<uint32_t>(l, kMaxLen);
  }
  if (too_long) return kErrCodeLen;

  // ---- canonical codewords: per-thread counts per length in symbol order -------
  std::vector<uint64_t> tc((size_t)(T + 1) * (kMaxLen + 1), 0);  // row t + 1: thread t's counts
  uint64_t bits = 0;
#pragma omp parallel num_threads(T) reduction(+ : bits)
  {
    const int t = omp_get_thread_num(), nt = omp_get_num_threads();
    uint64_t* c = tc.data() + (size_t)(t + 1) * (kMaxLen + 1);
    for (uint64_t s = part_lo(A, nt, t); s < part_lo(A, nt, t + 1); ++s) {
      c[cl[s]] += 1;
      bits += (uint64_t)hist[s] * cl[s];
    }
  }
  uint64_t cnt[kMaxLen + 1] = {0};
  for (int t = 1; t <= T; ++t)
    for (int l = 1; l <= kMaxLen; ++l) cnt[l] += tc[(size_t)t * (kMaxLen + 1) + l];
  uint32_t lmax = 0, lmin = 0;
  for (int l = 1; l <= kMaxLen; ++l)
    if (cnt[l]) {
      lmax = (uint32_t)l;
      if (!lmin) lmin = (uint32_t)l;
    }
  for (int l = (int)lmax - 1; l >= 1; --l) first[l] = (first[l + 1] + cnt[l + 1] + 1) / 2;
  uint64_t below = 0;
  for (int l = 0; l <= kMaxLen; ++l) {
    entry[l] = (uint32_t)below;
    if (l >= 1) below += cnt[l];
  }
  // row t becomes thread t's first rev slot per length
  for (int l = 1; l <= kMaxLen; ++l) {
    uint64_t run = entry[l];
    for (int t = 0; t < T; ++t) {
      const uint64_t c = tc[(size_t)(t + 1) * (kMaxLen + 1) + l];
      tc[(size_t)t * (kMaxLen + 1) + l] = run;
      run += c;
    }
  }
#pragma omp parallel num_threads(T)
  {
    const int t = omp_get_thread_num(), nt = omp_get_num_threads();
    uint64_t* next = tc.data() + (size_t)t * (kMaxLen + 1);
    for (uint64_t s = part_lo(A, nt, t); s < part_lo(A, nt, t + 1); ++s) {
      const uint32_t l = cl[s];
      if (!l) continue;
      const uint64_t slot = next[l]++;
      rev[slot] = (uint32_t)s;
      cw[s] = first[l] + (slot - entry[l]);
    }
  }
  info[0] = m;
  info[1] = lmax;
  info[2] = bits;
  info[3] = lmin;
  return kOk;
}

template <typename S>
int encode_impl(const S* x, uint64_t n, uint32_t A, const uint8_t* cl, const uint64_t* cw, uint32_t C,
                uint32_t* out, uint64_t cap, uint64_t* off, int T) {
  const uint64_t nch = (n + C - 1) / C;
  off[0] = 0;
  if (n == 0) return kOk;
  // chunk bit lengths, then an exclusive scan over them (two levels)
  std::vector<uint64_t> tsum(T + 1, 0);
  int bad = 0, used = T;
#pragma omp parallel num_threads(T) reduction(| : bad)
  {
    const int t = omp_get_thread_num(), nt = omp_get_num_threads();
#pragma omp single
    used = nt;
    uint64_t run = 0;
    for (uint64_t k = part_lo(nch, nt, t); k < part_lo(nch, nt, t + 1); ++k) {
      uint64_t B = 0;
      const uint64_t e = std::min<uint64_t>(n, (k + 1) * C);
      for (uint64_t i = k * C; i < e; ++i) {
        const uint32_t s = x[i];
        const uint32_t l = s < A ? cl[s] : 0u;
        bad |= l == 0;
        B += l;
      }
      off[k + 1] = B;
      run += B;
    }
    tsum[t + 1] = run;
  }
  if (bad) return kErrSymbol;
  for (int t = 0; t < used; ++t) tsum[t + 1] += tsum[t];
#pragma omp parallel num_threads(used)
  {
    const int t = omp_get_thread_num();
    uint64_t run = tsum[t];
    for (uint64_t k = part_lo(nch, used, t); k < part_lo(nch, used, t + 1); ++k) {
      run += off[k + 1];
      off[k + 1] = run;
    }
  }
  const uint64_t total = off[nch], nwords = (total + 31) / 32;
  if (nwords > cap) return kErrCapacity;
#pragma omp parallel for num_threads(used) schedule(static)
  for (int64_t w = 0; w < (int64_t)nwords; ++w) out[w] = 0;
  // each thread packs a run of chunks; only its first and last word can be
  // shared with a neighbour, so only those are ORed atomically
#pragma omp parallel num_threads(used)
  {
    const int t = omp_get_thread_num();
    const uint64_t k0 = part_lo(nch, used, t), k1 = part_lo(nch, used, t + 1);
    if (k0 < k1) {
      const uint64_t p0 = off[k0];
      uint64_t acc = 0, wi = p0 >> 5;
      uint32_t nb = (uint32_t)(p0 & 31);
      const uint64_t wshared = (p0 & 31) ? wi : ~0ull;
      auto put = [&](uint32_t v, uint32_t k) {
        acc = (k == 32 ? (acc << 32) : (acc << k)) | v;
        nb += k;
        if (nb >= 32) {
          nb -= 32;
          const uint32_t word = (uint32_t)(acc >> nb);
          if (wi == wshared) __atomic_fetch_or(&out[wi], word, __ATOMIC_RELAXED);
          else out[wi] = word;
          ++wi;
        }
      };
      const uint64_t e = std::min<uint64_t>(n, k1 * C);
      for (uint64_t i = k0 * C; i < e; ++i) {
        const uint32_t s = x[i];
        const uint32_t l = cl[s];
        const uint64_t c = cw[s];
        if (l > 32) {
          put((uint32_t)(c >> 32), l - 32);
          put((uint32_t)c, 32);
        } else {
          put((uint32_t)c, l);
        }
      }
      if (nb) __atomic_fetch_or(&out[wi], (uint32_t)(acc << (32 - nb)), __ATOMIC_RELAXED);
    }
  }
  return kOk;
}

bool valid(uint32_t sym_bytes, uint32_t A, uint64_t n) {
  return (sym_bytes == 1 || sym_bytes == 2) && A >= 1 && A <= 65536u && !(sym_bytes == 1 && A > 256u) &&
         n < (1ull << 32);
}

}  // namespace

extern "C" {

int hfc_threads(int nthreads) { return team(nthreads); }

int hfc_histogram(const void* sym, uint64_t n, uint32_t sym_bytes, uint32_t alphabet, uint32_t* hist,
                  int nthreads) {
  if (!valid(sym_bytes, alphabet, n) || !hist || (n && !sym)) return kErrArg;
  const int T = team(nthreads);
  return sym_bytes == 1 ? histogram_impl((const uint8_t*)sym, n, alphabet, hist, T)
                        : histogram_impl((const uint16_t*)sym, n, alphabet, hist, T);
}

int hfc_codebook(const uint32_t* hist, uint32_t alphabet, uint8_t* cl, uint64_t* cw, uint64_t* first,
                 uint32_t* entry, uint32_t* rev, uint64_t* info, int nthreads) {
  if (!hist || alphabet == 0 || alphabet > 65536u || !cl || !cw || !first || !entry || !rev || !info)
    return kErrArg;
  return codebook_impl(hist, alphabet, cl, cw, first, entry, rev, info, team(nthreads));
}

int hfc_encode(const void* sym, uint64_t n, uint32_t sym_bytes, uint32_t alphabet, const uint8_t* cl,
               const uint64_t* cw, uint32_t chunk, uint32_t* out, uint64_t cap_words, uint64_t* offsets,
               int nthreads) {
  if (!valid(sym_bytes, alphabet, n) || !cl || !cw || !offsets || (n && (!sym || !out))) return kErrArg;
  if (chunk < 256 || chunk > 65536 || (chunk & (chunk - 1))) return kErrArg;
  const int T = team(nthreads);
  return sym_bytes == 1 ? encode_impl((const uint8_t*)sym, n, alphabet, cl, cw, chunk, out, cap_words, offsets, T)
                        : encode_impl((const uint16_t*)sym, n, alphabet, cl, cw, chunk, out, cap_words, offsets, T);
}

}  // extern "C"
