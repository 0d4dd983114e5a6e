/*
 * huff_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, serial, obviously-correct CPU reference for the Huffman encoding
 * path of Tian et al., "Revisiting Huffman Coding: Toward Extreme Performance
 * on Modern GPU Architectures" (arXiv 2010.10039).  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load this library; the
 * product path never does.  It shares no code, header, table or helper with
 * the GPU library.
 *
 * Every result here has a plain textbook definition, so the oracle is that
 * definition written out (no blocking, no fusion, no parallel rounds):
 *
 *   oracle_histogram       Sec. 4.1 (histogramming): h[s] = #{i : x_i = s}.
 *   oracle_code_lengths    Sec. 2.3 / Sec. 4.2.1: an optimal (Huffman) prefix
 *                          code, built with a binary min-heap.  Ties are broken
 *                          by the key (weight, leaf-before-internal, rank):
 *                          leaves ranked by (h[s], s), internal nodes by their
 *                          creation order.  This is the two-queue order in which
 *                          the parallel construction of Algorithm 1 (GenerateCL)
 *                          consumes nodes when it combines everything no heavier
 *                          than the sum of the two lightest subtrees.
 *   oracle_canonical       Sec. 4.2.2 (canonizing): canonical codewords in which
 *                          longer codes are numerically smaller than shorter
 *                          ones at the same prefix length, plus the First and
 *                          Entry decode tables; within one length, codewords go
 *                          to symbols in ascending symbol order.
 *   oracle_encode          Sec. 4.3 (the Merge operator): the bits of code i+1
 *                          follow the bits of code i; MSB of each codeword
 *                          first; bit p of the stream is bit (31 - p%32) of
 *                          32-bit word p/32; the tail is zero padded.  Chunk k
 *                          covers symbols [kC, min((k+1)C, n)) and its start
 *                          offset is the exclusive prefix sum of chunk bit
 *                          lengths (Table 1, "get blockwise code len").
 *   oracle_decode          Sec. 4.2.2: treeless canonical decoding with First
 *                          and Entry.
 *
 * Error codes follow the C ABI of the GPU library numerically (they are
 * restated here, not shared): 0 ok, 1 bad argument, 16 symbol outside the
 * alphabet or without a code, 17 output capacity exceeded, 18 code longer
 * than 64 bits.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_ERR_ARG 1
#define OR_ERR_SYMBOL 16
#define OR_ERR_CAPACITY 17
#define OR_ERR_CODELEN 18
#define OR_MAXLEN 64

static uint32_t sym_at(const void* x, uint64_t i, int sym_bytes) {
  if (sym_bytes == 1) return ((const uint8_t*)x)[i];
  return ((const uint16_t*)x)[i];
}

/* ------------------------------------------------------------------ */
/* Sec. 4.1: frequency of every symbol.                                */
/* ------------------------------------------------------------------ */
int oracle_histogram(const void* x, uint64_t n, int sym_bytes, uint32_t alphabet, uint32_t* h) {
  if ((sym_bytes != 1 && sym_bytes != 2) || alphabet == 0) return OR_ERR_ARG;
  memset(h, 0, sizeof(uint32_t) * alphabet);
  int rc = OR_OK;
  for (uint64_t i = 0; i < n; ++i) {
    uint32_t s = sym_at(x, i, sym_bytes);
    if (s >= alphabet) { rc = OR_ERR_SYMBOL; continue; }
    h[s] += 1;
  }
  return rc;
}

/* ------------------------------------------------------------------ */
/* Huffman code lengths with a binary min-heap.                        */
/* ------------------------------------------------------------------ */
typedef struct {
  uint64_t w;   /* subtree weight */
  uint32_t cls; /* 0 = leaf, 1 = internal node */
  uint32_t idx; /* leaf: rank in (h, s) order; internal: creation number */
} or_node;

static int node_less(const or_node* a, const or_node* b) {
  if (a->w != b->w) return a->w < b->w;
  if (a->cls != b->cls) return a->cls < b->cls;
  return a->idx < b->idx;
}

static void heap_push(or_node* heap, uint32_t* size, or_node v) {
  uint32_t i = (*size)++;
  heap[i] = v;
  while (i > 0) {
    uint32_t p = (i - 1) / 2;
    if (!node_less(&heap[i], &heap[p])) break;
    or_node t = heap[i]; heap[i] = heap[p]; heap[p] = t;
    i = p;
  }
}

static or_node heap_pop(or_node* heap, uint32_t* size) {
  or_node top = heap[0];
  heap[0] = heap[--(*size)];
  uint32_t i = 0;
  for (;;) {
    uint32_t l = 2 * i + 1, r = l + 1, s = i;
    if (l < *size && node_less(&heap[l], &heap[s])) s = l;
    if (r < *size && node_less(&heap[r], &heap[s])) s = r;
    if (s == i) break;
    or_node t = heap[i]; heap[i] = heap[s]; heap[s] = t;
    i = s;
  }
  return top;
}

static const uint32_t* g_sort_h; /* qsort has no context argument */
static int cmp_leaf(const void* pa, const void* pb) {
  uint32_t a = *(const uint32_t*)pa, b = *(const uint32_t*)pb;
  if (g_sort_h[a] != g_sort_h[b]) return g_sort_h[a] < g_sort_h[b] ? -1 : 1;
  return a < b ? -1 : (a > b);
}

/*
 * cl[s] = depth of leaf s in the Huffman tree (0 for unused symbols).
 * One used symbol gets a 1-bit code.  *internal_weight_sum (optional) is the
 * sum of all internal node weights, which equals sum_s h[s]*cl[s].
 */
int oracle_code_lengths(const uint32_t* h, uint32_t alphabet, uint8_t* cl,
                        uint64_t* internal_weight_sum) {
  if (alphabet == 0) return OR_ERR_ARG;
  memset(cl, 0, alphabet);
  if (internal_weight_sum) *internal_weight_sum = 0;
  uint32_t m = 0;
  for (uint32_t s = 0; s < alphabet; ++s) m += (h[s] > 0);
  if (m == 0) return OR_OK;
  uint32_t* order = (uint32_t*)malloc(sizeof(uint32_t) * m);
  for (uint32_t s = 0, j = 0; s < alphabet; ++s)
    if (h[s] > 0) order[j++] = s;
  g_sort_h = h;
  qsort(order, m, sizeof(uint32_t), cmp_leaf);
  if (m == 1) {
    cl[order[0]] = 1;
    if (internal_weight_sum) *internal_weight_sum = h[order[0]];
    free(order);
    return OR_OK;
  }
  /* node ids: leaf of rank r -> r, internal node k -> m + k */
  uint32_t nnodes = 2 * m - 1;
  uint32_t* parent = (uint32_t*)malloc(sizeof(uint32_t) * nnodes);
  uint32_t* depth = (uint32_t*)malloc(sizeof(uint32_t) * nnodes);
  or_node* heap = (or_node*)malloc(sizeof(or_node) * m);
  uint32_t hs = 0;
  for (uint32_t r = 0; r < m; ++r) {
    or_node v = {h[order[r]], 0, r};
    heap_push(heap, &hs, v);
  }
  uint64_t wsum = 0;
  for (uint32_t k = 0; k + 1 < m; ++k) {
    or_node a = heap_pop(heap, &hs);
    or_node b = heap_pop(heap, &hs);
    uint32_t ida = a.cls ? m + a.idx : a.idx;
    uint32_t idb = b.cls ? m + b.idx : b.idx;
    parent[ida] = m + k;
    parent[idb] = m + k;
    or_node t = {a.w + b.w, 1, k};
    wsum += t.w;
    heap_push(heap, &hs, t);
  }
  /* the root is the last internal node; a parent is always created after
     its children, so one pass over decreasing ids fills every depth */
  uint32_t root = nnodes - 1;
  depth[root] = 0;
  int rc = OR_OK;
  for (int64_t id = (int64_t)root - 1; id >= 0; --id) depth[id] = depth[parent[id]] + 1;
  for (uint32_t r = 0; r < m; ++r) {
    if (depth[r] > OR_MAXLEN) rc = OR_ERR_CODELEN;
    cl[order[r]] = (uint8_t)(depth[r] > 255 ? 255 : depth[r]);
  }
  if (internal_weight_sum) *internal_weight_sum = wsum;
  free(heap); free(depth); free(parent); free(order);
  return rc;
}

/* ------------------------------------------------------------------ */
/* Sec. 4.2.2: canonical codewords and the First / Entry tables.       */
/* ------------------------------------------------------------------ */
/*
 * cnt[l]   = number of symbols with code length l (l >= 1).
 * first[L] = 0 for the longest length L; for shorter lengths
 *            first[l] = ceil((first[l+1] + cnt[l+1]) / 2).  The l-bit
 *            prefixes of all longer codes are then < first[l], which is what
 *            lets the decoder tell "need another bit" from "code complete".
 * entry[l] = number of codes shorter than l.
 * Symbols of length l receive first[l], first[l]+1, ... in ascending symbol
 * order; rev[entry[l] + j] is the symbol holding first[l] + j.
 * first[] and entry[] have 65 entries; first[l] = 0 for l = 0 and l > L,
 * entry[l] is defined for every l in [0, 64].  rev entries [m, alphabet)
 * are left untouched.  info = {m, L, 0, shortest length}.
 */
int oracle_canonical(const uint8_t* cl, uint32_t alphabet, uint64_t* cw, uint64_t* first,
                     uint32_t* entry, uint32_t* rev, uint64_t* info) {
  if (alphabet == 0) return OR_ERR_ARG;
  uint64_t cnt[OR_MAXLEN + 2];
  memset(cnt, 0, sizeof(cnt));
  uint32_t m = 0, lmax = 0, lmin = 0;
  for (uint32_t s = 0; s < alphabet; ++s) {
    uint32_t l = cl[s];
    if (l == 0) continue;
    if (l > OR_MAXLEN) return OR_ERR_CODELEN;
    cnt[l] += 1;
    m += 1;
    if (l > lmax) lmax = l;
    if (lmin == 0 || l < lmin) lmin = l;
  }
  for (int l = 0; l <= OR_MAXLEN; ++l) first[l] = 0;
  for (int l = (int)lmax - 1; l >= 1; --l) first[l] = (first[l + 1] + cnt[l + 1] + 1) / 2;
  uint64_t below = 0;
  for (int l = 0; l <= OR_MAXLEN; ++l) {
    entry[l] = (uint32_t)below;
    if (l >= 1) below += cnt[l];
  }
  uint64_t next_code[OR_MAXLEN + 1];
  uint64_t next_slot[OR_MAXLEN + 1];
  for (int l = 0; l <= OR_MAXLEN; ++l) {
    next_code[l] = first[l];
    next_slot[l] = entry[l];
  }
  for (uint32_t s = 0; s < alphabet; ++s) {
    uint32_t l = cl[s];
    if (l == 0) { cw[s] = 0; continue; }
    cw[s] = next_code[l]++;
    rev[next_slot[l]++] = s;
  }
  info[0] = m;
  info[1] = lmax;
  info[2] = 0;
  info[3] = lmin;
  return OR_OK;
}

/* Full codebook from a histogram: lengths, canonical codes, total bits. */
int oracle_codebook(const uint32_t* h, uint32_t alphabet, uint8_t* cl, uint64_t* cw,
                    uint64_t* first, uint32_t* entry, uint32_t* rev, uint64_t* info) {
  int rc = oracle_code_lengths(h, alphabet, cl, NULL);
  if (rc != OR_OK) return rc;
  rc = oracle_canonical(cl, alphabet, cw, first, entry, rev, info);
  if (rc != OR_OK) return rc;
  uint64_t bits = 0;
  for (uint32_t s = 0; s < alphabet; ++s) bits += (uint64_t)h[s] * cl[s];
  info[2] = bits;
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Sec. 4.3: serial concatenation of codewords, chunk offsets.         */
/* ------------------------------------------------------------------ */
/*
 * out must hold cap_words words; words [0, ceil(total/32)) are written.
 * offsets must hold ceil(n/chunk)+1 entries.  *total_bits receives the
 * stream length.  Returns OR_ERR_SYMBOL if a symbol is >= alphabet or has
 * no code, OR_ERR_CAPACITY if the stream does not fit.
 */
int oracle_encode(const void* x, uint64_t n, int sym_bytes, uint32_t alphabet,
                  const uint8_t* cl, const uint64_t* cw, uint64_t chunk, uint32_t* out,
                  uint64_t cap_words, uint64_t* offsets, uint64_t* total_bits) {
  if ((sym_bytes != 1 && sym_bytes != 2) || chunk == 0) return OR_ERR_ARG;
  uint64_t p = 0;
  uint64_t k = 0;
  for (uint64_t i = 0; i < n; ++i) {
    if (i % chunk == 0) offsets[k++] = p;
    uint32_t s = sym_at(x, i, sym_bytes);
    if (s >= alphabet || cl[s] == 0) return OR_ERR_SYMBOL;
    uint32_t l = cl[s];
    for (int j = (int)l - 1; j >= 0; --j) {
      uint64_t word = p >> 5;
      if (word >= cap_words) return OR_ERR_CAPACITY;
      if ((p & 31) == 0) out[word] = 0;
      if ((cw[s] >> j) & 1) out[word] |= 1u << (31 - (p & 31));
      p += 1;
    }
  }
  offsets[k] = p;
  if (total_bits) *total_bits = p;
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Sec. 4.2.2: treeless canonical decoding.                            */
/* ------------------------------------------------------------------ */
/*
 * Reads n symbols starting at bit `start` of `in` (nbits valid bits) for a
 * code with m codewords and longest length lmax:
 * v = next bit, l = 1; while v < first[l]: v = 2v + next bit, l += 1;
 * the code is valid when v - first[l] < cnt[l], and then
 * symbol = rev[entry[l] + v - first[l]].  *end_bit receives the bit position
 * after the last symbol.  Returns OR_ERR_SYMBOL on an invalid code or when
 * the stream runs out.
 */
int oracle_decode(const uint32_t* in, uint64_t start, uint64_t nbits, uint64_t n,
                  const uint64_t* first, const uint32_t* entry, const uint32_t* rev,
                  uint32_t m, uint32_t lmax, int sym_bytes, void* x_out, uint64_t* end_bit) {
  if ((sym_bytes != 1 && sym_bytes != 2) || lmax > OR_MAXLEN) return OR_ERR_ARG;
  uint64_t p = start;
  for (uint64_t i = 0; i < n; ++i) {
    if (p >= nbits) return OR_ERR_SYMBOL;
    uint64_t v = (in[p >> 5] >> (31 - (p & 31))) & 1;
    p += 1;
    uint32_t l = 1;
    while (l <= lmax && v < first[l]) {
      if (p >= nbits) return OR_ERR_SYMBOL;
      v = 2 * v + ((in[p >> 5] >> (31 - (p & 31))) & 1);
      p += 1;
      l += 1;
    }
    if (l > lmax) return OR_ERR_SYMBOL;
    uint64_t cnt_l = (l < OR_MAXLEN ? entry[l + 1] : m) - entry[l];
    if (v - first[l] >= cnt_l) return OR_ERR_SYMBOL;
    uint32_t s = rev[entry[l] + (v - first[l])];
    if (sym_bytes == 1) ((uint8_t*)x_out)[i] = (uint8_t)s;
    else ((uint16_t*)x_out)[i] = (uint16_t)s;
  }
  if (end_bit) *end_bit = p;
  return OR_OK;
}
