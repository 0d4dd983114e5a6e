/*
 * hf.h -- C ABI of libhf, an MI355X (gfx950) Huffman encoder for streams of
 * fixed-width integer symbols, after Tian et al., "Revisiting Huffman Coding:
 * Toward Extreme Performance on Modern GPU Architectures" (arXiv 2010.10039).
 *
 * The paper splits encoding into four stages (Sec. 4): histogramming,
 * codebook construction, canonization, and encoding with bit
 * concatenation.  hf_histogram is stage 1, hf_build_codebook is stages 2+3,
 * hf_encode is stage 4; hf_decode inverts it, and hf_decode_check re-reads the stream with the
 * canonical decode tables and compares it with the input.
 *
 * Conventions shared by every entry point:
 *  - Every buffer argument named d_* is DEVICE memory owned by the caller.
 *    libhf never allocates, frees or retains device memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls only enqueue work on that stream; they return before it runs.
 *  - The return value reports errors the host can detect (arguments,
 *    workspace size, launch failure).  Errors found while kernels run are
 *    written to *d_status (one uint32, caller-zeroed) with first-error-wins
 *    semantics; the caller reads it after synchronizing.
 *  - A workspace (d_ws, ws_bytes) is scratch device memory, at least
 *    hf_workspace_bytes() bytes, 256-byte aligned, with no required
 *    contents.  One workspace must not be used by two calls that can run at
 *    the same time.
 *  - Symbols are uint8 (sym_bytes = 1) or little-endian uint16
 *    (sym_bytes = 2); 1 <= alphabet <= 65536, alphabet <= 256 for uint8;
 *    n < 2^32 symbols per call.
 */
#ifndef HF_H
#define HF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HF_OK = 0,
  HF_ERR_ARG = 1,        /* bad argument (host) */
  HF_ERR_WORKSPACE = 2,  /* workspace missing or too small (host) */
  HF_ERR_LAUNCH = 3,     /* a kernel launch failed (host) */
  HF_ERR_SYMBOL = 16,    /* a symbol >= alphabet, or one without a code (device) */
  HF_ERR_CAPACITY = 17,  /* encoded stream longer than the output buffer (device) */
  HF_ERR_CODELEN = 18,   /* a code longer than 64 bits (device; unreachable for n < 2^32) */
  HF_ERR_MISMATCH = 19,  /* hf_decode_check found a difference (device) */
  HF_ERR_INTERNAL = 20,  /* a bounded wait or loop hit its limit (device; a bug guard) */
  HF_ERR_STREAM = 21,    /* hf_decode: a chunk does not decode with the codebook (device) */
  HF_ERR_VALUE = 22      /* hf_lorenzo_histogram: a value of the field is NaN or infinite (device) */
} hf_status;

#define HF_MAX_CODELEN 64

/*
 * The codebook: all pointers are device arrays owned by the caller.
 *   cl[alphabet]  uint8   code length of each symbol; 0 = symbol unused.
 *   cw[alphabet]  uint64  codeword in the low cl bits, sent MSB first; 0 if unused.
 *   first[65]     uint64  first (smallest) codeword of each length l in
 *                         [1, Lmax]; 0 for l = 0 and l > Lmax.
 *   entry[65]     uint32  number of codewords shorter than l, l in [0, 64].
 *   rev[alphabet] uint32  symbols ordered by (length, symbol); rev[entry[l] + j]
 *                         holds codeword first[l] + j.  Entries [m, alphabet)
 *                         are left untouched.
 *   info[4]       uint64  {m = used symbols, Lmax, total_bits = sum h[s]*cl[s],
 *                          shortest length}.
 * Canonical form (Sec. 4.2.2 and Algorithm 1, GenerateCW): at any prefix
 * length l, the l-bit prefix of a longer code is numerically smaller than
 * first[l]; first[Lmax] = 0 and first[l] = ceil((first[l+1] + cnt[l+1]) / 2);
 * codes of one length ascend with the symbol id.  One used symbol gets the
 * 1-bit code 0.
 */
typedef struct hf_codebook {
  uint32_t alphabet;
  uint8_t* cl;
  uint64_t* cw;
  uint64_t* first;
  uint32_t* entry;
  uint32_t* rev;
  uint64_t* info;
} hf_codebook;

/* Workspace bytes that suffice for every entry point below on a stream of n
 * symbols with this alphabet and chunk size (any reduce_log2). */
size_t hf_workspace_bytes(uint64_t n, uint32_t alphabet, uint32_t chunk_symbols);

/* Output words that always suffice without reading total_bits: a Huffman
 * code averages at most ceil(log2 alphabet) + 1 bits per symbol. */
uint64_t hf_bound_words(uint64_t n, uint32_t alphabet);

/* The paper's reduction-factor rule (Sec. 4.3, Interface):
 * floor(log2 beta) + r + 1 = log2(l_W) with l_W = 32 bits, for an average
 * code length beta (bits per symbol), clamped to [1, 6].  A performance
 * prior only; hf_encode's output does not depend on r. */
uint32_t hf_reduction_factor(double beta);

/* Human-readable name of a status code (static storage). */
const char* hf_status_string(uint32_t code);

/*
 * Slabs: the stream is cut into S slabs of whole 4096-symbol blocks, slab g
 * covering blocks [floor(g*nb/S), floor((g+1)*nb/S)) of nb = ceil(n/4096).
 * hf_slab_count() returns the S that keeps one encoder workgroup per slab
 * resident on this device (0 when per-slab counts are not worth keeping:
 * alphabets above 4096).  Per-slab counts let hf_encode place every slab's
 * bits without reading the input a second time.  Any slab count passed to
 * hf_histogram or hf_encode must satisfy 1 <= S <= min(nb, 16384).
 */
uint32_t hf_slab_count(uint64_t n, uint32_t alphabet);

/*
 * Stage 1, histogramming (Sec. 4.1): d_hist[s] = number of i < n with
 * d_sym[i] == s, for s < alphabet.  d_hist (uint32[alphabet]) is
 * overwritten.  If d_slab_hist is not NULL (then nslabs >= 1, alphabet <=
 * 4096), d_slab_hist[g * alphabet + s] (uint32[nslabs * alphabet]) receives
 * the count of s inside slab g.  Symbols >= alphabet are not counted and
 * raise HF_ERR_SYMBOL in *d_status.  Each workgroup counts its slab in
 * interleaved replicated sub-histograms in LDS and stores the slab's row of
 * counts (into d_slab_hist, or, when that is NULL and the alphabet is at
 * most 4096, into the workspace); a second kernel then sums the rows into
 * d_hist.  Alphabets above 4096 keep no rows: each workgroup adds its
 * totals to d_hist with one global atomic per non-zero bin, in passes over
 * bin windows that fit LDS.
 */
hf_status hf_histogram(const void* d_sym, uint64_t n, uint32_t sym_bytes, uint32_t alphabet,
                       uint32_t* d_hist, uint32_t nslabs, uint32_t* d_slab_hist, void* d_ws,
                       size_t ws_bytes, uint32_t* d_status, void* stream);

/*
 * Fused front end for the paper's multi-byte input (Sec. 5.1.3: the
 * quantization codes an SZ-style error-bounded compressor makes from a float
 * field), so that stage 1 needs no pass of its own over the codes.
 * d_field is float32[nz][ny][nx] in C order (flat index
 * f = (i * ny + j) * nx + k); n = nz * ny * nx < 2^32.  For every element:
 *   d = rint(x * inv_2eb) in float32 (ties to even), clamped to
 *       [-2^24, 2^24] -- inv_2eb is 1 / (2 eb) for an absolute error bound
 *       eb;
 *   e = the 3D Lorenzo residual of d: the mixed first difference along the
 *       three axes, with d = 0 outside the grid (eight neighbours, signs
 *       (-1)^(di + dj + dk));
 *   d_codes[f] (uint16[n]) = e + radius if 1 <= e + radius <= 2 radius - 1,
 *       else 0 (the outlier code); the alphabet is 2 radius.
 * d_hist (uint32[2 radius]) is overwritten with the counts of the codes.
 * If d_slab_hist is not NULL, it receives the per-slab counts exactly as
 * hf_histogram would for d_codes (same nslabs rules, 2 radius <= 4096), ready
 * for hf_encode.  Requirements (else HF_ERR_ARG): 1 <= radius <= 8192;
 * inv_2eb finite and > 0; nx <= 8192 when ny > 1; d_field 4-byte and d_codes
 * 2-byte aligned (16-byte alignment of both and nx % 8 == 0 take the
 * vector path); d_status not NULL.  A NaN or an infinity in the field is
 * outside an error-bounded quantizer's domain (no finite value lies within
 * eb of it): it raises HF_ERR_VALUE in *d_status, and the codes and counts
 * are then unspecified.  Workgroups stream their part of the field once
 * (four slabs one plane apart share their plane-back values when the shape
 * allows), and keep the previous row's partial differences in LDS.
 */
hf_status hf_lorenzo_histogram(const float* d_field, uint32_t nz, uint32_t ny, uint32_t nx, float inv_2eb,
                               uint32_t radius, uint16_t* d_codes, uint32_t* d_hist, uint32_t nslabs,
                               uint32_t* d_slab_hist, uint32_t* d_status, void* stream);

/*
 * The paper's own output format, kept as an ablation beside hf_encode's
 * exact dense stream (Sec. 4.3, Interface ReduceShuffleMerge<M, r>;
 * Sec. 5.2.2 and Table 3).  Chunks of 2^M symbols (chunk_log2 = M in
 * [8, 12]) are cut into groups of 2^r symbols (reduce_log2 = r in [1, 5]).
 * A group's codes, merged MSB first, form one word when they total at most
 * 32 bits; a group needing more is "breaking": it is left out of the stream
 * and recorded in a side channel, its global group index in
 * d_break_groups (uint64, ascending) and its 2^r raw symbols (zero padded
 * when the last group is short) in d_break_syms (the symbol type).  A
 * chunk's stream is the concatenation of its non-breaking group words,
 * padded to a whole 32-bit word; chunks follow one another, chunk k
 * starting at word d_chunk_word_offsets[k] (uint64[nchunks + 1], total
 * words at [nchunks]).  *d_nbreak (uint64) receives the number of breaking
 * groups.  Output beyond out_capacity_words words or break_capacity groups
 * is not written and raises HF_ERR_CAPACITY; a symbol outside the alphabet
 * or without a code raises HF_ERR_SYMBOL.  Workspace:
 * hf_paper_workspace_bytes(n, chunk_log2).
 */
size_t hf_paper_workspace_bytes(uint64_t n, uint32_t chunk_log2);
hf_status hf_encode_paper(const void* d_sym, uint64_t n, uint32_t sym_bytes, const hf_codebook* book,
                          uint32_t chunk_log2, uint32_t reduce_log2, uint32_t* d_out, uint64_t out_capacity_words,
                          uint64_t* d_chunk_word_offsets, uint64_t* d_break_groups, void* d_break_syms,
                          uint64_t break_capacity, uint64_t* d_nbreak, void* d_ws, size_t ws_bytes,
                          uint32_t* d_status, void* stream);

/*
 * Stages 2 and 3, codebook construction and canonization (Sec. 4.2,
 * Algorithm 1): from d_hist (uint32[book->alphabet]) fill every array of
 * *book (see hf_codebook).  Leaves are sorted by (count, symbol); code
 * lengths come from parallel rounds that combine every subtree no heavier
 * than the two lightest together, with ties taken leaf-first and then by
 * rank, which is exactly the code a heap-based Huffman construction gives
 * under that order; codewords are canonical as described above.  One
 * workgroup builds the book; the tree lives in LDS when at most 4096
 * symbols are used, else in the workspace.  For alphabets above 8192 with
 * more than 4096 used symbols the sort, the code lengths and the codewords
 * run over up to 64 workgroups (the rounds stay in one); the workspace
 * (hf_workspace_bytes) then also holds their buffers.  Enqueues up to five
 * kernels, none of which waits for the host.  Raises HF_ERR_CODELEN if a
 * code would exceed 64 bits, HF_ERR_INTERNAL if a bounded wait between the
 * grid-wide steps' workgroups ran out.
 */
hf_status hf_build_codebook(const uint32_t* d_hist, const hf_codebook* book, void* d_ws,
                            size_t ws_bytes, uint32_t* d_status, void* stream);

/*
 * hf_build_codebook with phase timestamps, for profiling the construction
 * of Sec. 4.2 (Table 2 splits it into code lengths and codewords).  Same
 * arguments, result and errors; in addition d_stamps (device, uint64[9],
 * caller-owned) receives the shader clock (s_memtime, core cycles) of the
 * single-workgroup build as it passes each phase: [0] start, [1] histogram
 * read and summed, [2] used symbols compacted, [3] sorted, [4] GenerateCL
 * rounds done, [5] depths, [6] code lengths, [7] First and Entry, [8] end.
 * Words of phases a build does not pass (no tree for fewer than two used
 * symbols; alphabets above 8192 with more than 4096 used symbols, whose
 * sort, lengths and codewords run over the whole grid) keep their
 * contents: zero them first.  HF_ERR_ARG if d_stamps is NULL.
 */
hf_status hf_build_codebook_traced(const uint32_t* d_hist, const hf_codebook* book, void* d_ws,
                                   size_t ws_bytes, uint32_t* d_status, uint64_t* d_stamps, void* stream);

/*
 * Stage 4, encoding (Sec. 4.3): the concatenation, in input order, of the
 * codewords of d_sym[0..n) (MSB of each codeword first), written bit-dense
 * into d_out: bit p of the stream is bit 31 - (p % 32) of d_out[p / 32]; the
 * last word is zero padded; words past ceil(total_bits / 32) are untouched.
 * d_chunk_bit_offsets (uint64[ceil(n / chunk_symbols) + 1]) receives the
 * starting bit of every chunk of chunk_symbols symbols and, last, the total
 * bit count, so that each chunk can be decoded independently (Sec. 3.1).
 *   chunk_symbols: a power of two in [256, 65536].
 *   reduce_log2:   r of the paper's ReduceShuffleMerge<M, r>; each lane
 *                  merges 2^r consecutive codewords in registers before the
 *                  workgroup-wide shuffle-merge; 1..6, or 0 for the library
 *                  default.  The output does not depend on it.
 *   nslabs, d_slab_hist: the slab partition and per-slab counts written by
 *                  hf_histogram for these same symbols, or d_slab_hist = NULL
 *                  (then nslabs = 0 picks hf_slab_count or a default, and
 *                  one extra pass over the input counts bits per slab).
 * The result is bit-identical for every chunk_symbols, reduce_log2 and
 * slab partition.  Raises HF_ERR_SYMBOL for a symbol >= alphabet or with
 * cl == 0, or when d_slab_hist does not hold these symbols' per-slab counts
 * (a slab's bits then differ from its counted total; the stream is
 * unspecified), and HF_ERR_CAPACITY when total_bits > 32 * out_capacity_words
 * (nothing is written at or past d_out[out_capacity_words]).
 */
hf_status hf_encode(const void* d_sym, uint64_t n, uint32_t sym_bytes, const hf_codebook* book,
                    uint32_t chunk_symbols, uint32_t reduce_log2, uint32_t nslabs,
                    const uint32_t* d_slab_hist, uint32_t* d_out, uint64_t out_capacity_words,
                    uint64_t* d_chunk_bit_offsets, void* d_ws, size_t ws_bytes,
                    uint32_t* d_status, void* stream);

/*
 * hf_encode without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Arguments, output and device errors
 * are exactly hf_encode's.  The workspace is instead a fixed array of
 * HF_NOALLOC_SCRATCH_BYTES in device memory, one per GPU, held from the
 * library's first use on that GPU until the process ends; this call
 * allocates nothing.  Returns HF_ERR_WORKSPACE if hf_encode's workspace for
 * this slab count and alphabet would not fit the array (it always fits for
 * the arguments hf_encode accepts: 16384 slabs take 192 KiB and the table of
 * a 65536-symbol alphabet 256 KiB), and HF_ERR_LAUNCH if the array's device
 * address cannot be found.  Nothing needs to start at zero.  All calls
 * on one GPU share the array: calls that can run at the same time on one
 * GPU (different streams, or different host threads) race on it and must
 * not be made; calls ordered on one stream are safe.
 */
#define HF_NOALLOC_SCRATCH_BYTES (512u << 10)
hf_status hf_encode_noalloc(const void* d_sym, uint64_t n, uint32_t sym_bytes, const hf_codebook* book,
                            uint32_t chunk_symbols, uint32_t reduce_log2, uint32_t nslabs,
                            const uint32_t* d_slab_hist, uint32_t* d_out, uint64_t out_capacity_words,
                            uint64_t* d_chunk_bit_offsets, uint32_t* d_status, void* stream);

/*
 * Decoder (the inverse path; the paper scopes decoding out, Sec. 1, and
 * gives its tables in Sec. 4.2.2 and Table 1): writes the n symbols encoded
 * in d_in (a stream from hf_encode with its chunk offsets, chunk_symbols as
 * used there, and the same codebook) to d_sym_out (n * sym_bytes bytes).
 * Treeless canonical decoding: the first l bits v form a code of length l
 * when First[l] <= v < First[l] + (Entry[l + 1] - Entry[l]) and l is the
 * smallest such length; its symbol is rev[Entry[l] + v - First[l]].  Each
 * chunk, from its offset, is decoded by one wave whose lanes start at fixed
 * bit strides and resynchronise (a decode begun off a code boundary falls
 * into step with the true one after a few codes), then decode again from
 * their true starts into their output positions.  A table of every 12-bit
 * prefix (its code, or its range of code lengths) is built in d_ws
 * (hf_decode_workspace_bytes(), 16 KiB, 256-byte aligned).  A chunk that
 * meets a bit pattern that is no code, ends off its next offset, or holds
 * another number of codes than its symbols raises HF_ERR_STREAM (its
 * symbols are then unspecified).  d_in must hold ceil(offsets[nchunks] / 32)
 * words.
 */
size_t hf_decode_workspace_bytes(void);
hf_status hf_decode(const uint32_t* d_in, const uint64_t* d_chunk_bit_offsets, uint64_t n,
                    uint32_t sym_bytes, uint32_t chunk_symbols, const hf_codebook* book, void* d_sym_out,
                    void* d_ws, size_t ws_bytes, uint32_t* d_status, void* stream);

/*
 * Checker: decodes every chunk of d_out from its offset with the canonical
 * First/Entry/rev tables (treeless decoding, Sec. 4.2.2), one bit at a time
 * and one lane per chunk, independently of hf_decode's tables, and compares
 * it with d_sym_expected.  It needs no workspace.  d_result (uint64[2]) receives {number of
 * mismatching symbols (a chunk whose decoding ends off its next offset
 * counts one more), index of the first mismatching symbol or n if none}.
 * Raises HF_ERR_MISMATCH in *d_status when the count is not zero.
 */
hf_status hf_decode_check(const uint32_t* d_out, const uint64_t* d_chunk_bit_offsets,
                          uint64_t n, uint32_t sym_bytes, uint32_t chunk_symbols,
                          const hf_codebook* book, const void* d_sym_expected,
                          uint64_t* d_result, uint32_t* d_status, void* stream);

/*
 * Batched encoding of many independent streams, each with its own symbol
 * width, alphabet and codebook (an extension beyond the paper, which
 * encodes one stream at a time).  Every stream gets exactly what
 * hf_histogram + hf_build_codebook + hf_encode would produce for it alone.
 * All pointers in a descriptor are device memory owned by the caller;
 * `book` is written.  hist may be NULL.  Limits per stream: n < 2^32,
 * book.alphabet <= 8192 (<= 256 for sym_bytes 1), chunk_symbols a power of
 * two in [256, 65536], reduce_log2 3, 4, 5 or 0 (the library default);
 * reserved must be 0.  The output is bit-identical whatever the other
 * streams of the batch are.
 */
typedef struct hf_stream_desc {
  const void* sym;
  uint64_t n;
  uint32_t sym_bytes;
  uint32_t chunk_symbols;
  uint32_t reduce_log2;
  uint32_t reserved;
  uint32_t* hist;
  hf_codebook book;
  uint32_t* out;
  uint64_t out_capacity_words;
  uint64_t* chunk_bit_offsets;
} hf_stream_desc;

/* Workspace bytes hf_encode_batch and hf_encode_batch_persistent need for
 * these descriptors (0 if one is invalid). */
size_t hf_batch_workspace_bytes(const hf_stream_desc* descs, uint32_t nstreams);

/*
 * Encodes all streams with one launch per stage, whatever their number:
 * per-slab histograms of every stream; their sum per stream (the stream's
 * histogram, written to hist when given); one workgroup per stream that
 * builds its book (as hf_build_codebook); the bit total of every slab; then
 * every slab of every stream is encoded as hf_encode does (Sec. 4.1-4.3
 * applied to each stream).
 * `descs` is a HOST array of nstreams descriptors; the plan derived from it
 * is copied to the workspace through library-owned pinned host buffers
 * (reused once their copy has completed) before the kernels run, so descs
 * may be reused when the call returns.  Calls on different streams do not
 * wait for each other.
 * d_status is uint32[nstreams], caller-zeroed; stream s's device errors go
 * to d_status[s].  Returns HF_ERR_ARG if any descriptor is invalid (nothing
 * is launched).
 */
hf_status hf_encode_batch(const hf_stream_desc* descs, uint32_t nstreams, void* d_ws, size_t ws_bytes,
                          uint32_t* d_status, void* stream);

/*
 * The same work as hf_encode_batch, with the same arguments, workspace
 * (hf_batch_workspace_bytes) and results, in ONE persistent launch: a grid
 * of resident workgroups takes work items from a device queue in the order
 * slab histograms, per-stream histogram sums, codebooks, slab bit totals,
 * slab encodings, and each item waits only for per-stream device counters
 * of earlier items (no grid-wide barrier), so the streams' stages overlap.
 * Every item of the queue depends only on earlier items, so the queue
 * always drains; a wait that exceeds its spin limit (a fraction of a
 * second) records HF_ERR_INTERNAL in its stream's status word and closes
 * the queue instead of hanging.  Calls that share a workspace must not
 * overlap.
 * CURRENTLY SWITCHED OFF: returns HF_ERR_LAUNCH and launches nothing (the
 * kernel's first run made a memory fault whose cause is not found yet).
 */
hf_status hf_encode_batch_persistent(const hf_stream_desc* descs, uint32_t nstreams, void* d_ws, size_t ws_bytes,
                                     uint32_t* d_status, void* stream);

/*
 * Profiling hook: for the next call of hf_histogram, hf_build_codebook,
 * hf_encode or hf_encode_batch made by this host thread, record hipEvent_t
 * `before` immediately before that call's main kernel (for hf_encode_batch:
 * its encoding launches) and `after` immediately after it, on the call's
 * stream.  Either may be NULL to clear the hook.  One-shot.
 */
hf_status hf_time_next_main_kernel(void* before_event, void* after_event);

#ifdef __cplusplus
}
#endif

#endif /* HF_H */
