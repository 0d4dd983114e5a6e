/*
 * hf_cpu.h -- C ABI of libhf_cpu, the multi-core CPU counterpart of libhf:
 * the paper's CPU parallel codebook construction (Sec. 5.2.1, Table 5: the
 * codebook built with OpenMP on the host's cores) and a thread-parallel
 * histogram + encoder (Sec. 5.2.2, Table 6: the multi-thread CPU encoder).
 *
 * It is a baseline to measure the GPU path against, not the oracle: its
 * tests check it against the oracle, never the reverse.  It shares no code
 * with the oracle or with the GPU library.
 *
 * Conventions:
 *  - Every pointer is HOST memory owned by the caller.
 *  - nthreads = 0 uses OpenMP's default team size (OMP_NUM_THREADS, else
 *    the host's cores); hfc_threads(0) says how many that is.
 *  - Return codes are libhf's status numbers: 0 ok, 1 bad argument,
 *    16 symbol outside the alphabet or without a code, 17 output capacity
 *    exceeded, 18 code longer than 64 bits.
 *  - Symbols are uint8 (sym_bytes = 1) or uint16 (sym_bytes = 2);
 *    1 <= alphabet <= 65536; n < 2^32.
 */
#ifndef HF_CPU_H
#define HF_CPU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Threads a call with this nthreads uses. */
int hfc_threads(int nthreads);

/* Sec. 4.1 on the host: hist[s] = number of i < n with sym[i] == s
 * (uint32[alphabet], overwritten).  Each thread counts a contiguous part of
 * the stream into private counters; the parts are summed per bin in
 * parallel.  Symbols >= alphabet are not counted and return 16. */
int hfc_histogram(const void* sym, uint64_t n, uint32_t sym_bytes, uint32_t alphabet, uint32_t* hist,
                  int nthreads);

/* Sec. 4.2 / Algorithm 1 on the host (Table 5): the same codebook as
 * hf_build_codebook (see hf_codebook in hf.h for the arrays: cl[alphabet],
 * cw[alphabet], first[65], entry[65], rev[alphabet], info[4] = {m, Lmax,
 * total bits, shortest length}).  Used symbols are sorted by (count,
 * symbol) with a parallel merge sort; GenerateCL runs as rounds that
 * combine every node no heavier than the two lightest together (ties leaf
 * first, then by rank), each round's merge split into equal output ranges
 * across the threads by co-rank searches; depths follow round by round from
 * the root; codewords are canonical, ranked within each length in symbol
 * order from per-thread counts. */
int hfc_codebook(const uint32_t* hist, uint32_t alphabet, uint8_t* cl, uint64_t* cw, uint64_t* first,
                 uint32_t* entry, uint32_t* rev, uint64_t* info, int nthreads);

/* Sec. 4.3 on the host: the bit-dense stream hf_encode writes (MSB of each
 * code first, bit p in bit 31 - p % 32 of word p / 32, zero-padded last
 * word) and the chunk bit offsets (uint64[ceil(n / chunk) + 1]).  Chunk bit
 * lengths are summed in parallel and prefix-summed; each thread then packs
 * a contiguous run of chunks at its offset, sharing only its first and last
 * word with its neighbours.  chunk: a power of two in [256, 65536].
 * Returns 17 (and writes no stream word) when the stream needs more than
 * cap_words words. */
int hfc_encode(const void* sym, uint64_t n, uint32_t sym_bytes, uint32_t alphabet, const uint8_t* cl,
               const uint64_t* cw, uint32_t chunk, uint32_t* out, uint64_t cap_words, uint64_t* offsets,
               int nthreads);

#ifdef __cplusplus
}
#endif

#endif /* HF_CPU_H */
