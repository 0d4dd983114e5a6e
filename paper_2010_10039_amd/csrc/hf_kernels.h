// hf_kernels.h -- host-side launchers of the libhf kernels (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hf.h"

namespace hf {

constexpr int kHistThreads = 256;
constexpr uint32_t kCbLdsMaxUsed = 4096;  // codebook tree kept in LDS up to this many used symbols
constexpr int kEncThreads = 256;
constexpr int kEncWaves = kEncThreads / 64;
constexpr int kEncMinR = 1;
constexpr int kEncMaxR = 6;
constexpr int kEncDefaultR = 4;
constexpr uint32_t kPackedMaxLen = 27;        // a left-aligned code plus 5 bits of 32 - cl fit 32 bits

// Slab partition shared by the histogram and the encoder: slab g of S
// covers blocks [g*nb/S, (g+1)*nb/S) of kSlabBlock symbols, nb = ceil(n / kSlabBlock).
constexpr uint64_t kSlabBlock = 4096;
constexpr uint32_t kSlabHistMaxAlphabet = 4096;  // per-slab counts kept up to this alphabet
constexpr uint32_t kMaxSlabs = 16384;  // each encoder workgroup sums all earlier slab totals
constexpr uint32_t kMaxInternalSlabs = 2048;  // per-slab counts the histogram keeps in the workspace

__host__ __device__ inline uint64_t slab_begin(uint64_t g, uint64_t nblocks, uint64_t nslabs, uint64_t n) {
  const uint64_t s = (g * nblocks / nslabs) * kSlabBlock;
  return s < n ? s : n;
}

// Records a pair of events around one stage's main kernel(s) when armed.
struct KernelTimer {
  hipEvent_t ev_before = nullptr;
  hipEvent_t ev_after = nullptr;
  void before(hipStream_t s) const {
    if (ev_before) (void)hipEventRecord(ev_before, s);
  }
  void after(hipStream_t s) const {
    if (ev_after) (void)hipEventRecord(ev_after, s);
  }
};

// Takes the one-shot timer armed by hf_time_next_main_kernel on this host
// thread (empty if none).
KernelTimer take_main_timer();

hipError_t launch_fill_u32(uint32_t* p, uint64_t count, uint32_t value, hipStream_t stream);
hipError_t launch_fill_u64(uint64_t* p, uint64_t count, uint64_t value, hipStream_t stream);

// Workgroups (= slabs) the histogram uses when the caller wants no per-slab
// counts; the counts then go to the workspace (0 = large alphabet, atomics).
uint32_t histogram_internal_slabs(uint64_t n, uint32_t alphabet, int num_cus);

hipError_t launch_histogram(const void* sym, uint64_t n, uint32_t sym_bytes, uint32_t alphabet,
                            uint32_t* hist, uint32_t nslabs, uint32_t* slab_hist, uint32_t* ws,
                            size_t ws_bytes, uint32_t* status, int num_cus, hipStream_t stream,
                            const KernelTimer& timer);

// hist[b] += sum over slabs of slab_hist[g * A + b] (hist zeroed beforehand).
hipError_t launch_slab_hist_reduce(const uint32_t* slab_hist, uint32_t nslabs, uint32_t A, uint32_t* hist,
                                   hipStream_t stream);

// Fused prequantization + 3D Lorenzo residual + histogram of a float field
// (nz, ny, nx) in C order; with slab_hist also the per-slab counts.
size_t lorenzo_lds_bytes(uint32_t ny, uint32_t nx, uint32_t radius);
hipError_t launch_lorenzo_histogram(const float* x, uint32_t nz, uint32_t ny, uint32_t nx, float r, uint32_t radius,
                                    uint16_t* codes, uint32_t* hist, uint32_t nslabs, uint32_t* slab_hist,
                                    uint32_t* status, int num_cus, hipStream_t stream, const KernelTimer& timer);

// The paper's own format (ReduceShuffleMerge<M, r> words, breaking groups
// in a side channel, word-aligned chunks): workspace and launch.
size_t paper_workspace_bytes(uint64_t n, uint32_t chunk_log2);
hipError_t launch_encode_paper(const void* sym, uint64_t n, uint32_t sym_bytes, const hf_codebook& book,
                               uint32_t M, uint32_t r, uint32_t* out, uint64_t cap_words, uint64_t* offsets,
                               uint64_t* brk_groups, void* brk_syms, uint64_t brk_cap, uint64_t* nbreak, void* ws,
                               uint32_t* status, uint32_t cus, hipStream_t stream, const KernelTimer& timer);

// Workspace bytes the codebook kernel needs when more than kCbLdsMaxUsed
// symbols are used.
size_t codebook_workspace_bytes(uint32_t alphabet, uint32_t tree_cap = kCbLdsMaxUsed);

// stamps: null, or 9 device words for the single-workgroup build's phase
// clocks (hf_build_codebook_traced)
hipError_t launch_codebook(const uint32_t* hist, const hf_codebook& book, void* ws, size_t ws_bytes,
                           uint32_t* status, hipStream_t stream, const KernelTimer& timer,
                           uint64_t* stamps = nullptr);

// Encoder workspace: per-slab bit totals and last-32-bit records.
size_t encode_workspace_bytes(uint32_t nslabs, uint32_t alphabet);

// Resident workgroups per CU of the default encoder for this alphabet.
int encode_blocks_per_cu(uint32_t alphabet, uint32_t sym_bytes);

hipError_t launch_encode(const void* sym, uint64_t n, uint32_t sym_bytes, const hf_codebook& book,
                         uint32_t chunk_log2, uint32_t r, uint32_t nslabs, const uint32_t* slab_hist,
                         uint32_t* out, uint64_t cap_words, uint64_t* offsets, void* ws,
                         uint32_t* status, hipStream_t stream, const KernelTimer& timer);

// One stream of a batched encode, as the batch kernels see it.  Slabs of a
// stream follow the same block partition as the single-stream path.
struct BatchStream {
  const void* sym;
  uint64_t n;
  uint64_t nblocks;
  uint32_t sym_bytes;
  uint32_t A;
  uint32_t nslabs;
  uint32_t item0;       // first (stream, slab) work item of this stream
  uint32_t r;           // reduce_log2 used for this stream
  uint32_t chunk_log2;
  uint64_t nchunks;
  uint32_t* part;       // [nslabs * A] per-slab counts
  uint32_t* hist;       // [A]
  hf_codebook book;
  char* cb_ws;          // codebook tree when more than kCbLdsMaxUsed symbols are used
  uint64_t* slab_bits;  // [nslabs] content bits of each slab
  uint32_t* slab_tail;  // [nslabs] last 32 content bits of each slab
  uint32_t* out;
  uint64_t cap_words;
  uint64_t* offsets;
  uint32_t* status;
};

// Arguments of the persistent batched launch (every stage in one kernel).
struct FusedArgs {
  const BatchStream* streams;
  const uint32_t* item_stream;  // [nitems] stream of every (stream, slab) item
  const uint32_t* hist_items;   // [nitems] queue order of the slab histograms
  const uint32_t* red_items;    // [nred] stream << 6 | bin chunk
  const uint32_t* enc_items;    // [nitems] queue order of the slab encodings
  uint32_t nitems, nred, nstreams;
  uint32_t lds_words;  // dynamic LDS words (the histogram's replicas)
  uint32_t* sync;      // [1 + 4 nstreams], zero: queue head, then per-stream counters
};
// Codebook tree kept in LDS up to this many used symbols in the persistent
// launch (beyond it, the stream's cb_ws).
constexpr uint32_t kFusedTreeCap = 1024;
// Dynamic LDS of the persistent launch: the largest need of any stage of any
// stream (host array of the streams' descriptors).
size_t batch_persistent_lds_bytes(const BatchStream* streams, uint32_t nstreams);
hipError_t launch_batch_persistent(const FusedArgs& f, size_t lds_bytes, int num_cus, hipStream_t stream);

// Histogram LDS words for a batch group whose alphabets are at most A.
uint32_t batch_hist_lds_words(uint32_t max_alphabet);
hipError_t launch_batch_histogram(const BatchStream* d_streams, const uint32_t* d_item_stream,
                                  const uint32_t* d_items, uint32_t nitems, uint32_t lds_words,
                                  hipStream_t stream);
// Bins one workgroup of the batched histogram reduction sums (alphabets up
// to 8192 give at most 32 chunks, encoded in 6 bits of a reduce item).
constexpr uint32_t kBatchReduceBins = 256;
hipError_t launch_batch_hist_reduce(const BatchStream* d_streams, const uint32_t* d_red_items, uint32_t nred,
                                    hipStream_t stream);
hipError_t launch_batch_codebook(const BatchStream* d_streams, uint32_t nstreams, hipStream_t stream);
hipError_t launch_batch_slab_bits(const BatchStream* d_streams, const uint32_t* d_item_stream, uint32_t nitems,
                                  hipStream_t stream);
// r in {3, 4, 5} (others run as 4); every item's alphabet is at most max_alphabet.
hipError_t launch_batch_encode(const BatchStream* d_streams, const uint32_t* d_item_stream,
                               const uint32_t* d_items, uint32_t nitems, uint32_t r, uint32_t max_alphabet,
                               hipStream_t stream);

// Decoder workspace: the prefix table.
size_t decode_workspace_bytes();

hipError_t launch_decode(const uint32_t* words, const uint64_t* offsets, uint64_t n, uint32_t sym_bytes,
                         uint32_t chunk_log2, const hf_codebook& book, void* out, void* ws, uint32_t* status,
                         int num_cus, hipStream_t stream, const KernelTimer& timer);

hipError_t launch_decode_check(const uint32_t* words, const uint64_t* offsets, uint64_t n,
                               uint32_t sym_bytes, uint32_t chunk_log2, const hf_codebook& book,
                               const void* expected, uint64_t* result, uint32_t* status,
                               hipStream_t stream);

}  // namespace hf
