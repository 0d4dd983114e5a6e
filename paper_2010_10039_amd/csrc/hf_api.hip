// hf_api.hip -- the extern "C" entry points of libhf: argument checks,
// workspace sizing and kernel launches on the caller's stream.
#include <math.h>

#include <algorithm>
#include <mutex>

#include "hf_kernels.h"

namespace {

using hf::KernelTimer;

thread_local KernelTimer t_timer;

KernelTimer take_timer() { return hf::take_main_timer(); }

int num_cus() {
  static std::mutex mu;
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  std::lock_guard<std::mutex> lock(mu);
  if (cache[dev] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
    cache[dev] = v;
  }
  return cache[dev];
}

bool is_pow2(uint64_t x) { return x && !(x & (x - 1)); }

uint32_t log2u(uint64_t x) {
  uint32_t l = 0;
  while ((1ull << l) < x) ++l;
  return l;
}

bool valid_symbols(uint32_t sym_bytes, uint32_t alphabet, uint64_t n) {
  if (sym_bytes != 1 && sym_bytes != 2) return false;
  if (alphabet == 0 || alphabet > 65536u) return false;
  if (sym_bytes == 1 && alphabet > 256u) return false;
  if (n >= (1ull << 32)) return false;
  return true;
}

bool valid_book(const hf_codebook* b) {
  return b && b->alphabet >= 1 && b->alphabet <= 65536u && b->cl && b->cw && b->first && b->entry &&
         b->rev && b->info;
}

bool valid_chunk(uint32_t chunk) { return is_pow2(chunk) && chunk >= 256u && chunk <= 65536u; }

uint32_t effective_r(uint32_t r) { return r == 0 ? (uint32_t)hf::kEncDefaultR : r; }

hf_status launch_result(hipError_t e) { return e == hipSuccess ? HF_OK : HF_ERR_LAUNCH; }

uint64_t blocks_of(uint64_t n) { return (n + hf::kSlabBlock - 1) / hf::kSlabBlock; }

// One encoder workgroup per slab, as many slabs as workgroups fit at once
// but at most four per CU: on the 134 M-symbol Lorenzo stream four per CU
// made the histogram 8 us faster (less LDS atomic contention, fewer
// per-slab counts) and the step 180 us against 184 us at five.
uint32_t default_slabs(uint64_t n, uint32_t alphabet, uint32_t sym_bytes) {
  const uint64_t nb = blocks_of(n);
  const uint64_t per_cu = std::min<uint64_t>(4, (uint64_t)hf::encode_blocks_per_cu(alphabet, sym_bytes));
  const uint64_t cap = (uint64_t)num_cus() * per_cu;
  uint64_t s = nb < cap ? nb : cap;
  if (s > hf::kMaxSlabs) s = hf::kMaxSlabs;
  return (uint32_t)(s > 0 ? s : 1);
}

// Argument rules shared by hf_encode and hf_encode_noalloc; *nslabs = 0 is
// replaced by the default slab count.
hf_status check_encode_args(const void* d_sym, uint64_t n, uint32_t sym_bytes, const hf_codebook* book,
                            uint32_t chunk_symbols, uint32_t reduce_log2, uint32_t* nslabs,
                            const uint32_t* d_slab_hist, const uint32_t* d_out, const uint64_t* d_offsets,
                            const uint32_t* d_status) {
  if (!valid_book(book) || !valid_symbols(sym_bytes, book->alphabet, n) || !valid_chunk(chunk_symbols) ||
      !d_offsets || !d_status || (n > 0 && (!d_sym || !d_out)))
    return HF_ERR_ARG;
  if (((uintptr_t)d_sym % sym_bytes) != 0) return HF_ERR_ARG;
  if (reduce_log2 > (uint32_t)hf::kEncMaxR) return HF_ERR_ARG;
  if (*nslabs > blocks_of(n) || *nslabs > hf::kMaxSlabs) return HF_ERR_ARG;
  if (d_slab_hist && (*nslabs == 0 || book->alphabet > hf::kSlabHistMaxAlphabet)) return HF_ERR_ARG;
  if (n > 0 && *nslabs == 0) *nslabs = default_slabs(n, book->alphabet, sym_bytes);
  return HF_OK;
}

// The allocation-free encoder's workspace: a fixed array in device memory,
// one copy per GPU, alive until the process ends.  Its name is a host-side
// stand-in; the device address of each GPU's copy is looked up once per
// device with hipGetSymbolAddress and used everywhere host code needs it.
__device__ __align__(256) unsigned char scratch[HF_NOALLOC_SCRATCH_BYTES];

void* device_scratch() {
  static std::mutex mu;
  static void* addr[64] = {nullptr};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  if (addr[dev] == nullptr) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return nullptr;
    addr[dev] = p;
  }
  return addr[dev];
}

}  // namespace

namespace hf {
KernelTimer take_main_timer() {
  KernelTimer t = t_timer;
  t_timer = KernelTimer{};
  return t;
}
}  // namespace hf

extern "C" {

size_t hf_workspace_bytes(uint64_t n, uint32_t alphabet, uint32_t chunk_symbols) {
  (void)chunk_symbols;
  const uint64_t nblocks = (n + hf::kSlabBlock - 1) / hf::kSlabBlock;
  const size_t enc = hf::encode_workspace_bytes((uint32_t)(nblocks > 0 ? nblocks : 1), alphabet);
  const size_t cb = hf::codebook_workspace_bytes(alphabet);
  const size_t hist = (size_t)hf::histogram_internal_slabs(n, alphabet, num_cus()) * alphabet * 4;
  size_t need = enc > cb ? enc : cb;
  if (hist > need) need = hist;
  return need < 256 ? 256 : need;
}

uint32_t hf_slab_count(uint64_t n, uint32_t alphabet) {
  if (alphabet == 0 || alphabet > hf::kSlabHistMaxAlphabet || n == 0) return 0;
  return default_slabs(n, alphabet, 2);
}

uint64_t hf_bound_words(uint64_t n, uint32_t alphabet) {
  const uint64_t bits_per = (uint64_t)log2u(alphabet > 0 ? alphabet : 1) + 1;
  return (n * bits_per + 31) / 32 + 1;
}

uint32_t hf_reduction_factor(double beta) {
  if (!(beta >= 1.0)) beta = 1.0;   // also NaN
  if (beta > 64.0) beta = 64.0;      // codes are at most 64 bits (also +inf)
  const int fl = (int)floor(log2(beta));
  int r = 5 - fl - 1;  // floor(log2 beta) + r + 1 = log2(32) = 5
  if (r < hf::kEncMinR) r = hf::kEncMinR;
  if (r > hf::kEncMaxR) r = hf::kEncMaxR;
  return (uint32_t)r;
}

const char* hf_status_string(uint32_t code) {
  switch (code) {
    case HF_OK: return "ok";
    case HF_ERR_ARG: return "invalid argument";
    case HF_ERR_WORKSPACE: return "workspace missing or too small";
    case HF_ERR_LAUNCH: return "kernel launch failed";
    case HF_ERR_SYMBOL: return "symbol outside the alphabet or without a code";
    case HF_ERR_CAPACITY: return "output capacity exceeded";
    case HF_ERR_CODELEN: return "code length above 64 bits";
    case HF_ERR_MISMATCH: return "decoded stream differs from the input";
    case HF_ERR_INTERNAL: return "internal bound exceeded";
    case HF_ERR_STREAM: return "stream does not decode with the codebook";
    case HF_ERR_VALUE: return "a value of the field is NaN or infinite";
    default: return "unknown status";
  }
}

hf_status hf_time_next_main_kernel(void* before_event, void* after_event) {
  t_timer.ev_before = (hipEvent_t)before_event;
  t_timer.ev_after = (hipEvent_t)after_event;
  return HF_OK;
}

hf_status hf_histogram(const void* d_sym, uint64_t n, uint32_t sym_bytes, uint32_t alphabet,
                       uint32_t* d_hist, uint32_t nslabs, uint32_t* d_slab_hist, void* d_ws,
                       size_t ws_bytes, uint32_t* d_status, void* stream) {
  const KernelTimer timer = take_timer();
  if (!valid_symbols(sym_bytes, alphabet, n) || !d_hist || !d_status || (n > 0 && !d_sym))
    return HF_ERR_ARG;
  if (((uintptr_t)d_sym % sym_bytes) != 0) return HF_ERR_ARG;
  if (d_slab_hist && (nslabs == 0 || nslabs > blocks_of(n) || nslabs > hf::kMaxSlabs ||
                      alphabet > hf::kSlabHistMaxAlphabet))
    return HF_ERR_ARG;
  if (d_ws && ((uintptr_t)d_ws & 255)) return HF_ERR_WORKSPACE;
  return launch_result(hf::launch_histogram(d_sym, n, sym_bytes, alphabet, d_hist, nslabs, d_slab_hist,
                                            (uint32_t*)d_ws, d_ws ? ws_bytes : 0, d_status, num_cus(),
                                            (hipStream_t)stream, timer));
}

hf_status hf_lorenzo_histogram(const float* d_field, uint32_t nz, uint32_t ny, uint32_t nx, float inv_2eb,
                               uint32_t radius, uint16_t* d_codes, uint32_t* d_hist, uint32_t nslabs,
                               uint32_t* d_slab_hist, uint32_t* d_status, void* stream) {
  const KernelTimer timer = take_timer();
  const uint64_t n = (uint64_t)nz * ny * nx;
  if (radius == 0 || radius > 8192u || !d_hist || !d_status || !isfinite(inv_2eb) || !(inv_2eb > 0.0f))
    return HF_ERR_ARG;
  if (n >= (1ull << 32) || (ny > 1 && nx > 8192u)) return HF_ERR_ARG;
  if (n > 0 && (!d_field || !d_codes || ((uintptr_t)d_field & 3) || ((uintptr_t)d_codes & 1))) return HF_ERR_ARG;
  if (d_slab_hist && (nslabs == 0 || nslabs > blocks_of(n) || nslabs > hf::kMaxSlabs ||
                      2 * radius > hf::kSlabHistMaxAlphabet))
    return HF_ERR_ARG;
  return launch_result(hf::launch_lorenzo_histogram(d_field, nz, ny, nx, inv_2eb, radius, d_codes, d_hist,
                                                    nslabs, d_slab_hist, d_status, num_cus(), (hipStream_t)stream,
                                                    timer));
}

hf_status hf_build_codebook(const uint32_t* d_hist, const hf_codebook* book, void* d_ws,
                            size_t ws_bytes, uint32_t* d_status, void* stream) {
  const KernelTimer timer = take_timer();
  if (!d_hist || !valid_book(book) || !d_status) return HF_ERR_ARG;
  const size_t need = hf::codebook_workspace_bytes(book->alphabet);
  if (need > 0 && (!d_ws || ws_bytes < need || ((uintptr_t)d_ws & 255))) return HF_ERR_WORKSPACE;
  return launch_result(hf::launch_codebook(d_hist, *book, d_ws, ws_bytes, d_status, (hipStream_t)stream, timer));
}

hf_status hf_build_codebook_traced(const uint32_t* d_hist, const hf_codebook* book, void* d_ws,
                                   size_t ws_bytes, uint32_t* d_status, uint64_t* d_stamps, void* stream) {
  const KernelTimer timer = take_timer();
  if (!d_hist || !valid_book(book) || !d_status || !d_stamps) return HF_ERR_ARG;
  const size_t need = hf::codebook_workspace_bytes(book->alphabet);
  if (need > 0 && (!d_ws || ws_bytes < need || ((uintptr_t)d_ws & 255))) return HF_ERR_WORKSPACE;
  return launch_result(
      hf::launch_codebook(d_hist, *book, d_ws, ws_bytes, d_status, (hipStream_t)stream, timer, d_stamps));
}

hf_status hf_encode(const void* d_sym, uint64_t n, uint32_t sym_bytes, const hf_codebook* book,
                    uint32_t chunk_symbols, uint32_t reduce_log2, uint32_t nslabs,
                    const uint32_t* d_slab_hist, uint32_t* d_out, uint64_t out_capacity_words,
                    uint64_t* d_chunk_bit_offsets, void* d_ws, size_t ws_bytes,
                    uint32_t* d_status, void* stream) {
  const KernelTimer timer = take_timer();
  const hf_status st = check_encode_args(d_sym, n, sym_bytes, book, chunk_symbols, reduce_log2, &nslabs,
                                         d_slab_hist, d_out, d_chunk_bit_offsets, d_status);
  if (st != HF_OK) return st;
  if (n > 0 && (!d_ws || ws_bytes < hf::encode_workspace_bytes(nslabs, book->alphabet) || ((uintptr_t)d_ws & 255)))
    return HF_ERR_WORKSPACE;
  return launch_result(hf::launch_encode(d_sym, n, sym_bytes, *book, log2u(chunk_symbols), effective_r(reduce_log2),
                                         nslabs, d_slab_hist, d_out, out_capacity_words, d_chunk_bit_offsets,
                                         d_ws, d_status, (hipStream_t)stream, timer));
}

hf_status hf_encode_noalloc(const void* d_sym, uint64_t n, uint32_t sym_bytes, const hf_codebook* book,
                            uint32_t chunk_symbols, uint32_t reduce_log2, uint32_t nslabs,
                            const uint32_t* d_slab_hist, uint32_t* d_out, uint64_t out_capacity_words,
                            uint64_t* d_chunk_bit_offsets, uint32_t* d_status, void* stream) {
  const KernelTimer timer = take_timer();
  const hf_status st = check_encode_args(d_sym, n, sym_bytes, book, chunk_symbols, reduce_log2, &nslabs,
                                         d_slab_hist, d_out, d_chunk_bit_offsets, d_status);
  if (st != HF_OK) return st;
  if (n > 0 && hf::encode_workspace_bytes(nslabs, book->alphabet) > HF_NOALLOC_SCRATCH_BYTES)
    return HF_ERR_WORKSPACE;
  void* ws = nullptr;
  if (n > 0 && (ws = device_scratch()) == nullptr) return HF_ERR_LAUNCH;
  return launch_result(hf::launch_encode(d_sym, n, sym_bytes, *book, log2u(chunk_symbols), effective_r(reduce_log2),
                                         nslabs, d_slab_hist, d_out, out_capacity_words, d_chunk_bit_offsets,
                                         ws, d_status, (hipStream_t)stream, timer));
}

size_t hf_paper_workspace_bytes(uint64_t n, uint32_t chunk_log2) {
  if (chunk_log2 < 8 || chunk_log2 > 12) return 0;
  return hf::paper_workspace_bytes(n, chunk_log2);
}

hf_status hf_encode_paper(const void* d_sym, uint64_t n, uint32_t sym_bytes, const hf_codebook* book,
                          uint32_t chunk_log2, uint32_t reduce_log2, uint32_t* d_out, uint64_t out_capacity_words,
                          uint64_t* d_chunk_word_offsets, uint64_t* d_break_groups, void* d_break_syms,
                          uint64_t break_capacity, uint64_t* d_nbreak, void* d_ws, size_t ws_bytes,
                          uint32_t* d_status, void* stream) {
  const KernelTimer timer = take_timer();
  if (!valid_book(book) || !valid_symbols(sym_bytes, book->alphabet, n) || !d_chunk_word_offsets || !d_nbreak ||
      !d_status || (n > 0 && (!d_sym || !d_out)))
    return HF_ERR_ARG;
  if (chunk_log2 < 8 || chunk_log2 > 12 || reduce_log2 < 1 || reduce_log2 > 5) return HF_ERR_ARG;
  if (((uintptr_t)d_sym % sym_bytes) != 0) return HF_ERR_ARG;
  if (break_capacity > 0 && (!d_break_groups || !d_break_syms)) return HF_ERR_ARG;
  if (n > 0 && (!d_ws || ws_bytes < hf::paper_workspace_bytes(n, chunk_log2) || ((uintptr_t)d_ws & 255)))
    return HF_ERR_WORKSPACE;
  return launch_result(hf::launch_encode_paper(d_sym, n, sym_bytes, *book, chunk_log2, reduce_log2, d_out,
                                               out_capacity_words, d_chunk_word_offsets, d_break_groups,
                                               d_break_syms, break_capacity, d_nbreak, d_ws, d_status,
                                               (uint32_t)num_cus(), (hipStream_t)stream, timer));
}

size_t hf_decode_workspace_bytes(void) { return hf::decode_workspace_bytes(); }

hf_status hf_decode(const uint32_t* d_in, const uint64_t* d_chunk_bit_offsets, uint64_t n, uint32_t sym_bytes,
                    uint32_t chunk_symbols, const hf_codebook* book, void* d_sym_out, void* d_ws,
                    size_t ws_bytes, uint32_t* d_status, void* stream) {
  if (!valid_book(book) || !valid_symbols(sym_bytes, book->alphabet, n) || !valid_chunk(chunk_symbols) ||
      !d_chunk_bit_offsets || !d_status || (n > 0 && (!d_in || !d_sym_out)))
    return HF_ERR_ARG;
  if (n > 0 && (!d_ws || ws_bytes < hf::decode_workspace_bytes() || ((uintptr_t)d_ws & 255)))
    return HF_ERR_WORKSPACE;
  return launch_result(hf::launch_decode(d_in, d_chunk_bit_offsets, n, sym_bytes, log2u(chunk_symbols), *book,
                                         d_sym_out, d_ws, d_status, num_cus(), (hipStream_t)stream,
                                         hf::take_main_timer()));
}

hf_status hf_decode_check(const uint32_t* d_out, const uint64_t* d_chunk_bit_offsets, uint64_t n,
                          uint32_t sym_bytes, uint32_t chunk_symbols, const hf_codebook* book,
                          const void* d_sym_expected, uint64_t* d_result, uint32_t* d_status,
                          void* stream) {
  if (!valid_book(book) || !valid_symbols(sym_bytes, book->alphabet, n) || !valid_chunk(chunk_symbols) ||
      !d_chunk_bit_offsets || !d_result || !d_status || (n > 0 && (!d_out || !d_sym_expected)))
    return HF_ERR_ARG;
  return launch_result(hf::launch_decode_check(d_out, d_chunk_bit_offsets, n, sym_bytes,
                                               log2u(chunk_symbols), *book, d_sym_expected, d_result,
                                               d_status, (hipStream_t)stream));
}

}  // extern "C"
