// Sanitizer driver (built by tests/test_sanitizers.py with
// -fsanitize=address,undefined): runs every routine of the serial oracle and
// of the multi-core CPU baseline on seeded streams -- empty, one symbol,
// ragged sizes, both symbol widths, long codes, error paths -- and checks
// that encode -> decode gives the input back and that the two agree.
// Exits non-zero on any disagreement; the sanitizers abort on any memory or
// undefined-behaviour error.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "hf_cpu.h"

extern "C" {
int oracle_histogram(const void* x, uint64_t n, int sym_bytes, uint32_t alphabet, uint32_t* h);
int oracle_codebook(const uint32_t* h, uint32_t alphabet, uint8_t* cl, uint64_t* cw, uint64_t* first,
                    uint32_t* entry, uint32_t* rev, uint64_t* info);
int oracle_encode(const void* x, uint64_t n, int sym_bytes, uint32_t alphabet, const uint8_t* cl,
                  const uint64_t* cw, uint64_t chunk, uint32_t* out, uint64_t cap_words, uint64_t* offsets,
                  uint64_t* total_bits);
int oracle_decode(const uint32_t* in, uint64_t start, uint64_t nbits, uint64_t n, const uint64_t* first,
                  const uint32_t* entry, const uint32_t* rev, uint32_t m, uint32_t lmax, int sym_bytes,
                  void* x_out, uint64_t* end_bit);
}

static uint64_t g_state = 0x9E3779B97F4A7C15ull;
static uint64_t next_rand() {  // splitmix64
  uint64_t z = (g_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static int fail(const char* what, int i) {
  std::printf("FAIL %s (case %d)\n", what, i);
  return 1;
}

template <typename S>
static int run_case(int id, uint64_t n, uint32_t A, int shape, uint32_t chunk) {
  const int sb = (int)sizeof(S);
  std::vector<S> x(n);
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t r = next_rand();
    uint32_t s;
    if (shape == 0) s = (uint32_t)(r % A);                              // flat
    else if (shape == 1) s = (uint32_t)(__builtin_ctzll(r | (1ull << 40)) % A);  // geometric: long codes
    else s = (uint32_t)((A / 2 + (r % 7) - 3) % A);                     // peaked
    x[i] = (S)s;
  }
  std::vector<uint32_t> h(A), h2(A);
  if (oracle_histogram(x.data(), n, sb, A, h.data())) return fail("oracle_histogram", id);
  if (hfc_histogram(x.data(), n, sb, A, h2.data(), 3)) return fail("hfc_histogram", id);
  if (h != h2) return fail("histograms differ", id);
  std::vector<uint8_t> cl(A), cl2(A);
  std::vector<uint64_t> cw(A), cw2(A), first(65), first2(65), info(4), info2(4);
  std::vector<uint32_t> entry(65), entry2(65), rev(A, 0xFFFFFFFFu), rev2(A, 0xFFFFFFFFu);
  if (oracle_codebook(h.data(), A, cl.data(), cw.data(), first.data(), entry.data(), rev.data(), info.data()))
    return fail("oracle_codebook", id);
  if (hfc_codebook(h.data(), A, cl2.data(), cw2.data(), first2.data(), entry2.data(), rev2.data(), info2.data(), 3))
    return fail("hfc_codebook", id);
  if (cl != cl2 || cw != cw2 || first != first2 || entry != entry2 || info != info2) return fail("books differ", id);
  if (std::memcmp(rev.data(), rev2.data(), 4 * info[0]) != 0) return fail("rev differs", id);
  const uint64_t total = info[2], words = (total + 31) / 32, nch = (n + chunk - 1) / chunk;
  std::vector<uint32_t> out(words + 1, 0), out2(words + 1, 0);
  std::vector<uint64_t> offs(nch + 1), offs2(nch + 1);
  uint64_t tb = 0;
  if (oracle_encode(x.data(), n, sb, A, cl.data(), cw.data(), chunk, out.data(), words + 1, offs.data(), &tb))
    return fail("oracle_encode", id);
  if (tb != total) return fail("total bits", id);
  if (hfc_encode(x.data(), n, sb, A, cl.data(), cw.data(), chunk, out2.data(), words + 1, offs2.data(), 3))
    return fail("hfc_encode", id);
  if (std::memcmp(out.data(), out2.data(), 4 * words) != 0 || offs != offs2) return fail("streams differ", id);
  if (n > 0) {
    std::vector<S> y(n);
    uint64_t end = 0;
    if (oracle_decode(out.data(), 0, total, n, first.data(), entry.data(), rev.data(), (uint32_t)info[0],
                      (uint32_t)info[1], sb, y.data(), &end))
      return fail("oracle_decode", id);
    if (y != x || end != total) return fail("round trip", id);
    // error paths: too little room, a symbol without a code
    if (words > 1 && hfc_encode(x.data(), n, sb, A, cl.data(), cw.data(), chunk, out2.data(), words - 1,
                                offs2.data(), 2) != 17)
      return fail("capacity error", id);
    if (words > 1 && oracle_encode(x.data(), n, sb, A, cl.data(), cw.data(), chunk, out.data(), words - 1,
                                   offs.data(), &tb) != 17)
      return fail("oracle capacity error", id);
  }
  return 0;
}

int main() {
  int bad = 0, id = 0;
  const uint64_t sizes[] = {0, 1, 2, 255, 4097, 100003};
  const uint32_t chunks[] = {256, 4096, 65536};
  for (uint64_t n : sizes)
    for (int shape = 0; shape < 3; ++shape) {
      bad |= run_case<uint16_t>(id++, n, 1024, shape, chunks[id % 3]);
      bad |= run_case<uint8_t>(id++, n, 256, shape, chunks[id % 3]);
      bad |= run_case<uint16_t>(id++, n, 65536, shape, chunks[id % 3]);
      bad |= run_case<uint8_t>(id++, n, 1, shape, chunks[id % 3]);
    }
  // a symbol outside the alphabet
  std::vector<uint16_t> x = {1, 2, 3, 900};
  std::vector<uint32_t> h(16);
  if (oracle_histogram(x.data(), x.size(), 2, 16, h.data()) != 16) bad |= fail("oracle symbol error", -1);
  if (hfc_histogram(x.data(), x.size(), 2, 16, h.data(), 2) != 16) bad |= fail("hfc symbol error", -1);
  std::printf(bad ? "sanitized run found errors\n" : "sanitized run clean: %d cases\n", id);
  return bad;
}
