// Sanitizer driver for libhf's host side (built by
// tests/test_sanitizers.py from every csrc/*.hip with the host pass under
// -fsanitize=address,undefined; no GPU is used): sizing functions, the
// reduction-factor rule, status strings, the batch planner over many seeded
// descriptor sets, and every entry point's argument checks with arguments
// they must refuse before any device work.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "hf.h"

static uint64_t g_state = 12345;
static uint64_t next_rand() {  // splitmix64
  uint64_t z = (g_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

#define EXPECT(c)                                              \
  do {                                                         \
    if (!(c)) {                                                \
      std::printf("FAIL line %d: %s\n", __LINE__, #c);         \
      return 1;                                                \
    }                                                          \
  } while (0)

int main() {
  // sizing and rules
  for (uint64_t n : {0ull, 1ull, 4095ull, 4096ull, 1000003ull, 134217728ull, 4294967295ull})
    for (uint32_t A : {1u, 2u, 255u, 256u, 1024u, 4096u, 8192u, 65536u}) {
      EXPECT(hf_workspace_bytes(n, A, 4096) >= 256);
      EXPECT(hf_bound_words(n, A) >= n / 32);
      (void)hf_slab_count(n, A);
    }
  for (double b : {-1.0, 0.0, 0.5, 1.0, 1.0272, 2.7307, 5.1639, 31.9, 64.0, 1e300, (double)NAN, (double)INFINITY})
    EXPECT(hf_reduction_factor(b) >= 1 && hf_reduction_factor(b) <= 6);
  for (uint32_t c = 0; c < 64; ++c) EXPECT(hf_status_string(c) != nullptr);
  EXPECT(hf_paper_workspace_bytes(1000000, 7) == 0 && hf_paper_workspace_bytes(1000000, 10) > 0);
  EXPECT(hf_decode_workspace_bytes() > 0);

  // the batch planner over seeded descriptor sets (fake device addresses:
  // sizing never dereferences them)
  hf_codebook book{};
  book.cl = (uint8_t*)0x4000;
  book.cw = (uint64_t*)0x4000;
  book.first = (uint64_t*)0x4000;
  book.entry = (uint32_t*)0x4000;
  book.rev = (uint32_t*)0x4000;
  book.info = (uint64_t*)0x4000;
  const uint32_t alphas[] = {1, 256, 1024, 4096, 8192, 8193};
  for (int trial = 0; trial < 200; ++trial) {
    const uint32_t ns = 1 + (uint32_t)(next_rand() % 600);
    std::vector<hf_stream_desc> d(ns);
    bool valid = true;
    for (uint32_t s = 0; s < ns; ++s) {
      hf_stream_desc& e = d[s];
      e.sym = (const void*)0x100000;
      e.n = next_rand() % (trial % 3 == 0 ? 70000000ull : 5000000ull);
      e.sym_bytes = 1 + (uint32_t)(next_rand() % 2);
      e.chunk_symbols = 1u << (8 + next_rand() % 9);
      e.reduce_log2 = (uint32_t)(next_rand() % 4) == 0 ? 0u : 3u + (uint32_t)(next_rand() % 3);
      e.reserved = 0;
      e.hist = nullptr;
      e.book = book;
      e.book.alphabet = alphas[next_rand() % (trial % 5 == 0 ? 6 : 5)];
      if (e.sym_bytes == 1 && e.book.alphabet > 256) e.book.alphabet = 256;
      e.out = (uint32_t*)0x200000;
      e.out_capacity_words = e.n;
      e.chunk_bit_offsets = (uint64_t*)0x300000;
      valid &= e.book.alphabet <= 8192;
    }
    const size_t need = hf_batch_workspace_bytes(d.data(), ns);
    EXPECT(valid ? need >= 256 : need == 0);
    if (!valid) EXPECT(hf_encode_batch(d.data(), ns, (void*)0x1000, need, (uint32_t*)0x5000, nullptr) == HF_ERR_ARG);
  }

  // argument checks: every call below must be refused before device work
  uint32_t* st = (uint32_t*)0x5000;
  void* p = (void*)0x10000;
  hf_codebook b = book;
  b.alphabet = 1024;
  EXPECT(hf_histogram(p, 100, 3, 1024, (uint32_t*)p, 0, nullptr, nullptr, 0, st, nullptr) == HF_ERR_ARG);
  EXPECT(hf_histogram(p, 100, 1, 1024, (uint32_t*)p, 0, nullptr, nullptr, 0, st, nullptr) == HF_ERR_ARG);
  EXPECT(hf_histogram(p, 100, 2, 1024, (uint32_t*)p, 0, nullptr, nullptr, 0, nullptr, nullptr) == HF_ERR_ARG);
  EXPECT(hf_histogram(p, 100, 2, 1024, (uint32_t*)p, 5, (uint32_t*)p, nullptr, 0, st, nullptr) == HF_ERR_ARG);
  EXPECT(hf_build_codebook(nullptr, &b, nullptr, 0, st, nullptr) == HF_ERR_ARG);
  hf_codebook big = b;
  big.alphabet = 65536;
  EXPECT(hf_build_codebook((uint32_t*)p, &big, nullptr, 0, st, nullptr) == HF_ERR_WORKSPACE);
  EXPECT(hf_encode(p, 100, 2, &b, 3000, 0, 0, nullptr, (uint32_t*)p, 10, (uint64_t*)p, p, 1 << 20, st, nullptr) ==
         HF_ERR_ARG);
  EXPECT(hf_encode(p, 100, 2, &b, 4096, 7, 0, nullptr, (uint32_t*)p, 10, (uint64_t*)p, p, 1 << 20, st, nullptr) ==
         HF_ERR_ARG);
  EXPECT(hf_encode(p, 100000, 2, &b, 4096, 0, 0, nullptr, (uint32_t*)p, 10, (uint64_t*)p, nullptr, 0, st,
                   nullptr) == HF_ERR_WORKSPACE);
  EXPECT(hf_decode((uint32_t*)p, (uint64_t*)p, 100, 2, 100, &b, p, p, 1 << 20, st, nullptr) == HF_ERR_ARG);
  EXPECT(hf_lorenzo_histogram((float*)p, 4, 4, 4, 1.0f, 0, (uint16_t*)p, (uint32_t*)p, 0, nullptr, st, nullptr) ==
         HF_ERR_ARG);
  EXPECT(hf_lorenzo_histogram((float*)p, 4, 4, 4, NAN, 8, (uint16_t*)p, (uint32_t*)p, 0, nullptr, st, nullptr) ==
         HF_ERR_ARG);
  EXPECT(hf_encode_paper(p, 100, 2, &b, 13, 3, (uint32_t*)p, 10, (uint64_t*)p, nullptr, nullptr, 0, (uint64_t*)p, p,
                         1 << 20, st, nullptr) == HF_ERR_ARG);
  std::printf("sanitized host run clean\n");
  return 0;
}
