// Runs the library's host-side builders and encoder (host_tables.cpp) over
// seeded random strips, built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_sanitizers.py; buffers are sized
// exactly as include/fptc.h states, and bad arguments must be refused.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "fptc.h"

static int fail(int code) {
  std::printf("failed %d\n", code);
  return code;
}

int main() {
  std::mt19937_64 rng(2605010861ull);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  static const int Ns[] = {4, 16, 32, 64, 256};
  for (int trial = 0; trial < 30; ++trial) {
    const int N = Ns[trial % 5];
    int E = N - (trial % 3) * (N / 4);
    if (E < 1) E = 1;
    fptc_quant_params q{};
    q.kind = (trial & 1) ? FPTC_QUANT_PAPER : FPTC_QUANT_AMPLITUDE;
    q.N = N;
    q.E = E;
    q.step_fine = 0.25, q.step_coarse = 2.0, q.threshold = 16.0;
    q.B1 = E < 2 ? E : 2;
    q.B2 = q.B1 + (E - q.B1) / 2;
    q.mu = 50.0, q.alpha1 = 0.004, q.A0 = 30.0, q.A1 = 20.0;
    // tables
    std::vector<float> basis((size_t)E * N);
    std::vector<double> table((size_t)E * (N + 1));
    if (fptc_build_basis(N, E, basis.data()) || fptc_build_dct_table(N, E, table.data())) return fail(1);
    std::vector<float> val(4 * 256);
    std::vector<uint8_t> zone(4 * 256), rob((size_t)E);
    int32_t rows = 0;
    if (fptc_build_dequant(&q, val.data(), zone.data(), rob.data(), &rows) || rows < 1 || rows > 4) return fail(2);
    // a batch of strips, one codebook trained on them
    const int n_streams = 1 + (int)(U(rng) * 6);
    std::vector<int64_t> so(n_streams + 1, 0);
    for (int s = 0; s < n_streams; ++s) so[s + 1] = so[s] + (int64_t)(U(rng) * (4 * N + 9));
    std::vector<float> x((size_t)so[n_streams]);
    for (auto &v : x) v = (float)(20.0 * (U(rng) - 0.5) * (U(rng) < 0.2 ? 10.0 : 1.0));
    std::vector<uint64_t> hist(256, 1);
    for (int s = 0; s < n_streams; ++s) {
      const int64_t L = so[s + 1] - so[s];
      // an empty strip writes nothing, but the output pointer must be valid
      std::vector<uint8_t> sym((size_t)((L + N - 1) / N * E) + 1);
      if (fptc_quantize_host(x.data() + so[s], L, &q, sym.data())) return fail(3);
      sym.pop_back();
      for (uint8_t v : sym) hist[v] += 1;
    }
    const int lmax = (trial & 2) ? 16 : 12;
    std::vector<uint8_t> len(256);
    std::vector<uint32_t> codes(256);
    if (fptc_code_lengths(hist.data(), lmax, len.data()) || fptc_canonical_codes(len.data(), codes.data())) return fail(4);
    if (lmax <= 12) {
      std::vector<uint16_t> lut((size_t)1 << lmax);
      if (fptc_build_lut(len.data(), lmax, lut.data())) return fail(5);
    }
    // encode each strip alone, then the batch on several threads, and compare
    std::vector<int64_t> cap_off(n_streams + 1, 0);
    for (int s = 0; s < n_streams; ++s) {
      const int64_t L = so[s + 1] - so[s];
      cap_off[s + 1] = cap_off[s] + (L + N - 1) / N * E + 1;
    }
    std::vector<uint64_t> words((size_t)cap_off[n_streams]);
    std::vector<uint8_t> symlen((size_t)cap_off[n_streams]);
    std::vector<int64_t> used(n_streams);
    std::vector<uint8_t> book((size_t)n_streams, 0);
    if (fptc_encode_batch_host(x.data(), so.data(), n_streams, book.data(), &q, len.data(), cap_off.data(),
                               words.data(), symlen.data(), used.data(), 4))
      return fail(6);
    for (int s = 0; s < n_streams; ++s) {
      const int64_t L = so[s + 1] - so[s], n = (L + N - 1) / N * E;
      std::vector<uint8_t> sym((size_t)n + 1);
      if (fptc_quantize_host(x.data() + so[s], L, &q, sym.data())) return fail(7);
      sym.pop_back();
      const int64_t cap = n + 1;
      std::vector<uint64_t> w((size_t)cap);
      std::vector<uint8_t> sl((size_t)cap);
      int64_t nw = -1;
      if (fptc_symlen_pack_host(sym.data(), n, len.data(), w.data(), sl.data(), cap, &nw)) return fail(8);
      if (nw != used[s] || std::memcmp(w.data(), words.data() + cap_off[s], (size_t)nw * 8) ||
          std::memcmp(sl.data(), symlen.data() + cap_off[s], (size_t)nw))
        return fail(9);
    }
  }
  // refusals: bad arguments return an error and touch nothing
  uint8_t len[256] = {0};
  uint16_t lut[16];
  fptc_quant_params bad{};
  bad.N = 3;
  if (fptc_build_lut(len, 0, lut) == 0 || fptc_build_basis(3, 1, nullptr) == 0) return fail(10);
  float v[1024];
  uint8_t z[1024], r[4];
  int32_t rows;
  if (fptc_build_dequant(&bad, v, z, r, &rows) == 0) return fail(11);
  std::printf("ok\n");
  return 0;
}
