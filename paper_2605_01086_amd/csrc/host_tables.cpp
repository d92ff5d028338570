// Host-side codec structures and the host encoder.
//
// These build what the GPU decoder consumes (decode lookup tables, the IDCT
// basis, dequantization tables) and produce SymLen bitstreams from float32
// strips.  Section references are to the FPTC paper.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "fptc_internal.h"

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

bool valid_n(int32_t N) {
  return N == 4 || N == 8 || N == 16 || N == 32 || N == 64 || N == 128 || N == 256;
}

// ---------------------------------------------------------------- quantizers
// Section 3.2.  Byte levels: 128 = zero, 129..255 positive, 0..127 negative.
// Rounding is floor(x + 1/2) (Eq. 3), applied to magnitudes.

struct Quant {
  const fptc_quant_params &q;
  long mT;  // AMPLITUDE: fine levels up to the threshold

  explicit Quant(const fptc_quant_params &qq) : q(qq), mT(0) {
    if (q.kind == FPTC_QUANT_AMPLITUDE) mT = std::lround(q.threshold / q.step_fine);
  }

  int zone_of_bin(int k) const { return k < q.B1 ? 0 : (k < q.B2 ? 1 : 2); }

  uint8_t quantize(double c, int k) const {
    if (q.kind == FPTC_QUANT_AMPLITUDE) {
      double a = std::fabs(c);
      long m = a <= q.threshold ? (long)std::floor(a / q.step_fine + 0.5)
                                : mT + (long)std::floor((a - q.threshold) / q.step_coarse + 0.5);
      if (c >= 0) return (uint8_t)(128 + std::min(m, 127L));
      return (uint8_t)(128 - std::min(m, 128L));
    }
    int z = zone_of_bin(k);
    if (z == 2) return 128;
    if (z == 0) {  // Eq. 2, |c| clipped to A0; levels as Eq. 3 with a zero deadzone
      if (c == 0.0) return 128;
      double a = std::min(std::fabs(c), q.A0);
      double u = std::log(1.0 + q.mu * a / q.A0) / std::log(1.0 + q.mu);
      if (c > 0) return (uint8_t)(129 + (long)std::floor(u * 126.0 + 0.5));
      return (uint8_t)(127 - (long)std::floor(u * 127.0 + 0.5));
    }
    double d1 = q.alpha1 * q.A1;  // Eq. 3, |c| clipped to A1
    double a = std::min(std::fabs(c), q.A1);
    if (c > d1) return (uint8_t)(129 + (long)std::floor((a - d1) / (q.A1 - d1) * 126.0 + 0.5));
    if (c < -d1) return (uint8_t)(127 - (long)std::floor((a - d1) / (q.A1 - d1) * 127.0 + 0.5));
    return 128;
  }

  // Value and zone of level s in table row r (rows: AMPLITUDE has one, PAPER
  // has one per frequency zone).
  double value(int s, int r) const {
    if (q.kind == FPTC_QUANT_AMPLITUDE) {
      long m = s >= 128 ? s - 128 : 128 - s;
      double mag = m <= mT ? m * q.step_fine : q.threshold + (double)(m - mT) * q.step_coarse;
      return s >= 128 ? mag : -mag;
    }
    if (r == 2 || s == 128) return 0.0;
    if (r == 0) {
      double u = s > 128 ? (s - 129) / 126.0 : (127 - s) / 127.0;
      double mag = q.A0 / q.mu * (std::pow(1.0 + q.mu, u) - 1.0);
      return s > 128 ? mag : -mag;
    }
    double d1 = q.alpha1 * q.A1;
    if (s > 128) return d1 + (s - 129) * (q.A1 - d1) / 126.0;
    return -(d1 + (127 - s) * (q.A1 - d1) / 127.0);
  }

  int zone(int s, int r) const {
    if (q.kind == FPTC_QUANT_AMPLITUDE) {
      long m = s >= 128 ? s - 128 : 128 - s;
      return m == 0 ? 0 : (m <= mT ? 1 : 2);
    }
    return r;
  }
};

int check_quant(const fptc_quant_params *q) {
  if (!q || !valid_n(q->N) || q->E < 1 || q->E > q->N) return FPTC_ERR_INVALID_ARG;
  if (q->kind == FPTC_QUANT_AMPLITUDE) {
    if (!(q->step_fine > 0) || !(q->step_coarse > 0) || !(q->threshold >= 0)) return FPTC_ERR_INVALID_ARG;
    double r = q->threshold / q->step_fine;
    if (std::fabs(r - std::round(r)) > 1e-9 || r > 127) return FPTC_ERR_INVALID_ARG;
    return FPTC_OK;
  }
  if (q->kind == FPTC_QUANT_PAPER) {
    if (q->B1 < 0 || q->B2 < q->B1 || q->B2 > q->E) return FPTC_ERR_INVALID_ARG;
    if (!(q->mu > 0) || !(q->A0 > 0) || !(q->A1 > 0) || !(q->alpha1 >= 0) || !(q->alpha1 < 1))
      return FPTC_ERR_INVALID_ARG;
    return FPTC_OK;
  }
  return FPTC_ERR_INVALID_ARG;
}

}  // namespace

int fptc::check_quant_params(const fptc_quant_params *q) { return check_quant(q); }

namespace {

// Orthonormal DCT-II basis in double: B[k][n] = a_k cos(pi/N (n + 1/2) k).
std::vector<double> basis64(int N, int E) {
  std::vector<double> B((size_t)E * N);
  for (int k = 0; k < E; ++k) {
    double a = k == 0 ? std::sqrt(1.0 / N) : std::sqrt(2.0 / N);
    for (int n = 0; n < N; ++n) B[(size_t)k * N + n] = a * std::cos(kPi / N * (n + 0.5) * k);
  }
  return B;
}

void quantize_strip(const float *x, int64_t L, const fptc_quant_params &q, const std::vector<double> &B,
                    uint8_t *out) {
  const int N = q.N, E = q.E;
  const int64_t nw = (L + N - 1) / N;
  Quant Q(q);
  std::vector<double> win(N);
  for (int64_t w = 0; w < nw; ++w) {
    for (int n = 0; n < N; ++n) {
      int64_t i = w * N + n;
      win[n] = i < L ? (double)x[i] : 0.0;
    }
    for (int k = 0; k < E; ++k) {
      const double *b = &B[(size_t)k * N];
      double s = 0.0;
      for (int n = 0; n < N; ++n) s += win[n] * b[n];
      out[w * E + k] = Q.quantize(s, k);
    }
  }
}

int canonical(const uint8_t *len, uint32_t *code) {
  int maxl = 0;
  for (int s = 0; s < 256; ++s) maxl = std::max(maxl, (int)len[s]);
  if (maxl > 32) return FPTC_ERR_INVALID_ARG;
  int count[33] = {0};
  for (int s = 0; s < 256; ++s)
    if (len[s]) count[len[s]]++;
  uint64_t next[34] = {0};
  uint64_t c = 0;
  for (int l = 1; l <= maxl; ++l) {
    c = (c + (uint64_t)count[l - 1]) << 1;
    if (l == 1) c = 0;
    next[l] = c;
  }
  // Kraft check: the last code of each length must fit in l bits.
  for (int l = 1; l <= maxl; ++l)
    if (count[l] && next[l] + (uint64_t)count[l] > (1ull << l)) return FPTC_ERR_INVALID_ARG;
  for (int s = 0; s < 256; ++s) code[s] = len[s] ? (uint32_t)next[len[s]]++ : 0u;
  return FPTC_OK;
}

int64_t pack(const uint8_t *sym, int64_t n, const uint8_t *len, const uint32_t *code, uint64_t *words,
             uint8_t *symlen, int64_t cap) {
  // Section 4.1, Algorithm 1: greedy, MSB-first, codewords never split.
  int64_t w = 0;
  uint64_t buf = 0;
  int bits = 0, cnt = 0;
  for (int64_t i = 0; i < n; ++i) {
    int l = len[sym[i]];
    if (l == 0) return -1;
    if (bits + l > 64) {
      if (w >= cap) return -1;
      words[w] = buf;
      symlen[w] = (uint8_t)cnt;
      ++w;
      buf = 0;
      bits = 0;
      cnt = 0;
    }
    buf |= (uint64_t)code[sym[i]] << (64 - bits - l);
    bits += l;
    ++cnt;
  }
  if (cnt > 0) {
    if (w >= cap) return -1;
    words[w] = buf;
    symlen[w] = (uint8_t)cnt;
    ++w;
  }
  return w;
}

}  // namespace

extern "C" {

int32_t fptc_abi_version(void) { return FPTC_ABI_VERSION; }

const char *fptc_status_string(int32_t st) {
  switch (st) {
    case FPTC_OK: return "ok";
    case FPTC_ERR_INVALID_ARG: return "invalid argument";
    case FPTC_ERR_UNSUPPORTED: return "unsupported request";
    case FPTC_ERR_WORKSPACE: return "workspace too small";
    case FPTC_ERR_HIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

int32_t fptc_canonical_codes(const uint8_t *code_len, uint32_t *codes_out) {
  if (!code_len || !codes_out) return FPTC_ERR_INVALID_ARG;
  return canonical(code_len, codes_out);
}

int32_t fptc_build_lut(const uint8_t *code_len, int32_t lmax, uint16_t *lut_out) {
  if (!code_len || !lut_out || lmax < 1 || lmax > fptc::kMaxLmax) return FPTC_ERR_INVALID_ARG;
  for (int s = 0; s < 256; ++s)
    if (code_len[s] > lmax) return FPTC_ERR_INVALID_ARG;
  uint32_t code[256];
  int rc = canonical(code_len, code);
  if (rc != FPTC_OK) return rc;
  const int size = 1 << lmax;
  std::fill(lut_out, lut_out + size, (uint16_t)0);
  for (int s = 0; s < 256; ++s) {
    int l = code_len[s];
    if (!l) continue;
    // every lmax-bit peek that starts with this code maps to (l, s)
    uint32_t first = code[s] << (lmax - l), span = 1u << (lmax - l);
    for (uint32_t p = 0; p < span; ++p) lut_out[first + p] = (uint16_t)((l << 8) | s);
  }
  return FPTC_OK;
}

int32_t fptc_code_lengths(const uint64_t *freq, int32_t lmax, uint8_t *len_out) {
  // Package-merge (Larmore-Hirschberg) over the symbols with nonzero count:
  // items carry the symbols they contain as a sorted list of leaves, so a
  // package is the union of two items; the 2(n-1) cheapest items of the
  // final level give the lengths.
  if (!freq || !len_out || lmax < 1 || lmax > 32) return FPTC_ERR_INVALID_ARG;
  std::vector<int> used;
  for (int s = 0; s < 256; ++s) {
    len_out[s] = 0;
    if (freq[s]) used.push_back(s);
  }
  const int n = (int)used.size();
  if (n == 0) return FPTC_OK;
  if (n == 1) {
    len_out[used[0]] = 1;
    return FPTC_OK;
  }
  if (lmax < 31 && (1 << lmax) < n) return FPTC_ERR_INVALID_ARG;
  std::stable_sort(used.begin(), used.end(), [&](int a, int b) { return freq[a] < freq[b]; });
  struct Item {
    unsigned long long w;
    std::vector<uint16_t> cnt;  // per sorted-leaf count
  };
  std::vector<Item> leaves(n), cur;
  for (int i = 0; i < n; ++i) {
    leaves[i].w = freq[used[i]];
    leaves[i].cnt.assign(n, 0);
    leaves[i].cnt[i] = 1;
  }
  cur = leaves;
  for (int r = 1; r < lmax; ++r) {
    std::vector<Item> pk;
    for (size_t i = 0; i + 1 < cur.size(); i += 2) {
      Item it;
      it.w = cur[i].w + cur[i + 1].w;
      it.cnt.resize(n);
      for (int j = 0; j < n; ++j) it.cnt[j] = (uint16_t)(cur[i].cnt[j] + cur[i + 1].cnt[j]);
      pk.push_back(std::move(it));
    }
    std::vector<Item> merged;
    merged.reserve(leaves.size() + pk.size());
    size_t a = 0, b = 0;
    while (a < leaves.size() || b < pk.size()) {
      if (b >= pk.size() || (a < leaves.size() && leaves[a].w <= pk[b].w)) merged.push_back(leaves[a++]);
      else merged.push_back(std::move(pk[b++]));
    }
    if ((int)merged.size() > 2 * n) merged.resize(2 * n);
    cur.swap(merged);
  }
  if ((int)cur.size() < 2 * n - 2) return FPTC_ERR_INVALID_ARG;
  std::vector<int> tot(n, 0);
  for (int i = 0; i < 2 * n - 2; ++i)
    for (int j = 0; j < n; ++j) tot[j] += cur[i].cnt[j];
  for (int j = 0; j < n; ++j) len_out[used[j]] = (uint8_t)tot[j];
  return FPTC_OK;
}

int32_t fptc_build_dct_table(int32_t N, int32_t E, double *table_out) {
  if (!table_out || !valid_n(N) || E < 1 || E > N) return FPTC_ERR_INVALID_ARG;
  for (int k = 0; k < E; ++k) {
    double *row = table_out + (size_t)k * (N + 1);
    for (int n = 0; n < N; ++n) row[n] = std::cos(kPi / N * (n + 0.5) * k);
    row[N] = k == 0 ? std::sqrt(1.0 / N) : std::sqrt(2.0 / N);
  }
  return FPTC_OK;
}

int32_t fptc_build_basis(int32_t N, int32_t E, float *basis_out) {
  if (!basis_out || !valid_n(N) || E < 1 || E > N) return FPTC_ERR_INVALID_ARG;
  std::vector<double> B = basis64(N, E);
  for (size_t i = 0; i < B.size(); ++i) basis_out[i] = (float)B[i];
  return FPTC_OK;
}

int32_t fptc_build_dequant(const fptc_quant_params *q, float *deq_val, uint8_t *deq_zone, uint8_t *row_of_bin,
                           int32_t *n_rows_out) {
  if (!deq_val || !deq_zone || !row_of_bin || !n_rows_out) return FPTC_ERR_INVALID_ARG;
  int rc = check_quant(q);
  if (rc != FPTC_OK) return rc;
  Quant Q(*q);
  int rows = q->kind == FPTC_QUANT_AMPLITUDE ? 1 : 3;
  for (int r = 0; r < rows; ++r)
    for (int s = 0; s < 256; ++s) {
      deq_val[r * 256 + s] = (float)Q.value(s, r);
      deq_zone[r * 256 + s] = (uint8_t)Q.zone(s, r);
    }
  for (int k = 0; k < q->E; ++k) row_of_bin[k] = (uint8_t)(q->kind == FPTC_QUANT_AMPLITUDE ? 0 : Q.zone_of_bin(k));
  *n_rows_out = rows;
  return FPTC_OK;
}

int32_t fptc_quantize_host(const float *x, int64_t L, const fptc_quant_params *q, uint8_t *symbols_out) {
  if ((!x && L > 0) || !symbols_out || L < 0) return FPTC_ERR_INVALID_ARG;
  int rc = check_quant(q);
  if (rc != FPTC_OK) return rc;
  quantize_strip(x, L, *q, basis64(q->N, q->N), symbols_out);
  return FPTC_OK;
}

int32_t fptc_symlen_pack_host(const uint8_t *symbols, int64_t n, const uint8_t *code_len, uint64_t *words,
                              uint8_t *symlen, int64_t cap, int64_t *n_words_out) {
  if ((!symbols && n > 0) || !code_len || !words || !symlen || !n_words_out || n < 0) return FPTC_ERR_INVALID_ARG;
  uint32_t code[256];
  int rc = canonical(code_len, code);
  if (rc != FPTC_OK) return rc;
  int64_t w = pack(symbols, n, code_len, code, words, symlen, cap);
  if (w < 0) return FPTC_ERR_INVALID_ARG;
  *n_words_out = w;
  return FPTC_OK;
}

int32_t fptc_encode_batch_host(const float *x, const int64_t *sample_off, int32_t n_streams,
                               const uint8_t *book_id, const fptc_quant_params *q, const uint8_t *code_len,
                               const int64_t *word_cap_off, uint64_t *words, uint8_t *symlen,
                               int64_t *n_words_out, int32_t n_threads) {
  if (!x || !sample_off || n_streams < 1 || !code_len || !word_cap_off || !words || !symlen || !n_words_out)
    return FPTC_ERR_INVALID_ARG;
  int rc = check_quant(q);
  if (rc != FPTC_OK) return rc;
  int n_books = 1;
  if (book_id)
    for (int s = 0; s < n_streams; ++s) n_books = std::max(n_books, (int)book_id[s] + 1);
  std::vector<uint32_t> codes((size_t)n_books * 256);
  for (int b = 0; b < n_books; ++b) {
    rc = canonical(code_len + 256 * b, &codes[256 * (size_t)b]);
    if (rc != FPTC_OK) return rc;
  }
  const std::vector<double> B = basis64(q->N, q->N);
  if (n_threads < 1) n_threads = (int)std::max(1u, std::thread::hardware_concurrency());
  std::vector<int> errs(n_threads, 0);
  auto work = [&](int tid) {
    std::vector<uint8_t> sym;
    for (int s = tid; s < n_streams; s += n_threads) {
      int64_t L = sample_off[s + 1] - sample_off[s];
      int64_t nw = (L + q->N - 1) / q->N;
      sym.resize((size_t)(nw * q->E));
      quantize_strip(x + sample_off[s], L, *q, B, sym.data());
      int b = book_id ? book_id[s] : 0;
      int64_t w = pack(sym.data(), (int64_t)sym.size(), code_len + 256 * b, &codes[256 * (size_t)b],
                       words + word_cap_off[s], symlen + word_cap_off[s], word_cap_off[s + 1] - word_cap_off[s]);
      if (w < 0) {
        errs[tid] = 1;
        n_words_out[s] = 0;
      } else {
        n_words_out[s] = w;
      }
    }
  };
  std::vector<std::thread> th;
  for (int t = 0; t < n_threads; ++t) th.emplace_back(work, t);
  for (auto &t : th) t.join();
  for (int e : errs)
    if (e) return FPTC_ERR_INVALID_ARG;
  return FPTC_OK;
}

}  // extern "C"
