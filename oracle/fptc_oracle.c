/*
 * FPTC reference oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, sequential, double-precision CPU implementation of what the FPTC
 * codec computes, written from the paper (Mechels et al., "FPTC: A Fast
 * Parallel Transform-based Codec for Efficient Asymmetric Signal
 * Compression").  It exists to check the HIP decoder; only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * code, header, table or helper with the GPU library.
 *
 * Every routine follows the plain definition of its step; nothing is blocked,
 * fused or reordered for speed.
 *
 * Sections followed:
 *   Section 3.1, Eq. (1)  windowed DCT-II (orthonormal scaling, see below)
 *   Section 3.2, Eq. (2)  zone-0 mu-law companding
 *   Section 3.2, Eq. (3)  zone-1 linear deadzone
 *   Section 3.2           zone-2 zeroing; 8-bit level layout (128 = zero)
 *   Section 3.3           length-limited Huffman lengths (package-merge),
 *                         canonical code assignment
 *   Section 4.1, Alg. 1   SymLen packing
 *   Section 4.2           per-word decode of exactly symlen[w] symbols
 *   Section 5.1, Eq. (4), (5)  compression ratio and PRD
 * Readings where the paper is silent are stated next to the code that uses
 * them.  Pins: every function is checked by the CPU test suite against
 * closed forms, library routines, invariants or brute force.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_PI 3.14159265358979323846264338327950288

/* ------------------------------------------------------------------------ */
/* Section 3.1: DCT-II.  The workloads use the orthonormal scaling:
 *   X[k] = a_k * sum_n x[n] cos(pi/N (n + 1/2) k),  a_0 = sqrt(1/N), a_k = sqrt(2/N).
 * Eq. (1) of the paper uses the factor 2/N for every k instead; that variant
 * is or_dct_eq1 below and differs from the orthonormal one by a per-bin scale. */

static double or_alpha(int k, int N) { return k == 0 ? sqrt(1.0 / N) : sqrt(2.0 / N); }

static double or_cosarg(int n, int k, int N) { return cos(OR_PI / N * (n + 0.5) * k); }

void or_dct_ortho(const double *x, int N, double *X) {
  for (int k = 0; k < N; ++k) {
    double s = 0.0;
    for (int n = 0; n < N; ++n) s += x[n] * or_cosarg(n, k, N);
    X[k] = or_alpha(k, N) * s;
  }
}

/* Eq. (1) exactly as printed: C[k] = (2/N) sum_n x[n] cos(pi/N (n+1/2) k). */
void or_dct_eq1(const double *x, int N, double *C) {
  for (int k = 0; k < N; ++k) {
    double s = 0.0;
    for (int n = 0; n < N; ++n) s += x[n] * or_cosarg(n, k, N);
    C[k] = 2.0 / N * s;
  }
}

/* The same transforms against a precomputed table cosv[k*N + n] =
 * cos(pi/N (n + 1/2) k): the table holds exactly the values the per-term code
 * evaluates and the sums run in the same order, so the results are identical
 * (a pinned property); stream-level routines use it to avoid N*N cos calls per
 * window. */
static double *or_cos_table(int N) {
  double *t = (double *)malloc(sizeof(double) * (size_t)N * (size_t)N);
  for (int k = 0; k < N; ++k)
    for (int n = 0; n < N; ++n) t[(size_t)k * N + n] = or_cosarg(n, k, N);
  return t;
}

static void or_dct_ortho_t(const double *x, int N, const double *cosv, double *X) {
  for (int k = 0; k < N; ++k) {
    double s = 0.0;
    for (int n = 0; n < N; ++n) s += x[n] * cosv[(size_t)k * N + n];
    X[k] = or_alpha(k, N) * s;
  }
}

static void or_idct_ortho_t(const double *X, int N, int E, const double *cosv, double *x) {
  for (int n = 0; n < N; ++n) {
    double s = 0.0;
    for (int k = 0; k < E; ++k) s += or_alpha(k, N) * X[k] * cosv[(size_t)k * N + n];
    x[n] = s;
  }
}

/* Test hook: table-based transforms of one window (must equal or_dct_ortho /
 * or_idct_ortho bit for bit). */
void or_dct_ortho_tab(const double *x, int N, double *X) {
  double *t = or_cos_table(N);
  or_dct_ortho_t(x, N, t, X);
  free(t);
}

void or_idct_ortho_tab(const double *X, int N, int E, double *x) {
  double *t = or_cos_table(N);
  or_idct_ortho_t(X, N, E, t, x);
  free(t);
}

/* Inverse of the orthonormal DCT-II (a DCT-III) from the first E coefficients;
 * bins k >= E are the ones discarded by spectral truncation (Section 3.1) and
 * count as zero. */
void or_idct_ortho(const double *X, int N, int E, double *x) {
  for (int n = 0; n < N; ++n) {
    double s = 0.0;
    for (int k = 0; k < E; ++k) s += or_alpha(k, N) * X[k] * or_cosarg(n, k, N);
    x[n] = s;
  }
}

/* ------------------------------------------------------------------------ */
/* Section 3.2: quantizers.  A symbol is one byte; 128 is the zero level,
 * 129..255 carry positive values and 0..127 negative values.
 *
 * Two families are implemented:
 *  (a) amplitude three-zone quantizer used by the evaluation workloads: a zero
 *      zone |c| < step_f/2, a fine zone of step step_f up to |c| = T, and a
 *      coarse zone of step step_c beyond T.  Rounding is floor(x + 1/2) on |c|
 *      (the paper's rounding rule, applied to the magnitude).  Magnitude levels
 *      saturate at 127 (positive side) and 128 (negative side).
 *  (b) the paper's frequency three-zone quantizer: bins [0, B1) mu-law (Eq. 2),
 *      [B1, B2) linear deadzone (Eq. 3), [B2, E) zeroed.
 * The paper prints only the forward maps; the reconstruction points are the
 * inverse of the rounding grid (reading). */

typedef struct {
  double step_f, step_c, T;
} or_amp_q;

static long or_floor_half(double v) { return (long)floor(v + 0.5); }

int or_quant_amp(double c, double step_f, double step_c, double T) {
  double a = fabs(c);
  long mT = or_floor_half(T / step_f);
  long m;
  if (a <= T)
    m = or_floor_half(a / step_f);
  else
    m = mT + or_floor_half((a - T) / step_c);
  if (c >= 0.0) {
    if (m > 127) m = 127;
    return (int)(128 + m);
  }
  if (m > 128) m = 128;
  return (int)(128 - m);
}

static long or_amp_level(int s) { return s >= 128 ? (long)(s - 128) : (long)(128 - s); }

double or_dequant_amp(int s, double step_f, double step_c, double T) {
  long m = or_amp_level(s);
  long mT = or_floor_half(T / step_f);
  double mag = (m <= mT) ? (double)m * step_f : T + (double)(m - mT) * step_c;
  return s >= 128 ? mag : -mag;
}

/* Zone of a symbol under (a): 0 = zero zone, 1 = fine, 2 = coarse. */
int or_zone_amp(int s, double step_f, double step_c, double T) {
  (void)step_c;
  long m = or_amp_level(s);
  long mT = or_floor_half(T / step_f);
  if (m == 0) return 0;
  return m <= mT ? 1 : 2;
}

/* (b) Paper quantizer.  zone(k) = 0 for k < B1, 1 for B1 <= k < B2, else 2. */
int or_zone_of_bin(int k, int B1, int B2) {
  if (k < B1) return 0;
  if (k < B2) return 1;
  return 2;
}

/* Eq. (2) with |c| clipped to A0 (Eq. 2 is stated for |c| <= A0).  The level
 * layout for zone 0 mirrors Eq. (3) with a zero deadzone (reading): positive
 * values take 129 + floor(126 q + 1/2), negative ones 127 - floor(127 q + 1/2),
 * exact zero takes 128. */
static int or_q_mulaw(double c, double mu, double A0) {
  if (c == 0.0) return 128;
  double a = fabs(c);
  if (a > A0) a = A0;
  double q = log(1.0 + mu * a / A0) / log(1.0 + mu);
  if (c > 0.0) return 129 + (int)or_floor_half(q * 126.0);
  return 127 - (int)or_floor_half(q * 127.0);
}

static double or_dq_mulaw(int s, double mu, double A0) {
  if (s == 128) return 0.0;
  double q = s > 128 ? (s - 129) / 126.0 : (127 - s) / 127.0;
  double mag = A0 / mu * (pow(1.0 + mu, q) - 1.0);
  return s > 128 ? mag : -mag;
}

/* Eq. (3), with |c| clipped to A1 so the level stays inside one byte. */
static int or_q_deadzone(double c, double A1, double alpha1) {
  double d1 = alpha1 * A1;
  double a = fabs(c);
  if (a > A1) a = A1;
  if (c > d1) return 129 + (int)or_floor_half((a - d1) / (A1 - d1) * 126.0);
  if (c < -d1) return 127 - (int)or_floor_half((a - d1) / (A1 - d1) * 127.0);
  return 128;
}

/* Reconstruction: level 129 + j -> d1 + j (A1 - d1)/126, 127 - j -> -(d1 + j (A1 - d1)/127). */
static double or_dq_deadzone(int s, double A1, double alpha1) {
  double d1 = alpha1 * A1;
  if (s == 128) return 0.0;
  if (s > 128) return d1 + (s - 129) * (A1 - d1) / 126.0;
  return -(d1 + (127 - s) * (A1 - d1) / 127.0);
}

int or_quant_paper(double c, int k, int B1, int B2, double mu, double alpha1, double A0, double A1) {
  int z = or_zone_of_bin(k, B1, B2);
  if (z == 0) return or_q_mulaw(c, mu, A0);
  if (z == 1) return or_q_deadzone(c, A1, alpha1);
  return 128;
}

double or_dequant_paper(int s, int k, int B1, int B2, double mu, double alpha1, double A0, double A1) {
  int z = or_zone_of_bin(k, B1, B2);
  if (z == 0) return or_dq_mulaw(s, mu, A0);
  if (z == 1) return or_dq_deadzone(s, A1, alpha1);
  return 0.0;
}

/* ------------------------------------------------------------------------ */
/* Section 3.3: length-limited code lengths by package-merge (Larmore and
 * Hirschberg).  Each symbol contributes one coin per level 1..lmax; at each
 * level the sorted list is paired into packages and merged with the leaves;
 * after lmax - 1 rounds the 2(n - 1) cheapest items are kept and a symbol's
 * code length is the number of kept items it occurs in.  Items carry an
 * explicit per-symbol count vector: slow and obvious.
 * Returns 0 on success, -1 if lmax is too small for the alphabet or the
 * arguments are invalid.  Symbols with freq 0 get length 0 (no code). */

typedef struct {
  double w;
  uint16_t cnt[256];
} or_item;

static int or_item_cmp(const void *a, const void *b) {
  const or_item *x = (const or_item *)a, *y = (const or_item *)b;
  if (x->w < y->w) return -1;
  if (x->w > y->w) return 1;
  return 0;
}

int or_package_merge(const uint64_t *freq, int nsym, int lmax, uint8_t *len) {
  if (nsym < 1 || nsym > 256 || lmax < 1 || lmax > 32) return -1;
  int used[256];
  int n = 0;
  for (int i = 0; i < nsym; ++i) {
    len[i] = 0;
    if (freq[i] > 0) used[n++] = i;
  }
  if (n == 0) return 0;
  if (n == 1) {
    len[used[0]] = 1;
    return 0;
  }
  if (lmax < 31 && (1L << lmax) < n) return -1;
  /* Leaves, sorted by weight; ties keep symbol order (stable insertion sort). */
  or_item *leaves = (or_item *)calloc((size_t)n, sizeof(or_item));
  or_item *list = (or_item *)calloc((size_t)(2 * n), sizeof(or_item));
  or_item *next = (or_item *)calloc((size_t)(3 * n), sizeof(or_item));
  if (!leaves || !list || !next) {
    free(leaves); free(list); free(next);
    return -1;
  }
  for (int i = 0; i < n; ++i) {
    leaves[i].w = (double)freq[used[i]];
    leaves[i].cnt[used[i]] = 1;
  }
  for (int i = 1; i < n; ++i) { /* stable insertion sort by weight */
    or_item t = leaves[i];
    int j = i - 1;
    while (j >= 0 && leaves[j].w > t.w) { leaves[j + 1] = leaves[j]; --j; }
    leaves[j + 1] = t;
  }
  int m = n;
  memcpy(list, leaves, sizeof(or_item) * (size_t)n);
  for (int round = 1; round < lmax; ++round) {
    /* package: pair consecutive items */
    int np = m / 2;
    int q = 0;
    for (int p = 0; p < np; ++p) {
      or_item pk;
      pk.w = list[2 * p].w + list[2 * p + 1].w;
      for (int s = 0; s < 256; ++s) pk.cnt[s] = (uint16_t)(list[2 * p].cnt[s] + list[2 * p + 1].cnt[s]);
      next[n + q++] = pk;
    }
    /* merge leaves and packages; a leaf goes first on equal weight */
    int a = 0, b = 0, o = 0;
    or_item *pk = next + n;
    or_item *merged = (or_item *)malloc(sizeof(or_item) * (size_t)(n + np));
    if (!merged) { free(leaves); free(list); free(next); return -1; }
    while (a < n || b < np) {
      if (b >= np || (a < n && leaves[a].w <= pk[b].w)) merged[o++] = leaves[a++];
      else merged[o++] = pk[b++];
    }
    m = o < 2 * n ? o : 2 * n; /* only the 2n cheapest can ever be selected */
    memcpy(list, merged, sizeof(or_item) * (size_t)m);
    free(merged);
  }
  int take = 2 * n - 2;
  if (take > m) { free(leaves); free(list); free(next); return -1; }
  int total[256] = {0};
  for (int i = 0; i < take; ++i)
    for (int s = 0; s < 256; ++s) total[s] += list[i].cnt[s];
  for (int i = 0; i < nsym; ++i) len[i] = (uint8_t)total[i];
  free(leaves); free(list); free(next);
  return 0;
}

/* Canonical codes (Section 3.3): order the coded symbols by (length, symbol);
 * the first gets code 0 and each next code is (previous + 1) shifted left by
 * the growth in length.  Codes are read MSB-first. */
void or_canonical_codes(const uint8_t *len, int nsym, uint32_t *code) {
  int maxl = 0;
  for (int i = 0; i < nsym; ++i) { code[i] = 0; if (len[i] > maxl) maxl = len[i]; }
  uint32_t c = 0;
  int prev = 0, first = 1;
  for (int l = 1; l <= maxl; ++l) {
    for (int s = 0; s < nsym; ++s) {
      if (len[s] != l) continue;
      if (first) { c = 0; first = 0; }
      else c = (c + 1) << (l - prev);
      prev = l;
      code[s] = c;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Section 4.1, Algorithm 1: SymLen packing.  Codewords are appended MSB-first
 * into a 64-bit buffer; when the next codeword does not fit, the buffer and
 * its symbol count are emitted and packing restarts in a fresh word.  A
 * codeword is never split.  Returns the number of words written, or -1 if a
 * symbol has no code or the output capacity is exceeded. */
int64_t or_symlen_pack(const uint8_t *sym, int64_t n, const uint32_t *code, const uint8_t *len,
                       uint64_t *out, uint8_t *symlen, int64_t cap) {
  int64_t i = 0, w = 0;
  uint64_t buffer = 0;
  int bits = 0, count = 0;
  while (i < n) {
    int cl = len[sym[i]];
    if (cl == 0) return -1;
    if (bits + cl > 64) {
      if (w >= cap) return -1;
      out[w] = buffer;
      symlen[w] = (uint8_t)count;
      ++w;
      buffer = 0;
      bits = 0;
      count = 0;
    } else {
      int shift = 64 - bits - cl;
      buffer |= ((uint64_t)code[sym[i]]) << shift;
      bits += cl;
      ++count;
      ++i;
    }
  }
  if (count > 0) {
    if (w >= cap) return -1;
    out[w] = buffer;
    symlen[w] = (uint8_t)count;
    ++w;
  }
  return w;
}

/* ------------------------------------------------------------------------ */
/* Decoder (Section 4.2): each word is decoded on its own, exactly symlen[w]
 * symbols, from its most significant bit.  This oracle reads one bit at a
 * time against the canonical first-code / count-per-length tables, not a
 * lookup table.
 * Returns the number of symbols written, or a negative error:
 *   -1 a codeword runs past bit 64 of its word (or no code matches),
 *   -2 the symbols decoded do not equal n_expected,
 *   -3 invalid code lengths. */
int64_t or_symlen_decode(const uint64_t *words, const uint8_t *symlen, int64_t n_words,
                         const uint8_t *len, int nsym, uint8_t *out, int64_t n_expected) {
  int count[33] = {0};
  int maxl = 0;
  for (int s = 0; s < nsym; ++s) {
    if (len[s] > 32) return -3;
    if (len[s]) { count[len[s]]++; if (len[s] > maxl) maxl = len[s]; }
  }
  /* symbols ordered by (length, symbol); first code and first index per length */
  int sorted[256], idx[34];
  uint32_t first[34];
  int o = 0;
  idx[1] = 0;
  for (int l = 1; l <= maxl; ++l) {
    idx[l] = o;
    for (int s = 0; s < nsym; ++s)
      if (len[s] == l) sorted[o++] = s;
  }
  uint32_t c = 0;
  for (int l = 1; l <= maxl; ++l) {
    if (l == 1) c = 0;
    else c = (c + (uint32_t)count[l - 1]) << 1;
    first[l] = c;
  }
  int64_t produced = 0;
  for (int64_t w = 0; w < n_words; ++w) {
    int pos = 0;
    for (int j = 0; j < symlen[w]; ++j) {
      uint32_t v = 0;
      int l = 0, found = -1;
      while (found < 0) {
        if (pos >= 64 || l >= maxl) return -1;
        int bit = (int)((words[w] >> (63 - pos)) & 1u);
        ++pos;
        v = (v << 1) | (uint32_t)bit;
        ++l;
        if (count[l] > 0 && v >= first[l] && v - first[l] < (uint32_t)count[l]) found = sorted[idx[l] + (int)(v - first[l])];
      }
      if (produced >= n_expected) return -2;
      out[produced++] = (uint8_t)found;
    }
  }
  if (produced != n_expected) return -2;
  return produced;
}

/* ------------------------------------------------------------------------ */
/* Stream-level encode.  A strip of L samples is cut into ceil(L/N)
 * non-overlapping windows (Section 3.1); the last partial window is padded
 * with zeros (reading).  Each window contributes its first E coefficients,
 * quantized, in ascending bin order (window-major symbol order).
 * quant_kind 0 = amplitude quantizer (params: step_f, step_c, T),
 * quant_kind 1 = paper quantizer (params: B1, B2, mu, alpha1, A0, A1). */

typedef struct {
  int32_t kind;
  int32_t N, E;
  int32_t B1, B2;
  double step_f, step_c, T;
  double mu, alpha1, A0, A1;
} or_qparams;

static int or_quantize(double c, int k, const or_qparams *p) {
  if (p->kind == 0) return or_quant_amp(c, p->step_f, p->step_c, p->T);
  return or_quant_paper(c, k, p->B1, p->B2, p->mu, p->alpha1, p->A0, p->A1);
}

double or_dequantize(int s, int k, const or_qparams *p) {
  if (p->kind == 0) return or_dequant_amp(s, p->step_f, p->step_c, p->T);
  return or_dequant_paper(s, k, p->B1, p->B2, p->mu, p->alpha1, p->A0, p->A1);
}

/* Zone that a per-zone reconstruction scale applies to (reading: for the
 * amplitude quantizer the amplitude zone of the level, for the paper
 * quantizer the frequency zone of the bin). */
int or_zone(int s, int k, const or_qparams *p) {
  if (p->kind == 0) return or_zone_amp(s, p->step_f, p->step_c, p->T);
  return or_zone_of_bin(k, p->B1, p->B2);
}

int64_t or_n_windows(int64_t L, int N) { return (L + N - 1) / N; }

/* Transform + quantize one strip: symbols[ceil(L/N) * E]. */
void or_quantize_stream(const float *x, int64_t L, const or_qparams *p, uint8_t *symbols) {
  int N = p->N, E = p->E;
  int64_t nw = or_n_windows(L, N);
  double *win = (double *)malloc(sizeof(double) * (size_t)N);
  double *X = (double *)malloc(sizeof(double) * (size_t)N);
  double *cosv = or_cos_table(N);
  for (int64_t w = 0; w < nw; ++w) {
    for (int n = 0; n < N; ++n) {
      int64_t i = w * N + n;
      win[n] = i < L ? (double)x[i] : 0.0;
    }
    or_dct_ortho_t(win, N, cosv, X);
    for (int k = 0; k < E; ++k) symbols[w * E + k] = (uint8_t)or_quantize(X[k], k, p);
  }
  free(cosv);
  free(win);
  free(X);
}

/* Same transform, returning the kept coefficients (for training statistics
 * and percentiles): coef[ceil(L/N) * E]. */
void or_dct_stream(const float *x, int64_t L, int N, int E, double *coef) {
  int64_t nw = or_n_windows(L, N);
  double *win = (double *)malloc(sizeof(double) * (size_t)N);
  double *X = (double *)malloc(sizeof(double) * (size_t)N);
  double *cosv = or_cos_table(N);
  for (int64_t w = 0; w < nw; ++w) {
    for (int n = 0; n < N; ++n) {
      int64_t i = w * N + n;
      win[n] = i < L ? (double)x[i] : 0.0;
    }
    or_dct_ortho_t(win, N, cosv, X);
    for (int k = 0; k < E; ++k) coef[w * E + k] = X[k];
  }
  free(cosv);
  free(win);
  free(X);
}

/* Symbol histogram (Section 3.3). */
void or_histogram(const uint8_t *sym, int64_t n, uint64_t *hist) {
  for (int s = 0; s < 256; ++s) hist[s] = 0;
  for (int64_t i = 0; i < n; ++i) hist[sym[i]]++;
}

/* ------------------------------------------------------------------------ */
/* Reconstruction (Section 4.2, lossy stage): dequantize every symbol, scale
 * it by the stream's per-zone factor gamma[zone] (1 when gamma is NULL), and
 * invert the transform window by window; the first L samples are kept.
 * Output in double precision. */
void or_reconstruct(const uint8_t *symbols, int64_t L, const or_qparams *p, const double *gamma, double *out) {
  int N = p->N, E = p->E;
  int64_t nw = or_n_windows(L, N);
  double *X = (double *)malloc(sizeof(double) * (size_t)E);
  double *x = (double *)malloc(sizeof(double) * (size_t)N);
  double *cosv = or_cos_table(N);
  for (int64_t w = 0; w < nw; ++w) {
    for (int k = 0; k < E; ++k) {
      int s = symbols[w * E + k];
      double g = gamma ? gamma[or_zone(s, k, p)] : 1.0;
      X[k] = g * or_dequantize(s, k, p);
    }
    or_idct_ortho_t(X, N, E, cosv, x);
    for (int n = 0; n < N; ++n) {
      int64_t i = w * N + n;
      if (i < L) out[i] = x[n];
    }
  }
  free(cosv);
  free(X);
  free(x);
}

/* Backward of reconstruction for a loss with output gradient gx = dLoss/dxhat
 * (length L).  Padded samples past L are not outputs, so their gradient is 0.
 *   grad_coef[w*E + k] = dLoss/dchat[w,k] = sum_n gx[w,n] a_k cos(pi/N (n+1/2) k)
 *   grad_gamma[z]      = sum over (w,k) with zone z of grad_coef[w,k] * v[w,k]
 * where v is the dequantized value before scaling.  grad_coef may be NULL. */
void or_backward(const uint8_t *symbols, int64_t L, const or_qparams *p, const double *gx,
                 double *grad_coef, double *grad_gamma) {
  int N = p->N, E = p->E;
  int64_t nw = or_n_windows(L, N);
  double *g = (double *)malloc(sizeof(double) * (size_t)N);
  double *G = (double *)malloc(sizeof(double) * (size_t)N);
  double *cosv = or_cos_table(N);
  grad_gamma[0] = grad_gamma[1] = grad_gamma[2] = 0.0;
  for (int64_t w = 0; w < nw; ++w) {
    for (int n = 0; n < N; ++n) {
      int64_t i = w * N + n;
      g[n] = i < L ? gx[i] : 0.0;
    }
    or_dct_ortho_t(g, N, cosv, G);
    for (int k = 0; k < E; ++k) {
      int s = symbols[w * E + k];
      if (grad_coef) grad_coef[w * E + k] = G[k];
      grad_gamma[or_zone(s, k, p)] += G[k] * or_dequantize(s, k, p);
    }
  }
  free(cosv);
  free(g);
  free(G);
}

/* Section 5.1, Eq. (5): PRD = 100 sqrt(sum (x - xhat)^2 / sum x^2). */
double or_prd(const float *x, const double *xhat, int64_t n) {
  double num = 0.0, den = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double d = (double)x[i] - xhat[i];
    num += d * d;
    den += (double)x[i] * (double)x[i];
  }
  return 100.0 * sqrt(num / den);
}

/* Section 5.1, Eq. (4): CR = original bytes / compressed bytes. */
double or_cr(int64_t orig_bytes, int64_t comp_bytes) { return (double)orig_bytes / (double)comp_bytes; }
