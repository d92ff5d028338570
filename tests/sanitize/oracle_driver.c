/* Runs the oracle's encode and decode functions over seeded random strips,
 * built with AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_sanitizers.py: every buffer is sized exactly, so an access past
 * one, a leak or undefined arithmetic ends the run with an error. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int32_t kind;
  int32_t N, E;
  int32_t B1, B2;
  double step_f, step_c, T;
  double mu, alpha1, A0, A1;
} or_qparams;

int64_t or_n_windows(int64_t L, int N);
void or_quantize_stream(const float *x, int64_t L, const or_qparams *p, uint8_t *symbols);
void or_dct_stream(const float *x, int64_t L, int N, int E, double *coef);
void or_histogram(const uint8_t *sym, int64_t n, uint64_t *hist);
int or_package_merge(const uint64_t *freq, int nsym, int lmax, uint8_t *len);
void or_canonical_codes(const uint8_t *len, int nsym, uint32_t *code);
int64_t or_symlen_pack(const uint8_t *sym, int64_t n, const uint32_t *code, const uint8_t *len, uint64_t *out,
                       uint8_t *symlen, int64_t cap);
int64_t or_symlen_decode(const uint64_t *words, const uint8_t *symlen, int64_t n_words, const uint8_t *len, int nsym,
                         uint8_t *out, int64_t n_expected);
void or_reconstruct(const uint8_t *symbols, int64_t L, const or_qparams *p, const double *gamma, double *out);
void or_backward(const uint8_t *symbols, int64_t L, const or_qparams *p, const double *gx, double *grad_coef,
                 double *grad_gamma);

static uint64_t g_state = 0x2605010860ull;
static double urand(void) {  /* xorshift64*, uniform in [0, 1) */
  g_state ^= g_state >> 12;
  g_state ^= g_state << 25;
  g_state ^= g_state >> 27;
  return (double)((g_state * 2685821657736338717ull) >> 11) * (1.0 / 9007199254740992.0);
}

static void *xmalloc(size_t n) { return malloc(n ? n : 1); }

int main(void) {
  static const int Ns[] = {4, 16, 32, 64, 256};
  for (int trial = 0; trial < 40; ++trial) {
    const int N = Ns[trial % 5];
    int E = N - (trial % 3) * (N / 4);
    if (E < 1) E = 1;
    const int64_t L = (int64_t)(urand() * (5 * N + 8));
    float *x = (float *)xmalloc(sizeof(float) * (size_t)L);
    for (int64_t i = 0; i < L; ++i) x[i] = (float)(20.0 * (urand() - 0.5) * (urand() < 0.2 ? 10.0 : 1.0));
    or_qparams p;
    memset(&p, 0, sizeof(p));
    p.kind = trial & 1;
    p.N = N;
    p.E = E;
    p.step_f = 0.25, p.step_c = 2.0, p.T = 16.0;
    p.B1 = E < 2 ? E : 2;
    p.B2 = p.B1 + (E - p.B1) / 2;
    p.mu = 50.0, p.alpha1 = 0.004, p.A0 = 30.0, p.A1 = 20.0;
    const int64_t nw = or_n_windows(L, N), n = nw * E;
    uint8_t *sym = (uint8_t *)xmalloc((size_t)n);
    double *coef = (double *)xmalloc(sizeof(double) * (size_t)n);
    or_quantize_stream(x, L, &p, sym);
    or_dct_stream(x, L, N, E, coef);
    uint64_t hist[256];
    or_histogram(sym, n, hist);
    for (int s = 0; s < 256; ++s) hist[s] += 1;  /* every byte gets a code */
    uint8_t len[256];
    uint32_t code[256];
    const int lmax = (trial & 2) ? 16 : 12;
    if (or_package_merge(hist, 256, lmax, len) != 0) return 2;
    or_canonical_codes(len, 256, code);
    const int64_t cap = n + 1;
    uint64_t *words = (uint64_t *)xmalloc(sizeof(uint64_t) * (size_t)cap);
    uint8_t *symlen = (uint8_t *)xmalloc((size_t)cap);
    const int64_t nwords = or_symlen_pack(sym, n, code, len, words, symlen, cap);
    if (nwords < 0 || nwords > cap) return 3;
    uint8_t *back = (uint8_t *)xmalloc((size_t)n);
    if (or_symlen_decode(words, symlen, nwords, len, 256, back, n) != n || (n && memcmp(back, sym, (size_t)n))) return 4;
    const double gamma[3] = {1.0, 1.1, 0.9};
    double *xr = (double *)xmalloc(sizeof(double) * (size_t)L);
    or_reconstruct(sym, L, &p, gamma, xr);
    double *gx = (double *)xmalloc(sizeof(double) * (size_t)L);
    for (int64_t i = 0; i < L; ++i) gx[i] = urand() - 0.5;
    double *gc = (double *)xmalloc(sizeof(double) * (size_t)n);
    double gg[3];
    or_backward(sym, L, &p, gx, gc, gg);
    free(x), free(sym), free(coef), free(words), free(symlen), free(back), free(xr), free(gx), free(gc);
  }
  printf("ok\n");
  return 0;
}
