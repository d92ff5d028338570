// The steps before the decode path, on the GPU: the encoder's forward
// transform and quantization (Section 3.1, Section 3.2), the symbol histogram
// a codebook is built from (Section 3.3), and the clipped zone maxima A0 / A1
// of the paper quantizer (Section 3.2, the Table 1 percentile).
//
// The forward transform runs in FP64 with every product and sum rounded
// separately (no fused multiply-adds), in the order of its definition
// X[k] = a_k * sum_n x[n] cos(pi/N (n + 1/2) k), on a table of cosines and
// a_k built on the host; the quantization decisions are taken on those FP64
// values, so the symbols are those of a sequential FP64 encoder.
#include <hip/hip_runtime.h>

#include "fptc_internal.h"

#pragma clang fp contract(off)

namespace fptc {
namespace {

constexpr int kThreads = 256;
constexpr int kStageDoubles = 4096;  // LDS staging of sample windows (32 KB)

// Section 3.2 quantizers on one coefficient c of bin k.  Levels: 128 = zero,
// above it positive, below negative; rounding floor(x + 1/2) on magnitudes.
struct DevQuant {
  fptc_quant_params q;
  long long mT;  // amplitude quantizer: fine levels up to the threshold

  __device__ int zone_of_bin(int k) const { return k < q.B1 ? 0 : (k < q.B2 ? 1 : 2); }

  __device__ uint8_t operator()(double c, int k) const {
    if (q.kind == FPTC_QUANT_AMPLITUDE) {
      const double a = fabs(c);
      const long long m = a <= q.threshold ? (long long)floor(a / q.step_fine + 0.5)
                                           : mT + (long long)floor((a - q.threshold) / q.step_coarse + 0.5);
      if (c >= 0) return (uint8_t)(128 + (m < 127 ? m : 127));
      return (uint8_t)(128 - (m < 128 ? m : 128));
    }
    const int z = zone_of_bin(k);
    if (z == 2) return 128;
    if (z == 0) {  // Eq. 2 with |c| clipped to A0, levels as Eq. 3 without a deadzone
      if (c == 0.0) return 128;
      const double a = fmin(fabs(c), q.A0);
      const double u = log(1.0 + q.mu * a / q.A0) / log(1.0 + q.mu);
      if (c > 0) return (uint8_t)(129 + (long long)floor(u * 126.0 + 0.5));
      return (uint8_t)(127 - (long long)floor(u * 127.0 + 0.5));
    }
    const double d1 = q.alpha1 * q.A1;  // Eq. 3, |c| clipped to A1
    const double a = fmin(fabs(c), q.A1);
    if (c > d1) return (uint8_t)(129 + (long long)floor((a - d1) / (q.A1 - d1) * 126.0 + 0.5));
    if (c < -d1) return (uint8_t)(127 - (long long)floor((a - d1) / (q.A1 - d1) * 127.0 + 0.5));
    return 128;
  }
};

// Stream of global window g: the last s with win_off[s] <= g, win_off[s] =
// sym_off[s] / E (streams with no windows share offsets; the last one holding
// g is the one whose range contains it).
__device__ inline int stream_of_window(const int64_t *sym_off, int n, int E, int64_t g) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sym_off[mid] / E <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// One workgroup takes G windows at a time: their samples are staged in LDS as
// doubles (zero past the stream's end), then thread t computes bin t % E of
// window t / E.
__global__ void __launch_bounds__(kThreads) k_fdct_quant(int n_streams, const int64_t *__restrict__ sample_off,
                                                         const int64_t *__restrict__ sym_off, int N, int E, int G,
                                                         DevQuant Q, const double *__restrict__ tab,
                                                         const float *__restrict__ x, uint8_t *__restrict__ symbols,
                                                         double *__restrict__ coef) {
  __shared__ double xs[kStageDoubles];
  __shared__ int64_t wbase[kThreads], wlen[kThreads], wsym[kThreads];
  const int64_t n_win = sym_off[n_streams] / E;
  for (int64_t g0 = (int64_t)blockIdx.x * G; g0 < n_win; g0 += (int64_t)gridDim.x * G) {
    __syncthreads();  // the previous group's reads are done
    if ((int)threadIdx.x < G) {
      const int64_t g = g0 + threadIdx.x;
      int64_t base = 0, len = 0, sb = -1;
      if (g < n_win) {
        const int s = stream_of_window(sym_off, n_streams, E, g);
        const int64_t j = g - sym_off[s] / E;  // window within the stream
        base = sample_off[s] + j * N;
        const int64_t rest = sample_off[s + 1] - base;
        len = rest < N ? rest : N;
        sb = sym_off[s] + j * E;
      }
      wbase[threadIdx.x] = base;
      wlen[threadIdx.x] = len;
      wsym[threadIdx.x] = sb;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < G * N; i += kThreads) {
      const int w = i / N, n = i % N;
      xs[i] = n < wlen[w] ? (double)x[wbase[w] + n] : 0.0;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < G * E; t += kThreads) {
      const int w = t / E, k = t % E;
      if (wsym[w] < 0) continue;
      const double *c = tab + (size_t)k * (N + 1);
      const double *xw = xs + w * N;
      double s = 0.0;
      for (int n = 0; n < N; ++n) s = s + xw[n] * c[n];
      const double X = c[N] * s;
      symbols[wsym[w] + k] = Q(X, k);
      if (coef) coef[wsym[w] + k] = X;
    }
  }
}

// Histogram of the symbols of every stream, per codebook: LDS counts per
// workgroup (32-bit, at most 2^32 - 1 symbols per workgroup pass), added to
// the global 64-bit counts at the end.
__global__ void __launch_bounds__(kThreads) k_histogram(int n_streams, const int64_t *__restrict__ sym_off,
                                                        const uint8_t *__restrict__ book_id, int n_books,
                                                        const uint8_t *__restrict__ symbols,
                                                        unsigned long long *__restrict__ counts) {
  __shared__ unsigned h[kMaxBooks * 256];
  for (int i = threadIdx.x; i < n_books * 256; i += kThreads) h[i] = 0;
  __syncthreads();
  // one stream at a time, all workgroups striding over its symbols
  for (int s = 0; s < n_streams; ++s) {
    const int bk = book_id ? book_id[s] : 0;
    if (bk >= n_books) continue;
    unsigned *hb = h + bk * 256;
    const int64_t a = sym_off[s], b = sym_off[s + 1];
    for (int64_t i = a + (int64_t)blockIdx.x * kThreads + threadIdx.x; i < b; i += (int64_t)gridDim.x * kThreads)
      atomicAdd(&hb[symbols[i]], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n_books * 256; i += kThreads)
    if (h[i]) atomicAdd(&counts[i], (unsigned long long)h[i]);
}

// ---------------------------------------------------------------- percentile
// Radix selection of the r-th smallest |coef[w][k]|, k0 <= k < k1, over the
// FP64 bit patterns (non-negative doubles order like their bits), one byte
// per pass from the top.  State in the workspace:
struct SelState {
  unsigned long long prefix, mask;  // bits fixed so far
  unsigned long long rank;          // rank still to skip among the candidates
  unsigned long long result[2];     // bits of the two order statistics
  unsigned long long hist[256];
};

__global__ void __launch_bounds__(kThreads) k_sel_count(const double *__restrict__ coef, int64_t n_windows, int E,
                                                        int k0, int k1, int shift, SelState *st) {
  __shared__ unsigned h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const unsigned long long prefix = st->prefix, mask = st->mask;
  const int nk = k1 - k0;
  const int64_t M = n_windows * nk;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < M; i += (int64_t)gridDim.x * kThreads) {
    const int64_t w = i / nk;
    const int k = k0 + (int)(i - w * nk);
    const unsigned long long v = (unsigned long long)__double_as_longlong(fabs(coef[w * E + k]));
    if ((v & mask) == prefix) atomicAdd(&h[(v >> shift) & 255u], 1u);
  }
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&st->hist[threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

// Fix the next byte: the bucket holding the remaining rank.  slot < 0: set up
// for rank `rank` (first pass); after the last pass the bits go to
// result[slot].  One thread.
__global__ void k_sel_pick(SelState *st, int shift, int slot, unsigned long long rank) {
  if (slot < 0) {
    st->prefix = 0;
    st->mask = 0;
    st->rank = rank;
    for (int i = 0; i < 256; ++i) st->hist[i] = 0;
    return;
  }
  unsigned long long r = st->rank, acc = 0;
  int b = 255;
  for (int i = 0; i < 256; ++i) {
    if (acc + st->hist[i] > r) {
      b = i;
      break;
    }
    acc += st->hist[i];
  }
  st->rank = r - acc;
  st->prefix |= (unsigned long long)b << shift;
  st->mask |= 255ull << shift;
  for (int i = 0; i < 256; ++i) st->hist[i] = 0;
  if (shift == 0) st->result[slot] = st->prefix;
}

// numpy's 'linear' percentile from the two order statistics: a + (b - a) t,
// or b - (b - a)(1 - t) when t >= 1/2.
__global__ void k_sel_finish(const SelState *st, double t, double *out) {
  const double a = __longlong_as_double((long long)st->result[0]);
  const double b = __longlong_as_double((long long)st->result[1]);
  const double d = b - a;
  out[0] = t >= 0.5 ? b - d * (1.0 - t) : a + d * t;
}

int grid_for(int64_t items) {
  const int64_t want = (items + kThreads - 1) / kThreads;
  const int64_t cap = (int64_t)device_cu_count() * 8;
  return (int)(want < 1 ? 1 : (want > cap ? cap : want));
}

}  // namespace

int launch_fdct_quant(const fptc_batch &b, const fptc_quant_params &q, const double *tab, const int64_t *sym_off,
                      const float *x, uint8_t *symbols, double *coef, int64_t n_windows, void *stream) {
  DevQuant Q{q, 0};
  if (q.kind == FPTC_QUANT_AMPLITUDE) Q.mT = (long long)llround(q.threshold / q.step_fine);
  int G = kThreads / q.E;
  if (G < 1) G = 1;
  if (G * q.N > kStageDoubles) G = kStageDoubles / q.N;
  const int blocks = grid_for((n_windows + G - 1) / G * kThreads);
  hipLaunchKernelGGL(k_fdct_quant, dim3(blocks), dim3(kThreads), 0, (hipStream_t)stream, b.n_streams, b.sample_off,
                     sym_off, q.N, q.E, G, Q, tab, x, symbols, coef);
  return (int)hipGetLastError();
}

int launch_histogram(const fptc_batch &b, const int64_t *sym_off, int n_books, const uint8_t *symbols,
                     uint64_t *counts, int64_t n_symbols, void *stream) {
  const int blocks = grid_for(n_symbols / 64 + 1);
  hipLaunchKernelGGL(k_histogram, dim3(blocks), dim3(kThreads), 0, (hipStream_t)stream, b.n_streams, sym_off,
                     b.book_id, n_books, symbols, reinterpret_cast<unsigned long long *>(counts));
  return (int)hipGetLastError();
}

size_t percentile_ws_bytes() { return sizeof(SelState); }

int launch_abs_percentile(const double *coef, int64_t n_windows, int E, int k0, int k1, double q, double *out,
                          void *ws, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  SelState *s = static_cast<SelState *>(ws);
  const int64_t M = n_windows * (int64_t)(k1 - k0);
  // numpy 'linear': virtual index h = (M - 1) q, neighbours floor(h) and
  // floor(h) + 1 (both M - 1 when h >= M - 1), weight h - floor(h)
  const double h = (double)(M - 1) * q;
  double lo_d = floor(h);
  unsigned long long lo = (unsigned long long)lo_d, hi = lo + 1;
  if (h >= (double)(M - 1)) lo = hi = (unsigned long long)(M - 1);
  const double t = h - lo_d;
  const int blocks = grid_for(M);
  const unsigned long long ranks[2] = {lo, hi};
  for (int slot = 0; slot < 2; ++slot) {
    hipLaunchKernelGGL(k_sel_pick, dim3(1), dim3(1), 0, st, s, 0, -1, ranks[slot]);
    for (int shift = 56; shift >= 0; shift -= 8) {
      hipLaunchKernelGGL(k_sel_count, dim3(blocks), dim3(kThreads), 0, st, coef, n_windows, E, k0, k1, shift, s);
      hipLaunchKernelGGL(k_sel_pick, dim3(1), dim3(1), 0, st, s, shift, slot, 0ull);
    }
  }
  hipLaunchKernelGGL(k_sel_finish, dim3(1), dim3(1), 0, st, s, t, out);
  return (int)hipGetLastError();
}

}  // namespace fptc
