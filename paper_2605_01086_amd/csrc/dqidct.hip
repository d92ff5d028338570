// Dequantization fused with the inverse DCT (Section 4.2, lossy stage).
//
// Windows of the whole batch are numbered globally (stream by stream, as the
// decoded symbols are stored), so every tile of windows has the same work
// regardless of stream boundaries: the paper's uniform per-sample work
// assignment, here at tile granularity.  Each window's coefficients are
// dequantized on load -- table value of the symbol in the row of its bin, times
// the stream's scale for the symbol's zone -- and contracted with the
// orthonormal IDCT basis.
//
// This file holds the plain FP32 SIMT form: one thread owns one output column
// n of 16 windows; basis and coefficients are staged in LDS in blocks of 64
// bins.
#include <hip/hip_runtime.h>

#include "fptc_internal.h"

namespace fptc {
namespace {

constexpr int kThreads = 256;
constexpr int kPerThread = 16;            // windows per thread
constexpr int kTileOut = kThreads * kPerThread;  // outputs per tile (4096)

// Bins per staged block: keeps the basis block at <= 32 KB of LDS.
__host__ __device__ inline int bins_per_block(int N) { return N >= 256 ? 32 : (N < 64 ? N : 64); }

__device__ inline int find_last_le(const int64_t *off, int n, int64_t g) {
  int lo = 0, hi = n;  // off[lo] <= g < off[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (off[mid] <= g) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Per-window facts of the tile, computed once per tile.
struct WinInfo {
  int64_t out;   // output index of sample 0 of the window
  int valid;     // samples of the window inside the stream (0 = skip)
  int book;
  float g[3];
};

__global__ void __launch_bounds__(kThreads) k_dqidct_f32(fptc_batch b, int N, int E, int n_books, int n_rows,
                                                         const float *deq_val, const uint8_t *deq_zone,
                                                         const uint8_t *row_of_bin, const float *basis,
                                                         const int64_t *hdr, const int64_t *win_off,
                                                         const uint8_t *symbols, const float *__restrict__ gamma, float *out) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int TW = kTileOut / N;  // windows per tile
  const int kKB = bins_per_block(N);
  float *Bs = reinterpret_cast<float *>(lds);               // [kKB][N]
  float *Cs = Bs + kKB * N;                                  // [TW][kKB]
  WinInfo *wi = reinterpret_cast<WinInfo *>(Cs + TW * kKB);  // [TW]

  const int64_t n_win = hdr[1];
  const int64_t n_tiles = (n_win + TW - 1) / TW;
  const int t = threadIdx.x;
  const int col = t % N;
  const int wrow = t / N;           // first window row of this thread
  const int rstep = kThreads / N;   // row stride between this thread's windows

  for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const int64_t g0 = tile * TW;
    for (int tw = t; tw < TW; tw += kThreads) {
      WinInfo w;
      const int64_t g = g0 + tw;
      w.valid = 0;
      w.out = 0;
      w.book = 0;
      w.g[0] = w.g[1] = w.g[2] = 1.0f;
      if (g < n_win) {
        const int s = find_last_le(win_off, b.n_streams, g);
        const int64_t j = g - win_off[s];
        const int64_t L = b.sample_off[s + 1] - b.sample_off[s];
        const int64_t o = b.sample_off[s] + j * N;
        int64_t v = L - j * N;
        v = v < N ? v : N;
        if (o < 0 || o + v > b.n_samples) v = 0;
        w.valid = v > 0 ? (int)v : 0;
        w.out = o;
        const int bk = b.book_id ? (int)b.book_id[s] : 0;
        w.book = bk < n_books ? bk : 0;
        if (gamma) {
          w.g[0] = gamma[3 * (int64_t)s + 0];
          w.g[1] = gamma[3 * (int64_t)s + 1];
          w.g[2] = gamma[3 * (int64_t)s + 2];
        }
      }
      wi[tw] = w;
    }
    float acc[kPerThread];
#pragma unroll
    for (int r = 0; r < kPerThread; ++r) acc[r] = 0.0f;

    // bins from the highest down: the DC term, often a large offset, enters
    // the FP32 sums last
    for (int kb = ((E - 1) / kKB) * kKB; kb >= 0; kb -= kKB) {
      const int kn = min(kKB, E - kb);
      __syncthreads();  // wi ready; previous block's LDS reads done
      for (int i = t; i < kKB * N; i += kThreads) {
        const int k = i / N;
        Bs[i] = k < kn ? basis[(int64_t)(kb + k) * N + (i % N)] : 0.0f;
      }
      for (int i = t; i < TW * kKB; i += kThreads) {
        const int w = i / kKB, k = i % kKB;
        float v = 0.0f;
        const WinInfo &W = wi[w];
        if (k < kn && W.valid > 0) {
          const int64_t si = (g0 + w) * (int64_t)E + kb + k;
          if (si < b.n_symbols) {
            const int sym = symbols[si];
            const int r0 = row_of_bin[W.book * E + kb + k];
            const int row = r0 < n_rows ? r0 : n_rows - 1;
            const int64_t ti = ((int64_t)W.book * n_rows + row) * 256 + sym;
            const int z = deq_zone[ti];
            v = W.g[z < 2 ? z : 2] * deq_val[ti];
          }
        }
        Cs[i] = v;
      }
      __syncthreads();
      for (int k = kn - 1; k >= 0; --k) {
        const float bv = Bs[k * N + col];
#pragma unroll
        for (int r = 0; r < kPerThread; ++r) acc[r] = fmaf(Cs[(wrow + r * rstep) * kKB + k], bv, acc[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < kPerThread; ++r) {
      const WinInfo &W = wi[wrow + r * rstep];
      if (col < W.valid) out[W.out + col] = acc[r];
    }
    __syncthreads();
  }
}

}  // namespace

int launch_dqidct(const fptc_batch &b, const fptc_codec &c, const Shape &s, const Plan &p, const uint8_t *symbols,
                  const float *gamma, int precision, float *out, void *stream) {
  if (precision != FPTC_FP32_SIMT) return (int)hipErrorInvalidValue;
  const int TW = kTileOut / c.N;
  const int kKB = bins_per_block(c.N);
  const size_t lds = sizeof(float) * ((size_t)kKB * c.N + (size_t)TW * kKB) + sizeof(WinInfo) * TW;
  int blocks = s.blocks > 0 ? s.blocks : device_cu_count() * 8;
  hipLaunchKernelGGL(k_dqidct_f32, dim3(blocks), dim3(kThreads), lds, (hipStream_t)stream, b, c.N, c.E, c.n_books,
                     c.n_rows, c.deq_val, c.deq_zone, c.row_of_bin, c.basis, p.hdr, p.win_off, symbols, gamma, out);
  return (int)hipGetLastError();
}

}  // namespace fptc
