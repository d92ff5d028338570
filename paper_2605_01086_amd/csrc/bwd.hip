// Backward of dequantization + inverse DCT.
//
// Forward (Section 4.2, lossy stage): x[w][n] = sum_k chat[w][k] B[k][n] with
// chat = gamma[stream][zone] * v, v the dequantized table value of the
// symbol.  For an output gradient gx = dL/dx (zero past each stream's end):
//   dL/dchat[w][k] = sum_n gx[w][n] B[k][n]              (a forward DCT-II of gx)
//   dL/dgamma[s][z] = sum over (w, k) of stream s with zone z of dL/dchat * v
// The first is computed in FP32 per chunk of windows (one stream per chunk,
// from the plan); the second is accumulated in FP64, first per chunk in a
// fixed reduction order, then per stream over its chunks in order, so the
// result is deterministic.
#include <hip/hip_runtime.h>

#include "fptc_internal.h"

namespace fptc {
namespace {

constexpr int kThreads = 256;

__host__ __device__ inline int bwd_bins_per_block(int N) { return N >= 256 ? 32 : (N < 64 ? N : 64); }

// One block per chunk at a time.  LDS: gx of the chunk [wpc][N] (zero-padded),
// basis block transposed [N][KB], per-zone FP64 reduction scratch.
__global__ void __launch_bounds__(kThreads) k_bwd_chunk(fptc_batch b, int N, int E, int wpc, int n_books, int n_rows,
                                                        const float *deq_val, const uint8_t *deq_zone,
                                                        const uint8_t *row_of_bin, const float *basis,
                                                        const int64_t *hdr, const ChunkMeta *meta,
                                                        const uint8_t *symbols, const float *gx, float *grad_coeff,
                                                        double *part) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int KB = bwd_bins_per_block(N);
  float *G = reinterpret_cast<float *>(lds);     // [wpc][N]
  float *Bt = G + (size_t)wpc * N;                // [N][KB]
  double *red = reinterpret_cast<double *>(Bt + (size_t)N * KB);  // [kThreads][3]
  const int t = threadIdx.x;
  const int64_t n_chunks = hdr[0];

  for (int64_t c = blockIdx.x; c < n_chunks; c += gridDim.x) {
    const ChunkMeta cm = meta[c];
    const int nwin = cm.n_windows;
    const int book = cm.book < n_books ? cm.book : 0;
    // stage the chunk's output gradient; samples past the stream are not
    // outputs and carry no gradient
    for (int i = t; i < wpc * N; i += kThreads) {
      float v = 0.0f;
      if (i < cm.out_len && cm.out_base + i < b.n_samples) v = gx[cm.out_base + i];
      G[i] = v;
    }
    double acc[3] = {0.0, 0.0, 0.0};
    for (int kb = 0; kb < E; kb += KB) {
      const int kn = min(KB, E - kb);
      __syncthreads();
      for (int i = t; i < N * KB; i += kThreads) {
        const int n = i / KB, k = i % KB;
        Bt[i] = k < kn ? basis[(int64_t)(kb + k) * N + n] : 0.0f;
      }
      __syncthreads();
      // (window, bin) pairs of this block, bins fastest: coalesced writes
      for (int i = t; i < nwin * kn; i += kThreads) {
        const int w = i / kn, k = i % kn;
        const float *g = G + (size_t)w * N;
        float s = 0.0f;
        for (int n = 0; n < N; ++n) s = fmaf(g[n], Bt[n * KB + k], s);
        const int kk = kb + k;
        const int64_t si = cm.sym_base + (int64_t)w * E + kk;
        if (si < b.n_symbols) {
          if (grad_coeff) grad_coeff[si] = s;
          const int r0 = row_of_bin[book * E + kk];
          const int row = r0 < n_rows ? r0 : n_rows - 1;
          const int64_t ti = ((int64_t)book * n_rows + row) * 256 + symbols[si];
          const int z = deq_zone[ti];
          const double prod = (double)s * (double)deq_val[ti];
          acc[0] += z == 0 ? prod : 0.0;
          acc[1] += z == 1 ? prod : 0.0;
          acc[2] += z >= 2 ? prod : 0.0;
        }
      }
    }
    // fixed-order tree reduction of the per-thread FP64 sums
    __syncthreads();
    red[3 * t] = acc[0];
    red[3 * t + 1] = acc[1];
    red[3 * t + 2] = acc[2];
    __syncthreads();
    for (int h = kThreads / 2; h > 0; h >>= 1) {
      if (t < h) {
        red[3 * t] += red[3 * (t + h)];
        red[3 * t + 1] += red[3 * (t + h) + 1];
        red[3 * t + 2] += red[3 * (t + h) + 2];
      }
      __syncthreads();
    }
    if (t < 3) part[3 * c + t] = red[t];
    __syncthreads();
  }
}

// One thread per (stream, zone): sum of the stream's chunk partials in order.
__global__ void k_bwd_streams(int n_streams, const int64_t *chunk_off, const ChunkMeta *meta, const double *part,
                              double *grad_gamma) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= 3 * (int64_t)n_streams) return;
  const int64_t s = i / 3;
  const int z = (int)(i % 3);
  double acc = 0.0;
  for (int64_t c = chunk_off[s]; c < chunk_off[s + 1]; ++c) acc += part[3 * c + z];
  grad_gamma[i] = acc;
}

}  // namespace

int set_bwd_attributes() { return lds_attr(k_bwd_chunk); }

size_t bwd_lds_bytes(const fptc_codec &c, const Shape &s) {
  const int KB = bwd_bins_per_block(c.N);
  return sizeof(float) * ((size_t)s.wpc * c.N + (size_t)c.N * KB) + sizeof(double) * 3 * kThreads;
}

int launch_bwd(const fptc_batch &b, const fptc_codec &c, const Shape &s, const Plan &p, const uint8_t *symbols,
               const float *grad_out, float *grad_coeff, double *grad_gamma, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  const size_t lds = bwd_lds_bytes(c, s);
  const int per_cu = (int)((160 * 1024) / lds);
  const int blocks = s.blocks > 0 ? s.blocks : device_cu_count() * (per_cu < 1 ? 1 : (per_cu > 8 ? 8 : per_cu));
  hipLaunchKernelGGL(k_bwd_chunk, dim3(blocks), dim3(kThreads), lds, st, b, c.N, c.E, s.wpc, c.n_books, c.n_rows,
                     c.deq_val, c.deq_zone, c.row_of_bin, c.basis, p.hdr, p.chunk_meta, symbols, grad_out, grad_coeff,
                     p.bwd_part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !grad_gamma) return (int)e;
  const int64_t nz = 3 * (int64_t)b.n_streams;
  hipLaunchKernelGGL(k_bwd_streams, dim3((unsigned)((nz + 255) / 256)), dim3(256), 0, st, b.n_streams, p.chunk_off,
                     p.chunk_meta, p.bwd_part, grad_gamma);
  return (int)hipGetLastError();
}

}  // namespace fptc
