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
#include "mfma_common.h"

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

// ---------------------------------------------------------------- matrix cores
// The same gradients with the coefficient gradient on v_mfma_f32_32x32x16_bf16
// for N in {32, 64, 128}: G[w][k] = sum_n gx[w][n] B[k][n] with the output
// gradient as the A operand (32 windows x 16 samples per k-step, read straight
// from memory, 32 bytes per lane) and the basis as the B operand (LDS, rows k,
// 16-bit pieces).  Both operands are split into three BF16 pieces (BF16X3:
// an FP32 value exactly, whatever its magnitude), and the six products down to
// the pieces' combined weight 2^-16 give FP32-level sums.  One wavefront per
// chunk of windows; its FP64 scale-gradient terms are summed per lane in a
// fixed order, then over the wave by a fixed butterfly, into the chunk's
// partial sums (the same per-stream reduction follows).
constexpr int kBwdWaves = 8;

// Basis rows k < Ep (zero past E) as BF16 pieces Bs[p][k][n], rows RS halves apart.
__device__ inline void stage_basis_rows(uint16_t *Bs, const float *basis, int N, int E, int Ep, int RS, int tid,
                                        int nthreads) {
  for (int i = tid; i < Ep * N; i += nthreads) {
    const int k = i / N, n = i % N;
    const float v = k < E ? basis[(int64_t)k * N + n] : 0.0f;
    uint16_t pc[3];
    split<false, 3>(v, pc);
#pragma unroll
    for (int q = 0; q < 3; ++q) Bs[((size_t)q * Ep + k) * RS + n] = pc[q];
  }
}

__device__ inline double wave_sum_f64(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  return v;
}

template <int NTK>
__global__ void __launch_bounds__(kBwdWaves * 64) k_bwd_mfma(fptc_batch b, int N, int E, int n_books, int n_rows,
                                                             const float *__restrict__ deq_val,
                                                             const uint8_t *__restrict__ deq_zone,
                                                             const uint8_t *__restrict__ row_of_bin,
                                                             const float *__restrict__ basis,
                                                             const int64_t *__restrict__ hdr,
                                                             const ChunkMeta *__restrict__ meta,
                                                             const uint8_t *__restrict__ symbols,
                                                             const float *__restrict__ gx, float *grad_coeff,
                                                             double *part) {
  constexpr int Ep = NTK * 32;  // output bins, padded
  const int RS = N + 8;        // LDS row stride of a basis piece, in halves
  const int S = N / 16, KH = N / 2;
  extern __shared__ __align__(16) unsigned char lds[];
  uint16_t *Bs = reinterpret_cast<uint16_t *>(lds);
  unsigned char *tables = lds + (size_t)3 * Ep * RS * 2;
  const DeqTables dt = deq_tables_at(tables, n_books, n_rows, E);
  stage_basis_rows(Bs, basis, N, E, Ep, RS, threadIdx.x, blockDim.x);
  stage_deq_tables<FPTC_BF16X3>(dt, deq_val, deq_zone, row_of_bin, n_books, n_rows, E, threadIdx.x, blockDim.x);

  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63, col = lane & 31, h = lane >> 5;
  const int64_t n_chunks = hdr[0];
  const bool gx16 = (reinterpret_cast<uintptr_t>(gx) & 15) == 0;
  for (int64_t c = (int64_t)blockIdx.x * kBwdWaves + wid; c < n_chunks; c += (int64_t)gridDim.x * kBwdWaves) {
    const ChunkMeta cm = meta_from_lanes(load_meta_lane(meta, c, n_chunks, lane), true);
    const int book = cm.book < n_books && cm.book >= 0 ? cm.book : 0;
    const uint8_t *rb = dt.rb + book * E;
    const float *tv = dt.tv + book * n_rows * 256;
    const uint8_t *tz = dt.tz + book * n_rows * 256;
    double z0 = 0.0, z1 = 0.0, z2 = 0.0;
    for (int tt = 0; tt * kTileWindows < cm.n_windows; ++tt) {
      const int wr = tt * kTileWindows + col;  // this lane's A row: window of the chunk
      // its output gradient, samples h N/2 .. h N/2 + N/2 (zero past the stream)
      const int64_t rbase = (int64_t)wr * N + KH * h;
      f16v acc[NTK];
#pragma unroll
      for (int t = 0; t < NTK; ++t) acc[t] = f16v{};
      for (int s = S - 1; s >= 0; --s) {
        float v[8];
        const int64_t o = rbase + 8 * s;
        if (gx16 && wr < cm.n_windows && o + 8 <= cm.out_len && ((cm.out_base + o) & 3) == 0) {
          const float4 *g4 = reinterpret_cast<const float4 *>(gx + cm.out_base + o);
          const float4 x0 = g4[0], x1 = g4[1];
          v[0] = x0.x, v[1] = x0.y, v[2] = x0.z, v[3] = x0.w, v[4] = x1.x, v[5] = x1.y, v[6] = x1.z, v[7] = x1.w;
        } else {
#pragma unroll
          for (int j = 0; j < 8; ++j) v[j] = (wr < cm.n_windows && o + j < cm.out_len) ? gx[cm.out_base + o + j] : 0.0f;
        }
        u8v a[3];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          uint16_t pc[3];
          split<false, 3>(v[j], pc);
          a[0][j] = pc[0], a[1][j] = pc[1], a[2][j] = pc[2];
        }
        mfma_step<FPTC_BF16X3, NTK>(acc, a, Bs + col * RS + KH * h + 8 * s, 32 * RS, Ep * RS, true);
      }
      // lane (col, h) holds G for bin 32 t + col of windows acc_window(r, h)
#pragma unroll
      for (int t = 0; t < NTK; ++t) {
        const int k = 32 * t + col;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int w = tt * kTileWindows + acc_window(r, h);
          if (k < E && w < cm.n_windows) {
            const int64_t si = cm.sym_base + (int64_t)w * E + k;
            if (si < b.n_symbols) {
              const float g = acc[t][r];
              if (grad_coeff) grad_coeff[si] = g;
              const int ti = rb[k] * 256 + symbols[si];
              const double prod = (double)g * (double)tv[ti];
              const int zz = tz[ti];
              z0 += zz == 0 ? prod : 0.0;
              z1 += zz == 1 ? prod : 0.0;
              z2 += zz >= 2 ? prod : 0.0;
            }
          }
        }
      }
    }
    z0 = wave_sum_f64(z0);
    z1 = wave_sum_f64(z1);
    z2 = wave_sum_f64(z2);
    if (lane == 0) {
      part[3 * c] = z0;
      part[3 * c + 1] = z1;
      part[3 * c + 2] = z2;
    }
  }
}

__host__ __device__ inline size_t bwd_mfma_lds(int N, int E, int n_books, int n_rows) {
  const int Ep = (E + 31) / 32 * 32;
  return (size_t)3 * Ep * (N + 8) * 2 + deq_table_bytes(3, n_books, n_rows, E);
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

int set_bwd_attributes() {
  return lds_attr(k_bwd_chunk) | lds_attr(k_bwd_mfma<1>) | lds_attr(k_bwd_mfma<2>) | lds_attr(k_bwd_mfma<3>) |
         lds_attr(k_bwd_mfma<4>);
}

size_t bwd_lds_bytes(const fptc_codec &c, const Shape &s) {
  const int KB = bwd_bins_per_block(c.N);
  return sizeof(float) * ((size_t)s.wpc * c.N + (size_t)c.N * KB) + sizeof(double) * 3 * kThreads;
}

int launch_bwd(const fptc_batch &b, const fptc_codec &c, const Shape &s, const Plan &p, const uint8_t *symbols,
               const float *grad_out, float *grad_coeff, double *grad_gamma, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  const size_t mlds = bwd_mfma_lds(c.N, c.E, c.n_books, c.n_rows);
  if ((c.N == 32 || c.N == 64 || c.N == 128) && mlds <= 160 * 1024) {
    const int per_cu = (int)((160 * 1024) / mlds);
    const int blocks = s.blocks > 0 ? s.blocks : device_cu_count() * (per_cu < 1 ? 1 : (per_cu > 2 ? 2 : per_cu));
    const int ntk = (c.E + 31) / 32;
    auto kern = ntk == 1 ? k_bwd_mfma<1> : ntk == 2 ? k_bwd_mfma<2> : ntk == 3 ? k_bwd_mfma<3> : k_bwd_mfma<4>;
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(kBwdWaves * 64), mlds, st, b, c.N, c.E, c.n_books, c.n_rows,
                       c.deq_val, c.deq_zone, c.row_of_bin, c.basis, p.hdr, p.chunk_meta, symbols, grad_out,
                       grad_coeff, p.bwd_part);
  } else {
    const size_t lds = bwd_lds_bytes(c, s);
    const int per_cu = (int)((160 * 1024) / lds);
    const int blocks = s.blocks > 0 ? s.blocks : device_cu_count() * (per_cu < 1 ? 1 : (per_cu > 8 ? 8 : per_cu));
    hipLaunchKernelGGL(k_bwd_chunk, dim3(blocks), dim3(kThreads), lds, st, b, c.N, c.E, s.wpc, c.n_books, c.n_rows,
                       c.deq_val, c.deq_zone, c.row_of_bin, c.basis, p.hdr, p.chunk_meta, symbols, grad_out,
                       grad_coeff, p.bwd_part);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !grad_gamma) return (int)e;
  const int64_t nz = 3 * (int64_t)b.n_streams;
  hipLaunchKernelGGL(k_bwd_streams, dim3((unsigned)((nz + 255) / 256)), dim3(256), 0, st, b.n_streams, p.chunk_off,
                     p.chunk_meta, p.bwd_part, grad_gamma);
  return (int)hipGetLastError();
}

}  // namespace fptc
