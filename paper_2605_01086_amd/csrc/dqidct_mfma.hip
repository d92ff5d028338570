// Dequantization fused with the inverse DCT on the matrix cores (Section 4.2,
// lossy stage, as a dense contraction).
//
// For a tile of 32 consecutive windows (global numbering) one wavefront forms
//     D[n][w] = sum_k B[k][n] * c[w][k]
// i.e. the transposed product basis^T x coefficients^T, with
// v_mfma_f32_32x32x16_{f16,bf16}: FP32 accumulation, 16-bit operands.  The
// transposed form leaves each lane holding four consecutive samples of one
// window, so the result leaves as 16-byte stores straight from registers.
//
// Bins are mapped to MFMA k-slots so that each lane's coefficients are one
// contiguous run of symbols: lane half h owns bins [h*Kp/2, (h+1)*Kp/2), k-step
// s covers the 8 bins h*Kp/2 + 8 s + j.  The basis operand uses the same map.
//
// FP32-level accuracy comes from splitting operands into 16-bit pieces:
//   FP16X2: basis = hi + lo (scaled by 2^10 so lo stays out of the FP16
//           subnormal range); a coefficient that is not exact in FP16 (any
//           per-zone scale != 1) is split too, and the pass with its lo piece
//           is skipped when every lane's lo piece is zero.
//   BF16X3: basis = hi + mid + lo in BF16, coefficients likewise.
// The basis pieces live in LDS (rows padded by 16 bytes to spread banks); the
// dequantization tables live in LDS; coefficients are dequantized in registers
// straight from the decoded symbols.
#include <hip/hip_runtime.h>

#include "fptc_internal.h"
#include "mfma_common.h"

namespace fptc {
namespace {

constexpr int kThreads = 256;

// LDS bytes of one instantiation: basis pieces and tables.
__host__ __device__ constexpr size_t mfma_lds_bytes(int bpieces, int N, int Kp, int n_books, int n_rows, int E) {
  return (size_t)bpieces * N * (Kp + 8) * 2 + (size_t)n_books * n_rows * 256 * 5 + (size_t)n_books * E + 16;
}

// NT = N / 32 output row tiles; S = Kp / 16 k-steps (Kp = E rounded up to 16).
template <int PREC, int NT>
__global__ void __launch_bounds__(kThreads) k_dqidct_mfma(fptc_batch b, int E, int S, int n_books, int n_rows,
                                                          const float *deq_val, const uint8_t *deq_zone,
                                                          const uint8_t *row_of_bin, const float *basis,
                                                          const int64_t *hdr, const int64_t *win_off,
                                                          const int32_t *tile_stream, const uint8_t *symbols,
                                                          const float *gamma, float *out) {
  using T = Traits<PREC>;
  constexpr int N = NT * 32;
  const int Kp = S * 16, KH = Kp / 2;
  const int RS = Kp + 8;  // LDS row stride of a basis piece, in halves
  constexpr int BP = T::kBPieces, AP = T::kAPieces;
  extern __shared__ __align__(16) unsigned char lds[];
  uint16_t *Bs = reinterpret_cast<uint16_t *>(lds);                         // [BP][N][RS]
  float *Tv = reinterpret_cast<float *>(lds + (size_t)BP * N * RS * 2);      // [books][rows][256]
  uint8_t *Tz = reinterpret_cast<uint8_t *>(Tv + n_books * n_rows * 256);    // [books][rows][256]
  uint8_t *Rb = Tz + n_books * n_rows * 256;                                 // [books][E]

  // Stage the split basis (transposed to [n][k], zero beyond E) and the tables.
  const float bscale = T::kF16 ? kBasisScaleF16 : 1.0f;
  stage_basis<PREC>(Bs, basis, N, E, Kp, RS, threadIdx.x, kThreads);
  for (int i = threadIdx.x; i < n_books * n_rows * 256; i += kThreads) {
    Tv[i] = deq_val[i];
    const int z = deq_zone[i];
    Tz[i] = (uint8_t)(z < 2 ? z : 2);
  }
  for (int i = threadIdx.x; i < n_books * E; i += kThreads) {
    const int r = row_of_bin[i];
    Rb[i] = (uint8_t)(r < n_rows ? r : n_rows - 1);
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, col = lane & 31, h = lane >> 5;
  const int wid = threadIdx.x >> 6;
  const int64_t n_win = hdr[1];
  const int64_t n_tiles = (n_win + kTileWindows - 1) / kTileWindows;
  const int64_t stride = (int64_t)gridDim.x * (kThreads / 64);
  const float oscale = 1.0f / bscale;
  const bool e_vec = (E % 16) == 0 && (reinterpret_cast<uintptr_t>(symbols) & 7) == 0;

  for (int64_t tile = (int64_t)blockIdx.x * (kThreads / 64) + wid; tile < n_tiles; tile += stride) {
    // ---- window of this lane's column
    const int64_t g = tile * kTileWindows + col;
    int valid = 0, book = 0;
    int64_t obase = 0;
    float gz0 = 1.0f, gz1 = 1.0f, gz2 = 1.0f;
    if (g < n_win) {
      int s = tile_stream[tile];
      s = s < 0 ? 0 : (s >= b.n_streams ? b.n_streams - 1 : s);
      while (s + 1 < b.n_streams && win_off[s + 1] <= g) ++s;
      const int64_t j = g - win_off[s];
      const int64_t L = b.sample_off[s + 1] - b.sample_off[s];
      const int64_t o = b.sample_off[s] + j * N;
      int64_t v = L - j * N;
      v = v < N ? v : N;
      if (o < 0 || o + v > b.n_samples || j < 0) v = 0;
      valid = v > 0 ? (int)v : 0;
      obase = o;
      const int bk = b.book_id ? (int)b.book_id[s] : 0;
      book = bk < n_books ? bk : 0;
      if (gamma) {
        gz0 = gamma[3 * (int64_t)s];
        gz1 = gamma[3 * (int64_t)s + 1];
        gz2 = gamma[3 * (int64_t)s + 2];
      }
    }
    // ---- contraction, one k-step at a time from the highest bins down
    f16v acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[t][r] = 0.0f;
    const int64_t sbase = g * (int64_t)E + h * KH;
#pragma unroll 1
    for (int s = S - 1; s >= 0; --s) {
      const int k0 = h * KH + 8 * s;
      uint8_t sy[8];
      if (valid > 0 && e_vec && sbase + 8 * s + 8 <= b.n_symbols) {
        const uint2 u = *reinterpret_cast<const uint2 *>(symbols + sbase + 8 * s);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          sy[j] = (uint8_t)(u.x >> (8 * j));
          sy[4 + j] = (uint8_t)(u.y >> (8 * j));
        }
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int64_t si = sbase + 8 * s + j;
          sy[j] = (valid > 0 && k0 + j < E && si < b.n_symbols) ? symbols[si] : (uint8_t)128;
        }
      }
      u8v a[AP];
      const bool r = dequant8<PREC>(sy, k0, E, valid > 0, Rb + book * E, Tv + book * n_rows * 256,
                                    Tz + book * n_rows * 256, gamma != nullptr, gz0, gz1, gz2, a);
      const bool any_rest = AP > 1 && __any(r);
      mfma_step<PREC, NT>(acc, a, Bs + col * RS + k0, 32 * RS, N * RS, any_rest);
    }
    // lane holds rows n = t*32 + 8*q + 4*h + (0..3) of its window
    if (valid > 0) {
#pragma unroll
      for (int t = 0; t < NT; ++t) store_block(out + obase, acc[t], t * 32, h, valid, oscale);
    }
  }
}

template <int PREC, int NT>
int launch_t(const fptc_batch &b, const fptc_codec &c, const Shape &sh, const Plan &p, const uint8_t *symbols,
             const float *gamma, float *out, void *stream) {
  constexpr int N = NT * 32;
  const int S = (c.E + 15) / 16, Kp = S * 16;
  const size_t lds = mfma_lds_bytes(Traits<PREC>::kBPieces, N, Kp, c.n_books, c.n_rows, c.E);
  auto kern = k_dqidct_mfma<PREC, NT>;
  static bool attr_set = false;  // one attribute call per instantiation
  if (!attr_set) {
    if (hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024) != hipSuccess)
      return (int)hipErrorInvalidValue;
    attr_set = true;
  }
  const int per_cu = (int)((160 * 1024) / lds);
  int blocks = sh.blocks > 0 ? sh.blocks : device_cu_count() * (per_cu < 1 ? 1 : (per_cu > 8 ? 8 : per_cu));
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(kThreads), lds, (hipStream_t)stream, b, c.E, S, c.n_books, c.n_rows,
                     c.deq_val, c.deq_zone, c.row_of_bin, c.basis, p.hdr, p.win_off, p.tile_stream, symbols, gamma,
                     out);
  return (int)hipGetLastError();
}

template <int PREC>
int launch_prec(const fptc_batch &b, const fptc_codec &c, const Shape &sh, const Plan &p, const uint8_t *symbols,
                const float *gamma, float *out, void *stream) {
  switch (c.N) {
    case 32: return launch_t<PREC, 1>(b, c, sh, p, symbols, gamma, out, stream);
    case 64: return launch_t<PREC, 2>(b, c, sh, p, symbols, gamma, out, stream);
    case 128: return launch_t<PREC, 4>(b, c, sh, p, symbols, gamma, out, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

}  // namespace

bool mfma_supported(int N, int E, int precision) {
  if (precision < FPTC_FP16 || precision > FPTC_BF16X3) return false;
  if (N != 32 && N != 64 && N != 128) return false;
  if (E < 1 || E > N) return false;
  // LDS: basis pieces + tables must fit in 160 KB (staging is optional)
  const int Kp = (E + 15) / 16 * 16;
  const int pieces = precision == FPTC_BF16X3 ? 3 : (precision == FPTC_FP16X2 ? 2 : 1);
  return mfma_lds_bytes(pieces, N, Kp, kMaxBooks, kMaxRows, E) <= 160 * 1024;
}

int launch_dqidct_mfma(const fptc_batch &b, const fptc_codec &c, const Shape &s, const Plan &p,
                       const uint8_t *symbols, const float *gamma, int precision, float *out, void *stream) {
  switch (precision) {
    case FPTC_FP16: return launch_prec<FPTC_FP16>(b, c, s, p, symbols, gamma, out, stream);
    case FPTC_FP16X2: return launch_prec<FPTC_FP16X2>(b, c, s, p, symbols, gamma, out, stream);
    case FPTC_BF16: return launch_prec<FPTC_BF16>(b, c, s, p, symbols, gamma, out, stream);
    case FPTC_BF16X3: return launch_prec<FPTC_BF16X3>(b, c, s, p, symbols, gamma, out, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

}  // namespace fptc
