// Device helpers shared by the matrix-core kernels: 16-bit operand splitting,
// the 32x32x16 MFMA wrappers, and a DPP wavefront scan.
#pragma once

#include <hip/hip_runtime.h>

#include "fptc_internal.h"

namespace fptc {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef uint16_t u8v __attribute__((ext_vector_type(8)));  // 8 raw 16-bit operand values
typedef float f16v __attribute__((ext_vector_type(16)));

constexpr float kBasisScaleF16 = 1024.0f;  // 2^10, undone exactly on the output

template <int PREC>
struct Traits;
template <>
struct Traits<FPTC_FP16> {
  static constexpr int kBPieces = 1, kAPieces = 1;
  static constexpr bool kF16 = true;
};
template <>
struct Traits<FPTC_FP16X2> {
  static constexpr int kBPieces = 2, kAPieces = 2;
  static constexpr bool kF16 = true;
};
template <>
struct Traits<FPTC_BF16> {
  static constexpr int kBPieces = 1, kAPieces = 1;
  static constexpr bool kF16 = false;
};
template <>
struct Traits<FPTC_BF16X3> {
  static constexpr int kBPieces = 3, kAPieces = 3;
  static constexpr bool kF16 = false;
};

// Split x into up to P 16-bit pieces whose sum approximates x.
template <bool F16, int P>
__device__ inline void split(float x, uint16_t *out) {
  float r = x;
#pragma unroll
  for (int i = 0; i < P; ++i) {
    if constexpr (F16) {
      _Float16 h = (_Float16)r;
      out[i] = __builtin_bit_cast(uint16_t, h);
      r -= (float)h;
    } else {
      __bf16 h = (__bf16)r;
      out[i] = __builtin_bit_cast(uint16_t, h);
      r -= (float)h;
    }
  }
}

template <bool F16>
__device__ inline f16v mfma(u8v a, u8v b, f16v acc) {
  // a: 8 basis values (rows n), b: 8 coefficient values (columns w)
  if constexpr (F16)
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(h8, a), __builtin_bit_cast(h8, b), acc, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(b8, a), __builtin_bit_cast(b8, b), acc, 0, 0,
                                                   0);
}

// Dequantize the 8 coefficients of one k-step (bins k0 + j, symbols sy) and
// split each into the precision's 16-bit pieces a[p].  Returns whether any
// lower piece is nonzero (a coefficient not exact in one piece).
//   rb: row of each bin (rb[0 .. E)), tv/tz: value and zone of (row, symbol),
//   g0..g2: the stream's per-zone scales (used when scaled).
// Loads use clamped indices and the value is selected afterwards, so there
// are no per-coefficient branches.
template <int PREC>
__device__ inline bool dequant8(const uint8_t (&sy)[8], int k0, int E, bool valid, const uint8_t *rb, const float *tv,
                                const uint8_t *tz, bool scaled, float g0, float g1, float g2,
                                u8v (&a)[Traits<PREC>::kAPieces]) {
  using T = Traits<PREC>;
  constexpr int AP = T::kAPieces;
  bool rest = false;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int k = k0 + j;
    const int ti = rb[k < E ? k : E - 1] * 256 + sy[j];
    float c = tv[ti];
    if (scaled) {
      const int z = tz[ti];
      c *= z == 0 ? g0 : (z == 1 ? g1 : g2);
    }
    c = (valid && k < E) ? c : 0.0f;
    uint16_t pc[AP];
    split<T::kF16, AP>(c, pc);
#pragma unroll
    for (int p = 0; p < AP; ++p) a[p][j] = pc[p];
#pragma unroll
    for (int p = 1; p < AP; ++p) rest |= (pc[p] & 0x7fff) != 0;
  }
  return rest;
}

// acc[t] += (basis rows of output tile t at this k-step) x (coefficient
// pieces a), smallest terms first.  brow: this lane's basis row of tile 0 at
// the k-step; tiles are tstride halves apart, pieces pstride halves apart.
// Callers run the k-steps from the highest bins down so that the low bins --
// the DC term in particular, often a large offset -- enter the FP32 sums last
// and the partial sums stay small.
template <int PREC, int NT>
__device__ inline void mfma_step(f16v (&acc)[NT], const u8v (&a)[Traits<PREC>::kAPieces], const uint16_t *brow,
                                 int tstride, int pstride, bool any_rest) {
  using T = Traits<PREC>;
  constexpr int BP = T::kBPieces;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    u8v bp[BP];
#pragma unroll
    for (int p = 0; p < BP; ++p) bp[p] = *reinterpret_cast<const u8v *>(brow + t * tstride + p * pstride);
    if constexpr (BP == 3) {
      acc[t] = mfma<T::kF16>(bp[2], a[0], acc[t]);
      if (any_rest) {
        acc[t] = mfma<T::kF16>(bp[1], a[1], acc[t]);
        acc[t] = mfma<T::kF16>(bp[0], a[2], acc[t]);
      }
      acc[t] = mfma<T::kF16>(bp[1], a[0], acc[t]);
      if (any_rest) acc[t] = mfma<T::kF16>(bp[0], a[1], acc[t]);
    } else if constexpr (BP == 2) {
      if (any_rest) acc[t] = mfma<T::kF16>(bp[0], a[1], acc[t]);
      acc[t] = mfma<T::kF16>(bp[1], a[0], acc[t]);
    }
    acc[t] = mfma<T::kF16>(bp[0], a[0], acc[t]);
  }
}

// Stage the split, transposed basis Bs[p][n][k] (row stride RS halves, zero
// for k >= E) from the float basis [E][N]; FP16 pieces are scaled by 2^10.
template <int PREC>
__device__ inline void stage_basis(uint16_t *Bs, const float *basis, int N, int E, int Kp, int RS, int tid,
                                   int nthreads) {
  using T = Traits<PREC>;
  constexpr int BP = T::kBPieces;
  const float bscale = T::kF16 ? kBasisScaleF16 : 1.0f;
  for (int i = tid; i < N * Kp; i += nthreads) {
    const int n = i / Kp, k = i % Kp;
    const float v = k < E ? basis[(int64_t)k * N + n] * bscale : 0.0f;
    uint16_t pc[BP];
    split<T::kF16, BP>(v, pc);
#pragma unroll
    for (int p = 0; p < BP; ++p) Bs[(p * N + n) * RS + k] = pc[p];
  }
}

typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));  // 16 bytes, 4-byte aligned

// Store this lane's results of one 32x32 output block: rows n = nbase + 8 q +
// 4 h + (0..3) of its window, whose samples start at dst; only the first
// `valid` samples of the window exist.  Four consecutive samples leave as one
// 16-byte store (global memory takes them at 4-byte alignment on gfx950).
__device__ inline void store_block(float *dst, const f16v &acc, int nbase, int h, int valid, float scale) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int n0 = nbase + 8 * q + 4 * h;
    const f4u v = {acc[4 * q] * scale, acc[4 * q + 1] * scale, acc[4 * q + 2] * scale, acc[4 * q + 3] * scale};
    if (n0 + 4 <= valid) {
      *reinterpret_cast<f4u *>(dst + n0) = v;
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (n0 + i < valid) dst[n0 + i] = v[i];
    }
  }
}

// Inclusive prefix sum across a 64-lane wavefront with DPP row shifts and row
// broadcasts (no LDS round trips).
__device__ inline int wave_incl_scan_dpp(int x) {
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, true);  // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, true);  // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, true);  // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, true);  // row_shr:8
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15 -> rows 1, 3
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31 -> rows 2, 3
  return x;
}

}  // namespace fptc
