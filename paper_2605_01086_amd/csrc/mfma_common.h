// Device helpers shared by the matrix-core kernels: 16-bit operand splitting,
// the 32x32x16 MFMA wrappers, and a DPP wavefront scan.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

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

// acc[w][n] += sum over the k-step of coef[w][k] * basis[k][n] for a 32-window
// by 32-sample block.  A operand = coefficients (lane l: window l % 32, bins
// of k-slots 8 (l / 32) + j), B operand = basis (lane l: sample l % 32, same
// k-slots).  The result leaves lane l with sample l % 32 of the windows
// acc_window(r, l / 32), r = 0 .. 15, so that a store of one accumulator
// element writes 32 consecutive samples of each of two windows.
template <bool F16>
__device__ inline f16v mfma(u8v basis, u8v coef, f16v acc) {
  if constexpr (F16)
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(h8, coef), __builtin_bit_cast(h8, basis), acc, 0,
                                                  0, 0);
  else
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(b8, coef), __builtin_bit_cast(b8, basis), acc,
                                                   0, 0, 0);
}

// Window (row of the 32 x 32 block) of accumulator element r in lane half h.
__device__ inline int acc_window(int r, int h) { return 8 * (r >> 2) + 4 * h + (r & 3); }

// Dequantize the 8 coefficients of one k-step (bins k0 + KS j, symbols sy) and
// split each into the precision's 16-bit pieces a[p].  MASK: bins may reach
// past E (zero coefficients there); else every bin is below E.  Returns whether any
// lower piece is nonzero (a coefficient not exact in one piece).
//   rb: row of each bin (rb[0 .. E)), tv/tz: value and zone of (row, symbol),
//   g0..g2: the stream's per-zone scales (used when scaled).
// Loads use clamped indices and the value is selected afterwards, so there
// are no per-coefficient branches.
template <int PREC, int KS = 1, bool MASK = true>
__device__ inline bool dequant8(const uint8_t (&sy)[8], int k0, int E, bool valid, const uint8_t *rb, const float *tv,
                                const uint8_t *tz, bool scaled, float g0, float g1, float g2,
                                u8v (&a)[Traits<PREC>::kAPieces]) {
  using T = Traits<PREC>;
  constexpr int AP = T::kAPieces;
  bool rest = false;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int k = k0 + KS * j;
    const int ti = rb[(!MASK || k < E) ? k : E - 1] * 256 + sy[j];
    float c = tv[ti];
    if (scaled) {
      const int z = tz[ti];
      c *= z == 0 ? g0 : (z == 1 ? g1 : g2);
    }
    c = (valid && (!MASK || k < E)) ? c : 0.0f;
    uint16_t pc[AP];
    split<T::kF16, AP>(c, pc);
#pragma unroll
    for (int p = 0; p < AP; ++p) a[p][j] = pc[p];
#pragma unroll
    for (int p = 1; p < AP; ++p) rest |= (pc[p] & 0x7fff) != 0;
  }
  return rest;
}

// FP16 operand range.  Coefficients are split into FP16 pieces, whose range
// ends at 65504, and a table value times a per-zone scale can lie far outside
// it (the paper quantizer's values reach the clipped zone maxima A0 / A1 of
// |c|, in the signal's own units).  So each chunk multiplies its coefficients
// by 2^-e, e chosen from its codebook's largest |value| times its stream's
// largest |scale| so that they lie below 2^15, and its output by 2^e.  A
// power-of-two factor changes no significand and the FP32 sums scale exactly
// with it, so results are those of unscaled arithmetic wherever that stays in
// range.  BF16 shares FP32's exponent range: e = 0.
template <int PREC>
__device__ inline int coef_exp(float vmax) {
  if constexpr (!Traits<PREC>::kF16) {
    return 0;
  } else {
    if (!(vmax > 0.0f) || !(vmax <= 3.0e38f)) return 0;  // zero, NaN or infinite: leave unscaled
    const int e = ((__float_as_int(vmax) >> 23) & 255) - 127 - 14;  // vmax * 2^-e in [2^14, 2^15)
    return e < -100 ? -100 : (e > 100 ? 100 : e);
  }
}
__device__ inline float pow2f(int e) { return __int_as_float((e + 127) << 23); }  // -126 <= e <= 127

// Largest |value| of each codebook's table (vmax[book]): LDS, zeroed, then
// raised by atomicMax on the float bits (non-negative floats order like
// their bit patterns).
__device__ inline void note_table_max(float *vmax, int book, float v) {
  atomicMax(reinterpret_cast<unsigned *>(vmax) + book, __float_as_uint(fabsf(v)));
}

// Table of pre-split dequantized values for the unscaled path (at most two
// pieces): one 32-bit entry per (book, row, symbol), the high piece in the
// low half and the low piece in the high half, exactly what dequant8 would
// produce for that symbol at the book's coefficient exponent (coef_exp of
// vmax[book]).  per_book: entries per codebook.
template <int PREC>
__device__ inline void stage_pieces(uint32_t *pq, const float *deq_val, const float *vmax, int per_book, int n, int tid,
                                    int nthreads) {
  using T = Traits<PREC>;
  constexpr int AP = T::kAPieces;
  static_assert(AP <= 2, "pre-split table holds at most two pieces");
  for (int i = tid; i < n; i += nthreads) {
    uint16_t pc[AP];
    split<T::kF16, AP>(deq_val[i] * pow2f(-coef_exp<PREC>(vmax[i / per_book])), pc);
    pq[i] = (uint32_t)pc[0] | (AP > 1 ? (uint32_t)pc[AP - 1] << 16 : 0u);
  }
}

// Dequantization tables of a workgroup in LDS: value and zone of each (book,
// row, symbol), the row of each bin, the largest |value| per book and, for at
// most two pieces, the pre-split values.
struct DeqTables {
  float *tv;
  uint8_t *tz;
  uint8_t *rb;
  float *vmax;   // [kMaxBooks]
  uint32_t *pq;  // pre-split values (at most two pieces)
};

__host__ __device__ inline size_t deq_table_bytes(int apieces, int n_books, int n_rows, int E) {
  const size_t a = (((size_t)n_books * n_rows * 256 * 5 + (size_t)n_books * E) + 15) & ~(size_t)15;
  return a + 4 * kMaxBooks + (apieces <= 2 ? (size_t)n_books * n_rows * 256 * 4 : 0);
}

__device__ inline DeqTables deq_tables_at(unsigned char *p, int n_books, int n_rows, int E) {
  DeqTables t;
  t.tv = reinterpret_cast<float *>(p);
  t.tz = reinterpret_cast<uint8_t *>(t.tv + n_books * n_rows * 256);
  t.rb = t.tz + n_books * n_rows * 256;
  t.vmax = reinterpret_cast<float *>(p + ((((size_t)n_books * n_rows * 256 * 5 + (size_t)n_books * E) + 15) &
                                          ~(size_t)15));
  t.pq = reinterpret_cast<uint32_t *>(t.vmax + kMaxBooks);
  return t;
}

// Stage the tables (ends with a workgroup barrier).  Zones above 2 read as 2
// and rows past the table as its last row, so corrupt tables index nothing
// outside LDS.
template <int PREC>
__device__ inline void stage_deq_tables(const DeqTables &t, const float *deq_val, const uint8_t *deq_zone,
                                        const uint8_t *row_of_bin, int n_books, int n_rows, int E, int tid,
                                        int nthreads) {
  if (tid < kMaxBooks) t.vmax[tid] = 0.0f;
  __syncthreads();
  const int per_book = n_rows * 256;
  for (int i = tid; i < n_books * per_book; i += nthreads) {
    const float v = deq_val[i];
    t.tv[i] = v;
    const int z = deq_zone[i];
    t.tz[i] = (uint8_t)(z < 2 ? z : 2);
    note_table_max(t.vmax, i / per_book, v);
  }
  for (int i = tid; i < n_books * E; i += nthreads) {
    const int r = row_of_bin[i];
    t.rb[i] = (uint8_t)(r < n_rows ? r : n_rows - 1);
  }
  __syncthreads();
  if constexpr (Traits<PREC>::kAPieces <= 2) stage_pieces<PREC>(t.pq, deq_val, t.vmax, per_book, n_books * per_book, tid, nthreads);
  __syncthreads();
}

// The coefficient factors of a chunk of stream s in codebook `book`:
// per-zone multipliers g0..g2 (the stream's scales, or 1, times 2^-e),
// whether they differ from 1 (scaled), and the output factor oscale * 2^e.
struct ChunkScales {
  float g0, g1, g2, out;
  bool scaled;
};
template <int PREC>
__device__ inline ChunkScales chunk_scales(const float *gamma, float g0, float g1, float g2, float vmax_book,
                                           float oscale) {
  const float gm = gamma ? fmaxf(fabsf(g0), fmaxf(fabsf(g1), fabsf(g2))) : 1.0f;
  const int e = coef_exp<PREC>(gamma ? vmax_book * gm : vmax_book);
  const float f = pow2f(-e);
  ChunkScales c;
  c.g0 = gamma ? g0 * f : f;
  c.g1 = gamma ? g1 * f : f;
  c.g2 = gamma ? g2 * f : f;
  c.scaled = gamma != nullptr || e != 0;
  c.out = oscale * pow2f(e);
  return c;
}

// Coefficient pieces of one k-step without per-stream scales: the 8 symbols
// (s0, s1: byte j is bin k0 + j) looked up in the pre-split table of their
// rows (pq: the book's table; rb: row of each bin when MULTI_ROW) and
// repacked pairwise with byte permutes.  Returns whether any low piece is
// nonzero.  Bins (k0 + KS j) must lie inside [0, E).
template <int PREC, bool MULTI_ROW, int KS = 1>
__device__ inline bool gather8(uint32_t s0, uint32_t s1, int k0, const uint32_t *pq, const uint8_t *rb,
                               u8v (&a)[Traits<PREC>::kAPieces]) {
  using T = Traits<PREC>;
  constexpr int AP = T::kAPieces;
  static_assert(AP <= 2, "pre-split table holds at most two pieces");
  uint32_t t[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const uint32_t sym = ((j < 4 ? s0 : s1) >> (8 * (j & 3))) & 255u;
    const uint32_t row = MULTI_ROW ? (uint32_t)rb[k0 + KS * j] : 0u;
    t[j] = pq[row * 256 + sym];
  }
  uint32_t hi[4], lo[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    hi[i] = __builtin_amdgcn_perm(t[2 * i + 1], t[2 * i], 0x05040100u);
    lo[i] = __builtin_amdgcn_perm(t[2 * i + 1], t[2 * i], 0x07060302u);
  }
  typedef uint32_t u4v __attribute__((ext_vector_type(4)));
  const u4v vh = {hi[0], hi[1], hi[2], hi[3]};
  a[0] = __builtin_bit_cast(u8v, vh);
  if constexpr (AP == 2) {
    const u4v vl = {lo[0], lo[1], lo[2], lo[3]};
    a[1] = __builtin_bit_cast(u8v, vl);
  }
  return AP > 1 && (((lo[0] | lo[1] | lo[2] | lo[3]) & 0x7fff7fffu) != 0);
}

// acc[t] += (basis rows of output tile t at this k-step) x (coefficient
// pieces a), smallest terms first.  brow: this lane's basis row of tile 0 at
// the k-step; tiles are tstride halves apart, pieces pstride halves apart.
// Callers run the k-steps from the highest bins down so that the low bins --
// the DC term in particular, often a large offset -- enter the FP32 sums last
// and the partial sums stay small.  FIRST: acc holds nothing yet, and the
// tile's first product takes a zero accumulator operand (no registers to
// clear beforehand; the same sums).
template <int PREC, int NT, bool FIRST = false>
__device__ inline void mfma_step(f16v (&acc)[NT], const u8v (&a)[Traits<PREC>::kAPieces], const uint16_t *brow,
                                 int tstride, int pstride, bool any_rest) {
  using T = Traits<PREC>;
  constexpr int BP = T::kBPieces;
  const f16v zero = {};
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    u8v bp[BP];
#pragma unroll
    for (int p = 0; p < BP; ++p) bp[p] = *reinterpret_cast<const u8v *>(brow + t * tstride + p * pstride);
    f16v c = FIRST ? zero : acc[t];
    if constexpr (BP == 3) {
      c = mfma<T::kF16>(bp[2], a[0], c);
      if (any_rest) {
        c = mfma<T::kF16>(bp[1], a[1], c);
        c = mfma<T::kF16>(bp[0], a[2], c);
      }
      c = mfma<T::kF16>(bp[1], a[0], c);
      if (any_rest) c = mfma<T::kF16>(bp[0], a[1], c);
    } else if constexpr (BP == 2) {
      if (any_rest) c = mfma<T::kF16>(bp[0], a[1], c);
      c = mfma<T::kF16>(bp[1], a[0], c);
    }
    acc[t] = mfma<T::kF16>(bp[0], a[0], c);
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

// One 32-window tile of a wavefront: acc[t] (output samples t*32 ..) of the
// tile's windows from their symbols at sb[base + bin] in LDS.  k-steps run
// from the highest bins down.  Two forms:
//  * contract_presplit: without scales, with E a multiple of 16 and at most
//    two pieces, coefficients come from the pre-split table pq (MULTI_ROW:
//    with the row lookup, else the book has one row);
//  * contract_dequant: any case, through dequant8.
// Lanes whose window is not valid compute on the clamped window's symbols;
// only their lower-piece flag is masked, so valid columns get exactly the
// general form's arithmetic.  Bs: split basis [piece][n][RS]; rb/tv/tz/pq:
// this book's tables.
template <int PREC, int NT, bool MULTI_ROW>
__device__ inline void contract_presplit(f16v (&acc)[NT], const unsigned char *sb, int base, int h, int col, int S,
                                         bool valid, const uint16_t *Bs, int RS, const uint8_t *rb,
                                         const uint32_t *pq) {
  constexpr int N = NT * 32, AP = Traits<PREC>::kAPieces;
  const int KH = S * 8;
  auto step = [&](int ss, auto first) {
    const int k0 = h * KH + 8 * ss;
    const uint2 u = *reinterpret_cast<const uint2 *>(sb + base + k0);
    u8v a[AP];
    const bool r = gather8<PREC, MULTI_ROW>(u.x, u.y, k0, pq, rb, a);
    const bool any_rest = AP > 1 && __any(r && valid);
    mfma_step<PREC, NT, decltype(first)::value>(acc, a, Bs + col * RS + k0, 32 * RS, N * RS, any_rest);
  };
  step(S - 1, std::true_type{});
#pragma unroll 1
  for (int ss = S - 2; ss >= 0; --ss) step(ss, std::false_type{});
}

template <int PREC, int NT>
__device__ inline void contract_dequant(f16v (&acc)[NT], const unsigned char *sb, int base, int h, int col, int S,
                                        int E, bool valid, const uint16_t *Bs, int RS, const uint8_t *rb,
                                        const float *tv, const uint8_t *tz, bool scaled, float g0, float g1,
                                        float g2) {
  using T = Traits<PREC>;
  constexpr int N = NT * 32;
  constexpr int AP = T::kAPieces;
  const int KH = S * 8;
  const bool e_vec = (E % 16) == 0;
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[t][r] = 0.0f;
#pragma unroll 1
  for (int ss = S - 1; ss >= 0; --ss) {
    const int k0 = h * KH + 8 * ss;
    uint8_t sy[8];
    if (e_vec) {  // the 8-bin group is inside [0, E) and 8-byte aligned
      const uint2 u = *reinterpret_cast<const uint2 *>(sb + base + k0);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        sy[j] = (uint8_t)(u.x >> (8 * j));
        sy[4 + j] = (uint8_t)(u.y >> (8 * j));
      }
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) sy[j] = sb[base + (k0 + j < E ? k0 + j : 0)];
    }
    u8v a[AP];
    const bool r = dequant8<PREC>(sy, k0, E, valid, rb, tv, tz, scaled, g0, g1, g2, a);
    const bool any_rest = AP > 1 && __any(r);
    mfma_step<PREC, NT>(acc, a, Bs + col * RS + k0, 32 * RS, N * RS, any_rest);
  }
}

// Contract a tile with the form that applies and hand the result to emit
// (each form keeps its own accumulators up to the stores).  Without per-stream
// scales the pre-split table already holds the book's coefficient factor.
template <int PREC, int NT, typename Emit>
__device__ inline void tile_contract_emit(const unsigned char *sb, int base, int h, int col, int S, int E, bool valid,
                                          const uint16_t *Bs, int RS, const uint8_t *rb, const float *tv,
                                          const uint8_t *tz, const uint32_t *pq, int n_rows, const float *gamma,
                                          const ChunkScales &cs, Emit &&emit) {
  if constexpr (Traits<PREC>::kAPieces <= 2) {
    if (!gamma && (E % 16) == 0) {
      if (n_rows > 1) {
        f16v acc[NT];
        contract_presplit<PREC, NT, true>(acc, sb, base, h, col, S, valid, Bs, RS, rb, pq);
        emit(acc);
      } else {
        f16v acc[NT];
        contract_presplit<PREC, NT, false>(acc, sb, base, h, col, S, valid, Bs, RS, rb, pq);
        emit(acc);
      }
      return;
    }
  }
  f16v acc[NT];
  contract_dequant<PREC, NT>(acc, sb, base, h, col, S, E, valid, Bs, RS, rb, tv, tz, cs.scaled, cs.g0, cs.g1, cs.g2);
  emit(acc);
}

typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));  // 16 bytes, 4-byte aligned

// Order a wavefront's LDS writes before its later LDS reads by other lanes.
__device__ inline void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

typedef float f4a __attribute__((ext_vector_type(4)));  // 16 bytes, 16-byte aligned

// Store a whole 32-window tile through LDS so that global memory sees
// contiguous, 16-byte aligned 16-byte stores.  The tile's windows are
// consecutive in one stream: win0 is the first sample of window 0 and rem
// the samples from there to the end of the tile's data.  Eight windows (a
// quarter, 8 N floats) at a time are scattered into `stage` in output order,
// shifted by the output's misalignment (0..3 floats), then read back as
// aligned 16-byte vectors, each lane writing whole 16-byte blocks (the
// floats of partial blocks at the quarter's ends spread over lanes 0..7 and
// written by one store instruction).  stage must be 16-byte
// aligned with 8 N + 4 floats of room (the caller passes its consumed symbol
// buffer, starting 16 bytes into the prefix before it).
template <int NT>
__device__ inline void store_tile_staged(float *win0, const f16v (&acc)[NT], float *stage, int h, int col, int lane,
                                         int rem, float scale) {
  constexpr int N = NT * 32, QF = 8 * N;
  const int delta = (int)((reinterpret_cast<uintptr_t>(win0) >> 2) & 3);
#pragma unroll 1
  for (int q = 0; q < 4; ++q) {
    const int qrem = rem - q * QF;  // wave-uniform
    if (qrem <= 0) break;
    const int qn = qrem < QF ? qrem : QF;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int j = 0; j < 4; ++j) stage[delta + (4 * h + j) * N + 32 * t + col] = acc[t][4 * q + j] * scale;
    wave_sync_lds();
    float *g = win0 + q * QF - delta;  // 16-byte aligned
    const int nvec = (qn + delta + 3) >> 2;
    // whole 16-byte blocks: every vector but possibly the first and the last
    for (int m = lane; m < nvec; m += 64) {
      const int i0 = 4 * m - delta;  // quarter-relative index of the block's first float
      if (i0 >= 0 && i0 + 4 <= qn) *reinterpret_cast<f4a *>(g + 4 * m) = *reinterpret_cast<const f4a *>(stage + 4 * m);
    }
    // the floats of a partial first or last block, one per lane (lanes 0..7),
    // so that they leave as a single store instruction
    if (lane < 8) {
      const int m = lane < 4 ? 0 : nvec - 1;
      const int i0 = 4 * m - delta, e = i0 + (lane & 3);
      const bool whole = i0 >= 0 && i0 + 4 <= qn;
      if (!whole && (lane < 4 || nvec > 1) && e >= 0 && e < qn) g[4 * m + (lane & 3)] = stage[4 * m + (lane & 3)];
    }
    wave_sync_lds();
  }
}

// Store a whole 32-window tile (rem >= 32 N) through LDS.  The quarters are
// cut on the output's 16-byte grid instead of at window boundaries: quarter q
// stages tile floats [q QF - delta, (q + 1) QF - delta), which takes in the
// last delta floats of quarter q - 1's windows.  Every block inside the tile
// is then whole and leaves with one 16-byte store; only the tile's first and
// last blocks are partial, and their floats (at most 3 + 3) leave together,
// one per lane, after the last quarter.  The whole blocks are non-temporal
// stores: each instruction writes 1 KB of whole 64-byte lines, so nothing has
// to be combined in L2, and the stream does not displace cached data.  Same
// stage buffer as store_tile_staged.
template <int NT>
__device__ inline void store_tile_whole(float *win0, const f16v (&acc)[NT], float *stage, int h, int col, int lane,
                                        float scale) {
  constexpr int N = NT * 32, QF = 8 * N, NV = QF / 256;  // NV: 16-byte vectors per lane per quarter
  const int delta = (int)((reinterpret_cast<uintptr_t>(win0) >> 2) & 3);
  float *const g0 = win0 - delta;  // 16-byte aligned
  float edge = 0.0f;  // lanes 4..7: block 0 of the tile; lanes 0..3: the floats past the last whole block
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    // this quarter's windows; their floats past index QF belong to the next
    // quarter (which writes them again) or, for the last, to the tail block
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int j = 0; j < 4; ++j) stage[delta + (4 * h + j) * N + 32 * t + col] = acc[t][4 * q + j] * scale;
    // the end of the previous quarter's last window (row 7, last delta samples)
    if (q > 0 && h == 1 && col >= 32 - delta) stage[col - 32 + delta] = acc[NT - 1][4 * q - 1] * scale;
    wave_sync_lds();
    float *g = g0 + q * QF;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const int m = lane + 64 * k;
      if (q > 0 || m > 0 || delta == 0)  // block 0 of a misaligned tile is partial
        __builtin_nontemporal_store(*reinterpret_cast<const f4a *>(stage + 4 * m), reinterpret_cast<f4a *>(g + 4 * m));
    }
    if (q == 0 && lane >= 4 && lane < 8) edge = stage[lane - 4];
    if (q == 3 && lane < 4) edge = stage[QF + lane];
    wave_sync_lds();
  }
  const bool tail = lane < delta, head = delta > 0 && lane >= 4 + delta && lane < 8;
  if (tail || head) g0[(tail ? 4 * QF : -4) + lane] = edge;
}

// Store output tile t (samples 32 t .. 32 t + 31 of every window) of a block
// of up to 32 consecutive windows of one stream: win0 = first sample of the
// block's window 0, rem = samples from there to the end of the block (window
// w holds samples [w N, w N + N) of it).  Lane (col, h) writes sample 32 t +
// col of its 16 windows; each instruction covers two 128-byte runs.
__device__ inline void store_rows(float *win0, int N, const f16v &acc, int t, int h, int col, int rem, float scale) {
  // offset of element r = lane part (window 4 h, sample 32 t + col) + a part
  // common to the wave, so each bound check is one compare with a scalar
  const int lane_off = 4 * h * N + 32 * t + col;
  float *p = win0 + lane_off;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int c = acc_window(r, 0) * N;
    if (lane_off < rem - c) p[c] = acc[r] * scale;
  }
}


// Chunk records (and per-stream scales) are read with vector loads, one dword
// per lane, then moved to scalar registers with readlane.  A scalar load
// would share its wait counter with LDS accesses and return out of order, so
// the first LDS wait after it -- the decode loop's first lookup -- would stall
// for the load's whole memory latency.  Vector loads retire in order with the
// word loads and are waited for together with them.
// Lanes 0..15: the dwords of record c; lanes 16..18: the first word and
// first symbol of record c + 1 (all ones when there is none).
__device__ inline uint32_t load_meta_lane(const ChunkMeta *meta, int64_t c, int64_t n, int lane) {
  if (c >= n || lane >= 19) return 0u;
  if (lane >= 16 && c + 1 >= n) return 0xffffffffu;
  return reinterpret_cast<const uint32_t *>(meta + c)[lane];
}
// The record whose dwords lanes 0..18 hold (load_meta_lane), its word_end
// resolved from the next record unless it is its stream's last chunk or the
// next chunk has no start; valid = false (no record) gives first_word = -1
// and no windows.
__device__ inline ChunkMeta meta_from_lanes(uint32_t d, bool valid) {
  uint32_t w[19];
#pragma unroll
  for (int i = 0; i < 19; ++i) w[i] = __builtin_amdgcn_readlane(d, i);
  ChunkMeta m;
  __builtin_memcpy(&m, w, sizeof(m));
  const int64_t nfw = (int64_t)(((uint64_t)w[17] << 32) | w[16]);
  if (!m.last && nfw >= 0) m.word_end = nfw + ((int32_t)w[18] < 0 ? 1 : 0);
  if (!valid) {
    m.first_word = -1;
    m.n_windows = 0;
  }
  return m;
}
// Chunk schedule of a persistent workgroup: in each of its rounds it takes
// per_round chunks, base + j step (j < per_round), the rounds `stride` chunks
// apart, in increasing order, handed out one at a time through a counter in
// LDS.  step 1 keeps a round's chunks adjacent (neighbouring output and
// input); step = the number of workgroups draws them from many streams, so
// that the rounds' costs even out across workgroups; small rounds of adjacent
// chunks do both.  A SIMD's arbiter favours its older waves, so with a fixed
// share per wave the younger ones fall behind and finish last while the older
// ones leave their SIMDs half empty; with the shared counter a wave takes the
// next chunk whenever it is ready.  Indices only grow, so a wave stops at the
// first one past the end.
struct BlockChunks {
  unsigned *ctr;  // LDS, zeroed before the loop
  int64_t base, stride, step;
  int per_round;
  __device__ int64_t next(int lane) const {
    unsigned t = 0;
    if (lane == 0) t = atomicAdd(ctr, 1u);
    t = __builtin_amdgcn_readfirstlane(t);
    return base + (int64_t)(t % (unsigned)per_round) * step + (int64_t)(t / (unsigned)per_round) * stride;
  }
};

// gamma[3 s + lane] in lanes 0..2 (1 without scales).
__device__ inline float load_gamma_lane(const float *gamma, int s, int lane) {
  return (gamma && lane < 3) ? gamma[3 * (int64_t)s + lane] : 1.0f;
}
__device__ inline float lane_float(float v, int i) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), i));
}
// Wait for a lane-loaded value here (see settle_chunk_words).
__device__ inline void settle_lane(uint32_t d) { asm volatile("" ::"v"(d) : "memory"); }
__device__ inline void settle_lane(float d) { asm volatile("" ::"v"(d) : "memory"); }

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
