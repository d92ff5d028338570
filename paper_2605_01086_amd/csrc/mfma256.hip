// Window 256 on the matrix cores (Section 4.2 lossy stage, Eq. 1 inverted).
//
// The inverse DCT rows obey B[k][N-1-n] = (-1)^k B[k][n].  With
//     E[w][n] = sum over even bins k of c[w][k] B[k][n],
//     O[w][n] = sum over odd bins  k of c[w][k] B[k][n],      n < 128,
// the samples are x[w][n] = E + O and x[w][255 - n] = E - O: two 128 x 128
// contractions instead of one 256 x 256, half the matrix-core work and half
// the basis.
//
// A workgroup has 8 waves.  Wave w owns parity p = w / 4 (even or odd bins)
// and the 32 output columns n = 32 (w % 4) + lane % 32 of the half; its slice
// of the split basis (up to 8 k-steps x the precision's 16-bit pieces) is
// loaded into registers once and never restaged.  Work comes in rounds of 8
// chunks (runs of up to wpc windows of one stream, from the plan):
//   1. each wave puts one chunk's symbols into its LDS buffer: the fused
//      kernel decodes them from the words (the same per-chunk decode as the
//      other fused kernel), the split kernel copies them from the symbol
//      array;
//   2. for every 32-window tile of the round's chunks, each wave contracts its
//      parity's dequantized coefficients of the tile's windows with its basis
//      slice on v_mfma_f32_32x32x16 (coefficients as the A operand), the even
//      and odd waves of a column tile swap their partial sums through LDS,
//      and the even wave writes x[n] = E + O, the odd wave x[255 - n] = E - O:
//      each store instruction writes 32 consecutive samples of two windows.
// Both kernels run the same contraction code, so their outputs are
// bit-identical.  The words of the next round are requested before the
// contraction and waited for before its first store; vector memory counters
// retire in order, so a later wait would also wait for the stores.
#include <hip/hip_runtime.h>

#include "decode_common.h"
#include "fptc_internal.h"
#include "mfma_common.h"

namespace fptc {
namespace {

constexpr int N256 = 256;
constexpr int kWaves256 = 8;
constexpr int kMaxSteps = 8;      // k-steps of 16 bins of one parity (128 bins)
constexpr int kPre256 = 12;       // rounds of 64 words requested a round ahead (768 words)
constexpr int kSymVec = 8;        // 16-byte symbol vectors per lane requested a round ahead (8 KB)
// Exchange buffer of a tile: the even waves' sums E[w][n] then the odd waves'
// O[w][n], 32 windows x 128 columns each, rows padded to 132 floats (so the
// two window rows a store of one accumulator element touches fall in
// different banks, and rows stay 16-byte aligned).
constexpr int kXRow = 132;
constexpr int kXchBytes = 2 * kTileWindows * kXRow * 4;
// Shared coefficient operands of a tile (one piece): for parity p, k-step s
// and lane l, the 8 halves lane l feeds the MFMA, at ((p * 8 + s) * 64 + l) * 16.
constexpr int kFrags = 2 * kMaxSteps * 64;
constexpr int kAfragBytes = kFrags * 16;

__host__ __device__ constexpr size_t a16(size_t x) { return (x + 15) & ~(size_t)15; }

// Per-wave symbol buffer: a prefix for symbols of the word before the chunk
// (decode), the chunk's symbols, and 256 bytes of slack: the contraction reads
// 256 bytes from the start of every window whatever E is.
__host__ __device__ inline size_t wave256_bytes(int wpc, int E) { return (size_t)kSymPrefix + a16((size_t)wpc * E + 256); }

// What every wave needs of each chunk of the round, written by its owner.
struct Slot {
  int64_t out_base;  // first output sample
  int32_t out_len;   // samples of the chunk
  int32_t n_win;     // windows (0: nothing to do)
  int32_t book;
  int32_t scaled;
  float g0, g1, g2, oscale;  // coefficient factors per zone, output factor (ChunkScales)
  int32_t pad[2];
};
static_assert(sizeof(Slot) == 48, "slot size");

// LDS: [decode tables] | dequantization tables | slots | exchange buffers |
// [shared coefficient operands] | wave symbol buffers.  The multi-symbol table build borrows lut1_temp_bytes
// right after the decode tables.
__host__ __device__ inline size_t w256_lds(bool fused, bool ms, int ap, int n_books, int n_rows, int lmax, int E,
                                           int wpc, int nxb, bool sh) {
  const size_t t = fused ? lut_lds_bytes(ms, n_books, lmax) : 0;
  const size_t need = t + a16(deq_table_bytes(ap, n_books, n_rows, E)) + kWaves256 * sizeof(Slot) +
                      (size_t)nxb * kXchBytes + (sh ? (size_t)ap * kAfragBytes + 16 : 0) +
                      kWaves256 * wave256_bytes(wpc, E);
  const size_t tmp = (fused && ms && lmax <= kShortLmax) ? t + lut1_temp_bytes(n_books, lmax) : 0;
  return need > tmp ? need : tmp;
}

// The 8 bytes of parity p (bytes p, p + 2, ..., p + 14) of a 16-byte group.
__device__ inline uint2 parity_bytes(uint4 u, int p) {
  const uint32_t sel = p ? 0x07050301u : 0x06040200u;
  return make_uint2(__builtin_amdgcn_perm(u.y, u.x, sel), __builtin_amdgcn_perm(u.w, u.z, sel));
}

// c += basis pieces x coefficient pieces for one k-step, smallest terms first
// (the order of mfma_step).
template <int PREC>
__device__ inline f16v mfma_pieces(const u8v (&bp)[Traits<PREC>::kBPieces], const u8v (&a)[Traits<PREC>::kAPieces],
                                   f16v c, bool any_rest) {
  using T = Traits<PREC>;
  constexpr int BP = T::kBPieces;
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
  return mfma<T::kF16>(bp[0], a[0], c);
}

// This wave's basis slice: for k-step s, lane (col, h) holds bins
// 2 (64 h + 8 s + j) + p, j < 8, at column n0 + col, split into pieces (FP16
// pieces scaled by 2^10); zero past E.
template <int PREC>
__device__ inline void load_basis_slice(u8v (&bv)[kMaxSteps][Traits<PREC>::kBPieces], const float *__restrict__ basis,
                                        int E, int p, int n0, int col, int h) {
  using T = Traits<PREC>;
  constexpr int BP = T::kBPieces;
  const float bscale = T::kF16 ? kBasisScaleF16 : 1.0f;
#pragma unroll
  for (int s = 0; s < kMaxSteps; ++s) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = 2 * (64 * h + 8 * s + j) + p;
      const float v = k < E ? basis[(int64_t)k * N256 + n0 + col] * bscale : 0.0f;
      uint16_t pc[BP];
      split<T::kF16, BP>(v, pc);
#pragma unroll
      for (int q = 0; q < BP; ++q) bv[s][q][j] = pc[q];
    }
  }
}

// Coefficient forms of a kernel: the pre-split table with one or several
// table rows (no per-stream scales, E = 256, at most two pieces), the general
// dequantization with every bin kept (E = 256), or with bins past E masked.
enum { kFormPresplit1 = 0, kFormPresplitRows = 1, kFormDequant = 2, kFormDequantE = 3 };

// The 8 coefficient pieces of k-step s for parity p of one window (row: its
// symbols from bin 128 h on), as dequant8 / gather8 make them for the
// contraction; returns whether a lower piece is nonzero (valid windows only).
template <int PREC, int FORM>
__device__ inline bool coef_frag(const unsigned char *row, int p, int s, int h, int E, bool valid, bool e_vec,
                                 const uint8_t *rb, const float *tv, const uint8_t *tz, const uint32_t *pq, bool scaled,
                                 float g0, float g1, float g2, u8v (&a)[Traits<PREC>::kAPieces]) {
  uint2 u;
  if (FORM != kFormDequantE || e_vec) {
    u = parity_bytes(*reinterpret_cast<const uint4 *>(row + 16 * s), p);
  } else {
    uint32_t w[2] = {0u, 0u};
#pragma unroll
    for (int j = 0; j < 8; ++j) w[j >> 2] |= (uint32_t)row[p + 16 * s + 2 * j] << (8 * (j & 3));
    u = make_uint2(w[0], w[1]);
  }
  const int k0 = 128 * h + p + 16 * s;
  if constexpr (FORM == kFormPresplit1 || FORM == kFormPresplitRows) {
    return gather8<PREC, FORM == kFormPresplitRows, 2>(u.x, u.y, k0, pq, rb, a) && valid;
  } else {
    uint8_t sy[8];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      sy[j] = (uint8_t)(u.x >> (8 * j));
      sy[4 + j] = (uint8_t)(u.y >> (8 * j));
    }
    return dequant8<PREC, 2, FORM == kFormDequantE>(sy, k0, E, valid, rb, tv, tz, scaled, g0, g1, g2, a);
  }
}

// Partial sums of one parity for a 32-window tile: lane (col, h) supplies the
// coefficients of window `col`, whose symbols start at sbw (bins 128 h + 16 s
// + 2 j + p for k-step s); the result leaves lane (col, h) with column n0 +
// col of windows acc_window(r, h).  All 8 k-steps run, from the highest bins
// down, the odd and even ones into two accumulators added at the end (the
// order of the shared form, so both forms give the same sums); bins past E
// have a zero basis row and a zero coefficient.  The
// symbol buffer holds at least 256 bytes past the start of any window, so
// every read stays inside it.
template <int PREC, int FORM>
__device__ inline f16v contract_parity(const u8v (&bv)[kMaxSteps][Traits<PREC>::kBPieces], const unsigned char *sbw,
                                       int p, int h, int E, bool valid, bool e_vec, const uint8_t *rb,
                                       const float *tv, const uint8_t *tz, const uint32_t *pq, bool scaled, float g0,
                                       float g1, float g2) {
  using T = Traits<PREC>;
  constexpr int AP = T::kAPieces;
  const unsigned char *row = sbw + 128 * h;   // this lane's symbols, 16-byte aligned when e_vec
  const int kh = 128 * h + p;                 // bin of step 0, j = 0
  f16v acc0 = {}, acc1 = {};                  // even and odd k-steps (the shared form's chains)
#pragma unroll
  for (int s = kMaxSteps - 1; s >= 0; --s) {
    uint2 u;
    if (FORM != kFormDequantE || e_vec) {
      u = parity_bytes(*reinterpret_cast<const uint4 *>(row + 16 * s), p);
    } else {
      uint32_t w[2] = {0u, 0u};
#pragma unroll
      for (int j = 0; j < 8; ++j) w[j >> 2] |= (uint32_t)row[p + 16 * s + 2 * j] << (8 * (j & 3));
      u = make_uint2(w[0], w[1]);
    }
    u8v a[AP];
    bool r;
    if constexpr (FORM == kFormPresplit1 || FORM == kFormPresplitRows) {
      r = gather8<PREC, FORM == kFormPresplitRows, 2>(u.x, u.y, kh + 16 * s, pq, rb, a) && valid;
    } else {
      uint8_t sy[8];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        sy[j] = (uint8_t)(u.x >> (8 * j));
        sy[4 + j] = (uint8_t)(u.y >> (8 * j));
      }
      r = dequant8<PREC, 2, FORM == kFormDequantE>(sy, kh + 16 * s, E, valid, rb, tv, tz, scaled, g0, g1, g2, a);
    }
    const bool any_rest = AP > 1 && __any(r);
    if (s & 1)
      acc1 = mfma_pieces<PREC>(bv[s], a, acc1, any_rest);
    else
      acc0 = mfma_pieces<PREC>(bv[s], a, acc0, any_rest);
  }
  return acc1 + acc0;
}

template <int PREC, bool FUSED, bool MS, int FORM, bool SH>
__global__ void __launch_bounds__(kWaves256 * 64) k_w256(const uint64_t *__restrict__ words,
                                                        const uint8_t *__restrict__ symlen,
                                                        const uint8_t *__restrict__ symbols, int64_t n_symbols,
                                                        int n_streams, int E, int lmax, int n_books, int n_rows,
                                                        int wpc, int nxb, const uint16_t *__restrict__ lut_g,
                                                        const float *__restrict__ deq_val,
                                                        const uint8_t *__restrict__ deq_zone,
                                                        const uint8_t *__restrict__ row_of_bin,
                                                        const float *__restrict__ basis,
                                                        const int64_t *__restrict__ hdr,
                                                        const ChunkMeta *__restrict__ meta,
                                                        const float *__restrict__ gamma, float *out, int32_t *status) {
  using T = Traits<PREC>;
  constexpr int AP = T::kAPieces, BP = T::kBPieces;
  extern __shared__ __align__(16) unsigned char lds[];
  const size_t lut_bytes = FUSED ? lut_lds_bytes(MS, n_books, lmax) : 0;
  unsigned char *tables = lds + lut_bytes;
  const DeqTables dt = deq_tables_at(tables, n_books, n_rows, E);
  Slot *slots = reinterpret_cast<Slot *>(tables + a16(deq_table_bytes(AP, n_books, n_rows, E)));
  float *xch = reinterpret_cast<float *>(slots + kWaves256);
  u8v *afrag = reinterpret_cast<u8v *>(reinterpret_cast<unsigned char *>(xch) + (size_t)nxb * kXchBytes);
  // two words: whether tile t (slot t % 2) has a nonzero lower piece
  unsigned *tflag = reinterpret_cast<unsigned *>(afrag + (SH ? AP * kFrags : 0));
  unsigned char *wave_base = reinterpret_cast<unsigned char *>(afrag) + (SH ? (size_t)AP * kAfragBytes + 16 : 0);

  if constexpr (FUSED) stage_decode_tables(MS, lds, lds + lut_bytes, lut_g, lmax, n_books, threadIdx.x, blockDim.x);
  stage_deq_tables<PREC>(dt, deq_val, deq_zone, row_of_bin, n_books, n_rows, E, threadIdx.x, blockDim.x);
  if (SH && threadIdx.x < 2) tflag[threadIdx.x] = 0;
  __syncthreads();

  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63, col = lane & 31, h = lane >> 5;
  const int p = wid >> 2, ct = wid & 3;
  const int n0 = 32 * ct;
  unsigned char *const sb_own = wave_base + (size_t)wid * wave256_bytes(wpc, E) + kSymPrefix;
  const float oscale = 1.0f / (T::kF16 ? kBasisScaleF16 : 1.0f);
  const bool e_vec = (E % 16) == 0;
  const bool sym_vec = e_vec && (reinterpret_cast<uintptr_t>(symbols) & 15) == 0;
  const int64_t n_chunks = hdr[0];
  const int64_t rstride = (int64_t)gridDim.x * kWaves256;

  u8v bv[kMaxSteps][BP];
  load_basis_slice<PREC>(bv, basis, E, p, n0, col, h);

  const uint8_t *cl = FUSED ? lds + ((size_t)n_books << lmax) * 4 : nullptr;
  const uint32_t *binfo = FUSED ? reinterpret_cast<const uint32_t *>(cl + n_books * 256) : nullptr;
  const int hs = 32 - lmax;

  // this wave's chunk of the first round, its words (or symbols), and the
  // record of its chunk in the next round
  int64_t c = (int64_t)blockIdx.x * kWaves256 + wid;
  ChunkMeta cm = meta_from_lanes(load_meta_lane(meta, c, n_chunks, lane), c < n_chunks);
  ChunkWordsT<kPre256> cw{};
  uint4 sv[kSymVec];
  auto load_syms = [&](const ChunkMeta &m, bool ok) {
    const int nbytes = ok ? min(m.n_windows, 32) * E : 0;
#pragma unroll
    for (int i = 0; i < kSymVec; ++i) {
      const int off = 16 * (lane + 64 * i);
      sv[i] = make_uint4(0u, 0u, 0u, 0u);
      if (off < nbytes) {
        const int64_t g = m.sym_base + off;
        if (sym_vec && g + 16 <= n_symbols) {
          sv[i] = *reinterpret_cast<const uint4 *>(symbols + g);
        } else {
          uint32_t w[4] = {0u, 0u, 0u, 0u};
          for (int j = 0; j < 16; ++j)
            if (g + j < n_symbols) w[j >> 2] |= (uint32_t)symbols[g + j] << (8 * (j & 3));
          sv[i] = make_uint4(w[0], w[1], w[2], w[3]);
        }
      }
    }
  };
  if constexpr (FUSED) {
    if (c < n_chunks) load_chunk_words(words, symlen, cm.first_word, cm.word_end, lane, cw);
  } else {
    load_syms(cm, c < n_chunks);
  }
  uint32_t vn = load_meta_lane(meta, c + rstride, n_chunks, lane);

  unsigned tix = 0;  // tiles done by the workgroup (the shared form's flag slots)
#pragma unroll 1
  for (int64_t c0 = (int64_t)blockIdx.x * kWaves256; c0 < n_chunks; c0 += rstride) {
    c = c0 + wid;
    // ---- 1. this wave's chunk of the round into its LDS buffer
    const bool have = c < n_chunks && (!FUSED || cm.first_word >= 0);
    const int s_id = cm.stream < 0 ? 0 : (cm.stream >= n_streams ? n_streams - 1 : cm.stream);
    const int book = cm.book < n_books && cm.book >= 0 ? cm.book : 0;
    const float vg = load_gamma_lane(have ? gamma : nullptr, s_id, lane);
    if constexpr (FUSED) {
      if (have) {
        const void *lb = MS ? (const void *)(reinterpret_cast<const uint32_t *>(lds) + (book << lmax))
                            : (const void *)(reinterpret_cast<const uint16_t *>(lds) + (book << lmax));
        const int err = decode_chunk<MS, kPre256, false>(words, symlen, cm.first_word, cm.first_sym, cm.n_windows * E,
                                                  cm.word_end, cw, lb, cl + book * 256, MS ? binfo[book] : 0u, hs,
                                                  sb_own, lane);
        if (err && status) atomicOr(&status[s_id], err);
      }
    } else {
      if (have) {
        const int nbytes = cm.n_windows * E;
#pragma unroll
        for (int i = 0; i < kSymVec; ++i) {
          const int off = 16 * (lane + 64 * i);
          if (off < nbytes && off < 32 * E) *reinterpret_cast<uint4 *>(sb_own + off) = sv[i];
        }
        // windows past the first 32 (wpc > 32): straight from memory
        for (int off = 32 * E + lane; off < nbytes; off += 64) {
          const int64_t g = cm.sym_base + off;
          sb_own[off] = g < n_symbols ? symbols[g] : (uint8_t)128;
        }
      }
    }
    settle_lane(vg);
    settle_lane(vn);
    const ChunkScales cs = chunk_scales<PREC>(gamma, lane_float(vg, 0), lane_float(vg, 1), lane_float(vg, 2),
                                              dt.vmax[book], oscale);
    if (lane == 0) {
      Slot sl;
      sl.out_base = cm.out_base;
      sl.out_len = cm.out_len;
      sl.n_win = have ? cm.n_windows : 0;
      sl.book = book;
      sl.scaled = cs.scaled ? 1 : 0;
      sl.g0 = cs.g0;
      sl.g1 = cs.g1;
      sl.g2 = cs.g2;
      sl.oscale = cs.out;
      slots[wid] = sl;
    }
    // the next round's chunk: its record (requested a round ago) and words
    const int64_t cn = c + rstride;
    cm = meta_from_lanes(vn, cn < n_chunks);
    vn = load_meta_lane(meta, cn + rstride, n_chunks, lane);
    if constexpr (FUSED) {
      cw = ChunkWordsT<kPre256>{};
      if (cn < n_chunks) load_chunk_words(words, symlen, cm.first_word, cm.word_end, lane, cw);
    } else {
      load_syms(cm, cn < n_chunks);
    }
    __syncthreads();

    // ---- 2. every 32-window tile of the round's chunks, in order
    int ntiles[kWaves256];
    int T = 0;
#pragma unroll
    for (int q = 0; q < kWaves256; ++q) {
      const int nw = __builtin_amdgcn_readfirstlane(slots[q].n_win);
      ntiles[q] = nw > 0 ? (nw + kTileWindows - 1) / kTileWindows : 0;
      T += ntiles[q];
    }
    // tile k of the round -> its chunk slot and the chunk's 32-window tile
    // (static indices only, so the counts stay in registers)
    int tend[kWaves256];  // tiles of slots 0 .. q
    {
      int acc_t = 0;
#pragma unroll
      for (int q = 0; q < kWaves256; ++q) tend[q] = (acc_t += ntiles[q]);
    }
    auto locate = [&](int k, int &jj, int &tt) {
      jj = 0;
      tt = k;
#pragma unroll
      for (int q = 0; q < kWaves256 - 1; ++q)
        if (k >= tend[q]) {
          ++jj;
          tt -= ntiles[q];
        }
    };
    struct TileP {
      const unsigned char *sb;
      const uint8_t *rb, *tz;
      const float *tv;
      const uint32_t *pq;
      int n_win, out_len, tt;
      int64_t out_base;
      float os, g0, g1, g2;
      bool scaled;
    };
    auto params = [&](int k) {
      int jj, tt;
      locate(k, jj, tt);
      const Slot &sl = slots[jj];
      TileP t;
      t.tt = tt;
      t.n_win = __builtin_amdgcn_readfirstlane(sl.n_win);
      const int bk = __builtin_amdgcn_readfirstlane(sl.book);
      t.out_len = __builtin_amdgcn_readfirstlane(sl.out_len);
      t.out_base = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(sl.out_base >> 32)) << 32) |
                             (uint32_t)__builtin_amdgcn_readfirstlane((int)sl.out_base));
      t.os = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(sl.oscale)));
      t.scaled = false;
      t.g0 = t.g1 = t.g2 = 1.0f;
      if constexpr (FORM == kFormDequant || FORM == kFormDequantE) {
        t.scaled = __builtin_amdgcn_readfirstlane(sl.scaled) != 0;
        t.g0 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(sl.g0)));
        t.g1 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(sl.g1)));
        t.g2 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(sl.g2)));
      }
      t.sb = wave_base + (size_t)jj * wave256_bytes(wpc, E) + kSymPrefix;
      t.rb = dt.rb + bk * E;
      t.tv = dt.tv + bk * n_rows * 256;
      t.tz = dt.tz + bk * n_rows * 256;
      t.pq = dt.pq + bk * n_rows * 256;
      return t;
    };
    // shared form: the tile's coefficients dequantized once, into the
    // operand layout every wave reads (2 x 8 x 64 fragments of 8 halves, two
    // per thread), and whether any lower piece is nonzero, ORed into the
    // tile's flag slot
    auto dequant_tile = [&](const TileP &t, unsigned slot) {
      bool lo_any = false;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int v = threadIdx.x + kWaves256 * 64 * i;
        const int pv = v >> 9, sv_ = (v >> 6) & 7, lv = v & 63;
        const int wv = t.tt * kTileWindows + (lv & 31);
        const bool okv = wv < t.n_win;
        const unsigned char *row = t.sb + (okv ? wv : t.n_win - 1) * E + 128 * (lv >> 5);
        u8v a[AP];
        lo_any |= coef_frag<PREC, FORM>(row, pv, sv_, (lv >> 5), E, okv, e_vec, t.rb, t.tv, t.tz, t.pq, t.scaled, t.g0,
                                        t.g1, t.g2, a);
#pragma unroll
        for (int q = 0; q < AP; ++q) afrag[q * kFrags + v] = a[q];
      }
      if (__any(lo_any) && lane == 0) atomicOr(&tflag[slot], 1u);
    };
    bool first = true;
    int xb = 0;
    if constexpr (SH)
      if (T > 0) dequant_tile(params(0), tix & 1);
#pragma unroll 1
    for (int k = 0; k < T; ++k) {
      const TileP t = params(k);
      f16v acc;
      if constexpr (SH) {
        // the fragments of tile k are complete, the exchange reads of tile
        // k - 1 done; the other flag slot (last read for tile k - 1) is
        // cleared for tile k + 1
        __syncthreads();
        const unsigned slot = tix & 1;
        const bool rest = tflag[slot] != 0;
        if (threadIdx.x == 0) tflag[slot ^ 1] = 0;
        ++tix;
        // two accumulation chains (odd and even k-steps, highest bins
        // first) halve the chain of dependent MFMAs
        f16v a0 = {}, a1 = {};
#pragma unroll
        for (int s2 = kMaxSteps - 1; s2 >= 0; --s2) {
          u8v a[AP];
          a[0] = afrag[(p * kMaxSteps + s2) * 64 + lane];
#pragma unroll
          for (int q = 1; q < AP; ++q)  // lower pieces only when the tile has any
            a[q] = rest ? afrag[q * kFrags + (p * kMaxSteps + s2) * 64 + lane] : u8v{};
          if (s2 & 1)
            a1 = mfma_pieces<PREC>(bv[s2], a, a1, AP > 1 && rest);
          else
            a0 = mfma_pieces<PREC>(bv[s2], a, a0, AP > 1 && rest);
        }
        acc = a1 + a0;
      } else {
        const int wr = t.tt * kTileWindows + col;  // chunk-relative window of this lane's A row
        const bool valid = wr < t.n_win;
        acc = contract_parity<PREC, FORM>(bv, t.sb + (valid ? wr : t.n_win - 1) * E, p, h, E, valid, e_vec, t.rb,
                                          t.tv, t.tz, t.pq, t.scaled, t.g0, t.g1, t.g2);
      }
      if (first) {  // the next round's loads have arrived by now; wait before any store
        if constexpr (FUSED) {
          settle_chunk_words(cw);
        } else {
#pragma unroll
          for (int i = 0; i < kSymVec; ++i)
            asm volatile("" ::"v"(sv[i].x), "v"(sv[i].y), "v"(sv[i].z), "v"(sv[i].w) : "memory");
        }
        first = false;
      }
      // partial sums into the tile's exchange buffer: E (even waves) or O
      float *xe = xch + (size_t)xb * (kXchBytes / 4);
      float *xo = xe + kTileWindows * kXRow;
      if (nxb == 1 && !SH) __syncthreads();  // the buffer's previous readers are done
      {
        float *mine = (p ? xo : xe) + n0 + col;
#pragma unroll
        for (int r = 0; r < 16; ++r) mine[acc_window(r, h) * kXRow] = acc[r];
      }
      __syncthreads();  // sums visible; every wave done with tile k's fragments
      float *win0 = out + t.out_base + (int64_t)t.tt * kTileWindows * N256;
      const int rem = t.out_len - t.tt * kTileWindows * N256;  // samples from win0 to the chunk's end
      if (rem >= kTileWindows * N256 && (reinterpret_cast<uintptr_t>(win0) & 15) == 0) {
        // whole, aligned tile: the workgroup writes its 32 KB as 16-byte
        // non-temporal stores, 1 KB of consecutive samples per instruction;
        // float4 m holds samples 4 (m % 64) .. + 3 of window m / 64
#pragma unroll
        for (int i = 0; i < kTileWindows * N256 / 4 / (kWaves256 * 64); ++i) {
          const int m = threadIdx.x + i * kWaves256 * 64;
          const int w = m >> 6, q = m & 63;
          f4a x;
          if (q < 32) {  // x[n] = E[n] + O[n], n = 4 q ..
            const f4a e = *reinterpret_cast<const f4a *>(xe + w * kXRow + 4 * q);
            const f4a o = *reinterpret_cast<const f4a *>(xo + w * kXRow + 4 * q);
            x = (e + o) * t.os;
          } else {  // x[n] = E[255 - n] - O[255 - n], n = 4 q ..: the float4 at 252 - 4 q, reversed
            const int b = 252 - 4 * q;
            const f4a e = *reinterpret_cast<const f4a *>(xe + w * kXRow + b);
            const f4a o = *reinterpret_cast<const f4a *>(xo + w * kXRow + b);
            const f4a d = e - o;
            x = f4a{d[3], d[2], d[1], d[0]} * t.os;
          }
          __builtin_nontemporal_store(x, reinterpret_cast<f4a *>(win0 + 4 * m));
        }
      } else {
        // partial or misaligned tile: each wave writes its own columns, the
        // even wave x[n] = E + O, the odd wave x[255 - n] = E - O
        const int n = p ? N256 - 1 - (n0 + col) : n0 + col;
        const float *theirs = (p ? xe : xo) + n0 + col;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const float o = theirs[acc_window(r, h) * kXRow];
          const float x = p ? o - acc[r] : acc[r] + o;
          const int off = acc_window(r, h) * N256 + n;
          if (off < rem) win0[off] = x * t.os;
        }
      }
      // the next tile's coefficients, beside this tile's stores
      if constexpr (SH)
        if (k + 1 < T) dequant_tile(params(k + 1), tix & 1);
      xb ^= nxb - 1;
    }
    // every wave is done with this round's slots, symbols and exchange
    // buffers before the next round overwrites them
    __syncthreads();
  }
}

int pieces(int precision) { return precision == FPTC_BF16X3 ? 3 : (precision == FPTC_FP16X2 ? 2 : 1); }

template <int PREC, int FORM, bool SH>
int attrs_form_sh() {
  return lds_attr(k_w256<PREC, false, false, FORM, SH>) | lds_attr(k_w256<PREC, true, true, FORM, SH>) |
         lds_attr(k_w256<PREC, true, false, FORM, SH>);
}

// The shared-operand form for at most two pieces (three pieces would need
// 48 KB of operands).
template <int PREC, int FORM>
int attrs_form() {
  int rc = attrs_form_sh<PREC, FORM, false>();
  if constexpr (Traits<PREC>::kAPieces <= 2) rc |= attrs_form_sh<PREC, FORM, true>();
  return rc;
}

template <int PREC>
int attrs_prec() {
  int rc = attrs_form<PREC, kFormDequant>() | attrs_form<PREC, kFormDequantE>();
  if constexpr (Traits<PREC>::kAPieces <= 2) rc |= attrs_form<PREC, kFormPresplit1>() | attrs_form<PREC, kFormPresplitRows>();
  return rc;
}

// Double exchange buffers (one barrier per tile) when they fit, else one.
int exchange_buffers(bool fused, bool ms, int ap, const fptc_codec &c, int wpc) {
  if (w256_lds(fused, ms, ap, c.n_books, c.n_rows, c.lmax, c.E, wpc, 2, false) <= 160 * 1024) return 2;
  if (w256_lds(fused, ms, ap, c.n_books, c.n_rows, c.lmax, c.E, wpc, 1, false) <= 160 * 1024) return 1;
  return 0;
}

// The shared-operand form (one exchange buffer, two barriers per tile, each
// coefficient dequantized once per tile instead of once per column wave)
// when its operand buffer fits.
bool shared_fits(bool fused, bool ms, int ap, const fptc_codec &c, int wpc) {
  return ap <= 2 && w256_lds(fused, ms, ap, c.n_books, c.n_rows, c.lmax, c.E, wpc, 1, true) <= 160 * 1024;
}

template <int PREC, bool FUSED, bool MS, int FORM>
int launch_form(const fptc_batch &b, const fptc_codec &c, const Shape &sh, const Plan &p, const uint8_t *symbols,
                const float *gamma, float *out, int32_t *status, void *stream) {
  constexpr int AP = Traits<PREC>::kAPieces;
  const bool shr = shared_fits(FUSED, MS, AP, c, sh.wpc);
  const int nxb = shr ? 1 : exchange_buffers(FUSED, MS, AP, c, sh.wpc);
  if (!nxb) return (int)hipErrorInvalidValue;
  const size_t lds = w256_lds(FUSED, MS, AP, c.n_books, c.n_rows, c.lmax, c.E, sh.wpc, nxb, shr);
  const int blocks = sh.blocks > 0 ? sh.blocks : device_cu_count();
  auto kern = k_w256<PREC, FUSED, MS, FORM, false>;
  if constexpr (AP <= 2)
    if (shr) kern = k_w256<PREC, FUSED, MS, FORM, true>;
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(kWaves256 * 64), lds, (hipStream_t)stream, b.words, b.symlen, symbols,
                     b.n_symbols, b.n_streams, c.E, c.lmax, c.n_books, c.n_rows, sh.wpc, nxb, c.lut, c.deq_val,
                     c.deq_zone, c.row_of_bin, c.basis, p.hdr, p.chunk_meta, gamma, out, status);
  return (int)hipGetLastError();
}

// The coefficient form: the pre-split table when there are no per-stream
// scales, every bin is kept and at most two pieces are needed; otherwise
// dequantization, masking bins past E only when some are dropped.
template <int PREC, bool FUSED, bool MS>
int launch_t(const fptc_batch &b, const fptc_codec &c, const Shape &sh, const Plan &p, const uint8_t *symbols,
             const float *gamma, float *out, int32_t *status, void *stream) {
  if constexpr (Traits<PREC>::kAPieces <= 2) {
    if (!gamma && c.E == N256) {
      if (c.n_rows > 1)
        return launch_form<PREC, FUSED, MS, kFormPresplitRows>(b, c, sh, p, symbols, gamma, out, status, stream);
      return launch_form<PREC, FUSED, MS, kFormPresplit1>(b, c, sh, p, symbols, gamma, out, status, stream);
    }
  }
  if (c.E == N256) return launch_form<PREC, FUSED, MS, kFormDequant>(b, c, sh, p, symbols, gamma, out, status, stream);
  return launch_form<PREC, FUSED, MS, kFormDequantE>(b, c, sh, p, symbols, gamma, out, status, stream);
}

template <int PREC>
int launch_fused_prec(const fptc_batch &b, const fptc_codec &c, const Shape &sh, const Plan &p, const float *gamma,
                      float *out, int32_t *status, void *stream) {
  // multi-symbol decode tables when they fit beside everything else
  if (exchange_buffers(true, true, Traits<PREC>::kAPieces, c, sh.wpc))
    return launch_t<PREC, true, true>(b, c, sh, p, nullptr, gamma, out, status, stream);
  return launch_t<PREC, true, false>(b, c, sh, p, nullptr, gamma, out, status, stream);
}

}  // namespace

int set_mfma256_attributes() {
  return attrs_prec<FPTC_FP16>() | attrs_prec<FPTC_FP16X2>() | attrs_prec<FPTC_BF16>() | attrs_prec<FPTC_BF16X3>();
}

bool mfma256_supported(const fptc_codec &c, int precision, int wpc) {
  if (precision < FPTC_FP16 || precision > FPTC_BF16X3) return false;
  if (c.E < 1 || c.E > N256) return false;
  return exchange_buffers(false, false, pieces(precision), c, wpc) > 0;
}

bool fused256_supported(const fptc_codec &c, int precision, int wpc, int waves) {
  if (precision < FPTC_FP16 || precision > FPTC_BF16X3 || waves != kWaves256) return false;
  if (c.lmax > kShortLmax) return false;  // codes longer than 12 bits: decode, then dequant+IDCT
  if (c.E < 1 || c.E > N256) return false;
  return exchange_buffers(true, false, pieces(precision), c, wpc) > 0;
}

int launch_dqidct_mfma256(const fptc_batch &b, const fptc_codec &c, const Shape &s, const Plan &p,
                          const uint8_t *symbols, const float *gamma, int precision, float *out, void *stream) {
  switch (precision) {
    case FPTC_FP16: return launch_t<FPTC_FP16, false, false>(b, c, s, p, symbols, gamma, out, nullptr, stream);
    case FPTC_FP16X2: return launch_t<FPTC_FP16X2, false, false>(b, c, s, p, symbols, gamma, out, nullptr, stream);
    case FPTC_BF16: return launch_t<FPTC_BF16, false, false>(b, c, s, p, symbols, gamma, out, nullptr, stream);
    case FPTC_BF16X3: return launch_t<FPTC_BF16X3, false, false>(b, c, s, p, symbols, gamma, out, nullptr, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

int launch_fused256(const fptc_batch &b, const fptc_codec &c, const Shape &s, const Plan &p, const float *gamma,
                    int precision, float *out, int32_t *status, void *stream) {
  switch (precision) {
    case FPTC_FP16: return launch_fused_prec<FPTC_FP16>(b, c, s, p, gamma, out, status, stream);
    case FPTC_FP16X2: return launch_fused_prec<FPTC_FP16X2>(b, c, s, p, gamma, out, status, stream);
    case FPTC_BF16: return launch_fused_prec<FPTC_BF16>(b, c, s, p, gamma, out, status, stream);
    case FPTC_BF16X3: return launch_fused_prec<FPTC_BF16X3>(b, c, s, p, gamma, out, status, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

}  // namespace fptc
