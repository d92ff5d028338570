// One-pass batch decompression: Huffman decode -> dequantization -> inverse
// DCT -> float samples, per chunk of windows, with the chunk's decoded symbols
// kept in LDS (Section 4.2's two stages fused; the symbol array between them
// disappears).
//
// Work item = one chunk of `wpc` windows of one stream, owned by one wavefront:
//  1. decode: 64 words at a time, one word per lane (the paper's one thread per
//     word), run offsets from a DPP wavefront prefix sum of symlen, each lane
//     decoding exactly symlen[w] symbols with lmax-bit peeks into the
//     codebook's lookup table in LDS.  Symbols of the chunk land in a per-wave
//     LDS buffer in window-major order; the next 64 words are loaded while the
//     current ones decode.
//  2. per 32 windows: dequantize from LDS into split 16-bit operands, contract
//     with the split IDCT basis on v_mfma_f32_32x32x16 (exactly the arithmetic
//     of the stand-alone MFMA kernel, so results are bit-identical) and store
//     each lane's four consecutive samples with one 16-byte write.
#include <hip/hip_runtime.h>

#include "fptc_internal.h"
#include "decode_common.h"
#include "mfma_common.h"

namespace fptc {
namespace {

__host__ __device__ constexpr size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

constexpr int kMaxFusedWaves = 16;
constexpr int kMaxFusedThreads = kMaxFusedWaves * 64;

// Per-wave LDS region: the chunk's decoded symbols.
__host__ __device__ inline size_t fused_wave_bytes(int N, int E, int wpc) {
  (void)N;
  return align16((size_t)wpc * E + 16);
}

__host__ __device__ inline size_t fused_lds_bytes(int bpieces, int N, int E, int Kp, int wpc, int waves, int n_books,
                                                  int n_rows, int lmax) {
  return align16((size_t)(n_books << lmax) * 2) + (size_t)bpieces * N * (Kp + 8) * 2 +
         align16((size_t)n_books * n_rows * 256 * 5 + (size_t)n_books * E) + (size_t)waves * fused_wave_bytes(N, E, wpc);
}

template <int PREC, int NT>
__global__ void __launch_bounds__(kMaxFusedThreads) k_fused(const uint64_t *__restrict__ words,
                                                            const uint8_t *__restrict__ symlen, int n_streams, int E,
                                                            int S,
                                                            int lmax, int n_books, int n_rows, int wpc,
                                                            const uint16_t *lut_g, const float *deq_val,
                                                            const uint8_t *deq_zone, const uint8_t *row_of_bin,
                                                            const float *basis, const int64_t *hdr,
                                                            const ChunkMeta *__restrict__ meta, const float *gamma,
                                                            float *out, int32_t *status) {
  using T = Traits<PREC>;
  constexpr int N = NT * 32;
  const int Kp = S * 16, KH = Kp / 2, RS = Kp + 8;
  constexpr int AP = T::kAPieces;
  extern __shared__ __align__(16) unsigned char lds[];
  const int nthreads = blockDim.x, waves = nthreads >> 6;
  uint16_t *lut = reinterpret_cast<uint16_t *>(lds);
  uint16_t *Bs = reinterpret_cast<uint16_t *>(lds + align16((size_t)(n_books << lmax) * 2));
  float *Tv = reinterpret_cast<float *>(Bs + (size_t)T::kBPieces * N * RS);
  uint8_t *Tz = reinterpret_cast<uint8_t *>(Tv + n_books * n_rows * 256);
  uint8_t *Rb = Tz + n_books * n_rows * 256;
  unsigned char *wave_base = reinterpret_cast<unsigned char *>(Tv) + align16((size_t)n_books * n_rows * 256 * 5 +
                                                                             (size_t)n_books * E);

  // ---- block setup: lookup tables, basis pieces, dequantization tables
  stage_lut(lut, lut_g, n_books << lmax, threadIdx.x, nthreads);
  stage_basis<PREC>(Bs, basis, N, E, Kp, RS, threadIdx.x, nthreads);
  for (int i = threadIdx.x; i < n_books * n_rows * 256; i += nthreads) {
    Tv[i] = deq_val[i];
    const int z = deq_zone[i];
    Tz[i] = (uint8_t)(z < 2 ? z : 2);
  }
  for (int i = threadIdx.x; i < n_books * E; i += nthreads) {
    const int r = row_of_bin[i];
    Rb[i] = (uint8_t)(r < n_rows ? r : n_rows - 1);
  }
  __syncthreads();

  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63, col = lane & 31, h = lane >> 5;
  unsigned char *sb = wave_base + (size_t)wid * fused_wave_bytes(N, E, wpc);
  const int hs = 32 - lmax;  // peek = top lmax bits of the word = hi32 >> hs
  const float oscale = 1.0f / (T::kF16 ? kBasisScaleF16 : 1.0f);
  const bool e_vec = (E % 16) == 0;
  const int64_t n_chunks = hdr[0];

  for (int64_t c = (int64_t)blockIdx.x * waves + wid; c < n_chunks; c += (int64_t)gridDim.x * waves) {
    const ChunkMeta cm = meta[c];
    if (cm.first_word < 0) continue;  // the stream's symbol count is wrong; already flagged
    const int s = cm.stream < 0 ? 0 : (cm.stream >= n_streams ? n_streams - 1 : cm.stream);
    const int book = cm.book < n_books ? cm.book : 0;
    const int w_cnt = cm.n_windows;
    float g0 = 1.0f, g1 = 1.0f, g2 = 1.0f;
    if (gamma) {
      g0 = gamma[3 * (int64_t)s];
      g1 = gamma[3 * (int64_t)s + 1];
      g2 = gamma[3 * (int64_t)s + 2];
    }

    // ---- 1. decode the chunk's symbols into sb[0 .. w_cnt * E)
    const int err = decode_range(words, symlen, cm.first_word, cm.first_sym, w_cnt * E, cm.word_end,
                                 lut + (book << lmax), hs, sb, lane);
    if (err && status) atomicOr(&status[s], err);
    wave_sync_lds();

    // ---- 2. per 32 windows: dequantize, contract, store
    for (int tt = 0; tt * kTileWindows < w_cnt; ++tt) {
      const int wr = tt * kTileWindows + col;  // chunk-relative window of this lane's column
      const int valid = wr < w_cnt ? min(N, cm.out_len - wr * N) : 0;
      // windows past the chunk read the last window's symbols (discarded)
      const int base = (wr < w_cnt ? wr : w_cnt - 1) * E;
      f16v acc[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[t][r] = 0.0f;
#pragma unroll 1
      for (int ss = S - 1; ss >= 0; --ss) {
        const int k0 = h * KH + 8 * ss;
        uint8_t sy[8];
        if (e_vec) {  // E % 16 == 0: the 8-bin group is inside [0, E) and 8-byte aligned
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
        const bool r = dequant8<PREC>(sy, k0, E, valid > 0, Rb + book * E, Tv + book * n_rows * 256,
                                      Tz + book * n_rows * 256, gamma != nullptr, g0, g1, g2, a);
        const bool any_rest = AP > 1 && __any(r);
        mfma_step<PREC, NT>(acc, a, Bs + col * RS + k0, 32 * RS, N * RS, any_rest);
      }
      // this lane's window starts at out_base + wr * N; all windows of a chunk
      // are consecutive in one stream
      if (valid > 0) {
        float *dst = out + cm.out_base + (int64_t)wr * N;
#pragma unroll
        for (int t = 0; t < NT; ++t) store_block(dst, acc[t], t * 32, h, valid, oscale);
      }
    }
  }
}

int pieces_of(int precision) {
  return precision == FPTC_BF16X3 ? 3 : (precision == FPTC_FP16X2 ? 2 : 1);
}

template <int PREC, int NT>
int launch_t(const fptc_batch &b, const fptc_codec &c, const Shape &sh, const Plan &p, const float *gamma, float *out,
             int32_t *status, void *stream) {
  constexpr int N = NT * 32;
  const int S = (c.E + 15) / 16, Kp = S * 16;
  const size_t lds = fused_lds_bytes(Traits<PREC>::kBPieces, N, c.E, Kp, sh.wpc, sh.waves, c.n_books, c.n_rows, c.lmax);
  auto kern = k_fused<PREC, NT>;
  static bool attr_set = false;  // one attribute call per instantiation
  if (!attr_set) {
    if (hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024) != hipSuccess)
      return (int)hipErrorInvalidValue;
    attr_set = true;
  }
  const int per_cu = (int)((160 * 1024) / lds);
  const int blocks = sh.blocks > 0 ? sh.blocks : device_cu_count() * (per_cu > 0 ? per_cu : 1);
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(sh.waves * 64), lds, (hipStream_t)stream, b.words, b.symlen,
                     b.n_streams, c.E, S, c.lmax, c.n_books, c.n_rows, sh.wpc, c.lut, c.deq_val, c.deq_zone,
                     c.row_of_bin, c.basis, p.hdr, p.chunk_meta, gamma, out, status);
  return (int)hipGetLastError();
}

template <int PREC>
int launch_prec(const fptc_batch &b, const fptc_codec &c, const Shape &sh, const Plan &p, const float *gamma,
                float *out, int32_t *status, void *stream) {
  switch (c.N) {
    case 32: return launch_t<PREC, 1>(b, c, sh, p, gamma, out, status, stream);
    case 64: return launch_t<PREC, 2>(b, c, sh, p, gamma, out, status, stream);
    case 128: return launch_t<PREC, 4>(b, c, sh, p, gamma, out, status, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

}  // namespace

bool fused_supported(int N, int E, int precision, int wpc, int waves, int n_books, int n_rows, int lmax) {
  if (precision < FPTC_FP16 || precision > FPTC_BF16X3) return false;
  if (waves < 1 || waves > kMaxFusedWaves) return false;
  if (N != 32 && N != 64 && N != 128) return false;
  if (E < 1 || E > N) return false;
  const int Kp = (E + 15) / 16 * 16;
  return fused_lds_bytes(pieces_of(precision), N, E, Kp, wpc, waves, n_books, n_rows, lmax) <= 160 * 1024;
}

int launch_fused(const fptc_batch &b, const fptc_codec &c, const Shape &s, const Plan &p, const float *gamma,
                 int precision, float *out, int32_t *status, void *stream) {
  switch (precision) {
    case FPTC_FP16: return launch_prec<FPTC_FP16>(b, c, s, p, gamma, out, status, stream);
    case FPTC_FP16X2: return launch_prec<FPTC_FP16X2>(b, c, s, p, gamma, out, status, stream);
    case FPTC_BF16: return launch_prec<FPTC_BF16>(b, c, s, p, gamma, out, status, stream);
    case FPTC_BF16X3: return launch_prec<FPTC_BF16X3>(b, c, s, p, gamma, out, status, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

}  // namespace fptc
