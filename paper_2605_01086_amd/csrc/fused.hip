// One-pass batch decompression: Huffman decode -> dequantization -> inverse
// DCT -> float samples, per chunk of windows, with the chunk's decoded symbols
// kept in LDS (Section 4.2's two stages fused; the symbol array between them
// disappears).
//
// Work item = one chunk of `wpc` windows of one stream, owned by one wavefront:
//  1. decode: 64 words at a time, one word per lane (the paper's one thread per
//     word), run offsets from a DPP wavefront prefix sum of symlen, each lane
//     decoding exactly symlen[w] symbols with lmax-bit peeks into the
//     codebook's lookup table in LDS (up to three symbols per peek when the
//     multi-symbol table fits).  Symbols of the chunk land in a per-wave LDS
//     buffer in window-major order.  The first 128 words of the next chunk are
//     loaded while this chunk is processed, later rounds one round ahead.
//  2. per 32 windows: dequantize from LDS into split 16-bit operands, contract
//     with the split IDCT basis on v_mfma_f32_32x32x16 (exactly the arithmetic
//     of the stand-alone MFMA kernel, so results are bit-identical) and store
//     rows of 32 consecutive samples per half-wave.
#include <hip/hip_runtime.h>

#include "fptc_internal.h"
#include "decode_common.h"
#include "mfma_common.h"

namespace fptc {
namespace {

__host__ __device__ constexpr size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

// Waves per block: up to 16; up to 8 at N = 128, whose basis leaves LDS for
// no more than that and whose four output tiles need the registers.
__host__ __device__ constexpr int max_fused_waves(int N) { return N >= 128 ? 8 : 16; }

// Per-wave LDS region: a prefix for symbols of the previous chunk, then the
// chunk's decoded symbols, then (E < N) a staging area for a quarter tile of
// output (8 N + 4 floats), which with E = N fits in the consumed symbols.
__host__ __device__ inline size_t fused_sym_bytes(int E, int wpc) { return align16((size_t)wpc * E + 16); }
__host__ __device__ inline size_t fused_wave_bytes(int E, int wpc, int N) {
  return (size_t)kSymPrefix + fused_sym_bytes(E, wpc) + (E < N ? align16((size_t)32 * N + 16) : 0);
}

// LDS: lookup tables | split basis | dequantization tables | wave buffers |
// chunk counter (16 B).  The multi-symbol build borrows lut1_temp_bytes right
// after the tables.
__host__ __device__ inline size_t fused_lds_bytes(bool ms, int bpieces, int N, int E, int Kp, int wpc, int waves,
                                                  int n_books, int n_rows, int lmax) {
  const size_t t = lut_lds_bytes(ms, n_books, lmax);
  const size_t need = t + (size_t)bpieces * N * (Kp + 8) * 2 + deq_table_bytes(bpieces, n_books, n_rows, E) +
                      (size_t)waves * fused_wave_bytes(E, wpc, N) + 16;
  const size_t tmp = (ms && lmax <= kShortLmax) ? t + lut1_temp_bytes(n_books, lmax) : 0;
  return need > tmp ? need : tmp;
}

template <int PREC, int NT, bool MS, bool LG>
__global__ void __launch_bounds__(64 * max_fused_waves(NT * 32)) k_fused(const uint64_t *__restrict__ words,
                                                            const uint8_t *__restrict__ symlen, int n_streams, int E,
                                                            int S, int lmax, int n_books, int n_rows, int wpc,
                                                            const uint16_t *__restrict__ lut_g,
                                                            const float *__restrict__ deq_val,
                                                            const uint8_t *__restrict__ deq_zone,
                                                            const uint8_t *__restrict__ row_of_bin,
                                                            const float *__restrict__ basis,
                                                            const int64_t *__restrict__ hdr,
                                                            const ChunkMeta *__restrict__ meta,
                                                            const float *__restrict__ gamma, float *out,
                                                            int32_t *status, int group) {
  using T = Traits<PREC>;
  constexpr int N = NT * 32;
  const int Kp = S * 16, KH = Kp / 2, RS = Kp + 8;
  constexpr int AP = T::kAPieces;
  extern __shared__ __align__(16) unsigned char lds[];
  const int nthreads = blockDim.x, waves = nthreads >> 6;
  const size_t lut_bytes = lut_lds_bytes(MS, n_books, lmax);
  uint16_t *Bs = reinterpret_cast<uint16_t *>(lds + lut_bytes);
  unsigned char *tables = reinterpret_cast<unsigned char *>(Bs + (size_t)T::kBPieces * N * RS);
  const DeqTables dt = deq_tables_at(tables, n_books, n_rows, E);
  unsigned char *wave_base = tables + deq_table_bytes(AP, n_books, n_rows, E);

  // ---- block setup: lookup tables, basis pieces, dequantization tables
  stage_decode_tables(MS, lds, lds + lut_bytes, lut_g, lmax, n_books, threadIdx.x, nthreads);
  stage_basis<PREC>(Bs, basis, N, E, Kp, RS, threadIdx.x, nthreads);
  stage_deq_tables<PREC>(dt, deq_val, deq_zone, row_of_bin, n_books, n_rows, E, threadIdx.x, nthreads);
  unsigned *chunk_ctr = reinterpret_cast<unsigned *>(wave_base + (size_t)waves * fused_wave_bytes(E, wpc, N));
  if (threadIdx.x == 0) *chunk_ctr = 0;
  __syncthreads();

  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63, col = lane & 31, h = lane >> 5;
  unsigned char *sb = wave_base + (size_t)wid * fused_wave_bytes(E, wpc, N) + kSymPrefix;
  const uint8_t *cl = lds + ((size_t)n_books << lmax) * 4;
  const uint32_t *binfo = reinterpret_cast<const uint32_t *>(cl + n_books * 256);  // multi-symbol form only
  const int hs = 32 - lmax;  // peek = top lmax bits of the word = hi32 >> hs
  const float oscale = 1.0f / (T::kF16 ? kBasisScaleF16 : 1.0f);
  const int64_t n_chunks = hdr[0];

  // Software pipeline over this wave's chunks (taken from the workgroup's
  // schedule): the words of chunk i+1 (and the record of chunk i+2) are
  // requested before chunk i decodes and are waited for right after that
  // decode, before chunk i's stores.  Vector memory counters retire in order,
  // so this one wait also covers chunk i-1's stores, which had the whole
  // decode to drain.
  //
  // The workgroup owns groups of `group` adjacent chunks spread over the
  // whole batch (group g goes to workgroup g mod grid size).  Decode cost
  // varies with the stream's bit rate, so many small groups from everywhere
  // even out the workgroups' totals; within a group, adjacent chunks keep
  // the words read and the samples written contiguous.
  const BlockChunks sched{chunk_ctr, (int64_t)blockIdx.x * group, (int64_t)gridDim.x * group, 1, group};
  int64_t c = sched.next(lane), cn = sched.next(lane);
  ChunkMeta cm = meta_from_lanes(load_meta_lane(meta, c, n_chunks, lane), c < n_chunks);
  const uint32_t vn = load_meta_lane(meta, cn, n_chunks, lane);
  ChunkWords cw{};
  if (c < n_chunks) load_chunk_words(words, symlen, cm.first_word, cm.word_end, lane, cw);
  ChunkMeta nm = meta_from_lanes(vn, cn < n_chunks);
  while (c < n_chunks) {
    const int64_t cmm = sched.next(lane);
    const bool ok = cm.first_word >= 0;  // else the stream's symbol count is wrong; already flagged
    const int s = cm.stream < 0 ? 0 : (cm.stream >= n_streams ? n_streams - 1 : cm.stream);
    const int book = cm.book < n_books && cm.book >= 0 ? cm.book : 0;
    const int w_cnt = cm.n_windows;
    const float vg = load_gamma_lane(gamma, s, lane);
    const uint32_t vm = load_meta_lane(meta, cmm, n_chunks, lane);
    ChunkWords nx{};
    if (cn < n_chunks) load_chunk_words(words, symlen, nm.first_word, nm.word_end, lane, nx);

    // ---- 1. decode the chunk's symbols into sb[0 .. w_cnt * E)
    int err = 0;
    if (ok) {
      const void *lb = LG   ? (const void *)(reinterpret_cast<const uint16_t *>(lds) +
                                             (size_t)book * (kLongPrefixes + kLongSub))
                       : MS ? (const void *)(reinterpret_cast<const uint32_t *>(lds) + (book << lmax))
                            : (const void *)(reinterpret_cast<const uint16_t *>(lds) + (book << lmax));
      err = decode_chunk<MS, kPreRounds, LG>(words, symlen, cm.first_word, cm.first_sym, w_cnt * E, cm.word_end, cw,
                                             lb, cl + book * 256, MS ? binfo[book] : 0u, hs, sb, lane, lmax);
    }
    settle_chunk_words(nx);
    settle_lane(vm);
    settle_lane(vg);
    const ChunkMeta mm = meta_from_lanes(vm, cmm < n_chunks);
    cw = nx;
    if (ok) {
      if (err && status) atomicOr(&status[s], err);
      const ChunkScales cs = chunk_scales<PREC>(gamma, lane_float(vg, 0), lane_float(vg, 1), lane_float(vg, 2),
                                                dt.vmax[book], oscale);
      wave_sync_lds();

      // ---- 2. per 32 windows: dequantize, contract, store
      for (int tt = 0; tt * kTileWindows < w_cnt; ++tt) {
        const int wr = tt * kTileWindows + col;  // chunk-relative window of this lane's column
        const int valid = wr < w_cnt ? min(N, cm.out_len - wr * N) : 0;
        // windows past the chunk read the last window's symbols (discarded)
        const int base = (wr < w_cnt ? wr : w_cnt - 1) * E;
        // the chunk's windows are consecutive in one stream
        float *win0 = out + cm.out_base + (int64_t)tt * kTileWindows * N;
        const int rem = cm.out_len - tt * kTileWindows * N;
        auto emit = [&](const f16v (&acc)[NT]) {
          if (E < N || wpc >= kTileWindows) {  // staged through LDS: E = N, the consumed symbols
            float *stage = E < N ? reinterpret_cast<float *>(sb + fused_sym_bytes(E, wpc))
                                 : reinterpret_cast<float *>(sb) - 4;
            if (rem >= kTileWindows * N)
              store_tile_whole<NT>(win0, acc, stage, h, col, lane, cs.out);
            else
              store_tile_staged<NT>(win0, acc, stage, h, col, lane, rem, cs.out);
          } else {
#pragma unroll
            for (int t = 0; t < NT; ++t) store_rows(win0, N, acc[t], t, h, col, rem, cs.out);
          }
        };
        tile_contract_emit<PREC, NT>(sb, base, h, col, S, E, valid > 0, Bs, RS, dt.rb + book * E,
                                     dt.tv + book * n_rows * 256, dt.tz + book * n_rows * 256,
                                     dt.pq + book * n_rows * 256, n_rows, gamma, cs, emit);
      }
      wave_sync_lds();
    }
    cm = nm;
    nm = mm;
    c = cn;
    cn = cmm;
  }
}

int pieces_of(int precision) {
  return precision == FPTC_BF16X3 ? 3 : (precision == FPTC_FP16X2 ? 2 : 1);
}

template <int PREC, int NT, bool MS, bool LG>
int launch_t(const fptc_batch &b, const fptc_codec &c, const Shape &sh, const Plan &p, const float *gamma, float *out,
             int32_t *status, void *stream) {
  constexpr int N = NT * 32;
  const int S = (c.E + 15) / 16, Kp = S * 16;
  const size_t lds =
      fused_lds_bytes(MS, Traits<PREC>::kBPieces, N, c.E, Kp, sh.wpc, sh.waves, c.n_books, c.n_rows, c.lmax);
  auto kern = k_fused<PREC, NT, MS, LG>;
  const int per_cu = (int)((160 * 1024) / lds);
  const int blocks = sh.blocks > 0 ? sh.blocks : device_cu_count() * (per_cu > 0 ? per_cu : 1);
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(sh.waves * 64), lds, (hipStream_t)stream, b.words, b.symlen,
                     b.n_streams, c.E, S, c.lmax, c.n_books, c.n_rows, sh.wpc, c.lut, c.deq_val, c.deq_zone,
                     c.row_of_bin, c.basis, p.hdr, p.chunk_meta, gamma, out, status, sh.group);
  return (int)hipGetLastError();
}

// Multi-symbol decode tables when they fit beside everything else.
template <int PREC, int NT>
int launch_ms(const fptc_batch &b, const fptc_codec &c, const Shape &sh, const Plan &p, const float *gamma,
              float *out, int32_t *status, void *stream) {
  const int Kp = (c.E + 15) / 16 * 16;
  if (c.lmax > kShortLmax) return launch_t<PREC, NT, false, true>(b, c, sh, p, gamma, out, status, stream);
  if (fused_lds_bytes(true, Traits<PREC>::kBPieces, NT * 32, c.E, Kp, sh.wpc, sh.waves, c.n_books, c.n_rows,
                      c.lmax) <= 160 * 1024)
    return launch_t<PREC, NT, true, false>(b, c, sh, p, gamma, out, status, stream);
  return launch_t<PREC, NT, false, false>(b, c, sh, p, gamma, out, status, stream);
}

template <int PREC>
int launch_prec(const fptc_batch &b, const fptc_codec &c, const Shape &sh, const Plan &p, const float *gamma,
                float *out, int32_t *status, void *stream) {
  switch (c.N) {
    case 32: return launch_ms<PREC, 1>(b, c, sh, p, gamma, out, status, stream);
    case 64: return launch_ms<PREC, 2>(b, c, sh, p, gamma, out, status, stream);
    case 128: return launch_ms<PREC, 4>(b, c, sh, p, gamma, out, status, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

template <int PREC, int NT>
int attrs_nt() {
  return lds_attr(k_fused<PREC, NT, true, false>) | lds_attr(k_fused<PREC, NT, false, false>) |
         lds_attr(k_fused<PREC, NT, false, true>);
}

template <int PREC>
int attrs_prec() {
  return attrs_nt<PREC, 1>() | attrs_nt<PREC, 2>() | attrs_nt<PREC, 4>();
}

}  // namespace

int set_fused_attributes() {
  return attrs_prec<FPTC_FP16>() | attrs_prec<FPTC_FP16X2>() | attrs_prec<FPTC_BF16>() | attrs_prec<FPTC_BF16X3>();
}

bool fused_supported(int N, int E, int precision, int wpc, int waves, int n_books, int n_rows, int lmax) {
  if (precision < FPTC_FP16 || precision > FPTC_BF16X3) return false;
  if (waves < 1 || waves > max_fused_waves(N)) return false;
  if (N != 32 && N != 64 && N != 128) return false;
  if (E < 1 || E > N) return false;
  const int Kp = (E + 15) / 16 * 16;
  return fused_lds_bytes(false, pieces_of(precision), N, E, Kp, wpc, waves, n_books, n_rows, lmax) <= 160 * 1024;
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
