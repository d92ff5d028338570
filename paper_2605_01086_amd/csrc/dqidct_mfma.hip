// Dequantization fused with the inverse DCT on the matrix cores (Section 4.2,
// lossy stage, as a dense contraction).
//
// For a tile of up to 32 consecutive windows of one stream (a chunk of the
// plan, or a 32-window part of it) one wavefront forms
//     D[w][n] = sum_k c[w][k] * B[k][n]
// with v_mfma_f32_32x32x16_{f16,bf16} (coefficients as the A operand, basis
// as B): FP32 accumulation, 16-bit operands.  A lane ends up holding one
// sample of 16 windows, so every store instruction writes 32 consecutive
// samples of two windows: whole 128-byte runs, the fewest write requests.
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
// The basis pieces live in LDS (rows padded by 16 bytes to spread banks), as do
// the dequantization tables and each wave's tile of symbols; coefficients are
// dequantized in registers from the symbols (tile_contract_emit).
#include <hip/hip_runtime.h>

#include "fptc_internal.h"
#include "mfma_common.h"

namespace fptc {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

__host__ __device__ constexpr size_t a16(size_t x) { return (x + 15) & ~(size_t)15; }

// Per-wave LDS: 16 bytes, one 32-window symbol tile, then (E < N) a staging
// area for a quarter tile of output (8 N + 4 floats); with E = N the consumed
// symbol tile holds it.
__host__ __device__ constexpr size_t tile_sym_bytes(int E) { return a16((size_t)kTileWindows * E + 16); }
__host__ __device__ constexpr size_t mfma_wave_bytes(int N, int E) {
  return 16 + tile_sym_bytes(E) + (E < N ? a16((size_t)32 * N + 16) : 0);
}

// LDS bytes of one instantiation: basis pieces, tables, the waves' regions,
// the chunk counter (16 B).
__host__ __device__ constexpr size_t mfma_lds_bytes(int bpieces, int N, int Kp, int n_books, int n_rows, int E) {
  return (size_t)bpieces * N * (Kp + 8) * 2 + deq_table_bytes(bpieces, n_books, n_rows, E) +
         (size_t)kWaves * mfma_wave_bytes(N, E) + 16;
}

// The symbols of a 32-window tile, 16 bytes per lane per round: R rounds of
// 64 lanes cover 32 windows of E <= 32 R symbols.
template <int R>
struct TileSyms {
  uint4 v[R];
};

template <int R>
__device__ inline void load_tile_syms(const uint8_t *__restrict__ symbols, int64_t n_symbols, int64_t base,
                                      int nbytes, bool vec16, int lane, TileSyms<R> &t) {
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int off = 16 * (lane + 64 * r);
    t.v[r] = make_uint4(0u, 0u, 0u, 0u);
    if (off < nbytes) {
      const int64_t g = base + off;
      if (vec16 && g + 16 <= n_symbols) {
        t.v[r] = *reinterpret_cast<const uint4 *>(symbols + g);
      } else {
        uint32_t w[4] = {0u, 0u, 0u, 0u};
        for (int j = 0; j < 16; ++j)
          if (g + j < n_symbols) w[j >> 2] |= (uint32_t)symbols[g + j] << (8 * (j & 3));
        t.v[r] = make_uint4(w[0], w[1], w[2], w[3]);
      }
    }
  }
}

template <int R>
__device__ inline void put_tile_syms(unsigned char *sb, int nbytes, int lane, const TileSyms<R> &t) {
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int off = 16 * (lane + 64 * r);
    if (off < nbytes) *reinterpret_cast<uint4 *>(sb + off) = t.v[r];
  }
}

// Pin the wait for prefetched symbols here (see settle_chunk_words).
template <int R>
__device__ inline void settle_tile_syms(const TileSyms<R> &t) {
#pragma unroll
  for (int r = 0; r < R; ++r)
    asm volatile("" ::"v"(t.v[r].x), "v"(t.v[r].y), "v"(t.v[r].z), "v"(t.v[r].w) : "memory");
}

// Work item = one chunk of the plan (up to wpc consecutive windows of one
// stream), in 32-window tiles; NT = N / 32 output row tiles, S = Kp / 16
// k-steps (Kp = E rounded up to 16).  A tile's symbols are one contiguous run:
// they are staged into the wave's LDS buffer with 16-byte loads, the first
// tile of the next chunk being loaded while this chunk computes.
template <int PREC, int NT>
__global__ void __launch_bounds__(kThreads, NT >= 4 ? 2 : (NT == 2 ? 3 : 4)) k_dqidct_mfma(fptc_batch b, int E, int S, int n_books, int n_rows,
                                                          const float *__restrict__ deq_val,
                                                          const uint8_t *__restrict__ deq_zone,
                                                          const uint8_t *__restrict__ row_of_bin,
                                                          const float *__restrict__ basis,
                                                          const int64_t *__restrict__ hdr,
                                                          const ChunkMeta *__restrict__ meta,
                                                          const uint8_t *__restrict__ symbols,
                                                          const float *__restrict__ gamma, float *out) {
  using T = Traits<PREC>;
  constexpr int N = NT * 32;
  const int Kp = S * 16;
  const int RS = Kp + 8;  // LDS row stride of a basis piece, in halves
  constexpr int BP = T::kBPieces, AP = T::kAPieces;
  extern __shared__ __align__(16) unsigned char lds[];
  uint16_t *Bs = reinterpret_cast<uint16_t *>(lds);                       // [BP][N][RS]
  unsigned char *tables = lds + (size_t)BP * N * RS * 2;
  const DeqTables dt = deq_tables_at(tables, n_books, n_rows, E);
  unsigned char *bufs = tables + deq_table_bytes(AP, n_books, n_rows, E);

  // Stage the split basis (transposed to [n][k], zero beyond E) and the tables.
  const float bscale = T::kF16 ? kBasisScaleF16 : 1.0f;
  stage_basis<PREC>(Bs, basis, N, E, Kp, RS, threadIdx.x, kThreads);
  stage_deq_tables<PREC>(dt, deq_val, deq_zone, row_of_bin, n_books, n_rows, E, threadIdx.x, kThreads);
  unsigned *chunk_ctr = reinterpret_cast<unsigned *>(bufs + (size_t)kWaves * mfma_wave_bytes(N, E));
  if (threadIdx.x == 0) *chunk_ctr = 0;
  __syncthreads();

  const int lane = threadIdx.x & 63, col = lane & 31, h = lane >> 5;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  unsigned char *sb = bufs + (size_t)wid * mfma_wave_bytes(N, E) + 16;
  const int64_t n_chunks = hdr[0];
  const int64_t cstride = (int64_t)gridDim.x * kWaves;
  const float oscale = 1.0f / bscale;
  const bool vec16 = (E % 16) == 0 && (reinterpret_cast<uintptr_t>(symbols) & 15) == 0;

  // chunks from the workgroup's schedule (BlockChunks)
  const BlockChunks sched{chunk_ctr, (int64_t)blockIdx.x * kWaves, cstride, 1, kWaves};
  int64_t c = sched.next(lane), cn = sched.next(lane);
  ChunkMeta cm = meta_from_lanes(load_meta_lane(meta, c, n_chunks, lane), c < n_chunks);
  const uint32_t vn = load_meta_lane(meta, cn, n_chunks, lane);
  TileSyms<NT> cur{};
  if (c < n_chunks)
    load_tile_syms(symbols, b.n_symbols, cm.sym_base, min(kTileWindows, cm.n_windows) * E, vec16, lane, cur);
  ChunkMeta nm = meta_from_lanes(vn, cn < n_chunks);
  auto stream_of = [&](const ChunkMeta &m) {
    return m.stream < 0 ? 0 : (m.stream >= b.n_streams ? b.n_streams - 1 : m.stream);
  };
  // per-stream scales of the current chunk, requested one chunk ahead
  float vg = load_gamma_lane(gamma, stream_of(cm), lane);
  settle_lane(vg);
  while (c < n_chunks) {
    const int book = cm.book < n_books && cm.book >= 0 ? cm.book : 0;
    const int w_cnt = cm.n_windows;
    const ChunkScales cs = chunk_scales<PREC>(gamma, lane_float(vg, 0), lane_float(vg, 1), lane_float(vg, 2),
                                              dt.vmax[book], oscale);
    const int64_t cmm = sched.next(lane);
    const uint32_t vm = load_meta_lane(meta, cmm, n_chunks, lane);
    const float vgn = load_gamma_lane(gamma, stream_of(nm), lane);
    TileSyms<NT> nx{};
    if (cn < n_chunks)
      load_tile_syms(symbols, b.n_symbols, nm.sym_base, min(kTileWindows, nm.n_windows) * E, vec16, lane, nx);
    for (int tt = 0; tt * kTileWindows < w_cnt; ++tt) {
      const int wt = min(kTileWindows, w_cnt - tt * kTileWindows);
      if (tt == 0) {
        put_tile_syms(sb, wt * E, lane, cur);
      } else {
        TileSyms<NT> t;
        load_tile_syms(symbols, b.n_symbols, cm.sym_base + (int64_t)tt * kTileWindows * E, wt * E, vec16, lane, t);
        put_tile_syms(sb, wt * E, lane, t);
      }
      wave_sync_lds();
      const int wr = tt * kTileWindows + col;
      const int valid = col < wt ? min(N, cm.out_len - wr * N) : 0;
      const int base = (col < wt ? col : wt - 1) * E;
      float *win0 = out + cm.out_base + (int64_t)tt * kTileWindows * N;
      const int rem = cm.out_len - tt * kTileWindows * N;
      auto emit = [&](const f16v (&acc)[NT]) {
        if (tt == 0) {  // before this chunk's stores
          settle_tile_syms(nx);
          settle_lane(vm);
          settle_lane(vgn);
        }
        {  // staged through LDS: the consumed symbol tile (E = N) or the wave's staging area
          float *stage = E < N ? reinterpret_cast<float *>(sb + tile_sym_bytes(E)) : reinterpret_cast<float *>(sb) - 4;
          if (rem >= kTileWindows * N)
            store_tile_whole<NT>(win0, acc, stage, h, col, lane, cs.out);
          else
            store_tile_staged<NT>(win0, acc, stage, h, col, lane, rem, cs.out);
        }
      };
      tile_contract_emit<PREC, NT>(sb, base, h, col, S, E, valid > 0, Bs, RS, dt.rb + book * E,
                                   dt.tv + book * n_rows * 256, dt.tz + book * n_rows * 256,
                                   dt.pq + book * n_rows * 256, n_rows, gamma, cs, emit);
      wave_sync_lds();
    }
    settle_tile_syms(nx);
    settle_lane(vm);
    settle_lane(vgn);
    cur = nx;
    cm = nm;
    nm = meta_from_lanes(vm, cmm < n_chunks);
    c = cn;
    cn = cmm;
    vg = vgn;
  }
}

template <int PREC, int NT>
int launch_t(const fptc_batch &b, const fptc_codec &c, const Shape &sh, const Plan &p, const uint8_t *symbols,
             const float *gamma, float *out, void *stream) {
  constexpr int N = NT * 32;
  const int S = (c.E + 15) / 16, Kp = S * 16;
  const size_t lds = mfma_lds_bytes(Traits<PREC>::kBPieces, N, Kp, c.n_books, c.n_rows, c.E);
  auto kern = k_dqidct_mfma<PREC, NT>;
  const int per_cu = (int)((160 * 1024) / lds);
  int blocks = sh.blocks > 0 ? sh.blocks : device_cu_count() * (per_cu < 1 ? 1 : (per_cu > 8 ? 8 : per_cu));
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(kThreads), lds, (hipStream_t)stream, b, c.E, S, c.n_books, c.n_rows,
                     c.deq_val, c.deq_zone, c.row_of_bin, c.basis, p.hdr, p.chunk_meta, symbols, gamma, out);
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

template <int PREC>
int attrs_prec() {
  return lds_attr(k_dqidct_mfma<PREC, 1>) | lds_attr(k_dqidct_mfma<PREC, 2>) | lds_attr(k_dqidct_mfma<PREC, 4>);
}

}  // namespace

int set_dqidct_mfma_attributes() {
  return attrs_prec<FPTC_FP16>() | attrs_prec<FPTC_FP16X2>() | attrs_prec<FPTC_BF16>() | attrs_prec<FPTC_BF16X3>();
}

bool mfma_supported(int N, int E, int precision, int n_books, int n_rows) {
  if (precision < FPTC_FP16 || precision > FPTC_BF16X3) return false;
  if (N != 32 && N != 64 && N != 128) return false;
  if (E < 1 || E > N) return false;
  // LDS: basis pieces, tables and the waves' symbol tiles must fit in 160 KB
  const int Kp = (E + 15) / 16 * 16;
  const int pieces = precision == FPTC_BF16X3 ? 3 : (precision == FPTC_FP16X2 ? 2 : 1);
  return mfma_lds_bytes(pieces, N, Kp, n_books, n_rows, E) <= 160 * 1024;
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
