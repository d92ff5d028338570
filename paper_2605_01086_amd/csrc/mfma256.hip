// Window 256 on the matrix cores: the split IDCT basis (256 x 256 in two or
// three 16-bit pieces) does not fit in LDS, so a workgroup stages it 64 bins
// at a time and every wave's 32-window tile accumulates over the staged
// blocks.  Same operand splitting, bin-to-k-slot map and accumulation order
// (k-steps from the highest bins down) as the resident kernels.
//
// Both kernels keep their loops uniform across the workgroup: every wave
// reaches every barrier, with idle waves (no chunk or tile) skipping only the
// arithmetic.
#include <hip/hip_runtime.h>

#include "decode_common.h"
#include "fptc_internal.h"
#include "mfma_common.h"

namespace fptc {
namespace {

constexpr int N256 = 256, NT256 = 8;
constexpr int kSB = 4;                 // k-steps per staged block (64 bins)
constexpr int kRSB = 16 * kSB + 8;     // LDS row stride of a staged block, in halves
constexpr int kMaxWaves256 = 8;

__host__ __device__ constexpr size_t a16(size_t x) { return (x + 15) & ~(size_t)15; }

__host__ __device__ inline size_t block_basis_bytes(int bpieces) { return (size_t)bpieces * N256 * kRSB * 2; }

// Stage k-steps [s0, s0 + kSB) of the split basis: for lane half h the bins
// h*KH + 8 s + j, stored at row n, column h*8*kSB + 8 (s - s0) + j.
template <int PREC>
__device__ inline void stage_basis_block(uint16_t *Bb, const float *basis, int E, int KH, int s0, int tid,
                                         int nthreads) {
  using T = Traits<PREC>;
  constexpr int BP = T::kBPieces;
  const float bscale = T::kF16 ? kBasisScaleF16 : 1.0f;
  constexpr int W = 16 * kSB;
  for (int i = tid; i < N256 * W; i += nthreads) {
    const int n = i % N256, r = i / N256;  // consecutive threads read consecutive n of one basis row
    const int h = r / (8 * kSB), o = r % (8 * kSB);
    const int k = h * KH + 8 * s0 + o;
    const float v = k < E ? basis[(int64_t)k * N256 + n] * bscale : 0.0f;
    uint16_t pc[BP];
    split<T::kF16, BP>(v, pc);
#pragma unroll
    for (int p = 0; p < BP; ++p) Bb[(p * N256 + n) * kRSB + r] = pc[p];
  }
}

constexpr int kMaxBlocks256 = (N256 / 16 + kSB - 1) / kSB;  // staged blocks at E = 256

// The split basis of every staged block, written once per call into the
// workspace in the exact LDS image of the block, so that staging a block in
// the main kernels is a plain 16-byte copy.  One workgroup per block.
template <int PREC>
__global__ void __launch_bounds__(256) k_split_basis256(const float *__restrict__ basis, int E, int KH,
                                                        uint16_t *bsplit) {
  using T = Traits<PREC>;
  const int blk = blockIdx.x;
  stage_basis_block<PREC>(bsplit + (size_t)blk * (block_basis_bytes(T::kBPieces) / 2), basis, E, KH, blk * kSB,
                          threadIdx.x, blockDim.x);
}

// Copy one staged block (bytes a multiple of 16) from the workspace to LDS.
__device__ inline void copy_basis_block(uint16_t *Bb, const uint16_t *__restrict__ src, int bytes, int tid,
                                        int nthreads) {
  const uint4 *s4 = reinterpret_cast<const uint4 *>(src);
  uint4 *d4 = reinterpret_cast<uint4 *>(Bb);
  for (int i = tid; i < bytes / 16; i += nthreads) d4[i] = s4[i];
}

// Contract k-steps [s0, s1) of one 32-window tile against the staged block;
// symbols come from `sym(k0)`: the 8 symbols of bins k0 .. k0 + 7, byte j of
// the pair being bin k0 + j.  (The pre-split table of the resident kernels
// is not used here: with eight 32-row output tiles the accumulators already
// take half of the 256 registers a wave has at eight waves per block.)
template <int PREC, typename SymFn>
__device__ inline void contract_block256(f16v (&acc)[NT256], const uint16_t *Bb, int s0, int s1, int KH, int h,
                                         int col, int E, bool valid, const uint8_t *rb, const float *tv,
                                         const uint8_t *tz, bool scaled, float g0, float g1, float g2, SymFn sym) {
  using T = Traits<PREC>;
  constexpr int AP = T::kAPieces;
#pragma unroll 1
  for (int s = s1 - 1; s >= s0; --s) {
    const int k0 = h * KH + 8 * s;
    const uint2 u = sym(k0);
    uint8_t sy[8];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      sy[j] = (uint8_t)(u.x >> (8 * j));
      sy[4 + j] = (uint8_t)(u.y >> (8 * j));
    }
    u8v a[AP];
    const bool r = dequant8<PREC>(sy, k0, E, valid, rb, tv, tz, scaled, g0, g1, g2, a);
    const bool any_rest = AP > 1 && __any(r);
    mfma_step<PREC, NT256>(acc, a, Bb + col * kRSB + h * 8 * kSB + 8 * (s - s0), 32 * kRSB, N256 * kRSB, any_rest);
  }
}

// ---------------------------------------------------------------- split path
template <int PREC>
__global__ void __launch_bounds__(kMaxWaves256 * 64) k_dqidct_mfma256(fptc_batch b, int E, int S, int n_books,
                                                                       int n_rows, const float *deq_val,
                                                                       const uint8_t *deq_zone,
                                                                       const uint8_t *row_of_bin,
                                                                       const uint16_t *__restrict__ bsplit,
                                                                       const int64_t *hdr, const int64_t *win_off,
                                                                       const int32_t *tile_stream,
                                                                       const uint8_t *symbols, const float *__restrict__ gamma,
                                                                       float *out) {
  using T = Traits<PREC>;
  extern __shared__ __align__(16) unsigned char lds[];
  const int nthreads = blockDim.x, waves = nthreads >> 6;
  uint16_t *Bb = reinterpret_cast<uint16_t *>(lds);
  float *Tv = reinterpret_cast<float *>(lds + block_basis_bytes(T::kBPieces));
  uint8_t *Tz = reinterpret_cast<uint8_t *>(Tv + n_books * n_rows * 256);
  uint8_t *Rb = Tz + n_books * n_rows * 256;
  for (int i = threadIdx.x; i < n_books * n_rows * 256; i += nthreads) {
    Tv[i] = deq_val[i];
    const int z = deq_zone[i];
    Tz[i] = (uint8_t)(z < 2 ? z : 2);
  }
  for (int i = threadIdx.x; i < n_books * E; i += nthreads) {
    const int r = row_of_bin[i];
    Rb[i] = (uint8_t)(r < n_rows ? r : n_rows - 1);
  }
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63, col = lane & 31, h = lane >> 5;
  const int KH = S * 8, nblk = (S + kSB - 1) / kSB;
  const int64_t n_win = hdr[1];
  const int64_t n_tiles = (n_win + kTileWindows - 1) / kTileWindows;
  const float oscale = 1.0f / (T::kF16 ? kBasisScaleF16 : 1.0f);

  for (int64_t t0 = (int64_t)blockIdx.x * waves; t0 < n_tiles; t0 += (int64_t)gridDim.x * waves) {
    const int64_t tile = t0 + wid;
    const int64_t g = tile * kTileWindows + col;
    int valid = 0, book = 0;
    int64_t obase = 0;
    float g0 = 1.0f, g1 = 1.0f, g2 = 1.0f;
    if (tile < n_tiles && g < n_win) {
      int s = tile_stream[tile];
      s = s < 0 ? 0 : (s >= b.n_streams ? b.n_streams - 1 : s);
      while (s + 1 < b.n_streams && win_off[s + 1] <= g) ++s;
      const int64_t j = g - win_off[s];
      const int64_t L = b.sample_off[s + 1] - b.sample_off[s];
      const int64_t o = b.sample_off[s] + j * N256;
      int64_t v = L - j * N256;
      v = v < N256 ? v : N256;
      if (o < 0 || o + v > b.n_samples || j < 0) v = 0;
      valid = v > 0 ? (int)v : 0;
      obase = o;
      const int bk = b.book_id ? (int)b.book_id[s] : 0;
      book = bk < n_books ? bk : 0;
      if (gamma) {
        g0 = gamma[3 * (int64_t)s];
        g1 = gamma[3 * (int64_t)s + 1];
        g2 = gamma[3 * (int64_t)s + 2];
      }
    }
    f16v acc[NT256];
#pragma unroll
    for (int t = 0; t < NT256; ++t)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[t][r] = 0.0f;
    const int64_t sbase = g * (int64_t)E;
    auto sym = [&](int k0) {
      uint32_t w[2] = {0u, 0u};
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int64_t si = sbase + k0 + j;
        const uint32_t v = (valid > 0 && k0 + j < E && si < b.n_symbols) ? symbols[si] : 128u;
        w[j >> 2] |= v << (8 * (j & 3));
      }
      return make_uint2(w[0], w[1]);
    };
    for (int blk = nblk - 1; blk >= 0; --blk) {
      __syncthreads();
      copy_basis_block(Bb, bsplit + (size_t)blk * (block_basis_bytes(T::kBPieces) / 2),
                       (int)block_basis_bytes(T::kBPieces), threadIdx.x, nthreads);
      __syncthreads();
      const int s1 = min(S, (blk + 1) * kSB);
      contract_block256<PREC>(acc, Bb, blk * kSB, s1, KH, h, col, E, valid > 0, Rb + book * E,
                              Tv + book * n_rows * 256, Tz + book * n_rows * 256, gamma != nullptr, g0, g1, g2, sym);
    }
    // the tile's windows may belong to different streams: each lane takes the
    // output offset and length of the windows it holds from their own lanes
    const int ob_lo = (int)(uint32_t)obase, ob_hi = (int)(obase >> 32);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int w = acc_window(r, h);
      const int v_w = __shfl(valid, w);
      const int64_t ob_w = ((int64_t)__shfl(ob_hi, w) << 32) | (int64_t)(uint32_t)__shfl(ob_lo, w);
#pragma unroll
      for (int t = 0; t < NT256; ++t) {
        const int n = 32 * t + col;
        if (n < v_w) out[ob_w + n] = acc[t][r] * oscale;
      }
    }
  }
}

// ---------------------------------------------------------------- fused path
// Dequantization tables: values, zones, row of each bin.
__host__ __device__ inline size_t table256_bytes(int bp, int n_books, int n_rows, int E) {
  (void)bp;
  return a16((size_t)n_books * n_rows * 256 * 5 + (size_t)n_books * E);
}

__host__ __device__ inline size_t wave256_bytes(int wpc, int E) { return (size_t)kSymPrefix + a16((size_t)wpc * E + 16); }

// LDS: lookup tables | staged basis block | dequantization tables | wave
// buffers; the multi-symbol build borrows lut1_temp_bytes after the tables.
__host__ __device__ inline size_t fused256_lds_ms(bool ms, int bp, int n_books, int lmax, int E, int wpc, int waves,
                                                  int n_rows) {
  const size_t t = lut_lds_bytes(ms, n_books, lmax);
  const size_t need = t + block_basis_bytes(bp) + table256_bytes(bp, n_books, n_rows, E) +
                      (size_t)waves * wave256_bytes(wpc, E);
  const size_t tmp = ms ? t + lut1_temp_bytes(n_books, lmax) : 0;
  return need > tmp ? need : tmp;
}

template <int PREC, bool MS>
__global__ void __launch_bounds__(kMaxWaves256 * 64) k_fused256(const uint64_t *__restrict__ words,
                                                                 const uint8_t *__restrict__ symlen, int n_streams,
                                                                 int E, int S, int lmax, int n_books, int n_rows,
                                                                 int wpc, const uint16_t *__restrict__ lut_g,
                                                                 const float *__restrict__ deq_val,
                                                                 const uint8_t *__restrict__ deq_zone,
                                                                 const uint8_t *__restrict__ row_of_bin,
                                                                 const uint16_t *__restrict__ bsplit,
                                                                 const int64_t *__restrict__ hdr,
                                                                 const ChunkMeta *__restrict__ meta,
                                                                 const float *__restrict__ gamma, float *out,
                                                                 int32_t *status) {
  using T = Traits<PREC>;
  extern __shared__ __align__(16) unsigned char lds[];
  const int nthreads = blockDim.x, waves = nthreads >> 6;
  const size_t lut_bytes = lut_lds_bytes(MS, n_books, lmax);
  uint16_t *Bb = reinterpret_cast<uint16_t *>(lds + lut_bytes);
  float *Tv = reinterpret_cast<float *>(reinterpret_cast<unsigned char *>(Bb) + block_basis_bytes(T::kBPieces));
  uint8_t *Tz = reinterpret_cast<uint8_t *>(Tv + n_books * n_rows * 256);
  uint8_t *Rb = Tz + n_books * n_rows * 256;
  unsigned char *wave_base = reinterpret_cast<unsigned char *>(Tv) + table256_bytes(T::kBPieces, n_books, n_rows, E);
  stage_decode_tables(MS, lds, lds + lut_bytes, lut_g, lmax, n_books, threadIdx.x, nthreads);
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
  const bool e_vec = (E % 16) == 0;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63, col = lane & 31, h = lane >> 5;
  unsigned char *sb = wave_base + (size_t)wid * wave256_bytes(wpc, E) + kSymPrefix;
  const uint8_t *cl = lds + ((size_t)n_books << lmax) * 4;
  const uint32_t *binfo = reinterpret_cast<const uint32_t *>(cl + n_books * 256);  // multi-symbol form only
  const int hs = 32 - lmax;
  const int KH = S * 8, nblk = (S + kSB - 1) / kSB;
  const int ntile_max = (wpc + kTileWindows - 1) / kTileWindows;
  const float oscale = 1.0f / (T::kF16 ? kBasisScaleF16 : 1.0f);
  const int64_t n_chunks = hdr[0];
  const int64_t cstride = (int64_t)gridDim.x * waves;

  // Software pipeline over this wave's chunks (see the resident fused
  // kernel): next chunk's words requested before this chunk decodes, waited
  // for right after the decode, before this chunk's stores.
  ChunkMeta cm, nm;
  ChunkWords cw{};
  {
    const int64_t c = (int64_t)blockIdx.x * waves + wid;
    cm = meta_from_lanes(load_meta_lane(meta, c, n_chunks, lane), c < n_chunks);
    const uint32_t vn = load_meta_lane(meta, c + cstride, n_chunks, lane);
    if (c < n_chunks) load_chunk_words(words, symlen, cm.first_word, cm.word_end, lane, cw);
    nm = meta_from_lanes(vn, c + cstride < n_chunks);
  }
  for (int64_t c0 = (int64_t)blockIdx.x * waves; c0 < n_chunks; c0 += cstride) {
    const int64_t c = c0 + wid;
    const bool active = c < n_chunks && cm.first_word >= 0;
    const int s = cm.stream < 0 ? 0 : (cm.stream >= n_streams ? n_streams - 1 : cm.stream);
    const int book = cm.book < n_books && cm.book >= 0 ? cm.book : 0;
    const int w_cnt = active ? cm.n_windows : 0;
    const float vg = load_gamma_lane(active ? gamma : nullptr, s, lane);
    const uint32_t vm = load_meta_lane(meta, c + 2 * cstride, n_chunks, lane);
    ChunkWords nx{};
    if (c + cstride < n_chunks) load_chunk_words(words, symlen, nm.first_word, nm.word_end, lane, nx);
    int err = 0;
    if (active) {
      const void *lb = MS ? (const void *)(reinterpret_cast<const uint32_t *>(lds) + (book << lmax))
                          : (const void *)(reinterpret_cast<const uint16_t *>(lds) + (book << lmax));
      err = decode_chunk<MS>(words, symlen, cm.first_word, cm.first_sym, w_cnt * E, cm.word_end, cw, lb,
                             cl + book * 256, MS ? binfo[book] : 0u, hs, sb, lane);
    }
    settle_chunk_words(nx);
    settle_lane(vm);
    settle_lane(vg);
    const ChunkMeta mm = meta_from_lanes(vm, c + 2 * cstride < n_chunks);
    cw = nx;
    if (err && status) atomicOr(&status[s], err);
    const float g0 = lane_float(vg, 0), g1 = lane_float(vg, 1), g2 = lane_float(vg, 2);
    wave_sync_lds();
    for (int tt = 0; tt < ntile_max; ++tt) {
      const int wr = tt * kTileWindows + col;
      const int valid = wr < w_cnt ? min(N256, cm.out_len - wr * N256) : 0;
      const int base = (wr < w_cnt ? wr : (w_cnt > 0 ? w_cnt - 1 : 0)) * E;
      f16v acc[NT256];
#pragma unroll
      for (int t = 0; t < NT256; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[t][r] = 0.0f;
      const bool tile_active = tt * kTileWindows < w_cnt;
      auto sym = [&](int k0) {
        if (e_vec) return *reinterpret_cast<const uint2 *>(sb + base + k0);
        uint32_t w[2] = {0u, 0u};
#pragma unroll
        for (int j = 0; j < 8; ++j) w[j >> 2] |= (uint32_t)sb[base + (k0 + j < E ? k0 + j : 0)] << (8 * (j & 3));
        return make_uint2(w[0], w[1]);
      };
      for (int blk = nblk - 1; blk >= 0; --blk) {
        __syncthreads();
        copy_basis_block(Bb, bsplit + (size_t)blk * (block_basis_bytes(T::kBPieces) / 2),
                       (int)block_basis_bytes(T::kBPieces), threadIdx.x, nthreads);
        __syncthreads();
        if (tile_active)
          contract_block256<PREC>(acc, Bb, blk * kSB, min(S, (blk + 1) * kSB), KH, h, col, E, valid > 0,
                                  Rb + book * E, Tv + book * n_rows * 256, Tz + book * n_rows * 256,
                                  gamma != nullptr, g0, g1, g2, sym);
      }
      float *win0 = out + cm.out_base + (int64_t)tt * kTileWindows * N256;
      const int rem = tile_active ? cm.out_len - tt * kTileWindows * N256 : 0;
      if (E == N256 && wpc >= kTileWindows && tile_active) {  // stage through the consumed symbol buffer
        if (rem >= kTileWindows * N256)
          store_tile_whole<NT256>(win0, acc, reinterpret_cast<float *>(sb) - 4, h, col, lane, oscale);
        else
          store_tile_staged<NT256>(win0, acc, reinterpret_cast<float *>(sb) - 4, h, col, lane, rem, oscale);
      } else {
#pragma unroll
        for (int t = 0; t < NT256; ++t) store_rows(win0, N256, acc[t], t, h, col, rem, oscale);
      }
    }
    wave_sync_lds();
    cm = nm;
    nm = mm;
  }
}

int pieces(int precision) { return precision == FPTC_BF16X3 ? 3 : (precision == FPTC_FP16X2 ? 2 : 1); }

size_t split256_lds(int bp, const fptc_codec &c) {
  return block_basis_bytes(bp) + a16((size_t)c.n_books * c.n_rows * 256 * 5 + (size_t)c.n_books * c.E);
}

size_t fused256_lds(int bp, const fptc_codec &c, int wpc, int waves, int n_rows) {
  return fused256_lds_ms(false, bp, c.n_books, c.lmax, c.E, wpc, waves, n_rows);
}

template <int PREC>
int attrs_prec() {
  return lds_attr(k_dqidct_mfma256<PREC>) | lds_attr(k_fused256<PREC, true>) | lds_attr(k_fused256<PREC, false>);
}

// Split the basis into the workspace (one workgroup per staged block).
template <int PREC>
int split_basis(const fptc_codec &c, int S, const Plan &p, void *stream) {
  const int nblk = (S + kSB - 1) / kSB;
  hipLaunchKernelGGL(k_split_basis256<PREC>, dim3(nblk), dim3(256), 0, (hipStream_t)stream, c.basis, c.E, S * 8,
                     p.basis_split);
  return (int)hipGetLastError();
}

template <int PREC>
int launch_split(const fptc_batch &b, const fptc_codec &c, const Shape &sh, const Plan &p, const uint8_t *symbols,
                 const float *gamma, float *out, void *stream) {
  const int S = (c.E + 15) / 16;
  int rc = split_basis<PREC>(c, S, p, stream);
  if (rc) return rc;
  const size_t lds = split256_lds(Traits<PREC>::kBPieces, c);
  const int per_cu = (int)((160 * 1024) / lds);
  const int blocks = sh.blocks > 0 ? sh.blocks : device_cu_count() * (per_cu < 1 ? 1 : per_cu);
  hipLaunchKernelGGL(k_dqidct_mfma256<PREC>, dim3(blocks), dim3(kMaxWaves256 * 64), lds, (hipStream_t)stream, b,
                     c.E, S, c.n_books, c.n_rows, c.deq_val, c.deq_zone, c.row_of_bin, p.basis_split, p.hdr, p.win_off,
                     p.tile_stream, symbols, gamma, out);
  return (int)hipGetLastError();
}

template <int PREC, bool MS>
int launch_fused_t(const fptc_batch &b, const fptc_codec &c, const Shape &sh, const Plan &p, const float *gamma,
                   float *out, int32_t *status, void *stream) {
  const int S = (c.E + 15) / 16;
  int rc = split_basis<PREC>(c, S, p, stream);
  if (rc) return rc;
  const size_t lds = fused256_lds_ms(MS, Traits<PREC>::kBPieces, c.n_books, c.lmax, c.E, sh.wpc, sh.waves, c.n_rows);
  const int per_cu = (int)((160 * 1024) / lds);
  const int blocks = sh.blocks > 0 ? sh.blocks : device_cu_count() * (per_cu < 1 ? 1 : per_cu);
  auto kern = k_fused256<PREC, MS>;
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(sh.waves * 64), lds, (hipStream_t)stream, b.words,
                     b.symlen, b.n_streams, c.E, S, c.lmax, c.n_books, c.n_rows, sh.wpc, c.lut, c.deq_val,
                     c.deq_zone, c.row_of_bin, p.basis_split, p.hdr, p.chunk_meta, gamma, out, status);
  return (int)hipGetLastError();
}

// Multi-symbol decode tables when they fit beside everything else.
template <int PREC>
int launch_fused_ms(const fptc_batch &b, const fptc_codec &c, const Shape &sh, const Plan &p, const float *gamma,
                    float *out, int32_t *status, void *stream) {
  if (fused256_lds_ms(true, Traits<PREC>::kBPieces, c.n_books, c.lmax, c.E, sh.wpc, sh.waves, c.n_rows) <=
      160 * 1024)
    return launch_fused_t<PREC, true>(b, c, sh, p, gamma, out, status, stream);
  return launch_fused_t<PREC, false>(b, c, sh, p, gamma, out, status, stream);
}

}  // namespace

int set_mfma256_attributes() {
  return attrs_prec<FPTC_FP16>() | attrs_prec<FPTC_FP16X2>() | attrs_prec<FPTC_BF16>() | attrs_prec<FPTC_BF16X3>();
}

bool mfma256_supported(int E, int precision) {
  if (precision < FPTC_FP16 || precision > FPTC_BF16X3) return false;
  return E >= 1 && E <= N256;
}

size_t basis_split256_bytes(int N) { return N == N256 ? (size_t)kMaxBlocks256 * block_basis_bytes(3) : 0; }

bool fused256_supported(const fptc_codec &c, int precision, int wpc, int waves) {
  if (!mfma256_supported(c.E, precision) || waves < 1 || waves > kMaxWaves256) return false;
  return fused256_lds(pieces(precision), c, wpc, waves, c.n_rows) <= 160 * 1024;
}

int launch_dqidct_mfma256(const fptc_batch &b, const fptc_codec &c, const Shape &s, const Plan &p,
                          const uint8_t *symbols, const float *gamma, int precision, float *out, void *stream) {
  switch (precision) {
    case FPTC_FP16: return launch_split<FPTC_FP16>(b, c, s, p, symbols, gamma, out, stream);
    case FPTC_FP16X2: return launch_split<FPTC_FP16X2>(b, c, s, p, symbols, gamma, out, stream);
    case FPTC_BF16: return launch_split<FPTC_BF16>(b, c, s, p, symbols, gamma, out, stream);
    case FPTC_BF16X3: return launch_split<FPTC_BF16X3>(b, c, s, p, symbols, gamma, out, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

int launch_fused256(const fptc_batch &b, const fptc_codec &c, const Shape &s, const Plan &p, const float *gamma,
                    int precision, float *out, int32_t *status, void *stream) {
  switch (precision) {
    case FPTC_FP16: return launch_fused_ms<FPTC_FP16>(b, c, s, p, gamma, out, status, stream);
    case FPTC_FP16X2: return launch_fused_ms<FPTC_FP16X2>(b, c, s, p, gamma, out, status, stream);
    case FPTC_BF16: return launch_fused_ms<FPTC_BF16>(b, c, s, p, gamma, out, status, stream);
    case FPTC_BF16X3: return launch_fused_ms<FPTC_BF16X3>(b, c, s, p, gamma, out, status, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

}  // namespace fptc
