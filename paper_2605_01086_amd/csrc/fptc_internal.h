// Internal declarations shared by the library's translation units: the
// workspace layout of a plan and the kernel launchers.  Not part of the ABI.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "../../include/fptc.h"

namespace fptc {

constexpr int kWave = 64;
constexpr int kDefaultWindowsPerChunk = 32;
constexpr int kDefaultWavesPerBlock = 4;
constexpr int kDefaultChunkGroup = 4;
constexpr int kMaxBooks = 8;
constexpr int kMaxRows = 4;
constexpr int kMaxLmax = 16;  // codes above 12 bits decode through two-level tables
constexpr int kTileWindows = 32;  // windows per MFMA tile (one 32x32 output block per wave)

// Everything a wavefront needs to decode one chunk, written by the plan.
struct ChunkMeta {
  // the whole record is written once, by the plan's chunk-start pass
  int64_t first_word;  // global index of the first word holding a symbol of the chunk; -1 = skip
  int32_t first_sym;   // chunk-relative index of the first word's first symbol (<= 0)
  int32_t last;        // 1 for a stream's last chunk
  // The chunk's words end at the next chunk's first word (inclusive when that
  // chunk starts inside it); a stream's last chunk ends at word_end, the end
  // of the stream's words.
  int64_t word_end;
  int64_t sym_base;    // global index of the chunk's first decoded symbol
  int64_t out_base;    // global index of the chunk's first output sample
  int32_t n_windows;   // windows in the chunk
  int32_t out_len;     // output samples of the chunk
  int32_t stream;
  int32_t book;
  int32_t pad[2];
};
static_assert(sizeof(ChunkMeta) == 64, "ChunkMeta is one 64-byte record");

// Resolved launch shape (defaults applied, validated).
struct Shape {
  int wpc;     // windows per chunk
  int waves;   // waves per block
  int blocks;  // persistent grid size (0 = launcher decides)
  int group;   // fused schedule: adjacent chunks per group
  bool auto_waves;  // waves_per_block was 0: each call may pick its own
};

// Workspace layout of a plan.  Every section starts on a 256-byte boundary.
//   hdr        int64[8]     [0] = chunk count, [1] = window count,
//                           [2] = segment count, [3] = segment capacity
//   win_off    int64[n+1]   exclusive prefix of ceil(L_s / N)
//   chunk_off  int64[n+1]   exclusive prefix of ceil(n_win_s / wpc) (0 for streams
//                           flagged by the stream pass)
//   seg_off    int64[n+1]   exclusive prefix of each stream's segment pieces
//   seg_map    int32[scap*2] stream and segment of each piece
//   gseg_sum   int32[nseg]  symbols of each 4096-word segment of the batch
//   gseg_lane  int32[nseg*64] exclusive prefix of its 64-word blocks
//   bwd_part   double[cap*3] backward partial sums per chunk and zone
//   chunk_meta ChunkMeta[cap] per-chunk decode record
struct Layout {
  size_t hdr, win_off, chunk_off, seg_off, bwd_part, seg_map, gseg_sum, gseg_lane, chunk_meta, total;
  int64_t chunk_cap, seg_cap, n_gseg;
};

Layout layout_for(const fptc_batch *b, const fptc_codec *c, const Shape &s);

// Pointers into a workspace.
struct Plan {
  int64_t *hdr;
  int64_t *win_off;
  int64_t *chunk_off;
  double *bwd_part;
  int64_t *seg_off;     // [n_streams + 1] symlen segments per stream, prefix
  int32_t *seg_map;     // [seg_cap * 2] stream and segment of each piece (a stream's words in one segment)
  int32_t *gseg_sum;    // [n_gseg] symbols of each segment of the batch
  int32_t *gseg_lane;   // [n_gseg * 64] exclusive prefix of each segment's 64-word blocks
  ChunkMeta *chunk_meta;
  int64_t chunk_cap, seg_cap, n_gseg;
};

Plan plan_view(void *ws, const Layout &L);

// Kernel launchers (return hipError_t as int).
int launch_plan(const fptc_batch &b, const fptc_codec &c, const Shape &s, const Plan &p, int32_t *status,
                void *stream);
size_t decode_lds_bytes(const fptc_codec &c, const Shape &s);
int launch_decode(const fptc_batch &b, const fptc_codec &c, const Shape &s, const Plan &p, uint8_t *symbols,
                  int32_t *status, void *stream);
int launch_dqidct(const fptc_batch &b, const fptc_codec &c, const Shape &s, const Plan &p,
                  const uint8_t *symbols, const float *gamma, int precision, float *out, void *stream);

bool mfma_supported(int N, int E, int precision, int n_books, int n_rows);
int launch_dqidct_mfma(const fptc_batch &b, const fptc_codec &c, const Shape &s, const Plan &p,
                       const uint8_t *symbols, const float *gamma, int precision, float *out, void *stream);

bool fused_supported(int N, int E, int precision, int wpc, int waves, int n_books, int n_rows, int lmax);
int launch_fused(const fptc_batch &b, const fptc_codec &c, const Shape &s, const Plan &p, const float *gamma,
                 int precision, float *out, int32_t *status, void *stream);

bool mfma256_supported(const fptc_codec &c, int precision, int wpc);
bool fused256_supported(const fptc_codec &c, int precision, int wpc, int waves);
int launch_dqidct_mfma256(const fptc_batch &b, const fptc_codec &c, const Shape &s, const Plan &p,
                          const uint8_t *symbols, const float *gamma, int precision, float *out, void *stream);
int launch_fused256(const fptc_batch &b, const fptc_codec &c, const Shape &s, const Plan &p, const float *gamma,
                    int precision, float *out, int32_t *status, void *stream);

size_t bwd_lds_bytes(const fptc_codec &c, const Shape &s);
int launch_bwd(const fptc_batch &b, const fptc_codec &c, const Shape &s, const Plan &p, const uint8_t *symbols,
               const float *grad_out, float *grad_coeff, double *grad_gamma, void *stream);

int device_cu_count();

// Encode-side steps (train.hip).
int launch_fdct_quant(const fptc_batch &b, const fptc_quant_params &q, const double *tab, const int64_t *sym_off,
                      const float *x, uint8_t *symbols, double *coef, int64_t n_windows, void *stream);
int launch_histogram(const fptc_batch &b, const int64_t *sym_off, int n_books, const uint8_t *symbols,
                     uint64_t *counts, int64_t n_symbols, void *stream);
size_t percentile_ws_bytes();
int launch_abs_percentile(const double *coef, int64_t n_windows, int E, int k0, int k1, double q, double *out,
                          void *ws, void *stream);
int check_quant_params(const fptc_quant_params *q);  // host_tables.cpp

// Host-side checks and launches of the ABI calls, shared by the entry points
// (return fptc_status codes).  check_decompress resolves the launch shape of
// fptc_decompress_batch (waves included) and validates every argument that
// needs no workspace.
int check_decompress(const fptc_batch *batch, const fptc_codec *codec, const fptc_launch *launch, int32_t precision,
                     const float *out, Shape *s);
int launch_decompress(const fptc_batch &b, const fptc_codec &c, const Shape &s, const Plan &p, const float *gamma,
                      int32_t precision, float *out, int32_t *stream_status, void *stream);
int launch_plan_status(const fptc_batch &b, const fptc_codec &c, const Shape &s, const Plan &p, int32_t *status,
                       void *stream);

// Library set-up on the current device, once per device (thread-safe):
// kernel attributes (dynamic LDS up to 160 KB) for every kernel
// instantiation.  Every device entry point runs it before enqueueing, so the
// launches themselves are the only runtime calls a call makes afterwards.
int ensure_device_init();
int set_decode_attributes();
int set_dqidct_mfma_attributes();
int set_fused_attributes();
int set_mfma256_attributes();
int set_bwd_attributes();
int init_noalloc_scratch();  // the no-allocation entry point's static workspace

#ifdef __HIPCC__
// Allow a kernel the whole 160 KB of a CU's LDS as dynamic shared memory.
template <typename K>
int lds_attr(K kern) {
  return hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                             160 * 1024) == hipSuccess
             ? 0
             : 1;
}
#endif

}  // namespace fptc
