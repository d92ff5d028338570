// C ABI entry points of the device path: argument checks on the host, the
// workspace layout, and the launches.  Every check runs before anything is
// enqueued, so an error return leaves the stream untouched.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "fptc_internal.h"

namespace fptc {

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool valid_n(int32_t N) {
  return N == 4 || N == 8 || N == 16 || N == 32 || N == 64 || N == 128 || N == 256;
}

int check_batch(const fptc_batch *b) {
  if (!b || b->n_streams < 1 || b->n_words < 0 || b->n_symbols < 0 || b->n_samples < 0) return FPTC_ERR_INVALID_ARG;
  if (!b->word_off || !b->sample_off) return FPTC_ERR_INVALID_ARG;
  if (b->n_words > 0 && (!b->words || !b->symlen)) return FPTC_ERR_INVALID_ARG;
  return FPTC_OK;
}

int check_codec(const fptc_codec *c) {
  if (!c || !valid_n(c->N) || c->E < 1 || c->E > c->N) return FPTC_ERR_INVALID_ARG;
  if (c->lmax < 1 || c->lmax > kMaxLmax || c->n_books < 1 || c->n_books > kMaxBooks) return FPTC_ERR_INVALID_ARG;
  if (c->n_rows < 1 || c->n_rows > kMaxRows) return FPTC_ERR_INVALID_ARG;
  if (!c->lut || !c->deq_val || !c->deq_zone || !c->row_of_bin || !c->basis) return FPTC_ERR_INVALID_ARG;
  return FPTC_OK;
}

int resolve_shape(const fptc_launch *l, const fptc_codec *c, Shape *s) {
  s->wpc = (l && l->windows_per_chunk) ? l->windows_per_chunk : kDefaultWindowsPerChunk;
  s->waves = (l && l->waves_per_block) ? l->waves_per_block : kDefaultWavesPerBlock;
  s->auto_waves = !(l && l->waves_per_block);
  s->blocks = l ? l->blocks : 0;
  s->group = (l && l->chunk_group) ? l->chunk_group : kDefaultChunkGroup;
  if (s->wpc < 1 || s->wpc > 1024 || s->waves < 1 || s->waves > 16 || s->blocks < 0) return FPTC_ERR_INVALID_ARG;
  if (s->group < 1 || s->group > 64) return FPTC_ERR_INVALID_ARG;
  (void)c;
  return FPTC_OK;
}

int status_of(int hip_err) { return hip_err == 0 ? FPTC_OK : FPTC_ERR_HIP; }

}  // namespace

Layout layout_for(const fptc_batch *b, const fptc_codec *c, const Shape &s) {
  Layout L{};
  const int64_t n = b->n_streams;
  const int64_t max_windows = b->n_symbols / c->E;
  L.chunk_cap = (max_windows + s.wpc - 1) / s.wpc + n + 1;
  size_t off = 0;
  L.hdr = off;
  off = align256(off + 8 * sizeof(int64_t));
  L.win_off = off;
  off = align256(off + (n + 1) * sizeof(int64_t));
  L.chunk_off = off;
  off = align256(off + (n + 1) * sizeof(int64_t));
  L.seg_off = off;
  off = align256(off + (n + 1) * sizeof(int64_t));
  // a stream's pieces are the 4096-word segments of the batch its words
  // touch: with disjoint word ranges at most n_words / 4096 + 2 n in all
  L.seg_cap = b->n_words / 4096 + 2 * n + 1;
  L.n_gseg = (b->n_words + 4095) / 4096;
  L.seg_map = off;
  off = align256(off + L.seg_cap * 2 * sizeof(int32_t));
  L.gseg_sum = off;
  off = align256(off + L.n_gseg * sizeof(int32_t));
  L.gseg_lane = off;
  off = align256(off + L.n_gseg * 64 * sizeof(int32_t));
  L.bwd_part = off;
  off = align256(off + L.chunk_cap * 3 * sizeof(double));
  L.chunk_meta = off;
  off = align256(off + L.chunk_cap * sizeof(ChunkMeta));
  L.total = off;
  return L;
}

Plan plan_view(void *ws, const Layout &L) {
  char *p = static_cast<char *>(ws);
  Plan v;
  v.hdr = reinterpret_cast<int64_t *>(p + L.hdr);
  v.win_off = reinterpret_cast<int64_t *>(p + L.win_off);
  v.chunk_off = reinterpret_cast<int64_t *>(p + L.chunk_off);
  v.bwd_part = reinterpret_cast<double *>(p + L.bwd_part);
  v.chunk_meta = reinterpret_cast<ChunkMeta *>(p + L.chunk_meta);
  v.seg_off = reinterpret_cast<int64_t *>(p + L.seg_off);
  v.seg_map = reinterpret_cast<int32_t *>(p + L.seg_map);
  v.gseg_sum = reinterpret_cast<int32_t *>(p + L.gseg_sum);
  v.gseg_lane = reinterpret_cast<int32_t *>(p + L.gseg_lane);
  v.chunk_cap = L.chunk_cap;
  v.seg_cap = L.seg_cap;
  v.n_gseg = L.n_gseg;
  return v;
}

int device_cu_count() {
  // Cached per device; guarded because several host threads may launch.
  static std::mutex mu;
  static std::vector<int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  std::lock_guard<std::mutex> g(mu);
  if ((int)cache.size() <= dev) cache.resize(dev + 1, 0);
  if (!cache[dev]) {
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0) cu = 256;
    cache[dev] = cu;
  }
  return cache[dev];
}

int check_decompress(const fptc_batch *batch, const fptc_codec *codec, const fptc_launch *launch, int32_t precision,
                     const float *out, Shape *s) {
  int rc;
  if ((rc = check_batch(batch)) || (rc = check_codec(codec)) || (rc = resolve_shape(launch, codec, s))) return rc;
  if (!out && batch->n_samples > 0) return FPTC_ERR_INVALID_ARG;
  if (precision < FPTC_FP32_SIMT || precision > FPTC_BF16X3) return FPTC_ERR_INVALID_ARG;
  const bool wide = codec->N == 256;
  auto fits = [&](int waves) {
    return wide ? fused256_supported(*codec, precision, s->wpc, waves)
                : fused_supported(codec->N, codec->E, precision, s->wpc, waves, codec->n_books, codec->n_rows,
                                  codec->lmax);
  };
  if (s->auto_waves) {  // the most waves (up to 16; 8 at N = 128 and 256) whose LDS fits
    s->waves = wide ? 8 : 16;
    while (s->waves > 1 && !fits(s->waves)) --s->waves;
  }
  if (!fits(s->waves)) return FPTC_ERR_UNSUPPORTED;
  return FPTC_OK;
}

int launch_decompress(const fptc_batch &b, const fptc_codec &c, const Shape &s, const Plan &p, const float *gamma,
                      int32_t precision, float *out, int32_t *stream_status, void *stream) {
  if (c.N == 256) return status_of(launch_fused256(b, c, s, p, gamma, precision, out, stream_status, stream));
  return status_of(launch_fused(b, c, s, p, gamma, precision, out, stream_status, stream));
}

int launch_plan_status(const fptc_batch &b, const fptc_codec &c, const Shape &s, const Plan &p, int32_t *status,
                       void *stream) {
  return status_of(launch_plan(b, c, s, p, status, stream));
}

}  // namespace fptc

using namespace fptc;

extern "C" {

int32_t fptc_init(void) { return ensure_device_init() ? FPTC_ERR_HIP : FPTC_OK; }

size_t fptc_workspace_size(const fptc_batch *batch, const fptc_codec *codec, const fptc_launch *launch) {
  Shape s;
  if (check_batch(batch) || check_codec(codec) || resolve_shape(launch, codec, &s)) return 0;
  return layout_for(batch, codec, s).total;
}

int32_t fptc_plan_batch(const fptc_batch *batch, const fptc_codec *codec, const fptc_launch *launch, void *ws,
                        size_t ws_bytes, int32_t *stream_status, void *stream) {
  Shape s;
  int rc;
  if ((rc = check_batch(batch)) || (rc = check_codec(codec)) || (rc = resolve_shape(launch, codec, &s))) return rc;
  if (!ws) return FPTC_ERR_INVALID_ARG;
  Layout L = layout_for(batch, codec, s);
  if (ws_bytes < L.total) return FPTC_ERR_WORKSPACE;
  if (ensure_device_init()) return FPTC_ERR_HIP;
  return status_of(launch_plan(*batch, *codec, s, plan_view(ws, L), stream_status, stream));
}

int32_t fptc_decode_batch(const fptc_batch *batch, const fptc_codec *codec, const fptc_launch *launch,
                          const void *ws, size_t ws_bytes, uint8_t *symbols_out, int32_t *stream_status,
                          void *stream) {
  Shape s;
  int rc;
  if ((rc = check_batch(batch)) || (rc = check_codec(codec)) || (rc = resolve_shape(launch, codec, &s))) return rc;
  if (!ws || (!symbols_out && batch->n_symbols > 0)) return FPTC_ERR_INVALID_ARG;
  if (s.auto_waves) {  // the most waves (up to 16) whose symbol buffers fit in LDS
    s.waves = 16;
    while (s.waves > 1 && decode_lds_bytes(*codec, s) > 160 * 1024) --s.waves;
  }
  if (decode_lds_bytes(*codec, s) > 160 * 1024) return FPTC_ERR_UNSUPPORTED;
  Layout L = layout_for(batch, codec, s);
  if (ws_bytes < L.total) return FPTC_ERR_WORKSPACE;
  if (ensure_device_init()) return FPTC_ERR_HIP;
  return status_of(
      launch_decode(*batch, *codec, s, plan_view(const_cast<void *>(ws), L), symbols_out, stream_status, stream));
}

int32_t fptc_dequant_idct(const fptc_batch *batch, const fptc_codec *codec, const fptc_launch *launch,
                          const void *ws, size_t ws_bytes, const uint8_t *symbols, const float *gamma,
                          int32_t precision, float *out, void *stream) {
  Shape s;
  int rc;
  if ((rc = check_batch(batch)) || (rc = check_codec(codec)) || (rc = resolve_shape(launch, codec, &s))) return rc;
  if (!ws || (!symbols && batch->n_symbols > 0) || (!out && batch->n_samples > 0)) return FPTC_ERR_INVALID_ARG;
  if (precision < FPTC_FP32_SIMT || precision > FPTC_BF16X3) return FPTC_ERR_INVALID_ARG;
  const bool wide = codec->N == 256;
  if (precision != FPTC_FP32_SIMT &&
      !(wide ? mfma256_supported(*codec, precision, s.wpc)
             : mfma_supported(codec->N, codec->E, precision, codec->n_books, codec->n_rows)))
    return FPTC_ERR_UNSUPPORTED;
  Layout L = layout_for(batch, codec, s);
  if (ws_bytes < L.total) return FPTC_ERR_WORKSPACE;
  if (ensure_device_init()) return FPTC_ERR_HIP;
  Plan pv = plan_view(const_cast<void *>(ws), L);
  if (precision == FPTC_FP32_SIMT)
    return status_of(launch_dqidct(*batch, *codec, s, pv, symbols, gamma, precision, out, stream));
  if (wide) return status_of(launch_dqidct_mfma256(*batch, *codec, s, pv, symbols, gamma, precision, out, stream));
  return status_of(launch_dqidct_mfma(*batch, *codec, s, pv, symbols, gamma, precision, out, stream));
}

int32_t fptc_dequant_idct_backward(const fptc_batch *batch, const fptc_codec *codec, const fptc_launch *launch,
                                   void *ws, size_t ws_bytes, const uint8_t *symbols, const float *grad_out,
                                   float *grad_coeff, double *grad_gamma, void *stream) {
  Shape s;
  int rc;
  if ((rc = check_batch(batch)) || (rc = check_codec(codec)) || (rc = resolve_shape(launch, codec, &s))) return rc;
  if (!ws || (!symbols && batch->n_symbols > 0) || (!grad_out && batch->n_samples > 0)) return FPTC_ERR_INVALID_ARG;
  if (!grad_coeff && !grad_gamma) return FPTC_ERR_INVALID_ARG;
  if (bwd_lds_bytes(*codec, s) > 160 * 1024) return FPTC_ERR_UNSUPPORTED;
  Layout L = layout_for(batch, codec, s);
  if (ws_bytes < L.total) return FPTC_ERR_WORKSPACE;
  if (ensure_device_init()) return FPTC_ERR_HIP;
  return status_of(launch_bwd(*batch, *codec, s, plan_view(ws, L), symbols, grad_out, grad_coeff, grad_gamma, stream));
}

int32_t fptc_decompress_batch(const fptc_batch *batch, const fptc_codec *codec, const fptc_launch *launch,
                              const void *ws, size_t ws_bytes, const float *gamma, int32_t precision, float *out,
                              int32_t *stream_status, void *stream) {
  Shape s;
  int rc;
  if ((rc = check_decompress(batch, codec, launch, precision, out, &s))) return rc;
  if (!ws) return FPTC_ERR_INVALID_ARG;
  Layout L = layout_for(batch, codec, s);
  if (ws_bytes < L.total) return FPTC_ERR_WORKSPACE;
  if (ensure_device_init()) return FPTC_ERR_HIP;
  return launch_decompress(*batch, *codec, s, plan_view(const_cast<void *>(ws), L), gamma, precision, out,
                           stream_status, stream);
}

int32_t fptc_quantize_batch(const fptc_batch *batch, const fptc_quant_params *q, const double *dct_table,
                            const int64_t *sym_off, const float *x, uint8_t *symbols_out, double *coef_out,
                            void *stream) {
  if (!batch || batch->n_streams < 1 || batch->n_samples < 0 || batch->n_symbols < 0 || !batch->sample_off)
    return FPTC_ERR_INVALID_ARG;
  if (check_quant_params(q)) return FPTC_ERR_INVALID_ARG;
  if (!dct_table || !sym_off || (!x && batch->n_samples > 0) || (!symbols_out && batch->n_symbols > 0))
    return FPTC_ERR_INVALID_ARG;
  if (batch->n_symbols % q->E) return FPTC_ERR_INVALID_ARG;
  if (batch->n_symbols == 0) return FPTC_OK;
  if (ensure_device_init()) return FPTC_ERR_HIP;
  return status_of(launch_fdct_quant(*batch, *q, dct_table, sym_off, x, symbols_out, coef_out,
                                     batch->n_symbols / q->E, stream));
}

int32_t fptc_histogram_batch(const fptc_batch *batch, const int64_t *sym_off, const uint8_t *symbols, int32_t n_books,
                             uint64_t *counts, void *stream) {
  if (!batch || batch->n_streams < 1 || batch->n_symbols < 0 || !sym_off || !counts) return FPTC_ERR_INVALID_ARG;
  if (n_books < 1 || n_books > kMaxBooks || (!symbols && batch->n_symbols > 0)) return FPTC_ERR_INVALID_ARG;
  if (batch->n_symbols == 0) return FPTC_OK;
  if (ensure_device_init()) return FPTC_ERR_HIP;
  return status_of(launch_histogram(*batch, sym_off, n_books, symbols, counts, batch->n_symbols, stream));
}

size_t fptc_percentile_workspace_size(void) { return percentile_ws_bytes(); }

int32_t fptc_abs_percentile(const double *coef, int64_t n_windows, int32_t E, int32_t k0, int32_t k1, double p,
                            double *out, void *ws, size_t ws_bytes, void *stream) {
  if (!coef || !out || !ws || n_windows < 1 || E < 1 || k0 < 0 || k1 <= k0 || k1 > E) return FPTC_ERR_INVALID_ARG;
  if (!(p >= 0.0 && p <= 100.0)) return FPTC_ERR_INVALID_ARG;
  if (ws_bytes < percentile_ws_bytes()) return FPTC_ERR_WORKSPACE;
  if (ensure_device_init()) return FPTC_ERR_HIP;
  return status_of(launch_abs_percentile(coef, n_windows, E, k0, k1, p / 100.0, out, ws, stream));
}

}  // extern "C"
