/*
 * fptc.h -- C ABI of the MI355X (gfx950) FPTC batch decoder.
 *
 * FPTC (Mechels et al., "FPTC: A Fast Parallel Transform-based Codec for
 * Efficient Asymmetric Signal Compression") compresses a strip of float32
 * samples by a windowed DCT-II (Section 3.1), a three-zone byte quantizer
 * (Section 3.2) and length-limited canonical Huffman coding packed into
 * 64-bit words with a per-word symbol count, the SymLen format (Section 3.3,
 * Section 4.1, Algorithm 1).  This library is the server side: it turns a
 * batch of SymLen streams already resident in GPU memory back into float32
 * samples in GPU memory (Section 4.2, throughput rule of Section 5.1).
 *
 * Conventions that hold for every call:
 *  - Pointers named "device" are GPU (HBM) addresses; "host" pointers are CPU
 *    memory read or written during the call only.  The caller owns every
 *    buffer.  No call allocates or frees GPU memory; scratch space comes from
 *    the caller's workspace.
 *  - Calls taking a `stream` (a hipStream_t passed as void*, NULL = the null
 *    stream) only enqueue work on it and return without synchronising.  All
 *    argument checks run on the host first: a call that returns an error has
 *    enqueued nothing.  Device buffers must stay alive until the enqueued work
 *    has finished.
 *  - Corrupt compressed data never makes a kernel read or write outside the
 *    buffers described by the batch; it is reported per stream in
 *    `stream_status` (bit flags FPTC_STREAM_*), without a host sync.  A flagged
 *    stream's outputs are unspecified, other streams are unaffected.
 *  - Return values are fptc_status codes.
 */
#ifndef FPTC_H
#define FPTC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FPTC_ABI_VERSION 1

#if defined(__GNUC__)
#define FPTC_API __attribute__((visibility("default")))
#else
#define FPTC_API
#endif

typedef enum {
  FPTC_OK = 0,
  FPTC_ERR_INVALID_ARG = 1, /* NULL pointer, size out of range, inconsistent sizes */
  FPTC_ERR_UNSUPPORTED = 2, /* valid request the library does not implement */
  FPTC_ERR_WORKSPACE = 3,   /* workspace smaller than fptc_workspace_size() */
  FPTC_ERR_HIP = 4          /* a HIP runtime call or kernel launch failed */
} fptc_status;

/* Per-stream data-error flags written to stream_status[s] (int32 bit set). */
#define FPTC_STREAM_BAD_COUNT 1   /* sum of symlen != ceil(L/N) * E (Section 4.1) */
#define FPTC_STREAM_OVERRUN 2     /* a codeword runs past bit 64 or no code matches */
#define FPTC_STREAM_BAD_SYMLEN 4  /* a symlen entry above 64 */
#define FPTC_STREAM_BAD_HEADER 8  /* offsets decrease or exceed the batch capacities */

/* Arithmetic of the inverse-DCT contraction (dequantized coefficients times the
 * IDCT basis).  FP32 accumulation in every case.
 *   FP32_SIMT: scalar FP32 fused multiply-adds.
 *   FP16 / BF16: one MFMA pass, operands rounded to 16 bits (fast, ~1e-3 rel).
 *   FP16X2: basis split into hi + lo FP16 halves (and the coefficient too
 *           when it is not exact in FP16): FP32-level accuracy on MFMA.
 *   BF16X3: basis split into three BF16 pieces, coefficient split likewise
 *           when needed: FP32-level accuracy on MFMA. */
typedef enum {
  FPTC_FP32_SIMT = 0,
  FPTC_FP16 = 1,
  FPTC_FP16X2 = 2,
  FPTC_BF16 = 3,
  FPTC_BF16X3 = 4
} fptc_precision;

/* A batch of independent compressed streams, concatenated (CSR layout).
 * Stream s holds L_s = sample_off[s+1] - sample_off[s] samples, cut into
 * n_win_s = ceil(L_s / N) windows (Section 3.1; the last window is zero-padded
 * by the encoder); its SymLen bitstream is words/symlen[word_off[s] ..
 * word_off[s+1]) and carries n_win_s * E symbols in window-major, ascending-bin
 * order.  Decoded symbols of stream s are stored at sym_off[s] = E * sum over
 * earlier streams of n_win; samples at sample_off[s]. */
typedef struct {
  int32_t n_streams;          /* >= 1 */
  int32_t reserved0;
  int64_t n_words;            /* host: elements of words[] and symlen[] */
  int64_t n_symbols;          /* host: elements of the decoded-symbol array */
  int64_t n_samples;          /* host: elements of the output array */
  const uint64_t *words;      /* device [n_words]; codewords MSB-first inside each word */
  const uint8_t *symlen;      /* device [n_words]; symbols in each word (Section 4.1) */
  const int64_t *word_off;    /* device [n_streams + 1], word_off[0] = 0 */
  const int64_t *sample_off;  /* device [n_streams + 1], sample_off[0] = 0 */
  const uint8_t *book_id;     /* device [n_streams] codebook per stream, or NULL = book 0 */
} fptc_batch;

/* Per-domain decoding structures (Section 3.4: built offline per signal
 * domain; Figure "Codec structures").  One transform size for the batch,
 * n_books codebooks / quantization tables. */
typedef struct {
  int32_t N;                  /* window (DCT size): 4, 8, 16, 32, 64, 128 or 256 */
  int32_t E;                  /* kept coefficients per window, 1 <= E <= N (Section 3.1) */
  int32_t lmax;               /* longest code, 1..16 (Section 3.3 length limit).  Above 12 the
                                 kernels decode through two-level tables built in LDS from
                                 lut; fptc_decompress_batch then supports N <= 128 only */
  int32_t n_books;            /* 1..8 */
  int32_t n_rows;             /* rows of the dequantization table, 1..4 */
  int32_t reserved0;
  const uint16_t *lut;        /* device [n_books][1 << lmax]: entry for an lmax-bit peek =
                                 (code length << 8) | symbol; 0 = no code (fptc_build_lut) */
  const float *deq_val;       /* device [n_books][n_rows][256]: value of a symbol */
  const uint8_t *deq_zone;    /* device [n_books][n_rows][256]: zone 0..2 of a symbol */
  const uint8_t *row_of_bin;  /* device [n_books][E]: table row used by bin k */
  const float *basis;         /* device [E][N]: orthonormal IDCT basis (fptc_build_basis) */
} fptc_codec;

/* Launch shape.  Zero fields take the library defaults. */
typedef struct {
  int32_t windows_per_chunk;  /* windows per decode work item (chunk); default 32 */
  int32_t waves_per_block;    /* 0: default (4; fptc_decode_batch: the most, up to 16, whose
                                 LDS fits; fptc_decompress_batch: the same, up to 8 at
                                 N = 128); at most 16 (fused: 8 at N = 128, else
                                 FPTC_ERR_UNSUPPORTED).  N = 256 (both MFMA calls): the
                                 kernels always run 8 waves (0 or 8, else
                                 FPTC_ERR_UNSUPPORTED for the fused call) */
  int32_t blocks;             /* persistent grid size; default: enough to fill the GPU */
  int32_t chunk_group;        /* fptc_decompress_batch at N <= 128: adjacent chunks per group, groups
                                 dealt round-robin over the grid (group g to block g mod blocks);
                                 0 = default (4), at most 64 */
} fptc_launch;

/* Quantizer description for the host table builders and host encoder
 * (Section 3.2, Table 1). */
typedef enum { FPTC_QUANT_AMPLITUDE = 0, FPTC_QUANT_PAPER = 1 } fptc_quant_kind;

typedef struct {
  int32_t kind;               /* fptc_quant_kind */
  int32_t N, E;
  int32_t B1, B2;             /* PAPER: zone boundaries 0 <= B1 <= B2 <= E */
  int32_t reserved0;
  double step_fine;           /* AMPLITUDE: fine step (zero zone is |c| < step_fine/2) */
  double step_coarse;         /* AMPLITUDE: coarse step beyond the threshold */
  double threshold;           /* AMPLITUDE: |c| where the coarse zone starts; a multiple of step_fine */
  double mu;                  /* PAPER: mu-law strength (Eq. 2) */
  double alpha1;              /* PAPER: deadzone ratio (Eq. 3) */
  double A0, A1;              /* PAPER: zone maxima (clipped percentiles) */
} fptc_quant_params;

/* ---------------------------------------------------------------- info */

FPTC_API int32_t fptc_abi_version(void);
FPTC_API const char *fptc_status_string(int32_t status);

/* --------------------------------------------------------- device calls */

/* Set up the library on the current device: every kernel is allowed the
 * whole 160 KB of a compute unit's LDS.  Done once per device and
 * thread-safe; every device call below runs it on its first use with a
 * device current, so calling it is optional.  Call it before capturing
 * library calls into a HIP graph: the captured calls then make no runtime
 * call besides their kernel launches.  FPTC_ERR_HIP when no device is
 * current or an attribute is refused. */
FPTC_API int32_t fptc_init(void);

/* Bytes of device workspace the calls below need for this batch, codec and
 * launch shape (plan tables, chunk tables, backward partial sums).  0 on
 * invalid arguments. */
FPTC_API size_t fptc_workspace_size(const fptc_batch *batch, const fptc_codec *codec, const fptc_launch *launch);

/* Plan a batch (stream and chunk setup, symlen prefix sums; Section 4.2: the
 * exclusive prefix sum over symlen that places each word's output).  Writes the
 * stream's symbol and window offsets and, for every chunk of windows, the
 * first word holding one of its symbols into `ws`, and initialises
 * stream_status (device [n_streams]) with the header and symbol-count checks.
 * The plan stays valid for the same batch contents, codec and launch. */
FPTC_API int32_t fptc_plan_batch(const fptc_batch *batch, const fptc_codec *codec, const fptc_launch *launch,
                        void *ws, size_t ws_bytes, int32_t *stream_status, void *stream);

/* Huffman decode with output compaction (Section 4.2, lossless stage): every
 * stream's SymLen words -> its n_win * E symbols, bit-exact, in symbols_out
 * (device [n_symbols], window-major per stream, at sym_off[s]).  Needs a plan
 * built by fptc_plan_batch in `ws`.  Decoding errors OR into stream_status. */
FPTC_API int32_t fptc_decode_batch(const fptc_batch *batch, const fptc_codec *codec, const fptc_launch *launch,
                          const void *ws, size_t ws_bytes, uint8_t *symbols_out, int32_t *stream_status,
                          void *stream);

/* Dequantization fused with the inverse DCT (Section 4.2, lossy stage):
 * symbols (device [n_symbols], as written by fptc_decode_batch) -> samples
 * out (device [n_samples]).  Coefficient k of a window of stream s is
 * gamma[3 s + z] * deq_val[book][row_of_bin[k]][sym] with
 * z = deq_zone[book][row_of_bin[k]][sym]; gamma (device [n_streams][3]) may be
 * NULL for all ones.  Only the first L_s samples of a stream are written.
 * Needs a plan in `ws`. */
FPTC_API int32_t fptc_dequant_idct(const fptc_batch *batch, const fptc_codec *codec, const fptc_launch *launch,
                          const void *ws, size_t ws_bytes, const uint8_t *symbols, const float *gamma,
                          int32_t precision, float *out, void *stream);

/* Backward of fptc_dequant_idct for an output gradient grad_out = dL/dx
 * (device [n_samples]; samples past a stream's length are not outputs).
 *   grad_coeff (device [n_symbols] or NULL): dL/dchat for every coefficient,
 *     chat = gamma * dequantized value, i.e. the first E bins of the
 *     orthonormal DCT-II (Section 3.1) of each window of grad_out; FP32.
 *   grad_gamma (device [n_streams][3] or NULL): dL/dgamma[s][z], the sum over
 *     the stream's coefficients of zone z of dL/dchat * dequantized value,
 *     accumulated in FP64 in a fixed order (deterministic).
 * At least one output must be given.  Needs a plan in `ws` (its backward
 * scratch is written); symbols as written by fptc_decode_batch. */
FPTC_API int32_t fptc_dequant_idct_backward(const fptc_batch *batch, const fptc_codec *codec,
                                            const fptc_launch *launch, void *ws, size_t ws_bytes,
                                            const uint8_t *symbols, const float *grad_out, float *grad_coeff,
                                            double *grad_gamma, void *stream);

/* Decode, dequantize and inverse-transform in one pass: the two stages of
 * Section 4.2 fused, the decoded symbols of a chunk of windows kept in LDS
 * instead of a global array.  Same result as fptc_decode_batch followed by
 * fptc_dequant_idct with the same precision (bit-identical samples), without
 * the symbol array.  Precisions: the MFMA ones (FP16, FP16X2, BF16, BF16X3)
 * for N in {32, 64, 128, 256}; FPTC_ERR_UNSUPPORTED otherwise.  Needs a plan in
 * `ws`; decoding errors OR into stream_status (device [n_streams]). */
FPTC_API int32_t fptc_decompress_batch(const fptc_batch *batch, const fptc_codec *codec, const fptc_launch *launch,
                                       const void *ws, size_t ws_bytes, const float *gamma, int32_t precision,
                                       float *out, int32_t *stream_status, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops and harnesses that forbid allocation):
 * fptc_plan_batch followed by fptc_decompress_batch, with the plan kept in a
 * static device array of the library, FPTC_NOALLOC_WS_BYTES per device,
 * reserved until the process ends, instead of a caller workspace.  The
 * caller passes inputs and outputs only; the call allocates nothing.
 * FPTC_ERR_WORKSPACE when the batch's plan needs more than that (compare
 * fptc_workspace_size); other errors as fptc_decompress_batch, all before
 * anything is enqueued.  Every call on a device uses that device's one
 * array and rewrites all of the plan it reads: calls that overlap on one
 * device (other streams, other host threads) race and must be ordered by
 * the caller. */
#define FPTC_NOALLOC_WS_BYTES (16u << 20)
FPTC_API int32_t fptc_decompress_batch_noalloc(const fptc_batch *batch, const fptc_codec *codec,
                                               const fptc_launch *launch, const float *gamma, int32_t precision,
                                               float *out, int32_t *stream_status, void *stream);

/* ------------------------------------------------ encode side (device calls)
 * The steps before the decode path: the encoder's transform and quantizer,
 * and the statistics a codebook and the paper quantizer are trained on.
 * For these calls the batch supplies n_streams, n_samples, n_symbols,
 * sample_off and book_id only (words may be NULL with n_words = 0). */

/* Transform and quantize (Section 3.1, Section 3.2): every stream's samples x
 * (device f32 [n_samples], CSR by batch->sample_off) cut into ceil(L/N)
 * windows (the last zero-padded), each transformed by the orthonormal DCT-II
 * X[k] = a_k * sum over n of x[n] cos(pi/N (n + 1/2) k) in FP64 (products and
 * sums rounded separately, n ascending), its first E coefficients quantized
 * by q: symbols_out (device u8 [n_symbols]) at sym_off[s], window-major.
 * dct_table: device FP64 [E][N + 1] from fptc_build_dct_table.  sym_off:
 * device [n_streams + 1], E times the exclusive prefix of ceil(L_s / N);
 * n_symbols = sym_off[n_streams].  coef_out (device FP64 [n_symbols] or
 * NULL) receives the coefficients X. */
FPTC_API int32_t fptc_quantize_batch(const fptc_batch *batch, const fptc_quant_params *q, const double *dct_table,
                                     const int64_t *sym_off, const float *x, uint8_t *symbols_out, double *coef_out,
                                     void *stream);

/* Symbol histogram per codebook (Section 3.3): adds the number of times each
 * byte value occurs among stream s's symbols (device [n_symbols], at
 * sym_off[s]) to counts[book_id[s]][value] (device u64 [n_books][256]; book 0
 * when book_id is NULL; streams of books >= n_books are skipped).  The caller
 * zeroes counts before the first call; exact integer counts. */
FPTC_API int32_t fptc_histogram_batch(const fptc_batch *batch, const int64_t *sym_off, const uint8_t *symbols,
                                      int32_t n_books, uint64_t *counts, void *stream);

/* Bytes of device workspace fptc_abs_percentile needs. */
FPTC_API size_t fptc_percentile_workspace_size(void);

/* Clipped zone maximum (Section 3.2; Table 1's percentile): the p-th
 * percentile, 0 <= p <= 100, of |coef[w][k]| over windows w < n_windows and
 * bins k0 <= k < k1 of coef (device FP64 [n_windows][E]), with linear
 * interpolation between order statistics: sorted values a, h = (M - 1) p/100,
 * result a[floor h] + (a[floor h + 1] - a[floor h]) (h - floor h) (taken from
 * the upper neighbour when that weight is at least 1/2).  The two order
 * statistics are found exactly by radix selection on the FP64 bit patterns.
 * out: device FP64 [1].  ws: device workspace, ws_bytes >=
 * fptc_percentile_workspace_size(); calls sharing ws must not overlap. */
FPTC_API int32_t fptc_abs_percentile(const double *coef, int64_t n_windows, int32_t E, int32_t k0, int32_t k1,
                                     double p, double *out, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------ host calls */

/* Decode lookup table of one codebook (Section 3.3: 2^lmax entries indexed by
 * the next lmax bits).  code_len (host [256]) holds each symbol's length
 * (0 = no code); codes are canonical in (length, symbol) order.  Fails on
 * lengths above lmax or a Kraft sum above 1.  lut_out: host [1 << lmax]. */
FPTC_API int32_t fptc_build_lut(const uint8_t *code_len, int32_t lmax, uint16_t *lut_out);

/* Canonical codes (host [256]) for the given lengths. */
FPTC_API int32_t fptc_canonical_codes(const uint8_t *code_len, uint32_t *codes_out);

/* Length-limited optimal code lengths by package-merge (Section 3.3) from a
 * 256-entry histogram (host); symbols with count 0 get no code. */
FPTC_API int32_t fptc_code_lengths(const uint64_t *freq, int32_t lmax, uint8_t *len_out);

/* Forward transform table for fptc_quantize_batch (host FP64 [E][N + 1]):
 * row k holds cos(pi/N (n + 1/2) k) for n < N, then a_k = sqrt(1/N) (k = 0)
 * or sqrt(2/N) in column N (Section 3.1, orthonormal scaling). */
FPTC_API int32_t fptc_build_dct_table(int32_t N, int32_t E, double *table_out);

/* Orthonormal IDCT basis B[k][n] = a_k cos(pi/N (n + 1/2) k), a_0 = sqrt(1/N),
 * a_k = sqrt(2/N), for k < E, n < N, rounded to float (host [E][N]). */
FPTC_API int32_t fptc_build_basis(int32_t N, int32_t E, float *basis_out);

/* Dequantization tables of one codebook (host): deq_val [n_rows][256],
 * deq_zone [n_rows][256], row_of_bin [E]; *n_rows_out receives the row count
 * (1 for AMPLITUDE, 3 for PAPER).  Buffers must hold 4 rows. */
FPTC_API int32_t fptc_build_dequant(const fptc_quant_params *q, float *deq_val, uint8_t *deq_zone,
                           uint8_t *row_of_bin, int32_t *n_rows_out);

/* Host encoder (Section 4.1): window, DCT-II, quantize one strip of L float32
 * samples into ceil(L/N) * E symbols (host). */
FPTC_API int32_t fptc_quantize_host(const float *x, int64_t L, const fptc_quant_params *q, uint8_t *symbols_out);

/* Host encoder (Section 4.1, Algorithm 1): pack symbols into SymLen words.
 * words/symlen hold `cap` entries; *n_words_out receives the count. */
FPTC_API int32_t fptc_symlen_pack_host(const uint8_t *symbols, int64_t n, const uint8_t *code_len, uint64_t *words,
                              uint8_t *symlen, int64_t cap, int64_t *n_words_out);

/* Batch host encoder, threads over streams: strips x (host, CSR by
 * sample_off[n+1]) with per-stream codebook index book_id[n] into the
 * code_len tables (host [n_books][256]).  word_cap_off (host [n+1]) gives each
 * stream's reserved word range; n_words_out (host [n]) receives the words
 * used.  Words of stream s are written at words[word_cap_off[s]]. */
FPTC_API int32_t fptc_encode_batch_host(const float *x, const int64_t *sample_off, int32_t n_streams,
                               const uint8_t *book_id, const fptc_quant_params *q, const uint8_t *code_len,
                               const int64_t *word_cap_off, uint64_t *words, uint8_t *symlen,
                               int64_t *n_words_out, int32_t n_threads);

#ifdef __cplusplus
}
#endif

#endif /* FPTC_H */
