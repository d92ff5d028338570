// Batch planning kernels (stream/chunk setup and the symlen prefix sums).
//
// Section 4.2 places each word's decoded symbols by an exclusive prefix sum of
// the per-word symbol counts.  Here the sum is taken per stream, and only the
// words where a chunk of `wpc` windows begins are recorded: a chunk then
// decodes from that word on its own, with no cross-chunk dependency.
#include <hip/hip_runtime.h>

#include "fptc_internal.h"
#include "mfma_common.h"

namespace fptc {
namespace {

constexpr int kPlanThreads = 1024;
constexpr int kScanThreads = 256;
constexpr int kWordsPerThread = 16;  // one 16-byte symlen load per thread and iteration

// Inclusive scan across one 64-lane wavefront.
template <typename T>
__device__ inline T wave_incl_scan(T v) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    T u = __shfl_up(v, d, kWave);
    if (lane >= d) v += u;
  }
  return v;
}

// Exclusive block scan; returns the exclusive prefix of v and the block total.
template <typename T, int THREADS>
__device__ inline T block_excl_scan(T v, T *lds, T &total) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  constexpr int NW = THREADS / kWave;
  T incl = wave_incl_scan(v);
  if (lane == kWave - 1) lds[wid] = incl;
  __syncthreads();
  if (wid == 0) {
    T x = lane < NW ? lds[lane] : T(0);
    T xi = wave_incl_scan(x);
    if (lane < NW) lds[lane] = xi - x;
    if (lane == NW - 1) lds[NW] = xi;
  }
  __syncthreads();
  T r = incl - v + lds[wid];
  total = lds[NW];
  __syncthreads();
  return r;
}

// One workgroup: per-stream window counts and chunk counts, their exclusive
// prefix sums, and header validation.
__global__ void __launch_bounds__(kPlanThreads) k_plan_streams(fptc_batch b, int N, int E, int wpc,
                                                               int64_t *hdr, int64_t *win_off, int64_t *chunk_off,
                                                               int32_t *status) {
  __shared__ int64_t lds[kPlanThreads / kWave + 1];
  const int n = b.n_streams;
  const int64_t win_cap = b.n_symbols / E;
  int64_t carry_w = 0, carry_c = 0;
  for (int base = 0; base < n; base += kPlanThreads) {
    const int s = base + threadIdx.x;
    int64_t nw = 0;
    int flag = 0;
    if (s < n) {
      const int64_t s0 = b.sample_off[s], s1 = b.sample_off[s + 1];
      const int64_t w0 = b.word_off[s], w1 = b.word_off[s + 1];
      if (s0 < 0 || s1 < s0 || s1 > b.n_samples || w0 < 0 || w1 < w0 || w1 > b.n_words) flag = FPTC_STREAM_BAD_HEADER;
      else nw = (s1 - s0 + N - 1) / N;
    }
    int64_t tot;
    const int64_t wo = carry_w + block_excl_scan<int64_t, kPlanThreads>(nw, lds, tot);
    carry_w += tot;
    if (s < n && !flag && (wo + nw) > win_cap) flag = FPTC_STREAM_BAD_HEADER;
    const int64_t nc = flag ? 0 : (nw + wpc - 1) / wpc;
    const int64_t co = carry_c + block_excl_scan<int64_t, kPlanThreads>(nc, lds, tot);
    carry_c += tot;
    if (s < n) {
      win_off[s] = wo;
      chunk_off[s] = co;
      if (status) status[s] = flag;
    }
  }
  if (threadIdx.x == 0) {
    win_off[n] = carry_w;
    chunk_off[n] = carry_c;
    hdr[0] = carry_c;
    hdr[1] = carry_w < win_cap ? carry_w : win_cap;
  }
}

// Exclusive block scan of int values with DPP wave scans; returns the
// exclusive prefix and the block total.
__device__ inline int block_excl_scan_dpp(int v, int *lds, int &total) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  constexpr int NW = kScanThreads / kWave;
  const int incl = wave_incl_scan_dpp(v);
  if (lane == kWave - 1) lds[wid] = incl;
  __syncthreads();
  int before = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    const int x = lds[i];
    before += i < wid ? x : 0;
    tot += x;
  }
  __syncthreads();
  total = tot;
  return before + incl - v;
}

// One workgroup per stream: exclusive scan of the stream's symlen; every word
// whose symbol range [p, p + symlen) contains the first symbol of a chunk
// (a multiple of wpc * E) is recorded in that chunk's record.  Also writes the
// per-chunk records, the 32-window tile owners, and checks the symbol total
// and the symlen bound.  4096 words per iteration, 16 per thread, the next
// iteration's bytes loaded while the current ones are scanned.
__global__ void __launch_bounds__(kScanThreads) k_plan_chunks(fptc_batch b, int N, int E, int wpc,
                                                              const int64_t *win_off, const int64_t *chunk_off,
                                                              int32_t *tile_stream, int64_t tile_cap,
                                                              ChunkMeta *meta, int32_t *status) {
  __shared__ int lds[kScanThreads / kWave];
  const int s = blockIdx.x;
  // Every stream, valid or not, records itself as the owner of the 32-window
  // tiles whose first window it holds, so a tile's first stream is one load.
  {
    const int64_t t0 = (win_off[s] + kTileWindows - 1) / kTileWindows;
    const int64_t t1 = (win_off[s + 1] + kTileWindows - 1) / kTileWindows;
    for (int64_t t = t0 + threadIdx.x; t < t1 && t < tile_cap; t += kScanThreads) tile_stream[t] = s;
  }
  const int64_t c0 = chunk_off[s], nc = chunk_off[s + 1] - c0;
  if (nc <= 0) return;  // empty stream or bad header (then status already flagged)
  const int64_t w0 = b.word_off[s], w1 = b.word_off[s + 1];
  const int64_t nw = win_off[s + 1] - win_off[s];
  const int64_t cb = (int64_t)wpc * E;  // symbols per chunk
  {
    const int64_t so = b.sample_off[s], L = b.sample_off[s + 1] - so;
    const int bk = b.book_id ? (int)b.book_id[s] : 0;
    for (int64_t i = threadIdx.x; i < nc; i += kScanThreads) {
      ChunkMeta cm;
      const int64_t wb = i * wpc;
      const int64_t nwc = nw - wb < wpc ? nw - wb : wpc;
      const int64_t ol = L - wb * N < nwc * N ? L - wb * N : nwc * N;
      cm.first_word = -1;
      cm.word_end = w1;
      cm.sym_base = win_off[s] * E + wb * E;
      cm.out_base = so + wb * N;
      cm.first_sym = 0;
      cm.n_windows = (int32_t)nwc;
      cm.out_len = (int32_t)ol;
      cm.stream = s;
      cm.book = bk;
      cm.pad[0] = cm.pad[1] = cm.pad[2] = 0;
      meta[c0 + i] = cm;
    }
  }
  __syncthreads();

  // iterate over 16-byte aligned groups of symlen bytes covering [w0, w1)
  const bool vec = (reinterpret_cast<uintptr_t>(b.symlen) & 15) == 0;
  const int64_t base0 = vec ? (w0 & ~(int64_t)15) : w0;
  constexpr int kIter = kScanThreads * kWordsPerThread;
  auto load16 = [&](int64_t first, uint8_t (&c)[kWordsPerThread]) {
    if (vec && first >= w0 && first + kWordsPerThread <= w1) {
      const uint4 u = *reinterpret_cast<const uint4 *>(b.symlen + first);
      const uint32_t x[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
      for (int j = 0; j < kWordsPerThread; ++j) c[j] = (uint8_t)(x[j >> 2] >> (8 * (j & 3)));
    } else {
#pragma unroll
      for (int j = 0; j < kWordsPerThread; ++j) {
        const int64_t w = first + j;
        c[j] = (w >= w0 && w < w1) ? b.symlen[w] : (uint8_t)0;
      }
    }
  };
  int64_t carry = 0;
  int bad = 0;
  uint8_t nxt[kWordsPerThread];
  load16(base0 + (int64_t)threadIdx.x * kWordsPerThread, nxt);
  for (int64_t base = base0; base < w1; base += kIter) {
    const int64_t wb = base + (int64_t)threadIdx.x * kWordsPerThread;
    int cnt[kWordsPerThread];
    int sum = 0;
#pragma unroll
    for (int j = 0; j < kWordsPerThread; ++j) {
      int c = nxt[j];
      if (c > 64) {
        bad |= FPTC_STREAM_BAD_SYMLEN;
        c = 64;
      }
      cnt[j] = c;
      sum += c;
    }
    if (base + kIter < w1) load16(wb + kIter, nxt);
    int tot;
    int64_t p = carry + block_excl_scan_dpp(sum, lds, tot);
    carry += tot;
    // chunk m starts at symbol m * cb; walk the boundaries inside this
    // thread's words from the first one at or after p
    int64_t m = (p + cb - 1) / cb;
    int64_t mb = m * cb;
#pragma unroll
    for (int j = 0; j < kWordsPerThread; ++j) {
      const int c = cnt[j];
      for (; mb < p + c && m < nc; ++m, mb += cb) {
        meta[c0 + m].first_word = wb + j;
        meta[c0 + m].first_sym = (int32_t)(p - mb);
      }
      p += c;
    }
  }
  if (threadIdx.x == 0 && carry != nw * E) bad |= FPTC_STREAM_BAD_COUNT;
  if (bad && status) atomicOr(&status[s], bad);
}

}  // namespace

int launch_plan(const fptc_batch &b, const fptc_codec &c, const Shape &s, const Plan &p, int32_t *status,
                void *stream) {
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_plan_streams, dim3(1), dim3(kPlanThreads), 0, st, b, c.N, c.E, s.wpc, p.hdr, p.win_off,
                     p.chunk_off, status);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return (int)e;
  hipLaunchKernelGGL(k_plan_chunks, dim3(b.n_streams), dim3(kScanThreads), 0, st, b, c.N, c.E, s.wpc, p.win_off,
                     p.chunk_off, p.tile_stream, p.tile_cap, p.chunk_meta, status);
  return (int)hipGetLastError();
}

}  // namespace fptc
