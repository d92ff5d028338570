// Batch planning kernels (stream/chunk setup and the symlen prefix sums).
//
// Section 4.2 places each word's decoded symbols by an exclusive prefix sum of
// the per-word symbol counts.  Here the sum is taken per stream, in two levels
// (4096-word segments, then the segments of each stream), and only the words
// where a chunk of `wpc` windows begins are recorded: a chunk then decodes
// from that word on its own, with no cross-chunk dependency.
#include <hip/hip_runtime.h>

#include "fptc_internal.h"
#include "mfma_common.h"

namespace fptc {
namespace {

constexpr int kPlanThreads = 1024;
constexpr int kScanThreads = 256;
constexpr int64_t kSegWords = 4096;  // words per segment
// The segment sums take a segment per wavefront (64 lanes x 64 words, four
// 16-byte symlen loads per lane): one-wave workgroups need no barrier in
// their scan, and more of them fit on a CU at once, which is what a
// latency-bound pass over many small segments needs.  The chunk-start pass
// walks every word's symbol range, so it keeps 256 threads x 16 words.
constexpr int kSumThreads = kWave;
constexpr int kChunkThreads = 256;

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

// One workgroup: per-stream window, chunk and symlen-segment counts, their
// exclusive prefix sums, header validation, and the segment -> stream map.
// Segments are kSegWords words on a 16-word grid aligned down from the
// stream's first word.  Each thread takes kStreamsPerThread consecutive
// streams (all their offsets loaded at once), so a batch of up to
// kPlanThreads * kStreamsPerThread streams needs one pass of block scans.
constexpr int kStreamsPerThread = 4;

__global__ void __launch_bounds__(kPlanThreads) k_plan_streams(fptc_batch b, int N, int E, int wpc,
                                                               int64_t *hdr, int64_t *win_off, int64_t *chunk_off,
                                                               int64_t *seg_off, int32_t *seg_stream,
                                                               int64_t seg_cap, int32_t *status) {
  __shared__ int64_t lds[kPlanThreads / kWave + 1];
  constexpr int K = kStreamsPerThread;
  __shared__ int64_t seg_at[kPlanThreads * K + 1];  // this pass's streams: first segment of each, then the end
  const int n = b.n_streams;
  const int64_t win_cap = b.n_symbols / E;
  int64_t carry_w = 0, carry_c = 0, carry_g = 0;
  for (int base = 0; base < n; base += kPlanThreads * K) {
    const int s0 = base + threadIdx.x * K;
    int64_t so[K + 1], wo[K + 1];
#pragma unroll
    for (int k = 0; k <= K; ++k) {
      const int s = s0 + k < n ? s0 + k : n;
      so[k] = b.sample_off[s];
      wo[k] = b.word_off[s];
    }
    int64_t nw[K], nc[K], ng[K];
    int flag[K];
    int64_t tw = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      flag[k] = 0;
      nw[k] = 0;
      if (s0 + k < n) {
        if (so[k] < 0 || so[k + 1] < so[k] || so[k + 1] > b.n_samples || wo[k] < 0 || wo[k + 1] < wo[k] ||
            wo[k + 1] > b.n_words)
          flag[k] = FPTC_STREAM_BAD_HEADER;
        else
          nw[k] = (so[k + 1] - so[k] + N - 1) / N;
      }
      tw += nw[k];
    }
    int64_t tot;
    int64_t w_at = carry_w + block_excl_scan<int64_t, kPlanThreads>(tw, lds, tot);
    carry_w += tot;
    int64_t tc = 0, tg = 0;
    int64_t wx[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      wx[k] = w_at;
      if (s0 + k < n && !flag[k] && w_at + nw[k] > win_cap) flag[k] = FPTC_STREAM_BAD_HEADER;
      w_at += nw[k];
      nc[k] = flag[k] ? 0 : (nw[k] + wpc - 1) / wpc;
      const int64_t a0 = wo[k] & ~(int64_t)15;
      ng[k] = (flag[k] || nc[k] == 0 || wo[k + 1] <= wo[k]) ? 0 : (wo[k + 1] - a0 + kSegWords - 1) / kSegWords;
      tc += nc[k];
      tg += ng[k];
    }
    int64_t c_at = carry_c + block_excl_scan<int64_t, kPlanThreads>(tc, lds, tot);
    carry_c += tot;
    int64_t g_at = carry_g + block_excl_scan<int64_t, kPlanThreads>(tg, lds, tot);
    carry_g += tot;
    const int64_t g_pass = carry_g - tot;  // this pass's first segment
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int s = s0 + k;
      if (s < n) {
        win_off[s] = wx[k];
        chunk_off[s] = c_at;
        seg_off[s] = g_at;
        if (status) status[s] = flag[k];
      }
      seg_at[threadIdx.x * K + k] = g_at;  // past n: the pass's end
      c_at += nc[k];
      g_at += ng[k];
    }
    if (threadIdx.x == 0) seg_at[kPlanThreads * K] = carry_g;
    __syncthreads();
    // segment -> stream map: each thread a contiguous range of this pass's
    // segments, its first stream by binary search, then walking forward
    const int64_t per = (tot + kPlanThreads - 1) / kPlanThreads;
    const int64_t g_lo = g_pass + (int64_t)threadIdx.x * per, g_hi = min(g_lo + per, carry_g);
    if (g_lo < g_hi) {
      int lo = 0, hi = kPlanThreads * K - 1;  // last local stream whose first segment is <= g_lo
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (seg_at[mid] <= g_lo) lo = mid;
        else hi = mid - 1;
      }
      int i = lo;
      for (int64_t g = g_lo; g < g_hi && g < seg_cap; ++g) {
        while (seg_at[i + 1] <= g) ++i;
        seg_stream[g] = base + i;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    win_off[n] = carry_w;
    chunk_off[n] = carry_c;
    seg_off[n] = carry_g;
    hdr[0] = carry_c;
    hdr[1] = carry_w < win_cap ? carry_w : win_cap;
    hdr[2] = carry_g < seg_cap ? carry_g : seg_cap;
    hdr[3] = seg_cap;
  }
}

// The words of one segment: this thread's WPT symlen bytes, packed four to a
// dword (words outside the stream read as 0), each clamped to 64 with the
// clamp reported.
template <int WPT>
struct SegWords {
  int64_t first;  // global index of this lane's first word
  uint32_t x[WPT / 4];
  __device__ int cnt(int j) const { return (int)((x[j >> 2] >> (8 * (j & 3))) & 255u); }
};

__device__ inline int clamp_stream(int s, int n) { return s < 0 ? 0 : (s >= n ? n - 1 : s); }

// An empty asm statement that reads a uniform value: the compiler must have
// loaded it here, so loads pinned this way are issued together and waited
// for once, instead of one round trip each as their uses come.
__device__ inline void pin(int64_t x) { asm volatile("" ::"s"(x)); }

// The segment's stream and its word range, loaded together with everything
// else the kernel needs of the stream, before any check waits on them.
struct SegStream {
  int64_t w0, w1, g0, g1;  // the stream's words, its segments
};

__device__ inline SegStream seg_stream_of(const fptc_batch &b, int s, const int64_t *seg_off) {
  SegStream t;
  t.w0 = b.word_off[s];
  t.w1 = b.word_off[s + 1];
  t.g0 = seg_off[s];
  t.g1 = seg_off[s + 1];
  return t;
}

template <int WPT>
__device__ inline int load_seg_words(const fptc_batch &b, int64_t g, const SegStream &t, SegWords<WPT> &sw) {
  static_assert(WPT % 16 == 0, "whole 16-byte symlen blocks per thread");
  const int64_t a0 = t.w0 & ~(int64_t)15;
  const int64_t first = a0 + (g - t.g0) * kSegWords + (int64_t)threadIdx.x * WPT;
  sw.first = first;
  const bool aligned = (reinterpret_cast<uintptr_t>(b.symlen) & 15) == 0;
#pragma unroll
  for (int q = 0; q < WPT / 16; ++q) {
    const int64_t f = first + 16 * q;
    uint32_t *x = sw.x + 4 * q;
    x[0] = x[1] = x[2] = x[3] = 0;
    if (f + 16 <= t.w0 || f >= t.w1) continue;  // no word of the stream
    if (aligned && f + 16 <= b.n_words) {
      // a whole 16-byte block inside the array (f is a multiple of 16);
      // bytes outside the stream are cleared below
      const uint4 u = *reinterpret_cast<const uint4 *>(b.symlen + f);
      x[0] = u.x, x[1] = u.y, x[2] = u.z, x[3] = u.w;
    } else {
#pragma unroll
      for (int j = 0; j < 16; ++j)
        if (f + j >= t.w0 && f + j < t.w1) x[j >> 2] |= (uint32_t)b.symlen[f + j] << (8 * (j & 3));
    }
  }
  // clear the bytes before the stream's first and from its last word on
  // (only the lanes at the stream's two ends have any)
  const int64_t lo64 = t.w0 - first, hi64 = t.w1 - first;
  if (lo64 > 0 || hi64 < WPT) {
    const int lo = lo64 > 0 ? (int)(lo64 < WPT ? lo64 : WPT) : 0;
    const int hi = hi64 < WPT ? (int)(hi64 > 0 ? hi64 : 0) : WPT;
#pragma unroll
    for (int d = 0; d < WPT / 4; ++d) {
      uint32_t m = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) m |= (4 * d + k >= lo && 4 * d + k < hi) ? (255u << (8 * k)) : 0u;
      sw.x[d] &= m;
    }
  }
  // a count above 64 (a byte of 65 or more) is clamped and reported
  int bad = 0;
#pragma unroll
  for (int d = 0; d < WPT / 4; ++d) {
    const uint32_t v = sw.x[d];
    if ((v & 0x80808080u) | (((v & 0x7f7f7f7fu) + 0x3f3f3f3fu) & 0x80808080u)) {
      uint32_t c = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t e = (v >> (8 * k)) & 255u;
        c |= (e > 64u ? 64u : e) << (8 * k);
      }
      sw.x[d] = c;
      bad = FPTC_STREAM_BAD_SYMLEN;
    }
  }
  return bad;
}

// The sum of a thread's counts.
template <int WPT>
__device__ inline int seg_words_sum(const SegWords<WPT> &sw) {
  uint32_t sum = 0;
#pragma unroll
  for (int d = 0; d < WPT / 4; ++d) sum = __builtin_amdgcn_sad_u8(sw.x[d], 0u, sum);
  return (int)sum;
}

// Exclusive block scan of int values (kChunkThreads threads) with DPP wave
// scans; returns the exclusive prefix and the block total.
__device__ inline int block_excl_scan_dpp(int v, int *lds, int &total) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  constexpr int NW = kChunkThreads / kWave;
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

// Exclusive scan across the segment's one wavefront; total = the wave's sum.
__device__ inline int seg_excl_scan(int v, int &total) {
  const int incl = wave_incl_scan_dpp(v);
  total = __builtin_amdgcn_readlane(incl, kWave - 1);
  return incl - v;
}

// One wavefront per segment: the segment's symbol count (symlen clamped to
// 64; a larger symlen is flagged).
__global__ void __launch_bounds__(kSumThreads) k_plan_seg_sums(fptc_batch b, const int64_t *hdr,
                                                                const int64_t *seg_off, const int32_t *seg_stream,
                                                                int32_t *seg_sum, int32_t *status) {
  if (b.n_streams <= 0) return;
  const int64_t g = blockIdx.x;
  // g < seg_cap, so this read is in bounds; past the plan's segments it may
  // hold anything, so it is clamped to a stream before the stream's offsets
  // are read with it (such a block then returns on the header check)
  const int s = clamp_stream(seg_stream[g], b.n_streams);
  const int64_t h2 = hdr[2], seg_cap = hdr[3];
  const SegStream t = seg_stream_of(b, s, seg_off);
  pin(t.w0), pin(t.w1), pin(t.g0), pin(t.g1), pin(h2), pin(seg_cap);
  if (g >= h2 || t.g1 > seg_cap) return;  // past the plan, or the stream's segments did not fit (flagged)
  SegWords<kSegWords / kSumThreads> sw;
  const int bad = load_seg_words(b, g, t, sw);
  int tot;
  seg_excl_scan(seg_words_sum(sw), tot);  // only the wave's total is kept
  if (threadIdx.x == 0) seg_sum[g] = tot;
  if (bad && status) atomicOr(&status[s], bad);
}

// One workgroup per stream: exclusive scan of its segment sums (symbols of
// the stream before each segment), the symbol-count check, the chunk
// records' fixed fields, and the 32-window tile owners.
__global__ void __launch_bounds__(kScanThreads) k_plan_stream_scan(fptc_batch b, int N, int E, int wpc,
                                                                   const int64_t *win_off, const int64_t *chunk_off,
                                                                   const int64_t *seg_off, int64_t seg_cap,
                                                                   const int32_t *seg_sum, int64_t *seg_base,
                                                                   int32_t *tile_stream,
                                                                   int64_t tile_cap, ChunkMeta *meta,
                                                                   int32_t *status) {
  __shared__ int64_t lds[kScanThreads / kWave + 1];
  const int s = blockIdx.x;
  // everything of the stream at once: one round trip before any use
  const int64_t wo0 = win_off[s], wo1 = win_off[s + 1];
  const int64_t c0 = chunk_off[s], nc = chunk_off[s + 1] - c0;
  const int64_t w1 = b.word_off[s + 1];
  const int64_t so = b.sample_off[s], L = b.sample_off[s + 1] - so;
  const int64_t g0 = seg_off[s], g1 = seg_off[s + 1];
  pin(wo0), pin(wo1), pin(c0), pin(nc), pin(w1), pin(so), pin(L), pin(g0), pin(g1);
  // Every stream, valid or not, records itself as the owner of the 32-window
  // tiles whose first window it holds, so a tile's first stream is one load.
  {
    const int64_t t0 = (wo0 + kTileWindows - 1) / kTileWindows;
    const int64_t t1 = (wo1 + kTileWindows - 1) / kTileWindows;
    for (int64_t t = t0 + threadIdx.x; t < t1 && t < tile_cap; t += kScanThreads) tile_stream[t] = s;
  }
  if (nc <= 0) return;  // empty stream or bad header (then status already flagged)
  const int64_t nw = wo1 - wo0;
  {
    const int bk = b.book_id ? (int)b.book_id[s] : 0;
    for (int64_t i = threadIdx.x; i < nc; i += kScanThreads) {
      ChunkMeta cm;
      const int64_t wb = i * wpc;
      const int64_t nwc = nw - wb < wpc ? nw - wb : wpc;
      const int64_t ol = L - wb * N < nwc * N ? L - wb * N : nwc * N;
      cm.first_word = -1;
      cm.first_sym = 0;
      cm.last = i == nc - 1;
      cm.word_end = w1;
      cm.sym_base = wo0 * E + wb * E;
      cm.out_base = so + wb * N;
      cm.n_windows = (int32_t)nwc;
      cm.out_len = (int32_t)ol;
      cm.stream = s;
      cm.book = bk;
      cm.pad[0] = cm.pad[1] = 0;
      meta[c0 + i] = cm;
    }
  }
  const int64_t ng = g1 - g0;
  if (g1 > seg_cap) {  // word ranges of streams overlap: no segment room
    if (threadIdx.x == 0 && status) atomicOr(&status[s], FPTC_STREAM_BAD_HEADER);
    return;  // its chunks keep first_word = -1
  }
  int64_t carry = 0;
  for (int64_t base = 0; base < ng; base += kScanThreads) {
    const int64_t i = base + threadIdx.x;
    const int64_t v = i < ng ? seg_sum[g0 + i] : 0;
    int64_t tot;
    const int64_t ex = block_excl_scan<int64_t, kScanThreads>(v, lds, tot);
    if (i < ng) seg_base[g0 + i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0 && carry != nw * E && status) atomicOr(&status[s], FPTC_STREAM_BAD_COUNT);
}

// One workgroup per segment: exclusive scan of its words' symlen on top of
// the segment's base; every word whose symbol range [p, p + symlen) holds the
// first symbol of a chunk (a multiple of wpc * E) becomes that chunk's first
// word (the chunk before it ends at that word, inclusive when the chunk
// starts inside the word).
__global__ void __launch_bounds__(kChunkThreads) k_plan_seg_chunks(fptc_batch b, int E, int wpc, const int64_t *hdr,
                                                                  const int64_t *chunk_off, const int64_t *seg_off,
                                                                  const int32_t *seg_stream,
                                                                  const int64_t *seg_base, ChunkMeta *meta) {
  if (b.n_streams <= 0) return;
  const int64_t g = blockIdx.x;
  // as in k_plan_seg_sums: the stream index is clamped before any read with it
  const int s = clamp_stream(seg_stream[g], b.n_streams);
  const int64_t gb = seg_base[g];
  const int64_t h2 = hdr[2], seg_cap = hdr[3];
  // everything of the stream at once: one round trip before the words
  const SegStream t = seg_stream_of(b, s, seg_off);
  const int64_t c0 = chunk_off[s], nc = chunk_off[s + 1] - c0;
  pin(t.w0), pin(t.w1), pin(t.g0), pin(t.g1), pin(h2), pin(seg_cap), pin(gb), pin(c0), pin(nc);
  if (g >= h2 || t.g1 > seg_cap) return;  // past the plan, or the stream's segments did not fit (flagged)
  constexpr int WPT = kSegWords / kChunkThreads;
  __shared__ int lds[kChunkThreads / kWave];
  SegWords<WPT> sw;
  load_seg_words(b, g, t, sw);
  int tot;
  const int ex = block_excl_scan_dpp(seg_words_sum(sw), lds, tot);
  const int64_t cb = (int64_t)wpc * E;  // symbols per chunk
  int64_t p = gb + ex;
  // the boundaries inside this thread's words, from the first at or after p
  int64_t m = (p + cb - 1) / cb;
  int64_t mb = m * cb;
#pragma unroll
  for (int j = 0; j < WPT; ++j) {
    const int c = sw.cnt(j);
    for (; mb < p + c && m < nc; ++m, mb += cb) {
      const int64_t w = sw.first + j;
      // first word, first symbol and the last flag: one 16-byte store (the
      // chunk before ends at this word, which its reader derives from these)
      *reinterpret_cast<uint4 *>(meta + c0 + m) =
          make_uint4((uint32_t)w, (uint32_t)((uint64_t)w >> 32), (uint32_t)(int32_t)(p - mb), m == nc - 1 ? 1u : 0u);
    }
    p += c;
  }
}

}  // namespace

int launch_plan(const fptc_batch &b, const fptc_codec &c, const Shape &s, const Plan &p, int32_t *status,
                void *stream) {
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_plan_streams, dim3(1), dim3(kPlanThreads), 0, st, b, c.N, c.E, s.wpc, p.hdr, p.win_off,
                     p.chunk_off, p.seg_off, p.seg_stream, p.seg_cap, status);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return (int)e;
  const unsigned nseg = (unsigned)(p.seg_cap > 0 ? p.seg_cap : 1);  // blocks past hdr[2] exit at once
  hipLaunchKernelGGL(k_plan_seg_sums, dim3(nseg), dim3(kSumThreads), 0, st, b, p.hdr, p.seg_off, p.seg_stream,
                     p.seg_sum, status);
  if ((e = hipGetLastError()) != hipSuccess) return (int)e;
  hipLaunchKernelGGL(k_plan_stream_scan, dim3(b.n_streams), dim3(kScanThreads), 0, st, b, c.N, c.E, s.wpc,
                     p.win_off, p.chunk_off, p.seg_off, p.seg_cap, p.seg_sum, p.seg_base, p.tile_stream, p.tile_cap,
                     p.chunk_meta, status);
  if ((e = hipGetLastError()) != hipSuccess) return (int)e;
  hipLaunchKernelGGL(k_plan_seg_chunks, dim3(nseg), dim3(kChunkThreads), 0, st, b, c.E, s.wpc, p.hdr, p.chunk_off,
                     p.seg_off, p.seg_stream, p.seg_base, p.chunk_meta);
  return (int)hipGetLastError();
}

}  // namespace fptc
