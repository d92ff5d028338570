// Batch planning kernels (stream/chunk setup and the symlen prefix sums).
//
// Section 4.2 places each word's decoded symbols by an exclusive prefix sum of
// the per-word symbol counts.  Here the sum is taken in two levels over the
// whole symlen array cut into 4096-word segments (each segment's total and
// its 64-word partial prefixes), and a stream's symbols before any of its
// words follow from those as differences; only the words where a chunk of
// `wpc` windows begins are recorded: a chunk then decodes from that word on
// its own, with no cross-chunk dependency.  Two launches: the stream pass
// (one workgroup) beside the segment sums (one wavefront per segment), which
// need nothing of each other, then the chunk starts (one wavefront per piece
// of a stream in a segment).
#include <hip/hip_runtime.h>

#include "fptc_internal.h"
#include "mfma_common.h"

namespace fptc {
namespace {

constexpr int kPlanThreads = 1024;
constexpr int64_t kSegWords = 4096;  // words per segment (a multiple of 64 x 64)
constexpr int kSegShift = 12;
static_assert(kSegWords == (int64_t)1 << kSegShift && kSegWords == kWave * 64, "segment geometry");
// Every pass takes a segment (or a stream's piece of one) per wavefront:
// 64 lanes x 64 words, four 16-byte symlen loads per lane, no barrier.
constexpr int kSumThreads = kWave;

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

// Exclusive block scan of two values at once (one set of barriers).
template <int THREADS>
__device__ inline void block_excl_scan2(int64_t a, int64_t b, int64_t *lds, int64_t &ea, int64_t &eb, int64_t &ta,
                                        int64_t &tb) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  constexpr int NW = THREADS / kWave;
  const int64_t ia = wave_incl_scan(a), ib = wave_incl_scan(b);
  if (lane == kWave - 1) lds[wid] = ia, lds[NW + 1 + wid] = ib;
  __syncthreads();
  if (wid == 0) {
    const int64_t x = lane < NW ? lds[lane] : 0, y = lane < NW ? lds[NW + 1 + lane] : 0;
    const int64_t xi = wave_incl_scan(x), yi = wave_incl_scan(y);
    if (lane < NW) lds[lane] = xi - x, lds[NW + 1 + lane] = yi - y;
    if (lane == NW - 1) lds[NW] = xi, lds[2 * NW + 1] = yi;
  }
  __syncthreads();
  ea = ia - a + lds[wid];
  eb = ib - b + lds[NW + 1 + wid];
  ta = lds[NW];
  tb = lds[2 * NW + 1];
  __syncthreads();
}

// ceil(a / d) for 0 <= a, 1 <= d: 32-bit division whenever the operands
// allow (the 64-bit one is a long instruction sequence).
__device__ inline int64_t ceil_div(int64_t a, int d) {
  const uint64_t x = (uint64_t)a + (uint64_t)(d - 1);
  if (x >> 32) return (int64_t)(x / (uint64_t)d);
  return (int64_t)((uint32_t)x / (uint32_t)d);
}

// One workgroup: per-stream window, segment-piece and chunk counts, their
// exclusive prefix sums, header validation, and the piece -> stream map.  A
// stream's pieces are the segments its words touch (segment k holds words
// [kSegWords k, kSegWords (k + 1)) of the batch).  A stream gets no chunks when its header is bad, when
// it has windows but no words (its symbol count is wrong) or when its
// segments do not fit the capacity (word ranges of streams overlap); it is
// flagged, and nothing later reads its words.  Each thread takes
// kStreamsPerThread consecutive streams (all their offsets loaded at once),
// so a batch of up to kPlanThreads * kStreamsPerThread streams needs one pass
// of block scans.
constexpr int kStreamsPerThread = 4;

__device__ void stream_pass(const fptc_batch &b, int N, int E, int wpc, int64_t *hdr, int64_t *win_off,
                            int64_t *chunk_off, int64_t *seg_off, int2 *seg_map, int64_t seg_cap,
                            int32_t *status) {
  __shared__ int64_t lds[2 * (kPlanThreads / kWave + 1)];
  constexpr int K = kStreamsPerThread;
  __shared__ int64_t seg_at[kPlanThreads * K + 1];  // this pass's streams: first piece of each, then the end
  __shared__ int32_t seg_g0[kPlanThreads * K];      // this pass's streams: the segment of each one's first word
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
    int64_t tw = 0, tg = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      flag[k] = 0;
      nw[k] = 0;
      if (s0 + k < n) {
        if (so[k] < 0 || so[k + 1] < so[k] || so[k + 1] > b.n_samples || wo[k] < 0 || wo[k + 1] < wo[k] ||
            wo[k + 1] > b.n_words)
          flag[k] = FPTC_STREAM_BAD_HEADER;
        else
          nw[k] = ceil_div(so[k + 1] - so[k], N);
      }
      if (!flag[k] && nw[k] > 0 && wo[k + 1] <= wo[k]) flag[k] = FPTC_STREAM_BAD_COUNT;  // windows, no words
      const int64_t a0 = wo[k] & ~(kSegWords - 1);
      ng[k] = (flag[k] || nw[k] == 0) ? 0 : ceil_div(wo[k + 1] - a0, (int)kSegWords);
      tw += nw[k];
      tg += ng[k];
    }
    int64_t w_at, g_at, tot, g_tot;
    block_excl_scan2<kPlanThreads>(tw, tg, lds, w_at, g_at, tot, g_tot);
    w_at += carry_w;
    g_at += carry_g;
    carry_w += tot;
    const int64_t g_pass = carry_g;  // this pass's first segment
    carry_g += g_tot;
    int64_t tc = 0;
    int64_t wx[K], gx[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      wx[k] = w_at;
      gx[k] = g_at;
      // windows past the batch's capacity, or segments past theirs (word
      // ranges of streams overlap): a bad header, which takes precedence
      if (s0 + k < n && !(flag[k] & FPTC_STREAM_BAD_HEADER) && (w_at + nw[k] > win_cap || g_at + ng[k] > seg_cap))
        flag[k] = FPTC_STREAM_BAD_HEADER;
      w_at += nw[k];
      g_at += ng[k];
      nc[k] = flag[k] ? 0 : ceil_div(nw[k], wpc);
      tc += nc[k];
    }
    int64_t c_at = carry_c + block_excl_scan<int64_t, kPlanThreads>(tc, lds, tot);
    carry_c += tot;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int s = s0 + k;
      if (s < n) {
        win_off[s] = wx[k];
        chunk_off[s] = c_at;
        seg_off[s] = gx[k];
        if (status) status[s] = flag[k];
      }
      seg_at[threadIdx.x * K + k] = gx[k];  // past n: the pass's end
      seg_g0[threadIdx.x * K + k] = (int32_t)(wo[k] >> kSegShift);
      c_at += nc[k];
    }
    if (threadIdx.x == 0) seg_at[kPlanThreads * K] = carry_g;
    __syncthreads();
    // piece -> (stream, segment) map: each thread a contiguous range of this
    // pass's pieces (an even number, so that aligned pairs leave as one
    // 16-byte store), its first stream by binary search, then walking forward
    const int64_t per = ((g_tot + kPlanThreads - 1) / kPlanThreads + 1) & ~(int64_t)1;
    const int64_t g_lo = g_pass + (int64_t)threadIdx.x * per;
    const int64_t g_hi = min(min(g_lo + per, carry_g), seg_cap);
    if (g_lo < g_hi) {
      int lo = 0, hi = kPlanThreads * K - 1;  // last local stream whose first piece is <= g_lo
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (seg_at[mid] <= g_lo) lo = mid;
        else hi = mid - 1;
      }
      int i = lo;
      for (int64_t g = g_lo; g < g_hi; g += 2) {
        int2 v[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          // g + q < g_hi <= the pass's end = seg_at[kPlanThreads * K]: the walk stops inside
          if (g + q < g_hi)
            while (seg_at[i + 1] <= g + q) ++i;
          v[q] = make_int2(base + i, seg_g0[i] + (int32_t)(g + q - seg_at[i]));
        }
        if (g + 2 <= g_hi && ((reinterpret_cast<uintptr_t>(seg_map + g) & 15) == 0)) {
          *reinterpret_cast<int4 *>(seg_map + g) = make_int4(v[0].x, v[0].y, v[1].x, v[1].y);
        } else {
#pragma unroll
          for (int q = 0; q < 2; ++q)
            if (g + q < g_hi) seg_map[g + q] = v[q];
        }
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

// Each byte of four packed symlen counts clamped to 64.
__device__ inline uint32_t clamp64x4(uint32_t v) {
  if (!((v & 0x80808080u) | (((v & 0x7f7f7f7fu) + 0x3f3f3f3fu) & 0x80808080u))) return v;
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t e = (v >> (8 * k)) & 255u;
    c |= (e > 64u ? 64u : e) << (8 * k);
  }
  return c;
}

// Segment G's symlen bytes for this lane: words [kSegWords G + WPT lane,
// + WPT), packed four to a dword; words past the array read as 0.  0 <= G.
template <int WPT>
__device__ inline void load_segment_words(const fptc_batch &b, int64_t G, SegWords<WPT> &sw) {
  static_assert(WPT % 16 == 0, "whole 16-byte symlen blocks per thread");
  const int64_t first = (G << kSegShift) + (int64_t)(threadIdx.x & (kWave - 1)) * WPT;
  sw.first = first;
  if ((reinterpret_cast<uintptr_t>(b.symlen) & 15) == 0 && first + WPT <= b.n_words) {
    // the lane's whole range inside the array: its 16-byte loads back to back
    // (first is a multiple of 16)
    const uint4 *src = reinterpret_cast<const uint4 *>(b.symlen + first);
#pragma unroll
    for (int q = 0; q < WPT / 16; ++q) {
      const uint4 u = src[q];
      sw.x[4 * q] = u.x, sw.x[4 * q + 1] = u.y, sw.x[4 * q + 2] = u.z, sw.x[4 * q + 3] = u.w;
    }
  } else {
#pragma unroll
    for (int d = 0; d < WPT / 4; ++d) sw.x[d] = 0;
    for (int j = 0; j < WPT && first + j < b.n_words; ++j) sw.x[j >> 2] |= (uint32_t)b.symlen[first + j] << (8 * (j & 3));
  }
}

// Keep the stream's words [w0, w1) of a loaded segment (the others read as
// 0); a count above 64 is clamped to 64 and reported.
template <int WPT>
__device__ inline int keep_stream_words(SegWords<WPT> &sw, const SegStream &t) {
  const int64_t lo64 = t.w0 - sw.first, hi64 = t.w1 - sw.first;
  if (lo64 > 0 || hi64 < WPT) {  // only the lanes at the stream's two ends, or outside it
    const int lo = lo64 > 0 ? (int)(lo64 < WPT ? lo64 : WPT) : 0;
    const int hi = hi64 < WPT ? (int)(hi64 > 0 ? hi64 : 0) : WPT;
#pragma unroll
    for (int d = 0; d < WPT / 4; ++d) {
      // bytes [lo - 4 d, hi - 4 d) of this dword, each bound clamped to [0, 4]
      const int a = min(max(lo - 4 * d, 0), 4), e = min(max(hi - 4 * d, 0), 4);
      const uint32_t keep_hi = (uint32_t)(((uint64_t)1 << (8 * e)) - 1);  // bytes below e
      const uint32_t drop_lo = (uint32_t)(((uint64_t)1 << (8 * a)) - 1);  // bytes below a
      sw.x[d] &= keep_hi & ~drop_lo;
    }
  }
  int bad = 0;
#pragma unroll
  for (int d = 0; d < WPT / 4; ++d) {
    const uint32_t c = clamp64x4(sw.x[d]);
    bad |= c != sw.x[d];
    sw.x[d] = c;
  }
  return bad ? FPTC_STREAM_BAD_SYMLEN : 0;
}

// The sum of a thread's counts.
template <int WPT>
__device__ inline int seg_words_sum(const SegWords<WPT> &sw) {
  uint32_t sum = 0;
#pragma unroll
  for (int d = 0; d < WPT / 4; ++d) sum = __builtin_amdgcn_sad_u8(sw.x[d], 0u, sum);
  return (int)sum;
}

// Exclusive scan across the segment's one wavefront; total = the wave's sum.
__device__ inline int seg_excl_scan(int v, int &total) {
  const int incl = wave_incl_scan_dpp(v);
  total = __builtin_amdgcn_readlane(incl, kWave - 1);
  return incl - v;
}

// One wavefront: segment G's symbol count and the exclusive prefix of its
// 64-word blocks (symlen clamped to 64, as everywhere in the plan; the flag
// for a larger one is raised where a stream's words are read).
__device__ void segment_sums(const fptc_batch &b, int64_t G, int32_t *gseg_sum, int32_t *gseg_lane) {
  const int lane = threadIdx.x & (kWave - 1);
  SegWords<kSegWords / kWave> sw;
  load_segment_words(b, G, sw);
  uint32_t sum = 0;
#pragma unroll
  for (int d = 0; d < kSegWords / kWave / 4; ++d) sum = __builtin_amdgcn_sad_u8(clamp64x4(sw.x[d]), 0u, sum);
  const int incl = wave_incl_scan_dpp((int)sum);
  gseg_lane[(G << 6) + lane] = incl - (int)sum;
  if (lane == kWave - 1) gseg_sum[G] = incl;
}

// The first launch: workgroup 0 runs the stream pass; every wavefront of the
// others sums one segment.  The two need nothing of each other.
constexpr int kSumWavesPerBlock = kPlanThreads / kWave;

__global__ void __launch_bounds__(kPlanThreads) k_plan_pass1(fptc_batch b, int N, int E, int wpc, int64_t *hdr,
                                                             int64_t *win_off, int64_t *chunk_off, int64_t *seg_off,
                                                             int2 *seg_map, int64_t seg_cap, int32_t *gseg_sum,
                                                             int32_t *gseg_lane, int64_t n_gseg, int32_t *status) {
  if (blockIdx.x == 0) {
    stream_pass(b, N, E, wpc, hdr, win_off, chunk_off, seg_off, seg_map, seg_cap, status);
    return;
  }
  const int64_t G = (int64_t)(blockIdx.x - 1) * kSumWavesPerBlock + (threadIdx.x >> 6);
  if (G < n_gseg) segment_sums(b, G, gseg_sum, gseg_lane);
}

// What the chunk records need of a stream.
struct StreamChunks {
  int64_t c0, nc;   // the stream's chunks
  int64_t wo0, nw;  // its windows
  int64_t so, L;    // its samples
  int64_t w1;       // the end of its words
  int s, book;
};

// Chunk m's whole record (Section 4.2's per-chunk offsets): where its words
// start (first_word, or -1 when no word starts it) and its fixed fields.
__device__ inline void put_record(ChunkMeta *meta, int64_t m, int64_t fw, int32_t fs, const StreamChunks &r, int N,
                                  int E, int wpc) {
  const int64_t wb = m * wpc;
  const int64_t nwc = r.nw - wb < wpc ? r.nw - wb : wpc;
  const int64_t ol = r.L - wb * N < nwc * N ? r.L - wb * N : nwc * N;
  const int64_t sym_base = (r.wo0 + wb) * E, out_base = r.so + wb * N;
  uint4 *d = reinterpret_cast<uint4 *>(meta + r.c0 + m);
  d[0] = make_uint4((uint32_t)fw, (uint32_t)((uint64_t)fw >> 32), (uint32_t)fs, m == r.nc - 1 ? 1u : 0u);
  d[1] = make_uint4((uint32_t)r.w1, (uint32_t)((uint64_t)r.w1 >> 32), (uint32_t)sym_base,
                    (uint32_t)((uint64_t)sym_base >> 32));
  d[2] = make_uint4((uint32_t)out_base, (uint32_t)((uint64_t)out_base >> 32), (uint32_t)nwc, (uint32_t)ol);
  d[3] = make_uint4((uint32_t)r.s, (uint32_t)r.book, 0u, 0u);
}
static_assert(offsetof(ChunkMeta, first_sym) == 8 && offsetof(ChunkMeta, last) == 12 &&
                  offsetof(ChunkMeta, word_end) == 16 && offsetof(ChunkMeta, sym_base) == 24 &&
                  offsetof(ChunkMeta, out_base) == 32 && offsetof(ChunkMeta, n_windows) == 40 &&
                  offsetof(ChunkMeta, out_len) == 44 && offsetof(ChunkMeta, stream) == 48 &&
                  offsetof(ChunkMeta, book) == 52,
              "put_record writes ChunkMeta as four 16-byte groups");

__device__ inline int64_t wave_sum64(int64_t v) {
#pragma unroll
  for (int d = kWave / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

// One wavefront per segment.  Its base is the symbols of the stream's
// earlier segments (their sums, added up); the chunks whose first symbol (a
// multiple of wpc * E) falls in the segment are [m_lo, m_hi), one per lane in
// turn, and each lane finds the word whose symbol range [p, p + symlen) holds
// its chunk's first symbol: the lane of the segment by a binary search over
// the lanes' exclusive prefixes, then the word among that lane's 64 counts,
// both kept in LDS.  Consecutive lanes then write consecutive records.  The
// stream's last segment also checks the stream's symbol count and writes the
// records of the chunks no word starts (-1: skipped), which exist only when
// the count is short; the two sets are disjoint, so every record is written
// exactly once.
__global__ void __launch_bounds__(kSumThreads) k_plan_seg_chunks(fptc_batch b, int N, int E, int wpc,
                                                                  const int64_t *hdr, const int64_t *win_off,
                                                                  const int64_t *chunk_off, const int64_t *seg_off,
                                                                  const int2 *seg_map, int64_t n_gseg,
                                                                  const int32_t *gseg_sum, const int32_t *gseg_lane,
                                                                  ChunkMeta *meta, int32_t *status) {
  constexpr int WPT = kSegWords / kSumThreads;
  __shared__ uint32_t counts[kSegWords / 4];  // lane l's packed counts at [l * WPT / 4, (l + 1) * WPT / 4)
  __shared__ int lane_at[kWave + 1];          // exclusive prefix of the lanes' totals, then the total
  if (b.n_streams <= 0 || n_gseg <= 0) return;
  const int64_t g = blockIdx.x;
  const int lane = threadIdx.x;
  // g < seg_cap, so this read is in bounds; past the plan's pieces it may
  // hold anything, so the stream and the segment are clamped before any read
  // with them (such a wavefront then returns on the check below)
  const int2 sg = seg_map[g];
  const int s = clamp_stream(sg.x, b.n_streams);
  const int64_t G = sg.y < 0 ? 0 : (sg.y >= n_gseg ? n_gseg - 1 : (int64_t)sg.y);
  // everything of the stream at once, then the segment's words beside it:
  // one round trip
  const int64_t h2 = hdr[2], seg_cap = hdr[3];
  const SegStream t = seg_stream_of(b, s, seg_off);
  StreamChunks r;
  r.c0 = chunk_off[s];
  r.nc = chunk_off[s + 1] - r.c0;
  r.wo0 = win_off[s];
  r.nw = win_off[s + 1] - r.wo0;
  r.so = b.sample_off[s];
  r.L = b.sample_off[s + 1] - r.so;
  r.w1 = t.w1;
  r.s = s;
  r.book = b.book_id ? (int)b.book_id[s] : 0;
  SegWords<WPT> sw;
  load_segment_words(b, G, sw);
  pin(t.w0), pin(t.w1), pin(t.g0), pin(t.g1), pin(h2), pin(seg_cap), pin(r.c0), pin(r.nc), pin(r.wo0), pin(r.nw),
      pin(r.so), pin(r.L);
  // past the plan, a stream without chunks, or (never, with the stream
  // pass's map) a piece outside its stream's pieces
  if (g >= h2 || t.g1 > seg_cap || r.nc <= 0 || g < t.g0 || g >= t.g1) return;
  // The stream's symbols before this piece: the whole segments from the
  // stream's first one up to this one, less what of the first precedes the
  // stream's first word w0 (its 64-word blocks before w0's, then w0's block
  // up to w0).  All of these words exist (w0 <= the piece's first word).
  int64_t before = 0;
  const int64_t j = g - t.g0;  // this piece's index in the stream
  if (j > 0) {
    const int64_t G0 = t.w0 >> kSegShift;
    const int l0 = (int)((t.w0 - (G0 << kSegShift)) >> 6);
    const int64_t blk = (G0 << kSegShift) + ((int64_t)l0 << 6);
    int64_t v = 0;
    const int32_t a0 = lane < j ? gseg_sum[G0 + lane] : 0;
    const int32_t a1 = lane + kWave < j ? gseg_sum[G0 + lane + kWave] : 0;
    const int pre = blk + lane < t.w0 ? (int)b.symlen[blk + lane] : 0;
    const int32_t pl = lane == 0 ? gseg_lane[(G0 << 6) + l0] : 0;
    v = (int64_t)a0 + a1 - (pre > 64 ? 64 : pre) - pl;
    for (int64_t i = lane + 2 * kWave; i < j; i += kWave) v += gseg_sum[G0 + i];  // streams of > 128 segments
    before = v;
  }
  const int bad = keep_stream_words(sw, t);
  if (bad && status) atomicOr(&status[s], bad);
#pragma unroll
  for (int q = 0; q < WPT / 16; ++q)
    *reinterpret_cast<uint4 *>(&counts[lane * (WPT / 4) + 4 * q]) =
        make_uint4(sw.x[4 * q], sw.x[4 * q + 1], sw.x[4 * q + 2], sw.x[4 * q + 3]);
  int tot;
  const int ex = seg_excl_scan(seg_words_sum(sw), tot);
  lane_at[lane] = ex;
  if (lane == 0) lane_at[kWave] = tot;
  if (j > 0) before = wave_sum64(before);
  wave_sync_lds();
  const int64_t cb = (int64_t)wpc * E;  // symbols per chunk
  const int64_t m_lo = (before + cb - 1) / cb;
  const int64_t m_end = (before + tot + cb - 1) / cb;
  const int64_t m_hi = m_end < r.nc ? m_end : r.nc;
  const int64_t first = sw.first - (int64_t)lane * WPT;  // the segment's first word
  for (int64_t m = m_lo + lane; m < m_hi; m += kWave) {
    const int at = (int)(m * cb - before);  // in [0, tot)
    int lo = 0, hi = kWave - 1;             // the last lane whose prefix is <= at
#pragma unroll
    for (int step = 0; step < 6; ++step) {
      const int mid = (lo + hi + 1) >> 1;
      if (lane_at[mid] <= at) lo = mid;
      else hi = mid - 1;
    }
    int q = lane_at[lo], j = 0;
    const uint32_t *cl = counts + lo * (WPT / 4);
    uint32_t v = cl[0];
    for (int d = 0; d < WPT / 4; ++d) {  // the dword, then the byte, holding symbol `at`
      v = cl[d];
      const int c4 = (int)__builtin_amdgcn_sad_u8(v, 0u, 0u);
      j = 4 * d;
      if (at < q + c4) break;
      q += c4;
    }
    for (int k = 0; k < 3; ++k, ++j) {
      const int c = (int)(v & 255u);
      if (at < q + c) break;
      q += c;
      v >>= 8;
    }
    put_record(meta, m, first + (int64_t)lo * WPT + j, q - at, r, N, E, wpc);
  }
  if (g == t.g1 - 1) {
    const int64_t total = before + tot;
    if (lane == 0 && total != r.nw * E && status) atomicOr(&status[s], FPTC_STREAM_BAD_COUNT);
    for (int64_t k = m_end + lane; k < r.nc; k += kWave) put_record(meta, k, -1, 0, r, N, E, wpc);
  }
}

}  // namespace

int launch_plan(const fptc_batch &b, const fptc_codec &c, const Shape &s, const Plan &p, int32_t *status,
                void *stream) {
  hipStream_t st = (hipStream_t)stream;
  const int64_t sum_blocks = (p.n_gseg + kSumWavesPerBlock - 1) / kSumWavesPerBlock;
  hipLaunchKernelGGL(k_plan_pass1, dim3((unsigned)(1 + sum_blocks)), dim3(kPlanThreads), 0, st, b, c.N, c.E, s.wpc,
                     p.hdr, p.win_off, p.chunk_off, p.seg_off, reinterpret_cast<int2 *>(p.seg_map), p.seg_cap,
                     p.gseg_sum, p.gseg_lane,
                     p.n_gseg, status);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return (int)e;
  const unsigned nseg = (unsigned)(p.seg_cap > 0 ? p.seg_cap : 1);  // wavefronts past hdr[2] exit at once
  hipLaunchKernelGGL(k_plan_seg_chunks, dim3(nseg), dim3(kSumThreads), 0, st, b, c.N, c.E, s.wpc, p.hdr, p.win_off,
                     p.chunk_off, p.seg_off, reinterpret_cast<const int2 *>(p.seg_map), p.n_gseg, p.gseg_sum,
                     p.gseg_lane, p.chunk_meta, status);
  return (int)hipGetLastError();
}

}  // namespace fptc
