// Huffman decode with output compaction (Section 4.2, lossless stage).
//
// Work item = one chunk of `wpc` windows of one stream, owned by one 64-lane
// wavefront.  The plan gives the first word holding a symbol of the chunk and
// that word's in-stream symbol index.  The wavefront then takes 64 words at a
// time, one word per lane (the paper's one-thread-per-word rule), forms the
// exclusive prefix sum of their symlen across the wave to place every lane's
// run, and each lane decodes exactly symlen[w] symbols by peeking lmax bits
// into the codebook's lookup table held in LDS.  Symbols that belong to the
// chunk are written into a per-wave LDS buffer laid out on the destination's
// 16-byte grid, and the buffer is then stored with 16-byte coalesced writes
// (the AMD counterpart of the paper's warp-broadcast compaction).
#include <hip/hip_runtime.h>

#include "fptc_internal.h"

namespace fptc {
namespace {

__device__ inline int wave_incl_scan_i32(int v) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    int u = __shfl_up(v, d, kWave);
    if (lane >= d) v += u;
  }
  return v;
}

// Index of the stream owning chunk c: the last s with chunk_off[s] <= c.
__device__ inline int find_stream(const int64_t *off, int n, int64_t c) {
  int lo = 0, hi = n;  // invariant off[lo] <= c < off[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (off[mid] <= c) lo = mid;
    else hi = mid;
  }
  return lo;
}

__global__ void k_decode(fptc_batch b, int N, int E, int lmax, int n_books, int wpc, const uint16_t *lut_g,
                         const int64_t *hdr, const int64_t *win_off, const int64_t *chunk_off,
                         const int64_t *chunk_word, const int64_t *chunk_wsym, uint8_t *symbols, int32_t *status) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int lut_entries = n_books << lmax;
  uint16_t *lut = reinterpret_cast<uint16_t *>(lds);
  const int lut_bytes = ((lut_entries * 2) + 15) & ~15;
  const int buf_bytes = ((wpc * E + 16) + 15) & ~15;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = threadIdx.x & (kWave - 1);
  unsigned char *buf = lds + lut_bytes + wid * buf_bytes;

  for (int i = threadIdx.x; i < lut_entries; i += blockDim.x) lut[i] = lut_g[i];
  __syncthreads();

  const int64_t n_chunks = hdr[0];
  const int waves_per_block = blockDim.x / kWave;
  const int64_t stride = (int64_t)gridDim.x * waves_per_block;
  const int shift = 64 - lmax;

  for (int64_t c = (int64_t)blockIdx.x * waves_per_block + wid; c < n_chunks; c += stride) {
    const int s = find_stream(chunk_off, b.n_streams, c);
    const int64_t fw = chunk_word[c];
    if (fw < 0) continue;  // the stream's symbol count is wrong; already flagged
    const int64_t m = c - chunk_off[s];
    const int64_t nw = win_off[s + 1] - win_off[s];
    const int64_t t_beg = m * wpc * (int64_t)E;
    const int64_t t_end = min((m + 1) * wpc, nw) * (int64_t)E;
    const int64_t w_end = b.word_off[s + 1];
    const int book = b.book_id ? (int)b.book_id[s] : 0;
    const uint16_t *L = lut + ((book < n_books ? book : 0) << lmax);
    uint8_t *dst = symbols + win_off[s] * (int64_t)E + t_beg;
    const int mis = (int)(reinterpret_cast<uintptr_t>(dst) & 15);
    int err = 0;

    int64_t P = chunk_wsym[c];
    for (int64_t w = fw; P < t_end && w < w_end; w += kWave) {
      const int64_t wi = w + lane;
      uint64_t word = 0;
      int n = 0;
      if (wi < w_end) {
        word = b.words[wi];
        n = b.symlen[wi];
        if (n > 64) {
          err |= FPTC_STREAM_BAD_SYMLEN;
          n = 64;
        }
      }
      const int incl = wave_incl_scan_i32(n);
      const int total = __shfl(incl, kWave - 1, kWave);
      const int64_t o = P + (incl - n);
      const int64_t hi = min(o + n, t_end);
      if (o < t_end && o + n > t_beg) {
        int pos = 0;
        const int cnt = (int)(hi - o);
        for (int j = 0; j < cnt; ++j) {
          if (pos >= 64) {
            err |= FPTC_STREAM_OVERRUN;
            break;
          }
          const uint32_t peek = (uint32_t)((word << pos) >> shift);
          const uint32_t e = L[peek];
          const int len = (int)(e >> 8);
          if (len == 0 || pos + len > 64) {
            err |= FPTC_STREAM_OVERRUN;
            break;
          }
          pos += len;
          const int64_t t = o + j;
          if (t >= t_beg) buf[mis + (int)(t - t_beg)] = (unsigned char)(e & 0xffu);
        }
      }
      P += total;
    }
    if (err && status) atomicOr(&status[s], err);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    // Store buf[mis .. mis + nbytes) to dst with 16-byte writes on the
    // destination's 16-byte grid; partial first/last blocks byte by byte.
    const int nbytes = (int)(t_end - t_beg);
    const int64_t sym_base = win_off[s] * (int64_t)E + t_beg;  // element index of dst[0]
    uint8_t *dst_al = dst - mis;
    const int nblk = (mis + nbytes + 15) >> 4;
    for (int k = lane; k < nblk; k += kWave) {
      const int lo = k * 16, hi2 = lo + 16;
      if (lo >= mis && hi2 <= mis + nbytes && sym_base - mis + hi2 <= b.n_symbols) {
        *reinterpret_cast<uint4 *>(dst_al + lo) = *reinterpret_cast<const uint4 *>(buf + lo);
      } else {
        for (int j = lo; j < hi2; ++j)
          if (j >= mis && j < mis + nbytes && sym_base + (j - mis) < b.n_symbols) dst_al[j] = buf[j];
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

}  // namespace

int launch_decode(const fptc_batch &b, const fptc_codec &c, const Shape &s, const Plan &p, uint8_t *symbols,
                  int32_t *status, void *stream) {
  const int threads = s.waves * kWave;
  const int lut_bytes = (((c.n_books << c.lmax) * 2) + 15) & ~15;
  const int buf_bytes = ((s.wpc * c.E + 16) + 15) & ~15;
  const size_t lds = (size_t)lut_bytes + (size_t)s.waves * buf_bytes;
  int blocks = s.blocks > 0 ? s.blocks : device_cu_count() * 8;
  hipLaunchKernelGGL(k_decode, dim3(blocks), dim3(threads), lds, (hipStream_t)stream, b, c.N, c.E, c.lmax, c.n_books,
                     s.wpc, c.lut, p.hdr, p.win_off, p.chunk_off, p.chunk_word, p.chunk_wsym, symbols, status);
  return (int)hipGetLastError();
}

}  // namespace fptc
