// Huffman decode with output compaction (Section 4.2, lossless stage).
//
// Work item = one chunk of `wpc` windows of one stream, owned by one 64-lane
// wavefront.  The plan gives the chunk's stream, the first word holding a
// symbol of the chunk and that word's in-stream symbol index.  The wavefront
// then takes 64 words at a time, one word per lane (the paper's
// one-thread-per-word rule), forms the exclusive prefix sum of their symlen
// across the wave to place every lane's run, and each lane decodes exactly
// symlen[w] symbols by peeking lmax bits into the codebook's lookup table held
// in LDS (decode_range).  Symbols that belong to the
// chunk are written into a per-wave LDS buffer laid out on the destination's
// 16-byte grid, and the buffer is then stored with 16-byte coalesced writes
// (the AMD counterpart of the paper's warp-broadcast compaction).
#include <hip/hip_runtime.h>

#include "decode_common.h"
#include "fptc_internal.h"

namespace fptc {
namespace {

__global__ void __launch_bounds__(1024) k_decode(const uint64_t *__restrict__ words, const uint8_t *__restrict__ symlen, int n_streams,
                         int64_t n_symbols, int E, int lmax, int n_books, int wpc, const uint16_t *lut_g,
                         const int64_t *hdr, const ChunkMeta *__restrict__ meta, uint8_t *symbols, int32_t *status) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int lut_entries = n_books << lmax;
  uint16_t *lut = reinterpret_cast<uint16_t *>(lds);
  const int lut_bytes = ((lut_entries * 2) + 15) & ~15;
  const int buf_bytes = ((wpc * E + 16) + 15) & ~15;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = threadIdx.x & (kWave - 1);
  unsigned char *buf = lds + lut_bytes + wid * buf_bytes;

  stage_lut(lut, lut_g, lut_entries, threadIdx.x, blockDim.x);
  __syncthreads();

  const int64_t n_chunks = hdr[0];
  const int waves_per_block = blockDim.x / kWave;
  const int hs = 32 - lmax;

  for (int64_t c = (int64_t)blockIdx.x * waves_per_block + wid; c < n_chunks; c += (int64_t)gridDim.x * waves_per_block) {
    const ChunkMeta cm = meta[c];
    if (cm.first_word < 0) continue;  // the stream's symbol count is wrong; already flagged
    const int s = cm.stream < 0 ? 0 : (cm.stream >= n_streams ? n_streams - 1 : cm.stream);
    const int book = cm.book < n_books ? cm.book : 0;
    const int nbytes = cm.n_windows * E;
    uint8_t *dst = symbols + cm.sym_base;
    const int mis = (int)(reinterpret_cast<uintptr_t>(dst) & 15);

    const int err = decode_range(words, symlen, cm.first_word, cm.first_sym, nbytes, cm.word_end,
                                 lut + (book << lmax), hs, buf + mis, lane);
    if (err && status) atomicOr(&status[s], err);
    wave_sync_lds();

    // Store buf[mis .. mis + nbytes) to dst with 16-byte writes on the
    // destination's 16-byte grid; partial first/last blocks byte by byte.
    uint8_t *dst_al = dst - mis;
    const int64_t sym_base = cm.sym_base;
    const int nblk = (mis + nbytes + 15) >> 4;
    for (int k = lane; k < nblk; k += kWave) {
      const int lo = k * 16, hi2 = lo + 16;
      if (lo >= mis && hi2 <= mis + nbytes && sym_base - mis + hi2 <= n_symbols) {
        *reinterpret_cast<uint4 *>(dst_al + lo) = *reinterpret_cast<const uint4 *>(buf + lo);
      } else {
        for (int j = lo; j < hi2; ++j)
          if (j >= mis && j < mis + nbytes && sym_base + (j - mis) < n_symbols) dst_al[j] = buf[j];
      }
    }
    wave_sync_lds();
  }
}

}  // namespace

size_t decode_lds_bytes(const fptc_codec &c, const Shape &s) {
  const size_t lut_bytes = (((size_t)(c.n_books << c.lmax) * 2) + 15) & ~(size_t)15;
  const size_t buf_bytes = (((size_t)s.wpc * c.E + 16) + 15) & ~(size_t)15;
  return lut_bytes + (size_t)s.waves * buf_bytes;
}

int launch_decode(const fptc_batch &b, const fptc_codec &c, const Shape &s, const Plan &p, uint8_t *symbols,
                  int32_t *status, void *stream) {
  const int threads = s.waves * kWave;
  const size_t lds = decode_lds_bytes(c, s);
  static bool attr_set = false;
  if (!attr_set) {
    if (hipFuncSetAttribute(reinterpret_cast<const void *>(k_decode), hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024) != hipSuccess)
      return (int)hipErrorInvalidValue;
    attr_set = true;
  }
  const int per_cu = (int)((160 * 1024) / lds);
  int blocks = s.blocks > 0 ? s.blocks : device_cu_count() * (per_cu < 1 ? 1 : (per_cu > 8 ? 8 : per_cu));
  hipLaunchKernelGGL(k_decode, dim3(blocks), dim3(threads), lds, (hipStream_t)stream, b.words, b.symlen, b.n_streams,
                     b.n_symbols, c.E, c.lmax, c.n_books, s.wpc, c.lut, p.hdr, p.chunk_meta, symbols, status);
  return (int)hipGetLastError();
}

}  // namespace fptc
