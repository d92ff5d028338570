// Huffman decode with output compaction (Section 4.2, lossless stage).
//
// Work item = one chunk of `wpc` windows of one stream, owned by one 64-lane
// wavefront.  The plan gives the chunk's stream, the first word holding a
// symbol of the chunk and that word's in-stream symbol index.  The wavefront
// then takes 64 words at a time, one word per lane (the paper's
// one-thread-per-word rule), forms the exclusive prefix sum of their symlen
// across the wave to place every lane's run, and each lane decodes exactly
// symlen[w] symbols by peeking lmax bits into the codebook's lookup table held
// in LDS (decode_chunk; three symbols per lookup where the multi-symbol table
// fits in LDS).  The next chunk's first words are loaded while the current
// chunk decodes.  Symbols that belong to the
// chunk are written into a per-wave LDS buffer laid out on the destination's
// 16-byte grid, and the buffer is then stored with 16-byte coalesced writes
// (the AMD counterpart of the paper's warp-broadcast compaction).
#include <hip/hip_runtime.h>

#include "decode_common.h"
#include "fptc_internal.h"

namespace fptc {
namespace {

// prefix | up to 15 bytes of destination misalignment | the chunk's symbols |
// room for the two bytes a decode lookup may write past the last run
__host__ __device__ inline size_t decode_wave_bytes(int wpc, int E) {
  return (size_t)kSymPrefix + ((((size_t)wpc * E + 32) + 15) & ~(size_t)15);
}

// LDS: lookup tables, then one symbol buffer per wave, then the chunk
// counter (16 B); the multi-symbol build borrows lut1_temp_bytes after the
// tables before the buffers are used.
__host__ __device__ inline size_t decode_lds(bool ms, int n_books, int lmax, int wpc, int E, int waves) {
  const size_t t = lut_lds_bytes(ms, n_books, lmax);
  const size_t need = t + (size_t)waves * decode_wave_bytes(wpc, E) + 16;
  const size_t tmp = (ms && lmax <= kShortLmax) ? t + lut1_temp_bytes(n_books, lmax) : 0;
  return need > tmp ? need : tmp;
}

template <bool MS, bool LG>
__global__ void __launch_bounds__(1024) k_decode(const uint64_t *__restrict__ words, const uint8_t *__restrict__ symlen,
                                                 int n_streams, int64_t n_symbols, int E, int lmax, int n_books,
                                                 int wpc, const uint16_t *__restrict__ lut_g,
                                                 const int64_t *__restrict__ hdr, const ChunkMeta *__restrict__ meta,
                                                 uint8_t *symbols, int32_t *status) {
  extern __shared__ __align__(16) unsigned char lds[];
  const size_t lut_bytes = lut_lds_bytes(MS, n_books, lmax);
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = threadIdx.x & (kWave - 1);
  unsigned char *buf = lds + lut_bytes + wid * decode_wave_bytes(wpc, E) + kSymPrefix;
  const void *lut = lds;
  const uint8_t *cl = lds + ((size_t)n_books << lmax) * 4;
  const uint32_t *binfo = reinterpret_cast<const uint32_t *>(cl + n_books * 256);  // multi-symbol form only

  stage_decode_tables(MS, lds, lds + lut_bytes, lut_g, lmax, n_books, threadIdx.x, blockDim.x);

  const int64_t n_chunks = hdr[0];
  const int waves_per_block = blockDim.x / kWave;
  const int64_t cstride = (int64_t)gridDim.x * waves_per_block;
  // the counter may share LDS with the table build's scratch: set after it
  unsigned *chunk_ctr = reinterpret_cast<unsigned *>(lds + lut_bytes + waves_per_block * decode_wave_bytes(wpc, E));
  if (threadIdx.x == 0) *chunk_ctr = 0;
  __syncthreads();
  const int hs = 32 - lmax;

  // Software pipeline over this wave's chunks: the words of the next chunk
  // (and the record of the one after) are requested before this chunk
  // decodes and waited for right after the decode, before this chunk's
  // stores; with in-order vector memory counters that wait also covers the
  // previous chunk's stores, which had the decode to drain.
  // (chunks from the workgroup's schedule, BlockChunks)
  const BlockChunks sched{chunk_ctr, (int64_t)blockIdx.x, cstride, (int64_t)gridDim.x, waves_per_block};
  int64_t c = sched.next(lane), cn = sched.next(lane);
  ChunkMeta cm = meta_from_lanes(load_meta_lane(meta, c, n_chunks, lane), c < n_chunks);
  const uint32_t vn = load_meta_lane(meta, cn, n_chunks, lane);
  ChunkWords cw{};
  if (c < n_chunks) load_chunk_words(words, symlen, cm.first_word, cm.word_end, lane, cw);
  ChunkMeta nm = meta_from_lanes(vn, cn < n_chunks);
  while (c < n_chunks) {
    const int64_t cmm = sched.next(lane);
    const uint32_t vm = load_meta_lane(meta, cmm, n_chunks, lane);
    ChunkWords nx{};
    if (cn < n_chunks) load_chunk_words(words, symlen, nm.first_word, nm.word_end, lane, nx);
    const bool ok = cm.first_word >= 0;  // else the stream's symbol count is wrong; already flagged
    const int s = cm.stream < 0 ? 0 : (cm.stream >= n_streams ? n_streams - 1 : cm.stream);
    const int book = cm.book < n_books && cm.book >= 0 ? cm.book : 0;
    const int nbytes = cm.n_windows * E;
    uint8_t *dst = symbols + cm.sym_base;
    const int mis = (int)(reinterpret_cast<uintptr_t>(dst) & 15);
    int err = 0;
    if (ok) {
      const void *lb = LG   ? (const void *)((const uint16_t *)lut + (size_t)book * (kLongPrefixes + kLongSub))
                       : MS ? (const void *)((const uint32_t *)lut + (book << lmax))
                            : (const void *)((const uint16_t *)lut + (book << lmax));
      err = decode_chunk<MS, kPreRounds, LG>(words, symlen, cm.first_word, cm.first_sym, nbytes, cm.word_end, cw, lb,
                                             cl + book * 256, MS ? binfo[book] : 0u, hs, buf + mis, lane, lmax);
    }
    settle_chunk_words(nx);
    settle_lane(vm);
    const ChunkMeta mm = meta_from_lanes(vm, cmm < n_chunks);
    cw = nx;
    if (ok) {
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
          // non-temporal: whole 16-byte blocks of a contiguous stream
          typedef uint32_t u4 __attribute__((ext_vector_type(4)));
          __builtin_nontemporal_store(*reinterpret_cast<const u4 *>(buf + lo), reinterpret_cast<u4 *>(dst_al + lo));
        } else {
          for (int j = lo; j < hi2; ++j)
            if (j >= mis && j < mis + nbytes && sym_base + (j - mis) < n_symbols) dst_al[j] = buf[j];
        }
      }
      wave_sync_lds();
    }
    cm = nm;
    nm = mm;
    c = cn;
    cn = cmm;
  }
}

template <bool MS, bool LG>
int launch_t(const fptc_batch &b, const fptc_codec &c, const Shape &s, const Plan &p, uint8_t *symbols,
             int32_t *status, void *stream) {
  const int threads = s.waves * kWave;
  const size_t lds = decode_lds(MS, c.n_books, c.lmax, s.wpc, c.E, s.waves);
  const int per_cu = (int)((160 * 1024) / lds);
  int blocks = s.blocks > 0 ? s.blocks : device_cu_count() * (per_cu < 1 ? 1 : (per_cu > 8 ? 8 : per_cu));
  hipLaunchKernelGGL((k_decode<MS, LG>), dim3(blocks), dim3(threads), lds, (hipStream_t)stream, b.words, b.symlen,
                     b.n_streams, b.n_symbols, c.E, c.lmax, c.n_books, s.wpc, c.lut, p.hdr, p.chunk_meta, symbols,
                     status);
  return (int)hipGetLastError();
}

}  // namespace

int set_decode_attributes() {
  return lds_attr(k_decode<true, false>) | lds_attr(k_decode<false, false>) | lds_attr(k_decode<false, true>);
}

// The smaller (single-symbol) layout: what the launch needs at least.
size_t decode_lds_bytes(const fptc_codec &c, const Shape &s) {
  return decode_lds(false, c.n_books, c.lmax, s.wpc, c.E, s.waves);
}

int launch_decode(const fptc_batch &b, const fptc_codec &c, const Shape &s, const Plan &p, uint8_t *symbols,
                  int32_t *status, void *stream) {
  if (c.lmax > kShortLmax) return launch_t<false, true>(b, c, s, p, symbols, status, stream);
  if (decode_lds(true, c.n_books, c.lmax, s.wpc, c.E, s.waves) <= 160 * 1024)
    return launch_t<true, false>(b, c, s, p, symbols, status, stream);
  return launch_t<false, false>(b, c, s, p, symbols, status, stream);
}

}  // namespace fptc
