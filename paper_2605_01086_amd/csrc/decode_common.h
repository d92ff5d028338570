// The per-chunk Huffman decode shared by the stand-alone decode kernel and the
// fused kernels (Section 4.2, lossless stage).
//
// Lookup tables held in LDS:
//  * single-symbol (uint16, the ABI's format): symbol | code length << 8; a
//    missing code (length 0) is staged as length 63 so that reading it
//    overruns the word and is reported.
//  * multi-symbol (uint32), built in LDS from the single-symbol table: the
//    lmax-bit peek resolves every whole code inside it, up to three:
//      bits  0..23  the symbols, first in the low byte (unused bytes 0)
//      bits 24..27  total length of those codes (what the word shifts by)
//      bits 28..29  how many symbols (1..3)
//      bit  30      the first code is missing (stream corrupt)
//    With a mean code length of a few bits this cuts the serial lookups per
//    word by 2-3x.  A per-codebook code-length table (symbol -> length) lets
//    the last lookup of a run discount symbols that lie past the run, so the
//    consumed-bit count stays exact for the overrun check.  Each lookup
//    writes all three symbol bytes; the at most two that fall past a lane's
//    run land on the first two positions of a later run, and every run writes
//    its first two symbols again once all lanes have finished.
#pragma once

#include <hip/hip_runtime.h>

#include "fptc_internal.h"
#include "mfma_common.h"

namespace fptc {

// Bytes reserved in front of a wavefront's symbol buffer: the first word of a
// chunk may start up to 63 symbols before the chunk, and the merged decode
// loop writes those symbols there instead of branching around them.
constexpr int kSymPrefix = 64;
// Rounds of 64 words whose loads are issued one chunk ahead.
constexpr int kPreRounds = 2;
constexpr uint32_t kLutMissing = 1u << 30;

__host__ __device__ inline size_t lut_lds_bytes(bool ms, int n_books, int lmax) {
  const size_t e = (size_t)n_books << lmax;
  return ((ms ? e * 4 + (size_t)n_books * 256 : e * 2) + 15) & ~(size_t)15;
}
__host__ __device__ inline size_t lut1_temp_bytes(int n_books, int lmax) {
  return (((size_t)n_books << lmax) * 2 + 15) & ~(size_t)15;
}

// Stage a codebook's single-symbol table into LDS (missing code -> length 63).
__device__ inline void stage_lut(uint16_t *lut, const uint16_t *lut_g, int entries, int tid, int nthreads) {
  for (int i = tid; i < entries; i += nthreads) {
    const uint16_t e = lut_g[i];
    lut[i] = (e >> 8) ? e : (uint16_t)((63u << 8) | (e & 0xffu));
  }
}

// Build the multi-symbol tables of n_books codebooks from single-symbol tables
// already in LDS (lut1, ABI format: length 0 = missing).  lut3 receives
// n_books << lmax entries, cl n_books * 256 code lengths.  A follow-on code is
// taken only when its whole length lies inside the peek: the bits after the
// first codes are then a prefix of the real stream, and prefix-freeness makes
// the table's answer for them the real next code.
__device__ inline void build_lut3(uint32_t *lut3, uint8_t *cl, const uint16_t *lut1, int lmax, int n_books, int tid,
                                  int nthreads) {
  const uint32_t mask = (1u << lmax) - 1;
  for (int i = tid; i < (n_books << lmax); i += nthreads) {
    const uint16_t *L = lut1 + (i & ~(int)mask);
    const uint32_t idx = (uint32_t)i & mask;
    const uint32_t e0 = L[idx];
    uint32_t len = e0 >> 8, out;
    if (len == 0) {
      out = kLutMissing | (1u << 28) | ((uint32_t)lmax << 24);
    } else {
      cl[(i >> lmax) * 256 + (e0 & 255u)] = (uint8_t)len;  // every entry of a symbol writes the same length
      out = e0 & 255u;
      uint32_t c = 1;
      for (int k = 1; k < 3; ++k) {
        const uint32_t e = L[(idx << len) & mask];
        const uint32_t l = e >> 8;
        if (l == 0 || len + l > (uint32_t)lmax) break;
        out |= (e & 255u) << (8 * c);
        len += l;
        ++c;
      }
      out |= (len << 24) | (c << 28);
    }
    lut3[i] = out;
  }
}

// Stage the lookup tables a decode kernel uses.  ms: multi-symbol tables at
// lut (then cl follows them); temp: LDS scratch of lut1_temp_bytes() that the
// caller overwrites only after a barrier.  Ends with a block barrier.
__device__ inline void stage_decode_tables(bool ms, unsigned char *lut, unsigned char *temp, const uint16_t *lut_g,
                                           int lmax, int n_books, int tid, int nthreads) {
  const int entries = n_books << lmax;
  if (ms) {
    uint16_t *t = reinterpret_cast<uint16_t *>(temp);
    for (int i = tid; i < entries; i += nthreads) t[i] = lut_g[i];
    __syncthreads();
    build_lut3(reinterpret_cast<uint32_t *>(lut), lut + (size_t)entries * 4, t, lmax, n_books, tid, nthreads);
  } else {
    stage_lut(reinterpret_cast<uint16_t *>(lut), lut_g, entries, tid, nthreads);
  }
  __syncthreads();
}

// The words of a chunk's first kPreRounds rounds, one per lane per round.
struct ChunkWords {
  uint64_t w[kPreRounds];
  int n[kPreRounds];
};

__device__ inline void load_chunk_words(const uint64_t *__restrict__ words, const uint8_t *__restrict__ symlen,
                                        int64_t fw, int64_t wend, int lane, ChunkWords &cw) {
#pragma unroll
  for (int r = 0; r < kPreRounds; ++r) {
    const int64_t w = fw + 64 * r + lane;
    cw.w[r] = 0;
    cw.n[r] = 0;
    if (fw >= 0 && w < wend) {
      cw.w[r] = words[w];
      cw.n[r] = symlen[w];
    }
  }
}

// Make the prefetched words available at this point of the program: an empty
// asm statement that reads them makes the compiler place its wait for their
// loads here rather than at the loop's back edge, where it would also wait
// for every store issued in between.
__device__ inline void settle_chunk_words(const ChunkWords &cw) {
#pragma unroll
  for (int r = 0; r < kPreRounds; ++r) asm volatile("" ::"v"(cw.w[r]), "v"(cw.n[r]) : "memory");
}

// Decode cnt > 0 symbols of one word into p[0 .. cnt); p may start up to 63
// bytes before the chunk (kSymPrefix).  Returns FPTC_STREAM_* bits.
template <bool MS>
__device__ inline int decode_word(uint64_t wd, unsigned char *p, int cnt, const void *lut, const uint8_t *cl, int hs) {
  unsigned char *const pe = p + cnt;
  int bits = 0, err = 0;
  if constexpr (MS) {
    const uint32_t *L = reinterpret_cast<const uint32_t *>(lut);
    const uint64_t w0 = wd;
    unsigned char *const p0 = p;
    uint32_t e, fl = 0;
    do {
      e = L[(uint32_t)(wd >> 32) >> hs];
      const int len = (e >> 24) & 15;
      wd <<= len;
      bits += len;
      fl |= e;
      // all three bytes, whatever the count: up to two may land past this
      // run, on the start of a later run, which writes its first two symbols
      // again after every lane's loop (below)
      p[0] = (unsigned char)e;
      p[1] = (unsigned char)(e >> 8);
      p[2] = (unsigned char)(e >> 16);
      p += (e >> 28) & 3;
    } while (p < pe);
    // symbols of the last lookup past the run are not part of this word's count
    const int c = (e >> 28) & 3;
    const int rem = (int)(pe - p) + c;  // symbols the last lookup still had to give
    const int l1 = cl[(e >> 8) & 255u], l2 = cl[(e >> 16) & 255u];
    bits -= (c > 1 && rem < 2) ? l1 : 0;
    bits -= (c > 2 && rem < 3) ? l2 : 0;
    if (fl & kLutMissing) err |= FPTC_STREAM_OVERRUN;
    // the first two symbols of this run, written again now that every lane of
    // the wave has left its loop
    const uint32_t f0 = L[(uint32_t)(w0 >> 32) >> hs];
    const uint32_t f1 = L[(uint32_t)((w0 << ((f0 >> 24) & 15)) >> 32) >> hs];
    p0[0] = (unsigned char)f0;
    if (cnt > 1) p0[1] = (unsigned char)(((f0 >> 28) & 3) > 1 ? (f0 >> 8) : f1);
  } else {
    const uint16_t *L = reinterpret_cast<const uint16_t *>(lut);
    do {
      const uint32_t e = L[(uint32_t)(wd >> 32) >> hs];
      const int len = (int)(e >> 8);
      wd <<= len;
      bits += len;
      *p++ = (unsigned char)e;
    } while (p < pe);
  }
  if (bits > 64) err |= FPTC_STREAM_OVERRUN;
  return err;
}

// One round: 64 words, one per lane; a DPP prefix sum of symlen places each
// lane's run at chunk-relative index o, and the lane decodes the run's part
// inside [.., t_cnt).  P advances by the round's symbol count.
template <bool MS>
__device__ inline void decode_round(uint64_t word, int n, int &P, int t_cnt, const void *lut, const uint8_t *cl,
                                    int hs, unsigned char *sb, int &err) {
  if (n > 64) {
    err |= FPTC_STREAM_BAD_SYMLEN;
    n = 64;
  }
  const int incl = wave_incl_scan_dpp(n);
  const int total = __builtin_amdgcn_readlane(incl, 63);
  const int o = P + incl - n;
  const int cnt = min(n, t_cnt - o);
  if (cnt > 0) err |= decode_word<MS>(word, sb + o, cnt, lut, cl, hs);
  P += total;
}

// Decode symbols [0, t_cnt) of a chunk into sb[0 .. t_cnt), one wavefront.
// fw is the first word holding a symbol of the chunk, p0 <= 0 the chunk-
// relative index of that word's first symbol, wend the stream's word end;
// cw holds the first kPreRounds rounds of words (load_chunk_words), later
// rounds are loaded here one round ahead.  Returns this lane's error bits.
template <bool MS>
__device__ inline int decode_chunk(const uint64_t *__restrict__ words, const uint8_t *__restrict__ symlen, int64_t fw,
                                   int p0, int t_cnt, int64_t wend, const ChunkWords &cw, const void *lut,
                                   const uint8_t *cl, int hs, unsigned char *sb, int lane) {
  int err = 0, P = p0;
  int64_t w = fw;
#pragma unroll
  for (int r = 0; r < kPreRounds; ++r) {
    if (P < t_cnt && w < wend) decode_round<MS>(cw.w[r], cw.n[r], P, t_cnt, lut, cl, hs, sb, err);
    w += 64;
  }
  if (P < t_cnt && w < wend) {
    uint64_t nword = 0;
    int nn = 0;
    if (w + lane < wend) {
      nword = words[w + lane];
      nn = symlen[w + lane];
    }
    while (P < t_cnt && w < wend) {
      const uint64_t word = nword;
      const int n = nn;
      nword = 0;
      nn = 0;
      if (w + 64 + lane < wend) {
        nword = words[w + 64 + lane];
        nn = symlen[w + 64 + lane];
      }
      decode_round<MS>(word, n, P, t_cnt, lut, cl, hs, sb, err);
      w += 64;
    }
  }
  return err;
}

}  // namespace fptc
