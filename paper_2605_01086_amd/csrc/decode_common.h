// The per-chunk Huffman decode loop shared by the stand-alone decode kernel and
// the fused kernel (Section 4.2, lossless stage).
#pragma once

#include <hip/hip_runtime.h>

#include "fptc_internal.h"
#include "mfma_common.h"

namespace fptc {

// Decode symbols [0, t_cnt) of a chunk into sb[0 .. t_cnt), one 64-lane
// wavefront.  fw is the first word holding a symbol of the chunk and p0 the
// chunk-relative index of that word's first symbol (<= 0); wend bounds the
// stream's words.  Words go 64 at a time, one per lane; a DPP prefix sum of
// their symlen places each lane's run; each lane decodes exactly symlen[w]
// symbols (fewer at the chunk's end) by peeking the top lmax bits (hi32 >> hs)
// into the lookup table Lb and shifting the word by the code length.  The
// next 64 words are loaded while the current ones decode.  Entries of Lb with
// length 63 mark missing codes.  Returns FPTC_STREAM_* error bits of this lane.
__device__ inline int decode_range(const uint64_t *__restrict__ words, const uint8_t *__restrict__ symlen, int64_t fw,
                                   int p0, int t_cnt, int64_t wend, const uint16_t *Lb, int hs, unsigned char *sb,
                                   int lane) {
  int err = 0;
  int P = p0;
  int64_t w = fw;
  uint64_t nword = 0;
  int nn = 0;
  if (w + lane < wend) {
    nword = words[w + lane];
    nn = symlen[w + lane];
  }
  while (P < t_cnt && w < wend) {
    const uint64_t word = nword;
    int n = nn;
    nword = 0;
    nn = 0;
    if (w + 64 + lane < wend) {
      nword = words[w + 64 + lane];
      nn = symlen[w + 64 + lane];
    }
    if (n > 64) {
      err |= FPTC_STREAM_BAD_SYMLEN;
      n = 64;
    }
    const int incl = wave_incl_scan_dpp(n);
    const int total = __builtin_amdgcn_readlane(incl, 63);
    const int o = P + incl - n;  // chunk-relative index of this lane's first symbol
    const int cnt = min(n, t_cnt - o);
    if (cnt > 0) {
      uint64_t wd = word;
      int bits = 0, j = 0;
      for (; j < cnt && o + j < 0; ++j) {  // symbols of the previous chunk
        const uint32_t e = Lb[(uint32_t)(wd >> 32) >> hs];
        const int len = (int)(e >> 8);
        wd <<= len;
        bits += len;
      }
      for (; j < cnt; ++j) {
        const uint32_t e = Lb[(uint32_t)(wd >> 32) >> hs];
        const int len = (int)(e >> 8);
        wd <<= len;
        bits += len;
        sb[o + j] = (unsigned char)e;
      }
      if (bits > 64) err |= FPTC_STREAM_OVERRUN;
    }
    P += total;
    w += 64;
  }
  return err;
}

// Stage a codebook's lookup table into LDS; a missing code (length 0) becomes
// length 63 so that reading it overruns the word and is reported.
__device__ inline void stage_lut(uint16_t *lut, const uint16_t *lut_g, int entries, int tid, int nthreads) {
  for (int i = tid; i < entries; i += nthreads) {
    const uint16_t e = lut_g[i];
    lut[i] = (e >> 8) ? e : (uint16_t)((63u << 8) | (e & 0xffu));
  }
}

__device__ inline void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace fptc
