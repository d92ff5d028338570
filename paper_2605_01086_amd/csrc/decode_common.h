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
//  * sparse multi-symbol (uint32), for a codebook whose fill symbol F (the
//    symbol of the all-zero peek, i.e. the shortest code) has a 1- or 2-bit
//    code, as for the zero level of sparse spectra: the chunk's symbol buffer
//    is first filled with F, and an entry resolves up to 15 whole codes of
//    which at most two are not F; only those are written:
//      bits  0..7   first non-F symbol (F if none)     bits  8..11 its offset
//      bits 12..15  total length of the codes
//      bits 16..23  second non-F symbol (the first's if none)
//      bits 24..27  its offset                         bits 28..31 count
//    An entry whose first code is missing has offset 15 in slot one (real
//    offsets are at most 14).  Writes past a lane's run are suppressed, so no
//    fix-up is needed.  A per-codebook info word records the form chosen:
//      bit 0 sparse, bits 8..15 F, bits 16..23 code length of F.
//  * two-level (uint16), for codes longer than kShortLmax = 12 bits (the
//    2^lmax-entry table of Section 3.3 would not fit in LDS): a primary table
//    indexed by the first 12 bits of the peek holds the single-symbol entry
//    of every code of at most 12 bits; a 12-bit prefix that starts longer
//    codes holds bit 15, its sub-table's offset (bits 0..11) and index width
//    d - 1 (bits 12..14, d = its longest code's length - 12), and the sub-table
//    entry for the next d bits of the peek is the code's single-symbol entry.
//    At most 256 prefixes start longer codes (each holds a symbol), so the
//    sub-tables never exceed 256 * 16 entries; 16 KB per codebook in all.
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

constexpr int kShortLmax = 12;  // longest code the one-level tables cover
constexpr int kLongPrefixes = 1 << kShortLmax;
constexpr int kLongSub = 256 * 16;  // sub-table entries per codebook, at most

// multi-symbol: entries | code lengths [book][256] | info word per book;
// codes longer than kShortLmax: the two-level tables (primary | sub) per book
__host__ __device__ inline size_t lut_lds_bytes(bool ms, int n_books, int lmax) {
  if (lmax > kShortLmax) return (size_t)n_books * (kLongPrefixes + kLongSub) * 2;
  const size_t e = (size_t)n_books << lmax;
  return ((ms ? e * 4 + (size_t)n_books * 260 : e * 2) + 15) & ~(size_t)15;
}
constexpr uint32_t kSparseMissing = (15u << 8) | (15u << 24) | (1u << 28);
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
__device__ inline void build_lut3(uint32_t *lut3, uint8_t *cl, uint32_t *info, const uint16_t *lut1, int lmax,
                                  int n_books, int tid, int nthreads) {
  const uint32_t mask = (1u << lmax) - 1;
  for (int i = tid; i < (n_books << lmax); i += nthreads) {
    const uint16_t *L = lut1 + (i & ~(int)mask);
    const uint32_t idx = (uint32_t)i & mask;
    // the book's fill symbol: the all-zero peek's code, the shortest one
    const uint32_t z = L[0], lf = z >> 8, fsym = z & 255u;
    const bool sparse = lf >= 1 && lf <= 2;
    if (idx == 0) info[i >> lmax] = (sparse ? 1u : 0u) | (fsym << 8) | (lf << 16);
    const uint32_t e0 = L[idx];
    uint32_t len = e0 >> 8, out;
    if (len == 0) {
      out = sparse ? (kSparseMissing | ((uint32_t)lmax << 12)) : (kLutMissing | (1u << 28) | ((uint32_t)lmax << 24));
    } else {
      cl[(i >> lmax) * 256 + (e0 & 255u)] = (uint8_t)len;  // every entry of a symbol writes the same length
      if (!sparse) {
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
      } else {
        uint32_t c = 1, nf = 0, sa = fsym, oa = 0, sb = 0, ob = 0;
        if ((e0 & 255u) != fsym) {
          sa = e0 & 255u;
          nf = 1;
        }
        while (c < 15) {
          // a run of fill codes is a run of lf-bit zero groups: take it whole
          // (leading zeros of the peek's remaining real bits), then one lookup
          // for the code after it
          const uint32_t v = (idx << len) & mask, real = (uint32_t)lmax - len;
          uint32_t zr = v ? (uint32_t)__clz(v) - (32u - (uint32_t)lmax) : (uint32_t)lmax;
          zr = zr < real ? zr : real;
          const uint32_t k = min(zr / lf, 15u - c);
          c += k;
          len += k * lf;
          if (c >= 15) break;
          const uint32_t e = L[(idx << len) & mask];
          const uint32_t l = e >> 8, s = e & 255u;
          if (l == 0 || len + l > (uint32_t)lmax) break;
          if (s != fsym) {
            if (nf == 2) break;
            if (nf == 0) {
              sa = s;
              oa = c;
            } else {
              sb = s;
              ob = c;
            }
            ++nf;
          }
          len += l;
          ++c;
        }
        if (nf < 2) {
          sb = sa;
          ob = oa;
        }
        out = sa | (oa << 8) | (len << 12) | (sb << 16) | (ob << 24) | (c << 28);
      }
    }
    lut3[i] = out;
  }
}

// An ABI table entry as a two-level table entry: lengths 0 (no code) and
// above lmax (not a valid table) read as length 63, which overruns the word.
__device__ inline uint16_t long_entry(uint16_t e, int lmax) {
  const int l = e >> 8;
  return (l >= 1 && l <= lmax) ? e : (uint16_t)((63u << 8) | (e & 0xffu));
}
// Longest valid code length among n ABI entries (0 if none).
__device__ inline int longest_code(const uint16_t *__restrict__ L, int n, int lmax) {
  int ml = 0;
  for (int j = 0; j < n; ++j) {
    const int l = L[j] >> 8;
    if (l <= lmax) ml = max(ml, l);
  }
  return ml;
}

// Two-level tables of n_books codebooks from the ABI's 2^lmax-entry tables
// (lmax > kShortLmax), one block: each thread sizes the sub-tables of a run
// of prefixes, a block-wide scan places them, then each fills its own.
// scan: LDS scratch of (blockDim / 64 + 1) ints.  Ends with a barrier.
__device__ inline void build_long_tables(uint16_t *tab, const uint16_t *__restrict__ lut_g, int lmax, int n_books,
                                         int tid, int nthreads, int *scan) {
  const int d = lmax - kShortLmax;
  const int per = (kLongPrefixes + nthreads - 1) / nthreads;
  const int lane = tid & 63, wid = tid >> 6;
  for (int b = 0; b < n_books; ++b) {
    const uint16_t *L = lut_g + ((size_t)b << lmax);
    uint16_t *prim = tab + (size_t)b * (kLongPrefixes + kLongSub), *sub = prim + kLongPrefixes;
    // longest code under each of this thread's prefixes (0: none longer than 12 bits)
    int total = 0;
    for (int i = 0; i < per; ++i) {
      const int pfx = tid * per + i;
      if (pfx >= kLongPrefixes) break;
      const int ml = longest_code(L + ((size_t)pfx << d), 1 << d, lmax);
      total += ml > kShortLmax ? 1 << (ml - kShortLmax) : 0;
    }
    // exclusive prefix of the totals over the block
    const int incl = wave_incl_scan_dpp(total);
    if (lane == 63) scan[wid] = incl;
    __syncthreads();
    int off = incl - total;
    for (int w = 0; w < wid; ++w) off += scan[w];
    __syncthreads();  // scan[] is read before the next book writes it
    for (int i = 0; i < per; ++i) {
      const int pfx = tid * per + i;
      if (pfx >= kLongPrefixes) break;
      const size_t base = (size_t)pfx << d;
      const int ml = longest_code(L + base, 1 << d, lmax);
      if (ml <= kShortLmax) {  // a code of at most 12 bits (or no code) covers the prefix
        prim[pfx] = long_entry(L[base], lmax);
        continue;
      }
      const int dp = ml - kShortLmax;
      if (off + (1 << dp) > kLongSub) {  // cannot happen with 256 symbols; refuse the codes
        prim[pfx] = (uint16_t)(63u << 8);
        continue;
      }
      prim[pfx] = (uint16_t)(0x8000u | ((unsigned)(dp - 1) << 12) | (unsigned)off);
      for (int j = 0; j < (1 << dp); ++j) sub[off + j] = long_entry(L[base + ((size_t)j << (d - dp))], lmax);
      off += 1 << dp;
    }
  }
  __syncthreads();
}

// Stage the lookup tables a decode kernel uses.  ms: multi-symbol tables at
// lut (then the code lengths and the info words follow them); temp: LDS scratch of lut1_temp_bytes() that the
// caller overwrites only after a barrier.  Ends with a block barrier.
__device__ inline void stage_decode_tables(bool ms, unsigned char *lut, unsigned char *temp, const uint16_t *lut_g,
                                           int lmax, int n_books, int tid, int nthreads) {
  const int entries = n_books << lmax;
  if (lmax > kShortLmax) {  // two-level tables; temp (at least 64 bytes) holds the scan
    build_long_tables(reinterpret_cast<uint16_t *>(lut), lut_g, lmax, n_books, tid, nthreads,
                      reinterpret_cast<int *>(temp));
    return;
  }
  if (ms) {
    uint16_t *t = reinterpret_cast<uint16_t *>(temp);
    for (int i = tid; i < entries; i += nthreads) t[i] = lut_g[i];
    __syncthreads();
    build_lut3(reinterpret_cast<uint32_t *>(lut), lut + (size_t)entries * 4,
               reinterpret_cast<uint32_t *>(lut + (size_t)entries * 4 + (size_t)n_books * 256), t, lmax, n_books, tid,
               nthreads);
  } else {
    stage_lut(reinterpret_cast<uint16_t *>(lut), lut_g, entries, tid, nthreads);
  }
  __syncthreads();
}

// The words of a chunk's first PR rounds, one per lane per round.
template <int PR = kPreRounds>
struct ChunkWordsT {
  uint64_t w[PR];
  int n[PR];
};
using ChunkWords = ChunkWordsT<kPreRounds>;

template <int PR>
__device__ inline void load_chunk_words(const uint64_t *__restrict__ words, const uint8_t *__restrict__ symlen,
                                        int64_t fw, int64_t wend, int lane, ChunkWordsT<PR> &cw) {
#pragma unroll
  for (int r = 0; r < PR; ++r) {
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
template <int PR>
__device__ inline void settle_chunk_words(const ChunkWordsT<PR> &cw) {
#pragma unroll
  for (int r = 0; r < PR; ++r) asm volatile("" ::"v"(cw.w[r]), "v"(cw.n[r]) : "memory");
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

// Two-level form of decode_word (codes up to lmax <= 16 bits): one primary
// lookup per code, a second one for codes longer than kShortLmax bits.
__device__ inline int decode_word_long(uint64_t wd, unsigned char *p, int cnt, const uint16_t *prim, int lmax,
                                       int hs) {
  unsigned char *const pe = p + cnt;
  const int d = lmax - kShortLmax;
  const uint16_t *sub = prim + kLongPrefixes;
  int bits = 0;
  do {
    const uint32_t peek = (uint32_t)(wd >> 32) >> hs;
    uint32_t e = prim[peek >> d];
    if (e & 0x8000u) {
      const int dp = (int)((e >> 12) & 7u) + 1;
      e = sub[(e & 0xfffu) + ((peek & ((1u << d) - 1)) >> (d - dp))];
    }
    const int len = (int)((e >> 8) & 63u);
    wd <<= len;
    bits += len;
    *p++ = (unsigned char)e;
  } while (p < pe);
  return bits > 64 ? FPTC_STREAM_OVERRUN : 0;
}

// Sparse-table form of decode_word: the buffer already holds the fill symbol
// at every position; lf is the fill symbol's code length.  While 16 or more
// symbols remain no entry can reach past the run, so the slot writes need no
// mask; the last few lookups drop slots past the run.
__device__ inline int decode_word_sparse(uint64_t wd, unsigned char *p, int cnt, const uint32_t *L, const uint8_t *cl,
                                         int hs, int lf) {
  unsigned char *const pe = p + cnt;
  int bits = 0, fl = 0;
  uint32_t e = 0;
  while ((int)(pe - p) >= 16) {
    e = L[(uint32_t)(wd >> 32) >> hs];
    const int len = (e >> 12) & 15;
    wd <<= len;
    bits += len;
    const int oa = (e >> 8) & 15;
    fl = max(fl, oa);
    p[oa] = (unsigned char)e;
    p[(e >> 24) & 15] = (unsigned char)(e >> 16);
    p += e >> 28;
  }
  while (p < pe) {
    e = L[(uint32_t)(wd >> 32) >> hs];
    const int len = (e >> 12) & 15;
    wd <<= len;
    bits += len;
    const int rem = (int)(pe - p);
    const int oa = (e >> 8) & 15, ob = (e >> 24) & 15;
    fl = max(fl, oa);
    if (oa < rem) p[oa] = (unsigned char)e;
    if (ob < rem) p[ob] = (unsigned char)(e >> 16);
    p += e >> 28;
  }
  // the last entry's codes past the run are not part of this word's count
  const int c = (int)(e >> 28), k = (int)(pe - (p - c));  // k: its symbols inside the run
  if (c > k) {
    const int oa = (e >> 8) & 15, ob = (e >> 24) & 15;
    const int a = oa < k, b = (ob < k) && (ob != oa);
    bits += (k - a - b) * lf + (a ? (int)cl[e & 255u] : 0) + (b ? (int)cl[(e >> 16) & 255u] : 0) -
            (int)((e >> 12) & 15);
  }
  return (fl == 15 || bits > 64) ? FPTC_STREAM_OVERRUN : 0;
}

// Fill sb[0 .. t_cnt) with the fill symbol (whole 16-byte blocks from sb's
// 16-byte boundary down, so a few bytes around the range are written too).
__device__ inline void prefill_symbols(unsigned char *sb, int t_cnt, uint32_t fsym, int lane) {
  const int mis = (int)(reinterpret_cast<uintptr_t>(sb) & 15);
  unsigned char *q = sb - mis;
  const uint32_t f4 = 0x01010101u * fsym;
  const uint4 v = make_uint4(f4, f4, f4, f4);
  const int nblk = (mis + t_cnt + 15) >> 4;
  for (int i = lane; i < nblk; i += 64) reinterpret_cast<uint4 *>(q)[i] = v;
}

// One round: 64 words, one per lane; a DPP prefix sum of symlen places each
// lane's run at chunk-relative index o, and the lane decodes the run's part
// inside [.., t_cnt).  P advances by the round's symbol count.
template <bool MS, bool LG = false>
__device__ inline void decode_round(uint64_t word, int n, int &P, int t_cnt, const void *lut, const uint8_t *cl,
                                    uint32_t binfo, int hs, unsigned char *sb, int &err, int lmax = 0) {
  if (n > 64) {
    err |= FPTC_STREAM_BAD_SYMLEN;
    n = 64;
  }
  const int incl = wave_incl_scan_dpp(n);
  const int total = __builtin_amdgcn_readlane(incl, 63);
  const int o = P + incl - n;
  const int cnt = min(n, t_cnt - o);
  if (cnt > 0) {
    if constexpr (LG)
      err |= decode_word_long(word, sb + o, cnt, reinterpret_cast<const uint16_t *>(lut), lmax, hs);
    else if (MS && (binfo & 1u))
      err |= decode_word_sparse(word, sb + o, cnt, reinterpret_cast<const uint32_t *>(lut), cl, hs,
                                (int)((binfo >> 16) & 255u));
    else
      err |= decode_word<MS>(word, sb + o, cnt, lut, cl, hs);
  }
  P += total;
}

// Decode symbols [0, t_cnt) of a chunk into sb[0 .. t_cnt), one wavefront.
// fw is the first word holding a symbol of the chunk, p0 <= 0 the chunk-
// relative index of that word's first symbol, wend the stream's word end;
// cw holds the first PR rounds of words (load_chunk_words), later
// rounds are loaded here one round ahead.  binfo: the codebook's info word
// (multi-symbol tables; 0 otherwise).  Returns this lane's error bits.
template <bool MS, int PR, bool LG = false>
__device__ inline int decode_chunk(const uint64_t *__restrict__ words, const uint8_t *__restrict__ symlen, int64_t fw,
                                   int p0, int t_cnt, int64_t wend, const ChunkWordsT<PR> &cw, const void *lut,
                                   const uint8_t *cl, uint32_t binfo, int hs, unsigned char *sb, int lane,
                                   int lmax = 0) {
  int err = 0, P = p0;
  if (MS && (binfo & 1u)) prefill_symbols(sb, t_cnt, (binfo >> 8) & 255u, lane);
  int64_t w = fw;
#pragma unroll
  for (int r = 0; r < PR; ++r) {
    if (P < t_cnt && w < wend) decode_round<MS, LG>(cw.w[r], cw.n[r], P, t_cnt, lut, cl, binfo, hs, sb, err, lmax);
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
      decode_round<MS, LG>(word, n, P, t_cnt, lut, cl, binfo, hs, sb, err, lmax);
      w += 64;
    }
  }
  return err;
}

}  // namespace fptc
