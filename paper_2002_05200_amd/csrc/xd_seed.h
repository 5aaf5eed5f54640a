// xd_seed.h -- seed choice on the GPU: one exact shared k-mer per read pair,
// picked by binning the pair's k-mer matches by diagonal.
//
// The paper's application (Section V) starts each extension from a k-mer the
// two reads share, chosen by binning: the positions of shared k-mers estimate
// the overlap, and the consensus bin supplies the seed.  Reading taken (the
// paper gives no formula): every exact match (p, q), A[p, p+k) == B[q, q+k),
// lies on diagonal q - p; diagonals fall into bins of `width`
// (bin floor((q - p) / width)); the bin with the most matches wins, the lower
// bin on a tie; the seed is that bin's match with the smallest p, then q.
//
// One workgroup per pair.  B's k-mers go into an open-addressing hash table
// in LDS whose 4-byte slots hold a k-mer's position and 19 further bits of
// its hash (a tag); the packed bases of B's segment sit in LDS beside it, so
// a probe compares tags first and verifies only a candidate whose tag agrees
// by re-reading its k-mer there.  Each thread walks a contiguous run of A's
// k-mers and rolls the k-mer code along it.  A is streamed through LDS in chunks, every
// k-mer of A probes the table, and each exact match adds to its diagonal
// bin's count and lowers the bin's smallest (p, q) with LDS atomics.  Reads
// longer than one table fill run segment by segment (A is scanned once per
// segment), and pairs with more diagonal bins than LDS holds run the bins
// window by window.  All of it is HBM-light: each base is read from HBM once
// per segment pass and the rest is LDS traffic.
#pragma once

#include <hip/hip_runtime.h>

#include "xdrop.h"

namespace xd {

constexpr int kSeedThreads = 512;
constexpr int kSeedTabBits = 13;
constexpr int kSeedTab = 1 << kSeedTabBits;   // hash slots: positions of B's k-mers
constexpr int kSeedSeg = kSeedTab / 2;        // k-mers of B per table fill (load <= 1/2)
constexpr int kSeedChunk = kSeedSeg;          // k-mers of A per LDS chunk
constexpr int kSeedBins = 2048;               // diagonal bins per window
// packed words of one segment or chunk: up to 15 bases of the first word
// before it, kSeedSeg k-mers of up to 31 bases, and the two words the last
// k-mer's three-word read may touch
constexpr int kSeedWords = (15 + kSeedSeg + 30 + 15) / 16 + 2;
constexpr uint32_t kSeedEmpty = 0u;          // slot = (tag << 13) | (position + 1)
constexpr int kSeedTagBits = 19;
static_assert(kSeedSeg <= (1 << 13) - 1, "positions + 1 fit the slot's 13 low bits");
constexpr int kSeedMaxK = 31;

struct SeedArgs {
  const uint32_t *A;
  const uint32_t *B;
  int64_t a_words, b_words;
  xd_pair *pairs;
  int64_t n_pairs;
  int32_t k;
  uint32_t width;
  int32_t set_pairs;
  xd_seed *out;
};

// The k-mer starting at base t of a packed LDS buffer, base t + s in bits
// 2s, 2s+1 (any fixed bijection serves: only equality is used).
__device__ __forceinline__ uint64_t seed_kmer(const uint32_t *w, uint32_t t, uint64_t mask) {
  const uint32_t wi = t >> 4, sh = (t & 15u) * 2u;
  uint64_t v = ((uint64_t)w[wi] | ((uint64_t)w[wi + 1] << 32)) >> sh;
  if (sh) v |= (uint64_t)w[wi + 2] << (64u - sh);
  return v & mask;
}

// Fibonacci (multiplicative) hashing of a k-mer code: the top bits index the
// table, the next kSeedTagBits bits are the tag kept in the slot.
__device__ __forceinline__ uint64_t seed_mix(uint64_t code) {
  return code * 0x9E3779B97F4A7C15ull;
}
__device__ __forceinline__ uint32_t seed_index(uint64_t mix) {
  return (uint32_t)(mix >> (64 - kSeedTabBits));
}
__device__ __forceinline__ uint32_t seed_tag(uint64_t mix) {
  return (uint32_t)(mix >> (64 - kSeedTabBits - kSeedTagBits)) & ((1u << kSeedTagBits) - 1u);
}

// Packed words [g0 / 16, g0 / 16 + nw) of an arena into LDS (zero past its end).
__device__ __forceinline__ void seed_load(uint32_t *dst, const uint32_t *src, int64_t words,
                                          int64_t g0, int nw) {
  const int64_t w0 = g0 >> 4;
  for (int i = threadIdx.x; i < nw; i += kSeedThreads) {
    const int64_t g = w0 + i;
    dst[i] = g < words ? src[g] : 0u;
  }
}

// (count, bin) of the better of two candidates: more matches, then lower bin.
__device__ __forceinline__ bool seed_better(unsigned long long c1, uint32_t b1,
                                            unsigned long long c2, uint32_t b2) {
  return c1 > c2 || (c1 == c2 && b1 < b2);
}

__global__ __launch_bounds__(kSeedThreads) void k_find_seeds(SeedArgs S) {
  __shared__ uint32_t tab[kSeedTab];
  __shared__ uint32_t bw[kSeedWords];
  __shared__ uint32_t aw[kSeedWords];
  __shared__ unsigned long long bcount[kSeedBins];
  __shared__ unsigned long long bkey[kSeedBins];
  __shared__ unsigned long long red_c[kSeedThreads / 64];
  __shared__ uint32_t red_b[kSeedThreads / 64];
  __shared__ unsigned long long s_total;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int64_t k = S.k;
  const uint64_t kmask = (k >= 32) ? ~0ull : ((1ull << (2 * k)) - 1ull);
  const uint64_t w = S.width;

  for (int64_t pi = blockIdx.x; pi < S.n_pairs; pi += gridDim.x) {
    __syncthreads();   // the previous pair's LDS readers are done
    const xd_pair pr = S.pairs[pi];
    const int64_t m = pr.a_len, n = pr.b_len;
    xd_seed res;
    res.a_seed = 0; res.b_seed = 0; res.found = 0; res.status = XD_OK;
    res.bin_matches = 0; res.matches = 0;
    const bool bad = (int64_t)(pr.a_off + pr.a_len) > S.a_words * 16 ||
                     (int64_t)(pr.b_off + pr.b_len) > S.b_words * 16 ||
                     pr.a_off > (uint64_t(1) << 60) || pr.b_off > (uint64_t(1) << 60);
    if (bad) {
      res.status = XD_EINVAL;
    } else if (m >= k && n >= k) {
      const int64_t nA = m - k + 1, nB = n - k + 1;
      // bin floor((q - p) / w) counted from the lowest possible one:
      // (q - p + off) / w with off = ceil((m - k) / w) * w
      const uint64_t off = ((uint64_t)(m - k) + w - 1) / w * w;
      const uint64_t nbins = ((uint64_t)(n - k) + off) / w + 1;
      unsigned long long best_c = 0, best_key = 0;
      if (tid == 0) s_total = 0;
      for (uint64_t win = 0; win < nbins; win += kSeedBins) {
        __syncthreads();
        for (int i = tid; i < kSeedBins; i += kSeedThreads) {
          bcount[i] = 0;
          bkey[i] = ~0ull;
        }
        unsigned long long my_total = 0;
        for (int64_t seg = 0; seg < nB; seg += kSeedSeg) {
          const int seg_n = (int)(nB - seg < kSeedSeg ? nB - seg : kSeedSeg);
          __syncthreads();   // earlier probes of the table and of bw are done
          for (int i = tid; i < kSeedTab; i += kSeedThreads) tab[i] = kSeedEmpty;
          const int64_t gb = (int64_t)pr.b_off + seg;
          const uint32_t sb = (uint32_t)(gb & 15);
          seed_load(bw, S.B, S.b_words, gb, (int)((sb + seg_n + k - 1 + 15) / 16) + 2);
          __syncthreads();
          for (int v = tid; v < seg_n; v += kSeedThreads) {
            const uint64_t mix = seed_mix(seed_kmer(bw, sb + v, kmask));
            const uint32_t entry = (seed_tag(mix) << 13) | (uint32_t)(v + 1);
            uint32_t h = seed_index(mix);
            while (atomicCAS(&tab[h], kSeedEmpty, entry) != kSeedEmpty)
              h = (h + 1) & (kSeedTab - 1);
          }
          for (int64_t ach = 0; ach < nA; ach += kSeedChunk) {
            const int a_n = (int)(nA - ach < kSeedChunk ? nA - ach : kSeedChunk);
            __syncthreads();   // inserts done; the previous chunk's readers done
            const int64_t ga = (int64_t)pr.a_off + ach;
            const uint32_t sa = (uint32_t)(ga & 15);
            seed_load(aw, S.A, S.a_words, ga, (int)((sa + a_n + k - 1 + 15) / 16) + 2);
            __syncthreads();
            // a contiguous run of A's k-mers per thread, the code rolled along it
            const int run = (a_n + kSeedThreads - 1) / kSeedThreads;
            const int u0 = tid * run, u1 = u0 + run < a_n ? u0 + run : a_n;
            uint64_t code = u0 < u1 ? seed_kmer(aw, sa + u0, kmask) : 0;
            for (int u = u0; u < u1; ++u) {
              if (u > u0) {   // base u + k - 1 enters at the top, base u - 1 leaves
                const uint32_t t = sa + (uint32_t)(u + k - 1);
                code = (code >> 2) | ((uint64_t)((aw[t >> 4] >> ((t & 15u) * 2u)) & 3u)
                                      << (2 * (k - 1)));
              }
              const uint64_t mix = seed_mix(code);
              const uint32_t tag = seed_tag(mix);
              uint32_t h = seed_index(mix);
              for (;;) {
                const uint32_t e = tab[h];
                if (e == kSeedEmpty) break;
                const uint32_t v = (e & 0x1FFFu) - 1u;
                if ((e >> 13) == tag && seed_kmer(bw, sb + v, kmask) == code) {
                  const uint64_t p = (uint64_t)(ach + u), q = (uint64_t)(seg + v);
                  const uint64_t bin = (q + off - p) / w;
                  if (win == 0) ++my_total;
                  if (bin >= win && bin < win + kSeedBins) {
                    atomicAdd(&bcount[bin - win], 1ull);
                    atomicMin(&bkey[bin - win], (unsigned long long)((p << 32) | q));
                  }
                }
                h = (h + 1) & (kSeedTab - 1);
              }
            }
          }
        }
        __syncthreads();   // every match of this window is counted
        // the window's best bin: most matches, lowest bin
        unsigned long long c = 0;
        uint32_t b = 0xFFFFFFFFu;
        for (int i = tid; i < kSeedBins; i += kSeedThreads)
          if (seed_better(bcount[i], (uint32_t)i, c, b)) { c = bcount[i]; b = (uint32_t)i; }
        for (int d = 32; d >= 1; d >>= 1) {
          const unsigned long long c2 = __shfl_xor(c, d);
          const uint32_t b2 = __shfl_xor(b, d);
          if (seed_better(c2, b2, c, b)) { c = c2; b = b2; }
        }
        unsigned long long t = my_total;
        for (int d = 32; d >= 1; d >>= 1) t += __shfl_xor(t, d);
        if (lane == 0) {
          red_c[wave] = c;
          red_b[wave] = b;
          if (win == 0) atomicAdd(&s_total, t);
        }
        __syncthreads();
        c = red_c[0];
        b = red_b[0];
        for (int v = 1; v < kSeedThreads / 64; ++v)
          if (seed_better(red_c[v], red_b[v], c, b)) { c = red_c[v]; b = red_b[v]; }
        if (c > best_c) {   // strict: a lower window keeps a tie
          best_c = c;
          best_key = bkey[b];
        }
      }
      __syncthreads();
      res.matches = s_total;
      if (best_c > 0) {
        res.found = 1;
        res.a_seed = (uint32_t)(best_key >> 32);
        res.b_seed = (uint32_t)(best_key & 0xFFFFFFFFull);
        res.bin_matches = best_c;
      }
    }
    if (tid == 0) {
      S.out[pi] = res;
      if (S.set_pairs && res.found) {
        S.pairs[pi].a_seed = res.a_seed;
        S.pairs[pi].b_seed = res.b_seed;
        S.pairs[pi].k = (uint32_t)k;
      }
    }
  }
}

}  // namespace xd
