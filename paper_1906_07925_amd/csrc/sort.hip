// Stable LSD radix sort of 32-bit cell keys with 32-bit payloads (gfx950, wave64).
//
// One pass over a digit of up to 8 bits is three kernels:
//   radix_hist    per-tile digit histograms (LDS counters)            -> hist[tile][digit]
//   radix_scan    per digit (one workgroup each): exclusive offsets over the tiles, in place,
//                 and the digit's total                               -> dsum[digit]
//   radix_scatter digit bases from the totals; every key of the tile ranked among the keys of its
//                 wave and item with the same digit (wave ballots), the (item, wave) counts turned
//                 into tile offsets per digit in LDS, the tile staged in LDS in sorted order and
//                 written out run by run (base + position in the digit's run).
// The order of equal keys is the input order, so the permutation is deterministic.
#include "sort.h"

#include <algorithm>

namespace mpsph {

constexpr int kSortThreads = 256;
// Keys per thread of a tile (measured on 2M keys: 16 beats 8 and 4, whose extra tiles cost the
// scan and the scatter more than their shorter ranking loops save).
#ifndef MPSPH_SORT_ITEMS
#define MPSPH_SORT_ITEMS 16
#endif
constexpr int kSortItems = MPSPH_SORT_ITEMS;
constexpr int kSortTile = kSortThreads * kSortItems;

__global__ __launch_bounds__(kSortThreads) void radix_hist(const uint32_t *__restrict__ keys, int n,
                                                           int shift, int bits,
                                                           uint32_t *__restrict__ hist) {
  __shared__ uint32_t cnt[256];
  const int radix = 1 << bits;
  const uint32_t mask = (uint32_t)radix - 1u;
  for (int t = threadIdx.x; t < radix; t += kSortThreads) cnt[t] = 0;
  __syncthreads();
  const int base = blockIdx.x * kSortTile;
#pragma unroll 4
  for (int it = 0; it < kSortItems; ++it) {
    int idx = base + it * kSortThreads + threadIdx.x;
    if (idx < n) atomicAdd(&cnt[(keys[idx] >> shift) & mask], 1u);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < radix; t += kSortThreads) hist[(size_t)blockIdx.x * radix + t] = cnt[t];
}

// Exclusive scan over the tiles of one digit's column of hist (one workgroup per digit), in
// place, and the digit's total into dsum[digit].  Thread t takes a contiguous run of tiles.
__global__ __launch_bounds__(kSortThreads) void radix_scan(uint32_t *__restrict__ hist, int ntiles, int bits,
                                                         uint32_t *__restrict__ dsum) {
  __shared__ uint32_t wsum[kSortThreads / 64];
  const int radix = 1 << bits;
  const int d = blockIdx.x;
  const int per = (ntiles + kSortThreads - 1) / kSortThreads;
  const int b0 = min(ntiles, (int)threadIdx.x * per), b1 = min(ntiles, b0 + per);
  uint32_t s = 0;
  for (int b = b0; b < b1; ++b) s += hist[(size_t)b * radix + d];
  // exclusive prefix of the thread sums: within the wave, then over the waves
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t incl = s;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t u = __shfl_up(incl, o, 64);
    if (lane >= o) incl += u;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  uint32_t run = incl - s;
  for (int ww = 0; ww < w; ++ww) run += wsum[ww];
  for (int b = b0; b < b1; ++b) {
    const uint32_t t = hist[(size_t)b * radix + d];
    hist[(size_t)b * radix + d] = run;
    run += t;
  }
  if (threadIdx.x == kSortThreads - 1) dsum[d] = run;
}

__global__ __launch_bounds__(kSortThreads) void radix_scatter(
    const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint32_t *__restrict__ kout,
    uint32_t *__restrict__ vout, int n, int shift, int bits, const uint32_t *__restrict__ offs,
    const uint32_t *__restrict__ dsum) {
  constexpr int kW = kSortThreads / 64;
  __shared__ uint32_t run[256];
  __shared__ uint32_t tstart[256];
  // per (item, wave) row and digit: the count of the wave's keys with that digit in that item,
  // then their offset in the tile (below 2^16: a tile holds kSortTile keys); afterwards the
  // staging area of the tile's keys and values (2 x kSortTile words, the same 32 KB)
  __shared__ uint16_t cnt[kSortItems * kW][256];
  static_assert(sizeof(cnt) >= 2 * kSortTile * sizeof(uint32_t), "staging area");
  const int radix = 1 << bits;
  const uint32_t mask = (uint32_t)radix - 1u;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  if (threadIdx.x < 64) {
    // digit bases: exclusive prefix of the (at most 256) digit totals, 4 per lane
    uint32_t v[4], tot = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int t = 4 * lane + q;
      v[q] = t < radix ? dsum[t] : 0u;
      tot += v[q];
    }
    uint32_t incl = tot;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t u = __shfl_up(incl, o, 64);
      if (lane >= o) incl += u;
    }
    uint32_t b = incl - tot;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int t = 4 * lane + q;
      if (t < radix) run[t] = b + offs[(size_t)blockIdx.x * radix + t];
      b += v[q];
    }
  }
  uint32_t *cnt32 = reinterpret_cast<uint32_t *>(&cnt[0][0]);
  for (int t = threadIdx.x; t < kSortItems * kW * 128; t += kSortThreads) cnt32[t] = 0u;
  const int base = blockIdx.x * kSortTile;
  uint32_t key[kSortItems], val[kSortItems], rank[kSortItems];
#pragma unroll
  for (int it = 0; it < kSortItems; ++it) {
    const int idx = base + it * kSortThreads + threadIdx.x;
    const bool valid = idx < n;
    key[it] = valid ? kin[idx] : 0u;
    val[it] = valid ? (vin ? vin[idx] : (uint32_t)idx) : 0u;
  }
  __syncthreads();
  // rank every key among the keys of its wave and item with the same digit
#pragma unroll
  for (int it = 0; it < kSortItems; ++it) {
    const bool valid = base + it * kSortThreads + (int)threadIdx.x < n;
    const uint32_t dig = (key[it] >> shift) & mask;
    uint64_t same = __ballot(valid);
    for (int b = 0; b < bits; ++b) {
      const bool bit = (dig >> b) & 1u;
      const uint64_t bal = __ballot(bit);
      same &= bit ? bal : ~bal;
    }
    rank[it] = (uint32_t)__popcll(same & lt);
    if (valid && rank[it] == 0u) cnt[it * kW + w][dig] = (uint16_t)__popcll(same);
  }
  __syncthreads();
  // per digit, offsets of the (item, wave) groups in input order, and the digit's count in the tile
  for (int d = threadIdx.x; d < radix; d += kSortThreads) {
    uint32_t s = 0;
    for (int q = 0; q < kSortItems * kW; ++q) {
      const uint32_t c = cnt[q][d];
      cnt[q][d] = (uint16_t)s;
      s += c;
    }
    tstart[d] = s;
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    // where each digit's keys start in the tile's sorted order: exclusive prefix of the counts
    uint32_t v[4], tot = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int t = 4 * lane + q;
      v[q] = t < radix ? tstart[t] : 0u;
      tot += v[q];
    }
    uint32_t incl = tot;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t u = __shfl_up(incl, o, 64);
      if (lane >= o) incl += u;
    }
    uint32_t b = incl - tot;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int t = 4 * lane + q;
      if (t < radix) tstart[t] = b;
      b += v[q];
    }
  }
  __syncthreads();
  // each key's place in the tile's sorted order (the counts are read for the last time here)
#pragma unroll
  for (int it = 0; it < kSortItems; ++it) {
    const uint32_t dig = (key[it] >> shift) & mask;
    rank[it] += tstart[dig] + cnt[it * kW + w][dig];
  }
  __syncthreads();
  // stage the tile in sorted order in the counts' memory, then write it out in that order, so
  // that consecutive threads store consecutive positions of a digit's run
  uint32_t *sk = cnt32, *sv = cnt32 + kSortTile;
#pragma unroll
  for (int it = 0; it < kSortItems; ++it) {
    if (base + it * kSortThreads + (int)threadIdx.x < n) {
      sk[rank[it]] = key[it];
      sv[rank[it]] = val[it];
    }
  }
  __syncthreads();
  const int tile_n = min(kSortTile, n - base);
  for (int l = threadIdx.x; l < tile_n; l += kSortThreads) {
    const uint32_t k = sk[l];
    const uint32_t dig = (k >> shift) & mask;
    const uint32_t pos = run[dig] + ((uint32_t)l - tstart[dig]);
    if (pos < (uint32_t)n) {
      kout[pos] = k;
      vout[pos] = sv[l];
    }
  }
}

size_t radix_hist_words(int n) {
  int tiles = (n + kSortTile - 1) / kSortTile;
  return (size_t)(tiles > 0 ? tiles : 1) * 256 + 256;   // tile histograms, then the digit totals
}

int radix_passes(int key_bits) { return key_bits <= 0 ? 0 : (key_bits + 7) / 8; }

hipError_t radix_sort(const uint32_t *keys_in, uint32_t *k0, uint32_t *v0, uint32_t *k1,
                      uint32_t *v1, uint32_t *hist, int n, int key_bits, hipStream_t stream,
                      const uint32_t **keys_out, const uint32_t **perm_out, LaunchHook *hook) {
  const int passes = radix_passes(key_bits);
  const int tiles = (n + kSortTile - 1) / kSortTile;
  uint32_t *dsum = hist + (size_t)std::max(tiles, 1) * 256;
  const uint32_t *kin = keys_in, *vin = nullptr;
  uint32_t *ko[2] = {k0, k1}, *vo[2] = {v0, v1};
  int shift = 0;
  for (int p = 0; p < passes; ++p) {
    int bits = (key_bits - shift + (passes - p) - 1) / (passes - p);
    if (bits > 8) bits = 8;
    if (hook) hook->begin("radix_hist");
    radix_hist<<<tiles, kSortThreads, 0, stream>>>(kin, n, shift, bits, hist);
    if (hook) hook->end();
    if (hook) hook->begin("radix_scan");
    radix_scan<<<1 << bits, kSortThreads, 0, stream>>>(hist, tiles, bits, dsum);
    if (hook) hook->end();
    if (hook) hook->begin("radix_scatter");
    radix_scatter<<<tiles, kSortThreads, 0, stream>>>(kin, vin, ko[p & 1], vo[p & 1], n, shift, bits, hist, dsum);
    if (hook) hook->end();
    kin = ko[p & 1];
    vin = vo[p & 1];
    shift += bits;
  }
  *keys_out = kin;
  *perm_out = vin;
  return hipGetLastError();
}

}  // namespace mpsph
