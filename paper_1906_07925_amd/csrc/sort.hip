// Stable LSD radix sort of 32-bit cell keys with 32-bit payloads (gfx950, wave64).
//
// One pass over a digit of up to 8 bits is three kernels:
//   radix_hist    per-tile digit histograms (LDS counters)            -> hist[tile][digit]
//   radix_scan    exclusive offsets in (digit, tile) order, in place  (one workgroup)
//   radix_scatter stable ranking inside the tile (wave ballots + per-wave counts in LDS) and
//                 scatter to hist offsets.
// The order of equal keys is the input order, so the permutation is deterministic.
#include "sort.h"

namespace mpsph {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
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

// Exclusive scan of hist[tile][digit] in digit-major order: offset(d, b) = sum of all counts of
// digits < d plus counts of digit d in tiles < b.  One workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void radix_scan(uint32_t *__restrict__ hist, int ntiles, int bits) {
  __shared__ uint32_t part[1024];
  __shared__ uint32_t dig_off[256];
  const int radix = 1 << bits;
  const int nparts = 1024 / radix;
  const int d = threadIdx.x % radix, p = threadIdx.x / radix;
  const int per = (ntiles + nparts - 1) / nparts;
  const int b0 = p * per, b1 = min(ntiles, b0 + per);
  uint32_t s = 0;
  if (p < nparts) {
    // independent loads in flight (the tile sums are order-free integers)
#pragma unroll 8
    for (int b = b0; b < b1; ++b) s += hist[(size_t)b * radix + d];
  }
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x < radix) {
    uint32_t run = 0;
    for (int q = 0; q < nparts; ++q) {
      uint32_t t = part[q * radix + threadIdx.x];
      part[q * radix + threadIdx.x] = run;
      run += t;
    }
    dig_off[threadIdx.x] = run;  // digit total for now
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    // exclusive scan of the (at most 256) digit totals by one wave: 4 per lane, then the lanes
    const int l = threadIdx.x;
    uint32_t v[4], tot = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int t = 4 * l + q;
      v[q] = t < radix ? dig_off[t] : 0u;
      tot += v[q];
    }
    uint32_t incl = tot;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t u = __shfl_up(incl, o, 64);
      if (l >= o) incl += u;
    }
    uint32_t run = incl - tot;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int t = 4 * l + q;
      if (t < radix) dig_off[t] = run;
      run += v[q];
    }
  }
  __syncthreads();
  if (p < nparts) {
    uint32_t run = dig_off[d] + part[threadIdx.x];
    // the loads do not depend on the running offset: the compiler can issue them ahead
#pragma unroll 8
    for (int b = b0; b < b1; ++b) {
      uint32_t t = hist[(size_t)b * radix + d];
      hist[(size_t)b * radix + d] = run;
      run += t;
    }
  }
}

__global__ __launch_bounds__(kSortThreads) void radix_scatter(
    const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint32_t *__restrict__ kout,
    uint32_t *__restrict__ vout, int n, int shift, int bits, const uint32_t *__restrict__ offs) {
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcnt[kSortThreads / 64][256];
  const int radix = 1 << bits;
  const uint32_t mask = (uint32_t)radix - 1u;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  for (int t = threadIdx.x; t < radix; t += kSortThreads) run[t] = offs[(size_t)blockIdx.x * radix + t];
  const int base = blockIdx.x * kSortTile;
  for (int it = 0; it < kSortItems; ++it) {
    for (int t = threadIdx.x; t < (kSortThreads / 64) * radix; t += kSortThreads) wcnt[t / radix][t % radix] = 0;
    __syncthreads();
    const int idx = base + it * kSortThreads + threadIdx.x;
    const bool valid = idx < n;
    uint32_t key = valid ? kin[idx] : 0u;
    uint32_t dig = (key >> shift) & mask;
    uint64_t same = __ballot(valid);
    for (int b = 0; b < bits; ++b) {
      bool bit = (dig >> b) & 1u;
      uint64_t bal = __ballot(bit);
      same &= bit ? bal : ~bal;
    }
    uint32_t rank = (uint32_t)__popcll(same & lt);
    if (valid && rank == 0) wcnt[w][dig] = (uint32_t)__popcll(same);
    __syncthreads();
    if (valid) {
      uint32_t pos = run[dig] + rank;
      for (int ww = 0; ww < w; ++ww) pos += wcnt[ww][dig];
      if (pos < (uint32_t)n) {
        kout[pos] = key;
        vout[pos] = vin ? vin[idx] : (uint32_t)idx;
      }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < radix; t += kSortThreads) {
      uint32_t s = 0;
      for (int ww = 0; ww < kSortThreads / 64; ++ww) s += wcnt[ww][t];
      run[t] += s;
    }
    __syncthreads();
  }
}

size_t radix_hist_words(int n) {
  int tiles = (n + kSortTile - 1) / kSortTile;
  return (size_t)(tiles > 0 ? tiles : 1) * 256;
}

int radix_passes(int key_bits) { return key_bits <= 0 ? 0 : (key_bits + 7) / 8; }

hipError_t radix_sort(const uint32_t *keys_in, uint32_t *k0, uint32_t *v0, uint32_t *k1,
                      uint32_t *v1, uint32_t *hist, int n, int key_bits, hipStream_t stream,
                      const uint32_t **keys_out, const uint32_t **perm_out, LaunchHook *hook) {
  const int passes = radix_passes(key_bits);
  const int tiles = (n + kSortTile - 1) / kSortTile;
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
    radix_scan<<<1, 1024, 0, stream>>>(hist, tiles, bits);
    if (hook) hook->end();
    if (hook) hook->begin("radix_scatter");
    radix_scatter<<<tiles, kSortThreads, 0, stream>>>(kin, vin, ko[p & 1], vo[p & 1], n, shift, bits, hist);
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
