// Stable LSD radix sort of (uint32 key, uint32 value) pairs with 8-bit
// digits, and a one-block exclusive scan, shared by the training pass and
// the device octree build.  Each sort pass: per-block digit histograms
// ([256][grid]), one exclusive scan of them, then a stable scatter (ranks
// within a wavefront from ballots, across wavefronts from LDS counts).
#pragma once

#include "ngl_device.h"

namespace ngl {

__device__ inline void sort_chunk(int64_t n, int64_t& begin, int64_t& end) {
  int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  chunk = (chunk + kBlock - 1) / kBlock * kBlock;
  begin = int64_t(blockIdx.x) * chunk;
  end = begin + chunk < n ? begin + chunk : n;
}

static __global__ __launch_bounds__(kBlock) void k_radix_hist(const uint32_t* __restrict__ key, int64_t n, int shift,
                                                       uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  int64_t begin, end;
  sort_chunk(n, begin, end);
  for (int64_t t = begin + threadIdx.x; t < end; t += kBlock) atomicAdd(&h[(key[t] >> shift) & 255u], 1u);
  __syncthreads();
  hist[threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of n uint32 values in place by one block of 1024 lanes
// (a must be 16-byte aligned); *total (nullable) receives the sum.  Each
// lane owns 32 consecutive values of a tile of 32 Ki values and loads them
// as eight 16-byte vectors, so a tile's loads are all in flight together
// (the radix-sort histograms, 256 x grid values, take a few tiles).
static __global__ __launch_bounds__(1024) void k_scan_inplace(uint32_t* __restrict__ a, int64_t n, uint32_t* total) {
  constexpr int ITEMS = 32;
  __shared__ uint32_t part[16];
  __shared__ uint32_t carry_s;
  if (threadIdx.x == 0) carry_s = 0;
  __syncthreads();
  for (int64_t base = 0; base < n; base += 1024 * ITEMS) {
    uint32_t v[ITEMS];
    const int64_t b0 = base + int64_t(threadIdx.x) * ITEMS;
    if (b0 + ITEMS <= n) {
      const uint4* src = reinterpret_cast<const uint4*>(a + b0);
#pragma unroll
      for (int q = 0; q < ITEMS / 4; ++q) {
        const uint4 u = src[q];
        v[4 * q] = u.x;
        v[4 * q + 1] = u.y;
        v[4 * q + 2] = u.z;
        v[4 * q + 3] = u.w;
      }
    } else {
#pragma unroll
      for (int q = 0; q < ITEMS; ++q) v[q] = b0 + q < n ? a[b0 + q] : 0u;
    }
    uint32_t local = 0;
#pragma unroll
    for (int q = 0; q < ITEMS; ++q) local += v[q];
    uint32_t x = local;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) part[threadIdx.x >> 6] = x;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < 16; ++w) {
      const uint32_t s = part[w];
      if (w < int(threadIdx.x >> 6)) pre += s;
      tot += s;
    }
    uint32_t run = carry_s + pre + x - local;
    if (b0 + ITEMS <= n) {
      uint4* dst = reinterpret_cast<uint4*>(a + b0);
#pragma unroll
      for (int q = 0; q < ITEMS / 4; ++q) {
        uint4 u;
        u.x = run;
        run += v[4 * q];
        u.y = run;
        run += v[4 * q + 1];
        u.z = run;
        run += v[4 * q + 2];
        u.w = run;
        run += v[4 * q + 3];
        dst[q] = u;
      }
    } else {
#pragma unroll
      for (int q = 0; q < ITEMS; ++q) {
        if (b0 + q < n) a[b0 + q] = run;
        run += v[q];
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) carry_s += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0 && total) *total = carry_s;
}

static __global__ __launch_bounds__(kBlock) void k_radix_scatter(const uint32_t* __restrict__ kin,
                                                          const uint32_t* __restrict__ vin,
                                                          uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                          int64_t n, int shift, const uint32_t* __restrict__ offs) {
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcnt[kBlock / 64][256];
  run[threadIdx.x] = offs[threadIdx.x * gridDim.x + blockIdx.x];
  int64_t begin, end;
  sort_chunk(n, begin, end);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int64_t base = begin; base < end; base += kBlock) {
#pragma unroll
    for (int q = 0; q < kBlock / 64; ++q) wcnt[q][threadIdx.x] = 0;
    __syncthreads();
    const int64_t t = base + threadIdx.x;
    const bool valid = t < end;
    const uint32_t k = valid ? kin[t] : 0u;
    const uint32_t dig = (k >> shift) & 255u;
    // lanes of this wavefront holding the same digit (stable rank by lane)
    uint64_t eq = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (dig >> b) & 1u;
      const uint64_t m = __ballot(bit);
      eq &= bit ? m : ~m;
    }
    const uint32_t rank = uint32_t(__popcll(eq & ((1ull << lane) - 1ull)));
    if (valid && rank == 0) wcnt[w][dig] = uint32_t(__popcll(eq));
    __syncthreads();
    if (valid) {
      uint32_t pos = run[dig] + rank;
      for (int q = 0; q < w; ++q) pos += wcnt[q][dig];
      kout[pos] = k;
      vout[pos] = vin[t];
    }
    __syncthreads();
    uint32_t add = 0;
#pragma unroll
    for (int q = 0; q < kBlock / 64; ++q) add += wcnt[q][threadIdx.x];
    run[threadIdx.x] += add;
    __syncthreads();
  }
}

// Sorts n pairs on `bits` low key bits (ceil(bits / 8) passes) between the
// two buffers; returns the index (0 or 1) of the buffer holding the result.
// hist: 256 * grid words.
inline int radix_sort_pairs(uint32_t* key[2], uint32_t* val[2], int64_t n, int bits, int grid, uint32_t* hist,
                            hipStream_t s) {
  int cur = 0;
  for (int shift = 0; shift < bits; shift += 8) {
    k_radix_hist<<<grid, kBlock, 0, s>>>(key[cur], n, shift, hist);
    k_scan_inplace<<<1, 1024, 0, s>>>(hist, int64_t(256) * grid, nullptr);
    k_radix_scatter<<<grid, kBlock, 0, s>>>(key[cur], val[cur], key[cur ^ 1], val[cur ^ 1], n, shift, hist);
    cur ^= 1;
  }
  return cur;
}

}  // namespace ngl
