// Compact index-list: per tile of kTile16 list positions and per direction
// an int32 base and per entry a uint16 offset o, so that the upstream list
// position is m = k + base + o.  kBounce16 marks a non-fluid upstream cell,
// kEscape16 an entry outside the tile's 16-bit window (its position is read
// from the int32 index-list).  The base is the smallest offset m - k of the
// tile when all offsets fit one window, else the start of the window that
// holds more of them.  Built once from the int32 index-list; the odd step
// then reads 2 instead of 4 bytes per index.
#include <limits.h>

#include "internal.hpp"

namespace lbm {

__device__ __forceinline__ int32_t wave_min(int32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const int32_t o = __shfl_xor(v, off, 64);
    v = o < v ? o : v;
  }
  return v;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ int32_t wave_max(int32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const int32_t o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  return v;
}

template <int Q>
__global__ __launch_bounds__(kTile16) void k_compress_index(const int32_t* __restrict__ index,
                                                             uint32_t S, uint32_t nf,
                                                             uint32_t ntiles, uint16_t* off,
                                                             int32_t* base, uint32_t* flags) {
  __shared__ int32_t smin[kTile16 / 64], smax[kTile16 / 64];
  __shared__ uint32_t scnt[kTile16 / 64];
  const uint32_t t = blockIdx.x;
  const uint32_t k = t * kTile16 + threadIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t escaped = 0;
  for (int i = 1; i < Q; ++i) {
    int32_t d = 0;
    bool fluid = false;
    if (k < nf) {
      const uint32_t p = (uint32_t)index[(size_t)(i - 1) * S + k];
      fluid = p >= (uint32_t)i * S && p < (uint32_t)(i + 1) * S;
      d = (int32_t)(p - (uint32_t)i * S) - (int32_t)k;
    }
    const int32_t mn = wave_min(fluid ? d : INT_MAX);
    const int32_t mx = wave_max(fluid ? d : INT_MIN);
    if (lane == 0) {
      smin[wv] = mn;
      smax[wv] = mx;
    }
    __syncthreads();
    int32_t bmin = INT_MAX, bmax = INT_MIN;
#pragma unroll
    for (int w = 0; w < kTile16 / 64; ++w) {
      bmin = smin[w] < bmin ? smin[w] : bmin;
      bmax = smax[w] > bmax ? smax[w] : bmax;
    }
    __syncthreads();
    int32_t b = bmin == INT_MAX ? 0 : bmin;
    if (bmax != INT_MIN && (int64_t)bmax - (int64_t)bmin > (int64_t)kMaxOff16) {
      // Two clusters: encode whichever window [bmin, bmin + max] or
      // [bmax - max, bmax] holds more entries; the rest escape.
      const int32_t b2 = bmax - (int32_t)kMaxOff16;
      const bool in1 = fluid && (int64_t)d - bmin <= (int64_t)kMaxOff16;
      const bool in2 = fluid && d >= b2;
      const uint32_t c1 = __popcll(__ballot(in1)), c2 = __popcll(__ballot(in2));
      if (lane == 0) scnt[wv] = c1 | (c2 << 16);
      __syncthreads();
      uint32_t t1 = 0, t2 = 0;
#pragma unroll
      for (int w = 0; w < kTile16 / 64; ++w) {
        t1 += scnt[w] & 0xffffu;
        t2 += scnt[w] >> 16;
      }
      __syncthreads();
      b = t1 >= t2 ? bmin : b2;
    }
    if (threadIdx.x == 0) base[(size_t)t * (Q - 1) + (i - 1)] = b;
    if (k < S) {
      uint16_t o = kBounce16;
      if (fluid) {
        const int64_t rel = (int64_t)d - b;
        if (rel >= 0 && rel <= (int64_t)kMaxOff16) {
          o = (uint16_t)rel;
        } else {
          o = kEscape16;
          ++escaped;
        }
      }
      off[(size_t)(i - 1) * S + k] = o;
    }
  }
  // escaped entries of the tile
  const uint32_t we = wave_sum_u32(escaped);
  if (lane == 0) scnt[wv] = we;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t tot = 0;
    for (int w = 0; w < kTile16 / 64; ++w) tot += scnt[w];
    flags[t] = tot;
  }
}

// One workgroup sums the per-tile escape counts into flags[ntiles] (fixed
// order, no atomics).
__global__ __launch_bounds__(256) void k_sum_flags(uint32_t* flags, uint32_t ntiles) {
  __shared__ uint32_t sh[256];
  uint32_t v = 0;
  for (uint32_t t = threadIdx.x; t < ntiles; t += 256) v += flags[t];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) flags[ntiles] = sh[0];
}

hipError_t launch_compress_index(int q, const int32_t* index, uint32_t S, uint32_t nf,
                                 uint32_t ntiles, uint16_t* off, int32_t* base, uint32_t* flags,
                                 hipStream_t st) {
  if (ntiles > 0) {
    if (q == 19)
      hipLaunchKernelGGL(k_compress_index<19>, dim3(ntiles), dim3(kTile16), 0, st, index, S, nf,
                         ntiles, off, base, flags);
    else
      hipLaunchKernelGGL(k_compress_index<27>, dim3(ntiles), dim3(kTile16), 0, st, index, S, nf,
                         ntiles, off, base, flags);
  }
  hipLaunchKernelGGL(k_sum_flags, dim3(1), dim3(256), 0, st, flags, ntiles);
  return hipGetLastError();
}

}  // namespace lbm
