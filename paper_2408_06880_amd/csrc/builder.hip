// Geometry -> sparse lists on the GPU (Section "Sparse Data Structure",
// "Sparse Boundary Conditions").
//
// The box is visited in list order by scanning a code space: Morton codes
// (bit b of x, y, z at bits 3b, 3b+1, 3b+2; codes outside the box skipped)
// or linear ids.  A three-kernel scan (per-chunk counts, one-workgroup
// exclusive scan, emit) gives each fluid cell its list position k without a
// sort; an inverse map lin -> k then lets one thread per fluid cell write
// its Q-1 pull indices, coalesced per direction.
#include "internal.hpp"

namespace lbm {

__device__ __forceinline__ uint32_t compact3(uint32_t v) {
  // keep bits 0, 3, 6, ... of v and pack them (10 bits max)
  v &= 0x09249249u;
  v = (v ^ (v >> 2)) & 0x030c30c3u;
  v = (v ^ (v >> 4)) & 0x0300f00fu;
  v = (v ^ (v >> 8)) & 0xff0000ffu;
  v = (v ^ (v >> 16)) & 0x000003ffu;
  return v;
}

__device__ __forceinline__ uint32_t compact2(uint32_t v) {
  // keep bits 0, 2, 4, ... of v and pack them (16 bits max)
  v &= 0x55555555u;
  v = (v | (v >> 1)) & 0x33333333u;
  v = (v | (v >> 2)) & 0x0f0f0f0fu;
  v = (v | (v >> 4)) & 0x00ff00ffu;
  v = (v | (v >> 8)) & 0x0000ffffu;
  return v;
}

// Decode a code into (x, y, z); false if it lies outside the box.
__device__ __forceinline__ bool decode(const BuildArgs& b, uint64_t code, int& x, int& y,
                                       int& z) {
  if (b.order == 2) {
    // blocks of nx * 8 * 8 cells in 2-D Morton order of (y/8, z/8)
    const uint64_t blk = (uint64_t)b.nx * (kBlockYZ * kBlockYZ);
    const uint32_t t = (uint32_t)(code / blk);
    const uint32_t local = (uint32_t)(code - (uint64_t)t * blk);
    x = (int)(local % (uint32_t)b.nx);
    const uint32_t r = local / (uint32_t)b.nx;
    y = (int)(compact2(t) * kBlockYZ + r % kBlockYZ);
    z = (int)(compact2(t >> 1) * kBlockYZ + r / kBlockYZ);
    return y < b.ny && z < b.nz;
  }
  if (b.order == 0) {
    const uint32_t c = (uint32_t)code;
    x = (int)compact3(c);
    y = (int)compact3(c >> 1);
    z = (int)compact3(c >> 2);
    return x < b.nx && y < b.ny && z < b.nz;
  }
  const uint64_t nxy = (uint64_t)b.nx * b.ny;
  z = (int)(code / nxy);
  const uint64_t r = code - (uint64_t)z * nxy;
  y = (int)(r / b.nx);
  x = (int)(r - (uint64_t)y * b.nx);
  return code < nxy * b.nz;
}

// Upstream cell x - c of (x, y, z); -1 when it leaves the box through a
// non-periodic face (a halfway no-slip wall).
__device__ __forceinline__ int64_t upstream(const BuildArgs& b, int x, int y, int z, int cx,
                                            int cy, int cz) {
  int p0 = x - cx, p1 = y - cy, p2 = z - cz;
  if (p0 < 0 || p0 >= b.nx) {
    if (!(b.periodic & 1u)) return -1;
    p0 = p0 < 0 ? p0 + b.nx : p0 - b.nx;
  }
  if (p1 < 0 || p1 >= b.ny) {
    if (!(b.periodic & 2u)) return -1;
    p1 = p1 < 0 ? p1 + b.ny : p1 - b.ny;
  }
  if (p2 < 0 || p2 >= b.nz) {
    if (!(b.periodic & 4u)) return -1;
    p2 = p2 < 0 ? p2 + b.nz : p2 - b.nz;
  }
  return (int64_t)p0 + (int64_t)b.nx * ((int64_t)p1 + (int64_t)b.ny * p2);
}

template <int Q>
__device__ __forceinline__ uint32_t count_links(const BuildArgs& b, int x, int y, int z) {
  using L = Lattice<Q>;
  uint32_t n = 0;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const int64_t yl = upstream(b, x, y, z, L::cx[i], L::cy[i], L::cz[i]);
    if (yl >= 0 && b.labels[yl] >= 2) ++n;
  }
  return n;
}

__device__ __forceinline__ int64_t lin_of(const BuildArgs& b, int x, int y, int z) {
  return (int64_t)x + (int64_t)b.nx * ((int64_t)y + (int64_t)b.ny * z);
}

// Exclusive scan of one value per thread within a workgroup of kBuildBlock.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* sh,
                                                         uint32_t& total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < kBuildBlock; off <<= 1) {
    const uint32_t add = t >= off ? sh[t - off] : 0u;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  total = sh[kBuildBlock - 1];
  const uint32_t incl = sh[t];
  __syncthreads();
  return incl - v;
}

template <int Q>
__global__ __launch_bounds__(kBuildBlock) void k_build_count(const BuildArgs b,
                                                             uint32_t* counts) {
  __shared__ uint32_t sh[kBuildBlock];
  const uint64_t c0 = (uint64_t)blockIdx.x * kChunk + (uint64_t)threadIdx.x * kCodesPerThread;
  uint32_t nf = 0, nl = 0;
  for (int j = 0; j < kCodesPerThread; ++j) {
    const uint64_t code = c0 + j;
    if (code >= b.n_codes) break;
    int x, y, z;
    if (!decode(b, code, x, y, z)) continue;
    if (b.labels[lin_of(b, x, y, z)] != 0) continue;
    ++nf;
    nl += count_links<Q>(b, x, y, z);
  }
  uint32_t tf, tl;
  block_exclusive_scan(nf, sh, tf);
  block_exclusive_scan(nl, sh, tl);
  if (threadIdx.x == 0) {
    counts[blockIdx.x] = tf;
    counts[b.n_chunks + 1 + blockIdx.x] = tl;
  }
}

// One workgroup: exclusive scan of narr consecutive count arrays of n + 1
// words each, in place (totals at [n]).
__global__ __launch_bounds__(1024) void k_build_scan(uint32_t n, uint32_t* counts, int narr) {
  __shared__ uint64_t sh[1024];
  for (int arr = 0; arr < narr; ++arr) {
    uint32_t* a = counts + (size_t)arr * (n + 1);
    const uint32_t per = (n + 1023) / 1024;
    const uint32_t lo = threadIdx.x * per;
    const uint32_t hi = lo + per < n ? lo + per : n;
    uint64_t s = 0;
    for (uint32_t i = lo; i < hi; ++i) s += a[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint64_t run = 0;
      for (int t = 0; t < 1024; ++t) {
        const uint64_t v = sh[t];
        sh[t] = run;
        run += v;
      }
      a[n] = (uint32_t)run;
    }
    __syncthreads();
    uint64_t run = sh[threadIdx.x];
    for (uint32_t i = lo; i < hi; ++i) {
      const uint32_t v = a[i];
      a[i] = (uint32_t)run;
      run += v;
    }
    __syncthreads();
  }
}

template <int Q>
__global__ __launch_bounds__(kBuildBlock) void k_build_emit(const BuildArgs b,
                                                            const uint32_t* counts, uint32_t S,
                                                            uint32_t n_fluid, uint32_t n_links,
                                                            int32_t* cells, int32_t* inv,
                                                            int32_t* links) {
  using L = Lattice<Q>;
  __shared__ uint32_t sh[kBuildBlock];
  const uint64_t c0 = (uint64_t)blockIdx.x * kChunk + (uint64_t)threadIdx.x * kCodesPerThread;
  uint32_t nf = 0, nl = 0;
  for (int j = 0; j < kCodesPerThread; ++j) {
    const uint64_t code = c0 + j;
    if (code >= b.n_codes) break;
    int x, y, z;
    if (!decode(b, code, x, y, z)) continue;
    if (b.labels[lin_of(b, x, y, z)] != 0) continue;
    ++nf;
    nl += count_links<Q>(b, x, y, z);
  }
  uint32_t tf, tl;
  uint32_t kf = counts[blockIdx.x] + block_exclusive_scan(nf, sh, tf);
  uint32_t kl = counts[b.n_chunks + 1 + blockIdx.x] + block_exclusive_scan(nl, sh, tl);
  for (int j = 0; j < kCodesPerThread; ++j) {
    const uint64_t code = c0 + j;
    if (code >= b.n_codes) break;
    int x, y, z;
    if (!decode(b, code, x, y, z)) continue;
    const int64_t lin = lin_of(b, x, y, z);
    if (b.labels[lin] != 0) continue;
    const uint32_t k = kf++;
    if (k >= n_fluid) continue;
    cells[k] = (int32_t)lin;
    inv[lin] = (int32_t)k;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const int64_t yl = upstream(b, x, y, z, L::cx[i], L::cy[i], L::cz[i]);
      if (yl < 0) continue;
      const int lab = b.labels[yl];
      if (lab < 2) continue;
      const uint32_t l = kl++;
      if (l >= n_links) continue;
      links[2 * (size_t)l] = (int32_t)((uint32_t)opp(i) * S + k);
      links[2 * (size_t)l + 1] = i | ((lab - 2) << 8);
    }
  }
}

template <int Q>
__global__ __launch_bounds__(256) void k_build_index(const BuildArgs b, const int32_t* cells,
                                                     const int32_t* inv, uint32_t S,
                                                     uint32_t n_fluid, int32_t* index) {
  using L = Lattice<Q>;
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= S) return;
  if (k >= n_fluid) {
#pragma unroll
    for (int i = 1; i < Q; ++i) index[(size_t)(i - 1) * S + k] = (int32_t)((uint32_t)opp(i) * S + k);
    return;
  }
  const int64_t lin = cells[k];
  const int64_t nxy = (int64_t)b.nx * b.ny;
  const int z = (int)(lin / nxy);
  const int64_t r = lin - (int64_t)z * nxy;
  const int y = (int)(r / b.nx);
  const int x = (int)(r - (int64_t)y * b.nx);
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const int64_t yl = upstream(b, x, y, z, L::cx[i], L::cy[i], L::cz[i]);
    uint32_t pos;
    if (yl >= 0 && b.labels[yl] == 0)
      pos = (uint32_t)i * S + (uint32_t)inv[yl];
    else
      pos = (uint32_t)opp(i) * S + k;
    index[(size_t)(i - 1) * S + k] = (int32_t)pos;
  }
}

hipError_t launch_build_count(const BuildArgs& b, uint32_t* counts, hipStream_t st) {
  dim3 g(b.n_chunks), blk(kBuildBlock);
  if (b.q == 19)
    hipLaunchKernelGGL(k_build_count<19>, g, blk, 0, st, b, counts);
  else
    hipLaunchKernelGGL(k_build_count<27>, g, blk, 0, st, b, counts);
  return hipGetLastError();
}

hipError_t launch_build_scan(uint32_t n_chunks, uint32_t* counts, hipStream_t st) {
  hipLaunchKernelGGL(k_build_scan, dim3(1), dim3(1024), 0, st, n_chunks, counts, 2);
  return hipGetLastError();
}

hipError_t launch_exclusive_scan(uint32_t n, uint32_t* v, hipStream_t st) {
  hipLaunchKernelGGL(k_build_scan, dim3(1), dim3(1024), 0, st, n, v, 1);
  return hipGetLastError();
}

hipError_t launch_build_emit(const BuildArgs& b, const uint32_t* counts, uint32_t S,
                             uint32_t n_fluid, uint32_t n_links, int32_t* cells, int32_t* inv,
                             int32_t* links, hipStream_t st) {
  dim3 g(b.n_chunks), blk(kBuildBlock);
  if (b.q == 19)
    hipLaunchKernelGGL(k_build_emit<19>, g, blk, 0, st, b, counts, S, n_fluid, n_links, cells,
                       inv, links);
  else
    hipLaunchKernelGGL(k_build_emit<27>, g, blk, 0, st, b, counts, S, n_fluid, n_links, cells,
                       inv, links);
  return hipGetLastError();
}

hipError_t launch_build_index(const BuildArgs& b, const int32_t* cells, const int32_t* inv,
                              uint32_t S, uint32_t n_fluid, int32_t* index, hipStream_t st) {
  if (S == 0) return hipSuccess;
  dim3 g((S + 255) / 256), blk(256);
  if (b.q == 19)
    hipLaunchKernelGGL(k_build_index<19>, g, blk, 0, st, b, cells, inv, S, n_fluid, index);
  else
    hipLaunchKernelGGL(k_build_index<27>, g, blk, 0, st, b, cells, inv, S, n_fluid, index);
  return hipGetLastError();
}

}  // namespace lbm
