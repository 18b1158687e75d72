// Run-compressed index-list.  In a list ordered along x rows, the upstream
// positions of consecutive cells usually rise by one: neighbouring cells of
// a row pull from neighbouring cells of the upstream row, or, along a wall,
// from their own consecutive bounce-back slots.  The list is cut into waves
// of kRunWave positions; per wave and direction a 64-bit mask marks the
// cells that start a run (lane 0 always does) and one int32 per run rebuilds
// every entry of it (value + lane).  Built from the int32 index-list in two
// passes around a prefix sum of the runs per wave.
#include "internal.hpp"

namespace lbm {

// Whether the calling lane starts a run: lane 0 always does, a lane inside
// the list does when its entry p is not its left neighbour's plus one, a
// lane past the list end never does.  Entries are unsigned positions.
__device__ __forceinline__ bool run_start(uint32_t p, uint32_t lane, bool in_list) {
  const uint32_t prev = (uint32_t)__shfl_up((int)p, 1, (int)kRunWave);
  return lane == 0 || (in_list && p != prev + 1u);
}

template <int Q>
__global__ __launch_bounds__(256) void k_runs_mask(const int32_t* __restrict__ index, uint32_t S,
                                                   uint32_t nw, uint64_t* __restrict__ mask,
                                                   uint32_t* __restrict__ cnt) {
  const uint32_t w = blockIdx.x * (256 / kRunWave) + threadIdx.x / kRunWave;
  if (w >= nw) return;  // whole waves only
  const uint32_t lane = threadIdx.x & (kRunWave - 1), k = w * kRunWave + lane;
  uint32_t total = 0;
  for (int i = 1; i < Q; ++i) {
    const uint32_t p = k < S ? (uint32_t)index[(size_t)(i - 1) * S + k] : 0u;
    const uint64_t m = __ballot(run_start(p, lane, k < S));
    if (lane == 0) mask[(size_t)w * (Q - 1) + (i - 1)] = m;
    total += (uint32_t)__popcll(m);
  }
  if (lane == 0) cnt[w] = total;
}

template <int Q>
__global__ __launch_bounds__(256) void k_runs_emit(const int32_t* __restrict__ index, uint32_t S,
                                                   uint32_t nw, const uint32_t* __restrict__ voff,
                                                   int32_t* __restrict__ val) {
  const uint32_t w = blockIdx.x * (256 / kRunWave) + threadIdx.x / kRunWave;
  if (w >= nw) return;
  const uint32_t lane = threadIdx.x & (kRunWave - 1), k = w * kRunWave + lane;
  uint32_t o = voff[w];
  for (int i = 1; i < Q; ++i) {
    const uint32_t p = k < S ? (uint32_t)index[(size_t)(i - 1) * S + k] : 0u;
    const bool st = run_start(p, lane, k < S);
    const uint64_t m = __ballot(st);
    if (st) {
      // number of run starts below this lane
      const uint32_t r = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
      val[o + r] = (int32_t)(p - lane);
    }
    o += (uint32_t)__popcll(m);
  }
}

hipError_t launch_runs_mask(int q, const int32_t* index, uint32_t S, uint32_t nw, uint64_t* mask,
                            uint32_t* cnt, hipStream_t st) {
  const dim3 g((nw + 3) / 4), b(256);
  if (q == 19)
    hipLaunchKernelGGL(k_runs_mask<19>, g, b, 0, st, index, S, nw, mask, cnt);
  else
    hipLaunchKernelGGL(k_runs_mask<27>, g, b, 0, st, index, S, nw, mask, cnt);
  return hipGetLastError();
}

hipError_t launch_runs_emit(int q, const int32_t* index, uint32_t S, uint32_t nw,
                            const uint32_t* voff, int32_t* val, hipStream_t st) {
  const dim3 g((nw + 3) / 4), b(256);
  if (q == 19)
    hipLaunchKernelGGL(k_runs_emit<19>, g, b, 0, st, index, S, nw, voff, val);
  else
    hipLaunchKernelGGL(k_runs_emit<27>, g, b, 0, st, index, S, nw, voff, val);
  return hipGetLastError();
}

}  // namespace lbm
