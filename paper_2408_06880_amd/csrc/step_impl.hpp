// Fused AA stream-collide kernels over the compacted fluid list
// (Section "In-place Streaming: AA Pattern").
//
// odd step  (t even): for cell k, population i >= 1 is gathered from
//   pos_i = index[(i-1)*S + k] (the upstream cell's slot, or the cell's own
//   opposite slot where the upstream cell is not fluid); after the
//   collision the opposite result f*_opp(i) is written back to pos_i, so
//   every slot is read and written by exactly one thread (the index-list
//   is a permutation of the slots) and one array suffices.
// even step (t odd): population i is read from the cell's own slot
//   opp(i)*S + k and f*_i is written to i*S + k -- purely local, no index
//   reads, fully coalesced.
//
// pull step (two arrays, Section "In-place Streaming: AA Pattern", the pull
//   pattern the paper compares against): gather exactly as the odd step,
//   collide, write f*_i to i*S + k of the second array; every step reads
//   the index-list.
//
// One thread updates one fluid cell; a workgroup covers BLOCK consecutive
// cells of one segment (solve).  Consecutive list positions are neighbours
// along the list order (blocked, lexicographic or Morton), so the gathers of
// a wavefront stay within a few cache lines per direction.
#pragma once

#include "cumulant.hpp"
#include "mrt.hpp"

#include <atomic>

namespace lbm {

template <int Q, int COLL, class R>
__device__ __forceinline__ void collide(R (&d)[Q], const CollParams<R>& p) {
  if constexpr (COLL == COLL_SRT) {
    collide_srt<Q, R>(d, p);
  } else if constexpr (COLL == COLL_TRT) {
    collide_trt<Q, R>(d, p);
  } else if constexpr (COLL == COLL_CUMULANT) {
    static_assert(Q == 27, "cumulant needs D3Q27");
    collide_cumulant<R>(d, p);
  } else if constexpr (COLL == COLL_CM) {
    static_assert(Q == 27, "central moments need D3Q27");
    collide_cm<R>(d, p);
  } else if constexpr (COLL == COLL_MRT) {
    static_assert(Q == 19, "MRT is defined for D3Q19");
    collide_mrt<R>(d, p);
  }
}

template <class R>
__device__ __forceinline__ CollParams<R> seg_params(const Seg& g) {
  CollParams<R> p;
  p.om1 = R(g.om1);
  p.om2 = R(g.om2);
  p.Fx = R(g.F[0]);
  p.Fy = R(g.F[1]);
  p.Fz = R(g.F[2]);
  for (int a = 0; a < 4; ++a) p.r[a] = R(g.rates[a]);
  return p;
}

#ifndef LBM_STEP_WAVES_PER_EU
#define LBM_STEP_WAVES_PER_EU 1
#endif
// Cache hints of the gather step (compile-time; measured defaults).  The
// index hint covers the int32 and 16-bit forms; run values stay cached
// (lanes of a run and neighbouring directions share their lines).
#ifndef LBM_NT_INDEX
#define LBM_NT_INDEX 1
#endif
#ifndef LBM_NT_GATHER
#define LBM_NT_GATHER 0
#endif
#ifndef LBM_NT_SCATTER
#define LBM_NT_SCATTER 0
#endif

template <bool NT, class T>
__device__ __forceinline__ T ld(const LBM_GLOBAL T* p) {
  if constexpr (NT)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}

template <bool NT, class T>
__device__ __forceinline__ void st(T v, LBM_GLOBAL T* p) {
  if constexpr (NT)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

// Run form: the wave's run-start masks and first value index are
// wave-uniform (scalar loads).  The entry of lane l is the value of the run
// holding l plus l; the run's number is the count of run starts in lanes
// 1..l (lane 0 always starts one).
template <int Q>
__device__ __forceinline__ void run_positions(const Seg& g, uint32_t k, uint32_t (&pos)[Q]) {
  const uint32_t lane = threadIdx.x & (kRunWave - 1);
  const uint32_t w = __builtin_amdgcn_readfirstlane(k / kRunWave);
  const LBM_GLOBAL uint64_t* __restrict__ mk = gp(g.rmask) + (size_t)w * (Q - 1);
  const LBM_GLOBAL int32_t* __restrict__ val = gp(g.rval) + gp(g.rvoff)[w];
  uint32_t vb = 0;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const uint64_t m = mk[i - 1];
    const uint64_t m1 = m >> 1;
    const uint32_t r = __builtin_amdgcn_mbcnt_hi((uint32_t)(m1 >> 32),
                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)m1, 0u));
    pos[i] = (uint32_t)val[vb + r] + lane;
    vb += (uint32_t)__builtin_popcountll(m);
  }
}

// Cells with boundary links hand their density and momentum sums at the
// new time to the link update before the next step, which would otherwise
// gather all Q populations of the cell (one cache line each) to form the
// velocity.  The sums are taken from the values as stored (stored(j):
// population j of cell k in the storage format), decoded exactly as the
// link update would read them.
// Only marked cells compute it, so the other cells pay one test.  WAVE: the
// wavefront's cells are one wave of the mask (one cell per thread), so the
// mask word is a scalar load.
template <int Q, int ST, bool WAVE, class Stored>
__device__ __forceinline__ void put_link_velocity(const Seg& g, uint32_t k, Stored&& stored) {
  using SP = Store<ST>;
  using R = typename SP::R;
  if (!g.lmask) return;
  const uint32_t w = WAVE ? __builtin_amdgcn_readfirstlane(k / kRunWave) : k / kRunWave;
  const uint64_t m = gp(g.lmask)[w];
  if (!((m >> (k & (kRunWave - 1))) & 1ull)) return;
  const R isc = R(g.inv_scale);
  R e[Q];
#pragma unroll
  for (int j = 0; j < Q; ++j) e[j] = SP::load(stored(j), R(Lattice<Q>::w(j)), isc);
  R sums[4];
  cell_sums<Q, R>(e, sums);
  LBM_GLOBAL R* v = gp(static_cast<R*>(g.lvel)) + 4 * (size_t)link_entry(m, gp(g.lwoff)[w], k);
#pragma unroll
  for (int a = 0; a < 4; ++a) v[a] = sums[a];
}

// One cell of an AA (or pull) step; `tile` is the workgroup's tile of the
// launch and g the segment that owns it.  LV = false leaves out the
// link-velocity epilogue (launches in which no solve has the buffer).
template <int Q, int COLL, int ST, int MODE, int IDX, bool LV = true>
__device__ __forceinline__ void aa_cell(const Seg& g, uint32_t tile) {
  constexpr bool GATHER = MODE != MODE_EVEN;
  using SP = Store<ST>;
  using T = typename SP::T;
  using R = typename SP::R;
  const uint32_t k = (tile - g.tile0) * blockDim.x + threadIdx.x;
  if (k >= g.nf) return;
  LBM_GLOBAL T* __restrict__ pdf = gp(static_cast<T*>(g.pdf));
  const uint32_t S = g.S;
  const R sc = R(g.scale), isc = R(g.inv_scale);
  R d[Q];
  if constexpr (GATHER) {
    uint32_t pos[Q];
    pos[0] = k;
    if constexpr (IDX == IDX_RUN) {
      run_positions<Q>(g, k, pos);
    } else if constexpr (IDX == IDX_16) {
      // All offset loads first, then the tile's bases (the workgroup lies in
      // one compact tile: the block size divides kTile16), then branch-free
      // positions; escaped entries are patched under a wave-uniform branch.
      const LBM_GLOBAL uint16_t* __restrict__ off = gp(g.off16);
      const uint32_t t16 = ((tile - g.tile0) * blockDim.x) / kTile16;
      const LBM_GLOBAL int32_t* __restrict__ base = gp(g.base16) + (size_t)t16 * (Q - 1);
      uint32_t o[Q];
      int32_t b[Q];
#pragma unroll
      for (int i = 1; i < Q; ++i) o[i] = ld<LBM_NT_INDEX>(off + (size_t)(i - 1) * S + k);
#pragma unroll
      for (int i = 1; i < Q; ++i) b[i] = base[i - 1];
      bool esc = false;
#pragma unroll
      for (int i = 1; i < Q; ++i) {
        const uint32_t fl = (uint32_t)i * S + k + (uint32_t)b[i] + o[i];
        const uint32_t bb = (uint32_t)opp(i) * S + k;
        const uint32_t m = 0u - (uint32_t)(o[i] == kBounce16);  // all ones: bounce-back
        pos[i] = (fl & ~m) | (bb & m);
        esc = esc || o[i] == kEscape16;
      }
      if (__ballot(esc)) {
        const LBM_GLOBAL int32_t* __restrict__ idx = gp(g.idx);
#pragma unroll
        for (int i = 1; i < Q; ++i)
          if (o[i] == kEscape16) pos[i] = (uint32_t)idx[(size_t)(i - 1) * S + k];
      }
    } else {
      const LBM_GLOBAL int32_t* __restrict__ idx = gp(g.idx);
#pragma unroll
      for (int i = 1; i < Q; ++i)
        pos[i] = static_cast<uint32_t>(ld<LBM_NT_INDEX>(idx + (size_t)(i - 1) * S + k));
    }
#pragma unroll
    for (int i = 0; i < Q; ++i)
      d[i] = SP::load(ld<LBM_NT_GATHER>(pdf + pos[i]), R(Lattice<Q>::w(i)), isc);
    collide<Q, COLL, R>(d, seg_params<R>(g));
    if constexpr (MODE == MODE_ODD) {
#pragma unroll
      for (int i = 0; i < Q; ++i)
        st<LBM_NT_SCATTER>(SP::store(d[opp(i)], R(Lattice<Q>::w(i)), sc), pdf + pos[i]);
      if constexpr (LV)
        put_link_velocity<Q, ST, true>(
            g, k, [&](int j) { return SP::store(d[j], R(Lattice<Q>::w(j)), sc); });
    } else {
      LBM_GLOBAL T* __restrict__ dst = gp(static_cast<T*>(g.dst));
#pragma unroll
      for (int i = 0; i < Q; ++i)
        __builtin_nontemporal_store(SP::store(d[i], R(Lattice<Q>::w(i)), sc),
                                    dst + (size_t)i * S + k);
      put_link_velocity<Q, ST, true>(
          g, k, [&](int j) { return SP::store(d[j], R(Lattice<Q>::w(j)), sc); });
    }
  } else {
#pragma unroll
    for (int i = 0; i < Q; ++i)
      d[i] = SP::load(__builtin_nontemporal_load(pdf + (size_t)opp(i) * S + k),
                      R(Lattice<Q>::w(i)), isc);
    collide<Q, COLL, R>(d, seg_params<R>(g));
#pragma unroll
    for (int i = 0; i < Q; ++i)
      __builtin_nontemporal_store(SP::store(d[i], R(Lattice<Q>::w(i)), sc),
                                  pdf + (size_t)i * S + k);
    put_link_velocity<Q, ST, true>(
        g, k, [&](int j) { return SP::store(d[j], R(Lattice<Q>::w(j)), sc); });
  }
}

template <int Q, int COLL, int ST, int MODE, int IDX, bool LV>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(LBM_STEP_WAVES_PER_EU))) void k_aa_step(const StepArgs a) {
  const uint32_t tile = xcd_tile(blockIdx.x, a.ntiles, a.xcd_remap);
  with_seg(a, tile, [&](const Seg& g) { aa_cell<Q, COLL, ST, MODE, IDX, LV>(g, tile); });
}

// Even step, two neighbouring cells per thread: every load and store moves a
// 2-vector (cells k, k+1 of one direction block), twice the bytes per
// memory instruction of the one-cell kernel.  v[j] holds slot j of both
// cells; cell k's results replace the .x halves once collided (its inputs
// are then dead), cell k+1's the .y halves.  The host launches it only for
// even strides, so the 2-wide accesses are aligned and, when n_fluid is
// odd, the last pair's second cell is a padding slot (k+1 < stride): it
// collides its own finite padding values, which only padding reads.
template <int Q, int COLL, int ST>
__device__ __forceinline__ void even_pair_cells(const Seg& g, uint32_t tile) {
  using SP = Store<ST>;
  using T = typename SP::T;
  using R = typename SP::R;
  typedef T T2 __attribute__((ext_vector_type(2)));
  const uint32_t k = 2 * ((tile - g.tile0) * blockDim.x + threadIdx.x);
  if (k >= g.nf) return;
  LBM_GLOBAL T* __restrict__ pdf = gp(static_cast<T*>(g.pdf));
  const uint32_t S = g.S;
  const R sc = R(g.scale), isc = R(g.inv_scale);
  const CollParams<R> p = seg_params<R>(g);
  T2 v[Q];
#pragma unroll
  for (int j = 0; j < Q; ++j)
    v[j] = __builtin_nontemporal_load(
        reinterpret_cast<const LBM_GLOBAL T2*>(pdf + (size_t)j * S + k));
  R d[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) d[i] = SP::load(v[opp(i)].x, R(Lattice<Q>::w(i)), isc);
  collide<Q, COLL, R>(d, p);
#pragma unroll
  for (int i = 0; i < Q; ++i) v[i].x = SP::store(d[i], R(Lattice<Q>::w(i)), sc);
#pragma unroll
  for (int i = 0; i < Q; ++i) d[i] = SP::load(v[opp(i)].y, R(Lattice<Q>::w(i)), isc);
  collide<Q, COLL, R>(d, p);
#pragma unroll
  for (int i = 0; i < Q; ++i) v[i].y = SP::store(d[i], R(Lattice<Q>::w(i)), sc);
#pragma unroll
  for (int j = 0; j < Q; ++j)
    __builtin_nontemporal_store(v[j], reinterpret_cast<LBM_GLOBAL T2*>(pdf + (size_t)j * S + k));
  put_link_velocity<Q, ST, false>(g, k, [&](int j) { return v[j].x; });
  put_link_velocity<Q, ST, false>(g, k + 1, [&](int j) { return v[j].y; });
}

template <int Q, int COLL, int ST>
__global__ __launch_bounds__(256) void k_even_pair(const StepArgs a) {
  const uint32_t tile = xcd_tile(blockIdx.x, a.ntiles, a.xcd_remap);
  with_seg(a, tile, [&](const Seg& g) { even_pair_cells<Q, COLL, ST>(g, tile); });
}

// Persistent, software-pipelined odd step (compact index-list).  Each
// workgroup walks tiles v, v + G, v + 2G, ... (G = grid size, a multiple of
// 8 so that every tile of a workgroup maps to the same XCD range); the
// offsets of the next tile are loaded before the current tile's gathers,
// so the index latency of one tile overlaps the gather/collide/scatter of
// the previous one.  Same arithmetic as k_aa_step<..., MODE_ODD, true>.
template <int Q>
__device__ __forceinline__ void pipe_load_offsets(const Seg& g, uint32_t tile, uint32_t (&o)[Q]) {
  const uint32_t k = (tile - g.tile0) * blockDim.x + threadIdx.x;
  if (k < g.nf) {
#pragma unroll
    for (int i = 1; i < Q; ++i) o[i] = ld<LBM_NT_INDEX>(gp(g.off16) + (size_t)(i - 1) * g.S + k);
  }
}

template <int Q, int COLL, int ST>
__global__ __launch_bounds__(256) void k_odd_pipe(const StepArgs a) {
  using SP = Store<ST>;
  using T = typename SP::T;
  using R = typename SP::R;
  const uint32_t G = gridDim.x;
  uint32_t v = blockIdx.x;
  if (v >= a.ntiles) return;
  uint32_t tile = xcd_tile(v, a.ntiles, a.xcd_remap);
  uint32_t o[Q];
  with_seg(a, tile, [&](const Seg& g) { pipe_load_offsets<Q>(g, tile, o); });
  while (true) {
    const uint32_t vn = v + G;
    const bool has_next = vn < a.ntiles;
    uint32_t tn = 0;
    uint32_t on[Q];
    if (has_next) {
      tn = xcd_tile(vn, a.ntiles, a.xcd_remap);
      with_seg(a, tn, [&](const Seg& gn) { pipe_load_offsets<Q>(gn, tn, on); });
    }
    with_seg(a, tile, [&](const Seg& g) {
      const uint32_t k = (tile - g.tile0) * blockDim.x + threadIdx.x;
      if (k < g.nf) {
        LBM_GLOBAL T* __restrict__ pdf = gp(static_cast<T*>(g.pdf));
        const uint32_t S = g.S;
        const R sc = R(g.scale), isc = R(g.inv_scale);
        const uint32_t t16 = ((tile - g.tile0) * blockDim.x) / kTile16;
        const LBM_GLOBAL int32_t* __restrict__ base = gp(g.base16) + (size_t)t16 * (Q - 1);
        uint32_t pos[Q];
        int32_t b[Q];
        pos[0] = k;
#pragma unroll
        for (int i = 1; i < Q; ++i) b[i] = base[i - 1];
        bool esc = false;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
          const uint32_t fl = (uint32_t)i * S + k + (uint32_t)b[i] + o[i];
          const uint32_t bb = (uint32_t)opp(i) * S + k;
          const uint32_t m = 0u - (uint32_t)(o[i] == kBounce16);
          pos[i] = (fl & ~m) | (bb & m);
          esc = esc || o[i] == kEscape16;
        }
        if (__ballot(esc)) {
#pragma unroll
          for (int i = 1; i < Q; ++i)
            if (o[i] == kEscape16) pos[i] = (uint32_t)gp(g.idx)[(size_t)(i - 1) * S + k];
        }
        R d[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i)
          d[i] = SP::load(ld<LBM_NT_GATHER>(pdf + pos[i]), R(Lattice<Q>::w(i)), isc);
        collide<Q, COLL, R>(d, seg_params<R>(g));
#pragma unroll
        for (int i = 0; i < Q; ++i)
          st<LBM_NT_SCATTER>(SP::store(d[opp(i)], R(Lattice<Q>::w(i)), sc), pdf + pos[i]);
        put_link_velocity<Q, ST, true>(
            g, k, [&](int j) { return SP::store(d[j], R(Lattice<Q>::w(j)), sc); });
      }
    });
    if (!has_next) break;
    v = vn;
    tile = tn;
#pragma unroll
    for (int i = 1; i < Q; ++i) o[i] = on[i];
  }
}

// Host-side dispatch over (collision, storage, parity) for one Q.  `lds`:
// dynamic LDS reserved per workgroup (the step kernels use none); it caps
// how many workgroups share a CU.  links: some solve of the launch has a
// link-velocity buffer (the odd kernel comes in a variant without the
// epilogue; the others test for it at run time).
template <int Q, int COLL, int ST>
inline hipError_t launch_aa_cs(int mode, int idx, const StepArgs& a, int block, uint32_t lds,
                               bool links, hipStream_t st) {
  dim3 grid(a.ntiles), blk(block);
  if (mode == MODE_ODD_PIPE) {
    // resident workgroups of this kernel, rounded down to a multiple of 8
    // (computed once per kernel instance: every device is the same gfx950)
    static std::atomic<int> resident{0};
    if (resident.load() == 0) {
      int per_cu = 0, dev = 0, cus = 0;
      hipError_t e = hipGetDevice(&dev);
      if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
      if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_odd_pipe<Q, COLL, ST>, 256, 0);
      if (e != hipSuccess) return e;
      resident.store(per_cu * cus < 8 ? 8 : per_cu * cus);
    }
    const int per = resident.load() * 256 / block;
    uint32_t g = a.ntiles < (uint32_t)per ? a.ntiles : (uint32_t)per;
    if (g >= 8) g &= ~7u;
    hipLaunchKernelGGL((k_odd_pipe<Q, COLL, ST>), dim3(g), blk, lds, st, a);
    return hipGetLastError();
  }
  if (mode == MODE_EVEN2) {
    hipLaunchKernelGGL((k_even_pair<Q, COLL, ST>), grid, blk, lds, st, a);
    return hipGetLastError();
  }
  if (mode == MODE_ODD && idx == IDX_RUN) {
    if (links)
      hipLaunchKernelGGL((k_aa_step<Q, COLL, ST, MODE_ODD, IDX_RUN, true>), grid, blk, lds, st, a);
    else
      hipLaunchKernelGGL((k_aa_step<Q, COLL, ST, MODE_ODD, IDX_RUN, false>), grid, blk, lds, st,
                         a);
  } else if (mode == MODE_ODD && idx == IDX_16) {
    if (links)
      hipLaunchKernelGGL((k_aa_step<Q, COLL, ST, MODE_ODD, IDX_16, true>), grid, blk, lds, st, a);
    else
      hipLaunchKernelGGL((k_aa_step<Q, COLL, ST, MODE_ODD, IDX_16, false>), grid, blk, lds, st, a);
  } else if (mode == MODE_ODD) {
    if (links)
      hipLaunchKernelGGL((k_aa_step<Q, COLL, ST, MODE_ODD, IDX_I32, true>), grid, blk, lds, st, a);
    else
      hipLaunchKernelGGL((k_aa_step<Q, COLL, ST, MODE_ODD, IDX_I32, false>), grid, blk, lds, st,
                         a);
  } else if (mode == MODE_PULL && idx == IDX_16) {
    hipLaunchKernelGGL((k_aa_step<Q, COLL, ST, MODE_PULL, IDX_16, true>), grid, blk, lds, st, a);
  } else if (mode == MODE_PULL) {
    hipLaunchKernelGGL((k_aa_step<Q, COLL, ST, MODE_PULL, IDX_I32, true>), grid, blk, lds, st, a);
  } else {
    hipLaunchKernelGGL((k_aa_step<Q, COLL, ST, MODE_EVEN, IDX_I32, true>), grid, blk, lds, st, a);
  }
  return hipGetLastError();
}

template <int Q, int COLL>
inline hipError_t launch_aa_c(int storage, int mode, int idx, const StepArgs& a, int block,
                              uint32_t lds, bool links, hipStream_t st) {
  switch (storage) {
    case ST_F64: return launch_aa_cs<Q, COLL, ST_F64>(mode, idx, a, block, lds, links, st);
    case ST_F32: return launch_aa_cs<Q, COLL, ST_F32>(mode, idx, a, block, lds, links, st);
    case ST_F16DEV: return launch_aa_cs<Q, COLL, ST_F16DEV>(mode, idx, a, block, lds, links, st);
    case ST_BF16DEV:
      return launch_aa_cs<Q, COLL, ST_BF16DEV>(mode, idx, a, block, lds, links, st);
    case ST_F32DEV: return launch_aa_cs<Q, COLL, ST_F32DEV>(mode, idx, a, block, lds, links, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace lbm
