// Dense direct-addressing AA comparator (Section "Single Node Results":
// the dense kernel traverses every cell, fluid or not, so no fluid branch is
// needed and its fluid-cell throughput falls linearly with the porosity).
// PDF element i*N + lin.  Neighbours by index arithmetic with periodic wrap;
// bounce-back where bit i of the cell's mask says the upstream cell is not
// fluid.  Non-fluid cells carry an all-ones mask and only touch their own
// slots, so they never disturb the fluid.
#include "step_impl.hpp"
#include "internal.hpp"

namespace lbm {

template <int Q>
__global__ __launch_bounds__(256) void k_dense_mask(const uint8_t* labels, int nx, int ny, int nz,
                                                    uint32_t periodic, uint32_t* mask) {
  using L = Lattice<Q>;
  const uint64_t N = (uint64_t)nx * ny * nz;
  const uint64_t lin = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (lin >= N) return;
  if (labels[lin] != 0) {
    mask[lin] = 0xffffffffu;
    return;
  }
  const int x = (int)(lin % nx), y = (int)((lin / nx) % ny), z = (int)(lin / ((uint64_t)nx * ny));
  uint32_t m = 0;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    int p[3] = {x - L::cx[i], y - L::cy[i], z - L::cz[i]};
    const int n[3] = {nx, ny, nz};
    bool out = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (p[a] < 0 || p[a] >= n[a]) {
        if (!((periodic >> a) & 1u)) out = true;
        p[a] = p[a] < 0 ? p[a] + n[a] : p[a] - n[a];
      }
    }
    if (out || labels[(uint64_t)p[0] + (uint64_t)nx * ((uint64_t)p[1] + (uint64_t)ny * p[2])] != 0)
      m |= 1u << i;
  }
  mask[lin] = m;
}

__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

template <int Q, int COLL, int ST, bool ODD>
__global__ __launch_bounds__(256) void k_dense_step(const DenseArgs a) {
  using SP = Store<ST>;
  using T = typename SP::T;
  using R = typename SP::R;
  using L = Lattice<Q>;
  const uint32_t tile = xcd_tile(blockIdx.x, a.ntiles, a.xcd_remap);
  const uint32_t lin = tile * blockDim.x + threadIdx.x;
  if (lin >= a.N) return;
  T* __restrict__ pdf = static_cast<T*>(a.pdf);
  const uint32_t N = a.N;
  const R sc = R(a.scale), isc = R(a.inv_scale);
  CollParams<R> p;
  p.om1 = R(a.om1);
  p.om2 = R(a.om2);
  for (int r = 0; r < 4; ++r) p.r[r] = R(a.rates[r]);
  p.Fx = R(a.F[0]);
  p.Fy = R(a.F[1]);
  p.Fz = R(a.F[2]);
  R d[Q];
  if constexpr (ODD) {
    const uint32_t m = a.mask[lin];
    const uint32_t nxy = (uint32_t)a.nx * (uint32_t)a.ny;
    const int z = (int)(lin / nxy);
    const uint32_t r = lin - (uint32_t)z * nxy;
    const int y = (int)(r / (uint32_t)a.nx);
    const int x = (int)(r - (uint32_t)y * (uint32_t)a.nx);
    uint32_t pos[Q];
    pos[0] = lin;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const uint32_t up = (uint32_t)wrap(x - L::cx[i], a.nx) +
                          (uint32_t)a.nx * ((uint32_t)wrap(y - L::cy[i], a.ny) +
                                            (uint32_t)a.ny * (uint32_t)wrap(z - L::cz[i], a.nz));
      pos[i] = ((m >> i) & 1u) ? (uint32_t)opp(i) * N + lin : (uint32_t)i * N + up;
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) d[i] = SP::load(pdf[pos[i]], R(L::w(i)), isc);
    collide<Q, COLL, R>(d, p);
#pragma unroll
    for (int i = 0; i < Q; ++i) pdf[pos[i]] = SP::store(d[opp(i)], R(L::w(i)), sc);
  } else {
#pragma unroll
    for (int i = 0; i < Q; ++i)
      d[i] = SP::load(__builtin_nontemporal_load(pdf + (size_t)opp(i) * N + lin), R(L::w(i)), isc);
    collide<Q, COLL, R>(d, p);
#pragma unroll
    for (int i = 0; i < Q; ++i)
      __builtin_nontemporal_store(SP::store(d[i], R(L::w(i)), sc), pdf + (size_t)i * N + lin);
  }
}

hipError_t launch_dense_mask(const uint8_t* labels, int nx, int ny, int nz, uint32_t periodic,
                             int q, uint32_t* mask, hipStream_t st) {
  const uint64_t N = (uint64_t)nx * ny * nz;
  dim3 g((unsigned)((N + 255) / 256)), b(256);
  if (q == 19)
    hipLaunchKernelGGL(k_dense_mask<19>, g, b, 0, st, labels, nx, ny, nz, periodic, mask);
  else
    hipLaunchKernelGGL(k_dense_mask<27>, g, b, 0, st, labels, nx, ny, nz, periodic, mask);
  return hipGetLastError();
}

template <int Q, int COLL, int ST>
static hipError_t launch_dense_qcs(bool odd, const DenseArgs& a, int block, hipStream_t st) {
  dim3 g(a.ntiles), b(block);
  if (odd)
    hipLaunchKernelGGL((k_dense_step<Q, COLL, ST, true>), g, b, 0, st, a);
  else
    hipLaunchKernelGGL((k_dense_step<Q, COLL, ST, false>), g, b, 0, st, a);
  return hipGetLastError();
}

template <int Q, int COLL>
static hipError_t launch_dense_qc(int storage, bool odd, const DenseArgs& a, int block,
                                  hipStream_t st) {
  switch (storage) {
    case ST_F64: return launch_dense_qcs<Q, COLL, ST_F64>(odd, a, block, st);
    case ST_F32: return launch_dense_qcs<Q, COLL, ST_F32>(odd, a, block, st);
    case ST_F16DEV: return launch_dense_qcs<Q, COLL, ST_F16DEV>(odd, a, block, st);
    case ST_BF16DEV: return launch_dense_qcs<Q, COLL, ST_BF16DEV>(odd, a, block, st);
    case ST_F32DEV: return launch_dense_qcs<Q, COLL, ST_F32DEV>(odd, a, block, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_dense_step(int q, int coll, int storage, bool odd, const DenseArgs& a,
                             int block, hipStream_t st) {
  if (q == 19) {
    if (coll == COLL_SRT) return launch_dense_qc<19, COLL_SRT>(storage, odd, a, block, st);
    if (coll == COLL_TRT) return launch_dense_qc<19, COLL_TRT>(storage, odd, a, block, st);
    if (coll == COLL_NONE) return launch_dense_qc<19, COLL_NONE>(storage, odd, a, block, st);
    if (coll == COLL_MRT) return launch_dense_qc<19, COLL_MRT>(storage, odd, a, block, st);
  } else if (q == 27) {
    if (coll == COLL_SRT) return launch_dense_qc<27, COLL_SRT>(storage, odd, a, block, st);
    if (coll == COLL_TRT) return launch_dense_qc<27, COLL_TRT>(storage, odd, a, block, st);
    if (coll == COLL_CUMULANT) return launch_dense_qc<27, COLL_CUMULANT>(storage, odd, a, block, st);
    if (coll == COLL_CM) return launch_dense_qc<27, COLL_CM>(storage, odd, a, block, st);
    if (coll == COLL_NONE) return launch_dense_qc<27, COLL_NONE>(storage, odd, a, block, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace lbm
