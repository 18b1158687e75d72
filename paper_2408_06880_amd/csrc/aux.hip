// Equilibrium initialisation, boundary-link updates, per-cell moments,
// deterministic FP64 reductions and the streaming copy kernel.
#include <string.h>

#include "collide.hpp"
#include "internal.hpp"

namespace lbm {

// Direction data for a runtime direction index (small kernels only).
template <int Q>
__device__ __forceinline__ void dir_of(int i, int& cx, int& cy, int& cz, double& w) {
  using L = Lattice<Q>;
  cx = cy = cz = 0;
  w = L::w(0);
#pragma unroll
  for (int j = 1; j < Q; ++j)
    if (j == i) {
      cx = L::cx[j];
      cy = L::cy[j];
      cz = L::cz[j];
      w = L::w(j);
    }
}

// ------------------------------------------------------------------ init
template <int Q, int ST>
__global__ __launch_bounds__(256) void k_init(void* pdf_, uint32_t S, uint32_t nf, double rho0,
                                              double ux, double uy, double uz, float scale) {
  using SP = Store<ST>;
  using T = typename SP::T;
  using R = typename SP::R;
  T* pdf = static_cast<T*>(pdf_);
  const uint64_t n = (uint64_t)Q * S;
  const double usq = ux * ux + uy * uy + uz * uz;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (uint64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / S);
    const uint32_t k = (uint32_t)(e - (uint64_t)i * S);
    int cx, cy, cz;
    double w;
    dir_of<Q>(i, cx, cy, cz, w);
    double dev = 0.0;
    if (k < nf) {
      const double cu = cx * ux + cy * uy + cz * uz;
      dev = w * ((rho0 - 1.0) + rho0 * (3.0 * cu + 4.5 * cu * cu - 1.5 * usq));
    }
    pdf[e] = SP::store(R(dev), R(w), R(scale));
  }
}

template <int Q>
static hipError_t launch_init_q(int storage, void* pdf, uint32_t S, uint32_t nf, double rho0,
                                const double u0[3], float scale, hipStream_t st) {
  const uint64_t n = (uint64_t)Q * S;
  uint64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks == 0) blocks = 1;
  dim3 g((unsigned)blocks), b(256);
  switch (storage) {
    case ST_F64: hipLaunchKernelGGL((k_init<Q, ST_F64>), g, b, 0, st, pdf, S, nf, rho0, u0[0], u0[1], u0[2], scale); break;
    case ST_F32: hipLaunchKernelGGL((k_init<Q, ST_F32>), g, b, 0, st, pdf, S, nf, rho0, u0[0], u0[1], u0[2], scale); break;
    case ST_F16DEV: hipLaunchKernelGGL((k_init<Q, ST_F16DEV>), g, b, 0, st, pdf, S, nf, rho0, u0[0], u0[1], u0[2], scale); break;
    case ST_BF16DEV: hipLaunchKernelGGL((k_init<Q, ST_BF16DEV>), g, b, 0, st, pdf, S, nf, rho0, u0[0], u0[1], u0[2], scale); break;
    case ST_F32DEV: hipLaunchKernelGGL((k_init<Q, ST_F32DEV>), g, b, 0, st, pdf, S, nf, rho0, u0[0], u0[1], u0[2], scale); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_init(int q, int storage, void* pdf, uint32_t S, uint32_t nf, double rho0,
                       const double u0[3], float scale, hipStream_t st) {
  if (q == 19) return launch_init_q<19>(storage, pdf, S, nf, rho0, u0, scale, st);
  if (q == 27) return launch_init_q<27>(storage, pdf, S, nf, rho0, u0, scale, st);
  return hipErrorInvalidValue;
}

// ----------------------------------------------------------- moments
// Post-collision deviations of cell k at the current time in natural order.
// Even t: natural slots.  Odd t: population opp(i) sits where the cell
// pulled population i from in the last (odd) step.  The run form is decoded
// by this thread alone, directions in storage order: the pull position of
// direction i is the value of the run holding lane k % 64 (the count of run
// starts in lanes 0..lane, minus one, after the runs of directions 1..i-1)
// plus the lane.  (The step kernels decode runs a whole wave at a time.)
template <int Q, int ST, bool ODD_T>
__device__ __forceinline__ void gather_post(const Seg& g, uint32_t k,
                                            typename Store<ST>::R (&d)[Q]) {
  using SP = Store<ST>;
  using T = typename SP::T;
  using R = typename SP::R;
  const LBM_GLOBAL T* pdf = gp(static_cast<const T*>(g.pdf));
  const R isc = R(g.inv_scale);
  uint32_t pos[Q];
#pragma unroll
  for (int j = 0; j < Q; ++j) pos[j] = (uint32_t)j * g.S + k;
  if (ODD_T) {
    if (g.rval) {
      const uint32_t w = k / kRunWave, lane = k % kRunWave;
      const LBM_GLOBAL uint64_t* mk = gp(g.rmask) + (size_t)w * (Q - 1);
      const LBM_GLOBAL int32_t* val = gp(g.rval) + gp(g.rvoff)[w];
      const uint64_t upto = lane == kRunWave - 1 ? ~0ull : ((2ull << lane) - 1ull);
      uint32_t vb = 0;
#pragma unroll
      for (int i = 1; i < Q; ++i) {
        const uint64_t m = mk[i - 1];
        const uint32_t r = (uint32_t)__popcll(m & upto) - 1u;
        pos[opp(i)] = (uint32_t)val[vb + r] + lane;
        vb += (uint32_t)__popcll(m);
      }
    } else {
      const uint32_t t16 = k / kTile16;
#pragma unroll
      for (int j = 1; j < Q; ++j)
        pos[j] = g.off16 ? pos16(g, Q, opp(j), j, k, t16)
                         : (uint32_t)gp(g.idx)[(size_t)(opp(j) - 1) * g.S + k];
    }
  }
#pragma unroll
  for (int j = 0; j < Q; ++j) d[j] = SP::load(pdf[pos[j]], R(Lattice<Q>::w(j)), isc);
}

// ------------------------------------------------------------- links
// Boundary link update, applied before every step to the slot that the
// link's cell pulls across the boundary (Section "Sparse Boundary
// Conditions", realised as an update of that slot instead of appended
// boundary PDFs), in deviation form:
//   UBB:      d <- d + 6 w_i (c_i . u_w)               (rho_w = 1)
//   pressure: d <- -d + 2 w_i (rho_out (1 + 9/2 (c_i.u)^2 - 3/2 u.u) - 1)
// with u the cell's velocity at the current time (anti-bounce-back: the
// sum of the two opposite second-order equilibria at (rho_out, u)).  The
// links are ordered by cell, so the first link of each cell updates all of
// that cell's links: it reads the velocity from the cell's populations
// before any of their slots changes, and no two threads touch one cell's
// slots.  A link slot holds a population of its own cell at both parities,
// so cells never touch each other's slots.
// Fluid cell of link l (its slot is opp(i) * S + k).
__device__ __forceinline__ uint32_t link_cell(const LinkArgs& a, uint32_t l) {
  const int i = a.links[2 * l + 1] & 0xff;
  return (uint32_t)a.links[2 * l] - (uint32_t)opp(i) * a.g.S;
}

// Updated value of one link slot v (direction and class in meta; class type
// 1 or 2) at the cell's velocity u.
template <int Q, int ST>
__device__ __forceinline__ typename Store<ST>::T link_slot(const LinkArgs& a, int meta,
                                                           typename Store<ST>::T v,
                                                           typename Store<ST>::R ux,
                                                           typename Store<ST>::R uy,
                                                           typename Store<ST>::R uz) {
  using SP = Store<ST>;
  using R = typename SP::R;
  const int i = meta & 0xff, cls = (meta >> 8) & 0xff;
  int cx, cy, cz;
  double w;
  dir_of<Q>(i, cx, cy, cz, w);
  R dv = SP::load(v, R(w), R(a.inv_scale));
  if (a.type[cls] == 1) {
    dv = dv + R(6.0 * w * (cx * a.u[cls][0] + cy * a.u[cls][1] + cz * a.u[cls][2]));
  } else {
    const R cu = R(cx) * ux + R(cy) * uy + R(cz) * uz;
    const R uu = ux * ux + uy * uy + uz * uz;
    dv = -dv + R(2.0 * w * (a.rho[cls] - 1.0)) +
         R(2.0 * w * a.rho[cls]) * (R(4.5) * cu * cu - R(1.5) * uu);
  }
  return SP::store(dv, R(w), R(a.scale));
}

__device__ __forceinline__ int link_type(const LinkArgs& a, int meta) {
  const int cls = (meta >> 8) & 0xff;
  return cls < a.n_classes ? a.type[cls] : 0;
}

template <int Q, int ST, bool ODD_T>
__global__ __launch_bounds__(256) void k_links(const LinkArgs a) {
  using SP = Store<ST>;
  using T = typename SP::T;
  using R = typename SP::R;
  const uint32_t l0 = blockIdx.x * blockDim.x + threadIdx.x;
  if (l0 >= a.n_links) return;
  const uint32_t k = link_cell(a, l0);
  if (l0 > 0 && link_cell(a, l0 - 1) == k) return;  // not the cell's first link
  // The cell's links are l0, l0 + 1, ... (at most Q - 1 of them; links are
  // ordered by cell).  All metadata and slot values are loaded before any
  // slot is written, so the loads overlap instead of waiting one by one.
  T* pdf = static_cast<T*>(a.pdf);
  uint32_t pos[Q - 1];
  int meta[Q - 1];
  T v[Q - 1];
  bool on[Q - 1];
  bool pressure = false;
#pragma unroll
  for (int m = 0; m < Q - 1; ++m) {
    const uint32_t l = l0 + (uint32_t)m;
    on[m] = l < a.n_links && link_cell(a, l) == k;
    pos[m] = 0;
    meta[m] = 0;
    if (on[m]) {
      pos[m] = (uint32_t)a.links[2 * l];
      meta[m] = a.links[2 * l + 1];
      pressure = pressure || link_type(a, meta[m]) == 2;
    }
  }
#pragma unroll
  for (int m = 0; m < Q - 1; ++m)
    if (on[m]) v[m] = pdf[pos[m]];
  R ux = 0, uy = 0, uz = 0;
  if (pressure) {
    R d[Q];
    gather_post<Q, ST, ODD_T>(a.g, k, d);
    R sums[4];
    cell_sums<Q, R>(d, sums);
    sums_velocity<R>(sums, a.g.F, ux, uy, uz);
  }
#pragma unroll
  for (int m = 0; m < Q - 1; ++m)
    if (on[m] && link_type(a, meta[m]) != 0)
      pdf[pos[m]] = link_slot<Q, ST>(a, meta[m], v[m], ux, uy, uz);
}

// The same update when the step kernel before it left the density and
// momentum sums of every cell with links in the link-velocity buffer: no
// thread reads a slot that another one writes, so one thread takes one
// link.
template <int Q, int ST>
__global__ __launch_bounds__(256) void k_links_vel(const LinkArgs a) {
  using SP = Store<ST>;
  using T = typename SP::T;
  using R = typename SP::R;
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= a.n_links) return;
  const uint32_t pos = (uint32_t)a.links[2 * l];
  const int meta = a.links[2 * l + 1];
  const int type = link_type(a, meta);
  if (type == 0) return;
  LBM_GLOBAL T* pdf = gp(static_cast<T*>(a.pdf));
  const T v = pdf[pos];
  R ux = 0, uy = 0, uz = 0;
  if (type == 2) {
    const uint32_t k = pos - (uint32_t)opp(meta & 0xff) * a.g.S;
    const uint32_t w = k / kRunWave;
    const LBM_GLOBAL R* p = gp(static_cast<const R*>(a.g.lvel)) +
                            4 * (size_t)link_entry(gp(a.g.lmask)[w], gp(a.g.lwoff)[w], k);
    const R sums[4] = {p[0], p[1], p[2], p[3]};
    sums_velocity<R>(sums, a.g.F, ux, uy, uz);
  }
  pdf[pos] = link_slot<Q, ST>(a, meta, v, ux, uy, uz);
}

template <int Q, int ST>
static void launch_links_vel_st(const LinkArgs& a, hipStream_t st) {
  hipLaunchKernelGGL((k_links_vel<Q, ST>), dim3((a.n_links + 255) / 256), dim3(256), 0, st, a);
}

template <int Q, bool ODD_T>
static hipError_t launch_links_qt(int storage, const LinkArgs& a, hipStream_t st) {
  dim3 g((a.n_links + 255) / 256), b(256);
  switch (storage) {
    case ST_F64: hipLaunchKernelGGL((k_links<Q, ST_F64, ODD_T>), g, b, 0, st, a); break;
    case ST_F32: hipLaunchKernelGGL((k_links<Q, ST_F32, ODD_T>), g, b, 0, st, a); break;
    case ST_F16DEV: hipLaunchKernelGGL((k_links<Q, ST_F16DEV, ODD_T>), g, b, 0, st, a); break;
    case ST_BF16DEV: hipLaunchKernelGGL((k_links<Q, ST_BF16DEV, ODD_T>), g, b, 0, st, a); break;
    case ST_F32DEV: hipLaunchKernelGGL((k_links<Q, ST_F32DEV, ODD_T>), g, b, 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int Q>
static hipError_t launch_links_q(int storage, const LinkArgs& a, hipStream_t st) {
  if (a.use_vel) {
    switch (storage) {
      case ST_F64: launch_links_vel_st<Q, ST_F64>(a, st); break;
      case ST_F32: launch_links_vel_st<Q, ST_F32>(a, st); break;
      case ST_F16DEV: launch_links_vel_st<Q, ST_F16DEV>(a, st); break;
      case ST_BF16DEV: launch_links_vel_st<Q, ST_BF16DEV>(a, st); break;
      case ST_F32DEV: launch_links_vel_st<Q, ST_F32DEV>(a, st); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  return a.natural ? launch_links_qt<Q, false>(storage, a, st)
                   : launch_links_qt<Q, true>(storage, a, st);
}

hipError_t launch_links(int storage, const LinkArgs& a, hipStream_t st) {
  if (a.n_links == 0) return hipSuccess;
  if (a.q == 19) return launch_links_q<19>(storage, a, st);
  if (a.q == 27) return launch_links_q<27>(storage, a, st);
  return hipErrorInvalidValue;
}

// Link-velocity buffer set-up: one bit per cell that has a link.
__global__ __launch_bounds__(256) void k_link_mask_clear(uint64_t* mask, uint32_t nw) {
  const uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w < nw) mask[w] = 0;
}

__global__ __launch_bounds__(256) void k_link_mask_mark(const int32_t* links, uint32_t n_links,
                                                        uint32_t S, uint32_t nw, uint64_t* mask) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= n_links) return;
  const int i = links[2 * l + 1] & 0xff;
  const uint32_t k = (uint32_t)links[2 * l] - (uint32_t)opp(i) * S;
  if (k / kRunWave < nw) atomicOr((unsigned long long*)&mask[k / kRunWave], 1ull << (k % kRunWave));
}

__global__ __launch_bounds__(256) void k_link_mask_count(const uint64_t* mask, uint32_t nw,
                                                         uint32_t* woff) {
  const uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w < nw) woff[w] = (uint32_t)__popcll(mask[w]);
}

hipError_t launch_link_mask(const int32_t* links, uint32_t n_links, uint32_t S,
                            uint32_t nw, uint64_t* mask, uint32_t* woff, hipStream_t st) {
  const dim3 b(256);
  hipLaunchKernelGGL(k_link_mask_clear, dim3((nw + 255) / 256), b, 0, st, mask, nw);
  if (n_links > 0)
    hipLaunchKernelGGL(k_link_mask_mark, dim3((n_links + 255) / 256), b, 0, st, links, n_links, S,
                       nw, mask);
  hipLaunchKernelGGL(k_link_mask_count, dim3((nw + 255) / 256), b, 0, st, mask, nw, woff);
  return hipGetLastError();
}

template <int Q, int ST, bool ODD_T, class O>
__global__ __launch_bounds__(256) void k_moments(const Seg g, O* rho, O* u) {
  using R = typename Store<ST>::R;
  using L = Lattice<Q>;
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= g.nf) return;
  R d[Q];
  gather_post<Q, ST, ODD_T>(g, k, d);
  R drho = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    drho += d[i];
    jx += R(L::cx[i]) * d[i];
    jy += R(L::cy[i]) * d[i];
    jz += R(L::cz[i]) * d[i];
  }
  const R r = R(1) + drho;
  rho[k] = O(r);
  u[k] = O((jx - R(0.5) * R(g.F[0])) / r);
  u[(size_t)g.S + k] = O((jy - R(0.5) * R(g.F[1])) / r);
  u[2 * (size_t)g.S + k] = O((jz - R(0.5) * R(g.F[2])) / r);
}

template <int Q, int ST>
static hipError_t launch_moments_qs(const Seg& g, bool odd_t, bool out_f64, void* rho, void* u,
                                    hipStream_t st) {
  dim3 gr((g.nf + 255) / 256), b(256);
  if (g.nf == 0) return hipSuccess;
  if (odd_t) {
    if (out_f64)
      hipLaunchKernelGGL((k_moments<Q, ST, true, double>), gr, b, 0, st, g, (double*)rho, (double*)u);
    else
      hipLaunchKernelGGL((k_moments<Q, ST, true, float>), gr, b, 0, st, g, (float*)rho, (float*)u);
  } else {
    if (out_f64)
      hipLaunchKernelGGL((k_moments<Q, ST, false, double>), gr, b, 0, st, g, (double*)rho, (double*)u);
    else
      hipLaunchKernelGGL((k_moments<Q, ST, false, float>), gr, b, 0, st, g, (float*)rho, (float*)u);
  }
  return hipGetLastError();
}

template <int Q>
static hipError_t launch_moments_q(int storage, const Seg& g, bool odd_t, bool out_f64,
                                   void* rho, void* u, hipStream_t st) {
  switch (storage) {
    case ST_F64: return launch_moments_qs<Q, ST_F64>(g, odd_t, out_f64, rho, u, st);
    case ST_F32: return launch_moments_qs<Q, ST_F32>(g, odd_t, out_f64, rho, u, st);
    case ST_F16DEV: return launch_moments_qs<Q, ST_F16DEV>(g, odd_t, out_f64, rho, u, st);
    case ST_BF16DEV: return launch_moments_qs<Q, ST_BF16DEV>(g, odd_t, out_f64, rho, u, st);
    case ST_F32DEV: return launch_moments_qs<Q, ST_F32DEV>(g, odd_t, out_f64, rho, u, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_moments(int q, int storage, const Seg& g, bool odd_t, bool out_f64, void* rho,
                          void* u, hipStream_t st) {
  if (q == 19) return launch_moments_q<19>(storage, g, odd_t, out_f64, rho, u, st);
  if (q == 27) return launch_moments_q<27>(storage, g, odd_t, out_f64, rho, u, st);
  return hipErrorInvalidValue;
}

// -------------------------------------------------------- reductions
// Deterministic two-pass FP64 sums.  Pass 1: one workgroup per tile of
// kRedBlock cells; each wavefront reduces with a fixed butterfly, the
// wavefront sums are added in wave order.  Pass 2: one workgroup per
// segment adds its tiles in a fixed strided order and a fixed tree.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sums of one thread's cell of a reduction tile into v (zeros past the
// segment's fluid cells).
template <int Q, int ST, bool ODD_T>
__device__ __forceinline__ void reduce_cell(const Seg& g, uint32_t tile, double (&v)[5]) {
  using R = typename Store<ST>::R;
  using L = Lattice<Q>;
  const uint32_t k = (tile - g.tile0) * kRedBlock + threadIdx.x;
  if (k < g.nf) {
    R d[Q];
    gather_post<Q, ST, ODD_T>(g, k, d);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const double x = (double)d[i];
      v[0] += x;
      v[1] += L::cx[i] * x;
      v[2] += L::cy[i] * x;
      v[3] += L::cz[i] * x;
    }
    v[1] -= 0.5 * g.F[0];
    v[2] -= 0.5 * g.F[1];
    v[3] -= 0.5 * g.F[2];
    bool fin = true;
#pragma unroll
    for (int m = 0; m < 4; ++m) fin = fin && __builtin_isfinite(v[m]);
    v[4] = fin ? 0.0 : 1.0;
  }
}

template <int Q, int ST, bool ODD_T>
__global__ __launch_bounds__(kRedBlock) void k_reduce_tiles(const StepArgs a, double* partials) {
  __shared__ double sh[kRedBlock / 64][5];
  const uint32_t tile = blockIdx.x;
  double v[5] = {0, 0, 0, 0, 0};
  with_seg(a, tile, [&](const Seg& g) { reduce_cell<Q, ST, ODD_T>(g, tile, v); });
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    const double t = wave_sum(v[m]);
    if (lane == 0) sh[wv][m] = t;
  }
  __syncthreads();
  if (threadIdx.x < 5) {
    double t = 0.0;
    for (int w = 0; w < kRedBlock / 64; ++w) t += sh[w][threadIdx.x];
    partials[(size_t)tile * 5 + threadIdx.x] = t;
  }
}

__global__ __launch_bounds__(256) void k_reduce_segs(const StepArgs a, const double* partials,
                                                     double* out) {
  __shared__ double sh[256][5];
  const int s = blockIdx.x;
  const uint32_t t0 = seg_tile0(a, s);
  const uint32_t t1 = (s + 1 < a.nseg) ? seg_tile0(a, s + 1) : a.ntiles;
  double v[5] = {0, 0, 0, 0, 0};
  for (uint32_t t = t0 + threadIdx.x; t < t1; t += 256)
    for (int m = 0; m < 5; ++m) v[m] += partials[(size_t)t * 5 + m];
  for (int m = 0; m < 5; ++m) sh[threadIdx.x][m] = v[m];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h)
      for (int m = 0; m < 5; ++m) sh[threadIdx.x][m] += sh[threadIdx.x + h][m];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double nf = (double)seg_nf(a, s);
    out[s * 8 + 0] = nf + sh[0][0];  // mass
    out[s * 8 + 1] = sh[0][0];       // sum of density deviations
    out[s * 8 + 2] = sh[0][1];
    out[s * 8 + 3] = sh[0][2];
    out[s * 8 + 4] = sh[0][3];
    out[s * 8 + 5] = sh[0][4];       // cells with non-finite values
    out[s * 8 + 6] = nf;
    out[s * 8 + 7] = 0.0;
  }
}

template <int Q, int ST>
static hipError_t launch_reduce_qs(const StepArgs& a, bool odd_t, double* partials, double* out,
                                   hipStream_t st) {
  dim3 g1(a.ntiles), b1(kRedBlock), g2(a.nseg), b2(256);
  if (a.ntiles > 0) {
    if (odd_t)
      hipLaunchKernelGGL((k_reduce_tiles<Q, ST, true>), g1, b1, 0, st, a, partials);
    else
      hipLaunchKernelGGL((k_reduce_tiles<Q, ST, false>), g1, b1, 0, st, a, partials);
  }
  hipLaunchKernelGGL(k_reduce_segs, g2, b2, 0, st, a, (const double*)partials, out);
  return hipGetLastError();
}

template <int Q>
static hipError_t launch_reduce_q(int storage, const StepArgs& a, bool odd_t, double* partials,
                                  double* out, hipStream_t st) {
  switch (storage) {
    case ST_F64: return launch_reduce_qs<Q, ST_F64>(a, odd_t, partials, out, st);
    case ST_F32: return launch_reduce_qs<Q, ST_F32>(a, odd_t, partials, out, st);
    case ST_F16DEV: return launch_reduce_qs<Q, ST_F16DEV>(a, odd_t, partials, out, st);
    case ST_BF16DEV: return launch_reduce_qs<Q, ST_BF16DEV>(a, odd_t, partials, out, st);
    case ST_F32DEV: return launch_reduce_qs<Q, ST_F32DEV>(a, odd_t, partials, out, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_reduce(int q, int storage, const StepArgs& a, bool odd_t, double* partials,
                         double* out, hipStream_t st) {
  if (q == 19) return launch_reduce_q<19>(storage, a, odd_t, partials, out, st);
  if (q == 27) return launch_reduce_q<27>(storage, a, odd_t, partials, out, st);
  return hipErrorInvalidValue;
}

// ------------------------------------------------------ segment tables
// A batch launch reads its segment table from device memory.  The host
// writes it with this kernel (up to kSegChunk entries per launch, from the
// kernel arguments) instead of a host-to-device copy, so the table travels
// in stream order, needs no pinned host buffer and can be captured.
struct SegChunk {
  uint32_t n;
  uint32_t pad;
  Seg seg[kSegChunk];
};

__global__ __launch_bounds__(256) void k_put_segs(const SegChunk c, Seg* dst) {
  static_assert(sizeof(Seg) % 8 == 0, "segments are copied as 8-byte words");
  const uint32_t words = c.n * (uint32_t)(sizeof(Seg) / 8);
  const uint64_t* src = reinterpret_cast<const uint64_t*>(c.seg);
  uint64_t* out = reinterpret_cast<uint64_t*>(dst);
  for (uint32_t w = threadIdx.x; w < words; w += blockDim.x) out[w] = src[w];
}

hipError_t launch_put_segs(const Seg* host, uint32_t n, Seg* dev, hipStream_t st) {
  for (uint32_t j = 0; j < n; j += kSegChunk) {
    SegChunk c;
    memset(&c, 0, sizeof(c));
    c.n = n - j < kSegChunk ? n - j : kSegChunk;
    memcpy(c.seg, host + j, c.n * sizeof(Seg));
    hipLaunchKernelGGL(k_put_segs, dim3(1), dim3(256), 0, st, c, dev + j);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// -------------------------------------------------------------- copy
// Bandwidth reference: one 16-byte vector per thread, non-temporal load and
// store, one workgroup per 4 KiB.
typedef float v4f __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_copy(const v4f* __restrict__ src, v4f* __restrict__ dst,
                                              uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// Storage conversion: every slot decoded to its deviation delta = f - w in
// FP64 and encoded in the destination format.  Opposite directions share
// their weight, so the slot's population (natural or swapped, by the AA
// parity) does not matter.
template <int Q, int SA, int SB>
__global__ __launch_bounds__(256) void k_convert(const void* src_, void* dst_, uint32_t S,
                                                 float inv_scale_a, float scale_b) {
  using A = Store<SA>;
  using B = Store<SB>;
  const typename A::T* src = static_cast<const typename A::T*>(src_);
  typename B::T* dst = static_cast<typename B::T*>(dst_);
  const uint64_t n = (uint64_t)Q * S;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (uint64_t)gridDim.x * blockDim.x) {
    int cx, cy, cz;
    double w;
    dir_of<Q>((int)(e / S), cx, cy, cz, w);
    const double dev =
        (double)A::load(src[e], typename A::R(w), typename A::R(inv_scale_a));
    dst[e] = B::store(typename B::R(dev), typename B::R(w), typename B::R(scale_b));
  }
}

template <int Q, int SA>
static hipError_t launch_convert_a(int sb, const void* src, void* dst, uint32_t S,
                                   float inv_scale_a, float scale_b, hipStream_t st) {
  const uint64_t n = (uint64_t)Q * S;
  uint64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks == 0) return hipSuccess;
  const dim3 g((unsigned)blocks), b(256);
  switch (sb) {
    case ST_F64: hipLaunchKernelGGL((k_convert<Q, SA, ST_F64>), g, b, 0, st, src, dst, S, inv_scale_a, scale_b); break;
    case ST_F32: hipLaunchKernelGGL((k_convert<Q, SA, ST_F32>), g, b, 0, st, src, dst, S, inv_scale_a, scale_b); break;
    case ST_F16DEV: hipLaunchKernelGGL((k_convert<Q, SA, ST_F16DEV>), g, b, 0, st, src, dst, S, inv_scale_a, scale_b); break;
    case ST_BF16DEV: hipLaunchKernelGGL((k_convert<Q, SA, ST_BF16DEV>), g, b, 0, st, src, dst, S, inv_scale_a, scale_b); break;
    case ST_F32DEV: hipLaunchKernelGGL((k_convert<Q, SA, ST_F32DEV>), g, b, 0, st, src, dst, S, inv_scale_a, scale_b); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int Q>
static hipError_t launch_convert_q(int sa, int sb, const void* src, void* dst, uint32_t S,
                                   float inv_scale_a, float scale_b, hipStream_t st) {
  switch (sa) {
    case ST_F64: return launch_convert_a<Q, ST_F64>(sb, src, dst, S, inv_scale_a, scale_b, st);
    case ST_F32: return launch_convert_a<Q, ST_F32>(sb, src, dst, S, inv_scale_a, scale_b, st);
    case ST_F16DEV: return launch_convert_a<Q, ST_F16DEV>(sb, src, dst, S, inv_scale_a, scale_b, st);
    case ST_BF16DEV: return launch_convert_a<Q, ST_BF16DEV>(sb, src, dst, S, inv_scale_a, scale_b, st);
    case ST_F32DEV: return launch_convert_a<Q, ST_F32DEV>(sb, src, dst, S, inv_scale_a, scale_b, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_convert(int q, int sa, int sb, const void* src, void* dst, uint32_t S,
                          float inv_scale_a, float scale_b, hipStream_t st) {
  if (q == 19) return launch_convert_q<19>(sa, sb, src, dst, S, inv_scale_a, scale_b, st);
  return launch_convert_q<27>(sa, sb, src, dst, S, inv_scale_a, scale_b, st);
}

hipError_t launch_copy(void* dst, const void* src, uint64_t bytes, hipStream_t st) {
  const uint64_t n = bytes / 16;
  if (n == 0) return hipSuccess;
  const uint64_t blocks = (n + 255) / 256;
  if (blocks > 0x7fffffffull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, st, (const v4f*)src,
                     (v4f*)dst, n);
  return hipGetLastError();
}

}  // namespace lbm
