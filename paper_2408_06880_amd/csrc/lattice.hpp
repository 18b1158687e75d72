// Velocity sets, storage codecs and launch-argument types of the sparse AA
// lattice Boltzmann kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// ---------------------------------------------------------------------------
// D3Q19 / D3Q27 velocity sets: rest, then opposite pairs (axes, edges,
// corners).  Weights 1/3, 1/18, 1/36 (D3Q19) and 8/27, 2/27, 1/54, 1/216
// (D3Q27); speed of sound c_s^2 = 1/3 (Section "Lattice Boltzmann Method").
// ---------------------------------------------------------------------------
template <int Q>
struct Lattice;

template <>
struct Lattice<19> {
  static constexpr int cx[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  static constexpr int cy[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  static constexpr int cz[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
  static constexpr double w(int i) { return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }
};

template <>
struct Lattice<27> {
  static constexpr int cx[27] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1,
                                 -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1};
  static constexpr int cy[27] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0,
                                 0, 1, -1, 1, -1, 1, -1, 1, -1, -1, 1, 1, -1};
  static constexpr int cz[27] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1,
                                 1, 1, -1, -1, 1, 1, -1, -1, 1, 1, -1, 1, -1};
  static constexpr double w(int i) {
    return i == 0 ? 8.0 / 27.0 : (i <= 6 ? 2.0 / 27.0 : (i <= 18 ? 1.0 / 54.0 : 1.0 / 216.0));
  }
};

// Opposite direction: pairs are stored as (odd, even) neighbours.
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// ---------------------------------------------------------------------------
// Storage formats of the PDF-list.  load() returns the deviation
// d = f - w from the rest weight in the compute type R; store() encodes a
// deviation.  Deviation ("zero-centred") storage keeps the small signal
// (u ~ 1e-3 .. 1e-1, F ~ 1e-6) away from the O(w) offset, which is what lets
// 16-bit storage work at all.
// ---------------------------------------------------------------------------
enum StoreKind { ST_F64 = 0, ST_F32 = 1, ST_F16DEV = 2, ST_BF16DEV = 3, ST_F32DEV = 4 };

template <int S>
struct Store;

template <>
struct Store<ST_F64> {
  using T = double;
  using R = double;
  __device__ static R load(T v, R w, R) { return v - w; }
  __device__ static T store(R d, R w, R) { return w + d; }
};

template <>
struct Store<ST_F32> {
  using T = float;
  using R = float;
  __device__ static R load(T v, R w, R) { return v - w; }
  __device__ static T store(R d, R w, R) { return w + d; }
};

template <>
struct Store<ST_F32DEV> {
  using T = float;
  using R = float;
  __device__ static R load(T v, R, R) { return v; }
  __device__ static T store(R d, R, R) { return d; }
};

template <>
struct Store<ST_F16DEV> {
  using T = uint16_t;
  using R = float;
  // scale = 2^dev_exp (exact power of two); conversion rounds to nearest even.
  __device__ static R load(T v, R, R inv_scale) {
    return static_cast<float>(__builtin_bit_cast(_Float16, v)) * inv_scale;
  }
  __device__ static T store(R d, R, R scale) {
    return __builtin_bit_cast(uint16_t, static_cast<_Float16>(d * scale));
  }
};

template <>
struct Store<ST_BF16DEV> {
  using T = uint16_t;
  using R = float;
  __device__ static R load(T v, R, R inv_scale) {
    return __uint_as_float(static_cast<uint32_t>(v) << 16) * inv_scale;
  }
  // float -> bfloat16, round to nearest, ties to even (NaN kept quiet).
  __device__ static T store(R d, R, R scale) {
    uint32_t u = __float_as_uint(d * scale);
    if ((u & 0x7fffffffu) > 0x7f800000u) return static_cast<T>((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return static_cast<T>(u >> 16);
  }
};

// Velocity of a cell from its post-collision deviations d (natural order) at
// the current time, for the pressure outlet's anti-bounce-back: the
// half-force velocity u = (sum_i c_i d_i - F/2) / rho, in two parts: the
// sums m = (rho - 1, j) and the velocity from them.  The link update and
// the step kernels that hand the sums on use these same expressions, so the
// two routes give the same bits (the force is that of the step taken).
template <int Q, class R>
__device__ __forceinline__ void cell_sums(const R (&d)[Q], R (&m)[4]) {
  R drho = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    drho += d[j];
    jx += R(Lattice<Q>::cx[j]) * d[j];
    jy += R(Lattice<Q>::cy[j]) * d[j];
    jz += R(Lattice<Q>::cz[j]) * d[j];
  }
  m[0] = drho;
  m[1] = jx;
  m[2] = jy;
  m[3] = jz;
}

template <class R>
__device__ __forceinline__ void sums_velocity(const R (&m)[4], const double (&F)[3], R& ux,
                                              R& uy, R& uz) {
  const R r = R(1) + m[0];
  ux = (m[1] - R(0.5) * R(F[0])) / r;
  uy = (m[2] - R(0.5) * R(F[1])) / r;
  uz = (m[3] - R(0.5) * R(F[2])) / r;
}

// ---------------------------------------------------------------------------
// Launch arguments.  One launch advances one or more independent solves
// ("segments"); segment s owns workgroup tiles [tile0_s, tile0_{s+1}).  A
// single segment travels in the kernel arguments; a batch of several reads
// its table from device memory (a caller workspace written by a small
// kernel before the launches), so a launch carries a pointer, not the table.
// ---------------------------------------------------------------------------

// Compact index-list: tiles of kTile16 list positions.
constexpr uint32_t kTile16 = 256;
constexpr uint16_t kBounce16 = 0xFFFFu;  // upstream cell not fluid
constexpr uint16_t kEscape16 = 0xFFFEu;  // read the int32 index-list
constexpr uint32_t kMaxOff16 = 0xFFFDu;  // largest stored offset

// Step kernels: even, odd, two-array pull, pipelined odd (compact
// index-list), even with two cells per thread.
enum StepMode { MODE_EVEN = 0, MODE_ODD = 1, MODE_PULL = 2, MODE_ODD_PIPE = 3, MODE_EVEN2 = 4 };

// Index-list forms read by the odd step.
enum IndexForm { IDX_I32 = 0, IDX_16 = 1, IDX_RUN = 2 };
// Run-compressed index-list: groups of kRunWave list positions (one wave).
constexpr uint32_t kRunWave = 64;

// Link-velocity buffer of a solve with boundary links (parts 256-byte
// aligned): uint64 mask[W] (bit l of wave w: cell 64w + l has a link),
// uint32 woff[W + 1] (exclusive prefix of the mask popcounts), then four
// values of the compute type per marked cell, in list order: its sums
// (rho - 1, j) at the current time (8 bytes per value reserved).  Entry of cell k: woff[k/64] + popcount of the mask bits
// below k % 64.
__device__ __forceinline__ uint32_t link_entry(uint64_t m, uint32_t woff, uint32_t k) {
  const uint32_t b = k & (kRunWave - 1);
  return woff + (uint32_t)__builtin_popcountll(m & ((1ull << b) - 1ull));
}

struct Seg {
  void* pdf;               // PDF-list of this solve
  void* dst;               // pull scheme only: the second PDF-list written this step
  const int32_t* idx;      // index-list (odd steps), or null when off16 is set
  const uint16_t* off16;   // compact index-list offsets, or null
  const int32_t* base16;   // compact index-list tile bases
  const uint32_t* rvoff;   // run form: first value of each wave, or null
  const uint64_t* rmask;   // run form: run-start masks [wave][direction]
  const int32_t* rval;     // run form: run values
  const uint64_t* lmask;   // link velocities: cells with links, bit per lane [wave]
  const uint32_t* lwoff;   // link velocities: first entry of each wave
  void* lvel;              // link velocities: 4 sums (compute type) per entry
  uint32_t ntiles16;       // tiles of the compact index-list
  uint32_t S;              // stride
  uint32_t nf;             // fluid cells
  uint32_t tile0;          // first tile of this segment in the launch
  double om1;            // SRT omega / TRT omega+ / cumulant shear rate
  double om2;            // TRT omega- / cumulant bulk rate
  double F[3];           // body force
  double rates[4];       // MRT epsilon, pi, q, m rates
  float scale;           // 2^dev_exp (16-bit storage)
  float inv_scale;       // 2^-dev_exp
};

struct StepArgs {
  int32_t nseg;
  uint32_t ntiles;
  int32_t xcd_remap;
  int32_t pad;
  const Seg* segs;         // device table of nseg segments when nseg > 1
  Seg seg0;                // the segment when nseg == 1
};

// Global-memory pointers.  Pointers in kernel arguments are known to the
// compiler to address global memory; a pointer read from a device table (a
// batch's segment table) is generic to it, and generic pointers compile to
// flat loads and stores, which are slower.  Kernels convert every buffer
// pointer of a segment with gp() before using it.  (The host compilation
// pass sees the same source without the address space.)
#if defined(__HIP_DEVICE_COMPILE__)
#define LBM_GLOBAL __attribute__((address_space(1)))
#else
#define LBM_GLOBAL
#endif

template <class T>
__device__ __forceinline__ LBM_GLOBAL T* gp(T* p) {
  return (LBM_GLOBAL T*)p;
}
template <class T>
__device__ __forceinline__ const LBM_GLOBAL T* gp(const T* p) {
  return (const LBM_GLOBAL T*)p;
}

// Pull position of population i of cell k from the compact index-list
// (t16 = the cell's compact tile; tile bases are stored [tile][direction]).
__device__ __forceinline__ uint32_t pos16(const Seg& g, int q, int i, int oi, uint32_t k,
                                          uint32_t t16) {
  const uint16_t o = gp(g.off16)[(size_t)(i - 1) * g.S + k];
  const int32_t b = gp(g.base16)[(size_t)t16 * (q - 1) + (i - 1)];
  if (o >= kEscape16)
    return o == kBounce16 ? (uint32_t)oi * g.S + k
                          : (uint32_t)gp(g.idx)[(size_t)(i - 1) * g.S + k];
  return (uint32_t)i * g.S + k + (uint32_t)b + (uint32_t)o;
}

// XCD-aware tile order.  Workgroups are dispatched round-robin over the 8
// XCDs (workgroup v runs on XCD v % 8).  mode 0: tile v (dispatch order).
// mode 1: the workgroups of one XCD take one contiguous eighth of the
// tiles.  mode m >= 2: chunks of m consecutive tiles are dealt round-robin
// to the XCDs (chunk c of XCD x is tiles (8c + x) m .. (8c + x) m + m - 1);
// tiles past the last full round of 8 m map to themselves.  Chunks keep the
// neighbour gathers of the odd step (upstream rows a few hundred to a few
// thousand list positions away) inside one XCD's L2 while all XCDs sweep
// the arrays together; one eighth per XCD makes 8 separate sweeps of every
// direction block.  Every mode is a bijection of [0, n).
__device__ __forceinline__ uint32_t xcd_tile(uint32_t v, uint32_t n, int32_t mode) {
  if (mode <= 0) return v;
  const uint32_t x = v & 7u, local = v >> 3;
  if (mode == 1) {
    const uint32_t per = n >> 3, rem = n & 7u;
    return x * per + (x < rem ? x : rem) + local;
  }
  const uint32_t m = (uint32_t)mode, round = 8u * m, full = n / round;
  if (v >= full * round) return v;
  const uint32_t c = local / m, r = local - c * m;
  return (c * 8u + x) * m + r;
}

// Segment of a tile: the last segment whose first tile is not after it
// (binary search; first tiles do not decrease with the segment number).
__device__ __forceinline__ int seg_of(const StepArgs& a, uint32_t tile) {
  if (a.nseg == 1) return 0;
  int lo = 0, hi = a.nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.segs[mid].tile0 <= tile)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Calls f(segment that owns `tile`).  A single segment is read from the
// kernel arguments, one of several from the device table; the two calls are
// kept apart (rather than selecting between the two sources) so that the
// segment's fields load with scalar loads on both paths.
template <class F>
__device__ __forceinline__ void with_seg(const StepArgs& a, uint32_t tile, F&& f) {
  if (a.nseg == 1) {
    f(a.seg0);
  } else {
    const Seg g = a.segs[seg_of(a, tile)];
    f(g);
  }
}

// First tile and fluid cells of segment s.
__device__ __forceinline__ uint32_t seg_tile0(const StepArgs& a, int s) {
  return a.nseg == 1 ? a.seg0.tile0 : a.segs[s].tile0;
}
__device__ __forceinline__ uint32_t seg_nf(const StepArgs& a, int s) {
  return a.nseg == 1 ? a.seg0.nf : a.segs[s].nf;
}

}  // namespace lbm
