// Host-side launch entry points shared between the translation units of
// liblbm.so (not part of the public C-ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lattice.hpp"

namespace lbm {

// AA step kernels (step_q19.hip, step_q27.hip); mode 0 even, 1 odd, 2 pull
// (lds: dynamic LDS bytes reserved per workgroup, to cap residency; links:
// some solve of the launch has a link-velocity buffer)
hipError_t launch_aa_q19(int coll, int storage, int mode, int idx, const StepArgs& a,
                         int block, uint32_t lds, bool links, hipStream_t st);
hipError_t launch_aa_q27(int coll, int storage, int mode, int idx, const StepArgs& a,
                         int block, uint32_t lds, bool links, hipStream_t st);

// Boundary-class coefficients of one solve, precomputed on the host:
// for class c, type[c] in {0 noslip, 1 UBB, 2 pressure}; u[c][3]; rho[c].
// g describes the solve (buffers, index forms, force, 16-bit scale) for the
// gather of a cell's velocity; natural = 1 when the populations sit in
// their natural slots (even t of the AA pattern, every pull step);
// use_vel = 1 reads the velocity that the last step kernel wrote into the
// link-velocity buffer (g.lmask, g.lwoff, g.lvel) instead of gathering it.
struct LinkArgs {
  void* pdf;
  const int32_t* links;
  uint32_t n_links;
  int32_t q;
  int32_t n_classes;
  int32_t natural;
  int32_t use_vel;
  int32_t pad;
  int32_t type[8];
  double u[8][3];
  double rho[8];
  float scale, inv_scale;
  Seg g;
};

// aux.hip
hipError_t launch_init(int q, int storage, void* pdf, uint32_t S, uint32_t nf, double rho0,
                       const double u0[3], float scale, hipStream_t st);
hipError_t launch_links(int storage, const LinkArgs& a, hipStream_t st);
// Link-velocity buffer: mark the cells of the n links in mask (nw words,
// cleared first) and write their popcounts to woff[0..nw) (the caller scans
// them).
hipError_t launch_link_mask(const int32_t* links, uint32_t n_links, uint32_t S,
                            uint32_t nw, uint64_t* mask, uint32_t* woff, hipStream_t st);
hipError_t launch_moments(int q, int storage, const Seg& g, bool odd_t, bool out_f64, void* rho,
                          void* u, hipStream_t st);
// Reductions: first pass writes 5 doubles per tile of kRedBlock cells into
// partials (tiles of all segments in launch order); the second pass writes
// 8 doubles per segment into out.
constexpr int kRedBlock = 256;
hipError_t launch_reduce(int q, int storage, const StepArgs& a, bool odd_t, double* partials,
                         double* out, hipStream_t st);
hipError_t launch_copy(void* dst, const void* src, uint64_t bytes, hipStream_t st);
// Write n segments from host memory into the device table `dev` (stream
// ordered; kernel launches carrying at most kSegChunk segments each).
constexpr uint32_t kSegChunk = 16;
hipError_t launch_put_segs(const Seg* host, uint32_t n, Seg* dev, hipStream_t st);
// Storage conversion of a whole PDF-list (q * S slots), format sa -> sb.
hipError_t launch_convert(int q, int sa, int sb, const void* src, void* dst, uint32_t S,
                          float inv_scale_a, float scale_b, hipStream_t st);

// builder.hip
struct BuildArgs {
  const uint8_t* labels;
  int32_t nx, ny, nz;
  uint32_t periodic;
  int32_t q, order;
  uint32_t bits;        // Morton bits per axis (order == Morton)
  uint64_t n_codes;     // codes to scan (8^bits for Morton, nx*ny*nz for lex)
  uint32_t n_chunks;    // ceil(n_codes / kChunk)
};
constexpr int kBuildBlock = 256;
constexpr int kBlockYZ = 8;  // y and z edge of a block in the blocked order
constexpr int kCodesPerThread = 16;
constexpr uint32_t kChunk = kBuildBlock * kCodesPerThread;
// counts: uint32[2*(n_chunks+1)] (fluid cells, links per chunk -> exclusive
// offsets after the scan, totals at [n_chunks]).
hipError_t launch_build_count(const BuildArgs& b, uint32_t* counts, hipStream_t st);
hipError_t launch_build_scan(uint32_t n_chunks, uint32_t* counts, hipStream_t st);
// Exclusive prefix sum of v[0..n) in place, total at v[n] (one workgroup).
hipError_t launch_exclusive_scan(uint32_t n, uint32_t* v, hipStream_t st);
hipError_t launch_build_emit(const BuildArgs& b, const uint32_t* counts, uint32_t S,
                             uint32_t n_fluid, uint32_t n_links, int32_t* cells, int32_t* inv,
                             int32_t* links, hipStream_t st);
hipError_t launch_build_index(const BuildArgs& b, const int32_t* cells, const int32_t* inv,
                              uint32_t S, uint32_t n_fluid, int32_t* index, hipStream_t st);

// index16.hip: compact index-list from the int32 one; flags gets one word
// per tile plus the OR of all of them at [ntiles].
hipError_t launch_compress_index(int q, const int32_t* index, uint32_t S, uint32_t nf,
                                 uint32_t ntiles, uint16_t* off, int32_t* base, uint32_t* flags,
                                 hipStream_t st);

// runs.hip: run-compressed index-list.  mask: uint64[nw][q-1]; cnt:
// uint32[nw+1] (runs per wave, then the exclusive scan of it); val: int32
// per run.
hipError_t launch_runs_mask(int q, const int32_t* index, uint32_t S, uint32_t nw, uint64_t* mask,
                            uint32_t* cnt, hipStream_t st);
hipError_t launch_runs_emit(int q, const int32_t* index, uint32_t S, uint32_t nw,
                            const uint32_t* voff, int32_t* val, hipStream_t st);

// dense.hip
struct DenseArgs {
  void* pdf;
  const uint32_t* mask;
  int32_t nx, ny, nz;
  uint32_t periodic;
  uint32_t N;
  int32_t xcd_remap;
  uint32_t ntiles;
  int32_t pad;
  double om1, om2, F[3];
  double rates[4];
  float scale, inv_scale;
};
hipError_t launch_dense_mask(const uint8_t* labels, int nx, int ny, int nz, uint32_t periodic,
                             int q, uint32_t* mask, hipStream_t st);
hipError_t launch_dense_step(int q, int coll, int storage, bool odd, const DenseArgs& a,
                             int block, hipStream_t st);

}  // namespace lbm
