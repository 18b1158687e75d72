// C-ABI of liblbm.so: argument validation, launch planning and kernel
// dispatch.  No entry point allocates device memory; all buffers and the
// stream belong to the caller.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "internal.hpp"

using namespace lbm;

namespace {

thread_local std::string g_err;

lbm_status fail(lbm_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

lbm_status hip_fail(hipError_t e, const char* where) {
  return fail(LBM_EDEVICE, "%s: %s", where, hipGetErrorString(e));
}

#define HIP_TRY(expr, where)              \
  do {                                    \
    hipError_t e_ = (expr);               \
    if (e_ != hipSuccess) return hip_fail(e_, where); \
  } while (0)

// ------------------------------------------------------- launch table
constexpr uint32_t kLdsPerCu = 160u * 1024u;  // LDS bytes per CU (gfx950)
std::mutex g_launch_mu;
lbm_launch g_launch[3][2][5];  // kernel x (q19, q27) x storage
bool g_launch_init = false;

bool is16(int s);

void launch_defaults() {
  if (g_launch_init) return;
  // Measured on MI355X: the gather/scatter (odd) kernel gains from keeping
  // neighbouring tiles on one XCD; the streaming kernels do not.  The even
  // kernel takes two cells per thread for 16-bit storage (2-byte lanes),
  // one otherwise.  Fewer resident workgroups than registers allow stream
  // better for D3Q19 on the 256^3 packing (block 256): FP32 and FP32-dev
  // odd step at 4 per CU (FP32 360 -> 355 us), even step at 3 (FP32-dev
  // 262 -> 253 us); the FP64 even step with 64-thread workgroups, two cells
  // per thread and 2 per CU (565 -> 516 us at porosity 0.6, 3-4 % faster
  // than 256 threads at 2 per CU for porosities 0.4-0.95); 16-bit storage,
  // the FP64 odd step and the D3Q27 kernels run fastest uncapped.
  for (int k = 0; k < 3; ++k)
    for (int qi = 0; qi < 2; ++qi)
      for (int st = 0; st < 5; ++st) {
        lbm_launch& c = g_launch[k][qi][st];
        c.block = 256;
        // odd step: chunks of 16 tiles dealt round-robin to the XCDs
        // (FP64 638 -> 618 us, FP32 357 -> 342 us against one contiguous
        // eighth per XCD; chunks of 12-32 tiles measure the same); D3Q19
        // 16-bit storage: chunks of 256 (FP16-dev 230.0 -> 227.7 us,
        // BF16-dev 232.4 -> 229.6 us against 16)
        c.xcd_remap = (k == LBM_KERNEL_ODD) ? ((qi == 0 && is16(st)) ? 256 : 16) : 0;
        c.pipelined = 0;
        c.cells_per_thread = (k == LBM_KERNEL_EVEN && is16(st)) ? 2 : 1;
        c.max_groups_per_cu = 0;
        if (qi == 0 && (st == LBM_STORE_F32 || st == LBM_STORE_F32DEV))
          c.max_groups_per_cu = k == LBM_KERNEL_ODD ? 4 : (k == LBM_KERNEL_EVEN ? 3 : 0);
        // D3Q27 FP32 odd step: about 1 % faster at 3 per CU on both the
        // vessel tree and the packing (its even step depends on geometry)
        if (qi == 1 && (st == LBM_STORE_F32 || st == LBM_STORE_F32DEV) && k == LBM_KERNEL_ODD)
          c.max_groups_per_cu = 3;
        if (qi == 0 && st == LBM_STORE_F64 && k == LBM_KERNEL_EVEN) {
          c.block = 64;
          c.cells_per_thread = 2;
          c.max_groups_per_cu = 2;
        }
      }
  g_launch_init = true;
}

// Dynamic LDS per workgroup that lets at most n workgroups share a CU's
// 160 KB (the step kernels use no LDS): just over 160 KB / (n + 1), in
// 512-byte units; 0 for no cap.
uint32_t cap_lds_bytes(int n) {
  if (n <= 0) return 0;
  return (kLdsPerCu / (uint32_t)(n + 1) / 512u + 1u) * 512u;
}

lbm_launch get_cfg(int kernel, int q, int storage) {
  std::lock_guard<std::mutex> lk(g_launch_mu);
  launch_defaults();
  return g_launch[kernel][q == 27 ? 1 : 0][storage];
}

// ------------------------------------------------------- validation
bool storage_ok(int s) { return s >= LBM_STORE_F64 && s <= LBM_STORE_F32DEV; }
bool is16(int s) { return s == LBM_STORE_F16DEV || s == LBM_STORE_BF16DEV; }

lbm_status check_layout(const lbm_layout& L) {
  if (L.q != 19 && L.q != 27) return fail(LBM_EINVAL, "layout.q must be 19 or 27 (got %d)", L.q);
  if (L.n_fluid < 0 || L.stride < L.n_fluid || L.n_links < 0)
    return fail(LBM_EINVAL, "inconsistent layout sizes (n_fluid %lld, stride %lld)",
                (long long)L.n_fluid, (long long)L.stride);
  if ((int64_t)L.q * L.stride >= (int64_t)1 << 32)
    return fail(LBM_ERANGE, "q*stride = %lld does not fit 32-bit positions",
                (long long)L.q * L.stride);
  return LBM_OK;
}

lbm_status check_state(const lbm_state* s) {
  if (!s) return fail(LBM_EINVAL, "state is NULL");
  lbm_status rc = check_layout(s->layout);
  if (rc) return rc;
  if (!storage_ok(s->storage)) return fail(LBM_EINVAL, "unknown storage %d", s->storage);
  if (is16(s->storage) && (s->dev_exp < 0 || s->dev_exp > 24))
    return fail(LBM_EINVAL, "dev_exp must be in [0, 24] (got %d)", s->dev_exp);
  if (s->layout.n_fluid > 0 && !s->pdf) return fail(LBM_EINVAL, "state pdf pointer is NULL");
  if (s->layout.n_fluid > 0 && !s->index && !s->runs)
    return fail(LBM_EINVAL, "state needs an index-list (index or runs)");
  if (s->index16 && !s->index)
    return fail(LBM_EINVAL, "the compact index-list needs the int32 one for escaped entries");
  if (s->layout.n_links > 0 && !s->links)
    return fail(LBM_EINVAL, "state has %lld links but links is NULL", (long long)s->layout.n_links);
  if (s->t < 0) return fail(LBM_EINVAL, "state.t is negative");
  return LBM_OK;
}

lbm_status check_coll(const lbm_collision* c, int q) {
  if (!c) return fail(LBM_EINVAL, "collision is NULL");
  if (c->kind < LBM_COLL_NONE || c->kind > LBM_COLL_CM)
    return fail(LBM_EINVAL, "unknown collision kind %d", c->kind);
  if (c->kind != LBM_COLL_NONE && !(c->tau > 0.5))
    return fail(LBM_EINVAL, "tau must be > 1/2 (got %g)", c->tau);
  if (c->kind == LBM_COLL_TRT && !(c->magic > 0.0))
    return fail(LBM_EINVAL, "TRT magic parameter must be > 0 (got %g)", c->magic);
  if (c->kind == LBM_COLL_CUMULANT && q != 27)
    return fail(LBM_EINVAL, "the cumulant operator needs D3Q27");
  if ((c->kind == LBM_COLL_CUMULANT || c->kind == LBM_COLL_MRT || c->kind == LBM_COLL_CM) &&
      !(c->omega_bulk > 0.0 && c->omega_bulk < 2.0))
    return fail(LBM_EINVAL, "omega_bulk must be in (0, 2) (got %g)", c->omega_bulk);
  if (c->kind == LBM_COLL_MRT && q != 19)
    return fail(LBM_EINVAL, "the MRT operator needs D3Q19");
  if (c->kind == LBM_COLL_CM && q != 27)
    return fail(LBM_EINVAL, "the central-moment operator needs D3Q27");
  if (c->kind == LBM_COLL_MRT || c->kind == LBM_COLL_CM)
    for (int a = 0; a < 4; ++a)
      if (!(c->rates[a] > 0.0 && c->rates[a] < 2.0))
        return fail(LBM_EINVAL, "rates must be in (0, 2) (rates[%d] = %g)", a, c->rates[a]);
  for (int a = 0; a < 3; ++a)
    if (!isfinite(c->force[a])) return fail(LBM_EINVAL, "force must be finite");
  return LBM_OK;
}

void coll_rates(const lbm_collision* c, double& om1, double& om2, double* rates) {
  om1 = om2 = 0.0;
  const bool has_rates = c->kind == LBM_COLL_MRT || c->kind == LBM_COLL_CM;
  for (int a = 0; a < 4; ++a) rates[a] = has_rates ? c->rates[a] : 0.0;
  if (c->kind == LBM_COLL_SRT) {
    om1 = om2 = 1.0 / c->tau;
  } else if (c->kind == LBM_COLL_TRT) {
    om1 = 1.0 / c->tau;
    om2 = 1.0 / (0.5 + c->magic / (c->tau - 0.5));
  } else if (c->kind == LBM_COLL_CUMULANT || c->kind == LBM_COLL_MRT || c->kind == LBM_COLL_CM) {
    om1 = 1.0 / c->tau;
    om2 = c->omega_bulk;
  }
}

// Sub-buffers of a compact index-list of `layout` starting at `p`.
struct Index16View {
  uint16_t* off;
  int32_t* base;
  uint32_t* flags;
  uint32_t ntiles;
  uint64_t bytes;
};

uint64_t align256(uint64_t v) { return (v + 255) & ~(uint64_t)255; }

Index16View index16_view(const lbm_layout& L, const void* p) {
  Index16View v;
  const uint64_t S = (uint64_t)L.stride, qm = (uint64_t)(L.q - 1);
  v.ntiles = (uint32_t)((S + kTile16 - 1) / kTile16);
  const uint64_t off_b = align256(2 * qm * S);
  const uint64_t base_b = align256(4 * qm * v.ntiles);
  const uint64_t flag_b = align256(4 * ((uint64_t)v.ntiles + 1));
  v.bytes = off_b + base_b + flag_b;
  v.off = nullptr;
  v.base = nullptr;
  v.flags = nullptr;
  if (p) {
    char* c = (char*)p;
    v.off = (uint16_t*)c;
    v.base = (int32_t*)(c + off_b);
    v.flags = (uint32_t*)(c + off_b + base_b);
  }
  return v;
}

// Sub-buffers of a run-compressed index-list of `layout` starting at `p`.
struct RunsView {
  uint32_t* voff;
  uint64_t* mask;
  int32_t* val;
  uint32_t nw;
  uint64_t header;
};

RunsView runs_view(const lbm_layout& L, const void* p) {
  RunsView v;
  v.nw = (uint32_t)(((uint64_t)L.stride + kRunWave - 1) / kRunWave);
  const uint64_t voff_b = align256(4 * ((uint64_t)v.nw + 1));
  const uint64_t mask_b = align256(8 * (uint64_t)v.nw * (uint64_t)(L.q - 1));
  v.header = voff_b + mask_b;
  v.voff = nullptr;
  v.mask = nullptr;
  v.val = nullptr;
  if (p) {
    char* c = (char*)p;
    v.voff = (uint32_t*)c;
    v.mask = (uint64_t*)(c + voff_b);
    v.val = (int32_t*)(c + v.header);
  }
  return v;
}

// Sub-buffers of a link-velocity buffer of `layout` starting at `p`.
struct LinkVelView {
  uint64_t* mask;
  uint32_t* woff;
  void* vel;
  uint32_t nw;
  uint64_t bytes;
};

LinkVelView link_vel_view(const lbm_layout& L, void* p) {
  LinkVelView v;
  v.nw = (uint32_t)(((uint64_t)L.stride + kRunWave - 1) / kRunWave);
  const uint64_t mask_b = align256(8 * (uint64_t)v.nw);
  const uint64_t woff_b = align256(4 * ((uint64_t)v.nw + 1));
  v.bytes = mask_b + woff_b + align256(4 * 8 * (uint64_t)L.n_links);
  v.mask = nullptr;
  v.woff = nullptr;
  v.vel = nullptr;
  if (p) {
    char* c = (char*)p;
    v.mask = (uint64_t*)c;
    v.woff = (uint32_t*)(c + mask_b);
    v.vel = c + mask_b + woff_b;
  }
  return v;
}

// Index form the odd step reads for a state: runs, else compact, else int32.
int index_form(const lbm_state* s) {
  return s->runs ? IDX_RUN : (s->index16 ? IDX_16 : IDX_I32);
}

Seg make_seg(const lbm_state* s, const lbm_collision* c) {
  Seg g;
  memset(&g, 0, sizeof(g));
  g.pdf = s->pdf;
  g.idx = s->index;
  g.S = (uint32_t)s->layout.stride;
  g.nf = (uint32_t)s->layout.n_fluid;
  if (s->index16) {
    Index16View v = index16_view(s->layout, s->index16);
    g.off16 = v.off;
    g.base16 = v.base;
    g.ntiles16 = v.ntiles;
  }
  if (s->runs) {
    RunsView r = runs_view(s->layout, s->runs);
    g.rvoff = r.voff;
    g.rmask = r.mask;
    g.rval = r.val;
  }
  if (s->link_vel && s->layout.n_links > 0) {
    LinkVelView v = link_vel_view(s->layout, s->link_vel);
    g.lmask = v.mask;
    g.lwoff = v.woff;
    g.lvel = v.vel;
  }
  if (c) {
    coll_rates(c, g.om1, g.om2, g.rates);
    for (int a = 0; a < 3; ++a) g.F[a] = c->force[a];
  }
  const int e = is16(s->storage) ? s->dev_exp : 0;
  g.scale = ldexpf(1.0f, e);
  g.inv_scale = ldexpf(1.0f, -e);
  return g;
}

// Boundary links of one state before a step.  natural: the populations sit
// in their natural slots (AA at even t, every pull step); the pressure rule
// reads the cell's velocity from them (coll supplies the force), or from the
// state's link-velocity buffer when a step kernel filled it at this t.
lbm_status link_update(const lbm_state* s, const lbm_collision* c, const lbm_bspec* bs,
                       bool natural, hipStream_t st) {
  if (s->layout.n_links == 0) return LBM_OK;
  LinkArgs la;
  memset(&la, 0, sizeof(la));
  la.g = make_seg(s, c);
  la.natural = natural ? 1 : 0;
  la.use_vel = (la.g.lmask && s->link_vel_t == s->t) ? 1 : 0;
  la.pdf = s->pdf;
  la.links = s->links;
  la.n_links = (uint32_t)s->layout.n_links;
  la.q = s->layout.q;
  la.n_classes = bs ? bs->n_classes : 0;
  if (la.n_classes < 0 || la.n_classes > 8)
    return fail(LBM_EINVAL, "bspec.n_classes must be in [0, 8]");
  for (int c = 0; c < la.n_classes; ++c) {
    const int ty = bs->cls[c].type;
    if (ty < LBM_BC_NOSLIP || ty > LBM_BC_PRESSURE)
      return fail(LBM_EINVAL, "unknown boundary type %d in class %d", ty, c);
    la.type[c] = ty;
    for (int a = 0; a < 3; ++a) la.u[c][a] = bs->cls[c].u[a];
    la.rho[c] = bs->cls[c].rho;
  }
  const int e = is16(s->storage) ? s->dev_exp : 0;
  la.scale = ldexpf(1.0f, e);
  la.inv_scale = ldexpf(1.0f, -e);
  HIP_TRY(launch_links(s->storage, la, st), "link update");
  return LBM_OK;
}

hipError_t launch_aa(int q, int coll, int storage, int mode, int idx, const StepArgs& a,
                     const lbm_launch& cfg, bool links, hipStream_t st) {
  const uint32_t lds = cap_lds_bytes(cfg.max_groups_per_cu);
  if (q == 19) return launch_aa_q19(coll, storage, mode, idx, a, cfg.block, lds, links, st);
  return launch_aa_q27(coll, storage, mode, idx, a, cfg.block, lds, links, st);
}

uint32_t ceil_div(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

}  // namespace

extern "C" {

int32_t lbm_abi_version(void) { return 7; }

const char* lbm_last_error(void) { return g_err.c_str(); }

lbm_status lbm_set_launch(int32_t kernel, int32_t q, int32_t storage, const lbm_launch* cfg) {
  if (kernel < 0 || kernel > 2 || (q != 19 && q != 27) || !storage_ok(storage) || !cfg)
    return fail(LBM_EINVAL, "lbm_set_launch: bad kernel/q/storage");
  if (cfg->block != 64 && cfg->block != 128 && cfg->block != 256)
    return fail(LBM_EINVAL, "block must be 64, 128 or 256 (got %d)", cfg->block);
  if (cfg->xcd_remap < 0 || cfg->xcd_remap > 65536)
    return fail(LBM_EINVAL, "xcd_remap must be in [0, 65536] (got %d)", cfg->xcd_remap);
  if (cfg->pipelined != 0 && (cfg->pipelined != 1 || kernel != LBM_KERNEL_ODD || cfg->block != 256))
    return fail(LBM_EINVAL, "pipelined applies to the odd kernel with block 256 only");
  if (cfg->cells_per_thread < 0 || cfg->cells_per_thread > 2 ||
      (cfg->cells_per_thread == 2 && kernel != LBM_KERNEL_EVEN))
    return fail(LBM_EINVAL, "cells_per_thread must be 0, 1, or 2 for the even kernel (got %d)",
                cfg->cells_per_thread);
  if (cfg->max_groups_per_cu != 0 &&
      (cfg->max_groups_per_cu < 2 || cfg->max_groups_per_cu > 16 ||
       kernel == LBM_KERNEL_DENSE || cfg->pipelined))
    return fail(LBM_EINVAL,
                "max_groups_per_cu must be 0, or 2..16 for the sparse step kernels (got %d)",
                cfg->max_groups_per_cu);
  std::lock_guard<std::mutex> lk(g_launch_mu);
  launch_defaults();
  g_launch[kernel][q == 27 ? 1 : 0][storage] = *cfg;
  return LBM_OK;
}

lbm_status lbm_get_launch(int32_t kernel, int32_t q, int32_t storage, lbm_launch* cfg) {
  if (kernel < 0 || kernel > 2 || (q != 19 && q != 27) || !storage_ok(storage) || !cfg)
    return fail(LBM_EINVAL, "lbm_get_launch: bad kernel/q/storage");
  *cfg = get_cfg(kernel, q, storage);
  return LBM_OK;
}

// ------------------------------------------------------------ builder
static bool build_dims_ok(int32_t nx, int32_t ny, int32_t nz) {
  return nx >= 1 && ny >= 1 && nz >= 1 && nx <= 1024 && ny <= 1024 && nz <= 1024;
}

static void build_plan(int32_t nx, int32_t ny, int32_t nz, int32_t order, uint32_t& bits,
                       uint64_t& n_codes, uint32_t& n_chunks) {
  const int32_t m = nx > ny ? (nx > nz ? nx : nz) : (ny > nz ? ny : nz);
  bits = 0;
  if (order == LBM_ORDER_BLOCKED) {
    const int32_t by = (ny + kBlockYZ - 1) / kBlockYZ, bz = (nz + kBlockYZ - 1) / kBlockYZ;
    const int32_t mb = by > bz ? by : bz;
    while ((1 << bits) < mb) ++bits;
    n_codes = ((uint64_t)1 << (2 * bits)) * (uint64_t)nx * (kBlockYZ * kBlockYZ);
  } else {
    while ((1 << bits) < m) ++bits;
    n_codes = order == LBM_ORDER_MORTON ? (uint64_t)1 << (3 * bits) : (uint64_t)nx * ny * nz;
  }
  n_chunks = ceil_div(n_codes, kChunk);
}

uint64_t lbm_build_workspace_bytes(int32_t nx, int32_t ny, int32_t nz, int32_t order) {
  if (!build_dims_ok(nx, ny, nz) || order < 0 || order > 2) return 0;
  uint32_t bits, n_chunks;
  uint64_t n_codes;
  build_plan(nx, ny, nz, order, bits, n_codes, n_chunks);
  return align256((uint64_t)8 * (n_chunks + 1)) + (uint64_t)4 * nx * ny * nz;
}

lbm_status lbm_build_sparse(const uint8_t* labels, int32_t nx, int32_t ny, int32_t nz,
                            uint32_t periodic, int32_t q, int32_t order, int32_t align,
                            void* workspace, lbm_layout* layout, int32_t* cells, int32_t* index,
                            int32_t* links, void* stream) {
  if (!labels || !workspace || !layout) return fail(LBM_EINVAL, "labels/workspace/layout is NULL");
  if (!build_dims_ok(nx, ny, nz)) return fail(LBM_EINVAL, "box sizes must be in [1, 1024]");
  if (q != 19 && q != 27) return fail(LBM_EINVAL, "q must be 19 or 27");
  if (order < LBM_ORDER_MORTON || order > LBM_ORDER_BLOCKED) return fail(LBM_EINVAL, "bad order");
  if (align < 1) return fail(LBM_EINVAL, "align must be >= 1");
  if (periodic > 7u) return fail(LBM_EINVAL, "periodic must be a 3-bit mask");
  hipStream_t st = (hipStream_t)stream;
  BuildArgs b;
  b.labels = labels;
  b.nx = nx;
  b.ny = ny;
  b.nz = nz;
  b.periodic = periodic;
  b.q = q;
  b.order = order;
  build_plan(nx, ny, nz, order, b.bits, b.n_codes, b.n_chunks);
  uint32_t* counts = (uint32_t*)workspace;
  int32_t* inv = (int32_t*)((char*)workspace + align256((uint64_t)8 * (b.n_chunks + 1)));
  HIP_TRY(launch_build_count(b, counts, st), "build count");
  HIP_TRY(launch_build_scan(b.n_chunks, counts, st), "build scan");
  if (!cells) {
    if (index || links) return fail(LBM_EINVAL, "plan call: index and links must be NULL");
    uint32_t tot[2];
    HIP_TRY(hipMemcpyAsync(&tot[0], counts + b.n_chunks, 4, hipMemcpyDeviceToHost, st), "plan copy");
    HIP_TRY(hipMemcpyAsync(&tot[1], counts + 2 * b.n_chunks + 1, 4, hipMemcpyDeviceToHost, st),
            "plan copy");
    HIP_TRY(hipStreamSynchronize(st), "plan sync");
    lbm_layout L;
    memset(&L, 0, sizeof(L));
    L.nx = nx;
    L.ny = ny;
    L.nz = nz;
    L.periodic = periodic;
    L.q = q;
    L.order = order;
    L.align = align;
    L.n_fluid = tot[0];
    L.stride = ((L.n_fluid + align - 1) / align) * align;
    L.n_links = tot[1];
    *layout = L;
    return check_layout(L);
  }
  const lbm_layout& L = *layout;
  if (L.nx != nx || L.ny != ny || L.nz != nz || L.q != q || L.order != order ||
      L.periodic != periodic || L.align != align)
    return fail(LBM_ESTATE, "fill call: layout does not match the arguments");
  lbm_status rc = check_layout(L);
  if (rc) return rc;
  if (!index) return fail(LBM_EINVAL, "fill call: index is NULL");
  if (L.n_links > 0 && !links) return fail(LBM_EINVAL, "fill call: links is NULL");
  HIP_TRY(launch_build_emit(b, counts, (uint32_t)L.stride, (uint32_t)L.n_fluid,
                            (uint32_t)L.n_links, cells, inv, links, st),
          "build emit");
  HIP_TRY(launch_build_index(b, cells, inv, (uint32_t)L.stride, (uint32_t)L.n_fluid, index, st),
          "build index");
  return LBM_OK;
}

// ------------------------------------------------ compact index-list
uint64_t lbm_index16_bytes(const lbm_layout* L) {
  if (!L || (L->q != 19 && L->q != 27) || L->stride < 0) return 0;
  return index16_view(*L, nullptr).bytes;
}

lbm_status lbm_compress_index(const lbm_layout* L, const int32_t* index, void* index16,
                              uint64_t* n_escaped, void* stream) {
  if (!L || !index || !index16) return fail(LBM_EINVAL, "layout/index/index16 is NULL");
  lbm_status rc = check_layout(*L);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  Index16View v = index16_view(*L, index16);
  HIP_TRY(launch_compress_index(L->q, index, (uint32_t)L->stride, (uint32_t)L->n_fluid, v.ntiles,
                                v.off, v.base, v.flags, st),
          "compress index");
  uint32_t esc = 0;
  HIP_TRY(hipMemcpyAsync(&esc, v.flags + v.ntiles, 4, hipMemcpyDeviceToHost, st), "index16 count");
  HIP_TRY(hipStreamSynchronize(st), "index16 sync");
  if (n_escaped) *n_escaped = esc;
  return LBM_OK;
}

// ------------------------------------------------ link-velocity buffer
uint64_t lbm_link_vel_bytes(const lbm_layout* L) {
  if (!L || (L->q != 19 && L->q != 27) || L->stride < 0 || L->n_links <= 0) return 0;
  return link_vel_view(*L, nullptr).bytes;
}

lbm_status lbm_link_vel_prepare(const lbm_layout* L, const int32_t* links, void* link_vel,
                                void* stream) {
  if (!L) return fail(LBM_EINVAL, "layout is NULL");
  lbm_status rc = check_layout(*L);
  if (rc) return rc;
  if (L->n_links == 0) return LBM_OK;
  if (!links || !link_vel) return fail(LBM_EINVAL, "links/link_vel is NULL");
  if (L->n_links > 0xffffffffll) return fail(LBM_ERANGE, "too many links");
  LinkVelView v = link_vel_view(*L, link_vel);
  if (v.nw == 0) return LBM_OK;
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(launch_link_mask(links, (uint32_t)L->n_links, (uint32_t)L->stride, v.nw, v.mask, v.woff,
                           st),
          "link cells");
  HIP_TRY(launch_exclusive_scan(v.nw, v.woff, st), "link entries");
  return LBM_OK;
}

// ------------------------------------------- run-compressed index-list
uint64_t lbm_runs_header_bytes(const lbm_layout* L) {
  if (!L || (L->q != 19 && L->q != 27) || L->stride < 0) return 0;
  return runs_view(*L, nullptr).header;
}

lbm_status lbm_compress_runs(const lbm_layout* L, const int32_t* index, void* runs,
                             uint64_t capacity, uint64_t* needed, void* stream) {
  if (!L || !index || !runs || !needed) return fail(LBM_EINVAL, "layout/index/runs/needed is NULL");
  lbm_status rc = check_layout(*L);
  if (rc) return rc;
  RunsView v = runs_view(*L, runs);
  if (capacity < v.header) {
    *needed = v.header;
    return fail(LBM_ENOMEM, "runs buffer of %llu bytes is below the header size %llu",
                (unsigned long long)capacity, (unsigned long long)v.header);
  }
  hipStream_t st = (hipStream_t)stream;
  const uint32_t S = (uint32_t)L->stride;
  uint32_t total = 0;
  if (v.nw > 0) {
    HIP_TRY(launch_runs_mask(L->q, index, S, v.nw, v.mask, v.voff, st), "run masks");
    HIP_TRY(launch_exclusive_scan(v.nw, v.voff, st), "run offsets");
    HIP_TRY(hipMemcpyAsync(&total, v.voff + v.nw, 4, hipMemcpyDeviceToHost, st), "run count");
    HIP_TRY(hipStreamSynchronize(st), "run count sync");
  } else {
    HIP_TRY(hipMemsetAsync(v.voff, 0, 4, st), "run offsets");
    HIP_TRY(hipStreamSynchronize(st), "run offsets sync");
  }
  *needed = v.header + 4 * (uint64_t)total;
  if (capacity < *needed)
    return fail(LBM_ENOMEM, "runs form needs %llu bytes (capacity %llu)",
                (unsigned long long)*needed, (unsigned long long)capacity);
  if (v.nw > 0) {
    HIP_TRY(launch_runs_emit(L->q, index, S, v.nw, v.voff, v.val, st), "run values");
    HIP_TRY(hipStreamSynchronize(st), "run values sync");
  }
  return LBM_OK;
}

// ------------------------------------------------------ storage change
lbm_status lbm_convert(const lbm_state* src, lbm_state* dst, void* stream) {
  lbm_status rc = check_state(src);
  if (rc) return rc;
  if (!dst) return fail(LBM_EINVAL, "dst is NULL");
  if (!storage_ok(dst->storage)) return fail(LBM_EINVAL, "unknown storage %d", dst->storage);
  if (is16(dst->storage) && (dst->dev_exp < 0 || dst->dev_exp > 24))
    return fail(LBM_EINVAL, "dev_exp must be in [0, 24] (got %d)", dst->dev_exp);
  if (dst->layout.q != src->layout.q || dst->layout.stride != src->layout.stride ||
      dst->layout.n_fluid != src->layout.n_fluid)
    return fail(LBM_EINVAL, "src and dst layouts differ");
  if (src->layout.stride > 0 && !dst->pdf) return fail(LBM_EINVAL, "dst pdf is NULL");
  if (src->layout.stride > 0 && dst->pdf == src->pdf)
    return fail(LBM_EINVAL, "src and dst must not share the PDF-list");
  const int ea = is16(src->storage) ? src->dev_exp : 0;
  const int eb = is16(dst->storage) ? dst->dev_exp : 0;
  HIP_TRY(launch_convert(src->layout.q, src->storage, dst->storage, src->pdf, dst->pdf,
                         (uint32_t)src->layout.stride, ldexpf(1.0f, -ea), ldexpf(1.0f, eb),
                         (hipStream_t)stream),
          "convert");
  dst->t = src->t;
  dst->link_vel_t = -1;
  return LBM_OK;
}

// ---------------------------------------------------------- stepping
lbm_status lbm_init_equilibrium(lbm_state* s, double rho0, const double* u0, void* stream) {
  lbm_status rc = check_state(s);
  if (rc) return rc;
  if (!u0 || !(rho0 > 0.0)) return fail(LBM_EINVAL, "rho0 must be > 0 and u0 non-NULL");
  const int e = is16(s->storage) ? s->dev_exp : 0;
  if (s->layout.stride > 0)
    HIP_TRY(launch_init(s->layout.q, s->storage, s->pdf, (uint32_t)s->layout.stride,
                        (uint32_t)s->layout.n_fluid, rho0, u0, ldexpf(1.0f, e),
                        (hipStream_t)stream),
            "init");
  s->t = 0;
  s->link_vel_t = -1;
  return LBM_OK;
}

// One launch group of a step: the segments [first, first + nseg) of the
// call's segment list, all read through one kernel (index form, mode).
struct LaunchGroup {
  int mode, form;
  uint32_t first, nseg, ntiles;
  bool links;  // some segment has a link-velocity buffer
};

static uint64_t seg_table_bytes(int64_t n) { return align256((uint64_t)n * sizeof(Seg)); }

// Advance n states by n_steps AA steps.  The segment lists of both parities
// are planned once per call; when a launch covers several states their table
// is written once into `table` (device, room for 2n segments) before the
// first step.
static lbm_status step_group(lbm_state* const* states, const lbm_collision* const* colls,
                             const lbm_bspec* const* bspecs, int32_t n, int32_t n_steps,
                             Seg* table, hipStream_t st) {
  const int q = states[0]->layout.q, storage = states[0]->storage;
  const int kind = colls[0]->kind;
  if (n_steps == 0) return LBM_OK;
  const lbm_launch cfg_odd = get_cfg(LBM_KERNEL_ODD, q, storage);
  lbm_launch cfg_even = get_cfg(LBM_KERNEL_EVEN, q, storage);
  // Two cells per thread need an even stride: the 2-wide accesses stay
  // aligned and the second cell of the last pair is a padding slot.
  bool even_strides = true;
  for (int32_t j = 0; j < n; ++j) even_strides = even_strides && (states[j]->layout.stride % 2 == 0);
  const uint32_t cpt = (cfg_even.cells_per_thread == 2 && even_strides) ? 2 : 1;
  // a residency cap chosen for the two-cell kernel does not carry over to
  // its one-cell fallback
  if (cfg_even.cells_per_thread == 2 && cpt == 1) cfg_even.max_groups_per_cu = 0;

  std::vector<Seg> segs;
  segs.reserve(2 * (size_t)n);
  std::vector<LaunchGroup> odd_groups, even_groups;
  // Odd steps run one launch per index form, each form being a kernel of
  // its own; even steps never read indices.
  for (int form = IDX_I32; form <= IDX_RUN; ++form) {
    LaunchGroup gr{form == IDX_16 && cfg_odd.pipelined == 1 ? MODE_ODD_PIPE : MODE_ODD, form,
                   (uint32_t)segs.size(), 0, 0, false};
    for (int32_t j = 0; j < n; ++j) {
      if (states[j]->layout.n_fluid == 0 || index_form(states[j]) != form) continue;
      Seg g = make_seg(states[j], colls[j]);
      g.tile0 = gr.ntiles;
      gr.ntiles += ceil_div(g.nf, (uint64_t)cfg_odd.block);
      gr.links = gr.links || g.lmask != nullptr;
      segs.push_back(g);
      gr.nseg += 1;
    }
    if (gr.nseg > 0) odd_groups.push_back(gr);
  }
  {
    LaunchGroup gr{cpt == 2 ? MODE_EVEN2 : MODE_EVEN, IDX_I32, (uint32_t)segs.size(), 0, 0, false};
    for (int32_t j = 0; j < n; ++j) {
      if (states[j]->layout.n_fluid == 0) continue;
      Seg g = make_seg(states[j], colls[j]);
      g.tile0 = gr.ntiles;
      gr.ntiles += ceil_div(g.nf, (uint64_t)cfg_even.block * cpt);
      gr.links = gr.links || g.lmask != nullptr;
      segs.push_back(g);
      gr.nseg += 1;
    }
    if (gr.nseg > 0) even_groups.push_back(gr);
  }
  bool need_table = false;
  for (const auto& gr : odd_groups) need_table = need_table || gr.nseg > 1;
  for (const auto& gr : even_groups) need_table = need_table || gr.nseg > 1;
  if (need_table) {
    if (!table) return fail(LBM_EINVAL, "a batch of several solves needs a workspace");
    HIP_TRY(launch_put_segs(segs.data(), (uint32_t)segs.size(), table, st), "segment table");
  }

  for (int32_t step = 0; step < n_steps; ++step) {
    const bool odd = (states[0]->t & 1) == 0;
    const lbm_launch& cfg = odd ? cfg_odd : cfg_even;
    for (int32_t j = 0; j < n; ++j) {
      lbm_status rc = link_update(states[j], colls[j], bspecs ? bspecs[j] : nullptr,
                                  (states[j]->t & 1) == 0, st);
      if (rc) return rc;
    }
    for (const LaunchGroup& gr : odd ? odd_groups : even_groups) {
      StepArgs a;
      memset(&a, 0, sizeof(a));
      a.xcd_remap = cfg.xcd_remap;
      a.nseg = (int32_t)gr.nseg;
      a.ntiles = gr.ntiles;
      if (gr.nseg == 1)
        a.seg0 = segs[gr.first];
      else
        a.segs = table + gr.first;
      HIP_TRY(launch_aa(q, kind, storage, gr.mode, gr.form, a, cfg, gr.links, st), "AA step");
    }
    // the step kernels wrote the velocities of the cells with links
    for (int32_t j = 0; j < n; ++j) {
      states[j]->t += 1;
      states[j]->link_vel_t = states[j]->link_vel ? states[j]->t : -1;
    }
  }
  return LBM_OK;
}

lbm_status lbm_step(lbm_state* s, int32_t n_steps, const lbm_collision* c, const lbm_bspec* bs,
                    void* stream) {
  lbm_status rc = check_state(s);
  if (rc) return rc;
  rc = check_coll(c, s->layout.q);
  if (rc) return rc;
  if (n_steps < 0) return fail(LBM_EINVAL, "n_steps must be >= 0");
  lbm_state* arr[1] = {s};
  const lbm_collision* carr[1] = {c};
  const lbm_bspec* barr[1] = {bs};
  return step_group(arr, carr, barr, 1, n_steps, nullptr, (hipStream_t)stream);
}

lbm_status lbm_step_pull(lbm_state* s, void** spare, int32_t n_steps, const lbm_collision* c,
                         const lbm_bspec* bs, void* stream) {
  lbm_status rc = check_state(s);
  if (rc) return rc;
  rc = check_coll(c, s->layout.q);
  if (rc) return rc;
  if (!spare || (s->layout.n_fluid > 0 && !*spare))
    return fail(LBM_EINVAL, "pull step needs a second PDF-list");
  if (n_steps < 0 || (n_steps & 1)) return fail(LBM_EINVAL, "n_steps must be even and >= 0");
  if (s->t & 1) return fail(LBM_ESTATE, "pull steps need the natural slot layout (even t)");
  hipStream_t st = (hipStream_t)stream;
  // the odd kernel's workgroup size and tile order; no residency cap (the
  // caps were measured for the AA kernels)
  lbm_launch cfg = get_cfg(LBM_KERNEL_ODD, s->layout.q, s->storage);
  cfg.max_groups_per_cu = 0;
  // the pull kernel reads the compact or the int32 index-list
  if (s->layout.n_fluid > 0 && !s->index)
    return fail(LBM_EINVAL, "pull steps need the int32 index-list");
  const int idx = s->index16 ? IDX_16 : IDX_I32;
  for (int32_t step = 0; step < n_steps; ++step) {
    rc = link_update(s, c, bs, true, st);
    if (rc) return rc;
    if (s->layout.n_fluid > 0) {
      StepArgs a;
      memset(&a, 0, sizeof(a));
      a.xcd_remap = cfg.xcd_remap;
      Seg g = make_seg(s, c);
      g.dst = *spare;
      g.tile0 = 0;
      a.seg0 = g;
      a.nseg = 1;
      a.ntiles = ceil_div(g.nf, (uint64_t)cfg.block);
      HIP_TRY(launch_aa(s->layout.q, c->kind, s->storage, MODE_PULL, idx, a, cfg, true, st),
              "pull step");
      void* tmp = s->pdf;
      s->pdf = *spare;
      *spare = tmp;
    }
    s->t += 1;
    s->link_vel_t = s->link_vel ? s->t : -1;
  }
  return LBM_OK;
}

uint64_t lbm_step_batch_workspace_bytes(int32_t n_states) {
  if (n_states < 1) return 0;
  return 2 * seg_table_bytes(n_states);
}

// Arguments of a batched step (both batch entry points).
static lbm_status check_batch(lbm_state* const* states, const lbm_collision* const* colls,
                              int32_t n, int32_t n_steps) {
  if (!states || !colls || n < 1) return fail(LBM_EINVAL, "lbm_step_batch: empty batch");
  if (n_steps < 0) return fail(LBM_EINVAL, "n_steps must be >= 0");
  for (int32_t j = 0; j < n; ++j) {
    lbm_status rc = check_state(states[j]);
    if (rc) return rc;
    rc = check_coll(colls[j], states[j]->layout.q);
    if (rc) return rc;
    if (states[j]->layout.q != states[0]->layout.q || states[j]->storage != states[0]->storage ||
        ((states[j]->t ^ states[0]->t) & 1) || colls[j]->kind != colls[0]->kind)
      return fail(LBM_ESTATE, "batch member %d differs in q, storage, parity or collision kind", j);
  }
  return LBM_OK;
}

lbm_status lbm_step_batch(lbm_state* const* states, const lbm_collision* const* colls,
                          const lbm_bspec* const* bspecs, int32_t n, int32_t n_steps,
                          void* workspace, uint64_t workspace_bytes, void* stream) {
  lbm_status rc = check_batch(states, colls, n, n_steps);
  if (rc) return rc;
  if (n > 1) {
    if (!workspace) return fail(LBM_EINVAL, "workspace is NULL");
    if (workspace_bytes < lbm_step_batch_workspace_bytes(n))
      return fail(LBM_ENOMEM, "workspace of %llu bytes is below the %llu bytes %d states need",
                  (unsigned long long)workspace_bytes,
                  (unsigned long long)lbm_step_batch_workspace_bytes(n), n);
  }
  return step_group(states, colls, bspecs, n, n_steps, (Seg*)workspace, (hipStream_t)stream);
}

// ------------------------------------------- batch without allocation
// Segment tables of lbm_step_batch_noalloc: room for
// LBM_STEP_BATCH_NOALLOC_MAX states, one copy per device, held until the
// process ends.  Host code must not pass `scratch` itself to a kernel (in
// host code the name stands for a host-side shadow, not the device
// address); it uses the address hipGetSymbolAddress returns for the device.
constexpr uint64_t kScratchBytes =
    2 * (((uint64_t)LBM_STEP_BATCH_NOALLOC_MAX * sizeof(Seg) + 255) / 256 * 256);
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};
}  // namespace

// Device address of this device's `scratch`, looked up once per device
// (with that device current) and kept.  The stream must belong to the
// current device.
static lbm_status scratch_table(hipStream_t st, void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(LBM_EINVAL, "device %d out of range", dev);
  if (st) {
    hipDevice_t sd = 0;
    HIP_TRY(hipStreamGetDevice(st, &sd), "hipStreamGetDevice");
    if ((int)sd != dev)
      return fail(LBM_EINVAL, "the stream belongs to device %d, the current device is %d",
                  (int)sd, dev);
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return LBM_OK;
}

lbm_status lbm_step_batch_noalloc(lbm_state* const* states, const lbm_collision* const* colls,
                                  const lbm_bspec* const* bspecs, int32_t n, int32_t n_steps,
                                  void* stream) {
  if (n > LBM_STEP_BATCH_NOALLOC_MAX)
    return fail(LBM_ENOMEM, "lbm_step_batch_noalloc takes at most %d states (got %d)",
                LBM_STEP_BATCH_NOALLOC_MAX, n);
  static_assert(2 * LBM_STEP_BATCH_NOALLOC_MAX * sizeof(Seg) <= kScratchBytes,
                "scratch holds the segment tables of both parities");
  lbm_status rc = check_batch(states, colls, n, n_steps);
  if (rc) return rc;
  void* table = nullptr;
  if (n > 1 && n_steps > 0) {
    rc = scratch_table((hipStream_t)stream, &table);
    if (rc) return rc;
  }
  return step_group(states, colls, bspecs, n, n_steps, (Seg*)table, (hipStream_t)stream);
}

lbm_status lbm_moments(const lbm_state* s, const lbm_collision* c, int32_t out_f64, void* rho,
                       void* u, void* stream) {
  lbm_status rc = check_state(s);
  if (rc) return rc;
  rc = check_coll(c, s->layout.q);
  if (rc) return rc;
  if (s->layout.n_fluid > 0 && (!rho || !u)) return fail(LBM_EINVAL, "rho/u is NULL");
  Seg g = make_seg(s, c);
  HIP_TRY(launch_moments(s->layout.q, s->storage, g, (s->t & 1) != 0, out_f64 != 0, rho, u,
                         (hipStream_t)stream),
          "moments");
  return LBM_OK;
}

uint64_t lbm_reduce_workspace_bytes(const lbm_layout* L) {
  if (!L || L->n_fluid < 0) return 0;
  // tile partials; 8 result doubles; this state's entry of a batch's
  // segment table
  return align256((uint64_t)ceil_div((uint64_t)L->n_fluid, kRedBlock) * 5 * sizeof(double)) + 256 +
         seg_table_bytes(1);
}

// Scratch bytes the reductions of n states need: tile partials, 8 result
// doubles per state and (n > 1) the segment table.
static uint64_t reduce_scratch_bytes(const lbm_state* const* states, int32_t n) {
  uint64_t tiles = 0;
  for (int32_t j = 0; j < n; ++j) tiles += ceil_div((uint64_t)states[j]->layout.n_fluid, kRedBlock);
  return align256(tiles * 5 * sizeof(double)) + align256((uint64_t)n * 8 * sizeof(double)) +
         (n > 1 ? seg_table_bytes(n) : 0);
}

// Reductions of n states into `ws` (laid out as reduce_scratch_bytes says);
// segs[n] and host[8n] are host buffers of the caller.  Fills out[n]; SYNC.
static lbm_status reduce_states(const lbm_state* const* states, const lbm_collision* const* colls,
                                int32_t n, char* ws, uint64_t ws_bytes, Seg* segs, double* host,
                                lbm_reduction* out, hipStream_t st) {
  const int q = states[0]->layout.q, storage = states[0]->storage;
  const bool odd_t = (states[0]->t & 1) != 0;
  const uint64_t need = reduce_scratch_bytes(states, n);
  if (need > ws_bytes)
    return fail(LBM_ENOMEM, "reduction of %d state(s) needs %llu bytes of scratch (%llu available)",
                n, (unsigned long long)need, (unsigned long long)ws_bytes);
  uint32_t tiles = 0;
  for (int32_t j = 0; j < n; ++j) {
    segs[j] = make_seg(states[j], colls[j]);
    segs[j].tile0 = tiles;
    tiles += ceil_div(segs[j].nf, kRedBlock);
  }
  const uint64_t part_b = align256((uint64_t)tiles * 5 * sizeof(double));
  const uint64_t out_b = align256((uint64_t)n * 8 * sizeof(double));
  double* partials = (double*)ws;
  double* dout = (double*)(ws + part_b);
  StepArgs a;
  memset(&a, 0, sizeof(a));
  a.nseg = n;
  a.ntiles = tiles;
  if (n == 1) {
    a.seg0 = segs[0];
  } else {
    Seg* table = (Seg*)(ws + part_b + out_b);
    HIP_TRY(launch_put_segs(segs, (uint32_t)n, table, st), "segment table");
    a.segs = table;
  }
  HIP_TRY(launch_reduce(q, storage, a, odd_t, partials, dout, st), "reduce");
  HIP_TRY(hipMemcpyAsync(host, dout, sizeof(double) * 8 * n, hipMemcpyDeviceToHost, st),
          "reduce copy");
  HIP_TRY(hipStreamSynchronize(st), "reduce sync");
  bool finite_all = true;
  for (int j = 0; j < n; ++j) {
    lbm_reduction& r = out[j];
    r.mass = host[j * 8 + 0];
    r.mom[0] = host[j * 8 + 2];
    r.mom[1] = host[j * 8 + 3];
    r.mom[2] = host[j * 8 + 4];
    r.n_fluid = (int64_t)host[j * 8 + 6];
    r.finite = (host[j * 8 + 5] == 0.0 && isfinite(r.mass) && isfinite(r.mom[0]) &&
                isfinite(r.mom[1]) && isfinite(r.mom[2]))
                   ? 1
                   : 0;
    r.reserved = 0;
    finite_all = finite_all && r.finite;
  }
  if (!finite_all) return fail(LBM_EUNSTABLE, "non-finite values in the reduction");
  return LBM_OK;
}

static lbm_status check_reduce_batch(const lbm_state* const* states,
                                     const lbm_collision* const* colls, int32_t n,
                                     lbm_reduction* out) {
  if (!states || !colls || n < 1 || !out) return fail(LBM_EINVAL, "lbm_reduce_batch: bad arguments");
  for (int32_t j = 0; j < n; ++j) {
    lbm_status rc = check_state(states[j]);
    if (rc) return rc;
    rc = check_coll(colls[j], states[j]->layout.q);
    if (rc) return rc;
    if (states[j]->layout.q != states[0]->layout.q || states[j]->storage != states[0]->storage ||
        ((states[j]->t ^ states[0]->t) & 1))
      return fail(LBM_ESTATE, "batch member %d differs in q, storage or parity", j);
  }
  return LBM_OK;
}

lbm_status lbm_reduce_batch(const lbm_state* const* states, const lbm_collision* const* colls,
                            int32_t n, void* workspace, lbm_reduction* out, void* stream) {
  lbm_status rc = check_reduce_batch(states, colls, n, out);
  if (rc) return rc;
  if (!workspace) return fail(LBM_EINVAL, "workspace is NULL");
  // the caller provides the sum of the states' workspace sizes
  uint64_t bytes = 0;
  for (int32_t j = 0; j < n; ++j) bytes += lbm_reduce_workspace_bytes(&states[j]->layout);
  std::vector<Seg> segs((size_t)n);
  std::vector<double> host((size_t)n * 8);
  return reduce_states(states, colls, n, (char*)workspace, bytes, segs.data(), host.data(), out,
                       (hipStream_t)stream);
}

lbm_status lbm_reduce(const lbm_state* s, const lbm_collision* c, void* workspace,
                      lbm_reduction* out, void* stream) {
  const lbm_state* arr[1] = {s};
  const lbm_collision* carr[1] = {c};
  return lbm_reduce_batch(arr, carr, 1, workspace, out, stream);
}

// ------------------------------------------------------------- dense
lbm_status lbm_dense_build_mask(const uint8_t* labels, int32_t nx, int32_t ny, int32_t nz,
                                uint32_t periodic, int32_t q, uint32_t* mask, void* stream) {
  if (!labels || !mask) return fail(LBM_EINVAL, "labels/mask is NULL");
  if (!build_dims_ok(nx, ny, nz)) return fail(LBM_EINVAL, "box sizes must be in [1, 1024]");
  if (q != 19 && q != 27) return fail(LBM_EINVAL, "q must be 19 or 27");
  if (periodic > 7u) return fail(LBM_EINVAL, "periodic must be a 3-bit mask");
  HIP_TRY(launch_dense_mask(labels, nx, ny, nz, periodic, q, mask, (hipStream_t)stream),
          "dense mask");
  return LBM_OK;
}

static lbm_status check_dense(const lbm_dense_state* s) {
  if (!s) return fail(LBM_EINVAL, "dense state is NULL");
  if (s->q != 19 && s->q != 27) return fail(LBM_EINVAL, "q must be 19 or 27");
  if (!build_dims_ok(s->nx, s->ny, s->nz)) return fail(LBM_EINVAL, "box sizes must be in [1, 1024]");
  if (!storage_ok(s->storage)) return fail(LBM_EINVAL, "unknown storage");
  if (is16(s->storage) && (s->dev_exp < 0 || s->dev_exp > 24))
    return fail(LBM_EINVAL, "dev_exp must be in [0, 24]");
  const int64_t N = (int64_t)s->nx * s->ny * s->nz;
  if ((int64_t)s->q * N >= (int64_t)1 << 31) return fail(LBM_ERANGE, "q*N does not fit int32");
  if (!s->pdf || !s->mask) return fail(LBM_EINVAL, "pdf/mask is NULL");
  return LBM_OK;
}

lbm_status lbm_dense_init_equilibrium(lbm_dense_state* s, double rho0, const double* u0,
                                      void* stream) {
  lbm_status rc = check_dense(s);
  if (rc) return rc;
  if (!u0 || !(rho0 > 0.0)) return fail(LBM_EINVAL, "rho0 must be > 0 and u0 non-NULL");
  const uint32_t N = (uint32_t)((int64_t)s->nx * s->ny * s->nz);
  const int e = is16(s->storage) ? s->dev_exp : 0;
  HIP_TRY(launch_init(s->q, s->storage, s->pdf, N, N, rho0, u0, ldexpf(1.0f, e),
                      (hipStream_t)stream),
          "dense init");
  s->t = 0;
  return LBM_OK;
}

lbm_status lbm_dense_step(lbm_dense_state* s, int32_t n_steps, const lbm_collision* c,
                          void* stream) {
  lbm_status rc = check_dense(s);
  if (rc) return rc;
  rc = check_coll(c, s->q);
  if (rc) return rc;
  if (n_steps < 0) return fail(LBM_EINVAL, "n_steps must be >= 0");
  const lbm_launch cfg = get_cfg(LBM_KERNEL_DENSE, s->q, s->storage);
  DenseArgs a;
  memset(&a, 0, sizeof(a));
  a.pdf = s->pdf;
  a.mask = s->mask;
  a.nx = s->nx;
  a.ny = s->ny;
  a.nz = s->nz;
  a.periodic = s->periodic;
  a.N = (uint32_t)((int64_t)s->nx * s->ny * s->nz);
  a.xcd_remap = cfg.xcd_remap;
  a.ntiles = ceil_div(a.N, (uint64_t)cfg.block);
  coll_rates(c, a.om1, a.om2, a.rates);
  for (int k = 0; k < 3; ++k) a.F[k] = c->force[k];
  const int e = is16(s->storage) ? s->dev_exp : 0;
  a.scale = ldexpf(1.0f, e);
  a.inv_scale = ldexpf(1.0f, -e);
  for (int32_t step = 0; step < n_steps; ++step) {
    const bool odd = (s->t & 1) == 0;
    HIP_TRY(launch_dense_step(s->q, c->kind, s->storage, odd, a, cfg.block, (hipStream_t)stream),
            "dense step");
    s->t += 1;
  }
  return LBM_OK;
}

// --------------------------------------------------------------- copy
lbm_status lbm_copy(void* dst, const void* src, uint64_t bytes, void* stream) {
  if (!dst || !src) return fail(LBM_EINVAL, "copy: NULL pointer");
  if ((bytes & 15) || ((uintptr_t)dst & 15) || ((uintptr_t)src & 15))
    return fail(LBM_EINVAL, "copy: pointers and size must be 16-byte aligned");
  HIP_TRY(launch_copy(dst, src, bytes, (hipStream_t)stream), "copy");
  return LBM_OK;
}

}  // extern "C"
