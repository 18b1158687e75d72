/*
 * lbm.h -- C-ABI of the MI355X (gfx950) sparse, indirect-addressing lattice
 * Boltzmann library (liblbm.so).
 *
 * The method is the sparse LBM of Suffa, Holzer, Koestler, Ruede,
 * arXiv 2408.06880: PDFs of fluid cells only, stored as a structure-of-arrays
 * "PDF-list"; neighbours reached through an int32 "index-list" with
 * bounce-back and periodicity folded in (Section "Sparse Data Structure",
 * "Sparse Boundary Conditions"); in-place AA streaming, alternating an
 * "odd" step (pull, collide, push back to the read positions) and an "even"
 * step (collide in place, opposite slots) so that one PDF array suffices
 * (Section "In-place Streaming: AA Pattern").
 *
 * Conventions
 *  - Every function returns lbm_status: LBM_OK (0) or a negative code.
 *    On error, lbm_last_error() (per calling thread) holds a message.
 *  - The caller owns all device memory and the HIP stream.  Pointers named
 *    "device" must be device (HBM) allocations of at least the stated size;
 *    "host" pointers are ordinary host memory.  `stream` is a hipStream_t
 *    (NULL = the default stream).
 *  - Calls are asynchronous on `stream` unless marked SYNC.  Kernel faults
 *    surface at the next synchronising call as LBM_EDEVICE.
 *  - No entry point allocates device memory.  Scratch comes in through a
 *    caller-provided `workspace` whose size a *_workspace_bytes() query
 *    returns.
 *  - A given lbm_state must not be used from two threads at once; separate
 *    states may be driven from different threads and streams.
 *
 * Lattice conventions (fixed; both the library and any reader of its
 * buffers rely on them)
 *  - Cell linear id: lin = x + nx*(y + ny*z).  Labels: uint8, 0 = fluid,
 *    1 = solid (no-slip), 2 + c = boundary class c (c < 8).  Periodicity:
 *    bit 0 = x, bit 1 = y, bit 2 = z.  A non-periodic box face is a no-slip
 *    wall located halfway between the outermost cell layer and the outside.
 *  - Directions: 0 = rest; then pairs (+e, -e): 1,2 = +-x; 3,4 = +-y;
 *    5,6 = +-z; 7..18 = the xy, xz, yz edge pairs (+x+y,-x-y), (+x-y,-x+y),
 *    (+x+z,-x-z), (+x-z,-x+z), (+y+z,-y-z), (+y-z,-y+z); D3Q27 adds the
 *    corners 19..26: (+++,---), (++-,--+), (+-+,-+-), (-++,+--).  The
 *    opposite of i >= 1 is i+1 for odd i and i-1 for even i.
 *  - PDF-list: element i*S + k = population i of the k-th fluid cell
 *    (S = stride >= n_fluid).  Index-list: element (i-1)*S + k = position
 *    in the PDF-list that cell k pulls population i from.
 */
#ifndef LBM_H
#define LBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lbm_status;

#define LBM_OK 0
#define LBM_EINVAL (-1)    /* invalid argument                                  */
#define LBM_ERANGE (-2)    /* q * stride does not fit 32-bit positions           */
#define LBM_ENOMEM (-3)    /* caller buffer / workspace too small                */
#define LBM_EDEVICE (-4)   /* a HIP call failed                                  */
#define LBM_EUNSTABLE (-5) /* a reduction saw NaN or Inf                          */
#define LBM_ESTATE (-6)    /* layout / parity / storage mismatch between inputs   */

enum { LBM_D3Q19 = 19, LBM_D3Q27 = 27 };
enum { LBM_COLL_NONE = 0, LBM_COLL_SRT = 1, LBM_COLL_TRT = 2, LBM_COLL_CUMULANT = 3,
       LBM_COLL_MRT = 4, LBM_COLL_CM = 5 };
/* Storage of the PDF-list.  *DEV formats store the deviation f_i - w_i
 * from the rest weights ("zero-centred" storage option, Section "Code
 * Generation for Sparse Kernels"), 16-bit ones scaled by 2^dev_exp.  All
 * arithmetic is FP32 except for LBM_STORE_F64, which computes in FP64. */
enum {
  LBM_STORE_F64 = 0,     /* double f_i                                            */
  LBM_STORE_F32 = 1,     /* float f_i                                             */
  LBM_STORE_F16DEV = 2,  /* IEEE half (f_i - w_i) * 2^dev_exp                     */
  LBM_STORE_BF16DEV = 3, /* bfloat16 (f_i - w_i) * 2^dev_exp                      */
  LBM_STORE_F32DEV = 4   /* float (f_i - w_i)                                     */
};
/* Fluid-cell order of the lists.  MORTON: Morton key of (x, y, z), bit b of
 * x, y, z at bits 3b, 3b+1, 3b+2.  LEX: linear id.  BLOCKED: the box is cut
 * into blocks of nx * 8 * 8 cells (whole x rows, 8 in y, 8 in z); blocks are
 * visited in 2-D Morton order of (y/8, z/8) (y bit at 2b, z bit at 2b+1)
 * and cells inside a block lexicographically (x, then y, then z). */
enum { LBM_ORDER_MORTON = 0, LBM_ORDER_LEX = 1, LBM_ORDER_BLOCKED = 2 };
enum { LBM_BC_NOSLIP = 0, LBM_BC_UBB = 1, LBM_BC_PRESSURE = 2 };

/* Sizes of one sparse domain.  Filled by lbm_build_sparse (plan call). */
typedef struct {
  int32_t nx, ny, nz;
  uint32_t periodic;
  int32_t q;         /* 19 or 27                                               */
  int32_t order;     /* LBM_ORDER_*                                            */
  int32_t align;     /* stride is a multiple of align (1 = unpadded)           */
  int32_t reserved;
  int64_t n_fluid;   /* N_F                                                    */
  int64_t stride;    /* S = round_up(N_F, align)                               */
  int64_t n_links;   /* boundary links (upstream cell carries label >= 2)      */
} lbm_layout;

/* ------------------------------------------------------------------ */
/* Builder: labels -> fluid list, index-list, boundary links.           */
/* Section "Sparse Data Structure" (PDF-list, index-list; N_F*(Q-1)     */
/* index entries since the rest population does not stream) and         */
/* "Sparse Boundary Conditions" (no-slip pull index redirected to the   */
/* same cell's opposite population; periodic pull index wrapped to the  */
/* other side of the domain).                                           */
/* ------------------------------------------------------------------ */

/* Device workspace bytes lbm_build_sparse needs for an nx*ny*nz box.
 * Host only; 0 for invalid sizes. */
uint64_t lbm_build_workspace_bytes(int32_t nx, int32_t ny, int32_t nz, int32_t order);

/* Two-phase build.
 *  labels     device, uint8[nx*ny*nz] (layout above); nx, ny, nz in [1, 1024].
 *  order      LBM_ORDER_MORTON, LBM_ORDER_LEX or LBM_ORDER_BLOCKED (above).
 *  align      stride multiple, >= 1 (64 recommended).
 *  workspace  device, >= lbm_build_workspace_bytes(nx, ny, nz, order).
 *  layout     host.  PLAN call (cells == NULL): SYNC; fills *layout; index
 *             and links must be NULL.  FILL call (cells != NULL): *layout
 *             must be the plan's result for the same labels (unchanged in
 *             between); writes
 *               cells  device int32[n_fluid]: lin of the k-th fluid cell;
 *               index  device int32[(q-1)*stride] holding unsigned 32-bit
 *                      PDF positions (q*S < 2^32): element (i-1)*S + k =
 *                      i*S + m if the upstream cell x_k - c_i (wrapped on
 *                      periodic axes) is fluid with list position m, else
 *                      opp(i)*S + k; padding k in [n_fluid, S) gets
 *                      opp(i)*S + k (in bounds; no step gathers through
 *                      a padding entry);
 *               links  device int32[2*n_links] (may be NULL iff n_links==0):
 *                      pairs (opp(i)*S + k, i | class << 8) for every
 *                      upstream cell with label 2 + class, ordered by (k, i).
 * Errors: LBM_EINVAL (sizes, q, order, align), LBM_ERANGE (q*S >= 2^32),
 *         LBM_EDEVICE. */
lbm_status lbm_build_sparse(const uint8_t* labels, int32_t nx, int32_t ny, int32_t nz,
                            uint32_t periodic, int32_t q, int32_t order, int32_t align,
                            void* workspace, lbm_layout* layout, int32_t* cells, int32_t* index,
                            int32_t* links, void* stream);

/* ------------------------------------------------------------------ */
/* State, collision parameters, boundary specification.                 */
/* ------------------------------------------------------------------ */

typedef struct {
  lbm_layout layout;
  int32_t storage;       /* LBM_STORE_*                                        */
  int32_t dev_exp;       /* 16-bit formats: stored = (f - w) * 2^dev_exp, 0..24 */
  void* pdf;             /* device, q*stride elements of the storage type      */
  const int32_t* index;  /* device, (q-1)*stride (from lbm_build_sparse); may  */
                         /* be NULL when runs is set (then no pull steps)      */
  const void* index16;   /* device, compact index-list (lbm_compress_index) of  */
                         /* the same index, or NULL; when set, index reads use  */
                         /* it and fall back to `index` for escaped entries     */
  const void* runs;      /* device, run-compressed index-list (lbm_compress_runs)*/
                         /* of the same index, or NULL; when set, odd steps and  */
                         /* moments/reductions at odd t read it instead of       */
                         /* index16 and index                                    */
  const int32_t* links;  /* device, 2*n_links or NULL when n_links == 0        */
  int64_t t;             /* steps taken. t even: populations in natural slots  */
  void* link_vel;        /* device link-velocity buffer of this state          */
                         /* (lbm_link_vel_prepare), or NULL                    */
  int64_t link_vel_t;    /* t at which link_vel holds the velocities (set by   */
                         /* every step); -1: holds nothing (set it so whenever */
                         /* the PDF-list is written other than by the library) */
} lbm_state;

/* Collision operator (Section "Lattice Boltzmann Method" and "Code
 * Generation for Sparse Kernels").  nu = (tau - 1/2)/3, tau > 1/2.
 *  SRT:      relax all populations with omega = 1/tau (BGK).
 *  TRT:      symmetric parts with omega+ = 1/tau, antisymmetric parts with
 *            omega- from magic = (1/omega+ - 1/2)(1/omega- - 1/2).
 *  CUMULANT: D3Q27 only; second-order shear/deviatoric moments relax with
 *            1/tau, the trace with omega_bulk, all higher cumulants -> 0.
 *  MRT:      D3Q19 only; the 19 orthogonal moments of d'Humieres et al.
 *            (2002) relax toward the moments of the same second-order
 *            equilibrium: shear moments (3p_xx, p_ww, p_xy, p_yz, p_xz)
 *            with 1/tau, energy e with omega_bulk, epsilon, pi_xx/pi_ww,
 *            energy flux q and third-order m with rates[0..3] (each in
 *            (0, 2)); the Guo source enters every moment with (1 - s/2).
 *            Even rates = 1/tau and odd rates = omega- give TRT exactly.
 *  CM:       central moments, D3Q27 only (the stencil with the complete
 *            per-axis central-moment basis); orders 0-2 as CUMULANT, each
 *            central moment of order n = 3..6 relaxes towards the
 *            Maxwellian's (rho times 1, 0, 1/3 per axis for exponent 0, 1,
 *            2) with rates[n - 3], each in (0, 2); all rates one give the
 *            product-form equilibrium, as the cumulant operator does.
 *  force:    constant body force density (Guo scheme, half-force velocity).
 */
typedef struct {
  int32_t kind;          /* LBM_COLL_*                                         */
  int32_t reserved;
  double tau;
  double magic;          /* TRT Lambda, e.g. 3/16                               */
  double omega_bulk;     /* cumulant trace rate, MRT energy rate, e.g. 1       */
  double force[3];
  double rates[4];       /* MRT: epsilon, pi, q, m rates; CM: orders 3, 4, 5, 6 */
} lbm_collision;

/* Boundary classes for labels 2..9.  UBB: moving wall u (bounce-back plus
 * 6 w_i rho_w c_i.u, rho_w = 1); PRESSURE: anti-bounce-back to density rho,
 * -f + 2 w_i rho (1 + 9/2 (c_i.u)^2 - 3/2 u.u) with u the fluid cell's
 * velocity at the current time (its u member is unused); NOSLIP: plain
 * bounce-back.  The paper specifies the no-slip and velocity rules; the
 * pressure rule is this library's outlet. */
typedef struct {
  int32_t type;          /* LBM_BC_*                                           */
  int32_t reserved;
  double u[3];
  double rho;
} lbm_bclass;
typedef struct {
  int32_t n_classes;     /* 0..8                                               */
  int32_t reserved;
  lbm_bclass cls[8];
} lbm_bspec;

/* Compact index-list.  The list positions are cut into tiles of 256
 * cells; for tile t and direction i the library stores one int32 base b,
 * and per cell a uint16 o: 0xFFFF = upstream cell not fluid (position
 * opp(i)*S + k), 0xFFFE = escaped (position read from the int32
 * index-list), else position i*S + k + b + o.  b is chosen per tile and
 * direction so that as many entries as possible fit the 16-bit window.
 * Buffer: uint16 o[(q-1)][S]; then (256-byte aligned) int32 b[tiles][q-1];
 * then (aligned) uint32 per-tile escape counts and their total.
 * Halves the index bytes read by each odd step.
 *  lbm_index16_bytes: device bytes of the compact form (host only).
 *  lbm_compress_index: index device int32[(q-1)*S] from lbm_build_sparse;
 *      index16 device buffer of lbm_index16_bytes(layout); n_escaped host
 *      (may be NULL) receives the number of escaped entries.  SYNC.
 *      lbm_state.index stays required next to index16. */
uint64_t lbm_index16_bytes(const lbm_layout* layout);
lbm_status lbm_compress_index(const lbm_layout* layout, const int32_t* index, void* index16,
                              uint64_t* n_escaped, void* stream);

/* Run-compressed index-list (same entries as the int32 index-list of
 * Section "Sparse Data Structure", fewer bytes).  The list positions are
 * cut into waves of 64 (wave w: positions 64w .. 64w+63, W = ceil(S/64)
 * waves).  For wave w and direction i a run is a maximal stretch of lanes
 * whose entries rise by one from lane to lane; it is stored as one int32
 * v = (entry of its first lane l0) - l0, so that lane l of the run has the
 * entry v + l.  Rows of a list ordered along x make most entries continue a
 * run (neighbouring cells pull from neighbouring cells or from consecutive
 * bounce-back slots), so the form needs a few bytes per cell instead of
 * 4*(q-1).
 * Buffer (device), parts 256-byte aligned in this order:
 *   uint32 voff[W + 1]: index of wave w's first value; voff[W] = all values;
 *   uint64 mask[W][q-1]: bit l set = lane l starts a run (bit 0 always);
 *   int32 val[voff[W]]: wave w's values, direction 1's runs in lane order,
 *                       then direction 2's, ... .
 *  lbm_runs_header_bytes: bytes of voff and mask (host only).
 *  lbm_compress_runs: index device int32[(q-1)*S] from lbm_build_sparse;
 *      runs device buffer of `capacity` >= lbm_runs_header_bytes(layout)
 *      bytes; *needed (host, required) receives the size of the whole form.
 *      If capacity >= *needed, writes it and returns LBM_OK; otherwise
 *      writes voff and mask only and returns LBM_ENOMEM: allocate *needed
 *      bytes and call again.  A capacity below the header size returns
 *      LBM_ENOMEM with *needed = the header size and writes nothing.  SYNC.
 *      A state with runs may drop its int32 index (lbm_state.index = NULL):
 *      steps, moments and reductions then read only the run form; pull
 *      steps still need the int32 index. */
uint64_t lbm_runs_header_bytes(const lbm_layout* layout);
lbm_status lbm_compress_runs(const lbm_layout* layout, const int32_t* index, void* runs,
                             uint64_t capacity, uint64_t* needed, void* stream);

/* Link-velocity buffer (optional; no counterpart in the paper).  The
 * pressure rule of Section "Sparse Boundary Conditions" as this library
 * states it needs the velocity of each cell that has an outlet link before
 * every step; without the buffer the link update gathers all q populations
 * of such a cell (one cache line each).  With it, every step kernel also
 * writes the density and momentum sums of the cells that have links, the
 * step calls set lbm_state.link_vel_t = t after each step, and a link
 * update at time t forms the velocities from those sums (with the force
 * of the step it precedes) when link_vel_t == t, else it gathers.
 * lbm_init_equilibrium and lbm_convert set link_vel_t = -1 on the state
 * they write; a caller that writes a PDF-list by other means (an upload, a
 * restored checkpoint) sets it to -1 too.  Results are bitwise the same
 * with and without the buffer.
 *  lbm_link_vel_bytes: device bytes for `layout` (0 when it has no links;
 *      host only).
 *  lbm_link_vel_prepare: links device int32[2*n_links] from
 *      lbm_build_sparse (same layout); link_vel device buffer of
 *      lbm_link_vel_bytes(layout) bytes: marks the cells with links, in
 *      stream order (asynchronous).  Set lbm_state.link_vel to it.  One
 *      buffer belongs to one state: states stepped in one batch, or
 *      concurrently, need buffers of their own. */
uint64_t lbm_link_vel_bytes(const lbm_layout* layout);
lbm_status lbm_link_vel_prepare(const lbm_layout* layout, const int32_t* links, void* link_vel,
                                void* stream);

/* Change a state's storage format (the deviation storage of the FP16/BF16
 * formats; no counterpart in the paper): every slot of src's PDF-list,
 * padding included, is decoded to delta = f - w in FP64 and encoded in
 * dst->storage (16-bit formats round to nearest even at dst->dev_exp);
 * dst->t = src->t.  FP16/BF16/FP32 deviations convert to FP32-deviation or
 * FP64 exactly.  The parity does not matter (opposite directions share a
 * weight).  dst: a state of the same layout (q, stride, n_fluid) whose pdf
 * holds q*stride elements of its storage and does not overlap src's; its
 * index, index16, runs and links are not touched.  Errors: LBM_EINVAL,
 * LBM_EDEVICE. */
lbm_status lbm_convert(const lbm_state* src, lbm_state* dst, void* stream);

/* Initialise every fluid cell to the equilibrium of (rho0, u0) and set
 * state->t = 0.  u0: host double[3].  Padding slots are zeroed (deviation)
 * or set to the weights.  Errors: LBM_EINVAL, LBM_EDEVICE. */
lbm_status lbm_init_equilibrium(lbm_state* state, double rho0, const double* u0, void* stream);

/* Advance n_steps >= 0 AA steps (Section "In-place Streaming: AA Pattern").
 * For each step: apply the boundary links (if n_links > 0), then run the
 * odd kernel when t is even (gather through the index-list, collide, write
 * each result back to the slot its opposite population came from) or the
 * even kernel when t is odd (collide reading opposite slots, write natural
 * slots); t += 1.  bspec may be NULL when n_links == 0.
 * Errors: LBM_EINVAL (tau <= 1/2, cumulant with q != 27, storage/dev_exp),
 *         LBM_ESTATE, LBM_EDEVICE. */
lbm_status lbm_step(lbm_state* state, int32_t n_steps, const lbm_collision* coll,
                    const lbm_bspec* bspec, void* stream);

/* Two-array pull scheme over the same lists (the pattern the paper's AA
 * section compares against): every step gathers through the index-list,
 * collides and writes f*_i to slot i*S + k of the other array, then the two
 * arrays swap.  *spare is a device buffer of the same size as state->pdf;
 * on return state->pdf holds the current populations and *spare the other
 * buffer.  The slot layout stays natural, so t must be even on entry and
 * n_steps even (then the state continues seamlessly with lbm_step).  The
 * launch configuration of LBM_KERNEL_ODD is used without its residency cap.
 * The pull kernel reads the int32 index-list (or the compact form with
 * it): a state whose int32 list was dropped is refused with LBM_EINVAL.
 * Errors as lbm_step. */
lbm_status lbm_step_pull(lbm_state* state, void** spare, int32_t n_steps,
                         const lbm_collision* coll, const lbm_bspec* bspec, void* stream);

/* Density and velocity of every fluid cell at the current t (either
 * parity), from the post-collision populations: rho = sum f*,
 * u = (sum c f* - F/2) / rho.
 *  rho  device, stride elements; u device, 3*stride elements (u_x block,
 *       u_y block, u_z block); element type double if out_f64 else float.
 * Entries k >= n_fluid are left as they were.  Errors: LBM_EINVAL (state,
 * collision), LBM_EDEVICE. */
lbm_status lbm_moments(const lbm_state* state, const lbm_collision* coll, int32_t out_f64,
                       void* rho, void* u, void* stream);

/* FP64 global reductions over fluid cells (either parity):
 * mass = sum rho, mom = sum rho*u.  Deterministic: fixed per-tile tree then
 * a fixed-order second pass.  SYNC.  Returns LBM_EUNSTABLE (with the
 * result filled and finite = 0) if any value was NaN or Inf. */
typedef struct {
  double mass;
  double mom[3];
  int64_t n_fluid;
  int32_t finite;
  int32_t reserved;
} lbm_reduction;

uint64_t lbm_reduce_workspace_bytes(const lbm_layout* layout);
lbm_status lbm_reduce(const lbm_state* state, const lbm_collision* coll, void* workspace,
                      lbm_reduction* host_out, void* stream);

/* ------------------------------------------------------------------ */
/* Batching: one launch per step advances many independent states in     */
/* lockstep parity.  Each state keeps its own buffers; kernels never mix */
/* two states in one workgroup, so every result is bitwise identical to  */
/* running the state alone with the same launch configuration.           */
/* ------------------------------------------------------------------ */

/* Device workspace bytes lbm_step_batch needs for n_states states (host
 * only; 0 for n_states < 1): room for the batch's segment tables (each
 * state's buffers, sizes and collision parameters, about 160 bytes per state
 * and parity), which the launches read from device memory.  */
uint64_t lbm_step_batch_workspace_bytes(int32_t n_states);

/* states[n], colls[n], bspecs[n] (bspecs may be NULL): every state must
 * have the same q, storage and parity (t & 1).  No limit on n.
 *  workspace        device, >= lbm_step_batch_workspace_bytes(n) bytes
 *                   (may be NULL when n == 1).  The call writes the
 *                   segment tables into it on `stream` (kernels, no host
 *                   copies) before the first step; it must not be reused
 *                   by another call on another stream until this call's
 *                   launches have run.
 *  workspace_bytes  its size.
 * Errors: LBM_ESTATE when the states differ, LBM_ENOMEM when the workspace
 * is too small, otherwise as lbm_step. */
lbm_status lbm_step_batch(lbm_state* const* states, const lbm_collision* const* colls,
                          const lbm_bspec* const* bspecs, int32_t n_states, int32_t n_steps,
                          void* workspace, uint64_t workspace_bytes, void* stream);

/* lbm_step_batch for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same steps, launches and results as lbm_step_batch with
 * the same arguments, but the segment tables go into a fixed device array
 * inside the library instead of a caller workspace.  The array holds the
 * tables of LBM_STEP_BATCH_NOALLOC_MAX states (about 370 KiB); each device
 * the library runs on keeps its own copy until the process ends, and the
 * call allocates nothing.
 *  n_states  1 .. LBM_STEP_BATCH_NOALLOC_MAX; more returns LBM_ENOMEM.
 *  stream    must belong to the calling thread's current device
 *            (LBM_EINVAL otherwise).
 * Every call on one device writes that device's array (each call writes
 * the whole table it reads before its first launch, so nothing is carried
 * over), so calls whose launches may overlap on one device -- from several
 * threads or on several streams without ordering between them -- race;
 * serialise them.  Errors as lbm_step_batch. */
#define LBM_STEP_BATCH_NOALLOC_MAX 1024
lbm_status lbm_step_batch_noalloc(lbm_state* const* states, const lbm_collision* const* colls,
                                  const lbm_bspec* const* bspecs, int32_t n_states,
                                  int32_t n_steps, void* stream);

/* Per-state reductions of lbm_reduce for n states at once (no limit on n),
 * bitwise equal to calling lbm_reduce on each.  workspace >= sum of
 * lbm_reduce_workspace_bytes over the states (it also holds the batch's
 * segment table).  host_out[n].  SYNC. */
lbm_status lbm_reduce_batch(const lbm_state* const* states, const lbm_collision* const* colls,
                            int32_t n_states, void* workspace, lbm_reduction* host_out,
                            void* stream);

/* ------------------------------------------------------------------ */
/* Dense direct-addressing comparator (Section "Single Node Results":    */
/* the dense kernel traverses every cell, fluid or not, without a fluid  */
/* branch).  AA pattern over all N = nx*ny*nz cells, PDF element i*N +   */
/* lin; bounce-back from a per-cell uint32 mask (bit i set: the upstream */
/* cell x - c_i is not fluid).  Labels >= 2 act as no-slip here.         */
/* ------------------------------------------------------------------ */

typedef struct {
  int32_t nx, ny, nz;
  uint32_t periodic;
  int32_t q;
  int32_t storage;
  int32_t dev_exp;
  int32_t reserved;
  void* pdf;             /* device, q*N elements                               */
  const uint32_t* mask;  /* device, N                                          */
  int64_t t;
} lbm_dense_state;

/* labels device uint8[N]; mask device uint32[N]. */
lbm_status lbm_dense_build_mask(const uint8_t* labels, int32_t nx, int32_t ny, int32_t nz,
                                uint32_t periodic, int32_t q, uint32_t* mask, void* stream);
lbm_status lbm_dense_init_equilibrium(lbm_dense_state* state, double rho0, const double* u0,
                                      void* stream);
lbm_status lbm_dense_step(lbm_dense_state* state, int32_t n_steps, const lbm_collision* coll,
                          void* stream);

/* ------------------------------------------------------------------ */
/* Launch configuration and measurement helpers.                        */
/* ------------------------------------------------------------------ */

enum { LBM_KERNEL_ODD = 0, LBM_KERNEL_EVEN = 1, LBM_KERNEL_DENSE = 2 };
typedef struct {
  int32_t block;      /* threads per workgroup: 64, 128 or 256                 */
  int32_t xcd_remap;  /* tile order over the 8 XCDs (workgroup v runs on XCD  */
                      /* v % 8): 0 = dispatch order; 1 = each XCD takes one    */
                      /* contiguous eighth of the tiles; m in [2, 65536] =     */
                      /* chunks of m consecutive tiles dealt round-robin to    */
                      /* the XCDs                                              */
  int32_t pipelined;  /* odd kernel, block 256, compact index-list only: 1 =   */
                      /* persistent workgroups that load the next tile's       */
                      /* offsets during the current tile (same results)        */
  int32_t cells_per_thread; /* even kernel: 2 = two neighbouring cells per    */
                      /* thread with 2-wide loads/stores, used when every      */
                      /* state of the launch has an even stride (one cell      */
                      /* otherwise); 0 or 1 = one cell (the only choice for    */
                      /* the other kernels)                                    */
  int32_t max_groups_per_cu; /* odd and even AA kernels: 0 = as many resident */
                      /* workgroups per CU as registers allow; n in [2, 16] =  */
                      /* at most n (dynamic LDS is reserved for the purpose;   */
                      /* the kernels use none).  Not for pipelined or dense    */
                      /* launches; pull steps run uncapped.                    */
} lbm_launch;

/* Set / get the launch configuration used for (kernel, q, storage) from
 * now on, process-wide (e.g. from an autotuner cache).  Changing it does
 * not change results except through workgroup-to-tile assignment, which
 * the arithmetic does not depend on.  Defaults (measured on MI355X): block
 * 256; XCD-aware tile order for the odd kernel only (chunks of 16 tiles,
 * 256 for D3Q19 in 16-bit storage);
 * two cells per thread for even steps in 16-bit storage; D3Q19 FP32 and
 * FP32-dev at most 4
 * (odd) and 3 (even) workgroups per CU; D3Q19 FP64 even steps with block
 * 64, two cells per thread, at most 2 per CU; D3Q27 FP32 and FP32-dev
 * odd steps at most 3 per CU; everything else uncapped. */
lbm_status lbm_set_launch(int32_t kernel, int32_t q, int32_t storage, const lbm_launch* cfg);
lbm_status lbm_get_launch(int32_t kernel, int32_t q, int32_t storage, lbm_launch* cfg);

/* Streaming copy dst[0..bytes) = src[0..bytes) with 16-byte vector loads;
 * device pointers, 16-byte aligned, bytes a multiple of 16.  Reference for
 * the achievable HBM bandwidth and for hardware byte counters.
 * Errors: LBM_EINVAL (alignment, size), LBM_EDEVICE. */
lbm_status lbm_copy(void* dst, const void* src, uint64_t bytes, void* stream);

/* Message of the last failing call on the calling thread (owned by the
 * library, valid until that thread's next call; empty when none failed). */
const char* lbm_last_error(void);
/* Version of this interface: 7 (launch table with residency caps, unsigned
 * 32-bit positions, optional int32 index-list next to the run form, batch
 * segment tables in a caller workspace, batch steps without allocation,
 * link-velocity buffer in the state). */
int32_t lbm_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
