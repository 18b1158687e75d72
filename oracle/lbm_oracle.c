/*
 * Plain FP64 CPU oracle for the sparse, indirect-addressing lattice Boltzmann
 * method (Suffa, Holzer, Koestler, Ruede: "Architecture Specific Generation of
 * Large Scale Lattice Boltzmann Methods for Sparse Complex Geometries",
 * arXiv 2408.06880).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link or call
 * this file; it exists so that tests, the smoke check and the CPU baseline
 * timing have an obviously correct reference to compare the HIP kernels with.
 * It shares no code, header, table or constant with the GPU library.
 *
 * Two independent schemes live here:
 *   1. dense two-array pull LBM over every box cell (Section "Lattice
 *      Boltzmann Method", eqs. (1)-(6); pull pattern of Section "In-place
 *      Streaming: AA Pattern");
 *   2. a sparse CPU variant with its own list builder (Section "Sparse Data
 *      Structure", "Sparse Boundary Conditions") and in-place AA streaming
 *      (Section "In-place Streaming: AA Pattern").
 * After every even number of steps both must give the same PDFs.
 *
 * Everything is FP64, no fused multiply-add contraction (built with
 * -ffp-contract=off), no reassociation.  Readings where the paper is silent
 * (direction order, Guo forcing, TRT magic parameter, cumulant details,
 * inlet/outlet links, Morton order) are listed in the repository design notes
 * and restated at each function below.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Loops over fewer cells than this run on one thread: on tiny test boxes a
 * parallel region per step costs more than the step.  Every cell is
 * computed on its own, so the thread count never changes a result. */
#define ORC_PAR_MIN 32768

/* ------------------------------------------------------------------ */
/* Velocity sets.                                                      */
/* D3Q19 / D3Q27 with the pairwise order: 0 rest, then (+e,-e) pairs:  */
/* axes, xy/xz/yz edges, and (D3Q27) the four corner diagonals.        */
/* Weights: D3Q19 1/3, 1/18, 1/36; D3Q27 8/27, 2/27, 1/54, 1/216.       */
/* The opposite direction is found by search, not by an index rule.     */
/* ------------------------------------------------------------------ */

typedef struct {
  int q;
  int c[27][3];
  double w[27];
  int opp[27];
} orc_stencil;

static const int ORC_DIRS[27][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1},
    {1, 1, 1},  {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1},
    {1, -1, 1}, {-1, 1, -1}, {-1, 1, 1}, {1, -1, -1}};

static int orc_stencil_init(orc_stencil* s, int q) {
  if (q != 19 && q != 27) return -1;
  s->q = q;
  for (int i = 0; i < q; ++i) {
    int n2 = 0;
    for (int a = 0; a < 3; ++a) {
      s->c[i][a] = ORC_DIRS[i][a];
      n2 += ORC_DIRS[i][a] * ORC_DIRS[i][a];
    }
    if (q == 19) {
      s->w[i] = (n2 == 0) ? 1.0 / 3.0 : (n2 == 1) ? 1.0 / 18.0 : 1.0 / 36.0;
    } else {
      s->w[i] = (n2 == 0)   ? 8.0 / 27.0
                : (n2 == 1) ? 2.0 / 27.0
                : (n2 == 2) ? 1.0 / 54.0
                            : 1.0 / 216.0;
    }
  }
  for (int i = 0; i < q; ++i) {
    s->opp[i] = -1;
    for (int j = 0; j < q; ++j)
      if (s->c[j][0] == -s->c[i][0] && s->c[j][1] == -s->c[i][1] &&
          s->c[j][2] == -s->c[i][2])
        s->opp[i] = j;
  }
  return 0;
}

/* Exported so tests can check the tables against lattice isotropy. */
int orc_stencil_tables(int q, int32_t* c_out /* [q*3] */, double* w_out /* [q] */,
                       int32_t* opp_out /* [q] */) {
  orc_stencil s;
  if (orc_stencil_init(&s, q)) return -1;
  for (int i = 0; i < q; ++i) {
    for (int a = 0; a < 3; ++a) c_out[3 * i + a] = s.c[i][a];
    w_out[i] = s.w[i];
    opp_out[i] = s.opp[i];
  }
  return 0;
}

/* Threads the OpenMP loops use (reported with CPU timings). */
int orc_num_threads(void) { return omp_get_max_threads(); }

/* Sets the thread count of later parallel loops (CPU timings only). */
void orc_set_num_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

/* ------------------------------------------------------------------ */
/* Parameters.                                                          */
/* ------------------------------------------------------------------ */

enum { ORC_NONE = 0, ORC_SRT = 1, ORC_TRT = 2, ORC_CUMULANT = 3, ORC_MRT = 4, ORC_CM = 5 };
enum { ORC_BC_NOSLIP = 0, ORC_BC_UBB = 1, ORC_BC_PRESSURE = 2 };

typedef struct {
  int32_t q;
  int32_t kind;         /* ORC_NONE / SRT / TRT / CUMULANT / MRT            */
  double tau;           /* relaxation time, nu = (tau - 1/2)/3              */
  double magic;         /* TRT magic parameter Lambda                       */
  double omega_bulk;    /* cumulant trace / MRT energy (bulk) rate          */
  double rates[4];      /* MRT: epsilon, pi, q, m rates; CM: orders 3-6     */
  double force[3];      /* constant body force density F                    */
  int32_t n_classes;    /* boundary classes for labels >= 2                 */
  int32_t cls_type[8];  /* ORC_BC_*                                         */
  double cls_u[8][3];   /* UBB wall velocity                                */
  double cls_rho[8];    /* pressure-outlet density (UBB uses rho_w = 1)     */
} orc_params;

/* ------------------------------------------------------------------ */
/* Collision (one cell). Input: pre-collision f[q]. Output: f*[q].       */
/* Section "Lattice Boltzmann Method": rho and rho*u from the PDFs      */
/* (eq. 1), equilibrium (second-order polynomial, c_s^2 = 1/3), SRT     */
/* operator, nu = c_s^2 (tau - 1/2).  Force: Guo scheme with the        */
/* half-force velocity (the paper only names a "force model" option).   */
/* ------------------------------------------------------------------ */

static void orc_macros(const orc_stencil* s, const double* f, const double F[3], double* rho,
                       double u[3]) {
  double r = 0.0, j[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < s->q; ++i) {
    r += f[i];
    for (int a = 0; a < 3; ++a) j[a] += s->c[i][a] * f[i];
  }
  *rho = r;
  for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * F[a]) / r;
}

static double orc_feq(const orc_stencil* s, int i, double rho, const double u[3]) {
  double cu = s->c[i][0] * u[0] + s->c[i][1] * u[1] + s->c[i][2] * u[2];
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  double cs2 = 1.0 / 3.0;
  return s->w[i] * rho * (1.0 + cu / cs2 + (cu * cu) / (2.0 * cs2 * cs2) - uu / (2.0 * cs2));
}

/* Guo source term S_i = w_i [ (c_i - u)/cs^2 + (c_i.u) c_i / cs^4 ] . F */
static double orc_guo(const orc_stencil* s, int i, const double u[3], const double F[3]) {
  double cs2 = 1.0 / 3.0;
  double cu = s->c[i][0] * u[0] + s->c[i][1] * u[1] + s->c[i][2] * u[2];
  double acc = 0.0;
  for (int a = 0; a < 3; ++a)
    acc += ((s->c[i][a] - u[a]) / cs2 + cu * s->c[i][a] / (cs2 * cs2)) * F[a];
  return s->w[i] * acc;
}

static void orc_collide_srt(const orc_stencil* s, const orc_params* P, const double* f,
                            double* out) {
  double rho, u[3];
  orc_macros(s, f, P->force, &rho, u);
  double om = 1.0 / P->tau;
  for (int i = 0; i < s->q; ++i) {
    double feq = orc_feq(s, i, rho, u);
    double S = orc_guo(s, i, u, P->force);
    out[i] = f[i] - om * (f[i] - feq) + (1.0 - 0.5 * om) * S;
  }
}

/* Two-relaxation-time operator (Ginzburg): symmetric parts relax with
 * omega+ = 1/tau, antisymmetric parts with omega- chosen from the magic
 * parameter Lambda = (1/omega+ - 1/2)(1/omega- - 1/2).  The source term is
 * split the same way into its symmetric and antisymmetric halves. */
static void orc_collide_trt(const orc_stencil* s, const orc_params* P, const double* f,
                            double* out) {
  double rho, u[3];
  orc_macros(s, f, P->force, &rho, u);
  double omp = 1.0 / P->tau;
  double omm = 1.0 / (0.5 + P->magic / (P->tau - 0.5));
  double feq[27], S[27];
  for (int i = 0; i < s->q; ++i) {
    feq[i] = orc_feq(s, i, rho, u);
    S[i] = orc_guo(s, i, u, P->force);
  }
  for (int i = 0; i < s->q; ++i) {
    int o = s->opp[i];
    double fp = 0.5 * (f[i] + f[o]), fm = 0.5 * (f[i] - f[o]);
    double ep = 0.5 * (feq[i] + feq[o]), em = 0.5 * (feq[i] - feq[o]);
    double sp = 0.5 * (S[i] + S[o]), sm = 0.5 * (S[i] - S[o]);
    out[i] = f[i] - omp * (fp - ep) - omm * (fm - em) + (1.0 - 0.5 * omp) * sp +
             (1.0 - 0.5 * omm) * sm;
  }
}

/* Cumulant operator for D3Q27 (Geier et al. 2015, cited by the paper as the
 * cumulant model), in the fully specified variant used here: second-order
 * shear/deviatoric moments relax with omega1 = 1/tau, the trace with
 * omega_bulk, every cumulant of order >= 3 is set to zero (all higher rates
 * equal to one), no limiter.
 *
 *  a. central moments k_abc = sum_i f_i (cx-ux)^a (cy-uy)^b (cz-uz)^c,
 *     by direct 27-term sums;
 *  b. relax the second order;
 *  c. zero cumulants of order >= 3: odd orders vanish, even orders follow
 *     from the second-order moments (Isserlis / Wick relations);
 *  d. first order = F/2 so that the momentum gains F per step;
 *  e. back to populations through the exact inverse of the per-axis
 *     central-moment transform. */
static int orc_dir_of(const orc_stencil* s, int cx, int cy, int cz) {
  for (int i = 0; i < s->q; ++i)
    if (s->c[i][0] == cx && s->c[i][1] == cy && s->c[i][2] == cz) return i;
  return -1;
}

static double orc_ipow(double x, int n) {
  double r = 1.0;
  for (int k = 0; k < n; ++k) r *= x;
  return r;
}

/* Central moments k_abc about u by direct 27-term sums (step a). */
static void orc_central_moments(const orc_stencil* s, const double* f, const double u[3],
                                double k[3][3][3]) {
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      for (int c = 0; c < 3; ++c) {
        double acc = 0.0;
        for (int i = 0; i < s->q; ++i)
          acc += f[i] * orc_ipow(s->c[i][0] - u[0], a) * orc_ipow(s->c[i][1] - u[1], b) *
                 orc_ipow(s->c[i][2] - u[2], c);
        k[a][b][c] = acc;
      }
}

/* Orders 0-2 after collision (steps b, d): density, F/2, and the second
 * order with off-diagonal and deviatoric parts at omega1 = 1/tau, the trace
 * towards rho at omega_bulk. */
static void orc_relax_low_orders(const orc_params* P, double rho, double k[3][3][3],
                                 double p[3][3][3]) {
  double w1 = 1.0 / P->tau, w2 = P->omega_bulk;
  memset(p, 0, sizeof(double) * 27);
  p[0][0][0] = rho;
  p[1][0][0] = 0.5 * P->force[0];
  p[0][1][0] = 0.5 * P->force[1];
  p[0][0][1] = 0.5 * P->force[2];
  p[1][1][0] = (1.0 - w1) * k[1][1][0];
  p[1][0][1] = (1.0 - w1) * k[1][0][1];
  p[0][1][1] = (1.0 - w1) * k[0][1][1];
  double dxy = (1.0 - w1) * (k[2][0][0] - k[0][2][0]);
  double dxz = (1.0 - w1) * (k[2][0][0] - k[0][0][2]);
  double tr = k[2][0][0] + k[0][2][0] + k[0][0][2];
  tr = tr + w2 * (rho - tr);
  p[2][0][0] = (dxy + dxz + tr) / 3.0;
  p[0][2][0] = (tr - 2.0 * dxy + dxz) / 3.0;
  p[0][0][2] = (tr + dxy - 2.0 * dxz) / 3.0;
}

static void orc_central_inverse(const orc_stencil* s, double p[3][3][3], const double u[3],
                                double* out);

static void orc_collide_cumulant(const orc_stencil* s, const orc_params* P, const double* f,
                                 double* out) {
  double rho, u[3];
  orc_macros(s, f, P->force, &rho, u);
  double k[3][3][3], p[3][3][3];
  orc_central_moments(s, f, u, k);
  orc_relax_low_orders(P, rho, k, p);
  double p110 = p[1][1][0], p101 = p[1][0][1], p011 = p[0][1][1];
  double p200 = p[2][0][0], p020 = p[0][2][0], p002 = p[0][0][2];
  /* order 3 and 5: zero (already). order 4: */
  p[2][2][0] = (p200 * p020 + 2.0 * p110 * p110) / rho;
  p[2][0][2] = (p200 * p002 + 2.0 * p101 * p101) / rho;
  p[0][2][2] = (p020 * p002 + 2.0 * p011 * p011) / rho;
  p[2][1][1] = (p200 * p011 + 2.0 * p110 * p101) / rho;
  p[1][2][1] = (p020 * p101 + 2.0 * p110 * p011) / rho;
  p[1][1][2] = (p002 * p110 + 2.0 * p101 * p011) / rho;
  /* order 6 */
  p[2][2][2] = (p200 * p020 * p002 +
                2.0 * (p110 * p110 * p002 + p101 * p101 * p020 + p011 * p011 * p200) +
                8.0 * p110 * p101 * p011) /
               (rho * rho);
  orc_central_inverse(s, p, u, out);
}

/* Step e: exact inverse, one axis at a time: central (k0,k1,k2) about v ->
 * raw (m0,m1,m2) -> values at c = -1, 0, +1, stored at position c+1. */
static void orc_central_inverse(const orc_stencil* s, double p[3][3][3], const double u[3],
                                double* out) {
  double g[3][3][3];
  /* z axis: p[a][b][n] -> g[a][b][cz+1] */
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double v = u[2];
      double m0 = p[a][b][0];
      double m1 = p[a][b][1] + v * p[a][b][0];
      double m2 = p[a][b][2] + 2.0 * v * p[a][b][1] + v * v * p[a][b][0];
      g[a][b][1] = m0 - m2;
      g[a][b][2] = 0.5 * (m2 + m1);
      g[a][b][0] = 0.5 * (m2 - m1);
    }
  double h[3][3][3];
  for (int a = 0; a < 3; ++a)
    for (int z = 0; z < 3; ++z) {
      double v = u[1];
      double m0 = g[a][0][z];
      double m1 = g[a][1][z] + v * g[a][0][z];
      double m2 = g[a][2][z] + 2.0 * v * g[a][1][z] + v * v * g[a][0][z];
      h[a][1][z] = m0 - m2;
      h[a][2][z] = 0.5 * (m2 + m1);
      h[a][0][z] = 0.5 * (m2 - m1);
    }
  double r[3][3][3];
  for (int y = 0; y < 3; ++y)
    for (int z = 0; z < 3; ++z) {
      double v = u[0];
      double m0 = h[0][y][z];
      double m1 = h[1][y][z] + v * h[0][y][z];
      double m2 = h[2][y][z] + 2.0 * v * h[1][y][z] + v * v * h[0][y][z];
      r[1][y][z] = m0 - m2;
      r[2][y][z] = 0.5 * (m2 + m1);
      r[0][y][z] = 0.5 * (m2 - m1);
    }
  for (int x = 0; x < 3; ++x)
    for (int y = 0; y < 3; ++y)
      for (int z = 0; z < 3; ++z) {
        int i = orc_dir_of(s, x - 1, y - 1, z - 1);
        out[i] = r[x][y][z];
      }
}

/* Central-moment operator for D3Q27 (the paper names the central-moment
 * operator among its collision models; the complete per-axis central-moment
 * basis exists on D3Q27).  Central moments about the local velocity:
 * orders 0-2 exactly as the cumulant operator (density, F/2, shear at
 * 1/tau, trace at omega_bulk); every central moment of order n = 3..6
 * relaxes towards the central moment of the Maxwellian,
 *   k^eq_abc = rho e(a) e(b) e(c),  e(0) = 1, e(1) = 0, e(2) = 1/3,
 * with rate rates[n - 3]; back to populations by the exact inverse. */
static void orc_collide_cm(const orc_stencil* s, const orc_params* P, const double* f,
                           double* out) {
  double rho, u[3];
  orc_macros(s, f, P->force, &rho, u);
  double k[3][3][3], p[3][3][3];
  orc_central_moments(s, f, u, k);
  orc_relax_low_orders(P, rho, k, p);
  const double e[3] = {1.0, 0.0, 1.0 / 3.0};
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      for (int c = 0; c < 3; ++c) {
        int n = a + b + c;
        if (n < 3) continue;
        double keq = rho * e[a] * e[b] * e[c];
        double sn = P->rates[n - 3];
        p[a][b][c] = k[a][b][c] - sn * (k[a][b][c] - keq);
      }
  orc_central_inverse(s, p, u, out);
}

/* Multiple-relaxation-time operator for D3Q19 (the paper lists MRT with
 * the classical operators, Section "Lattice Boltzmann Method"; moment basis
 * of d'Humieres et al. 2002).  The 19 moments are the polynomials below in
 * the lattice velocity; they are mutually orthogonal over the D3Q19 set, so
 * M^-1 = M^T diag(1 / |row|^2).  Every moment relaxes toward the moment of
 * the same second-order equilibrium the SRT/TRT operators use, with its own
 * rate; Guo's source enters in moment space with weight (1 - s/2).
 * Rates: density and momentum are conserved (rate irrelevant, 1 used);
 * energy e: omega_bulk; epsilon: rates[0]; the shear moments 3p_xx, p_ww,
 * p_xy, p_yz, p_xz: 1/tau; pi_xx, pi_ww: rates[1]; energy flux q:
 * rates[2]; third-order m: rates[3]. */
static double orc_mrt_poly(int k, const int c[3]) {
  double x = c[0], y = c[1], z = c[2], c2 = x * x + y * y + z * z;
  switch (k) {
    case 0: return 1.0;
    case 1: return 19.0 * c2 - 30.0;
    case 2: return (21.0 * c2 * c2 - 53.0 * c2 + 24.0) / 2.0;
    case 3: return x;
    case 4: return (5.0 * c2 - 9.0) * x;
    case 5: return y;
    case 6: return (5.0 * c2 - 9.0) * y;
    case 7: return z;
    case 8: return (5.0 * c2 - 9.0) * z;
    case 9: return 3.0 * x * x - c2;
    case 10: return (3.0 * c2 - 5.0) * (3.0 * x * x - c2);
    case 11: return y * y - z * z;
    case 12: return (3.0 * c2 - 5.0) * (y * y - z * z);
    case 13: return x * y;
    case 14: return y * z;
    case 15: return x * z;
    case 16: return (y * y - z * z) * x;
    case 17: return (z * z - x * x) * y;
    default: return (x * x - y * y) * z;
  }
}

static double orc_mrt_rate(const orc_params* P, int k) {
  switch (k) {
    case 0: case 3: case 5: case 7: return 1.0;
    case 1: return P->omega_bulk;
    case 2: return P->rates[0];
    case 9: case 11: case 13: case 14: case 15: return 1.0 / P->tau;
    case 10: case 12: return P->rates[1];
    case 4: case 6: case 8: return P->rates[2];
    default: return P->rates[3];
  }
}

static void orc_collide_mrt(const orc_stencil* s, const orc_params* P, const double* f,
                            double* out) {
  double rho, u[3];
  orc_macros(s, f, P->force, &rho, u);
  /* equilibrium, Guo source and squared row norms, each computed once */
  double feq[19], src[19], norm[19];
  for (int i = 0; i < 19; ++i) {
    feq[i] = orc_feq(s, i, rho, u);
    src[i] = orc_guo(s, i, u, P->force);
  }
  for (int k = 0; k < 19; ++k) {
    norm[k] = 0.0;
    for (int j = 0; j < 19; ++j) norm[k] += orc_mrt_poly(k, s->c[j]) * orc_mrt_poly(k, s->c[j]);
  }
  double mstar[19];
  for (int k = 0; k < 19; ++k) {
    double m = 0.0, meq = 0.0, ms = 0.0;
    for (int i = 0; i < 19; ++i) {
      double pk = orc_mrt_poly(k, s->c[i]);
      m += pk * f[i];
      meq += pk * feq[i];
      ms += pk * src[i];
    }
    double sk = orc_mrt_rate(P, k);
    mstar[k] = m - sk * (m - meq) + (1.0 - 0.5 * sk) * ms;
  }
  for (int i = 0; i < 19; ++i) {
    double acc = 0.0;
    for (int k = 0; k < 19; ++k) acc += orc_mrt_poly(k, s->c[i]) * mstar[k] / norm[k];
    out[i] = acc;
  }
}

/* Moment matrix of the MRT basis (row k, column i) for tests. */
int orc_mrt_matrix(double* M) {
  orc_stencil s;
  if (orc_stencil_init(&s, 19)) return -1;
  for (int k = 0; k < 19; ++k)
    for (int i = 0; i < 19; ++i) M[k * 19 + i] = orc_mrt_poly(k, s.c[i]);
  return 0;
}

static void orc_collide(const orc_stencil* s, const orc_params* P, const double* f,
                        double* out) {
  switch (P->kind) {
    case ORC_SRT: orc_collide_srt(s, P, f, out); break;
    case ORC_TRT: orc_collide_trt(s, P, f, out); break;
    case ORC_CUMULANT: orc_collide_cumulant(s, P, f, out); break;
    case ORC_MRT: orc_collide_mrt(s, P, f, out); break;
    case ORC_CM: orc_collide_cm(s, P, f, out); break;
    default:
      for (int i = 0; i < s->q; ++i) out[i] = f[i];
  }
}

/* Batch collision for unit tests: f_in/f_out are [n][q]. */
int orc_collide_cells(const orc_params* P, int64_t n, const double* f_in, double* f_out) {
  orc_stencil s;
  if (orc_stencil_init(&s, P->q)) return -1;
  if ((P->kind == ORC_CUMULANT || P->kind == ORC_CM) && P->q != 27) return -1;
  if (P->kind == ORC_MRT && P->q != 19) return -1;
  for (int64_t k = 0; k < n; ++k) orc_collide(&s, P, f_in + k * s.q, f_out + k * s.q);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Boundary rule for one pulled population (Section "Sparse Boundary    */
/* Conditions" describes no-slip and velocity bounce-back; the pressure */
/* outlet is this build's reading).  `own_opp` is the cell's own        */
/* post-collision population in the opposite direction and u the       */
/* cell's velocity at the same time (orc_cell_velocity; read for        */
/* pressure only).  Labels: 0 fluid, 1 solid (halfway bounce-back), 2+c */
/* boundary class c.  UBB: moving-wall bounce-back with rho_w = 1;      */
/* pressure: anti-bounce-back,                                          */
/*   f_i = -own_opp + 2 w_i rho_out (1 + 9/2 (c_i.u)^2 - 3/2 u.u),       */
/* i.e. the sum of the two opposite second-order equilibria at          */
/* (rho_out, u), so a cell in equilibrium at rho_out gets the           */
/* equilibrium back.                                                    */
/* ------------------------------------------------------------------ */

/* rho = sum f*, u = (sum c f* - F/2) / rho of one cell's post-collision
 * populations (the velocity the moments output reports). */
static void orc_cell_velocity(const orc_stencil* s, const orc_params* P, const double* fs,
                              double u[3]) {
  double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < s->q; ++a) {
    rho += fs[a];
    for (int d = 0; d < 3; ++d) j[d] += s->c[a][d] * fs[a];
  }
  for (int d = 0; d < 3; ++d) u[d] = (j[d] - 0.5 * P->force[d]) / rho;
}

static double orc_wall_value(const orc_stencil* s, const orc_params* P, int i, int label,
                             double own_opp, const double u[3]) {
  if (label <= 1) return own_opp;
  int cls = label - 2;
  if (cls >= P->n_classes) return own_opp;
  int type = P->cls_type[cls];
  if (type == ORC_BC_UBB) {
    double cu = s->c[i][0] * P->cls_u[cls][0] + s->c[i][1] * P->cls_u[cls][1] +
                s->c[i][2] * P->cls_u[cls][2];
    return own_opp + 6.0 * s->w[i] * 1.0 * cu;
  }
  if (type == ORC_BC_PRESSURE) {
    double cu = s->c[i][0] * u[0] + s->c[i][1] * u[1] + s->c[i][2] * u[2];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return -own_opp + 2.0 * s->w[i] * P->cls_rho[cls] * (1.0 + 4.5 * cu * cu - 1.5 * uu);
  }
  return own_opp;
}

/* Neighbour of (x,y,z) displaced by d; returns -1 when it leaves the box
 * through a non-periodic face (treated as solid), otherwise its linear id. */
static int64_t orc_neighbour(int x, int y, int z, int dx, int dy, int dz, int nx, int ny, int nz,
                             uint32_t periodic) {
  int p[3] = {x + dx, y + dy, z + dz};
  int n[3] = {nx, ny, nz};
  for (int a = 0; a < 3; ++a) {
    if (p[a] < 0 || p[a] >= n[a]) {
      if (!((periodic >> a) & 1u)) return -1;
      p[a] = (p[a] + n[a]) % n[a];
    }
  }
  return (int64_t)p[0] + (int64_t)nx * ((int64_t)p[1] + (int64_t)ny * (int64_t)p[2]);
}

/* ------------------------------------------------------------------ */
/* 1. Dense two-array pull scheme over all box cells.                    */
/* A and B are [q][N] with N = nx*ny*nz, x fastest.  A holds the        */
/* post-collision state at time t; B receives the state at t+1.         */
/* Non-fluid cells are copied unchanged.                                 */
/* ------------------------------------------------------------------ */

int orc_dense_step(const orc_params* P, const uint8_t* labels, int nx, int ny, int nz,
                   uint32_t periodic, const double* A, double* B) {
  orc_stencil s;
  if (orc_stencil_init(&s, P->q)) return -1;
  if ((P->kind == ORC_CUMULANT || P->kind == ORC_CM) && P->q != 27) return -1;
  if (P->kind == ORC_MRT && P->q != 19) return -1;
  const int64_t N = (int64_t)nx * ny * nz;
  const int q = s.q;
#pragma omp parallel for schedule(static) if ((int64_t)nx * ny * nz >= ORC_PAR_MIN)
  for (int z = 0; z < nz; ++z) {
    double f[27], fs[27];
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        int64_t lin = (int64_t)x + (int64_t)nx * ((int64_t)y + (int64_t)ny * z);
        if (labels[lin] != 0) {
          for (int i = 0; i < q; ++i) B[i * N + lin] = A[i * N + lin];
          continue;
        }
        /* the cell's own velocity at time t, for pressure outlets */
        double own[27], u[3];
        for (int i = 0; i < q; ++i) own[i] = A[i * N + lin];
        orc_cell_velocity(&s, P, own, u);
        f[0] = A[lin];
        for (int i = 1; i < q; ++i) {
          /* pull: f_i(x) comes from x - c_i */
          int64_t y_lin = orc_neighbour(x, y, z, -s.c[i][0], -s.c[i][1], -s.c[i][2], nx, ny,
                                        nz, periodic);
          int lab = (y_lin < 0) ? 1 : labels[y_lin];
          if (lab == 0)
            f[i] = A[i * N + y_lin];
          else
            f[i] = orc_wall_value(&s, P, i, lab, A[s.opp[i] * N + lin], u);
        }
        orc_collide(&s, P, f, fs);
        for (int i = 0; i < q; ++i) B[i * N + lin] = fs[i];
      }
  }
  return 0;
}

/* Runs n steps; A is both input and output; B is scratch of the same size. */
int orc_dense_run(const orc_params* P, const uint8_t* labels, int nx, int ny, int nz,
                  uint32_t periodic, int64_t n_steps, double* A, double* B) {
  const int64_t N = (int64_t)nx * ny * nz;
  for (int64_t t = 0; t < n_steps; ++t) {
    int rc = orc_dense_step(P, labels, nx, ny, nz, periodic, A, B);
    if (rc) return rc;
    memcpy(A, B, sizeof(double) * (size_t)(P->q) * (size_t)N);
  }
  return 0;
}

/* Equilibrium initialisation of every fluid cell (solid cells get the
 * rest weights so that the arrays are fully defined). */
int orc_dense_init(int q, const uint8_t* labels, int64_t N, double rho0, const double u0[3],
                   double* A) {
  orc_stencil s;
  if (orc_stencil_init(&s, q)) return -1;
  for (int i = 0; i < q; ++i) {
    const double feq = orc_feq(&s, i, rho0, u0);
#pragma omp parallel for schedule(static) if (N >= ORC_PAR_MIN)
    for (int64_t lin = 0; lin < N; ++lin) A[i * N + lin] = labels[lin] == 0 ? feq : s.w[i];
  }
  return 0;
}

/* Macroscopic output of a post-collision state: rho = sum f*,
 * u = (sum c f* - F/2) / rho.  Non-fluid cells get rho = 0, u = 0. */
int orc_dense_moments(const orc_params* P, const uint8_t* labels, int64_t N, const double* A,
                      double* rho_out, double* u_out /* [3][N] */) {
  orc_stencil s;
  if (orc_stencil_init(&s, P->q)) return -1;
  for (int64_t lin = 0; lin < N; ++lin) {
    if (labels[lin] != 0) {
      rho_out[lin] = 0.0;
      for (int a = 0; a < 3; ++a) u_out[a * N + lin] = 0.0;
      continue;
    }
    double r = 0.0, j[3] = {0, 0, 0};
    for (int i = 0; i < s.q; ++i) {
      r += A[i * N + lin];
      for (int a = 0; a < 3; ++a) j[a] += s.c[i][a] * A[i * N + lin];
    }
    rho_out[lin] = r;
    for (int a = 0; a < 3; ++a) u_out[a * N + lin] = (j[a] - 0.5 * P->force[a]) / r;
  }
  return 0;
}

/* Kahan-compensated sums over fluid cells, in linear-id order:
 * out[0] = mass sum rho, out[1..3] = sum rho*u, out[4] = fluid cell count. */
int orc_dense_reduce(const orc_params* P, const uint8_t* labels, int64_t N, const double* A,
                     double* out) {
  orc_stencil s;
  if (orc_stencil_init(&s, P->q)) return -1;
  double sum[4] = {0, 0, 0, 0}, comp[4] = {0, 0, 0, 0};
  int64_t nf = 0;
  for (int64_t lin = 0; lin < N; ++lin) {
    if (labels[lin] != 0) continue;
    ++nf;
    double v[4] = {0, 0, 0, 0};
    for (int i = 0; i < s.q; ++i) {
      v[0] += A[i * N + lin];
      for (int a = 0; a < 3; ++a) v[1 + a] += s.c[i][a] * A[i * N + lin];
    }
    for (int a = 0; a < 3; ++a) v[1 + a] -= 0.5 * P->force[a];
    for (int m = 0; m < 4; ++m) {
      double yk = v[m] - comp[m];
      double tk = sum[m] + yk;
      comp[m] = (tk - sum[m]) - yk;
      sum[m] = tk;
    }
  }
  for (int m = 0; m < 4; ++m) out[m] = sum[m];
  out[4] = (double)nf;
  return 0;
}

/* ------------------------------------------------------------------ */
/* 2. Sparse CPU variant: own builder + in-place AA streaming.           */
/* ------------------------------------------------------------------ */

/* Morton key: bit b of x, y, z goes to bit 3b, 3b+1, 3b+2 (x lowest). */
uint64_t orc_morton_key(uint32_t x, uint32_t y, uint32_t z) {
  uint64_t key = 0;
  for (int b = 0; b < 21; ++b) {
    key |= (uint64_t)((x >> b) & 1u) << (3 * b);
    key |= (uint64_t)((y >> b) & 1u) << (3 * b + 1);
    key |= (uint64_t)((z >> b) & 1u) << (3 * b + 2);
  }
  return key;
}

/* Blocked order: blocks of nx*8*8 cells (whole x rows), visited in 2-D
 * Morton order of (y/8, z/8) with y at bit 2b and z at bit 2b+1; inside a
 * block x fastest, then y, then z. */
uint64_t orc_blocked_key(uint32_t x, uint32_t y, uint32_t z, uint32_t nx) {
  uint32_t ty = y / 8, tz = z / 8, ly = y % 8, lz = z % 8;
  uint64_t t = 0;
  for (int b = 0; b < 16; ++b) {
    t |= (uint64_t)((ty >> b) & 1u) << (2 * b);
    t |= (uint64_t)((tz >> b) & 1u) << (2 * b + 1);
  }
  return t * ((uint64_t)nx * 64) + x + (uint64_t)nx * (ly + 8 * lz);
}

typedef struct {
  uint64_t key;
  int64_t lin;
} orc_keyed;

static int orc_keyed_cmp(const void* a, const void* b) {
  const orc_keyed* x = (const orc_keyed*)a;
  const orc_keyed* y = (const orc_keyed*)b;
  if (x->key < y->key) return -1;
  if (x->key > y->key) return 1;
  return 0;
}

/* Sparse list construction (Section "Sparse Data Structure"):
 *   cells[k]          linear id of the k-th fluid cell (order 0: Morton,
 *                     order 1: ascending linear id, order 2: blocked);
 *   index[(i-1)*S+k]  for direction i >= 1, the PDF-list position cell k
 *                     pulls population i from: i*S + m when the upstream
 *                     cell x_k - c_i is fluid with list index m, otherwise
 *                     opp(i)*S + k (bounce-back folded into the table);
 *   links[2*l]        = position opp(i)*S + k, links[2*l+1] = i | class<<8,
 *                     for every upstream cell carrying a boundary class,
 *                     ordered by (k, i).
 * S = n_fluid rounded up to a multiple of `align`.
 * Call with cells == NULL to obtain n_fluid, stride and n_links only. */
int orc_sparse_build(const uint8_t* labels, int nx, int ny, int nz, uint32_t periodic, int q,
                     int order, int align, int64_t* n_fluid, int64_t* stride, int64_t* n_links,
                     int32_t* cells, int32_t* index, int32_t* links) {
  orc_stencil s;
  if (orc_stencil_init(&s, q) || align < 1 || order < 0 || order > 2) return -1;
  const int64_t N = (int64_t)nx * ny * nz;
  int64_t nf = 0;
  for (int64_t lin = 0; lin < N; ++lin) nf += labels[lin] == 0;
  int64_t S = ((nf + align - 1) / align) * align;
  /* links count */
  int64_t nl = 0;
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        int64_t lin = (int64_t)x + (int64_t)nx * ((int64_t)y + (int64_t)ny * z);
        if (labels[lin] != 0) continue;
        for (int i = 1; i < q; ++i) {
          int64_t yl = orc_neighbour(x, y, z, -s.c[i][0], -s.c[i][1], -s.c[i][2], nx, ny, nz,
                                     periodic);
          if (yl >= 0 && labels[yl] >= 2) ++nl;
        }
      }
  *n_fluid = nf;
  *stride = S;
  *n_links = nl;
  if (!cells) return 0;

  orc_keyed* kv = (orc_keyed*)malloc(sizeof(orc_keyed) * (size_t)(nf > 0 ? nf : 1));
  int32_t* inv = (int32_t*)malloc(sizeof(int32_t) * (size_t)(N > 0 ? N : 1));
  if (!kv || !inv) {
    free(kv);
    free(inv);
    return -3;
  }
  int64_t k = 0;
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        int64_t lin = (int64_t)x + (int64_t)nx * ((int64_t)y + (int64_t)ny * z);
        if (labels[lin] != 0) continue;
        kv[k].lin = lin;
        kv[k].key = order == 0   ? orc_morton_key((uint32_t)x, (uint32_t)y, (uint32_t)z)
                    : order == 2 ? orc_blocked_key((uint32_t)x, (uint32_t)y, (uint32_t)z,
                                                   (uint32_t)nx)
                                 : (uint64_t)lin;
        ++k;
      }
  qsort(kv, (size_t)nf, sizeof(orc_keyed), orc_keyed_cmp);
  for (int64_t lin = 0; lin < N; ++lin) inv[lin] = -1;
  for (k = 0; k < nf; ++k) {
    cells[k] = (int32_t)kv[k].lin;
    inv[kv[k].lin] = (int32_t)k;
  }
  int64_t l = 0;
  for (k = 0; k < nf; ++k) {
    int64_t lin = kv[k].lin;
    int x = (int)(lin % nx), y = (int)((lin / nx) % ny), z = (int)(lin / ((int64_t)nx * ny));
    for (int i = 1; i < q; ++i) {
      int64_t yl = orc_neighbour(x, y, z, -s.c[i][0], -s.c[i][1], -s.c[i][2], nx, ny, nz,
                                 periodic);
      int lab = yl < 0 ? 1 : labels[yl];
      int64_t pos;
      if (lab == 0)
        pos = (int64_t)i * S + inv[yl];
      else
        pos = (int64_t)s.opp[i] * S + k;
      index[(int64_t)(i - 1) * S + k] = (int32_t)pos;
      if (lab >= 2) {
        links[2 * l] = (int32_t)((int64_t)s.opp[i] * S + k);
        links[2 * l + 1] = i | ((lab - 2) << 8);
        ++l;
      }
    }
  }
  for (k = nf; k < S; ++k)
    for (int i = 1; i < q; ++i) index[(int64_t)(i - 1) * S + k] = -1;
  free(kv);
  free(inv);
  return 0;
}

/* Boundary-link update applied before every AA step: the slot that will be
 * pulled across a boundary link gets the wall rule of orc_wall_value
 * applied to the value it currently holds (the cell's own opposite-direction
 * population, in both parities).  The velocity of every link's cell is
 * taken first, from the state before any link of this step is applied
 * (as the dense scheme reads it from the unmodified previous array): the
 * cell's post-collision populations sit in its natural slots at even t and
 * where it pulled the opposite populations from at odd t. */
static int orc_sparse_links(const orc_stencil* s, const orc_params* P, int64_t n_links,
                            const int32_t* links, double* pdf, int64_t S,
                            const int32_t* index, int64_t t) {
  if (n_links <= 0) return 0;
  double* uu = (double*)malloc(sizeof(double) * 3 * (size_t)n_links);
  if (!uu) return -1;
  for (int64_t l = 0; l < n_links; ++l) {
    int i = links[2 * l + 1] & 0xff;
    int64_t k = links[2 * l] - (int64_t)s->opp[i] * S;
    double fs[27];
    for (int a = 0; a < s->q; ++a)
      fs[a] = ((t & 1) == 0 || a == 0) ? pdf[(int64_t)a * S + k]
                                       : pdf[index[(int64_t)(s->opp[a] - 1) * S + k]];
    orc_cell_velocity(s, P, fs, uu + 3 * l);
  }
  for (int64_t l = 0; l < n_links; ++l) {
    int64_t pos = links[2 * l];
    int i = links[2 * l + 1] & 0xff;
    int cls = (links[2 * l + 1] >> 8) & 0xff;
    pdf[pos] = orc_wall_value(s, P, i, cls + 2, pdf[pos], uu + 3 * l);
  }
  free(uu);
  return 0;
}

/* One AA step (Section "In-place Streaming: AA Pattern").
 * t even ("odd" step of the paper): gather f_i = pdf[index_i(k)], collide,
 *   write the opposite population back to where f_i came from;
 * t odd ("even" step): f_i = pdf[opp(i)*S + k], collide, f*_i -> pdf[i*S+k]. */
int orc_sparse_step(const orc_params* P, int64_t n_fluid, int64_t S, const int32_t* index,
                    int64_t n_links, const int32_t* links, int64_t t, double* pdf) {
  orc_stencil s;
  if (orc_stencil_init(&s, P->q)) return -1;
  if ((P->kind == ORC_CUMULANT || P->kind == ORC_CM) && P->q != 27) return -1;
  if (P->kind == ORC_MRT && P->q != 19) return -1;
  const int q = s.q;
  if (orc_sparse_links(&s, P, n_links, links, pdf, S, index, t)) return -1;
  if ((t & 1) == 0) {
#pragma omp parallel for schedule(static) if (n_fluid >= ORC_PAR_MIN)
    for (int64_t k = 0; k < n_fluid; ++k) {
      double f[27], fs[27];
      int64_t pos[27];
      pos[0] = k;
      for (int i = 1; i < q; ++i) pos[i] = index[(int64_t)(i - 1) * S + k];
      for (int i = 0; i < q; ++i) f[i] = pdf[pos[i]];
      orc_collide(&s, P, f, fs);
      for (int i = 0; i < q; ++i) pdf[pos[i]] = fs[s.opp[i]];
    }
  } else {
#pragma omp parallel for schedule(static) if (n_fluid >= ORC_PAR_MIN)
    for (int64_t k = 0; k < n_fluid; ++k) {
      double f[27], fs[27];
      for (int i = 0; i < q; ++i) f[i] = pdf[(int64_t)s.opp[i] * S + k];
      orc_collide(&s, P, f, fs);
      for (int i = 0; i < q; ++i) pdf[(int64_t)i * S + k] = fs[i];
    }
  }
  return 0;
}

/* Post-collision populations of cell k at time t in natural order, whatever
 * the parity: at even t they sit in the natural slots; at odd t population
 * j of cell k sits where direction opp(j) of cell k was pulled from. */
int orc_sparse_gather(int q, int64_t n_fluid, int64_t S, const int32_t* index, int64_t t,
                      const double* pdf, double* out /* [q][n_fluid] */) {
  orc_stencil s;
  if (orc_stencil_init(&s, q)) return -1;
  for (int64_t k = 0; k < n_fluid; ++k) {
    for (int j = 0; j < q; ++j) {
      double v;
      if ((t & 1) == 0 || j == 0)
        v = pdf[(int64_t)j * S + k];
      else
        v = pdf[index[(int64_t)(s.opp[j] - 1) * S + k]];
      out[(int64_t)j * n_fluid + k] = v;
    }
  }
  return 0;
}
