/* Exercises every entry point of the oracle in one process so that the
 * CPU test suite can run it under AddressSanitizer and
 * UndefinedBehaviorSanitizer: dense pull runs and sparse AA runs for each
 * stencil, collision kind and periodicity on a small random mask with
 * velocity and pressure classes, the builder's two phases, parity-aware
 * gathers, moments, reductions, single-cell collisions and the MRT matrix.
 * It also checks that sparse AA equals dense pull after an even number of
 * steps.  Exit status 0 on success. */
#include "../../oracle/lbm_oracle.c"

#include <stdio.h>

static uint32_t g_rng = 2408u;
static uint32_t next_u32(void) {
  g_rng = g_rng * 1664525u + 1013904223u;
  return g_rng >> 8;
}

static int run_case(int q, int kind, uint32_t periodic, int order, const uint8_t* lab, int nx,
                    int ny, int nz, double* worst) {
  const int64_t N = (int64_t)nx * ny * nz;
  orc_params P;
  memset(&P, 0, sizeof(P));
  P.q = q;
  P.kind = kind;
  P.tau = 0.8;
  P.magic = 3.0 / 16.0;
  P.omega_bulk = 1.1;
  for (int a = 0; a < 4; ++a) P.rates[a] = 1.1 + 0.1 * a;
  P.force[0] = 1e-4;
  P.force[1] = -2e-5;
  P.n_classes = 2;
  P.cls_type[0] = ORC_BC_UBB;
  P.cls_u[0][2] = 0.01;
  P.cls_type[1] = ORC_BC_PRESSURE;
  P.cls_rho[1] = 1.001;
  const double u0[3] = {0.01, 0.0, -0.005};
  double* A = malloc(sizeof(double) * q * N);
  double* B = malloc(sizeof(double) * q * N);
  if (!A || !B || orc_dense_init(q, lab, N, 1.0, u0, A)) return 1;
  int64_t nf = 0, S = 0, nl = 0;
  if (orc_sparse_build(lab, nx, ny, nz, periodic, q, order, 8, &nf, &S, &nl, NULL, NULL, NULL))
    return 2;
  int32_t* cells = malloc(sizeof(int32_t) * (nf > 0 ? nf : 1));
  int32_t* index = malloc(sizeof(int32_t) * (q - 1) * (S > 0 ? S : 1));
  int32_t* links = malloc(sizeof(int32_t) * 2 * (nl > 0 ? nl : 1));
  double* pdf = calloc((size_t)q * (S > 0 ? S : 1), sizeof(double));
  double* got = malloc(sizeof(double) * q * (nf > 0 ? nf : 1));
  if (!cells || !index || !links || !pdf || !got) return 3;
  if (orc_sparse_build(lab, nx, ny, nz, periodic, q, order, 8, &nf, &S, &nl, cells, index, links))
    return 4;
  for (int i = 0; i < q; ++i)
    for (int64_t k = 0; k < nf; ++k) pdf[(int64_t)i * S + k] = A[(int64_t)i * N + cells[k]];
  const int steps = 6;
  for (int t = 0; t < steps; ++t) {
    if (orc_sparse_step(&P, nf, S, index, nl, links, t, pdf)) return 5;
    if (orc_sparse_gather(q, nf, S, index, t + 1, pdf, got)) return 6;
  }
  if (orc_dense_run(&P, lab, nx, ny, nz, periodic, steps, A, B)) return 7;
  for (int i = 0; i < q; ++i)
    for (int64_t k = 0; k < nf; ++k) {
      const double d = fabs(got[(int64_t)i * nf + k] - A[(int64_t)i * N + cells[k]]);
      if (!(d <= *worst)) *worst = d;
    }
  double* rho = malloc(sizeof(double) * N);
  double* u = malloc(sizeof(double) * 3 * N);
  double red[8];
  if (!rho || !u || orc_dense_moments(&P, lab, N, A, rho, u) || orc_dense_reduce(&P, lab, N, A, red))
    return 8;
  double fin[27], fout[27];
  for (int i = 0; i < q; ++i) fin[i] = A[(int64_t)i * N + (nf > 0 ? cells[0] : 0)];
  if (orc_collide_cells(&P, 1, fin, fout)) return 9;
  free(A); free(B); free(cells); free(index); free(links); free(pdf); free(got); free(rho); free(u);
  return 0;
}

int main(void) {
  const int nx = 9, ny = 8, nz = 7;
  uint8_t lab[9 * 8 * 7];
  for (int i = 0; i < nx * ny * nz; ++i) {
    const uint32_t r = next_u32() % 100u;
    lab[i] = r < 68 ? 0 : (r < 90 ? 1 : (r < 95 ? 2 : 3));
  }
  double M[19 * 19];
  if (orc_mrt_matrix(M)) return 10;
  int32_t c[27 * 3], opp[27];
  double w[27];
  if (orc_stencil_tables(27, c, w, opp)) return 11;
  const int kinds19[] = {ORC_NONE, ORC_SRT, ORC_TRT, ORC_MRT};
  const int kinds27[] = {ORC_NONE, ORC_SRT, ORC_TRT, ORC_CUMULANT, ORC_CM};
  double worst = 0.0;
  for (int order = 0; order < 3; ++order)
    for (uint32_t per = 0; per < 8; per += 7) {
      for (int j = 0; j < 4; ++j) {
        const int rc = run_case(19, kinds19[j], per, order, lab, nx, ny, nz, &worst);
        if (rc) return 20 + rc;
      }
      for (int j = 0; j < 5; ++j) {
        const int rc = run_case(27, kinds27[j], per, order, lab, nx, ny, nz, &worst);
        if (rc) return 40 + rc;
      }
    }
  printf("max |sparse AA - dense pull| after 6 steps: %.3e\n", worst);
  return worst <= 1e-12 ? 0 : 60;
}
