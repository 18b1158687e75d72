// Cumulant collision for D3Q27 in deviation form (Geier et al. 2015, the
// cumulant model the paper names among its operators): second-order
// off-diagonal and deviatoric central moments relax with om1 = 1/tau, the
// trace relaxes towards rho with om2, every cumulant of order >= 3 is set to
// zero (all higher rates one), first-order central moments become F/2.
//
// Conditioning.  The stored deviations d = f - w are transformed to central
// moments K^d about u with the per-axis ("chimera") transform.  The central
// moments of the rest weights are known in closed form,
//     K^w_abc = k(a,ux) k(b,uy) k(c,uz),  k(0,u) = 1, k(1,u) = -u,
//     k(2,u) = 1/3 + u^2,
// so the full moments are K = K^w + K^d.  The post-collision moments K* are
// written as deviations D* = K* - K^w using only small quantities (drho, u,
// K^d), and the exact inverse transform of D* yields d* = f* - w, because
// the inverse transform of K^w is w itself.  No O(1) quantity is ever
// subtracted from another in FP32.
#pragma once

#include "collide.hpp"

namespace lbm {

// Forward per-axis transform of the values at c = -1, 0, +1 (slots 0, 1, 2)
// into central moments of order 0, 1, 2 about v.
template <class R>
__device__ __forceinline__ void chimera_fwd(R& a, R& b, R& c, R v) {
  const R k0 = a + b + c;
  const R m1 = c - a;
  const R k1 = m1 - v * k0;
  const R k2 = (c + a) - R(2) * v * m1 + v * v * k0;
  a = k0;
  b = k1;
  c = k2;
}

// Exact inverse: central moments (k0, k1, k2) about v -> values at -1, 0, +1.
template <class R>
__device__ __forceinline__ void chimera_bwd(R& a, R& b, R& c, R v) {
  const R k0 = a, k1 = b, k2 = c;
  const R m1 = k1 + v * k0;
  const R m2 = k2 + R(2) * v * k1 + v * v * k0;
  a = R(0.5) * (m2 - m1);
  b = k0 - m2;
  c = R(0.5) * (m2 + m1);
}

template <class R>
__device__ __forceinline__ void collide_cumulant(R (&d)[27], const CollParams<R>& p) {
  using L = Lattice<27>;
  const Macro<27, R> mac = macros<27, R>(d, p);
  const R ux = mac.ux, uy = mac.uy, uz = mac.uz;
  R m[3][3][3];
#pragma unroll
  for (int i = 0; i < 27; ++i) m[L::cx[i] + 1][L::cy[i] + 1][L::cz[i] + 1] = d[i];
  // forward: z, y, x
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) chimera_fwd(m[a][b][0], m[a][b][1], m[a][b][2], uz);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) chimera_fwd(m[a][0][c], m[a][1][c], m[a][2][c], uy);
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int c = 0; c < 3; ++c) chimera_fwd(m[0][b][c], m[1][b][c], m[2][b][c], ux);

  const R w1 = p.om1, w2 = p.om2;
  const R drho = mac.drho, rho = mac.rho, inv_rho = R(1) / rho;
  const R ux2 = ux * ux, uy2 = uy * uy, uz2 = uz * uz;
  const R A = R(1) / R(3) + ux2, B = R(1) / R(3) + uy2, C = R(1) / R(3) + uz2;

  // second order
  const R e0 = (R(1) - w1) * m[1][1][0] - w1 * ux * uy;
  const R f0 = (R(1) - w1) * m[1][0][1] - w1 * ux * uz;
  const R g0 = (R(1) - w1) * m[0][1][1] - w1 * uy * uz;
  const R dxy = (R(1) - w1) * ((ux2 - uy2) + (m[2][0][0] - m[0][2][0]));
  const R dxz = (R(1) - w1) * ((ux2 - uz2) + (m[2][0][0] - m[0][0][2]));
  const R tm1 = (R(1) - w2) * ((ux2 + uy2 + uz2) + (m[2][0][0] + m[0][2][0] + m[0][0][2])) +
                w2 * drho;
  const R a2 = (dxy + dxz + tm1) * (R(1) / R(3)) - ux2;
  const R b2 = (tm1 - R(2) * dxy + dxz) * (R(1) / R(3)) - uy2;
  const R c2 = (tm1 + dxy - R(2) * dxz) * (R(1) / R(3)) - uz2;
  const R e = ux * uy + e0, f = ux * uz + f0, g = uy * uz + g0;
  const R Ap = A + a2, Bp = B + b2, Cp = C + c2;

  R D[3][3][3];
  D[0][0][0] = drho;
  D[1][0][0] = R(0.5) * p.Fx + ux;
  D[0][1][0] = R(0.5) * p.Fy + uy;
  D[0][0][1] = R(0.5) * p.Fz + uz;
  D[1][1][0] = e0;
  D[1][0][1] = f0;
  D[0][1][1] = g0;
  D[2][0][0] = a2;
  D[0][2][0] = b2;
  D[0][0][2] = c2;
  // third order: K* = 0  ->  D* = -K^w
  D[1][1][1] = ux * uy * uz;
  D[2][1][0] = A * uy;
  D[2][0][1] = A * uz;
  D[1][2][0] = B * ux;
  D[0][2][1] = B * uz;
  D[1][0][2] = C * ux;
  D[0][1][2] = C * uy;
  // fourth order (Isserlis relations written as deviations)
  D[2][2][0] = (A * b2 + a2 * B + a2 * b2 + R(2) * e * e - drho * A * B) * inv_rho;
  D[2][0][2] = (A * c2 + a2 * C + a2 * c2 + R(2) * f * f - drho * A * C) * inv_rho;
  D[0][2][2] = (B * c2 + b2 * C + b2 * c2 + R(2) * g * g - drho * B * C) * inv_rho;
  D[2][1][1] = (A * g0 + a2 * g + R(2) * e * f - drho * A * uy * uz) * inv_rho;
  D[1][2][1] = (B * f0 + b2 * f + R(2) * e * g - drho * B * ux * uz) * inv_rho;
  D[1][1][2] = (C * e0 + c2 * e + R(2) * f * g - drho * C * ux * uy) * inv_rho;
  // fifth order: K* = 0
  D[2][2][1] = A * B * uz;
  D[2][1][2] = A * C * uy;
  D[1][2][2] = B * C * ux;
  // sixth order
  {
    const R lin = A * B * c2 + A * b2 * C + a2 * B * C;
    const R quad = A * b2 * c2 + a2 * B * c2 + a2 * b2 * C;
    const R cub = a2 * b2 * c2;
    const R iss = R(2) * (e * e * Cp + f * f * Bp + g * g * Ap) + R(8) * e * f * g;
    D[2][2][2] = (lin + quad + cub - drho * (R(2) + drho) * A * B * C + iss) * (inv_rho * inv_rho);
  }

  // backward: x, y, z
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int c = 0; c < 3; ++c) chimera_bwd(D[0][b][c], D[1][b][c], D[2][b][c], ux);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) chimera_bwd(D[a][0][c], D[a][1][c], D[a][2][c], uy);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) chimera_bwd(D[a][b][0], D[a][b][1], D[a][b][2], uz);
#pragma unroll
  for (int i = 0; i < 27; ++i) d[i] = D[L::cx[i] + 1][L::cy[i] + 1][L::cz[i] + 1];
}

}  // namespace lbm
