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

// Deviations d (indexed by direction) -> central moments K^d[a][b][c] of
// the deviations about u: z, y, x axis passes.
template <class R>
__device__ __forceinline__ void central_forward(const R (&d)[27], R ux, R uy, R uz,
                                                R (&m)[3][3][3]) {
  using L = Lattice<27>;
#pragma unroll
  for (int i = 0; i < 27; ++i) m[L::cx[i] + 1][L::cy[i] + 1][L::cz[i] + 1] = d[i];
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
}

// Post-collision deviation moments D*[a][b][c] -> deviations d*: x, y, z
// axis passes of the exact inverse.
template <class R>
__device__ __forceinline__ void central_backward(R (&D)[3][3][3], R ux, R uy, R uz,
                                                 R (&d)[27]) {
  using L = Lattice<27>;
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

// Orders 0-2 after collision, written as deviations D* = K* - K^w (shared
// by the cumulant and central-moment operators): density, F/2 for the
// first order, off-diagonal and deviatoric second order at om1, the trace
// towards rho at om2.  Also returns the post-collision full second-order
// moments' small parts used by the cumulant's higher orders.
template <class R>
struct LowOrders {
  R a2, b2, c2, e0, f0, g0;  // D* of 200, 020, 002, 110, 101, 011
};

template <class R>
__device__ __forceinline__ LowOrders<R> relax_low_orders(const R (&m)[3][3][3],
                                                         const Macro<27, R>& mac,
                                                         const CollParams<R>& p,
                                                         R (&D)[3][3][3]) {
  const R ux = mac.ux, uy = mac.uy, uz = mac.uz;
  const R w1 = p.om1, w2 = p.om2;
  const R drho = mac.drho;
  const R ux2 = ux * ux, uy2 = uy * uy, uz2 = uz * uz;
  LowOrders<R> o;
  o.e0 = (R(1) - w1) * m[1][1][0] - w1 * ux * uy;
  o.f0 = (R(1) - w1) * m[1][0][1] - w1 * ux * uz;
  o.g0 = (R(1) - w1) * m[0][1][1] - w1 * uy * uz;
  const R dxy = (R(1) - w1) * ((ux2 - uy2) + (m[2][0][0] - m[0][2][0]));
  const R dxz = (R(1) - w1) * ((ux2 - uz2) + (m[2][0][0] - m[0][0][2]));
  const R tm1 = (R(1) - w2) * ((ux2 + uy2 + uz2) + (m[2][0][0] + m[0][2][0] + m[0][0][2])) +
                w2 * drho;
  o.a2 = (dxy + dxz + tm1) * (R(1) / R(3)) - ux2;
  o.b2 = (tm1 - R(2) * dxy + dxz) * (R(1) / R(3)) - uy2;
  o.c2 = (tm1 + dxy - R(2) * dxz) * (R(1) / R(3)) - uz2;
  D[0][0][0] = drho;
  D[1][0][0] = R(0.5) * p.Fx + ux;
  D[0][1][0] = R(0.5) * p.Fy + uy;
  D[0][0][1] = R(0.5) * p.Fz + uz;
  D[1][1][0] = o.e0;
  D[1][0][1] = o.f0;
  D[0][1][1] = o.g0;
  D[2][0][0] = o.a2;
  D[0][2][0] = o.b2;
  D[0][0][2] = o.c2;
  return o;
}

template <class R>
__device__ __forceinline__ void collide_cumulant(R (&d)[27], const CollParams<R>& p) {
  const Macro<27, R> mac = macros<27, R>(d, p);
  const R ux = mac.ux, uy = mac.uy, uz = mac.uz;
  R m[3][3][3];
  central_forward(d, ux, uy, uz, m);

  const R drho = mac.drho, rho = mac.rho, inv_rho = R(1) / rho;
  const R ux2 = ux * ux, uy2 = uy * uy, uz2 = uz * uz;
  const R A = R(1) / R(3) + ux2, B = R(1) / R(3) + uy2, C = R(1) / R(3) + uz2;

  R D[3][3][3];
  const LowOrders<R> lo = relax_low_orders(m, mac, p, D);
  const R e0 = lo.e0, f0 = lo.f0, g0 = lo.g0, a2 = lo.a2, b2 = lo.b2, c2 = lo.c2;
  // second order (full moments' small parts)
  const R e = ux * uy + e0, f = ux * uz + f0, g = uy * uz + g0;
  const R Ap = A + a2, Bp = B + b2, Cp = C + c2;
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

  central_backward(D, ux, uy, uz, d);
}

// Central-moment operator for D3Q27 (the paper names the central-moment
// model among its operators; D3Q27 holds the complete per-axis basis).
// Orders 0-2 as the cumulant operator; every central moment of order
// n = 3..6 relaxes towards the Maxwellian's, K^eq_abc = rho e(a) e(b) e(c)
// with e = (1, 0, 1/3), at rate p.r[n - 3]:
//   D* = K* - K^w = (1 - s) K^d + s (K^eq - K^w),
// with K^eq - K^w in closed form of the small quantities (drho, u):
//   any exponent 1:  K^eq = 0, K^w = product of k(a, u_a), k(1, u) = -u;
//   220-type:        rho/9  - A B   = drho/9 - (ux^2 + uy^2)/3 - ux^2 uy^2;
//   222:             rho/27 - A B C = drho/27 - |u|^2/9
//                                     - (ux^2 uy^2 + ux^2 uz^2 + uy^2 uz^2)/3
//                                     - ux^2 uy^2 uz^2.
template <class R>
__device__ __forceinline__ void collide_cm(R (&d)[27], const CollParams<R>& p) {
  const Macro<27, R> mac = macros<27, R>(d, p);
  const R ux = mac.ux, uy = mac.uy, uz = mac.uz;
  R m[3][3][3];
  central_forward(d, ux, uy, uz, m);
  R D[3][3][3];
  relax_low_orders(m, mac, p, D);
  const R drho = mac.drho;
  const R ux2 = ux * ux, uy2 = uy * uy, uz2 = uz * uz;
  const R A = R(1) / R(3) + ux2, B = R(1) / R(3) + uy2, C = R(1) / R(3) + uz2;
  const R s3 = p.r[0], s4 = p.r[1], s5 = p.r[2], s6 = p.r[3];
  const R t3 = R(1) - s3, t4 = R(1) - s4, t5 = R(1) - s5, t6 = R(1) - s6;
  // order 3: K^eq = 0, D* = (1 - s3) K^d - s3 K^w
  D[1][1][1] = t3 * m[1][1][1] + s3 * (ux * uy * uz);
  D[2][1][0] = t3 * m[2][1][0] + s3 * (A * uy);
  D[2][0][1] = t3 * m[2][0][1] + s3 * (A * uz);
  D[1][2][0] = t3 * m[1][2][0] + s3 * (B * ux);
  D[0][2][1] = t3 * m[0][2][1] + s3 * (B * uz);
  D[1][0][2] = t3 * m[1][0][2] + s3 * (C * ux);
  D[0][1][2] = t3 * m[0][1][2] + s3 * (C * uy);
  // order 4
  const R r9 = R(1) / R(9), r3 = R(1) / R(3);
  D[2][2][0] = t4 * m[2][2][0] + s4 * (drho * r9 - (ux2 + uy2) * r3 - ux2 * uy2);
  D[2][0][2] = t4 * m[2][0][2] + s4 * (drho * r9 - (ux2 + uz2) * r3 - ux2 * uz2);
  D[0][2][2] = t4 * m[0][2][2] + s4 * (drho * r9 - (uy2 + uz2) * r3 - uy2 * uz2);
  D[2][1][1] = t4 * m[2][1][1] - s4 * (A * uy * uz);
  D[1][2][1] = t4 * m[1][2][1] - s4 * (B * ux * uz);
  D[1][1][2] = t4 * m[1][1][2] - s4 * (C * ux * uy);
  // order 5: K^w_221 = -A B uz
  D[2][2][1] = t5 * m[2][2][1] + s5 * (A * B * uz);
  D[2][1][2] = t5 * m[2][1][2] + s5 * (A * C * uy);
  D[1][2][2] = t5 * m[1][2][2] + s5 * (B * C * ux);
  // order 6
  D[2][2][2] = t6 * m[2][2][2] +
               s6 * (drho * (R(1) / R(27)) - (ux2 + uy2 + uz2) * r9 -
                     (ux2 * uy2 + ux2 * uz2 + uy2 * uz2) * r3 - ux2 * uy2 * uz2);
  central_backward(D, ux, uy, uz, d);
}

}  // namespace lbm
