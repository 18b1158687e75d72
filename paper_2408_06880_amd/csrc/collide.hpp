// Collision operators in deviation form: the input d[i] = f_i - w_i is the
// pre-collision population minus its rest weight, the output the
// post-collision deviation.  Never forms w_i + d_i, so FP32 keeps the
// resolution of the small non-equilibrium signal.
//
//   rho = 1 + sum d,  j = sum c d  (sum w c = 0),  u = (j + F/2) / rho
//   f^eq_i - w_i = w_i [ drho + rho (3 c.u + 4.5 (c.u)^2 - 1.5 u.u) ]
//   Guo source S_i = w_i [ 3 c.F - 3 u.F + 9 (c.u)(c.F) ]
//
// (Section "Lattice Boltzmann Method": moments eq. (1), SRT operator,
// second-order equilibrium with c_s^2 = 1/3, nu = c_s^2 (tau - 1/2).)
#pragma once

#include "lattice.hpp"

namespace lbm {

enum CollKind {
  COLL_NONE = 0, COLL_SRT = 1, COLL_TRT = 2, COLL_CUMULANT = 3, COLL_MRT = 4, COLL_CM = 5
};

template <class R>
struct CollParams {
  R om1, om2;  // SRT: omega; TRT: omega+, omega-; cumulant, MRT, CM: shear, bulk
  R Fx, Fy, Fz;
  R r[4];      // MRT: epsilon, pi, q, m rates; CM: orders 3-6
};

template <int Q, class R>
struct Macro {
  R drho, rho, ux, uy, uz;
};

template <int Q, class R>
__device__ __forceinline__ Macro<Q, R> macros(const R (&d)[Q], const CollParams<R>& p) {
  using L = Lattice<Q>;
  R drho = R(0), jx = R(0), jy = R(0), jz = R(0);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    drho += d[i];
    if (L::cx[i] > 0) jx += d[i];
    if (L::cx[i] < 0) jx -= d[i];
    if (L::cy[i] > 0) jy += d[i];
    if (L::cy[i] < 0) jy -= d[i];
    if (L::cz[i] > 0) jz += d[i];
    if (L::cz[i] < 0) jz -= d[i];
  }
  Macro<Q, R> m;
  m.drho = drho;
  m.rho = R(1) + drho;
  const R inv = R(1) / m.rho;
  m.ux = (jx + R(0.5) * p.Fx) * inv;
  m.uy = (jy + R(0.5) * p.Fy) * inv;
  m.uz = (jz + R(0.5) * p.Fz) * inv;
  return m;
}

template <int Q, class R>
__device__ __forceinline__ void collide_srt(R (&d)[Q], const CollParams<R>& p) {
  using L = Lattice<Q>;
  const Macro<Q, R> m = macros<Q, R>(d, p);
  const R usq = m.ux * m.ux + m.uy * m.uy + m.uz * m.uz;
  const R uF = m.ux * p.Fx + m.uy * p.Fy + m.uz * p.Fz;
  const R om = p.om1, sf = R(1) - R(0.5) * p.om1;
  const R base = R(-1.5) * usq;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const R w = R(L::w(i));
    const R cu = R(L::cx[i]) * m.ux + R(L::cy[i]) * m.uy + R(L::cz[i]) * m.uz;
    const R cF = R(L::cx[i]) * p.Fx + R(L::cy[i]) * p.Fy + R(L::cz[i]) * p.Fz;
    const R deq = w * (m.drho + m.rho * (R(3) * cu + R(4.5) * cu * cu + base));
    const R S = w * (R(3) * cF - R(3) * uF + R(9) * cu * cF);
    d[i] = d[i] - om * (d[i] - deq) + sf * S;
  }
}

// Two-relaxation-time operator: symmetric halves of (f - f^eq) and of the
// source relax with omega+, antisymmetric halves with omega-.  Written per
// opposite pair (i, i+1) with the even/odd parts in closed form:
//   eq+ = w [drho + rho(4.5 cu^2 - 1.5 u.u)],  eq- = 3 w rho cu,
//   S+  = w [9 cu cF - 3 u.F],                 S-  = 3 w cF.
template <int Q, class R>
__device__ __forceinline__ void collide_trt(R (&d)[Q], const CollParams<R>& p) {
  using L = Lattice<Q>;
  const Macro<Q, R> m = macros<Q, R>(d, p);
  const R usq = m.ux * m.ux + m.uy * m.uy + m.uz * m.uz;
  const R uF = m.ux * p.Fx + m.uy * p.Fy + m.uz * p.Fz;
  const R omp = p.om1, omm = p.om2;
  const R sfp = R(1) - R(0.5) * omp, sfm = R(1) - R(0.5) * omm;
  const R base = R(-1.5) * usq;
  {
    const R w = R(L::w(0));
    const R deq = w * (m.drho + m.rho * base);
    d[0] = d[0] - omp * (d[0] - deq) + sfp * (w * R(-3) * uF);
  }
#pragma unroll
  for (int i = 1; i < Q; i += 2) {
    const int j = i + 1;
    const R w = R(L::w(i));
    const R cu = R(L::cx[i]) * m.ux + R(L::cy[i]) * m.uy + R(L::cz[i]) * m.uz;
    const R cF = R(L::cx[i]) * p.Fx + R(L::cy[i]) * p.Fy + R(L::cz[i]) * p.Fz;
    const R eqp = w * (m.drho + m.rho * (R(4.5) * cu * cu + base));
    const R eqm = w * m.rho * R(3) * cu;
    const R sp = w * (R(9) * cu * cF - R(3) * uF);
    const R sm = w * R(3) * cF;
    const R dp = R(0.5) * (d[i] + d[j]);
    const R dm = R(0.5) * (d[i] - d[j]);
    const R relp = -omp * (dp - eqp) + sfp * sp;
    const R relm = -omm * (dm - eqm) + sfm * sm;
    d[i] = d[i] + relp + relm;
    d[j] = d[j] + relp - relm;
  }
}

}  // namespace lbm
