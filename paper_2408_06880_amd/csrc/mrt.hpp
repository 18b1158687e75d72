// Multiple-relaxation-time operator for D3Q19 in deviation form (the paper
// lists MRT among the classical operators, Section "Lattice Boltzmann
// Method"; moment basis of d'Humieres et al. 2002).
//
// The 19 basis polynomials are each even or odd under c -> -c, so a moment
// needs only the symmetric pair sums (even moments) or the antisymmetric
// pair differences (odd moments) of its input: 10 even moments from 10
// symmetric inputs (rest + 9 pairs), 9 odd moments from 9 antisymmetric
// ones.  With D = f - f^eq and G the Guo source, moment k changes by
//   -s_k (M D)_k + (1 - s_k / 2) (M G)_k,
// and the populations by M^T diag(1 / |row k|^2) of that (the rows are
// orthogonal).  Density and momentum are conserved: the density row sees
// no change and each momentum row changes by the force exactly.
#pragma once

#include "collide.hpp"

namespace lbm {

namespace mrt {

// Basis polynomial k at the integer velocity (x, y, z).
constexpr int poly(int k, int x, int y, int z) {
  const int c2 = x * x + y * y + z * z;
  switch (k) {
    case 0: return 1;
    case 1: return 19 * c2 - 30;
    case 2: return (21 * c2 * c2 - 53 * c2 + 24) / 2;
    case 3: return x;
    case 4: return (5 * c2 - 9) * x;
    case 5: return y;
    case 6: return (5 * c2 - 9) * y;
    case 7: return z;
    case 8: return (5 * c2 - 9) * z;
    case 9: return 3 * x * x - c2;
    case 10: return (3 * c2 - 5) * (3 * x * x - c2);
    case 11: return y * y - z * z;
    case 12: return (3 * c2 - 5) * (y * y - z * z);
    case 13: return x * y;
    case 14: return y * z;
    case 15: return x * z;
    case 16: return (y * y - z * z) * x;
    case 17: return (z * z - x * x) * y;
    default: return (x * x - y * y) * z;
  }
}

constexpr int P(int k, int i) {
  return poly(k, Lattice<19>::cx[i], Lattice<19>::cy[i], Lattice<19>::cz[i]);
}

constexpr int norm(int k) {
  int s = 0;
  for (int i = 0; i < 19; ++i) s += P(k, i) * P(k, i);
  return s;
}

// Even (symmetric) and odd (antisymmetric) moments, in basis order.
constexpr int kEven[10] = {0, 1, 2, 9, 10, 11, 12, 13, 14, 15};
constexpr int kOdd[9] = {3, 4, 5, 6, 7, 8, 16, 17, 18};

}  // namespace mrt

// Rates: p.om1 shear (1/tau), p.om2 energy (bulk); p.r[0..3] the epsilon,
// pi, q and m groups.
template <class R>
__device__ __forceinline__ void collide_mrt(R (&d)[19], const CollParams<R>& p) {
  using L = Lattice<19>;
  const Macro<19, R> m = macros<19, R>(d, p);
  const R usq = m.ux * m.ux + m.uy * m.uy + m.uz * m.uz;
  const R uF = m.ux * p.Fx + m.uy * p.Fy + m.uz * p.Fz;
  const R base = R(-1.5) * usq;
  // symmetric / antisymmetric parts of D = d - d^eq and of G, per pair
  R Dp[10], Gp[10], Dm[9], Gm[9];
  {
    const R w = R(L::w(0));
    Dp[0] = d[0] - w * (m.drho + m.rho * base);
    Gp[0] = w * R(-3) * uF;
  }
#pragma unroll
  for (int n = 0; n < 9; ++n) {
    const int i = 2 * n + 1, j = i + 1;
    const R w = R(L::w(i));
    const R cu = R(L::cx[i]) * m.ux + R(L::cy[i]) * m.uy + R(L::cz[i]) * m.uz;
    const R cF = R(L::cx[i]) * p.Fx + R(L::cy[i]) * p.Fy + R(L::cz[i]) * p.Fz;
    const R eqp = w * (m.drho + m.rho * (R(4.5) * cu * cu + base));
    const R eqm = w * m.rho * R(3) * cu;
    Dp[n + 1] = (d[i] + d[j]) - R(2) * eqp;
    Dm[n] = (d[i] - d[j]) - R(2) * eqm;
    Gp[n + 1] = R(2) * w * (R(9) * cu * cF - R(3) * uF);
    Gm[n] = R(2) * w * R(3) * cF;
  }
  // moment changes divided by the row norms; density: none, momentum: F
  R de[10], dodd[9];
  de[0] = R(0);
#pragma unroll
  for (int e = 1; e < 10; ++e) {
    const int k = mrt::kEven[e];
    R a = R(0), b = R(0);
#pragma unroll
    for (int n = 0; n < 10; ++n) {
      const int i = n == 0 ? 0 : 2 * n - 1;
      const int c = mrt::P(k, i);
      if (c != 0) {
        a += R(c) * Dp[n];
        b += R(c) * Gp[n];
      }
    }
    R s;
    switch (k) {
      case 1: s = p.om2; break;
      case 2: s = p.r[0]; break;
      case 10: case 12: s = p.r[1]; break;
      default: s = p.om1; break;
    }
    de[e] = (s * a - (R(1) - R(0.5) * s) * b) * R(1.0 / mrt::norm(k));
  }
  dodd[0] = R(-1.0 / mrt::norm(3)) * p.Fx;
  dodd[2] = R(-1.0 / mrt::norm(5)) * p.Fy;
  dodd[4] = R(-1.0 / mrt::norm(7)) * p.Fz;
#pragma unroll
  for (int o = 0; o < 9; ++o) {
    const int k = mrt::kOdd[o];
    if (k == 3 || k == 5 || k == 7) continue;
    R a = R(0), b = R(0);
#pragma unroll
    for (int n = 0; n < 9; ++n) {
      const int c = mrt::P(k, 2 * n + 1);
      if (c != 0) {
        a += R(c) * Dm[n];
        b += R(c) * Gm[n];
      }
    }
    const R s = (k == 4 || k == 6 || k == 8) ? p.r[2] : p.r[3];
    dodd[o] = (s * a - (R(1) - R(0.5) * s) * b) * R(1.0 / mrt::norm(k));
  }
  // back to populations: d_i -= sum_k P(k, i) delta_k
  {
    R acc = R(0);
#pragma unroll
    for (int e = 0; e < 10; ++e) {
      const int c = mrt::P(mrt::kEven[e], 0);
      if (c != 0) acc += R(c) * de[e];
    }
    d[0] -= acc;
  }
#pragma unroll
  for (int n = 0; n < 9; ++n) {
    const int i = 2 * n + 1, j = i + 1;
    R ev = R(0), od = R(0);
#pragma unroll
    for (int e = 0; e < 10; ++e) {
      const int c = mrt::P(mrt::kEven[e], i);
      if (c != 0) ev += R(c) * de[e];
    }
#pragma unroll
    for (int o = 0; o < 9; ++o) {
      const int c = mrt::P(mrt::kOdd[o], i);
      if (c != 0) od += R(c) * dodd[o];
    }
    d[i] -= ev + od;
    d[j] -= ev - od;
  }
}

}  // namespace lbm
