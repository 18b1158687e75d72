// Host build of the library's collision operators (deviation form), for
// comparing their arithmetic with the oracle on the CPU.
#include "cumulant.hpp"
#include "mrt.hpp"

using namespace lbm;

template <int Q, int C, class R>
static void run(const double* P, long n, const double* fin, double* fout) {
  CollParams<R> p;
  p.om1 = (R)P[0];
  p.om2 = (R)P[1];
  p.Fx = (R)P[2];
  p.Fy = (R)P[3];
  p.Fz = (R)P[4];
  for (int a = 0; a < 4; ++a) p.r[a] = (R)P[5 + a];
  for (long k = 0; k < n; ++k) {
    R d[Q];
    for (int i = 0; i < Q; ++i) d[i] = (R)(fin[k * Q + i] - Lattice<Q>::w(i));
    if constexpr (C == COLL_SRT) collide_srt<Q, R>(d, p);
    if constexpr (C == COLL_TRT) collide_trt<Q, R>(d, p);
    if constexpr (C == COLL_CUMULANT && Q == 27) collide_cumulant<R>(d, p);
    if constexpr (C == COLL_MRT && Q == 19) collide_mrt<R>(d, p);
    if constexpr (C == COLL_CM && Q == 27) collide_cm<R>(d, p);
    for (int i = 0; i < Q; ++i) fout[k * Q + i] = Lattice<Q>::w(i) + (double)d[i];
  }
}

extern "C" int host_collide(int q, int kind, int f64, const double* P, long n, const double* fin,
                            double* fout) {
#define DISPATCH(Q, C)                          \
  if (q == Q && kind == C) {                    \
    if (f64)                                    \
      run<Q, C, double>(P, n, fin, fout);       \
    else                                        \
      run<Q, C, float>(P, n, fin, fout);        \
    return 0;                                   \
  }
  DISPATCH(19, COLL_SRT)
  DISPATCH(19, COLL_TRT)
  DISPATCH(27, COLL_SRT)
  DISPATCH(27, COLL_TRT)
  DISPATCH(27, COLL_CUMULANT)
  DISPATCH(19, COLL_MRT)
  DISPATCH(27, COLL_CM)
  return -1;
}
