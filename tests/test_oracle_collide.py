"""Pins of the oracle's velocity sets and single-cell collision operators.

Each test checks the oracle against something other than itself: lattice
isotropy conditions, conservation laws, fixed points, operator identities,
closed forms, and (for the cumulant) an independent computation of cumulants
through the logarithm of the moment-generating function.
"""
import itertools
import math

import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("q", [19, 27])
def test_lattice_isotropy(q):
    """Weights and velocities satisfy the isotropy conditions of a
    fourth-order lattice with c_s^2 = 1/3 (Section 'Lattice Boltzmann Method')."""
    c, w, opp = oracle.stencil(q)
    c = c.astype(np.float64)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.all(w > 0)
    # odd moments vanish
    assert np.allclose(w @ c, 0.0, atol=1e-16)
    for a, b, g in itertools.product(range(3), repeat=3):
        assert abs(np.sum(w * c[:, a] * c[:, b] * c[:, g])) < 1e-16
    # second moment = delta/3
    M2 = np.einsum("i,ia,ib->ab", w, c, c)
    assert np.allclose(M2, np.eye(3) / 3.0, atol=1e-15)
    # fourth moment = (d_ab d_cd + d_ac d_bd + d_ad d_bc)/9
    M4 = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    d = np.eye(3)
    ref = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
           + np.einsum("ad,bc->abcd", d, d)) / 9.0
    assert np.allclose(M4, ref, atol=1e-15)
    # all directions distinct, opposite is an involution with c_opp = -c
    assert len({tuple(v) for v in c.astype(int)}) == q
    assert np.all(opp[opp] == np.arange(q))
    assert np.all(c[opp] == -c)
    assert tuple(c[0]) == (0, 0, 0)


def test_d3q27_weights_are_tensor_products():
    c, w, _ = oracle.stencil(27)
    W1 = {0: 2.0 / 3.0, 1: 1.0 / 6.0, -1: 1.0 / 6.0}
    for i in range(27):
        assert abs(w[i] - W1[c[i, 0]] * W1[c[i, 1]] * W1[c[i, 2]]) < 1e-16


def _feq(q, rho, u):
    c, w, _ = oracle.stencil(q)
    cu = c @ u
    return w * rho * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * (u @ u))


def _product_eq(q, rho, u):
    """Product-form equilibrium: rho * prod_a g(c_a, u_a)."""
    c, _, _ = oracle.stencil(q)
    out = np.empty(q)
    for i in range(q):
        v = rho
        for a in range(3):
            ua = u[a]
            if c[i, a] == 0:
                v *= 2.0 / 3.0 - ua * ua
            else:
                v *= (1.0 / 3.0 + ua * ua + c[i, a] * ua) / 2.0
        out[i] = v
    return out


def _random_states(q, n, seed, amp=1e-2):
    rng = np.random.default_rng(seed)
    out = np.empty((n, q))
    for k in range(n):
        rho = 1.0 + 0.05 * rng.standard_normal()
        u = 0.05 * rng.standard_normal(3)
        out[k] = _feq(q, rho, u) * (1.0 + amp * rng.standard_normal(q))
    return out


KINDS = [(19, oracle.SRT), (19, oracle.TRT), (27, oracle.SRT), (27, oracle.TRT),
         (27, oracle.CUMULANT), (19, oracle.MRT), (27, oracle.CM)]


@pytest.mark.parametrize("q,kind", KINDS)
def test_mass_and_momentum_balance(q, kind):
    """Collision conserves mass and adds exactly F to the momentum density
    (Guo forcing with the half-force velocity)."""
    c, _, _ = oracle.stencil(q)
    F = np.array([1e-4, -2e-4, 3e-5])
    p = oracle.params(q=q, kind=kind, tau=0.7, magic=3 / 16, omega_bulk=1.3, force=F)
    f = _random_states(q, 50, seed=3)
    fs = oracle.collide(p, f)
    assert np.allclose(fs.sum(1), f.sum(1), rtol=0, atol=2e-15)
    assert np.allclose(fs @ c, f @ c + F[None, :], rtol=0, atol=2e-15)


@pytest.mark.parametrize("q,kind", KINDS)
def test_forced_equilibrium_moves_to_the_new_velocity(q, kind):
    """A forced collision of the operator's equilibrium at (rho, u0), at
    general rates, gives density, momentum and second moments of the
    equilibrium at u0 + F/rho up to O(F^2): the error falls by 4 when F
    halves.  Mass and momentum balance alone would not see a wrong force
    term in the stress (the second-order part of the source, or the
    half-force shift of the cumulant frame), which leaves an O(F) error."""
    c, _, _ = oracle.stencil(q)
    eq = _product_eq if kind in (oracle.CUMULANT, oracle.CM) else _feq
    rho, u0 = 1.03, np.array([0.02, -0.01, 0.015])
    errs = []
    for scale in (1.0, 0.5, 0.25):
        F = scale * np.array([4e-4, -3e-4, 2e-4])
        p = oracle.params(q=q, kind=kind, tau=0.71, magic=3 / 16, omega_bulk=1.27, force=F,
                          rates=(1.3, 1.6, 1.1, 1.45))
        fs = oracle.collide(p, eq(q, rho, u0)[None])[0]
        target = eq(q, rho, u0 + F / rho)
        m0 = abs(fs.sum() - target.sum())
        m1 = np.max(np.abs(fs @ c - target @ c))
        m2 = np.max(np.abs(np.einsum("i,ia,ib->ab", fs - target, c, c)))
        assert m0 < 1e-15 and m1 < 1e-15
        errs.append(m2)
    assert errs[0] < 1e-7
    for a, b in zip(errs, errs[1:]):
        assert 3.9 < a / b < 4.1


@pytest.mark.parametrize("q,kind", KINDS)
def test_equilibrium_fixed_point(q, kind):
    """Without force, the operator's equilibrium is a fixed point: the
    polynomial f^eq for SRT/TRT, the product form for the cumulant."""
    rng = np.random.default_rng(5)
    p = oracle.params(q=q, kind=kind, tau=0.63, magic=0.25, omega_bulk=1.1)
    for _ in range(10):
        rho = 1.0 + 0.1 * rng.standard_normal()
        u = 0.08 * rng.standard_normal(3)
        f = (_product_eq if kind in (oracle.CUMULANT, oracle.CM) else _feq)(q, rho, u)
        fs = oracle.collide(p, f[None])[0]
        assert np.max(np.abs(fs - f)) < 5e-16


@pytest.mark.parametrize("q", [19, 27])
def test_trt_reduces_to_srt(q):
    """TRT with Lambda = (tau - 1/2)^2 has omega- = omega+ and equals SRT."""
    tau = 0.83
    F = (1e-4, 2e-5, -3e-5)
    f = _random_states(q, 30, seed=7)
    a = oracle.collide(oracle.params(q=q, kind=oracle.SRT, tau=tau, force=F), f)
    b = oracle.collide(oracle.params(q=q, kind=oracle.TRT, tau=tau, magic=(tau - 0.5) ** 2,
                                     force=F), f)
    assert np.max(np.abs(a - b)) < 1e-16


def test_srt_relaxes_non_equilibrium():
    """SRT without force: f* - f^eq = (1 - omega)(f - f^eq), with f^eq built
    here from eq. (5) of the paper on the cell's own rho, u."""
    q = 19
    c, _, _ = oracle.stencil(q)
    tau = 0.9
    f = _random_states(q, 20, seed=9)
    fs = oracle.collide(oracle.params(q=q, kind=oracle.SRT, tau=tau), f)
    for k in range(f.shape[0]):
        rho = f[k].sum()
        u = (c.T @ f[k]) / rho
        feq = _feq(q, rho, u)
        assert np.allclose(fs[k] - feq, (1 - 1 / tau) * (f[k] - feq), atol=1e-16)


def test_trt_relaxes_parities_separately():
    """TRT: even part of f - f^eq scales by (1 - omega+), odd part by (1 - omega-)."""
    q = 19
    c, _, opp = oracle.stencil(q)
    tau, lam = 0.7, 3.0 / 16.0
    wp = 1 / tau
    wm = 1 / (0.5 + lam / (tau - 0.5))
    f = _random_states(q, 20, seed=11)
    fs = oracle.collide(oracle.params(q=q, kind=oracle.TRT, tau=tau, magic=lam), f)
    for k in range(f.shape[0]):
        rho = f[k].sum()
        u = (c.T @ f[k]) / rho
        neq = f[k] - _feq(q, rho, u)
        neqs = fs[k] - _feq(q, rho, u)
        assert np.allclose(0.5 * (neqs + neqs[opp]), (1 - wp) * 0.5 * (neq + neq[opp]), atol=1e-16)
        assert np.allclose(0.5 * (neqs - neqs[opp]), (1 - wm) * 0.5 * (neq - neq[opp]), atol=1e-16)


# ---------------------------------------------------------------- cumulant

def _series_mul(a, b):
    """Product in R[x,y,z]/(x^3, y^3, z^3); arrays [3,3,3] of coefficients."""
    out = np.zeros((3, 3, 3))
    for i, j, k in itertools.product(range(3), repeat=3):
        if a[i, j, k] == 0.0:
            continue
        for l, m, n in itertools.product(range(3 - i), range(3 - j), range(3 - k)):
            out[i + l, j + m, k + n] += a[i, j, k] * b[l, m, n]
    return out


def _cumulants(f, c):
    """Cumulants C_abc (a,b,c <= 2) of a discrete distribution: a!b!c! times
    the coefficients of log(M(xi)/M(0)), M the moment-generating function,
    computed in the truncated power-series ring (exact: the logarithm of
    1 + X with X nilpotent is a finite series).  Independent of the oracle's
    central-moment / Isserlis arithmetic."""
    M = np.zeros((3, 3, 3))
    for a, b, g in itertools.product(range(3), repeat=3):
        M[a, b, g] = np.sum(f * c[:, 0] ** a * c[:, 1] ** b * c[:, 2] ** g) / (
            math.factorial(a) * math.factorial(b) * math.factorial(g))
    X = M / M[0, 0, 0]
    X[0, 0, 0] = 0.0
    L = np.zeros((3, 3, 3))
    P = X.copy()
    for n in range(1, 7):
        L += ((-1) ** (n + 1)) * P / n
        P = _series_mul(P, X)
    C = np.zeros((3, 3, 3))
    for a, b, g in itertools.product(range(3), repeat=3):
        C[a, b, g] = L[a, b, g] * math.factorial(a) * math.factorial(b) * math.factorial(g)
    return C


def test_cumulant_series_helper_on_product_distribution():
    """Sanity of the helper: a product of independent 1-D distributions has
    vanishing mixed cumulants, and its 1-D cumulants match direct formulas."""
    c, _, _ = oracle.stencil(27)
    px = np.array([0.2, 0.5, 0.3])  # values at -1, 0, 1
    py = np.array([0.1, 0.6, 0.3])
    pz = np.array([0.25, 0.5, 0.25])
    f = np.array([px[ci[0] + 1] * py[ci[1] + 1] * pz[ci[2] + 1] for ci in c])
    C = _cumulants(f, c.astype(float))
    mean_x = px[2] - px[0]
    var_x = px[2] + px[0] - mean_x ** 2
    assert abs(C[1, 0, 0] - mean_x) < 1e-15
    assert abs(C[2, 0, 0] - var_x) < 1e-15
    for a, b, g in itertools.product(range(3), repeat=3):
        if sum(x > 0 for x in (a, b, g)) >= 2:
            assert abs(C[a, b, g]) < 1e-15


def test_cumulant_higher_cumulants_vanish_after_collision():
    """At F = 0 the post-collision state has zero cumulants of order >= 3,
    the momentum is conserved, and the second-order central moments are
    relaxed: off-diagonal and deviatoric parts by (1 - omega1), the trace
    towards rho with omega_bulk."""
    q = 27
    c, _, _ = oracle.stencil(q)
    cf = c.astype(float)
    tau, wb = 0.62, 1.4
    w1 = 1.0 / tau
    f = _random_states(q, 25, seed=13, amp=5e-2)
    fs = oracle.collide(oracle.params(q=q, kind=oracle.CUMULANT, tau=tau, omega_bulk=wb), f)
    for k in range(f.shape[0]):
        rho = f[k].sum()
        j = cf.T @ f[k]
        assert abs(fs[k].sum() - rho) < 1e-15
        assert np.allclose(cf.T @ fs[k], j, atol=1e-16)
        Cs = _cumulants(fs[k], cf)
        for a, b, g in itertools.product(range(3), repeat=3):
            if a + b + g >= 3:
                assert abs(Cs[a, b, g]) < 2e-14, (a, b, g, Cs[a, b, g])
        u = j / rho
        d = cf - u[None, :]
        K = np.einsum("i,ia,ib->ab", f[k], d, d)
        Ks = np.einsum("i,ia,ib->ab", fs[k], d, d)
        for a, b in ((0, 1), (0, 2), (1, 2)):
            assert abs(Ks[a, b] - (1 - w1) * K[a, b]) < 1e-15
        assert abs((Ks[0, 0] - Ks[1, 1]) - (1 - w1) * (K[0, 0] - K[1, 1])) < 1e-15
        assert abs((Ks[0, 0] - Ks[2, 2]) - (1 - w1) * (K[0, 0] - K[2, 2])) < 1e-15
        T, Ts = np.trace(K), np.trace(Ks)
        assert abs(Ts - (T + wb * (rho - T))) < 1e-15


def test_cumulant_omega_one_gives_product_equilibrium():
    """With omega1 = omega_bulk = 1 and F = 0, one collision lands exactly on
    the product-form equilibrium rho * prod g(c_a, u_a),
    g(0, u) = 2/3 - u^2, g(+-1, u) = (1/3 + u^2 +- u)/2."""
    q = 27
    c, _, _ = oracle.stencil(q)
    f = _random_states(q, 25, seed=17, amp=5e-2)
    fs = oracle.collide(oracle.params(q=q, kind=oracle.CUMULANT, tau=1.0, omega_bulk=1.0), f)
    for k in range(f.shape[0]):
        rho = f[k].sum()
        u = (c.T @ f[k]) / rho
        assert np.max(np.abs(fs[k] - _product_eq(q, rho, u))) < 1e-15


def test_none_is_identity():
    f = _random_states(19, 5, seed=1)
    assert np.array_equal(oracle.collide(oracle.params(q=19, kind=oracle.NONE), f), f)


def test_cumulant_rejects_d3q19():
    with pytest.raises(RuntimeError):
        oracle.collide(oracle.params(q=19, kind=oracle.CUMULANT), _random_states(19, 1, 0))


# ------------------------------------------------------------------- MRT
def test_mrt_basis_orthogonal_with_published_norms():
    """The D3Q19 moment basis of d'Humieres et al. (2002) is orthogonal over
    the lattice; M M^T is diagonal with the norms published there.  Rows are
    either even or odd under c -> -c, so the basis splits the populations
    into the symmetric and antisymmetric halves TRT works with."""
    M = oracle.mrt_matrix()
    G = M @ M.T
    assert np.array_equal(G, np.diag(np.diag(G)))
    assert np.diag(G).tolist() == [19, 2394, 252, 10, 40, 10, 40, 10, 40, 36, 72, 12, 24,
                                   4, 4, 4, 8, 8, 8]
    _, _, opp = oracle.stencil(19)
    odd = {3, 4, 5, 6, 7, 8, 16, 17, 18}
    for k in range(19):
        sign = -1 if k in odd else 1
        assert np.array_equal(M[k, opp], sign * M[k])
    # the conserved rows are density and momentum
    c, _, _ = oracle.stencil(19)
    assert np.array_equal(M[0], np.ones(19))
    assert np.array_equal(M[[3, 5, 7]], c.T)


def test_mrt_reduces_to_trt_and_srt():
    """Even moments at omega+, odd ones at omega- is TRT (any magic);
    every rate at 1/tau is SRT."""
    tau, magic = 0.77, 0.21
    F = (2e-4, -1e-4, 5e-5)
    omp, omm = 1 / tau, 1 / (0.5 + magic / (tau - 0.5))
    f = _random_states(19, 40, seed=11)
    mrt = oracle.collide(oracle.params(19, oracle.MRT, tau=tau, omega_bulk=omp, force=F,
                                       rates=(omp, omp, omm, omm)), f)
    trt = oracle.collide(oracle.params(19, oracle.TRT, tau=tau, magic=magic, force=F), f)
    assert np.max(np.abs(mrt - trt)) < 1e-15
    mrt = oracle.collide(oracle.params(19, oracle.MRT, tau=tau, omega_bulk=omp, force=F,
                                       rates=(omp,) * 4), f)
    srt = oracle.collide(oracle.params(19, oracle.SRT, tau=tau, force=F), f)
    assert np.max(np.abs(mrt - srt)) < 1e-15


def test_mrt_relaxes_each_moment_group_at_its_rate():
    """Unforced: the non-equilibrium part of moment k is multiplied by
    (1 - s_k), with s_k the rate of its group; conserved moments keep their
    values."""
    tau, wb, rates = 0.9, 1.19, (1.4, 1.1, 1.2, 1.98)
    rate = {1: wb, 2: rates[0], 10: rates[1], 12: rates[1], 4: rates[2], 6: rates[2],
            8: rates[2], 16: rates[3], 17: rates[3], 18: rates[3]}
    for k in (9, 11, 13, 14, 15):
        rate[k] = 1 / tau
    M = oracle.mrt_matrix()
    c, _, _ = oracle.stencil(19)
    f = _random_states(19, 20, seed=2)
    fs = oracle.collide(oracle.params(19, oracle.MRT, tau=tau, omega_bulk=wb, rates=rates), f)
    for n in range(f.shape[0]):
        rho = f[n].sum()
        u = f[n] @ c / rho
        meq = M @ _feq(19, rho, u)
        m, ms = M @ f[n], M @ fs[n]
        for k in range(19):
            if k in (0, 3, 5, 7):
                assert abs(ms[k] - m[k]) < 1e-15
            else:
                assert abs((ms[k] - meq[k]) - (1 - rate[k]) * (m[k] - meq[k])) < 1e-14


# ----------------------------------------------------- central moments
def _central(f, c, u):
    """Central moments k[a, b, g] = sum_i f_i (c - u)_x^a (c - u)_y^b (c - u)_z^g."""
    d = c.astype(float) - u[None, :]
    K = np.zeros((3, 3, 3))
    for a, b, g in itertools.product(range(3), repeat=3):
        K[a, b, g] = np.sum(f * d[:, 0] ** a * d[:, 1] ** b * d[:, 2] ** g)
    return K


def test_cm_relaxes_each_order_to_the_maxwellian():
    """Unforced: central moments of order n = 3..6 approach the Maxwellian's
    (rho times 1, 0, 1/3 per axis for exponents 0, 1, 2) by the factor
    (1 - rate_n); orders 0-2 follow the cumulant operator's rules, which the
    cumulant test pins (same second order)."""
    q = 27
    c, _, _ = oracle.stencil(q)
    tau, wb, rates = 0.7, 1.3, (1.2, 0.8, 1.5, 1.9)
    e = (1.0, 0.0, 1.0 / 3.0)
    f = _random_states(q, 20, seed=19, amp=5e-2)
    fs = oracle.collide(oracle.params(q=q, kind=oracle.CM, tau=tau, omega_bulk=wb,
                                      rates=rates), f)
    cu = oracle.collide(oracle.params(q=q, kind=oracle.CUMULANT, tau=tau, omega_bulk=wb), f)
    for k in range(f.shape[0]):
        rho = f[k].sum()
        u = (c.T @ f[k]) / rho
        K, Ks, Kc = _central(f[k], c, u), _central(fs[k], c, u), _central(cu[k], c, u)
        for a, b, g in itertools.product(range(3), repeat=3):
            n = a + b + g
            if n <= 2:
                assert abs(Ks[a, b, g] - Kc[a, b, g]) < 1e-15
            else:
                keq = rho * e[a] * e[b] * e[g]
                assert abs((Ks[a, b, g] - keq) - (1 - rates[n - 3]) * (K[a, b, g] - keq)) < 1e-15


def test_cm_unit_rates_give_product_equilibrium():
    """All rates one and F = 0: every central moment takes the Maxwellian
    value, which the product-form equilibrium has exactly -- the same state
    the cumulant operator reaches at unit rates."""
    q = 27
    c, _, _ = oracle.stencil(q)
    f = _random_states(q, 25, seed=23, amp=5e-2)
    fs = oracle.collide(oracle.params(q=q, kind=oracle.CM, tau=1.0, omega_bulk=1.0,
                                      rates=(1, 1, 1, 1)), f)
    for k in range(f.shape[0]):
        rho = f[k].sum()
        u = (c.T @ f[k]) / rho
        assert np.max(np.abs(fs[k] - _product_eq(q, rho, u))) < 1e-15


def test_cm_at_rest_with_equal_rates_is_srt():
    """At u = 0 and F = 0 the central moments are raw moments and the
    Maxwellian's equal the moments of f^eq = w rho (the D3Q27 weights carry
    them up to sixth order), so every rate = omega reduces the operator to
    SRT."""
    q = 27
    c, w, _ = oracle.stencil(q)
    rng = np.random.default_rng(29)
    tau = 0.74
    om = 1 / tau
    for _ in range(10):
        f = w * (1 + 0.05 * rng.standard_normal(q))
        f -= w * ((c.T @ f) @ c.T) * 3       # remove the momentum: u = 0 exactly
        assert np.max(np.abs(c.T @ f)) < 1e-16
        a = oracle.collide(oracle.params(q=q, kind=oracle.CM, tau=tau, omega_bulk=om,
                                         rates=(om,) * 4), f[None])[0]
        b = oracle.collide(oracle.params(q=q, kind=oracle.SRT, tau=tau), f[None])[0]
        assert np.max(np.abs(a - b)) < 1e-15


def test_cm_rejects_d3q19():
    with pytest.raises(RuntimeError):
        oracle.collide(oracle.params(q=19, kind=oracle.CM), _random_states(19, 1, 0))
