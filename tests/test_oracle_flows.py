"""Flow-level pins of the dense FP64 oracle: conservation, fixed points,
pure streaming, the analytic Poiseuille profile and shear-wave viscosity."""
import numpy as np
import pytest

import oracle
from paper_2408_06880_amd import inputs


def _feq_field(q, rho, u):
    """Polynomial equilibrium for per-cell rho [Z,Y,X] and u [3,Z,Y,X]."""
    c, w, _ = oracle.stencil(q)
    cu = np.einsum("ia,a...->i...", c.astype(float), u)
    uu = np.sum(u * u, axis=0)
    return w[:, None, None, None] * rho[None] * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * uu[None])


def _product_eq_field(q, rho, u):
    c, _, _ = oracle.stencil(q)
    out = np.empty((q,) + rho.shape)
    for i in range(q):
        v = rho.copy()
        for a in range(3):
            if c[i, a] == 0:
                v = v * (2.0 / 3.0 - u[a] ** 2)
            else:
                v = v * (1.0 / 3.0 + u[a] ** 2 + c[i, a] * u[a]) / 2.0
        out[i] = v
    return out


@pytest.mark.parametrize("kind,tau,magic,tol", [
    (oracle.TRT, 0.8, 3.0 / 16.0, 1e-9),        # TRT magic 3/16: halfway walls exact
    (oracle.TRT, 1.4, 3.0 / 16.0, 1e-9),
    (oracle.SRT, 0.5 + np.sqrt(3.0 / 16.0), 0.0, 1e-9),  # SRT at Lambda = 3/16
    (oracle.SRT, 0.8, 0.0, 1e-2),               # SRT elsewhere: small viscosity-dependent slip
])
def test_poiseuille_body_force(kind, tau, magic, tol):
    """Body-forced channel, walls halfway outside the first/last fluid layer:
    u(y) = F/(2 rho nu) (y + 1/2)(H - 1/2 - y), nu = (tau - 1/2)/3."""
    H, F = 12, 1e-6
    lab, per = inputs.channel(2, H, 2)
    p = oracle.params(q=19, kind=kind, tau=tau, magic=magic, force=(F, 0, 0))
    A = oracle.dense_run(p, lab, per, 12000, oracle.dense_init(19, lab))
    rho, u = oracle.dense_moments(p, lab, A)
    nu = (tau - 0.5) / 3.0
    y = np.arange(H)
    ua = F / (2 * nu) * (y + 0.5) * (H - 0.5 - y)
    ux = u[0, 0, :, 0]
    assert np.max(np.abs(rho - 1.0)) < 1e-12
    assert np.max(np.abs(ux - ua)) / ua.max() < tol
    # symmetric about the centre line, no wall-normal flow
    assert np.max(np.abs(ux - ux[::-1])) < 1e-12 * ua.max() + 1e-20
    assert np.max(np.abs(u[1])) < 1e-10 * ua.max()


@pytest.mark.parametrize("tau,even", [(0.8, (1.4, 1.4)), (0.8, (1.1, 1.7)), (1.4, (1.6, 0.9))])
def test_poiseuille_mrt(tau, even):
    """MRT with both odd groups (q, m) at the omega- of Lambda = 3/16 puts
    the halfway walls exactly, whatever the even non-hydrodynamic rates;
    d'Humieres' rates (q 1.2, m 1.98) leave a slip error."""
    H, F = 12, 1e-6
    lab, per = inputs.channel(2, H, 2)
    omm = 1 / (0.5 + (3 / 16) / (tau - 0.5))
    nu = (tau - 0.5) / 3.0
    y = np.arange(H)
    ua = F / (2 * nu) * (y + 0.5) * (H - 0.5 - y)
    errs = []
    for rates in ((even[0], even[1], omm, omm), oracle.MRT_RATES):
        p = oracle.params(q=19, kind=oracle.MRT, tau=tau, omega_bulk=1.19, force=(F, 0, 0),
                          rates=rates)
        A = oracle.dense_run(p, lab, per, 12000, oracle.dense_init(19, lab))
        _, u = oracle.dense_moments(p, lab, A)
        errs.append(np.max(np.abs(u[0, 0, :, 0] - ua)) / ua.max())
    assert errs[0] < 1e-9
    assert errs[1] > 1e-3


def _shear_wave_rate(kind, tau, L, U0=0.0, q=27, steps=(200, 600)):
    lab, per = inputs.periodic_box(1, L, 1)
    y = np.arange(L)
    rho = np.ones((1, L, 1))
    u = np.zeros((3, 1, L, 1))
    U = 1e-4
    u[0, 0, :, 0] = U0 + U * np.sin(2 * np.pi * y / L)
    eq = _product_eq_field if kind in (oracle.CUMULANT, oracle.CM) else _feq_field
    A = eq(q, rho, u)
    p = oracle.params(q=q, kind=kind, tau=tau, magic=3.0 / 16.0)
    amps = []
    t = 0
    for t_next in steps:
        A = oracle.dense_run(p, lab, per, t_next - t, A)
        t = t_next
        _, uu = oracle.dense_moments(p, lab, A)
        amps.append(2.0 / L * np.sum((uu[0, 0, :, 0] - U0) * np.sin(2 * np.pi * y / L)))
    rate = -np.log(amps[1] / amps[0]) / (steps[1] - steps[0])
    nu = (tau - 0.5) / 3.0
    return rate / (nu * (2 * np.pi / L) ** 2)


@pytest.mark.parametrize("kind,q", [(oracle.SRT, 19), (oracle.TRT, 19), (oracle.CUMULANT, 27),
                                    (oracle.MRT, 19), (oracle.CM, 27)])
def test_shear_wave_viscosity(kind, q):
    """A shear wave decays as exp(-nu k^2 t); the lattice error is O(k^2), so
    the relative rate error must shrink about 4x when L doubles."""
    e32 = abs(_shear_wave_rate(kind, 0.8, 32, q=q, steps=(100, 300)) - 1.0)
    e64 = abs(_shear_wave_rate(kind, 0.8, 64, q=q, steps=(400, 1200)) - 1.0)
    assert e64 < 1e-2
    assert e64 < 0.35 * e32 or e64 < 1e-6


@pytest.mark.parametrize("kind", [oracle.CUMULANT, oracle.CM])
def test_shear_wave_galilean(kind):
    """Cumulant and central moments: the same decay rate on top of a
    uniform background flow."""
    r0 = _shear_wave_rate(kind, 0.8, 32, steps=(100, 300))
    r1 = _shear_wave_rate(kind, 0.8, 32, U0=0.05, steps=(100, 300))
    assert abs(r1 - r0) < 2e-2


@pytest.fixture(scope="module")
def small_packing():
    lab, info = inputs.rsa_spheres(20, 2.0, 3.5, 0.6, seed=3, max_rejects=2000)
    return lab


def test_mass_conservation_packing(small_packing):
    """Bounce-back and periodic streaming move populations without loss and
    the Guo source has zero sum: mass is conserved to rounding."""
    lab = small_packing
    p = oracle.params(q=19, kind=oracle.SRT, tau=0.8, force=(1e-6, 0, 0))
    A0 = oracle.dense_init(19, lab)
    m0, _, nf = oracle.dense_reduce(p, lab, A0)
    A = oracle.dense_run(p, lab, 7, 200, A0)
    m1, J, _ = oracle.dense_reduce(p, lab, A)
    assert abs(m1 - m0) / m0 < 1e-13
    assert nf == int(np.count_nonzero(lab == 0))
    assert 0 < J[0] / nf < 200 * 1e-6


@pytest.mark.parametrize("q,kind", [(19, oracle.SRT), (19, oracle.TRT), (27, oracle.CUMULANT)])
def test_momentum_growth_periodic(q, kind):
    """Fully fluid periodic box: total momentum grows by N*F every step."""
    rng = np.random.default_rng(2)
    lab, per = inputs.periodic_box(6, 5, 4)
    rho = 1 + 0.01 * rng.standard_normal(lab.shape)
    u = 0.01 * rng.standard_normal((3,) + lab.shape)
    A0 = _feq_field(q, rho, u) * (1 + 1e-3 * rng.standard_normal((q,) + lab.shape))
    F = np.array([1e-5, -2e-6, 3e-6])
    p = oracle.params(q=q, kind=kind, tau=0.7, force=F)
    _, J0, _ = oracle.dense_reduce(p, lab, A0)
    n = 40
    A = oracle.dense_run(p, lab, per, n, A0)
    _, J, nf = oracle.dense_reduce(p, lab, A)
    assert np.allclose(J - J0, n * nf * F, rtol=1e-10, atol=1e-15)


def test_rest_state_is_fixed_point(small_packing):
    lab = small_packing
    p = oracle.params(q=19, kind=oracle.TRT, tau=0.8)
    A0 = oracle.dense_init(19, lab)
    A = oracle.dense_run(p, lab, 7, 50, A0)
    assert np.max(np.abs(A - A0)) < 1e-15


@pytest.mark.parametrize("q", [19, 27])
def test_pure_streaming_translates(q):
    """Collision NONE: after n steps each population is shifted by n*c_i
    (periodic box), bit for bit."""
    rng = np.random.default_rng(4)
    lab, per = inputs.periodic_box(5, 6, 7)
    A0 = rng.random((q,) + lab.shape)
    n = 3
    A = oracle.dense_run(oracle.params(q=q, kind=oracle.NONE), lab, per, n, A0)
    c, _, _ = oracle.stencil(q)
    for i in range(q):
        ref = np.roll(A0[i], shift=(n * c[i, 2], n * c[i, 1], n * c[i, 0]), axis=(0, 1, 2))
        assert np.array_equal(A[i], ref)


def test_pure_streaming_bounces_off_walls():
    """Collision NONE in a closed 1-cell-wide column along x: a population
    travelling +x reaches the wall, reflects into -x, and returns; after
    2*nx steps every x-population is back where it started."""
    nx = 5
    lab = np.zeros((1, 1, nx), np.uint8)
    rng = np.random.default_rng(8)
    A0 = rng.random((19,) + lab.shape)
    A = oracle.dense_run(oracle.params(q=19, kind=oracle.NONE), lab, 0, 2 * nx, A0)
    assert np.array_equal(A[1], A0[1]) and np.array_equal(A[2], A0[2])


@pytest.mark.parametrize("kind,tau", [(oracle.SRT, 0.8), (oracle.TRT, 1.2)])
def test_couette_moving_wall(kind, tau):
    """Moving-wall (UBB) layer below the fluid, no-slip box face above:
    steady Couette flow u(y') = U (H - 1/2 - y') / H with both walls halfway
    between lattice nodes, reproduced to rounding."""
    H, U = 8, 0.01
    lab = np.zeros((2, H + 1, 2), np.uint8)
    lab[:, 0, :] = 2                       # class 0 = moving wall
    p = oracle.params(q=19, kind=kind, tau=tau, magic=3 / 16,
                      classes=[(oracle.BC_UBB, (U, 0.0, 0.0), 1.0)])
    per = inputs.PERIODIC_X | inputs.PERIODIC_Z
    A = oracle.dense_run(p, lab, per, 6000, oracle.dense_init(19, lab))
    rho, u = oracle.dense_moments(p, lab, A)
    yp = np.arange(H)
    ua = U * (H - 0.5 - yp) / H
    assert np.max(np.abs(u[0, 0, 1:, 0] - ua)) < 1e-10 * U
    assert np.max(np.abs(rho[0, 1:, 0] - 1.0)) < 1e-10


def test_pressure_outlet_returns_equilibrium_with_velocity():
    """Anti-bounce-back at a pressure outlet returns the sum of the two
    opposite second-order equilibria at (rho_out, u): a cell in equilibrium
    at rho_out moving with u gets exactly the equilibrium population back
    through the outlet, O(u^2) term included (pure streaming, no collision,
    so the pulled values are the boundary rule's output)."""
    lab = np.zeros((1, 1, 3), np.uint8)
    lab[0, 0, 2] = 2                      # x = 2: pressure outlet; periodic in y and z
    rho_out, u0 = 1.003, (0.05, 0.02, -0.01)
    p = oracle.params(q=19, kind=oracle.NONE,
                      classes=[(oracle.BC_PRESSURE, (0, 0, 0), rho_out)])
    rho = np.full((1, 1, 3), rho_out)
    u = np.zeros((3, 1, 1, 3))
    for a in range(3):
        u[a] = u0[a]
    A = _feq_field(19, rho, u)
    B = oracle.dense_run(p, lab, 6, 1, A)
    c, _, _ = oracle.stencil(19)
    from_outlet = [i for i in range(1, 19) if c[i, 0] == -1]   # pulled from x + 1 = outlet
    assert len(from_outlet) == 5
    for i in from_outlet:
        assert abs(B[i, 0, 0, 1] - A[i, 0, 0, 1]) <= 1e-14 * A[i, 0, 0, 1]
    # without the velocity terms the returned value would be off by
    # 2 w rho (9/2 (c.u)^2 - 3/2 u.u), far above rounding
    assert abs(4.5 * 0.05 ** 2 - 1.5 * (0.05 ** 2 + 0.02 ** 2 + 0.01 ** 2)) > 1e-4


def test_pressure_outlet_sets_density():
    """Closed box with one pressure-outlet face and no force: the fluid
    relaxes to rest at the outlet density (anti-bounce-back rule)."""
    lab = np.zeros((3, 4, 5), np.uint8)
    lab[:, :, 4] = 2                      # class 0 = pressure outlet at x = 4
    rho_out = 1.01
    p = oracle.params(q=19, kind=oracle.SRT, tau=0.9,
                      classes=[(oracle.BC_PRESSURE, (0, 0, 0), rho_out)])
    A = oracle.dense_run(p, lab, 0, 4000, oracle.dense_init(19, lab))
    rho, u = oracle.dense_moments(p, lab, A)
    fl = lab == 0
    assert np.max(np.abs(rho[fl] - rho_out)) < 1e-9
    assert np.max(np.abs(u[:, fl])) < 1e-9
