"""Pins of the Rykov diatomic-model oracle (Eqs. GHR_equ, equ11-equ13,
updat_W, equ8, equ19) against closed forms of Gaussian moments, reached to
round-off by the mid-point rule on a fine velocity mesh.  CPU only."""
import math

import numpy as np
import pytest

from oracle import avs_oracle as O
from oracle import avs_rykov as RY


def fine(D):
    n, half = (160, 10.0) if D == 2 else (56, 9.0)
    t = O.base_forest(D, [-half] * D, [half] * D, [n] * D, 0)
    return t.centres(), t.weights()


def state(D):
    rho, Tt, Tr = 1.3, 1.1, 0.8
    U = np.array([0.4, -0.3, 0.2][:D])
    qt = np.array([0.06, -0.09, 0.04][:D])
    qr = np.array([-0.05, 0.03, 0.07][:D])
    return rho, U, Tt, Tr, qt, qr


@pytest.mark.parametrize("D", [2, 3])
def test_parts_moments_closed_form(D):
    """t part: mass rho, momentum rho U, translational energy 3/2 rho R T_t,
    int R^t = rho R T_r; r part the same at T (T_r replaced by T); the
    Shakhov-type corrections carry no mass, momentum or energy."""
    gas = RY.RykovGas(R=0.5)
    xi, A = fine(D)
    rho, U, Tt, Tr, qt, qr = state(D)
    T = (3 * Tt + 2 * Tr) / 5
    t, r = RY.rykov_parts(rho, U, Tt, Tr, qt, qr, xi, gas)
    for part, Ttr, Trot in ((t, Tt, Tr), (r, T, T)):
        m = RY.moments(part, xi, A)
        np.testing.assert_allclose(m[0], rho, rtol=1e-12)
        np.testing.assert_allclose(m[1:1 + D], rho * U, rtol=1e-12, atol=1e-13)
        e_tr = 0.5 * rho * U @ U + 1.5 * rho * gas.R * Ttr
        np.testing.assert_allclose(m[1 + D] - m[2 + D], e_tr, rtol=1e-12)
        np.testing.assert_allclose(m[2 + D], rho * gas.R * Trot, rtol=1e-12)
    if D == 3:
        assert np.all(t[1] == 0) and np.all(r[1] == 0)


@pytest.mark.parametrize("D", [2, 3])
def test_parts_heat_fluxes_closed_form(D):
    """q_t of the t part is q_t/3 and of the r part omega_0 q_t/3 (a
    Shakhov correction with coefficient 1/15 = (1 - 2/3)/5); int c R^t =
    (1 - delta)(T_r/T_t) q_r and int c R^r = omega_1 (1 - delta) q_r."""
    gas = RY.RykovGas(R=0.5)
    xi, A = fine(D)
    rho, U, Tt, Tr, qt, qr = state(D)
    t, r = RY.rykov_parts(rho, U, Tt, Tr, qt, qr, xi, gas)
    qtt, qrt = RY.heat_fluxes(t, xi, A, U)
    qtr, qrr = RY.heat_fluxes(r, xi, A, U)
    np.testing.assert_allclose(qtt, qt / 3, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(qtr, gas.omega0 * qt / 3, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(qrt, (1 - gas.delta) * (Tr / Tt) * qr, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(qrr, gas.omega1 * (1 - gas.delta) * qr, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("D", [2, 3])
def test_collision_conserves_and_exchanges_rotational_energy(D):
    """The Rykov equilibrium has the mass, momentum and total energy of the
    state (the collision conserves them), and its rotational energy moves
    1/Z of the way from rho R T_r to rho R T: (int g^R - rho E_rot)/tau is
    the source (rho R T - rho E_rot)/(Z tau) of Eq. equ19."""
    gas = RY.RykovGas(R=0.5, Z_rot=3.5)
    xi, A = fine(D)
    rho, U, Tt, Tr, qt, qr = state(D)
    W = RY.conserved(rho, U, Tt, Tr, gas.R)
    g = RY.rykov_equilibrium(rho, U, Tt, Tr, qt, qr, xi, gas)
    m = RY.moments(g, xi, A)
    np.testing.assert_allclose(m[:2 + D], W[:2 + D], rtol=1e-12, atol=1e-13)
    tau = 0.37
    np.testing.assert_allclose((m[2 + D] - W[2 + D]) / tau, RY.rotational_source(W, tau, gas), rtol=1e-11)
    rho_, U_, Tt_, Tr_, T_ = RY.temperatures(W, gas.R)
    assert abs(Tt_ - Tt) < 1e-14 and abs(Tr_ - Tr) < 1e-14 and abs(T_ - (3 * Tt + 2 * Tr) / 5) < 1e-14


def test_relaxation_number_limits():
    """Z = 1: the equilibrium is the r part alone (full exchange at every
    collision); Z -> infinity: the t part (no exchange)."""
    xi, A = fine(2)
    rho, U, Tt, Tr, qt, qr = state(2)
    t, r = RY.rykov_parts(rho, U, Tt, Tr, qt, qr, xi, RY.RykovGas(R=0.5))
    g1 = RY.rykov_equilibrium(rho, U, Tt, Tr, qt, qr, xi, RY.RykovGas(R=0.5, Z_rot=1.0))
    assert np.array_equal(g1, r)
    ginf = RY.rykov_equilibrium(rho, U, Tt, Tr, qt, qr, xi, RY.RykovGas(R=0.5, Z_rot=1e300))
    assert np.allclose(ginf, t, rtol=0, atol=1e-300 + 1e-15 * np.abs(t).max())


def test_equal_temperatures_and_zero_heat_flux_give_maxwellians():
    """At T_t = T_r and zero heat fluxes every part is the Maxwellian pair:
    G = g(T), H = (3 - D) R T g(T), R = R T g(T)."""
    gas = RY.RykovGas(R=0.7)
    xi, A = fine(2)
    rho, U, T = 0.9, np.array([0.2, 0.5]), 1.3
    z = np.zeros(2)
    g = RY.rykov_equilibrium(rho, U, T, T, z, z, xi, gas)
    m = O.maxwell(rho, U, T, xi, gas.R)
    np.testing.assert_allclose(g[0], m, rtol=1e-14, atol=1e-300)
    np.testing.assert_allclose(g[1], gas.R * T * m, rtol=1e-14, atol=1e-300)
    np.testing.assert_allclose(g[2], gas.R * T * m, rtol=1e-14, atol=1e-300)


def test_interface_rotational_relaxation_limits():
    gas = RY.RykovGas(R=0.5, Z_rot=4.0)
    assert RY.interface_rotational_energy(2.0, 3.0, 0.0, 0.1, gas) == 2.0
    assert abs(RY.interface_rotational_energy(2.0, 3.0, 1e12, 0.1, gas) - 3.0) < 1e-9
    # linear in its inputs: the weights sum to one
    a = RY.interface_rotational_energy(1.0, 0.0, 0.3, 0.1, gas)
    b = RY.interface_rotational_energy(0.0, 1.0, 0.3, 0.1, gas)
    assert abs(a + b - 1.0) < 1e-15 and abs(b - 0.3 / (0.4 + 0.3)) < 1e-15


def periodic_case(nx=5, ny=4, seed=1, omega=0.74, dt=2e-3, Tr_amp=0.1, uamp=0.3, max_level=0):
    from workloads import meshes as MM
    mesh = MM.box2d(nx, ny, periodic=(True, True))
    tree = O.base_forest(2, [-6.0, -6.0], [6.0, 6.0], [16, 16], max_level)
    vgas = dict(R=0.5, Pr=2 / 3, omega=omega, mu_ref=0.05, T_ref=1.0, model=1)
    gas = RY.RykovGas(R=0.5, Z_rot=3.5)
    rng = np.random.default_rng(seed)
    n = nx * ny
    prim = np.concatenate([1 + 0.1 * rng.uniform(-1, 1, (n, 1)), uamp * rng.uniform(-1, 1, (n, 2)),
                           1 + 0.1 * rng.uniform(-1, 1, (n, 1)), 0.8 + Tr_amp * rng.uniform(-1, 1, (n, 1))], axis=1)
    return RY.DiatomicSolver(mesh, tree, vgas, gas, dt, 1.0, prim)


def test_diatomic_step_conserves_and_keeps_moments():
    """Periodic box: mass, momentum and total energy are kept to round-off
    (the rotational energy is exchanged with the translational one), and the
    moments of phi equal W after every step (the closed target and the
    point-implicit exchange use the same tau)."""
    s = periodic_case()
    tot0 = s.totals()
    np.testing.assert_allclose(s.vdf_moments(), s.W, rtol=0, atol=1e-14)
    for _ in range(3):
        s.step(1)
        np.testing.assert_allclose(s.vdf_moments(), s.W, rtol=0, atol=1e-13)
    tot = s.totals()
    np.testing.assert_allclose(tot[:4], tot0[:4], rtol=1e-14, atol=1e-14)
    assert abs(tot[4] - tot0[4]) > 1e-5             # energy does move into rotation


def test_homogeneous_rotational_relaxation_closed_form():
    """A uniform gas at rest with T_r < T_t: with omega = 1 the relaxation
    time mu(T_t)/p_t is constant, so the rotational energy obeys implicit
    Euler on dE/dt = (rho R T - E)/(Z tau) exactly:
    E_n = rho R T + (E_0 - rho R T) (1 + dt/(Z tau))^-n, T fixed by the
    internal energy."""
    s = periodic_case(nx=2, ny=2, omega=1.0, dt=0.01, Tr_amp=0.0, uamp=0.0)
    s.W[:] = s.W[0]
    s.phi[:] = s.phi[:, :1]
    rho, U, Tt, Tr, T = RY.temperatures(s.W[0], 0.5)
    tau = 0.05 / (rho * 0.5 * 1.0)                   # mu_ref (T/T_ref)^1 / (rho R T)
    E0, Eeq = s.W[0, 4], rho * 0.5 * T
    k = 0.01 / (3.5 * tau)
    for nstep in range(1, 6):
        s.step(1)
        np.testing.assert_allclose(s.W[:, 4], Eeq + (E0 - Eeq) * (1 + k) ** -nstep, rtol=1e-13)
        assert abs(RY.temperatures(s.W[0], 0.5)[4] - T) < 1e-14


def test_diatomic_criterion_sums_and_remap_conserves():
    """When M[phi] = W the criterion's terms are fractions: sum_k M1 = sum_k
    M2 = 1 in every cell (mass and internal energy, rotation included).
    After an adaptation with splits and merges the remapped state has the
    moments W to round-off; a split followed by the merge of the same
    leaves returns the consanguinity values exactly."""
    s = periodic_case(nx=3, ny=2, max_level=1)
    xi, A = s.tree.centres(), s.tree.weights()
    for i in range(s.mesh.nc):
        Mk = RY.criterion_dia(s.phi[:, i:i + 1], s.W[i:i + 1], s.tree)
        # one cell: Mk = max(M1, M2); recompute both sums through the definition
        rho, U, Tt, Tr, T = RY.temperatures(s.W[i], 0.5)
        c = xi - U[None, :]
        eint = s.W[i, 3] - 0.5 * rho * U @ U
        M1 = A * s.phi[0, i] / rho
        M2 = A * (0.5 * (np.sum(c * c, axis=1) * s.phi[0, i] + s.phi[1, i]) + s.phi[2, i]) / eint
        assert abs(M1.sum() - 1) < 1e-13 and abs(M2.sum() - 1) < 1e-13
        assert np.array_equal(Mk, np.maximum(M1, M2)) or np.allclose(Mk, np.maximum(M1, M2), rtol=1e-15)
    s.step(1)
    Mk = RY.criterion_dia(s.phi, s.W, s.tree)
    C1 = np.quantile(Mk, 0.8)
    eff, plan, _ = s.adapt(C1, np.quantile(Mk, 0.2))
    assert (eff == 1).any()
    s.remap()
    np.testing.assert_allclose(s.vdf_moments(), s.W, rtol=0, atol=1e-13)
    # split everything, then merge everything back: consanguinity is exact
    s = periodic_case(nx=3, ny=2, max_level=1)
    phi0, tree0 = s.phi.copy(), s.tree
    s.adapt(-1.0, -2.0)
    p_split = O.remap(s.phi, s.plan, 2)
    t_split = s.plan.tree
    eff = O.resolve_merges(O.raw_flags(np.zeros(t_split.n), t_split, 1.0, 0.5), t_split)
    back = O.make_plan(eff, t_split)
    assert back.tree.n == tree0.n
    assert np.array_equal(O.remap(p_split, back, 2), phi0)


# ------------------------------------------------------------ implicit step
@pytest.mark.parametrize("D", [2, 3])
def test_diatomic_euler_flux_and_its_spectral_radius(D):
    """With E_rot = 0 the first D + 2 rows are the monatomic Euler flux (an
    independent function); the rotational row is E_rot U.n; the spectral
    radius of the flux Jacobian (central differences) is the inviscid r,
    |U.n| + sqrt(5/3 R T_t): E_rot is only carried and does not enter p."""
    from oracle import avs_implicit as IM
    rng = np.random.default_rng(40 + D)
    R = 0.6
    n = rng.normal(size=D)
    n /= np.linalg.norm(n)
    rho, U, Tt, Tr = 1.3, rng.uniform(-0.5, 0.5, D), 1.1, 0.8
    W = RY.conserved(rho, U, Tt, Tr, R)
    W0 = W.copy()
    W0[1 + D] -= W0[2 + D]
    W0[2 + D] = 0.0
    Fm = IM.euler_flux(W0[:D + 2], n, R)
    np.testing.assert_allclose(RY.euler_flux_dia(W0, n, R)[:D + 2], Fm, rtol=1e-15, atol=1e-15)
    F = RY.euler_flux_dia(W, n, R)
    assert abs(F[2 + D] - W[2 + D] * float(U @ n)) < 1e-15
    J = np.empty((D + 3, D + 3))
    for m in range(D + 3):
        e = np.zeros(D + 3)
        e[m] = 1e-6 * max(1.0, abs(W[m]))
        J[:, m] = (RY.euler_flux_dia(W + e, n, R) - RY.euler_flux_dia(W - e, n, R)) / (2 * e[m])
    rad = np.max(np.abs(np.linalg.eigvals(J)))
    r0 = RY.roe_radius_dia(rho, U, Tt, 0.0, n, 1.0, R)
    assert abs(rad - r0) < 1e-7 * r0
    assert abs(r0 - abs(float(U @ n)) - math.sqrt(5 / 3 * R * Tt)) < 1e-14


def test_implicit_diatomic_homogeneous_relaxation_closed_form():
    """A uniform gas at rest with T_r < T_t, omega = 1 (constant tau):
    converged predictor sweeps give the implicit-Euler increment of Eq.
    SGS_wrot, dE = k (rho R T - E)/(1 + k) with k = dt/(Z tau), and nothing
    else moves; W^{n+1} follows the same closed-form sequence; with converged
    micro sweeps the moments of phi equal W."""
    s = periodic_case(nx=2, ny=2, omega=1.0, dt=0.01, Tr_amp=0.0, uamp=0.0)
    s.W[:] = s.W[0]
    s.phi[:] = s.phi[:, :1]
    rho, U, Tt, Tr, T = RY.temperatures(s.W[0], 0.5)
    tau = 0.05 / (rho * 0.5 * 1.0)
    E0, Eeq = s.W[0, 4], rho * 0.5 * T
    k = 0.01 / (3.5 * tau)
    for nstep in range(1, 4):
        E = s.W[0, 4]
        W = s.W.copy()
        s.step_implicit(1, 40, 40)
        dW = s.predicted - W
        np.testing.assert_allclose(dW[:, 4], k * (Eeq - E) / (1 + k), rtol=1e-12)
        assert np.abs(dW[:, :4]).max() < 1e-15
        np.testing.assert_allclose(s.W[:, 4], Eeq + (E0 - Eeq) * (1 + k) ** -nstep, rtol=1e-13)
        np.testing.assert_allclose(s.vdf_moments(), s.W, rtol=0, atol=1e-12)


def test_implicit_diatomic_conserves_and_tends_to_the_explicit_step():
    """Periodic box: after two sweeps of each kind the implicit step keeps
    mass, momentum and total energy to round-off (flux form); its difference
    from the explicit step, relative to the step's change, halves with dt
    (both are first order; they differ at O(dt^2))."""
    s = periodic_case()
    tot0 = s.totals()
    s.step_implicit(2, 2, 2)
    tot = s.totals()
    np.testing.assert_allclose(tot[:4], tot0[:4], rtol=1e-14, atol=1e-14)
    e = []
    for dt in (4e-3, 2e-3, 1e-3):
        c = periodic_case(dt=dt)
        pe, We = RY.step_dia(c.mesh, c.tree, c.vgas, c.gas, dt, c.Kv, c.phi, c.W)
        pi, Wi, _ = RY.step_implicit_dia(c.mesh, c.tree, c.vgas, c.gas, dt, c.Kv, c.phi, c.W, 30, 30)
        e.append((np.abs(pi - pe).max() / np.abs(pe - c.phi).max(), np.abs(Wi - We).max() / np.abs(We - c.W).max()))
    for a, b in zip(e, e[1:]):
        assert 1.8 < a[0] / b[0] < 2.2 and 1.8 < a[1] / b[1] < 2.2


def test_diatomic_criterion_probe_equals_an_equilibrium_cell():
    """A probe state is counted as an equilibrium cell: with one cell set to
    the equilibrium triple of (rho, U, T), the criterion of that cell alone
    equals the criterion of the probe (rho, U, T) alone to round-off, and a
    probe only ever raises M_k."""
    s = periodic_case(nx=2, ny=2, max_level=1)
    xi = s.tree.centres()
    rho, U, T = 0.8, np.array([0.3, -0.2]), 1.2
    phi = RY.triple(rho, U, T, xi, 0.5)[:, None, :]
    W = RY.conserved(rho, U, T, T, 0.5)[None, :]
    m_cell = RY.criterion_dia(phi, W, s.tree)
    m_probe = RY.criterion_dia(phi[:, :0], W[:0], s.tree, probes=[[rho, *U, T]], R=0.5)
    np.testing.assert_allclose(m_probe, m_cell, rtol=1e-14)
    base = RY.criterion_dia(s.phi, s.W, s.tree)
    both = RY.criterion_dia(s.phi, s.W, s.tree, probes=[[rho, *U, T]], R=0.5)
    assert np.all(both >= base) and np.array_equal(both, np.maximum(base, m_probe))


def test_implicit_diatomic_without_sweeps_is_the_explicit_macro_update():
    """No sweeps: dW = 0, so the implicit flux is F^n exactly and W^{n+1}
    equals the explicit step's bit for bit (transport, then the same
    rotational exchange); with no micro sweeps phi is unchanged."""
    s = periodic_case()
    pe, We = RY.step_dia(s.mesh, s.tree, s.vgas, s.gas, s.dt, s.Kv, s.phi, s.W)
    pi, Wi, Wp = RY.step_implicit_dia(s.mesh, s.tree, s.vgas, s.gas, s.dt, s.Kv, s.phi, s.W, 0, 0)
    assert np.array_equal(Wi, We) and np.array_equal(Wp, s.W) and np.array_equal(pi, s.phi)
