"""Pins of the implicit-step oracle (Sec. 2.3.1-2.3.2, Eqs. equ_delw to
SGS_phi) against closed forms and invariants.  CPU only.

None of them re-derives an expected value with the oracle's own sweep:
the converged sweeps are compared with Fourier solutions of the circulant
systems they solve on periodic strips (numpy's FFT), with the exact
conservation the predictor inherits from the Roe form on closed meshes,
with the spectral radius of a numerical Euler Jacobian, and with the
explicit update in the small-step limit."""
import math

import numpy as np
import pytest

from oracle import avs_implicit as I
from oracle import avs_oracle as O
from workloads import fields as F
from workloads import meshes as MM


def strip(n):
    """n unit cells in a periodic row (the y direction wraps onto the cell)."""
    return O.Mesh(MM.box2d(n, 1, lx=float(n), ly=1.0, periodic=(True, True)))


def test_colouring_is_proper_and_greedy():
    """No two face neighbours share a colour; a Cartesian grid gets the two
    colours of a checkerboard; a triangle mesh needs at most max degree + 1."""
    box = O.Mesh(MM.box2d(6, 5, periodic=(False, False), sides={'left': 0, 'right': 0, 'bottom': 0, 'top': 0},
                          bcs=[(0, (1, 0, 0, 1))]))
    col = I.cell_colours(box)
    ix, iy = np.arange(30) % 6, np.arange(30) // 6
    assert np.array_equal(col, (ix + iy) % 2)
    tri = O.Mesh(MM.tri_box(7, 6, 3, sides={'left': 0, 'right': 0, 'bottom': 0, 'top': 0}, bcs=[(0, (1, 0, 0, 1))]))
    for m in (box, tri, O.Mesh(MM.box2d(5, 3, periodic=(True, True)))):
        c = I.cell_colours(m)
        for i in range(m.nc):
            for s in m.slots[i]:
                if s.nbr >= 0 and s.nbr != i:
                    assert c[i] != c[s.nbr]
        assert c.max() + 1 <= max(len(sl) for sl in m.slots) + 1
    order = I.sweep_order(I.cell_colours(tri))
    assert sorted(order) == list(range(tri.nc))
    assert all(I.cell_colours(tri)[a] <= I.cell_colours(tri)[b] for a, b in zip(order, order[1:]))


@pytest.mark.parametrize("n", [9, 12])
def test_micro_sweeps_solve_the_upwind_system(n):
    """On a periodic strip with a uniform tau the micro system of Eq.
    SGS_phi is, for each velocity node, circulant: (V/dt + V/tau + A|xi_x|)
    dphi_i - A|xi_x| dphi_upwind = Res_i.  The converged symmetric
    Gauss-Seidel sweeps equal its Fourier solution."""
    mesh = strip(n)
    tree = O.base_forest(2, [-3.0, -3.0], [3.0, 3.0], [4, 4], 0)
    xi = tree.centres()
    rng = np.random.default_rng(n)
    res = rng.standard_normal((2, n, tree.n))
    dt, tau = 0.7, 0.4
    order = I.sweep_order(I.cell_colours(mesh))
    dphi = I.micro_sgs(mesh, xi, dt, np.full(n, tau), res, 80, order)
    expect = np.empty_like(res)
    for k in range(tree.n):
        a = 1.0 / dt + 1.0 / tau + abs(xi[k, 0])
        c = np.zeros(n)
        c[0] = a
        if xi[k, 0] > 0:
            c[1] = -xi[k, 0]          # row i couples to i - 1
        elif xi[k, 0] < 0:
            c[n - 1] = xi[k, 0]       # row i couples to i + 1
        for p in range(2):
            expect[p, :, k] = np.real(np.fft.ifft(np.fft.fft(res[p, :, k]) / np.fft.fft(c)))
    np.testing.assert_allclose(dphi, expect, rtol=1e-12, atol=1e-12)
    # two sweeps (the paper's count) are not yet the solution: the test would see a wrong count
    assert np.abs(I.micro_sgs(mesh, xi, dt, np.full(n, tau), res, 2, order) - expect).max() > 1e-8


def euler_jacobian_x(W, gamma=5.0 / 3.0):
    """Textbook Jacobian dG_x/dW of the 2-D Euler flux with p = (gamma - 1)
    (rho E - rho |U|^2 / 2)."""
    rho, mx, my, E = W
    u, v = mx / rho, my / rho
    q2 = u * u + v * v
    p = (gamma - 1.0) * (E - 0.5 * rho * q2)
    H = (E + p) / rho
    g1 = gamma - 1.0
    return np.array([
        [0.0, 1.0, 0.0, 0.0],
        [0.5 * g1 * q2 - u * u, (3.0 - gamma) * u, -g1 * v, g1],
        [-u * v, v, u, 0.0],
        [u * (0.5 * g1 * q2 - H), H - g1 * u * u, -g1 * u * v, gamma * u],
    ])


def test_predictor_solves_its_linearisation():
    """About a uniform state W0 on a periodic strip, with a tiny right-hand
    side, the predictor of Eq. SGS_w is linear: for each Fourier mode theta
    [V/dt + A r (1 - cos theta) + i A J_x sin theta] w = rhs, J_x the Euler
    Jacobian.  The converged PRSGS increment equals that solution to the
    size of the neglected quadratic terms."""
    n = 10
    mesh = strip(n)
    W0 = O.conserved(np.array([1.2, 0.35, -0.2, 0.9]), 1.0)
    W = np.tile(W0, (n, 1))
    eps = 1e-7
    rhs = eps * np.random.default_rng(5).standard_normal((n, 4))
    r0 = 2.5
    dt = 0.5
    dW = I.macro_sgs(mesh, dt, 1.0, W, rhs, np.full(mesh.nf, r0), 120, I.sweep_order(I.cell_colours(mesh)))
    J = euler_jacobian_x(W0)
    rh = np.fft.fft(rhs, axis=0)
    wh = np.empty_like(rh)
    for m in range(n):
        th = 2.0 * math.pi * m / n
        M = (1.0 / dt + r0 * (1.0 - math.cos(th))) * np.eye(4) + 1j * math.sin(th) * J
        wh[m] = np.linalg.solve(M, rh[m])
    expect = np.real(np.fft.ifft(wh, axis=0))
    assert np.abs(dW - expect).max() < 1e-5 * np.abs(expect).max()


def test_converged_predictor_conserves_on_closed_meshes():
    """Sum_i V_i dW_i = 0 on a periodic mesh once the sweeps have converged:
    the Euler terms dropped from Eq. SGS_w sum to zero over every closed
    cell, so the system is the conservative Roe form in disguise."""
    desc = MM.box2d(5, 4, periodic=(True, True))
    mesh = O.Mesh(desc)
    W = O.conserved(F.perturbed_uniform(mesh.nc, 2, 8, amp=0.2, uamp=0.5), 1.0)
    rng = np.random.default_rng(9)
    Ff = rng.standard_normal((mesh.nf, 4))
    rhs = np.zeros_like(W)
    for i in range(mesh.nc):
        for s in mesh.slots[i]:
            rhs[i] -= s.sigma * mesh.area[s.face] * Ff[s.face]
    r = 2.0 + rng.uniform(0.0, 1.0, mesh.nf)
    dW = I.macro_sgs(mesh, 0.05, 1.0, W, rhs, r, 150, I.sweep_order(I.cell_colours(mesh)))
    tot = np.sum(mesh.vol[:, None] * dW, axis=0)
    assert np.abs(dW).max() > 1e-3
    assert np.abs(tot).max() < 1e-12 * np.abs(mesh.vol[:, None] * dW).sum()


@pytest.mark.parametrize("D", [2, 3])
def test_roe_radius_inviscid_limit(D):
    """r without its viscous part is the spectral radius |U.n| + a of the
    Euler flux Jacobian (eigenvalues of a central-difference Jacobian); the
    viscous part falls off like 1/dl."""
    gas = O.Gas(R=0.7, Pr=2 / 3, omega=0.74, mu_ref=0.3, T_ref=1.0)
    rng = np.random.default_rng(D)
    for _ in range(4):
        rho, T = rng.uniform(0.5, 2.0), rng.uniform(0.5, 3.0)
        U = rng.uniform(-1.0, 1.0, D)
        n = rng.standard_normal(D)
        n /= np.linalg.norm(n)
        W = O.conserved(np.concatenate([[rho], U, [T]]), gas.R)
        J = np.empty((D + 2, D + 2))
        for c in range(D + 2):
            h = 1e-6 * max(1.0, abs(W[c]))
            e = np.zeros(D + 2)
            e[c] = h
            J[:, c] = (I.euler_flux(W + e, n, gas.R) - I.euler_flux(W - e, n, gas.R)) / (2 * h)
        rad = np.max(np.abs(np.linalg.eigvals(J)))
        r_inf = I.roe_radius(rho, U, T, n, 1e300, gas)
        assert abs(r_inf - rad) < 1e-6 * rad
        v1 = I.roe_radius(rho, U, T, n, 0.1, gas) - r_inf
        v2 = I.roe_radius(rho, U, T, n, 0.4, gas) - r_inf
        assert v1 > 0 and abs(v1 / v2 - 4.0) < 1e-9


def test_small_step_limits_are_the_explicit_updates():
    """As dt -> 0 the predictor gives dW/dt -> rhs / V (Eq. equ18 explicit)
    and the micro sweeps dphi/dt -> Res / V, with errors of order dt."""
    desc = MM.box2d(4, 3, periodic=(True, True))
    mesh = O.Mesh(desc)
    W = O.conserved(F.perturbed_uniform(mesh.nc, 2, 4, amp=0.2, uamp=0.5), 1.0)
    rng = np.random.default_rng(4)
    rhs = rng.standard_normal(W.shape)
    r = np.full(mesh.nf, 3.0)
    order = I.sweep_order(I.cell_colours(mesh))
    errs = []
    for dt in (1e-3, 5e-4):
        dW = I.macro_sgs(mesh, dt, 1.0, W, rhs, r, 20, order)
        errs.append(np.abs(dW / dt - rhs / mesh.vol[:, None]).max() / np.abs(rhs / mesh.vol[:, None]).max())
    assert errs[0] < 0.05 and 1.8 < errs[0] / errs[1] < 2.2
    tree = O.base_forest(2, [-3.0, -3.0], [3.0, 3.0], [4, 4], 0)
    res = rng.standard_normal((2, mesh.nc, tree.n))
    errs = []
    for dt in (1e-3, 5e-4):
        dphi = I.micro_sgs(mesh, tree.centres(), dt, np.full(mesh.nc, 0.3), res, 20, order)
        errs.append(np.abs(dphi / dt - res / mesh.vol[None, :, None]).max() / np.abs(res / mesh.vol[None, :, None]).max())
    assert errs[0] < 0.05 and 1.8 < errs[0] / errs[1] < 2.2


def test_uniform_periodic_state_keeps_W():
    """No flux on a uniform periodic state: the predictor has a zero
    right-hand side, so W is unchanged, and once the micro sweeps have
    converged the distribution changes the same way in every cell (after
    two sweeps it does not: Gauss-Seidel is not translation invariant)."""
    desc = MM.box2d(4, 3, periodic=(True, True))
    vs = dict(dim=2, lo=(-5.0, -5.0), hi=(5.0, 5.0), base=(8, 8), max_level=1)
    gas = dict(R=1.0, Pr=2 / 3, omega=0.5, mu_ref=0.05, T_ref=1.0, model=1)
    s = O.Solver(desc, vs, gas, 0.05, 1.0, F.uniform(desc['ncells'], 1.1, (0.3, -0.2), 1.2))
    phi, W, _ = I.step_implicit(s.mesh, s.tree, s.gas, s.dt, s.Kv, s.phi, s.W, 10, 40)
    np.testing.assert_allclose(W, s.W, rtol=0, atol=1e-14)
    assert np.abs(phi - phi[:, :1]).max() < 1e-12 * np.abs(phi).max()
    phi2, _, _ = I.step_implicit(s.mesh, s.tree, s.gas, s.dt, s.Kv, s.phi, s.W, 10, 2)
    assert np.abs(phi2 - phi2[:, :1]).max() > 1e-10 * np.abs(phi2).max()


def test_half_step_cap_closed_form():
    """On a Cartesian box of dx x dy cells and a velocity box reaching X_d,
    every cell's outflow over the box is (dy X_x + dx X_y) per unit content
    dx dy, so the interface half step is min(dt/2, dx dy / (2 (dy X_x + dx X_y)));
    below that bound it is dt/2 exactly."""
    nx, ny, lx, ly = 6, 4, 1.5, 1.0
    mesh = O.Mesh(MM.box2d(nx, ny, lx=lx, ly=ly, periodic=(True, False), sides={'bottom': 0, 'top': 0},
                           bcs=[(0, (1, 0, 0, 1))]))
    tree = O.base_forest(2, [-3.0, -5.0], [7.0, 4.0], [4, 4], 0)
    dx, dy = lx / nx, ly / ny
    cap = dx * dy / (2.0 * (dy * 7.0 + dx * 5.0))
    assert abs(O.half_step(mesh, tree, 1.0) - cap) < 1e-15
    assert O.half_step(mesh, tree, 0.5 * cap) == 0.25 * cap


def test_step_conserves_and_converged_step_is_the_prediction():
    """W^{n+1} from the flux form of Eq. equ18 with the Roe-type implicit
    flux: on a periodic mesh the totals sum_i V_i W_i are kept to round-off
    even after two predictor sweeps (W~ = W^n + dW is not); with converged
    sweeps W^{n+1} equals W~."""
    from oracle import avs_implicit as II
    desc = MM.box2d(5, 4, periodic=(True, True))
    vs = dict(dim=2, lo=(-5.0, -5.0), hi=(5.0, 5.0), base=(8, 8), max_level=1)
    gas = dict(R=1.0, Pr=2 / 3, omega=0.81, mu_ref=0.03, T_ref=1.0, model=1)
    prim = F.perturbed_uniform(desc['ncells'], 2, 12, amp=0.15, uamp=0.5)
    s = O.Solver(desc, vs, gas, 0.05, 1.0, prim)
    tot0 = s.totals()
    _, W2, d2 = II.step_implicit(s.mesh, s.tree, s.gas, s.dt, s.Kv, s.phi, s.W, 2, 2)
    tot2 = np.sum(s.mesh.vol[:, None] * W2, axis=0)
    np.testing.assert_allclose(tot2, tot0, rtol=1e-14, atol=1e-14)
    drift = np.sum(s.mesh.vol[:, None] * d2.predicted, axis=0) - tot0
    assert np.abs(drift).max() > 1e-8
    _, W60, d60 = II.step_implicit(s.mesh, s.tree, s.gas, s.dt, s.Kv, s.phi, s.W, 120, 2)
    assert np.abs(W60 - d60.predicted).max() < 1e-12 * np.abs(W60).max()


def test_walls_pass_no_mass():
    """In a box closed by isothermal walls the implicit step keeps the total
    mass to round-off after two predictor sweeps: the explicit wall flux has
    zero net mass flux (diffuse reflection) and the mirror state cancels the
    mass and energy increments through the wall, leaving only the normal
    momentum flux p + rho (U.n)^2 from each side."""
    from oracle import avs_implicit as II
    n = np.array([0.6, -0.8])
    Wc = O.conserved(np.array([1.3, 0.4, -0.25, 0.9]), 1.0)
    Wm = II.mirror(Wc, n)
    assert np.allclose(II.mirror(Wm, n), Wc, rtol=0, atol=1e-15)
    Gc, Gm = II.euler_flux(Wc, n, 1.0), II.euler_flux(Wm, n, 1.0)
    assert abs(Gc[0] + Gm[0]) < 1e-15 and abs(Gc[3] + Gm[3]) < 1e-14
    # the normal momentum flux doubles, p + rho (U.n)^2 from each side
    un = 0.4 * 0.6 + (-0.25) * (-0.8)
    np.testing.assert_allclose(Gc[1:3] + Gm[1:3], 2.0 * (1.3 * 0.9 + 1.3 * un * un) * n, rtol=1e-14)
    desc = MM.box2d(5, 4, sides={'left': 0, 'right': 0, 'bottom': 0, 'top': 1},
                    bcs=[(0, (1.0, 0.0, 0.0, 1.0)), (0, (1.0, 0.3, 0.0, 1.2))])
    vs = dict(dim=2, lo=(-5.0, -5.0), hi=(5.0, 5.0), base=(8, 8), max_level=1)
    gas = dict(R=1.0, Pr=2 / 3, omega=0.81, mu_ref=0.03, T_ref=1.0, model=1)
    s = O.Solver(desc, vs, gas, 0.05, 1.0, F.perturbed_uniform(desc['ncells'], 2, 13, amp=0.15, uamp=0.4))
    m0 = s.totals()[0]
    _, W2, d2 = II.step_implicit(s.mesh, s.tree, s.gas, s.dt, s.Kv, s.phi, s.W, 2, 2)
    assert abs(np.sum(s.mesh.vol * W2[:, 0]) - m0) < 1e-14 * m0
