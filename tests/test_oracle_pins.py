"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

Each test names what it pins.  None of them re-derives a value by calling the
same oracle routine twice: expected values come from closed forms, invariants,
special cases, independent brute force, or numbers printed in the paper.
"""
import math

import numpy as np
import pytest

from oracle import avs_oracle as O
from workloads import fields as F
from workloads import meshes as MM


def fine_mesh(D, n, half):
    t = O.base_forest(D, [-half] * D, [half] * D, [n] * D, 0)
    return t.centres(), t.weights()


# ---------------------------------------------------------------- P1 ------
@pytest.mark.parametrize("D,n", [(2, 160), (3, 56)])
def test_maxwell_and_shakhov_moments_closed_form(D, n):
    """Continuous moments of the Maxwellian (rho, rho U, rho|U|^2/2 + 3/2 rho R T,
    zero heat flux) and of the Shakhov equilibrium (same W, heat flux (1-Pr) q),
    Eqs. Maxwell_df, equ14-equ17; reached to round-off by the mid-point rule on
    a fine mesh because the integrands are smooth and decay like Gaussians."""
    R = 0.5
    rho, U, T = 1.3, np.array([0.4, -0.3, 0.2][:D]), 1.1
    xi, A = fine_mesh(D, n, 9.0)
    gas = O.Gas(R=R, Pr=2.0 / 3.0, omega=0.81, mu_ref=1.0, T_ref=1.0, model=1)
    W_exact = np.concatenate([[rho], rho * U, [0.5 * rho * U @ U + 1.5 * rho * R * T]])
    geq = O.eq_pair(rho, U, T, xi, R)
    np.testing.assert_allclose(O.moments(geq, xi, A), W_exact, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(O.heat_flux(geq, xi, A, U), 0.0, atol=1e-12)
    q = np.array([0.05, -0.08, 0.03][:D])
    sh = O.shakhov(rho, U, T, q, xi, gas)
    np.testing.assert_allclose(O.moments(sh, xi, A), W_exact, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(O.heat_flux(sh, xi, A, U), (1 - gas.Pr) * q, rtol=1e-10, atol=1e-12)
    gas.model = 0
    np.testing.assert_allclose(O.heat_flux(O.shakhov(rho, U, T, q, xi, gas), xi, A, U), 0.0, atol=1e-12)


def test_reduced_H_carries_the_missing_translational_energy():
    """In 2-D, H integrates to rho R T (one hidden translational dof, Eq. equ16
    with K=0); in 3-D there is no H and 1/2 int |c|^2 G = 3/2 rho R T."""
    R, rho, T = 1.0, 0.7, 1.9
    xi, A = fine_mesh(2, 160, 12.0)
    e = O.eq_pair(rho, np.zeros(2), T, xi, R)
    assert abs(np.sum(A * e[1]) - rho * R * T) < 1e-12
    xi3, A3 = fine_mesh(3, 64, 12.0)
    g = O.eq_pair(rho, np.zeros(3), T, xi3, R)[0]
    assert abs(0.5 * np.sum(A3 * np.sum(xi3 * xi3, 1) * g) - 1.5 * rho * R * T) < 1e-11


# -------------------------------------------------------- closure ---------
@pytest.mark.parametrize("D", [2, 3])
def test_closure_hits_target_and_stays_in_equilibrium_span(D):
    """C(phi, W*) has moments W* to round-off, and the correction it adds is
    (a + b.c + e|c|^2) g_eq(W*): dividing by g_eq leaves a quadratic in c."""
    R = 1.0
    t = O.base_forest(D, [-6] * D, [6] * D, [12] * D, 0)
    xi, A = t.centres(), t.weights()
    rng = np.random.default_rng(3)
    U = np.array([0.3, -0.2, 0.1][:D])
    ph = O.eq_pair(1.0, U, 1.0, xi, R) * (1 + 0.05 * rng.standard_normal((2 if D == 2 else 1, t.n)))
    Wstar = O.conserved(np.concatenate([[1.02], U + 0.01, [0.97]]), R)
    out = O.closure(ph, Wstar, xi, A, R)
    np.testing.assert_allclose(O.moments(out, xi, A), Wstar, rtol=1e-13, atol=1e-14)
    r, Us, Ts = O.primitive(Wstar, R)
    g = O.maxwell(r, Us, Ts, xi, R)
    ratio = (out[0] - ph[0]) / g
    c = xi - Us
    Bm = np.column_stack([np.ones(t.n)] + [c[:, d] for d in range(D)] + [np.sum(c * c, 1)])
    coef, *_ = np.linalg.lstsq(Bm, ratio, rcond=None)
    assert np.max(np.abs(Bm @ coef - ratio)) < 1e-8 * np.max(np.abs(ratio))


# ------------------------------------------------------------ tau, Kn ----
def test_hard_sphere_mean_free_path_and_Kn_Ma_Re():
    """Eq. equ4 at omega = 1/2 is the textbook hard-sphere mean free path
    lambda = 16 mu / (5 rho sqrt(2 pi R T)); Eq. equ5's Ma/Re form agrees."""
    R, T, rho = 1.0, 1.0, 1.0
    mu = O.mu_ref_from_kn(0.075, 0.5, R, T, rho, 1.0)
    assert abs(16 * mu / (5 * rho * math.sqrt(2 * math.pi * R * T)) - 0.075) < 1e-15
    gamma, Ma, omega = 5 / 3, 5.0, 0.81
    mu = O.mu_ref_from_kn(0.1, omega, 0.5, 1.0, 1.0, 1.0)
    Re = rho * Ma * math.sqrt(gamma * 0.5 * 1.0) * 1.0 / mu
    kn = math.sqrt(gamma / math.pi) * math.sqrt(2) * (5 - 2 * omega) * (7 - 2 * omega) / 15 * Ma / Re
    assert abs(kn - 0.1) < 1e-14
    gas = O.Gas(R=0.5, Pr=2 / 3, omega=omega, mu_ref=mu, T_ref=1.0)
    # VHS: tau p / mu_ref = (T/T_ref)^omega
    assert abs(O.tau(2.0, 3.0, gas) * 2.0 * 0.5 * 3.0 / mu - 3.0 ** omega) < 1e-14


# --------------------------------------------------- gradient, limiter ---
def test_lsq_gradient_exact_for_linear_fields():
    """A least-squares gradient reproduces any linear field exactly, on the
    Cartesian box and on the distorted quads of the O-grid (interior cells)."""
    for desc in (MM.box2d(5, 4, periodic=(False, False), sides={'left': 0, 'right': 0, 'bottom': 0, 'top': 0},
                          bcs=[(0, (1, 0, 0, 1))]), MM.ogrid(6, 12)):
        mesh = O.Mesh(desc)
        a = np.array([0.7, -1.3])
        lin = desc['cell_ctr'] @ a
        for i in range(mesh.nc):
            g = sum(c * (lin[s.nbr] - lin[i]) for s, c in zip(mesh.slots[i], mesh.lsq[i]) if s.nbr >= 0)
            np.testing.assert_allclose(g, a, rtol=1e-10, atol=1e-10)


def strip(values, K):
    """A periodic row of cells (unit spacing) carrying ``values`` at one node."""
    n = len(values)
    desc = MM.box2d(n, 1, lx=float(n), ly=1.0, periodic=(True, True))
    mesh = O.Mesh(desc)
    phi = np.asarray(values, np.float64).reshape(1, n, 1)
    return mesh, phi


def test_venkatakrishnan_properties():
    """Limiter properties:
    * a linear profile is not limited (psi = 1 on both faces) for any eps;
    * a smooth extremum has zero gradient, so nothing is reconstructed;
    * (eps = 0) when the slope would overshoot a neighbour by far, the limited
      increment tends to the distance to that neighbour (L * D2 -> D1), and it
      never exceeds it, also for VDF values near the bottom of the FP64 range."""
    box = O.Mesh(MM.box2d(4, 4, sides={'left': 0, 'right': 0, 'bottom': 0, 'top': 0}, bcs=[(0, (1, 0, 0, 1))]))
    lin = (box.ctr @ np.array([0.3, 0.7])).reshape(1, -1, 1)
    for K in (0.0, 0.7, 2.0):          # linear data is never limited, whatever eps
        lg = O.limited_gradient(5, lin, box, K)
        np.testing.assert_allclose(lg[0, 0], [0.3, 0.7], rtol=1e-14)
    mesh, phi = strip([0.0, 1.0, 0.0], 0.0)
    assert np.all(O.limited_gradient(1, phi, mesh, 0.0) == 0.0)
    for delta in (1e-3, 1e-5):
        mesh, phi = strip([0.0, 1.0, 1.0 + delta, 1.0 + delta, 0.5], 0.0)
        lg = O.limited_gradient(1, phi, mesh, 0.0)
        inc = lg[0, 0, 0] * 0.5          # limited increment to the east face
        assert abs(inc / delta - 1.0) < 10 * delta ** 0.5
    for scale in (1.0, 1e-200, 1e-300):
        mesh, phi = strip([0.0, scale, 1.3 * scale, 0.2 * scale], 0.0)
        lg = O.limited_gradient(1, phi, mesh, 0.0)
        assert np.isfinite(lg).all() and 0.0 < lg[0, 0, 0] * 0.5 <= 0.3 * scale
    # eps -> infinity switches the limiter off (psi -> 1)
    mesh, phi = strip([0.0, 1.0, 1.2, 0.1], 1e6)
    lg = O.limited_gradient(1, phi, mesh, 1e6)
    assert abs(lg[0, 0, 0] - 0.6) < 1e-12


# --------------------------------------------------- P2, P3: remap -------
def small_tree(D, seed, splits=2):
    t = O.base_forest(D, [-4] * D, [4] * D, [4] * D, 3)
    rng = np.random.default_rng(seed)
    for _ in range(splits):
        eff = np.where((rng.random(t.n) < 0.3) & (t.level < t.max_level), 1, 0).astype(np.int8)
        t = O.make_plan(eff, t).tree
    return t


@pytest.mark.parametrize("D", [2, 3])
def test_split_conservation_closed_form(D):
    """Copying a parent into its 2^D children keeps mass and momentum exactly
    (children's centres average to the parent's) and adds energy
    A_p G_p D h_p^2 / 32 per split leaf (Sec. 3.2, P2)."""
    t = small_tree(D, 1)
    rng = np.random.default_rng(2)
    P = 2 if D == 2 else 1
    phi = rng.random((P, 3, t.n))
    eff = np.where(t.level < t.max_level, 1, 0).astype(np.int8)
    plan = O.make_plan(eff, t)
    new = O.remap(phi, plan, D)
    xi, A = t.centres(), t.weights()
    xn, An = plan.tree.centres(), plan.tree.weights()
    h = t.widths()[:, 0]
    for i in range(3):
        W0, W1 = O.moments(phi[:, i], xi, A), O.moments(new[:, i], xn, An)
        np.testing.assert_allclose(W1[:1 + D], W0[:1 + D], rtol=1e-14, atol=1e-15)
        gain = np.sum(np.where(eff == 1, A * phi[0, i] * D * h * h / 32.0, 0.0))
        assert abs((W1[1 + D] - W0[1 + D]) - gain) < 1e-13 * abs(W0[1 + D])


@pytest.mark.parametrize("D", [2, 3])
def test_merge_conservation_closed_form(D):
    """Averaging 2^D children into the parent keeps mass exactly and changes
    momentum by -(A_p/2^D) sum_c G_c (xi_c - xi_p) (Sec. 3.2, P2)."""
    t = O.base_forest(D, [-4] * D, [4] * D, [2] * D, 2)
    t = O.make_plan(np.ones(t.n, np.int8), t).tree
    rng = np.random.default_rng(5)
    P = 2 if D == 2 else 1
    phi = rng.random((P, 1, t.n))
    plan = O.make_plan(-np.ones(t.n, np.int8), t)
    new = O.remap(phi, plan, D)
    xi, A = t.centres(), t.weights()
    xn, An = plan.tree.centres(), plan.tree.weights()
    W0, W1 = O.moments(phi[:, 0], xi, A), O.moments(new[:, 0], xn, An)
    assert abs(W1[0] - W0[0]) < 1e-14 * W0[0]
    dmom = np.zeros(D)
    for j in range(plan.tree.n):
        k = plan.src[j]
        for c in range(2 ** D):
            dmom -= (An[j] / 2 ** D) * phi[0, 0, k + c] * (xi[k + c] - xn[j])
    np.testing.assert_allclose(W1[1:1 + D] - W0[1:1 + D], dmom, atol=1e-13)


@pytest.mark.parametrize("D", [2, 3])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_split_then_merge_is_bit_exact(D, dtype):
    """Split followed by merge of the unchanged children returns the parent
    bit for bit (pairwise sum of 2^D equal values times 2^-D, P3)."""
    t = small_tree(D, 7)
    rng = np.random.default_rng(8)
    P = 2 if D == 2 else 1
    phi = rng.standard_normal((P, 4, t.n)).astype(dtype) * dtype(1e3)
    eff = np.where(t.level < t.max_level, 1, 0).astype(np.int8)
    p1 = O.make_plan(eff, t)
    mid = O.remap(phi, p1, D).astype(dtype)
    back_eff = np.zeros(p1.tree.n, np.int8)
    back_eff[p1.kind == O.SPLIT] = -1
    p2 = O.make_plan(O.resolve_merges(back_eff, p1.tree), p1.tree)
    out = O.remap(mid, p2, D).astype(dtype)
    assert np.array_equal(p2.tree.level, t.level) and np.array_equal(p2.tree.idx, t.idx)
    assert np.array_equal(out.view(np.uint8), phi.view(np.uint8))


# ---------------------------------------------------------------- P4 -----
@pytest.mark.parametrize("D", [2, 3])
def test_criterion_terms_sum_to_one(D):
    """sum_k M1_ik = sum_k M2_ik = 1 when W_i = M[phi_i] (the M's are density
    and internal-energy fractions, Sec. 3.4), H included in M2."""
    t = small_tree(D, 11)
    R = 0.5
    xi, A = t.centres(), t.weights()
    rng = np.random.default_rng(12)
    for U, T in ((np.array([0.5, -1.0, 0.3][:D]), 2.0), (np.zeros(D), 0.8)):
        ph = O.eq_pair(1.0, U, T, xi, R) * (1 + 0.2 * rng.random((2 if D == 2 else 1, t.n)))
        W = O.moments(ph, xi, A)
        M1, M2 = O.criterion_terms(ph[0], ph[1] if D == 2 else 0.0, W, xi, A)
        assert abs(M1.sum() - 1) < 1e-13 and abs(M2.sum() - 1) < 1e-12


# ------------------------------------------------------ P11: tree rules ---
def brute_force_adapt(tree, raw):
    """Independent tree update on a set of (level, index-tuple) leaves."""
    D = tree.dim
    leaves = {(int(l), tuple(int(v) for v in ix)): int(r) for l, ix, r in zip(tree.level, tree.idx, raw)}
    out = set()
    parents = {}
    for (l, ix), r in leaves.items():
        if r == -1:
            parents.setdefault((l - 1, tuple(v // 2 for v in ix)), []).append((l, ix))
    merged = {p for p, ch in parents.items() if len(ch) == 2 ** D}
    for (l, ix), r in leaves.items():
        if r == 1:
            for c in range(2 ** D):
                out.add((l + 1, tuple(2 * ix[d] + ((c >> d) & 1) for d in range(D))))
        elif r == -1 and (l - 1, tuple(v // 2 for v in ix)) in merged:
            out.add((l - 1, tuple(v // 2 for v in ix)))
        else:
            out.add((l, ix))
    # depth-first order from the roots, children in x-fastest binary order
    order = []

    def visit(l, ix):
        if (l, ix) in out:
            order.append((l, ix))
            return
        for c in range(2 ** D):
            visit(l + 1, tuple(2 * ix[d] + ((c >> d) & 1) for d in range(D)))
    # the roots' own order (Z14: Morton order) without the oracle's key: the
    # base^D roots are the leaves of one virtual tree, log2(base) levels
    # above them, visited depth first with children in x-fastest binary order
    base = [int(b) for b in tree.base]
    top = max(base).bit_length() - 1
    assert all(1 << top >= b for b in base)

    def visit_virtual(l, ix):
        if any(v << -l >= base[d] for d, v in enumerate(ix)):
            return                               # wholly outside the root grid
        if l == 0:
            visit(0, ix)
            return
        for c in range(2 ** D):
            visit_virtual(l + 1, tuple(2 * ix[d] + ((c >> d) & 1) for d in range(D)))
    visit_virtual(-top, (0,) * D)
    return order


@pytest.mark.parametrize("D,seed", [(2, 0), (2, 1), (3, 2)])
def test_flags_and_plan_match_brute_force_tree(D, seed):
    t = small_tree(D, seed, splits=3)
    rng = np.random.default_rng(100 + seed)
    raw = rng.choice(np.array([-1, 0, 1], np.int8), t.n, p=[0.6, 0.25, 0.15])
    raw[(raw == 1) & (t.level == t.max_level)] = 0
    raw[(raw == -1) & (t.level == 0)] = 0
    eff = O.resolve_merges(raw, t)
    plan = O.make_plan(eff, t)
    expect = brute_force_adapt(t, raw)
    got = [(int(l), tuple(int(v) for v in ix)) for l, ix in zip(plan.tree.level, plan.tree.idx)]
    assert got == expect
    # plan consistency: every old leaf is accounted for exactly once
    cover = np.zeros(t.n, int)
    for j in range(plan.tree.n):
        k = plan.src[j]
        if plan.kind[j] == O.MERGE:
            cover[k:k + 2 ** D] += 1
        elif plan.kind[j] == O.COPY or plan.child[j] == 0:
            cover[k] += 1
    assert np.all(cover == 1)


@pytest.mark.parametrize("D,base", [(2, (4, 4)), (2, (8, 2)), (3, (2, 4, 2))])
def test_root_order_is_the_virtual_tree_depth_first_order(D, base):
    """The level-0 roots (Z12, Z14) come in the depth-first order of one
    virtual tree above them, children in x-fastest binary order; checked
    with base counts that differ per axis."""
    t = O.base_forest(D, [-1.0] * D, [1.0] * D, list(base), 2)
    got = [tuple(int(v) for v in ix) for ix in t.idx]
    expect = brute_force_adapt(t, np.zeros(t.n, np.int8))
    assert got == [ix for _, ix in expect]
    # 2-D base (4, 4): the first quadrant's four roots, then the second's
    if D == 2 and base == (4, 4):
        assert got[:8] == [(0, 0), (1, 0), (0, 1), (1, 1), (2, 0), (3, 0), (2, 1), (3, 1)]


# ------------------------------------------------------ stepping pins -----
def periodic_setup(nx=6, ny=5, base=8, level=1, model=1, mu=0.05, prim=None, seed=0, half=5.0):
    desc = MM.box2d(nx, ny, periodic=(True, True))
    vs = dict(dim=2, lo=(-half, -half), hi=(half, half), base=(base, base), max_level=level)
    gas = O.Gas(R=1.0, Pr=2 / 3, omega=0.5, mu_ref=mu, T_ref=1.0, model=model)
    if prim is None:
        prim = F.perturbed_uniform(desc['ncells'], 2, seed, amp=0.05, uamp=0.2)
    return O.Solver(desc, vs, gas, dt=0.004, venkat_K=1.0, prim0=prim)


def test_uniform_rest_maxwellian_is_invariant():
    """A uniform Maxwellian at rest stays put (P5): periodic box to round-off;
    closed diffuse-wall cavity whose walls are at rest at the gas temperature
    to quadrature accuracy (the walls re-emit the plain discrete Maxwellian,
    the interior holds its moment-closed version; on a +-8 sqrt(RT) box with
    h = 1/2 the two differ by ~1e-14)."""
    s = periodic_setup(prim=F.uniform(30, 1.0, (0.0, 0.0), 1.0))
    phi0 = s.phi.copy()
    s.step(3)
    assert np.max(np.abs(s.phi - phi0)) < 1e-14 * np.max(phi0)
    c = F.cavity(n=6, Ma=0.0, box=8.0, base=32, max_level=0)
    s = O.Solver(c['mesh'], c['vspace'], c['gas'], c['dt'], 1.0, c['prim0'])
    phi0 = s.phi.copy()
    s.step(3)
    assert np.max(np.abs(s.phi - phi0)) < 1e-12 * np.max(phi0)


def test_periodic_conservation_and_vdf_moments():
    """Periodic box: sum V W conserved to round-off (telescoping fluxes), and
    the VDF's moments equal the authoritative W after every step (P6)."""
    s = periodic_setup()
    s.tree = O.make_plan(np.where(np.arange(s.tree.n) % 3 == 0, 1, 0).astype(np.int8), s.tree).tree
    s.phi = s.initial_vdf(s.W)
    tot0 = s.totals()
    for _ in range(4):
        s.step(1)
        np.testing.assert_allclose(s.vdf_moments(), s.W, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(s.totals(), tot0, rtol=1e-13, atol=1e-13)


def test_cavity_conserves_mass():
    """Closed cavity with a moving lid: the diffuse walls carry no net mass, so
    total mass is conserved to round-off while momentum and energy change."""
    c = F.cavity(n=6, base=8, max_level=1)
    s = O.Solver(c['mesh'], c['vspace'], c['gas'], c['dt'], 1.0, c['prim0'])
    m0 = s.totals()[0]
    s.step(5)
    assert abs(s.totals()[0] - m0) < 1e-13 * m0
    np.testing.assert_allclose(s.vdf_moments(), s.W, rtol=1e-12, atol=1e-13)


def homogeneous(model, Pr=2 / 3):
    """Spatially uniform bimodal (non-equilibrium) VDF in a periodic box."""
    s = periodic_setup(nx=2, ny=2, base=48, level=0, model=model, mu=0.01, half=8.0)
    s.gas.Pr = Pr
    xi, A = s.tree.centres(), s.tree.weights()
    f = 0.6 * O.eq_pair(1.0, np.array([0.8, 0.0]), 0.7, xi, 1.0) + 0.4 * O.eq_pair(1.0, np.array([-0.9, 0.3]), 1.2, xi, 1.0)
    s.phi = np.repeat(f[:, None, :], s.mesh.nc, axis=1)
    s.W = np.repeat(O.moments(f, xi, A)[None, :], s.mesh.nc, axis=0)
    return s, xi, A


def test_homogeneous_bgk_relaxation_closed_form():
    """BGK (P7): with no gradients the update is (phi - g~) <- (phi - g~)/(1+dt/tau),
    so phi^n - g~ = (1 + dt/tau)^-n (phi^0 - g~) exactly."""
    s, xi, A = homogeneous(model=0)
    phi0 = s.phi[:, 0].copy()
    r, U, T = O.primitive(s.W[0], 1.0)
    gt = O.closure(O.eq_pair(r, U, T, xi, 1.0), s.W[0], xi, A, 1.0)
    fac = 1.0 + s.dt / O.tau(r, T, s.gas)
    s.step(6)
    np.testing.assert_allclose(s.phi[:, 0] - gt, (phi0 - gt) * fac ** -6, atol=1e-13)


def test_homogeneous_shakhov_heat_flux_decay():
    """Shakhov (P7): the heat flux decays per step by
    (1 + (1-Pr) dt/tau) / (1 + dt/tau), i.e. at rate Pr/tau (to quadrature accuracy)."""
    s, xi, A = homogeneous(model=1)
    r, U, T = O.primitive(s.W[0], 1.0)
    fac = s.dt / O.tau(r, T, s.gas)
    q0 = O.heat_flux(s.phi[:, 0], xi, A, U)
    s.step(1)
    q1 = O.heat_flux(s.phi[:, 0], xi, A, U)
    expect = (1 + (1 - s.gas.Pr) * fac) / (1 + fac)
    np.testing.assert_allclose(q1 / q0, expect, rtol=2e-5)


def test_free_transport_matches_fourier_symbol():
    """tau -> infinity (P8): each node is advected by the scheme
    phi_{i+1/2} = phi_i + (phi_{i+1} - phi_{i-1})(1 - nu)/4 (central LSQ slope,
    limiter off, reconstruction at x_f - xi h), whose amplification factor
    for a Fourier mode of wavenumber theta is
    G = 1 - nu[(1 - e^{-i theta}) + (1-nu)/4 (e^{i theta} - e^{-i theta} - 1 + e^{-2 i theta})]."""
    nx = 16
    desc = MM.box2d(nx, 1, lx=1.0, ly=1.0 / nx, periodic=(True, True))
    vs = dict(dim=2, lo=(-3, -3), hi=(3, 3), base=(6, 6), max_level=0)
    gas = O.Gas(R=1.0, Pr=2 / 3, omega=0.5, mu_ref=1e30, T_ref=1.0, model=1)
    s = O.Solver(desc, vs, gas, dt=0.01, venkat_K=1e6, prim0=F.uniform(nx, 1.0, (0.0, 0.0), 1.0))
    th = 2 * np.pi * 3 / nx
    x = np.arange(nx)
    prof = 1.0 + 0.1 * np.cos(th * x)
    s.phi = np.repeat(prof[None, :, None], s.tree.n, axis=2) * np.ones((2, 1, 1))
    s.W = s.vdf_moments()
    s.step(1)
    dx = 1.0 / nx
    for k in range(s.tree.n):
        v = s.tree.centres()[k, 0]
        nu = abs(v) * s.dt / dx
        b = (1 - nu) / 4
        G = 1 - nu * ((1 - np.exp(-1j * th)) + b * (np.exp(1j * th) - np.exp(-1j * th) - 1 + np.exp(-2j * th)))
        xs = x if v >= 0 else -x
        expect = 1.0 + 0.1 * np.real(G * np.exp(1j * th * xs))
        np.testing.assert_allclose(s.phi[0, :, k], expect, atol=1e-13)


def test_full_refinement_equals_uniform_fine_mesh():
    """C1 below every M_k, C2 = -inf refines every leaf to the maximum level (P9): the
    node set equals the uniform fine mesh (same points, weights and order), and
    a step from the same initial state is bit-identical."""
    s = periodic_setup(nx=4, ny=3, base=4, level=2)
    for _ in range(2):
        s.adapt(-1.0, -np.inf)
        s.remap(correction=2)
    fine = periodic_setup(nx=4, ny=3, base=16, level=0)
    assert np.array_equal(s.tree.centres(), fine.tree.centres())
    assert np.array_equal(s.tree.weights(), fine.tree.weights())
    s.phi = s.initial_vdf(s.W)
    s.step(2)
    fine.step(2)
    assert np.array_equal(s.phi, fine.phi) and np.array_equal(s.W, fine.W)


def test_remap_correction_restores_W():
    """After split/merge + literal correction + closure, M[f] = W to round-off
    (Sec. 3.3, P6); the literal correction alone leaves a small defect."""
    s = periodic_setup(base=8, level=2)
    s.step(2)
    eff, plan, Mk = s.adapt(0.002, math.exp(-8) * 0.002)
    assert (eff == 1).any()
    W = s.W.copy()
    s.remap(correction=2)
    np.testing.assert_allclose(s.vdf_moments(), W, rtol=1e-12, atol=1e-13)


def _moments_by_hand(phi, xi, A):
    """Sum A (G, xi G, (|xi|^2 G + H)/2) written out per leaf (Eq. updat_W)."""
    D = xi.shape[1]
    G = phi[0]
    H = phi[1] if D == 2 else np.zeros_like(G)
    out = [float(np.sum(A * G))]
    out += [float(np.sum(A * xi[:, d] * G)) for d in range(D)]
    out.append(float(np.sum(0.5 * A * (np.sum(xi * xi, axis=1) * G + H))))
    return np.array(out)


@pytest.mark.parametrize("D,n,half", [(2, 48, 12.0), (3, 28, 9.0)])
def test_literal_correction_conserves_exactly_where_the_quadrature_is_exact(D, n, half):
    """The literal correction of Sec. 3.3 alone (no closure): f = f' + g(W) -
    g(W') has moments W' + M[g(W)] - M[g(W')].  On a uniform mesh over a box
    of many thermal speeds the mid-point rule integrates a Maxwellian to
    round-off (its error decays like exp(-2 pi^2 sigma^2 / h^2)), so M[f] = W
    there for any f' and any W.  A flipped sign would give 2 W' - W, a
    dropped term W' or M[g(W)], a wrong H pairing a wrong energy."""
    R = 1.0
    t = O.base_forest(D, [-half] * D, [half] * D, [n] * D, 0)
    xi, A = t.centres(), t.weights()
    rng = np.random.default_rng(31 + D)
    Ub = np.array([0.3, -0.2, 0.1][:D])
    base = O.eq_pair(1.0, Ub, 1.0, xi, R)
    ncell = 3
    fp = np.stack([base * (1.0 + 0.2 * rng.random(base.shape)) for _ in range(ncell)], axis=1)
    Wp = np.array([_moments_by_hand(fp[:, i], xi, A) for i in range(ncell)])
    W = Wp * (1.0 + 0.01 * rng.uniform(-1, 1, Wp.shape))          # a different authoritative state
    W[:, 1 + D] = np.abs(W[:, 1 + D]) + 0.05                      # keep it hot enough to be physical
    out = O.correct(fp, W, t, R, close=False)
    for i in range(ncell):
        np.testing.assert_allclose(_moments_by_hand(out[:, i], xi, A), W[i], rtol=1e-11, atol=1e-12)
        assert np.max(np.abs(Wp[i] - W[i])) > 1e-4                 # the correction had work to do


def test_literal_correction_after_split_and_merge_on_a_fine_mesh():
    """The same through the remap of Sec. 3.2-3.3: a uniform fine mesh,
    every brother group merged (the new mesh is uniform too), literal
    correction without the closure: the moments return to W to round-off,
    while the consanguinity reconstruction alone moves them (momentum of a
    merge, P2)."""
    R = 1.0
    t = O.base_forest(2, [-12.0] * 2, [12.0] * 2, [48] * 2, 1)
    t = O.make_plan(np.ones(t.n, np.int8), t).tree                   # 96 x 96 uniform at level 1
    xi, A = t.centres(), t.weights()
    rng = np.random.default_rng(5)
    phi = O.eq_pair(1.1, np.array([0.4, 0.1]), 0.9, xi, R)[:, None, :] * (1 + 0.3 * rng.random((2, 2, t.n)))
    W = np.array([_moments_by_hand(phi[:, i], xi, A) for i in range(2)])
    plan = O.make_plan(-np.ones(t.n, np.int8), t)
    assert plan.tree.n * 4 == t.n
    fp = O.remap(phi, plan, 2)
    xn, An = plan.tree.centres(), plan.tree.weights()
    Wp = np.array([_moments_by_hand(fp[:, i], xn, An) for i in range(2)])
    assert np.max(np.abs(Wp - W)) > 1e-4
    out = O.correct(fp, W, plan.tree, R, close=False)
    for i in range(2):
        np.testing.assert_allclose(_moments_by_hand(out[:, i], xn, An), W[i], rtol=1e-11, atol=1e-12)


def test_criterion_is_the_max_over_cells_and_probes():
    """M_k runs over the whole physical mesh (text of Sec. 3.4): the
    criterion of a mesh is the leafwise maximum of the criteria of its cells
    taken one at a time, and a probe state counts as one more cell holding its
    discrete Maxwellian.  Two cells with Maxwellians far apart: at the leaf
    under each peak the criterion takes that cell's value, which exceeds the
    other cell's by orders of magnitude, and the peak value is A_k times the
    Maxwellian's peak density over rho, 1/(2 pi R T) (M1 with G at c = 0)."""
    R = 1.0
    t = O.base_forest(2, [-8.0] * 2, [8.0] * 2, [16, 16], 1)
    xi, A = t.centres(), t.weights()
    T = 0.25
    Ua, Ub = np.array([-4.5, 0.5]), np.array([4.5, 0.5])       # leaf centres: the peaks sit on leaves
    ea, eb = O.eq_pair(1.0, Ua, T, xi, R), O.eq_pair(2.0, Ub, T, xi, R)
    phi = np.stack([ea, eb], axis=1)
    pa, pb = np.array([1.0, Ua[0], Ua[1], T]), np.array([2.0, Ub[0], Ub[1], T])
    W = np.array([O.conserved(pa, R), O.conserved(pb, R)])     # exact states (the coarse mesh is not)
    both = O.criterion(phi, W, t, R)
    one_a = O.criterion(phi[:, :1], W[:1], t, R)
    one_b = O.criterion(phi[:, 1:], W[1:], t, R)
    assert np.array_equal(both, np.maximum(one_a, one_b))
    ka = int(np.argmin(np.sum((xi - Ua) ** 2, 1)))
    kb = int(np.argmin(np.sum((xi - Ub) ** 2, 1)))
    assert np.allclose(xi[ka], Ua) and np.allclose(xi[kb], Ub)
    assert both[ka] == one_a[ka] and both[kb] == one_b[kb]
    assert one_a[ka] > 1e6 * one_b[ka] and one_b[kb] > 1e6 * one_a[kb]
    for k, i in ((ka, 0), (kb, 1)):
        np.testing.assert_allclose(both[k], A[k] / (2 * math.pi * R * T), rtol=1e-14)
    # a probe holding cell b's state adds cell b's criterion to a one-cell mesh
    with_probe = O.criterion(phi[:, :1], W[:1], t, R, probes=pb)
    assert np.array_equal(with_probe, np.maximum(one_a, one_b))


def test_equilibrium_bypass():
    """End of Sec. 3.3: f = g_eq(W) on the new leaves.  Closed (mode 4) it
    has the moments W to round-off; literal (mode 3) it conserves to the
    quadrature error of the discrete Maxwellian only (here the truncation
    of the Gaussian tails at the box edge, +-5 thermal speeds); both
    discard the previous VDF entirely."""
    s = periodic_setup(base=8, level=2)
    s.step(2)
    s.adapt(0.002, math.exp(-8) * 0.002)
    W = s.W.copy()
    s.remap(correction=4)
    np.testing.assert_allclose(s.vdf_moments(), W, rtol=1e-12, atol=1e-13)
    defects = []
    for base in (4, 8, 16):
        t = periodic_setup(base=base, level=1)
        t.adapt(-1.0, -2.0)                     # split everything once
        Wt = t.W.copy()
        t.remap(correction=3)
        defects.append(np.max(np.abs(t.vdf_moments() - Wt)) / np.max(np.abs(Wt)))
    assert all(1e-9 < d < 1e-3 for d in defects)
    # the result depends on W alone: a different VDF with the same W gives the same f
    u = periodic_setup(base=8, level=1, seed=3)
    u.adapt(-1.0, -2.0)
    v = periodic_setup(base=8, level=1, seed=3)
    v.phi = v.phi * (1.0 + 0.01 * np.random.default_rng(1).standard_normal(v.phi.shape))
    v.adapt(-1.0, -2.0)
    u.remap(correction=3)
    v.remap(correction=3)
    assert np.array_equal(u.phi, v.phi)
