"""GPU implicit step (IUGKS, Sec. 2.3.1-2.3.2) through the C ABI against the
FP64 oracle on identical seeded inputs, with the same colour-major sweep
order on both sides: FP64 to 1e-12 per step, FP32 within 1e-5
field-normalised.  Time steps are several times the explicit stability
bound."""
import math

import numpy as np
import pytest

from oracle import avs_oracle as O
from workloads import fields as F
from workloads import meshes as MM

from test_gpu_parity import fieldrel, make_pair, random_tree, rel, resolved_tree

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def avs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_05645_amd import avs as mod
    return mod


def test_implicit_periodic(avs):
    """Periodic box (two colours), random tree, CFL about 4: the paper's
    sweep counts (60 macro, 2 micro) and a short run of both."""
    mesh = MM.box2d(6, 5, periodic=(True, True))
    vs = dict(dim=2, lo=(-6, -6), hi=(6, 6), base=(8, 8), max_level=2)
    gas = dict(R=1.0, Pr=2 / 3, omega=0.81, mu_ref=0.02, T_ref=1.0, model=1)
    prim = F.perturbed_uniform(mesh['ncells'], 2, 61, amp=0.1, uamp=0.4)
    dt = 4.0 * F._cfl_dt(mesh, 1.0, (6.0, 6.0))
    cs, o = make_pair(avs, mesh, vs, gas, dt, prim, tree=random_tree(vs, 62, 2), noise=0.02, seed=63)
    for _ in range(2):
        r = cs.step_implicit(1, 60, 2, residual=True)
        ro = o.step_implicit(1, 60, 2)
        v, W = cs.get_state()
        assert rel(v, o.phi) < 1e-12 and rel(W, o.W) < 1e-12
        assert rel(r, ro) < 1e-8
    _, tot = cs.moments(fields=False)
    assert np.all(np.isfinite(tot))


def test_implicit_cavity(avs):
    """Walls and a moving lid (boundary faces hold their increments at zero)."""
    c = F.cavity(n=8, base=8, max_level=2)
    t = random_tree(c['vspace'], 64, 2)
    cs, o = make_pair(avs, c['mesh'], c['vspace'], c['gas'], 5.0 * c['dt'], c['prim0'], tree=t, noise=0.02, seed=65)
    cs.step_implicit(2, 30, 3)
    o.step_implicit(2, 30, 3)
    v, W = cs.get_state()
    assert rel(v, o.phi) < 1e-12 and rel(W, o.W) < 1e-12


def test_implicit_ogrid_and_triangles(avs):
    """Far field and wall on the O-grid, then a triangle mesh whose greedy
    colouring needs more than two colours."""
    c = F.cylinder(nr=6, nth=16, Ma=2.0, box=8.0, base=16, max_level=2, r1=2.5, first=0.1)
    cs, o = make_pair(avs, c['mesh'], c['vspace'], c['gas'], 3.0 * c['dt'], c['prim0'], tree=resolved_tree(c['vspace'], 66),
                      noise=0.01, seed=67, Kv=c['venkat_K'])
    cs.step_implicit(2, 20, 2)
    o.step_implicit(2, 20, 2)
    v, W = cs.get_state()
    assert rel(v, o.phi) < 1e-12 and rel(W, o.W) < 1e-12
    U = 1.2 * math.sqrt(5.0 / 3.0)
    mesh = MM.tri_box(7, 6, 68, sides=dict(left=1, right=1, bottom=0, top=0),
                      bcs=[(MM.WALL, (1.0, 0.0, 0.0, 1.0)), (MM.FARFIELD, (1.0, U, 0.0, 1.0))])
    from oracle import avs_implicit as I
    assert I.cell_colours(O.Mesh(mesh)).max() >= 2
    vs = dict(dim=2, lo=(-6.0, -6.0), hi=(7.0, 6.0), base=(8, 8), max_level=2)
    gas = dict(R=1.0, Pr=2 / 3, omega=0.81, mu_ref=0.02, T_ref=1.0, model=1)
    prim = F.perturbed_uniform(mesh['ncells'], 2, 69, amp=0.1, uamp=0.4)
    dt = 3.0 * F._cfl_dt(mesh, 1.0, (7.0, 6.0))
    cs, o = make_pair(avs, mesh, vs, gas, dt, prim, tree=random_tree(vs, 70, 2), noise=0.01, seed=71, Kv=0.0)
    cs.step_implicit(2, 20, 2)
    o.step_implicit(2, 20, 2)
    v, W = cs.get_state()
    assert rel(v, o.phi) < 1e-12 and rel(W, o.W) < 1e-12


def test_implicit_3d(avs):
    mesh = MM.box3d(3, 3, 2, periodic=(True, True, True))
    vs = dict(dim=3, lo=(-5.0,) * 3, hi=(5.0,) * 3, base=(4, 4, 4), max_level=2)
    gas = dict(R=1.0, Pr=2 / 3, omega=0.5, mu_ref=0.05, T_ref=1.0, model=1)
    prim = F.perturbed_uniform(mesh['ncells'], 3, 72, amp=0.1, uamp=0.4)
    dt = 3.0 * F._cfl_dt(mesh, 1.0, (5.0, 5.0, 5.0))
    cs, o = make_pair(avs, mesh, vs, gas, dt, prim, tree=random_tree(vs, 73, 2), noise=0.01, seed=74)
    cs.step_implicit(1, 20, 2)
    o.step_implicit(1, 20, 2)
    v, W = cs.get_state()
    assert rel(v, o.phi) < 1e-12 and rel(W, o.W) < 1e-12


def test_implicit_fp32_form(avs):
    c = F.cavity(n=8, base=8, max_level=2)
    t = random_tree(c['vspace'], 75, 2)
    cs, o = make_pair(avs, c['mesh'], c['vspace'], c['gas'], 5.0 * c['dt'], c['prim0'], tree=t, noise=0.02, seed=76,
                      precision=1)
    cs.step_implicit(3, 30, 2)
    o.step_implicit(3, 30, 2)
    f, _ = cs.moments(fields=True, totals=False)
    assert fieldrel(cs.get_W(), o.W) < 1e-5


def test_implicit_arguments(avs):
    c = F.cavity(n=4, base=8, max_level=1)
    cs = avs.Case(c['mesh'], c['vspace'], c['gas'], c['dt'], 1.0, c['prim0'])
    with pytest.raises(avs.AvsError):
        cs.step_implicit(1, -1, 2)
    import ctypes as C
    small = cs._torch.empty(256, dtype=cs._torch.uint8, device=cs.device)
    assert avs.lib.avs_step_implicit(cs.ctx, 1, 2, 2, small.data_ptr(), 256, None) == avs.AVS_E_INVALID
    cs.step_implicit(1, 2, 2)
    cs.close()


def test_implicit_steady_state_is_the_explicit_one(avs):
    """At a steady state phi^{n+1} = phi^n and W^{n+1} = W^n the implicit
    equations (Eqs. SGS_w, SGS_phi with zero increments) reduce to the
    explicit ones with the same interface half step.  A small cavity run to
    steady state explicitly at the stability bound (h = dt/2 = the cap) and
    implicitly at 50 times that step reaches the same fields."""
    c = F.cavity(n=12, Kn=0.02, base=8, max_level=1, cfl=1.0)
    cs = avs.Case(c['mesh'], c['vspace'], c['gas'], c['dt'], 1.0, c['prim0'])
    ci = avs.Case(c['mesh'], c['vspace'], c['gas'], 50.0 * c['dt'], 1.0, c['prim0'])
    for k in (cs, ci):
        k.adapt(-1.0, -2.0)
        k.remap(2)
    r0 = None
    for it in range(200):
        r = cs.step(500, residual=True)
        r0 = r0 if r0 is not None else np.max(r)
        if np.max(r) < 1e-9 * r0:
            break
    assert np.max(r) < 1e-9 * r0, (it, np.max(r) / r0)
    for it in range(100):
        ri = ci.step_implicit(20, 30, 4, residual=True)
        if np.max(ri) < 1e-9 * r0:
            break
    assert np.max(ri) < 1e-9 * r0, (it, np.max(ri) / r0)
    We, Wi = cs.get_W(), ci.get_W()
    assert fieldrel(Wi, We) < 1e-6
    cs.close()
    ci.close()


def test_implicit_with_adaptation_sutherland_and_bypass(avs):
    """Implicit steps interleaved with the adaptation of Sec. 3: flags
    bit exact, closed remap, then the equilibrium bypass, on an O-grid gas
    with Sutherland's viscosity; FP64 to 1e-12 throughout."""
    c = F.cylinder(nr=6, nth=16, Ma=2.0, box=8.0, base=16, max_level=2, r1=2.5, first=0.1)
    gas = dict(c['gas'], law=1, C_s=2.5)
    cs, o = make_pair(avs, c['mesh'], c['vspace'], gas, 4.0 * c['dt'], c['prim0'], tree=resolved_tree(c['vspace'], 80),
                      noise=0.01, seed=81, Kv=c['venkat_K'])
    cs.step_implicit(2, 20, 2)
    o.step_implicit(2, 20, 2)
    flags, nn = cs.adapt(2e-3, 1e-5)
    eff, plan, _ = o.adapt(2e-3, 1e-5)
    assert np.array_equal(flags, eff) and nn == plan.tree.n
    assert (eff == 1).any() or (eff == -1).any()
    cs.remap(2)
    o.remap(2)
    cs.step_implicit(1, 20, 2)
    o.step_implicit(1, 20, 2)
    v, W = cs.get_state()
    assert rel(v, o.phi) < 1e-12 and rel(W, o.W) < 1e-12
    cs.adapt(2e-3, 1e-5)
    o.adapt(2e-3, 1e-5)
    cs.remap(4)
    o.remap(4)
    cs.step_implicit(1, 20, 2)
    o.step_implicit(1, 20, 2)
    v, W = cs.get_state()
    assert rel(v, o.phi) < 1e-12 and rel(W, o.W) < 1e-12


def test_single_cell_periodic_mesh(avs):
    """Degenerate mesh: one cell whose two faces both join it to itself
    (periodic in x and y).  Explicit and implicit steps against the oracle;
    W cannot change."""
    mesh = MM.box2d(1, 1, periodic=(True, True))
    vs = dict(dim=2, lo=(-5, -5), hi=(5, 5), base=(8, 8), max_level=2)
    gas = dict(R=1.0, Pr=2 / 3, omega=0.81, mu_ref=0.05, T_ref=1.0, model=1)
    prim = F.perturbed_uniform(1, 2, 3, amp=0.1, uamp=0.3)
    for implicit in (False, True):
        cs, o = make_pair(avs, mesh, vs, gas, 0.01, prim, tree=random_tree(vs, 4, 2), noise=0.02, seed=5)
        W0 = o.W.copy()
        if implicit:
            cs.step_implicit(2, 10, 2)
            o.step_implicit(2, 10, 2)
        else:
            cs.step(2)
            o.step(2)
        v, W = cs.get_state()
        assert rel(v, o.phi) < 1e-12
        np.testing.assert_allclose(W, W0, rtol=1e-14, atol=1e-15)
        cs.close()


def test_zero_sweeps_reduce_to_the_explicit_macro_update(avs):
    """With no predictor sweep the increment is zero, the implicit flux is
    F^n and W^{n+1} is the explicit finite-volume update, bit for bit; with
    no micro sweep phi is unchanged."""
    c = F.cavity(n=8, base=8, max_level=2)
    t = random_tree(c['vspace'], 90, 2)
    a, _ = make_pair(avs, c['mesh'], c['vspace'], c['gas'], c['dt'], c['prim0'], tree=t, noise=0.02, seed=91)
    b, _ = make_pair(avs, c['mesh'], c['vspace'], c['gas'], c['dt'], c['prim0'], tree=t, noise=0.02, seed=91)
    v0, _ = a.get_state()
    a.step(1)
    b.step_implicit(1, 0, 0)
    assert np.array_equal(a.get_W(), b.get_W())
    vb, _ = b.get_state()
    assert np.array_equal(vb, v0)


@pytest.mark.parametrize("D,prec", [(2, 0), (3, 0), (2, 1)])
def test_rykov_equilibrium_matches_oracle(avs, D, prec):
    """Rykov equilibrium (G, H, R) of the diatomic model on a random tree
    of several hundred leaves (ragged row), for seeded states with unequal
    translational and rotational temperatures and both heat fluxes: FP64 to
    1e-12 of each component's scale, FP32 to 1e-6."""
    from oracle import avs_rykov as RY
    if D == 2:
        mesh = MM.box2d(3, 2, periodic=(True, True))
        vs = dict(dim=2, lo=(-6, -5), hi=(7, 6), base=(8, 8), max_level=2)
    else:
        mesh = MM.box3d(2, 2, 1, periodic=(True, True, True))
        vs = dict(dim=3, lo=(-5.0,) * 3, hi=(5.0,) * 3, base=(4, 4, 4), max_level=2)
    gas = dict(R=0.5, Pr=2 / 3, omega=0.74, mu_ref=0.05, T_ref=1.0, model=1)
    prim = F.perturbed_uniform(mesh['ncells'], D, 95, amp=0.1, uamp=0.3)
    t = random_tree(vs, 96, 2)
    cs = avs.Case(mesh, vs, gas, 1e-3, 1.0, prim, precision=prec)
    cs.set_leaves(t.level, t.idx)
    rng = np.random.default_rng(97)
    n = 37
    states = np.concatenate([rng.uniform(0.5, 2.0, (n, 1)), rng.uniform(-1.0, 1.0, (n, D)),
                             rng.uniform(0.6, 2.5, (n, 2)), 0.1 * rng.standard_normal((n, 2 * D))], axis=1)
    out = cs.rykov_equilibrium(states, Z_rot=3.5).cpu().numpy()[:, :, :t.n]
    g = RY.RykovGas(R=0.5, Z_rot=3.5)
    xi = t.centres()
    tol = 1e-12 if prec == 0 else 1e-6
    for i in range(n):
        s = states[i]
        ref = RY.rykov_equilibrium(s[0], s[1:1 + D], s[1 + D], s[2 + D], s[3 + D:3 + 2 * D], s[3 + 2 * D:], xi, g)
        for p in range(3):
            scale = max(np.abs(ref[p]).max(), 1e-300)
            assert np.abs(out[p, i] - ref[p]).max() <= tol * scale, (i, p)
    with pytest.raises(avs.AvsError):
        cs.rykov_equilibrium(states, Z_rot=0.5)
    cs.close()


def dia_pair(avs, mesh, vs, vgas, dt, prim5, tree, Kv=1.0, Z=3.5, max_leaves=None):
    from oracle import avs_rykov as RY
    D = vs['dim']
    cs = avs.Case(mesh, vs, vgas, dt, Kv, np.ascontiguousarray(prim5[:, :D + 2]))
    cs.set_leaves(tree.level, tree.idx)
    dia = avs.Diatomic(cs, prim5, Z_rot=Z, max_leaves=max_leaves)
    o = RY.DiatomicSolver(mesh, tree, vgas, RY.RykovGas(R=vgas['R'], Z_rot=Z), dt, Kv, prim5)
    return cs, dia, o


def test_diatomic_periodic_against_oracle(avs):
    """Rykov diatomic steps (2-D FP64) on a periodic box with a random tree
    and unequal translational and rotational temperatures: the closed
    initial state and three steps equal the oracle's to 1e-12; mass,
    momentum and total energy are kept."""
    mesh = MM.box2d(5, 4, periodic=(True, True))
    vs = dict(dim=2, lo=(-6.0, -6.0), hi=(6.0, 6.0), base=(8, 8), max_level=2)
    vgas = dict(R=0.5, Pr=0.72, omega=0.74, mu_ref=0.05, T_ref=1.0, model=1)
    rng = np.random.default_rng(101)
    n = mesh['ncells']
    prim = np.concatenate([1 + 0.1 * rng.uniform(-1, 1, (n, 1)), 0.3 * rng.uniform(-1, 1, (n, 2)),
                           1 + 0.1 * rng.uniform(-1, 1, (n, 1)), 0.8 + 0.1 * rng.uniform(-1, 1, (n, 1))], axis=1)
    cs, dia, o = dia_pair(avs, mesh, vs, vgas, 2e-3, prim, random_tree(vs, 102, 2))
    v, W = dia.get_state()
    assert rel(v, o.phi) < 1e-12 and rel(W, o.W) < 1e-13
    tot0 = np.sum(o.mesh.vol[:, None] * W, axis=0)
    for _ in range(3):
        dia.step(1)
        o.step(1)
        v, W = dia.get_state()
        assert rel(v, o.phi) < 1e-12 and rel(W, o.W) < 1e-12
    tot = np.sum(o.mesh.vol[:, None] * W, axis=0)
    np.testing.assert_allclose(tot[:4], tot0[:4], rtol=1e-13, atol=1e-14)
    dia.close()
    cs.close()


def test_diatomic_3d_walls_and_adaptation(avs):
    """The 3-D diatomic path (H identically zero) on a box with isothermal
    walls in y and periodic x and z: the closed initial state, a step,
    bit-exact flags of an adaptation with splits and merges, the remapped
    state, and a step on the new leaves against the oracle; mass is kept."""
    mesh = MM.box3d(3, 3, 2, periodic=(True, False, True))
    vs = dict(dim=3, lo=(-5.0,) * 3, hi=(5.0,) * 3, base=(4, 4, 4), max_level=2)
    vgas = dict(R=0.5, Pr=0.72, omega=0.74, mu_ref=0.05, T_ref=1.0, model=1)
    rng = np.random.default_rng(121)
    n = mesh['ncells']
    prim = np.concatenate([1 + 0.1 * rng.uniform(-1, 1, (n, 1)), 0.3 * rng.uniform(-1, 1, (n, 3)),
                           1 + 0.2 * rng.uniform(-1, 1, (n, 1)), 0.7 + 0.1 * rng.uniform(-1, 1, (n, 1))], axis=1)
    from oracle import avs_rykov as RY
    cs, dia, o = dia_pair(avs, mesh, vs, vgas, 2e-3, prim, random_tree(vs, 122, 2), max_leaves=2048)
    v, W = dia.get_state()
    assert W.shape == (n, 6) and not v[1].any()
    assert rel(v, o.phi) < 1e-12 and rel(W, o.W) < 1e-13
    m0 = np.sum(o.mesh.vol * W[:, 0])
    dia.step(1)
    o.step(1)
    v, W = dia.get_state()
    assert rel(v, o.phi) < 1e-12 and rel(W, o.W) < 1e-12
    Mk = np.sort(RY.criterion_dia(o.phi, o.W, o.tree))
    j1, j2 = int(0.85 * len(Mk)), int(0.25 * len(Mk))
    C1, C2 = 0.5 * (Mk[j1] + Mk[j1 + 1]), 0.5 * (Mk[j2] + Mk[j2 + 1])
    assert Mk[j1 + 1] - Mk[j1] > 1e-9 * Mk[j1] and Mk[j2 + 1] - Mk[j2] > 1e-9 * Mk[j2]
    flags, nn = dia.adapt(C1, C2)
    eff, plan, _ = o.adapt(C1, C2)
    assert np.array_equal(flags, eff) and nn == plan.tree.n
    assert (eff == 1).any() and (eff == -1).any()
    dia.remap()
    o.remap()
    v, W = dia.get_state()
    assert rel(v, o.phi) < 1e-12 and rel(W, o.W) < 1e-13
    dia.step(1)
    o.step(1)
    v, W = dia.get_state()
    assert rel(v, o.phi) < 1e-12 and rel(W, o.W) < 1e-12
    assert abs(np.sum(o.mesh.vol * W[:, 0]) - m0) < 1e-13 * m0
    dia.close()
    cs.close()


def test_diatomic_ogrid_wall_and_farfield(avs):
    """Nitrogen-like gas past a cylinder (O-grid with an isothermal wall and
    a far field, Ma 2): two steps against the oracle to 1e-12; the context's
    leaves may not change under the diatomic state."""
    c = F.cylinder(nr=5, nth=14, Ma=2.0, box=8.0, base=8, max_level=2, r1=2.5, first=0.1)
    vgas = dict(c['gas'], Pr=0.72, omega=0.74)
    p = c['prim0']
    prim = np.concatenate([p[:, :3], p[:, 3:4], 0.9 * p[:, 3:4]], axis=1)
    cs, dia, o = dia_pair(avs, c['mesh'], c['vspace'], vgas, c['dt'], prim, resolved_tree(c['vspace'], 103), Kv=0.0)
    dia.step(2)
    o.step(2)
    v, W = dia.get_state()
    assert rel(v, o.phi) < 1e-12 and rel(W, o.W) < 1e-12
    cs.adapt(1e-3, 1e-5)
    cs.remap(2)
    with pytest.raises(avs.AvsError):
        dia.step(1)
    dia.close()
    cs.close()


def test_diatomic_adaptation_against_oracle(avs):
    """Adaptation driven by the diatomic state: flags bit exact against the
    oracle's criterion (splits and merges), the remapped and closed state to
    1e-12 with moments equal to W, then a step on the new leaves; the
    context follows the new leaves."""
    mesh = MM.box2d(5, 4, periodic=(True, True))
    vs = dict(dim=2, lo=(-6.0, -6.0), hi=(6.0, 6.0), base=(8, 8), max_level=2)
    vgas = dict(R=0.5, Pr=0.72, omega=0.74, mu_ref=0.05, T_ref=1.0, model=1)
    rng = np.random.default_rng(111)
    n = mesh['ncells']
    prim = np.concatenate([1 + 0.1 * rng.uniform(-1, 1, (n, 1)), 0.4 * rng.uniform(-1, 1, (n, 2)),
                           1 + 0.2 * rng.uniform(-1, 1, (n, 1)), 0.7 + 0.1 * rng.uniform(-1, 1, (n, 1))], axis=1)
    from oracle import avs_rykov as RY
    tree = random_tree(vs, 112, 2)
    prim4 = np.concatenate([prim[:, :3], prim[:, 3:4]], axis=1)
    cs = avs.Case(mesh, vs, vgas, 2e-3, 1.0, prim4)
    cs.set_leaves(tree.level, tree.idx)
    dia = avs.Diatomic(cs, prim, max_leaves=1024)
    o = RY.DiatomicSolver(mesh, tree, vgas, RY.RykovGas(R=0.5, Z_rot=3.5), 2e-3, 1.0, prim)
    dia.step(1)
    o.step(1)
    # thresholds halfway between neighbouring values of M_k, so that the
    # decisions do not hang on the rounding differences of the two sides
    Mk = np.sort(RY.criterion_dia(o.phi, o.W, o.tree))
    j1, j2 = int(0.85 * len(Mk)), int(0.25 * len(Mk))
    C1, C2 = 0.5 * (Mk[j1] + Mk[j1 + 1]), 0.5 * (Mk[j2] + Mk[j2 + 1])
    assert Mk[j1 + 1] - Mk[j1] > 1e-9 * Mk[j1] and Mk[j2 + 1] - Mk[j2] > 1e-9 * Mk[j2]
    flags, nn = dia.adapt(C1, C2)
    eff, plan, _ = o.adapt(C1, C2)
    assert np.array_equal(flags, eff) and nn == plan.tree.n
    assert (eff == 1).any() and (eff == -1).any()
    dia.remap()
    o.remap()
    assert cs.nleaves() == o.tree.n
    v, W = dia.get_state()
    assert rel(v, o.phi) < 1e-12 and rel(W, o.W) < 1e-13
    np.testing.assert_allclose(o.vdf_moments(), W, rtol=0, atol=1e-13)
    dia.step(1)
    o.step(1)
    v, W = dia.get_state()
    assert rel(v, o.phi) < 1e-12 and rel(W, o.W) < 1e-12
    dia.close()
    cs.close()


def test_diatomic_implicit_periodic_against_oracle(avs):
    """Implicit diatomic steps (predictor with the rotational row, micro
    sweeps over G, H, R) on a periodic box at a step 20x the explicit one:
    three steps with 4/2 sweeps and one with no sweeps against the oracle
    to 1e-11; mass, momentum and total energy kept."""
    from oracle import avs_rykov as RY
    mesh = MM.box2d(5, 4, periodic=(True, True))
    vs = dict(dim=2, lo=(-6.0, -6.0), hi=(6.0, 6.0), base=(8, 8), max_level=2)
    vgas = dict(R=0.5, Pr=0.72, omega=0.74, mu_ref=0.05, T_ref=1.0, model=1)
    rng = np.random.default_rng(131)
    n = mesh['ncells']
    prim = np.concatenate([1 + 0.1 * rng.uniform(-1, 1, (n, 1)), 0.3 * rng.uniform(-1, 1, (n, 2)),
                           1 + 0.1 * rng.uniform(-1, 1, (n, 1)), 0.8 + 0.1 * rng.uniform(-1, 1, (n, 1))], axis=1)
    cs, dia, o = dia_pair(avs, mesh, vs, vgas, 0.04, prim, random_tree(vs, 132, 2))
    tot0 = o.totals()
    for sweeps in [(4, 2), (4, 2), (4, 2), (0, 0)]:
        dia.step_implicit(1, *sweeps)
        o.step_implicit(1, *sweeps)
        v, W = dia.get_state()
        assert rel(v, o.phi) < 1e-11 and rel(W, o.W) < 1e-11, sweeps
    tot = o.totals()
    np.testing.assert_allclose(tot[:4], tot0[:4], rtol=1e-13, atol=1e-13)
    dia.close()
    cs.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_diatomic_implicit_walls_against_oracle(avs, dim):
    """Implicit diatomic steps with boundaries: an O-grid with an isothermal
    wall and a Ma 2 far field (2-D), a box with walls in y (3-D); two steps
    against the oracle to 1e-11."""
    from oracle import avs_rykov as RY
    if dim == 2:
        c = F.cylinder(nr=5, nth=14, Ma=2.0, box=8.0, base=8, max_level=2, r1=2.5, first=0.1)
        vgas = dict(c['gas'], Pr=0.72, omega=0.74)
        p = c['prim0']
        prim = np.concatenate([p[:, :3], p[:, 3:4], 0.9 * p[:, 3:4]], axis=1)
        cs, dia, o = dia_pair(avs, c['mesh'], c['vspace'], vgas, 4 * c['dt'], prim, resolved_tree(c['vspace'], 133),
                              Kv=0.0)
    else:
        mesh = MM.box3d(3, 3, 2, periodic=(True, False, True))
        vs = dict(dim=3, lo=(-5.0,) * 3, hi=(5.0,) * 3, base=(4, 4, 4), max_level=2)
        vgas = dict(R=0.5, Pr=0.72, omega=0.74, mu_ref=0.05, T_ref=1.0, model=1)
        rng = np.random.default_rng(134)
        n = mesh['ncells']
        prim = np.concatenate([1 + 0.1 * rng.uniform(-1, 1, (n, 1)), 0.3 * rng.uniform(-1, 1, (n, 3)),
                               1 + 0.2 * rng.uniform(-1, 1, (n, 1)), 0.7 + 0.1 * rng.uniform(-1, 1, (n, 1))], axis=1)
        cs, dia, o = dia_pair(avs, mesh, vs, vgas, 0.02, prim, random_tree(vs, 135, 2))
    for _ in range(2):
        dia.step_implicit(1, 3, 2)
        o.step_implicit(1, 3, 2)
        v, W = dia.get_state()
        assert rel(v, o.phi) < 1e-11 and rel(W, o.W) < 1e-11
    with pytest.raises(avs.AvsError):
        dia.step_implicit(1, -1, 2)
    dia.close()
    cs.close()


def test_diatomic_sphere_explicit_and_implicit(avs):
    """The paper's sphere case with the Rykov gas, small: a spherical grid
    with an isothermal wall and a Ma 2 far field in 3-D, T_r = 0.9 T_t;
    two explicit steps, then one implicit step with 3/2 sweeps, against
    the oracle to 1e-11."""
    c = F.sphere(nr=3, nth=4, nph=4, Ma=2.0, box=5.0, base=8, max_level=1, r1=1.5, first=0.2)
    vgas = dict(c['gas'], Pr=0.72, omega=0.74)
    p = c['prim0']
    prim = np.concatenate([p[:, :4], p[:, 4:5], 0.9 * p[:, 4:5]], axis=1)
    cs, dia, o = dia_pair(avs, c['mesh'], c['vspace'], vgas, c['dt'], prim, resolved_tree(c['vspace'], 136), Kv=0.0)
    dia.step(2)
    o.step(2)
    v, W = dia.get_state()
    assert W.shape[1] == 6 and rel(v, o.phi) < 1e-11 and rel(W, o.W) < 1e-11
    dia.step_implicit(1, 3, 2)
    o.step_implicit(1, 3, 2)
    v, W = dia.get_state()
    assert rel(v, o.phi) < 1e-11 and rel(W, o.W) < 1e-11
    dia.close()
    cs.close()


def test_diatomic_adaptation_with_probe_states(avs):
    """Probe states in the diatomic criterion: a fast, hot equilibrium
    probe outside the cells' states adds splits where no cell needs them;
    flags bit exact against the oracle (thresholds between neighbouring
    M_k), and different from the flags without the probe."""
    from oracle import avs_rykov as RY
    mesh = MM.box2d(4, 3, periodic=(True, True))
    vs = dict(dim=2, lo=(-8.0, -8.0), hi=(8.0, 8.0), base=(8, 8), max_level=2)
    vgas = dict(R=0.5, Pr=0.72, omega=0.74, mu_ref=0.05, T_ref=1.0, model=1)
    rng = np.random.default_rng(141)
    n = mesh['ncells']
    prim = np.concatenate([1 + 0.1 * rng.uniform(-1, 1, (n, 1)), 0.2 * rng.uniform(-1, 1, (n, 2)),
                           1 + 0.1 * rng.uniform(-1, 1, (n, 1)), 0.9 + 0.05 * rng.uniform(-1, 1, (n, 1))], axis=1)
    probe = np.array([[0.7, 3.0, 1.0, 1.6]])
    cs, dia, o = dia_pair(avs, mesh, vs, vgas, 2e-3, prim, random_tree(vs, 142, 1), max_leaves=1024)
    Mk = np.sort(RY.criterion_dia(o.phi, o.W, o.tree, probe, 0.5))

    def gap(j):                      # the nearest index above j with a gap to the next value
        while not Mk[j + 1] - Mk[j] > 1e-9 * Mk[j]:
            j += 1
        return j
    j1, j2 = gap(int(0.8 * len(Mk))), gap(int(0.2 * len(Mk)))
    C1, C2 = 0.5 * (Mk[j1] + Mk[j1 + 1]), 0.5 * (Mk[j2] + Mk[j2 + 1])
    flags0, _ = dia.adapt(C1, C2)
    flags, nn = dia.adapt(C1, C2, probes=probe)
    eff, plan, _ = o.adapt(C1, C2, probe)
    assert np.array_equal(flags, eff) and nn == plan.tree.n
    assert not np.array_equal(flags, flags0)
    dia.remap()
    o.remap()
    v, W = dia.get_state()
    assert rel(v, o.phi) < 1e-12 and rel(W, o.W) < 1e-13
    dia.close()
    cs.close()


def test_diatomic_argument_errors(avs):
    """The diatomic entry points refuse bad arguments with an error and
    leave the state usable: Rykov parameters out of range, a non-physical
    or misshaped initial state, max_leaves beyond the capacity, negative
    step or sweep counts, probe rows of the wrong width."""
    mesh = MM.box2d(3, 3, periodic=(True, True))
    vs = dict(dim=2, lo=(-6.0, -6.0), hi=(6.0, 6.0), base=(8, 8), max_level=1)
    vgas = dict(R=0.5, Pr=0.72, omega=0.74, mu_ref=0.05, T_ref=1.0, model=1)
    n = mesh['ncells']
    prim = np.tile([1.0, 0.1, 0.0, 1.0, 0.9], (n, 1))
    cs = avs.Case(mesh, vs, vgas, 2e-3, 1.0, np.ascontiguousarray(prim[:, :4]))
    for kw in (dict(Z_rot=0.5), dict(delta=0.0), dict(delta=1.5), dict(omega0=float('nan'))):
        with pytest.raises(avs.AvsError):
            avs.Diatomic(cs, prim, **kw)
    bad = prim.copy()
    bad[4, 4] = -1.0
    with pytest.raises(avs.AvsError):
        avs.Diatomic(cs, bad)
    with pytest.raises(ValueError):
        avs.Diatomic(cs, prim[:, :4])
    with pytest.raises(avs.AvsError):
        avs.Diatomic(cs, prim, max_leaves=10 ** 6)
    dia = avs.Diatomic(cs, prim)
    for call in (lambda: dia.step(-1), lambda: dia.step_implicit(1, 2, -1), lambda: dia.step_implicit(-1, 2, 2)):
        with pytest.raises(avs.AvsError):
            call()
    with pytest.raises(ValueError):
        dia.adapt(1e-3, 1e-6, probes=[[1.0, 0.0, 1.0]])
    dia.step(1)
    dia.step_implicit(1, 2, 2)
    v, W = dia.get_state()
    assert np.isfinite(v).all() and np.allclose(W[:, 0], 1.0, rtol=1e-12)
    dia.close()
    cs.close()


def test_diatomic_remap_refuses_a_plan_it_did_not_make(avs):
    """A plan made by the monatomic adaptation of the context (bounded only
    by the context's leaf capacity) is refused by the diatomic remap before
    any device work, also when it would outgrow the diatomic rows; the
    diatomic state stays usable and its own plan is accepted afterwards."""
    mesh = MM.box2d(3, 3, periodic=(True, True))
    vs = dict(dim=2, lo=(-6.0, -6.0), hi=(6.0, 6.0), base=(8, 8), max_level=2)
    vgas = dict(R=0.5, Pr=0.72, omega=0.74, mu_ref=0.05, T_ref=1.0, model=1)
    n = mesh['ncells']
    prim = np.tile([1.0, 0.1, 0.0, 1.0, 0.9], (n, 1))
    cs = avs.Case(mesh, vs, vgas, 2e-3, 1.0, np.ascontiguousarray(prim[:, :4]), leaf_capacity=1024)
    dia = avs.Diatomic(cs, prim)                # rows for the current 64 leaves only
    n0 = cs.nleaves()
    _, nn = cs.adapt(-1.0, -2.0)                # split everything: 256 leaves > 64 rows
    assert nn == 4 * n0
    with pytest.raises(avs.AvsError, match="not made by avs_dia_adapt"):
        dia.remap()
    assert cs.nleaves() == n0
    dia.step(1)
    v, W = dia.get_state()
    assert np.isfinite(v).all() and np.allclose(W[:, 0], 1.0, rtol=1e-12)
    # its own plan (merge-free, no split: keeps the leaf count) is accepted
    _, nn2 = dia.adapt(1e30, -1.0)
    assert nn2 == n0
    dia.remap()
    dia.step(1)
    v2, _ = dia.get_state()
    assert np.isfinite(v2).all() and v2.shape == v.shape
    # a diatomic plan is not taken by another diatomic state
    dia_b = avs.Diatomic(cs, prim)
    dia.adapt(1e30, -1.0)
    with pytest.raises(avs.AvsError, match="not made by avs_dia_adapt"):
        dia_b.remap()
    dia.remap()
    dia_b.close()
    dia.close()
    cs.close()

