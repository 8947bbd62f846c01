"""GPU (HIP, through the C ABI) vs FP64 oracle on identical seeded inputs.

Tolerances: FP64 path 1e-12 relative per step on the VDF and W (the two
sides differ only by summation order and fused multiply-adds), 1e-10 on the
macroscopic fields over a run; integer work (flags, plan, leaf tables) bit
exact; FP32 form 1e-5 field-normalised with FP64 conservation.
Leaf counts of a few hundred span several 256-leaf chunks with a ragged tail.
"""
import math

import numpy as np
import pytest

from oracle import avs_oracle as O
from workloads import fields as F
from workloads import meshes as MM
from workloads import trees as TR

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def avs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_05645_amd import avs as mod
    return mod


def rel(a, b):
    """Largest error of a row relative to that row's largest reference
    value; a row is the last axis (the leaves of one cell and component, or
    one cell's W), so a cell of small density is judged on its own scale."""
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    if b.ndim < 2:
        return float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))), 1e-300))
    a2, b2 = a.reshape(-1, b.shape[-1]), b.reshape(-1, b.shape[-1])
    den = np.maximum(np.max(np.abs(b2), axis=1), 1e-300)
    return float(np.max(np.max(np.abs(a2 - b2), axis=1) / den))


def tailrel(a, b, floor=1e-8):
    """Elementwise error relative to the value itself, floored at ``floor``
    times its row's largest value: a leaf down to 1e-8 of the row's peak is
    judged on its own size, so a wrong upwind side or boundary branch on a
    tail leaf is seen (it changes the value by order one)."""
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    a2, b2 = a.reshape(-1, b.shape[-1]), b.reshape(-1, b.shape[-1])
    den = np.abs(b2) + floor * np.max(np.abs(b2), axis=1, keepdims=True) + 1e-300
    return float(np.max(np.abs(a2 - b2) / den))


def fieldrel(a, b):
    """max_i |a - b| / max_i |b| per column (field-normalised)."""
    a, b = np.asarray(a), np.asarray(b)
    return max(float(np.max(np.abs(a[:, j] - b[:, j])) / max(float(np.max(np.abs(b[:, j]))), 1e-300))
               for j in range(b.shape[1]))


def otree(vspace, level, idx):
    """The oracle's view of a generated leaf list."""
    D = vspace['dim']
    return O.Tree(D, np.asarray(vspace['lo'], np.float64)[:D], np.asarray(vspace['hi'], np.float64)[:D],
                  np.asarray(vspace['base'], np.int64)[:D], int(vspace['max_level']),
                  np.asarray(level, np.int64), np.asarray(idx, np.int64))


def random_tree(vspace, seed, rounds, p=0.35):
    return otree(vspace, *TR.random_tree(vspace['dim'], vspace['base'], vspace['max_level'], seed, rounds, p))


def resolved_tree(vspace, seed, p=0.35):
    """Every root split once, then a random fraction split again."""
    return otree(vspace, *TR.resolved_tree(vspace['dim'], vspace['base'], vspace['max_level'], seed, p))


def make_pair(avs, mesh, vspace, gas, dt, prim0, tree=None, precision=0, noise=0.0, seed=0, Kv=1.0, cap=None):
    o = O.Solver(mesh, vspace, gas, dt, Kv, prim0)
    # each side derives mu_ref from Kn itself (the gas dict carries Kn, or mu_ref directly)
    cs = avs.Case(mesh, vspace, gas, dt, Kv, prim0, precision=precision, leaf_capacity=cap)
    if tree is not None:
        o.tree = tree
        o.phi = o.initial_vdf(o.W)
        cs.set_leaves(tree.level, tree.idx)
    if noise > 0:
        # the same seeded relative perturbation of each side's own initial state;
        # W follows as the moments of the perturbed VDF on each side
        fac = 1.0 + noise * np.random.default_rng(seed).standard_normal(o.phi.shape)
        o.phi = o.phi * fac
        o.W = o.vdf_moments()
        v0, _ = cs.get_state()
        cs.set_state(v0 * fac, None)
    return cs, o


def gas_of(cfg_gas, model=1):
    g = dict(cfg_gas)
    g['model'] = model
    return g


# ------------------------------------------------------------ init, steps ---
def test_initial_state_and_leaf_table(avs):
    c = F.cavity(n=8, base=8, max_level=2)
    t = random_tree(c['vspace'], 1, 2)
    cs, o = make_pair(avs, c['mesh'], c['vspace'], c['gas'], c['dt'], c['prim0'], tree=t)
    L = cs.leaves()
    assert np.array_equal(L['level'], t.level) and np.array_equal(L['idx'], t.idx)
    assert np.array_equal(L['xi'], t.centres()) and np.array_equal(L['w'], t.weights())
    v, W = cs.get_state()
    assert rel(v, o.phi) < 1e-13 and np.array_equal(W, o.W)


@pytest.mark.parametrize("model", [0, 1])
def test_cavity_steps(avs, model):
    c = F.cavity(n=8, base=8, max_level=2)
    t = random_tree(c['vspace'], 2, 2)
    cs, o = make_pair(avs, c['mesh'], c['vspace'], gas_of(c['gas'], model), c['dt'], c['prim0'], tree=t,
                      noise=0.02, seed=3)
    for n in range(4):
        r = cs.step(1, residual=True)
        ro = o.step(1)
        v, W = cs.get_state()
        assert rel(v, o.phi) < 1e-12, n
        assert rel(W, o.W) < 1e-13, n
        assert rel(r, ro) < 1e-8, n
    f, tot = cs.moments()
    assert fieldrel(f.cpu().numpy(), o.fields()) < 1e-10
    np.testing.assert_allclose(tot, o.totals(), rtol=1e-13, atol=1e-15)


def test_periodic_conservation_random_tree(avs):
    mesh = MM.box2d(7, 5, periodic=(True, True))
    vs = dict(dim=2, lo=(-6, -6), hi=(6, 6), base=(8, 8), max_level=2)
    gas = dict(R=1.0, Pr=2 / 3, omega=0.81, mu_ref=0.03, T_ref=1.0, model=1)
    prim = F.perturbed_uniform(mesh['ncells'], 2, 7, amp=0.1, uamp=0.4)
    cs, o = make_pair(avs, mesh, vs, gas, 0.004, prim, tree=random_tree(vs, 4, 2))
    _, tot0 = cs.moments(fields=False)
    cs.step(5)
    o.step(5)
    v, W = cs.get_state()
    assert rel(v, o.phi) < 1e-12 and rel(W, o.W) < 1e-13
    _, tot = cs.moments(fields=False)
    np.testing.assert_allclose(tot, tot0, rtol=1e-13, atol=1e-13)


def test_ogrid_wall_and_farfield(avs):
    c = F.cylinder(nr=6, nth=24, Ma=2.0, box=8.0, base=16, max_level=2, r1=2.5, first=0.1)
    cs, o = make_pair(avs, c['mesh'], c['vspace'], c['gas'], c['dt'], c['prim0'], tree=resolved_tree(c['vspace'], 5),
                      noise=0.01, seed=5)
    cs.step(3)
    o.step(3)
    v, W = cs.get_state()
    assert rel(v, o.phi) < 1e-12 and rel(W, o.W) < 1e-12


@pytest.mark.parametrize("prec", [0, 1])
def test_sutherland_viscosity(avs, prec):
    """Sutherland's law for tau (Eq. Sutherland; C_s = 111 K over a 43.22 K
    freestream, the sphere's nitrogen at Ma 5.45) on the O-grid with walls
    and far field: FP64 to 1e-12 per step, FP32 form within 1e-5."""
    c = F.cylinder(nr=6, nth=24, Ma=2.0, box=8.0, base=16, max_level=2, r1=2.5, first=0.1)
    gas = dict(c['gas'], law=1, C_s=111.0 / 43.22)
    cs, o = make_pair(avs, c['mesh'], c['vspace'], gas, c['dt'], c['prim0'], tree=resolved_tree(c['vspace'], 5),
                      noise=0.01, seed=5, precision=prec)
    assert o.gas.law == 1
    nstep = 3 if prec == 0 else 5
    cs.step(nstep)
    o.step(nstep)
    v, W = cs.get_state()
    if prec == 0:
        assert rel(v, o.phi) < 1e-12 and rel(W, o.W) < 1e-12
    else:
        assert fieldrel(W, o.W) < 1e-5
    # the power law on the same state gives a different result
    cp, op = make_pair(avs, c['mesh'], c['vspace'], c['gas'], c['dt'], c['prim0'], tree=resolved_tree(c['vspace'], 5),
                       noise=0.01, seed=5, precision=prec)
    cp.step(nstep)
    assert rel(cp.get_state()[1], W) > 1e-9


@pytest.mark.parametrize("D", [2, 3])
def test_cells_with_fewer_faces_than_slots(avs, D):
    """A cut-out block of a body-fitted grid whose outermost ring has
    incomplete face lists (cells with 1-3 of 4, or 2-5 of 6, faces; the
    dropped faces carry no flux on either side), so every slot kind is
    exercised: interior, wall or far-field boundary, and unused."""
    if D == 2:
        c = F.cylinder(nr=8, nth=24, Ma=2.0, box=8.0, base=16, max_level=2, r1=2.5, first=0.1)
        block = [r * 24 + t for r in range(0, 3) for t in range(5, 9)] + [7 * 24 + 15]
    else:
        c = F.sphere(nr=4, nth=6, nph=6, Ma=2.0, box=5.0, base=8, max_level=1, r1=1.5, first=0.2)
        block = [0, 1, 7, 40, 41]
    sub, keep = MM.submesh(c['mesh'], block, halo=1)
    nslot = np.bincount(np.asarray(sub['face_lr'])[:, 0], minlength=sub['ncells']) + \
        np.bincount(np.asarray(sub['face_lr'])[:, 1][np.asarray(sub['face_lr'])[:, 1] >= 0], minlength=sub['ncells'])
    assert nslot.min() < 2 * D and (nslot == 2 * D).any()
    tree = resolved_tree(c['vspace'], 8)
    cs, o = make_pair(avs, sub, c['vspace'], c['gas'], c['dt'], c['prim0'][keep], tree=tree, noise=0.01, seed=8,
                      Kv=c['venkat_K'])
    cs.step(3)
    o.step(3)
    v, W = cs.get_state()
    assert rel(v, o.phi) < 1e-12 and rel(W, o.W) < 1e-12


@pytest.mark.parametrize("dim,Ma", [(2, 2.0), (2, 6.0), (3, 4.25)])
def test_initial_avs_matches_oracle(avs, dim, Ma):
    """Step-0 velocity space of Sec. 3.5 through the C ABI: the leaves after
    the uniform splits and the probes-only adaptation equal the oracle's bit
    for bit, and the state is the closed Maxwellian of W on them."""
    from oracle import avs_params as AP
    if dim == 2:
        c = F.cylinder(nr=6, nth=16, Ma=Ma, box=8.0, base=16, max_level=2, r1=2.5, first=0.1)
        gamma = 5.0 / 3.0
    else:
        c = F.sphere(nr=3, nth=4, nph=4, Ma=Ma, box=5.0, base=8, max_level=1, r1=1.5, first=0.2)
        gamma = 1.4
    flow = dict(dim=dim, R=c['gas']['R'], gamma=gamma, Ma=Ma, T_inf=1.0, T_wall=1.0)
    params, vs = avs.auto_params(**flow)
    C1 = 1e-3
    C2 = params['k_sigma'] * C1
    cs = avs.Case(c['mesh'], vs, c['gas'], c['dt'], c['venkat_K'], c['prim0'], leaf_capacity=vs['leaf_capacity'])
    n = cs.initial_avs(C1, C2, **flow)
    f = AP.Flow(**flow)
    t0, eff, t1 = AP.initial_tree(f, C1=C1, C2=C2)
    L = cs.leaves()
    assert n == t1.n == len(L['level'])
    assert np.array_equal(L['level'], t1.level) and np.array_equal(L['idx'], t1.idx)
    assert (eff == 1).any()
    o = O.Solver(c['mesh'], vs, c['gas'], c['dt'], c['venkat_K'], c['prim0'])
    o.tree = t1
    o.phi = o.initial_vdf(o.W)
    v, W = cs.get_state()
    assert rel(v, o.phi) < 1e-12 and rel(W, o.W) < 1e-12
    # a velocity space that is not the one of this flow is refused
    with pytest.raises(avs.AvsError):
        cs.initial_avs(C1, C2, **dict(flow, Ma=Ma + 1.0))
    cs.close()


@pytest.mark.parametrize("dim,Ma,Tw", [(2, 6.0, 3.0), (3, 4.25, 3.0)])
def test_initial_avs_separated_matches_oracle(avs, dim, Ma, Tw):
    """Separating flow with a warm wall: the step-0 velocity space with the
    separated zone of Sec. 3.5 equals the oracle's leaf for leaf (and is not
    the plain one); the zone stays on the context, so after two steps the
    next adaptation's flags equal the oracle's under the same floor; a zone
    with crossed radii is refused and a negative level removes it."""
    from oracle import avs_params as AP
    if dim == 2:
        c = F.cylinder(nr=6, nth=16, Ma=Ma, box=13.0, base=16, max_level=2, r1=2.5, first=0.1)
        gamma = 5.0 / 3.0
    else:
        c = F.sphere(nr=3, nth=4, nph=4, Ma=Ma, box=8.0, base=8, max_level=1, r1=1.5, first=0.2)
        gamma = 1.4
    flow = dict(dim=dim, R=c['gas']['R'], gamma=gamma, Ma=Ma, T_inf=1.0, T_wall=Tw)
    params, vs = avs.auto_params(**flow)
    C1 = 1e-3
    C2 = params['k_sigma'] * C1
    cs = avs.Case(c['mesh'], vs, c['gas'], c['dt'], c['venkat_K'], c['prim0'], leaf_capacity=vs['leaf_capacity'])
    n = cs.initial_avs(C1, C2, **flow, separated=True)
    p = AP.auto_params(AP.Flow(**flow))
    _, _, t1 = AP.initial_tree(AP.Flow(**flow, separated=True), p, C1=C1, C2=C2)
    _, _, plain = AP.initial_tree(AP.Flow(**flow), p, C1=C1, C2=C2)
    L = cs.leaves()
    assert n == t1.n and np.array_equal(L['level'], t1.level) and np.array_equal(L['idx'], t1.idx)
    assert t1.n != plain.n
    o = O.Solver(c['mesh'], vs, c['gas'], c['dt'], c['venkat_K'], c['prim0'])
    o.tree = t1
    o.phi = o.initial_vdf(o.W)
    o.separated = AP.separated_zone(p)
    cs.step(2)
    o.step(2)
    v, W = cs.get_state()
    assert rel(v, o.phi) < 1e-12 and rel(W, o.W) < 1e-12
    # thresholds under which the zone holds merges back after the steps
    C1b, C2b = 1e-2, 3e-3
    flags, nn = cs.adapt(C1b, C2b)
    eff, plan, _ = o.adapt(C1b, C2b)
    assert np.array_equal(flags, eff) and nn == plan.tree.n
    o.separated = None
    eff0, _, _ = o.adapt(C1b, C2b)
    assert not np.array_equal(eff0, eff)
    with pytest.raises(avs.AvsError):
        cs.set_separated(2.0, 1.0, 1)
    cs.set_separated(0.0, 1.0, -1)
    flags0, _ = cs.adapt(C1b, C2b)
    assert np.array_equal(flags0, eff0)
    cs.close()


# ------------------------------------------------ unstructured meshes ------
def test_unstructured_triangles(avs):
    """Triangles of a jittered lattice with random diagonals (three faces
    per cell, corner cells with one interior neighbour take the
    pseudo-inverse gradient), walls below and above, far field left and
    right: steps, one adaptation (flags bit exact) with the closed remap,
    and more steps, FP64 to 1e-12."""
    U = 1.5 * math.sqrt(5.0 / 3.0)
    mesh = MM.tri_box(10, 8, 41, lx=1.25, ly=1.0, sides=dict(left=1, right=1, bottom=0, top=0),
                      bcs=[(MM.WALL, (1.0, 0.0, 0.0, 1.3)), (MM.FARFIELD, (1.0, U, 0.0, 1.0))])
    vs = dict(dim=2, lo=(-6.0, -6.0), hi=(8.0, 6.0), base=(8, 8), max_level=2)
    gas = dict(R=1.0, Pr=2 / 3, omega=0.81, mu_ref=0.02, T_ref=1.0, model=1)
    prim = F.perturbed_uniform(mesh['ncells'], 2, 42, amp=0.1, uamp=0.5)
    cs, o = make_pair(avs, mesh, vs, gas, 2e-3, prim, tree=random_tree(vs, 43, 2), noise=0.01, seed=44, Kv=0.0)
    cs.step(3)
    o.step(3)
    v, W = cs.get_state()
    assert rel(v, o.phi) < 1e-12 and rel(W, o.W) < 1e-12
    flags, nn = cs.adapt(5e-3, 1e-4)
    eff, plan, _ = o.adapt(5e-3, 1e-4)
    assert np.array_equal(flags, eff) and nn == plan.tree.n
    cs.remap(2)
    o.remap(2)
    cs.step(2)
    o.step(2)
    v, W = cs.get_state()
    assert rel(v, o.phi) < 1e-12 and rel(W, o.W) < 1e-12


def test_unstructured_tetrahedra(avs):
    """Tetrahedra (six per jittered hexahedron, four faces each) with walls
    on every side, FP64 steps to 1e-12."""
    mesh = MM.tet_box(3, 3, 2, 51)
    vs = dict(dim=3, lo=(-5.0,) * 3, hi=(5.0,) * 3, base=(4, 4, 4), max_level=2)
    gas = dict(R=1.0, Pr=2 / 3, omega=0.5, mu_ref=0.05, T_ref=1.0, model=1)
    prim = F.perturbed_uniform(mesh['ncells'], 3, 52, amp=0.1, uamp=0.4)
    cs, o = make_pair(avs, mesh, vs, gas, 1e-3, prim, tree=random_tree(vs, 53, 2), noise=0.01, seed=54)
    cs.step(2)
    o.step(2)
    v, W = cs.get_state()
    assert rel(v, o.phi) < 1e-12 and rel(W, o.W) < 1e-12


def test_blunt_wedge_full_size(avs):
    """The unstructured blunt-wedge workload at full size (about 11 900
    triangles, Ma 8.1): the step-0 velocity space of Sec. 3.5 built by the
    library equals the oracle's leaf for leaf; after one step in the
    benchmark's launch configuration, sampled cells (wall, nose, flank,
    base, far field) are recomputed by the oracle from their two-ring
    neighbourhood and compared element by element."""
    from oracle import avs_params as AP
    flow = F.wedge_flow()
    params, vs = avs.auto_params(**flow)
    c = F.blunt_wedge(vs)
    C1 = 1e-3
    C2 = params['k_sigma'] * C1
    cs = avs.Case(c['mesh'], vs, c['gas'], c['dt'], c['venkat_K'], c['prim0'], leaf_capacity=vs['leaf_capacity'])
    n = cs.initial_avs(C1, C2, **flow)
    _, _, t = AP.initial_tree(AP.Flow(**flow), C1=C1, C2=C2)
    L = cs.leaves()
    assert n == t.n and np.array_equal(L['level'], t.level) and np.array_equal(L['idx'], t.idx)
    cs.step(1)
    m = c['mesh']
    lr = m['face_lr']
    wall = lr[lr[:, 1] == -1, 0]
    far = lr[lr[:, 1] == -2, 0]
    ctr = m['cell_ctr']
    sample = sorted(set([int(wall[0]), int(wall[len(wall) // 2]), int(far[0]), int(far[-1]),
                         int(np.argmin(np.hypot(ctr[:, 0] + 0.3, ctr[:, 1]))),      # ahead of the nose
                         int(np.argmin(np.hypot(ctr[:, 0] - 7.0, ctr[:, 1]))),      # behind the base
                         int(np.argmin(np.hypot(ctr[:, 0] - 3.0, ctr[:, 1] - 2.0))),  # above the flank
                         m['ncells'] - 1]))
    got = cs.get_cells(sample)
    Wg = cs.get_W()[sample]
    sub, keep = MM.submesh(m, sample, halo=2)
    gas = O.gas_from(c['gas'])
    o = O.Solver(sub, vs, gas, c['dt'], c['venkat_K'], c['prim0'][keep])
    o.tree = t
    o.phi = o.initial_vdf(o.W)
    loc = [int(np.searchsorted(keep, i)) for i in sample]
    phi1, W1, _ = O.step(o.mesh, t, gas, c['dt'], c['venkat_K'], o.phi, o.W, cells=loc)
    assert rel(got, phi1[:, loc]) < 1e-12
    assert rel(Wg, W1[loc]) < 1e-13
    cs.close()


@pytest.mark.parametrize("which", ["box", "sphere"])
def test_3d_steps(avs, which):
    if which == "box":
        mesh = MM.box3d(3, 3, 2, periodic=(True, False, True))
        prim = F.perturbed_uniform(mesh['ncells'], 3, 9, amp=0.05, uamp=0.3)
        vs = dict(dim=3, lo=(-5,) * 3, hi=(5,) * 3, base=(4,) * 3, max_level=1)
        gas = dict(R=1.0, Pr=2 / 3, omega=0.74, mu_ref=0.05, T_ref=1.0, model=1)
        dt = 0.004
    else:
        c = F.sphere(nr=3, nth=4, nph=4, Ma=2.0, box=5.0, base=8, max_level=1, r1=1.5, first=0.2)
        mesh, prim, vs, gas, dt = c['mesh'], c['prim0'], c['vspace'], c['gas'], c['dt']
    tree = random_tree(vs, 6, 1, p=0.25) if which == "box" else resolved_tree(vs, 6)
    cs, o = make_pair(avs, mesh, vs, gas, dt, prim, tree=tree, noise=0.01, seed=6, Kv=0.0 if which == "sphere" else 1.0)
    cs.step(3)
    o.step(3)
    v, W = cs.get_state()
    assert rel(v, o.phi) < 1e-12 and rel(W, o.W) < 1e-12
    assert tailrel(v, o.phi) < 1e-6


def test_3d_fp32_form_against_fp64_oracle(avs):
    """The 3-D FP32 form (the sphere workload's form) on a small spherical
    grid: fields within 1e-5 field-normalised after 5 steps, FP64 totals."""
    c = F.sphere(nr=3, nth=4, nph=4, Ma=2.0, box=5.0, base=8, max_level=1, r1=1.5, first=0.2)
    cs, o = make_pair(avs, c['mesh'], c['vspace'], c['gas'], c['dt'], c['prim0'], tree=resolved_tree(c['vspace'], 8),
                      precision=1, noise=0.01, seed=8, Kv=0.0)
    cs.step(5)
    o.step(5)
    f, tot = cs.moments()
    assert fieldrel(f.cpu().numpy(), o.fields()) < 1e-5
    ot = o.totals()
    assert np.max(np.abs(tot - ot)) < 1e-5 * np.max(np.abs(ot))


def test_capacity_error_leaves_state_usable(avs):
    """An adaptation that would exceed leaf_capacity reports AVS_E_CAPACITY,
    builds no plan, and leaves the case stepping exactly as before."""
    c = F.cavity(n=8, base=8, max_level=2)
    tree = random_tree(c['vspace'], 12, 1, p=0.2)
    cs, o = make_pair(avs, c['mesh'], c['vspace'], c['gas'], c['dt'], c['prim0'], tree=tree, cap=tree.n + 10)
    with pytest.raises(avs.AvsError) as e:
        cs.adapt(-1.0, -2.0)                 # split everything: far beyond the capacity
    assert e.value.status == avs.AVS_E_CAPACITY
    with pytest.raises(avs.AvsError) as e:
        cs.remap(2)
    assert e.value.status == avs.AVS_E_STATE
    assert cs.nleaves() == tree.n
    cs.step(2)
    o.step(2)
    v, W = cs.get_state()
    assert rel(v, o.phi) < 1e-12 and rel(W, o.W) < 1e-12


# ------------------------------------------------------------- adaptation --
@pytest.mark.parametrize("D,seed", [(2, 0), (2, 1), (3, 2)])
def test_adapt_flags_plan_bit_exact(avs, D, seed):
    """Criterion over cells only is bit-exact (same operation order, no
    contraction); effective flags, remap plan and new leaf table too."""
    if D == 2:
        mesh = MM.box2d(5, 4, periodic=(True, True))
        vs = dict(dim=2, lo=(-6, -6), hi=(6, 6), base=(8, 8), max_level=3)
    else:
        mesh = MM.box3d(2, 2, 2)
        vs = dict(dim=3, lo=(-6,) * 3, hi=(6,) * 3, base=(4,) * 3, max_level=2)
    gas = dict(R=1.0, Pr=2 / 3, omega=0.5, mu_ref=0.05, T_ref=1.0, model=1)
    prim = F.perturbed_uniform(mesh['ncells'], D, seed, amp=0.2, uamp=0.8)
    cs, o = make_pair(avs, mesh, vs, gas, 1e-3, prim, tree=random_tree(vs, 10 + seed, 2), noise=0.05, seed=seed)
    for C1 in (3e-3, 1e-2):
        C2 = math.exp(-8.0) * C1 * 50
        v, W = cs.get_state()
        o.phi, o.W = v, W
        fl, nn = cs.adapt(C1, C2)
        eff, plan, Mk = o.adapt(C1, C2)
        assert np.array_equal(cs.criterion(len(fl)), Mk)
        assert np.array_equal(fl, eff)
        assert (eff == 1).any() and (eff == -1).any()
        kind, src, child = cs.plan(nn)
        assert nn == plan.tree.n
        assert np.array_equal(kind, plan.kind) and np.array_equal(src, plan.src) and np.array_equal(child, plan.child)
        cs.remap(0)
        o.remap(0)
        L = cs.leaves()
        assert np.array_equal(L['level'], o.tree.level) and np.array_equal(L['idx'], o.tree.idx)
        assert np.array_equal(L['xi'], o.tree.centres()) and np.array_equal(L['w'], o.tree.weights())
        v, _ = cs.get_state()
        assert np.array_equal(v, o.phi)     # consanguinity gather is exact arithmetic


def test_adapt_with_probe_states(avs):
    """Probe VDFs are discrete Maxwellians evaluated with each side's exp:
    M_k agrees to 1e-15 and flags are identical away from ties."""
    c = F.cavity(n=6, base=16, max_level=2)
    cs, o = make_pair(avs, c['mesh'], c['vspace'], c['gas'], c['dt'], c['prim0'])
    for _ in range(2):
        fl, nn = cs.adapt(c['C1'], c['C2'], probes=c['probes'])
        eff, plan, Mk = o.adapt(c['C1'], c['C2'], probes=c['probes'])
        Mg = cs.criterion(len(fl))
        assert rel(Mg, Mk) < 1e-15
        near = (np.abs(Mk - c['C1']) < 1e-14 * c['C1']) | (np.abs(Mk - c['C2']) < 1e-14 * c['C2'])
        assert np.array_equal(fl[~near], eff[~near])
        cs.remap(2)
        o.remap(2)
    assert o.tree.n == 496 and cs.nleaves() == 496


@pytest.mark.parametrize("correction", [1, 2, 3, 4])
def test_remap_correction(avs, correction):
    """Corrections 1/2 of Sec. 3.3 and the equilibrium bypass 3/4 (end of
    Sec. 3.3) against the oracle's remap of the same plan."""
    mesh = MM.box2d(5, 4, periodic=(True, True))
    vs = dict(dim=2, lo=(-6, -6), hi=(6, 6), base=(8, 8), max_level=3)
    gas = dict(R=1.0, Pr=2 / 3, omega=0.5, mu_ref=0.05, T_ref=1.0, model=1)
    prim = F.perturbed_uniform(mesh['ncells'], 2, 21, amp=0.2, uamp=0.8)
    cs, o = make_pair(avs, mesh, vs, gas, 1e-3, prim, tree=random_tree(vs, 22, 2), noise=0.05, seed=23)
    cs.adapt(5e-3, 1e-4)
    o.adapt(5e-3, 1e-4)
    with pytest.raises(avs.AvsError):
        cs.remap(5)
    cs.remap(correction)
    o.remap(correction)
    v, W = cs.get_state()
    assert rel(v, o.phi) < 1e-12
    if correction in (2, 4):
        np.testing.assert_allclose(o.vdf_moments(), W, rtol=1e-12, atol=1e-13)
    # W is the cell state; only the closed forms reproduce it from the new VDF
    np.testing.assert_allclose(W, o.W, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("D,prec,correction", [(2, 0, 1), (2, 0, 2), (2, 1, 2), (3, 0, 2), (3, 1, 2)])
def test_remap_moments_equal_recomputed(avs, D, prec, correction):
    """The correction kernel leaves the moments and heat flux of the new
    state for the next step; a twin case that recomputes them through the
    moments pass after the same remap steps to the same state bit for bit."""
    if D == 2:
        mesh = MM.box2d(5, 4, periodic=(True, True))
        vs = dict(dim=2, lo=(-6, -6), hi=(6, 6), base=(8, 8), max_level=3)
    else:
        mesh = MM.box3d(3, 3, 2, periodic=(True, True, True))
        vs = dict(dim=3, lo=(-5, -5, -5), hi=(5, 5, 5), base=(4, 4, 4), max_level=2)
    gas = dict(R=1.0, Pr=2 / 3, omega=0.5, mu_ref=0.05, T_ref=1.0, model=1)
    prim = F.perturbed_uniform(mesh['ncells'], D, 41, amp=0.2, uamp=0.6)
    tree = random_tree(vs, 42, 2)
    cases = []
    for _ in range(2):
        cs, _ = make_pair(avs, mesh, vs, gas, 1e-3, prim, tree=tree, precision=prec, noise=0.05, seed=43)
        n = cs.adapt(5e-3, 1e-4)[1]
        cs.remap(correction)
        cases.append((cs, n))
    assert cases[0][1] == cases[1][1] and cases[0][1] != tree.n
    cases[1][0].moments(fields=True, totals=False)     # recomputes the moments and heat flux
    states = []
    for cs, _ in cases:
        cs.step(2)
        v, W = cs.get_state()
        states.append((np.asarray(v), np.asarray(W)))
    assert np.array_equal(states[0][0], states[1][0]) and np.array_equal(states[0][1], states[1][1])


@pytest.mark.parametrize("correction", [3, 4])
def test_bypass_remap_3d(avs, correction):
    mesh = MM.box3d(3, 3, 2, periodic=(True, True, True))
    vs = dict(dim=3, lo=(-5, -5, -5), hi=(5, 5, 5), base=(4, 4, 4), max_level=2)
    gas = dict(R=1.0, Pr=2 / 3, omega=0.5, mu_ref=0.05, T_ref=1.0, model=1)
    prim = F.perturbed_uniform(mesh['ncells'], 3, 31, amp=0.2, uamp=0.6)
    cs, o = make_pair(avs, mesh, vs, gas, 1e-3, prim, tree=random_tree(vs, 32, 2), noise=0.05, seed=33)
    cs.adapt(5e-3, 1e-4)
    o.adapt(5e-3, 1e-4)
    cs.remap(correction)
    o.remap(correction)
    v, W = cs.get_state()
    assert cs.nleaves() == o.tree.n
    assert rel(v, o.phi) < 1e-12
    if correction == 4:
        np.testing.assert_allclose(o.vdf_moments(), W, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("D,prec", [(2, 0), (3, 0), (2, 1)])
def test_split_then_merge_identity_on_gpu(avs, D, prec):
    """Split every leaf down to the maximum level, then merge every brother
    group back up: the VDF returns bit for bit (P3), FP64 and FP32 storage."""
    if D == 2:
        mesh = MM.box2d(3, 3, periodic=(True, True))
        vs = dict(dim=2, lo=(-6, -6), hi=(6, 6), base=(4, 4), max_level=2)
    else:
        mesh = MM.box3d(2, 2, 2)
        vs = dict(dim=3, lo=(-4,) * 3, hi=(4,) * 3, base=(4,) * 3, max_level=2)
    gas = dict(R=1.0, Pr=2 / 3, omega=0.5, mu_ref=0.05, T_ref=1.0, model=1)
    prim = F.perturbed_uniform(mesh['ncells'], D, 31)
    cs, o = make_pair(avs, mesh, vs, gas, 1e-3, prim, noise=0.1, seed=33, precision=prec)
    v0, _ = cs.get_state()
    L0 = cs.leaves()
    for _ in range(vs['max_level']):
        cs.adapt(-1.0, -np.inf)
        cs.remap(0)
    assert np.all(cs.leaves()['level'] == vs['max_level'])
    for _ in range(vs['max_level']):
        cs.adapt(np.inf, np.inf)
        cs.remap(0)
    v1, _ = cs.get_state()
    L1 = cs.leaves()
    assert np.array_equal(L1['level'], L0['level']) and np.array_equal(L1['idx'], L0['idx'])
    assert np.array_equal(v1.view(np.uint8), v0.view(np.uint8))


# ------------------------------------------------------------- FP32 form ---
def test_fp32_form_against_fp64_oracle(avs):
    c = F.cylinder(nr=8, nth=32, Ma=2.0, box=8.0, base=16, max_level=2, r1=2.5, first=0.1)
    t = resolved_tree(c['vspace'], 41)
    cs, o = make_pair(avs, c['mesh'], c['vspace'], c['gas'], c['dt'], c['prim0'], tree=t, precision=1)
    _, tot0 = cs.moments(fields=False)
    cs.step(10)
    o.step(10)
    f, tot = cs.moments()
    assert fieldrel(f.cpu().numpy(), o.fields()) < 1e-5
    # totals move through wall and far-field fluxes computed from FP32 VDFs
    ot = o.totals()
    assert np.max(np.abs(tot - ot)) < 1e-5 * np.max(np.abs(ot))


def test_fp32_periodic_conservation(avs):
    mesh = MM.box2d(6, 6, periodic=(True, True))
    vs = dict(dim=2, lo=(-6, -6), hi=(6, 6), base=(8, 8), max_level=2)
    gas = dict(R=1.0, Pr=2 / 3, omega=0.81, mu_ref=0.03, T_ref=1.0, model=1)
    prim = F.perturbed_uniform(mesh['ncells'], 2, 44, amp=0.1, uamp=0.4)
    cs, o = make_pair(avs, mesh, vs, gas, 0.004, prim, tree=random_tree(vs, 45, 2), precision=1)
    _, tot0 = cs.moments(fields=False)
    cs.step(20)
    _, tot = cs.moments(fields=False)
    np.testing.assert_allclose(tot, tot0, rtol=1e-12, atol=1e-12)


# ------------------------------------------------- the C1 cavity workload --
def test_cavity_workload_with_adaptation(avs):
    """32x32 cavity, base 16^2, two levels, C1 = 0.01: step-0 adaptation on the
    lid and rest probe states, 20 steps, a run-time adaptation and 4 more
    steps; fields within 1e-10 of the oracle."""
    c = F.cavity()
    cs, o = make_pair(avs, c['mesh'], c['vspace'], c['gas'], c['dt'], c['prim0'])
    for _ in range(2):
        cs.adapt(c['C1'], c['C2'], probes=c['probes'])
        o.adapt(c['C1'], c['C2'], probes=c['probes'])
        cs.remap(2)
        o.remap(2)
    cs.set_state(None, cs.get_W())          # re-close from the GPU's own (unchanged) W
    o.phi = o.initial_vdf(o.W)
    cs.step(20)
    o.step(20)
    fl, nn = cs.adapt(c['C1'], c['C2'])
    v, W = cs.get_state()
    eff, plan, Mk = o.adapt(c['C1'], c['C2'])
    assert nn == plan.tree.n
    cs.remap(2)
    o.remap(2)
    cs.step(4)
    o.step(4)
    f, _ = cs.moments()
    assert fieldrel(f.cpu().numpy(), o.fields()) < 1e-10


# ----------------------------------------- full size, sampled outputs ------
def test_full_size_cylinder_sampled(avs):
    """The cylinder workload at full size (O-grid 128 x 256, 32^2 roots, 3
    levels), one step in the launch configuration the benchmark times, on a
    seeded random tree of all three levels (about 16 k leaves); both sides
    start from the same primitive field.  Sampled cells (wall, shock layer,
    wake, far field) are recomputed by the oracle from their two-ring
    neighbourhood and compared element by element."""
    c = F.cylinder()
    vs = c['vspace']
    t = random_tree(vs, 77, 3, p=0.5)
    assert 2000 < t.n < 40000
    gas = O.gas_from(c['gas'])
    cs = avs.Case(c['mesh'], vs, c['gas'], c['dt'], c['venkat_K'], c['prim0'], leaf_capacity=t.n)
    cs.set_leaves(t.level, t.idx)
    cs.step(1)
    nth = c['mesh']['shape'][1]
    sample = [0, 5, 128, 20 * nth + 7, 40 * nth + 128, 60 * nth + 64, 64 * nth + 200, 90 * nth + 31,
              127 * nth + 0, 127 * nth + 255]
    got = cs.get_cells(sample)
    Wg = cs.get_W()[sample]
    from workloads import meshes
    sub, keep = meshes.submesh(c['mesh'], sample, halo=2)
    o = O.Solver(sub, vs, gas, c['dt'], c['venkat_K'], c['prim0'][keep])
    o.tree = t
    o.phi = o.initial_vdf(o.W)
    loc = [int(np.searchsorted(keep, i)) for i in sample]
    phi1, W1, _ = O.step(o.mesh, t, gas, c['dt'], c['venkat_K'], o.phi, o.W, cells=loc)
    assert rel(got, phi1[:, loc]) < 1e-12
    assert tailrel(got, phi1[:, loc]) < 1e-6
    assert rel(Wg, W1[loc]) < 1e-13


@pytest.mark.parametrize("prec", [0, 1])
def test_full_size_sphere_sampled(avs, prec):
    """The sphere workload at full size (64 x 64 x 32 spherical grid, 16^3
    roots, 2 levels), one step in the launch configuration the benchmark
    times, on a seeded random tree (about 11 k leaves), FP64 and the FP32
    form.  Sampled cells (wall, pole, shock layer, wake, outer boundary) are
    recomputed by the FP64 oracle from their two-ring neighbourhood: FP64
    row by row to 1e-12, FP32 within 1e-5 of each row (its storage rounding
    is 6e-8)."""
    c = F.sphere()
    vs = c['vspace']
    t = random_tree(vs, 79, 1, p=0.25)
    assert 8000 < t.n < 16000
    gas = O.gas_from(c['gas'])
    cs = avs.Case(c['mesh'], vs, c['gas'], c['dt'], c['venkat_K'], c['prim0'], precision=prec, leaf_capacity=t.n)
    cs.set_leaves(t.level, t.idx)
    cs.step(1)
    nr, nth, nph = c['mesh']['shape']
    cell = lambda ir, it, ip: (ir * nth + it) * nph + ip
    sample = [cell(0, 0, 0), cell(0, 31, 5), cell(0, 63, 31), cell(10, 20, 17), cell(30, 32, 8),
              cell(40, 5, 30), cell(63, 0, 0), cell(63, 40, 12)]
    got = cs.get_cells(sample)
    Wg = cs.get_W()[sample]
    sub, keep = MM.submesh(c['mesh'], sample, halo=2)
    o = O.Solver(sub, vs, gas, c['dt'], c['venkat_K'], c['prim0'][keep])
    o.tree = t
    o.phi = o.initial_vdf(o.W)
    loc = [int(np.searchsorted(keep, i)) for i in sample]
    phi1, W1, _ = O.step(o.mesh, t, gas, c['dt'], c['venkat_K'], o.phi, o.W, cells=loc)
    if prec == 0:
        assert rel(got, phi1[:, loc]) < 1e-12
        assert tailrel(got, phi1[:, loc]) < 1e-6
        assert rel(Wg, W1[loc]) < 1e-13
    else:
        assert rel(got, phi1[:, loc]) < 1e-5
        assert rel(Wg, W1[loc]) < 1e-6
    cs.close()


# ------------------------------------------------------------ batched form --
@pytest.mark.parametrize("prec", [0, 1])
def test_batch_matches_single_cases_bit_for_bit(avs, prec):
    """Three different cases advanced by the batched kernels (eager and
    graph-replayed, odd and even step counts) hold exactly the state the
    same cases reach when advanced one by one."""
    import torch
    stream = torch.cuda.Stream()
    specs = []
    c = F.cavity(n=8, base=8, max_level=2)
    specs.append((c['mesh'], c['vspace'], c['gas'], c['dt'], 1.0, c['prim0'], random_tree(c['vspace'], 61, 2)))
    c = F.cylinder(nr=6, nth=24, Ma=2.0, box=8.0, base=16, max_level=2, r1=2.5, first=0.1)
    specs.append((c['mesh'], c['vspace'], c['gas'], c['dt'], 0.0, c['prim0'], resolved_tree(c['vspace'], 62)))
    mesh = MM.box2d(7, 5, periodic=(True, True))
    vs = dict(dim=2, lo=(-6, -6), hi=(6, 6), base=(8, 8), max_level=2)
    specs.append((mesh, vs, dict(R=1.0, Pr=2 / 3, omega=0.81, mu_ref=0.03, T_ref=1.0, model=1), 0.004, 1.0,
                  F.perturbed_uniform(mesh['ncells'], 2, 63, amp=0.1, uamp=0.4), random_tree(vs, 64, 2)))

    def build():
        out = []
        for mesh, vs, gas, dt, K, prim, tree in specs:
            cs = avs.Case(mesh, vs, gas, dt, K, prim, precision=prec, stream=stream)
            cs.set_leaves(tree.level, tree.idx)
            out.append(cs)
        return out
    with torch.cuda.stream(stream):
        solo, grouped = build(), build()
        batch = avs.Batch(grouped)
        for n, graph in ((3, False), (4, True), (4, True), (1, True)):
            for cs in solo:
                cs.step(n)
            batch.step(n, graph=graph)
            batch.check()
            for a, b in zip(solo, grouped):
                va, Wa = a.get_state()
                vb, Wb = b.get_state()
                assert np.array_equal(va, vb) and np.array_equal(Wa, Wb)
        # members stay usable on their own after batch steps
        for cs in grouped + solo:
            cs.adapt(0.01, 1e-6)
            cs.remap(2)
        batch.step(2)
        for cs in solo:
            cs.step(2)
        for a, b in zip(solo, grouped):
            assert np.array_equal(a.get_state()[0], b.get_state()[0])
        # batched adaptation and remap equal the per-case calls (per-case thresholds)
        C1 = [0.02, 1e-3, 0.005]
        nn_solo = []
        for cs, c1 in zip(solo, C1):
            nn_solo.append(cs.adapt(c1, math.exp(-8) * c1)[1])
            cs.remap(2)
        nn = batch.adapt(C1, [math.exp(-8) * c1 for c1 in C1])
        batch.remap(2)
        assert list(nn) == nn_solo
        for a, b in zip(solo, grouped):
            la, lb = a.leaves(), b.leaves()
            assert np.array_equal(la['level'], lb['level']) and np.array_equal(la['idx'], lb['idx'])
            va, Wa = a.get_state()
            vb, Wb = b.get_state()
            assert np.array_equal(va, vb) and np.array_equal(Wa, Wb)
        # every correction of the batched remap (0-2 span all members, 3-4 per member)
        for corr in (0, 1, 3, 4):
            batch.step(1)
            for cs in solo:
                cs.step(1)
            C1 = [0.01, 2e-3, 0.004]
            for cs, c1 in zip(solo, C1):
                cs.adapt(c1, math.exp(-8) * c1)
                cs.remap(corr)
            batch.adapt(C1, [math.exp(-8) * c1 for c1 in C1])
            batch.remap(corr)
            for a, b in zip(solo, grouped):
                va, Wa = a.get_state()
                vb, Wb = b.get_state()
                assert np.array_equal(va, vb) and np.array_equal(Wa, Wb), corr
        batch.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_3d_matches_single_cases_bit_for_bit(avs, prec):
    """Three 3-D cases (a box with walls, a small sphere grid, tetrahedra)
    advanced by the batched kernels through the captured graph, then one
    batched adaptation and the batched remap: states, leaf counts and leaves
    equal the same cases advanced one by one, bit for bit."""
    import torch
    stream = torch.cuda.Stream()
    specs = []
    mesh = MM.box3d(3, 3, 2, periodic=(True, False, True))
    vs = dict(dim=3, lo=(-5,) * 3, hi=(5,) * 3, base=(4,) * 3, max_level=1)
    specs.append((mesh, vs, dict(R=1.0, Pr=2 / 3, omega=0.74, mu_ref=0.05, T_ref=1.0, model=1), 0.004, 1.0,
                  F.perturbed_uniform(mesh['ncells'], 3, 9, amp=0.05, uamp=0.3), random_tree(vs, 6, 1, p=0.25)))
    c = F.sphere(nr=3, nth=4, nph=4, Ma=2.0, box=5.0, base=8, max_level=1, r1=1.5, first=0.2)
    specs.append((c['mesh'], c['vspace'], c['gas'], c['dt'], 0.0, c['prim0'], resolved_tree(c['vspace'], 6)))
    mesh = MM.tet_box(2, 2, 2, 51)
    vs = dict(dim=3, lo=(-5.0,) * 3, hi=(5.0,) * 3, base=(4, 4, 4), max_level=1)
    specs.append((mesh, vs, dict(R=1.0, Pr=2 / 3, omega=0.5, mu_ref=0.05, T_ref=1.0, model=1), 1e-3, 1.0,
                  F.perturbed_uniform(mesh['ncells'], 3, 52, amp=0.1, uamp=0.4), random_tree(vs, 53, 1)))

    def build():
        out = []
        for mesh, vs, gas, dt, K, prim, tree in specs:
            cs = avs.Case(mesh, vs, gas, dt, K, prim, precision=prec, stream=stream)
            cs.set_leaves(tree.level, tree.idx)
            out.append(cs)
        return out
    with torch.cuda.stream(stream):
        solo, grouped = build(), build()
        batch = avs.Batch(grouped)
        batch.step(3, graph=True)
        for cs in solo:
            cs.step(3)
        C1 = [1e-3, 2e-3, 5e-4]
        n0 = [cs.nleaves() for cs in grouped]
        nn_solo = []
        for cs, c1 in zip(solo, C1):
            nn_solo.append(cs.adapt(c1, math.exp(-8) * c1)[1])
            cs.remap(2)
        nn = batch.adapt(C1, [math.exp(-8) * c1 for c1 in C1])
        batch.remap(2)
        assert list(nn) == nn_solo and list(nn) != n0
        batch.step(2, graph=True)
        for cs in solo:
            cs.step(2)
        for a, b in zip(solo, grouped):
            la, lb = a.leaves(), b.leaves()
            assert np.array_equal(la['level'], lb['level']) and np.array_equal(la['idx'], lb['idx'])
            va, Wa = a.get_state()
            vb, Wb = b.get_state()
            assert np.array_equal(va, vb) and np.array_equal(Wa, Wb)
        batch.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_tuning_leaves_the_state_unchanged(avs, prec):
    """avs_batch_tune times its candidates on steps it does not take: the
    members' state (VDF, W, and the heat flux the next step's target uses)
    is bit for bit what it was, and tuned batched steps agree with the same
    cases advanced alone (to rounding: pass A's leaf chunk sets the order in
    which a face's moments are summed)."""
    import torch
    stream = torch.cuda.Stream()
    c = F.cavity(n=8, base=8, max_level=2)
    specs = [(c['mesh'], c['vspace'], c['gas'], c['dt'], 1.0, c['prim0'], random_tree(c['vspace'], 91, 2))]
    c = F.cylinder(nr=6, nth=24, Ma=2.0, box=8.0, base=16, max_level=2, r1=2.5, first=0.1)
    specs.append((c['mesh'], c['vspace'], c['gas'], c['dt'], 0.0, c['prim0'], resolved_tree(c['vspace'], 92)))
    with torch.cuda.stream(stream):
        solo, grouped = [], []
        for dst in (solo, grouped):
            for mesh, vs, gas, dt, K, prim, tree in specs:
                cs = avs.Case(mesh, vs, gas, dt, K, prim, precision=prec, stream=stream)
                cs.set_leaves(tree.level, tree.idx)
                cs.step(1)
                dst.append(cs)
        batch = avs.Batch(grouped)
        choice = batch.tune()
        assert len(choice) == 5 and choice[4] in (1, 2)
        for a, b in zip(solo, grouped):
            va, Wa = a.get_state()
            vb, Wb = b.get_state()
            assert np.array_equal(va, vb) and np.array_equal(Wa, Wb)
        batch.step(3, graph=True)
        for cs in solo:
            cs.step(3)
        for a, b in zip(solo, grouped):
            va, Wa = a.get_state()
            vb, Wb = b.get_state()
            if prec == 0:
                assert rel(vb, va) < 1e-12 and rel(Wb, Wa) < 1e-12
            else:
                assert rel(vb, va) < 1e-5 and rel(Wb, Wa) < 1e-6
        batch.close()


def _gap_thresholds(Mk, lo_q, hi_q, rgap):
    """C1, C2 halfway between neighbouring values of M_k with a relative
    gap above rgap, near the given quantiles (no leaf sits near either)."""
    m = np.sort(Mk)

    def gap(j):
        while not m[j + 1] - m[j] > rgap * m[j + 1]:
            j += 1
        return j
    j1, j2 = gap(int(hi_q * len(m))), gap(int(lo_q * len(m)))
    return 0.5 * (m[j1] + m[j1 + 1]), 0.5 * (m[j2] + m[j2 + 1])


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_members_match_the_oracle(avs, prec):
    """A mixed batch (cavity, cylinder, periodic box; different Kn, Ma and
    leaf counts) advanced by the batched kernels against the FP64 oracle
    advancing each case alone: FP64 members row by row to 1e-12, FP32
    members within 1e-5 field-normalised with FP64 totals; then one batched
    adaptation with per-case thresholds placed in gaps of the oracle's M_k:
    flags and leaf counts bit exact, and after the batched remap and two
    more batched steps the states again within the same tolerances."""
    import torch
    stream = torch.cuda.Stream()
    specs = []
    c = F.cavity(n=8, Kn=0.3, Ma=0.4, base=8, max_level=2)
    specs.append((c['mesh'], c['vspace'], c['gas'], c['dt'], 1.0, c['prim0'], random_tree(c['vspace'], 81, 2)))
    c = F.cylinder(nr=6, nth=24, Ma=3.0, Kn=0.05, box=8.0, base=16, max_level=2, r1=2.5, first=0.1)
    specs.append((c['mesh'], c['vspace'], c['gas'], c['dt'], 0.0, c['prim0'], resolved_tree(c['vspace'], 82)))
    mesh = MM.box2d(5, 4, periodic=(True, True))
    vs = dict(dim=2, lo=(-6, -6), hi=(6, 6), base=(4, 4), max_level=3)
    specs.append((mesh, vs, dict(R=1.0, Pr=2 / 3, omega=0.5, mu_ref=0.2, T_ref=1.0, model=1), 0.004, 1.0,
                  F.perturbed_uniform(mesh['ncells'], 2, 83, amp=0.1, uamp=0.4), random_tree(vs, 84, 3)))
    with torch.cuda.stream(stream):
        members, oracles = [], []
        for mesh, vs, gas, dt, K, prim, tree in specs:
            cs = avs.Case(mesh, vs, gas, dt, K, prim, precision=prec, stream=stream)
            cs.set_leaves(tree.level, tree.idx)
            o = O.Solver(mesh, vs, gas, dt, K, prim)
            o.tree = tree
            o.phi = o.initial_vdf(o.W)
            members.append(cs)
            oracles.append(o)
        assert len({cs.nleaves() for cs in members}) == len(members)
        batch = avs.Batch(members)

        def compare():
            for cs, o in zip(members, oracles):
                v, W = cs.get_state()
                if prec == 0:
                    assert rel(v, o.phi) < 1e-12 and rel(W, o.W) < 1e-12
                else:
                    f, tot = cs.moments()
                    assert fieldrel(f.cpu().numpy(), o.fields()) < 1e-5
                    ot = o.totals()
                    assert np.max(np.abs(tot - ot)) <= 1e-12 * np.max(np.abs(ot)) + 1e-5 * np.max(np.abs(ot))
        batch.step(3, graph=False)
        for o in oracles:
            o.step(3)
        compare()
        batch.step(2, graph=True)
        for o in oracles:
            o.step(2)
        compare()
        C1, C2 = [], []
        for o in oracles:
            Mk = O.criterion(o.phi, o.W, o.tree, o.gas.R)
            a, b = _gap_thresholds(Mk, 0.2, 0.85, 1e-9 if prec == 0 else 1e-4)
            C1.append(a)
            C2.append(b)
        nn = batch.adapt(C1, C2)
        nsplit = nmerge = 0
        for cs, o, a, b, n in zip(members, oracles, C1, C2, nn):
            eff, plan, _ = o.adapt(a, b)
            assert n == plan.tree.n
            kind, src, child = cs.plan(int(n))      # the plan follows from the effective flags
            assert np.array_equal(kind, plan.kind) and np.array_equal(src, plan.src)
            assert np.array_equal(child, plan.child)
            nsplit += int((eff == 1).sum())
            nmerge += int((eff == -1).sum())
        assert nsplit > 0 and nmerge > 0
        batch.remap(2)
        for o in oracles:
            o.remap(2)
        for cs, o in zip(members, oracles):
            lv = cs.leaves()
            assert np.array_equal(lv['level'], o.tree.level) and np.array_equal(lv['idx'], o.tree.idx)
        batch.step(2, graph=True)
        for o in oracles:
            o.step(2)
        compare()
        batch.close()


def test_degenerate_cases(avs):
    """Degenerate inputs: zero steps leave the state bit for bit and a
    residual over zero steps is refused; a velocity space without levels
    (4^2 roots, 16 leaves: one ragged chunk) steps like the oracle, and its
    adaptation can neither split (maximum level) nor merge (roots); an
    adaptation that flags nothing (C1 = inf, C2 = 0) keeps every leaf and
    its copy remap returns the state bit for bit."""
    c = F.cavity(n=8, base=4, max_level=0)
    cs, o = make_pair(avs, c['mesh'], c['vspace'], c['gas'], c['dt'], c['prim0'], Kv=1.0)
    assert cs.nleaves() == 16
    v0, W0 = cs.get_state()
    cs.step(0)
    v1, W1 = cs.get_state()
    assert np.array_equal(v0, v1) and np.array_equal(W0, W1)
    with pytest.raises(avs.AvsError):
        cs.step(0, residual=True)
    cs.step(2)
    o.step(2)
    v, W = cs.get_state()
    assert rel(v, o.phi) < 1e-12 and rel(W, o.W) < 1e-12
    flags, nn = cs.adapt(0.0, 1e300)         # every leaf over C1 and under C2
    assert nn == 16 and not flags.any()
    cs.remap(0)
    c = F.cavity(n=8, base=8, max_level=2)
    cs, o = make_pair(avs, c['mesh'], c['vspace'], c['gas'], c['dt'], c['prim0'],
                      tree=random_tree(c['vspace'], 71, 2), Kv=1.0)
    cs.step(1)
    v0, W0 = cs.get_state()
    n0 = cs.nleaves()
    flags, nn = cs.adapt(math.inf, 0.0)
    assert nn == n0 and not flags.any()
    cs.remap(0)
    v1, W1 = cs.get_state()
    assert np.array_equal(v0, v1) and np.array_equal(W0, W1)
    cs.close()


def test_full_batch_sampled_members(avs):
    """The batched workload at full size: the 64 seeded cases (cavities and
    cylinders, grids 32^2..96^2, FP32) on seeded random trees of 16^2 roots
    and 3 levels spanning the workload's leaf counts, tuned like the
    benchmark (pass-A chunk per bucket, pass-C leaves in flight), one step
    through the captured graph.  In every eighth member and the largest one,
    a wall or lid cell and an interior cell are recomputed by the FP64
    oracle from their two-ring neighbourhood: within 1e-5 of each row (the
    FP32 storage rounding is 6e-8), W within 1e-6."""
    import torch
    specs = F.batch_cases(seed=0, ncase=64)
    stream = torch.cuda.Stream()
    lo, hi = math.log(256.0), math.log(16384.0)
    with torch.cuda.stream(stream):
        members, trees = [], []
        for i, c in enumerate(specs):
            p = 0.05 + 0.85 * (math.log(c['target_leaves']) - lo) / (hi - lo)
            t = random_tree(c['vspace'], 900 + i, 3, p=p)
            cs = avs.Case(c['mesh'], c['vspace'], c['gas'], c['dt'], c['venkat_K'], c['prim0'], precision=1,
                          leaf_capacity=t.n, stream=stream)
            cs.set_leaves(t.level, t.idx)
            members.append(cs)
            trees.append(t)
        n = [t.n for t in trees]
        assert min(n) < 1000 and max(n) > 8000
        batch = avs.Batch(members)
        batch.tune()
        batch.step(1, graph=True)
        torch.cuda.synchronize()
        pick = sorted(set(range(0, 64, 8)) | {int(np.argmax(n))})
        for i in pick:
            c, cs, t = specs[i], members[i], trees[i]
            m = c['mesh']
            lr = np.asarray(m['face_lr'])
            wall = int(lr[lr[:, 1] == -1, 0][0])
            sample = sorted({wall, m['ncells'] // 2 + 3})
            got = cs.get_cells(sample)
            Wg = cs.get_W()[sample]
            sub, keep = MM.submesh(m, sample, halo=2)
            gas = O.gas_from(c['gas'])
            o = O.Solver(sub, c['vspace'], gas, c['dt'], c['venkat_K'], c['prim0'][keep])
            o.tree = t
            o.phi = o.initial_vdf(o.W)
            loc = [int(np.searchsorted(keep, j)) for j in sample]
            phi1, W1, _ = O.step(o.mesh, t, gas, c['dt'], c['venkat_K'], o.phi, o.W, cells=loc)
            assert rel(got, phi1[:, loc]) < 1e-5, (i, c['geometry'], t.n)
            assert rel(Wg, W1[loc]) < 1e-6, (i, c['geometry'], t.n)
        batch.close()
        for cs in members:
            cs.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_fine_velocity_grids_beyond_64_kib_of_lds(avs, dim):
    """Velocity grids whose per-axis Maxwellian tables need more than the
    default 64 KiB of LDS per workgroup in pass C (2-D: 2 x 16 x 2^5 = 1024
    half-finest points per axis, 80 KiB; 3-D: 2 x 8 x 2^5 = 512, 86 KiB) step
    like the oracle (1e-12 per step); a grid beyond gfx950's 160 KiB is
    refused at set-up."""
    if dim == 2:
        mesh = MM.box2d(3, 2, periodic=(True, True))
        vs = dict(dim=2, lo=(-6.0, -6.0), hi=(6.0, 6.0), base=(16, 16), max_level=5)
    else:
        mesh = MM.box3d(2, 2, 2, periodic=(True, True, True))
        vs = dict(dim=3, lo=(-5.0,) * 3, hi=(5.0,) * 3, base=(8, 8, 8), max_level=5)
    gas = dict(R=1.0, Pr=2 / 3, omega=0.81, mu_ref=0.05, T_ref=1.0, model=1)
    prim = F.perturbed_uniform(mesh['ncells'], dim, 17, amp=0.05, uamp=0.3)
    tree = random_tree(vs, 18, 2, p=0.03)
    cs, o = make_pair(avs, mesh, vs, gas, 2e-3, prim, tree=tree, noise=0.01, seed=19, cap=4096)
    cs.step(2)
    o.step(2)
    v, W = cs.get_state()
    assert rel(v, o.phi) < 1e-12 and rel(W, o.W) < 1e-12
    cs.close()
    if dim == 2:
        too_fine = dict(dim=2, lo=(-6.0, -6.0), hi=(6.0, 6.0), base=(32, 32), max_level=6)
        with pytest.raises(avs.AvsError, match="too fine"):
            avs.Case(mesh, too_fine, gas, 2e-3, 1.0, prim, leaf_capacity=4096)
