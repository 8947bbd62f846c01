"""Seeded synthetic macroscopic states and workload configurations.

Inputs only: primitive fields ``(rho, U_1..U_D, T)`` per cell, shaped like the
flows of the paper's test cases (Sec. 4: lid-driven cavity, supersonic
cylinder, supersonic sphere), and the physical/velocity-space parameters of
each workload.  Nothing here evaluates a distribution function, a moment or a
gas-model relation: the conversion to conserved variables and the viscosity
law belong to the two implementations that consume these inputs.
The published flow solutions are not available, so smooth analytic stand-ins
with seeded perturbations are used.
"""
from __future__ import annotations

import math

import numpy as np

from . import meshes


def prim(rho, U, T):
    """Stack primitive fields into rows ``(rho, U_1..U_D, T)``."""
    rho = np.asarray(rho, np.float64)
    U = np.asarray(U, np.float64)
    T = np.asarray(T, np.float64)
    rho, T = np.broadcast_arrays(rho, T)
    return np.concatenate([rho[..., None], np.broadcast_to(U, rho.shape + U.shape[-1:]), T[..., None]], axis=-1)


def uniform(ncells, rho, U, T):
    return prim(np.full(ncells, rho), np.asarray(U, np.float64), np.full(ncells, T))


def perturbed_uniform(ncells, dim, seed, amp=0.05, uamp=0.3):
    """Unit state with seeded cell-wise random perturbations of rho, U and T."""
    rng = np.random.default_rng(seed)
    rho = 1.0 + amp * rng.uniform(-1, 1, ncells)
    U = uamp * rng.uniform(-1, 1, (ncells, dim))
    T = 1.0 + amp * rng.uniform(-1, 1, ncells)
    return prim(rho, U, T)


def normal_shock(Ma, gamma=5.0 / 3.0):
    """Rankine-Hugoniot ratios (rho2/rho1, u2/u1, T2/T1) across a normal shock."""
    m2 = Ma * Ma
    rr = (gamma + 1) * m2 / ((gamma - 1) * m2 + 2)
    pr = 1 + 2 * gamma / (gamma + 1) * (m2 - 1)
    return rr, 1.0 / rr, pr / rr


def blunt_body_field(ctr, radius, Ma, R, T_inf=1.0, rho_inf=1.0, seed=0, amp=0.02, gamma=5.0 / 3.0):
    """Bow-shock shaped blend of freestream, post-shock and wake states.

    Flow along +x around a body of ``radius`` at the origin (2-D or 3-D; the
    distance from the x-axis is used).  Billig-type hyperbolic shock shape,
    tanh transitions, and seeded +-``amp`` perturbations of rho and T.
    Returns ``(prim, probes)`` where ``probes`` are the four reference states
    (freestream, static, post-shock, wake) as primitive rows.
    """
    rng = np.random.default_rng(seed)
    D = ctr.shape[1]
    U_inf = Ma * math.sqrt(gamma * R * T_inf)
    rr, ur, Tr = normal_shock(max(Ma, 1.0), gamma)
    x = ctr[:, 0]
    y = np.sqrt(np.sum(ctr[:, 1:] ** 2, axis=1))
    if Ma <= 1.05:                       # subsonic: no bow shock, freestream plus wake
        Ma_s = 1.05
    else:
        Ma_s = Ma
    standoff = radius * 0.386 * math.exp(4.67 / (Ma_s * Ma_s))
    Rc = radius * 1.386 * math.exp(1.8 / max(Ma_s - 1.0, 0.3) ** 0.75)
    beta = math.asin(min(1.0, 1.0 / Ma_s))
    xs = -(radius + standoff) + Rc / math.tan(beta) ** 2 * (np.sqrt(1 + (y * math.tan(beta) / Rc) ** 2) - 1)
    a_sh = 0.5 * (1 + np.tanh((xs - x) / (0.05 * radius)))           # 1 upstream of shock
    if Ma <= 1.05:
        a_sh = np.where(x < 0, 1.0, a_sh)
    wake = 0.5 * (1 + np.tanh(x / (0.5 * radius))) * np.exp(-(y / (radius * (1.2 + 0.15 * np.maximum(x, 0)))) ** 2)
    rho_ps, T_ps, u_ps = rho_inf * rr, T_inf * Tr, U_inf * ur
    rho_w, T_w, u_w = 0.3 * rho_inf, 0.6 * T_ps, 0.2 * U_inf
    rho = a_sh * rho_inf + (1 - a_sh) * ((1 - wake) * rho_ps + wake * rho_w)
    T = a_sh * T_inf + (1 - a_sh) * ((1 - wake) * T_ps + wake * T_w)
    u = a_sh * U_inf + (1 - a_sh) * ((1 - wake) * u_ps + wake * u_w)
    rho = rho * (1 + amp * rng.uniform(-1, 1, len(x)))
    T = T * (1 + amp * rng.uniform(-1, 1, len(x)))
    U = np.zeros((len(x), D))
    U[:, 0] = u
    e0 = np.zeros(D)
    e0[0] = 1.0
    probes = np.stack([prim(rho_inf, U_inf * e0, T_inf), prim(rho_inf, 0 * e0, T_inf),
                       prim(rho_ps, u_ps * e0, T_ps), prim(rho_w, u_w * e0, T_w)])
    return prim(rho, U, T), probes


# ---------------------------------------------------------------------------
# Workload configurations (shapes of the paper's test cases)
# ---------------------------------------------------------------------------

def cavity(n=32, Ma=0.16, Kn=0.075, omega=0.5, box=5.0, base=16, max_level=2, C1=0.01, cfl=0.8):
    """2-D lid-driven cavity on the unit square (Sec. 4.2 shape), units sqrt(R T0), R=1."""
    R, T0, gamma = 1.0, 1.0, 5.0 / 3.0
    Uw = Ma * math.sqrt(gamma * R * T0)
    mesh = meshes.box2d(n, n, sides={'left': 0, 'right': 0, 'bottom': 0, 'top': 1},
                        bcs=[(meshes.WALL, (1.0, 0.0, 0.0, T0)), (meshes.WALL, (1.0, Uw, 0.0, T0))])
    W0 = uniform(mesh['ncells'], 1.0, (0.0, 0.0), T0)
    probes = np.stack([prim(1.0, (Uw, 0.0), T0), prim(1.0, (0.0, 0.0), T0)])
    dt = _cfl_dt(mesh, cfl, box)
    return dict(name='cavity', dim=2, mesh=mesh, prim0=W0, probes=probes,
                vspace=dict(dim=2, lo=(-box, -box), hi=(box, box), base=(base, base), max_level=max_level),
                gas=dict(R=R, Pr=2.0 / 3.0, omega=omega, Kn=Kn, L_ref=1.0, rho_ref=1.0, T_ref=T0, model=1),
                dt=dt, venkat_K=1.0, C1=C1, C2=math.exp(-8.0) * C1, nu=20, steps=200)


def cylinder(nr=128, nth=256, Ma=5.0, Kn=0.1, omega=0.81, box=15.0, base=32, max_level=3, C1=2e-4, cfl=0.8, seed=0,
             r1=15.0, first=0.01):
    """2-D supersonic flow past a cylinder (Sec. 4.1 shape), units sqrt(R Tinf) with R=1/2."""
    R, Tinf, gamma = 0.5, 1.0, 5.0 / 3.0
    mesh = meshes.ogrid(nr, nth, r0=0.5, r1=r1, first=first)
    U_inf = Ma * math.sqrt(gamma * R * Tinf)
    mesh['bc_state'][0] = (1.0, 0.0, 0.0, Tinf)
    mesh['bc_state'][1] = (1.0, U_inf, 0.0, Tinf)
    W0, probes = blunt_body_field(mesh['cell_ctr'], 0.5, Ma, R, Tinf, seed=seed)
    dt = _cfl_dt(mesh, cfl, box)
    return dict(name='cylinder', dim=2, mesh=mesh, prim0=W0, probes=probes,
                vspace=dict(dim=2, lo=(-box, -box), hi=(box, box), base=(base, base), max_level=max_level),
                gas=dict(R=R, Pr=2.0 / 3.0, omega=omega, Kn=Kn, L_ref=1.0, rho_ref=1.0, T_ref=Tinf, model=1),
                dt=dt, venkat_K=0.0, C1=C1, C2=math.exp(-8.0) * C1, nu=20, steps=100)


def sphere(nr=64, nth=64, nph=32, Ma=4.0, Kn=0.05, omega=0.74, box=12.0, base=16, max_level=2, C1=2e-5, cfl=0.8, seed=0,
           r1=8.0, first=0.02):
    """3-D supersonic flow past a sphere (Sec. 4.6 shape), monatomic, R=1/2."""
    R, Tinf, gamma = 0.5, 1.0, 5.0 / 3.0
    U_inf = Ma * math.sqrt(gamma * R * Tinf)
    mesh = meshes.sphere_grid(nr, nth, nph, r0=0.5, r1=r1, first=first,
                              wall_state=(1.0, 0.0, 0.0, 0.0, Tinf), far_state=(1.0, U_inf, 0.0, 0.0, Tinf))
    W0, probes = blunt_body_field(mesh['cell_ctr'], 0.5, Ma, R, Tinf, seed=seed)
    dt = _cfl_dt(mesh, cfl, box)
    return dict(name='sphere', dim=3, mesh=mesh, prim0=W0, probes=probes,
                vspace=dict(dim=3, lo=(-box,) * 3, hi=(box,) * 3, base=(base,) * 3, max_level=max_level),
                gas=dict(R=R, Pr=2.0 / 3.0, omega=omega, Kn=Kn, L_ref=1.0, rho_ref=1.0, T_ref=Tinf, model=1),
                dt=dt, venkat_K=0.0, C1=C1, C2=math.exp(-8.0) * C1, nu=20, steps=50)


def _cfl_dt(mesh, cfl, xmax):
    """Explicit time step: cfl * min_i V_i / (1/2 sum_f A_f sum_d |n_fd| xmax_d).

    The denominator bounds, for every velocity node of the box (|xi_d| <=
    xmax_d), the outflow rate sum_out A_f xi.n_f of a closed cell (outflow
    and inflow areas balance, so the outflow is half of sum_f A_f |xi.n_f|).
    At cfl <= 1 the first-order upwind update keeps every node positive,
    also at the corners of the box, where a one-dimensional bound would
    allow a CFL up to D times larger."""
    nc, D = mesh['ncells'], mesh['dim']
    xm = np.broadcast_to(np.asarray(xmax, dtype=float), (D,))
    lr = mesh['face_lr']
    rate = mesh['face_area'] * (np.abs(mesh['face_nrm']) @ xm)
    out = np.zeros(nc)
    np.add.at(out, lr[:, 0], rate)
    inner = lr[:, 1] >= 0
    np.add.at(out, lr[inner, 1], rate[inner])
    return cfl * float(np.min(mesh['cell_vol'] / (0.5 * out)))


def batch_cases(seed=0, ncase=64):
    """Independent 2-D cases for the batched form: Kn log-uniform in
    [1e-3, 1], Ma uniform in [0.1, 6], cavity or cylinder with equal
    probability, grid side uniform in {32..96}, quadtree with 16^2 roots and
    3 levels, target step-0 leaf count log-uniform in [256, 16384].  Cylinder
    velocity boxes follow the paper's sizing (Sec. 3.5): radius 4 sigma_0 with
    T0 = Tinf (1 + (gamma-1)/2 Ma^2), centred at (0.4 Uinf, 0)."""
    rng = np.random.default_rng(seed)
    out = []
    for c in range(ncase):
        Kn = 10.0 ** rng.uniform(-3.0, 0.0)
        Ma = rng.uniform(0.1, 6.0)
        geo = 'cavity' if rng.random() < 0.5 else 'cylinder'
        side = int(rng.integers(32, 97))
        target = int(round(10.0 ** rng.uniform(math.log10(256), math.log10(16384))))
        if geo == 'cavity':
            lid = Ma * math.sqrt(5.0 / 3.0)
            cfg = cavity(n=side, Ma=Ma, Kn=Kn, omega=0.5, box=5.0 + lid, base=16, max_level=3)
        else:
            gamma, R = 5.0 / 3.0, 0.5
            T0 = 1.0 + 0.5 * (gamma - 1.0) * Ma * Ma
            rdv = 4.0 * math.sqrt(R * T0)
            cx = 0.4 * Ma * math.sqrt(gamma * R)
            cfg = cylinder(nr=side, nth=side, Ma=Ma, Kn=Kn, box=rdv, base=16, max_level=3, seed=seed * 1000 + c)
            cfg['vspace'] = dict(dim=2, lo=(cx - rdv, -rdv), hi=(cx + rdv, rdv), base=(16, 16), max_level=3)
            cfg['dt'] = _cfl_dt(cfg['mesh'], 0.8, (abs(cx) + rdv, rdv))
        cfg.update(case=c, Kn=Kn, Ma=Ma, geometry=geo, side=side, target_leaves=target)
        out.append(cfg)
    return out


def wedge_flow(Ma=8.1):
    """Freestream of the hypersonic blunt-wedge case (Sec. 4.3 shape):
    argon (gamma 5/3), units sqrt(R T_inf) with R = 1/2, wall at 273 K
    against a 189 K freestream, flow along +x."""
    return dict(dim=2, R=0.5, gamma=5.0 / 3.0, Ma=Ma, T_inf=1.0, T_wall=273.0 / 189.0)


def blunt_wedge(vspace, Ma=8.1, Kn=0.338, omega=0.81, C1=1e-3, cfl=0.8, seed=0, **mesh_kw):
    """2-D hypersonic flow over a blunt wedge on an unstructured triangle
    mesh (Sec. 4.3 shape: nose radius 1, half angle 10 deg, base height
    3.736 nose radii, about 11 900 cells; Kn 0.338 on the nose radius).
    ``vspace`` is the velocity space (the automatic one of Sec. 3.5 for
    ``wedge_flow(Ma)`` in the paper's run); the time step follows from it."""
    fl = wedge_flow(Ma)
    R, Tinf, gamma = fl['R'], fl['T_inf'], fl['gamma']
    mesh = meshes.blunt_wedge(seed=seed, **mesh_kw)
    U_inf = Ma * math.sqrt(gamma * R * Tinf)
    mesh['bc_state'][0] = (1.0, 0.0, 0.0, fl['T_wall'])
    mesh['bc_state'][1] = (1.0, U_inf, 0.0, Tinf)
    # the nose circle is centred one radius behind the tip
    W0, probes = blunt_body_field(mesh['cell_ctr'] - np.array([1.0, 0.0]), 1.0, Ma, R, Tinf, seed=seed)
    lo, hi = np.asarray(vspace['lo'], np.float64), np.asarray(vspace['hi'], np.float64)
    dt = _cfl_dt(mesh, cfl, np.maximum(np.abs(lo), np.abs(hi)))
    return dict(name='blunt_wedge', dim=2, mesh=mesh, prim0=W0, probes=probes, vspace=dict(vspace), flow=fl,
                gas=dict(R=R, Pr=2.0 / 3.0, omega=omega, Kn=Kn, L_ref=1.0, rho_ref=1.0, T_ref=Tinf, model=1),
                dt=dt, venkat_K=0.0, C1=C1, C2=math.exp(-8.0) * C1, nu=20, steps=50)
