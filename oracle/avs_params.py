"""Plain CPU oracle of the adaptive-parameter configuration and of the
step-0 velocity space (Sec. 3.5 of arXiv 2212.05645).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no
code with the GPU library and imports nothing from it; the tree operations
of the step-0 build come from ``oracle.avs_oracle``.

What it computes, from the freestream (Ma, T_inf, rho_inf, direction), the
wall temperature and the gas (R, gamma):

* the three standard deviations sigma_inf, sigma_0, sigma_w = sqrt(R T) of
  the freestream, total and wall temperatures, with the total temperature
  of Eq. totaltemperature;
* the velocity domain: a square (cube) of half-width R_dv = k sigma_0
  (k = 4, or more for hot walls) centred at 0.4 U_inf;
* the levels: L_max = the smallest L with 2^L >= 2 R_dv / h_std (h_std =
  0.6), the finest interval h_inf = 2 R_dv / 2^L_max, the wall level L_w
  (L_max, or L_max - 1 when T_w / T_inf >= 4), the minimum level L_min (4
  for D = 2 above Ma 5, else 3) and the separated-zone level
  max(L_min, L_w - 1);
* the thresholds C1 = 13.749 Ma^-1.465 (Eq. C1_Ma) and C2 = k_sigma C1 with
  k_sigma = f(4) / f(0) of the standard normal density (Eq. c2c1; the
  printed value 3.3546e-4 is this ratio, the formula beside it is written
  the other way up);
* the step-0 velocity space: one element of half-width R_dv split L_w - 1
  times, then one adaptation whose criterion runs over the freestream and
  the static state (rho_inf, 0, T_inf) only;
* for a flow that separates, the separated zone: elements whose discrete
  velocity lies in 3 sigma_w < |xi| < 5 sigma_w keep at least L_sep
  (a floor on the flags of every adaptation, ``avs_oracle.separated_floor``).

Mapping onto the forest of the solver (Sec. 3.1 reading: level-0 roots that
never merge): the paper's single root with levels L_min..L_max is a forest
of 2^L_min roots per axis with L_max - L_min levels below them (when L_max
< L_min the roots sit at L_max and no level is added).  A uniform split
count below L_min gives the roots themselves.

Pinned by the values the paper prints (tests/golden): the L_max column of
the cylinder table, the h_inf column of the sphere table, the C1 values the
runs quote from Eq. C1_Ma, the normal-density constants and the sphere's
total temperatures.  The separated-zone floor is pinned by hand-counted
trees (which centre decides, split below the level, merge kept) and by the
invariant it guarantees.  Parity unpinned: the element counts of the step-0
space (they depend on the normalisation of the criterion against C1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import avs_oracle as O

H_STD = 0.6          # standard velocity interval (Sec. 3.5)


@dataclass
class Flow:
    dim: int
    R: float
    gamma: float
    Ma: float
    T_inf: float
    T_wall: float
    rho_inf: float = 1.0
    direction: tuple = (1.0, 0.0, 0.0)   # unit vector of the freestream velocity
    rdv_sigmas: float = 4.0              # R_dv in units of sigma_0
    h_std: float = H_STD
    separated: bool = False              # the flow separates: refine the separated zone


def total_temperature(T_inf, gamma, Ma):
    """Eq. totaltemperature: T_0 = T_inf (1 + (gamma - 1) / 2 Ma^2)."""
    return T_inf * (1.0 + 0.5 * (gamma - 1.0) * Ma * Ma)


def sound_speed(R, gamma, T):
    """a = sqrt(gamma R T) (Sec. 4.2 quotes a this way)."""
    return math.sqrt(gamma * R * T)


def standard_deviation(R, T):
    """sigma = sqrt(R T): the standard deviation of a Maxwellian per axis
    (Sec. 3.5, comparing Eqs. Maxwell_df and Normal_df)."""
    return math.sqrt(R * T)


def level_std(R_dv, h_std=H_STD):
    """The smallest level L with 2^L >= 2 R_dv / h_std (Sec. 3.5)."""
    need = 2.0 * R_dv / h_std
    L = 0
    while 2.0 ** L < need:
        L += 1
    return L


def wall_level(L_max, T_wall, T_inf):
    """L_w = L_max if T_w / T_inf < 4, else L_max - 1 (Sec. 3.5)."""
    return L_max if T_wall / T_inf < 4.0 else L_max - 1


def min_level(dim, Ma):
    """L_min = 4 for D = 2 and Ma > 5, otherwise 3 (Sec. 3.5)."""
    return 4 if (dim == 2 and Ma > 5.0) else 3


def normal_pdf(x):
    """Standard normal density (Eq. Normal_df_std)."""
    return math.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def k_sigma():
    """C2 / C1 = f(4 sigma) / f(0) of the standard normal density (Eq. c2c1)."""
    return normal_pdf(4.0) / normal_pdf(0.0)


def c1_of_ma(Ma):
    """Eq. C1_Ma: C1 = 13.749 Ma^-1.465 (infinite at Ma = 0: nothing splits)."""
    return math.inf if Ma == 0.0 else 13.749 * Ma ** -1.465


def auto_params(flow: Flow):
    """Every adaptive parameter of Sec. 3.5 for one freestream."""
    D = flow.dim
    T0 = total_temperature(flow.T_inf, flow.gamma, flow.Ma)
    s_inf = standard_deviation(flow.R, flow.T_inf)
    s_0 = standard_deviation(flow.R, T0)
    s_w = standard_deviation(flow.R, flow.T_wall)
    U_inf = flow.Ma * sound_speed(flow.R, flow.gamma, flow.T_inf)
    e = np.asarray(flow.direction, np.float64)[:D]
    R_dv = flow.rdv_sigmas * s_0
    centre = 0.4 * U_inf * e
    L_max = level_std(R_dv, flow.h_std)
    h_min = 2.0 * R_dv / 2.0 ** L_max
    L_w = wall_level(L_max, flow.T_wall, flow.T_inf)
    L_min = min_level(D, flow.Ma)
    L_sep = max(L_min, L_w - 1)
    C1 = c1_of_ma(flow.Ma)
    ks = k_sigma()
    return dict(T0=T0, sigma_inf=s_inf, sigma_0=s_0, sigma_w=s_w, U_inf=U_inf, R_dv=R_dv, centre=centre,
                L_max=L_max, h_min=h_min, L_w=L_w, L_min=L_min, L_sep=L_sep, C1=C1, k_sigma=ks, C2=ks * C1)


def vspace_of(p, dim):
    """The solver's velocity box and forest for the parameters ``p``: roots
    at level min(L_min, L_max) (2^that per axis), L_max - that levels below."""
    lr = min(p['L_min'], p['L_max'])
    lo = p['centre'] - p['R_dv']
    hi = p['centre'] + p['R_dv']
    return dict(dim=dim, lo=lo, hi=hi, base=(1 << lr,) * dim, max_level=p['L_max'] - lr)


def separated_zone(p):
    """The separated zone of Sec. 3.5 on the solver's forest: the annulus
    3 sigma_w < |xi| < 5 sigma_w about the origin (the wall is at rest) and
    its level L_sep relative to the roots at min(L_min, L_max)."""
    lr = min(p['L_min'], p['L_max'])
    return (3.0 * p['sigma_w'], 5.0 * p['sigma_w'], p['L_sep'] - lr)


def uniform_tree(vs, level):
    """Every cell of the forest at ``level`` (relative to the roots), in
    depth-first order."""
    D = vs['dim']
    n = np.asarray(vs['base'], np.int64) << level
    grids = np.meshgrid(*[np.arange(m) for m in n], indexing='ij')
    idx = np.stack([g.ravel() for g in grids], 1).astype(np.int64)
    t = O.Tree(D, np.asarray(vs['lo'], np.float64), np.asarray(vs['hi'], np.float64),
               np.asarray(vs['base'], np.int64), int(vs['max_level']), np.full(len(idx), level, np.int64), idx)
    return t.sorted()


def probe_states(flow: Flow, p):
    """The freestream W_inf = (rho_inf, U_inf e, T_inf) and the static state
    W_0 = (rho_inf, 0, T_inf) of the step-0 adaptation, as primitive rows."""
    D = flow.dim
    e = np.asarray(flow.direction, np.float64)[:D]
    w_inf = np.concatenate([[flow.rho_inf], p['U_inf'] * e, [flow.T_inf]])
    w_0 = np.concatenate([[flow.rho_inf], np.zeros(D), [flow.T_inf]])
    return np.stack([w_inf, w_0])


def initial_tree(flow: Flow, p=None, C1=None, C2=None):
    """The step-0 velocity space of Sec. 3.5: one element of half-width R_dv
    centred at 0.4 U_inf, split L_w - 1 times, then one adaptation over the
    two probe states only (no cell contributes; for a separating flow the
    separated zone's level is a floor on its flags).  C1 and C2 default to the
    fit of Eq. C1_Ma and k_sigma C1; with the criterion as printed (M_k at
    most the mass fraction of one element) that C1 never splits, so callers
    pass the threshold their normalisation needs.
    Returns (tree after the uniform splits, effective flags, final tree)."""
    p = auto_params(flow) if p is None else p
    C1 = p['C1'] if C1 is None else C1
    C2 = p['k_sigma'] * C1 if C2 is None else C2
    vs = vspace_of(p, flow.dim)
    lr = min(p['L_min'], p['L_max'])
    level = min(max(p['L_w'] - 1 - lr, 0), vs['max_level'])
    t0 = uniform_tree(vs, level)
    P = 2 if flow.dim == 2 else 1
    no_cells = np.zeros((P, 0, t0.n))
    Mk = O.criterion(no_cells, np.zeros((0, flow.dim + 2)), t0, flow.R, probes=probe_states(flow, p))
    raw = O.raw_flags(Mk, t0, C1, C2)
    if flow.separated:
        raw = O.separated_floor(raw, t0, separated_zone(p))
    eff = O.resolve_merges(raw, t0)
    return t0, eff, O.make_plan(eff, t0).tree
