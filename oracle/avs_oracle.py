"""Plain FP64 CPU oracle of the global adaptive-velocity-space (AVS) sweep.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no
code with the GPU library and imports nothing from it.

What it computes (paper: Chen, Liu, Zhang, Zhong, Yang, Zhuo, "A global
adaptive velocity space for general discrete velocity framework", arXiv
2212.05645):

* reduced distributions G, H of a monatomic gas (Sec. 2.2, Eq. equ6); in 3-D
  only G (H vanishes for D = 3, K = 0, Eq. equ16);
* moments W = (rho, rho U, rho E) and heat flux q (Eqs. updat_W, equ8),
  Maxwellian and Shakhov equilibria (Eqs. Maxwell_df, equ14-equ17), VHS
  relaxation time (Eq. equ3) with the reference viscosity of Eq. equ4;
* one time step of the discrete-velocity scheme of Sec. 2.3 in its explicit
  limit (implicit flux increments set to zero in Eqs. equ_delw and
  delta_phi): least-squares gradient and Venkatakrishnan limiter, upwind
  Taylor reconstruction at x_ij - xi h, interface moments and equilibrium
  (Eq. w_interface), characteristic-line interface VDF (Eq. equ28),
  macroscopic finite-volume update (Eq. equ18), point-implicit relaxation
  towards the conservative Shakhov target;
* velocity-tree adaptation of Sec. 3: forest of quadtrees/octrees (Sec. 3.1),
  criterion M1/M2 and split/merge rules (Sec. 3.4, Eqs. criterion_rho,
  criterion_e, criterion_mk), "consanguinity" remap (Sec. 3.2) and the
  conservation correction f = f' + g(W) - g(W') (Sec. 3.3).

Where the paper leaves a point open, the docstring states the reading
taken; each function below names the passage it follows.

Parity unpinned (readings that no closed form, invariant or printed value
of the paper can check; both implementations share them as conventions):
the interface heat-flux factor tau/(tau + h Pr) in ``face_vdf``, the
Venkatakrishnan constant K of ``venkat_psi`` (eps^2 = (K V^(1/D))^3), the
wall and far-field treatment of incoming leaves in ``face_vdf`` beyond zero
net mass flux, and the threshold C1 of ``raw_flags``.  Every array is float64.
Nothing here is blocked, fused or reordered for speed: loops run over cells
and faces, NumPy vectorises over the velocity axis only.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

WALL = 0
FARFIELD = 1
COPY, SPLIT, MERGE = 0, 1, 2


# ---------------------------------------------------------------------------
# Velocity tree (Sec. 3.1) -- forest of level-0 roots; leaves are the mesh
# ---------------------------------------------------------------------------

@dataclass
class Tree:
    """Leaves of a forest of quadtrees (D=2) / octrees (D=3).

    ``base[d]`` level-0 roots per axis over the box ``[lo, hi]``; a leaf at
    level ``l`` has integer index ``idx`` in the uniform grid of
    ``base * 2**l`` cells per axis.  Leaves are kept in depth-first order
    (Morton order of their lower corner on the finest grid), which places a
    parent exactly where its first child was.
    """
    dim: int
    lo: np.ndarray
    hi: np.ndarray
    base: np.ndarray
    max_level: int
    level: np.ndarray            # int64 [Nv]
    idx: np.ndarray              # int64 [Nv, D]

    @property
    def n(self):
        return len(self.level)

    def widths(self):
        """Per-leaf cell widths h_d = (hi_d - lo_d) / (base_d 2^level)."""
        cnt = self.base[None, :].astype(np.int64) << self.level[:, None]
        return (self.hi - self.lo)[None, :] / cnt.astype(np.float64)

    def centres(self):
        """Quadrature points: the centres of the leaf cells (Sec. 3, mid-point rule)."""
        return self.lo[None, :] + (self.idx.astype(np.float64) + 0.5) * self.widths()

    def weights(self):
        """Quadrature weights: leaf area (2-D) / volume (3-D) (Sec. 3, mid-point rule)."""
        h = self.widths()
        a = h[:, 0] * h[:, 1]
        if self.dim == 3:
            a = a * h[:, 2]
        return a

    def morton(self):
        """Interleaved bits of the lower corner on the finest grid (x lowest)."""
        X = self.idx << (self.max_level - self.level)[:, None]
        key = np.zeros(self.n, dtype=np.uint64)
        for b in range(64 // self.dim):
            for d in range(self.dim):
                key |= ((X[:, d] >> b) & 1).astype(np.uint64) << np.uint64(self.dim * b + d)
        return key

    def sorted(self):
        o = np.argsort(self.morton(), kind='stable')
        return Tree(self.dim, self.lo, self.hi, self.base, self.max_level, self.level[o], self.idx[o])


def base_forest(dim, lo, hi, base, max_level):
    """The level-0 roots (they split but never merge, Sec. 3.1)."""
    base = np.asarray(base, np.int64)[:dim]
    grids = np.meshgrid(*[np.arange(b) for b in base], indexing='ij')
    idx = np.stack([g.ravel() for g in grids], 1).astype(np.int64)
    t = Tree(dim, np.asarray(lo, np.float64)[:dim], np.asarray(hi, np.float64)[:dim], base, int(max_level),
             np.zeros(len(idx), np.int64), idx)
    return t.sorted()


# ---------------------------------------------------------------------------
# Gas model (Sec. 2.1-2.2)
# ---------------------------------------------------------------------------

@dataclass
class Gas:
    R: float
    Pr: float
    omega: float
    mu_ref: float
    T_ref: float
    model: int = 1               # 0 BGK, 1 Shakhov
    law: int = 0                 # viscosity: 0 power law (VHS, Eq. equ3), 1 Sutherland (Eq. Sutherland)
    C_s: float = 0.0             # Sutherland constant, in the units of T


def mu_ref_from_kn(Kn, omega, R, T_ref=1.0, rho_ref=1.0, L_ref=1.0):
    """mu that gives lambda = Kn L_ref at the reference state (Eqs. equ4, equ5)."""
    return Kn * L_ref * 15.0 * rho_ref * math.sqrt(2.0 * math.pi * R * T_ref) / (2.0 * (5.0 - 2.0 * omega) * (7.0 - 2.0 * omega))


def conserved(prim, R):
    """(rho, U, T) -> W = (rho, rho U, rho E), rho E = rho|U|^2/2 + 3/2 rho R T (Eq. updat_W)."""
    prim = np.asarray(prim, np.float64)
    D = prim.shape[-1] - 2
    rho = prim[..., 0]
    U = prim[..., 1:1 + D]
    T = prim[..., 1 + D]
    ke = 0.5 * rho * np.sum(U * U, axis=-1)
    out = np.empty(prim.shape)
    out[..., 0] = rho
    out[..., 1:1 + D] = rho[..., None] * U
    out[..., 1 + D] = ke + 1.5 * rho * R * T
    return out


def primitive(W, R):
    """W -> (rho, U, T) for a monatomic gas (internal energy 3/2 rho R T)."""
    D = len(W) - 2
    rho = W[0]
    U = W[1:1 + D] / rho
    T = (W[1 + D] - 0.5 * rho * np.dot(U, U)) / (1.5 * rho * R)
    return rho, U, T


def viscosity(T, gas):
    """mu(T): power law mu_ref (T/T_ref)^omega of the VHS model (Eq. equ3), or
    Sutherland's law mu_ref (T/T_ref)^(3/2) (T_ref + C_s)/(T + C_s) (Eq.
    Sutherland, Sec. 4.6, with the reference state in place of the
    freestream)."""
    if gas.law == 1:
        return gas.mu_ref * (T / gas.T_ref) ** 1.5 * (gas.T_ref + gas.C_s) / (T + gas.C_s)
    return gas.mu_ref * (T / gas.T_ref) ** gas.omega


def tau(rho, T, gas):
    """Relaxation time tau = mu / p (Eq. equ3)."""
    return viscosity(T, gas) / (rho * gas.R * T)


def maxwell(rho, U, T, xi, R):
    """g_eq = rho (2 pi R T)^(-D/2) exp(-|xi-U|^2 / 2RT) (Eq. Maxwell_df)."""
    D = xi.shape[1]
    c = xi - U[None, :]
    c2 = np.sum(c * c, axis=1)
    return rho * (2.0 * math.pi * R * T) ** (-0.5 * D) * np.exp(-c2 / (2.0 * R * T))


def shakhov(rho, U, T, q, xi, gas):
    """Shakhov target (g^G, g^H) for K = 0 (Eqs. equ14-equ17); BGK if model 0.

    Returns an array [P, Nv] with P = 2 (G, H) in 2-D and P = 1 (G) in 3-D.
    """
    D = xi.shape[1]
    R = gas.R
    g = maxwell(rho, U, T, xi, R)
    c = xi - U[None, :]
    c2 = np.sum(c * c, axis=1)
    if gas.model == 1:
        cq = c @ q
        fac = (1.0 - gas.Pr) * cq / (5.0 * rho * R * T * R * T)
        G = g + fac * (c2 / (R * T) - D - 2) * g
        H = (3 - D) * R * T * g + fac * (c2 / (R * T) - D) * (3 - D) * R * T * g
    else:
        G = g
        H = (3 - D) * R * T * g
    return np.stack([G, H]) if D == 2 else G[None, :]


def eq_pair(rho, U, T, xi, R):
    """Maxwellian pair (g, (3-D) R T g) for the reduced VDFs (Eq. equ16, K=0)."""
    D = xi.shape[1]
    g = maxwell(rho, U, T, xi, R)
    return np.stack([g, (3 - D) * R * T * g]) if D == 2 else g[None, :]


def moments(phi, xi, A):
    """W = sum_k A_k (G, xi G, (|xi|^2 G + H)/2) (Eq. updat_W, mid-point rule)."""
    D = xi.shape[1]
    G = phi[0]
    H = phi[1] if D == 2 else 0.0
    xi2 = np.sum(xi * xi, axis=1)
    out = np.empty(D + 2)
    out[0] = np.sum(A * G)
    for d in range(D):
        out[1 + d] = np.sum(A * xi[:, d] * G)
    out[1 + D] = np.sum(A * 0.5 * (xi2 * G + H))
    return out


def heat_flux(phi, xi, A, U):
    """q = 1/2 sum_k A_k c (c^2 G + H), c = xi - U (Eq. equ8, translational part)."""
    D = xi.shape[1]
    G = phi[0]
    H = phi[1] if D == 2 else 0.0
    c = xi - U[None, :]
    c2 = np.sum(c * c, axis=1)
    return np.array([0.5 * np.sum(A * c[:, d] * (c2 * G + H)) for d in range(D)])


def closure(phi_hat, Wstar, xi, A, R):
    """Smallest equilibrium-shaped correction that makes the moments equal W*.

    The paper keeps conservation with the discrete deviation of the
    equilibrium (Sec. 3.3): the correction is spanned by the derivatives of
    g_eq(W*) with respect to W, i.e. by (1, c, |c|^2) g_eq(W*) with
    c = xi - U* (H part (3-D) R T* times the same).  The coefficients solve
    the (D+2)x(D+2) system J lambda = W* - M[phi_hat], J_lm = M_l[e_m]
    (dense LU with partial pivoting).
    """
    D = xi.shape[1]
    rho, U, T = primitive(Wstar, R)
    g = maxwell(rho, U, T, xi, R)
    c = xi - U[None, :]
    basis = [np.ones(len(A))] + [c[:, d] for d in range(D)] + [np.sum(c * c, axis=1)]
    E = []
    for b in basis:
        e = b * g
        E.append(np.stack([e, (3 - D) * R * T * e]) if D == 2 else e[None, :])
    J = np.stack([moments(e, xi, A) for e in E], axis=1)
    lam = np.linalg.solve(J, np.asarray(Wstar, np.float64) - moments(phi_hat, xi, A))
    out = np.array(phi_hat, dtype=np.float64, copy=True)
    for m, e in enumerate(E):
        out = out + lam[m] * e
    return out


# ---------------------------------------------------------------------------
# Physical mesh: per-cell face lists and least-squares coefficients
# ---------------------------------------------------------------------------

@dataclass
class Slot:
    face: int
    sigma: float                 # +1 if the cell is the face's L side, -1 if R
    nbr: int                     # neighbour cell, -1 for a boundary face
    d: np.ndarray                # face midpoint minus cell centre (cell's frame)
    dx: np.ndarray | None        # neighbour centre minus cell centre (cell's frame)


class Mesh:
    """Finite-volume mesh with the geometric data each cell needs.

    Least-squares gradient (Sec. 2.3.3, reconstruction paragraph): weights
    1/|dx_ij|^2 over interior neighbours, ``grad = sum_j c_ij (phi_j - phi_i)``
    with ``c_ij = M^+ w_j dx_ij``, ``M = sum_j w_j dx_ij dx_ij^T`` (pseudo-inverse
    when M is rank deficient).
    """

    def __init__(self, desc):
        self.dim = int(desc['dim'])
        self.nc = int(desc['ncells'])
        self.nf = int(desc['nfaces'])
        self.vol = np.asarray(desc['cell_vol'], np.float64)
        self.ctr = np.asarray(desc['cell_ctr'], np.float64)
        self.lr = np.asarray(desc['face_lr'], np.int64)
        self.area = np.asarray(desc['face_area'], np.float64)
        self.nrm = np.asarray(desc['face_nrm'], np.float64)
        self.fctr = np.asarray(desc['face_ctr'], np.float64)
        self.shift = np.asarray(desc['face_shift'], np.float64)
        self.bc_kind = np.asarray(desc['bc_kind'], np.int32)
        self.bc_state = np.asarray(desc['bc_state'], np.float64)
        self.slots = [[] for _ in range(self.nc)]
        for f in range(self.nf):
            L, R = int(self.lr[f, 0]), int(self.lr[f, 1])
            if R >= 0:
                xR = self.ctr[R] + self.shift[f]
                self.slots[L].append(Slot(f, 1.0, R, self.fctr[f] - self.ctr[L], xR - self.ctr[L]))
                self.slots[R].append(Slot(f, -1.0, L, self.fctr[f] - xR, self.ctr[L] - xR))
            else:
                self.slots[L].append(Slot(f, 1.0, -1, self.fctr[f] - self.ctr[L], None))
        self.lsq = []
        for i in range(self.nc):
            M = np.zeros((self.dim, self.dim))
            for s in self.slots[i]:
                if s.nbr >= 0:
                    M += np.outer(s.dx, s.dx) / np.dot(s.dx, s.dx)
            Minv = np.linalg.pinv(M)
            self.lsq.append([Minv @ (s.dx / np.dot(s.dx, s.dx)) if s.nbr >= 0 else np.zeros(self.dim)
                             for s in self.slots[i]])


# ---------------------------------------------------------------------------
# One explicit step (Sec. 2.3 in the limit of zero implicit increments)
# ---------------------------------------------------------------------------

def limited_gradient(i, phi, mesh, Kv):
    """L * grad(phi_i) per component and node: LSQ gradient + Venkatakrishnan limiter.

    Venkatakrishnan (the limiter the paper cites for the reconstruction):
    for every face f of the cell, D2 = grad . (x_f - x_i), D1 = phimax - phi_i
    if D2 > 0 else phimin - phi_i, psi_f = [(D1^2+eps^2) D2 + 2 D2^2 D1] /
    [D2 (D1^2 + 2 D2^2 + D1 D2 + eps^2)] (psi_f = 1 when D2 = 0), limiter =
    min_f psi_f, eps^2 = (K V^(1/D))^3.  Returns [P, Nv, D].
    """
    D = mesh.dim
    slots = mesh.slots[i]
    p_i = phi[:, i, :]
    grad = np.zeros(p_i.shape + (D,))
    pmax = p_i.copy()
    pmin = p_i.copy()
    for s, c in zip(slots, mesh.lsq[i]):
        if s.nbr >= 0:
            dphi = phi[:, s.nbr, :] - p_i
            grad += dphi[..., None] * c[None, None, :]
            pmax = np.maximum(pmax, phi[:, s.nbr, :])
            pmin = np.minimum(pmin, phi[:, s.nbr, :])
    eps2 = (Kv * mesh.vol[i] ** (1.0 / D)) ** 3
    lim = np.full(p_i.shape, np.inf)
    for s in slots:
        d2 = grad @ s.d
        d1 = np.where(d2 > 0, pmax - p_i, pmin - p_i)
        lim = np.minimum(lim, venkat_psi(d1, d2, eps2))
    if not slots:
        lim[:] = 1.0
    return lim[..., None] * grad


def normal_speed(xi, n):
    """s_k = xi_k . n as the ordered sum xi_1 n_1 + xi_2 n_2 (+ xi_3 n_3),
    without fused multiply-adds: the sign of s decides the upwind side, so it
    is evaluated exactly the same way wherever it is compared with zero."""
    s = xi[:, 0] * n[0]
    for d in range(1, xi.shape[1]):
        s = s + xi[:, d] * n[d]
    return s


def venkat_psi(d1, d2, eps2):
    """psi = [(D1^2+eps^2) D2 + 2 D2^2 D1] / [D2 (D1^2 + 2 D2^2 + D1 D2 + eps^2)], 1 if D2 = 0.

    Evaluated after dividing through by D2, and for eps = 0 through the ratio
    t = D2/D1 >= 0 as (1 + 2t) / (1 + t + 2t^2) when t <= 1, or through
    u = 1/t as u (u + 2) / (u^2 + u + 2) when t > 1: the same function, but
    free of underflow and overflow for VDF values near the ends of the range.
    """
    with np.errstate(divide='ignore', invalid='ignore', over='ignore'):
        if eps2 > 0:
            psi = (d1 * d1 + eps2 + 2.0 * d1 * d2) / (d1 * d1 + 2.0 * d2 * d2 + d1 * d2 + eps2)
        else:
            small = np.abs(d2) <= np.abs(d1)
            t = d2 / d1
            u = d1 / d2
            psi = np.where(small, (1.0 + 2.0 * t) / (1.0 + t + 2.0 * t * t), u * (u + 2.0) / (u * u + u + 2.0))
    return np.where(d2 == 0.0, 1.0, psi)


def reconstruct(phi_c, lg_c, d, xi, h):
    """phi(x_f - xi h) = phi_C + L grad phi_C . (x_f - xi h - x_C) (Sec. 2.3.3)."""
    r = d[None, :] - xi * h
    return phi_c + np.sum(lg_c * r[None, :, :], axis=2)


@dataclass
class StepDiag:
    face_W: np.ndarray = None
    face_tau: np.ndarray = None
    rho_w: dict = field(default_factory=dict)
    residual: np.ndarray = None


def half_step(mesh, tree, dt):
    """h of the interface VDF (Eq. equ27): dt/2, but at most half of the
    step at which the outflow of every cell, for every node of the velocity
    box, equals its content: h <= 1/2 min_i V_i / (1/2 sum_f A_f sum_d
    |n_fd| X_d), X_d = max(|lo_d|, |hi_d|).  The Taylor expansion of the
    reconstruction holds for x_ij - xi h inside the upwind cell (Sec.
    2.3.3); an implicit step longer than the explicit bound would move that
    point cells away, so the flux keeps the largest half step for which
    the point stays within reach of its cell (below the bound, h = dt/2)."""
    X = np.maximum(np.abs(tree.lo), np.abs(tree.hi))
    out = np.zeros(mesh.nc)
    for i in range(mesh.nc):
        for s in mesh.slots[i]:
            out[i] += 0.5 * mesh.area[s.face] * float(np.dot(np.abs(mesh.nrm[s.face]), X))
    return min(0.5 * dt, 0.5 * float(np.min(mesh.vol / out)))


def face_vdf(f, phi, LG, mesh, xi, A, gas, h):
    """Interface VDF at t_n + h for face f (S4-S7).

    Interior face: upwind reconstruction (C = L if xi.n >= 0 else R), face
    moments (Eq. w_interface), tau at the face (Eq. equ3), face heat flux
    relaxed over h at Shakhov's rate Pr/tau, Shakhov equilibrium, and the
    characteristic-line blend of Eq. equ28.  Boundary face: outgoing nodes
    keep the reconstructed VDF; incoming nodes take the diffuse-wall
    Maxwellian with zero net mass flux, or the far-field Maxwellian.
    ``h`` is the half step of ``half_step``.
    Returns (phi_f [P,Nv], diag): ('face', (W_f, tau_f)), ('wall', rho_w) or ('far', None).
    """
    D = mesh.dim
    L, R = int(mesh.lr[f, 0]), int(mesh.lr[f, 1])
    n = mesh.nrm[f]
    s = normal_speed(xi, n)
    slotL = next(sl for sl in mesh.slots[L] if sl.face == f and sl.sigma > 0)
    recL = reconstruct(phi[:, L, :], LG[L], slotL.d, xi, h)
    if R >= 0:
        slotR = next(sl for sl in mesh.slots[R] if sl.face == f and sl.sigma < 0)
        recR = reconstruct(phi[:, R, :], LG[R], slotR.d, xi, h)
        pbar = np.where((s >= 0)[None, :], recL, recR)
        Wf = moments(pbar, xi, A)
        rho, U, T = primitive(Wf, gas.R)
        qbar = heat_flux(pbar, xi, A, U)
        tf = tau(rho, T, gas)
        q = tf / (tf + h * gas.Pr) * qbar
        g = shakhov(rho, U, T, q, xi, gas)
        return tf / (tf + h) * pbar + h / (tf + h) * g, ('face', (Wf, tf))
    b = -1 - R
    st = mesh.bc_state[b]
    Ub, Tb = st[1:1 + D], st[1 + D]
    out = (s >= 0)[None, :]
    if mesh.bc_kind[b] == WALL:
        gw = eq_pair(1.0, Ub, Tb, xi, gas.R)
        num = np.sum(np.where(s > 0, A * s * recL[0], 0.0))
        den = np.sum(np.where(s < 0, A * (-s) * gw[0], 0.0))
        rho_w = num / den
        return np.where(out, recL, rho_w * gw), ('wall', rho_w)
    ginf = eq_pair(st[0], Ub, Tb, xi, gas.R)
    return np.where(out, recL, ginf), ('far', None)


def flux_moments(phi_f, xi, A, n):
    """F = sum_k A_k (xi_k . n) (G, xi G, (|xi|^2 G + H)/2) at the face."""
    s = normal_speed(xi, n)
    return moments(phi_f * s[None, :], xi, A)


def interfaces(mesh, tree, gas, dt, Kv, phi, want):
    """S2-S7 for the faces of the cells ``want``: limited gradients of the
    cells those faces touch, interface VDFs (face_vdf) and their flux
    moments.  Returns (phi_f, F, diag) keyed by face."""
    xi = tree.centres()
    A = tree.weights()
    need_faces = sorted({s.face for i in want for s in mesh.slots[i]})
    need_lg = set()
    for f in need_faces:
        L, R = mesh.lr[f]
        need_lg.add(int(L))
        if R >= 0:
            need_lg.add(int(R))
    LG = {c: limited_gradient(c, phi, mesh, Kv) for c in sorted(need_lg)}
    phif, F, diag = {}, {}, StepDiag(face_W={}, face_tau={})
    h = half_step(mesh, tree, dt)
    for f in need_faces:
        pf, dg = face_vdf(f, phi, LG, mesh, xi, A, gas, h)
        phif[f] = pf
        F[f] = flux_moments(pf, xi, A, mesh.nrm[f])
        if dg[0] == 'wall':
            diag.rho_w[f] = dg[1]
        elif dg[0] == 'face':
            diag.face_W[f], diag.face_tau[f] = dg[1]
    return phif, F, diag


def step(mesh, tree, gas, dt, Kv, phi, W, cells=None):
    """Advance (phi, W) by one step; returns (phi_new, W_new, diag).

    ``phi`` is [P, Nc, Nv], ``W`` is [Nc, D+2] (authoritative conserved
    variables).  ``cells`` optionally restricts the update to a subset (the
    other rows of the result are left as NaN); only the faces and limited
    gradients those cells need are evaluated.

    S1: q_i^n = heat flux of phi_i^n about U_i^n (Eq. equ8).
    S2-S7: interface VDFs (face_vdf).
    S8: W_i^{n+1} = W_i^n - dt/V_i sum_f sigma A_f F_f (Eq. equ18, explicit).
    S9: target g~ = closure(Shakhov(W^{n+1}, q^n), W^{n+1}); tau~ = tau(W^{n+1}).
    S10: phi^{n+1} = [phi^n + dt/tau~ g~ - dt/V sum_f sigma A_f (xi.n) phi_f]
         / (1 + dt/tau~)  (Eq. delta_phi with the implicit increments dropped).
    """
    D = mesh.dim
    xi = tree.centres()
    A = tree.weights()
    want = range(mesh.nc) if cells is None else list(cells)
    phif, F, diag = interfaces(mesh, tree, gas, dt, Kv, phi, want)
    phi_new = np.full(phi.shape, np.nan)
    W_new = np.full(W.shape, np.nan)
    for i in want:
        rho_n, U_n, _ = primitive(W[i], gas.R)
        q_n = heat_flux(phi[:, i, :], xi, A, U_n)
        div = np.zeros(phi.shape[0::2])
        Fsum = np.zeros(D + 2)
        for s in mesh.slots[i]:
            af = s.sigma * mesh.area[s.face]
            Fsum += af * F[s.face]
            div += af * normal_speed(xi, mesh.nrm[s.face])[None, :] * phif[s.face]
        Wn1 = W[i] - dt / mesh.vol[i] * Fsum
        rho, U, T = primitive(Wn1, gas.R)
        if not (rho > 0 and T > 0):
            raise FloatingPointError(f'non-physical state in cell {i}: rho={rho} T={T}')
        ghat = shakhov(rho, U, T, q_n, xi, gas)
        tt = tau(rho, T, gas)
        gt = closure(ghat, Wn1, xi, A, gas.R)
        phi_new[:, i, :] = (phi[:, i, :] + dt / tt * gt - dt / mesh.vol[i] * div) / (1.0 + dt / tt)
        W_new[i] = Wn1
    if cells is None:
        diag.residual = np.sqrt(np.sum((W_new - W) ** 2, axis=0)) / dt
    return phi_new, W_new, diag


# ---------------------------------------------------------------------------
# Adaptation (Sec. 3.2-3.4)
# ---------------------------------------------------------------------------

def criterion(phi, W, tree, R, probes=None):
    """M_k = max over cells (and probe states) of max(M1, M2) (Eqs. criterion_rho,
    criterion_e, criterion_mk; the max runs over the whole physical mesh).

    M1 = A_k G_ik / rho_i, M2 = 0.5 A_k (|xi_k - U_i|^2 G_ik + H_ik) /
    (rho E_i - 0.5 rho_i |U_i|^2), with the authoritative W_i.  Operations are
    done in exactly this order (no fused multiply-add), so that the result is
    reproducible bit for bit.  ``probes`` are primitive rows whose VDF is the
    discrete Maxwellian pair.
    """
    D = tree.dim
    xi = tree.centres()
    A = tree.weights()
    Mk = np.full(tree.n, -np.inf)

    def one(G, H, Wi):
        M1, M2 = criterion_terms(G, H, Wi, xi, A)
        return np.maximum(M1, M2)

    for i in range(phi.shape[1]):
        H = phi[1, i] if D == 2 else 0.0
        Mk = np.maximum(Mk, one(phi[0, i], H, W[i]))
    if probes is not None:
        for p in np.atleast_2d(probes):
            Wp = conserved(p, R)
            e = eq_pair(p[0], p[1:1 + D], p[1 + D], xi, R)
            Mk = np.maximum(Mk, one(e[0], e[1] if D == 2 else 0.0, Wp))
    return Mk


def criterion_terms(G, H, Wi, xi, A):
    """(M1, M2) of one state over all leaves, in the fixed operation order."""
    D = xi.shape[1]
    rho = Wi[0]
    U = [Wi[1 + d] / rho for d in range(D)]
    ke = U[0] * U[0]
    for d in range(1, D):
        ke = ke + U[d] * U[d]
    eint = Wi[1 + D] - 0.5 * rho * ke
    c = xi[:, 0] - U[0]
    c2 = c * c
    for d in range(1, D):
        c = xi[:, d] - U[d]
        c2 = c2 + c * c
    M1 = (A * G) / rho
    M2 = (0.5 * (A * (c2 * G + H))) / eint
    return M1, M2


def raw_flags(Mk, tree, C1, C2):
    """Rules (a)-(c) of Sec. 3.4: split if M_k > C1 (below the maximum level),
    merge-candidate if M_k < C2 (roots never merge), keep otherwise."""
    raw = np.zeros(tree.n, np.int8)
    raw[(Mk > C1) & (tree.level < tree.max_level)] = 1
    raw[(Mk < C2) & (tree.level > 0)] = -1
    return raw


def separated_floor(raw, tree, zone):
    """The separated-zone level of Sec. 3.5 as a floor on the raw flags.
    ``zone = (r_lo, r_hi, S)``: an element whose discrete velocity (its
    centre) lies in the open annulus r_lo < |xi| < r_hi about the origin
    keeps at least level S (relative to the roots).  A leaf in the annulus
    below S is split (below the maximum level); a merge candidate whose
    parent would sit in the annulus below S is kept.  Radii are compared
    squared, |xi|^2 summed axis by axis."""
    r_lo, r_hi, S = zone
    lo2, hi2 = r_lo * r_lo, r_hi * r_hi
    out = raw.copy()
    xi = tree.centres()
    for k in range(tree.n):
        l = int(tree.level[k])
        s = 0.0
        for d in range(tree.dim):
            s = s + xi[k, d] * xi[k, d]
        if lo2 < s < hi2 and l < S and l < tree.max_level:
            out[k] = 1
        if out[k] == -1 and l - 1 < S:
            s = 0.0
            for d in range(tree.dim):
                h = (tree.hi[d] - tree.lo[d]) / float(int(tree.base[d]) << (l - 1))
                c = tree.lo[d] + (float(int(tree.idx[k, d]) >> 1) + 0.5) * h
                s = s + c * c
            if lo2 < s < hi2:
                out[k] = 0
    return out


def resolve_merges(raw, tree):
    """A brother group merges only if all 2^D brothers are leaves and all are
    merge candidates (Sec. 3.1); other candidates are kept."""
    D = tree.dim
    groups = {}
    for k in range(tree.n):
        if tree.level[k] > 0:
            key = (int(tree.level[k]),) + tuple(int(v) >> 1 for v in tree.idx[k])
            groups.setdefault(key, []).append(k)
    eff = raw.copy()
    for k in range(tree.n):
        if raw[k] == -1:
            key = (int(tree.level[k]),) + tuple(int(v) >> 1 for v in tree.idx[k])
            g = groups[key]
            if not (len(g) == 2 ** D and all(raw[m] == -1 for m in g)):
                eff[k] = 0
    return eff


@dataclass
class Plan:
    tree: Tree                   # new leaves
    kind: np.ndarray             # COPY / SPLIT / MERGE per new leaf
    src: np.ndarray              # old leaf index (first brother for MERGE)
    child: np.ndarray            # child number for SPLIT (x bit 0, y bit 1, z bit 2)


def make_plan(eff, tree):
    """New leaf list in depth-first order: keep -> itself, split -> its 2^D
    children, a merging brother group -> the parent at the first brother's
    position (Sec. 3.1)."""
    D = tree.dim
    lev, idx, kind, src, child = [], [], [], [], []
    for k in range(tree.n):
        if eff[k] == 0:
            lev.append(tree.level[k]); idx.append(tree.idx[k]); kind.append(COPY); src.append(k); child.append(0)
        elif eff[k] == 1:
            for c in range(2 ** D):
                bits = np.array([(c >> d) & 1 for d in range(D)], np.int64)
                lev.append(tree.level[k] + 1); idx.append(2 * tree.idx[k] + bits)
                kind.append(SPLIT); src.append(k); child.append(c)
        else:
            cnum = sum(((int(tree.idx[k][d]) & 1) << d) for d in range(D))
            if cnum == 0:
                lev.append(tree.level[k] - 1); idx.append(tree.idx[k] >> 1)
                kind.append(MERGE); src.append(k); child.append(0)
    nt = Tree(D, tree.lo, tree.hi, tree.base, tree.max_level,
              np.array(lev, np.int64), np.array(idx, np.int64).reshape(-1, D))
    return Plan(nt, np.array(kind, np.int8), np.array(src, np.int64), np.array(child, np.int8))


def remap(phi, plan, dim):
    """Consanguinity reconstruction (Sec. 3.2): a child copies its parent; a
    merged parent is the mean of its 2^D children, summed as a balanced
    pairwise tree ((f0+f1)+(f2+f3)) [+ ((f4+f5)+(f6+f7))] times 2^-D."""
    out = np.empty(phi.shape[:2] + (plan.tree.n,))
    for j in range(plan.tree.n):
        k = plan.src[j]
        if plan.kind[j] == MERGE:
            f = [phi[:, :, k + c] for c in range(2 ** dim)]
            if dim == 2:
                out[:, :, j] = ((f[0] + f[1]) + (f[2] + f[3])) * 0.25
            else:
                out[:, :, j] = (((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7]))) * 0.125
        else:
            out[:, :, j] = phi[:, :, k]
    return out


def correct(phi_p, W, tree, R, close=True):
    """Conservation correction of Sec. 3.3: f = f' + g_eq(W) - g_eq(W') with
    W' = M[f'] on the new leaves (H paired as (3-D) R T g), then, when
    ``close``, the closure that makes M[f] = W to round-off."""
    xi = tree.centres()
    A = tree.weights()
    out = np.empty(phi_p.shape)
    for i in range(phi_p.shape[1]):
        Wp = moments(phi_p[:, i], xi, A)
        r1, U1, T1 = primitive(W[i], R)
        r2, U2, T2 = primitive(Wp, R)
        f = phi_p[:, i] + eq_pair(r1, U1, T1, xi, R) - eq_pair(r2, U2, T2, xi, R)
        out[:, i] = closure(f, W[i], xi, A, R) if close else f
    return out


def bypass(W, tree, R, close=False):
    """Equilibrium bypass of the reconstruction (end of Sec. 3.3): f =
    g_eq(W) on the new leaves (H paired as (3-D) R T g), conserving only to
    quadrature error; with ``close`` followed by the closure C(., W)."""
    xi = tree.centres()
    A = tree.weights()
    D = tree.dim
    out = np.empty((2 if D == 2 else 1, W.shape[0], tree.n))
    for i in range(W.shape[0]):
        rho, U, T = primitive(W[i], R)
        f = eq_pair(rho, U, T, xi, R)
        out[:, i] = closure(f, W[i], xi, A, R) if close else f
    return out


# ---------------------------------------------------------------------------
# Driver mirroring the library's entry points
# ---------------------------------------------------------------------------

def gas_from(cfg):
    """Gas parameters from a workload description (mu_ref from Kn via Eq. equ4)."""
    if isinstance(cfg, Gas):
        return cfg
    mu = cfg.get('mu_ref')
    if mu is None:
        mu = mu_ref_from_kn(cfg['Kn'], cfg['omega'], cfg['R'], cfg['T_ref'], cfg.get('rho_ref', 1.0), cfg.get('L_ref', 1.0))
    return Gas(R=cfg['R'], Pr=cfg['Pr'], omega=cfg['omega'], mu_ref=mu, T_ref=cfg['T_ref'], model=cfg.get('model', 1),
               law=cfg.get('law', 0), C_s=cfg.get('C_s', 0.0))


class Solver:
    """init / step / moments / adapt / remap on the CPU, in FP64."""

    def __init__(self, desc, vspace, gas, dt, venkat_K, prim0):
        self.mesh = Mesh(desc)
        self.gas = gas_from(gas)
        self.dt = float(dt)
        self.Kv = float(venkat_K)
        self.tree = base_forest(vspace['dim'], vspace['lo'], vspace['hi'], vspace['base'], vspace['max_level'])
        self.W = conserved(prim0, self.gas.R)
        self.phi = self.initial_vdf(self.W)
        self.plan = None
        self.separated = None    # (r_lo, r_hi, level) floor of every adaptation, or None

    @property
    def dim(self):
        return self.mesh.dim

    def initial_vdf(self, W):
        """phi0 = closure(g_eq(W0), W0) on the current leaves."""
        xi, A = self.tree.centres(), self.tree.weights()
        P = 2 if self.dim == 2 else 1
        phi = np.empty((P, self.mesh.nc, self.tree.n))
        for i in range(self.mesh.nc):
            r, U, T = primitive(W[i], self.gas.R)
            phi[:, i] = closure(eq_pair(r, U, T, xi, self.gas.R), W[i], xi, A, self.gas.R)
        return phi

    def step(self, n=1):
        res = None
        for _ in range(n):
            self.phi, self.W, d = step(self.mesh, self.tree, self.gas, self.dt, self.Kv, self.phi, self.W)
            res = d.residual
        return res

    def step_implicit(self, n=1, macro=60, micro=2):
        """Implicit steps (oracle.avs_implicit.step_implicit)."""
        from .avs_implicit import step_implicit
        res = None
        for _ in range(n):
            self.phi, self.W, d = step_implicit(self.mesh, self.tree, self.gas, self.dt, self.Kv, self.phi, self.W,
                                                macro, micro)
            res = d.residual
        return res

    def fields(self):
        """rho, U, T from the authoritative W and q from phi about U."""
        xi, A = self.tree.centres(), self.tree.weights()
        D = self.dim
        out = np.empty((self.mesh.nc, 2 * D + 2))
        for i in range(self.mesh.nc):
            r, U, T = primitive(self.W[i], self.gas.R)
            out[i, 0], out[i, 1:1 + D], out[i, 1 + D] = r, U, T
            out[i, 2 + D:] = heat_flux(self.phi[:, i], xi, A, U)
        return out

    def totals(self):
        return np.sum(self.mesh.vol[:, None] * self.W, axis=0)

    def vdf_moments(self):
        xi, A = self.tree.centres(), self.tree.weights()
        return np.stack([moments(self.phi[:, i], xi, A) for i in range(self.mesh.nc)])

    def adapt(self, C1, C2, probes=None):
        Mk = criterion(self.phi, self.W, self.tree, self.gas.R, probes)
        raw = raw_flags(Mk, self.tree, C1, C2)
        if self.separated is not None:
            raw = separated_floor(raw, self.tree, self.separated)
        eff = resolve_merges(raw, self.tree)
        self.plan = make_plan(eff, self.tree)
        return eff, self.plan, Mk

    def remap(self, correction=2):
        """Commit the plan.  correction 0: consanguinity only (Sec. 3.2); 1:
        plus f' + g(W) - g(W'); 2: plus the closure (Sec. 3.3); 3: the
        equilibrium bypass f = g_eq(W) for weakly non-equilibrium flow (end
        of Sec. 3.3); 4: the bypass closed onto W."""
        p = self.plan
        self.tree = p.tree
        if correction in (3, 4):
            self.phi = bypass(self.W, self.tree, self.gas.R, close=(correction == 4))
        else:
            phi_p = remap(self.phi, p, self.dim)
            if correction:
                phi_p = correct(phi_p, self.W, self.tree, self.gas.R, close=(correction == 2))
            self.phi = phi_p
        self.plan = None
