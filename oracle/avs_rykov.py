"""Plain FP64 CPU oracle of the Rykov diatomic model (Sec. 2.2-2.3 of arXiv
2212.05645: Eqs. equ6, updat_W, equ8, GHR_equ, equ11-equ13, equ19 and the
rotational interface relaxation after Eq. w_interface).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no
code with the GPU library and imports nothing from it.

A diatomic gas carries three reduced distributions on the D-dimensional
velocity mesh: G (mass), H (the 3 - D hidden translational degrees of
freedom; zero in 3-D) and R (rotational energy, two rotational degrees of
freedom).  The conserved variables are W = (rho, rho U, rho E, rho E_rot)
with (Eq. updat_W)
    rho = int G,  rho U = int xi G,  rho E = int [(|xi|^2 G + H)/2 + R],
    rho E_rot = int R.
Temperatures: rho E_rot = rho R T_r (two rotational degrees of freedom),
rho E - rho |U|^2/2 - rho E_rot = 3/2 rho R T_t, and the equilibrium
temperature T = (3 T_t + 2 T_r)/5 shares the internal energy over five
degrees of freedom.  Heat fluxes (Eq. equ8): q_t = 1/2 int c (c^2 G + H),
q_r = int c R.

Readings (the paper leaves these open):
* Z_rot is a parameter of the gas (the paper names it without a value);
* the relaxation time is tau = mu(T_t) / p_t with p_t = rho R T_t;
* the rotational interface state (the formula after Eq. w_interface is
  printed with its relaxation factor in the numerator) is the implicit
  relaxation over h: rho R T_rot = (int R + h/(Z tau) rho R T) / (1 + h/(Z tau)).

The implicit step (``step_implicit_dia``) extends the monatomic IUGKS of
``avs_implicit`` with the rotational row.  Readings:
* the predictor's Euler flux carries rho E_rot U.n and uses the
  translational pressure rho R T_t, so its sound speed in r_ij is the
  frozen one, sqrt(5/3 R T_t), and mu/rho = tau R T_t;
* tau and rho R T of Eq. SGS_wrot are taken at the cell's current iterate
  W + dW in every sweep (rho R T does not depend on the rotational share);
* W^{n+1} is the flux form with the implicit flux, followed by the
  point-implicit rotational exchange of the explicit step, so that the
  same target and tau~ drive the micro system.

Pins (tests/test_rykov_pins.py): the equilibrium's moments and heat fluxes
against closed forms of Gaussian moments (mass, momentum, the translational
energy 3/2 rho R T_t of the t part and 3/2 rho R T of the r part, int R^t =
rho R T_r, int R^r = rho R T, q_t of (G^t, H^t) = q_t/3, of (G^r, H^r) =
omega_0 q_t/3, int c R^t = (1 - delta)(T_r/T_t) q_r, int c R^r = omega_1
(1 - delta) q_r); energy conservation of the collision; the rotational
moment of the collision term equal to the source of Eq. equ19; the limits
Z -> 1 and Z -> infinity; the interface relaxation's limits.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class RykovGas:
    R: float
    Z_rot: float = 3.5
    delta: float = 1.0 / 1.55      # nitrogen (Sec. 2.2)
    omega0: float = 0.2354
    omega1: float = 0.3049


def temperatures(W, R):
    """W = (rho, rho U, rho E, rho E_rot) -> (rho, U, T_t, T_r, T)."""
    D = len(W) - 3
    rho = W[0]
    U = W[1:1 + D] / rho
    Erot = W[2 + D]
    Tr = Erot / (rho * R)
    Tt = (W[1 + D] - 0.5 * rho * float(np.dot(U, U)) - Erot) / (1.5 * rho * R)
    T = (3.0 * Tt + 2.0 * Tr) / 5.0
    return rho, U, Tt, Tr, T


def conserved(rho, U, Tt, Tr, R):
    U = np.asarray(U, np.float64)
    D = len(U)
    out = np.empty(D + 3)
    out[0] = rho
    out[1:1 + D] = rho * U
    out[2 + D] = rho * R * Tr
    out[1 + D] = 0.5 * rho * float(np.dot(U, U)) + 1.5 * rho * R * Tt + out[2 + D]
    return out


def maxwell(rho, U, T, xi, R):
    """g_eq(T) = rho (2 pi R T)^(-D/2) exp(-|xi - U|^2 / 2RT) (Eq. Maxwell_df)."""
    D = xi.shape[1]
    c = xi - U[None, :]
    return rho * (2.0 * math.pi * R * T) ** (-0.5 * D) * np.exp(-np.sum(c * c, axis=1) / (2.0 * R * T))


def rykov_parts(rho, U, Tt, Tr, qt, qr, xi, gas):
    """The translational and rotational parts (G, H, R)^t and (G, H, R)^r of
    Eqs. equ11-equ13, each [3, Nv] (H is zero in 3-D)."""
    D = xi.shape[1]
    R = gas.R
    T = (3.0 * Tt + 2.0 * Tr) / 5.0
    c = xi - np.asarray(U)[None, :]
    c2 = np.sum(c * c, axis=1)
    cqt = c @ np.asarray(qt)
    cqr = c @ np.asarray(qr)
    pt, p = rho * R * Tt, rho * R * T
    gt = maxwell(rho, np.asarray(U), Tt, xi, R)
    g = maxwell(rho, np.asarray(U), T, xi, R)
    at = cqt / (15.0 * pt * R * Tt)
    ar = gas.omega0 * cqt / (15.0 * p * R * T)
    Gt = gt * (1.0 + at * (c2 / (R * Tt) - D - 2))
    Gr = g * (1.0 + ar * (c2 / (R * T) - D - 2))
    Ht = R * Tt * gt * (3 - D) * (1.0 + at * (c2 / (R * Tt) - D))
    Hr = R * T * g * (3 - D) * (1.0 + ar * (c2 / (R * T) - D))
    Rt = R * Tr * (Gt + (1.0 - gas.delta) * cqr / (pt * R * Tt) * gt)
    Rr = R * T * (Gr + gas.omega1 * (1.0 - gas.delta) * cqr / (p * R * T) * g)
    return np.stack([Gt, Ht, Rt]), np.stack([Gr, Hr, Rr])


def rykov_equilibrium(rho, U, Tt, Tr, qt, qr, xi, gas):
    """g^phi = (1 - 1/Z) phi^t + (1/Z) phi^r for phi = G, H, R (Eq. GHR_equ)."""
    t, r = rykov_parts(rho, U, Tt, Tr, qt, qr, xi, gas)
    return (1.0 - 1.0 / gas.Z_rot) * t + (1.0 / gas.Z_rot) * r


def moments(f, xi, A):
    """(rho, rho U, rho E, rho E_rot) of f = [G, H, R] (Eq. updat_W)."""
    G, H, Rr = f
    D = xi.shape[1]
    xi2 = np.sum(xi * xi, axis=1)
    out = np.empty(D + 3)
    out[0] = np.sum(A * G)
    out[1:1 + D] = (A * G) @ xi
    out[1 + D] = np.sum(A * (0.5 * (xi2 * G + H) + Rr))
    out[2 + D] = np.sum(A * Rr)
    return out


def heat_fluxes(f, xi, A, U):
    """q_t = 1/2 int c (c^2 G + H), q_r = int c R (Eq. equ8)."""
    G, H, Rr = f
    c = xi - np.asarray(U)[None, :]
    c2 = np.sum(c * c, axis=1)
    qt = (A * 0.5 * (c2 * G + H)) @ c
    qr = (A * Rr) @ c
    return qt, qr


def rotational_source(W, tau, gas):
    """S_rot = (rho E_rot,eq - rho E_rot) / (Z tau) with rho E_rot,eq = rho R T (Eq. equ19)."""
    rho, U, Tt, Tr, T = temperatures(W, gas.R)
    return (rho * gas.R * T - W[-1]) / (gas.Z_rot * tau)


def interface_rotational_energy(int_R, rhoRT, h, tau, gas):
    """rho R T_rot at the interface: implicit relaxation of int R towards
    rho R T over h at the rate 1/(Z tau) (the relation after Eq. w_interface,
    read with its relaxation factor as a divisor)."""
    k = h / (gas.Z_rot * tau)
    return (int_R + k * rhoRT) / (1.0 + k)


# ---------------------------------------------------------------------------
# One explicit step of the diatomic model (Sec. 2.3 in its explicit limit,
# with the Rykov equilibrium of Eq. GHR_equ and the source of Eq. equ19)
# ---------------------------------------------------------------------------
#
# Further readings for the step (the paper states them for the monatomic
# case or not at all):
# * interface heat fluxes relax over h at the rates the collision gives
#   them: the Rykov equilibrium carries lambda_t q_t and lambda_r q_r with
#   lambda_t = (1 - 1/Z)/3 + omega_0/(3Z) and lambda_r = (1 - delta)
#   ((1 - 1/Z) T_r/T_t + omega_1/Z), so q_f = q_bar / (1 + (1 - lambda) h/tau)
#   (for a monatomic Shakhov gas this is the factor tau/(tau + h Pr) of the
#   explicit step);
# * the interface translational temperature follows from the rotational
#   relaxation at fixed internal energy;
# * the rotational exchange is point-implicit with tau from the state after
#   transport, W*: rho E_rot^{n+1} = (rho E_rot* + k rho R T) / (1 + k),
#   k = dt/(Z tau*), and the relaxation of phi uses the same tau, so that the
#   moments of phi^{n+1} equal W^{n+1} exactly;
# * the target's rotational moment is (1 - 1/Z) rho E_rot^{n+1} + rho R T / Z
#   (the rotational energy of the Rykov equilibrium of W^{n+1}), its other
#   moments those of W^{n+1}; the closure spans (1, c, |c|^2) times the
#   Maxwellian triple (g, (3 - D) R T g, R T g) at T and the rotational
#   direction (0, 0, R T g);
# * boundary Maxwellians are in equilibrium (T_t = T_r = the wall's or the
#   far field's temperature): (g, (3 - D) R T g, R T g);
# * the initial state is the translational part at (T_t, T_r) with zero
#   heat fluxes, closed onto W.

from . import avs_oracle as _O


def tau_t(rho, Tt, vgas):
    """tau = mu(T_t) / p_t (reading)."""
    return _O.viscosity(Tt, vgas) / (rho * vgas.R * Tt)


def triple(rho, U, T, xi, R):
    """Equilibrium triple (g, (3 - D) R T g, R T g) at one temperature."""
    D = xi.shape[1]
    g = maxwell(rho, np.asarray(U, np.float64), T, xi, R)
    return np.stack([g, (3 - D) * R * T * g, R * T * g])


def closure_dia(f_hat, target, W, xi, A, R):
    """f_hat + sum_m lambda_m e_m with moments equal to ``target``; the e_m
    are (1, c, |c|^2) times the equilibrium triple at T of W, and (0, 0, R T g)."""
    D = xi.shape[1]
    rho, U, Tt, Tr, T = temperatures(W, R)
    tri = triple(rho, U, T, xi, R)
    c = xi - U[None, :]
    basis = [np.ones(len(A))] + [c[:, d] for d in range(D)] + [np.sum(c * c, axis=1)]
    E = [b[None, :] * tri for b in basis]
    E.append(np.stack([np.zeros(len(A)), np.zeros(len(A)), tri[2]]))
    J = np.stack([moments(e, xi, A) for e in E], axis=1)
    lam = np.linalg.solve(J, np.asarray(target, np.float64) - moments(f_hat, xi, A))
    out = np.array(f_hat, dtype=np.float64, copy=True)
    for m, e in enumerate(E):
        out = out + lam[m] * e
    return out


def heat_rates(Tt, Tr, gas):
    lt = (1.0 - 1.0 / gas.Z_rot) / 3.0 + gas.omega0 / (3.0 * gas.Z_rot)
    lr = (1.0 - gas.delta) * ((1.0 - 1.0 / gas.Z_rot) * Tr / Tt + gas.omega1 / gas.Z_rot)
    return lt, lr


def face_vdf_dia(f, phi, LG, mesh, xi, A, vgas, gas, h, state=None):
    """Interface VDF (3 components) of face f at t_n + h.  For an interior
    face, ``state`` (a dict, if given) receives the interface moment state
    (rho, U, T_t) and its tau."""
    D = mesh.dim
    R = gas.R
    L, Rc = int(mesh.lr[f, 0]), int(mesh.lr[f, 1])
    n = mesh.nrm[f]
    s = _O.normal_speed(xi, n)
    slotL = next(sl for sl in mesh.slots[L] if sl.face == f and sl.sigma > 0)
    recL = _O.reconstruct(phi[:, L, :], LG[L], slotL.d, xi, h)
    if Rc >= 0:
        slotR = next(sl for sl in mesh.slots[Rc] if sl.face == f and sl.sigma < 0)
        recR = _O.reconstruct(phi[:, Rc, :], LG[Rc], slotR.d, xi, h)
        pbar = np.where((s >= 0)[None, :], recL, recR)
        Wf = moments(pbar, xi, A)
        rho, U, Tt_b, Tr_b, T = temperatures(Wf, R)
        qt_b, qr_b = heat_fluxes(pbar, xi, A, U)
        tf = tau_t(rho, Tt_b, vgas)
        if state is not None:
            state[f] = (rho, U, Tt_b, tf)
        ERf = interface_rotational_energy(Wf[2 + D], rho * R * T, h, tf, gas)
        Tr = ERf / (rho * R)
        Tt = Tt_b + (2.0 / 3.0) * (Tr_b - Tr)
        lt, lr = heat_rates(Tt, Tr, gas)
        qt = qt_b / (1.0 + (1.0 - lt) * h / tf)
        qr = qr_b / (1.0 + (1.0 - lr) * h / tf)
        g = rykov_equilibrium(rho, U, Tt, Tr, qt, qr, xi, gas)
        return tf / (tf + h) * pbar + h / (tf + h) * g
    b = -1 - Rc
    st = mesh.bc_state[b]
    Ub, Tb = st[1:1 + D], st[1 + D]
    out = (s >= 0)[None, :]
    if mesh.bc_kind[b] == _O.WALL:
        gw = triple(1.0, Ub, Tb, xi, R)
        num = np.sum(np.where(s > 0, A * s * recL[0], 0.0))
        den = np.sum(np.where(s < 0, A * (-s) * gw[0], 0.0))
        return np.where(out, recL, (num / den) * gw)
    return np.where(out, recL, triple(st[0], Ub, Tb, xi, R))


def flux_moments(phi_f, xi, A, n):
    return moments(phi_f * _O.normal_speed(xi, n)[None, :], xi, A)


def step_dia(mesh, tree, vgas, gas, dt, Kv, phi, W):
    """One explicit step of the diatomic model; phi [3, Nc, Nv], W [Nc, D+3]."""
    D = mesh.dim
    R = gas.R
    xi, A = tree.centres(), tree.weights()
    h = _O.half_step(mesh, tree, dt)
    LG = {c: _O.limited_gradient(c, phi, mesh, Kv) for c in range(mesh.nc)}
    phif, F = {}, {}
    for f in range(mesh.nf):
        phif[f] = face_vdf_dia(f, phi, LG, mesh, xi, A, vgas, gas, h)
        F[f] = flux_moments(phif[f], xi, A, mesh.nrm[f])
    phi_new = np.empty_like(phi)
    W_new = np.empty_like(W)
    for i in range(mesh.nc):
        _, U_n, _, _, _ = temperatures(W[i], R)
        qt_n, qr_n = heat_fluxes(phi[:, i, :], xi, A, U_n)
        Fs = np.zeros(D + 3)
        div = np.zeros(phi.shape[0::2])
        for s in mesh.slots[i]:
            af = s.sigma * mesh.area[s.face]
            Fs += af * F[s.face]
            div += af * _O.normal_speed(xi, mesh.nrm[s.face])[None, :] * phif[s.face]
        Ws = W[i] - dt / mesh.vol[i] * Fs
        rho, U, Tt_s, Tr_s, T = temperatures(Ws, R)
        if not (rho > 0 and Tt_s > 0 and Tr_s > 0):
            raise FloatingPointError(f'non-physical state in cell {i}')
        tt = tau_t(rho, Tt_s, vgas)
        k = dt / (gas.Z_rot * tt)
        Wn = Ws.copy()
        Wn[2 + D] = (Ws[2 + D] + k * rho * R * T) / (1.0 + k)
        _, _, Tt, Tr, _ = temperatures(Wn, R)
        target = Wn.copy()
        target[2 + D] = (1.0 - 1.0 / gas.Z_rot) * Wn[2 + D] + rho * R * T / gas.Z_rot
        g = rykov_equilibrium(rho, U, Tt, Tr, qt_n, qr_n, xi, gas)
        gt = closure_dia(g, target, Wn, xi, A, R)
        phi_new[:, i, :] = (phi[:, i, :] + dt / tt * gt - dt / mesh.vol[i] * div) / (1.0 + dt / tt)
        W_new[i] = Wn
    return phi_new, W_new


def euler_flux_dia(W, n, R):
    """Euler flux of a diatomic state through n (the flux of the implicit
    predictor with the rotational row): (rho U.n, rho U U.n + p n,
    (rho E + p) U.n, rho E_rot U.n) with the translational pressure
    p = rho R T_t."""
    D = len(n)
    rho, U, Tt, _, _ = temperatures(W, R)
    p = rho * R * Tt
    un = float(np.dot(U, n))
    out = np.empty(D + 3)
    out[0] = rho * un
    out[1:1 + D] = rho * U * un + p * np.asarray(n)
    out[1 + D] = (W[1 + D] + p) * un
    out[2 + D] = W[2 + D] * un
    return out


def roe_radius_dia(rho, U, Tt, tau, n, dl, R):
    """r = |U.n| + a + 2 mu / (rho dl) with the frozen sound speed
    a = sqrt(5/3 R T_t) of the flux above (E_rot is only carried) and
    mu / rho = tau R T_t."""
    return abs(float(np.dot(U, n))) + math.sqrt(5.0 / 3.0 * R * Tt) + 2.0 * tau * R * Tt / dl


def step_implicit_dia(mesh, tree, vgas, gas, dt, Kv, phi, W, n_macro, n_micro, order=None):
    """One implicit step of the diatomic model (Sec. 2.3.1-2.3.2 with the
    rotational row of Eqs. S_rot, SGS_wrot); phi [3, Nc, Nv], W [Nc, D+3].
    Returns (phi_new, W_new, predicted W~)."""
    from . import avs_implicit as _I
    D = mesh.dim
    R = gas.R
    xi, A = tree.centres(), tree.weights()
    if order is None:
        order = _I.sweep_order(_I.cell_colours(mesh))
    h = _O.half_step(mesh, tree, dt)
    LG = {c: _O.limited_gradient(c, phi, mesh, Kv) for c in range(mesh.nc)}
    phif, F, fst = {}, {}, {}
    for f in range(mesh.nf):
        phif[f] = face_vdf_dia(f, phi, LG, mesh, xi, A, vgas, gas, h, state=fst)
        F[f] = flux_moments(phif[f], xi, A, mesh.nrm[f])
    rhs = np.zeros_like(W)
    div = np.zeros_like(phi)
    for i in range(mesh.nc):
        for s in mesh.slots[i]:
            af = s.sigma * mesh.area[s.face]
            rhs[i] -= af * F[s.face]
            div[:, i, :] += af * _O.normal_speed(xi, mesh.nrm[s.face])[None, :] * phif[s.face]
    # r_ij from the interface moment state; a boundary face from its cell's W^n
    r = np.zeros(mesh.nf)
    for f in range(mesh.nf):
        L, Rc = int(mesh.lr[f, 0]), int(mesh.lr[f, 1])
        n = mesh.nrm[f]
        if Rc >= 0:
            rho, U, Tt, tf = fst[f]
            dl = float(np.linalg.norm(mesh.ctr[Rc] + mesh.shift[f] - mesh.ctr[L]))
        else:
            rho, U, Tt, _, _ = temperatures(W[L], R)
            tf = tau_t(rho, Tt, vgas)
            dl = 2.0 * float(np.dot(mesh.fctr[f] - mesh.ctr[L], n))
        r[f] = roe_radius_dia(rho, U, Tt, tf, n, dl, R)

    # Eq. SGS_wrot: the rotational row gains V/(Z tau) on its diagonal and
    # V ((rho R T) - rho E_rot^n)/(Z tau) on its right-hand side, tau and
    # rho R T taken at the cell's current iterate W + dW
    def rot_source(i, Wc):
        rho, _, Tt, _, T = temperatures(Wc, R)
        k = mesh.vol[i] / (gas.Z_rot * tau_t(rho, Tt, vgas))
        d = np.zeros(D + 3)
        b = np.zeros(D + 3)
        d[2 + D] = k
        b[2 + D] = k * (rho * R * T - W[i][2 + D])
        return d, b

    dW = _I.macro_sgs(mesh, dt, R, W, rhs, r, n_macro, order, flux=euler_flux_dia, source=rot_source)
    Fh = _I.implicit_flux(mesh, gas, W, dW, F, r, flux=euler_flux_dia)
    res = np.empty_like(phi)
    tau_c = np.empty(mesh.nc)
    W_new = np.empty_like(W)
    for i in range(mesh.nc):
        _, U_n, _, _, _ = temperatures(W[i], R)
        qt_n, qr_n = heat_fluxes(phi[:, i, :], xi, A, U_n)
        Fs = np.zeros(D + 3)
        for s in mesh.slots[i]:
            Fs += s.sigma * mesh.area[s.face] * Fh[s.face]
        # W^{n+1}: flux form with the implicit flux, then the rotational
        # exchange as in the explicit step
        Ws = W[i] - dt / mesh.vol[i] * Fs
        rho, U, Tt_s, Tr_s, T = temperatures(Ws, R)
        if not (rho > 0 and Tt_s > 0 and Tr_s > 0):
            raise FloatingPointError(f'non-physical state in cell {i}')
        tt = tau_t(rho, Tt_s, vgas)
        k = dt / (gas.Z_rot * tt)
        Wn = Ws.copy()
        Wn[2 + D] = (Ws[2 + D] + k * rho * R * T) / (1.0 + k)
        _, _, Tt, Tr, _ = temperatures(Wn, R)
        target = Wn.copy()
        target[2 + D] = (1.0 - 1.0 / gas.Z_rot) * Wn[2 + D] + rho * R * T / gas.Z_rot
        gt = closure_dia(rykov_equilibrium(rho, U, Tt, Tr, qt_n, qr_n, xi, gas), target, Wn, xi, A, R)
        tau_c[i] = tt
        res[:, i, :] = mesh.vol[i] * (gt - phi[:, i, :]) / tt - div[:, i, :]
        W_new[i] = Wn
    phi_new = phi + _I.micro_sgs(mesh, xi, dt, tau_c, res, n_micro, order)
    return phi_new, W_new, W + dW


class DiatomicSolver:
    """Explicit diatomic steps on a fixed velocity tree, in FP64.
    ``prim0`` rows are (rho, U, T_t, T_r); the physical gas ``vgas`` gives R
    and the viscosity law; ``gas`` the Rykov constants."""

    def __init__(self, desc, tree, vgas, gas, dt, venkat_K, prim0):
        self.mesh = _O.Mesh(desc)
        self.tree = tree
        self.vgas = _O.gas_from(vgas)
        self.gas = gas
        self.dt = float(dt)
        self.Kv = float(venkat_K)
        D = self.mesh.dim
        P0 = np.asarray(prim0, np.float64)
        self.W = np.stack([conserved(p[0], p[1:1 + D], p[1 + D], p[2 + D], gas.R) for p in P0])
        self.phi = self.initial_vdf(self.W)

    def initial_vdf(self, W):
        xi, A = self.tree.centres(), self.tree.weights()
        out = np.empty((3, self.mesh.nc, self.tree.n))
        z = np.zeros(self.mesh.dim)
        for i in range(self.mesh.nc):
            rho, U, Tt, Tr, _ = temperatures(W[i], self.gas.R)
            t, _ = rykov_parts(rho, U, Tt, Tr, z, z, xi, self.gas)
            out[:, i] = closure_dia(t, W[i], W[i], xi, A, self.gas.R)
        return out

    def step(self, n=1):
        for _ in range(n):
            self.phi, self.W = step_dia(self.mesh, self.tree, self.vgas, self.gas, self.dt, self.Kv, self.phi, self.W)

    def step_implicit(self, n, n_macro, n_micro):
        for _ in range(n):
            self.phi, self.W, self.predicted = step_implicit_dia(self.mesh, self.tree, self.vgas, self.gas, self.dt,
                                                                 self.Kv, self.phi, self.W, n_macro, n_micro)

    def vdf_moments(self):
        xi, A = self.tree.centres(), self.tree.weights()
        return np.stack([moments(self.phi[:, i], xi, A) for i in range(self.mesh.nc)])

    def totals(self):
        return np.sum(self.mesh.vol[:, None] * self.W, axis=0)


# ---------------------------------------------------------------------------
# Adaptation of the diatomic state (Sec. 3.2-3.4 with the diatomic energy)
# ---------------------------------------------------------------------------
#
# Readings: M2 measures the internal energy including rotation,
# M2 = A (1/2 (|c|^2 G + H) + R) / (rho E - rho |U|^2 / 2); the remap is the
# consanguinity reconstruction of each component followed by the closure
# onto W (the diatomic counterpart of correction 2 without its literal
# equilibrium difference); no probe states.

def _crit_dia_one(G, H, Rr, Wi, xi, A):
    """max(M1, M2) of one state over all leaves, in the fixed operation order."""
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
    M2 = (A * (0.5 * (c2 * G + H) + Rr)) / eint
    return np.maximum(M1, M2)


def criterion_dia(phi, W, tree, probes=None, R=None):
    """M_k = max over cells (and over probe states) of max(M1, M2), in a
    fixed operation order (no fused multiply-add) so that it can be compared
    bit for bit.  ``probes`` are rows (rho, U, T) of equilibrium states
    (T_t = T_r = T) whose VDF is the equilibrium triple; R is the gas
    constant."""
    xi, A = tree.centres(), tree.weights()
    Mk = np.full(tree.n, -np.inf)
    for i in range(phi.shape[1]):
        Mk = np.maximum(Mk, _crit_dia_one(phi[0, i], phi[1, i], phi[2, i], W[i], xi, A))
    if probes is not None:
        D = tree.dim
        for p in np.atleast_2d(probes):
            rho, U, T = p[0], np.asarray(p[1:1 + D], np.float64), p[1 + D]
            tri = triple(rho, U, T, xi, R)
            Mk = np.maximum(Mk, _crit_dia_one(tri[0], tri[1], tri[2], conserved(rho, U, T, T, R), xi, A))
    return Mk


def remap_dia(phi, plan, W, R):
    """Consanguinity reconstruction of G, H and R, then the closure onto W."""
    D = plan.tree.dim
    out = _O.remap(phi, plan, D)
    xi, A = plan.tree.centres(), plan.tree.weights()
    for i in range(out.shape[1]):
        out[:, i] = closure_dia(out[:, i], W[i], W[i], xi, A, R)
    return out


def _adapt(self, C1, C2, probes=None):
    Mk = criterion_dia(self.phi, self.W, self.tree, probes, self.gas.R)
    raw = _O.raw_flags(Mk, self.tree, C1, C2)
    if getattr(self, 'separated', None) is not None:
        raw = _O.separated_floor(raw, self.tree, self.separated)
    eff = _O.resolve_merges(raw, self.tree)
    self.plan = _O.make_plan(eff, self.tree)
    return eff, self.plan, Mk


def _remap(self):
    self.phi = remap_dia(self.phi, self.plan, self.W, self.gas.R)
    self.tree = self.plan.tree
    self.plan = None


DiatomicSolver.adapt = _adapt
DiatomicSolver.remap = _remap
