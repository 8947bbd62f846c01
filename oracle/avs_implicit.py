"""Plain FP64 CPU oracle of the implicit step of Sec. 2.3.1-2.3.2 (IUGKS)
of arXiv 2212.05645, for the monatomic Shakhov/BGK gas of ``avs_oracle``.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no
code with the GPU library and imports nothing from it; the interface stage
(reconstruction, interface VDF, flux moments) is ``avs_oracle.interfaces``.

One step, in the paper's order:

1. interface VDFs phi_ij^n and fluxes F_ij^n at t_n + h, as in the
   explicit step (Sec. 2.3.3; h = dt/2 capped by ``avs_oracle.half_step``);
2. macroscopic predictor (Eqs. equ_delw, delta_Flux, Roe, SGS_w): the
   increment dW solves
       (V_i/dt + 1/2 sum_j A_ij r_ij) dW_i - 1/2 sum_j A_ij r_ij dW_j
           = -sum_j A_ij F_ij^n - 1/2 sum_j A_ij [G_ij(W_j + dW_j) - G_ij(W_j)]
   with G the Euler flux through the outward normal of i and
   r_ij = |U_ij . n_ij| + a_ij + 2 mu_ij / (rho_ij dl_ij); it is solved by
   point-relaxation symmetric Gauss-Seidel sweeps (PRSGS); W~ = W^n + dW;
3. W^{n+1} (below), target g~ = closure(Shakhov(W^{n+1}, q^n), W^{n+1})
   and tau~ = tau(W^{n+1}), as in the explicit step;
4. microscopic increment (Eqs. delta_phi, SGS_phi): per velocity node,
       (V_i/dt + V_i/tau~_i + sum_{j in N+} A_ij xi.n_ij) dphi_i
           + sum_{j in N-} A_ij xi.n_ij dphi_j = Res_i,
       Res_i = V_i (g~_i - phi_i^n)/tau~_i - sum_j A_ij xi.n_ij phi_ij^n,
   N+ the faces with xi.n_ij >= 0, solved by symmetric Gauss-Seidel sweeps;
5. phi^{n+1} = phi^n + dphi.

W^{n+1} follows from the flux form of Eq. equ18 with the implicit flux of
Eqs. delta_Flux and Roe: W_i^{n+1} = W_i^n - dt/V_i sum_j A_ij Fh_ij,
    Fh_ij = F_ij^n + 1/2 [G_ij(W~_i) - G_ij(W_i) + G_ij(W~_j) - G_ij(W_j)]
            + 1/2 r_ij (dW_i - dW_j)
with the outside state of a boundary face described below.  With converged
sweeps and no boundary face this is W~ exactly (the terms dropped from Eq.
SGS_w sum to zero over a closed cell); after any number of sweeps it
conserves mass, momentum and energy between cells exactly, and no mass
crosses a wall, which W~ does not guarantee.  The target (step 3) is built
from this W^{n+1}.

Readings (the paper leaves these open):
* sweep order: the cells in colour-major order of the greedy colouring of
  the face-neighbour graph in cell order (each cell takes the smallest
  colour that no lower-numbered neighbour holds); one symmetric sweep runs
  the colours up, then down.  This is a Gauss-Seidel order like any other
  cell numbering, and the cells of one colour do not depend on each other;
* the interface state of r_ij is the interface moment state W_ij of Eq.
  w_interface (the state the interface equilibrium is built from); a
  boundary face takes its cell's W^n and dl = 2 (x_f - x_i) . n;
* outside a boundary face, in the predictor and in Fh: a far-field face
  holds the outside at W^n (increment 0); a wall face takes the mirror
  state (normal momentum reversed) of the cell's own W and dW, so that the
  mass and energy increments through the wall cancel and only the
  pressure increment acts.  The micro system holds the outside increment
  at zero on every boundary face, so an outgoing node adds A xi.n to its
  diagonal;
* a = sqrt(gamma R T) with gamma = 5/3 (three translational degrees of
  freedom, the gas of Eq. updat_W);
* W^{n+1} is the conservative update above: the predicted state itself
  drifts in mass when the sweeps stop short, and a Roe increment against
  a fixed outside state would carry mass through walls during the
  transient; either way the steady state of a closed domain would depend
  on the path to it.
  The micro system takes q^n about U^n like the explicit step.

Pins (tests/test_implicit_pins.py): the converged micro sweeps against the
Fourier solution of the circulant upwind system on a periodic strip; the
converged predictor against the Fourier solution of its linearisation about
a uniform state (Euler Jacobian in closed form) and, on periodic meshes,
its exact conservation; r_ij against the spectral radius of a numerical
Euler Jacobian in the inviscid limit; the explicit update as the small-dt
limit of the predictor; the step's W^{n+1} conserving the totals after two
sweeps and equal to W~ after converged sweeps.
"""
from __future__ import annotations

import math

import numpy as np

from . import avs_oracle as O

GAMMA = 5.0 / 3.0


def cell_colours(mesh):
    """Greedy colouring of the face-neighbour graph in cell order."""
    col = np.full(mesh.nc, -1, np.int64)
    for i in range(mesh.nc):
        used = {int(col[s.nbr]) for s in mesh.slots[i] if 0 <= s.nbr < i}
        c = 0
        while c in used:
            c += 1
        col[i] = c
    return col


def sweep_order(col):
    """Cells of colour 0 first, then colour 1, ...; increasing index within
    a colour.  A symmetric sweep visits this list, then its reverse."""
    return [int(i) for i in np.lexsort((np.arange(len(col)), col))]


def euler_flux(W, n, R):
    """G(W) . n = (rho U.n, rho U (U.n) + p n, (rho E + p) U.n), p = rho R T."""
    D = len(n)
    rho, U, T = O.primitive(W, R)
    p = rho * R * T
    un = float(np.dot(U, n))
    out = np.empty(D + 2)
    out[0] = rho * un
    out[1:1 + D] = rho * U * un + p * np.asarray(n)
    out[1 + D] = (W[1 + D] + p) * un
    return out


def roe_radius(rho, U, T, n, dl, gas):
    """r = |U.n| + a + 2 mu / (rho dl) (the coefficient of Eq. Roe)."""
    a = math.sqrt(GAMMA * gas.R * T)
    return abs(float(np.dot(U, n))) + a + 2.0 * O.viscosity(T, gas) / (rho * dl)


def face_radii(mesh, gas, W, face_W):
    """r per face: interior faces from the interface state W_ij, boundary
    faces from the cell's W^n with the mirrored distance."""
    r = np.zeros(mesh.nf)
    for f in range(mesh.nf):
        L, Rc = int(mesh.lr[f, 0]), int(mesh.lr[f, 1])
        n = mesh.nrm[f]
        if Rc >= 0:
            rho, U, T = O.primitive(face_W[f], gas.R)
            dl = float(np.linalg.norm(mesh.ctr[Rc] + mesh.shift[f] - mesh.ctr[L]))
        else:
            rho, U, T = O.primitive(W[L], gas.R)
            dl = 2.0 * float(np.dot(mesh.fctr[f] - mesh.ctr[L], n))
        r[f] = roe_radius(rho, U, T, n, dl, gas)
    return r


def mirror(W, n):
    """W reflected in a wall of unit normal n (normal momentum reversed)."""
    D = len(n)
    out = np.array(W, dtype=np.float64)
    m = out[1:1 + D].copy()
    out[1:1 + D] = m - 2.0 * float(np.dot(m, n)) * np.asarray(n)
    return out


def is_wall(mesh, f):
    Rc = int(mesh.lr[f, 1])
    return Rc < 0 and mesh.bc_kind[-1 - Rc] == O.WALL


def macro_sgs(mesh, dt, R, W, rhs, r, n_sweeps, order, flux=None, source=None):
    """PRSGS sweeps on the predictor (Eq. SGS_w).  ``rhs[i]`` = -sum_j A_ij
    F_ij^n (outward normals).  ``flux(W, n, R)`` is the Euler flux (the
    monatomic one by default); ``source(i, W_i + dW_i)``, if given, returns
    (d, b): an implicit source adds d to the cell's diagonal and b to its
    right-hand side (Eq. SGS_wrot).  Returns dW."""
    euler = flux or euler_flux
    nc = mesh.nc
    dW = np.zeros_like(W)
    diag = np.array([mesh.vol[i] / dt + 0.5 * sum(mesh.area[s.face] * r[s.face] for s in mesh.slots[i])
                     for i in range(nc)])
    for _ in range(n_sweeps):
        for i in list(order) + list(reversed(order)):
            acc = rhs[i].copy()
            for s in mesh.slots[i]:
                A = mesh.area[s.face]
                n_out = s.sigma * mesh.nrm[s.face]
                if s.nbr >= 0:
                    Wj, dWj = W[s.nbr], dW[s.nbr]
                elif is_wall(mesh, s.face):
                    Wj, dWj = mirror(W[i], n_out), mirror(dW[i], n_out)
                else:
                    continue
                acc -= 0.5 * A * (euler(Wj + dWj, n_out, R) - euler(Wj, n_out, R))
                acc += 0.5 * A * r[s.face] * dWj
            if source is None:
                dW[i] = acc / diag[i]
            else:
                d, b = source(i, W[i] + dW[i])
                dW[i] = (acc + b) / (diag[i] + d)
    return dW


def micro_sgs(mesh, xi, dt, tau_c, res, n_sweeps, order):
    """Symmetric Gauss-Seidel sweeps on the upwind micro system (Eq.
    SGS_phi).  ``res`` is [P, Nc, Nv], ``tau_c`` the cells' tau~.
    Returns dphi."""
    nc = mesh.nc
    dphi = np.zeros_like(res)
    diag = []
    for i in range(nc):
        d = np.full(xi.shape[0], mesh.vol[i] / dt + mesh.vol[i] / tau_c[i])
        for s in mesh.slots[i]:
            sn = s.sigma * mesh.area[s.face] * O.normal_speed(xi, mesh.nrm[s.face])
            d = d + np.where(sn >= 0, sn, 0.0)
        diag.append(d)
    for _ in range(n_sweeps):
        for i in list(order) + list(reversed(order)):
            acc = res[:, i, :].copy()
            for s in mesh.slots[i]:
                if s.nbr < 0:
                    continue
                sn = s.sigma * mesh.area[s.face] * O.normal_speed(xi, mesh.nrm[s.face])
                acc -= np.where(sn < 0, sn, 0.0)[None, :] * dphi[:, s.nbr, :]
            dphi[:, i, :] = acc / diag[i][None, :]
    return dphi


def implicit_flux(mesh, gas, W, dW, F, r, flux=None):
    """Fh_f = F_f + 1/2 [G(W~_L) - G(W_L) + G(W~_R) - G(W_R)] + 1/2 r_f (dW_L - dW_R)
    through the face normal (L to R); the outside of a boundary face as in
    the predictor (mirror state at a wall, increment 0 at the far field)."""
    euler = flux or euler_flux
    Fh = {}
    for f in F:
        L, Rc = int(mesh.lr[f, 0]), int(mesh.lr[f, 1])
        n = mesh.nrm[f]
        if Rc >= 0:
            WR, dWR = W[Rc], dW[Rc]
        elif is_wall(mesh, f):
            WR, dWR = mirror(W[L], n), mirror(dW[L], n)
        else:
            WR, dWR = None, np.zeros_like(dW[L])
        v = F[f] + 0.5 * (euler(W[L] + dW[L], n, gas.R) - euler(W[L], n, gas.R))
        if WR is not None:
            v = v + 0.5 * (euler(WR + dWR, n, gas.R) - euler(WR, n, gas.R))
        v = v + 0.5 * r[f] * (dW[L] - dWR)
        Fh[f] = v
    return Fh


def step_implicit(mesh, tree, gas, dt, Kv, phi, W, n_macro, n_micro, order=None):
    """One implicit step; returns (phi_new, W_new, diag) with diag.residual =
    |W^{n+1} - W^n| / dt per component, like the explicit step."""
    D = mesh.dim
    xi = tree.centres()
    A = tree.weights()
    if order is None:
        order = sweep_order(cell_colours(mesh))
    phif, F, diag = O.interfaces(mesh, tree, gas, dt, Kv, phi, range(mesh.nc))
    rhs = np.zeros_like(W)
    div = np.zeros_like(phi)
    for i in range(mesh.nc):
        for s in mesh.slots[i]:
            af = s.sigma * mesh.area[s.face]
            rhs[i] -= af * F[s.face]
            div[:, i, :] += af * O.normal_speed(xi, mesh.nrm[s.face])[None, :] * phif[s.face]
    r = face_radii(mesh, gas, W, diag.face_W)
    dW = macro_sgs(mesh, dt, gas.R, W, rhs, r, n_macro, order)
    Fh = implicit_flux(mesh, gas, W, dW, F, r)
    Wt = np.empty_like(W)
    for i in range(mesh.nc):
        Fs = np.zeros(D + 2)
        for s in mesh.slots[i]:
            Fs += s.sigma * mesh.area[s.face] * Fh[s.face]
        Wt[i] = W[i] - dt / mesh.vol[i] * Fs
    diag.predicted = W + dW
    res = np.empty_like(phi)
    tau_c = np.empty(mesh.nc)
    for i in range(mesh.nc):
        _, U_n, _ = O.primitive(W[i], gas.R)
        q_n = O.heat_flux(phi[:, i, :], xi, A, U_n)
        rho, U, T = O.primitive(Wt[i], gas.R)
        if not (rho > 0 and T > 0):
            raise FloatingPointError(f'non-physical state in cell {i}: rho={rho} T={T}')
        tau_c[i] = O.tau(rho, T, gas)
        gt = O.closure(O.shakhov(rho, U, T, q_n, xi, gas), Wt[i], xi, A, gas.R)
        res[:, i, :] = mesh.vol[i] * (gt - phi[:, i, :]) / tau_c[i] - div[:, i, :]
    phi_new = phi + micro_sgs(mesh, xi, dt, tau_c, res, n_micro, order)
    diag.residual = np.sqrt(np.sum((Wt - W) ** 2, axis=0)) / dt
    return phi_new, Wt, diag
