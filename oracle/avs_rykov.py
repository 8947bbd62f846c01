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
