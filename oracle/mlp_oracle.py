"""FP64 CPU oracle of the learned refinement proposal.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no
code with the GPU library and imports nothing from it.

The learned proposal is not part of the paper.  It predicts, for every leaf
of the shared velocity tree, the decision that the criterion of Sec. 3.4
(Eqs. criterion_rho, criterion_e, criterion_mk and rules (a)-(c)) takes after
the brother-group rule of Sec. 3.1: keep (class 0), split (1) or merge (2).
The criterion reads every (cell, leaf) value of the distribution; the
proposal reads only the leaf's own geometry and a 24-number summary of the
macroscopic fields.  This module is the definition of that form:

* features of leaf k (28): its centre relative to the box centre over the
  box half-width (2), its width over the box width (1), level / max level
  (1), and the lower quantiles at 0, 1/5, ..., 1 (element j (n-1) / 5 of the
  sorted values, integer division) of rho / rho_ref, U_x / sqrt(R T_ref),
  U_y / sqrt(R T_ref) and T / T_ref over the cells (24);
* network 28 -> 128 -> 128 -> 3 with ReLU after both hidden layers; inputs,
  weights and hidden activations are held in bfloat16 (round to nearest,
  ties to even), biases and logits in float32;
* loss: mean softmax cross-entropy over a batch; backward deltas are
  rounded to bfloat16 where the forward rounds its activations;
* optimiser: Adam with bias correction (Kingma and Ba, 2015);
* proposal: class of the largest logit (the lowest class on ties), split only
  below the maximum level, merge only above the roots, then the brother-group
  rule of Sec. 3.1;
* judge: the proposal is accepted only if, on the proposed leaf set, the
  discrete density and energy of the Maxwellian of every probe state (given
  states plus the cells holding the minimum and maximum of each field) are
  within a tolerance of their exact values; otherwise the plain criterion
  decides.

``bf16=False`` runs the same network in plain float64 (used to pin the
gradient against finite differences).  Every array is float64.
"""
from __future__ import annotations

import math

import numpy as np

NIN, NH, NOUT = 28, 128, 3
SHAPES = [("W1", (NIN, NH)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NH, NOUT)), ("b3", (NOUT,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)   # 20611


def unpack(p):
    """Flat parameter vector -> dict of views (row-major, input index first)."""
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(p[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


def bf16_round(x):
    """Nearest bfloat16 (8 significant bits, ties to even) of float64 values,
    returned as float64.  Written from the format's definition: x = m 2^e with
    m in [0.5, 1); keep round(m 2^8) with halves to even."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)
    return np.ldexp(np.rint(m * 256.0), e - 8)


def lower_quantile(a, j, parts=5):
    """Element j (n - 1) // parts of the ascending sort of a."""
    s = np.sort(np.asarray(a, dtype=np.float64))
    return s[(j * (len(s) - 1)) // parts]


def cell_fields(prim, R, rho_ref, T_ref):
    """rho / rho_ref, U_x / sqrt(R T_ref), U_y / sqrt(R T_ref), T / T_ref."""
    c = math.sqrt(R * T_ref)
    return [prim[:, 0] / rho_ref, prim[:, 1] / c, prim[:, 2] / c, prim[:, 3] / T_ref]


def primitive_2d(W, R):
    """(rho, U, T) of 2-D conserved moments, rho E = rho |U|^2 / 2 + 3/2 rho R T
    (three translational degrees of freedom carried by G and H, Sec. 2.2)."""
    rho = W[:, 0]
    U = W[:, 1:3] / rho[:, None]
    ke = U[:, 0] * U[:, 0] + U[:, 1] * U[:, 1]
    T = (W[:, 3] - 0.5 * rho * ke) / (1.5 * rho * R)
    return np.column_stack([rho, U, T])


def features(level, idx, base, max_level, prim, R, rho_ref, T_ref):
    """Feature rows [n_leaves, 28] (float64, before the bfloat16 rounding)."""
    level = np.asarray(level, np.int64)
    idx = np.asarray(idx, np.int64).reshape(-1, 2)
    n = len(level)
    F = np.zeros((n, NIN))
    scale = 2.0 ** level
    for d in range(2):
        F[:, d] = (2 * idx[:, d] + 1) / (base[d] * scale) - 1.0
    F[:, 2] = 1.0 / (base[0] * scale)
    F[:, 3] = level / max_level if max_level > 0 else 0.0
    for f, a in enumerate(cell_fields(prim, R, rho_ref, T_ref)):
        for j in range(6):
            F[:, 4 + 6 * f + j] = lower_quantile(a, j)
    return F


def forward(p, X, bf16=True):
    """Logits [n, 3] and the values the backward pass needs."""
    r = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    q = unpack(p)
    X = r(X)
    W1, W2, W3 = r(q["W1"]), r(q["W2"]), r(q["W3"])
    H1 = r(np.maximum(X @ W1 + q["b1"], 0.0))
    H2 = r(np.maximum(H1 @ W2 + q["b2"], 0.0))
    Z = H2 @ W3 + q["b3"]
    return Z, (X, H1, H2, W1, W2, W3)


def loss_and_grad(p, X, y, bf16=True):
    """Mean softmax cross-entropy and its gradient (flat, like p)."""
    r = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    y = np.asarray(y, np.int64)
    Z, (X, H1, H2, W1, W2, W3) = forward(p, X, bf16)
    n = len(y)
    zmax = Z.max(axis=1, keepdims=True)
    E = np.exp(Z - zmax)
    S = E.sum(axis=1, keepdims=True)
    P = E / S
    loss = float(np.mean(np.log(S[:, 0]) + zmax[:, 0] - Z[np.arange(n), y]))
    onehot = np.zeros_like(P)
    onehot[np.arange(n), y] = 1.0
    dZ = r((P - onehot) / n)
    g = {"W3": H2.T @ dZ, "b3": dZ.sum(axis=0)}
    dH2 = r((dZ @ W3.T) * (H2 > 0))
    g["W2"], g["b2"] = H1.T @ dH2, dH2.sum(axis=0)
    dH1 = r((dH2 @ W2.T) * (H1 > 0))
    g["W1"], g["b1"] = X.T @ dH1, dH1.sum(axis=0)
    flat = np.concatenate([g[name].ravel() for name, _ in SHAPES])
    return loss, flat


def adam(p, m, v, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba, 2015, Algorithm 1), t counted from 1."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def labels_from_flags(eff):
    """Effective flags (+1 split, 0 keep, -1 merge) -> classes (1, 0, 2)."""
    eff = np.asarray(eff)
    return np.where(eff == 1, 1, np.where(eff == -1, 2, 0)).astype(np.int64)


def proposal_raw(Z, level, max_level):
    """Raw flags from logits: arg max (lowest class on ties), split only
    below the maximum level, merge only above the roots."""
    c = np.argmax(Z, axis=1)
    raw = np.where(c == 1, 1, np.where(c == 2, -1, 0)).astype(np.int8)
    level = np.asarray(level)
    raw[(raw == 1) & (level >= max_level)] = 0
    raw[(raw == -1) & (level <= 0)] = 0
    return raw


def probe_states(prim, given=None):
    """Given probe states, then the cells holding the minimum and the maximum
    of rho, U_x, U_y and T (lowest cell index on ties), as primitive rows."""
    rows = [] if given is None else [np.asarray(g, np.float64) for g in given]
    for f in range(4):
        rows.append(prim[int(np.argmin(prim[:, f]))])
        rows.append(prim[int(np.argmax(prim[:, f]))])
    return np.array(rows)


def tail_errors(xi, A, probes, R):
    """Relative error of the discrete density and energy of each probe's
    Maxwellian on a leaf set (centres xi [n, 2], areas A [n]).  The 2-D
    reduced pair carries g and H = R T g (Sec. 2.2), so the energy is
    sum A (|xi|^2 g + R T g) / 2 against rho |U|^2 / 2 + 3/2 rho R T."""
    out = []
    for pr in probes:
        rho, U, T = pr[0], pr[1:3], pr[3]
        RT = R * T
        c2 = (xi[:, 0] - U[0]) ** 2 + (xi[:, 1] - U[1]) ** 2
        g = rho / (2.0 * math.pi * RT) * np.exp(-c2 / (2.0 * RT))
        x2 = xi[:, 0] ** 2 + xi[:, 1] ** 2
        s0 = np.sum(A * g)
        se = np.sum(A * 0.5 * (x2 * g + RT * g))
        rhoE = 0.5 * rho * (U[0] ** 2 + U[1] ** 2) + 1.5 * rho * RT
        out.append(max(abs(s0 - rho) / rho, abs(se - rhoE) / rhoE))
    return np.array(out)
