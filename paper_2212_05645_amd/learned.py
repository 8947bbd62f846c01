"""Training driver of the learned refinement proposal.

Collects (features, plain-criterion decision) pairs on the device while a
case runs, then trains the network with the library's own kernels (fused
forward/backward per 64-sample tile on MFMA, deterministic gradient
reduction, Adam).  Host code here only draws the initial weights and the
minibatch order from seeded generators and sequences library calls.
"""
from __future__ import annotations

import math

import numpy as np

from . import avs

NPARAM = 20611
SHAPES = [(28, 128), (128,), (128, 128), (128,), (128, 3), (3,)]


def init_params(seed=0):
    """He-uniform weights (bound sqrt(6 / fan_in)), zero biases, float32."""
    rng = np.random.default_rng(seed)
    parts = []
    for shp in SHAPES:
        if len(shp) == 2:
            b = math.sqrt(6.0 / shp[0])
            parts.append(rng.uniform(-b, b, size=shp[0] * shp[1]))
        else:
            parts.append(np.zeros(shp[0]))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == NPARAM
    return p


class Dataset:
    """Device rows of features (bfloat16 bit patterns) and effective flags."""

    def __init__(self, capacity, device="cuda:0"):
        import torch
        self.torch = torch
        self.feat = torch.zeros((capacity, 32), dtype=torch.int16, device=device)
        self.flags = torch.zeros(capacity, dtype=torch.int8, device=device)
        self.n = 0
        self.events = []          # (start, count) per adaptation event

    def room(self):
        return self.feat.shape[0] - self.n


def _label_event(case, mlp, ds, C1, C2, probes):
    n = case.nleaves()
    if ds.room() < n:
        return False
    case.features(mlp, out=ds.feat[ds.n:])
    case.adapt(C1, C2, probes=probes, flags_out=ds.flags[ds.n:])
    ds.events.append((ds.n, n))
    ds.n += n
    return True


def collect(case, mlp, ds, C1, C2, events, sweeps_between, base, levels=(0, 1, 2), probes=None, exact_restore=True):
    """Run ``events`` adaptation events on ``case``.  At each event, store
    the features and the plain criterion's effective flags (a) of the current
    leaves and (b) of uniform trees at each of ``levels`` (``base`` = the
    level-0 roots as (level, idx)) carrying the moment-closed Maxwellian of
    the current W, so that every decision (split, keep, merge) is sampled;
    then restore the state (exactly, or from W when ``exact_restore`` is
    false), remap the current-tree decision (correction 2) and advance
    ``sweeps_between`` sweeps."""
    for _ in range(events):
        L = case.leaves()
        vdf, W = case.get_state() if exact_restore else (None, case.get_W())
        for lv in levels:
            case.set_leaves(*base)
            for _ in range(lv):
                case.adapt(-1.0, -2.0)          # M_k >= 0 > C1: split every leaf
                case.remap(0)
            case.set_state(None, W)
            if not _label_event(case, mlp, ds, C1, C2, probes):
                break
        case.set_leaves(L['level'], L['idx'])
        case.set_state(vdf, W)
        if not _label_event(case, mlp, ds, C1, C2, probes):
            break
        case.remap(2)
        if sweeps_between:
            case.step(sweeps_between)


def balanced_epoch(flags, pool, g, torch):
    """One epoch's row order in which every class (keep, split, merge) present
    in ``pool`` is drawn as often as the largest one: the rows of the smaller
    classes repeat (drawn with replacement from the seeded generator ``g``),
    so that the mean cross-entropy weighs the three decisions alike."""
    lab = flags[pool.long()]
    parts = [pool[lab == c] for c in (0, 1, -1)]
    parts = [p for p in parts if len(p) > 0]
    n = max(len(p) for p in parts)
    out = []
    for p in parts:
        if len(p) == n:
            out.append(p)
        else:
            out.append(p[torch.randint(len(p), (n,), generator=g)])
    cat = torch.cat(out)
    return cat[torch.randperm(len(cat), generator=g)]


def train(mlp, ds, epochs=3, batch=8192, lr=2e-3, seed=0, rows=None, log_every=0, balance=False):
    """Adam over shuffled minibatches of the dataset rows ``rows`` (all rows
    by default); with ``balance`` each epoch draws the three decisions
    equally often (balanced_epoch).  Returns the losses sampled every
    ``log_every`` steps."""
    torch = ds.torch
    g = torch.Generator().manual_seed(seed)
    pool = torch.arange(ds.n, dtype=torch.int32) if rows is None else torch.as_tensor(rows, dtype=torch.int32)
    flags = ds.flags[:ds.n].cpu() if balance else None
    losses, step = [], 0
    for _ in range(epochs):
        order = balanced_epoch(flags, pool, g, torch) if balance else pool[torch.randperm(len(pool), generator=g)]
        perm = order.to(ds.feat.device)
        for s in range(0, len(perm), batch):
            r = perm[s:s + batch]
            want = log_every and step % log_every == 0
            out = mlp.train_step(ds.feat, ds.flags, rows=r, lr=lr, loss=bool(want))
            if want:
                losses.append(out)
            step += 1
    return losses


def confusion(mlp, ds, rows=None):
    """3x3 counts [label, predicted class] of the network on dataset rows."""
    torch = ds.torch
    idx = torch.arange(ds.n, device=ds.feat.device) if rows is None else torch.as_tensor(rows, device=ds.feat.device)
    feat = ds.feat[idx].contiguous()
    z = mlp.forward(feat)
    pred = torch.argmax(z, dim=1)
    f = ds.flags[idx].to(torch.int64)
    lab = torch.where(f == 1, 1, torch.where(f == -1, 2, 0))
    cm = torch.zeros(9, dtype=torch.int64, device=feat.device)
    cm.index_add_(0, lab * 3 + pred, torch.ones_like(lab))
    return cm.view(3, 3).cpu().numpy()
