"""Seeded velocity-tree generators shared by both implementations' tests.

A tree is given as its leaves: ``level`` [n] and ``idx`` [n, dim] (integer
index of the leaf in the uniform grid of ``base * 2**level`` cells per axis),
listed in depth-first order, i.e. ascending Z-order (bit-interleaved, x
lowest) of each leaf's lower corner on the finest grid.  Only integer
bookkeeping happens here: no velocity, weight or distribution value.
"""
from __future__ import annotations

import numpy as np


def _z_key(level, idx, max_level):
    X = np.asarray(idx, np.int64) << (max_level - np.asarray(level, np.int64))[:, None]
    dim = X.shape[1]
    key = np.zeros(len(X), dtype=np.uint64)
    for b in range(64 // dim):
        for d in range(dim):
            key |= ((X[:, d] >> b) & 1).astype(np.uint64) << np.uint64(dim * b + d)
    return key


def _ordered(level, idx, max_level):
    o = np.argsort(_z_key(level, idx, max_level), kind="stable")
    return level[o], idx[o]


def roots(dim, base):
    """The level-0 roots of a base[0] x ... forest."""
    grids = np.meshgrid(*[np.arange(int(b)) for b in base[:dim]], indexing="ij")
    idx = np.stack([g.ravel() for g in grids], 1).astype(np.int64)
    return np.zeros(len(idx), np.int64), idx


def _split(level, idx, which):
    """Replace the leaves flagged in ``which`` by their 2^dim children."""
    dim = idx.shape[1]
    keep_l, keep_i = level[~which], idx[~which]
    pl, pi = level[which], idx[which]
    kids_l, kids_i = [], []
    for c in range(2 ** dim):
        bits = np.array([(c >> d) & 1 for d in range(dim)], np.int64)
        kids_l.append(pl + 1)
        kids_i.append(2 * pi + bits)
    return np.concatenate([keep_l] + kids_l), np.concatenate([keep_i] + kids_i)


def random_tree(dim, base, max_level, seed, rounds, p=0.35):
    """``rounds`` passes, each splitting every leaf below max_level with
    probability p (seeded)."""
    rng = np.random.default_rng(seed)
    level, idx = roots(dim, base)
    for _ in range(rounds):
        which = (rng.random(len(level)) < p) & (level < max_level)
        level, idx = _split(level, idx, which)
    return _ordered(level, idx, max_level)


def resolved_tree(dim, base, max_level, seed, p=0.35):
    """Every root split once, then a random fraction of the leaves again."""
    level, idx = roots(dim, base)
    if max_level >= 1:
        level, idx = _split(level, idx, np.ones(len(level), bool))
    rng = np.random.default_rng(seed)
    which = (rng.random(len(level)) < p) & (level < max_level)
    level, idx = _split(level, idx, which)
    return _ordered(level, idx, max_level)


def sized_tree(dim, base, max_level, seed, target):
    """Random refinement, one level at a time, until about ``target`` leaves."""
    rng = np.random.default_rng(seed)
    level, idx = roots(dim, base)
    while len(level) < target:
        room = (target - len(level)) / (2 ** dim - 1)
        cand = np.flatnonzero(level < max_level)
        if len(cand) == 0:
            break
        take = rng.permutation(cand)[:max(1, min(len(cand), int(room)))]
        which = np.zeros(len(level), bool)
        which[take] = True
        level, idx = _split(level, idx, which)
    return _ordered(level, idx, max_level)
