"""Pins of the learned-proposal oracle against closed forms, an independent
rounding route, finite differences and brute force (CPU only)."""
import math

import numpy as np
import pytest

from oracle import avs_oracle as O
from oracle import mlp_oracle as M


def rand_params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    parts = []
    for name, shp in M.SHAPES:
        fan_in = shp[0] if len(shp) == 2 else 1
        s = scale * math.sqrt(2.0 / fan_in) if len(shp) == 2 else 0.1 * scale
        parts.append(rng.uniform(-s, s, size=int(np.prod(shp))))
    return np.concatenate(parts)


def test_parameter_count():
    assert M.NPARAM == 28 * 128 + 128 + 128 * 128 + 128 + 128 * 3 + 3 == 20611


def test_bf16_round_hand_values():
    e = 2.0 ** -8
    assert M.bf16_round(1.0) == 1.0
    assert M.bf16_round(1.0 + e) == 1.0                  # halfway, even neighbour is 1
    assert M.bf16_round(1.0 + 3 * e) == 1.0 + 4 * e      # halfway, even neighbour is 1 + 2^-6
    assert M.bf16_round(1.0 + 1.5 * e) == 1.0 + 2 * e    # above halfway
    assert M.bf16_round(-3.0) == -3.0
    assert M.bf16_round(0.0) == 0.0
    assert M.bf16_round(1.0 / 3.0) == 0.333984375        # 0x3EAB


def test_bf16_round_matches_integer_route_on_float32():
    # independent route: round-to-nearest-even on the top 16 bits of float32
    rng = np.random.default_rng(1)
    x = (rng.standard_normal(20000) * 10.0 ** rng.uniform(-20, 20, 20000)).astype(np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    ref = r.astype(np.uint32).view(np.float32).astype(np.float64)
    np.testing.assert_array_equal(M.bf16_round(x.astype(np.float64)), ref)


def test_lower_quantile_definition():
    rng = np.random.default_rng(2)
    for n in (1, 2, 5, 6, 7, 11, 100, 1001):
        a = rng.integers(0, 7, n).astype(float)      # many ties
        for j in range(6):
            v = M.lower_quantile(a, j)
            k = j * (n - 1) // 5
            assert np.sum(a < v) <= k < np.sum(a <= v)
    a = rng.standard_normal(1001)                      # j (n-1) / 5 integral: library 'lower' agrees
    for j in range(6):
        assert M.lower_quantile(a, j) == np.quantile(a, j / 5, method="lower")


def test_features_against_tree_geometry():
    tree = O.base_forest(2, (-3.0, -5.0), (7.0, 5.0), (4, 6), 2)
    # split the first root twice over to get several levels
    lev = np.array([2, 2, 1, 0], np.int64)
    idx = np.array([[0, 0], [1, 0], [1, 1], [3, 5]], np.int64)
    t = O.Tree(2, tree.lo, tree.hi, tree.base, tree.max_level, lev, idx)
    prim = np.array([[1.0, 0.5, -0.5, 2.0], [3.0, 1.5, 0.0, 1.0], [2.0, -1.0, 2.0, 4.0]])
    F = M.features(lev, idx, t.base, t.max_level, prim, 0.5, 2.0, 1.0)
    lo, hi = np.array(t.lo), np.array(t.hi)
    ctr = 0.5 * (lo + hi)
    half = 0.5 * (hi - lo)
    np.testing.assert_allclose(F[:, :2], (t.centres() - ctr) / half, rtol=0, atol=1e-15)
    np.testing.assert_allclose(F[:, 2], t.widths()[:, 0] / (hi[0] - lo[0]), rtol=1e-15)
    np.testing.assert_array_equal(F[:, 3], lev / 2.0)
    # quantiles of rho / rho_ref: sorted (0.5, 1.0, 1.5); n = 3 -> indices 0,0,0,1,1,2
    np.testing.assert_array_equal(F[0, 4:10], [0.5, 0.5, 0.5, 1.0, 1.0, 1.5])
    c = math.sqrt(0.5)
    np.testing.assert_array_equal(F[0, 10:16], np.array([-1.0, -1.0, -1.0, 0.5, 0.5, 1.5]) / c)
    np.testing.assert_array_equal(F[0, 22:28], [1.0, 1.0, 1.0, 2.0, 2.0, 4.0])
    assert np.all(F[1:, 4:] == F[0, 4:])


def test_softmax_cross_entropy_at_zero_weights():
    p = np.zeros(M.NPARAM)
    X = np.random.default_rng(3).standard_normal((10, 28))
    y = np.array([0, 1, 2, 0, 0, 1, 2, 2, 2, 1])
    loss, g = M.loss_and_grad(p, X, y, bf16=False)
    assert abs(loss - math.log(3.0)) < 1e-15
    q = M.unpack(g)
    onehot = np.eye(3)[y]
    np.testing.assert_allclose(q["b3"], np.mean(1.0 / 3.0 - onehot, axis=0), atol=1e-16)
    assert np.all(q["W1"] == 0) and np.all(q["W2"] == 0)      # no signal through zero weights


def test_gradient_matches_central_differences_fp64():
    p = rand_params(4)
    rng = np.random.default_rng(5)
    X = rng.standard_normal((16, 28))
    y = rng.integers(0, 3, 16)
    loss, g = M.loss_and_grad(p, X, y, bf16=False)
    picks = np.concatenate([rng.choice(M.NPARAM, 60, replace=False), np.arange(M.NPARAM - 3, M.NPARAM)])
    h = 1e-6
    for k in picks:
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (M.loss_and_grad(pp, X, y, bf16=False)[0] - M.loss_and_grad(pm, X, y, bf16=False)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1e-3, abs(g[k])) + 1e-9, (k, fd, g[k])


def test_bf16_network_close_to_fp64_network():
    # same bf16-representable weights and inputs: only activation/delta rounding differs
    p = M.bf16_round(rand_params(6))
    rng = np.random.default_rng(7)
    X = M.bf16_round(rng.standard_normal((64, 28)))
    y = rng.integers(0, 3, 64)
    l1, g1 = M.loss_and_grad(p, X, y, bf16=True)
    l0, g0 = M.loss_and_grad(p, X, y, bf16=False)
    assert abs(l1 - l0) < 1e-2 * abs(l0)
    for name, _ in M.SHAPES:
        a, b = M.unpack(g1)[name], M.unpack(g0)[name]
        assert np.linalg.norm(a - b) <= 5e-2 * np.linalg.norm(b), name


def test_adam_constant_gradient_closed_form():
    # m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2, so each step moves lr g / (|g| + eps)
    rng = np.random.default_rng(8)
    p0 = rng.standard_normal(50)
    g = rng.standard_normal(50)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    lr, eps = 1e-3, 1e-8
    for t in range(1, 8):
        p, m, v = M.adam(p, m, v, g, t, lr, eps=eps)
        np.testing.assert_allclose(p, p0 - t * lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-15)


def test_labels_and_proposal_rules():
    np.testing.assert_array_equal(M.labels_from_flags([1, 0, -1, 0]), [1, 0, 2, 0])
    Z = np.array([[1.0, 2.0, 0.0], [0.0, 0.0, 5.0], [3.0, 3.0, 3.0], [0.0, 9.0, 1.0], [0.0, 0.0, 7.0]])
    raw = M.proposal_raw(Z, level=np.array([1, 2, 1, 3, 0]), max_level=3)
    np.testing.assert_array_equal(raw, [1, -1, 0, 0, 0])   # tie -> keep; no split at max; no merge of a root


def test_tail_errors_fine_and_coarse_meshes():
    # midpoint sums of a Maxwellian on a fine uniform mesh are exact to round-off
    R = 0.5
    pr = np.array([[1.3, 0.4, -0.2, 1.1]])
    for n, expect_small in ((128, True), (8, False)):
        t = O.base_forest(2, (-6.0, -6.0), (6.0, 6.0), (n, n), 0)
        err = M.tail_errors(t.centres(), t.weights(), pr, R)
        assert (err[0] < 1e-10) == expect_small, (n, err)
    # a box that cuts the Maxwellian loses mass: error of the order of the lost tail
    t = O.base_forest(2, (-1.0, -6.0), (6.0, 6.0), (128, 128), 0)
    err = M.tail_errors(t.centres(), t.weights(), pr, R)[0]
    lost = 0.5 * math.erfc((0.4 + 1.0) / math.sqrt(2 * R * 1.1))
    assert 0.5 * lost < err < 5 * lost


def test_probe_states_pick_extreme_cells():
    prim = np.array([[1.0, 0.0, 0.0, 1.0], [0.5, 2.0, -1.0, 3.0], [2.0, -1.0, 1.0, 0.5], [0.5, 2.0, 4.0, 3.0]])
    P = M.probe_states(prim, given=[[9.0, 0.0, 0.0, 9.0]])
    assert P.shape == (9, 4)
    np.testing.assert_array_equal(P[0], [9.0, 0.0, 0.0, 9.0])
    np.testing.assert_array_equal(P[1:], prim[[1, 2, 2, 1, 1, 3, 2, 1]])
