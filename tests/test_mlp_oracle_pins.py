"""Pins of the learned-weights oracle (oracle/mlp_oracle.py) against what
the mathematics fixes: exact BF16 roundings, hand-computed features, a
network whose output has a closed form, finite differences of the loss,
the closed form of the first AdamW steps, and the properties of the
softmax-KL loss and of the selection weights."""

from fractions import Fraction

import numpy as np
import pytest

from oracle import mlp_oracle as M
from paper_2608_30239_amd import instances as I


def test_parameter_count():
    assert M.N_PARAMS == 4801   # 8*64 + 64 + 64*64 + 64 + 64 + 1


@pytest.mark.parametrize("value,expected", [
    (1.0, 1.0),
    (1.0 + 2.0 ** -8, 1.0),                    # half way, kept part even: down
    (1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -6),   # half way, kept part odd: up
    (1.0 + 2.0 ** -8 + 2.0 ** -20, 1.0 + 2.0 ** -7),   # just above half: up
    (-(1.0 + 3 * 2.0 ** -8), -(1.0 + 2.0 ** -6)),
    (2.0 - 2.0 ** -9, 2.0),                    # rounds up across the exponent
    (0.0, 0.0),
])
def test_bf16_round_exact(value, expected):
    assert float(M.bf16_round(np.float32(value))) == expected


def test_bf16_round_is_nearest():
    rng = np.random.default_rng(0)
    x = rng.standard_normal(2000).astype(np.float32) * 10
    r = M.bf16_round(x)
    for xi, ri in zip(x[:200], r[:200]):
        # ri has at most 8 significant bits and no bf16 value is closer
        fr = Fraction(float(ri))
        e = int(np.floor(np.log2(abs(float(ri))))) if ri != 0 else 0
        unit = Fraction(2) ** (e - 7)
        assert (fr / unit).denominator == 1
        assert abs(Fraction(float(xi)) - fr) <= unit / 2


def test_features_by_hand():
    # 4 clones, 3 pools; rows: 0:{0,1} 1:{1,2} 2:{2} 3:{0,2}; y = (1, 0, 1)
    A = np.array([[1, 0, 0, 1],
                  [1, 1, 0, 0],
                  [0, 1, 1, 1]], np.uint8)
    inst = I.from_dense("hand", A, np.array([1, 0, 1], np.uint8), 0.05, 0.1, 0.2)
    X = M.features(inst)
    # pool sizes: 2, 2, 3
    assert X[0, :5].tolist() == [1 / 8, 1 / 8, 2 / 64, 2 / 64, 2 / 64]
    assert X[1, :5].tolist() == [1 / 8, 1 / 8, 3 / 64, 2 / 64, 3 / 64]
    assert X[2, :5].tolist() == [1 / 8, 0.0, 3 / 64, 0.0, 3 / 64]
    assert X[3, :5].tolist() == [2 / 8, 0.0, 2.5 / 64, 0.0, 2 / 64]
    # score s_i = sum d_j a_j: a+ = log(0.9/0.05), a- = log(0.1/0.95)
    ap, an = np.log(0.9) - np.log(0.05), np.log(0.1) - np.log(0.95)
    s = np.array([2 * ap + 2 * an, 2 * an + 3 * ap, 3 * ap, 2 * ap + 3 * ap])
    c = np.log(400.0) * (s - s.max()) / (s.max() - s.min())
    np.testing.assert_allclose(M.base_logits(inst), c, rtol=0, atol=1e-13)
    np.testing.assert_allclose(X[:, 5], c / 16, rtol=0, atol=1e-14)
    assert X[3, 5] == 0.0 and abs(X[0, 5] + np.log(400.0) / 16) < 1e-14   # top and bottom
    assert (X[:, 6] == 0.5).all() and (X[:, 7] == 1.0).all()


def test_base_logits_give_the_score_weights():
    inst, _ = I.tiny_plain()
    _, w = __import__("oracle.oracle", fromlist=["x"]).score_weights(inst)
    c = M.base_logits(inst)
    # a network that outputs zero gives back the paper's weights
    np.testing.assert_allclose(M.selection_weights(np.zeros(inst.n), c, 0.5), w, rtol=1e-13)
    assert abs(c.max()) == 0.0 and abs(c.min() + np.log(100.0 * inst.n)) < 1e-12


def test_features_equal_scores_give_zero():
    inst = I.identity_instance(5, 0.1, 0.1, 0.2)
    inst.y[:] = 0
    X = M.features(inst)
    assert (X[:, 5] == 0).all()
    assert (X[:, 0] == 0).all() and (X[:, 1] == 1 / 8).all()


def closed_form_net():
    """W1 = [I_8; 0], W2 = I_64, W3 = (1,...,1,0,...) over the first 8: the
    network computes sum_f relu(x_f) + b3."""
    theta = np.zeros(M.N_PARAMS)
    W1, b1, W2, b2, W3, b3 = M.split(theta)
    W1[:8, :8] = np.eye(8)
    W2[:, :] = np.eye(64)
    W3[:8] = 1.0
    b3[0] = 0.25
    return theta


def test_forward_closed_form():
    theta = closed_form_net()
    rng = np.random.default_rng(1)
    X = rng.standard_normal((50, 8))
    g, _ = M.forward(M.bf16_round(theta), X)
    np.testing.assert_allclose(g, np.maximum(X, 0).sum(axis=1) + 0.25, rtol=0, atol=1e-15)


def _random_problem(seed=2, rows=40, segs=(0, 13, 27, 40)):
    rng = np.random.default_rng(seed)
    theta = rng.uniform(-0.5, 0.5, M.N_PARAMS)
    X = rng.uniform(0, 1.5, (rows, 8))
    signal = rng.uniform(-0.05, 1.05, rows)
    base = -rng.uniform(0, 8, rows)
    seg = np.array(segs)
    t = M.targets(signal, base, seg, 0.7, 0.5, 1e-3)
    return theta, X, t, seg, base


def test_targets_normalised_and_special_cases():
    theta, X, t, seg, base = _random_problem()
    for a, b in zip(seg[:-1], seg[1:]):
        assert abs(t[a:b].sum() - 1.0) < 1e-14
    assert (t > 0).all()
    c = np.array([0.0, -1.0, -2.5, -4.0])
    # beta = 1, gamma = 0: the score softmax itself
    t1 = M.targets(np.array([0.3, 0.9, -0.2, 1.4]), c, np.array([0, 4]), 1.0, 0.0, 0.5)
    np.testing.assert_allclose(t1, np.exp(c) / np.exp(c).sum(), rtol=1e-15)
    # beta = 0, gamma = 1: proportional to clip(signal) + eps
    t2 = M.targets(np.array([0.25, 1.0, 1.3, -0.5]), c, np.array([0, 4]), 0.0, 1.0, 0.25)
    np.testing.assert_allclose(t2, np.array([0.5, 1.25, 1.25, 0.25]) / 3.25, rtol=1e-15)
    # beta = gamma = 0: uniform
    np.testing.assert_allclose(M.targets(np.zeros(4), c, np.array([0, 4]), 0.0, 0.0, 1.0), 0.25)


def test_loss_zero_at_target_and_gradient():
    rng = np.random.default_rng(3)
    f = rng.standard_normal(10)
    base = -rng.uniform(0, 5, 10)
    g = base + f
    seg = np.array([0, 4, 10])
    t = np.concatenate([np.exp(g[:4]) / np.exp(g[:4]).sum(), np.exp(g[4:]) / np.exp(g[4:]).sum()])
    loss, dg = M.loss_and_dg(f, base, t, seg)
    assert abs(loss) < 1e-15 and np.max(np.abs(dg)) < 1e-15
    t2 = M.targets(rng.uniform(0, 1, 10), base, seg, 0.5, 0.5, 1e-3)
    loss, dg = M.loss_and_dg(f, base, t2, seg)
    assert loss > 0
    h = 1e-6
    for i in range(10):
        e = np.zeros(10); e[i] = h
        fd = (M.loss_and_dg(f + e, base, t2, seg)[0] - M.loss_and_dg(f - e, base, t2, seg)[0]) / (2 * h)
        assert abs(fd - dg[i]) < 1e-8


def test_backward_matches_finite_differences():
    theta, X, t, seg, base = _random_problem()

    def loss_of(th):
        g, _ = M.forward(th, X)
        return M.loss_and_dg(g, base, t, seg)[0]

    g, c = M.forward(theta, X)
    # keep away from ReLU kinks so that central differences are valid
    assert min(np.min(np.abs(c["z1"])), np.min(np.abs(c["z2"]))) > 1e-4
    _, dg = M.loss_and_dg(g, base, t, seg)
    grad = M.backward(theta, X, dg)
    rng = np.random.default_rng(4)
    idx = np.concatenate([rng.choice(512, 20, replace=False),            # W1
                          512 + rng.choice(64, 8, replace=False),         # b1
                          576 + rng.choice(4096, 40, replace=False),      # W2
                          4672 + rng.choice(64, 8, replace=False),        # b2
                          4736 + rng.choice(64, 8, replace=False),        # W3
                          [4800]])                                        # b3
    h = 1e-6
    for i in idx:
        e = np.zeros_like(theta); e[i] = h
        fd = (loss_of(theta + e) - loss_of(theta - e)) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-7 + 1e-5 * abs(fd), (i, fd, grad[i])


def test_adamw_first_steps_closed_form():
    theta = np.array([0.5, -1.0, 2.0])
    g1 = np.array([0.2, -0.3, 0.0])
    lr, b1, b2, eps, wd = 0.01, 0.9, 0.999, 1e-8, 0.1
    th1, m1, v1 = M.adamw_step(theta, np.zeros(3), np.zeros(3), g1, 1, lr, b1, b2, eps, wd)
    # step 1: mhat = g, vhat = g^2, so the move is lr (g / (|g| + eps) + wd theta)
    np.testing.assert_allclose(th1, theta - lr * (g1 / (np.abs(g1) + eps) + wd * theta), rtol=1e-15)
    g2 = np.array([0.1, 0.4, -0.5])
    th2, _, _ = M.adamw_step(th1, m1, v1, g2, 2, lr, b1, b2, eps, wd)
    m2 = b1 * (1 - b1) * g1 + (1 - b1) * g2
    v2 = b2 * (1 - b2) * g1 ** 2 + (1 - b2) * g2 ** 2
    upd = (m2 / (1 - b1 ** 2)) / (np.sqrt(v2 / (1 - b2 ** 2)) + eps)
    np.testing.assert_allclose(th2, th1 - lr * (upd + wd * th1), rtol=1e-14)


def test_selection_weights_floor_and_sum():
    rng = np.random.default_rng(5)
    g = rng.standard_normal(100) * 5
    w = M.selection_weights(g, np.zeros(100), 0.5)
    assert abs(w.sum() - 1) < 1e-14 and (w >= 0.5 / 100).all()
    np.testing.assert_allclose(M.selection_weights(np.full(7, 3.0), np.zeros(7)), 1 / 7, rtol=1e-15)
    # only c + f matters
    np.testing.assert_allclose(M.selection_weights(g - 1.5, np.full(100, 1.5)), w, rtol=1e-14)
