"""GPU parity of the learned-weights kernels (features, forward, loss and
gradient, AdamW, weights from the network) against the FP64 oracle in
oracle/mlp_oracle.py.

Tolerances follow from the arithmetic: the kernels accumulate in FP32
(unit roundoff 2^-24) over at most 64 terms per unit, and over the rows of
a chunk then over blocks for the gradient; the oracle is FP64.  Features are
FP64 values rounded once to FP32.  BF16 roundings and the integer masses
derived from given weights are compared exactly."""

import numpy as np
import pytest

from oracle import mlp_oracle as MO
from oracle import oracle as O
from paper_2608_30239_amd import instances as I

pytestmark = pytest.mark.gpu

N = pytest.importorskip("paper_2608_30239_amd.native")


@pytest.fixture(scope="module", autouse=True)
def _lib():
    N.load()


def bf16_bits(x32):
    return (MO.bf16_round(x32).view(np.uint32) >> 16).astype(np.uint16)


def some_instances():
    hand = I.from_dense("hand", np.array([[1, 0, 0, 1], [1, 1, 0, 0], [0, 1, 1, 1]], np.uint8),
                        np.array([1, 0, 1], np.uint8), 0.05, 0.1, 0.2)
    tiny, _ = I.tiny_plain()
    paper, _ = I.paper_shaped()
    big = I.make_instance("u3000", 3000, 225, (3, 7), 5, 0.12, 0.07, prior=5 / 3000, seed=9)
    eq = I.identity_instance(5, 0.1, 0.1, 0.2)
    eq.y[:] = 0
    return [hand, tiny, paper, big, eq]


@pytest.mark.parametrize("k", range(5))
def test_features_match_oracle(k):
    inst = some_instances()[k]
    dec = N.Decoder(inst)
    try:
        X, c = N.mcpd_features(dec)
    finally:
        dec.close()
    ref = MO.features(inst)
    # FP64 values rounded once to FP32 (the base logits may differ from the
    # oracle's in the last bit of log(100 n))
    np.testing.assert_allclose(c, MO.base_logits(inst), rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(X, ref.astype(np.float32), rtol=2.0 ** -23, atol=1e-12)
    assert np.array_equal(X[:, [0, 1, 2, 3, 4, 6, 7]], ref[:, [0, 1, 2, 3, 4, 6, 7]].astype(np.float32))


def test_forward_and_bf16_copy():
    theta = I.mlp_init(1)
    net = N.Mlp(theta)
    try:
        master, bf = net.params()
        assert np.array_equal(master, theta)
        assert np.array_equal(bf, bf16_bits(theta))
        rng = np.random.default_rng(2)
        for rows in (1, 255, 256, 257, 10007):
            X = rng.uniform(0, 2, (rows, 8)).astype(np.float32)
            g = net.forward(X)
            ref, c = MO.forward(MO.bf16_round(theta), X.astype(np.float64))
            # FP32 accumulation over <= 65 terms per unit: a few hundred units
            # of 2^-24 of the magnitudes that flow into g
            W3 = MO.split(MO.bf16_round(theta).astype(np.float64))[4]
            scale = 1.0 + np.abs(c["h2"]) @ np.abs(W3) + np.abs(ref)
            assert np.all(np.abs(g - ref) <= 1e-5 * scale), rows
    finally:
        net.close()


def _training_rows(seed=3, sizes=(1, 255, 256, 257, 3000)):
    rng = np.random.default_rng(seed)
    rows = sum(sizes)
    X = rng.uniform(0, 1.5, (rows, 8)).astype(np.float32)
    signal = rng.uniform(-0.05, 1.05, rows)
    base = -rng.uniform(0, 12, rows)
    seg = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return X, base, signal, seg


@pytest.mark.parametrize("beta,gamma,eps", [(1.0, 0.0, 1e-3), (0.75, 0.5, 1e-2), (0.0, 1.0, 1e-4)])
def test_loss_and_gradient_match_oracle(beta, gamma, eps):
    theta = I.mlp_init(4)
    X, base, signal, seg = _training_rows()
    net = N.Mlp(theta)
    try:
        net.set_training_rows(X, base, signal, seg, beta, gamma, eps)
        loss, grad = net.loss_grad()
    finally:
        net.close()
    tb = MO.bf16_round(theta).astype(np.float64)
    g, _ = MO.forward(tb, X.astype(np.float64))
    t = MO.targets(signal, base, seg, beta, gamma, eps)
    ref_loss, dg = MO.loss_and_dg(g, base, t, seg)
    ref_grad = MO.backward(tb, X.astype(np.float64), dg)
    assert abs(loss - ref_loss) <= 1e-5 * abs(ref_loss)
    assert np.max(np.abs(grad - ref_grad)) <= 1e-4 * np.max(np.abs(ref_grad))


def test_single_row_segments_have_zero_loss():
    theta = I.mlp_init(5)
    X, base, signal, _ = _training_rows(sizes=(1, 1, 1))
    net = N.Mlp(theta)
    try:
        net.set_training_rows(X, base, signal, np.array([0, 1, 2, 3]))
        loss, grad = net.loss_grad()
    finally:
        net.close()
    assert abs(loss) < 1e-12 and np.max(np.abs(grad)) < 1e-12


def test_adamw_steps_match_oracle():
    theta = I.mlp_init(6)
    X, base, signal, seg = _training_rows(seed=7)
    hp = dict(lr=1e-2, beta1=0.9, beta2=0.99, eps=1e-6, weight_decay=0.05)
    net = N.Mlp(theta)
    try:
        net.set_training_rows(X, base, signal, seg, 0.75, 0.5, 1e-2)
        th = theta.astype(np.float64)
        m = np.zeros_like(th)
        v = np.zeros_like(th)
        for step in (1, 2, 3):
            _, grad = net.loss_grad()
            net.train(1, **hp)
            master, bf = net.params()
            th, m, v = MO.adamw_step(th, m, v, grad.astype(np.float64), step, hp["lr"], hp["beta1"],
                                     hp["beta2"], hp["eps"], hp["weight_decay"])
            assert np.max(np.abs(master - th)) <= 1e-6 * (1 + np.max(np.abs(th)))
            assert np.array_equal(bf, bf16_bits(master))
            th = master.astype(np.float64)   # continue from the device state
    finally:
        net.close()


def test_training_lowers_the_loss():
    theta = I.mlp_init(8)
    X, base, signal, seg = _training_rows(seed=9, sizes=(700, 900, 1300))
    net = N.Mlp(theta)
    try:
        net.set_training_rows(X, base, signal, seg, 0.5, 0.5, 1e-3)
        hist = net.train(150, lr=3e-3)
        loss, _ = net.loss_grad()
    finally:
        net.close()
    assert hist[0] > 0 and loss < 0.8 * hist[0]
    assert np.all(np.isfinite(hist))


def test_learned_weights_match_oracle_and_feed_the_sampler():
    inst, rp = I.paper_shaped()
    theta = I.mlp_init(10)
    net = N.Mlp(theta)
    dec = N.Decoder(inst)
    try:
        X, c = N.mcpd_features(dec)
        w = net.apply(dec, alpha=0.5)
        _, mass = dec.weights()
    finally:
        dec.close()
        net.close()
    f, _ = MO.forward(MO.bf16_round(theta), X.astype(np.float64))
    ref = MO.selection_weights(f, c, 0.5)
    assert np.max(np.abs(w - ref) / ref) <= 1e-5
    assert w.min() >= 0.5 / inst.n and abs(w.sum() - 1) < 1e-12
    assert np.array_equal(mass, O.quantize(w))


@pytest.mark.parametrize("make", [I.tiny_plain, I.paper_shaped])
def test_zero_network_gives_back_the_score_weights(make):
    inst, _ = make()
    net = N.Mlp(np.zeros(N.MLP_PARAMS, np.float32))
    dec = N.Decoder(inst)
    try:
        _, score_mass = dec.weights()
        w = net.apply(dec, alpha=0.5)
        _, mass = dec.weights()
    finally:
        dec.close()
        net.close()
    _, ws = O.score_weights(inst)
    assert np.array_equal(w, ws)
    assert np.array_equal(mass, score_mass)


def test_backward_entry_point_matches_oracle():
    theta = I.mlp_init(11)
    X, base, signal, seg = _training_rows(seed=12)
    rng = np.random.default_rng(13)
    dg = rng.normal(size=X.shape[0]).astype(np.float32)
    net = N.Mlp(theta)
    try:
        grad = net.backward(X, dg)
    finally:
        net.close()
    ref = MO.backward(MO.bf16_round(theta).astype(np.float64), X.astype(np.float64), dg.astype(np.float64))
    assert np.max(np.abs(grad - ref)) <= 1e-4 * np.max(np.abs(ref))


def test_adamw_step_entry_point_equals_fused_training_step():
    """loss_grad then adamw_step gives the state train(1) gives, bit for
    bit, and the step follows the closed form."""
    theta = I.mlp_init(14)
    X, base, signal, seg = _training_rows(seed=15)
    hp = dict(lr=1e-2, beta1=0.9, beta2=0.99, eps=1e-6, weight_decay=0.05)
    a, b = N.Mlp(theta), N.Mlp(theta)
    try:
        for net in (a, b):
            net.set_training_rows(X, base, signal, seg, 0.75, 0.5, 1e-2)
        th = theta.astype(np.float64)
        m = np.zeros_like(th)
        v = np.zeros_like(th)
        for step in (1, 2):
            _, grad = a.loss_grad()
            a.adamw_step(grad, **hp)
            b.train(1, **hp)
            sa, sb = a.state(), b.state()
            for x, y in zip(sa[:4], sb[:4]):
                assert np.array_equal(x, y)
            assert sa[4] == sb[4] == step
            th, m, v = MO.adamw_step(th, m, v, grad.astype(np.float64), step, hp["lr"], hp["beta1"], hp["beta2"],
                                     hp["eps"], hp["weight_decay"])
            assert np.max(np.abs(sa[0] - th)) <= 1e-6 * (1 + np.max(np.abs(th)))
            th = sa[0].astype(np.float64)
        with pytest.raises(N.McpdError):
            a.adamw_step(np.full(N.MLP_PARAMS, np.nan, np.float32), **hp)
    finally:
        a.close()
        b.close()


def test_checkpoint_resume_continues_bit_for_bit(tmp_path):
    """Train, save the whole optimiser state, restore it into a new network
    and train both on: master, BF16 copy, moments and step stay identical."""
    from paper_2608_30239_amd import selection as S
    theta = I.mlp_init(16)
    X, base, signal, seg = _training_rows(seed=17, sizes=(300, 500, 700))
    hp = dict(lr=3e-3, weight_decay=1e-4)
    net = N.Mlp(theta)
    path = str(tmp_path / "ckpt.npz")
    try:
        net.set_training_rows(X, base, signal, seg, 0.7, 0.3, 1e-3)
        net.train(7, **hp)
        S.save_checkpoint(net, path, note="after 7 steps")
        back = S.load_checkpoint(path)
        try:
            assert back.state()[4] == 7
            back.set_training_rows(X, base, signal, seg, 0.7, 0.3, 1e-3)
            h1 = net.train(5, **hp)
            h2 = back.train(5, **hp)
            assert np.array_equal(h1, h2)
            for x, y in zip(net.state(), back.state()):
                assert np.array_equal(x, y)
        finally:
            back.close()
        # a damaged checkpoint is refused
        z = dict(np.load(path, allow_pickle=False))
        z["adam_m"] = z["adam_m"] + np.float32(1e-3)
        np.savez(path, **z)
        with pytest.raises(ValueError, match="hash"):
            S.load_checkpoint(path)
    finally:
        net.close()
