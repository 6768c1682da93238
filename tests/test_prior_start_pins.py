"""Pins of the oracle's prior initial distribution (init_mode 1; Algorithm 3
draws Z_0 ~ nu and sets X_0 = Y_0 = Z_0, and the estimator is unbiased for
any nu, Theorem 1): the literal H_{k:l} sums from stored paths that now start
from Z_0, the rate at which clones start positive, unbiasedness against
exact marginals, and the reduction to the all-negative start when
floor(q 2^32) = 0."""

import numpy as np
import pytest

from oracle import oracle as O
from paper_2608_30239_amd import instances as I
from tests import exact
from tests.test_oracle_pins import literal_numerators, twelve_clone_instance


@pytest.mark.parametrize("k,ell", [(0, 0), (3, 12), (10, 50)])
def test_prior_start_numerators_equal_literal_definition(k, ell):
    inst = twelve_clone_instance(seed=3, fp=0.15, fn=0.15, q=0.3)
    M = O.Model(inst)
    started_positive = 0
    for p in range(16):
        for r in (1, 2):
            tr = M.trace(p, r, max_len=20000, k=k, m=ell, budget=0, slots=1, seed=4, init_mode=1)
            assert np.array_equal(tr["X"][0], tr["Y"][0])          # X_0 = Y_0 = Z_0
            started_positive += int(tr["X"][0].any())
            assert list(tr["numer"]) == [int(v) for v in literal_numerators(tr, k, ell)]
    assert started_positive > 20


def test_prior_start_rate():
    """Clones start positive independently with probability
    floor(q 2^32) / 2^32 (binomial z-scores per clone and overall)."""
    q = 0.3
    inst = twelve_clone_instance(seed=2, fp=0.1, fn=0.1, q=q)
    M = O.Model(inst)
    qt = np.floor(q * 2.0 ** 32) / 2.0 ** 32
    Z = []
    for p in range(700):
        for r in (1, 2, 3):
            Z.append(M.trace(p, r, max_len=20000, k=0, m=1, budget=0, slots=1, seed=7, init_mode=1)["X"][0])
    Z = np.array(Z, dtype=np.float64)
    N = Z.shape[0]
    z_clone = (Z.mean(axis=0) - qt) / np.sqrt(qt * (1 - qt) / N)
    assert np.max(np.abs(z_clone)) < 4.5, z_clone
    # pairs of clones drawn from the same block and from different blocks are uncorrelated
    c = np.corrcoef(Z.T)
    off = c[~np.eye(inst.n, dtype=bool)]
    assert np.max(np.abs(off)) < 4.5 / np.sqrt(N)


def test_prior_start_unbiased():
    inst = twelve_clone_instance(seed=3, fp=0.15, fn=0.15, q=0.3)
    pe = np.array([float(v) for v in exact.exact_marginals(inst)])
    M = O.Model(inst)
    r = M.run(0, 1 << 19, 3, 12, seed=21, init_mode=1)
    z = (r["marginals"] - pe) / r["stderr"]
    assert np.max(np.abs(z)) < 4.5, z
    # with refill over a horizon of 2.5 windows as well
    P = 1 << 17
    r = M.run(P * 30, P, 3, 12, seed=22, init_mode=1)
    assert r["stats"]["reps_retained"] > P
    z = (r["marginals"] - pe) / r["stderr"]
    assert np.max(np.abs(z)) < 4.5, z


def test_prior_below_resolution_is_the_all_negative_start():
    inst, rp = I.tiny_plain()
    inst.prior = 2.0 ** -33                  # floor(q 2^32) = 0: nobody starts positive
    M = O.Model(inst)
    a = M.run(rp.slots * 120, rp.slots, rp.k, rp.m, seed=5, init_mode=1)
    b = M.run(rp.slots * 120, rp.slots, rp.k, rp.m, seed=5, init_mode=0)
    assert np.array_equal(a["marginals"], b["marginals"])
    assert np.array_equal(a["stderr"], b["stderr"])
    assert np.array_equal(a["hist"], b["hist"])


def test_init_mode_out_of_range_is_rejected():
    inst, rp = I.tiny_plain()
    with pytest.raises(ValueError):
        O.Model(inst).run(0, 16, rp.k, rp.m, init_mode=2)


def test_prior_start_uses_documented_words():
    """Clone i reads word i mod 4 of block (floor(i/4), r, p, g + 2^25) and
    starts positive when it is below floor(q 2^32)."""
    q = 0.3
    inst = twelve_clone_instance(seed=2, fp=0.1, fn=0.1, q=q)
    M = O.Model(inst)
    seed = 0x0123456789ABCDEF
    key = [seed & 0xFFFFFFFF, seed >> 32]
    Q = int(np.floor(q * 2.0 ** 32))
    for p, r, g in ((0, 1, 0), (5, 3, 0), (17, 2, 9)):
        tr = M.trace(p, r, max_len=20000, k=0, m=1, budget=0, slots=1, seed=seed, init_mode=1, instance_id=g)
        want = [int(O.philox([i // 4, r, p, g + (1 << 25)], key)[i % 4]) < Q for i in range(inst.n)]
        assert tr["X"][0].astype(bool).tolist() == want
