"""Pins of the oracle's pruning (``oracle.naive_rank``) and of the restricted
instance (``instances.restrict``) against what the paper fixes: the naive
ranking R_i as a product of likelihood ratios (Section "Knill's Method"), a
ranking worked by hand, the tie rule, and the pruned posterior as the full
posterior conditioned on the pruned clones being negative (exact
enumeration)."""

import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O
from paper_2608_30239_amd import instances as I
from tests import exact as E


def hand_instance():
    # pools 0 and 2 positive, 1 and 3 negative
    #   clone 0: {0, 1}   one +, one -      clone 3: {2}       one +
    #   clone 1: {0, 2}   two +             clone 4: {0, 1}    one +, one - (ties clone 0)
    #   clone 2: {1, 3}   two -             clone 5: {3}       one -
    a = np.zeros((4, 6), np.uint8)
    for i, pools in enumerate(([0, 1], [0, 2], [1, 3], [2], [0, 1], [3])):
        a[pools, i] = 1
    return I.from_dense("hand6", a, [1, 0, 1, 0], fp=0.1, fn=0.2, prior=0.05)


def test_ranking_by_hand():
    inst = hand_instance()
    # a+ = log(0.8/0.1) > 0 > a- = log(0.2/0.9): keys 2a+ (1) > a+ (3) >
    # a+ + a- (0, 4: a tie, lower index first) > a- (5) > 2a- (2)
    assert O.naive_rank(inst, 1).tolist() == [1]
    assert O.naive_rank(inst, 2).tolist() == [1, 3]
    assert O.naive_rank(inst, 3).tolist() == [0, 1, 3]
    assert O.naive_rank(inst, 4).tolist() == [0, 1, 3, 4]
    assert O.naive_rank(inst, 5).tolist() == [0, 1, 3, 4, 5]
    assert O.naive_rank(inst, 6).tolist() == list(range(6))


def log_r_product(inst, i):
    """log of R_i = prod over the clone's pools of Pr{y|xi=1} / Pr{y|xi=0}."""
    r = 1.0
    for j in inst.pool_idx[inst.row_ptr[i]:inst.row_ptr[i + 1]]:
        r *= ((1 - inst.fn) / inst.fp) if inst.y[j] else (inst.fn / (1 - inst.fp))
    return math.log(r)


@pytest.mark.parametrize("fn,fp", [(0.05, 0.05), (0.10, 0.05), (0.05, 0.10), (0.10, 0.10)])
def test_ranking_follows_the_likelihood_ratio(fn, fp):
    inst = I.knill_degree3(fn=fn, fp=fp)
    lr = np.array([log_r_product(inst, i) for i in range(inst.n)])
    keep = O.naive_rank(inst, 333)
    assert len(keep) == 333 and np.all(np.diff(keep) > 0)
    kept = np.zeros(inst.n, bool)
    kept[keep] = True
    # every kept clone scores at least as high as every dropped one
    assert lr[kept].min() >= lr[~kept].max() - 1e-9
    # and the clones at the cut have equal scores (a tie split by index)
    cut = lr[kept].min()
    if lr[~kept].max() > cut - 1e-9:
        tied = np.nonzero(np.abs(lr - cut) <= 1e-9)[0]
        assert np.all(kept[tied[:kept[tied].sum()]]) and not np.any(kept[tied[kept[tied].sum():]])


def test_ties_go_to_the_lower_index():
    inst = I.identity_instance(10, 0.1, 0.1, 0.2)
    inst.y[:] = 1                       # every clone has one positive pool: all tie
    assert O.naive_rank(inst, 4).tolist() == [0, 1, 2, 3]
    inst.y[7] = 0                       # clone 7 drops to the bottom
    assert O.naive_rank(inst, 9).tolist() == [0, 1, 2, 3, 4, 5, 6, 8, 9]


def test_rankings_are_nested():
    inst = I.knill_degree3(fn=0.1, fp=0.05, seed=3)
    prev = set()
    for k in (50, 100, 200, 333, 700, 1298):
        cur = set(O.naive_rank(inst, k).tolist())
        assert prev <= cur and len(cur) == k
        prev = cur


def test_pruned_posterior_is_the_conditional_posterior():
    """pi_A(z_A) = pi(z_A, z_{A^c} = 0) / sum over z_A: the marginals of the
    restricted instance equal those of the full posterior conditioned on the
    pruned clones being negative (exact rationals)."""
    full = I.make_instance("prune12", 12, 6, 2, 2, 0.1, 0.15, prior=0.1, seed=5)
    keep = O.naive_rank(full, 8)
    w = E.unnormalized_weights(full)
    Z = E.all_states(full.n)
    mask_out = np.ones(full.n, bool)
    mask_out[keep] = False
    ok = ~np.any(Z[:, mask_out] == 1, axis=1)
    denom = sum((w[s] for s in np.nonzero(ok)[0]), Fraction(0))
    cond = [sum((w[s] for s in np.nonzero(ok & (Z[:, c] == 1))[0]), Fraction(0)) / denom for c in keep]
    pruned = I.restrict(full, keep)
    assert pruned.n == 8 and pruned.m == full.m and pruned.prior == full.prior
    assert E.exact_marginals(pruned) == cond
