"""Exact reference quantities for small pooling instances, by enumeration.

Written directly from the posterior of the paper (Section "Knill's Method"):
  pi(z | y) ~ prod_i q^{z_i} (1-q)^{1-z_i} prod_j Pr{y_j | xi_j(z)},
  xi_j(z) = 1{sum_i A_ji z_i > 0},
with Pr{y=1 | xi=1} = 1 - fn and Pr{y=1 | xi=0} = fp.  Arithmetic is exact
(``fractions.Fraction`` of the binary values of q, fp, fn).  Independent of
the oracle and of the HIP path: it never computes a log-odds or a
conditional by the count formula; it only evaluates pi on whole states.
"""

from __future__ import annotations

from fractions import Fraction

import numpy as np


def all_states(n: int) -> np.ndarray:
    """uint8 [2^n, n]; row s holds the bits of s (clone i = bit i)."""
    s = np.arange(1 << n, dtype=np.int64)
    return ((s[:, None] >> np.arange(n)) & 1).astype(np.uint8)


def _rates(inst):
    q = Fraction(inst.prior)
    fp = Fraction(inst.fp)
    fn = Fraction(inst.fn)
    # like[xi][y] = Pr{y | xi}
    like = {1: {1: 1 - fn, 0: fn}, 0: {1: fp, 0: 1 - fp}}
    return q, like


def unnormalized_weights(inst):
    """Exact pi(z) up to the common normaliser, for every state (n <= 14)."""
    n = inst.n
    assert n <= 14, "enumeration is meant for tiny instances"
    A = inst.dense().astype(np.int64)
    q, like = _rates(inst)
    Z = all_states(n).astype(np.int64)
    xi = (Z @ A.T > 0).astype(np.int64)           # [S, m]
    k = Z.sum(axis=1)
    out = []
    qpow = [q ** a * (1 - q) ** (n - a) for a in range(n + 1)]
    for s in range(Z.shape[0]):
        w = qpow[int(k[s])]
        for j in range(inst.m):
            w *= like[int(xi[s, j])][int(inst.y[j])]
        out.append(w)
    return out


def exact_marginals(inst):
    """Exact p_i = E_pi[Z_i] for n <= 20, grouping states by (|z|, xi).

    Returns a list of Fractions."""
    n, m = inst.n, inst.m
    assert n <= 20 and m <= 20
    A = inst.dense().astype(np.int64)
    q, like = _rates(inst)
    Z = all_states(n).astype(np.int64)
    xi_code = ((Z @ A.T > 0).astype(np.int64) << np.arange(m)).sum(axis=1)
    k = Z.sum(axis=1)
    key = k * (1 << m) + xi_code
    nkeys = (n + 1) << m
    tot = np.bincount(key, minlength=nkeys)
    per_clone = [np.bincount(key, weights=None, minlength=nkeys) * 0 for _ in range(n)]
    for i in range(n):
        per_clone[i] = np.bincount(key[Z[:, i] == 1], minlength=nkeys)
    lik_cache = {}

    def weight(kk, code):
        if code not in lik_cache:
            w = Fraction(1)
            for j in range(m):
                w *= like[(code >> j) & 1][int(inst.y[j])]
            lik_cache[code] = w
        return q ** kk * (1 - q) ** (n - kk) * lik_cache[code]

    nz = np.nonzero(tot)[0]
    denom = Fraction(0)
    numer = [Fraction(0)] * n
    for key_ in nz:
        kk, code = divmod(int(key_), 1 << m)
        w = weight(kk, code)
        denom += int(tot[key_]) * w
        for i in range(n):
            c = int(per_clone[i][key_])
            if c:
                numer[i] += c * w
    return [x / denom for x in numer]


def exact_conditional(weights, n, x_index: int, i: int) -> Fraction:
    """pi(x^{i<-1}) / (pi(x^{i<-1}) + pi(x^{i<-0})) from whole-state weights."""
    s1 = x_index | (1 << i)
    s0 = x_index & ~(1 << i)
    return weights[s1] / (weights[s1] + weights[s0])


def identity_marginals(inst):
    """A = I: clones are independent, p_i = q L1 / (q L1 + (1-q) L0)."""
    q, like = _rates(inst)
    out = []
    for i in range(inst.n):
        yi = int(inst.y[i])
        a = q * like[1][yi]
        b = (1 - q) * like[0][yi]
        out.append(a / (a + b))
    return out
