"""Seeded synthetic pooling instances (inputs only; no decoding arithmetic).

This module is the single source of inputs shared by the HIP path and by the
CPU oracle.  It draws pooling designs, latent positive clones and noisy pool
outcomes; it computes nothing of the decoding method itself.

Shapes follow the paper's workloads (Experiments, "Synthetic data"; the
supplementary "Details of the Experimental Setup"): a Knill-type random
k-sets design in which each clone joins ``d`` distinct pools chosen uniformly,
a handful of true positives, and pool outcomes drawn with the same
false-positive / false-negative rates that are later used for decoding.  The
paper's own instance and the Tapestry matrices are not published with it, so
these generators stand in for them.

All randomness comes from ``numpy.random.default_rng(seed)`` (PCG64).
"""

from __future__ import annotations

import dataclasses
import hashlib
from typing import List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Instance:
    """A decoding instance: design as clone->pool CSR plus observed outcomes."""

    name: str
    n: int                    # clones
    m: int                    # pools
    row_ptr: np.ndarray       # int32 [n+1]
    pool_idx: np.ndarray      # int32 [nnz], strictly ascending within a row
    y: np.ndarray             # uint8 [m], observed pool outcomes
    fp: float                 # false-positive rate alpha_fp
    fn: float                 # false-negative rate beta_fn
    prior: float              # clone prior q
    positives: np.ndarray     # int32, the latent positives used to draw y

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int32)

    def dense(self) -> np.ndarray:
        """Pooling matrix A in {0,1}^{m x n} (small instances only)."""
        a = np.zeros((self.m, self.n), dtype=np.uint8)
        for i in range(self.n):
            a[self.pool_idx[self.row_ptr[i]:self.row_ptr[i + 1]], i] = 1
        return a

    def digest(self) -> str:
        h = hashlib.sha256()
        for arr in (self.row_ptr, self.pool_idx, self.y):
            h.update(np.ascontiguousarray(arr).tobytes())
        h.update(np.array([self.fp, self.fn, self.prior], dtype=np.float64).tobytes())
        return h.hexdigest()[:16]


def _csr_from_rows(rows: Sequence[np.ndarray]) -> (np.ndarray, np.ndarray):
    row_ptr = np.zeros(len(rows) + 1, dtype=np.int32)
    for i, r in enumerate(rows):
        row_ptr[i + 1] = row_ptr[i] + len(r)
    pool_idx = (np.concatenate([np.sort(r) for r in rows]).astype(np.int32)
                if rows else np.zeros(0, np.int32))
    return row_ptr, pool_idx


def random_ksets_design(n: int, m: int, degree, rng: np.random.Generator):
    """Each clone joins ``degree`` distinct pools drawn uniformly.

    ``degree`` is an int, or a (lo, hi) pair for a per-clone degree drawn
    uniformly from {lo..hi}.
    """
    rows = []
    for _ in range(n):
        d = degree if np.isscalar(degree) else int(rng.integers(degree[0], degree[1] + 1))
        rows.append(rng.choice(m, size=int(d), replace=False))
    return _csr_from_rows(rows)


def simulate_outcomes(row_ptr, pool_idx, m, positives, fp, fn, rng):
    """Pool j is latently positive iff it holds a positive clone; the observed
    outcome flips with probability fn (positive pool) or fp (negative pool)."""
    latent = np.zeros(m, dtype=bool)
    for i in positives:
        latent[pool_idx[row_ptr[i]:row_ptr[i + 1]]] = True
    u = rng.random(m)
    y = np.where(latent, u >= fn, u < fp).astype(np.uint8)
    return y


def make_instance(name, n, m, degree, n_pos, fp, fn, prior=None, seed=0,
                  design_seed: Optional[int] = None) -> Instance:
    """Random k-sets design + positives + outcomes.

    With ``design_seed`` given, the design comes from that seed and the
    positives/outcomes from ``seed``; otherwise everything comes from ``seed``.
    """
    if design_seed is None:
        rng = np.random.default_rng(seed)
        row_ptr, pool_idx = random_ksets_design(n, m, degree, rng)
    else:
        row_ptr, pool_idx = random_ksets_design(n, m, degree, np.random.default_rng(design_seed))
        rng = np.random.default_rng([design_seed, seed])
    positives = np.sort(rng.choice(n, size=n_pos, replace=False)).astype(np.int32)
    y = simulate_outcomes(row_ptr, pool_idx, m, positives, fp, fn, rng)
    q = float(prior) if prior is not None else n_pos / n
    return Instance(name, n, m, row_ptr, pool_idx, y, float(fp), float(fn), q, positives)


def identity_instance(n: int, fp: float, fn: float, prior: float, seed: int = 0) -> Instance:
    """A = I: every pool holds exactly one clone (closed-form posterior)."""
    rng = np.random.default_rng(seed)
    row_ptr = np.arange(n + 1, dtype=np.int32)
    pool_idx = np.arange(n, dtype=np.int32)
    y = (rng.random(n) < 0.5).astype(np.uint8)
    return Instance(f"identity{n}", n, n, row_ptr, pool_idx, y, fp, fn, prior,
                    np.zeros(0, np.int32))


def from_dense(name, a: np.ndarray, y, fp, fn, prior) -> Instance:
    m, n = a.shape
    rows = [np.nonzero(a[:, i])[0] for i in range(n)]
    row_ptr, pool_idx = _csr_from_rows(rows)
    return Instance(name, n, m, row_ptr, pool_idx, np.asarray(y, np.uint8), fp, fn, prior,
                    np.zeros(0, np.int32))


def restrict(inst: Instance, active, name: Optional[str] = None) -> Instance:
    """The design restricted to the clones ``active`` (ascending), relabelled
    0..len-1 in that order; every pool, the outcomes, the rates and the prior
    are kept.  Clones outside ``active`` are fixed to 0, so this is the
    instance of the pruned posterior."""
    active = np.asarray(active, np.int64)
    rows = [inst.pool_idx[inst.row_ptr[i]:inst.row_ptr[i + 1]] for i in active]
    row_ptr, pool_idx = _csr_from_rows(rows)
    where = {int(c): j for j, c in enumerate(active)}
    pos = np.array([where[int(c)] for c in inst.positives if int(c) in where], np.int32)
    return Instance(name or f"{inst.name}_top{len(active)}", len(active), inst.m, row_ptr, pool_idx,
                    inst.y.copy(), inst.fp, inst.fn, inst.prior, pos)


def regular_design(n: int, m: int, degree: int, pool_size: int, rng: np.random.Generator):
    """A random design in which every clone is in ``degree`` distinct pools
    and every pool holds ``pool_size`` clones (n * degree = m * pool_size):
    pool slots dealt at random, then repeated pools inside a clone swapped
    away with random slots of other clones."""
    assert n * degree == m * pool_size
    slots = np.repeat(np.arange(m, dtype=np.int32), pool_size)
    rng.shuffle(slots)
    rows = slots.reshape(n, degree)
    for _ in range(1000 * n):
        bad = [i for i in range(n) if len(set(rows[i].tolist())) < degree]
        if not bad:
            break
        for i in bad:
            e = int(rng.integers(degree))
            j, f = int(rng.integers(n)), int(rng.integers(degree))
            a, b = rows[i, e], rows[j, f]
            if j != i and b not in rows[i] and a not in rows[j]:
                rows[i, e], rows[j, f] = b, a
    else:
        raise RuntimeError("no regular design found")
    return _csr_from_rows([np.sort(r) for r in rows])


# --------------------------------------------------------------------------
# Estimator-length recipe (supplementary, "Details of the Experimental Setup"
# and Table S1): M_s = s * n_a updates, b_s = round(0.1 M_s), k = b_s + 1,
# l = M_s.  Table S1 fixes the rounding of exact halves to the even neighbour
# (M = 1665 -> 166, M = 1235 -> 124).
# --------------------------------------------------------------------------

def round_half_even_tenth(M: int) -> int:
    """round(M / 10) with ties to even, in exact integer arithmetic."""
    q, rem = divmod(int(M), 10)
    if rem > 5 or (rem == 5 and q % 2 == 1):
        q += 1
    return q


def window_for_sweeps(s: int, n_a: int):
    """(k, l) for an estimator of ``s`` sweeps over ``n_a`` clones."""
    M = s * n_a
    b = round_half_even_tenth(M)
    return b + 1, M


# --------------------------------------------------------------------------
# Workloads.  Each returns plain inputs plus the run parameters.
# --------------------------------------------------------------------------

@dataclasses.dataclass
class RunParams:
    budget: int     # total progress units (coupled updates); B = budget // slots
    slots: int      # logical slots P
    k: int
    m: int          # window end l (Jacob's m)
    seed: int


def tiny_plain(seed: int = 0) -> (Instance, RunParams):
    """16 clones, 8 pools, degree 3, 2 positives, fp=0.02, fn=0.05, q=0.01;
    4096 pairs (budget 0: one pair per slot), window 10:50."""
    inst = make_instance("tiny16x8", 16, 8, 3, 2, 0.02, 0.05, prior=0.01, seed=seed)
    return inst, RunParams(budget=0, slots=4096, k=10, m=50, seed=0)


def paper_shaped(seed: int = 0) -> (Instance, RunParams):
    """1298 clones, 97 pools, degree 5, 3 positives, fp=0.05, fn=0.10,
    q = 3/1298; budget 2^28 over 65536 slots (B = 4096); window of one sweep
    (k = 131, l = 1298)."""
    inst = make_instance("knill1298x97", 1298, 97, 5, 3, 0.05, 0.10, prior=3 / 1298, seed=seed)
    k, l = window_for_sweeps(1, 1298)
    return inst, RunParams(budget=1 << 28, slots=65536, k=k, m=l, seed=0)


NOISE_LEVELS = (0.01, 0.05, 0.10, 0.20)


def noise_sweep(n_seeds: int = 8, design_seed: int = 0) -> (List[Instance], RunParams):
    """The 1298x97 degree-5 design held fixed; fp, fn each in NOISE_LEVELS,
    times ``n_seeds`` positive/outcome seeds (128 instances by default), 3
    positives each; 2^24 updates per instance over 4096 slots."""
    insts = []
    for fp in NOISE_LEVELS:
        for fn in NOISE_LEVELS:
            for s in range(n_seeds):
                insts.append(make_instance(f"noise_fp{fp}_fn{fn}_s{s}", 1298, 97, 5, 3, fp, fn,
                                           prior=3 / 1298, seed=s, design_seed=design_seed))
    k, l = window_for_sweeps(1, 1298)
    return insts, RunParams(budget=1 << 24, slots=4096, k=k, m=l, seed=0)


def uneven_batch(count: int = 256, seed: int = 4, n_lo: int = 200, n_hi: int = 20000):
    """Uneven instances: n ~ U{n_lo..n_hi}, m = round(0.075 n), per-clone
    degree ~ U{3..7}, positives ~ U{1..10}, fp, fn ~ U[0.01, 0.20], q =
    positives / n.  Returns (instances, per-instance (budget, slots, k, l))."""
    rng = np.random.default_rng(seed)
    insts, params = [], []
    for c in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        m = max(8, int(round(0.075 * n)))
        npos = int(rng.integers(1, 11))
        fp = float(rng.uniform(0.01, 0.20))
        fn = float(rng.uniform(0.01, 0.20))
        inst = make_instance(f"uneven{c}_n{n}", n, m, (3, 7), npos, fp, fn,
                             prior=npos / n, seed=int(rng.integers(1 << 31)))
        budget = 1 << 24
        slots = 64 * -(-budget // (4 * n * 64))
        k, l = window_for_sweeps(1, n)
        insts.append(inst)
        params.append(RunParams(budget=budget, slots=slots, k=k, m=l, seed=0))
    return insts, params


def mlp_init(seed: int = 0) -> np.ndarray:
    """Initial FP32 parameters of the 8-64-64-1 selection-weight network,
    flat in the layout W1 [64][8], b1 [64], W2 [64][64], b2 [64], W3 [64], b3:
    every weight and bias of a layer uniform in +-1/sqrt(fan_in)."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, count in ((8, 64 * 8), (8, 64), (64, 64 * 64), (64, 64), (64, 64), (64, 1)):
        b = 1.0 / np.sqrt(fan_in)
        parts.append(rng.uniform(-b, b, count))
    return np.concatenate(parts).astype(np.float32)


def heldout_large(seed: int, n: int = 20000, budget: int = 1 << 28) -> (Instance, RunParams):
    """A fresh large instance drawn like the uneven batch (m = 7.5% of n,
    degree ~ U{3..7}, positives ~ U{1..10}, fp, fn ~ U[0.01, 0.20], q =
    positives / n), run at the given budget (2^28 by default) with B about
    four sweeps."""
    rng = np.random.default_rng(seed)
    m = int(round(0.075 * n))
    npos = int(rng.integers(1, 11))
    fp = float(rng.uniform(0.01, 0.20))
    fn = float(rng.uniform(0.01, 0.20))
    inst = make_instance(f"heldout{seed}_n{n}", n, m, (3, 7), npos, fp, fn, prior=npos / n,
                         seed=int(rng.integers(1 << 31)))
    slots = 64 * -(-budget // (4 * n * 64))
    k, l = window_for_sweeps(1, n)
    return inst, RunParams(budget=budget, slots=slots, k=k, m=l, seed=0)


# --------------------------------------------------------------------------
# The designs of the paper's experiments (Section "Experimental Setup"), as
# synthetic stand-ins: its 1298 x 97 instance and the Tapestry data are not
# available, so designs of the same shape are drawn here.
# --------------------------------------------------------------------------

KNILL3_NOISE = ((0.05, 0.05), (0.05, 0.10), (0.10, 0.05), (0.10, 0.10))   # (fn, fp)


def knill_degree3(fn: float = 0.10, fp: float = 0.10, seed: int = 0, design_seed: int = 0) -> Instance:
    """1298 clones, 97 pools, every clone in 3 pools (random k-sets), 3
    positives, q = 2.6 / 1298; the design held fixed over noise levels and
    outcome seeds."""
    return make_instance(f"knill3_fn{fn}_fp{fp}_s{seed}", 1298, 97, 3, 3, fp, fn, prior=2.6 / 1298,
                         seed=seed, design_seed=design_seed)


def tapestry_shaped(which: int = 320, seed: int = 0) -> (Instance, int):
    """A design shaped like Tapestry 320 (320 samples, 48 pools of 20, 5
    positives, fn = fp = 0.01, q = 5/320, all clones kept) or Tapestry 961
    (961 samples, 93 pools of 31, 10 positives, fn = 1/23, fp = 0.01,
    q = 10/961, 247 clones kept); every sample in 3 pools.  Returns the
    instance and the number of clones the paper's analysis keeps."""
    if which == 320:
        n, m, size, npos, fn, fp, keep = 320, 48, 20, 5, 0.01, 0.01, 320
    elif which == 961:
        n, m, size, npos, fn, fp, keep = 961, 93, 31, 10, 1.0 / 23.0, 0.01, 247
    else:
        raise ValueError("which must be 320 or 961")
    rng = np.random.default_rng([which, seed])
    row_ptr, pool_idx = regular_design(n, m, 3, size, rng)
    positives = np.sort(rng.choice(n, size=npos, replace=False)).astype(np.int32)
    y = simulate_outcomes(row_ptr, pool_idx, m, positives, fp, fn, rng)
    inst = Instance(f"tapestry{which}_s{seed}", n, m, row_ptr, pool_idx, y, fp, fn, npos / n, positives)
    return inst, keep
