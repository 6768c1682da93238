"""Shared comparison of a GPU result with the oracle's (GPU tests only).

Integer results (N* buckets of the exact numerators, sums of squares,
meeting-time histograms, per-clone mismatch times, per-slot N* and S_p,
retained-pair counters) must be bit-identical.  The FP64 marginals and
standard errors are formed on each side from those integers in a different
order (the oracle averages slot means in slot order, the library divides the
per-N* sums): they must agree
within 1e-12 relative to the scale of the estimates (standard errors within
1e-10, since they pass through a difference of sums of squares).

Per element, the GPU's marginals and standard errors are also checked
against the values the integer buckets define exactly (the buckets being
bit-identical to the oracle's): theta_j = (1/(P W)) sum_n S1[n][j] / n,
formed here in extended precision.  The bound is the rounding of a short
FP64 sum of the nb terms S1[n][j] / n (each converted and divided once):
(nb + 8) ulp of the sum of their magnitudes, so a small marginal is held to
its own scale, not to the largest one's.
"""

import numpy as np

from oracle import oracle as O


def expected_device_stats(orc, B, cmin):
    """What the device must report, derived from the oracle's per-slot
    records: a replication that can no longer be retained is never started
    when S + max(l,1) > B, otherwise it is stopped after B - S + 1 draws and
    replayed once with negated contributions."""
    sret = orc["slot_sret"].astype(np.int64)
    disc = orc["slot_disc"].astype(np.int64)
    started_disc = (disc > 0) & (sret + cmin <= B)
    aborted = int(started_disc.sum())
    rollback = int(((B - sret + 1) * started_disc).sum())
    st = orc["stats"]
    return dict(reps_aborted=aborted, rollback_units=rollback,
                progress_units=st["retained_units"] + 2 * rollback,
                reps_started=st["reps_retained"] + aborted)


def oracle_run(inst, budget, slots, k, m, seed=0, weights=None, nthreads=0, **opt):
    """The oracle's run with the options a GPU run takes; returns (orc, nb)."""
    hist_bins = opt.get("hist_bins", 64)
    hist_width = opt.get("hist_width", 0) or inst.n
    M = O.Model(inst, weights=weights)
    B = budget // slots
    nb = max(1, B // max(m, 1))
    orc = M.run(budget, slots, k, m, seed=seed, nthreads=nthreads, slot_records=True, buckets=nb,
                max_steps=opt.get("max_steps", 0), refill=opt.get("refill", 1),
                hist_bins=hist_bins, hist_width=hist_width, u_hi_bits=opt.get("u_hi_bits", 32),
                instance_id=opt.get("instance_id", 0), init_mode=opt.get("init_mode", 0))
    orc["masses"] = M.masses()
    orc["W"] = m - k + 1
    return orc, nb


EPS = float(np.finfo(np.float64).eps)


def check_elementwise(gpu, orc, slots):
    """GPU marginals and standard errors, clone by clone, against the values
    the integer buckets define (see the module docstring)."""
    ld = np.longdouble
    W = orc["W"]
    S1 = orc["bucket1"]
    S2 = orc["bucket2"]
    nb = S1.shape[0]
    nn = np.arange(1, nb + 1, dtype=ld)[:, None]
    terms = S1.astype(ld) / nn
    PW = ld(slots) * ld(W)
    ref = terms.sum(axis=0) / PW
    mag = np.abs(terms).sum(axis=0) / PW
    err = np.abs(gpu["marginals"].astype(ld) - ref)
    bound = (nb + 8) * EPS * mag + ld(1e-300)
    bad = np.nonzero(err > bound)[0]
    assert bad.size == 0, f"marginal of clone {bad[0]}: {gpu['marginals'][bad[0]]!r} vs {float(ref[bad[0]])!r}"
    if slots < 2:
        return
    # sums of A_pj = V_pj / (W N*_p) and of their squares
    sq = (S2[:, :, 1].astype(ld) * ld(2.0) ** 64 + S2[:, :, 0].astype(ld)) / (nn * nn)
    sumA = terms.sum(axis=0) / ld(W)
    sumA2 = sq.sum(axis=0) / (ld(W) * ld(W))
    var = (sumA2 - sumA * sumA / ld(slots)) / ld(slots - 1)
    var = np.maximum(var, ld(0))
    se2_ref = var / ld(slots)
    se2 = gpu["stderr"].astype(ld) ** 2
    bound2 = 2 * (nb + 8) * EPS * sumA2 / (ld(slots) * ld(slots - 1)) + 4 * EPS * se2_ref + ld(1e-300)
    bad = np.nonzero(np.abs(se2 - se2_ref) > bound2)[0]
    assert bad.size == 0, f"standard error of clone {bad[0]}: {gpu['stderr'][bad[0]]!r} vs {float(np.sqrt(se2_ref[bad[0]]))!r}"


def check(gpu, orc, budget, slots, m, tol=1e-12):
    """gpu: dict with bucket_sum, bucket_sumsq, hist, stats, marginals,
    stderr and optionally slot_nstar, slot_units."""
    B = budget // slots
    cmin = max(m, 1)
    assert np.array_equal(gpu["bucket_sum"], orc["bucket1"])
    assert np.array_equal(gpu["bucket_sumsq"], orc["bucket2"])
    assert np.array_equal(gpu["hist"], orc["hist"])
    if "mismatch" in gpu:
        assert np.array_equal(gpu["mismatch"], orc["mismatch"])
    if "slot_nstar" in gpu:
        assert np.array_equal(gpu["slot_nstar"], orc["slot_nstar"])
        assert np.array_equal(gpu["slot_units"], orc["slot_sret"])
    gs, os_ = gpu["stats"], orc["stats"]
    for key in ("retained_units", "single_site_updates", "reps_retained", "cap_hits",
                "zero_completion_slots", "tau_sum", "tau_max", "nstar_max"):
        assert gs[key] == os_[key], key
    for key, val in expected_device_stats(orc, B, cmin).items():
        assert gs[key] == val, key
    if "W" in orc:
        check_elementwise(gpu, orc, slots)
    scale = max(1e-300, float(np.max(np.abs(orc["marginals"]))))
    assert np.max(np.abs(gpu["marginals"] - orc["marginals"])) <= tol * scale
    if slots > 1:
        sscale = max(1e-300, float(np.max(orc["stderr"])))
        assert np.max(np.abs(gpu["stderr"] - orc["stderr"])) <= 1e-10 * sscale
    else:
        assert np.all(np.isnan(gpu["stderr"])) and np.all(np.isnan(orc["stderr"]))
