"""GPU suite: a run split into shares of its slots (first_slot).  Slots are
i.i.d. (Assumption 2) and keyed by their global index in the random-number
counter, so the shares' integer sums, histograms and counters add up exactly
to the whole run's; this is what a run over several GPUs relies on (one
share per GPU, then one sum of integers)."""

import numpy as np
import pytest

from paper_2608_30239_amd import instances as I
from test_gpu_parity import kern  # noqa: F401  (kern is a fixture)

pytestmark = pytest.mark.gpu

N = pytest.importorskip("paper_2608_30239_amd.native")

SUMMED = ("progress_units", "retained_units", "single_site_updates", "reps_started", "reps_retained",
          "reps_aborted", "cap_hits", "zero_completion_slots", "tau_sum", "rollback_units")


def wide(b2):
    """128-bit sums of squares (lo, hi words) as Python integers."""
    return b2[..., 0].astype(object) + b2[..., 1].astype(object) * (1 << 64)


@pytest.mark.parametrize("init_mode", [0, 1])
def test_shares_add_up_to_the_whole_run(kern, init_mode):
    inst, rp = I.paper_shaped()
    B, P = 4096, 8192
    nb = B // rp.m
    dec = N.Decoder(inst)
    try:
        full = dec.run(B * P, P, rp.k, rp.m, 5, buckets=nb, slot_records=True, init_mode=init_mode, **kern)
        parts = [dec.run(B * n, n, rp.k, rp.m, 5, buckets=nb, slot_records=True, first_slot=f,
                         init_mode=init_mode, **kern)
                 for f, n in ((0, 3000), (3000, 5192))]
    finally:
        dec.close()
    assert np.array_equal(sum(p["bucket_sum"] for p in parts), full["bucket_sum"])
    assert (sum(wide(p["bucket_sumsq"]) for p in parts) == wide(full["bucket_sumsq"])).all()
    assert np.array_equal(sum(p["hist"] for p in parts), full["hist"])
    assert np.array_equal(np.concatenate([p["slot_nstar"] for p in parts]), full["slot_nstar"])
    assert np.array_equal(np.concatenate([p["slot_units"] for p in parts]), full["slot_units"])
    for key in SUMMED:
        assert sum(p["stats"][key] for p in parts) == full["stats"][key], key
    for key in ("tau_max", "nstar_max"):
        assert max(p["stats"][key] for p in parts) == full["stats"][key], key
    # the whole run's marginals are the slot-weighted mean of the shares'
    m = (3000 * parts[0]["marginals"] + 5192 * parts[1]["marginals"]) / P
    assert np.max(np.abs(m - full["marginals"])) <= 1e-12 * np.max(np.abs(full["marginals"]))


def test_first_slot_range_checked():
    inst, rp = I.tiny_plain()
    dec = N.Decoder(inst)
    try:
        with pytest.raises(N.McpdError):
            dec.run(16 * 100, 16, rp.k, rp.m, 1, first_slot=(1 << 32) - 8)
        dec.run(16 * 100, 16, rp.k, rp.m, 1, first_slot=(1 << 32) - 16)
    finally:
        dec.close()
