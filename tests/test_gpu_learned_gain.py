"""What the trained selection network gains over the paper's score weights
at equal budget (paper_2608_30239_amd/selection.py has the protocol), on the
five held-out evaluation instances: the paper-shaped 1298 x 97 instance and
four 20000-clone instances (the network saw only the uneven batch).  Equal
budget means equal progress units and slots; the gain is the ratio of
1 / (MSE x device seconds), MSE against the mean of 1024 independent
reference runs with its own variance removed, over 1024 runs per weighting.
The learned weights use the floor selection.FLOOR, chosen on four other
20000-clone instances (selection.choose_floor), not on these.

Every run has a fixed seed, so every figure here is a function of the
inputs and the shipped network alone.  On the 20000-clone instances the
run-level error is heavy-tailed (the mean over runs is set by the few runs
that drew a pair taking very long to meet), so each gain comes with a 90%
bootstrap interval and the median run's gain beside it."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

N = pytest.importorskip("paper_2608_30239_amd.native")
S = pytest.importorskip("paper_2608_30239_amd.selection")
from paper_2608_30239_amd import instances as I  # noqa: E402


def test_trained_network_against_score_weights_on_the_evaluation_set():
    params, report = S.load_trained()
    assert params.shape == (N.MLP_PARAMS,) and np.isfinite(params).all()
    net = N.Mlp(params)
    try:
        res = S.evaluate(net, nref=1024, nrep=1024, log=lambda m: print(m, flush=True))
    finally:
        net.close()
    rows = {r["instance"]: r for r in res["rows"]}
    for name, r in rows.items():
        print(f"{name}: gain {r['gain']:.2f} (90% CI {r['gain_ci90'][0]:.2f}-{r['gain_ci90'][1]:.2f}), "
              f"median run {r['median_gain']:.2f}, runs {r['runs']}", flush=True)
        assert np.isfinite(r["gain"]) and r["gain"] > 0
        lo, hi = r["gain_ci90"]
        assert lo <= r["gain"] <= hi
        # the typical run gains everywhere
        assert r["median_gain"] > 1.0
    print(f"geometric mean gain {res['gain_geomean']:.2f}", flush=True)
    # the paper-shaped instance: a clear win, its whole interval above one
    k = rows["knill1298x97"]
    assert k["gain"] > 1.5 and k["gain_ci90"][0] > 1.0
    assert res["gain_geomean"] > 1.5


def test_zero_residual_network_is_the_score_weights():
    """The fallback: a network whose output is zero, at the score weights'
    own floor of 1/2, reproduces the score weights exactly, hence the same
    runs bit for bit."""
    inst, rp = I.paper_shaped()
    net = N.Mlp(np.zeros(N.MLP_PARAMS, np.float32))
    dec = N.Decoder(inst)
    try:
        a = dec.run(rp.budget // 16, rp.slots // 16, rp.k, rp.m, 5)
        net.apply(dec, 0.5)
        b = dec.run(rp.budget // 16, rp.slots // 16, rp.k, rp.m, 5)
    finally:
        dec.close()
        net.close()
    assert np.array_equal(a["marginals"], b["marginals"]) and np.array_equal(a["hist"], b["hist"])
