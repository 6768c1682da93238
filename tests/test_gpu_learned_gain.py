"""What the trained selection network gains over the paper's score weights
at equal budget, with the score weights as judge (paper_2608_30239_amd/
selection.py has the protocol).  Equal budget means equal progress units
and slots; the gain is the ratio of 1 / (MSE x device seconds), MSE against
an independent long reference run with its own variance removed.

Measured on the paper-shaped instance (1298 clones, 97 pools, budget 2^28,
65536 slots), held out from training (the network saw only the uneven batch
of 256 instances).  Runs take about 12 ms each."""

import numpy as np
import pytest

from paper_2608_30239_amd import instances as I

pytestmark = pytest.mark.gpu

N = pytest.importorskip("paper_2608_30239_amd.native")
S = pytest.importorskip("paper_2608_30239_amd.selection")


def test_trained_network_beats_score_weights_on_paper_shaped_instance():
    params, report = S.load_trained()
    assert params.shape == (N.MLP_PARAMS,) and np.isfinite(params).all()
    net = N.Mlp(params)
    try:
        res = S.evaluate(net, nref=48, nrep=24, instances=[I.paper_shaped()], log=print)
    finally:
        net.close()
    row = res["rows"][0]
    print(f"gain {row['gain']:.2f} (variance-based {row['var_gain']:.2f}), judge chose {row['judge_choice']}, "
          f"judged gain {row['judged_gain']:.2f}")
    # both measures of the same quantity agree on the direction and the size
    assert row["gain"] > 1.3 and row["var_gain"] > 1.3
    assert row["judge_choice"] == "learned" and row["judged_gain"] > 1.2
    assert row["rmse_learned"] < row["rmse_score"]


def test_zero_residual_network_is_the_score_weights():
    """The fallback: a network whose output is zero reproduces the score
    weights exactly, hence the same runs bit for bit."""
    inst, rp = I.paper_shaped()
    net = N.Mlp(np.zeros(N.MLP_PARAMS, np.float32))
    dec = N.Decoder(inst)
    try:
        a = dec.run(rp.budget // 16, rp.slots // 16, rp.k, rp.m, 5)
        net.apply(dec)
        b = dec.run(rp.budget // 16, rp.slots // 16, rp.k, rp.m, 5)
    finally:
        dec.close()
        net.close()
    assert np.array_equal(a["marginals"], b["marginals"]) and np.array_equal(a["hist"], b["hist"])
