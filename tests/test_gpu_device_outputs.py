"""GPU suite: mcpd_run_unbiased_dev (outputs left in device memory) against
mcpd_run_unbiased on the same inputs and against the oracle.  The device
forms the marginals and standard errors in FP64 from the same integer sums
the host forms in extended precision, so they agree to rounding; the
histogram and the counters are integers and agree exactly."""

import numpy as np
import pytest

import parity as P
from paper_2608_30239_amd import instances as I
from test_gpu_parity import kern  # noqa: F401  (kern is a fixture)

pytestmark = pytest.mark.gpu

N = pytest.importorskip("paper_2608_30239_amd.native")
torch = pytest.importorskip("torch")


def dev_run(dec, n, budget, slots, k, m, seed, hist_bins=64, with_se=True, with_hist=True, **opt):
    marg = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
    se = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
    hist = torch.full((hist_bins,), -1, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    st = dec.run_dev(budget, slots, k, m, seed, marg.data_ptr(), se.data_ptr() if with_se else 0,
                     hist.data_ptr() if with_hist else 0, hist_bins=hist_bins, **opt)
    torch.cuda.synchronize()
    return marg.cpu().numpy(), se.cpu().numpy(), hist.cpu().numpy().view(np.uint64), st


def close(a, b, rel):
    scale = max(1e-300, float(np.max(np.abs(b))))
    assert np.max(np.abs(a - b)) <= rel * scale


@pytest.mark.parametrize("full", [False, True], ids=["4096-slots", "benchmark-size"])
def test_device_outputs_equal_host_outputs(kern, full):
    """Also at the benchmark's size (2^28 updates over 65536 slots), the
    configuration whose device-output runs the benchmark times."""
    inst, rp = I.paper_shaped()
    budget, slots = (rp.budget, rp.slots) if full else (4096 * 4096, 4096)
    dec = N.Decoder(inst)
    try:
        host = dec.run(budget, slots, rp.k, rp.m, 21, **kern)
        marg, se, hist, st = dev_run(dec, inst.n, budget, slots, rp.k, rp.m, 21, **kern)
    finally:
        dec.close()
    close(marg, host["marginals"], 1e-12)
    close(se, host["stderr"], 1e-10)
    assert np.array_equal(hist, host["hist"])
    for key, val in host["stats"].items():
        if key != "kernel_ms":
            assert st[key] == val, key
    orc, _ = P.oracle_run(inst, budget, slots, rp.k, rp.m, seed=21)
    close(marg, orc["marginals"], 1e-12)
    close(se, orc["stderr"], 1e-10)
    # clone by clone against the value the (bit-identical) integer sums define
    P.check_elementwise(dict(marginals=marg, stderr=se), orc, slots)


def test_device_outputs_optional_parts_and_one_slot():
    inst, rp = I.tiny_plain()
    dec = N.Decoder(inst)
    try:
        host = dec.run(200, 1, rp.k, rp.m, 3)
        marg, se, hist, _ = dev_run(dec, inst.n, 200, 1, rp.k, rp.m, 3, with_se=False, with_hist=False)
        close(marg, host["marginals"], 1e-12)
        assert np.all(se == -1.0) and np.all(hist.view(np.int64) == -1)   # untouched
        marg, se, _, _ = dev_run(dec, inst.n, 200, 1, rp.k, rp.m, 3)
        assert np.all(np.isnan(se))                                        # one slot: no SE
        with pytest.raises(N.McpdError):
            dec.run_dev(200, 1, rp.k, rp.m, 3, 0)                          # marginals are required
        m = torch.zeros(inst.n, dtype=torch.float64, device="cuda")
        with pytest.raises(N.McpdError):
            dec.run_dev(200, 1, rp.k, rp.m, 3, m.data_ptr(), bucket_rows=1, bucket_sum=1)
    finally:
        dec.close()
