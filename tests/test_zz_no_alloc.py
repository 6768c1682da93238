"""The allocation-free entry point (mcpd_run_unbiased_dev_noalloc) against
mcpd_run_unbiased_dev, through the C ABI: same marginals, standard errors,
histogram and counters bit for bit, on calls in a row that change the
input's size (the paper-shaped workload at the benchmark's size, then a
16-clone instance, then the large one again, so a call never depends on
what the previous one left in the shared scratch array).  Sizes beyond the
array are refused with MCPD_EINVAL before any launch."""

import numpy as np
import pytest

import parity as P
from paper_2608_30239_amd import instances as I

pytestmark = pytest.mark.gpu

N = pytest.importorskip("paper_2608_30239_amd.native")
torch = pytest.importorskip("torch")


def outputs(fn, dec, budget, slots, k, m, seed, **opt):
    n = dec.n
    marg = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
    se = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
    hist = torch.full((64,), -1, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    st = fn(dec.h, budget, slots, k, m, seed, marg.data_ptr(), se.data_ptr(), hist.data_ptr(), hist_bins=64, **opt)
    torch.cuda.synchronize()
    return marg.cpu().numpy(), se.cpu().numpy(), hist.cpu().numpy().view(np.uint64), st


def assert_same(a, b):
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[1], b[1], equal_nan=True)
    assert np.array_equal(a[2], b[2])
    for key, val in a[3].items():
        if key != "kernel_ms":
            assert b[3][key] == val, key


def test_noalloc_equals_dev_entry_point_on_changing_sizes():
    big, rp = I.paper_shaped()
    small, srp = I.tiny_plain()
    dbig, dsmall = N.Decoder(big), N.Decoder(small)
    try:
        calls = [(dbig, (rp.budget, rp.slots, rp.k, rp.m, 31)),
                 (dsmall, (1000 * 125, 1000, srp.k, srp.m, 32)),
                 (dbig, (rp.budget // 4, rp.slots // 4, rp.k, rp.m, 33))]
        for dec, args in calls:
            print(f"[call] n={dec.n} budget={args[0]} slots={args[1]}", flush=True)
            ref = outputs(N.mcpd_run_unbiased_dev, dec, *args)
            got = outputs(N.mcpd_run_unbiased_dev_noalloc, dec, *args)
            assert_same(ref, got)
            assert got[3]["kernel_ms"] == 0.0
        # the small call against the oracle, clone by clone
        budget, slots, k, m, seed = calls[1][1]
        orc, _ = P.oracle_run(small, budget, slots, k, m, seed=seed)
        got = outputs(N.mcpd_run_unbiased_dev_noalloc, dsmall, budget, slots, k, m, seed)
        P.check_elementwise(dict(marginals=got[0], stderr=got[1]), orc, slots)
        assert np.array_equal(got[2], orc["hist"])
        # both kernels and every group width through the scratch array
        for opt in (dict(kernel=1), dict(kernel=2, group_lanes=8), dict(kernel=2, group_lanes=64)):
            ref = outputs(N.mcpd_run_unbiased_dev, dsmall, budget, slots, k, m, seed, **opt)
            got = outputs(N.mcpd_run_unbiased_dev_noalloc, dsmall, budget, slots, k, m, seed, **opt)
            assert_same(ref, got)
    finally:
        dbig.close()
        dsmall.close()


def test_noalloc_refuses_runs_beyond_the_scratch_array():
    """2^18 clones on the lane kernel need 256 x 2^18 x 8 bytes of numerator
    rows for one workgroup, twice the array: MCPD_EINVAL, nothing runs, and
    the instance still runs through the allocating entry point."""
    n = 1 << 18
    inst = I.make_instance(f"n{n}", n, 8000, 3, 8, 0.05, 0.1, prior=8 / n, seed=3)
    dec = N.Decoder(inst)
    try:
        marg = torch.zeros(n, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        with pytest.raises(N.McpdError) as e:
            N.mcpd_run_unbiased_dev_noalloc(dec.h, 256 * 2000, 256, 200, 2000, 1, marg.data_ptr(), kernel=1)
        assert e.value.code == N.MCPD_EINVAL and "scratch" in str(e.value)
        st = N.mcpd_run_unbiased_dev(dec.h, 256 * 2000, 256, 200, 2000, 1, marg.data_ptr(), kernel=1)
        torch.cuda.synchronize()
        assert st["reps_retained"] >= 256
    finally:
        dec.close()
