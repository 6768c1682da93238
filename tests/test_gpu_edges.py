"""GPU parity at the edges of the input domain (criteria in tests/parity.py):
one clone and one pool, clones in no pool, a pool of the largest size, the
largest degree with the most pools, rates near 0 and 1, extreme selection
weights, a horizon shorter than the window, and the largest clone count the
numerator workspace allows at the paper's window."""

import numpy as np
import pytest

from paper_2608_30239_amd import instances as I
from test_gpu_parity import compare, kern  # noqa: F401  (kern is a fixture)

pytestmark = pytest.mark.gpu

N = pytest.importorskip("paper_2608_30239_amd.native")


def from_rows(name, rows, m, y, fp, fn, q):
    row_ptr, pool_idx = I._csr_from_rows([np.asarray(sorted(r), np.int32) for r in rows])
    return I.Instance(name, len(rows), m, row_ptr, pool_idx, np.asarray(y, np.uint8), fp, fn, q,
                      np.zeros(0, np.int32))


@pytest.mark.parametrize("y", [0, 1])
def test_one_clone_one_pool(y, kern):
    inst = from_rows("one", [[0]], 1, [y], 0.1, 0.2, 0.3)
    compare(inst, 64 * 40, 64, 0, 10, seed=1, **kern)
    compare(inst, 64 * 40, 64, 2, 10, seed=2, init_mode=1, **kern)


def test_clones_in_no_pool(kern):
    rng = np.random.default_rng(4)
    rows = [sorted(rng.choice(6, size=2, replace=False).tolist()) if i % 2 else [] for i in range(20)]
    inst = from_rows("isolated", rows, 6, [1, 0, 1, 0, 0, 1], 0.1, 0.1, 0.2)
    compare(inst, 300 * 120, 300, 5, 40, seed=3, **kern)


def test_pool_of_largest_size(kern):
    # every clone is in pool 0 (255 clones) and in two of seven other pools
    rng = np.random.default_rng(5)
    rows = [[0] + sorted((1 + rng.choice(7, size=2, replace=False)).tolist()) for _ in range(255)]
    inst = from_rows("pool255", rows, 8, [1, 1, 0, 1, 0, 0, 1, 0], 0.05, 0.1, 0.3)
    assert np.bincount(inst.pool_idx).max() == 255
    compare(inst, 256 * 3 * 255, 256, 26, 255, seed=4, **kern)
    compare(inst, 256 * 3 * 255, 256, 26, 255, seed=5, init_mode=1, **kern)


def test_largest_degree_and_most_pools(kern):
    inst = I.make_instance("deg12_m32767", 4000, 32767, 12, 6, 0.05, 0.1, prior=6 / 4000, seed=9)
    assert inst.degrees().max() == 12 and inst.m == 32767
    if kern["kernel"] == 2:
        # 16384 count words per slot: no group state fits in LDS, and the
        # cooperative kernel says so instead of running
        dec = N.Decoder(inst)
        try:
            with pytest.raises(N.McpdError, match="do not fit"):
                dec.run(512 * 2 * 4000, 512, 401, 4000, 6, **kern)
        finally:
            dec.close()
        return
    compare(inst, 512 * 2 * 4000, 512, 401, 4000, seed=6, **kern)


@pytest.mark.parametrize("fp,fn", [(1e-9, 0.999999), (0.999999, 1e-9), (0.5, 0.5)])
def test_extreme_rates(fp, fn, kern):
    inst = I.make_instance("rates", 200, 30, 3, 3, min(fp, 0.5), min(fn, 0.5), prior=0.05, seed=2)
    inst.fp, inst.fn = fp, fn
    compare(inst, 512 * 600, 512, 20, 200, seed=7, **kern)


def test_extreme_weights(kern):
    inst, rp = I.tiny_plain()
    w = np.array([1e-300] * 8 + [1.0] * 7 + [1e300 * 1e-290], np.float64)
    compare(inst, 1024 * 200, 1024, rp.k, rp.m, seed=8, weights=w, **kern)


def test_horizon_shorter_than_window(kern):
    inst, rp = I.tiny_plain()
    # B = l / 2: every slot keeps its first pair (the zero-completion rule)
    gpu, orc = compare(inst, 2048 * (rp.m // 2), 2048, rp.k, rp.m, seed=9, **kern)
    assert gpu["stats"]["zero_completion_slots"] == 2048


@pytest.mark.parametrize("n,opt", [(1 << 17, dict(kernel=1, wg_per_cu=1)), (1 << 16, dict(kernel=2, group_lanes=64)),
                                   (1 << 17, dict(kernel=2, group_lanes=64))],
                         ids=["lane-global-state-131072", "coop64-65536", "coop64-131072-refused"])
def test_largest_clone_count(n, opt):
    """The lane kernel keeps chain states of 2^17 clones in global memory;
    the cooperative kernel holds a group's state in LDS, 4 groups per
    workgroup at least, so 2^16 clones (32 KB per group) run and 2^17
    (49 KB) are refused with MCPD_EINVAL."""
    inst = I.make_instance(f"n{n}", n, 8000, 3, 8, 0.05, 0.1, prior=8 / n, seed=3)
    args = (256 * 2 * n, 256, n // 10 + 1, n)
    if n == (1 << 17) and opt["kernel"] == 2:
        dec = N.Decoder(inst)
        try:
            with pytest.raises(N.McpdError, match="do not fit"):
                dec.run(*args, 10, **opt)
        finally:
            dec.close()
        return
    gpu, _ = compare(inst, *args, seed=10, **opt)
    if opt["kernel"] == 1:
        assert not (gpu["stats"]["placement"] & 1)      # state in global memory
    else:
        assert gpu["stats"]["placement"] & 4


def test_strict_cap_reports_mcpd_ecap(kern):
    """strict_cap: a run in which a retained pair hits the meeting cap
    returns MCPD_ECAP; the same run without it returns the capped estimate,
    which matches the oracle's truncated one."""
    inst, rp = I.tiny_plain()
    cap = rp.m   # the smallest cap allowed: max(m, 1) draws
    gpu, orc = compare(inst, 2048 * 3 * rp.m, 2048, rp.k, rp.m, seed=11, max_steps=cap, **kern)
    assert gpu["stats"]["cap_hits"] > 0 and orc["stats"]["cap_hits"] == gpu["stats"]["cap_hits"]
    dec = N.Decoder(inst)
    try:
        with pytest.raises(N.McpdError) as e:
            dec.run(2048 * 3 * rp.m, 2048, rp.k, rp.m, 11, max_steps=cap, strict_cap=1, **kern)
        assert e.value.code == N.MCPD_ECAP
        # no pair reaches a cap of 2^32 - 1 draws: strict mode returns normally
        ok = dec.run(2048 * 3 * rp.m, 2048, rp.k, rp.m, 11, strict_cap=1, **kern)
        assert ok["stats"]["cap_hits"] == 0
    finally:
        dec.close()


def test_numerator_workspace_limit_reports_mcpd_enomem():
    """The lane kernel's dense numerator rows (lanes x n x 8 bytes) are
    capped at 64 GiB: 2^17 clones with enough slots (2^20) to fill two
    workgroups of 256 lanes on every CU would need 128 GiB, so the run
    returns MCPD_ENOMEM before allocating anything or launching, and the
    instance still runs afterwards."""
    n = 1 << 17
    inst = I.make_instance(f"n{n}", n, 8000, 3, 8, 0.05, 0.1, prior=8 / n, seed=3)
    dec = N.Decoder(inst)
    try:
        slots = 1 << 20
        with pytest.raises(N.McpdError) as e:
            dec.run(slots * n, slots, n // 10 + 1, n, 10, kernel=1, wg_per_cu=2)
        assert e.value.code == N.MCPD_ENOMEM
        ok = dec.run(256 * 2000, 256, 200, 2000, 10, kernel=1, wg_per_cu=1)
        assert ok["stats"]["reps_retained"] >= 256
    finally:
        dec.close()
