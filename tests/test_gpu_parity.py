"""GPU parity of single runs (mcpd_run_unbiased): the HIP path through the
C ABI against the CPU oracle (criteria in tests/parity.py)."""

import numpy as np
import pytest

import parity as P
from paper_2608_30239_amd import instances as I

pytestmark = pytest.mark.gpu

N = pytest.importorskip("paper_2608_30239_amd.native")


@pytest.fixture(scope="module", autouse=True)
def _lib():
    N.load()


# every generic case runs on both kernels: one slot per lane, and one slot
# per group of 8, 16 or 64 lanes drawing speculatively
@pytest.fixture(params=[dict(kernel=1), dict(kernel=2, group_lanes=8), dict(kernel=2, group_lanes=16),
                        dict(kernel=2, group_lanes=64)], ids=["lane", "coop8", "coop16", "coop64"])
def kern(request):
    return request.param


def compare(inst, budget, slots, k, m, seed=0, weights=None, tol=1e-12, **opt):
    """Run both sides and compare everything; returns (gpu, oracle)."""
    orc, nb = P.oracle_run(inst, budget, slots, k, m, seed, weights=weights, **opt)
    dec = N.Decoder(inst)
    try:
        if weights is not None:
            dec.set_weights(weights)
        w_exact, mass = dec.weights()
        assert np.array_equal(mass, orc["masses"])
        gpu = dec.run(budget, slots, k, m, seed, slot_records=True, buckets=nb, mismatch=True, **opt)
    finally:
        dec.close()
    P.check(gpu, orc, budget, slots, m, tol)
    return gpu, orc


def test_tiny_plain_one_pair_per_slot(kern):
    inst, rp = I.tiny_plain()
    gpu, orc = compare(inst, rp.budget, rp.slots, rp.k, rp.m, rp.seed, **kern)
    assert gpu["stats"]["kernel"] == kern["kernel"]
    assert gpu["stats"]["group_lanes"] == kern.get("group_lanes", 1)
    assert gpu["stats"]["reps_retained"] == rp.slots


@pytest.mark.parametrize("slots,mult,k,m", [(1000, 2.5, 10, 50), (333, 4.0, 0, 0), (257, 3.3, 7, 7),
                                            (64, 9.0, 0, 20), (1, 5.0, 3, 30)])
def test_tiny_refill_ragged(slots, mult, k, m, kern):
    inst, _ = I.tiny_plain()
    B = int(mult * max(m, 1))
    gpu, orc = compare(inst, B * slots, slots, k, m, seed=3, hist_width=1, **kern)
    if mult > 1:
        assert gpu["stats"]["reps_retained"] > slots


def test_refill_off_and_instance_id(kern):
    inst, _ = I.tiny_plain()
    compare(inst, 4096 * 200, 4096, 10, 50, seed=5, refill=0, instance_id=77, **kern)


@pytest.mark.parametrize("degree", [(1, 4), (1, 5), (4, 5)], ids=["u8x4-mixed", "u8x5-mixed", "u8x5-4or5"])
def test_one_byte_rows_with_padding(degree, kern):
    """Rows of one-byte entries (m <= 127) whose clones have fewer pools than
    a row holds: the padding entries must never count as free pools, on the
    lane kernel and on the cooperative kernel, which takes the threshold
    index of 4- and 5-entry rows from its pattern table."""
    inst = I.make_instance("pad", 400, 60, degree, 4, 0.08, 0.12, prior=4 / 400, seed=11)
    d = inst.degrees()
    assert d.min() < d.max() == degree[1] and inst.m <= 127
    compare(inst, 256 * 3 * 400, 256, 41, 400, seed=12, **kern)
    compare(inst, 256 * 3 * 400, 256, 41, 400, seed=13, init_mode=1, **kern)


def test_one_decoder_through_changing_shapes():
    """One decoder (its launch plan, workspace and output block reused) through
    runs whose shapes change: slot counts that are and are not multiples of
    the per-XCD slot ranges, fewer slots than ranges, one slot, both kernels
    and several group sizes, both initial distributions, an empty window;
    every run against the oracle."""
    inst, _ = I.tiny_plain()
    runs = [(4096 * 120, 4096, 10, 50, dict()),
            (7 * 200, 7, 10, 50, dict(kernel=2, group_lanes=8)),
            (1 * 300, 1, 3, 30, dict(kernel=1)),
            (1000 * 130, 1000, 0, 0, dict(kernel=2, group_lanes=64, init_mode=1)),
            (8191 * 55, 8191, 5, 20, dict(kernel=2, group_lanes=16)),
            (333 * 400, 333, 10, 50, dict(kernel=1, init_mode=1)),
            (4096 * 120, 4096, 10, 50, dict())]
    dec = N.Decoder(inst)
    try:
        for i, (budget, slots, k, m, opt) in enumerate(runs):
            orc, nb = P.oracle_run(inst, budget, slots, k, m, seed=40 + i, **opt)
            gpu = dec.run(budget, slots, k, m, 40 + i, slot_records=True, buckets=nb, **opt)
            P.check(gpu, orc, budget, slots, m)
    finally:
        dec.close()


def test_meeting_cap_truncation(kern):
    inst = I.make_instance("noisy12", 12, 6, 3, 2, 0.25, 0.25, prior=0.3, seed=3)
    gpu, orc = compare(inst, 2000 * 30, 2000, 2, 6, seed=9, max_steps=8, hist_width=1, **kern)
    assert orc["stats"]["cap_hits"] > 0


def test_low_bit_refinement_path(kern):
    # u_hi_bits = 2 makes the high part of U tie with the threshold often,
    # so the low-bit block decides many draws
    inst, _ = I.tiny_plain()
    compare(inst, 512 * 150, 512, 10, 50, seed=2, u_hi_bits=2, **kern)
    compare(inst, 512 * 150, 512, 10, 50, seed=2, u_hi_bits=13, **kern)


def test_user_weights(kern):
    inst, _ = I.tiny_plain()
    w = np.linspace(1.0, 3.0, inst.n)
    compare(inst, 2048 * 120, 2048, 10, 50, seed=4, weights=w, **kern)


def test_degree_up_to_twelve_and_wide_pools(kern):
    inst = I.make_instance("deg12", 300, 200, (6, 12), 4, 0.08, 0.12, prior=4 / 300, seed=7)
    k, m = I.window_for_sweeps(1, inst.n)
    compare(inst, 1024 * 4 * m, 1024, k, m, seed=1, **kern)


def test_global_state_path():
    # chain state and tables in global memory (forced)
    inst = I.make_instance("big", 12000, 900, (3, 7), 6, 0.1, 0.1, prior=6 / 12000, seed=2)
    k, m = 10, 200
    gpu, _ = compare(inst, 512 * 700, 512, k, m, seed=6, plan=4)
    assert gpu["stats"]["placement"] == 0 and gpu["stats"]["wg_slots"] == 256 and gpu["stats"]["kernel"] == 1


def test_narrow_lds_layout():
    # 4.8 KB of state per lane: by default a workgroup runs 33 lanes with the
    # state in LDS; the same run with wide layouts only keeps it in global memory
    inst = I.make_instance("big", 12000, 900, (3, 7), 6, 0.1, 0.1, prior=6 / 12000, seed=2)
    gpu, _ = compare(inst, 512 * 700, 512, 10, 200, seed=6, kernel=1)
    assert gpu["stats"]["placement"] == 1 and 8 <= gpu["stats"]["wg_slots"] < 256
    gpu2, _ = compare(inst, 512 * 700, 512, 10, 200, seed=6, narrow_lanes=256, kernel=1)
    assert gpu2["stats"]["placement"] in (0, 2) and gpu2["stats"]["wg_slots"] == 256
    gpu3, _ = compare(inst, 512 * 700, 512, 10, 200, seed=6, kernel=2, group_lanes=32)
    assert gpu3["stats"]["placement"] & 5 == 5 and gpu3["stats"]["wg_slots"] == 8


def test_lds_state_global_tables():
    # state fills LDS at 256 lanes, the tables no longer fit beside it
    inst = I.make_instance("lds_state_only", 1600, 110, 5, 3, 0.05, 0.1, prior=3 / 1600, seed=4)
    gpu, _ = compare(inst, 2048 * 2000, 2048, 60, 600, seed=2, kernel=1)
    assert gpu["stats"]["placement"] == 1


def test_global_state_lds_tables():
    inst = I.make_instance("lds_tables_only", 3000, 400, (3, 7), 5, 0.1, 0.05, prior=5 / 3000, seed=5)
    gpu, _ = compare(inst, 1024 * 1500, 1024, 30, 500, seed=3, plan=3, kernel=1)
    assert gpu["stats"]["placement"] == 2


def test_narrow_layout_with_tables_and_ragged_lanes():
    # state 1.5 KB per lane: narrow layouts with and without the tables
    inst = I.make_instance("lds_tables_only", 3000, 400, (3, 7), 5, 0.1, 0.05, prior=5 / 3000, seed=5)
    gpu, _ = compare(inst, 1000 * 1500, 1000, 30, 500, seed=4, kernel=1)
    assert gpu["stats"]["placement"] & 1 and gpu["stats"]["wg_slots"] < 256
    gpu, _ = compare(inst, 1000 * 1500, 1000, 30, 500, seed=4, plan=1, narrow_lanes=8, kernel=1)
    assert gpu["stats"]["placement"] == 3 and gpu["stats"]["wg_slots"] < 256
    gpu, _ = compare(inst, 1000 * 1500, 1000, 30, 500, seed=4, plan=2, kernel=2)
    assert gpu["stats"]["placement"] == 5


def test_deterministic_repeat(kern):
    inst, rp = I.tiny_plain()
    dec = N.Decoder(inst)
    try:
        a = dec.run(4096 * 150, 4096, 10, 50, seed=8, buckets=3, **kern)
        b = dec.run(4096 * 150, 4096, 10, 50, seed=8, buckets=3, **kern)
    finally:
        dec.close()
    assert np.array_equal(a["marginals"], b["marginals"])
    assert np.array_equal(a["bucket_sum"], b["bucket_sum"])
    assert np.array_equal(a["hist"], b["hist"])


def test_invalid_arguments_raise():
    inst, _ = I.tiny_plain()
    dec = N.Decoder(inst)
    try:
        with pytest.raises(N.McpdError):
            dec.run(0, 0, 1, 2)               # slots = 0
        with pytest.raises(N.McpdError):
            dec.run(0, 16, 5, 4)              # k > m
        with pytest.raises(N.McpdError):
            dec.run(0, 16, 1, 10, max_steps=5)  # cap below m
        with pytest.raises(N.McpdError):
            dec.set_weights(np.zeros(inst.n))
        with pytest.raises(N.McpdError):
            dec.run(0, 16, 1, 2, init_mode=2)  # no such initial distribution
    finally:
        dec.close()


# the prior as initial distribution: clones start positive in both chains,
# which adds window terms, count changes and touched-list entries at the
# start of every replication (and of every replay)
@pytest.mark.parametrize("slots,mult,k,m", [(1000, 2.5, 10, 50), (257, 3.3, 7, 7), (64, 9.0, 0, 20),
                                            (1, 5.0, 3, 30)])
def test_prior_start_ragged(slots, mult, k, m, kern):
    inst, _ = I.tiny_plain()
    inst.prior = 0.2
    B = int(mult * max(m, 1))
    gpu, orc = compare(inst, B * slots, slots, k, m, seed=3, hist_width=1, init_mode=1, **kern)
    assert gpu["stats"]["reps_retained"] >= slots


def test_prior_start_paper_shaped(kern):
    inst, rp = I.paper_shaped()
    compare(inst, 4096 * 4096, 4096, rp.k, rp.m, seed=8, init_mode=1, **kern)


def test_prior_start_pruned_with_cap(kern):
    full = I.knill_degree3(fn=0.1, fp=0.1)
    inst = I.restrict(full, N.mcpd_prune(full, 333))
    inst.prior = 0.01
    k, l = I.window_for_sweeps(1, inst.n)
    compare(inst, 20 * inst.n * 2048, 2048, k, l, seed=2, max_steps=20 * inst.n, init_mode=1, **kern)


def test_paper_shaped_full_size(kern):
    inst, rp = I.paper_shaped()
    gpu, orc = compare(inst, rp.budget, rp.slots, rp.k, rp.m, rp.seed, **kern)
    assert gpu["stats"]["placement"] & 1          # chain state in LDS
    assert gpu["stats"]["nstar_max"] >= 3


# Slots whose events touch more clones than their group has lanes: the
# group's per-lane numerator entries are evicted into its global row in
# turn, and the slot's flush goes through the touched list, or scans the row
# once the list has overflowed (its capacity here is 64 entries)
@pytest.mark.parametrize("design", [(300, 40, 3, 10, 0.1, 0.1), (600, 60, 4, 12, 0.15, 0.15)], ids=["n300", "n600"])
@pytest.mark.parametrize("lanes", [8, 16, 64])
@pytest.mark.parametrize("init_mode", [0, 1], ids=["zero_start", "prior_start"])
def test_numerator_entries_evicted(design, lanes, init_mode):
    from oracle import oracle as O
    n = design[0]
    inst = I.make_instance("evict", *design, prior=design[3] / n, seed=3)
    k, m, cap = n // 10, n, 20 * n
    # how many clones a replication leaves a nonzero numerator on (a lower
    # bound on the clones its events touch), on the oracle
    M = O.Model(inst)
    touched = np.array([(M.trace(p, 1, max_len=cap, k=k, m=m, budget=0, slots=1, seed=5, max_steps=cap)["numer"]
                         != 0).sum() for p in range(16)])
    if lanes < 64 or n == 600:
        assert (touched > lanes).mean() >= 0.25
    slots = 256
    # the prior start (init_mode 1) also puts the window terms of the clones
    # that start positive in the row and the touched list before any event
    gpu, _ = compare(inst, slots * 3 * m, slots, k, m, seed=5, max_steps=cap, kernel=2, group_lanes=lanes,
                     init_mode=init_mode)
    assert gpu["stats"]["group_lanes"] == lanes
