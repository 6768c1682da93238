"""GPU parity of batched runs: many instances of different sizes in one
persistent launch (mcpd_batch_*), against the CPU oracle instance by
instance (criteria in tests/parity.py).  Instance i of a batch draws its
random numbers with g = instance_id + i, so the oracle runs it with that id.
"""

import numpy as np
import pytest

import parity as P
from paper_2608_30239_amd import instances as I

pytestmark = pytest.mark.gpu

N = pytest.importorskip("paper_2608_30239_amd.native")


@pytest.fixture(scope="module", autouse=True)
def _lib():
    N.load()


def mixed_batch():
    """Small and large instances, LDS-resident and global chain state, narrow
    and wide rows, ragged slot counts, refill with several pairs per slot."""
    tiny, _ = I.tiny_plain()
    a = I.make_instance("deg12", 300, 200, (6, 12), 4, 0.08, 0.12, prior=4 / 300, seed=7)
    b = I.make_instance("lds_state_only", 1600, 110, 5, 3, 0.05, 0.1, prior=3 / 1600, seed=4)
    c = I.make_instance("lds_tables_only", 3000, 400, (3, 7), 5, 0.1, 0.05, prior=5 / 3000, seed=5)
    d = I.make_instance("big", 12000, 900, (3, 7), 6, 0.1, 0.1, prior=6 / 12000, seed=2)
    e = I.make_instance("noisy12", 12, 6, 3, 2, 0.25, 0.25, prior=0.3, seed=3)
    ka, ma = I.window_for_sweeps(1, a.n)
    return [
        (tiny, 1000 * 125, 1000, 10, 50),
        (a, 700 * 3 * ma, 700, ka, ma),
        (b, 1300 * 1500, 1300, 60, 600),
        (c, 257 * 1400, 257, 30, 500),
        (d, 300 * 700, 300, 10, 200),
        (e, 999 * 30, 999, 2, 6),
        (tiny, 64 * 9 * 20, 64, 0, 20),
    ]


def run_batch(spec, seed, runs=1, **opt):
    decs = [N.Decoder(inst) for inst, *_ in spec]
    bt = N.Batch(decs, [s[1:] for s in spec], **opt)
    try:
        outs = [bt.run(seed) for _ in range(runs)]
        for i, (inst, budget, slots, k, m) in enumerate(spec):
            nb = max(1, (budget // slots) // max(m, 1))
            b1, b2 = bt.buckets(i, nb)
            outs[-1][i].update(bucket_sum=b1, bucket_sumsq=b2)
            if opt.get("keep_mismatch"):
                outs[-1][i].update(mismatch=bt.mismatch(i))
            if opt.get("keep_slot_records"):
                ns, su = bt.slot_records(i)
                outs[-1][i].update(slot_nstar=ns, slot_units=su)
        cfg = bt.config()
    finally:
        bt.close()
        for d in decs:
            d.close()
    return outs, cfg


@pytest.mark.parametrize("kern", [dict(kernel=1), dict(kernel=2, group_lanes=16), dict(kernel=2, group_lanes=32),
                                  dict(kernel=2)], ids=["lane", "coop16", "coop32", "coop_per_instance"])
def test_mixed_batch_matches_oracle_with_graph_replays(kern):
    spec = mixed_batch()
    base = 40
    outs, cfg = run_batch(spec, seed=11, runs=3, instance_id=base, keep_slot_records=1, keep_mismatch=1, **kern)
    # every replay of the captured graph gives the same answer
    for r in outs[:-1]:
        for i in range(len(spec)):
            assert np.array_equal(r[i]["marginals"], outs[-1][i]["marginals"])
            assert np.array_equal(r[i]["hist"], outs[-1][i]["hist"])
    if kern["kernel"] == 1:
        assert set(cfg["placement"].tolist()) >= {1, 3}
        assert (cfg["wg_slots"] < 256).any() and (cfg["wg_slots"] == 256).any()
    elif "group_lanes" in kern:
        assert ((cfg["placement"] & 5) == 5).all()
        assert (cfg["wg_slots"] == 256 // kern["group_lanes"]).all()
    else:
        # group sizes of 16, 32 or 64 lanes, one per instance
        assert ((cfg["placement"] & 5) == 5).all()
        assert set(cfg["wg_slots"].tolist()) <= {16, 8, 4}
    for i, (inst, budget, slots, k, m) in enumerate(spec):
        orc, nb = P.oracle_run(inst, budget, slots, k, m, seed=11, instance_id=base + i)
        P.check(outs[-1][i], orc, budget, slots, m)


def test_batch_prior_start_with_graph_replays():
    spec = mixed_batch()
    outs, _ = run_batch(spec, seed=19, runs=2, instance_id=7, init_mode=1, kernel=2, group_lanes=16)
    for i in range(len(spec)):
        assert np.array_equal(outs[0][i]["marginals"], outs[1][i]["marginals"])
    for i, (inst, budget, slots, k, m) in enumerate(spec):
        orc, nb = P.oracle_run(inst, budget, slots, k, m, seed=19, instance_id=7 + i, init_mode=1)
        P.check(outs[-1][i], orc, budget, slots, m)


def test_batch_cap_in_sweeps_of_each_instance():
    """cap_sweeps caps every instance at max(cap_sweeps * n_i, m_i) draws:
    the oracle run of instance i with that max_steps."""
    spec = mixed_batch()
    outs, _ = run_batch(spec, seed=23, runs=1, instance_id=3, cap_sweeps=2)
    capped = 0
    for i, (inst, budget, slots, k, m) in enumerate(spec):
        orc, nb = P.oracle_run(inst, budget, slots, k, m, seed=23, instance_id=3 + i,
                               max_steps=max(2 * inst.n, m, 1))
        P.check(outs[-1][i], orc, budget, slots, m)
        capped += int(outs[-1][i]["stats"]["cap_hits"])
    assert capped > 0
    tiny, _ = I.tiny_plain()
    dec = N.Decoder(tiny)
    try:
        a = dec.run(64 * 200, 64, 3, 40, 5, cap_sweeps=3)
        b = dec.run(64 * 200, 64, 3, 40, 5, max_steps=48)
        assert np.array_equal(a["marginals"], b["marginals"]) and a["stats"]["cap_hits"] > 0
        with pytest.raises(N.McpdError):
            dec.run(64 * 200, 64, 3, 40, 5, cap_sweeps=3, max_steps=48)
    finally:
        dec.close()


def test_batch_invariant_to_launch_shape():
    spec = mixed_batch()
    ref, _ = run_batch(spec, seed=5)
    shapes = [dict(kernel=1, wg_per_cu=2, ticket_slots=4), dict(kernel=1, wg_per_cu=3, ticket_slots=2),
              dict(plan=4, wg_per_cu=1), dict(kernel=1, use_graph=0, ticket_slots=8),
              dict(kernel=1, narrow_lanes=256), dict(kernel=1, narrow_lanes=32, wg_per_cu=2),
              dict(kernel=2, wg_per_cu=3, ticket_slots=1, group_lanes=64),
              dict(kernel=2, plan=2, use_graph=0, group_lanes=8),
              dict(kernel=2, wg_per_cu=1), dict(kernel=2, wg_per_cu=4, ticket_slots=2)]
    for sh in shapes:
        got, cfg = run_batch(spec, seed=5, **sh)
        if "wg_per_cu" in sh:
            assert cfg["wg_per_cu"] == sh["wg_per_cu"]
        if sh.get("plan") == 4:
            assert not cfg["placement"].any()
        if sh.get("narrow_lanes") == 256:
            assert (cfg["wg_slots"] == 256).all() and (cfg["placement"] == 0).any()
        if sh.get("kernel") == 2 and "group_lanes" in sh:
            assert (cfg["wg_slots"] == 256 // sh["group_lanes"]).all()
        for a, b in zip(ref[0], got[0]):
            assert np.array_equal(a["bucket_sum"], b["bucket_sum"]), sh
            assert np.array_equal(a["bucket_sumsq"], b["bucket_sumsq"]), sh
            assert np.array_equal(a["marginals"], b["marginals"]), sh
            assert np.array_equal(a["hist"], b["hist"]), sh
            for key in ("retained_units", "reps_retained", "tau_sum", "progress_units"):
                assert a["stats"][key] == b["stats"][key], (sh, key)


def test_batch_equals_single_runs_and_seed_changes():
    spec = mixed_batch()[:4]
    decs = [N.Decoder(inst) for inst, *_ in spec]
    try:
        bt = N.Batch(decs, [s[1:] for s in spec], instance_id=7)
        r1 = bt.run(21)
        r2 = bt.run(22)
        r3 = bt.run(21)
        bt.close()
        for i, (inst, budget, slots, k, m) in enumerate(spec):
            single = decs[i].run(budget, slots, k, m, 21, instance_id=7 + i)
            assert np.array_equal(single["marginals"], r1[i]["marginals"])
            assert np.array_equal(single["hist"], r1[i]["hist"])
            assert np.array_equal(r1[i]["marginals"], r3[i]["marginals"])
            assert not np.array_equal(r1[i]["marginals"], r2[i]["marginals"])
    finally:
        for d in decs:
            d.close()


def test_mismatch_times_only_when_asked_and_change_nothing_else():
    spec = mixed_batch()
    plain, _ = run_batch(spec, seed=13)
    kept, _ = run_batch(spec, seed=13, keep_mismatch=1)
    for a, b in zip(plain[0], kept[0]):
        assert np.array_equal(a["marginals"], b["marginals"]) and np.array_equal(a["hist"], b["hist"])
        assert np.array_equal(a["bucket_sumsq"], b["bucket_sumsq"])
    assert sum(int(r["mismatch"].sum()) for r in kept[0]) > 0
    decs = [N.Decoder(inst) for inst, *_ in spec[:1]]
    try:
        bt = N.Batch(decs, [spec[0][1:]])
        bt.run(1)
        with pytest.raises(N.McpdError, match="not kept"):
            bt.mismatch(0)
        bt.close()
    finally:
        for d in decs:
            d.close()


def test_autotuner_keeps_results():
    spec = mixed_batch()
    decs = [N.Decoder(inst) for inst, *_ in spec]
    try:
        bt = N.Batch(decs, [s[1:] for s in spec])
        before = bt.run(3)
        entries = bt.tune(3)
        assert len(entries) >= 3 and all(e["ms"] > 0 for e in entries)
        best = min(entries, key=lambda e: e["ms"])
        cfg = bt.config()
        assert (cfg["wg_per_cu"], cfg["ticket_slots"]) == (best["wg_per_cu"], best["ticket_slots"])
        after = bt.run(3)
        bt.close()
        for a, b in zip(before, after):
            assert np.array_equal(a["marginals"], b["marginals"])
            assert np.array_equal(a["hist"], b["hist"])
    finally:
        for d in decs:
            d.close()


def test_batch_rejects_bad_arguments():
    tiny, _ = I.tiny_plain()
    dec = N.Decoder(tiny)
    try:
        with pytest.raises(N.McpdError):
            N.Batch([dec], [(0, 0, 1, 2)])                 # slots = 0
        with pytest.raises(N.McpdError):
            N.Batch([dec, dec], [(0, 16, 5, 4), (0, 16, 1, 2)])   # k > m
        with pytest.raises(N.McpdError):
            N.Batch([dec], [(0, 16, 1, 2)], instance_id=(1 << 24) - 1 + 1)
        bt = N.Batch([dec], [(0, 16, 1, 2)])
        with pytest.raises(N.McpdError):
            bt.slot_records(0)                             # not kept
        assert N.load().mcpd_batch_buckets(bt.h, 1, 1, None, None) == N.MCPD_EINVAL   # no instance 1
        assert N.load().mcpd_batch_buckets(bt.h, -1, 1, None, None) == N.MCPD_EINVAL
        bt.close()
    finally:
        dec.close()


def test_noise_sweep_full_size_every_instance():
    """128 instances (the 1298x97 design, 16 noise settings x 8 seeds), 2^24
    updates each over 4096 slots, in one launch: every instance bit-exact."""
    insts, rp = I.noise_sweep()
    spec = [(x, rp.budget, rp.slots, rp.k, rp.m) for x in insts]
    outs, cfg = run_batch(spec, seed=rp.seed, keep_slot_records=1, keep_mismatch=1)
    assert ((cfg["placement"] & 3) == 3).all()
    for i, (inst, budget, slots, k, m) in enumerate(spec):
        orc, _ = P.oracle_run(inst, budget, slots, k, m, seed=rp.seed, instance_id=i)
        P.check(outs[0][i], orc, budget, slots, m)


def test_uneven_batch_full_size_every_instance():
    """256 uneven instances (n in [200, 20000]) in one launch at full size:
    every instance in full against the oracle, and against the invariants
    of its slot records."""
    insts, params = I.uneven_batch()
    spec = [(x, p.budget, p.slots, p.k, p.m) for x, p in zip(insts, params)]
    outs, cfg = run_batch(spec, seed=0, keep_slot_records=1, keep_mismatch=1)
    res = outs[0]
    for i, (inst, budget, slots, k, m) in enumerate(spec):
        st = res[i]["stats"]
        B = budget // slots
        assert int(res[i]["slot_units"].sum()) == st["retained_units"]
        assert (res[i]["slot_nstar"] >= 1).all()
        assert int(res[i]["slot_nstar"].max()) == st["nstar_max"]
        # a slot's retained units stay within B unless its first pair overran
        over = res[i]["slot_units"] > B
        assert int(over.sum()) == st["zero_completion_slots"]
        assert int(res[i]["hist"].sum()) + st["cap_hits"] == st["reps_retained"]
    for i, (inst, budget, slots, k, m) in enumerate(spec):
        print(f"[oracle] uneven instance {i}: n={inst.n} m={inst.m} slots={slots}", flush=True)
        orc, _ = P.oracle_run(inst, budget, slots, k, m, seed=0, instance_id=i)
        P.check(res[i], orc, budget, slots, m)


def test_uneven_batch_capped_every_instance():
    """The same batch with the paper's meeting cap of 20 sweeps per instance
    (cap_sweeps = 20): pairs stopped by the cap keep the truncated estimator,
    every instance in full against the oracle run with that cap."""
    insts, params = I.uneven_batch()
    spec = [(x, p.budget, p.slots, p.k, p.m) for x, p in zip(insts, params)]
    outs, cfg = run_batch(spec, seed=1, keep_slot_records=1, keep_mismatch=1, cap_sweeps=20)
    res = outs[0]
    assert sum(r["stats"]["cap_hits"] for r in res) > 0
    # one launch, group sizes chosen per instance (small instances run
    # groups of 16 lanes, the largest groups of 64)
    assert len({r["stats"]["group_lanes"] for r in res}) > 1
    for i, (inst, budget, slots, k, m) in enumerate(spec):
        print(f"[oracle] capped uneven instance {i}: n={inst.n} m={inst.m} slots={slots}", flush=True)
        orc, _ = P.oracle_run(inst, budget, slots, k, m, seed=1, instance_id=i, max_steps=20 * inst.n)
        P.check(res[i], orc, budget, slots, m)
