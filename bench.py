"""Benchmark: coupled Gibbs updates per second of the unbiased MCPD hot path.

One step = one full fixed-budget run (mcpd_run_unbiased_dev) of the
paper-shaped workload: 1298 clones, 97 pools, degree 5, 3 positives, fp 0.05,
fn 0.10, q = 3/1298, budget 2^28 progress units over 65536 slots (B = 4096),
window k = 131, l = 1298 (one sweep), score weights.  The instance tables are
resident in device memory before the timed region; every step runs the
sampler kernel, the integer bucket reduction and the final FP64 division on
the device, with a new seed per step, and leaves the marginals, standard
errors and histogram in device memory.  The same runs with host outputs
(mcpd_run_unbiased, PCIe-inclusive) are reported beside it.

Also reported on the same line: the batched workloads (128-instance noise
sweep, 256-instance uneven batch uncapped and with the paper's meeting cap
of 20 sweeps per instance) as one persistent launch replayed from a captured
graph, and the learned selection weights against the score
weights on the same paper-shaped workload at equal budget (RMSE against an
independent long reference run, device seconds, efficiency 1/(MSE s)).

Prints one JSON line.  Only one GPU is used; --gpus N > 1 exits.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Iterations of each peak-rate probe (about 10-30 ms of device time each).
PROBE_ITERS = {"lds_b32": 40000, "lds_b64": 20000, "lds_b128": 10000, "lds_b32_random": 20000,
               "valu_add": 40000, "valu_mul_lo": 10000, "valu_mul_hi": 10000, "valu_bitop3": 40000,
               "valu_mul64": 10000, "philox10": 20000}


def lds_bytes_per_update(d: float) -> float:
    """Algorithmic LDS bytes of one coupled update at dword granularity: per
    pair the bit word holding x_I and y_I (4) and one dword per pool of the
    drawn clone (4d); shared per instance the alias column (8) and the clone
    row (8).  20 + 4d = 40 B at degree 5."""
    return 4.0 + 4.0 * d + 8.0 + 8.0


def alg_full_rate_ops(d: float) -> float:
    """Algorithmic full-rate 32-bit lane operations of one update besides its
    random numbers: the alias site draw (shift, mask, compare, select) = 4,
    the free test and pattern step of each of the d pools = 4d, the
    threshold index and 53-bit comparison = 4."""
    return 4.0 + 4.0 * d + 4.0


def measure_peaks():
    """Peak rates of the device measured by the library's probes."""
    from paper_2608_30239_amd import native as N
    return {k: N.mcpd_probe(k, PROBE_ITERS[k]) for k in N.PROBES}


def roofline_of(peaks, d: float, units_per_launch: float, kernel_s: float, kernel_name: str):
    """Achieved rates of one launch against the measured peaks.

    LDS: algorithmic bytes (lds_bytes_per_update x the launch's retained
    updates) over the launch's time, against the best streaming LDS read
    rate the probes measured.  VALU: the algorithmic work of one update is
    half a Philox4x32-10 block (one block serves two draws) plus
    alg_full_rate_ops full-rate lane operations; at the measured Philox
    block rate and 32-bit add rate that bounds the update rate at
    1 / (0.5 / philox_per_s + ops / add_per_s)."""
    lds_peak = max(peaks[k]["per_second"] for k in ("lds_b32", "lds_b64", "lds_b128"))
    best = max(("lds_b32", "lds_b64", "lds_b128"), key=lambda k: peaks[k]["per_second"])
    lds_ach = lds_bytes_per_update(d) * units_per_launch / kernel_s
    upd = units_per_launch / kernel_s
    alu_roof = 1.0 / (0.5 / peaks["philox10"]["per_second"] + alg_full_rate_ops(d) / peaks["valu_add"]["per_second"])
    return {
        "bound": "lds",
        "achieved": lds_ach / 1e12,
        "peak": lds_peak / 1e12,
        "unit": "TB/s",
        "frac": lds_ach / lds_peak,
        "traffic": measured_traffic(),
        "kernel": kernel_name,
        "lds_bytes_per_update": lds_bytes_per_update(d),
        "lds_peak_probe": best,
        "lds_peak_bytes_per_cu_per_clock": peaks[best]["per_cu_per_clock"],
        "alu": {
            "achieved_updates_per_s": upd,
            "peak_updates_per_s": alu_roof,
            "frac": upd / alu_roof,
            "philox_blocks_per_s": peaks["philox10"]["per_second"],
            "add_lane_ops_per_s": peaks["valu_add"]["per_second"],
            "full_rate_ops_per_update": alg_full_rate_ops(d),
        },
        "binding": "valu issue (SQ counters: VALU busy is high while LDS runs far below its peak)",
        "peaks_measured": {k: {"per_cu_per_clock": v["per_cu_per_clock"], "per_second": v["per_second"],
                               "clock_hz": v["clock_hz"]} for k, v in peaks.items()},
    }


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 summary, or None when
    the sampler source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "sampler_knill1298x97_hbm.md")
    src = os.path.join(ROOT, "paper_2608_30239_amd", "csrc", "mcpd_sampler.hip")
    try:
        text = open(path).read()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    fields = dict(line.split(": ", 1) for line in text.splitlines() if ": " in line and
                  line.split(": ", 1)[0] in ("kernel_sha256", "traffic_bytes_per_launch"))
    if fields.get("kernel_sha256") != sha:
        return None
    return float(fields["traffic_bytes_per_launch"])


def cpu_baseline(inst, rp, threads: int, min_seconds: float = 10.0, max_runs: int = 12):
    """The oracle on the same workload, whole runs with new seeds until at
    least min_seconds of CPU time have passed."""
    from oracle import oracle as O
    M = O.Model(inst)
    units, dt, runs = 0, 0.0, 0
    while runs < max_runs and (runs == 0 or dt < min_seconds):
        t0 = time.perf_counter()
        r = M.run(rp.budget, rp.slots, rp.k, rp.m, seed=rp.seed + runs, nthreads=threads)
        dt += time.perf_counter() - t0
        units += r["stats"]["retained_units"]
        runs += 1
    return dict(value=units / dt, unit="coupled Gibbs updates/s", cores=threads, kind="oracle",
                seconds_per_run=dt / runs,
                sample=f"{runs} whole runs of the workload ({rp.slots} slots, budget {rp.budget}); "
                       f"{units} retained coupled updates in {dt:.2f} s (the oracle also runs the "
                       f"replications it discards to their end; they are not counted)")


def cpu_baseline_one_thread(inst, rp, slots: int = 4096, min_seconds: float = 3.0):
    """The oracle on one thread, on a bounded sample of the same workload:
    its first `slots` slots at the same per-slot horizon B, new seeds until
    at least min_seconds have passed."""
    from oracle import oracle as O
    M = O.Model(inst)
    B = rp.budget // rp.slots
    units, dt, runs = 0, 0.0, 0
    while runs == 0 or dt < min_seconds:
        t0 = time.perf_counter()
        r = M.run(B * slots, slots, rp.k, rp.m, seed=rp.seed + runs, nthreads=1)
        dt += time.perf_counter() - t0
        units += r["stats"]["retained_units"]
        runs += 1
    return dict(value=units / dt, unit="coupled Gibbs updates/s", cores=1, kind="oracle",
                sample=f"{runs} runs of the first {slots} slots of the workload (B = {B}); "
                       f"{units} retained coupled updates in {dt:.2f} s")


def batch_lines(steps: int):
    """One persistent launch per batched workload, autotuned, then replayed
    from its captured graph."""
    from paper_2608_30239_amd import instances as I
    from paper_2608_30239_amd import native as N
    out = {}
    insts, rp = I.noise_sweep()
    work = {"noise_sweep_128x1298": (insts, [(rp.budget, rp.slots, rp.k, rp.m)] * len(insts))}
    insts, params = I.uneven_batch()
    work["uneven_256"] = (insts, [(p.budget, p.slots, p.k, p.m) for p in params])
    # the same batch with the paper's meeting cap of 20 sweeps per instance
    work["uneven_256_cap20sweeps"] = (insts, work["uneven_256"][1], dict(cap_sweeps=20))
    for name, spec in work.items():
        insts, params = spec[0], spec[1]
        decs = [N.Decoder(x) for x in insts]
        bt = N.Batch(decs, params, **(spec[2] if len(spec) > 2 else {}))
        try:
            tuned = bt.tune(12345)
            bt.run(12345, outputs=False)
            ms, units = [], 0
            for s in range(steps):
                r = bt.run(s, outputs=False)
                ms.append(r[0]["stats"]["kernel_ms"])
                units += sum(x["stats"]["retained_units"] for x in r)
            cfg = bt.config()
            out[name] = dict(instances=len(insts), graph_ms=sum(ms) / len(ms),
                             updates_per_s=units / (sum(ms) / 1e3), kernel=r[0]["stats"]["kernel"],
                             group_lanes={str(g): sum(x["stats"]["group_lanes"] == g for x in r)
                                          for g in sorted({x["stats"]["group_lanes"] for x in r})},
                             wg_per_cu=cfg["wg_per_cu"],
                             ticket_slots=cfg["ticket_slots"], tuner_candidates=len(tuned),
                             tau_max=max(x["stats"]["tau_max"] for x in r),
                             cap_hits=sum(x["stats"]["cap_hits"] for x in r))
        finally:
            bt.close()
            for d in decs:
                d.close()
    return out


def learned_line(nref: int, nrep: int):
    """Learned against score weights at equal budget on the five held-out
    evaluation instances (the paper-shaped one and four with 20000 clones),
    each with a bootstrap interval of the gain."""
    from paper_2608_30239_amd import native as N
    from paper_2608_30239_amd import selection as S
    params, rep = S.load_trained()
    net = N.Mlp(params)
    try:
        res = S.evaluate(net, nref=nref, nrep=nrep, log=lambda m: None)
    finally:
        net.close()
    keep = ("rmse_score", "rmse_learned", "seconds_score", "seconds_learned", "gain", "gain_ci90", "median_gain",
            "var_gain", "tau_max_p99")
    return dict(instances={r["instance"]: {k: r[k] for k in keep} for r in res["rows"]},
                gain_geomean=res["gain_geomean"], median_gain_geomean=res["median_gain_geomean"],
                reference_runs=nref, runs=nrep, weight_floor=S.FLOOR,
                metric="efficiency 1/(MSE x device seconds), learned over score weights; 90% bootstrap interval")


def copy_calibration(mib: int, reps: int):
    """A plain device copy of known size, for scaling FETCH_SIZE/WRITE_SIZE."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n * 4, "reps": reps}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batches", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run a device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: the library runs one process on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.copy_calibration_mib:
        copy_calibration(args.copy_calibration_mib, max(1, args.steps))
        return

    from paper_2608_30239_amd import instances as I
    from paper_2608_30239_amd import native as N

    import torch

    inst, rp = I.paper_shaped()
    d_mean = float(inst.degrees().mean())
    dec = N.Decoder(inst)
    # outputs stay in device memory (mcpd_run_unbiased_dev): the timed steps
    # move no marginals over PCIe; only the run's counters come back
    marg = torch.empty(inst.n, dtype=torch.float64, device="cuda")
    se = torch.empty(inst.n, dtype=torch.float64, device="cuda")
    hist = torch.empty(64, dtype=torch.int64, device="cuda")

    def step(seed):
        return dec.run_dev(rp.budget, rp.slots, rp.k, rp.m, seed, marg.data_ptr(), se.data_ptr(), hist.data_ptr(),
                           hist_bins=64)

    for i in range(args.warmup):
        step(rp.seed + 1000 + i)
    # value counts the method's updates: the draws of retained replications.
    # A replication that can no longer be retained is stopped and its draws
    # are replayed negated; those draws are counted apart (rollback_units).
    units = 0
    progress = 0
    rollback = 0
    kernel_ms = []
    site_updates = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        st = step(rp.seed + i)
        units += st["retained_units"]
        progress += st["progress_units"]
        rollback += st["rollback_units"]
        site_updates += st["single_site_updates"]
        kernel_ms.append(st["kernel_ms"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # the same runs with host outputs (mcpd_run_unbiased): integer sums copied
    # back and divided on the host, so this rate includes the PCIe transfer
    host_steps = max(1, min(args.steps, 10))
    host_units = 0
    dec.run(rp.budget, rp.slots, rp.k, rp.m, rp.seed + 2000)   # warm-up of the host-output path
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for i in range(host_steps):
        host_units += dec.run(rp.budget, rp.slots, rp.k, rp.m, rp.seed + i)["stats"]["retained_units"]
    torch.cuda.synchronize()
    dt_host = time.perf_counter() - t1
    dec.close()
    kernel_name = {1: "sampler_kernel (one slot per lane)",
                   2: f"coop_kernel (one slot per {st['group_lanes']} lanes drawing speculatively)"}[st["kernel"]]
    kernel_name += (f", {st['wg_per_cu']} workgroups of 256 lanes per CU, chain state "
                    f"{'and tables ' if st['placement'] & 2 else ''}in LDS, 5-entry rows")

    value = units / dt
    avg_kernel_s = sum(kernel_ms) / len(kernel_ms) / 1e3
    units_per_launch = units / args.steps
    roofline = roofline_of(measure_peaks(), d_mean, units_per_launch, avg_kernel_s, kernel_name)
    out = {
        "metric": "coupled Gibbs updates/s + marginal RMSE per GPU-second (learned vs score weights)",
        "value": value,
        "unit": "coupled Gibbs updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64 estimator, u32 state (fp64 thresholds)",
        "data": "synthetic",
        "config": {"workload": "knill1298x97 paper-shaped: n=1298, m=97, degree 5, 3 positives, "
                               "fp=0.05, fn=0.10, q=3/1298, budget 2^28 over 65536 slots, k=131, l=1298",
                   "slots": rp.slots, "budget": rp.budget, "k": rp.k, "m": rp.m},
        "kernel_ms": avg_kernel_s * 1e3,
        "kernel_ms_median": sorted(kernel_ms)[len(kernel_ms) // 2],
        "kernel_updates_per_s": units_per_launch / avg_kernel_s,
        "single_site_updates_per_s": site_updates / dt,
        "progress_units_per_s": progress / dt,
        "rollback_units_per_run": rollback / args.steps,
        "note_units": "value counts retained replications' draws; progress units add the draws of "
                      "replications stopped once they could no longer be retained, and their replay",
        "host_outputs": {"updates_per_s": host_units / dt_host, "ms_per_step": dt_host / host_steps * 1e3,
                         "steps": host_steps, "note": "marginals, SE and histogram returned to host memory "
                                                       "(PCIe-inclusive); not the value"},
        "roofline": roofline,
    }
    if not args.no_batches:
        out["batches"] = batch_lines(3)
    if not args.no_learned:
        # the GPU test's own comparison (1024 runs per weighting, the same
        # seeds): on the 20000-clone instances a few hundred runs do not
        # settle the mean of a heavy-tailed error
        out["learned_vs_score"] = learned_line(1024, 1024)
    if not args.no_cpu_baseline:
        threads = min(16, os.cpu_count() or 1)
        out["cpu_baseline"] = cpu_baseline(inst, rp, threads)
        out["cpu_baseline_1thread"] = cpu_baseline_one_thread(inst, rp)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
