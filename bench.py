"""Benchmark: coupled Gibbs updates per second of the unbiased MCPD hot path.

One step = one full fixed-budget run (mcpd_run_unbiased) of the paper-shaped
workload: 1298 clones, 97 pools, degree 5, 3 positives, fp 0.05, fn 0.10,
q = 3/1298, budget 2^28 progress units over 65536 slots (B = 4096), window
k = 131, l = 1298 (one sweep), score weights.  The instance tables are
resident in device memory before the timed region; every step runs the
sampler kernel, the integer bucket reduction and the final FP64 division.

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

# Algorithmic cost per progress unit ("Roofline"):
#   VALU issue slots of the minimal per-draw work at degree d,
#   LDS bytes of the per-pair state touched at degree d.
PHILOX_SLOTS_PER_DRAW = 50          # half a Philox4x32-10 block: 10 x (2 quarter-rate mad_u64 + 2 xor3) / 2


def valu_slots_per_draw(d: float) -> float:
    # site draw 3 + state bit read 3 + per pool 9 + threshold/decision 5 + loop 3
    return PHILOX_SLOTS_PER_DRAW + 3 + 3 + 9 * d + 5 + 3


def lds_bytes_per_draw(d: float) -> float:
    # one dword of state bits + one count dword per pool of the drawn clone
    return 4.0 * (1 + d)


MI355X = dict(cus=256, clock_hz=2.4e9, simd_per_cu=4, lanes_per_simd_clk=16, hbm_Bps=8.0e12)


def alu_peak_slots_per_s():
    c = MI355X
    return c["cus"] * c["simd_per_cu"] * c["lanes_per_simd_clk"] * c["clock_hz"]


def cpu_baseline(inst, rp, threads: int, slots: int):
    from oracle import oracle as O
    M = O.Model(inst)
    B = rp.budget // rp.slots
    t0 = time.perf_counter()
    r = M.run(B * slots, slots, rp.k, rp.m, seed=rp.seed, nthreads=threads)
    dt = time.perf_counter() - t0
    units = r["stats"]["retained_units"] + r["stats"]["discarded_units"]
    return dict(value=units / dt, unit="coupled Gibbs updates/s", cores=threads, kind="oracle",
                sample=f"{slots} of {rp.slots} slots of the same workload (B={B}), "
                       f"{units} progress units in {dt:.2f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-slots", type=int, default=16384)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    from paper_2608_30239_amd import instances as I
    from paper_2608_30239_amd import native as N

    inst, rp = I.paper_shaped()
    d_mean = float(inst.degrees().mean())
    dec = N.Decoder(inst)
    for _ in range(args.warmup):
        dec.run(rp.budget, rp.slots, rp.k, rp.m, rp.seed)
    units = 0
    kernel_ms = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        r = dec.run(rp.budget, rp.slots, rp.k, rp.m, rp.seed + i)
        units += r["stats"]["progress_units"]
        kernel_ms.append(r["stats"]["kernel_ms"])
    dt = time.perf_counter() - t0
    dec.close()

    value = units / dt
    avg_kernel_s = sum(kernel_ms) / len(kernel_ms) / 1e3
    units_per_launch = units / args.steps
    slots_alg = valu_slots_per_draw(d_mean) * units_per_launch
    achieved = slots_alg / avg_kernel_s
    peak = alu_peak_slots_per_s()
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "Tslot/s",
                "frac": achieved / peak, "traffic": None,
                "lds_achieved_TBps": lds_bytes_per_draw(d_mean) * units_per_launch / avg_kernel_s / 1e12}
    out = {
        "metric": "coupled Gibbs updates/s",
        "value": value,
        "unit": "coupled Gibbs updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64/u32 (fp64 thresholds)",
        "data": "synthetic",
        "config": {"workload": "knill1298x97 paper-shaped: n=1298, m=97, d=5, 3 positives, "
                               "fp=0.05, fn=0.10, budget 2^28, 65536 slots, k=131, l=1298",
                   "slots": rp.slots, "budget": rp.budget},
        "kernel_ms": avg_kernel_s * 1e3,
        "kernel_updates_per_s": units_per_launch / avg_kernel_s,
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        threads = min(16, os.cpu_count() or 1)
        out["cpu_baseline"] = cpu_baseline(inst, rp, threads, args.cpu_slots)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
