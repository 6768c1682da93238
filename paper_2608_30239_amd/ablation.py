"""The paper's ablations, run on synthetic designs shaped like its own
(Section "Experimental Setup"; Section "Results": "Slot refill ablation",
"Meeting time"; supplementary "Details of the Experimental Setup": the cap
audit).

Every run follows the paper's recipe: n_a retained clones (pruning by the
naive ranking), an estimator of s sweeps (k = b_s + 1, l = s n_a,
b_s = round(0.1 s n_a)), a per-slot horizon of 20 sweeps, a meeting cap of
20 sweeps, 1,000,000 logical slots, 10 executions (seeds) per cell.

* Refill ablation: the all-clone MAE against a reference, refill on and off,
  at s in {1, 3, 5, 10, 20}.
* Meeting time: per execution the largest meeting time (in sweeps) of any
  retained pair that met; its mean over the executions of every estimator
  length (refill on), for coupled random update (uniform weights) and
  coupled score-weighted update.
* Cap audit: pairs stopped by the cap over pairs started, per method and
  design, over all estimator lengths.

The reference is the mean of independent 20-sweep runs with the score
weights (the paper uses long systematic-scan chains, a comparison system not
built here); its own standard error is reported next to each MAE.

All sampling runs in the library's kernels; this module only sequences runs
and keeps score.
"""

from __future__ import annotations

import json
import sys
import time

import numpy as np

from . import instances as I
from . import native as N

SWEEPS = (1, 3, 5, 10, 20)
HORIZON = 20       # sweeps per slot
CAP = 20           # meeting cap in sweeps


def designs():
    """(label, instance) of every design, pruned as in the paper."""
    out = []
    for fn, fp in I.KNILL3_NOISE:
        full = I.knill_degree3(fn=fn, fp=fp)
        out.append((f"knill3 fn={fn} fp={fp}", I.restrict(full, N.mcpd_prune(full, 333))))
    for which in (320, 961):
        full, keep = I.tapestry_shaped(which)
        inst = I.restrict(full, N.mcpd_prune(full, keep)) if keep < full.n else full
        out.append((f"tapestry{which}-shaped", inst))
    return out


def run(dec, n_a, s, slots, seed, refill=1):
    k, l = I.window_for_sweeps(s, n_a)
    return dec.run(HORIZON * n_a * slots, slots, k, l, seed, max_steps=CAP * n_a, refill=refill)


def study(inst, slots=1_000_000, seeds=10, ref_runs=32, log=print):
    """All three ablations on one design; returns a dict of results."""
    n_a = inst.n
    dec = N.Decoder(inst)
    try:
        dec.set_weights(None)
        ref_m = np.array([run(dec, n_a, HORIZON, slots, 10_000 + r)["marginals"] for r in range(ref_runs)])
        ref = ref_m.mean(axis=0)
        ref_se = float(np.mean(ref_m.std(axis=0, ddof=1) / np.sqrt(ref_runs)))
        log(f"  reference: {ref_runs} runs, mean per-clone SE {ref_se:.3g}")
        out = dict(n_a=n_a, slots=slots, seeds=seeds, ref_runs=ref_runs, ref_se=ref_se, mae={},
                   meeting={}, cap={})
        audit = {}
        for method in ("score", "uniform"):
            dec.set_weights(None if method == "score" else np.ones(n_a))
            started = capped = 0
            maxima = []
            for s in SWEEPS:
                for refill in ((1, 0) if method == "score" else (1,)):
                    maes = []
                    for seed in range(seeds):
                        r = run(dec, n_a, s, slots, seed, refill)
                        st = r["stats"]
                        maes.append(float(np.mean(np.abs(r["marginals"] - ref))))
                        if refill:
                            started += st["reps_started"]
                            capped += st["cap_hits"]
                            maxima.append(st["tau_max"] / n_a)
                    if method == "score":
                        out["mae"][f"s={s} refill={refill}"] = dict(
                            mean=float(np.mean(maes)), se=float(np.std(maes, ddof=1) / np.sqrt(seeds)))
                log(f"  {method} s={s} done")
            out["meeting"][method] = dict(mean_max_sweeps=float(np.mean(maxima)),
                                          se=float(np.std(maxima, ddof=1) / np.sqrt(len(maxima))))
            audit[method] = dict(pairs=int(started), capped=int(capped),
                                 rate_percent=100.0 * capped / max(started, 1))
        out["cap"] = audit
        m1, m0 = out["mae"]["s=1 refill=1"]["mean"], out["mae"]["s=1 refill=0"]["mean"]
        out["refill_mae_reduction_s1_percent"] = 100.0 * (1.0 - m1 / m0)
        return out
    finally:
        dec.close()


def main(path=None, slots=1_000_000, seeds=10, ref_runs=32, log=print):
    t0 = time.perf_counter()
    report = {}
    for label, inst in designs():
        log(f"{label}: n_a = {inst.n}")
        report[label] = study(inst, slots, seeds, ref_runs, log)
        log(json.dumps({label: report[label]}))
    report["seconds"] = time.perf_counter() - t0
    if path:
        with open(path, "w") as f:
            json.dump(report, f, indent=1)
    return report


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else None, log=lambda m: print(m, flush=True))
