"""Learned selection weights: training on the method's own outputs and the
equal-budget comparison with the paper's score weights.

Everything numerical runs in the library's kernels (sampler, features,
network, loss, AdamW); this module only sequences calls and keeps score.

Training signal.  With random-scan weights w, the variance of clone j's
estimate behaves like sigma_j^2 / w_j per unit of budget, and the method's
own standard errors give sigma_j ~ SE_j sqrt(w_j).  The allocation that
minimises sum_j sigma_j^2 / w_j is w ~ sigma.  The network learns, from
per-clone features only, a move of the score softmax towards it: the target
of an instance is t ~ exp((1 - rho) c) (v + eps)^rho with c the score
log-weights and v = sigma / max sigma measured on the uneven batch.

Comparison at equal budget (the weights change neither the budget nor the
slots): for each instance, a reference is the mean of `nref` independent
runs with the score weights (seeds 1000...); each weighting is then run
`nrep` times (seeds 0...) and scored by
    MSE = mean over runs of mean_j (theta_hat_j - ref_j)^2 - mean_j Var(ref_j)
(the reference's own variance removed) and by the mean device time per run;
efficiency = 1 / (MSE * seconds), and the gain of a weighting is its
efficiency over the score weights' efficiency.

The estimator is unbiased (Theorem 2), so its MSE is its variance, which
each run also estimates from its own slots: VAR = mean over runs of
mean_j SE_j^2.  That estimate pools every slot of every run instead of
`nrep` run-level errors, so it is far less noisy under the heavy tails of
the per-slot estimates; `var_efficiency` = 1 / (VAR * seconds) is what the
choice of the training target uses.
"""

from __future__ import annotations

import json
import os
import time
from typing import Dict

import numpy as np

from . import instances as I
from . import native as N

PKG = os.path.dirname(os.path.abspath(__file__))
TRAINED = os.path.join(PKG, "selection_mlp.npz")


def initial_params(seed=0):
    """The uniform initialisation with the output layer zeroed, so that
    training starts from the score weights (f = 0)."""
    theta = I.mlp_init(seed)
    theta[-(N.MLP_HIDDEN + 1):] = 0.0
    return theta


def uneven_outputs(seed: int = 4, runs: int = 4):
    """Decoders of the uneven batch (256 instances, 2^24 updates each) and,
    per instance, the training signal v = sigma / max sigma from `runs`
    batched launches with the score weights."""
    insts, params = I.uneven_batch(seed=seed)
    decs = [N.Decoder(x) for x in insts]
    bt = N.Batch(decs, [(p.budget, p.slots, p.k, p.m) for p in params])
    try:
        res = [bt.run(r) for r in range(runs)]
    finally:
        bt.close()
    signals = []
    for i, d in enumerate(decs):
        se2 = np.mean([r[i]["stderr"] ** 2 for r in res], axis=0)
        w, _ = d.weights()
        sig = np.sqrt(se2 * w)
        signals.append(sig / sig.max() if sig.max() > 0 else np.zeros_like(sig))
    return decs, signals, res


def train(decs, signals, rho, eps, steps=600, lr=3e-3, weight_decay=1e-4, init_seed=0):
    net = N.Mlp(initial_params(init_seed))
    net.set_training_data(decs, signals, 1.0 - rho, rho, eps)
    t0 = time.perf_counter()
    hist = net.train(steps, lr=lr, weight_decay=weight_decay)
    return net, hist, time.perf_counter() - t0


class Comparison:
    """Equal-budget runs of one instance under several weightings."""

    def __init__(self, inst, rp, nref=64, ref_seed=100000):
        self.inst, self.rp = inst, rp
        self.dec = N.Decoder(inst)
        self.dec.set_weights(None)
        runs = [self._run(ref_seed + s) for s in range(nref)]
        M = np.array([r["marginals"] for r in runs])
        self.ref = M.mean(axis=0)
        self.ref_var = float((M.var(axis=0, ddof=1) / nref).mean())
        self.nref = nref
        self.results: Dict[str, dict] = {}

    def _run(self, seed):
        rp = self.rp
        return self.dec.run(rp.budget, rp.slots, rp.k, rp.m, seed)

    def measure(self, name, set_weights, nrep):
        set_weights(self.dec)
        errs, ms, var, tau = [], [], [], []
        for s in range(nrep):
            r = self._run(s)
            errs.append(float(np.mean((r["marginals"] - self.ref) ** 2)))
            var.append(float(np.mean(r["stderr"] ** 2)))
            ms.append(r["stats"]["kernel_ms"])
            tau.append(int(r["stats"]["tau_max"]))
        self.dec.set_weights(None)
        mse = float(np.mean(errs)) - self.ref_var
        # the median run: the per-slot estimates are heavy-tailed (a pair
        # that takes very long to meet makes one run's error large), so the
        # mean over runs is decided by its largest runs; the median shows the
        # typical run next to it
        mse_med = float(np.median(errs)) - self.ref_var
        v = float(np.mean(var))
        sec = float(np.mean(ms)) / 1e3
        out = dict(mse=mse, rmse=float(np.sqrt(max(mse, 0.0))), seconds=sec,
                   efficiency=(1.0 / (mse * sec)) if mse > 0 else float("inf"),
                   mse_median=mse_med,
                   median_efficiency=(1.0 / (mse_med * sec)) if mse_med > 0 else float("inf"),
                   var=v, var_efficiency=1.0 / (v * sec), run_mse=errs, run_var=var, run_ms=ms, run_tau_max=tau)
        self.results[name] = out
        return out

    def gain(self, name, base="score", key="efficiency"):
        return self.results[name][key] / self.results[base][key]

    def gain_ci(self, name, base="score", level=0.9, resamples=2000, seed=0):
        """Bootstrap interval of the efficiency gain: the runs of each
        weighting resampled with replacement (the reference held fixed)."""
        rng = np.random.default_rng(seed)
        a = np.asarray(self.results[base]["run_mse"])
        b = np.asarray(self.results[name]["run_mse"])
        sa, sb = self.results[base]["seconds"], self.results[name]["seconds"]
        g = []
        for _ in range(resamples):
            ma = a[rng.integers(0, len(a), len(a))].mean() - self.ref_var
            mb = b[rng.integers(0, len(b), len(b))].mean() - self.ref_var
            g.append((ma * sa) / (mb * sb) if mb > 0 else float("inf"))
        lo, hi = np.percentile(g, [50 * (1 - level), 50 * (1 + level)])
        return float(lo), float(hi)

    def close(self):
        self.dec.close()


def score_weights(dec):
    dec.set_weights(None)


# The floor of the learned weights, w = (1 - FLOOR) softmax(c + f) + FLOOR / n:
# chosen by choose_floor on floor_validation_set() for the shipped network
# (the largest geometric-mean efficiency gain over the score weights, 1024
# runs per weighting and instance).  Any floor in (0, 1] keeps the weights
# fixed and positive; at 0.5, the score weights' own floor, a network whose
# output is zero reproduces the score weights.
FLOOR = 0.05
FLOOR_CANDIDATES = (0.02, 0.05, 0.1, 0.2, 0.35, 0.5, 0.65, 0.8)
TRAINING_FLOOR = 0.5   # the floor at which main() compares its targets


def learned_weights(net, alpha=FLOOR):
    return lambda dec: net.apply(dec, alpha)


def judge(dec, net, rp, frac=16, seed=1 << 20, alpha=FLOOR):
    """The score weights as judge: a pilot on 1/frac of the slots at the same
    horizon B with each weighting (slots are i.i.d., so the per-slot variance
    is the same as in the full run), then the weighting with the larger
    1 / (sum_j SE_j^2 * P_pilot * seconds) is kept.  Returns (choice, pilot
    seconds)."""
    P = max(64, rp.slots // frac)
    budget = (rp.budget // rp.slots) * P
    eff, sec = {}, 0.0
    for name in ("score", "learned"):
        if name == "score":
            dec.set_weights(None)
        else:
            net.apply(dec, alpha)
        r = dec.run(budget, P, rp.k, rp.m, seed)
        s = r["stats"]["kernel_ms"] / 1e3
        sec += s
        eff[name] = 1.0 / (float(np.mean(r["stderr"] ** 2)) * P * s)
    choice = "learned" if eff["learned"] > eff["score"] else "score"
    if choice == "score":
        dec.set_weights(None)
    else:
        net.apply(dec, alpha)
    return choice, sec


def validation_set():
    """Held-out instances for choosing the target (not used for the final
    comparison): n = 3000, 6000, 12000 drawn like the uneven batch, at
    budget 2^26, and the paper-shaped design with new outcomes."""
    out = [I.heldout_large(2000 + i, n=n, budget=1 << 26) for i, n in enumerate((3000, 6000, 12000))]
    inst = I.make_instance("knill_val", 1298, 97, 5, 3, 0.05, 0.10, prior=3 / 1298, seed=77, design_seed=1)
    k, l = I.window_for_sweeps(1, 1298)
    out.append((inst, I.RunParams(budget=1 << 26, slots=16384, k=k, m=l, seed=0)))
    return out


def evaluation_set():
    """The final comparison: the paper-shaped instance and four fresh
    20000-clone instances, at budget 2^28."""
    return [I.paper_shaped()] + [I.heldout_large(1000 + i) for i in range(4)]


def floor_validation_set():
    """Four further 20000-clone instances, drawn like the evaluation set's
    but from other seeds, for choosing the floor of the learned weights."""
    return [I.heldout_large(2010 + i) for i in range(4)]


def choose_floor(net, floors=FLOOR_CANDIDATES, nrep=1024, instances=None, log=print):
    """The floor with the largest geometric mean of the efficiency gain
    over the score weights on the floor-validation instances; returns
    (floor, {floor: [gain per instance]})."""
    gains = {a: [] for a in floors}
    for inst, rp in (instances or floor_validation_set()):
        cmp_ = Comparison(inst, rp, nref=nrep)
        cmp_.measure("score", score_weights, nrep)
        for a in floors:
            cmp_.measure(f"floor{a}", learned_weights(net, a), nrep)
            gains[a].append(cmp_.gain(f"floor{a}"))
        log(f"floor validation {inst.name}: " + ", ".join(f"{a}: {g[-1]:.2f}" for a, g in gains.items()))
        cmp_.dec.set_weights(None)
        cmp_.close()
    geo = {a: float(np.exp(np.mean(np.log(np.maximum(g, 1e-12))))) for a, g in gains.items()}
    return max(geo, key=geo.get), gains


# (rho, eps) of the target t ~ exp((1 - rho) c) (v + eps)^rho
CANDIDATES = ((0.1, 1e-3), (0.15, 1e-3), (0.2, 1e-3), (0.3, 1e-3), (0.15, 1e-2), (0.3, 1e-2))


def main(out=TRAINED, steps=600, nrep=12, log=print):
    t0 = time.perf_counter()
    decs, signals, res = uneven_outputs()
    log(f"uneven batch: {len(res)} runs of {sum(r['stats']['progress_units'] for r in res[0])} updates, "
        f"{res[0][0]['stats']['kernel_ms']:.1f} ms each")
    nets = {}
    for rho, eps in CANDIDATES:
        net, hist, sec = train(decs, signals, rho, eps, steps=steps)
        nets[(rho, eps)] = net
        log(f"target rho={rho} eps={eps}: loss {hist[0]:.4f} -> {hist[-1]:.4f} in {sec:.2f} s")
    for d in decs:
        d.close()
    gains = {c: [] for c in CANDIDATES}
    for inst, rp in validation_set():
        cmp_ = Comparison(inst, rp, nref=16)
        cmp_.measure("score", score_weights, nrep)
        for c, net in nets.items():
            cmp_.measure(str(c), learned_weights(net, TRAINING_FLOOR), nrep)
            gains[c].append(cmp_.gain(str(c), key="var_efficiency"))
        log(f"validation {inst.name}: " + ", ".join(f"{c}: {g[-1]:.2f}" for c, g in gains.items()))
        cmp_.close()
    geo = {c: float(np.exp(np.mean(np.log(np.maximum(g, 1e-12))))) for c, g in gains.items()}
    best = max(geo, key=geo.get)
    master, _ = nets[best].params()
    report = dict(target=dict(rho=best[0], eps=best[1]), steps=steps,
                  validation_var_gain_geomean={str(c): v for c, v in geo.items()},
                  validation_var_gains={str(c): g for c, g in gains.items()},
                  seconds=time.perf_counter() - t0)
    np.savez(out, params=master, report=json.dumps(report))
    for net in nets.values():
        net.close()
    log(json.dumps(report))
    return report


def evaluate(net, nref=1024, nrep=1024, instances=None, log=print, with_judge=False):
    """Learned against score weights on the evaluation set at equal budget:
    per instance the reference-based MSE (mean and median run), a bootstrap
    interval of the efficiency gain, the variance from the runs' own
    standard errors, device seconds and the runs' largest meeting times.
    Runs use fixed seeds (reference 100000..., compared runs 0...), so the
    figures are a function of the inputs and the network alone."""
    rows = []
    for inst, rp in (instances or evaluation_set()):
        cmp_ = Comparison(inst, rp, nref=nref)
        s = cmp_.measure("score", score_weights, nrep)
        l = cmp_.measure("learned", learned_weights(net), nrep)
        lo, hi = cmp_.gain_ci("learned")
        row = dict(instance=inst.name, n=inst.n, budget=rp.budget, slots=rp.slots, runs=nrep, reference_runs=nref,
                   rmse_score=s["rmse"], rmse_learned=l["rmse"],
                   var_score=s["var"], var_learned=l["var"],
                   seconds_score=s["seconds"], seconds_learned=l["seconds"],
                   gain=cmp_.gain("learned"), gain_ci90=[lo, hi],
                   var_gain=cmp_.gain("learned", key="var_efficiency"),
                   median_gain=cmp_.gain("learned", key="median_efficiency"),
                   tau_max_p50=[float(np.median(s["run_tau_max"])), float(np.median(l["run_tau_max"]))],
                   tau_max_p99=[float(np.percentile(s["run_tau_max"], 99)), float(np.percentile(l["run_tau_max"], 99))],
                   ref_var=cmp_.ref_var)
        if with_judge:
            choice, pilot_sec = judge(cmp_.dec, net, rp)
            j = cmp_.results[choice]
            # the judged weighting pays for its pilot once per instance,
            # spread over the runs it serves
            judged_eff = 1.0 / (j["mse"] * (j["seconds"] + pilot_sec / nrep)) if j["mse"] > 0 else float("inf")
            row.update(judge_choice=choice, judge_pilot_seconds=pilot_sec, judged_gain=judged_eff / s["efficiency"])
        cmp_.dec.set_weights(None)
        rows.append(row)
        log(json.dumps(row))
        cmp_.close()

    def geomean(key):
        return float(np.exp(np.mean(np.log([max(r[key], 1e-12) for r in rows]))))
    out = dict(rows=rows, gain_geomean=geomean("gain"), var_gain_geomean=geomean("var_gain"),
               median_gain_geomean=geomean("median_gain"))
    if with_judge:
        out["judged_gain_geomean"] = geomean("judged_gain")
    return out


def _state_hash(master, bf16, m, v, step):
    import hashlib
    h = hashlib.sha256()
    for a in (master, bf16, m, v):
        h.update(np.ascontiguousarray(a).tobytes())
    h.update(int(step).to_bytes(8, "little", signed=True))
    return h.hexdigest()


def save_checkpoint(net, path, **extra):
    """The network's whole optimiser state: FP32 master parameters, their
    BF16 copy, AdamW moments and step counter, with a SHA-256 over all of
    them (extra: JSON-serialisable metadata)."""
    master, bf16, m, v, step = net.state()
    np.savez(path, master=master, bf16=bf16, adam_m=m, adam_v=v, step=np.int64(step),
             sha256=_state_hash(master, bf16, m, v, step), meta=json.dumps(extra))


def load_checkpoint(path, stream=None):
    """A network restored from save_checkpoint, after checking the hash and
    that the BF16 copy it rebuilds equals the saved one."""
    with np.load(path, allow_pickle=False) as z:
        master, bf16, m, v = (z[k] for k in ("master", "bf16", "adam_m", "adam_v"))
        step = int(z["step"])
        if _state_hash(master, bf16, m, v, step) != str(z["sha256"]):
            raise ValueError(f"{path}: checkpoint hash mismatch")
    net = N.Mlp(master, stream)
    net.set_state(master, m, v, step)
    if not np.array_equal(net.state()[1], bf16):
        net.close()
        raise ValueError(f"{path}: BF16 copy differs from the one rebuilt from the master")
    return net


def load_trained(path=TRAINED):
    """(FP32 master parameters, report dict) of the shipped network."""
    with np.load(path, allow_pickle=False) as z:
        return z["params"].astype(np.float32), json.loads(str(z["report"]))


if __name__ == "__main__":
    import sys
    main(out=sys.argv[1] if len(sys.argv) > 1 else TRAINED, log=lambda m: print(m, flush=True))
