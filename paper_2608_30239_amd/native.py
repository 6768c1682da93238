"""ctypes binding of the C ABI in ``include/mcpd.h`` (``libmcpd.so``).

Argument marshalling only: every step of the decoding runs in the library's
HIP kernels and its host setup.  There is no fallback: if the library is
missing or the device is unusable the calls raise.
"""

from __future__ import annotations

import ctypes as C
import os
import threading
from typing import Optional

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmcpd.so")

MCPD_OK = 0
MCPD_EINVAL = -1
MCPD_ENOMEM = -2
MCPD_EDEVICE = -3
MCPD_ECAP = -4


class McpdError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__(f"{where}: {detail} (code {code})")
        self.code = code


class RunOpts(C.Structure):
    _fields_ = [
        ("max_steps", C.c_uint64),
        ("refill", C.c_uint32),
        ("strict_cap", C.c_uint32),
        ("hist_bins", C.c_uint32),
        ("hist_width", C.c_uint32),
        ("u_hi_bits", C.c_uint32),
        ("instance_id", C.c_uint32),
        ("plan", C.c_uint32),
        ("wg_per_cu", C.c_uint32),
        ("ticket_slots", C.c_uint32),
        ("use_graph", C.c_uint32),
        ("keep_slot_records", C.c_uint32),
        ("narrow_lanes", C.c_uint32),
        ("bucket_rows", C.c_uint32),
        ("kernel", C.c_uint32),
        ("group_lanes", C.c_uint32),
        ("init_mode", C.c_uint32),
        ("cap_sweeps", C.c_uint32),
        ("first_slot", C.c_uint32),
        ("keep_mismatch", C.c_uint32),
        ("reserved0", C.c_uint32),
        ("slot_nstar", C.c_void_p),
        ("slot_units", C.c_void_p),
        ("bucket_sum", C.c_void_p),
        ("bucket_sumsq", C.c_void_p),
        ("mismatch", C.c_void_p),
    ]


STAT_FIELDS = ("progress_units", "retained_units", "single_site_updates", "reps_started",
               "reps_retained", "reps_aborted", "cap_hits", "zero_completion_slots", "tau_sum",
               "tau_max", "nstar_max", "rollback_units", "list_overflows", "lanes")


class RunStats(C.Structure):
    _fields_ = [(f, C.c_uint64) for f in STAT_FIELDS] + [
        ("placement", C.c_uint32), ("wg_per_cu", C.c_uint32), ("wg_slots", C.c_uint32),
        ("kernel", C.c_uint32), ("group_lanes", C.c_uint32), ("reserved", C.c_uint32),
        ("kernel_ms", C.c_double)]

    def as_dict(self):
        d = {f: int(getattr(self, f)) for f in STAT_FIELDS}
        d["placement"] = int(self.placement)
        d["wg_per_cu"] = int(self.wg_per_cu)
        d["wg_slots"] = int(self.wg_slots)
        d["kernel"] = int(self.kernel)
        d["group_lanes"] = int(self.group_lanes)
        d["kernel_ms"] = float(self.kernel_ms)
        return d


class TuneEntry(C.Structure):
    _fields_ = [("wg_per_cu", C.c_uint32), ("ticket_slots", C.c_uint32), ("narrow_lanes", C.c_uint32),
                ("kernel", C.c_uint32), ("group_lanes", C.c_uint32), ("per_instance", C.c_uint32),
                ("ms", C.c_double)]


# Every symbol include/mcpd.h declares.
EXPORTS = ("mcpd_run_opts_init", "mcpd_score_weights", "mcpd_prune", "mcpd_create", "mcpd_set_weights",
           "mcpd_get_weights", "mcpd_run_unbiased", "mcpd_run_unbiased_dev", "mcpd_run_unbiased_dev_noalloc",
           "mcpd_destroy", "mcpd_batch_create",
           "mcpd_batch_run", "mcpd_batch_tune", "mcpd_batch_config", "mcpd_batch_buckets",
           "mcpd_batch_slot_records", "mcpd_batch_mismatch", "mcpd_batch_destroy", "mcpd_run_batch", "mcpd_features",
           "mcpd_mlp_create", "mcpd_mlp_get_params", "mcpd_mlp_set_params", "mcpd_mlp_forward",
           "mcpd_mlp_set_training_rows", "mcpd_mlp_set_training_data", "mcpd_mlp_loss_grad",
           "mcpd_mlp_train", "mcpd_mlp_backward", "mcpd_mlp_adamw_step", "mcpd_mlp_get_state", "mcpd_mlp_set_state",
           "mcpd_set_learned_weights", "mcpd_mlp_destroy", "mcpd_probe", "mcpd_strerror",
           "mcpd_last_error")

MLP_FEATURES = 8
MLP_HIDDEN = 64
MLP_PARAMS = 4801


PROBES = ("lds_b32", "lds_b64", "lds_b128", "lds_b32_random", "valu_add", "valu_mul_lo", "valu_mul_hi",
          "valu_bitop3", "valu_mul64", "philox10")


class ProbeResult(C.Structure):
    _fields_ = [("per_cu_per_clock", C.c_double), ("per_second", C.c_double), ("clock_hz", C.c_double),
                ("ms", C.c_double), ("cus", C.c_uint32), ("reserved", C.c_uint32)]


class AdamW(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("weight_decay", C.c_float)]

_lock = threading.Lock()
_lib = None


def load(path: Optional[str] = None):
    """Load libmcpd.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        p = path or LIB_PATH
        if not os.path.exists(p):
            raise FileNotFoundError(f"{p} is missing: build it with paper_2608_30239_amd/build.py")
        L = C.CDLL(p)
        vp = C.c_void_p
        L.mcpd_run_opts_init.argtypes = [C.POINTER(RunOpts)]
        L.mcpd_run_opts_init.restype = None
        L.mcpd_score_weights.argtypes = [C.c_int32, C.c_int32, vp, vp, vp, C.c_double, C.c_double,
                                         C.c_double, vp, vp]
        L.mcpd_prune.argtypes = [C.c_int32, C.c_int32, vp, vp, vp, C.c_double, C.c_double, C.c_int32, vp]
        L.mcpd_create.argtypes = [C.c_int32, C.c_int32, vp, vp, vp, C.c_double, C.c_double,
                                  C.c_double, vp, C.POINTER(vp)]
        L.mcpd_set_weights.argtypes = [vp, vp]
        L.mcpd_get_weights.argtypes = [vp, vp, vp]
        L.mcpd_run_unbiased.argtypes = [vp, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                        C.c_uint64, C.POINTER(RunOpts), vp, vp, vp,
                                        C.POINTER(RunStats)]
        L.mcpd_run_unbiased_dev.argtypes = L.mcpd_run_unbiased.argtypes
        L.mcpd_run_unbiased_dev_noalloc.argtypes = L.mcpd_run_unbiased.argtypes
        L.mcpd_destroy.argtypes = [vp]
        L.mcpd_destroy.restype = None
        L.mcpd_batch_create.argtypes = [vp, C.c_int32, vp, vp, vp, vp, C.POINTER(RunOpts), vp, C.POINTER(vp)]
        L.mcpd_batch_run.argtypes = [vp, C.c_uint64, vp, vp, vp, vp]
        L.mcpd_batch_tune.argtypes = [vp, C.c_uint64, vp, C.c_uint32, vp]
        L.mcpd_batch_config.argtypes = [vp, vp, vp, vp, vp, vp]
        L.mcpd_batch_buckets.argtypes = [vp, C.c_int32, C.c_uint32, vp, vp]
        L.mcpd_batch_slot_records.argtypes = [vp, C.c_int32, vp, vp]
        L.mcpd_batch_mismatch.argtypes = [vp, C.c_int32, vp]
        L.mcpd_batch_destroy.argtypes = [vp]
        L.mcpd_batch_destroy.restype = None
        L.mcpd_run_batch.argtypes = [vp, C.c_int32, vp, vp, vp, vp, C.c_uint64, C.POINTER(RunOpts), vp, vp,
                                     vp, vp]
        L.mcpd_features.argtypes = [vp, vp, vp]
        L.mcpd_mlp_create.argtypes = [vp, vp, C.POINTER(vp)]
        L.mcpd_mlp_get_params.argtypes = [vp, vp, vp]
        L.mcpd_mlp_set_params.argtypes = [vp, vp]
        L.mcpd_mlp_forward.argtypes = [vp, vp, C.c_int64, vp]
        L.mcpd_mlp_set_training_rows.argtypes = [vp, vp, vp, vp, C.c_int64, vp, C.c_int32, C.c_double,
                                                 C.c_double, C.c_double]
        L.mcpd_mlp_set_training_data.argtypes = [vp, vp, vp, C.c_int32, C.c_double, C.c_double, C.c_double]
        L.mcpd_mlp_loss_grad.argtypes = [vp, vp, vp]
        L.mcpd_mlp_train.argtypes = [vp, C.c_int32, C.POINTER(AdamW), vp]
        L.mcpd_set_learned_weights.argtypes = [vp, vp, C.c_double, vp]
        L.mcpd_mlp_backward.argtypes = [vp, vp, C.c_int64, vp, vp]
        L.mcpd_mlp_adamw_step.argtypes = [vp, vp, C.POINTER(AdamW)]
        L.mcpd_mlp_get_state.argtypes = [vp, vp, vp, vp, vp, C.POINTER(C.c_int64)]
        L.mcpd_mlp_set_state.argtypes = [vp, vp, vp, vp, C.c_int64]
        L.mcpd_mlp_destroy.argtypes = [vp]
        L.mcpd_mlp_destroy.restype = None
        L.mcpd_probe.argtypes = [C.c_int, C.c_uint32, C.POINTER(ProbeResult)]
        L.mcpd_strerror.argtypes = [C.c_int]
        L.mcpd_strerror.restype = C.c_char_p
        L.mcpd_last_error.argtypes = []
        L.mcpd_last_error.restype = C.c_char_p
        _lib = L
        return L


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _check(rc: int, where: str):
    if rc != MCPD_OK:
        L = load()
        raise McpdError(rc, where, f"{L.mcpd_strerror(rc).decode()}: {L.mcpd_last_error().decode()}")


def _design(inst):
    return (np.ascontiguousarray(inst.row_ptr, np.int32), np.ascontiguousarray(inst.pool_idx, np.int32),
            np.ascontiguousarray(inst.y, np.uint8))


def mcpd_score_weights(inst):
    rp, pi, y = _design(inst)
    s = np.zeros(inst.n)
    w = np.zeros(inst.n)
    _check(load().mcpd_score_weights(inst.n, inst.m, _p(rp), _p(pi), _p(y), inst.fp, inst.fn,
                                     inst.prior, _p(s), _p(w)), "mcpd_score_weights")
    return s, w


def mcpd_prune(inst, n_active: int) -> np.ndarray:
    """Indices (ascending) of the n_active clones the naive ranking keeps."""
    rp, pi, y = _design(inst)
    out = np.zeros(max(int(n_active), 1), np.int32)
    _check(load().mcpd_prune(inst.n, inst.m, _p(rp), _p(pi), _p(y), inst.fp, inst.fn, int(n_active), _p(out)),
           "mcpd_prune")
    return out


def mcpd_create(inst, stream: Optional[int] = None):
    rp, pi, y = _design(inst)
    h = C.c_void_p()
    _check(load().mcpd_create(inst.n, inst.m, _p(rp), _p(pi), _p(y), inst.fp, inst.fn, inst.prior,
                              C.c_void_p(stream) if stream else None, C.byref(h)), "mcpd_create")
    return h


def mcpd_set_weights(h, w=None):
    w = None if w is None else np.ascontiguousarray(w, np.float64)
    _check(load().mcpd_set_weights(h, _p(w)), "mcpd_set_weights")


def mcpd_get_weights(h, n):
    w = np.zeros(n)
    mass = np.zeros(n, np.uint64)
    _check(load().mcpd_get_weights(h, _p(w), _p(mass)), "mcpd_get_weights")
    return w, mass


def run_opts(**kw) -> RunOpts:
    o = RunOpts()
    load().mcpd_run_opts_init(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def mcpd_run_unbiased(h, n, budget, slots, k, m, seed=0, slot_records=False, buckets=0, mismatch=False, **opt):
    """Returns dict(marginals, stderr, hist, stats[, slot_nstar, slot_units, bucket_sum, bucket_sumsq,
    mismatch])."""
    o = run_opts(**opt)
    out = {}
    keep = []
    if mismatch:
        mis = np.zeros(n, np.uint64)
        o.mismatch = _p(mis).value
        out.update(mismatch=mis)
        keep.append(mis)
    if slot_records:
        ns = np.zeros(slots, np.uint32)
        su = np.zeros(slots, np.uint64)
        o.slot_nstar, o.slot_units = _p(ns).value, _p(su).value
        out.update(slot_nstar=ns, slot_units=su)
        keep += [ns, su]
    if buckets:
        b1 = np.zeros((buckets, n), np.int64)
        b2 = np.zeros((buckets, n, 2), np.uint64)
        o.bucket_sum, o.bucket_sumsq, o.bucket_rows = _p(b1).value, _p(b2).value, buckets
        out.update(bucket_sum=b1, bucket_sumsq=b2)
        keep += [b1, b2]
    marg = np.zeros(n)
    se = np.zeros(n)
    hist = np.zeros(o.hist_bins, np.uint64)
    st = RunStats()
    _check(load().mcpd_run_unbiased(h, budget, slots, k, m, seed, C.byref(o), _p(marg), _p(se), _p(hist),
                                    C.byref(st)), "mcpd_run_unbiased")
    out.update(marginals=marg, stderr=se, hist=hist, stats=st.as_dict())
    return out


def mcpd_run_unbiased_dev(h, budget, slots, k, m, seed, marginals_ptr, stderr_ptr=0, hist_ptr=0, **opt):
    """Device outputs: the pointers are device addresses (ints) of n doubles,
    n doubles and hist_bins uint64 on the instance's device.  Returns the
    statistics dict."""
    o = run_opts(**opt)
    st = RunStats()
    _check(load().mcpd_run_unbiased_dev(h, budget, slots, k, m, seed, C.byref(o), C.c_void_p(marginals_ptr),
                                        C.c_void_p(stderr_ptr or None), C.c_void_p(hist_ptr or None),
                                        C.byref(st)), "mcpd_run_unbiased_dev")
    return st.as_dict()


def mcpd_run_unbiased_dev_noalloc(h, budget, slots, k, m, seed, marginals_ptr, stderr_ptr=0, hist_ptr=0, **opt):
    """mcpd_run_unbiased_dev without any allocation (the library's static
    scratch array).  Returns the statistics dict."""
    o = run_opts(**opt)
    st = RunStats()
    _check(load().mcpd_run_unbiased_dev_noalloc(h, budget, slots, k, m, seed, C.byref(o), C.c_void_p(marginals_ptr),
                                                C.c_void_p(stderr_ptr or None), C.c_void_p(hist_ptr or None),
                                                C.byref(st)), "mcpd_run_unbiased_dev_noalloc")
    return st.as_dict()


def mcpd_destroy(h):
    if h:
        load().mcpd_destroy(h)


def _ptr_array(arrays):
    return (C.c_void_p * len(arrays))(*[a.ctypes.data for a in arrays])


class Batch:
    """Many instances in one persistent launch (mcpd_batch_*).

    ``params`` holds (budget, slots, k, m) per instance.  Instance i draws its
    random numbers with g = instance_id + i."""

    def __init__(self, decoders, params, stream: Optional[int] = None, **opt):
        self.decoders = list(decoders)   # keeps the instances alive
        self.count = len(self.decoders)
        if len(params) != self.count:
            raise ValueError("one (budget, slots, k, m) per instance")
        self.budget = np.array([p[0] for p in params], np.uint64)
        self.slots = np.array([p[1] for p in params], np.uint32)
        self.k = np.array([p[2] for p in params], np.uint32)
        self.m = np.array([p[3] for p in params], np.uint32)
        self.opts = run_opts(**opt)
        insts = (C.c_void_p * self.count)(*[d.h.value for d in self.decoders])
        h = C.c_void_p()
        _check(load().mcpd_batch_create(insts, self.count, _p(self.budget), _p(self.slots), _p(self.k),
                                        _p(self.m), C.byref(self.opts),
                                        C.c_void_p(stream) if stream else None, C.byref(h)),
               "mcpd_batch_create")
        self.h = h

    def run(self, seed=0, outputs=True):
        """Returns a list of dict(marginals, stderr, hist, stats) per instance."""
        n = [d.n for d in self.decoders]
        hb = self.opts.hist_bins
        marg = [np.zeros(x) for x in n] if outputs else None
        se = [np.zeros(x) for x in n] if outputs else None
        hist = [np.zeros(hb, np.uint64) for _ in n]
        st = (RunStats * self.count)()
        _check(load().mcpd_batch_run(self.h, seed, _ptr_array(marg) if outputs else None,
                                     _ptr_array(se) if outputs else None, _ptr_array(hist), st),
               "mcpd_batch_run")
        out = []
        for i in range(self.count):
            r = dict(hist=hist[i], stats=st[i].as_dict())
            if outputs:
                r.update(marginals=marg[i], stderr=se[i])
            out.append(r)
        return out

    def tune(self, seed=0):
        cap = 64
        ent = (TuneEntry * cap)()
        cnt = C.c_uint32()
        _check(load().mcpd_batch_tune(self.h, seed, ent, cap, C.byref(cnt)), "mcpd_batch_tune")
        return [dict(wg_per_cu=int(e.wg_per_cu), ticket_slots=int(e.ticket_slots),
                     narrow_lanes=int(e.narrow_lanes), kernel=int(e.kernel),
                     group_lanes=int(e.group_lanes), per_instance=bool(e.per_instance), ms=float(e.ms))
                for e in ent[:cnt.value]]

    def config(self):
        wg, ts, lanes = C.c_uint32(), C.c_uint32(), C.c_uint32()
        place = np.zeros(self.count, np.uint32)
        wl = np.zeros(self.count, np.uint32)
        _check(load().mcpd_batch_config(self.h, C.byref(wg), C.byref(ts), C.byref(lanes), _p(place), _p(wl)),
               "mcpd_batch_config")
        return dict(wg_per_cu=wg.value, ticket_slots=ts.value, lanes=lanes.value, placement=place, wg_slots=wl)

    def buckets(self, i, rows):
        n = self.decoders[i].n
        b1 = np.zeros((rows, n), np.int64)
        b2 = np.zeros((rows, n, 2), np.uint64)
        _check(load().mcpd_batch_buckets(self.h, i, rows, _p(b1), _p(b2)), "mcpd_batch_buckets")
        return b1, b2

    def mismatch(self, i):
        """Mismatch times of instance i of the last run (n values)."""
        out = np.zeros(self.decoders[i].n, np.uint64)
        _check(load().mcpd_batch_mismatch(self.h, i, _p(out)), "mcpd_batch_mismatch")
        return out

    def slot_records(self, i):
        P = int(self.slots[i])
        ns = np.zeros(P, np.uint32)
        su = np.zeros(P, np.uint64)
        _check(load().mcpd_batch_slot_records(self.h, i, _p(ns), _p(su)), "mcpd_batch_slot_records")
        return ns, su

    def close(self):
        if getattr(self, "h", None):
            load().mcpd_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mcpd_probe(kind: str, iters: int):
    """One peak-rate probe (mcpd_probe): dict(per_cu_per_clock, per_second,
    clock_hz, ms, cus)."""
    r = ProbeResult()
    _check(load().mcpd_probe(PROBES.index(kind), int(iters), C.byref(r)), "mcpd_probe")
    return dict(per_cu_per_clock=r.per_cu_per_clock, per_second=r.per_second, clock_hz=r.clock_hz,
                ms=r.ms, cus=int(r.cus))


def mcpd_features(dec):
    """(features [n, 8] float32, base logits [n] float64)."""
    X = np.zeros((dec.n, MLP_FEATURES), np.float32)
    c = np.zeros(dec.n)
    _check(load().mcpd_features(dec.h, _p(X), _p(c)), "mcpd_features")
    return X, c


class Mlp:
    """The selection-weight network (mcpd_mlp_*): FP32 master parameters,
    BF16 working copy, training and inference on the device."""

    def __init__(self, params, stream: Optional[int] = None):
        p = np.ascontiguousarray(params, np.float32)
        if p.shape != (MLP_PARAMS,):
            raise ValueError(f"need {MLP_PARAMS} parameters")
        h = C.c_void_p()
        _check(load().mcpd_mlp_create(_p(p), C.c_void_p(stream) if stream else None, C.byref(h)),
               "mcpd_mlp_create")
        self.h = h

    def params(self):
        master = np.zeros(MLP_PARAMS, np.float32)
        bf16 = np.zeros(MLP_PARAMS, np.uint16)
        _check(load().mcpd_mlp_get_params(self.h, _p(master), _p(bf16)), "mcpd_mlp_get_params")
        return master, bf16

    def set_params(self, params):
        p = np.ascontiguousarray(params, np.float32)
        _check(load().mcpd_mlp_set_params(self.h, _p(p)), "mcpd_mlp_set_params")

    def forward(self, X):
        X = np.ascontiguousarray(X, np.float32)
        g = np.zeros(X.shape[0], np.float32)
        _check(load().mcpd_mlp_forward(self.h, _p(X), X.shape[0], _p(g)), "mcpd_mlp_forward")
        return g

    def set_training_rows(self, X, base, signal, seg_ptr, beta=1.0, gamma=0.0, eps=1e-3):
        X = np.ascontiguousarray(X, np.float32)
        base = np.ascontiguousarray(base, np.float64)
        signal = np.ascontiguousarray(signal, np.float64)
        seg = np.ascontiguousarray(seg_ptr, np.int64)
        _check(load().mcpd_mlp_set_training_rows(self.h, _p(X), _p(base), _p(signal), X.shape[0], _p(seg),
                                                 len(seg) - 1, beta, gamma, eps), "mcpd_mlp_set_training_rows")

    def set_training_data(self, decoders, signals, beta=1.0, gamma=0.0, eps=1e-3):
        ph = [np.ascontiguousarray(p, np.float64) for p in signals]
        insts = (C.c_void_p * len(decoders))(*[d.h.value for d in decoders])
        _check(load().mcpd_mlp_set_training_data(self.h, insts, _ptr_array(ph), len(decoders), beta, gamma, eps),
               "mcpd_mlp_set_training_data")

    def loss_grad(self):
        loss = C.c_double()
        grad = np.zeros(MLP_PARAMS, np.float32)
        _check(load().mcpd_mlp_loss_grad(self.h, C.byref(loss), _p(grad)), "mcpd_mlp_loss_grad")
        return loss.value, grad

    def train(self, steps, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
        hp = AdamW(lr, beta1, beta2, eps, weight_decay)
        hist = np.zeros(max(steps, 1))
        _check(load().mcpd_mlp_train(self.h, steps, C.byref(hp), _p(hist)), "mcpd_mlp_train")
        return hist[:steps]

    def backward(self, X, dg):
        """Parameter gradient of sum_r dg_r g_r (mcpd_mlp_backward)."""
        X = np.ascontiguousarray(X, np.float32)
        dg = np.ascontiguousarray(dg, np.float32)
        grad = np.zeros(MLP_PARAMS, np.float32)
        _check(load().mcpd_mlp_backward(self.h, _p(X), X.shape[0], _p(dg), _p(grad)), "mcpd_mlp_backward")
        return grad

    def adamw_step(self, grad, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
        """One AdamW step with a given gradient (mcpd_mlp_adamw_step)."""
        grad = np.ascontiguousarray(grad, np.float32)
        hp = AdamW(lr, beta1, beta2, eps, weight_decay)
        _check(load().mcpd_mlp_adamw_step(self.h, _p(grad), C.byref(hp)), "mcpd_mlp_adamw_step")

    def state(self):
        """(master FP32, BF16 bits, AdamW m, AdamW v, step)."""
        master = np.zeros(MLP_PARAMS, np.float32)
        bf16 = np.zeros(MLP_PARAMS, np.uint16)
        m = np.zeros(MLP_PARAMS, np.float32)
        v = np.zeros(MLP_PARAMS, np.float32)
        step = C.c_int64()
        _check(load().mcpd_mlp_get_state(self.h, _p(master), _p(bf16), _p(m), _p(v), C.byref(step)),
               "mcpd_mlp_get_state")
        return master, bf16, m, v, int(step.value)

    def set_state(self, master, m, v, step):
        master = np.ascontiguousarray(master, np.float32)
        m = np.ascontiguousarray(m, np.float32)
        v = np.ascontiguousarray(v, np.float32)
        _check(load().mcpd_mlp_set_state(self.h, _p(master), _p(m), _p(v), int(step)), "mcpd_mlp_set_state")

    def apply(self, dec, alpha=0.5):
        """Set dec's selection weights from the network; returns w."""
        w = np.zeros(dec.n)
        _check(load().mcpd_set_learned_weights(dec.h, self.h, alpha, _p(w)), "mcpd_set_learned_weights")
        return w

    def close(self):
        if getattr(self, "h", None):
            load().mcpd_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Decoder:
    """Owns one mcpd instance."""

    def __init__(self, inst, stream: Optional[int] = None):
        self.inst = inst
        self.n = inst.n
        self.h = mcpd_create(inst, stream)

    def set_weights(self, w=None):
        mcpd_set_weights(self.h, w)

    def weights(self):
        return mcpd_get_weights(self.h, self.n)

    def run(self, budget, slots, k, m, seed=0, **kw):
        return mcpd_run_unbiased(self.h, self.n, budget, slots, k, m, seed, **kw)

    def run_dev(self, budget, slots, k, m, seed, marginals_ptr, stderr_ptr=0, hist_ptr=0, **kw):
        """Outputs written to device memory (addresses as ints)."""
        return mcpd_run_unbiased_dev(self.h, budget, slots, k, m, seed, marginals_ptr, stderr_ptr, hist_ptr, **kw)

    def close(self):
        if getattr(self, "h", None):
            mcpd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
