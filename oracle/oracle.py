"""ctypes binding of the plain FP64 CPU oracle (``mcpd_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and
the CPU-baseline leg of the benchmark, never by the product path.  It takes
plain numpy inputs (for instance the arrays of
``paper_2608_30239_amd.instances.Instance``) and imports nothing from the
HIP package.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mcpd_oracle.c")
LIB = os.path.join(HERE, "libmcpd_oracle.so")

# Strict IEEE evaluation: no contraction into FMA, no fast-math, no -march.
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
          "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter"]

STAT_NAMES = ("retained_units", "single_site_updates", "reps_retained", "cap_hits",
              "zero_completion_slots", "tau_sum", "tau_max", "reps_discarded",
              "discarded_units", "nstar_max")

_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (a second or two)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class Params(C.Structure):
    _fields_ = [(name, C.c_uint64) for name in (
        "budget", "slots", "k", "ell", "seed", "max_steps", "refill", "hist_bins",
        "hist_width", "u_hi_bits", "instance_id", "init_mode")]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            path = build()
            L = C.CDLL(path)
            vp = C.c_void_p
            L.mo_philox4x32_10.argtypes = [vp, vp, vp]
            L.mo_draw.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64,
                                  C.c_uint32, vp, vp]
            L.mo_log_odds_terms.argtypes = [C.c_double, C.c_double, C.c_double, vp]
            L.mo_score_weights.argtypes = [C.c_int32, C.c_int32, vp, vp, vp, C.c_double,
                                           C.c_double, C.c_double, vp, vp]
            L.mo_quantize.argtypes = [C.c_int32, vp, vp]
            L.mo_model_create.restype = vp
            L.mo_model_create.argtypes = [C.c_int32, C.c_int32, vp, vp, vp, C.c_double,
                                          C.c_double, C.c_double, vp]
            L.mo_model_free.argtypes = [vp]
            L.mo_model_masses.argtypes = [vp, vp]
            L.mo_model_alias.restype = C.c_int32
            L.mo_model_alias.argtypes = [vp, vp, vp]
            L.mo_site.restype = C.c_int32
            L.mo_site.argtypes = [vp, C.c_uint32]
            L.mo_conditional.restype = C.c_double
            L.mo_conditional.argtypes = [vp, vp, C.c_int32]
            L.mo_gibbs_step.argtypes = [vp, vp, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                        C.c_uint64, C.c_uint32, vp, vp]
            L.mo_trace.argtypes = [vp, C.POINTER(Params), C.c_uint32, C.c_uint32, C.c_uint64,
                                   vp, vp, vp, vp, vp, vp, vp]
            L.mo_run.argtypes = [vp, C.POINTER(Params), vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                 C.c_uint64, vp, C.c_int32]
            L.mo_slot.argtypes = [vp, C.POINTER(Params), C.c_uint32, vp, vp]
            _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().mo_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def draw(seed, g, p, r, t, b=32):
    s = np.zeros(1, np.uint32)
    u = np.zeros(1, np.uint64)
    lib().mo_draw(seed, g, p, r, t, b, _ptr(s), _ptr(u))
    return int(s[0]), int(u[0])


def log_odds_terms(fp, fn, q):
    out = np.zeros(3)
    lib().mo_log_odds_terms(fp, fn, q, _ptr(out))
    return out  # (logit q, a for y=1, a for y=0)


def _design(inst):
    return (np.ascontiguousarray(inst.row_ptr, np.int32), np.ascontiguousarray(inst.pool_idx, np.int32),
            np.ascontiguousarray(inst.y, np.uint8))


def score_weights(inst):
    rp, pi, y = _design(inst)
    s = np.zeros(inst.n)
    w = np.zeros(inst.n)
    rc = lib().mo_score_weights(inst.n, inst.m, _ptr(rp), _ptr(pi), _ptr(y), inst.fp, inst.fn,
                                inst.prior, _ptr(s), _ptr(w))
    if rc:
        raise ValueError(f"mo_score_weights failed ({rc})")
    return s, w


def naive_rank(inst, n_active):
    """The clones kept by pruning (Section "Knill's Method", naive ranking
    R_i; Section "Score-Weighted Update Gibbs Sampler", eta_i): the n_active
    clones of largest log R_i, ties to the lower index, returned in
    ascending order.  log R_i = sum over the clone's pools of
    log Pr{y_j|xi=1} - log Pr{y_j|xi=0}; grouped by outcome it is
    n+_i a+ + n-_i a-, and that grouping is what is evaluated (in FP64), so
    clones with the same outcome counts tie exactly."""
    _, a_pos, a_neg = log_odds_terms(inst.fp, inst.fn, 0.5)
    rp, pi, y = _design(inst)
    n_pos = np.zeros(inst.n)
    n_neg = np.zeros(inst.n)
    for i in range(inst.n):
        outs = y[pi[rp[i]:rp[i + 1]]]
        n_pos[i] = float(np.count_nonzero(outs))
        n_neg[i] = float(len(outs) - np.count_nonzero(outs))
    key = n_pos * a_pos + n_neg * a_neg
    # sort by key descending, then by index ascending
    order = sorted(range(inst.n), key=lambda i: (-key[i], i))
    return np.array(sorted(order[:n_active]), np.int32)


def quantize(w):
    w = np.ascontiguousarray(w, np.float64)
    mass = np.zeros(len(w), np.uint64)
    rc = lib().mo_quantize(len(w), _ptr(w), _ptr(mass))
    if rc:
        raise ValueError(f"mo_quantize failed ({rc})")
    return mass


class Model:
    """Oracle model of one instance (score weights unless ``weights`` given)."""

    def __init__(self, inst, weights=None):
        self.inst = inst
        rp, pi, y = _design(inst)
        self._keep = (rp, pi, y)
        w = None if weights is None else np.ascontiguousarray(weights, np.float64)
        self.h = lib().mo_model_create(inst.n, inst.m, _ptr(rp), _ptr(pi), _ptr(y), inst.fp,
                                       inst.fn, inst.prior, _ptr(w))
        if not self.h:
            raise ValueError("oracle rejected the instance")
        self.n = inst.n

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().mo_model_free(h)
            self.h = None

    def masses(self):
        out = np.zeros(self.n, np.uint64)
        lib().mo_model_masses(self.h, _ptr(out))
        return out

    def alias_table(self):
        a = lib().mo_model_alias(self.h, None, None)
        thr = np.zeros(1 << a, np.uint32)
        alias = np.zeros(1 << a, np.uint32)
        lib().mo_model_alias(self.h, _ptr(thr), _ptr(alias))
        return a, thr, alias

    def site(self, word):
        return lib().mo_site(self.h, word)

    def conditional(self, x, i):
        x = np.ascontiguousarray(x, np.uint8)
        return lib().mo_conditional(self.h, _ptr(x), i)

    def gibbs_step(self, x, seed, g, p, r, t, b=32):
        x = np.ascontiguousarray(x, np.uint8)
        out = np.zeros(self.n, np.uint8)
        site = np.zeros(1, np.int32)
        rc = lib().mo_gibbs_step(self.h, _ptr(x), seed, g, p, r, t, b, _ptr(out), _ptr(site))
        if rc:
            raise ValueError(f"mo_gibbs_step failed ({rc})")
        return out, int(site[0])

    @staticmethod
    def params(budget, slots, k, m, seed=0, max_steps=0, refill=1, hist_bins=64,
               hist_width=None, u_hi_bits=32, instance_id=0, init_mode=0, n=None):
        return Params(budget, slots, k, m, seed, max_steps, refill, hist_bins,
                      hist_width if hist_width else max(1, n or 1), u_hi_bits, instance_id, init_mode)

    def _params(self, **kw):
        kw.setdefault("n", self.n)
        return self.params(**kw)

    def trace(self, p, r, max_len=4096, **kw):
        P = self._params(**kw)
        n = self.n
        X = np.zeros((max_len + 1, n), np.uint8)
        Y = np.zeros((max_len, n), np.uint8)
        I = np.zeros(max_len, np.int32)
        U = np.zeros(max_len, np.uint64)
        numer = np.zeros(n, np.int64)
        mis = np.zeros(n, np.int64)
        out = np.zeros(3, np.uint64)
        rc = lib().mo_trace(self.h, C.byref(P), p, r, max_len, _ptr(X), _ptr(Y), _ptr(I), _ptr(U),
                            _ptr(numer), _ptr(mis), _ptr(out))
        if rc:
            raise ValueError(f"mo_trace failed ({rc})")
        Cn, tau, capped = (int(v) for v in out)
        return dict(X=X[:Cn + 1], Y=Y[:Cn], I=I[:Cn], U=U[:Cn], numer=numer, mismatch=mis, C=Cn, tau=tau,
                    capped=bool(capped))

    def run(self, budget, slots, k, m, seed=0, nthreads=0, slot_records=False, buckets=None,
            **kw):
        P = self._params(budget=budget, slots=slots, k=k, m=m, seed=seed, **kw)
        n = self.n
        marg = np.zeros(n)
        se = np.zeros(n)
        hist = np.zeros(P.hist_bins, np.uint64)
        stats = np.zeros(len(STAT_NAMES), np.uint64)
        ns = sr = sd = None
        if slot_records:
            ns = np.zeros(slots, np.uint32)
            sr = np.zeros(slots, np.uint64)
            sd = np.zeros(slots, np.uint64)
        b1 = b2 = None
        if buckets:
            b1 = np.zeros((buckets, n), np.int64)
            b2 = np.zeros((buckets, n, 2), np.uint64)
        mis = np.zeros(n, np.uint64)
        rc = lib().mo_run(self.h, C.byref(P), _ptr(marg), _ptr(se), _ptr(hist), _ptr(stats),
                          _ptr(ns), _ptr(sr), _ptr(sd), _ptr(b1), _ptr(b2), buckets or 0, _ptr(mis), nthreads)
        if rc:
            raise ValueError(f"mo_run failed ({rc})")
        res = dict(marginals=marg, stderr=se, hist=hist, mismatch=mis,
                   stats={k_: int(v) for k_, v in zip(STAT_NAMES, stats)})
        if slot_records:
            res.update(slot_nstar=ns, slot_sret=sr, slot_disc=sd)
        if buckets:
            res.update(bucket1=b1, bucket2=b2)
        return res

    def slot(self, p, budget, slots, k, m, seed=0, **kw):
        P = self._params(budget=budget, slots=slots, k=k, m=m, seed=seed, **kw)
        numer = np.zeros(self.n, np.int64)
        out = np.zeros(3, np.uint64)
        rc = lib().mo_slot(self.h, C.byref(P), p, _ptr(numer), _ptr(out))
        if rc:
            raise ValueError(f"mo_slot failed ({rc})")
        return numer, int(out[0]), int(out[1]), int(out[2])
