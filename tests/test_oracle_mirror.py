"""The oracle's entry points in the library's call shape (oracle/mcpd_oracle.h):
every declared symbol is exported, and a run, a trace and the weights
through them equal the oracle's own functions on the same inputs."""

import ctypes as C
import os
import re

import numpy as np

from oracle import oracle as O
from paper_2608_30239_amd import instances as I

HERE = os.path.dirname(os.path.abspath(O.__file__))


class Opts(C.Structure):
    _fields_ = [("max_steps", C.c_uint64), ("refill", C.c_uint32), ("hist_bins", C.c_uint32),
                ("hist_width", C.c_uint32), ("u_hi_bits", C.c_uint32), ("instance_id", C.c_uint32),
                ("init_mode", C.c_uint32), ("nthreads", C.c_int32), ("bucket_rows", C.c_uint32),
                ("slot_nstar", C.c_void_p), ("slot_units", C.c_void_p), ("bucket_sum", C.c_void_p),
                ("bucket_sumsq", C.c_void_p), ("mismatch", C.c_void_p)]


class Stats(C.Structure):
    _fields_ = [(f, C.c_uint64) for f in O.STAT_NAMES]


def lib():
    L = O.lib()
    vp = C.c_void_p
    L.mcpd_oracle_opts_init.argtypes = [C.POINTER(Opts)]
    L.mcpd_oracle_opts_init.restype = None
    L.mcpd_oracle_create.argtypes = [C.c_int32, C.c_int32, vp, vp, vp, C.c_double, C.c_double, C.c_double,
                                     C.POINTER(vp)]
    L.mcpd_oracle_set_weights.argtypes = [vp, vp]
    L.mcpd_oracle_get_weights.argtypes = [vp, vp, vp]
    L.mcpd_oracle_run_unbiased.argtypes = [vp, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64,
                                           C.POINTER(Opts), vp, vp, vp, C.POINTER(Stats)]
    L.mcpd_oracle_trace.argtypes = [vp, C.c_uint32, C.c_uint32, C.c_uint64, C.c_uint32, C.c_uint32,
                                    C.POINTER(Opts), C.c_uint64, vp, vp, vp, vp, vp, vp, vp]
    L.mcpd_oracle_destroy.argtypes = [vp]
    L.mcpd_oracle_destroy.restype = None
    return L


def p(a):
    return a.ctypes.data_as(C.c_void_p)


def create(inst):
    rp_, pi, y = (np.ascontiguousarray(inst.row_ptr, np.int32), np.ascontiguousarray(inst.pool_idx, np.int32),
                  np.ascontiguousarray(inst.y, np.uint8))
    h = C.c_void_p()
    assert lib().mcpd_oracle_create(inst.n, inst.m, p(rp_), p(pi), p(y), inst.fp, inst.fn, inst.prior,
                                    C.byref(h)) == 0
    return h


def test_header_declares_every_exported_mirror_symbol():
    text = open(os.path.join(HERE, "mcpd_oracle.h")).read()
    names = set(re.findall(r"^\s*(?:int|void)\s+(mcpd_oracle_\w+)\s*\(", text, re.M))
    assert names == {"mcpd_oracle_opts_init", "mcpd_oracle_create", "mcpd_oracle_set_weights",
                     "mcpd_oracle_get_weights", "mcpd_oracle_run_unbiased", "mcpd_oracle_trace",
                     "mcpd_oracle_destroy"}
    L = lib()
    assert all(hasattr(L, n) for n in names)


def test_run_through_mirror_equals_oracle_run():
    inst, _ = I.tiny_plain()
    slots, k, m, seed = 300, 5, 40, 9
    budget = slots * 130
    nb = (budget // slots) // m
    ref = O.Model(inst).run(budget, slots, k, m, seed=seed, slot_records=True, buckets=nb)
    h = create(inst)
    try:
        o = Opts()
        lib().mcpd_oracle_opts_init(C.byref(o))
        ns = np.zeros(slots, np.uint32)
        su = np.zeros(slots, np.uint64)
        b1 = np.zeros((nb, inst.n), np.int64)
        b2 = np.zeros((nb, inst.n, 2), np.uint64)
        mis = np.zeros(inst.n, np.uint64)
        o.slot_nstar, o.slot_units, o.bucket_sum, o.bucket_sumsq, o.mismatch = (p(ns).value, p(su).value, p(b1).value,
                                                                               p(b2).value, p(mis).value)
        o.bucket_rows = nb
        marg, se = np.zeros(inst.n), np.zeros(inst.n)
        hist = np.zeros(64, np.uint64)
        st = Stats()
        assert lib().mcpd_oracle_run_unbiased(h, budget, slots, k, m, seed, C.byref(o), p(marg), p(se), p(hist),
                                              C.byref(st)) == 0
    finally:
        lib().mcpd_oracle_destroy(h)
    assert np.array_equal(marg, ref["marginals"]) and np.array_equal(se, ref["stderr"])
    assert np.array_equal(hist, ref["hist"]) and np.array_equal(mis, ref["mismatch"])
    assert np.array_equal(ns, ref["slot_nstar"]) and np.array_equal(su, ref["slot_sret"])
    assert np.array_equal(b1, ref["bucket1"]) and np.array_equal(b2, ref["bucket2"])
    assert {f: getattr(st, f) for f in O.STAT_NAMES} == ref["stats"]


def test_trace_and_weights_through_mirror():
    inst, _ = I.tiny_plain()
    M = O.Model(inst)
    h = create(inst)
    try:
        tr = M.trace(3, 2, max_len=500, k=4, m=30, budget=0, slots=1, seed=6)
        n, L_ = inst.n, 500
        X = np.zeros((L_ + 1, n), np.uint8)
        Y = np.zeros((L_, n), np.uint8)
        Ib = np.zeros(L_, np.int32)
        U = np.zeros(L_, np.uint64)
        numer = np.zeros(n, np.int64)
        mis = np.zeros(n, np.int64)
        out = np.zeros(3, np.uint64)
        assert lib().mcpd_oracle_trace(h, 3, 2, 6, 4, 30, None, L_, p(X), p(Y), p(Ib), p(U), p(numer), p(mis),
                                       p(out)) == 0
        Cn = int(out[0])
        assert Cn == tr["C"] and int(out[1]) == tr["tau"]
        assert np.array_equal(X[:Cn + 1], tr["X"]) and np.array_equal(Ib[:Cn], tr["I"])
        assert np.array_equal(numer, tr["numer"]) and np.array_equal(mis, tr["mismatch"])
        # weights: score weights by default, caller weights after set_weights
        w, mass = np.zeros(n), np.zeros(n, np.uint64)
        assert lib().mcpd_oracle_get_weights(h, p(w), p(mass)) == 0
        assert np.array_equal(mass, M.masses())
        wn = np.linspace(1.0, 3.0, n)
        assert lib().mcpd_oracle_set_weights(h, p(wn)) == 0
        assert lib().mcpd_oracle_get_weights(h, None, p(mass)) == 0
        assert np.array_equal(mass, O.Model(inst, weights=wn).masses())
        assert lib().mcpd_oracle_set_weights(h, None) == 0
        assert lib().mcpd_oracle_get_weights(h, None, p(mass)) == 0
        assert np.array_equal(mass, M.masses())
        bad = wn.copy()
        bad[2] = -1.0
        assert lib().mcpd_oracle_set_weights(h, p(bad)) != 0
    finally:
        lib().mcpd_oracle_destroy(h)
