"""C ABI checks that need no GPU: symbols, defaults, host-side setup, and
argument validation (which runs before any device call)."""

import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_2608_30239_amd import instances as I
from paper_2608_30239_amd import native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "mcpd.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*\**(mcpd_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    L = N.load()
    names = declared_functions()
    assert len(names) >= 17
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(names) == set(N.EXPORTS)


def test_struct_layouts_match_header():
    # mcpd_run_opts: u64, 20 x u32, 5 pointers; mcpd_run_stats: 14 x u64, 6 x u32, double
    assert C.sizeof(N.RunOpts) == 8 + 20 * 4 + 5 * 8
    assert C.sizeof(N.RunStats) == 14 * 8 + 6 * 4 + 8
    assert C.sizeof(N.TuneEntry) == 32
    assert C.sizeof(N.ProbeResult) == 4 * 8 + 2 * 4


def test_probe_rejects_bad_arguments_before_any_device_call():
    L = N.load()
    r = N.ProbeResult()
    assert L.mcpd_probe(-1, 10, C.byref(r)) == N.MCPD_EINVAL
    assert L.mcpd_probe(len(N.PROBES), 10, C.byref(r)) == N.MCPD_EINVAL
    assert L.mcpd_probe(0, 0, C.byref(r)) == N.MCPD_EINVAL
    assert L.mcpd_probe(0, 10, None) == N.MCPD_EINVAL


def test_run_opts_defaults():
    o = N.run_opts()
    assert (o.max_steps, o.refill, o.strict_cap, o.hist_bins, o.hist_width, o.u_hi_bits,
            o.instance_id, o.plan, o.wg_per_cu, o.ticket_slots, o.use_graph,
            o.keep_slot_records, o.narrow_lanes, o.kernel, o.group_lanes, o.init_mode, o.cap_sweeps, o.first_slot) == \
        (0, 1, 0, 64, 0, 32, 0, 0, 0, 0, 1, 0, 0, 0, 0, 0, 0, 0)


def test_strerror_names_codes():
    L = N.load()
    for code in (N.MCPD_OK, N.MCPD_EINVAL, N.MCPD_ENOMEM, N.MCPD_EDEVICE, N.MCPD_ECAP):
        assert L.mcpd_strerror(code)
    assert L.mcpd_strerror(-99) == b"unknown error"


@pytest.mark.parametrize("make", [I.tiny_plain, I.paper_shaped])
def test_host_score_weights_equal_oracle_bitwise(make):
    inst, _ = make()
    s1, w1 = N.mcpd_score_weights(inst)
    s2, w2 = O.score_weights(inst)
    assert np.array_equal(s1, s2) and np.array_equal(w1, w2)


def _bad_designs():
    inst, _ = I.tiny_plain()
    good = dict(n=inst.n, m=inst.m, rp=inst.row_ptr.copy(), pi=inst.pool_idx.copy(), y=inst.y.copy(),
                fp=inst.fp, fn=inst.fn, q=inst.prior)
    cases = []
    c = dict(good); c["pi"] = c["pi"].copy(); c["pi"][0], c["pi"][1] = c["pi"][1], c["pi"][0]
    cases.append(("unsorted row", c))
    c = dict(good); c["pi"] = c["pi"].copy(); c["pi"][2] = c["m"]
    cases.append(("pool out of range", c))
    c = dict(good); c["pi"] = c["pi"].copy(); c["pi"][1] = c["pi"][0]
    cases.append(("duplicate pool", c))
    c = dict(good); c["fp"] = 0.0
    cases.append(("fp = 0", c))
    c = dict(good); c["fn"] = 1.0
    cases.append(("fn = 1", c))
    c = dict(good); c["q"] = 1.5
    cases.append(("prior > 1", c))
    c = dict(good); c["y"] = c["y"].copy(); c["y"][0] = 2
    cases.append(("outcome 2", c))
    c = dict(good); c["rp"] = c["rp"].copy(); c["rp"][0] = 1
    cases.append(("row_ptr[0] != 0", c))
    c = dict(good); c["n"] = 0
    cases.append(("no clones", c))
    return cases


@pytest.mark.parametrize("name,c", _bad_designs())
def test_invalid_designs_rejected_before_device(name, c):
    L = N.load()
    h = C.c_void_p()
    p = lambda a: a.ctypes.data_as(C.c_void_p)
    rc = L.mcpd_create(c["n"], c["m"], p(c["rp"]), p(c["pi"]), p(c["y"]), c["fp"], c["fn"], c["q"],
                       None, C.byref(h))
    assert rc == N.MCPD_EINVAL, (name, rc)
    assert not h.value
    w = np.zeros(max(c["n"], 1))
    rc = L.mcpd_score_weights(c["n"], c["m"], p(c["rp"]), p(c["pi"]), p(c["y"]), c["fp"], c["fn"],
                              c["q"], None, p(w))
    assert rc == N.MCPD_EINVAL


def test_degree_and_pool_size_limits_rejected():
    L = N.load()
    p = lambda a: a.ctypes.data_as(C.c_void_p)
    # a clone in 13 pools exceeds the supported degree
    rp = np.array([0, 13], np.int32)
    pi = np.arange(13, dtype=np.int32)
    y = np.zeros(13, np.uint8)
    h = C.c_void_p()
    assert L.mcpd_create(1, 13, p(rp), p(pi), p(y), 0.1, 0.1, 0.1, None, C.byref(h)) == N.MCPD_EINVAL
    # a pool with 256 clones exceeds the 8-bit counts
    n = 256
    rp = np.arange(n + 1, dtype=np.int32)
    pi = np.zeros(n, np.int32)
    y = np.zeros(1, np.uint8)
    assert L.mcpd_create(n, 1, p(rp), p(pi), p(y), 0.1, 0.1, 0.1, None, C.byref(h)) == N.MCPD_EINVAL
