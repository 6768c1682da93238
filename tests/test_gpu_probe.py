"""The peak-rate probes behind the benchmark's roofline: every probe runs,
reports a shader clock within the part's range, and orders as the hardware
must (wider streaming LDS reads move at least as many bytes per clock as
narrower ones; random reads no more than streaming ones; a 32-bit add
issues at least as fast as any product)."""

import pytest

pytestmark = pytest.mark.gpu

N = pytest.importorskip("paper_2608_30239_amd.native")


def test_every_probe_runs_and_orders():
    res = {k: N.mcpd_probe(k, 256) for k in N.PROBES}
    for k, r in res.items():
        print(k, {x: (round(v, 4) if isinstance(v, float) else v) for x, v in r.items()}, flush=True)
        assert r["per_second"] > 0 and r["per_cu_per_clock"] > 0, k
        assert 0.3e9 < r["clock_hz"] < 4.0e9, k
        assert r["cus"] > 0
    lds = [res[k]["per_cu_per_clock"] for k in ("lds_b32", "lds_b64", "lds_b128")]
    assert lds[1] >= 0.9 * lds[0] and lds[2] >= 0.9 * lds[1]
    assert res["lds_b32_random"]["per_cu_per_clock"] <= 1.1 * lds[0]
    add = res["valu_add"]["per_cu_per_clock"]
    for k in ("valu_mul_lo", "valu_mul_hi", "valu_mul64"):
        assert res[k]["per_cu_per_clock"] <= 1.1 * add, k
    # a 64-lane wavefront issues at most 64 lane operations per clock per SIMD
    assert add <= 4 * 64 * 1.1
