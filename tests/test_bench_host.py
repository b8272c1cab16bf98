"""Host-side checks of bench.py's CPU legs (no GPU needed): the oracle timing
reports what the measurement contract asks for."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_cpu_baseline_fields():
    import bench
    from paper_1610_07114_amd import workloads as W
    r = bench.cpu_baseline([W.couette()], seconds_target=0.05)
    assert set(r) == {"value", "unit", "cores", "kind", "sample"}
    assert r["unit"] == "MLUPS" and r["kind"] == "oracle" and r["value"] > 0 and r["cores"] >= 1
    assert r["sample"].startswith("couette 8x32, ")


def test_cpu_baseline_detail_one_and_all_threads():
    import bench
    import oracle as O
    full = O.num_threads()
    d = bench.cpu_baseline_detail(seconds_target=0.02)
    assert O.num_threads() == full                      # thread count restored
    assert d["nproc"] >= 1 and d["cpu_model"]
    assert d["threads"] == sorted({1, full})
    assert set(d["cases"]) == {"couette_8x32", "shock_tube_8192x4", "rayleigh_benard_512x256"}
    for row in d["cases"].values():
        for t in d["threads"]:
            assert row[f"threads_{t}"] > 0 and row[f"steps_{t}"] >= 2
