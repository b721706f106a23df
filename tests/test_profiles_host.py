"""The committed counter summaries the benchmark line quotes (profiles/
consume_<workload>_pmc.json and _traffic.json) describe the kernels in the
tree: their kernel hash is that of the current sources, and each holds the
split and launch shapes the summaries name.  A kernel change without new
summaries fails here instead of leaving the benchmark line without them."""
import importlib.util
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_for_tests", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("workload", ["walk_99p_20s", "qaoa_12v_p2"])
def test_counter_summaries_match_the_kernels(workload):
    bench = _bench()
    kh = bench.kernels_hash()
    with open(os.path.join(ROOT, "profiles", f"consume_{workload}_pmc.json")) as f:
        pmc = json.load(f)
    with open(os.path.join(ROOT, "profiles", f"consume_{workload}_traffic.json")) as f:
        traffic = json.load(f)
    assert pmc["kernels_hash"] == kh and traffic["kernels_hash"] == kh
    assert pmc["runs"] and traffic["splits"]
    for key, run in pmc["runs"].items():
        split, launch = key.split("|")
        part = [int(v) for v in split.split(",")]
        shape = [int(v) for v in launch.split(",")]
        assert bench.pmc_from_profile(workload, part, shape) == run
        assert run["valu_insts"] > 0 and run["leaves"] > 0
        # every split with counters also has its HBM traffic
        assert bench.traffic_from_profile(workload, part) > 0
