"""Long runs judged by ensembles: 16 GPU runs (Philox seeds 0-15) against
the oracle's 16 runs of the same workloads (tests/golden/ensemble_*.json,
written by make_ensembles.py from the oracle alone).  Each observable's
ensemble mean must agree within 3 sigma of the two ensembles' combined
standard error; observables that do not vary in either ensemble must agree
exactly."""
import json
import os
import sys

import numpy as np
import pytest

import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_ensembles as M  # noqa: E402

pytestmark = pytest.mark.gpu


def run_gpu(name, seed):
    from paper_2606_05893_amd import pic as G
    e = M.ENSEMBLES[name]
    p = M.params(name, seed)
    gpu = G.Pic(p, capacity=(60000, 60000, 60000), max_events=8192)
    if e["preload"]:
        n0 = 0
        for s, (pos, vel, ids) in W.preload(p, seed=100 + seed).items():
            gpu.load(s, pos, vel, ids)
            n0 += pos.shape[0]
        gpu.set_clock(0, n0)
    obs = M.new_obs()
    for k in range(e["steps"]):
        _, d = gpu.step(p["dt"])
        assert d["solve"]["converged"] == 1
        M.accumulate(obs, d, k, e["steps"])
    for s, key in ((0, "n_e"), (1, "n_n"), (2, "n_ion")):
        obs[key] = gpu.count(s)
    return obs


@pytest.mark.parametrize("name", ["c1", "c2s"])
def test_ensemble_matches_oracle(gpu_lib, name):
    with open(os.path.join(HERE, "golden", f"ensemble_{name}.json")) as f:
        ref = json.load(f)
    seeds = ref["seeds"]
    gpu = [run_gpu(name, s) for s in seeds]
    n = len(seeds)
    report = {}
    for key in ref["runs"][0]:
        o = np.array([r[key] for r in ref["runs"]], dtype=np.float64)
        g = np.array([r[key] for r in gpu], dtype=np.float64)
        so, sg = o.std(ddof=1), g.std(ddof=1)
        report[key] = (o.mean(), g.mean(), so, sg)
        if so == 0.0 and sg == 0.0:
            assert o.mean() == g.mean(), (key, o.mean(), g.mean())
        else:
            se = np.sqrt(so ** 2 / n + sg ** 2 / n)
            assert abs(g.mean() - o.mean()) <= 3.0 * se, (key, report[key])
    print(name, "oracle mean, GPU mean, oracle sd, GPU sd:")
    for k, v in report.items():
        print(f"  {k:14s} {v[0]:12.3f} {v[1]:12.3f} {v[2]:10.3f} {v[3]:10.3f}")
