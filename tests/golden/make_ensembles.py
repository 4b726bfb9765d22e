"""Writes the oracle's 16-seed ensembles that the GPU ensemble tests compare
against (ensemble_c1.json, ensemble_c2s.json).  Calls only the oracle and
the seeded input generators:

    python tests/golden/make_ensembles.py [--seeds 16]

c1: the 32x32x64-cell, dx = 4 nm, 1 GV/m gap with the disk source of 100
electrons and 50 Cu neutrals per step, Lotz ionisation and elastic
collisions, 200 steps of 5e-16 s; Philox seed s for run s.
c2s: the 128x128x512 workload scaled to 16x16x32 cells with a preload of
3000 e + 3000 Cu+ + 2000 Cu (preload seed 100 + s), Fowler-Nordheim disk
and neutral source, 60 steps of 2e-16 s; Philox seed s.
Per run the observables of ensemble_observables() are stored.
"""
import argparse
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import pic as O  # noqa: E402
from oracle import poisson as P  # noqa: E402

ENSEMBLES = {
    "c1": dict(steps=200, preload=False),
    "c2s": dict(steps=60, preload=True),
}


def params(name, seed):
    if name == "c1":
        p = W.config("c1")
    else:
        p = W.scaled(W.config("c2"), 16, 16, 32, n_e=3000, n_ion=3000, n_n=2000)
    p = dict(p)
    p["seed"] = seed
    return p


def accumulate(obs, d, k, steps):
    """Fold one step's diagnostics into the run's observables."""
    obs["anode_e"] += d["anode"][0]
    if k >= steps // 2:
        obs["anode_e_late"] += d["anode"][0]
    obs["cathode_e"] += d["cathode"][0]
    obs["cathode_ion"] += d["cathode"][2]
    obs["ionisations"] += d["ionisations"]
    obs["elastic"] += d["elastic"]
    obs["fn_emitted"] += d["fn_emitted"]


def new_obs():
    return dict(anode_e=0, anode_e_late=0, cathode_e=0, cathode_ion=0,
                ionisations=0, elastic=0, fn_emitted=0)


def run_oracle(name, seed):
    e = ENSEMBLES[name]
    p = params(name, seed)
    g = P.Grid(p["nx"], p["ny"], p["nz"], p["dx"], p["bc_lo"], p["bc_hi"],
               p["v_lo"], p["v_hi"])
    st = O.State(g, seed=seed, w_sp=p["w_sp"])
    if e["preload"]:
        n0 = 0
        for s, (pos, vel, ids) in W.preload(p, seed=100 + seed).items():
            st.load(s, pos, vel, ids)
            n0 += pos.shape[0]
        st.next_id = n0
    obs = new_obs()
    for k in range(e["steps"]):
        _, d, _ = O.step(st, p, p["dt"])
        accumulate(obs, d, k, e["steps"])
    for s, key in ((0, "n_e"), (1, "n_n"), (2, "n_ion")):
        obs[key] = st.count(s)
    return obs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--seeds", type=int, default=16)
    ap.add_argument("--only", default=None)
    a = ap.parse_args()
    for name in ENSEMBLES:
        if a.only and name != a.only:
            continue
        runs = [run_oracle(name, s) for s in range(a.seeds)]
        out = {"ensemble": name, "steps": ENSEMBLES[name]["steps"],
               "seeds": list(range(a.seeds)), "runs": runs}
        with open(os.path.join(HERE, f"ensemble_{name}.json"), "w") as f:
            json.dump(out, f, indent=1)
        print(name, {k: sum(r[k] for r in runs) / len(runs) for k in runs[0]})


if __name__ == "__main__":
    main()
