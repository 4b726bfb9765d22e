"""The C3 workload as configured: the C1 grid (32x32x64 cells of 4 nm, 0 V /
256 V, disk source of 100 electrons and 50 atoms a step) in mixed precision
with four multigrid levels, 200 steps, against the FP64 oracle's C1 run and
the FP64 GPU run from the same seed.

Both GPU runs are judged against the oracle per quantity: particle counts
at the end, particles absorbed at each face, collisions over the run, and
the kinetic and field energies at the end.  The error of each is printed
(with the first step at which any count differs) and bounded by the
quantity's statistical spread (four standard deviations of a Poisson
count) or, for energies, 5 %: over 200 steps a collision decided by a
near-threshold draw, or a particle that crosses a cell face a rounding
apart, sends the runs apart, more soon in mixed precision.
"""
import time

import numpy as np
import pytest

import workloads as W
from oracle import pic as O
from oracle import poisson as P

pytestmark = pytest.mark.gpu

STEPS = 200


def grid_of(p):
    return P.Grid(p["nx"], p["ny"], p["nz"], p["dx"], p["bc_lo"], p["bc_hi"],
                  p["v_lo"], p["v_hi"])


def gpu_run(p):
    from paper_2606_05893_amd import pic as G
    gpu = G.Pic(p, capacity=(200_000, 200_000, 200_000), max_events=1 << 16)
    gpu.set_clock(0, 0)
    out = []
    for _ in range(STEPS):
        _, d = gpu.step(p["dt"])
        out.append(d)
    return out


def totals(diags, key, s=None):
    return sum(int(d[key][s] if s is not None else d[key]) for d in diags)


def test_c3_mixed_against_fp64_oracle(gpu_lib):
    t0 = time.time()
    c1, c3 = W.config("c1"), W.config("c3")
    assert c3["precision"] == "mixed" and c3["mg_levels"] == 4
    g = grid_of(c1)
    st = O.State(g, seed=c1["seed"], w_sp=c1["w_sp"])
    ora = []
    for _ in range(STEPS):
        _, do, _ = O.step(st, c1, c1["dt"])
        ora.append(do)
    print(f"oracle C1: {STEPS} steps in {time.time() - t0:.1f} s", flush=True)
    f64 = gpu_run(c1)
    mix = gpu_run(c3)
    print(f"GPU C1 and C3 runs done at {time.time() - t0:.1f} s", flush=True)

    names = {0: "electrons", 1: "atoms", 2: "Cu+"}

    def table(run):
        """(quantity, GPU, oracle, relative error, bound) rows."""
        rows = []

        def row(name, got, ref, bound):
            rows.append((name, got, ref, abs(got - ref) / max(abs(ref), 1e-300), bound))

        for s in range(3):
            ref = ora[-1]["counts"][s]
            row(f"{names[s]} at step {STEPS}", run[-1]["counts"][s], ref,
                4.0 / np.sqrt(max(ref, 1)))
            for key, what in (("cathode", "to the cathode"), ("anode", "to the anode")):
                ref = totals(ora, key, s)
                if ref:
                    row(f"{names[s]} {what}", totals(run, key, s), ref, 4.0 / np.sqrt(ref))
        for key in ("elastic", "ionisations"):
            ref = totals(ora, key)
            row(f"{key} in {STEPS} steps", totals(run, key), ref,
                4.0 / np.sqrt(max(ref, 1)))
        for s in (0, 2):
            row(f"{names[s]} kinetic energy at step {STEPS}", run[-1]["kinetic"][s],
                ora[-1]["kinetic"][s], 0.05)
        row(f"field energy at step {STEPS}", run[-1]["field_energy"],
            ora[-1]["field_energy"], 0.05)
        return rows

    def first_difference(run):
        for k, (a, b) in enumerate(zip(run, ora)):
            if any(a["counts"][s] != b["counts"][s] for s in range(3)):
                return k + 1
        return None

    ok = True
    for label, run in (("C1 in FP64 on the GPU", f64), ("C3 (mixed) on the GPU", mix)):
        rows = table(run)
        print(f"{label} against the C1 oracle (first step with a count difference: "
              f"{first_difference(run)}):")
        for name, got, ref, err, bound in rows:
            print(f"  {name:38s} {got:14.6g} {ref:14.6g}  rel {err:9.3e}  bound {bound:9.3e}")
            ok &= err <= bound
    assert all(d["solve"]["rel_residual"] <= 1e-10 for d in mix + f64)
    assert ok
