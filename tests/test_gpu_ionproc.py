"""Recombination, ionisation of Cu+ into Cu2+ and charge exchange on the
GPU against the oracle, with cross sections raised so that every process
happens hundreds of times a step.

* Fixed field, several advances: the event counts exactly, all four
  species by id, positions bit for bit, velocities within 1e-12 (the
  processes call exp, log, sqrt, sin, cos); the Cu2+ made in one step are
  pushed (charge 2) in the next and reach the cathode list.
* A full step with Coulomb collisions too: the potential within 1e-6 and
  the total charge exact, Cu2+ counted twice.
* Mixed precision: counts close to the oracle's.
"""
import numpy as np
import pytest

import workloads as W
from oracle import constants as C
from oracle import pic as O
from oracle import poisson as P

pytestmark = pytest.mark.gpu

IONP = dict(enabled=True, sigma_rec_1eV=1e-17, lotz_a2=4.5e-16, I2_eV=20.29,
            cx_a=3.1622776601683795e-08, cx_b=0.0)


def grid_of(p):
    return P.Grid(p["nx"], p["ny"], p["nz"], p["dx"], p.get("bc_lo", 0),
                  p.get("bc_hi", 0), p.get("v_lo", 0.0), p.get("v_hi", 0.0))


def by_id(pos, vel, ids):
    ids = np.asarray(ids).astype(np.uint64)
    o = np.argsort(ids)
    return ids[o], np.asarray(pos)[o], np.asarray(vel)[o]


def oracle_arrays(sp):
    o = np.argsort(sp["id"])
    return (sp["id"][o], np.stack([sp[k] for k in ("x", "y", "z")], 1)[o],
            np.stack([sp[k] for k in ("vx", "vy", "vz")], 1)[o])


def make(p, cap=60000):
    from paper_2606_05893_amd import pic as G
    return G.Pic(p, capacity=(cap, cap, cap, cap), flags=G.FLAG_CELL_GROUPS)


def case(precision="fp64", seed=6):
    p = W.scaled(W.config("c2"), 16, 16, 16, n_e=8000, n_ion=8000, n_n=6000)
    p["preload"]["kT_e_eV"] = 40.0
    p["precision"] = precision
    p["seed"] = seed
    p["ion_processes"] = IONP
    p["sources"] = {}
    return p


def load(p, gpu, st, seed):
    pre = W.preload(p, seed=seed)
    for s, (pos, vel, ids) in pre.items():
        st.load(s, pos, vel, ids)
        gpu.load(s, pos, vel, ids)
    n0 = sum(v[0].shape[0] for v in pre.values())
    st.next_id = n0
    gpu.set_clock(0, n0)


def compare_all(gpu, st, p, tol, tag):
    for s in range(4):
        pos, vel, ids = (t.cpu().numpy() for t in gpu.read(s))
        ig, pg, vg = by_id(pos, vel, ids)
        io, po, vo = oracle_arrays(st.sp[s])
        assert np.array_equal(ig, io), (tag, s, ig.size, io.size)
        if io.size == 0:
            continue
        sc = np.maximum(np.abs(vo), np.sqrt(np.mean(vo ** 2)))
        assert np.all(np.abs(vg - vo) <= tol * sc), (tag, s)
        assert np.all(np.abs(pg - po) <= tol * np.maximum(np.abs(po), p["dx"])), (tag, s)


def test_ion_processes_fixed_field_fp64(gpu_lib):
    p = case()
    g = grid_of(p)
    gpu = make(p)
    st = O.State(g, seed=p["seed"])
    load(p, gpu, st, 61)
    phi = P.solve_exact(P.add_boundary_terms(np.zeros(g.shape), g), g)
    gpu.set_phi(phi)
    E = O.efield(phi, g)
    seen = {"recombinations": 0, "ionisations2": 0, "charge_exchanges": 0}
    for k in range(3):
        ab_g, dg = gpu.advance(p["dt"])
        ab_o, do = O.advance(st, p, E, p["dt"])
        print("step", k, {key: do[key] for key in seen}, "starved",
              do["f3_starved"], flush=True)
        assert dg["near_threshold"] == sum(do["near"].values())
        for key in seen:
            assert dg[key] == do[key], (k, key)
            seen[key] += do[key]
        assert dg["ion_starved"] == do["f3_starved"]
        for s in range(4):
            assert dg["counts"][s] == do["counts"][s], (k, s)
            assert dg["cathode"][s] == do["cathode"][s], (k, s)
        compare_all(gpu, st, p, 1e-12, k)
        assert ab_g["n"] == ab_o["id"].size
    for key, v in seen.items():
        assert v >= 50, (key, v)


def test_full_step_with_coulomb_and_ion_processes(gpu_lib):
    p = case(seed=8)
    p["coulomb"] = dict(enabled=True, ln_lambda=10.0)
    g = grid_of(p)
    gpu = make(p)
    st = O.State(g, seed=p["seed"])
    load(p, gpu, st, 62)
    for k in range(3):
        _, dg = gpu.step(p["dt"])
        _, do, phi_o = O.step(st, p, p["dt"])
        assert dg["total_charge_units"] == do["total_charge_units"], k
        _, phi_g, _ = gpu.read_fields()
        phi_g = phi_g.cpu().numpy()
        assert np.max(np.abs(phi_g - phi_o)) <= 1e-6 * np.max(np.abs(phi_o))
        for key in ("recombinations", "ionisations2", "charge_exchanges"):
            assert dg[key] == do[key], (k, key)
        compare_all(gpu, st, p, 1e-6, k)
    assert st.count(C.ION2) > 0


def test_ion_processes_mixed_tracks_oracle(gpu_lib):
    p = case("mixed", seed=9)
    g = grid_of(p)
    gpu = make(p)
    st = O.State(g, seed=p["seed"])
    load(p, gpu, st, 63)
    phi = P.solve_exact(P.add_boundary_terms(np.zeros(g.shape), g), g)
    gpu.set_phi(phi)
    _, dg = gpu.advance(p["dt"])
    _, do = O.advance(st, p, O.efield(phi, g), p["dt"])
    for key in ("recombinations", "ionisations2", "charge_exchanges"):
        assert abs(dg[key] - do[key]) <= max(3, 0.02 * do[key]), key
    assert abs(dg["counts"][3] - do["counts"][3]) <= max(3, 0.02 * do["counts"][3])


def crowded_load(p, gpu, st, seed, cells):
    """A thin base population plus crowded cells, each given as
    ((i, j, k), electrons, Cu+, atoms), particles well inside the cell."""
    pre = W.preload(p, seed=seed)
    rng = np.random.default_rng(seed + 1)
    sig = {C.ELECTRON: np.sqrt(40.0 * C.E_CHARGE / C.M_E),
           C.ION: np.sqrt(C.K_B * 3000.0 / C.M_CU)}
    sig[C.NEUTRAL] = sig[C.ION]
    nid = sum(v[0].shape[0] for v in pre.values())
    out = {s: list(v) for s, v in pre.items()}
    for ijk, *counts in cells:
        for s, n in zip((C.ELECTRON, C.ION, C.NEUTRAL), counts):
            if n == 0:
                continue
            pos = (np.array(ijk) + 0.3 + 0.4 * rng.random((n, 3))) * p["dx"]
            vel = rng.standard_normal((n, 3)) * sig[s]
            ids = np.arange(nid, nid + n, dtype=np.uint64)
            nid += n
            out[s] = [np.concatenate([out[s][0], pos]),
                      np.concatenate([out[s][1], vel]),
                      np.concatenate([out[s][2], ids])]
    for s, (pos, vel, ids) in out.items():
        st.load(s, pos, vel, ids)
        gpu.load(s, pos, vel, ids)
    st.next_id = nid
    gpu.set_clock(0, nid)


def test_crowded_cells_windows_of_atoms(gpu_lib):
    """Cells of thousands of atoms: the charge exchanges take the atoms a
    window at a time, the order restarting when the Cu+ outnumber them."""
    p = W.scaled(W.config("c2"), 16, 16, 16, n_e=2000, n_ion=2000, n_n=2000)
    p["seed"] = 12
    p["sources"] = {}
    p["ion_processes"] = dict(IONP, cx_a=3e-9)
    g = grid_of(p)
    gpu = make(p)
    st = O.State(g, seed=p["seed"])
    cells = [((3, 4, 5), 200, 1500, 3000),    # several windows of atoms
             ((10, 10, 10), 0, 1300, 1100),   # windows, then the order restarts
             ((5, 12, 2), 5, 40, 30),          # restarts within one window
             ((8, 8, 8), 0, 600, 2500)]
    crowded_load(p, gpu, st, 71, cells)
    phi = P.solve_exact(P.add_boundary_terms(np.zeros(g.shape), g), g)
    gpu.set_phi(phi)
    E = O.efield(phi, g)
    for k in range(2):
        ab_g, dg = gpu.advance(p["dt"])
        ab_o, do = O.advance(st, p, E, p["dt"])
        print("step", k, do["charge_exchanges"], do["recombinations"],
              do["ionisations2"], flush=True)
        assert dg["near_threshold"] == sum(do["near"].values())
        for key in ("recombinations", "ionisations2", "charge_exchanges"):
            assert dg[key] == do[key], (k, key)
        assert dg["ion_starved"] == do["f3_starved"]
        compare_all(gpu, st, p, 1e-12, k)
    assert do["charge_exchanges"] >= 500


def test_crowded_cell_beyond_lds_is_reported(gpu_lib):
    from paper_2606_05893_amd import pic as G
    p = W.scaled(W.config("c2"), 16, 16, 16, n_e=10, n_ion=10, n_n=10)
    p["sources"] = {}
    p["collisions"] = dict(p["collisions"], enabled=False)
    p["ion_processes"] = IONP
    g = grid_of(p)
    gpu = make(p)
    st = O.State(g, seed=p["seed"])
    crowded_load(p, gpu, st, 72, [((8, 8, 8), 1000, 1100, 10)])
    gpu.set_phi(np.zeros(g.shape))
    with pytest.raises(G.PicError) as e:
        gpu.advance(1e-18)
    assert e.value.status == -2
