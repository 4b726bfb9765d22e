"""Parity at full size for the nanoparticle absorber and the Debye-length
check, on the 128x128x512-cell workload with its preload of 10 M electrons
+ 10 M Cu+ + 5 M Cu, in the launch configuration the benchmark times.

One advance in a fixed field with a 20 nm electron-absorbing nanoparticle
in the gap: the oracle pushes every preloaded electron in the same field
(the emitted ones start at the cathode, far below the ball), and the GPU
must absorb exactly the electrons whose path touches the ball, with the
same heat tally.  On the state the advance leaves, the Debye check over all
8.4 M blocks of one cell and over the blocks of 8^3 cells must give the
oracle's Debye length in every block to 1e-9 and its counts."""
import numpy as np
import pytest

import workloads as W
from oracle import constants as C
from oracle import pic as O
from oracle import poisson as P

pytestmark = pytest.mark.gpu


def test_full_size_absorber_and_debye_check(gpu_lib):
    from paper_2606_05893_amd import pic as G
    p = W.config("c2")
    p["sources"] = dict(p["sources"])
    sph = dict(cx=p["nx"] * p["dx"] / 2, cy=p["ny"] * p["dx"] / 2, cz=200e-9,
               radius=20e-9, n=0, T_K=3500.0, absorb=True, alpha_eh=0.5)
    p["sources"]["sphere"] = sph
    g = P.Grid(p["nx"], p["ny"], p["nz"], p["dx"], p["bc_lo"], p["bc_hi"],
               p["v_lo"], p["v_hi"])
    phi = P.solve_exact(P.add_boundary_terms(np.zeros(g.shape), g), g)
    E = O.efield(phi, g)
    pl = p["preload"]
    cap = (pl["n_e"] + 2_000_000, pl["n_n"] + 1_000_000, pl["n_ion"] + 2_000_000)
    gpu = G.Pic(p, capacity=cap, max_events=1 << 17, queue_capacity=1 << 10)
    pre = W.preload(p, seed=1)
    n0 = 0
    for s, (pos, vel, ids) in pre.items():
        gpu.load(s, pos, vel, ids)
        n0 += pos.shape[0]
    gpu.set_clock(0, n0)
    gpu.set_phi(phi)
    _, d = gpu.advance(p["dt"])
    # The oracle's push of every preloaded electron.
    pos, vel, ids = pre[C.ELECTRON]
    del pre
    sp = dict(x=pos[:, 0].copy(), y=pos[:, 1].copy(), z=pos[:, 2].copy(),
              vx=vel[:, 0].copy(), vy=vel[:, 1].copy(), vz=vel[:, 2].copy(),
              id=ids.astype(np.uint64))
    O.push(sp, C.ELECTRON, E, g, p["dt"], sph)
    hit = sp["np_hit"]
    v2 = (sp["vx"][hit] ** 2 + sp["vy"][hit] ** 2) + sp["vz"][hit] ** 2
    heat = sph["alpha_eh"] * float(np.sum(0.5 * C.M_E * v2))
    print("absorbed", int(hit.sum()), "GPU", d["np_absorbed"], "heat", heat,
          d["np_heat"], flush=True)
    assert int(hit.sum()) >= 100
    assert d["np_absorbed"] == int(hit.sum())
    assert abs(d["np_heat"] - heat) <= 1e-12 * heat
    st = O.State(g, w_sp=p["w_sp"])
    for s in range(3):
        pos, vel, gid = (t.cpu().numpy() for t in gpu.read(s))
        st.load(s, pos, vel, gid.astype(np.uint64))
    left = np.sort(st.sp[C.ELECTRON]["id"])
    at = np.searchsorted(left, sp["id"][hit])
    gone = (at >= left.size) | (left[np.minimum(at, left.size - 1)] != sp["id"][hit])
    assert gone.all()
    # The Debye check on the state the advance leaves.
    for block in (1, 8):
        info, lam = gpu.debye_check(block, 0.5)
        ref = O.debye_check(st, block, 0.5)
        lam = lam.cpu().numpy()
        fin = np.isfinite(ref["lambda_D"])
        assert np.array_equal(np.isfinite(lam), fin), block
        assert np.all(np.abs(lam[fin] - ref["lambda_D"][fin])
                      <= 1e-9 * ref["lambda_D"][fin]), block
        assert info["checked"] == ref["checked"], block
        ratio = p["dx"] / (3.4 * 0.5 * ref["lambda_D"][fin])
        edge = int(np.count_nonzero(np.abs(ratio - 1.0) < 1e-9))
        assert abs(info["unresolved"] - ref["unresolved"]) <= edge, block
        assert abs(info["lambda_min"] - ref["lambda_min"]) <= 1e-9 * ref["lambda_min"]
        assert abs(info["ratio_max"] - ref["ratio_max"]) <= 1e-9 * ref["ratio_max"]
        print("block", block, info, flush=True)
