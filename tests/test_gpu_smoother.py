"""The fused two-sweep smoothing pass against one launch per colour and
sweep: the same red-black Gauss-Seidel arithmetic, so the potential and the
V-cycle count are identical bit for bit, on grids with ragged tiles in x and
y and with Dirichlet and Neumann z faces, in FP64 and in the mixed form."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

GRIDS = [
    dict(nx=64, ny=64, nz=128, bc_lo=0, bc_hi=0),
    dict(nx=40, ny=20, nz=36, bc_lo=1, bc_hi=0),
    dict(nx=96, ny=48, nz=62, bc_lo=0, bc_hi=1),
]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("gi", range(len(GRIDS)))
def test_fused_smoother_matches_plain(gpu_lib, gi, precision):
    from paper_2606_05893_amd import pic as G
    gd = GRIDS[gi]
    p = W.scaled(W.config("c2"), gd["nx"], gd["ny"], gd["nz"], n_e=10, n_ion=10, n_n=10)
    p.update(bc_lo=gd["bc_lo"], bc_hi=gd["bc_hi"], precision=precision)
    if gd["bc_lo"] == 1:
        p["v_lo"] = -2e8
    if gd["bc_hi"] == 1:
        p["v_hi"] = 3e8
    rng = np.random.default_rng(gi)
    rho = rng.standard_normal((gd["nz"] + 1, gd["ny"], gd["nx"])) * 1e6
    out = []
    for flags in (0, G.FLAG_PLAIN_SMOOTHER):
        # Ragged grids stop coarsening early: a well-solved coarsest level
        # keeps the cycle count small.
        gpu = G.Pic(p, capacity=(64, 64, 64), flags=flags, coarse_sweeps=1024)
        phi, info = gpu.poisson_solve(rho)
        assert info["converged"] == 1
        out.append((phi.cpu().numpy(), info["vcycles"]))
    assert out[0][1] == out[1][1]
    assert np.array_equal(out[0][0], out[1][0])


# Grids whose first coarse level takes the FFT path with unequal axes
# (64 x 16) and with lines shorter than one register DFT (8 x 4).
SPEC_GRIDS = GRIDS + [
    dict(nx=128, ny=32, nz=40, bc_lo=1, bc_hi=0),
    dict(nx=16, ny=8, nz=24, bc_lo=0, bc_hi=1),
]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("gi", range(len(SPEC_GRIDS)))
def test_spectral_coarse_level_matches_full_multigrid(gpu_lib, gi, precision):
    """The exact solve of the first small coarse level (DFT in x, y,
    tridiagonal in z per mode) against the V-cycle run down to the
    coarsest level: both reach the 1e-10 residual, the potentials agree to
    the solver tolerance, and the exact coarse level takes no more
    V-cycles."""
    from paper_2606_05893_amd import pic as G
    gd = SPEC_GRIDS[gi]
    p = W.scaled(W.config("c2"), gd["nx"], gd["ny"], gd["nz"], n_e=10, n_ion=10, n_n=10)
    p.update(bc_lo=gd["bc_lo"], bc_hi=gd["bc_hi"], precision=precision)
    # Emitters shrunk to fit the smallest grid (this test solves Poisson only).
    rmax = 0.4 * min(gd["nx"], gd["ny"]) * p["dx"]
    p["sources"] = {k: dict(v, radius=min(v["radius"], rmax)) if "radius" in v else v
                    for k, v in p["sources"].items()}
    if gd["bc_lo"] == 1:
        p["v_lo"] = -2e8
    if gd["bc_hi"] == 1:
        p["v_hi"] = 3e8
    rng = np.random.default_rng(10 + gi)
    rho = rng.standard_normal((gd["nz"] + 1, gd["ny"], gd["nx"])) * 1e6
    out = []
    for flags in (0, G.FLAG_MG_ALL_LEVELS):
        gpu = G.Pic(p, capacity=(64, 64, 64), flags=flags, coarse_sweeps=1024)
        phi, info = gpu.poisson_solve(rho)
        assert info["converged"] == 1 and info["rel_residual"] <= 1e-10
        out.append((phi.cpu().numpy(), info["vcycles"]))
    (a, va), (b, vb) = out
    print("V-cycles, exact coarse level:", va, "all levels:", vb)
    assert va <= vb
    assert np.max(np.abs(a - b)) <= 1e-8 * np.max(np.abs(b))
