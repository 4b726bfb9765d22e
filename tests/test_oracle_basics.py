"""Oracle pins: constants, Philox, Poisson (CPU only).

Each test ties the oracle to something other than itself: published
constants and test vectors, an independent Philox implementation, a dense
linear solve assembled from the stencil, closed forms and the paper's own
parallel-plate numbers.
"""
import json
import os
import subprocess
import tempfile

import numpy as np
import pytest
import scipy.constants as sc
import scipy.fft
import scipy.sparse
import scipy.sparse.linalg

from oracle import constants as C
from oracle import poisson as P
from oracle.philox import philox4x32_10, uniforms

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_constants_match_codata_2022():
    assert C.E_CHARGE == sc.e
    assert C.M_E == sc.m_e
    assert C.EPS0 == sc.epsilon_0
    assert C.K_B == sc.k
    assert C.AMU == sc.atomic_mass
    assert C.H_PLANCK == sc.h
    assert C.TWO_PI == 2 * np.pi
    assert C.E_EULER == np.e


def _kat_rows():
    rows = []
    with open(os.path.join(GOLD, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            rows.append([int(t, 16) for t in line.split()])
    return rows


def test_philox_known_answers():
    for r in _kat_rows():
        out = philox4x32_10(*r[:6])
        assert [int(v) for v in out] == r[6:]


TORCH_PHILOX_SRC = r"""
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cstdint>
int main() {
  // (seed, subsequence, offset) -> key = seed, counter = (offset, subseq).
  uint64_t seeds[4] = {0ull, 0x123456789abcdef0ull, 42ull, ~0ull};
  uint64_t subs[4] = {0ull, 7ull, 0xfedcba9876543210ull, 99ull};
  uint64_t offs[4] = {0ull, 3ull, 1ull << 40, 12345ull};
  for (int t = 0; t < 4; ++t) {
    at::philox_engine e(seeds[t], subs[t], offs[t]);
    uint32_t r0 = e(), r1 = e(), r2 = e(), r3 = e();  // one block's words
    std::printf("%llu %llu %llu %u %u %u %u\n",
                (unsigned long long)seeds[t], (unsigned long long)subs[t],
                (unsigned long long)offs[t], r0, r1, r2, r3);
  }
  return 0;
}
"""


def test_philox_matches_torch_engine():
    """Cross-check against PyTorch's header-only Philox4x32-10 engine,
    compiled here for the test only (an independent implementation)."""
    import torch.utils.cpp_extension as ce
    inc = ce.include_paths()
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "t.cpp")
        exe = os.path.join(d, "t")
        with open(src, "w") as f:
            f.write(TORCH_PHILOX_SRC)
        cmd = ["g++", "-std=c++17", "-O1", src, "-o", exe]
        for p in inc:
            cmd += ["-I", p]
        try:
            subprocess.run(cmd, check=True, capture_output=True, timeout=240)
        except (subprocess.CalledProcessError, FileNotFoundError) as e:
            pytest.skip(f"cannot compile torch Philox header: {e}")
        out = subprocess.run([exe], check=True, capture_output=True,
                             text=True).stdout
    for line in out.strip().splitlines():
        seed, sub, off, *words = (int(t) for t in line.split())
        got = philox4x32_10(off & 0xFFFFFFFF, off >> 32, sub & 0xFFFFFFFF,
                            sub >> 32, seed & 0xFFFFFFFF, seed >> 32)
        assert [int(v) for v in got] == words


def test_uniforms_range_and_moments():
    ids = np.arange(200000, dtype=np.uint64)
    ua, ub = uniforms(ids, 5, 0, 0)
    for u in (ua, ub):
        assert u.min() >= 0.0 and u.max() < 1.0
        assert abs(u.mean() - 0.5) < 4 * np.sqrt(1 / 12 / u.size)
        assert abs((u * u).mean() - 1 / 3) < 4 * np.sqrt(4 / 45 / u.size)
    assert abs(np.corrcoef(ua, ub)[0, 1]) < 4 / np.sqrt(ids.size)
    # 53 random bits: the low bit is set about half the time.
    lowbit = (ua * 2.0 ** 53).astype(np.uint64) & np.uint64(1)
    assert abs(lowbit.mean() - 0.5) < 0.01
    # Different tags, steps and seeds give different streams.
    assert not np.array_equal(ua, uniforms(ids, 5, 1, 0)[0])
    assert not np.array_equal(ua, uniforms(ids, 6, 0, 0)[0])
    assert not np.array_equal(ua, uniforms(ids, 5, 0, 1)[0])


# --------------------------------------------------------------------------
# Poisson
# --------------------------------------------------------------------------
def _dense_matrix(g):
    """Sparse matrix of the scaled 7-point operator over the unknowns,
    assembled node by node from the stencil."""
    k0, k1 = g.k_range
    planes = list(range(k0, k1 + 1))
    idx = {}
    for k in planes:
        for j in range(g.ny):
            for i in range(g.nx):
                idx[(i, j, k)] = len(idx)
    rows, cols, vals = [], [], []
    for (i, j, k), r in idx.items():
        rows.append(r)
        cols.append(r)
        vals.append(6.0)
        for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
            rows.append(r)
            cols.append(idx[((i + di) % g.nx, (j + dj) % g.ny, k)])
            vals.append(-1.0)
        for dk in (1, -1):
            kk = k + dk
            if kk < 0:
                kk = 1                      # Neumann mirror at the cathode
            if kk > g.nz:
                kk = g.nz - 1               # Neumann mirror at the anode
            if (i, j, kk) in idx:
                rows.append(r)
                cols.append(idx[(i, j, kk)])
                vals.append(-1.0)
    A = scipy.sparse.csr_matrix((vals, (rows, cols)), shape=(len(idx),) * 2)
    return A, idx


@pytest.mark.parametrize("bc", [(0, 0), (1, 0), (0, 1)])
def test_exact_solve_matches_assembled_matrix(bc):
    g = P.Grid(4, 6, 8, 1e-9, bc_lo=bc[0], bc_hi=bc[1], v_lo=3.0, v_hi=-7.0)
    rng = np.random.default_rng(1)
    b = P.add_boundary_terms(rng.standard_normal(g.shape), g)
    phi = P.solve_exact(b, g)
    A, idx = _dense_matrix(g)
    bv = np.array([b[k, j, i] for (i, j, k) in idx])
    x = scipy.sparse.linalg.spsolve(A.tocsc(), bv)
    got = np.array([phi[k, j, i] for (i, j, k) in idx])
    assert np.max(np.abs(got - x)) <= 1e-12 * np.max(np.abs(x))
    assert P.rel_residual(phi, b, g) < 1e-13
    if bc[0] == 0:
        assert np.all(phi[0] == 3.0)
    if bc[1] == 0:
        assert np.all(phi[g.nz] == -7.0)


def test_exact_solve_matches_dst_for_dirichlet():
    """Dirichlet in z: a sine transform diagonalises z as well."""
    g = P.Grid(8, 4, 16, 1e-9)
    rng = np.random.default_rng(2)
    b = P.add_boundary_terms(rng.standard_normal(g.shape), g)
    inner = b[1:g.nz]
    bh = scipy.fft.dst(np.fft.fft2(inner, axes=(1, 2)), type=1, axis=0)
    m = np.arange(1, g.nz)[:, None, None]
    p = np.arange(g.nx)[None, None, :]
    q = np.arange(g.ny)[None, :, None]
    lam = (4 * np.sin(np.pi * m / (2 * g.nz)) ** 2
           + 4 * np.sin(np.pi * p / g.nx) ** 2
           + 4 * np.sin(np.pi * q / g.ny) ** 2)
    x = np.fft.ifft2(scipy.fft.idst(bh / lam, type=1, axis=0),
                     axes=(1, 2)).real
    phi = P.solve_exact(b, g)
    assert np.max(np.abs(phi[1:g.nz] - x)) <= 1e-12 * np.max(np.abs(x))


def test_parallel_plate_paper_cases():
    """The paper's gap (1200 a, a = 3.64 A) with its three anode voltages:
    no charge gives phi = V0 z / h_gap and E_z = -F_ext at every node."""
    with open(os.path.join(GOLD, "paper_parallel_plate.json")) as f:
        gold = json.load(f)
    a = gold["lattice_a_m"]
    nz = 120
    dx = gold["gap_in_a"] * a / nz          # 3.64 nm cells
    for case in gold["cases"]:
        V0 = case["V0"]
        g = P.Grid(4, 4, nz, dx, v_lo=0.0, v_hi=V0)
        b = P.add_boundary_terms(np.zeros(g.shape), g)
        phi = P.solve_exact(b, g)
        z = np.arange(nz + 1) * dx
        assert np.allclose(phi[:, 0, 0], V0 * z / g.lz, rtol=0, atol=1e-12 * V0)
        from oracle.pic import efield
        E = efield(phi, g)
        F = case["F_ext_V_per_m"]
        assert np.allclose(E[..., 2], -F, rtol=2e-5, atol=0)
        assert np.max(np.abs(E[..., :2])) < 1e-9 * F


def test_neumann_quadratic_is_exact():
    """Uniform charge, Neumann cathode (slope g), Dirichlet anode: the
    continuum solution is a quadratic in z, which second differences and
    the mirror ghost reproduce exactly at the nodes."""
    nz, dx = 32, 1e-9
    rho0, gslope, V = 3.0e5, 2.0e8, 5.0
    g = P.Grid(4, 4, nz, dx, bc_lo=P.NEUMANN, bc_hi=P.DIRICHLET,
               v_lo=gslope, v_hi=V)
    rho = np.full(g.shape, rho0)
    b = P.rhs_from_density(rho, g)
    phi = P.solve_exact(b, g)
    z = np.arange(nz + 1) * dx
    L = nz * dx
    a2 = -rho0 / (2 * C.EPS0)
    ref = a2 * z * z + gslope * z + (V - a2 * L * L - gslope * L)
    assert np.max(np.abs(phi[:, 1, 2] - ref)) <= 1e-9 * np.max(np.abs(ref))


def test_manufactured_solution_second_order():
    """phi = sin(2 pi x/Lx) cos(2 pi y/Ly) sin(pi z/Lz) + V z/Lz; error of
    the discrete solution falls ~4x per halving of dx."""
    errs = []
    L = 64e-9
    V = 10.0
    for n in (8, 16, 32):
        dx = L / n
        g = P.Grid(n, n, n, dx, v_hi=V)
        x = np.arange(n) * dx
        z = np.arange(n + 1) * dx
        X = x[None, None, :]
        Y = x[None, :, None]
        Z = z[:, None, None]
        k2 = (2 * np.pi / L) ** 2 * 2 + (np.pi / L) ** 2
        s = np.sin(2 * np.pi * X / L) * np.cos(2 * np.pi * Y / L) \
            * np.sin(np.pi * Z / L)
        exact = s + V * Z / L
        rho = C.EPS0 * k2 * s                      # -eps0 lap(phi)
        phi = P.solve_exact(P.rhs_from_density(rho, g), g)
        errs.append(np.max(np.abs(phi - exact)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.8 < r1 < 4.2 and 3.8 < r2 < 4.2


def test_both_neumann_rejected():
    with pytest.raises(ValueError):
        P.Grid(4, 4, 4, 1e-9, bc_lo=P.NEUMANN, bc_hi=P.NEUMANN)
