"""Oracle pins for deposition, field gather, push, sources, emission and
collisions (CPU only).

Pins are closed forms, exact invariants, special cases, published constants
and statistical laws (3-4 sigma), chosen so that a dropped term, a wrong sign
or index, or a transposed operand in the oracle fails at least one of them
(the planted-mistake tests at the end check a few such mutations).
"""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import constants as C
from oracle import pic as O
from oracle import poisson as P

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def small_grid(nx=8, ny=8, nz=16, dx=4e-9, v_hi=64.0, **kw):
    return P.Grid(nx, ny, nz, dx, v_lo=0.0, v_hi=v_hi, **kw)


def one(state, species, pos, vel=None, ids=None):
    pos = np.atleast_2d(np.asarray(pos, dtype=np.float64))
    vel = np.zeros_like(pos) if vel is None else np.atleast_2d(vel)
    ids = np.arange(pos.shape[0], dtype=np.uint64) if ids is None else ids
    state.load(species, pos, vel, ids)


# --------------------------------------------------------------------------
# Deposition
# --------------------------------------------------------------------------
def test_deposit_node_and_cell_centre():
    g = small_grid()
    st = O.State(g)
    dx = g.dx
    one(st, C.ION, [(3 * dx, 2 * dx, 5 * dx)])
    acc = O.deposit(st)
    assert acc[5, 2, 3] == 2 ** 39 and np.count_nonzero(acc) == 1
    one(st, C.ION, [(3.5 * dx, 2.5 * dx, 5.5 * dx)])
    acc = O.deposit(st)
    nz_ = np.argwhere(acc)
    assert len(nz_) == 8 and np.all(acc[acc != 0] == 2 ** 36)
    assert set(map(tuple, nz_)) == {(k, j, i) for k in (5, 6) for j in (2, 3)
                                    for i in (3, 4)}


def test_deposit_off_centre_weights_by_axis():
    """Fractions 1/4, 1/2, 3/4 along x, y, z give distinct corner values:
    a transposed weight or index changes which node gets which."""
    g = small_grid()
    st = O.State(g)
    dx = g.dx
    one(st, C.ION, [((2 + 0.25) * dx, (3 + 0.5) * dx, (4 + 0.75) * dx)])
    acc = O.deposit(st)
    for c, wz in ((0, 2048), (1, 6144)):
        for b, wy in ((0, 4096), (1, 4096)):
            for a, wx in ((0, 6144), (1, 2048)):
                assert acc[4 + c, 3 + b, 2 + a] == wx * wy * wz


def test_deposit_periodic_seam_and_top_plane():
    g = small_grid()
    st = O.State(g)
    dx = g.dx
    z_top = np.nextafter(g.nz * dx, 0)
    while z_top * g.inv_dx >= g.nz:
        z_top = np.nextafter(z_top, 0)
    one(st, C.ELECTRON, [((g.nx - 0.5) * dx, (g.ny - 0.5) * dx, z_top)])
    acc = O.deposit(st)
    assert acc.sum() == -(2 ** 39)
    # Charge lands on x in {nx-1, 0}, y in {ny-1, 0}, z planes nz-1 / nz.
    ks, js, is_ = np.nonzero(acc)
    assert set(is_) <= {g.nx - 1, 0} and set(js) <= {g.ny - 1, 0}
    assert set(ks) <= {g.nz - 1, g.nz}


def test_deposit_total_charge_exact():
    p = W.scaled(W.config("c1"), 8, 8, 16)
    g = small_grid()
    st = O.State(g)
    pe, ve, ie = W.random_particles(5000, p, 1)
    pi, vi, ii = W.random_particles(3000, p, 2, id0=5000)
    st.load(C.ELECTRON, pe, ve, ie)
    st.load(C.ION, pi, vi, ii)
    assert O.deposit(st).sum() == 2 ** 39 * (3000 - 5000)


# --------------------------------------------------------------------------
# Field at particles and push
# --------------------------------------------------------------------------
def test_gather_reproduces_linear_field_on_weight_lattice():
    """CIC interpolation of a field linear in x, y, z is exact for positions
    on the 1/8192-cell lattice of the quantised weights."""
    g = small_grid(nx=16, ny=16, nz=16)
    rng = np.random.default_rng(3)
    n = 500
    frac = rng.integers(0, 8192, size=(n, 3)) / 8192.0
    cells = rng.integers(1, 14, size=(n, 3))
    pos = (cells + frac) * g.dx
    k, j, i = np.meshgrid(np.arange(g.nz + 1), np.arange(g.ny),
                          np.arange(g.nx), indexing="ij")
    E = np.stack([1.0 * i + 0.0 * j, 3.0 * j + 0.5 * k, -2.0 * k + 0.25 * i],
                 axis=-1).astype(np.float64)
    sp = dict(x=pos[:, 0], y=pos[:, 1], z=pos[:, 2])
    ex, ey, ez = O.gather(sp, E, g)
    gi, gj, gk = cells[:, 0] + frac[:, 0], cells[:, 1] + frac[:, 1], \
        cells[:, 2] + frac[:, 2]
    assert np.allclose(ex, gi, rtol=1e-14, atol=1e-13)
    assert np.allclose(ey, 3.0 * gj + 0.5 * gk, rtol=1e-14, atol=1e-13)
    assert np.allclose(ez, -2.0 * gk + 0.25 * gi, rtol=1e-14, atol=1e-13)


def test_single_electron_uniform_field_closed_form():
    """Leapfrog in a uniform field: x_n = x0 + n v0 dt + a dt^2 n(n+1)/2
    (discrete closed form), with the field of the paper's parallel-plate
    gap rescaled to a small box."""
    with open(os.path.join(GOLD, "paper_parallel_plate.json")) as f:
        F = json.load(f)["cases"][1]["F_ext_V_per_m"]          # 500 MV/m
    nz, dx = 64, 4e-9
    g = small_grid(nz=nz, dx=dx, v_hi=F * nz * dx)
    phi = P.solve_exact(P.add_boundary_terms(np.zeros(g.shape), g), g)
    E = O.efield(phi, g)
    dt = 1e-16
    x0 = np.array([1.3e-9, 7.7e-9, 2.1e-9])
    v0 = np.array([2.0e5, -1.0e5, 3.0e4])
    sp = dict(x=x0[:1].copy(), y=x0[1:2].copy(), z=x0[2:].copy(),
              vx=v0[:1].copy(), vy=v0[1:2].copy(), vz=v0[2:].copy(),
              id=np.zeros(1, np.uint64))
    a = (-C.E_CHARGE / C.M_E) * (-F)          # electron pulled to +z
    for n in range(1, 81):
        cath, an, _, _ = O.push(sp, C.ELECTRON, E, g, dt)
        assert not cath[0] and not an[0]
        zn = x0[2] + n * v0[2] * dt + a * dt * dt * n * (n + 1) / 2
        assert abs(sp["z"][0] - zn) <= 1e-11 * zn
        xn = (x0[0] + n * v0[0] * dt) % g.lx
        assert abs(sp["x"][0] - xn) <= 1e-12 * g.lx
        assert abs(sp["vz"][0] - (v0[2] + a * n * dt)) <= 1e-11 * abs(a * n * dt)


def test_electron_reaches_anode_with_eV():
    """Energy gained crossing the gap from rest equals e V (to O(dt))."""
    nz, dx, V = 32, 4e-9, 100.0
    g = small_grid(nz=nz, dx=dx, v_hi=V)
    phi = P.solve_exact(P.add_boundary_terms(np.zeros(g.shape), g), g)
    E = O.efield(phi, g)
    res = []
    for dt in (4e-17, 2e-17):
        sp = dict(x=np.array([1e-9]), y=np.array([1e-9]), z=np.array([0.0]),
                  vx=np.zeros(1), vy=np.zeros(1), vz=np.zeros(1),
                  id=np.zeros(1, np.uint64))
        for _ in range(100000):
            v_before = sp["vz"][0]
            _, an, _, _ = O.push(sp, C.ELECTRON, E, g, dt)
            if an[0]:
                break
        ke = 0.5 * C.M_E * sp["vz"][0] * v_before / C.E_CHARGE
        res.append(abs(ke - V))
    assert res[0] < 0.05 * V and res[1] < res[0]


def test_cathode_absorption_crossing_point():
    g = small_grid()
    st = O.State(g)
    pos = np.array([[1e-9, 2e-9, 0.5e-9]])
    vel = np.array([[1e6, -2e6, -1e7]])
    st.load(C.NEUTRAL, pos, vel, np.array([7], np.uint64))
    E = np.zeros(g.shape + (3,))
    ab, diag = O.advance(st, {"collisions": {"enabled": False}}, E, 1e-16)
    assert ab["id"].tolist() == [7] and ab["species"].tolist() == [1]
    tc = -(0.5e-9 - 1e-9) / -1e7            # time back to z = 0 (negative)
    assert np.isclose(ab["x"][0], 1e-9 + 1e6 * (1e-16 + tc), rtol=1e-12)
    assert np.isclose(ab["y"][0], 2e-9 - 2e6 * (1e-16 + tc), rtol=1e-12)
    assert st.count(C.NEUTRAL) == 0 and diag["cathode"][1] == 1


# --------------------------------------------------------------------------
# Collisions
# --------------------------------------------------------------------------
def test_lotz_cross_section_properties():
    co = O.Collisions(lotz_a=4.5e-18, ion_I_eV=7.73)
    E = np.linspace(0.0, 7.73, 50)
    assert np.all(co.sigma_ion(E) == 0.0)
    grid = np.linspace(8.0, 60.0, 200001)
    s = co.sigma_ion(grid)
    assert abs(grid[np.argmax(s)] - np.e * 7.73) < 1e-3
    assert np.isclose(s.max(), 4.5e-18 / (np.e * 7.73 ** 2), rtol=1e-9)
    big = np.array([1e4, 1e5, 1e6])
    assert np.allclose(co.sigma_ion(big) * big / np.log(big / 7.73),
                       4.5e-18 / 7.73, rtol=1e-14)
    assert np.isclose(co.sigma_ion_max, s.max(), rtol=1e-9)


def _mcc_state(n, E_eV, rng, g, seed=0):
    st = O.State(g, seed=seed)
    v = np.sqrt(2 * E_eV * C.E_CHARGE / C.M_E)
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    pos = (rng.random((n, 3)) * np.array([g.lx, g.ly, g.lz]))
    st.load(C.ELECTRON, pos, d * v, np.arange(n, dtype=np.uint64))
    return st, v


def test_null_collision_reduces_to_eq4_with_tight_majorant():
    """Elastic only and E_max equal to the electrons' energy: the null-
    collision selection is exactly the collision probability of Eq. 4."""
    g = small_grid()
    rng = np.random.default_rng(4)
    E_eV, n = 50.0, 200000
    st, v = _mcc_state(n, E_eV, rng, g)
    co = O.Collisions(sigma_el=1e-19, lotz_a=0.0, ion_model="const",
                      sigma_ion_const=0.0, E_max_eV=E_eV)
    Nc = 3
    ncount = np.full(g.nx * g.ny * g.nz, Nc, dtype=np.int64)
    dt = 1e-15
    near = {"cand": 0, "proc": 0, "fn": 0}
    diag = {}
    ion_idx, _ = O.mcc(st, co, ncount, dt, near, diag)
    dens = Nc / g.dx ** 3
    P4 = 1.0 - np.exp(-v * dens * 1e-19 * dt)            # Eq. 4
    frac = diag["elastic"] / n
    assert ion_idx.size == 0
    assert abs(frac - P4) < 4 * np.sqrt(P4 * (1 - P4) / n)
    assert diag["elastic"] <= diag["candidates"]


def test_null_collision_process_fractions():
    """General majorant: P(process) = (1 - exp(-nu* dt)) nu_p / nu*."""
    g = small_grid()
    rng = np.random.default_rng(5)
    E_eV, n = 30.0, 300000
    st, v = _mcc_state(n, E_eV, rng, g, seed=3)
    co = O.Collisions(sigma_el=1e-19, E_max_eV=400.0)
    Nc = 2
    ncount = np.full(g.nx * g.ny * g.nz, Nc, dtype=np.int64)
    dt = 2e-15
    diag = {}
    ion_idx, _ = O.mcc(st, co, ncount, dt, {"cand": 0, "proc": 0, "fn": 0},
                       diag)
    nu_star = Nc / g.dx ** 3 * co.g_max
    pstar = 1 - np.exp(-nu_star * dt)
    s_ion = co.lotz_a * np.log(E_eV / co.I) / (E_eV * co.I)
    for count, p in ((ion_idx.size, pstar * s_ion * v / co.g_max),
                     (diag["elastic"], pstar * 1e-19 * v / co.g_max),
                     (diag["candidates"], pstar)):
        assert abs(count / n - p) < 4 * np.sqrt(p * (1 - p) / n)


def test_elastic_kinematics():
    g = small_grid()
    rng = np.random.default_rng(6)
    n = 100000
    st, v = _mcc_state(n, 20.0, rng, g)
    v_old = np.stack([st.sp[0][k].copy() for k in ("vx", "vy", "vz")], 1)
    co = O.Collisions(sigma_el=1e-17, ion_model="const", sigma_ion_const=0.0,
                      E_max_eV=20.0)
    ncount = np.full(g.nx * g.ny * g.nz, 50, dtype=np.int64)
    diag = {}
    O.mcc(st, co, ncount, 1e-14, {"cand": 0, "proc": 0, "fn": 0}, diag)
    v_new = np.stack([st.sp[0][k] for k in ("vx", "vy", "vz")], 1)
    hit = np.any(v_new != v_old, axis=1)
    assert hit.sum() == diag["elastic"] and hit.sum() > 0.9 * n
    vo, vn = v_old[hit], v_new[hit]
    so, sn = np.linalg.norm(vo, axis=1), np.linalg.norm(vn, axis=1)
    cosx = np.sum(vo * vn, axis=1) / (so * sn)
    ratio = 2 * C.M_E / C.M_CU
    assert np.allclose(sn ** 2 / so ** 2, 1 - ratio * (1 - cosx), rtol=1e-12)
    d = vn / sn[:, None]
    m = d.shape[0]
    assert np.all(np.abs(d.mean(0)) < 4 * np.sqrt(1 / 3 / m))
    assert np.all(np.abs((d ** 2).mean(0) - 1 / 3) < 4 * np.sqrt(4 / 45 / m))


def _ionisation_setup(n_e, n_n, seed=0, E_eV=60.0, g=None):
    g = g or small_grid(nx=4, ny=4, nz=4)
    rng = np.random.default_rng(seed)
    st, v = _mcc_state(n_e, E_eV, rng, g, seed=seed)
    pos = rng.random((n_n, 3)) * np.array([g.lx, g.ly, g.lz])
    vel = rng.standard_normal((n_n, 3)) * 300.0
    st.load(C.NEUTRAL, pos, vel,
            np.arange(10 ** 6, 10 ** 6 + n_n, dtype=np.uint64)[::-1].copy())
    st.next_id = 2 * 10 ** 6
    return st, g


def test_ionisation_kinematics_matching_and_ids():
    st, g = _ionisation_setup(4000, 40)
    co = O.Collisions(sigma_el=0.0, ion_model="const", sigma_ion_const=1e-14,
                      E_max_eV=60.0)
    e_before = {int(i): (x, y, z, vx, vy, vz) for i, x, y, z, vx, vy, vz in
                zip(st.sp[0]["id"], st.sp[0]["x"], st.sp[0]["y"],
                    st.sp[0]["z"], st.sp[0]["vx"], st.sp[0]["vy"],
                    st.sp[0]["vz"])}
    n_before = {int(i): (x, y, z, vx, vy, vz) for i, x, y, z, vx, vy, vz in
                zip(st.sp[1]["id"], st.sp[1]["x"], st.sp[1]["y"],
                    st.sp[1]["z"], st.sp[1]["vx"], st.sp[1]["vy"],
                    st.sp[1]["vz"])}
    E = np.zeros(g.shape + (3,))
    dt = 1e-18        # positions barely move: cells stay as loaded
    ab, diag = O.advance(st, {"collisions_obj": co}, E, dt)
    ni = diag["ionisations"]
    assert ni > 0 and diag["starved"] > 0          # more events than targets
    assert ni + st.count(1) == 40 and st.count(2) == ni
    lost = diag["cathode"][0] + diag["anode"][0]
    assert st.count(0) == 4000 - lost + ni
    # Cu+ are the consumed neutrals, unchanged.
    for k, i in enumerate(st.sp[2]["id"]):
        x, y, z, vx, vy, vz = n_before[int(i)]
        assert st.sp[2]["vx"][k] == vx and st.sp[2]["id"][k] == i
        assert abs(st.sp[2]["z"][k] - (z + vz * dt)) < 1e-20
    # Secondaries: consecutive ids from next_id, in primary-id order, at the
    # primary's position; energy conservation E = Ep + Es + I.
    sec = st.sp[0]["id"] >= 2 * 10 ** 6
    sec_ids = np.sort(st.sp[0]["id"][sec])
    assert sec_ids.tolist() == list(range(2 * 10 ** 6, 2 * 10 ** 6 + ni))
    half_me = 0.5 * C.M_E / C.E_CHARGE
    ids = st.sp[0]["id"]
    pos_by_id = {int(i): k for k, i in enumerate(ids)}
    changed = [int(i) for i in ids
               if int(i) < 10 ** 6
               and st.sp[0]["vx"][pos_by_id[int(i)]] != e_before[int(i)][3]]
    assert len(changed) == ni
    changed.sort()
    for r, pid in enumerate(changed):
        kp = pos_by_id[pid]
        ks = pos_by_id[2 * 10 ** 6 + r]
        Ep = half_me * (st.sp[0]["vx"][kp] ** 2 + st.sp[0]["vy"][kp] ** 2
                        + st.sp[0]["vz"][kp] ** 2)
        Es = half_me * (st.sp[0]["vx"][ks] ** 2 + st.sp[0]["vy"][ks] ** 2
                        + st.sp[0]["vz"][ks] ** 2)
        assert abs(Ep + Es + co.I - 60.0) < 1e-9
        assert st.sp[0]["x"][ks] == st.sp[0]["x"][kp]


def test_ionisation_rank_rule_picks_lowest_ids():
    """With one neutral per cell wanted by several electrons, the electron
    with the smallest id wins it."""
    g = small_grid(nx=1, ny=1, nz=1, dx=4e-9, v_hi=0.0)
    st = O.State(g)
    st.load(C.NEUTRAL, [[1e-9, 1e-9, 1e-9], [2e-9, 2e-9, 2e-9]],
            np.zeros((2, 3)), np.array([50, 40], np.uint64))
    v = np.sqrt(2 * 60 * C.E_CHARGE / C.M_E)
    n = 64
    pos = np.tile([[2e-9, 2e-9, 2e-9]], (n, 1))
    vel = np.tile([[v, 0.0, 0.0]], (n, 1))
    st.load(C.ELECTRON, pos, vel, np.arange(100, 100 + n, dtype=np.uint64))
    st.next_id = 1000
    co = O.Collisions(sigma_el=0.0, ion_model="const", sigma_ion_const=1e-15,
                      E_max_eV=60.0)
    near, diag = {"cand": 0, "proc": 0, "fn": 0}, {}
    ncell = O.cell_index(st.sp[1], g)
    ncount = np.bincount(ncell, minlength=1)
    idx, cell = O.mcc(st, co, ncount, 1e-14, near, diag)
    events = np.sort(st.sp[0]["id"][idx])
    assert events.size >= 2
    sec, consumed, ions = O.ionise(st, co, idx, cell, ncell, diag)
    assert diag["ionisations"] == 2 and diag["starved"] == events.size - 2
    # Lowest-id electron takes the lowest-id neutral (40), next takes 50.
    assert ions["id"].tolist() == [40, 50]
    assert sec["id"].tolist() == [1000, 1001]


# --------------------------------------------------------------------------
# Sources and emission
# --------------------------------------------------------------------------
def test_disk_and_sphere_sources_moments():
    g = small_grid(nx=32, ny=32, nz=64)
    R = 10e-9
    src = dict(disk=dict(cx=g.lx / 2, cy=g.ly / 2, radius=R, n_e=60000,
                         kT_e_eV=0.5, n_n=60000, T_n_K=3000.0),
               sphere=dict(cx=g.lx / 2, cy=g.ly / 2, cz=100e-9, radius=5e-9,
                           n=60000, T_K=3500.0))
    st = O.State(g, seed=9)
    st.next_id = 17
    E = np.zeros(g.shape + (3,))
    near = {"cand": 0, "proc": 0, "fn": 0}
    new, n_fn = O.sources(st, {"sources": src}, E, 1e-16, near)
    (xe, ye, ze, vxe, vye, vze, ide), = new[0]
    (xn, yn, zn, vxn, vyn, vzn, idn), (xs, ys, zs, vxs, vys, vzs, ids_) = new[1]
    assert ide.tolist() == list(range(17, 17 + 60000))
    assert idn[0] == 17 + 60000 and ids_[0] == 17 + 120000
    assert st.next_id == 17 + 180000 and n_fn == 0
    n = 60000
    r2 = (xe - g.lx / 2) ** 2 + (ye - g.ly / 2) ** 2
    assert r2.max() <= R * R * (1 + 1e-12) and np.all(ze == 0)
    assert abs(r2.mean() - R * R / 2) < 4 * (R * R / np.sqrt(12) / np.sqrt(n))
    kT = 0.5 * C.E_CHARGE
    vm, v2 = np.sqrt(np.pi * kT / (2 * C.M_E)), 2 * kT / C.M_E
    assert np.all(vxe == 0) and np.all(vze > 0)
    assert abs(vze.mean() - vm) < 4 * np.sqrt((v2 - vm ** 2) / n)
    assert abs((vze ** 2).mean() - v2) < 4 * v2 / np.sqrt(n)
    kTn = C.K_B * 3000.0
    assert abs((vxn ** 2).mean() - kTn / C.M_CU) < 4 * np.sqrt(2 / n) * kTn / C.M_CU
    assert abs(vxn.mean()) < 4 * np.sqrt(kTn / C.M_CU / n)
    assert abs((vzn ** 2).mean() - 2 * kTn / C.M_CU) < 4 * 2 * kTn / C.M_CU / np.sqrt(n)
    c = np.array([g.lx / 2, g.ly / 2, 100e-9])
    rel = np.stack([xs, ys, zs], 1) - c
    assert np.allclose(np.linalg.norm(rel, axis=1), 5e-9, rtol=1e-12)
    nrm = rel / 5e-9
    vs = np.stack([vxs, vys, vzs], 1)
    assert np.all(np.sum(vs * nrm, 1) >= -1e-9)
    kTs = C.K_B * 3500.0
    assert abs((vs ** 2).sum(1).mean() - 3 * kTs / C.M_CU) < 4 * np.sqrt(6 / n) * kTs / C.M_CU
    assert np.all(np.abs(nrm.mean(0)) < 4 * np.sqrt(1 / 3 / n))


def test_fowler_nordheim_against_published_constants():
    with open(os.path.join(GOLD, "fn_forbes_constants.json")) as f:
        gold = json.load(f)
    a, b = gold["a_A_eV_per_V2"], gold["b_eV_m32_V_per_nm"]
    phi = 4.5
    for F_V_per_nm in (1.0, 3.0, 6.0, 10.0):
        J_ref = a / phi * F_V_per_nm ** 2 * np.exp(-b * phi ** 1.5 / F_V_per_nm)
        J = O.fn_current_density(F_V_per_nm * 1e9, phi) * 1e-18  # A/nm^2
        # Seven-digit constants: the exponent b phi^1.5/F carries ~1e-7 rel.
        assert abs(J / J_ref - 1) < 2e-6 * b * phi ** 1.5 / F_V_per_nm + 2e-6
    assert O.fn_current_density(-1e9, phi) == 0.0
    assert O.fn_current_density(0.0, phi) == 0.0


def test_fowler_nordheim_emitted_count_mean():
    """Stochastic rounding: the mean count per node is J dx^2 dt / e."""
    g = small_grid(nx=16, ny=16, nz=8, dx=2e-9)
    F = 7e9
    E = np.zeros(g.shape + (3,))
    E[0, :, :, 2] = -F
    fn = dict(cx=g.lx / 2, cy=g.ly / 2, radius=1e-6, phi_w_eV=4.5,
              kT_e_eV=0.5)
    dt = 2e-16
    J = O.fn_current_density(F, 4.5)
    mean = J * g.dx * g.dx * dt / C.E_CHARGE
    tot = 0
    steps = 200
    st = O.State(g, seed=5)
    for s in range(steps):
        st.step = s
        _, n_fn = O.sources(st, {"sources": {"fn": fn}}, E, dt,
                            {"cand": 0, "proc": 0, "fn": 0})
        tot += n_fn
    nodes = g.nx * g.ny
    exp_ = mean * nodes * steps
    fr = mean - np.floor(mean)
    var = fr * (1 - fr) * nodes * steps
    assert abs(tot - exp_) < 4 * np.sqrt(var) + 1e-9


# --------------------------------------------------------------------------
# Multi-step closed forms
# --------------------------------------------------------------------------
def test_neutral_decay_constant_cross_section():
    """Field off, x-directed 100 eV electrons, neutrals at rest, constant
    sigma_ion: N_n(t) = N_n0 exp(-n_e sigma v t), checked over 16 seeds."""
    nx, ny, nz, dx = 16, 16, 32, 4e-9
    g = P.Grid(nx, ny, nz, dx)
    vol = g.lx * g.ly * g.lz
    n_e, n_n, steps, dt, sig = 12500, 100, 200, 5e-16, 1e-20
    v = np.sqrt(2 * 100.0 * C.E_CHARGE / C.M_E)
    co = O.Collisions(sigma_el=0.0, ion_model="const", sigma_ion_const=sig,
                      E_max_eV=100.0)
    params = {"collisions_obj": co, "field_solve": 0}
    E = np.zeros(g.shape + (3,))
    left = []
    for seed in range(16):
        rng = np.random.default_rng(100 + seed)
        st = O.State(g, seed=seed)
        pos = rng.random((n_e, 3)) * np.array([g.lx, g.ly, g.lz])
        vel = np.zeros((n_e, 3))
        vel[:, 0] = v
        st.load(0, pos, vel, np.arange(n_e, dtype=np.uint64))
        posn = rng.random((n_n, 3)) * np.array([g.lx, g.ly, g.lz])
        st.load(1, posn, np.zeros((n_n, 3)),
                np.arange(n_e, n_e + n_n, dtype=np.uint64))
        st.next_id = n_e + n_n
        for _ in range(steps):
            O.advance(st, params, E, dt)
        left.append(st.count(1))
    rate = n_e / vol * sig * v * dt
    p = np.exp(-rate * steps)
    tot = 16 * n_n
    assert abs(sum(left) - tot * p) < 3 * np.sqrt(tot * p * (1 - p))


@pytest.mark.slow
def test_child_langmuir_space_charge_limited_current():
    """Cold full-plane injection at 3x the limit: the transmitted current
    settles at J_CL = (4 eps0/9) sqrt(2e/m) V^1.5 / d^2 (within 5%)."""
    nx, ny, nz, dx, V = 16, 16, 64, 4e-9, 2560.0
    g = P.Grid(nx, ny, nz, dx, v_hi=V)
    dt = 1e-16
    jcl = 4 * C.EPS0 / 9 * np.sqrt(2 * C.E_CHARGE / C.M_E) * V ** 1.5 \
        / g.lz ** 2
    per_step = jcl * g.lx * g.ly * dt / C.E_CHARGE
    n_inj = int(round(3 * per_step))
    co = O.Collisions(enabled=False)
    params = {"collisions_obj": co}
    st = O.State(g, seed=0)
    rng = np.random.default_rng(7)
    vz0 = np.sqrt(2 * 0.01 * C.E_CHARGE / C.M_E)
    arrived = []
    prof = []
    for s in range(900):
        pos = np.zeros((n_inj, 3))
        pos[:, 0] = rng.random(n_inj) * g.lx
        pos[:, 1] = rng.random(n_inj) * g.ly
        vel = np.zeros((n_inj, 3))
        vel[:, 2] = vz0
        st.inject(0, pos, vel)
        _, diag, phi = O.step(st, params, dt)
        arrived.append(diag["anode"][0])
        if s >= 400:
            prof.append(phi.mean(axis=(1, 2)))
    got = np.mean(arrived[400:])
    assert abs(got / per_step - 1) < 0.05, (got, per_step)
    # Space-charge-limited potential: phi / V = (z / d)^(4/3).
    z = np.arange(nz + 1) / nz
    assert np.max(np.abs(np.mean(prof, 0) / V - z ** (4 / 3))) < 0.02


# --------------------------------------------------------------------------
# Planted mistakes: each mutation of the oracle must fail a pin.
# --------------------------------------------------------------------------
def test_planted_field_sign_fails_pin(monkeypatch):
    orig = O.efield
    monkeypatch.setattr(O, "efield", lambda phi, g: -orig(phi, g))
    with pytest.raises(AssertionError):
        test_single_electron_uniform_field_closed_form()


def test_planted_transposed_gather_fails_pin(monkeypatch):
    orig = O.gather
    monkeypatch.setattr(O, "gather", lambda sp, E, g: orig(
        dict(x=sp["y"], y=sp["x"], z=sp["z"]), E, g))
    with pytest.raises(AssertionError):
        test_gather_reproduces_linear_field_on_weight_lattice()


def test_planted_dropped_neumann_term_fails_pin(monkeypatch):
    orig = P.add_boundary_terms

    def dropped(b, g):
        g2 = P.Grid(g.nx, g.ny, g.nz, g.dx, g.bc_lo, g.bc_hi,
                    0.0 if g.bc_lo == P.NEUMANN else g.v_lo, g.v_hi)
        return orig(b, g2)
    monkeypatch.setattr(P, "add_boundary_terms", dropped)
    from tests.test_oracle_basics import test_neumann_quadratic_is_exact
    with pytest.raises(AssertionError):
        test_neumann_quadratic_is_exact()


def test_planted_wrong_deposit_sign_fails_pin(monkeypatch):
    orig = O.deposit
    monkeypatch.setattr(O, "deposit", lambda st: -orig(st))
    with pytest.raises(AssertionError):
        test_deposit_total_charge_exact()
