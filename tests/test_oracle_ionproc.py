"""Pins of recombination, ionisation of Cu+ and charge exchange (CPU only;
the paper's Monte Carlo collisions include charge exchange and
recombination, and its ions reach several charge levels).

* Eq. 4 evaluated per electron: the fraction of electrons at one energy
  that recombine (or ionise Cu+) in one step is 1 - exp(-n_i sigma v dt)
  when the cell has Cu+ to spare; the split between the two processes
  follows their cross sections.
* Kinematics: the recombined atom has the pair's centre-of-mass velocity
  and the ion's position and id; an ionisation conserves energy minus the
  threshold; the Cu2+ keeps the ion's state; secondary ids follow the
  primaries' id order from next_id.
* Starvation: one Cu+ in a cell is taken by the first colliding electron
  of the random order only.
* Charge exchange: the fraction of ions that exchange is
  1 - exp(-n_n sigma_cx u dt); an exchange swaps the two records.
* Charge: the deposited total follows N(Cu+) + 2 N(Cu2+) - N(e).
* Cu2+ moves with acceleration 2 e E / M in a uniform field.
Planted mistakes each fail a pin.
"""
import numpy as np
import pytest

from oracle import constants as C
from oracle import ionproc as I
from oracle import pic as O
from oracle import poisson as P


def _grid(n=8, dx=2e-9):
    return P.Grid(n, n, n, dx)


def _cells_state(g, n_cells, e_per, i_per, n_per=0, E_eV=5.0, seed=3,
                 ion_v=0.0):
    st = O.State(g, seed=seed)
    rng = np.random.default_rng(seed)
    cells = np.arange(n_cells)
    base = np.stack([cells % g.nx, (cells // g.nx) % g.ny,
                     cells // (g.nx * g.ny)], 1).astype(float)
    v = np.sqrt(2 * E_eV * C.E_CHARGE / C.M_E)

    def fill(per, vel_fn):
        pos = (np.repeat(base, per, 0) + 0.05 + 0.9 * rng.random((n_cells * per, 3))) * g.dx
        return pos, vel_fn(n_cells * per)
    pe, ve = fill(e_per, lambda k: np.tile([0.0, 0.0, v], (k, 1)))
    pi_, vi = fill(i_per, lambda k: np.tile([ion_v, 0.0, 0.0], (k, 1)))
    st.load(C.ELECTRON, pe, ve, np.arange(pe.shape[0], dtype=np.uint64))
    st.load(C.ION, pi_, vi, np.arange(pi_.shape[0], dtype=np.uint64) + 10 ** 7)
    if n_per:
        pn, vn = fill(n_per, lambda k: np.zeros((k, 3)))
        st.load(C.NEUTRAL, pn, vn, np.arange(pn.shape[0], dtype=np.uint64) + 2 * 10 ** 7)
    st.next_id = 3 * 10 ** 7
    return st, v


def _run(st, cfg, dt):
    near, diag = {}, {}
    I.ion_processes(st, {"ion_processes": cfg}, dt, near, diag)
    return diag, near


def test_recombination_rate_and_kinematics():
    g = _grid()
    st, v = _cells_state(g, 512, 1, 40, E_eV=2.0)
    cfg = dict(enabled=True, sigma_rec_1eV=2e-20, lotz_a2=0.0)
    dt = 2e-16
    el0 = {k: a.copy() for k, a in st.sp[C.ELECTRON].items()}
    io0 = {k: a.copy() for k, a in st.sp[C.ION].items()}
    diag, _ = _run(st, cfg, dt)
    n_i = 40 / g.dx ** 3
    sig = 2e-20 * (1.0 / 2.0)
    p = 1 - np.exp(-n_i * sig * v * dt)
    n = 512
    assert abs(diag["recombinations"] / n - p) < 4 * np.sqrt(p * (1 - p) / n), (diag, p)
    assert diag["ionisations2"] == 0 and diag["f3_starved"] == 0
    nu = st.sp[C.NEUTRAL]
    assert nu["x"].size == diag["recombinations"]
    # Each atom: an ion's id and position, the pair's centre-of-mass velocity.
    for k in range(nu["x"].size):
        j = np.nonzero(io0["id"] == nu["id"][k])[0][0]
        assert nu["x"][k] == io0["x"][j] and nu["z"][k] == io0["z"][j]
        cell = (np.floor(io0["x"][j] * g.inv_dx) + g.nx * np.floor(io0["y"][j] * g.inv_dx)
                + g.nx * g.ny * np.floor(io0["z"][j] * g.inv_dx))
        ce = (np.floor(el0["x"] * g.inv_dx) + g.nx * np.floor(el0["y"] * g.inv_dx)
              + g.nx * g.ny * np.floor(el0["z"] * g.inv_dx))
        e = np.nonzero(ce == cell)[0][0]
        vz = (C.M_CU * io0["vz"][j] + C.M_E * el0["vz"][e]) / (C.M_CU + C.M_E)
        assert nu["vz"][k] == vz
    assert st.sp[C.ION]["x"].size == io0["x"].size - diag["recombinations"]
    assert st.sp[C.ELECTRON]["x"].size == n - diag["recombinations"]


def test_planted_ion_only_velocity_fails_pin(monkeypatch):
    orig = I.ion_processes

    def wrong(state, params, dt, near, diag):
        orig(state, params, dt, near, diag)
        state.sp[C.NEUTRAL]["vz"] = state.sp[C.NEUTRAL]["vz"] * 0.0
    monkeypatch.setattr(I, "ion_processes", wrong)
    with pytest.raises(AssertionError):
        test_recombination_rate_and_kinematics()


def test_ionisation_of_cu_plus_rate_energy_and_ids():
    g = _grid()
    E = 80.0
    st, v = _cells_state(g, 512, 1, 40, E_eV=E, seed=5)
    cfg = dict(enabled=True, sigma_rec_1eV=0.0, lotz_a2=4.5e-16, I2_eV=20.29)
    dt = 2e-16
    el0 = {k: a.copy() for k, a in st.sp[C.ELECTRON].items()}
    io0 = {k: a.copy() for k, a in st.sp[C.ION].items()}
    next0 = st.next_id
    diag, _ = _run(st, cfg, dt)
    n_i = 40 / g.dx ** 3
    sig = 4.5e-16 * np.log(E / 20.29) / (E * 20.29)
    p = 1 - np.exp(-n_i * sig * v * dt)
    n = 512
    k = diag["ionisations2"]
    assert abs(k / n - p) < 4 * np.sqrt(p * (1 - p) / n), (k, p)
    el = st.sp[C.ELECTRON]
    assert el["x"].size == n + k
    sec = el["id"] >= np.uint64(next0)
    assert np.array_equal(np.sort(el["id"][sec]),
                          np.arange(next0, next0 + k, dtype=np.uint64))
    # Energy: primary + secondary = E - I2, secondary at the primary's spot.
    prim_ids = el0["id"][[np.any(np.abs(el["x"][sec] - x) == 0) for x in el0["x"]]]
    assert prim_ids.size == k
    order = np.argsort(prim_ids)
    sec_sorted = np.argsort(el["id"][sec])
    ke = 0.5 * C.M_E * (el["vx"] ** 2 + el["vy"] ** 2 + el["vz"] ** 2) / C.E_CHARGE
    for r in range(k):
        pid = prim_ids[order[r]]
        pe = np.nonzero(el["id"] == pid)[0][0]
        se = np.nonzero(sec)[0][sec_sorted[r]]
        assert el["x"][se] == el["x"][pe]
        assert abs(ke[pe] + ke[se] - (E - 20.29)) <= 1e-12 * E
    ion2 = st.sp[C.ION2]
    assert ion2["x"].size == k
    assert np.all(np.isin(ion2["id"], io0["id"]))
    assert st.sp[C.ION]["x"].size == io0["x"].size - k


def test_one_ion_is_taken_by_the_first_colliding_electron():
    g = _grid()
    st, v = _cells_state(g, 64, 6, 1, E_eV=3.0, seed=8)
    cfg = dict(enabled=True, sigma_rec_1eV=1e-12, lotz_a2=0.0)
    diag, _ = _run(st, cfg, 2e-16)
    # Every electron collides (huge cross section): one recombination and
    # five starved events per cell.
    assert diag["recombinations"] == 64 and diag["f3_starved"] == 64 * 5
    assert st.sp[C.ION]["x"].size == 0
    # The electron that recombined is the first of its cell's random order.
    left = set(st.sp[C.ELECTRON]["id"].tolist())
    key = I.order_key(np.arange(64 * 6, dtype=np.uint64), 0, 8)
    for c in range(64):
        ids = np.arange(6 * c, 6 * c + 6, dtype=np.uint64)
        first = ids[np.lexsort((ids, key[6 * c:6 * c + 6]))[0]]
        assert int(first) not in left
        assert all(int(i) in left for i in ids if i != first)


def test_charge_exchange_rate_and_swap():
    g = _grid()
    u = 2e4
    st, _ = _cells_state(g, 512, 0, 1, n_per=30, seed=11, ion_v=u)
    sig = 5e-19
    cfg = dict(enabled=True, sigma_rec_1eV=0.0, lotz_a2=0.0,
               cx_a=np.sqrt(sig), cx_b=0.0)
    io0 = {k: a.copy() for k, a in st.sp[C.ION].items()}
    nu0 = {k: a.copy() for k, a in st.sp[C.NEUTRAL].items()}
    dt = 2e-15
    diag, _ = _run(st, cfg, dt)
    n_n = 30 / g.dx ** 3
    p = 1 - np.exp(-n_n * sig * u * dt)
    k = diag["charge_exchanges"]
    assert abs(k / 512 - p) < 4 * np.sqrt(p * (1 - p) / 512), (k, p)
    io, nu = st.sp[C.ION], st.sp[C.NEUTRAL]
    swapped = io["id"] != io0["id"]
    assert swapped.sum() == k
    for j in np.nonzero(swapped)[0]:
        a = np.nonzero(nu0["id"] == io["id"][j])[0][0]
        assert io["x"][j] == nu0["x"][a] and io["vx"][j] == nu0["vx"][a]
        b = np.nonzero(nu["id"] == io0["id"][j])[0][0]
        assert nu["x"][b] == io0["x"][j] and nu["vx"][b] == u


def test_planted_cx_rate_fails_pin(monkeypatch):
    orig = I.IonProcesses.sigma_cx
    monkeypatch.setattr(I.IonProcesses, "sigma_cx",
                        lambda self, eps: 2.0 * orig(self, eps))
    with pytest.raises(AssertionError):
        test_charge_exchange_rate_and_swap()


def test_deposit_counts_cu2_twice():
    g = _grid()
    st = O.State(g)
    rng = np.random.default_rng(2)
    for s, n in ((C.ELECTRON, 300), (C.ION, 200), (C.ION2, 50)):
        pos = rng.random((n, 3)) * [g.lx, g.ly, g.lz]
        st.load(s, pos, np.zeros_like(pos), np.arange(n, dtype=np.uint64) + 1000 * s)
    assert O.deposit(st).sum() == 2 ** 39 * (200 + 2 * 50 - 300)


def test_cu2_uniform_field_closed_form():
    g = P.Grid(4, 4, 64, 5e-9, v_lo=0.0, v_hi=-100.0)
    E = O.efield(P.solve_exact(P.add_boundary_terms(np.zeros(g.shape), g), g), g)
    Ez = E[10, 1, 1, 2]
    st = O.State(g)
    x0 = np.array([[1e-9, 1e-9, 2e-7]])
    st.load(C.ION2, x0, np.zeros((1, 3)), np.array([5], dtype=np.uint64))
    dt = 1e-14
    sp = st.sp[C.ION2]
    for n in range(1, 6):
        O.push(sp, C.ION2, E, g, dt)
        a = 2 * C.E_CHARGE * Ez / C.M_CU
        z = x0[0, 2] + a * dt * dt * n * (n + 1) / 2
        assert abs(sp["z"][0] - z) <= 1e-12 * abs(z)


def test_planted_cu2_single_charge_fails_pin(monkeypatch):
    monkeypatch.setattr(C, "CHARGE_SIGN", (-1, 0, 1, 1))
    with pytest.raises(AssertionError):
        test_cu2_uniform_field_closed_form()
