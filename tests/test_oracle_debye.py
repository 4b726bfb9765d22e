"""Pins of the Debye-length resolution check (CPU only; Appendix A: mesh
criterion d_max = 3.4 lambda_D alpha_D with alpha_D = 0.5, lambda_D of the
electrons and ions).

* Closed forms: two electrons with opposite velocities in one block give
  k T = m (2 v^2) / 3 exactly (unbiased variance over the three
  components), so lambda_D^2 = eps0 k T / (n e^2) with n = 2 w / V; adding
  two ions adds their term to 1 / lambda_D^2.
* A drifting Maxwellian of many electrons per block recovers the textbook
  lambda_D = sqrt(eps0 k T / (n e^2)) of its temperature (drift removed).
* The criterion: blocks are flagged exactly when dx > 3.4 alpha_D lambda_D.
Planted mistakes (biased variance, drift kept in the temperature, ions
dropped) each fail one of them.
"""
import numpy as np
import pytest

from oracle import constants as C
from oracle import pic as O
from oracle import poisson as P


def _state(nx=8, ny=8, nz=8, dx=2e-9, w=1):
    return O.State(P.Grid(nx, ny, nz, dx), w_sp=w)


def test_two_electrons_closed_form():
    st = _state(w=3)
    g = st.grid
    v = 1.7e6
    pos = np.array([[1.2, 3.4, 5.6], [1.7, 3.1, 5.2]]) * g.dx
    vel = np.array([[v, 0.0, 0.0], [-v, 0.0, 0.0]])
    st.load(C.ELECTRON, pos, vel, np.arange(2, dtype=np.uint64))
    out = O.debye_check(st, block=1)
    kT = C.M_E * (2 * v * v) / 3.0
    n = 2 * 3 / g.dx ** 3
    lam = np.sqrt(C.EPS0 * kT / (n * C.E_CHARGE ** 2))
    got = out["lambda_D"][5, 3, 1]
    assert out["checked"] == 1
    assert abs(got - lam) <= 1e-14 * lam
    assert np.isinf(out["lambda_D"][0, 0, 0])


def test_electrons_and_ions_add_inverse_squares():
    st = _state()
    g = st.grid
    v, u = 9e5, 2.5e3
    st.load(C.ELECTRON, np.array([[0.5, 0.5, 0.5], [0.6, 0.4, 0.3]]) * g.dx,
            np.array([[0.0, v, 0.0], [0.0, -v, 0.0]]),
            np.arange(2, dtype=np.uint64))
    st.load(C.ION, np.array([[0.2, 0.7, 0.9], [0.9, 0.1, 0.1]]) * g.dx,
            np.array([[u, u, 0.0], [-u, -u, 0.0]]),
            np.arange(2, 4, dtype=np.uint64))
    out = O.debye_check(st, block=1)
    n = 2 / g.dx ** 3
    kTe = C.M_E * (2 * v * v) / 3.0
    kTi = C.M_CU * (4 * u * u) / 3.0
    inv = n * C.E_CHARGE ** 2 / C.EPS0 * (1 / kTe + 1 / kTi)
    assert abs(out["lambda_D"][0, 0, 0] - inv ** -0.5) <= 1e-14 * inv ** -0.5


def test_drifting_maxwellian_recovers_textbook_length():
    st = _state(nx=16, ny=16, nz=16, dx=5e-9)
    g = st.grid
    rng = np.random.default_rng(7)
    n_per = 5000
    kT_eV = 5.0
    pos = rng.random((8 * n_per, 3)) * np.array([g.lx, g.ly, g.lz])
    vel = rng.standard_normal((8 * n_per, 3)) * np.sqrt(kT_eV * C.E_CHARGE / C.M_E)
    vel[:, 2] += 3e6                                   # drift
    st.load(C.ELECTRON, pos, vel, np.arange(pos.shape[0], dtype=np.uint64))
    out = O.debye_check(st, block=8)
    n = n_per / (8 * g.dx) ** 3
    lam = np.sqrt(C.EPS0 * kT_eV * C.E_CHARGE / (n * C.E_CHARGE ** 2))
    rel = np.abs(out["lambda_D"] / lam - 1)
    assert out["checked"] == 8 and rel.max() < 0.03, rel


def test_criterion_flags_exactly_the_underresolved_blocks():
    st = _state(nx=4, ny=4, nz=8, dx=2e-9)
    g = st.grid
    rng = np.random.default_rng(3)
    pos, vel = [], []
    # Every cell holds two electrons with opposite velocities whose speed
    # puts dx / d_max between about 0.6 and 1.8.
    temps = []
    for k in range(g.nz):
        for j in range(g.ny):
            for i in range(g.nx):
                v = 7e5 * (1 + 2 * rng.random())
                temps.append(v)
                c = np.array([i + 0.5, j + 0.5, k + 0.5]) * g.dx
                pos += [c, c]
                vel += [[v, 0, 0], [-v, 0, 0]]
    st.load(C.ELECTRON, np.array(pos), np.array(vel),
            np.arange(len(pos), dtype=np.uint64))
    alpha = 0.5
    out = O.debye_check(st, block=1, alpha_D=alpha)
    lam = out["lambda_D"].reshape(-1)
    expect = g.dx > 3.4 * alpha * lam
    assert 0 < expect.sum() < lam.size
    assert out["unresolved"] == int(expect.sum())
    assert np.isclose(out["ratio_max"], np.max(g.dx / (3.4 * alpha * lam)),
                      rtol=1e-15)


def test_planted_biased_variance_fails_pin(monkeypatch):
    orig = O.debye_check

    def biased(state, block=1, alpha_D=0.5):
        out = orig(state, block, alpha_D)
        # N instead of N - 1 for two particles: kT halved, lambda / sqrt(2).
        out["lambda_D"] = out["lambda_D"] / np.sqrt(2.0)
        return out
    monkeypatch.setattr(O, "debye_check", biased)
    with pytest.raises(AssertionError):
        test_two_electrons_closed_form()


def test_planted_drift_kept_fails_pin(monkeypatch):
    def with_drift(state, block=1, alpha_D=0.5):
        sp = state.sp[C.ELECTRON]
        g = state.grid
        v2 = (sp["vx"] ** 2 + sp["vy"] ** 2 + sp["vz"] ** 2).sum() / 8
        n = sp["x"].size / 8 / (block * g.dx) ** 3
        kT = C.M_E * v2 / (3 * (sp["x"].size / 8 - 1))
        lam = np.full((2, 2, 2), np.sqrt(C.EPS0 * kT / (n * C.E_CHARGE ** 2)))
        return dict(lambda_D=lam, checked=8, unresolved=0,
                    lambda_min=float(lam.min()), ratio_max=0.0)
    monkeypatch.setattr(O, "debye_check", with_drift)
    with pytest.raises(AssertionError):
        test_drifting_maxwellian_recovers_textbook_length()


def test_planted_ions_dropped_fails_pin(monkeypatch):
    orig = O.debye_check

    def no_ions(state, block=1, alpha_D=0.5):
        saved = state.sp[C.ION]
        state.sp[C.ION] = O.empty_species()
        try:
            return orig(state, block, alpha_D)
        finally:
            state.sp[C.ION] = saved
    monkeypatch.setattr(O, "debye_check", no_ions)
    with pytest.raises(AssertionError):
        test_electrons_and_ions_add_inverse_squares()
