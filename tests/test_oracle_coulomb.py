"""Pins of the Coulomb binary collisions (CPU only; the paper's Monte Carlo
collisions include Coulomb collisions, after Takizuka & Abe).

* Geometry of one collision: the relative velocity keeps its length and
  turns by theta = 2 atan(delta); its change has the components
  u sin(theta) cos(phi) and u sin(theta) sin(phi) on the two axes
  perpendicular to u (the one in the plane of u and z, and the one in the
  x-y plane) and -u (1 - cos(theta)) along u; momentum and energy are kept.
* Variance: a cold electron beam through cold Cu+ ions loses velocity
  along the beam at the mean rate <1 - cos(theta)> u per collision, with
  the normal delta of the stated variance; to first order in delta^2 that
  is the textbook slowing-down rate e^4 n lnL / (4 pi eps0^2 m_r^2 u^2).
* Pairing: the particles of a cell pair as the random order says (pairs
  keep their own momentum), an odd triplet keeps its momentum as a group.
* A random plasma keeps its total momentum and energy over a call.
Planted mistakes (variance off by two, an azimuth sign) fail pins.
"""
import numpy as np
import pytest

from oracle import constants as C
from oracle import coulomb as K
from oracle import pic as O
from oracle import poisson as P


def _frame(u):
    ux, uy, uz = u
    un = np.linalg.norm(u)
    up = np.hypot(ux, uy)
    e1 = np.array([ux * uz / (up * un), uy * uz / (up * un), -up / un])
    e2 = np.array([-uy / up, ux / up, 0.0])
    return u / un, e1, e2


@pytest.mark.parametrize("delta, phi", [(0.3, 0.7), (-1.7, 4.0), (0.02, 2.5)])
def test_one_collision_geometry(delta, phi):
    rng = np.random.default_rng(1)
    v1 = rng.standard_normal(3) * 1e6
    v2 = rng.standard_normal(3) * 3e3
    m1, m2 = C.M_E, C.M_CU
    n1, n2 = K.scatter(v1, v2, m1, m2, delta, phi)
    n1, n2 = np.array(n1), np.array(n2)
    u = v1 - v2
    du = (n1 - n2) - u
    un = np.linalg.norm(u)
    th = 2 * np.arctan(delta)
    uh, e1, e2 = _frame(u)
    assert np.isclose(np.linalg.norm(n1 - n2), un, rtol=1e-13)
    assert np.isclose(du @ uh, -un * (1 - np.cos(th)), rtol=1e-10, atol=1e-9 * un)
    assert np.isclose(du @ e1, un * np.sin(th) * np.cos(phi), rtol=1e-10, atol=1e-9 * un)
    assert np.isclose(du @ e2, un * np.sin(th) * np.sin(phi), rtol=1e-10, atol=1e-9 * un)
    p0, p1 = m1 * v1 + m2 * v2, m1 * n1 + m2 * n2
    assert np.allclose(p1, p0, rtol=0, atol=1e-13 * np.linalg.norm(m1 * v1))
    e0 = 0.5 * (m1 * v1 @ v1 + m2 * v2 @ v2)
    e1_ = 0.5 * (m1 * n1 @ n1 + m2 * n2 @ n2)
    assert abs(e1_ - e0) <= 1e-12 * e0


def test_collision_along_z_is_the_explicit_rotation():
    v1 = np.array([0.0, 0.0, 2e6])
    v2 = np.zeros(3)
    n1, n2 = K.scatter(v1, v2, C.M_E, C.M_E, 0.5, 1.0)
    du = (np.array(n1) - np.array(n2)) - v1
    th = 2 * np.arctan(0.5)
    ref = 2e6 * np.array([np.sin(th) * np.cos(1.0), np.sin(th) * np.sin(1.0),
                          -(1 - np.cos(th))])
    assert np.allclose(du, ref, rtol=1e-13, atol=1e-6)


def test_planted_azimuth_sign_fails_pin(monkeypatch):
    orig = K.scatter
    monkeypatch.setattr(K, "scatter", lambda v1, v2, m1, m2, d, p: orig(
        v1, v2, m1, m2, d, -p))
    with pytest.raises(AssertionError):
        test_one_collision_geometry(0.3, 0.7)


def _beam_state(n_cells=4096, u=1.2e6, ions_per_cell=1):
    g = P.Grid(16, 16, 16, 2e-9)
    st = O.State(g, seed=9)
    cells = np.arange(n_cells)
    i, j, k = cells % 16, (cells // 16) % 16, cells // 256
    centre = (np.stack([i, j, k], 1) + 0.5) * g.dx
    vel = np.zeros((n_cells, 3))
    vel[:, 2] = u
    st.load(C.ELECTRON, centre, vel, np.arange(n_cells, dtype=np.uint64))
    ip = np.repeat(centre, ions_per_cell, axis=0) + 0.1 * g.dx
    st.load(C.ION, ip, np.zeros_like(ip),
            np.arange(n_cells * ions_per_cell, dtype=np.uint64) + 10 ** 6)
    return st


def test_beam_slowing_down_rate():
    u, dt, lnl = 1.2e6, 1e-16, 10.0
    st = _beam_state(u=u)
    g = st.grid
    params = {"coulomb": {"enabled": True, "ln_lambda": lnl}}
    K.coulomb(st, params, dt)
    dv = st.sp[C.ELECTRON]["vz"] - u
    n = 1.0 / g.dx ** 3
    mr = C.M_E * C.M_CU / (C.M_E + C.M_CU)
    var = (C.E_CHARGE ** 4 * n * lnl * dt) / (8 * np.pi * C.EPS0 ** 2 * mr ** 2 * u ** 3)
    # E[1 - cos theta] = E[2 d^2 / (1 + d^2)], d ~ N(0, var): Gauss-Hermite.
    x, w = np.polynomial.hermite_e.hermegauss(80)
    d2 = var * x * x
    e_omc = np.sum(w * 2 * d2 / (1 + d2)) / np.sqrt(2 * np.pi)
    expect = -(mr / C.M_E) * u * e_omc
    se = np.std(dv) / np.sqrt(dv.size)
    assert abs(dv.mean() - expect) < 4 * se, (dv.mean(), expect, se)
    # First order in <delta^2>: the textbook slowing-down rate.
    rate = C.E_CHARGE ** 4 * n * lnl / (4 * np.pi * C.EPS0 ** 2 * mr ** 2 * u ** 2)
    assert abs(expect / dt * (C.M_E / mr) + rate) < 0.15 * rate


def test_planted_variance_factor_fails_pin(monkeypatch):
    orig = K.variance
    monkeypatch.setattr(K, "variance", lambda *a: 2.0 * orig(*a))
    with pytest.raises(AssertionError):
        test_beam_slowing_down_rate()


def test_pairs_follow_the_random_order():
    g = P.Grid(4, 4, 4, 2e-9)
    st = O.State(g, seed=3)
    rng = np.random.default_rng(5)
    N = 7                                      # triplet + two pairs
    pos = (np.array([1.5, 2.5, 0.5]) + 0.3 * rng.random((N, 3))) * g.dx
    vel = rng.standard_normal((N, 3)) * 1e6
    ids = np.arange(N, dtype=np.uint64) * 13 + 5
    st.load(C.ELECTRON, pos, vel, ids)
    K.coulomb(st, {"coulomb": {"enabled": True, "ln_lambda": 10.0}}, 2e-16)
    new = np.stack([st.sp[0][k] for k in ("vx", "vy", "vz")], 1)
    order = np.lexsort((ids, K.order_key(ids, 0, 3)))
    groups = [order[:3], order[3:5], order[5:7]]
    for grp in groups:
        assert np.allclose(new[grp].sum(0), vel[grp].sum(0), rtol=0,
                           atol=1e-9 * np.abs(vel).max())
        assert not np.allclose(new[grp], vel[grp])
    # Any other grouping of the same size would not keep its momentum.
    wrong = np.r_[order[3], order[5]]
    assert not np.allclose(new[wrong].sum(0), vel[wrong].sum(0), rtol=0,
                           atol=1e-9 * np.abs(vel).max())


def test_plasma_keeps_momentum_and_energy():
    g = P.Grid(8, 8, 8, 2e-9)
    st = O.State(g, seed=4)
    rng = np.random.default_rng(6)
    for s, n, m, sc in ((C.ELECTRON, 3000, C.M_E, 1e6),
                        (C.ION, 2000, C.M_CU, 2e3)):
        pos = rng.random((n, 3)) * np.array([g.lx, g.ly, g.lz])
        st.load(s, pos, rng.standard_normal((n, 3)) * sc,
                np.arange(n, dtype=np.uint64) + 10 ** 5 * s)

    def totals():
        p = np.zeros(3)
        e = 0.0
        for s, m in ((C.ELECTRON, C.M_E), (C.ION, C.M_CU)):
            v = np.stack([st.sp[s][k] for k in ("vx", "vy", "vz")], 1)
            p += m * v.sum(0)
            e += 0.5 * m * np.sum(v * v)
        return p, e
    p0, e0 = totals()
    n_like, n_ei = K.coulomb(st, {"coulomb": {"enabled": True}}, 2e-16)
    p1, e1 = totals()
    assert n_like > 1000 and n_ei > 1000
    scale = C.M_E * 1e6 * 3000
    assert np.allclose(p1, p0, rtol=0, atol=1e-12 * scale)
    assert abs(e1 - e0) <= 1e-12 * e0
