"""Oracle pins of the surface-sink completion (CPU only): the nanoparticle
as an electron absorber with its electron-heating tally, and the hand-back
of cathode ions to MD (Appendix A: NP electron heating; transfer of
bombarding ions).

* alpha_EH from the paper's worked estimate (R = 0.15, d = 1 nm,
  ell = 7 A, phi = 4.5 eV, E_e = 20 eV): the printed factors 0.85 and 0.76
  and the result of about 0.5.
* A beam of electrons moving straight up through the ball's z extent in
  one step (field zero): an electron is absorbed exactly when its
  transverse distance to the centre is below R (closed form per electron),
  so the absorbed fraction of a uniform beam is pi R^2 / A.
* Paths that end short of the ball, move away from it, start inside it or
  cross the periodic seam to reach it.
* The heat tally: alpha_EH times the kinetic energy of each absorbed
  electron's half-step velocity.
* MD return: offset of exactly three lattice constants against the
  velocity, above the surface for an incoming ion.
"""
import numpy as np
import pytest

import workloads as W
from oracle import constants as C
from oracle import pic as O
from oracle import poisson as P

A_CU = 3.64e-10   # the paper's Cu lattice constant (gap of 1200 a = 436.8 nm)


def test_alpha_eh_worked_estimate():
    a = O.alpha_eh(0.15, 1e-9, 7e-10, 4.5, 20.0)
    assert round(1.0 - 0.15, 2) == 0.85
    assert round(1.0 - np.exp(-1e-9 / 7e-10), 2) == 0.76
    assert round(1.0 - 4.5 / 20.0, 3) == 0.775
    assert abs(a - 0.85 * 0.76 * 0.775) < 1e-3
    assert abs(a - 0.5) < 0.005


def test_planted_printed_exponent_fails_pin(monkeypatch):
    monkeypatch.setattr(O, "alpha_eh", lambda R, d, ell, phi, E: (
        (1 - R) * np.exp(-d / ell) * (1 - phi / E)))
    with pytest.raises(AssertionError):
        test_alpha_eh_worked_estimate()


def _grid():
    return P.Grid(16, 16, 32, 2e-9, v_lo=0.0, v_hi=0.0)


def _sphere(g, R=5e-9, cx=None, cy=None):
    return dict(cx=g.lx / 2 if cx is None else cx,
                cy=g.ly / 2 if cy is None else cy, cz=30e-9, radius=R,
                n=0, T_K=3500.0, absorb=True, alpha_eh=0.5)


def _step(g, sph, pos, vel, dt=1e-15):
    st = O.State(g)
    st.load(C.ELECTRON, pos, vel, np.arange(pos.shape[0], dtype=np.uint64))
    params = dict(sources=dict(sphere=sph),
                  collisions=dict(enabled=False, sigma_el=0.0,
                                  ion_model="const", sigma_ion_const=0.0))
    E = np.zeros(g.shape + (3,))
    ab, diag = O.advance(st, params, E, dt)
    return st, diag


def test_beam_absorbed_exactly_inside_the_disc_of_the_ball():
    """Electrons from z = cz - 7 nm move up by 14 nm in one step, so every
    path crosses the ball's whole z extent; absorbed iff (x-cx)^2 + (y-cy)^2
    < R^2 (tangent paths excluded by the seeded positions)."""
    g = _grid()
    sph = _sphere(g)
    rng = np.random.default_rng(3)
    n = 20000
    half = 8e-9
    pos = np.empty((n, 3))
    pos[:, 0] = sph["cx"] + (2 * rng.random(n) - 1) * half
    pos[:, 1] = sph["cy"] + (2 * rng.random(n) - 1) * half
    pos[:, 2] = sph["cz"] - 7e-9
    dt = 1e-15
    vel = np.zeros((n, 3))
    vel[:, 2] = 14e-9 / dt
    st, diag = _step(g, sph, pos, vel, dt)
    r2 = (pos[:, 0] - sph["cx"]) ** 2 + (pos[:, 1] - sph["cy"]) ** 2
    inside = r2 < sph["radius"] ** 2
    left = np.sort(st.sp[C.ELECTRON]["id"])
    assert np.array_equal(left, np.nonzero(~inside)[0].astype(np.uint64))
    assert diag["np_hits"] == int(inside.sum())
    frac = diag["np_hits"] / n
    expect = np.pi * sph["radius"] ** 2 / (2 * half) ** 2
    sig = np.sqrt(expect * (1 - expect) / n)
    assert abs(frac - expect) < 4 * sig, (frac, expect)
    # Heat: alpha_EH * 1/2 m v^2 per absorbed electron.
    e1 = 0.5 * C.M_E * (14e-9 / dt) ** 2
    assert np.isclose(diag["np_heat"], 0.5 * e1 * diag["np_hits"], rtol=1e-12)
    assert diag["anode"][0] == 0 and diag["cathode"][0] == 0


def test_paths_short_away_inside_and_across_the_seam():
    g = _grid()
    R = 5e-9
    dt = 1e-15
    # Short: ends 0.1 nm below the ball's bottom.  Away: starts just above
    # the top and moves up.  Inside: starts at the centre.  Grazing: passes
    # 1e-3 nm outside the rim.
    sph = _sphere(g, R)
    cx, cy, cz = sph["cx"], sph["cy"], sph["cz"]
    pos = np.array([[cx, cy, cz - R - 3e-9],
                    [cx, cy, cz + R + 1e-10],
                    [cx, cy, cz],
                    [cx + R + 1e-12, cy, cz - 8e-9]])
    vel = np.array([[0, 0, 2.9e-9 / dt], [0, 0, 5e-9 / dt], [1e5, 0, 0],
                    [0, 0, 16e-9 / dt]])
    st, diag = _step(g, sph, pos, vel, dt)
    assert np.array_equal(np.sort(st.sp[0]["id"]), np.array([0, 1, 3], np.uint64))
    # Across the seam: the ball sits at x = 1 nm, the electron starts at
    # x = L - 3 nm and moves +x by 4 nm through the periodic boundary.
    sph2 = _sphere(g, 1.5e-9, cx=1e-9)
    pos2 = np.array([[g.lx - 3e-9, sph2["cy"], sph2["cz"]]])
    vel2 = np.array([[4e-9 / dt, 0.0, 0.0]])
    st2, diag2 = _step(g, sph2, pos2, vel2, dt)
    assert diag2["np_hits"] == 1 and st2.count(0) == 0


def test_planted_absorber_ignored_fails_pin(monkeypatch):
    monkeypatch.setattr(O, "sphere_hit", lambda *a, **k: np.zeros(
        np.asarray(a[0]).shape, dtype=bool))
    with pytest.raises(AssertionError):
        test_beam_absorbed_exactly_inside_the_disc_of_the_ball()


def test_md_return_offset_three_lattice_constants():
    rng = np.random.default_rng(9)
    n = 50
    ab = dict(species=np.r_[np.zeros(10, int), np.full(n, C.ION)],
              id=np.arange(10 + n, dtype=np.uint64),
              x=rng.random(10 + n) * 3e-8, y=rng.random(10 + n) * 3e-8,
              z=np.zeros(10 + n),
              vx=rng.standard_normal(10 + n) * 1e3,
              vy=rng.standard_normal(10 + n) * 1e3,
              vz=-np.abs(rng.standard_normal(10 + n)) * 1e4)
    md = O.md_return(ab, A_CU)
    assert np.array_equal(md["id"], ab["id"][10:])
    d = np.stack([md["x"] - ab["x"][10:], md["y"] - ab["y"][10:],
                  md["z"] - ab["z"][10:]], 1)
    v = np.stack([ab["vx"][10:], ab["vy"][10:], ab["vz"][10:]], 1)
    L = np.linalg.norm(d, axis=1)
    assert np.allclose(L, 3 * A_CU, rtol=1e-14, atol=0)
    cosang = np.sum(d * v, 1) / (L * np.linalg.norm(v, axis=1))
    assert np.allclose(cosang, -1.0, atol=1e-12)
    assert np.all(md["z"] > 0)
    # Wrapped into the periodic box: an ion at the seam moving -x comes
    # back on the far side.
    g = P.Grid(8, 8, 8, 2e-9)
    one = {k: v[:1].copy() for k, v in ab.items()}
    one.update(species=np.array([C.ION]), x=np.array([1e-10]),
               y=np.array([5e-9]), vx=np.array([1e4]), vy=np.array([0.0]),
               vz=np.array([-1e4]))
    w = O.md_return(one, A_CU, g)
    assert 0.0 <= w["x"][0] < g.lx and w["x"][0] > g.lx - 1e-9


def test_planted_forward_offset_fails_pin(monkeypatch):
    orig = O.md_return

    def forward(ab, a, grid=None, species=(C.ION,)):
        return orig(ab, -a, grid, species)
    monkeypatch.setattr(O, "md_return", forward)
    with pytest.raises(AssertionError):
        test_md_return_offset_three_lattice_constants()
