"""Coulomb collisions by binary pairing within cells (Takizuka & Abe 1977,
the reference the paper gives for its Monte Carlo collisions, which list
Coulomb collisions among them), plain numpy float64.

Test infrastructure only (see the package docstring).

One call after the electron-neutral collisions of a step, on the charged
particles of every cell (cell of the position after the push):

  * Order.  A cell's electrons and its ions are each put in a random order:
    ascending (a, id) with a the 53-bit integer of the first Philox word
    pair of (id, step, TAG_ORDER).
  * Like pairs.  Consecutive particles of the order collide: (0, 1),
    (2, 3), ...; with an odd number N >= 3 the first three collide as
    (0, 1), (1, 2), (2, 0) in that sequence, each with half the variance,
    and the pairs start at 3.  The density is that species' n = N w / dx^3.
  * Electron-ion.  With N_e and N_i >= 1, K = max(N_e, N_i) collisions,
    collision k between electron k mod N_e and ion k mod N_i, in
    ascending k (sequential: a particle of the smaller group collides
    several times).  The density is the lower one, n_L = min(N_e, N_i)
    w / dx^3.  Like pairs act first, then the electron-ion sequence.
  * One collision of particles 1, 2 (masses m1, m2, charges q1, q2) with
    relative velocity u = v1 - v2: delta = tan(theta/2) is normal with
    zero mean and variance
        <delta^2> = q1^2 q2^2 n lnL dt / (8 pi eps0^2 m_r^2 |u|^3)
    (times 1/2 inside a triplet), m_r = m1 m2 / (m1 + m2); phi uniform
    in [0, 2 pi).  With u_perp = sqrt(u_x^2 + u_y^2),
    sin(theta) = 2 delta / (1 + delta^2), 1 - cos(theta) = 2 delta^2 /
    (1 + delta^2):
        du_x = (u_x/u_perp) u_z sin cos(phi) - (u_y/u_perp) |u| sin sin(phi)
               - u_x (1 - cos)
        du_y = (u_y/u_perp) u_z sin cos(phi) + (u_x/u_perp) |u| sin sin(phi)
               - u_y (1 - cos)
        du_z = -u_perp sin cos(phi) - u_z (1 - cos)
    (u_perp = 0: du = (|u| sin cos(phi), |u| sin sin(phi),
    -u_z (1 - cos))), then v1 += (m_r/m1) du, v2 -= (m_r/m2) du: the
    relative velocity turns by theta about itself, momentum and energy are
    kept.  |u| = 0: no collision.
  * Draws: (U1, U2) of (id_c, step, TAG_DELTA) give the normal
    sqrt(-2 ln(1 - U1)) cos(2 pi U2); U3 of (id_c, step, TAG_PHI) gives
    phi = 2 pi U3.  id_c is the first particle of a like pair (each
    particle of a triplet is first once), and for an electron-ion
    collision the particle of the larger group (the electron when equal),
    with the electron-ion tags.
"""
import numpy as np

from . import constants as C
from .philox import philox4x32_10, uniforms

TAG_ORDER = 20
TAG_DELTA, TAG_PHI = 21, 22          # like pairs
TAG_DELTA_EI, TAG_PHI_EI = 23, 24    # electron-ion


def order_key(ids, step, seed):
    """53-bit integer of the order draw of each id (ties broken by id)."""
    ids = np.asarray(ids, dtype=np.uint64)
    seed = int(seed)
    w = philox4x32_10(ids & np.uint64(0xFFFFFFFF), ids >> np.uint64(32),
                      np.uint64(step & 0xFFFFFFFF), np.uint64(TAG_ORDER),
                      np.uint64(seed & 0xFFFFFFFF),
                      np.uint64((seed >> 32) & 0xFFFFFFFF))
    return ((w[0].astype(np.uint64) << np.uint64(21))
            ^ (w[1].astype(np.uint64) >> np.uint64(11)))


def _normal_phi(id_c, step, seed, tag_d, tag_p):
    u1, u2 = uniforms(np.array([id_c], dtype=np.uint64), step, tag_d, seed)
    u3, _ = uniforms(np.array([id_c], dtype=np.uint64), step, tag_p, seed)
    g = np.sqrt(-2.0 * np.log(1.0 - u1[0])) * np.cos(C.TWO_PI * u2[0])
    return g, C.TWO_PI * u3[0]


def scatter(v1, v2, m1, m2, delta, phi):
    """New velocities of one binary collision with deflection
    delta = tan(theta/2) and azimuth phi (see the module docstring)."""
    ux = v1[0] - v2[0]
    uy = v1[1] - v2[1]
    uz = v1[2] - v2[2]
    u = np.sqrt((ux * ux + uy * uy) + uz * uz)
    uperp = np.sqrt(ux * ux + uy * uy)
    d2 = delta * delta
    s = (2.0 * delta) / (1.0 + d2)
    omc = (2.0 * d2) / (1.0 + d2)
    cp, sp = np.cos(phi), np.sin(phi)
    if uperp > 0.0:
        dux = ((ux / uperp) * uz) * s * cp - ((uy / uperp) * u) * s * sp - ux * omc
        duy = ((uy / uperp) * uz) * s * cp + ((ux / uperp) * u) * s * sp - uy * omc
        duz = -(uperp * s) * cp - uz * omc
    else:
        dux = (u * s) * cp
        duy = (u * s) * sp
        duz = -(uz * omc)
    mr = (m1 * m2) / (m1 + m2)
    a1, a2 = mr / m1, mr / m2
    n1 = (v1[0] + a1 * dux, v1[1] + a1 * duy, v1[2] + a1 * duz)
    n2 = (v2[0] - a2 * dux, v2[1] - a2 * duy, v2[2] - a2 * duz)
    return n1, n2


def variance(q1q2_sq, n, ln_lambda, dt, mr, u):
    """<delta^2> of one binary collision (u > 0)."""
    return ((q1q2_sq * n) * ln_lambda * dt) / (
        ((8.0 * np.pi) * (C.EPS0 * C.EPS0)) * ((mr * mr) * ((u * u) * u)))


def _collide(sp1, i1, m1, sp2, i2, m2, n, lnl, dt, id_c, step, seed, tags,
             half=False):
    v1 = (sp1["vx"][i1], sp1["vy"][i1], sp1["vz"][i1])
    v2 = (sp2["vx"][i2], sp2["vy"][i2], sp2["vz"][i2])
    ux, uy, uz = v1[0] - v2[0], v1[1] - v2[1], v1[2] - v2[2]
    u = np.sqrt((ux * ux + uy * uy) + uz * uz)
    if not u > 0.0:
        return
    mr = (m1 * m2) / (m1 + m2)
    e2 = C.E_CHARGE * C.E_CHARGE
    var = variance(e2 * e2, n, lnl, dt, mr, u)
    if half:
        var = 0.5 * var
    g, phi = _normal_phi(id_c, step, seed, *tags)
    delta = np.sqrt(var) * g
    n1, n2 = scatter(v1, v2, m1, m2, delta, phi)
    sp1["vx"][i1], sp1["vy"][i1], sp1["vz"][i1] = n1
    sp2["vx"][i2], sp2["vy"][i2], sp2["vz"][i2] = n2


def _cells(sp, grid):
    i = np.floor(sp["x"] * grid.inv_dx).astype(np.int64) % grid.nx
    j = np.floor(sp["y"] * grid.inv_dx).astype(np.int64) % grid.ny
    k = np.floor(sp["z"] * grid.inv_dx).astype(np.int64)
    return (k * grid.ny + j) * grid.nx + i


def _groups(sp, grid, step, seed):
    """{cell: indices of the species' particles in the cell, in random
    order}."""
    if sp["x"].size == 0:
        return {}
    cell = _cells(sp, grid)
    key = order_key(sp["id"], step, seed)
    o = np.lexsort((sp["id"], key, cell))
    cs = cell[o]
    out = {}
    starts = np.r_[0, np.nonzero(np.diff(cs))[0] + 1]
    ends = np.r_[starts[1:], cs.size]
    for a, b in zip(starts, ends):
        out[int(cs[a])] = o[a:b]
    return out


def _like(sp, idx, m, n, lnl, dt, step, seed):
    """Like-species pairs of one cell; returns the collisions formed."""
    N = idx.size
    if N < 2:
        return 0
    tags = (TAG_DELTA, TAG_PHI)
    start = 0
    if N % 2 == 1:
        a, b, c = idx[0], idx[1], idx[2]
        for p, q in ((a, b), (b, c), (c, a)):
            _collide(sp, p, m, sp, q, m, n, lnl, dt, sp["id"][p], step, seed,
                     tags, half=True)
        start = 3
    for k in range(start, N - 1, 2):
        p, q = idx[k], idx[k + 1]
        _collide(sp, p, m, sp, q, m, n, lnl, dt, sp["id"][p], step, seed, tags)
    return (3 if start else 0) + (N - start) // 2


def coulomb(state, params, dt):
    """Apply one step of Coulomb collisions in place; returns the numbers of
    binary collisions formed (like pairs, a triplet counting three;
    electron-ion), including those skipped for zero relative speed."""
    cfg = params.get("coulomb") or {}
    if not cfg.get("enabled"):
        return 0, 0
    lnl = float(cfg.get("ln_lambda", 10.0))
    g = state.grid
    step, seed = state.step, state.seed
    w_dx3 = float(state.w_sp) * ((g.inv_dx * g.inv_dx) * g.inv_dx)
    el, io = state.sp[C.ELECTRON], state.sp[C.ION]
    ge = _groups(el, g, step, seed)
    gi = _groups(io, g, step, seed)
    n_like = n_ei = 0
    for sp, groups, m in ((el, ge, C.M_E), (io, gi, C.M_CU)):
        for cell, idx in groups.items():
            N = idx.size
            if N >= 2:
                n_like += _like(sp, idx, m, float(N) * w_dx3, lnl, dt, step,
                                seed)
    for cell, ie in ge.items():
        ii = gi.get(cell)
        if ii is None:
            continue
        Ne, Ni = ie.size, ii.size
        nL = float(min(Ne, Ni)) * w_dx3
        for k in range(max(Ne, Ni)):
            a, b = ie[k % Ne], ii[k % Ni]
            id_c = el["id"][a] if Ne >= Ni else io["id"][b]
            _collide(el, a, C.M_E, io, b, C.M_CU, nL, lnl, dt, id_c, step,
                     seed, (TAG_DELTA_EI, TAG_PHI_EI))
            n_ei += 1
    return n_like, n_ei
