"""Recombination, electron-impact ionisation of Cu+ and resonant charge
exchange, plain numpy float64: the remaining processes of the paper's
Monte Carlo collisions ("elastic, Coulomb, ionization, charge exchange and
recombination") and the ions "at various charge levels" they lead to.

Test infrastructure only (see the package docstring).

The paper gives no cross sections for these processes (it defers to its
references), so they are parameters:
  * radiative recombination e + Cu+ -> Cu: sigma_rec(E) = s_rec (1 eV / E),
    E the electron energy in eV (at least 1e-3 eV);
  * ionisation of Cu+, e + Cu+ -> 2e + Cu2+: one-subshell Lotz
    a2 ln(E / I2) / (E I2) above I2 (Cu+ -> Cu2+: 20.29 eV), zero below;
  * resonant charge exchange Cu+ + Cu -> Cu + Cu+:
    sigma_cx = max(a_cx - b_cx ln(eps / 1 eV), 0)^2 with eps the energy of
    the relative motion, m_r u^2 / 2 in eV (at least 1e-6 eV).

One call after the Coulomb collisions of a step (cells of the positions
after the push; tags 25-30 of the particle's Philox stream):

  A. Electrons on Cu+.  A cell's electrons and Cu+ are each put in a random
     order (ascending 53-bit draw of (id, step, 25), then id).  Each
     electron in turn collides with probability
     P = 1 - exp(-n_i (sigma_rec + sigma_ion2) v dt), n_i = N_i w / dx^3
     the cell's Cu+ density and v the electron speed (Eq. 4 evaluated per
     electron): U1 < P with (U1, U2) of tag 26.  The r-th colliding electron
     of the cell takes the r-th Cu+ of the order; with none left it is
     starved (no change).  U2 < sigma_rec / (sigma_rec + sigma_ion2):
     recombination, the electron and the ion leave and a Cu atom appears
     at the ion's position with the ion's id and the pair's centre-of-mass
     velocity (M v_i + m v_e) / (M + m).  Otherwise ionisation of Cu+: the
     energy above I2 is shared uniformly (U3), both electrons leave
     isotropically ((U4, U5), (U6, U7) of tags 27-29), the secondary starts
     at the electron's position, and the ion becomes Cu2+ with its own
     position, velocity and id.  Secondary ids are next_id + rank among
     these events ordered by primary id (after those of the electron-neutral
     ionisations of the step).
  B. Charge exchange.  The Cu+ that are left, in the same order, meet the
     cell's Cu atoms (present before A) in their random order: ion k with
     atom k mod N_n, sequentially.  With u the relative speed,
     P = 1 - exp(-n_n sigma_cx u dt), n_n = N_n w / dx^3, and U1 of tag 30
     below P, the electron passes from the atom to the ion: the two records
     exchange position, velocity and id (each atom keeps its motion; the
     charge moves).
Draws within 1e-6 of a threshold are counted as near-threshold.
"""
import numpy as np

from . import constants as C
from .coulomb import _cells
from .philox import philox4x32_10, uniforms

TAG_ORDER = 25
TAG_EI0, TAG_EI1, TAG_EI2, TAG_EI3 = 26, 27, 28, 29
TAG_CX = 30
NEAR = 1e-6


class IonProcesses:
    def __init__(self, enabled=False, sigma_rec_1eV=1e-24, lotz_a2=4.5e-18,
                 I2_eV=20.29, cx_a=7.0710678118654755e-10, cx_b=0.0):
        self.enabled = bool(enabled)
        self.s_rec = float(sigma_rec_1eV)
        self.a2 = float(lotz_a2)
        self.I2 = float(I2_eV)
        self.cx_a = float(cx_a)
        self.cx_b = float(cx_b)

    def sigma_rec(self, E_eV):
        return self.s_rec * (1.0 / max(E_eV, 1e-3))

    def sigma_ion2(self, E_eV):
        if not E_eV > self.I2:
            return 0.0
        return (self.a2 * np.log(E_eV / self.I2)) / (E_eV * self.I2)

    def sigma_cx(self, eps_eV):
        t = self.cx_a - self.cx_b * np.log(max(eps_eV, 1e-6))
        t = max(t, 0.0)
        return t * t


def order_key(ids, step, seed):
    ids = np.asarray(ids, dtype=np.uint64)
    seed = int(seed)
    w = philox4x32_10(ids & np.uint64(0xFFFFFFFF), ids >> np.uint64(32),
                      np.uint64(step & 0xFFFFFFFF), np.uint64(TAG_ORDER),
                      np.uint64(seed & 0xFFFFFFFF),
                      np.uint64((seed >> 32) & 0xFFFFFFFF))
    return ((w[0].astype(np.uint64) << np.uint64(21))
            ^ (w[1].astype(np.uint64) >> np.uint64(11)))


def _groups(sp, grid, step, seed):
    if sp["x"].size == 0:
        return {}
    cell = _cells(sp, grid)
    key = order_key(sp["id"], step, seed)
    o = np.lexsort((sp["id"], key, cell))
    cs = cell[o]
    starts = np.r_[0, np.nonzero(np.diff(cs))[0] + 1]
    ends = np.r_[starts[1:], cs.size]
    return {int(cs[a]): o[a:b] for a, b in zip(starts, ends)}


def _u(sp, i):
    return sp["vx"][i], sp["vy"][i], sp["vz"][i]


def _isotropic(uc, up):
    c = 1.0 - 2.0 * uc
    s = np.sqrt(1.0 - c * c)
    ps = C.TWO_PI * up
    return s * np.cos(ps), s * np.sin(ps), c


def _take(sp, keep):
    return {k: v[keep] for k, v in sp.items()}


def _append(sp, rows):
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        sp[k] = np.concatenate([sp[k], np.array([r[k] for r in rows],
                                                dtype=np.float64)])
    sp["id"] = np.concatenate([sp["id"], np.array([r["id"] for r in rows],
                                                  dtype=np.uint64)])


def ion_processes(state, params, dt, near, diag):
    """Apply one step of recombination, Cu+ ionisation and charge exchange
    in place; fills diag (recombinations, ionisations2, charge_exchanges,
    f3_starved) and near["f3"]."""
    for k in ("recombinations", "ionisations2", "charge_exchanges",
              "f3_starved"):
        diag[k] = 0
    near.setdefault("f3", 0)
    cfg = params.get("ion_processes") or {}
    proc = IonProcesses(**cfg)
    if not proc.enabled:
        return
    g = state.grid
    step, seed = state.step, state.seed
    w_dx3 = float(state.w_sp) * ((g.inv_dx * g.inv_dx) * g.inv_dx)
    el, io, nu = (state.sp[C.ELECTRON], state.sp[C.ION], state.sp[C.NEUTRAL])
    ge = _groups(el, g, step, seed)
    gi = _groups(io, g, step, seed)
    gn = _groups(nu, g, step, seed)
    dead_e = np.zeros(el["x"].size, dtype=bool)
    dead_i = np.zeros(io["x"].size, dtype=bool)
    new_n, ion2_events = [], []
    M, m = C.M_CU, C.M_E
    # A. electrons on Cu+.
    for cell, ie in ge.items():
        ii = gi.get(cell)
        if ii is None:
            continue
        Ni = ii.size
        ni = float(Ni) * w_dx3
        r = 0
        for e in ie:
            vx, vy, vz = _u(el, e)
            v2 = (vx * vx + vy * vy) + vz * vz
            v = np.sqrt(v2)
            E = ((0.5 * C.M_E) * v2) / C.E_CHARGE
            s_rec, s_i2 = proc.sigma_rec(E), proc.sigma_ion2(E)
            s_tot = s_rec + s_i2
            P = 1.0 - np.exp(-(((ni * s_tot) * v) * dt))
            u1, u2 = uniforms(np.array([el["id"][e]]), step, TAG_EI0, seed)
            u1, u2 = u1[0], u2[0]
            frac = s_rec / s_tot
            if abs(u1 - P) < NEAR:
                near["f3"] += 1
            if not u1 < P:
                continue
            if r >= Ni:
                diag["f3_starved"] += 1
                continue
            if abs(u2 - frac) < NEAR:
                near["f3"] += 1
            i = ii[r]
            r += 1
            dead_i[i] = True
            if u2 < frac:
                dead_e[e] = True
                ivx, ivy, ivz = _u(io, i)
                den = M + m
                new_n.append(dict(x=io["x"][i], y=io["y"][i], z=io["z"][i],
                                  vx=(M * ivx + m * vx) / den,
                                  vy=(M * ivy + m * vy) / den,
                                  vz=(M * ivz + m * vz) / den,
                                  id=io["id"][i]))
                diag["recombinations"] += 1
            else:
                ion2_events.append((el["id"][e], e, i, E))
    # Ionisation of Cu+: kinematics, secondaries in primary-id order.
    ion2_events.sort(key=lambda t: int(t[0]))
    sec, ion2 = [], []
    for rank, (pid, e, i, E) in enumerate(ion2_events):
        u3, u4 = uniforms(np.array([pid]), step, TAG_EI1, seed)
        u5, u6 = uniforms(np.array([pid]), step, TAG_EI2, seed)
        u7, _ = uniforms(np.array([pid]), step, TAG_EI3, seed)
        avail = E - proc.I2
        Es = u3[0] * avail
        Ep = avail - Es
        k = (2.0 * C.E_CHARGE) / C.M_E
        vp = np.sqrt(Ep * k)
        vs = np.sqrt(Es * k)
        px, py, pz = _isotropic(u4[0], u5[0])
        sx, sy, sz = _isotropic(u6[0], u7[0])
        el["vx"][e], el["vy"][e], el["vz"][e] = vp * px, vp * py, vp * pz
        sec.append(dict(x=el["x"][e], y=el["y"][e], z=el["z"][e],
                        vx=vs * sx, vy=vs * sy, vz=vs * sz,
                        id=np.uint64(state.next_id + rank)))
        ion2.append({kk: io[kk][i] for kk in ("x", "y", "z", "vx", "vy",
                                                "vz", "id")})
    state.next_id += len(ion2_events)
    diag["ionisations2"] = len(ion2_events)
    # B. charge exchange of the Cu+ left with the atoms present before A.
    n_cx = 0
    for cell, ii in gi.items():
        jn = gn.get(cell)
        if jn is None:
            continue
        live = [i for i in ii if not dead_i[i]]
        Nn = jn.size
        nn = float(Nn) * w_dx3
        for k, i in enumerate(live):
            a = jn[k % Nn]
            ux = io["vx"][i] - nu["vx"][a]
            uy = io["vy"][i] - nu["vy"][a]
            uz = io["vz"][i] - nu["vz"][a]
            u2 = (ux * ux + uy * uy) + uz * uz
            u = np.sqrt(u2)
            mr = 0.5 * M
            eps = ((0.5 * mr) * u2) / C.E_CHARGE
            P = 1.0 - np.exp(-(((nn * proc.sigma_cx(eps)) * u) * dt))
            u1, _ = uniforms(np.array([io["id"][i]]), step, TAG_CX, seed)
            if abs(u1[0] - P) < NEAR:
                near["f3"] += 1
            if u1[0] < P:
                for kk in ("x", "y", "z", "vx", "vy", "vz", "id"):
                    io[kk][i], nu[kk][a] = nu[kk][a], io[kk][i]
                n_cx += 1
    diag["charge_exchanges"] = n_cx
    # Commit: removals and appends.
    state.sp[C.ELECTRON] = _take(el, ~dead_e)
    if sec:
        _append(state.sp[C.ELECTRON], sec)
    state.sp[C.ION] = _take(io, ~dead_i)
    if new_n:
        _append(state.sp[C.NEUTRAL], new_n)
    if ion2:
        _append(state.sp[C.ION2], ion2)
