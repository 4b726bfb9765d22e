"""One electrostatic PIC-MCC step, plain numpy float64.

Test infrastructure only (see the package docstring).

The step follows the paper's statement of the plasma model (superparticles
injected as emitted electrons and evaporated or sputtered neutrals; charge
density from electrons and ions feeding Poisson's equation, Eq. 1; motion
under electric forces; Monte Carlo collisions with probability
P = 1 - exp(-u n sigma(E) dt), Eq. 4, here in its null-collision form;
ions that reach the cathode handed back to the surface, Appendix A) and the
order of the FEM+PIC step in Appendix A: field and emission first, then push
and collisions.

Readings where the paper is silent (each is used identically by the HIP
library, which implements them independently):
  * Cloud-in-cell shape, per-axis weights quantised to 13 bits
    (fq = floor(frac * 8192 + 0.5)), charge summed in int64 units of
    2^-39 superparticle charges; the field is gathered with the same weights
    so a particle exerts no force on itself.
  * Cell coordinate g = x * (1/dx); x, y wrap once per step; z < 0 (g < 0)
    is absorbed at the cathode, g >= nz at the anode.
  * Non-relativistic leapfrog; a new particle's sampled velocity is taken as
    its half-step velocity.
  * Target density of Eq. 4: the number of neutrals in the electron's cell
    after the push, times the superparticle weight, over dx^3; relative speed
    u = electron speed (the target is at rest on the electron's scale).
  * Null-collision majorant g_max = (sigma_el + sigma_ion,max) v_max with
    v_max from E_max; process order ionisation, then elastic.
  * Ionisation cross section of Lotz form a ln(E/I)/(E I) (one subshell,
    q = 1), or a constant one for closed-form tests.
  * Ionisation: the energy above threshold is shared uniformly at random,
    both electrons leave isotropically; the neutral becomes the Cu+ ion with
    its own position, velocity and id; the secondary starts at the primary's
    position.  Within a cell, ionising electrons taken in increasing id order
    consume the cell's neutrals in increasing id order; an electron without a
    neutral left is a null event ("starved").  Secondaries get ids in
    increasing order of their primary's id.
  * Elastic: isotropic new direction, energy loss fraction
    (2 m_e / M)(1 - cos chi).
"""
import numpy as np

from . import constants as C
from .philox import uniforms
from .poisson import (DIRICHLET, NEUMANN, Grid, add_boundary_terms,
                      solve_exact)

QBITS = 8192                      # 13-bit quantisation of CIC weights
QSCALE = 2.0 ** -39               # (2^13)^3 weight product -> fraction
NEAR = 1e-6                       # near-threshold window for draws

TAG_MCC0, TAG_MCC1, TAG_MCC2, TAG_MCC3 = 0, 1, 2, 3
TAG_SRC0, TAG_SRC1, TAG_SRC2 = 8, 9, 10
TAG_FN = 12
FN_NODE_BIT = np.uint64(1) << np.uint64(63)


# --------------------------------------------------------------------------
# State
# --------------------------------------------------------------------------
def empty_species():
    z = np.zeros(0, dtype=np.float64)
    return dict(x=z.copy(), y=z.copy(), z=z.copy(), vx=z.copy(), vy=z.copy(),
                vz=z.copy(), id=np.zeros(0, dtype=np.uint64))


class State:
    """Particles (three species), clock, id counter and injection queue."""

    def __init__(self, grid, seed=0, w_sp=1):
        self.grid = grid
        self.seed = int(seed)
        self.w_sp = int(w_sp)
        self.sp = [empty_species() for _ in range(C.NSPECIES)]
        self.step = 0
        self.next_id = 0
        self.queue = []                 # (species, pos (n,3), vel (n,3))
        self.phi = None                 # last potential (warm start)

    def load(self, species, pos, vel, ids):
        """Replace a species' population (arrays copied)."""
        pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
        vel = np.asarray(vel, dtype=np.float64).reshape(-1, 3)
        self.sp[species] = dict(
            x=pos[:, 0].copy(), y=pos[:, 1].copy(), z=pos[:, 2].copy(),
            vx=vel[:, 0].copy(), vy=vel[:, 1].copy(), vz=vel[:, 2].copy(),
            id=np.asarray(ids, dtype=np.uint64).copy())

    def inject(self, species, pos, vel):
        """Queue caller particles; they receive ids at the next step."""
        self.queue.append((int(species),
                           np.asarray(pos, dtype=np.float64).reshape(-1, 3),
                           np.asarray(vel, dtype=np.float64).reshape(-1, 3)))

    def count(self, species):
        return int(self.sp[species]["x"].size)


def _append(sp, x, y, z, vx, vy, vz, ids):
    for key, val in (("x", x), ("y", y), ("z", z), ("vx", vx), ("vy", vy),
                     ("vz", vz)):
        sp[key] = np.concatenate([sp[key], np.asarray(val, np.float64)])
    sp["id"] = np.concatenate([sp["id"], np.asarray(ids, np.uint64)])


def _select(sp, keep):
    return {k: v[keep] for k, v in sp.items()}


# --------------------------------------------------------------------------
# Cloud-in-cell weights
# --------------------------------------------------------------------------
def cic_axis(coord, inv_dx):
    """Cell index (floor of coord/dx) and the quantised upper weight fq."""
    g = coord * inv_dx
    i = np.floor(g)
    f = g - i
    fq = np.floor(f * float(QBITS) + 0.5).astype(np.int64)
    return i.astype(np.int64), fq


def deposit(state):
    """int64 node charges: sum over charged particles of s * Wa * Wb * Wc.

    One unit is 2^-39 of a superparticle's charge (times w_sp, applied in the
    right-hand side).  Sum over all nodes =
    2^39 * (N_ion + 2 N_ion2 - N_electron).
    """
    g = state.grid
    acc = np.zeros(g.shape, dtype=np.int64)
    flat = acc.reshape(-1)
    for s, sign in ((C.ELECTRON, -1), (C.ION, +1), (C.ION2, +2)):
        sp = state.sp[s]
        if sp["x"].size == 0:
            continue
        ix, fx = cic_axis(sp["x"], g.inv_dx)
        iy, fy = cic_axis(sp["y"], g.inv_dx)
        iz, fz = cic_axis(sp["z"], g.inv_dx)
        wx = (QBITS - fx, fx)
        wy = (QBITS - fy, fy)
        wz = (QBITS - fz, fz)
        for c in (0, 1):
            for b in (0, 1):
                for a in (0, 1):
                    node = (((iz + c) * g.ny + (iy + b) % g.ny) * g.nx
                            + (ix + a) % g.nx)
                    np.add.at(flat, node, sign * (wx[a] * wy[b] * wz[c]))
    return acc


# --------------------------------------------------------------------------
# Field: right-hand side, Poisson, E
# --------------------------------------------------------------------------
def charge_scale(grid, w_sp):
    """c_rho: b = acc * c_rho, i.e. dx^2 rho/eps0 for one 2^-39 unit."""
    return ((float(w_sp) * C.E_CHARGE) * QSCALE) / (C.EPS0 * grid.dx)


def rhs(acc, grid, w_sp):
    """Scaled right-hand side b of A phi = b from the int64 node charges.

    A Neumann face node owns half a cell, so its density is doubled.
    """
    b = acc.astype(np.float64) * charge_scale(grid, w_sp)
    if grid.bc_lo == NEUMANN:
        b[0] = b[0] * 2.0
    if grid.bc_hi == NEUMANN:
        b[grid.nz] = b[grid.nz] * 2.0
    return add_boundary_terms(b, grid)


def efield(phi, grid):
    """E = -grad(phi) at nodes, shape grid.shape + (3,).

    Central differences in x, y (periodic) and inside in z; second-order
    one-sided differences on the two z faces.
    """
    h = 0.5 * grid.inv_dx
    nz = grid.nz
    E = np.empty(grid.shape + (3,), dtype=np.float64)
    E[..., 0] = (np.roll(phi, 1, axis=2) - np.roll(phi, -1, axis=2)) * h
    E[..., 1] = (np.roll(phi, 1, axis=1) - np.roll(phi, -1, axis=1)) * h
    E[1:nz, :, :, 2] = (phi[0:nz - 1] - phi[2:nz + 1]) * h
    E[0, :, :, 2] = ((3.0 * phi[0] - 4.0 * phi[1]) + phi[2]) * h
    E[nz, :, :, 2] = ((-3.0 * phi[nz] + 4.0 * phi[nz - 1]) - phi[nz - 2]) * h
    return E


def field_energy(acc, phi, grid, w_sp):
    """Electrostatic energy 1/2 sum_n q_n phi_n, J."""
    q = acc.astype(np.float64) * ((float(w_sp) * C.E_CHARGE) * QSCALE)
    return 0.5 * float(np.sum(q * phi))


def solve_field(state, params):
    """Deposit -> b -> exact phi -> E.  Returns (acc, b, phi, E)."""
    g = state.grid
    acc = deposit(state)
    if params.get("field_solve", 1):
        b = rhs(acc, g, state.w_sp)
    else:
        b = add_boundary_terms(np.zeros(g.shape), g)
    phi = solve_exact(b, g)
    return acc, b, phi, efield(phi, g)


# --------------------------------------------------------------------------
# Sources
# --------------------------------------------------------------------------
def _wrap(v, length):
    v = np.where(v < 0.0, v + length, v)
    return np.where(v >= length, v - length, v)


def _flux_vz(u, vth2):
    """Flux-weighted half-Maxwellian normal speed, vth2 = kT/m."""
    return np.sqrt((-2.0 * vth2) * np.log(1.0 - u))


def _disk_positions(ids, step, seed, cx, cy, radius, grid):
    u1, u2 = uniforms(ids, step, TAG_SRC0, seed)
    r = radius * np.sqrt(u1)
    th = C.TWO_PI * u2
    x = _wrap(cx + r * np.cos(th), grid.lx)
    y = _wrap(cy + r * np.sin(th), grid.ly)
    return x, y, np.zeros_like(x)


def fn_current_density(F, phi_w_eV):
    """Elementary Fowler-Nordheim current density, A/m^2.

    J = (a/phi) F^2 exp(-b phi^(3/2) / F) with a = e^3/(8 pi h) and
    b = 8 pi sqrt(2 m_e) / (3 e h) in SI (phi in J, F in V/m); F <= 0 gives 0.
    """
    phi_j = phi_w_eV * C.E_CHARGE
    a_fn = (C.E_CHARGE ** 3) / (8.0 * np.pi * C.H_PLANCK)
    b_fn = (8.0 * np.pi * np.sqrt(2.0 * C.M_E)) / (3.0 * C.E_CHARGE
                                                   * C.H_PLANCK)
    a_phi = a_fn / phi_j
    b_phi = b_fn * phi_j * np.sqrt(phi_j)
    F = np.asarray(F, dtype=np.float64)
    Fp = np.where(F > 0.0, F, 1.0)
    J = ((a_phi * Fp) * Fp) * np.exp(-(b_phi / Fp))
    return np.where(F > 0.0, J, 0.0)


def sources(state, params, E, dt, near):
    """New particles of this step, with ids next_id + rank in fixed order:
    injection queue (call order), disk electrons, disk neutrals, sphere
    neutrals, Fowler-Nordheim electrons (node order, last because only
    their number depends on the field).

    Returns per-species lists of (x, y, z, vx, vy, vz, ids) and the number of
    emitted electrons by source.
    """
    g = state.grid
    step, seed = state.step, state.seed
    new = {s: [] for s in range(C.NSPECIES)}
    nid = state.next_id

    def take(n):
        nonlocal nid
        ids = np.arange(nid, nid + n, dtype=np.uint64)
        nid += n
        return ids

    for s, pos, vel in state.queue:
        ids = take(pos.shape[0])
        new[s].append((pos[:, 0], pos[:, 1], pos[:, 2],
                       vel[:, 0], vel[:, 1], vel[:, 2], ids))
    state.queue = []

    src = params.get("sources", {})
    disk = src.get("disk")
    if disk:
        cx, cy, rad = disk["cx"], disk["cy"], disk["radius"]
        ne = int(disk.get("n_e", 0))
        if ne:
            ids = take(ne)
            x, y, z = _disk_positions(ids, step, seed, cx, cy, rad, g)
            vth2 = (disk["kT_e_eV"] * C.E_CHARGE) / C.M_E
            u3, _ = uniforms(ids, step, TAG_SRC1, seed)
            vz = _flux_vz(u3, vth2)
            zero = np.zeros(ne)
            new[C.ELECTRON].append((x, y, z, zero, zero.copy(), vz, ids))
        nn = int(disk.get("n_n", 0))
        if nn:
            ids = take(nn)
            x, y, z = _disk_positions(ids, step, seed, cx, cy, rad, g)
            vth2 = (C.K_B * disk["T_n_K"]) / C.M_CU
            u3, u4 = uniforms(ids, step, TAG_SRC1, seed)
            rr = np.sqrt((-2.0 * vth2) * np.log(1.0 - u3))
            th = C.TWO_PI * u4
            u5, _ = uniforms(ids, step, TAG_SRC2, seed)
            new[C.NEUTRAL].append((x, y, z, rr * np.cos(th), rr * np.sin(th),
                                   _flux_vz(u5, vth2), ids))

    sph = src.get("sphere")
    if sph and int(sph.get("n", 0)):
        n = int(sph["n"])
        ids = take(n)
        u1, u2 = uniforms(ids, step, TAG_SRC0, seed)
        c = 1.0 - 2.0 * u1
        s = np.sqrt(1.0 - c * c)
        ps = C.TWO_PI * u2
        nx_, ny_, nz_ = s * np.cos(ps), s * np.sin(ps), c
        x = _wrap(sph["cx"] + sph["radius"] * nx_, g.lx)
        y = _wrap(sph["cy"] + sph["radius"] * ny_, g.ly)
        z = sph["cz"] + sph["radius"] * nz_
        sig = np.sqrt((C.K_B * sph["T_K"]) / C.M_CU)
        u3, u4 = uniforms(ids, step, TAG_SRC1, seed)
        rr = np.sqrt(-2.0 * np.log(1.0 - u3))
        g1, g2 = rr * np.cos(C.TWO_PI * u4), rr * np.sin(C.TWO_PI * u4)
        u5, u6 = uniforms(ids, step, TAG_SRC2, seed)
        g3 = np.sqrt(-2.0 * np.log(1.0 - u5)) * np.cos(C.TWO_PI * u6)
        vx, vy, vz = sig * g1, sig * g2, sig * g3
        vn = (vx * nx_ + vy * ny_) + vz * nz_
        inward = vn < 0.0
        t = 2.0 * vn
        vx = np.where(inward, vx - t * nx_, vx)
        vy = np.where(inward, vy - t * ny_, vy)
        vz = np.where(inward, vz - t * nz_, vz)
        new[C.NEUTRAL].append((x, y, z, vx, vy, vz, ids))

    n_fn = 0
    fn = src.get("fn")
    if fn:
        i = np.arange(g.nx)
        j = np.arange(g.ny)
        xi = i.astype(np.float64) * g.dx
        yj = j.astype(np.float64) * g.dx
        ddx = (xi - fn["cx"])[None, :]
        ddy = (yj - fn["cy"])[:, None]
        inside = (ddx * ddx + ddy * ddy) <= fn["radius"] * fn["radius"]
        nodes = np.nonzero(inside.reshape(-1))[0].astype(np.uint64)
        F = -E[0, :, :, 2].reshape(-1)[nodes.astype(np.int64)]
        J = fn_current_density(F, fn["phi_w_eV"])
        c_fn = ((g.dx * g.dx) * dt) / C.E_CHARGE
        mean = J * c_fn
        fl = np.floor(mean)
        u, _ = uniforms(nodes | FN_NODE_BIT, step, TAG_FN, seed)
        frac = mean - fl
        near["fn"] += int(np.count_nonzero(np.abs(u - frac) < NEAR))
        cnt = fl.astype(np.int64) + (u < frac).astype(np.int64)
        n_fn = int(cnt.sum())
        if n_fn:
            ids = take(n_fn)
            node_of = np.repeat(nodes.astype(np.int64), cnt)
            u1, u2 = uniforms(ids, step, TAG_SRC0, seed)
            x = _wrap((node_of % g.nx).astype(np.float64) * g.dx
                      + (u1 - 0.5) * g.dx, g.lx)
            y = _wrap((node_of // g.nx).astype(np.float64) * g.dx
                      + (u2 - 0.5) * g.dx, g.ly)
            vth2 = (fn["kT_e_eV"] * C.E_CHARGE) / C.M_E
            u3, _ = uniforms(ids, step, TAG_SRC1, seed)
            zero = np.zeros(n_fn)
            new[C.ELECTRON].append((x, y, zero, zero.copy(), zero.copy(),
                                    _flux_vz(u3, vth2), ids))

    state.next_id = nid
    return new, n_fn


# --------------------------------------------------------------------------
# Push
# --------------------------------------------------------------------------
def gather(sp, E, grid):
    """CIC field at particles with the deposit's quantised weights.

    Accumulated in the fixed order z-corner, y-corner, x-corner (0 then 1).
    """
    ix, fx = cic_axis(sp["x"], grid.inv_dx)
    iy, fy = cic_axis(sp["y"], grid.inv_dx)
    iz, fz = cic_axis(sp["z"], grid.inv_dx)
    wx = (QBITS - fx, fx)
    wy = (QBITS - fy, fy)
    wz = (QBITS - fz, fz)
    Ef = E.reshape(-1, 3)
    ex = np.zeros(sp["x"].size)
    ey = np.zeros(sp["x"].size)
    ez = np.zeros(sp["x"].size)
    for c in (0, 1):
        for b in (0, 1):
            for a in (0, 1):
                node = (((iz + c) * grid.ny + (iy + b) % grid.ny) * grid.nx
                        + (ix + a) % grid.nx)
                w = (wx[a] * wy[b] * wz[c]).astype(np.float64) * QSCALE
                e = Ef[node]
                ex = ex + w * e[:, 0]
                ey = ey + w * e[:, 1]
                ez = ez + w * e[:, 2]
    return ex, ey, ez


def qm_dt(species, dt):
    q = C.CHARGE_SIGN[species] * C.E_CHARGE
    return (q / C.MASS[species]) * dt


def sphere_hit(x0, y0, z0, vx, vy, vz, dt, sph, grid):
    """Does the straight path x0 + v t, 0 <= t <= dt, of a particle touch
    the closed ball of a nanoparticle (Appendix A: electrons that hit an NP
    heat it)?  x and y use the nearest periodic image of the centre.

    With d = x0 - c and s = v dt the path is d + tau s, tau in [0, 1]; it
    touches the ball if it starts inside (|d|^2 <= R^2), or moves towards
    the centre (d.s < 0) with a real root of |d + tau s|^2 = R^2 whose
    smaller value tau_in = (-(d.s) - sqrt((d.s)^2 - |s|^2 (|d|^2 - R^2)))
    / |s|^2 is at most 1.
    """
    dxx = x0 - sph["cx"]
    dyy = y0 - sph["cy"]
    hx, hy = 0.5 * grid.lx, 0.5 * grid.ly
    dxx = np.where(dxx > hx, dxx - grid.lx, np.where(dxx < -hx, dxx + grid.lx, dxx))
    dyy = np.where(dyy > hy, dyy - grid.ly, np.where(dyy < -hy, dyy + grid.ly, dyy))
    dzz = z0 - sph["cz"]
    sx, sy, sz = vx * dt, vy * dt, vz * dt
    r2 = sph["radius"] * sph["radius"]
    c0 = ((dxx * dxx + dyy * dyy) + dzz * dzz) - r2
    b = (dxx * sx + dyy * sy) + dzz * sz
    a = (sx * sx + sy * sy) + sz * sz
    disc = b * b - a * c0
    with np.errstate(invalid="ignore", divide="ignore"):
        tau = (-b - np.sqrt(np.where(disc >= 0.0, disc, 0.0))) / np.where(
            a > 0.0, a, 1.0)
    moving_in = (b < 0.0) & (disc >= 0.0) & (a > 0.0) & (tau <= 1.0)
    return (c0 <= 0.0) | moving_in


def alpha_eh(R, d, ell, phi_w_eV, E_e_eV):
    """Electron energy-loss fraction of a nanoparticle (Appendix A, NP
    electron heating): not reflected (1 - R), stopped inside the particle
    (1 - exp(-d / ell), the complement of passing through it within an
    inelastic mean free path), and leaving with the work function
    (1 - phi / E_e).  The paper prints the middle factor as exp(-d/ell) but
    evaluates it as 0.76 = 1 - exp(-1 nm / 0.7 nm); this reading follows
    the value."""
    return (1.0 - R) * (1.0 - np.exp(-d / ell)) * (1.0 - phi_w_eV / E_e_eV)


def md_return(ab, lattice_a, grid=None, species=(C.ION,)):
    """Atoms handed back to MD from the cathode-absorbed list (Appendix A,
    transfer of bombarding ions): each selected particle's crossing point
    offset backwards along its velocity by three lattice constants,
    x_MD = x_c - 3 a v / |v| (x, y wrapped into the periodic box when grid
    is given), with its velocity and id, in the list's (species, id)
    order."""
    sel = np.isin(ab["species"], np.asarray(species))
    vx, vy, vz = ab["vx"][sel], ab["vy"][sel], ab["vz"][sel]
    inv = 1.0 / np.sqrt((vx * vx + vy * vy) + vz * vz)
    off = (3.0 * lattice_a) * inv
    x = ab["x"][sel] - off * vx
    y = ab["y"][sel] - off * vy
    if grid is not None:
        x, y = _wrap(x, grid.lx), _wrap(y, grid.ly)
    return dict(species=ab["species"][sel], id=ab["id"][sel], x=x, y=y,
                z=ab["z"][sel] - off * vz, vx=vx.copy(), vy=vy.copy(),
                vz=vz.copy())


def push(sp, species, E, grid, dt, sphere=None):
    """Leapfrog push of one species in place; returns (cathode, anode)
    masks and the cathode crossing points (x, y) of absorbed particles.
    With sphere (an electron-absorbing nanoparticle, electrons only) the
    returned cathode and anode masks exclude the electrons whose path
    touched the ball, and sp gains the mask "np_hit" of them (they are
    removed like the absorbed ones; the ball lies inside the domain, so a
    straight path that leaves through a face cannot meet it afterwards).
    """
    if species != C.NEUTRAL and sp["x"].size:
        ex, ey, ez = gather(sp, E, grid)
        k = qm_dt(species, dt)
        sp["vx"] = sp["vx"] + k * ex
        sp["vy"] = sp["vy"] + k * ey
        sp["vz"] = sp["vz"] + k * ez
    x0, y0, z0 = sp["x"], sp["y"], sp["z"]
    x = sp["x"] + sp["vx"] * dt
    y = sp["y"] + sp["vy"] * dt
    z = sp["z"] + sp["vz"] * dt
    gz = z * grid.inv_dx
    cath = gz < 0.0
    anode = gz >= float(grid.nz)
    if sphere is not None and species == C.ELECTRON:
        hit = sphere_hit(x0, y0, z0, sp["vx"], sp["vy"], sp["vz"], dt,
                         sphere, grid)
        cath = cath & ~hit
        anode = anode & ~hit
        sp["np_hit"] = hit
    with np.errstate(divide="ignore", invalid="ignore"):
        tc = np.where(cath, -z / np.where(cath, sp["vz"], 1.0), 0.0)
    xc = _wrap(x + sp["vx"] * tc, grid.lx)
    yc = _wrap(y + sp["vy"] * tc, grid.ly)
    sp["x"] = _wrap(x, grid.lx)
    sp["y"] = _wrap(y, grid.ly)
    sp["z"] = z
    return cath, anode, xc, yc


def cell_index(sp, grid):
    """Linear index (k*ny + j)*nx + i of the cell holding each particle."""
    i = np.floor(sp["x"] * grid.inv_dx).astype(np.int64) % grid.nx
    j = np.floor(sp["y"] * grid.inv_dx).astype(np.int64) % grid.ny
    k = np.floor(sp["z"] * grid.inv_dx).astype(np.int64)
    return (k * grid.ny + j) * grid.nx + i


# --------------------------------------------------------------------------
# Collisions
# --------------------------------------------------------------------------
class Collisions:
    """Cross sections and the null-collision majorant (host constants)."""

    def __init__(self, sigma_el=1e-19, ion_model="lotz", lotz_a=4.5e-18,
                 ion_I_eV=7.73, sigma_ion_const=0.0, E_max_eV=612.0,
                 enabled=True):
        self.sigma_el = float(sigma_el)
        self.ion_model = ion_model
        self.lotz_a = float(lotz_a)       # m^2 eV^2
        self.I = float(ion_I_eV)
        self.sigma_ion_const = float(sigma_ion_const)
        self.E_max = float(E_max_eV)
        self.enabled = bool(enabled)
        if ion_model == "lotz":
            self.sigma_ion_max = self.lotz_a / (C.E_EULER * self.I * self.I)
        else:
            self.sigma_ion_max = self.sigma_ion_const
        self.v_max = np.sqrt((2.0 * (self.E_max * C.E_CHARGE)) / C.M_E)
        self.g_max = (self.sigma_el + self.sigma_ion_max) * self.v_max
        self.inv_gmax = 1.0 / self.g_max if self.g_max > 0 else 0.0

    def sigma_ion(self, E_eV):
        """Ionisation cross section, m^2 (zero at or below threshold)."""
        E_eV = np.asarray(E_eV, dtype=np.float64)
        above = E_eV > self.I
        if self.ion_model == "lotz":
            Es = np.where(above, E_eV, 2.0 * self.I)
            s = (self.lotz_a * np.log(Es / self.I)) / (Es * self.I)
        else:
            s = np.full(E_eV.shape, self.sigma_ion_const)
        return np.where(above, s, 0.0)


def isotropic(u_c, u_psi):
    c = 1.0 - 2.0 * u_c
    s = np.sqrt(1.0 - c * c)
    ps = C.TWO_PI * u_psi
    return s * np.cos(ps), s * np.sin(ps), c


def mcc(state, coll, ncount, dt, near, diag):
    """Null-collision MCC of electrons against the per-cell neutral counts.

    Elastic collisions are applied in place.  Returns the ionisation events
    (electron indices) in arbitrary order; their kinematics are applied after
    target matching.
    """
    g = state.grid
    el = state.sp[C.ELECTRON]
    n = el["x"].size
    if n == 0 or not coll.enabled or coll.g_max <= 0:
        return np.zeros(0, dtype=np.int64), np.zeros(0, dtype=np.int64)
    cell = cell_index(el, g)
    nc = ncount[cell]
    inv_dx3 = (g.inv_dx * g.inv_dx) * g.inv_dx
    c_coll = ((coll.g_max * dt) * float(state.w_sp)) * inv_dx3
    pstar = 1.0 - np.exp(-(nc.astype(np.float64) * c_coll))
    u1, u2 = uniforms(el["id"], state.step, TAG_MCC0, state.seed)
    has = nc > 0
    near["cand"] += int(np.count_nonzero(has & (np.abs(u1 - pstar) < NEAR)))
    cand = np.nonzero(has & (u1 < pstar))[0]
    diag["candidates"] = int(cand.size)
    vx, vy, vz = el["vx"][cand], el["vy"][cand], el["vz"][cand]
    v2 = (vx * vx + vy * vy) + vz * vz
    v = np.sqrt(v2)
    E_eV = ((0.5 * C.M_E) * v2) / C.E_CHARGE
    diag["over_majorant"] = int(np.count_nonzero(E_eV > coll.E_max))
    p_ion = (coll.sigma_ion(E_eV) * v) * coll.inv_gmax
    p_el = (coll.sigma_el * v) * coll.inv_gmax
    u2c = u2[cand]
    p_tot = p_ion + p_el
    near["proc"] += int(np.count_nonzero(
        ((p_ion > 0) & (np.abs(u2c - p_ion) < NEAR))
        | (np.abs(u2c - p_tot) < NEAR)))
    is_ion = u2c < p_ion
    is_el = (~is_ion) & (u2c < p_tot)
    # Elastic: isotropic new direction, energy loss (2m/M)(1 - cos chi).
    ei = cand[is_el]
    diag["elastic"] = int(ei.size)
    if ei.size:
        u3, u4 = uniforms(el["id"][ei], state.step, TAG_MCC1, state.seed)
        nx_, ny_, nz_ = isotropic(u3, u4)
        sv = v[is_el]
        cosx = ((el["vx"][ei] * nx_ + el["vy"][ei] * ny_)
                + el["vz"][ei] * nz_) / sv
        ratio = (2.0 * C.M_E) / C.M_CU
        fac = np.sqrt(1.0 - ratio * (1.0 - cosx))
        sp_new = sv * fac
        el["vx"][ei] = sp_new * nx_
        el["vy"][ei] = sp_new * ny_
        el["vz"][ei] = sp_new * nz_
    ion_idx = cand[is_ion]
    return ion_idx, cell[ion_idx]


def ionise(state, coll, ion_idx, ion_cell, ncell_neutral, diag):
    """Match ionisation events to neutrals and apply the kinematics.

    Returns (secondaries dict of arrays, consumed neutral mask,
    new ion arrays).
    """
    el = state.sp[C.ELECTRON]
    nu = state.sp[C.NEUTRAL]
    step, seed = state.step, state.seed
    consumed = np.zeros(nu["x"].size, dtype=bool)
    diag["ionisations"] = 0
    diag["starved"] = 0
    if ion_idx.size == 0:
        return None, consumed, None
    eid = el["id"][ion_idx]
    # Events ordered by (cell, electron id); rank within the cell.
    order = np.lexsort((eid, ion_cell))
    ev_idx, ev_cell = ion_idx[order], ion_cell[order]
    first = np.searchsorted(ev_cell, ev_cell, side="left")
    rank = np.arange(ev_cell.size) - first
    # Neutrals ordered by (cell, id).
    nord = np.lexsort((nu["id"], ncell_neutral))
    ncell_sorted = ncell_neutral[nord]
    lo = np.searchsorted(ncell_sorted, ev_cell, side="left")
    hi = np.searchsorted(ncell_sorted, ev_cell, side="right")
    ok = rank < (hi - lo)
    diag["starved"] = int(np.count_nonzero(~ok))
    ev_idx, lo, rank = ev_idx[ok], lo[ok], rank[ok]
    tgt = nord[lo + rank]
    # Successful events in increasing primary id order give secondary ids.
    porder = np.argsort(el["id"][ev_idx], kind="stable")
    ev_idx, tgt = ev_idx[porder], tgt[porder]
    n = ev_idx.size
    diag["ionisations"] = int(n)
    consumed[tgt] = True
    pid = el["id"][ev_idx]
    u3, u4 = uniforms(pid, step, TAG_MCC1, seed)
    u5, u6 = uniforms(pid, step, TAG_MCC2, seed)
    u7, _ = uniforms(pid, step, TAG_MCC3, seed)
    vx, vy, vz = el["vx"][ev_idx], el["vy"][ev_idx], el["vz"][ev_idx]
    v2 = (vx * vx + vy * vy) + vz * vz
    E_eV = ((0.5 * C.M_E) * v2) / C.E_CHARGE
    avail = E_eV - coll.I
    Es = u3 * avail
    Ep = avail - Es
    k = (2.0 * C.E_CHARGE) / C.M_E
    vp = np.sqrt(Ep * k)
    vs = np.sqrt(Es * k)
    px, py, pz = isotropic(u4, u5)
    sx, sy, sz = isotropic(u6, u7)
    el["vx"][ev_idx] = vp * px
    el["vy"][ev_idx] = vp * py
    el["vz"][ev_idx] = vp * pz
    sec_ids = np.arange(state.next_id, state.next_id + n, dtype=np.uint64)
    state.next_id += n
    sec = dict(x=el["x"][ev_idx].copy(), y=el["y"][ev_idx].copy(),
               z=el["z"][ev_idx].copy(), vx=vs * sx, vy=vs * sy, vz=vs * sz,
               id=sec_ids)
    ions = {key: nu[key][tgt].copy() for key in nu}
    return sec, consumed, ions


# --------------------------------------------------------------------------
# One step
# --------------------------------------------------------------------------
def kinetic_energy(sp, species):
    v2 = (sp["vx"] * sp["vx"] + sp["vy"] * sp["vy"]) + sp["vz"] * sp["vz"]
    return float(0.5 * C.MASS[species] * np.sum(v2))


def advance(state, params, E, dt, progress=None):
    """Everything after the field solve: sources, push, MCC, ionisation,
    compaction.  Returns (absorbed dict, diagnostics dict).  progress, if
    given, is called with a short label after each stage (long runs at full
    size report where they are).
    """
    def done(label):
        if progress is not None:
            progress(label)
    g = state.grid
    coll = params.get("collisions_obj")
    if coll is None:
        coll = Collisions(**params.get("collisions", {}))
    near = {"cand": 0, "proc": 0, "fn": 0}
    diag = {"candidates": 0, "elastic": 0, "ionisations": 0, "starved": 0,
            "over_majorant": 0}
    new, n_fn = sources(state, params, E, dt, near)
    done("sources")
    emitted = {s: 0 for s in range(C.NSPECIES)}
    for s in range(C.NSPECIES):
        for parts in new[s]:
            _append(state.sp[s], *parts)
            emitted[s] += parts[0].size
    absorbed = []
    anode = [0] * C.NSPECIES
    cath_count = [0] * C.NSPECIES
    ke = [0.0] * C.NSPECIES
    sph = params.get("sources", {}).get("sphere")
    absorber = sph if (sph and sph.get("absorb")) else None
    np_hits, np_heat = 0, 0.0
    for s in (C.NEUTRAL, C.ION, C.ION2, C.ELECTRON):
        sp = state.sp[s]
        cath, an, xc, yc = push(sp, s, E, g, dt, absorber)
        ke[s] = kinetic_energy(sp, s)
        hit = sp.pop("np_hit", None)
        if hit is None:
            hit = np.zeros(sp["x"].size, dtype=bool)
        elif np.any(hit):
            # Heat of the nanoparticle: alpha_EH E_e per electron, E_e the
            # kinetic energy of the half-step velocity it arrives with.
            v2 = ((sp["vx"][hit] * sp["vx"][hit] + sp["vy"][hit] * sp["vy"][hit])
                  + sp["vz"][hit] * sp["vz"][hit])
            np_hits = int(np.count_nonzero(hit))
            np_heat = float(absorber.get("alpha_eh", 0.5)
                            * np.sum((0.5 * C.M_E) * v2))
        if np.any(cath):
            absorbed.append(dict(species=np.full(int(cath.sum()), s),
                                 id=sp["id"][cath], x=xc[cath], y=yc[cath],
                                 z=np.zeros(int(cath.sum())),
                                 vx=sp["vx"][cath], vy=sp["vy"][cath],
                                 vz=sp["vz"][cath]))
        cath_count[s] = int(cath.sum())
        anode[s] = int(an.sum())
        state.sp[s] = _select(sp, ~(cath | an | hit))
        done(f"push of species {s}")
    ncell_neutral = cell_index(state.sp[C.NEUTRAL], g)
    ncount = np.bincount(ncell_neutral,
                         minlength=g.nx * g.ny * g.nz).astype(np.int64)
    ion_idx, ion_cell = mcc(state, coll, ncount, dt, near, diag)
    done("mcc")
    sec, consumed, ions = ionise(state, coll, ion_idx, ion_cell,
                                 ncell_neutral, diag)
    if sec is not None:
        _append(state.sp[C.ELECTRON], sec["x"], sec["y"], sec["z"],
                sec["vx"], sec["vy"], sec["vz"], sec["id"])
        _append(state.sp[C.ION], ions["x"], ions["y"], ions["z"],
                ions["vx"], ions["vy"], ions["vz"], ions["id"])
        state.sp[C.NEUTRAL] = _select(state.sp[C.NEUTRAL], ~consumed)
    # Coulomb collisions of the charged particles the step leaves.
    from .coulomb import coulomb
    diag["coulomb_like"], diag["coulomb_ei"] = coulomb(state, params, dt)
    # Recombination, ionisation of Cu+ and charge exchange.
    from .ionproc import ion_processes
    ion_processes(state, params, dt, near, diag)
    if absorbed:
        ab = {k: np.concatenate([a[k] for a in absorbed]) for k in absorbed[0]}
        order = np.lexsort((ab["id"], ab["species"]))
        ab = {k: v[order] for k, v in ab.items()}
    else:
        ab = dict(species=np.zeros(0, np.int64), id=np.zeros(0, np.uint64),
                  x=np.zeros(0), y=np.zeros(0), z=np.zeros(0),
                  vx=np.zeros(0), vy=np.zeros(0), vz=np.zeros(0))
    diag.update(near=near, emitted=emitted, fn_emitted=n_fn,
                cathode=cath_count, anode=anode, kinetic=ke,
                np_hits=np_hits, np_heat=np_heat,
                counts=[state.count(s) for s in range(C.NSPECIES)])
    state.step += 1
    return ab, diag


def step(state, params, dt):
    """One full PIC-MCC step.  Returns (absorbed, diagnostics, phi)."""
    acc, b, phi, E = solve_field(state, params)
    state.phi = phi
    ab, diag = advance(state, params, E, dt)
    diag["total_charge_units"] = int(acc.sum())
    diag["field_energy"] = field_energy(acc, phi, state.grid, state.w_sp)
    return ab, diag, phi


# --------------------------------------------------------------------------
# Resolution check against the Debye length
# --------------------------------------------------------------------------
def debye_check(state, block=1, alpha_D=0.5):
    """Debye length of the electrons and ions per block of block^3 cells
    and the mesh criterion the paper applies to its elements (Appendix A:
    maximum element size d_max = 3.4 lambda_D alpha_D, alpha_D = 0.5).

    Per block and charged species s with N_s >= 2 particles: density
    n_s = N_s w / (block dx)^3, temperature k T_s = m_s S_s / (3 (N_s - 1))
    with S_s the sum over the block's particles of |v - mean v|^2 (the
    unbiased variance of the three velocity components, drift removed), and
    1 / lambda_D^2 = sum_s n_s e^2 / (eps0 k T_s) over the species with
    N_s >= 2 and T_s > 0.  A block where no species qualifies has no Debye
    length (infinite: nothing to resolve).  The grid resolves a block when
    dx <= d_max.

    Returns dict(lambda_D (bz, by, bx) array, checked = blocks with a finite
    lambda_D, unresolved = of them with dx > d_max, lambda_min, ratio_max =
    largest dx / d_max).
    """
    g = state.grid
    if g.nx % block or g.ny % block or g.nz % block:
        raise ValueError("block must divide the grid")
    bx, by, bz = g.nx // block, g.ny // block, g.nz // block
    nb = bx * by * bz
    vol = (float(block) * g.dx) ** 3
    inv_l2 = np.zeros(nb)
    for s in (C.ELECTRON, C.ION):
        sp = state.sp[s]
        if sp["x"].size == 0:
            continue
        i = (np.floor(sp["x"] * g.inv_dx).astype(np.int64) % g.nx) // block
        j = (np.floor(sp["y"] * g.inv_dx).astype(np.int64) % g.ny) // block
        k = np.floor(sp["z"] * g.inv_dx).astype(np.int64) // block
        key = (k * by + j) * bx + i
        N = np.bincount(key, minlength=nb).astype(np.float64)
        Nq = np.where(N > 0, N, 1.0)
        ss = np.zeros(nb)
        for comp in ("vx", "vy", "vz"):
            mean = np.bincount(key, sp[comp], minlength=nb) / Nq
            dev = sp[comp] - mean[key]
            ss += np.bincount(key, dev * dev, minlength=nb)
        ok = N >= 2
        kT = np.where(ok, (C.MASS[s] * ss) / (3.0 * np.where(ok, N - 1.0, 1.0)),
                      0.0)
        n = (N * float(state.w_sp)) / vol
        use = ok & (kT > 0.0)
        term = np.where(use, (n * (C.E_CHARGE * C.E_CHARGE))
                        / (C.EPS0 * np.where(use, kT, 1.0)), 0.0)
        inv_l2 += term
    has = inv_l2 > 0.0
    lam = np.full(nb, np.inf)
    lam[has] = 1.0 / np.sqrt(inv_l2[has])
    dmax = (3.4 * alpha_D) * lam
    ratio = np.where(has, g.dx / dmax, 0.0)
    return dict(lambda_D=lam.reshape(bz, by, bx), checked=int(has.sum()),
                unresolved=int(np.count_nonzero(ratio > 1.0)),
                lambda_min=float(lam[has].min()) if has.any() else np.inf,
                ratio_max=float(ratio.max()) if nb else 0.0)
