"""Seeded synthetic workloads: run parameters and initial particle states.

This module is the only code that both the oracle's tests and the HIP path's
tests, benchmark and smoke check use.  It holds no arithmetic of the method:
only the parameter sets of the workloads and numpy-seeded generators of
initial particle populations (positions uniform in the box, Maxwellian
velocities), which are inputs to the step, not part of it.

Workloads (sizes in cells, dx in metres):
  c1  32x32x64, dx 4 nm, anode +256 V (1 GV/m), disk source of 100 electrons
      (0.5 eV) and 50 Cu neutrals (3000 K) per step, radius 10 nm, Lotz
      ionisation (I = 7.73 eV) and 1e-19 m^2 elastic, dt 5e-16 s, 200 steps.
  c2  128x128x512, dx 2 nm, anode +1024 V (1 GV/m), Fowler-Nordheim emission
      (4.5 eV) over a 20 nm disk, 1e5 Cu neutrals per step at 3000 K,
      dt 2e-16 s; preloaded with 10 M electrons (5 eV), 10 M Cu+ at the same
      positions and 5 M neutrals (3000 K), uniform over the box.
  c3  c1 in mixed precision (FP32 particles, FP32 multigrid smoothing with
      FP64 refinement, 4 levels).
  c5  256x256x1024, dx 2 nm, anode +2048 V, c1's surface source plus a 5 nm
      sphere at z = 200 nm emitting 2e5 Cu neutrals per step at 3500 K;
      preloaded with 40 M electrons, 40 M Cu+ and 20 M neutrals.
"""
import numpy as np

# Physical constants needed only to draw initial velocities (not used by the
# step).  CODATA 2022.
_E = 1.602176634e-19
_ME = 9.1093837139e-31
_KB = 1.380649e-23
_MCU = 63.546 * 1.66053906892e-27

ELECTRON, NEUTRAL, ION = 0, 1, 2


def _collisions(v_top):
    return dict(sigma_el=1e-19, ion_model="lotz", lotz_a=4.5e-18,
                ion_I_eV=7.73, sigma_ion_const=0.0,
                E_max_eV=2.0 * abs(v_top) + 100.0, enabled=True)


def config(name):
    """Parameter dict of a named workload."""
    if name in ("c1", "c3"):
        nx, ny, nz, dx, v = 32, 32, 64, 4e-9, 256.0
        p = dict(nx=nx, ny=ny, nz=nz, dx=dx, bc_lo=0, bc_hi=0, v_lo=0.0,
                 v_hi=v, seed=0, w_sp=1, dt=5e-16, steps=200,
                 field_solve=1, collisions=_collisions(v),
                 sources=dict(disk=dict(cx=nx * dx / 2, cy=ny * dx / 2,
                                        radius=10e-9, n_e=100, kT_e_eV=0.5,
                                        n_n=50, T_n_K=3000.0)),
                 precision="fp64" if name == "c1" else "mixed",
                 mg_levels=0 if name == "c1" else 4)
        return p
    if name == "c2":
        nx, ny, nz, dx, v = 128, 128, 512, 2e-9, 1024.0
        return dict(nx=nx, ny=ny, nz=nz, dx=dx, bc_lo=0, bc_hi=0, v_lo=0.0,
                    v_hi=v, seed=0, w_sp=1, dt=2e-16, steps=2000,
                    field_solve=1, collisions=_collisions(v),
                    sources=dict(
                        disk=dict(cx=nx * dx / 2, cy=ny * dx / 2,
                                  radius=20e-9, n_e=0, kT_e_eV=0.5,
                                  n_n=100000, T_n_K=3000.0),
                        fn=dict(cx=nx * dx / 2, cy=ny * dx / 2, radius=20e-9,
                                phi_w_eV=4.5, kT_e_eV=0.5)),
                    preload=dict(n_e=10_000_000, n_ion=10_000_000,
                                 n_n=5_000_000, kT_e_eV=5.0, T_K=3000.0),
                    precision="fp64", mg_levels=0)
    if name == "c5":
        nx, ny, nz, dx, v = 256, 256, 1024, 2e-9, 2048.0
        return dict(nx=nx, ny=ny, nz=nz, dx=dx, bc_lo=0, bc_hi=0, v_lo=0.0,
                    v_hi=v, seed=0, w_sp=1, dt=2e-16, steps=5000,
                    field_solve=1, collisions=_collisions(v),
                    sources=dict(
                        disk=dict(cx=nx * dx / 2, cy=ny * dx / 2,
                                  radius=10e-9, n_e=100, kT_e_eV=0.5,
                                  n_n=50, T_n_K=3000.0),
                        sphere=dict(cx=nx * dx / 2, cy=ny * dx / 2,
                                    cz=200e-9, radius=5e-9, n=200000,
                                    T_K=3500.0)),
                    preload=dict(n_e=40_000_000, n_ion=40_000_000,
                                 n_n=20_000_000, kT_e_eV=5.0, T_K=3000.0),
                    precision="mixed", mg_levels=0)
    raise KeyError(name)


def scaled(p, nx, ny, nz, n_e=None, n_ion=None, n_n=None):
    """Copy of a workload on a smaller grid (same dx, field, sources scaled
    to the grid) for tests the oracle finishes in seconds."""
    q = dict(p)
    field = p["v_hi"] / (p["nz"] * p["dx"])
    q.update(nx=nx, ny=ny, nz=nz, v_hi=field * nz * p["dx"])
    q["collisions"] = dict(p["collisions"])
    q["collisions"]["E_max_eV"] = 2.0 * abs(q["v_hi"]) + 100.0
    src = {}
    for k, s in p.get("sources", {}).items():
        s = dict(s)
        if "cx" in s:
            s["cx"], s["cy"] = nx * p["dx"] / 2, ny * p["dx"] / 2
        if k == "disk" and s.get("n_n", 0) > 1000:
            s["n_n"] = 200
        if k == "sphere":
            s["n"] = min(s["n"], 500)
            s["cz"] = min(s["cz"], 0.5 * nz * p["dx"])
        src[k] = s
    q["sources"] = src
    if "preload" in p:
        pl = dict(p["preload"])
        if n_e is not None:
            pl["n_e"] = n_e
        if n_ion is not None:
            pl["n_ion"] = n_ion
        if n_n is not None:
            pl["n_n"] = n_n
        q["preload"] = pl
    return q


def preload(p, seed=1234):
    """Initial populations: dict species -> (pos (n,3), vel (n,3), ids).

    Electrons: uniform in the box, isotropic Maxwellian at kT_e; Cu+ at the
    electrons' positions (zero net charge), Maxwellian at T; neutrals uniform,
    Maxwellian at T.  Ids run 0 .. N-1 over electrons, ions, neutrals.
    """
    pl = p["preload"]
    rng = np.random.default_rng(seed)
    L = np.array([p["nx"], p["ny"], p["nz"]], dtype=np.float64) * p["dx"]
    ne, ni, nn = int(pl["n_e"]), int(pl["n_ion"]), int(pl["n_n"])
    out = {}
    pos_e = rng.random((ne, 3)) * L
    sig_e = np.sqrt(pl["kT_e_eV"] * _E / _ME)
    out[ELECTRON] = (pos_e, rng.standard_normal((ne, 3)) * sig_e,
                     np.arange(0, ne, dtype=np.uint64))
    sig_i = np.sqrt(_KB * pl["T_K"] / _MCU)
    m = min(ni, ne)
    pos_i = np.concatenate([pos_e[:m], rng.random((ni - m, 3)) * L])
    out[ION] = (pos_i, rng.standard_normal((ni, 3)) * sig_i,
                np.arange(ne, ne + ni, dtype=np.uint64))
    out[NEUTRAL] = (rng.random((nn, 3)) * L,
                    rng.standard_normal((nn, 3)) * sig_i,
                    np.arange(ne + ni, ne + ni + nn, dtype=np.uint64))
    return out


def random_particles(n, p, seed, kT_eV=5.0, mass=_ME, z_margin=0.0,
                     id0=0):
    """n particles uniform in the box (z kept z_margin cells from the
    faces), Maxwellian velocities; for kernel-level tests."""
    rng = np.random.default_rng(seed)
    L = np.array([p["nx"], p["ny"], p["nz"]], dtype=np.float64) * p["dx"]
    pos = rng.random((n, 3)) * L
    if z_margin:
        lo = z_margin * p["dx"]
        pos[:, 2] = lo + rng.random(n) * (L[2] - 2 * lo)
    vel = rng.standard_normal((n, 3)) * np.sqrt(kT_eV * _E / mass)
    return pos, vel, np.arange(id0, id0 + n, dtype=np.uint64)


def edge_positions(p, seed):
    """Positions on nodes, cell centres, faces, the periodic seam and
    just inside the top face (edge cases of the weights)."""
    rng = np.random.default_rng(seed)
    dx = p["dx"]
    nx, ny, nz = p["nx"], p["ny"], p["nz"]
    pts = []
    for _ in range(64):
        i, j, k = rng.integers(0, nx), rng.integers(0, ny), rng.integers(0, nz)
        pts.append((i * dx, j * dx, k * dx))
        pts.append(((i + 0.5) * dx, (j + 0.5) * dx, (k + 0.5) * dx))
    # Largest z whose cell coordinate z * (1/dx) is still below nz.
    top = np.nextafter(nz * dx, 0.0)
    while top * (1.0 / dx) >= nz:
        top = np.nextafter(top, 0.0)
    pts += [(0.0, 0.0, 0.0), (np.nextafter(nx * dx, 0.0), 0.0, 0.0),
            (0.0, np.nextafter(ny * dx, 0.0), top),
            (np.nextafter(nx * dx, 0.0), np.nextafter(ny * dx, 0.0), top),
            ((nx - 0.5) * dx, (ny - 0.5) * dx, (nz - 0.5) * dx)]
    return np.array(pts, dtype=np.float64)


def unet_init(seed=0):
    """He-normal initial parameters of the warm-start U-Net (flat FP32
    vector in the documented layout); biases zero, head small."""
    layers = ((2, 16), (16, 16), (16, 32), (32, 32), (32, 64), (64, 64),
              (64, 128), (128, 128), (192, 64), (64, 64), (96, 32),
              (32, 32), (48, 16), (16, 16))
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co in layers:
        parts.append(rng.standard_normal(co * 27 * ci)
                     * np.sqrt(2.0 / (27 * ci)))
        parts.append(np.zeros(co))
    parts.append(rng.standard_normal(16) * 0.1)
    parts.append(np.zeros(1))
    return np.concatenate(parts).astype(np.float32)
