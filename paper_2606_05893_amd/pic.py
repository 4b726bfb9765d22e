"""Python binding of libpic.so (ctypes): argument marshalling only.

Every step of the PIC-MCC path runs in the HIP library; torch supplies the
device memory (the workspace and the tensors handed across the C ABI) and
the stream.  There is no fallback: if the library or a GPU is missing the
calls raise.
"""
import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpic.so")

ELECTRON, NEUTRAL, ION, ION2 = 0, 1, 2, 3
NSPECIES = 4
DIRICHLET, NEUMANN = 0, 1
FP64, MIXED = 0, 1
ION_LOTZ, ION_CONST = 0, 1
FLAG_PLAIN_SMOOTHER = 1
FLAG_MG_ALL_LEVELS = 2
FLAG_CELL_GROUPS = 4

STATUS = {0: "PIC_OK", -1: "PIC_ERR_ARG", -2: "PIC_ERR_CAPACITY",
          -3: "PIC_ERR_NOCONV", -4: "PIC_ERR_NONFINITE", -5: "PIC_ERR_HIP",
          -6: "PIC_ERR_STATE"}

_c_d = ctypes.c_double
_c_i32 = ctypes.c_int32
_c_i64 = ctypes.c_int64
_c_u32 = ctypes.c_uint32
_c_u64 = ctypes.c_uint64
_c_p = ctypes.c_void_p


class Config(ctypes.Structure):
    _fields_ = [("nx", _c_i32), ("ny", _c_i32), ("nz", _c_i32), ("dx", _c_d),
                ("bc_lo", _c_i32), ("bc_hi", _c_i32), ("v_lo", _c_d),
                ("v_hi", _c_d), ("precision", _c_i32),
                ("field_solve", _c_i32), ("mg_levels", _c_i32),
                ("max_vcycles", _c_i32), ("nu_pre", _c_i32),
                ("nu_post", _c_i32), ("coarse_sweeps", _c_i32),
                ("sort_every", _c_i32), ("rel_tol", _c_d), ("seed", _c_u64),
                ("w_sp", _c_u32), ("flags", _c_u32),
                ("capacity", _c_i64 * 4), ("queue_capacity", _c_i64),
                ("max_events", _c_i64)]


class Collisions(ctypes.Structure):
    _fields_ = [("enabled", _c_i32), ("ion_model", _c_i32),
                ("sigma_el", _c_d), ("lotz_a", _c_d), ("ion_I_eV", _c_d),
                ("sigma_ion_const", _c_d), ("E_max_eV", _c_d)]


class Sources(ctypes.Structure):
    _fields_ = [("disk_on", _c_i32), ("fn_on", _c_i32), ("sphere_on", _c_i32),
                ("sph_absorb", _c_i32), ("disk_cx", _c_d), ("disk_cy", _c_d),
                ("disk_radius", _c_d), ("disk_n_e", _c_i64),
                ("disk_kT_e_eV", _c_d), ("disk_n_n", _c_i64),
                ("disk_T_n_K", _c_d), ("fn_cx", _c_d), ("fn_cy", _c_d),
                ("fn_radius", _c_d), ("fn_phi_w_eV", _c_d),
                ("fn_kT_e_eV", _c_d), ("sph_cx", _c_d), ("sph_cy", _c_d),
                ("sph_cz", _c_d), ("sph_radius", _c_d), ("sph_n", _c_i64),
                ("sph_T_K", _c_d), ("sph_alpha_eh", _c_d)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("vcycles", _c_i32), ("converged", _c_i32),
                ("rel_residual", _c_d), ("b_norm", _c_d),
                ("rel_residual0", _c_d), ("warm_ratio", _c_d),
                ("warm_used", _c_i32), ("warm_rejected", _c_i32),
                ("refinements", _c_i32)]


class Diag(ctypes.Structure):
    _fields_ = [("counts", _c_i64 * 4), ("emitted", _c_i64 * 4),
                ("fn_emitted", _c_i64), ("cathode", _c_i64 * 4),
                ("anode", _c_i64 * 4), ("candidates", _c_i64),
                ("elastic", _c_i64), ("ionisations", _c_i64),
                ("starved", _c_i64), ("over_majorant", _c_i64),
                ("near_threshold", _c_i64), ("total_charge_units", _c_i64),
                ("kinetic", _c_d * 4), ("field_energy", _c_d),
                ("solve", SolveInfo), ("step", _c_i64), ("next_id", _c_u64),
                ("np_absorbed", _c_i64), ("np_heat", _c_d),
                ("coulomb_like", _c_i64), ("coulomb_ei", _c_i64),
                ("recombinations", _c_i64), ("ionisations2", _c_i64),
                ("charge_exchanges", _c_i64), ("ion_starved", _c_i64)]


class Coulomb(ctypes.Structure):
    _fields_ = [("enabled", _c_i32), ("reserved", _c_i32),
                ("ln_lambda", _c_d)]


class IonProcesses(ctypes.Structure):
    _fields_ = [("enabled", _c_i32), ("reserved", _c_i32),
                ("sigma_rec_1eV", _c_d), ("lotz_a2", _c_d),
                ("ion2_I_eV", _c_d), ("cx_a", _c_d), ("cx_b", _c_d)]


class DebyeInfo(ctypes.Structure):
    _fields_ = [("blocks", _c_i64), ("checked", _c_i64),
                ("unresolved", _c_i64), ("lambda_min", _c_d),
                ("ratio_max", _c_d)]


class Absorbed(ctypes.Structure):
    _fields_ = [("n", _c_i64), ("species", _c_p), ("id", _c_p),
                ("pos", _c_p), ("vel", _c_p)]


EXPORTS = {
    "pic_abi_version": (_c_i32, []),
    "pic_last_error": (ctypes.c_char_p, [_c_p]),
    "pic_workspace_bytes": (_c_i32, [ctypes.POINTER(Config),
                                     ctypes.POINTER(ctypes.c_size_t)]),
    "pic_init": (_c_i32, [ctypes.POINTER(Config), _c_p, ctypes.c_size_t, _c_p,
                          ctypes.POINTER(_c_p)]),
    "pic_destroy": (None, [_c_p]),
    "pic_set_collisions": (_c_i32, [_c_p, ctypes.POINTER(Collisions)]),
    "pic_set_sources": (_c_i32, [_c_p, ctypes.POINTER(Sources)]),
    "pic_inject": (_c_i32, [_c_p, _c_i32, _c_i64, _c_p, _c_p]),
    "pic_step": (_c_i32, [_c_p, _c_d, ctypes.POINTER(Absorbed),
                          ctypes.POINTER(Diag)]),
    "poisson_solve": (_c_i32, [_c_p, _c_p, _c_p, _c_i32,
                               ctypes.POINTER(SolveInfo)]),
    "pic_deposit": (_c_i32, [_c_p]),
    "pic_field": (_c_i32, [_c_p, ctypes.POINTER(SolveInfo)]),
    "pic_set_phi": (_c_i32, [_c_p, _c_p]),
    "pic_advance": (_c_i32, [_c_p, _c_d, ctypes.POINTER(Absorbed),
                             ctypes.POINTER(Diag)]),
    "pic_load_particles": (_c_i32, [_c_p, _c_i32, _c_i64, _c_p, _c_p, _c_p]),
    "pic_count": (_c_i32, [_c_p, _c_i32, ctypes.POINTER(_c_i64)]),
    "pic_read_particles": (_c_i32, [_c_p, _c_i32, _c_i64, _c_p, _c_p, _c_p,
                                    ctypes.POINTER(_c_i64)]),
    "pic_read_fields": (_c_i32, [_c_p, _c_p, _c_p, _c_p]),
    "pic_set_clock": (_c_i32, [_c_p, _c_i64, _c_u64]),
    "pic_get_diag": (_c_i32, [_c_p, ctypes.POINTER(Diag)]),
    "pic_set_warm_start": (_c_i32, [_c_p, _c_i32, _c_p]),
    "pic_checkpoint_bytes": (_c_i32, [_c_p, ctypes.POINTER(ctypes.c_size_t)]),
    "pic_checkpoint_save": (_c_i32, [_c_p, _c_p, ctypes.c_size_t]),
    "pic_checkpoint_load": (_c_i32, [_c_p, _c_p, ctypes.c_size_t]),
    "pic_warm_pair": (_c_i32, [_c_p, _c_p, _c_p]),
    "pic_enable_timing": (_c_i32, [_c_p, _c_i32]),
    "pic_phase_times": (_c_i32, [_c_p, ctypes.POINTER(_c_d),
                                 ctypes.POINTER(_c_i64)]),
    "pic_md_return": (_c_i32, [_c_p, _c_d, _c_u32, _c_i64, _c_p, _c_p, _c_p,
                               _c_p, ctypes.POINTER(_c_i64)]),
    "pic_alpha_eh": (_c_d, [_c_d, _c_d, _c_d, _c_d, _c_d]),
    "pic_set_coulomb": (_c_i32, [_c_p, ctypes.POINTER(Coulomb)]),
    "pic_set_ion_processes": (_c_i32, [_c_p, ctypes.POINTER(IonProcesses)]),
    "pic_debye_check": (_c_i32, [_c_p, _c_i32, _c_d, _c_p,
                                 ctypes.POINTER(DebyeInfo)]),
    "poisson_solve_static": (_c_i32, [ctypes.POINTER(Config), _c_p, _c_p,
                                      _c_i32, ctypes.POINTER(SolveInfo),
                                      _c_p]),
}

PHASES = ("deposit", "rhs", "poisson", "efield", "sources", "push_neutral",
          "push_ion", "push_electron", "collide", "absorbed", "bin", "warm",
          "smooth_l0", "debye", "coulomb", "ion_coll")
WARM_MODES = {"prev": 0, "record": 1, "unet": 2, "extrap": 3}

_lib = None


def load_library(path=LIB_PATH):
    """Load libpic.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} (run "
                           "__graft_entry__.build())")
    lib = ctypes.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class PicError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _soa(a, dtype=torch.float64):
    """(n, 3) -> contiguous (3, n) device tensor (x block, y, z)."""
    t = torch.as_tensor(a, dtype=dtype, device="cuda")
    return t.reshape(-1, 3).t().contiguous()


def make_config(p, capacity=(1 << 16,) * 3, queue_capacity=1 << 16,
                max_events=1 << 16, rel_tol=1e-10, max_vcycles=100,
                nu_pre=2, nu_post=2, coarse_sweeps=64, flags=0):
    c = Config()
    c.nx, c.ny, c.nz, c.dx = p["nx"], p["ny"], p["nz"], p["dx"]
    c.bc_lo, c.bc_hi = p.get("bc_lo", 0), p.get("bc_hi", 0)
    c.v_lo, c.v_hi = p.get("v_lo", 0.0), p.get("v_hi", 0.0)
    c.precision = MIXED if p.get("precision", "fp64") == "mixed" else FP64
    c.field_solve = int(p.get("field_solve", 1))
    c.mg_levels = int(p.get("mg_levels", 0))
    c.max_vcycles, c.nu_pre, c.nu_post = max_vcycles, nu_pre, nu_post
    c.coarse_sweeps, c.sort_every = coarse_sweeps, 1
    c.rel_tol = rel_tol
    c.seed = int(p.get("seed", 0))
    c.w_sp = int(p.get("w_sp", 1))
    c.flags = int(flags)
    # A fourth capacity (Cu2+) defaults to at most 65536.
    caps = list(capacity)
    if len(caps) == 3:
        caps.append(min(int(caps[2]), 1 << 16))
    for s in range(NSPECIES):
        c.capacity[s] = int(caps[s])
    c.queue_capacity, c.max_events = int(queue_capacity), int(max_events)
    return c


def make_collisions(d):
    k = Collisions()
    d = d or {}
    k.enabled = int(bool(d.get("enabled", False)))
    k.ion_model = ION_LOTZ if d.get("ion_model", "lotz") == "lotz" else ION_CONST
    k.sigma_el = d.get("sigma_el", 0.0)
    k.lotz_a = d.get("lotz_a", 0.0)
    k.ion_I_eV = d.get("ion_I_eV", 7.73)
    k.sigma_ion_const = d.get("sigma_ion_const", 0.0)
    k.E_max_eV = d.get("E_max_eV", 1.0)
    return k


def make_sources(d):
    s = Sources()
    d = d or {}
    if "disk" in d:
        q = d["disk"]
        s.disk_on = 1
        s.disk_cx, s.disk_cy, s.disk_radius = q["cx"], q["cy"], q["radius"]
        s.disk_n_e, s.disk_kT_e_eV = int(q.get("n_e", 0)), q.get("kT_e_eV", 0.5)
        s.disk_n_n, s.disk_T_n_K = int(q.get("n_n", 0)), q.get("T_n_K", 3000.0)
    if "fn" in d:
        q = d["fn"]
        s.fn_on = 1
        s.fn_cx, s.fn_cy, s.fn_radius = q["cx"], q["cy"], q["radius"]
        s.fn_phi_w_eV, s.fn_kT_e_eV = q["phi_w_eV"], q.get("kT_e_eV", 0.5)
    if "sphere" in d:
        q = d["sphere"]
        s.sphere_on = 1
        s.sph_cx, s.sph_cy, s.sph_cz = q["cx"], q["cy"], q["cz"]
        s.sph_radius, s.sph_n, s.sph_T_K = q["radius"], int(q["n"]), q["T_K"]
        s.sph_absorb = int(bool(q.get("absorb", False)))
        s.sph_alpha_eh = float(q.get("alpha_eh", 0.5))
    return s


class Pic:
    """One PIC-MCC context on the current torch device and stream."""

    def __init__(self, p, **kw):
        self.lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible")
        self.p = p
        self.cfg = make_config(p, **kw)
        nbytes = ctypes.c_size_t()
        self._check(self.lib.pic_workspace_bytes(ctypes.byref(self.cfg),
                                                 ctypes.byref(nbytes)), None)
        self.ws = torch.empty(nbytes.value + 256, dtype=torch.uint8,
                              device="cuda")
        base = (self.ws.data_ptr() + 255) // 256 * 256
        self.stream = torch.cuda.current_stream()
        ctx = ctypes.c_void_p()
        self._check(self.lib.pic_init(ctypes.byref(self.cfg),
                                      ctypes.c_void_p(base), nbytes.value,
                                      ctypes.c_void_p(self.stream.cuda_stream),
                                      ctypes.byref(ctx)), None)
        self.ctx = ctx
        self._keep = []
        self.grid_shape = (p["nz"] + 1, p["ny"], p["nx"])
        self.set_collisions(p.get("collisions"))
        self.set_sources(p.get("sources"))
        if p.get("coulomb"):
            self.set_coulomb(p["coulomb"])
        if p.get("ion_processes"):
            self.set_ion_processes(p["ion_processes"])

    def __del__(self):
        if getattr(self, "ctx", None) and self.lib is not None:
            self.lib.pic_destroy(self.ctx)
            self.ctx = None

    def _check(self, status, ctx):
        if status != 0:
            msg = (self.lib.pic_last_error(ctx) or b"").decode() if ctx else ""
            raise PicError(status, msg)

    def _call(self, name, *args):
        # Inputs prepared on the caller's current stream are complete before
        # the context's stream reads them.
        cur = torch.cuda.current_stream()
        if cur != self.stream:
            self.stream.wait_stream(cur)
        self._check(getattr(self.lib, name)(self.ctx, *args), self.ctx)

    def _hand_over(self, *tensors):
        """Tensors allocated and filled on the context's stream become safe
        to use (and to free) on the caller's current stream."""
        cur = torch.cuda.current_stream()
        if cur != self.stream:
            cur.wait_stream(self.stream)
            for t in tensors:
                t.record_stream(cur)

    def set_collisions(self, d):
        self._coll = make_collisions(d)
        self._call("pic_set_collisions", ctypes.byref(self._coll))

    def set_coulomb(self, d):
        k = Coulomb()
        d = d or {}
        k.enabled = int(bool(d.get("enabled", False)))
        k.ln_lambda = float(d.get("ln_lambda", 10.0))
        self._coul = k
        self._call("pic_set_coulomb", ctypes.byref(k))

    def set_ion_processes(self, d):
        k = IonProcesses()
        d = d or {}
        k.enabled = int(bool(d.get("enabled", False)))
        k.sigma_rec_1eV = float(d.get("sigma_rec_1eV", 1e-24))
        k.lotz_a2 = float(d.get("lotz_a2", 4.5e-18))
        k.ion2_I_eV = float(d.get("I2_eV", 20.29))
        k.cx_a = float(d.get("cx_a", 7.0710678118654755e-10))
        k.cx_b = float(d.get("cx_b", 0.0))
        self._ionp = k
        self._call("pic_set_ion_processes", ctypes.byref(k))

    def set_sources(self, d):
        self._src = make_sources(d)
        self._call("pic_set_sources", ctypes.byref(self._src))

    def inject(self, species, pos, vel):
        pos, vel = _soa(pos), _soa(vel)
        n = pos.shape[1]
        self._keep += [pos, vel]
        self._call("pic_inject", int(species), n, _ptr(pos), _ptr(vel))

    def load(self, species, pos, vel, ids):
        pos, vel = _soa(pos), _soa(vel)
        ids = torch.as_tensor(ids, device="cuda").to(torch.int64).contiguous()
        self._call("pic_load_particles", int(species), pos.shape[1], _ptr(pos),
                   _ptr(vel), _ptr(ids))

    def count(self, species):
        n = _c_i64()
        self._call("pic_count", int(species), ctypes.byref(n))
        return n.value

    def read(self, species):
        n = self.count(species)
        with torch.cuda.stream(self.stream):
            pos = torch.empty((3, max(n, 1)), dtype=torch.float64,
                              device="cuda")
            vel = torch.empty_like(pos)
            ids = torch.empty(max(n, 1), dtype=torch.int64, device="cuda")
        got = _c_i64()
        self._call("pic_read_particles", int(species), n, _ptr(pos), _ptr(vel),
                   _ptr(ids), ctypes.byref(got))
        self._hand_over(pos, vel, ids)
        return (pos[:, :n].t().contiguous(), vel[:, :n].t().contiguous(),
                ids[:n])

    def read_fields(self):
        shp = self.grid_shape
        with torch.cuda.stream(self.stream):
            acc = torch.empty(shp, dtype=torch.int64, device="cuda")
            phi = torch.empty(shp, dtype=torch.float64, device="cuda")
            E = torch.empty((3,) + shp, dtype=torch.float64, device="cuda")
        self._call("pic_read_fields", _ptr(acc), _ptr(phi), _ptr(E))
        self._hand_over(acc, phi, E)
        return acc, phi, E.permute(1, 2, 3, 0).contiguous()

    def deposit(self):
        self._call("pic_deposit")

    def field(self):
        info = SolveInfo()
        self._call("pic_field", ctypes.byref(info))
        return _struct_dict(info)

    def set_phi(self, phi):
        phi = torch.as_tensor(phi, dtype=torch.float64, device="cuda").contiguous()
        self._keep.append(phi)
        self._call("pic_set_phi", _ptr(phi))

    def _absorbed(self, ab):
        n = ab.n
        out = {"n": n}
        if n > 0:
            st = self.stream.cuda_stream
            with torch.cuda.stream(self.stream):
                sp = _wrap_dev(ab.species, n, torch.int32, st)
                ids = _wrap_dev(ab.id, n, torch.int64, st)
                pos = _wrap_dev(ab.pos, 3 * n, torch.float64, st)
                vel = _wrap_dev(ab.vel, 3 * n, torch.float64, st)
            self._hand_over(sp, ids, pos, vel)
            out["species"] = sp
            out["id"] = ids
            out["pos"] = pos.reshape(3, n).t()
            out["vel"] = vel.reshape(3, n).t()
        return out

    def advance(self, dt):
        ab, dg = Absorbed(), Diag()
        self._call("pic_advance", float(dt), ctypes.byref(ab), ctypes.byref(dg))
        self._keep = []
        return self._absorbed(ab), _struct_dict(dg)

    def step(self, dt):
        ab, dg = Absorbed(), Diag()
        self._call("pic_step", float(dt), ctypes.byref(ab), ctypes.byref(dg))
        self._keep = []
        return self._absorbed(ab), _struct_dict(dg)

    def poisson_solve(self, rho, phi=None):
        rho = torch.as_tensor(rho, dtype=torch.float64, device="cuda").contiguous()
        warm = phi is not None
        out = (torch.as_tensor(phi, dtype=torch.float64, device="cuda").clone()
               if warm else torch.zeros(self.grid_shape, dtype=torch.float64,
                                        device="cuda"))
        info = SolveInfo()
        self._call("poisson_solve", _ptr(rho), _ptr(out), 1 if warm else 0,
                   ctypes.byref(info))
        return out, _struct_dict(info)

    def enable_timing(self, on=True):
        self._call("pic_enable_timing", 1 if on else 0)

    def phase_times(self):
        """{phase: (total ms, timed executions)} since timing was enabled."""
        ms = (_c_d * len(PHASES))()
        calls = (_c_i64 * len(PHASES))()
        self._call("pic_phase_times", ms, calls)
        return {k: (ms[i], calls[i]) for i, k in enumerate(PHASES)}

    def set_warm_start(self, mode, net=None):
        """mode: "prev", "record" or "unet" (net: a UNet on this device)."""
        self.net = net  # keeps the network alive while attached
        self._call("pic_set_warm_start", WARM_MODES[mode],
                   net.u if net is not None else None)

    def warm_pair(self):
        """(input (nz, ny, nx, 2), target (nz, ny, nx)) FP32 of the last
        recorded solve."""
        nz, ny, nx = self.p["nz"], self.p["ny"], self.p["nx"]
        with torch.cuda.stream(self.stream):
            x = torch.empty((nz, ny, nx, 2), dtype=torch.float32,
                            device="cuda")
            t = torch.empty((nz, ny, nx), dtype=torch.float32, device="cuda")
        self._call("pic_warm_pair", _ptr(x), _ptr(t))
        self._hand_over(x, t)
        return x, t

    def checkpoint(self):
        """The context's checkpoint as bytes (host memory)."""
        n = ctypes.c_size_t()
        self._call("pic_checkpoint_bytes", ctypes.byref(n))
        buf = ctypes.create_string_buffer(n.value)
        self._call("pic_checkpoint_save", buf, n.value)
        return buf.raw

    def restore(self, data):
        buf = ctypes.create_string_buffer(bytes(data), len(data))
        self._call("pic_checkpoint_load", buf, len(data))

    def md_return(self, lattice_a, species=(ION,)):
        """Atoms handed back to MD from the last step's cathode list: dict
        of species, id, pos (n, 3), vel (n, 3) device tensors."""
        mask = 0
        for sp in species:
            mask |= 1 << int(sp)
        n = _c_i64()
        # First call with no room: the count (PIC_ERR_CAPACITY if non-zero).
        st = self.lib.pic_md_return(self.ctx, float(lattice_a), mask, 0, None,
                                    None, None, None, ctypes.byref(n))
        if st not in (0, -2):
            self._check(st, self.ctx)
        k = n.value
        with torch.cuda.stream(self.stream):
            pos = torch.empty((3, max(k, 1)), dtype=torch.float64,
                              device="cuda")
            vel = torch.empty_like(pos)
            ids = torch.empty(max(k, 1), dtype=torch.int64, device="cuda")
            sp_t = torch.empty(max(k, 1), dtype=torch.int32, device="cuda")
        self._call("pic_md_return", float(lattice_a), mask, k, _ptr(pos),
                   _ptr(vel), _ptr(ids), _ptr(sp_t), ctypes.byref(n))
        self._hand_over(pos, vel, ids, sp_t)
        return {"species": sp_t[:k], "id": ids[:k],
                "pos": pos[:, :k].t(), "vel": vel[:, :k].t()}

    def debye_check(self, block=1, alpha_D=0.5, with_lambda=True):
        """(info dict, lambda_D per block (bz, by, bx) device tensor or
        None)."""
        lam = None
        if with_lambda:
            shp = (self.p["nz"] // block, self.p["ny"] // block,
                   self.p["nx"] // block)
            with torch.cuda.stream(self.stream):
                lam = torch.empty(shp, dtype=torch.float64, device="cuda")
        info = DebyeInfo()
        self._call("pic_debye_check", int(block), float(alpha_D), _ptr(lam),
                   ctypes.byref(info))
        if lam is not None:
            self._hand_over(lam)
        return _struct_dict(info), lam

    def set_clock(self, step, next_id):
        self._call("pic_set_clock", int(step), int(next_id))


def poisson_solve_static(p, rho, phi=None, **kw):
    """rho -> phi through the allocation-free entry point (no context, no
    workspace) on the current stream; kw as for make_config."""
    lib = load_library()
    cfg = make_config(p, capacity=(0, 0, 0), queue_capacity=0, max_events=1,
                      **kw)
    shape = (p["nz"] + 1, p["ny"], p["nx"])
    rho = torch.as_tensor(rho, dtype=torch.float64, device="cuda").contiguous()
    warm = phi is not None
    out = (torch.as_tensor(phi, dtype=torch.float64, device="cuda").clone()
           if warm else torch.zeros(shape, dtype=torch.float64, device="cuda"))
    info = SolveInfo()
    st = lib.poisson_solve_static(
        ctypes.byref(cfg), _ptr(rho), _ptr(out), 1 if warm else 0,
        ctypes.byref(info),
        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if st != 0:
        raise PicError(st, "poisson_solve_static")
    return out, _struct_dict(info)


def _struct_dict(s):
    d = {}
    for name, typ in s._fields_:
        v = getattr(s, name)
        if isinstance(v, ctypes.Structure):
            v = _struct_dict(v)
        elif hasattr(v, "__len__") and not isinstance(v, (bytes, str)):
            v = list(v)
        d[name] = v
    return d


def _wrap_dev(ptr, n, dtype, stream):
    """Copy n elements of library-owned device memory into a torch tensor,
    queued on the context's stream (so before the next step overwrites
    them).  The caller allocates under that stream (torch.cuda.stream) and
    hands the tensor over to its own stream afterwards."""
    out = torch.empty(n, dtype=dtype, device="cuda")
    nbytes = n * out.element_size()
    _hip_d2d(out.data_ptr(), ptr, nbytes, stream)
    return out


_hip = None


def _hip_d2d(dst, src, nbytes, stream):
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpyAsync.restype = ctypes.c_int
        _hip.hipMemcpyAsync.argtypes = [_c_p, _c_p, ctypes.c_size_t,
                                        ctypes.c_int, _c_p]
    rc = _hip.hipMemcpyAsync(ctypes.c_void_p(dst), ctypes.c_void_p(src),
                             ctypes.c_size_t(nbytes), 3,  # device to device
                             ctypes.c_void_p(stream))
    if rc != 0:
        raise RuntimeError(f"hipMemcpyAsync failed: {rc}")


UNET_EXPORTS = {
    "pic_unet_param_count": (_c_i64, []),
    "pic_unet_workspace_bytes": (_c_i32, [_c_i32, _c_i32, _c_i32,
                                          ctypes.POINTER(ctypes.c_size_t)]),
    "pic_unet_init": (_c_i32, [_c_i32, _c_i32, _c_i32, _c_p, ctypes.c_size_t,
                               _c_p, ctypes.POINTER(_c_p)]),
    "pic_unet_destroy": (None, [_c_p]),
    "pic_unet_set_params": (_c_i32, [_c_p, _c_p]),
    "pic_unet_get_params": (_c_i32, [_c_p, _c_p]),
    "pic_unet_forward": (_c_i32, [_c_p, _c_p, _c_i32, _c_i32, _c_i32, _c_p]),
    "pic_unet_gradients": (_c_i32, [_c_p, _c_p, _c_p, _c_i32, _c_i32, _c_i32,
                                    _c_p, ctypes.POINTER(_c_d)]),
    "pic_unet_train_step": (_c_i32, [_c_p, _c_p, _c_p, _c_i32, _c_i32, _c_i32,
                                     ctypes.c_float, ctypes.c_float,
                                     ctypes.c_float, ctypes.c_float,
                                     ctypes.POINTER(_c_d)]),
    "pic_unet_last_error": (ctypes.c_char_p, [_c_p]),
    "pic_unet_set_loss": (_c_i32, [_c_p, _c_i32, _c_i32]),
}


def _unet_lib():
    lib = load_library()
    if not getattr(lib, "_unet_bound", False):
        for name, (res, args) in UNET_EXPORTS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        lib._unet_bound = True
    return lib


class UNet:
    """The learned warm-start network on the current device and stream.
    Inputs are channels-last FP32 tensors: x (D, H, W, 2), target (D, H, W).
    """

    def __init__(self, D, H, W, params=None):
        self.lib = _unet_lib()
        self.shape = (int(D), int(H), int(W))
        n = ctypes.c_size_t()
        self._check(self.lib.pic_unet_workspace_bytes(D, H, W, ctypes.byref(n)))
        self.ws = torch.empty(n.value + 256, dtype=torch.uint8, device="cuda")
        base = (self.ws.data_ptr() + 255) // 256 * 256
        u = ctypes.c_void_p()
        self._check(self.lib.pic_unet_init(
            D, H, W, ctypes.c_void_p(base), n.value,
            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
            ctypes.byref(u)))
        self.u = u
        self.n_params = int(self.lib.pic_unet_param_count())
        if params is not None:
            self.set_params(params)

    @staticmethod
    def param_count():
        return int(_unet_lib().pic_unet_param_count())

    def __del__(self):
        if getattr(self, "u", None):
            self.lib.pic_unet_destroy(self.u)
            self.u = None

    def _check(self, status):
        if status != 0:
            msg = ""
            if getattr(self, "u", None):
                msg = (self.lib.pic_unet_last_error(self.u) or b"").decode()
            raise PicError(status, msg)

    def set_loss(self, mode="mse", k0=1):
        """mode "mse" or "residual" (k0: first unknown plane)."""
        self._check(self.lib.pic_unet_set_loss(
            self.u, {"mse": 0, "residual": 1}[mode], int(k0)))

    def set_params(self, params):
        p = torch.as_tensor(params, dtype=torch.float32, device="cuda").contiguous()
        assert p.numel() == self.n_params
        self._check(self.lib.pic_unet_set_params(self.u, _ptr(p)))

    def get_params(self):
        p = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        self._check(self.lib.pic_unet_get_params(self.u, _ptr(p)))
        return p

    def _dims(self, x):
        D, H, W = x.shape[:3]
        return int(D), int(H), int(W)

    def forward(self, x):
        x = torch.as_tensor(x, dtype=torch.float32, device="cuda").contiguous()
        D, H, W = self._dims(x)
        out = torch.empty((D, H, W), dtype=torch.float32, device="cuda")
        self._check(self.lib.pic_unet_forward(self.u, _ptr(x), D, H, W, _ptr(out)))
        return out

    def gradients(self, x, t):
        x = torch.as_tensor(x, dtype=torch.float32, device="cuda").contiguous()
        t = torch.as_tensor(t, dtype=torch.float32, device="cuda").contiguous()
        D, H, W = self._dims(x)
        g = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        loss = _c_d()
        self._check(self.lib.pic_unet_gradients(self.u, _ptr(x), _ptr(t), D, H,
                                                W, _ptr(g), ctypes.byref(loss)))
        return g, loss.value

    def train_step(self, x, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        x = torch.as_tensor(x, dtype=torch.float32, device="cuda").contiguous()
        t = torch.as_tensor(t, dtype=torch.float32, device="cuda").contiguous()
        D, H, W = self._dims(x)
        loss = _c_d()
        self._check(self.lib.pic_unet_train_step(self.u, _ptr(x), _ptr(t), D, H,
                                                 W, lr, beta1, beta2, eps,
                                                 ctypes.byref(loss)))
        return loss.value
