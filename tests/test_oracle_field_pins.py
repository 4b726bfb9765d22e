"""Pins of the oracle's field-side arithmetic that no closed form elsewhere
reaches (CPU only).

* E_z on the two z faces (one-sided second-order differences, the field the
  Fowler-Nordheim source reads): exact for the quadratic potential of a
  uniform charge between Dirichlet plates (Eq. 1 in one dimension).
* The doubled charge density of a Neumann face node in rhs(): a lattice of
  ions at cell centres is a uniform density, and only with the face node's
  half-cell volume taken into account does the solve give the closed-form
  quadratic of that density with the prescribed face slope.
* field_energy(): the discrete Green identity.  With zero-potential plates,
  sum_n q_n phi_n = eps0 dx sum over grid edges of (phi_a - phi_b)^2, since
  A phi = b = q / (eps0 dx) node by node (summation by parts of the 7-point
  operator).
* adam_step(): five steps against torch.optim.Adam in float64.

Each pin has a planted-mistake test: the mutated oracle must fail it.
"""
import numpy as np
import pytest

from oracle import constants as C
from oracle import pic as O
from oracle import poisson as P
from oracle import unet as U


# --------------------------------------------------------------------------
# E_z on the z faces
# --------------------------------------------------------------------------
def _uniform_charge_between_plates(nz=24, dx=2e-9, rho0=-4.0e6, V=30.0):
    g = P.Grid(4, 6, nz, dx, v_lo=0.0, v_hi=V)
    phi = P.solve_exact(P.rhs_from_density(np.full(g.shape, rho0), g), g)
    # Continuum: phi'' = -rho0/eps0, phi(0) = 0, phi(L) = V.
    L = nz * dx
    a2 = -rho0 / (2.0 * C.EPS0)
    c1 = (V - a2 * L * L) / L
    return g, phi, a2, c1, L


def test_uniform_charge_potential_is_the_quadratic():
    g, phi, a2, c1, L = _uniform_charge_between_plates()
    z = np.arange(g.nz + 1) * g.dx
    ref = a2 * z * z + c1 * z
    assert np.max(np.abs(phi[:, 2, 1] - ref)) <= 1e-11 * np.max(np.abs(ref))


def test_ez_faces_exact_for_uniform_charge_between_plates():
    """-dphi/dz of the quadratic at z = 0 and z = L, and central
    differences inside, to 1e-12 of the field scale."""
    g, phi, a2, c1, L = _uniform_charge_between_plates()
    E = O.efield(phi, g)
    z = np.arange(g.nz + 1) * g.dx
    ref = -(2.0 * a2 * z + c1)
    scale = np.max(np.abs(ref))
    got = E[:, 3, 2, 2]
    assert abs(got[0] - ref[0]) <= 1e-12 * scale, (got[0], ref[0])
    assert abs(got[-1] - ref[-1]) <= 1e-12 * scale, (got[-1], ref[-1])
    assert np.max(np.abs(got - ref)) <= 1e-12 * scale
    # The transverse components of a z-only potential vanish.
    assert np.max(np.abs(E[..., :2])) <= 1e-12 * scale


def test_planted_first_order_face_field_fails_pin(monkeypatch):
    orig = O.efield

    def first_order(phi, g):
        E = orig(phi, g)
        E[0, :, :, 2] = (phi[0] - phi[1]) * g.inv_dx
        return E
    monkeypatch.setattr(O, "efield", first_order)
    with pytest.raises(AssertionError):
        test_ez_faces_exact_for_uniform_charge_between_plates()


def test_planted_top_face_sign_fails_pin(monkeypatch):
    orig = O.efield

    def flipped(phi, g):
        E = orig(phi, g)
        E[g.nz, :, :, 2] = -E[g.nz, :, :, 2]
        return E
    monkeypatch.setattr(O, "efield", flipped)
    with pytest.raises(AssertionError):
        test_ez_faces_exact_for_uniform_charge_between_plates()


# --------------------------------------------------------------------------
# Neumann face: doubled density of the half-cell node
# --------------------------------------------------------------------------
def test_neumann_face_charge_from_ion_lattice():
    """One Cu+ at every cell centre deposits 1/8 of its charge on each of
    the cell's nodes: interior nodes collect a full unit, the cathode face
    node only half (it borders cells on one side).  Density e/dx^3
    everywhere once the face node's half volume is used, so the solve with
    slope g at the Neumann cathode and V at the anode is the quadratic
    phi = a2 z^2 + g z + c, a2 = -rho0/(2 eps0)."""
    nx, ny, nz, dx = 4, 4, 16, 3e-9
    gslope, V = 2.0e7, 1.5
    g = P.Grid(nx, ny, nz, dx, bc_lo=P.NEUMANN, bc_hi=P.DIRICHLET,
               v_lo=gslope, v_hi=V)
    st = O.State(g, w_sp=1)
    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz),
                          indexing="ij")
    pos = (np.stack([i.ravel(), j.ravel(), k.ravel()], 1) + 0.5) * dx
    st.load(C.ION, pos, np.zeros_like(pos),
            np.arange(pos.shape[0], dtype=np.uint64))
    acc = O.deposit(st)
    unit = 2 ** 39
    assert np.all(acc[1:nz] == unit) and np.all(acc[0] == unit // 2)
    phi = P.solve_exact(O.rhs(acc, g, st.w_sp), g)
    rho0 = C.E_CHARGE / dx ** 3
    z = np.arange(nz + 1) * dx
    L = nz * dx
    a2 = -rho0 / (2.0 * C.EPS0)
    ref = a2 * z * z + gslope * z + (V - a2 * L * L - gslope * L)
    assert np.max(np.abs(phi[:, 1, 2] - ref)) <= 1e-9 * np.max(np.abs(ref))


def test_planted_missing_neumann_doubling_fails_pin(monkeypatch):
    def undoubled(acc, grid, w_sp):
        b = acc.astype(np.float64) * O.charge_scale(grid, w_sp)
        return P.add_boundary_terms(b, grid)
    monkeypatch.setattr(O, "rhs", undoubled)
    with pytest.raises(AssertionError):
        test_neumann_face_charge_from_ion_lattice()


# --------------------------------------------------------------------------
# Field energy: discrete Green identity
# --------------------------------------------------------------------------
def _edge_energy(phi, g):
    """eps0 dx / 2 times the sum over every grid edge of (phi_a - phi_b)^2:
    x and y edges of all planes (periodic), z edges between planes."""
    ex = phi - np.roll(phi, -1, axis=2)
    ey = phi - np.roll(phi, -1, axis=1)
    ez = phi[1:] - phi[:-1]
    s = np.sum(ex * ex) + np.sum(ey * ey) + np.sum(ez * ez)
    return 0.5 * C.EPS0 * g.dx * s


def test_field_energy_green_identity():
    g = P.Grid(8, 6, 12, 2e-9, v_lo=0.0, v_hi=0.0)
    st = O.State(g, w_sp=3)
    rng = np.random.default_rng(21)
    L = np.array([g.lx, g.ly, g.lz])
    for s, n in ((C.ELECTRON, 700), (C.ION, 400)):
        pos = rng.random((n, 3)) * L
        st.load(s, pos, np.zeros_like(pos),
                np.arange(n, dtype=np.uint64) + 1000 * s)
    acc = O.deposit(st)
    phi = P.solve_exact(O.rhs(acc, g, st.w_sp), g)
    got = O.field_energy(acc, phi, g, st.w_sp)
    ref = _edge_energy(phi, g)
    assert ref > 0
    assert abs(got - ref) <= 1e-10 * ref, (got, ref)


def test_planted_field_energy_factor_fails_pin(monkeypatch):
    orig = O.field_energy
    monkeypatch.setattr(O, "field_energy",
                        lambda acc, phi, g, w: 2.0 * orig(acc, phi, g, w))
    with pytest.raises(AssertionError):
        test_field_energy_green_identity()


def test_planted_field_energy_weight_fails_pin(monkeypatch):
    orig = O.field_energy
    monkeypatch.setattr(O, "field_energy",
                        lambda acc, phi, g, w: orig(acc, phi, g, 1))
    with pytest.raises(AssertionError):
        test_field_energy_green_identity()


# --------------------------------------------------------------------------
# Adam
# --------------------------------------------------------------------------
def test_adam_five_steps_match_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    p0 = rng.standard_normal(40)
    grads = [rng.standard_normal(40) * 10.0 ** rng.uniform(-3, 1, 40)
             for _ in range(5)]
    lr, b1, b2, eps = 3e-3, 0.8, 0.95, 1e-6
    p = p0.copy()
    m, v = np.zeros(40), np.zeros(40)
    tp = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=lr, betas=(b1, b2), eps=eps)
    for t, gr in enumerate(grads, start=1):
        U.adam_step(p, m, v, gr, t, lr, beta1=b1, beta2=b2, eps=eps)
        opt.zero_grad()
        tp.grad = torch.tensor(gr, dtype=torch.float64)
        opt.step()
        ref = tp.detach().numpy()
        assert np.allclose(p, ref, rtol=1e-12, atol=1e-15), t


def test_planted_swapped_adam_betas_fails_pin(monkeypatch):
    orig = U.adam_step

    def swapped(params, m, v, grad, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        return orig(params, m, v, grad, t, lr, beta1=beta2, beta2=beta1,
                    eps=eps)
    monkeypatch.setattr(U, "adam_step", swapped)
    with pytest.raises(AssertionError):
        test_adam_five_steps_match_torch()
