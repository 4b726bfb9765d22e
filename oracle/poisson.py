"""Discrete Poisson problem of the PIC field solve, solved exactly.

Test infrastructure only (see the package docstring).

The paper solves Poisson's equation, Eq. 1 (Laplacian of phi equals minus
rho over epsilon_0), in the vacuum gap with Dirichlet or Neumann conditions.
On the uniform node-centred grid used here (nodes i in [0, nx), j in [0, ny)
periodic; k in [0, nz] from cathode to anode, spacing dx) the equation is
discretised with the 7-point stencil and scaled by dx^2:

    (A phi)_n = 6 phi_n - sum of the 6 neighbours = b_n,
    b_n = dx^2 rho_n / epsilon_0.

z faces:
  * Dirichlet: phi fixed to the face value; the face node is not an unknown,
    its value enters b of the next-inner node.
  * Neumann with prescribed g = d(phi)/dz (V/m) at the face: the face node is
    an unknown, its out-of-domain neighbour is the mirror ghost
    phi_ghost = phi_inner -/+ 2 dx g (minus at the cathode face, plus at the
    anode face), and the face node owns half a cell of volume, so its charge
    density is doubled (finite-volume reading of the boundary node).

Both faces Neumann is singular with periodic x, y and is rejected.

The exact solve diagonalises the periodic x, y part with a 2-D DFT; every
(p, q) mode is then a tridiagonal system in z, solved with the Thomas
algorithm.  It reaches the discrete solution up to rounding, with no
iteration choice.
"""
import numpy as np

DIRICHLET, NEUMANN = 0, 1


class Grid:
    """Uniform grid description shared by every oracle function."""

    def __init__(self, nx, ny, nz, dx, bc_lo=DIRICHLET, bc_hi=DIRICHLET,
                 v_lo=0.0, v_hi=0.0):
        if bc_lo == NEUMANN and bc_hi == NEUMANN:
            raise ValueError("both z faces Neumann: singular operator")
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.dx = float(dx)
        self.bc_lo, self.bc_hi = int(bc_lo), int(bc_hi)
        self.v_lo, self.v_hi = float(v_lo), float(v_hi)
        self.inv_dx = 1.0 / self.dx
        self.lx = float(self.nx) * self.dx
        self.ly = float(self.ny) * self.dx
        self.lz = float(self.nz) * self.dx

    @property
    def shape(self):
        """Node array shape, z slowest, x fastest."""
        return (self.nz + 1, self.ny, self.nx)

    @property
    def k_range(self):
        """First and last k plane holding unknowns."""
        k0 = 1 if self.bc_lo == DIRICHLET else 0
        k1 = self.nz - 1 if self.bc_hi == DIRICHLET else self.nz
        return k0, k1


def rhs_from_density(rho, grid):
    """b = dx^2 rho / eps0 at every node, plus the boundary terms.

    rho: charge density at nodes, C/m^3, shape grid.shape (the density of a
    Neumann face node is the charge in its half-cell divided by its half-cell
    volume, i.e. the caller's value is used as given).
    Returns b with zeros on Dirichlet planes.
    """
    from .constants import EPS0
    scale = (grid.dx * grid.dx) / EPS0
    b = np.asarray(rho, dtype=np.float64) * scale
    return add_boundary_terms(b, grid)


def add_boundary_terms(b, grid):
    """Move the known boundary data of the z faces into b (copy)."""
    b = np.array(b, dtype=np.float64, copy=True)
    nz = grid.nz
    if grid.bc_lo == DIRICHLET:
        b[0] = 0.0
        b[1] += grid.v_lo
    else:
        b[0] -= 2.0 * grid.dx * grid.v_lo
    if grid.bc_hi == DIRICHLET:
        b[nz] = 0.0
        b[nz - 1] += grid.v_hi
    else:
        b[nz] += 2.0 * grid.dx * grid.v_hi
    return b


def apply_operator(phi, grid):
    """(A phi) on the unknown planes; zero on Dirichlet planes.

    phi holds the Dirichlet face values on Dirichlet planes; those values do
    not enter the result (they belong to b).  Used for residuals in tests.
    """
    phi = np.asarray(phi, dtype=np.float64)
    nz = grid.nz
    out = np.zeros_like(phi)
    k0, k1 = grid.k_range
    # Dirichlet face values are data, not unknowns: zero them for A.
    ph = phi.copy()
    if grid.bc_lo == DIRICHLET:
        ph[0] = 0.0
    if grid.bc_hi == DIRICHLET:
        ph[nz] = 0.0
    for k in range(k0, k1 + 1):
        p = ph[k]
        xy = (np.roll(p, 1, axis=1) + np.roll(p, -1, axis=1)
              + np.roll(p, 1, axis=0) + np.roll(p, -1, axis=0))
        if k == 0:
            zz = 2.0 * ph[1]
        elif k == nz:
            zz = 2.0 * ph[nz - 1]
        else:
            zz = ph[k - 1] + ph[k + 1]
        out[k] = 6.0 * p - xy - zz
    return out


def residual(phi, b, grid):
    """r = b - A phi on unknown planes (zero elsewhere)."""
    r = b - apply_operator(phi, grid)
    k0, k1 = grid.k_range
    r[:k0] = 0.0
    r[k1 + 1:] = 0.0
    return r


def solve_exact(b, grid):
    """Exact discrete solution of A phi = b (b from add_boundary_terms).

    Returns phi on all nodes, with the Dirichlet face values set.
    """
    nx, ny, nz = grid.nx, grid.ny, grid.nz
    k0, k1 = grid.k_range
    m = k1 - k0 + 1
    bh = np.fft.fft2(np.asarray(b, dtype=np.float64)[k0:k1 + 1], axes=(1, 2))
    p = np.arange(nx)
    q = np.arange(ny)
    lam = (4.0 * np.sin(np.pi * q / ny)[:, None] ** 2
           + 4.0 * np.sin(np.pi * p / nx)[None, :] ** 2)
    diag = 2.0 + lam                                   # (ny, nx)
    # Tridiagonal rows: lower[r] * x[r-1] + diag * x[r] + upper[r] * x[r+1].
    lower = -np.ones(m)
    upper = -np.ones(m)
    lower[0] = 0.0
    upper[m - 1] = 0.0
    if grid.bc_lo == NEUMANN:
        upper[0] = -2.0
    if grid.bc_hi == NEUMANN:
        lower[m - 1] = -2.0
    # Thomas algorithm, vectorised over the (q, p) modes.
    cp = np.empty((m, ny, nx), dtype=np.complex128)
    dp = np.empty((m, ny, nx), dtype=np.complex128)
    cp[0] = upper[0] / diag
    dp[0] = bh[0] / diag
    for r in range(1, m):
        den = diag - lower[r] * cp[r - 1]
        cp[r] = upper[r] / den
        dp[r] = (bh[r] - lower[r] * dp[r - 1]) / den
    xh = np.empty_like(dp)
    xh[m - 1] = dp[m - 1]
    for r in range(m - 2, -1, -1):
        xh[r] = dp[r] - cp[r] * xh[r + 1]
    phi = np.zeros(grid.shape, dtype=np.float64)
    phi[k0:k1 + 1] = np.fft.ifft2(xh, axes=(1, 2)).real
    if grid.bc_lo == DIRICHLET:
        phi[0] = grid.v_lo
    if grid.bc_hi == DIRICHLET:
        phi[nz] = grid.v_hi
    return phi


def rel_residual(phi, b, grid):
    """||b - A phi||_2 / ||b||_2 over the unknown planes."""
    r = residual(phi, b, grid)
    bn = np.sqrt(np.sum(b * b))
    return float(np.sqrt(np.sum(r * r)) / bn) if bn > 0 else 0.0
