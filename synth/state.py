"""Synthetic flow state: a pressure field consistent with the permeability field.

The paper's Jacobians are linearisations at states of a running simulation, where the
pressure nearly satisfies the total mass balance, so the Darcy fluxes are close to
divergence free away from wells.  A pressure made of a linear ramp plus cell noise is
not: on a heterogeneous field every cell becomes a strong source or sink, which makes
the saturation rows of the Jacobian far from diagonally dominant (inflow derivatives
thousands of times the cell's own coefficient) -- a property of the input, not of the
method.  The state used here is instead

  p = p_hydro + p_drive,

p_hydro the water-hydrostatic part and p_drive the steady single-phase pressure of a
line drive along x: div(T grad p_drive) = 0 on the TPFA stencil of the same
transmissibilities (App. A), with p_drive fixed at `dp` on one x face and 0 on the
other through half-cell transmissibilities, no flow through the other faces.  The
closed system the Jacobian describes then sees the two end columns of cells as the
injection and production wells of the drive.

p_drive is found by conjugate gradients to a relative residual of 1e-10 (flux imbalance
at interior cells of order 1e-8 of the cell's throughput), preconditioned by a
two-level scheme (a Jacobi sweep, a correction from the Galerkin projection of the
Laplacian onto piecewise-constant boxes of about 4 x 4 x 4 cells solved directly, a
second Jacobi sweep) so that the large grids take seconds.  This is input preparation;
it holds none of the solver's method.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .jacobian import faces, transmissibility


def _laplacian(kperm, nx, ny, nz, h):
    n = nx * ny * nz
    K, L, _ = faces(nx, ny, nz)
    T = transmissibility(kperm, h, K, L)
    rows = np.concatenate([K, L, K, L])
    cols = np.concatenate([K, L, L, K])
    vals = np.concatenate([T, T, -T, -T])
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def drive_pressure(kperm, nx, ny, nz, h, dp, drive=1.0, rtol=1e-10, maxit=20000):
    """Steady line-drive pressure (Pa) per cell, x fastest.

    drive = +1: p_drive = dp on the x = L face and 0 on x = 0 (flow towards -x);
    drive = -1: the reverse (injection at x = 0).
    """
    n = nx * ny * nz
    A = _laplacian(kperm, nx, ny, nz, h)
    ci = np.tile(np.arange(nx), ny * nz)
    tb = 2.0 * h * kperm                     # half-cell transmissibility to a boundary face
    d = np.zeros(n)
    b = np.zeros(n)
    hi_face = ci == (nx - 1 if drive > 0 else 0)
    lo_face = ci == (0 if drive > 0 else nx - 1)
    d[hi_face] += tb[hi_face]
    d[lo_face] += tb[lo_face]
    b[hi_face] += tb[hi_face] * dp
    A = (A + sp.diags(d)).tocsr()
    dinv = 1.0 / A.diagonal()
    # boxes of about 4 x 4 x 4 cells (at most ~12k of them) for the coarse correction
    box = []
    for m in (nx, ny, nz):
        a = 4
        while m / a > 24:
            a *= 2
        box.append(min(a, m))
    ci_ = np.arange(n)
    ix, iy, iz = ci_ % nx, (ci_ // nx) % ny, ci_ // (nx * ny)
    bx, by = -(-nx // box[0]), -(-ny // box[1])
    agg = ix // box[0] + bx * (iy // box[1] + by * (iz // box[2]))
    P = sp.csr_matrix((np.ones(n), (ci_, agg)), shape=(n, int(agg.max()) + 1))
    lu = spla.splu((P.T @ A @ P).tocsc())

    def precond(r):
        z = dinv * r
        z += P @ lu.solve(P.T @ (r - A @ z))
        z += dinv * (r - A @ z)
        return z

    # preconditioned conjugate gradients from the linear ramp
    xc = (ci + 0.5) / nx
    x = dp * (xc if drive > 0 else 1.0 - xc)
    r = b - A @ x
    z = precond(r)
    p = z.copy()
    rz = r @ z
    bn = np.linalg.norm(b)
    for _ in range(maxit):
        if np.linalg.norm(r) <= rtol * bn:
            break
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        z = precond(r)
        rz_new = r @ z
        p *= rz_new / rz
        p += z
        rz = rz_new
    else:
        raise RuntimeError("drive pressure: conjugate gradients did not converge")
    return x
