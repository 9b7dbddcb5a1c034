"""Seeded synthetic fully-implicit multiphase-poromechanics Jacobians.

This module is *input generation* shared by the tests, the oracle checks and the
benchmark.  It holds none of the solver's arithmetic (no preconditioner, no Krylov
method); it only discretises the physics of Sec. 2-3 and App. A-B of the paper on a
structured hexahedral grid and linearises it at a synthetic state.

Discretisation (paper Sec. 3, App. A, App. B):
  * Q1 finite elements for the displacement (3 dof per node), drained isotropic
    elasticity, Biot coefficient b, gravity body force of the mixture density
    (App. B.2, A_uu / A_up / A_us element terms).
  * P0 cell-centred unknowns for the flow: saturation dof(s) then pressure, per
    cell, interleaved (the permutation P of Sec. 5.3 is the identity).
  * TPFA fluxes with single-point upstream weighting and averaged face density
    (eqs. num_flux_approx, avg_density), harmonic transmissibility (App. A).
  * Backward-Euler mass accumulation (App. B.1) with fluid density
    rho = rho0 (1 + c (p - p0)) and incompressible grains, b = 1 (Sec. 6).
  * Fixed-stress diagonals D_sp = V b^2/K_dr s rho_w, D_pp = V b^2/K_dr (1-s) rho_nw
    (eq. FS_Dps_Dpp); for three phases D_sp holds one entry per saturation dof
    (remark after eq. FS_Dps_Dpp).

Readings where the paper is silent or inconsistent:
  * Face-term sign: the residual is written with the physically consistent sign,
    whose Jacobian is the +[[psi]] dt dF/dx form of App. B.2, so the TPFA part of
    the pressure block has a positive diagonal.
  * Block-row/column scaling (remark in Sec. 4): A~ = C A C with one factor per
    field (displacement; each cell dof) c = mean(|a_ii|)^(-1/2); the fixed-stress
    diagonals are scaled the same way.
  * Boundary conditions: bottom face fixed, roller sides, top free; every node is
    kept and a constrained component becomes a decoupled row (row and column
    zeroed, diagonal kept) with zero right-hand side.
  * Synthetic state: p = 20 MPa + rho_w0 g (z_top - z) + 10 MPa x/L_x + N(0, 0.1 MPa),
    p0 = the hydrostatic part; upwind tie (zero potential) -> lower-index cell.
  * No wells (the configurations define none).
  * The displacement block is constant over a simulation (Sec. 5.2: the elasticity
    operator does not change), so its gravity term uses the mixture-density derivative
    at a reference state (reference densities, equal phase saturations) rather than
    the current state; systems on the same grid with the same moduli then share A_uu.
"""
from dataclasses import dataclass, field
import numpy as np

GRAV = 9.81


@dataclass
class BSR:
    """Block CSR with sorted column indices; vals has shape (nblocks, br, bc)."""
    rowptr: np.ndarray
    colind: np.ndarray
    vals: np.ndarray
    nbcols: int

    @property
    def nbrows(self):
        return self.rowptr.shape[0] - 1

    @property
    def br(self):
        return self.vals.shape[1]

    @property
    def bc(self):
        return self.vals.shape[2]

    @property
    def nblocks(self):
        return self.colind.shape[0]


@dataclass
class PoroSystem:
    nx: int
    ny: int
    nz: int
    nf: int
    p_index: int
    Auu: BSR
    Auf: BSR
    Afu: BSR
    Aff: BSR
    d_sp: np.ndarray          # (n_cells, nf-1)
    d_pp: np.ndarray          # (n_cells,)
    constrained: np.ndarray   # (3*n_nodes,) bool
    scale_u: float = 1.0
    scale_f: np.ndarray = None
    meta: dict = field(default_factory=dict)
    ml_part: np.ndarray = None    # optional subdomain id per cell (processor-local BILU)

    @property
    def n_nodes(self):
        return self.Auu.nbrows

    @property
    def n_cells(self):
        return self.Aff.nbrows

    @property
    def n_u(self):
        return 3 * self.n_nodes

    @property
    def n_f(self):
        return self.nf * self.n_cells

    @property
    def N(self):
        return self.n_u + self.n_f


# --------------------------------------------------------------------------
# Phase models (Sec. 6: density model, Corey relative permeabilities)
# --------------------------------------------------------------------------
class Phases:
    """Immiscible phases; the last phase's saturation is 1 - sum(others).

    Cell dofs are [s_0 .. s_{nph-2}, p]; equation rows are the mass balances of
    phases 0..nph-1 in the same order, so the last (pressure) row is the last
    phase's balance.
    """

    def __init__(self, rho0, comp, mu, corey_residual=None):
        self.rho0 = np.asarray(rho0, float)
        self.comp = np.asarray(comp, float)
        self.mu = np.asarray(mu, float)
        self.nph = len(rho0)
        self.res = corey_residual  # (s_wr, s_nwr) for the two-phase Corey model

    def saturations(self, S):
        """S: (n, nph-1) saturation dofs -> (n, nph) phase saturations."""
        return np.concatenate([S, 1.0 - S.sum(axis=1, keepdims=True)], axis=1)

    def dsat(self):
        """d s_l / d S_j, shape (nph, nph-1)."""
        d = np.zeros((self.nph, self.nph - 1))
        d[: self.nph - 1] = np.eye(self.nph - 1)
        d[self.nph - 1] = -1.0
        return d

    def kr(self, S):
        """Relative permeabilities (n, nph) and derivatives d kr_l / d S_j (n, nph, nph-1)."""
        n = S.shape[0]
        if self.nph == 2 and self.res is not None:
            swr, snwr = self.res
            span = 1.0 - swr - snwr
            sh = (S[:, 0] - swr) / span
            kr = np.stack([sh ** 2, (1.0 - sh) ** 2], axis=1)
            dkr = np.zeros((n, 2, 1))
            dkr[:, 0, 0] = 2.0 * sh / span
            dkr[:, 1, 0] = -2.0 * (1.0 - sh) / span
            return kr, dkr
        s = self.saturations(S)
        kr = s ** 2
        dkr = 2.0 * s[:, :, None] * self.dsat()[None, :, :]
        return kr, dkr


def two_phase(mu_w=1e-3, mu_o=5e-3):
    # Table 1: water 1035 kg/m3, 4.34e-4 1/MPa; oil 863 kg/m3, 1.98e-4 1/MPa;
    # residual saturations 0.2 / 0.2.  Viscosities from the workload definition.
    return Phases([1035.0, 863.0], [4.34e-10, 1.98e-10], [mu_w, mu_o], corey_residual=(0.2, 0.2))


def three_phase():
    # water, gas, oil; gas density 200 kg/m3 is a chosen value (not in the paper).
    return Phases([1035.0, 200.0, 863.0], [4.34e-10, 1e-7, 1.98e-10], [1e-3, 2e-5, 5e-3])


# --------------------------------------------------------------------------
# Q1 reference-element integrals on a cube of side h
# --------------------------------------------------------------------------
def q1_cube(h, nu):
    """Returns (Kref, Gd, Gn, V) for a cube of side h.

    Kref[a, r, b, c]: stiffness for E = 1, Poisson ratio nu (local nodes a, b;
                      components r, c).
    Gd[a, c]        : integral of dN_a/dx_c.
    Gn[a, b, c]     : integral of N_a dN_b/dx_c.
    Local node a = ax + 2 ay + 4 az.  2x2x2 Gauss quadrature is exact here.
    """
    g = 1.0 / np.sqrt(3.0)
    pts = [-g, g]
    lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = 1.0 / (2.0 * (1.0 + nu))
    signs = np.array([[2 * (a & 1) - 1, 2 * ((a >> 1) & 1) - 1, 2 * ((a >> 2) & 1) - 1]
                      for a in range(8)], float)
    detJ = (h / 2.0) ** 3
    K = np.zeros((8, 3, 8, 3))
    Gd = np.zeros((8, 3))
    Gn = np.zeros((8, 8, 3))
    for xi in pts:
        for eta in pts:
            for zeta in pts:
                q = np.array([xi, eta, zeta])
                f = (1.0 + signs * q) / 2.0          # (8, 3) factors
                N = f.prod(axis=1)
                dN = np.zeros((8, 3))
                for d in range(3):
                    others = [e for e in range(3) if e != d]
                    dN[:, d] = signs[:, d] / 2.0 * f[:, others[0]] * f[:, others[1]] * (2.0 / h)
                dot = dN @ dN.T
                for r in range(3):
                    for c in range(3):
                        K[:, r, :, c] += detJ * (lam * np.outer(dN[:, r], dN[:, c])
                                                 + mu * np.outer(dN[:, c], dN[:, r])
                                                 + (mu * dot if r == c else 0.0))
                Gd += detJ * dN
                Gn += detJ * N[:, None, None] * dN[None, :, :]
    return K, Gd, Gn, h ** 3


# --------------------------------------------------------------------------
# Structured-grid patterns
# --------------------------------------------------------------------------
def _node_ijk(nx, ny, nz):
    k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    return i.ravel(), j.ravel(), k.ravel()


def _cell_ijk(nx, ny, nz):
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return i.ravel(), j.ravel(), k.ravel()


def _pattern(valid, nbr):
    """valid/nbr: (nrows, nslots) in increasing-column order -> rowptr, colind, slotmap."""
    counts = valid.sum(axis=1)
    rowptr = np.zeros(valid.shape[0] + 1, np.int64)
    np.cumsum(counts, out=rowptr[1:])
    colind = nbr[valid].astype(np.int32)
    slotmap = np.cumsum(valid.ravel()) - 1
    slotmap = np.where(valid.ravel(), slotmap, -1).reshape(valid.shape)
    return rowptr.astype(np.int32), colind, slotmap


def node_node_pattern(nx, ny, nz):
    i, j, k = _node_ijk(nx, ny, nz)
    sx, sxy = nx + 1, (nx + 1) * (ny + 1)
    valid = []
    nbr = []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                ok = ((i + dx >= 0) & (i + dx <= nx) & (j + dy >= 0) & (j + dy <= ny)
                      & (k + dz >= 0) & (k + dz <= nz))
                valid.append(ok)
                nbr.append((i + dx) + sx * (j + dy) + sxy * (k + dz))
    return _pattern(np.stack(valid, 1), np.stack(nbr, 1))


def node_cell_pattern(nx, ny, nz):
    i, j, k = _node_ijk(nx, ny, nz)
    valid = []
    nbr = []
    for oz in (-1, 0):
        for oy in (-1, 0):
            for ox in (-1, 0):
                ci, cj, ck = i + ox, j + oy, k + oz
                ok = (ci >= 0) & (ci < nx) & (cj >= 0) & (cj < ny) & (ck >= 0) & (ck < nz)
                valid.append(ok)
                nbr.append(ci + nx * (cj + ny * ck))
    return _pattern(np.stack(valid, 1), np.stack(nbr, 1))


def cell_node_pattern(nx, ny, nz):
    i, j, k = _cell_ijk(nx, ny, nz)
    sx, sxy = nx + 1, (nx + 1) * (ny + 1)
    base = i + sx * j + sxy * k
    nbr = np.stack([base + (a & 1) + sx * ((a >> 1) & 1) + sxy * ((a >> 2) & 1) for a in range(8)], 1)
    valid = np.ones_like(nbr, bool)
    return _pattern(valid, nbr)


CELL_OFFSETS = [(0, 0, -1), (0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]


def cell_cell_pattern(nx, ny, nz):
    i, j, k = _cell_ijk(nx, ny, nz)
    valid = []
    nbr = []
    for dx, dy, dz in CELL_OFFSETS:
        ok = ((i + dx >= 0) & (i + dx < nx) & (j + dy >= 0) & (j + dy < ny)
              & (k + dz >= 0) & (k + dz < nz))
        valid.append(ok)
        nbr.append((i + dx) + nx * ((j + dy) + ny * (k + dz)))
    return _pattern(np.stack(valid, 1), np.stack(nbr, 1))


# --------------------------------------------------------------------------
# Flow state, fluxes and residual (used for the Jacobian and for FD checks)
# --------------------------------------------------------------------------
def faces(nx, ny, nz):
    """Internal faces: (K, L, axis) with L = K + stride, K < L."""
    i, j, k = _cell_ijk(nx, ny, nz)
    cid = np.arange(nx * ny * nz)
    out = []
    for axis, (ok, stride) in enumerate([(i < nx - 1, 1), (j < ny - 1, nx), (k < nz - 1, nx * ny)]):
        K = cid[ok]
        out.append((K, K + stride, np.full(K.shape, axis)))
    K = np.concatenate([o[0] for o in out])
    L = np.concatenate([o[1] for o in out])
    ax = np.concatenate([o[2] for o in out])
    return K, L, ax


def transmissibility(kperm, h, K, L):
    """App. A: harmonic mean of half transmissibilities on a cube grid.

    For a cube, Upsilon^{f,K} = |f| kappa_K / (h/2) = 2 h kappa_K.
    """
    tK = 2.0 * h * kperm[K]
    tL = 2.0 * h * kperm[L]
    return tK * tL / (tK + tL)


def flow_residual(S, p, epsv, props):
    """Flow residual (mass balance of each phase) per cell, shape (n_cells, nph).

    Accumulation at the new time level only (the old-time term is a constant of the
    linearisation); face terms with the physically consistent sign.
    """
    ph, V, h, dt = props["phases"], props["V"], props["h"], props["dt"]
    phi = props["phi0"] + props["biot"] * epsv
    rho = ph.rho0[None, :] * (1.0 + ph.comp[None, :] * (p - props["p0"])[:, None])
    s = ph.saturations(S)
    kr, _ = ph.kr(S)
    lam = kr / ph.mu[None, :]
    R = V * phi[:, None] * rho * s
    K, L, T, zc = props["fK"], props["fL"], props["T"], props["zc"]
    for l in range(ph.nph):
        rav = 0.5 * (rho[K, l] + rho[L, l])
        Phi = T * ((p[L] - p[K]) + rav * GRAV * (zc[L] - zc[K]))
        up = np.where(Phi > 0, L, K)
        F = rho[up, l] * lam[up, l] * Phi
        np.add.at(R[:, l], K, -dt * F)
        np.add.at(R[:, l], L, dt * F)
    return R


def flow_jacobian(S, p, props):
    """Analytic flow Jacobian d R / d [S, p], App. B formulas, as dense per-face
    contributions.  Returns (diag_blocks (n,nph,nf), face list of (K, L, dK, dL))
    where dK/dL are d(F-terms)/d(cell K or L dofs) added to rows K (with -dt) and L (+dt).
    """
    ph, V, dt = props["phases"], props["V"], props["dt"]
    n, nph, nf = S.shape[0], ph.nph, ph.nph
    phi = props["phi0"]
    rho = ph.rho0[None, :] * (1.0 + ph.comp[None, :] * (p - props["p0"])[:, None])
    drho = (ph.rho0 * ph.comp)[None, :] * np.ones((n, 1))
    s = ph.saturations(S)
    kr, dkr = ph.kr(S)
    lam = kr / ph.mu[None, :]
    ds = ph.dsat()
    acc = np.zeros((n, nph, nf))
    for l in range(nph):
        acc[:, l, : nf - 1] = V * phi[:, None] * rho[:, l: l + 1] * ds[l][None, :]
        acc[:, l, nf - 1] = V * phi * s[:, l] * drho[:, l]
    K, L, T, zc = props["fK"], props["fL"], props["T"], props["zc"]
    nfaces = K.shape[0]
    dK = np.zeros((nfaces, nph, nf))   # dF_l / d dofs of K
    dL = np.zeros((nfaces, nph, nf))
    for l in range(nph):
        rav = 0.5 * (rho[K, l] + rho[L, l])
        dz = zc[L] - zc[K]
        Phi = T * ((p[L] - p[K]) + rav * GRAV * dz)
        upL = Phi > 0
        up = np.where(upL, L, K)
        rup, lup = rho[up, l], lam[up, l]
        # pressure derivatives
        common = rup * lup * T
        dK[:, l, nf - 1] = common * (-1.0 + 0.5 * drho[K, l] * GRAV * dz)
        dL[:, l, nf - 1] = common * (1.0 + 0.5 * drho[L, l] * GRAV * dz)
        dup_p = drho[up, l] * lup * Phi
        dK[:, l, nf - 1] += np.where(upL, 0.0, dup_p)
        dL[:, l, nf - 1] += np.where(upL, dup_p, 0.0)
        # saturation derivatives: only through the upwind cell's mobility
        dsat = (rup / ph.mu[l] * Phi)[:, None] * dkr[up, l, :]
        dK[:, l, : nf - 1] += np.where(upL[:, None], 0.0, dsat)
        dL[:, l, : nf - 1] += np.where(upL[:, None], dsat, 0.0)
    return acc, dK, dL


# --------------------------------------------------------------------------
# Assembly
# --------------------------------------------------------------------------
def assemble(nx, ny, nz, fields, phases, h=10.0, dt=86400.0, nu=0.25, biot=1.0, rho_s=2650.0):
    """Unscaled Jacobian blocks and fixed-stress diagonals for the given cell fields.

    fields: dict with per-cell arrays E, kperm, phi, S (n, nph-1), p, p0.
    """
    nc = nx * ny * nz
    nn = (nx + 1) * (ny + 1) * (nz + 1)
    nph = phases.nph
    nf = nph
    E, kperm, phi, S, p, p0 = (fields[k] for k in ("E", "kperm", "phi", "S", "p", "p0"))
    Kref, Gd, Gn, V = q1_cube(h, nu)
    ci, cj, ck = _cell_ijk(nx, ny, nz)
    sx, sxy = nx + 1, (nx + 1) * (ny + 1)
    base = ci + sx * cj + sxy * ck
    loc = [(a & 1, (a >> 1) & 1, (a >> 2) & 1) for a in range(8)]
    node_of = [base + ax + sx * ay + sxy * az for (ax, ay, az) in loc]

    s = phases.saturations(S)
    rho = phases.rho0[None, :] * (1.0 + phases.comp[None, :] * (p - p0)[:, None])
    # mixture-density derivatives (App. B.2), b = 1 and incompressible grains; the one in
    # A_uu at the reference state (equal saturations, reference densities)
    drho_deps = np.full(nc, (-rho_s + phases.rho0.mean()) * biot)
    drho_dp = phi * (s * (phases.rho0 * phases.comp)[None, :]).sum(1)
    drho_dS = phi[:, None] * (rho @ phases.dsat())        # (n, nph-1)

    # ---- A_uu -------------------------------------------------------------
    rp, ci_, slot = node_node_pattern(nx, ny, nz)
    Auu = np.zeros((ci_.shape[0], 3, 3))
    for a in range(8):
        ax, ay, az = loc[a]
        na = node_of[a]
        for b in range(8):
            bx, by, bz = loc[b]
            d = (bz - az + 1) * 9 + (by - ay + 1) * 3 + (bx - ax + 1)
            sl = slot[na, d]
            blk = E[:, None, None] * Kref[a, :, b, :][None, :, :]
            # gravity term: -int eta_i . (drho/deps g) div eta_j ; g = (0, 0, -GRAV)
            blk[:, 2, :] += GRAV * drho_deps[:, None] * Gn[a, b, :][None, :]
            Auu[sl] += blk
    A_uu = BSR(rp, ci_, Auu, nn)

    # ---- A_uf (node rows, cell cols): columns [S_0..S_{nf-2}, p] ------------
    rp, ci_, slot = node_cell_pattern(nx, ny, nz)
    Auf = np.zeros((ci_.shape[0], 3, nf))
    for a in range(8):
        ax, ay, az = loc[a]
        sl = slot[node_of[a], (1 - az) * 4 + (1 - ay) * 2 + (1 - ax)]
        blk = np.zeros((nc, 3, nf))
        blk[:, :, nf - 1] = -biot * Gd[a][None, :]
        blk[:, 2, nf - 1] += GRAV * drho_dp * V / 8.0
        blk[:, 2, : nf - 1] += GRAV * drho_dS * V / 8.0
        Auf[sl] += blk
    A_uf = BSR(rp, ci_, Auf, nc)

    # ---- A_fu (cell rows, node cols) ----------------------------------------
    rp, ci_, _ = cell_node_pattern(nx, ny, nz)
    Afu = np.zeros((nc, 8, nf, 3))
    for a in range(8):
        Afu[:, a, :, :] = (s * rho)[:, :, None] * biot * Gd[a][None, None, :]
    A_fu = BSR(rp, ci_, Afu.reshape(nc * 8, nf, 3), nn)

    # ---- A_ff ---------------------------------------------------------------
    rp, ci_, slot = cell_cell_pattern(nx, ny, nz)
    Aff = np.zeros((ci_.shape[0], nf, nf))
    zc = (ck + 0.5) * h
    fK, fL, fax = faces(nx, ny, nz)
    T = transmissibility(kperm, h, fK, fL)
    props = dict(phases=phases, V=V, h=h, dt=dt, phi0=phi, biot=biot, p0=p0,
                 fK=fK, fL=fL, T=T, zc=zc)
    acc, dK, dL = flow_jacobian(S, p, props)
    Aff[slot[:, 3]] += acc
    # slots: offset index of L seen from K is the "+axis" offset, of K seen from L the "-axis"
    plus = {0: 4, 1: 5, 2: 6}
    minus = {0: 2, 1: 1, 2: 0}
    sKK = slot[fK, 3]
    sLL = slot[fL, 3]
    sKL = slot[fK, np.vectorize(plus.get)(fax)] if fK.size else fK
    sLK = slot[fL, np.vectorize(minus.get)(fax)] if fK.size else fK
    # rows K get -dt * dF, rows L get +dt * dF (no duplicate slots within one call)
    np.add.at(Aff, sKK, -dt * dK)
    np.add.at(Aff, sKL, -dt * dL)
    np.add.at(Aff, sLK, dt * dK)
    np.add.at(Aff, sLL, dt * dL)
    A_ff = BSR(rp, ci_, Aff, nc)

    # ---- fixed-stress diagonals (eq. FS_Dps_Dpp) ----------------------------
    Kdr = E / (3.0 * (1.0 - 2.0 * nu))
    fs = V * biot ** 2 / Kdr
    d_sp = fs[:, None] * s[:, : nf - 1] * rho[:, : nf - 1]
    d_pp = fs * s[:, nf - 1] * rho[:, nf - 1]
    return dict(Auu=A_uu, Auf=A_uf, Afu=A_fu, Aff=A_ff, d_sp=d_sp, d_pp=d_pp,
                props=props, nn=nn, nc=nc)


def constrained_mask(nx, ny, nz):
    """Bottom fixed (all comps), x-sides u_x = 0, y-sides u_y = 0, top free."""
    i, j, k = _node_ijk(nx, ny, nz)
    m = np.zeros((i.shape[0], 3), bool)
    m[k == 0, :] = True
    m[(i == 0) | (i == nx), 0] = True
    m[(j == 0) | (j == ny), 1] = True
    return m


def apply_bc(parts, mask):
    A = parts["Auu"]
    rows = np.repeat(np.arange(A.nbrows), np.diff(A.rowptr))
    cols = A.colind
    kill = mask[rows][:, :, None] | mask[cols][:, None, :]
    diag = (rows == cols)[:, None, None] & np.eye(3, dtype=bool)[None]
    A.vals[kill & ~diag] = 0.0
    B = parts["Auf"]
    rows = np.repeat(np.arange(B.nbrows), np.diff(B.rowptr))
    B.vals[mask[rows]] = 0.0
    C = parts["Afu"]
    C.vals[np.broadcast_to(mask[C.colind][:, None, :], C.vals.shape)] = 0.0


def apply_scaling(parts, nf):
    A = parts["Auu"]
    rows = np.repeat(np.arange(A.nbrows), np.diff(A.rowptr))
    dmask = rows == A.colind
    du = np.abs(np.diagonal(A.vals[dmask], axis1=1, axis2=2)).ravel()
    cu = float(np.mean(du) ** -0.5)
    F = parts["Aff"]
    rows = np.repeat(np.arange(F.nbrows), np.diff(F.rowptr))
    fd = np.abs(np.diagonal(F.vals[rows == F.colind], axis1=1, axis2=2))   # (nc, nf)
    cf = np.mean(fd, axis=0) ** -0.5
    A.vals *= cu * cu
    parts["Auf"].vals *= cu * cf[None, None, :]
    parts["Afu"].vals *= cf[None, :, None] * cu
    F.vals *= cf[None, :, None] * cf[None, None, :]
    parts["d_sp"] = parts["d_sp"] * (cf[: nf - 1] * cf[nf - 1])[None, :]
    parts["d_pp"] = parts["d_pp"] * cf[nf - 1] ** 2
    return cu, cf


def build_system(nx, ny, nz, fields, phases, **kw):
    parts = assemble(nx, ny, nz, fields, phases, **kw)
    mask = constrained_mask(nx, ny, nz)
    apply_bc(parts, mask)
    cu, cf = apply_scaling(parts, phases.nph)
    nf = phases.nph
    return PoroSystem(nx=nx, ny=ny, nz=nz, nf=nf, p_index=nf - 1,
                      Auu=parts["Auu"], Auf=parts["Auf"], Afu=parts["Afu"], Aff=parts["Aff"],
                      d_sp=np.ascontiguousarray(parts["d_sp"]), d_pp=np.ascontiguousarray(parts["d_pp"]),
                      constrained=mask.ravel(), scale_u=cu, scale_f=cf)


def make_rhs(system, seed):
    """N(0, 1) right-hand side on the scaled system, zero on constrained dofs."""
    rng = np.random.Generator(np.random.PCG64(seed))
    b = rng.standard_normal(system.N)
    b[: system.n_u][system.constrained] = 0.0
    return b


def box_partition(nx, ny, nz, bx, by, bz):
    """Subdomain id per cell for a partition into bx x by x bz-cell boxes (x fastest)."""
    i = np.tile(np.arange(nx), ny * nz)
    j = np.tile(np.repeat(np.arange(ny), nx), nz)
    k = np.repeat(np.arange(nz), nx * ny)
    px, py = -(-nx // bx), -(-ny // by)
    return ((i // bx) + px * ((j // by) + py * (k // bz))).astype(np.int32)
