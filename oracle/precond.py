"""Two-stage block preconditioner: setup and Algorithm 1 (oracle).

Paper Sec. 5.  The Jacobian is re-partitioned as [[A_uu, A_uf], [A_fu, A_ff]]
(eq. LU) and preconditioned with the block lower-triangular operator of
eq. blk_tr_prec, where
  * M_uu^{-1} = amg(A_uu^(sdc)), the separate-displacement-component approximation
    blockdiag(A_xx, A_yy, A_zz) (Sec. 5.2), i.e. one scalar AMG on the three
    components in component-major order;
  * A_us is dropped, so A_uf never enters the preconditioner (Sec. 5.1);
  * M_ff^{-1} = M_G^{-1} + M_L^{-1}(I - S_ff^(fs) M_G^{-1}) (eq. mult_prec_op), with
    S_ff^(fs) the fixed-stress Schur approximation (eq. Schur_1_FS: D_sp added to
    the (s, p) entries and D_pp to the (p, p) entry of each diagonal cell block),
    M_G^{-1} the quasi-IMPES global stage of eq. S1_prec (D_ss = diagm(A_ss),
    D_ps = diagm(A_ps), M_pp = amg(S_pp), full A_ps kept), and M_L the local stage.
Algorithm 1 applies it as: z_u = M_uu^{-1} v_u; y = v_f - A_fu z_u;
z_s = D_ss^{-1} y_s; w_p = y_p - A_ps z_s; z_p = M_pp^{-1} w_p;
w = y - S_ff^(fs) [z_s; z_p]; dz = M_L^{-1} w; z_f = [z_s; z_p] + dz.

Readings:
  * Multi-component flow (remarks in Sec. 5.1 / 5.3): D_ss and D_ps are the
    (nf-1)x(nf-1) and 1x(nf-1) parts of each diagonal cell block; small inverses
    use Cramer's rule.  nf = 2: t_i = D_ps,i / D_ss,i; nf = 3: t_i = D_ps,i D_ss,i^{-1}.
    S_pp[i, j] = A_pp^(fs)[i, j] - t_i . A_sp^(fs)[i, j] on the TPFA pattern.
  * Step 6 uses S_ff^(fs) (the matrix M_ff approximates), not A_ff.
  * Alternatives of Sec. 5.1 / 5.3: true-IMPES (column-sum lumping, eq. CPR_CSL; cell
    blocks summed over the block column for nf = 3) and the row-sum-lumped fixed-stress
    diagonals (eq. FS_RSL, A_uu^{-1} approximated by Richardson steps with M_uu).
  * The local stage acts on all flow (cell) unknowns; displacement is untouched.
Test infrastructure only.
"""
from dataclasses import dataclass
import numpy as np
import scipy.sparse as sp

from . import amg
from . import local


@dataclass
class Options:
    restart: int = 100
    maxit: int = 1000
    theta: float = 0.25
    coarse_max: int = 256
    max_levels: int = 25
    smoother: str = "cheb2"        # "cheb2" | "l1jac"
    ml_kind: str = "bilu0"         # "bilu0" | "bjacobi" | "mcgs"
    ml_sweeps: int = 1             # sweeps of the local stage (BILU(0) or block Jacobi)
    method: str = "fgmres"         # "fgmres" | "richardson" (sequential fixed-stress scheme)
    reduction: str = "quasi"       # "quasi" | "true" (IMPES reduction, Sec. 5.3)
    fixed_stress: str = "given"    # "given" (the system's d_sp, d_pp) | "rsl" (eq. FS_RSL)
    fs_iters: int = 10             # RSL: Richardson steps with the mechanics V-cycle for A_uu^-1
    orth: str = "cgs2"             # FGMRES Arnoldi step: "cgs2" | "dcgs2" (delayed re-orthogonalisation)


def bsr_to_csr(rowptr, colind, vals, ncols_blocks):
    """Scalar CSR expansion of a block CSR matrix (explicit zeros kept)."""
    rowptr = np.asarray(rowptr, np.int64)
    colind = np.asarray(colind, np.int64)
    vals = np.asarray(vals, np.float64)
    nb, br, bc = vals.shape
    nbr = rowptr.shape[0] - 1
    brow = np.repeat(np.arange(nbr), np.diff(rowptr))
    r = (brow[:, None, None] * br + np.arange(br)[None, :, None]) + 0 * np.arange(bc)[None, None, :]
    c = (colind[:, None, None] * bc + np.arange(bc)[None, None, :]) + 0 * np.arange(br)[None, :, None]
    M = sp.csr_matrix((vals.ravel(), (r.ravel(), c.ravel())), shape=(nbr * br, ncols_blocks * bc))
    M.sort_indices()
    return M


def system_matrices(system):
    """Scalar CSR matrices of the four blocks and of the full Jacobian."""
    s = system
    Auu = bsr_to_csr(s.Auu.rowptr, s.Auu.colind, s.Auu.vals, s.n_nodes)
    Auf = bsr_to_csr(s.Auf.rowptr, s.Auf.colind, s.Auf.vals, s.n_cells)
    Afu = bsr_to_csr(s.Afu.rowptr, s.Afu.colind, s.Afu.vals, s.n_nodes)
    Aff = bsr_to_csr(s.Aff.rowptr, s.Aff.colind, s.Aff.vals, s.n_cells)
    A = sp.bmat([[Auu, Auf], [Afu, Aff]], format="csr")
    A.sort_indices()
    return dict(A=A, Auu=Auu, Auf=Auf, Afu=Afu, Aff=Aff)


def _diag_positions(rowptr, colind):
    n = rowptr.shape[0] - 1
    brow = np.repeat(np.arange(n), np.diff(rowptr))
    pos = np.nonzero(brow == colind)[0]
    if pos.shape[0] != n:
        raise ValueError("every block row needs its diagonal block")
    return pos


def fixed_stress(system, d_sp=None, d_pp=None):
    """Block values of S_ff^(fs) (eq. Schur_1_FS with the diagonals of eq. FS_Dps_Dpp,
    or the given ones)."""
    nf = system.nf
    d_sp = system.d_sp if d_sp is None else d_sp
    d_pp = system.d_pp if d_pp is None else d_pp
    vals = np.array(system.Aff.vals, np.float64, copy=True)
    dpos = _diag_positions(system.Aff.rowptr, system.Aff.colind)
    for l in range(nf - 1):
        vals[dpos, l, nf - 1] += d_sp[:, l]
    vals[dpos, nf - 1, nf - 1] += d_pp
    return vals


def rsl_diagonals(system, mats, sdc, smoother, iters):
    """Fixed-stress diagonals by row-sum lumping (remark after eq. FS_Dps_Dpp, eq. FS_RSL):
    D_sp = -diag(A_su A_uu^{-1} A_up e), D_pp = -diag(A_pu A_uu^{-1} A_up e), e = 1 on the
    pressure unknowns.  The paper allows a good preconditioner of A_uu in place of the
    inverse; reading: y = A_uu^{-1} g is approximated by `iters` Richardson steps
    y += M_uu^{-1}(g - A_uu y) from y = 0, M_uu the mechanics V-cycle of step 1.
    Returns (d_sp (n_cells, nf-1), d_pp (n_cells,))."""
    nf, nc = system.nf, system.n_cells
    e = np.zeros(nf * nc)
    e[nf - 1::nf] = 1.0
    g = mats["Auf"] @ e                      # A_up e (the saturation columns get 0)
    Auu = mats["Auu"]
    y = np.zeros(g.shape[0])
    for _ in range(iters):
        y = y + _sdc_apply(sdc, g - Auu @ y, smoother)
    w = (mats["Afu"] @ y).reshape(nc, nf)     # rows s and p of A_fu y
    return -w[:, : nf - 1].copy(), -w[:, nf - 1].copy()


def column_sum_blocks(system):
    """Per cell i the sum over block rows k of A_ff[k, i] (nf x nf), rows k in increasing
    order: the column-sum lumping of eq. CPR_CSL (true-IMPES), whose s-column part gives
    D_ss = diag(A_ss^T e) and D_ps = diag(A_ps^T e); for nf = 3 the cell blocks of the
    multi-component remark (Sec. 5.3)."""
    nf = system.nf
    out = np.zeros((system.n_cells, nf, nf))
    np.add.at(out, system.Aff.colind, system.Aff.vals)
    return out


def inv2(a, b, c, d):
    """Cramer inverse of [[a, b], [c, d]] (arrays), returned as four arrays."""
    det = a * d - b * c
    return d / det, -b / det, -c / det, a / det


def quasi_impes(system, sff_vals, reduction="quasi"):
    """IMPES-reduced pressure matrix S_pp (scalar CSR on the cell pattern) and D_ss^{-1}:
    quasi-IMPES (D_ss, D_ps from the diagonal cell blocks, diagm) or true-IMPES (from the
    column sums, eq. CPR_CSL)."""
    nf = system.nf
    rowptr, colind = system.Aff.rowptr, system.Aff.colind
    aff = system.Aff.vals
    if reduction == "true":
        D = column_sum_blocks(system)
    else:
        D = aff[_diag_positions(rowptr, colind)]
    Dss = D[:, : nf - 1, : nf - 1]
    Dps = D[:, nf - 1, : nf - 1]
    if nf == 2:
        t = (Dps[:, 0] / Dss[:, 0, 0])[:, None]
        dss_inv = (1.0 / Dss[:, 0, 0])[:, None, None]
    elif nf == 3:
        i00, i01, i10, i11 = inv2(Dss[:, 0, 0], Dss[:, 0, 1], Dss[:, 1, 0], Dss[:, 1, 1])
        t = np.stack([Dps[:, 0] * i00 + Dps[:, 1] * i10, Dps[:, 0] * i01 + Dps[:, 1] * i11], 1)
        dss_inv = np.stack([np.stack([i00, i01], 1), np.stack([i10, i11], 1)], 1)
    else:
        raise ValueError("nf must be 2 or 3")
    brow = np.repeat(np.arange(system.n_cells), np.diff(rowptr))
    app = sff_vals[:, nf - 1, nf - 1]
    asp = sff_vals[:, : nf - 1, nf - 1]
    if nf == 2:
        spp = app - t[brow, 0] * asp[:, 0]
    else:
        spp = app - (t[brow, 0] * asp[:, 0] + t[brow, 1] * asp[:, 1])
    S = sp.csr_matrix((spp, colind.astype(np.int64), rowptr.astype(np.int64)),
                      shape=(system.n_cells, system.n_cells))
    return S, dss_inv


def sdc_matrix(system):
    """A_uu^(sdc) = blockdiag(A_xx, A_yy, A_zz) in component-major order (Sec. 5.2)."""
    nn = system.n_nodes
    rowptr, colind, vals = system.Auu.rowptr, system.Auu.colind, system.Auu.vals
    blocks = []
    for c in range(3):
        blocks.append(sp.csr_matrix((vals[:, c, c].copy(), colind.astype(np.int64),
                                     rowptr.astype(np.int64)), shape=(nn, nn)))
    A = sp.block_diag(blocks, format="csr")
    A.sort_indices()
    return A


@dataclass
class Setup:
    system: object
    opts: Options
    mats: dict
    sff_vals: np.ndarray
    Sff: sp.csr_matrix
    Spp: sp.csr_matrix
    dss_inv: np.ndarray
    Aps: sp.csr_matrix
    sdc: list
    pres: list
    ml: tuple


def setup(system, opts=None, mechanics=None):
    """Setup phase (Sec. 5.4): operators and sub-preconditioners.

    mechanics: an existing SDC hierarchy to reuse (the elasticity AMG is set up once
    per simulation, Sec. 5.2).
    """
    opts = opts or Options()
    if system.p_index != system.nf - 1:
        raise ValueError("pressure must be the last cell dof")
    mats = system_matrices(system)
    kw = dict(theta=opts.theta, coarse_max=opts.coarse_max, max_levels=opts.max_levels,
              smoother=opts.smoother)
    sdc = mechanics if mechanics is not None else amg.build(sdc_matrix(system), **kw)
    if opts.fixed_stress == "rsl":
        d_sp, d_pp = rsl_diagonals(system, mats, sdc, opts.smoother, opts.fs_iters)
    else:
        d_sp, d_pp = system.d_sp, system.d_pp
    sff_vals = fixed_stress(system, d_sp, d_pp)
    Sff = bsr_to_csr(system.Aff.rowptr, system.Aff.colind, sff_vals, system.n_cells)
    Spp, dss_inv = quasi_impes(system, sff_vals, opts.reduction)
    nf = system.nf
    # A_ps: pressure rows, saturation columns of A_ff (unchanged by fixed stress)
    Aps = bsr_to_csr(system.Aff.rowptr, system.Aff.colind,
                     np.ascontiguousarray(system.Aff.vals[:, nf - 1: nf, : nf - 1]), system.n_cells)
    pres = amg.build(Spp, **kw)
    part = getattr(system, "ml_part", None)
    if opts.ml_kind == "bilu0" and part is not None:
        rp, ci, vals = local.restrict_to_parts(system.Aff.rowptr, system.Aff.colind, sff_vals, part)
        ml = ("bilu0",) + local.bilu0_factor(rp, ci, vals) + (rp, ci)
    elif opts.ml_kind == "bilu0":
        ml = ("bilu0",) + local.bilu0_factor(system.Aff.rowptr, system.Aff.colind, sff_vals) + (
            system.Aff.rowptr, system.Aff.colind)
    elif opts.ml_kind == "bjacobi":
        ml = ("bjacobi", local.block_diag_inv(system.Aff.rowptr, system.Aff.colind, sff_vals))
    elif opts.ml_kind == "mcgs":
        ml = ("mcgs", local.block_diag_inv(system.Aff.rowptr, system.Aff.colind, sff_vals),
              local.greedy_colors(system.Aff.rowptr, system.Aff.colind))
    else:
        raise ValueError(opts.ml_kind)
    return Setup(system, opts, mats, sff_vals, Sff, Spp, dss_inv, Aps, sdc, pres, ml)


def alg1(v, n_u, nf, Muu, Afu, dss_solve, Aps, Mpp, Sff, ML):
    """Algorithm 1 with the sub-operators passed in (steps 1-8)."""
    v_u, v_f = v[:n_u], v[n_u:]
    z_u = Muu(v_u)                                    # step 1
    y = v_f - Afu @ z_u                               # step 2
    yc = y.reshape(-1, nf)
    z_s = dss_solve(yc[:, : nf - 1])                  # step 3
    w_p = yc[:, nf - 1] - Aps @ z_s.ravel()           # step 4
    z_p = Mpp(w_p)                                    # step 5
    zf = np.concatenate([z_s, z_p[:, None]], axis=1).ravel()
    w = y - Sff @ zf                                  # step 6
    dz = ML(w)                                        # step 7
    return np.concatenate([z_u, zf + dz])             # step 8


def _sdc_apply(levels, v_u, kind):
    nn = v_u.shape[0] // 3
    x = amg.vcycle(levels, v_u.reshape(nn, 3).T.ravel(), kind)
    return x.reshape(3, nn).T.ravel()


def apply_precond(st, v):
    """z = M^{-1} v for the configured preconditioner."""
    s, o = st.system, st.opts
    nf = s.nf

    def Muu(vu):
        return _sdc_apply(st.sdc, vu, o.smoother)

    def dss_solve(ys):
        return np.einsum("nij,nj->ni", st.dss_inv, ys)

    def Mpp(wp):
        return amg.vcycle(st.pres, wp, o.smoother)

    if st.ml[0] == "bilu0":
        _, F, Dinv, diag, lrp, lci = st.ml

        def ML(w):
            return local.bilu0_sweeps(lrp, lci, F, Dinv, diag, st.Sff, w.reshape(-1, nf), o.ml_sweeps).ravel()
    elif st.ml[0] == "mcgs":
        Dinv, colors = st.ml[1], st.ml[2]

        def ML(w):
            return local.mcgs_apply(st.Sff, Dinv, colors, w.reshape(-1, nf), o.ml_sweeps).ravel()
    else:
        Dinv = st.ml[1]

        def ML(w):
            return local.bjacobi_apply(st.Sff, Dinv, w.reshape(-1, nf), o.ml_sweeps).ravel()

    return alg1(v, s.n_u, nf, Muu, st.mats["Afu"], dss_solve, st.Aps, Mpp, st.Sff, ML)
