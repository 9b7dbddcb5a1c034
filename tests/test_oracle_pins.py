"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: dense direct
solves, closed forms, brute force on tiny inputs, or a different formula the paper
states for the same operator.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from synth import workload
from oracle import Options, solve
from oracle import amg, local
from oracle import precond as P
from oracle.fgmres import fgmres
from oracle.rng import splitmix64


# ---------------------------------------------------------------------------- rng
def test_splitmix64_reference_value():
    # First output of SplitMix64 seeded with 0 (published reference implementation).
    with np.errstate(over="ignore"):
        assert int(splitmix64(np.uint64(0))) == 0xE220A8397B1DCDAF


# ---------------------------------------------------------------------------- fixtures
def tiny(kind="iid", grid=(3, 3, 2), seed=11):
    return workload(grid=grid, kind=kind, seed=seed, rhs_seed=seed + 100)


def dense(m):
    return np.asarray(m.todense())


def perms(s):
    """Index arrays splitting the interleaved cell vector into s- and p-parts."""
    nf = s.nf
    cells = np.arange(s.n_cells)
    sidx = (cells[:, None] * nf + np.arange(nf - 1)[None, :]).ravel()
    pidx = cells * nf + nf - 1
    return sidx, pidx


# ---------------------------------------------------------------------------- solve
ORTHS = ("cgs2", "dcgs2")


@pytest.mark.parametrize("orth", ORTHS)
def test_fgmres_matches_dense_direct_solve(iid8, orth):
    s, b = iid8
    out = solve(s, b, rtol=1e-10, opts=Options(orth=orth))
    A = dense(out["setup"].mats["A"])
    x = np.linalg.solve(A, b)
    assert out["status"] == 0 and out["rel_residual"] <= 1e-10
    # relative error bounded by cond(A) * relative residual
    cond = np.linalg.cond(A)
    err = np.linalg.norm(out["x"] - x) / np.linalg.norm(x)
    assert err <= cond * out["rel_residual"]
    assert err <= 1e-6


def test_exact_solution_recovery():
    s, _ = tiny(grid=(4, 3, 3))
    st = P.setup(s)
    xs = np.random.default_rng(7).standard_normal(s.N)
    xs[: s.n_u][s.constrained] = 0.0
    b = st.mats["A"] @ xs
    out = solve(s, b, rtol=1e-12, setup_result=st)
    assert np.linalg.norm(out["x"] - xs) / np.linalg.norm(xs) < 1e-6


def test_exact_subsolves_converge_in_two_iterations():
    """With M_uu = A_uu^{-1} and the true Schur complement S_ff handled exactly,
    L^{-1} A = U has all eigenvalues 1 and (U - I)^2 = 0 (Sec. 5.1), so FGMRES stops in
    at most two iterations."""
    s, b = tiny(grid=(3, 2, 2))
    st = P.setup(s)
    M = st.mats
    Auu, Auf, Afu, Aff = (dense(M[k]) for k in ("Auu", "Auf", "Afu", "Aff"))
    Auu_inv = np.linalg.inv(Auu)
    S_true = Aff - Afu @ Auu_inv @ Auf
    S_inv = np.linalg.inv(S_true)
    nf = s.nf

    def prec(v):
        return P.alg1(v, s.n_u, nf, lambda vu: Auu_inv @ vu, M["Afu"],
                      lambda ys: np.einsum("nij,nj->ni", st.dss_inv, ys), st.Aps,
                      lambda wp: amg.vcycle(st.pres, wp), sp.csr_matrix(S_true),
                      lambda w: S_inv @ w)

    A = M["A"]
    # (A M^{-1} - I)^2 = L (U - I)^2 L^{-1} = 0 up to rounding
    B = dense(A) @ _mat_of(prec, s.N) - np.eye(s.N)
    assert np.abs(B @ B).max() <= 1e-12 * np.abs(B).max() ** 2
    # so the second FGMRES iterate is exact up to cond(S_ff) * eps (cond ~ 1e10 here)
    out = fgmres(lambda v: A @ v, prec, b, rtol=1e-30, restart=20, maxit=2)
    assert out["history"][1] <= 1e-8


def _mat_of(fn, n):
    return np.stack([fn(e) for e in np.eye(n)], axis=1)


@pytest.mark.parametrize("ml_kind,sweeps", [("bilu0", 1), ("bilu0", 2), ("bjacobi", 3), ("mcgs", 3)])
def test_algorithm1_equals_multistage_formula(ml_kind, sweeps):
    """Steps 3-8 of Alg. 1 equal M_G^{-1} + M_L^{-1}(I - S M_G^{-1}) (eq. mult_prec_op) with
    M_G^{-1} the product of eq. S1_prec, and the whole of Alg. 1 equals the product form of
    eq. blk_tr_prec."""
    s, _ = tiny(grid=(3, 2, 2))
    opts = Options(ml_kind=ml_kind, ml_sweeps=sweeps)
    st = P.setup(s, opts)
    nf, nu, nfl = s.nf, s.n_u, s.n_f
    sidx, pidx = perms(s)
    ns = sidx.size
    Sff = dense(st.Sff)
    # dense sub-operators (all linear maps)
    Mpp = _mat_of(lambda w: amg.vcycle(st.pres, w), s.n_cells)
    Dss_inv = sla.block_diag(*st.dss_inv)
    Aps = dense(st.Aps)
    # M_G^{-1} in (s, p)-partitioned order, eq. S1_prec
    I_s, I_p = np.eye(ns), np.eye(s.n_cells)
    T1 = sla.block_diag(Dss_inv, I_p)
    T2 = np.block([[I_s, np.zeros((ns, s.n_cells))], [-Aps, I_p]])
    T3 = sla.block_diag(I_s, Mpp)
    MG_part = T3 @ T2 @ T1
    perm = np.concatenate([sidx, pidx])
    MG = np.zeros((nfl, nfl))
    MG[np.ix_(perm, perm)] = MG_part
    if ml_kind == "bilu0":
        _, F, Dinv, diag = st.ml[:4]
        ML1 = _mat_of(lambda w: local.bilu0_apply(s.Aff.rowptr, s.Aff.colind, F, Dinv, diag,
                                                   w.reshape(-1, nf)).ravel(), nfl)
    elif ml_kind == "mcgs":
        ML1 = _mat_of(lambda w: local.mcgs_apply(st.Sff, st.ml[1], st.ml[2], w.reshape(-1, nf), 1).ravel(), nfl)
    else:
        ML1 = sla.block_diag(*st.ml[1])
    # k sweeps of a stationary iteration with B: M_L = sum_{i<k} (I - B S)^i B
    ML = np.zeros_like(ML1)
    E = np.eye(nfl)
    for _ in range(sweeps):
        ML += E @ ML1
        E = E @ (np.eye(nfl) - ML1 @ Sff)
    Mff = MG + ML @ (np.eye(nfl) - Sff @ MG)
    # top level, eq. blk_tr_prec: [I; Mff] [I; -Afu I] [Muu; I]
    Muu = _mat_of(lambda v: P._sdc_apply(st.sdc, v, opts.smoother), nu)
    Afu = dense(st.mats["Afu"])
    N = s.N
    L1 = sla.block_diag(Muu, np.eye(nfl))
    L2 = np.block([[np.eye(nu), np.zeros((nu, nfl))], [-Afu, np.eye(nfl)]])
    L3 = sla.block_diag(np.eye(nu), Mff)
    M_formula = L3 @ L2 @ L1
    M_alg = _mat_of(lambda v: P.apply_precond(st, v), N)
    assert np.abs(M_alg - M_formula).max() <= 1e-10 * np.abs(M_formula).max()


def test_exact_local_stage_gives_exact_schur_inverse():
    """With M_L = S^{-1}, M_ff^{-1} = S^{-1} whatever M_G is (eq. mult_prec_op)."""
    s, _ = tiny(grid=(3, 2, 2))
    st = P.setup(s)
    S = dense(st.Sff)
    S_inv = np.linalg.inv(S)
    w = np.random.default_rng(1).standard_normal(s.n_f)
    z = P.alg1(np.concatenate([np.zeros(s.n_u), w]), s.n_u, s.nf, lambda vu: np.zeros_like(vu),
               st.mats["Afu"], lambda ys: np.einsum("nij,nj->ni", st.dss_inv, ys), st.Aps,
               lambda wp: amg.vcycle(st.pres, wp), st.Sff, lambda r: S_inv @ r)[s.n_u:]
    assert np.allclose(z, S_inv @ w, rtol=1e-9, atol=1e-12 * np.abs(S_inv @ w).max())


# ---------------------------------------------------------------------------- setup
@pytest.mark.parametrize("kind", ["iid", "iid3"])
def test_fixed_stress_and_quasi_impes_dense(kind):
    s, _ = tiny(kind=kind, grid=(3, 3, 2))
    st = P.setup(s)
    nf = s.nf
    sidx, pidx = perms(s)
    Aff = dense(st.mats["Aff"])
    Sff = dense(st.Sff)
    # fixed stress only adds D_sp to (s, p) and D_pp to (p, p) of each cell's diagonal
    D = Sff - Aff
    expect = np.zeros_like(D)
    for c in range(s.n_cells):
        for l in range(nf - 1):
            expect[c * nf + l, c * nf + nf - 1] = s.d_sp[c, l]
        expect[c * nf + nf - 1, c * nf + nf - 1] = s.d_pp[c]
    assert np.all(np.abs(D - expect) <= 4e-16 * (np.abs(Aff) + np.abs(expect)))
    assert np.all(D[expect == 0] == 0.0)
    # quasi-IMPES: S_pp = A_pp^fs - D_ps D_ss^{-1} A_sp^fs with diagm (block-diagonal) parts
    Ass = Aff[np.ix_(sidx, sidx)]
    Aps = Aff[np.ix_(pidx, sidx)]
    m = nf - 1
    Dss = np.zeros_like(Ass)
    Dps = np.zeros_like(Aps)
    for c in range(s.n_cells):
        sl = slice(c * m, (c + 1) * m)
        Dss[sl, sl] = Ass[sl, sl]
        Dps[c, sl] = Aps[c, sl]
    Spp = Sff[np.ix_(pidx, pidx)] - Dps @ np.linalg.inv(Dss) @ Sff[np.ix_(sidx, pidx)]
    assert np.allclose(dense(st.Spp), Spp, rtol=1e-12, atol=1e-12 * np.abs(Spp).max())
    # sparsity: the TPFA 7-point stencil
    pat = np.zeros_like(Spp, bool)
    rows = np.repeat(np.arange(s.n_cells), np.diff(s.Aff.rowptr))
    pat[rows, s.Aff.colind] = True
    assert np.all(Spp[~pat] == 0.0)


def test_sdc_is_component_diagonal_part():
    s, _ = tiny(grid=(2, 2, 2))
    A = dense(P.system_matrices(s)["Auu"])
    nn = s.n_nodes
    perm = np.concatenate([np.arange(nn) * 3 + c for c in range(3)])
    Ap = A[np.ix_(perm, perm)]
    expect = np.zeros_like(Ap)
    for c in range(3):
        sl = slice(c * nn, (c + 1) * nn)
        expect[sl, sl] = Ap[sl, sl]
    assert np.array_equal(dense(P.sdc_matrix(s)), expect)


# ---------------------------------------------------------------------------- AMG
def poisson1d(n):
    return sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1], format="csr")


def poisson2d(n):
    T = poisson1d(n)
    I = sp.eye(n)
    return (sp.kron(T, I) + sp.kron(I, T)).tocsr()


def test_direct_interpolation_is_linear_on_1d_poisson():
    n = 9
    A = poisson1d(n)
    split = np.where(np.arange(n) % 2 == 1, amg.C_PT, amg.F_PT)
    lv = amg.build(A, coarse_max=1, max_levels=2, forced_split=[split], smoother="l1jac")
    P_ = dense(lv[0].P)
    expect = np.zeros((n, 4))
    for J in range(4):
        f = 2 * J + 1
        expect[f, J] = 1.0
        expect[f - 1, J] = 0.5
        expect[f + 1, J] = 0.5
    assert np.allclose(P_, expect, rtol=0, atol=1e-15)
    # Galerkin operator of linear interpolation: (1/2) tridiag(-1, 2, -1)
    assert np.allclose(dense(lv[1].A), 0.5 * dense(poisson1d(4)), rtol=0, atol=1e-15)


def test_pmis_split_invariants():
    A = poisson2d(20)
    smask = amg.strength(A, 0.25)
    state = amg.pmis(A, smask)
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    assert set(np.unique(state)) <= {amg.C_PT, amg.F_PT}
    # every F point with strong connections has a strong C neighbour (interpolation exists)
    hasc = np.zeros(A.shape[0], bool)
    hasc[rows[smask & (state[A.indices] == amg.C_PT)]] = True
    nS = np.bincount(rows[smask], minlength=A.shape[0])
    assert np.all(hasc | (state == amg.C_PT) | (nS == 0))
    nC = np.sum(state == amg.C_PT)
    assert 0.1 * A.shape[0] < nC < 0.6 * A.shape[0]
    # C points before promotion are never strongly connected to each other
    pre = amg.pmis(A, smask, promote=False)
    cpos = rows[smask]
    assert not np.any((pre[cpos] == amg.C_PT) & (pre[A.indices[smask]] == amg.C_PT))


def _aniso_graph(nx=7, ny=6, seed=5):
    """Non-symmetric 9-point operator on an nx x ny grid with random, anisotropic
    couplings, so that S is not symmetric and the weights differ from point to point."""
    rng = np.random.default_rng(seed)
    n = nx * ny
    A = sp.lil_matrix((n, n))
    for j in range(ny):
        for i in range(nx):
            r = i + nx * j
            for dj in (-1, 0, 1):
                for di in (-1, 0, 1):
                    ii, jj = i + di, j + dj
                    if (di, dj) == (0, 0) or not (0 <= ii < nx and 0 <= jj < ny):
                        continue
                    base = 1.0 if dj == 0 else (0.35 if di == 0 else 0.12)
                    A[r, ii + nx * jj] = -base * (0.5 + rng.random())
            A[r, r] = 6.0
    A = A.tocsr()
    A.sort_indices()
    return A


def _brute_pmis(A, theta):
    """PMIS (De Sterck, Yang, Heys) written out point by point from its definition:
    returns (state after round 1, state after all rounds, state after C-promotion),
    each a dict i -> 'C' | 'F' | 'U'."""
    from oracle.rng import unit
    n = A.shape[0]
    Ad = A.toarray()
    S = []
    for i in range(n):
        offs = {j: -Ad[i, j] for j in range(n) if j != i and A[i, j] != 0}
        m = max(offs.values()) if offs else -np.inf
        S.append({j for j, v in offs.items() if m > 0 and v >= theta * m})
    ST = [{k for k in range(n) if i in S[k]} for i in range(n)]
    w = [len(ST[i]) + float(unit(np.uint64(i))) for i in range(n)]
    state = {i: ("F" if len(ST[i]) == 0 else "U") for i in range(n)}
    snaps = []
    while any(v == "U" for v in state.values()):
        und = [i for i in range(n) if state[i] == "U"]
        newc = [i for i in und
                if all((w[i], i) > (w[j], j) for j in (S[i] | ST[i]) if state[j] == "U")]
        for i in newc:
            state[i] = "C"
        for k in und:
            if state[k] == "U" and any(state[c] == "C" and c in newc for c in S[k]):
                state[k] = "F"
        snaps.append(dict(state))
    after = dict(state)
    for i in range(n):
        if state[i] == "F" and S[i] and not any(state[j] == "C" for j in S[i]):
            state[i] = "C"
    return snaps[0], after, dict(state), S


def _as_letters(state):
    return {i: {amg.C_PT: "C", amg.F_PT: "F", amg.UNDEC: "U"}[int(v)] for i, v in enumerate(state)}


def test_pmis_brute_force_rounds():
    """PMIS round by round against a point-by-point brute force on a small
    non-symmetric graph: the first round's C set is exactly the points whose (w_i, i)
    beats every undecided neighbour in S_i u S_i^T, its F set the undecided points that
    strongly depend on a new C point; the final splitting (before and after C-promotion)
    matches, and C before promotion is independent in S u S^T."""
    A = _aniso_graph()
    smask = amg.strength(A, 0.25)
    first, before, final, S = _brute_pmis(A, 0.25)
    assert sum(v == "U" for v in first.values()) > 0          # the graph needs several rounds
    assert _as_letters(amg.pmis(A, smask, rounds=1, promote=False)) == first
    assert _as_letters(amg.pmis(A, smask, promote=False)) == before
    assert _as_letters(amg.pmis(A, smask)) == final
    C = [i for i, v in before.items() if v == "C"]
    for i in C:
        for j in C:
            assert j not in S[i], (i, j)
    # every F point with strong connections depends on a C point after promotion
    for i, v in final.items():
        if v == "F" and S[i]:
            assert any(final[j] == "C" for j in S[i])


def test_direct_interpolation_hand_computed_row():
    """One F row of direct interpolation worked by hand (Stueben): row 0 has a strong C
    neighbour (col 1, -2), a weak C neighbour (col 2, -0.3 < 0.25 * 2), a positive entry
    (col 3, +0.5) and a strong F neighbour (col 4, -1).
      atil_00 = 4 + 0.5 = 4.5 (positive entries lumped into the diagonal)
      alpha_0 = (-2 - 0.3 - 1) / (-2) = 1.65
      P_01    = -alpha_0 * (-2) / atil_00 = 3.3 / 4.5
    and no weight on the weak C neighbour or on the positive entry's column."""
    A = sp.csr_matrix(np.array([
        [4.0, -2.0, -0.3, 0.5, -1.0],
        [-1.0, 3.0, -1.0, 0.0, 0.0],
        [0.0, -1.0, 3.0, -1.0, 0.0],
        [0.0, 0.0, -1.0, 3.0, -1.0],
        [-1.0, 0.0, 0.0, -1.5, 4.0],
    ]))
    A.sort_indices()
    smask = amg.strength(A, 0.25)
    state = np.array([amg.F_PT, amg.C_PT, amg.C_PT, amg.C_PT, amg.F_PT], np.int8)
    P_ = dense(amg.direct_interpolation(A, smask, state))
    assert P_.shape == (5, 3)
    assert abs(P_[0, 0] - 3.3 / 4.5) < 1e-15
    assert P_[0, 1] == 0.0 and P_[0, 2] == 0.0
    # row 4: strong neighbours 0 (F, -1) and 3 (C, -1.5); no positive entries
    #   alpha = (-1 - 1.5) / (-1.5), P_43 = -alpha * (-1.5) / 4 = 2.5 / 4
    assert abs(P_[4, 2] - 2.5 / 4.0) < 1e-15
    assert np.array_equal(P_[1:4], np.eye(3))


def test_strength_definition_brute_force():
    rng = np.random.default_rng(3)
    A = sp.random(30, 30, density=0.3, random_state=4, format="csr") - sp.random(30, 30, density=0.3, random_state=5, format="csr")
    A = (A + sp.diags(np.full(30, 5.0))).tocsr()
    A.sort_indices()
    smask = amg.strength(A, 0.25)
    Ad = dense(A)
    rows = np.repeat(np.arange(30), np.diff(A.indptr))
    for t in range(A.nnz):
        i, j = rows[t], A.indices[t]
        offs = [-Ad[i, k] for k in range(30) if k != i and A[i, k] != 0]
        m = max(offs) if offs else -np.inf
        expect = (i != j) and m > 0 and (-Ad[i, j] >= 0.25 * m)
        assert smask[t] == expect


@pytest.mark.parametrize("kind", ["l1jac", "cheb2"])
def test_two_level_error_propagation_closed_form(kind):
    """Two-level V(1,1): E = S_post (I - P A_c^{-1} R A) S_pre, with the smoother written as its
    error polynomial: l1-Jacobi I - D_l1^{-1} A; Chebyshev T_2((theta - D^{-1}A)/delta)/T_2(theta/delta)."""
    A = poisson2d(9)
    lv = amg.build(A, coarse_max=30, max_levels=2, smoother=kind)
    assert len(lv) == 2
    L0 = lv[0]
    Ad = dense(A)
    n = A.shape[0]
    if kind == "l1jac":
        Smat = np.eye(n) - np.diag(1.0 / L0.dl1) @ Ad
    else:
        lam = L0.lam
        lo, hi = 0.3 * lam, lam
        th, de = (hi + lo) / 2, (hi - lo) / 2
        X = (th * np.eye(n) - np.diag(1.0 / np.diag(Ad)) @ Ad) / de
        Smat = (2 * X @ X - np.eye(n)) / (2 * (th / de) ** 2 - 1)
    P_, R_ = dense(L0.P), dense(L0.R)
    Ac = R_ @ Ad @ P_
    CGC = np.eye(n) - P_ @ np.linalg.solve(Ac, R_ @ Ad)
    E_formula = Smat @ CGC @ Smat
    E_oracle = _mat_of(lambda e: e - amg.vcycle(lv, Ad @ e, kind), n)
    assert np.abs(E_oracle - E_formula).max() < 1e-12
    rho = np.abs(np.linalg.eigvals(E_formula)).max()
    assert rho < 0.5


def test_vcycle_observed_rate_matches_spectral_radius():
    A = poisson2d(24)
    lv = amg.build(A, coarse_max=40, smoother="cheb2")
    assert len(lv) >= 3
    n = A.shape[0]
    E = _mat_of(lambda e: e - amg.vcycle(lv, A @ e), n)
    rho = np.abs(np.linalg.eigvals(E)).max()
    e = np.random.default_rng(0).standard_normal(n)
    ratios = []
    for _ in range(60):
        e_new = e - amg.vcycle(lv, A @ e)
        ratios.append(np.linalg.norm(e_new) / np.linalg.norm(e))
        e = e_new / np.linalg.norm(e_new)
    assert rho < 0.6
    assert abs(ratios[-1] - rho) < 0.02


def test_galerkin_product_equals_dense():
    A = poisson2d(12)
    lv = amg.build(A, coarse_max=20, smoother="l1jac")
    for L, Lc in zip(lv[:-1], lv[1:]):
        assert np.allclose(dense(Lc.A), dense(L.P).T @ dense(L.A) @ dense(L.P), rtol=0,
                           atol=1e-13 * np.abs(dense(L.A)).max())


def test_isolated_rows_solved_exactly():
    A = poisson2d(10).tolil()
    for i in (0, 37, 55):
        A[i, :] = 0
        A[:, i] = 0
        A[i, i] = 3.0
    A = A.tocsr()
    lv = amg.build(A, coarse_max=20, smoother="cheb2")
    b = np.random.default_rng(2).standard_normal(100)
    x = amg.vcycle(lv, b)
    for i in (0, 37, 55):
        assert x[i] == b[i] / 3.0 or abs(x[i] - b[i] / 3.0) < 1e-15


# ---------------------------------------------------------------------------- BILU(0)
def _blocks(s, vals):
    return s.Aff.rowptr, s.Aff.colind, vals


def test_bilu0_reproduces_matrix_on_pattern():
    s, _ = tiny(grid=(4, 3, 3))
    st = P.setup(s)
    rowptr, colind, vals = _blocks(s, st.sff_vals)
    F, Dinv, diag = local.bilu0_factor(rowptr, colind, vals)
    n, nf = s.n_cells, s.nf
    L = np.eye(n * nf)
    U = np.zeros((n * nf, n * nf))
    for i in range(n):
        for t in range(rowptr[i], rowptr[i + 1]):
            j = colind[t]
            blk = np.linalg.inv(Dinv[i]) if j == i else F[t]
            if j < i:
                L[i * nf:(i + 1) * nf, j * nf:(j + 1) * nf] = blk
            else:
                U[i * nf:(i + 1) * nf, j * nf:(j + 1) * nf] = blk
    LU = L @ U
    S = dense(st.Sff)
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    for t in range(colind.size):
        i, j = rows[t], colind[t]
        a = S[i * nf:(i + 1) * nf, j * nf:(j + 1) * nf]
        assert np.allclose(LU[i * nf:(i + 1) * nf, j * nf:(j + 1) * nf], a, rtol=1e-10,
                           atol=1e-12 * np.abs(S).max())


def test_bilu0_exact_on_block_tridiagonal_chain():
    s, _ = tiny(grid=(6, 1, 1))
    st = P.setup(s)
    rowptr, colind, vals = _blocks(s, st.sff_vals)
    F, Dinv, diag = local.bilu0_factor(rowptr, colind, vals)
    w = np.random.default_rng(0).standard_normal(s.n_f)
    dz = local.bilu0_apply(rowptr, colind, F, Dinv, diag, w.reshape(-1, s.nf)).ravel()
    assert np.allclose(dz, np.linalg.solve(dense(st.Sff), w), rtol=1e-10)


def _scalar_ilu0(Ad, pattern):
    """Textbook pointwise ILU(0) (IKJ) on a dense copy restricted to `pattern`."""
    a = Ad.copy()
    n = a.shape[0]
    for i in range(1, n):
        for k in range(i):
            if not pattern[i, k]:
                continue
            a[i, k] /= a[k, k]
            for j in range(k + 1, n):
                if pattern[i, j]:
                    a[i, j] -= a[i, k] * a[k, j]
    L = np.tril(a, -1) + np.eye(n)
    U = np.triu(a)
    return L, U


def test_block_ilu0_equals_pointwise_ilu0_on_block_pattern():
    s, _ = tiny(grid=(4, 3, 2))
    st = P.setup(s)
    rowptr, colind, vals = _blocks(s, st.sff_vals)
    F, Dinv, diag = local.bilu0_factor(rowptr, colind, vals)
    n, nf = s.n_cells, s.nf
    S = dense(st.Sff)
    pattern = np.zeros_like(S, bool)
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    for t in range(colind.size):
        i, j = rows[t], colind[t]
        pattern[i * nf:(i + 1) * nf, j * nf:(j + 1) * nf] = True
    L, U = _scalar_ilu0(S, pattern)
    w = np.random.default_rng(5).standard_normal(n * nf)
    z_point = sla.solve_triangular(U, sla.solve_triangular(L, w, lower=True, unit_diagonal=True))
    z_block = local.bilu0_apply(rowptr, colind, F, Dinv, diag, w.reshape(-1, nf)).ravel()
    assert np.allclose(z_block, z_point, rtol=1e-9, atol=1e-12 * np.abs(z_point).max())


# ---------------------------------------------------------------------------- FGMRES
@pytest.mark.parametrize("orth", ORTHS)
def test_fgmres_arnoldi_relation_and_orthogonality(orth):
    s, b = tiny(grid=(4, 4, 3))
    st = P.setup(s)
    A = st.mats["A"]
    out = fgmres(lambda v: A @ v, lambda v: P.apply_precond(st, v), b, rtol=1e-30,
                 restart=12, maxit=12, debug=True, orth=orth)
    d = out["debug"]
    V, Z, H = d["V"], d["Z"], d["H"]
    # columns whose next basis vector was formed (CGS2 stores none after the last column;
    # DCGS2 forms it when it finishes that column)
    k = Z.shape[0] - (0 if orth == "dcgs2" else 1)
    assert k >= 11
    AZ = np.stack([A @ z for z in Z[:k]], axis=1)
    rel = np.abs(AZ - V[: k + 1].T @ H[: k + 1, :k]).max() / sp.linalg.norm(A, np.inf)
    assert rel <= 1e-12
    G = V[: k + 1] @ V[: k + 1].T
    assert np.abs(G - np.eye(k + 1)).max() <= 1e-12


@pytest.mark.parametrize("orth", ORTHS)
def test_fgmres_residual_estimates_monotone(iid8, orth):
    s, b = iid8
    out = solve(s, b, rtol=1e-9, opts=Options(orth=orth))
    h = np.array(out["history"])
    assert np.all(np.diff(h) <= 1e-15)


@pytest.mark.parametrize("orth", ORTHS)
def test_fgmres_equals_minimal_residual_with_fixed_preconditioner(orth):
    """With a fixed linear M, iterate k minimises |b - A x| over x in M^{-1} K_k(A M^{-1}, b)."""
    rng = np.random.default_rng(9)
    n = 40
    A = np.eye(n) * 4 + rng.standard_normal((n, n))
    Minv = np.linalg.inv(np.diag(np.diag(A)) + np.tril(A, -1))
    b = rng.standard_normal(n)
    out = fgmres(lambda v: A @ v, lambda v: Minv @ v, b, rtol=1e-30, restart=30, maxit=8,
                 record_iterates=True, orth=orth)
    B = A @ Minv
    K = [b]
    for k in range(1, 9):
        Q, _ = np.linalg.qr(np.stack(K, 1))
        y, *_ = np.linalg.lstsq(B @ Q, b, rcond=None)
        x_ref = Minv @ (Q @ y)
        x_k = out["iterates"][k - 1]
        assert np.linalg.norm(x_k - x_ref) <= 1e-9 * np.linalg.norm(x_ref)
        K.append(B @ K[-1])


@pytest.mark.parametrize("orth", ORTHS)
def test_unpreconditioned_gmres_converges_in_n_steps(orth):
    rng = np.random.default_rng(2)
    Q = rng.standard_normal((12, 12))
    A = Q @ Q.T + 12 * np.eye(12)
    b = rng.standard_normal(12)
    out = fgmres(lambda v: A @ v, lambda v: v, b, rtol=1e-12, restart=50, maxit=50, orth=orth)
    assert out["status"] == 0 and out["iterations"] <= 12
    assert np.allclose(out["x"], np.linalg.solve(A, b), rtol=1e-9)


@pytest.mark.parametrize("orth", ORTHS)
def test_zero_rhs_returns_zero(orth):
    s, _ = tiny()
    out = solve(s, np.zeros(s.N), opts=Options(orth=orth))
    assert out["iterations"] == 0 and not out["x"].any() and out["status"] == 0


@pytest.mark.parametrize("restart", [100, 7])
def test_dcgs2_iterates_equal_cgs2_iterates(restart):
    """Delayed re-orthogonalisation changes only when the second Gram-Schmidt pass and the
    normalisation happen: in exact arithmetic both variants build the same basis and the
    same iterates, so on a well-conditioned system (two-stage preconditioner, restarts
    included) they agree to rounding and stop at the same iteration."""
    s, b = tiny(grid=(4, 4, 3))
    st = P.setup(s)
    A = st.mats["A"]
    runs = [fgmres(lambda v: A @ v, lambda v: P.apply_precond(st, v), b, rtol=1e-9, restart=restart,
                   maxit=60, record_iterates=True, orth=o) for o in ORTHS]
    a, c = runs
    assert a["status"] == c["status"] == 0 and a["iterations"] == c["iterations"]
    assert a["restarts"] == c["restarts"]
    for xa, xc in zip(a["iterates"], c["iterates"]):
        assert np.linalg.norm(xa - xc) <= 1e-11 * np.linalg.norm(xa)
    # residual estimates (above the rounding floor of this cond ~ 1e10 system)
    ha, hc = np.array(a["history"]), np.array(c["history"])
    big = ha >= 1e-7
    assert big.sum() >= 10 and np.allclose(ha[big], hc[big], rtol=1e-6)


@pytest.mark.parametrize("orth", ORTHS)
def test_fgmres_orthogonality_under_cancellation(orth):
    """A flexible preconditioner that returns z_j = |v_j| (z_{j-1} / |z_{j-1}| + 1e-9 v_j / |v_j|)
    makes every A z_j lie within 1e-9 of span(V): one classical Gram-Schmidt pass then loses orthogonality
    completely (checked here), while both two-pass variants keep V orthonormal and
    A Z = V H to rounding.  (Drops the second pass, the normalisation by alpha or the
    s.p term of t in the delayed variant, and this fails.)"""
    rng = np.random.default_rng(5)
    n, k = 120, 25
    A = np.eye(n) * 3 + rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n)
    state = {}

    def prec(v):
        nv = np.linalg.norm(v)
        z = v.copy() if "z" not in state else nv * (state["z"] / np.linalg.norm(state["z"]) + 1e-9 * v / nv)
        state["z"] = z
        return z

    V1 = np.zeros((k + 1, n))               # one classical Gram-Schmidt pass
    V1[0] = b / np.linalg.norm(b)
    for j in range(k):
        w = A @ prec(V1[j])
        w = w - V1[: j + 1].T @ (V1[: j + 1] @ w)
        V1[j + 1] = w / np.linalg.norm(w)
    assert np.abs(V1 @ V1.T - np.eye(k + 1)).max() > 1e-3
    state.clear()
    out = fgmres(lambda v: A @ v, prec, b, rtol=1e-30, restart=k, maxit=k, debug=True, orth=orth)
    d = out["debug"]
    V, Z, H = d["V"], d["Z"], d["H"]
    kk = Z.shape[0] - (0 if orth == "dcgs2" else 1)
    assert kk >= k - 1
    assert np.abs(V[: kk + 1] @ V[: kk + 1].T - np.eye(kk + 1)).max() <= 1e-13
    AZ = np.stack([A @ z for z in Z[:kk]], axis=1)
    assert np.abs(AZ - V[: kk + 1].T @ H[: kk + 1, :kk]).max() <= 1e-13 * np.abs(AZ).max()


def test_multicolour_gs_is_block_gs_in_colour_order():
    """One multicolour sweep equals a block Gauss-Seidel sweep, (D + L)^{-1} w, on the matrix
    permuted to colour order; the greedy colouring of a 7-point stencil is a checkerboard."""
    s, _ = tiny(grid=(4, 3, 3))
    st = P.setup(s, Options(ml_kind="mcgs"))
    colors = st.ml[2]
    ci, cj, ck = np.meshgrid(np.arange(4), np.arange(3), np.arange(3), indexing="xy")
    i = np.tile(np.arange(4), 9)
    j = np.tile(np.repeat(np.arange(3), 4), 3)
    k = np.repeat(np.arange(3), 12)
    assert np.array_equal(colors, (i + j + k) % 2)
    nf = s.nf
    order = np.argsort(colors, kind="stable")
    perm = (order[:, None] * nf + np.arange(nf)[None, :]).ravel()
    S = dense(st.Sff)[np.ix_(perm, perm)]
    # block lower triangle including the diagonal cell blocks
    n = s.n_cells
    DL = np.zeros_like(S)
    for a in range(n):
        for b in range(a + 1):
            DL[a * nf:(a + 1) * nf, b * nf:(b + 1) * nf] = S[a * nf:(a + 1) * nf, b * nf:(b + 1) * nf]
    w = np.random.default_rng(4).standard_normal(s.n_f)
    z_ref = np.zeros(s.n_f)
    z_ref[perm] = np.linalg.solve(DL, w[perm])
    z = local.mcgs_apply(st.Sff, st.ml[1], colors, w.reshape(-1, nf), 1).ravel()
    assert np.allclose(z, z_ref, rtol=1e-10, atol=1e-12 * np.abs(z_ref).max())


def test_processor_local_bilu_reduces_to_known_cases():
    """One cell per subdomain: processor-local BILU(0) is block Jacobi.  One x-line per
    subdomain: it is the exact inverse of each line's block-tridiagonal matrix."""
    from synth.jacobian import box_partition
    s, _ = tiny(grid=(5, 3, 2))
    nf, n = s.nf, s.n_cells
    w = np.random.default_rng(6).standard_normal(s.n_f)
    for bx, expect in ((1, "jacobi"), (5, "lines")):
        s.ml_part = box_partition(5, 3, 2, bx, 1, 1)
        st = P.setup(s)
        z = P.apply_precond(st, np.concatenate([np.zeros(s.n_u), w]))  # noqa: F841 (exercise)
        _, F, Dinv, diag, lrp, lci = st.ml
        dz = local.bilu0_apply(lrp, lci, F, Dinv, diag, w.reshape(-1, nf)).ravel()
        S = dense(st.Sff)
        keep = np.zeros_like(S, bool)
        for i in range(n):
            for j in range(n):
                if s.ml_part[i] == s.ml_part[j]:
                    keep[i * nf:(i + 1) * nf, j * nf:(j + 1) * nf] = True
        ref = np.linalg.solve(np.where(keep, S, 0.0), w)
        assert np.allclose(dz, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max()), expect
    s.ml_part = None


def test_power_iteration_estimate_brute_force_and_bound():
    """Chebyshev's eigenvalue estimate: ten normalised power steps on D^{-1} A from
    v_0 = 1 + u equal |B^10 v_0| / |B^9 v_0| (B = D^{-1} A, dense brute force), and on
    tridiag(-1, 2, -1) stay below the closed-form spectral radius 1 + cos(pi/(n+1))."""
    n = 15
    A = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1], format="csr")
    d = A.diagonal()
    lam = amg.power_lambda(A, d)
    B = np.diag(1.0 / d) @ A.toarray()
    from oracle.rng import unit
    v0 = 1.0 + unit(np.arange(n, dtype=np.uint64))
    w9 = np.linalg.matrix_power(B, 9) @ v0
    assert abs(lam - np.linalg.norm(B @ w9) / np.linalg.norm(w9)) <= 1e-13 * lam
    rho = 1.0 + np.cos(np.pi / (n + 1))
    assert lam <= rho * (1 + 1e-12) and lam > 0.5 * rho


# ---------------------------------------------------------------------------- alternatives
@pytest.mark.parametrize("kind", ["iid", "iid3"])
def test_true_impes_column_sum_lumping_dense(kind):
    """True-IMPES (eq. CPR_CSL): D_ss = diag(A_ss^T e), D_ps = diag(A_ps^T e) -- for
    nf = 3 the s-s and p-s cell blocks summed down each block column -- and S_pp and
    step 3 built from them, by dense brute force."""
    s, _ = tiny(kind=kind, grid=(3, 3, 2))
    st = P.setup(s, Options(reduction="true"))
    nf, m = s.nf, s.nf - 1
    sidx, pidx = perms(s)
    Aff = dense(st.mats["Aff"])
    Sff = dense(st.Sff)
    Ass = Aff[np.ix_(sidx, sidx)]
    Aps = Aff[np.ix_(pidx, sidx)]
    Dss = np.zeros_like(Ass)
    Dps = np.zeros_like(Aps)
    for c in range(s.n_cells):
        sl = slice(c * m, (c + 1) * m)
        for k in range(s.n_cells):               # block column c: rows of every cell k
            Dss[sl, sl] += Ass[k * m:(k + 1) * m, sl]
            Dps[c, sl] += Aps[k, sl]
    if nf == 2:                                   # the scalar case is exactly e^T A_ss
        assert np.allclose(np.diag(Dss), Ass.sum(axis=0), rtol=1e-13)
        assert np.allclose(np.diag(Dps), Aps.sum(axis=0), rtol=1e-13)
    Spp = Sff[np.ix_(pidx, pidx)] - Dps @ np.linalg.inv(Dss) @ Sff[np.ix_(sidx, pidx)]
    assert np.allclose(dense(st.Spp), Spp, rtol=1e-12, atol=1e-12 * np.abs(Spp).max())
    dss_inv = np.zeros_like(Dss)
    for c in range(s.n_cells):
        sl = slice(c * m, (c + 1) * m)
        dss_inv[sl, sl] = st.dss_inv[c]
    assert np.allclose(dss_inv, np.linalg.inv(Dss), rtol=1e-12, atol=1e-12 * np.abs(dss_inv).max())
    # and it differs from quasi-IMPES whenever fluxes couple the saturations
    qi = P.setup(s, Options())
    assert not np.allclose(dense(qi.Spp), dense(st.Spp))


def test_true_impes_equals_quasi_impes_without_saturation_flux_terms():
    """With no saturation derivatives off the diagonal (A_ss, A_ps block-diagonal), the
    column sums are the diagonal blocks and the two reductions coincide."""
    s, _ = tiny(kind="iid", grid=(3, 2, 2))
    rows = np.repeat(np.arange(s.n_cells), np.diff(s.Aff.rowptr))
    off = rows != s.Aff.colind
    s.Aff.vals[off, :, : s.nf - 1] = 0.0
    a = P.setup(s, Options(reduction="true"))
    b = P.setup(s, Options())
    assert np.array_equal(dense(a.Spp), dense(b.Spp))
    assert np.array_equal(a.dss_inv, b.dss_inv)


def test_rsl_diagonals_converge_to_the_exact_row_sums():
    """eq. FS_RSL with A_uu^{-1} applied exactly: -diag(A_fu A_uu^{-1} A_up e) by a dense
    solve; the oracle's V-cycle Richardson approximation approaches it as the number of
    steps grows (and is the exact Schur complement's row sums over the pressure columns)."""
    s, _ = tiny(kind="iid3", grid=(3, 3, 2))
    mats = P.system_matrices(s)
    nf, nc = s.nf, s.n_cells
    Auu, Auf, Afu = dense(mats["Auu"]), dense(mats["Auf"]), dense(mats["Afu"])
    sidx, pidx = perms(s)
    Aup = Auf[:, pidx]
    y = np.linalg.solve(Auu, Aup @ np.ones(nc))
    w = Afu @ y
    exact_sp = -w[sidx].reshape(nc, nf - 1)
    exact_pp = -w[pidx]
    # the same numbers are the row sums of the exact first-level Schur complement's
    # coupling part  -A_fu A_uu^{-1} A_up  (Sec. 5.1)
    C = -Afu @ np.linalg.solve(Auu, Aup)
    assert np.allclose(C.sum(axis=1), np.concatenate([exact_sp, exact_pp[:, None]], 1).ravel(), rtol=1e-10)
    sdc = amg.build(P.sdc_matrix(s), smoother="cheb2")
    errs = []
    for its in (1, 5, 40):
        d_sp, d_pp = P.rsl_diagonals(s, mats, sdc, "cheb2", its)
        errs.append(max(np.abs(d_sp - exact_sp).max() / np.abs(exact_sp).max(),
                        np.abs(d_pp - exact_pp).max() / np.abs(exact_pp).max()))
    assert errs[0] > errs[1] > errs[2] and errs[2] <= 1e-8, errs
    # fixed stress with RSL diagonals: S_ff = A_ff + the lumped diagonals, nothing else
    st = P.setup(s, Options(fixed_stress="rsl", fs_iters=40), mechanics=sdc)
    D = dense(st.Sff) - dense(mats["Aff"])
    expect = np.zeros_like(D)
    for c in range(nc):
        for l in range(nf - 1):
            expect[c * nf + l, c * nf + nf - 1] = exact_sp[c, l]
        expect[c * nf + nf - 1, c * nf + nf - 1] = exact_pp[c]
    assert np.allclose(D, expect, rtol=1e-7, atol=1e-8 * np.abs(expect).max())


def test_richardson_iterates_equal_the_stationary_closed_form():
    """x_k of the preconditioned Richardson iteration from x_0 = 0 is
    sum_{i<k} (I - M A)^i M b for a linear M (dense matrices, brute force), and with
    M = A^{-1} it converges in one step."""
    from oracle.fgmres import richardson
    s, b = tiny(kind="iid", grid=(2, 2, 2))
    st = P.setup(s)
    A = dense(st.mats["A"])
    n = A.shape[0]
    M = np.column_stack([P.apply_precond(st, e) for e in np.eye(n)])
    out = richardson(lambda v: A @ v, lambda v: M @ v, b, rtol=1e-300, maxit=6, record_iterates=True)
    G = np.eye(n) - M @ A
    acc = np.zeros(n)
    term = M @ b
    for k in range(6):
        acc = acc + term
        term = G @ term
        assert np.allclose(out["iterates"][k], acc, rtol=1e-10, atol=1e-12 * np.abs(acc).max())
    one = richardson(lambda v: A @ v, lambda v: np.linalg.solve(A, v), b, rtol=1e-6, maxit=5)
    assert one["iterations"] == 1 and one["status"] == 0
    assert np.allclose(one["x"], np.linalg.solve(A, b), rtol=1e-8)


def test_eisenstat_walker_forcing_values():
    """The forcing of the Sec. 4 remark with gamma = 0.9, omega = 2, eta_0 = 0.1, by hand."""
    from oracle.newton import ew_eta
    assert ew_eta(0, 5.0, None, None) == 0.1
    assert np.isclose(ew_eta(1, 1.0, 2.0, 0.1), 0.9 * 0.25)               # 0.9 * 0.1^2 < 0.1
    assert np.isclose(ew_eta(2, 1.0, 100.0, 0.5), 0.9 * 0.25)             # safeguard 0.225 > 0.1
    assert np.isclose(ew_eta(2, 1.0, 100.0, 0.2), 0.9 * 1e-4)             # 0.036 <= 0.1: no safeguard
    assert ew_eta(3, 10.0, 1.0, 0.5) == 0.9                               # capped


def test_oracle_newton_converges_fast_near_the_solution():
    """Newton on one backward-Euler day of a tiny i.i.d. grid: the scaled residual falls at
    every step and reaches 1e-8 of the initial one, the last two steps by 100x or more."""
    from synth.nonlinear import time_step
    from oracle.newton import newton
    out = newton(time_step((5, 4, 3), kind="iid", seed=3), tol=1e-8, max_steps=10,
                 opts=Options(smoother="l1jac"))
    res = [st["residual"] for st in out["steps"]]
    assert out["converged"] and all(b < a for a, b in zip(res, res[1:]))
    assert res[-1] < 0.01 * res[-2] and res[-2] < 0.01 * res[-3]
