"""Classical algebraic multigrid, written plainly (oracle; test infrastructure only).

The paper uses AMG for both scalar sub-problems -- the separate-displacement-
component elasticity operator (Sec. 5.2, M_uu = amg(A_uu^sdc)) and the
quasi-IMPES pressure operator (Sec. 5.3, eq. S1_prec, M_pp = amg(S_pp)) -- but its
concrete AMG (Hypre BoomerAMG with HMIS/aggressive coarsening and hybrid
l1-Gauss-Seidel, Sec. 6) is a CPU-cluster choice.  The method computed here is the
published parallel alternative, fixed in every detail so that two independent
implementations produce the same hierarchy:

  strength   j in S_i  iff  j != i and -a_ij >= theta * max_{k != i}(-a_ik) > 0.
  PMIS       (De Sterck, Yang, Heys 2006) weights w_i = |S^T_i| + u_i with u_i from
             SplitMix64 of the row index; ties compared on (w_i, i).  Points that
             influence nobody start as F.  Each round every undecided point that
             beats all undecided neighbours in S u S^T becomes C, then every
             undecided point strongly depending on a new C point becomes F.
  promotion  in increasing i, an F point with S_i non-empty and no C point in S_i
             becomes C.
  interp.    direct interpolation (Stueben): C rows identity; F row i with
             C_i = S_i n C:  P_ij = -(alpha_i a_ij) / atil_ii,  j in C_i, with
             alpha_i = sum_{j != i, a_ij < 0} a_ij / sum_{k in C_i} a_ik and
             atil_ii = a_ii + sum_{j != i, a_ij > 0} a_ij (positive entries lumped).
             All sums run in increasing column order starting from 0.
  coarse     R = P^T, A_c = R (A P), exact zeros dropped.  Stop when n <= coarse_max,
             at max_levels levels, or when n_c == 0 or n_c > 0.9 n; the last level is
             solved with dense LU with partial pivoting.
  smoothing  V(1,1), pre-smoother from x = 0.  l1-Jacobi: x += (b - A x) / d,
             d_i = a_ii + sum_{j != i} |a_ij|.  Chebyshev degree 2 on D^{-1} A over
             [0.3 l', l'], l' = 1.1 l, l = |D^{-1} A v_10| after 10 normalised power
             steps from v_0 = 1 + u (Saad, Iterative Methods, Alg. 12.1 recurrence);
             rows without off-diagonal entries are solved exactly.
"""
from dataclasses import dataclass
import numpy as np
import scipy.sparse as sp
import scipy.linalg as sla

from .rng import unit

F_PT, UNDEC, C_PT = -1, 0, 1


def _row_ids(A):
    return np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))


def strength(A, theta):
    """Boolean mask over A's stored entries: True where j in S_i."""
    n = A.shape[0]
    rows = _row_ids(A)
    off = rows != A.indices
    neg = np.where(off, -A.data, -np.inf)
    m = np.full(n, -np.inf)
    np.maximum.at(m, rows, neg)
    return off & (m[rows] > 0) & (neg >= theta * m[rows])


def _strength_matrix(A, smask):
    rows = _row_ids(A)
    n = A.shape[0]
    return sp.csr_matrix((np.ones(int(smask.sum()), np.int32), (rows[smask], A.indices[smask])),
                         shape=(n, n))


def pmis(A, smask, rounds=None, promote=True):
    """C/F splitting (array of C_PT / F_PT), PMIS followed by C-promotion.

    rounds: stop after this many PMIS rounds (undecided points stay UNDEC); promote:
    apply the C-promotion pass.  Both exist so that tests can inspect the rounds.
    """
    n = A.shape[0]
    S = _strength_matrix(A, smask)
    ST = S.T.tocsr()
    lam = np.diff(ST.indptr).astype(np.float64)   # |S^T_i|
    nS = np.diff(S.indptr)
    w = lam + unit(np.arange(n, dtype=np.uint64))
    state = np.zeros(n, np.int8)
    state[lam == 0] = F_PT
    G = (S + ST).tocoo()
    gi, gj = G.row, G.col
    done = 0
    while np.any(state == UNDEC) and (rounds is None or done < rounds):
        done += 1
        und = state == UNDEC
        e = und[gi] & und[gj]
        bigger = (w[gj] > w[gi]) | ((w[gj] == w[gi]) & (gj > gi))
        beaten = np.zeros(n, bool)
        beaten[gi[e & bigger]] = True
        newc = und & ~beaten
        state[newc] = C_PT
        hit = (S @ newc.astype(np.int32)) > 0
        state[(state == UNDEC) & hit] = F_PT
    if not promote:
        return state
    # C-promotion, sequential in increasing i
    hasc = (S @ (state == C_PT).astype(np.int32)) > 0
    for i in np.nonzero((state == F_PT) & (nS > 0) & ~hasc)[0]:
        nb = S.indices[S.indptr[i]:S.indptr[i + 1]]
        if not np.any(state[nb] == C_PT):
            state[i] = C_PT
    return state


def direct_interpolation(A, smask, state):
    n = A.shape[0]
    isc = state == C_PT
    cidx = np.cumsum(isc) - 1
    nc = int(isc.sum())
    rows = _row_ids(A)
    cols = A.indices
    a = A.data
    off = rows != cols
    diag = np.zeros(n)
    diag[rows[~off]] = a[~off]
    pos = np.bincount(rows[off & (a > 0)], weights=a[off & (a > 0)], minlength=n)
    negs = np.bincount(rows[off & (a < 0)], weights=a[off & (a < 0)], minlength=n)
    cstrong = smask & isc[cols]
    den = np.bincount(rows[cstrong], weights=a[cstrong], minlength=n)
    atil = diag + pos
    frow = ~isc[rows]
    sel = cstrong & frow
    alpha = np.zeros(n)
    ok = den != 0
    alpha[ok] = negs[ok] / den[ok]
    r = rows[sel]
    vals = -(alpha[r] * a[sel]) / atil[r]
    ci = np.nonzero(isc)[0]
    prow = np.concatenate([ci, r])
    pcol = np.concatenate([cidx[ci], cidx[cols[sel]]])
    pval = np.concatenate([np.ones(nc), vals])
    P = sp.csr_matrix((pval, (prow, pcol)), shape=(n, nc))
    P.sort_indices()
    return P


def galerkin(A, P):
    R = P.T.tocsr()
    R.sort_indices()
    Ac = R @ (A @ P)
    Ac.eliminate_zeros()
    Ac.sort_indices()
    return R, Ac.tocsr()


@dataclass
class Level:
    A: sp.csr_matrix
    P: sp.csr_matrix = None
    R: sp.csr_matrix = None
    dl1: np.ndarray = None
    c0: np.ndarray = None
    c1: np.ndarray = None
    cm: np.ndarray = None
    lam: float = None
    lu: tuple = None
    state: np.ndarray = None


def power_lambda(A, d, its=10):
    """Largest-eigenvalue estimate of D^{-1} A: |D^{-1} A v_its| after normalised steps."""
    n = A.shape[0]
    v = 1.0 + unit(np.arange(n, dtype=np.uint64))
    v = v / np.linalg.norm(v)
    lam = 0.0
    for _ in range(its):
        wv = (A @ v) / d
        lam = np.linalg.norm(wv)
        v = wv / lam
    return lam


def smoother_setup(L, kind):
    A = L.A
    rows = _row_ids(A)
    off = rows != A.indices
    d = np.zeros(A.shape[0])
    d[rows[~off]] = A.data[~off]
    iso = np.bincount(rows[off & (A.data != 0)], minlength=A.shape[0]) == 0
    if kind == "l1jac":
        L.dl1 = d + np.bincount(rows[off], weights=np.abs(A.data[off]), minlength=A.shape[0])
    elif kind == "cheb2":
        lam = 1.1 * power_lambda(A, d)
        lo, hi = 0.3 * lam, lam
        theta, delta = (hi + lo) / 2.0, (hi - lo) / 2.0
        sigma = theta / delta
        rho0 = 1.0 / sigma
        rho1 = 1.0 / (2.0 * sigma - rho0)
        L.lam = lam
        L.c0 = np.where(iso, 1.0 / d, 1.0 / (theta * d))
        L.cm = np.where(iso, 0.0, rho1 * rho0)
        L.c1 = np.where(iso, 0.0, 2.0 * rho1 / (delta * d))
    else:
        raise ValueError(kind)


def build(A, theta=0.25, coarse_max=256, max_levels=25, smoother="cheb2", max_dense=6000,
          forced_split=None):
    """AMG hierarchy for scalar CSR matrix A (list of Level, coarsest last).

    forced_split: optional list of C/F arrays that replace PMIS on the first levels
    (used only by tests pinning interpolation against closed forms).
    """
    A = sp.csr_matrix(A)
    A.sort_indices()
    levels = []
    while A.shape[0] > coarse_max and len(levels) + 1 < max_levels:
        smask = strength(A, theta)
        if forced_split is not None and len(levels) < len(forced_split):
            state = np.asarray(forced_split[len(levels)], np.int8)
        else:
            state = pmis(A, smask)
        nc = int(np.sum(state == C_PT))
        if nc == 0 or nc > 0.9 * A.shape[0]:
            break
        P = direct_interpolation(A, smask, state)
        R, Ac = galerkin(A, P)
        L = Level(A=A, P=P, R=R, state=state)
        smoother_setup(L, smoother)
        levels.append(L)
        A = Ac
    if A.shape[0] > max_dense:
        raise RuntimeError("coarsest level too large for a dense solve: %d" % A.shape[0])
    dense = A.toarray()
    lu = sla.lu_factor(dense, check_finite=True)
    if np.any(np.diag(lu[0]) == 0):
        raise np.linalg.LinAlgError("singular coarsest matrix")
    levels.append(Level(A=A, lu=lu))
    return levels


def presmooth(L, b, kind):
    if kind == "l1jac":
        return b / L.dl1
    d0 = L.c0 * b
    x1 = d0
    r1 = b - L.A @ x1
    return x1 + (L.cm * d0 + L.c1 * r1)


def postsmooth(L, b, x, kind):
    if kind == "l1jac":
        return x + (b - L.A @ x) / L.dl1
    r0 = b - L.A @ x
    d0 = L.c0 * r0
    x1 = x + d0
    r1 = b - L.A @ x1
    return x1 + (L.cm * d0 + L.c1 * r1)


def vcycle(levels, b, kind="cheb2", lvl=0):
    """One V(1,1)-cycle for A_0 x = b starting from x = 0."""
    L = levels[lvl]
    if L.lu is not None:
        return sla.lu_solve(L.lu, b)
    x = presmooth(L, b, kind)
    r = b - L.A @ x
    ec = vcycle(levels, L.R @ r, kind, lvl + 1)
    x = x + L.P @ ec
    return postsmooth(L, b, x, kind)


def operator_complexity(levels):
    return sum(L.A.nnz for L in levels) / levels[0].A.nnz
