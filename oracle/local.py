"""Second-stage local preconditioners M_L on the interleaved flow system (oracle).

Sec. 5.3: after the global stage, the approximate Schur complement S_ff^(fs) is
viewed as one monolithic system in interleaved ordering ({s_i, p_i} per cell), which
gives dense nf x nf cell blocks coupled by the TPFA stencil; the paper uses either
hybrid block Gauss-Seidel sweeps or one sweep of pointwise ILU(0) on it.

  BILU(0)   block incomplete LU with zero fill on the block pattern, in the given
            cell order (IKJ form): for each block row i and each k < i in the row
            (increasing), L_ik = A_ik D_k^{-1}, then A_ij -= L_ik U_kj for every j > k
            present in both row i and row k; finally D_i = A_ii.  Apply: forward
            y_i = w_i - sum_{k<i} L_ik y_k, backward dz_i = D_i^{-1} (y_i - sum_{j>i}
            U_ij dz_j).  Reading: the block form on nf x nf cell blocks equals
            pointwise ILU(0) on the block-dense pattern (tested).  With k > 1 sweeps
            the factorisation is used as a stationary iteration:
            dz_1 = B^{-1} w, dz_{i+1} = dz_i + B^{-1}(w - S dz_i).
            Processor-local form (the paper's second example, Sec. 6): with a cell
            partition, B is the BILU(0) of S with the couplings between cells of
            different subdomains removed (block Jacobi over subdomains).
  Jacobi    `sweeps` block-Jacobi sweeps dz += D^{-1}(w - S dz) from dz = 0 with the
            diagonal cell blocks D (a fully parallel relaxation option).
  block GS  the paper's option 1, hybrid block Gauss-Seidel (several sweeps), in its
            parallel multicolour form: cells are coloured greedily in increasing index
            order (each cell takes the smallest colour not used by an already coloured
            neighbour; two colours on a 7-point stencil), and one sweep visits the
            colours in increasing order, updating every cell of a colour from the
            latest values: dz_i = D_i^{-1}(w_i - sum_{j != i} S_ij dz_j), dz = 0 at start.
Test infrastructure only.
"""
import numpy as np


class SingularBlock(ArithmeticError):
    pass


def _inv(blk):
    inv = np.linalg.inv(blk)
    if not np.all(np.isfinite(inv)):
        raise SingularBlock("singular diagonal block")
    return inv


def bilu0_factor(rowptr, colind, vals):
    """Returns (F, Dinv, diag) with F the factor values in the input block pattern."""
    n = rowptr.shape[0] - 1
    F = np.array(vals, dtype=np.float64, copy=True)
    nf = F.shape[1]
    diag = np.full(n, -1, np.int64)
    for i in range(n):
        for t in range(rowptr[i], rowptr[i + 1]):
            if colind[t] == i:
                diag[i] = t
    if np.any(diag < 0):
        raise ValueError("missing diagonal block")
    Dinv = np.zeros((n, nf, nf))
    for i in range(n):
        lo, hi = rowptr[i], rowptr[i + 1]
        pos = {int(colind[t]): t for t in range(lo, hi)}
        for t in range(lo, hi):
            k = int(colind[t])
            if k >= i:
                break
            F[t] = F[t] @ Dinv[k]
            for u in range(diag[k] + 1, rowptr[k + 1]):
                j = int(colind[u])
                q = pos.get(j)
                if q is not None:
                    F[q] -= F[t] @ F[u]
        Dinv[i] = _inv(F[diag[i]])
    return F, Dinv, diag


def bilu0_apply(rowptr, colind, F, Dinv, diag, w):
    """w: (n, nf) -> dz: (n, nf)."""
    n = rowptr.shape[0] - 1
    y = np.array(w, dtype=np.float64, copy=True)
    for i in range(n):
        for t in range(rowptr[i], diag[i]):
            y[i] -= F[t] @ y[colind[t]]
    z = np.zeros_like(y)
    for i in range(n - 1, -1, -1):
        acc = y[i].copy()
        for t in range(diag[i] + 1, rowptr[i + 1]):
            acc -= F[t] @ z[colind[t]]
        z[i] = Dinv[i] @ acc
    return z


def restrict_to_parts(rowptr, colind, vals, part):
    """Block CSR of S keeping only blocks (i, j) with part[i] == part[j]."""
    n = rowptr.shape[0] - 1
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    keep = part[rows] == part[colind]
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(rows[keep], minlength=n), out=rp[1:])
    return rp, colind[keep], vals[keep]


def bilu0_sweeps(rowptr, colind, F, Dinv, diag, S, w, sweeps):
    """`sweeps` BILU(0) sweeps as a stationary iteration; w: (n, nf)."""
    n, nf = w.shape
    dz = bilu0_apply(rowptr, colind, F, Dinv, diag, w)
    for _ in range(sweeps - 1):
        r = (w.ravel() - S @ dz.ravel()).reshape(n, nf)
        dz = dz + bilu0_apply(rowptr, colind, F, Dinv, diag, r)
    return dz


def greedy_colors(rowptr, colind):
    """Colour of each block row: smallest colour unused by lower-index neighbours."""
    n = rowptr.shape[0] - 1
    col = np.full(n, -1, np.int64)
    for i in range(n):
        used = {int(col[j]) for j in colind[rowptr[i]:rowptr[i + 1]] if j < i}
        c = 0
        while c in used:
            c += 1
        col[i] = c
    return col


def mcgs_apply(S, Dinv, colors, w, sweeps):
    """`sweeps` multicolour block Gauss-Seidel sweeps from dz = 0; w: (n, nf)."""
    n, nf = w.shape
    dz = np.zeros_like(w)
    groups = [np.nonzero(colors == c)[0] for c in range(int(colors.max()) + 1)]
    for _ in range(sweeps):
        for rows in groups:
            r = (w.ravel() - S @ dz.ravel()).reshape(n, nf)
            dz[rows] = dz[rows] + np.einsum("nij,nj->ni", Dinv[rows], r[rows])
    return dz


def block_diag_inv(rowptr, colind, vals):
    n = rowptr.shape[0] - 1
    nf = vals.shape[1]
    Dinv = np.zeros((n, nf, nf))
    for i in range(n):
        for t in range(rowptr[i], rowptr[i + 1]):
            if colind[t] == i:
                Dinv[i] = _inv(vals[t])
    return Dinv


def bjacobi_apply(S, Dinv, w, sweeps):
    """S: scalar CSR of the interleaved system; w: (n, nf)."""
    n, nf = w.shape
    dz = np.zeros_like(w)
    for _ in range(sweeps):
        r = (w.ravel() - S @ dz.ravel()).reshape(n, nf)
        dz = dz + np.einsum("nij,nj->ni", Dinv, r)
    return dz
