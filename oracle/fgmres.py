"""Right-preconditioned flexible GMRES(m) in FP64 (oracle; test infrastructure only).

The paper solves each Jacobian system with right-preconditioned GMRES (Sec. 4,
(A M^{-1}) dy = -r, dx = M^{-1} dy).  Readings where it is silent: restart length
m = 100, flexible variant (Saad, SIAM J. Sci. Comput. 14, 1993) so that a
preconditioner applied in reduced precision stays consistent, classical
Gram-Schmidt applied twice (CGS2) for the Arnoldi step, Givens rotations for the
Hessenberg least-squares problem, x0 = 0, convergence when the true residual
|b - A x| <= rtol |b| at the end of a cycle, a cycle also ends on a happy breakdown
h_{j+1,j} <= 1e-14 |A z_j|, and at most `maxit` iterations in total.
"""
import numpy as np
import scipy.linalg as sla

OK, EMAXIT, EBREAKDOWN = 0, -6, -9


def fgmres(matvec, precond, b, rtol=1e-8, restart=100, maxit=1000, record_iterates=False,
           debug=False):
    """Returns dict(x, iterations, restarts, status, rel_residual, history, iterates).

    history[k] is the Givens residual estimate |g_{k+1}| / |b| after iteration k+1.
    iterates[k] (when recorded) is the iterate x_{k+1} = x_cycle + Z_k H_k^{-1} g_k.
    debug: keep the last cycle's V, Z and unrotated Hessenberg matrix in the result.
    """
    b = np.asarray(b, np.float64)
    n = b.shape[0]
    x = np.zeros(n)
    beta_b = np.linalg.norm(b)
    res = dict(x=x, iterations=0, restarts=0, status=OK, rel_residual=0.0, history=[],
               iterates=[] if record_iterates else None)
    if beta_b == 0.0:
        return res
    m = restart
    its = 0
    r = b.copy()
    cycles = 0
    while True:
        beta = np.linalg.norm(r)
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        if debug:
            Hraw = np.zeros((m + 1, m))
        k = 0
        breakdown = False
        for j in range(m):
            Z[j] = precond(V[j])
            w = matvec(Z[j])
            norm_az = np.linalg.norm(w)
            h = V[: j + 1] @ w
            w = w - V[: j + 1].T @ h
            h2 = V[: j + 1] @ w
            w = w - V[: j + 1].T @ h2
            h = h + h2
            hn = np.linalg.norm(w)
            H[: j + 1, j] = h
            H[j + 1, j] = hn
            if debug:
                Hraw[: j + 2, j] = H[: j + 2, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            rho = np.hypot(H[j, j], H[j + 1, j])
            k = j + 1
            its += 1
            if rho == 0.0:
                breakdown = True
                break
            cs[j] = H[j, j] / rho
            sn[j] = H[j + 1, j] / rho
            H[j, j] = rho
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            res["history"].append(abs(g[j + 1]) / beta_b)
            if record_iterates:
                y = sla.solve_triangular(H[:k, :k], g[:k])
                res["iterates"].append(x + Z[:k].T @ y)
            if abs(g[j + 1]) <= rtol * beta_b or hn <= 1e-14 * norm_az or its >= maxit:
                break
            V[j + 1] = w / hn
        if breakdown:
            k -= 1
        if debug:
            res["debug"] = dict(V=V[: k + 1].copy(), Z=Z[:k].copy(), H=Hraw[: k + 1, :k].copy(),
                                last_normalised=(k < m and V[k].any()))
        if k > 0:
            y = sla.solve_triangular(H[:k, :k], g[:k])
            x = x + Z[:k].T @ y
        r = b - matvec(x)
        rel = np.linalg.norm(r) / beta_b
        res.update(x=x, iterations=its, restarts=cycles, rel_residual=rel)
        if rel <= rtol:
            res["status"] = OK
            return res
        if breakdown:
            res["status"] = EBREAKDOWN
            return res
        if its >= maxit:
            res["status"] = EMAXIT
            return res
        cycles += 1


def richardson(matvec, precond, b, rtol=1e-8, maxit=1000, record_iterates=False):
    """Preconditioned Richardson iteration x_{k+1} = x_k + M^{-1}(b - A x_k), x_0 = 0.

    The paper's remark after Algorithm 1: the two-stage preconditioner inside a
    fixed-point (Richardson) iteration is the sequential fixed-stress scheme -- step 1
    corrects the displacement, steps 2-8 then update the flow unknowns.  Stops when the
    FP64 residual |b - A x_k| <= rtol |b| (checked after every step) or after maxit steps.
    history[k] = |b - A x_{k+1}| / |b|; iterates[k] = x_{k+1} when recorded.
    """
    b = np.asarray(b, np.float64)
    x = np.zeros(b.shape[0])
    beta_b = np.linalg.norm(b)
    res = dict(x=x, iterations=0, restarts=0, status=OK, rel_residual=0.0, history=[],
               iterates=[] if record_iterates else None)
    if beta_b == 0.0:
        return res
    r = b.copy()
    its = 0
    while True:
        x = x + precond(r)
        r = b - matvec(x)
        its += 1
        rel = np.linalg.norm(r) / beta_b
        res["history"].append(rel)
        if record_iterates:
            res["iterates"].append(x.copy())
        if rel <= rtol or its >= maxit:
            res.update(x=x, iterations=its, rel_residual=rel, status=OK if rel <= rtol else EMAXIT)
            return res


def solve(system, b, rtol=1e-8, opts=None, setup_result=None, record_iterates=False):
    """FGMRES (or, with opts.method == "richardson", the preconditioned Richardson
    iteration) with the two-stage preconditioner on a synthetic system."""
    from .precond import setup as _setup, apply_precond, Options
    opts = opts or Options()
    st = setup_result or _setup(system, opts)
    A = st.mats["A"]
    if getattr(opts, "method", "fgmres") == "richardson":
        out = richardson(lambda v: A @ v, lambda v: apply_precond(st, v), b, rtol=rtol,
                         maxit=opts.maxit, record_iterates=record_iterates)
    else:
        out = fgmres(lambda v: A @ v, lambda v: apply_precond(st, v), b, rtol=rtol,
                     restart=opts.restart, maxit=opts.maxit, record_iterates=record_iterates)
    out["setup"] = st
    return out
