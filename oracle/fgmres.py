"""Right-preconditioned flexible GMRES(m) in FP64 (oracle; test infrastructure only).

The paper solves each Jacobian system with right-preconditioned GMRES (Sec. 4,
(A M^{-1}) dy = -r, dx = M^{-1} dy).  Readings where it is silent: restart length
m = 100, flexible variant (Saad, SIAM J. Sci. Comput. 14, 1993) so that a
preconditioner applied in reduced precision stays consistent, classical
Gram-Schmidt applied twice (CGS2) for the Arnoldi step, Givens rotations for the
Hessenberg least-squares problem, x0 = 0, convergence when the true residual
|b - A x| <= rtol |b| at the end of a cycle, a cycle also ends on a happy breakdown
h_{j+1,j} <= 1e-14 |A z_j|, and at most `maxit` iterations in total.

orth = "dcgs2": the same method with the Arnoldi step orthogonalised by classical
Gram-Schmidt with delayed re-orthogonalisation and lagged normalisation (Bielich, Langou,
Thomas, Swirydowicz, Yamazaki, Boman, Parallel Computing 112, 2022).  The vector u_j that
enters the preconditioner has had one Gram-Schmidt pass against the finished basis
v_0..v_{j-1}; its second pass and its normalisation happen in the next iteration, in the
same pass over the basis that projects w = A z_j:

    s = V_j^T u_j,   p = V_j^T w,   alpha = sqrt(u_j.u_j - s.s),   t = (u_j.w - s.p) / alpha,
    v_j = (u_j - V_j s) / alpha,   r_j = w - V_j p - t v_j,   u_{j+1} = r_j / |w|.

Scaling by |w| = |A z_j| (known before the second pass) keeps |u_{j+1}| <= 1 without a pass
of its own, and, unlike leaving u unscaled, does not compound over the iterations.  Column j
of the Hessenberg matrix is (p, t) until the next iteration adds |w| s' and sets
h_{j+1,j} = |w| alpha' (s', alpha' of u_{j+1}); FGMRES keeps z_j = M^{-1} u_j, so
A Z_k = V_{k+1} H_k holds with the finished columns (the flexible method allows any z_j, and
every formula above is invariant to the scale of u_j).  The stopping test after iteration j
uses the Givens estimate of the unfinished column, with |r_j| as its subdiagonal; when the
cycle ends its last column is finished with one more product V^T u_{j+1}.  In exact
arithmetic the iterates equal those of CGS2.
"""
import numpy as np
import scipy.linalg as sla

OK, EMAXIT, EBREAKDOWN = 0, -6, -9


def fgmres(matvec, precond, b, rtol=1e-8, restart=100, maxit=1000, record_iterates=False,
           debug=False, orth="cgs2"):
    """Returns dict(x, iterations, restarts, status, rel_residual, history, iterates).

    history[k] is the Givens residual estimate |g_{k+1}| / |b| after iteration k+1.
    iterates[k] (when recorded) is the iterate x_{k+1} = x_cycle + Z_k H_k^{-1} g_k.
    debug: keep the last cycle's V, Z and unrotated Hessenberg matrix in the result.
    """
    if orth == "dcgs2":
        return _fgmres_dcgs2(matvec, precond, b, rtol, restart, maxit, record_iterates, debug)
    if orth != "cgs2":
        raise ValueError(orth)
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


def _rotate(col, cs, sn, nrot):
    """Apply the first nrot Givens rotations to a Hessenberg column (in place)."""
    for i in range(nrot):
        t = cs[i] * col[i] + sn[i] * col[i + 1]
        col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1]
        col[i] = t


def _finished_column(raw, naz, V, u_next, want_v=False):
    """Column j of H from its first-pass entries raw (length j+1), the scale naz = |A z_j|
    and the vector u_next = r_j / naz that pass left: adds naz s' and sets h_{j+1,j} =
    naz alpha', s' = V_{j+1}^T u_next, alpha' = sqrt(|u_next|^2 - s'.s') (naz = 0: nothing
    to add).  want_v: also return v_{j+1} = (u_next - V_{j+1} s') / alpha' (None when
    alpha' = 0)."""
    j = raw.shape[0] - 1
    col = np.zeros(j + 2)
    col[: j + 1] = raw
    if naz == 0.0:
        return (col, None) if want_v else col
    sp = V[: j + 1] @ u_next
    a2 = u_next @ u_next - sp @ sp
    alpha = np.sqrt(a2) if a2 > 0.0 else 0.0
    col[: j + 1] += naz * sp
    col[j + 1] = naz * alpha
    if want_v:
        return col, ((u_next - V[: j + 1].T @ sp) / alpha if alpha > 0.0 else None)
    return col


def _fgmres_dcgs2(matvec, precond, b, rtol, restart, maxit, record_iterates, debug=False):
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
        V = np.zeros((m + 1, n))          # V[:j] finished; V[j] = u_j while iteration j runs
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))          # finished columns, rotated
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        raw_prev, naz_prev = None, 0.0
        Hraw = np.zeros((m + 1, m))       # finished columns before rotation
        v_last = None
        k = 0
        breakdown = False
        last_open = False                 # the last column still lacks its second pass
        for j in range(m):
            last_open = False
            u = V[j]
            Z[j] = precond(u)
            w = matvec(Z[j])
            norm_az = np.linalg.norm(w)
            # one pass over the finished basis and u_j
            s = V[:j] @ u
            p = V[:j] @ w
            a2 = u @ u - s @ s
            alpha = np.sqrt(a2) if a2 > 0.0 else 0.0
            t = (u @ w - s @ p) / alpha
            v = (u - V[:j].T @ s) / alpha
            V[j] = v
            w = w - V[:j].T @ p - t * v
            hn = np.linalg.norm(w)
            u_next = w / norm_az if norm_az > 0.0 else np.zeros(n)
            if j > 0:
                # column j-1 finished with s and alpha of u_j
                col = np.zeros(j + 1)
                col[:j] = raw_prev + naz_prev * s
                col[j] = naz_prev * alpha
                Hraw[: j + 1, j - 1] = col
                _rotate(col, cs, sn, j - 1)
                rho = np.hypot(col[j - 1], col[j])
                cs[j - 1] = col[j - 1] / rho
                sn[j - 1] = col[j] / rho
                col[j - 1] = rho
                col[j] = 0.0
                H[: j + 1, j - 1] = col
                g[j] = -sn[j - 1] * g[j - 1]
                g[j - 1] = cs[j - 1] * g[j - 1]
            raw = np.concatenate([p, [t]])
            # Givens estimate with the unfinished column j (rotation not kept)
            col = np.concatenate([raw, [hn]])
            _rotate(col, cs, sn, j)
            rho = np.hypot(col[j], col[j + 1])
            k = j + 1
            its += 1
            if rho == 0.0:
                breakdown = True
                break
            est = abs(col[j + 1] / rho * g[j])
            res["history"].append(est / beta_b)
            if record_iterates:
                colf = _finished_column(raw, norm_az, V, u_next)
                _rotate(colf, cs, sn, j)
                rf = np.hypot(colf[j], colf[j + 1])
                Hk = H[:k, :k].copy()
                Hk[: j + 1, j] = colf[: j + 1]
                Hk[j, j] = rf
                gk = g[:k].copy()
                gk[j] = colf[j] / rf * g[j]
                y = sla.solve_triangular(Hk, gk)
                res["iterates"].append(x + Z[:k].T @ y)
            if est <= rtol * beta_b or hn <= 1e-14 * norm_az or its >= maxit:
                # finish the last column, keep its rotation
                col, v_last = _finished_column(raw, norm_az, V, u_next, want_v=True)
                Hraw[: j + 2, j] = col
                _rotate(col, cs, sn, j)
                rho = np.hypot(col[j], col[j + 1])
                cs[j] = col[j] / rho
                sn[j] = col[j + 1] / rho
                col[j] = rho
                col[j + 1] = 0.0
                H[: j + 2, j] = col
                g[j + 1] = -sn[j] * g[j]
                g[j] = cs[j] * g[j]
                break
            V[j + 1] = u_next
            raw_prev, naz_prev = raw, norm_az
            last_open = True
        if last_open:
            # the cycle ran to the restart length: finish its last column
            j = m - 1
            col, v_last = _finished_column(raw, naz_prev, V, V[m], want_v=True)
            Hraw[: j + 2, j] = col
            _rotate(col, cs, sn, j)
            rho = np.hypot(col[j], col[j + 1])
            cs[j] = col[j] / rho
            sn[j] = col[j + 1] / rho
            col[j] = rho
            col[j + 1] = 0.0
            H[: j + 2, j] = col
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
        if breakdown:
            k -= 1
        if debug:
            Vf = V[: k + 1].copy()
            if not breakdown and v_last is not None:
                Vf[k] = v_last
            res["debug"] = dict(V=Vf, Z=Z[:k].copy(), H=Hraw[: k + 1, :k].copy(),
                                last_normalised=not breakdown and v_last is not None)
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
                     restart=opts.restart, maxit=opts.maxit, record_iterates=record_iterates,
                     orth=getattr(opts, "orth", "cgs2"))
    out["setup"] = st
    return out
