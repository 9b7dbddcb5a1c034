"""Inexact Newton loop with the oracle's linear solve (test infrastructure only).

Sec. 4: Newton's method on the nonlinear residual, each linear system solved to the
relative tolerance eta_k of the Eisenstat-Walker forcing given in the remark there --
eta_0 = 0.1, eta_k = 0.9 (|r_k| / |r_{k-1}|)^2, raised to 0.9 eta_{k-1}^2 when that
exceeds 0.1 -- and, as a reading (the paper keeps eta in [0, 1]), at most 0.9.  The
mechanics hierarchy is built at the first step and reused (Sec. 5.2); the flow stage is
set up again at every step (Sec. 5.4).  Norms are of the scaled residual C r.

Globalisation (the paper applies a backtracking line search when a step fails the
descent condition, remark in Sec. 4).  Reading: the update dx is first scaled so that no
saturation changes by more than 0.2 in one step (lambda_0 = min(1, 0.2 / max |dS|)), then
halved (at most 8 times) until |C r(x + lambda dx)| <= (1 - 1e-4 lambda) |C r(x)|, the
residual scaled with the current state's C.
"""
import numpy as np

from . import amg
from .fgmres import solve
from .precond import Options, setup, sdc_matrix


def ew_eta(k, rnorm, rnorm_prev, eta_prev):
    """Forcing term of Newton step k (k = 0: eta_0)."""
    if k == 0:
        return 0.1
    eta = 0.9 * (rnorm / rnorm_prev) ** 2
    if 0.9 * eta_prev ** 2 > 0.1:
        eta = max(eta, 0.9 * eta_prev ** 2)
    return min(eta, 0.9)


def step_length(problem, x, dx, c, norm):
    """Saturation-limited, backtracked step length (module docstring)."""
    _, dS, _ = problem.split(dx)
    big = float(np.abs(dS).max()) if dS.size else 0.0
    lam = 1.0 if big <= 0.2 else 0.2 / big
    for _ in range(8):
        if np.linalg.norm(c * problem.residual(x + lam * dx)) <= (1.0 - 1e-4 * lam) * norm:
            break
        lam *= 0.5
    return lam


def newton(problem, tol=1e-6, max_steps=10, opts=None, fixed_eta=None):
    opts = opts or Options()
    x = problem.initial_state()
    sdc = None
    steps = []
    norm0 = prev = eta = None
    for k in range(max_steps + 1):
        r = problem.residual(x)
        system = problem.system(x)
        c = problem.scale_vector(system)
        rs = c * r
        norm = float(np.linalg.norm(rs))
        norm0 = norm if k == 0 else norm0
        eta = (fixed_eta if fixed_eta is not None else ew_eta(k, norm, prev, eta))
        steps.append(dict(residual=norm))
        if norm <= tol * norm0 or k == max_steps:
            return dict(x=x, converged=norm <= tol * norm0, steps=steps)
        if sdc is None:
            sdc = amg.build(sdc_matrix(system), theta=opts.theta, coarse_max=opts.coarse_max,
                            max_levels=opts.max_levels, smoother=opts.smoother)
        st = setup(system, opts, mechanics=sdc)
        out = solve(system, -rs, rtol=eta, opts=opts, setup_result=st)
        dx = c * out["x"]
        lam = step_length(problem, x, dx, c, norm)
        steps[-1].update(eta=eta, iterations=out["iterations"], status=out["status"],
                         rel_residual=out["rel_residual"], step=lam)
        x = x + lam * dx
        prev = norm
