"""Inexact Newton loop around the library's linear solve (Sec. 4).

Each Newton step solves the scaled Jacobian system J~ dy = -C r to the relative tolerance
eta_k of the Eisenstat-Walker forcing the paper recommends (remark in Sec. 4):

    eta_0 = 0.1,   eta_k = gamma (|r_k| / |r_{k-1}|)^omega,   gamma = 0.9, omega = 2,
    eta_k <- max(eta_k, gamma eta_{k-1}^omega)  whenever  gamma eta_{k-1}^omega > 0.1,

capped at eta_max = 0.9 (reading: the paper leaves eta in [0, 1]).  The mechanics AMG is
built once, with the first setup, and reused by every step (Sec. 5.2: A_uu does not change);
each later step passes the new state's flow blocks, fixed-stress terms and coupling values
through ps_update_flow and rebuilds only the flow stage with ps_setup (Sec. 5.4).

Globalisation (the paper backtracks when a step fails the descent condition, remark in
Sec. 4): the update is scaled so that no saturation changes by more than 0.2, then halved
(at most 8 times) until |C r(x + lambda dx)| <= (1 - 1e-4 lambda) |C r(x)|.

The residual and the Jacobian at a state come from the caller's problem object (physics,
outside the library): initial_state(), residual(x), system(x) (a scaled system with
scale_u / scale_f) and scale_vector(system).  This module holds only the loop; every
linear-algebra step runs in the library.
"""
import numpy as np

from . import ps

GAMMA, OMEGA, ETA0, ETA_MAX = 0.9, 2.0, 0.1, 0.9


def forcing(rnorm, rnorm_prev, eta_prev):
    """Eisenstat-Walker forcing term of the Sec. 4 remark."""
    eta = GAMMA * (rnorm / rnorm_prev) ** OMEGA
    safe = GAMMA * eta_prev ** OMEGA
    if safe > 0.1:
        eta = max(eta, safe)
    return min(eta, ETA_MAX)


def _step_length(problem, x, dx, c, norm):
    _, dS, _ = problem.split(dx)
    big = float(np.abs(dS).max()) if dS.size else 0.0
    lam = 1.0 if big <= 0.2 else 0.2 / big
    for _ in range(8):
        if np.linalg.norm(c * problem.residual(x + lam * dx)) <= (1.0 - 1e-4 * lam) * norm:
            return lam
        lam *= 0.5
    return lam


def newton(ctx, problem, tol=1e-6, max_steps=10, mech_key=1, fixed_eta=None, **opts):
    """Newton iterations until |C r_k| <= tol |C r_0| (scaled residual).

    fixed_eta: a constant linear tolerance instead of the forcing (the paper's own runs).
    Returns dict(x, converged, steps=[dict(residual, eta, iterations, status, rel_residual,
    setup_s, solve_s)]).
    """
    import torch

    x = problem.initial_state()
    r = problem.residual(x)
    sysm = problem.system(x)
    c = problem.scale_vector(sysm)
    sv = ps.Solver(ctx, sysm, mech_key=mech_key, **opts)
    steps = []
    norm0 = prev = None
    eta = None
    converged = False
    try:
        sv.setup()
        for k in range(max_steps + 1):
            rs = c * r
            norm = float(np.linalg.norm(rs))
            if k == 0:
                norm0 = norm
                eta = ETA0 if fixed_eta is None else fixed_eta
            elif fixed_eta is None:
                eta = forcing(norm, prev, eta)
            steps.append(dict(residual=norm))
            if norm <= tol * norm0:
                converged = True
                break
            if k == max_steps:
                break
            b = torch.as_tensor(-rs, dtype=torch.float64, device="cuda")
            dy = torch.zeros_like(b)
            res = sv.solve(b, dy, eta)
            if res["status"] not in (ps.PS_OK, ps.PS_EMAXIT):
                raise ps.PsError(res["status"], "ps_solve in Newton step %d" % k)
            steps[-1].update(eta=eta, iterations=res["iterations"], status=res["status"],
                             rel_residual=res["rel_residual"], setup_s=res["setup_s"], solve_s=res["solve_s"])
            dx = c * dy.cpu().numpy()
            lam = _step_length(problem, x, dx, c, norm)
            steps[-1]["step"] = lam
            x = x + lam * dx
            prev = norm
            r = problem.residual(x)
            sysm = problem.system(x)
            c = problem.scale_vector(sysm)
            ps.ps_update_flow(sv.h, sysm.Afu.vals, sysm.Aff.vals, sysm.d_sp, sysm.d_pp, sysm.Auf.vals)
            sv.setup()
    finally:
        sv.close()
    return dict(x=x, converged=converged, steps=steps)
