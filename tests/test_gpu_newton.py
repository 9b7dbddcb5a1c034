"""Inexact Newton loop (Sec. 4) with the library's solve against the same loop driven by
the oracle: per Newton step, the linear iteration count equal to the oracle's +-1, the
forcing terms and residual norms the same to 1e-6 relative.

The step: one backward-Euler day of the 8^3 i.i.d. two-phase recipe (synth.nonlinear),
mechanics AMG built once and reused, flow blocks updated through ps_update_flow and the
flow stage rebuilt on the device at every step, BILU(0) on 4^3-cell subdomains, l1-Jacobi.
"""
import numpy as np
import pytest

from synth.nonlinear import time_step
from synth.jacobian import box_partition
from oracle import Options
from oracle.newton import newton as oracle_newton

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1812_05540_amd import ps  # noqa: E402
from paper_1812_05540_amd.newton import newton  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    ps.load()
    c = ps.ps_ctx_create(0, 0)
    yield c
    ps.ps_ctx_destroy(c)


def problem():
    return time_step((8, 8, 8), kind="iid", seed=1, ml_part=box_partition(8, 8, 8, 4, 4, 4))


def test_newton_three_steps_match_oracle_loop(ctx):
    ref = oracle_newton(problem(), tol=1e-12, max_steps=3, opts=Options(smoother="l1jac"))
    out = newton(ctx, problem(), tol=1e-12, max_steps=3, mech_key=88, precision=ps.PS_FP64,
                 smoother=ps.PS_L1JAC)
    assert len(out["steps"]) == len(ref["steps"]) == 4
    for k, (a, b) in enumerate(zip(out["steps"], ref["steps"])):
        print("step %d: residual %.6e / %.6e" % (k, a["residual"], b["residual"]), a.get("iterations"),
              b.get("iterations"), flush=True)
        assert abs(a["residual"] - b["residual"]) <= 1e-6 * b["residual"]
        if "iterations" in b:
            assert abs(a["eta"] - b["eta"]) <= 1e-6 * b["eta"]
            assert abs(a["iterations"] - b["iterations"]) <= 1
            assert a["status"] == ps.PS_OK and a["step"] == b["step"]
    # the residual falls at every step
    res = [st["residual"] for st in ref["steps"]]
    assert all(r1 < r0 for r0, r1 in zip(res, res[1:]))


def test_newton_converges_with_the_fp32_preconditioner(ctx):
    out = newton(ctx, problem(), tol=1e-8, max_steps=10, mech_key=89, precision=ps.PS_FP32_PREC,
                 smoother=ps.PS_L1JAC)
    assert out["converged"], out["steps"]
