"""The HIP path against the FP64 oracle at the benchmarked size and configuration.

grf64 (64^3 cells, 1,348,163 unknowns) with the benchmark's options -- l1-Jacobi
smoothing, BILU(0) on 16 x 16 x 16-cell subdomains with two sweeps, FGMRES with delayed
re-orthogonalisation -- and ps_setup run
twice, so that the operators the timed steps use (fixed stress, quasi-IMPES, pressure AMG
and subdomain factors built on the device) are the ones compared:
  * one preconditioner application, field by field, in FP64 and FP32;
  * the FGMRES iterates x_5 and x_10 against the oracle's (FP64 path);
  * the full solve's iteration count against the oracle's count stored in
    tests/golden/grf64_bench_oracle.json (written by tests/golden/make_grf64_oracle.py,
    which calls only the oracle), +-1.
"""
import json
import os

import numpy as np
import pytest

from synth import workload
from synth.jacobian import box_partition
from oracle import Options
from oracle import precond as P
from oracle.fgmres import fgmres

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1812_05540_amd import ps  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN_PATH = os.path.join(HERE, "golden", "grf64_bench_oracle.json")
# the configuration the golden file was written for (tests/golden/make_grf64_oracle.py)
CFG = dict(workload="grf64", smoother="l1jac", ml_kind="bilu0", ml_sweeps=2, ml_part=(16, 16, 16),
           restart=100, rtol=1e-8, orth="dcgs2")
OPTS = dict(smoother=ps.PS_L1JAC, ml_kind=ps.PS_BILU0, ml_sweeps=CFG["ml_sweeps"], orth=ps.PS_DCGS2)
# field-by-field bounds, as in test_gpu_parity (FP64: summation order only; FP32: the
# FP32 rounding amplified by the cancellation that forms the saturation field)
FP64_BLOCK_TOL = 1e-11
FP32_BLOCK_TOL = (1e-6, 1e-3, 1e-6)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def block_errors(z, ref, s):
    nu, nf = s.n_u, s.nf
    out = []
    for sl in (lambda a: a[:nu], lambda a: a[nu:].reshape(-1, nf)[:, : nf - 1],
               lambda a: a[nu:].reshape(-1, nf)[:, nf - 1]):
        out.append(np.linalg.norm(sl(z) - sl(ref)) / np.linalg.norm(sl(ref)))
    return out


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    ps.load()
    c = ps.ps_ctx_create(0, 0)
    yield c
    ps.ps_ctx_destroy(c)


@pytest.fixture(scope="module")
def case():
    s, b = workload(CFG["workload"])
    s.ml_part = box_partition(*s.meta["grid"], *CFG["ml_part"])
    print("oracle setup, grf64 benchmark configuration", flush=True)
    st = P.setup(s, Options(smoother=CFG["smoother"], ml_kind=CFG["ml_kind"], ml_sweeps=CFG["ml_sweeps"]))
    return s, b, st


def solver(ctx, s, **kw):
    sv = ps.Solver(ctx, s, **dict(OPTS, **kw))
    sv.setup()
    sv.setup()            # the timed steps' setup: operators rebuilt on the device
    return sv


def test_bench_config_precond_matches_oracle_by_field(ctx, case):
    s, _, st = case
    v = np.random.default_rng(11).standard_normal(s.N)
    ref = P.apply_precond(st, v)
    for prec, tol in ((ps.PS_FP64, (FP64_BLOCK_TOL,) * 3), (ps.PS_FP32_PREC, FP32_BLOCK_TOL)):
        print("precond parity, precision", prec, flush=True)
        sv = solver(ctx, s, precision=prec)
        z = dev(np.zeros(s.N))
        sv.apply_precond(dev(v), z)
        errs = block_errors(host(z), ref, s)
        sv.close()
        print("  field errors u %.2e s %.2e p %.2e" % tuple(errs), flush=True)
        assert all(e <= t for e, t in zip(errs, tol)), (prec, errs)


def test_bench_config_iterates_match_oracle(ctx, case):
    s, b, st = case
    A = st.mats["A"]
    print("oracle FGMRES, 10 iterations", flush=True)
    out = fgmres(lambda v: A @ v, lambda v: P.apply_precond(st, v), b, rtol=1e-30, restart=100, maxit=10,
                 record_iterates=True, orth=CFG["orth"])
    for k in (5, 10):
        sv = solver(ctx, s, precision=ps.PS_FP64, maxit=k)
        x = dev(np.zeros(s.N))
        r = sv.solve(dev(b), x, 1e-30)
        sv.close()
        assert r["status"] == ps.PS_EMAXIT and r["iterations"] == k
        xo = out["iterates"][k - 1]
        err = np.linalg.norm(host(x) - xo) / np.linalg.norm(xo)
        print("  x_%d relative difference %.2e" % (k, err), flush=True)
        assert err <= 1e-9, (k, err)


def test_bench_config_iteration_count_matches_stored_oracle(ctx, case):
    with open(GOLDEN_PATH) as f:
        golden = json.load(f)
    assert golden["config"] == dict(CFG, ml_part=list(CFG["ml_part"]))
    s, b, _ = case
    for prec in (ps.PS_FP64, ps.PS_FP32_PREC):
        sv = solver(ctx, s, precision=prec)
        x = dev(np.zeros(s.N))
        r = sv.solve(dev(b), x, CFG["rtol"])
        sv.close()
        print("  precision %d: %d iterations (oracle %d)" % (prec, r["iterations"], golden["iterations"]),
              flush=True)
        assert r["status"] == ps.PS_OK and r["rel_residual"] <= CFG["rtol"]
        if prec == ps.PS_FP64:
            assert abs(r["iterations"] - golden["iterations"]) <= 1
