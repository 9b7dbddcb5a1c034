"""ps_solve_noalloc (FGMRES workspace in the library's static device scratch) against
ps_solve (workspace allocated by the handle), through the C ABI.

Both run the same kernels on the same handle data; only the workspace addresses differ,
and every reduction has a fixed order, so the iterates are expected to agree bit for
bit: iteration counts and statuses equal, solutions equal to 1e-14 relative (the FP64
parity bar of the other tests, tightened because nothing differs but addresses).  Two
calls in a row, the second on a smaller system, so that the second call finds the
first call's contents in the scratch.
"""
import numpy as np
import pytest

from synth import workload

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1812_05540_amd import ps  # noqa: E402


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    ps.load()
    c = ps.ps_ctx_create(0, 0)
    yield c
    ps.ps_ctx_destroy(c)


CASES = [
    (dict(grid=(12, 11, 10), kind="grf", seed=2, rhs_seed=102), dict(precision=ps.PS_FP32_PREC)),
    (dict(grid=(8, 8, 8), kind="iid", seed=1, rhs_seed=101), dict(precision=ps.PS_FP32_PREC)),
    (dict(grid=(9, 8, 7), kind="iid3", seed=3, rhs_seed=103), dict()),
    (dict(grid=(7, 6, 5), kind="iid3", seed=3, rhs_seed=103), dict(smoother=ps.PS_L1JAC)),
    (dict(grid=(12, 11, 10), kind="grf", seed=2, rhs_seed=102), dict(precision=ps.PS_FP32_PREC, orth=ps.PS_DCGS2)),
    (dict(grid=(8, 8, 8), kind="iid", seed=1, rhs_seed=101), dict(orth=ps.PS_DCGS2)),
]


@pytest.mark.parametrize("first,second", [(0, 1), (2, 3), (4, 5)])
def test_noalloc_solve_equals_allocating_solve(ctx, first, second):
    for idx in (first, second):                # the second system is smaller than the first
        spec, opts = CASES[idx]
        s, b = workload(**spec)
        print("no-alloc case", idx, spec["grid"], spec["kind"], opts, flush=True)
        sv = ps.Solver(ctx, s, **opts)
        sv.setup()
        bd = dev(b)
        x_ref = dev(np.zeros(s.N))
        r_ref = sv.solve(bd, x_ref, 1e-8)
        x = dev(np.full(s.N, 7.0))             # x is overwritten (x0 = 0)
        r = ps.ps_solve_noalloc(sv.h, bd, x, 1e-8)
        torch.cuda.synchronize()
        assert r["status"] == r_ref["status"] == ps.PS_OK, (r, r_ref)
        assert r["iterations"] == r_ref["iterations"]
        assert abs(r["rel_residual"] - r_ref["rel_residual"]) <= 1e-14 * max(1.0, r_ref["rel_residual"])
        xr = x_ref.cpu().numpy()
        err = np.linalg.norm(x.cpu().numpy() - xr) / np.linalg.norm(xr)
        assert err <= 1e-14, err
        sv.close()


def test_noalloc_rejects_a_workspace_beyond_the_scratch(ctx):
    """A system whose workspace exceeds the static array is refused on the host,
    before any launch."""
    s, b = workload(grid=(32, 32, 32), kind="iid", seed=1, rhs_seed=101)   # N = 173,347
    sv = ps.Solver(ctx, s)                    # FP64, restart 100: 1616 N bytes = 280 MB > 256 MiB
    sv.setup()
    x = dev(np.zeros(s.N))
    r = ps.ps_solve_noalloc(sv.h, dev(b), x, 1e-8)
    assert r["status"] == ps.PS_EINVAL
    assert "scratch" in ps.ps_last_error()
    sv.close()
