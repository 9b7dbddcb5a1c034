"""GPU checks at the full sizes of the benchmark workloads, in the configuration bench.py
times (processor-local BILU(0) on 32x16x16-cell subdomains, l1-Jacobi smoothing).

The oracle cannot run the whole solve at these sizes, so the checks are the ones that
hold at any size: the system SpMV on sampled rows computed one by one from the block
matrices, the true FP64 residual of the returned x, the FP32- and FP64-preconditioned
paths agreeing with each other, and the device-built pressure hierarchy equal to the
host build on every level.  (The oracle comparison in the benchmarked configuration is
in test_gpu_bench_config.py.)
"""
import numpy as np
import pytest

from synth import workload
from synth.jacobian import box_partition

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1812_05540_amd import ps  # noqa: E402


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    ps.load()
    c = ps.ps_ctx_create(0, 0)
    yield c
    ps.ps_ctx_destroy(c)


_cache = {}


def big(name):
    if name not in _cache:
        s, b = workload(name)
        nx, ny, nz = s.meta["grid"]
        s.ml_part = box_partition(nx, ny, nz, 32, 16, 16)
        _cache[name] = (s, b)
    return _cache[name]


def row_of(s, g, x):
    """(row g of A) . x and sum |a_gj x_j|, from the block matrices, entry by entry."""
    nu = 3 * s.n_nodes
    if g < nu:
        i, c = divmod(g, 3)
        blocks = [(s.Auu, 3, 0), (s.Auf, s.nf, nu)]
    else:
        i, c = divmod(g - nu, s.nf)
        blocks = [(s.Afu, 3, 0), (s.Aff, s.nf, nu)]
    acc = mag = 0.0
    for B, bc, off in blocks:
        for t in range(B.rowptr[i], B.rowptr[i + 1]):
            j0 = off + bc * int(B.colind[t])
            xv = x[j0:j0 + bc]
            acc += float(np.dot(B.vals[t, c, :], xv))
            mag += float(np.dot(abs(B.vals[t, c, :]), abs(xv)))
    return acc, mag


def spmv(sv, x):
    y = dev(np.zeros(x.shape[0]))
    sv.spmv(dev(x), y)
    return host(y)


def check_spmv_rows(sv, s, k):
    rng = np.random.default_rng(5)
    x = rng.standard_normal(s.N)
    y = spmv(sv, x)
    for g in rng.choice(s.N, k, replace=False):
        ref, mag = row_of(s, int(g), x)
        assert abs(y[g] - ref) <= 1e-14 * max(mag, 1e-300)


def solve(ctx, s, b, **kw):
    sv = ps.Solver(ctx, s, smoother=ps.PS_L1JAC, **kw)
    sv.setup()
    x = dev(np.zeros(s.N))
    r = sv.solve(dev(b), x, 1e-8)
    xh = host(x)
    # true residual of the returned x, with the library's A x (checked row by row above)
    res = b - spmv(sv, xh)
    sv.close()
    true_rel = np.linalg.norm(res) / np.linalg.norm(b)
    return r, xh, true_rel


def test_grf64_spmv_rows_and_solves(ctx):
    s, b = big("grf64")
    sv = ps.Solver(ctx, s)
    check_spmv_rows(sv, s, 3000)
    sv.close()
    out = {}
    for prec in (ps.PS_FP32_PREC, ps.PS_FP64):
        r, x, true_rel = solve(ctx, s, b, precision=prec, ml_sweeps=2)
        assert r["status"] == ps.PS_OK, r
        assert true_rel <= 1.01e-8 and abs(true_rel - r["rel_residual"]) <= 1e-10, (true_rel, r)
        out[prec] = (r["iterations"], x)
    (i32, x32), (i64, x64) = out[ps.PS_FP32_PREC], out[ps.PS_FP64]
    assert abs(i32 - i64) <= 3
    assert np.linalg.norm(x32 - x64) / np.linalg.norm(x64) <= 1e-6


def test_grf64_pressure_hierarchy_device_equals_host(ctx, monkeypatch):
    s, _ = big("grf64")
    levels = {}
    for mode in (None, "host"):
        if mode:
            monkeypatch.setenv("PS_GALERKIN", mode)
        else:
            monkeypatch.delenv("PS_GALERKIN", raising=False)
        sv = ps.Solver(ctx, s, precision=ps.PS_FP32_PREC, smoother=ps.PS_L1JAC)
        sv.setup()
        nl = sv.pressure_level(0)["nlevels"]
        levels[mode] = [sv.pressure_level(l) for l in range(nl)]
        sv.close()
    monkeypatch.delenv("PS_GALERKIN", raising=False)
    assert len(levels[None]) == len(levels["host"]) >= 3
    for a, h in zip(levels[None], levels["host"]):
        for key in ("rowptr", "colind", "vals", "cf"):
            assert np.array_equal(a[key], h[key])
    _cache.pop("grf64", None)


def both_paths(ctx, name, **kw):
    """FP32- and FP64-preconditioned solves of one workload: both reach rtol 1e-8 with the
    reported true residual, and their solutions agree to 1e-6 (the FP32 path's error
    against the plain FP64 solve, the spec criterion)."""
    s, b = big(name)
    sv = ps.Solver(ctx, s)
    check_spmv_rows(sv, s, 1000)
    sv.close()
    out = {}
    for prec in (ps.PS_FP32_PREC, ps.PS_FP64):
        print(name, "precision", prec, kw, flush=True)
        r, x, true_rel = solve(ctx, s, b, precision=prec, **kw)
        assert r["status"] == ps.PS_OK, r
        assert true_rel <= 1.01e-8 and abs(true_rel - r["rel_residual"]) <= 1e-10, (true_rel, r)
        out[prec] = (r["iterations"], x)
    (i32, x32), (i64, x64) = out[ps.PS_FP32_PREC], out[ps.PS_FP64]
    diff = np.linalg.norm(x32 - x64) / np.linalg.norm(x64)
    print(name, "iterations fp32 %d fp64 %d, solution difference %.2e" % (i32, i64, diff), flush=True)
    assert abs(i32 - i64) <= 3
    assert diff <= 1e-6, diff
    _cache.pop(name, None)


def test_layered128_both_paths(ctx):
    """128 x 128 x 96 cells, 7,988,259 unknowns, facies contrast ~1e6 (the precision
    variant): FP32-preconditioned against plain FP64, three local-stage sweeps."""
    both_paths(ctx, "layered128", ml_sweeps=3)


def test_three_phase_96_both_paths(ctx):
    """96 x 96 x 64 three-phase (3 x 3 flow blocks), 3,604,227 unknowns: both paths reach
    rtol 1e-8, three local-stage sweeps."""
    both_paths(ctx, "grf3ph96", ml_sweeps=3)
