"""GPU parity of the HIP path with the FP64 oracle (all calls go through the C ABI).

Tolerances: FP64 kernels differ from the oracle only in summation order and fused
multiply-adds, so single operators agree to ~1e-13 relative; a preconditioner
application chains V-cycles and triangular sweeps and is compared field by field
(displacement, saturation, pressure), each against its own oracle norm, with the
bounds FP64_BLOCK_TOL / FP32_BLOCK_TOL below.  FP64 solves: iteration count
equal to the oracle's +-1 and the solution within 1e-9 of the oracle's iterate at
the same iteration.  FP32 preconditioner: true FP64 residual <= rtol and solution
error vs a tightly converged oracle solution <= 1e-6 or, when the problem's
conditioning makes the FP64 path itself miss that, no worse than 10x the FP64
path's own error.
"""
import numpy as np
import pytest

from synth import workload
from oracle import Options, solve as oracle_solve
from oracle import precond as P

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
    ps.load()                      # fails loudly if the library is missing
    c = ps.ps_ctx_create(0, 0)
    yield c
    ps.ps_ctx_destroy(c)


SMALL = {
    "iid8": dict(grid=(8, 8, 8), kind="iid", seed=1, rhs_seed=101),
    "grf12": dict(grid=(12, 11, 10), kind="grf", seed=2, rhs_seed=102),
    "grf12s1": dict(grid=(12, 11, 10), kind="grf", seed=2, rhs_seed=102, sigma=1.0),
    "iid3ph": dict(grid=(7, 6, 5), kind="iid3", seed=3, rhs_seed=103),
}
_cache = {}


def small(name):
    if name not in _cache:
        _cache[name] = workload(**SMALL[name])
    return _cache[name]


def make_solver(ctx, s, **opts):
    sv = ps.Solver(ctx, s, **opts)
    sv.setup()
    return sv


# Per-field bounds on a preconditioner output, each relative to the oracle's field norm.
# FP64: the kernels differ from the oracle only in summation order and fused multiply-
# adds; measured at most 1.1e-12 (the saturation field, which step 6 forms by
# cancellation: w_s = y_s - S_ss z_s - S_sp z_p with z_s ~ D_ss^-1 y_s), bound 1e-11.
# FP32 preconditioner (unit roundoff 6e-8): measured at most 1.2e-7 (u), 2.6e-7 (p) and
# 1.8e-4 (s, the same cancellation amplifying FP32 rounding by ~1e3); bounds 1e-6, 1e-3,
# 1e-6.
FP64_BLOCK_TOL = 1e-11
FP32_BLOCK_TOL = (1e-6, 1e-3, 1e-6)


def block_errors(z, ref, s):
    """Relative error of each field of a preconditioner output, each against its own
    oracle norm: (z_u, z_s, z_p).  One norm over the whole vector would be dominated
    by the pressure block (|z_u|/|z| ~ 1e-6 on the random fields)."""
    nu, nf = s.n_u, s.nf
    out = []
    for sl in (lambda a: a[:nu], lambda a: a[nu:].reshape(-1, nf)[:, : nf - 1],
               lambda a: a[nu:].reshape(-1, nf)[:, nf - 1]):
        out.append(np.linalg.norm(sl(z) - sl(ref)) / np.linalg.norm(sl(ref)))
    return out


def oracle_opts(**opts):
    return Options(smoother={ps.PS_CHEB2: "cheb2", ps.PS_L1JAC: "l1jac"}[opts.get("smoother", ps.PS_CHEB2)],
                   ml_kind={ps.PS_BILU0: "bilu0", ps.PS_BJACOBI: "bjacobi",
                            ps.PS_MCGS: "mcgs"}[opts.get("ml_kind", ps.PS_BILU0)],
                   ml_sweeps=opts.get("ml_sweeps", 1), restart=opts.get("restart", 100),
                   maxit=opts.get("maxit", 1000),
                   method={ps.PS_FGMRES: "fgmres", ps.PS_RICHARDSON: "richardson"}[opts.get("method", ps.PS_FGMRES)],
                   reduction={ps.PS_QUASI_IMPES: "quasi", ps.PS_TRUE_IMPES: "true"}[
                       opts.get("reduction", ps.PS_QUASI_IMPES)],
                   fixed_stress={ps.PS_FS_GIVEN: "given", ps.PS_FS_RSL: "rsl"}[opts.get("fixed_stress", ps.PS_FS_GIVEN)],
                   fs_iters=opts.get("fs_iters", 10),
                   orth={ps.PS_CGS2: "cgs2", ps.PS_DCGS2: "dcgs2"}[opts.get("orth", ps.PS_CGS2)])


@pytest.mark.parametrize("name", list(SMALL))
def test_spmv_matches_oracle(ctx, name):
    s, _ = small(name)
    A = P.system_matrices(s)["A"]
    x = np.random.default_rng(0).standard_normal(s.N)
    sv = make_solver(ctx, s)
    y = dev(np.zeros(s.N))
    sv.spmv(dev(x), y)
    ref = A @ x
    assert np.abs(host(y) - ref).max() <= 1e-13 * np.abs(ref).max()
    sv.close()


PRECOND_CASES = [
    ("iid8", dict()),
    ("grf12", dict()),
    ("grf12", dict(smoother=ps.PS_L1JAC)),
    ("grf12", dict(ml_sweeps=3)),
    ("grf12", dict(ml_kind=ps.PS_BJACOBI, ml_sweeps=3)),
    ("iid3ph", dict()),
    ("iid3ph", dict(ml_kind=ps.PS_BJACOBI, ml_sweeps=2, smoother=ps.PS_L1JAC)),
    ("grf12", dict(ml_kind=ps.PS_MCGS, ml_sweeps=3)),
    ("iid3ph", dict(ml_kind=ps.PS_MCGS, ml_sweeps=2)),
    # the alternative reductions of Sec. 5.1 / 5.3 (true-IMPES, row-sum-lumped fixed stress)
    ("grf12", dict(reduction=ps.PS_TRUE_IMPES)),
    ("iid3ph", dict(reduction=ps.PS_TRUE_IMPES, smoother=ps.PS_L1JAC)),
    ("grf12", dict(fixed_stress=ps.PS_FS_RSL)),
    ("iid3ph", dict(fixed_stress=ps.PS_FS_RSL, fs_iters=4, smoother=ps.PS_L1JAC)),
]


@pytest.mark.parametrize("name,opts", PRECOND_CASES)
def test_precond_fp64_matches_oracle(ctx, name, opts):
    s, _ = small(name)
    st = P.setup(s, oracle_opts(**opts))
    sv = make_solver(ctx, s, **opts)
    rng = np.random.default_rng(1)
    for _ in range(2):
        v = rng.standard_normal(s.N)
        z = dev(np.zeros(s.N))
        sv.apply_precond(dev(v), z)
        ref = P.apply_precond(st, v)
        errs = block_errors(host(z), ref, s)
        assert max(errs) <= FP64_BLOCK_TOL, errs
    sv.close()


@pytest.mark.parametrize("layout", ["all", "off"])
@pytest.mark.parametrize("name,opts", [("grf12", dict()), ("grf12", dict(smoother=ps.PS_L1JAC)),
                                       ("iid3ph", dict(smoother=ps.PS_L1JAC))])
def test_level_layouts_match_oracle(ctx, name, opts, layout, monkeypatch):
    """Every AMG operator in SELL-64 (one lane per row), or every one in CSR (G lanes per
    row): both give the oracle's preconditioner, in FP64 and in FP32."""
    monkeypatch.setenv("PS_SELL", layout)
    s, _ = small(name)
    st = P.setup(s, oracle_opts(**opts))
    v = np.random.default_rng(4).standard_normal(s.N)
    ref = P.apply_precond(st, v)
    for prec, tol in ((ps.PS_FP64, (FP64_BLOCK_TOL,) * 3), (ps.PS_FP32_PREC, FP32_BLOCK_TOL)):
        sv = make_solver(ctx, s, precision=prec, **opts)
        z = dev(np.zeros(s.N))
        sv.apply_precond(dev(v), z)
        errs = block_errors(host(z), ref, s)
        assert all(e <= t for e, t in zip(errs, tol)), (prec, errs)
        sv.close()


@pytest.mark.parametrize("name", ["iid8", "grf12"])
def test_precond_fp32_close_to_fp64(ctx, name):
    s, _ = small(name)
    sv = make_solver(ctx, s, precision=ps.PS_FP32_PREC)
    st = P.setup(s, Options())
    v = np.random.default_rng(2).standard_normal(s.N)
    z = dev(np.zeros(s.N))
    sv.apply_precond(dev(v), z)
    ref = P.apply_precond(st, v)
    errs = block_errors(host(z), ref, s)
    assert all(e <= t for e, t in zip(errs, FP32_BLOCK_TOL)), errs
    sv.close()


@pytest.mark.parametrize("name,opts", [("iid8", dict()), ("grf12", dict()), ("grf12", dict(smoother=ps.PS_L1JAC)),
                                       ("grf12", dict(ml_sweeps=2)), ("grf12s1", dict(ml_sweeps=2)),
                                       ("iid3ph", dict(smoother=ps.PS_L1JAC)),
                                       ("grf12", dict(ml_kind=ps.PS_MCGS, ml_sweeps=3)),
                                       # (true-IMPES stalls on the sigma = 2 and three-phase fields,
                                       # whose D_ss keeps only accumulation where transport dominates)
                                       ("iid8", dict(reduction=ps.PS_TRUE_IMPES)),
                                       ("iid3ph", dict(fixed_stress=ps.PS_FS_RSL)),
                                       ("iid8", dict(method=ps.PS_RICHARDSON)),
                                       ("iid3ph", dict(method=ps.PS_RICHARDSON, smoother=ps.PS_L1JAC)),
                                       # delayed re-orthogonalisation against the oracle's DCGS2
                                       ("iid8", dict(orth=ps.PS_DCGS2)),
                                       ("grf12", dict(orth=ps.PS_DCGS2)),
                                       ("grf12", dict(orth=ps.PS_DCGS2, smoother=ps.PS_L1JAC, ml_sweeps=2)),
                                       ("iid3ph", dict(orth=ps.PS_DCGS2, smoother=ps.PS_L1JAC))])
def test_fp64_solve_matches_oracle(ctx, name, opts):
    s, b = small(name)
    out = oracle_solve(s, b, rtol=1e-8, opts=oracle_opts(**opts), record_iterates=True)
    sv = make_solver(ctx, s, **opts)
    x = dev(np.zeros(s.N))
    r = sv.solve(dev(b), x, 1e-8)
    assert r["status"] == ps.PS_OK and r["rel_residual"] <= 1e-8
    assert abs(r["iterations"] - out["iterations"]) <= 1
    k = min(r["iterations"], len(out["iterates"]))
    xo = out["iterates"][k - 1]
    err = np.linalg.norm(host(x) - xo) / np.linalg.norm(xo)
    assert err <= 1e-9, err
    sv.close()


@pytest.mark.parametrize("opts", [dict(ml_sweeps=2), dict(ml_kind=ps.PS_MCGS, ml_sweeps=3),
                                  dict(ml_sweeps=2, orth=ps.PS_DCGS2)])
def test_fp64_iterates_match_oracle_at_matched_k_on_ill_conditioned_field(ctx, opts):
    """sigma = 2 field (cond ~1e10): x_k (GPU stopped by maxit = k) against the oracle's
    x_k at k = 5, 15, 30, each within 1e-9.  Rounding differences (a few 1e-16 per
    operation) grow along the iteration by at most ~1e5 on this field (oracle against
    itself with 1e-13 relative noise on every preconditioner output: drift 4e-9 at k = 5,
    falling to 1e-13 by k = 30), and the GPU's drift measured 2e-10 at most."""
    s, b = small("grf12")
    out = oracle_solve(s, b, rtol=1e-30, opts=oracle_opts(maxit=30, **opts), record_iterates=True)
    errs = []
    for k, tol in ((5, 1e-9), (15, 1e-9), (30, 1e-9)):
        sv = make_solver(ctx, s, maxit=k, **opts)
        x = dev(np.zeros(s.N))
        r = sv.solve(dev(b), x, 1e-30)
        assert r["status"] == ps.PS_EMAXIT and r["iterations"] == k
        xo = out["iterates"][k - 1]
        err = np.linalg.norm(host(x) - xo) / np.linalg.norm(xo)
        errs.append(err)
        sv.close()
        assert err <= tol, (k, err)


@pytest.mark.parametrize("name,orth", [("iid8", ps.PS_CGS2), ("grf12", ps.PS_CGS2), ("iid3ph", ps.PS_CGS2),
                                       ("grf12", ps.PS_DCGS2)])
def test_fp32_solve_reaches_fp64_accuracy(ctx, name, orth):
    s, b = small(name)
    tight = oracle_solve(s, b, rtol=1e-12)["x"]
    A = P.system_matrices(s)["A"]
    res = {}
    for prec in (ps.PS_FP64, ps.PS_FP32_PREC):
        sv = make_solver(ctx, s, precision=prec, orth=orth)
        x = dev(np.zeros(s.N))
        r = sv.solve(dev(b), x, 1e-8)
        xh = host(x)
        assert r["status"] == ps.PS_OK
        true_res = np.linalg.norm(b - A @ xh) / np.linalg.norm(b)
        # the library's FP64 residual and a SciPy recomputation differ by the cancellation
        # error of b - A x, bounded by a few eps |A| |x| / |b|
        cancel = 16 * np.finfo(float).eps * np.linalg.norm(abs(A) @ abs(xh)) / np.linalg.norm(b)
        assert true_res <= 1.01e-8 + cancel and abs(true_res - r["rel_residual"]) <= max(cancel, 1e-13)
        res[prec] = np.linalg.norm(xh - tight) / np.linalg.norm(tight)
        sv.close()
    assert res[ps.PS_FP32_PREC] <= max(1e-6, 10 * res[ps.PS_FP64])


def test_processor_local_bilu_matches_oracle(ctx):
    from synth.jacobian import box_partition
    s, b = workload(grid=(12, 11, 10), kind="grf", seed=2, rhs_seed=102, sigma=1.0)
    s.ml_part = box_partition(12, 11, 10, 6, 6, 5)
    st = P.setup(s, Options())
    sv = make_solver(ctx, s)
    v = np.random.default_rng(3).standard_normal(s.N)
    z = dev(np.zeros(s.N))
    sv.apply_precond(dev(v), z)
    ref = P.apply_precond(st, v)
    assert max(block_errors(host(z), ref, s)) <= FP64_BLOCK_TOL
    out = oracle_solve(s, b, rtol=1e-8, setup_result=st)
    x = dev(np.zeros(s.N))
    r = sv.solve(dev(b), x, 1e-8)
    assert r["status"] == ps.PS_OK and abs(r["iterations"] - out["iterations"]) <= 1
    sv.close()


SUB_CASES = {
    "grf_boxes": (dict(grid=(12, 11, 10), kind="grf", seed=2, rhs_seed=102, sigma=1.0), (6, 6, 5), 1),
    "grf_ragged_2sweeps": (dict(grid=(12, 11, 10), kind="grf", seed=4, rhs_seed=104, sigma=1.0), (5, 4, 3), 2),
    "three_phase": (dict(grid=(7, 6, 5), kind="iid3", seed=3, rhs_seed=103), (4, 3, 5), 1),
    "one_cell_parts": (dict(grid=(5, 4, 3), kind="iid", seed=6, rhs_seed=106), (1, 1, 1), 1),
}


@pytest.mark.parametrize("precision", [ps.PS_FP64, ps.PS_FP32_PREC])
@pytest.mark.parametrize("case", list(SUB_CASES))
def test_subdomain_bilu_kernel_matches_level_kernels(ctx, case, precision, monkeypatch):
    """The LDS-resident subdomain kernel (default with ml_part) and the one-launch-per-
    level kernels compute every row with the same operations in the same order."""
    from synth.jacobian import box_partition
    spec, box, sweeps = SUB_CASES[case]
    s, b = workload(**spec)
    s.ml_part = box_partition(*spec["grid"], *box)
    v = dev(np.random.default_rng(7).standard_normal(s.N))
    out = []
    for mode in (None, "levels"):
        if mode:
            monkeypatch.setenv("PS_BILU_LAUNCH", mode)
        else:
            monkeypatch.delenv("PS_BILU_LAUNCH", raising=False)
        sv = make_solver(ctx, s, precision=precision, ml_sweeps=sweeps)
        z = dev(np.zeros(s.N))
        sv.apply_precond(v, z)
        x = dev(np.zeros(s.N))
        r = sv.solve(dev(b), x, 1e-8)
        out.append((host(z), r, host(x)))
        sv.close()
    monkeypatch.delenv("PS_BILU_LAUNCH", raising=False)
    (za, ra, xa), (zb, rb, xb) = out
    assert np.array_equal(za, zb)
    assert ra["status"] == rb["status"] == ps.PS_OK and ra["iterations"] == rb["iterations"]
    assert np.array_equal(xa, xb)
    if precision == ps.PS_FP64:
        st = P.setup(s, Options(ml_sweeps=sweeps))
        ref = P.apply_precond(st, host(v))
        assert max(block_errors(za, ref, s)) <= FP64_BLOCK_TOL


@pytest.mark.parametrize("precision", [ps.PS_FP64, ps.PS_FP32_PREC])
@pytest.mark.parametrize("case", list(SUB_CASES))
def test_device_bilu_factor_equals_host_factor(ctx, case, precision, monkeypatch):
    """From the second setup of a handle on, the subdomain BILU(0) factor is computed on
    the device from A_ff and the fixed-stress terms; it is the host's factor bit for bit,
    also after new flow values arrive through ps_update_flow."""
    from synth.jacobian import box_partition
    spec, box, sweeps = SUB_CASES[case]
    s, _ = workload(**spec)
    s.ml_part = box_partition(*spec["grid"], *box)
    s2, _ = workload(**dict(spec, seed=spec["seed"] + 10))
    v = dev(np.random.default_rng(8).standard_normal(s.N))
    out = []
    for mode in ("host", None):
        if mode:
            monkeypatch.setenv("PS_BILU_FACTOR", mode)
        else:
            monkeypatch.delenv("PS_BILU_FACTOR", raising=False)
        sv = make_solver(ctx, s, precision=precision, ml_sweeps=sweeps)   # first setup: host factor
        sv.setup()                                                         # then the device's
        z1 = dev(np.zeros(s.N))
        sv.apply_precond(v, z1)
        ps.ps_update_flow(sv.h, s2.Afu.vals, s2.Aff.vals, s2.d_sp, s2.d_pp)
        sv.setup()
        z2 = dev(np.zeros(s.N))
        sv.apply_precond(v, z2)
        out.append((host(z1), host(z2)))
        sv.close()
    monkeypatch.delenv("PS_BILU_FACTOR", raising=False)
    (a1, a2), (b1, b2) = out
    assert np.array_equal(a1, b1)
    assert np.array_equal(a2, b2)
    assert not np.array_equal(a1, a2)


@pytest.mark.parametrize("precision", [ps.PS_FP64, ps.PS_FP32_PREC])
@pytest.mark.parametrize("case", ["grf_boxes", "three_phase"])
def test_device_operators_equal_host_operators(ctx, case, precision, monkeypatch):
    """From the second setup of an l1-Jacobi handle on, S_pp and D_ss (quasi-IMPES) and
    the local-stage factor are formed on the device from the system's A_ff and the
    fixed-stress terms: every pressure level, the preconditioner and the solve are those
    of the host-formed operators bit for bit, also after ps_update_flow."""
    from synth.jacobian import box_partition
    spec, box, sweeps = SUB_CASES[case]
    s, b = workload(**spec)
    s.ml_part = box_partition(*spec["grid"], *box)
    s2, _ = workload(**dict(spec, seed=spec["seed"] + 10))
    v = dev(np.random.default_rng(9).standard_normal(s.N))
    out = []
    for mode in ("host", None):
        for var in ("PS_OPERATORS", "PS_BILU_FACTOR"):
            if mode:
                monkeypatch.setenv(var, mode)
            else:
                monkeypatch.delenv(var, raising=False)
        sv = make_solver(ctx, s, precision=precision, ml_sweeps=sweeps, smoother=ps.PS_L1JAC)
        res = []
        for new_values in (False, True):
            if new_values:
                ps.ps_update_flow(sv.h, s2.Afu.vals, s2.Aff.vals, s2.d_sp, s2.d_pp)
            sv.setup()
            nl = sv.pressure_level(0)["nlevels"]
            levels = [sv.pressure_level(l) for l in range(nl)]
            z = dev(np.zeros(s.N))
            sv.apply_precond(v, z)
            x = dev(np.zeros(s.N))
            r = sv.solve(dev(b), x, 1e-8)
            res.append((levels, host(z), r, host(x)))
        out.append(res)
        sv.close()
    for var in ("PS_OPERATORS", "PS_BILU_FACTOR"):
        monkeypatch.delenv(var, raising=False)
    for (la, za, ra, xa), (lb, zb, rb, xb) in zip(out[0], out[1]):
        assert len(la) == len(lb)
        for p, q in zip(la, lb):
            for key in ("rowptr", "colind", "vals", "cf"):
                assert np.array_equal(p[key], q[key]), key
        assert np.array_equal(za, zb)
        assert ra["status"] == rb["status"] and ra["iterations"] == rb["iterations"]
        assert np.array_equal(xa, xb)


@pytest.mark.parametrize("orth", [ps.PS_CGS2, ps.PS_DCGS2])
def test_solves_are_deterministic(ctx, orth):
    s, b = small("grf12")
    sv = make_solver(ctx, s, orth=orth)
    xs = []
    for _ in range(2):
        x = dev(np.zeros(s.N))
        r = sv.solve(dev(b), x, 1e-8)
        xs.append(host(x))
    assert np.array_equal(xs[0], xs[1])
    sv.close()


@pytest.mark.parametrize("orth", [ps.PS_CGS2, ps.PS_DCGS2])
def test_edge_cases(ctx, orth):
    s, b = small("iid8")
    sv = ps.Solver(ctx, s, orth=orth)
    x = dev(np.zeros(s.N))
    r = sv.solve(dev(b), x, 1e-8)
    assert r["status"] == ps.PS_ENOTSETUP
    sv.setup()
    # zero right-hand side: x = 0 after zero iterations
    x = dev(np.ones(s.N))
    r = sv.solve(dev(np.zeros(s.N)), x, 1e-8)
    assert r["status"] == ps.PS_OK and r["iterations"] == 0 and not host(x).any()
    # invalid tolerance
    r = sv.solve(dev(b), x, 0.0)
    assert r["status"] == ps.PS_EINVAL
    # non-finite right-hand side
    bn = b.copy()
    bn[5] = np.nan
    r = sv.solve(dev(bn), x, 1e-8)
    assert r["status"] == ps.PS_EINVAL
    sv.close()
    # iteration cap: status EMAXIT with the last iterate, which has reduced the residual
    sv = make_solver(ctx, s, maxit=3, orth=orth)
    x = dev(np.zeros(s.N))
    r = sv.solve(dev(b), x, 1e-12)
    assert r["status"] == ps.PS_EMAXIT and r["iterations"] == 3 and r["rel_residual"] < 1.0
    sv.close()


@pytest.mark.parametrize("restart", [1, 2, 3])
def test_dcgs2_shortest_restart_lengths_match_oracle(ctx, restart):
    """Restart lengths 1-3 (twelve iterations, so four to twelve cycles): every cycle ends
    right after its first columns, so the last column is finished at nearly every
    iteration (the delayed pass's corner cases).  The iterate after twelve iterations
    against the oracle's."""
    s, b = small("iid8")
    out = oracle_solve(s, b, rtol=1e-30, opts=oracle_opts(restart=restart, maxit=12, orth=ps.PS_DCGS2))
    sv = make_solver(ctx, s, restart=restart, maxit=12, orth=ps.PS_DCGS2)
    x = dev(np.zeros(s.N))
    r = sv.solve(dev(b), x, 1e-30)
    sv.close()
    assert out["status"] == -6 and r["status"] == ps.PS_EMAXIT and r["iterations"] == 12
    assert r["restarts"] == out["restarts"]
    err = np.linalg.norm(host(x) - out["x"]) / np.linalg.norm(out["x"])
    assert err <= 1e-9, err
    assert abs(r["rel_residual"] - out["rel_residual"]) <= 1e-9 * out["rel_residual"]


@pytest.mark.parametrize("orth", [ps.PS_CGS2, ps.PS_DCGS2])
def test_restarted_solve_matches_oracle(ctx, orth):
    s, b = small("iid8")
    out = oracle_solve(s, b, rtol=1e-8, opts=oracle_opts(restart=7, orth=orth))
    sv = make_solver(ctx, s, restart=7, orth=orth)
    x = dev(np.zeros(s.N))
    r = sv.solve(dev(b), x, 1e-8)
    assert r["status"] == ps.PS_OK
    assert abs(r["iterations"] - out["iterations"]) <= 1 and r["restarts"] >= 3
    assert np.linalg.norm(host(x) - out["x"]) <= 1e-7 * np.linalg.norm(out["x"])
    sv.close()


def test_mech_key_shares_hierarchy_without_changing_results(ctx):
    s, b = small("grf12")
    ref_sv = make_solver(ctx, s)
    x0 = dev(np.zeros(s.N))
    ref_sv.solve(dev(b), x0, 1e-8)
    a = make_solver(ctx, s, mech_key=77)
    bsv = ps.Solver(ctx, s, mech_key=77)
    bsv.setup()
    fa, fb = a.footprint(), bsv.footprint()
    for sv in (a, bsv):
        x = dev(np.zeros(s.N))
        sv.solve(dev(b), x, 1e-8)
        assert np.array_equal(host(x), host(x0))
    assert fa > 0 and fb > 0
    for sv in (ref_sv, a, bsv):
        sv.close()


def test_update_flow_matches_fresh_handle(ctx):
    s, b = small("grf12")
    s2, _ = workload(grid=(12, 11, 10), kind="grf", seed=8, rhs_seed=102)
    sv = make_solver(ctx, s)
    ps.ps_update_flow(sv.h, s2.Afu.vals, s2.Aff.vals, s2.d_sp, s2.d_pp)
    sv.setup()
    # the fresh system with the original displacement block and the new flow blocks
    s3, _ = workload(grid=(12, 11, 10), kind="grf", seed=2, rhs_seed=102)
    s3.Afu, s3.Aff, s3.d_sp, s3.d_pp = s2.Afu, s2.Aff, s2.d_sp, s2.d_pp
    s3.Auf = s.Auf
    ref = make_solver(ctx, s3)
    xa, xb = dev(np.zeros(s.N)), dev(np.zeros(s.N))
    ra = sv.solve(dev(b), xa, 1e-8)
    rb = ref.solve(dev(b), xb, 1e-8)
    assert ra["iterations"] == rb["iterations"]
    assert np.array_equal(host(xa), host(xb))
    sv.close()
    ref.close()


GAL_CASES = {
    "grf12_cheb2": (dict(grid=(12, 11, 10), kind="grf", seed=2, rhs_seed=102, sigma=1.0), ps.PS_CHEB2),
    "grf24_l1jac": (dict(grid=(24, 24, 24), kind="grf", seed=5, rhs_seed=105, sigma=2.0), ps.PS_L1JAC),
    "three_phase": (dict(grid=(12, 10, 8), kind="iid3", seed=3, rhs_seed=103), ps.PS_CHEB2),
    "three_phase_l1jac": (dict(grid=(12, 10, 8), kind="iid3", seed=3, rhs_seed=103), ps.PS_L1JAC),
    "iid8_l1jac": (dict(grid=(8, 8, 8), kind="iid", seed=1, rhs_seed=101), ps.PS_L1JAC),
    "grf12_l1jac": (dict(grid=(12, 11, 10), kind="grf", seed=2, rhs_seed=102, sigma=2.0), ps.PS_L1JAC),
}


@pytest.mark.parametrize("case", list(GAL_CASES))
def test_device_galerkin_hierarchy_equals_oracle_bitwise(ctx, case):
    """Pressure AMG with R (A P) formed on the device (expansion, stable sort, ordered
    sums) -- with l1-Jacobi the whole coarsening too (strength, PMIS, C-promotion, direct
    interpolation): every level operator and C/F splitting equals the oracle's bit for bit."""
    spec, sm = GAL_CASES[case]
    s, _ = workload(**spec)
    sv = make_solver(ctx, s, smoother=sm)
    st = P.setup(s, oracle_opts(smoother=sm))
    assert sv.pressure_level(0)["nlevels"] == len(st.pres) >= 2
    for l, O in enumerate(st.pres):
        L = sv.pressure_level(l)
        assert L["n"] == O.A.shape[0]
        assert np.array_equal(L["rowptr"], O.A.indptr) and np.array_equal(L["colind"], O.A.indices)
        assert np.array_equal(L["vals"], O.A.data), "level %d operator differs" % l
        if O.P is not None:
            assert np.array_equal(L["cf"], O.state)
    sv.close()


def test_device_and_host_galerkin_give_identical_solves(ctx, monkeypatch):
    s, b = workload(**GAL_CASES["grf24_l1jac"][0])
    out = []
    for mode in (None, "host"):
        if mode:
            monkeypatch.setenv("PS_GALERKIN", mode)
        else:
            monkeypatch.delenv("PS_GALERKIN", raising=False)
        sv = make_solver(ctx, s, precision=ps.PS_FP32_PREC, smoother=ps.PS_L1JAC)
        sv.setup()                       # a second setup reuses the recycled device buffers
        v = dev(np.random.default_rng(11).standard_normal(s.N))
        z = dev(np.zeros(s.N))
        sv.apply_precond(v, z)
        x = dev(np.zeros(s.N))
        r = sv.solve(dev(b), x, 1e-8)
        out.append((host(z), r, host(x)))
        sv.close()
    monkeypatch.delenv("PS_GALERKIN", raising=False)
    (za, ra, xa), (zb, rb, xb) = out
    assert np.array_equal(za, zb)
    assert ra["status"] == rb["status"] == ps.PS_OK and ra["iterations"] == rb["iterations"]
    assert np.array_equal(xa, xb)
