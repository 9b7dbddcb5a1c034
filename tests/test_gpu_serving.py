"""Serving loop: continuous batching of mixed-size solves (C ABI ps_submit / ps_poll / ps_wait).

Each request runs the same kernels on its own stream whether it is alone or in a
mix, with fixed-order reductions, so its result must be bitwise identical in both
cases; admission under a tiny memory budget must serialise requests without
changing results.
"""
import time

import numpy as np
import pytest

from synth import workload

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1812_05540_amd import ps  # noqa: E402

GRIDS = [8, 12, 10, 8, 12, 6]


def requests():
    out = []
    for i, n in enumerate(GRIDS):
        s, b = workload(grid=(n, n, n), kind="grf", seed=5000 + i, rhs_seed=9000 + i,
                        sigma=1.0 + 0.3 * i, e_seed=n)
        out.append((n, s, b))
    return out


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.fixture(scope="module")
def reqs():
    return requests()


def run_alone(ctx, reqs, **opts):
    res = []
    for n, s, b in reqs:
        sv = ps.Solver(ctx, s, mech_key=n, **opts)
        sv.setup()
        x = dev(np.zeros(s.N))
        r = sv.solve(dev(b), x, 1e-8)
        torch.cuda.synchronize()
        res.append((r, x.cpu().numpy()))
        sv.close()
    return res


def run_mix(ctx, reqs, **opts):
    solvers, xs, tickets = [], [], []
    for n, s, b in reqs:
        sv = ps.Solver(ctx, s, mech_key=n, **opts)
        sv.setup()
        solvers.append(sv)
    torch.cuda.synchronize()
    bs = [dev(b) for _, _, b in reqs]
    for sv, (n, s, b), bd in zip(solvers, reqs, bs):
        x = dev(np.zeros(s.N))
        xs.append(x)
        tickets.append(sv.submit(bd, x, 1e-8))
    out = []
    pending = set(range(len(tickets)))
    polled = {}
    t0 = time.time()
    while pending and time.time() - t0 < 60:
        for i in list(pending):
            r = ps.ps_poll(ctx, tickets[i])
            if r["status"] != ps.PS_PENDING:
                polled[i] = r
                pending.discard(i)
        time.sleep(0.001)
    assert not pending, "requests did not finish"
    torch.cuda.synchronize()
    for i in range(len(tickets)):
        out.append((polled[i], xs[i].cpu().numpy()))
    for sv in solvers:
        sv.close()
    return out


@pytest.mark.parametrize("precision,orth", [(ps.PS_FP64, ps.PS_CGS2), (ps.PS_FP32_PREC, ps.PS_CGS2),
                                            (ps.PS_FP32_PREC, ps.PS_DCGS2)])
def test_results_identical_alone_and_in_mix(reqs, precision, orth):
    """Every request bitwise equal alone and in the mix, where requests of one grid size
    share step-1 launches (batched V-cycles over the shared mechanics hierarchy)."""
    ps.load()
    ctx = ps.ps_ctx_create(0, 0)
    try:
        alone = run_alone(ctx, reqs, precision=precision, orth=orth)
        launches0, _ = ps.ps_ctx_batches(ctx)
        mix = run_mix(ctx, reqs, precision=precision, orth=orth)
        launches, covered = ps.ps_ctx_batches(ctx)
    finally:
        ps.ps_ctx_destroy(ctx)
    for (ra, xa), (rm, xm) in zip(alone, mix):
        assert ra["status"] == ps.PS_OK and rm["status"] == ps.PS_OK
        assert ra["iterations"] == rm["iterations"]
        assert np.array_equal(xa, xm)
        assert rm["rel_residual"] <= 1e-8
    # the mix has two requests on each of the 8^3 and 12^3 grids: they shared launches
    print("batched step-1 launch sequences %d covering %d requests" % (launches, covered), flush=True)
    assert launches0 == 0 and launches > 0 and covered >= 2 * launches


def test_admission_under_small_budget_serialises(reqs):
    ps.load()
    ctx = ps.ps_ctx_create(0, 1)          # 1 byte: at most one request on the device at a time
    try:
        alone = run_alone(ctx, reqs[:3])
        mix = run_mix(ctx, reqs[:3])
    finally:
        ps.ps_ctx_destroy(ctx)
    for (ra, xa), (rm, xm) in zip(alone, mix):
        assert rm["status"] == ps.PS_OK and np.array_equal(xa, xm)


def test_wait_and_busy_handle(reqs):
    ps.load()
    ctx = ps.ps_ctx_create(0, 0)
    try:
        n, s, b = reqs[1]
        sv = ps.Solver(ctx, s)
        sv.setup()
        x = dev(np.zeros(s.N))
        t = sv.submit(dev(b), x, 1e-8)
        # a handle with a request in flight refuses a second one (or has just finished it)
        try:
            t2 = sv.submit(dev(b), dev(np.zeros(s.N)), 1e-8)
            ps.ps_wait(ctx, t2)
        except ps.PsError as e:
            assert e.code == ps.PS_EBUSY
        r = ps.ps_wait(ctx, t)
        assert r["status"] == ps.PS_OK and r["iterations"] > 0
        assert ps.ps_wait(ctx, t)["status"] == ps.PS_EINVAL     # a finished ticket is consumed
        sv.close()
    finally:
        ps.ps_ctx_destroy(ctx)


def test_released_handle_is_reused_with_the_same_results():
    """A set-up handle released by ps_destroy is taken by the next ps_create of a system
    with the same mech_key, options and patterns (another field on the same grid): its
    first setup runs the device path, and its solve equals, bit for bit, the solve of a
    fresh handle (host-built first setup) on the same system."""
    from synth.jacobian import box_partition
    ps.load()
    ctx = ps.ps_ctx_create(0, 0)
    try:
        systems = []
        for i in range(2):
            s, b = workload(grid=(10, 10, 10), kind="grf", seed=7100 + i, rhs_seed=9100 + i, sigma=1.5, e_seed=10)
            s.ml_part = box_partition(10, 10, 10, 5, 5, 5)
            systems.append((s, b))
        opts = dict(precision=ps.PS_FP32_PREC, smoother=ps.PS_L1JAC)
        sv = ps.Solver(ctx, systems[0][0], mech_key=10, **opts)
        sv.setup()
        x = dev(np.zeros(systems[0][0].N))
        assert sv.solve(dev(systems[0][1]), x, 1e-8)["status"] == ps.PS_OK
        first = sv.h
        sv.close()                                       # kept by the context
        s, b = systems[1]
        out = []
        for key in (10, 0):                             # reused handle, then a fresh one
            sv = ps.Solver(ctx, s, mech_key=key, **opts)
            if key == 10:
                assert sv.h == first
            sv.setup()
            x = dev(np.zeros(s.N))
            r = sv.solve(dev(b), x, 1e-8)
            torch.cuda.synchronize()
            out.append((r, x.cpu().numpy()))
            sv.close()
        (ra, xa), (rb, xb) = out
        assert ra["status"] == rb["status"] == ps.PS_OK and ra["iterations"] == rb["iterations"]
        assert np.array_equal(xa, xb)
    finally:
        ps.ps_ctx_destroy(ctx)
