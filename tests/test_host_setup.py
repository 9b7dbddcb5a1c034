"""CPU checks of the native library: exported symbols, input validation, and the
host-side setup phase compared with the oracle (bit-for-bit where the arithmetic
is the same sequence of operations)."""
import ctypes
import os
import re

import numpy as np
import pytest

from synth import workload
from oracle import Options
from oracle import precond as P

ps = pytest.importorskip("paper_1812_05540_amd.ps")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    try:
        return ps.load()
    except OSError as e:
        pytest.skip(str(e))


def declared_functions():
    names = []
    for h in ("ps.h", "ps_host.h"):
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"\b(ps_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = _lib()
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(ps.exported_symbols())


def test_header_constants_match_binding():
    """Every integer #define of the two headers has the same value in the Python binding."""
    n = 0
    for h in ("ps.h", "ps_host.h"):
        text = open(os.path.join(ROOT, "include", h)).read()
        for name, val in re.findall(r"^#define\s+(PS_[A-Z0-9_]+)\s+\(?(-?\d+)\)?(?:\s|/\*|$)", text, flags=re.M):
            assert getattr(ps, name) == int(val), name
            n += 1
    assert n >= 20


def test_strerror_and_defaults():
    _lib()
    assert ps.ps_strerror(ps.PS_EINVAL) == "invalid argument"
    o = ps.options()
    assert (o.restart, o.maxit, o.coarse_max, o.max_levels, o.ml_sweeps) == (100, 1000, 256, 25, 1)
    assert o.theta == 0.25 and o.precision == ps.PS_FP64


def _with(system, **changes):
    class S:
        pass
    s = S()
    for k in ("n_nodes", "n_cells", "nf", "p_index", "Auu", "Auf", "Afu", "Aff", "d_sp", "d_pp"):
        setattr(s, k, getattr(system, k))
    for k, v in changes.items():
        setattr(s, k, v)
    return s


@pytest.mark.parametrize("case", ["unsorted", "nan", "missing_diag", "bad_nf", "bad_p_index", "bad_block"])
def test_validation_rejects_bad_input(case):
    _lib()
    s, _ = workload(grid=(3, 2, 2), kind="iid", seed=5, rhs_seed=6)
    from synth.jacobian import BSR
    A = s.Aff
    if case == "unsorted":
        ci = A.colind.copy()
        ci[[0, 1]] = ci[[1, 0]]
        bad = _with(s, Aff=BSR(A.rowptr, ci, A.vals, A.nbcols))
    elif case == "nan":
        v = A.vals.copy()
        v[3, 0, 1] = np.nan
        bad = _with(s, Aff=BSR(A.rowptr, A.colind, v, A.nbcols))
    elif case == "missing_diag":
        rows = np.repeat(np.arange(A.nbrows), np.diff(A.rowptr))
        keep = ~((rows == 0) & (A.colind == 0))
        rp = np.concatenate([[0], np.cumsum(np.bincount(rows[keep], minlength=A.nbrows))]).astype(np.int32)
        bad = _with(s, Aff=BSR(rp, A.colind[keep], A.vals[keep], A.nbcols))
    elif case == "bad_nf":
        bad = _with(s, nf=4)
    elif case == "bad_p_index":
        bad = _with(s, p_index=0)
    else:
        bad = _with(s, Auu=BSR(s.Auu.rowptr, s.Auu.colind, s.Auu.vals[:, :2, :], s.Auu.nbcols))
    with pytest.raises(ps.PsError) as e:
        ps.HostSetup(bad)
    assert e.value.code == ps.PS_EINVAL


def test_bad_options_rejected():
    _lib()
    s, _ = workload(grid=(3, 2, 2), kind="iid", seed=5, rhs_seed=6)
    for kw in (dict(restart=0), dict(ml_sweeps=0), dict(theta=0.0), dict(smoother=7), dict(precision=3)):
        with pytest.raises(ps.PsError) as e:
            ps.HostSetup(s, ps.options(**kw))
        assert e.value.code == ps.PS_EINVAL


def _compare(hs, st, which, levels):
    assert hs.levels(which) == len(levels)
    for l, O in enumerate(levels):
        L = hs.level(which, l)
        assert L["n"] == O.A.shape[0]
        assert np.array_equal(L["rowptr"], O.A.indptr) and np.array_equal(L["colind"], O.A.indices)
        assert np.array_equal(L["vals"], O.A.data), "level %d operator differs" % l
        if O.P is not None:
            assert np.array_equal(L["cf"], O.state)
            assert np.array_equal(L["p_rowptr"], O.P.indptr) and np.array_equal(L["p_colind"], O.P.indices)
            assert np.array_equal(L["p_vals"], O.P.data)
            if O.lam is not None:
                assert abs(hs.lam(which, l) - O.lam) <= 1e-13 * O.lam


@pytest.mark.parametrize("spec,smoother", [
    (dict(grid=(8, 8, 8), kind="iid", seed=1), "cheb2"),
    (dict(grid=(12, 10, 9), kind="grf", seed=7), "cheb2"),
    (dict(grid=(8, 7, 6), kind="iid3", seed=3), "l1jac"),
])
def test_host_setup_matches_oracle_bitwise(spec, smoother):
    _lib()
    s, _ = workload(rhs_seed=1, **spec)
    sm = ps.PS_CHEB2 if smoother == "cheb2" else ps.PS_L1JAC
    hs = ps.HostSetup(s, ps.options(smoother=sm))
    st = P.setup(s, Options(smoother=smoother))
    _compare(hs, st, ps.PS_H_SDC, st.sdc)
    _compare(hs, st, ps.PS_H_PRES, st.pres)
    assert np.array_equal(hs.spp(), st.Spp.data)
    F = hs.bilu()
    _, Fo, Dinv, diag = st.ml[:4]
    Fo = Fo.copy()
    Fo[diag] = Dinv
    assert np.abs(F - Fo).max() <= 1e-12 * np.abs(Fo).max()


def test_processor_local_bilu_matches_oracle():
    _lib()
    from synth.jacobian import box_partition
    s, _ = workload(grid=(12, 10, 8), kind="grf", seed=7, rhs_seed=1)
    s.ml_part = box_partition(12, 10, 8, 4, 5, 4)
    hs = ps.HostSetup(s)
    st = P.setup(s, Options())
    _, Fo, Dinv, diag, lrp, lci = st.ml
    Fo = Fo.copy()
    Fo[diag] = Dinv
    F = hs.bilu()
    # the library exports the factor on the full A_ff pattern; blocks outside the
    # subdomains are not part of the factor
    rows = np.repeat(np.arange(s.n_cells), np.diff(s.Aff.rowptr))
    keep = s.ml_part[rows] == s.ml_part[s.Aff.colind]
    assert np.abs(F[: keep.sum()] - Fo).max() <= 1e-12 * np.abs(Fo).max()
    # 4 + 5 + 4 - 2 wavefronts inside a 4 x 5 x 4 box instead of 12 + 10 + 8 - 2
    assert hs.bilu_levels() == (11, 11)


def test_bilu_level_schedule_counts():
    _lib()
    s, _ = workload(grid=(8, 8, 8), kind="iid", seed=1, rhs_seed=1)
    hs = ps.HostSetup(s)
    # natural order on a 7-point stencil: nx + ny + nz - 2 wavefronts each way
    assert hs.bilu_levels() == (22, 22)
