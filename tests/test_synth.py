"""Checks of the synthetic-Jacobian generator against closed forms and finite differences."""
import numpy as np
import pytest

from synth import jacobian as J
from synth import workload
from synth.configs import fields_iid


def test_sizes_match_structured_grid_counts(iid8):
    s, b = iid8
    # 8^3 cells: 729 nodes, 27-point node stencil, 8 nodes per cell, 7-point cell stencil
    assert (s.n_nodes, s.n_cells, s.N) == (729, 512, 3211)
    assert s.Auu.nblocks == 25 ** 3
    assert s.Auf.nblocks == s.Afu.nblocks == 8 * 512
    assert s.Aff.nblocks == 512 + 2 * 3 * 8 * 8 * 7
    assert b.shape == (3211,)


def test_q1_stiffness_symmetric_psd_with_rigid_modes():
    K, Gd, Gn, V = J.q1_cube(10.0, 0.25)
    K = K.reshape(24, 24)
    assert np.array_equal(K, K.T)
    w = np.linalg.eigvalsh(K)
    assert w.min() > -1e-12 * w.max()
    assert np.sum(np.abs(w) < 1e-10 * w.max()) == 6       # 3 translations + 3 rotations


def test_q1_divergence_integrals():
    K, Gd, Gn, V = J.q1_cube(10.0, 0.25)
    coords = np.array([[(a >> d) & 1 for d in range(3)] for a in range(8)], float) * 10.0
    assert np.allclose(Gd.sum(0), 0.0, atol=1e-12)           # constants have zero divergence
    assert np.allclose(coords.T @ Gd, V * np.eye(3))          # div(x) integrates to 3V
    # sum_a N_a = 1  ->  sum_a Gn[a, b, c] = Gd[b, c]
    assert np.allclose(Gn.sum(0), Gd)


@pytest.mark.parametrize("nph", [2, 3])
def test_flow_jacobian_matches_finite_differences(nph):
    fld = fields_iid(3, 3, 2, 1)
    if nph == 3:
        rng = np.random.default_rng(3)
        fld["S"] = 0.05 + 0.85 * rng.dirichlet(np.ones(3), 18)[:, :2]
        ph = J.three_phase()
    else:
        ph = J.two_phase()
    parts = J.assemble(3, 3, 2, fld, ph)
    props = parts["props"]
    A = parts["Aff"]
    nc, nf = 18, nph
    D = np.zeros((nc * nf, nc * nf))
    for i in range(nc):
        for t in range(A.rowptr[i], A.rowptr[i + 1]):
            j = A.colind[t]
            D[i * nf:(i + 1) * nf, j * nf:(j + 1) * nf] = A.vals[t]
    S, p = fld["S"], fld["p"]
    eps = np.zeros(nc)
    Dfd = np.zeros_like(D)
    for j in range(nc):
        for d in range(nf):
            h = 1e-6 if d < nf - 1 else 1.0
            Sp, pp, Sm, pm = S.copy(), p.copy(), S.copy(), p.copy()
            if d < nf - 1:
                Sp[j, d] += h
                Sm[j, d] -= h
            else:
                pp[j] += h
                pm[j] -= h
            Dfd[:, j * nf + d] = ((J.flow_residual(Sp, pp, eps, props)
                                   - J.flow_residual(Sm, pm, eps, props)) / (2 * h)).ravel()
    assert np.abs(D - Dfd).max() <= 1e-8 * np.abs(D).max()


def test_flow_to_mechanics_coupling_matches_porosity_derivative():
    """A_fu = d(flow residual)/d(u) through phi = phi0 + b eps_v (eq. linearized_porosity)."""
    fld = fields_iid(2, 2, 2, 4)
    ph = J.two_phase()
    parts = J.assemble(2, 2, 2, fld, ph)
    props = parts["props"]
    K, Gd, Gn, V = J.q1_cube(10.0, 0.25)
    A = parts["Afu"]
    # dR/deps_v by FD, chained with deps_v/du = Gd / V
    h = 1e-7
    R0p = J.flow_residual(fld["S"], fld["p"], np.full(8, h), props)
    R0m = J.flow_residual(fld["S"], fld["p"], np.full(8, -h), props)
    dR = (R0p - R0m) / (2 * h)            # (cells, nph): each cell's own eps_v
    for c in range(8):
        for a in range(8):
            blk = A.vals[c * 8 + a]
            assert np.allclose(blk, dR[c][:, None] * Gd[a][None, :] / V, rtol=1e-6, atol=0)


def test_fixed_stress_diagonals_closed_form(iid8):
    s, _ = iid8
    fld = fields_iid(8, 8, 8, 1)
    E, S, p, p0 = fld["E"], fld["S"][:, 0], fld["p"], fld["p0"]
    rho_w = 1035.0 * (1 + 4.34e-10 * (p - p0))
    rho_o = 863.0 * (1 + 1.98e-10 * (p - p0))
    Kdr = E / (3 * (1 - 2 * 0.25))
    cs, cp = s.scale_f
    assert np.allclose(s.d_sp[:, 0], 1000.0 / Kdr * S * rho_w * cs * cp, rtol=1e-13)
    assert np.allclose(s.d_pp, 1000.0 / Kdr * (1 - S) * rho_o * cp * cp, rtol=1e-13)


def test_constrained_rows_are_decoupled(iid8):
    s, b = iid8
    A = s.Auu
    mask = s.constrained.reshape(-1, 3)
    rows = np.repeat(np.arange(A.nbrows), np.diff(A.rowptr))
    for blk in range(A.nblocks):
        i, j = rows[blk], A.colind[blk]
        for r in range(3):
            for c in range(3):
                if (mask[i, r] or mask[j, c]) and not (i == j and r == c):
                    assert A.vals[blk, r, c] == 0.0
    assert np.all(b[: s.n_u][s.constrained] == 0.0)
    assert np.all(s.Auf.vals[np.repeat(mask, np.diff(s.Auf.rowptr), axis=0)] == 0.0)


def test_scaled_field_diagonals_have_unit_mean(iid8):
    s, _ = iid8
    rows = np.repeat(np.arange(s.n_cells), np.diff(s.Aff.rowptr))
    d = np.abs(np.diagonal(s.Aff.vals[rows == s.Aff.colind], axis1=1, axis2=2))
    assert np.allclose(d.mean(0), 1.0)
    rows = np.repeat(np.arange(s.n_nodes), np.diff(s.Auu.rowptr))
    du = np.abs(np.diagonal(s.Auu.vals[rows == s.Auu.colind], axis1=1, axis2=2))
    assert np.isclose(du.mean(), 1.0)


def test_generator_is_deterministic():
    a, ba = workload(grid=(4, 3, 2), kind="grf", seed=9, rhs_seed=19)
    b, bb = workload(grid=(4, 3, 2), kind="grf", seed=9, rhs_seed=19)
    assert np.array_equal(a.Auu.vals, b.Auu.vals) and np.array_equal(a.Aff.vals, b.Aff.vals)
    assert np.array_equal(ba, bb)


def test_three_phase_layout():
    s, b = workload(grid=(4, 4, 3), kind="iid3", seed=3, rhs_seed=5)
    assert s.nf == 3 and s.p_index == 2
    assert s.Aff.vals.shape[1:] == (3, 3) and s.Afu.vals.shape[1:] == (3, 3)
    assert s.d_sp.shape == (48, 2)


@pytest.mark.parametrize("kind", ["iid", "iid3"])
def test_time_step_jacobian_matches_finite_differences(kind):
    """The Jacobian system of synth.nonlinear (unscaled: C^-1 J~ C^-1) against central
    differences of its residual at a perturbed state (u != 0)."""
    from synth.nonlinear import time_step
    from oracle import precond as P
    ts = time_step((4, 3, 3), kind=kind, seed=3)
    rng = np.random.default_rng(0)
    nf, nu = ts.nf, 3 * ts.nn
    scale = np.concatenate([np.full(nu, 1e-9), np.tile([1e-6] * (nf - 1) + [0.1], ts.nc)])
    x = ts.initial_state() + scale * rng.standard_normal(nu + nf * ts.nc)
    system = ts.system(x)
    c = ts.scale_vector(system)
    J = P.system_matrices(system)["A"].toarray() / c[:, None] / c[None, :]
    for _ in range(3):
        v = rng.standard_normal(x.shape) * np.concatenate([np.full(nu, 1e-4), np.tile([1e-3] * (nf - 1) + [1e2], ts.nc)])
        v[:nu][ts.mask] = 0.0
        eps = 1e-4
        fd = (ts.residual(x + eps * v) - ts.residual(x - eps * v)) / (2 * eps)
        jv = J @ v
        for sl in (slice(0, nu), slice(nu, None)):
            assert np.linalg.norm(fd[sl] - jv[sl]) <= 1e-7 * np.linalg.norm(fd[sl])
    # the step starts in mechanical equilibrium with no accumulation change
    r0 = ts.residual(ts.initial_state())
    assert np.all(r0[:nu] == 0.0)
