"""A nonlinear time step of the synthetic poromechanics problem, for Newton loops.

Input side (physics, no solver arithmetic): the residual r(x) of one backward-Euler step
(Sec. 3, eq. NL_res) at a state x = (u, S, p) and the Jacobian system at that state in
the same scaled block form as `build_system` (App. B).  The time step starts from the
synthetic state of the workload (u = 0, S_0, p_0), which is taken to be in mechanical
equilibrium, so

  r_u(x) = A_uu u + B (p - p_0) + G(S, p) - G(S_0, p_0),
           B: the Biot coupling -b int div(eta) per cell, G: the fluid part of the
           gravity body force, g (V / 8) phi_0 sum_l s_l rho_l(p) on the z component of
           each of the cell's nodes (A_uu is the constant elasticity block, Sec. 5.2);
  r_f(x) = R_flow(S, p, eps_v(u)) - R_acc(S_0, p_0),
           R_flow the mass balance of each phase with the porosity phi_0 + b eps_v(u)
           (`flow_residual`), R_acc the accumulation at the start of the step and
           eps_v(u) = (1 / V) sum_a int grad(N_a) . u_a per cell.

The Jacobian blocks are those `assemble` forms at (S, p) -- the flow accumulation and
the coupling terms at phi_0 -- so the Newton iteration is exact up to the O(b eps_v)
porosity change in those terms.  Residuals and solutions cross the library in the scaled
variables: J~ = C J C, J~ dy = -C r, dx = C dy.
"""
import numpy as np

from .jacobian import (assemble, apply_bc, apply_scaling, constrained_mask, flow_residual, q1_cube,
                       PoroSystem, _cell_ijk, GRAV)


class TimeStep:
    def __init__(self, nx, ny, nz, fields, phases, h=10.0, dt=86400.0, nu=0.25, biot=1.0, ml_part=None):
        self.grid = (nx, ny, nz)
        self.ml_part = ml_part                 # subdomain id per cell, attached to every system
        self.fields = dict(fields)
        self.phases = phases
        self.h, self.dt, self.nu, self.biot = h, dt, nu, biot
        self.nf = phases.nph
        self.nc = nx * ny * nz
        self.nn = (nx + 1) * (ny + 1) * (nz + 1)
        _, self.Gd, _, self.V = q1_cube(h, nu)
        ci, cj, ck = _cell_ijk(nx, ny, nz)
        sx, sxy = nx + 1, (nx + 1) * (ny + 1)
        base = ci + sx * cj + sxy * ck
        self.node_of = np.stack([base + (a & 1) + sx * ((a >> 1) & 1) + sxy * ((a >> 2) & 1)
                                 for a in range(8)], 1)                          # (nc, 8)
        self.mask = constrained_mask(nx, ny, nz).ravel()
        self.S0 = np.array(fields["S"], np.float64)
        self.p0 = np.array(fields["p"], np.float64)
        parts = assemble(nx, ny, nz, self.fields, phases, h=h, dt=dt, nu=nu, biot=biot)
        self.props = parts["props"]
        # constant elasticity block (unscaled, constrained rows decoupled)
        apply_bc(parts, constrained_mask(nx, ny, nz))
        A = parts["Auu"]
        self._auu = (A.rowptr, A.colind, A.vals.copy())
        self.R_acc0 = self._accumulation(self.S0, self.p0, np.zeros(self.nc))
        self.G0 = self._gravity(self.S0, self.p0)

    # ------------------------------------------------------------------ pieces
    def eps_v(self, u):
        U = u.reshape(self.nn, 3)
        return np.einsum("cad,ad->c", U[self.node_of], self.Gd) / self.V

    def _accumulation(self, S, p, epsv):
        ph = self.phases
        phi = self.props["phi0"] + self.biot * epsv
        rho = ph.rho0[None, :] * (1.0 + ph.comp[None, :] * (p - self.props["p0"])[:, None])
        return self.V * phi[:, None] * rho * ph.saturations(S)

    def _gravity(self, S, p):
        """Fluid gravity force per node (z component), (nn,)."""
        ph = self.phases
        rho = ph.rho0[None, :] * (1.0 + ph.comp[None, :] * (p - self.props["p0"])[:, None])
        f = GRAV * (self.V / 8.0) * self.props["phi0"] * (ph.saturations(S) * rho).sum(1)
        out = np.zeros(self.nn)
        np.add.at(out, self.node_of.ravel(), np.repeat(f, 8))
        return out

    def _auu_dot(self, u):
        rp, ci, vals = self._auu
        U = u.reshape(self.nn, 3)
        rows = np.repeat(np.arange(self.nn), np.diff(rp))
        y = np.zeros((self.nn, 3))
        np.add.at(y, rows, np.einsum("bij,bj->bi", vals, U[ci]))
        return y.ravel()

    # ------------------------------------------------------------------ residual
    def split(self, x):
        nu = 3 * self.nn
        xf = x[nu:].reshape(self.nc, self.nf)
        return x[:nu], xf[:, : self.nf - 1], xf[:, self.nf - 1]

    def join(self, u, S, p):
        return np.concatenate([u, np.concatenate([S, p[:, None]], 1).ravel()])

    def initial_state(self):
        return self.join(np.zeros(3 * self.nn), self.S0, self.p0)

    def residual(self, x):
        """Unscaled residual r(x), constrained displacement rows zero."""
        u, S, p = self.split(x)
        # mechanics: elasticity + Biot coupling + fluid gravity, relative to the start
        ru = self._auu_dot(u)
        dp = p - self.p0
        bforce = np.zeros((self.nn, 3))
        for a in range(8):
            np.add.at(bforce, self.node_of[:, a], -self.biot * dp[:, None] * self.Gd[a][None, :])
        ru = ru + bforce.ravel()
        g = self._gravity(S, p) - self.G0
        ru.reshape(self.nn, 3)[:, 2] += g
        ru[self.mask] = 0.0
        rf = flow_residual(S, p, self.eps_v(u), self.props) - self.R_acc0
        return np.concatenate([ru, rf.ravel()])

    # ------------------------------------------------------------------ Jacobian
    def system(self, x):
        """Scaled Jacobian system at x (a PoroSystem, as build_system returns)."""
        u, S, p = self.split(x)
        f = dict(self.fields)
        f["S"] = np.ascontiguousarray(S)
        f["p"] = np.ascontiguousarray(p)
        nx, ny, nz = self.grid
        parts = assemble(nx, ny, nz, f, self.phases, h=self.h, dt=self.dt, nu=self.nu, biot=self.biot)
        mask = constrained_mask(nx, ny, nz)
        apply_bc(parts, mask)
        cu, cf = apply_scaling(parts, self.nf)
        return PoroSystem(nx=nx, ny=ny, nz=nz, nf=self.nf, p_index=self.nf - 1,
                          Auu=parts["Auu"], Auf=parts["Auf"], Afu=parts["Afu"], Aff=parts["Aff"],
                          d_sp=np.ascontiguousarray(parts["d_sp"]), d_pp=np.ascontiguousarray(parts["d_pp"]),
                          constrained=mask.ravel(), scale_u=cu, scale_f=cf, ml_part=self.ml_part)

    def scale_vector(self, system):
        """The diagonal of C (per unknown) for a system returned by `system`."""
        return np.concatenate([np.full(3 * self.nn, system.scale_u),
                               np.tile(system.scale_f, self.nc)])


def time_step(grid=(6, 5, 4), kind="iid", seed=1, **kw):
    """A TimeStep on a workload recipe of synth.configs (fields and phases)."""
    from . import configs as C
    nx, ny, nz = grid
    if kind == "iid":
        f, ph = C.fields_iid(nx, ny, nz, seed), C.two_phase()
    elif kind == "grf":
        f, ph = C.fields_grf(nx, ny, nz, seed, sigma=kw.pop("sigma", 2.0)), C.two_phase()
    elif kind == "iid3":
        f = C.fields_iid(nx, ny, nz, seed)
        rng = C._rng(seed + 7777)
        f["S"] = 0.05 + 0.85 * rng.dirichlet(np.ones(3), nx * ny * nz)[:, :2]
        ph = C.three_phase()
    else:
        raise ValueError(kind)
    return TimeStep(nx, ny, nz, f, ph, **kw)
