"""Seeded synthetic workloads.

Every workload is a structured grid of 10 m cubes (x fastest), drawn with numpy's
PCG64 generator from a matrix seed; the right-hand side uses its own seed.

  small-iid  : i.i.d. fields -- E lognormal (median 10 GPa, sigma_ln 0.5), Poisson 0.25,
               Biot 1, log10 k ~ N(-13, 1) m^2, porosity U(0.15, 0.3), s_w U(0.2, 0.8);
               two-phase water/oil, viscosities 1 cP / 5 cP, dt = 1 day.  8^3 cells
               (3,211 unknowns) is the reference small case.
  grf        : log10 k a Gaussian random field (correlation 200 m horizontal, 20 m
               vertical, mean -13, sigma 2 unless given), clipped above at LOG10K_MAX;
               porosity 0.15 + 0.15 Phi(g) and ln E = ln(10 GPa) - 0.5 g from the
               standardised field g.  64^3 cells (1,348,163 unknowns) is the reference
               large case.
  layered    : 96 alternating facies layers, channelised (2-D field, 400 m x 40 m,
               mean -12, sigma 1.5) and tight (isotropic 200 m, mean -16, sigma 1).
  grf3       : the grf recipe with three phases (water, gas, oil), saturations uniform
               on the simplex with every saturation >= 0.05.
The paper's SPE10-derived and staircase benchmarks are not available; these
synthetic fields with the paper's property ranges stand in for them.
"""
import numpy as np
from scipy.special import erfc, ndtr

from .grf import gaussian_field, gaussian_field_2d
from .jacobian import build_system, make_rhs, two_phase, three_phase, GRAV
from .state import drive_pressure

H = 10.0
DRIVE = 10e6            # pressure difference of the line drive across the grid (Pa)
# Largest log10 permeability of the random-field workloads (about 20 D, the upper end of
# reservoir rock such as the SPE10 data of the paper's second example).
LOG10K_MAX = -10.7


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _state(nx, ny, nz, kperm, h=H, drive=1.0):
    """Synthetic pressure state and reference pressure (hydrostatic part).

    p = p0 + p_drive: p0 = 20 MPa + rho_w0 g (z_top - z), and p_drive the steady
    single-phase pressure of a 10 MPa line drive along x through the permeability field
    (synth.state.drive_pressure), so that the Darcy fluxes are divergence free inside the
    domain.  drive = +1: pressure rises along x; -1: falls along x (injection at x = 0).
    """
    ck = np.repeat(np.arange(nz), nx * ny)
    zc = (ck + 0.5) * h
    ztop = nz * h
    p0 = 20e6 + 1035.0 * GRAV * (ztop - zc)
    p = p0 + drive_pressure(kperm, nx, ny, nz, h, DRIVE, drive)
    return p, p0


def flood_saturation(nx, ny, nz, g, front=0.4, width=0.05, swr=0.2, snwr=0.2):
    """Waterflood state: water injected across the x = 0 face from s = s_wr (the paper's
    initial state, Sec. 6), front further along permeable streaks.  A time-of-flight
    proxy tau = (x / L_x) exp(-g / 2) (g: standardised log-permeability) sets
    s = s_wr + (1 - s_wr - s_nwr) * erfc((tau - front) / width) / 2."""
    ci = np.tile(np.arange(nx), ny * nz)
    tau = (ci + 0.5) / nx * np.exp(-0.5 * g)
    return (swr + (1.0 - swr - snwr) * 0.5 * erfc((tau - front) / width))[:, None]


def fields_iid(nx, ny, nz, seed):
    rng = _rng(seed)
    n = nx * ny * nz
    E = 10e9 * np.exp(rng.normal(0.0, 0.5, n))
    logk = rng.normal(-13.0, 1.0, n)
    phi = rng.uniform(0.15, 0.3, n)
    S = rng.uniform(0.2, 0.8, (n, 1))
    kperm = 10.0 ** logk
    p, p0 = _state(nx, ny, nz, kperm)
    return dict(E=E, kperm=kperm, phi=phi, S=S, p=p, p0=p0)


def fields_grf(nx, ny, nz, seed, sigma=2.0, mean=-13.0, nph=2, e_seed=None, sat="iid"):
    rng = _rng(seed)
    g = gaussian_field(rng, (nz, ny, nx), H, (20.0, 200.0, 200.0)).ravel()
    if e_seed is not None:
        # mechanics fields fixed per grid (shared displacement block across requests)
        ge = gaussian_field(_rng(e_seed), (nz, ny, nx), H, (20.0, 200.0, 200.0)).ravel()
    else:
        ge = g
    n = nx * ny * nz
    logk = np.minimum(mean + sigma * g, LOG10K_MAX)
    phi = 0.15 + 0.15 * ndtr(g)
    E = np.exp(np.log(10e9) - 0.5 * ge)
    drive = 1.0
    if nph == 2 and sat == "flood":
        S = flood_saturation(nx, ny, nz, g)
        drive = -1.0
    elif nph == 2:
        S = rng.uniform(0.2, 0.8, (n, 1))
    else:
        S = 0.05 + 0.85 * rng.dirichlet(np.ones(3), n)[:, :2]
    kperm = 10.0 ** logk
    p, p0 = _state(nx, ny, nz, kperm, drive=drive)
    return dict(E=E, kperm=kperm, phi=phi, S=S, p=p, p0=p0)


def fields_layered(nx, ny, nz, seed):
    rng = _rng(seed)
    g = np.zeros((nz, ny, nx))
    logk = np.zeros((nz, ny, nx))
    for k in range(nz):
        if k % 2 == 0:
            gk = gaussian_field_2d(rng, (ny, nx), H, (40.0, 400.0))
            logk[k] = -12.0 + 1.5 * gk
        else:
            gk = gaussian_field_2d(rng, (ny, nx), H, (200.0, 200.0))
            logk[k] = -16.0 + 1.0 * gk
        g[k] = gk
    g = g.ravel()
    n = nx * ny * nz
    phi = 0.15 + 0.15 * ndtr(g)
    E = np.exp(np.log(10e9) - 0.5 * g)
    S = rng.uniform(0.2, 0.8, (n, 1))
    kperm = 10.0 ** np.minimum(logk.ravel(), LOG10K_MAX)
    p, p0 = _state(nx, ny, nz, kperm)
    return dict(E=E, kperm=kperm, phi=phi, S=S, p=p, p0=p0)


# name -> (grid, nf, recipe, matrix seed, rhs seed)
WORKLOADS = {
    "iid8": dict(grid=(8, 8, 8), kind="iid", seed=1, rhs_seed=101),
    "grf64": dict(grid=(64, 64, 64), kind="grf", seed=2, rhs_seed=102),
    "layered128": dict(grid=(128, 128, 96), kind="layered", seed=3, rhs_seed=103),
    "grf3ph96": dict(grid=(96, 96, 64), kind="grf3", seed=4, rhs_seed=104, sigma=2.5),
}


def workload(name=None, grid=None, kind="iid", seed=1, rhs_seed=101, sigma=2.0, e_seed=None, sat="iid"):
    """Return (system, rhs) for a named workload or an explicit recipe."""
    if name is not None:
        spec = dict(WORKLOADS[name])
        grid, kind, seed, rhs_seed = spec["grid"], spec["kind"], spec["seed"], spec["rhs_seed"]
        sigma = spec.get("sigma", sigma)
        sat = spec.get("sat", sat)
    nx, ny, nz = grid
    if kind == "iid":
        f, ph = fields_iid(nx, ny, nz, seed), two_phase()
    elif kind == "grf":
        f, ph = fields_grf(nx, ny, nz, seed, sigma=sigma, e_seed=e_seed, sat=sat), two_phase()
    elif kind == "layered":
        f, ph = fields_layered(nx, ny, nz, seed), two_phase()
    elif kind == "grf3":
        f, ph = fields_grf(nx, ny, nz, seed, sigma=sigma, nph=3), three_phase()
    elif kind == "iid3":
        f = fields_iid(nx, ny, nz, seed)
        rng = _rng(seed + 7777)
        f["S"] = 0.05 + 0.85 * rng.dirichlet(np.ones(3), nx * ny * nz)[:, :2]
        ph = three_phase()
    else:
        raise ValueError(kind)
    system = build_system(nx, ny, nz, f, ph)
    system.meta.update(dict(grid=(nx, ny, nz), kind=kind, seed=seed, rhs_seed=rhs_seed, sigma=sigma, sat=sat))
    return system, make_rhs(system, rhs_seed)


def serving_request_spec(i):
    """(n, sigma) of request i of the mixed-size serving stream: grid n^3 drawn uniformly
    from 16, 24, 32, 48, 64 and the log-permeability sigma from U(1, 3)."""
    rng = _rng(77_000 + i)
    n = int(rng.choice([16, 24, 32, 48, 64]))
    sigma = float(rng.uniform(1.0, 3.0))
    return n, sigma


def serving_request(i):
    """Request i of the mixed-size serving stream: its own field (seed 5000 + i) and rhs
    (seed 9000 + i); E fixed per grid size (seed n), so requests of one size share A_uu."""
    n, sigma = serving_request_spec(i)
    return workload(grid=(n, n, n), kind="grf", seed=5000 + i, rhs_seed=9000 + i,
                    sigma=sigma, e_seed=n)
