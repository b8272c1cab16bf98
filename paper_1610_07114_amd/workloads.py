"""Seeded synthetic workloads shaped like the paper's test problems.

This module only sets up problems: lattice sizes, relaxation parameters derived
from the physical numbers, boundary descriptions and initial macroscopic
fields (rho, u, T) as float64 host arrays indexed [y, x].  It holds none of the
method's arithmetic (no equilibria, moments or collision), so both the HIP
library's callers and the CPU reference can draw their inputs from here.

Lattice units throughout: R = 1/3, T0 = 1, so R*T0 = c_s^2 = 1/3.

Problems (Fei & Luo, arXiv:1610.07114, Section 5, and the project's scaled
workloads):
  couette        thermal Couette flow between a resting and a moving wall
  rayleigh_benard  2:1 box, hot bottom / cold top, gravity as body force
  shock_tube     low-Mach shock tube, bounce-back ends
  taylor_green   steady forced Taylor-Green flow (athermal)
  uniform_noise  periodic box with seeded smooth perturbations (parity work)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional, Tuple

import numpy as np

R_LAT = 1.0 / 3.0
T_REF = 1.0

PERIODIC, BOUNCEBACK, WALL, WALL_ADIABATIC = 0, 1, 2, 3
XLO, XHI, YLO, YHI = 0, 1, 2, 3


@dataclass
class Case:
    name: str
    nx: int
    ny: int
    tau_f: float
    w2: float = 1.0
    w3: float = 1.0
    w4: float = 1.0
    gamma: float = 1.4
    Pr: float = 0.71
    R: float = R_LAT
    T0: float = T_REF
    ax: float = 0.0
    ay: float = 0.0
    thermal: int = 1
    correction: int = 1
    bc: Tuple[int, int, int, int] = (PERIODIC, PERIODIC, PERIODIC, PERIODIC)
    wall_ux: Tuple[float, float, float, float] = (0.0, 0.0, 0.0, 0.0)
    wall_uy: Tuple[float, float, float, float] = (0.0, 0.0, 0.0, 0.0)
    wall_T: Tuple[float, float, float, float] = (1.0, 1.0, 1.0, 1.0)
    rho: Optional[np.ndarray] = None
    ux: Optional[np.ndarray] = None
    uy: Optional[np.ndarray] = None
    T: Optional[np.ndarray] = None
    ax_field: Optional[np.ndarray] = None
    ay_field: Optional[np.ndarray] = None
    viscosity_mode: int = 0              # 1: mu = mu0 T/T0 (Section 5B)
    mu0: float = 0.0
    energy_df: int = 0                   # 1: internal-energy DF (Section 5D)
    steps: int = 0                       # nominal run length of the problem
    meta: dict = field(default_factory=dict)

    @property
    def nodes(self) -> int:
        return self.nx * self.ny

    def fields(self):
        return self.rho, self.ux, self.uy, self.T

    def with_(self, **kw) -> "Case":
        return replace(self, **kw)


def _full(ny, nx, v):
    return np.full((ny, nx), float(v), dtype=np.float64)


def tau_from_nu(nu: float, R: float = R_LAT, T0: float = T_REF) -> float:
    """Kinematic viscosity at the reference state -> 1/w1 (nu = R T0 (1/w1 - 1/2))."""
    return nu / (R * T0) + 0.5


# --------------------------------------------------------------------------------
def couette(nx: int = 8, ny: int = 32, u0: float = 0.05, T_bottom: float = 1.0, T_top: float = 1.02,
            nu: float = 0.05, gamma: float = 1.4, Pr: float = 0.71, w2: float = 1.1, w3: float = 1.6,
            w4: float = 0.3, steps: int = 20000) -> Case:
    """Thermal Couette flow: periodic in x, node walls at y = 0 (resting, T_bottom)
    and y = ny-1 (moving at u0, T_top); H = ny - 1.  Starts from rest with the
    linear conduction profile and uniform density.  w2..w4 default to the
    paper's Couette set (Section 5B)."""
    H = ny - 1
    y = np.arange(ny, dtype=np.float64)[:, None] * np.ones((1, nx))
    T = T_bottom + (T_top - T_bottom) * y / H
    return Case(
        name="couette", nx=nx, ny=ny, tau_f=tau_from_nu(nu), w2=w2, w3=w3, w4=w4, gamma=gamma, Pr=Pr,
        bc=(PERIODIC, PERIODIC, WALL, WALL), wall_ux=(0.0, 0.0, 0.0, u0), wall_T=(1.0, 1.0, T_bottom, T_top),
        rho=_full(ny, nx, 1.0), ux=_full(ny, nx, 0.0), uy=_full(ny, nx, 0.0), T=T, steps=steps,
        meta=dict(u0=u0, H=H, T_bottom=T_bottom, T_top=T_top, nu=nu))


def couette_closed_form(case: Case) -> Tuple[np.ndarray, np.ndarray]:
    """Constant-property plane Couette flow with viscous heating (dynamic
    viscosity and conductivity uniform because the pressure is):
    u = u0 eta,  T = Tb + dT eta + Pr u0^2/(2 c_p) eta (1 - eta),  eta = y/H,
    c_p = (b + 2) R / 2 with b = 2/(gamma - 1)."""
    m = case.meta
    eta = np.arange(case.ny) / m["H"]
    b = 2.0 / (case.gamma - 1.0)
    cp = (b + 2.0) * case.R / 2.0
    u = m["u0"] * eta
    T = m["T_bottom"] + (m["T_top"] - m["T_bottom"]) * eta + case.Pr * m["u0"] ** 2 / (2.0 * cp) * eta * (1 - eta)
    return u, T


def couette_variable_viscosity(Pr: float = 5.0, gamma: float = 5.0 / 3.0, Ma: float = 0.35, nx: int = 5,
                               ny: int = 40, mu0: float = 0.35, w2: float = 1.1, w3: float = 1.6, w4: float = 0.3,
                               steps: int = 120000) -> Case:
    """The thermal Couette flow of Section 5B: dynamic viscosity mu = mu0 T/T0
    (mu0 = 0.35), constant Pr; the upper plate (node wall at y = ny-1) moves at
    U = Ma sqrt(gamma R T0) with T = T0; the lower plate (y = 0) is fixed and
    adiabatic; periodic in x; 5 x 40 nodes, w2, w3, w4 = 1.1, 1.6, 0.3.  Starts
    from rest at T0 and unit density.  tau_f records 1/w1 at unit density."""
    U = Ma * math.sqrt(gamma * R_LAT * T_REF)
    return Case(
        name="couette_mu_T", nx=nx, ny=ny, tau_f=mu0 / (R_LAT * T_REF) + 0.5, w2=w2, w3=w3, w4=w4, gamma=gamma,
        Pr=Pr, bc=(PERIODIC, PERIODIC, WALL_ADIABATIC, WALL), wall_ux=(0.0, 0.0, 0.0, U),
        wall_T=(1.0, 1.0, T_REF, T_REF), rho=_full(ny, nx, 1.0), ux=_full(ny, nx, 0.0), uy=_full(ny, nx, 0.0),
        T=_full(ny, nx, T_REF), viscosity_mode=1, mu0=mu0, steps=steps,
        meta=dict(U=U, Ma=Ma, H=ny - 1, mu0=mu0))


# --------------------------------------------------------------------------------
def rb_parameters(ny: int, Ra: float, Pr: float, dT: float = 0.02, uc: float = 0.08, T0: float = T_REF,
                  R: float = R_LAT):
    """Rayleigh-Benard parameters: H = ny - 1 (node walls), beta = 1/T0,
    u_c = sqrt(g beta dT H), Ra = g beta dT H^3 Pr / nu^2
    => g = u_c^2/(beta dT H), nu = u_c H sqrt(Pr/Ra)."""
    H = ny - 1
    beta = 1.0 / T0
    g = uc * uc / (beta * dT * H)
    nu = uc * H * math.sqrt(Pr / Ra)
    return dict(H=H, g=g, nu=nu, tau_f=tau_from_nu(nu, R, T0), kappa=nu / Pr, dT=dT, uc=uc)


def rayleigh_benard(nx: int = 512, ny: int = 256, Ra: float = 1e5, Pr: float = 0.71, gamma: float = 1.4,
                    dT: float = 0.02, uc: float = 0.08, noise: float = 1e-4, seed: int = 0,
                    steps: int = 200000) -> Case:
    """Rayleigh-Benard convection: periodic in x, node walls at y = 0 (hot,
    T0 + dT/2) and y = ny-1 (cold, T0 - dT/2), gravity a_y = -g as a body
    force (no Boussinesq approximation), w2 = w3 = w4 = 1.

    Initial state: linear conduction profile plus seeded uniform noise of the
    given amplitude on T (interior nodes), u = 0, and the hydrostatic density of
    the conduction profile, p(y) = p_b (T(y)/T_b)^(g H/(R dT)), rho = p/(R T),
    scaled to mean 1."""
    P = rb_parameters(ny, Ra, Pr, dT, uc)
    H = P["H"]
    Tb, Tt = T_REF + 0.5 * dT, T_REF - 0.5 * dT
    y = np.arange(ny, dtype=np.float64)
    Tcond = Tb - dT * y / H
    expo = P["g"] * H / (R_LAT * dT)
    p = (Tcond / Tb) ** expo
    rho_row = p / (R_LAT * Tcond)
    rho_row /= rho_row.mean()
    rng = np.random.default_rng(seed)
    T = np.repeat(Tcond[:, None], nx, axis=1)
    T[1:-1, :] += rng.uniform(-noise, noise, size=(ny - 2, nx))
    rho = np.repeat(rho_row[:, None], nx, axis=1)
    return Case(
        name="rayleigh_benard", nx=nx, ny=ny, tau_f=P["tau_f"], w2=1.0, w3=1.0, w4=1.0, gamma=gamma, Pr=Pr,
        ay=-P["g"], bc=(PERIODIC, PERIODIC, WALL, WALL), wall_T=(1.0, 1.0, Tb, Tt),
        rho=rho, ux=_full(ny, nx, 0.0), uy=_full(ny, nx, 0.0), T=T, steps=steps,
        meta=dict(Ra=Ra, H=H, dT=dT, kappa=P["kappa"], nu=P["nu"], g=P["g"], uc=uc, seed=seed))


TABLE3_RA = (2500.0, 5000.0, 10000.0, 30000.0, 50000.0)
# Nu printed in Section 5D, Table 3: (the paper's scheme, the reference solution)
TABLE3_NU = {2500.0: (1.468, 1.475), 5000.0: (2.106, 2.116), 10000.0: (2.650, 2.661),
             30000.0: (3.629, 3.662), 50000.0: (4.181, 4.245)}


def rb_table3(Ra: float) -> Case:
    """Section 5D's Nu(Ra) runs: 6% temperature difference about T0 = 1,
    u_c = 0.08, Pr = 0.71, w2 = w3 = w4 = 1, a 2:1 box with N_y = 80 below
    Ra = 1e4, 100 below 5e4 and 150 above, the internal-energy DF.  Start:
    the conduction state with a density perturbation of relative amplitude
    1e-3 shaped like the critical mode, cos(2 pi x/nx) sin(pi y/H), i.e. one
    pair of rolls across the box (the paper perturbs the density without
    saying how; random noise grows four rolls at Ra 3e4 and 5e4, a state
    that Table 3's reference values do not describe)."""
    ny = 80 if Ra < 1e4 else (100 if Ra < 5e4 else 150)
    c = rayleigh_benard(nx=2 * ny, ny=ny, Ra=Ra, Pr=0.71, dT=0.06, uc=0.08, noise=0.0)
    H = c.meta["H"]
    y = np.arange(ny, dtype=np.float64)[:, None]
    x = np.arange(2 * ny, dtype=np.float64)[None, :]
    mode = np.cos(2.0 * math.pi * x / (2 * ny)) * np.sin(math.pi * y / H)
    return c.with_(rho=c.rho * (1.0 + 1e-3 * mode), energy_df=1)


# --------------------------------------------------------------------------------
def shock_tube(nx: int = 8192, ny: int = 4, rho_left: float = 1.5, rho_right: float = 1.0, T: float = 1.0,
               w1: float = 1.887, gamma: float = 1.4, Pr: float = 0.71, steps: int = 4000) -> Case:
    """Low-Mach shock tube: left half (x < nx/2) at rho_left, right half at
    rho_right, uniform T, at rest; periodic in y, halfway bounce-back ends;
    w1 = 1.887, w2 = w3 = w4 = 1 (Section 5C)."""
    x = np.arange(nx)
    rho = np.repeat(np.where(x < nx // 2, rho_left, rho_right)[None, :].astype(np.float64), ny, axis=0)
    return Case(
        name="shock_tube", nx=nx, ny=ny, tau_f=1.0 / w1, w2=1.0, w3=1.0, w4=1.0, gamma=gamma, Pr=Pr,
        bc=(BOUNCEBACK, BOUNCEBACK, PERIODIC, PERIODIC),
        rho=rho, ux=_full(ny, nx, 0.0), uy=_full(ny, nx, 0.0), T=_full(ny, nx, T), steps=steps,
        meta=dict(rho_left=rho_left, rho_right=rho_right, T=T))


# --------------------------------------------------------------------------------
def taylor_green(N: int = 64, u0: float = 0.05, nu_phys: float = 0.002) -> Case:
    """Steady forced Taylor-Green flow on [0, 2 pi)^2 with N x N nodes (Section 5A):
    model viscosity nu_m = nu_phys N/(2 pi), all four rates equal (BGK limit),
    body acceleration a = 2 nu_m k^2 u0 (sin kx sin ky, cos kx cos ky), k = 2 pi/N,
    athermal, starting from rest at unit density."""
    nu_m = nu_phys * N / (2.0 * math.pi)
    tau = tau_from_nu(nu_m)
    k = 2.0 * math.pi / N
    i = np.arange(N, dtype=np.float64)
    X, Y = np.meshgrid(i, i)
    amp = 2.0 * nu_m * k * k * u0
    w = 1.0 / tau
    return Case(
        name="taylor_green", nx=N, ny=N, tau_f=tau, w2=w, w3=w, w4=w, thermal=0, correction=0,
        rho=_full(N, N, 1.0), ux=_full(N, N, 0.0), uy=_full(N, N, 0.0), T=_full(N, N, T_REF),
        ax_field=amp * np.sin(k * X) * np.sin(k * Y), ay_field=amp * np.cos(k * X) * np.cos(k * Y),
        meta=dict(u0=u0, k=k, nu_m=nu_m,
                  ux_exact=u0 * np.sin(k * X) * np.sin(k * Y), uy_exact=u0 * np.cos(k * X) * np.cos(k * Y)))


# --------------------------------------------------------------------------------
def _smooth_noise(rng, ny, nx, modes=3):
    """Sum of a few random periodic Fourier modes, unit max amplitude."""
    y = np.arange(ny)[:, None]
    x = np.arange(nx)[None, :]
    out = np.zeros((ny, nx))
    for _ in range(modes):
        kx, ky = rng.integers(0, 4), rng.integers(0, 4)
        ph = rng.uniform(0, 2 * np.pi)
        out += rng.uniform(-1, 1) * np.cos(2 * np.pi * (kx * x / nx + ky * y / ny) + ph)
    m = np.abs(out).max()
    return out / m if m > 0 else out


def uniform_noise(nx: int, ny: int, seed: int = 0, amp_rho: float = 0.05, amp_u: float = 0.05,
                  amp_T: float = 0.05, Tmean: float = 1.0, tau_f: float = 0.7, w2: float = 1.2, w3: float = 1.4,
                  w4: float = 0.9, ax: float = 0.0, ay: float = 0.0, gamma: float = 1.4, Pr: float = 0.71,
                  pointwise: float = 0.0) -> Case:
    """Periodic box with smooth seeded perturbations of rho, u and T (plus optional
    pointwise noise), unequal relaxation rates and an optional uniform force:
    a parity workload that exercises every term of the step, including the
    correction (T != T0 everywhere)."""
    rng = np.random.default_rng(seed)
    rho = 1.0 + amp_rho * _smooth_noise(rng, ny, nx)
    ux = amp_u * _smooth_noise(rng, ny, nx)
    uy = amp_u * _smooth_noise(rng, ny, nx)
    T = Tmean + amp_T * _smooth_noise(rng, ny, nx)
    if pointwise > 0:
        rho += pointwise * rng.uniform(-1, 1, size=(ny, nx))
        ux += pointwise * rng.uniform(-1, 1, size=(ny, nx))
        uy += pointwise * rng.uniform(-1, 1, size=(ny, nx))
        T += pointwise * rng.uniform(-1, 1, size=(ny, nx))
    return Case(name="uniform_noise", nx=nx, ny=ny, tau_f=tau_f, w2=w2, w3=w3, w4=w4, gamma=gamma, Pr=Pr,
                ax=ax, ay=ay, rho=rho, ux=ux, uy=uy, T=T, meta=dict(seed=seed))


# --------------------------------------------------------------------------------
# Below this 1/w1 the default thermal scheme is linearly unstable (spectral
# radius of the linearised step above 1): such lattices blow up whatever the
# arithmetic precision.
TAU_STABLE = 0.55


def rb_tau_f(N: int, Ra: float, Pr: float) -> float:
    """1/w1 of a 2N x N Rayleigh-Benard instance (rb_parameters' viscosity)."""
    return rb_parameters(N, Ra, Pr)["tau_f"]


def batched_rb_specs(n: int = 256, seed: int = 0, nmin: int = 32, nmax: int = 512, Ra_range=(1e4, 1e6),
                     Pr_range=(0.5, 7.0), tau_min: float = TAU_STABLE, rejected: Optional[list] = None) -> List[dict]:
    """Seeded instance list of the batched Rayleigh-Benard workload: N log-uniform
    on [nmin, nmax] (lattice 2N x N), Ra log-uniform, Pr uniform; per-instance
    noise seed = seed + i.  Draws whose 1/w1 falls below `tau_min` (small
    lattices at high Ra and low Pr: too little viscosity for the scheme's
    stability limit) are skipped, so the list holds n instances of the same
    distribution conditioned on linear stability; `rejected` (a list), when
    given, receives the skipped draws.  tau_min = 0 keeps every draw."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        N = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        Ra = math.exp(rng.uniform(math.log(Ra_range[0]), math.log(Ra_range[1])))
        Pr = rng.uniform(*Pr_range)
        spec = dict(nx=2 * N, ny=N, Ra=Ra, Pr=Pr, seed=seed + len(out))
        if rb_tau_f(N, Ra, Pr) < tau_min:
            if rejected is not None:
                rejected.append(spec)
            continue
        out.append(spec)
    return out


def rb_from_spec(spec: dict, steps: int = 0) -> Case:
    c = rayleigh_benard(nx=spec["nx"], ny=spec["ny"], Ra=spec["Ra"], Pr=spec["Pr"], seed=spec["seed"])
    return c.with_(steps=steps)
