"""Shared test helpers: D2Q9 velocity tables written out in the tests themselves
(so that checks on the oracle do not reuse its tables) and adapters from a
workload Case to the oracle."""
from __future__ import annotations

import numpy as np

import oracle as O

# Section 2 velocity set, written independently of the oracle source.
ANG = [None] + [(k - 1) * np.pi / 2 for k in range(1, 5)] + [(k - 4.5) * np.pi / 2 for k in range(5, 9)]
EX = np.array([0] + [int(round(np.cos(ANG[k]) * (1 if k <= 4 else np.sqrt(2)))) for k in range(1, 9)])
EY = np.array([0] + [int(round(np.sin(ANG[k]) * (1 if k <= 4 else np.sqrt(2)))) for k in range(1, 9)])


def moments_np(f, cx=0.0, cy=0.0):
    """rho and the nine-moment set about (cx, cy), directly from the definition
    sum_a f_a (e_ax - cx)^p (e_ay - cy)^q / rho, in the order
    [M00, M10, M01, E, N, Pi, M21, M12, M22]."""
    f = np.asarray(f, dtype=np.float64)
    dx, dy = EX - cx, EY - cy
    M = lambda p, q: float(np.sum(f * dx ** p * dy ** q))
    rho = M(0, 0)
    out = np.array([M(0, 0), M(1, 0), M(0, 1), M(2, 0) + M(0, 2), M(2, 0) - M(0, 2), M(1, 1), M(2, 1), M(1, 2),
                    M(2, 2)]) / rho
    return rho, out


def oracle_params(case, **over) -> O.Params:
    kw = dict(nx=case.nx, ny=case.ny, R=case.R, T0=case.T0, gamma=case.gamma, Pr=case.Pr, tau_f=case.tau_f,
              w2=case.w2, w3=case.w3, w4=case.w4, ax=case.ax, ay=case.ay, thermal=case.thermal,
              correction=case.correction, bc=case.bc, wall_ux=case.wall_ux, wall_uy=case.wall_uy,
              wall_T=case.wall_T, ax_field=case.ax_field, ay_field=case.ay_field,
              viscosity_mode=case.viscosity_mode, mu0=case.mu0, energy_df=case.energy_df)
    kw.update(over)
    return O.Params(**kw)


def oracle_lattice(case, **over) -> O.Lattice:
    return O.Lattice(oracle_params(case, **over), case.rho, case.ux, case.uy, case.T)


def random_pops(rng, rho=1.0, spread=0.2):
    """A positive, non-equilibrium population set of total mass rho."""
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    f = w * (1.0 + spread * rng.uniform(-1, 1, 9))
    return rho * f / f.sum()


def taylor_green_e2(N, u0, max_blocks=400, rates=None, threads=None):
    """E2 of the oracle's steady forced Taylor-Green flow (Section 5A) at the
    paper's convergence criterion, E_R < 1e-8 over 1000 steps.  Module-level
    so that worker processes can run several amplitudes side by side."""
    from paper_1610_07114_amd import workloads as W
    if threads:
        O.set_num_threads(threads)
    case = W.taylor_green(N=N, u0=u0)
    if rates:
        case = case.with_(w2=rates[0], w3=rates[1], w4=rates[2])
    L = oracle_lattice(case)
    prev = None
    for _ in range(max_blocks):
        L.step(1000)
        _, ux, uy, _ = L.macros()
        if prev is not None:
            ER = np.sqrt(((ux - prev[0]) ** 2 + (uy - prev[1]) ** 2).sum() / (ux ** 2 + uy ** 2).sum())
            if ER < 1e-8:
                break
        prev = (ux, uy)
    ue, ve = case.meta["ux_exact"], case.meta["uy_exact"]
    return float(np.sqrt(((ux - ue) ** 2 + (uy - ve) ** 2).sum() / (ue ** 2 + ve ** 2).sum()))


def couette_mu_T_fields(Pr, gamma, steps=60000, threads=None, **over):
    """Fields (rho, ux, uy, T) of the Section 5B Couette case with
    mu = mu0 T/T0 after `steps` steps, with oracle option overrides."""
    from paper_1610_07114_amd import workloads as W
    if threads:
        O.set_num_threads(threads)
    case = W.couette_variable_viscosity(Pr=Pr, gamma=gamma)
    return oracle_lattice(case, **over).step(steps).macros()
