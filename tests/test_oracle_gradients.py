"""Pins of the oracle's correction-term derivatives (Section 4):
Dx = d/dx[u_x (1 - theta)], Dy = d/dy[u_y (1 - theta)] by second-order
differences, central in the bulk and across periodic wraps, one-sided second
order, (-3 Q0 + 4 Q1 - Q2)/2, on non-periodic edges.  A second-order
difference is exact for a quadratic, so a state whose Q is quadratic along an
axis must give the analytic derivative at every node, edge rows included, to
round-off.  A first-order or mis-signed edge formula, a wrong neighbour or a
dropped factor 1/2 fails these checks."""
import numpy as np
import pytest

import oracle as O


def _quadratic_state(nx, ny, theta, cx, cy, xbc):
    """Fields with Q_x = cx[0] + cx[1] x + cx[2] x^2 on the interior rows and
    Q_y = cy[0] + cy[1] y + cy[2] y^2 everywhere, at uniform temperature theta
    (Q = u (1 - theta)), with node walls on both y sides whose imposed velocity
    and temperature continue the same profiles."""
    x = np.arange(nx, dtype=np.float64)[None, :] * np.ones((ny, 1))
    y = np.arange(ny, dtype=np.float64)[:, None] * np.ones((1, nx))
    qx = cx[0] + cx[1] * x + cx[2] * x * x
    qy = cy[0] + cy[1] * y + cy[2] * y * y
    ux, uy = qx / (1.0 - theta), qy / (1.0 - theta)
    # the wall rows carry the imposed wall velocity, uniform along the wall
    uxw_lo, uxw_hi = 0.01, -0.02
    ux[0, :], ux[-1, :] = uxw_lo, uxw_hi
    uyw_lo, uyw_hi = uy[0, 0], uy[-1, 0]
    p = O.Params(nx=nx, ny=ny, tau_f=0.8, w2=1.1, w3=1.2, w4=0.9,
                 bc=(xbc, xbc, O.WALL, O.WALL), wall_ux=(0.0, 0.0, uxw_lo, uxw_hi),
                 wall_uy=(0.0, 0.0, uyw_lo, uyw_hi), wall_T=(1.0, 1.0, theta, theta))
    rho = 1.0 + 0.01 * np.sin(0.3 * x + 0.2 * y)
    T = np.full((ny, nx), theta)
    return p, rho, ux, uy, T, x, y


@pytest.mark.parametrize("theta", [1.2, 0.85])
def test_one_sided_edge_derivatives_are_exact_for_quadratics(theta):
    nx, ny = 11, 9
    cx = (0.003, -0.0021, 0.00037)
    cy = (-0.002, 0.0017, -0.00029)
    p, rho, ux, uy, T, x, y = _quadratic_state(nx, ny, theta, cx, cy, O.BOUNCEBACK)
    L = O.Lattice(p, rho, ux, uy, T)
    Dx, Dy = L.gradients()
    dy_exact = cy[1] + 2.0 * cy[2] * y
    scale = np.abs(dy_exact).max()
    # every row, the wall rows 0 and ny-1 and their neighbours 1 and ny-2 included
    assert np.abs(Dy - dy_exact).max() < 1e-12 * scale
    for row in (0, 1, ny - 2, ny - 1):
        assert np.abs(Dy[row] - dy_exact[row]).max() < 1e-12 * scale
    # the edge values differ from what a first-order difference would give
    assert abs(Dy[0, 0] - (cy[1])) < 1e-12 * scale
    assert abs((Dy[0, 0]) - (uy[1, 0] - uy[0, 0]) * (1 - theta)) > 1e-2 * scale
    # x: bounce-back sides are non-periodic, so columns 0 and nx-1 take the
    # one-sided difference; interior rows carry the quadratic Q_x, the wall rows
    # a uniform wall velocity (derivative zero)
    dx_exact = cx[1] + 2.0 * cx[2] * x
    sx = np.abs(dx_exact).max()
    assert np.abs(Dx[1:-1] - dx_exact[1:-1]).max() < 1e-12 * sx
    for col in (0, 1, nx - 2, nx - 1):
        assert np.abs(Dx[1:-1, col] - dx_exact[1:-1, col]).max() < 1e-12 * sx
    assert np.abs(Dx[[0, -1]]).max() < 1e-15


def test_periodic_derivative_is_the_central_difference_across_the_wrap():
    """Periodic x: Dx at column 0 and nx-1 uses the neighbour across the wrap."""
    nx, ny = 10, 7
    theta = 1.1
    k = 2 * np.pi / nx
    x = np.arange(nx, dtype=np.float64)[None, :] * np.ones((ny, 1))
    qx = 0.004 * np.sin(k * x + 0.3)
    p = O.Params(nx=nx, ny=ny, tau_f=0.8)
    L = O.Lattice(p, np.ones((ny, nx)), qx / (1 - theta), np.zeros((ny, nx)), np.full((ny, nx), theta))
    Dx, Dy = L.gradients()
    exact = 0.5 * (np.roll(qx, -1, axis=1) - np.roll(qx, 1, axis=1))
    assert np.abs(Dx - exact).max() < 1e-15
    # the central difference of a sine is sin(k)/k times the derivative
    assert np.abs(Dx - np.sin(k) * 0.004 * np.cos(k * x + 0.3)).max() < 1e-15
    assert np.abs(Dy).max() < 1e-15


def test_step_uses_the_exported_gradients():
    """The collision inside a step applies exactly the exported Dx, Dy: one
    oracle step equals the per-node collision with those values followed by
    pull streaming (periodic box)."""
    from paper_1610_07114_amd import workloads as W
    from helpers import EX, EY, oracle_params
    case = W.uniform_noise(9, 8, seed=5, ax=2e-5, ay=-1e-5)
    p = oracle_params(case)
    L = O.Lattice(p, case.rho, case.ux, case.uy, case.T)
    Dx, Dy = L.gradients()
    r, u, v, T = L.macros()
    fo = np.zeros_like(L.f)
    ho = np.zeros_like(L.h)
    for yy in range(case.ny):
        for xx in range(case.nx):
            fo[:, yy, xx], ho[:, yy, xx] = O.collide_node(p, L.f[:, yy, xx], L.h[:, yy, xx], r[yy, xx], u[yy, xx],
                                                          v[yy, xx], T[yy, xx], Dx[yy, xx], Dy[yy, xx], case.ax,
                                                          case.ay)
    f_next = np.stack([np.roll(fo[a], (EY[a], EX[a]), axis=(0, 1)) for a in range(9)])
    h_next = np.stack([np.roll(ho[a], (EY[a], EX[a]), axis=(0, 1)) for a in range(9)])
    L.step(1)
    assert np.abs(L.f - f_next).max() < 1e-15
    assert np.abs(L.h - h_next).max() < 1e-14
