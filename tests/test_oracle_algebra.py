"""Pins of the oracle's per-node algebra against identities the paper and the
mathematics fix (Sections 2-4).  Every expected value here is computed by an
independent route: moments straight from their definitions in numpy, the
product-form equilibrium, Maxwellian moments, conservation sums."""
import numpy as np
import pytest

import oracle as O
from helpers import EX, EY, moments_np, random_pops

RT0 = 1.0 / 3.0
rng_seeds = list(range(6))


def test_velocity_set_matches_section2():
    # e_a for a = 1..4 on the axes, 5..8 on the diagonals, counter-clockwise.
    assert list(EX) == [0, 1, 0, -1, 0, 1, -1, -1, 1]
    assert list(EY) == [0, 0, 1, 0, -1, 1, 1, -1, -1]


@pytest.mark.parametrize("seed", rng_seeds)
def test_eq3_inverts_eq1(seed):
    """P1: Eq. (3) is the exact inverse of the nine raw moments of Eq. (1)-(2)."""
    rng = np.random.default_rng(seed)
    f = random_pops(rng, rho=rng.uniform(0.5, 2.0), spread=0.6)
    rho, m = moments_np(f)
    np.testing.assert_allclose(O.pops_from_moments(rho, m), f, rtol=0, atol=1e-15)
    # and the other way round: arbitrary moments -> populations -> same moments
    m2 = np.concatenate([[1.0], rng.uniform(-0.3, 0.3, 8)])
    g = O.pops_from_moments(1.7, m2)
    rho2, back = moments_np(g)
    assert rho2 == pytest.approx(1.7, abs=1e-14)
    np.testing.assert_allclose(back, m2, atol=1e-14)
    # the oracle's own moment routine agrees with the definition
    r3, m3 = O.raw_moments(f)
    assert r3 == pytest.approx(rho, abs=1e-15)
    np.testing.assert_allclose(m3, m, atol=1e-15)


@pytest.mark.parametrize("seed", rng_seeds)
def test_eq9_inverts_eq4(seed):
    """P2: Eq. (9) recovers the raw moments from the central moments of Eq. (4)
    when M10 = ux, M01 = uy (the frame velocity is the DF's own velocity)."""
    rng = np.random.default_rng(100 + seed)
    f = random_pops(rng, rho=rng.uniform(0.5, 2.0), spread=0.8)
    rho, raw = moments_np(f)
    ux, uy = raw[1], raw[2]
    _, cen = moments_np(f, ux, uy)
    _, cen_orc = O.central_moments(f, ux, uy)
    np.testing.assert_allclose(cen_orc, cen, atol=1e-15)
    np.testing.assert_allclose(O.raw_from_central(cen, ux, uy), raw, atol=1e-14)


@pytest.mark.parametrize("seed", rng_seeds)
def test_eq18_is_raw_from_central_of_fbar(seed):
    """P3: Eq. (18) is the exact central->raw map for the transformed DF whose
    first moments are u - a/2 (u the fluid velocity of Eq. (20))."""
    rng = np.random.default_rng(200 + seed)
    fb = random_pops(rng, rho=rng.uniform(0.5, 2.0), spread=0.8)
    ax, ay = rng.uniform(-0.05, 0.05, 2)
    rho, raw = moments_np(fb)
    ux, uy = raw[1] + 0.5 * ax, raw[2] + 0.5 * ay
    _, cen = moments_np(fb, ux, uy)
    np.testing.assert_allclose(O.post_collision_raw(cen, ux, uy, ax, ay), raw, atol=1e-14)


def product_form_feq(rho, ux, uy, RT):
    """D2Q9 equilibrium as a product of 1-D three-velocity factors that match the
    Gaussian moments 1, u, RT + u^2 in each direction."""
    def psi(e, u):
        return 1.0 - RT - u * u if e == 0 else 0.5 * (RT + u * u + e * u)
    return np.array([rho * psi(EX[a], ux) * psi(EY[a], uy) for a in range(9)])


@pytest.mark.parametrize("seed", rng_seeds)
def test_feq_product_form_and_maxwellian_moments(seed):
    """P4: Eq. (7) (T0 -> T) through Eq. (9) and Eq. (3) is the product-form
    equilibrium, whose moments are the continuous Maxwellian's up to the
    lattice-fixed diagonal third moments."""
    rng = np.random.default_rng(300 + seed)
    rho = rng.uniform(0.5, 2.0)
    ux, uy = rng.uniform(-0.15, 0.15, 2)
    RT = RT0 * rng.uniform(0.8, 1.2)
    feq = O.feq(rho, ux, uy, RT)
    np.testing.assert_allclose(feq, product_form_feq(rho, ux, uy, RT), atol=1e-15)
    r, m = moments_np(feq)
    assert r == pytest.approx(rho, rel=1e-14)
    np.testing.assert_allclose(m[1:3], [ux, uy], atol=1e-15)
    np.testing.assert_allclose(m[3], 2 * RT + ux * ux + uy * uy, atol=1e-15)         # trace
    np.testing.assert_allclose(m[4], ux * ux - uy * uy, atol=1e-15)                  # normal difference
    np.testing.assert_allclose(m[5], ux * uy, atol=1e-15)                            # off-diagonal
    np.testing.assert_allclose(m[6], uy * RT + ux * ux * uy, atol=1e-15)             # M21^eq, Section 4
    np.testing.assert_allclose(m[7], ux * RT + uy * uy * ux, atol=1e-15)
    _, c = moments_np(feq, ux, uy)
    np.testing.assert_allclose(c[8], RT * RT, atol=1e-15)                            # Gaussian 4th central
    # third-order diagonal moments are fixed by the lattice (e^3 = e), Section 4
    assert np.sum(feq * EX ** 3) == pytest.approx(np.sum(feq * EX), abs=1e-15)


@pytest.mark.parametrize("seed", rng_seeds)
def test_bgk_limit(seed):
    """P5: equal rates, no force, no correction: the cascaded step is BGK on the
    product-form equilibrium (the limit the paper uses for Taylor-Green)."""
    rng = np.random.default_rng(400 + seed)
    w = rng.uniform(0.6, 1.8)
    p = O.Params(nx=3, ny=3, tau_f=1 / w, w2=w, w3=w, w4=w, thermal=0, correction=0)
    fb = random_pops(rng, rho=rng.uniform(0.7, 1.5), spread=0.5)
    rho, ux, uy, T = O.node_macros(p, fb, np.zeros(9))
    fo, _ = O.collide_node(p, fb, np.zeros(9), rho, ux, uy, T, 0.0, 0.0, 0.0, 0.0)
    np.testing.assert_allclose(fo, fb - w * (fb - product_form_feq(rho, ux, uy, RT0)), atol=1e-15)


@pytest.mark.parametrize("seed", rng_seeds)
def test_source_moments(seed):
    """P6: S_a has zero mass, momentum rho a, and zero central moments of order
    >= 2 within the D2Q9 set (third-order terms dropped, Section 3)."""
    rng = np.random.default_rng(500 + seed)
    rho = rng.uniform(0.5, 2.0)
    ax, ay, ux, uy = rng.uniform(-0.1, 0.1, 4)
    S = O.pops_from_moments(rho, O.source_moments(ax, ay, ux, uy))
    assert S.sum() == pytest.approx(0.0, abs=1e-15)
    assert np.sum(S * EX) == pytest.approx(rho * ax, abs=1e-15)
    assert np.sum(S * EY) == pytest.approx(rho * ay, abs=1e-15)
    dx, dy = EX - ux, EY - uy
    for p_, q_ in [(1, 1), (2, 0), (0, 2), (2, 1), (1, 2), (2, 2)]:
        assert np.sum(S * dx ** p_ * dy ** q_) == pytest.approx(0.0, abs=1e-15)


@pytest.mark.parametrize("seed", rng_seeds)
def test_correction_moments(seed):
    """P7: C_a has no mass or momentum; its central trace and normal difference
    are Dx + Dy and Dx - Dy; Pi, M21, M12 central vanish; the fourth central
    moment is -(uy^2 Dx + ux^2 Dy), the O(u^2 D) term the paper neglects."""
    rng = np.random.default_rng(600 + seed)
    rho = rng.uniform(0.5, 2.0)
    Dx, Dy, ux, uy = rng.uniform(-0.05, 0.05, 4)
    C = O.pops_from_moments(rho, O.correction_moments(Dx, Dy, ux, uy))
    assert C.sum() == pytest.approx(0.0, abs=1e-15)
    assert np.sum(C * EX) == pytest.approx(0.0, abs=1e-15)
    assert np.sum(C * EY) == pytest.approx(0.0, abs=1e-15)
    dx, dy = EX - ux, EY - uy
    cm = lambda p_, q_: np.sum(C * dx ** p_ * dy ** q_) / rho
    assert cm(2, 0) + cm(0, 2) == pytest.approx(Dx + Dy, abs=1e-15)
    assert cm(2, 0) - cm(0, 2) == pytest.approx(Dx - Dy, abs=1e-15)
    for pq in [(1, 1), (2, 1), (1, 2)]:
        assert cm(*pq) == pytest.approx(0.0, abs=1e-15)
    assert cm(2, 2) == pytest.approx(-(uy * uy * Dx + ux * ux * Dy), abs=1e-15)


@pytest.mark.parametrize("seed", rng_seeds)
@pytest.mark.parametrize("mode", [0, 1])
def test_heq_moments(seed, mode):
    """P8: h^eq (Section 4) has the six prescribed moments in both forms; its
    total is rho E."""
    rng = np.random.default_rng(700 + seed)
    rho = rng.uniform(0.5, 2.0)
    ux, uy = rng.uniform(-0.15, 0.15, 2)
    RT = RT0 * rng.uniform(0.8, 1.2)
    b = rng.choice([3.0, 4.0, 5.0])
    E = 0.5 * (b * RT + ux * ux + uy * uy)
    h = O.heq(rho, ux, uy, RT, b, mode)
    M = lambda p_, q_: np.sum(h * EX ** p_ * EY ** q_) / rho
    assert M(0, 0) == pytest.approx(E, rel=1e-14)
    assert M(1, 0) == pytest.approx((E + RT) * ux, abs=1e-15)
    assert M(0, 1) == pytest.approx((E + RT) * uy, abs=1e-15)
    assert M(2, 0) == pytest.approx((E + 2 * RT) * ux * ux + RT * (E + RT), rel=1e-14)
    assert M(0, 2) == pytest.approx((E + 2 * RT) * uy * uy + RT * (E + RT), rel=1e-14)
    assert M(1, 1) == pytest.approx((E + 2 * RT) * ux * uy, abs=1e-15)
    if mode == 1:  # the paper's explicit form: higher raw moments zero
        for pq in [(2, 1), (1, 2), (2, 2)]:
            assert M(*pq) == pytest.approx(0.0, abs=1e-15)


def _continuous_energy_central_moment(p_, q_, ux, uy, RT, b, n=40):
    """Central moment of (|xi|^2/2 + (b-2)RT/2) f^M(xi) about u for a unit-density
    2-D Maxwellian at (u, RT), by Gauss-Hermite quadrature (exact for these
    polynomial integrands)."""
    x, w = np.polynomial.hermite_e.hermegauss(n)   # weight exp(-x^2/2)
    w = w / np.sqrt(2 * np.pi)
    s = np.sqrt(RT)
    cx, cy = np.meshgrid(s * x, s * x, indexing="ij")
    W2 = np.outer(w, w)
    xi2 = (cx + ux) ** 2 + (cy + uy) ** 2
    dens = 0.5 * xi2 + 0.5 * (b - 2.0) * RT
    return float(np.sum(W2 * dens * cx ** p_ * cy ** q_))


@pytest.mark.parametrize("seed", rng_seeds)
def test_heq_continuous_form_matches_maxwellian(seed):
    """The default h^eq takes every moment of the nine-moment set, including
    the three the paper leaves free, from the continuous total-energy density of
    a Maxwellian (computed here by quadrature)."""
    rng = np.random.default_rng(750 + seed)
    rho = rng.uniform(0.5, 2.0)
    ux, uy = rng.uniform(-0.15, 0.15, 2)
    RT = RT0 * rng.uniform(0.8, 1.2)
    b = rng.choice([3.0, 4.0, 5.0])
    h = O.heq(rho, ux, uy, RT, b, 0)
    dx, dy = EX - ux, EY - uy
    for p_, q_ in [(0, 0), (1, 0), (0, 1), (2, 0), (0, 2), (1, 1), (2, 1), (1, 2), (2, 2)]:
        got = np.sum(h * dx ** p_ * dy ** q_) / rho
        assert got == pytest.approx(_continuous_energy_central_moment(p_, q_, ux, uy, RT, b), abs=1e-14), (p_, q_)


def _thermal_params(seed):
    rng = np.random.default_rng(seed)
    return rng, O.Params(nx=3, ny=3, tau_f=rng.uniform(0.55, 1.2), w2=rng.uniform(0.5, 1.8),
                         w3=rng.uniform(0.5, 1.8), w4=rng.uniform(0.5, 1.8), gamma=rng.choice([1.4, 5 / 3]),
                         Pr=rng.uniform(0.5, 3.0))


@pytest.mark.parametrize("seed", rng_seeds)
def test_collision_conservation(seed):
    """P9 and the conservation laws of one collision: mass kept, momentum raised
    by rho a (Eq. (20) with the source of Section 3), and sum hbar kept, which
    holds exactly iff sum_a K_a = 0."""
    rng, p = _thermal_params(800 + seed)
    fb = random_pops(rng, rho=rng.uniform(0.7, 1.4), spread=0.5)
    hb = random_pops(rng, rho=rng.uniform(0.7, 1.4), spread=0.5) * 0.8
    ax, ay = rng.uniform(-0.02, 0.02, 2)
    Dx, Dy = rng.uniform(-0.02, 0.02, 2)
    rho, ux, uy, T = O.node_macros(p, fb, hb, ax, ay)
    fo, ho = O.collide_node(p, fb, hb, rho, ux, uy, T, Dx, Dy, ax, ay)
    assert fo.sum() == pytest.approx(rho, rel=1e-14)
    assert np.sum(fo * EX) == pytest.approx(np.sum(fb * EX) + rho * ax, abs=1e-15)
    assert np.sum(fo * EY) == pytest.approx(np.sum(fb * EY) + rho * ay, abs=1e-15)
    assert ho.sum() == pytest.approx(hb.sum(), rel=1e-14)
    # and the energy DF really is coupled (K != 0 pointwise) when Pr != 1
    p1 = O.Params(**{**p.__dict__, "Pr": 1.0, "_keep": []})
    _, ho1 = O.collide_node(p1, fb, hb, rho, ux, uy, T, Dx, Dy, ax, ay)
    assert np.abs(ho - ho1).max() > 1e-6


def test_collision_relaxes_each_central_moment():
    """Eq. (8): with the source and correction switched off, each central moment
    about u after the collision is w*eq + (1 - w)*pre, rate by rate."""
    rng = np.random.default_rng(900)
    w1, w2, w3, w4 = 1.3, 0.7, 1.6, 0.4
    p = O.Params(nx=3, ny=3, tau_f=1 / w1, w2=w2, w3=w3, w4=w4, thermal=0, correction=0)
    fb = random_pops(rng, rho=1.2, spread=0.6)
    rho, ux, uy, T = O.node_macros(p, fb, np.zeros(9))
    fo, _ = O.collide_node(p, fb, np.zeros(9), rho, ux, uy, T, 0, 0, 0, 0)
    _, c0 = moments_np(fb, ux, uy)
    _, c1 = moments_np(fo, ux, uy)
    eq = {3: 2 * RT0, 4: 0.0, 5: 0.0, 6: 0.0, 7: 0.0, 8: RT0 * RT0}
    rate = {3: w2, 4: w1, 5: w1, 6: w3, 7: w3, 8: w4}
    for i in range(3, 9):
        assert c1[i] == pytest.approx(rate[i] * eq[i] + (1 - rate[i]) * c0[i], abs=1e-14), i
