// tclbm_node.h -- per-node arithmetic of the thermal cascaded LBM step, written
// for the GPU (also compiled for the host by the node-level tests).
//
// Route: all population <-> moment maps go through central moments about the
// local fluid velocity, factored into three-point transforms along x and then y
// (a D2Q9 population set is a 3x3 array over (e_x, e_y) in {-1,0,1}^2).  The
// relaxation (Eq. (8)), the force source S (Section 3) and the correction C
// (Section 4) are all applied in central-moment space, so one inverse transform
// yields fbar* + S + C directly.  Moments are rho-weighted throughout
// (kappa_pq = sum_a f_a (e_ax - u_x)^p (e_ay - u_y)^q).
//
// Deviation arithmetic: the state is held as d_a = fbar_a - r_a and
// g_a = hbar_a - s_a, where r and s are the rest-state equilibria of the row
// (density rho_r, theta_r = R T_r).  The central moments of r about u are known
// in closed form (r is a product of 1-D factors with moments 1, -u, theta_r +
// u^2), so every quantity below is formed as a difference of small numbers and
// FP32 rounding acts on deviations, not on O(1) populations.  theta = R T.
#pragma once

#if defined(__HIPCC__) || defined(__HIP__)
#include <hip/hip_runtime.h>
#else
// plain host compiler (node-level tests): no HIP qualifiers
#define __host__
#define __device__
#define __forceinline__ inline
#endif

namespace tclbm {

#define TC_HD __host__ __device__ __forceinline__

// Forward three-point transform: populations at e = -1, 0, +1 -> central
// moments of order 0, 1, 2 about u.
template <class R>
TC_HD void fwd3(R m, R z, R p, R u, R &k0, R &k1, R &k2) {
  k0 = m + z + p;
  R d = p - m;
  k1 = d - u * k0;
  k2 = (p + m) - u * (R(2) * d - u * k0);
}

// Inverse three-point transform: central moments (c0, c1, c2) about u ->
// populations at e = -1, 0, +1.
template <class R>
TC_HD void inv3(R c0, R c1, R c2, R u, R &m, R &z, R &p) {
  R r1 = c1 + u * c0;         // first raw moment
  R r2 = c2 + u * (c1 + r1);  // second raw moment
  z = c0 - r2;
  p = R(0.5) * (r2 + r1);
  m = R(0.5) * (r2 - r1);
}

// Central moments k[i][j] (i: x order, j: y order) of a population set.
template <class R>
TC_HD void central9(const R *f, R ux, R uy, R k[3][3]) {
  R am[3], a0[3], ap[3];  // x moments of the e_y = -1, 0, +1 rows
  fwd3(f[7], f[4], f[8], ux, am[0], am[1], am[2]);
  fwd3(f[3], f[0], f[1], ux, a0[0], a0[1], a0[2]);
  fwd3(f[6], f[2], f[5], ux, ap[0], ap[1], ap[2]);
#pragma unroll
  for (int i = 0; i < 3; ++i) fwd3(am[i], a0[i], ap[i], uy, k[i][0], k[i][1], k[i][2]);
}

// Populations from central moments c[i][j] about (ux, uy).
template <class R>
TC_HD void pops9(const R c[3][3], R ux, R uy, R *f) {
  R bm[3], b0[3], bp[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) inv3(c[i][0], c[i][1], c[i][2], uy, bm[i], b0[i], bp[i]);
  inv3(bm[0], bm[1], bm[2], ux, f[7], f[4], f[8]);
  inv3(b0[0], b0[1], b0[2], ux, f[3], f[0], f[1]);
  inv3(bp[0], bp[1], bp[2], ux, f[6], f[2], f[5]);
}

// Rest-state reference of one row: r = rho_r psi(e_x) psi(e_y) with
// psi(0) = 1 - theta_r, psi(+-1) = theta_r/2 (the density equilibrium at rest),
// s = the energy equilibrium at rest; E = b theta_r/2, S2 = theta_r(E + theta_r)
// and S22 its second and fourth raw moments per unit mass.
template <class R>
struct RowRef {
  R rho, th, E, S2, S22;
};

// Rest reference of a row.  heq_mode 0/1: total-energy DF (raw moments E,
// S2 = th (E + th), S22 = th^2 (E + 2 th) or 0); heq_mode 2: internal-energy
// DF, whose rest populations are e times the density ones (S2 = th E,
// S22 = th^2 E).
template <class R>
TC_HD RowRef<R> make_ref(R rho, R th, R b, int heq_mode) {
  RowRef<R> q;
  q.rho = rho;
  q.th = th;
  q.E = R(0.5) * b * th;
  if (heq_mode == 2) {
    q.S2 = th * q.E;
    q.S22 = th * th * q.E;
    return q;
  }
  q.S2 = th * (q.E + th);
  q.S22 = (heq_mode == 1) ? R(0) : th * th * (q.E + R(2) * th);
  return q;
}

// Rest populations of the reference (host tables and tests).
template <class R>
TC_HD void ref_pops(const RowRef<R> &q, int thermal, int heq_mode, R *r, R *s) {
  const R p0 = R(1) - q.th, p1 = R(0.5) * q.th;
  r[0] = q.rho * p0 * p0;
  r[1] = r[2] = r[3] = r[4] = q.rho * p0 * p1;
  r[5] = r[6] = r[7] = r[8] = q.rho * p1 * p1;
  if (!thermal) {
    for (int a = 0; a < 9; ++a) s[a] = R(0);
    return;
  }
  (void)heq_mode;
  // raw moments M00 = E, M20 = M02 = S2, M22 = S22 (odd ones zero) through Eq. (3)
  s[0] = q.rho * (q.E - R(2) * q.S2 + q.S22);
  s[1] = s[2] = s[3] = s[4] = R(0.5) * q.rho * (q.S2 - q.S22);
  s[5] = s[6] = s[7] = s[8] = R(0.25) * q.rho * q.S22;
}

// Central moments about u of the density reference: rho_r m_i(ux) m_j(uy).
template <class R>
TC_HD void ref_central(const RowRef<R> &q, R ux, R uy, R k[3][3]) {
  const R mx[3] = {R(1), -ux, q.th + ux * ux};
  const R my[3] = {R(1), -uy, q.th + uy * uy};
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) k[i][j] = q.rho * mx[i] * my[j];
}

template <class R>
struct Consts {
  R R_, T0, b, w1, w2, w3, w4, wh, inv_tau_hf;
  int thermal, correction, heq_mode, h_coll, h_force;
  R two_b, inv_RT0;  // 2/b and 1/(R T0)
  // R T0 in the compute type and its rounding error, R T0 - RT0f (formed in
  // double): theta - R T0 = ((theta_r - RT0f) + dRT0) + dtheta, where the
  // first difference is exact (both near 1/3)
  R RT0f, dRT0;
};

// 1 - theta/theta0 of a node from its row reference and deviation, without
// rounding the O(1) temperature itself (the correction term's
// u(1 - theta) is a small difference)
template <class R>
TC_HD R one_minus_theta(const Consts<R> &c, R th_ref, R dth) {
  return -(((th_ref - c.RT0f) + c.dRT0) + dth) * c.inv_RT0;
}

// 1/x: IEEE division in FP64; in FP32 on the GPU the hardware reciprocal
// refined by one Newton step (within an ulp or so, no division sequence).
TC_HD double recip(double x) { return 1.0 / x; }
TC_HD float recip(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  float r = __builtin_amdgcn_rcpf(x);
  return r * (2.0f - x * r);
#else
  return 1.0f / x;
#endif
}

// Macroscopic state of a node (Eq. (20), the temperature of Section 4), with
// the deviations from the row reference kept separately.
template <class R>
struct Macro {
  R drho, rho, ux, uy, dth, th;  // th = R T
  R sg;                          // sum of g = rho E - rho_r E_r
};

template <class R>
TC_HD Macro<R> macros(const Consts<R> &c, const RowRef<R> &q, const R *d, const R *g, R ax, R ay) {
  Macro<R> m;
  m.drho = ((d[0] + d[1]) + (d[2] + d[3])) + ((d[4] + d[5]) + (d[6] + d[7])) + d[8];
  m.rho = q.rho + m.drho;
  const R jx = (d[1] - d[3]) + (d[5] - d[6]) + (d[8] - d[7]);
  const R jy = (d[2] - d[4]) + (d[5] - d[7]) + (d[6] - d[8]);
  const R ir = recip(m.rho);
  m.ux = jx * ir + R(0.5) * ax;
  m.uy = jy * ir + R(0.5) * ay;
  if (c.thermal) {
    m.sg = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7])) + g[8];
    // theta - theta_r = (2/b) ((sum g - drho E_r)/rho - u^2/2); the
    // internal-energy DF (heq_mode 2) carries no kinetic part
    if (c.heq_mode == 2)
      m.dth = c.two_b * ((m.sg - m.drho * q.E) * ir);
    else
      m.dth = c.two_b * ((m.sg - m.drho * q.E) * ir - R(0.5) * (m.ux * m.ux + m.uy * m.uy));
  } else {
    m.sg = R(0);
    m.dth = c.R_ * c.T0 - q.th;
  }
  m.th = q.th + m.dth;
  return m;
}

// Deviation of the density equilibrium at (rho, u, th) from the reference r:
// central moments of f^eq about its own u are rho (1, 0, th) x (1, 0, th).
template <class R>
TC_HD void feq_dev(const RowRef<R> &q, R drho, R ux, R uy, R dth, R *out) {
  const R rho = q.rho + drho, th = q.th + dth;
  const R dP = drho * th + q.rho * dth;                   // rho th - rho_r th_r
  const R dP2 = drho * th * th + q.rho * dth * (th + q.th);  // rho th^2 - rho_r th_r^2
  const R rr = q.rho, u2 = ux * ux + uy * uy;
  R c[3][3];
  c[0][0] = drho;
  c[1][0] = rr * ux;
  c[0][1] = rr * uy;
  c[1][1] = -rr * ux * uy;
  c[2][0] = dP - rr * ux * ux;
  c[0][2] = dP - rr * uy * uy;
  c[2][1] = rr * (q.th + ux * ux) * uy;
  c[1][2] = rr * (q.th + uy * uy) * ux;
  c[2][2] = dP2 - rr * (q.th * u2 + ux * ux * uy * uy);
  (void)rho;
  pops9(c, ux, uy, out);
}

// Deviation of the energy equilibrium from the reference s, E = (b th + u^2)/2.
// mode 0: central moments about u of the continuous total-energy density
//   (rho E, rho th u, rho th (E + th) on both axes, rho th^2 u_y, rho th^2 u_x,
//    rho th^2 (E + 2 th)); mode 1: the explicit form of Section 4 (higher raw
//   moments zero).  sg = rho E - rho_r E_r (the deviation of the total energy).
template <class R>
TC_HD void heq_dev(const Consts<R> &c, const RowRef<R> &q, R drho, R ux, R uy, R dth, R sg, R *out) {
  const R rho = q.rho + drho, th = q.th + dth;
  const R rr = q.rho, rE = rr * q.E, rS2 = rr * q.S2;
  const R ux2 = ux * ux, uy2 = uy * uy;
  if (c.heq_mode == 2) {
    // internal-energy DF: g^eq = e f^eq, e = b th/2; against the reference
    // e_r r: e (f^eq - r) + (e - e_r) r
    R fd[9];
    feq_dev(q, drho, ux, uy, dth, fd);
    const R de = R(0.5) * c.b * dth, e = q.E + de;
    const R p0 = R(1) - q.th, p1 = R(0.5) * q.th;
    const R r0 = rr * p0 * p0, r1 = rr * p0 * p1, r5 = rr * p1 * p1;
    out[0] = e * fd[0] + de * r0;
#pragma unroll
    for (int a = 1; a <= 4; ++a) out[a] = e * fd[a] + de * r1;
#pragma unroll
    for (int a = 5; a <= 8; ++a) out[a] = e * fd[a] + de * r5;
    (void)sg;
    (void)rho;
    return;
  }
  if (c.heq_mode == 1) {
    R E = R(0.5) * (c.b * th + ux2 + uy2);
    R A = E + th, B = E + R(2) * th, C = th * A, u2 = ux2 + uy2;
    R hx = R(0.5) * rho, hq = R(0.25) * rho * B * ux * uy;
    R s0 = rr * (q.E - R(2) * q.S2), s1 = R(0.5) * rr * q.S2;
    out[0] = rho * (E - B * u2 - R(2) * C) - s0;
    R sx = B * ux2 + C, sy = B * uy2 + C;
    out[1] = hx * (A * ux + sx) - s1;
    out[3] = hx * (-A * ux + sx) - s1;
    out[2] = hx * (A * uy + sy) - s1;
    out[4] = hx * (-A * uy + sy) - s1;
    out[5] = hq;
    out[6] = -hq;
    out[7] = hq;
    out[8] = -hq;
    return;
  }
  const R dP2 = drho * th * th + rr * dth * (th + q.th);
  const R A = rE * dth + th * sg + dP2;  // rho th (E+th) - rho_r th_r (E_r+th_r)
  const R rth2 = rho * th * th;
  const R B = rE * dth * (th + q.th) + th * th * sg +
              R(2) * (drho * th * th * th + rr * dth * (th * th + th * q.th + q.th * q.th));
  R h[3][3];
  h[0][0] = sg;
  h[1][0] = ux * (rho * th + rE);
  h[0][1] = uy * (rho * th + rE);
  h[1][1] = -ux * uy * rE;
  h[2][0] = A - ux2 * rE;
  h[0][2] = A - uy2 * rE;
  h[2][1] = uy * (rth2 + rS2 + ux2 * rE);
  h[1][2] = ux * (rth2 + rS2 + uy2 * rE);
  h[2][2] = B - (ux2 + uy2) * rS2 - ux2 * uy2 * rE;
  pops9(h, ux, uy, out);
}

// The energy update conserves the total energy sum_a h_a (the relaxation
// keeps the zeroth moment, K and the force source carry none): the rest
// population takes the balance.
template <class R>
TC_HD R energy_balance(R sg, const R *Q) {
  return sg - (((Q[1] + Q[2]) + (Q[3] + Q[4])) + ((Q[5] + Q[6]) + (Q[7] + Q[8])));
}

// One node's collision in deviation form.  Inputs: d, g before collision, the
// node's macroscopic state, Dx = d/dx[u_x(1-theta)], Dy = d/dy[u_y(1-theta)],
// the node acceleration.  Outputs the deviations (from the same row
// reference) of what streams: P = fbar* + S + C (Eq. (27)) and Q = updated hbar.
template <class R, bool kBalance = true>
TC_HD void collide(const Consts<R> &c, const RowRef<R> &q, const R *d, const R *g, const Macro<R> &m, R Dx, R Dy,
                   R ax, R ay, R *P, R *Q) {
  const R rho = m.rho, ux = m.ux, uy = m.uy, th = m.th;
  const R rr = q.rho, ux2 = ux * ux, uy2 = uy * uy, u2 = ux2 + uy2;
  if (!(c.correction && c.thermal)) {
    Dx = R(0);
    Dy = R(0);
  }
  R kd[3][3], kr[3][3];
  central9(d, ux, uy, kd);
  ref_central(q, ux, uy, kr);

  const R dP = m.drho * th + rr * m.dth;                      // rho th - rho_r th_r
  const R dP2 = m.drho * th * th + rr * m.dth * (th + q.th);  // rho th^2 - rho_r th_r^2
  const R rDx = rho * Dx, rDy = rho * Dy;
  const R ccorr = rho * (uy2 * Dx + ux2 * Dy);  // 4th central moment of C is -ccorr

  // Eq. (8) towards the equilibria of the transformed DF (Section 4), written
  // as deviations from the reference's central moments.
  const R dE = kd[2][0] + kd[0][2], dN = kd[2][0] - kd[0][2];
  const R dEs = (R(1) - c.w2) * dE + c.w2 * (R(2) * dP - rr * u2 - R(0.5) * (rDx + rDy));
  const R dNs = (R(1) - c.w1) * dN + c.w1 * (R(0.5) * (rDy - rDx) - rr * (ux2 - uy2));
  R qd[3][3];
  qd[0][0] = m.drho;
  qd[1][0] = R(0.5) * rho * ax + rr * ux;  // (-rho a/2 + rho a) - kr10
  qd[0][1] = R(0.5) * rho * ay + rr * uy;
  qd[1][1] = (R(1) - c.w1) * kd[1][1] - c.w1 * kr[1][1];
  qd[2][0] = R(0.5) * (dEs + dNs) + rDx;  // + C
  qd[0][2] = R(0.5) * (dEs - dNs) + rDy;
  qd[2][1] = (R(1) - c.w3) * kd[2][1] - c.w3 * kr[2][1];
  qd[1][2] = (R(1) - c.w3) * kd[1][2] - c.w3 * kr[1][2];
  qd[2][2] = (R(1) - c.w4) * kd[2][2] + c.w4 * (dP2 - rr * (q.th * u2 + ux2 * uy2)) - ccorr;
  pops9(qd, ux, uy, P);
  // The collision conserves mass and momentum exactly (the force adds rho a):
  // impose both on the computed populations, so that FP32 rounding in the
  // transforms does not accumulate into a drift of the conserved sums.  (With
  // 16-bit storage the unbiased storage rounding is larger by orders of
  // magnitude; the balance is not applied there.)
  if (kBalance) {
    const R jx = rho * ux + R(0.5) * rho * ax, jy = rho * uy + R(0.5) * rho * ay;
    const R dx = jx - ((P[1] - P[3]) + ((P[5] - P[6]) + (P[8] - P[7])));
    const R dy = jy - ((P[2] - P[4]) + ((P[5] - P[7]) + (P[6] - P[8])));
    P[1] += R(0.5) * dx;
    P[3] -= R(0.5) * dx;
    P[2] += R(0.5) * dy;
    P[4] -= R(0.5) * dy;
    P[0] = m.drho - (((P[1] + P[2]) + (P[3] + P[4])) + ((P[5] + P[6]) + (P[7] + P[8])));
  }

  if (!c.thermal) return;

  if (c.heq_mode == 2) {
    // Internal-energy DF: BGK towards e f^eq, plus the force source whose
    // only moment is e rho a (half on each axis link), with the (1 - w_h/2)
    // factor; no coupling source.
    R he[9];
    heq_dev(c, q, m.drho, ux, uy, m.dth, m.sg, he);
    const R ge = R(0.5) * (R(1) - R(0.5) * c.wh) * rho * (R(0.5) * c.b * th);
#pragma unroll
    for (int a = 0; a < 9; ++a) Q[a] = g[a] - c.wh * (g[a] - he[a]);
    Q[1] += ge * ax;
    Q[3] -= ge * ax;
    Q[2] += ge * ay;
    Q[4] -= ge * ay;
    if (kBalance) Q[0] = energy_balance(m.sg, Q);
    return;
  }

  // f - f^eq with f = fbar + S/2 + C/2: central moments, then populations.
  R dd[3][3];
  dd[0][0] = R(0);
  dd[1][0] = R(0);
  dd[0][1] = R(0);
  dd[1][1] = kd[1][1] + kr[1][1];
  dd[2][0] = kd[2][0] + R(0.5) * rDx - dP + rr * ux2;
  dd[0][2] = kd[0][2] + R(0.5) * rDy - dP + rr * uy2;
  dd[2][1] = kd[2][1] + kr[2][1];
  dd[1][2] = kd[1][2] + kr[1][2];
  dd[2][2] = kd[2][2] - R(0.5) * ccorr - (dP2 - rr * (q.th * u2 + ux2 * uy2));
  R dl[9];
  pops9(dd, ux, uy, dl);

  R he[9];  // h^eq - s
  heq_dev(c, q, m.drho, ux, uy, m.dth, m.sg, he);

  // K_a = Z_a/tau_hf (f_a - f_a^eq), Z_a = e_a.u - u^2/2 (Eq. (22))
  const R hu2 = R(0.5) * u2;
  R K[9];
  K[0] = -hu2 * dl[0];
  K[1] = (ux - hu2) * dl[1];
  K[2] = (uy - hu2) * dl[2];
  K[3] = (-ux - hu2) * dl[3];
  K[4] = (-uy - hu2) * dl[4];
  K[5] = (ux + uy - hu2) * dl[5];
  K[6] = (uy - ux - hu2) * dl[6];
  K[7] = (-ux - uy - hu2) * dl[7];
  K[8] = (ux - uy - hu2) * dl[8];
#pragma unroll
  for (int a = 0; a < 9; ++a) K[a] *= c.inv_tau_hf;

  // Body-force source of the energy DF: the force changes the equilibrium
  // energy flux (rho E + p) u by (rho E + p) a per step, which the printed
  // scheme leaves to the Chapman-Enskog flux as a spurious -(1/w_h - 1/2)
  // (rho E + p) a.  Populations: half of each component on the two axis
  // links, entering with the (1 - w_h/2) factor of the transformed scheme.
  const R kk = R(1) - R(0.5) * c.wh;
  R Fx = R(0), Fy = R(0);
  if (c.h_force) {
    const R hf = R(0.5) * kk * rho * ((R(0.5) * c.b + R(1)) * th + hu2);  // th = R T
    Fx = hf * ax;
    Fy = hf * ay;
  }

  if (c.h_coll == 1) {
    // BGK update of the transformed energy DF (Section 4)
#pragma unroll
    for (int a = 0; a < 9; ++a) Q[a] = g[a] - c.wh * (g[a] - he[a]) + kk * K[a];
    Q[1] += Fx;
    Q[3] -= Fx;
    Q[2] += Fy;
    Q[4] -= Fy;
    if (kBalance) Q[0] = energy_balance(m.sg, Q);
    return;
  }
  // Two-rate update: energy-flux moments relax with w_h, all others with 1.
  // In populations: Q = h^eq + K/2 + (1 - w_h)/2 e_a.G on the axis links,
  // G = sum_a (hbar_a - h^eq_a + K_a/2) e_a (the reference has no flux).
  R n[9];
#pragma unroll
  for (int a = 0; a < 9; ++a) n[a] = g[a] - he[a] + R(0.5) * K[a];
  const R Gx = (n[1] - n[3]) + (n[5] - n[6]) + (n[8] - n[7]);
  const R Gy = (n[2] - n[4]) + (n[5] - n[7]) + (n[6] - n[8]);
  const R gg = R(0.5) * (R(1) - c.wh);
#pragma unroll
  for (int a = 0; a < 9; ++a) Q[a] = he[a] + R(0.5) * K[a];
  Q[1] += gg * Gx + Fx;
  Q[3] -= gg * Gx + Fx;
  Q[2] += gg * Gy + Fy;
  Q[4] -= gg * Gy + Fy;
  if (kBalance) Q[0] = energy_balance(m.sg, Q);
}

// Force source S (Section 3) as populations: its only non-zero central moments
// about u are the first ones, rho a.
template <class R>
TC_HD void source9(R rho, R ux, R uy, R ax, R ay, R *S) {
  R c[3][3] = {{R(0), R(0), R(0)}, {R(0), R(0), R(0)}, {R(0), R(0), R(0)}};
  c[1][0] = rho * ax;
  c[0][1] = rho * ay;
  pops9(c, ux, uy, S);
}

#undef TC_HD

}  // namespace tclbm
