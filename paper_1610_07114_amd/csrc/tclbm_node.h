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
  R r1 = c1 + u * c0;           // first raw moment
  R r2 = c2 + u * (c1 + r1);    // second raw moment
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

// Cascaded equilibrium of the density DF in product form:
// f_a = rho psi(e_ax, ux) psi(e_ay, uy), psi(0,u) = 1 - RT - u^2,
// psi(+-1,u) = (RT + u^2 +- u)/2 (Eq. (7) with the local T, through Eq. (9)).
template <class R>
TC_HD void feq9(R rho, R ux, R uy, R RT, R *f) {
  R x0 = R(1) - RT - ux * ux, xs = R(0.5) * (RT + ux * ux);
  R xp = xs + R(0.5) * ux, xm = xs - R(0.5) * ux;
  R y0 = R(1) - RT - uy * uy, ys = R(0.5) * (RT + uy * uy);
  R yp = rho * (ys + R(0.5) * uy), ym = rho * (ys - R(0.5) * uy);
  y0 *= rho;
  f[0] = x0 * y0;
  f[1] = xp * y0;
  f[2] = x0 * yp;
  f[3] = xm * y0;
  f[4] = x0 * ym;
  f[5] = xp * yp;
  f[6] = xm * yp;
  f[7] = xm * ym;
  f[8] = xp * ym;
}

// Equilibrium of the total-energy DF, E = (b RT + u^2)/2.
// mode 0: central moments about u of the continuous total-energy density
//   (rho E, rho RT u, rho RT(E+RT) on both axes, rho u_y RT^2, rho u_x RT^2,
//    rho RT^2 (E + 2RT)); mode 1: the explicit form of Section 4 (higher raw
//   moments zero).
template <class R>
TC_HD void heq9(R rho, R ux, R uy, R RT, R b, int mode, R *h) {
  R u2 = ux * ux + uy * uy;
  R E = R(0.5) * (b * RT + u2);
  if (mode == 1) {
    R A = E + RT, B = E + R(2) * RT, C = RT * A;
    R hx = R(0.5) * rho, hq = R(0.25) * rho * B * ux * uy;
    h[0] = rho * (E - B * u2 - R(2) * C);
    R sx = B * ux * ux + C, sy = B * uy * uy + C;
    h[1] = hx * (A * ux + sx);
    h[3] = hx * (-A * ux + sx);
    h[2] = hx * (A * uy + sy);
    h[4] = hx * (-A * uy + sy);
    h[5] = hq;
    h[6] = -hq;
    h[7] = hq;
    h[8] = -hq;
    return;
  }
  R rRT = rho * RT;
  R c[3][3];
  c[0][0] = rho * E;
  c[1][0] = rRT * ux;
  c[0][1] = rRT * uy;
  c[2][0] = rRT * (E + RT);
  c[0][2] = c[2][0];
  c[1][1] = R(0);
  c[2][1] = rRT * RT * uy;
  c[1][2] = rRT * RT * ux;
  c[2][2] = rRT * RT * (E + R(2) * RT);
  pops9(c, ux, uy, h);
}

template <class R>
struct Consts {
  R R_, T0, b, w1, w2, w3, w4, wh, inv_tau_hf, inv_bR2;
  int thermal, correction, heq_mode, h_coll;
};

template <class R>
struct Macro {
  R rho, ux, uy, T;
};

// Eq. (20) and the temperature of Section 4 from the transformed DFs.
template <class R>
TC_HD Macro<R> macros(const Consts<R> &c, const R *f, const R *h, R ax, R ay) {
  Macro<R> m;
  R rho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
  R jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
  R jy = (f[2] - f[4]) + (f[5] - f[7]) + (f[6] - f[8]);
  R ir = R(1) / rho;
  m.rho = rho;
  m.ux = jx * ir + R(0.5) * ax;
  m.uy = jy * ir + R(0.5) * ay;
  if (c.thermal) {
    R hs = ((h[0] + h[1]) + (h[2] + h[3])) + ((h[4] + h[5]) + (h[6] + h[7])) + h[8];
    m.T = c.inv_bR2 * (hs * ir - R(0.5) * (m.ux * m.ux + m.uy * m.uy));
  } else {
    m.T = c.T0;
  }
  return m;
}

// One node's collision.  Inputs: transformed DFs fbar, hbar before collision,
// their macroscopic values, Dx = d/dx[u_x(1-theta)], Dy = d/dy[u_y(1-theta)]
// and the node acceleration.  Outputs what streams: P = fbar* + S + C
// (Eq. (27)) and Q = the updated hbar.
template <class R>
TC_HD void collide(const Consts<R> &c, const R *f, const R *h, const Macro<R> &m, R Dx, R Dy, R ax, R ay,
                   R *P, R *Q) {
  const R rho = m.rho, ux = m.ux, uy = m.uy;
  const R RT = c.R_ * m.T;
  if (!(c.correction && c.thermal)) {
    Dx = R(0);
    Dy = R(0);
  }
  R k[3][3];
  central9(f, ux, uy, k);

  // Eq. (8) on the trace / normal difference / off-diagonal / 3rd / 4th order
  // central moments, towards the equilibria of the transformed DF (Section 4).
  const R Et = k[2][0] + k[0][2], Nt = k[2][0] - k[0][2];
  const R rDx = rho * Dx, rDy = rho * Dy;
  const R Es = (R(1) - c.w2) * Et + c.w2 * (R(2) * rho * RT - R(0.5) * (rDx + rDy));
  const R Ns = (R(1) - c.w1) * Nt + c.w1 * (R(0.5) * (rDy - rDx));
  const R ccorr = rho * (uy * uy * Dx + ux * ux * Dy);  // 4th central moment of C is -ccorr
  R q[3][3];
  q[0][0] = rho;
  q[1][0] = R(0.5) * rho * ax;  // -rho a/2 (fbar*) + rho a (S)
  q[0][1] = R(0.5) * rho * ay;
  q[1][1] = (R(1) - c.w1) * k[1][1];
  q[2][0] = R(0.5) * (Es + Ns) + rDx;  // + C
  q[0][2] = R(0.5) * (Es - Ns) + rDy;
  q[2][1] = (R(1) - c.w3) * k[2][1];
  q[1][2] = (R(1) - c.w3) * k[1][2];
  q[2][2] = (R(1) - c.w4) * k[2][2] + c.w4 * rho * RT * RT - ccorr;
  pops9(q, ux, uy, P);

  if (!c.thermal) return;

  // f - f^eq with f = fbar + S/2 + C/2: central moments, then populations.
  R d[3][3];
  d[0][0] = R(0);
  d[1][0] = R(0);
  d[0][1] = R(0);
  d[1][1] = k[1][1];
  d[2][0] = k[2][0] + R(0.5) * rDx - rho * RT;
  d[0][2] = k[0][2] + R(0.5) * rDy - rho * RT;
  d[2][1] = k[2][1];
  d[1][2] = k[1][2];
  d[2][2] = k[2][2] - R(0.5) * ccorr - rho * RT * RT;
  R dl[9];
  pops9(d, ux, uy, dl);

  R he[9];
  heq9(rho, ux, uy, RT, c.b, c.heq_mode, he);

  // K_a = Z_a/tau_hf (f_a - f_a^eq), Z_a = e_a.u - u^2/2 (Eq. (22))
  const R hu2 = R(0.5) * (ux * ux + uy * uy);
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

  if (c.h_coll == 1) {
    // BGK update of the transformed energy DF (Section 4)
    const R kk = R(1) - R(0.5) * c.wh;
#pragma unroll
    for (int a = 0; a < 9; ++a) Q[a] = h[a] - c.wh * (h[a] - he[a]) + kk * K[a];
    return;
  }
  // Two-rate update: energy-flux moments relax with w_h, all others with 1.
  // In populations: Q = h^eq + K/2 + (1 - w_h)/2 e_a.G on the axis links,
  // G = sum_a (hbar_a - h^eq_a + K_a/2) e_a.
  R n[9];
#pragma unroll
  for (int a = 0; a < 9; ++a) n[a] = h[a] - he[a] + R(0.5) * K[a];
  const R Gx = (n[1] - n[3]) + (n[5] - n[6]) + (n[8] - n[7]);
  const R Gy = (n[2] - n[4]) + (n[5] - n[7]) + (n[6] - n[8]);
  const R g = R(0.5) * (R(1) - c.wh);
#pragma unroll
  for (int a = 0; a < 9; ++a) Q[a] = he[a] + R(0.5) * K[a];
  Q[1] += g * Gx;
  Q[3] -= g * Gx;
  Q[2] += g * Gy;
  Q[4] -= g * Gy;
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
