// Host build of the GPU per-node arithmetic (tclbm_node.h) for the node-level
// tests; not part of the library.
#include "../paper_1610_07114_amd/csrc/tclbm_node.h"

using namespace tclbm;

static Consts<double> consts(const double *c) {
  return Consts<double>{c[0], c[1], c[2], c[3], c[4], c[5], c[6], c[7], c[8],
                        (int)c[9], (int)c[10], (int)c[11], (int)c[12], (int)c[13], 2.0 / c[2], 1.0 / (c[0] * c[1]),
                        c[0] * c[1], 0.0};
}

extern "C" {
// ref = {rho_r, theta_r}; f, h absolute populations; out: rho, ux, uy, T
void shim_macros(const double *cst, const double *ref, const double *f, const double *h, double ax, double ay,
                 double *out) {
  Consts<double> c = consts(cst);
  RowRef<double> q = make_ref<double>(ref[0], ref[1], c.b, c.heq_mode);
  double r[9], s[9], d[9], g[9];
  ref_pops(q, c.thermal, c.heq_mode, r, s);
  for (int a = 0; a < 9; ++a) {
    d[a] = f[a] - r[a];
    g[a] = h[a] - s[a];
  }
  Macro<double> m = macros(c, q, d, g, ax, ay);
  out[0] = m.rho;
  out[1] = m.ux;
  out[2] = m.uy;
  out[3] = m.th / c.R_;
}
// P, Q returned as absolute populations (reference added back)
void shim_collide(const double *cst, const double *ref, const double *f, const double *h, double Dx, double Dy,
                  double ax, double ay, double *P, double *Q) {
  Consts<double> c = consts(cst);
  RowRef<double> q = make_ref<double>(ref[0], ref[1], c.b, c.heq_mode);
  double r[9], s[9], d[9], g[9];
  ref_pops(q, c.thermal, c.heq_mode, r, s);
  for (int a = 0; a < 9; ++a) {
    d[a] = f[a] - r[a];
    g[a] = h[a] - s[a];
  }
  Macro<double> m = macros(c, q, d, g, ax, ay);
  collide(c, q, d, g, m, Dx, Dy, ax, ay, P, Q);
  for (int a = 0; a < 9; ++a) {
    P[a] += r[a];
    Q[a] += s[a];
  }
}
// equilibria (absolute) through the deviation forms
void shim_feq(const double *cst, const double *ref, double rho, double ux, double uy, double T, double *f) {
  Consts<double> c = consts(cst);
  RowRef<double> q = make_ref<double>(ref[0], ref[1], c.b, c.heq_mode);
  double r[9], s[9];
  ref_pops(q, c.thermal, c.heq_mode, r, s);
  feq_dev(q, rho - q.rho, ux, uy, c.R_ * T - q.th, f);
  for (int a = 0; a < 9; ++a) f[a] += r[a];
}
void shim_heq(const double *cst, const double *ref, double rho, double ux, double uy, double T, double *h) {
  Consts<double> c = consts(cst);
  RowRef<double> q = make_ref<double>(ref[0], ref[1], c.b, c.heq_mode);
  double r[9], s[9];
  ref_pops(q, c.thermal, c.heq_mode, r, s);
  const double th = c.R_ * T, E = 0.5 * (c.b * th + ux * ux + uy * uy);
  heq_dev(c, q, rho - q.rho, ux, uy, th - q.th, rho * E - q.rho * q.E, h);
  for (int a = 0; a < 9; ++a) h[a] += s[a];
}
}
