// Host build of the GPU per-node arithmetic (tclbm_node.h) for the node-level
// tests; not part of the library.
#include "../paper_1610_07114_amd/csrc/tclbm_node.h"

using namespace tclbm;

extern "C" {
void shim_macros(const double *cst, const double *f, const double *h, double ax, double ay, double *out) {
  Consts<double> c{cst[0], cst[1], cst[2], cst[3], cst[4], cst[5], cst[6], cst[7], cst[8], cst[9],
                   (int)cst[10], (int)cst[11], (int)cst[12], (int)cst[13]};
  Macro<double> m = macros(c, f, h, ax, ay);
  out[0] = m.rho; out[1] = m.ux; out[2] = m.uy; out[3] = m.T;
}
void shim_collide(const double *cst, const double *f, const double *h, const double *mac, double Dx, double Dy,
                  double ax, double ay, double *P, double *Q) {
  Consts<double> c{cst[0], cst[1], cst[2], cst[3], cst[4], cst[5], cst[6], cst[7], cst[8], cst[9],
                   (int)cst[10], (int)cst[11], (int)cst[12], (int)cst[13]};
  Macro<double> m{mac[0], mac[1], mac[2], mac[3]};
  collide(c, f, h, m, Dx, Dy, ax, ay, P, Q);
}
void shim_feq(double rho, double ux, double uy, double RT, double *f) { feq9(rho, ux, uy, RT, f); }
void shim_heq(double rho, double ux, double uy, double RT, double b, int mode, double *h) {
  heq9(rho, ux, uy, RT, b, mode, h);
}
void shim_source(double rho, double ux, double uy, double ax, double ay, double *S) {
  source9(rho, ux, uy, ax, ay, S);
}
}
