/*
 * tclbm_oracle.c -- plain, slow, FP64 CPU reference of the thermal cascaded
 * lattice Boltzmann method (TCLBM) of Fei & Luo, "Thermal cascaded lattice
 * Boltzmann method" (arXiv:1610.07114).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file; only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or helper with the HIP
 * implementation.
 *
 * It follows the paper's steps in the paper's order and notation:
 *   - central moments are computed by their definition, Eq. (4), as explicit
 *     sums over the nine populations (never by a binomial shortcut);
 *   - post-collision raw moments come from Eq. (18) (Eq. (9) for equilibria);
 *   - every population set (f*, S, C, f^eq) is built through Eq. (3);
 *   - the energy DF uses the explicit h^eq of Section 4 and the BGK update with
 *     the coupling source K.
 *
 * Readings where the paper is silent or ambiguous (each is listed, with its
 * justification, in the design notes of the repository):
 *   units      R = 1/3 and T0 = 1 are expected, so that R*T0 = c_s^2 and
 *              theta = T/T0 (Section 4's third-moment deviation needs it);
 *   gradients  d/dx[u_x(1-theta)], d/dy[u_y(1-theta)] at the collision's time
 *              level, second-order central differences (Section 4), periodic
 *              wrap, and one-sided second-order differences on non-periodic
 *              edges; rho multiplies the Eq. (3) form of C_a, outside the
 *              derivatives;
 *   tau_hf     1/tau_hf = w1 (Pr - 1), i.e. tau_hf = (mu/p + 1/2)/(Pr - 1) with
 *              mu/p = 1/w1 - 1/2 (Eq. (29));
 *   K_a        uses f_a = fbar_a + S_a/2 + C_a/2 and the cascaded equilibrium
 *              f^eq at the local (rho, u, T);
 *   walls      node walls imposed by non-equilibrium extrapolation of both DFs
 *              from the adjacent interior node, applied before the collision;
 *              halfway, resting bounce-back on BOUNCEBACK sides;
 *   init       fbar = f^eq - S/2 and hbar = h^eq from given (rho, u, T);
 *   wall rho   the density of a wall node is fixed by the populations that
 *              reached it after streaming, rho_w = (k0 + 2 kin)/(1 + u_n - a_n/2)
 *              (k0: rest and tangential, kin: arrived from the fluid, u_n, a_n
 *              outward-normal wall velocity and acceleration), the mass balance
 *              of the non-equilibrium bounce-back scheme the paper cites; the
 *              literal rho_w = rho_f and a pressure extrapolation are options;
 *   h^eq       the moments the paper leaves free take their continuous
 *              (Maxwellian) values (the paper's zero choice kept as an option);
 *   h update   two-rate form of the transformed BGK update: energy-flux moments
 *              at w_h, the other moments at rate 1 (BGK kept as an option);
 *   h force    the energy DF receives the change that the body force makes to
 *              its equilibrium energy flux (rho E + p) u within a step: a source
 *              with first moment (rho E + p) a and no other moment (Section 4
 *              prints no force term for the energy DF; without one the
 *              Chapman-Enskog energy flux carries -(1/w_h - 1/2)(rho E + p) a,
 *              which heats the top of a resting isothermal column; the printed
 *              form is kept as an option); no work term rho u.a is added to
 *              the total energy, as in Section 4;
 *   wall NEQ   the stored f is the transformed fbar, so the equilibrium part
 *              used in the extrapolation is f^eq - S/2 at each node;
 *   adiabatic  the fixed lower plate of the Couette test of Section 5B: a node
 *              wall whose temperature makes the one-sided second-order normal
 *              derivative vanish, T_w = (4 T_1 - T_2)/3 from the two nodes
 *              inside, extrapolated like any other wall (T_w = T_1 leaks the
 *              viscous heat of the first cell: 3% low bottom temperature at
 *              H = 39);
 *   mu(T)      mu = mu0 T/T0 of Section 5B enters through Eq. (29) at each node,
 *              1/w1 = mu/p + 1/2 = mu0/(rho R T0) + 1/2, and w_h, tau_hf follow
 *              from that w1 at constant Pr as everywhere else;
 *   e-DF       Section 5D's internal-energy DF, which the paper cites without
 *              stating: g^eq = e f^eq, BGK at w_h, a force source with first
 *              moment e rho a (orc_geq).
 *
 * Build:  gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------------------
 * D2Q9 lattice, Section 2: e_0 = 0; e_1..4 = E, N, W, S; e_5..8 = NE, NW, SW, SE.
 * ------------------------------------------------------------------------- */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

/* Order of the nine-moment set used with Eq. (3):
 * M00, M10, M01, E = M20 + M02, N = M20 - M02, Pi = M11, M21, M12, M22 (Eq. (2)). */
enum { I00 = 0, I10, I01, IE, IN, IPI, I21, I12, I22 };

/* Boundary kinds (one per side). */
enum { ORC_PERIODIC = 0, ORC_BOUNCEBACK = 1, ORC_WALL = 2, ORC_WALL_ADIABATIC = 3 };

static int is_wall(int kind) { return kind == ORC_WALL || kind == ORC_WALL_ADIABATIC; }
enum { ORC_XLO = 0, ORC_XHI = 1, ORC_YLO = 2, ORC_YHI = 3 };

typedef struct {
  int32_t nx, ny;
  double R, T0;      /* lattice gas constant and reference temperature */
  double gamma, Pr;  /* specific-heat ratio, Prandtl number */
  double tau_f;      /* 1/w1 */
  double w2, w3, w4; /* bulk, third- and fourth-order relaxation rates */
  double ax, ay;     /* uniform body acceleration (F = rho a) */
  int32_t thermal;   /* 1: TCLBM; 0: athermal CLBM of Sections 2-3 (T == T0) */
  int32_t correction;/* 1: include the correction term C_a of Section 4 */
  int32_t bc[4];     /* ORC_* per side, indexed by ORC_XLO.. */
  double wall_ux[4], wall_uy[4], wall_T[4];
  int32_t wall_rho;  /* density of a wall node: 0 from the populations that reached
                      * it (k0 + 2 kin, force-corrected), 1 rho_f, 2 from the
                      * pressure of the fluid neighbour plus the static step */
  int32_t heq_moments; /* unprescribed moments of h^eq: 0 continuous values, 1 raw zero */
  int32_t h_collision; /* energy DF collision: 0 two-rate, 1 BGK */
  const double *ax_field; /* optional per-node acceleration (nullable) */
  const double *ay_field;
  int32_t h_force;     /* energy DF body-force source: 1 the flux term (default),
                        * 0 none (Section 4 as printed) */
  int32_t viscosity_mode; /* 0: w1 = 1/tau_f; 1: mu = mu0 T/T0 (Section 5B) */
  double mu0;
  int32_t energy_df;   /* 0: total-energy DF (Section 4); 1: internal-energy DF
                        * (Section 5D's Rayleigh-Benard runs), see orc_geq */
} orc_params;

static double pw(double v, int n) {
  double r = 1.0;
  for (int i = 0; i < n; ++i) r *= v;
  return r;
}

/* Eq. (3): populations from the nine raw moments (per unit mass) times rho. */
void orc_pops_from_moments(double rho, const double m[9], double f[9]) {
  f[0] = rho * (m[I00] - m[IE] + m[I22]);
  f[1] = 0.5 * rho * (m[I10] + 0.5 * (m[IE] + m[IN]) - m[I12] - m[I22]);
  f[2] = 0.5 * rho * (m[I01] + 0.5 * (m[IE] - m[IN]) - m[I21] - m[I22]);
  f[3] = 0.5 * rho * (-m[I10] + 0.5 * (m[IE] + m[IN]) + m[I12] - m[I22]);
  f[4] = 0.5 * rho * (-m[I01] + 0.5 * (m[IE] - m[IN]) + m[I21] - m[I22]);
  f[5] = 0.25 * rho * (m[IPI] + m[I21] + m[I12] + m[I22]);
  f[6] = 0.25 * rho * (-m[IPI] + m[I21] - m[I12] + m[I22]);
  f[7] = 0.25 * rho * (m[IPI] - m[I21] - m[I12] + m[I22]);
  f[8] = 0.25 * rho * (-m[IPI] - m[I21] + m[I12] + m[I22]);
}

/* Moments about a shifted origin (cx, cy), per unit mass:
 * rho*M_pq = sum_a f_a (e_ax - cx)^p (e_ay - cy)^q.  With (cx, cy) = 0 this is
 * Eq. (1); with the local velocity it is the central-moment definition Eq. (4).
 * Returned in the nine-moment order (E, N, Pi recombined as in Eq. (2)). */
static void moments_about(const double f[9], double cx, double cy, double *rho_out, double m[9]) {
  double M[3][3];
  for (int p = 0; p < 3; ++p)
    for (int q = 0; q < 3; ++q) {
      double s = 0.0;
      for (int a = 0; a < 9; ++a) s += f[a] * pw(EX[a] - cx, p) * pw(EY[a] - cy, q);
      M[p][q] = s;
    }
  double rho = M[0][0];
  m[I00] = 1.0;
  m[I10] = M[1][0] / rho;
  m[I01] = M[0][1] / rho;
  m[IE] = (M[2][0] + M[0][2]) / rho;
  m[IN] = (M[2][0] - M[0][2]) / rho;
  m[IPI] = M[1][1] / rho;
  m[I21] = M[2][1] / rho;
  m[I12] = M[1][2] / rho;
  m[I22] = M[2][2] / rho;
  if (rho_out) *rho_out = rho;
}

/* Eq. (1)-(2): raw moments of a population set. */
void orc_raw_moments(const double f[9], double *rho, double m[9]) { moments_about(f, 0.0, 0.0, rho, m); }

/* Eq. (4): central moments about (ux, uy), by definition. */
void orc_central_moments(const double f[9], double ux, double uy, double *rho, double m[9]) {
  moments_about(f, ux, uy, rho, m);
}

/* Eq. (9): raw moments from central moments with M00 = 1, M10 = ux, M01 = uy. */
void orc_raw_from_central(const double c[9], double ux, double uy, double r[9]) {
  double u2 = ux * ux + uy * uy;
  r[I00] = 1.0;
  r[I10] = ux;
  r[I01] = uy;
  r[IPI] = c[IPI] + ux * uy;
  r[IN] = c[IN] + ux * ux - uy * uy;
  r[IE] = c[IE] + u2;
  r[I21] = c[I21] + 2.0 * ux * r[IPI] + 0.5 * uy * (r[IE] + r[IN]) - 2.0 * ux * ux * uy;
  r[I12] = c[I12] + 2.0 * uy * r[IPI] + 0.5 * ux * (r[IE] - r[IN]) - 2.0 * uy * uy * ux;
  r[I22] = c[I22] + 2.0 * ux * r[I12] + 2.0 * uy * r[I21] - 0.5 * u2 * r[IE] +
           0.5 * (ux * ux - uy * uy) * r[IN] - 4.0 * ux * uy * r[IPI] + 3.0 * ux * ux * uy * uy;
}

/* Eq. (18): post-collision raw moments of the transformed DF fbar, whose
 * conserved moments are Mbar00 = 1, Mbar10 = ux - ax/2, Mbar01 = uy - ay/2
 * (Section 3), from its post-collision central moments about u. */
void orc_post_collision_raw(const double c[9], double ux, double uy, double ax, double ay, double r[9]) {
  double u2 = ux * ux + uy * uy;
  r[I00] = 1.0;
  r[I10] = ux - 0.5 * ax;
  r[I01] = uy - 0.5 * ay;
  r[IPI] = c[IPI] + ux * uy - 0.5 * (ax * uy + ay * ux);
  r[IN] = c[IN] + ux * ux - uy * uy - (ax * ux - ay * uy);
  r[IE] = c[IE] + u2 - (ax * ux + ay * uy);
  r[I21] = c[I21] + 2.0 * ux * r[IPI] + 0.5 * uy * (r[IE] + r[IN]) - 2.0 * ux * ux * uy +
           0.5 * ay * ux * ux + ax * ux * uy;
  r[I12] = c[I12] + 2.0 * uy * r[IPI] + 0.5 * ux * (r[IE] - r[IN]) - 2.0 * uy * uy * ux +
           0.5 * ax * uy * uy + ay * ux * uy;
  r[I22] = c[I22] + 2.0 * ux * r[I12] + 2.0 * uy * r[I21] - 0.5 * u2 * r[IE] +
           0.5 * (ux * ux - uy * uy) * r[IN] - 4.0 * ux * uy * r[IPI] + 3.0 * ux * ux * uy * uy -
           ax * ux * uy * uy - ay * uy * ux * ux;
}

/* Section 3: raw moments of the force source S_a (third-order central moments
 * of S dropped, as the paper does). */
void orc_source_moments(double ax, double ay, double ux, double uy, double s[9]) {
  s[I00] = 0.0;
  s[I10] = ax;
  s[I01] = ay;
  s[IE] = 2.0 * (ax * ux + ay * uy);
  s[IN] = 2.0 * (ax * ux - ay * uy);
  s[IPI] = ax * uy + ay * ux;
  s[I21] = ay * ux * ux + 2.0 * ax * ux * uy;
  s[I12] = ax * uy * uy + 2.0 * ay * ux * uy;
  s[I22] = 2.0 * ax * ux * uy * uy + 2.0 * ay * uy * ux * ux;
}

/* Section 4: raw moments of the correction term C_a, with
 * Dx = d/dx[u_x (1 - theta)], Dy = d/dy[u_y (1 - theta)]. */
void orc_correction_moments(double Dx, double Dy, double ux, double uy, double c[9]) {
  c[I00] = 0.0;
  c[I10] = 0.0;
  c[I01] = 0.0;
  c[IPI] = 0.0;
  c[IE] = Dx + Dy;
  c[IN] = Dx - Dy;
  c[I21] = uy * Dx;
  c[I12] = ux * Dy;
  c[I22] = 0.0;
}

/* Eq. (7) with T0 replaced by the local T (Section 4), then Eq. (9), then Eq. (3):
 * the discrete equilibrium of the density DF. */
void orc_feq(double rho, double ux, double uy, double RT, double feq[9]) {
  double c[9] = {0};
  c[I00] = 1.0;
  c[IPI] = 0.0;
  c[IN] = 0.0;
  c[I21] = 0.0;
  c[I12] = 0.0;
  c[IE] = 2.0 * RT;
  c[I22] = RT * RT;
  double r[9];
  orc_raw_from_central(c, ux, uy, r);
  orc_pops_from_moments(rho, r, feq);
}

/* Raw moments (per unit mass) from central moments about (ux, uy) with arbitrary
 * lower-order central moments c00, c10, c01: the binomial theorem written out for
 * the nine-moment set, (e - u + u)^p. */
static void raw_from_central_general(const double C[3][3], double ux, double uy, double M[3][3]) {
  M[0][0] = C[0][0];
  M[1][0] = C[1][0] + ux * C[0][0];
  M[0][1] = C[0][1] + uy * C[0][0];
  M[2][0] = C[2][0] + 2.0 * ux * C[1][0] + ux * ux * C[0][0];
  M[0][2] = C[0][2] + 2.0 * uy * C[0][1] + uy * uy * C[0][0];
  M[1][1] = C[1][1] + ux * C[0][1] + uy * C[1][0] + ux * uy * C[0][0];
  M[2][1] = C[2][1] + 2.0 * ux * C[1][1] + uy * C[2][0] + ux * ux * C[0][1] + 2.0 * ux * uy * C[1][0] +
            ux * ux * uy * C[0][0];
  M[1][2] = C[1][2] + 2.0 * uy * C[1][1] + ux * C[0][2] + uy * uy * C[1][0] + 2.0 * ux * uy * C[0][1] +
            ux * uy * uy * C[0][0];
  M[2][2] = C[2][2] + 2.0 * uy * C[2][1] + 2.0 * ux * C[1][2] + uy * uy * C[2][0] + ux * ux * C[0][2] +
            4.0 * ux * uy * C[1][1] + 2.0 * ux * uy * uy * C[1][0] + 2.0 * ux * ux * uy * C[0][1] +
            ux * ux * uy * uy * C[0][0];
}

static void set_from_pq(const double M[3][3], double m[9]) {
  m[I00] = M[0][0];
  m[I10] = M[1][0];
  m[I01] = M[0][1];
  m[IE] = M[2][0] + M[0][2];
  m[IN] = M[2][0] - M[0][2];
  m[IPI] = M[1][1];
  m[I21] = M[2][1];
  m[I12] = M[1][2];
  m[I22] = M[2][2];
}

/* Section 4: equilibrium of the total-energy DF, with E = (b R T + u^2)/2 the
 * total energy per unit mass.
 *
 * mode 1 (the paper's explicit form): the six prescribed moments, the higher
 * raw moments M21 = M12 = M22 = 0.
 * mode 0 (default): the same six prescribed moments; the three moments the paper
 * leaves free are given their continuous values, the central moments of the
 * total-energy density (xi^2/2 + internal energy) f^M of a Maxwellian at (u, T):
 * C21 = uy (RT)^2, C12 = ux (RT)^2, C22 = (RT)^2 (E + 2RT) -- the same principle
 * the paper applies to the density DF in Eq. (5).  The paper's zero choice gives
 * an energy DF whose checkerboard modes grow on any 2-D lattice. */
void orc_heq_mode(double rho, double ux, double uy, double RT, double b, int mode, double heq[9]) {
  double u2 = ux * ux + uy * uy;
  double E = 0.5 * (b * RT + u2);
  if (mode == 1) {
    heq[0] = rho * (E - (E + 2.0 * RT) * u2 - 2.0 * RT * (E + RT));
    for (int a = 1; a <= 4; ++a) {
      double eu = EX[a] * ux + EY[a] * uy;
      double sq = EX[a] * EX[a] * ux * ux + EY[a] * EY[a] * uy * uy;
      heq[a] = 0.5 * rho * ((E + RT) * eu + (E + 2.0 * RT) * sq + RT * (E + RT));
    }
    for (int a = 5; a <= 8; ++a) heq[a] = 0.25 * rho * ((E + 2.0 * RT) * EX[a] * EY[a] * ux * uy);
    return;
  }
  double C[3][3], M[3][3], m[9];
  C[0][0] = E;
  C[1][0] = RT * ux;
  C[0][1] = RT * uy;
  C[2][0] = RT * (E + RT);
  C[0][2] = RT * (E + RT);
  C[1][1] = 0.0;
  C[2][1] = uy * RT * RT;
  C[1][2] = ux * RT * RT;
  C[2][2] = RT * RT * (E + 2.0 * RT);
  raw_from_central_general(C, ux, uy, M);
  set_from_pq(M, m);
  orc_pops_from_moments(rho, m, heq);
}

void orc_heq(double rho, double ux, double uy, double RT, double b, double heq[9]) {
  orc_heq_mode(rho, ux, uy, RT, b, 1, heq);
}

/* Section 5D runs Rayleigh-Benard convection with an internal-energy DF in
 * place of the total-energy one, so that no viscous heating enters; the paper
 * cites the model without stating it.  Reading: the DF g carries rho e, with
 * e = b R T/2 the internal energy per unit mass, and its equilibrium is the
 * density equilibrium scaled by e, g^eq_a = e f^eq_a (moments rho e, rho e u,
 * e (p I + rho u u)).  A Chapman-Enskog expansion of the BGK update
 * g* = g - w_h (g - g^eq) + (1 - w_h/2) G then gives
 *   d(rho e)/dt + div(rho e u) = div(p (1/w_h - 1/2) grad e),
 * i.e. rho c_v DT/Dt = div(kappa grad T) with thermal diffusivity
 * R T (1/w_h - 1/2) = nu/Pr at the same w_h as the total-energy DF: no
 * viscous dissipation and no pressure work.  Without a source the expansion
 * leaves a spurious flux -(1/w_h - 1/2) e rho a under a body force (the force
 * changes the equilibrium flux rho e u within a step); G, with first moment
 * e rho a on the axis links and no other moment, supplies that change. */
void orc_geq(double rho, double ux, double uy, double RT, double b, double geq[9]) {
  double feq[9];
  orc_feq(rho, ux, uy, RT, feq);
  double e = 0.5 * b * RT;
  for (int a = 0; a < 9; ++a) geq[a] = e * feq[a];
}

/* Derived relaxation constants. */
typedef struct {
  double b, RT0, w1, wh, inv_tau_hf;
} orc_derived;

static orc_derived derive(const orc_params *p) {
  orc_derived d;
  d.b = 2.0 / (p->gamma - 1.0);          /* gamma = (b + 2)/b, Section 5 */
  d.RT0 = p->R * p->T0;
  d.w1 = 1.0 / p->tau_f;
  /* 1/w_h = 2 lambda/(p R (b+2)) + 1/2 with Pr = mu c_p/lambda,
   * c_p = (b+2)R/2 and mu = p(1/w1 - 1/2) (Eq. (29)). */
  d.wh = 1.0 / ((1.0 / d.w1 - 0.5) / p->Pr + 0.5);
  /* tau_hf = (mu/p + 1/2)/(Pr - 1) = (1/w1)/(Pr - 1). */
  d.inv_tau_hf = d.w1 * (p->Pr - 1.0);
  return d;
}

/* The rates at a node of density rho.  Under mu = mu0 T/T0 (Section 5B),
 * Eq. (29) with p = rho R T gives mu/p = mu0/(rho R T0): w1 depends on rho
 * alone; w_h and tau_hf follow from it as in derive(). */
static orc_derived derive_node(const orc_params *p, double rho) {
  orc_derived d = derive(p);
  if (p->viscosity_mode != 1) return d;
  double mu_p = p->mu0 / (rho * p->R * p->T0);
  d.w1 = 1.0 / (mu_p + 0.5);
  d.wh = 1.0 / (mu_p / p->Pr + 0.5);
  d.inv_tau_hf = d.w1 * (p->Pr - 1.0);
  return d;
}

static double node_ax(const orc_params *p, long i) { return p->ax_field ? p->ax_field[i] : p->ax; }
static double node_ay(const orc_params *p, long i) { return p->ay_field ? p->ay_field[i] : p->ay; }

/* Eq. (20) and the temperature of Section 4:
 * rho = sum fbar, rho u = sum fbar e + F/2 (F = rho a),
 * T = 2/(b R) (sum hbar / rho - u^2/2);
 * with the internal-energy DF (orc_geq) T = 2/(b R) sum g / rho. */
void orc_node_macros(const orc_params *p, const double fb[9], const double hb[9], double ax, double ay,
                     double *rho, double *ux, double *uy, double *T) {
  orc_derived d = derive(p);
  double r = 0.0, jx = 0.0, jy = 0.0;
  for (int a = 0; a < 9; ++a) {
    r += fb[a];
    jx += fb[a] * EX[a];
    jy += fb[a] * EY[a];
  }
  double vx = jx / r + 0.5 * ax;
  double vy = jy / r + 0.5 * ay;
  double t = p->T0;
  if (p->thermal) {
    double hs = 0.0;
    for (int a = 0; a < 9; ++a) hs += hb[a];
    if (p->energy_df == 1)
      t = 2.0 / (d.b * p->R) * (hs / r);
    else
      t = 2.0 / (d.b * p->R) * (hs / r - 0.5 * (vx * vx + vy * vy));
  }
  *rho = r;
  *ux = vx;
  *uy = vy;
  *T = t;
}

/* One node's collision: cascaded relaxation of fbar with force and correction
 * sources (Sections 2-4, Eq. (8), Eq. (18), Eq. (27)) and the BGK update of hbar
 * with the coupling source K (Section 4).  Outputs the post-collision values
 * that stream: fout = fbar* + S + C, hout = hbar - w_h(hbar - h^eq) + (1 - w_h/2) K. */
void orc_collide_node(const orc_params *p, const double fb[9], const double hb[9], double rho, double ux,
                      double uy, double T, double Dx, double Dy, double ax, double ay, double fout[9],
                      double hout[9]) {
  orc_derived d = derive_node(p, rho);
  double RT = p->R * T;
  if (!p->correction || !p->thermal) {
    Dx = 0.0;
    Dy = 0.0;
  }

  /* Central moments of fbar about u, Eq. (4).  For p+q >= 2 they equal those of f
   * up to the C shift (Sections 3-4). */
  double c[9], rho_c;
  orc_central_moments(fb, ux, uy, &rho_c, c);
  (void)rho_c;

  /* Equilibrium central moments of the transformed DF (Section 4; Eq. (7) with
   * T0 -> T, shifted by half the C moments). */
  double Pi_eq = 0.0, M21_eq = 0.0, M12_eq = 0.0;
  double N_eq = 0.5 * Dy - 0.5 * Dx;
  double E_eq = 2.0 * RT - 0.5 * Dx - 0.5 * Dy;
  double M22_eq = RT * RT;

  /* Eq. (8): separate relaxation of each central moment. */
  double w1 = d.w1;
  double cs[9];
  cs[I00] = 1.0;
  cs[I10] = 0.0;
  cs[I01] = 0.0;
  cs[IPI] = w1 * Pi_eq + (1.0 - w1) * c[IPI];
  cs[IN] = w1 * N_eq + (1.0 - w1) * c[IN];
  cs[IE] = p->w2 * E_eq + (1.0 - p->w2) * c[IE];
  cs[I21] = p->w3 * M21_eq + (1.0 - p->w3) * c[I21];
  cs[I12] = p->w3 * M12_eq + (1.0 - p->w3) * c[I12];
  cs[I22] = p->w4 * M22_eq + (1.0 - p->w4) * c[I22];

  /* Eq. (18) then Eq. (3): post-collision transformed populations. */
  double rs[9], fstar[9];
  orc_post_collision_raw(cs, ux, uy, ax, ay, rs);
  orc_pops_from_moments(rho, rs, fstar);

  /* Source and correction populations in the form of Eq. (3). */
  double sm[9], cm[9], S[9], C[9];
  orc_source_moments(ax, ay, ux, uy, sm);
  orc_pops_from_moments(rho, sm, S);
  orc_correction_moments(Dx, Dy, ux, uy, cm);
  orc_pops_from_moments(rho, cm, C);

  /* Eq. (27): what streams is fbar* + S + C. */
  for (int a = 0; a < 9; ++a) fout[a] = fstar[a] + S[a] + C[a];

  if (!p->thermal) {
    for (int a = 0; a < 9; ++a) hout[a] = 0.0;
    return;
  }

  if (p->energy_df == 1) {
    /* internal-energy DF (orc_geq): BGK towards e f^eq with the force source G */
    double geq[9], G[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    orc_geq(rho, ux, uy, RT, d.b, geq);
    double ge = 0.5 * rho * (0.5 * d.b * RT); /* half of rho e */
    G[1] = ge * ax;
    G[3] = -ge * ax;
    G[2] = ge * ay;
    G[4] = -ge * ay;
    for (int a = 0; a < 9; ++a) hout[a] = hb[a] - d.wh * (hb[a] - geq[a]) + (1.0 - 0.5 * d.wh) * G[a];
    return;
  }

  /* Energy DF, Section 4. */
  double feq[9], heq[9], K[9];
  orc_feq(rho, ux, uy, RT, feq);
  orc_heq_mode(rho, ux, uy, RT, d.b, p->heq_moments, heq);
  double u2 = ux * ux + uy * uy;
  for (int a = 0; a < 9; ++a) {
    double fa = fb[a] + 0.5 * S[a] + 0.5 * C[a];        /* undo the transform of Eq. (27) */
    double Z = EX[a] * ux + EY[a] * uy - 0.5 * u2;       /* Z_a = e_a . u - u^2/2, Eq. (22) */
    K[a] = Z * d.inv_tau_hf * (fa - feq[a]);              /* K_a = Z_a/tau_hf (f_a - f_a^eq) */
  }
  /* Body-force source of the energy DF (option): the force changes u inside
   * the step, hence the equilibrium energy flux (rho E + p) u, by (rho E + p) a
   * per unit time; nothing in the energy DF supplies that change, and the
   * Chapman-Enskog flux then carries -(1/w_h - 1/2)(rho E + p) a.  F has first
   * moment (rho E + p) a on the axis links and no other moment. */
  double F[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (p->h_force == 1) {
    double Etot = 0.5 * (d.b * RT + u2);
    double g = rho * (Etot + RT);
    F[1] = 0.5 * g * ax;
    F[3] = -0.5 * g * ax;
    F[2] = 0.5 * g * ay;
    F[4] = -0.5 * g * ay;
  }
  if (p->h_collision == 1) {
    /* the paper's BGK update of the transformed energy DF */
    for (int a = 0; a < 9; ++a)
      hout[a] = hb[a] - d.wh * (hb[a] - heq[a]) + (1.0 - 0.5 * d.wh) * (K[a] + F[a]);
    return;
  }
  /* Two-rate update: the same transformed scheme written moment by moment.  The
   * energy-flux moments (first order) relax with w_h, which fixes the thermal
   * conductivity exactly as the BGK update does; every other non-conserved moment
   * relaxes with rate 1.  Source moments carry the matching (1 - w/2) factors.
   * The total (zeroth moment) is untouched since sum (hbar - h^eq) = sum K = 0. */
  double neq[9], mn[9], mk[9], post[9], rho_n;
  for (int a = 0; a < 9; ++a) neq[a] = hb[a] - heq[a];
  double Mn[3][3], Mk[3][3];
  for (int p2 = 0; p2 < 3; ++p2)
    for (int q2 = 0; q2 < 3; ++q2) {
      double sn = 0.0, sk = 0.0;
      for (int a = 0; a < 9; ++a) {
        double w = pw(EX[a], p2) * pw(EY[a], q2);
        sn += neq[a] * w;
        sk += K[a] * w;
      }
      Mn[p2][q2] = sn;
      Mk[p2][q2] = sk;
    }
  (void)rho_n;
  set_from_pq(Mn, mn);
  set_from_pq(Mk, mk);
  const double kf = 1.0 - d.wh, sf = 1.0 - 0.5 * d.wh; /* flux moments */
  const double ko = 0.0, so = 0.5;                     /* other moments, rate 1 */
  double mp[9];
  mp[I00] = 0.0;
  mp[I10] = kf * mn[I10] + sf * (mk[I10] + (F[1] - F[3]));
  mp[I01] = kf * mn[I01] + sf * (mk[I01] + (F[2] - F[4]));
  for (int i = IE; i <= I22; ++i) mp[i] = ko * mn[i] + so * mk[i];
  orc_pops_from_moments(1.0, mp, post);
  for (int a = 0; a < 9; ++a) hout[a] = heq[a] + post[a];
}

/* ---------------------------------------------------------------------------
 * Whole-lattice operations.  Storage: X[a*nx*ny + y*nx + x], FP64.
 * ------------------------------------------------------------------------- */
#define IDX(x, y) ((long)(y) * nx + (x))

static int wrap(int v, int n) { return ((v % n) + n) % n; }

/* Non-equilibrium extrapolation on WALL sides (y sides only):
 * X(x_b) = X^eq(rho_f, u_w, T_w) + [X(x_f) - X^eq(rho_f, u_f, T_f)] for both DFs. */
static void wall_prestep(const orc_params *p, double *f, double *h) {
  const int nx = p->nx, ny = p->ny;
  const long n = (long)nx * ny;
  orc_derived d = derive(p);
  for (int side = ORC_YLO; side <= ORC_YHI; ++side) {
    if (!is_wall(p->bc[side])) continue;
    int yb = (side == ORC_YLO) ? 0 : ny - 1;
    int yf = (side == ORC_YLO) ? 1 : ny - 2;
    for (int x = 0; x < nx; ++x) {
      long ib = IDX(x, yb), i_f = IDX(x, yf);
      double fb[9], hb[9];
      for (int a = 0; a < 9; ++a) {
        fb[a] = f[a * n + i_f];
        hb[a] = p->thermal ? h[a * n + i_f] : 0.0;
      }
      double r, vx, vy, t;
      orc_node_macros(p, fb, hb, node_ax(p, i_f), node_ay(p, i_f), &r, &vx, &vy, &t);
      double Tw = !p->thermal ? p->T0 : p->wall_T[side];
      if (p->thermal && p->bc[side] == ORC_WALL_ADIABATIC) {
        /* zero normal temperature gradient at the wall node, to second order:
         * -3 T_w + 4 T_1 - T_2 = 0 with T_1, T_2 one and two nodes inside */
        int y2 = (side == ORC_YLO) ? 2 : ny - 3;
        long i2 = IDX(x, y2);
        double f2[9], h2[9], r2, vx2, vy2, t2;
        for (int a = 0; a < 9; ++a) {
          f2[a] = f[a * n + i2];
          h2[a] = h[a * n + i2];
        }
        orc_node_macros(p, f2, h2, node_ax(p, i2), node_ay(p, i2), &r2, &vx2, &vy2, &t2);
        Tw = (4.0 * t - t2) / 3.0;
      }
      /* wall pressure: the fluid neighbour's, carried one node along the
       * outward normal by the static momentum balance grad p = rho a */
      double an = (side == ORC_YLO) ? -node_ay(p, i_f) : node_ay(p, i_f);
      double rw = (p->wall_rho == 2) ? (r * p->R * t + r * an) / (p->R * Tw) : r;
      if (p->wall_rho == 0) {
        /* density from the populations that reached the wall node: rest and
         * tangential ones (k0) and those that arrived from the fluid (kin) */
        double k0 = 0.0, kin = 0.0;
        for (int a = 0; a < 9; ++a) {
          int en = (side == ORC_YLO) ? -EY[a] : EY[a]; /* e_a . outward normal */
          if (en == 0) k0 += f[a * n + ib];
          else if (en > 0) kin += f[a * n + ib];
        }
        double un = (side == ORC_YLO) ? -p->wall_uy[side] : p->wall_uy[side];
        double anw = (side == ORC_YLO) ? -node_ay(p, ib) : node_ay(p, ib);
        rw = (k0 + 2.0 * kin) / (1.0 + un - 0.5 * anw);
      }
      double fw[9], ff[9], hw[9], hf[9];
      orc_feq(rw, p->wall_ux[side], p->wall_uy[side], p->R * Tw, fw);
      orc_feq(r, vx, vy, p->R * t, ff);
      /* the stored DF is the transformed one, fbar = f - S/2 - C/2, so its
       * equilibrium part is f^eq - S/2 at either node (C has no mass or
       * momentum; its share stays in the extrapolated non-equilibrium part) */
      double smw[9], smf[9], Sw[9], Sf[9];
      orc_source_moments(node_ax(p, ib), node_ay(p, ib), p->wall_ux[side], p->wall_uy[side], smw);
      orc_pops_from_moments(rw, smw, Sw);
      orc_source_moments(node_ax(p, i_f), node_ay(p, i_f), vx, vy, smf);
      orc_pops_from_moments(r, smf, Sf);
      for (int a = 0; a < 9; ++a) f[a * n + ib] = (fw[a] - 0.5 * Sw[a]) + (fb[a] - (ff[a] - 0.5 * Sf[a]));
      if (p->thermal && p->energy_df == 1) {
        orc_geq(rw, p->wall_ux[side], p->wall_uy[side], p->R * Tw, d.b, hw);
        orc_geq(r, vx, vy, p->R * t, d.b, hf);
        for (int a = 0; a < 9; ++a) h[a * n + ib] = hw[a] + (hb[a] - hf[a]);
      } else if (p->thermal) {
        orc_heq_mode(rw, p->wall_ux[side], p->wall_uy[side], p->R * Tw, d.b, p->heq_moments, hw);
        orc_heq_mode(r, vx, vy, p->R * t, d.b, p->heq_moments, hf);
        for (int a = 0; a < 9; ++a) h[a * n + ib] = hw[a] + (hb[a] - hf[a]);
      }
    }
  }
}

/* Second-order derivative of q along one axis at index i of n samples:
 * central difference in the bulk or across a periodic wrap, one-sided
 * second-order difference on a non-periodic edge. */
static double deriv(const double *q, int i, int n, long stride, int periodic) {
  if (periodic) {
    return 0.5 * (q[(long)wrap(i + 1, n) * stride] - q[(long)wrap(i - 1, n) * stride]);
  }
  if (i == 0) return 0.5 * (-3.0 * q[0] + 4.0 * q[stride] - q[2 * stride]);
  if (i == n - 1)
    return 0.5 * (3.0 * q[(long)(n - 1) * stride] - 4.0 * q[(long)(n - 2) * stride] + q[(long)(n - 3) * stride]);
  return 0.5 * (q[(long)(i + 1) * stride] - q[(long)(i - 1) * stride]);
}

int orc_check_params(const orc_params *p) {
  if (p->nx < 3 || p->ny < 3) return 1;
  if (!(p->tau_f > 0.5) || !(p->gamma > 1.0) || !(p->Pr > 0.0) || !(p->R > 0.0) || !(p->T0 > 0.0)) return 1;
  for (int s = 0; s < 4; ++s)
    if (p->bc[s] < 0 || p->bc[s] > 3) return 1;
  if (p->viscosity_mode < 0 || p->viscosity_mode > 1 || (p->viscosity_mode == 1 && !(p->mu0 > 0.0))) return 1;
  if (p->wall_rho < 0 || p->wall_rho > 2 || p->heq_moments < 0 || p->heq_moments > 1 || p->h_collision < 0 || p->h_collision > 1 || p->h_force < 0 || p->h_force > 1) return 1;
  if (p->energy_df < 0 || p->energy_df > 1) return 1;
  if ((p->bc[ORC_XLO] == ORC_PERIODIC) != (p->bc[ORC_XHI] == ORC_PERIODIC)) return 1;
  if ((p->bc[ORC_YLO] == ORC_PERIODIC) != (p->bc[ORC_YHI] == ORC_PERIODIC)) return 1;
  if (is_wall(p->bc[ORC_XLO]) || is_wall(p->bc[ORC_XHI])) return 1; /* walls on y sides only */
  return 0;
}

/* Initial state (fbar = f^eq - S/2, hbar = h^eq or g^eq) from macroscopic fields. */
int orc_init(const orc_params *p, const double *rho, const double *ux, const double *uy, const double *T,
             double *f, double *h) {
  if (orc_check_params(p)) return 1;
  const int nx = p->nx, ny = p->ny;
  const long n = (long)nx * ny;
  orc_derived d = derive(p);
  for (long i = 0; i < n; ++i) {
    double t = p->thermal ? T[i] : p->T0;
    double RT = p->R * t;
    double feq[9], sm[9], S[9], heq[9];
    orc_feq(rho[i], ux[i], uy[i], RT, feq);
    orc_source_moments(node_ax(p, i), node_ay(p, i), ux[i], uy[i], sm);
    orc_pops_from_moments(rho[i], sm, S);
    if (p->energy_df == 1)
      orc_geq(rho[i], ux[i], uy[i], RT, d.b, heq);
    else
      orc_heq_mode(rho[i], ux[i], uy[i], RT, d.b, p->heq_moments, heq);
    for (int a = 0; a < 9; ++a) {
      f[a * n + i] = feq[a] - 0.5 * S[a];
      h[a * n + i] = p->thermal ? heq[a] : 0.0;
    }
  }
  return 0;
}

/* Macroscopic fields of the state as the next step would see it (wall nodes
 * after their non-equilibrium extrapolation). */
int orc_macros(const orc_params *p, const double *f_in, const double *h_in, double *rho, double *ux,
               double *uy, double *T) {
  if (orc_check_params(p)) return 1;
  const int nx = p->nx, ny = p->ny;
  const long n = (long)nx * ny;
  double *f = (double *)malloc(sizeof(double) * 9 * n);
  double *h = (double *)malloc(sizeof(double) * 9 * n);
  if (!f || !h) {
    free(f);
    free(h);
    return 2;
  }
  memcpy(f, f_in, sizeof(double) * 9 * n);
  memcpy(h, h_in, sizeof(double) * 9 * n);
  wall_prestep(p, f, h);
  for (long i = 0; i < n; ++i) {
    double fb[9], hb[9];
    for (int a = 0; a < 9; ++a) {
      fb[a] = f[a * n + i];
      hb[a] = h[a * n + i];
    }
    orc_node_macros(p, fb, hb, node_ax(p, i), node_ay(p, i), &rho[i], &ux[i], &uy[i], &T[i]);
  }
  free(f);
  free(h);
  return 0;
}

/* Macroscopic fields and Q = u (1 - theta), theta = T/T0, of a state whose
 * wall nodes have already been extrapolated (Section 4's correction needs Q). */
static void macro_fields(const orc_params *p, const double *f, const double *h, double *Rho, double *Ux,
                         double *Uy, double *Tt, double *Qx, double *Qy) {
  const long n = (long)p->nx * p->ny;
#pragma omp parallel for schedule(static)
  for (long i = 0; i < n; ++i) {
    double fb[9], hb[9];
    for (int a = 0; a < 9; ++a) {
      fb[a] = f[a * n + i];
      hb[a] = h[a * n + i];
    }
    orc_node_macros(p, fb, hb, node_ax(p, i), node_ay(p, i), &Rho[i], &Ux[i], &Uy[i], &Tt[i]);
    double theta = Tt[i] / p->T0;
    Qx[i] = Ux[i] * (1.0 - theta);
    Qy[i] = Uy[i] * (1.0 - theta);
  }
}

/* Section 4: Dx = d/dx[u_x (1 - theta)] and Dy = d/dy[u_y (1 - theta)] at node
 * (x, y) from the Q fields, by second-order differences (central in the bulk
 * and across periodic wraps, one-sided on non-periodic edges). */
static void node_gradients(const orc_params *p, const double *Qx, const double *Qy, int x, int y, double *Dx,
                           double *Dy) {
  const int nx = p->nx, ny = p->ny;
  const int xper = p->bc[ORC_XLO] == ORC_PERIODIC, yper = p->bc[ORC_YLO] == ORC_PERIODIC;
  *Dx = deriv(Qx + IDX(0, y), x, nx, 1, xper);
  *Dy = deriv(Qy + x, y, ny, nx, yper);
}

/* The correction gradients Dx, Dy (nx*ny each, index y*nx + x) that the next
 * collision of the state (f_in, h_in) uses: walls extrapolated first, as in
 * orc_step. */
int orc_gradients(const orc_params *p, const double *f_in, const double *h_in, double *Dx, double *Dy) {
  if (orc_check_params(p)) return 1;
  const int nx = p->nx, ny = p->ny;
  const long n = (long)nx * ny;
  double *f = (double *)malloc(sizeof(double) * 9 * n);
  double *h = (double *)malloc(sizeof(double) * 9 * n);
  double *mr = (double *)malloc(sizeof(double) * 6 * n);
  if (!f || !h || !mr) {
    free(f);
    free(h);
    free(mr);
    return 2;
  }
  memcpy(f, f_in, sizeof(double) * 9 * n);
  memcpy(h, h_in, sizeof(double) * 9 * n);
  wall_prestep(p, f, h);
  macro_fields(p, f, h, mr, mr + n, mr + 2 * n, mr + 3 * n, mr + 4 * n, mr + 5 * n);
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) node_gradients(p, mr + 4 * n, mr + 5 * n, x, y, &Dx[IDX(x, y)], &Dy[IDX(x, y)]);
  free(f);
  free(h);
  free(mr);
  return 0;
}

/* nsteps full time steps, in place on (f, h).  Step order: walls, macroscopic
 * variables, gradients of u(1 - theta), collision of f and h, pull streaming. */
int orc_step(const orc_params *p, double *f, double *h, int64_t nsteps) {
  if (orc_check_params(p)) return 1;
  const int nx = p->nx, ny = p->ny;
  const long n = (long)nx * ny;
  double *fp = (double *)malloc(sizeof(double) * 9 * n);
  double *hp = (double *)malloc(sizeof(double) * 9 * n);
  double *mr = (double *)malloc(sizeof(double) * 6 * n);
  if (!fp || !hp || !mr) {
    free(fp);
    free(hp);
    free(mr);
    return 2;
  }
  double *Rho = mr, *Ux = mr + n, *Uy = mr + 2 * n, *Tt = mr + 3 * n, *Qx = mr + 4 * n, *Qy = mr + 5 * n;
  const int xper = p->bc[ORC_XLO] == ORC_PERIODIC, yper = p->bc[ORC_YLO] == ORC_PERIODIC;

  for (int64_t s = 0; s < nsteps; ++s) {
    /* 0. walls */
    wall_prestep(p, f, h);

    /* 1. macroscopic variables, and Q = u (1 - theta) with theta = T/T0 */
    macro_fields(p, f, h, Rho, Ux, Uy, Tt, Qx, Qy);

    /* 2-4. gradients and collision */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
      for (int x = 0; x < nx; ++x) {
        long i = IDX(x, y);
        double Dx, Dy;
        node_gradients(p, Qx, Qy, x, y, &Dx, &Dy);
        double fb[9], hb[9], fo[9], ho[9];
        for (int a = 0; a < 9; ++a) {
          fb[a] = f[a * n + i];
          hb[a] = h[a * n + i];
        }
        orc_collide_node(p, fb, hb, Rho[i], Ux[i], Uy[i], Tt[i], Dx, Dy, node_ax(p, i), node_ay(p, i), fo, ho);
        for (int a = 0; a < 9; ++a) {
          fp[a * n + i] = fo[a];
          hp[a * n + i] = ho[a];
        }
      }
    }

    /* 5. pull streaming: X_a(x, t+1) = X*_a(x - e_a, t) */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
      for (int x = 0; x < nx; ++x) {
        long i = IDX(x, y);
        for (int a = 0; a < 9; ++a) {
          int sx = x - EX[a], sy = y - EY[a];
          int out_side = -1;
          if (sx < 0 && !xper) out_side = ORC_XLO;
          else if (sx >= nx && !xper) out_side = ORC_XHI;
          else if (sy < 0 && !yper) out_side = ORC_YLO;
          else if (sy >= ny && !yper) out_side = ORC_YHI;
          double fv, hv;
          if (out_side < 0) {
            long j = IDX(wrap(sx, nx), wrap(sy, ny));
            fv = fp[a * n + j];
            hv = hp[a * n + j];
          } else if (p->bc[out_side] == ORC_BOUNCEBACK) {
            /* halfway bounce-back at rest: the population sent towards the
             * side returns reversed to the same node */
            fv = fp[OPP[a] * n + i];
            hv = hp[OPP[a] * n + i];
          } else {
            /* wall node: replaced at the start of the next step */
            fv = fp[a * n + i];
            hv = hp[a * n + i];
          }
          f[a * n + i] = fv;
          h[a * n + i] = hv;
        }
      }
    }
  }
  free(fp);
  free(hp);
  free(mr);
  return 0;
}

/* Number of OpenMP threads the whole-lattice loops use. */
int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
