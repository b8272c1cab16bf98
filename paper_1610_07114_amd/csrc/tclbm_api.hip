// tclbm_api.hip -- host side of the C ABI declared in include/tclbm.h:
// parameter validation and derivation, the memory plan inside the caller's
// device buffer, initial state, stepping (with HIP-graph replay of fixed step
// chunks), FP64 moments and error reporting.  Every HIP failure becomes a
// status code; nothing here aborts.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/tclbm.h"
#include "tclbm_internal.h"
#include "tclbm_node.h"

using namespace tclbm;

struct tclbm_ctx {
  tclbm_params p;
  KParams k;             // template for launches (src/dst filled per step)
  hipStream_t stream;
  char *base;
  void *buf[2];
  int cur;               // index of the buffer holding the current state
  size_t esz;
  double *partials;
  int nparts;
  double *fields;        // library-owned, lazily allocated (4 * n doubles)
  int64_t steps;
  bool unstable;
  uint64_t version;      // bumped whenever the launch template changes
  int strip_rows_req;
  int graph_chunk;
  hipGraphExec_t graph;  // replays graph_chunk steps starting from buffer 0
  bool graph_ok;
  std::vector<double> th_ref;  // theta_r of each row, as the kernels see it
  int dev;                     // device current at create
  char err[512];
};

namespace {

constexpr size_t kAlign = 256;
size_t up(size_t v, size_t a) { return (v + a - 1) / a * a; }

void set_err(tclbm_ctx *c, const char *fmt, ...) {
  if (!c) return;
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(c->err, sizeof(c->err), fmt, ap);
  va_end(ap);
}

bool valid_params(const tclbm_params *p) {
  if (!p) return false;
  if (p->nx < 3 || p->ny < 3) return false;
  if ((long long)p->nx * p->ny > (1LL << 28)) return false;
  // kernels index a state buffer (all of its planes) with 32-bit element offsets
  {
    const size_t tw = (p->bc[kXlo] == kPeriodic) ? 62 : 61;  // tile_w_of
    if ((((size_t)p->nx + tw - 1) / tw) * 64 * (size_t)p->ny * (size_t)(p->thermal ? 18 : 9) >= (1ULL << 32))
      return false;
  }
  if (!(std::isfinite(p->R) && std::isfinite(p->T0) && p->R > 0 && p->T0 > 0)) return false;
  if (std::fabs(p->R * p->T0 - 1.0 / 3.0) > 1e-12) return false;
  if (!(p->gamma > 1.0) || !(p->Pr > 0.0) || !std::isfinite(p->gamma) || !std::isfinite(p->Pr)) return false;
  if (!(p->tau_f > 0.5) || !std::isfinite(p->tau_f)) return false;
  for (double w : {p->w2, p->w3, p->w4})
    if (!(w > 0.0 && w < 2.0)) return false;
  if (!std::isfinite(p->ax) || !std::isfinite(p->ay)) return false;
  if (p->thermal != 0 && p->thermal != 1) return false;
  if (p->correction != 0 && p->correction != 1) return false;
  if (p->storage < kF32 || p->storage > kF64) return false;
  if (p->wall_rho < 0 || p->wall_rho > 2) return false;
  if (p->heq_moments < 0 || p->heq_moments > 1) return false;
  if (p->h_collision < 0 || p->h_collision > 1) return false;
  if (p->h_force < 0 || p->h_force > 1) return false;
  if (p->energy_df != 0 && p->energy_df != 1) return false;
  if (p->accel_field != 0 && p->accel_field != 1) return false;
  if (p->viscosity_mode != 0 && p->viscosity_mode != 1) return false;
  if (p->viscosity_mode == 1 && !(p->mu0 > 0.0 && std::isfinite(p->mu0))) return false;
  for (int q = 0; q < 4; ++q) {
    if (p->bc[q] < kPeriodic || p->bc[q] > kWallAdiabatic) return false;
    if (!(std::isfinite(p->wall_ux[q]) && std::isfinite(p->wall_uy[q]) && std::isfinite(p->wall_T[q]))) return false;
    if (p->bc[q] == kWall && !(p->wall_T[q] > 0)) return false;
    // the adiabatic wall temperature uses the two rows inside the wall
    if (p->bc[q] == kWallAdiabatic && p->ny < 4) return false;
  }
  if (is_wall_kind(p->bc[kXlo]) || is_wall_kind(p->bc[kXhi])) return false;
  if ((p->bc[kXlo] == kPeriodic) != (p->bc[kXhi] == kPeriodic)) return false;
  if ((p->bc[kYlo] == kPeriodic) != (p->bc[kYhi] == kPeriodic)) return false;
  return true;
}

int pitch_of(const tclbm_params *p) { return (int)up((size_t)p->nx, 64); }
int planes_of(const tclbm_params *p) { return p->thermal ? 18 : 9; }
// x tiling of the waves and of the state blocks: a wave covers 64 lanes,
// lane_off halo lanes on the left, tile_w columns it evaluates and stores
// (62 with periodic x; 61 otherwise, for the second left neighbour that the
// one-sided difference at the right edge needs)
int lane_off_of(const tclbm_params *p) { return p->bc[kXlo] == kPeriodic ? 1 : 2; }
int tile_w_of(const tclbm_params *p) { return 63 - lane_off_of(p); }
// 64-slot blocks per stored row (one per x tile) and slots per plane
size_t blocks_of(const tclbm_params *p) { return ((size_t)p->nx + tile_w_of(p) - 1) / tile_w_of(p); }
size_t slots_of(const tclbm_params *p) { return blocks_of(p) * 64 * (size_t)p->ny; }

struct Plan {
  size_t buf, ref, acc, part, ctr, total;
};

Plan plan_of(const tclbm_params *p) {
  Plan pl;
  const size_t esz = store_bytes(p->storage);
  const size_t plane = (size_t)pitch_of(p) * p->ny;
  pl.buf = up(slots_of(p) * planes_of(p) * esz, kAlign);
  const size_t rsz = (p->storage == kF64) ? 8 : 4;
  pl.ref = up(rsz * (2 + 2 * 9) * (size_t)p->ny, kAlign);
  pl.acc = p->accel_field ? up(2 * plane * rsz, kAlign) : 0;
  const long long n = (long long)p->nx * p->ny;
  pl.part = up(sizeof(double) * kNumSums * (size_t)((n + 255) / 256), kAlign);
  pl.ctr = kAlign;  // two 32-bit step counters
  pl.total = 2 * pl.buf + pl.ref + pl.acc + pl.part + pl.ctr;
  return pl;
}

// Derived relaxation constants (Sections 4-5): b from gamma, w1 = 1/tau_f,
// 1/w_h = (1/w1 - 1/2)/Pr + 1/2, 1/tau_hf = w1 (Pr - 1).
void fill_kparams(tclbm_ctx *c) {
  const tclbm_params &p = c->p;
  KParams &k = c->k;
  memset(&k, 0, sizeof(k));
  k.nx = p.nx;
  k.ny = p.ny;
  k.pitch = pitch_of(&p);
  k.plane = (long long)k.pitch * p.ny;
  // state layout (tclbm_internal.h): one 64-slot block per x tile and plane,
  // the planes of a tile row contiguous
  const int np = planes_of(&p);
  k.lane_off = lane_off_of(&p);
  k.tile_w = tile_w_of(&p);
  k.slots = (long long)slots_of(&p);
  k.pstride = 64;
  k.tstride = np * 64;
  k.rstride = (unsigned)(np * 64 * blocks_of(&p));
  k.thermal = p.thermal;
  k.correction = p.correction;
  k.heq_mode = p.heq_moments;
  k.h_coll = p.h_collision;
  k.h_force = p.h_force;
  if (p.energy_df == 1) {
    // internal-energy DF: equilibrium mode 2 (e f^eq), BGK with its own force
    // source (the total-energy switches do not apply)
    k.heq_mode = 2;
    k.h_coll = 1;
    k.h_force = 0;
  }
  k.wall_rho = p.wall_rho;
  k.visc_mode = p.viscosity_mode;
  k.mu0_RT0 = p.mu0 / (p.R * p.T0);
  k.Pr = p.Pr;
  k.R = p.R;
  k.T0 = p.T0;
  k.b = 2.0 / (p.gamma - 1.0);
  k.w1 = 1.0 / p.tau_f;
  k.w2 = p.w2;
  k.w3 = p.w3;
  k.w4 = p.w4;
  k.wh = 1.0 / ((p.tau_f - 0.5) / p.Pr + 0.5);
  k.inv_tau_hf = k.w1 * (p.Pr - 1.0);
  k.ax = p.ax;
  k.ay = p.ay;
  for (int s = 0; s < 4; ++s) {
    k.bc[s] = p.bc[s];
    k.wall_ux[s] = p.wall_ux[s];
    k.wall_uy[s] = p.wall_uy[s];
    k.wall_T[s] = (p.bc[s] == kWall) ? p.wall_T[s] : p.T0;
  }
}

// Row-tiles per wave strip that the automatic strip height aims at, by storage
// (one wave-row is one 62-column tile row; see decompose and batch_auto_rows).
static long long strip_target(int storage) {
  return (storage == kF32) ? 81920 : (storage == kF64 ? 65536 : 20480);
}

void decompose(tclbm_ctx *c) {
  KParams &k = c->k;
  // lane_off and tile_w are fixed at create with the state layout
  k.n_xtiles = (k.nx + k.tile_w - 1) / k.tile_w;
  int rows = c->strip_rows_req;
  if (rows <= 0) {
    // enough waves to fill 256 CUs many times over: strips of a few rows when
    // the lattice is large, down to a single row when it is small.  Halo rows
    // are re-pulled once per strip, yet on 8192x4096 strips of 6-8 rows
    // measured fastest for FP32 (2 rows: 1048 us, 3: 983, 4: 973, 6: 967,
    // 8: 966, 16: 998, 32: 1024) and 24-32 rows for 16-bit storage (FP16
    // 8 rows: 680 us, 16: 654, 24: 650, 32: 644, 48: 665).
    long long r = ((long long)k.ny * k.n_xtiles) / strip_target(c->p.storage);
    rows = (int)(r < 1 ? 1 : (r > 64 ? 64 : r));
  }
  if (rows > k.ny) rows = k.ny;
  k.strip_rows = rows;
  k.n_strips = (k.ny + rows - 1) / rows;
}

// Wall temperatures as deviations from the wall row's reference theta_r (see
// KParams::wall_dth), formed in double from the references the kernels use.
void set_wall_dth(tclbm_ctx *c) {
  KParams &k = c->k;
  const int ny = k.ny;
  for (int side = 0; side < 4; ++side) {
    k.wall_dth[side] = 0.0;
    if (side < kYlo || c->th_ref.size() != (size_t)ny) continue;
    const int yw = (side == kYlo) ? 0 : ny - 1, y1 = (side == kYlo) ? 1 : ny - 2, y2 = (side == kYlo) ? 2 : ny - 3;
    if (k.bc[side] == kWall) k.wall_dth[side] = k.R * k.wall_T[side] - c->th_ref[yw];
    else if (k.bc[side] == kWallAdiabatic && ny >= 4)
      k.wall_dth[side] = (4.0 * c->th_ref[y1] - c->th_ref[y2] - 3.0 * c->th_ref[yw]) / 3.0;
  }
  fill_f32_consts(k);
}

bool bc_pairs_ok(const KParams &k) {
  if ((k.bc[kXlo] == kPeriodic) != (k.bc[kXhi] == kPeriodic)) return false;
  if ((k.bc[kYlo] == kPeriodic) != (k.bc[kYhi] == kPeriodic)) return false;
  return true;
}

#define HIP_TRY(ctx, expr)                                                    \
  do {                                                                        \
    hipError_t e_ = (expr);                                                   \
    if (e_ != hipSuccess) {                                                   \
      set_err(ctx, "%s failed: %s", #expr, hipGetErrorString(e_));           \
      return TCLBM_E_DEVICE;                                                  \
    }                                                                         \
  } while (0)

// Per-row rest-state reference: (rho_r, theta_r) from the row means of the
// initial fields, and the pull shifts r_a(y - e_ay) - r_a(y), s_a(...) - s_a(y),
// evaluated in double from the values the kernels will see (rounded to the
// compute type) so that writer and reader agree exactly.
template <class R>
void build_refs(const tclbm_params &p, const double *rho, const double *T, std::vector<R> &out) {
  const int ny = p.ny, nx = p.nx;
  const bool yper = p.bc[kYlo] == kPeriodic;
  const double b = 2.0 / (p.gamma - 1.0);
  out.assign((size_t)(2 + 18) * ny, R(0));
  R *rr = out.data();
  R *shF = rr + 2 * ny;
  R *shH = shF + 9 * ny;
  std::vector<double> rpop(9 * (size_t)ny), spop(9 * (size_t)ny);
  for (int y = 0; y < ny; ++y) {
    double rs = 0, ts = 0;
    for (int x = 0; x < nx; ++x) {
      rs += rho[(size_t)y * nx + x];
      ts += p.thermal ? T[(size_t)y * nx + x] : p.T0;
    }
    rr[2 * y] = (R)(rs / nx);
    rr[2 * y + 1] = (R)(p.R * (p.thermal ? ts / nx : p.T0));
    const int hm = p.energy_df ? 2 : p.heq_moments;
    RowRef<double> q = make_ref<double>((double)rr[2 * y], (double)rr[2 * y + 1], b, hm);
    ref_pops<double>(q, p.thermal, hm, &rpop[9 * (size_t)y], &spop[9 * (size_t)y]);
  }
  static const int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  for (int y = 0; y < ny; ++y)
    for (int a = 0; a < 9; ++a) {
      int sy = y - ey[a];
      if (ey[a] == 0) continue;
      if (yper) sy = (sy + ny) % ny;
      else if (sy < 0 || sy >= ny) continue;
      shF[9 * y + a] = (R)(rpop[9 * (size_t)sy + a] - rpop[9 * (size_t)y + a]);
      shH[9 * y + a] = (R)(spop[9 * (size_t)sy + a] - spop[9 * (size_t)y + a]);
    }
}

tclbm_status launch_steps(tclbm_ctx *c, int64_t n) {
  for (int64_t s = 0; s < n; ++s) {
    KParams k = c->k;
    k.src = c->buf[c->cur];
    k.dst = c->buf[1 - c->cur];
    k.par = c->cur;
    HIP_TRY(c, launch_step(k, c->p.storage, c->stream));
    c->cur = 1 - c->cur;
    ++c->steps;
  }
  return TCLBM_OK;
}

void drop_graph(tclbm_ctx *c) {
  if (c->graph_ok) hipGraphExecDestroy(c->graph);
  c->graph_ok = false;
}

tclbm_status build_graph(tclbm_ctx *c) {
  drop_graph(c);
  hipGraph_t g;
  HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  hipError_t lerr = hipSuccess;
  for (int s = 0; s < c->graph_chunk && lerr == hipSuccess; ++s) {
    KParams k = c->k;
    k.src = c->buf[s & 1];
    k.dst = c->buf[1 - (s & 1)];
    k.par = s & 1;
    lerr = launch_step(k, c->p.storage, c->stream);
  }
  hipError_t e = hipStreamEndCapture(c->stream, &g);
  if (lerr != hipSuccess || e != hipSuccess) {
    set_err(c, "graph capture failed: %s", hipGetErrorString(lerr != hipSuccess ? lerr : e));
    if (e == hipSuccess) hipGraphDestroy(g);
    return TCLBM_E_DEVICE;
  }
  e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (e != hipSuccess) {
    set_err(c, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
    return TCLBM_E_DEVICE;
  }
  c->graph_ok = true;
  return TCLBM_OK;
}

tclbm_status do_steps(tclbm_ctx *c, int64_t n) {
  if (!c) return TCLBM_E_INVALID;
  if (c->unstable) return TCLBM_E_STATE;
  if (n < 0) return TCLBM_E_INVALID;
  if (!bc_pairs_ok(c->k)) {
    set_err(c, "periodic sides must come in pairs");
    return TCLBM_E_INVALID;
  }
  // the legacy NULL stream cannot be captured: plain launches there
  const int ch = c->stream ? c->graph_chunk : 0;
  if (ch >= 2 && n >= 2 * (int64_t)ch) {
    if (c->cur != 0) {
      tclbm_status st = launch_steps(c, 1);
      if (st != TCLBM_OK) return st;
      --n;
    }
    if (!c->graph_ok) {
      tclbm_status st = build_graph(c);
      if (st != TCLBM_OK) return st;
    }
    while (n >= ch) {
      HIP_TRY(c, hipGraphLaunch(c->graph, c->stream));
      c->steps += ch;
      n -= ch;
    }
  }
  return launch_steps(c, n);
}

// FP64 sums: block partials added in block order (deterministic), then the
// instability check shared by both moments entry points.
void sums_begin(tclbm_sums &s, double &bad) {
  memset(&s, 0, sizeof(s));
  s.rho_min = 1e300;
  s.T_min = 1e300;
  bad = 0;
}

void sums_add(tclbm_sums &s, double &bad, const double *part, int nblocks) {
  for (int b = 0; b < nblocks; ++b) {
    const double *v = &part[(size_t)b * kNumSums];
    s.mass += v[kSumMass];
    s.momx += v[kSumMx];
    s.momy += v[kSumMy];
    s.energy += v[kSumE];
    s.kinetic += v[kSumKin];
    s.nu_num += v[kSumNu];
    s.rho_min = std::fmin(s.rho_min, v[kSumRhoMin]);
    s.T_min = std::fmin(s.T_min, v[kSumTMin]);
    bad += v[kSumBad];
  }
}

tclbm_status sums_end(tclbm_ctx *c, tclbm_sums &s, double bad, tclbm_sums *out) {
  s.nonfinite = (int64_t)bad;
  if (out) *out = s;
  if (s.nonfinite > 0 || !(s.rho_min > 0) || !(s.T_min > 0)) {
    c->unstable = true;
    set_err(c, "unstable state: %lld non-finite nodes, rho_min %g, T_min %g", (long long)s.nonfinite, s.rho_min,
            s.T_min);
    return TCLBM_E_UNSTABLE;
  }
  return TCLBM_OK;
}

}  // namespace

extern "C" {

void tclbm_default_params(int32_t nx, int32_t ny, tclbm_params *p) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->nx = nx;
  p->ny = ny;
  p->R = 1.0 / 3.0;
  p->T0 = 1.0;
  p->gamma = 1.4;
  p->Pr = 0.71;
  p->tau_f = 0.8;
  p->w2 = p->w3 = p->w4 = 1.0;
  p->thermal = 1;
  p->correction = 1;
  p->h_force = 1;
  p->storage = TCLBM_STORE_F32;
  for (int q = 0; q < 4; ++q) {
    p->bc[q] = TCLBM_BC_PERIODIC;
    p->wall_T[q] = 1.0;
  }
}

size_t tclbm_state_bytes(const tclbm_params *p) {
  if (!valid_params(p)) return 0;
  return plan_of(p).total;
}

tclbm_status tclbm_create(const tclbm_params *p, void *dev_buf, size_t dev_bytes, void *hip_stream,
                          const double *rho, const double *ux, const double *uy, const double *T,
                          const double *ax_field, const double *ay_field, tclbm_handle *out) {
  if (!out) return TCLBM_E_INVALID;
  *out = nullptr;
  if (!valid_params(p) || !dev_buf || !rho || !ux || !uy || (p->thermal && !T)) return TCLBM_E_INVALID;
  if ((p->accel_field != 0) != (ax_field != nullptr && ay_field != nullptr)) return TCLBM_E_INVALID;
  if ((reinterpret_cast<uintptr_t>(dev_buf) & (kAlign - 1)) != 0) return TCLBM_E_INVALID;
  const Plan pl = plan_of(p);
  if (dev_bytes < pl.total) return TCLBM_E_NOMEM;
  const long long n = (long long)p->nx * p->ny;
  for (long long i = 0; i < n; ++i) {
    if (!(std::isfinite(rho[i]) && rho[i] > 0 && std::isfinite(ux[i]) && std::isfinite(uy[i])))
      return TCLBM_E_INVALID;
    if (p->thermal && !(std::isfinite(T[i]) && T[i] > 0)) return TCLBM_E_INVALID;
    if (ax_field && !(std::isfinite(ax_field[i]) && std::isfinite(ay_field[i]))) return TCLBM_E_INVALID;
  }

  tclbm_ctx *c = new (std::nothrow) tclbm_ctx();
  if (!c) return TCLBM_E_NOMEM;
  if (hipGetDevice(&c->dev) != hipSuccess) {
    delete c;
    return TCLBM_E_DEVICE;
  }
  c->p = *p;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  c->base = reinterpret_cast<char *>(dev_buf);
  c->esz = store_bytes(p->storage);
  c->buf[0] = c->base;
  c->buf[1] = c->base + pl.buf;
  char *refs = c->base + 2 * pl.buf;
  const size_t rsz = (p->storage == kF64) ? 8 : 4;
  char *acc = c->base + 2 * pl.buf + pl.ref;
  c->partials = reinterpret_cast<double *>(acc + pl.acc);
  unsigned *ctr = reinterpret_cast<unsigned *>(acc + pl.acc + pl.part);
  c->nparts = (int)((n + 255) / 256);
  c->cur = 0;
  c->graph_chunk = 32;
  fill_kparams(c);
  c->k.rowref = refs;
  c->k.shiftF = refs + rsz * 2 * p->ny;
  c->k.shiftH = refs + rsz * (2 + 9) * p->ny;
  c->k.ctr = ctr;
  decompose(c);

  tclbm_status st = TCLBM_OK;
  double *tmp = nullptr;
  do {
    // per-row rest-state references of the deviation storage
    hipError_t e;
    c->th_ref.resize(p->ny);
    if (p->storage == kF64) {
      std::vector<double> ref;
      build_refs<double>(*p, rho, T, ref);
      for (int y = 0; y < p->ny; ++y) c->th_ref[y] = ref[2 * y + 1];
      e = hipMemcpyAsync(refs, ref.data(), ref.size() * sizeof(double), hipMemcpyHostToDevice, c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    } else {
      std::vector<float> ref;
      build_refs<float>(*p, rho, T, ref);
      for (int y = 0; y < p->ny; ++y) c->th_ref[y] = (double)ref[2 * y + 1];
      e = hipMemcpyAsync(refs, ref.data(), ref.size() * sizeof(float), hipMemcpyHostToDevice, c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    }
    set_wall_dth(c);
    if (e == hipSuccess) e = hipMemsetAsync(ctr, 0, 2 * sizeof(unsigned), c->stream);
    if (e != hipSuccess) { set_err(c, "ref upload: %s", hipGetErrorString(e)); st = TCLBM_E_DEVICE; break; }
    if (p->accel_field) {
      const size_t plane = (size_t)c->k.plane;
      if (p->storage == kF64) {
        std::vector<double> a(2 * plane, 0.0);
        for (int y = 0; y < p->ny; ++y)
          for (int x = 0; x < p->nx; ++x) {
            a[(size_t)y * c->k.pitch + x] = ax_field[(size_t)y * p->nx + x];
            a[plane + (size_t)y * c->k.pitch + x] = ay_field[(size_t)y * p->nx + x];
          }
        e = hipMemcpyAsync(acc, a.data(), a.size() * sizeof(double), hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        c->k.axf = acc;
        c->k.ayf = acc + plane * sizeof(double);
      } else {
        std::vector<float> a(2 * plane, 0.0f);
        for (int y = 0; y < p->ny; ++y)
          for (int x = 0; x < p->nx; ++x) {
            a[(size_t)y * c->k.pitch + x] = (float)ax_field[(size_t)y * p->nx + x];
            a[plane + (size_t)y * c->k.pitch + x] = (float)ay_field[(size_t)y * p->nx + x];
          }
        e = hipMemcpyAsync(acc, a.data(), a.size() * sizeof(float), hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        c->k.axf = acc;
        c->k.ayf = acc + plane * sizeof(float);
      }
      if (e != hipSuccess) { set_err(c, "accel upload: %s", hipGetErrorString(e)); st = TCLBM_E_DEVICE; break; }
    }
    // stage the initial fields and build the pre-pulled initial state
    e = hipMalloc(&tmp, sizeof(double) * 4 * (size_t)n);
    if (e != hipSuccess) { set_err(c, "hipMalloc: %s", hipGetErrorString(e)); st = TCLBM_E_NOMEM; tmp = nullptr; break; }
    const double *srcs[4] = {rho, ux, uy, p->thermal ? T : rho};
    for (int q = 0; q < 4 && e == hipSuccess; ++q)
      e = hipMemcpyAsync(tmp + (size_t)q * n, srcs[q], sizeof(double) * n, hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) { set_err(c, "field upload: %s", hipGetErrorString(e)); st = TCLBM_E_DEVICE; break; }
    KParams k = c->k;
    k.dst = c->buf[0];
    e = launch_init(k, p->storage, tmp, tmp + n, tmp + 2 * n, tmp + 3 * n, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) { set_err(c, "init: %s", hipGetErrorString(e)); st = TCLBM_E_DEVICE; break; }
  } while (0);
  if (tmp) hipFree(tmp);
  if (st != TCLBM_OK) {
    delete c;
    return st;
  }
  *out = c;
  return TCLBM_OK;
}

tclbm_status tclbm_set_bc(tclbm_handle c, int32_t side, int32_t kind, double ux_w, double uy_w, double T_w) {
  if (!c) return TCLBM_E_INVALID;
  if (side < 0 || side > 3 || kind < 0 || kind > kWallAdiabatic) return TCLBM_E_INVALID;
  if (is_wall_kind(kind) && side < kYlo) {
    set_err(c, "WALL is supported on y sides only");
    return TCLBM_E_INVALID;
  }
  if (kind == kWallAdiabatic && c->p.ny < 4) {
    set_err(c, "an adiabatic wall needs ny >= 4");
    return TCLBM_E_INVALID;
  }
  if (!(std::isfinite(ux_w) && std::isfinite(uy_w) && std::isfinite(T_w)) || (kind == kWall && !(T_w > 0)))
    return TCLBM_E_INVALID;
  if (side < kYlo && (kind == kPeriodic) != (c->p.bc[kXlo] == kPeriodic)) {
    set_err(c, "x periodicity is fixed at create (the state layout depends on it)");
    return TCLBM_E_INVALID;
  }
  c->k.bc[side] = kind;
  c->k.wall_ux[side] = ux_w;
  c->k.wall_uy[side] = uy_w;
  c->k.wall_T[side] = (kind == kWall) ? T_w : c->p.T0;
  set_wall_dth(c);
  decompose(c);
  drop_graph(c);
  ++c->version;
  return TCLBM_OK;
}

tclbm_status tclbm_set_tuning(tclbm_handle c, int32_t strip_rows, int32_t graph_chunk) {
  if (!c || strip_rows < 0 || graph_chunk < 0 || graph_chunk == 1 || (graph_chunk & 1)) return TCLBM_E_INVALID;
  c->strip_rows_req = strip_rows;
  c->graph_chunk = graph_chunk;
  decompose(c);
  drop_graph(c);
  ++c->version;
  return TCLBM_OK;
}

tclbm_status tclbm_step(tclbm_handle c, int64_t nsteps) { return do_steps(c, nsteps); }

tclbm_status tclbm_step_timed(tclbm_handle c, int64_t nsteps, double *ms) {
  if (!c || !ms) return TCLBM_E_INVALID;
  hipEvent_t e0, e1;
  HIP_TRY(c, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return TCLBM_E_DEVICE;
  }
  tclbm_status st = TCLBM_OK;
  hipError_t e = hipEventRecord(e0, c->stream);
  if (e == hipSuccess) {
    st = do_steps(c, nsteps);
    e = hipEventRecord(e1, c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float f = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&f, e0, e1);
    *ms = f;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st != TCLBM_OK) return st;
  if (e != hipSuccess) {
    set_err(c, "timing: %s", hipGetErrorString(e));
    return TCLBM_E_DEVICE;
  }
  return TCLBM_OK;
}

tclbm_status tclbm_moments(tclbm_handle c, double *rho, double *ux, double *uy, double *T, tclbm_sums *sums) {
  if (!c) return TCLBM_E_INVALID;
  if (!bc_pairs_ok(c->k)) return TCLBM_E_INVALID;
  const long long n = (long long)c->p.nx * c->p.ny;
  const bool want = rho || ux || uy || T;
  if (want && !c->fields) {
    hipError_t e = hipMalloc(&c->fields, sizeof(double) * 4 * (size_t)n);
    if (e != hipSuccess) {
      c->fields = nullptr;
      set_err(c, "hipMalloc fields: %s", hipGetErrorString(e));
      return TCLBM_E_NOMEM;
    }
  }
  double *F = c->fields;
  KParams k = c->k;
  k.src = c->buf[c->cur];
  int nb = 0;
  HIP_TRY(c, launch_moments(k, c->p.storage, want ? F : nullptr, want ? F + n : nullptr,
                            want ? F + 2 * n : nullptr, want ? F + 3 * n : nullptr, c->partials, &nb, c->stream));
  std::vector<double> part((size_t)nb * kNumSums);
  HIP_TRY(c, hipMemcpyAsync(part.data(), c->partials, part.size() * sizeof(double), hipMemcpyDeviceToHost,
                            c->stream));
  double *outs[4] = {rho, ux, uy, T};
  for (int q = 0; q < 4; ++q)
    if (outs[q])
      HIP_TRY(c, hipMemcpyAsync(outs[q], F + (size_t)q * n, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  tclbm_sums s;
  double bad;
  sums_begin(s, bad);
  sums_add(s, bad, part.data(), nb);
  return sums_end(c, s, bad, sums);
}

}  // extern "C"

// ---------------------------------------------- moments without allocation ---
// Device scratch of tclbm_moments_noalloc: a file-scope array, so every GPU the
// library runs on holds its own copy (at its own address) until the process
// ends.  In host code `scratch` names a host-side stand-in, not device memory:
// host code uses only the address hipGetSymbolAddress returns for each device.
constexpr size_t kScratchBytes = (size_t)4 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
static unsigned char *g_scratch[kMaxDevices];  // per device, set once
static std::mutex g_scratch_mu;
// block partials of one chunk, copied to the caller's thread stack
constexpr int kChunkBlocks = 512;

// Address of the scratch array on device `dev`, which must be current.
static tclbm_status scratch_on(tclbm_ctx *c, int dev, unsigned char **out) {
  if (dev < 0 || dev >= kMaxDevices) {
    set_err(c, "device %d beyond the %d the scratch table holds", dev, kMaxDevices);
    return TCLBM_E_DEVICE;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_err(c, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
      return TCLBM_E_DEVICE;
    }
    g_scratch[dev] = reinterpret_cast<unsigned char *>(p);
  }
  *out = g_scratch[dev];
  return TCLBM_OK;
}

static tclbm_status moments_noalloc(tclbm_ctx *c, double *rho, double *ux, double *uy, double *T, tclbm_sums *sums) {
  unsigned char *base = nullptr;
  tclbm_status st = scratch_on(c, c->dev, &base);
  if (st != TCLBM_OK) return st;
  const long long n = (long long)c->p.nx * c->p.ny;
  const int bn = moments_block_nodes();
  const long long nb = (n + bn - 1) / bn;
  double *outs[4] = {rho, ux, uy, T};
  const bool want = rho || ux || uy || T;
  // per chunk: partials of its blocks, then (when fields are asked for) the
  // four fields of its nodes; both rewritten in full by every chunk
  const size_t per_block = sizeof(double) * (kNumSums + (want ? 4 * (size_t)bn : 0));
  const int chunk = (int)std::min<size_t>(kChunkBlocks, kScratchBytes / per_block);
  double *d_part = reinterpret_cast<double *>(base);
  double *d_f = d_part + (size_t)chunk * kNumSums;
  const size_t fstride = (size_t)chunk * bn;
  double part[kChunkBlocks * kNumSums];
  KParams k = c->k;
  k.src = c->buf[c->cur];
  tclbm_sums s;
  double bad;
  sums_begin(s, bad);
  for (long long b0 = 0; b0 < nb; b0 += chunk) {
    const int m = (int)std::min<long long>(chunk, nb - b0);
    const long long i0 = b0 * bn, cnt = std::min<long long>((long long)m * bn, n - i0);
    HIP_TRY(c, launch_moments_range(k, c->p.storage, b0, m, want ? d_f : nullptr, want ? d_f + fstride : nullptr,
                                    want ? d_f + 2 * fstride : nullptr, want ? d_f + 3 * fstride : nullptr, d_part,
                                    c->stream));
    HIP_TRY(c, hipMemcpyAsync(part, d_part, sizeof(double) * kNumSums * m, hipMemcpyDeviceToHost, c->stream));
    for (int q = 0; q < 4; ++q)
      if (outs[q])
        HIP_TRY(c, hipMemcpyAsync(outs[q] + i0, d_f + q * fstride, sizeof(double) * cnt, hipMemcpyDeviceToHost,
                                  c->stream));
    // the next chunk reuses the scratch and `part`
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    sums_add(s, bad, part, m);
  }
  return sums_end(c, s, bad, sums);
}

extern "C" {

tclbm_status tclbm_moments_noalloc(tclbm_handle c, double *rho, double *ux, double *uy, double *T,
                                   tclbm_sums *sums) {
  if (!c) return TCLBM_E_INVALID;
  if (!bc_pairs_ok(c->k)) return TCLBM_E_INVALID;
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess) return TCLBM_E_DEVICE;
  if (prev != c->dev && hipSetDevice(c->dev) != hipSuccess) return TCLBM_E_DEVICE;
  const tclbm_status st = moments_noalloc(c, rho, ux, uy, T, sums);
  if (prev != c->dev) (void)hipSetDevice(prev);
  return st;
}

int64_t tclbm_steps_done(tclbm_handle c) { return c ? c->steps : -1; }

const char *tclbm_step_kernel(tclbm_handle c) { return c ? step_kernel_name(c->k, c->p.storage) : nullptr; }

tclbm_status tclbm_read_state(tclbm_handle c, double *out) {
  if (!c || !out) return TCLBM_E_INVALID;
  const size_t cnt = (size_t)c->p.nx * c->p.ny * (c->p.thermal ? 18 : 9);
  double *d = nullptr;
  hipError_t e = hipMalloc(&d, cnt * sizeof(double));
  if (e != hipSuccess) {
    set_err(c, "hipMalloc: %s", hipGetErrorString(e));
    return TCLBM_E_NOMEM;
  }
  KParams k = c->k;
  k.src = c->buf[c->cur];
  e = launch_read_state(k, c->p.storage, d, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(out, d, cnt * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  hipFree(d);
  if (e != hipSuccess) {
    set_err(c, "read_state: %s", hipGetErrorString(e));
    return TCLBM_E_DEVICE;
  }
  return TCLBM_OK;
}

tclbm_status tclbm_destroy(tclbm_handle c) {
  if (!c) return TCLBM_E_INVALID;
  hipStreamSynchronize(c->stream);
  drop_graph(c);
  if (c->fields) hipFree(c->fields);
  delete c;
  return TCLBM_OK;
}

const char *tclbm_status_str(tclbm_status s) {
  switch (s) {
    case TCLBM_OK: return "ok";
    case TCLBM_E_INVALID: return "invalid argument";
    case TCLBM_E_NOMEM: return "out of memory";
    case TCLBM_E_DEVICE: return "device error";
    case TCLBM_E_STATE: return "handle unusable";
    case TCLBM_E_UNSTABLE: return "unstable state";
    default: return "unknown status";
  }
}

const char *tclbm_last_error(tclbm_handle c) { return c ? c->err : "no handle"; }

tclbm_status tclbm_hbm_copy(void *dst, const void *src, size_t bytes, void *hip_stream) {
  if (!dst || !src || (bytes & 15) || (reinterpret_cast<uintptr_t>(dst) & 15) ||
      (reinterpret_cast<uintptr_t>(src) & 15))
    return TCLBM_E_INVALID;
  hipError_t e = launch_copy(dst, src, bytes, reinterpret_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? TCLBM_OK : TCLBM_E_DEVICE;
}

}  // extern "C"

// ------------------------------------------------------------------ batches ---
struct tclbm_batch {
  std::vector<tclbm_handle> m;  // members, in table order
  std::vector<uint64_t> version;  // members' launch-template versions when tabled
  std::vector<int64_t> steps;     // members' step counts the table's parity assumes
  int storage;
  hipStream_t stream;
  KParams *d_tab;    // device table: n entries for even steps, n with src/dst swapped
  int *d_start;      // device prefix sums of waves per member
  int total_waves;
  int graph_chunk;
  hipGraphExec_t graph;
  bool graph_ok;
  int parity;        // 0: members' current state in the table's src
  int strip_rows_req;  // batch strip height (0: automatic), overrides the members'
  int strip_rows;      // the height in use
  bool all_default;    // every member runs the default scheme (leaner kernel)
  bool all_fit;        // every member's state buffers allow buffer addressing
  // persistent launches (tclbm_batch_set_persistent)
  int persist_steps;       // steps per launch (0: one launch per step)
  int persist_max_grid;    // blocks that fit on the device at once
  long long wait_ticks;    // longest barrier wait, wall-clock ticks
  PersistCtl *d_ctl;       // barrier counter and failure word
  unsigned *h_fail;        // pinned copy of the failure word after each launch
  unsigned arrive_base;    // barrier arrivals so far
  char err[256];
};

// Strip height for a whole batch: the single-lattice rule applied to the
// members' row-tiles together (256 uneven RB lattices: FP32 6 rows and FP16
// 26, within 1% of the fastest heights measured for that batch: FP32 2 rows
// 1004 us, 4: 946, 6: 937, 8: 939, 16: 989; FP16 16: 635, 24: 631, 32: 636),
// capped at 32.
static int batch_auto_rows(const tclbm_batch *b) {
  long long rowtiles = 0;
  for (tclbm_handle h : b->m) rowtiles += (long long)h->k.ny * h->k.n_xtiles;
  long long r = rowtiles / strip_target(b->storage);
  return (int)(r < 1 ? 1 : (r > 32 ? 32 : r));
}

// Launch table and wave prefix sums for the current members, strip height,
// and parity 0 = members' current buffers as src (device copies; synchronous).
static hipError_t batch_upload(tclbm_batch *b) {
  const int n = (int)b->m.size();
  b->strip_rows = b->strip_rows_req > 0 ? b->strip_rows_req : batch_auto_rows(b);
  std::vector<KParams> tab(2 * n);  // [0, n): even steps; [n, 2n): odd steps (src, dst swapped)
  std::vector<int> start(n + 1, 0);
  b->all_default = true;
  b->all_fit = true;
  for (int i = 0; i < n; ++i) {
    tclbm_handle h = b->m[i];
    b->all_default = b->all_default && default_scheme(h->k);
    b->all_fit = b->all_fit && buffer_fits(h->k, b->storage);
    tab[i] = h->k;
    tab[i].src = h->buf[h->cur];
    tab[i].dst = h->buf[1 - h->cur];
    tab[i].par = h->cur;
    const int rows = b->strip_rows < h->k.ny ? b->strip_rows : h->k.ny;
    tab[i].strip_rows = rows;
    tab[i].n_strips = (h->k.ny + rows - 1) / rows;
    start[i + 1] = start[i] + tab[i].n_xtiles * tab[i].n_strips;
    tab[n + i] = tab[i];
    tab[n + i].src = tab[i].dst;
    tab[n + i].dst = const_cast<void *>(tab[i].src);
    tab[n + i].par = 1 - h->cur;
  }
  b->total_waves = start[n];
  b->parity = 0;
  hipError_t e = hipMemcpy(b->d_tab, tab.data(), sizeof(KParams) * 2 * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->d_start, start.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice);
  return e;
}

static void batch_drop_graph(tclbm_batch *b) {
  if (b->graph_ok) hipGraphExecDestroy(b->graph);
  b->graph_ok = false;
}

// n plain launches, one step each; *done counts those enqueued
static tclbm_status batch_launch(tclbm_batch *b, int64_t n, int64_t *done) {
  for (int64_t s = 0; s < n; ++s) {
    hipError_t e = launch_batch_step(b->d_tab, b->d_start, (int)b->m.size(), b->total_waves, b->storage, b->parity,
                                     b->all_default, b->all_fit, b->stream);
    if (e != hipSuccess) {
      snprintf(b->err, sizeof(b->err), "batch launch: %s", hipGetErrorString(e));
      return TCLBM_E_DEVICE;
    }
    b->parity ^= 1;
    ++*done;
  }
  return TCLBM_OK;
}

// A persistent launch whose barrier wait ran out leaves every member's state
// undefined: the members are marked unstable and the batch refuses to step.
static bool batch_persist_failed(tclbm_batch *b) {
  if (!b->h_fail || __atomic_load_n(b->h_fail, __ATOMIC_ACQUIRE) == 0u) return false;
  for (tclbm_handle h : b->m) h->unstable = true;
  snprintf(b->err, sizeof(b->err),
           "persistent batch: a block waited longer than the barrier limit; the members' states are undefined");
  return true;
}

// n steps in launches of at most persist_steps steps each
static tclbm_status batch_persist_run(tclbm_batch *b, int64_t n, int64_t *done) {
  const int nwork = (b->total_waves + step_waves_per_block() - 1) / step_waves_per_block();
  const int grid = nwork < b->persist_max_grid ? nwork : b->persist_max_grid;
  while (n > 0) {
    const int k = (int)(n < b->persist_steps ? n : b->persist_steps);
    hipError_t e = launch_batch_persistent(b->d_tab, b->d_start, (int)b->m.size(), b->total_waves, b->storage,
                                           b->parity, k, b->d_ctl, b->arrive_base, b->wait_ticks, grid, b->stream);
    if (e != hipSuccess) {
      snprintf(b->err, sizeof(b->err), "persistent batch launch: %s", hipGetErrorString(e));
      return TCLBM_E_DEVICE;
    }
    b->arrive_base += (unsigned)(k - 1) * (unsigned)grid;
    b->parity ^= (k & 1);
    *done += k;
    n -= k;
    e = hipMemcpyAsync(b->h_fail, &b->d_ctl->fail, sizeof(unsigned), hipMemcpyDeviceToHost, b->stream);
    if (e != hipSuccess) {
      snprintf(b->err, sizeof(b->err), "persistent batch: %s", hipGetErrorString(e));
      return TCLBM_E_DEVICE;
    }
  }
  return TCLBM_OK;
}

// Enqueue n steps: replays of the captured chunk while at least two chunks
// remain (after one plain step if the parity is odd), plain launches for the
// rest.  *done counts the steps actually enqueued, also on a failure.
static tclbm_status batch_run(tclbm_batch *b, int64_t n, int64_t *done) {
  if (b->persist_steps > 0) {
    // a cooperative launch cannot be recorded into a graph: under stream
    // capture the batch records per-step launches instead
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(b->stream, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone)
      return batch_persist_run(b, n, done);
  }
  const int ch = b->stream ? b->graph_chunk : 0;
  if (ch >= 2 && n >= 2 * (int64_t)ch) {
    if (b->parity) {
      tclbm_status st = batch_launch(b, 1, done);
      if (st != TCLBM_OK) return st;
      --n;
    }
    if (!b->graph_ok) {
      // capture records launches without running them: a failed capture
      // enqueues nothing
      hipGraph_t g;
      hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
      hipError_t le = hipSuccess;
      for (int s = 0; s < ch && le == hipSuccess && e == hipSuccess; ++s)
        le = launch_batch_step(b->d_tab, b->d_start, (int)b->m.size(), b->total_waves, b->storage, s & 1,
                               b->all_default, b->all_fit, b->stream);
      hipError_t ee = (e == hipSuccess) ? hipStreamEndCapture(b->stream, &g) : e;
      if (e != hipSuccess || le != hipSuccess || ee != hipSuccess) {
        if (e == hipSuccess && ee == hipSuccess) hipGraphDestroy(g);
        snprintf(b->err, sizeof(b->err), "batch capture failed");
        return TCLBM_E_DEVICE;
      }
      ee = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
      hipGraphDestroy(g);
      if (ee != hipSuccess) {
        snprintf(b->err, sizeof(b->err), "batch graph instantiation: %s", hipGetErrorString(ee));
        return TCLBM_E_DEVICE;
      }
      b->graph_ok = true;
    }
    while (n >= ch) {
      hipError_t e = hipGraphLaunch(b->graph, b->stream);
      if (e != hipSuccess) {
        snprintf(b->err, sizeof(b->err), "batch graph launch: %s", hipGetErrorString(e));
        return TCLBM_E_DEVICE;
      }
      *done += ch;  // an even chunk leaves the parity unchanged
      n -= ch;
    }
  }
  return batch_launch(b, n, done);
}

extern "C" {

tclbm_status tclbm_batch_create(tclbm_handle *members, int32_t n, tclbm_batch_handle *out) {
  if (!out) return TCLBM_E_INVALID;
  *out = nullptr;
  if (!members || n <= 0) return TCLBM_E_INVALID;
  for (int i = 0; i < n; ++i) {
    tclbm_handle h = members[i];
    if (!h || h->unstable) return TCLBM_E_INVALID;
    if (h->p.storage != members[0]->p.storage || h->stream != members[0]->stream) return TCLBM_E_INVALID;
    if (!bc_pairs_ok(h->k)) return TCLBM_E_INVALID;
    for (int j = 0; j < i; ++j)
      if (members[j] == h) return TCLBM_E_INVALID;
  }
  tclbm_batch *b = new (std::nothrow) tclbm_batch();
  if (!b) return TCLBM_E_NOMEM;
  b->m.assign(members, members + n);
  // largest members first: their waves start first and the tail is short ones
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  auto work = [&](int i) { return (long long)b->m[i]->k.n_xtiles * b->m[i]->k.ny; };
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work(x) > work(y); });
  std::vector<tclbm_handle> sorted(n);
  for (int i = 0; i < n; ++i) sorted[i] = b->m[order[i]];
  b->m = sorted;
  for (tclbm_handle h : b->m) {
    b->version.push_back(h->version);
    b->steps.push_back(h->steps);
  }
  b->storage = members[0]->p.storage;
  b->stream = members[0]->stream;
  b->graph_chunk = 16;
  b->strip_rows_req = 0;
  hipError_t e = hipMalloc(&b->d_tab, sizeof(KParams) * 2 * n);
  if (e == hipSuccess) e = hipMalloc(&b->d_start, sizeof(int) * (n + 1));
  if (e == hipSuccess) e = hipMalloc(&b->d_ctl, sizeof(PersistCtl));
  if (e == hipSuccess) e = hipMemset(b->d_ctl, 0, sizeof(PersistCtl));
  if (e == hipSuccess) e = hipHostMalloc((void **)&b->h_fail, sizeof(unsigned), hipHostMallocDefault);
  if (e == hipSuccess) {
    *b->h_fail = 0u;
    e = batch_upload(b);
  }
  if (e != hipSuccess) {
    if (b->d_tab) hipFree(b->d_tab);
    if (b->d_start) hipFree(b->d_start);
    if (b->d_ctl) hipFree(b->d_ctl);
    if (b->h_fail) hipHostFree(b->h_fail);
    delete b;
    return TCLBM_E_DEVICE;
  }
  *out = b;
  return TCLBM_OK;
}

tclbm_status tclbm_batch_step(tclbm_batch_handle b, int64_t nsteps) {
  if (!b || nsteps < 0) return TCLBM_E_INVALID;
  if (batch_persist_failed(b)) return TCLBM_E_STATE;
  for (size_t i = 0; i < b->m.size(); ++i) {
    tclbm_handle h = b->m[i];
    if (h->unstable) return TCLBM_E_STATE;
    // a member stepped alone or re-tuned since the table was built: the table's
    // buffers or launch shape no longer describe it
    if (h->version != b->version[i] || h->steps != b->steps[i]) {
      snprintf(b->err, sizeof(b->err), "member %zu changed outside the batch", i);
      return TCLBM_E_STATE;
    }
  }
  int64_t done = 0;
  const tclbm_status st = batch_run(b, nsteps, &done);
  // members' bookkeeping on every exit path: the state now lives in the buffer
  // the parity names, after the steps actually enqueued
  for (size_t i = 0; i < b->m.size(); ++i) {
    tclbm_handle h = b->m[i];
    h->steps += done;
    b->steps[i] = h->steps;
    if (done & 1) h->cur = 1 - h->cur;
  }
  return st;
}

tclbm_status tclbm_batch_step_timed(tclbm_batch_handle b, int64_t nsteps, double *ms) {
  if (!b || !ms) return TCLBM_E_INVALID;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return TCLBM_E_DEVICE;
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return TCLBM_E_DEVICE;
  }
  hipEventRecord(e0, b->stream);
  tclbm_status st = tclbm_batch_step(b, nsteps);
  hipEventRecord(e1, b->stream);
  hipError_t e = hipEventSynchronize(e1);
  float f = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&f, e0, e1);
  *ms = f;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != TCLBM_OK) return st;
  if (e != hipSuccess) return TCLBM_E_DEVICE;
  return batch_persist_failed(b) ? TCLBM_E_DEVICE : TCLBM_OK;
}

int32_t tclbm_batch_size(tclbm_batch_handle b) { return b ? (int32_t)b->m.size() : -1; }

int64_t tclbm_batch_waves(tclbm_batch_handle b) { return b ? b->total_waves : -1; }

tclbm_status tclbm_batch_set_graph_chunk(tclbm_batch_handle b, int32_t chunk) {
  if (!b || chunk < 0 || chunk == 1 || (chunk & 1)) return TCLBM_E_INVALID;
  b->graph_chunk = chunk;
  batch_drop_graph(b);
  return TCLBM_OK;
}

tclbm_status tclbm_batch_set_strip_rows(tclbm_batch_handle b, int32_t rows) {
  if (!b || rows < 0) return TCLBM_E_INVALID;
  // the table is rebuilt from the members' bookkeeping (current buffers),
  // which restarts the parity at 0
  (void)hipStreamSynchronize(b->stream);
  b->strip_rows_req = rows;
  batch_drop_graph(b);
  if (batch_upload(b) != hipSuccess) return TCLBM_E_DEVICE;
  return TCLBM_OK;
}

int32_t tclbm_batch_strip_rows(tclbm_batch_handle b) { return b ? b->strip_rows : -1; }

tclbm_status tclbm_batch_set_persistent(tclbm_batch_handle b, int32_t steps_per_launch, int32_t wait_us) {
  if (!b || steps_per_launch < 0 || wait_us < 0) return TCLBM_E_INVALID;
  if (steps_per_launch == 0) {
    b->persist_steps = 0;
    return TCLBM_OK;
  }
  if (b->storage == kF64 || !b->all_default || !b->all_fit) {
    snprintf(b->err, sizeof(b->err),
             "persistent batch: FP32 or 16-bit storage, every member on the default scheme and within 4 GiB");
    return TCLBM_E_INVALID;
  }
  int dev = 0, coop = 0, khz = 0, maxb = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
  if (e == hipSuccess) e = persistent_max_blocks(b->storage, &maxb);
  if (e != hipSuccess || !coop || khz <= 0 || maxb <= 0) {
    snprintf(b->err, sizeof(b->err), "persistent batch: no cooperative launch on this device");
    return TCLBM_E_DEVICE;
  }
  b->persist_steps = steps_per_launch;
  b->persist_max_grid = maxb;
  b->wait_ticks = (long long)(wait_us > 0 ? wait_us : 1000000) * khz / 1000;
  return TCLBM_OK;
}

int32_t tclbm_batch_persistent(tclbm_batch_handle b) { return b ? b->persist_steps : -1; }

const char *tclbm_batch_step_kernel(tclbm_batch_handle b) {
  if (!b) return nullptr;
  return b->persist_steps > 0 ? batch_persistent_kernel_name(b->storage) : batch_step_kernel_name(b->storage);
}

tclbm_status tclbm_batch_destroy(tclbm_batch_handle b) {
  if (!b) return TCLBM_E_INVALID;
  (void)hipStreamSynchronize(b->stream);
  batch_drop_graph(b);
  (void)hipFree(b->d_tab);
  (void)hipFree(b->d_start);
  (void)hipFree(b->d_ctl);
  (void)hipHostFree(b->h_fail);
  delete b;
  return TCLBM_OK;
}

}  // extern "C"
