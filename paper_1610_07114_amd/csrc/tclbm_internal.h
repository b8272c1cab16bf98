// tclbm_internal.h -- declarations shared by the HIP kernels and the C-ABI host
// code of libtclbm (not installed; the public interface is include/tclbm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace tclbm {

enum StoreKind { kF32 = 0, kF16 = 1, kBF16 = 2, kF64 = 3 };
enum BcKind { kPeriodic = 0, kBounceBack = 1, kWall = 2, kWallAdiabatic = 3 };

// node walls (imposed velocity; imposed or adiabatic temperature)
__host__ __device__ inline bool is_wall_kind(int kind) { return kind == kWall || kind == kWallAdiabatic; }
enum Side { kXlo = 0, kXhi = 1, kYlo = 2, kYhi = 3 };

// Everything a kernel needs, passed by value.  Physical constants are double
// here and converted to the kernel's arithmetic type on entry.
struct KParams {
  const void *src;  // population buffer read this step (storage type)
  void *dst;        // population buffer written this step
  int nx, ny;
  int pitch;        // columns per stored row (nx rounded up to 64)
  long long plane;  // nodes per population plane (pitch * ny); the buffer holds 9 or 18 planes
  // State layout: every x tile of tile_w columns (see below) owns one block
  // of 64 slots per row and plane, the planes of a tile row contiguous.
  // Population a of node (x, y) sits at
  //   y * rstride + (x / tile_w) * tstride + a * pstride + lane_off + x % tile_w,
  // i.e. in the slot of the lane that evaluates it; pstride = 64,
  // tstride = planes * 64, rstride = planes * 64 * blocks per row.  The
  // other slots of a block hold nothing that is read.
  long long slots;  // slots per plane (64 * blocks per row * ny)
  long long pstride;
  int tstride;
  unsigned rstride;
  int thermal, correction, heq_mode, h_coll, h_force, wall_rho;
  int visc_mode;  // 1: per-node rates from mu = mu0 T/T0 (mu0 here as mu0/(R T0))
  double mu0_RT0, Pr;
  int bc[4];
  double wall_ux[4], wall_uy[4], wall_T[4];
  // wall temperatures as deviations of theta = R T from the wall row's
  // reference, formed in double on the host: WALL sides R T_w - theta_r(wall);
  // WALL_ADIABATIC sides the reference part of (4 theta_1 - theta_2)/3 -
  // theta_r(wall), (4 theta_r(1) - theta_r(2) - 3 theta_r(wall))/3, with rows
  // 1 and 2 counted inwards
  double wall_dth[4];
  double R, T0, b, w1, w2, w3, w4, wh, inv_tau_hf, ax, ay;
  // the constants in FP32, rounded once on the host (the FP32 kernels would
  // otherwise convert the doubles with vector instructions wherever the
  // compiler reloads them)
  struct F32 {
    float R, T0, b, w1, w2, w3, w4, wh, inv_tau_hf, two_b, inv_RT0, RT0f, dRT0, ax, ay;
    float wall_ux[4], wall_uy[4], wall_dth[4];
  } f32;
  const void *axf, *ayf;          // per-node acceleration, compute type, pitch layout (nullable)
  // per-row rest-state reference (compute type): rowref[2y] = rho_r,
  // rowref[2y+1] = theta_r = R T_r; shiftF/H[9y + a] = r_a(row y - e_ay) - r_a(y)
  // (zero where that row is outside a non-periodic side)
  const void *rowref, *shiftF, *shiftH;
  // march decomposition
  int tile_w, lane_off, n_xtiles, strip_rows, n_strips;
  // step counter of the lattice (16-bit stochastic rounding): ctr[par] holds
  // the number of the step this launch computes, where par is the index of
  // the source buffer; the launch writes ctr[1 - par] = ctr[par] + 1
  unsigned *ctr;
  int par;
};

// The default thermal scheme (the step kernels have a compile-time
// instantiation of it): correction on, continuous h^eq moments, two-rate
// energy update with its force source, wall density from the known
// populations, uniform acceleration, constant w1.
__host__ __device__ inline bool default_scheme(const KParams &k) {
  return k.thermal == 1 && k.correction == 1 && k.heq_mode == 0 && k.h_coll == 0 && k.h_force == 1 &&
         k.wall_rho == 0 && k.axf == nullptr && k.visc_mode == 0;
}

// Buffer-resource addressing of the default scheme (FP32 and 16-bit storage):
// one descriptor per state buffer, so its 18 planes must span less than 4 GiB.
__host__ __device__ inline bool buffer_fits(const KParams &k, int storage) {
  unsigned long long esz = (storage == kF32) ? 4ull : ((storage == kF16 || storage == kBF16) ? 2ull : 0ull);
  if (esz == 0) return false;
  return 18ull * (unsigned long long)k.slots * esz < (1ull << 32);
}

// FP32 copies of the launch constants (KParams::f32), rounded as the kernels
// would round them.
inline void fill_f32_consts(KParams &k) {
  KParams::F32 &f = k.f32;
  f.R = (float)k.R;
  f.T0 = (float)k.T0;
  f.b = (float)k.b;
  f.w1 = (float)k.w1;
  f.w2 = (float)k.w2;
  f.w3 = (float)k.w3;
  f.w4 = (float)k.w4;
  f.wh = (float)k.wh;
  f.inv_tau_hf = (float)k.inv_tau_hf;
  f.two_b = (float)(2.0 / k.b);
  f.inv_RT0 = (float)(1.0 / (k.R * k.T0));
  f.RT0f = (float)(k.R * k.T0);
  f.dRT0 = (float)(k.R * k.T0 - (double)f.RT0f);
  f.ax = (float)k.ax;
  f.ay = (float)k.ay;
  for (int s = 0; s < 4; ++s) {
    f.wall_ux[s] = (float)k.wall_ux[s];
    f.wall_uy[s] = (float)k.wall_uy[s];
    f.wall_dth[s] = (float)k.wall_dth[s];
  }
}

// Reduction record written per block by the moments kernel.
enum { kSumMass = 0, kSumMx, kSumMy, kSumE, kSumKin, kSumNu, kSumRhoMin, kSumTMin, kSumBad, kNumSums };

size_t store_bytes(int storage);

hipError_t launch_step(const KParams &k, int storage, hipStream_t s);
const char *step_kernel_name(const KParams &k, int storage);
int step_waves_per_block();
const char *batch_step_kernel_name(int storage);
// one step of every lattice in a device-side descriptor table (see tclbm_batch_*)
hipError_t launch_batch_step(const KParams *d_tab, const int *d_wave_start, int n_inst, int total_waves,
                             int storage, int parity, bool all_default, bool all_fit, hipStream_t s);
// Persistent batch: barrier state in device memory (zeroed at creation)
struct PersistCtl {
  unsigned arrive;  // barrier arrivals so far (grows by the grid size per barrier)
  unsigned fail;    // set by a block that waited too long; stays set
};
// blocks of the persistent kernel that fit on the device at once
hipError_t persistent_max_blocks(int storage, int *blocks);
hipError_t launch_batch_persistent(const KParams *d_tab, const int *d_wave_start, int n_inst, int total_waves,
                                   int storage, int parity, int nsteps, PersistCtl *ctl, unsigned base,
                                   long long wait_ticks, int grid, hipStream_t s);
const char *batch_persistent_kernel_name(int storage);
hipError_t launch_init(const KParams &k, int storage, const double *d_rho, const double *d_ux,
                       const double *d_uy, const double *d_T, hipStream_t s);
// fields (device, double, nx*ny each, nullable) and per-block partial sums
hipError_t launch_moments(const KParams &k, int storage, double *d_rho, double *d_ux, double *d_uy,
                          double *d_T, double *d_partials, int *nblocks_out, hipStream_t s);
int moments_blocks(const KParams &k);
int moments_block_nodes();  // nodes per moments block
// blocks [block0, block0 + nblocks) of launch_moments; fields written from the
// block's first node on (at index 0 for block0), partials at 0 for block0
hipError_t launch_moments_range(const KParams &k, int storage, long long block0, int nblocks, double *d_rho,
                                double *d_ux, double *d_uy, double *d_T, double *d_partials, hipStream_t s);
hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t s);
hipError_t launch_read_state(const KParams &k, int storage, double *d_out, hipStream_t s);

}  // namespace tclbm
