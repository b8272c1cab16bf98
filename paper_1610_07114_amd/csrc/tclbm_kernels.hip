// tclbm_kernels.hip -- gfx950 kernels of the thermal cascaded LBM step.
//
// Data layout (per population buffer): 9 planes of f then 9 planes of h
// (h omitted when athermal), each plane ny rows of `pitch` elements, x fastest.
// A buffer holds post-collision populations at their own node, stored as
// deviations from the rest-state reference of their row; the next step pulls
// them (f_a(x, t+1) = P_a(x - e_a, t)) and adds the per-row shift
// r_a(source row) - r_a(own row).  One step reads 18 and writes 18 values per
// node: one HBM pass.
//
// Step kernel decomposition: one wave64 owns a tile of tile_w consecutive
// columns (plus one halo column on each side, two on the left when x is not
// periodic) and marches upwards through a strip of strip_rows rows.  Each lane
// keeps the pulled populations of the current row in registers together with
// u(1 - theta) of the rows below; the x-derivative of the correction term comes
// from neighbouring lanes through wave shuffles, the y-derivative from the
// register window, so every node's macroscopic values are computed once per
// row visit and the halo costs 2/64 lanes plus two rows per strip.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "tclbm_internal.h"
#include "tclbm_node.h"

namespace tclbm {

namespace {

// D2Q9 order of Section 2: 0 rest, 1 E, 2 N, 3 W, 4 S, 5 NE, 6 NW, 7 SW, 8 SE.
constexpr int kEx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int kEy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int kOpp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

// ---------------------------------------------------------------- storage ---
// 16-bit stores round stochastically and without bias: random bits below the
// target's last place are added to the FP32 pattern, which is then cut.  The
// bits come from a counter-based generator keyed by (step, node, plane), never
// by the value being rounded (bits derived from the value itself made the
// rounding of a slowly varying value a fixed rule with a bias: a thermal
// Couette flow then heated up and blew up).  Round-to-nearest freezes a stored
// value whose per-step change is below half a unit in the last place (with
// it, BF16 Rayleigh-Benard runs never left the conduction state).  Per node,
// the "lowbias32" integer hash (C. Wellons' hash-prospector) of the node
// index and the step; per plane, a multiplicative spread of that word.  The
// result depends only on (step, node, plane), so it is the same for any
// launch shape or batch composition.  The per-plane spread multiplies the
// low 24 bits (a full-rate multiply; a 32-bit one issues at a quarter of the
// rate) and the encoders take the top bits of the product.
__device__ __forceinline__ unsigned sr_node(unsigned node, unsigned step) {
  unsigned x = node ^ (step * 0x9E3779B9u);
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}
__device__ __forceinline__ unsigned sr_word(unsigned hn, int plane) {
  return __umul24(hn ^ ((unsigned)plane * 0x632BE5ABu), 0xEBCA6Bu);  // use the top bits
}
constexpr unsigned kInitStep = 0xFFFFFFFFu;  // generator step of the initial state

// Cache policy of the state's buffer-addressed stores: non-temporal (the
// stored rows are next read in the following step, by then out of L2 for any
// lattice larger than the caches).  Against plain stores, on the same box:
// 8192x4096 FP32 967 -> 931 us, FP16 647 -> 636 us, the 256-lattice batch
// 937 -> 901 us (FP16 638 -> 623 us), 512x256 7.96 -> 7.52 us.
#ifndef TCLBM_STORE_AUX
#define TCLBM_STORE_AUX 2
#endif

template <int S>
struct Store;
template <>
struct Store<kF32> {
  using T = float;
  static __device__ __forceinline__ float ld(const T *p, long long i) { return p[i]; }
  static __device__ __forceinline__ void st(T *p, long long i, float v, unsigned) { p[i] = v; }
  static __device__ __forceinline__ T enc(float v, unsigned) { return v; }
  // buffer addressing: byte offsets within one state buffer (below 4 GiB)
  static __device__ __forceinline__ float ldb(__amdgpu_buffer_rsrc_t r, unsigned vb, unsigned sb) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, vb, sb, 0));
  }
  static __device__ __forceinline__ void stb(__amdgpu_buffer_rsrc_t r, unsigned vb, unsigned sb, float v,
                                             unsigned) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, vb, sb, TCLBM_STORE_AUX);
  }
};
template <>
struct Store<kF64> {
  using T = double;
  static __device__ __forceinline__ double ld(const T *p, long long i) { return p[i]; }
  static __device__ __forceinline__ void st(T *p, long long i, double v, unsigned) { p[i] = v; }
  static __device__ __forceinline__ T enc(double v, unsigned) { return v; }
};
template <>
struct Store<kF16> {
  // IEEE half of the deviation times 2^10.  The power of two scales exactly;
  // it moves half's normal range (6.1e-5 .. 65504) to deviations 6.0e-8 .. 64,
  // so the tiny perturbations from which an instability grows keep 11
  // significant bits instead of falling into subnormals.  |deviation| >= 64
  // overflows to inf (reported as unstable).  Stochastic rounding: random
  // bits below half's last place are added to the FP32 pattern, which is then
  // cut to half precision (exact for normal halfs).
  using T = unsigned short;
  static __device__ __forceinline__ float dec(T b) { return __half2float(__ushort_as_half(b)) * 0x1p-10f; }
  static __device__ __forceinline__ float ld(const T *p, long long i) { return dec(p[i]); }
  // the pulls keep the loaded bits (zero-extended, in a float register) and
  // decode them together with the row shift: one mixed-precision
  // multiply-add, bits x 2^-10 + add
  static __device__ __forceinline__ float ld_raw(const T *p, long long i) { return __uint_as_float(p[i]); }
  static __device__ __forceinline__ float ldb_raw(__amdgpu_buffer_rsrc_t r, unsigned vb, unsigned sb) {
    return __uint_as_float((unsigned)__builtin_amdgcn_raw_buffer_load_b16(r, vb, sb, 0));
  }
  static __device__ __forceinline__ float dec_add(float raw, float add) {
    const _Float16 hv = __builtin_bit_cast(_Float16, (T)__float_as_uint(raw));
    return __builtin_fmaf((float)hv, 0x1p-10f, add);
  }
  static __device__ __forceinline__ void st(T *p, long long i, float v, unsigned rnd) { p[i] = enc(v, rnd); }
  static __device__ __forceinline__ float ldb(__amdgpu_buffer_rsrc_t r, unsigned vb, unsigned sb) {
    return dec(__builtin_amdgcn_raw_buffer_load_b16(r, vb, sb, 0));
  }
  static __device__ __forceinline__ void stb(__amdgpu_buffer_rsrc_t r, unsigned vb, unsigned sb, float v,
                                             unsigned rnd) {
    __builtin_amdgcn_raw_buffer_store_b16(enc(v, rnd), r, vb, sb, TCLBM_STORE_AUX);
  }
  // rnd: 32 random bits, of which the top 13 are used
  static __device__ __forceinline__ T enc(float v, unsigned rnd) {
    unsigned b = __float_as_uint(v * 0x1p10f);
    b = (b + (rnd >> 19)) & ~0x1FFFu;
    return __half_as_ushort(__float2half_rn(__uint_as_float(b)));
  }
};
template <>
struct Store<kBF16> {  // bfloat16: the upper half of the FP32 pattern, stochastic rounding
  using T = unsigned short;
  static __device__ __forceinline__ float dec(T b) { return __bfloat162float(__ushort_as_bfloat16(b)); }
  static __device__ __forceinline__ float ld(const T *p, long long i) { return dec(p[i]); }
  static __device__ __forceinline__ float ld_raw(const T *p, long long i) { return __uint_as_float(p[i]); }
  static __device__ __forceinline__ float ldb_raw(__amdgpu_buffer_rsrc_t r, unsigned vb, unsigned sb) {
    return __uint_as_float((unsigned)__builtin_amdgcn_raw_buffer_load_b16(r, vb, sb, 0));
  }
  static __device__ __forceinline__ float dec_add(float raw, float add) {
    return __uint_as_float(__float_as_uint(raw) << 16) + add;
  }
  static __device__ __forceinline__ void st(T *p, long long i, float v, unsigned rnd) { p[i] = enc(v, rnd); }
  static __device__ __forceinline__ float ldb(__amdgpu_buffer_rsrc_t r, unsigned vb, unsigned sb) {
    return dec(__builtin_amdgcn_raw_buffer_load_b16(r, vb, sb, 0));
  }
  static __device__ __forceinline__ void stb(__amdgpu_buffer_rsrc_t r, unsigned vb, unsigned sb, float v,
                                             unsigned rnd) {
    __builtin_amdgcn_raw_buffer_store_b16(enc(v, rnd), r, vb, sb, TCLBM_STORE_AUX);
  }
  // rnd: 32 random bits, of which the top 16 are used
  static __device__ __forceinline__ T enc(float v, unsigned rnd) {
    const unsigned b = __float_as_uint(v);
    return (T)((b + (rnd >> 16)) >> 16);
  }
};


template <int S>
struct Real {
  using T = float;
};
template <>
struct Real<kF64> {
  using T = double;
};

// ------------------------------------------------------------- utilities ---
// Scheme variants of the march.  M = 0 reads every scheme switch from the
// launch descriptor.  M = 1 is the default thermal scheme with its switches
// fixed at compile time (thermal, with the correction term, continuous h^eq
// moments, the two-rate energy update with its force source, the wall density
// from the known populations, uniform acceleration): its pulls, collision and
// stores are then straight-line code without uniform branches in between.
// M = 2 is the same scheme with buffer-resource addressing: each state buffer
// (below 4 GiB) is one descriptor, a population plane a scalar byte offset and
// a lane's node a 32-bit byte offset, so no 64-bit address is formed per load
// or store.  The host picks it for 16-bit storage when the buffers fit (FP16
// on 8192x4096: 784 -> 697 us); FP32 measured the same either way and keeps
// the global addressing of its LDS pipeline.

struct Flags {
  int thermal, wall_rho;
  bool field;  // per-node acceleration
  bool visc;   // per-node rates from mu = mu0 T/T0
};

template <int M>
__device__ __forceinline__ Flags flags(const KParams &k) {
  if (M >= 1) return Flags{1, 0, false, false};
  return Flags{k.thermal, k.wall_rho, k.axf != nullptr, k.visc_mode == 1};
}

// Launch constants in the compute type: FP32 from the host-rounded copies,
// FP64 from the doubles.

template <class R, int M = 0>
__device__ __forceinline__ Consts<R> make_consts(const KParams &k) {
  Consts<R> c;
  if constexpr (sizeof(R) == 4) {
    const KParams::F32 &f = k.f32;
    c.R_ = f.R;
    c.T0 = f.T0;
    c.b = f.b;
    c.w1 = f.w1;
    c.w2 = f.w2;
    c.w3 = f.w3;
    c.w4 = f.w4;
    c.wh = f.wh;
    c.inv_tau_hf = f.inv_tau_hf;
    c.two_b = f.two_b;
    c.inv_RT0 = f.inv_RT0;
    c.RT0f = f.RT0f;
    c.dRT0 = f.dRT0;
  } else {
    c.R_ = (R)k.R;
    c.T0 = (R)k.T0;
    c.b = (R)k.b;
    c.w1 = (R)k.w1;
    c.w2 = (R)k.w2;
    c.w3 = (R)k.w3;
    c.w4 = (R)k.w4;
    c.wh = (R)k.wh;
    c.inv_tau_hf = (R)k.inv_tau_hf;
    c.two_b = (R)(2.0 / k.b);
    c.inv_RT0 = (R)(1.0 / (k.R * k.T0));
    c.RT0f = (R)(k.R * k.T0);
    c.dRT0 = (R)(k.R * k.T0 - (double)c.RT0f);
  }
  c.thermal = (M >= 1) ? 1 : k.thermal;
  c.correction = (M >= 1) ? 1 : k.correction;
  c.heq_mode = (M >= 1) ? 0 : k.heq_mode;
  c.h_coll = (M >= 1) ? 0 : k.h_coll;
  c.h_force = (M >= 1) ? 1 : k.h_force;
  return c;
}

// Blocks are handed to the 8 XCDs round-robin; renumber them so that each XCD
// receives one contiguous range of logical blocks (neighbouring tiles share
// their halo lines in that XCD's L2).
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int nx = 8;
  int q = nb / nx, r = nb - q * nx;
  int x = b % nx, i = b / nx;
  return (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Column bookkeeping of one lane.
struct Col {
  int xc;         // column whose node this lane evaluates
  int xm, xp;     // source columns of links with e_x = +1 / -1
  unsigned oc, om, op;  // their element offsets within a stored row (state layout)
  unsigned ow;          // the lane's slot in its wave's own block (stores)
  bool wst;             // the lane stores that slot (buffer-addressed stores)
  bool outL, outR;  // those links come from outside (non-periodic x)
};

// Element offset of column x within a stored row of the state (see
// KParams::slots): the slot of the lane that evaluates x, in the block of
// its x tile.
__device__ __forceinline__ unsigned col_off(const KParams &k, int x) {
  const unsigned t = (unsigned)x / (unsigned)k.tile_w;
  return t * (unsigned)k.tstride + (unsigned)k.lane_off + ((unsigned)x - t * (unsigned)k.tile_w);
}

__device__ __forceinline__ Col make_col(const KParams &k, int xl) {
  Col c;
  if (k.bc[kXlo] == kPeriodic) {
    int x = xl % k.nx;
    if (x < 0) x += k.nx;
    c.xc = x;
    c.xm = (x == 0) ? k.nx - 1 : x - 1;
    c.xp = (x == k.nx - 1) ? 0 : x + 1;
    c.outL = false;
    c.outR = false;
  } else {
    int x = xl < 0 ? 0 : (xl >= k.nx ? k.nx - 1 : xl);
    c.xc = x;
    c.outL = (x == 0);
    c.outR = (x == k.nx - 1);
    c.xm = c.outL ? x : x - 1;
    c.xp = c.outR ? x : x + 1;
  }
  c.oc = col_off(k, c.xc);
  c.om = col_off(k, c.xm);
  c.op = col_off(k, c.xp);
  c.ow = c.oc;
  c.wst = true;
  return c;
}

template <class R, int M = 0>
__device__ __forceinline__ void node_accel(const KParams &k, int y, int x, R &ax, R &ay) {
  if (flags<M>(k).field) {
    long long i = (long long)y * k.pitch + x;
    ax = reinterpret_cast<const R *>(k.axf)[i];
    ay = reinterpret_cast<const R *>(k.ayf)[i];
  } else if constexpr (sizeof(R) == 4) {
    ax = k.f32.ax;
    ay = k.f32.ay;
  } else {
    ax = (R)k.ax;
    ay = (R)k.ay;
  }
}

// The per-row tables (references and shifts) are written once at create and
// only read by the step kernels: read them through the constant address space,
// so that row-uniform reads become scalar loads instead of vector loads that
// the compiler must order behind the kernel's own stores.
template <class R>
using ConstPtr = const __attribute__((address_space(4))) R *;

template <class R>
__device__ __forceinline__ ConstPtr<R> const_table(const void *p) {
  return (ConstPtr<R>)(reinterpret_cast<const R *>(p));
}

// Descriptors of the source and destination state buffers (18 planes; the
// buffer addressing is used for the thermal default scheme only).  Reads and
// writes outside the buffer are dropped by the hardware.
template <int S>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t state_rsrc(const void *p, const KParams &k) {
  const unsigned bytes = (unsigned)(18ull * (unsigned long long)k.slots * sizeof(typename Store<S>::T));
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}
template <int S>
__device__ __forceinline__ unsigned plane_bytes(const KParams &k, int a) {
  return (unsigned)((unsigned long long)a * (unsigned long long)k.pstride * sizeof(typename Store<S>::T));
}

template <class R>
__device__ __forceinline__ RowRef<R> row_ref(const KParams &k, const Consts<R> &c, int y) {
  const ConstPtr<R> rr = const_table<R>(k.rowref);
  return make_ref<R>(rr[2 * y], rr[2 * y + 1], c.b, c.heq_mode);
}

// Pull the populations that arrive at (col.xc, y): f_a = P_a(x - e_a).  Links
// from outside a non-periodic side bounce back halfway at rest:
// f_a = P_opp(a)(x) (for WALL rows those values are never used).
// Row geometry of a pull: source rows of the three e_y classes and whether
// links come from outside a non-periodic y side.
struct RowSrc {
  unsigned rm, rc, rp;  // element offsets of rows y-1 (e_y = +1 links), y, y+1
  bool outB, outT;
};

__device__ __forceinline__ RowSrc row_src(const KParams &k, int y) {
  RowSrc r;
  int ym, yp;
  if (k.bc[kYlo] == kPeriodic) {
    ym = (y == 0) ? k.ny - 1 : y - 1;
    yp = (y == k.ny - 1) ? 0 : y + 1;
    r.outB = r.outT = false;
  } else {
    r.outB = (y == 0);
    r.outT = (y == k.ny - 1);
    ym = r.outB ? y : y - 1;
    yp = r.outT ? y : y + 1;
  }
  r.rm = (unsigned)ym * k.rstride;
  r.rc = (unsigned)y * k.rstride;
  r.rp = (unsigned)yp * k.rstride;
  return r;
}

// Phase 1 of a pull: issue the loads of the populations that arrive at
// (col.xc, y), f_a = P_a(x - e_a), as stored (deviations of the source row).
// Links from outside a non-periodic side bounce back halfway at rest,
// f_a = P_opp(a)(x).  Interior tiles and rows take a select-free path.
// What a pull keeps in a register until pull_shift: the value (FP32, FP64),
// or the loaded 16-bit pattern, which pull_shift decodes together with the
// row shift.
template <int S>
struct Pull {
  static constexpr bool kRaw = (S == kF16 || S == kBF16);
  using R = typename Real<S>::T;
  using ST = typename Store<S>::T;
  static __device__ __forceinline__ R ld(const ST *p, long long i) {
    if constexpr (kRaw) return Store<S>::ld_raw(p, i);
    else return Store<S>::ld(p, i);
  }
  static __device__ __forceinline__ R ldb(__amdgpu_buffer_rsrc_t r, unsigned vb, unsigned sb) {
    if constexpr (kRaw) return Store<S>::ldb_raw(r, vb, sb);
    else return Store<S>::ldb(r, vb, sb);
  }
};

template <int S, int M = 0>
__device__ __forceinline__ void pull_issue(const KParams &k, int y, const Col &col,
                                           typename Real<S>::T *f, typename Real<S>::T *h) {
  using ST = typename Store<S>::T;
  const ST *src = reinterpret_cast<const ST *>(k.src);
  const RowSrc rs = row_src(k, y);
  const long long hoff = 9 * k.pstride;
  if constexpr (M == 2) {
    // all offsets are non-negative and inside the buffer
    const __amdgpu_buffer_rsrc_t r = state_rsrc<S>(k.src, k);
    if (k.bc[kXlo] == kPeriodic && !rs.outB && !rs.outT) {
#pragma unroll
      for (int a = 0; a < 9; ++a) {
        const unsigned off = (kEy[a] > 0 ? rs.rm : (kEy[a] < 0 ? rs.rp : rs.rc)) +
                             (kEx[a] > 0 ? col.om : (kEx[a] < 0 ? col.op : col.oc));
        const unsigned vb = off * (unsigned)sizeof(ST);
        f[a] = Pull<S>::ldb(r, vb, plane_bytes<S>(k, a));
        h[a] = Pull<S>::ldb(r, vb, plane_bytes<S>(k, a + 9));
      }
      return;
    }
    // a bounce-back link reads the opposite population of the node itself: the
    // plane may differ per lane, so it goes into the lane's byte offset
#pragma unroll
    for (int a = 0; a < 9; ++a) {
      const unsigned sx = kEx[a] > 0 ? col.om : (kEx[a] < 0 ? col.op : col.oc);
      const bool ox = kEx[a] > 0 ? col.outL : (kEx[a] < 0 ? col.outR : false);
      const unsigned sr = kEy[a] > 0 ? rs.rm : (kEy[a] < 0 ? rs.rp : rs.rc);
      const bool oy = kEy[a] > 0 ? rs.outB : (kEy[a] < 0 ? rs.outT : false);
      const bool bb = ox || oy;
      const int pa = bb ? kOpp[a] : a;
      const unsigned off = bb ? rs.rc + col.oc : sr + sx;
      const unsigned vb = off * (unsigned)sizeof(ST);
      f[a] = Pull<S>::ldb(r, vb + plane_bytes<S>(k, pa), 0u);
      h[a] = Pull<S>::ldb(r, vb + plane_bytes<S>(k, pa + 9), 0u);
    }
    return;
  }
  if (k.bc[kXlo] == kPeriodic && !rs.outB && !rs.outT) {
#pragma unroll
    for (int a = 0; a < 9; ++a) {
      const unsigned off = (kEy[a] > 0 ? rs.rm : (kEy[a] < 0 ? rs.rp : rs.rc)) +
                           (kEx[a] > 0 ? col.om : (kEx[a] < 0 ? col.op : col.oc));
      const ST *base = src + a * k.pstride;
      f[a] = Pull<S>::ld(base, off);
      if (flags<M>(k).thermal) h[a] = Pull<S>::ld(base + hoff, off);
    }
    return;
  }
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    const unsigned sx = kEx[a] > 0 ? col.om : (kEx[a] < 0 ? col.op : col.oc);
    const bool ox = kEx[a] > 0 ? col.outL : (kEx[a] < 0 ? col.outR : false);
    const unsigned sr = kEy[a] > 0 ? rs.rm : (kEy[a] < 0 ? rs.rp : rs.rc);
    const bool oy = kEy[a] > 0 ? rs.outB : (kEy[a] < 0 ? rs.outT : false);
    const bool bb = ox || oy;
    const ST *base = src + (bb ? kOpp[a] : a) * k.pstride;
    const unsigned off = bb ? rs.rc + col.oc : sr + sx;
    f[a] = Pull<S>::ld(base, off);
    if (flags<M>(k).thermal) h[a] = Pull<S>::ld(base + hoff, off);
  }
}

// Phase 2: re-express the pulled deviations against this row's reference,
// adding r_a(source row) - r_a(y) (bounced links stay in the row: the rest
// state is symmetric, no shift).
template <int S, int M = 0>
__device__ __forceinline__ void pull_shift(const KParams &k, int y, const Col &col,
                                           typename Real<S>::T *f, typename Real<S>::T *h) {
  using R = typename Real<S>::T;
  const ConstPtr<R> shF = const_table<R>(k.shiftF) + 9 * y;
  const ConstPtr<R> shH = const_table<R>(k.shiftH) + 9 * y;
  const RowSrc rs = row_src(k, y);
  const bool th = flags<M>(k).thermal;
  if constexpr (Pull<S>::kRaw) {
    // 16-bit patterns: decode every plane, adding the shift (wave-uniform
    // unless the x ends bounce back, where it depends on the lane)
    R af[9], ah[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) {
      const bool keep = kEy[a] != 0 && !(kEy[a] > 0 ? rs.outB : rs.outT);
      af[a] = keep ? shF[a] : R(0);
      ah[a] = (keep && th) ? shH[a] : R(0);
    }
    if (k.bc[kXlo] == kPeriodic) {
#pragma unroll
      for (int a = 0; a < 9; ++a) {
        f[a] = Store<S>::dec_add(f[a], af[a]);
        if (th) h[a] = Store<S>::dec_add(h[a], ah[a]);
      }
    } else {
#pragma unroll
      for (int a = 0; a < 9; ++a) {
        const bool ox = kEx[a] > 0 ? col.outL : (kEx[a] < 0 ? col.outR : false);
        f[a] = Store<S>::dec_add(f[a], ox ? R(0) : af[a]);
        if (th) h[a] = Store<S>::dec_add(h[a], ox ? R(0) : ah[a]);
      }
    }
    return;
  }
  // the table entries are read unconditionally (always in bounds) and applied
  // by selection, so that their loads are not tied to branches
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    if (kEy[a] == 0) continue;
    const R sfa = shF[a];
    const R sha = flags<M>(k).thermal ? shH[a] : R(0);
    const bool ox = kEx[a] > 0 ? col.outL : (kEx[a] < 0 ? col.outR : false);
    const bool oy = kEy[a] > 0 ? rs.outB : rs.outT;
    const bool bb = ox || oy;
    f[a] += bb ? R(0) : sfa;
    if (flags<M>(k).thermal) h[a] += bb ? R(0) : sha;
  }
}

template <int S, int M = 0>
__device__ __forceinline__ void pull(const KParams &k, int y, const Col &col,
                                     typename Real<S>::T *f, typename Real<S>::T *h) {
  pull_issue<S, M>(k, y, col, f, h);
  pull_shift<S, M>(k, y, col, f, h);
}

// Asynchronous pulls (FP32 storage): the loads of a row go straight into a
// per-wave LDS slot (one 64-lane line per plane) with global_load_lds, so the
// wave keeps no registers for loads in flight and computes the previous row
// meanwhile.  The compiler does not track these LDS writes: lds_wait_loads()
// must separate the issue from the reads, and lds_wait_reads() the reads of a
// slot from the next issue into it.
using LdsF = __attribute__((address_space(3))) float;
constexpr int kLdsSlot = 18 * 64;  // floats per slot: 18 planes x 64 lanes

__device__ __forceinline__ void lds_wait_loads() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
__device__ __forceinline__ void lds_wait_reads() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

template <int M>
__device__ __forceinline__ void pull_issue_lds(const KParams &k, int y, const Col &col, LdsF *slot) {
  using GV = __attribute__((address_space(1))) const void;
  using LV = __attribute__((address_space(3))) void;
  const float *src = reinterpret_cast<const float *>(k.src);
  const RowSrc rs = row_src(k, y);
  if constexpr (M == 2) {
    // buffer addressing: one descriptor for the state buffer; plane and row
    // (wave-uniform) in the scalar offset, the lane's column in the vector
    // offset; bounce-back links carry their plane in the lane's offset
    const __amdgpu_buffer_rsrc_t r = state_rsrc<kF32>(k.src, k);
    if (k.bc[kXlo] == kPeriodic && !rs.outB && !rs.outT) {
      const unsigned cm = col.om * 4u, cz = col.oc * 4u, cp = col.op * 4u;
#pragma unroll
      for (int a = 0; a < 9; ++a) {
        const unsigned rb = (kEy[a] > 0 ? rs.rm : (kEy[a] < 0 ? rs.rp : rs.rc)) * 4u;
        const unsigned vb = kEx[a] > 0 ? cm : (kEx[a] < 0 ? cp : cz);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (LV *)(slot + a * 64), 4, vb, plane_bytes<kF32>(k, a) + rb, 0, 0);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (LV *)(slot + (9 + a) * 64), 4, vb,
                                                 plane_bytes<kF32>(k, a + 9) + rb, 0, 0);
      }
      return;
    }
#pragma unroll
    for (int a = 0; a < 9; ++a) {
      const unsigned sx = kEx[a] > 0 ? col.om : (kEx[a] < 0 ? col.op : col.oc);
      const bool ox = kEx[a] > 0 ? col.outL : (kEx[a] < 0 ? col.outR : false);
      const unsigned sr = kEy[a] > 0 ? rs.rm : (kEy[a] < 0 ? rs.rp : rs.rc);
      const bool oy = kEy[a] > 0 ? rs.outB : (kEy[a] < 0 ? rs.outT : false);
      const bool bb = ox || oy;
      const int pa = bb ? kOpp[a] : a;
      const unsigned vb = (bb ? rs.rc + col.oc : sr + sx) * 4u + plane_bytes<kF32>(k, pa);
      __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (LV *)(slot + a * 64), 4, vb, 0u, 0, 0);
      __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (LV *)(slot + (9 + a) * 64), 4, vb + plane_bytes<kF32>(k, 9), 0u,
                                               0, 0);
    }
    return;
  }
  const long long hoff = 9 * k.pstride;
  const bool th = flags<M>(k).thermal;
  if (k.bc[kXlo] == kPeriodic && !rs.outB && !rs.outT) {
#pragma unroll
    for (int a = 0; a < 9; ++a) {
      const unsigned off = (kEy[a] > 0 ? rs.rm : (kEy[a] < 0 ? rs.rp : rs.rc)) +
                           (kEx[a] > 0 ? col.om : (kEx[a] < 0 ? col.op : col.oc));
      const float *base = src + a * k.pstride;
      __builtin_amdgcn_global_load_lds((GV *)(base + off), (LV *)(slot + a * 64), 4, 0, 0);
      if (th) __builtin_amdgcn_global_load_lds((GV *)(base + hoff + off), (LV *)(slot + (9 + a) * 64), 4, 0, 0);
    }
    return;
  }
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    const unsigned sx = kEx[a] > 0 ? col.om : (kEx[a] < 0 ? col.op : col.oc);
    const bool ox = kEx[a] > 0 ? col.outL : (kEx[a] < 0 ? col.outR : false);
    const unsigned sr = kEy[a] > 0 ? rs.rm : (kEy[a] < 0 ? rs.rp : rs.rc);
    const bool oy = kEy[a] > 0 ? rs.outB : (kEy[a] < 0 ? rs.outT : false);
    const bool bb = ox || oy;
    const float *base = src + (bb ? kOpp[a] : a) * k.pstride;
    const unsigned off = bb ? rs.rc + col.oc : sr + sx;
    __builtin_amdgcn_global_load_lds((GV *)(base + off), (LV *)(slot + a * 64), 4, 0, 0);
    if (th) __builtin_amdgcn_global_load_lds((GV *)(base + hoff + off), (LV *)(slot + (9 + a) * 64), 4, 0, 0);
  }
}


// Populations of a WALL row node by non-equilibrium extrapolation from the
// adjacent fluid node (I):
// X(x_b) = X^eq(rho_w, u_w, T_w) + [X(x_f) - X^eq(rho_f, u_f, T_f)],
// in deviations: d_w = (f^eq_w - r_w) - (f^eq_I - r_I) + d_I.  The stored f is
// the transformed fbar = f - S/2 - C/2, whose equilibrium part is f^eq - S/2
// (at each node's own rho, u and a); C, without mass or momentum, stays in the
// extrapolated non-equilibrium part.
// On entry dw holds the deviations pulled at the wall node; those that came
// from the fluid and the tangential ones fix rho_w (default reading): with the
// rest reference, k0 + 2 k_in = rho_r + the same combination of deviations.
template <class R, int M = 0>
__device__ __forceinline__ void wall_node(const KParams &k, const Consts<R> &c, int side, const RowRef<R> &qw,
                                          const RowRef<R> &qI, const R *dI, const R *gI, const Macro<R> &mI,
                                          R axI, R ayI, R axW, R ayW, R dthw, R *dw, R *gw) {
  const R thw = qw.th + dthw;
  const R aI_n = (side == kYlo) ? -ayI : ayI;
  const R aW_n = (side == kYlo) ? -ayW : ayW;
  R uwx, uwy;
  if constexpr (sizeof(R) == 4) {
    uwx = k.f32.wall_ux[side];
    uwy = k.f32.wall_uy[side];
  } else {
    uwx = (R)k.wall_ux[side];
    uwy = (R)k.wall_uy[side];
  }
  const Flags fl = flags<M>(k);
  R drw;
  if (fl.wall_rho == 1) {
    drw = mI.drho + (qI.rho - qw.rho);
  } else if (fl.wall_rho == 2) {
    drw = (mI.rho * mI.th + mI.rho * aI_n) / thw - qw.rho;
  } else {
    // bottom: links from the fluid are e_y = -1 (4, 7, 8); top: e_y = +1 (2, 5, 6)
    const R D = (dw[0] + dw[1] + dw[3]) +
                R(2) * ((side == kYlo) ? (dw[4] + dw[7] + dw[8]) : (dw[2] + dw[5] + dw[6]));
    const R un = (side == kYlo) ? -uwy : uwy;
    const R den = R(1) + un - R(0.5) * aW_n;
    drw = (D - qw.rho * (un - R(0.5) * aW_n)) / den;
  }
  R ew[9], ef[9], sw[9], sf[9];
  feq_dev(qw, drw, uwx, uwy, dthw, ew);
  feq_dev(qI, mI.drho, mI.ux, mI.uy, mI.dth, ef);
  source9(qw.rho + drw, uwx, uwy, axW, ayW, sw);
  source9(mI.rho, mI.ux, mI.uy, axI, ayI, sf);
#pragma unroll
  for (int a = 0; a < 9; ++a) dw[a] = (ew[a] - ef[a]) - R(0.5) * (sw[a] - sf[a]) + dI[a];
  if (fl.thermal) {
    const R Ew = R(0.5) * (c.b * thw + uwx * uwx + uwy * uwy);
    const R sgw = drw * Ew + qw.rho * (R(0.5) * c.b * dthw + R(0.5) * (uwx * uwx + uwy * uwy));
    heq_dev(c, qw, drw, uwx, uwy, dthw, sgw, ew);
    heq_dev(c, qI, mI.drho, mI.ux, mI.uy, mI.dth, mI.sg, ef);
#pragma unroll
    for (int a = 0; a < 9; ++a) gw[a] = ew[a] - ef[a] + gI[a];
  }
}

template <class R>
struct RowState {
  R f[9], h[9];  // deviations from the row reference
  RowRef<R> q;
  Macro<R> m;
  R qx, qy;  // u (1 - theta)
};

template <class R, int M = 0>
__device__ __forceinline__ void finish(const KParams &k, const Consts<R> &c, int y, int xc, RowState<R> &s) {
  R ax, ay;
  node_accel<R, M>(k, y, xc, ax, ay);
  s.m = macros(c, s.q, s.f, s.h, ax, ay);
  R om = one_minus_theta(c, s.q.th, s.m.dth);
  s.qx = s.m.ux * om;
  s.qy = s.m.uy * om;
}

__device__ __forceinline__ bool is_wall_row(const KParams &k, int y) {
  return (y == 0 && is_wall_kind(k.bc[kYlo])) || (y == k.ny - 1 && is_wall_kind(k.bc[kYhi]));
}

// State of row y (not a WALL row): pull and evaluate.
template <int S, int M = 0>
__device__ __forceinline__ void get_row(const KParams &k, const Consts<typename Real<S>::T> &c, int y,
                                        const Col &col, RowState<typename Real<S>::T> &s) {
  s.q = row_ref(k, c, y);
  pull<S, M>(k, y, col, s.f, s.h);
  finish<typename Real<S>::T, M>(k, c, y, col.xc, s);
}

// State of row y (not a WALL row) from a slot whose loads have landed.
template <int M>
__device__ __forceinline__ void get_row_lds(const KParams &k, const Consts<float> &c, int y, const Col &col,
                                            const LdsF *slot, int lane, RowState<float> &s) {
  s.q = row_ref(k, c, y);
  const bool th = flags<M>(k).thermal;
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    s.f[a] = slot[a * 64 + lane];
    if (th) s.h[a] = slot[(9 + a) * 64 + lane];
  }
  pull_shift<kF32, M>(k, y, col, s.f, s.h);
  finish<float, M>(k, c, y, col.xc, s);
}

// State of the WALL row y whose fluid neighbour state is `in`.  issued: the
// loads of its known populations were already issued into s.f, s.h (by
// pull_issue; needed only when its density comes from them).
template <int S, int M = 0>
__device__ __forceinline__ void get_wall_row(const KParams &k, const Consts<typename Real<S>::T> &c, int y,
                                             const Col &col, const RowState<typename Real<S>::T> &in,
                                             RowState<typename Real<S>::T> &s, bool issued = false) {
  using R = typename Real<S>::T;
  const int side = (y == 0) ? kYlo : kYhi;
  const int yf = (y == 0) ? 1 : y - 1;
  s.q = row_ref(k, c, y);
  if (flags<M>(k).wall_rho == 0) {
    if (!issued) pull_issue<S, M>(k, y, col, s.f, s.h);
    pull_shift<S, M>(k, y, col, s.f, s.h);
  }
  R axI, ayI, axW, ayW;
  node_accel<R, M>(k, yf, col.xc, axI, ayI);
  node_accel<R, M>(k, y, col.xc, axW, ayW);
  // wall temperature as a deviation from the wall row's reference; the O(1)
  // parts are formed in double on the host (wall_dth)
  R dthw = c.R_ * c.T0 - s.q.th;
  if (flags<M>(k).thermal) {
    if constexpr (sizeof(R) == 4) dthw = k.f32.wall_dth[side];
    else dthw = (R)k.wall_dth[side];
  }
  if (flags<M>(k).thermal && k.bc[side] == kWallAdiabatic) {
    // zero normal temperature gradient to second order, -3 T_w + 4 T_1 - T_2 = 0,
    // with the row two inside the wall evaluated here (ny >= 4: a fluid row)
    RowState<R> two;
    get_row<S, M>(k, c, (y == 0) ? 2 : y - 2, col, two);
    dthw += (R(4) * in.m.dth - two.m.dth) * (R(1) / R(3));
  }
  wall_node<R, M>(k, c, side, s.q, in.q, in.f, in.h, in.m, axI, ayI, axW, ayW, dthw, s.f, s.h);
  finish<R, M>(k, c, y, col.xc, s);
}

template <class R>
__device__ __forceinline__ R shfl_dn(R v, int d) {
  return __shfl_down(v, d, 64);
}
template <class R>
__device__ __forceinline__ R shfl_up(R v, int d) {
  return __shfl_up(v, d, 64);
}

// d/dx[u_x (1 - theta)] at this lane's node: central difference with the
// neighbouring lanes, one-sided second order on a non-periodic edge.  Every
// lane of the wave must call it (shuffles).
template <class R>
__device__ __forceinline__ R ddx(const KParams &k, R q, int xl) {
  R qp = shfl_dn(q, 1), qm = shfl_up(q, 1);
  if (k.bc[kXlo] == kPeriodic) return R(0.5) * (qp - qm);
  R qpp = shfl_dn(q, 2), qmm = shfl_up(q, 2);
  if (xl == 0) return R(0.5) * (R(-3) * q + R(4) * qp - qpp);
  if (xl == k.nx - 1) return R(0.5) * (R(3) * q - R(4) * qm + qmm);
  return R(0.5) * (qp - qm);
}

// Collide the current row and store it.
template <int S, int M = 0>
__device__ __forceinline__ void collide_store(const KParams &k, const Consts<typename Real<S>::T> &c, int y,
                                              const Col &col, bool store, const RowState<typename Real<S>::T> &s,
                                              typename Real<S>::T Dy, int xl, unsigned step) {
  using R = typename Real<S>::T;
  using ST = typename Store<S>::T;
  const R Dx = ddx<R>(k, s.qx, xl);
  R ax, ay;
  node_accel<R, M>(k, y, col.xc, ax, ay);
  R P[9], Q[9];
  Consts<R> cn = c;
  if (flags<M>(k).visc) {
    // mu = mu0 T/T0 in Eq. (29), p = rho R T: 1/w1 = mu0/(rho R T0) + 1/2; w_h and
    // tau_hf follow from that w1 at constant Pr
    const R mp = (R)k.mu0_RT0 / s.m.rho;
    cn.w1 = R(1) / (mp + R(0.5));
    cn.wh = R(1) / (mp / (R)k.Pr + R(0.5));
    cn.inv_tau_hf = cn.w1 * ((R)k.Pr - R(1));
  }
  collide<R, (S == kF32 || S == kF64)>(cn, s.q, s.f, s.h, s.m, Dx, Dy, ax, ay, P, Q);
  // buffer-addressed stores cover every 128-byte line of the wave's block
  // that holds one of its nodes (the halo lanes and lanes past nx write
  // slots that are never read), so no store request fills a line in part;
  // the others store the tile's own nodes
  if (M == 2 ? !col.wst : !store) return;
  ST *dst = reinterpret_cast<ST *>(k.dst);
  // the node's number (y * pitch + x) keys the rounding generator; its
  // address follows the state layout
  const unsigned node = (unsigned)y * k.pitch + (unsigned)col.xc;
  const unsigned hn = (S == kF16 || S == kBF16) ? sr_node(node, step) : 0u;
  const unsigned own = (unsigned)y * k.rstride + col.oc;
  if constexpr (M == 2) {
    // row and plane in the scalar offset, the lane's slot in the vector offset
    const __amdgpu_buffer_rsrc_t r = state_rsrc<S>(k.dst, k);
    const unsigned vb = col.ow * (unsigned)sizeof(ST);
    const unsigned rb = (unsigned)y * k.rstride * (unsigned)sizeof(ST);
#pragma unroll
    for (int a = 0; a < 9; ++a) {
      Store<S>::stb(r, vb, plane_bytes<S>(k, a) + rb, P[a], sr_word(hn, a));
      Store<S>::stb(r, vb, plane_bytes<S>(k, a + 9) + rb, Q[a], sr_word(hn, a + 9));
    }
    return;
  }
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    (dst + a * k.pstride)[own] = Store<S>::enc(P[a], sr_word(hn, a));
    if (flags<M>(k).thermal) (dst + (a + 9) * k.pstride)[own] = Store<S>::enc(Q[a], sr_word(hn, a + 9));
  }
}

}  // namespace

// ------------------------------------------------------------ step kernel ---
// Build-time switches of the step kernels (defaults chosen by measurement on
// MI355X; the others exist for A/B comparisons):
//   TCLBM_STEP_WAVES          waves per block (4)
//   TCLBM_LDS_PULL            FP32 rows pulled one row ahead into LDS (1)
//   TCLBM_SCHEME_SPECIAL      compile-time instantiation of the default scheme (1)
//   TCLBM_BUFFER_ADDR         buffer-resource addressing for it, 16-bit storage (1)
//   TCLBM_F32_WAVES_PER_EU    occupancy cap of the FP32 step kernels (3)
//   TCLBM_WAVES_PER_EU        occupancy cap of the 16-bit step kernels (3)
//   TCLBM_BATCH_WAVES_PER_EU  occupancy cap of the 16-bit batch kernels (3)
//   TCLBM_BATCH32_WAVES_PER_EU  occupancy cap of the FP32 batch kernels (3)
//   TCLBM_ROW_GROUP           rows per block for FP32 lattices of single-row
//                             strips, neighbours' u_y(1 - theta) shared in LDS
//                             (4; 1: one independent wave per row)
//   TCLBM_BATCH_ALT_MARCH     batch kernels: odd interior strips march
//                             downwards (1)
#ifndef TCLBM_STEP_WAVES
#define TCLBM_STEP_WAVES 4
#endif
constexpr int kStepWaves = TCLBM_STEP_WAVES;

#ifndef TCLBM_LDS_PULL
#define TCLBM_LDS_PULL 1
#endif
#ifndef TCLBM_SCHEME_SPECIAL
#define TCLBM_SCHEME_SPECIAL 1
#endif
#ifndef TCLBM_BUFFER_ADDR
#define TCLBM_BUFFER_ADDR 1
#endif
#ifndef TCLBM_F32_WAVES_PER_EU
#define TCLBM_F32_WAVES_PER_EU 3
#endif
#if TCLBM_F32_WAVES_PER_EU > 0
#define TCLBM_F32_OCC __attribute__((amdgpu_waves_per_eu(TCLBM_F32_WAVES_PER_EU, TCLBM_F32_WAVES_PER_EU)))
#else
#define TCLBM_F32_OCC
#endif
#ifndef TCLBM_WAVES_PER_EU
#define TCLBM_WAVES_PER_EU 3
#endif
#if TCLBM_WAVES_PER_EU > 0
#define TCLBM_OCC __attribute__((amdgpu_waves_per_eu(TCLBM_WAVES_PER_EU, TCLBM_WAVES_PER_EU)))
#else
#define TCLBM_OCC
#endif
#ifndef TCLBM_BATCH_WAVES_PER_EU
#define TCLBM_BATCH_WAVES_PER_EU 3
#endif
#ifndef TCLBM_ROW_GROUP
#define TCLBM_ROW_GROUP 4
#endif
#ifndef TCLBM_BATCH_ALT_MARCH
#define TCLBM_BATCH_ALT_MARCH 1
#endif
constexpr bool kBatchAlt = TCLBM_BATCH_ALT_MARCH;
constexpr int kRowGroup = TCLBM_ROW_GROUP;
#if TCLBM_BATCH_WAVES_PER_EU > 0
#define TCLBM_BATCH_OCC __attribute__((amdgpu_waves_per_eu(TCLBM_BATCH_WAVES_PER_EU, TCLBM_BATCH_WAVES_PER_EU)))
#else
#define TCLBM_BATCH_OCC
#endif
// occupancy cap of the FP32 batch kernels (0: none).  Their default-scheme
// instantiations fit in 128 registers, but 4 waves per SIMD measured slower
// than 3 (256-lattice batch 1150 vs 1086 us, 8192x4096 alone 1266 vs
// 1179 us): the kernels are bound by their memory access pattern, and more
// waves in flight only spread it over more rows.
#ifndef TCLBM_BATCH32_WAVES_PER_EU
#define TCLBM_BATCH32_WAVES_PER_EU 3
#endif
#if TCLBM_BATCH32_WAVES_PER_EU > 0
#define TCLBM_BATCH32_OCC \
  __attribute__((amdgpu_waves_per_eu(TCLBM_BATCH32_WAVES_PER_EU, TCLBM_BATCH32_WAVES_PER_EU)))
#else
#define TCLBM_BATCH32_OCC
#endif

// A lane's own-block slot and whether it stores it under buffer addressing:
// the lanes of every 128-byte line (32 slots of FP32, 64 of 16-bit storage)
// that holds one of the tile's nodes.
template <int S>
__device__ __forceinline__ void own_slot(const KParams &k, int xt, int lane, Col &col) {
  col.ow = (unsigned)xt * (unsigned)k.tstride + (unsigned)lane;
  const int valid = min(k.tile_w, k.nx - xt * k.tile_w);
  const int last = k.lane_off + valid - 1;
  constexpr int sh = (sizeof(typename Store<S>::T) == 2) ? 6 : 5;
  col.wst = (lane >> sh) <= (last >> sh);
}

// The march of one wave over its (x tile, strip) of lattice k.
template <int S, int M = 0, bool Alt = false>
__device__ __forceinline__ void march(const KParams &k, int wave, int lane, LdsF *lds) {
  using R = typename Real<S>::T;
  const int strip = wave / k.n_xtiles;
  const int xt = wave - strip * k.n_xtiles;
  const int r0 = strip * k.strip_rows;
  const int r1 = min(r0 + k.strip_rows, k.ny);
  const int xl = xt * k.tile_w - k.lane_off + lane;
  const bool store = (lane >= k.lane_off) && (lane < k.lane_off + k.tile_w) && (xl < k.nx);
  Col col = make_col(k, xl);
  own_slot<S>(k, xt, lane, col);
  const Consts<R> c = make_consts<R, M>(k);
  const bool yper = (k.bc[kYlo] == kPeriodic);
  const int ny = k.ny;

  RowState<R> cur, nxt;
  R qy_m1 = R(0), qy_m2 = R(0);
  int j;
  // step number for the 16-bit rounding generator; the lattice's first wave
  // advances the counter for the next launch (the other cell: no race)
  constexpr bool k16 = (S == kF16 || S == kBF16);
  const unsigned step = k16 ? k.ctr[k.par] : 0u;
  if (k16 && wave == 0 && lane == 0) k.ctr[1 - k.par] = step + 1u;
  if (r1 - r0 == 1 && (yper || (r0 >= 3 && r0 <= ny - 4))) {
    // single-row strip away from the edges (small lattices): the three rows it
    // needs are independent, so all their loads are issued before any is used
    const int ya = (r0 == 0) ? ny - 1 : r0 - 1, yb = (r0 == ny - 1) ? 0 : r0 + 1;
    RowState<R> lo, hi;
    pull_issue<S, M>(k, ya, col, lo.f, lo.h);
    pull_issue<S, M>(k, r0, col, cur.f, cur.h);
    pull_issue<S, M>(k, yb, col, hi.f, hi.h);
    lo.q = row_ref(k, c, ya);
    pull_shift<S, M>(k, ya, col, lo.f, lo.h);
    finish<R, M>(k, c, ya, col.xc, lo);
    hi.q = row_ref(k, c, yb);
    pull_shift<S, M>(k, yb, col, hi.f, hi.h);
    finish<R, M>(k, c, yb, col.xc, hi);
    cur.q = row_ref(k, c, r0);
    pull_shift<S, M>(k, r0, col, cur.f, cur.h);
    finish<R, M>(k, c, r0, col.xc, cur);
    collide_store<S, M>(k, c, r0, col, store, cur, R(0.5) * (hi.qy - lo.qy), xl, step);
    return;
  }
  // Alt (the batch kernels): an odd strip whose rows and halo rows are all
  // pulled fluid rows marches downwards (d = -1).  It then pulls the rows it
  // shares with each neighbouring strip at the same end of the march as that
  // neighbour does, so the second pull of a shared row finds it in L2 (the
  // 256-lattice batch: counted reads 1.41x -> 1.07x of the algorithmic
  // bytes, 902 -> 895 us per step).  On one large lattice the strips that
  // share a row run too far apart for that, and it measured slower (8192x4096
  // 929 -> 945 us).  Each row's collision depends only on its own and its two
  // neighbouring rows, so the result does not depend on the direction.
  const bool down = Alt && (strip & 1) && r1 - r0 >= 2 && (yper || (r0 >= 2 && r1 <= ny - 2));
  const int d = down ? -1 : 1;
  if (down) {
    get_row<S, M>(k, c, r1 == ny ? 0 : r1, col, nxt);  // row above the strip
    qy_m1 = nxt.qy;
    get_row<S, M>(k, c, r1 - 1, col, cur);
    j = r1 - 1;
  } else if (!yper && r0 == 0) {
    // bottom edge: row 0 needs u(1-theta) of rows 1 and 2 (one-sided difference)
    get_row<S, M>(k, c, 1, col, nxt);                       // row 1 (ny >= 3: a fluid row)
    RowState<R> two;
    if (is_wall_row(k, 2)) get_wall_row<S, M>(k, c, 2, col, nxt, two);
    else get_row<S, M>(k, c, 2, col, two);
    if (is_wall_row(k, 0)) get_wall_row<S, M>(k, c, 0, col, nxt, cur);
    else get_row<S, M>(k, c, 0, col, cur);
    const R Dy = R(0.5) * (R(-3) * cur.qy + R(4) * nxt.qy - two.qy);
    collide_store<S, M>(k, c, 0, col, store, cur, Dy, xl, step);
    qy_m1 = cur.qy;
    cur = nxt;
    j = 1;
  } else {
    const int ya = yper ? (r0 == 0 ? ny - 1 : r0 - 1) : r0 - 1;  // row below the strip
    if (!yper && ya == 0 && is_wall_row(k, 0)) {
      get_row<S, M>(k, c, r0, col, cur);
      get_wall_row<S, M>(k, c, 0, col, cur, nxt);
      qy_m1 = nxt.qy;
    } else {
      get_row<S, M>(k, c, ya, col, nxt);
      qy_m1 = nxt.qy;
      if (!yper && r1 == ny && r0 >= 2) {
        // strip holds the top edge: also u(1-theta) two rows below its start
        RowState<R> low;
        if (r0 - 2 == 0 && is_wall_row(k, 0)) get_wall_row<S, M>(k, c, 0, col, nxt, low);
        else get_row<S, M>(k, c, r0 - 2, col, low);
        qy_m2 = low.qy;
      }
      if (is_wall_row(k, r0)) get_wall_row<S, M>(k, c, r0, col, nxt, cur);
      else get_row<S, M>(k, c, r0, col, cur);
    }
    j = r0;
  }

  // FP32 storage pipelines the pulls through two LDS slots: the row the next
  // iteration needs is loaded while this one collides.
  constexpr bool kAsync = (S == kF32) && TCLBM_LDS_PULL;
  bool pending = false;  // the loads of the march's next row are in lds slot `slot`
  int slot = 0;
  // the row after y in the march's direction (periodic wrap)
  const auto step_row = [&](int y) { return d > 0 ? (y == ny - 1 ? 0 : y + 1) : (y == 0 ? ny - 1 : y - 1); };
  const auto next_pulled = [&](int jj) {
    // the row after jj is pulled (not derived) by iteration jj of this strip
    if (d < 0) return jj >= r0;
    if (jj >= r1 || (!yper && jj == ny - 1)) return false;
    const int y1 = (jj == ny - 1) ? 0 : jj + 1;
    return yper || !is_wall_row(k, y1);
  };
  if (kAsync && next_pulled(j)) {
    pull_issue_lds<M>(k, step_row(j), col, lds);
    pending = true;
  }
  const int jend = d > 0 ? r1 : r0 - 1;
  for (; j != jend; j += d) {
    if (!yper && j == ny - 1) {  // top edge: one-sided difference with the rows below
      const R Dy = R(0.5) * (R(3) * cur.qy - R(4) * qy_m1 + qy_m2);
      collide_store<S, M>(k, c, j, col, store, cur, Dy, xl, step);
      break;
    }
    const int yn = step_row(j);
    if constexpr (kAsync) {
      if (pending) {
        lds_wait_loads();
        get_row_lds<M>(k, c, yn, col, lds + slot * kLdsSlot, lane, nxt);
      } else if (!yper && is_wall_row(k, yn)) {
        get_wall_row<S, M>(k, c, yn, col, cur, nxt);
      } else {
        get_row<S, M>(k, c, yn, col, nxt);
      }
      pending = false;
      if (next_pulled(j + d)) {
        // the other slot was last read an iteration ago
        lds_wait_reads();
        slot ^= 1;
        pull_issue_lds<M>(k, step_row(yn), col, lds + slot * kLdsSlot);
        pending = true;
      }
    } else {
      if (!yper && is_wall_row(k, yn)) get_wall_row<S, M>(k, c, yn, col, cur, nxt);
      else get_row<S, M>(k, c, yn, col, nxt);
    }
    // central difference, row above minus row below, whichever way the march goes
    const R Dy = R(0.5) * (d > 0 ? nxt.qy - qy_m1 : qy_m1 - nxt.qy);
    collide_store<S, M>(k, c, j, col, store, cur, Dy, xl, step);
    qy_m2 = qy_m1;
    qy_m1 = cur.qy;
    cur = nxt;
  }
}

// W waves per block: kStepWaves, or 1 for default-scheme lattices of single-row
// strips when row groups are switched off (their 2-3 waves per SIMD then spread
// evenly over the CUs: 512x256 10.4 -> 10.2 us).
template <int S, int M, int W>
__global__ __launch_bounds__(64 * W) TCLBM_F32_OCC void step_kernel(KParams k) {
  // wave-uniform: rows, strips and table reads stay scalar
  const int wave = __builtin_amdgcn_readfirstlane(xcd_block(blockIdx.x, gridDim.x) * W + (threadIdx.x >> 6));
  if (wave >= k.n_xtiles * k.n_strips) return;  // whole wave leaves together
  __shared__ float lds[W * 2 * kLdsSlot];
  march<S, M>(k, wave, threadIdx.x & 63, (LdsF *)(lds + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) * 2 * kLdsSlot));
}
// Lattices of single-row strips, G consecutive rows of one tile column per
// block, one wave per row.  A row's collision needs u_y(1 - theta) of the rows
// above and below it (central difference; one-sided at a non-periodic edge
// row), so a lone wave pulls three rows to collide one.  In a group every wave
// pulls and evaluates its own row and the waves read their neighbours' values
// from LDS: (G + 2) / G pulls per collided row instead of 3.  The first and
// last wave also pull the row just outside the group; in the group that holds
// a non-periodic edge row, the edge row's wave pulls the row next to it
// instead, which a WALL edge row is derived from (so the wall row is derived
// once per group, not by two waves).  The arithmetic per node is that of the
// lone-wave path, value for value.  Groups that overhang the lattice, or whose
// outside rows are WALL rows, run every row as a lone wave; the choice is the
// same for the whole block, so either all G waves meet the barrier or none does.
// E: the lattice has non-periodic y sides (edge groups exist); lattices
// periodic in y take the instantiation without the edge roles.
template <int S, int M, int G, bool E>
__device__ __forceinline__ void row_group(const KParams &k, int grp, int xt, int w, int lane,
                                          LdsF *qy_share, LdsF *lds) {
  static_assert(S == kF32, "row groups serve FP32 storage");
  using R = typename Real<S>::T;
  const int ny = k.ny;
  const int g0 = grp * G, y = g0 + w;
  const bool yper = !E || (k.bc[kYlo] == kPeriodic);  // E = false is launched for periodic y only
  // 1: central differences only; 2: holds the bottom row; 3: holds the top row
  int kind = 0;
  if (g0 + G <= ny) {
    if (yper || (g0 >= 1 && g0 + G <= ny - 1 && !is_wall_row(k, g0 - 1) && !is_wall_row(k, g0 + G))) kind = 1;
    else if (E && G >= 3 && g0 == 0 && G <= ny - 2) kind = 2;  // one-sided: rows 1 and 2 in the group
    else if (E && G >= 3 && g0 + G == ny && g0 >= 1 && !is_wall_row(k, g0 - 1)) kind = 3;
  }
  if (kind == 0) {
    if (y < ny) march<S, M>(k, y * k.n_xtiles + xt, lane, lds);  // strip y of one row
    return;
  }
  const int xl = xt * k.tile_w - k.lane_off + lane;
  const bool store = (lane >= k.lane_off) && (lane < k.lane_off + k.tile_w) && (xl < k.nx);
  Col col = make_col(k, xl);
  own_slot<S>(k, xt, lane, col);
  const Consts<R> c = make_consts<R, M>(k);
  // wave-uniform roles
  const bool edge_lo = E && (kind == 2 && w == 0), edge_hi = E && (kind == 3 && w == G - 1);
  const bool halo_lo = (w == 0 && kind != 2), halo_hi = (w == G - 1 && kind != 3);
  const bool wall = E && (edge_lo || edge_hi) && is_wall_row(k, y);
  const bool other = halo_lo || halo_hi || wall;  // a second row: outside the group, or the wall's neighbour
  const int yo = halo_lo ? (y == 0 ? ny - 1 : y - 1) : halo_hi ? (y == ny - 1 ? 0 : y + 1) : (edge_lo ? 1 : ny - 2);
  RowState<R> cur, out;
  if (!wall || flags<M>(k).wall_rho == 0) pull_issue<S, M>(k, y, col, cur.f, cur.h);
  if (other) pull_issue<S, M>(k, yo, col, out.f, out.h);
  if (other) {
    out.q = row_ref(k, c, yo);
    pull_shift<S, M>(k, yo, col, out.f, out.h);
    finish<R, M>(k, c, yo, col.xc, out);
  }
  if (E && wall) {
    get_wall_row<S, M>(k, c, y, col, out, cur, true);
  } else {
    cur.q = row_ref(k, c, y);
    pull_shift<S, M>(k, y, col, cur.f, cur.h);
    finish<R, M>(k, c, y, col.xc, cur);
  }
  qy_share[(w + 1) * 64 + lane] = cur.qy;  // slot s: row g0 + s - 1
  if (halo_lo) qy_share[lane] = out.qy;
  if (halo_hi) qy_share[(G + 1) * 64 + lane] = out.qy;
  __syncthreads();
  R Dy;
  if (E && edge_lo) {
    Dy = R(0.5) * (R(-3) * cur.qy + R(4) * qy_share[2 * 64 + lane] - qy_share[3 * 64 + lane]);
  } else if (E && edge_hi) {
    Dy = R(0.5) * (R(3) * cur.qy - R(4) * qy_share[(G - 1) * 64 + lane] + qy_share[(G - 2) * 64 + lane]);
  } else {
    const R lo = qy_share[w * 64 + lane], hi = qy_share[(w + 2) * 64 + lane];
    Dy = R(0.5) * (hi - lo);
  }
  collide_store<S, M>(k, c, y, col, store, cur, Dy, xl, 0u);
}

template <int S, int M, int G, bool E>
__global__ __launch_bounds__(64 * G) TCLBM_F32_OCC void row_group_kernel(KParams k) {
  const int b = xcd_block(blockIdx.x, gridDim.x);  // uniform: one group and tile per block
  const int grp = b / k.n_xtiles;
  const int xt = b - grp * k.n_xtiles;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  __shared__ float lds[G * 2 * kLdsSlot];
  __shared__ float qy_share[(G + 2) * 64];
  row_group<S, M, G, E>(k, grp, xt, w, threadIdx.x & 63, (LdsF *)qy_share, (LdsF *)(lds + w * 2 * kLdsSlot));
}

// 16-bit storage: the stochastic-rounding stores need a few more registers;
// capped to keep 3 waves per SIMD (a handful of spills)
template <int S, int M>
__global__ __launch_bounds__(64 * kStepWaves) TCLBM_OCC void step_kernel_16(KParams k) {
  const int wave = __builtin_amdgcn_readfirstlane(xcd_block(blockIdx.x, gridDim.x) * kStepWaves + (threadIdx.x >> 6));
  if (wave >= k.n_xtiles * k.n_strips) return;
  march<S, M>(k, wave, threadIdx.x & 63, nullptr);
}
template <int M>
__global__ __launch_bounds__(64 * kStepWaves) void step_kernel_f64(KParams k) {
  const int wave = __builtin_amdgcn_readfirstlane(xcd_block(blockIdx.x, gridDim.x) * kStepWaves + (threadIdx.x >> 6));
  if (wave >= k.n_xtiles * k.n_strips) return;
  march<kF64, M>(k, wave, threadIdx.x & 63, nullptr);
}

// Batched step: one launch advances every lattice of a table by one step.
// wave_start[i] is the first global wave of instance i (prefix sum of
// n_xtiles * n_strips, wave_start[n] = total); waves of one instance are
// contiguous, in table order (largest lattices first).

// MB = 1 or 2: every member runs the default scheme (the host checked), so
// only that instantiation (2: with buffer addressing, every member fits) is
// compiled in; MB = 0: chosen per member.
template <int S, int MB>
__device__ __forceinline__ void batch_body(const KParams *__restrict__ tab, const int *__restrict__ wave_start,
                                           int n_inst, int parity, int lblock) {
  const int wave = __builtin_amdgcn_readfirstlane(lblock * kStepWaves + (threadIdx.x >> 6));
  if (wave >= wave_start[n_inst]) return;
  int lo = 0, hi = n_inst - 1;  // last instance whose start <= wave
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (wave_start[mid] <= wave) lo = mid;
    else hi = mid - 1;
  }
  lo = __builtin_amdgcn_readfirstlane(lo);
  // the table holds each member twice: entries [0, n) for even steps and
  // [n, 2n) with source and destination swapped for odd steps; the
  // descriptor is read in place (like a kernel argument), not copied
  const KParams &k = tab[parity * n_inst + lo];
  LdsF *lds = nullptr;
  if constexpr (S == kF32) {
    __shared__ float buf[kStepWaves * 2 * kLdsSlot];
    lds = (LdsF *)(buf + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) * 2 * kLdsSlot);
  }
  if constexpr (MB >= 1) {
    march<S, MB, kBatchAlt>(k, wave - wave_start[lo], threadIdx.x & 63, lds);
  } else {
    if (TCLBM_SCHEME_SPECIAL && default_scheme(k))
      march<S, 1, kBatchAlt>(k, wave - wave_start[lo], threadIdx.x & 63, lds);
    else march<S, 0, kBatchAlt>(k, wave - wave_start[lo], threadIdx.x & 63, lds);
  }
}

// 32- and 16-bit storage may take a register cap (occupancy); FP64 never does
template <int S, int MB>
__global__ __launch_bounds__(64 * kStepWaves) TCLBM_BATCH_OCC void batch_step_kernel(
    const KParams *__restrict__ tab, const int *__restrict__ wave_start, int n_inst, int parity) {
  batch_body<S, MB>(tab, wave_start, n_inst, parity, xcd_block(blockIdx.x, gridDim.x));
}
template <int MB>
__global__ __launch_bounds__(64 * kStepWaves) TCLBM_BATCH32_OCC void batch_step_kernel_f32(
    const KParams *__restrict__ tab, const int *__restrict__ wave_start, int n_inst, int parity) {
  batch_body<kF32, MB>(tab, wave_start, n_inst, parity, xcd_block(blockIdx.x, gridDim.x));
}
template <int MB>
__global__ __launch_bounds__(64 * kStepWaves) void batch_step_kernel_f64(const KParams *__restrict__ tab,
                                                                         const int *__restrict__ wave_start,
                                                                         int n_inst, int parity) {
  batch_body<kF64, MB>(tab, wave_start, n_inst, parity, xcd_block(blockIdx.x, gridDim.x));
}

// Persistent batched steps: one cooperative launch (the runtime refuses a
// grid whose blocks cannot all be resident at once) runs nsteps steps of every
// member.  Its blocks take the per-step grid's logical blocks in turn, strided
// by the grid size, and meet at a grid barrier between steps.  The barrier is
// an arrival counter that only grows (the launch is told the count it starts
// from; comparisons are modulo 2^32) and a failure word that stays set.  A
// block that waits longer than wait_ticks of the wall clock at a barrier sets
// the failure word and leaves; every other block leaves at its next barrier,
// and a launch that finds the word set runs no step, so every wave ends.
// Agent-scope fences around the barrier make the stores of one step visible
// to the loads of the next across the XCDs' separate L2 caches.  That is an
// L2 write-back per block and barrier, where a kernel boundary needs one per
// XCD: on MI355X these launches measured slower than per-step launches
// replayed from a graph (512x256: 85 vs 9.2 us per step; 256 lattices: 1504
// vs 940 us), so they are not the default.
// Only the lean default-scheme instantiation with buffer addressing (MB = 2).
__device__ __forceinline__ bool persist_flag_clear(PersistCtl *ctl) {
  __shared__ int clear;
  __syncthreads();
  if (threadIdx.x == 0) clear = __hip_atomic_load(&ctl->fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u;
  __syncthreads();
  return clear != 0;
}

__device__ __forceinline__ bool grid_barrier(PersistCtl *ctl, unsigned target, long long wait_ticks) {
  __builtin_amdgcn_s_waitcnt(0);  // this wave's stores have reached L2
  __syncthreads();
  __shared__ int ok;
  if (threadIdx.x == 0) {
    // one wave per block fences for the whole block (every wave of it waited
    // for its stores above): release of the block's stores to every XCD
    __threadfence();
    int good = 1;
    __hip_atomic_fetch_add(&ctl->arrive, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    const long long t0 = wall_clock64();
    while ((int)(__hip_atomic_load(&ctl->arrive, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) - target) < 0) {
      if (__hip_atomic_load(&ctl->fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
          wall_clock64() - t0 >= wait_ticks) {
        __hip_atomic_store(&ctl->fail, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        good = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __threadfence();  // acquire, for the caches the block's waves share
    ok = good;
  }
  __syncthreads();
  return ok != 0;
}

template <int S>
__device__ __forceinline__ void persist_body(const KParams *__restrict__ tab, const int *__restrict__ wave_start,
                                             int n_inst, int parity, int nsteps, PersistCtl *ctl, unsigned base,
                                             long long wait_ticks) {
  if (!persist_flag_clear(ctl)) return;
  const int nwork = (wave_start[n_inst] + kStepWaves - 1) / kStepWaves;
  const int G = gridDim.x;
  const int lb0 = xcd_block(blockIdx.x, G);
  for (int s = 0; s < nsteps; ++s) {
    for (int lb = lb0; lb < nwork; lb += G) batch_body<S, 2>(tab, wave_start, n_inst, parity ^ (s & 1), lb);
    if (s + 1 < nsteps && !grid_barrier(ctl, base + (unsigned)(s + 1) * (unsigned)G, wait_ticks)) return;
  }
}

__global__ __launch_bounds__(64 * kStepWaves) TCLBM_BATCH32_OCC void batch_persistent_kernel_f32(
    const KParams *__restrict__ tab, const int *__restrict__ wave_start, int n_inst, int parity, int nsteps,
    PersistCtl *ctl, unsigned base, long long wait_ticks) {
  persist_body<kF32>(tab, wave_start, n_inst, parity, nsteps, ctl, base, wait_ticks);
}
template <int S>
__global__ __launch_bounds__(64 * kStepWaves) TCLBM_BATCH_OCC void batch_persistent_kernel(
    const KParams *__restrict__ tab, const int *__restrict__ wave_start, int n_inst, int parity, int nsteps,
    PersistCtl *ctl, unsigned base, long long wait_ticks) {
  persist_body<S>(tab, wave_start, n_inst, parity, nsteps, ctl, base, wait_ticks);
}

static const void *persistent_kernel(int storage) {
  switch (storage) {
    case kF32: return reinterpret_cast<const void *>(&batch_persistent_kernel_f32);
    case kF16: return reinterpret_cast<const void *>(&batch_persistent_kernel<kF16>);
    case kBF16: return reinterpret_cast<const void *>(&batch_persistent_kernel<kBF16>);
    default: return nullptr;
  }
}

hipError_t persistent_max_blocks(int storage, int *blocks) {
  *blocks = 0;
  const void *f = persistent_kernel(storage);
  if (!f) return hipErrorInvalidValue;
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, 64 * kStepWaves, 0);
  if (e == hipSuccess) *blocks = per_cu * cus;
  return e;
}

hipError_t launch_batch_persistent(const KParams *d_tab, const int *d_wave_start, int n_inst, int total_waves,
                                   int storage, int parity, int nsteps, PersistCtl *ctl, unsigned base,
                                   long long wait_ticks, int grid, hipStream_t s) {
  const void *f = persistent_kernel(storage);
  if (!f || grid <= 0 || nsteps <= 0 || total_waves <= 0) return hipErrorInvalidValue;
  void *args[] = {(void *)&d_tab, (void *)&d_wave_start, (void *)&n_inst, (void *)&parity, (void *)&nsteps,
                  (void *)&ctl,   (void *)&base,         (void *)&wait_ticks};
  return hipLaunchCooperativeKernel(f, dim3(grid), dim3(64 * kStepWaves), args, 0, s);
}

hipError_t launch_batch_step(const KParams *d_tab, const int *d_wave_start, int n_inst, int total_waves,
                             int storage, int parity, bool all_default, bool all_fit, hipStream_t s) {
  if (total_waves <= 0) return hipSuccess;
  const int blocks = (total_waves + kStepWaves - 1) / kStepWaves;
  dim3 grid(blocks), block(64 * kStepWaves);
  const bool d = TCLBM_SCHEME_SPECIAL && all_default;
  const bool b = d && TCLBM_BUFFER_ADDR && all_fit && storage != kF64;
#define TCLBM_BATCH_LAUNCH(K0, K1, K2)                                                       \
  do {                                                                                       \
    if (b) hipLaunchKernelGGL(K2, grid, block, 0, s, d_tab, d_wave_start, n_inst, parity);      \
    else if (d) hipLaunchKernelGGL(K1, grid, block, 0, s, d_tab, d_wave_start, n_inst, parity); \
    else hipLaunchKernelGGL(K0, grid, block, 0, s, d_tab, d_wave_start, n_inst, parity);        \
  } while (0)
  switch (storage) {
    case kF32:
      TCLBM_BATCH_LAUNCH((batch_step_kernel_f32<0>), (batch_step_kernel_f32<1>), (batch_step_kernel_f32<2>));
      break;
    case kF16:
      TCLBM_BATCH_LAUNCH((batch_step_kernel<kF16, 0>), (batch_step_kernel<kF16, 1>), (batch_step_kernel<kF16, 2>));
      break;
    case kBF16:
      TCLBM_BATCH_LAUNCH((batch_step_kernel<kBF16, 0>), (batch_step_kernel<kBF16, 1>),
                         (batch_step_kernel<kBF16, 2>));
      break;
    case kF64:
      TCLBM_BATCH_LAUNCH((batch_step_kernel_f64<0>), (batch_step_kernel_f64<1>), (batch_step_kernel_f64<1>));
      break;
    default: return hipErrorInvalidValue;
  }
#undef TCLBM_BATCH_LAUNCH
  return hipGetLastError();
}

int step_waves_per_block() { return kStepWaves; }

const char *batch_persistent_kernel_name(int storage) {
  switch (storage) {
    case kF32: return "batch_persistent_kernel_f32";
    case kF16:
    case kBF16: return "batch_persistent_kernel";
    default: return "";
  }
}

const char *batch_step_kernel_name(int storage) {
  switch (storage) {
    case kF32: return "batch_step_kernel_f32";
    case kF16:
    case kBF16: return "batch_step_kernel";
    case kF64: return "batch_step_kernel_f64";
    default: return "";
  }
}

hipError_t launch_step(const KParams &k, int storage, hipStream_t s) {
  const int waves = k.n_xtiles * k.n_strips;
  const int blocks = (waves + kStepWaves - 1) / kStepWaves;
  dim3 grid(blocks), block(64 * kStepWaves);
  const bool d = TCLBM_SCHEME_SPECIAL && default_scheme(k);
  const bool b = d && TCLBM_BUFFER_ADDR && buffer_fits(k, storage);
  switch (storage) {
    case kF32:
      if (d && k.strip_rows == 1 && kRowGroup > 1) {
        const int groups = (k.ny + kRowGroup - 1) / kRowGroup;
        const dim3 gg(groups * k.n_xtiles), gb(64 * kRowGroup);
        if (k.bc[kYlo] == kPeriodic) {
          if (b) hipLaunchKernelGGL((row_group_kernel<kF32, 2, kRowGroup, false>), gg, gb, 0, s, k);
          else hipLaunchKernelGGL((row_group_kernel<kF32, 1, kRowGroup, false>), gg, gb, 0, s, k);
        } else {
          if (b) hipLaunchKernelGGL((row_group_kernel<kF32, 2, kRowGroup, true>), gg, gb, 0, s, k);
          else hipLaunchKernelGGL((row_group_kernel<kF32, 1, kRowGroup, true>), gg, gb, 0, s, k);
        }
      } else if (d && k.strip_rows == 1 && kStepWaves != 1) {
        if (b) hipLaunchKernelGGL((step_kernel<kF32, 2, 1>), dim3(waves), dim3(64), 0, s, k);
        else hipLaunchKernelGGL((step_kernel<kF32, 1, 1>), dim3(waves), dim3(64), 0, s, k);
      } else if (b) hipLaunchKernelGGL((step_kernel<kF32, 2, kStepWaves>), grid, block, 0, s, k);
      else if (d) hipLaunchKernelGGL((step_kernel<kF32, 1, kStepWaves>), grid, block, 0, s, k);
      else hipLaunchKernelGGL((step_kernel<kF32, 0, kStepWaves>), grid, block, 0, s, k);
      break;
    case kF16:
      if (b) hipLaunchKernelGGL((step_kernel_16<kF16, 2>), grid, block, 0, s, k);
      else if (d) hipLaunchKernelGGL((step_kernel_16<kF16, 1>), grid, block, 0, s, k);
      else hipLaunchKernelGGL((step_kernel_16<kF16, 0>), grid, block, 0, s, k);
      break;
    case kBF16:
      if (b) hipLaunchKernelGGL((step_kernel_16<kBF16, 2>), grid, block, 0, s, k);
      else if (d) hipLaunchKernelGGL((step_kernel_16<kBF16, 1>), grid, block, 0, s, k);
      else hipLaunchKernelGGL((step_kernel_16<kBF16, 0>), grid, block, 0, s, k);
      break;
    case kF64:
      if (d) hipLaunchKernelGGL((step_kernel_f64<1>), grid, block, 0, s, k);
      else hipLaunchKernelGGL((step_kernel_f64<0>), grid, block, 0, s, k);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

const char *step_kernel_name(const KParams &k, int storage) {
  const bool d = TCLBM_SCHEME_SPECIAL && default_scheme(k);
  switch (storage) {
    case kF32: return (d && k.strip_rows == 1 && kRowGroup > 1) ? "row_group_kernel" : "step_kernel";
    case kF16:
    case kBF16: return "step_kernel_16";
    case kF64: return "step_kernel_f64";
    default: return "";
  }
}

size_t store_bytes(int storage) {
  switch (storage) {
    case kF32: return 4;
    case kF16:
    case kBF16: return 2;
    case kF64: return 8;
    default: return 0;
  }
}

// ------------------------------------------------------------ init kernel ---
// P_a(x) = fbar^init_a(x + e_a) so that the first pull returns the initial
// state fbar = f^eq - S/2, hbar = h^eq (Sections 3-4); the stored deviation is
// taken against the storing row (the reader adds r_a(source) - r_a(own) back).
// A link leaving through a non-periodic side stores the opposite population of
// the same node (the value that bounces back into it).
template <int S>
__global__ __launch_bounds__(256) void init_kernel(KParams k, const double *rho, const double *ux,
                                                   const double *uy, const double *T) {
  using R = typename Real<S>::T;
  using ST = typename Store<S>::T;
  const long long n = (long long)k.nx * k.ny;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int y = (int)(i / k.nx), x = (int)(i - (long long)y * k.nx);
  const Consts<R> c = make_consts<R>(k);
  const bool xper = k.bc[kXlo] == kPeriodic, yper = k.bc[kYlo] == kPeriodic;
  ST *dst = reinterpret_cast<ST *>(k.dst);
  const long long own = (long long)y * k.pitch + x;  // node number (rounding generator key)
  const long long at = (long long)y * k.rstride + col_off(k, x);  // its address in the state layout
#pragma unroll 1
  for (int a = 0; a < 9; ++a) {
    int tx = x + kEx[a], ty = y + kEy[a];
    bool out = false;
    if (xper) tx = (tx + k.nx) % k.nx;
    else if (tx < 0 || tx >= k.nx) out = true;
    if (yper) ty = (ty + k.ny) % k.ny;
    else if (ty < 0 || ty >= k.ny) out = true;
    int comp = a;
    if (out) {
      tx = x;
      ty = y;
      comp = kOpp[a];
    }
    const long long j = (long long)ty * k.nx + tx;
    const RowRef<R> q = row_ref(k, c, ty);
    // deviations from the row reference formed in double from the double
    // inputs: the O(1) density and temperature are never rounded to the
    // compute type before the subtraction
    const R drho = (R)(rho[j] - (double)q.rho);
    const R dth = (R)(k.R * (k.thermal ? T[j] : k.T0) - (double)q.th);
    const R r = q.rho + drho, th = q.th + dth;
    const R vx = (R)ux[j], vy = (R)uy[j];
    R ax, ay;
    node_accel<R>(k, ty, tx, ax, ay);
    R fe[9], se[9], he[9];
    feq_dev(q, drho, vx, vy, dth, fe);
    source9(r, vx, vy, ax, ay, se);
    // shift of the reader at (tx, ty) for direction a: r_a(y) - r_a(ty)
    R shf = R(0), shh = R(0);
    if (!out && kEy[a] != 0) {
      shf = reinterpret_cast<const R *>(k.shiftF)[9 * ty + a];
      shh = reinterpret_cast<const R *>(k.shiftH)[9 * ty + a];
    }
    const unsigned hn = sr_node((unsigned)own, kInitStep);
    Store<S>::st(dst, (long long)a * k.pstride + at, fe[comp] - R(0.5) * se[comp] - shf, sr_word(hn, a));
    if (k.thermal) {
      const R E = R(0.5) * (c.b * th + vx * vx + vy * vy);
      const R sg = drho * E + q.rho * (R(0.5) * c.b * dth + R(0.5) * (vx * vx + vy * vy));
      heq_dev(c, q, drho, vx, vy, dth, sg, he);
      Store<S>::st(dst, (long long)(a + 9) * k.pstride + at, he[comp] - shh, sr_word(hn, a + 9));
    }
  }
}

hipError_t launch_init(const KParams &k, int storage, const double *d_rho, const double *d_ux,
                       const double *d_uy, const double *d_T, hipStream_t s) {
  const long long n = (long long)k.nx * k.ny;
  dim3 grid((unsigned)((n + 255) / 256)), block(256);
  switch (storage) {
    case kF32: hipLaunchKernelGGL(init_kernel<kF32>, grid, block, 0, s, k, d_rho, d_ux, d_uy, d_T); break;
    case kF16: hipLaunchKernelGGL(init_kernel<kF16>, grid, block, 0, s, k, d_rho, d_ux, d_uy, d_T); break;
    case kBF16: hipLaunchKernelGGL(init_kernel<kBF16>, grid, block, 0, s, k, d_rho, d_ux, d_uy, d_T); break;
    case kF64: hipLaunchKernelGGL(init_kernel<kF64>, grid, block, 0, s, k, d_rho, d_ux, d_uy, d_T); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// --------------------------------------------------------- moments kernel ---
// Macroscopic fields of the state the next step sees (WALL rows after their
// extrapolation) and FP64 block sums (fixed-order tree in LDS, so repeated
// calls give bitwise-identical sums).
constexpr int kMomThreads = 256;

// Nodes i0 + [0, gridDim.x * kMomThreads) (i0 a multiple of kMomThreads, so
// that the blocks and their sums are those of a launch over the whole
// lattice); fields are written at i - i0, partials at the block index.
template <int S>
__global__ __launch_bounds__(kMomThreads) void moments_kernel(KParams k, long long i0, double *frho, double *fux,
                                                              double *fuy, double *fT, double *partials) {
  using R = typename Real<S>::T;
  __shared__ double red[kNumSums][kMomThreads];
  const long long n = (long long)k.nx * k.ny;
  const long long i = i0 + (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long o = i - i0;
  const Consts<R> c = make_consts<R>(k);
  double v[kNumSums];
#pragma unroll
  for (int q = 0; q < kNumSums; ++q) v[q] = 0.0;
  v[kSumRhoMin] = 1e300;
  v[kSumTMin] = 1e300;
  if (i < n) {
    const int y = (int)(i / k.nx), x = (int)(i - (long long)y * k.nx);
    const Col col = make_col(k, x);
    RowState<R> s;
    if (is_wall_row(k, y)) {
      RowState<R> in;
      get_row<S>(k, c, (y == 0) ? 1 : y - 1, col, in);
      get_wall_row<S>(k, c, y, col, in, s);
    } else {
      get_row<S>(k, c, y, col, s);
    }
    const double r = (double)s.q.rho + (double)s.m.drho, u = (double)s.m.ux, w = (double)s.m.uy;
    const double tmt0 = ((double)s.q.th - k.R * k.T0 + (double)s.m.dth) / k.R;  // T - T0
    const double t = k.T0 + tmt0;
    if (frho) frho[o] = r;
    if (fux) fux[o] = u;
    if (fuy) fuy[o] = w;
    if (fT) fT[o] = t;
    const double hs = k.thermal ? (double)s.q.rho * (double)s.q.E + (double)s.m.sg : 0.0;
    const bool bad = !(isfinite(r) && isfinite(u) && isfinite(w) && isfinite(t));
    v[kSumMass] = r;
    v[kSumMx] = r * u;
    v[kSumMy] = r * w;
    v[kSumE] = hs;
    v[kSumKin] = 0.5 * r * (u * u + w * w);
    v[kSumNu] = w * tmt0;
    v[kSumRhoMin] = bad ? -1.0 : r;
    v[kSumTMin] = bad ? -1.0 : t;
    v[kSumBad] = bad ? 1.0 : 0.0;
  }
#pragma unroll
  for (int q = 0; q < kNumSums; ++q) red[q][threadIdx.x] = v[q];
  __syncthreads();
  for (int st = kMomThreads / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
#pragma unroll
      for (int q = 0; q < kNumSums; ++q) {
        double o = red[q][threadIdx.x + st];
        if (q == kSumRhoMin || q == kSumTMin) red[q][threadIdx.x] = fmin(red[q][threadIdx.x], o);
        else red[q][threadIdx.x] += o;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < kNumSums; ++q) partials[(long long)blockIdx.x * kNumSums + q] = red[q][0];
  }
}

int moments_blocks(const KParams &k) {
  const long long n = (long long)k.nx * k.ny;
  return (int)((n + kMomThreads - 1) / kMomThreads);
}

int moments_block_nodes() { return kMomThreads; }

hipError_t launch_moments(const KParams &k, int storage, double *d_rho, double *d_ux, double *d_uy, double *d_T,
                          double *d_partials, int *nblocks_out, hipStream_t s) {
  const int nb = moments_blocks(k);
  if (nblocks_out) *nblocks_out = nb;
  return launch_moments_range(k, storage, 0, nb, d_rho, d_ux, d_uy, d_T, d_partials, s);
}

hipError_t launch_moments_range(const KParams &k, int storage, long long block0, int nblocks, double *d_rho,
                                double *d_ux, double *d_uy, double *d_T, double *d_partials, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  const long long i0 = block0 * kMomThreads;
  dim3 grid(nblocks), block(kMomThreads);
  switch (storage) {
    case kF32:
      hipLaunchKernelGGL(moments_kernel<kF32>, grid, block, 0, s, k, i0, d_rho, d_ux, d_uy, d_T, d_partials);
      break;
    case kF16:
      hipLaunchKernelGGL(moments_kernel<kF16>, grid, block, 0, s, k, i0, d_rho, d_ux, d_uy, d_T, d_partials);
      break;
    case kBF16:
      hipLaunchKernelGGL(moments_kernel<kBF16>, grid, block, 0, s, k, i0, d_rho, d_ux, d_uy, d_T, d_partials);
      break;
    case kF64:
      hipLaunchKernelGGL(moments_kernel<kF64>, grid, block, 0, s, k, i0, d_rho, d_ux, d_uy, d_T, d_partials);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ----------------------------------------------------- raw state readback ---
template <int S>
__global__ __launch_bounds__(256) void read_state_kernel(KParams k, double *out) {
  using R = typename Real<S>::T;
  using ST = typename Store<S>::T;
  const long long n = (long long)k.nx * k.ny;
  const int np = k.thermal ? 18 : 9;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * np) return;
  const int a = (int)(i / n);
  const long long node = i - (long long)a * n;
  const int y = (int)(node / k.nx), x = (int)(node - (long long)y * k.nx);
  const ST *src = reinterpret_cast<const ST *>(k.src);
  const R *rr = reinterpret_cast<const R *>(k.rowref);
  const RowRef<double> q = make_ref<double>((double)rr[2 * y], (double)rr[2 * y + 1], k.b, k.heq_mode);
  double r[9], s[9];
  ref_pops<double>(q, k.thermal, k.heq_mode, r, s);
  const double ref = (a < 9) ? r[a] : s[a - 9];
  out[i] = ref + (double)Store<S>::ld(src, (long long)a * k.pstride + (long long)y * k.rstride + col_off(k, x));
}

hipError_t launch_read_state(const KParams &k, int storage, double *d_out, hipStream_t s) {
  const long long n = (long long)k.nx * k.ny * (k.thermal ? 18 : 9);
  dim3 grid((unsigned)((n + 255) / 256)), block(256);
  switch (storage) {
    case kF32: hipLaunchKernelGGL(read_state_kernel<kF32>, grid, block, 0, s, k, d_out); break;
    case kF16: hipLaunchKernelGGL(read_state_kernel<kF16>, grid, block, 0, s, k, d_out); break;
    case kBF16: hipLaunchKernelGGL(read_state_kernel<kBF16>, grid, block, 0, s, k, d_out); break;
    case kF64: hipLaunchKernelGGL(read_state_kernel<kF64>, grid, block, 0, s, k, d_out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// -------------------------------------------------------- HBM copy probe ---
// Streaming copy used to measure the achievable HBM bandwidth and to
// calibrate byte counters: one 16-byte element per thread, a plain load and a
// non-temporal store (the access types of the step kernels' pulls and
// stores).  Copies of 2 GiB measured with 1, 2, 4, 8 and 16 elements per
// thread in flight: one was the fastest (plain loads and stores 6.14 TB/s
// against 5.69-5.71 at two to four, non-temporal loads and stores 6.51 TB/s).
typedef unsigned int CopyV __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void copy_kernel(const CopyV *__restrict__ src, CopyV *__restrict__ dst,
                                                   long long n16) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < n16) __builtin_nontemporal_store(src[i], dst + i);
}

hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t s) {
  const long long n16 = (long long)(bytes / 16);
  if (n16 <= 0) return hipSuccess;
  const long long blocks = (n16 + 255) / 256;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, s, reinterpret_cast<const CopyV *>(src),
                     reinterpret_cast<CopyV *>(dst), n16);
  return hipGetLastError();
}

}  // namespace tclbm
