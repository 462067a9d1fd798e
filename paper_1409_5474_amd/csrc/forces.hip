// Direct-summation force kernels for gfx950 (CDNA4).
//
// Computes, for every i in the active set and every j of the j-set,
//   r = x_j - x_i, u = v_j - v_i, s = |r|^2 + eps2, q = s^{-1/2}
//   a += m_j q^3 r,   jdot += m_j q^3 (u - 3 (r.u) q^2 r),   phi -= m_j q
// (the i-particle / j-particle split of the paper's section "Optimizations
// for the GPU"; G = 1, Plummer softening).
//
// Mapping onto the chip (one family of kernels, three tiling axes):
//  * j-tiles of kTile particles are read once per workgroup from the
//    caller's row-major arrays with contiguous (coalesced) loads, converted
//    to the kernel's layout and staged in LDS; the next tile is prefetched
//    into registers while the current one is consumed.
//  * K i-particles per lane: every LDS read of a j-particle feeds K pair
//    evaluations, and the K independent chains hide VALU latency.
//  * L lanes per i-particle: lane `sub` of a group takes j = sub, sub+L, ...
//    of each tile; the L partial sums are combined by butterfly shuffles
//    inside the wavefront and, for L > 64, through LDS across wavefronts.
//  * S j-subsets: the j-range is cut into S chunks, one workgroup each; the
//    partial sums go to a workspace and a second kernel adds them in a fixed
//    order (the paper's two-kernel scheme).  Nothing uses float atomics, so
//    every result is bitwise reproducible run to run.
// The pair loop is VALU-bound (the pairwise reciprocal square root is not a
// dense contraction), so the work is plain vector arithmetic, not MFMA.
//
// Precision policies
//  * F64:   all pair arithmetic in double; per-tile double sums folded into a
//           compensated (TwoSum) double-double accumulator.
//  * Mixed: r = x_j - x_i formed in double and rounded to float, u, m and all
//           pair arithmetic in float, float sums over runs of NB_FP32_RUN
//           pairs (acceleration, potential) or one tile (jerk) added into
//           double accumulators (the paper's remedy for single precision: the
//           largest error sits in the inter-particle distance, which is
//           therefore formed in higher precision).
// The self pair (j == i) is not skipped in the loop: with eps2 > 0 it adds
// exactly zero to a and jdot and m_i q(eps2) to the potential sum, which is
// removed afterwards using the identical value.  With eps2 == 0 the MASK
// variant drops every pair with s == 0 instead.
#include <map>
#include <mutex>

// Unroll factor of the pair loop over a staged tile: more unrolling gives
// the scheduler more independent LDS reads, fewer leaves VGPRs for more
// resident waves (which the dual VALU issue of gfx950 needs).
#ifndef NB_JJ_UNROLL
#define NB_JJ_UNROLL 2
#endif

// Length of the float runs of the mixed policies: every NB_FP32_RUN pairs
// a lane adds its float sums of acceleration and potential into the double
// accumulators.  A float sum that already holds one dominant term (a
// heavy neighbour, or the self pair m_i/eps) rounds every later small term
// to its own ulp, with an error that has a sign bias and so grows linearly
// with the run length; 32 keeps it near the float rounding of one pair for
// mass ratios of 1e3 at a cost of two instructions per component per run.
// The jerk error is set by the float velocity differences instead and is
// folded once per tile.
#ifndef NB_FP32_RUN
#define NB_FP32_RUN 32
#endif

#include "nb_internal.h"
#include "hermite_step.h"

namespace nb {
namespace {

// Reciprocal square root in double: hardware estimate refined by one
// third-order Newton step, y <- y (1 + e/2 + 3 e^2/8) with e = 1 - s y^2.
__device__ __forceinline__ double rsqrt_f64(double s) {
  const double y = __builtin_amdgcn_rsq(s);
  const double e = fma(-(s * y), y, 1.0);
  return fma(y, e * fma(e, 0.375, 0.5), y);
}

// A wave-uniform value copied into a VGPR.  gfx950 pairs two independent
// VALU instructions of a wave per issue cycle only when neither reads an
// SGPR, so a loop-invariant operand such as eps2 is kept in a VGPR.
__device__ __forceinline__ float in_vgpr(float x) {
  float r;
  asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "s"(x));
  return r;
}
__device__ __forceinline__ double in_vgpr(double x) {
  double r;
  asm volatile("v_mov_b64 %0, %1" : "=v"(r) : "s"(x));
  return r;
}

__device__ __forceinline__ float add_nocontract(float a, float b) {
#pragma clang fp contract(off)
  return a + b;
}

__device__ __forceinline__ void two_sum_add(double& hi, double& lo, double x) {
  const double s = hi + x;
  const double bp = s - hi;
  const double err = (hi - (s - bp)) + (x - bp);
  hi = s;
  lo += err;
}

// ------------------------------------------------------------------ F64 ----
struct F64 {
  using T = double;
  template <int TT>
  struct JTileT {
    double2 xy[TT];
    double2 zm[TT];
    double2 vxy[TT];
    double vz[TT];
  };
  using JTile = JTileT<kTile>;
  struct JReg {
    double x, y, z, vx, vy, vz, m;
  };
  struct IPart {
    double x, y, z, vx, vy, vz;
  };
  struct Tot {
    double hi[7], lo[7];
  };
  static __device__ __forceinline__ JReg load(const double* pos, const double* vel, const double* mass,
                                              int64_t j, bool valid) {
    JReg r;
    if (valid) {
      r.x = pos[3 * j]; r.y = pos[3 * j + 1]; r.z = pos[3 * j + 2];
      r.vx = vel[3 * j]; r.vy = vel[3 * j + 1]; r.vz = vel[3 * j + 2];
      r.m = mass[j];
    } else {
      r.x = r.y = r.z = r.vx = r.vy = r.vz = r.m = 0.0;
    }
    return r;
  }
  template <class Tile>
  static __device__ __forceinline__ void store(Tile& t, int s, const JReg& r) {
    t.xy[s] = make_double2(r.x, r.y);
    t.zm[s] = make_double2(r.z, r.m);
    t.vxy[s] = make_double2(r.vx, r.vy);
    t.vz[s] = r.vz;
  }
  static __device__ __forceinline__ IPart load_i(const double* pos, const double* vel, int64_t i) {
    IPart p;
    p.x = pos[3 * i]; p.y = pos[3 * i + 1]; p.z = pos[3 * i + 2];
    p.vx = vel[3 * i]; p.vy = vel[3 * i + 1]; p.vz = vel[3 * i + 2];
    return p;
  }
  static __device__ __forceinline__ T eps(double eps2) { return eps2; }

  template <bool MASK>
  static __device__ __forceinline__ void pair(const IPart& I, const double2 xy, const double2 zm,
                                              const double2 vxy, const double vz, const T e2, T* A) {
    const double dx = xy.x - I.x, dy = xy.y - I.y, dz = zm.x - I.z;
    const double s = fma(dz, dz, fma(dy, dy, fma(dx, dx, e2)));
    double q = rsqrt_f64(s);
    if (MASK) q = (s > 0.0) ? q : 0.0;
    const double ux = vxy.x - I.vx, uy = vxy.y - I.vy, uz = vz - I.vz;
    const double rv = fma(dz, uz, fma(dy, uy, dx * ux));
    const double q2 = q * q;
    const double mq = zm.y * q;
    const double mq3 = mq * q2;
    const double c = -3.0 * (rv * q2);
    A[0] = fma(mq3, dx, A[0]);
    A[1] = fma(mq3, dy, A[1]);
    A[2] = fma(mq3, dz, A[2]);
    A[3] = fma(mq3, fma(c, dx, ux), A[3]);
    A[4] = fma(mq3, fma(c, dy, uy), A[4]);
    A[5] = fma(mq3, fma(c, dz, uz), A[5]);
    A[6] += mq;
  }
  template <bool MASK, class Tile>
  static __device__ __forceinline__ void pair_tile(const Tile& t, int s, const IPart* I, T e2, T (*A)[7],
                                                   int kcount) {
    const double2 xy = t.xy[s];
    const double2 zm = t.zm[s];
    const double2 vxy = t.vxy[s];
    const double vz = t.vz[s];
#pragma unroll
    for (int k = 0; k < kcount; ++k) pair<MASK>(I[k], xy, zm, vxy, vz, e2, A[k]);
  }
  static __device__ __forceinline__ void zero(Tot& t) {
#pragma unroll
    for (int c = 0; c < 7; ++c) t.hi[c] = t.lo[c] = 0.0;
  }
  static __device__ __forceinline__ void fold(Tot& t, T* A) {
#pragma unroll
    for (int c = 0; c < 7; ++c) {
      two_sum_add(t.hi[c], t.lo[c], A[c]);
      A[c] = 0.0;
    }
  }
  // Double tile sums are folded once per tile only.
  static constexpr int kRun = kTile;
  static __device__ __forceinline__ void fold_run(Tot&, T*) {}
  static __device__ __forceinline__ double value(const Tot& t, int c) { return t.hi[c] + t.lo[c]; }
  // The value the pair loop adds to the potential sum for the self pair.
  static __device__ __forceinline__ double self_term(double m, double eps2) { return m * rsqrt_f64(eps2); }
  // The pair from a j-record held in (scalar) registers.
  template <bool MASK>
  static __device__ __forceinline__ void pair_reg(const JReg& r, const IPart* I, T e2, T (*A)[7], int kcount) {
#pragma unroll
    for (int k = 0; k < kcount; ++k)
      pair<MASK>(I[k], make_double2(r.x, r.y), make_double2(r.z, r.m), make_double2(r.vx, r.vy), r.vz, e2, A[k]);
  }
};

// ---------------------------------------------------------------- Mixed ----
struct Mixed {
  using T = float;
  template <int TT>
  struct JTileT {
    double2 xy[TT];
    double z[TT];
    float4 vm[TT];
  };
  using JTile = JTileT<kTile>;
  struct JReg {
    double x, y, z;
    float vx, vy, vz, m;
  };
  struct IPart {
    double x, y, z;
    float vx, vy, vz;
  };
  struct Tot {
    double v[7];
  };
  static __device__ __forceinline__ JReg load(const double* pos, const double* vel, const double* mass,
                                              int64_t j, bool valid) {
    JReg r;
    if (valid) {
      r.x = pos[3 * j]; r.y = pos[3 * j + 1]; r.z = pos[3 * j + 2];
      r.vx = (float)vel[3 * j]; r.vy = (float)vel[3 * j + 1]; r.vz = (float)vel[3 * j + 2];
      r.m = (float)mass[j];
    } else {
      r.x = r.y = r.z = 0.0;
      r.vx = r.vy = r.vz = r.m = 0.0f;
    }
    return r;
  }
  template <class Tile>
  static __device__ __forceinline__ void store(Tile& t, int s, const JReg& r) {
    t.xy[s] = make_double2(r.x, r.y);
    t.z[s] = r.z;
    t.vm[s] = make_float4(r.vx, r.vy, r.vz, r.m);
  }
  static __device__ __forceinline__ IPart load_i(const double* pos, const double* vel, int64_t i) {
    IPart p;
    p.x = pos[3 * i]; p.y = pos[3 * i + 1]; p.z = pos[3 * i + 2];
    p.vx = (float)vel[3 * i]; p.vy = (float)vel[3 * i + 1]; p.vz = (float)vel[3 * i + 2];
    return p;
  }
  static __device__ __forceinline__ T eps(double eps2) { return (float)eps2; }

  template <bool MASK>
  static __device__ __forceinline__ void pair(const IPart& I, const double2 xy, const double zj,
                                              const float4 vm, const T e2, T* A) {
    const float dx = (float)(xy.x - I.x);
    const float dy = (float)(xy.y - I.y);
    const float dz = (float)(zj - I.z);
    const float s = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, e2)));
    float q = __builtin_amdgcn_rsqf(s);
    if (MASK) q = (s > 0.0f) ? q : 0.0f;
    const float ux = vm.x - I.vx, uy = vm.y - I.vy, uz = vm.z - I.vz;
    const float rv = fmaf(dz, uz, fmaf(dy, uy, dx * ux));
    const float q2 = q * q;
    const float mq = vm.w * q;
    const float mq3 = mq * q2;
    const float c = -3.0f * (rv * q2);
    A[0] = fmaf(mq3, dx, A[0]);
    A[1] = fmaf(mq3, dy, A[1]);
    A[2] = fmaf(mq3, dz, A[2]);
    A[3] = fmaf(mq3, fmaf(c, dx, ux), A[3]);
    A[4] = fmaf(mq3, fmaf(c, dy, uy), A[4]);
    A[5] = fmaf(mq3, fmaf(c, dz, uz), A[5]);
    // a separate add (no contraction): fused into an FMA the mass, often an
    // SGPR, would be read twice per pair, and SGPR-operand instructions never
    // dual-issue
    A[6] = add_nocontract(A[6], mq);
  }
  template <bool MASK, class Tile>
  static __device__ __forceinline__ void pair_tile(const Tile& t, int s, const IPart* I, T e2, T (*A)[7],
                                                   int kcount) {
    const double2 xy = t.xy[s];
    const double z = t.z[s];
    const float4 vm = t.vm[s];
#pragma unroll
    for (int k = 0; k < kcount; ++k) pair<MASK>(I[k], xy, z, vm, e2, A[k]);
  }
  static __device__ __forceinline__ void zero(Tot& t) {
#pragma unroll
    for (int c = 0; c < 7; ++c) t.v[c] = 0.0;
  }
  static __device__ __forceinline__ void fold(Tot& t, T* A) {
#pragma unroll
    for (int c = 0; c < 7; ++c) {
      t.v[c] += (double)A[c];
      A[c] = 0.0f;
    }
  }
  // Acceleration and potential leave their float sums every kRun pairs.
  static constexpr int kRun = NB_FP32_RUN;
  static_assert(kRun > 0 && (kRun & (kRun - 1)) == 0 && kTile % kRun == 0, "float run must divide the tile");
  static __device__ __forceinline__ void fold_run(Tot& t, T* A) {
#pragma unroll
    for (int c = 0; c < 7; ++c) {
      if (c >= 3 && c < 6) continue;
      t.v[c] += (double)A[c];
      A[c] = 0.0f;
    }
  }
  static __device__ __forceinline__ double value(const Tot& t, int c) { return t.v[c]; }
  static __device__ __forceinline__ double self_term(double m, double eps2) {
    return (double)((float)m * __builtin_amdgcn_rsqf((float)eps2));
  }
  template <bool MASK>
  static __device__ __forceinline__ void pair_reg(const JReg& r, const IPart* I, T e2, T (*A)[7], int kcount) {
#pragma unroll
    for (int k = 0; k < kcount; ++k)
      pair<MASK>(I[k], make_double2(r.x, r.y), r.z, make_float4(r.vx, r.vy, r.vz, r.m), e2, A[k]);
  }
};

// ------------------------------------------------------------- MixedDS -----
// As Mixed, but the separation is formed in emulated double precision on
// float hardware (the paper's remedy for single-precision devices): every
// position is split once, at staging, into x = hi + lo (two floats), and
//   r = (x_j,hi - x_i,hi) + (x_j,lo - x_i,lo)
// costs three float operations instead of a double subtraction and a
// conversion.  The error of r stays within a few float ulps of |r|.
struct MixedDS {
  using T = float;
  template <int TT>
  struct JTileT {
    float4 hm[TT];   // x_hi, y_hi, z_hi, m
    float4 lv[TT];   // x_lo, y_lo, z_lo, vx
    float2 vyz[TT];  // vy, vz
  };
  using JTile = JTileT<kTile>;
  struct JReg {
    float4 hm, lv;
    float2 vyz;
  };
  struct IPart {
    float xh, yh, zh, xl, yl, zl, vx, vy, vz;
  };
  struct Tot {
    double v[7];
  };
  static __device__ __forceinline__ void split(double x, float& hi, float& lo) {
    hi = (float)x;
    lo = (float)(x - (double)hi);
  }
  static __device__ __forceinline__ JReg load(const double* pos, const double* vel, const double* mass,
                                              int64_t j, bool valid) {
    JReg r;
    if (valid) {
      float xh, xl, yh, yl, zh, zl;
      split(pos[3 * j], xh, xl);
      split(pos[3 * j + 1], yh, yl);
      split(pos[3 * j + 2], zh, zl);
      r.hm = make_float4(xh, yh, zh, (float)mass[j]);
      r.lv = make_float4(xl, yl, zl, (float)vel[3 * j]);
      r.vyz = make_float2((float)vel[3 * j + 1], (float)vel[3 * j + 2]);
    } else {
      r.hm = make_float4(0.f, 0.f, 0.f, 0.f);
      r.lv = make_float4(0.f, 0.f, 0.f, 0.f);
      r.vyz = make_float2(0.f, 0.f);
    }
    return r;
  }
  template <class Tile>
  static __device__ __forceinline__ void store(Tile& t, int s, const JReg& r) {
    t.hm[s] = r.hm;
    t.lv[s] = r.lv;
    t.vyz[s] = r.vyz;
  }
  static __device__ __forceinline__ IPart load_i(const double* pos, const double* vel, int64_t i) {
    IPart p;
    split(pos[3 * i], p.xh, p.xl);
    split(pos[3 * i + 1], p.yh, p.yl);
    split(pos[3 * i + 2], p.zh, p.zl);
    p.vx = (float)vel[3 * i]; p.vy = (float)vel[3 * i + 1]; p.vz = (float)vel[3 * i + 2];
    return p;
  }
  static __device__ __forceinline__ T eps(double eps2) { return (float)eps2; }

  template <bool MASK>
  static __device__ __forceinline__ void pair(const IPart& I, const float4 hm, const float4 lv, const float2 vyz,
                                              const T e2, T* A) {
    const float dx = (hm.x - I.xh) + (lv.x - I.xl);
    const float dy = (hm.y - I.yh) + (lv.y - I.yl);
    const float dz = (hm.z - I.zh) + (lv.z - I.zl);
    const float s = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, e2)));
    float q = __builtin_amdgcn_rsqf(s);
    if (MASK) q = (s > 0.0f) ? q : 0.0f;
    const float ux = lv.w - I.vx, uy = vyz.x - I.vy, uz = vyz.y - I.vz;
    const float rv = fmaf(dz, uz, fmaf(dy, uy, dx * ux));
    const float q2 = q * q;
    const float mq = hm.w * q;
    const float mq3 = mq * q2;
    const float c = -3.0f * (rv * q2);
    A[0] = fmaf(mq3, dx, A[0]);
    A[1] = fmaf(mq3, dy, A[1]);
    A[2] = fmaf(mq3, dz, A[2]);
    A[3] = fmaf(mq3, fmaf(c, dx, ux), A[3]);
    A[4] = fmaf(mq3, fmaf(c, dy, uy), A[4]);
    A[5] = fmaf(mq3, fmaf(c, dz, uz), A[5]);
    A[6] = add_nocontract(A[6], mq);
  }
  template <bool MASK, class Tile>
  static __device__ __forceinline__ void pair_tile(const Tile& t, int s, const IPart* I, T e2, T (*A)[7],
                                                   int kcount) {
    const float4 hm = t.hm[s];
    const float4 lv = t.lv[s];
    const float2 vyz = t.vyz[s];
#pragma unroll
    for (int k = 0; k < kcount; ++k) pair<MASK>(I[k], hm, lv, vyz, e2, A[k]);
  }
  static __device__ __forceinline__ void zero(Tot& t) {
#pragma unroll
    for (int c = 0; c < 7; ++c) t.v[c] = 0.0;
  }
  static __device__ __forceinline__ void fold(Tot& t, T* A) {
#pragma unroll
    for (int c = 0; c < 7; ++c) {
      t.v[c] += (double)A[c];
      A[c] = 0.0f;
    }
  }
  // Acceleration and potential leave their float sums every kRun pairs.
  static constexpr int kRun = NB_FP32_RUN;
  static_assert(kRun > 0 && (kRun & (kRun - 1)) == 0 && kTile % kRun == 0, "float run must divide the tile");
  static __device__ __forceinline__ void fold_run(Tot& t, T* A) {
#pragma unroll
    for (int c = 0; c < 7; ++c) {
      if (c >= 3 && c < 6) continue;
      t.v[c] += (double)A[c];
      A[c] = 0.0f;
    }
  }
  static __device__ __forceinline__ double value(const Tot& t, int c) { return t.v[c]; }
  static __device__ __forceinline__ double self_term(double m, double eps2) {
    return (double)((float)m * __builtin_amdgcn_rsqf((float)eps2));
  }
  template <bool MASK>
  static __device__ __forceinline__ void pair_reg(const JReg& r, const IPart* I, T e2, T (*A)[7], int kcount) {
#pragma unroll
    for (int k = 0; k < kcount; ++k) pair<MASK>(I[k], r.hm, r.lv, r.vyz, e2, A[k]);
  }
};

// The j-split chosen on the device (device-count mode) and on the host
// alike: enough work items to fill the chip, chunks of at least one tile.
__host__ __device__ inline int choose_S(int64_t n_act, int IB, int target_items, int64_t n, int tile = kTile) {
  const int64_t n_iblk = (n_act + IB - 1) / IB;
  if (n_iblk <= 0) return 1;
  int64_t s = (target_items + n_iblk - 1) / n_iblk;
  const int64_t max_s = (n + tile - 1) / tile;
  if (s > max_s) s = max_s;
  if (s < 1) s = 1;
  return (int)s;
}

// The work-item target of a device-count launch for count d (see n_sub).
// The loop is unrolled so that every table entry is read at a fixed offset
// of the kernel arguments: an index known only at run time would make the
// compiler copy the arguments to scratch memory, which upsets the register
// allocation of the whole kernel.
__device__ __forceinline__ int target_for(const ForceArgs& a, int64_t d) {
  int t = a.target_items;
#pragma unroll
  for (int r = 0; r < kMaxSubRegimes; ++r)
    if (r < a.n_sub && d >= a.sub_lo[r]) t = a.sub_items[r];
  return t;
}

// An i-set entry: its row, or -1 when it lies outside [lo, hi) -- the row is
// then skipped and the context's error word flags it for nb_sync.
__device__ __forceinline__ int64_t checked_row(const int32_t* active, int64_t k, int64_t lo, int64_t hi,
                                               unsigned int* err) {
  const int64_t r = active[k];
  if (row_in_range(r, lo, hi)) return r;
  if (err) atomicOr(err, kErrActiveRange);
  return -1;
}

__host__ __device__ inline int64_t chunk_len(int64_t n, int S, int tile = kTile) {
  const int64_t per = (n + S - 1) / S;
  return ((per + tile - 1) / tile) * tile;
}

// Work queues of the persistent force grids.  The items -- (i-block,
// j-chunk) pairs in chunk-major order -- are cut into kXcd equal ranges, one
// per XCD: the hardware hands workgroups to the chip's 8 XCDs round-robin by
// blockIdx, so range x is worked by the workgroups on XCD x, and that XCD's
// L2 holds only the j-chunks of its own range.  Within a range, workgroups
// take items from a counter in device memory (wq[x]), so a faster compute
// unit takes more; once its own range is exhausted, a workgroup takes from
// the other ranges in turn, so the XCDs (whose clocks differ by a few
// percent) also finish together.  Each item is computed the same way
// whichever workgroup takes it: results do not depend on the assignment.
// wq[0..kXcd-1] are the range counters and wq[kXcd] counts finished
// workgroups; all are zero before a launch and the last workgroup to finish
// sets them back to zero.  Without a queue (wq null) the grid strides over
// the items in the same order.
constexpr int kXcd = 8;
constexpr int kQueueWords = kXcd + 1;
static_assert(kQueueWords <= kWorkQueueWords, "work queue larger than its buffer");

// Thread 0 turns an own-range take into an item: `own` is the counter value
// the take returned.  When that range is exhausted it reads every range's
// counter at once (independent loads, one round of latency: device-scope
// atomics cost about a microsecond each, so the ranges are not visited one
// by one) and takes from the first range with items left, in the order
// x0 + 1, x0 + 2, ...  Returns the item, or `items` once all are exhausted.
__device__ __forceinline__ int64_t queue_pick(unsigned int* wq, int64_t items, unsigned int own) {
  const int x0 = blockIdx.x % kXcd;
  const int64_t lo0 = items * x0 / kXcd, len0 = items * (x0 + 1) / kXcd - lo0;
  if ((int64_t)own < len0) return lo0 + own;
  for (int attempt = 0; attempt < kXcd; ++attempt) {
    unsigned int cnt[kXcd];
#pragma unroll
    for (int x = 0; x < kXcd; ++x) cnt[x] = __hip_atomic_load(&wq[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int pick = -1, best = kXcd;
#pragma unroll
    for (int x = 0; x < kXcd; ++x) {
      const int64_t len = items * (x + 1) / kXcd - items * x / kXcd;
      const int order = (x - x0 - 1 + 2 * kXcd) % kXcd;  // 0 for range x0 + 1
      if ((int64_t)cnt[x] < len && order < best) {
        best = order;
        pick = x;
      }
    }
    if (pick < 0) return items;
    const int64_t lo = items * pick / kXcd, len = items * (pick + 1) / kXcd - lo;
    const int64_t k = atomicAdd(&wq[pick], 1u);
    if (k < len) return lo + k;
  }
  return items;
}

// The first item of a workgroup (w_stride: its item without a queue).
__device__ __forceinline__ int64_t queue_take(unsigned int* wq, unsigned int& slot, int64_t items,
                                              int64_t w_stride) {
  if (!wq) return w_stride;
  if (threadIdx.x == 0) slot = (unsigned int)queue_pick(wq, items, atomicAdd(&wq[blockIdx.x % kXcd], 1u));
  __syncthreads();
  // one value for the whole wave: read into a scalar register, so everything
  // derived from the item (chunk bounds, record addresses) stays uniform
  return (int64_t)(unsigned int)__builtin_amdgcn_readfirstlane((int)slot);
}

// A workgroup's next item (w_stride: its next item without a queue).
__device__ __forceinline__ int64_t queue_next(unsigned int* wq, unsigned int& slot, int64_t items, int64_t w_stride) {
  if (!wq) return w_stride;
  __syncthreads();  // every thread has read `slot` before it is replaced
  if (threadIdx.x == 0) slot = (unsigned int)queue_pick(wq, items, atomicAdd(&wq[blockIdx.x % kXcd], 1u));
  __syncthreads();
  return (int64_t)(unsigned int)__builtin_amdgcn_readfirstlane((int)slot);
}

// Only the first min(items, grid) workgroups take part in a launch's queue
// (one item each at least; the rest return at once, so a launch sized for
// its largest count costs little at a small one).  Every member calls
// queue_done once, after its last queue_next; the last one resets the queue.
__device__ __forceinline__ bool queue_member(int64_t items) { return (int64_t)blockIdx.x < items; }

__device__ __forceinline__ void queue_done(unsigned int* wq, int64_t items) {
  const unsigned int members = items < (int64_t)gridDim.x ? (unsigned int)items : gridDim.x;
  if (wq && threadIdx.x == 0 && atomicAdd(&wq[kXcd], 1u) == members - 1) {
    for (int x = 0; x < kQueueWords; ++x) atomicExch(&wq[x], 0u);
  }
}

// Shared body: one workgroup processes one (i-block, j-chunk) item.
// Outputs: final rows (acc/jerk/pot at out_row0 + k) when `final_out`,
// otherwise partial sums part[c * n_act + k] for c = 0..6.
template <class P, int K, int L, bool MASK, int T = kTile, int WG = kWG, bool ATOMIC = false>
__device__ __forceinline__ void process_item(typename P::template JTileT<T>& tile, double* red, const double* __restrict__ pos,
                                             const double* __restrict__ vel, const double* __restrict__ mass,
                                             const double* __restrict__ ipos, const double* __restrict__ ivel,
                                             const double* __restrict__ smass,
                                             int64_t jbeg, int64_t jend, const int32_t* __restrict__ active,
                                             int64_t n_act, int64_t k0, double eps2, bool final_out,
                                             double* __restrict__ acc, double* __restrict__ jerk,
                                             double* __restrict__ pot, double* __restrict__ part, int64_t row_lo,
                                             int64_t row_hi, unsigned int* err) {
  static_assert(L <= T && T <= WG && WG <= kWG, "a tile holds a pair for every lane and one record per thread");
  constexpr int SLOTS = WG / L;
  constexpr int PER = T / L;                              // pairs per lane and tile
  constexpr int RUN = P::kRun < PER ? P::kRun : PER;      // pairs per float run
  const int t = threadIdx.x;
  const int slot = t / L;
  const int sub = t % L;

  typename P::IPart I[K];
  int64_t irow[K];
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    const int64_t k = k0 + kk * SLOTS + slot;
    irow[kk] = (k < n_act) ? checked_row(active, k, row_lo, row_hi, err) : -1;
    I[kk] = P::load_i(ipos, ivel, irow[kk] >= 0 ? irow[kk] : 0);
  }
  const typename P::T e2 = in_vgpr(P::eps(eps2));

  typename P::T A[K][7];
  typename P::Tot Tt[K];
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    P::zero(Tt[kk]);
#pragma unroll
    for (int c = 0; c < 7; ++c) A[kk][c] = 0;
  }

  // threads t < T stage one record each
  typename P::JReg nxt = P::load(pos, vel, mass, jbeg + t, t < T && jbeg + t < jend);
  for (int64_t base = jbeg; base < jend; base += T) {
    __syncthreads();  // every lane is done with the previous tile
    if (T == WG || t < T) P::store(tile, t, nxt);
    __syncthreads();
    const int64_t nb = base + T;
    if (nb < jend) nxt = P::load(pos, vel, mass, nb + t, t < T && nb + t < jend);
#pragma unroll 1
    for (int jb = 0; jb < T; jb += RUN * L) {
#pragma unroll NB_JJ_UNROLL
      for (int jj = jb + sub; jj < jb + RUN * L; jj += L) P::template pair_tile<MASK>(tile, jj, I, e2, A, K);
      if constexpr (RUN < PER) {
        if (jb + RUN * L < T) {
#pragma unroll
          for (int kk = 0; kk < K; ++kk) P::fold_run(Tt[kk], A[kk]);
        }
      }
    }
#pragma unroll
    for (int kk = 0; kk < K; ++kk) P::fold(Tt[kk], A[kk]);
  }

  // Combine the L lanes of each i-particle, in a fixed order.
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    double v[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) v[c] = P::value(Tt[kk], c);
    if constexpr (L > 1) {
      constexpr int LW = L < 64 ? L : 64;
#pragma unroll
      for (int o = LW / 2; o > 0; o >>= 1) {
#pragma unroll
        for (int c = 0; c < 7; ++c) v[c] += __shfl_xor(v[c], o, 64);
      }
    }
    if constexpr (L > 64) {
      constexpr int NW = L / 64;  // wavefronts per i-particle
      __syncthreads();
      if ((t & 63) == 0) {
#pragma unroll
        for (int c = 0; c < 7; ++c) red[(t >> 6) * 7 + c] = v[c];
      }
      __syncthreads();
      if (sub == 0) {
        const int w0 = t >> 6;
#pragma unroll
        for (int c = 0; c < 7; ++c) {
          double s = red[w0 * 7 + c];
#pragma unroll
          for (int w = 1; w < NW; ++w) s += red[(w0 + w) * 7 + c];
          v[c] = s;
        }
      }
    }
    const int64_t k = k0 + kk * SLOTS + slot;
    if (sub == 0 && irow[kk] >= 0) {
      if (final_out) {
        const double self = (e2 > 0 && smass) ? P::self_term(smass[irow[kk]], eps2) : 0.0;
        acc[3 * k] = v[0]; acc[3 * k + 1] = v[1]; acc[3 * k + 2] = v[2];
        jerk[3 * k] = v[3]; jerk[3 * k + 1] = v[4]; jerk[3 * k + 2] = v[5];
        pot[k] = -(v[6] - self);
      } else if constexpr (ATOMIC) {
        // the paper's alternative to the two-kernel sum: every j-subset adds
        // its part into the outputs (seeded by k_atomic_init) with device-scope
        // atomics, in whatever order the work items finish
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          atomicAdd(&acc[3 * k + c], v[c]);
          atomicAdd(&jerk[3 * k + c], v[3 + c]);
        }
        atomicAdd(&pot[k], -v[6]);
      } else {
#pragma unroll
        for (int c = 0; c < 7; ++c) part[c * n_act + k] = v[c];
      }
    }
  }
}

template <class P, int L, int T = kTile, int WG = kWG>
struct Smem {
  typename P::template JTileT<T> tile;
  double red[(L > 64 ? WG / 64 : 1) * 7];
};

// The items of one launch shape: (i-block, j-chunk) pairs taken from the
// work queue until none is left.
template <class P, int K, int L, bool MASK, int T = kTile, int WG = kWG, bool ATOMIC = false>
__device__ __forceinline__ void run_items(typename P::template JTileT<T>& tile, double* red, unsigned int& slot,
                                          const ForceArgs& a, int64_t n_act, int S) {
  constexpr int IB = (WG / L) * K;
  const int64_t n_iblk = (n_act + IB - 1) / IB;
  const int64_t items = n_iblk * S;
  const int64_t clen = chunk_len(a.n, S, T);
  if (!queue_member(items)) return;
  int64_t w = queue_take(a.wq, slot, items, blockIdx.x);
  while (w < items) {
    const int64_t chunk = w / n_iblk;
    const int64_t iblk = w - chunk * n_iblk;
    const int64_t jb = chunk * clen;
    const int64_t je = jb + clen < a.n ? jb + clen : a.n;
    process_item<P, K, L, MASK, T, WG, ATOMIC>(tile, red, a.pos, a.vel, a.mass, a.ipos ? a.ipos : a.pos,
                                a.ivel ? a.ivel : a.vel, a.no_self ? nullptr : a.mass, jb, je, a.active, n_act, iblk * IB,
                                a.eps2, S == 1, a.acc, a.jerk, a.pot, a.part + chunk * 7 * n_act, a.row_lo, a.row_hi,
                                a.err);
    w = queue_next(a.wq, slot, items, w + gridDim.x);
  }
  queue_done(a.wq, items);
}

// One shape (those outside the families below), with its j-tile length T
// and workgroup size WG.
template <class P, int K, int L, bool MASK, int T = kTile, int WG = kWG>
__global__ __launch_bounds__(WG) void k_forces(ForceArgs a) {
  __shared__ Smem<P, L, T, WG> sm;
  __shared__ unsigned int slot;
  constexpr int IB = (WG / L) * K;
  int64_t n_act = a.n_active;
  int S = a.S;
  if (a.n_active_dev) {
    const int64_t d = *a.n_active_dev;
    if (d < a.act_lo || (d > a.n_active && !a.last)) return;  // another regime's launch
    n_act = d < n_act ? (d < 0 ? 0 : d) : n_act;
    S = choose_S(n_act, IB, target_for(a, d), a.n, T);
    if (a.s_dev && blockIdx.x == 0 && threadIdx.x == 0) *a.s_dev = S;  // for the shared reduce
  }
  run_items<P, K, L, MASK, T, WG>(sm.tile, sm.red, slot, a, n_act, S);
}

// The shape of a family launch for count d (unrolled like target_for).
__device__ __forceinline__ int shape_for(const ForceArgs& a, int64_t d) {
  int t = a.shape;
#pragma unroll
  for (int r = 0; r < kMaxSubRegimes; ++r)
    if (r < a.n_sub && d >= a.sub_lo[r]) t = a.sub_shape[r];
  return t;
}

// A kernel family (family_of): the shape -- fixed by the host, or in
// device-count mode the one of the regime holding the count -- selects one
// of the compiled bodies, so the regimes of a block step share one launch
// whatever their shapes.  Every body is the single-shape kernel's, so a
// shape gives the same sums in either kernel.
template <class P, int FAM, bool MASK, bool ATOMIC = false>
__global__ __launch_bounds__(kWG) void k_forces_fam(ForceArgs a) {
  __shared__ Smem<P, 256> sm;
  __shared__ unsigned int slot;
  int64_t n_act = a.n_active;
  int S = a.S;
  int shape = a.shape;
  if (a.n_active_dev) {
    const int64_t d = *a.n_active_dev;
    if (d < a.act_lo || (d > a.n_active && !a.last)) return;  // another launch's range
    n_act = d < n_act ? (d < 0 ? 0 : d) : n_act;
    shape = shape_for(a, d);
    const int K = shape >> 16, L = shape & 0xffff;
    S = choose_S(n_act, (kWG / L) * K, target_for(a, d), a.n);
    if (a.s_dev && blockIdx.x == 0 && threadIdx.x == 0) *a.s_dev = S;
  }
#define NB_RUN(KK, LL)                                                           \
  if (shape == shape_code(KK, LL)) {                                             \
    run_items<P, KK, LL, MASK, kTile, kWG, ATOMIC>(sm.tile, sm.red, slot, a, n_act, S); \
    return;                                                                      \
  }
  NB_RUN(1, 1) NB_RUN(1, 4) NB_RUN(1, 16) NB_RUN(1, 64) NB_RUN(1, 256)
  if constexpr (FAM == 2 && !MASK) {
    NB_RUN(2, 1) NB_RUN(2, 4) NB_RUN(2, 16)
  }
  if constexpr (FAM == 4 && !MASK) {
    NB_RUN(4, 4)
  }
#undef NB_RUN
  // a shape outside the family (the host never launches one): no items, queue untouched
}

// Fixed-order sum of the S partial blocks, self-term removal, output.
// With a device count and s_dev set, one reduce serves every regime of the
// call: the regime that worked left its S in *s_dev.
template <class P>
__global__ __launch_bounds__(256) void k_reduce(ForceArgs a, int S_host, int IB) {
  int64_t n_act = a.n_active;
  int S = S_host;
  if (a.n_active_dev) {
    const int64_t d = *a.n_active_dev;
    if (a.s_dev) {
      n_act = d < n_act ? (d < 0 ? 0 : d) : n_act;
      S = *a.s_dev;
    } else {
      if (d < a.act_lo || (d > a.n_active && !a.last)) return;
      n_act = d < n_act ? (d < 0 ? 0 : d) : n_act;
      S = choose_S(n_act, IB, target_for(a, d), a.n);
    }
  }
  if (S <= 1) return;
  const int64_t total = 7 * n_act;
  const bool self_on = P::eps(a.eps2) > 0;
  // g lanes per output (a power of two dividing the 256-thread block, so the
  // index below is the same across each output's lanes)
  const int g = chunk_lanes(S);
  const int lg = __builtin_ctz(g);
  const int lane = threadIdx.x & (g - 1);
  for (int64_t idx = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> lg; idx < total;
       idx += ((int64_t)gridDim.x * blockDim.x) >> lg) {
    const int64_t c = idx / n_act;
    const int64_t k = idx - c * n_act;
    const double s = sum_blocks(a.part + c * n_act + k, 7 * n_act, S, lane, g);
    if (lane != 0) continue;
    if (!row_in_range(a.active[k], a.row_lo, a.row_hi)) continue;  // skipped row (flagged by the force pass)
    if (c < 3) {
      a.acc[3 * k + c] = s;
    } else if (c < 6) {
      a.jerk[3 * k + c - 3] = s;
    } else {
      const double self = (self_on && !a.no_self) ? P::self_term(a.mass[a.active[k]], a.eps2) : 0.0;
      a.pot[k] = -(s - self);
    }
  }
}


// Block steps: the fixed-order sum of the S partial blocks of every active
// row (the same sums, lane for lane, as k_reduce) followed by that row's
// Hermite correction (the same arithmetic as the corrector kernel), so a
// block step runs one kernel after its force pass instead of two.  Each of a
// row's 7 outputs is summed by its own group of g = chunk_lanes(S) lanes, as
// in k_reduce, so a block takes R = 256 / (7 g) rows at a time (at least
// one): the sums of a pass run side by side, never one after another.  With
// S = 1 the force kernel has written the final rows and only the
// correction runs.
constexpr int kReduceCorrectThreads = 512;

template <class P>
__global__ __launch_bounds__(kReduceCorrectThreads) void k_reduce_correct(ForceArgs a, StepArgs s) {
  int64_t n_act = a.n_active;
  int S = 1;
  if (a.n_active_dev) {
    const int64_t d = *a.n_active_dev;
    n_act = d < n_act ? (d < 0 ? 0 : d) : n_act;
    S = a.s_dev ? *a.s_dev : 1;
  }
  if (s.step_dev && n_act > 0 && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(s.step_dev, 1ull);
  const bool self_on = P::eps(a.eps2) > 0;
  // g lanes per row (the lane grouping of sum_blocks, so every sum is the one
  // k_reduce forms); each group adds all seven outputs of its row, two
  // blocks ahead so the loads of both are in flight together
  const int g = S > 1 ? chunk_lanes(S) : 1;
  const int lane = threadIdx.x & (g - 1);
  // wavefronts are dealt to the blocks in turn (a few rows then run on as
  // many compute units), rows consecutive within a wavefront (coalesced
  // when g is small)
  const int rpw = 64 / g;
  const int64_t wave = (int64_t)(threadIdx.x >> 6) * gridDim.x + blockIdx.x;
  const int64_t nwave = (int64_t)(kReduceCorrectThreads >> 6) * gridDim.x;
  const int64_t stride = 7 * n_act;
  for (int64_t k = wave * rpw + (threadIdx.x & 63) / g; k < n_act; k += nwave * rpw) {
    const int64_t i = a.active[k];
    double v[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) v[c] = 0.0;
    if (S > 1) {
      const double* p = a.part + k;
      int ch = lane;
      for (; ch + g < S; ch += 2 * g) {
        double x[7], y[7];
#pragma unroll
        for (int c = 0; c < 7; ++c) {
          x[c] = p[(int64_t)ch * stride + c * n_act];
          y[c] = p[(int64_t)(ch + g) * stride + c * n_act];
        }
#pragma unroll
        for (int c = 0; c < 7; ++c) {
          v[c] += x[c];
          v[c] += y[c];
        }
      }
      if (ch < S) {
#pragma unroll
        for (int c = 0; c < 7; ++c) v[c] += p[(int64_t)ch * stride + c * n_act];
      }
      for (int m = g >> 1; m > 0; m >>= 1) {
#pragma unroll
        for (int c = 0; c < 7; ++c) v[c] += __shfl_xor(v[c], m);
      }
    }
    if (lane != 0) continue;
    if (!row_in_range(i, a.row_lo, a.row_hi)) {
      if (a.err) atomicOr(a.err, kErrActiveRange);
      continue;
    }
    double a1[3], j1[3];
    if (S > 1) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        a1[c] = v[c];
        j1[c] = v[3 + c];
        a.acc[3 * k + c] = a1[c];
        a.jerk[3 * k + c] = j1[c];
      }
      const double self = (self_on && !a.no_self) ? P::self_term(a.mass[i], a.eps2) : 0.0;
      a.pot[k] = -(v[6] - self);
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        a1[c] = a.acc[3 * k + c];
        j1[c] = a.jerk[3 * k + c];
      }
    }
    correct_particle(i, a1, j1, s.pos_p, s.vel_p, s.pos, s.vel, s.acc, s.jerk, s.t_tick, s.level, s.eta, s.dt_max,
                     s.max_level, s.clamp_dev);
  }
}

// ------------------------------------------------------- scalar j-path -----
// Variant of the i-parallel layout (L = 1) without LDS: the j-records are
// first converted once per call into the kernel's layout (a mirror array),
// and every wavefront then walks them with a wave-uniform index, so the
// compiler reads them through the scalar data cache into SGPRs (one-ahead
// prefetch).  No barriers, no LDS, no VGPRs for j-data; the VALU
// instructions take their j operand from an SGPR.
template <class P>
__global__ __launch_bounds__(256) void k_mirror(const double* __restrict__ pos, const double* __restrict__ vel,
                                                const double* __restrict__ mass, int64_t n,
                                                typename P::JReg* __restrict__ rec) {
  // records 0..n-1 and one zero padding record at n (read by the prefetch
  // of the last pair, never used)
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j <= n; j += (int64_t)gridDim.x * 256)
    rec[j] = P::load(pos, vel, mass, j, j < n);
}

template <class P, int K, bool MASK, int WG = kWG>
__device__ __forceinline__ void process_item_sj(const typename P::JReg* __restrict__ rec,
                                                const double* __restrict__ ipos, const double* __restrict__ ivel,
                                                const double* __restrict__ smass, int64_t jbeg, int64_t jend,
                                                const int32_t* __restrict__ active, int64_t n_act, int64_t k0,
                                                double eps2, bool final_out, double* __restrict__ acc,
                                                double* __restrict__ jerk, double* __restrict__ pot,
                                                double* __restrict__ part, int64_t row_lo,
                                                int64_t row_hi, unsigned int* err) {
  constexpr int RUN = P::kRun;  // pairs per float run
  const int t = threadIdx.x;
  typename P::IPart I[K];
  int64_t irow[K];
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    const int64_t k = k0 + kk * WG + t;
    irow[kk] = (k < n_act) ? checked_row(active, k, row_lo, row_hi, err) : -1;
    I[kk] = P::load_i(ipos, ivel, irow[kk] >= 0 ? irow[kk] : 0);
  }
  const typename P::T e2 = in_vgpr(P::eps(eps2));
  typename P::T A[K][7];
  typename P::Tot Tt[K];
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    P::zero(Tt[kk]);
#pragma unroll
    for (int c = 0; c < 7; ++c) A[kk][c] = 0;
  }
  if (jbeg < jend) {
    typename P::JReg nxt = rec[jbeg];
    for (int64_t base = jbeg; base < jend; base += kTile) {
      if (base + kTile <= jend) {
        // the prefetch of the tile's last pair wraps to jbeg on the last tile;
        // the test is kept on 32-bit uniform values so it stays on the scalar
        // unit (an unclamped index made the compiler hoist loads further ahead
        // at a cost of 14 VGPRs, one resident wave per SIMD, for K = 2)
        const bool last = base + kTile >= jend;
#pragma unroll 1
        for (int jb = 0; jb < kTile; jb += RUN) {
#pragma unroll NB_JJ_UNROLL
          for (int jj = jb; jj < jb + RUN; ++jj) {
            const typename P::JReg r = nxt;
            nxt = rec[(jj + 1 < kTile || !last) ? base + jj + 1 : jbeg];
            P::template pair_reg<MASK>(r, I, e2, A, K);
          }
          if constexpr (RUN < kTile) {
            if (jb + RUN < kTile) {
#pragma unroll
              for (int kk = 0; kk < K; ++kk) P::fold_run(Tt[kk], A[kk]);
            }
          }
        }
      } else {
        const int cnt = (int)(jend - base);
        for (int o = 0; o < cnt; ++o) {
          const typename P::JReg r = nxt;
          nxt = rec[o + 1 < cnt ? base + o + 1 : jbeg];
          P::template pair_reg<MASK>(r, I, e2, A, K);
          if constexpr (RUN < kTile) {
            if ((o & (RUN - 1)) == RUN - 1) {
#pragma unroll
              for (int kk = 0; kk < K; ++kk) P::fold_run(Tt[kk], A[kk]);
            }
          }
        }
      }
#pragma unroll
      for (int kk = 0; kk < K; ++kk) P::fold(Tt[kk], A[kk]);
    }
  }
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    const int64_t k = k0 + kk * WG + t;
    if (irow[kk] >= 0) {
      double v[7];
#pragma unroll
      for (int c = 0; c < 7; ++c) v[c] = P::value(Tt[kk], c);
      if (final_out) {
        const double self = (e2 > 0 && smass) ? P::self_term(smass[irow[kk]], eps2) : 0.0;
        acc[3 * k] = v[0]; acc[3 * k + 1] = v[1]; acc[3 * k + 2] = v[2];
        jerk[3 * k] = v[3]; jerk[3 * k + 1] = v[4]; jerk[3 * k + 2] = v[5];
        pot[k] = -(v[6] - self);
      } else {
#pragma unroll
        for (int c = 0; c < 7; ++c) part[c * n_act + k] = v[c];
      }
    }
  }
}

// Waves per SIMD the scalar j-path asks the register allocator for: with
// two i-particles per lane the float kernels then fit five waves (86
// VGPRs), measured 12% faster than four waves (110 VGPRs) with a deeper
// scalar-load pipeline.
template <class P, int K>
struct SjWaves {
  static constexpr int value = (K == 2 && sizeof(typename P::T) == 4) ? 5 : 1;
};

template <class P, int K, bool MASK, int WG = kWG>
__global__ __launch_bounds__(WG, (SjWaves<P, K>::value)) void k_forces_sj(ForceArgs a,
                                                                       const typename P::JReg* __restrict__ rec) {
  constexpr int IB = WG * K;
  int64_t n_act = a.n_active;
  int S = a.S;
  if (a.n_active_dev) {
    const int64_t d = *a.n_active_dev;
    if (d < a.act_lo || (d > a.n_active && !a.last)) return;
    n_act = d < n_act ? (d < 0 ? 0 : d) : n_act;
    S = choose_S(n_act, IB, target_for(a, d), a.n);
    if (a.s_dev && blockIdx.x == 0 && threadIdx.x == 0) *a.s_dev = S;  // for the shared reduce
  }
  const int64_t n_iblk = (n_act + IB - 1) / IB;
  const int64_t items = n_iblk * S;
  const int64_t clen = chunk_len(a.n, S);
  __shared__ unsigned int slot;
  if (!queue_member(items)) return;
  int64_t w = queue_take(a.wq, slot, items, blockIdx.x);
  while (w < items) {
    const int64_t chunk = w / n_iblk;
    const int64_t iblk = w - chunk * n_iblk;
    const int64_t jb = chunk * clen;
    const int64_t je = jb + clen < a.n ? jb + clen : a.n;
    process_item_sj<P, K, MASK, WG>(rec, a.ipos ? a.ipos : a.pos, a.ivel ? a.ivel : a.vel, a.no_self ? nullptr : a.mass,
                                jb, je, a.active, n_act, iblk * IB, a.eps2, S == 1,
                                a.acc, a.jerk, a.pot, a.part + chunk * 7 * n_act, a.row_lo, a.row_hi, a.err);
    w = queue_next(a.wq, slot, items, w + gridDim.x);
  }
  queue_done(a.wq, items);
}


// Hybrid of the two j-paths for the mixed policy (launch shape L = -1):
// positions come through the scalar cache (they feed double subtractions,
// which never dual-issue anyway) while velocities and masses are staged per
// tile into LDS, so the velocity differences and m q read VGPR operands and
// can pair with their neighbours.
template <int K>
__device__ __forceinline__ void process_item_hy(const Mixed::JReg* __restrict__ rec, float4* vm_tile,
                                                const double* __restrict__ ipos, const double* __restrict__ ivel,
                                                const double* __restrict__ smass, int64_t jbeg, int64_t jend,
                                                const int32_t* __restrict__ active, int64_t n_act, int64_t k0,
                                                double eps2, bool final_out, double* __restrict__ acc,
                                                double* __restrict__ jerk, double* __restrict__ pot,
                                                double* __restrict__ part, int64_t row_lo,
                                                int64_t row_hi, unsigned int* err) {
  using P = Mixed;
  constexpr int RUN = P::kRun;  // pairs per float run
  const int t = threadIdx.x;
  P::IPart I[K];
  int64_t irow[K];
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    const int64_t k = k0 + kk * kWG + t;
    irow[kk] = (k < n_act) ? checked_row(active, k, row_lo, row_hi, err) : -1;
    I[kk] = P::load_i(ipos, ivel, irow[kk] >= 0 ? irow[kk] : 0);
  }
  const float e2 = in_vgpr(P::eps(eps2));
  float A[K][7];
  P::Tot Tt[K];
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    P::zero(Tt[kk]);
#pragma unroll
    for (int c = 0; c < 7; ++c) A[kk][c] = 0;
  }
  for (int64_t base = jbeg; base < jend; base += kTile) {
    __syncthreads();  // every lane is done with the previous tile
    {
      const int64_t j = base + t;
      const P::JReg r = rec[j < jend ? j : jend];  // record jend exists (padding)
      vm_tile[t] = make_float4(r.vx, r.vy, r.vz, j < jend ? r.m : 0.0f);
    }
    __syncthreads();
    double2 nxy = make_double2(rec[base].x, rec[base].y);
    double nz = rec[base].z;
    if (base + kTile <= jend) {
#pragma unroll 1
      for (int jb = 0; jb < kTile; jb += RUN) {
#pragma unroll NB_JJ_UNROLL
        for (int jj = jb; jj < jb + RUN; ++jj) {
          const double2 xy = nxy;
          const double z = nz;
          const int64_t jn = base + jj + 1 < jend ? base + jj + 1 : jbeg;
          nxy = make_double2(rec[jn].x, rec[jn].y);
          nz = rec[jn].z;
          const float4 vm = vm_tile[jj];
#pragma unroll
          for (int kk = 0; kk < K; ++kk) P::pair<false>(I[kk], xy, z, vm, e2, A[kk]);
        }
        if constexpr (RUN < kTile) {
          if (jb + RUN < kTile) {
#pragma unroll
            for (int kk = 0; kk < K; ++kk) P::fold_run(Tt[kk], A[kk]);
          }
        }
      }
    } else {
      const int cnt = (int)(jend - base);
      for (int jj = 0; jj < cnt; ++jj) {
        const double2 xy = nxy;
        const double z = nz;
        const int64_t jn = base + jj + 1 < jend ? base + jj + 1 : jbeg;
        nxy = make_double2(rec[jn].x, rec[jn].y);
        nz = rec[jn].z;
        const float4 vm = vm_tile[jj];
#pragma unroll
        for (int kk = 0; kk < K; ++kk) P::pair<false>(I[kk], xy, z, vm, e2, A[kk]);
        if constexpr (RUN < kTile) {
          if ((jj & (RUN - 1)) == RUN - 1) {
#pragma unroll
            for (int kk = 0; kk < K; ++kk) P::fold_run(Tt[kk], A[kk]);
          }
        }
      }
    }
#pragma unroll
    for (int kk = 0; kk < K; ++kk) P::fold(Tt[kk], A[kk]);
  }
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    const int64_t k = k0 + kk * kWG + t;
    if (irow[kk] >= 0) {
      double v[7];
#pragma unroll
      for (int c = 0; c < 7; ++c) v[c] = P::value(Tt[kk], c);
      if (final_out) {
        const double self = (e2 > 0 && smass) ? P::self_term(smass[irow[kk]], eps2) : 0.0;
        acc[3 * k] = v[0]; acc[3 * k + 1] = v[1]; acc[3 * k + 2] = v[2];
        jerk[3 * k] = v[3]; jerk[3 * k + 1] = v[4]; jerk[3 * k + 2] = v[5];
        pot[k] = -(v[6] - self);
      } else {
#pragma unroll
        for (int c = 0; c < 7; ++c) part[c * n_act + k] = v[c];
      }
    }
  }
}

template <int K>
__global__ __launch_bounds__(kWG, (K == 2 ? 5 : 1)) void k_forces_hy(ForceArgs a, const Mixed::JReg* __restrict__ rec) {
  __shared__ float4 vm_tile[kTile];
  constexpr int IB = kWG * K;
  int64_t n_act = a.n_active;
  int S = a.S;
  if (a.n_active_dev) {
    const int64_t d = *a.n_active_dev;
    if (d < a.act_lo || (d > a.n_active && !a.last)) return;
    n_act = d < n_act ? (d < 0 ? 0 : d) : n_act;
    S = choose_S(n_act, IB, target_for(a, d), a.n);
    if (a.s_dev && blockIdx.x == 0 && threadIdx.x == 0) *a.s_dev = S;  // for the shared reduce
  }
  const int64_t n_iblk = (n_act + IB - 1) / IB;
  const int64_t items = n_iblk * S;
  const int64_t clen = chunk_len(a.n, S);
  __shared__ unsigned int slot;
  if (!queue_member(items)) return;
  int64_t w = queue_take(a.wq, slot, items, blockIdx.x);
  while (w < items) {
    const int64_t chunk = w / n_iblk;
    const int64_t iblk = w - chunk * n_iblk;
    const int64_t jb = chunk * clen;
    const int64_t je = jb + clen < a.n ? jb + clen : a.n;
    process_item_hy<K>(rec, vm_tile, a.ipos ? a.ipos : a.pos, a.ivel ? a.ivel : a.vel,
                       a.no_self ? nullptr : a.mass, jb, je, a.active, n_act, iblk * IB, a.eps2, S == 1,
                       a.acc, a.jerk, a.pot, a.part + chunk * 7 * n_act, a.row_lo, a.row_hi, a.err);
    w = queue_next(a.wq, slot, items, w + gridDim.x);
  }
  queue_done(a.wq, items);
}

// ---------------------------------------------------------------- batch ----
template <class P, int K, int L, bool MASK>
__global__ __launch_bounds__(kWG) void k_forces_batch(const BatchItem* __restrict__ items, int n_items,
                                                      const int* __restrict__ n_items_dev,
                                                      const BatchSys* __restrict__ sys, const double* pos,
                                                      const double* vel, const double* mass,
                                                      const int32_t* active, double* acc, double* jerk,
                                                      double* pot, double* part, unsigned int* err) {
  __shared__ Smem<P, L> sm;
  constexpr int IB = (kWG / L) * K;
  if (n_items_dev) {
    const int d = *n_items_dev;
    n_items = d < n_items ? (d < 0 ? 0 : d) : n_items;
  }
  for (int w = blockIdx.x; w < n_items; w += gridDim.x) {
    const BatchItem it = items[w];
    const BatchSys sy = sys[it.sys];
    const int64_t nj = sy.j1 - sy.j0;
    const int64_t n_act = sy.a1 - sy.a0;
    const int64_t clen = chunk_len(nj, it.nchunk);
    const int64_t jb = sy.j0 + (int64_t)it.chunk * clen;
    const int64_t je = jb + clen < sy.j1 ? jb + clen : sy.j1;
    process_item<P, K, L, MASK>(sm.tile, sm.red, pos, vel, mass, pos, vel, mass, jb, je, active + sy.a0, n_act,
                                (int64_t)it.iblk * IB, sy.eps2, it.nchunk == 1, acc + 3 * sy.a0,
                                jerk + 3 * sy.a0, pot + sy.a0,
                                part + (sy.part_off + (int64_t)it.chunk * n_act) * 7, sy.j0, sy.j1, err);
  }
}

// The same work list on the scalar j-path: j-records of the whole batch come
// from one mirror through the scalar cache, each system's rows with its own
// softening; an i-block is kBatchSjWG * K of the system's active rows.
template <class P, int K, bool MASK>
__global__ __launch_bounds__(kBatchSjWG, (SjWaves<P, K>::value)) void k_forces_batch_sj(
    const BatchItem* __restrict__ items, int n_items, const int* __restrict__ n_items_dev,
    const BatchSys* __restrict__ sys, const typename P::JReg* __restrict__ rec, const double* pos, const double* vel,
    const double* mass, const int32_t* active, double* acc, double* jerk, double* pot, double* part,
    unsigned int* err) {
  constexpr int IB = kBatchSjWG * K;
  if (n_items_dev) {
    const int d = *n_items_dev;
    n_items = d < n_items ? (d < 0 ? 0 : d) : n_items;
  }
  for (int w = blockIdx.x; w < n_items; w += gridDim.x) {
    const BatchItem it = items[w];
    const BatchSys sy = sys[it.sys];
    const int64_t nj = sy.j1 - sy.j0;
    const int64_t n_act = sy.a1 - sy.a0;
    const int64_t clen = chunk_len(nj, it.nchunk);
    const int64_t jb = sy.j0 + (int64_t)it.chunk * clen;
    const int64_t je = jb + clen < sy.j1 ? jb + clen : sy.j1;
    process_item_sj<P, K, MASK, kBatchSjWG>(rec, pos, vel, mass, jb, je, active + sy.a0, n_act, (int64_t)it.iblk * IB, sy.eps2,
                                it.nchunk == 1, acc + 3 * sy.a0, jerk + 3 * sy.a0, pot + sy.a0,
                                part + (sy.part_off + (int64_t)it.chunk * n_act) * 7, sy.j0, sy.j1, err);
  }
}

// Systems with more than one chunk (grid y) over a few workgroups each (grid
// x); each output is the fixed-order sum of its chunks.
template <class P>
__global__ __launch_bounds__(256) void k_batch_reduce(const BatchSys* __restrict__ sys,
                                                      const int32_t* __restrict__ nchunk, int n_sys,
                                                      const double* mass, const int32_t* active, double* acc,
                                                      double* jerk, double* pot, const double* part) {
  for (int cs = blockIdx.y; cs < n_sys; cs += gridDim.y) {  // more systems than grid rows
  const BatchSys sy = sys[cs];
  const int S = nchunk[cs];
  if (S <= 1) continue;
  const int64_t n_act = sy.a1 - sy.a0;
  const double* pb = part + sy.part_off * 7;
  const bool self_on = P::eps(sy.eps2) > 0;
  const int g = chunk_lanes(S);
  const int lg = __builtin_ctz(g);
  const int lane = threadIdx.x & (g - 1);
  for (int64_t idx = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> lg; idx < 7 * n_act;
       idx += ((int64_t)gridDim.x * blockDim.x) >> lg) {
    const int64_t c = idx / n_act;
    const int64_t k = idx - c * n_act;
    const double s = sum_blocks(pb + c * n_act + k, 7 * n_act, S, lane, g);
    if (lane != 0) continue;
    const int64_t row = sy.a0 + k;
    if (!row_in_range(active[row], sy.j0, sy.j1)) continue;  // skipped row (flagged by the force pass)
    if (c < 3) {
      acc[3 * row + c] = s;
    } else if (c < 6) {
      jerk[3 * row + c - 3] = s;
    } else {
      const double self = self_on ? P::self_term(mass[active[row]], sy.eps2) : 0.0;
      pot[row] = -(s - self);
    }
  }
  }
}


// Batched block step: the chunk sums of k_batch_reduce and the corrector in
// one pass.  Grid row y is system y (no search for a row's system); its
// blocks stride over the system's active rows with g lanes per row (the
// grouping of sum_blocks, so every sum is the one k_batch_reduce forms),
// each group adding all seven outputs of its row two chunks ahead; lane 0
// of the group then corrects the particle.
template <class P>
__global__ __launch_bounds__(256) void k_batch_reduce_correct(const BatchSys* __restrict__ sys,
                                                              const int32_t* __restrict__ nchunk, int C,
                                                              const int64_t* __restrict__ n_act_dev,
                                                              const double* __restrict__ mass,
                                                              const int32_t* __restrict__ active, double* acc1,
                                                              double* jerk1, double* pot1, const double* part,
                                                              StepArgs s, unsigned int* err) {
  if (s.step_dev && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0 && *n_act_dev > 0)
    atomicAdd(s.step_dev, 1ull);
  for (int cs = blockIdx.y; cs < C; cs += gridDim.y) {  // more systems than grid rows
  const BatchSys sy = sys[cs];
  const int64_t na = sy.a1 - sy.a0;
  if (na <= 0) continue;
  const int S = nchunk[cs];
  const int g = S > 1 ? chunk_lanes(S) : 1;
  const int lane = threadIdx.x & (g - 1);
  // wavefronts dealt to the system's blocks in turn, rows consecutive within one
  const int rpw = 64 / g;
  const int64_t wave = (int64_t)(threadIdx.x >> 6) * gridDim.x + blockIdx.x;
  const int64_t nwave = (int64_t)4 * gridDim.x;
  const double* pb = part + sy.part_off * 7;
  const int64_t stride = 7 * na;
  for (int64_t kk = wave * rpw + (threadIdx.x & 63) / g; kk < na; kk += nwave * rpw) {
    const int64_t k = sy.a0 + kk;
    const int64_t i = active[k];
    double v[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) v[c] = 0.0;
    if (S > 1) {
      const double* p = pb + kk;
      int ch = lane;
      for (; ch + g < S; ch += 2 * g) {
        double x[7], y[7];
#pragma unroll
        for (int c = 0; c < 7; ++c) {
          x[c] = p[(int64_t)ch * stride + c * na];
          y[c] = p[(int64_t)(ch + g) * stride + c * na];
        }
#pragma unroll
        for (int c = 0; c < 7; ++c) {
          v[c] += x[c];
          v[c] += y[c];
        }
      }
      if (ch < S) {
#pragma unroll
        for (int c = 0; c < 7; ++c) v[c] += p[(int64_t)ch * stride + c * na];
      }
      for (int m = g >> 1; m > 0; m >>= 1) {
#pragma unroll
        for (int c = 0; c < 7; ++c) v[c] += __shfl_xor(v[c], m);
      }
    }
    if (lane != 0) continue;
    if (!row_in_range(i, sy.j0, sy.j1)) {
      if (err) atomicOr(err, kErrActiveRange);
      continue;
    }
    double a1[3], j1[3];
    if (S > 1) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        a1[c] = v[c];
        j1[c] = v[3 + c];
        acc1[3 * k + c] = a1[c];
        jerk1[3 * k + c] = j1[c];
      }
      const double self = P::eps(sy.eps2) > 0 ? P::self_term(mass[i], sy.eps2) : 0.0;
      pot1[k] = -(v[6] - self);
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        a1[c] = acc1[3 * k + c];
        j1[c] = jerk1[3 * k + c];
      }
    }
    correct_particle(i, a1, j1, s.pos_p, s.vel_p, s.pos, s.vel, s.acc, s.jerk, s.t_tick, s.level, s.eta, s.dt_max,
                     s.max_level, s.clamp_dev);
  }
  }
}

// ------------------------------------------------------------ batch plan ---
// One workgroup turns the scheduled active set of a batch of independent
// systems into the work list of the batched force kernel, entirely on the
// device (so a block step over the batch can be captured in a graph):
//   per system: its rows of the (ascending) active list by binary search,
//   n_iblk = ceil(n_act / IB); a common chunk length J chosen so the whole
//   batch yields about `target` items; S_c = ceil(nj / J) chunks (at least
//   one tile each); items (system, i-block, chunk) and partial-sum offsets
//   by exclusive scans over the systems.
// The searches start in LDS, on every stride-th entry of the active list
// (one entry per thread), and finish within one stride in global memory:
// log2(stride) dependent loads instead of log2(n_active).  The sums and
// scans over the threads use shuffles within each wavefront and one
// exchange of the wavefront totals.
constexpr int kPlanThreads = 1024;
constexpr int kPlanWaves = kPlanThreads / 64;

// First index k in [0, n) with active[k] >= key (n if none).  samp[t] =
// active[t * stride] for t < ns = ceil(n / stride).
__device__ int64_t plan_lower_bound(const int32_t* active, int64_t n, const int32_t* samp, int ns, int64_t stride,
                                    int64_t key) {
  int lo = 0, hi = ns;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if ((int64_t)samp[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  // every entry up to (lo - 1) stride is below key; entry lo stride (or n) is not
  if (lo == 0) return 0;
  int64_t a = (int64_t)(lo - 1) * stride + 1;
  int64_t b = lo < ns ? (int64_t)lo * stride : n;
  while (a < b) {
    const int64_t mid = (a + b) >> 1;
    if ((int64_t)active[mid] < key) a = mid + 1;
    else b = mid;
  }
  return a;
}

// Sum of one value per thread.
__device__ int64_t plan_sum(int64_t v, int64_t* wred) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if (lane == 0) wred[wave] = v;
  __syncthreads();
  int64_t r = 0;
#pragma unroll
  for (int w = 0; w < kPlanWaves; ++w) r += wred[w];
  __syncthreads();  // wred is free again for the next call
  return r;
}

// Exclusive scan of one value per thread (thread order); returns the total.
__device__ int64_t plan_exscan(int64_t v, int64_t* wred, int64_t* excl) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int64_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wred[wave] = x;
  __syncthreads();
  int64_t before = 0, total = 0;
#pragma unroll
  for (int w = 0; w < kPlanWaves; ++w) {
    const int64_t t = wred[w];
    before += w < wave ? t : 0;
    total += t;
  }
  __syncthreads();
  *excl = before + x - v;
  return total;
}

__global__ __launch_bounds__(kPlanThreads) void k_batch_plan(const int64_t* __restrict__ off,
                                                            const double* __restrict__ eps2, int C,
                                                            const int32_t* __restrict__ active,
                                                            const int64_t* __restrict__ n_act_dev, int IB, int target,
                                                            BatchSys* __restrict__ sys, int32_t* __restrict__ nchunk,
                                                            BatchItem* __restrict__ items, int max_items,
                                                            int* __restrict__ n_items_dev, int64_t part_cap_rows) {
  __shared__ int64_t red[kPlanWaves];
  __shared__ int32_t samp[kPlanThreads];
  __shared__ int64_t J_s;
  int64_t n_act = *n_act_dev;
  if (n_act < 0) n_act = 0;
  const int per = (C + kPlanThreads - 1) / kPlanThreads;
  const int c0 = threadIdx.x * per;
  const int c1 = c0 + per < C ? c0 + per : C;
  // 1. active rows per system and the total work (i-slots x j)
  const int64_t stride = n_act > kPlanThreads ? (n_act + kPlanThreads - 1) / kPlanThreads : 1;
  const int ns = (int)((n_act + stride - 1) / stride);
  if ((int)threadIdx.x < ns) samp[threadIdx.x] = active[(int64_t)threadIdx.x * stride];
  __syncthreads();
  int64_t work = 0;
  int64_t a1 = c0 < c1 ? plan_lower_bound(active, n_act, samp, ns, stride, off[c0]) : 0;
  for (int c = c0; c < c1; ++c) {
    const int64_t a0 = a1;
    a1 = plan_lower_bound(active, n_act, samp, ns, stride, off[c + 1]);
    const int64_t nib = (a1 - a0 + IB - 1) / IB;
    work += nib * IB * (off[c + 1] - off[c]);
    sys[c].j0 = off[c];
    sys[c].j1 = off[c + 1];
    sys[c].a0 = a0;
    sys[c].a1 = a1;
    sys[c].eps2 = eps2[c];
  }
  const int64_t W = plan_sum(work, red);
  if (threadIdx.x == 0) {
    int64_t J = (W + (int64_t)IB * target - 1) / ((int64_t)IB * target);
    J = (J + kTile - 1) / kTile * kTile;
    J_s = J < kTile ? kTile : J;
  }
  __syncthreads();
  const int64_t J = J_s;
  // 2. chunks, items and partial rows per system
  int64_t my_items = 0, my_parts = 0;
  for (int c = c0; c < c1; ++c) {
    const int64_t nj = sys[c].j1 - sys[c].j0;
    const int64_t na = sys[c].a1 - sys[c].a0;
    int64_t S = (nj + J - 1) / J;
    const int64_t max_s = (nj + kTile - 1) / kTile;
    if (S > max_s) S = max_s;
    if (S < 1) S = 1;
    nchunk[c] = (int32_t)S;
    my_items += ((na + IB - 1) / IB) * S;
    if (S > 1) my_parts += S * na;
  }
  int64_t item_base, part_base;
  const int64_t total_items = plan_exscan(my_items, red, &item_base);
  const int64_t total_parts = plan_exscan(my_parts, red, &part_base);
  const bool fits = total_items <= max_items && total_parts <= part_cap_rows;
  // 3. the work list, system by system
  for (int c = c0; c < c1; ++c) {
    const int64_t na = sys[c].a1 - sys[c].a0;
    const int32_t S = fits ? nchunk[c] : 1;
    if (!fits) nchunk[c] = 1;
    const int64_t nib = (na + IB - 1) / IB;
    sys[c].part_off = (S > 1) ? part_base : 0;
    if (S > 1) part_base += (int64_t)S * na;
    if (fits) {
      for (int32_t ch = 0; ch < S; ++ch)
        for (int64_t b = 0; b < nib; ++b)
          items[item_base + (int64_t)ch * nib + b] = BatchItem{(int32_t)c, (int32_t)b, ch, S};
      item_base += nib * S;
    }
  }
  if (!fits) {
    // The bounds of the host sizing make this unreachable; fall back to one
    // chunk per system (no partials), written in a second ordered pass.
    __syncthreads();
    int64_t mine = 0;
    for (int c = c0; c < c1; ++c) mine += (sys[c].a1 - sys[c].a0 + IB - 1) / IB;
    int64_t base;
    const int64_t tot = plan_exscan(mine, red, &base);
    for (int c = c0; c < c1; ++c) {
      const int64_t nib = (sys[c].a1 - sys[c].a0 + IB - 1) / IB;
      for (int64_t b = 0; b < nib; ++b)
        if (base + b < max_items) items[base + b] = BatchItem{(int32_t)c, (int32_t)b, 0, 1};
      base += nib;
    }
    if (threadIdx.x == 0) *n_items_dev = (int)(tot < max_items ? tot : max_items);
  } else if (threadIdx.x == 0) {
    *n_items_dev = (int)total_items;
  }
}

// Seeds of the atomic j-split sum: zero acceleration and jerk, and the
// potential at +self term, so that after every subset has added -(its part)
// it is -(sum - self), as the fixed-order reduce writes it.
template <class P>
__global__ __launch_bounds__(256) void k_atomic_init(ForceArgs a) {
  const bool self_on = P::eps(a.eps2) > 0 && !a.no_self;
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < a.n_active; k += (int64_t)gridDim.x * 256) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      a.acc[3 * k + c] = 0.0;
      a.jerk[3 * k + c] = 0.0;
    }
    const int64_t i = a.active[k];
    a.pot[k] = (self_on && row_in_range(i, a.row_lo, a.row_hi)) ? P::self_term(a.mass[i], a.eps2) : 0.0;
  }
}

// ------------------------------------------------------------- dispatch ----
using ForceFn = void (*)(ForceArgs);
using BatchFn = void (*)(const BatchItem*, int, const int*, const BatchSys*, const double*, const double*,
                         const double*, const int32_t*, double*, double*, double*, double*, unsigned int*);

// Shapes with another j-tile length or workgroup size (no masked variant).
template <class P, int T, int WG>
ForceFn pick_force_tw(int K, int L) {
#define NB_CASE(KK, LL) \
  if (K == KK && L == LL) return k_forces<P, KK, LL, false, T, WG>;
  NB_CASE(1, 1) NB_CASE(1, 4) NB_CASE(1, 16) NB_CASE(2, 1) NB_CASE(2, 4)
#undef NB_CASE
  return nullptr;
}

// Single-shape kernels: the shapes no family holds.
template <class P, bool MASK>
ForceFn pick_force(int K, int L, int T = kTile, int WG = kWG) {
  if constexpr (!MASK) {
    if (T == 128 && WG == 256) return pick_force_tw<P, 128, 256>(K, L);
    if (T == 128 && WG == 128) return pick_force_tw<P, 128, 128>(K, L);
    if (T == 64 && WG == 64) return pick_force_tw<P, 64, 64>(K, L);
  }
  if (T != kTile || WG != kWG) return nullptr;
#define NB_CASE(KK, LL) \
  if (K == KK && L == LL) return k_forces<P, KK, LL, MASK>;
  NB_CASE(1, 2) NB_CASE(1, 8) NB_CASE(1, 32) NB_CASE(1, 128)
  if constexpr (!MASK) {
    NB_CASE(2, 2) NB_CASE(2, 8) NB_CASE(2, 32) NB_CASE(2, 64)
    NB_CASE(4, 1) NB_CASE(4, 2) NB_CASE(4, 8) NB_CASE(4, 16)
  }
#undef NB_CASE
  return nullptr;
}

template <class P, bool MASK>
ForceFn pick_fam(int fam) {
  if (fam == 1) return k_forces_fam<P, 1, MASK>;
  if constexpr (!MASK) {
    if (fam == 2) return k_forces_fam<P, 2, MASK>;
    if (fam == 4) return k_forces_fam<P, 4, MASK>;
  }
  return nullptr;
}

// The LDS kernel of a shape: its family's (cfg.fam, else the smallest
// family holding it), else its single-shape kernel.
template <class P, bool MASK>
ForceFn pick_lds(const Launch& cfg, int K) {
  const int fam = cfg.fam > 0 ? cfg.fam : (default_tile(cfg) ? family_of(K, cfg.L) : 0);
  return fam ? pick_fam<P, MASK>(fam) : pick_force<P, MASK>(K, cfg.L, cfg.T, cfg.WG);
}

template <class P, bool MASK>
using SjFn = void (*)(ForceArgs, const typename P::JReg*);

template <class P, bool MASK>
SjFn<P, MASK> pick_sj(int K, int WG = kWG) {
  if (WG == 128) {
    if constexpr (!MASK) {
      if (K == 1) return k_forces_sj<P, 1, MASK, 128>;
      if (K == 2) return k_forces_sj<P, 2, MASK, 128>;
    }
    return nullptr;
  }
  if (WG != kWG) return nullptr;
  if (K == 1) return k_forces_sj<P, 1, MASK>;
  if constexpr (!MASK) {
    if (K == 2) return k_forces_sj<P, 2, MASK>;
    if (K == 3) return k_forces_sj<P, 3, MASK>;
    if (K == 4) return k_forces_sj<P, 4, MASK>;
  }
  return nullptr;
}

template <class P, bool MASK>
hipError_t launch_sj_p(int K, int WG, const ForceArgs& a, hipStream_t st, int grid_override, int max_grid) {
  SjFn<P, MASK> fn = pick_sj<P, MASK>(K, WG);
  if (!fn || !a.rec) return hipErrorInvalidValue;
  typename P::JReg* rec = static_cast<typename P::JReg*>(a.rec);
  int64_t mg = (a.n + 255) / 256;
  if (mg > 8192) mg = 8192;
  hipLaunchKernelGGL(k_mirror<P>, dim3((int)mg), dim3(256), 0, st, a.pos, a.vel, a.mass, a.n, rec);
  Launch shape{K, 1, a.S};
  shape.WG = WG;
  int grid = grid_override > 0 ? grid_override : items_for(shape, a.n_active, a.S);
  if (max_grid > 0 && grid > max_grid) grid = max_grid;
  if (grid <= 0) return hipGetLastError();
  hipLaunchKernelGGL(fn, dim3(grid), dim3(WG), 0, st, a, rec);
  return hipGetLastError();
}

using HyFn = void (*)(ForceArgs, const Mixed::JReg*);
HyFn pick_hy(int K) {
  if (K == 1) return k_forces_hy<1>;
  if (K == 2) return k_forces_hy<2>;
  if (K == 3) return k_forces_hy<3>;
  if (K == 4) return k_forces_hy<4>;
  return nullptr;
}

template <class P>
using BatchSjFn = void (*)(const BatchItem*, int, const int*, const BatchSys*, const typename P::JReg*,
                           const double*, const double*, const double*, const int32_t*, double*, double*, double*,
                           double*, unsigned int*);

template <class P, bool MASK>
BatchSjFn<P> pick_batch_sj(int K) {
  if (K == 1) return k_forces_batch_sj<P, 1, MASK>;
  if constexpr (!MASK) {
    if (K == 2) return k_forces_batch_sj<P, 2, MASK>;
  }
  return nullptr;
}

template <class P, bool MASK>
hipError_t launch_batch_sj_p(int K, const BatchItem* items, int n_items, const int* n_items_dev, const BatchSys* sys,
                             void* rec_buf, int64_t n_total, const double* pos, const double* vel, const double* mass,
                             const int32_t* active, double* acc, double* jerk, double* pot, double* part,
                             int max_grid, unsigned int* err, hipStream_t st) {
  BatchSjFn<P> fn = pick_batch_sj<P, MASK>(K);
  if (!fn || !rec_buf) return hipErrorInvalidValue;
  typename P::JReg* rec = static_cast<typename P::JReg*>(rec_buf);
  int64_t mg = (n_total + 256) / 256;
  if (mg > 8192) mg = 8192;
  hipLaunchKernelGGL(k_mirror<P>, dim3((int)mg), dim3(256), 0, st, pos, vel, mass, n_total, rec);
  if (n_items <= 0) return hipGetLastError();
  int grid = n_items;
  if (max_grid > 0 && grid > max_grid) grid = max_grid;
  hipLaunchKernelGGL(fn, dim3(grid), dim3(kBatchSjWG), 0, st, items, n_items, n_items_dev, sys, rec, pos, vel, mass,
                     active, acc, jerk, pot, part, err);
  return hipGetLastError();
}

template <class P, bool MASK>
BatchFn pick_batch(int K, int L) {
#define NB_CASE(KK, LL) \
  if (K == KK && L == LL) return k_forces_batch<P, KK, LL, MASK>;
  NB_CASE(1, 1) NB_CASE(1, 4) NB_CASE(1, 16) NB_CASE(1, 64)
  if constexpr (!MASK) {
    NB_CASE(2, 1) NB_CASE(2, 4) NB_CASE(2, 16)
  }
#undef NB_CASE
  return nullptr;
}

template <class P>
ForceFn pick_fam_atomic(int fam) {
  if (fam == 1) return k_forces_fam<P, 1, false, true>;
  if (fam == 2) return k_forces_fam<P, 2, false, true>;
  return nullptr;
}

}  // namespace

bool atomic_split_supported(const Launch& c) {
  const int fam = default_tile(c) && c.L >= 1 ? family_of(c.K, c.L) : 0;
  return fam == 1 || fam == 2;
}

hipError_t launch_forces_atomic(int prec, const Launch& cfg, const ForceArgs& a, hipStream_t st, int max_grid) {
  if (!atomic_split_supported(cfg)) return hipErrorInvalidValue;
  const int fam = family_of(cfg.K, cfg.L);
  ForceFn fn = prec == NB_PREC_FP64 ? pick_fam_atomic<F64>(fam)
               : prec == NB_PREC_MIXED_DS ? pick_fam_atomic<MixedDS>(fam) : pick_fam_atomic<Mixed>(fam);
  if (!fn) return hipErrorInvalidValue;
  int64_t g0 = (a.n_active + 255) / 256;
  g0 = g0 < 1 ? 1 : (g0 > 1024 ? 1024 : g0);
  if (prec == NB_PREC_FP64)
    hipLaunchKernelGGL(k_atomic_init<F64>, dim3((unsigned)g0), dim3(256), 0, st, a);
  else if (prec == NB_PREC_MIXED_DS)
    hipLaunchKernelGGL(k_atomic_init<MixedDS>, dim3((unsigned)g0), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(k_atomic_init<Mixed>, dim3((unsigned)g0), dim3(256), 0, st, a);
  Launch shape = cfg;
  shape.S = a.S;
  int grid = items_for(shape, a.n_active, a.S);
  if (max_grid > 0 && grid > max_grid) grid = max_grid;
  if (grid <= 0) return hipGetLastError();
  ForceArgs b = a;
  b.shape = shape_code(cfg.K, cfg.L);
  hipLaunchKernelGGL(fn, dim3(grid), dim3(kWG), 0, st, b);
  return hipGetLastError();
}

bool launch_supported(const Launch& c) {
  if (c.S < 1) return false;
  if (c.L < 0) return pick_hy(c.K) != nullptr && default_tile(c);
  if (c.L == 0) return pick_sj<F64, false>(c.K, c.WG) != nullptr && c.T == kTile;
  if (default_tile(c) && family_of(c.K, c.L)) return true;
  return pick_force<F64, false>(c.K, c.L, c.T, c.WG) != nullptr;
}

size_t mirror_bytes(int prec, int64_t n) {
  const size_t rec = prec == NB_PREC_FP64 ? sizeof(F64::JReg)
                     : prec == NB_PREC_MIXED_DS ? sizeof(MixedDS::JReg) : sizeof(Mixed::JReg);
  return rec * (size_t)((n > 0 ? n : 1) + 1);  // one padding record
}

int items_for(const Launch& c, int64_t n_active, int S) {
  const int64_t IB = ib_of(c);
  return (int)(((n_active + IB - 1) / IB) * S);
}

hipError_t launch_forces(int prec, const Launch& cfg_in, bool mask, const ForceArgs& a, hipStream_t st,
                         int grid_override, int max_grid) {
  const Launch cfg = mask ? masked(cfg_in) : cfg_in;
  const int K = cfg.K;
  if (cfg.L < 0) {
    // hybrid path: mixed precision with eps2 > 0 only (otherwise the scalar j-path)
    if (prec != NB_PREC_MIXED || mask) {
      Launch c2 = cfg;
      c2.L = 0;
      return launch_forces(prec, c2, mask, a, st, grid_override, max_grid);
    }
    HyFn fn = pick_hy(K);
    if (!fn || !a.rec) return hipErrorInvalidValue;
    Mixed::JReg* rec = static_cast<Mixed::JReg*>(a.rec);
    int64_t mg = (a.n + 256) / 256;
    if (mg > 8192) mg = 8192;
    hipLaunchKernelGGL(k_mirror<Mixed>, dim3((int)mg), dim3(256), 0, st, a.pos, a.vel, a.mass, a.n, rec);
    int grid = grid_override > 0 ? grid_override : items_for(Launch{K, 1, a.S}, a.n_active, a.S);
    if (max_grid > 0 && grid > max_grid) grid = max_grid;
    if (grid <= 0) return hipGetLastError();
    hipLaunchKernelGGL(fn, dim3(grid), dim3(kWG), 0, st, a, rec);
    return hipGetLastError();
  }
  if (cfg.L == 0) {
    const int WG = cfg.WG;
    if (prec == NB_PREC_FP64)
      return mask ? launch_sj_p<F64, true>(K, WG, a, st, grid_override, max_grid)
                  : launch_sj_p<F64, false>(K, WG, a, st, grid_override, max_grid);
    if (prec == NB_PREC_MIXED_DS)
      return mask ? launch_sj_p<MixedDS, true>(K, WG, a, st, grid_override, max_grid)
                  : launch_sj_p<MixedDS, false>(K, WG, a, st, grid_override, max_grid);
    return mask ? launch_sj_p<Mixed, true>(K, WG, a, st, grid_override, max_grid)
                : launch_sj_p<Mixed, false>(K, WG, a, st, grid_override, max_grid);
  }
  ForceFn fn = nullptr;
  if (prec == NB_PREC_FP64)
    fn = mask ? pick_lds<F64, true>(cfg, K) : pick_lds<F64, false>(cfg, K);
  else if (prec == NB_PREC_MIXED_DS)
    fn = mask ? pick_lds<MixedDS, true>(cfg, K) : pick_lds<MixedDS, false>(cfg, K);
  else
    fn = mask ? pick_lds<Mixed, true>(cfg, K) : pick_lds<Mixed, false>(cfg, K);
  if (!fn) return hipErrorInvalidValue;
  Launch shape = cfg;
  shape.S = a.S;
  int grid = grid_override > 0 ? grid_override : items_for(shape, a.n_active, a.S);
  if (max_grid > 0 && grid > max_grid) grid = max_grid;
  if (grid <= 0) return hipSuccess;
  if (a.n_sub == 0 && a.shape == 0) {
    // a host-chosen shape: the family kernel runs the body of this shape
    ForceArgs b = a;
    b.shape = shape_code(K, cfg.L);
    hipLaunchKernelGGL(fn, dim3(grid), dim3(cfg.WG), 0, st, b);
  } else {
    hipLaunchKernelGGL(fn, dim3(grid), dim3(cfg.WG), 0, st, a);
  }
  return hipGetLastError();
}

// Workgroups of this kernel that one compute unit holds at once (from the
// occupancy calculator, cached per kernel).  A grid of num_CUs times this
// runs as one round, with no tail of lightly loaded SIMDs.
int resident_wgs(int prec, const Launch& cfg_in, bool mask) {
  static std::mutex mu;
  static std::map<const void*, int> cache;
  const Launch cfg = mask ? masked(cfg_in) : cfg_in;
  const int K = cfg.K;
  const void* fn = nullptr;
  if (cfg.L < 0 && prec == NB_PREC_MIXED && !mask) {
    fn = (const void*)pick_hy(K);
  } else if (cfg.L <= 0) {
    if (prec == NB_PREC_FP64)
      fn = mask ? (const void*)pick_sj<F64, true>(K, cfg.WG) : (const void*)pick_sj<F64, false>(K, cfg.WG);
    else if (prec == NB_PREC_MIXED_DS)
      fn = mask ? (const void*)pick_sj<MixedDS, true>(K, cfg.WG) : (const void*)pick_sj<MixedDS, false>(K, cfg.WG);
    else
      fn = mask ? (const void*)pick_sj<Mixed, true>(K, cfg.WG) : (const void*)pick_sj<Mixed, false>(K, cfg.WG);
  } else if (prec == NB_PREC_FP64) {
    fn = mask ? (const void*)pick_lds<F64, true>(cfg, K) : (const void*)pick_lds<F64, false>(cfg, K);
  } else if (prec == NB_PREC_MIXED_DS) {
    fn = mask ? (const void*)pick_lds<MixedDS, true>(cfg, K) : (const void*)pick_lds<MixedDS, false>(cfg, K);
  } else {
    fn = mask ? (const void*)pick_lds<Mixed, true>(cfg, K) : (const void*)pick_lds<Mixed, false>(cfg, K);
  }
  if (!fn) return 1;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(reinterpret_cast<const void*>(fn));
  if (it != cache.end()) return it->second;
  int nblk = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nblk, fn, cfg.WG, 0) != hipSuccess || nblk < 1) {
    (void)hipGetLastError();
    nblk = 1;
  }
  cache[reinterpret_cast<const void*>(fn)] = nblk;
  return nblk;
}

hipError_t launch_reduce_correct(int prec, const ForceArgs& a, const StepArgs& s, hipStream_t st) {
  // enough blocks for one row per thread at the largest count (a row takes
  // up to 64 lanes when its split is wide, and the count is then small); a
  // grid-stride loop covers the rest
  int64_t grid = (a.n_active + kReduceCorrectThreads - 1) / kReduceCorrectThreads;
  if (grid > 1024) grid = 1024;
  if (grid < 1) grid = 1;
  if (prec == NB_PREC_FP64)
    hipLaunchKernelGGL(k_reduce_correct<F64>, dim3((int)grid), dim3(kReduceCorrectThreads), 0, st, a, s);
  else if (prec == NB_PREC_MIXED_DS)
    hipLaunchKernelGGL(k_reduce_correct<MixedDS>, dim3((int)grid), dim3(kReduceCorrectThreads), 0, st, a, s);
  else
    hipLaunchKernelGGL(k_reduce_correct<Mixed>, dim3((int)grid), dim3(kReduceCorrectThreads), 0, st, a, s);
  return hipGetLastError();
}

hipError_t launch_reduce_ib(int prec, const ForceArgs& a, int S, int IB, hipStream_t st) {
  if (!a.n_active_dev && S <= 1) return hipSuccess;
  // threads: 7 outputs per row times the lanes per output; with the count
  // and S on the device, at least the rows' threads, and up to 1024 blocks
  // for a small count with many blocks to add (a grid-stride loop covers the
  // rest)
  const int64_t rows = 7 * a.n_active;
  int64_t threads = rows * chunk_lanes(S);
  if (a.n_active_dev) {
    threads = rows * 64 < (int64_t)1024 * 256 ? rows * 64 : (int64_t)1024 * 256;
    if (threads < rows) threads = rows;
  }
  int64_t grid = (threads + 255) / 256;
  if (grid > 4096) grid = 4096;
  if (grid < 1) grid = 1;
  if (prec == NB_PREC_FP64)
    hipLaunchKernelGGL(k_reduce<F64>, dim3((unsigned)grid), dim3(256), 0, st, a, S, IB);
  else if (prec == NB_PREC_MIXED_DS)
    hipLaunchKernelGGL(k_reduce<MixedDS>, dim3((unsigned)grid), dim3(256), 0, st, a, S, IB);
  else
    hipLaunchKernelGGL(k_reduce<Mixed>, dim3((unsigned)grid), dim3(256), 0, st, a, S, IB);
  return hipGetLastError();
}

bool batch_supported(const Launch& c) {
  if (c.L == 0) return pick_batch_sj<F64, false>(c.K) != nullptr;
  return pick_batch<F64, false>(c.K, c.L) != nullptr;
}

template <class P>
const void* batch_kernel(const Launch& cfg, bool mask) {
  if (cfg.L == 0)
    return mask ? (const void*)pick_batch_sj<P, true>(cfg.K) : (const void*)pick_batch_sj<P, false>(cfg.K);
  return mask ? (const void*)pick_batch<P, true>(cfg.K, cfg.L) : (const void*)pick_batch<P, false>(cfg.K, cfg.L);
}

int batch_resident_wgs(int prec, const Launch& cfg, bool mask) {
  static std::mutex mu;
  static std::map<const void*, int> cache;
  const void* fn = prec == NB_PREC_FP64        ? batch_kernel<F64>(cfg, mask)
                   : prec == NB_PREC_MIXED_DS ? batch_kernel<MixedDS>(cfg, mask)
                                              : batch_kernel<Mixed>(cfg, mask);
  if (!fn) return 1;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(fn);
  if (it != cache.end()) return it->second;
  int nblk = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nblk, fn, cfg.L == 0 ? kBatchSjWG : kWG, 0) != hipSuccess ||
      nblk < 1) {
    (void)hipGetLastError();
    nblk = 1;
  }
  cache[fn] = nblk;
  return nblk;
}

hipError_t launch_batch(int prec, const Launch& cfg, const BatchItem* items, int n_items, const int* n_items_dev,
                        const BatchSys* sys, const double* pos, const double* vel, const double* mass,
                        const int32_t* active, double* acc, double* jerk, double* pot, double* part,
                        int64_t part_rows, bool any_mask, int max_grid, unsigned int* err, void* rec,
                        int64_t n_total, hipStream_t st) {
  (void)part_rows;
  const int K = any_mask ? 1 : cfg.K;
  if (cfg.L == 0) {
#define NB_SJ(P)                                                                                                    \
  (any_mask ? launch_batch_sj_p<P, true>(K, items, n_items, n_items_dev, sys, rec, n_total, pos, vel, mass, active, \
                                         acc, jerk, pot, part, max_grid, err, st)                                   \
            : launch_batch_sj_p<P, false>(K, items, n_items, n_items_dev, sys, rec, n_total, pos, vel, mass,       \
                                          active, acc, jerk, pot, part, max_grid, err, st))
    if (prec == NB_PREC_FP64) return NB_SJ(F64);
    if (prec == NB_PREC_MIXED_DS) return NB_SJ(MixedDS);
    return NB_SJ(Mixed);
#undef NB_SJ
  }
  BatchFn fn = nullptr;
  if (prec == NB_PREC_FP64)
    fn = any_mask ? pick_batch<F64, true>(K, cfg.L) : pick_batch<F64, false>(K, cfg.L);
  else if (prec == NB_PREC_MIXED_DS)
    fn = any_mask ? pick_batch<MixedDS, true>(K, cfg.L) : pick_batch<MixedDS, false>(K, cfg.L);
  else
    fn = any_mask ? pick_batch<Mixed, true>(K, cfg.L) : pick_batch<Mixed, false>(K, cfg.L);
  if (!fn) return hipErrorInvalidValue;
  if (n_items <= 0) return hipSuccess;
  int grid = n_items;
  if (max_grid > 0 && grid > max_grid) grid = max_grid;
  hipLaunchKernelGGL(fn, dim3(grid), dim3(kWG), 0, st, items, n_items, n_items_dev, sys, pos, vel, mass, active, acc,
                     jerk, pot, part, err);
  return hipGetLastError();
}

hipError_t launch_batch_reduce(int prec, const BatchSys* sys, int n_sys, const int32_t* chunks_per_sys,
                               const double* mass, const int32_t* active, int64_t n_act_total, double* acc,
                               double* jerk, double* pot, const double* part, hipStream_t st) {
  if (n_sys <= 0) return hipSuccess;
  // blocks per system (grid x): enough for a system with the mean share of
  // the rows, at up to 16 lanes per output, to give each thread a few sums; a
  // system's blocks past its rows return at once
  int64_t nx = (7 * 16 * (n_act_total > 0 ? n_act_total : 1) + (int64_t)n_sys * 1024 - 1) / ((int64_t)n_sys * 1024);
  nx = nx < 1 ? 1 : (nx > 32 ? 32 : nx);
  const dim3 grid((unsigned)nx, (unsigned)(n_sys < 65535 ? n_sys : 65535));
  if (prec == NB_PREC_FP64)
    hipLaunchKernelGGL(k_batch_reduce<F64>, grid, dim3(256), 0, st, sys, chunks_per_sys, n_sys, mass, active, acc,
                       jerk, pot, part);
  else if (prec == NB_PREC_MIXED_DS)
    hipLaunchKernelGGL(k_batch_reduce<MixedDS>, grid, dim3(256), 0, st, sys, chunks_per_sys, n_sys, mass, active,
                       acc, jerk, pot, part);
  else
    hipLaunchKernelGGL(k_batch_reduce<Mixed>, grid, dim3(256), 0, st, sys, chunks_per_sys, n_sys, mass, active,
                       acc, jerk, pot, part);
  return hipGetLastError();
}

hipError_t launch_batch_reduce_correct(int prec, const BatchSys* sys, const int32_t* chunks_per_sys, int C,
                                       const int64_t* n_act_dev, int64_t n_max, const double* mass,
                                       const int32_t* active, double* acc1, double* jerk1, double* pot1,
                                       const double* part, const StepArgs& s, unsigned int* err, hipStream_t st) {
  if (C <= 0) return hipSuccess;
  // blocks per system (grid x) as for k_batch_reduce: enough for a system of
  // the mean size at up to 16 lanes per row; a system's blocks past its rows
  // return at once
  int64_t nx = (16 * (n_max > 0 ? n_max : 1) + (int64_t)C * 256 - 1) / ((int64_t)C * 256);
  nx = nx < 1 ? 1 : (nx > 32 ? 32 : nx);
  const dim3 grid((unsigned)nx, (unsigned)(C < 65535 ? C : 65535));
#define NB_RC(P)                                                                                                  \
  hipLaunchKernelGGL(k_batch_reduce_correct<P>, grid, dim3(256), 0, st, sys, chunks_per_sys, C, n_act_dev, mass, \
                     active, acc1, jerk1, pot1, part, s, err)
  if (prec == NB_PREC_FP64) NB_RC(F64);
  else if (prec == NB_PREC_MIXED_DS) NB_RC(MixedDS);
  else NB_RC(Mixed);
#undef NB_RC
  return hipGetLastError();
}

hipError_t launch_batch_plan(const int64_t* off, const double* eps2, int C, const int32_t* active,
                             const int64_t* n_act_dev, int IB, int target, BatchSys* sys, int32_t* nchunk,
                             BatchItem* items, int max_items, int* n_items_dev, int64_t part_cap_rows,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_batch_plan, dim3(1), dim3(kPlanThreads), 0, st, off, eps2, C, active, n_act_dev, IB, target,
                     sys, nchunk, items, max_items, n_items_dev, part_cap_rows);
  return hipGetLastError();
}

int host_choose_S(int64_t n_act, int IB, int target_items, int64_t n, int tile) {
  return choose_S(n_act, IB, target_items, n, tile);
}

}  // namespace nb
