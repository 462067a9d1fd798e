// Sixth-order Hermite block-step kernels: predictor of position, velocity
// and acceleration, corrector from the quintic through (a, jdot, snap) at
// both ends of the step, the order-six step criterion and the start-up
// levels.  HBM-bound element-wise passes in double precision; the block
// scheduler is the fourth-order one (hermite.hip).
//
// The scheme (one reading of the higher-order Hermite integrators the paper
// cites for its direct method; it writes none of them down):
//  predict   x_p = x + v d + a d^2/2 + j d^3/6 + s d^4/24 + c d^5/120,
//            v_p = v + a d + j d^2/2 + s d^3/6 + c d^4/24,
//            a_p = a + j d + s d^2/2 + c d^3/6      (c: crackle of the last step)
//  correct   the quintic a(t) through (a0, j0, s0) at 0 and (a1, j1, s1) at h
//            has, with A = a1 - (a0 + j0 h + s0 h^2/2), B = (j1 - j0 - s0 h) h,
//            C = (s1 - s0) h^2,
//              c0 = (60 A - 24 B + 3 C) / h^3, p0 = (-360 A + 168 B - 24 C) / h^4,
//              q0 = (720 A - 360 B + 60 C) / h^5;
//            x1, v1 are its exact integrals from (x0, v0); c1 = c0 + p0 h + q0 h^2/2,
//            p1 = p0 + q0 h
//  new step  dt* = eta ((sqrt(|a1||s1|) + |j1|) / (sqrt(|c1||q0|) + |p1|))^(1/3),
//            dt_max when the denominator is 0; power-of-two levels as the
//            fourth-order corrector
//  start-up  dt* = eta_s min(|a|/|j|, sqrt(|a|/|s|)) over the finite terms.
#include "nb_internal.h"

namespace nb {
namespace {

constexpr int kB6 = 256;

__device__ __forceinline__ double norm3_6(const double* v) { return sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); }

inline int grid6(int64_t work, int cap) {
  const int64_t g = (work + kB6 - 1) / kB6;
  return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

// One thread per (particle, component), unit stride everywhere.
__global__ __launch_bounds__(kB6) void k_predict6(const double* __restrict__ pos, const double* __restrict__ vel,
                                                  const double* __restrict__ acc, const double* __restrict__ jerk,
                                                  const double* __restrict__ snap, const double* __restrict__ crackle,
                                                  const int64_t* __restrict__ t_tick, int64_t t_next_host,
                                                  const int64_t* __restrict__ t_next_dev, double dt_min, int64_t n3,
                                                  double* __restrict__ pos_p, double* __restrict__ vel_p,
                                                  double* __restrict__ acc_p) {
  const int64_t t_next = t_next_dev ? *t_next_dev : t_next_host;
  for (int64_t e = (int64_t)blockIdx.x * kB6 + threadIdx.x; e < n3; e += (int64_t)gridDim.x * kB6) {
    const double d = (double)(t_next - t_tick[e / 3]) * dt_min;
    const double x = pos[e], v = vel[e], a = acc[e], j = jerk[e], s = snap[e], c = crackle[e];
    pos_p[e] = x + d * (v + d * (0.5 * a + d * ((1.0 / 6.0) * j + d * ((1.0 / 24.0) * s + d * ((1.0 / 120.0) * c)))));
    vel_p[e] = v + d * (a + d * (0.5 * j + d * ((1.0 / 6.0) * s + d * ((1.0 / 24.0) * c))));
    acc_p[e] = a + d * (j + d * (0.5 * s + d * ((1.0 / 6.0) * c)));
  }
}

__device__ __forceinline__ int new_level6(int L, double ds, int64_t t_new, double dt_max, int max_level,
                                          bool* clamped) {
  double dt = ldexp(dt_max, -L);
  *clamped = false;
  if (ds < dt) {
    while (dt > ds && L < max_level) {
      ++L;
      dt = ldexp(dt_max, -L);
    }
    *clamped = dt > ds;
  } else if (ds >= 2.0 * dt && L > 0) {
    const int64_t two_dt_ticks = (int64_t)1 << (max_level - L + 1);
    if (t_new % two_dt_ticks == 0) --L;
  }
  return L;
}

__global__ __launch_bounds__(kB6) void k_correct6(const int32_t* __restrict__ active, int64_t n_active_host,
                                                  const int64_t* __restrict__ n_active_dev, int64_t n_rows,
                                                  unsigned int* __restrict__ err,
                                                  const double* __restrict__ acc1, const double* __restrict__ jerk1,
                                                  const double* __restrict__ snap1, double* __restrict__ pos,
                                                  double* __restrict__ vel, double* __restrict__ acc,
                                                  double* __restrict__ jerk, double* __restrict__ snap,
                                                  double* __restrict__ crackle, int64_t* __restrict__ t_tick,
                                                  int32_t* __restrict__ level, double eta, double dt_max,
                                                  int max_level, unsigned long long* __restrict__ clamp_dev,
                                                  unsigned long long* __restrict__ step_dev) {
  int64_t n_act = n_active_host;
  if (n_active_dev) {
    const int64_t d = *n_active_dev;
    n_act = d < n_act ? (d < 0 ? 0 : d) : n_act;
  }
  if (step_dev && n_act > 0 && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(step_dev, 1ull);
  for (int64_t k = (int64_t)blockIdx.x * kB6 + threadIdx.x; k < n_act; k += (int64_t)gridDim.x * kB6) {
    const int64_t i = active[k];
    if (!row_in_range(i, 0, n_rows)) {  // not a particle: skipped, and reported by nb_sync
      if (err) atomicOr(err, kErrActiveRange);
      continue;
    }
    const int L = level[i];
    const double h = ldexp(dt_max, -L);
    const double h2 = h * h, h3 = h2 * h;
    double a1[3], j1[3], s1[3], c1[3], p1[3], q0[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double a0 = acc[3 * i + c], j0 = jerk[3 * i + c], s0 = snap[3 * i + c];
      a1[c] = acc1[3 * k + c];
      j1[c] = jerk1[3 * k + c];
      s1[c] = snap1[3 * k + c];
      const double A = a1[c] - (a0 + h * (j0 + h * (0.5 * s0)));
      const double B = (j1[c] - (j0 + h * s0)) * h;
      const double C = (s1[c] - s0) * h2;
      const double cc = (60.0 * A - 24.0 * B + 3.0 * C) / h3;
      const double pp = (-360.0 * A + 168.0 * B - 24.0 * C) / (h3 * h);
      const double qq = (720.0 * A - 360.0 * B + 60.0 * C) / (h3 * h2);
      const double x0 = pos[3 * i + c], v0 = vel[3 * i + c];
      const double v1 = v0 + h * (a0 + h * (0.5 * j0 + h * ((1.0 / 6.0) * s0 + h * ((1.0 / 24.0) * cc +
                                 h * ((1.0 / 120.0) * pp + h * ((1.0 / 720.0) * qq))))));
      const double x1 = x0 + h * (v0 + h * (0.5 * a0 + h * ((1.0 / 6.0) * j0 + h * ((1.0 / 24.0) * s0 +
                                 h * ((1.0 / 120.0) * cc + h * ((1.0 / 720.0) * pp + h * ((1.0 / 5040.0) * qq)))))));
      pos[3 * i + c] = x1;
      vel[3 * i + c] = v1;
      acc[3 * i + c] = a1[c];
      jerk[3 * i + c] = j1[c];
      snap[3 * i + c] = s1[c];
      c1[c] = cc + h * (pp + h * (0.5 * qq));
      p1[c] = pp + h * qq;
      q0[c] = qq;
      crackle[3 * i + c] = c1[c];
    }
    const double num = sqrt(norm3_6(a1) * norm3_6(s1)) + norm3_6(j1);
    const double den = sqrt(norm3_6(c1) * norm3_6(q0)) + norm3_6(p1);
    const double ds = den > 0.0 ? eta * cbrt(num / den) : dt_max;
    const int64_t t_new = t_tick[i] + ((int64_t)1 << (max_level - L));
    t_tick[i] = t_new;
    bool clamped;
    level[i] = new_level6(L, ds, t_new, dt_max, max_level, &clamped);
    if (clamped && clamp_dev) atomicAdd(clamp_dev, 1ull);
  }
}

__global__ __launch_bounds__(kB6) void k_startup6(const double* __restrict__ acc, const double* __restrict__ jerk,
                                                  const double* __restrict__ snap, int64_t n, double eta_s,
                                                  double dt_max, int max_level, int32_t* __restrict__ level) {
  for (int64_t i = (int64_t)blockIdx.x * kB6 + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB6) {
    const double na = norm3_6(acc + 3 * i), nj = norm3_6(jerk + 3 * i), ns = norm3_6(snap + 3 * i);
    double target = -1.0;
    if (nj > 0.0) target = na / nj;
    if (ns > 0.0) {
      const double t2 = sqrt(na / ns);
      target = (target < 0.0 || t2 < target) ? t2 : target;
    }
    int L = 0;
    if (target >= 0.0) {
      target *= eta_s;
      while (ldexp(dt_max, -L) > target && L < max_level) ++L;
    }
    level[i] = L;
  }
}

}  // namespace

hipError_t launch_predict6(const double* pos, const double* vel, const double* acc, const double* jerk,
                           const double* snap, const double* crackle, const int64_t* t_tick, int64_t t_next,
                           const int64_t* t_next_dev, double dt_min, int64_t n, double* pos_p, double* vel_p,
                           double* acc_p, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_predict6, dim3(grid6(3 * n, 8192)), dim3(kB6), 0, st, pos, vel, acc, jerk, snap, crackle,
                     t_tick, t_next, t_next_dev, dt_min, 3 * n, pos_p, vel_p, acc_p);
  return hipGetLastError();
}

hipError_t launch_correct6(const int32_t* active, int64_t n_max, const int64_t* n_active_dev, int64_t n_rows,
                           unsigned int* err, const double* acc1, const double* jerk1, const double* snap1,
                           double* pos, double* vel, double* acc, double* jerk, double* snap, double* crackle,
                           int64_t* t_tick, int32_t* level, double eta, double dt_max, int max_level,
                           int64_t* clamp_dev, int64_t* step_dev, hipStream_t st) {
  if (n_max <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_correct6, dim3(grid6(n_max, 1024)), dim3(kB6), 0, st, active, n_max, n_active_dev, n_rows,
                     err, acc1,
                     jerk1, snap1, pos, vel, acc, jerk, snap, crackle, t_tick, level, eta, dt_max, max_level,
                     reinterpret_cast<unsigned long long*>(clamp_dev),
                     reinterpret_cast<unsigned long long*>(step_dev));
  return hipGetLastError();
}

hipError_t launch_startup6(const double* acc, const double* jerk, const double* snap, int64_t n, double eta_s,
                           double dt_max, int max_level, int32_t* level, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_startup6, dim3(grid6(n, 4096)), dim3(kB6), 0, st, acc, jerk, snap, n, eta_s, dt_max,
                     max_level, level);
  return hipGetLastError();
}

}  // namespace nb
