// One particle's fourth-order Hermite correction and new time-step level,
// shared by the corrector kernel and the fused reduce-and-correct kernel of
// the block steps (so both give the same bits).
//
// Makino-Aarseth form (the paper names a fourth-order Hermite integrator for
// its direct code and gives no formulas): from the start-of-step a0, j0 and
// the end-of-step a1, j1 over dt,
//   a2 = [-6 (a0 - a1) - dt (4 j0 + 2 j1)] / dt^2,
//   a3 = [12 (a0 - a1) + 6 dt (j0 + j1)] / dt^3,
//   x1 = x_p + a2 dt^4/24 + a3 dt^5/120,   v1 = v_p + a2 dt^3/6 + a3 dt^4/24;
// then Aarseth's criterion with a2 taken at the end of the step,
//   dt* = sqrt(eta (|a1||a2 + a3 dt| + |j1|^2) / (|j1||a3| + |a2 + a3 dt|^2)),
// and the power-of-two level rules (halve while dt > dt*, capped at
// max_level and counted in *clamp_dev; double once when dt* >= 2 dt and the
// new time is a multiple of 2 dt).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace nb {

__device__ __forceinline__ double norm3_d(double x, double y, double z) { return sqrt(x * x + y * y + z * z); }

__device__ __forceinline__ void correct_particle(int64_t i, const double a1[3], const double j1[3],
                                                 const double* __restrict__ pos_p,
                                                 const double* __restrict__ vel_p, double* __restrict__ pos,
                                                 double* __restrict__ vel, double* __restrict__ acc,
                                                 double* __restrict__ jerk, int64_t* __restrict__ t_tick,
                                                 int32_t* __restrict__ level, double eta, double dt_max,
                                                 int max_level, unsigned long long* __restrict__ clamp_dev) {
  const int L = level[i];
  const double dt = ldexp(dt_max, -L);
  const double dt2 = dt * dt, dt3 = dt2 * dt;
  double a2[3], a3[3], a2e[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double a0 = acc[3 * i + c], j0 = jerk[3 * i + c];
    a2[c] = (-6.0 * (a0 - a1[c]) - dt * (4.0 * j0 + 2.0 * j1[c])) / dt2;
    a3[c] = (12.0 * (a0 - a1[c]) + 6.0 * dt * (j0 + j1[c])) / dt3;
    const double dt4 = dt2 * dt2;
    pos[3 * i + c] = pos_p[3 * i + c] + a2[c] * (dt4 / 24.0) + a3[c] * (dt4 * dt / 120.0);
    vel[3 * i + c] = vel_p[3 * i + c] + a2[c] * (dt3 / 6.0) + a3[c] * (dt4 / 24.0);
    acc[3 * i + c] = a1[c];
    jerk[3 * i + c] = j1[c];
    a2e[c] = a2[c] + a3[c] * dt;
  }
  const double na1 = norm3_d(a1[0], a1[1], a1[2]);
  const double nj1 = norm3_d(j1[0], j1[1], j1[2]);
  const double na2 = norm3_d(a2e[0], a2e[1], a2e[2]);
  const double na3 = norm3_d(a3[0], a3[1], a3[2]);
  const double num = na1 * na2 + nj1 * nj1;
  const double den = nj1 * na3 + na2 * na2;
  const double ds = den > 0.0 ? sqrt(eta * num / den) : dt_max;
  const int64_t t_new = t_tick[i] + ((int64_t)1 << (max_level - L));
  int Ln = L;
  double dtc = dt;
  if (ds < dtc) {
    while (dtc > ds && Ln < max_level) {
      ++Ln;
      dtc = ldexp(dt_max, -Ln);
    }
    if (dtc > ds && clamp_dev) atomicAdd(clamp_dev, 1ull);
  } else if (ds >= 2.0 * dtc && Ln > 0) {
    const int64_t two_dt = (int64_t)1 << (max_level - Ln + 1);
    if (t_new % two_dt == 0) --Ln;
  }
  t_tick[i] = t_new;
  level[i] = Ln;
}

}  // namespace nb
