// Element-wise kernels of the second-order Hamiltonian split (section "The
// multi-scale approach": H = H_A + H_B, evolved as e^{dt/2 A} e^{dt B}
// e^{dt/2 A}).  A kick is the flow of a potential term: velocities move by
// h a and positions stay.  The field subsystem's own evolution under H_g is
// a shared-step leapfrog whose first half is a kick followed by a drift,
// fused here into one pass.
//
// Both passes are HBM-bound (24 B read and 24 B written per particle for a
// kick, 72 B read and 48 B written for a kick-drift); one thread takes one
// component of one particle, so every array is read and written with unit
// stride.  Each update is a multiply and then an add (no fused multiply-add)
// so that the result is the same in every evaluation order that rounds after
// each operation.
#include "nb_internal.h"

namespace nb {
namespace {

constexpr int kB = 256;

__device__ __forceinline__ double axpy_rounded(double y, double h, double x) {
#pragma clang fp contract(off)
  return y + h * x;
}

__global__ __launch_bounds__(kB) void k_kick(double* __restrict__ vel, const double* __restrict__ acc, double h,
                                             int64_t n3) {
  for (int64_t e = (int64_t)blockIdx.x * kB + threadIdx.x; e < n3; e += (int64_t)gridDim.x * kB)
    vel[e] = axpy_rounded(vel[e], h, acc[e]);
}

__global__ __launch_bounds__(kB) void k_kick_drift(double* __restrict__ pos, double* __restrict__ vel,
                                                   const double* __restrict__ acc, double h_kick, double h_drift,
                                                   int64_t n3) {
  for (int64_t e = (int64_t)blockIdx.x * kB + threadIdx.x; e < n3; e += (int64_t)gridDim.x * kB) {
    const double v = axpy_rounded(vel[e], h_kick, acc[e]);
    vel[e] = v;
    pos[e] = axpy_rounded(pos[e], h_drift, v);
  }
}

inline int grid_for(int64_t work, int cap) {
  const int64_t g = (work + kB - 1) / kB;
  return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace

hipError_t launch_kick(double* vel, const double* acc, double h, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_kick, dim3(grid_for(3 * n, 8192)), dim3(kB), 0, st, vel, acc, h, 3 * n);
  return hipGetLastError();
}

hipError_t launch_kick_drift(double* pos, double* vel, const double* acc, double h_kick, double h_drift, int64_t n,
                             hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_kick_drift, dim3(grid_for(3 * n, 8192)), dim3(kB), 0, st, pos, vel, acc, h_kick, h_drift,
                     3 * n);
  return hipGetLastError();
}

}  // namespace nb
