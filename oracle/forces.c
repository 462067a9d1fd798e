/*
 * oracle/forces.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct CPU evaluation of the direct-summation
 * Plummer-softened gravitational acceleration, jerk and potential that the
 * GPU library computes.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this file's shared object; the
 * product path never does.  It shares no code with the HIP library.
 *
 * What is computed (paper, section "Optimizations for the GPU": the
 * j-particles exert a force and the i-particles receive it; every i-force is
 * an independent sum over the j-set; with Newton's law of gravity, G = 1, and
 * Plummer softening eps^2 as the standard reading of the direct method):
 *
 *   for i = active[k], r = x_j - x_i, u = v_j - v_i, s = |r|^2 + eps2:
 *     a_i   =  sum_{j != i}  m_j r / s^{3/2}
 *     jdot_i=  sum_{j != i}  m_j [ u / s^{3/2} - 3 (r.u) r / s^{5/2} ]
 *     phi_i = -sum_{j != i}  m_j / s^{1/2}
 *
 * The self pair is excluded by index.  A pair with s == 0 (two distinct
 * particles on the same spot with eps2 == 0) contributes nothing; the number
 * of such pairs is returned.
 *
 * Two evaluations of the same definition:
 *   oracle_forces_f64 : IEEE double, j ascending, plain accumulation.
 *   oracle_forces_ld  : the same loops in x87 extended precision (64-bit
 *                       significand); also returns, per i, the sums of the
 *                       magnitudes of the pair terms, which set the scale of
 *                       any rounding error (the condition of each sum).
 * Arrays: pos/vel [N][3] row-major doubles, mass [N], active [n_active]
 * int32 indices, outputs compact per active row: acc/jerk [n_active][3],
 * pot [n_active]; optional magnitude sums abs_acc/abs_jerk/abs_pot
 * [n_active] (may be NULL).
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int64_t oracle_forces_f64(const double *pos, const double *vel, const double *mass,
                          int64_t n, const int32_t *active, int64_t n_active, double eps2,
                          double *acc, double *jerk, double *pot, int nthreads)
{
    int64_t skipped = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(static) reduction(+ : skipped)
    for (int64_t k = 0; k < n_active; ++k) {
        const int64_t i = active[k];
        const double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
        const double vxi = vel[3 * i], vyi = vel[3 * i + 1], vzi = vel[3 * i + 2];
        double ax = 0, ay = 0, az = 0, jx = 0, jy = 0, jz = 0, ph = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            const double rx = pos[3 * j] - xi, ry = pos[3 * j + 1] - yi, rz = pos[3 * j + 2] - zi;
            const double ux = vel[3 * j] - vxi, uy = vel[3 * j + 1] - vyi, uz = vel[3 * j + 2] - vzi;
            const double s = rx * rx + ry * ry + rz * rz + eps2;
            if (s == 0.0) { ++skipped; continue; }
            const double inv_sqrt_s = 1.0 / sqrt(s);          /* s^{-1/2} */
            const double inv_s = inv_sqrt_s * inv_sqrt_s;      /* s^{-1}   */
            const double w = mass[j] * inv_sqrt_s * inv_s;     /* m s^{-3/2} */
            const double ru = rx * ux + ry * uy + rz * uz;
            const double c = 3.0 * ru * inv_s;                 /* 3 (r.u) / s */
            ax += w * rx; ay += w * ry; az += w * rz;
            jx += w * (ux - c * rx); jy += w * (uy - c * ry); jz += w * (uz - c * rz);
            ph -= mass[j] * inv_sqrt_s;
        }
        acc[3 * k] = ax; acc[3 * k + 1] = ay; acc[3 * k + 2] = az;
        jerk[3 * k] = jx; jerk[3 * k + 1] = jy; jerk[3 * k + 2] = jz;
        pot[k] = ph;
    }
    return skipped;
}

int64_t oracle_forces_ld(const double *pos, const double *vel, const double *mass,
                         int64_t n, const int32_t *active, int64_t n_active, double eps2,
                         double *acc, double *jerk, double *pot,
                         double *abs_acc, double *abs_jerk, double *abs_pot, int nthreads)
{
    int64_t skipped = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(static) reduction(+ : skipped)
    for (int64_t k = 0; k < n_active; ++k) {
        const int64_t i = active[k];
        const long double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
        const long double vxi = vel[3 * i], vyi = vel[3 * i + 1], vzi = vel[3 * i + 2];
        long double ax = 0, ay = 0, az = 0, jx = 0, jy = 0, jz = 0, ph = 0;
        long double sa = 0, sj = 0, sp = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            const long double rx = (long double)pos[3 * j] - xi;
            const long double ry = (long double)pos[3 * j + 1] - yi;
            const long double rz = (long double)pos[3 * j + 2] - zi;
            const long double ux = (long double)vel[3 * j] - vxi;
            const long double uy = (long double)vel[3 * j + 1] - vyi;
            const long double uz = (long double)vel[3 * j + 2] - vzi;
            const long double s = rx * rx + ry * ry + rz * rz + (long double)eps2;
            if (s == 0.0L) { ++skipped; continue; }
            const long double inv_sqrt_s = 1.0L / sqrtl(s);
            const long double inv_s = 1.0L / s;
            const long double m = mass[j];
            const long double w = m * inv_sqrt_s * inv_s;
            const long double ru = rx * ux + ry * uy + rz * uz;
            const long double c = 3.0L * ru * inv_s;
            const long double tx = w * rx, ty = w * ry, tz = w * rz;
            const long double qx = w * (ux - c * rx), qy = w * (uy - c * ry), qz = w * (uz - c * rz);
            ax += tx; ay += ty; az += tz;
            jx += qx; jy += qy; jz += qz;
            ph -= m * inv_sqrt_s;
            sa += sqrtl(tx * tx + ty * ty + tz * tz);
            sj += sqrtl(qx * qx + qy * qy + qz * qz);
            sp += fabsl(m * inv_sqrt_s);
        }
        acc[3 * k] = (double)ax; acc[3 * k + 1] = (double)ay; acc[3 * k + 2] = (double)az;
        jerk[3 * k] = (double)jx; jerk[3 * k + 1] = (double)jy; jerk[3 * k + 2] = (double)jz;
        pot[k] = (double)ph;
        if (abs_acc) abs_acc[k] = (double)sa;
        if (abs_jerk) abs_jerk[k] = (double)sj;
        if (abs_pot) abs_pot[k] = (double)sp;
    }
    return skipped;
}

/* Total potential energy W = -sum_{i<j} m_i m_j / sqrt(|x_i - x_j|^2 + eps2),
 * evaluated pair by pair in extended precision (pairs with s == 0 skipped).
 * Used to pin W = 1/2 sum_i m_i phi_i. */
double oracle_pair_potential_energy(const double *pos, const double *mass, int64_t n, double eps2)
{
    long double w = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j) {
            const long double rx = (long double)pos[3 * j] - pos[3 * i];
            const long double ry = (long double)pos[3 * j + 1] - pos[3 * i + 1];
            const long double rz = (long double)pos[3 * j + 2] - pos[3 * i + 2];
            const long double s = rx * rx + ry * ry + rz * rz + (long double)eps2;
            if (s == 0.0L) continue;
            w -= (long double)mass[i] * (long double)mass[j] / sqrtl(s);
        }
    return (double)w;
}
