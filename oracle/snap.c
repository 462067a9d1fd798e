/*
 * oracle/snap.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain CPU evaluation of the force terms a sixth-order Hermite scheme needs
 * (the higher-order Hermite integrators the paper cites in section
 * "Simulating Collisional systems with direct force evaluation methods"):
 * acceleration, jerk, snap (the second time derivative of the acceleration)
 * and potential of the i-set active[0..n_active) in the field of all n
 * particles, each particle moving with its own position, velocity and
 * acceleration at the instant of evaluation.  With G = 1, Plummer softening
 * and, for i = active[k],
 *   r = x_j - x_i,  u = v_j - v_i,  w = a_j - a_i,  s = |r|^2 + eps2:
 *
 *   a_i    =  sum_{j != i} m_j r s^{-3/2}
 *   jdot_i =  sum_{j != i} m_j [ u s^{-3/2} - 3 (r.u) r s^{-5/2} ]
 *   snap_i =  sum_{j != i} m_j [ w s^{-3/2} - 6 (r.u) u s^{-5/2}
 *                                - 3 (u.u + r.w) r s^{-5/2} + 15 (r.u)^2 r s^{-7/2} ]
 *   phi_i  = -sum_{j != i} m_j s^{-1/2}
 *
 * (snap is the time derivative of the jerk term with dr/dt = u, du/dt = w,
 * ds/dt = 2 r.u, written out term by term).  The self pair is excluded by
 * index; a pair with s == 0 contributes nothing and is counted.
 *
 * One evaluation in x87 extended precision (64-bit significand), j ascending,
 * rounded to double at the end; per i it also returns the sums of the
 * magnitudes of the pair terms (the scale of any rounding error).
 * Arrays: pos/vel/acc [n][3] row-major doubles, mass [n], active [n_active]
 * int32; outputs compact per active row: acc/jerk/snap [n_active][3],
 * pot [n_active]; abs_* [n_active] may be NULL.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static long double norm3l(long double x, long double y, long double z) { return sqrtl(x * x + y * y + z * z); }

int64_t oracle_snap_ld(const double *pos, const double *vel, const double *accj, const double *mass,
                       int64_t n, const int32_t *active, int64_t n_active, double eps2,
                       double *acc, double *jerk, double *snap, double *pot,
                       double *abs_acc, double *abs_jerk, double *abs_snap, double *abs_pot, int nthreads)
{
    int64_t skipped = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(static) reduction(+ : skipped)
    for (int64_t k = 0; k < n_active; ++k) {
        const int64_t i = active[k];
        long double A[3] = {0, 0, 0}, J[3] = {0, 0, 0}, S[3] = {0, 0, 0}, ph = 0;
        long double sa = 0, sj = 0, ss = 0, sp = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            long double r[3], u[3], w[3];
            for (int c = 0; c < 3; ++c) {
                r[c] = (long double)pos[3 * j + c] - (long double)pos[3 * i + c];
                u[c] = (long double)vel[3 * j + c] - (long double)vel[3 * i + c];
                w[c] = (long double)accj[3 * j + c] - (long double)accj[3 * i + c];
            }
            const long double s = r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + (long double)eps2;
            if (s == 0.0L) { ++skipped; continue; }
            const long double m = mass[j];
            const long double s12 = sqrtl(s);
            const long double s32 = s * s12, s52 = s32 * s, s72 = s52 * s;
            const long double ru = r[0] * u[0] + r[1] * u[1] + r[2] * u[2];
            const long double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
            const long double rw = r[0] * w[0] + r[1] * w[1] + r[2] * w[2];
            long double ta[3], tj[3], ts[3];
            for (int c = 0; c < 3; ++c) {
                ta[c] = m * r[c] / s32;
                tj[c] = m * (u[c] / s32 - 3.0L * ru * r[c] / s52);
                ts[c] = m * (w[c] / s32 - 6.0L * ru * u[c] / s52 - 3.0L * (uu + rw) * r[c] / s52
                             + 15.0L * ru * ru * r[c] / s72);
                A[c] += ta[c]; J[c] += tj[c]; S[c] += ts[c];
            }
            ph -= m / s12;
            sa += norm3l(ta[0], ta[1], ta[2]);
            sj += norm3l(tj[0], tj[1], tj[2]);
            ss += norm3l(ts[0], ts[1], ts[2]);
            sp += fabsl(m / s12);
        }
        for (int c = 0; c < 3; ++c) {
            acc[3 * k + c] = (double)A[c];
            jerk[3 * k + c] = (double)J[c];
            snap[3 * k + c] = (double)S[c];
        }
        pot[k] = (double)ph;
        if (abs_acc) abs_acc[k] = (double)sa;
        if (abs_jerk) abs_jerk[k] = (double)sj;
        if (abs_snap) abs_snap[k] = (double)ss;
        if (abs_pot) abs_pot[k] = (double)sp;
    }
    return skipped;
}
