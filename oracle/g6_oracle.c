/*
 * g6_oracle.c -- plain CPU reference for the direct-summation force
 * evaluation that a 4th-order Hermite block-time-step integrator consumes
 * (Gaburov, Harfst & Portegies Zwart 2009, "SAPPORO", Sec. 2).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is loaded by the test-suite, by
 * the smoke check and by the CPU-baseline leg of the benchmark, nothing
 * else.  It includes nothing from the GPU tree and the GPU library never
 * links or calls it.
 *
 * Everything is IEEE float64, evaluated term by term in the order of the
 * definitions below, with no blocking, fusion or reordering.  Build with
 *     gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared
 * so that the compiler contracts no multiply-add.  The only parallelism is
 * over i-particles; each i-particle's sum over j runs sequentially in
 * ascending slot order, so the results do not depend on the thread count.
 *
 * Functions and what pins them (tests/test_oracle_pins.py):
 *   oracle_predict -- Eq. (1) and Eq. (2), Sec. 2.2.  Pinned by exact cubic
 *                     trajectories and by d(x_pred)/dt = v_pred.
 *   oracle_force   -- acceleration, jerk and potential of Plummer-softened
 *                     Newtonian gravity (G = 1), summed over all j-particles
 *                     except the i-particle itself (Sec. 2 and 2.3); nearest
 *                     neighbour and neighbour list (Sec. 2.5 and 4).  Pinned
 *                     by closed-form configurations, -grad(phi), d(acc)/dt
 *                     along straight-line motion, Newton's third law,
 *                     the Plummer-model potential energy and a k-d tree.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- threads */

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* -------------------------------------------------------------- predictor */
/*
 * Sec. 2.2, Eq. (1) and (2): with tau = t_i - t_k the time since particle
 * k was last corrected,
 *     x_pred = x0 + v0 tau + a0 tau^2 / 2 + j0 tau^3 / 6
 *     v_pred = v0 + a0 tau + j0 tau^2 / 2.
 * A GRAPE-6 client stores the pre-scaled coefficients a2 = a0/2 and
 * j6 = j0/6, so the terms are a2 tau^2, j6 tau^3, 2 a2 tau and 3 j6 tau^2.
 * Arrays are row-major [n][3].
 */
void oracle_predict(int64_t nj, double ti, const double *t,
                    const double *x, const double *v,
                    const double *a2, const double *j6,
                    double *xp, double *vp)
{
    for (int64_t k = 0; k < nj; ++k) {
        double tau = ti - t[k];
        double tau2 = tau * tau;
        double tau3 = tau2 * tau;
        for (int d = 0; d < 3; ++d) {
            int64_t e = 3 * k + d;
            xp[e] = x[e] + v[e] * tau + a2[e] * tau2 + j6[e] * tau3;
            vp[e] = v[e] + 2.0 * a2[e] * tau + 3.0 * j6[e] * tau2;
        }
    }
}

/* ------------------------------------------------------------------ force */

static int cmp_int(const void *a, const void *b)
{
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

/*
 * For every i-particle (position xi, velocity vi, particle index iindex)
 * and every j-slot k whose particle index differs from iindex[i]:
 *     r  = x_k - x_i,  w = v_k - v_i,  r2u = r.r,  s = r2u + eps2
 *     acc_i  +=  m_k r / s^{3/2}
 *     jerk_i +=  m_k ( w / s^{3/2} - 3 (r.w) r / s^{5/2} )
 *     pot_i  -=  m_k / s^{1/2}
 * The jerk is the time derivative of the acceleration along the motion.
 * A pair with s == 0 (eps2 = 0 and coincident positions) is counted as
 * degenerate and skipped.
 *
 * Nearest neighbour: the j-particle with the smallest unsoftened r2u,
 * ties broken by the smaller particle index; (-1, +inf) if there is none.
 * Neighbour list: all particle indices with r2u < h2[i], in ascending
 * order.  nb_count[i] is the true number of neighbours; nb_list holds the
 * first min(count, nb_cap) of them in row i (row length nb_cap), the rest of
 * the row is -1.
 *
 * Optional outputs acc_abs[i] = sum_k |m_k r / s^{3/2}| and jerk_abs[i] =
 * sum_k |jerk term of pair k| (NULL to skip) measure how much the sums
 * cancel: |acc_i| / acc_abs[i] is 1 when all pair forces are parallel.
 *
 * Returns the number of degenerate pairs.
 */
int64_t oracle_force(int64_t nj, const double *xj, const double *vj,
                     const double *mj, const int *jindex,
                     int64_t ni, const double *xi, const double *vi,
                     const int *iindex, double eps2, const double *h2,
                     int nb_cap,
                     double *acc, double *jerk, double *pot,
                     int *nn_index, double *nn_r2,
                     int64_t *nb_count, int *nb_list,
                     double *acc_abs, double *jerk_abs)
{
    int64_t degenerate = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : degenerate)
    for (int64_t i = 0; i < ni; ++i) {
        double ax = 0.0, ay = 0.0, az = 0.0;
        double jx = 0.0, jy = 0.0, jz = 0.0;
        double phi = 0.0;
        double sa = 0.0, sj = 0.0;
        double best_r2 = INFINITY;
        int best_idx = -1;
        int64_t count = 0, cap = 16;
        int *found = (int *)malloc((size_t)cap * sizeof(int));
        const double px = xi[3 * i + 0], py = xi[3 * i + 1], pz = xi[3 * i + 2];
        const double qx = vi[3 * i + 0], qy = vi[3 * i + 1], qz = vi[3 * i + 2];
        const double hh = h2 ? h2[i] : 0.0;

        for (int64_t k = 0; k < nj; ++k) {
            if (jindex[k] == iindex[i]) continue; /* the particle itself */
            double rx = xj[3 * k + 0] - px;
            double ry = xj[3 * k + 1] - py;
            double rz = xj[3 * k + 2] - pz;
            double wx = vj[3 * k + 0] - qx;
            double wy = vj[3 * k + 1] - qy;
            double wz = vj[3 * k + 2] - qz;
            double r2u = rx * rx + ry * ry + rz * rz;

            /* nearest neighbour: smallest r2u, then smallest index */
            if (r2u < best_r2 || (r2u == best_r2 && jindex[k] < best_idx)) {
                best_r2 = r2u;
                best_idx = jindex[k];
            }
            /* neighbour list: strict r2u < h2 */
            if (r2u < hh) {
                if (count == cap) {
                    cap *= 2;
                    found = (int *)realloc(found, (size_t)cap * sizeof(int));
                }
                found[count++] = jindex[k];
            }

            double s = r2u + eps2;
            if (s == 0.0) {
                degenerate += 1;
                continue;
            }
            double q = 1.0 / sqrt(s);     /* 1/|r|, softened */
            double q2 = q * q;
            double q3 = q2 * q;
            double rw = rx * wx + ry * wy + rz * wz;
            double m = mj[k];
            ax += m * q3 * rx;
            ay += m * q3 * ry;
            az += m * q3 * rz;
            jx += m * (q3 * wx - 3.0 * rw * q3 * q2 * rx);
            jy += m * (q3 * wy - 3.0 * rw * q3 * q2 * ry);
            jz += m * (q3 * wz - 3.0 * rw * q3 * q2 * rz);
            phi -= m * q;
            if (acc_abs || jerk_abs) {
                double ex = m * (q3 * wx - 3.0 * rw * q3 * q2 * rx);
                double ey = m * (q3 * wy - 3.0 * rw * q3 * q2 * ry);
                double ez = m * (q3 * wz - 3.0 * rw * q3 * q2 * rz);
                sa += fabs(m) * q3 * sqrt(r2u);
                sj += sqrt(ex * ex + ey * ey + ez * ez);
            }
        }

        acc[3 * i + 0] = ax;
        acc[3 * i + 1] = ay;
        acc[3 * i + 2] = az;
        jerk[3 * i + 0] = jx;
        jerk[3 * i + 1] = jy;
        jerk[3 * i + 2] = jz;
        pot[i] = phi;
        if (acc_abs) acc_abs[i] = sa;
        if (jerk_abs) jerk_abs[i] = sj;
        if (nn_index) nn_index[i] = best_idx;
        if (nn_r2) nn_r2[i] = best_r2;
        if (nb_count) nb_count[i] = count;
        if (nb_list && nb_cap > 0) {
            qsort(found, (size_t)count, sizeof(int), cmp_int);
            for (int64_t s = 0; s < nb_cap; ++s)
                nb_list[i * nb_cap + s] = s < count ? found[s] : -1;
        }
        free(found);
    }
    return degenerate;
}
