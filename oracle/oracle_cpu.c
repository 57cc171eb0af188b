/*
 * FP64 CPU oracle for the direct-summation N-body hot path, in plain C.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path. It shares no code,
 * header or constant with the GPU library.
 *
 * The pair sum is the force equation of Section 3 (sum over all j != i of
 * G m_j (r_j - r_i) / r_ij^3, here per unit target mass), with Plummer
 * softening eps added to r_ij^2; eps = 0 is the paper's unsoftened sum. The
 * potential is phi_i = -G sum_{j != i} m_j / sqrt(r_ij^2 + eps^2). It is the
 * naive double-precision brute force the paper validates against (Section 3,
 * correctness paragraph): OpenMP over targets, a sequential loop over sources
 * in ascending index order, IEEE double arithmetic (built without
 * -ffast-math and with -ffp-contract=off).
 *
 * The kick-drift-kick step is the leapfrog the GPU path drives:
 * v += dt/2 a; x += dt v; a = A(x); v += dt/2 a.
 */
#include <math.h>
#include <stdint.h>
#include <omp.h>

/* acc: [nt][3], pot: [nt] (pot may be NULL); targets may be NULL (= all). */
void oracle_accel_pot(const double *pos, const double *mass, int64_t n,
                      const int64_t *targets, int64_t nt, double eps, double G,
                      double *acc, double *pot, int nthreads)
{
    const double eps2 = eps * eps;
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t i = targets ? targets[t] : t;
        const double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
        double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            const double dx = pos[3 * j] - xi;
            const double dy = pos[3 * j + 1] - yi;
            const double dz = pos[3 * j + 2] - zi;
            const double r2 = dx * dx + dy * dy + dz * dz + eps2;
            const double r = sqrt(r2);
            const double w = mass[j] / r;
            const double w3 = w / r2;
            ax += w3 * dx;
            ay += w3 * dy;
            az += w3 * dz;
            ph -= w;
        }
        acc[3 * t] = G * ax;
        acc[3 * t + 1] = G * ay;
        acc[3 * t + 2] = G * az;
        if (pot) pot[t] = G * ph;
    }
}

/* n_steps of kick-drift-kick. acc must hold A(pos) on entry and holds
 * A(pos_final) on return; pot (nullable) gets the final potentials. */
void oracle_kdk(double *pos, double *vel, double *acc, double *pot,
                const double *mass, int64_t n, double eps, double G, double dt,
                int32_t n_steps, int nthreads)
{
    const double h = 0.5 * dt;
    for (int32_t s = 0; s < n_steps; ++s) {
        for (int64_t k = 0; k < 3 * n; ++k) {
            vel[k] += h * acc[k];
            pos[k] += dt * vel[k];
        }
        oracle_accel_pot(pos, mass, n, 0, n, eps, G, acc, pot, nthreads);
        for (int64_t k = 0; k < 3 * n; ++k) vel[k] += h * acc[k];
    }
}

/* Accelerations, jerks (time derivative of the acceleration) and
 * potentials: jerk_i = G sum_{j != i} m_j [w/q^{3/2} - 3 (d.w) d/q^{5/2}],
 * d = x_j - x_i, w = v_j - v_i, q = |d|^2 + eps^2. */
void oracle_accel_jerk(const double *pos, const double *vel, const double *mass, int64_t n,
                       const int64_t *targets, int64_t nt, double eps, double G,
                       double *acc, double *jerk, double *pot, int nthreads)
{
    const double eps2 = eps * eps;
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t i = targets ? targets[t] : t;
        double ax = 0.0, ay = 0.0, az = 0.0, jx = 0.0, jy = 0.0, jz = 0.0, ph = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            const double dx = pos[3 * j] - pos[3 * i];
            const double dy = pos[3 * j + 1] - pos[3 * i + 1];
            const double dz = pos[3 * j + 2] - pos[3 * i + 2];
            const double wx = vel[3 * j] - vel[3 * i];
            const double wy = vel[3 * j + 1] - vel[3 * i + 1];
            const double wz = vel[3 * j + 2] - vel[3 * i + 2];
            const double q = dx * dx + dy * dy + dz * dz + eps2;
            const double r = sqrt(q);
            const double m1 = mass[j] / r;
            const double m3 = m1 / q;
            const double m5 = m3 / q;
            const double dw = dx * wx + dy * wy + dz * wz;
            ax += m3 * dx;
            ay += m3 * dy;
            az += m3 * dz;
            jx += m3 * wx - 3.0 * m5 * dw * dx;
            jy += m3 * wy - 3.0 * m5 * dw * dy;
            jz += m3 * wz - 3.0 * m5 * dw * dz;
            ph -= m1;
        }
        acc[3 * t] = G * ax;
        acc[3 * t + 1] = G * ay;
        acc[3 * t + 2] = G * az;
        jerk[3 * t] = G * jx;
        jerk[3 * t + 1] = G * jy;
        jerk[3 * t + 2] = G * jz;
        if (pot) pot[t] = G * ph;
    }
}

int oracle_max_threads(void) { return omp_get_max_threads(); }
