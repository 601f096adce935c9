/*
 * precision_probe.c -- what the stability monitor after Eq. (5) measures.
 *
 * TEST INFRASTRUCTURE ONLY, like scivr_oracle.c (built into the same library).
 *
 * The monitor discards a trajectory once |det(M)^2 - 1| = |det(M^T M) - 1|
 * exceeds 1e-6.  For the exact flow M is symplectic and det M = 1, and the
 * fourth-order composition's discrete map is symplectic too, so any
 * deviation comes from floating-point rounding.  Two places could produce
 * it: the determinant of the stored M taken by Gaussian elimination (M is
 * ill-conditioned: a symplectic M has cond_2(M) = ||M||_2^2), or the stored M
 * itself, whose rounding errors accumulated along the trajectory.  This file
 * separates the two.  Along one trajectory, every `every` steps, it reports:
 *   - ||M||_F of the FP64 trajectory (the oracle's own integration);
 *   - |det^2 - 1| of that M by the oracle's FP64 elimination;
 *   - |det^2 - 1| of the same stored M by elimination in binary128 (the
 *     determinant of exactly the matrix the monitor sees);
 *   - |det^2 - 1| of M integrated in 80-bit long double from the same
 *     initial point with the same stages, its determinant in binary128;
 *   - ||M^T J M - J||_F / ||M||_F^2 of the FP64 M in binary128, J = [[0, I],
 *     [-I, 0]] in the (p, q) ordering.
 * The long-double integration restates the oracle's drift and kick with the
 * same potential and the same Yoshida / Forest-Ruth stages.
 *
 * Build: with scivr_oracle.c, -lquadmath.
 */
#include <math.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __float128 quad;

/* The oracle's problem statement and trajectory interface (scivr_oracle.c). */
typedef struct {
    int32_t F;
    const double *k_harm, *morse_D, *morse_a, *lam, *gamma, *p_eq, *q_eq;
    double dt;
    int32_t n_steps;
    double e_min, e_max;
    int32_t n_energies;
    double det_tol;
    int32_t check_every;
} orc_problem;
int64_t orc_state_size(int32_t F);
void orc_traj_init(const orc_problem *P, const double *p0, const double *q0, double *st, double *amp0);
int orc_traj_advance(const orc_problem *P, double *st, int32_t nsteps, double *amp_out);
double orc_det_real(int32_t n, double *a);

/* det of the n x n matrix a (row-major) by elimination with partial pivoting in binary128. */
static quad det_q(int n, const quad *a0, quad *a)
{
    memcpy(a, a0, sizeof(quad) * (size_t)n * n);
    quad det = 1;
    for (int k = 0; k < n; ++k) {
        int p = k;
        quad best = fabsq(a[k * n + k]);
        for (int i = k + 1; i < n; ++i)
            if (fabsq(a[i * n + k]) > best) {
                best = fabsq(a[i * n + k]);
                p = i;
            }
        if (best == 0) return 0;
        if (p != k) {
            for (int j = 0; j < n; ++j) {
                const quad t = a[k * n + j];
                a[k * n + j] = a[p * n + j];
                a[p * n + j] = t;
            }
            det = -det;
        }
        const quad piv = a[k * n + k];
        det *= piv;
        for (int i = k + 1; i < n; ++i) {
            const quad l = a[i * n + k] / piv;
            for (int j = k + 1; j < n; ++j) a[i * n + j] -= l * a[k * n + j];
        }
    }
    return det;
}

/* ||M^T J M - J||_F in binary128 for the 2F x 2F M ordered (p, q). */
static quad symplectic_defect_q(int F, const quad *M)
{
    const int n = 2 * F;
    quad s = 0;
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
            /* (M^T J M)_ab = sum_i M_{p_i a} M_{q_i b} - M_{q_i a} M_{p_i b} */
            quad v = 0;
            for (int i = 0; i < F; ++i) v += M[i * n + a] * M[(F + i) * n + b] - M[(F + i) * n + a] * M[i * n + b];
            if (a < F && b == a + F) v -= 1;
            if (a >= F && b == a - F) v += 1;
            s += v * v;
        }
    return sqrtq(s);
}

/* One step of the composition in long double: drifts d, kicks c (as the oracle). */
static void step_ld(const orc_problem *P, long double dt, const long double *d, const long double *c,
                    long double *p, long double *q, long double *M, long double *g, long double *H, long double *tmp)
{
    const int F = P->F, n = 2 * F;
    for (int s = 0; s < 4; ++s) {
        const long double h = d[s] * dt;
        for (int i = 0; i < F; ++i) q[i] += h * p[i];
        for (int i = 0; i < F; ++i)
            for (int j = 0; j < n; ++j) M[(F + i) * n + j] += h * M[i * n + j];
        if (s == 3) break;
        const long double hk = c[s] * dt;
        for (int i = 0; i < F; ++i) {
            const long double a = P->morse_a[i], D = P->morse_D[i], k = P->k_harm[i];
            const long double e = expl(-a * q[i]);
            g[i] = k * q[i] + 2.0L * D * a * e * (1.0L - e);
            for (int j = 0; j < F; ++j) H[i * F + j] = 0;
            H[i * F + i] = k + 2.0L * D * a * a * e * (2.0L * e - 1.0L);
        }
        for (int i = 0; i < F; ++i)
            for (int j = i + 1; j < F; ++j) {
                const long double l = P->lam[i * F + j], qi2 = q[i] * q[i], qj2 = q[j] * q[j];
                g[i] += 2.0L * l * q[i] * qj2;
                g[j] += 2.0L * l * q[j] * qi2;
                H[i * F + i] += 2.0L * l * qj2;
                H[j * F + j] += 2.0L * l * qi2;
                H[i * F + j] += 4.0L * l * q[i] * q[j];
                H[j * F + i] += 4.0L * l * q[i] * q[j];
            }
        for (int i = 0; i < F; ++i) p[i] -= hk * g[i];
        for (int i = 0; i < F; ++i)
            for (int j = 0; j < n; ++j) {
                long double sm = 0;
                for (int k = 0; k < F; ++k) sm += H[i * F + k] * M[(F + k) * n + j];
                tmp[i * n + j] = sm;
            }
        for (int i = 0; i < F; ++i)
            for (int j = 0; j < n; ++j) M[i * n + j] -= hk * tmp[i * n + j];
    }
}

/*
 * Rows of `out` (5 doubles each, nsteps / every rows): ||M||_F, FP64 |det^2 - 1|,
 * binary128 |det^2 - 1| of the same M, binary128 |det^2 - 1| of the long-double
 * M, and ||M^T J M - J||_F / ||M||_F^2.  Returns 0, or -1 if memory ran out.
 */
int orc_monitor_probe(const orc_problem *P, const double *p0, const double *q0, int32_t nsteps, int32_t every,
                      double *out)
{
    const int F = P->F, n = 2 * F;
    const int64_t ss = orc_state_size(F);
    double *st = malloc(sizeof(double) * (size_t)ss), *Mc = malloc(sizeof(double) * n * n);
    long double *p = malloc(sizeof(long double) * F), *q = malloc(sizeof(long double) * F);
    long double *M = calloc((size_t)n * n, sizeof(long double)), *g = malloc(sizeof(long double) * F);
    long double *H = malloc(sizeof(long double) * F * F), *tmp = malloc(sizeof(long double) * F * n);
    quad *Mq = malloc(sizeof(quad) * n * n), *wq = malloc(sizeof(quad) * n * n);
    int rc = -1;
    if (!st || !Mc || !p || !q || !M || !g || !H || !tmp || !Mq || !wq) goto done;
    orc_traj_init(P, p0, q0, st, NULL);
    for (int i = 0; i < F; ++i) {
        p[i] = p0[i];
        q[i] = q0[i];
    }
    for (int i = 0; i < n; ++i) M[i * n + i] = 1;
    const long double cb = cbrtl(2.0L), w1 = 1.0L / (2.0L - cb), w0 = -cb / (2.0L - cb);
    const long double d[4] = {0.5L * w1, 0.5L * (w0 + w1), 0.5L * (w0 + w1), 0.5L * w1}, c[3] = {w1, w0, w1};
    const double *Md = st + 2 * F + 8; /* the oracle's state: p, q, 8 scalars, then M */
    for (int s = 1; s <= nsteps; ++s) {
        if (orc_traj_advance(P, st, 1, NULL) != 0) goto done;
        step_ld(P, (long double)P->dt, d, c, p, q, M, g, H, tmp);
        if (s % every) continue;
        double *row = out + (size_t)(s / every - 1) * 5;
        double nm = 0;
        for (int i = 0; i < n * n; ++i) nm += Md[i] * Md[i];
        nm = sqrt(nm);
        memcpy(Mc, Md, sizeof(double) * n * n);
        const double d64 = orc_det_real(n, Mc);
        for (int i = 0; i < n * n; ++i) Mq[i] = Md[i];
        const quad dq = det_q(n, Mq, wq);
        const quad defect = symplectic_defect_q(F, Mq) / ((quad)nm * nm);
        for (int i = 0; i < n * n; ++i) Mq[i] = M[i];
        const quad dl = det_q(n, Mq, wq);
        row[0] = nm;
        row[1] = fabs(d64 * d64 - 1.0);
        row[2] = (double)fabsq(dq * dq - 1);
        row[3] = (double)fabsq(dl * dl - 1);
        row[4] = (double)defect;
    }
    rc = 0;
done:
    free(st); free(Mc); free(p); free(q); free(M); free(g); free(H); free(tmp); free(Mq); free(wq);
    return rc;
}
