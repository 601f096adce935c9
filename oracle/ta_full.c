/*
 * ta_full.c -- the time-averaged SC-IVR spectral density without the
 * separable approximation: Eq. (9) with the Herman-Kluk prefactor of each
 * trajectory segment.
 *
 * TEST INFRASTRUCTURE ONLY, like scivr_oracle.c (built into the same library).
 *
 * Eq. (9) integrates over two times t1 <= t2 of one trajectory: the
 * prefactor C_{t2}(p(t1), q(t1)) belongs to the trajectory that starts at the
 * phase-space point (p(t1), q(t1)) and runs to t2, i.e. sqrt(det A) of Eq. (5)
 * built from the tangent map of the segment [t1, t2], with the square-root
 * branch continuous in t2 from C = 1 at t2 = t1.  The separable approximation
 * after Eq. (9) replaces it by exp(i (phi(t2) - phi(t1))) and reduces the
 * double sum to |sum_t ...|^2 (Eq. (10)).  Discretised on the same time samples
 * as Eq. (11), with the diagonal t1 = t2 weighted 1/2 (so that the separable
 * prefactor gives exactly Eq. (11)):
 *
 *   I(E_k) = dt^2 / (pi T G) sum_j w_j good_j
 *            Re sum_{c1 <= c2} omega_{c1 c2} C_j(c1, c2) a_j(c2) conj(a_j(c1)) e^{i E_k (c2 - c1) dt},
 *   a_j(c) = <chi|p_j(c dt), q_j(c dt)> e^{i S_j(c dt)},  omega = 1/2 on the diagonal, 1 above,
 *
 * with w_j, good_j and G as in Eq. (11) (this file returns the sum without the
 * factor dt^2 / (2 pi T G), written as 2 Re of the lag sum: the convention of
 * the separable form's |A_j|^2).  The segment is run by the oracle's own
 * trajectory routine from the stored state at c1 (fresh tangent map, action
 * and branch), which repeats the main trajectory's arithmetic exactly, so the
 * points z_j(c) are the same; the segment's action is S(c2) - S(c1).
 * The sum is regrouped by lag tau = c2 - c1: R_j(tau) = sum_{c1} omega C a conj(a).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

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
void orc_overlap(const orc_problem *P, const double *p, const double *q, double *re, double *im);
void orc_prefactor_matrix(const orc_problem *P, const double *M, double *are, double *aim);
void orc_det_complex(int32_t n, double *re, double *im, double *det_re, double *det_im);
void orc_energy_grid(const orc_problem *P, double *E);

enum { TS_S = 0, TS_PHI = 3, TS_GOOD = 4, TS_NSCALAR = 8 }; /* the oracle's state layout after p, q */

/*
 * Lag sums of one trajectory from (p0, q0): R[tau] (complex, 2 (n_steps + 1)
 * doubles) and its good flag.  Returns 0, or -1 if memory ran out.
 */
int orc_ta_full_lags(const orc_problem *P, const double *p0, const double *q0, double *R, int32_t *good)
{
    const int F = P->F, ns = P->n_steps;
    const int64_t ss = orc_state_size(F);
    double *traj = malloc(sizeof(double) * (size_t)ss * (ns + 1)); /* the main trajectory's states */
    double *seg = malloc(sizeof(double) * (size_t)ss);
    double *are = malloc(sizeof(double) * F * F), *aim = malloc(sizeof(double) * F * F);
    if (!traj || !seg || !are || !aim) {
        free(traj); free(seg); free(are); free(aim);
        return -1;
    }
    orc_traj_init(P, p0, q0, traj, NULL);
    for (int c = 1; c <= ns; ++c) {
        memcpy(traj + (size_t)c * ss, traj + (size_t)(c - 1) * ss, sizeof(double) * (size_t)ss);
        orc_traj_advance(P, traj + (size_t)c * ss, 1, NULL);
    }
    *good = traj[(size_t)ns * ss + 2 * F + TS_GOOD] != 0.0;
    for (int k = 0; k < 2 * (ns + 1); ++k) R[k] = 0.0;
    for (int c1 = 0; c1 <= ns; ++c1) {
        /* the segment from z(c1): fresh tangent map, action and branch */
        const double *st1 = traj + (size_t)c1 * ss;
        orc_traj_init(P, st1, st1 + F, seg, NULL);
        for (int c2 = c1; c2 <= ns; ++c2) {
            if (c2 > c1) orc_traj_advance(P, seg, 1, NULL);
            /* C = |det A|^(1/2) e^{i phi}, phi the continuous half-argument */
            double dr, di;
            orc_prefactor_matrix(P, seg + 2 * F + TS_NSCALAR, are, aim);
            orc_det_complex(F, are, aim, &dr, &di);
            const double mod = sqrt(hypot(dr, di));
            const double phi = seg[2 * F + TS_PHI];
            const double cr = mod * cos(phi), ci = mod * sin(phi);
            /* the segment's own overlap and action at c2: the main trajectory's point */
            double ore, oim;
            orc_overlap(P, seg, seg + F, &ore, &oim);
            const double S = seg[2 * F + TS_S];
            const double br = ore * cos(S) - oim * sin(S), bi = ore * sin(S) + oim * cos(S);
            /* omega C b conj(<chi|z_c1>) ; the segment's action starts at 0 */
            double o1r, o1i;
            orc_overlap(P, st1, st1 + F, &o1r, &o1i);
            const double xr = cr * br - ci * bi, xi = cr * bi + ci * br;
            const double w = (c2 == c1) ? 0.5 : 1.0;
            R[2 * (c2 - c1)] += w * (xr * o1r + xi * o1i);
            R[2 * (c2 - c1) + 1] += w * (xi * o1r - xr * o1i);
        }
    }
    free(traj); free(seg); free(are); free(aim);
    return 0;
}

/*
 * The estimator over n trajectories (p0, q0 [F][n], logrho [n]): spec_sum[K] =
 * sum_j good_j w_j 2 Re sum_tau R_j(tau) e^{i E_k tau dt} (the separable form's
 * sum_j good_j w_j |A_j(E_k)|^2 in the separable approximation), n_good, and the
 * per-trajectory lag sums if lags is not NULL ([n][n_steps + 1][2]).
 */
int orc_ta_full_run(const orc_problem *P, int64_t n, const double *p0, const double *q0, const double *logrho,
                    double *spec_sum, int64_t *n_good, double *good_out, double *lags)
{
    const int F = P->F, ns = P->n_steps, K = P->n_energies;
    double *E = malloc(sizeof(double) * K);
    double *tot = calloc((size_t)2 * (ns + 1), sizeof(double));
    if (!E || !tot) {
        free(E); free(tot);
        return -1;
    }
    orc_energy_grid(P, E);
    int err = 0;
    int64_t ng = 0;
    /* trajectories in parallel, the weighted lag sums added in trajectory order */
    double *Rall = malloc(sizeof(double) * (size_t)2 * (ns + 1) * (size_t)n);
    int32_t *gall = malloc(sizeof(int32_t) * (size_t)n);
    if (!Rall || !gall) {
        free(E); free(tot); free(Rall); free(gall);
        return -1;
    }
#pragma omp parallel for schedule(dynamic)
    for (int64_t j = 0; j < n; ++j) {
        double *pz = malloc(sizeof(double) * 2 * F);
        if (!pz) {
#pragma omp atomic write
            err = -1;
            continue;
        }
        for (int i = 0; i < F; ++i) {
            pz[i] = p0[(int64_t)i * n + j];
            pz[F + i] = q0[(int64_t)i * n + j];
        }
        if (orc_ta_full_lags(P, pz, pz + F, Rall + (size_t)j * 2 * (ns + 1), &gall[j]) != 0) {
#pragma omp atomic write
            err = -1;
        }
        free(pz);
    }
    for (int64_t j = 0; j < n; ++j) {
        if (good_out) good_out[j] = gall[j];
        if (lags) memcpy(lags + (size_t)j * 2 * (ns + 1), Rall + (size_t)j * 2 * (ns + 1),
                         sizeof(double) * 2 * (ns + 1));
        if (!gall[j]) continue;
        ++ng;
        const double w = exp(-logrho[j] - (double)F * log(2.0 * 3.14159265358979323846));
        for (int t = 0; t < 2 * (ns + 1); ++t) tot[t] += w * Rall[(size_t)j * 2 * (ns + 1) + t];
    }
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (int tau = 0; tau <= ns; ++tau) {
            const double ph = E[k] * (double)tau * P->dt;
            s += tot[2 * tau] * cos(ph) - tot[2 * tau + 1] * sin(ph);
        }
        spec_sum[k] = 2.0 * s;
    }
    *n_good = ng;
    free(E); free(tot); free(Rall); free(gall);
    return err;
}
