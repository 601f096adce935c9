/*
 * scivr_oracle.c -- plain, slow, FP64 CPU oracle of the time-averaged
 * semiclassical initial value representation (TA-SC-IVR) power spectrum
 * with the separable prefactor approximation.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * with the HIP library: every formula below is written out again from the
 * paper (Tamascelli, Dambrosio, Conte, Ceotto, "Graphics Processing Units
 * Accelerated Semiclassical Initial Value Representation Molecular
 * Dynamics").
 *
 * What is computed, in the order of the section "Monte-Carlo SC-IVR
 * algorithm" and Eq. (11):
 *   - initial phase-space points drawn from the Husimi distribution of the
 *     reference coherent state chi (Philox4x64-10 + Box-Muller, each written
 *     from its published definition);
 *   - for every point, a classical trajectory under a fourth-order symplectic
 *     integrator, with the action S_t, the 2F x 2F monodromy matrix M(t)
 *     (Eq. (5) and the text after it), the phase phi_t of the Herman-Kluk
 *     prefactor C_t kept on a continuous branch (separable approximation
 *     after Eq. (9)), and the stability monitor on det(M^T M) = det(M)^2;
 *   - the amplitude <chi|p_t,q_t> exp(i (S_t + phi_t)) at every time sample;
 *   - its Fourier sum over an equally spaced energy grid and the weighted,
 *     n_good-normalised Monte Carlo average of |.|^2 (Eqs. (10) and (11)).
 *
 * Readings of the paper taken here (the paper is silent or ambiguous):
 *   - coherent states are normalised per mode, <q|p,q> = prod_i
 *     (gamma_i/pi)^(1/4) exp(...), so <chi|chi> = 1 (Eq. (3) prints the
 *     exponent F/4 on each factor);
 *   - the fourth-order symplectic scheme is the drift-kick-drift triple jump
 *     of Yoshida / Forest-Ruth (w1 = 1/(2 - 2^(1/3)), w0 = -2^(1/3) w1), which
 *     evaluates the Hessian three times per step;
 *   - the action is the discrete Lagrangian of the same stages:
 *     +h |p|^2/2 per drift of length h, -h V per kick of length h;
 *   - the prefactor matrix is the holomorphic block of the tangent map in
 *     the variables z = Gamma^(1/2) q + i Gamma^(-1/2) p; its determinant
 *     equals that of the bracket in Eq. (5) and only its phase is used;
 *   - the square-root branch is made continuous in time by unwrapping the
 *     argument of det(A) exp(i t sum_i gamma_i) step by step;
 *   - a trajectory is bad once |det(M)^2 - 1| exceeds det_tol (1e-6) at any
 *     checked step (every step by default); bad trajectories keep running to
 *     T but contribute nothing;
 *   - the Husimi weight is w_j = 1 / ((2 pi)^F rho(z_j)) for a sampling
 *     density rho, i.e. 1/|<z_j|chi>|^2 for Husimi sampling;
 *   - the time sum runs over c = 0 .. n_steps inclusive, T = n_steps dt, and
 *     the spectrum is I_k = dt^2 / (2 pi T n_good) sum_j good_j w_j |A_jk|^2.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846264338327950288

/* Problem statement (arrays are borrowed for the duration of a call). */
typedef struct {
    int32_t F;
    const double *k_harm;  /* [F] quadratic coefficients k_i (V += k_i q_i^2 / 2) */
    const double *morse_D; /* [F] Morse well depths D_i */
    const double *morse_a; /* [F] Morse range parameters a_i */
    const double *lam;     /* [F*F] row-major symmetric quartic couplings; only i<j is read */
    const double *gamma;   /* [F] coherent-state widths gamma_i */
    const double *p_eq;    /* [F] reference state momentum */
    const double *q_eq;    /* [F] reference state position */
    double dt;
    int32_t n_steps;
    double e_min, e_max;
    int32_t n_energies;
    double det_tol;
    int32_t check_every;
} orc_problem;

/*
 * Per-trajectory state, a flat array of orc_state_size(F) doubles:
 *   [0, F)        p
 *   [F, 2F)       q
 *   2F + 0        S        action
 *   2F + 1        theta    unwrapped argument of det(A) e^{i t sum gamma}
 *   2F + 2        rprev    last principal argument
 *   2F + 3        phi      prefactor phase at the current time
 *   2F + 4        good     1 or 0 (sticky)
 *   2F + 5        detM     det(M) at the last checked step
 *   2F + 6        maxdev   max |det(M)^2 - 1| over checked steps
 *   2F + 7        step     number of steps taken
 *   2F + 8 ...    M        2F x 2F row-major, rows/cols ordered (p, q)
 */
enum { ST_S = 0, ST_THETA, ST_RPREV, ST_PHI, ST_GOOD, ST_DETM, ST_MAXDEV, ST_STEP, ST_NSCALAR };

int64_t orc_state_size(int32_t F) { return 2 * (int64_t)F + ST_NSCALAR + 4 * (int64_t)F * F; }

static double *st_M(double *st, int F) { return st + 2 * F + ST_NSCALAR; }

/* ------------------------------------------------------------------------ */
/* Potential energy surface: value, gradient and Hessian.                    */
/*   V = sum_i [k_i q_i^2/2 + D_i (1 - e_i)^2] + sum_{i<j} lam_ij q_i^2 q_j^2 */
/*   with e_i = exp(-a_i q_i).                                               */
/* ------------------------------------------------------------------------ */
void orc_potential(const orc_problem *P, const double *q, double *V, double *g, double *H)
{
    const int F = P->F;
    double v = 0.0;
    for (int i = 0; i < F; ++i) {
        const double e = exp(-P->morse_a[i] * q[i]);
        const double D = P->morse_D[i], a = P->morse_a[i], k = P->k_harm[i];
        v += 0.5 * k * q[i] * q[i] + D * (1.0 - e) * (1.0 - e);
        g[i] = k * q[i] + 2.0 * D * a * e * (1.0 - e);
        for (int j = 0; j < F; ++j) H[i * F + j] = 0.0;
        H[i * F + i] = k + 2.0 * D * a * a * e * (2.0 * e - 1.0);
    }
    for (int i = 0; i < F; ++i) {
        for (int j = i + 1; j < F; ++j) {
            const double l = P->lam[i * F + j];
            const double qi2 = q[i] * q[i], qj2 = q[j] * q[j];
            v += l * qi2 * qj2;
            g[i] += 2.0 * l * q[i] * qj2;
            g[j] += 2.0 * l * q[j] * qi2;
            H[i * F + i] += 2.0 * l * qj2;
            H[j * F + j] += 2.0 * l * qi2;
            H[i * F + j] += 4.0 * l * q[i] * q[j];
            H[j * F + i] += 4.0 * l * q[i] * q[j];
        }
    }
    *V = v;
}

/* ------------------------------------------------------------------------ */
/* Determinants by Gaussian elimination with partial pivoting (the first    */
/* entry of largest modulus in the column is the pivot).  The input is      */
/* overwritten.                                                             */
/* ------------------------------------------------------------------------ */
double orc_det_real(int32_t n, double *a)
{
    double det = 1.0;
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = fabs(a[k * n + k]);
        for (int i = k + 1; i < n; ++i) {
            if (fabs(a[i * n + k]) > best) {
                best = fabs(a[i * n + k]);
                p = i;
            }
        }
        if (best == 0.0) return 0.0;
        if (p != k) {
            for (int j = 0; j < n; ++j) {
                double t = a[k * n + j];
                a[k * n + j] = a[p * n + j];
                a[p * n + j] = t;
            }
            det = -det;
        }
        const double piv = a[k * n + k];
        det *= piv;
        for (int i = k + 1; i < n; ++i) {
            const double l = a[i * n + k] / piv;
            for (int j = k + 1; j < n; ++j) a[i * n + j] -= l * a[k * n + j];
        }
    }
    return det;
}

void orc_det_complex(int32_t n, double *re, double *im, double *det_re, double *det_im)
{
    double dr = 1.0, di = 0.0;
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = hypot(re[k * n + k], im[k * n + k]);
        for (int i = k + 1; i < n; ++i) {
            const double m = hypot(re[i * n + k], im[i * n + k]);
            if (m > best) {
                best = m;
                p = i;
            }
        }
        if (best == 0.0) {
            *det_re = 0.0;
            *det_im = 0.0;
            return;
        }
        if (p != k) {
            for (int j = 0; j < n; ++j) {
                double t = re[k * n + j];
                re[k * n + j] = re[p * n + j];
                re[p * n + j] = t;
                t = im[k * n + j];
                im[k * n + j] = im[p * n + j];
                im[p * n + j] = t;
            }
            dr = -dr;
            di = -di;
        }
        const double pr = re[k * n + k], pi = im[k * n + k];
        /* det *= pivot */
        const double nr = dr * pr - di * pi;
        const double ni = dr * pi + di * pr;
        dr = nr;
        di = ni;
        const double pm2 = pr * pr + pi * pi;
        for (int i = k + 1; i < n; ++i) {
            /* l = a_ik / a_kk */
            const double ar = re[i * n + k], ai = im[i * n + k];
            const double lr = (ar * pr + ai * pi) / pm2;
            const double li = (ai * pr - ar * pi) / pm2;
            for (int j = k + 1; j < n; ++j) {
                const double br = re[k * n + j], bi = im[k * n + j];
                re[i * n + j] -= lr * br - li * bi;
                im[i * n + j] -= lr * bi + li * br;
            }
        }
    }
    *det_re = dr;
    *det_im = di;
}

/* ------------------------------------------------------------------------ */
/* Coherent-state overlap <chi|p,q> for chi = |p_eq, q_eq>, Eq. (3) with     */
/* per-mode normalisation:                                                   */
/*   prod_i exp( -gamma_i (q_eq,i - q_i)^2 / 4 - (p_eq,i - p_i)^2 / (4 gamma_i) */
/*               + (i/2) (q_eq,i - q_i)(p_eq,i + p_i) )                       */
/* ------------------------------------------------------------------------ */
void orc_overlap(const orc_problem *P, const double *p, const double *q, double *re, double *im)
{
    double ex = 0.0, ph = 0.0;
    for (int i = 0; i < P->F; ++i) {
        const double dq = P->q_eq[i] - q[i];
        const double dp = P->p_eq[i] - p[i];
        ex += -P->gamma[i] * dq * dq / 4.0 - dp * dp / (4.0 * P->gamma[i]);
        ph += 0.5 * dq * (P->p_eq[i] + p[i]);
    }
    const double m = exp(ex);
    *re = m * cos(ph);
    *im = m * sin(ph);
}

/* ------------------------------------------------------------------------ */
/* Herman-Kluk prefactor matrix (Eq. (5)), written with G = Gamma:           */
/*   A = 1/2 [ G^{1/2} M_qq G^{-1/2} + G^{-1/2} M_pp G^{1/2}                  */
/*             - i G^{1/2} M_qp G^{1/2} + i G^{-1/2} M_pq G^{-1/2} ]           */
/* where M_pp = dp_t/dp_0, M_pq = dp_t/dq_0, M_qp = dq_t/dp_0, M_qq = dq_t/dq_0. */
/* ------------------------------------------------------------------------ */
void orc_prefactor_matrix(const orc_problem *P, const double *M, double *are, double *aim)
{
    const int F = P->F, n = 2 * F;
    for (int i = 0; i < F; ++i) {
        const double si = sqrt(P->gamma[i]);
        for (int j = 0; j < F; ++j) {
            const double sj = sqrt(P->gamma[j]);
            const double mpp = M[i * n + j];
            const double mpq = M[i * n + F + j];
            const double mqp = M[(F + i) * n + j];
            const double mqq = M[(F + i) * n + F + j];
            are[i * F + j] = 0.5 * (si * mqq / sj + mpp * sj / si);
            aim[i * F + j] = 0.5 * (-si * mqp * sj + mpq / (si * sj));
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Fourth-order symplectic triple jump (drift-kick-drift composition).       */
/* ------------------------------------------------------------------------ */
void orc_yoshida_coefficients(double *d /*[4]*/, double *c /*[3]*/)
{
    const double cbrt2 = cbrt(2.0);
    const double w1 = 1.0 / (2.0 - cbrt2);
    const double w0 = -cbrt2 / (2.0 - cbrt2);
    d[0] = 0.5 * w1;
    d[1] = 0.5 * (w0 + w1);
    d[2] = 0.5 * (w0 + w1);
    d[3] = 0.5 * w1;
    c[0] = w1;
    c[1] = w0;
    c[2] = w1;
}

/* Drift of length h: q += h p, S += h |p|^2 / 2, dq/dz0 += h dp/dz0. */
static void drift(int F, double h, double *st)
{
    double *p = st, *q = st + F, *M = st_M(st, F);
    const int n = 2 * F;
    double kin = 0.0;
    for (int i = 0; i < F; ++i) kin += 0.5 * p[i] * p[i];
    for (int i = 0; i < F; ++i) q[i] += h * p[i];
    st[2 * F + ST_S] += h * kin;
    for (int i = 0; i < F; ++i)
        for (int j = 0; j < n; ++j) M[(F + i) * n + j] += h * M[i * n + j];
}

/* Kick of length h: p -= h grad V(q), S -= h V(q), dp/dz0 -= h Hess V(q) dq/dz0. */
static void kick(const orc_problem *P, double h, double *st, double *g, double *H, double *tmp)
{
    const int F = P->F, n = 2 * F;
    double *p = st, *q = st + F, *M = st_M(st, F);
    double V;
    orc_potential(P, q, &V, g, H);
    for (int i = 0; i < F; ++i) p[i] -= h * g[i];
    st[2 * F + ST_S] -= h * V;
    /* tmp = H * M_q (F x 2F), then M_p -= h tmp */
    for (int i = 0; i < F; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int k = 0; k < F; ++k) s += H[i * F + k] * M[(F + k) * n + j];
            tmp[i * n + j] = s;
        }
    for (int i = 0; i < F; ++i)
        for (int j = 0; j < n; ++j) M[i * n + j] -= h * tmp[i * n + j];
}

static double sum_gamma(const orc_problem *P)
{
    double s = 0.0;
    for (int i = 0; i < P->F; ++i) s += P->gamma[i];
    return s;
}

/* Amplitude <chi|p,q> exp(i (S + phi)), zero for a bad trajectory. */
static void amplitude(const orc_problem *P, const double *st, double *re, double *im)
{
    const int F = P->F;
    if (st[2 * F + ST_GOOD] == 0.0) {
        *re = 0.0;
        *im = 0.0;
        return;
    }
    double ore, oim;
    orc_overlap(P, st, st + F, &ore, &oim);
    const double th = st[2 * F + ST_S] + st[2 * F + ST_PHI];
    const double c = cos(th), s = sin(th);
    *re = ore * c - oim * s;
    *im = ore * s + oim * c;
}

/* Start a trajectory at (p0, q0): S = 0, M = I, phi = 0, good. */
void orc_traj_init(const orc_problem *P, const double *p0, const double *q0, double *st, double *amp0 /*[2] or NULL*/)
{
    const int F = P->F, n = 2 * F;
    memset(st, 0, sizeof(double) * (size_t)orc_state_size(F));
    for (int i = 0; i < F; ++i) {
        st[i] = p0[i];
        st[F + i] = q0[i];
    }
    st[2 * F + ST_GOOD] = 1.0;
    st[2 * F + ST_DETM] = 1.0;
    double *M = st_M(st, F);
    for (int i = 0; i < n; ++i) M[i * n + i] = 1.0;
    if (amp0) amplitude(P, st, &amp0[0], &amp0[1]);
}

static double wrap_pi(double x)
{
    while (x > ORC_PI) x -= 2.0 * ORC_PI;
    while (x <= -ORC_PI) x += 2.0 * ORC_PI;
    return x;
}

/* Advance a trajectory by n steps; amp_out receives 2*n doubles (re, im) per step. */
int orc_traj_advance(const orc_problem *P, double *st, int32_t nsteps, double *amp_out)
{
    const int F = P->F, n = 2 * F;
    double d[4], c[3];
    orc_yoshida_coefficients(d, c);
    double *g = (double *)malloc(sizeof(double) * F);
    double *H = (double *)malloc(sizeof(double) * F * F);
    double *tmp = (double *)malloc(sizeof(double) * F * n);
    double *Mc = (double *)malloc(sizeof(double) * n * n);
    double *are = (double *)malloc(sizeof(double) * F * F);
    double *aim = (double *)malloc(sizeof(double) * F * F);
    if (!g || !H || !tmp || !Mc || !are || !aim) {
        free(g); free(H); free(tmp); free(Mc); free(are); free(aim);
        return -1;
    }
    const double sg = sum_gamma(P);
    const double dt = P->dt;
    for (int s = 0; s < nsteps; ++s) {
        /* one step: drift d0, kick c0, drift d1, kick c1, drift d2, kick c2, drift d3 */
        for (int stage = 0; stage < 4; ++stage) {
            drift(F, d[stage] * dt, st);
            if (stage < 3) kick(P, c[stage] * dt, st, g, H, tmp);
        }
        const int64_t step = (int64_t)st[2 * F + ST_STEP] + 1;
        st[2 * F + ST_STEP] = (double)step;
        const double t = (double)step * dt;
        double *M = st_M(st, F);

        /* prefactor phase on a continuous branch */
        double dre, dim;
        orc_prefactor_matrix(P, M, are, aim);
        orc_det_complex(F, are, aim, &dre, &dim);
        const double rc = cos(sg * t), rs = sin(sg * t);
        const double zr = dre * rc - dim * rs, zi = dre * rs + dim * rc;
        const double r = atan2(zi, zr);
        st[2 * F + ST_THETA] += wrap_pi(r - st[2 * F + ST_RPREV]);
        st[2 * F + ST_RPREV] = r;
        st[2 * F + ST_PHI] = 0.5 * (st[2 * F + ST_THETA] - sg * t);

        /* stability monitor on det(M^T M) = det(M)^2 */
        const int checked = (P->check_every <= 1) || (step % P->check_every == 0) || (step == P->n_steps);
        if (checked) {
            memcpy(Mc, M, sizeof(double) * n * n);
            const double dM = orc_det_real(n, Mc);
            const double dev = fabs(dM * dM - 1.0);
            st[2 * F + ST_DETM] = dM;
            if (!(dev <= st[2 * F + ST_MAXDEV])) st[2 * F + ST_MAXDEV] = dev; /* NaN propagates */
            if (!(dev <= P->det_tol)) st[2 * F + ST_GOOD] = 0.0;
        }
        if (!isfinite(st[2 * F + ST_PHI]) || !isfinite(st[2 * F + ST_S])) st[2 * F + ST_GOOD] = 0.0;
        if (amp_out) amplitude(P, st, &amp_out[2 * s], &amp_out[2 * s + 1]);
    }
    free(g); free(H); free(tmp); free(Mc); free(are); free(aim);
    return 0;
}

/* The energy axis E_k = e_min + k (e_max - e_min) / (K - 1). */
void orc_energy_grid(const orc_problem *P, double *E)
{
    const int K = P->n_energies;
    for (int k = 0; k < K; ++k) E[k] = P->e_min + (double)k * (P->e_max - P->e_min) / (double)(K - 1);
}

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11) and Box-Muller.         */
/* ------------------------------------------------------------------------ */
static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    const unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(M0, x0, &hi0, &lo0);
        mulhilo64(M1, x2, &hi1, &lo1);
        const uint64_t y0 = hi1 ^ x1 ^ k0;
        const uint64_t y2 = hi0 ^ x3 ^ k1;
        x0 = y0;
        x1 = lo1;
        x2 = y2;
        x3 = lo0;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

/* A 64-bit word to a uniform double in the open interval (0, 1). */
static double u01(uint64_t x) { return ((double)(x >> 11) + 0.5) * (1.0 / 9007199254740992.0); }

/* The 2F standard normals of trajectory `index`: counter (index, block, 0, 0),
 * key (seed, 0); each block gives four uniforms, i.e. two Box-Muller pairs. */
void orc_normals(uint64_t seed, uint64_t index, int32_t count, double *out)
{
    const uint64_t key[2] = {seed, 0};
    for (int b = 0; 4 * b < count; ++b) {
        const uint64_t ctr[4] = {index, (uint64_t)b, 0, 0};
        uint64_t r[4];
        orc_philox4x64_10(ctr, key, r);
        for (int h = 0; h < 2; ++h) {
            const double u1 = u01(r[2 * h]), u2 = u01(r[2 * h + 1]);
            const double rad = sqrt(-2.0 * log(u1));
            const double ang = 2.0 * ORC_PI * u2;
            const int i0 = 4 * b + 2 * h;
            if (i0 < count) out[i0] = rad * cos(ang);
            if (i0 + 1 < count) out[i0 + 1] = rad * sin(ang);
        }
    }
}

/*
 * Husimi sampling of chi = |p_eq, q_eq>: the density is
 *   rho(p,q) = |<p,q|chi>|^2 / (2 pi)^F
 *            = prod_i (1/(2 pi)) exp(-gamma_i (q_i-q_eq,i)^2/2 - (p_i-p_eq,i)^2/(2 gamma_i)),
 * so q_i = q_eq,i + xi_i / sqrt(gamma_i), p_i = p_eq,i + eta_i sqrt(gamma_i), with
 * xi_i = normal #2i and eta_i = normal #(2i+1) of the trajectory.
 * Outputs are structure-of-arrays [F][n]; logrho is ln rho(p,q).
 */
void orc_sample_husimi(const orc_problem *P, uint64_t seed, uint64_t first_index, int64_t n,
                       double *p0, double *q0, double *logrho)
{
    const int F = P->F;
#pragma omp parallel
    {
        double *z = (double *)malloc(sizeof(double) * 2 * F);
#pragma omp for schedule(static)
        for (int64_t j = 0; j < n; ++j) {
            orc_normals(seed, first_index + (uint64_t)j, 2 * F, z);
            double sq = 0.0;
            for (int i = 0; i < F; ++i) {
                const double xi = z[2 * i], eta = z[2 * i + 1];
                q0[(int64_t)i * n + j] = P->q_eq[i] + xi / sqrt(P->gamma[i]);
                p0[(int64_t)i * n + j] = P->p_eq[i] + eta * sqrt(P->gamma[i]);
                sq += xi * xi + eta * eta;
            }
            logrho[j] = -(double)F * log(2.0 * ORC_PI) - 0.5 * sq;
        }
        free(z);
    }
}

/*
 * The whole estimator.  p0, q0 are [F][n] (structure of arrays), logrho [n].
 * Outputs (any may be NULL except spec_sum and n_good):
 *   spec_sum[K]   sum_j good_j w_j |A_j(E_k)|^2 (not yet normalised)
 *   n_good        number of good trajectories
 *   final_state   [n][orc_state_size(F)]
 *   contrib[n]    w_j sum_k |A_j(E_k)|^2 for good trajectories, else 0
 *   amps          [n][n_steps+1][2] amplitude time series
 * Partial sums are combined in thread order, so the result is reproducible
 * for a fixed thread count.
 */
int orc_run(const orc_problem *P, int64_t n, const double *p0, const double *q0, const double *logrho,
            double *spec_sum, int64_t *n_good, double *final_state, double *contrib, double *amps,
            int32_t n_threads)
{
    const int F = P->F, K = P->n_energies;
    const int64_t nt = (int64_t)P->n_steps + 1;
    const int64_t ss = orc_state_size(F);
    double *E = (double *)malloc(sizeof(double) * K);
    double *ctab = (double *)malloc(sizeof(double) * (size_t)(nt * K));
    double *stab = (double *)malloc(sizeof(double) * (size_t)(nt * K));
    if (!E || !ctab || !stab) {
        free(E); free(ctab); free(stab);
        return -1;
    }
    orc_energy_grid(P, E);
    for (int64_t c = 0; c < nt; ++c)
        for (int k = 0; k < K; ++k) {
            const double ph = E[k] * ((double)c * P->dt);
            ctab[c * K + k] = cos(ph);
            stab[c * K + k] = sin(ph);
        }
#ifdef _OPENMP
    int nth = n_threads > 0 ? n_threads : omp_get_max_threads();
#else
    int nth = 1;
    (void)n_threads;
#endif
    double *partial = (double *)calloc((size_t)nth * K, sizeof(double));
    int64_t *pgood = (int64_t *)calloc((size_t)nth, sizeof(int64_t));
    int err = 0;
#pragma omp parallel num_threads(nth)
    {
#ifdef _OPENMP
        const int tid = omp_get_thread_num();
#else
        const int tid = 0;
#endif
        double *st = (double *)malloc(sizeof(double) * (size_t)ss);
        double *amp = (double *)malloc(sizeof(double) * (size_t)(2 * nt));
        double *pz = (double *)malloc(sizeof(double) * 2 * F);
        double *my = partial + (size_t)tid * K;
        if (!st || !amp || !pz) {
#pragma omp atomic write
            err = -1;
        }
#pragma omp for schedule(static)
        for (int64_t j = 0; j < n; ++j) {
            if (!st || !amp || !pz) continue;
            for (int i = 0; i < F; ++i) {
                pz[i] = p0[(int64_t)i * n + j];
                pz[F + i] = q0[(int64_t)i * n + j];
            }
            orc_traj_init(P, pz, pz + F, st, amp);
            orc_traj_advance(P, st, P->n_steps, amp + 2);
            const int good = st[2 * F + ST_GOOD] != 0.0;
            const double w = exp(-logrho[j] - (double)F * log(2.0 * ORC_PI));
            double csum = 0.0;
            if (good) {
                pgood[tid] += 1;
                for (int k = 0; k < K; ++k) {
                    double ar = 0.0, ai = 0.0;
                    for (int64_t c = 0; c < nt; ++c) {
                        const double xr = amp[2 * c], xi = amp[2 * c + 1];
                        const double cr = ctab[c * K + k], ci = stab[c * K + k];
                        ar += xr * cr - xi * ci;
                        ai += xr * ci + xi * cr;
                    }
                    const double v = w * (ar * ar + ai * ai);
                    my[k] += v;
                    csum += v;
                }
            }
            if (contrib) contrib[j] = csum;
            if (final_state) memcpy(final_state + j * ss, st, sizeof(double) * (size_t)ss);
            if (amps) memcpy(amps + j * 2 * nt, amp, sizeof(double) * (size_t)(2 * nt));
        }
        free(st);
        free(amp);
        free(pz);
    }
    for (int k = 0; k < K; ++k) spec_sum[k] = 0.0;
    int64_t ng = 0;
    for (int t = 0; t < nth; ++t) {
        for (int k = 0; k < K; ++k) spec_sum[k] += partial[(size_t)t * K + k];
        ng += pgood[t];
    }
    *n_good = ng;
    free(partial);
    free(pgood);
    free(E);
    free(ctab);
    free(stab);
    return err;
}

/* I_k = dt^2 / (2 pi T n_good) spec_sum_k, T = n_steps dt; zero if n_good = 0. */
void orc_normalise(const orc_problem *P, const double *spec_sum, int64_t n_good, double *I)
{
    const double T = (double)P->n_steps * P->dt;
    for (int k = 0; k < P->n_energies; ++k)
        I[k] = n_good > 0 ? P->dt * P->dt / (2.0 * ORC_PI * T * (double)n_good) * spec_sum[k] : 0.0;
}
