// Time-averaged SC-IVR spectral density without the separable approximation
// (Eq. (9) with the Herman-Kluk prefactor of each trajectory segment), FP64,
// F <= 16.
//
// Eq. (9) integrates over two times t1 <= t2 of one trajectory, and the
// prefactor C_{t2}(z(t1)) belongs to the trajectory that starts at the
// phase-space point z(t1) and runs to t2: sqrt(det A) of Eq. (5) built from
// the tangent map of the segment [t1, t2], on the square-root branch that is
// continuous in t2 from C = 1 at t2 = t1.  On the time samples of Eq. (11),
// with the diagonal weighted 1/2 (so that the separable prefactor
// exp(i (phi(t2) - phi(t1))) gives Eq. (11) exactly), the sum over t1 <= t2
// regroups by lag tau = c2 - c1 into
//
//   R_j(tau) = sum_{c1} omega C_j(c1, c1 + tau) a_j(c1 + tau) conj(a_j(c1)),
//   a_j(c) = <chi|z_j(c)> e^{i S_j(c)},   omega = 1/2 at tau = 0, else 1,
//
// and sum_j w_j good_j 2 Re sum_tau R_j(tau) e^{i E tau dt} takes the place of
// sum_j w_j good_j |A_j(E)|^2 (normalised as Eq. (11)).  The segment's own
// action S(c1 + tau) - S(c1) and amplitude <chi|z(c1 + tau)> e^{i S_seg}
// give the product a(c2) conj(a(c1)) = <chi|z(c2)> e^{i S_seg} conj(<chi|z(c1)>).
//
// Kernels:
//  * ta_full_kernel: one wave per (trajectory j, split s).  A group of F
//    lanes runs one segment at a time, laid out as the small-F trajectory
//    kernel lays out a trajectory (lane c: mode c and tangent columns c, F + c).
//    In round r the wave's W = 64 / F groups run the segments c1 = r W + g
//    (g the group), and the split s takes the rounds r = s, s + S, ...  Each
//    group also carries a cursor on the trajectory itself (positions only,
//    the same step code), advanced to its next c1 between rounds.  A segment
//    propagates its tangent map from the identity, takes det A by complex
//    elimination every step and keeps the branch as the main kernel does.
//    Each lag leaves det A, the action and the modes' q and p in the group's
//    ring; every eight lags (every F at F < 8) lanes 0..7 of the group finish
//    one lag each (|C|, the branch with its increments added in lag order, the
//    overlap, exp and sincos), and lanes 0..7 of the wave sum the groups'
//    terms of those lags in group order into the wave's rows part[s][tau][j]
//    (each row belongs to one wave: no atomics).
//    Segments do not run the stability monitor: only the trajectory's own
//    flag (from the propagation) enters the estimate.
//  * ta_lags_kernel: C(tau) = sum_j weight_j sum_s part[s][tau][j], in fixed
//    order, with the zero lag doubled for the spectrum evaluation.
#include <math.h>

#include "group_lu.h"
#include "scivr_internal.h"
#include "traj_common.h"

namespace scivr {
namespace {

template <int F>
struct alignas(16) FullGroupLds {
    static constexpr int RB = F < 8 ? F : 8;  // lags per ring
    double pivA[2 * F];
    unsigned keys[(F + 3) & ~3];
    double qv[F], pm[F], ph[F], pv[F];
    // ring of the last RB lags: each mode's q and p, the raw det(A), the
    // action, and the argument that advances the branch
    double rq[RB][F], rp[RB][F];
    double rdr[RB], rdi[RB], rS[RB], ra[RB];
};

// One fourth-order triple-jump step of the group's trajectory: positions,
// momenta and (TANGENT) the action and the two tangent columns of lane c.
template <int F, bool TANGENT>
__device__ inline void full_step(const ProblemDev *P0, FullGroupLds<F> &L, const double *lam_lds, int c, double &pc,
                                 double &qc, double &S, double (&dpP)[F], double (&dqP)[F], double (&dpQ)[F],
                                 double (&dqQ)[F])
{
    ConstProblem Pc = opaque(P0);
    const double kc = Pc->k[c], Dc = Pc->D[c], ac = Pc->a[c];
#pragma unroll 1
    for (int s = 0; s < 4; ++s) {
        ConstProblem Pk = opaque(P0);
        const double h = Pk->hd[s];
        if (TANGENT && c == 0) {
            double kin = 0.0;
#pragma unroll
            for (int i = 0; i < F; ++i) kin += 0.5 * L.pm[i] * L.pm[i];
            S += h * kin;
        }
        qc = fma(h, pc, qc);
        if constexpr (TANGENT) {
#pragma unroll
            for (int i = 0; i < F; ++i) {
                dqP[i] = fma(h, dpP[i], dqP[i]);
                dqQ[i] = fma(h, dpQ[i], dqQ[i]);
            }
        }
        lds_order();
        L.qv[c] = qc;
        lds_order();
        if (s == 3) break;
        const double hk = Pk->hc[s];
        double q[F];
#pragma unroll
        for (int i = 0; i < F; ++i) q[i] = L.qv[i];
        double sm = 0.0;
#pragma unroll
        for (int i = 0; i < F; ++i) sm = fma(lam_lds[c * F + i], q[i] * q[i], sm);
        const double e = dexp(-ac * qc, &Pk->mc);
        const double one_e = 1.0 - e;
        const double gc = kc * qc + 2.0 * Dc * ac * e * one_e + 2.0 * qc * sm;
        const double hc = kc + 2.0 * Dc * ac * ac * e * (2.0 * e - 1.0) + 2.0 * sm;
        const double vc = 0.5 * kc * qc * qc + Dc * one_e * one_e + 0.5 * qc * qc * sm;
        pc = fma(-hk, gc, pc);
        L.ph[c] = hc;
        L.pv[c] = vc;
        L.pm[c] = pc;
        lds_order();
        if constexpr (TANGENT) {
            if (c == 0) {
                double V = 0.0;
#pragma unroll
                for (int i = 0; i < F; ++i) V += L.pv[i];
                S -= hk * V;
            }
            // dp -= hk (h o dq + 4 q o Lambda (q o dq)), column by column
#pragma unroll
            for (int col = 0; col < 2; ++col) {
                double(&dp)[F] = col ? dpQ : dpP;
                double(&dq)[F] = col ? dqQ : dqP;
                double u[F], w[F];
#pragma unroll
                for (int i = 0; i < F; ++i) {
                    u[i] = q[i] * dq[i];
                    w[i] = 0.0;
                }
#pragma unroll
                for (int i = 0; i < F; ++i)
#pragma unroll
                    for (int jj = i + 1; jj < F; ++jj) {
                        const double l = Pk->lam[i * FMAX + jj];
                        w[i] = fma(l, u[jj], w[i]);
                        w[jj] = fma(l, u[i], w[jj]);
                    }
#pragma unroll
                for (int i = 0; i < F; ++i) dp[i] = fma(-hk, fma(L.ph[i], dq[i], 4.0 * q[i] * w[i]), dp[i]);
            }
        }
        lds_order();
    }
}

// exponent and phase of <chi_m|p,q> (reference state m, 0 = chi) for the
// modes' positions q[i] and momenta p[i]
template <int F>
__device__ inline double overlap_of(ConstProblem P, int m, const double *q, const double *p, double &ph)
{
    double ex = 0.0;
    ph = 0.0;
#pragma unroll
    for (int i = 0; i < F; ++i) {
        const double dqe = P->ref_q[m][i] - q[i];
        const double dpe = P->ref_p[m][i] - p[i];
        ex += -0.25 * P->gamma[i] * dqe * dqe - dpe * dpe * P->inv4gamma[i];
        ph += 0.5 * dqe * (P->ref_p[m][i] + p[i]);
    }
    return ex;
}

// det(A) rescaled by a power of two (the branch only needs its argument)
__device__ inline void rescale(double &dr, double &di)
{
    int e2;
    (void)frexp(fmax(fabs(dr), fabs(di)), &e2);
    dr = ldexp(dr, -e2);
    di = ldexp(di, -e2);
}

// Waves per SIMD the register allocator must allow (unified 512-register
// file).  For 7 <= F <= 16 the kernel would take more than 256 registers and
// run one wave per SIMD, where nothing hides the LDS round trips of the
// eliminations; two waves with some spilling are faster.  Smaller F already
// fits two or more waves.
template <int F>
constexpr int full_waves() { return (F >= 7 && F <= 16) ? 2 : 1; }

template <int F>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(full_waves<F>(), 8)))
ta_full_kernel(FullArgs A, const ProblemDev *__restrict__ P0)
{
    constexpr int W = 64 / F;
    __shared__ FullGroupLds<F> lds_all[W];
    __shared__ double lam_lds[F * F];
    constexpr int RB = FullGroupLds<F>::RB;
    __shared__ double2 term[W][RB];
    const int lane = threadIdx.x;
    for (int idx = lane; idx < F * F; idx += 64) lam_lds[idx] = P0->lam[(idx / F) * FMAX + idx % F];
    const int g = lane / F;
    if (g >= W) return;  // lanes beyond the last group; nothing below synchronises the workgroup
    const int c = lane - g * F;
    FullGroupLds<F> &L = lds_all[g];
    const int64_t j = blockIdx.x / A.splits;
    const int split = (int)(blockIdx.x % A.splits);
    const int64_t NP = A.npad;
    const int ns = A.n_steps;
    ConstProblem P = opaque(P0);
    const double sgc = P->sqrt_gamma[c], isgc = P->inv_sqrt_gamma[c];

    // the cursor on trajectory j (positions only), at time sample `cur`
    double pm = A.p0[c * NP + j], qm = A.q0[c * NP + j];
    int cur = 0;
    double dpP[F], dqP[F], dpQ[F], dqQ[F];
    double2 *out = A.part + ((int64_t)split * A.nt) * NP + j;  // row part[split][tau][j]

    for (int r = split; r * W <= ns; r += A.splits) {
        const int c1 = r * W + g;
        // advance the group's cursor to its c1 (groups past the end stop at ns)
        const int target = min(c1, ns);
        for (; cur < target; ++cur) {
            double Sx = 0.0;
            L.pm[c] = pm;
            L.qv[c] = qm;
            lds_order();
            full_step<F, false>(P0, L, lam_lds, c, pm, qm, Sx, dpP, dqP, dpQ, dqQ);
        }
        // the segment from z(c1): identity tangent map, zero action, branch at C = 1
        const bool seg = c1 <= ns;
        double pc = pm, qc = qm, S = 0.0;
#pragma unroll
        for (int i = 0; i < F; ++i) {
            dpP[i] = (i == c) ? 1.0 : 0.0;
            dqP[i] = 0.0;
            dpQ[i] = 0.0;
            dqQ[i] = (i == c) ? 1.0 : 0.0;
        }
        L.pm[c] = pc;
        L.qv[c] = qc;
        lds_order();
        double ph1;
        const double ex1 = overlap_of<F>(P, A.ref, L.qv, L.pm, ph1);  // <chi_m|z(c1)>
        // the branch through the lags finished so far: theta, and det(A) of the
        // last of them rescaled (kept by the lanes c < RB that finish lags)
        double theta = 0.0, prev_r = 1.0, prev_i = 0.0;
        const int len = ns - r * W;  // lags of the round's longest segment (g = 0)
        {
            // lag 0: C = 1, (1/2) |<chi|z(c1)>|^2
            ConstProblem Ps = opaque(P0);
            const double x0 = (c == 0) ? 0.5 * dexp(2.0 * ex1, &Ps->mc) : 0.0;
            const bool live = seg && isfinite(x0);
            lds_order();
            if (c == 0) term[g][0] = make_double2(live ? x0 : 0.0, 0.0);
            lds_order();
            if (lane == 0) {
                double sr = 0.0, si = 0.0;
                for (int gg = 0; gg < W; ++gg) {
                    sr += term[gg][0].x;
                    si += term[gg][0].y;
                }
                double2 *o = out;
                double2 v = *o;
                v.x += sr;
                v.y += si;
                *o = v;
            }
            lds_order();
        }
        int nk = 0;  // lags in the ring
        for (int tau = 1; tau <= len; ++tau) {
            ConstProblem Ps = opaque(P0);
            full_step<F, true>(P0, L, lam_lds, c, pc, qc, S, dpP, dqP, dpQ, dqQ);
            double are[F], aim[F];
#pragma unroll
            for (int i = 0; i < F; ++i) {
                const double si = Ps->sqrt_gamma[i], isi = Ps->inv_sqrt_gamma[i];
                are[i] = 0.5 * (si * dqQ[i] * isgc + dpP[i] * sgc * isi);
                aim[i] = 0.5 * (-si * dqP[i] * sgc + dpQ[i] * isi * isgc);
            }
            double dAr, dAi;
            lu_det_complex<F>(are, aim, c, L.pivA, L.keys, dAr, dAi);
            L.rq[nk][c] = qc;
            L.rp[nk][c] = pc;
            if (c == 0) {
                L.rdr[nk] = dAr;
                L.rdi[nk] = dAi;
                L.rS[nk] = S;
            }
            ++nk;
            if (nk < RB && tau < len) continue;
            // Finish the ring's lags tau0 .. tau0 + nk - 1, lane c < nk taking
            // lag tau0 + c: |C| = |det A|^(1/2); the branch as in the
            // propagation (theta accumulates the principal argument of
            // det(A_t) conj(det(A_{t-dt})) e^{i dt sum gamma}, on det(A) rescaled
            // by a power of two), its arguments added in lag order.
            const int tau0 = tau - nk + 1;
            lds_order();
            double mod = 0.0;
            if (c < nk) {
                double dr = L.rdr[c], di = L.rdi[c];
                mod = sqrt(hypot(dr, di));
                rescale(dr, di);
                double qr = prev_r, qi = prev_i;
                if (c > 0) {
                    qr = L.rdr[c - 1];
                    qi = L.rdi[c - 1];
                    rescale(qr, qi);
                }
                const double ur = dr * qr + di * qi;
                const double ui = di * qr - dr * qi;
                const double zr = ur * Ps->cos_gdt - ui * Ps->sin_gdt;
                const double zi = ur * Ps->sin_gdt + ui * Ps->cos_gdt;
                L.ra[c] = datan2(zi, zr, &Ps->mc);
            }
            lds_order();
            if (c < nk) {
                const int tk = tau0 + c;
                double th = theta;
                for (int kk = 0; kk <= c; ++kk) th += L.ra[kk];
                const double phi = 0.5 * (th - Ps->sum_gamma * ((double)tk * Ps->dt));
                double ph;
                const double ex = overlap_of<F>(Ps, A.ref, L.rq[c], L.rp[c], ph);
                const double mag = mod * dexp(ex + ex1, &Ps->mc);
                double sn, cs;
                dsincos(phi + ph + L.rS[c] - ph1, &Ps->mc, &sn, &cs);
                const double xr = mag * cs, xi = mag * sn;
                const bool live = seg && c1 + tk <= ns && isfinite(xr) && isfinite(xi);
                term[g][c] = make_double2(live ? xr : 0.0, live ? xi : 0.0);
                // the branch carried to the next ring (the same on every such lane)
                for (int kk = c + 1; kk < nk; ++kk) th += L.ra[kk];
                theta = th;
                prev_r = L.rdr[nk - 1];
                prev_i = L.rdi[nk - 1];
                rescale(prev_r, prev_i);
            }
            lds_order();
            // the groups' terms of each lag, summed in group order by lane tau - tau0
            if (lane < nk) {
                double sr = 0.0, si = 0.0;
                for (int gg = 0; gg < W; ++gg) {
                    sr += term[gg][lane].x;
                    si += term[gg][lane].y;
                }
                double2 *o = out + (int64_t)(tau0 + lane) * NP;
                double2 v = *o;
                v.x += sr;
                v.y += si;
                *o = v;
            }
            lds_order();
            nk = 0;
        }
    }
}

// C(tau) = sum_j weight_j sum_s part[s][tau][j] (fixed order), zero lag doubled:
// the spectrum then adds C(0) + 2 Re sum_{tau >= 1} C(tau) e^{i E tau dt}.
__global__ void __launch_bounds__(256) ta_lags_kernel(const double2 *__restrict__ part, const double *__restrict__ weight,
                                                      int64_t n, int64_t npad, int nt, int splits,
                                                      double2 *__restrict__ C)
{
    __shared__ double2 red[256];
    const int tau = blockIdx.x;
    const int t = threadIdx.x;
    double sr = 0.0, si = 0.0;
    for (int64_t j = t; j < n; j += 256) {
        const double w = weight[j];
        if (w == 0.0) continue;
        double rr = 0.0, ri = 0.0;
        for (int s = 0; s < splits; ++s) {
            const double2 v = part[((int64_t)s * nt + tau) * npad + j];
            rr += v.x;
            ri += v.y;
        }
        sr = fma(w, rr, sr);
        si = fma(w, ri, si);
    }
    red[t] = make_double2(sr, si);
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) {
            red[t].x += red[t + h].x;
            red[t].y += red[t + h].y;
        }
        __syncthreads();
    }
    if (t == 0) C[tau] = tau == 0 ? make_double2(2.0 * red[0].x, 2.0 * red[0].y) : red[0];
}

template <int F>
hipError_t launch_full_F(const FullArgs &a, hipStream_t s)
{
    const int64_t blocks = a.n * a.splits;
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL((ta_full_kernel<F>), dim3((unsigned)blocks), dim3(64), 0, s, a, a.prob);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_ta_full(int F, const FullArgs &a, hipStream_t s)
{
    switch (F) {
    case 1: return launch_full_F<1>(a, s);
    case 2: return launch_full_F<2>(a, s);
    case 3: return launch_full_F<3>(a, s);
    case 4: return launch_full_F<4>(a, s);
    case 5: return launch_full_F<5>(a, s);
    case 6: return launch_full_F<6>(a, s);
    case 7: return launch_full_F<7>(a, s);
    case 8: return launch_full_F<8>(a, s);
    case 9: return launch_full_F<9>(a, s);
    case 10: return launch_full_F<10>(a, s);
    case 11: return launch_full_F<11>(a, s);
    case 12: return launch_full_F<12>(a, s);
    case 13: return launch_full_F<13>(a, s);
    case 14: return launch_full_F<14>(a, s);
    case 15: return launch_full_F<15>(a, s);
    case 16: return launch_full_F<16>(a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_ta_lags(const FullArgs &a, const double *weight, double2 *C, hipStream_t s)
{
    hipLaunchKernelGGL(ta_lags_kernel, dim3((unsigned)a.nt), dim3(256), 0, s, a.part, weight, a.n, a.npad, a.nt,
                       a.splits, C);
    return hipGetLastError();
}

}  // namespace scivr
