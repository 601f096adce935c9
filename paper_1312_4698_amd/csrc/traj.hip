// Trajectory kernel of the TA-SC-IVR spectrum for gfx950, F <= 16, in the FP64
// and the mixed-precision form.
//
// One trajectory is owned by a group of F lanes of a wave64 (floor(64/F)
// trajectories per wave).  Lane c owns degree of freedom c:
//  * during the symplectic step it carries two columns of the 2F x 2F
//    monodromy matrix M = d(p_t, q_t)/d(p_0, q_0): the tangent vectors of the
//    initial directions p0_c and q0_c; it also carries the trajectory's p and
//    q, and evaluates the Morse terms of mode c, which it shares with the
//    group through LDS;
//  * after each step the group takes det(A) of the Herman-Kluk prefactor
//    matrix of Eq. (5) (complex, F x F) and det(M) (real, 2F x 2F; the
//    stability monitor after Eq. (5)) as the determinants of the transposes,
//    whose rows are the columns lane c already holds: column c of A (one row of
//    A^T per lane) and columns c, F + c of M (two rows of M^T per lane), so
//    no transpose is needed.  Gaussian elimination with partial pivoting runs
//    across the group's lanes: each lane publishes one packed (|a|, position)
//    key, every lane reads the group's keys back and takes their maximum, the
//    pivot lane publishes its row, the live rows read it back as a broadcast.
//
// The fourth-order symplectic step is the drift-kick-drift triple jump
// (Yoshida / Forest-Ruth); each kick evaluates gradient, Hessian and potential
// of V = sum_i [k_i q_i^2/2 + D_i (1 - e^{-a_i q_i})^2] + sum_{i<j} l_ij q_i^2 q_j^2
// and applies the Hessian to each tangent column in factored form,
//   H dq = h o dq + 4 q o (Lambda (q o dq)),  h_i = d^2V/dq_i^2,
// with Lambda the symmetric zero-diagonal coupling matrix (scalar operands).
// The action follows the discrete Lagrangian of the stages (+h |p|^2/2 per
// drift, -h V per kick).  The prefactor phase is kept on a continuous branch
// by accumulating the principal argument of det(A_t) conj(det(A_{t-dt}))
// e^{i dt sum gamma}; phi = (theta - t sum gamma)/2 (the separable
// approximation after Eq. (9)).  Each step writes the amplitude
// <chi|p_t,q_t> e^{i (S_t + phi_t)} (zero once the trajectory is flagged) into
// the left operand of the Fourier GEMM: a time-major [t][trajectory] FP64
// matrix, or in the mixed form FP16 hi/lo planes [t / 8][trajectory][t % 8].
#include <math.h>

#include <type_traits>

#include "scivr_internal.h"
#include "traj_common.h"
#include "group_lu.h"

namespace scivr {
namespace {

// Waves per SIMD the register allocator must allow (unified 512-register file).
template <int F>
constexpr int traj_waves() { return F <= 3 ? 4 : (F <= 6 ? 3 : (F <= 12 ? 2 : 1)); }

template <int F, bool MULTI>
struct GroupCore {
    static constexpr int N2 = 2 * F;
    static constexpr int KS = (F + 3) & ~3;
    static constexpr int RB = F < 8 ? F : 8;  // time samples per amplitude ring
    // the overlap's mode terms and the action's parts go through the ring (one
    // per lane) where the kernel runs at most two waves per SIMD; with more
    // waves the LDS it takes would cost occupancy, and lane 0 sums them itself.
    // With several reference states (MULTI) every lane puts its mode's q and p
    // into the ring instead, and the lanes that finish a time sample form each
    // reference state's overlap from them.
    static constexpr bool OVL = traj_waves<F>() <= 2;
    static constexpr int OT = (OVL || MULTI) ? F : 1;
    static constexpr int ST = OVL ? F : 1;
    double pivM[N2];                   // pivot row of the real elimination
    double pivA[N2];                   // pivot row of the complex elimination (re, im interleaved)
    unsigned keys[KS];                 // one pivot key per lane of the group
    // amplitude ring: per time sample, each mode's terms of the exponent and
    // the phase of <chi|p,q>, the action, the det(A) ratio z whose argument
    // advances the prefactor branch, the status flag, and the branch increment
    double rex[RB][OT], rph[RB][OT];  // without OVL: lane 0's sums, the phase with the action added; MULTI: q, p
    double rS[RB][ST];                 // with OVL: each lane's part of the action; MULTI without OVL: lane 0's
    double rzr[RB], rzi[RB], rinc[RB];
    double rtheta, rphi;               // branch and prefactor phase after the last finished sample
    double prev_r, prev_i;             // det(A) of the last step, rescaled
    double detM, maxdev;               // the monitor's last det(M) and largest |det(M)^2 - 1|
    int rflag[RB];
    int rgood;
};

// A group's LDS block, padded to an odd multiple of 16 B: the groups of a
// wave then start 4 * odd banks apart modulo the 64 four-byte banks, so up to
// 16 groups' simultaneous 16-byte broadcast reads fall into different banks.
template <int F, bool MULTI>
struct alignas(16) GroupLds : GroupCore<F, MULTI> {
    static constexpr int BYTES = (int)((sizeof(GroupCore<F, MULTI>) + 15) & ~(size_t)15);
    static constexpr int PADB = ((BYTES / 16) % 2 == 0) ? 16 : 0;
    static constexpr int PADN = (BYTES - (int)sizeof(GroupCore<F, MULTI>)) + PADB;
    char pad[PADN > 0 ? PADN : 32];  // 32 keeps the parity where no padding is needed
};

// The trajectory kernel.  MIXED = false: every trajectory quantity in FP64.
// MIXED = true: the trajectory (p, q), the potential, gradient and Hessian
// diagonal and the action (Kahan-compensated) in FP32; the tangent columns,
// det(A), det(M) and the phase branch stay in FP64; the amplitude, scaled by a
// per-trajectory power of two 2^e (e = min(floor(-log2 |<chi|z_0>|) + 3, 15)) so
// that both FP16 parts of its components stay normal and none can overflow, is stored as FP16 hi/lo planes
// [re_hi, re_lo, im_hi, im_lo][t / 8][trajectory][t % 8] for the FP16 GEMM.
// MULTI (FP64 only): amplitudes for each of A.n_refs reference states of the
// problem's widths, [t][ref][trajectory].
template <int F, bool MIXED, bool MULTI>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(traj_waves<F>(), 8)))
traj_kernel(TrajArgs A, const ProblemDev *__restrict__ P0)
{
    static_assert(!(MIXED && MULTI), "several reference states run in the FP64 form");
    typedef typename std::conditional<MIXED, float, double>::type R;
    constexpr int N2 = 2 * F;
    constexpr int TPW = 64 / F;
    __shared__ GroupLds<F, MULTI> lds_all[TPW];
    __shared__ double lam_lds[F * F];  // coupling matrix, shared by the wave's groups
    static_assert((sizeof(GroupLds<F, MULTI>) / 16) % 2 == 1, "group stride must be an odd multiple of 16 B");
    __shared__ R qv_all[TPW][F + (F & 1)], pm_all[TPW][F + (F & 1)];
    __shared__ R ph_all[TPW][F + (F & 1)], pv_all[TPW][F + (F & 1)];
    // The p halves of the lane's two monodromy columns wait in LDS while the
    // eliminations run where the register file cannot hold them, the rows of
    // M^T and the pivot traffic at once (F <= 6, three or four waves per SIMD;
    // at two waves per SIMD the LDS round trip costs more than it saves).
    constexpr bool STASH = F <= 6;
    constexpr bool OVL = GroupCore<F, MULTI>::OVL;
    const int NR = MULTI ? A.n_refs : 1;  // reference states
    __shared__ double stash_all[STASH ? TPW : 1][2][F][F];

    const int lane = threadIdx.x;
    const ProblemDev *__restrict__ P = P0;
    for (int idx = lane; idx < F * F; idx += 64) lam_lds[idx] = P->lam[(idx / F) * FMAX + idx % F];
    const int grp = lane / F;
    // Lanes beyond the last full group own no trajectory.  They leave once the
    // shared table is written; nothing below synchronises the workgroup, so the
    // rest of the wave runs on with them masked off.
    if (grp >= TPW) return;
    const int c = lane - grp * F;  // degree of freedom owned by this lane
    GroupLds<F, MULTI> &L = lds_all[grp];
    R *qv = qv_all[grp], *pm = pm_all[grp], *phd = ph_all[grp], *pv = pv_all[grp];
    const int64_t j = (int64_t)blockIdx.x * TPW + grp;
    const bool live = j < A.n;
    const int64_t jr = live ? j : 0;
    const int64_t NP = A.npad;

    // constants of the lane's own mode c
    const R kc = (R)P->k[c], Dc = (R)P->D[c], ac = (R)P->a[c];
    const double sgc = P->sqrt_gamma[c], isgc = P->inv_sqrt_gamma[c];

    // pc, qc: the trajectory's momentum and position of mode c (the group's
    // full p and q live in LDS); columns c ("P": d/dp0_c) and F + c ("Q":
    // d/dq0_c) of M, split into their p and q halves.
    double dpP[F], dqP[F], dpQ[F], dqQ[F];
    R pc, qc;
    Action<MIXED> S;
    double theta, prev_r, prev_i, phi, detM, maxdev;  // held in the group's LDS block while the steps run
    int escale = 0;  // amplitude scale exponent (mixed form)
    bool good;
    if (A.step_begin == 0) {
#pragma unroll
        for (int i = 0; i < F; ++i) {
            dpP[i] = (i == c) ? 1.0 : 0.0;
            dqP[i] = 0.0;
            dpQ[i] = 0.0;
            dqQ[i] = (i == c) ? 1.0 : 0.0;
        }
        pc = (R)A.p0[c * NP + jr];
        qc = (R)A.q0[c * NP + jr];
        theta = phi = prev_i = 0.0;
        prev_r = 1.0;  // det(A) = 1 at t = 0
        detM = 1.0;
        maxdev = 0.0;
        good = true;
    } else {
#pragma unroll
        for (int i = 0; i < F; ++i) {
            dpP[i] = A.Mst[(int64_t)(i * N2 + c) * NP + jr];
            dqP[i] = A.Mst[(int64_t)((F + i) * N2 + c) * NP + jr];
            dpQ[i] = A.Mst[(int64_t)(i * N2 + F + c) * NP + jr];
            dqQ[i] = A.Mst[(int64_t)((F + i) * N2 + F + c) * NP + jr];
        }
        pc = (R)A.p[c * NP + jr];
        qc = (R)A.q[c * NP + jr];
        if constexpr (OVL)
            S.unpack(A.spart[c * NP + jr]);  // this lane's part, bit for bit
        else if (c == 0)
            S.load(A.scal[SC_S * NP + jr], A.scal[SC_SCOMP * NP + jr]);
        theta = A.scal[SC_THETA * NP + jr];
        prev_r = A.scal[SC_PREV_RE * NP + jr];
        prev_i = A.scal[SC_PREV_IM * NP + jr];
        phi = A.scal[SC_PHI * NP + jr];
        good = A.scal[SC_GOOD * NP + jr] != 0.0;
        detM = A.scal[SC_DETM * NP + jr];
        maxdev = A.scal[SC_MAXDEV * NP + jr];
        escale = (int)A.scal[SC_ESCALE * NP + jr];
    }
    qv[c] = qc;
    pm[c] = pc;
    if (c == 0) {
        L.rtheta = theta;
        L.rphi = phi;
        L.prev_r = prev_r;
        L.prev_i = prev_i;
        L.detM = detM;
        L.maxdev = maxdev;
    }
    lds_order();

    // exponent of <chi|p,q> of the published state
    auto overlap = [&](auto PP, double &ph) -> double {
        double ex = 0.0;
        ph = 0.0;
#pragma unroll
        for (int i = 0; i < F; ++i) {
            const double qi = (double)qv[i], pi = (double)pm[i];
            const double dqe = PP->q_eq[i] - qi;
            const double dpe = PP->p_eq[i] - pi;
            ex += -0.25 * PP->gamma[i] * dqe * dqe - dpe * dpe * PP->inv4gamma[i];
            ph += 0.5 * dqe * (PP->p_eq[i] + pi);
        }
        return ex;
    };
    // exponent and phase of <chi_m|p,q> for reference state m from the modes' q, p
    auto overlap_ref = [&](auto PP, int m, const double *qs, const double *ps, double &ph) -> double {
        double ex = 0.0;
        ph = 0.0;
#pragma unroll
        for (int i = 0; i < F; ++i) {
            const double dqe = PP->ref_q[m][i] - qs[i];
            const double dpe = PP->ref_p[m][i] - ps[i];
            ex += -0.25 * PP->gamma[i] * dqe * dqe - dpe * dpe * PP->inv4gamma[i];
            ph += 0.5 * dqe * (PP->ref_p[m][i] + ps[i]);
        }
        return ex;
    };
    // store the amplitude e^{ex} e^{i phase} of time sample t (zero when bad)
    auto put_amplitude = [&](auto PP, int t, double ex, double phase, bool g, int m = 0) {
        double s, co;
        dsincos(phase, &PP->mc, &s, &co);
        if constexpr (!MIXED) {
            const double mag = dexp(ex, &PP->mc);
            double2 r;
            r.x = g ? mag * co : 0.0;
            r.y = g ? mag * s : 0.0;
            A.amp[((int64_t)t * NR + m) * NP + jr] = r;
        } else {
            const double mag = ldexp(dexp(ex, &PP->mc), escale);
            const float re = g ? (float)(mag * co) : 0.f, im = g ? (float)(mag * s) : 0.f;
            _Float16 h[4];
            split_f16(re, h[0], h[1]);
            split_f16(im, h[2], h[3]);
            const int64_t e = ((int64_t)(t >> 3) * NP + jr) * 8 + (t & 7);
#pragma unroll
            for (int pl = 0; pl < 4; ++pl) A.amp16[pl * A.plane + e] = h[pl];
        }
    };
    // the amplitude <chi|p,q> e^{i(S + phi)} of the published state (each reference state's)
    auto store_amplitude = [&](auto PP, int t) {
        if constexpr (MULTI) {
            double qs[F], ps[F];
#pragma unroll
            for (int i = 0; i < F; ++i) {
                qs[i] = (double)qv[i];
                ps[i] = (double)pm[i];
            }
            for (int m = 0; m < NR; ++m) {
                double ph;
                const double ex = overlap_ref(PP, m, qs, ps, ph);
                put_amplitude(PP, t, ex, ph + S.value() + phi, good, m);
            }
        } else {
            double ph;
            const double ex = overlap(PP, ph);
            put_amplitude(PP, t, ex, ph + S.value() + phi, good);
        }
    };

    if (A.step_begin == 0) {
        if constexpr (MIXED) {  // every lane: the ring's lanes store with it
            double ph;
            const double ex0 = overlap(P, ph);
            // 2^escale: the power of two that puts |<chi|z_0>| 2^escale in (4, 8], so
            // both FP16 parts stay normal (about 22 bits), capped at 2^15: since
            // |<chi|z_t>| <= 1, no later amplitude can then exceed 2^15 < 65504
            escale = (int)fmin(floor(-ex0 * 1.4426950408889634) + 3.0, 15.0);
        }
        if (c == 0 && live) store_amplitude(P, 0);
    }

    for (int step = A.step_begin; step < A.step_end; ++step) {
        ConstProblem Ps = opaque(P0);
#pragma unroll 1
        for (int s = 0; s < 4; ++s) {
            ConstProblem Pk = opaque(P0);
            // ---- drift ----
            const double h = Pk->hd[s];
            if constexpr (OVL) {  // each lane carries its mode's part of the action
                S.add(h * (double)((R)0.5 * pc * pc));
            } else if (c == 0) {  // lane 0 carries the whole action
                R kin = 0;
#pragma unroll
                for (int i = 0; i < F; ++i) {
                    const R pi = pm[i];
                    kin += (R)0.5 * pi * pi;
                }
                S.add(h * (double)kin);
            }
            qc = fma((R)h, pc, qc);
#pragma unroll
            for (int i = 0; i < F; ++i) {
                dqP[i] = fma(h, dpP[i], dqP[i]);
                dqQ[i] = fma(h, dpQ[i], dqQ[i]);
            }
            lds_order();
            qv[c] = qc;
            lds_order();
            if (s == 3) break;
            // ---- kick: mode c's terms, shared through LDS ----
            const double hk = Pk->hc[s];
            R q[F];
#pragma unroll
            for (int i = 0; i < F; ++i) q[i] = qv[i];
            R sm = 0;
#pragma unroll
            for (int i = 0; i < F; ++i) sm = fma((R)lam_lds[c * F + i], q[i] * q[i], sm);
            R e;
            if constexpr (MIXED)
                e = expf(-ac * qc);
            else
                e = dexp(-ac * qc, &Pk->mc);
            const R one_e = (R)1 - e;
            const R gc = kc * qc + (R)2 * Dc * ac * e * one_e + (R)2 * qc * sm;
            const R hc = kc + (R)2 * Dc * ac * ac * e * ((R)2 * e - (R)1) + (R)2 * sm;
            const R vc = (R)0.5 * kc * qc * qc + Dc * one_e * one_e + (R)0.5 * qc * qc * sm;
            pc = fma(-(R)hk, gc, pc);
            phd[c] = hc;
            if constexpr (!OVL) pv[c] = vc;
            pm[c] = pc;
            lds_order();
            if constexpr (OVL) {
                S.add(-hk * (double)vc);
            } else if (c == 0) {
                R V = 0;
#pragma unroll
                for (int i = 0; i < F; ++i) V += pv[i];
                S.add(-hk * (double)V);
            }
            // tangent kick, one column after the other: dp -= hk (h o dq + 4 q o Lambda (q o dq))
#pragma unroll
            for (int col = 0; col < 2; ++col) {
                double(&dp)[F] = col ? dpQ : dpP;
                double(&dq)[F] = col ? dqQ : dqP;
                double u[F], w[F];
#pragma unroll
                for (int i = 0; i < F; ++i) {
                    u[i] = (double)q[i] * dq[i];
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
                for (int i = 0; i < F; ++i)
                    dp[i] = fma(-hk, fma((double)phd[i], dq[i], 4.0 * (double)q[i] * w[i]), dp[i]);
            }
            lds_order();
        }

        const int stp = step + 1;

        // det(A) = det(A^T) and det(M) = det(M^T): the rows of the transposes are
        // columns, and lane c already holds columns c (d/dp0_c) and F + c
        // (d/dq0_c) of M, so it forms column c of A and rows c, F + c of M^T
        // from its own registers, with no transpose.
        double dAr, dAi;
        {
            double are[F], aim[F];
#pragma unroll
            for (int i = 0; i < F; ++i) {
                const double si = Ps->sqrt_gamma[i], isi = Ps->inv_sqrt_gamma[i];
                // A[i][c] = (1/2)[sqrt(g_i) Mqq[i][c] / sqrt(g_c) + Mpp[i][c] sqrt(g_c) / sqrt(g_i)]
                //         + (i/2)[-sqrt(g_i) Mqp[i][c] sqrt(g_c) + Mpq[i][c] / (sqrt(g_i) sqrt(g_c))]
                are[i] = 0.5 * (si * dqQ[i] * isgc + dpP[i] * sgc * isi);
                aim[i] = 0.5 * (-si * dqP[i] * sgc + dpQ[i] * isi * isgc);
            }
            if constexpr (STASH) {
#pragma unroll
                for (int i = 0; i < F; ++i) {
                    stash_all[grp][0][i][c] = dpP[i];
                    stash_all[grp][1][i][c] = dpQ[i];
                }
            }
            lu_det_complex<F>(are, aim, c, L.pivA, L.keys, dAr, dAi);
        }

        // stability monitor |det(M)^2 - 1| on checked steps
        const bool checked = (A.check_every <= 1) || (stp % A.check_every == 0) || (stp == A.n_steps);
        if (checked) {
            double r0[N2], r1[N2];  // rows c and F + c of M^T, entries ordered (p rows, q rows) of M
#pragma unroll
            for (int i = 0; i < F; ++i) {
                r0[i] = STASH ? stash_all[STASH ? grp : 0][0][i][c] : dpP[i];
                r0[F + i] = dqP[i];
                r1[i] = STASH ? stash_all[STASH ? grp : 0][1][i][c] : dpQ[i];
                r1[F + i] = dqQ[i];
            }
            const double dM = lu_det_real2<N2, F>(r0, r1, c, L.pivM, L.keys);
            const double dev = fabs(dM * dM - 1.0);
            if (c == 0) {
                L.detM = dM;
                if (!(dev <= L.maxdev)) L.maxdev = dev;
            }
            if (!(dev <= Ps->det_tol)) good = false;
        }
        if constexpr (STASH) {
#pragma unroll
            for (int i = 0; i < F; ++i) {
                dpP[i] = stash_all[grp][0][i][c];
                dpQ[i] = stash_all[grp][1][i][c];
            }
            lds_order();
        }

        // continuous branch: theta accumulates the principal argument of
        // det(A_t) conj(det(A_{t-dt})) e^{i dt sum gamma}, which equals the step of
        // arg(det(A) e^{i t sum gamma}) wrapped to (-pi, pi]; det(A) is rescaled by
        // a power of two (argument unchanged) so the products cannot overflow.
        // Lane 0 puts the step's inputs of the amplitude into the group's ring
        // (each lane adds its mode's terms of the overlap);
        // every RB steps (and at the last step of the launch) RB lanes finish
        // one time sample each: the argument, the branch as the running sum of
        // the arguments in time order, phi, the status, exp and sincos.
        constexpr int RB = GroupCore<F, MULTI>::RB;
        const int slot = stp % RB;
        if (c == 0) {
            int ex;
            (void)frexp(fmax(fabs(dAr), fabs(dAi)), &ex);
            dAr = ldexp(dAr, -ex);
            dAi = ldexp(dAi, -ex);
            const double pr_ = L.prev_r, pi_ = L.prev_i;
            const double ur = dAr * pr_ + dAi * pi_;
            const double ui = dAi * pr_ - dAr * pi_;
            L.rzr[slot] = ur * Ps->cos_gdt - ui * Ps->sin_gdt;
            L.rzi[slot] = ur * Ps->sin_gdt + ui * Ps->cos_gdt;
            L.prev_r = dAr;
            L.prev_i = dAi;
            if constexpr (OVL) {
                L.rflag[slot] = good ? 1 : 0;  // the finite-action test is on the sum
            } else if constexpr (MULTI) {
                L.rflag[slot] = (good && isfinite(S.value())) ? 1 : 0;
                L.rS[slot][0] = S.value();
            } else {
                L.rflag[slot] = (good && isfinite(S.value())) ? 1 : 0;
                double ph;
                L.rex[slot][0] = overlap(Ps, ph);
                L.rph[slot][0] = ph + S.value();
            }
        }
        if constexpr (MULTI) {  // mode c's coordinates
            L.rex[slot][c] = (double)qc;
            L.rph[slot][c] = (double)pc;
        } else if constexpr (OVL) {  // mode c's terms of <chi|p,q>
            const double dqe = Ps->q_eq[c] - (double)qc;
            const double dpe = Ps->p_eq[c] - (double)pc;
            L.rex[slot][c] = -0.25 * Ps->gamma[c] * dqe * dqe - dpe * dpe * Ps->inv4gamma[c];
            L.rph[slot][c] = 0.5 * dqe * (Ps->p_eq[c] + (double)pc);
        }
        if constexpr (OVL) L.rS[slot][c] = S.value();  // mode c's part of the action
        if (slot == RB - 1 || stp == A.step_end) {
            const int first = max(stp - slot, A.step_begin + 1);  // first time sample in the ring
            const int cnt = stp - first + 1;
            const int sl = (first + c) % RB;                       // this lane's sample, if c < cnt
            lds_order();
            if (c < cnt) L.rinc[sl] = datan2(L.rzi[sl], L.rzr[sl], &Ps->mc);
            lds_order();
            if (c < cnt) {
                double th = L.rtheta;
#pragma unroll
                for (int u = 0; u < RB; ++u)
                    if (u <= c) th += L.rinc[(first + u) % RB];
                const int ts = first + c;
                const double ph_ = 0.5 * (th - Ps->sum_gamma * ((double)ts * Ps->dt));
                // the flag holds the sticky status at that step; a non-finite
                // branch stays non-finite for every later sample
                bool g = L.rflag[sl] != 0 && isfinite(ph_);
                if constexpr (MULTI) {
                    double St = 0.0;
#pragma unroll
                    for (int i = 0; i < GroupCore<F, MULTI>::ST; ++i) St += L.rS[sl][i];
                    g = g && isfinite(St);
                    double qs[F], ps[F];
#pragma unroll
                    for (int i = 0; i < F; ++i) {
                        qs[i] = L.rex[sl][i];
                        ps[i] = L.rph[sl][i];
                    }
                    for (int m = 0; m < NR; ++m) {
                        double ph;
                        const double ex = overlap_ref(Ps, m, qs, ps, ph);
                        if (live) put_amplitude(Ps, ts, ex, ph + St + ph_, g, m);
                    }
                } else {
                    double ex = 0.0, ph = 0.0;
#pragma unroll
                    for (int i = 0; i < GroupCore<F, MULTI>::OT; ++i) {
                        ex += L.rex[sl][i];
                        ph += L.rph[sl][i];
                    }
                    if constexpr (OVL) {
                        double St = 0.0;
#pragma unroll
                        for (int i = 0; i < F; ++i) St += L.rS[sl][i];
                        g = g && isfinite(St);  // the parts are running sums: once non-finite, always
                        ph = ph + St;
                    }
                    if (live) put_amplitude(Ps, ts, ex, ph + ph_, g);
                }
                if (c == cnt - 1) {
                    L.rtheta = th;
                    L.rphi = ph_;
                    L.rgood = g ? 1 : 0;
                }
            }
            lds_order();

            good = L.rgood != 0;
            lds_order();
        }
    }

    if constexpr (OVL) {  // each lane's part for a continuation, the whole action into lane 0
        if (live) A.spart[c * NP + jr] = S.pack();
        lds_order();
        L.rS[0][c] = S.value();
        lds_order();
        if (c == 0) {
            double St = 0.0;
#pragma unroll
            for (int i = 0; i < F; ++i) St += L.rS[0][i];
            S.set_total(St);
        }
        lds_order();
    }

    // ---- save the state for a later continuation and for inspection ----
    if (live) {
        A.p[c * NP + jr] = (double)pc;
        A.q[c * NP + jr] = (double)qc;
        if (c == 0) {
            A.scal[SC_S * NP + jr] = S.hi();
            A.scal[SC_SCOMP * NP + jr] = S.lo();
            A.scal[SC_THETA * NP + jr] = L.rtheta;
            A.scal[SC_PREV_RE * NP + jr] = L.prev_r;
            A.scal[SC_PREV_IM * NP + jr] = L.prev_i;
            A.scal[SC_PHI * NP + jr] = L.rphi;
            A.scal[SC_GOOD * NP + jr] = good ? 1.0 : 0.0;
            A.scal[SC_DETM * NP + jr] = L.detM;
            A.scal[SC_MAXDEV * NP + jr] = L.maxdev;
            A.scal[SC_ESCALE * NP + jr] = (double)escale;
        }
#pragma unroll
        for (int i = 0; i < F; ++i) {
            A.Mst[(int64_t)(i * N2 + c) * NP + jr] = dpP[i];
            A.Mst[(int64_t)((F + i) * N2 + c) * NP + jr] = dqP[i];
            A.Mst[(int64_t)(i * N2 + F + c) * NP + jr] = dpQ[i];
            A.Mst[(int64_t)((F + i) * N2 + F + c) * NP + jr] = dqQ[i];
        }
    }
}

template <int F, bool MIXED>
hipError_t launch_F(const TrajArgs &a, hipStream_t s)
{
    constexpr int TPW = 64 / F;
    const int64_t blocks = (a.n + TPW - 1) / TPW;
    if (blocks <= 0) return hipSuccess;
    if constexpr (!MIXED) {
        if (a.n_refs > 1) {
            hipLaunchKernelGGL((traj_kernel<F, false, true>), dim3((unsigned)blocks), dim3(64), 0, s, a, a.prob);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((traj_kernel<F, MIXED, false>), dim3((unsigned)blocks), dim3(64), 0, s, a, a.prob);
    return hipGetLastError();
}

template <bool MIXED>
hipError_t launch_any(int F, const TrajArgs &a, hipStream_t s)
{
    switch (F) {
    case 1: return launch_F<1, MIXED>(a, s);
    case 2: return launch_F<2, MIXED>(a, s);
    case 3: return launch_F<3, MIXED>(a, s);
    case 4: return launch_F<4, MIXED>(a, s);
    case 5: return launch_F<5, MIXED>(a, s);
    case 6: return launch_F<6, MIXED>(a, s);
    case 7: return launch_F<7, MIXED>(a, s);
    case 8: return launch_F<8, MIXED>(a, s);
    case 9: return launch_F<9, MIXED>(a, s);
    case 10: return launch_F<10, MIXED>(a, s);
    case 11: return launch_F<11, MIXED>(a, s);
    case 12: return launch_F<12, MIXED>(a, s);
    case 13: return launch_F<13, MIXED>(a, s);
    case 14: return launch_F<14, MIXED>(a, s);
    case 15: return launch_F<15, MIXED>(a, s);
    case 16: return launch_F<16, MIXED>(a, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_traj(int F, bool mixed, const TrajArgs &a, hipStream_t s)
{
    if (F > 16) return launch_traj_big(F, mixed, a, s);
    return mixed ? launch_any<true>(F, a, s) : launch_any<false>(F, a, s);
}

}  // namespace scivr
