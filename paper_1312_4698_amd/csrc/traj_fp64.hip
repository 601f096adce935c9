// FP64 trajectory kernel of the TA-SC-IVR spectrum for gfx950.
//
// One trajectory is owned by a group of G = 2F lanes of a wave64 (64/G
// trajectories per wave).  During propagation lane c holds column c of the
// 2F x 2F monodromy matrix M = d(p_t, q_t)/d(p_0, q_0), i.e. the tangent
// vector (dp, dq) of one initial direction; every lane also holds the
// trajectory's p and q, and lane c evaluates the potential terms of mode
// c mod F.  After each step M is transposed through LDS so that lane r holds
// row r, and det(M) (stability monitor after Eq. (5)) and det(A) (the
// Herman-Kluk prefactor matrix of Eq. (5)) are taken by Gaussian elimination
// with partial pivoting across the lanes of the group: the pivot is chosen by
// an LDS max over packed (|a|, position) keys and broadcast through LDS.
//
// The fourth-order symplectic step is the drift-kick-drift triple jump
// (Yoshida / Forest-Ruth); each kick evaluates the gradient and the Hessian
// of V = sum_i [k_i q_i^2/2 + D_i (1 - e^{-a_i q_i})^2] + sum_{i<j} l_ij q_i^2 q_j^2
// and applies the Hessian to the tangent column in factored form,
//   H dq = h o dq + 4 q o (Lambda (q o dq)),  h_i = d^2V/dq_i^2,
// with Lambda the symmetric zero-diagonal coupling matrix (kept in scalar
// registers).  The action follows the discrete Lagrangian of the stages
// (+h |p|^2/2 per drift, -h V per kick).  The prefactor phase is kept on a
// continuous branch by unwrapping arg(det(A) e^{i t sum gamma}) step by step,
// phi = (theta - t sum gamma)/2 (separable approximation after Eq. (9)).
// Each step writes the amplitude <chi|p_t,q_t> e^{i (S_t + phi_t)} (zero once
// the trajectory is flagged) into a time-major [t][trajectory] matrix, the
// left operand of the Fourier GEMM.
#include <math.h>

#include "scivr_internal.h"

namespace scivr {
namespace {

template <int F>
struct alignas(16) GroupLds {
    static constexpr int N2 = 2 * F;
    static constexpr int RS = N2 + 2;  // row stride of the transposed matrix (keeps 16-byte rows)
    double M[N2 * RS];                 // transposed monodromy matrix, row r at r * RS
    double pivM[N2];                   // pivot row of the real elimination
    double pivA[N2];                   // pivot row of the complex elimination (re, im interleaved)
    double pg[F + (F & 1)], ph[F + (F & 1)], pv[F + (F & 1)];
    unsigned long long slotM[N2];      // per-step argmax keys of the two eliminations
    unsigned long long slotA[F + (F & 1)];
};

__device__ inline unsigned long long dbits(double x) { return (unsigned long long)__double_as_longlong(x); }

// Workgroups are one wave, and a wave's LDS instructions execute in issue
// order, so a write by one lane is visible to a later read by another lane of
// the same wave without waiting; only the compiler must keep the order.
__device__ inline void lds_order()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

typedef const __attribute__((address_space(4))) ProblemDev *ConstProblem;

// A fresh, opaque handle to the trajectory-independent constants.  Calling it
// at the top of every step keeps their ~100 uniform doubles as scalar-cache
// loads inside the loop instead of letting them be hoisted into (and spilled
// out of) the scalar register file.
__device__ inline ConstProblem opaque(const ProblemDev *P)
{
    uint64_t v = (uint64_t)P;
    asm volatile("" : "+s"(v));
    return (ConstProblem)v;
}

// Gaussian elimination with partial pivoting across the lanes of a group.
// Lane-local a[] is the row at position `pos` (lanes with alive == false hold
// no row).  Each step takes the column maximum with one LDS atomic max over
// packed (|a_k|, 63 - pos) keys (ties go to the lowest position, as in a
// row-swapping LU); only the winning lane then publishes its row into the
// pivot buffer, which the group reads back as a broadcast.  The row at
// position k and the pivot swap positions; the sign of the determinant flips
// when they differ.  Apart from the pivot's store, everything is branch-free.
template <int N>
__device__ inline double lu_det_real(double (&a)[N], int pos, bool alive, double *piv, unsigned long long *slot)
{
    if (alive) slot[pos] = 0ull;
    double det = 1.0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        lds_order();
        if (alive) atomicMax(&slot[k], (dbits(fabs(a[k])) & ~63ull) | (unsigned long long)(63 - pos));
        lds_order();
        const unsigned long long win = __hip_atomic_load(&slot[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        const int ppos = 63 - (int)(win & 63ull);
        const bool isp = alive && pos == ppos;
        if (isp) {
#pragma unroll
            for (int jj = k; jj < N; ++jj) piv[jj] = a[jj];
        }
        lds_order();
        const double pk = piv[k];
        det *= (ppos != k) ? -pk : pk;
        pos = (alive && pos == k) ? ppos : pos;
        alive = alive && !isp;
        if (alive) {  // rows already eliminated (and the pivot) skip the broadcast read
            const double l = a[k] * rcp_nr(pk);
#pragma unroll
            for (int jj = k + 1; jj < N; ++jj) a[jj] = fma(-l, piv[jj], a[jj]);
        }
    }
    lds_order();
    return det;
}

// Complex version: rows (ar, ai); pivot on |a_k|^2; the pivot row is stored
// interleaved (re, im).
template <int N>
__device__ inline void lu_det_complex(double (&ar)[N], double (&ai)[N], int pos, bool alive, double *piv,
                                      unsigned long long *slot, double &dr, double &di)
{
    if (alive) slot[pos] = 0ull;
    double zr = 1.0, zi = 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const double m2 = fma(ar[k], ar[k], ai[k] * ai[k]);
        lds_order();
        if (alive) atomicMax(&slot[k], (dbits(m2) & ~63ull) | (unsigned long long)(63 - pos));
        lds_order();
        const unsigned long long win = __hip_atomic_load(&slot[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        const int ppos = 63 - (int)(win & 63ull);
        const bool isp = alive && pos == ppos;
        if (isp) {
#pragma unroll
            for (int jj = k; jj < N; ++jj) {
                piv[2 * jj] = ar[jj];
                piv[2 * jj + 1] = ai[jj];
            }
        }
        lds_order();
        const double pr = piv[2 * k], pi = piv[2 * k + 1];
        const double nr = zr * pr - zi * pi;
        const double ni = zr * pi + zi * pr;
        zr = (ppos != k) ? -nr : nr;
        zi = (ppos != k) ? -ni : ni;
        pos = (alive && pos == k) ? ppos : pos;
        alive = alive && !isp;
        if (alive) {
            const double inv = rcp_nr(fma(pr, pr, pi * pi));
            const double lr = (ar[k] * pr + ai[k] * pi) * inv;
            const double li = (ai[k] * pr - ar[k] * pi) * inv;
#pragma unroll
            for (int jj = k + 1; jj < N; ++jj) {
                const double br = piv[2 * jj], bi = piv[2 * jj + 1];
                ar[jj] = ar[jj] - (lr * br - li * bi);
                ai[jj] = ai[jj] - (lr * bi + li * br);
            }
        }
    }
    lds_order();
    dr = zr;
    di = zi;
}

// Waves per SIMD the register allocator must allow (unified 512-register file):
// small F keeps several waves resident to hide LDS and transcendental latency.
template <int F>
constexpr int traj_waves() { return F <= 2 ? 4 : (F <= 6 ? 3 : (F <= 12 ? 2 : 1)); }

template <int F>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(traj_waves<F>(), 8))) traj_fp64_kernel(TrajArgs A, const ProblemDev *__restrict__ P0)
{
    constexpr int G = 2 * F;
    constexpr int TPW = 64 / G;
    constexpr int RS = GroupLds<F>::RS;
    __shared__ GroupLds<F> lds_all[TPW];

    const int lane = threadIdx.x;
    const int grp = lane / G;
    // Lanes beyond the last full group own no trajectory.  They leave at once;
    // nothing below synchronises the workgroup, so the rest of the wave runs on
    // with them masked off.
    if (grp >= TPW) return;
    const int c = lane - grp * G;
    const int m = (c < F) ? c : c - F;
    GroupLds<F> &L = lds_all[grp];
    const int64_t j = (int64_t)blockIdx.x * TPW + grp;
    const bool live = j < A.n;
    const int64_t jr = live ? j : 0;
    const int64_t NP = A.npad;

    const ProblemDev *__restrict__ P = P0;
    // constants of the lane's own mode m
    const double km = P->k[m], Dm = P->D[m], am = P->a[m];
    const double sgc = P->sqrt_gamma[m], isgc = P->inv_sqrt_gamma[m];
    double lamrow[F];
#pragma unroll
    for (int i = 0; i < F; ++i) lamrow[i] = P->lam[m * FMAX + i];

    double p[F], q[F], dp[F], dq[F];
    double pm, qm, S, theta, prev_r, prev_i, phi, detM, maxdev;
    bool good;
    if (A.step_begin == 0) {
#pragma unroll
        for (int i = 0; i < F; ++i) {
            p[i] = A.p0[i * NP + jr];
            q[i] = A.q0[i * NP + jr];
            dp[i] = (i == c) ? 1.0 : 0.0;
            dq[i] = (F + i == c) ? 1.0 : 0.0;
        }
        pm = A.p0[m * NP + jr];
        qm = A.q0[m * NP + jr];
        S = theta = phi = prev_i = 0.0;
        prev_r = 1.0;  // det(A) = 1 at t = 0
        detM = 1.0;
        maxdev = 0.0;
        good = true;
    } else {
#pragma unroll
        for (int i = 0; i < F; ++i) {
            p[i] = A.p[i * NP + jr];
            q[i] = A.q[i * NP + jr];
            dp[i] = A.Mst[(int64_t)(i * G + c) * NP + jr];
            dq[i] = A.Mst[(int64_t)((F + i) * G + c) * NP + jr];
        }
        pm = A.p[m * NP + jr];
        qm = A.q[m * NP + jr];
        S = A.scal[SC_S * NP + jr];
        theta = A.scal[SC_THETA * NP + jr];
        prev_r = A.scal[SC_PREV_RE * NP + jr];
        prev_i = A.scal[SC_PREV_IM * NP + jr];
        phi = A.scal[SC_PHI * NP + jr];
        good = A.scal[SC_GOOD * NP + jr] != 0.0;
        detM = A.scal[SC_DETM * NP + jr];
        maxdev = A.scal[SC_MAXDEV * NP + jr];
    }

    // amplitude <chi|p,q> e^{i(S + phi)} of the current state (zero when bad)
    auto amplitude = [&](auto PP) -> double2 {
        double ex = 0.0, ph = 0.0;
#pragma unroll
        for (int i = 0; i < F; ++i) {
            const double dqe = PP->q_eq[i] - q[i];
            const double dpe = PP->p_eq[i] - p[i];
            ex += -0.25 * PP->gamma[i] * dqe * dqe - dpe * dpe * PP->inv4gamma[i];
            ph += 0.5 * dqe * (PP->p_eq[i] + p[i]);
        }
        double s, co;
        dsincos(ph + S + phi, &PP->mc, &s, &co);
        const double mag = dexp(ex, &PP->mc);
        double2 r;
        r.x = good ? mag * co : 0.0;
        r.y = good ? mag * s : 0.0;
        return r;
    };

    if (A.step_begin == 0 && live && c == 0) A.amp[jr] = amplitude(P);

    for (int step = A.step_begin; step < A.step_end; ++step) {
        ConstProblem P = opaque(P0);
#pragma unroll 1
        for (int s = 0; s < 4; ++s) {
            // ---- drift ----
            const double h = P->hd[s];
            double kin = 0.0;
#pragma unroll
            for (int i = 0; i < F; ++i) kin += 0.5 * p[i] * p[i];
#pragma unroll
            for (int i = 0; i < F; ++i) {
                q[i] = fma(h, p[i], q[i]);
                dq[i] = fma(h, dp[i], dq[i]);
            }
            qm = fma(h, pm, qm);
            S = fma(h, kin, S);
            if (s == 3) break;
            // ---- kick ----
            ConstProblem Pk = opaque(P0);
            const double hk = Pk->hc[s];
            double q2[F];
#pragma unroll
            for (int i = 0; i < F; ++i) q2[i] = q[i] * q[i];
            double sm = 0.0;
#pragma unroll
            for (int i = 0; i < F; ++i) sm = fma(lamrow[i], q2[i], sm);
            const double e = dexp(-am * qm, &Pk->mc);
            const double one_e = 1.0 - e;
            const double gm = km * qm + 2.0 * Dm * am * e * one_e + 2.0 * qm * sm;
            const double hm = km + 2.0 * Dm * am * am * e * (2.0 * e - 1.0) + 2.0 * sm;
            const double vm = 0.5 * km * qm * qm + Dm * one_e * one_e + 0.5 * qm * qm * sm;
            if (c < F) {
                L.pg[c] = gm;
                L.ph[c] = hm;
                L.pv[c] = vm;
            }
            lds_order();
            double V = 0.0;
#pragma unroll
            for (int i = 0; i < F; ++i) {
                p[i] = fma(-hk, L.pg[i], p[i]);
                V += L.pv[i];
            }
            pm = fma(-hk, gm, pm);
            S = fma(-hk, V, S);
            // tangent kick: dp -= hk (h o dq + 4 q o Lambda (q o dq))
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
                    const double l = P->lam[i * FMAX + jj];
                    w[i] = fma(l, u[jj], w[i]);
                    w[jj] = fma(l, u[i], w[jj]);
                }
#pragma unroll
            for (int i = 0; i < F; ++i) dp[i] = fma(-hk, fma(L.ph[i], dq[i], 4.0 * q[i] * w[i]), dp[i]);
            lds_order();
        }

        const int stp = step + 1;
        const double t = (double)stp * P->dt;

        // ---- transpose M through LDS: column c -> rows ----
#pragma unroll
        for (int i = 0; i < F; ++i) {
            L.M[i * RS + c] = dp[i];
            L.M[(F + i) * RS + c] = dq[i];
        }
        lds_order();

        // prefactor matrix row c: A[c][jj] from M rows c and F+c, then det(A);
        // only lanes c < F take part (they alone carry the phase, lane 0 writes
        // the amplitude), the upper half of the group is masked off meanwhile
        double dAr = 0.0, dAi = 0.0;
        if (c < F) {
            double are[F], aim[F];
#pragma unroll
            for (int jj = 0; jj < F; ++jj) {
                const double mpp = L.M[c * RS + jj], mpq = L.M[c * RS + F + jj];
                const double mqp = L.M[(F + c) * RS + jj], mqq = L.M[(F + c) * RS + F + jj];
                const double sj = P->sqrt_gamma[jj], isj = P->inv_sqrt_gamma[jj];
                are[jj] = 0.5 * (sgc * mqq * isj + mpp * sj * isgc);
                aim[jj] = 0.5 * (-sgc * mqp * sj + mpq * isgc * isj);
            }
            lu_det_complex<F>(are, aim, c, true, L.pivA, L.slotA, dAr, dAi);
        }

        // stability monitor |det(M)^2 - 1| on checked steps
        const bool checked = (A.check_every <= 1) || (stp % A.check_every == 0) || (stp == A.n_steps);
        if (checked) {
            double row[G];
#pragma unroll
            for (int jj = 0; jj < G; ++jj) row[jj] = L.M[c * RS + jj];
            const double dM = lu_det_real<G>(row, c, true, L.pivM, L.slotM);
            const double dev = fabs(dM * dM - 1.0);
            detM = dM;
            if (!(dev <= maxdev)) maxdev = dev;
            if (!(dev <= P->det_tol)) good = false;
        }

        // continuous branch: theta accumulates the principal argument of
        // det(A_t) conj(det(A_{t-dt})) e^{i dt sum gamma}, which equals the step of
        // arg(det(A) e^{i t sum gamma}) wrapped to (-pi, pi]; det(A) is rescaled by
        // a power of two (argument unchanged) so the products cannot overflow.
        if (c < F) {
            int ex;
            (void)frexp(fmax(fabs(dAr), fabs(dAi)), &ex);
            dAr = ldexp(dAr, -ex);
            dAi = ldexp(dAi, -ex);
            const double ur = dAr * prev_r + dAi * prev_i;
            const double ui = dAi * prev_r - dAr * prev_i;
            const double zr = ur * P->cos_gdt - ui * P->sin_gdt;
            const double zi = ur * P->sin_gdt + ui * P->cos_gdt;
            theta += datan2(zi, zr, &P->mc);
            prev_r = dAr;
            prev_i = dAi;
            phi = 0.5 * (theta - P->sum_gamma * t);
        }
        if (!isfinite(phi) || !isfinite(S)) good = false;

        if (live && c == 0) A.amp[(int64_t)stp * NP + jr] = amplitude(P);
    }

    // ---- save the state for a later continuation and for inspection ----
    if (live) {
        if (c == 0) {
#pragma unroll
            for (int i = 0; i < F; ++i) {
                A.p[i * NP + jr] = p[i];
                A.q[i * NP + jr] = q[i];
            }
            A.scal[SC_S * NP + jr] = S;
            A.scal[SC_THETA * NP + jr] = theta;
            A.scal[SC_PREV_RE * NP + jr] = prev_r;
            A.scal[SC_PREV_IM * NP + jr] = prev_i;
            A.scal[SC_PHI * NP + jr] = phi;
            A.scal[SC_GOOD * NP + jr] = good ? 1.0 : 0.0;
            A.scal[SC_DETM * NP + jr] = detM;
            A.scal[SC_MAXDEV * NP + jr] = maxdev;
        }
#pragma unroll
        for (int i = 0; i < F; ++i) {
            A.Mst[(int64_t)(i * G + c) * NP + jr] = dp[i];
            A.Mst[(int64_t)((F + i) * G + c) * NP + jr] = dq[i];
        }
    }
}

template <int F>
hipError_t launch_F(const TrajArgs &a, hipStream_t s)
{
    constexpr int TPW = 64 / (2 * F);
    const int64_t blocks = (a.n + TPW - 1) / TPW;
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(traj_fp64_kernel<F>, dim3((unsigned)blocks), dim3(64), 0, s, a, a.prob);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_traj_fp64(int F, const TrajArgs &a, hipStream_t s)
{
    switch (F) {
    case 1: return launch_F<1>(a, s);
    case 2: return launch_F<2>(a, s);
    case 3: return launch_F<3>(a, s);
    case 4: return launch_F<4>(a, s);
    case 5: return launch_F<5>(a, s);
    case 6: return launch_F<6>(a, s);
    case 7: return launch_F<7>(a, s);
    case 8: return launch_F<8>(a, s);
    case 9: return launch_F<9>(a, s);
    case 10: return launch_F<10>(a, s);
    case 11: return launch_F<11>(a, s);
    case 12: return launch_F<12>(a, s);
    case 13: return launch_F<13>(a, s);
    case 14: return launch_F<14>(a, s);
    case 15: return launch_F<15>(a, s);
    case 16: return launch_F<16>(a, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace scivr
