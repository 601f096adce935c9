// Trajectory kernel of the TA-SC-IVR spectrum for large F (17 <= F <= 32):
// one wave64 per trajectory.
//
// Lane c < 2F owns column c of the 2F x 2F monodromy matrix M = d(p_t, q_t) /
// d(p_0, q_0) (the tangent vector of initial direction c, its p half dp[] and
// q half dq[]); lane i < F also owns mode i of the trajectory (p_i, q_i and the
// Morse terms of that mode), shared with the wave through LDS.  Per step:
//  * the fourth-order symplectic triple jump (Yoshida / Forest-Ruth drifts
//    and kicks), each kick applying the Hessian to all tangent columns in
//    factored form H dq = h o dq + 4 q o (Lambda (q o dq)); the product of the
//    coupling matrix Lambda with the 2F columns q o dq is one 32 x 32 by
//    32 x 64 FP64 matrix-core product per kick (the batched monodromy product),
//    staged through LDS between the column-per-lane and the MFMA layouts;
//  * det(A) of the Herman-Kluk prefactor matrix of Eq. (5) and det(M) (the
//    stability monitor after Eq. (5)) are taken as the determinants of the
//    transposes: lane c < 2F's own column is row c of M^T; row i of A^T
//    (column i of A) has its real parts in lane i and its imaginary parts in
//    lane 32 + i, both formed from columns i and F + i of an LDS copy of M
//    (written column by column; each lane also reloads its column from it
//    afterwards, so the register copy is dead while the eliminations run).
//    Gaussian elimination with partial pivoting runs across the lanes, one
//    row (or one part of a complex row) per lane: a wave-wide DPP maximum
//    over packed (|a|, position) keys picks each pivot (the trajectory is the
//    whole wave, so the pivot is wave-uniform) and the pivot row reaches
//    every lane through readlane into scalar registers, with no LDS round
//    trip in the elimination;
//  * the action, the overlap terms and the continuous prefactor phase are
//    summed across the mode lanes; lane 0 writes the amplitude of the time
//    sample.
// The state layout, the branch tracking and the amplitude storage (FP64
// time-major, or FP16 hi/lo planes in the mixed form) are the small-F
// kernel's.
#include <math.h>

#include <type_traits>

#include "scivr_internal.h"
#include "traj_common.h"

namespace scivr {
namespace {

template <int F>
struct alignas(16) BigLds {
    static constexpr int N2 = 2 * F;
    static constexpr int RS = N2 + 1;  // odd row stride of the copy of M
    static constexpr bool SM_MFMA = N2 < 64;  // a spare product column for sum_k Lambda_ik q_k^2
    static constexpr int RB = 8;              // time samples per amplitude ring
    union {
        double T[N2 * RS];  // M, row r at T + r RS (after the step)
        double U[32];       // the kicks' mode terms sum_k Lambda_ik q_k^2, row i at U + i
    };
    // coupling matrix, row-major, zero diagonal (read only where the product
    // has no spare column for the mode terms)
    double lam[SM_MFMA ? 1 : F * F];
    // amplitude ring: per time sample, the raw det(A), the action, the
    // monitor's flag and every reference state's overlap exponent and phase;
    // ra holds the branch increments while a ring is finished
    double rdr[RB], rdi[RB], rS[RB], ra[RB];
    double rex[RB][MAX_REFS], rph[RB][MAX_REFS];
    int rgood[RB];
};

typedef double d4 __attribute__((ext_vector_type(4)));

// lane 0's value in every lane (both 32-bit halves through scalar registers)
__device__ __attribute__((always_inline)) inline double from_lane0(double v)
{
    const unsigned long long u = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)u);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(u >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// det(A) rescaled by a power of two (the branch only needs its argument)
__device__ __attribute__((always_inline)) inline void rescale_det(double &dr, double &di)
{
    int ex;
    (void)frexp(fmax(fabs(dr), fabs(di)), &ex);
    dr = ldexp(dr, -ex);
    di = ldexp(di, -ex);
}

// Largest 32-bit key over the wave (every lane gets it).  DPP row shifts
// 1, 2, 4, 8 leave each row's maximum in its lane 15, row broadcasts 15 and 31
// carry it to lane 63; lanes without a source take the identity 0.
__device__ __attribute__((always_inline)) inline unsigned wave_max_u32(unsigned v)
{
#define SCIVR_DPP_MAX(ctrl, rmask) \
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, ctrl, rmask, 0xf, false));
    SCIVR_DPP_MAX(0x111, 0xf)  // row_shr:1
    SCIVR_DPP_MAX(0x112, 0xf)  // row_shr:2
    SCIVR_DPP_MAX(0x114, 0xf)  // row_shr:4
    SCIVR_DPP_MAX(0x118, 0xf)  // row_shr:8
    SCIVR_DPP_MAX(0x142, 0xa)  // row_bcast:15 into rows 1 and 3
    SCIVR_DPP_MAX(0x143, 0xc)  // row_bcast:31 into rows 2 and 3
#undef SCIVR_DPP_MAX
    return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

// The value of v in lane l (l uniform across the wave), into scalar registers.
__device__ __attribute__((always_inline)) inline double readlane_f64(double v, int l)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// v from the lane selected by the DPP control CTRL (rows in ROW_MASK), 0 where
// there is no source lane.
template <int CTRL, int ROW_MASK>
__device__ __attribute__((always_inline)) inline float dpp_src(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, false));
}
template <int CTRL, int ROW_MASK>
__device__ __attribute__((always_inline)) inline double dpp_src(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xf, false);
    return __hiloint2double(hi, lo);
}

// Sum of v over lanes 0..31, returned to every lane: prefix sums within each
// row of 16 lanes (row shifts 1, 2, 4, 8), then row 0's total added into
// row 1 (row broadcast 15), read from lane 31.
template <typename T>
__device__ __attribute__((always_inline)) inline T wave_sum32(T v)
{
    v += dpp_src<0x111, 0xf>(v);
    v += dpp_src<0x112, 0xf>(v);
    v += dpp_src<0x114, 0xf>(v);
    v += dpp_src<0x118, 0xf>(v);
    v += dpp_src<0x142, 0xa>(v);
    if constexpr (sizeof(T) == 8)
        return readlane_f64(v, 31);
    else
        return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 31));
}

// det of the real N x N matrix whose row r lives in a[] of lane r (`active`
// on lanes 0..N-1; rows stay in place).  The pivot of each column is the live
// row with the largest |a_k|, compared as 32-bit keys (the magnitude's high
// word with the row's tag 63 - r in its low six bits, so ties go to the lowest
// row) by a wave-wide maximum, which names the pivot lane directly; the pivot
// row is read into scalar registers lane by lane, so the elimination needs no
// LDS.  The determinant is the product of the pivots times the sign of the
// pivot order r_0, r_1, ..., whose inversions are the live rows below each
// r_k (a popcount of the wave-uniform set of rows not yet used).  Every lane
// returns det.
template <int N>
__device__ __attribute__((always_inline)) inline double lu_det_rows(double (&a)[N], bool active)
{
    const int lane = threadIdx.x;
    bool alive = active;
    unsigned long long live = __ballot(active);
    unsigned inversions = 0;
    double det = 1.0;
    // lookahead: column k + 1 is updated first and its pivot search runs
    // while the rest of the row is eliminated
    unsigned win = wave_max_u32(alive ? pivot_key32(fabs(a[0]), lane) : 0u);
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const int pl = 63 - (int)(win & 63u);
        const double pk = readlane_f64(a[k], pl);
        det *= pk;
        // the product is taken here, in a vector register: left to the
        // scheduler, the 2N pivot halves stay live in scalar registers until
        // the end and push the kernel into scalar spills
        asm volatile("" : "+v"(det));
        inversions += __builtin_popcountll(live & ((1ull << pl) - 1ull));
        live &= ~(1ull << pl);
        alive = alive && lane != pl;
        if (k + 1 < N) {
            // rows out of play (used pivots, lanes beyond N) are updated too:
            // their keys are masked, so their values are never read again
            const double l = a[k] * rcp_nr(pk);
            a[k + 1] = fma(-l, readlane_f64(a[k + 1], pl), a[k + 1]);
            win = wave_max_u32(alive ? pivot_key32(fabs(a[k + 1]), lane) : 0u);
            // the pivot row arrives four entries at a time, so several
            // readlanes are in flight before their scalar registers are used
#pragma unroll
            for (int j0 = k + 2; j0 < N; j0 += 4) {
                double b[4];
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (j0 + u < N) b[u] = readlane_f64(a[j0 + u], pl);
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (j0 + u < N) a[j0 + u] = fma(-l, b[u], a[j0 + u]);
            }
        }
    }
    return (inversions & 1u) ? -det : det;
}

// 4 x 4 transpose between the wave's four row groups of 16 lanes and four
// registers: on return v[c] in row group k holds what v[k] held in row group c
// (same lane within the group).  Per 32-bit half, v_permlane32_swap on (v0, v2)
// and (v1, v3), then v_permlane16_swap on (v0, v1) and (v2, v3) (lane layouts
// checked on the device: permlane32_swap(a, b) gives [a0 a1 b0 b1] and
// [a2 a3 b2 b3] by row group, permlane16_swap(a, b) gives [a0 b0 a2 b2] and
// [a1 b1 a3 b3]).
__device__ __attribute__((always_inline)) inline void group_transpose(double (&v)[4])
{
    int lo[4], hi[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        lo[r] = __double2loint(v[r]);
        hi[r] = __double2hiint(v[r]);
    }
    auto stage = [](int (&w)[4]) {
        auto a = __builtin_amdgcn_permlane32_swap(w[0], w[2], false, false);
        auto b = __builtin_amdgcn_permlane32_swap(w[1], w[3], false, false);
        auto c = __builtin_amdgcn_permlane16_swap(a[0], b[0], false, false);
        auto d = __builtin_amdgcn_permlane16_swap(a[1], b[1], false, false);
        w[0] = c[0];
        w[1] = c[1];
        w[2] = d[0];
        w[3] = d[1];
    };
    stage(lo);
    stage(hi);
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = __hiloint2double(hi[r], lo[r]);
}

// The value of v in lane (lane & 31) and in lane (lane & 31) + 32, to every
// lane: two v_permlane32_swap, one per 32-bit half (each swaps the upper half
// of one copy with the lower half of the other).
__device__ __attribute__((always_inline)) inline void half_pair(double v, double &lower, double &upper)
{
    const auto a = __builtin_amdgcn_permlane32_swap(__double2loint(v), __double2loint(v), false, false);
    const auto b = __builtin_amdgcn_permlane32_swap(__double2hiint(v), __double2hiint(v), false, false);
    lower = __hiloint2double(b[0], a[0]);
    upper = __hiloint2double(b[1], a[1]);
}

// det of the complex N x N matrix (N <= 32) whose row r has its real parts in
// x[] of lane r and its imaginary parts in x[] of lane r + 32 (`active` on
// both lanes of rows 0..N-1; `imag` on the upper half).  Pivot on |a_k|^2
// (keys from the real-part lanes), otherwise as lu_det_rows.  Each lane
// updates one part, so every entry costs the pivot row's four readlanes and
// two FMAs per lane; a whole complex row per lane would take four FMAs and
// leave the upper half of the wave idle.  Every lane returns det.
template <int N>
__device__ __attribute__((always_inline)) inline void lu_det_rows_complex_split(double (&x)[N], bool active, bool imag,
                                                                                double &dr, double &di)
{
    const int row = threadIdx.x & 31;
    bool alive = active;
    unsigned live = (unsigned)__ballot(active && !imag);
    unsigned inversions = 0;
    double zr = 1.0, zi = 0.0;
    double re, im;  // this row's entry in the column being eliminated
    half_pair(x[0], re, im);
    unsigned win = wave_max_u32((alive && !imag) ? pivot_key32(fma(re, re, im * im), row) : 0u);
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const int pl = 63 - (int)(win & 63u);  // the pivot row's real-part lane
        const double pr = readlane_f64(x[k], pl), pi = readlane_f64(x[k], pl + 32);
        const double nr = zr * pr - zi * pi;
        const double ni = zr * pi + zi * pr;
        zr = nr;
        zi = ni;
        asm volatile("" : "+v"(zr), "+v"(zi));  // as in lu_det_rows
        inversions += __builtin_popcount(live & ((1u << pl) - 1u));
        live &= ~(1u << pl);
        alive = alive && row != pl;
        if (k + 1 < N) {
            const double inv = rcp_nr(fma(pr, pr, pi * pi));
            const double lr = (re * pr + im * pi) * inv;  // rows out of play: as in lu_det_rows
            const double li = (im * pr - re * pi) * inv;
            // x -= l b: the real part loses lr br - li bi, the imaginary part
            // lr bi + li br; both as fma(-u, br, fma(v, bi, x)), so every lane
            // takes the broadcast operands in the same order
            const double u = imag ? li : lr, v = imag ? -lr : li;
            {
                const double br = readlane_f64(x[k + 1], pl), bi = readlane_f64(x[k + 1], pl + 32);
                x[k + 1] = fma(-u, br, fma(v, bi, x[k + 1]));
            }
            half_pair(x[k + 1], re, im);
            win = wave_max_u32((alive && !imag) ? pivot_key32(fma(re, re, im * im), row) : 0u);
#pragma unroll
            for (int j0 = k + 2; j0 < N; j0 += 2) {
                double br[2], bi[2];
#pragma unroll
                for (int w = 0; w < 2; ++w)
                    if (j0 + w < N) {
                        br[w] = readlane_f64(x[j0 + w], pl);
                        bi[w] = readlane_f64(x[j0 + w], pl + 32);
                    }
#pragma unroll
                for (int w = 0; w < 2; ++w)
                    if (j0 + w < N) x[j0 + w] = fma(-u, br[w], fma(v, bi[w], x[j0 + w]));
            }
        }
    }
    dr = (inversions & 1u) ? -zr : zr;
    di = (inversions & 1u) ? -zi : zi;
}

template <int F, bool MIXED>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1)))
traj_big_kernel(TrajArgs A, const ProblemDev *__restrict__ P0)
{
    typedef typename std::conditional<MIXED, float, double>::type R;
    constexpr int N2 = 2 * F;
    constexpr int RS = BigLds<F>::RS;
    constexpr int FP = F + (F & 1);
    constexpr bool SM_MFMA = BigLds<F>::SM_MFMA;
    constexpr int RB = BigLds<F>::RB;
    __shared__ BigLds<F> L;
    __shared__ R qv[FP], pm[FP];
    __shared__ double2 qh[F];  // (4 q_i, h_i) of the kick's Hessian diagonal terms

    const int lane = threadIdx.x;
    const ProblemDev *__restrict__ P = P0;
    if constexpr (!SM_MFMA)
        for (int idx = lane; idx < F * F; idx += 64) L.lam[idx] = P->lam[(idx / F) * FMAX + idx % F];
    const int64_t jr = blockIdx.x;  // one trajectory per workgroup, grid = batch size
    const int64_t NP = A.npad;
    const bool colLane = lane < N2;
    const bool modeLane = lane < F;
    const int cm = modeLane ? lane : 0;

    const R kc = (R)P->k[cm], Dc = (R)P->D[cm], ac = (R)P->a[cm];
    // the prefactor matrix's rows: lane rc and lane 32 + rc hold row rc of A^T
    const bool imagLane = lane >= 32;
    const bool rowLane = (lane & 31) < F;
    const int rc = rowLane ? (lane & 31) : 0;
    const double sgr = P->sqrt_gamma[rc], isgr = P->inv_sqrt_gamma[rc];
    const double alphaA = imagLane ? -sgr : isgr, betaA = imagLane ? isgr : sgr;
    const int colU = imagLane ? rc : F + rc, colV = imagLane ? F + rc : rc;
    const int li = lane & 15, kg = lane >> 4;
    // A-operand fragments of Lambda (32 x 32, zero-padded): block (ib, kb) holds
    // Lambda[16 ib + li][4 kb + kg] in this lane
    double lamA[2][8];
#pragma unroll
    for (int ib = 0; ib < 2; ++ib)
#pragma unroll
        for (int kb = 0; kb < 8; ++kb) {
            const int r = 16 * ib + li, cc = 4 * kb + kg;
            lamA[ib][kb] = (r < F && cc < F) ? P->lam[r * FMAX + cc] : 0.0;
        }

    double dp[F], dq[F];  // column `lane` of M: p rows and q rows
    R pc = 0, qc = 0;     // mode `lane` of the trajectory (lanes < F)
    Action<MIXED> S;
    double theta, prev_r, prev_i, phi, detM, maxdev;
    int escale = 0;
    bool good;
    if (A.step_begin == 0) {
#pragma unroll
        for (int i = 0; i < F; ++i) {
            dp[i] = (lane == i) ? 1.0 : 0.0;
            dq[i] = (lane == F + i) ? 1.0 : 0.0;
        }
        if (modeLane) {
            pc = (R)A.p0[lane * NP + jr];
            qc = (R)A.q0[lane * NP + jr];
        }
        theta = phi = prev_i = 0.0;
        prev_r = 1.0;
        detM = 1.0;
        maxdev = 0.0;
        good = true;
    } else {
        const int cc = colLane ? lane : 0;
#pragma unroll
        for (int i = 0; i < F; ++i) {
            dp[i] = colLane ? A.Mst[(int64_t)(i * N2 + cc) * NP + jr] : 0.0;
            dq[i] = colLane ? A.Mst[(int64_t)((F + i) * N2 + cc) * NP + jr] : 0.0;
        }
        if (modeLane) {
            pc = (R)A.p[lane * NP + jr];
            qc = (R)A.q[lane * NP + jr];
        }
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
    if (modeLane) {
        qv[lane] = qc;
        pm[lane] = pc;
    }
    lds_order();

    // exponent and phase of <chi_m|p,q> (reference state m; m = 0 is chi): each
    // mode lane forms its own terms from its (q, p), summed across the wave
    // (every lane calls this)
    const double g4c = 0.25 * P->gamma[cm], i4gc = P->inv4gamma[cm];
    const double rq0 = P->ref_q[0][cm], rp0 = P->ref_p[0][cm];
    auto overlap = [&](auto PP, int m, double &ph) -> double {
        double ex = 0.0, phm = 0.0;
        if (modeLane) {
            const double qi = (double)qc, pi = (double)pc;
            const double rq = m == 0 ? rq0 : PP->ref_q[m][lane], rp = m == 0 ? rp0 : PP->ref_p[m][lane];
            const double dqe = rq - qi, dpe = rp - pi;
            ex = -g4c * dqe * dqe - dpe * dpe * i4gc;
            phm = 0.5 * dqe * (rp + pi);
        }
        ph = wave_sum32(phm);
        return wave_sum32(ex);
    };
    // amplitude of time sample t (lane 0 stores; ex0, ph0 are reference 0's
    // overlap terms, the others are formed here with every lane)
    auto store_amplitude = [&](auto PP, int t, double ex0, double ph0) {
        if constexpr (!MIXED) {
            // each reference state's amplitude, [t][ref][trajectory]
            for (int m = 0; m < A.n_refs; ++m) {
                double ex = ex0, ph = ph0;
                if (m > 0) ex = overlap(PP, m, ph);
                if (lane == 0) {
                    double s, co;
                    dsincos(ph + S.value() + phi, &PP->mc, &s, &co);
                    const double mag = dexp(ex, &PP->mc);
                    double2 r;
                    r.x = good ? mag * co : 0.0;
                    r.y = good ? mag * s : 0.0;
                    A.amp[((int64_t)t * A.n_refs + m) * NP + jr] = r;
                }
            }
        } else if (lane == 0) {
            const double ex = ex0, ph = ph0;
            double s, co;
            dsincos(ph + S.value() + phi, &PP->mc, &s, &co);
            const double mag = ldexp(dexp(ex, &PP->mc), escale);
            const float re = good ? (float)(mag * co) : 0.f, im = good ? (float)(mag * s) : 0.f;
            _Float16 h[4];
            split_f16(re, h[0], h[1]);
            split_f16(im, h[2], h[3]);
            const int64_t e = ((int64_t)(t >> 3) * NP + jr) * 8 + (t & 7);
#pragma unroll
            for (int pl = 0; pl < 4; ++pl) A.amp16[pl * A.plane + e] = h[pl];
        }
    };

    auto store_zero = [&](int t) {
        if constexpr (!MIXED) {
            for (int m = 0; m < A.n_refs; ++m) A.amp[((int64_t)t * A.n_refs + m) * NP + jr] = make_double2(0.0, 0.0);
        } else {
            const int64_t e = ((int64_t)(t >> 3) * NP + jr) * 8 + (t & 7);
#pragma unroll
            for (int pl = 0; pl < 4; ++pl) A.amp16[pl * A.plane + e] = (_Float16)0.0f;
        }
    };

    // Finish the ring's nk time samples t0 .. t0 + nk - 1, lane k < nk taking
    // sample t0 + k: the argument of det(A_t) conj(det(A_{t-dt})) e^{i dt sum
    // gamma} (on det(A) rescaled by a power of two) advances the continuous
    // branch, the increments added in time order as one lane per step would;
    // a non-finite phase or action makes its sample and every later one bad;
    // then the amplitudes of every reference state.
    int nk = 0;
    auto finish_ring = [&](ConstProblem PP, int t0) {
        lds_order();
        const bool fin = lane < nk;
        const int k = fin ? lane : 0;
        if (fin) {
            double dr = L.rdr[k], di = L.rdi[k];
            rescale_det(dr, di);
            double qr = prev_r, qi = prev_i;
            if (k > 0) {
                qr = L.rdr[k - 1];
                qi = L.rdi[k - 1];
                rescale_det(qr, qi);
            }
            const double ur = dr * qr + di * qi;
            const double ui = di * qr - dr * qi;
            const double zr = ur * PP->cos_gdt - ui * PP->sin_gdt;
            const double zi = ur * PP->sin_gdt + ui * PP->cos_gdt;
            L.ra[k] = datan2(zi, zr, &PP->mc);
        }
        lds_order();
        double th = theta, phk = 0.0, Sk = 0.0;
        bool bad = false;
        if (fin) {
            for (int kk = 0; kk <= k; ++kk) th += L.ra[kk];
            phk = 0.5 * (th - PP->sum_gamma * ((double)(t0 + k) * PP->dt));
            Sk = L.rS[k];
            bad = !isfinite(phk) || !isfinite(Sk);
        }
        const unsigned long long badm = __ballot(fin && bad);
        if (fin) {
            const bool g = L.rgood[k] != 0 && (badm & ((2ull << k) - 1ull)) == 0;
            const int t = t0 + k;
            if constexpr (!MIXED) {
                for (int m = 0; m < A.n_refs; ++m) {
                    double sn, co;
                    dsincos(L.rph[k][m] + Sk + phk, &PP->mc, &sn, &co);
                    const double mag = dexp(L.rex[k][m], &PP->mc);
                    double2 r;
                    r.x = g ? mag * co : 0.0;
                    r.y = g ? mag * sn : 0.0;
                    A.amp[((int64_t)t * A.n_refs + m) * NP + jr] = r;
                }
            } else {
                double sn, co;
                dsincos(L.rph[k][0] + Sk + phk, &PP->mc, &sn, &co);
                const double mag = ldexp(dexp(L.rex[k][0], &PP->mc), escale);
                const float re = g ? (float)(mag * co) : 0.f, im = g ? (float)(mag * sn) : 0.f;
                _Float16 h[4];
                split_f16(re, h[0], h[1]);
                split_f16(im, h[2], h[3]);
                const int64_t e = ((int64_t)(t >> 3) * NP + jr) * 8 + (t & 7);
#pragma unroll
                for (int pl = 0; pl < 4; ++pl) A.amp16[pl * A.plane + e] = h[pl];
            }
            for (int kk = k + 1; kk < nk; ++kk) th += L.ra[kk];
        }
        // the branch through the ring's last sample, in every lane
        theta = from_lane0(th);
        prev_r = L.rdr[nk - 1];
        prev_i = L.rdi[nk - 1];
        rescale_det(prev_r, prev_i);
        phi = 0.5 * (theta - PP->sum_gamma * ((double)(t0 + nk - 1) * PP->dt));
        if (badm != 0) good = false;
        lds_order();
        nk = 0;
    };

    if (A.step_begin == 0) {
        double ph0;
        const double ex0 = overlap(P, 0, ph0);
        if constexpr (MIXED) escale = (int)fmin(floor(-ex0 * 1.4426950408889634) + 3.0, 15.0);
        store_amplitude(P, 0, ex0, ph0);
    }

    for (int step = A.step_begin; step < A.step_end; ++step) {
        ConstProblem Ps = opaque(P0);
        // a flagged trajectory contributes nothing: when asked, it stops here
        // (its amplitudes stay zero; lane 0's flag also covers a non-finite
        // phase or action)
        if (A.stop_flagged && !__builtin_amdgcn_readfirstlane((int)good)) {
            if (nk > 0) finish_ring(Ps, step - nk + 1);
            if (lane == 0) store_zero(step + 1);
            continue;
        }
#pragma unroll 1
        for (int s = 0; s < 4; ++s) {
            ConstProblem Pk = opaque(P0);
            // ---- drift ----
            const double h = Pk->hd[s];
            S.add(h * (double)wave_sum32(modeLane ? (R)0.5 * pc * pc : (R)0));
            if (modeLane) qc = fma((R)h, pc, qc);
#pragma unroll
            for (int i = 0; i < F; ++i) dq[i] = fma(h, dp[i], dq[i]);
            lds_order();
            if (modeLane) qv[lane] = qc;
            lds_order();
            if (s == 3) break;
            // ---- kick ----
            const double hk = Pk->hc[s];
            // the product W = Lambda (q o dQ) of the tangent kick on the matrix
            // cores, a 32 x 32 by 32 x 64 FP64 product (v_mfma_f64_16x16x4f64:
            // A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k, D[i][j] in lane
            // j + 16 (i mod 4), register i / 4).  Lane c's own column reaches the
            // B layout, four rows at a time, through a row-group transpose; the
            // result comes back the same way in the tangent kick below.  Column
            // 2F, when there is one, carries q o q, so that row i of its product
            // is the mode term sum_k Lambda_ik q_k^2.
            d4 acc[2][4];
#pragma unroll
            for (int ib = 0; ib < 2; ++ib)
#pragma unroll
                for (int cb = 0; cb < 4; ++cb) acc[ib][cb] = (d4){0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kb = 0; kb < 8; ++kb) {
                double b[4];  // rows 4 kb .. 4 kb + 3 of this lane's column
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = 4 * kb + r;
                    const double qi = (double)qv[i < F ? i : 0];
                    b[r] = (i >= F) ? 0.0 : colLane ? qi * dq[i < F ? i : 0] : (SM_MFMA && lane == N2) ? qi * qi : 0.0;
                }
                group_transpose(b);  // b[cb]: column 16 cb + li, row 4 kb + kg
#pragma unroll
                for (int ib = 0; ib < 2; ++ib)
#pragma unroll
                    for (int cb = 0; cb < 4; ++cb)
                        acc[ib][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(lamA[ib][kb], b[cb], acc[ib][cb], 0, 0, 0);
            }
            if constexpr (SM_MFMA) {
                // column 2F's rows to LDS for the mode lanes: row 16 ib + 4 r + kg
                // sits in lane (2F mod 16) + 16 kg, register r of block 2F / 16
                if (li == (N2 & 15)) {
#pragma unroll
                    for (int ib = 0; ib < 2; ++ib)
#pragma unroll
                        for (int r = 0; r < 4; ++r) L.U[16 * ib + 4 * r + kg] = acc[ib][N2 >> 4][r];
                }
                lds_order();
            }
            // mode terms on lanes < F: gradient, Hessian diagonal and potential
            R vc = 0;
            if (modeLane) {
                R sm;
                if constexpr (SM_MFMA) {
                    sm = (R)L.U[lane];
                } else {
                    sm = 0;
#pragma unroll
                    for (int i = 0; i < F; ++i) {
                        const R qi = qv[i];
                        sm = fma((R)L.lam[lane * F + i], qi * qi, sm);
                    }
                }
                R e;
                if constexpr (MIXED)
                    e = expf(-ac * qc);
                else
                    e = dexp(-ac * qc, &Pk->mc);
                const R one_e = (R)1 - e;
                const R gc = kc * qc + (R)2 * Dc * ac * e * one_e + (R)2 * qc * sm;
                const R hc = kc + (R)2 * Dc * ac * ac * e * ((R)2 * e - (R)1) + (R)2 * sm;
                vc = (R)0.5 * kc * qc * qc + Dc * one_e * one_e + (R)0.5 * qc * qc * sm;
                pc = fma(-(R)hk, gc, pc);
                qh[lane] = make_double2(4.0 * (double)qc, (double)hc);
                pm[lane] = pc;
            }
            S.add(-hk * (double)wave_sum32(vc));
            lds_order();
            // tangent kick of every column: dp -= hk (h o dq + 4 q o W), the rows
            // of W in this lane's column four at a time: after the transpose
            // w[c] is row 16 ib + 4 r + c
#pragma unroll
            for (int ib = 0; ib < 2; ++ib)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (16 * ib + 4 * r >= F) continue;
                    double w[4] = {acc[ib][0][r], acc[ib][1][r], acc[ib][2][r], acc[ib][3][r]};
                    group_transpose(w);
                    if (colLane) {
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            const int i = 16 * ib + 4 * r + c;
                            if (i < F) {
                                const double2 g = qh[i];
                                dp[i] = fma(-hk, fma(g.y, dq[i], g.x * w[c]), dp[i]);
                            }
                        }
                    }
                }
            lds_order();
        }

        const int stp = step + 1;

        // ---- M to LDS, column `lane` ----
        if (colLane) {
#pragma unroll
            for (int i = 0; i < F; ++i) {
                L.T[i * RS + lane] = dp[i];
                L.T[(F + i) * RS + lane] = dq[i];
            }
        }
        lds_order();

        // det(A) = det(A^T) and det(M) = det(M^T).  Row c of A^T (column c of A)
        // has its real parts in lane c and its imaginary parts in lane 32 + c,
        // formed from columns c and F + c of M in LDS:
        //   Re A[i][c] = (1/2)[sqrt(g_i) Mqq[i][c] / sqrt(g_c) + Mpp[i][c] sqrt(g_c) / sqrt(g_i)]
        //   Im A[i][c] = (1/2)[-sqrt(g_i) Mqp[i][c] sqrt(g_c) + Mpq[i][c] / (sqrt(g_i) sqrt(g_c))]
        // i.e. (1/2)(sqrt(g_i) u alpha + v beta / sqrt(g_i)) with (u, v, alpha, beta)
        // = (Mqq, Mpp, 1/sqrt(g_c), sqrt(g_c)) or (Mqp, Mpq, -sqrt(g_c), 1/sqrt(g_c)).
        // Lane c < 2F holds row c of M^T, its own column.
        double dAr, dAi;
        {
            double x[F];
#pragma unroll
            for (int i = 0; i < F; ++i) {
                const double si = Ps->sqrt_gamma[i], isi = Ps->inv_sqrt_gamma[i];
                const double u = L.T[(F + i) * RS + colU], v = L.T[i * RS + colV];
                x[i] = 0.5 * (si * u * alphaA + v * isi * betaA);
            }
            lu_det_rows_complex_split<F>(x, rowLane, imagLane, dAr, dAi);
        }

        // stability monitor |det(M)^2 - 1| on checked steps
        const bool checked = (A.check_every <= 1) || (stp % A.check_every == 0) || (stp == A.n_steps);
        if (checked) {
            double a[N2];
#pragma unroll
            for (int i = 0; i < F; ++i) {
                a[i] = dp[i];
                a[F + i] = dq[i];
            }
            const double dM = lu_det_rows<N2>(a, colLane);
            const double dev = fabs(dM * dM - 1.0);
            detM = dM;
            if (!(dev <= maxdev)) maxdev = dev;
            if (!(dev <= Ps->det_tol)) good = false;
        }

        // column `lane` back from LDS: the copy in registers is dead across the
        // two eliminations, which keeps them within the register file
        {
            const int cc = colLane ? lane : 0;
#pragma unroll
            for (int i = 0; i < F; ++i) {
                dp[i] = colLane ? L.T[i * RS + cc] : 0.0;
                dq[i] = colLane ? L.T[(F + i) * RS + cc] : 0.0;
            }
        }

        // this time sample into the ring (the branch and the amplitudes are
        // finished eight samples at a time, on samples 8a .. 8a + 7)
        {
            double ph0;
            const double ex0 = overlap(Ps, 0, ph0);
            if (lane == 0) {
                L.rdr[nk] = dAr;
                L.rdi[nk] = dAi;
                L.rS[nk] = S.value();
                L.rgood[nk] = good ? 1 : 0;
                L.rex[nk][0] = ex0;
                L.rph[nk][0] = ph0;
            }
            if constexpr (!MIXED) {
                for (int m = 1; m < A.n_refs; ++m) {
                    double ph;
                    const double ex = overlap(Ps, m, ph);
                    if (lane == 0) {
                        L.rex[nk][m] = ex;
                        L.rph[nk][m] = ph;
                    }
                }
            }
            ++nk;
            if ((stp & (RB - 1)) == RB - 1) finish_ring(Ps, stp - nk + 1);
        }
    }
    if (nk > 0) finish_ring(opaque(P0), A.step_end - nk + 1);

    // ---- save the state ----
    if (modeLane) {
        A.p[lane * NP + jr] = (double)pc;
        A.q[lane * NP + jr] = (double)qc;
    }
    if (lane == 0) {
        A.scal[SC_S * NP + jr] = S.hi();
        A.scal[SC_SCOMP * NP + jr] = S.lo();
        A.scal[SC_THETA * NP + jr] = theta;
        A.scal[SC_PREV_RE * NP + jr] = prev_r;
        A.scal[SC_PREV_IM * NP + jr] = prev_i;
        A.scal[SC_PHI * NP + jr] = phi;
        A.scal[SC_GOOD * NP + jr] = good ? 1.0 : 0.0;
        A.scal[SC_DETM * NP + jr] = detM;
        A.scal[SC_MAXDEV * NP + jr] = maxdev;
        A.scal[SC_ESCALE * NP + jr] = (double)escale;
    }
    if (colLane) {
#pragma unroll
        for (int i = 0; i < F; ++i) {
            A.Mst[(int64_t)(i * N2 + lane) * NP + jr] = dp[i];
            A.Mst[(int64_t)((F + i) * N2 + lane) * NP + jr] = dq[i];
        }
    }
}

template <int F, bool MIXED>
hipError_t launch_big_F(const TrajArgs &a, hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL((traj_big_kernel<F, MIXED>), dim3((unsigned)a.n), dim3(64), 0, s, a, a.prob);
    return hipGetLastError();
}

template <bool MIXED>
hipError_t launch_big_any(int F, const TrajArgs &a, hipStream_t s)
{
    switch (F) {
    case 17: return launch_big_F<17, MIXED>(a, s);
    case 18: return launch_big_F<18, MIXED>(a, s);
    case 19: return launch_big_F<19, MIXED>(a, s);
    case 20: return launch_big_F<20, MIXED>(a, s);
    case 21: return launch_big_F<21, MIXED>(a, s);
    case 22: return launch_big_F<22, MIXED>(a, s);
    case 23: return launch_big_F<23, MIXED>(a, s);
    case 24: return launch_big_F<24, MIXED>(a, s);
    case 25: return launch_big_F<25, MIXED>(a, s);
    case 26: return launch_big_F<26, MIXED>(a, s);
    case 27: return launch_big_F<27, MIXED>(a, s);
    case 28: return launch_big_F<28, MIXED>(a, s);
    case 29: return launch_big_F<29, MIXED>(a, s);
    case 30: return launch_big_F<30, MIXED>(a, s);
    case 31: return launch_big_F<31, MIXED>(a, s);
    case 32: return launch_big_F<32, MIXED>(a, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_traj_big(int F, bool mixed, const TrajArgs &a, hipStream_t s)
{
    return mixed ? launch_big_any<true>(F, a, s) : launch_big_any<false>(F, a, s);
}

}  // namespace scivr
