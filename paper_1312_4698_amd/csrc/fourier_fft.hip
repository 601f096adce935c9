// Exact FFT-autocorrelation form of the Fourier accumulation of the TA-SC-IVR
// estimator (Eq. (11)), an alternative to the GEMM:
//
//   sum_j w_j |A_j(E)|^2 = C(0) + 2 Re sum_{tau >= 1} C(tau) e^{i E tau dt},
//   C(tau) = sum_j w_j R_j(tau),  R_j(tau) = sum_c amp_j[c + tau] conj(amp_j[c]),
//
// because |sum_c a_c e^{i E c dt}|^2 is a trigonometric polynomial in E dt
// whose coefficients are the autocorrelation of the sequence.  With the
// sequence zero-padded to a power of two L >= 2 (n_t - 1), R_j is the
// circular autocorrelation (1/L) sum_m |X_j[m]|^2 e^{2 pi i m tau / L}, X_j =
// DFT_L(amp_j), for every lag 0 <= tau < n_t except tau = L / 2 when
// L = 2 (n_t - 1): there the lags +-L/2 fold onto one bin, so that single lag
// is summed directly.  The result equals the GEMM's to rounding.
//
// Kernels:
//  * fft_power_kernel: one workgroup of 512 threads (two waves per SIMD) per
//    trajectory at a time, the whole
//    length-L FP64 sequence in LDS (L <= 8192: 128 KB), an in-place radix-2
//    decimation-in-frequency FFT with the passes fused in pairs and the
//    twiddles in registers (bit-reversed output), and w_j |X_j[m]|^2
//    accumulated in registers at fixed bins per thread over the workgroup's
//    trajectories; concurrently running workgroups of one XCD take
//    consecutive trajectories, so the 128-byte lines of the time-major
//    amplitude buffer are shared in that XCD's L2;
//  * fft_reduce_kernel: the workgroups' partial sums in a fixed order, bins
//    back to natural order;
//  * fft_lags_kernel: C(tau) for tau < n_t by direct inverse DFT;
//  * fft_spectrum_kernel: the trigonometric sum at every energy, added to the
//    running spectrum like the GEMM's reduction.
#include <math.h>

#include "scivr_internal.h"

namespace scivr {
namespace {

constexpr int FFT_THREADS = 512;

__device__ inline double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ inline unsigned bitrev(unsigned v, int bits) { return __builtin_bitreverse32(v) >> (32 - bits); }

template <int LOG2L, bool MIXED>
__global__ void __launch_bounds__(FFT_THREADS, 1) fft_power_kernel(FftArgs G)
{
    constexpr int L = 1 << LOG2L;
    constexpr int PER = L / FFT_THREADS > 0 ? L / FFT_THREADS : 1;      // bins per thread
    __shared__ double2 X[L];
    const int t = threadIdx.x;

    // Passes are fused in pairs (radix 2^2): thread group g = t + T m (T threads) takes
    // the four elements i0, i0 + q, i0 + h, i0 + h + q (i0 = (g / q) 2h + g mod q)
    // through the passes of half-spans h and q = h / 2, which is exactly those
    // two radix-2 passes (output stays bit-reversed).  Its twiddles, with
    // p = g mod q and exponent step ts = L / (2h): W^{p ts}, W^{(p + q) ts} for
    // the first pass and W^{2 p ts} for the second, repeat with period
    // max(1, q / T) in m.  They are computed once into registers; reading
    // them from an LDS table costs bank conflicts of up to 32 ways.
    constexpr int NPAIR = LOG2L / 2;
    constexpr int NG = L / 4 / FFT_THREADS > 0 ? L / 4 / FFT_THREADS : 1;  // groups per thread per pair
    double2 tw1[NPAIR > 0 ? NPAIR : 1][NG], tw2[NPAIR > 0 ? NPAIR : 1][NG], tw3[NPAIR > 0 ? NPAIR : 1][NG];
#pragma unroll
    for (int pr = 0; pr < NPAIR; ++pr) {
        const int sft = 2 * pr, h = L >> (sft + 1), q = h >> 1;
        const int rep = q > FFT_THREADS ? q / FFT_THREADS : 1;
#pragma unroll
        for (int m = 0; m < NG; ++m) {
            if (m >= rep) break;
            const int p = (t + FFT_THREADS * m) & (q - 1);
            double sn, cs;
            sincospi(2.0 * (double)(p << sft) / (double)L, &sn, &cs);
            tw1[pr][m] = make_double2(cs, -sn);
            sincospi(2.0 * (double)((p + q) << sft) / (double)L, &sn, &cs);
            tw2[pr][m] = make_double2(cs, -sn);
            sincospi(2.0 * (double)(p << (sft + 1)) / (double)L, &sn, &cs);
            tw3[pr][m] = make_double2(cs, -sn);
        }
    }

    double acc[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r) acc[r] = 0.0;
    double2 corr = make_double2(0.0, 0.0);

    // workgroup wg runs on XCD wg % 8 as local slot wg / 8; in iteration `it` the
    // XCD's slots take trajectories [(it * 8 + xcd) * per, +per)
    const int nwg = gridDim.x;
    const int xcd = blockIdx.x % 8, slot = blockIdx.x / 8, per = nwg / 8;
    const int nt = G.nt;
    auto traj_of = [&](int64_t it) { return (it * 8 + xcd) * per + slot; };

    for (int64_t it = 0;; ++it) {
        if ((it * 8) * per >= G.n) break;  // every workgroup leaves after the same iteration
        const int64_t j = traj_of(it);
        const bool have = j < G.n;
        const double w = have ? G.weight[j] : 0.0;
        __syncthreads();  // the previous trajectory's bins have been read
        if constexpr (!MIXED) {
            for (int c = t; c < L; c += FFT_THREADS)
                X[c] = (have && c < nt) ? G.amp[(int64_t)c * G.npad + j] : make_double2(0.0, 0.0);
        } else {
            // FP16 hi/lo planes [t / 8][trajectory][t % 8]: one 16-byte chunk per plane per 8 samples
            typedef _Float16 h8 __attribute__((ext_vector_type(8)));
            for (int bch = t; bch < L / 8; bch += FFT_THREADS) {
                h8 rh = (h8)0, rl = (h8)0, ih = (h8)0, il = (h8)0;
                if (have && 8 * bch < nt) {
                    const _Float16 *a = G.amp16 + ((int64_t)bch * G.npad + j) * 8;
                    rh = *(const h8 *)(a);
                    rl = *(const h8 *)(a + G.plane);
                    ih = *(const h8 *)(a + 2 * G.plane);
                    il = *(const h8 *)(a + 3 * G.plane);
                }
#pragma unroll
                for (int s = 0; s < 8; ++s) {
                    const int c = 8 * bch + s;
                    const double re = (double)((float)rh[s] + (float)rl[s]);
                    const double im = (double)((float)ih[s] + (float)il[s]);
                    X[c] = (c < nt) ? make_double2(re, im) : make_double2(0.0, 0.0);
                }
            }
        }
        __syncthreads();
        if (G.fold && t == 0 && have) {  // the lag L / 2, summed directly
            const double2 a = X[L / 2], b0 = X[0];
            corr.x += w * (a.x * b0.x + a.y * b0.y);
            corr.y += w * (a.y * b0.x - a.x * b0.y);
        }
        // radix-2 decimation in frequency, in place, two passes at a time
#pragma unroll
        for (int pr = 0; pr < NPAIR; ++pr) {
            const int h = L >> (2 * pr + 1), q = h >> 1, lq = LOG2L - 2 * pr - 2;  // q = 2^lq
            const int rep = q > FFT_THREADS ? q / FFT_THREADS : 1;
#pragma unroll
            for (int m = 0; m < NG; ++m) {
                const int g = t + FFT_THREADS * m;
                if (g < L / 4) {
                    const int p = g & (q - 1);
                    const int i0 = ((g >> lq) << (lq + 2)) + p;
                    const double2 a = X[i0], b = X[i0 + q], c = X[i0 + h], d = X[i0 + h + q];
                    const double2 a1 = make_double2(a.x + c.x, a.y + c.y);
                    const double2 c1 = cmul(make_double2(a.x - c.x, a.y - c.y), tw1[pr][m % rep]);
                    const double2 b1 = make_double2(b.x + d.x, b.y + d.y);
                    const double2 d1 = cmul(make_double2(b.x - d.x, b.y - d.y), tw2[pr][m % rep]);
                    const double2 w3 = tw3[pr][m % rep];
                    X[i0] = make_double2(a1.x + b1.x, a1.y + b1.y);
                    X[i0 + q] = cmul(make_double2(a1.x - b1.x, a1.y - b1.y), w3);
                    X[i0 + h] = make_double2(c1.x + d1.x, c1.y + d1.y);
                    X[i0 + h + q] = cmul(make_double2(c1.x - d1.x, c1.y - d1.y), w3);
                }
            }
            __syncthreads();
        }
        if constexpr (LOG2L % 2 == 1) {  // the last pass (half-span 1, twiddle 1) alone
            for (int b = t; b < L / 2; b += FFT_THREADS) {
                const double2 u = X[2 * b], v = X[2 * b + 1];
                X[2 * b] = make_double2(u.x + v.x, u.y + v.y);
                X[2 * b + 1] = make_double2(u.x - v.x, u.y - v.y);
            }
            __syncthreads();
        }
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int p = t + r * FFT_THREADS;
            if (p < L) {
                const double2 x = X[p];
                acc[r] = fma(w, fma(x.x, x.x, x.y * x.y), acc[r]);
            }
        }
    }
    double *part = G.part + (int64_t)blockIdx.x * L;
#pragma unroll
    for (int r = 0; r < PER; ++r)
        if (t + r * FFT_THREADS < L) part[t + r * FFT_THREADS] = acc[r];
    if (t == 0) G.part_corr[blockIdx.x] = corr;
}

// S[m] = sum over workgroups of their bins, in natural order.
__global__ void fft_reduce_kernel(const double *__restrict__ part, const double2 *__restrict__ part_corr, int nwg,
                                  int log2L, double *__restrict__ S, double2 *__restrict__ corr)
{
    const int L = 1 << log2L;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < L) {
        double s = 0.0;
        for (int w = 0; w < nwg; ++w) s += part[(int64_t)w * L + p];
        S[bitrev((unsigned)p, log2L)] = s;
    }
    if (p == 0) {
        double2 c = make_double2(0.0, 0.0);
        for (int w = 0; w < nwg; ++w) {
            c.x += part_corr[w].x;
            c.y += part_corr[w].y;
        }
        *corr = c;
    }
}

// C(tau) = (1/L) sum_m S[m] e^{2 pi i m tau / L} for tau < nt (S is real);
// the folded lag takes its direct sum.
__global__ void fft_lags_kernel(const double *__restrict__ S, const double2 *__restrict__ corr, int log2L, int nt,
                                int fold, double2 *__restrict__ C)
{
    const int L = 1 << log2L;
    const int tau = blockIdx.x * blockDim.x + threadIdx.x;
    if (tau >= nt) return;
    if (fold && tau == L / 2) {
        C[tau] = *corr;
        return;
    }
    double re = 0.0, im = 0.0;
    for (int m = 0; m < L; ++m) {
        const int e = (int)(((int64_t)m * tau) & (L - 1));
        double s, c;
        sincospi(2.0 * (double)e / (double)L, &s, &c);
        re = fma(S[m], c, re);
        im = fma(S[m], s, im);
    }
    C[tau] = make_double2(re / L, im / L);
}

// total[k] += C(0) + 2 Re sum_{tau >= 1} C(tau) e^{i E_k tau dt}
__global__ void fft_spectrum_kernel(const double2 *__restrict__ C, int nt, int K, double e_min, double de, double dt,
                                    double *__restrict__ total)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    const double E = e_min + (double)k * de;
    double s = 0.0;
    for (int tau = nt - 1; tau >= 1; --tau) {
        double sn, cs;
        sincos(E * (double)tau * dt, &sn, &cs);
        s = fma(C[tau].x, cs, fma(-C[tau].y, sn, s));
    }
    total[k] += C[0].x + 2.0 * s;
}

template <bool MIXED>
hipError_t launch_power(int log2L, const FftArgs &a, int nwg, hipStream_t st)
{
    switch (log2L) {
#define SCIVR_FFT_CASE(n) \
    case n: hipLaunchKernelGGL((fft_power_kernel<n, MIXED>), dim3(nwg), dim3(FFT_THREADS), 0, st, a); break;
        SCIVR_FFT_CASE(3)
        SCIVR_FFT_CASE(4)
        SCIVR_FFT_CASE(5)
        SCIVR_FFT_CASE(6)
        SCIVR_FFT_CASE(7)
        SCIVR_FFT_CASE(8)
        SCIVR_FFT_CASE(9)
        SCIVR_FFT_CASE(10)
        SCIVR_FFT_CASE(11)
        SCIVR_FFT_CASE(12)
        SCIVR_FFT_CASE(13)
#undef SCIVR_FFT_CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

int fft_log2_length(int nt)
{
    int lg = 3;
    while ((1 << lg) < 2 * (nt - 1)) ++lg;
    return lg;
}

hipError_t launch_fft_spectrum(const double2 *C, int nt, int K, double e_min, double de, double dt, double *total,
                               hipStream_t st)
{
    hipLaunchKernelGGL(fft_spectrum_kernel, dim3((K + 127) / 128), dim3(128), 0, st, C, nt, K, e_min, de, dt, total);
    return hipGetLastError();
}

hipError_t launch_fourier_fft(const FftArgs &a, bool mixed, double e_min, double de, double dt, int K, double *S,
                              double2 *corr, double2 *C, double *total, hipStream_t st)
{
    const int lg = fft_log2_length(a.nt);
    if (lg > FFT_MAX_LOG2) return hipErrorInvalidValue;
    const int L = 1 << lg;
    hipError_t e = mixed ? launch_power<true>(lg, a, a.nwg, st) : launch_power<false>(lg, a, a.nwg, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fft_reduce_kernel, dim3((L + 255) / 256), dim3(256), 0, st, a.part, a.part_corr, a.nwg, lg, S,
                       corr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(fft_lags_kernel, dim3((a.nt + 127) / 128), dim3(128), 0, st, S, corr, lg, a.nt, a.fold, C);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(fft_spectrum_kernel, dim3((K + 127) / 128), dim3(128), 0, st, C, a.nt, K, e_min, de, dt, total);
    return hipGetLastError();
}

}  // namespace scivr
