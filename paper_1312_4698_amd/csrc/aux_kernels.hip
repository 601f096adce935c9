// Small kernels around the two hot ones: Husimi sampling, the time x energy
// phase table, per-trajectory weights, deterministic reductions.
#include <math.h>

#include "philox.h"
#include "scivr_internal.h"

namespace scivr {
namespace {

// One thread per trajectory: 2F normals from ceil(2F/4) Philox blocks with
// counter (index, block, 0, 0) and key (seed, 0), Box-Muller on uniform pairs;
// q = q_eq + xi / sqrt(gamma), p = p_eq + eta sqrt(gamma), ln rho of the
// product Gaussian (Husimi density of chi).
__global__ void sample_husimi_kernel(const ProblemDev *__restrict__ P, int F, uint64_t seed, uint64_t first,
                                     int64_t n, int64_t npad, double *p0, double *q0, double *logrho)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double sq = 0.0;
    const int count = 2 * F;
    for (int b = 0; 4 * b < count; ++b) {
        uint64_t r[4];
        philox4x64_10(first + (uint64_t)j, (uint64_t)b, 0, 0, seed, 0, r);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int i0 = 4 * b + 2 * h;
            if (i0 >= count) break;
            double xi, eta;  // normals i0 and i0 + 1
            box_muller(r[2 * h], r[2 * h + 1], xi, eta);
            const int mode = i0 / 2;
            q0[mode * npad + j] = P->q_eq[mode] + xi / P->sqrt_gamma[mode];
            p0[mode * npad + j] = P->p_eq[mode] + eta * P->sqrt_gamma[mode];
            sq += xi * xi + eta * eta;
        }
    }
    logrho[j] = -P->F_log_2pi - 0.5 * sq;
}

// phase[c][k] = exp(i E_k c dt), E_k = e_min + k (e_max - e_min)/(K - 1); zero padding.
__global__ void phase_table_kernel(double e_min, double e_max, int K, int kpad, int nt, int nt_pad, double dt,
                                   double2 *phase)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)nt_pad * kpad) return;
    const int c = (int)(idx / kpad), k = (int)(idx % kpad);
    double2 v;
    v.x = 0.0;
    v.y = 0.0;
    if (c < nt && k < K) {
        const double E = e_min + (double)k * (e_max - e_min) / (double)(K - 1);
        double s, co;
        sincos(E * ((double)c * dt), &s, &co);
        v.x = co;
        v.y = s;
    }
    phase[idx] = v;
}

// weight_j = good_j exp(-ln rho_j - F ln 2 pi) 4^-e_j for j < n, 0 in the padding
// (e_j: the power-of-two scale the mixed form applied to trajectory j's
// amplitudes, 0 in the FP64 form); counts good trajectories, and gives each
// good trajectory its ratio r_j = Husimi density / sampling density (1 for a
// Husimi batch), whose sum replaces n_good in the normalisation of Eq. (11).
__global__ void weights_kernel(const ProblemDev *__restrict__ P, int F, const double *__restrict__ good_row,
                               const double *__restrict__ escale_row, const double *__restrict__ logrho,
                               const double *__restrict__ p0, const double *__restrict__ q0, int husimi, int64_t n,
                               int64_t npad, double *weight, double *goodw_row, unsigned long long *n_good)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool g = false;
    if (j < npad) {
        double w = 0.0, r = 0.0;
        if (j < n && good_row[j] != 0.0) {
            // in the log domain: for a point far in the sampling density's tail
            // exp(-ln rho) alone overflows while the scaled weight is moderate
            w = exp(-logrho[j] - P->F_log_2pi - 2.0 * escale_row[j] * 0.69314718055994530942);
            g = true;
            r = 1.0;
            if (!husimi) {
                double sq = 0.0;
                for (int i = 0; i < F; ++i) {
                    const double xi = (q0[i * npad + j] - P->q_eq[i]) * P->sqrt_gamma[i];
                    const double eta = (p0[i * npad + j] - P->p_eq[i]) * P->inv_sqrt_gamma[i];
                    sq += xi * xi + eta * eta;
                }
                r = exp(-P->F_log_2pi - 0.5 * sq - logrho[j]);
            }
        }
        weight[j] = w;
        goodw_row[j] = r;
    }
    const unsigned long long cnt = __popcll(__ballot(g));
    if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(n_good, cnt);
}

// r_j = good_j H_m(z_j) / rho(z_j) for the Husimi density H_m of reference
// state m (centre ref_p[m], ref_q[m], the problem's widths): each good
// trajectory's share of reference m's good count (reading of Eq. (11)'s
// n_good for points not drawn from H_m).
__global__ void ref_good_weights_kernel(const ProblemDev *__restrict__ P, int F, int m,
                                        const double *__restrict__ good_row, const double *__restrict__ logrho,
                                        const double *__restrict__ p0, const double *__restrict__ q0, int64_t n,
                                        int64_t npad, double *goodw_row)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= npad) return;
    double r = 0.0;
    if (j < n && good_row[j] != 0.0) {
        double sq = 0.0;
        for (int i = 0; i < F; ++i) {
            const double xi = (q0[i * npad + j] - P->ref_q[m][i]) * P->sqrt_gamma[i];
            const double eta = (p0[i * npad + j] - P->ref_p[m][i]) * P->inv_sqrt_gamma[i];
            sq += xi * xi + eta * eta;
        }
        r = exp(-P->F_log_2pi - 0.5 * sq - logrho[j]);
    }
    goodw_row[j] = r;
}

// total += sum_j row[j] over j < n in a fixed order (one workgroup).
__global__ void row_sum_kernel(const double *__restrict__ row, int64_t n, double *total)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t j = threadIdx.x; j < n; j += 256) s += row[j];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) total[0] += red[0];
}

// total[k] += sum over row tiles of part[rt][k], in row-tile order (deterministic).
__global__ void spectrum_reduce_kernel(const double *__restrict__ part, int row_tiles, int K, int kpad,
                                       double *total)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    double s = 0.0;
    for (int rt = 0; rt < row_tiles; ++rt) s += part[(int64_t)rt * kpad + k];
    total[k] += s;
}

// contrib[j] = weight_j * sum over column tiles of part[ct][j].
__global__ void contrib_reduce_kernel(const double *__restrict__ part, int ctiles, const double *__restrict__ weight,
                                      int64_t n, int64_t npad, double *contrib)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double s = 0.0;
    for (int ct = 0; ct < ctiles; ++ct) s += part[(int64_t)ct * npad + j];
    contrib[j] = weight[j] * s;
}

__global__ void fill_zero_kernel(double *p, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0.0;
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_sample_husimi(const ProblemDev *P, int F, uint64_t seed, uint64_t first, int64_t n, int64_t npad,
                                double *p0, double *q0, double *logrho, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(sample_husimi_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, P, F, seed, first, n, npad,
                       p0, q0, logrho);
    return hipGetLastError();
}

hipError_t launch_phase_table(double e_min, double e_max, int K, int kpad, int nt, int nt_pad, double dt,
                              double2 *phase, hipStream_t s)
{
    const int64_t total = (int64_t)nt_pad * kpad;
    hipLaunchKernelGGL(phase_table_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, s, e_min, e_max, K, kpad, nt,
                       nt_pad, dt, phase);
    return hipGetLastError();
}

hipError_t launch_weights(const ProblemDev *P, int F, const double *good_row, const double *escale_row,
                          const double *logrho, const double *p0, const double *q0, bool husimi, int64_t n,
                          int64_t npad, double *weight, double *goodw_row, unsigned long long *n_good,
                          double *goodw_total, hipStream_t s)
{
    hipLaunchKernelGGL(weights_kernel, dim3(blocks_for(npad, 256)), dim3(256), 0, s, P, F, good_row, escale_row,
                       logrho, p0, q0, husimi ? 1 : 0, n, npad, weight, goodw_row, n_good);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(row_sum_kernel, dim3(1), dim3(256), 0, s, goodw_row, n, goodw_total);
    return hipGetLastError();
}

hipError_t launch_ref_good_weights(const ProblemDev *P, int F, int ref, const double *good_row, const double *logrho,
                                  const double *p0, const double *q0, int64_t n, int64_t npad, double *goodw_row,
                                  double *goodw_total, hipStream_t s)
{
    hipLaunchKernelGGL(ref_good_weights_kernel, dim3(blocks_for(npad, 256)), dim3(256), 0, s, P, F, ref, good_row,
                       logrho, p0, q0, n, npad, goodw_row);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(row_sum_kernel, dim3(1), dim3(256), 0, s, goodw_row, n, goodw_total);
    return hipGetLastError();
}

hipError_t launch_spectrum_reduce(const double *part_spec, int row_tiles, int K, int kpad, double *total,
                                  hipStream_t s)
{
    hipLaunchKernelGGL(spectrum_reduce_kernel, dim3(blocks_for(K, 256)), dim3(256), 0, s, part_spec, row_tiles, K,
                       kpad, total);
    return hipGetLastError();
}

hipError_t launch_contrib_reduce(const double *part_contrib, int ctiles, const double *weight, int64_t n,
                                 int64_t npad, double *contrib, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(contrib_reduce_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, part_contrib, ctiles, weight,
                       n, npad, contrib);
    return hipGetLastError();
}

hipError_t launch_fill_zero(double *p, int64_t count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_zero_kernel, dim3(blocks_for(count, 256)), dim3(256), 0, s, p, count);
    return hipGetLastError();
}

}  // namespace scivr
