// Kernels of the learned importance-sampling proposal: an affine-coupling
// flow over the whitened initial conditions, trained by weighted maximum
// likelihood on the per-trajectory contributions of Eq. (11) and sampled as
// a defensive mixture with the Husimi density.  Training runs in FP32 on
// tiled vector-ALU GEMMs (the matrices are at most 128 wide, so the work is
// small next to the trajectory kernel); inference for sampling runs the
// same networks in BF16 on the matrix cores with FP32 accumulation.
#include <math.h>

#include "flow_internal.h"
#include "philox.h"

namespace scivr {
namespace {

constexpr double LOG_2PI = 1.8378770664093454836;

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// ---------------------------------------------------------------- FP32 GEMM
// TM x 64 output tile per 256-thread workgroup (TM = 64 or 32), TM / 16 x 4
// outputs per thread, operands staged through LDS in k-slices of 32.  The
// next slice's global loads are issued into registers before the current
// slice is multiplied, so their latency overlaps the arithmetic.  The 32-row
// tile doubles the workgroups of products too small to fill the chip.  Each
// output sums its k terms in ascending order.
constexpr int GEMM_KS = 32;

template <bool AT, bool BNK, int TM>
struct F32Slice {
    static constexpr int NA = TM * GEMM_KS / 256, NB = 64 * GEMM_KS / 256;
    float a[NA], b[NB];

    __device__ void load(const GemmF32 &g, int tid, int m0, int n0, int64_t k0, int64_t ke)
    {
#pragma unroll
        for (int r = 0; r < NA; ++r) {
            const int e = tid + 256 * r;
            const int mm = AT ? (e % TM) : (e / GEMM_KS);
            const int kk = AT ? (e / TM) : (e % GEMM_KS);
            const int m = m0 + mm;
            const int64_t k = k0 + kk;
            a[r] = (m < g.M && k < ke) ? (AT ? g.A[k * g.lda + m] : g.A[(int64_t)m * g.lda + k]) : 0.f;
        }
#pragma unroll
        for (int r = 0; r < NB; ++r) {
            const int e = tid + 256 * r;
            const int nn = BNK ? (e / GEMM_KS) : (e & 63);
            const int kk = BNK ? (e % GEMM_KS) : (e >> 6);
            const int n = n0 + nn;
            const int64_t k = k0 + kk;
            float v = 0.f;
            if (n < g.N && k < ke) {
                if (n == g.ones_col)
                    v = 1.f;
                else
                    v = BNK ? g.B[(int64_t)n * g.ldb + k] : g.B[k * g.ldb + n];
            }
            b[r] = v;
        }
    }

    __device__ void store(float (*As)[TM + 4], float (*Bs)[64 + 4], int tid) const
    {
#pragma unroll
        for (int r = 0; r < NA; ++r) {
            const int e = tid + 256 * r;
            As[AT ? (e / TM) : (e % GEMM_KS)][AT ? (e % TM) : (e / GEMM_KS)] = a[r];
        }
#pragma unroll
        for (int r = 0; r < NB; ++r) {
            const int e = tid + 256 * r;
            Bs[BNK ? (e % GEMM_KS) : (e >> 6)][BNK ? (e / GEMM_KS) : (e & 63)] = b[r];
        }
    }
};

template <bool AT, bool BNK, int EPI, int TM>
__global__ void __launch_bounds__(256) gemm_f32_kernel(GemmF32 g)
{
    constexpr int RI = TM / 16;  // rows per thread
    __shared__ float As[GEMM_KS][TM + 4];
    __shared__ float Bs[GEMM_KS][64 + 4];
    const int tid = threadIdx.x;
    const int m0 = blockIdx.x * TM, n0 = blockIdx.y * 64;
    const int64_t kb = (int64_t)blockIdx.z * g.k_chunk;
    const int64_t ke = min(g.K, kb + g.k_chunk);
    const int tx = tid & 15, ty = tid >> 4;
    float acc[RI][4];
#pragma unroll
    for (int i = 0; i < RI; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.f;

    F32Slice<AT, BNK, TM> sl;
    sl.load(g, tid, m0, n0, kb, ke);
    for (int64_t k0 = kb; k0 < ke; k0 += GEMM_KS) {
        sl.store(As, Bs, tid);
        __syncthreads();
        if (k0 + GEMM_KS < ke) sl.load(g, tid, m0, n0, k0 + GEMM_KS, ke);
#pragma unroll
        for (int kk = 0; kk < GEMM_KS; ++kk) {
            float a[RI], b[4];
#pragma unroll
            for (int i = 0; i < RI; ++i) a[i] = As[kk][ty * RI + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx * 4 + j];
#pragma unroll
            for (int i = 0; i < RI; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
    float *C = g.C + (int64_t)blockIdx.z * g.c_stride;
#pragma unroll
    for (int i = 0; i < RI; ++i) {
        const int m = m0 + ty * RI + i;
        if (m >= g.M) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int n = n0 + tx * 4 + j;
            if (n >= g.N) continue;
            float v = acc[i][j];
            if (EPI == EPI_BIAS_TANH) v = tanhf(v + g.bias[n]);
            if (EPI == EPI_BIAS) v = v + g.bias[n];
            if (EPI == EPI_DTANH) {
                const float h = g.aux[(int64_t)m * g.ldaux + n];
                v = v * (1.f - h * h);
            }
            C[(int64_t)m * g.ldc + n] = v;
        }
    }
}

template <bool AT, bool BNK, int TM>
hipError_t gemm_epi(const GemmF32 &g, dim3 grid, hipStream_t s)
{
    switch (g.epi) {
    case EPI_BIAS_TANH:
        hipLaunchKernelGGL((gemm_f32_kernel<AT, BNK, EPI_BIAS_TANH, TM>), grid, dim3(256), 0, s, g);
        break;
    case EPI_BIAS: hipLaunchKernelGGL((gemm_f32_kernel<AT, BNK, EPI_BIAS, TM>), grid, dim3(256), 0, s, g); break;
    case EPI_DTANH: hipLaunchKernelGGL((gemm_f32_kernel<AT, BNK, EPI_DTANH, TM>), grid, dim3(256), 0, s, g); break;
    default: hipLaunchKernelGGL((gemm_f32_kernel<AT, BNK, EPI_PLAIN, TM>), grid, dim3(256), 0, s, g); break;
    }
    return hipGetLastError();
}

template <int TM>
hipError_t gemm_tiles(const GemmF32 &g, hipStream_t s)
{
    const int64_t chunks = (g.K + g.k_chunk - 1) / g.k_chunk;
    const dim3 grid(blocks_for(g.M, TM), blocks_for(g.N, 64), (unsigned)chunks);
    if (g.a_trans) return g.b_nk ? gemm_epi<true, true, TM>(g, grid, s) : gemm_epi<true, false, TM>(g, grid, s);
    return g.b_nk ? gemm_epi<false, true, TM>(g, grid, s) : gemm_epi<false, false, TM>(g, grid, s);
}

// ---------------------------------------------------------------- BF16 GEMM
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Round to nearest even (inputs are finite).
__device__ inline unsigned short f32_to_bf16(float x)
{
    unsigned u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

// v_mfma_f32_16x16x32_bf16 operand layout on gfx950: A[i][k] in lane i + 16 (k / 8),
// slot k % 8; B[k][j] in lane j + 16 (k / 8), slot k % 8; D[i][j] in lane
// j + 16 (i / 4), register i % 4.  Each wave computes 32 rows x one group of up
// to 128 columns (blockIdx.y selects the group); four waves per workgroup.
__global__ void __launch_bounds__(256) gemm_bf16_kernel(const float *__restrict__ X, int64_t ldx,
                                                         const unsigned short *__restrict__ W,
                                                         const float *__restrict__ bias, float *__restrict__ Y,
                                                         int64_t ldy, int M, int N, int K, int act)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int li = lane & 15, kg = lane >> 4;
    const int64_t m0 = (int64_t)blockIdx.x * 128 + wave * 32;
    const int n_base = blockIdx.y * 128;  // column group of up to 128
    const int NB = min(8, (N - n_base + 15) >> 4);
    f4 acc[2][8];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 8; ++b) acc[a][b] = (f4){0.f, 0.f, 0.f, 0.f};

    for (int k0 = 0; k0 < K; k0 += 32) {
        bf8 av[2];
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
            const int64_t row = m0 + 16 * mb + li;
            us8 t;
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const int k = k0 + 8 * kg + s;
                const float v = (row < M && k < K) ? X[row * ldx + k] : 0.f;
                t[s] = f32_to_bf16(v);
            }
            av[mb] = __builtin_bit_cast(bf8, t);
        }
#pragma unroll
        for (int nb = 0; nb < 8; ++nb) {
            if (nb >= NB) break;
            const int n = n_base + 16 * nb + li;
            us8 t;
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const int k = k0 + 8 * kg + s;
                t[s] = (n < N && k < K) ? W[(int64_t)n * K + k] : (unsigned short)0;
            }
            const bf8 bv = __builtin_bit_cast(bf8, t);
#pragma unroll
            for (int mb = 0; mb < 2; ++mb) acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[mb], bv, acc[mb][nb], 0, 0, 0);
        }
    }
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 8; ++nb) {
            if (nb >= NB) break;
            const int col = n_base + 16 * nb + li;
            if (col >= N) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = m0 + 16 * mb + 4 * kg + r;
                if (row >= M) continue;
                const float v = acc[mb][nb][r] + bias[col];
                Y[row * ldy + col] = act ? tanhf(v) : v;
            }
        }
}

// ---------------------------------------------------------------- elementwise
__global__ void to_bf16_kernel(const float *src, int64_t n, unsigned short *dst)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = f32_to_bf16(src[i]);
}

__global__ void whiten_kernel(const ProblemDev *__restrict__ P, int F, const double *__restrict__ p0,
                              const double *__restrict__ q0, int64_t pitch, int64_t n, float *X)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    for (int i = 0; i < F; ++i) {
        X[j * 2 * F + i] = (float)((q0[i * pitch + j] - P->q_eq[i]) * P->sqrt_gamma[i]);
        X[j * 2 * F + F + i] = (float)((p0[i * pitch + j] - P->p_eq[i]) * P->inv_sqrt_gamma[i]);
    }
}

__global__ void copy_kernel(const float *src, int64_t n, float *dst)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

__global__ void fill_kernel(float *p, int64_t n, float v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// offsets of the conditioning and transformed halves of layer `layer`
__device__ inline int cond_off(int F, int layer) { return (layer & 1) ? F : 0; }
__device__ inline int trans_off(int F, int layer) { return (layer & 1) ? 0 : F; }

__global__ void gather_kernel(const float *Z, int64_t n, int F, int layer, float *A)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int co = cond_off(F, layer);
    for (int i = 0; i < F; ++i) A[j * F + i] = Z[j * 2 * F + co + i];
}

// density direction: b <- (b - t) exp(-s); sum_s += sum_i s_i
__global__ void inv_step_kernel(float *Z, const float *O, int64_t n, int F, int layer, float *S_save, float *B_save,
                                float *sum_s)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int to = trans_off(F, layer);
    float ss = 0.f;
    for (int i = 0; i < F; ++i) {
        const float s = FLOW_S_CLAMP * tanhf(O[j * 2 * F + i] * (1.f / FLOW_S_CLAMP));
        const float t = O[j * 2 * F + F + i];
        const float b = (Z[j * 2 * F + to + i] - t) * expf(-s);
        Z[j * 2 * F + to + i] = b;
        if (S_save) {
            S_save[j * F + i] = s;
            B_save[j * F + i] = b;
        }
        ss += s;
    }
    sum_s[j] += ss;
}

// generation direction: b <- b exp(s) + t
__global__ void gen_step_kernel(float *Z, const float *O, int64_t n, int F, int layer)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int to = trans_off(F, layer);
    for (int i = 0; i < F; ++i) {
        const float s = FLOW_S_CLAMP * tanhf(O[j * 2 * F + i] * (1.f / FLOW_S_CLAMP));
        const float t = O[j * 2 * F + F + i];
        Z[j * 2 * F + to + i] = Z[j * 2 * F + to + i] * expf(s) + t;
    }
}

// Start of the backward pass: m_j = -c_j / sum c (dL/dlog q_j), log q_j,
// G = dL/du = -u m_j, and block partial sums of the loss sum_j m_j log q_j.
__global__ void seed_kernel(const float *U, const float *sum_s, const double *c, double inv_csum, int64_t n, int F,
                            float *G, float *m, double *loss_part)
{
    __shared__ double red[256];
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double lossj = 0.0;
    if (j < n) {
        const double mj = -c[j] * inv_csum;
        double sq = 0.0;
        for (int k = 0; k < 2 * F; ++k) {
            const double u = U[j * 2 * F + k];
            sq += u * u;
            G[j * 2 * F + k] = (float)(-u * mj);
        }
        const double logq = -(double)F * LOG_2PI - 0.5 * sq - (double)sum_s[j];
        m[j] = (float)mj;
        lossj = mj * logq;
    }
    red[threadIdx.x] = lossj;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

// Backward through one density-direction coupling step:
//   g_s = -g_b b - m (through b and the -sum s term), g_t = -g_b exp(-s),
//   g_b(in) = g_b exp(-s); output-layer gradient Go = (g_s (1 - (s/C)^2), g_t).
__global__ void coupling_bwd_kernel(float *G, const float *S, const float *Bsv, const float *m, int64_t n, int F,
                                    int layer, float *Go)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int to = trans_off(F, layer);
    const float mj = m[j];
    for (int i = 0; i < F; ++i) {
        const float gb = G[j * 2 * F + to + i];
        const float s = S[j * F + i], b = Bsv[j * F + i];
        const float e = expf(-s);
        const float sc = s * (1.f / FLOW_S_CLAMP);
        Go[j * 2 * F + i] = (-gb * b - mj) * (1.f - sc * sc);
        Go[j * 2 * F + F + i] = -gb * e;
        G[j * 2 * F + to + i] = gb * e;
    }
}

__global__ void add_cond_kernel(float *G, const float *GA, int64_t n, int F, int layer)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int co = cond_off(F, layer);
    for (int i = 0; i < F; ++i) G[j * 2 * F + co + i] += GA[j * F + i];
}

// Sum the split-K partials [chunks][N][K + 1] in chunk order: column K is the bias gradient.
// Sum of the split-K partials.  A workgroup takes 64 consecutive entries;
// its four waves sum the partials z = w, w + 4, ... in order, and wave 0 adds
// the four sums in wave order, so the result does not depend on timing.
__global__ void __launch_bounds__(256) reduce_wgrad_kernel(const float *part, int chunks, int N, int K, float *gW,
                                                           float *gb)
{
    __shared__ float sums[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t idx = (int64_t)blockIdx.x * 64 + lane;
    const int64_t per = (int64_t)N * (K + 1);
    float s = 0.f;
    if (idx < per) {
        int z = w;
        for (; z + 12 < chunks; z += 16) {
            const float a = part[(int64_t)z * per + idx], b = part[(int64_t)(z + 4) * per + idx];
            const float c = part[(int64_t)(z + 8) * per + idx], d = part[(int64_t)(z + 12) * per + idx];
            s = (((s + a) + b) + c) + d;
        }
        for (; z < chunks; z += 4) s += part[(int64_t)z * per + idx];
    }
    sums[w][lane] = s;
    __syncthreads();
    if (w != 0 || idx >= per) return;
    s = ((sums[0][lane] + sums[1][lane]) + sums[2][lane]) + sums[3][lane];
    const int nn = (int)(idx / (K + 1)), k = (int)(idx % (K + 1));
    if (k < K)
        gW[(int64_t)nn * K + k] = s;
    else
        gb[nn] = s;
}

// Adam (Kingma & Ba) with bias corrections bc1 = 1 - beta1^t, bc2 = 1 - beta2^t.
__global__ void adam_kernel(float *p, const float *g, float *m, float *v, int64_t count, float lr, float bc1, float bc2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + 1e-8f);
}

// sums[b] = sum of c over [b batch, min(n, (b+1) batch)), one workgroup per batch.
__global__ void batch_sums_kernel(const double *c, int64_t n, int64_t batch, double *sums)
{
    __shared__ double red[256];
    const int64_t b0 = (int64_t)blockIdx.x * batch;
    const int64_t b1 = min(n, b0 + batch);
    double s = 0.0;
    for (int64_t j = b0 + threadIdx.x; j < b1; j += 256) s += c[j];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = red[0];
}

__global__ void logq_kernel(const float *U, const float *sum_s, int64_t n, int F, double *logq)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double sq = 0.0;
    for (int k = 0; k < 2 * F; ++k) {
        const double u = U[j * 2 * F + k];
        sq += u * u;
    }
    logq[j] = -(double)F * LOG_2PI - 0.5 * sq - (double)sum_s[j];
}

// Normals of point `first + j` exactly as the Husimi sampler draws them
// (counter (index, block, 0, 0), key (seed, 0); xi_i, eta_i from normals 2i,
// 2i + 1) and the component uniform from counter (index, 0, 1, 0).
__global__ void draw_kernel(uint64_t seed, uint64_t first, int64_t n, int F, double alpha, double *U64,
                            uint8_t *from_normal, float *Z)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int count = 2 * F;
    for (int b = 0; 4 * b < count; ++b) {
        uint64_t r[4];
        philox4x64_10(first + (uint64_t)j, (uint64_t)b, 0, 0, seed, 0, r);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int i0 = 4 * b + 2 * h;
            if (i0 >= count) break;
            double xi, eta;
            box_muller(r[2 * h], r[2 * h + 1], xi, eta);
            const int mode = i0 / 2;
            U64[j * count + mode] = xi;
            U64[j * count + F + mode] = eta;
            Z[j * count + mode] = (float)xi;
            Z[j * count + F + mode] = (float)eta;
        }
    }
    uint64_t r[4];
    philox4x64_10(first + (uint64_t)j, 0, 1, 0, seed, 0, r);
    from_normal[j] = u01(r[0]) < alpha ? 1 : 0;
}

// Pick the point (normal draw or its image under the flow), write the
// initial conditions with the Husimi sampler's formulas, keep x in FP64 and FP32.
__global__ void select_kernel(const ProblemDev *__restrict__ P, int F, const double *U64, const uint8_t *from_normal,
                              const float *Zgen, int64_t n, int64_t npad, double *p0, double *q0, double *X64, float *Z)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const bool nrm = from_normal[j] != 0;
    const int count = 2 * F;
    for (int k = 0; k < count; ++k) {
        const double x = nrm ? U64[j * count + k] : (double)Zgen[j * count + k];
        X64[j * count + k] = x;
        Z[j * count + k] = nrm ? (float)x : Zgen[j * count + k];
    }
    for (int mode = 0; mode < F; ++mode) {
        const double xi = X64[j * count + mode], eta = X64[j * count + F + mode];
        q0[mode * npad + j] = P->q_eq[mode] + xi / P->sqrt_gamma[mode];
        p0[mode * npad + j] = P->p_eq[mode] + eta * P->sqrt_gamma[mode];
    }
}

// log of alpha N(x) + (1 - alpha) q(x), and block sums of r = N(x) / density
// and r^2 for the effective sample size.
__global__ void mixture_kernel(const double *X64, const double *logq, int64_t n, int F, double F_log_2pi,
                               double alpha, double *logrho, double *ess_part)
{
    __shared__ double red[2][256];
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double r = 0.0;
    if (j < n) {
        double sq = 0.0;
        for (int mode = 0; mode < F; ++mode) {
            const double xi = X64[j * 2 * F + mode], eta = X64[j * 2 * F + F + mode];
            sq += xi * xi + eta * eta;
        }
        const double ln = -F_log_2pi - 0.5 * sq;
        double lr;
        if (alpha >= 1.0) {
            lr = ln;
        } else if (alpha <= 0.0) {
            lr = logq[j];
        } else {
            const double a = log(alpha) + ln, b = log1p(-alpha) + logq[j];
            const double hi = fmax(a, b), lo = fmin(a, b);
            lr = hi + log1p(exp(lo - hi));
        }
        logrho[j] = lr;
        r = exp(ln - lr);
    }
    red[0][threadIdx.x] = r;
    red[1][threadIdx.x] = r * r;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        ess_part[2 * blockIdx.x] = red[0][0];
        ess_part[2 * blockIdx.x + 1] = red[1][0];
    }
}

// W1 and W2 entries N(0, 1) / sqrt(fan-in) (Philox counter (index, 0, 2, 0), key
// (seed, 0), Box-Muller on the first two words); biases and the output layer zero,
// so the initial flow is the identity and its density the Husimi density.
__global__ void init_params_kernel(float *p, int F, int H, int L, uint64_t seed)
{
    const int64_t per = flow_layer_size(F, H);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= per * L) return;
    const int64_t o = i % per;
    const int64_t w1 = 0, b1 = (int64_t)H * F, w2 = b1 + H, b2 = w2 + (int64_t)H * H;
    double scale = 0.0;
    if (o >= w1 && o < b1) scale = 1.0 / sqrt((double)F);
    if (o >= w2 && o < b2) scale = 1.0 / sqrt((double)H);
    float v = 0.f;
    if (scale != 0.0) {
        uint64_t r[4];
        philox4x64_10((uint64_t)i, 0, 2, 0, seed, 0, r);
        double z0, z1;
        box_muller(r[0], r[1], z0, z1);
        v = (float)(z0 * scale);
    }
    p[i] = v;
}

}  // namespace

hipError_t launch_flow_init_params(float *p, int F, int H, int L, uint64_t seed, hipStream_t s)
{
    const int64_t n = flow_layer_size(F, H) * L;
    hipLaunchKernelGGL(init_params_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, F, H, L, seed);
    return hipGetLastError();
}

hipError_t launch_gemm_f32(const GemmF32 &g, hipStream_t s)
{
    if (g.M <= 0 || g.N <= 0 || g.K <= 0) return hipSuccess;
    const int64_t tiles = (int64_t)blocks_for(g.M, 64) * blocks_for(g.N, 64) * ((g.K + g.k_chunk - 1) / g.k_chunk);
    return tiles < 512 ? gemm_tiles<32>(g, s) : gemm_tiles<64>(g, s);
}

hipError_t launch_gemm_bf16(const float *X, int64_t ldx, const uint16_t *W, const float *bias, float *Y, int64_t ldy,
                            int M, int N, int K, bool tanh_act, hipStream_t s)
{
    if (M <= 0 || N <= 0) return hipSuccess;
    hipLaunchKernelGGL(gemm_bf16_kernel, dim3(blocks_for(M, 128), blocks_for(N, 128)), dim3(256), 0, s, X, ldx,
                       (const unsigned short *)W, bias, Y, ldy, M, N, K, tanh_act ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_flow_to_bf16(const float *src, int64_t n, uint16_t *dst, hipStream_t s)
{
    hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, src, n, (unsigned short *)dst);
    return hipGetLastError();
}

hipError_t launch_flow_whiten(const ProblemDev *P, int F, const double *p0, const double *q0, int64_t pitch, int64_t n,
                              float *X, hipStream_t s)
{
    hipLaunchKernelGGL(whiten_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, P, F, p0, q0, pitch, n, X);
    return hipGetLastError();
}

hipError_t launch_flow_copy(const float *src, int64_t count, float *dst, hipStream_t s)
{
    hipLaunchKernelGGL(copy_kernel, dim3(blocks_for(count, 256)), dim3(256), 0, s, src, count, dst);
    return hipGetLastError();
}

hipError_t launch_flow_fill(float *p, int64_t count, float v, hipStream_t s)
{
    hipLaunchKernelGGL(fill_kernel, dim3(blocks_for(count, 256)), dim3(256), 0, s, p, count, v);
    return hipGetLastError();
}

hipError_t launch_flow_gather(const float *Z, int64_t n, int F, int layer, float *A, hipStream_t s)
{
    hipLaunchKernelGGL(gather_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, Z, n, F, layer, A);
    return hipGetLastError();
}

hipError_t launch_flow_inv_step(float *Z, const float *O, int64_t n, int F, int layer, float *S_save, float *B_save,
                                float *sum_s, hipStream_t s)
{
    hipLaunchKernelGGL(inv_step_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, Z, O, n, F, layer, S_save, B_save,
                       sum_s);
    return hipGetLastError();
}

hipError_t launch_flow_gen_step(float *Z, const float *O, int64_t n, int F, int layer, hipStream_t s)
{
    hipLaunchKernelGGL(gen_step_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, Z, O, n, F, layer);
    return hipGetLastError();
}

hipError_t launch_flow_seed(const float *U, const float *sum_s, const double *c, double inv_csum, int64_t n, int F,
                            float *G, float *m, double *loss_part, hipStream_t s)
{
    hipLaunchKernelGGL(seed_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, U, sum_s, c, inv_csum, n, F, G, m,
                       loss_part);
    return hipGetLastError();
}

hipError_t launch_flow_coupling_bwd(float *G, const float *S, const float *Bsv, const float *m, int64_t n, int F,
                                    int layer, float *Go, hipStream_t s)
{
    hipLaunchKernelGGL(coupling_bwd_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, G, S, Bsv, m, n, F, layer, Go);
    return hipGetLastError();
}

hipError_t launch_flow_add_cond(float *G, const float *GA, int64_t n, int F, int layer, hipStream_t s)
{
    hipLaunchKernelGGL(add_cond_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, G, GA, n, F, layer);
    return hipGetLastError();
}

hipError_t launch_flow_reduce_wgrad(const float *part, int chunks, int N, int K, float *gW, float *gb, hipStream_t s)
{
    const int64_t per = (int64_t)N * (K + 1);
    hipLaunchKernelGGL(reduce_wgrad_kernel, dim3(blocks_for(per, 64)), dim3(256), 0, s, part, chunks, N, K, gW, gb);
    return hipGetLastError();
}

hipError_t launch_flow_adam(float *p, const float *g, float *m, float *v, int64_t count, float lr, float bc1,
                            float bc2, hipStream_t s)
{
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(count, 256)), dim3(256), 0, s, p, g, m, v, count, lr, bc1, bc2);
    return hipGetLastError();
}

hipError_t launch_flow_batch_sums(const double *c, int64_t n, int64_t batch, double *sums, hipStream_t s)
{
    hipLaunchKernelGGL(batch_sums_kernel, dim3(blocks_for(n, (int)batch)), dim3(256), 0, s, c, n, batch, sums);
    return hipGetLastError();
}

hipError_t launch_flow_logq(const float *U, const float *sum_s, int64_t n, int F, double *logq, hipStream_t s)
{
    hipLaunchKernelGGL(logq_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, U, sum_s, n, F, logq);
    return hipGetLastError();
}

hipError_t launch_flow_draw(uint64_t seed, uint64_t first, int64_t n, int F, double alpha, double *U64,
                            uint8_t *from_normal, float *Z, hipStream_t s)
{
    hipLaunchKernelGGL(draw_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, seed, first, n, F, alpha, U64,
                       from_normal, Z);
    return hipGetLastError();
}

hipError_t launch_flow_select(const ProblemDev *P, int F, const double *U64, const uint8_t *from_normal,
                              const float *Zgen, int64_t n, int64_t npad, double *p0, double *q0, double *X64,
                              float *Z, hipStream_t s)
{
    hipLaunchKernelGGL(select_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, P, F, U64, from_normal, Zgen, n, npad,
                       p0, q0, X64, Z);
    return hipGetLastError();
}

hipError_t launch_flow_mixture(const double *X64, const double *logq, int64_t n, int F, double F_log_2pi,
                               double alpha, double *logrho, double *ess_part, hipStream_t s)
{
    hipLaunchKernelGGL(mixture_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, X64, logq, n, F, F_log_2pi, alpha,
                       logrho, ess_part);
    return hipGetLastError();
}

}  // namespace scivr
