// Kernels of the learned importance-sampling proposal (affine-coupling flow
// over the whitened initial conditions), declared for the flow entry points.
//
// Coordinates x = (xi_1..xi_F, eta_1..eta_F), xi_i = sqrt(gamma_i)(q_i - q_eq,i),
// eta_i = (p_i - p_eq,i)/sqrt(gamma_i): the Husimi density is N(0, I) in x and
// the map (p, q) -> x has unit Jacobian.  Layer l conditions on xi (even l) or
// eta (odd l) and transforms the other half with b -> b exp(s) + t, where
// (s_raw, t) come from a tanh MLP F -> H -> H -> 2F and s = 2 tanh(s_raw / 2).
// Per-layer parameters, FP32, flat: W1 [H][F], b1 [H], W2 [H][H], b2 [H],
// W3 [2F][H], b3 [2F].  Activations are row-major [sample][feature].
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "scivr_internal.h"

namespace scivr {

constexpr float FLOW_S_CLAMP = 2.0f;

struct FlowShape {
    int F, H, L;
    int64_t per_layer;  // parameters of one coupling layer
    int64_t W1() const { return 0; }
    int64_t b1() const { return (int64_t)H * F; }
    int64_t W2() const { return b1() + H; }
    int64_t b2() const { return W2() + (int64_t)H * H; }
    int64_t W3() const { return b2() + H; }
    int64_t b3() const { return W3() + 2LL * F * H; }
};

__host__ __device__ inline int64_t flow_layer_size(int F, int H) { return (int64_t)H * F + H + (int64_t)H * H + H + 2LL * F * H + 2 * F; }

enum FlowEpi { EPI_BIAS_TANH = 0, EPI_BIAS = 1, EPI_DTANH = 2, EPI_PLAIN = 3 };

// C[m][n] (+ blockIdx.z * c_stride) = epi(sum over k of A(m, k) B(k, n)), k in
// the z-th chunk [z k_chunk, min((z+1) k_chunk, K)).
//   A(m, k) = a_trans ? A[k lda + m] : A[m lda + k]
//   B(k, n) = b_nk ? B[n ldb + k] : B[k ldb + n]; B(k, ones_col) = 1 if ones_col >= 0
//   epi: tanh(acc + bias[n]) | acc + bias[n] | acc (1 - aux[m][n]^2) | acc
struct GemmF32 {
    const float *A = nullptr;
    int64_t lda = 0;
    bool a_trans = false;
    const float *B = nullptr;
    int64_t ldb = 0;
    bool b_nk = false;
    float *C = nullptr;
    int64_t ldc = 0;
    int M = 0, N = 0;
    int64_t K = 0, k_chunk = 0, c_stride = 0;
    int ones_col = -1;
    const float *bias = nullptr;
    const float *aux = nullptr;
    int64_t ldaux = 0;
    int epi = EPI_PLAIN;
};

hipError_t launch_gemm_f32(const GemmF32 &g, hipStream_t s);

// Y[m][n] = act(sum_k X[m][k] W[n][k] + bias[n]) with X rounded to BF16 and
// W given in BF16 (raw 16-bit words), FP32 accumulation on the matrix cores.
hipError_t launch_gemm_bf16(const float *X, int64_t ldx, const uint16_t *W, const float *bias, float *Y, int64_t ldy,
                            int M, int N, int K, bool tanh_act, hipStream_t s);

hipError_t launch_flow_init_params(float *p, int F, int H, int L, uint64_t seed, hipStream_t s);
hipError_t launch_flow_to_bf16(const float *src, int64_t n, uint16_t *dst, hipStream_t s);
hipError_t launch_flow_whiten(const ProblemDev *P, int F, const double *p0, const double *q0, int64_t pitch, int64_t n,
                              float *X, hipStream_t s);
hipError_t launch_flow_copy(const float *src, int64_t count, float *dst, hipStream_t s);
hipError_t launch_flow_fill(float *p, int64_t count, float v, hipStream_t s);
hipError_t launch_flow_gather(const float *Z, int64_t n, int F, int layer, float *A, hipStream_t s);
hipError_t launch_flow_inv_step(float *Z, const float *O, int64_t n, int F, int layer, float *S_save, float *B_save,
                                float *sum_s, hipStream_t s);
hipError_t launch_flow_gen_step(float *Z, const float *O, int64_t n, int F, int layer, hipStream_t s);
hipError_t launch_flow_seed(const float *U, const float *sum_s, const double *c, double inv_csum, int64_t n, int F,
                            float *G, float *m, double *loss_part, hipStream_t s);
hipError_t launch_flow_coupling_bwd(float *G, const float *S, const float *Bsv, const float *m, int64_t n, int F,
                                    int layer, float *Go, hipStream_t s);
hipError_t launch_flow_add_cond(float *G, const float *GA, int64_t n, int F, int layer, hipStream_t s);
hipError_t launch_flow_reduce_wgrad(const float *part, int chunks, int N, int K, float *gW, float *gb, hipStream_t s);
hipError_t launch_flow_adam(float *p, const float *g, float *m, float *v, int64_t count, float lr, float bc1,
                            float bc2, hipStream_t s);
hipError_t launch_flow_batch_sums(const double *c, int64_t n, int64_t batch, double *sums, hipStream_t s);
hipError_t launch_flow_logq(const float *U, const float *sum_s, int64_t n, int F, double *logq, hipStream_t s);
hipError_t launch_flow_draw(uint64_t seed, uint64_t first, int64_t n, int F, double alpha, double *U64,
                            uint8_t *from_normal, float *Z, hipStream_t s);
hipError_t launch_flow_select(const ProblemDev *P, int F, const double *U64, const uint8_t *from_normal,
                              const float *Zgen, int64_t n, int64_t npad, double *p0, double *q0, double *X64,
                              float *Z, hipStream_t s);
hipError_t launch_flow_mixture(const double *X64, const double *logq, int64_t n, int F, double F_log_2pi,
                               double alpha, double *logrho, double *ess_part, hipStream_t s);

}  // namespace scivr
