// C ABI of the learned importance-sampling proposal (declared in
// include/scivr.h): flow parameters and Adam state, training on the
// per-trajectory contributions, density evaluation, and the defensive-mixture
// sampler that fills a context's initial conditions.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <cmath>
#include <new>
#include <algorithm>
#include <vector>

#include "ctx.h"
#include "flow_internal.h"

using namespace scivr;

struct scivr_flow {
    scivr_ctx *ctx = nullptr;
    FlowShape sh{};
    int64_t P = 0;
    int64_t adam_t = 0;
    float *d_params = nullptr, *d_grad = nullptr, *d_m = nullptr, *d_v = nullptr;
    uint16_t *d_wbf16 = nullptr;
    bool bf16_stale = true;

    // inference workspace, capacity cap_inf points
    int64_t cap_inf = 0;
    float *i_Z = nullptr, *i_Zgen = nullptr, *i_A = nullptr, *i_H1 = nullptr, *i_H2 = nullptr, *i_O = nullptr,
          *i_sums = nullptr;
    double *i_U64 = nullptr, *i_X64 = nullptr, *i_logq = nullptr, *i_ess = nullptr, *i_pq = nullptr;
    uint8_t *i_sel = nullptr;

    // training data (cap_data points) and one mini-batch (cap_batch points)
    int64_t cap_data = 0, cap_batch = 0;
    float *t_X = nullptr;
    double *t_c = nullptr, *t_bsums = nullptr, *t_pq = nullptr;
    float *t_Z = nullptr, *t_O = nullptr, *t_G = nullptr, *t_Go = nullptr, *t_GA = nullptr, *t_Gp1 = nullptr,
          *t_Gp2 = nullptr, *t_m = nullptr, *t_sums = nullptr, *t_part = nullptr;
    float *t_A = nullptr, *t_S = nullptr, *t_B = nullptr, *t_H1 = nullptr, *t_H2 = nullptr;
    double *t_loss = nullptr;
};

namespace {

// Batch rows per split-K partial of the weight gradients: about 64 partials
// per gradient, so that a batch of a few thousand rows spreads over the whole
// chip, with 64 to 512 rows in each.
int64_t wgrad_chunk(int64_t rows)
{
    return std::min<int64_t>(512, std::max<int64_t>(64, ((rows + 63) / 64 + 15) / 16 * 16));
}
constexpr int FLOW_KIND = 4;          // kernel-time slot of the flow kernels

template <typename T>
hipError_t falloc(T **p, int64_t count)
{
    return hipMalloc((void **)p, (size_t)count * sizeof(T) + 256);
}

template <typename T>
void ffree(T *&p)
{
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

void free_inference(scivr_flow *f)
{
    ffree(f->i_Z), ffree(f->i_Zgen), ffree(f->i_A), ffree(f->i_H1), ffree(f->i_H2), ffree(f->i_O), ffree(f->i_sums);
    ffree(f->i_U64), ffree(f->i_X64), ffree(f->i_logq), ffree(f->i_ess), ffree(f->i_pq), ffree(f->i_sel);
    f->cap_inf = 0;
}

void free_data(scivr_flow *f)
{
    ffree(f->t_X), ffree(f->t_c), ffree(f->t_bsums), ffree(f->t_pq);
    f->cap_data = 0;
}

void free_batch(scivr_flow *f)
{
    ffree(f->t_Z), ffree(f->t_O), ffree(f->t_G), ffree(f->t_Go), ffree(f->t_GA), ffree(f->t_Gp1), ffree(f->t_Gp2);
    ffree(f->t_m), ffree(f->t_sums), ffree(f->t_part), ffree(f->t_A), ffree(f->t_S), ffree(f->t_B), ffree(f->t_H1);
    ffree(f->t_H2), ffree(f->t_loss);
    f->cap_batch = 0;
}

int64_t chunks_of(int64_t rows) { return (rows + wgrad_chunk(rows) - 1) / wgrad_chunk(rows); }
// the most partials any batch of at most B rows takes
int64_t max_chunks(int64_t B) { return std::max<int64_t>(64, (B + 511) / 512); }

hipError_t ensure_inference(scivr_flow *f, int64_t n)
{
    if (n <= f->cap_inf) return hipSuccess;
    free_inference(f);
    const int F = f->sh.F, H = f->sh.H;
    hipError_t e;
    if ((e = falloc(&f->i_Z, n * 2 * F)) != hipSuccess) return e;
    if ((e = falloc(&f->i_Zgen, n * 2 * F)) != hipSuccess) return e;
    if ((e = falloc(&f->i_A, n * F)) != hipSuccess) return e;
    if ((e = falloc(&f->i_H1, n * H)) != hipSuccess) return e;
    if ((e = falloc(&f->i_H2, n * H)) != hipSuccess) return e;
    if ((e = falloc(&f->i_O, n * 2 * F)) != hipSuccess) return e;
    if ((e = falloc(&f->i_sums, n)) != hipSuccess) return e;
    if ((e = falloc(&f->i_U64, n * 2 * F)) != hipSuccess) return e;
    if ((e = falloc(&f->i_X64, n * 2 * F)) != hipSuccess) return e;
    if ((e = falloc(&f->i_logq, n)) != hipSuccess) return e;
    if ((e = falloc(&f->i_ess, 2 * ((n + 255) / 256))) != hipSuccess) return e;
    if ((e = falloc(&f->i_pq, n * 2 * F)) != hipSuccess) return e;
    if ((e = falloc(&f->i_sel, n)) != hipSuccess) return e;
    f->cap_inf = n;
    return hipSuccess;
}

hipError_t ensure_data(scivr_flow *f, int64_t n)
{
    if (n <= f->cap_data) return hipSuccess;
    free_data(f);
    const int F = f->sh.F;
    hipError_t e;
    if ((e = falloc(&f->t_X, n * 2 * F)) != hipSuccess) return e;
    if ((e = falloc(&f->t_c, n)) != hipSuccess) return e;
    if ((e = falloc(&f->t_bsums, n)) != hipSuccess) return e;
    if ((e = falloc(&f->t_pq, n * 2 * F)) != hipSuccess) return e;
    f->cap_data = n;
    return hipSuccess;
}

hipError_t ensure_batch(scivr_flow *f, int64_t B)
{
    if (B <= f->cap_batch) return hipSuccess;
    free_batch(f);
    const int F = f->sh.F, H = f->sh.H, L = f->sh.L;
    const int64_t part = max_chunks(B) * std::max<int64_t>(std::max<int64_t>(2LL * F * (H + 1), (int64_t)H * (H + 1)),
                                                          (int64_t)H * (F + 1));
    hipError_t e;
    if ((e = falloc(&f->t_Z, B * 2 * F)) != hipSuccess) return e;
    if ((e = falloc(&f->t_O, B * 2 * F)) != hipSuccess) return e;
    if ((e = falloc(&f->t_G, B * 2 * F)) != hipSuccess) return e;
    if ((e = falloc(&f->t_Go, B * 2 * F)) != hipSuccess) return e;
    if ((e = falloc(&f->t_GA, B * F)) != hipSuccess) return e;
    if ((e = falloc(&f->t_Gp1, B * H)) != hipSuccess) return e;
    if ((e = falloc(&f->t_Gp2, B * H)) != hipSuccess) return e;
    if ((e = falloc(&f->t_m, B)) != hipSuccess) return e;
    if ((e = falloc(&f->t_sums, B)) != hipSuccess) return e;
    if ((e = falloc(&f->t_part, part)) != hipSuccess) return e;
    if ((e = falloc(&f->t_A, (int64_t)L * B * F)) != hipSuccess) return e;
    if ((e = falloc(&f->t_S, (int64_t)L * B * F)) != hipSuccess) return e;
    if ((e = falloc(&f->t_B, (int64_t)L * B * F)) != hipSuccess) return e;
    if ((e = falloc(&f->t_H1, (int64_t)L * B * H)) != hipSuccess) return e;
    if ((e = falloc(&f->t_H2, (int64_t)L * B * H)) != hipSuccess) return e;
    if ((e = falloc(&f->t_loss, (B + 255) / 256)) != hipSuccess) return e;
    f->cap_batch = B;
    return hipSuccess;
}

GemmF32 fwd_gemm(const float *X, int64_t ldx, const float *W, const float *bias, float *Y, int64_t ldy, int M, int N,
                 int K, int epi)
{
    GemmF32 g;
    g.A = X;
    g.lda = ldx;
    g.B = W;
    g.ldb = K;
    g.b_nk = true;
    g.C = Y;
    g.ldc = ldy;
    g.M = M;
    g.N = N;
    g.K = K;
    g.k_chunk = K;
    g.bias = bias;
    g.epi = epi;
    return g;
}

// The layer network on rows A [rows][F]: H1, H2 (kept for the backward pass) and O [rows][2F].
hipError_t layer_net(scivr_flow *f, int l, const float *A, int64_t rows, float *H1, float *H2, float *O, bool bf16,
                     hipStream_t s)
{
    const int F = f->sh.F, H = f->sh.H;
    const int64_t base = (int64_t)l * f->sh.per_layer;
    const float *p = f->d_params + base;
    hipError_t e;
    if (bf16) {
        const uint16_t *w = f->d_wbf16 + base;
        if ((e = launch_gemm_bf16(A, F, w + f->sh.W1(), p + f->sh.b1(), H1, H, (int)rows, H, F, true, s)) !=
            hipSuccess)
            return e;
        if ((e = launch_gemm_bf16(H1, H, w + f->sh.W2(), p + f->sh.b2(), H2, H, (int)rows, H, H, true, s)) !=
            hipSuccess)
            return e;
        return launch_gemm_bf16(H2, H, w + f->sh.W3(), p + f->sh.b3(), O, 2 * F, (int)rows, 2 * F, H, false, s);
    }
    if ((e = launch_gemm_f32(fwd_gemm(A, F, p + f->sh.W1(), p + f->sh.b1(), H1, H, (int)rows, H, F, EPI_BIAS_TANH),
                             s)) != hipSuccess)
        return e;
    if ((e = launch_gemm_f32(fwd_gemm(H1, H, p + f->sh.W2(), p + f->sh.b2(), H2, H, (int)rows, H, H, EPI_BIAS_TANH),
                             s)) != hipSuccess)
        return e;
    return launch_gemm_f32(fwd_gemm(H2, H, p + f->sh.W3(), p + f->sh.b3(), O, 2 * F, (int)rows, 2 * F, H, EPI_BIAS), s);
}

// dW [N][K], db [N] = sum over rows of G[r][n] [X[r][k] | 1]
hipError_t weight_grad(scivr_flow *f, const float *G, int N, const float *X, int K, int64_t rows, float *gW, float *gb,
                       hipStream_t s)
{
    GemmF32 g;
    g.A = G;
    g.lda = N;
    g.a_trans = true;
    g.B = X;
    g.ldb = K;
    g.b_nk = false;
    g.C = f->t_part;
    g.ldc = K + 1;
    g.M = N;
    g.N = K + 1;
    g.K = rows;
    g.k_chunk = wgrad_chunk(rows);
    g.c_stride = (int64_t)N * (K + 1);
    g.ones_col = K;
    g.epi = EPI_PLAIN;
    hipError_t e = launch_gemm_f32(g, s);
    if (e != hipSuccess) return e;
    return launch_flow_reduce_wgrad(f->t_part, (int)chunks_of(rows), N, K, gW, gb, s);
}

// Y [rows][K] = (G [rows][N] W [N][K]) (1 - aux^2 if aux)
hipError_t data_grad(const float *G, int N, const float *W, int K, int64_t rows, const float *aux, float *Y,
                     hipStream_t s)
{
    GemmF32 g;
    g.A = G;
    g.lda = N;
    g.B = W;
    g.ldb = K;
    g.b_nk = false;
    g.C = Y;
    g.ldc = K;
    g.M = (int)rows;
    g.N = K;
    g.K = N;
    g.k_chunk = N;
    g.aux = aux;
    g.ldaux = K;
    g.epi = aux ? EPI_DTANH : EPI_PLAIN;
    return launch_gemm_f32(g, s);
}

// Gradient of L = -sum c_j log q(x_j) / sum c over rows X [rows][2F] into d_grad.
hipError_t compute_grad(scivr_flow *f, const float *X, const double *c, int64_t rows, double inv_csum, hipStream_t s)
{
    const int F = f->sh.F, H = f->sh.H, L = f->sh.L;
    const int64_t B = f->cap_batch;
    hipError_t e;
#define TRY(x)                              \
    do {                                    \
        if ((e = (x)) != hipSuccess) return e; \
    } while (0)
    TRY(launch_flow_copy(X, rows * 2 * F, f->t_Z, s));
    TRY(launch_flow_fill(f->t_sums, rows, 0.f, s));
    for (int l = L - 1; l >= 0; --l) {
        float *A = f->t_A + (int64_t)l * B * F, *S = f->t_S + (int64_t)l * B * F, *Bs = f->t_B + (int64_t)l * B * F;
        float *H1 = f->t_H1 + (int64_t)l * B * H, *H2 = f->t_H2 + (int64_t)l * B * H;
        TRY(launch_flow_gather(f->t_Z, rows, F, l, A, s));
        TRY(layer_net(f, l, A, rows, H1, H2, f->t_O, false, s));
        TRY(launch_flow_inv_step(f->t_Z, f->t_O, rows, F, l, S, Bs, f->t_sums, s));
    }
    TRY(launch_flow_seed(f->t_Z, f->t_sums, c, inv_csum, rows, F, f->t_G, f->t_m, f->t_loss, s));
    for (int l = 0; l < L; ++l) {
        const float *A = f->t_A + (int64_t)l * B * F, *S = f->t_S + (int64_t)l * B * F,
                    *Bs = f->t_B + (int64_t)l * B * F;
        const float *H1 = f->t_H1 + (int64_t)l * B * H, *H2 = f->t_H2 + (int64_t)l * B * H;
        const int64_t base = (int64_t)l * f->sh.per_layer;
        const float *p = f->d_params + base;
        float *gp = f->d_grad + base;
        TRY(launch_flow_coupling_bwd(f->t_G, S, Bs, f->t_m, rows, F, l, f->t_Go, s));
        TRY(weight_grad(f, f->t_Go, 2 * F, H2, H, rows, gp + f->sh.W3(), gp + f->sh.b3(), s));
        TRY(data_grad(f->t_Go, 2 * F, p + f->sh.W3(), H, rows, H2, f->t_Gp2, s));
        TRY(weight_grad(f, f->t_Gp2, H, H1, H, rows, gp + f->sh.W2(), gp + f->sh.b2(), s));
        TRY(data_grad(f->t_Gp2, H, p + f->sh.W2(), H, rows, H1, f->t_Gp1, s));
        TRY(weight_grad(f, f->t_Gp1, H, A, F, rows, gp + f->sh.W1(), gp + f->sh.b1(), s));
        TRY(data_grad(f->t_Gp1, H, p + f->sh.W1(), F, rows, nullptr, f->t_GA, s));
        TRY(launch_flow_add_cond(f->t_G, f->t_GA, rows, F, l, s));
    }
#undef TRY
    return hipSuccess;
}

// Density direction on Z [rows][2F] (overwritten by u) into logq [rows].
hipError_t density_pass(scivr_flow *f, float *Z, int64_t rows, bool bf16, double *logq, hipStream_t s)
{
    const int F = f->sh.F;
    hipError_t e;
    if ((e = launch_flow_fill(f->i_sums, rows, 0.f, s)) != hipSuccess) return e;
    for (int l = f->sh.L - 1; l >= 0; --l) {
        if ((e = launch_flow_gather(Z, rows, F, l, f->i_A, s)) != hipSuccess) return e;
        if ((e = layer_net(f, l, f->i_A, rows, f->i_H1, f->i_H2, f->i_O, bf16, s)) != hipSuccess) return e;
        if ((e = launch_flow_inv_step(Z, f->i_O, rows, F, l, nullptr, nullptr, f->i_sums, s)) != hipSuccess) return e;
    }
    return launch_flow_logq(Z, f->i_sums, rows, F, logq, s);
}

hipError_t generation_pass(scivr_flow *f, float *Z, int64_t rows, bool bf16, hipStream_t s)
{
    const int F = f->sh.F;
    hipError_t e;
    for (int l = 0; l < f->sh.L; ++l) {
        if ((e = launch_flow_gather(Z, rows, F, l, f->i_A, s)) != hipSuccess) return e;
        if ((e = layer_net(f, l, f->i_A, rows, f->i_H1, f->i_H2, f->i_O, bf16, s)) != hipSuccess) return e;
        if ((e = launch_flow_gen_step(Z, f->i_O, rows, F, l, s)) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t refresh_bf16(scivr_flow *f, hipStream_t s)
{
    if (!f->bf16_stale) return hipSuccess;
    hipError_t e = launch_flow_to_bf16(f->d_params, f->P, f->d_wbf16, s);
    if (e == hipSuccess) f->bf16_stale = false;
    return e;
}

// Whitened FP32 points of (p0, q0) SoA [F][pitch] into X; host arrays are staged through `stage`.
hipError_t load_points(scivr_flow *f, int64_t n, const double *p0, const double *q0, int32_t mem_kind, double *stage,
                       float *X, hipStream_t s)
{
    const int F = f->sh.F;
    hipError_t e;
    const double *dp = p0, *dq = q0;
    if (mem_kind == SCIVR_MEM_HOST) {
        if ((e = hipMemcpyAsync(stage, p0, sizeof(double) * F * n, hipMemcpyHostToDevice, s)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(stage + F * n, q0, sizeof(double) * F * n, hipMemcpyHostToDevice, s)) != hipSuccess)
            return e;
        dp = stage;
        dq = stage + F * n;
    }
    return launch_flow_whiten(f->ctx->d_prob, F, dp, dq, n, n, X, s);
}

#define FLOW_FAIL(f, st, ...) scivr::ctx_fail((f)->ctx, st, __VA_ARGS__)
#define FLOWCALL(f, expr) HIPCALL((f)->ctx, expr)
#define CHECK_FLOW(f)                          \
    do {                                       \
        if (!(f)) return SCIVR_EINVAL;         \
        CHECK_CTX((f)->ctx);                   \
    } while (0)

scivr_status train_core(scivr_flow *f, int64_t n, int32_t epochs, int64_t batch, float lr, hipStream_t s,
                        double *last_loss)
{
    if (batch > n) batch = n;
    FLOWCALL(f, ensure_batch(f, batch));
    const int64_t nb = (n + batch - 1) / batch;
    FLOWCALL(f, launch_flow_batch_sums(f->t_c, n, batch, f->t_bsums, s));
    std::vector<double> sums(nb);
    FLOWCALL(f, hipMemcpyAsync(sums.data(), f->t_bsums, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
    FLOWCALL(f, hipStreamSynchronize(s));
    const int F = f->sh.F;
    int64_t last_rows = 0;
    Timed tm(f->ctx, s, FLOW_KIND);
    for (int32_t ep = 0; ep < epochs; ++ep)
        for (int64_t b = 0; b < nb; ++b) {
            if (!(sums[b] > 0.0)) continue;
            const int64_t r0 = b * batch, rows = std::min(batch, n - r0);
            FLOWCALL(f, compute_grad(f, f->t_X + r0 * 2 * F, f->t_c + r0, rows, 1.0 / sums[b], s));
            f->adam_t += 1;
            const double bc1 = 1.0 - pow(0.9, (double)f->adam_t), bc2 = 1.0 - pow(0.999, (double)f->adam_t);
            FLOWCALL(f, launch_flow_adam(f->d_params, f->d_grad, f->d_m, f->d_v, f->P, lr, (float)bc1, (float)bc2, s));
            last_rows = rows;
        }
    tm.done();
    f->bf16_stale = true;
    if (last_loss) {
        *last_loss = 0.0;
        if (last_rows > 0) {
            const int64_t nblk = (last_rows + 255) / 256;
            std::vector<double> lp(nblk);
            FLOWCALL(f, hipMemcpyAsync(lp.data(), f->t_loss, sizeof(double) * nblk, hipMemcpyDeviceToHost, s));
            FLOWCALL(f, hipStreamSynchronize(s));
            for (double v : lp) *last_loss += v;
        }
    }
    return SCIVR_OK;
}

}  // namespace

extern "C" {

scivr_status scivr_flow_create(scivr_ctx *ctx, int32_t n_layers, int32_t width, uint64_t seed, scivr_flow **out)
{
    if (!out) return SCIVR_EINVAL;
    *out = nullptr;
    CHECK_CTX(ctx);
    if (n_layers < 1 || n_layers > 64) return ctx_fail(ctx, SCIVR_EINVAL, "n_layers %d outside [1, 64]", n_layers);
    if (width < 1 || width > 1024) return ctx_fail(ctx, SCIVR_EINVAL, "width %d outside [1, 1024]", width);
    scivr_flow *f = new (std::nothrow) scivr_flow();
    if (!f) return ctx_fail(ctx, SCIVR_ENOMEM, "out of host memory");
    f->ctx = ctx;
    f->sh.F = ctx->F;
    f->sh.H = width;
    f->sh.L = n_layers;
    f->sh.per_layer = flow_layer_size(ctx->F, width);
    f->P = f->sh.per_layer * n_layers;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = falloc(&f->d_params, f->P);
    if (e == hipSuccess) e = falloc(&f->d_grad, f->P);
    if (e == hipSuccess) e = falloc(&f->d_m, f->P);
    if (e == hipSuccess) e = falloc(&f->d_v, f->P);
    if (e == hipSuccess) e = falloc(&f->d_wbf16, f->P);
    if (e == hipSuccess) e = launch_flow_init_params(f->d_params, f->sh.F, f->sh.H, f->sh.L, seed, nullptr);
    if (e == hipSuccess) e = launch_flow_fill(f->d_m, f->P, 0.f, nullptr);
    if (e == hipSuccess) e = launch_flow_fill(f->d_v, f->P, 0.f, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        scivr_flow_destroy(f);
        return ctx_fail(ctx, e == hipErrorOutOfMemory ? SCIVR_ENOMEM : SCIVR_EDEVICE, "flow create: %s",
                        hipGetErrorString(e));
    }
    *out = f;
    return SCIVR_OK;
}

void scivr_flow_destroy(scivr_flow *f)
{
    if (!f) return;
    if (f->ctx && hipSetDevice(f->ctx->device) == hipSuccess) (void)hipDeviceSynchronize();
    free_inference(f);
    free_data(f);
    free_batch(f);
    ffree(f->d_params), ffree(f->d_grad), ffree(f->d_m), ffree(f->d_v), ffree(f->d_wbf16);
    delete f;
}

int64_t scivr_flow_param_count(const scivr_flow *f) { return f ? f->P : -1; }

scivr_status scivr_flow_set_params(scivr_flow *f, const float *params, int64_t count, int32_t mem_kind, void *stream)
{
    CHECK_FLOW(f);
    if (!params) return FLOW_FAIL(f, SCIVR_EINVAL, "null params");
    if (count != f->P) return FLOW_FAIL(f, SCIVR_EINVAL, "count %lld != %lld parameters", (long long)count,
                                        (long long)f->P);
    if (mem_kind != SCIVR_MEM_HOST && mem_kind != SCIVR_MEM_DEVICE)
        return FLOW_FAIL(f, SCIVR_EINVAL, "bad mem_kind %d", mem_kind);
    hipStream_t s = (hipStream_t)stream;
    FLOWCALL(f, hipMemcpyAsync(f->d_params, params, sizeof(float) * count,
                               mem_kind == SCIVR_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, s));
    FLOWCALL(f, launch_flow_fill(f->d_m, f->P, 0.f, s));
    FLOWCALL(f, launch_flow_fill(f->d_v, f->P, 0.f, s));
    if (mem_kind == SCIVR_MEM_HOST) FLOWCALL(f, hipStreamSynchronize(s));
    f->adam_t = 0;
    f->bf16_stale = true;
    return SCIVR_OK;
}

scivr_status scivr_flow_get_params(scivr_flow *f, float *params, int64_t count)
{
    CHECK_FLOW(f);
    if (!params) return FLOW_FAIL(f, SCIVR_EINVAL, "null params");
    if (count != f->P) return FLOW_FAIL(f, SCIVR_EINVAL, "count %lld != %lld parameters", (long long)count,
                                        (long long)f->P);
    FLOWCALL(f, hipDeviceSynchronize());
    FLOWCALL(f, hipMemcpy(params, f->d_params, sizeof(float) * count, hipMemcpyDeviceToHost));
    return SCIVR_OK;
}

static scivr_status check_points(scivr_flow *f, int64_t n, const double *p0, const double *q0, int32_t mem_kind)
{
    if (n < 1) return FLOW_FAIL(f, SCIVR_EINVAL, "n %lld < 1", (long long)n);
    if (!p0 || !q0) return FLOW_FAIL(f, SCIVR_EINVAL, "null point arrays");
    if (mem_kind != SCIVR_MEM_HOST && mem_kind != SCIVR_MEM_DEVICE)
        return FLOW_FAIL(f, SCIVR_EINVAL, "bad mem_kind %d", mem_kind);
    return SCIVR_OK;
}

scivr_status scivr_flow_train(scivr_flow *f, int64_t n, const double *p0, const double *q0, const double *c,
                              int32_t mem_kind, int32_t epochs, int32_t batch, float lr, void *stream,
                              double *last_loss)
{
    CHECK_FLOW(f);
    scivr_status st = check_points(f, n, p0, q0, mem_kind);
    if (st != SCIVR_OK) return st;
    if (!c) return FLOW_FAIL(f, SCIVR_EINVAL, "null contributions");
    if (epochs < 0 || batch < 1 || !(lr >= 0.f) || !std::isfinite(lr))
        return FLOW_FAIL(f, SCIVR_EINVAL, "bad epochs %d / batch %d / lr %g", epochs, batch, (double)lr);
    hipStream_t s = (hipStream_t)stream;
    FLOWCALL(f, ensure_data(f, n));
    FLOWCALL(f, load_points(f, n, p0, q0, mem_kind, f->t_pq, f->t_X, s));
    FLOWCALL(f, hipMemcpyAsync(f->t_c, c, sizeof(double) * n,
                               mem_kind == SCIVR_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, s));
    return train_core(f, n, epochs, batch, lr, s, last_loss);
}

scivr_status scivr_flow_train_on_batch(scivr_flow *f, int32_t epochs, int32_t batch, float lr, void *stream,
                                       double *last_loss)
{
    CHECK_FLOW(f);
    scivr_ctx *ctx = f->ctx;
    if (!ctx->accumulated) return FLOW_FAIL(f, SCIVR_ESTATE, "the context's batch has not been accumulated");
    if (!ctx->contrib_valid)
        return FLOW_FAIL(f, SCIVR_ESTATE, "the batch was accumulated without per-trajectory contributions (FFT form)");
    if (epochs < 0 || batch < 1 || !(lr >= 0.f) || !std::isfinite(lr))
        return FLOW_FAIL(f, SCIVR_EINVAL, "bad epochs %d / batch %d / lr %g", epochs, batch, (double)lr);
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = ctx->n_traj;
    FLOWCALL(f, ensure_data(f, n));
    FLOWCALL(f, launch_flow_whiten(ctx->d_prob, f->sh.F, ctx->d_p0, ctx->d_q0, ctx->npad, n, f->t_X, s));
    FLOWCALL(f, hipMemcpyAsync(f->t_c, ctx->d_contrib, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    return train_core(f, n, epochs, batch, lr, s, last_loss);
}

scivr_status scivr_flow_loss_grad(scivr_flow *f, int64_t n, const double *p0, const double *q0, const double *c,
                                  int32_t mem_kind, double *loss, float *grad)
{
    CHECK_FLOW(f);
    scivr_status st = check_points(f, n, p0, q0, mem_kind);
    if (st != SCIVR_OK) return st;
    if (!c) return FLOW_FAIL(f, SCIVR_EINVAL, "null contributions");
    hipStream_t s = nullptr;
    FLOWCALL(f, ensure_data(f, n));
    FLOWCALL(f, ensure_batch(f, n));
    FLOWCALL(f, load_points(f, n, p0, q0, mem_kind, f->t_pq, f->t_X, s));
    FLOWCALL(f, hipMemcpyAsync(f->t_c, c, sizeof(double) * n,
                               mem_kind == SCIVR_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, s));
    FLOWCALL(f, launch_flow_batch_sums(f->t_c, n, n, f->t_bsums, s));
    double csum = 0.0;
    FLOWCALL(f, hipMemcpyAsync(&csum, f->t_bsums, sizeof(double), hipMemcpyDeviceToHost, s));
    FLOWCALL(f, hipStreamSynchronize(s));
    if (!(csum > 0.0)) {
        if (loss) *loss = 0.0;
        if (grad) memset(grad, 0, sizeof(float) * f->P);
        return SCIVR_OK;
    }
    FLOWCALL(f, compute_grad(f, f->t_X, f->t_c, n, 1.0 / csum, s));
    FLOWCALL(f, hipStreamSynchronize(s));
    if (loss) {
        const int64_t nblk = (n + 255) / 256;
        std::vector<double> lp(nblk);
        FLOWCALL(f, hipMemcpy(lp.data(), f->t_loss, sizeof(double) * nblk, hipMemcpyDeviceToHost));
        *loss = 0.0;
        for (double v : lp) *loss += v;
    }
    if (grad) FLOWCALL(f, hipMemcpy(grad, f->d_grad, sizeof(float) * f->P, hipMemcpyDeviceToHost));
    return SCIVR_OK;
}

scivr_status scivr_flow_log_density(scivr_flow *f, int64_t n, const double *p0, const double *q0, int32_t mem_kind,
                                    int32_t use_bf16, double *logq, float *u)
{
    CHECK_FLOW(f);
    scivr_status st = check_points(f, n, p0, q0, mem_kind);
    if (st != SCIVR_OK) return st;
    if (!logq) return FLOW_FAIL(f, SCIVR_EINVAL, "null logq");
    hipStream_t s = nullptr;
    FLOWCALL(f, ensure_inference(f, n));
    if (use_bf16) FLOWCALL(f, refresh_bf16(f, s));
    FLOWCALL(f, load_points(f, n, p0, q0, mem_kind, f->i_pq, f->i_Z, s));
    FLOWCALL(f, density_pass(f, f->i_Z, n, use_bf16 != 0, f->i_logq, s));
    FLOWCALL(f, hipStreamSynchronize(s));
    FLOWCALL(f, hipMemcpy(logq, f->i_logq, sizeof(double) * n, hipMemcpyDeviceToHost));
    if (u) FLOWCALL(f, hipMemcpy(u, f->i_Z, sizeof(float) * n * 2 * f->sh.F, hipMemcpyDeviceToHost));
    return SCIVR_OK;
}

scivr_status scivr_flow_sample(scivr_flow *f, uint64_t seed, uint64_t first_index, int64_t n, double alpha,
                               double min_ess_frac, double *ess_frac, int32_t *used_flow, void *stream)
{
    CHECK_FLOW(f);
    scivr_ctx *ctx = f->ctx;
    if (n < 1 || n > ctx->max_traj)
        return FLOW_FAIL(f, SCIVR_EINVAL, "n_traj %lld outside [1, %lld]", (long long)n, (long long)ctx->max_traj);
    if (!(alpha >= 0.0 && alpha <= 1.0)) return FLOW_FAIL(f, SCIVR_EINVAL, "alpha %g outside [0, 1]", alpha);
    if (!(min_ess_frac >= 0.0 && min_ess_frac <= 1.0))
        return FLOW_FAIL(f, SCIVR_EINVAL, "min_ess_frac %g outside [0, 1]", min_ess_frac);
    hipStream_t s = (hipStream_t)stream;
    const int F = f->sh.F;
    FLOWCALL(f, ensure_inference(f, n));
    // one draw of m points from the mixture at Philox indices [first, first + m)
    // into the context's batch, with its effective sample size fraction
    auto draw = [&](uint64_t first, int64_t m, double *ess) -> scivr_status {
        {
            Timed tm(ctx, s, FLOW_KIND);
            if (alpha < 1.0) FLOWCALL(f, refresh_bf16(f, s));
            FLOWCALL(f, launch_flow_draw(seed, first, m, F, alpha, f->i_U64, f->i_sel, f->i_Zgen, s));
            if (alpha < 1.0) FLOWCALL(f, generation_pass(f, f->i_Zgen, m, true, s));
            FLOWCALL(f, launch_flow_select(ctx->d_prob, F, f->i_U64, f->i_sel, f->i_Zgen, m, ctx->npad, ctx->d_p0,
                                           ctx->d_q0, f->i_X64, f->i_Z, s));
            if (alpha < 1.0) FLOWCALL(f, density_pass(f, f->i_Z, m, true, f->i_logq, s));
            FLOWCALL(f, launch_flow_mixture(f->i_X64, f->i_logq, m, F, ctx->host_prob.F_log_2pi, alpha, ctx->d_logrho,
                                            f->i_ess, s));
            tm.done();
        }
        const int64_t nblk = (m + 255) / 256;
        std::vector<double> ep(2 * nblk);
        FLOWCALL(f, hipMemcpyAsync(ep.data(), f->i_ess, sizeof(double) * 2 * nblk, hipMemcpyDeviceToHost, s));
        FLOWCALL(f, hipStreamSynchronize(s));
        double s1 = 0.0, s2 = 0.0;
        for (int64_t b = 0; b < nblk; ++b) {
            s1 += ep[2 * b];
            s2 += ep[2 * b + 1];
        }
        *ess = (s2 > 0.0) ? s1 * s1 / ((double)m * s2) : 0.0;
        return SCIVR_OK;
    };
    // the fallback is decided on a pilot draw from indices disjoint from the
    // batch's, so the choice of estimator does not depend on the batch itself
    double ess = 0.0;
    scivr_status st = draw(first_index + SCIVR_FLOW_PILOT_OFFSET, std::min<int64_t>(n, SCIVR_FLOW_PILOT_SIZE), &ess);
    if (st != SCIVR_OK) return st;
    if (ess_frac) *ess_frac = ess;
    const bool flow_used = ess >= min_ess_frac;
    if (flow_used) {
        double ess_batch = 0.0;
        st = draw(first_index, n, &ess_batch);
        if (st != SCIVR_OK) return st;
    } else {
        FLOWCALL(f, launch_sample_husimi(ctx->d_prob, F, seed, first_index, n, ctx->npad, ctx->d_p0, ctx->d_q0,
                                         ctx->d_logrho, s));
    }
    if (used_flow) *used_flow = flow_used ? 1 : 0;
    ctx->n_traj = n;
    ctx->steps_done = 0;
    ctx->have_initial = true;
    ctx->husimi_batch = !flow_used;
    ctx->accumulated = false;
    ctx->full_valid = false;
    return SCIVR_OK;
}

}  // extern "C"
