// C ABI of libscivr (declared in include/scivr.h): argument validation,
// device buffers of one batch, kernel launches and host-side bookkeeping.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>

#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "ctx.h"

using namespace scivr;

namespace scivr {

scivr_status ctx_fail(scivr_ctx *c, scivr_status st, const char *fmt, ...)
{
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
        if (st == SCIVR_EDEVICE) c->device_error = true;
    }
    return st;
}

}  // namespace scivr

namespace {

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

bool finite_all(const double *a, int n)
{
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}

template <typename T>
hipError_t dalloc(T **p, size_t count)
{
    return hipMalloc((void **)p, count * sizeof(T) + 256);
}

void free_all(scivr_ctx *c)
{
    void *ptrs[] = {c->d_prob,   c->d_p0,        c->d_q0,           c->d_logrho,  c->d_p,     c->d_q,
                    c->d_scal,   c->d_M,         c->d_amp,          c->d_amp16,   c->d_phase, c->d_weight,
                    c->d_part_spec, c->d_part_contrib, c->d_contrib, c->d_total, c->d_ngood, c->d_goodw,
                    c->d_goodw_row, c->d_spart, c->d_fft_part, c->d_fft_S, c->d_fft_pcorr, c->d_fft_corr,
                    c->d_fft_C,  c->d_full_part, c->d_full_C};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (auto &e : c->events) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    c->events.clear();
}


// Coefficients and reduction constants of the kernel's exp, sincos and atan2.
// The split constants are pi/2 and ln 2 rounded to a double, then the
// remainders rounded in turn (from a 80-digit pi by Machin's formula and
// ln 2 at the same precision).
void fill_math_consts(MathConsts &m)
{
    double f = 1.0;  // n! is exact in double for n <= 18
    for (int n = 0; n < 14; ++n) {
        if (n > 0) f *= n;
        m.exp_c[n] = 1.0 / f;
    }
    double fo = 1.0, fe = 1.0;  // (2n+1)!, (2n)!
    for (int n = 0; n < 10; ++n) {
        if (n > 0) {
            fe = fo * (2 * n);
            fo = fe * (2 * n + 1);
        }
        const double sg = (n & 1) ? -1.0 : 1.0;
        if (n < 9) m.sin_c[n] = sg / fo;
        m.cos_c[n] = sg / fe;
    }
    for (int n = 0; n < 12; ++n) m.atan_c[n] = ((n & 1) ? -1.0 : 1.0) / (2 * n + 1);
    m.log2e = 0x1.71547652b82fep+0;
    m.ln2_hi = 0x1.62e42fefa39efp-1;
    m.ln2_lo = 0x1.abc9e3b39803fp-56;
    m.two_over_pi = 0x1.45f306dc9c883p-1;
    m.pio2_1 = 0x1.921fb54442d18p+0;
    m.pio2_2 = 0x1.1a62633145c07p-54;
    m.pio2_3 = -0x1.f1976b7ed8fbcp-110;
    m.pi = 0x1.921fb54442d18p+1;
    m.pio2 = 0x1.921fb54442d18p+0;
    m.pio4 = 0x1.921fb54442d18p-1;
    m.pio8 = 0x1.921fb54442d18p-2;
    m.tan_pio8 = sqrt(2.0) - 1.0;
    m.tan_pio16 = tan(m.pi / 16.0);
    m.tan_3pio16 = tan(3.0 * m.pi / 16.0);
}

// Scratch of the FFT-autocorrelation accumulation: per-workgroup bins and
// folded lags, their sums, and the lags C(tau).
struct FftScratch {
    double *part, *S;
    double2 *pcorr, *corr, *C;
};

// Byte offsets of those buffers in the static scratch (each 256-byte aligned),
// sized for FFT_NWG workgroups and the longest sequence, L = 2^FFT_MAX_LOG2.
constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr size_t STATIC_LMAX = (size_t)1 << FFT_MAX_LOG2;
constexpr size_t STATIC_OFF_PART = 0;
constexpr size_t STATIC_OFF_S = STATIC_OFF_PART + align256(sizeof(double) * FFT_NWG * STATIC_LMAX);
constexpr size_t STATIC_OFF_PCORR = STATIC_OFF_S + align256(sizeof(double) * STATIC_LMAX);
constexpr size_t STATIC_OFF_CORR = STATIC_OFF_PCORR + align256(sizeof(double2) * FFT_NWG);
constexpr size_t STATIC_OFF_C = STATIC_OFF_CORR + align256(sizeof(double2));
constexpr size_t STATIC_SCRATCH_BYTES = STATIC_OFF_C + align256(sizeof(double2) * (STATIC_LMAX / 2 + 1));
static_assert(STATIC_SCRATCH_BYTES == SCIVR_FFT_STATIC_SCRATCH_BYTES, "header states the static scratch size");

// The no-allocation FFT accumulation's scratch: one copy per device, held
// until the process ends, shared by every context on that device.
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

// Device address of each device's copy of `scratch`, looked up once per
// device with that device current (at context creation).
constexpr int STATIC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[STATIC_MAX_DEVICES] = {};

hipError_t static_scratch_address(int device, void **out)
{
    if (device < 0 || device >= STATIC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

scivr_status fft_accumulate_check(scivr_ctx *ctx)
{
    if (!ctx->have_initial || ctx->steps_done != ctx->n_steps)
        return ctx_fail(ctx, SCIVR_ESTATE, "accumulate needs a fully propagated batch (%d of %d steps)", ctx->steps_done,
                        ctx->n_steps);
    if (ctx->accumulated) return ctx_fail(ctx, SCIVR_ESTATE, "batch already accumulated");
    if (fft_log2_length(ctx->nt) > FFT_MAX_LOG2)
        return ctx_fail(ctx, SCIVR_EUNSUPPORTED, "the FFT accumulation holds at most %d steps (the problem has %d)",
                        1 << (FFT_MAX_LOG2 - 1), ctx->n_steps);
    return SCIVR_OK;
}

// Weights, the FFT form's kernels into the given scratch, and the running
// totals; `timed` brackets the Fourier step with the context's timing events.
scivr_status fft_accumulate(scivr_ctx *ctx, hipStream_t s, const FftScratch &b, bool timed)
{
    const int L = 1 << fft_log2_length(ctx->nt);
    HIPCALL(ctx, launch_weights(ctx->d_prob, ctx->F, ctx->d_scal + SC_GOOD * ctx->npad,
                                ctx->d_scal + SC_ESCALE * ctx->npad, ctx->d_logrho, ctx->d_p0, ctx->d_q0,
                                ctx->husimi_batch, ctx->n_traj, ctx->npad, ctx->d_weight, ctx->d_goodw_row,
                                ctx->d_ngood, ctx->d_goodw, s));
    for (int m = 1; m < ctx->n_refs; ++m)
        HIPCALL(ctx, launch_ref_good_weights(ctx->d_prob, ctx->F, m, ctx->d_scal + SC_GOOD * ctx->npad, ctx->d_logrho,
                                             ctx->d_p0, ctx->d_q0, ctx->n_traj, ctx->npad, ctx->d_goodw_row,
                                             ctx->d_goodw + m, s));
    FftArgs a;
    a.amp16 = ctx->d_amp16;
    a.plane = (int64_t)ctx->nt16 * ctx->npad;
    a.weight = ctx->d_weight;
    a.part = b.part;
    a.part_corr = b.pcorr;
    a.n = ctx->n_traj;
    // FP64 amplitudes are [t][reference state][trajectory]: a time row of one
    // state is n_refs row blocks apart (several states run in FP64 only)
    a.npad = (int64_t)ctx->n_refs * ctx->npad;
    a.nt = ctx->nt;
    a.nwg = FFT_NWG;
    a.fold = (L == 2 * (ctx->nt - 1)) ? 1 : 0;
    {
        Timed tm(timed ? ctx : nullptr, s, 2);
        // one pass per reference state through the same scratch, in stream order
        for (int m = 0; m < ctx->n_refs; ++m) {
            a.amp = ctx->d_amp + (int64_t)m * ctx->npad;
            HIPCALL(ctx, launch_fourier_fft(a, ctx->precision == SCIVR_PRECISION_MIXED, ctx->e_min,
                                            (ctx->e_max - ctx->e_min) / (double)(ctx->n_energies - 1), ctx->dt,
                                            ctx->n_energies, b.S, b.corr, b.C,
                                            ctx->d_total + (int64_t)m * ctx->n_energies, s));
        }
        tm.done();
    }
    ctx->n_total += ctx->n_traj;
    ctx->accumulated = true;
    ctx->contrib_valid = false;
    ctx->full_valid = false;
    return SCIVR_OK;
}

}  // namespace

extern "C" {

int32_t scivr_abi_version(void) { return SCIVR_ABI_VERSION; }

const char *scivr_last_error(const scivr_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

scivr_status scivr_create(const scivr_problem *p, int32_t device, scivr_ctx **out)
{
    if (!out) return SCIVR_EINVAL;
    *out = nullptr;
    if (!p) return SCIVR_EINVAL;
    const int F = p->F;
    if (F < 1 || F > SCIVR_F_MAX) return SCIVR_EINVAL;
    if (!p->k_harm || !p->morse_D || !p->morse_a || !p->lambda || !p->gamma || !p->p_eq || !p->q_eq)
        return SCIVR_EINVAL;
    if (p->n_steps < 1 || p->n_energies < 2 || !(p->e_max > p->e_min) || !(p->dt > 0) || p->check_every < 1 ||
        p->max_traj < 1 || !(p->det_tol >= 0))
        return SCIVR_EINVAL;
    if (!std::isfinite(p->dt) || !std::isfinite(p->e_min) || !std::isfinite(p->e_max) || !std::isfinite(p->det_tol))
        return SCIVR_EINVAL;
    if (!finite_all(p->k_harm, F) || !finite_all(p->morse_D, F) || !finite_all(p->morse_a, F) ||
        !finite_all(p->lambda, F * F) || !finite_all(p->gamma, F) || !finite_all(p->p_eq, F) ||
        !finite_all(p->q_eq, F))
        return SCIVR_EINVAL;
    for (int i = 0; i < F; ++i)
        if (!(p->gamma[i] > 0)) return SCIVR_EINVAL;
    if (p->precision != SCIVR_PRECISION_FP64 && p->precision != SCIVR_PRECISION_MIXED) return SCIVR_EINVAL;
    if ((int64_t)p->n_steps + 1 > (int64_t)INT32_MAX - 64 || p->n_energies > (1 << 24) || p->max_traj > (1ll << 31))
        return SCIVR_EINVAL;

    scivr_ctx *c = new (std::nothrow) scivr_ctx();
    if (!c) return SCIVR_ENOMEM;
    c->device = device;
    c->F = F;
    c->n_steps = p->n_steps;
    c->n_energies = p->n_energies;
    c->check_every = p->check_every;
    c->precision = p->precision;
    c->dt = p->dt;
    c->e_min = p->e_min;
    c->e_max = p->e_max;
    c->det_tol = p->det_tol;
    c->max_traj = p->max_traj;
    c->npad = round_up(p->max_traj, GEMM_BM);
    c->nt = p->n_steps + 1;
    c->nt_pad = (int32_t)round_up(c->nt, GEMM_BK);
    c->nt_alloc = c->nt_pad + 2 * GEMM_BK;  // the FP64 GEMM prefetches two time blocks ahead
    c->kpad = (int32_t)round_up(p->n_energies, GEMM_BN);
    c->nt16 = (int32_t)round_up(c->nt, GEMM16_BK);
    c->row_tiles = (int32_t)(c->npad / GEMM_BM);
    c->col_tiles = c->kpad / GEMM_BN;

    // trajectory-independent constants
    ProblemDev &h = c->host_prob;
    memset(&h, 0, sizeof h);
    double sg = 0.0;
    for (int i = 0; i < F; ++i) {
        h.k[i] = p->k_harm[i];
        h.D[i] = p->morse_D[i];
        h.a[i] = p->morse_a[i];
        h.gamma[i] = p->gamma[i];
        h.sqrt_gamma[i] = sqrt(p->gamma[i]);
        h.inv_sqrt_gamma[i] = 1.0 / h.sqrt_gamma[i];
        h.inv4gamma[i] = 1.0 / (4.0 * p->gamma[i]);
        h.p_eq[i] = p->p_eq[i];
        h.q_eq[i] = p->q_eq[i];
        h.ref_p[0][i] = p->p_eq[i];
        h.ref_q[0][i] = p->q_eq[i];
        sg += p->gamma[i];
    }
    for (int i = 0; i < F; ++i)
        for (int j = i + 1; j < F; ++j) {
            h.lam[i * FMAX + j] = p->lambda[i * F + j];
            h.lam[j * FMAX + i] = p->lambda[i * F + j];
        }
    // fourth-order triple jump: w1 = 1/(2 - 2^(1/3)), w0 = -2^(1/3) w1
    const double cbrt2 = cbrt(2.0);
    const double w1 = 1.0 / (2.0 - cbrt2);
    const double w0 = -cbrt2 / (2.0 - cbrt2);
    const double dco[4] = {0.5 * w1, 0.5 * (w0 + w1), 0.5 * (w0 + w1), 0.5 * w1};
    const double cco[3] = {w1, w0, w1};
    for (int s = 0; s < 4; ++s) h.hd[s] = dco[s] * p->dt;
    for (int s = 0; s < 3; ++s) h.hc[s] = cco[s] * p->dt;
    h.dt = p->dt;
    h.sum_gamma = sg;
    h.cos_gdt = cos(sg * p->dt);
    h.sin_gdt = sin(sg * p->dt);
    h.det_tol = p->det_tol;
    h.F_log_2pi = (double)F * log(2.0 * M_PI);
    h.e_min = p->e_min;
    h.e_max = p->e_max;
    fill_math_consts(h.mc);
    h.n_refs = 1;

    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) {
        delete c;
        return SCIVR_EDEVICE;
    }
    if (static_scratch_address(device, &c->d_static_scratch) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return SCIVR_EDEVICE;
    }
    const int64_t NP = c->npad;
    const int64_t G2 = 4ll * F * F;
    hipError_t ea = hipSuccess;
    auto A = [&](hipError_t r) {
        if (r != hipSuccess && ea == hipSuccess) ea = r;
    };
    A(dalloc(&c->d_prob, 1));
    A(dalloc(&c->d_p0, F * NP));
    A(dalloc(&c->d_q0, F * NP));
    A(dalloc(&c->d_logrho, NP));
    A(dalloc(&c->d_p, F * NP));
    A(dalloc(&c->d_q, F * NP));
    A(dalloc(&c->d_spart, F * NP));
    A(dalloc(&c->d_scal, NSCAL * NP));
    A(dalloc(&c->d_M, G2 * NP));
    const bool mixed = c->precision == SCIVR_PRECISION_MIXED;
    if (mixed) {
        A(dalloc(&c->d_amp16, 4ll * c->nt16 * NP));
    } else {
        A(dalloc(&c->d_amp, (int64_t)c->nt_alloc * NP));
        A(dalloc(&c->d_phase, (int64_t)c->nt_alloc * c->kpad));
    }
    A(dalloc(&c->d_weight, NP));
    A(dalloc(&c->d_part_spec, (int64_t)c->row_tiles * c->kpad));
    A(dalloc(&c->d_part_contrib, (int64_t)(c->kpad / 64) * NP));
    A(dalloc(&c->d_contrib, NP));
    A(dalloc(&c->d_total, c->n_energies));
    A(dalloc(&c->d_ngood, 1));
    A(dalloc(&c->d_goodw, 1));
    A(dalloc(&c->d_goodw_row, NP));
    if (ea != hipSuccess) {
        const bool oom = (ea == hipErrorOutOfMemory || ea == hipErrorMemoryAllocation);
        free_all(c);
        delete c;
        (void)hipGetLastError();
        return oom ? SCIVR_ENOMEM : SCIVR_EDEVICE;
    }
    hipStream_t s0 = nullptr;
    e = hipMemcpy(c->d_prob, &h, sizeof h, hipMemcpyHostToDevice);
    if (e == hipSuccess && !mixed) e = launch_fill_zero((double *)c->d_amp, 2ll * c->nt_alloc * NP, s0);
    if (e == hipSuccess && mixed) e = launch_fill_zero((double *)c->d_amp16, (int64_t)c->nt16 * NP, s0);
    if (e == hipSuccess) e = launch_fill_zero(c->d_logrho, NP, s0);
    if (e == hipSuccess) e = launch_fill_zero(c->d_scal, NSCAL * NP, s0);
    if (e == hipSuccess) e = launch_fill_zero(c->d_total, c->n_energies, s0);
    if (e == hipSuccess) e = launch_fill_zero((double *)c->d_ngood, 1, s0);
    if (e == hipSuccess) e = launch_fill_zero(c->d_goodw, 1, s0);
    if (e == hipSuccess && !mixed)
        e = launch_phase_table(p->e_min, p->e_max, p->n_energies, c->kpad, c->nt, c->nt_alloc, p->dt, c->d_phase, s0);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        free_all(c);
        delete c;
        return SCIVR_EDEVICE;
    }
    *out = c;
    return SCIVR_OK;
}

void scivr_destroy(scivr_ctx *ctx)
{
    if (!ctx) return;
    if (hipSetDevice(ctx->device) == hipSuccess) (void)hipDeviceSynchronize();
    free_all(ctx);
    delete ctx;
}

scivr_status scivr_sample_husimi(scivr_ctx *ctx, uint64_t seed, uint64_t first_index, int64_t n_traj, void *stream)
{
    CHECK_CTX(ctx);
    if (n_traj < 1 || n_traj > ctx->max_traj)
        return ctx_fail(ctx, SCIVR_EINVAL, "n_traj %lld outside [1, %lld]", (long long)n_traj, (long long)ctx->max_traj);
    hipStream_t s = (hipStream_t)stream;
    Timed tm(ctx, s, 0);
    HIPCALL(ctx, launch_sample_husimi(ctx->d_prob, ctx->F, seed, first_index, n_traj, ctx->npad, ctx->d_p0,
                                      ctx->d_q0, ctx->d_logrho, s));
    tm.done();
    ctx->n_traj = n_traj;
    ctx->steps_done = 0;
    ctx->have_initial = true;
    ctx->husimi_batch = true;
    ctx->accumulated = false;
    ctx->full_valid = false;
    return SCIVR_OK;
}

scivr_status scivr_set_initial(scivr_ctx *ctx, int64_t n_traj, const double *p0, const double *q0,
                               const double *log_density, int32_t mem_kind, void *stream)
{
    CHECK_CTX(ctx);
    if (n_traj < 1 || n_traj > ctx->max_traj)
        return ctx_fail(ctx, SCIVR_EINVAL, "n_traj %lld outside [1, %lld]", (long long)n_traj, (long long)ctx->max_traj);
    if (!p0 || !q0 || !log_density) return ctx_fail(ctx, SCIVR_EINVAL, "null initial-condition pointer");
    if (mem_kind != SCIVR_MEM_HOST && mem_kind != SCIVR_MEM_DEVICE)
        return ctx_fail(ctx, SCIVR_EINVAL, "bad mem_kind %d", mem_kind);
    hipStream_t s = (hipStream_t)stream;
    const hipMemcpyKind kind = mem_kind == SCIVR_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    const size_t row = (size_t)n_traj * sizeof(double), pitch = (size_t)ctx->npad * sizeof(double);
    HIPCALL(ctx, hipMemcpy2DAsync(ctx->d_p0, pitch, p0, row, row, ctx->F, kind, s));
    HIPCALL(ctx, hipMemcpy2DAsync(ctx->d_q0, pitch, q0, row, row, ctx->F, kind, s));
    HIPCALL(ctx, hipMemcpyAsync(ctx->d_logrho, log_density, row, kind, s));
    if (mem_kind == SCIVR_MEM_HOST) HIPCALL(ctx, hipStreamSynchronize(s));
    ctx->n_traj = n_traj;
    ctx->steps_done = 0;
    ctx->have_initial = true;
    ctx->husimi_batch = false;
    ctx->accumulated = false;
    ctx->full_valid = false;
    return SCIVR_OK;
}

scivr_status scivr_propagate(scivr_ctx *ctx, int32_t step_begin, int32_t step_end, void *stream)
{
    CHECK_CTX(ctx);
    if (!ctx->have_initial) return ctx_fail(ctx, SCIVR_ESTATE, "propagate before initial conditions");
    if (step_begin != ctx->steps_done)
        return ctx_fail(ctx, SCIVR_ESTATE, "step_begin %d but %d steps done", step_begin, ctx->steps_done);
    if (step_end <= step_begin || step_end > ctx->n_steps)
        return ctx_fail(ctx, SCIVR_EINVAL, "step_end %d outside (%d, %d]", step_end, step_begin, ctx->n_steps);
    hipStream_t s = (hipStream_t)stream;
    TrajArgs a;
    a.prob = ctx->d_prob;
    a.p0 = ctx->d_p0;
    a.q0 = ctx->d_q0;
    a.p = ctx->d_p;
    a.q = ctx->d_q;
    a.scal = ctx->d_scal;
    a.spart = ctx->d_spart;
    a.Mst = ctx->d_M;
    a.amp = ctx->d_amp;
    a.amp16 = ctx->d_amp16;
    a.plane = (int64_t)ctx->nt16 * ctx->npad;
    a.n = ctx->n_traj;
    a.npad = ctx->npad;
    a.step_begin = step_begin;
    a.step_end = step_end;
    a.n_steps = ctx->n_steps;
    a.check_every = ctx->check_every;
    a.n_refs = ctx->n_refs;
    a.stop_flagged = ctx->stop_flagged;
    Timed tm(ctx, s, 1);
    HIPCALL(ctx, launch_traj(ctx->F, ctx->precision == SCIVR_PRECISION_MIXED, a, s));
    tm.done();
    ctx->steps_done = step_end;
    ctx->accumulated = false;
    ctx->full_valid = false;
    return SCIVR_OK;
}

scivr_status scivr_set_stop_flagged(scivr_ctx *ctx, int32_t enable)
{
    CHECK_CTX(ctx);
    ctx->stop_flagged = enable != 0;
    return SCIVR_OK;
}

scivr_status scivr_accumulate_spectrum(scivr_ctx *ctx, void *stream)
{
    CHECK_CTX(ctx);
    if (!ctx->have_initial || ctx->steps_done != ctx->n_steps)
        return ctx_fail(ctx, SCIVR_ESTATE, "accumulate needs a fully propagated batch (%d of %d steps)", ctx->steps_done,
                    ctx->n_steps);
    if (ctx->accumulated) return ctx_fail(ctx, SCIVR_ESTATE, "batch already accumulated");
    hipStream_t s = (hipStream_t)stream;
    HIPCALL(ctx, launch_weights(ctx->d_prob, ctx->F, ctx->d_scal + SC_GOOD * ctx->npad,
                                ctx->d_scal + SC_ESCALE * ctx->npad, ctx->d_logrho, ctx->d_p0, ctx->d_q0,
                                ctx->husimi_batch, ctx->n_traj, ctx->npad, ctx->d_weight, ctx->d_goodw_row,
                                ctx->d_ngood, ctx->d_goodw, s));
    // the good count of every further reference state (its Husimi mass of the batch)
    for (int m = 1; m < ctx->n_refs; ++m)
        HIPCALL(ctx, launch_ref_good_weights(ctx->d_prob, ctx->F, m, ctx->d_scal + SC_GOOD * ctx->npad, ctx->d_logrho,
                                             ctx->d_p0, ctx->d_q0, ctx->n_traj, ctx->npad, ctx->d_goodw_row,
                                             ctx->d_goodw + m, s));
    // only the row tiles that hold trajectories of this batch
    const int32_t row_tiles = (int32_t)((ctx->n_traj + GEMM_BM - 1) / GEMM_BM);
    if (ctx->precision == SCIVR_PRECISION_MIXED) {
        GemmF16Args g;
        g.amp16 = ctx->d_amp16;
        g.plane = (int64_t)ctx->nt16 * ctx->npad;
        g.weight = ctx->d_weight;
        g.part_spec = ctx->d_part_spec;
        g.part_contrib = ctx->d_part_contrib;
        g.npad = ctx->npad;
        g.kpad = ctx->kpad;
        g.nt_pad = ctx->nt16;
        g.K = ctx->n_energies;
        g.row_tiles = row_tiles;
        g.col_tiles = ctx->col_tiles;
        g.e_min = ctx->e_min;
        g.de = (ctx->e_max - ctx->e_min) / (double)(ctx->n_energies - 1);
        g.dt = ctx->dt;
        Timed tm(ctx, s, 2);
        HIPCALL(ctx, launch_fourier_f16(g, s));
        tm.done();
    } else {
        GemmArgs g;
        g.amp = ctx->d_amp;
        g.phase = ctx->d_phase;
        g.weight = ctx->d_weight;
        g.part_spec = ctx->d_part_spec;
        g.part_contrib = ctx->d_part_contrib;
        g.npad = (int64_t)ctx->n_refs * ctx->npad;  // the reference states' row blocks side by side
        g.ref_rows = ctx->npad;
        g.kpad = ctx->kpad;
        g.nt_pad = ctx->nt_pad;
        g.tiles_per_ref = row_tiles;
        g.row_tiles = ctx->n_refs * row_tiles;
        g.col_tiles = ctx->col_tiles;
        Timed tm(ctx, s, 2);
        HIPCALL(ctx, launch_fourier_fp64(g, s));
        tm.done();
    }
    {
        Timed tm(ctx, s, 3);
        for (int m = 0; m < ctx->n_refs; ++m)
            HIPCALL(ctx, launch_spectrum_reduce(ctx->d_part_spec + (int64_t)m * row_tiles * ctx->kpad, row_tiles,
                                                ctx->n_energies, ctx->kpad, ctx->d_total + (int64_t)m * ctx->n_energies,
                                                s));
        // per-trajectory contributions of reference state 0
        HIPCALL(ctx, launch_contrib_reduce(ctx->d_part_contrib, ctx->kpad / 64, ctx->d_weight, ctx->n_traj,
                                           (int64_t)ctx->n_refs * ctx->npad, ctx->d_contrib, s));
        tm.done();
    }
    ctx->n_total += ctx->n_traj;
    ctx->accumulated = true;
    ctx->contrib_valid = true;
    ctx->full_valid = false;
    return SCIVR_OK;
}

scivr_status scivr_accumulate_spectrum_fft(scivr_ctx *ctx, void *stream)
{
    CHECK_CTX(ctx);
    scivr_status st = fft_accumulate_check(ctx);
    if (st != SCIVR_OK) return st;
    if (!ctx->d_fft_part) {  // scratch for the longest sequence the library takes, on first use
        const int Lmax = 1 << FFT_MAX_LOG2;
        FftScratch b{};
        const bool ok = dalloc(&b.part, (int64_t)FFT_NWG * Lmax) == hipSuccess && dalloc(&b.S, Lmax) == hipSuccess &&
                        dalloc(&b.pcorr, FFT_NWG) == hipSuccess && dalloc(&b.corr, 1) == hipSuccess &&
                        dalloc(&b.C, Lmax / 2 + 1) == hipSuccess;
        if (!ok) {
            for (void *q : {(void *)b.part, (void *)b.S, (void *)b.pcorr, (void *)b.corr, (void *)b.C})
                if (q) (void)hipFree(q);
            (void)hipGetLastError();
            return ctx_fail(ctx, SCIVR_ENOMEM, "FFT scratch allocation failed");
        }
        ctx->d_fft_part = b.part;
        ctx->d_fft_S = b.S;
        ctx->d_fft_pcorr = b.pcorr;
        ctx->d_fft_corr = b.corr;
        ctx->d_fft_C = b.C;
    }
    const FftScratch b{ctx->d_fft_part, ctx->d_fft_S, ctx->d_fft_pcorr, ctx->d_fft_corr, ctx->d_fft_C};
    return fft_accumulate(ctx, (hipStream_t)stream, b, true);
}

scivr_status scivr_accumulate_spectrum_fft_noalloc(scivr_ctx *ctx, void *stream)
{
    CHECK_CTX(ctx);
    scivr_status st = fft_accumulate_check(ctx);
    if (st != SCIVR_OK) return st;
    // the device address of this device's copy of `scratch`, looked up when
    // the context was created; the array's name is not a device address here
    char *base = static_cast<char *>(ctx->d_static_scratch);
    if (!base) return ctx_fail(ctx, SCIVR_EDEVICE, "no device address for the static FFT scratch");
    FftScratch b;
    b.part = reinterpret_cast<double *>(base + STATIC_OFF_PART);
    b.S = reinterpret_cast<double *>(base + STATIC_OFF_S);
    b.pcorr = reinterpret_cast<double2 *>(base + STATIC_OFF_PCORR);
    b.corr = reinterpret_cast<double2 *>(base + STATIC_OFF_CORR);
    b.C = reinterpret_cast<double2 *>(base + STATIC_OFF_C);
    return fft_accumulate(ctx, (hipStream_t)stream, b, false);
}

scivr_status scivr_accumulate_spectrum_full(scivr_ctx *ctx, void *stream)
{
    CHECK_CTX(ctx);
    if (!ctx->have_initial || ctx->steps_done != ctx->n_steps)
        return ctx_fail(ctx, SCIVR_ESTATE, "accumulate needs a fully propagated batch (%d of %d steps)", ctx->steps_done,
                        ctx->n_steps);
    if (ctx->accumulated) return ctx_fail(ctx, SCIVR_ESTATE, "batch already accumulated");
    if (ctx->precision != SCIVR_PRECISION_FP64)
        return ctx_fail(ctx, SCIVR_EUNSUPPORTED, "the double-time form runs in the FP64 form only");
    if (ctx->F > 16) return ctx_fail(ctx, SCIVR_EUNSUPPORTED, "the double-time form takes F <= 16 (F = %d)", ctx->F);
    // splits of each trajectory's segment rounds: enough waves to fill the
    // device, at most one split per round
    const int W = 64 / ctx->F;
    const int rounds = ctx->n_steps / W + 1;
    const int64_t want = (4096 + ctx->max_traj - 1) / ctx->max_traj;
    const int splits = (int)std::max<int64_t>(1, std::min<int64_t>(want, rounds));
    if (!ctx->d_full_part) {
        double2 *part = nullptr, *C = nullptr;
        const bool ok = dalloc(&part, (int64_t)splits * ctx->nt * ctx->npad) == hipSuccess &&
                        dalloc(&C, ctx->nt) == hipSuccess;
        if (!ok) {
            if (part) (void)hipFree(part);
            if (C) (void)hipFree(C);
            (void)hipGetLastError();
            return ctx_fail(ctx, SCIVR_ENOMEM, "double-time lag buffer allocation failed (%d x %d x %lld)", splits,
                            ctx->nt, (long long)ctx->npad);
        }
        ctx->d_full_part = part;
        ctx->d_full_C = C;
        ctx->full_splits = splits;
    }
    hipStream_t s = (hipStream_t)stream;
    HIPCALL(ctx, launch_weights(ctx->d_prob, ctx->F, ctx->d_scal + SC_GOOD * ctx->npad,
                                ctx->d_scal + SC_ESCALE * ctx->npad, ctx->d_logrho, ctx->d_p0, ctx->d_q0,
                                ctx->husimi_batch, ctx->n_traj, ctx->npad, ctx->d_weight, ctx->d_goodw_row,
                                ctx->d_ngood, ctx->d_goodw, s));
    // the good count of every further reference state (its Husimi mass of the batch)
    for (int m = 1; m < ctx->n_refs; ++m)
        HIPCALL(ctx, launch_ref_good_weights(ctx->d_prob, ctx->F, m, ctx->d_scal + SC_GOOD * ctx->npad, ctx->d_logrho,
                                             ctx->d_p0, ctx->d_q0, ctx->n_traj, ctx->npad, ctx->d_goodw_row,
                                             ctx->d_goodw + m, s));
    FullArgs a;
    a.prob = ctx->d_prob;
    a.p0 = ctx->d_p0;
    a.q0 = ctx->d_q0;
    a.part = ctx->d_full_part;
    a.n = ctx->n_traj;
    a.npad = ctx->npad;
    a.nt = ctx->nt;
    a.n_steps = ctx->n_steps;
    a.splits = ctx->full_splits;
    {
        Timed tm(ctx, s, 2);
        // one pass per reference state through the same lag buffer, in stream
        // order; reference 0 last, so that scivr_read_lags returns chi's sums
        for (int m = ctx->n_refs - 1; m >= 0; --m) {
            a.ref = m;
            HIPCALL(ctx, hipMemsetAsync(a.part, 0, sizeof(double2) * (size_t)a.splits * a.nt * a.npad, s));
            HIPCALL(ctx, launch_ta_full(ctx->F, a, s));
            HIPCALL(ctx, launch_ta_lags(a, ctx->d_weight, ctx->d_full_C, s));
            HIPCALL(ctx, launch_fft_spectrum(ctx->d_full_C, ctx->nt, ctx->n_energies, ctx->e_min,
                                             (ctx->e_max - ctx->e_min) / (double)(ctx->n_energies - 1), ctx->dt,
                                             ctx->d_total + (int64_t)m * ctx->n_energies, s));
        }
        tm.done();
    }
    ctx->n_total += ctx->n_traj;
    ctx->accumulated = true;
    ctx->contrib_valid = false;
    ctx->full_valid = true;
    return SCIVR_OK;
}

scivr_status scivr_read_lags(scivr_ctx *ctx, double *R)
{
    CHECK_CTX(ctx);
    if (!R) return ctx_fail(ctx, SCIVR_EINVAL, "null output");
    if (!ctx->full_valid) return ctx_fail(ctx, SCIVR_ESTATE, "the last accumulation was not the double-time form");
    HIPCALL(ctx, hipDeviceSynchronize());
    const int64_t n = ctx->n_traj, nt = ctx->nt, np = ctx->npad;
    std::vector<double2> buf((size_t)nt * np);
    for (int64_t j = 0; j < n; ++j)
        for (int64_t t = 0; t < nt; ++t) R[(j * nt + t) * 2] = R[(j * nt + t) * 2 + 1] = 0.0;
    for (int sp = 0; sp < ctx->full_splits; ++sp) {
        HIPCALL(ctx, hipMemcpy(buf.data(), ctx->d_full_part + (size_t)sp * nt * np, sizeof(double2) * buf.size(),
                               hipMemcpyDeviceToHost));
        for (int64_t t = 0; t < nt; ++t)
            for (int64_t j = 0; j < n; ++j) {
                R[(j * nt + t) * 2] += buf[(size_t)t * np + j].x;
                R[(j * nt + t) * 2 + 1] += buf[(size_t)t * np + j].y;
            }
    }
    return SCIVR_OK;
}

scivr_status scivr_read_spectrum_ref(scivr_ctx *ctx, int32_t ref, double *I_host, int64_t *n_good,
                                     int64_t *n_total)
{
    CHECK_CTX(ctx);
    if (ref < 0 || ref >= ctx->n_refs)
        return ctx_fail(ctx, SCIVR_EINVAL, "reference state %d of %d", ref, ctx->n_refs);
    HIPCALL(ctx, hipDeviceSynchronize());
    unsigned long long ng = 0;
    HIPCALL(ctx, hipMemcpy(&ng, ctx->d_ngood, sizeof ng, hipMemcpyDeviceToHost));
    if (n_good) *n_good = (int64_t)ng;
    if (n_total) *n_total = ctx->n_total;
    double gw = 0.0;
    HIPCALL(ctx, hipMemcpy(&gw, ctx->d_goodw + ref, sizeof gw, hipMemcpyDeviceToHost));
    if (I_host) {
        if (ng == 0 || !(gw > 0.0)) {
            for (int k = 0; k < ctx->n_energies; ++k) I_host[k] = 0.0;
        } else {
            HIPCALL(ctx, hipMemcpy(I_host, ctx->d_total + (int64_t)ref * ctx->n_energies,
                                   sizeof(double) * ctx->n_energies, hipMemcpyDeviceToHost));
            const double T = (double)ctx->n_steps * ctx->dt;
            const double scale = ctx->dt * ctx->dt / (2.0 * M_PI * T * gw);
            for (int k = 0; k < ctx->n_energies; ++k) I_host[k] *= scale;
        }
    }
    return ng == 0 ? SCIVR_ENOGOOD : SCIVR_OK;
}

scivr_status scivr_read_spectrum(scivr_ctx *ctx, double *I_host, int64_t *n_good, int64_t *n_total)
{
    return scivr_read_spectrum_ref(ctx, 0, I_host, n_good, n_total);
}

scivr_status scivr_set_references(scivr_ctx *ctx, int32_t n_extra, const double *p_eq, const double *q_eq)
{
    CHECK_CTX(ctx);
    if (n_extra < 0 || n_extra > MAX_REFS - 1 || (n_extra > 0 && (!p_eq || !q_eq)))
        return ctx_fail(ctx, SCIVR_EINVAL, "%d further reference states (0 to %d)", n_extra, MAX_REFS - 1);
    if (n_extra > 0 && ctx->precision != SCIVR_PRECISION_FP64)
        return ctx_fail(ctx, SCIVR_EUNSUPPORTED, "several reference states run in the FP64 form only");
    if (ctx->have_initial && !ctx->accumulated)
        return ctx_fail(ctx, SCIVR_ESTATE, "a batch is in flight (accumulate it first)");
    const int F = ctx->F;
    for (int64_t i = 0; i < (int64_t)n_extra * F; ++i)
        if (!std::isfinite(p_eq[i]) || !std::isfinite(q_eq[i]))
            return ctx_fail(ctx, SCIVR_EINVAL, "non-finite reference state");
    const int M = n_extra + 1;
    // the buffers whose size follows the number of reference states, allocated
    // before the old ones are released (on failure the context is unchanged)
    double2 *amp = nullptr;
    double *part_spec = nullptr, *part_contrib = nullptr, *total = nullptr, *goodw = nullptr;
    const bool ok = dalloc(&amp, (int64_t)ctx->nt_alloc * M * ctx->npad) == hipSuccess &&
                    dalloc(&part_spec, (int64_t)M * ctx->row_tiles * ctx->kpad) == hipSuccess &&
                    dalloc(&part_contrib, (int64_t)(ctx->kpad / 64) * M * ctx->npad) == hipSuccess &&
                    dalloc(&total, (int64_t)M * ctx->n_energies) == hipSuccess && dalloc(&goodw, M) == hipSuccess;
    if (!ok) {
        for (void *q : {(void *)amp, (void *)part_spec, (void *)part_contrib, (void *)total, (void *)goodw})
            if (q) (void)hipFree(q);
        (void)hipGetLastError();
        return ctx_fail(ctx, SCIVR_ENOMEM, "buffers for %d reference states", M);
    }
    HIPCALL(ctx, hipDeviceSynchronize());
    HIPCALL(ctx, launch_fill_zero((double *)amp, 2ll * ctx->nt_alloc * M * ctx->npad, nullptr));
    for (void *q : {(void *)ctx->d_amp, (void *)ctx->d_part_spec, (void *)ctx->d_part_contrib, (void *)ctx->d_total,
                    (void *)ctx->d_goodw})
        if (q) HIPCALL(ctx, hipFree(q));
    ctx->d_amp = amp;
    ctx->d_part_spec = part_spec;
    ctx->d_part_contrib = part_contrib;
    ctx->d_total = total;
    ctx->d_goodw = goodw;
    ctx->n_refs = M;
    ProblemDev &h = ctx->host_prob;
    h.n_refs = M;
    for (int m = 1; m < M; ++m)
        for (int i = 0; i < F; ++i) {
            h.ref_p[m][i] = p_eq[(m - 1) * F + i];
            h.ref_q[m][i] = q_eq[(m - 1) * F + i];
        }
    HIPCALL(ctx, hipMemcpy(ctx->d_prob, &h, sizeof h, hipMemcpyHostToDevice));
    // a fresh estimate: every reference state's totals, n_good and n_total
    HIPCALL(ctx, launch_fill_zero(ctx->d_total, (int64_t)M * ctx->n_energies, nullptr));
    HIPCALL(ctx, launch_fill_zero((double *)ctx->d_ngood, 1, nullptr));
    HIPCALL(ctx, launch_fill_zero(ctx->d_goodw, M, nullptr));
    HIPCALL(ctx, hipDeviceSynchronize());
    ctx->n_total = 0;
    ctx->have_initial = false;
    ctx->accumulated = false;
    ctx->contrib_valid = false;
    ctx->full_valid = false;
    ctx->steps_done = 0;
    return SCIVR_OK;
}

scivr_status scivr_read_totals(scivr_ctx *ctx, double *total, double *good_weight, int64_t *n_good,
                               int64_t *n_total)
{
    CHECK_CTX(ctx);
    HIPCALL(ctx, hipDeviceSynchronize());
    if (total)
        HIPCALL(ctx, hipMemcpy(total, ctx->d_total, sizeof(double) * ctx->n_energies, hipMemcpyDeviceToHost));
    if (good_weight) HIPCALL(ctx, hipMemcpy(good_weight, ctx->d_goodw, sizeof(double), hipMemcpyDeviceToHost));
    if (n_good) {
        unsigned long long ng = 0;
        HIPCALL(ctx, hipMemcpy(&ng, ctx->d_ngood, sizeof ng, hipMemcpyDeviceToHost));
        *n_good = (int64_t)ng;
    }
    if (n_total) *n_total = ctx->n_total;
    return SCIVR_OK;
}

scivr_status scivr_reset_spectrum(scivr_ctx *ctx, void *stream)
{
    CHECK_CTX(ctx);
    hipStream_t s = (hipStream_t)stream;
    HIPCALL(ctx, launch_fill_zero(ctx->d_total, (int64_t)ctx->n_refs * ctx->n_energies, s));
    HIPCALL(ctx, launch_fill_zero((double *)ctx->d_ngood, 1, s));
    HIPCALL(ctx, launch_fill_zero(ctx->d_goodw, ctx->n_refs, s));
    ctx->n_total = 0;
    return SCIVR_OK;
}

scivr_status scivr_batch_info(const scivr_ctx *ctx, int64_t *n_traj, int32_t *steps_done)
{
    if (!ctx) return SCIVR_EINVAL;
    if (n_traj) *n_traj = ctx->have_initial ? ctx->n_traj : 0;
    if (steps_done) *steps_done = ctx->steps_done;
    return SCIVR_OK;
}

static scivr_status copy_rows(scivr_ctx *ctx, double *dst, const double *src, int rows)
{
    const size_t row = (size_t)ctx->n_traj * sizeof(double), pitch = (size_t)ctx->npad * sizeof(double);
    HIPCALL(ctx, hipMemcpy2D(dst, row, src, pitch, row, rows, hipMemcpyDeviceToHost));
    return SCIVR_OK;
}

scivr_status scivr_read_initial(scivr_ctx *ctx, double *p0, double *q0, double *log_density)
{
    CHECK_CTX(ctx);
    if (!ctx->have_initial) return ctx_fail(ctx, SCIVR_ESTATE, "no initial conditions");
    HIPCALL(ctx, hipDeviceSynchronize());
    scivr_status st;
    if (p0 && (st = copy_rows(ctx, p0, ctx->d_p0, ctx->F)) != SCIVR_OK) return st;
    if (q0 && (st = copy_rows(ctx, q0, ctx->d_q0, ctx->F)) != SCIVR_OK) return st;
    if (log_density && (st = copy_rows(ctx, log_density, ctx->d_logrho, 1)) != SCIVR_OK) return st;
    return SCIVR_OK;
}

scivr_status scivr_read_state(scivr_ctx *ctx, double *p, double *q, double *S, double *phi, double *M, uint8_t *good,
                              double *detM, double *maxdev)
{
    CHECK_CTX(ctx);
    if (!ctx->have_initial || ctx->steps_done == 0) return ctx_fail(ctx, SCIVR_ESTATE, "no propagated state");
    HIPCALL(ctx, hipDeviceSynchronize());
    const int64_t n = ctx->n_traj, NP = ctx->npad;
    scivr_status st;
    if (p && (st = copy_rows(ctx, p, ctx->d_p, ctx->F)) != SCIVR_OK) return st;
    if (q && (st = copy_rows(ctx, q, ctx->d_q, ctx->F)) != SCIVR_OK) return st;
    if (S && (st = copy_rows(ctx, S, ctx->d_scal + SC_S * NP, 1)) != SCIVR_OK) return st;
    if (phi && (st = copy_rows(ctx, phi, ctx->d_scal + SC_PHI * NP, 1)) != SCIVR_OK) return st;
    if (detM && (st = copy_rows(ctx, detM, ctx->d_scal + SC_DETM * NP, 1)) != SCIVR_OK) return st;
    if (maxdev && (st = copy_rows(ctx, maxdev, ctx->d_scal + SC_MAXDEV * NP, 1)) != SCIVR_OK) return st;
    if (good) {
        std::vector<double> g(n);
        if ((st = copy_rows(ctx, g.data(), ctx->d_scal + SC_GOOD * NP, 1)) != SCIVR_OK) return st;
        for (int64_t j = 0; j < n; ++j) good[j] = g[j] != 0.0 ? 1 : 0;
    }
    if (M) {
        const int G = 2 * ctx->F;
        std::vector<double> buf((size_t)G * G * n);
        if ((st = copy_rows(ctx, buf.data(), ctx->d_M, G * G)) != SCIVR_OK) return st;
        for (int64_t j = 0; j < n; ++j)
            for (int e = 0; e < G * G; ++e) M[j * G * G + e] = buf[(size_t)e * n + j];
    }
    return SCIVR_OK;
}

scivr_status scivr_read_amplitudes(scivr_ctx *ctx, int64_t j0, int64_t count, double *amp)
{
    CHECK_CTX(ctx);
    if (!amp || j0 < 0 || count < 1 || j0 + count > ctx->n_traj)
        return ctx_fail(ctx, SCIVR_EINVAL, "amplitude range [%lld, %lld) outside the batch", (long long)j0,
                    (long long)(j0 + count));
    HIPCALL(ctx, hipDeviceSynchronize());
    const int nt = ctx->nt;
    if (ctx->precision != SCIVR_PRECISION_MIXED) {
        std::vector<double2> buf((size_t)nt * count);
        HIPCALL(ctx, hipMemcpy2D(buf.data(), count * sizeof(double2), ctx->d_amp + j0,
                                 ctx->n_refs * ctx->npad * sizeof(double2), count * sizeof(double2), nt,
                                 hipMemcpyDeviceToHost));
        for (int64_t j = 0; j < count; ++j)
            for (int c = 0; c < nt; ++c) {
                amp[(j * nt + c) * 2] = buf[(size_t)c * count + j].x;
                amp[(j * nt + c) * 2 + 1] = buf[(size_t)c * count + j].y;
            }
        return SCIVR_OK;
    }
    // mixed form: planes [nt16 / 8][npad][8] of FP16 hi/lo, scaled by 2^escale_j
    const int64_t nb = ctx->nt16 / 8, plane = (int64_t)ctx->nt16 * ctx->npad;
    std::vector<_Float16> buf((size_t)4 * nb * count * 8);
    for (int pl = 0; pl < 4; ++pl)
        HIPCALL(ctx, hipMemcpy2D(buf.data() + (size_t)pl * nb * count * 8, count * 8 * sizeof(_Float16),
                                 ctx->d_amp16 + pl * plane + j0 * 8, ctx->npad * 8 * sizeof(_Float16),
                                 count * 8 * sizeof(_Float16), nb, hipMemcpyDeviceToHost));
    std::vector<double> esc(count);
    HIPCALL(ctx, hipMemcpy(esc.data(), ctx->d_scal + SC_ESCALE * ctx->npad + j0, count * sizeof(double),
                           hipMemcpyDeviceToHost));
    auto at = [&](int pl, int64_t j, int c) {
        return (double)(float)buf[(((size_t)pl * nb + c / 8) * count + j) * 8 + c % 8];
    };
    for (int64_t j = 0; j < count; ++j)
        for (int c = 0; c < nt; ++c) {
            amp[(j * nt + c) * 2] = ldexp(at(0, j, c) + at(1, j, c), -(int)esc[j]);
            amp[(j * nt + c) * 2 + 1] = ldexp(at(2, j, c) + at(3, j, c), -(int)esc[j]);
        }
    return SCIVR_OK;
}

scivr_status scivr_read_contributions(scivr_ctx *ctx, double *c)
{
    CHECK_CTX(ctx);
    if (!c) return ctx_fail(ctx, SCIVR_EINVAL, "null output");
    if (!ctx->accumulated) return ctx_fail(ctx, SCIVR_ESTATE, "batch not accumulated");
    if (!ctx->contrib_valid)
        return ctx_fail(ctx, SCIVR_ESTATE, "the FFT accumulation produces no per-trajectory contributions");
    HIPCALL(ctx, hipDeviceSynchronize());
    HIPCALL(ctx, hipMemcpy(c, ctx->d_contrib, sizeof(double) * ctx->n_traj, hipMemcpyDeviceToHost));
    return SCIVR_OK;
}

scivr_status scivr_timing_enable(scivr_ctx *ctx, int32_t on)
{
    CHECK_CTX(ctx);
    HIPCALL(ctx, hipDeviceSynchronize());
    for (auto &e : ctx->events) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    ctx->events.clear();
    ctx->timing = on != 0;
    return SCIVR_OK;
}

scivr_status scivr_kernel_times(scivr_ctx *ctx, int64_t *launches, double *ms)
{
    CHECK_CTX(ctx);
    for (int k = 0; k < SCIVR_KERNEL_KINDS; ++k) {
        if (launches) launches[k] = 0;
        if (ms) ms[k] = 0.0;
    }
    for (auto &e : ctx->events) {
        HIPCALL(ctx, hipEventSynchronize(e.b));
        float t = 0.f;
        HIPCALL(ctx, hipEventElapsedTime(&t, e.a, e.b));
        if (launches) launches[e.kind] += 1;
        if (ms) ms[e.kind] += (double)t;
    }
    for (auto &e : ctx->events) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    ctx->events.clear();
    return SCIVR_OK;
}

}  // extern "C"
