// Host-side state of a context, shared by the translation units that
// implement the C ABI (context, batch and flow entry points).
#pragma once

#include <stdarg.h>

#include <string>
#include <vector>

#include "scivr.h"
#include "scivr_internal.h"

struct EventPair {
    hipEvent_t a, b;
    int kind;
};

struct scivr_ctx {
    int device = 0;
    int F = 0;
    int32_t n_steps = 0, n_energies = 0, check_every = 1, precision = 0;
    double dt = 0, e_min = 0, e_max = 0, det_tol = 0;
    int64_t max_traj = 0, npad = 0;
    int32_t nt = 0, nt_pad = 0, nt_alloc = 0, kpad = 0, row_tiles = 0, col_tiles = 0;

    scivr::ProblemDev host_prob{};
    scivr::ProblemDev *d_prob = nullptr;
    double *d_p0 = nullptr, *d_q0 = nullptr, *d_logrho = nullptr;
    double *d_p = nullptr, *d_q = nullptr, *d_scal = nullptr, *d_M = nullptr;
    double *d_spart = nullptr;      // per-mode parts of the action between launches [F][npad]
    double2 *d_amp = nullptr, *d_phase = nullptr;  // FP64 form
    _Float16 *d_amp16 = nullptr;                    // mixed form: 4 planes [nt16 / 8][npad][8]
    int32_t nt16 = 0;                               // time samples per plane (multiple of 32)
    double *d_weight = nullptr, *d_part_spec = nullptr, *d_part_contrib = nullptr, *d_contrib = nullptr;
    double *d_total = nullptr;
    unsigned long long *d_ngood = nullptr;
    double *d_goodw = nullptr;      // running sum of good_j r_j (r_j = Husimi / sampling density)
    double *d_goodw_row = nullptr;  // good_j r_j of the current batch [npad]
    bool husimi_batch = false;      // the batch was drawn by the Husimi sampler (r_j = 1 exactly)
    int32_t stop_flagged = 0;       // scivr_set_stop_flagged
    int32_t n_refs = 1;             // reference states of the spectra (d_amp [t][ref][npad], d_total [ref][K])

    int64_t n_traj = 0;      // current batch size
    int32_t steps_done = 0;
    bool have_initial = false, accumulated = false;
    bool contrib_valid = false;  // the last accumulation produced per-trajectory contributions (the GEMM does)
    // FFT-autocorrelation accumulation: scratch allocated on first use, and
    // the device address of the device's static scratch (no-allocation form)
    void *d_static_scratch = nullptr;
    double *d_fft_part = nullptr, *d_fft_S = nullptr;
    double2 *d_fft_pcorr = nullptr, *d_fft_corr = nullptr, *d_fft_C = nullptr;
    // double-time form of Eq. (9): per-split lag sums and the weighted lags, on first use
    double2 *d_full_part = nullptr, *d_full_C = nullptr;
    int32_t full_splits = 0;
    bool full_valid = false;  // the last accumulation was the double-time form (its lags can be read)
    int64_t n_total = 0;     // trajectories accumulated so far

    bool device_error = false;
    std::string err;

    bool timing = false;
    std::vector<EventPair> events;
};

namespace scivr {

// Record the message and the status on the context (sticky for device errors).
scivr_status ctx_fail(scivr_ctx *c, scivr_status st, const char *fmt, ...) __attribute__((format(printf, 3, 4)));

// Bracket a launch with timing events when enabled.
struct Timed {
    scivr_ctx *c;
    hipStream_t s;
    int kind;
    hipEvent_t a = nullptr, b = nullptr;
    Timed(scivr_ctx *c_, hipStream_t s_, int k) : c(c_), s(s_), kind(k)
    {
        if (c && c->timing) {
            if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
                a = b = nullptr;
                return;
            }
            (void)hipEventRecord(a, s);
        }
    }
    void done()
    {
        if (a && b) {
            (void)hipEventRecord(b, s);
            c->events.push_back({a, b, kind});
            a = b = nullptr;
        }
    }
    ~Timed()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

}  // namespace scivr

#define HIPCALL(ctx, expr)                                                                                  \
    do {                                                                                                    \
        hipError_t e_ = (expr);                                                                             \
        if (e_ != hipSuccess)                                                                               \
            return scivr::ctx_fail((ctx), SCIVR_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                        __LINE__);                                                                          \
    } while (0)

#define CHECK_CTX(ctx)                                                                        \
    do {                                                                                      \
        if (!(ctx)) return SCIVR_EINVAL;                                                      \
        if ((ctx)->device_error) return SCIVR_EDEVICE;                                        \
        hipError_t e_ = hipSetDevice((ctx)->device);                                          \
        if (e_ != hipSuccess) return scivr::ctx_fail((ctx), SCIVR_EDEVICE, "hipSetDevice: %s", hipGetErrorString(e_)); \
    } while (0)

