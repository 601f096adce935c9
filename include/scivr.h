/*
 * scivr.h -- C ABI of the MI355X (gfx950) TA-SC-IVR power-spectrum library.
 *
 * The library computes the time-averaged semiclassical initial value
 * representation spectral density with the separable prefactor
 * approximation (Tamascelli, Dambrosio, Conte, Ceotto, "Graphics Processing
 * Units Accelerated Semiclassical Initial Value Representation Molecular
 * Dynamics", Eq. (10)) by the Monte Carlo estimator of Eq. (11):
 *
 *   I(E_k) = dt^2 / (2 pi T n_good) * sum_j good_j w_j
 *            | sum_{c=0}^{n_steps} <chi|p_j(c dt), q_j(c dt)> e^{i (S_j + E_k c dt + phi_j)} |^2
 *
 * with T = n_steps dt, w_j = 1 / ((2 pi)^F rho(p0_j, q0_j)) for initial
 * points drawn from a density rho (Husimi sampling of the reference coherent
 * state chi gives w_j = 1/|<p0_j,q0_j|chi>|^2), the energy grid
 * E_k = e_min + k (e_max - e_min)/(K - 1) of the section "Monte-Carlo SC-IVR
 * algorithm", and good_j = 0 for a trajectory whose |det(M)^2 - 1| exceeded
 * det_tol at a checked step (the accuracy monitor after Eq. (5)).
 *
 * Units: atomic units, hbar = 1, mass-weighted coordinates.  The potential is
 *   V(q) = sum_i [k_i q_i^2/2 + D_i (1 - exp(-a_i q_i))^2] + sum_{i<j} lambda_ij q_i^2 q_j^2.
 *
 * Conventions common to every call:
 *  - Return values are scivr_status codes (<= 0).  No C++ exception, abort or
 *    exit crosses the ABI.  After an error, scivr_last_error(ctx) describes it.
 *  - A device error (a failed HIP call) is sticky: every later call on that
 *    context returns SCIVR_EDEVICE.
 *  - `stream` is a hipStream_t passed as void*; NULL means the legacy default
 *    stream.  Calls taking a stream are asynchronous on it unless stated.
 *  - One context per host thread at a time; a context is not thread-safe.
 *  - Phase-space arrays are structure-of-arrays [F][n] (all trajectories'
 *    values of degree of freedom 0, then of degree of freedom 1, ...), the
 *    coalesced layout described in the section "GP-GPU Implementation".
 */
#ifndef SCIVR_H
#define SCIVR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SCIVR_ABI_VERSION 2
/* Largest number of degrees of freedom of the FP64 trajectory kernel. */
#define SCIVR_F_MAX 32

typedef int32_t scivr_status;
#define SCIVR_OK 0
#define SCIVR_EINVAL (-1)       /* invalid argument */
#define SCIVR_ENOMEM (-2)       /* device or host allocation failed */
#define SCIVR_EDEVICE (-3)      /* a HIP call failed (sticky) */
#define SCIVR_ESTATE (-4)       /* call out of order (e.g. propagate before initial conditions) */
#define SCIVR_ENOGOOD (-5)      /* no good trajectory accumulated yet; spectrum zero-filled */
#define SCIVR_EUNSUPPORTED (-6) /* valid request the library does not implement */

#define SCIVR_PRECISION_FP64 0  /* every step in FP64 */
#define SCIVR_PRECISION_MIXED 1 /* FP32 trajectory and Kahan action, FP64 monodromy/prefactor/branch, split-FP16 Fourier GEMM */

#define SCIVR_MEM_HOST 0
#define SCIVR_MEM_DEVICE 1

/*
 * Problem statement.  All arrays are read during scivr_create and copied;
 * the caller keeps ownership.  `lambda` is F x F row-major and symmetric;
 * only the entries i < j are read (the diagonal is ignored).
 */
typedef struct scivr_problem {
    int32_t F;               /* degrees of freedom, 1 <= F <= SCIVR_F_MAX */
    const double *k_harm;    /* [F] harmonic coefficients k_i */
    const double *morse_D;   /* [F] Morse depths D_i */
    const double *morse_a;   /* [F] Morse range parameters a_i */
    const double *lambda;    /* [F*F] quartic couplings lambda_ij */
    const double *gamma;     /* [F] coherent-state widths gamma_i > 0 (Eq. (3)) */
    const double *p_eq;      /* [F] reference state chi = |p_eq, q_eq> */
    const double *q_eq;      /* [F] */
    double dt;               /* time step (> 0) */
    int32_t n_steps;         /* steps per trajectory (>= 1); T = n_steps dt */
    double e_min, e_max;     /* energy window, e_max > e_min */
    int32_t n_energies;      /* K >= 2 grid points, both ends included */
    double det_tol;          /* stability threshold on |det(M)^2 - 1| (paper: 1e-6) */
    int32_t check_every;     /* check det(M) every this many steps (and at the last step); 1 = every step */
    int32_t precision;       /* SCIVR_PRECISION_* */
    int64_t max_traj;        /* batch capacity: largest n_traj of one batch (>= 1) */
} scivr_problem;

typedef struct scivr_ctx scivr_ctx;

/* Version of this ABI (SCIVR_ABI_VERSION of the built library). */
int32_t scivr_abi_version(void);

/*
 * Validate the problem, select `device`, copy the parameters and allocate
 * every device buffer of a batch of max_traj trajectories (initial
 * conditions, state, the amplitude matrix of n_steps+1 samples per
 * trajectory, spectrum accumulators; FP64: complex [n_steps+1][max_traj] and
 * the time x energy phase table; MIXED: four FP16 planes hi/lo of re/im in
 * the time-blocked layout [t/8][max_traj][t%8]).
 * Errors: SCIVR_EINVAL (F out of range, n_steps < 1, n_energies < 2,
 * e_max <= e_min, gamma_i <= 0, dt <= 0, check_every < 1, max_traj < 1, a
 * non-finite parameter, NULL pointer, precision not FP64/MIXED),
 * SCIVR_ENOMEM, SCIVR_EDEVICE.  On error *out is NULL and
 * nothing is leaked.
 */
scivr_status scivr_create(const scivr_problem *p, int32_t device, scivr_ctx **out);

/* Free every resource of the context (synchronises its device first). NULL is ignored. */
void scivr_destroy(scivr_ctx *ctx);

/* Message of the last error on this context ("" if none).  Valid until the next call. */
const char *scivr_last_error(const scivr_ctx *ctx);

/*
 * Husimi sampling of chi (section "Monte-Carlo SC-IVR algorithm"): for
 * trajectory j of the batch, global index g = first_index + j, the 2F
 * standard normals are Box-Muller pairs of the uniforms of Philox4x64-10
 * blocks with key (seed, 0) and counter (g, b, 0, 0), b = 0, 1, ...; normal
 * 2i is xi_i and normal 2i+1 is eta_i, and
 *   q0_i = q_eq,i + xi_i / sqrt(gamma_i),  p0_i = p_eq,i + eta_i sqrt(gamma_i),
 *   ln rho = -F ln(2 pi) - sum_i (xi_i^2 + eta_i^2)/2.
 * Sets the batch size to n_traj (1 <= n_traj <= max_traj) and resets the
 * propagation state.  Disjoint first_index ranges give independent batches.
 */
scivr_status scivr_sample_husimi(scivr_ctx *ctx, uint64_t seed, uint64_t first_index, int64_t n_traj,
                                 void *stream);

/*
 * Use caller-given initial conditions: p0, q0 are [F][n_traj], log_density
 * [n_traj] is ln rho(p0, q0) of the density they were drawn from (it sets
 * the weight w_j = exp(-ln rho_j - F ln 2 pi)).  mem_kind says whether the
 * pointers are host or device memory; device pointers are read on `stream`
 * and must stay valid until that work completes.  Sets the batch size and
 * resets the propagation state.
 */
scivr_status scivr_set_initial(scivr_ctx *ctx, int64_t n_traj, const double *p0, const double *q0,
                               const double *log_density, int32_t mem_kind, void *stream);

/*
 * Integrate the batch over steps [step_begin, step_end) (0 <= step_begin <
 * step_end <= n_steps): the fourth-order symplectic triple jump with three
 * Hessian evaluations per step, the action, the 2F x 2F monodromy matrix, the
 * continuous phase of the Herman-Kluk prefactor (Eq. (5)), the stability
 * monitor, and the amplitude of every time sample.  Calls must continue
 * where the last one stopped (step_begin == steps done), else SCIVR_ESTATE;
 * SCIVR_ESTATE also without initial conditions.
 */
scivr_status scivr_propagate(scivr_ctx *ctx, int32_t step_begin, int32_t step_end, void *stream);

/*
 * Stop integrating a trajectory at the step where the stability monitor flags
 * it (enable != 0), as the sequential code of the paper's implementation
 * section interrupts such a trajectory, instead of running it to T as its GPU
 * design does.  A flagged trajectory contributes nothing to the estimate, so
 * the spectra, the good counts and the contributions are those of the full
 * run, bit for bit; its amplitudes after the flag stay zero.  What changes is
 * scivr_read_state for flagged trajectories: their p, q, S, phi, M and the
 * largest |det(M)^2 - 1| are those of the step at which they were flagged.
 * It takes effect in the kernel for F > 16, where one wave holds one
 * trajectory and stopping it costs no divergence; for F <= 16 (several
 * trajectories per wave) the setting is kept and has no effect.  Off by
 * default; applies to later scivr_propagate calls.
 */
scivr_status scivr_set_stop_flagged(scivr_ctx *ctx, int32_t enable);

/*
 * After all n_steps are done: the Fourier sums A_jk = sum_c amp_jc e^{i E_k c dt}
 * of the batch, and ADD sum_j good_j w_j |A_jk|^2 and the batch's n_good
 * and n_traj into the context's running totals (so several batches form one
 * estimate).  Also stores each trajectory's contribution w_j sum_k |A_jk|^2.
 * SCIVR_ESTATE if the batch is not fully propagated or was already added.
 */
scivr_status scivr_accumulate_spectrum(scivr_ctx *ctx, void *stream);

/*
 * The same addition to the running totals as scivr_accumulate_spectrum, by
 * the exact autocorrelation form of the Fourier sums (Eq. (11)): for each
 * trajectory, |sum_c amp_jc e^{i E c dt}|^2 is a trigonometric polynomial in
 * E dt whose coefficients are the autocorrelation of amp_j, obtained from a
 * zero-padded FFT of length L = 2^ceil(log2(2 n_steps)); the weighted
 * autocorrelation summed over the batch is then evaluated on the energy grid.
 * The spectrum agrees with scivr_accumulate_spectrum's to rounding.  No
 * per-trajectory contributions are produced: scivr_read_contributions and
 * the flow's training on this batch then return SCIVR_ESTATE.  With several
 * reference states (scivr_set_references) each state's spectrum is added, one
 * transform pass per state.  At most 4096 steps (L <= 8192), else
 * SCIVR_EUNSUPPORTED.  The first call allocates about
 * 17 MB of scratch on the context's device (SCIVR_ENOMEM if that fails).
 * Other errors as scivr_accumulate_spectrum.
 */
scivr_status scivr_accumulate_spectrum_fft(scivr_ctx *ctx, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * addition as scivr_accumulate_spectrum_fft, with bit-identical results, that
 * allocates nothing.  Its scratch is a static device array of
 * SCIVR_FFT_STATIC_SCRATCH_BYTES (about 16.1 MiB) of which each device the
 * library runs on holds one copy until the process ends; its device address
 * is looked up when a context is created on that device.  Every call on one
 * device shares that copy, and nothing in it needs to start at zero (each
 * call writes every element it reads), so calls that overlap on one device
 * (from several host threads or streams) race and give wrong spectra: order
 * them on one stream.  Limit: at most 4096 steps (L <= 8192), else
 * SCIVR_EUNSUPPORTED, as the allocating form.  No timing events are recorded.
 * Other errors as scivr_accumulate_spectrum_fft.
 */
#define SCIVR_FFT_STATIC_SCRATCH_BYTES 16912896
scivr_status scivr_accumulate_spectrum_fft_noalloc(scivr_ctx *ctx, void *stream);

/*
 * The same addition to the running totals without the separable
 * approximation: the double-time form of Eq. (9), in which every segment
 * [t1, t2] of a trajectory carries the Herman-Kluk prefactor C_{t2}(z(t1)) of
 * the trajectory started at z(t1) (sqrt(det A) of Eq. (5) from the segment's
 * own tangent map, on the branch continuous in t2 from C = 1 at t2 = t1).  On
 * the time samples of Eq. (11), with the diagonal t1 = t2 weighted 1/2,
 *   total_k += sum_j good_j w_j 2 Re sum_tau R_j(tau) e^{i E_k tau dt},
 *   R_j(tau) = sum_c omega C_j(c, c + tau) a_j(c + tau) conj(a_j(c)),
 *   a_j(c) = <chi|z_j(c dt)> e^{i S_j(c dt)},
 * which equals scivr_accumulate_spectrum's addition when the prefactor is
 * replaced by exp(i (phi(t2) - phi(t1))).  The trajectories' own stability
 * flags (from the propagation) select the good ones; segments are not
 * monitored.  Cost: about n_steps^2 / 2 segment steps per trajectory, and
 * with several reference states (scivr_set_references) one such pass per
 * state, each adding its own spectrum (scivr_read_lags then returns chi's lag
 * sums).  FP64 form and F <= 16 only (else SCIVR_EUNSUPPORTED).  The first call allocates
 * a lag buffer of about 16 * n_t * max(max_traj, 4096) bytes (SCIVR_ENOMEM if
 * that fails).  Other errors as scivr_accumulate_spectrum.
 */
scivr_status scivr_accumulate_spectrum_full(scivr_ctx *ctx, void *stream);

/*
 * After scivr_accumulate_spectrum_full: the batch's lag sums R_j(tau) as
 * complex pairs, R [n][n_steps + 1][2] (caller-owned host memory).
 * Synchronises.  SCIVR_ESTATE if the batch's last accumulation was another form.
 */
scivr_status scivr_read_lags(scivr_ctx *ctx, double *R);

/*
 * Synchronise and write I_k = dt^2/(2 pi T G) * total_k to I_host[K]
 * (caller-owned), and the running n_good and n_total.  G is the good count of
 * Eq. (11) estimated for the sampling density rho of each batch,
 * G = sum_j good_j H(z_j) / rho(z_j) with H the Husimi density of the
 * reference state: exactly n_good for Husimi batches, the importance-weighted
 * count for batches drawn from another density (the learned proposal).  If
 * n_good is 0 the spectrum is zero-filled and SCIVR_ENOGOOD is returned.  Any
 * output pointer may be NULL.
 */
scivr_status scivr_read_spectrum(scivr_ctx *ctx, double *I_host, int64_t *n_good, int64_t *n_total);

/*
 * Several reference states on one trajectory batch (the paper's runs with
 * different coherent-state combinations, Results and discussion): besides
 * the problem's chi (reference 0), n_extra more coherent states of the same
 * widths, centred at p_eq[m][F], q_eq[m][F] (row-major host arrays, read and
 * copied).  Every later batch then feeds one spectrum per reference state
 * from the same trajectories: the amplitudes carry <chi_m|z_t>, the weights
 * w_j = 1/((2 pi)^F rho(z_j)) are shared, and reference m's good count is its
 * own Husimi mass of the batch, sum_j good_j H_m(z_j) / rho(z_j) (Eq. (11)'s
 * n_good for points not drawn from H_m).  The Fourier step becomes one product
 * with a right-hand side per reference state (the phase matrix is shared).
 * Resets the running totals and discards the current batch.  0 <= n_extra
 * <= 7 (SCIVR_EINVAL otherwise); FP64 form only (SCIVR_EUNSUPPORTED for the
 * mixed form); SCIVR_ESTATE while a propagated batch awaits accumulation;
 * SCIVR_ENOMEM if the amplitude buffer for the n_extra + 1 states cannot be
 * allocated (the context is then unchanged).  Per-trajectory contributions
 * (scivr_read_contributions) and amplitudes (scivr_read_amplitudes) are
 * reference 0's.
 */
scivr_status scivr_set_references(scivr_ctx *ctx, int32_t n_extra, const double *p_eq, const double *q_eq);

/*
 * scivr_read_spectrum for reference state `ref` (0 = the problem's chi):
 * I_k = dt^2/(2 pi T G_ref) total_ref,k with G_ref that state's good count.
 * SCIVR_EINVAL for a reference outside [0, n_extra].
 */
scivr_status scivr_read_spectrum_ref(scivr_ctx *ctx, int32_t ref, double *I_host, int64_t *n_good,
                                     int64_t *n_total);

/*
 * Synchronise and write the raw running sums: total[K] = sum over accumulated
 * batches of sum_j good_j w_j |A_j(E_k)|^2 (or its double-time form), the good
 * weight G of scivr_read_spectrum, n_good and n_total.  Several contexts (or
 * shards of one estimate on several devices) combine by adding these and
 * normalising once as scivr_read_spectrum does.  Any output pointer may be NULL.
 */
scivr_status scivr_read_totals(scivr_ctx *ctx, double *total, double *good_weight, int64_t *n_good,
                               int64_t *n_total);

/* Zero the running spectrum totals and counts (asynchronous on `stream`). */
scivr_status scivr_reset_spectrum(scivr_ctx *ctx, void *stream);

/* ---- inspection (parity checks and diagnostics); all synchronise and write host memory ---- */

/* Current batch size (0 before initial conditions) and steps done. */
scivr_status scivr_batch_info(const scivr_ctx *ctx, int64_t *n_traj, int32_t *steps_done);

/* Initial conditions of the batch: p0, q0 [F][n], log_density [n]. Any may be NULL. */
scivr_status scivr_read_initial(scivr_ctx *ctx, double *p0, double *q0, double *log_density);

/*
 * State after the last propagate call: p, q [F][n]; S, phi, detM (det M at
 * the last checked step), maxdev (max |det(M)^2 - 1| over checked steps) [n];
 * M [n][2F][2F] row-major with rows and columns ordered (p, q), i.e.
 * M[j][r][c] = d(p,q)_r(t) / d(p0,q0)_c; good [n] (1 or 0).  Any may be NULL.
 */
scivr_status scivr_read_state(scivr_ctx *ctx, double *p, double *q, double *S, double *phi, double *M,
                              uint8_t *good, double *detM, double *maxdev);

/* Amplitudes of trajectories [j0, j0 + count) at every time sample: amp[count][n_steps+1][2] (re, im). */
scivr_status scivr_read_amplitudes(scivr_ctx *ctx, int64_t j0, int64_t count, double *amp);

/* Per-trajectory contributions w_j sum_k |A_jk|^2 (0 for bad) of the last accumulated batch: c[n]. */
scivr_status scivr_read_contributions(scivr_ctx *ctx, double *c);

/*
 * Kernel timing.  While enabled, every kernel launch of the context is
 * bracketed by HIP events on its stream.  scivr_kernel_times synchronises
 * and returns, per kernel kind, the number of launches and their summed
 * duration in milliseconds since the last reset (enable resets).  Kinds:
 * 0 = sample, 1 = trajectory, 2 = Fourier GEMM, 3 = spectrum reduction,
 * 4 = flow proposal (training and sampling).
 */
#define SCIVR_KERNEL_KINDS 5
scivr_status scivr_timing_enable(scivr_ctx *ctx, int32_t on);
scivr_status scivr_kernel_times(scivr_ctx *ctx, int64_t *launches /*[SCIVR_KERNEL_KINDS]*/,
                                double *ms /*[SCIVR_KERNEL_KINDS]*/);

/* ---- learned importance-sampling proposal ----
 *
 * Not part of the paper's method: the paper draws initial conditions from
 * the Husimi density of chi and weights trajectory j by 1/|<z_j|chi>|^2 =
 * 1/((2 pi)^F rho_j) (section "Monte-Carlo SC-IVR algorithm", Eq. (11)).
 * Any other sampling density keeps the estimator unbiased with the same
 * weight formula, rho being that density; scivr_set_initial and
 * scivr_flow_sample pass it as log_density.
 *
 * The proposal is an affine-coupling normalising flow over the whitened
 * coordinates x = (xi, eta), xi_i = sqrt(gamma_i)(q_i - q_eq,i), eta_i =
 * (p_i - p_eq,i)/sqrt(gamma_i), in which the Husimi density is N(0, I) and
 * which have unit Jacobian.  n_layers coupling layers: layer l conditions on
 * xi (l even) or eta (l odd) and maps the other half b to b exp(s) + t, with
 * (s_raw, t) from a tanh MLP F -> width -> width -> 2F and s = 2 tanh(s_raw/2).
 * Parameters (FP32, one flat array, per layer): W1 [width][F], b1 [width],
 * W2 [width][width], b2 [width], W3 [2F][width], b3 [2F]; W3 rows 0..F-1
 * give s_raw and F..2F-1 give t.
 *
 * A flow belongs to one context (it reads the context's problem and writes
 * its initial conditions); destroy it before the context.
 */
typedef struct scivr_flow scivr_flow;

/*
 * New flow with W1, W2 entries N(0,1)/sqrt(fan-in) from Philox4x64-10 (key
 * (seed, 0), counter (parameter index, 0, 2, 0)) and zero biases and output
 * layer: the initial flow is the identity, its density the Husimi density.
 * Errors: SCIVR_EINVAL (n_layers outside [1, 64], width outside [1, 1024]),
 * SCIVR_ENOMEM, SCIVR_EDEVICE.  On error *out is NULL.
 */
scivr_status scivr_flow_create(scivr_ctx *ctx, int32_t n_layers, int32_t width, uint64_t seed, scivr_flow **out);

/* Free the flow (synchronises its device first).  NULL is ignored. */
void scivr_flow_destroy(scivr_flow *flow);

/* Number of FP32 parameters (-1 for NULL). */
int64_t scivr_flow_param_count(const scivr_flow *flow);

/* Replace the parameters (count must equal the parameter count) and reset the Adam state. */
scivr_status scivr_flow_set_params(scivr_flow *flow, const float *params, int64_t count, int32_t mem_kind,
                                   void *stream);

/* Synchronise and copy the parameters to host memory. */
scivr_status scivr_flow_get_params(scivr_flow *flow, float *params, int64_t count);

/*
 * Weighted maximum likelihood: points (p0, q0 [F][n]) drawn from some
 * density r, with contributions c[n] = w_j sum_k |A_jk|^2 (w_j = 1/((2 pi)^F
 * r_j), as scivr_read_contributions returns them), are proportional to the
 * ideal sampling density divided by r; minimise L = -sum c_j log q(x_j) /
 * sum c_j with Adam (lr, beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected),
 * in FP32, over contiguous mini-batches [b batch, (b+1) batch) of the data in
 * order, `epochs` times; a mini-batch with sum c = 0 is skipped.  The Adam
 * state carries over between calls.  mem_kind: host or device arrays.
 * *last_loss (may be NULL) receives L of the last mini-batch.  Synchronises.
 */
scivr_status scivr_flow_train(scivr_flow *flow, int64_t n, const double *p0, const double *q0, const double *c,
                              int32_t mem_kind, int32_t epochs, int32_t batch, float lr, void *stream,
                              double *last_loss);

/* As scivr_flow_train on the context's current batch: its initial conditions
 * and the contributions of its last accumulate call (SCIVR_ESTATE if none). */
scivr_status scivr_flow_train_on_batch(scivr_flow *flow, int32_t epochs, int32_t batch, float lr, void *stream,
                                       double *last_loss);

/* One full-batch evaluation of L and dL/dparams (FP32) without a step; loss
 * and grad [param count] are host outputs, either may be NULL.  Synchronises. */
scivr_status scivr_flow_loss_grad(scivr_flow *flow, int64_t n, const double *p0, const double *q0, const double *c,
                                  int32_t mem_kind, double *loss, float *grad);

/*
 * log q(p0, q0) of the flow alone (FP32 networks, or BF16 matrix-core
 * networks as the sampler uses when use_bf16 != 0): logq [n] and, if u is
 * not NULL, the latent points u [n][2F] (FP32), both host outputs.
 * Synchronises.
 */
scivr_status scivr_flow_log_density(scivr_flow *flow, int64_t n, const double *p0, const double *q0,
                                    int32_t mem_kind, int32_t use_bf16, double *logq, float *u);

/*
 * Fill the context's initial conditions with n (<= max_traj) points of the
 * defensive mixture alpha N + (1 - alpha) q: point j (global index g =
 * first_index + j) draws its 2F normals exactly as scivr_sample_husimi does
 * and one uniform from counter (g, 0, 1, 0); if the uniform is below alpha
 * the point is those normals (the Husimi draw), otherwise their image under
 * the flow (BF16 networks on the matrix cores, FP32 affine steps).
 * log_density is ln(alpha N(x) + (1 - alpha) q(x)).  Whether the mixture is
 * used is decided before the batch is drawn, on a pilot draw of
 * min(n, SCIVR_FLOW_PILOT_SIZE) mixture points from the disjoint indices
 * first_index + SCIVR_FLOW_PILOT_OFFSET + j of the same seed: the effective
 * sample size of their ratios N(x)/density(x), divided by their count, goes
 * to *ess_frac; if it is below min_ess_frac the batch is drawn from the
 * Husimi density with the same seed and indices and *used_flow is 0 (else 1).
 * The choice of estimator therefore does not depend on the batch's own
 * points, and either estimator is unbiased.  alpha = 1 gives exactly
 * scivr_sample_husimi.  Resets the propagation state.  Synchronises.
 */
#define SCIVR_FLOW_PILOT_SIZE 4096
#define SCIVR_FLOW_PILOT_OFFSET (1ull << 62)
scivr_status scivr_flow_sample(scivr_flow *flow, uint64_t seed, uint64_t first_index, int64_t n, double alpha,
                               double min_ess_frac, double *ess_frac, int32_t *used_flow, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SCIVR_H */
