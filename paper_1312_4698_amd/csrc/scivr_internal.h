// Internal declarations shared by the HIP sources of libscivr (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "scivr_math.h"

namespace scivr {

constexpr int FMAX = 32;
// Reference states whose spectra one batch can feed (the problem's chi and
// up to MAX_REFS - 1 more of the same widths).
constexpr int MAX_REFS = 8;

// Tile sizes of the Fourier GEMM: a workgroup covers GEMM_BM trajectories x
// GEMM_BN energies; the time axis is consumed GEMM_BK samples per MFMA step.
constexpr int GEMM_BM = 128;
constexpr int GEMM_BN = 128;
constexpr int GEMM_BK = 4;

// Scalar per-trajectory state rows, structure of arrays [NSCAL][npad].
enum ScalarRow {
    SC_S = 0, SC_SCOMP, SC_THETA, SC_PREV_RE, SC_PREV_IM, SC_PHI, SC_GOOD, SC_DETM, SC_MAXDEV, SC_ESCALE, NSCAL
};

// Trajectory-independent constants, read with uniform (scalar) loads.
struct ProblemDev {
    double k[FMAX], D[FMAX], a[FMAX];
    double gamma[FMAX], sqrt_gamma[FMAX], inv_sqrt_gamma[FMAX], inv4gamma[FMAX];
    double p_eq[FMAX], q_eq[FMAX];
    double lam[FMAX * FMAX];  // symmetric, zero diagonal, row stride FMAX
    double hd[4];             // drift lengths d_s * dt
    double hc[3];             // kick lengths c_s * dt
    double dt, sum_gamma, det_tol;
    double cos_gdt, sin_gdt;  // exp(i dt sum gamma)
    double F_log_2pi;         // F ln(2 pi)
    double e_min, e_max;
    MathConsts mc;            // coefficients of the kernel's exp, sincos, atan2
    int32_t n_refs;           // reference states of the batch's spectra (1: the problem's chi)
    double ref_p[MAX_REFS][FMAX], ref_q[MAX_REFS][FMAX];  // their centres; ref 0 = (p_eq, q_eq)
};

struct TrajArgs {
    const ProblemDev *prob;
    const double *p0, *q0;  // [F][npad]
    double *p, *q;          // [F][npad] state
    double *scal;           // [NSCAL][npad]
    double *spart;          // [F][npad] per-mode parts of the action, kept between launches
                            // where the small-F kernel splits the action over its lanes
    double *Mst;            // [(2F)^2][npad], element r*2F + c
    double2 *amp;           // FP64 form: [nt_alloc][n_refs][npad]
    _Float16 *amp16;        // mixed form: 4 planes [nt_alloc / 8][npad][8]
    int64_t plane;          // elements per plane of amp16
    int64_t n, npad;
    int32_t step_begin, step_end, n_steps, check_every;
    int32_t n_refs;         // FP64 form: amplitudes for each reference state
    int32_t stop_flagged;   // stop a trajectory once flagged (F > 16 kernel)
};

// Time samples per FP16 MFMA k-step of the mixed-form Fourier GEMM.
constexpr int GEMM16_BK = 32;

struct GemmF16Args {
    const _Float16 *amp16;  // planes re_hi, re_lo, im_hi, im_lo: [nt_alloc / 8][npad][8]
    int64_t plane;
    const double *weight;
    double *part_spec;
    double *part_contrib;
    int64_t npad;
    int32_t kpad, nt_pad, K;
    int32_t row_tiles, col_tiles;
    double e_min, de, dt;
};

// FFT-autocorrelation form of the Fourier accumulation: sequences of length
// L = 2^lg >= 2 (n_t - 1), lg <= FFT_MAX_LOG2 (the whole sequence in LDS).
constexpr int FFT_MAX_LOG2 = 13;
constexpr int FFT_NWG = 256;  // workgroups of the per-trajectory transform (one per CU)
struct FftArgs {
    const double2 *amp;      // FP64 form: [nt_alloc][npad]
    const _Float16 *amp16;   // mixed form: 4 planes [nt16 / 8][npad][8]
    int64_t plane;
    const double *weight;    // [npad] w_j good_j (2^-2 escale_j in the mixed form)
    double *part;            // [nwg][L] per-workgroup sums of w_j |X_j[m]|^2, bit-reversed bins
    double2 *part_corr;      // [nwg] per-workgroup sums of the folded lag
    int64_t n, npad;
    int32_t nt, nwg, fold;   // fold: L == 2 (n_t - 1), lag L/2 summed directly
};
int fft_log2_length(int nt);
hipError_t launch_fourier_fft(const FftArgs &a, bool mixed, double e_min, double de, double dt, int K, double *S,
                              double2 *corr, double2 *C, double *total, hipStream_t st);

// Double-time form of Eq. (9) (each segment's own Herman-Kluk prefactor).
struct FullArgs {
    const ProblemDev *prob;
    const double *p0, *q0;  // [F][npad] initial conditions of the batch
    double2 *part;          // [splits][nt][npad] per-split lag sums R_j(tau)
    int64_t n, npad;
    int32_t nt, n_steps, splits;
    int32_t ref;            // reference state whose overlaps form the lag sums (0 = chi)
};
hipError_t launch_ta_full(int F, const FullArgs &a, hipStream_t s);
hipError_t launch_ta_lags(const FullArgs &a, const double *weight, double2 *C, hipStream_t s);
hipError_t launch_fft_spectrum(const double2 *C, int nt, int K, double e_min, double de, double dt, double *total,
                               hipStream_t s);

struct GemmArgs {
    const double2 *amp;     // [nt_pad][npad]: rows are (reference, trajectory) pairs, ref_rows apart
    const double2 *phase;   // [nt_pad][kpad]
    const double *weight;   // [ref_rows] good_j * w_j, the same for every reference state
    double *part_spec;      // [row_tiles][kpad]
    double *part_contrib;   // [kpad / 64][npad]
    int64_t npad;           // row stride of amp (n_refs x ref_rows)
    int64_t ref_rows;       // rows of one reference state (the batch capacity)
    int32_t kpad, nt_pad;
    int32_t row_tiles, col_tiles;
    int32_t tiles_per_ref;  // row tiles holding trajectories, per reference state
};

hipError_t launch_traj(int F, bool mixed, const TrajArgs &a, hipStream_t s);
hipError_t launch_traj_big(int F, bool mixed, const TrajArgs &a, hipStream_t s);  // 17 <= F <= 32
hipError_t launch_sample_husimi(const ProblemDev *P, int F, uint64_t seed, uint64_t first, int64_t n, int64_t npad,
                                double *p0, double *q0, double *logrho, hipStream_t s);
hipError_t launch_phase_table(double e_min, double e_max, int K, int kpad, int nt, int nt_pad, double dt,
                              double2 *phase, hipStream_t s);
hipError_t launch_ref_good_weights(const ProblemDev *P, int F, int ref, const double *good_row, const double *logrho,
                                  const double *p0, const double *q0, int64_t n, int64_t npad, double *goodw_row,
                                  double *goodw_total, hipStream_t s);
hipError_t launch_weights(const ProblemDev *P, int F, const double *good_row, const double *escale_row,
                          const double *logrho, const double *p0, const double *q0, bool husimi, int64_t n,
                          int64_t npad, double *weight, double *goodw_row, unsigned long long *n_good,
                          double *goodw_total, hipStream_t s);
hipError_t launch_fourier_fp64(const GemmArgs &a, hipStream_t s);
hipError_t launch_fourier_f16(const GemmF16Args &a, hipStream_t s);
hipError_t launch_spectrum_reduce(const double *part_spec, int row_tiles, int K, int kpad, double *total,
                                  hipStream_t s);
hipError_t launch_contrib_reduce(const double *part_contrib, int ctiles, const double *weight, int64_t n,
                                 int64_t npad, double *contrib, hipStream_t s);
hipError_t launch_fill_zero(double *p, int64_t count, hipStream_t s);

}  // namespace scivr
