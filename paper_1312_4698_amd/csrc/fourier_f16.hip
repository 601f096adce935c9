// Mixed-form Fourier accumulation of the TA-SC-IVR estimator (Eq. (11)) as a
// split-FP16 GEMM on the gfx950 matrix cores with FP32 accumulation:
//
//   A_jk = sum_c amp[c][j] * exp(i E_k c dt)
//
// Both factors are carried as FP16 pairs x ~ x_hi + x_lo (about 22 bits), and
// each real product is x_hi y_hi + x_hi y_lo + x_lo y_hi, so a complex 16 x 16
// block over 32 time samples costs twelve v_mfma_f32_16x16x32_f16.  The
// amplitudes (already scaled per trajectory by a power of two, undone in the
// weights) stream from HBM in the time-blocked layout [t / 8][trajectory][t % 8]
// that is exactly one MFMA operand fragment per lane.  The phase factors are
// never stored: each lane generates exp(i E_k t dt) for its eight time samples
// from an FP64 start value advanced by exp(i E_k 32 dt) per k-step, with an
// FP32 recurrence inside the fragment, and splits them on the fly.  A
// workgroup of four waves covers 128 trajectories x 128 energies; the epilogue
// is the same weighted |A|^2 reduction as the FP64 kernel, in FP64.
//
// v_mfma_f32_16x16x32_f16 lane layout on gfx950 (checked with a one-hot probe):
// A[i][k] in lane i + 16 (k / 8), slot k % 8; B[k][j] in lane j + 16 (k / 8),
// slot k % 8; D[i][j] in lane j + 16 (i / 4), register i % 4.
#include <math.h>

#include "scivr_internal.h"

namespace scivr {
namespace {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ inline f4 mma(h8 a, h8 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }

__global__ void __launch_bounds__(256, 1) fourier_f16_kernel(GemmF16Args G)
{
    const int wg = blockIdx.x;
    const int nwg = G.row_tiles * G.col_tiles;
    int rt, ct;
    if (nwg % 8 == 0) {  // each XCD walks contiguous trajectory tiles, energy tiles innermost
        const int per = nwg / 8;
        const int lin = (wg % 8) * per + wg / 8;
        rt = lin / G.col_tiles;
        ct = lin % G.col_tiles;
    } else {
        rt = wg / G.col_tiles;
        ct = wg % G.col_tiles;
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wr = wave >> 1, wc = wave & 1;
    const int64_t row0 = (int64_t)rt * GEMM_BM + wr * 64;
    const int col0 = ct * GEMM_BN + wc * 64;
    const int kq = lane >> 4, ii = lane & 15;

    f4 cr[4][4], ci[4][4];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj) {
            cr[bi][bj] = (f4){0.f, 0.f, 0.f, 0.f};
            ci[bi][bj] = (f4){0.f, 0.f, 0.f, 0.f};
        }

    // phase generators of this lane's four energies: z = exp(i E t0 dt) at the
    // lane's first time sample t0 = 8 kq, advanced by exp(i E 32 dt) per k-step
    double zr[4], zi[4], sr[4], si[4];
    float s1r[4], s1i[4];
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) {
        const double E = G.e_min + (double)(col0 + bj * 16 + ii) * G.de;
        double s, c;
        sincos(E * (8.0 * kq) * G.dt, &s, &c);
        zr[bj] = c;
        zi[bj] = s;
        sincos(E * (double)GEMM16_BK * G.dt, &s, &c);
        sr[bj] = c;
        si[bj] = s;
        sincos(E * G.dt, &s, &c);
        s1r[bj] = (float)c;
        s1i[bj] = (float)s;
    }

    const int64_t P = G.plane;
    const _Float16 *ap = G.amp16 + ((int64_t)kq * G.npad + row0 + ii) * 8;
    const int64_t astep = (int64_t)(GEMM16_BK / 8) * G.npad * 8;

    // amplitude fragments of one k-step; the next k-step's are in flight while
    // the current one is multiplied (the last prefetch re-reads the last k-step)
    h8 arh[4], arl[4], aih[4], ail[4];
    auto load = [&](const _Float16 *base, h8(&rh)[4], h8(&rl)[4], h8(&ih)[4], h8(&il)[4]) {
#pragma unroll
        for (int bi = 0; bi < 4; ++bi) {
            const _Float16 *a = base + bi * 16 * 8;
            rh[bi] = *(const h8 *)(a);
            rl[bi] = *(const h8 *)(a + P);
            ih[bi] = *(const h8 *)(a + 2 * P);
            il[bi] = *(const h8 *)(a + 3 * P);
        }
    };
    load(ap, arh, arl, aih, ail);
    for (int t0 = 0; t0 < G.nt_pad; t0 += GEMM16_BK) {
        if (t0 + GEMM16_BK < G.nt_pad) ap += astep;
        h8 nrh[4], nrl[4], nih_[4], nil_[4];
        load(ap, nrh, nrl, nih_, nil_);
#pragma unroll
        for (int bj = 0; bj < 4; ++bj) {
            // exp(i E t dt) for t = t0 + 8 kq + s, s = 0..7, split into FP16 pairs
            h8 prh, prl, pih, pil, nih, nil;
            float wr_ = (float)zr[bj], wi_ = (float)zi[bj];
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const _Float16 rh = (_Float16)wr_, ih = (_Float16)wi_;
                const _Float16 rl = (_Float16)(wr_ - (float)rh), il = (_Float16)(wi_ - (float)ih);
                prh[s] = rh;
                prl[s] = rl;
                pih[s] = ih;
                pil[s] = il;
                nih[s] = -ih;
                nil[s] = -il;
                const float nr = wr_ * s1r[bj] - wi_ * s1i[bj];
                const float ni = wr_ * s1i[bj] + wi_ * s1r[bj];
                wr_ = nr;
                wi_ = ni;
            }
            const double nzr = zr[bj] * sr[bj] - zi[bj] * si[bj];
            const double nzi = zr[bj] * si[bj] + zi[bj] * sr[bj];
            zr[bj] = nzr;
            zi[bj] = nzi;
#pragma unroll
            for (int bi = 0; bi < 4; ++bi) {
                f4 r = cr[bi][bj], m = ci[bi][bj];
                r = mma(arh[bi], prh, r);
                r = mma(arh[bi], prl, r);
                r = mma(arl[bi], prh, r);
                r = mma(aih[bi], nih, r);
                r = mma(aih[bi], nil, r);
                r = mma(ail[bi], nih, r);
                m = mma(arh[bi], pih, m);
                m = mma(arh[bi], pil, m);
                m = mma(arl[bi], pih, m);
                m = mma(aih[bi], prh, m);
                m = mma(aih[bi], prl, m);
                m = mma(ail[bi], prh, m);
                cr[bi][bj] = r;
                ci[bi][bj] = m;
            }
        }
#pragma unroll
        for (int bi = 0; bi < 4; ++bi) {
            arh[bi] = nrh[bi];
            arl[bi] = nrl[bi];
            aih[bi] = nih_[bi];
            ail[bi] = nil_[bi];
        }
    }

    // ---- epilogue: element r of block (bi, bj) in this lane is row 4 kq + r, column ii ----
    double w[4][4];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int r = 0; r < 4; ++r) w[bi][r] = G.weight[row0 + bi * 16 + 4 * kq + r];

    __shared__ double lds_spec[2][GEMM_BN];
    double rowsum[4][4];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int r = 0; r < 4; ++r) rowsum[bi][r] = 0.0;
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) {
        double colsum = 0.0;
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const double re = cr[bi][bj][r], im = ci[bi][bj][r];
                const double m2 = re * re + im * im;
                rowsum[bi][r] += m2;
                colsum += (w[bi][r] != 0.0) ? w[bi][r] * m2 : 0.0;
            }
        colsum += __shfl_xor(colsum, 16);
        colsum += __shfl_xor(colsum, 32);
        if (kq == 0) lds_spec[wr][wc * 64 + bj * 16 + ii] = colsum;
    }
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            double v = rowsum[bi][r];
            v += __shfl_xor(v, 1);
            v += __shfl_xor(v, 2);
            v += __shfl_xor(v, 4);
            v += __shfl_xor(v, 8);
            if (ii == 0) G.part_contrib[(int64_t)(ct * 2 + wc) * G.npad + row0 + bi * 16 + 4 * kq + r] = v;
        }
    __syncthreads();
    if (threadIdx.x < GEMM_BN) {
        const int x = threadIdx.x;
        G.part_spec[(int64_t)rt * G.kpad + ct * GEMM_BN + x] = lds_spec[0][x] + lds_spec[1][x];
    }
}

}  // namespace

hipError_t launch_fourier_f16(const GemmF16Args &a, hipStream_t s)
{
    const int nwg = a.row_tiles * a.col_tiles;
    if (nwg <= 0) return hipSuccess;
    hipLaunchKernelGGL(fourier_f16_kernel, dim3(nwg), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace scivr
