// FP64 Fourier accumulation of the TA-SC-IVR estimator (Eq. (11)) as a GEMM
// on the gfx950 matrix cores:
//
//   A_jk = sum_c amp[c][j] * exp(i E_k c dt)          (trajectories x energies)
//   part_spec[tile][k]    = sum_{j in tile} weight_j |A_jk|^2
//
// Several reference states on one batch make it a multi-right-hand-side
// product: their amplitude matrices stack as row blocks of one left operand
// (time-major [t][ref][trajectory]) against the one phase matrix, and each
// row tile's |A|^2 reduction goes to its own reference state's partial sums.
//   part_contrib[ctile][j] = sum_{k in ctile} |A_jk|^2
//
// The complex product is four real v_mfma_f64_16x16x4 per 16x16 block
// (Cr += Ar Br - Ai Bi, Ci += Ar Bi + Ai Br).  Both operands are time-major, so
// each MFMA operand fragment (16 consecutive trajectories or energies at one
// time sample per lane quarter) is a coalesced 256-byte load straight into
// registers; the time block after next is prefetched while the current one
// is multiplied.  A workgroup of eight waves covers 128 trajectories x 128
// energies (2 x 4 waves of 64 x 32, two waves per SIMD: each wave's 128
// accumulator registers fit beside its operands, so the accumulators are not
// shuffled between register files); |A|^2 never leaves registers: the epilogue
// reduces it over trajectories (weighted, for the spectrum) and over energies
// (for the per-trajectory contributions).  Workgroups are mapped so that each
// of the eight XCDs walks a contiguous range of trajectory tiles with the
// energy tiles innermost, which keeps the amplitude tile resident in that
// XCD's L2 while all energy tiles consume it.
#include "scivr_internal.h"

namespace scivr {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2))) fourier_fp64_kernel(GemmArgs G)
{
    const int wg = blockIdx.x;
    const int nwg = G.row_tiles * G.col_tiles;
    int rt, ct;
    if (nwg % 8 == 0) {
        const int per = nwg / 8;
        const int lin = (wg % 8) * per + wg / 8;
        rt = lin / G.col_tiles;
        ct = lin % G.col_tiles;
    } else {
        rt = wg / G.col_tiles;
        ct = wg % G.col_tiles;
    }
    // eight waves: 2 x 4 of 64 trajectories x 32 energies
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wr = wave >> 2, wc = wave & 3;
    // row tile rt is tile rt % tiles_per_ref of reference state rt / tiles_per_ref
    const int ref = rt / G.tiles_per_ref;
    const int64_t lrow0 = (int64_t)(rt - ref * G.tiles_per_ref) * GEMM_BM + wr * 64;  // trajectory of the tile's row
    const int64_t row0 = ref * G.ref_rows + lrow0;
    const int col0 = ct * GEMM_BN + wc * 32;
    const int kk = lane >> 4, ii = lane & 15;

    d4 cr[4][2], ci[4][2];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
            cr[bi][bj] = (d4){0.0, 0.0, 0.0, 0.0};
            ci[bi][bj] = (d4){0.0, 0.0, 0.0, 0.0};
        }

    const double2 *Ap = G.amp + (int64_t)kk * G.npad + row0 + ii;
    const double2 *Bp = G.phase + (int64_t)kk * G.kpad + col0 + ii;
    const int64_t astep = (int64_t)GEMM_BK * G.npad;
    const int64_t bstep = (int64_t)GEMM_BK * G.kpad;

    // operands of the current time block (a, b), the next (an, bn) and the one
    // after (loaded while the current one is multiplied).  The buffers hold
    // two zero time blocks beyond nt_pad, so the prefetch never leaves them.
    double2 a[4], b[2], an[4], bn[2];
#pragma unroll
    for (int x = 0; x < 4; ++x) {
        a[x] = Ap[x * 16];
        an[x] = Ap[astep + x * 16];
    }
#pragma unroll
    for (int x = 0; x < 2; ++x) {
        b[x] = Bp[x * 16];
        bn[x] = Bp[bstep + x * 16];
    }
    Ap += astep;
    Bp += bstep;
    for (int t0 = 0; t0 < G.nt_pad; t0 += GEMM_BK) {
        Ap += astep;
        Bp += bstep;
        double2 a2[4], b2[2];
#pragma unroll
        for (int x = 0; x < 4; ++x) a2[x] = Ap[x * 16];
#pragma unroll
        for (int x = 0; x < 2; ++x) b2[x] = Bp[x * 16];
        // the four real products in four sweeps over the 8 blocks, so that the
        // two updates of one accumulator are 8 independent MFMAs apart
        double nai[4];
#pragma unroll
        for (int bi = 0; bi < 4; ++bi) nai[bi] = -a[bi].y;
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
                cr[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi].x, b[bj].x, cr[bi][bj], 0, 0, 0);
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
                ci[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi].x, b[bj].y, ci[bi][bj], 0, 0, 0);
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
                cr[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(nai[bi], b[bj].y, cr[bi][bj], 0, 0, 0);
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
                ci[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi].y, b[bj].x, ci[bi][bj], 0, 0, 0);
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            a[x] = an[x];
            an[x] = a2[x];
        }
#pragma unroll
        for (int x = 0; x < 2; ++x) {
            b[x] = bn[x];
            bn[x] = b2[x];
        }
    }

    // ---- epilogue ----
    // v_mfma_f64_16x16x4f64 leaves D[i][j] in lane j + 16 (i mod 4), register i / 4:
    // element r of block (bi, bj) in this lane is row 4 r + kk, column ii of the block.
    double w[4][4];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int r = 0; r < 4; ++r) w[bi][r] = G.weight[lrow0 + bi * 16 + 4 * r + kk];

    __shared__ double lds_spec[2][GEMM_BN];
    __shared__ double lds_row[8][64];
    double rowsum[4][4];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int r = 0; r < 4; ++r) rowsum[bi][r] = 0.0;
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
        double colsum = 0.0;
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const double m2 = cr[bi][bj][r] * cr[bi][bj][r] + ci[bi][bj][r] * ci[bi][bj][r];
                rowsum[bi][r] += m2;
                colsum += (w[bi][r] != 0.0) ? w[bi][r] * m2 : 0.0;
            }
        colsum += __shfl_xor(colsum, 16);
        colsum += __shfl_xor(colsum, 32);
        if (kk == 0) lds_spec[wr][wc * 32 + bj * 16 + ii] = colsum;
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
            if (ii == 0) lds_row[wave][bi * 16 + 4 * r + kk] = v;
        }
    __syncthreads();
    // per-trajectory sums over each 64-energy half of the tile: waves wc and
    // wc + 1 cover one half
    if ((wc & 1) == 0)
        G.part_contrib[(int64_t)(ct * 2 + (wc >> 1)) * G.npad + row0 + lane] = lds_row[wave][lane] + lds_row[wave + 1][lane];
    if (threadIdx.x < GEMM_BN) {
        const int x = threadIdx.x;
        G.part_spec[(int64_t)rt * G.kpad + ct * GEMM_BN + x] = lds_spec[0][x] + lds_spec[1][x];
    }
}

}  // namespace

hipError_t launch_fourier_fp64(const GemmArgs &a, hipStream_t s)
{
    const int nwg = a.row_tiles * a.col_tiles;
    if (nwg <= 0) return hipSuccess;
    hipLaunchKernelGGL(fourier_fp64_kernel, dim3(nwg), dim3(512), 0, s, a);
    return hipGetLastError();
}

}  // namespace scivr
