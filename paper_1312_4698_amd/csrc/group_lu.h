// Gaussian elimination with partial pivoting across a group of lanes of one
// wave (the small-F trajectory kernels: a trajectory owns G consecutive
// lanes, one or two matrix rows per lane).  Workgroups are single waves, so
// the LDS exchanges need only the compiler ordering of lds_order().
#pragma once

#include "traj_common.h"

namespace scivr {

// Publishes one element of a pivot row.  The stores stay single 8-byte
// stores: merged into 16-byte stores they need their two doubles in four
// consecutive registers, and the register copies that packs them cost more
// than the extra LDS instructions.
__device__ inline void publish(double *row, int j, double v)
{
    typedef __attribute__((address_space(3))) volatile double lds_vf64;
    ((lds_vf64 *)row)[j] = v;
}

// Pivot search of one elimination step: lane `lane` of the group of G lanes
// publishes its best key, and every lane reads the G keys back (16-byte
// broadcast reads) and takes their maximum.  The slots are rewritten at the
// next step; the wave's LDS instructions run in order, so this step's reads
// complete before any lane's next write.
template <int G>
__device__ inline unsigned group_max_key(unsigned *keys, int lane, unsigned mine)
{
    lds_order();
    keys[lane] = mine;
    lds_order();
    constexpr int NQ = (G + 3) / 4;
    unsigned v[4 * NQ];
#pragma unroll
    for (int qd = 0; qd < NQ; ++qd) {
        const uint4 t = reinterpret_cast<const uint4 *>(keys)[qd];
        v[4 * qd] = t.x;
        v[4 * qd + 1] = t.y;
        v[4 * qd + 2] = t.z;
        v[4 * qd + 3] = t.w;
    }
    // a tree of three-input maxima (v_max3_u32)
    unsigned t[(G + 2) / 3];
    int nt = 0;
#pragma unroll
    for (int i = 0; i < G; i += 3)
        t[nt++] = (i + 2 < G) ? max(max(v[i], v[i + 1]), v[i + 2]) : (i + 1 < G ? max(v[i], v[i + 1]) : v[i]);
    unsigned m = t[0];
    int i = 1;
#pragma unroll
    for (; i + 1 < nt; i += 2) m = max(max(m, t[i]), t[i + 1]);
    if (i < nt) m = max(m, t[i]);
    return m;
}

// Pivot bookkeeping of an elimination that leaves rows where they are.
// Row r of the matrix keeps its tag 63 - r and its key (|a|, tag)
// (pivot_key32); the pivot of step k is the live row with the largest key, so
// ties go to the lowest row index.  The determinant is the product of the
// pivots times the sign of the pivot order r_0, r_1, ...: its inversions are
// counted as the number of live rows below r_k at step k (`live` is the
// group-uniform set of rows not yet used as pivots).
struct PivotOrder {
    unsigned live, inversions = 0;
    __device__ explicit PivotOrder(int n) : live(n >= 32 ? ~0u : ((1u << n) - 1u)) {}
    // take the pivot row r = 63 - tag
    __device__ void take(unsigned tag)
    {
        const unsigned r = 63u - tag;
        inversions += __builtin_popcount(live & ((1u << r) - 1u));
        live &= ~(1u << r);
    }
    __device__ double sign(double det) const { return (inversions & 1u) ? -det : det; }
};

// key of a live row from an element's bits: the magnitude's high word with
// the sign bit and the low six bits cleared, and the row's tag in their place
__device__ inline unsigned row_key(double a, unsigned tag) { return ((unsigned)(dbits(a) >> 32) & 0x7FFFFFC0u) | tag; }

// det of the real N x N matrix (N = 2G) whose rows r0 = lane, r1 = G + lane
// live in lane-local a0[], a1[] of lane `lane` of a group of G lanes.  Each
// step picks the pivot as the largest key (group_max_key) of the live rows'
// entries in column k; the lane holding the winner publishes that row; every
// row updates (rows already used as pivots too: they are no longer
// candidates, so their values are never read again).  Lookahead: each step
// updates column k + 1 first and sends the pivot search of step k + 1 off
// before eliminating the rest of the row, so the search's LDS round trip
// overlaps that arithmetic (every element sees the same operations in the
// same order as without it).
template <int N, int G>
__device__ inline double lu_det_real2(double (&a0)[N], double (&a1)[N], int lane, double *piv, unsigned *keys)
{
    const unsigned t0 = 63u - (unsigned)lane, t1 = 63u - (unsigned)(G + lane);
    bool live0 = true, live1 = true;
    PivotOrder order(N);
    double det = 1.0;
    unsigned win = group_max_key<G>(keys, lane, max(row_key(a0[0], t0), row_key(a1[0], t1)));
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const unsigned wt = win & 63u;
        const bool isp0 = live0 && t0 == wt;
        const bool isp1 = live1 && t1 == wt;
        lds_order();
        if (isp0) {
#pragma unroll
            for (int jj = k; jj < N; ++jj) publish(piv, jj, a0[jj]);
        }
        if (isp1) {
#pragma unroll
            for (int jj = k; jj < N; ++jj) publish(piv, jj, a1[jj]);
        }
        lds_order();
        const double pk = piv[k];
        det *= pk;
        order.take(wt);
        live0 = live0 && !isp0;
        live1 = live1 && !isp1;
        if (k + 1 < N) {
            const double inv = rcp_nr(pk);
            const double l0 = a0[k] * inv;
            const double l1 = a1[k] * inv;
            const double v = piv[k + 1];
            a0[k + 1] = fma(-l0, v, a0[k + 1]);
            a1[k + 1] = fma(-l1, v, a1[k + 1]);
            const unsigned k0 = live0 ? row_key(a0[k + 1], t0) : 0u;
            const unsigned k1 = live1 ? row_key(a1[k + 1], t1) : 0u;
            win = group_max_key<G>(keys, lane, max(k0, k1));
#pragma unroll
            for (int jj = k + 2; jj < N; ++jj) {
                const double w = piv[jj];
                a0[jj] = fma(-l0, w, a0[jj]);
                a1[jj] = fma(-l1, w, a1[jj]);
            }
        }
    }
    lds_order();
    return order.sign(det);
}

// det of the complex N x N matrix (N = G) whose row `lane` lives in (ar, ai)
// of lane `lane`; pivot on |a_k|^2; the pivot row is published interleaved
// (re, im).  Same pivot bookkeeping and lookahead as the real elimination.
template <int N>
__device__ inline void lu_det_complex(double (&ar)[N], double (&ai)[N], int lane, double *piv, unsigned *keys,
                                      double &dr, double &di)
{
    const unsigned tg = 63u - (unsigned)lane;
    bool live = true;
    PivotOrder order(N);
    double zr = 1.0, zi = 0.0;
    unsigned win = group_max_key<N>(keys, lane, row_key(fma(ar[0], ar[0], ai[0] * ai[0]), tg));
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const unsigned wt = win & 63u;
        const bool isp = live && tg == wt;
        lds_order();
        if (isp) {
#pragma unroll
            for (int jj = k; jj < N; ++jj) {
                publish(piv, 2 * jj, ar[jj]);
                publish(piv, 2 * jj + 1, ai[jj]);
            }
        }
        lds_order();
        const double pr = piv[2 * k], pi = piv[2 * k + 1];
        const double nr = zr * pr - zi * pi;
        const double ni = zr * pi + zi * pr;
        zr = nr;
        zi = ni;
        order.take(wt);
        live = live && !isp;
        if (k + 1 < N) {
            const double inv = rcp_nr(fma(pr, pr, pi * pi));
            const double lr = (ar[k] * pr + ai[k] * pi) * inv;  // a used pivot row is updated too, never read again
            const double li = (ai[k] * pr - ar[k] * pi) * inv;
            {
                const double br = piv[2 * (k + 1)], bi = piv[2 * (k + 1) + 1];
                ar[k + 1] = fma(-lr, br, fma(li, bi, ar[k + 1]));
                ai[k + 1] = fma(-lr, bi, fma(-li, br, ai[k + 1]));
            }
            const double m2 = fma(ar[k + 1], ar[k + 1], ai[k + 1] * ai[k + 1]);
            win = group_max_key<N>(keys, lane, live ? row_key(m2, tg) : 0u);
#pragma unroll
            for (int jj = k + 2; jj < N; ++jj) {
                const double br = piv[2 * jj], bi = piv[2 * jj + 1];
                ar[jj] = fma(-lr, br, fma(li, bi, ar[jj]));
                ai[jj] = fma(-lr, bi, fma(-li, br, ai[jj]));
            }
        }
    }
    lds_order();
    dr = order.sign(zr);
    di = order.sign(zi);
}

}  // namespace scivr
