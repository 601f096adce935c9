// Device helpers shared by the trajectory kernels (small F: F lanes per
// trajectory; large F: one wave per trajectory).
#pragma once

#include <math.h>

#include "scivr_internal.h"

namespace scivr {

__device__ inline unsigned long long dbits(double x) { return (unsigned long long)__double_as_longlong(x); }

// Workgroups are one wave, and a wave's LDS instructions execute in issue
// order, so a write by one lane is visible to a later read by another lane of
// the same wave without waiting; only the compiler must keep the order.
__device__ inline void lds_order()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

typedef const __attribute__((address_space(4))) ProblemDev *ConstProblem;

// A fresh, opaque handle to the trajectory-independent constants.  Taking it
// inside the time loop keeps their uniform doubles as scalar-cache loads there
// instead of letting them be hoisted into (and spilled out of) the scalar
// register file.
__device__ inline ConstProblem opaque(const ProblemDev *P)
{
    uint64_t v = (uint64_t)P;
    asm volatile("" : "+s"(v));
    return (ConstProblem)v;
}

// 32-bit pivot key: the high word of the (non-negative) magnitude's bits with
// its low six bits replaced by 63 - pos.  Keys order as the magnitudes
// truncated to 14 mantissa bits, ties going to the lowest position (partial
// pivoting up to a factor 1 + 2^-14 in the pivot's size); 0 marks a row that
// is no longer a candidate.
__device__ inline unsigned pivot_key32(double mag, int pos)
{
    return ((unsigned)(dbits(mag) >> 32) & ~63u) | (unsigned)(63 - pos);
}

// Kahan-compensated running sum (used for the FP32 action of the mixed form).
struct Kahan {
    float s = 0.f, c = 0.f;
    __device__ void add(float x)
    {
        const float y = x - c;
        const float t = s + y;
        c = (t - s) - y;
        s = t;
    }
    __device__ double value() const { return (double)s - (double)c; }
};

template <bool MIXED>
struct Action;
template <>
struct Action<false> {
    double s = 0.0;
    __device__ void add(double x) { s += x; }
    __device__ double value() const { return s; }
    __device__ void load(double v, double) { s = v; }
    __device__ void set_total(double v) { s = v; }
    __device__ double pack() const { return s; }
    __device__ void unpack(double v) { s = v; }
    __device__ double hi() const { return s; }
    __device__ double lo() const { return 0.0; }
};
template <>
struct Action<true> {
    Kahan k;
    __device__ void add(double x) { k.add((float)x); }
    __device__ double value() const { return k.value(); }
    __device__ void load(double v, double comp)
    {
        k.s = (float)v;
        k.c = (float)comp;
    }
    // the compensated pair (s, c) with s - c ~ v
    __device__ void set_total(double v)
    {
        k.s = (float)v;
        k.c = (float)((double)k.s - v);
    }
    // the pair (s, c) bit for bit in one 64-bit word
    __device__ double pack() const { return __hiloint2double(__float_as_int(k.c), __float_as_int(k.s)); }
    __device__ void unpack(double v)
    {
        k.s = __int_as_float(__double2loint(v));
        k.c = __int_as_float(__double2hiint(v));
    }
    __device__ double hi() const { return (double)k.s; }
    __device__ double lo() const { return (double)k.c; }
};

// Split x into FP16 hi + lo with x ~ hi + lo to about 22 bits.
__device__ inline void split_f16(float x, _Float16 &hi, _Float16 &lo)
{
    hi = (_Float16)x;
    lo = (_Float16)(x - (float)hi);
}

}  // namespace scivr
