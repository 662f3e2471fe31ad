// Device helpers for gfx950: complex arithmetic, wave64 cross-lane moves,
// DPP wave reductions and the PML stretch.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace raspml {

// Right-hand side of a batched band solve: v itself, or (ks non-null) for
// each subdomain v + ks[problem].kp * stride -- the Krylov vector of its
// problem's current GMRES step, read on the device so that the launch's
// arguments do not change from step to step.
struct SolveSrc {
    const double2 *v;
    const KState *ks;
    long long stride;
};

// Destination of a PoU-weighted sum: z, or z + ks[problem].kp * stride.
struct SumDst {
    double2 *z;
    const KState *ks;
    long long stride;
};

// Dispatch of a batched band solve: one wave per subdomain (queue null or
// waves >= subdomains), or `waves` persistent waves taking subdomains from
// the atomic counter `queue` (two words, zero between launches).
struct SolveDispatch {
    unsigned int *queue;
    int waves;
};


template <typename T>
struct cplx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cplx<T> mk(T r, T i) { return cplx<T>{r, i}; }

template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a - b * c with fused multiply-adds
template <typename T>
__device__ __forceinline__ cplx<T> cfms(cplx<T> a, cplx<T> b, cplx<T> c) {
    cplx<T> r;
    r.re = fma(-b.re, c.re, a.re);
    r.re = fma(b.im, c.im, r.re);
    r.im = fma(-b.re, c.im, a.im);
    r.im = fma(-b.im, c.re, r.im);
    return r;
}
// a + b * c
template <typename T>
__device__ __forceinline__ cplx<T> cfma(cplx<T> a, cplx<T> b, cplx<T> c) {
    cplx<T> r;
    r.re = fma(b.re, c.re, a.re);
    r.re = fma(-b.im, c.im, r.re);
    r.im = fma(b.re, c.im, a.im);
    r.im = fma(b.im, c.re, r.im);
    return r;
}
// conj(a) * b accumulated
template <typename T>
__device__ __forceinline__ cplx<T> cdotacc(cplx<T> acc, cplx<T> a, cplx<T> b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(-a.im, b.re, acc.im);
    return acc;
}
template <typename T>
__device__ __forceinline__ cplx<T> cscale(cplx<T> a, T s) { return {a.re * s, a.im * s}; }
template <typename T>
__device__ __forceinline__ cplx<T> crecip(cplx<T> a) {
    // scaled to avoid overflow in |a|^2
    T s = fmax(fabs(a.re), fabs(a.im));
    T ar = a.re / s, ai = a.im / s;
    T d = (ar * ar + ai * ai) * s;
    return {ar / d, -ai / d};
}
template <typename T>
__device__ __forceinline__ T cabs2(cplx<T> a) { return a.re * a.re + a.im * a.im; }
// c ? a : b per component (keeps the select in registers)
template <typename T>
__device__ __forceinline__ cplx<T> csel(bool c, cplx<T> a, cplx<T> b) {
    cplx<T> r;
    r.re = c ? a.re : b.re;
    r.im = c ? a.im : b.im;
    return r;
}

template <typename T, typename U>
__device__ __forceinline__ cplx<T> ccast(cplx<U> a) {
    return {static_cast<T>(a.re), static_cast<T>(a.im)};
}

__device__ __forceinline__ int lane_id() {
    return __builtin_amdgcn_mbcnt_hi(-1, __builtin_amdgcn_mbcnt_lo(-1, 0));
}

// ---- wave64 cross-lane moves (lane index must be wave-uniform)
__device__ __forceinline__ float readlane(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double readlane(double v, int l) {
    long long b = __double_as_longlong(v);
    int lo = __builtin_amdgcn_readlane(static_cast<int>(b), l);
    int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), l);
    return __longlong_as_double((static_cast<long long>(hi) << 32) |
                                static_cast<unsigned int>(lo));
}
// Replace lane l of `old` by the (wave-uniform) value v: v_writelane_b32.
// The compiler exposes the instruction only as an LLVM intrinsic.
extern "C" __device__ int raspml_writelane_i32(int v, int lane, int old) __asm(
    "llvm.amdgcn.writelane.i32");
__device__ __forceinline__ float writelane(float old, float v, int l) {
    return __int_as_float(raspml_writelane_i32(__float_as_int(v), l, __float_as_int(old)));
}
__device__ __forceinline__ double writelane(double old, double v, int l) {
    const long long o = __double_as_longlong(old), b = __double_as_longlong(v);
    const int lo = raspml_writelane_i32(static_cast<int>(b), l, static_cast<int>(o));
    const int hi = raspml_writelane_i32(static_cast<int>(b >> 32), l, static_cast<int>(o >> 32));
    return __longlong_as_double((static_cast<long long>(hi) << 32) |
                                static_cast<unsigned int>(lo));
}
template <typename T>
__device__ __forceinline__ cplx<T> readlane(cplx<T> v, int l) {
    return {readlane(v.re, l), readlane(v.im, l)};
}
template <typename T>
__device__ __forceinline__ cplx<T> writelane(cplx<T> old, cplx<T> v, int l) {
    return {writelane(old.re, v.re, l), writelane(old.im, v.im, l)};
}

// ---- DPP wave64 sum; the total ends in lane 63.
// quad_perm [1,0,3,2] = 0xB1, [2,3,0,1] = 0x4E, row_half_mirror 0x141,
// row_mirror 0x140, row_bcast:15 0x142 (rows 1,3), row_bcast:31 0x143 (rows 2,3)
template <int CTRL, int ROWMASK>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWMASK, 0xF, false);
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(dpp_i<CTRL, ROWMASK>(__float_as_int(v)));
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_d(double v) {
    long long b = __double_as_longlong(v);
    int lo = dpp_i<CTRL, ROWMASK>(static_cast<int>(b));
    int hi = dpp_i<CTRL, ROWMASK>(static_cast<int>(b >> 32));
    return __longlong_as_double((static_cast<long long>(hi) << 32) |
                                static_cast<unsigned int>(lo));
}
__device__ __forceinline__ float wave_sum_to63(float v) {
    v += dpp_f<0xB1, 0xF>(v);
    v += dpp_f<0x4E, 0xF>(v);
    v += dpp_f<0x141, 0xF>(v);
    v += dpp_f<0x140, 0xF>(v);
    v += dpp_f<0x142, 0xA>(v);
    v += dpp_f<0x143, 0xC>(v);
    return v;
}
__device__ __forceinline__ double wave_sum_to63(double v) {
    v += dpp_d<0xB1, 0xF>(v);
    v += dpp_d<0x4E, 0xF>(v);
    v += dpp_d<0x141, 0xF>(v);
    v += dpp_d<0x140, 0xF>(v);
    v += dpp_d<0x142, 0xA>(v);
    v += dpp_d<0x143, 0xC>(v);
    return v;
}
template <typename T>
__device__ __forceinline__ cplx<T> wave_sum(cplx<T> v) {
    cplx<T> s{wave_sum_to63(v.re), wave_sum_to63(v.im)};
    return readlane(s, 63);
}

// ---- PML stretch gamma = 1 + i g'(x), g(x) = sigma x^3 beyond the edge.
// Section 1 (global profile: distance to [0,1]) and Section 2 (local
// profile: beyond the Omega_{j,int} edges a, b on sides with an added PML).
__device__ __forceinline__ cplx<double> gamma_at(double x, double sigma, bool lo, double a,
                                                 bool hi, double b) {
    double d;
    if (hi && x >= b)
        d = x - b;
    else if (lo && x <= a)
        d = a - x;
    else
        d = fmax(0.0, fmax(-x, x - 1.0));
    return {1.0, 3.0 * sigma * d * d};
}

}  // namespace raspml
