// Per-point arithmetic of the kinetic update shared by the sweep kernels
// (internal): division, exponential and the reference distributions g / tau
// evaluated from a cell's sweep parameters.
#pragma once
#include "gsis_common.h"

namespace gsis {

template <typename T> struct Arith;
// Division by the hardware reciprocal: one rounding more than IEEE division
// (FP32: v_rcp_f32, about 1 ulp; FP64: v_rcp_f64 refined by two Newton steps
// and a residual correction), the same code for every tile shape.  FP32
// exponential: the hardware exp2; FP64: exp_nonpos below.
template <> struct Arith<float> {
    static __device__ __forceinline__ float ex(float x) { return __expf(x); }
    static __device__ __forceinline__ float div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
};
// e^x for x <= 0 (the argument of every Maxwellian factor here): exp_core,
// with arguments below -745 clamped there, where e^x is zero in FP64.
__device__ __forceinline__ double exp_nonpos(double x) { return exp_core(fmax(x, -745.0)); }

template <> struct Arith<double> {
    static __device__ __forceinline__ double ex(double x) { return exp_nonpos(x); }
    static __device__ __forceinline__ double div(double a, double b)
    {
        double r = __builtin_amdgcn_rcp(b);
        double e = fma(-b, r, 1.0);
        r = fma(r, e, r);
        e = fma(-b, r, 1.0);
        r = fma(r, e, r);
        double q = a * r;
        double res = fma(-b, q, a);
        return fma(r, res, q);
    }
};

// g / tau at node (cx, cy, cz) = xi - u of a monatomic cell
template <typename T>
__device__ __forceinline__ T ref_mono(const T *p, T cx, T cy, T cz, T it)
{
#pragma clang fp contract(off)
    const T c2 = fma(cz, cz, fma(cy, cy, cx * cx));
    const T t = c2 * it;
    const T E = p[4] * Arith<T>::ex(-t);
    const T q = fma(p[12], cz, fma(p[11], cy, p[10] * cx));
    const T poly = fma(q, t - T(2.5), fma(p[9], c2, fma(p[8], cz, fma(p[7], cy, fma(p[6], cx, p[5])))));
    return E * poly;
}

// g0 / tau, g1 / tau of a diatomic cell (Rykov mixture of the four components)
template <typename T>
__device__ __forceinline__ void ref_dia(const T *p, T cx, T cy, T cz, T itt, T itr, T &g0, T &g1)
{
#pragma clang fp contract(off)
    const T c2 = fma(cz, cz, fma(cy, cy, cx * cx));
    const T tt = c2 * itt, tr = c2 * itr;
    const T Et = p[5] * Arith<T>::ex(-tt);
    const T Er = p[6] * Arith<T>::ex(-tr);
    const T sht = fma(p[14], cz, fma(p[13], cy, p[12] * cx)) * (tt - T(2.5));
    const T shr = fma(p[22], cz, fma(p[21], cy, p[20] * cx)) * (tr - T(2.5));
    const T lt = fma(p[11], c2, fma(p[10], cz, fma(p[9], cy, fma(p[8], cx, p[7]))));
    const T lr = fma(p[19], c2, fma(p[18], cz, fma(p[17], cy, fma(p[16], cx, p[15]))));
    const T rt = fma(p[26], cz, fma(p[25], cy, fma(p[24], cx, fma(p[23], T(1) + sht, p[27]))));
    const T rr = fma(p[31], cz, fma(p[30], cy, fma(p[29], cx, fma(p[28], T(1) + shr, p[32]))));
    g0 = fma(Et, lt + sht, Er * (lr + shr));
    g1 = fma(Et, rt, Er * rr);
}

}  // namespace gsis
