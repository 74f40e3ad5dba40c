// Forward-mode dual numbers for the adjoint of the face flux.
//
// Dual<N> carries a value and N directional derivatives.  The overloads below
// let the same templated flux code (fv_device.hpp) run on duals, so the
// Jacobian of a face flux with respect to its face states is exact for the
// branch the forward pass takes (min/max, selects and the positivity guards
// pick the derivative of the selected operand).
#pragma once

#include <hip/hip_runtime.h>

namespace fvk {

template <int N> struct Dual {
    float v;
    float d[N];
    __device__ __forceinline__ Dual() {}
    __device__ __forceinline__ Dual(float x) : v(x)
    {
#pragma unroll
        for (int i = 0; i < N; i++) d[i] = 0.0f;
    }
};

template <int N> __device__ __forceinline__ Dual<N> seed(float x, int dir)
{
    Dual<N> r(x);
    r.d[dir] = 1.0f;
    return r;
}

#define DUAL_BIN(OP, DEXPR)                                                                          \
    template <int N> __device__ __forceinline__ Dual<N> operator OP(const Dual<N> &a, const Dual<N> &b) \
    {                                                                                                \
        Dual<N> r;                                                                                   \
        r.v = a.v OP b.v;                                                                            \
        _Pragma("unroll") for (int i = 0; i < N; i++) r.d[i] = DEXPR;                                \
        return r;                                                                                    \
    }
DUAL_BIN(+, a.d[i] + b.d[i])
DUAL_BIN(-, a.d[i] - b.d[i])
DUAL_BIN(*, a.d[i] * b.v + a.v * b.d[i])
#undef DUAL_BIN

template <int N> __device__ __forceinline__ Dual<N> operator-(const Dual<N> &a)
{
    Dual<N> r;
    r.v = -a.v;
#pragma unroll
    for (int i = 0; i < N; i++) r.d[i] = -a.d[i];
    return r;
}
template <int N> __device__ __forceinline__ Dual<N> &operator+=(Dual<N> &a, const Dual<N> &b)
{
    a = a + b;
    return a;
}
template <int N> __device__ __forceinline__ bool operator<(const Dual<N> &a, const Dual<N> &b) { return a.v < b.v; }
template <int N> __device__ __forceinline__ bool operator>(const Dual<N> &a, const Dual<N> &b) { return a.v > b.v; }
template <int N> __device__ __forceinline__ bool operator<=(const Dual<N> &a, const Dual<N> &b) { return a.v <= b.v; }
template <int N> __device__ __forceinline__ bool operator>=(const Dual<N> &a, const Dual<N> &b) { return a.v >= b.v; }
template <int N> __device__ __forceinline__ bool operator==(const Dual<N> &a, const Dual<N> &b) { return a.v == b.v; }

template <int N> __device__ __forceinline__ Dual<N> rcp(const Dual<N> &a)
{
    Dual<N> r;
    r.v = __builtin_amdgcn_rcpf(a.v);
    float s = -r.v * r.v;
#pragma unroll
    for (int i = 0; i < N; i++) r.d[i] = s * a.d[i];
    return r;
}
template <int N> __device__ __forceinline__ Dual<N> fsqrt(const Dual<N> &a)
{
    Dual<N> r;
    r.v = __builtin_amdgcn_sqrtf(a.v);
    float s = r.v > 0.0f ? 0.5f * __builtin_amdgcn_rcpf(r.v) : 0.0f;
#pragma unroll
    for (int i = 0; i < N; i++) r.d[i] = s * a.d[i];
    return r;
}
template <int N> __device__ __forceinline__ Dual<N> tmin(const Dual<N> &a, const Dual<N> &b) { return b.v < a.v ? b : a; }
template <int N> __device__ __forceinline__ Dual<N> tmax(const Dual<N> &a, const Dual<N> &b) { return b.v > a.v ? b : a; }
template <int N> __device__ __forceinline__ Dual<N> tabs(const Dual<N> &a) { return a.v < 0.0f ? -a : a; }

}  // namespace fvk
