// Shared device helpers of the mfdkc HIP library (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace mfd {

// Interleaved complex of precision R: float2 / double2.
template <class R> struct cx;
template <> struct cx<float> { using T = float2; };
template <> struct cx<double> { using T = double2; };
template <class R> using cplx = typename cx<R>::T;

template <class T> __host__ __device__ __forceinline__ T mk(double re, double im) {
    T r; r.x = (decltype(r.x))re; r.y = (decltype(r.y))im; return r;
}
template <class T> __device__ __forceinline__ T cadd(T a, T b) { a.x += b.x; a.y += b.y; return a; }
template <class T> __device__ __forceinline__ T csub(T a, T b) { a.x -= b.x; a.y -= b.y; return a; }
template <class T> __device__ __forceinline__ T cmul(T a, T b) {
    T r; r.x = a.x * b.x - a.y * b.y; r.y = a.x * b.y + a.y * b.x; return r;
}
// conj(a) * b
template <class T> __device__ __forceinline__ T cmulc(T a, T b) {
    T r; r.x = a.x * b.x + a.y * b.y; r.y = a.x * b.y - a.y * b.x; return r;
}
template <class T> __device__ __forceinline__ T cconj(T a) { a.y = -a.y; return a; }
template <class T, class S> __device__ __forceinline__ T cscale(T a, S s) { a.x *= s; a.y *= s; return a; }
// acc + a * b
template <class T> __device__ __forceinline__ T cfma(T acc, T a, T b) {
    acc.x = fma(a.x, b.x, acc.x); acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y); acc.y = fma(a.y, b.x, acc.y);
    return acc;
}
// acc + conj(a) * b
template <class T> __device__ __forceinline__ T cfmac(T acc, T a, T b) {
    acc.x = fma(a.x, b.x, acc.x); acc.x = fma(a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y); acc.y = fma(-a.y, b.x, acc.y);
    return acc;
}
template <class T> __device__ __forceinline__ auto cabs2(T a) { return a.x * a.x + a.y * a.y; }

// Workgroups are dispatched round-robin over the 8 XCDs of MI355X (block i
// runs on XCD i mod 8).  Remap so that a run of consecutive logical blocks
// lands on one XCD and shares its L2: logical = (i mod 8) * (G / 8) + i / 8,
// valid when G is a multiple of 8 (otherwise the identity is used).
__device__ __forceinline__ int xcd_remap(int i, int G) {
    if (G & 7) return i;
    return (i & 7) * (G >> 3) + (i >> 3);
}

}  // namespace mfd
