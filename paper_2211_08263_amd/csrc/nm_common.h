// Shared device/host helpers of the Newmark FFT solver library (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nm {

template <typename T> struct Cx;
template <> struct Cx<double> { using type = double2; };
template <> struct Cx<float> { using type = float2; };
template <typename T> using cx_t = typename Cx<T>::type;

template <typename V> __device__ __forceinline__ V cadd(V a, V b) { return V{a.x + b.x, a.y + b.y}; }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { return V{a.x - b.x, a.y - b.y}; }
template <typename V> __device__ __forceinline__ V cmul(V a, V b)
{
    return V{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename V> __device__ __forceinline__ V cmulc(V a, V b)
{
    return V{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename V> __device__ __forceinline__ V conjv(V a) { return V{a.x, -a.y}; }
// multiply by (DIR * i): DIR = -1 -> -i, DIR = +1 -> +i
template <int DIR, typename V> __device__ __forceinline__ V mul_di(V a)
{
    return DIR < 0 ? V{a.y, -a.x} : V{-a.y, a.x};
}
template <typename V, typename S> __device__ __forceinline__ V cscale(V a, S s) { return V{a.x * s, a.y * s}; }

// Streaming access of a complex element read or written once by a pass: NT bit 0 marks the
// load nontemporal, bit 1 the store (a cache-policy hint; the values are unchanged).
template <int NT, typename V> __device__ __forceinline__ V ld_nt(const V* p)
{
    if constexpr ((NT & 1) != 0) {
        using E = decltype(V{}.x);
        typedef E N2 __attribute__((ext_vector_type(2)));
        const N2 r = __builtin_nontemporal_load((const N2*)p);
        return V{r.x, r.y};
    } else {
        return *p;
    }
}
template <int NT, typename V> __device__ __forceinline__ void st_nt(V* p, V v)
{
    if constexpr ((NT & 2) != 0) {
        using E = decltype(V{}.x);
        typedef E N2 __attribute__((ext_vector_type(2)));
        N2 r;
        r.x = v.x;
        r.y = v.y;
        __builtin_nontemporal_store(r, (N2*)p);
    } else {
        *p = v;
    }
}

// Spatial frequency of DFT index k on an axis of n points, box length L.
// Standard DFT order; the Nyquist bin (k = n/2) and n == 1 give 0.
__host__ __device__ __forceinline__ double freq_of(int k, int n, double L)
{
    if (n == 1 || 2 * k == n) return 0.0;
    int kk = (2 * k < n) ? k : k - n;
    return 6.283185307179586476925286766559 * (double)kk / L;
}

// Signed DFT index of bin k on an axis of n points (0 for the Nyquist bin and n == 1);
// the frequency is this times 2 pi / L.
__host__ __device__ __forceinline__ int freq_index(int k, int n)
{
    if (n == 1 || 2 * k == n) return 0;
    return (2 * k < n) ? k : k - n;
}

constexpr int kBlock = 256;

} // namespace nm
