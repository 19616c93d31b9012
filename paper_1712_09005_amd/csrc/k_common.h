// Device helpers shared by the point-side kernels (binning, spreading,
// gathering, update): element loads, the interval of a coordinate, and one
// point's coordinates moved as one vector.
#pragma once

#include <math.h>

#include "launch.h"

namespace tsne {

template <typename T> __device__ __forceinline__ T ld(const void* p, int64_t i)
{
    return static_cast<const T*>(p)[i];
}

// Interval of a coordinate value and its local coordinate:
// u = (y - o) / w, l = clamp(floor(u), 0, n_int - 1), t = u - l.
// Evaluated in double for both element types: the input value is exact in
// double, so the interval is the same in every kernel and t carries no error
// from the box offset (FP32 t would lose |u| * 2^-24 absolute).
template <typename T>
__device__ __forceinline__ int locate(T y, double o, double w, int n_int, T& t)
{
#pragma clang fp contract(off)
    const double u = ((double)y - o) / w;
    const double f = floor(u);
    int c;
    if (!(f >= 0.0)) c = 0;
    else if (f > (double)(n_int - 1)) c = n_int - 1;
    else c = (int)f;
    t = (T)(u - (double)c);
    return c;
}

// One point's S coordinates, moved with one vector access when S = 2 (the
// [N, S] arrays are 8- or 16-byte aligned per point).
template <typename T, int S> struct Pt {
    T v[S];
    __device__ __forceinline__ static Pt load(const T* a, int64_t i)
    {
        Pt p;
#pragma unroll
        for (int d = 0; d < S; ++d) p.v[d] = a[i * S + d];
        return p;
    }
    __device__ __forceinline__ void store(T* a, int64_t i) const
    {
#pragma unroll
        for (int d = 0; d < S; ++d) a[i * S + d] = v[d];
    }
};
template <typename T> struct Pt2Vec;
template <> struct Pt2Vec<float> { typedef float2 t; };
template <> struct Pt2Vec<double> { typedef double2 t; };
template <typename T> struct Pt<T, 2> {
    typedef typename Pt2Vec<T>::t V;
    T v[2];
    __device__ __forceinline__ static Pt load(const T* a, int64_t i)
    {
        const V q = reinterpret_cast<const V*>(a)[i];
        Pt p;
        p.v[0] = q.x;
        p.v[1] = q.y;
        return p;
    }
    __device__ __forceinline__ void store(T* a, int64_t i) const
    {
        V q;
        q.x = v[0];
        q.y = v[1];
        reinterpret_cast<V*>(a)[i] = q;
    }
};

// Cell of a point: x interval + n_int * y interval (s >= 2) + n_int n_int_y
// * z interval (s = 3), as the binning and every later kernel see it.
template <typename T, int S>
__device__ __forceinline__ int cell_of(const Pt<T, S>& y, const Geom& G)
{
    T t;
    int key = locate<T>(y.v[0], G.origin[0], G.w, G.n_int, t);
    if (S >= 2) key += G.n_int * locate<T>(y.v[1], G.origin[1], G.w, G.n_int_y, t);
    if (S == 3) key += G.n_int * G.n_int_y * locate<T>(y.v[S - 1], G.origin[S - 1], G.w, G.n_int, t);
    return key;
}

// 1 / prod_{k != m} (m - k), the denominator of the Lagrange basis on nodes
// m + 1/2 (in units of the node spacing).
__host__ __device__ constexpr double lag_inv_denom(int P, int m)
{
    double d = 1.0;
    for (int k = 0; k < P; ++k)
        if (k != m) d *= (double)(m - k);
    return 1.0 / d;
}

// Lagrange basis of Section 2.1 on the p equispaced nodes (m + 1/2)/p of the
// unit interval, evaluated at t in [0, 1] (eq. (equinodes) for the nodes).
template <typename T, int P>
__device__ __forceinline__ void lagrange(T t, T (&L)[P])
{
    const T sv = t * (T)P;
    T a[P];
#pragma unroll
    for (int k = 0; k < P; ++k) a[k] = sv - ((T)k + (T)0.5);
#pragma unroll
    for (int m = 0; m < P; ++m) {
        T prod = (T)lag_inv_denom(P, m);
#pragma unroll
        for (int k = 0; k < P; ++k)
            if (k != m) prod *= a[k];
        L[m] = prod;
    }
}

// Charges and potentials per form: A {1, y'(d)} -> K1*1, K2*1, K2*y'(d);
// B adds |y'|^2 and takes K2*|y'|^2 in place of K1*1; V (vector kernels)
// has the one charge 1 -> K1*1 and (z_d K2)*1 for each dimension d.
template <int S, int FORM> struct Shape {
    static constexpr int NC = (FORM == 0) ? S + 1 : (FORM == 1) ? S + 2 : 1;
    static constexpr int NP = (FORM == 2) ? S + 1 : S + 2;
};

}  // namespace tsne
