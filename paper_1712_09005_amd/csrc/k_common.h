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

// Cell of a point: x interval + n_int * y interval (s = 2), as the binning
// and every later kernel see it.
template <typename T, int S>
__device__ __forceinline__ int cell_of(const Pt<T, S>& y, const Geom& G)
{
    T t;
    int key = locate<T>(y.v[0], G.origin[0], G.w, G.n_int, t);
    if (S == 2) key += G.n_int * locate<T>(y.v[S - 1], G.origin[1], G.w, G.n_int_y, t);
    return key;
}

}  // namespace tsne
