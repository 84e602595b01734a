// Wave-wide small-matrix algebra (gfx950, 64-lane wavefronts).
//
// One matrix per wavefront: its logical row i sits in the registers of lane
// Map::lane(i) as an array of C values.  A Householder LQ sweep (Tria, eq.
// tria of section 2.2) then costs each lane one row's worth of arithmetic per
// reflection instead of the whole trailing block: the reflecting row is
// broadcast with v_readlane (one lane's value copied into scalar registers),
// every lane forms the reflector from the broadcast copy -- the same uniform
// arithmetic in every lane, so all lanes agree bit for bit -- and the lanes
// holding rows below it apply it to their own row.  Rows that no lane holds
// are simply absent; a lane outside the matrix carries rho = -1 and is never
// updated.
//
// The reflector is the one of pss::lq_rows (pivot taken cancellation-free,
// tau = -1 / (r v0), FP32 rows scaled by a power of two, a tail below machine
// epsilon relative to a positive pivot left alone), so a wave sweep and a
// one-thread sweep of the same matrix differ only in where each row's
// arithmetic runs.
#pragma once

#include "device_math.hpp"

namespace pss {
namespace wave {

// value of x in lane `lane` (a wave-uniform constant), in every lane
__device__ __forceinline__ float bcast(float x, int lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), lane));
}
__device__ __forceinline__ double bcast(double x, int lane)
{
    const long long v = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffffLL), lane);
    const int hi = __builtin_amdgcn_readlane((int)(v >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// rows 0..R-1 on lanes OFF..OFF+R-1
template <int OFF> struct Contig {
    static constexpr int lane(int i) { return OFF + i; }
};

// rows 0..NA-1 on lanes OA.., rows NA.. on lanes OB..
template <int NA, int OA, int OB> struct Split {
    static constexpr int lane(int i) { return i < NA ? OA + i : OB + (i - NA); }
};

// Reduce logical rows 0..K-1 of the wave's matrix in turn (lq_rows' contract:
// on return row i < K holds row i of Tria(A) in columns 0..i; entries right
// of the diagonal of reduced rows are stale).  `a` is this lane's row, `rho`
// its logical index (-1: no row).  Z0 is lq_rows' structural-zero bound.
template <int K, int Z0, class Map, typename T, int C>
__device__ __forceinline__ void lq_rows(T (&a)[C], int rho)
{
    constexpr bool kScale = sizeof(T) == 4;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int jend = cmin(C, Z0 + i + 1);
        T x[C];
#pragma unroll
        for (int j = i; j < jend; ++j)
            x[j] = bcast(a[j], Map::lane(i));
        int ex = 0;
        if constexpr (kScale) {
            T sc = pabs(x[i]);
#pragma unroll
            for (int j = i + 1; j < jend; ++j)
                sc = pmax(sc, pabs(x[j]));
            ex = pexp(sc);
#pragma unroll
            for (int j = i; j < jend; ++j)
                x[j] = pldexp(x[j], -ex);
        }
        T sig = T(0);
#pragma unroll
        for (int j = i + 1; j < jend; ++j)
            sig = pfma(x[j], x[j], sig);
        const T al = x[i];
        const T nr = psqrt(pfma(al, al, sig));
        const T v0 = (al > T(0)) ? -sig * prcp(al + nr) : (al - nr);
        const T p = nr * v0;
        const bool skip = !(p < T(0)) || (al > T(0) && sig <= Eps<T>::v * Eps<T>::v * al * al);
        const T tau = skip ? T(0) : -prcp(p);
        if (rho > i) {
            T w = a[i] * v0;
#pragma unroll
            for (int j = i + 1; j < jend; ++j)
                w = pfma(a[j], x[j], w);
            const T tw = tau * w;
            a[i] = pfma(-tw, v0, a[i]);
#pragma unroll
            for (int j = i + 1; j < jend; ++j)
                a[j] = pfma(-tw, x[j], a[j]);
        }
        if (rho == i) {
            const T d = (skip && al > T(0)) ? al : nr;
            a[i] = kScale ? pldexp(d, ex) : d;
        }
    }
}

// L[i][j] (j <= i < N) = column c0 + j of logical row i (rows on Map's lanes)
template <class Map, int N, int c0 = 0, typename T, int C>
__device__ __forceinline__ void bcast_lower(const T (&a)[C], T (&L)[N][N])
{
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j)
            L[i][j] = bcast(a[c0 + j], Map::lane(i));
}

// v[i] = x of the lane holding logical row i
template <class Map, int N, typename T>
__device__ __forceinline__ void bcast_vec(T x, T (&v)[N])
{
#pragma unroll
    for (int i = 0; i < N; ++i)
        v[i] = bcast(x, Map::lane(i));
}

} // namespace wave
} // namespace pss
