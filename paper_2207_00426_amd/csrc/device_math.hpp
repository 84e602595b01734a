// Device small-matrix algebra for the parallel square-root smoother (gfx950).
//
// Every object here lives in registers of ONE thread: the matrices are at
// most 2*NX x 2*NX with NX <= 8, every loop has a compile-time trip count and
// is fully unrolled, so all indices are constants and no scratch memory is
// touched.  Lower-triangular factors are stored in full [N][N] arrays whose
// upper triangle is never read; loops that consume them are bounded by the
// triangle, so structural zeros cost no instructions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define PSS_INL __host__ __device__ __forceinline__

namespace pss {

__host__ __device__ constexpr int tri_size(int n) { return n * (n + 1) / 2; }
__host__ __device__ constexpr int tri_idx(int i, int j) { return i * (i + 1) / 2 + j; }
__host__ __device__ constexpr int cmin(int a, int b) { return a < b ? a : b; }

PSS_INL double psqrt(double x) { return sqrt(x); }
PSS_INL float psqrt(float x) { return sqrtf(x); }
PSS_INL double plog(double x) { return log(x); }
PSS_INL float plog(float x) { return logf(x); }
PSS_INL double pfma(double a, double b, double c) { return fma(a, b, c); }
PSS_INL float pfma(float a, float b, float c) { return fmaf(a, b, c); }

// --------------------------------------------------------------------------
// Reciprocal: the hardware estimate refined by Newton-Raphson steps
// r <- r + r (1 - x r), each roughly doubling the correct bits (two steps in
// FP64, one in FP32, from the estimate's ~2^-23 relative error); ~1 ulp, not
// correctly rounded.  Zero gives an infinity or NaN; callers select such
// results away.
// --------------------------------------------------------------------------
PSS_INL double prcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}
PSS_INL float prcp(float x)
{
    float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// exact power-of-two scaling of a row: 2^-e with sc = m 2^e, m in [0.5, 1)
PSS_INL int pexp(double x) { return __builtin_amdgcn_frexp_exp(x); }
PSS_INL int pexp(float x) { return __builtin_amdgcn_frexp_expf(x); }
PSS_INL double pldexp(double x, int e) { return __builtin_amdgcn_ldexp(x, e); }
PSS_INL float pldexp(float x, int e) { return __builtin_amdgcn_ldexpf(x, e); }

// --------------------------------------------------------------------------
// Tria by Householder reflections applied from the right (an LQ sweep).
//
// On entry A is R x C; rows 0..K-1 are reduced in turn: reflection i maps row
// i onto (|row i|, 0, ...) in columns i..C-1 and is applied to every row
// below it.  On return A[i][j], j <= i < K, hold the first K rows of
// Tria(A) (with K = R: the whole lower factor, diagonal >= 0); entries right
// of the diagonal of reduced rows are stale and must not be read.
//
// Z0 describes structural zeros that reflections preserve: when row i has
// no non-zero beyond column Z0 + i before it is reduced (true for [X | L]
// with X of Z0 columns and L lower or diagonal, and for the stacked blocks
// of Lemmas 1-3), the sweep never touches those columns.  Z0 = C disables
// the shortcut.
//
// Reflector of row x = (a, t) (pivot a, tail t, s = |t|^2, r = |x|):
// v = (a - r, t), with the pivot entry taken as -s / (a + r) when a > 0 so
// nothing cancels; since |v|^2 = -2 r v0, the reflection is
// I - tau v v^T with tau = -1 / (r v0) for either sign of a, and maps x to
// (+r, 0, ...) without a sign fix-up.  Two reciprocals per row.  In FP32 each
// row is first scaled by a power of two near its largest magnitude, so
// squares neither overflow nor fall into the subnormal range (a tail with
// s ~ 1e-39 would otherwise give an infinite tau); FP64's exponent range makes
// that unnecessary for these models.  A tail below machine epsilon relative
// to a positive pivot is left alone (its reflection is the identity to
// working precision), and an all-zero row is untouched.
// --------------------------------------------------------------------------
template <typename T> struct Eps;
template <> struct Eps<double> { static constexpr double v = 2.220446049250313e-16; };
template <> struct Eps<float> { static constexpr float v = 1.1920929e-07f; };

PSS_INL double pabs(double x) { return fabs(x); }
PSS_INL float pabs(float x) { return fabsf(x); }
PSS_INL double pmax(double a, double b) { return fmax(a, b); }
PSS_INL float pmax(float a, float b) { return fmaxf(a, b); }

template <int K, int Z0, typename T, int R, int C>
PSS_INL void lq_rows(T (&A)[R][C])
{
    static_assert(K <= R && K <= C, "lq_rows: need K <= R and K <= C");
    constexpr bool kScale = sizeof(T) == 4;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int jend = cmin(C, Z0 + i + 1);
        int ex = 0;
        if constexpr (kScale) {
            T sc = pabs(A[i][i]);
#pragma unroll
            for (int j = i + 1; j < jend; ++j)
                sc = pmax(sc, pabs(A[i][j]));
            ex = pexp(sc);
#pragma unroll
            for (int j = i; j < jend; ++j)
                A[i][j] = pldexp(A[i][j], -ex);
        }
        T sig = T(0);
#pragma unroll
        for (int j = i + 1; j < jend; ++j)
            sig = pfma(A[i][j], A[i][j], sig);
        const T al = A[i][i];
        const T nr = psqrt(pfma(al, al, sig));
        const T v0 = (al > T(0)) ? -sig * prcp(al + nr) : (al - nr);
        const T p = nr * v0;
        const bool skip = !(p < T(0)) || (al > T(0) && sig <= Eps<T>::v * Eps<T>::v * al * al);
        const T tau = skip ? T(0) : -prcp(p);
#pragma unroll
        for (int r = i + 1; r < R; ++r) {
            T w = A[r][i] * v0;
#pragma unroll
            for (int j = i + 1; j < jend; ++j)
                w = pfma(A[r][j], A[i][j], w);
            const T tw = tau * w;
            A[r][i] = pfma(-tw, v0, A[r][i]);
#pragma unroll
            for (int j = i + 1; j < jend; ++j)
                A[r][j] = pfma(-tw, A[i][j], A[r][j]);
        }
        const T d = (skip && al > T(0)) ? al : nr;
        A[i][i] = kScale ? pldexp(d, ex) : d;
    }
}

// Tria of a rectangular R x C matrix into an R x R lower factor L (C may be
// smaller than R: the missing columns are zeros).
template <typename T, int R, int C>
PSS_INL void tria_rect(const T (&X)[R][C], T (&L)[R][R])
{
    constexpr int W = (C > R) ? C : R;
    T A[R][W];
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j < W; ++j)
            A[i][j] = (j < C) ? X[i][j] : T(0);
    lq_rows<R, (C < W ? C : W)>(A);
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j)
            L[i][j] = A[i][j];
}

// Tria([X, L2]) with X dense R x R and L2 lower R x R, into lower L.
template <typename T, int R>
PSS_INL void tria_dense_lower(const T (&X)[R][R], const T (&L2)[R][R], T (&L)[R][R])
{
    T A[R][2 * R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
#pragma unroll
        for (int j = 0; j < R; ++j)
            A[i][j] = X[i][j];
#pragma unroll
        for (int j = 0; j <= i; ++j)
            A[i][R + j] = L2[i][j];
    }
    lq_rows<R, R>(A);
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j)
            L[i][j] = A[i][j];
}

// Tria([X, L2]) with X dense R x NC and L2 lower R x R, into lower L.
template <typename T, int R, int NC>
PSS_INL void tria_cols_lower(const T (&X)[R][NC], const T (&L2)[R][R], T (&L)[R][R])
{
    T A[R][NC + R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
#pragma unroll
        for (int j = 0; j < NC; ++j)
            A[i][j] = X[i][j];
#pragma unroll
        for (int j = 0; j < R; ++j)
            A[i][NC + j] = (j <= i) ? L2[i][j] : T(0);
    }
    lq_rows<R, NC>(A);
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j)
            L[i][j] = A[i][j];
}

// --------------------------------------------------------------------------
// triangular solves (L lower with non-zero diagonal)
// --------------------------------------------------------------------------
// X = B L^{-1}  (X L = B), B is R x N
template <typename T, int R, int N>
PSS_INL void rsolve_lower(const T (&B)[R][N], const T (&L)[N][N], T (&X)[R][N])
{
    T inv[N];
#pragma unroll
    for (int j = 0; j < N; ++j)
        inv[j] = prcp(L[j][j]);
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int j = N - 1; j >= 0; --j) {
            T s = B[r][j];
#pragma unroll
            for (int t = j + 1; t < N; ++t)
                s = pfma(-X[r][t], L[t][j], s);
            X[r][j] = s * inv[j];
        }
}

// X = B L^{-T}  (X L^T = B), B is R x N
template <typename T, int R, int N>
PSS_INL void rsolve_lower_t(const T (&B)[R][N], const T (&L)[N][N], T (&X)[R][N])
{
    T inv[N];
#pragma unroll
    for (int j = 0; j < N; ++j)
        inv[j] = prcp(L[j][j]);
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int j = 0; j < N; ++j) {
            T s = B[r][j];
#pragma unroll
            for (int t = 0; t < j; ++t)
                s = pfma(-X[r][t], L[j][t], s);
            X[r][j] = s * inv[j];
        }
}

// x = L^{-1} b
template <typename T, int N>
PSS_INL void lsolve_lower(const T (&L)[N][N], const T (&b)[N], T (&x)[N])
{
#pragma unroll
    for (int i = 0; i < N; ++i) {
        T s = b[i];
#pragma unroll
        for (int t = 0; t < i; ++t)
            s = pfma(-L[i][t], x[t], s);
        x[i] = s * prcp(L[i][i]);
    }
}

// --------------------------------------------------------------------------
// small products
// --------------------------------------------------------------------------
template <typename T, int R, int K, int C>
PSS_INL void mm(const T (&A)[R][K], const T (&B)[K][C], T (&O)[R][C])
{
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j < C; ++j) {
            T s = A[i][0] * B[0][j];
#pragma unroll
            for (int t = 1; t < K; ++t)
                s = pfma(A[i][t], B[t][j], s);
            O[i][j] = s;
        }
}

// O = A L with L lower (K x K)
template <typename T, int R, int K>
PSS_INL void mm_lower(const T (&A)[R][K], const T (&L)[K][K], T (&O)[R][K])
{
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j < K; ++j) {
            T s = A[i][j] * L[j][j];
#pragma unroll
            for (int t = j + 1; t < K; ++t)
                s = pfma(A[i][t], L[t][j], s);
            O[i][j] = s;
        }
}

// O = L1^T L2 with L1, L2 lower (N x N); general result
template <typename T, int N>
PSS_INL void mm_lowerT_lower(const T (&L1)[N][N], const T (&L2)[N][N], T (&O)[N][N])
{
#pragma unroll
    for (int a = 0; a < N; ++a)
#pragma unroll
        for (int c = 0; c < N; ++c) {
            const int t0 = a > c ? a : c;
            T s = L1[t0][a] * L2[t0][c];
#pragma unroll
            for (int t = t0 + 1; t < N; ++t)
                s = pfma(L1[t][a], L2[t][c], s);
            O[a][c] = s;
        }
}

// O = A^T B  (A is K x R, B is K x C)
template <typename T, int K, int R, int C>
PSS_INL void mtm(const T (&A)[K][R], const T (&B)[K][C], T (&O)[R][C])
{
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j < C; ++j) {
            T s = A[0][i] * B[0][j];
#pragma unroll
            for (int t = 1; t < K; ++t)
                s = pfma(A[t][i], B[t][j], s);
            O[i][j] = s;
        }
}

template <typename T, int R, int C>
PSS_INL void mv(const T (&A)[R][C], const T (&x)[C], T (&y)[R])
{
#pragma unroll
    for (int i = 0; i < R; ++i) {
        T s = A[i][0] * x[0];
#pragma unroll
        for (int j = 1; j < C; ++j)
            s = pfma(A[i][j], x[j], s);
        y[i] = s;
    }
}

// y = A^T x  (A is R x C)
template <typename T, int R, int C>
PSS_INL void mtv(const T (&A)[R][C], const T (&x)[R], T (&y)[C])
{
#pragma unroll
    for (int j = 0; j < C; ++j) {
        T s = A[0][j] * x[0];
#pragma unroll
        for (int i = 1; i < R; ++i)
            s = pfma(A[i][j], x[i], s);
        y[j] = s;
    }
}

// y = L x, L lower
template <typename T, int N>
PSS_INL void lower_mv(const T (&L)[N][N], const T (&x)[N], T (&y)[N])
{
#pragma unroll
    for (int i = 0; i < N; ++i) {
        T s = L[i][0] * x[0];
#pragma unroll
        for (int j = 1; j <= i; ++j)
            s = pfma(L[i][j], x[j], s);
        y[i] = s;
    }
}

// y = L^T x, L lower
template <typename T, int N>
PSS_INL void lowerT_mv(const T (&L)[N][N], const T (&x)[N], T (&y)[N])
{
#pragma unroll
    for (int j = 0; j < N; ++j) {
        T s = L[j][j] * x[j];
#pragma unroll
        for (int i = j + 1; i < N; ++i)
            s = pfma(L[i][j], x[i], s);
        y[j] = s;
    }
}

} // namespace pss
