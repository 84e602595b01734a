// Positive-weight sigma-point rules (Section 4.3) and the generalised
// statistical linear regression built on them (the GSLR moments of Section
// 2.3), with the models' images written as deviations from a reference
// value so that no difference of two large numbers is formed.  Used by the
// unscented and Gauss-Hermite rules of both nonlinear models and by every
// linearisation of the Ricker-Poisson model (Section 6.1).
#pragma once

#include "common.hpp"
#include "device_ops.hpp"

namespace pss {

PSS_INL double vexp(double x) { return exp(x); }
PSS_INL float vexp(float x) { return expf(x); }
PSS_INL double vexpm1(double x) { return expm1(x); }
PSS_INL float vexpm1(float x) { return expm1f(x); }

// A rule with unit points xi_i and weights w_i > 0 (sum one) that
// integrates the first two moments of N(0, I) exactly:
//   kind 0 (cubature)  +-spread e_j, weight wi (spread = sqrt(nx));
//   kind 1 (unscented) the centre with weight w0 (when w0 > 0), then
//                      +-spread e_j with weight wi;
//   kind 2 (Gauss-Hermite) point i = sum_j d_j p^j (d_0 the first
//                      coordinate): xi_j = gx[d_j], w = prod_j gw[d_j].
template <typename T>
struct RuleSpec {
    int kind, np, p;
    T w0, wi, spread;
    T gx[kMaxGH], gw[kMaxGH];
};

template <typename T, int NX>
PSS_INL T rule_point(const RuleSpec<T> &R, int i, T (&xi)[NX])
{
#pragma unroll
    for (int j = 0; j < NX; ++j)
        xi[j] = T(0);
    if (R.kind == 2) {
        T w = T(1);
        int r = i;
#pragma unroll
        for (int j = 0; j < NX; ++j) {
            const int d = r % R.p;
            r /= R.p;
            xi[j] = R.gx[d];
            w *= R.gw[d];
        }
        return w;
    }
    int q = i;
    if (R.w0 > T(0)) {
        if (q == 0)
            return R.w0;
        --q;
    }
    const bool neg = q >= NX;
    const int a = neg ? q - NX : q;
#pragma unroll
    for (int j = 0; j < NX; ++j)
        if (j == a)
            xi[j] = neg ? -R.spread : R.spread;
    return R.wi;
}

// L L^T + v v^T = L' L'^T for a lower factor with a positive diagonal
// (rank-one Cholesky update by plane rotations; v is overwritten)
template <typename T, int N>
PSS_INL void chol_update(T (&L)[N][N], T (&v)[N])
{
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const T lkk = L[k][k];
        const T r = psqrt(pfma(lkk, lkk, v[k] * v[k]));
        const T il = T(1) / lkk;
        const T ic = lkk / r; // 1 / c
        const T s = v[k] * il, c = r * il;
        L[k][k] = r;
#pragma unroll
        for (int i = k + 1; i < N; ++i) {
            const T l = (L[i][k] + s * v[i]) * ic;
            v[i] = c * v[i] - s * l;
            L[i][k] = l;
        }
    }
}

// Generalised SLR at N(m, N N^T) in deviation form.  img(dl, e, v) returns
// the image deviation e = E[z | x = m + dl] - r and, for VAR models (NZ = 1),
// the conditional variance v = V[z | x = m + dl].  With the rule's points
// (sum w xi = 0, sum w xi xi^T = I):
//   ebar = sum w_i e_i,  D = sum w_i e_i xi_i^T,  G = D N^{-1},
//   off  = r + ebar - G m,
//   S S^T = noise + sum w_i rho_i rho_i^T,  rho_i = e_i - ebar - D xi_i,
// where noise is Sn Sn^T (additive) or sum w_i v_i (VAR: the E[V[z|x]] term).
// sum w rho rho^T equals Zx Zx^T - G N N^T G^T, so S is the paper's
// DownDate(Tria([noise, Zx]), G N) without the subtraction.
template <typename T, int NX, int NZ, bool VAR, class Img>
PSS_INL void rule_slr(const RuleSpec<T> &R, const Marg<T, NX> &mg, const T (&r)[NZ],
                      const T (&Sn)[NZ][NZ], Img img, T (&G)[NZ][NX], T (&off)[NZ],
                      T (&S)[NZ][NZ])
{
    static_assert(!VAR || NZ == 1, "state-dependent noise is built for scalar outputs");
    T ebar[NZ], D[NZ][NX];
    T vs = T(0);
#pragma unroll
    for (int a = 0; a < NZ; ++a) {
        ebar[a] = T(0);
#pragma unroll
        for (int j = 0; j < NX; ++j)
            D[a][j] = T(0);
    }
    for (int i = 0; i < R.np; ++i) {
        T xi[NX], dl[NX], e[NZ], v = T(0);
        const T w = rule_point(R, i, xi);
#pragma unroll
        for (int a = 0; a < NX; ++a) {
            T s = T(0);
#pragma unroll
            for (int b = 0; b <= a; ++b)
                s = pfma(mg.N[a][b], xi[b], s);
            dl[a] = s;
        }
        img(dl, e, v);
        vs = pfma(w, v, vs);
#pragma unroll
        for (int a = 0; a < NZ; ++a) {
            ebar[a] = pfma(w, e[a], ebar[a]);
#pragma unroll
            for (int j = 0; j < NX; ++j)
                D[a][j] = pfma(w * e[a], xi[j], D[a][j]);
        }
    }
    rsolve_lower(D, mg.N, G);
    T Gm[NZ];
    mv(G, mg.m, Gm);
#pragma unroll
    for (int a = 0; a < NZ; ++a)
        off[a] = (r[a] + ebar[a]) - Gm[a];
    if constexpr (NZ == 1) {
        T acc = VAR ? vs : Sn[0][0] * Sn[0][0];
        for (int i = 0; i < R.np; ++i) {
            T xi[NX], dl[NX], e[1], v;
            const T w = rule_point(R, i, xi);
#pragma unroll
            for (int a = 0; a < NX; ++a) {
                T s = T(0);
#pragma unroll
                for (int b = 0; b <= a; ++b)
                    s = pfma(mg.N[a][b], xi[b], s);
                dl[a] = s;
            }
            img(dl, e, v);
            T rho = e[0] - ebar[0];
#pragma unroll
            for (int j = 0; j < NX; ++j)
                rho = pfma(-D[0][j], xi[j], rho);
            acc = pfma(w * rho, rho, acc);
        }
        S[0][0] = psqrt(acc);
    } else {
#pragma unroll
        for (int a = 0; a < NZ; ++a)
#pragma unroll
            for (int b = 0; b < NZ; ++b)
                S[a][b] = (b <= a) ? Sn[a][b] : T(0);
        for (int i = 0; i < R.np; ++i) {
            T xi[NX], dl[NX], e[NZ], v;
            const T w = rule_point(R, i, xi);
#pragma unroll
            for (int a = 0; a < NX; ++a) {
                T s = T(0);
#pragma unroll
                for (int b = 0; b <= a; ++b)
                    s = pfma(mg.N[a][b], xi[b], s);
                dl[a] = s;
            }
            img(dl, e, v);
            const T sw = psqrt(w);
            T rho[NZ];
#pragma unroll
            for (int a = 0; a < NZ; ++a) {
                T t = e[a] - ebar[a];
#pragma unroll
                for (int j = 0; j < NX; ++j)
                    t = pfma(-D[a][j], xi[j], t);
                rho[a] = sw * t;
            }
            chol_update(S, rho);
        }
    }
}

// --------------------------------------------------------------------------
// coordinated-turn model with a general rule (the same deviation images as
// the dedicated cubature code: the transition through phi, the bearings as
// angles from the bearing of the mean, on the branch nearest to y)
// --------------------------------------------------------------------------
template <typename T>
PSS_INL void ct_rule_transition(const RuleSpec<T> &R, const CTParams<T> &P, const Marg<T, 5> &mg,
                                T (&F)[5][5], T (&c)[5], T (&S)[5][5])
{
    CTPhiMean<T> b;
    ct_phi_mean(P, mg, b);
    rule_slr<T, 5, 5, false>(
        R, mg, b.phi, P.LQ,
        [&](const T (&dl)[5], T (&e)[5], T &v) {
            ct_phi_dev(P, b, dl[2], dl[3], dl[4], e);
            v = T(0);
        },
        F, c, S);
#pragma unroll
    for (int i = 0; i < 5; ++i)
        F[i][i] += T(1);
}

template <typename T>
PSS_INL void ct_rule_bearings(const RuleSpec<T> &R, const CTParams<T> &P, const Marg<T, 5> &mg,
                              const T (&y)[2], T (&H)[2][5], T (&d)[2], T (&S)[2][2])
{
    // bearings and their branch in BranchPrec<T> (FP64 for FP32 kernels)
    using W = typename BranchPrec<T>::type;
    const W pi = W(3.14159265358979323846);
    const W tp = W(6.28318530717958647692);
    W ux[2], uy[2], r2[2], D0[2];
    T r[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const W sx = W(q == 0 ? P.s1x : P.s2x), sy = W(q == 0 ? P.s1y : P.s2y);
        ux[q] = W(mg.m[0]) - sx;
        uy[q] = W(mg.m[1]) - sy;
        r2[q] = ux[q] * ux[q] + uy[q] * uy[q];
        W a = patan2(uy[q], ux[q]) - W(y[q]);
        D0[q] = a - tp * pfloor((a + pi) / tp);
        r[q] = T(W(y[q]) + D0[q]);
    }
    const T Sn[2][2] = {{P.sigma, T(0)}, {T(0), P.sigma}};
    rule_slr<T, 5, 2, false>(
        R, mg, r, Sn,
        [&](const T (&dl)[5], T (&e)[2], T &v) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const W cr = ux[q] * W(dl[1]) - uy[q] * W(dl[0]);
                const W dt = ux[q] * W(dl[0]) + uy[q] * W(dl[1]);
                const W ang = patan2(cr, r2[q] + dt);
                e[q] = T(ang - tp * pfloor((D0[q] + ang + pi) / tp));
            }
            v = T(0);
        },
        H, d, S);
}

// --------------------------------------------------------------------------
// Ricker-Poisson model (Section 6.1), nx = ny = 1:
//   f(x) = x + phi(x), phi(x) = log a - exp(x), noise sqrt(Q);
//   E[y|x] = V[y|x] = b exp(x).
// Deviations at m + dl: phi: -exp(m) expm1(dl); counts: b exp(m) expm1(dl).
// The identity part of f is regressed exactly, so F = 1 + G_phi.
// --------------------------------------------------------------------------
template <typename T>
struct RickerParams {
    T loga, b, sqQ;
};

template <typename T>
PSS_INL void ricker_rule_transition(const RuleSpec<T> &R, const RickerParams<T> &P,
                                    const Marg<T, 1> &mg, T (&F)[1][1], T (&c)[1], T (&S)[1][1])
{
    const T em = vexp(mg.m[0]);
    const T r[1] = {P.loga - em};
    const T Sn[1][1] = {{P.sqQ}};
    rule_slr<T, 1, 1, false>(
        R, mg, r, Sn,
        [&](const T (&dl)[1], T (&e)[1], T &v) {
            e[0] = -em * vexpm1(dl[0]);
            v = T(0);
        },
        F, c, S);
    F[0][0] += T(1);
}

template <typename T>
PSS_INL void ricker_rule_poisson(const RuleSpec<T> &R, const RickerParams<T> &P,
                                 const Marg<T, 1> &mg, T (&H)[1][1], T (&d)[1], T (&S)[1][1])
{
    const T lam = P.b * vexp(mg.m[0]);
    const T r[1] = {lam};
    const T Sn[1][1] = {{T(0)}};
    rule_slr<T, 1, 1, true>(
        R, mg, r, Sn,
        [&](const T (&dl)[1], T (&e)[1], T &v) {
            e[0] = lam * vexpm1(dl[0]);
            v = lam + e[0];
        },
        H, d, S);
}

// first-order Taylor expansion at the mean (Section 4.2)
template <typename T>
PSS_INL void ricker_taylor(const RickerParams<T> &P, const Marg<T, 1> &mt, const Marg<T, 1> &mo,
                           bool trans, bool obs, T (&F)[1][1], T (&c)[1], T (&SL)[1][1],
                           T (&H)[1][1], T (&d)[1], T (&SO)[1][1])
{
    if (trans) {
        const T m = mt.m[0], em = vexp(m);
        F[0][0] = T(1) - em;
        c[0] = (P.loga - em) + em * m; // f(m) - F m
        SL[0][0] = P.sqQ;
    }
    if (obs) {
        const T m = mo.m[0], lam = P.b * vexp(m);
        H[0][0] = lam;
        d[0] = lam - lam * m;
        SO[0][0] = psqrt(lam);
    }
}

} // namespace pss
