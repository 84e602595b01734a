// Standard (covariance-form) parallel filter and smoother elements and
// operators: the left columns of Tables 1-5.  They reuse the square-root
// path's storage: in a filter element {A, b, C, eta, J} the symmetric C and J
// occupy the packed lower triangles that hold U and Z in square-root form,
// a smoother element {E, g, L} puts L where D is, and a marginal keeps the
// packed lower triangle of its covariance P where the factor N is.  Views
// are read the same way (U(i, j), Z(i, j), D(i, j) with j <= i).
#pragma once

#include "device_ops.hpp"

namespace pss {

// ---- small dense helpers -----------------------------------------------------
// full symmetric matrix from a packed-lower accessor
template <typename T, int N, class Get>
PSS_INL void sym_full(T (&S)[N][N], Get &&get)
{
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            const T v = get(i, j);
            S[i][j] = v;
            S[j][i] = v;
        }
}

// inverse by Gauss-Jordan elimination with partial pivoting (rows swapped by
// selects, so the code stays branch-free and fully unrolled)
template <typename T, int N>
PSS_INL void inv_gj(const T (&M)[N][N], T (&X)[N][N])
{
    T a[N][N];
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) {
            a[i][j] = M[i][j];
            X[i][j] = (i == j) ? T(1) : T(0);
        }
#pragma unroll
    for (int k = 0; k < N; ++k) {
#pragma unroll
        for (int r = k + 1; r < N; ++r) {
            const bool sw = pabs(a[r][k]) > pabs(a[k][k]);
#pragma unroll
            for (int c = 0; c < N; ++c) {
                const T t = a[k][c], u = X[k][c];
                a[k][c] = sw ? a[r][c] : t;
                a[r][c] = sw ? t : a[r][c];
                X[k][c] = sw ? X[r][c] : u;
                X[r][c] = sw ? u : X[r][c];
            }
        }
        const T p = prcp(a[k][k]);
#pragma unroll
        for (int c = 0; c < N; ++c) {
            a[k][c] *= p;
            X[k][c] *= p;
        }
#pragma unroll
        for (int r = 0; r < N; ++r) {
            if (r == k)
                continue;
            const T f = a[r][k];
#pragma unroll
            for (int c = 0; c < N; ++c) {
                a[r][c] = pfma(-f, a[k][c], a[r][c]);
                X[r][c] = pfma(-f, X[k][c], X[r][c]);
            }
        }
    }
}

// lower Cholesky factor of a symmetric positive definite matrix
template <typename T, int N>
PSS_INL void chol_lower(const T (&S)[N][N], T (&L)[N][N])
{
#pragma unroll
    for (int j = 0; j < N; ++j) {
        T s = S[j][j];
#pragma unroll
        for (int t = 0; t < j; ++t)
            s = pfma(-L[j][t], L[j][t], s);
        const T d = psqrt(s);
        L[j][j] = d;
        const T r = prcp(d);
#pragma unroll
        for (int i = j + 1; i < N; ++i) {
            T v = S[i][j];
#pragma unroll
            for (int t = 0; t < j; ++t)
                v = pfma(-L[i][t], L[j][t], v);
            L[i][j] = v * r;
        }
#pragma unroll
        for (int i = 0; i < j; ++i)
            L[i][j] = T(0);
    }
}

// X = B S^{-1} for S = L L^T (B is R x N)
template <typename T, int R, int N>
PSS_INL void rsolve_spd(const T (&B)[R][N], const T (&L)[N][N], T (&X)[R][N])
{
    T W[R][N];
    rsolve_lower_t(B, L, W); // W = B L^{-T}
    rsolve_lower(W, L, X);   // X = W L^{-1}
}

template <typename T, int N>
PSS_INL void gram_full(const T (&L)[N][N], T (&S)[N][N])
{ // S = L L^T, L lower
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            T s = T(0);
#pragma unroll
            for (int t = 0; t <= j; ++t)
                s = pfma(L[i][t], L[j][t], s);
            S[i][j] = s;
            S[j][i] = s;
        }
}

// ---- filter elements (Tables 1 and 2, standard column) -----------------------
// the measurement update shared by both elements: from the predicted (mp, Pp)
// of the element, S = H Pp H^T + Omega, K = Pp H^T S^{-1},
// b = mp + K (y - H mp - d), C = Pp - K S K^T, and, with the transition of the
// element, eta = F^T H^T S^{-1} (y - H c - d), J = F^T H^T S^{-1} H F.
template <typename T, int NX, int NY>
PSS_INL void cov_update(const T (&F)[NX][NX], const T (&c)[NX], const T (&H)[NY][NX],
                        const T (&d)[NY], const T (&Om)[NY][NY], const T (&y)[NY],
                        const T (&mp)[NX], const T (&Pp)[NX][NX], FElem<T, NX> &e,
                        T (&KT)[NX][NY])
{
    T HP[NY][NX], S[NY][NY], LS[NY][NY];
    mm(H, Pp, HP);
#pragma unroll
    for (int a = 0; a < NY; ++a)
#pragma unroll
        for (int q = 0; q < NY; ++q) {
            T s = Om[a][q];
#pragma unroll
            for (int j = 0; j < NX; ++j)
                s = pfma(HP[a][j], H[q][j], s);
            S[a][q] = s;
        }
    chol_lower(S, LS);
    {
        T PH[NX][NY];
#pragma unroll
        for (int i = 0; i < NX; ++i)
#pragma unroll
            for (int a = 0; a < NY; ++a)
                PH[i][a] = HP[a][i];
        rsolve_spd(PH, LS, KT); // K = Pp H^T S^{-1}
    }
    T Hm[NY], v[NY];
    mv(H, mp, Hm);
#pragma unroll
    for (int a = 0; a < NY; ++a)
        v[a] = y[a] - Hm[a] - d[a];
#pragma unroll
    for (int i = 0; i < NX; ++i) {
        T s = mp[i];
#pragma unroll
        for (int a = 0; a < NY; ++a)
            s = pfma(KT[i][a], v[a], s);
        e.b[i] = s;
    }
    // C = Pp - K H Pp (symmetrised)
    T C[NX][NX];
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j < NX; ++j) {
            T s = Pp[i][j];
#pragma unroll
            for (int a = 0; a < NY; ++a)
                s = pfma(-KT[i][a], HP[a][j], s);
            C[i][j] = s;
        }
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j)
            e.U[i][j] = T(0.5) * (C[i][j] + C[j][i]);
    // eta, J with HF = H F and W = S^{-1} H F
    T HF[NY][NX], Hc[NY], r[NY];
    mm(H, F, HF);
    mv(H, c, Hc);
#pragma unroll
    for (int a = 0; a < NY; ++a)
        r[a] = y[a] - Hc[a] - d[a];
    T HFt[NX][NY], WT[NX][NY];
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int a = 0; a < NY; ++a)
            HFt[i][a] = HF[a][i];
    rsolve_spd(HFt, LS, WT); // (S^{-1} H F)^T
#pragma unroll
    for (int i = 0; i < NX; ++i) {
        T s = T(0);
#pragma unroll
        for (int a = 0; a < NY; ++a)
            s = pfma(WT[i][a], r[a], s);
        e.eta[i] = s;
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            T t = T(0);
#pragma unroll
            for (int a = 0; a < NY; ++a)
                t = pfma(WT[i][a], HF[a][j], t);
            e.Z[i][j] = t;
        }
    }
}

// Table 2 (1 < k <= n): mp = c, Pp = Lambda; A = (I - K H) F
template <typename T, int NX, int NY>
PSS_INL void filter_element_cov(const T (&F)[NX][NX], const T (&c)[NX], const T (&SL)[NX][NX],
                                const T (&H)[NY][NX], const T (&d)[NY], const T (&SO)[NY][NY],
                                const T (&y)[NY], FElem<T, NX> &e)
{
    T Lam[NX][NX], Om[NY][NY], KT[NX][NY];
    gram_full(SL, Lam);
    gram_full(SO, Om);
    cov_update(F, c, H, d, Om, y, c, Lam, e, KT);
    // A = (I - K H) F = F - K (H F)
    T HF[NY][NX];
    mm(H, F, HF);
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j < NX; ++j) {
            T s = F[i][j];
#pragma unroll
            for (int a = 0; a < NY; ++a)
                s = pfma(-KT[i][a], HF[a][j], s);
            e.A[i][j] = s;
        }
}

// Table 1 (k = 1): mp = F m0 + c, Pp = F P0 F^T + Lambda; A = 0
template <typename T, int NX, int NY>
PSS_INL void filter_element_first_cov(const T (&m0)[NX], const T (&N0)[NX][NX],
                                      const T (&F)[NX][NX], const T (&c)[NX],
                                      const T (&SL)[NX][NX], const T (&H)[NY][NX],
                                      const T (&d)[NY], const T (&SO)[NY][NY], const T (&y)[NY],
                                      FElem<T, NX> &e)
{
    T mp[NX], P0[NX][NX], FP[NX][NX], Pp[NX][NX], Om[NY][NY];
    mv(F, m0, mp);
#pragma unroll
    for (int i = 0; i < NX; ++i)
        mp[i] += c[i];
    gram_full(N0, P0);
    gram_full(SL, Pp);
    gram_full(SO, Om);
    mm(F, P0, FP);
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j < NX; ++j) {
            T s = Pp[i][j];
#pragma unroll
            for (int t = 0; t < NX; ++t)
                s = pfma(FP[i][t], F[j][t], s);
            Pp[i][j] = s;
        }
    T KT[NX][NY];
    cov_update(F, c, H, d, Om, y, mp, Pp, e, KT);
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j < NX; ++j)
            e.A[i][j] = T(0);
}

// ---- filter operator (Table 3, standard column) ------------------------------
//   M = I + C_i J_j,
//   A = A_j M^{-1} A_i,  b = A_j M^{-1} (b_i + C_i eta_j) + b_j,
//   C = A_j M^{-1} C_i A_j^T + C_j,
//   eta = A_i^T M^{-T} (eta_j - J_j b_i) + eta_i,  J = A_i^T M^{-T} J_j A_i + J_i
// (M^{-T} = (I + J_j C_i)^{-1} since C and J are symmetric).  Output fields
// are written after the last read of the input fields they may overwrite.
template <typename T, int NX, class VI, class VJ, class VO>
PSS_INL void filter_combine_cov_v(const VI &ei, const VJ &ej, const VO &o)
{
    T Ci[NX][NX], Jj[NX][NX], Mi[NX][NX];
    sym_full(Ci, [&](int i, int j) { return ei.U(i, j); });
    sym_full(Jj, [&](int i, int j) { return ej.Z(i, j); });
    {
        T M[NX][NX];
        mm(Ci, Jj, M);
#pragma unroll
        for (int i = 0; i < NX; ++i)
            M[i][i] += T(1);
        inv_gj(M, Mi);
    }
    T bi[NX], etj[NX], u[NX], w[NX];
#pragma unroll
    for (int i = 0; i < NX; ++i) {
        bi[i] = ei.b(i);
        etj[i] = ej.eta(i);
    }
    mv(Ci, etj, u);
    T Jb[NX];
    mv(Jj, bi, Jb);
#pragma unroll
    for (int i = 0; i < NX; ++i) {
        u[i] += bi[i];       // b_i + C_i eta_j
        w[i] = etj[i] - Jb[i]; // eta_j - J_j b_i
    }
    T AM[NX][NX];
    {
        T Aj[NX][NX];
        load_A(ej, Aj);
        mm(Aj, Mi, AM);
        T q[NX];
        mv(AM, u, q);
#pragma unroll
        for (int i = 0; i < NX; ++i)
            o.sb(i, q[i] + ej.b(i));
        // C = AM C_i A_j^T + C_j
        T ACi[NX][NX];
        mm(AM, Ci, ACi);
#pragma unroll
        for (int i = 0; i < NX; ++i)
#pragma unroll
            for (int j = 0; j <= i; ++j) {
                T s = ej.U(i, j), t = ej.U(i, j);
#pragma unroll
                for (int k = 0; k < NX; ++k) {
                    s = pfma(ACi[i][k], Aj[j][k], s);
                    t = pfma(ACi[j][k], Aj[i][k], t);
                }
                o.sU(i, j, T(0.5) * (s + t));
            }
    }
    T Ai[NX][NX];
    load_A(ei, Ai);
    // X = M^{-1} A_i, so that A_i^T M^{-T} = X^T
    T X[NX][NX];
    mm(Mi, Ai, X);
    {
        T q[NX];
        mtv(X, w, q);
#pragma unroll
        for (int i = 0; i < NX; ++i)
            o.seta(i, q[i] + ei.eta(i));
    }
    {
        // J = X^T J_j A_i + J_i
        T JA[NX][NX];
        mm(Jj, Ai, JA);
#pragma unroll
        for (int i = 0; i < NX; ++i)
#pragma unroll
            for (int j = 0; j <= i; ++j) {
                T s = ei.Z(i, j), t = ei.Z(i, j);
#pragma unroll
                for (int k = 0; k < NX; ++k) {
                    s = pfma(X[k][i], JA[k][j], s);
                    t = pfma(X[k][j], JA[k][i], t);
                }
                o.sZ(i, j, T(0.5) * (s + t));
            }
    }
    {
        T An[NX][NX];
        mm(AM, Ai, An);
#pragma unroll
        for (int i = 0; i < NX; ++i)
#pragma unroll
            for (int j = 0; j < NX; ++j)
                o.sA(i, j, An[i][j]);
    }
}

// a true prefix (A = 0) on the left: (m, P) (x) e_j
template <typename T, int NX, class VJ>
PSS_INL void filter_apply_cov_v(const Marg<T, NX> &p, const VJ &ej, Marg<T, NX> &o)
{
    T P[NX][NX], Jj[NX][NX], Mi[NX][NX];
    sym_full(P, [&](int i, int j) { return p.N[i][j]; });
    sym_full(Jj, [&](int i, int j) { return ej.Z(i, j); });
    {
        T M[NX][NX];
        mm(P, Jj, M);
#pragma unroll
        for (int i = 0; i < NX; ++i)
            M[i][i] += T(1);
        inv_gj(M, Mi);
    }
    T etj[NX], u[NX];
#pragma unroll
    for (int i = 0; i < NX; ++i)
        etj[i] = ej.eta(i);
    mv(P, etj, u);
#pragma unroll
    for (int i = 0; i < NX; ++i)
        u[i] += p.m[i];
    T Aj[NX][NX], AM[NX][NX];
    load_A(ej, Aj);
    mm(Aj, Mi, AM);
    T q[NX];
    mv(AM, u, q);
#pragma unroll
    for (int i = 0; i < NX; ++i)
        o.m[i] = q[i] + ej.b(i);
    T AP[NX][NX];
    mm(AM, P, AP);
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            T s = ej.U(i, j), t = ej.U(i, j);
#pragma unroll
            for (int k = 0; k < NX; ++k) {
                s = pfma(AP[i][k], Aj[j][k], s);
                t = pfma(AP[j][k], Aj[i][k], t);
            }
            o.N[i][j] = T(0.5) * (s + t);
        }
}

// ---- smoother elements and operator (Tables 4 and 5, standard column) ---------
//   E = P F^T (F P F^T + Lambda)^{-1},  g = m - E (F m + c),  L = P - E F P;
//   last element {0, m^f_n, P^f_n};  (i) (x) (j) = {E_i E_j, E_i g_j + g_i,
//   E_i L_j E_i^T + L_i}
template <typename T, int NX>
PSS_INL void smoother_element_cov(const T (&F)[NX][NX], const T (&c)[NX], const T (&SL)[NX][NX],
                                  const Marg<T, NX> &f, SElem<T, NX> &e)
{
    T P[NX][NX], FP[NX][NX], Pp[NX][NX], LP[NX][NX];
    sym_full(P, [&](int i, int j) { return f.N[i][j]; });
    mm(F, P, FP);
    gram_full(SL, Pp);
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j < NX; ++j) {
            T s = Pp[i][j];
#pragma unroll
            for (int t = 0; t < NX; ++t)
                s = pfma(FP[i][t], F[j][t], s);
            Pp[i][j] = s;
        }
    chol_lower(Pp, LP);
    {
        T PF[NX][NX];
#pragma unroll
        for (int i = 0; i < NX; ++i)
#pragma unroll
            for (int j = 0; j < NX; ++j)
                PF[i][j] = FP[j][i];
        rsolve_spd(PF, LP, e.E);
    }
    T Fm[NX], Eg[NX];
    mv(F, f.m, Fm);
#pragma unroll
    for (int i = 0; i < NX; ++i)
        Fm[i] += c[i];
    mv(e.E, Fm, Eg);
#pragma unroll
    for (int i = 0; i < NX; ++i) {
        e.g[i] = f.m[i] - Eg[i];
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            T s = P[i][j], t = P[i][j];
#pragma unroll
            for (int k = 0; k < NX; ++k) {
                s = pfma(-e.E[i][k], FP[k][j], s);
                t = pfma(-e.E[j][k], FP[k][i], t);
            }
            e.D[i][j] = T(0.5) * (s + t);
        }
    }
}

template <typename T, int NX, class VI, class VJ, class VO>
PSS_INL void smoother_combine_cov_v(const VI &ei, const VJ &ej, const VO &o)
{
    T Ei[NX][NX], EE[NX][NX], Eg[NX], ELE[NX][NX];
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j < NX; ++j)
            Ei[i][j] = ei.E(i, j);
    {
        T Lj[NX][NX], gj[NX], Ej[NX][NX], EL[NX][NX];
        sym_full(Lj, [&](int i, int j) { return ej.D(i, j); });
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            gj[i] = ej.g(i);
#pragma unroll
            for (int j = 0; j < NX; ++j)
                Ej[i][j] = ej.E(i, j);
        }
        mm(Ei, Lj, EL);
#pragma unroll
        for (int i = 0; i < NX; ++i)
#pragma unroll
            for (int j = 0; j < NX; ++j) {
                T s = T(0);
#pragma unroll
                for (int k = 0; k < NX; ++k)
                    s = pfma(EL[i][k], Ei[j][k], s);
                ELE[i][j] = s;
            }
        mv(Ei, gj, Eg);
        mm(Ei, Ej, EE);
    }
#pragma unroll
    for (int i = 0; i < NX; ++i) {
        o.sg(i, Eg[i] + ei.g(i));
#pragma unroll
        for (int j = 0; j <= i; ++j)
            o.sD(i, j, T(0.5) * (ELE[i][j] + ELE[j][i]) + ei.D(i, j));
    }
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j < NX; ++j)
            o.sE(i, j, EE[i][j]);
}

// element (x) true suffix (E_j = 0): the smoothing marginal (m^s, P^s)
template <typename T, int NX, class VI>
PSS_INL void smoother_apply_cov_v(const VI &ei, const Marg<T, NX> &s, Marg<T, NX> &o)
{
    T Ei[NX][NX], P[NX][NX], EP[NX][NX], Eg[NX];
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j < NX; ++j)
            Ei[i][j] = ei.E(i, j);
    sym_full(P, [&](int i, int j) { return s.N[i][j]; });
    mm(Ei, P, EP);
    mv(Ei, s.m, Eg);
#pragma unroll
    for (int i = 0; i < NX; ++i) {
        o.m[i] = Eg[i] + ei.g(i);
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            T a = ei.D(i, j), b = ei.D(i, j);
#pragma unroll
            for (int k = 0; k < NX; ++k) {
                a = pfma(EP[i][k], Ei[j][k], a);
                b = pfma(EP[j][k], Ei[i][k], b);
            }
            o.N[i][j] = T(0.5) * (a + b);
        }
    }
}

} // namespace pss
