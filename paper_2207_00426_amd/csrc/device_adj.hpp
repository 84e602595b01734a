// Reverse-mode adjoint of the square-root filter's pseudo-log-likelihood
// (Section 5.1 eq. log-likelihood, Section 5.2 eq. gradient at a frozen
// nominal), per-thread register code for gfx950.
//
// The filtering marginals are the prefixes y_k = y_{k-1} (.) a_k of the
// scan of Lemma 2 (Algorithm 1), and y_{k-1} (.) a_k(Gamma_k) is one Kalman
// step from (m_{k-1}, P_{k-1}) with the linearisation Gamma_k.  The
// log-likelihood is l = sum_k l_k(y_{k-1}, Gamma_k).  Cotangents of the
// Cholesky factors are never formed: every quantity is a function of the
// Grams (P = N N^T, Lambda = S_L S_L^T, Omega = S_O S_O^T), so cotangents
// travel as symmetric Gram cotangents P_bar, Lambda_bar, Omega_bar.
//
// Scan VJP.  With lambda_k = dl/d(m_k, P_k) (total, through every later
// term), the Jacobian of one step with respect to its prefix is
//   dm_k = Phi_k (dm + dP u_k),  dP_k = Phi_k dP Phi_k^T,
//   Phi_k = (I - K_k H_k) F_{k-1},  u_k = F^T H^T W_k v_k,
// (K gain, W = S^{-1} the innovation precision, v the innovation), and l_k
// adds (u_k, (u_k u_k^T - J_k) / 2) with J_k = F^T H^T W H F.  Hence
//   lambda_{k-1} = T_k(lambda_k),
//   T(m_bar, P_bar) = (Phi^T m_bar + u,
//                      Phi^T P_bar Phi + sym(Phi^T m_bar u^T) + Gam),
// an affine map whose family {Phi, u, Gam (symmetric)} is closed under
// composition:  T1 o T2 = {Phi2 Phi1, Phi1^T u2 + u1,
//                          Phi1^T Gam2 Phi1 + sym(Phi1^T u2 u1^T) + Gam1}.
// So the VJP of the filter scan is itself an associative scan, run in
// reverse time from lambda_n = 0 over the same tile / level machinery as the
// smoother: the exclusive suffix of T_k is lambda_k.
//
// Step VJP.  The VJP of y_{k-1} (.) a_k(Gamma_k) plus l_k with respect to
// Gamma_k, given lambda_k = (m_bar, P_bar) -- the apply VJP (Table 3 with a
// true prefix) composed with the element VJP (Lemma 1, Table 2) -- in closed
// form from the step's gain:
//   c_bar     = (I - K H)^T m_bar + H^T W v
//   d_bar     = -K^T m_bar + W v
//   Lam_bar   = (I-KH)^T P_bar (I-KH) + sym((I-KH)^T m_bar (H^T W v)^T)
//               + H^T Sl H,                 Sl = (W v v^T W - W) / 2
//   Om_bar    = K^T P_bar K - sym(K^T m_bar (W v)^T) + Sl
//   F_bar     = c_bar m^T + 2 Lam_bar F P
//   H_bar     = 2 Sl H P^- + W v (m^- + P_k m_bar)^T - (K^T m_bar) m_k^T
//               - 2 K^T P_bar P_k
// Factor cotangents follow from Gram cotangents as X_bar = 2 G_bar X.
#pragma once

#include "device_ops.hpp"

namespace pss {

// full symmetric matrix from a lower-triangle accessor
template <typename T, int N, class Fn>
PSS_INL void sym_from_lower(T (&S)[N][N], Fn &&lo)
{
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            const T v = lo(i, j);
            S[i][j] = v;
            S[j][i] = v;
        }
}

// ---------------------------------------------------------------------------
// One Kalman step in square-root form from the filtering marginal (m, N) of
// state k-1 and Gamma_k: the quantities both halves of the adjoint use.
// ---------------------------------------------------------------------------
template <typename T, int NX, int NY>
struct StepQ {
    T K[NX][NY];   // gain P^- H^T W
    T HF[NY][NX];  // H F
    T G[NY][NX];   // Y^{-1} H F  (J = G^T G)
    T Yi[NY][NY];  // Y^{-1} (lower), Y Y^T = S the innovation covariance
    T w[NY];       // Y^{-1} v
    T Wv[NY];      // W v = Y^{-T} Y^{-1} v
    T u[NX];       // F^T H^T W v = G^T w
};

// Y = Tria([H N^-, S_O]) with N^- = Tria([F N, S_L]); [[Y, 0], [Psi21, Psi22]]
// = Tria([[H N^-, S_O], [N^-, 0]]) gives K = Psi21 Y^{-1} (the blocks of the
// Lemma 1 step, eq. sqrt-filter-step1).  Np / P22 / mp receive N^-, Psi22 and
// m^- when the caller needs them (the Gamma cotangent), else may be ignored.
template <typename T, int NX, int NY>
PSS_INL void adj_step(const T (&F)[NX][NX], const T (&c)[NX], const T (&SL)[NX][NX],
                      const T (&H)[NY][NX], const T (&d)[NY], const T (&SO)[NY][NY],
                      const T (&y)[NY], const Marg<T, NX> &f, StepQ<T, NX, NY> &q,
                      T (&Np)[NX][NX], T (&P22)[NX][NX], T (&mp)[NX])
{
    {
        T FN[NX][NX];
        mm_lower(F, f.N, FN);
        tria_dense_lower(FN, SL, Np);
    }
    T Y[NY][NY], P21[NX][NY];
    psi_blocks(H, Np, SO, Y, P21, P22);
    rsolve_lower(P21, Y, q.K);
    mv(F, f.m, mp);
#pragma unroll
    for (int i = 0; i < NX; ++i)
        mp[i] += c[i];
    T v[NY];
    {
        T Hm[NY];
        mv(H, mp, Hm);
#pragma unroll
        for (int a = 0; a < NY; ++a)
            v[a] = y[a] - Hm[a] - d[a];
    }
    // Y^{-1} by forward substitution on the unit columns
#pragma unroll
    for (int j = 0; j < NY; ++j)
#pragma unroll
        for (int a = 0; a < NY; ++a) {
            if (a < j) {
                q.Yi[a][j] = T(0);
                continue;
            }
            T s = (a == j) ? T(1) : T(0);
#pragma unroll
            for (int t = j; t < a; ++t)
                s = pfma(-Y[a][t], q.Yi[t][j], s);
            q.Yi[a][j] = s * prcp(Y[a][a]);
        }
#pragma unroll
    for (int a = 0; a < NY; ++a) {
        T s = T(0);
#pragma unroll
        for (int t = 0; t <= a; ++t)
            s = pfma(q.Yi[a][t], v[t], s);
        q.w[a] = s;
    }
#pragma unroll
    for (int a = 0; a < NY; ++a) {
        T s = T(0);
#pragma unroll
        for (int t = a; t < NY; ++t)
            s = pfma(q.Yi[t][a], q.w[t], s);
        q.Wv[a] = s;
    }
    mm(H, F, q.HF);
#pragma unroll
    for (int a = 0; a < NY; ++a)
#pragma unroll
        for (int j = 0; j < NX; ++j) {
            T s = T(0);
#pragma unroll
            for (int t = 0; t <= a; ++t)
                s = pfma(q.Yi[a][t], q.HF[t][j], s);
            q.G[a][j] = s;
        }
    mtv(q.G, q.w, q.u);
}

// T_k = {Phi = F - K HF, u, Gam = (u u^T - G^T G) / 2} stored in a smoother
// element's fields (E <- Phi, g <- u, D <- lower triangle of Gam).
template <typename T, int NX, int NY>
PSS_INL void adj_element(const T (&F)[NX][NX], const StepQ<T, NX, NY> &q, SElem<T, NX> &e)
{
#pragma unroll
    for (int i = 0; i < NX; ++i) {
#pragma unroll
        for (int j = 0; j < NX; ++j) {
            T s = F[i][j];
#pragma unroll
            for (int a = 0; a < NY; ++a)
                s = pfma(-q.K[i][a], q.HF[a][j], s);
            e.E[i][j] = s;
        }
        e.g[i] = q.u[i];
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            T s = q.u[i] * q.u[j];
#pragma unroll
            for (int a = 0; a < NY; ++a)
                s = pfma(-q.G[a][i], q.G[a][j], s);
            e.D[i][j] = T(0.5) * s;
        }
    }
}

// (T1 o T2) with T2 applied first, through views; o may view t1 or t2.
// Every field of t2 is read before the first write; t1's Phi and u are read
// before any write, its Gam before the write of Gam.
template <typename T, int NX, class V1, class V2, class VO>
PSS_INL void adj_combine_v(const V1 &t1, const V2 &t2, const VO &o)
{
    T P1[NX][NX], u1[NX], a[NX], PP[NX][NX], X[NX][NX];
#pragma unroll
    for (int i = 0; i < NX; ++i) {
        u1[i] = t1.g(i);
#pragma unroll
        for (int j = 0; j < NX; ++j)
            P1[i][j] = t1.E(i, j);
    }
    {
        T u2[NX], P2[NX][NX], G2[NX][NX];
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            u2[i] = t2.g(i);
#pragma unroll
            for (int j = 0; j < NX; ++j)
                P2[i][j] = t2.E(i, j);
        }
        sym_from_lower(G2, [&](int i, int j) { return t2.D(i, j); });
        mtv(P1, u2, a);   // Phi1^T u2
        mm(P2, P1, PP);   // Phi2 Phi1
        mm(G2, P1, X);    // Gam2 Phi1
    }
    // Gam = Phi1^T X + sym(a u1^T) + Gam1
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            T s = t1.D(i, j);
            s = pfma(T(0.5) * a[i], u1[j], s);
            s = pfma(T(0.5) * u1[i], a[j], s);
#pragma unroll
            for (int t = 0; t < NX; ++t)
                s = pfma(P1[t][i], X[t][j], s);
            o.sD(i, j, s);
        }
#pragma unroll
    for (int i = 0; i < NX; ++i) {
        o.sg(i, a[i] + u1[i]);
#pragma unroll
        for (int j = 0; j < NX; ++j)
            o.sE(i, j, PP[i][j]);
    }
}

// T(lambda) for a suffix value lambda = (m_bar, P_bar) held in a marginal
// (m <- m_bar, N <- lower triangle of P_bar); o must not be lam.
template <typename T, int NX, class V>
PSS_INL void adj_apply_v(const V &t, const Marg<T, NX> &lam, Marg<T, NX> &o)
{
    T Ph[NX][NX], Pb[NX][NX], X[NX][NX], a[NX];
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j < NX; ++j)
            Ph[i][j] = t.E(i, j);
    sym_from_lower(Pb, [&](int i, int j) { return lam.N[i][j]; });
    mtv(Ph, lam.m, a);
    mm(Pb, Ph, X);
#pragma unroll
    for (int i = 0; i < NX; ++i) {
        const T ui = t.g(i);
        o.m[i] = a[i] + ui;
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            T s = t.D(i, j);
            s = pfma(T(0.5) * a[i], t.g(j), s);
            s = pfma(T(0.5) * ui, a[j], s);
#pragma unroll
            for (int q = 0; q < NX; ++q)
                s = pfma(Ph[q][i], X[q][j], s);
            o.N[i][j] = s;
        }
    }
}

// Gram cotangents Lambda_bar (NX x NX, full symmetric) and Omega_bar of the
// step with the suffix cotangent lam = lambda_k; also (I - KH)^T m_bar + H^T
// W v (= c_bar) and -K^T m_bar + W v (= d_bar).
template <typename T, int NX, int NY>
PSS_INL void adj_gram_bars(const T (&H)[NY][NX], const StepQ<T, NX, NY> &q,
                           const Marg<T, NX> &lam, T (&Lb)[NX][NX], T (&Ob)[NY][NY],
                           T (&cb)[NX], T (&db)[NY])
{
    T IKH[NX][NX], Pb[NX][NX], X[NX][NX], h[NX], kb[NY], Sl[NY][NY];
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j < NX; ++j) {
            T s = (i == j) ? T(1) : T(0);
#pragma unroll
            for (int a = 0; a < NY; ++a)
                s = pfma(-q.K[i][a], H[a][j], s);
            IKH[i][j] = s;
        }
    sym_from_lower(Pb, [&](int i, int j) { return lam.N[i][j]; });
    mtv(IKH, lam.m, cb);   // (I - KH)^T m_bar
    mtv(H, q.Wv, h);       // H^T W v
    mtv(q.K, lam.m, kb);   // K^T m_bar
    // Sl = (W v v^T W - W) / 2 with W = Y^{-T} Y^{-1}
#pragma unroll
    for (int a = 0; a < NY; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            T s = T(0);
#pragma unroll
            for (int t = a; t < NY; ++t)
                s = pfma(q.Yi[t][a], q.Yi[t][b], s);
            const T v = T(0.5) * (q.Wv[a] * q.Wv[b] - s);
            Sl[a][b] = v;
            Sl[b][a] = v;
        }
    T SH[NY][NX];
    mm(Sl, H, SH);
    mm(Pb, IKH, X);
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            T s = T(0.5) * (cb[i] * h[j] + h[i] * cb[j]);
#pragma unroll
            for (int a = 0; a < NY; ++a)
                s = pfma(H[a][i], SH[a][j], s);
#pragma unroll
            for (int t = 0; t < NX; ++t)
                s = pfma(IKH[t][i], X[t][j], s);
            Lb[i][j] = s;
            Lb[j][i] = s;
        }
    T KX[NX][NY];
    mm(Pb, q.K, KX);
#pragma unroll
    for (int a = 0; a < NY; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            T s = Sl[a][b] - T(0.5) * (kb[a] * q.Wv[b] + q.Wv[a] * kb[b]);
#pragma unroll
            for (int t = 0; t < NX; ++t)
                s = pfma(q.K[t][a], KX[t][b], s);
            Ob[a][b] = s;
            Ob[b][a] = s;
        }
#pragma unroll
    for (int i = 0; i < NX; ++i)
        cb[i] += h[i];
#pragma unroll
    for (int a = 0; a < NY; ++a)
        db[a] = q.Wv[a] - kb[a];
}

} // namespace pss
