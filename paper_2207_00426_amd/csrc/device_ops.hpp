// Square-root parallel filter / smoother elements and associative operators
// (Lemmas 1-4 and Tables 1-5 of the paper), cubature statistical linear
// regression (Section 4.3) and the coordinated-turn bearings model
// (Section 6.2), as per-thread register code for gfx950.
#pragma once

#include "device_math.hpp"

namespace pss {

// filtering / smoothing marginal: mean and lower factor
template <typename T, int NX>
struct Marg {
    T m[NX];
    T N[NX][NX];
};

// filter element Pi^f = {A, b, U, eta, Z} (eq. pi-f); U, Z lower
template <typename T, int NX>
struct FElem {
    T A[NX][NX];
    T b[NX];
    T U[NX][NX];
    T eta[NX];
    T Z[NX][NX];
};

// smoother element Pi^s = {E, g, D}; D lower
template <typename T, int NX>
struct SElem {
    T E[NX][NX];
    T g[NX];
    T D[NX][NX];
};

// ---- component visitors: the flat SoA component order of each object ----
template <typename T, int NX, class Fn>
PSS_INL void visit(Marg<T, NX> &x, Fn &&f)
{
    int c = 0;
#pragma unroll
    for (int i = 0; i < NX; ++i)
        f(c++, x.m[i]);
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j)
            f(c++, x.N[i][j]);
}

template <typename T, int NX, class Fn>
PSS_INL void visit(FElem<T, NX> &x, Fn &&f)
{
    int c = 0;
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j < NX; ++j)
            f(c++, x.A[i][j]);
#pragma unroll
    for (int i = 0; i < NX; ++i)
        f(c++, x.b[i]);
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j)
            f(c++, x.U[i][j]);
#pragma unroll
    for (int i = 0; i < NX; ++i)
        f(c++, x.eta[i]);
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j)
            f(c++, x.Z[i][j]);
}

template <typename T, int NX, class Fn>
PSS_INL void visit(SElem<T, NX> &x, Fn &&f)
{
    int c = 0;
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j < NX; ++j)
            f(c++, x.E[i][j]);
#pragma unroll
    for (int i = 0; i < NX; ++i)
        f(c++, x.g[i]);
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j)
            f(c++, x.D[i][j]);
}

template <int NX> struct Sizes {
    static constexpr int P = tri_size(NX);
    static constexpr int marg = NX + P;
    static constexpr int felem = NX * NX + NX + P + NX + P;
    static constexpr int selem = NX * NX + NX + P;
};

// --------------------------------------------------------------------------
// Lemma 1: filter elements.
// --------------------------------------------------------------------------

// Psi = Tria([[H L, S_Omega], [L, 0]]) (eq. sqrt-filter-init-2 with L =
// S_Lambda_{k-1}; eq. sqrt-filter-step1 with L = N_1^-), returning the blocks
// Psi11 (ny x ny), Psi21 (nx x ny), Psi22 (nx x nx).
template <typename T, int NX, int NY>
PSS_INL void psi_blocks(const T (&H)[NY][NX], const T (&L)[NX][NX], const T (&SO)[NY][NY],
                        T (&P11)[NY][NY], T (&P21)[NX][NY], T (&P22)[NX][NX])
{
    constexpr int R = NY + NX, C = NX + NY;
    T M[R][C];
    T HL[NY][NX];
    mm_lower(H, L, HL);
#pragma unroll
    for (int i = 0; i < NY; ++i) {
#pragma unroll
        for (int j = 0; j < NX; ++j)
            M[i][j] = HL[i][j];
#pragma unroll
        for (int j = 0; j < NY; ++j)
            M[i][NX + j] = (j <= i) ? SO[i][j] : T(0);
    }
#pragma unroll
    for (int i = 0; i < NX; ++i) {
#pragma unroll
        for (int j = 0; j < NX; ++j)
            M[NY + i][j] = (j <= i) ? L[i][j] : T(0);
#pragma unroll
        for (int j = 0; j < NY; ++j)
            M[NY + i][NX + j] = T(0);
    }
    lq_rows<R, NX>(M);
#pragma unroll
    for (int i = 0; i < NY; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j)
            P11[i][j] = M[i][j];
#pragma unroll
    for (int i = 0; i < NX; ++i) {
#pragma unroll
        for (int j = 0; j < NY; ++j)
            P21[i][j] = M[NY + i][j];
#pragma unroll
        for (int j = 0; j <= i; ++j)
            P22[i][j] = M[NY + i][NY + j];
    }
}

// Z_k = F^T H^T Y^{-T} (nx x ny), stored squared as Tria([Z_k, 0]); and
// eta_k = Z_k Y^{-1} r with r = y_k - H_k c_{k-1} - d_k.
template <typename T, int NX, int NY>
PSS_INL void info_part(const T (&F)[NX][NX], const T (&H)[NY][NX], const T (&Y)[NY][NY],
                       const T (&r)[NY], FElem<T, NX> &e)
{
    T HF[NY][NX];
    mm(H, F, HF);
    T HFt[NX][NY];
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int a = 0; a < NY; ++a)
            HFt[i][a] = HF[a][i];
    T Zr[NX][NY];
    rsolve_lower_t(HFt, Y, Zr);
    T u[NY];
    lsolve_lower(Y, r, u);
    mv(Zr, u, e.eta);
    tria_rect(Zr, e.Z);
}

// Table 2 (1 < k <= n), square-root column.  b_k uses d_k.
template <typename T, int NX, int NY>
PSS_INL void filter_element(const T (&F)[NX][NX], const T (&c)[NX], const T (&SL)[NX][NX],
                            const T (&H)[NY][NX], const T (&d)[NY], const T (&SO)[NY][NY],
                            const T (&y)[NY], FElem<T, NX> &e)
{
    T P11[NY][NY], P21[NX][NY];
    psi_blocks(H, SL, SO, P11, P21, e.U);
    T K[NX][NY];
    rsolve_lower(P21, P11, K);
    // A = (I - K H) F
    T IKH[NX][NX];
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j < NX; ++j) {
            T s = (i == j) ? T(1) : T(0);
#pragma unroll
            for (int a = 0; a < NY; ++a)
                s = pfma(-K[i][a], H[a][j], s);
            IKH[i][j] = s;
        }
    mm(IKH, F, e.A);
    T Hc[NY], r[NY];
    mv(H, c, Hc);
#pragma unroll
    for (int a = 0; a < NY; ++a)
        r[a] = y[a] - Hc[a] - d[a];
    T Kr[NX];
    mv(K, r, Kr);
#pragma unroll
    for (int i = 0; i < NX; ++i)
        e.b[i] = c[i] + Kr[i];
    info_part(F, H, P11, r, e);
}

// Table 1 (k = 1), square-root column.
template <typename T, int NX, int NY>
PSS_INL void filter_element_first(const T (&m0)[NX], const T (&N0)[NX][NX], const T (&F)[NX][NX],
                                  const T (&c)[NX], const T (&SL)[NX][NX], const T (&H)[NY][NX],
                                  const T (&d)[NY], const T (&SO)[NY][NY], const T (&y)[NY],
                                  FElem<T, NX> &e)
{
    T mp[NX];
    mv(F, m0, mp);
#pragma unroll
    for (int i = 0; i < NX; ++i)
        mp[i] += c[i];
    T FN[NX][NX], Np[NX][NX];
    mm_lower(F, N0, FN);
    tria_dense_lower(FN, SL, Np);
    T P11[NY][NY], P21[NX][NY];
    psi_blocks(H, Np, SO, P11, P21, e.U);
    T K[NX][NY];
    rsolve_lower(P21, P11, K);
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j < NX; ++j)
            e.A[i][j] = T(0);
    T Hm[NY], v[NY];
    mv(H, mp, Hm);
#pragma unroll
    for (int a = 0; a < NY; ++a)
        v[a] = y[a] - Hm[a] - d[a];
    T Kv[NX];
    mv(K, v, Kv);
#pragma unroll
    for (int i = 0; i < NX; ++i)
        e.b[i] = mp[i] + Kv[i];
    T Hc[NY], r[NY];
    mv(H, c, Hc);
#pragma unroll
    for (int a = 0; a < NY; ++a)
        r[a] = y[a] - Hc[a] - d[a];
    info_part(F, H, P11, r, e);
}

// --------------------------------------------------------------------------
// Lemma 2: the square-root filtering operator  (i) (x) (j)  (Table 3).
//   Xi = Tria([[U_i^T Z_j, I], [Z_j, 0]])
//   Tm = U_i Xi11^{-T},  G = I - Tm Xi21^T  (= (I + C_i J_j)^{-1})
//   A  = A_j G A_i,  b = A_j G (b_i + U_i U_i^T eta_j) + b_j
//   U  = Tria([A_j Tm, U_j])
//   eta = A_i^T G^T (eta_j - Z_j Z_j^T b_i) + eta_i
//   Z  = Tria([A_i^T Xi22, Z_i])
// --------------------------------------------------------------------------
// Xi input block [[U_i^T Z_j, I], [Z_j, 0]] of Table 3 with Z_j given as its
// first NZ columns (lower trapezoidal NX x NZ).  NZ = NX is the general
// case; a finest-level element stores Z_j = Tria([Z_k, 0]) with Z_k of ny
// columns (Lemma 1), whose columns from ny on are exactly zero, so NZ = ny
// drops them and the block has NZ + NX columns instead of 2 NX.  Columns can
// be dropped or reordered freely: Tria only depends on the Gram matrix.
template <typename T, int NX, int NZ>
PSS_INL void xi_block(const T (&Ui)[NX][NX], const T (&Zj)[NX][NZ], T (&M)[2 * NX][NZ + NX])
{
#pragma unroll
    for (int r = 0; r < NX; ++r) {
#pragma unroll
        for (int a = 0; a < NZ; ++a) {
            const int t0 = r > a ? r : a;
            T s = Ui[t0][r] * Zj[t0][a];
#pragma unroll
            for (int t = t0 + 1; t < NX; ++t)
                s = pfma(Ui[t][r], Zj[t][a], s);
            M[r][a] = s;
            M[NX + r][a] = Zj[r][a];
        }
#pragma unroll
        for (int j = 0; j < NX; ++j) {
            M[r][NZ + j] = (r == j) ? T(1) : T(0);
            M[NX + r][NZ + j] = T(0);
        }
    }
}

// ---- element views ---------------------------------------------------------
// The operators below read their operands through views, one field at a time
// and only when it is needed, so an operand may stay in LDS or memory instead
// of occupying registers for the whole operator.  FRegV views an element in
// registers; FSlotV views one stored flat, component c at p[c * ld] in the
// component order of visit() (an LDS slot: p = lds + slot, ld = threads).
// Setters write through the view.
template <typename T, int NX>
struct FRegV {
    FElem<T, NX> *e;
    PSS_INL T A(int i, int j) const { return e->A[i][j]; }
    PSS_INL T b(int i) const { return e->b[i]; }
    PSS_INL T U(int i, int j) const { return e->U[i][j]; }
    PSS_INL T eta(int i) const { return e->eta[i]; }
    PSS_INL T Z(int i, int j) const { return e->Z[i][j]; }
    PSS_INL void sA(int i, int j, T v) const { e->A[i][j] = v; }
    PSS_INL void sb(int i, T v) const { e->b[i] = v; }
    PSS_INL void sU(int i, int j, T v) const { e->U[i][j] = v; }
    PSS_INL void seta(int i, T v) const { e->eta[i] = v; }
    PSS_INL void sZ(int i, int j, T v) const { e->Z[i][j] = v; }
};

template <typename T, int NX, typename I>
struct FSlotV {
    T *p;
    I ld;
    static constexpr int oA = 0, ob = NX * NX, oU = ob + NX, oe = oU + tri_size(NX),
                         oZ = oe + NX;
    PSS_INL T A(int i, int j) const { return p[(I)(oA + i * NX + j) * ld]; }
    PSS_INL T b(int i) const { return p[(I)(ob + i) * ld]; }
    PSS_INL T U(int i, int j) const { return p[(I)(oU + tri_idx(i, j)) * ld]; }
    PSS_INL T eta(int i) const { return p[(I)(oe + i) * ld]; }
    PSS_INL T Z(int i, int j) const { return p[(I)(oZ + tri_idx(i, j)) * ld]; }
    PSS_INL void sA(int i, int j, T v) const { p[(I)(oA + i * NX + j) * ld] = v; }
    PSS_INL void sb(int i, T v) const { p[(I)(ob + i) * ld] = v; }
    PSS_INL void sU(int i, int j, T v) const { p[(I)(oU + tri_idx(i, j)) * ld] = v; }
    PSS_INL void seta(int i, T v) const { p[(I)(oe + i) * ld] = v; }
    PSS_INL void sZ(int i, int j, T v) const { p[(I)(oZ + tri_idx(i, j)) * ld] = v; }
};

template <typename T, int NX, class VS, class VD>
PSS_INL void felem_copy(const VS &s, const VD &d)
{
#pragma unroll
    for (int i = 0; i < NX; ++i) {
#pragma unroll
        for (int j = 0; j < NX; ++j)
            d.sA(i, j, s.A(i, j));
        d.sb(i, s.b(i));
        d.seta(i, s.eta(i));
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            d.sU(i, j, s.U(i, j));
            d.sZ(i, j, s.Z(i, j));
        }
    }
}

template <typename T, int NX, class V>
PSS_INL void load_lower_U(const V &v, T (&L)[NX][NX])
{
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j < NX; ++j)
            L[i][j] = (j <= i) ? v.U(i, j) : T(0);
}

template <typename T, int NX, class V>
PSS_INL void load_lower_Z(const V &v, T (&L)[NX][NX])
{
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j < NX; ++j)
            L[i][j] = (j <= i) ? v.Z(i, j) : T(0);
}

template <typename T, int NX, int NZ, class V>
PSS_INL void load_Z_cols(const V &v, T (&Z)[NX][NZ])
{
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int a = 0; a < NZ; ++a)
            Z[i][a] = (a <= i) ? v.Z(i, a) : T(0);
}

template <typename T, int NX, class V>
PSS_INL void load_A(const V &v, T (&A)[NX][NX])
{
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j < NX; ++j)
            A[i][j] = v.A(i, j);
}

// Table 3 through views.  The output is written field by field, b, U, eta,
// Z, A, each after the last read of the input fields it may overwrite, so
// `o` may view the same storage as `ei` or as `ej`.  Only the first NZ
// columns of Z_j are read (see xi_block).
//
// The mean is formed in update form: with G = (I + C_i J_j)^{-1},
//   G (b_i + C_i eta_j) = b_i + G C_i (eta_j - J_j b_i)
//                       = b_i + Tm Tm^T (eta_j - J_j b_i),
// since G C_i = U_i (I + U_i^T J_j U_i)^{-1} U_i^T = Tm Tm^T.  It equals the
// printed b of Table 3 but never multiplies the (possibly large) mean by G:
// G itself is formed as I - Tm Xi21^T, which cancels when C_i J_j is large
// (a broad prefix against the information of a long span, or a fold of
// several steps), and in FP32 that cancellation cost ~3 digits of the mean.
template <typename T, int NX, int NZ, class VI, class VJ, class VO>
PSS_INL void filter_combine_v(const VI &ei, const VJ &ej, const VO &o)
{
    constexpr int C = NZ + NX;
    constexpr int K = cmin(2 * NX, C);
    // bi and q = eta_j - Z_j Z_j^T b_i need the inputs only; computing them
    // first keeps U_i, Z_j out of the Tria below
    T v[NX], q[NX];
    T M[2 * NX][C];
    {
        T Ui[NX][NX], Zj[NX][NZ], etj[NX], bi[NX];
        load_lower_U(ei, Ui);
        load_Z_cols(ej, Zj);
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            etj[i] = ej.eta(i);
            bi[i] = ei.b(i);
        }
        T zt[NZ];
#pragma unroll
        for (int a = 0; a < NZ; ++a) {
            T s = Zj[a][a] * bi[a];
#pragma unroll
            for (int i = a + 1; i < NX; ++i)
                s = pfma(Zj[i][a], bi[i], s);
            zt[a] = s;
        }
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            T s = Zj[i][0] * zt[0];
#pragma unroll
            for (int a = 1; a < NZ && a <= i; ++a)
                s = pfma(Zj[i][a], zt[a], s);
            v[i] = bi[i];
            q[i] = etj[i] - s;
        }
        // Xi = Tria([[U_i^T Z_j, I], [Z_j, 0]])
        xi_block(Ui, Zj, M);
    }
    lq_rows<K, NZ>(M);
    // Tm = U_i Xi11^{-T}, G = I - Tm Xi21^T
    T Tm[NX][NX], G[NX][NX];
    {
        T Ui[NX][NX], X11[NX][NX];
        load_lower_U(ei, Ui);
#pragma unroll
        for (int i = 0; i < NX; ++i)
#pragma unroll
            for (int j = 0; j < NX; ++j)
                X11[i][j] = M[i][j];
        rsolve_lower_t(Ui, X11, Tm);
    }
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j < NX; ++j) {
            T s = (i == j) ? T(1) : T(0);
#pragma unroll
            for (int t = 0; t < NX; ++t)
                s = pfma(-Tm[i][t], M[NX + j][t], s);
            G[i][j] = s;
        }
    T gq[NX];
    mtv(G, q, gq);
    // v <- b_i + Tm Tm^T q (the filtered mean of the span's start)
    {
        T tq[NX], u[NX];
        mtv(Tm, q, tq);
        mv(Tm, tq, u);
#pragma unroll
        for (int i = 0; i < NX; ++i)
            v[i] += u[i];
    }
    // A_j G and A_j Tm; then b = A_j v + b_j
    T AG[NX][NX], AT[NX][NX];
    {
        T Aj[NX][NX];
        load_A(ej, Aj);
        mm(Aj, G, AG);
        mm(Aj, Tm, AT);
        T w[NX];
        mv(Aj, v, w);
#pragma unroll
        for (int i = 0; i < NX; ++i)
            o.sb(i, w[i] + ej.b(i));
    }
    // U = Tria([A_j Tm, U_j])
    {
        T Uj[NX][NX], Un[NX][NX];
        load_lower_U(ej, Uj);
        tria_dense_lower(AT, Uj, Un);
#pragma unroll
        for (int i = 0; i < NX; ++i)
#pragma unroll
            for (int j = 0; j <= i; ++j)
                o.sU(i, j, Un[i][j]);
    }
    T Ai[NX][NX];
    load_A(ei, Ai);
    // eta = A_i^T G^T (eta_j - Z_j Z_j^T b_i) + eta_i
    {
        T aq[NX];
        mtv(Ai, gq, aq);
#pragma unroll
        for (int i = 0; i < NX; ++i)
            o.seta(i, aq[i] + ei.eta(i));
    }
    // Z = Tria([A_i^T Xi22, Z_i]); Xi22 is NX x NZ lower trapezoidal
    {
        T AX[NX][NZ];
#pragma unroll
        for (int a = 0; a < NX; ++a)
#pragma unroll
            for (int c = 0; c < NZ; ++c) {
                T s = Ai[c][a] * M[NX + c][NX + c];
#pragma unroll
                for (int t = c + 1; t < NX; ++t)
                    s = pfma(Ai[t][a], M[NX + t][NX + c], s);
                AX[a][c] = s;
            }
        T Zi[NX][NX], Zn[NX][NX];
        load_lower_Z(ei, Zi);
        tria_cols_lower(AX, Zi, Zn);
#pragma unroll
        for (int i = 0; i < NX; ++i)
#pragma unroll
            for (int j = 0; j <= i; ++j)
                o.sZ(i, j, Zn[i][j]);
    }
    // A = A_j G A_i
    {
        T An[NX][NX];
        mm(AG, Ai, An);
#pragma unroll
        for (int i = 0; i < NX; ++i)
#pragma unroll
            for (int j = 0; j < NX; ++j)
                o.sA(i, j, An[i][j]);
    }
}

template <typename T, int NX>
PSS_INL void filter_combine(const FElem<T, NX> &ei, const FElem<T, NX> &ej, FElem<T, NX> &o)
{
    filter_combine_v<T, NX, NX>(FRegV<T, NX>{const_cast<FElem<T, NX> *>(&ei)},
                            FRegV<T, NX>{const_cast<FElem<T, NX> *>(&ej)}, FRegV<T, NX>{&o});
}

// The operator with a true prefix on the left: every prefix a_1 (x) ... (x)
// a_k has A = 0 (A_1 = 0 in Table 1), so only its b and U, i.e. the
// filtering marginal (m, N), matter, and the result is again such a prefix.
// This is Table 3 with A_i = 0, b_i = m, U_i = N: the Xi22 block and the
// eta/Z outputs drop out.  `o` must not be `p`.
template <typename T, int NX, int NZ, class VJ>
PSS_INL void filter_apply_v(const Marg<T, NX> &p, const VJ &ej, Marg<T, NX> &o)
{
    T Nf[NX][NX];
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j < NX; ++j)
            Nf[i][j] = (j <= i) ? p.N[i][j] : T(0);
    T q[NX];
    T M[2 * NX][NZ + NX];
    {
        // q = eta_j - Z_j Z_j^T m
        T Zj[NX][NZ], zt[NZ];
        load_Z_cols(ej, Zj);
#pragma unroll
        for (int a = 0; a < NZ; ++a) {
            T s = Zj[a][a] * p.m[a];
#pragma unroll
            for (int i = a + 1; i < NX; ++i)
                s = pfma(Zj[i][a], p.m[i], s);
            zt[a] = s;
        }
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            T s = Zj[i][0] * zt[0];
#pragma unroll
            for (int a = 1; a < NZ && a <= i; ++a)
                s = pfma(Zj[i][a], zt[a], s);
            q[i] = ej.eta(i) - s;
        }
        xi_block(Nf, Zj, M);
    }
    lq_rows<NX, NZ>(M);
    // Tm = N Xi11^{-T}; the mean in update form (see filter_combine_v):
    // m' = A_j (m + Tm Tm^T q) + b_j, and N' = Tria([A_j Tm, U_j])
    T Tm[NX][NX];
    {
        T X11[NX][NX];
#pragma unroll
        for (int i = 0; i < NX; ++i)
#pragma unroll
            for (int j = 0; j < NX; ++j)
                X11[i][j] = M[i][j];
        rsolve_lower_t(Nf, X11, Tm);
    }
    T v[NX];
    {
        T tq[NX], u[NX];
        mtv(Tm, q, tq);
        mv(Tm, tq, u);
#pragma unroll
        for (int i = 0; i < NX; ++i)
            v[i] = p.m[i] + u[i];
    }
    T AT[NX][NX];
    {
        T Aj[NX][NX], w[NX];
        load_A(ej, Aj);
        mm(Aj, Tm, AT);
        mv(Aj, v, w);
#pragma unroll
        for (int i = 0; i < NX; ++i)
            o.m[i] = w[i] + ej.b(i);
    }
    T Uj[NX][NX];
    load_lower_U(ej, Uj);
    tria_dense_lower(AT, Uj, o.N);
}

template <typename T, int NX>
PSS_INL void filter_apply(const Marg<T, NX> &p, const FElem<T, NX> &ej, Marg<T, NX> &o)
{
    filter_apply_v<T, NX, NX>(p, FRegV<T, NX>{const_cast<FElem<T, NX> *>(&ej)}, o);
}

// --------------------------------------------------------------------------
// Lemma 3: smoother element (Table 4) for 0 <= k < n.
//   Phi = Tria([[F N^f, S_Lambda], [N^f, 0]]),  E = Phi21 Phi11^{-1},
//   g = m^f - E (F m^f + c),  D = Phi22.
// --------------------------------------------------------------------------
template <typename T, int NX>
PSS_INL void smoother_element(const T (&F)[NX][NX], const T (&c)[NX], const T (&SL)[NX][NX],
                              const Marg<T, NX> &f, SElem<T, NX> &e)
{
    T M[2 * NX][2 * NX];
    T FN[NX][NX];
    mm_lower(F, f.N, FN);
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j < NX; ++j) {
            M[i][j] = FN[i][j];
            M[i][NX + j] = (j <= i) ? SL[i][j] : T(0);
            M[NX + i][j] = (j <= i) ? f.N[i][j] : T(0);
            M[NX + i][NX + j] = T(0);
        }
    lq_rows<2 * NX, NX>(M);
    T P11[NX][NX], P21[NX][NX];
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j < NX; ++j) {
            P11[i][j] = M[i][j];
            P21[i][j] = M[NX + i][j];
        }
    rsolve_lower(P21, P11, e.E);
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
        for (int j = 0; j <= i; ++j)
            e.D[i][j] = M[NX + i][NX + j];
    }
}

// last element of a sequence: E = 0, g = m^f_n, D = N^f_n
template <typename T, int NX>
PSS_INL void smoother_element_last(const Marg<T, NX> &f, SElem<T, NX> &e)
{
#pragma unroll
    for (int i = 0; i < NX; ++i) {
        e.g[i] = f.m[i];
#pragma unroll
        for (int j = 0; j < NX; ++j)
            e.E[i][j] = T(0);
#pragma unroll
        for (int j = 0; j <= i; ++j)
            e.D[i][j] = f.N[i][j];
    }
}

// Smoother element views (as for the filter element): registers, or a flat
// slot with component c at p[c * ld].
template <typename T, int NX>
struct SRegV {
    SElem<T, NX> *e;
    PSS_INL T E(int i, int j) const { return e->E[i][j]; }
    PSS_INL T g(int i) const { return e->g[i]; }
    PSS_INL T D(int i, int j) const { return e->D[i][j]; }
    PSS_INL void sE(int i, int j, T v) const { e->E[i][j] = v; }
    PSS_INL void sg(int i, T v) const { e->g[i] = v; }
    PSS_INL void sD(int i, int j, T v) const { e->D[i][j] = v; }
};

template <typename T, int NX, typename I>
struct SSlotV {
    T *p;
    I ld;
    static constexpr int oE = 0, og = NX * NX, oD = og + NX;
    PSS_INL T E(int i, int j) const { return p[(I)(oE + i * NX + j) * ld]; }
    PSS_INL T g(int i) const { return p[(I)(og + i) * ld]; }
    PSS_INL T D(int i, int j) const { return p[(I)(oD + tri_idx(i, j)) * ld]; }
    PSS_INL void sE(int i, int j, T v) const { p[(I)(oE + i * NX + j) * ld] = v; }
    PSS_INL void sg(int i, T v) const { p[(I)(og + i) * ld] = v; }
    PSS_INL void sD(int i, int j, T v) const { p[(I)(oD + tri_idx(i, j)) * ld] = v; }
};

template <typename T, int NX, class VS, class VD>
PSS_INL void selem_copy(const VS &s, const VD &d)
{
#pragma unroll
    for (int i = 0; i < NX; ++i) {
#pragma unroll
        for (int j = 0; j < NX; ++j)
            d.sE(i, j, s.E(i, j));
        d.sg(i, s.g(i));
#pragma unroll
        for (int j = 0; j <= i; ++j)
            d.sD(i, j, s.D(i, j));
    }
}

// Lemma 4 / Table 5:  (i) (x) (j) = {E_i E_j, E_i g_j + g_i, Tria([E_i D_j, D_i])}
// Every field of `ej` is read before the first write and each field of `ei`
// before the write of the same field, so `o` may view `ei` or `ej`.
template <typename T, int NX, class VI, class VJ, class VO>
PSS_INL void smoother_combine_v(const VI &ei, const VJ &ej, const VO &o)
{
    T Ei[NX][NX], ED[NX][NX], Eg[NX], EE[NX][NX];
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j < NX; ++j)
            Ei[i][j] = ei.E(i, j);
    {
        T Dj[NX][NX], gj[NX], Ej[NX][NX];
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            gj[i] = ej.g(i);
#pragma unroll
            for (int j = 0; j < NX; ++j) {
                Dj[i][j] = (j <= i) ? ej.D(i, j) : T(0);
                Ej[i][j] = ej.E(i, j);
            }
        }
        mm_lower(Ei, Dj, ED);
        mv(Ei, gj, Eg);
        mm(Ei, Ej, EE);
    }
    {
        T Di[NX][NX], Dn[NX][NX];
#pragma unroll
        for (int i = 0; i < NX; ++i)
#pragma unroll
            for (int j = 0; j < NX; ++j)
                Di[i][j] = (j <= i) ? ei.D(i, j) : T(0);
        tria_dense_lower(ED, Di, Dn);
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            o.sg(i, Eg[i] + ei.g(i));
#pragma unroll
            for (int j = 0; j <= i; ++j)
                o.sD(i, j, Dn[i][j]);
        }
    }
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j < NX; ++j)
            o.sE(i, j, EE[i][j]);
}

template <typename T, int NX>
PSS_INL void smoother_combine(const SElem<T, NX> &ei, const SElem<T, NX> &ej, SElem<T, NX> &o)
{
    smoother_combine_v<T, NX>(SRegV<T, NX>{const_cast<SElem<T, NX> *>(&ei)},
                              SRegV<T, NX>{const_cast<SElem<T, NX> *>(&ej)}, SRegV<T, NX>{&o});
}

// element (x) true suffix: a suffix a_k (x) ... (x) a_n has E = 0, so it is a
// smoothing marginal (g, D) = (m^s, N^s); Table 5 with E_j = 0.
template <typename T, int NX, class VI>
PSS_INL void smoother_apply_v(const VI &ei, const Marg<T, NX> &s, Marg<T, NX> &o)
{
    T Ei[NX][NX], ED[NX][NX], Eg[NX], Di[NX][NX];
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j < NX; ++j)
            Ei[i][j] = ei.E(i, j);
    mm_lower(Ei, s.N, ED);
    mv(Ei, s.m, Eg);
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j < NX; ++j)
            Di[i][j] = (j <= i) ? ei.D(i, j) : T(0);
    tria_dense_lower(ED, Di, o.N);
#pragma unroll
    for (int i = 0; i < NX; ++i)
        o.m[i] = Eg[i] + ei.g(i);
}

template <typename T, int NX>
PSS_INL void smoother_apply(const SElem<T, NX> &ei, const Marg<T, NX> &s, Marg<T, NX> &o)
{
    smoother_apply_v<T, NX>(SRegV<T, NX>{const_cast<SElem<T, NX> *>(&ei)}, s, o);
}

// --------------------------------------------------------------------------
// Coordinated-turn bearings-only model (Section 6.2).
// --------------------------------------------------------------------------
template <typename T>
struct CTParams {
    T dt;
    T s1x, s1y, s2x, s2y;
    T sigma;
    T LQ[5][5]; // lower factor of Q(theta)
};

PSS_INL double psin(double x) { return sin(x); }
PSS_INL float psin(float x) { return sinf(x); }
PSS_INL double pcos(double x) { return cos(x); }
PSS_INL float pcos(float x) { return cosf(x); }
PSS_INL double patan2(double y, double x) { return atan2(y, x); }
PSS_INL float patan2(float y, float x) { return atan2f(y, x); }
PSS_INL double pfloor(double x) { return floor(x); }
PSS_INL float pfloor(float x) { return floorf(x); }

template <typename T>
PSS_INL T sinc_(T u)
{
    return (fabs(u) < T(1e-4)) ? T(1) - u * u / T(6) : psin(u) / u;
}

// transition mean: the exact flow of p' = v, v' = w J v, w' = 0 over dt
template <typename T>
PSS_INL void ct_f(const CTParams<T> &P, const T (&x)[5], T (&o)[5])
{
    const T a = x[4] * P.dt;
    const T h = T(0.5) * a;
    const T sh = sinc_(h);
    const T s1 = P.dt * sinc_(a);        // sin(w dt) / w
    const T s2 = P.dt * h * sh * sh;     // (1 - cos(w dt)) / w
    const T ca = pcos(a), sa = psin(a);
    o[0] = x[0] + s1 * x[2] - s2 * x[3];
    o[1] = x[1] + s2 * x[2] + s1 * x[3];
    o[2] = ca * x[2] - sa * x[3];
    o[3] = sa * x[2] + ca * x[3];
    o[4] = x[4];
}

// Precision in which the bearings are formed and their branch is chosen.  An
// image crossing the cut opposite the measurement jumps by 2 pi, so which
// side a point falls on is an integer decision; FP32 kernels take it in FP64
// (from the same FP32 inputs), as the FP64 reference does, and round the
// small deviations it yields back afterwards.  Without this an FP32 sigma
// point 1e-7 rad from the cut chose the other branch than FP64 did.
template <typename T>
struct BranchPrec {
    using type = T;
};
template <>
struct BranchPrec<float> {
    using type = double;
};

template <typename T>
PSS_INL T wrap_near(T a, T ref)
{ // ref + (a - ref) reduced to [-pi, pi)
    const T pi = T(3.14159265358979323846);
    const T tp = T(6.28318530717958647692);
    T dlt = a - ref;
    dlt = dlt - tp * pfloor((dlt + pi) / tp);
    return ref + dlt;
}

// bearings of both sensors, on the branch nearest to y
template <typename T>
PSS_INL void ct_h(const CTParams<T> &P, const T (&x)[5], const T (&y)[2], T (&o)[2])
{
    using W = typename BranchPrec<T>::type;
    o[0] = T(wrap_near(patan2(W(x[1]) - W(P.s1y), W(x[0]) - W(P.s1x)), W(y[0])));
    o[1] = T(wrap_near(patan2(W(x[1]) - W(P.s2y), W(x[0]) - W(P.s2x)), W(y[1])));
}

// --------------------------------------------------------------------------
// First-order Taylor linearisation (Section 4.2, the iterated extended
// smoother): F = Jacobian of f at the nominal mean m, c = f(m) - F m,
// S_Lambda = chol Q; H = Jacobian of the bearings at m, d = h~(m) - H m
// (h~ on the branch nearest to y), S_Omega = sigma I.  The nominal factor is
// not used.
// --------------------------------------------------------------------------
// g1 = d/dw [sin(w dt)/w] / dt^2 = (a cos a - sin a) / a^2 and
// g2 = d/dw [(1 - cos(w dt))/w] / dt^2 = (a sin a - 1 + cos a) / a^2, a = w dt.
// Both closed forms cancel as a -> 0 (relative error ~ eps / a^2), so below
// a type-dependent switch point their power series are used.
template <typename T> struct TaylorSwitch;
template <> struct TaylorSwitch<double> { static constexpr double a = 1e-2; };
template <> struct TaylorSwitch<float> { static constexpr float a = 0.3f; };

template <typename T>
PSS_INL void ct_dsw(T a, T &g1, T &g2)
{
    if (fabs(a) < TaylorSwitch<T>::a) {
        const T a2 = a * a;
        g1 = a * (T(-1) / T(3) + a2 * (T(1) / T(30) + a2 * (T(-1) / T(840) + a2 / T(45360))));
        g2 = T(0.5) + a2 * (T(-1) / T(8) + a2 * (T(1) / T(144) - a2 / T(5760)));
    } else {
        const T ca = pcos(a), sa = psin(a), r = T(1) / (a * a);
        g1 = (a * ca - sa) * r;
        g2 = (a * sa - T(1) + ca) * r;
    }
}

template <typename T>
PSS_INL void ct_taylor_transition(const CTParams<T> &P, const Marg<T, 5> &mg, T (&F)[5][5],
                                  T (&c)[5], T (&S)[5][5])
{
    const T dt = P.dt, a = mg.m[4] * dt, h = T(0.5) * a;
    const T sh = sinc_(h);
    const T s1 = dt * sinc_(a), s2 = dt * h * sh * sh;
    const T ca = pcos(a), sa = psin(a), vx = mg.m[2], vy = mg.m[3];
    T g1, g2;
    ct_dsw(a, g1, g2);
    const T d1 = dt * dt * g1, d2 = dt * dt * g2;
#pragma unroll
    for (int i = 0; i < 5; ++i)
#pragma unroll
        for (int j = 0; j < 5; ++j)
            F[i][j] = T(0);
    F[0][0] = T(1);
    F[0][2] = s1;
    F[0][3] = -s2;
    F[0][4] = d1 * vx - d2 * vy;
    F[1][1] = T(1);
    F[1][2] = s2;
    F[1][3] = s1;
    F[1][4] = d2 * vx + d1 * vy;
    F[2][2] = ca;
    F[2][3] = -sa;
    F[2][4] = -dt * (sa * vx + ca * vy);
    F[3][2] = sa;
    F[3][3] = ca;
    F[3][4] = dt * (ca * vx - sa * vy);
    F[4][4] = T(1);
    T fx[5];
    ct_f(P, mg.m, fx);
    T Fm[5];
    mv(F, mg.m, Fm);
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        c[i] = fx[i] - Fm[i];
#pragma unroll
        for (int j = 0; j < 5; ++j)
            S[i][j] = P.LQ[i][j];
    }
}

template <typename T>
PSS_INL void ct_taylor_bearings(const CTParams<T> &P, const Marg<T, 5> &mg, const T (&y)[2],
                                T (&H)[2][5], T (&d)[2], T (&S)[2][2])
{
    const T sx[2] = {P.s1x, P.s2x}, sy[2] = {P.s1y, P.s2y};
    T hx[2];
    ct_h(P, mg.m, y, hx);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const T dx = mg.m[0] - sx[s], dy = mg.m[1] - sy[s];
        const T r = T(1) / (dx * dx + dy * dy);
        H[s][0] = -dy * r;
        H[s][1] = dx * r;
        H[s][2] = H[s][3] = H[s][4] = T(0);
        d[s] = hx[s] - (H[s][0] * mg.m[0] + H[s][1] * mg.m[1]);
        S[s][0] = s == 0 ? P.sigma : T(0);
        S[s][1] = s == 1 ? P.sigma : T(0);
    }
}

// --------------------------------------------------------------------------
// Cubature SLR (Section 4.3) in the residual form.  With the sigma points
// X+-_i = m +- sqrt(nx) N e_i (equal weights 1/(2 nx)) and their images
// written as z+-_i = r + e+-_i (a common reference r plus deviations),
//   zbar = r + mean(e),
//   G    = [(e+_i - e-_i) / (2 sqrt(nx))]_i N^{-1},   off = zbar - G m,
//   S    = Tria([R, S_noise]),  R = [((e+_i + e-_i)/2 - mean(e)) / sqrt(nx)]_i.
// R R^T equals Zx Zx^T - G N N^T G^T exactly, so S is the paper's
// DownDate(Tria([S_noise, Zx]), G N) without the subtraction.  Passing
// deviations instead of raw images keeps the differences free of
// cancellation when |r| >> |e| (positions far from the origin, bearings).
// --------------------------------------------------------------------------
template <typename T, int NX, int NZ>
PSS_INL void cubature_from_dev(const Marg<T, NX> &mg, const T (&Sn)[NZ][NZ],
                               const T (&ep)[NZ][NX], const T (&em)[NZ][NX], const T (&r)[NZ],
                               T (&G)[NZ][NX], T (&off)[NZ], T (&S)[NZ][NZ])
{
    const T sq = psqrt(T(NX));
    const T w = T(1) / T(2 * NX);
    T Dp[NZ][NX], ebar[NZ];
#pragma unroll
    for (int a = 0; a < NZ; ++a) {
        T s = T(0);
#pragma unroll
        for (int i = 0; i < NX; ++i)
            s += ep[a][i] + em[a][i];
        ebar[a] = s * w;
    }
    const T hd = T(1) / (T(2) * sq);
#pragma unroll
    for (int a = 0; a < NZ; ++a)
#pragma unroll
        for (int i = 0; i < NX; ++i)
            Dp[a][i] = (ep[a][i] - em[a][i]) * hd;
    rsolve_lower(Dp, mg.N, G);
    T Gm[NZ];
    mv(G, mg.m, Gm);
#pragma unroll
    for (int a = 0; a < NZ; ++a)
        off[a] = (r[a] + ebar[a]) - Gm[a];
    const T rs = T(1) / sq;
    T A[NZ][NX + NZ];
#pragma unroll
    for (int a = 0; a < NZ; ++a) {
#pragma unroll
        for (int i = 0; i < NX; ++i)
            A[a][i] = (T(0.5) * (ep[a][i] + em[a][i]) - ebar[a]) * rs;
#pragma unroll
        for (int b = 0; b < NZ; ++b)
            A[a][NX + b] = (b <= a) ? Sn[a][b] : T(0);
    }
    lq_rows<NZ, NX>(A);
#pragma unroll
    for (int a = 0; a < NZ; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b)
            S[a][b] = A[a][b];
}

// column i of sqrt(nx) N: the sigma-point offset d_i
template <typename T, int NX>
PSS_INL void sigma_offset(const Marg<T, NX> &mg, int i, T (&dlt)[NX])
{
    const T sq = psqrt(T(NX));
#pragma unroll
    for (int j = 0; j < NX; ++j)
        dlt[j] = (j >= i) ? sq * mg.N[j][i] : T(0);
}

// Transition SLR of the CT model.  The mean map is f(x) = x + phi(v, w)
// with phi = (s1 vx - s2 vy, s2 vx + s1 vy, -w (s2 vx + s1 vy),
// w (s1 vx - s2 vy), 0), s1 = sin(w dt)/w, s2 = (1 - cos(w dt))/w.  SLR is
// linear in the map and exact for the identity, so F = I + G_phi,
// c = off_phi and the residual is phi's alone; phi only sees the velocity
// and turn-rate coordinates of the sigma points.
//
// The images go to the SLR as phi(m) plus deviations formed directly, never
// as two absolute images subtracted: once the nominal is tight, a sigma
// point's image differs from phi(m) by a small fraction of |v| dt, and the
// subtraction lost that many digits (FP32 relative errors of F up to 1e-4).

// sinc(x + d) - sinc(x) without cancellation.  sinc is even, so the
// difference is taken between X = |x| and X1 = |x + d| with step
// D = X1 - X (a step across zero becomes a small one).  While both are
// below 1/2 the power series is differenced term by term, each term
// carrying the exact factor X1^2 - X^2 = D (X1 + X) (FP32 keeps 4 terms,
// FP64 7: the rest is below a quarter ulp of the leading term); otherwise a
// step below X/2 uses the identity
//   X sin(X + D) - (X + D) sin X
//     = -2 X sin X sin^2(D/2) + X cos X (sin D - D) + D (X cos X - sin X)
// over X (X + D), which leaves only products of small factors (sin D - D
// from its own series), and a larger step differences directly.
template <typename T>
struct SincTerms {
    static constexpr int n = Eps<T>::v > 1e-10 ? 4 : 7;
};
// (-1)^k / (2k + 1)!, k = 1, 2, ...
__host__ __device__ constexpr double sinc_coef(int k)
{
    constexpr double c[8] = {-1.66666666666666657e-01, 8.33333333333333322e-03,
                             -1.98412698412698413e-04, 2.75573192239858925e-06,
                             -2.50521083854417202e-08, 1.60590438368216133e-10,
                             -7.64716373181981641e-13, 2.81145725434552060e-15};
    return c[k - 1];
}

template <typename T>
PSS_INL T sin_minus_id(T d)
{ // sin d - d
    if (fabs(d) < T(0.5)) {
        const T d2 = d * d;
        T t = d * d2, s = T(0);
#pragma unroll
        for (int k = 1; k <= SincTerms<T>::n; ++k) {
            s = s + T(sinc_coef(k)) * t;
            t = t * d2;
        }
        return s;
    }
    return psin(d) - d;
}

template <typename T>
PSS_INL T dsinc(T x, T d)
{
    const T x1 = x + d;
    const T X = fabs(x), X1 = fabs(x1);
    const bool same = (x < T(0)) == (x1 < T(0));
    const T D = same ? (x < T(0) ? -d : d) : X1 - X;
    if (X < T(0.5) && X1 < T(0.5)) {
        const T u = X * X, u1 = X1 * X1, q = D * (X1 + X);
        T h = T(1), uk = u, s = T(0);
#pragma unroll
        for (int k = 1; k <= SincTerms<T>::n; ++k) {
            s = s + T(sinc_coef(k)) * h; // h = sum of u1^i u^(k-1-i)
            h = u1 * h + uk;
            uk = uk * u;
        }
        return q * s;
    }
    if (fabs(D) < T(0.5) * X) {
        const T sx = psin(X), cx = pcos(X), sh = psin(T(0.5) * D);
        const T num = T(-2) * X * sx * sh * sh + X * cx * sin_minus_id(D) + D * (X * cx - sx);
        return num / (X * X1);
    }
    return sinc_(X1) - sinc_(X);
}

// phi at the nominal mean, with the parts its deviations reuse
template <typename T>
struct CTPhiMean {
    T vx, vy, w, a, s1, s2, S, phi[5];
};

template <typename T>
PSS_INL void ct_phi_mean(const CTParams<T> &P, const Marg<T, 5> &mg, CTPhiMean<T> &b)
{
    b.vx = mg.m[2];
    b.vy = mg.m[3];
    b.w = mg.m[4];
    b.a = b.w * P.dt;
    b.S = sinc_(T(0.5) * b.a);
    b.s1 = P.dt * sinc_(b.a);
    b.s2 = P.dt * (T(0.5) * b.a) * b.S * b.S;
    b.phi[0] = b.s1 * b.vx - b.s2 * b.vy;
    b.phi[1] = b.s2 * b.vx + b.s1 * b.vy;
    b.phi[2] = -b.w * b.phi[1];
    b.phi[3] = b.w * b.phi[0];
    b.phi[4] = T(0);
}

// phi(v + dv, w + dw) - phi(v, w): with a = w dt, s1 = dt sinc(a) and
// s2 = dt (a/2) sinc(a/2)^2, the differences of s1 and s2 come from dsinc
// and the rest is products of the offsets.
template <typename T>
PSS_INL void ct_phi_dev(const CTParams<T> &P, const CTPhiMean<T> &b, T dvx, T dvy, T dw,
                        T (&e)[5])
{
    const T da = dw * P.dt;
    const T ds1 = P.dt * dsinc(b.a, da);
    const T dS = dsinc(T(0.5) * b.a, T(0.5) * da), S1 = b.S + dS;
    const T ds2 = P.dt * (T(0.5) * da * S1 * S1 + T(0.5) * b.a * dS * (S1 + b.S));
    const T s1 = b.s1 + ds1, s2 = b.s2 + ds2;
    e[0] = s1 * dvx - s2 * dvy + ds1 * b.vx - ds2 * b.vy;
    e[1] = s2 * dvx + s1 * dvy + ds2 * b.vx + ds1 * b.vy;
    e[2] = -(dw * (b.phi[1] + e[1]) + b.w * e[1]);
    e[3] = dw * (b.phi[0] + e[0]) + b.w * e[0];
    e[4] = T(0);
}

template <typename T>
PSS_INL void ct_slr_transition(const CTParams<T> &P, const Marg<T, 5> &mg, T (&F)[5][5],
                               T (&c)[5], T (&S)[5][5])
{
    CTPhiMean<T> b;
    ct_phi_mean(P, mg, b);
    T ep[5][5], em[5][5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        T dlt[5], zp[5], zm[5];
        sigma_offset(mg, i, dlt);
        ct_phi_dev(P, b, dlt[2], dlt[3], dlt[4], zp);
        ct_phi_dev(P, b, -dlt[2], -dlt[3], -dlt[4], zm);
#pragma unroll
        for (int a = 0; a < 5; ++a) {
            ep[a][i] = zp[a];
            em[a][i] = zm[a];
        }
    }
    cubature_from_dev(mg, P.LQ, ep, em, b.phi, F, c, S);
#pragma unroll
    for (int i = 0; i < 5; ++i)
        F[i][i] += T(1);
}

// Measurement SLR of the two bearings.  With u0 = p(m) - s and a sigma point
// at u0 + du, the bearing is the bearing of u0 plus the angle from u0 to
// u0 + du, atan2(u0 x du, |u0|^2 + u0 . du), so deviations never subtract
// two absolute angles.  Images are read on the branch nearest to y: with
// D0 = wrap(bearing(u0) - y), image - y = wrap(D0 + angle); the deviation
// from D0 carries the 2 pi branch jumps explicitly.
template <typename T>
PSS_INL void ct_slr_bearings(const CTParams<T> &P, const Marg<T, 5> &mg, const T (&y)[2],
                             T (&H)[2][5], T (&d)[2], T (&S)[2][2])
{
    using W = typename BranchPrec<T>::type;
    const W pi = W(3.14159265358979323846);
    const W tp = W(6.28318530717958647692);
    const W sq = psqrt(W(5));
    T ep[2][5], em[2][5], r[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const W sx = W(q == 0 ? P.s1x : P.s2x), sy = W(q == 0 ? P.s1y : P.s2y);
        const W ux = W(mg.m[0]) - sx, uy = W(mg.m[1]) - sy;
        const W r2 = ux * ux + uy * uy;
        W D0 = patan2(uy, ux) - W(y[q]);
        D0 = D0 - tp * pfloor((D0 + pi) / tp);
        r[q] = T(W(y[q]) + D0);
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            // position part of column i of sqrt(nx) N (lower: rows >= i)
            const W d0 = (i == 0) ? sq * W(mg.N[0][0]) : W(0);
            const W d1 = (i <= 1) ? sq * W(mg.N[1][i]) : W(0);
            const W cr = ux * d1 - uy * d0;
            const W dt = ux * d0 + uy * d1;
            const W ap = patan2(cr, r2 + dt);
            const W am = patan2(-cr, r2 - dt);
            // branch jumps of D0 + angle back into [-pi, pi)
            const W kp = pfloor((D0 + ap + pi) / tp);
            const W km = pfloor((D0 + am + pi) / tp);
            ep[q][i] = T(ap - tp * kp);
            em[q][i] = T(am - tp * km);
        }
    }
    const T Sn[2][2] = {{P.sigma, T(0)}, {T(0), P.sigma}};
    cubature_from_dev(mg, Sn, ep, em, r, H, d, S);
}

} // namespace pss
