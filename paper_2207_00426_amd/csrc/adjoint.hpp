// Adjoint (reverse-mode) pass of the square-root filter's pseudo-log-
// likelihood: the VJP of the filter scan as a reverse associative scan of
// affine cotangent maps (device_adj.hpp), its finest level built from the
// filtering marginals and the linearisation, and the per-step VJP with
// respect to the linearisation Gamma_k (Section 5.2, eq. gradient, at a
// frozen nominal).
#pragma once

#include "device_adj.hpp"
#include "kernels.hpp"

namespace pss {

// Reverse scan of the cotangent maps T_k, run as a forward scan over the
// time-reversed maps (scan position p holds T_{n-p}); a scan prefix covers
// later times and composes as "later map first".  Elements use the smoother
// element's storage (E <- Phi, g <- u, D <- Gam), prefixes the marginal's
// (m <- m_bar, N <- P_bar, both lower triangles of symmetric matrices).
template <typename T_, int NX_>
struct AdjScan {
    using T = T_;
    static constexpr int NX = NX_;
    using Elem = SElem<T, NX>;
    using Pre = Marg<T, NX>;
    static constexpr int NE = Sizes<NX>::selem;
    static constexpr int NP = Sizes<NX>::marg;
    static constexpr const char *name = "adjoint";
    PSS_INL static SSlotV<T, NX, int> slot(T *lds, int Tb, int s)
    {
        return SSlotV<T, NX, int>{lds + s, Tb};
    }
    PSS_INL static SRegV<T, NX> reg(Elem &e) { return SRegV<T, NX>{&e}; }
    template <int NZ = NX, class VA, class VB, class VO>
    PSS_INL static void combine_v(const VA &a, const VB &b, const VO &o)
    {
        adj_combine_v<T, NX>(b, a, o);
    }
    template <int NZ = NX, class VA>
    PSS_INL static void apply_v(const Pre &p, const VA &a, Pre &o)
    {
        adj_apply_v<T, NX>(a, p, o);
    }
    template <class VS, class VD>
    PSS_INL static void copy_v(const VS &src, const VD &dst)
    {
        selem_copy<T, NX>(src, dst);
    }
};

// theta contraction of the coordinated-turn model: dl/dtheta_j =
// sum_k tr(Lam_bar_k dQ/dtheta_j) + tr(Om_bar_k dR/dtheta_j) with
// dQ/dlog q1 = q1 Qv, dQ/dlog q2 = q2 Qw, dR/dlog sigma = 2 sigma^2 I.
template <typename T, int NX>
struct AdjTheta {
    T dQ1[NX][NX];
    T dQ2[NX][NX];
    T dR;
};

// output of the step VJP: per-step theta terms (terms[c * T_y + t], FP64)
template <typename T, int NX, int NY>
struct ThetaOut {
    static constexpr bool kGamma = false;
    AdjTheta<T, NX> th;
    double *terms;
    int64_t T_y;
};

// output of the step VJP: the cotangent of every input of the step in the
// library's representation (pss_gamma fields at step slot t, factors as
// packed lower triangles), scaled by the sequence's cotangent w_b
template <typename T, int NX, int NY>
struct GammaOut {
    static constexpr bool kGamma = true;
    GammaRef<T, NX, NY> bar; // stride 1, ld = T_y
    const double *w;         // [B] or null (ones)
};

// the finest level of the adjoint scan: element p of sequence b is the map
// of step k = n - p, built from the filtering marginal of state k - 1 and
// Gamma at step slot y_off[b] + k - 1.  down_apply also forms the step's
// cotangents with the suffix lambda_k.
template <typename T, int NX, int NY, class Out>
struct AdjSrc {
    static constexpr bool lazy_up = false, lazy_down = false, fused_down = true;
    static constexpr int leaf_nz = 0;
    GammaRef<T, NX, NY> gam;
    MargRef<T, NX> filt; // ld = T_x
    const T *y;
    int64_t T_y;
    Out out;

    PSS_INL void load(const TileInfo &ti, int64_t p, int64_t &t, T (&F)[NX][NX], T (&c)[NX],
                      T (&SL)[NX][NX], T (&H)[NY][NX], T (&d)[NY], T (&SO)[NY][NY],
                      T (&yy)[NY], Marg<T, NX> &f) const
    {
        t = ti.off + ti.cnt - 1 - p; // step slot of step k = n - p
        gam.load_trans(t, F, c, SL);
        gam.load_obs(t, H, d, SO);
#pragma unroll
        for (int a = 0; a < NY; ++a)
            yy[a] = y[a * T_y + t];
        filt.load(t + ti.b, f); // state k - 1
    }

    PSS_INL void up(const TileInfo &ti, int64_t p, SElem<T, NX> &e) const
    {
        int64_t t;
        T F[NX][NX], c[NX], SL[NX][NX], H[NY][NX], d[NY], SO[NY][NY], yy[NY];
        Marg<T, NX> f;
        load(ti, p, t, F, c, SL, H, d, SO, yy, f);
        StepQ<T, NX, NY> q;
        T Np[NX][NX], P22[NX][NX], mp[NX];
        adj_step(F, c, SL, H, d, SO, yy, f, q, Np, P22, mp);
        adj_element(F, q, e);
    }

    PSS_INL void down_apply(const TileInfo &ti, int64_t p, const Marg<T, NX> &lam,
                            Marg<T, NX> &o) const
    {
        int64_t t;
        T F[NX][NX], c[NX], SL[NX][NX], H[NY][NX], d[NY], SO[NY][NY], yy[NY];
        Marg<T, NX> f;
        load(ti, p, t, F, c, SL, H, d, SO, yy, f);
        StepQ<T, NX, NY> q;
        T Np[NX][NX], P22[NX][NX], mp[NX];
        adj_step(F, c, SL, H, d, SO, yy, f, q, Np, P22, mp);
        {
            SElem<T, NX> e;
            adj_element(F, q, e);
            adj_apply_v<T, NX>(SRegV<T, NX>{&e}, lam, o);
        }
        T Lb[NX][NX], Ob[NY][NY], cb[NX], db[NY];
        adj_gram_bars(H, q, lam, Lb, Ob, cb, db);
        if constexpr (!Out::kGamma) {
            double g1 = 0.0, g2 = 0.0, g3 = 0.0;
#pragma unroll
            for (int i = 0; i < NX; ++i)
#pragma unroll
                for (int j = 0; j < NX; ++j) {
                    g1 += (double)(Lb[i][j] * out.th.dQ1[i][j]);
                    g2 += (double)(Lb[i][j] * out.th.dQ2[i][j]);
                }
#pragma unroll
            for (int a = 0; a < NY; ++a)
                g3 += (double)(Ob[a][a] * out.th.dR);
            out.terms[t] = g1;
            out.terms[out.T_y + t] = g2;
            out.terms[2 * out.T_y + t] = g3;
        } else {
            const T w = out.w ? (T)out.w[ti.b] : T(1);
            // Sl = (W v v^T W - W) / 2
            T Sl[NY][NY];
#pragma unroll
            for (int a = 0; a < NY; ++a)
#pragma unroll
                for (int b = 0; b <= a; ++b) {
                    T s = T(0);
#pragma unroll
                    for (int u = a; u < NY; ++u)
                        s = pfma(q.Yi[u][a], q.Yi[u][b], s);
                    Sl[a][b] = Sl[b][a] = T(0.5) * (q.Wv[a] * q.Wv[b] - s);
                }
            // factor cotangents of S_L and S_O: lower triangles of 2 G_bar S
            T SLb[NX][NX], SOb[NY][NY];
            mm_lower(Lb, SL, SLb);
            mm_lower(Ob, SO, SOb);
            // F_bar = c_bar m^T + 2 Lam_bar F N N^T
            T Fb[NX][NX];
            {
                T FN[NX][NX], X[NX][NX];
                mm_lower(F, f.N, FN);
                mm(Lb, FN, X);
#pragma unroll
                for (int i = 0; i < NX; ++i)
#pragma unroll
                    for (int j = 0; j < NX; ++j) {
                        T s = cb[i] * f.m[j];
#pragma unroll
                        for (int u = 0; u <= j; ++u)
                            s = pfma(T(2) * X[i][u], f.N[j][u], s);
                        Fb[i][j] = s;
                    }
            }
            // H_bar = 2 Sl H P^- + W v (m^- + P_k m_bar)^T - (K^T m_bar) m_k^T
            //         - 2 K^T P_bar P_k,  P^- = Np Np^T, P_k = P22 P22^T,
            //         m_k = m^- + K v with v = Y w
            T Hb[NY][NX];
            {
                T Pm[NX][NX], Pk[NX][NX], Pb[NX][NX], kb[NY], mk[NX], pm[NX];
                sym_from_lower(Pm, [&](int i, int j) {
                    T s = T(0);
                    for (int u = 0; u <= j; ++u)
                        s = pfma(Np[i][u], Np[j][u], s);
                    return s;
                });
                sym_from_lower(Pk, [&](int i, int j) {
                    T s = T(0);
                    for (int u = 0; u <= j; ++u)
                        s = pfma(P22[i][u], P22[j][u], s);
                    return s;
                });
                sym_from_lower(Pb, [&](int i, int j) { return lam.N[i][j]; });
                mtv(q.K, lam.m, kb);
                // K v = Psi21 w (K = Psi21 Y^{-1}) -- recovered as K (Y w)
                T v[NY];
#pragma unroll
                for (int a = 0; a < NY; ++a) {
                    // Y = Yi^{-1}: solve Yi v = w
                    T s = q.w[a];
#pragma unroll
                    for (int u = 0; u < a; ++u)
                        s = pfma(-q.Yi[a][u], v[u], s);
                    v[a] = s * prcp(q.Yi[a][a]);
                }
                mv(Pk, lam.m, pm);
#pragma unroll
                for (int i = 0; i < NX; ++i) {
                    T s = mp[i];
#pragma unroll
                    for (int a = 0; a < NY; ++a)
                        s = pfma(q.K[i][a], v[a], s);
                    mk[i] = s;
                }
                T SH[NY][NX], KP[NY][NX];
                mm(Sl, H, SH);
#pragma unroll
                for (int a = 0; a < NY; ++a)
#pragma unroll
                    for (int j = 0; j < NX; ++j) {
                        T s = T(0);
#pragma unroll
                        for (int u = 0; u < NX; ++u)
                            s = pfma(q.K[u][a], Pb[u][j], s);
                        KP[a][j] = s;
                    }
#pragma unroll
                for (int a = 0; a < NY; ++a)
#pragma unroll
                    for (int j = 0; j < NX; ++j) {
                        T s = q.Wv[a] * (mp[j] + pm[j]) - kb[a] * mk[j];
#pragma unroll
                        for (int u = 0; u < NX; ++u) {
                            s = pfma(T(2) * SH[a][u], Pm[u][j], s);
                            s = pfma(T(-2) * KP[a][u], Pk[u][j], s);
                        }
                        Hb[a][j] = s;
                    }
            }
            // scale by the sequence's cotangent and store
#pragma unroll
            for (int i = 0; i < NX; ++i) {
                cb[i] *= w;
#pragma unroll
                for (int j = 0; j < NX; ++j) {
                    Fb[i][j] *= w;
                    SLb[i][j] *= T(2) * w;
                }
            }
#pragma unroll
            for (int a = 0; a < NY; ++a) {
                db[a] *= w;
#pragma unroll
                for (int j = 0; j < NX; ++j)
                    Hb[a][j] *= w;
#pragma unroll
                for (int j = 0; j < NY; ++j)
                    SOb[a][j] *= T(2) * w;
            }
            out.bar.store_trans(t, Fb, cb, SLb);
            out.bar.store_obs(t, Hb, db, SOb);
        }
    }
};

// finest-level sink of the adjoint scan: the inclusive suffix at the last
// scan position is lambda_0, the cotangent of the prior (m0, P0); with
// m0_bar set it is stored per sequence as (m0_bar [NX][B], N0_bar [P][B],
// N0_bar = lower triangle of 2 P0_bar N0), scaled by w_b
template <typename T, int NX>
struct AdjDst {
    static constexpr bool stageable = false, stage_excl = false;
    T *m0_bar;
    T *N0_bar;
    const T *N0; // packed prior factor
    const double *w;
    int B;
    PSS_INL void put(const TileInfo &ti, int64_t p, const Marg<T, NX> &excl,
                     const Marg<T, NX> &incl) const
    {
        if (!m0_bar || p != ti.cnt - 1)
            return;
        const T s = w ? (T)w[ti.b] : T(1);
        T Pb[NX][NX], L[NX][NX];
        sym_from_lower(Pb, [&](int i, int j) { return incl.N[i][j]; });
#pragma unroll
        for (int i = 0; i < NX; ++i)
#pragma unroll
            for (int j = 0; j < NX; ++j)
                L[i][j] = (j <= i) ? N0[tri_idx(i, j)] : T(0);
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            m0_bar[(int64_t)i * B + ti.b] = s * incl.m[i];
#pragma unroll
            for (int j = 0; j <= i; ++j) {
                T a = T(0);
#pragma unroll
                for (int u = j; u < NX; ++u)
                    a = pfma(Pb[i][u], L[u][j], a);
                N0_bar[(int64_t)tri_idx(i, j) * B + ti.b] = T(2) * s * a;
            }
        }
    }
};

} // namespace pss
