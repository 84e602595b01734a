// Counts the floating-point operations of the library's per-thread register
// code for the coordinated-turn shapes (nx = 5, ny = 2) by instantiating the
// same templates on a counting number type on the host.  Convention: add,
// subtract, multiply, divide, reciprocal and square root count 1, a fused
// multiply-add 2; sign flips, comparisons, selects, absolute values and
// exponent scaling count 0; sin, cos, atan2, log and floor are counted apart
// as transcendentals.  Prints one "name flops transcendentals" line per
// operator.  Test infrastructure: compiled and run by tests/test_flop_counts_cpu.py.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>

namespace fc {
long long g_flop = 0, g_trans = 0;

struct C {
    double v = 0.0;
    C() = default;
    constexpr C(double x) : v(x) {}
};
inline C operator+(C a, C b) { ++g_flop; return C(a.v + b.v); }
inline C operator-(C a, C b) { ++g_flop; return C(a.v - b.v); }
inline C operator*(C a, C b) { ++g_flop; return C(a.v * b.v); }
inline C operator/(C a, C b) { ++g_flop; return C(a.v / b.v); }
inline C operator-(C a) { return C(-a.v); }
inline C &operator+=(C &a, C b) { a = a + b; return a; }
inline C &operator-=(C &a, C b) { a = a - b; return a; }
inline C &operator*=(C &a, C b) { a = a * b; return a; }
inline bool operator<(C a, C b) { return a.v < b.v; }
inline bool operator>(C a, C b) { return a.v > b.v; }
inline bool operator<=(C a, C b) { return a.v <= b.v; }
inline bool operator>=(C a, C b) { return a.v >= b.v; }
inline C pfma(C a, C b, C c) { g_flop += 2; return C(std::fma(a.v, b.v, c.v)); }
inline C prcp(C x) { ++g_flop; return C(1.0 / x.v); }
inline C psqrt(C x) { ++g_flop; return C(std::sqrt(x.v)); }
inline C pabs(C x) { return C(std::fabs(x.v)); }
inline C fabs(C x) { return C(std::fabs(x.v)); }
inline C pmax(C a, C b) { return C(std::fmax(a.v, b.v)); }
inline int pexp(C x) { int e; std::frexp(x.v, &e); return e; }
inline C pldexp(C x, int e) { return C(std::ldexp(x.v, e)); }
inline C plog(C x) { ++g_trans; return C(std::log(x.v)); }
inline C psin(C x) { ++g_trans; return C(std::sin(x.v)); }
inline C pcos(C x) { ++g_trans; return C(std::cos(x.v)); }
inline C patan2(C y, C x) { ++g_trans; return C(std::atan2(y.v, x.v)); }
inline C pfloor(C x) { ++g_trans; return C(std::floor(x.v)); }
} // namespace fc

#include "../paper_2207_00426_amd/csrc/device_adj.hpp"

namespace pss {
template <> struct Eps<fc::C> { static constexpr double v = 2.220446049250313e-16; };
} // namespace pss

using fc::C;
using namespace pss;
constexpr int NX = 5, NY = 2;

// deterministic, well-conditioned operands: every branch of the code takes
// its general path (no skipped reflections)
static double g_seed = 0.1234;
static double rnd()
{
    g_seed = std::fmod(g_seed * 997.0 + 0.31415, 1.0);
    return g_seed - 0.5;
}
template <int R, int K>
static void fill(C (&A)[R][K], bool lower = false, double diag = 0.0)
{
    for (int i = 0; i < R; ++i)
        for (int j = 0; j < K; ++j)
            A[i][j] = (lower && j > i) ? C(0.0) : C(rnd() + (i == j ? diag : 0.0));
}
template <int R>
static void fillv(C (&a)[R])
{
    for (int i = 0; i < R; ++i)
        a[i] = C(rnd());
}
static void felem(FElem<C, NX> &e)
{
    fill(e.A);
    fillv(e.b);
    fill(e.U, true, 2.0);
    fillv(e.eta);
    fill(e.Z, true, 2.0);
}
static void selem(SElem<C, NX> &e)
{
    fill(e.E);
    fillv(e.g);
    fill(e.D, true, 2.0);
}
static void marg(Marg<C, NX> &m)
{
    fillv(m.m);
    fill(m.N, true, 2.0);
}

template <class Fn>
static void count(const char *name, Fn &&fn)
{
    fc::g_flop = fc::g_trans = 0;
    fn();
    printf("%s %lld %lld\n", name, fc::g_flop, fc::g_trans);
}

int main()
{
    count("filter_combine", [] {
        FElem<C, NX> a, b, o;
        felem(a);
        felem(b);
        filter_combine_v<C, NX, NX>(FRegV<C, NX>{&a}, FRegV<C, NX>{&b}, FRegV<C, NX>{&o});
    });
    count("filter_combine_leaf", [] {
        FElem<C, NX> a, b, o;
        felem(a);
        felem(b);
        filter_combine_v<C, NX, NY>(FRegV<C, NX>{&a}, FRegV<C, NX>{&b}, FRegV<C, NX>{&o});
    });
    count("filter_apply", [] {
        FElem<C, NX> b;
        Marg<C, NX> p, o;
        felem(b);
        marg(p);
        filter_apply_v<C, NX, NX>(p, FRegV<C, NX>{&b}, o);
    });
    count("filter_apply_leaf", [] {
        FElem<C, NX> b;
        Marg<C, NX> p, o;
        felem(b);
        marg(p);
        filter_apply_v<C, NX, NY>(p, FRegV<C, NX>{&b}, o);
    });
    count("smoother_combine", [] {
        SElem<C, NX> a, b, o;
        selem(a);
        selem(b);
        smoother_combine_v<C, NX>(SRegV<C, NX>{&a}, SRegV<C, NX>{&b}, SRegV<C, NX>{&o});
    });
    count("smoother_apply", [] {
        SElem<C, NX> a;
        Marg<C, NX> s, o;
        selem(a);
        marg(s);
        smoother_apply_v<C, NX>(SRegV<C, NX>{&a}, s, o);
    });
    count("filter_element", [] {
        C F[NX][NX], c[NX], SL[NX][NX], H[NY][NX], d[NY], SO[NY][NY], y[NY];
        fill(F);
        fillv(c);
        fill(SL, true, 2.0);
        fill(H);
        fillv(d);
        fill(SO, true, 2.0);
        fillv(y);
        FElem<C, NX> e;
        filter_element(F, c, SL, H, d, SO, y, e);
    });
    count("smoother_element", [] {
        C F[NX][NX], c[NX], SL[NX][NX];
        fill(F);
        fillv(c);
        fill(SL, true, 2.0);
        Marg<C, NX> f;
        marg(f);
        SElem<C, NX> e;
        smoother_element(F, c, SL, f, e);
    });
    CTParams<C> P;
    P.dt = C(0.01);
    P.s1x = C(-1.5);
    P.s1y = C(0.5);
    P.s2x = C(1.0);
    P.s2y = C(1.0);
    P.sigma = C(0.05);
    fill(P.LQ, true, 1.0);
    count("slr_transition", [&] {
        Marg<C, NX> mg;
        marg(mg);
        mg.m[4] = C(0.7); // a turning target: the general sinc branch
        C F[NX][NX], c[NX], S[NX][NX];
        ct_slr_transition(P, mg, F, c, S);
    });
    count("slr_bearings", [&] {
        Marg<C, NX> mg;
        marg(mg);
        C y[NY] = {C(0.3), C(-0.2)}, H[NY][NX], d[NY], S[NY][NY];
        ct_slr_bearings(P, mg, y, H, d, S);
    });
    // adjoint: the map T_k (built in the up-sweep), its combine and apply,
    // and the down-sweep's per-step work (map, apply, Gram cotangents and the
    // theta contraction)
    static C F[NX][NX], c[NX], SL[NX][NX], H[NY][NX], d[NY], SO[NY][NY], y[NY];
    fill(F);
    fillv(c);
    fill(SL, true, 2.0);
    fill(H);
    fillv(d);
    fill(SO, true, 2.0);
    fillv(y);
    count("adjoint_element", [] {
        Marg<C, NX> f;
        marg(f);
        StepQ<C, NX, NY> q;
        C Np[NX][NX], P22[NX][NX], mp[NX];
        adj_step(F, c, SL, H, d, SO, y, f, q, Np, P22, mp);
        SElem<C, NX> e;
        adj_element(F, q, e);
    });
    count("adjoint_combine", [] {
        SElem<C, NX> a, b, o;
        selem(a);
        selem(b);
        adj_combine_v<C, NX>(SRegV<C, NX>{&a}, SRegV<C, NX>{&b}, SRegV<C, NX>{&o});
    });
    count("adjoint_apply", [] {
        SElem<C, NX> a;
        Marg<C, NX> s, o;
        selem(a);
        marg(s);
        adj_apply_v<C, NX>(SRegV<C, NX>{&a}, s, o);
    });
    {
        static Marg<C, NX> f, lam;
        marg(f);
        marg(lam);
        static StepQ<C, NX, NY> q;
        C Np[NX][NX], P22[NX][NX], mp[NX];
        adj_step(F, c, SL, H, d, SO, y, f, q, Np, P22, mp);
        count("adjoint_cotangents", [] {
            C Lb[NX][NX], Ob[NY][NY], cb[NX], db[NY];
            adj_gram_bars(H, q, lam, Lb, Ob, cb, db);
            // theta contraction: tr(Lam_bar dQ1), tr(Lam_bar dQ2), tr(Om_bar) dR
            C g1 = C(0.0), g2 = C(0.0), g3 = C(0.0);
            for (int i = 0; i < NX; ++i)
                for (int j = 0; j < NX; ++j) {
                    g1 = g1 + Lb[i][j] * F[i][j];
                    g2 = g2 + Lb[i][j] * F[j][i];
                }
            for (int a = 0; a < NY; ++a)
                g3 = g3 + Ob[a][a] * c[0];
        });
    }
    return 0;
}
