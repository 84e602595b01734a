// Host-side launch logic: workspace layout, scan level planning and the
// per-(dtype, nx, ny) implementations behind the C ABI.
#pragma once

#include <algorithm>
#include <type_traits>

#include "adjoint.hpp"
#include "common.hpp"
#include "kernels.hpp"

namespace pss {

template <typename T>
inline const T *cptr(const void *p) { return static_cast<const T *>(p); }
template <typename T>
inline T *mptr(void *p) { return static_cast<T *>(p); }

// default launch shapes (overridable through pss_problem).  One 64-lane
// wave per tile; the filter folds 4 elements per thread, the smoother 2 (its
// operator is cheaper, and with 2 its level-0 reads and stash writes stay
// closer to whole cache lines).  The filter's finest level is flat: its
// per-thread aggregates are the next level's elements, so no in-tile tree
// runs there (a tree step keeps the whole wave busy for one operator while
// half of its lanes or fewer have work); its next level, n/4 elements, folds
// 4 per thread, the levels above it 2.  The smoother's operator is cheap
// next to its element construction, so its finest level keeps the tree and
// saves a level; its upper levels fold 2.
template <typename T, int NX>
struct Defaults {
    static constexpr int T0 = 64;
    static constexpr int E0_filter = 4;
    static constexpr int E0_smoother = 2;
    static constexpr int Tup = 64;
    static constexpr int E1_filter = 4;
    static constexpr int E1_smoother = 2;
    static constexpr int Eup_filter = 2;
    static constexpr int Eup_smoother = 2;
    static constexpr bool flat_filter = true;
    static constexpr bool flat_smoother = false;
};

template <typename T, int NX, int NY>
struct Core {
    using FS = FilterScan<T, NX>;
    using SS = SmootherScan<T, NX>;
    static constexpr int P = tri_size(NX);
    static constexpr int PY = tri_size(NY);
    static constexpr bool kFlatF = Defaults<T, NX>::flat_filter;
    static constexpr bool kFlatS = Defaults<T, NX>::flat_smoother;

    // ------------------------------------------------------------------
    static void shapes(const Ctx &c, bool smoother, int &T0, int &E0, int &Tup, int &E1,
                       int &Eup)
    {
        T0 = c.p->scan_threads > 0 ? c.p->scan_threads : Defaults<T, NX>::T0;
        E0 = c.p->scan_elems > 0 ? c.p->scan_elems
                                 : (smoother ? Defaults<T, NX>::E0_smoother
                                             : Defaults<T, NX>::E0_filter);
        Tup = Defaults<T, NX>::Tup;
        E1 = smoother ? Defaults<T, NX>::E1_smoother : Defaults<T, NX>::E1_filter;
        Eup = smoother ? Defaults<T, NX>::Eup_smoother : Defaults<T, NX>::Eup_filter;
        if (Tup > T0)
            Tup = T0;
    }

    // workspace of one scan; with base == nullptr only sizes
    template <class Op>
    struct ScanWs {
        int64_t *tile_off[kMaxLevels];
        int64_t *elem_off[kMaxLevels]; // element offsets of level l >= 1
        T *agg[kMaxLevels];  // elements of level l >= 1
        T *pre[kMaxLevels];  // exclusive prefixes of level l >= 1
        T *tree[kMaxLevels]; // LDS tree of a tree level l < L-1
    };

    template <class Op>
    static ScanWs<Op> carve_scan(Carver &cv, const Ctx &c, const ScanShape &sh)
    {
        ScanWs<Op> w{};
        for (int l = 0; l < sh.L; ++l)
            w.tile_off[l] = cv.template take<int64_t>(c.B + 1);
        for (int l = 1; l < sh.L; ++l) {
            w.elem_off[l] = cv.template take<int64_t>(c.B + 1);
            w.agg[l] = cv.template take<T>((size_t)Op::NE * sh.nelem[l]);
            w.pre[l] = cv.template take<T>((size_t)Op::NP * sh.nelem[l]);
        }
        for (int l = 0; l + 1 < sh.L; ++l)
            if (!sh.flat[l])
                w.tree[l] = cv.template take<T>((size_t)Op::NE * sh.ntiles[l] * sh.T[l]);
        return w;
    }

    static FElemRef<T, NX> felem_ref(T *base, int64_t ld)
    {
        FElemRef<T, NX> r;
        r.ld = ld;
        r.A = base;
        r.b = r.A + (int64_t)NX * NX * ld;
        r.U = r.b + (int64_t)NX * ld;
        r.eta = r.U + (int64_t)P * ld;
        r.Z = r.eta + (int64_t)NX * ld;
        return r;
    }
    static SElemRef<T, NX> selem_ref(T *base, int64_t ld)
    {
        SElemRef<T, NX> r;
        r.ld = ld;
        r.E = base;
        r.g = r.E + (int64_t)NX * NX * ld;
        r.D = r.g + (int64_t)NX * ld;
        return r;
    }
    static MargRef<T, NX> marg_ref(T *base, int64_t ld)
    {
        MargRef<T, NX> r;
        r.ld = ld;
        r.m = base;
        r.N = base + (int64_t)NX * ld;
        return r;
    }
    static MargRef<T, NX> marg_ref2(const void *m, const void *N, int64_t ld)
    {
        MargRef<T, NX> r;
        r.ld = ld;
        r.m = const_cast<T *>(cptr<T>(m));
        r.N = const_cast<T *>(cptr<T>(N));
        return r;
    }
    static GammaRef<T, NX, NY> gamma_ref(const pss_gamma *g, int64_t T_y)
    {
        GammaRef<T, NX, NY> r;
        r.F = mptr<T>(g->F);
        r.c = mptr<T>(g->c);
        r.SL = mptr<T>(g->SL);
        r.H = mptr<T>(g->H);
        r.d = mptr<T>(g->d);
        r.SO = mptr<T>(g->SO);
        r.stride = g->stride;
        r.ld = g->stride ? T_y : 1;
        return r;
    }
    // a linearisation buffer carved from the workspace (stride 1)
    static pss_gamma carve_gamma(Carver &cv, int64_t T_y)
    {
        pss_gamma g;
        g.F = cv.template take<T>((size_t)NX * NX * T_y);
        g.c = cv.template take<T>((size_t)NX * T_y);
        g.SL = cv.template take<T>((size_t)P * T_y);
        g.H = cv.template take<T>((size_t)NY * NX * T_y);
        g.d = cv.template take<T>((size_t)NY * T_y);
        g.SO = cv.template take<T>((size_t)PY * T_y);
        g.stride = 1;
        return g;
    }

    template <class Op>
    static size_t lds_bytes(int Tb, int E, bool stage)
    {
        return scan_lds(Op::NE, Op::NP, Tb, E, sizeof(T), stage);
    }

    template <class K>
    static int prep_lds(K kernel, size_t bytes)
    {
        return hip_check(hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)bytes),
                         "hipFuncSetAttribute");
    }

    // generic multi-level scan driver; Flat: level 0 may be flat (then it
    // is, see plan_scan, and level 1 is stored tile-interleaved)
    // stop > 0 (and < sh.L): run only the levels below `stop`, whose
    // exclusive prefixes w.pre[stop] the caller provides (a checkpoint):
    // the up-sweeps that rebuild those levels' trees and elements, then their
    // down-sweeps; the levels from `stop` up are not run.
    template <class Op, bool Flat, class Src0, class Dst0, class AggRef, class Start>
    static int run_scan(const Ctx &c, const ScanShape &sh, const ScanWs<Op> &w, int extra,
                        const Src0 &src0, const Dst0 &dst0, const Start &start,
                        AggRef (*agg_ref)(T *, int64_t), int stop = 0)
    {
        const int top = (stop > 0 && stop < sh.L) ? stop : sh.L;
        const bool partial = top < sh.L;
        int rc = launch_plan(c, sh, extra, w.tile_off, w.elem_off);
        if (rc)
            return rc;
        using LvSrc = RefSrc<Op, AggRef>;
        using LvSrcI = RefSrc<Op, AggRef, true>;
        using LvDst = PreDst<Op, MargRef<T, NX>>;
        auto geom = [&](int l) {
            LevelGeom g;
            g.y_off = c.p->y_off;
            g.elem_off = l > 0 ? w.elem_off[l] : nullptr;
            g.tile_off = w.tile_off[l];
            g.level = l;
            g.extra = extra;
            g.B = c.B;
            g.E = sh.E[l];
            g.stage = scan_stage(Op::NE, Op::NP, sh.T[l], sh.E[l], sizeof(T));
            return g;
        };
        // calls launch(src) with the element source of level l >= 1
        auto with_src = [&](int l, auto &&launch) -> int {
            if constexpr (Flat) {
                if (l == 1 && sh.flat[0])
                    return launch(LvSrcI{agg_ref(w.agg[l], sh.nelem[l])});
            }
            return launch(LvSrc{agg_ref(w.agg[l], sh.nelem[l])});
        };
        // up-sweeps of the lower levels (below a checkpoint: all levels
        // under it; a flat level right under it needs no up-sweep, its
        // down-sweep reads the stored prefixes per thread)
        for (int l = 0; l + 1 < sh.L && l < top; ++l) {
            if (partial && l == top - 1 && sh.flat[l])
                continue;
            const LevelGeom g = geom(l);
            const int64_t tree_ld = sh.ntiles[l] * sh.T[l];
            AggRef agg = agg_ref(w.agg[l + 1], sh.nelem[l + 1]);
            const size_t lb = lds_bytes<Op>(sh.T[l], sh.E[l], g.stage);
            KTime kt(c.s, Op::name, "up", l);
            if (l == 0) {
                bool flat = false;
                if constexpr (Flat) {
                    if ((flat = sh.flat[0])) {
                        auto k = k_scan_up_flat<Op, Src0, AggRef>;
                        if ((rc = prep_lds(k, lb)))
                            return rc;
                        hipLaunchKernelGGL(k, dim3((unsigned)sh.ntiles[l]), dim3(sh.T[l]), lb,
                                           c.s, g, src0, agg, w.elem_off[1], sh.T[1], sh.E[1]);
                    }
                }
                if (!flat) {
                    auto k = k_scan_up<Op, Src0, AggRef>;
                    if ((rc = prep_lds(k, lb)))
                        return rc;
                    hipLaunchKernelGGL(k, dim3((unsigned)sh.ntiles[l]), dim3(sh.T[l]), lb, c.s,
                                       g, src0, agg, w.tree[l], tree_ld);
                }
            } else {
                rc = with_src(l, [&](auto s) -> int {
                    auto k = k_scan_up<Op, decltype(s), AggRef>;
                    if (int r = prep_lds(k, lb))
                        return r;
                    hipLaunchKernelGGL(k, dim3((unsigned)sh.ntiles[l]), dim3(sh.T[l]), lb, c.s,
                                       g, s, agg, w.tree[l], tree_ld);
                    return 0;
                });
                if (rc)
                    return rc;
            }
            if ((rc = hip_check(hipGetLastError(), "scan up launch")))
                return rc;
        }
        // top level
        if (!partial) {
            const int l = sh.L - 1;
            const LevelGeom g = geom(l);
            const size_t lb = lds_bytes<Op>(sh.T[l], sh.E[l], g.stage);
            KTime kt(c.s, Op::name, "top", l);
            if (l == 0) {
                auto k = k_scan_top<Op, Src0, Dst0, Start>;
                if ((rc = prep_lds(k, lb)))
                    return rc;
                hipLaunchKernelGGL(k, dim3((unsigned)sh.ntiles[l]), dim3(sh.T[l]), lb, c.s, g,
                                   src0, dst0, start);
            } else {
                LvDst d{marg_ref(w.pre[l], sh.nelem[l])};
                rc = with_src(l, [&](auto s) -> int {
                    auto k = k_scan_top<Op, decltype(s), LvDst, Start>;
                    if (int r = prep_lds(k, lb))
                        return r;
                    hipLaunchKernelGGL(k, dim3((unsigned)sh.ntiles[l]), dim3(sh.T[l]), lb, c.s,
                                       g, s, d, start);
                    return 0;
                });
                if (rc)
                    return rc;
            }
            if ((rc = hip_check(hipGetLastError(), "scan top launch")))
                return rc;
        }
        // down-sweeps of the lower levels
        for (int l = top - (partial ? 1 : 2); l >= 0; --l) {
            const LevelGeom g = geom(l);
            const int64_t tree_ld = sh.ntiles[l] * sh.T[l];
            const size_t lb = lds_bytes<Op>(sh.T[l], sh.E[l], g.stage);
            MargRef<T, NX> pin = marg_ref(w.pre[l + 1], sh.nelem[l + 1]);
            KTime kt(c.s, Op::name, "down", l);
            if (l == 0) {
                bool flat = false;
                if constexpr (Flat) {
                    if ((flat = sh.flat[0])) {
                        auto k = k_scan_down_flat<Op, Src0, Dst0, MargRef<T, NX>>;
                        if ((rc = prep_lds(k, lb)))
                            return rc;
                        hipLaunchKernelGGL(k, dim3((unsigned)sh.ntiles[l]), dim3(sh.T[l]), lb,
                                           c.s, g, src0, dst0, w.elem_off[1], pin);
                    }
                }
                if (!flat) {
                    auto k = k_scan_down<Op, Src0, Dst0, MargRef<T, NX>>;
                    if ((rc = prep_lds(k, lb)))
                        return rc;
                    hipLaunchKernelGGL(k, dim3((unsigned)sh.ntiles[l]), dim3(sh.T[l]), lb, c.s,
                                       g, src0, dst0, w.tree[l], tree_ld, pin);
                }
            } else {
                LvDst d{marg_ref(w.pre[l], sh.nelem[l])};
                rc = with_src(l, [&](auto s) -> int {
                    auto k = k_scan_down<Op, decltype(s), LvDst, MargRef<T, NX>>;
                    if (int r = prep_lds(k, lb))
                        return r;
                    hipLaunchKernelGGL(k, dim3((unsigned)sh.ntiles[l]), dim3(sh.T[l]), lb, c.s,
                                       g, s, d, w.tree[l], tree_ld, pin);
                    return 0;
                });
                if (rc)
                    return rc;
            }
            if ((rc = hip_check(hipGetLastError(), "scan down launch")))
                return rc;
        }
        return PSS_OK;
    }

    // ------------------------------------------------------------------
    // filter scan (elements read from `el`)
    static ScanShape filter_shape(const Ctx &c)
    {
        int T0, E0, Tup, E1, Eup;
        shapes(c, false, T0, E0, Tup, E1, Eup);
        return plan_scan(c, 0, T0, E0, Tup, E1, Eup, kFlatF);
    }
    static ScanShape smoother_shape(const Ctx &c)
    {
        int T0, E0, Tup, E1, Eup;
        shapes(c, true, T0, E0, Tup, E1, Eup);
        return plan_scan(c, 1, T0, E0, Tup, E1, Eup, kFlatS);
    }

    // the adjoint scan (reverse time, one element per step): tree level 0
    // with 2 elements per thread, as the smoother (its element -- a Kalman
    // step from the filtering marginal -- dominates the operator)
    static ScanShape adj_shape(const Ctx &c)
    {
        const int T0 = c.p->scan_threads > 0 ? c.p->scan_threads : Defaults<T, NX>::T0;
        const int Tup = std::min(T0, (int)Defaults<T, NX>::Tup);
        return plan_scan(c, 0, T0, 2, Tup, 2, 2, false);
    }
    static size_t ascan_bytes(const Ctx &c)
    {
        Carver cv{nullptr};
        carve_scan<AdjScan<T, NX>>(cv, c, adj_shape(c));
        return cv.used;
    }

    static size_t fscan_bytes(const Ctx &c)
    {
        Carver cv{nullptr};
        carve_scan<FS>(cv, c, filter_shape(c));
        return cv.used;
    }
    static size_t sscan_bytes(const Ctx &c)
    {
        Carver cv{nullptr};
        carve_scan<SS>(cv, c, smoother_shape(c));
        cv.template take<T>((size_t)Sizes<NX>::selem * c.T_x); // element stash
        return cv.used;
    }

    // ilv: the elements are stored tile-interleaved for this scan's level 0
    // (as written by felem(..., true)); the library's own passes use that
    // cov: the standard (covariance-form) scan of the same storage layout
    // ck_pre (square-root form only): the exclusive prefixes of the filter
    // scan's level ck_level (1 <= ck_level < levels) -- written there by a
    // full scan, or, with resume, read from there and only the levels below
    // re-run (the backward pass of a checkpointed log-likelihood)
    static int fscan(const Ctx &c, const pss_felem *el, void *mf, void *Nf, void *ws,
                     bool ilv = false, bool cov = false, int ck_level = 0, T *ck_pre = nullptr,
                     bool resume = false)
    {
        const ScanShape sh = filter_shape(c);
        Carver cv{static_cast<char *>(ws)};
        auto w = carve_scan<FS>(cv, c, sh);
        const bool ck = ck_pre && ck_level >= 1 && ck_level < sh.L;
        if (ck)
            w.pre[ck_level] = ck_pre;
        const int stop = (ck && resume) ? ck_level : 0;
        FElemRef<T, NX> er;
        er.A = mptr<T>(el->A);
        er.b = mptr<T>(el->b);
        er.U = mptr<T>(el->U);
        er.eta = mptr<T>(el->eta);
        er.Z = mptr<T>(el->Z);
        er.ld = c.T_y;
        FiltDst<T, NX> dst{marg_ref2(mf, Nf, c.T_x), c.p->y_off};
        dst.dev_m = cptr<T>(c.dev_m);
        StartPre<T, NX> st{cptr<T>(c.p->m0), cptr<T>(c.p->N0)};
        // finest-level elements: Z = Tria([Z_k, 0]) with Z_k of ny columns
        constexpr int LZ = NY < NX ? NY : NX;
        if (cov) {
            using FSC = FilterScanCov<T, NX>;
            StartPreCov<T, NX> stc{cptr<T>(c.p->m0), cptr<T>(c.p->N0)};
            Carver cc{static_cast<char *>(ws)};
            auto wc = carve_scan<FSC>(cc, c, sh);
            if (ilv) {
                RefSrc<FSC, FElemRef<T, NX>, true> src{er};
                return run_scan<FSC, kFlatF>(c, sh, wc, 0, src, dst, stc, &felem_ref);
            }
            RefSrc<FSC, FElemRef<T, NX>> src{er};
            return run_scan<FSC, kFlatF>(c, sh, wc, 0, src, dst, stc, &felem_ref);
        }
        if (ilv) {
            RefSrc<FS, FElemRef<T, NX>, true, LZ> src{er};
            return run_scan<FS, kFlatF>(c, sh, w, 0, src, dst, st, &felem_ref, stop);
        }
        RefSrc<FS, FElemRef<T, NX>, false, LZ> src{er};
        return run_scan<FS, kFlatF>(c, sh, w, 0, src, dst, st, &felem_ref, stop);
    }

    static int sscan(const Ctx &c, const pss_gamma *g, const void *mf, const void *Nf, void *ms,
                     void *Ns, void *ws, bool cov = false)
    {
        const ScanShape sh = smoother_shape(c);
        Carver cv{static_cast<char *>(ws)};
        auto w = carve_scan<SS>(cv, c, sh);
        T *stash = cv.template take<T>((size_t)Sizes<NX>::selem * c.T_x);
        SmoothDst<T, NX> dst{marg_ref2(ms, Ns, c.T_x)};
        dst.dev_m = cptr<T>(c.dev_m);
        StartPre<T, NX> st{nullptr, nullptr};
        if (cov) {
            using SSC = SmootherScanCov<T, NX>;
            Carver cc{static_cast<char *>(ws)};
            auto wc = carve_scan<SSC>(cc, c, sh);
            SmootherSrc<T, NX, NY, true> src{gamma_ref(g, c.T_y), marg_ref2(mf, Nf, c.T_x),
                                             selem_ref(stash, c.T_x), c.p->y_off};
            return run_scan<SSC, kFlatS>(c, sh, wc, 1, src, dst, st, &selem_ref);
        }
        SmootherSrc<T, NX, NY> src{gamma_ref(g, c.T_y), marg_ref2(mf, Nf, c.T_x),
                                   selem_ref(stash, c.T_x), c.p->y_off};
        return run_scan<SS, kFlatS>(c, sh, w, 1, src, dst, st, &selem_ref);
    }

    // the adjoint scan: the reverse scan of the cotangent maps T_k from the
    // filtering marginals (mf, Nf) and the linearisation, emitting through
    // `out` the step cotangents and through `dst` the prior's
    template <class Out>
    static int ascan(const Ctx &c, const pss_gamma *g, const void *y, const void *mf,
                     const void *Nf, const Out &out, const AdjDst<T, NX> &dst, void *ws)
    {
        using AS = AdjScan<T, NX>;
        const ScanShape sh = adj_shape(c);
        Carver cv{static_cast<char *>(ws)};
        auto w = carve_scan<AS>(cv, c, sh);
        AdjSrc<T, NX, NY, Out> src{gamma_ref(g, c.T_y), marg_ref2(mf, Nf, c.T_x), cptr<T>(y),
                                   c.T_y, out};
        StartPre<T, NX> st{nullptr, nullptr};
        return run_scan<AS, false>(c, sh, w, 0, src, dst, st, &selem_ref);
    }

    static int felem(const Ctx &c, const pss_gamma *g, const void *y, const pss_felem *out,
                     bool ilv = false, bool cov = false)
    {
        int ilv_T = 0, ilv_E = 0;
        if (ilv) {
            const ScanShape sh = filter_shape(c);
            ilv_T = sh.T[0];
            ilv_E = sh.E[0];
        }
        FElemRef<T, NX> er;
        er.A = mptr<T>(out->A);
        er.b = mptr<T>(out->b);
        er.U = mptr<T>(out->U);
        er.eta = mptr<T>(out->eta);
        er.Z = mptr<T>(out->Z);
        er.ld = c.T_y;
        // a block covers a whole level-0 tile (64 x 4): the strided reads of
        // its tile-interleaved elements meet the same cache lines in one L2
        const int tb = 256;
        KTime kt(c.s, cov ? "filter_elements_cov" : "filter_elements", "", 0);
        const dim3 grid((unsigned)((c.T_y + tb - 1) / tb));
        if (cov)
            hipLaunchKernelGGL((k_filter_elements<T, NX, NY, true>), grid, dim3(tb), 0, c.s,
                               c.p->y_off, c.B, c.T_y, gamma_ref(g, c.T_y), cptr<T>(y),
                               cptr<T>(c.p->m0), cptr<T>(c.p->N0), er, ilv_T, ilv_E,
                               cptr<T>(c.dev_m), c.T_x);
        else
            hipLaunchKernelGGL((k_filter_elements<T, NX, NY>), grid, dim3(tb), 0, c.s,
                               c.p->y_off, c.B, c.T_y, gamma_ref(g, c.T_y), cptr<T>(y),
                               cptr<T>(c.p->m0), cptr<T>(c.p->N0), er, ilv_T, ilv_E,
                               cptr<T>(c.dev_m), c.T_x);
        return hip_check(hipGetLastError(), "filter elements launch");
    }

    // ------------------------------------------------------------------
    // model-specific pieces
    static int slr(const Ctx &c, const void *m, const void *N, const void *y,
                   const pss_gamma *out);
    // the CT model with cubature or Taylor linearisation in FP32: slr and
    // the (tile-interleaved) filter elements in one kernel; returns 1,
    // launching nothing, for every other case.  (In FP64 the fused kernel's
    // register footprint made it slower than the two kernels it replaces:
    // 0.47 ms against 0.17 + 0.23 ms at n = 10^6; in FP32 0.16 against
    // 0.08 + 0.13 ms.)
    static int slr_felem(const Ctx &c, const void *m, const void *N, const void *y,
                         const pss_gamma *g, const pss_felem *el, bool cov, bool store_obs);
    static int grad_terms(const Ctx &c, const pss_gamma *g, const void *y, const void *mf,
                          const void *Nf, const void *ms, const void *Ns, double *gterms);

    // ------------------------------------------------------------------
    // composite operations
    static size_t felem_bytes(const Ctx &c)
    {
        return align256((size_t)Sizes<NX>::felem * c.T_y * sizeof(T));
    }
    static size_t marg_bytes(const Ctx &c)
    {
        return align256((size_t)Sizes<NX>::marg * c.T_x * sizeof(T));
    }
    static size_t gamma_bytes(const Ctx &c)
    {
        Carver cv{nullptr};
        carve_gamma(cv, c.T_y);
        return cv.used;
    }
    // nonlinear models are linearised on every pass; a linear one is given
    static bool nonlinear(const Ctx &c) { return c.p->model != PSS_MODEL_LINEAR; }

    static size_t ws_size(const Ctx &c, int op)
    {
        const size_t scans = fscan_bytes(c) > sscan_bytes(c) ? fscan_bytes(c) : sscan_bytes(c);
        const size_t fwd = gamma_bytes(c) + felem_bytes(c) + marg_bytes(c) +
                           align256(c.T_y * sizeof(double));
        switch (op) {
        case PSS_OP_SLR:
        case PSS_OP_FILTER_ELEMENTS:
            return 0;
        case PSS_OP_FILTER_SCAN:
            return fscan_bytes(c);
        case PSS_OP_SMOOTHER_SCAN:
            return sscan_bytes(c);
        case PSS_OP_IPLS:
            return gamma_bytes(c) + felem_bytes(c) + marg_bytes(c) + scans;
        case PSS_OP_LOGLIK:
            return fwd + std::max(fscan_bytes(c), seq_sum_bytes(c, 1));
        case PSS_OP_LOGLIK_GRAD:
            return fwd + std::max({fscan_bytes(c), ascan_bytes(c), seq_sum_bytes(c, 3)}) +
                   align256(3 * c.T_y * sizeof(double)) + align256(3 * c.B * sizeof(double));
        case PSS_OP_LOGLIK_VJP:
            return fwd + std::max({fscan_bytes(c), ascan_bytes(c), seq_sum_bytes(c, 1)});
        case PSS_OP_SCORE_FISHER:
            return gamma_bytes(c) + felem_bytes(c) + marg_bytes(c) +
                   align256(c.T_y * sizeof(double)) + std::max(scans, seq_sum_bytes(c, 3)) +
                   marg_bytes(c) + align256(3 * c.T_y * sizeof(double)) +
                   align256(3 * c.B * sizeof(double));
        case PSS_OP_SEQUENTIAL:
            return gamma_bytes(c) + marg_bytes(c);
        default:
            return 0;
        }
    }

    // ------------------------------------------------------------------
    // checkpoints of the log-likelihood's filter pass (pss_ckpt): the
    // per-sequence log-likelihoods, then what the level keeps -- level 0
    // every filtering marginal, level l in [1, levels) the exclusive
    // prefixes of the filter scan's level-l elements, higher levels nothing
    struct CkView {
        int level = 0;
        double *ll = nullptr;
        T *marg = nullptr; // level 0: [Sizes::marg][T_x]
        T *pre = nullptr;  // level l: [Sizes::marg][nelem_l]
    };
    static size_t ckpt_bytes(const Ctx &c, int level)
    {
        Carver cv{nullptr};
        cv.template take<double>((size_t)c.B);
        if (level == 0) {
            cv.template take<T>((size_t)Sizes<NX>::marg * c.T_x);
        } else {
            const ScanShape sh = filter_shape(c);
            if (level < sh.L)
                cv.template take<T>((size_t)Sizes<NX>::marg * sh.nelem[level]);
        }
        return cv.used;
    }
    static CkView ckpt_view(const Ctx &c, const pss_ckpt *ck)
    {
        CkView v;
        if (!ck)
            return v;
        v.level = ck->level;
        Carver cv{static_cast<char *>(ck->buf)};
        v.ll = cv.template take<double>((size_t)c.B);
        if (ck->level == 0) {
            v.marg = cv.template take<T>((size_t)Sizes<NX>::marg * c.T_x);
        } else {
            const ScanShape sh = filter_shape(c);
            if (ck->level < sh.L)
                v.pre = cv.template take<T>((size_t)Sizes<NX>::marg * sh.nelem[ck->level]);
        }
        return v;
    }
    // the filter scan's level count for this problem (checkpoint levels
    // from it up keep nothing but the log-likelihoods)
    static int filter_levels(const Ctx &c) { return filter_shape(c).L; }

    static int ipls(const Ctx &c, const pss_gamma *gin, const void *y, int n_iter, void *m_nom,
                    void *N_nom, void *mf_out, void *Nf_out, void *ws)
    {
        Carver cv{static_cast<char *>(ws)};
        pss_gamma gw = carve_gamma(cv, c.T_y);
        T *fel = cv.template take<T>((size_t)Sizes<NX>::felem * c.T_y);
        T *mfb = cv.template take<T>((size_t)Sizes<NX>::marg * c.T_x);
        void *scan_ws = cv.base + cv.used;
        const pss_gamma *g = nonlinear(c) ? &gw : gin;
        // FP32: the CT model's passes run in deviation coordinates relative
        // to the nominal means (see Ctx), unless the caller takes the
        // filtering marginals (those are absolute).  On the 10^6-step track
        // this cut the late passes' mean error about 5x; FP64 loses nothing
        // measurable in absolute coordinates and keeps them (the offsets and
        // the smoother's read of the nominal cost 0.04 ms per pass there).
        Ctx cs = c;
        if (sizeof(T) == 4 && c.p->model == PSS_MODEL_CT_BEARINGS && !mf_out)
            cs.dev_m = m_nom;
        FElemRef<T, NX> fr = felem_ref(fel, c.T_y);
        pss_felem el{fr.A, fr.b, fr.U, fr.eta, fr.Z};
        void *mf = mf_out ? mf_out : (void *)mfb;
        void *Nf = mf_out ? Nf_out : (void *)(mfb + (size_t)NX * c.T_x);
        int rc = PSS_OK;
        const bool cov = c.p->form == PSS_FORM_COV;
        for (int it = 0; it < n_iter && rc == PSS_OK; ++it) {
            const int fused =
                nonlinear(c) ? slr_felem(cs, m_nom, N_nom, y, &gw, &el, cov, false) : 1;
            if (fused < 0) {
                rc = fused;
                break;
            }
            if (fused) {
                if (nonlinear(c) && (rc = slr(cs, m_nom, N_nom, y, &gw)))
                    break;
                if ((rc = felem(cs, g, y, &el, true, cov)))
                    break;
            }
            if ((rc = fscan(cs, &el, mf, Nf, scan_ws, true, cov)))
                break;
            rc = sscan(cs, g, mf, Nf, m_nom, N_nom, scan_ws, cov);
        }
        return rc;
    }

    // linearisation (nonlinear models) and level-0 filter elements
    // (tile-interleaved) at the nominal; the transition and measurement
    // parts of Gamma are both stored
    static int lin_elements(const Ctx &c, const pss_gamma *gin, const void *m_nom,
                            const void *N_nom, const void *y, const pss_gamma &gw,
                            const pss_felem *el)
    {
        int rc;
        const bool cov = c.p->form == PSS_FORM_COV;
        const int fused = nonlinear(c) ? slr_felem(c, m_nom, N_nom, y, &gw, el, cov, true) : 1;
        if (fused < 0)
            return fused;
        if (fused) {
            if (nonlinear(c) && (rc = slr(c, m_nom, N_nom, y, &gw)))
                return rc;
            if ((rc = felem(c, nonlinear(c) ? &gw : gin, y, el, true, cov)))
                return rc;
        }
        return PSS_OK;
    }

    // filter pass shared by loglik and the gradients; returns the carved
    // state.  With a checkpoint (square-root form) the filtering marginals
    // go to it (level 0) or the scan's level-`level` prefixes do, and the
    // log-likelihoods are copied into it.
    static int loglik_core(const Ctx &c, const pss_gamma *gin, const void *m_nom,
                           const void *N_nom, const void *y, double *ll, Carver &cv,
                           pss_gamma &gw, T *&mfb, void *&scan_ws, const CkView &ck = CkView{},
                           bool use_ck = false)
    {
        gw = carve_gamma(cv, c.T_y);
        T *fel = cv.template take<T>((size_t)Sizes<NX>::felem * c.T_y);
        mfb = cv.template take<T>((size_t)Sizes<NX>::marg * c.T_x);
        double *ell = cv.template take<double>((size_t)c.T_y);
        scan_ws = cv.base + cv.used;
        if (!nonlinear(c))
            gw = *gin;
        const pss_gamma *g = &gw;
        if (use_ck && ck.level == 0)
            mfb = ck.marg;
        FElemRef<T, NX> fr = felem_ref(fel, c.T_y);
        pss_felem el{fr.A, fr.b, fr.U, fr.eta, fr.Z};
        int rc;
        const bool cov = c.p->form == PSS_FORM_COV;
        if ((rc = lin_elements(c, gin, m_nom, N_nom, y, gw, &el)))
            return rc;
        if ((rc = fscan(c, &el, mfb, mfb + (size_t)NX * c.T_x, scan_ws, true, cov,
                        use_ck ? ck.level : 0, use_ck ? ck.pre : nullptr, false)))
            return rc;
        const int tb = 128;
        {
            KTime kt(c.s, "loglik_terms", "", 0);
            const dim3 grid((unsigned)((c.T_y + tb - 1) / tb));
            if (cov)
                hipLaunchKernelGGL((k_loglik_terms_cov<T, NX, NY>), grid, dim3(tb), 0, c.s,
                                   c.p->y_off, c.B, c.T_y, c.T_x, gamma_ref(g, c.T_y), cptr<T>(y),
                                   marg_ref(mfb, c.T_x), ell);
            else
                hipLaunchKernelGGL((k_loglik_terms<T, NX, NY>), grid, dim3(tb), 0, c.s,
                                   c.p->y_off, c.B, c.T_y, c.T_x, gamma_ref(g, c.T_y), cptr<T>(y),
                                   marg_ref(mfb, c.T_x), ell);
            if ((rc = hip_check(hipGetLastError(), "loglik launch")))
                return rc;
        }
        if ((rc = launch_seq_sum(c, 1, ell, c.T_y, ll, scan_ws)))
            return rc;
        if (use_ck)
            rc = hip_check(hipMemcpyAsync(ck.ll, ll, (size_t)c.B * sizeof(double),
                                          hipMemcpyDeviceToDevice, c.s),
                           "checkpoint log-likelihood copy");
        return rc;
    }

    static int loglik(const Ctx &c, const pss_gamma *gin, const void *m_nom, const void *N_nom,
                      const void *y, double *ll, const pss_ckpt *ckpt, void *ws)
    {
        Carver cv{static_cast<char *>(ws)};
        pss_gamma gw;
        T *mfb;
        void *scan_ws;
        return loglik_core(c, gin, m_nom, N_nom, y, ll, cv, gw, mfb, scan_ws, ckpt_view(c, ckpt),
                           ckpt != nullptr);
    }

    // forward state of a gradient pass: the linearisation and the filtering
    // marginals at the nominal, from a checkpoint (re-running the filter
    // scan's levels under it) or from a full filter pass; ll receives the
    // log-likelihoods
    static int grad_forward(const Ctx &c, const pss_gamma *gin, const void *m_nom,
                            const void *N_nom, const void *y, const pss_ckpt *ckpt, double *ll,
                            Carver &cv, pss_gamma &gw, T *&mf, void *&scan_ws)
    {
        if (!ckpt) {
            T *mfb;
            int rc = loglik_core(c, gin, m_nom, N_nom, y, ll, cv, gw, mfb, scan_ws);
            mf = mfb;
            return rc;
        }
        const CkView ck = ckpt_view(c, ckpt);
        gw = carve_gamma(cv, c.T_y);
        T *fel = cv.template take<T>((size_t)Sizes<NX>::felem * c.T_y);
        T *mfb = cv.template take<T>((size_t)Sizes<NX>::marg * c.T_x);
        cv.template take<double>((size_t)c.T_y);
        scan_ws = cv.base + cv.used;
        if (!nonlinear(c))
            gw = *gin;
        int rc;
        if (ck.level == 0) {
            // every marginal is stored: only the linearisation is redone
            if (nonlinear(c) && (rc = slr(c, m_nom, N_nom, y, &gw)))
                return rc;
            mf = ck.marg;
        } else {
            FElemRef<T, NX> fr = felem_ref(fel, c.T_y);
            pss_felem el{fr.A, fr.b, fr.U, fr.eta, fr.Z};
            if ((rc = lin_elements(c, gin, m_nom, N_nom, y, gw, &el)))
                return rc;
            // levels under the checkpoint re-run from its prefixes; without
            // stored prefixes (a level at or above the top) the whole scan
            if ((rc = fscan(c, &el, mfb, mfb + (size_t)NX * c.T_x, scan_ws, true, false,
                            ck.level, ck.pre, true)))
                return rc;
            mf = mfb;
        }
        return hip_check(hipMemcpyAsync(ll, ck.ll, (size_t)c.B * sizeof(double),
                                        hipMemcpyDeviceToDevice, c.s),
                         "checkpoint log-likelihood copy");
    }

    // gradient with respect to theta (coordinated-turn model) by the
    // reverse-mode adjoint: the cotangent scan from the filtering marginals,
    // the step VJP contracted with dQ/dtheta and dR/dtheta, fixed-order
    // per-sequence sums
    static int loglik_grad(const Ctx &c, const void *m_nom, const void *N_nom, const void *y,
                           const double *ll_bar, const pss_ckpt *ckpt, double *ll, double *grad,
                           double *theta_bar, void *ws)
    {
        if constexpr (NX == 5 && NY == 2) {
            const size_t scans = std::max({fscan_bytes(c), ascan_bytes(c), seq_sum_bytes(c, 3)});
            Carver tail{static_cast<char *>(ws) + gamma_bytes(c) + felem_bytes(c) +
                        marg_bytes(c) + align256(c.T_y * sizeof(double)) + scans};
            double *gterms = tail.template take<double>((size_t)3 * c.T_y);
            double *gseq = tail.template take<double>((size_t)3 * c.B);
            Carver cv{static_cast<char *>(ws)};
            pss_gamma gw;
            T *mf;
            void *scan_ws;
            int rc = grad_forward(c, nullptr, m_nom, N_nom, y, ckpt, ll, cv, gw, mf, scan_ws);
            if (rc)
                return rc;
            const CTHost h = ct_host(c.p);
            ThetaOut<T, NX, NY> out;
            for (int i = 0; i < 5; ++i)
                for (int j = 0; j < 5; ++j) {
                    double a1 = 0.0, a2 = 0.0;
                    for (int q = 0; q < 5; ++q) {
                        a1 += h.L1[i][q] * h.L1[j][q];
                        a2 += h.L2[i][q] * h.L2[j][q];
                    }
                    out.th.dQ1[i][j] = (T)a1;
                    out.th.dQ2[i][j] = (T)a2;
                }
            out.th.dR = (T)(2.0 * h.sigma * h.sigma);
            out.terms = gterms;
            out.T_y = c.T_y;
            AdjDst<T, NX> dst{nullptr, nullptr, nullptr, nullptr, c.B};
            if ((rc = ascan(c, &gw, y, mf, mf + (size_t)NX * c.T_x, out, dst, scan_ws)))
                return rc;
            double *gout = grad ? grad : gseq;
            if ((rc = launch_seq_sum(c, 3, gterms, c.T_y, gout, scan_ws)))
                return rc;
            if (theta_bar)
                rc = launch_weighted_grad(c, gout, ll_bar, theta_bar);
            return rc;
        } else {
            set_error("the theta gradient needs the coordinated-turn model");
            return PSS_EUNSUPPORTED;
        }
    }

    // VJP of the log-likelihood with respect to the linearisation (every
    // step's Gamma in the library's representation) and the prior
    static int loglik_vjp(const Ctx &c, const pss_gamma *gin, const void *m_nom,
                          const void *N_nom, const void *y, const double *ll_bar,
                          const pss_ckpt *ckpt, double *ll, const pss_gamma *gbar, void *m0_bar,
                          void *N0_bar, void *ws)
    {
        Carver cv{static_cast<char *>(ws)};
        pss_gamma gw;
        T *mf;
        void *scan_ws;
        int rc = grad_forward(c, gin, m_nom, N_nom, y, ckpt, ll, cv, gw, mf, scan_ws);
        if (rc)
            return rc;
        GammaOut<T, NX, NY> out;
        out.bar = gamma_ref(gbar, c.T_y);
        out.w = ll_bar;
        AdjDst<T, NX> dst{mptr<T>(m0_bar), mptr<T>(N0_bar), cptr<T>(c.p->N0), ll_bar, c.B};
        return ascan(c, &gw, y, mf, mf + (size_t)NX * c.T_x, out, dst, scan_ws);
    }

    // the frozen-nominal score by Fisher's identity from the parallel
    // smoother (a cross-check of the adjoint)
    static int score_fisher(const Ctx &c, const void *m_nom, const void *N_nom, const void *y,
                            const double *ll_bar, double *ll, double *grad, double *theta_bar,
                            void *ws)
    {
        // layout: [gamma | felem | mf | ell | scan ws ...] then the score part
        // after the largest scan workspace
        Carver cv{static_cast<char *>(ws)};
        pss_gamma gw;
        T *mfb;
        void *scan_ws;
        const size_t scans = std::max(std::max(fscan_bytes(c), sscan_bytes(c)),
                                      seq_sum_bytes(c, 3));
        Carver tail{static_cast<char *>(ws) + gamma_bytes(c) + felem_bytes(c) + marg_bytes(c) +
                    align256(c.T_y * sizeof(double)) + scans};
        T *msb = tail.template take<T>((size_t)Sizes<NX>::marg * c.T_x);
        double *gterms = tail.template take<double>((size_t)3 * c.T_y);
        double *gseq = tail.template take<double>((size_t)3 * c.B);
        int rc = loglik_core(c, nullptr, m_nom, N_nom, y, ll, cv, gw, mfb, scan_ws);
        if (rc)
            return rc;
        T *mf = mfb, *Nf = mfb + (size_t)NX * c.T_x;
        T *ms = msb, *Ns = msb + (size_t)NX * c.T_x;
        if ((rc = sscan(c, &gw, mf, Nf, ms, Ns, scan_ws)))
            return rc;
        if ((rc = grad_terms(c, &gw, y, mf, Nf, ms, Ns, gterms)))
            return rc;
        double *gout = grad ? grad : gseq;
        // per-sequence sums land component-major [3][B]
        if ((rc = launch_seq_sum(c, 3, gterms, c.T_y, gout, scan_ws)))
            return rc;
        if (theta_bar)
            rc = launch_weighted_grad(c, gout, ll_bar, theta_bar);
        return rc;
    }

    static int sequential(const Ctx &c, const pss_gamma *gin, const void *y, int n_iter,
                          void *m_nom, void *N_nom, void *mf_out, void *Nf_out, void *ws)
    {
        Carver cv{static_cast<char *>(ws)};
        pss_gamma gw = carve_gamma(cv, c.T_y);
        T *mfb = cv.template take<T>((size_t)Sizes<NX>::marg * c.T_x);
        const pss_gamma *g = nonlinear(c) ? &gw : gin;
        void *mf = mf_out ? mf_out : (void *)mfb;
        void *Nf = mf_out ? Nf_out : (void *)(mfb + (size_t)NX * c.T_x);
        int rc = PSS_OK;
        for (int it = 0; it < n_iter && rc == PSS_OK; ++it) {
            if (nonlinear(c) && (rc = slr(c, m_nom, N_nom, y, &gw)))
                break;
            const int tb = 64;
            const dim3 grid((unsigned)((c.B + tb - 1) / tb));
            KTime kt(c.s, "sequential", "", 0);
            if (c.p->form == PSS_FORM_COV)
                hipLaunchKernelGGL((k_sequential_cov<T, NX, NY>), grid, dim3(tb), 0, c.s,
                                   c.p->y_off, c.B, c.T_y, gamma_ref(g, c.T_y), cptr<T>(y),
                                   cptr<T>(c.p->m0), cptr<T>(c.p->N0), marg_ref2(mf, Nf, c.T_x),
                                   marg_ref2(m_nom, N_nom, c.T_x));
            else if constexpr (NX == 1) // scalar state: one thread per sequence
                hipLaunchKernelGGL((k_sequential_1t<T, NX, NY>), grid, dim3(tb), 0, c.s,
                                   c.p->y_off, c.B, c.T_y, gamma_ref(g, c.T_y), cptr<T>(y),
                                   cptr<T>(c.p->m0), cptr<T>(c.p->N0), marg_ref2(mf, Nf, c.T_x),
                                   marg_ref2(m_nom, N_nom, c.T_x));
            else // one wavefront per sequence
                hipLaunchKernelGGL((k_sequential<T, NX, NY>), dim3((unsigned)c.B), dim3(64), 0, c.s,
                                   c.p->y_off, c.B, c.T_y, gamma_ref(g, c.T_y), cptr<T>(y),
                                   cptr<T>(c.p->m0), cptr<T>(c.p->N0), marg_ref2(mf, Nf, c.T_x),
                                   marg_ref2(m_nom, N_nom, c.T_x));
            rc = hip_check(hipGetLastError(), "sequential launch");
        }
        return rc;
    }
};

template <typename T>
static bool rule_spec(const pss_problem *p, int nx, RuleSpec<T> &R)
{
    RuleHost h;
    if (!rule_host(p, nx, h))
        return false;
    R.kind = h.kind;
    R.np = h.np;
    R.p = h.p;
    R.w0 = (T)h.w0;
    R.wi = (T)h.wi;
    R.spread = (T)h.spread;
    for (int q = 0; q < kMaxGH; ++q) {
        R.gx[q] = (T)h.gx[q];
        R.gw[q] = (T)h.gw[q];
    }
    return true;
}

// device-side CT constants in the kernel's precision
template <typename T>
CTParams<T> ct_params(const CTHost &h)
{
    CTParams<T> P;
    P.dt = (T)h.dt;
    P.s1x = (T)h.s1x;
    P.s1y = (T)h.s1y;
    P.s2x = (T)h.s2x;
    P.s2y = (T)h.s2y;
    P.sigma = (T)h.sigma;
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 5; ++j)
            P.LQ[i][j] = (T)h.LQ[i][j];
    return P;
}

template <typename T, int NX, int NY>
int Core<T, NX, NY>::slr_felem(const Ctx &c, const void *m, const void *N, const void *y,
                               const pss_gamma *g, const pss_felem *el, bool cov,
                               bool store_obs)
{
    if constexpr (NX == 5 && NY == 2 && std::is_same_v<T, float>) {
        const int lin = c.p->linearization;
        if (c.p->model == PSS_MODEL_CT_BEARINGS &&
            (lin == PSS_LIN_CUBATURE || lin == PSS_LIN_TAYLOR)) {
            const CTParams<T> P = ct_params<T>(ct_host(c.p));
            const ScanShape sh = filter_shape(c);
            FElemRef<T, NX> er;
            er.A = mptr<T>(el->A);
            er.b = mptr<T>(el->b);
            er.U = mptr<T>(el->U);
            er.eta = mptr<T>(el->eta);
            er.Z = mptr<T>(el->Z);
            er.ld = c.T_y;
            const int tb = 256; // one level-0 filter tile per block, as felem
            const dim3 grid((unsigned)((c.T_y + tb - 1) / tb));
            const int taylor = lin == PSS_LIN_TAYLOR ? 1 : 0;
            KTime kt(c.s, "slr_felem", "", 0);
            if (cov)
                hipLaunchKernelGGL((k_slr_felem_ct<T, true>), grid, dim3(tb), 0, c.s, c.p->y_off,
                                   c.B, c.T_y, P, marg_ref2(m, N, c.T_x), cptr<T>(y),
                                   cptr<T>(c.p->m0), cptr<T>(c.p->N0), gamma_ref(g, c.T_y),
                                   store_obs ? 1 : 0, er, sh.T[0], sh.E[0], taylor, 1,
                                   c.dev_m ? 1 : 0);
            else
                hipLaunchKernelGGL((k_slr_felem_ct<T, false>), grid, dim3(tb), 0, c.s,
                                   c.p->y_off, c.B, c.T_y, P, marg_ref2(m, N, c.T_x), cptr<T>(y),
                                   cptr<T>(c.p->m0), cptr<T>(c.p->N0), gamma_ref(g, c.T_y),
                                   store_obs ? 1 : 0, er, sh.T[0], sh.E[0], taylor, 0,
                                   c.dev_m ? 1 : 0);
            return hip_check(hipGetLastError(), "slr + filter elements launch");
        }
    }
    return 1;
}

template <typename T, int NX, int NY>
int Core<T, NX, NY>::slr(const Ctx &c, const void *m, const void *N, const void *y,
                         const pss_gamma *out)
{
    const int tb = 128;
    const dim3 grid((unsigned)((c.T_x + tb - 1) / tb));
    const int lin = c.p->linearization;
    const int cov = c.p->form == PSS_FORM_COV ? 1 : 0;
    if constexpr (NX == 5 && NY == 2) {
        if (c.p->model == PSS_MODEL_CT_BEARINGS) {
            const CTParams<T> P = ct_params<T>(ct_host(c.p));
            if (lin == PSS_LIN_CUBATURE || lin == PSS_LIN_TAYLOR) {
                KTime kt(c.s, "slr", "", 0);
                hipLaunchKernelGGL((k_slr_ct<T>), grid, dim3(tb), 0, c.s, c.p->y_off, c.B, c.T_x,
                                   c.T_y, P, marg_ref2(m, N, c.T_x), cptr<T>(y),
                                   gamma_ref(out, c.T_y), lin == PSS_LIN_TAYLOR ? 1 : 0, cov,
                                   c.dev_m ? 1 : 0);
            } else {
                RuleSpec<T> R;
                if (!rule_spec(c.p, NX, R))
                    return PSS_EINVAL;
                KTime kt(c.s, "slr", "", 0);
                hipLaunchKernelGGL((k_slr_ct_rule<T>), grid, dim3(tb), 0, c.s, c.p->y_off, c.B,
                                   c.T_x, c.T_y, P, marg_ref2(m, N, c.T_x), cptr<T>(y),
                                   gamma_ref(out, c.T_y), R, cov, c.dev_m ? 1 : 0);
            }
            return hip_check(hipGetLastError(), "slr launch");
        }
    }
    if constexpr (NX == 1 && NY == 1) {
        if (c.p->model == PSS_MODEL_RICKER_POISSON) {
            const RickerHost h = ricker_host(c.p);
            RickerParams<T> P;
            P.loga = (T)h.loga;
            P.b = (T)h.b;
            P.sqQ = (T)h.sqQ;
            RuleSpec<T> R{};
            if (lin != PSS_LIN_TAYLOR && !rule_spec(c.p, NX, R))
                return PSS_EINVAL;
            KTime kt(c.s, "slr", "", 0);
            hipLaunchKernelGGL((k_slr_ricker<T>), grid, dim3(tb), 0, c.s, c.p->y_off, c.B, c.T_x, P,
                               marg_ref2(m, N, c.T_x), gamma_ref(out, c.T_y),
                               lin == PSS_LIN_TAYLOR ? 1 : 0, R, cov);
            return hip_check(hipGetLastError(), "slr launch");
        }
    }
    (void)y;
    set_error("no linearisation is built for this model and dimension pair");
    return PSS_EUNSUPPORTED;
}

template <typename T, int NX, int NY>
int Core<T, NX, NY>::grad_terms(const Ctx &c, const pss_gamma *g, const void *y, const void *mf,
                                const void *Nf, const void *ms, const void *Ns, double *gterms)
{
    if constexpr (NX == 5 && NY == 2) {
        const CTHost h = ct_host(c.p);
        CTGradParams<T> gp;
        for (int i = 0; i < 5; ++i)
            for (int j = 0; j < 5; ++j) {
                gp.L1[i][j] = (T)h.L1[i][j];
                gp.L2[i][j] = (T)h.L2[i][j];
            }
        gp.sig2 = (T)(h.sigma * h.sigma);
        const int tb = 128;
        KTime kt(c.s, "grad_terms", "", 0);
        hipLaunchKernelGGL((k_grad_ct<T>), dim3((unsigned)((c.T_y + tb - 1) / tb)), dim3(tb), 0,
                           c.s, c.p->y_off, c.B, c.T_y, gamma_ref(g, c.T_y), cptr<T>(y),
                           marg_ref2(mf, Nf, c.T_x), marg_ref2(ms, Ns, c.T_x), gp, gterms);
        return hip_check(hipGetLastError(), "grad launch");
    } else {
        set_error("the gradient needs the coordinated-turn model");
        return PSS_EUNSUPPORTED;
    }
}

// forwarding definitions of the public per-dimension interface
template <typename T, int NX, int NY>
size_t Impl<T, NX, NY>::ws_size(const Ctx &c, int op) { return Core<T, NX, NY>::ws_size(c, op); }
template <typename T, int NX, int NY>
int Impl<T, NX, NY>::slr(const Ctx &c, const void *m, const void *N, const void *y,
                         const pss_gamma *out)
{
    return Core<T, NX, NY>::slr(c, m, N, y, out);
}
template <typename T, int NX, int NY>
int Impl<T, NX, NY>::felem(const Ctx &c, const pss_gamma *g, const void *y, const pss_felem *out)
{
    return Core<T, NX, NY>::felem(c, g, y, out);
}
template <typename T, int NX, int NY>
int Impl<T, NX, NY>::fscan(const Ctx &c, const pss_felem *el, void *mf, void *Nf, void *ws)
{
    return Core<T, NX, NY>::fscan(c, el, mf, Nf, ws);
}
template <typename T, int NX, int NY>
int Impl<T, NX, NY>::sscan(const Ctx &c, const pss_gamma *g, const void *mf, const void *Nf,
                           void *ms, void *Ns, void *ws)
{
    return Core<T, NX, NY>::sscan(c, g, mf, Nf, ms, Ns, ws);
}
template <typename T, int NX, int NY>
int Impl<T, NX, NY>::ipls(const Ctx &c, const pss_gamma *g, const void *y, int n_iter,
                          void *m_nom, void *N_nom, void *mf_out, void *Nf_out, void *ws)
{
    return Core<T, NX, NY>::ipls(c, g, y, n_iter, m_nom, N_nom, mf_out, Nf_out, ws);
}
template <typename T, int NX, int NY>
int Impl<T, NX, NY>::loglik(const Ctx &c, const pss_gamma *g, const void *m_nom,
                            const void *N_nom, const void *y, double *ll, const pss_ckpt *ckpt,
                            void *ws)
{
    return Core<T, NX, NY>::loglik(c, g, m_nom, N_nom, y, ll, ckpt, ws);
}
template <typename T, int NX, int NY>
int Impl<T, NX, NY>::loglik_grad(const Ctx &c, const void *m_nom, const void *N_nom,
                                 const void *y, const double *ll_bar, const pss_ckpt *ckpt,
                                 double *ll, double *grad, double *theta_bar, void *ws)
{
    return Core<T, NX, NY>::loglik_grad(c, m_nom, N_nom, y, ll_bar, ckpt, ll, grad, theta_bar,
                                        ws);
}
template <typename T, int NX, int NY>
int Impl<T, NX, NY>::loglik_vjp(const Ctx &c, const pss_gamma *g, const void *m_nom,
                                const void *N_nom, const void *y, const double *ll_bar,
                                const pss_ckpt *ckpt, double *ll, const pss_gamma *gbar,
                                void *m0_bar, void *N0_bar, void *ws)
{
    return Core<T, NX, NY>::loglik_vjp(c, g, m_nom, N_nom, y, ll_bar, ckpt, ll, gbar, m0_bar,
                                       N0_bar, ws);
}
template <typename T, int NX, int NY>
int Impl<T, NX, NY>::score_fisher(const Ctx &c, const void *m_nom, const void *N_nom,
                                  const void *y, const double *ll_bar, double *ll, double *grad,
                                  double *theta_bar, void *ws)
{
    return Core<T, NX, NY>::score_fisher(c, m_nom, N_nom, y, ll_bar, ll, grad, theta_bar, ws);
}
template <typename T, int NX, int NY>
size_t Impl<T, NX, NY>::ckpt_bytes(const Ctx &c, int level)
{
    return Core<T, NX, NY>::ckpt_bytes(c, level);
}
template <typename T, int NX, int NY>
int Impl<T, NX, NY>::filter_levels(const Ctx &c)
{
    return Core<T, NX, NY>::filter_levels(c);
}
template <typename T, int NX, int NY>
int Impl<T, NX, NY>::sequential(const Ctx &c, const pss_gamma *g, const void *y, int n_iter,
                                void *m_nom, void *N_nom, void *mf_out, void *Nf_out, void *ws)
{
    return Core<T, NX, NY>::sequential(c, g, y, n_iter, m_nom, N_nom, mf_out, Nf_out, ws);
}

} // namespace pss
