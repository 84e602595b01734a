// Persistent, work-queue form of one IPLS pass for ragged batches of several
// model groups in ONE launch (gfx950).
//
// Work items are (group, sequence, tile) triples handed out in a fixed order
// by one atomic counter: first every filter tile of every group, then every
// smoother tile (smoother tiles in reverse time order).  For batches of many
// sequences the order is time-major (tile 0 of every sequence, then tile 1,
// ...), so the blocks running at the same time work on different sequences
// and a tile's predecessor has long finished; otherwise it is sequence by
// sequence, tiles in order.  A filter tile builds its elements on the fly (SLR at the previous
// nominal for the CT model, then Lemma 1), folds them, runs the in-LDS
// up-sweep, then chains with its predecessor: it waits for tile t-1's
// published inclusive prefix (a filtering marginal), publishes its own
// inclusive prefix = prefix(t-1) (x) aggregate(t), and finishes with the
// down-sweep and the apply pass.  Smoother tiles mirror this backwards in
// time, after waiting for the filter tiles whose marginals and transition
// parameters they read.  Every wait is on an item with a SMALLER index, so
// the lowest unfinished item never waits and the queue always drains; waits
// are bounded and raise an error flag instead of spinning forever.
// The bracketing inside and across tiles depends only on the sequence
// lengths and launch shape, so results are bitwise reproducible.
#pragma once

#include "kernels.hpp"

namespace pss {

constexpr int kMaxGroups = 4;
constexpr int kGroupCT = 1;      // coordinated-turn bearings, nx 5, ny 2
constexpr int kGroupLinear4 = 2; // linear model, nx 4, ny 2

template <typename T>
struct PGroup {
    int kind;
    int B;
    int E_f, E_s;
    int stage_f, stage_s; // outputs staged through LDS (see apply_phase)
    int taylor;           // CT: first-order Taylor instead of cubature SLR
    const int64_t *y_off;
    int64_t T_y, T_x;
    const T *y;
    const T *m0, *N0;
    // nominal trajectory: read from *_in, smoothing marginals written to *_out
    const T *nom_in_m, *nom_in_N;
    T *nom_out_m, *nom_out_N;
    // workspace
    T *mf, *Nf;            // filtering marginals [P_marg][T_x]
    T *fstash;             // filter elements [NE_f][T_y]
    T *gstash;             // transition linearisation [NX^2 + NX + P][T_y]
    T *sstash;             // smoother elements [NE_s][T_x]
    T *pre_f, *pre_s;      // published inclusive prefixes / suffixes [P_marg][tiles]
    int *flag_f, *done_f;  // per filter tile: prefix published, outputs written
    int *flag_s;           // per smoother tile: suffix published
    const int64_t *tile_f, *tile_s; // per-sequence tile offsets [B+1]
    int64_t item_f0, item_s0;       // first global item of this group's phases
    int seq0;                       // first global sequence index of this group
    int64_t ntiles_f, ntiles_s;
    // linear model parameters (kind == kGroupLinear4)
    const T *gF, *gc, *gSL, *gH, *gd, *gSO;
    int64_t gstride;
    // CT model constants (kind == kGroupCT)
    CTParams<T> ct;
};

template <typename T>
struct PArgs {
    PGroup<T> g[kMaxGroups];
    int n_groups;
    int64_t total_items;
    // time-major order (rr != 0): filter item r = t * B_all + s is tile t of
    // global sequence s (skipped if that sequence has fewer tiles), for t <
    // maxt_f; then the smoother items likewise; otherwise items run group by
    // group, sequence by sequence, tile by tile
    int rr;
    int B_all;
    int64_t n_f_items;
    int *counter;   // work counter (reset before each pass)
    int *error;     // set if a wait exceeded its bound
    int spin_limit; // bounded waits
};

// ---- synchronisation helpers (vector atomics on global memory) ------------
PSS_INL int flag_load(int *p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
PSS_INL void flag_store(int *p, int v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
// thread 0 waits until *p != 0 (bounded); returns false on timeout
PSS_INL bool wait_flag(int *p, int limit)
{
    for (int it = 0; it < limit; ++it) {
        if (flag_load(p) != 0)
            return true;
        __builtin_amdgcn_s_sleep(4);
    }
    return false;
}

template <typename T, int NX>
PSS_INL MargRef<T, NX> pre_ref(T *base, int64_t ld)
{
    MargRef<T, NX> r;
    r.ld = ld;
    r.m = base;
    r.N = base + (int64_t)NX * ld;
    return r;
}

template <typename T, int NX>
PSS_INL FElemRef<T, NX> felem_ref_dev(T *base, int64_t ld)
{
    FElemRef<T, NX> r;
    r.ld = ld;
    r.A = base;
    r.b = r.A + (int64_t)NX * NX * ld;
    r.U = r.b + (int64_t)NX * ld;
    r.eta = r.U + (int64_t)tri_size(NX) * ld;
    r.Z = r.eta + (int64_t)NX * ld;
    return r;
}

template <typename T, int NX>
PSS_INL SElemRef<T, NX> selem_ref_dev(T *base, int64_t ld)
{
    SElemRef<T, NX> r;
    r.ld = ld;
    r.E = base;
    r.g = r.E + (int64_t)NX * NX * ld;
    r.D = r.g + (int64_t)NX * ld;
    return r;
}

// transition part of a linearisation, stashed per step slot by filter tiles
template <typename T, int NX>
struct TransRef {
    T *F, *c, *SL;
    int64_t ld;
    PSS_INL void store(int64_t t, const T (&Fm)[NX][NX], const T (&cv)[NX],
                       const T (&S)[NX][NX]) const
    {
#pragma unroll
        for (int i = 0; i < NX; ++i) {
#pragma unroll
            for (int j = 0; j < NX; ++j)
                F[(i * NX + j) * ld + t] = Fm[i][j];
            c[i * ld + t] = cv[i];
#pragma unroll
            for (int j = 0; j <= i; ++j)
                SL[tri_idx(i, j) * ld + t] = S[i][j];
        }
    }
    PSS_INL void load(int64_t t, T (&Fm)[NX][NX], T (&cv)[NX], T (&S)[NX][NX]) const
    {
#pragma unroll
        for (int i = 0; i < NX; ++i) {
#pragma unroll
            for (int j = 0; j < NX; ++j)
                Fm[i][j] = F[(i * NX + j) * ld + t];
            cv[i] = c[i * ld + t];
#pragma unroll
            for (int j = 0; j <= i; ++j)
                S[i][j] = SL[tri_idx(i, j) * ld + t];
        }
    }
};

template <typename T, int NX>
PSS_INL TransRef<T, NX> trans_ref_dev(T *base, int64_t ld)
{
    TransRef<T, NX> r;
    r.ld = ld;
    r.F = base;
    r.c = r.F + (int64_t)NX * NX * ld;
    r.SL = r.c + (int64_t)NX * ld;
    return r;
}

// ---- element sources of the fused pass ------------------------------------
// filter: element of step position p (slot off + p) built from the model
template <typename T, int NX, int NY, bool CT>
struct FusedFiltSrc {
    const PGroup<T> *G;
    int64_t x0; // first state slot of the sequence
    PSS_INL void store(const TileInfo &ti, int64_t p, FElem<T, NX> &e) const
    {
        felem_ref_dev<T, NX>(G->fstash, G->T_y).store(ilv_slot(ti, p), e);
    }
    PSS_INL void build(const TileInfo &ti, int64_t p, FElem<T, NX> &e) const
    {
        const int64_t s = ti.off + p;
        T F[NX][NX], c[NX], SL[NX][NX], H[NY][NX], d[NY], SO[NY][NY], yy[NY];
#pragma unroll
        for (int a = 0; a < NY; ++a)
            yy[a] = G->y[a * G->T_y + s];
        if constexpr (CT) {
            MargRef<T, NX> nom;
            nom.m = const_cast<T *>(G->nom_in_m);
            nom.N = const_cast<T *>(G->nom_in_N);
            nom.ld = G->T_x;
            Marg<T, NX> prev, cur;
            nom.load(x0 + p, prev);
            nom.load(x0 + p + 1, cur);
            if (G->taylor) {
                ct_taylor_transition(G->ct, prev, F, c, SL);
                ct_taylor_bearings(G->ct, cur, yy, H, d, SO);
            } else {
                ct_slr_transition(G->ct, prev, F, c, SL);
                ct_slr_bearings(G->ct, cur, yy, H, d, SO);
            }
            trans_ref_dev<T, NX>(G->gstash, G->T_y).store(s, F, c, SL);
        } else {
            GammaRef<T, NX, NY> gr;
            gr.F = const_cast<T *>(G->gF);
            gr.c = const_cast<T *>(G->gc);
            gr.SL = const_cast<T *>(G->gSL);
            gr.H = const_cast<T *>(G->gH);
            gr.d = const_cast<T *>(G->gd);
            gr.SO = const_cast<T *>(G->gSO);
            gr.stride = G->gstride;
            gr.ld = G->gstride ? G->T_y : 1;
            gr.load_trans(s, F, c, SL);
            gr.load_obs(s, H, d, SO);
        }
        if (p == 0) {
            T m[NX], N[NX][NX];
#pragma unroll
            for (int i = 0; i < NX; ++i) {
                m[i] = G->m0[i];
#pragma unroll
                for (int j = 0; j <= i; ++j)
                    N[i][j] = G->N0[tri_idx(i, j)];
            }
            filter_element_first(m, N, F, c, SL, H, d, SO, yy, e);
        } else {
            filter_element(F, c, SL, H, d, SO, yy, e);
        }
    }
    static constexpr bool lazy_up = false, lazy_down = true;
    static constexpr int leaf_nz = NY < NX ? NY : NX; // Z = Tria([Z_k, 0])
    PSS_INL FRefV<T, NX> dview(const TileInfo &ti, int64_t p) const
    {
        return view_of(felem_ref_dev<T, NX>(G->fstash, G->T_y), ilv_slot(ti, p));
    }
};

// smoother: element of state k = n - p (Table 4) from the stashed transition
// parameters (CT) or the model (linear) and the filtering marginal
template <typename T, int NX, int NY, bool CT>
struct FusedSmoothSrc {
    const PGroup<T> *G;
    int64_t ybase; // y_off[b]
    PSS_INL void store(const TileInfo &ti, int64_t p, SElem<T, NX> &e) const
    {
        selem_ref_dev<T, NX>(G->sstash, G->T_x).store(ilv_slot(ti, p), e);
    }
    PSS_INL void build(const TileInfo &ti, int64_t p, SElem<T, NX> &e) const
    {
        const int64_t n = ti.cnt - 1, k = n - p;
        Marg<T, NX> f;
        pre_ref<T, NX>(G->mf, G->T_x).load(ti.off + k, f);
        if (k == n) {
            smoother_element_last(f, e);
        } else {
            T F[NX][NX], c[NX], SL[NX][NX];
            if constexpr (CT) {
                trans_ref_dev<T, NX>(G->gstash, G->T_y).load(ybase + k, F, c, SL);
            } else {
                GammaRef<T, NX, NY> gr;
                gr.F = const_cast<T *>(G->gF);
                gr.c = const_cast<T *>(G->gc);
                gr.SL = const_cast<T *>(G->gSL);
                gr.H = const_cast<T *>(G->gH);
                gr.d = const_cast<T *>(G->gd);
                gr.SO = const_cast<T *>(G->gSO);
                gr.stride = G->gstride;
                gr.ld = G->gstride ? G->T_y : 1;
                gr.load_trans(ybase + k, F, c, SL);
            }
            smoother_element(F, c, SL, f, e);
        }
    }
    static constexpr bool lazy_up = false, lazy_down = true;
    static constexpr int leaf_nz = 0;
    PSS_INL SRefV<T, NX> dview(const TileInfo &ti, int64_t p) const
    {
        return view_of(selem_ref_dev<T, NX>(G->sstash, G->T_x), ilv_slot(ti, p));
    }
};

// A tile first builds all its elements into the tile-interleaved stash, lane
// q on elements q, q + Tb, ... (consecutive lanes read consecutive steps of
// the nominal, y and the stashed linearisation, whole lines per load), then
// folds them back lazily: the model linearisation and element construction
// never share registers with the fold's operator, so the kernel's register
// peak is the larger of the two phases rather than their sum.
template <class Src>
struct Stashed {
    static constexpr bool lazy_up = true, lazy_down = true;
    static constexpr int leaf_nz = Src::leaf_nz;
    Src src;
    PSS_INL auto uview(const TileInfo &ti, int64_t p) const { return src.dview(ti, p); }
    PSS_INL auto dview(const TileInfo &ti, int64_t p) const { return src.dview(ti, p); }
};

// The block calls this uniformly.  Round r builds elements r Tb .. r Tb +
// Tb - 1, lane q on element r Tb + q (consecutive lanes read consecutive
// steps), into LDS; the lanes then take the round's elements grouped by
// interleaved position -- element t E + j of the round goes to lane
// j (Tb / E) + (t - t0) -- so each store writes runs of Tb / E consecutive
// words of the stash rather than E runs of Tb / E / E (the direct order is
// kept when E does not divide Tb).  The last barrier publishes the stash to
// the lanes whose fold reads it and frees the LDS for the tree.
template <class Op, class Src>
PSS_INL void build_phase(const TileInfo &ti, const Src &src, typename Op::T *lds)
{
    const int Tb = blockDim.x, tid = threadIdx.x, E = ti.E;
    const bool grouped = Tb % E == 0;
    const int m = Tb / E;
    for (int r0 = 0; r0 < ti.tcnt; r0 += Tb) {
        __syncthreads(); // the previous round's readers are done with the LDS
        typename Op::Elem e;
        if (r0 + tid < ti.tcnt) {
            src.build(ti, ti.start + r0 + tid, e);
            lds_put(e, lds, Tb, tid);
        }
        __syncthreads();
        const int qi = grouped ? (tid % m) * E + tid / m : tid; // element of the round
        if (r0 + qi < ti.tcnt) {
            lds_get(e, lds, Tb, qi);
            src.store(ti, ti.start + r0 + qi, e);
        }
    }
    __syncthreads();
}

// ---- one tile of a phase ----------------------------------------------------// ---- one tile of a phase ----------------------------------------------------
template <typename T, int NX, int NY, bool CT>
PSS_INL void filter_tile(const PArgs<T> &a, const PGroup<T> &G, int64_t gt, T *lds)
{
    using Op = FilterScan<T, NX>;
    const int b = find_seq(G.tile_f, G.B, gt, 0);
    const int64_t t = gt - G.tile_f[b];
    LevelGeom g;
    g.y_off = G.y_off;
    g.elem_off = nullptr;
    g.tile_off = G.tile_f;
    g.level = 0;
    g.extra = 0;
    g.B = G.B;
    g.E = G.E_f;
    g.stage = G.stage_f;
    TileInfo ti;
    ti.b = b;
    seq_range(g, b, ti.off, ti.cnt);
    const int64_t TS = (int64_t)blockDim.x * g.E;
    ti.start = t * TS;
    const int64_t rem = ti.cnt - ti.start;
    ti.tcnt = (int)(rem < TS ? rem : TS);
    ti.nvalid = (ti.tcnt + g.E - 1) / g.E;
    ti.E = g.E;
    const int Tb = blockDim.x;
    FusedFiltSrc<T, NX, NY, CT> build{&G, G.y_off[b] + b};
    build_phase<Op>(ti, build, lds);
    Stashed<FusedFiltSrc<T, NX, NY, CT>> src{build};
    fold_phase<Op>(g, ti, src, lds, Tb);
    tree_up<Op>(lds, Tb, ti.nvalid);
    typename Op::Pre excl;
    if (threadIdx.x == 0) {
        MargRef<T, NX> pub = pre_ref<T, NX>(G.pre_f, G.ntiles_f);
        if (t == 0) {
            StartPre<T, NX>{G.m0, G.N0}.get(excl);
        } else {
            if (!wait_flag(G.flag_f + gt - 1, a.spin_limit))
                atomicOr(a.error, 1);
            pub.load(gt - 1, excl);
        }
        typename Op::Pre incl;
        Op::apply_v(excl, Op::slot(lds, Tb, Tb - 1), incl);
        pub.store(gt, incl);
        flag_store(G.flag_f + gt, 1);
    }
    tree_down<Op>(lds, Tb, ti.nvalid, excl);
    FiltDst<T, NX> dst{pre_ref<T, NX>(G.mf, G.T_x), G.y_off};
    apply_phase<Op>(g, ti, src, dst, lds, Tb);
    __threadfence(); // every thread's outputs visible device-wide before the flag
    __syncthreads();
    if (threadIdx.x == 0)
        flag_store(G.done_f + gt, 1);
}

template <typename T, int NX, int NY, bool CT>
PSS_INL void smoother_tile(const PArgs<T> &a, const PGroup<T> &G, int64_t gu, T *lds)
{
    using Op = SmootherScan<T, NX>;
    const int b = find_seq(G.tile_s, G.B, gu, 0);
    const int64_t u = gu - G.tile_s[b];
    LevelGeom g;
    g.y_off = G.y_off;
    g.elem_off = nullptr;
    g.tile_off = G.tile_s;
    g.level = 0;
    g.extra = 1;
    g.B = G.B;
    g.E = G.E_s;
    g.stage = G.stage_s;
    TileInfo ti;
    ti.b = b;
    seq_range(g, b, ti.off, ti.cnt);
    const int64_t TS = (int64_t)blockDim.x * g.E;
    ti.start = u * TS;
    const int64_t rem = ti.cnt - ti.start;
    ti.tcnt = (int)(rem < TS ? rem : TS);
    ti.nvalid = (ti.tcnt + g.E - 1) / g.E;
    ti.E = g.E;
    const int Tb = blockDim.x;
    const int64_t n = ti.cnt - 1;
    // states [klo, khi] of this tile; wait for the filter tiles that wrote
    // their marginals and the transition parameters of steps klo+1..khi+1
    if (threadIdx.x == 0) {
        const int64_t khi = n - ti.start, klo = n - (ti.start + ti.tcnt - 1);
        const int64_t s_lo = klo > 1 ? klo : 1;
        const int64_t s_hi = (khi + 1) < n ? (khi + 1) : n;
        const int64_t TSf = (int64_t)blockDim.x * G.E_f;
        const int64_t f0 = G.tile_f[b];
        for (int64_t tf = (s_lo - 1) / TSf; tf <= (s_hi - 1) / TSf; ++tf)
            if (!wait_flag(G.done_f + f0 + tf, a.spin_limit))
                atomicOr(a.error, 2);
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    FusedSmoothSrc<T, NX, NY, CT> build{&G, G.y_off[b]};
    build_phase<Op>(ti, build, lds);
    Stashed<FusedSmoothSrc<T, NX, NY, CT>> src{build};
    fold_phase<Op>(g, ti, src, lds, Tb);
    tree_up<Op>(lds, Tb, ti.nvalid);
    typename Op::Pre excl;
    if (threadIdx.x == 0) {
        MargRef<T, NX> pub = pre_ref<T, NX>(G.pre_s, G.ntiles_s);
        if (u == 0) {
            StartPre<T, NX>{nullptr, nullptr}.get(excl);
        } else {
            if (!wait_flag(G.flag_s + gu - 1, a.spin_limit))
                atomicOr(a.error, 4);
            pub.load(gu - 1, excl);
        }
        typename Op::Pre incl;
        Op::apply_v(excl, Op::slot(lds, Tb, Tb - 1), incl);
        pub.store(gu, incl);
        flag_store(G.flag_s + gu, 1);
    }
    tree_down<Op>(lds, Tb, ti.nvalid, excl);
    SmoothDst<T, NX> dst{pre_ref<T, NX>(G.nom_out_m, G.T_x)};
    dst.out.N = G.nom_out_N;
    apply_phase<Op>(g, ti, src, dst, lds, Tb);
    __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(256) void k_ipls_persistent(PArgs<T> a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);
    __shared__ int item_sh;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0)
            item_sh = atomicAdd(a.counter, 1);
        __syncthreads();
        const int64_t item = item_sh;
        if (item >= a.total_items)
            break;
        // filter items of all groups first, then smoother items
        if (a.rr) {
            const bool smooth = item >= a.n_f_items;
            const int64_t r = smooth ? item - a.n_f_items : item;
            const int64_t t = r / a.B_all;
            const int sg = (int)(r - t * a.B_all);
            int gi = 0;
            while (gi + 1 < a.n_groups && sg >= a.g[gi + 1].seq0)
                ++gi;
            const PGroup<T> &G = a.g[gi];
            const int sq = sg - G.seq0;
            const int64_t *toff = smooth ? G.tile_s : G.tile_f;
            const int64_t t0 = toff[sq];
            if (t < toff[sq + 1] - t0) {
                if (!smooth) {
                    if (G.kind == kGroupCT)
                        filter_tile<T, 5, 2, true>(a, G, t0 + t, lds);
                    else
                        filter_tile<T, 4, 2, false>(a, G, t0 + t, lds);
                } else {
                    if (G.kind == kGroupCT)
                        smoother_tile<T, 5, 2, true>(a, G, t0 + t, lds);
                    else
                        smoother_tile<T, 4, 2, false>(a, G, t0 + t, lds);
                }
            }
            continue;
        }
        for (int gi = 0; gi < a.n_groups; ++gi) {
            const PGroup<T> &G = a.g[gi];
            if (item >= G.item_f0 && item < G.item_f0 + G.ntiles_f) {
                const int64_t gt = item - G.item_f0;
                if (G.kind == kGroupCT)
                    filter_tile<T, 5, 2, true>(a, G, gt, lds);
                else
                    filter_tile<T, 4, 2, false>(a, G, gt, lds);
            } else if (item >= G.item_s0 && item < G.item_s0 + G.ntiles_s) {
                const int64_t gu = item - G.item_s0;
                if (G.kind == kGroupCT)
                    smoother_tile<T, 5, 2, true>(a, G, gu, lds);
                else
                    smoother_tile<T, 4, 2, false>(a, G, gu, lds);
            }
        }
    }
}

// clears the per-pass flags and the work counter (a kernel, so that the pass
// can be captured in a graph without memset nodes)
__global__ __launch_bounds__(256) void k_clear_ints(int *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

template <typename T>
__global__ __launch_bounds__(256) void k_copy(const T *src, T *dst, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

} // namespace pss
