// HIP kernels of the parallel square-root smoother for gfx950.
//
// Scan structure (one per direction): a reduce-then-scan over tiles with a
// fixed bracketing, so results are bitwise reproducible and a sequence's
// result does not depend on the rest of its batch.
//   level 0 elements are the paper's elements; a tile is TS = T * E
//   consecutive elements of ONE sequence, handled by a block of T threads:
//     fold    - thread t folds its E elements left to right (full operator)
//     up      - in-LDS up-sweep over the T thread aggregates (Blelloch)
//     down    - in-LDS down-sweep seeded with the tile's exclusive prefix;
//               prefixes are true prefixes (A = 0 / E = 0), so only the
//               marginal (m, N) travels and the cheap "apply" form is used
//     apply   - thread t walks its E elements again, producing the outputs
//   the tile aggregates of level l are the elements of level l + 1, until a
//   level has one tile per sequence; that top level runs fold, up, down and
//   apply in one kernel; lower levels run an "up" kernel (fold + up-sweep,
//   LDS tree saved to global) and later a "down" kernel.
// LDS holds one object per thread, component-major ([c * T + slot]) so that
// consecutive lanes touch consecutive words.
#pragma once

#include <type_traits>

#include "common.hpp"
#include "device_cov.hpp"
#include "device_ops.hpp"
#include "device_rules.hpp"
#include "device_wave.hpp"

namespace pss {

// ---------------------------------------------------------------------------
// SoA references and loads / stores
// ---------------------------------------------------------------------------
template <typename T, int NX>
struct MargRef {
    T *m;
    T *N;
    int64_t ld;
    PSS_INL void load(int64_t t, Marg<T, NX> &x) const
    {
#pragma unroll
        for (int i = 0; i < NX; ++i)
            x.m[i] = m[i * ld + t];
#pragma unroll
        for (int i = 0; i < NX; ++i)
#pragma unroll
            for (int j = 0; j <= i; ++j)
                x.N[i][j] = N[tri_idx(i, j) * ld + t];
    }
    PSS_INL void store(int64_t t, const Marg<T, NX> &x) const
    {
#pragma unroll
        for (int i = 0; i < NX; ++i)
            m[i * ld + t] = x.m[i];
#pragma unroll
        for (int i = 0; i < NX; ++i)
#pragma unroll
            for (int j = 0; j <= i; ++j)
                N[tri_idx(i, j) * ld + t] = x.N[i][j];
    }
};

template <typename T, int NX>
struct FElemRef {
    T *A, *b, *U, *eta, *Z;
    int64_t ld;
    PSS_INL void load(int64_t t, FElem<T, NX> &e) const
    {
#pragma unroll
        for (int i = 0; i < NX; ++i) {
#pragma unroll
            for (int j = 0; j < NX; ++j)
                e.A[i][j] = A[(i * NX + j) * ld + t];
            e.b[i] = b[i * ld + t];
            e.eta[i] = eta[i * ld + t];
#pragma unroll
            for (int j = 0; j <= i; ++j) {
                e.U[i][j] = U[tri_idx(i, j) * ld + t];
                e.Z[i][j] = Z[tri_idx(i, j) * ld + t];
            }
        }
    }
    PSS_INL void store(int64_t t, const FElem<T, NX> &e) const
    {
#pragma unroll
        for (int i = 0; i < NX; ++i) {
#pragma unroll
            for (int j = 0; j < NX; ++j)
                A[(i * NX + j) * ld + t] = e.A[i][j];
            b[i * ld + t] = e.b[i];
            eta[i * ld + t] = e.eta[i];
#pragma unroll
            for (int j = 0; j <= i; ++j) {
                U[tri_idx(i, j) * ld + t] = e.U[i][j];
                Z[tri_idx(i, j) * ld + t] = e.Z[i][j];
            }
        }
    }
};

template <typename T, int NX>
struct SElemRef {
    T *E, *g, *D;
    int64_t ld;
    PSS_INL void load(int64_t t, SElem<T, NX> &e) const
    {
#pragma unroll
        for (int i = 0; i < NX; ++i) {
#pragma unroll
            for (int j = 0; j < NX; ++j)
                e.E[i][j] = E[(i * NX + j) * ld + t];
            e.g[i] = g[i * ld + t];
#pragma unroll
            for (int j = 0; j <= i; ++j)
                e.D[i][j] = D[tri_idx(i, j) * ld + t];
        }
    }
    PSS_INL void store(int64_t t, const SElem<T, NX> &e) const
    {
#pragma unroll
        for (int i = 0; i < NX; ++i) {
#pragma unroll
            for (int j = 0; j < NX; ++j)
                E[(i * NX + j) * ld + t] = e.E[i][j];
            g[i * ld + t] = e.g[i];
#pragma unroll
            for (int j = 0; j <= i; ++j)
                D[tri_idx(i, j) * ld + t] = e.D[i][j];
        }
    }
};

// views of element t of an SoA reference (fields read and written in place)
template <typename T, int NX>
struct FRefV {
    FElemRef<T, NX> r;
    int64_t t;
    PSS_INL T A(int i, int j) const { return r.A[(i * NX + j) * r.ld + t]; }
    PSS_INL T b(int i) const { return r.b[i * r.ld + t]; }
    PSS_INL T U(int i, int j) const { return r.U[tri_idx(i, j) * r.ld + t]; }
    PSS_INL T eta(int i) const { return r.eta[i * r.ld + t]; }
    PSS_INL T Z(int i, int j) const { return r.Z[tri_idx(i, j) * r.ld + t]; }
    PSS_INL void sA(int i, int j, T v) const { r.A[(i * NX + j) * r.ld + t] = v; }
    PSS_INL void sb(int i, T v) const { r.b[i * r.ld + t] = v; }
    PSS_INL void sU(int i, int j, T v) const { r.U[tri_idx(i, j) * r.ld + t] = v; }
    PSS_INL void seta(int i, T v) const { r.eta[i * r.ld + t] = v; }
    PSS_INL void sZ(int i, int j, T v) const { r.Z[tri_idx(i, j) * r.ld + t] = v; }
};

template <typename T, int NX>
struct SRefV {
    SElemRef<T, NX> r;
    int64_t t;
    PSS_INL T E(int i, int j) const { return r.E[(i * NX + j) * r.ld + t]; }
    PSS_INL T g(int i) const { return r.g[i * r.ld + t]; }
    PSS_INL T D(int i, int j) const { return r.D[tri_idx(i, j) * r.ld + t]; }
    PSS_INL void sE(int i, int j, T v) const { r.E[(i * NX + j) * r.ld + t] = v; }
    PSS_INL void sg(int i, T v) const { r.g[i * r.ld + t] = v; }
    PSS_INL void sD(int i, int j, T v) const { r.D[tri_idx(i, j) * r.ld + t] = v; }
};

template <typename T, int NX>
PSS_INL FRefV<T, NX> view_of(const FElemRef<T, NX> &r, int64_t t)
{
    return FRefV<T, NX>{r, t};
}

template <typename T, int NX>
PSS_INL SRefV<T, NX> view_of(const SElemRef<T, NX> &r, int64_t t)
{
    return SRefV<T, NX>{r, t};
}

// linearisation parameters (stride 0: one shared set)
template <typename T, int NX, int NY>
struct GammaRef {
    T *F, *c, *SL, *H, *d, *SO;
    int64_t ld;     // T_y (or 1 when shared)
    int64_t stride; // 0 or 1
    PSS_INL void load_trans(int64_t t, T (&Fm)[NX][NX], T (&cv)[NX], T (&S)[NX][NX]) const
    {
        const int64_t u = t * stride;
#pragma unroll
        for (int i = 0; i < NX; ++i) {
#pragma unroll
            for (int j = 0; j < NX; ++j)
                Fm[i][j] = F[(i * NX + j) * ld + u];
            cv[i] = c[i * ld + u];
#pragma unroll
            for (int j = 0; j <= i; ++j)
                S[i][j] = SL[tri_idx(i, j) * ld + u];
        }
    }
    PSS_INL void load_obs(int64_t t, T (&Hm)[NY][NX], T (&dv)[NY], T (&S)[NY][NY]) const
    {
        const int64_t u = t * stride;
#pragma unroll
        for (int a = 0; a < NY; ++a) {
#pragma unroll
            for (int j = 0; j < NX; ++j)
                Hm[a][j] = H[(a * NX + j) * ld + u];
            dv[a] = d[a * ld + u];
#pragma unroll
            for (int j = 0; j <= a; ++j)
                S[a][j] = SO[tri_idx(a, j) * ld + u];
        }
    }
    PSS_INL void store_trans(int64_t t, const T (&Fm)[NX][NX], const T (&cv)[NX],
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
    PSS_INL void store_obs(int64_t t, const T (&Hm)[NY][NX], const T (&dv)[NY],
                           const T (&S)[NY][NY]) const
    {
#pragma unroll
        for (int a = 0; a < NY; ++a) {
#pragma unroll
            for (int j = 0; j < NX; ++j)
                H[(a * NX + j) * ld + t] = Hm[a][j];
            d[a * ld + t] = dv[a];
#pragma unroll
            for (int j = 0; j <= a; ++j)
                SO[tri_idx(a, j) * ld + t] = S[a][j];
        }
    }
};

// ---------------------------------------------------------------------------
// sequence lookup
// ---------------------------------------------------------------------------
// largest b in [0, B) with off[b] + b * shift <= v
PSS_INL int find_seq(const int64_t *off, int B, int64_t v, int shift)
{
    int lo = 0, hi = B - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] + (int64_t)mid * shift <= v)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// scan operator policies
// ---------------------------------------------------------------------------
template <typename T_, int NX_>
struct FilterScan {
    using T = T_;
    static constexpr int NX = NX_;
    using Elem = FElem<T, NX>;
    using Pre = Marg<T, NX>;
    static constexpr int NE = Sizes<NX>::felem;
    static constexpr int NP = Sizes<NX>::marg;
    static constexpr const char *name = "filter";
    PSS_INL static void combine(const Elem &a, const Elem &b, Elem &o) { filter_combine(a, b, o); }
    PSS_INL static void apply(const Pre &p, const Elem &a, Pre &o) { filter_apply(p, a, o); }
    // view forms: `o` may view the storage of `a` or `b`
    PSS_INL static FSlotV<T, NX, int> slot(T *lds, int Tb, int s)
    {
        return FSlotV<T, NX, int>{lds + s, Tb};
    }
    PSS_INL static FRegV<T, NX> reg(Elem &e) { return FRegV<T, NX>{&e}; }
    // NZ: columns of the right element's Z that can be non-zero (xi_block)
    template <int NZ = NX, class VA, class VB, class VO>
    PSS_INL static void combine_v(const VA &a, const VB &b, const VO &o)
    {
        filter_combine_v<T, NX, NZ>(a, b, o);
    }
    template <int NZ = NX, class VA>
    PSS_INL static void apply_v(const Pre &p, const VA &a, Pre &o)
    {
        filter_apply_v<T, NX, NZ>(p, a, o);
    }
    template <class VS, class VD>
    PSS_INL static void copy_v(const VS &src, const VD &dst)
    {
        felem_copy<T, NX>(src, dst);
    }
};

// Reverse associative scan of the smoother, run as a forward scan over the
// time-reversed elements with the arguments of the operator swapped.
template <typename T_, int NX_>
struct SmootherScan {
    using T = T_;
    static constexpr int NX = NX_;
    using Elem = SElem<T, NX>;
    using Pre = Marg<T, NX>;
    static constexpr int NE = Sizes<NX>::selem;
    static constexpr int NP = Sizes<NX>::marg;
    static constexpr const char *name = "smoother";
    PSS_INL static void combine(const Elem &a, const Elem &b, Elem &o) { smoother_combine(b, a, o); }
    PSS_INL static void apply(const Pre &p, const Elem &a, Pre &o) { smoother_apply(a, p, o); }
    PSS_INL static SSlotV<T, NX, int> slot(T *lds, int Tb, int s)
    {
        return SSlotV<T, NX, int>{lds + s, Tb};
    }
    PSS_INL static SRegV<T, NX> reg(Elem &e) { return SRegV<T, NX>{&e}; }
    template <int NZ = NX, class VA, class VB, class VO>
    PSS_INL static void combine_v(const VA &a, const VB &b, const VO &o)
    {
        smoother_combine_v<T, NX>(b, a, o);
    }
    template <int NZ = NX, class VA>
    PSS_INL static void apply_v(const Pre &p, const VA &a, Pre &o)
    {
        smoother_apply_v<T, NX>(a, p, o);
    }
    template <class VS, class VD>
    PSS_INL static void copy_v(const VS &src, const VD &dst)
    {
        selem_copy<T, NX>(src, dst);
    }
};

// Standard (covariance-form) scans over the same storage (device_cov.hpp)
template <typename T_, int NX_>
struct FilterScanCov {
    using T = T_;
    static constexpr int NX = NX_;
    using Elem = FElem<T, NX>;
    using Pre = Marg<T, NX>;
    static constexpr int NE = Sizes<NX>::felem;
    static constexpr int NP = Sizes<NX>::marg;
    static constexpr const char *name = "filter_cov";
    PSS_INL static FSlotV<T, NX, int> slot(T *lds, int Tb, int s)
    {
        return FSlotV<T, NX, int>{lds + s, Tb};
    }
    PSS_INL static FRegV<T, NX> reg(Elem &e) { return FRegV<T, NX>{&e}; }
    template <int NZ = NX, class VA, class VB, class VO>
    PSS_INL static void combine_v(const VA &a, const VB &b, const VO &o)
    {
        filter_combine_cov_v<T, NX>(a, b, o);
    }
    template <int NZ = NX, class VA>
    PSS_INL static void apply_v(const Pre &p, const VA &a, Pre &o)
    {
        filter_apply_cov_v<T, NX>(p, a, o);
    }
    template <class VS, class VD>
    PSS_INL static void copy_v(const VS &src, const VD &dst)
    {
        felem_copy<T, NX>(src, dst);
    }
};

template <typename T_, int NX_>
struct SmootherScanCov {
    using T = T_;
    static constexpr int NX = NX_;
    using Elem = SElem<T, NX>;
    using Pre = Marg<T, NX>;
    static constexpr int NE = Sizes<NX>::selem;
    static constexpr int NP = Sizes<NX>::marg;
    static constexpr const char *name = "smoother_cov";
    PSS_INL static SSlotV<T, NX, int> slot(T *lds, int Tb, int s)
    {
        return SSlotV<T, NX, int>{lds + s, Tb};
    }
    PSS_INL static SRegV<T, NX> reg(Elem &e) { return SRegV<T, NX>{&e}; }
    template <int NZ = NX, class VA, class VB, class VO>
    PSS_INL static void combine_v(const VA &a, const VB &b, const VO &o)
    {
        smoother_combine_cov_v<T, NX>(b, a, o);
    }
    template <int NZ = NX, class VA>
    PSS_INL static void apply_v(const Pre &p, const VA &a, Pre &o)
    {
        smoother_apply_cov_v<T, NX>(a, p, o);
    }
    template <class VS, class VD>
    PSS_INL static void copy_v(const VS &src, const VD &dst)
    {
        selem_copy<T, NX>(src, dst);
    }
};

// LDS object access, component-major
template <class Obj, typename T>
PSS_INL void lds_get(Obj &o, const T *lds, int Tb, int s)
{
    visit(o, [&](int c, T &v) { v = lds[c * Tb + s]; });
}
template <class Obj, typename T>
PSS_INL void lds_put(Obj &o, T *lds, int Tb, int s)
{
    visit(o, [&](int c, T &v) { lds[c * Tb + s] = v; });
}

// ---------------------------------------------------------------------------
// in-LDS Blelloch sweeps over the T thread aggregates of a tile.  Slots past
// `nvalid` hold no data; a node whose right half is empty takes its left
// half, a node whose left half is empty is empty.  Active jobs are packed
// onto the lowest threads.
// ---------------------------------------------------------------------------
template <class Op>
PSS_INL void tree_up(typename Op::T *lds, int Tb, int nvalid)
{
    using T = typename Op::T;
    for (int d = 1; d < Tb; d <<= 1) {
        __syncthreads();
        const int jobs = Tb / (2 * d);
        const int j = threadIdx.x;
        if (j < jobs) {
            const int r = (j + 1) * 2 * d - 1, l = r - d;
            if (r - 2 * d + 1 < nvalid) {
                if (r - d + 1 < nvalid) {
                    // slot r <- slot l (x) slot r, operands read in place
                    Op::combine_v(Op::slot(lds, Tb, l), Op::slot(lds, Tb, r), Op::slot(lds, Tb, r));
                } else {
                    for (int c = 0; c < Op::NE; ++c)
                        lds[c * Tb + r] = lds[c * Tb + l];
                }
            }
        }
    }
    __syncthreads();
}

// Exclusive down-sweep: on return slot t (t < nvalid) holds, in its first NP
// components, the prefix preceding thread t's first element.
template <class Op>
PSS_INL void tree_down(typename Op::T *lds, int Tb, int nvalid, const typename Op::Pre &root)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        typename Op::Pre r0 = root;
        lds_put(r0, lds, Tb, Tb - 1);
    }
    for (int d = Tb / 2; d >= 1; d >>= 1) {
        __syncthreads();
        const int jobs = Tb / (2 * d);
        const int j = threadIdx.x;
        if (j < jobs) {
            const int r = (j + 1) * 2 * d - 1, l = r - d;
            if (r - 2 * d + 1 < nvalid) {
                typename Op::Pre P;
                lds_get(P, lds, Tb, r);
                if (r - d + 1 < nvalid) {
                    // the element in slot l is read before P overwrites it
                    typename Op::Pre Q;
                    Op::apply_v(P, Op::slot(lds, Tb, l), Q);
                    lds_put(Q, lds, Tb, r);
                }
                lds_put(P, lds, Tb, l);
            }
        }
    }
    __syncthreads();
}

// geometry of one scan level
struct LevelGeom {
    const int64_t *y_off;      // level 0: measurement offsets
    const int64_t *elem_off;   // level >= 1: this level's element offsets [B + 1]
    const int64_t *tile_off;   // this level's tile offsets [B + 1]
    int level;
    int extra; // level 0: elements per sequence = n_b + extra, element offset y_off[b] + extra*b
    int B;
    int E;
    int stage; // outputs staged in LDS and written by the whole block (needs
               // NP * T * E values of LDS)
};

PSS_INL void seq_range(const LevelGeom &g, int b, int64_t &off, int64_t &cnt)
{
    if (g.level == 0) {
        const int64_t a = g.y_off[b], z = g.y_off[b + 1];
        off = a + (int64_t)g.extra * b;
        cnt = z - a + g.extra;
    } else {
        off = g.elem_off[b];
        cnt = g.elem_off[b + 1] - off;
    }
}

struct TileInfo {
    int b;
    int64_t off, cnt, start;
    int tcnt, nvalid, E;
};

// Tile-interleaved position of the tile's element q (thread q / E, its j-th
// element, j = q % E): the j-th elements of all threads are contiguous, so a
// wave's j-th accesses touch consecutive words.  A bijection of [0, tcnt)
// also for a ragged last tile, whose last thread holds r <= E elements.
PSS_INL int ilv(int q, int tcnt, int E)
{
    const int nv = (tcnt + E - 1) / E, r = tcnt - (nv - 1) * E;
    const int t = q / E, j = q - t * E;
    return j < r ? j * nv + t : r * nv + (j - r) * (nv - 1) + t;
}

// inverse of ilv: the tile element stored at interleaved position r
PSS_INL int ilv_inv(int r, int tcnt, int E)
{
    const int nv = (tcnt + E - 1) / E, rr = tcnt - (nv - 1) * E;
    int t, j;
    if (r < rr * nv) {
        j = r / nv;
        t = r - j * nv;
    } else {
        const int r2 = r - rr * nv;
        j = rr + r2 / (nv - 1);
        t = r2 - (j - rr) * (nv - 1);
    }
    return t * E + j;
}

// slot of element p of the tile's sequence in storage private to the scan
PSS_INL int64_t ilv_slot(const TileInfo &ti, int64_t p)
{
    return ti.off + ti.start + ilv((int)(p - ti.start), ti.tcnt, ti.E);
}

PSS_INL TileInfo tile_info(const LevelGeom &g)
{
    TileInfo ti;
    const int64_t tile = blockIdx.x;
    ti.b = find_seq(g.tile_off, g.B, tile, 0);
    const int64_t tin = tile - g.tile_off[ti.b];
    seq_range(g, ti.b, ti.off, ti.cnt);
    const int64_t TS = (int64_t)blockDim.x * g.E;
    ti.start = tin * TS;
    const int64_t rem = ti.cnt - ti.start;
    ti.tcnt = (int)(rem < TS ? rem : TS);
    ti.nvalid = (ti.tcnt + g.E - 1) / g.E;
    ti.E = g.E;
    return ti;
}

// --- element sources --------------------------------------------------------
// plain SoA source (filter elements, or aggregates of a level below)
// A source either builds element p in registers (up / down) or, when
// lazy_up / lazy_down is set, hands out a view of it (uview / dview) that the
// operators read field by field.
// (ILV: the level's elements are stored tile-interleaved, see ilv.  LEAF_NZ
// > 0: finest-level filter elements, whose Z has only LEAF_NZ columns that
// can be non-zero; leaf_nz = 0 for everything else.)
template <class Op, class Ref, bool ILV = false, int LEAF_NZ = 0>
struct RefSrc {
    static constexpr bool lazy_up = true, lazy_down = true;
    static constexpr int leaf_nz = LEAF_NZ;
    Ref ref;
    PSS_INL int64_t slot(const TileInfo &ti, int64_t p) const
    {
        return ILV ? ilv_slot(ti, p) : ti.off + p;
    }
    PSS_INL auto uview(const TileInfo &ti, int64_t p) const { return view_of(ref, slot(ti, p)); }
    PSS_INL auto dview(const TileInfo &ti, int64_t p) const { return view_of(ref, slot(ti, p)); }
};

// smoother level 0: element of state k = n - p built from the transition
// linearisation of slot (b, k) and the filtering marginal at k (Table 4),
// stashed (tile-interleaved) during the up phase and re-read afterwards.
template <typename T, int NX, int NY, bool COV = false>
struct SmootherSrc {
    static constexpr bool lazy_up = false, lazy_down = true;
    static constexpr int leaf_nz = 0;
    GammaRef<T, NX, NY> gam;
    MargRef<T, NX> filt; // ld = T_x
    SElemRef<T, NX> stash; // ld = T_x
    const int64_t *y_off;
    PSS_INL void up(const TileInfo &ti, int64_t p, SElem<T, NX> &e) const
    {
        const int64_t n = ti.cnt - 1, k = n - p;
        Marg<T, NX> f;
        filt.load(ti.off + k, f);
        if (k == n) {
            smoother_element_last(f, e); // {0, m, N}: also {0, m, P} in covariance form
        } else {
            T F[NX][NX], c[NX], S[NX][NX];
            gam.load_trans(y_off[ti.b] + k, F, c, S);
            if constexpr (COV)
                smoother_element_cov(F, c, S, f, e);
            else
                smoother_element(F, c, S, f, e);
        }
        stash.store(ilv_slot(ti, p), e);
    }
    PSS_INL SRefV<T, NX> dview(const TileInfo &ti, int64_t p) const
    {
        return view_of(stash, ilv_slot(ti, p));
    }
};

// --- output sinks -------------------------------------------------------------
// put(ti, p, excl, incl) receives the exclusive and inclusive prefix of
// element p.  A sink with `stageable` also has first(ti, excl), called with
// the exclusive prefix of a sequence's first element, and store(ti, p, x):
// apply_phase may then collect a tile's prefixes in LDS (the exclusive ones
// when `stage_excl`, else the inclusive ones) and store them with
// consecutive lanes on consecutive elements.
// levels >= 1: exclusive prefix of each element
template <class Op, class Ref>
struct PreDst {
    static constexpr bool stageable = true, stage_excl = true;
    Ref ref;
    PSS_INL void first(const TileInfo &ti, const typename Op::Pre &excl) const {}
    PSS_INL void store(const TileInfo &ti, int64_t p, const typename Op::Pre &excl) const
    {
        ref.store(ti.off + p, excl);
    }
    PSS_INL void put(const TileInfo &ti, int64_t p, const typename Op::Pre &excl,
                     const typename Op::Pre &incl) const
    {
        ref.store(ti.off + p, excl);
    }
};

// filter level 0: inclusive prefix of step p+1 is the filtering marginal of
// state p+1; the first step also writes state 0 (its exclusive prefix, the
// prior)
template <typename T, int NX>
struct FiltDst {
    static constexpr bool stageable = true, stage_excl = false;
    MargRef<T, NX> out; // ld = T_x
    const int64_t *y_off;
    // deviation coordinates (nominal means, ld T_x): the start value is the
    // prior, whose mean is stored relative to r_0 like every later state's
    const T *dev_m = nullptr;
    PSS_INL void first(const TileInfo &ti, const Marg<T, NX> &excl) const
    {
        const int64_t s = y_off[ti.b] + ti.b;
        if (dev_m) {
            Marg<T, NX> x = excl;
#pragma unroll
            for (int i = 0; i < NX; ++i)
                x.m[i] -= dev_m[i * out.ld + s];
            out.store(s, x);
            return;
        }
        out.store(s, excl);
    }
    PSS_INL void store(const TileInfo &ti, int64_t p, const Marg<T, NX> &incl) const
    {
        out.store(y_off[ti.b] + ti.b + p + 1, incl);
    }
    PSS_INL void put(const TileInfo &ti, int64_t p, const Marg<T, NX> &excl,
                     const Marg<T, NX> &incl) const
    {
        if (p == 0)
            first(ti, excl);
        store(ti, p, incl);
    }
};

// smoother level 0: inclusive suffix of position p is the smoothing marginal
// of state n - p
template <typename T, int NX>
struct SmoothDst {
    static constexpr bool stageable = true, stage_excl = false;
    MargRef<T, NX> out;
    // deviation coordinates: the output mean is r_k plus the deviation,
    // r_k read from dev_m (ld = out.ld; may be out.m itself: each slot is
    // read and then written by one thread)
    const T *dev_m = nullptr;
    PSS_INL void first(const TileInfo &ti, const Marg<T, NX> &excl) const {}
    PSS_INL void store(const TileInfo &ti, int64_t p, const Marg<T, NX> &incl) const
    {
        const int64_t s = ti.off + (ti.cnt - 1 - p);
        if (dev_m) {
            Marg<T, NX> x = incl;
#pragma unroll
            for (int i = 0; i < NX; ++i)
                x.m[i] += dev_m[i * out.ld + s];
            out.store(s, x);
            return;
        }
        out.store(s, incl);
    }
    PSS_INL void put(const TileInfo &ti, int64_t p, const Marg<T, NX> &excl,
                     const Marg<T, NX> &incl) const
    {
        store(ti, p, incl);
    }
};

// sequence-start prefix: the prior for the filter, zero for the smoother (the
// first element in scan order has A = 0 / E = 0, so its value never matters)
template <typename T, int NX>
struct StartPre {
    const T *m0; // may be null: zeros
    const T *N0; // packed lower
    PSS_INL void get(Marg<T, NX> &p) const
    {
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            p.m[i] = m0 ? m0[i] : T(0);
#pragma unroll
            for (int j = 0; j <= i; ++j)
                p.N[i][j] = m0 ? N0[tri_idx(i, j)] : T(0);
        }
    }
};

// covariance form: the prior (m0, P0 = N0 N0^T)
template <typename T, int NX>
struct StartPreCov {
    const T *m0;
    const T *N0; // packed lower factor
    PSS_INL void get(Marg<T, NX> &p) const
    {
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            p.m[i] = m0[i];
#pragma unroll
            for (int j = 0; j <= i; ++j) {
                T s = T(0);
#pragma unroll
                for (int t = 0; t <= j; ++t)
                    s = pfma(N0[tri_idx(i, t)], N0[tri_idx(j, t)], s);
                p.N[i][j] = s;
            }
        }
    }
};

// ---------------------------------------------------------------------------
// scan kernels
// ---------------------------------------------------------------------------
template <class Op, class Src, class V>
PSS_INL void src_first(const Src &src, const TileInfo &ti, int64_t p, const V &acc)
{
    if constexpr (Src::lazy_up) {
        Op::copy_v(src.uview(ti, p), acc);
    } else {
        typename Op::Elem e;
        src.up(ti, p, e);
        Op::copy_v(Op::reg(e), acc);
    }
}

template <class Src, int NX>
constexpr int leaf_cols()
{
    return Src::leaf_nz > 0 ? Src::leaf_nz : NX;
}

template <class Op, class Src, class V>
PSS_INL void src_fold(const Src &src, const TileInfo &ti, int64_t p, const V &acc)
{
    constexpr int nz = leaf_cols<Src, Op::NX>();
    if constexpr (Src::lazy_up) {
        Op::template combine_v<nz>(acc, src.uview(ti, p), acc);
    } else {
        typename Op::Elem e;
        src.up(ti, p, e);
        Op::template combine_v<nz>(acc, Op::reg(e), acc);
    }
}

// A source with fused_down (the adjoint's finest level) applies element p to
// the prefix itself and may emit per-element results from both.
template <class S, class = void>
struct fused_down_of : std::false_type {};
template <class S>
struct fused_down_of<S, std::void_t<decltype(S::fused_down)>>
    : std::integral_constant<bool, S::fused_down> {};

template <class Op, class Src>
PSS_INL void src_apply(const Src &src, const TileInfo &ti, int64_t p, const typename Op::Pre &P,
                       typename Op::Pre &Q)
{
    constexpr int nz = leaf_cols<Src, Op::NX>();
    if constexpr (fused_down_of<Src>::value) {
        src.down_apply(ti, p, P, Q);
    } else if constexpr (Src::lazy_down) {
        Op::template apply_v<nz>(P, src.dview(ti, p), Q);
    } else {
        typename Op::Elem e;
        src.down(ti, p, e);
        Op::template apply_v<nz>(P, Op::reg(e), Q);
    }
}

// Thread t folds its elements left to right.  The accumulator stays in
// registers when the element is small (FP32); an FP64 filter element would
// not fit beside the operator's work space, so there the thread's LDS slot
// doubles as the accumulator.  Either way the fold ends in that slot.
template <class Op>
constexpr bool reg_accumulator()
{
    return sizeof(typename Op::T) * Op::NE <= 260;
}

template <class Op, class Src, bool RegAcc = reg_accumulator<Op>()>
PSS_INL void fold_phase(const LevelGeom &g, const TileInfo &ti, const Src &src,
                        typename Op::T *lds, int Tb)
{
    const int tid = threadIdx.x;
    if (tid < ti.nvalid) {
        const int64_t p0 = ti.start + (int64_t)tid * g.E;
        int64_t pe = p0 + g.E;
        if (pe > ti.start + ti.tcnt)
            pe = ti.start + ti.tcnt;
        if constexpr (RegAcc) {
            typename Op::Elem a;
            const auto acc = Op::reg(a);
            src_first<Op>(src, ti, p0, acc);
            for (int64_t p = p0 + 1; p < pe; ++p)
                src_fold<Op>(src, ti, p, acc);
            lds_put(a, lds, Tb, tid);
        } else {
            const auto acc = Op::slot(lds, Tb, tid);
            src_first<Op>(src, ti, p0, acc);
            for (int64_t p = p0 + 1; p < pe; ++p)
                src_fold<Op>(src, ti, p, acc);
        }
    }
}

// Thread t walks its elements again from its exclusive prefix (left in its
// LDS slot by the down-sweep).  With g.stage (stageable sinks only) the
// inclusive prefixes are first collected in LDS, component-major over the
// tile's elements, and then stored by the whole block, consecutive lanes on
// consecutive elements; the block must call this uniformly.
template <class Op, class Src, class Dst>
PSS_INL void apply_phase(const LevelGeom &g, const TileInfo &ti, const Src &src, const Dst &dst,
                         typename Op::T *lds, int Tb)
{
    const int tid = threadIdx.x;
    const bool act = tid < ti.nvalid;
    const int64_t p0 = ti.start + (int64_t)tid * g.E;
    int64_t pe = p0 + g.E;
    if (pe > ti.start + ti.tcnt)
        pe = ti.start + ti.tcnt;
    typename Op::Pre P;
    if (act)
        lds_get(P, lds, Tb, tid);
    if constexpr (Dst::stageable) {
        if (g.stage) {
            const int ld = Tb * g.E;
            __syncthreads(); // every prefix is in registers: LDS is free
            if (act) {
                for (int64_t p = p0; p < pe; ++p) {
                    typename Op::Pre Q;
                    src_apply<Op>(src, ti, p, P, Q);
                    if (p == 0)
                        dst.first(ti, P);
                    if constexpr (Dst::stage_excl)
                        lds_put(P, lds, ld, (int)(p - ti.start));
                    else
                        lds_put(Q, lds, ld, (int)(p - ti.start));
                    P = Q;
                }
            }
            __syncthreads();
            for (int q = tid; q < ti.tcnt; q += Tb) {
                typename Op::Pre x;
                lds_get(x, lds, ld, q);
                dst.store(ti, ti.start + q, x);
            }
            return;
        }
    }
    if (act) {
        for (int64_t p = p0; p < pe; ++p) {
            typename Op::Pre Q;
            src_apply<Op>(src, ti, p, P, Q);
            dst.put(ti, p, P, Q);
            P = Q;
        }
    }
}

// lower levels, first half: fold + up-sweep; saves the LDS tree and the
// tile aggregate (an element of the next level)
template <class Op, class Src, class AggRef>
__global__ __launch_bounds__(256) void k_scan_up(LevelGeom g, Src src, AggRef agg,
                                                 typename Op::T *tree, int64_t tree_ld)
{
    using T = typename Op::T;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);
    const int Tb = blockDim.x;
    const TileInfo ti = tile_info(g);
    fold_phase<Op>(g, ti, src, lds, Tb);
    tree_up<Op>(lds, Tb, ti.nvalid);
    const int64_t base = (int64_t)blockIdx.x * Tb + threadIdx.x;
    for (int c = 0; c < Op::NE; ++c)
        tree[c * tree_ld + base] = lds[c * Tb + threadIdx.x];
    if (threadIdx.x == 0)
        Op::copy_v(Op::slot(lds, Tb, Tb - 1), view_of(agg, (int64_t)blockIdx.x));
}

// lower levels, second half: restore the tree, down-sweep from the tile's
// exclusive prefix (written by the level above), apply, emit
template <class Op, class Src, class Dst, class PreRef>
__global__ __launch_bounds__(256) void k_scan_down(LevelGeom g, Src src, Dst dst,
                                                   const typename Op::T *tree, int64_t tree_ld,
                                                   PreRef pre_in)
{
    using T = typename Op::T;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);
    const int Tb = blockDim.x;
    const TileInfo ti = tile_info(g);
    const int64_t base = (int64_t)blockIdx.x * Tb + threadIdx.x;
    for (int c = 0; c < Op::NE; ++c)
        lds[c * Tb + threadIdx.x] = tree[c * tree_ld + base];
    typename Op::Pre root;
    pre_in.load(blockIdx.x, root);
    tree_down<Op>(lds, Tb, ti.nvalid, root);
    apply_phase<Op>(g, ti, src, dst, lds, Tb);
}

// flat level, first half: every thread's fold is element v of the next
// level (v = the thread's rank in its sequence), stored tile-interleaved for
// that level's tiles of nT threads x nE elements; no tree
template <class Op, class Src, class AggRef>
__global__ __launch_bounds__(256) void k_scan_up_flat(LevelGeom g, Src src, AggRef agg,
                                                      const int64_t *next_off, int nT, int nE)
{
    using T = typename Op::T;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);
    const int Tb = blockDim.x;
    const TileInfo ti = tile_info(g);
    fold_phase<Op>(g, ti, src, lds, Tb);
    if (threadIdx.x < ti.nvalid) {
        const int64_t v = ti.start / g.E + threadIdx.x;
        const int64_t off = next_off[ti.b], cnt = next_off[ti.b + 1] - off;
        const int64_t TS = (int64_t)nT * nE, start = (v / TS) * TS;
        const int tcnt = (int)((cnt - start) < TS ? (cnt - start) : TS);
        const int64_t slot = off + start + ilv((int)(v - start), tcnt, nE);
        Op::copy_v(Op::slot(lds, Tb, threadIdx.x), view_of(agg, slot));
    }
}

// flat level, second half: each thread takes its exclusive prefix from the
// level above, then applies and emits as a tree level does
template <class Op, class Src, class Dst, class PreRef>
__global__ __launch_bounds__(256) void k_scan_down_flat(LevelGeom g, Src src, Dst dst,
                                                        const int64_t *next_off, PreRef pre_in)
{
    using T = typename Op::T;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);
    const int Tb = blockDim.x;
    const TileInfo ti = tile_info(g);
    if (threadIdx.x < ti.nvalid) {
        typename Op::Pre P;
        pre_in.load(next_off[ti.b] + ti.start / g.E + threadIdx.x, P);
        lds_put(P, lds, Tb, threadIdx.x);
    }
    apply_phase<Op>(g, ti, src, dst, lds, Tb);
}

// top level (one tile per sequence): everything in one kernel
template <class Op, class Src, class Dst, class Start>
__global__ __launch_bounds__(256) void k_scan_top(LevelGeom g, Src src, Dst dst, Start start)
{
    using T = typename Op::T;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);
    const int Tb = blockDim.x;
    const TileInfo ti = tile_info(g);
    fold_phase<Op>(g, ti, src, lds, Tb);
    tree_up<Op>(lds, Tb, ti.nvalid);
    typename Op::Pre root;
    start.get(root);
    tree_down<Op>(lds, Tb, ti.nvalid, root);
    apply_phase<Op>(g, ti, src, dst, lds, Tb);
}

// tile offsets of every level, one thread per sequence + a block scan
struct PlanArgs {
    const int64_t *y_off;
    int B;
    int extra;
    int L;
    int64_t TS[kMaxLevels]; // tile size of level l
    int64_t D[kMaxLevels];  // elements of level l per element of level l + 1
    int64_t *tile_off[kMaxLevels];
    int64_t *elem_off[kMaxLevels]; // may be null
};

__global__ __launch_bounds__(1024) void k_plan(PlanArgs a);

// ---------------------------------------------------------------------------
// element-wise kernels
// ---------------------------------------------------------------------------
template <typename T, int NX, int NY, bool COV = false>
__global__ __launch_bounds__(256) void k_filter_elements(const int64_t *y_off, int B, int64_t T_y,
                                                         GammaRef<T, NX, NY> gam, const T *y,
                                                         const T *m0, const T *N0,
                                                         FElemRef<T, NX> out, int ilv_T,
                                                         int ilv_E, const T *dev_m, int64_t T_x)
{
    // thread i fills stored slot i; with ilv_E > 0 the elements are stored
    // tile-interleaved for a level-0 filter scan of ilv_T threads x ilv_E
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= T_y)
        return;
    const int b = find_seq(y_off, B, i, 0);
    int64_t k = i - y_off[b];
    if (ilv_E > 0) {
        const int64_t TS = (int64_t)ilv_T * ilv_E, cnt = y_off[b + 1] - y_off[b];
        const int64_t start = (k / TS) * TS;
        const int tcnt = (int)((cnt - start) < TS ? (cnt - start) : TS);
        k = start + ilv_inv((int)(k - start), tcnt, ilv_E);
    }
    const int64_t t = y_off[b] + k; // logical step slot
    T F[NX][NX], c[NX], SL[NX][NX], H[NY][NX], d[NY], SO[NY][NY], yy[NY];
    gam.load_trans(t, F, c, SL);
    gam.load_obs(t, H, d, SO);
#pragma unroll
    for (int a = 0; a < NY; ++a)
        yy[a] = y[a * T_y + t];
    FElem<T, NX> e;
    if (k == 0) {
        T m[NX], N[NX][NX];
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            // deviation coordinates: the prior mean relative to r_0
            m[i] = dev_m ? m0[i] - dev_m[i * T_x + y_off[b] + b] : m0[i];
#pragma unroll
            for (int j = 0; j <= i; ++j)
                N[i][j] = N0[tri_idx(i, j)];
        }
        if constexpr (COV)
            filter_element_first_cov(m, N, F, c, SL, H, d, SO, yy, e);
        else
            filter_element_first(m, N, F, c, SL, H, d, SO, yy, e);
    } else {
        if constexpr (COV)
            filter_element_cov(F, c, SL, H, d, SO, yy, e);
        else
            filter_element(F, c, SL, H, d, SO, yy, e);
    }
    out.store(i, e);
}

// pseudo-log-likelihood terms (Section 5.1) from the filtering marginal of the
// previous state: ell[t] = log N(y; H m^- + d, Y Y^T)
template <typename T, int NX, int NY>
__global__ __launch_bounds__(128) void k_loglik_terms(const int64_t *y_off, int B, int64_t T_y,
                                                      int64_t T_x, GammaRef<T, NX, NY> gam,
                                                      const T *y, MargRef<T, NX> filt,
                                                      double *ell)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T_y)
        return;
    const int b = find_seq(y_off, B, t, 0);
    T F[NX][NX], c[NX], SL[NX][NX], H[NY][NX], d[NY], SO[NY][NY];
    gam.load_trans(t, F, c, SL);
    gam.load_obs(t, H, d, SO);
    Marg<T, NX> f;
    filt.load(t + b, f);
    T mp[NX], FN[NX][NX], Np[NX][NX];
    mv(F, f.m, mp);
#pragma unroll
    for (int i = 0; i < NX; ++i)
        mp[i] += c[i];
    mm_lower(F, f.N, FN);
    tria_dense_lower(FN, SL, Np);
    T HN[NY][NX];
    mm_lower(H, Np, HN);
    T M[NY][NX + NY];
#pragma unroll
    for (int a = 0; a < NY; ++a) {
#pragma unroll
        for (int j = 0; j < NX; ++j)
            M[a][j] = HN[a][j];
#pragma unroll
        for (int j = 0; j < NY; ++j)
            M[a][NX + j] = (j <= a) ? SO[a][j] : T(0);
    }
    lq_rows<NY, NX>(M);
    T Y[NY][NY], v[NY], Hm[NY], u[NY];
#pragma unroll
    for (int a = 0; a < NY; ++a)
#pragma unroll
        for (int j = 0; j <= a; ++j)
            Y[a][j] = M[a][j];
    mv(H, mp, Hm);
#pragma unroll
    for (int a = 0; a < NY; ++a)
        v[a] = y[a * T_y + t] - Hm[a] - d[a];
    lsolve_lower(Y, v, u);
    double l = -0.5 * NY * 1.8378770664093454835606594728112; // log(2 pi)
#pragma unroll
    for (int a = 0; a < NY; ++a)
        l -= (double)plog(Y[a][a]) + 0.5 * (double)u[a] * (double)u[a];
    ell[t] = l;
}

// Deterministic per-sequence sums in two stages.  Stage 1: one block per
// chunk of kSumChunk consecutive step slots of ONE sequence (chunk offsets
// from the tile plan with tile size kSumChunk); fixed thread strides, then a
// fixed LDS tree.  Stage 2: one block per sequence adds its chunk partials in
// order.  The bracketing depends only on the sequence lengths.
constexpr int kSumChunk = 8192;

template <int NC>
__global__ __launch_bounds__(256) void k_chunk_sum(const int64_t *y_off, const int64_t *chunk_off,
                                                   int B, const double *terms, int64_t ld,
                                                   double *partial, int64_t nchunks)
{
    __shared__ double red[NC][256];
    const int64_t ch = blockIdx.x;
    const int b = find_seq(chunk_off, B, ch, 0);
    const int64_t a = y_off[b] + (ch - chunk_off[b]) * kSumChunk;
    int64_t z = a + kSumChunk;
    if (z > y_off[b + 1])
        z = y_off[b + 1];
    double s[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c)
        s[c] = 0.0;
#pragma unroll 8
    for (int64_t t = a + threadIdx.x; t < z; t += blockDim.x)
#pragma unroll
        for (int c = 0; c < NC; ++c)
            s[c] += terms[c * ld + t];
#pragma unroll
    for (int c = 0; c < NC; ++c)
        red[c][threadIdx.x] = s[c];
    for (int w = blockDim.x / 2; w >= 1; w >>= 1) {
        __syncthreads();
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int c = 0; c < NC; ++c)
                red[c][threadIdx.x] += red[c][threadIdx.x + w];
    }
    if (threadIdx.x == 0)
#pragma unroll
        for (int c = 0; c < NC; ++c)
            partial[c * nchunks + ch] = red[c][0];
}

template <int NC>
__global__ __launch_bounds__(64) void k_seq_total(const int64_t *chunk_off, const double *partial,
                                                  int64_t nchunks, int B, double *out)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B)
        return;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double s = 0.0;
        for (int64_t k = chunk_off[b]; k < chunk_off[b + 1]; ++k)
            s += partial[c * nchunks + k];
        out[(int64_t)c * B + b] = s;
    }
}

// theta_bar[c] = sum_b w[b] grad[c][b] in a fixed order (one block)
__global__ __launch_bounds__(256) void k_weighted_grad(const double *grad, const double *w, int B,
                                                       double *theta_bar);

// Sequential square-root comparator, one wavefront per sequence: the filter
// recursion forward (eqs. sqrt-filter-step1/2: predict with
// Tria([F N, S_Lambda]), update with Psi = Tria([[H N^-, S_Omega], [N^-, 0]]);
// m^f, N^f stored) and the RTS recursion back through the Table 4 element
// (Phi = Tria([[F N^f, S_Lambda], [N^f, 0]]), E = Phi21 Phi11^{-1}, then
// N^s = Tria([E N^s_{k+1}, D])).  Every Tria runs over the wave with its rows
// on lanes (pss::wave): lane NX + r holds row r of the state (m[r] and row r
// of N), lanes 0..NX-1 the upper rows of Phi, lanes 2NX.. the measurement
// rows of Psi.  The steps are serial; the wave spreads each step's rows.
// Used for nx >= 2 (a scalar state runs k_sequential_1t below).
template <typename T, int NX, int NY>
__global__ __launch_bounds__(64) void k_sequential(const int64_t *y_off, int B, int64_t T_y,
                                                   GammaRef<T, NX, NY> gam, const T *y,
                                                   const T *m0, const T *N0,
                                                   MargRef<T, NX> filt, MargRef<T, NX> smooth)
{
    static_assert(2 * NX + NY <= 64, "k_sequential: 2 nx + ny rows must fit one wave");
    using St = wave::Contig<NX>;                 // state rows
    using Ps = wave::Split<NY, 2 * NX, NX>;      // Psi: measurement rows, then state rows
    using Ph = wave::Contig<0>;                  // Phi: upper rows on 0..NX-1, lower on the state lanes
    const int b = blockIdx.x;
    if (b >= B)
        return;
    const int lane = threadIdx.x;
    const int r = lane - NX, oa = lane - 2 * NX;
    const bool st = r >= 0 && r < NX, ob = oa >= 0 && oa < NY, up = lane < NX;
    const int rs = st ? r : 0, os = ob ? oa : 0, us = up ? lane : 0; // clamped rows for loads
    const int64_t a = y_off[b], n = y_off[b + 1] - a, x0 = a + b;
    const int64_t ld = gam.ld, gs = gam.stride;
    // this lane's state row: m[r], N[r][0..r] (zeros right of the diagonal)
    T m_r, Nr[NX];
    auto tri = [](int i, int j) { return i * (i + 1) / 2 + (j < i ? j : i); };
    auto store_state = [&](const MargRef<T, NX> &M, int64_t t) {
        if (st) {
            M.m[r * M.ld + t] = m_r;
#pragma unroll
            for (int j = 0; j < NX; ++j)
                if (j <= r)
                    M.N[tri(r, j) * M.ld + t] = Nr[j];
        }
    };
    m_r = m0[rs];
#pragma unroll
    for (int j = 0; j < NX; ++j)
        Nr[j] = (j <= rs) ? N0[tri(rs, j)] : T(0);
    store_state(filt, x0);
    for (int64_t k = 0; k < n; ++k) {
        const int64_t u = (a + k) * gs;
        T mb[NX], Nb[NX][NX];
        wave::bcast_vec<St>(m_r, mb);
        wave::bcast_lower<St, NX>(Nr, Nb);
        // predict on the state lanes: mp[r] = F[r] m + c[r]; row r of [F N, S_Lambda]
        T Fr[NX], row[2 * NX];
#pragma unroll
        for (int j = 0; j < NX; ++j)
            Fr[j] = gam.F[(rs * NX + j) * ld + u];
        T mp_r = Fr[0] * mb[0];
#pragma unroll
        for (int j = 1; j < NX; ++j)
            mp_r = pfma(Fr[j], mb[j], mp_r);
        mp_r += gam.c[rs * ld + u];
#pragma unroll
        for (int j = 0; j < NX; ++j) {
            T s = Fr[j] * Nb[j][j];
#pragma unroll
            for (int t = j + 1; t < NX; ++t)
                s = pfma(Fr[t], Nb[t][j], s);
            row[j] = s;
            row[NX + j] = (j <= rs) ? gam.SL[tri(rs, j) * ld + u] : T(0);
        }
        wave::lq_rows<NX, NX, St>(row, st ? r : -1);
        // Psi: measurement rows [H N^-, S_Omega] on lanes 2NX.., state rows [N^-, 0]
        T Pb[NX][NX], mpb[NX];
        wave::bcast_lower<St, NX>(row, Pb);
        wave::bcast_vec<St>(mp_r, mpb);
        T Ho[NX];
#pragma unroll
        for (int j = 0; j < NX; ++j)
            Ho[j] = gam.H[(os * NX + j) * ld + u];
        T psi[NX + NY];
#pragma unroll
        for (int j = 0; j < NX; ++j) {
            T s = Ho[j] * Pb[j][j];
#pragma unroll
            for (int t = j + 1; t < NX; ++t)
                s = pfma(Ho[t], Pb[t][j], s);
            psi[j] = ob ? s : ((st && j <= r) ? row[j] : T(0));
        }
#pragma unroll
        for (int j = 0; j < NY; ++j)
            psi[NX + j] = (ob && j <= oa) ? gam.SO[tri(os, j) * ld + u] : T(0);
        wave::lq_rows<NY + NX, NX, Ps>(psi, ob ? oa : (st ? NY + r : -1));
        // innovation v = y - H mp - d on the measurement lanes; u = Psi11^{-1} v
        T Hm = Ho[0] * mpb[0];
#pragma unroll
        for (int j = 1; j < NX; ++j)
            Hm = pfma(Ho[j], mpb[j], Hm);
        const T v_o = y[os * T_y + a + k] - Hm - gam.d[os * ld + u];
        T vb[NY], P11[NY][NY], ub[NY];
        wave::bcast_vec<wave::Contig<2 * NX>>(v_o, vb);
        wave::bcast_lower<wave::Contig<2 * NX>, NY>(psi, P11);
        lsolve_lower(P11, vb, ub);
        // update on the state lanes: m = mp + Psi21 u, N = Psi22
        T Ku = psi[0] * ub[0];
#pragma unroll
        for (int q = 1; q < NY; ++q)
            Ku = pfma(psi[q], ub[q], Ku);
        m_r = mp_r + Ku;
#pragma unroll
        for (int j = 0; j < NX; ++j)
            Nr[j] = (j <= rs) ? psi[NY + j] : T(0);
        store_state(filt, x0 + k + 1);
    }
    store_state(smooth, x0 + n);
    // the filtered marginals are read back by other lanes of this wave
    __threadfence_block();
    for (int64_t k = n - 1; k >= 0; --k) {
        const int64_t u = (a + k) * gs, xk = x0 + k;
        // Phi rows: upper (lanes 0..NX-1) [F N^f, S_Lambda], lower (state lanes) [N^f, 0]
        T fm[NX], fN[NX][NX];
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            fm[i] = filt.m[i * filt.ld + xk];
#pragma unroll
            for (int j = 0; j <= i; ++j)
                fN[i][j] = filt.N[tri_idx(i, j) * filt.ld + xk];
        }
        T Fu[NX], ph[2 * NX];
#pragma unroll
        for (int j = 0; j < NX; ++j)
            Fu[j] = gam.F[(us * NX + j) * ld + u];
#pragma unroll
        for (int j = 0; j < NX; ++j) {
            T s = Fu[j] * fN[j][j];
#pragma unroll
            for (int t = j + 1; t < NX; ++t)
                s = pfma(Fu[t], fN[t][j], s);
            ph[j] = up ? s : ((st && j <= r) ? filt.N[tri(rs, j) * filt.ld + xk] : T(0));
            ph[NX + j] = (up && j <= lane) ? gam.SL[tri(us, j) * ld + u] : T(0);
        }
        wave::lq_rows<2 * NX, NX, Ph>(ph, (up || st) ? lane : -1);
        // E row r = Phi21[r] Phi11^{-1} on the state lanes
        T P11[NX][NX], inv[NX], E[NX];
        wave::bcast_lower<Ph, NX>(ph, P11);
#pragma unroll
        for (int j = 0; j < NX; ++j)
            inv[j] = prcp(P11[j][j]);
#pragma unroll
        for (int j = NX - 1; j >= 0; --j) {
            T s = ph[j];
#pragma unroll
            for (int t = j + 1; t < NX; ++t)
                s = pfma(-E[t], P11[t][j], s);
            E[j] = s * inv[j];
        }
        // g = m^f - E (F m^f + c): F m^f + c on the upper lanes
        T Fm_u = Fu[0] * fm[0];
#pragma unroll
        for (int j = 1; j < NX; ++j)
            Fm_u = pfma(Fu[j], fm[j], Fm_u);
        Fm_u += gam.c[us * ld + u];
        T Fmb[NX];
        wave::bcast_vec<Ph>(Fm_u, Fmb);
        T Eg = E[0] * Fmb[0];
#pragma unroll
        for (int j = 1; j < NX; ++j)
            Eg = pfma(E[j], Fmb[j], Eg);
        const T g_r = filt.m[rs * filt.ld + xk] - Eg;
        // apply to the smoothed marginal of step k+1: m = E m^s + g,
        // N = Tria([E N^s, D]) with D = Phi22
        T sb[NX], sN[NX][NX], ap[2 * NX];
        wave::bcast_vec<St>(m_r, sb);
        wave::bcast_lower<St, NX>(Nr, sN);
#pragma unroll
        for (int j = 0; j < NX; ++j) {
            T s = E[j] * sN[j][j];
#pragma unroll
            for (int t = j + 1; t < NX; ++t)
                s = pfma(E[t], sN[t][j], s);
            ap[j] = s;
            ap[NX + j] = (j <= rs) ? ph[NX + j] : T(0);
        }
        wave::lq_rows<NX, NX, St>(ap, st ? r : -1);
        T Es = E[0] * sb[0];
#pragma unroll
        for (int j = 1; j < NX; ++j)
            Es = pfma(E[j], sb[j], Es);
        m_r = Es + g_r;
#pragma unroll
        for (int j = 0; j < NX; ++j)
            Nr[j] = (j <= rs) ? ap[j] : T(0);
        store_state(smooth, xk);
    }
}

// The same comparator with one thread per sequence, for a scalar state
// (nx = 1): its Trias have one row, nothing to spread over lanes, and the
// wave form's broadcasts only add latency there.
template <typename T, int NX, int NY>
__global__ __launch_bounds__(64) void k_sequential_1t(const int64_t *y_off, int B, int64_t T_y,
                                                   GammaRef<T, NX, NY> gam, const T *y,
                                                   const T *m0, const T *N0,
                                                   MargRef<T, NX> filt, MargRef<T, NX> smooth)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B)
        return;
    const int64_t a = y_off[b], n = y_off[b + 1] - a, x0 = a + b;
    Marg<T, NX> f;
#pragma unroll
    for (int i = 0; i < NX; ++i) {
        f.m[i] = m0[i];
#pragma unroll
        for (int j = 0; j <= i; ++j)
            f.N[i][j] = N0[tri_idx(i, j)];
    }
    filt.store(x0, f);
    for (int64_t k = 0; k < n; ++k) {
        T F[NX][NX], c[NX], SL[NX][NX], H[NY][NX], d[NY], SO[NY][NY];
        gam.load_trans(a + k, F, c, SL);
        gam.load_obs(a + k, H, d, SO);
        T mp[NX], FN[NX][NX], Np[NX][NX];
        mv(F, f.m, mp);
#pragma unroll
        for (int i = 0; i < NX; ++i)
            mp[i] += c[i];
        mm_lower(F, f.N, FN);
        tria_dense_lower(FN, SL, Np);
        T P11[NY][NY], P21[NX][NY];
        psi_blocks(H, Np, SO, P11, P21, f.N);
        T Hm[NY], v[NY], u[NY], Ku[NX];
        mv(H, mp, Hm);
#pragma unroll
        for (int q = 0; q < NY; ++q)
            v[q] = y[q * T_y + a + k] - Hm[q] - d[q];
        lsolve_lower(P11, v, u);
        mv(P21, u, Ku);
#pragma unroll
        for (int i = 0; i < NX; ++i)
            f.m[i] = mp[i] + Ku[i];
        filt.store(x0 + k + 1, f);
    }
    Marg<T, NX> s = f;
    smooth.store(x0 + n, s);
    for (int64_t k = n - 1; k >= 0; --k) {
        T F[NX][NX], c[NX], SL[NX][NX];
        gam.load_trans(a + k, F, c, SL);
        Marg<T, NX> fk, o;
        filt.load(x0 + k, fk);
        SElem<T, NX> e;
        smoother_element(F, c, SL, fk, e);
        smoother_apply(e, s, o);
        s = o;
        smooth.store(x0 + k, s);
    }
}

// sequential covariance-form comparator (the standard Kalman filter and RTS
// smoother, one thread per sequence): predict mp = F m + c,
// Pp = F P F^T + Lambda; update with S = H Pp H^T + Omega = Y Y^T,
// K = Pp H^T S^{-1}, m = mp + K (y - H mp - d), P = Pp - K H Pp (symmetrised);
// the backward pass applies the smoother element of Table 4 (standard
// column), which is the RTS step.  Marginals hold (m, packed P).
template <typename T, int NX, int NY>
__global__ __launch_bounds__(64) void k_sequential_cov(const int64_t *y_off, int B, int64_t T_y,
                                                       GammaRef<T, NX, NY> gam, const T *y,
                                                       const T *m0, const T *N0,
                                                       MargRef<T, NX> filt, MargRef<T, NX> smooth)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B)
        return;
    const int64_t a = y_off[b], n = y_off[b + 1] - a, x0 = a + b;
    T m[NX], P[NX][NX];
    {
        T L0[NX][NX];
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            m[i] = m0[i];
#pragma unroll
            for (int j = 0; j < NX; ++j)
                L0[i][j] = j <= i ? N0[tri_idx(i, j)] : T(0);
        }
        gram_full(L0, P);
    }
    Marg<T, NX> f;
#pragma unroll
    for (int i = 0; i < NX; ++i) {
        f.m[i] = m[i];
#pragma unroll
        for (int j = 0; j <= i; ++j)
            f.N[i][j] = P[i][j];
    }
    filt.store(x0, f);
    for (int64_t k = 0; k < n; ++k) {
        T F[NX][NX], c[NX], SL[NX][NX], H[NY][NX], d[NY], SO[NY][NY];
        gam.load_trans(a + k, F, c, SL);
        gam.load_obs(a + k, H, d, SO);
        T mp[NX], FP[NX][NX], Pp[NX][NX];
        mv(F, m, mp);
#pragma unroll
        for (int i = 0; i < NX; ++i)
            mp[i] += c[i];
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
        T HP[NY][NX], S[NY][NY], Y[NY][NY], PHt[NX][NY], K[NX][NY];
        mm(H, Pp, HP);
        gram_full(SO, S);
#pragma unroll
        for (int q = 0; q < NY; ++q)
#pragma unroll
            for (int r = 0; r < NY; ++r) {
                T s = S[q][r];
#pragma unroll
                for (int t = 0; t < NX; ++t)
                    s = pfma(HP[q][t], H[r][t], s);
                S[q][r] = s;
            }
        chol_lower(S, Y);
#pragma unroll
        for (int i = 0; i < NX; ++i)
#pragma unroll
            for (int q = 0; q < NY; ++q)
                PHt[i][q] = HP[q][i];
        rsolve_spd(PHt, Y, K);
        T Hm[NY], v[NY];
        mv(H, mp, Hm);
#pragma unroll
        for (int q = 0; q < NY; ++q)
            v[q] = y[q * T_y + a + k] - Hm[q] - d[q];
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            T s = mp[i];
#pragma unroll
            for (int q = 0; q < NY; ++q)
                s = pfma(K[i][q], v[q], s);
            m[i] = s;
        }
#pragma unroll
        for (int i = 0; i < NX; ++i)
#pragma unroll
            for (int j = 0; j <= i; ++j) {
                T s = Pp[i][j], t = Pp[i][j];
#pragma unroll
                for (int q = 0; q < NY; ++q) {
                    s = pfma(-K[i][q], HP[q][j], s);
                    t = pfma(-K[j][q], HP[q][i], t);
                }
                P[i][j] = P[j][i] = T(0.5) * (s + t);
            }
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            f.m[i] = m[i];
#pragma unroll
            for (int j = 0; j <= i; ++j)
                f.N[i][j] = P[i][j];
        }
        filt.store(x0 + k + 1, f);
    }
    Marg<T, NX> s = f;
    smooth.store(x0 + n, s);
    for (int64_t k = n - 1; k >= 0; --k) {
        T F[NX][NX], c[NX], SL[NX][NX];
        gam.load_trans(a + k, F, c, SL);
        Marg<T, NX> fk, o;
        filt.load(x0 + k, fk);
        SElem<T, NX> e;
        smoother_element_cov(F, c, SL, fk, e);
        smoother_apply_cov_v<T, NX>(SRegV<T, NX>{&e}, s, o);
        s = o;
        smooth.store(x0 + k, s);
    }
}

// ---------------------------------------------------------------------------
// coordinated-turn model kernels
// ---------------------------------------------------------------------------
// one thread per state: transition SLR from state k (slot k, k < n) and
// measurement SLR from state k (slot k-1, k >= 1)
// Offsets in deviation coordinates relative to the nominal means (the CT
// model's IPLS pass): with r_k the nominal mean of state k, step k's
// transition x~_{k+1} = F x~_k + (F r_k + c - r_{k+1}) + noise and its
// measurement y = H x~_{k+1} + (d + H r_{k+1}) + noise.  The means the
// scans then carry are deviations, small next to positions of order 100,
// whose information vectors eta ~ J m lose far fewer digits in FP32.  The
// offsets are summed in BranchPrec (FP64 for FP32 kernels).
template <typename T, int NX>
PSS_INL void dev_trans_offset(const T (&F)[NX][NX], const T (&rk)[NX], const T (&rk1)[NX],
                              T (&c)[NX])
{
    using W = typename BranchPrec<T>::type;
#pragma unroll
    for (int i = 0; i < NX; ++i) {
        W v = W(c[i]) - W(rk1[i]);
#pragma unroll
        for (int j = 0; j < NX; ++j)
            v = pfma(W(F[i][j]), W(rk[j]), v);
        c[i] = T(v);
    }
}
template <typename T, int NX, int NY>
PSS_INL void dev_obs_offset(const T (&H)[NY][NX], const T (&r)[NX], T (&d)[NY])
{
    using W = typename BranchPrec<T>::type;
#pragma unroll
    for (int a = 0; a < NY; ++a) {
        W v = W(d[a]);
#pragma unroll
        for (int j = 0; j < NX; ++j)
            v = pfma(W(H[a][j]), W(r[j]), v);
        d[a] = T(v);
    }
}

// (TAYLOR_ONLY: an instance that holds the Taylor linearisation alone; the
// runtime flag then has to be set)
template <typename T, bool TAYLOR_ONLY = false>
__global__ __launch_bounds__(128) void k_slr_ct(const int64_t *y_off, int B, int64_t T_x,
                                                int64_t T_y, CTParams<T> P, MargRef<T, 5> nom,
                                                const T *y, GammaRef<T, 5, 2> out, int taylor,
                                                int nominal_cov, int dev)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= T_x)
        return;
    const int b = find_seq(y_off, B, s, 1);
    const int64_t x0 = y_off[b] + b, k = s - x0, n = y_off[b + 1] - y_off[b];
    Marg<T, 5> mg;
    nom.load(s, mg);
    if (nominal_cov && !taylor) {
        // covariance form: the nominal holds P; the sigma points need a factor
        T P[5][5], L[5][5];
        sym_full(P, [&](int i, int j) { return mg.N[i][j]; });
        chol_lower(P, L);
#pragma unroll
        for (int i = 0; i < 5; ++i)
#pragma unroll
            for (int j = 0; j <= i; ++j)
                mg.N[i][j] = L[i][j];
    }
    if (k < n) {
        T G[5][5], off[5], S[5][5];
        if constexpr (TAYLOR_ONLY)
            ct_taylor_transition(P, mg, G, off, S);
        else if (taylor)
            ct_taylor_transition(P, mg, G, off, S);
        else
            ct_slr_transition(P, mg, G, off, S);
        if (dev) {
            T r1[5];
#pragma unroll
            for (int i = 0; i < 5; ++i)
                r1[i] = nom.m[i * nom.ld + s + 1];
            dev_trans_offset(G, mg.m, r1, off);
        }
        out.store_trans(y_off[b] + k, G, off, S);
    }
    if (k >= 1) {
        const int64_t t = y_off[b] + k - 1;
        T yy[2] = {y[t], y[T_y + t]};
        T G[2][5], off[2], S[2][2];
        if constexpr (TAYLOR_ONLY)
            ct_taylor_bearings(P, mg, yy, G, off, S);
        else if (taylor)
            ct_taylor_bearings(P, mg, yy, G, off, S);
        else
            ct_slr_bearings(P, mg, yy, G, off, S);
        if (dev)
            dev_obs_offset(G, mg.m, off);
        out.store_obs(t, G, off, S);
    }
}

// The CT model with cubature (or Taylor, taylor != 0) linearisation fused
// with the filter elements: one thread per stored element slot i (stored
// tile-interleaved as k_filter_elements does) linearises its step slot t --
// the transition at state k and the bearings at state k + 1, as k_slr_ct --
// and builds the element of that step from the result in registers.  The
// transition part is stored for the smoother; the measurement part only
// with store_obs.
template <typename T, bool COV>
__global__ __launch_bounds__(256) void k_slr_felem_ct(const int64_t *y_off, int B, int64_t T_y,
                                                      CTParams<T> P, MargRef<T, 5> nom,
                                                      const T *y, const T *m0, const T *N0,
                                                      GammaRef<T, 5, 2> gam, int store_obs,
                                                      FElemRef<T, 5> out, int ilv_T, int ilv_E,
                                                      int taylor, int nominal_cov, int dev)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= T_y)
        return;
    const int b = find_seq(y_off, B, i, 0);
    int64_t k = i - y_off[b];
    if (ilv_E > 0) {
        const int64_t TS = (int64_t)ilv_T * ilv_E, cnt = y_off[b + 1] - y_off[b];
        const int64_t start = (k / TS) * TS;
        const int tcnt = (int)((cnt - start) < TS ? (cnt - start) : TS);
        k = start + ilv_inv((int)(k - start), tcnt, ilv_E);
    }
    const int64_t t = y_off[b] + k; // step slot
    const int64_t s = t + b;        // state slot of state k
    auto load_nom = [&](int64_t st, Marg<T, 5> &mg) {
        nom.load(st, mg);
        if (nominal_cov && !taylor) {
            T Pm[5][5], L[5][5];
            sym_full(Pm, [&](int r, int q) { return mg.N[r][q]; });
            chol_lower(Pm, L);
#pragma unroll
            for (int r = 0; r < 5; ++r)
#pragma unroll
                for (int q = 0; q <= r; ++q)
                    mg.N[r][q] = L[r][q];
        }
    };
    T F[5][5], c[5], SL[5][5], rk[5], rk1[5];
    {
        Marg<T, 5> mg;
        load_nom(s, mg);
        if (taylor)
            ct_taylor_transition(P, mg, F, c, SL);
        else
            ct_slr_transition(P, mg, F, c, SL);
#pragma unroll
        for (int r = 0; r < 5; ++r)
            rk[r] = mg.m[r];
    }
    T yy[2] = {y[t], y[T_y + t]};
    T H[2][5], d[2], SO[2][2];
    {
        Marg<T, 5> mg;
        load_nom(s + 1, mg);
        if (taylor)
            ct_taylor_bearings(P, mg, yy, H, d, SO);
        else
            ct_slr_bearings(P, mg, yy, H, d, SO);
#pragma unroll
        for (int r = 0; r < 5; ++r)
            rk1[r] = mg.m[r];
    }
    if (dev) {
        dev_trans_offset(F, rk, rk1, c);
        dev_obs_offset(H, rk1, d);
    }
    gam.store_trans(t, F, c, SL);
    if (store_obs)
        gam.store_obs(t, H, d, SO);
    FElem<T, 5> e;
    if (k == 0) {
        T m[5], N[5][5];
#pragma unroll
        for (int r = 0; r < 5; ++r) {
            m[r] = dev ? T(typename BranchPrec<T>::type(m0[r]) - rk[r]) : m0[r];
#pragma unroll
            for (int q = 0; q <= r; ++q)
                N[r][q] = N0[tri_idx(r, q)];
        }
        if constexpr (COV)
            filter_element_first_cov(m, N, F, c, SL, H, d, SO, yy, e);
        else
            filter_element_first(m, N, F, c, SL, H, d, SO, yy, e);
    } else {
        if constexpr (COV)
            filter_element_cov(F, c, SL, H, d, SO, yy, e);
        else
            filter_element(F, c, SL, H, d, SO, yy, e);
    }
    out.store(i, e);
}

// the CT model with the unscented or Gauss-Hermite rule (one thread per
// state, the slots as k_slr_ct)
template <typename T>
__global__ __launch_bounds__(128) void k_slr_ct_rule(const int64_t *y_off, int B, int64_t T_x,
                                                     int64_t T_y, CTParams<T> P,
                                                     MargRef<T, 5> nom, const T *y,
                                                     GammaRef<T, 5, 2> out, RuleSpec<T> R,
                                                     int nominal_cov, int dev)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= T_x)
        return;
    const int b = find_seq(y_off, B, s, 1);
    const int64_t x0 = y_off[b] + b, k = s - x0, n = y_off[b + 1] - y_off[b];
    Marg<T, 5> mg;
    nom.load(s, mg);
    if (nominal_cov) {
        T Pm[5][5], L[5][5];
        sym_full(Pm, [&](int i, int j) { return mg.N[i][j]; });
        chol_lower(Pm, L);
#pragma unroll
        for (int i = 0; i < 5; ++i)
#pragma unroll
            for (int j = 0; j <= i; ++j)
                mg.N[i][j] = L[i][j];
    }
    if (k < n) {
        T G[5][5], off[5], S[5][5];
        ct_rule_transition(R, P, mg, G, off, S);
        if (dev) {
            T r1[5];
#pragma unroll
            for (int i = 0; i < 5; ++i)
                r1[i] = nom.m[i * nom.ld + s + 1];
            dev_trans_offset(G, mg.m, r1, off);
        }
        out.store_trans(y_off[b] + k, G, off, S);
    }
    if (k >= 1) {
        const int64_t t = y_off[b] + k - 1;
        T yy[2] = {y[t], y[T_y + t]};
        T G[2][5], off[2], S[2][2];
        ct_rule_bearings(R, P, mg, yy, G, off, S);
        if (dev)
            dev_obs_offset(G, mg.m, off);
        out.store_obs(t, G, off, S);
    }
}

// Ricker-Poisson model: first-order Taylor (taylor != 0) or the rule R
template <typename T>
__global__ __launch_bounds__(128) void k_slr_ricker(const int64_t *y_off, int B, int64_t T_x,
                                                    RickerParams<T> P, MargRef<T, 1> nom,
                                                    GammaRef<T, 1, 1> out, int taylor,
                                                    RuleSpec<T> R, int nominal_cov)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= T_x)
        return;
    const int b = find_seq(y_off, B, s, 1);
    const int64_t x0 = y_off[b] + b, k = s - x0, n = y_off[b + 1] - y_off[b];
    Marg<T, 1> mg;
    nom.load(s, mg);
    if (nominal_cov) // the nominal holds the variance
        mg.N[0][0] = psqrt(mg.N[0][0]);
    T F[1][1], c[1], SL[1][1], H[1][1], d[1], SO[1][1];
    if (taylor) {
        ricker_taylor(P, mg, mg, k < n, k >= 1, F, c, SL, H, d, SO);
    } else {
        if (k < n)
            ricker_rule_transition(R, P, mg, F, c, SL);
        if (k >= 1)
            ricker_rule_poisson(R, P, mg, H, d, SO);
    }
    if (k < n)
        out.store_trans(y_off[b] + k, F, c, SL);
    if (k >= 1)
        out.store_obs(y_off[b] + k - 1, H, d, SO);
}

// covariance form of the log-likelihood terms: P^- = F P^f F^T + Lambda,
// S = H P^- H^T + Omega = Y Y^T (Cholesky), ell = log N(y; H m^- + d, S)
template <typename T, int NX, int NY>
__global__ __launch_bounds__(128) void k_loglik_terms_cov(const int64_t *y_off, int B,
                                                          int64_t T_y, int64_t T_x,
                                                          GammaRef<T, NX, NY> gam, const T *y,
                                                          MargRef<T, NX> filt, double *ell)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T_y)
        return;
    const int b = find_seq(y_off, B, t, 0);
    T F[NX][NX], c[NX], SL[NX][NX], H[NY][NX], d[NY], SO[NY][NY];
    gam.load_trans(t, F, c, SL);
    gam.load_obs(t, H, d, SO);
    Marg<T, NX> f;
    filt.load(t + b, f);
    T mp[NX], P[NX][NX], FP[NX][NX], Pp[NX][NX], Om[NY][NY];
    mv(F, f.m, mp);
#pragma unroll
    for (int i = 0; i < NX; ++i)
        mp[i] += c[i];
    sym_full(P, [&](int i, int j) { return f.N[i][j]; });
    mm(F, P, FP);
    gram_full(SL, Pp);
    gram_full(SO, Om);
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j < NX; ++j) {
            T s = Pp[i][j];
#pragma unroll
            for (int k = 0; k < NX; ++k)
                s = pfma(FP[i][k], F[j][k], s);
            Pp[i][j] = s;
        }
    T HP[NY][NX], S[NY][NY], Y[NY][NY];
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
    chol_lower(S, Y);
    T Hm[NY], v[NY], u[NY];
    mv(H, mp, Hm);
#pragma unroll
    for (int a = 0; a < NY; ++a)
        v[a] = y[a * T_y + t] - Hm[a] - d[a];
    lsolve_lower(Y, v, u);
    double l = -0.5 * NY * 1.8378770664093454835606594728112; // log(2 pi)
#pragma unroll
    for (int a = 0; a < NY; ++a)
        l -= (double)plog(Y[a][a]) + 0.5 * (double)u[a] * (double)u[a];
    ell[t] = l;
}

// Score terms at a frozen nominal (Fisher's identity on the linearised
// model): for slot t (transition x_k -> x_{k+1}, measurement y_{k+1})
//   Sig  = r r^T + Var(x_{k+1} - F x_k | y),  r = m^s_{k+1} - F m^s_k - c,
//          Var = Tria([(I - F E_k) N^s_{k+1}, F D_k])^2 (smoother element
//          of Table 4: x_k = E_k x_{k+1} + g_k + N(0, D_k D_k^T)),
//   dl/dtheta_j += 1/2 tr(Lam^{-1} Sig Lam^{-1} dQ_j) - 1/2 tr(Lam^{-1} dQ_j)
//   and the same for the measurement with Sig' = v v^T + H P^s_{k+1} H^T.
// dQ_j = L_j L_j^T are passed as lower factors; dR/dlog sigma = 2 sigma^2 I.
template <typename T>
struct CTGradParams {
    T L1[5][5];
    T L2[5][5];
    T sig2; // sigma^2
};

template <typename T>
__global__ __launch_bounds__(128) void k_grad_ct(const int64_t *y_off, int B, int64_t T_y,
                                                 GammaRef<T, 5, 2> gam, const T *y,
                                                 MargRef<T, 5> filt, MargRef<T, 5> smooth,
                                                 CTGradParams<T> gp, double *gterms)
{
    constexpr int NX = 5, NY = 2;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T_y)
        return;
    const int b = find_seq(y_off, B, t, 0);
    const int64_t xs = t + b; // state k
    T F[NX][NX], c[NX], SL[NX][NX], H[NY][NX], d[NY], SO[NY][NY];
    gam.load_trans(t, F, c, SL);
    gam.load_obs(t, H, d, SO);
    Marg<T, NX> fk, sk, sk1;
    filt.load(xs, fk);
    smooth.load(xs, sk);
    smooth.load(xs + 1, sk1);
    SElem<T, NX> e;
    smoother_element(F, c, SL, fk, e);
    // V = Tria([(I - F E) N^s_{k+1}, F D])
    T FE[NX][NX], IFE[NX][NX], X1[NX][NX], X2[NX][NX];
    mm(F, e.E, FE);
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j < NX; ++j)
            IFE[i][j] = ((i == j) ? T(1) : T(0)) - FE[i][j];
    mm_lower(IFE, sk1.N, X1);
    mm_lower(F, e.D, X2);
    T Wm[NX][2 * NX + 1];
    T Fm[NX];
    mv(F, sk.m, Fm);
#pragma unroll
    for (int i = 0; i < NX; ++i) {
#pragma unroll
        for (int j = 0; j < NX; ++j) {
            Wm[i][j] = X1[i][j];
            Wm[i][NX + j] = X2[i][j];
        }
        Wm[i][2 * NX] = sk1.m[i] - Fm[i] - c[i];
    }
    // K = S^{-T} S^{-1} [V1 V2 r]  (columns of Lam^{-1} [sqrt(Sig)])
    T Kc[NX][2 * NX + 1];
#pragma unroll
    for (int col = 0; col < 2 * NX + 1; ++col) {
        T x[NX], z[NX], w[NX];
#pragma unroll
        for (int i = 0; i < NX; ++i)
            x[i] = Wm[i][col];
        lsolve_lower(SL, x, z);
        // w = S^{-T} z
#pragma unroll
        for (int i = NX - 1; i >= 0; --i) {
            T s = z[i];
#pragma unroll
            for (int q = i + 1; q < NX; ++q)
                s = pfma(-SL[q][i], w[q], s);
            w[i] = s / SL[i][i];
        }
#pragma unroll
        for (int i = 0; i < NX; ++i)
            Kc[i][col] = w[i];
    }
    double g1 = 0.0, g2 = 0.0;
    // 1/2 sum_cols |L_j^T k|^2
#pragma unroll
    for (int col = 0; col < 2 * NX + 1; ++col) {
#pragma unroll
        for (int q = 0; q < NX; ++q) {
            T s1 = T(0), s2 = T(0);
#pragma unroll
            for (int i = q; i < NX; ++i) {
                s1 = pfma(gp.L1[i][q], Kc[i][col], s1);
                s2 = pfma(gp.L2[i][q], Kc[i][col], s2);
            }
            g1 += 0.5 * (double)s1 * (double)s1;
            g2 += 0.5 * (double)s2 * (double)s2;
        }
    }
    // - 1/2 |S^{-1} L_j|_F^2
#pragma unroll
    for (int q = 0; q < NX; ++q) {
        T x1[NX], x2[NX], z1[NX], z2[NX];
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            x1[i] = (i >= q) ? gp.L1[i][q] : T(0);
            x2[i] = (i >= q) ? gp.L2[i][q] : T(0);
        }
        lsolve_lower(SL, x1, z1);
        lsolve_lower(SL, x2, z2);
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            g1 -= 0.5 * (double)z1[i] * (double)z1[i];
            g2 -= 0.5 * (double)z2[i] * (double)z2[i];
        }
    }
    // measurement: Sig' = [v, H N^s_{k+1}] [...]^T, dR = 2 sigma^2 I
    T HN[NY][NX], Hm[NY];
    mm_lower(H, sk1.N, HN);
    mv(H, sk1.m, Hm);
    double g3 = 0.0;
#pragma unroll
    for (int col = 0; col <= NX; ++col) {
        T x[NY], z[NY], w[NY];
#pragma unroll
        for (int a = 0; a < NY; ++a)
            x[a] = (col < NX) ? HN[a][col] : (y[a * T_y + t] - Hm[a] - d[a]);
        lsolve_lower(SO, x, z);
#pragma unroll
        for (int i = NY - 1; i >= 0; --i) {
            T s = z[i];
#pragma unroll
            for (int q = i + 1; q < NY; ++q)
                s = pfma(-SO[q][i], w[q], s);
            w[i] = s / SO[i][i];
        }
#pragma unroll
        for (int a = 0; a < NY; ++a)
            g3 += (double)gp.sig2 * (double)w[a] * (double)w[a];
    }
#pragma unroll
    for (int q = 0; q < NY; ++q) {
        T x[NY], z[NY];
#pragma unroll
        for (int a = 0; a < NY; ++a)
            x[a] = (a == q) ? T(1) : T(0);
        lsolve_lower(SO, x, z);
#pragma unroll
        for (int a = 0; a < NY; ++a)
            g3 -= (double)gp.sig2 * (double)z[a] * (double)z[a];
    }
    gterms[0 * T_y + t] = g1;
    gterms[1 * T_y + t] = g2;
    gterms[2 * T_y + t] = g3;
}

} // namespace pss
