// Gradient of the pseudo-log-likelihood at the IPLS fixed point (Section 5.2,
// eq. implicity_function_theorem, Algorithm 4) for the coordinated-turn model.
//
// At the fixed point n* = KS(n*, theta) the total derivative of
// l(theta) = lhat(theta, n*(theta)) needs dn*/dtheta, which solves the linear
// fixed point dn = dKS/dn dn + dKS/dtheta.  Algorithm 4 iterates that
// equation; here each iteration is one pass of the parallel covariance-form
// smoother (SLR, filter elements, filter scan, smoother scan) run on numbers
// that carry three tangents (Dual<S, 3> for S = double or float, one per theta
// component; this file is compiled once per S, with PSS_IFT_T set): with
// the nominal's value held at n* and its tangents set to the previous
// iterate, the pass's output tangents are exactly dKS/dn dn + dKS/dtheta.
// The same scans, operators and storage layouts as the value pass are used,
// instantiated for the dual type; every step keeps the O(log n) span.  The
// covariance form is used (as Algorithm 4 states it): its operators are
// smooth wherever they are defined, whereas the square-root form's Tria is
// not differentiable where a factor loses rank (leaf elements have rank ny).
// A final dual pass evaluates the log-likelihood terms, whose tangents are
// the gradient.
#include <math.h>

#include <string>

#include "ift.hpp"

namespace pss {

// value-only dual copy of an array
template <typename S>
__global__ __launch_bounds__(256) void k_to_dual(const S *x, Dual<S, 3> *out, int64_t n)
{
    using D = Dual<S, 3>;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        out[i] = D(x[i]);
}

// dual nominal from the caller's fixed point (m [5][T_x], N packed [15][T_x],
// a factor when is_factor, else the covariance): the covariance form's
// (m, P); tangents zeroed (value_only = 0) or kept (value_only = 1).  With
// value_only, stat[s] receives the largest change of state s's tangents
// since the previous call relative to max(1, their size), and prev keeps
// the tangents for the next call ([20 values][3 tangents][T_x]).
template <typename S>
__global__ __launch_bounds__(128) void k_ift_nominal(int64_t T_x, const S *m, const S *N,
                                                     int is_factor, Dual<S, 3> *nm,
                                                     Dual<S, 3> *nP, int value_only,
                                                     double *prev, double *stat)
{
    using D = Dual<S, 3>;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= T_x)
        return;
    double dmax = 0.0, amax = 0.0;
    bool finite = true;
    auto track = [&](int q, const D &x) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int64_t at = ((int64_t)q * 3 + k) * T_x + s;
            const double t = value_only ? (double)x.d[k] : 0.0;
            finite = finite && isfinite(t);
            dmax = fmax(dmax, fabs(t - prev[at]));
            amax = fmax(amax, fabs(t));
            prev[at] = t;
        }
    };
#pragma unroll
    for (int i = 0; i < 5; ++i)
        track(i, nm[(int64_t)i * T_x + s]);
#pragma unroll
    for (int q = 0; q < 15; ++q)
        track(5 + q, nP[(int64_t)q * T_x + s]);
    // a tangent that overflowed reports an infinite change
    stat[s] = finite ? dmax / fmax(1.0, amax) : INFINITY;
    S L[5][5];
#pragma unroll
    for (int i = 0; i < 5; ++i)
#pragma unroll
        for (int j = 0; j < 5; ++j)
            L[i][j] = j <= i ? N[(int64_t)tri_idx(i, j) * T_x + s] : S(0);
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const S v = m[(int64_t)i * T_x + s];
        if (value_only)
            nm[(int64_t)i * T_x + s].v = v;
        else
            nm[(int64_t)i * T_x + s] = D(v);
    }
#pragma unroll
    for (int i = 0; i < 5; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            S v = L[i][j];
            if (is_factor) {
                v = S(0);
#pragma unroll
                for (int t = 0; t <= j; ++t)
                    v = pfma(L[i][t], L[j][t], v);
            }
            const int64_t at = (int64_t)tri_idx(i, j) * T_x + s;
            if (value_only)
                nP[at].v = v;
            else
                nP[at] = D(v);
        }
}

// per sequence: the largest stat over its states (one block per sequence)
static __global__ __launch_bounds__(256) void k_seq_max(const int64_t *y_off,
                                                        const double *stat, double *out)
{
    __shared__ double red[256];
    const int b = blockIdx.x;
    const int64_t x0 = y_off[b] + b, x1 = y_off[b + 1] + b + 1;
    double v = 0.0;
    for (int64_t s = x0 + threadIdx.x; s < x1; s += blockDim.x)
        v = fmax(v, stat[s]);
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0)
        out[b] = red[0];
}

// covariance-form log-likelihood terms (as k_loglik_terms_cov) in dual
// numbers: ell[0][t] the value, ell[1 + k][t] its tangent k
template <typename S>
__global__ __launch_bounds__(128) void k_loglik_terms_cov_dual(const int64_t *y_off, int B,
                                                               int64_t T_y,
                                                               GammaRef<Dual<S, 3>, 5, 2> gam,
                                                               const S *y,
                                                               MargRef<Dual<S, 3>, 5> filt,
                                                               double *ell)
{
    using D = Dual<S, 3>;
    constexpr int NX = 5, NY = 2;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T_y)
        return;
    const int b = find_seq(y_off, B, t, 0);
    D F[NX][NX], c[NX], SL[NX][NX], H[NY][NX], d[NY], SO[NY][NY];
    gam.load_trans(t, F, c, SL);
    gam.load_obs(t, H, d, SO);
    Marg<D, NX> f;
    filt.load(t + b, f);
    D mp[NX], P[NX][NX], FP[NX][NX], Pp[NX][NX], Om[NY][NY];
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
            D s = Pp[i][j];
#pragma unroll
            for (int k = 0; k < NX; ++k)
                s = pfma(FP[i][k], F[j][k], s);
            Pp[i][j] = s;
        }
    D HP[NY][NX], Sy[NY][NY], Y[NY][NY];
    mm(H, Pp, HP);
#pragma unroll
    for (int a = 0; a < NY; ++a)
#pragma unroll
        for (int q = 0; q < NY; ++q) {
            D s = Om[a][q];
#pragma unroll
            for (int j = 0; j < NX; ++j)
                s = pfma(HP[a][j], H[q][j], s);
            Sy[a][q] = s;
        }
    chol_lower(Sy, Y);
    D Hm[NY], v[NY], u[NY];
    mv(H, mp, Hm);
#pragma unroll
    for (int a = 0; a < NY; ++a)
        v[a] = (D(y[a * T_y + t]) - Hm[a]) - d[a];
    lsolve_lower(Y, v, u);
    // the sum in FP64 for both precisions, as the value pass does
    double lv = -0.5 * NY * 1.8378770664093454835606594728112; // log(2 pi)
    double ld[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < NY; ++a) {
        const D q = plog(Y[a][a]) + S(0.5) * (u[a] * u[a]);
        lv -= (double)q.v;
#pragma unroll
        for (int k = 0; k < 3; ++k)
            ld[k] -= (double)q.d[k];
    }
    ell[t] = lv;
#pragma unroll
    for (int k = 0; k < 3; ++k)
        ell[(int64_t)(1 + k) * T_y + t] = ld[k];
}

template <typename S>
static size_t scan_ws_bytes(const Ctx &c)
{
    using D = Dual<S, 3>;
    using C = IftC<S>;
    using FSC = FilterScanCov<D, 5>;
    using SSC = SmootherScanCov<D, 5>;
    Carver a{nullptr};
    C::template carve_scan<FSC>(a, c, C::filter_shape(c));
    Carver b{nullptr};
    C::template carve_scan<SSC>(b, c, C::smoother_shape(c));
    b.take<D>((size_t)Sizes<5>::selem * c.T_x); // smoother element stash
    return std::max(std::max(a.used, b.used), seq_sum_bytes(c, 3));
}

template <typename S>
static IftBufs<S> carve_ift(const Ctx &c, void *base)
{
    using D = Dual<S, 3>;
    using C = IftC<S>;
    Carver cv{static_cast<char *>(base)};
    IftBufs<S> w;
    w.nm = cv.take<D>((size_t)5 * c.T_x);
    w.nP = cv.take<D>((size_t)15 * c.T_x);
    w.mf = cv.take<D>((size_t)5 * c.T_x);
    w.Pf = cv.take<D>((size_t)15 * c.T_x);
    w.yd = cv.take<D>((size_t)2 * c.T_y);
    w.m0d = cv.take<D>(5);
    w.N0d = cv.take<D>(15);
    w.gam = C::carve_gamma(cv, c.T_y);
    D *fel = cv.take<D>((size_t)Sizes<5>::felem * c.T_y);
    w.fel = C::felem_ref(fel, c.T_y);
    w.ell = cv.take<double>((size_t)4 * c.T_y);
    w.prev = cv.take<double>((size_t)60 * c.T_x);
    w.stat = cv.take<double>((size_t)c.T_x);
    w.scan_ws = cv.base ? cv.base + cv.used : nullptr;
    w.used = cv.used + scan_ws_bytes<S>(c);
    return w;
}

template <typename S>
static int launch_slr(const Ctx &c, const IftBufs<S> &w)
{
    using D = Dual<S, 3>;
    using C = IftC<S>;
    const CTHost h = ct_host(c.p);
    CTParams<D> P;
    P.dt = D(h.dt);
    P.s1x = D(h.s1x);
    P.s1y = D(h.s1y);
    P.s2x = D(h.s2x);
    P.s2y = D(h.s2y);
    // theta = (log q1, log q2, log sigma): the q1 part of the factor scales
    // as sqrt(q1), the q2 part as sqrt(q2), sigma as e^theta3
    P.sigma = D(h.sigma);
    P.sigma.d[2] = (S)h.sigma;
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 5; ++j) {
            P.LQ[i][j] = D(h.LQ[i][j]);
            P.LQ[i][j].d[0] = (S)(0.5 * h.L1[i][j]);
            P.LQ[i][j].d[1] = (S)(0.5 * h.L2[i][j]);
        }
    const int tb = 128;
    const dim3 grid((unsigned)((c.T_x + tb - 1) / tb));
    const int lin = c.p->linearization;
    KTime kt(c.s, "ift_slr", "", 0);
    // Cubature goes through the general rule kernel too (the same rule, 2 nx
    // points of weight 1/(2 nx)): it accumulates the sigma-point moments
    // point by point, while the dedicated kernel holds every image at once.
    // In Dual<float, 3> that kernel reached the 512-register ceiling and its
    // results disagreed with the same steps run on the host; the rule kernel
    // stays well inside the limit.
    if (lin == PSS_LIN_TAYLOR) {
        hipLaunchKernelGGL((k_slr_ct<D, true>), grid, dim3(tb), 0, c.s, c.p->y_off, c.B, c.T_x,
                           c.T_y, P, C::marg_ref2(w.nm, w.nP, c.T_x), w.yd,
                           C::gamma_ref(&w.gam, c.T_y), 1, 1, 0);
    } else {
        RuleSpec<double> Rd;
        if (!rule_spec(c.p, 5, Rd))
            return PSS_EINVAL;
        // the rule's nodes and weights enter with zero tangents
        RuleSpec<D> R;
        R.kind = Rd.kind;
        R.np = Rd.np;
        R.p = Rd.p;
        R.w0 = D(Rd.w0);
        R.wi = D(Rd.wi);
        R.spread = D(Rd.spread);
        for (int q = 0; q < kMaxGH; ++q) {
            R.gx[q] = D(Rd.gx[q]);
            R.gw[q] = D(Rd.gw[q]);
        }
        hipLaunchKernelGGL((k_slr_ct_rule<D>), grid, dim3(tb), 0, c.s, c.p->y_off, c.B, c.T_x,
                           c.T_y, P, C::marg_ref2(w.nm, w.nP, c.T_x), w.yd,
                           C::gamma_ref(&w.gam, c.T_y), R, 1, 0);
    }
    return hip_check(hipGetLastError(), "ift slr launch");
}

template <typename S>
static int launch_felem(const Ctx &c, const IftBufs<S> &w)
{
    using D = Dual<S, 3>;
    using C = IftC<S>;
    const ScanShape sh = C::filter_shape(c);
    const int tb = 128;
    KTime kt(c.s, "ift_filter_elements", "", 0);
    hipLaunchKernelGGL((k_filter_elements<D, 5, 2, true>), dim3((unsigned)((c.T_y + tb - 1) / tb)),
                       dim3(tb), 0, c.s, c.p->y_off, c.B, c.T_y, C::gamma_ref(&w.gam, c.T_y), w.yd,
                       w.m0d, w.N0d, w.fel, sh.T[0], sh.E[0], static_cast<const D *>(nullptr),
                       c.T_x);
    return hip_check(hipGetLastError(), "ift filter elements launch");
}

template <typename S>
static int run_fscan(const Ctx &c, const IftBufs<S> &w)
{
    using D = Dual<S, 3>;
    using C = IftC<S>;
    using FSC = FilterScanCov<D, 5>;
    const ScanShape sh = C::filter_shape(c);
    Carver cv{static_cast<char *>(w.scan_ws)};
    auto sw = C::template carve_scan<FSC>(cv, c, sh);
    FiltDst<D, 5> dst{C::marg_ref2(w.mf, w.Pf, c.T_x), c.p->y_off};
    StartPreCov<D, 5> st{w.m0d, w.N0d};
    RefSrc<FSC, FElemRef<D, 5>, true> src{w.fel};
    return C::template run_scan<FSC, C::kFlatF>(c, sh, sw, 0, src, dst, st, &C::felem_ref);
}

template <typename S>
size_t ift_ws(const pss_problem *p)
{
    Ctx c;
    c.p = p;
    c.B = p->B;
    c.T_y = p->y_off_host[p->B];
    c.T_x = c.T_y + p->B;
    c.s = nullptr;
    return carve_ift<S>(c, nullptr).used;
}

template <typename S>
int ift_run(const pss_problem *p, const void *m_nom, const void *N_nom, const void *y,
            int32_t n_iter, double *ll, double *grad, double *delta, void *ws,
            hipStream_t stream)
{
    using C = IftC<S>;
    Ctx c;
    c.p = p;
    c.B = p->B;
    c.T_y = p->y_off_host[p->B];
    c.T_x = c.T_y + p->B;
    c.s = stream;
    const IftBufs<S> w = carve_ift<S>(c, ws);
    const int is_factor = p->form == PSS_FORM_SQRT ? 1 : 0;
    const dim3 blk(256);
    const S *ys = static_cast<const S *>(y);
    hipLaunchKernelGGL(k_to_dual<S>, dim3((unsigned)((2 * c.T_y + 255) / 256)), blk, 0, stream, ys,
                       w.yd, 2 * c.T_y);
    hipLaunchKernelGGL(k_to_dual<S>, dim3(1), blk, 0, stream, static_cast<const S *>(p->m0), w.m0d,
                       (int64_t)5);
    hipLaunchKernelGGL(k_to_dual<S>, dim3(1), blk, 0, stream, static_cast<const S *>(p->N0), w.N0d,
                       (int64_t)15);
    const dim3 gx((unsigned)((c.T_x + 127) / 128));
    const S *mn = static_cast<const S *>(m_nom);
    const S *Nn = static_cast<const S *>(N_nom);
    hipLaunchKernelGGL(k_ift_nominal<S>, gx, dim3(128), 0, stream, c.T_x, mn, Nn, is_factor, w.nm,
                       w.nP, 0, w.prev, w.stat);
    int rc;
    if ((rc = hip_check(hipGetLastError(), "ift setup launch")))
        return rc;
    for (int it = 0; it < n_iter; ++it) {
        if ((rc = launch_slr<S>(c, w)) || (rc = launch_felem<S>(c, w)) ||
            (rc = run_fscan<S>(c, w)) || (rc = run_sscan<S>(c, w)))
            return rc;
        // hold the value at the fixed point; keep the new tangents
        hipLaunchKernelGGL(k_ift_nominal<S>, gx, dim3(128), 0, stream, c.T_x, mn, Nn, is_factor,
                           w.nm, w.nP, 1, w.prev, w.stat);
        if ((rc = hip_check(hipGetLastError(), "ift nominal launch")))
            return rc;
    }
    if (delta) {
        hipLaunchKernelGGL(k_seq_max, dim3((unsigned)c.B), dim3(256), 0, stream, p->y_off, w.stat,
                           delta);
        if ((rc = hip_check(hipGetLastError(), "ift delta launch")))
            return rc;
    }
    // log-likelihood of the linearisation at (n*, dn*/dtheta)
    if ((rc = launch_slr<S>(c, w)) || (rc = launch_felem<S>(c, w)) || (rc = run_fscan<S>(c, w)))
        return rc;
    {
        KTime kt(stream, "ift_loglik_terms", "", 0);
        hipLaunchKernelGGL(k_loglik_terms_cov_dual<S>, dim3((unsigned)((c.T_y + 127) / 128)),
                           dim3(128), 0, stream, p->y_off, c.B, c.T_y, C::gamma_ref(&w.gam, c.T_y),
                           ys, C::marg_ref2(w.mf, w.Pf, c.T_x), w.ell);
        if ((rc = hip_check(hipGetLastError(), "ift loglik launch")))
            return rc;
    }
    if ((rc = launch_seq_sum(c, 1, w.ell, c.T_y, ll, w.scan_ws)))
        return rc;
    return launch_seq_sum(c, 3, w.ell + c.T_y, c.T_y, grad, w.scan_ws);
}

#if !defined(PSS_IFT_T)
#error "compile with -DPSS_IFT_T=<double|float>"
#endif
template size_t ift_ws<PSS_IFT_T>(const pss_problem *p);
template int ift_run<PSS_IFT_T>(const pss_problem *p, const void *m_nom, const void *N_nom,
                                const void *y, int32_t n_iter, double *ll, double *grad,
                                double *delta, void *ws, hipStream_t stream);

} // namespace pss
