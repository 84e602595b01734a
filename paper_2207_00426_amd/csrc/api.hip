// C ABI of the parallel square-root smoother: validation, dispatch on
// (dtype, nx, ny), scan planning and the few non-template kernels.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "rules_host.hpp"
#include "common.hpp"
#include "kernels.hpp"

namespace pss {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

int hip_check(hipError_t e, const char *what)
{
    if (e == hipSuccess)
        return PSS_OK;
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return PSS_EHIP;
}

// ---------------------------------------------------------------------------
// per-launch kernel timing (instrumentation)
// ---------------------------------------------------------------------------
namespace {
struct KRec {
    std::string key;
    int level;
    hipEvent_t a, b;
};
std::atomic<bool> g_kt_on{false};
std::mutex g_kt_mu;
std::vector<KRec> g_kt_recs;
std::vector<hipEvent_t> g_kt_pool;

hipEvent_t kt_event()
{
    hipEvent_t e = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_kt_mu);
        if (!g_kt_pool.empty()) {
            e = g_kt_pool.back();
            g_kt_pool.pop_back();
            return e;
        }
    }
    if (hipEventCreate(&e) != hipSuccess)
        return nullptr;
    return e;
}

void kt_release(hipEvent_t e)
{
    if (!e)
        return;
    std::lock_guard<std::mutex> lk(g_kt_mu);
    g_kt_pool.push_back(e);
}

bool kt_capturing(hipStream_t s)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess)
        return true; // unknown: do not record
    return st != hipStreamCaptureStatusNone;
}
} // namespace

KTime::KTime(hipStream_t s_, const char *name_, const char *phase_, int level_)
    : s(s_), name(name_), phase(phase_), level(level_)
{
    if (!g_kt_on.load(std::memory_order_relaxed) || kt_capturing(s))
        return;
    a = kt_event();
    if (a && hipEventRecord(a, s) != hipSuccess) {
        kt_release(a);
        a = nullptr;
    }
}

KTime::~KTime()
{
    if (!a)
        return;
    hipEvent_t b = kt_event();
    if (!b || hipEventRecord(b, s) != hipSuccess) {
        kt_release(a);
        kt_release(b);
        return;
    }
    std::string key = name;
    if (phase && phase[0])
        key += std::string("_") + phase;
    std::lock_guard<std::mutex> lk(g_kt_mu);
    g_kt_recs.push_back(KRec{key, level, a, b});
}

// ---------------------------------------------------------------------------
// scan planning (host side mirrors k_plan exactly)
// ---------------------------------------------------------------------------
ScanShape plan_scan(const Ctx &c, int extra, int T0, int E0, int Tup, int E1, int Eup,
                    bool flat0)
{
    ScanShape sh;
    std::vector<int64_t> cnt(c.B);
    int64_t total = 0;
    for (int b = 0; b < c.B; ++b) {
        cnt[b] = c.p->y_off_host[b + 1] - c.p->y_off_host[b] + extra;
        total += cnt[b];
    }
    sh.nelem[0] = total;
    for (int l = 0; l < kMaxLevels; ++l) {
        sh.T[l] = l == 0 ? T0 : Tup;
        sh.E[l] = l == 0 ? E0 : (l == 1 ? E1 : Eup);
        const int64_t TS = (int64_t)sh.T[l] * sh.E[l];
        int64_t nt = 0, mx = 0;
        for (int b = 0; b < c.B; ++b) {
            mx = std::max(mx, cnt[b]);
            nt += (cnt[b] + TS - 1) / TS;
        }
        sh.ntiles[l] = nt;
        // a flat level 0 is never the top, also where one tile would hold
        // every sequence: a sequence's bracketing must not depend on the
        // lengths of the others in its batch (a level that holds a sequence
        // in one tile passes it through bitwise unchanged)
        sh.flat[l] = l == 0 && flat0;
        if (mx <= TS && !sh.flat[l]) {
            sh.L = l + 1;
            break;
        }
        const int64_t D = sh.flat[l] ? sh.E[l] : TS;
        int64_t ne = 0;
        for (int b = 0; b < c.B; ++b) {
            cnt[b] = (cnt[b] + D - 1) / D;
            ne += cnt[b];
        }
        if (l + 1 < kMaxLevels)
            sh.nelem[l + 1] = ne;
    }
    return sh;
}

// exclusive block-wide prefix sums of one value per sequence, written to
// out[0..B] (one block of 1024 threads; the block calls it uniformly)
template <class F>
__device__ void plan_offsets(int B, int64_t *out, int64_t *sh, int64_t &carry, F value)
{
    if (threadIdx.x == 0) {
        carry = 0;
        out[0] = 0;
    }
    for (int base = 0; base < B; base += 1024) {
        const int b = base + threadIdx.x;
        const int64_t t = b < B ? value(b) : 0;
        __syncthreads();
        sh[threadIdx.x] = t;
        for (int d = 1; d < 1024; d <<= 1) {
            __syncthreads();
            const int64_t v = (int)threadIdx.x >= d ? sh[threadIdx.x - d] : 0;
            __syncthreads();
            sh[threadIdx.x] += v;
        }
        __syncthreads();
        if (b < B)
            out[b + 1] = carry + sh[threadIdx.x];
        __syncthreads();
        if (threadIdx.x == 0)
            carry += sh[1023];
        __syncthreads();
    }
}

__global__ __launch_bounds__(1024) void k_plan(PlanArgs a)
{
    __shared__ int64_t sh[1024];
    __shared__ int64_t carry;
    if (a.B <= 64) {
        // few sequences: one thread, no block-wide scans
        if (threadIdx.x != 0)
            return;
        for (int l = 0; l < a.L; ++l) {
            int64_t t_acc = 0, e_acc = 0;
            a.tile_off[l][0] = 0;
            if (l > 0 && a.elem_off[l])
                a.elem_off[l][0] = 0;
            for (int b = 0; b < a.B; ++b) {
                int64_t cn = a.y_off[b + 1] - a.y_off[b] + a.extra;
                for (int q = 0; q < l; ++q)
                    cn = (cn + a.D[q] - 1) / a.D[q];
                t_acc += (cn + a.TS[l] - 1) / a.TS[l];
                e_acc += cn;
                a.tile_off[l][b + 1] = t_acc;
                if (l > 0 && a.elem_off[l])
                    a.elem_off[l][b + 1] = e_acc;
            }
        }
        return;
    }
    for (int l = 0; l < a.L; ++l) {
        // elements of sequence b at level l
        auto elems = [&](int b) {
            int64_t cn = a.y_off[b + 1] - a.y_off[b] + a.extra;
            for (int q = 0; q < l; ++q)
                cn = (cn + a.D[q] - 1) / a.D[q];
            return cn;
        };
        plan_offsets(a.B, a.tile_off[l], sh, carry,
                     [&](int b) { return (elems(b) + a.TS[l] - 1) / a.TS[l]; });
        if (l > 0 && a.elem_off[l])
            plan_offsets(a.B, a.elem_off[l], sh, carry, elems);
    }
}

int launch_plan(const Ctx &c, const ScanShape &sh, int extra, int64_t *const *tile_off,
                int64_t *const *elem_off)
{
    PlanArgs a;
    a.y_off = c.p->y_off;
    a.B = c.B;
    a.extra = extra;
    a.L = sh.L;
    for (int l = 0; l < kMaxLevels; ++l) {
        const bool in = l < sh.L;
        a.TS[l] = in ? (int64_t)sh.T[l] * sh.E[l] : 1;
        a.D[l] = in ? (sh.flat[l] ? sh.E[l] : a.TS[l]) : 1;
        a.tile_off[l] = in ? tile_off[l] : nullptr;
        a.elem_off[l] = in && elem_off ? elem_off[l] : nullptr;
    }
    hipLaunchKernelGGL(k_plan, dim3(1), dim3(1024), 0, c.s, a);
    return hip_check(hipGetLastError(), "plan launch");
}

static int64_t seq_chunks(const Ctx &c)
{
    int64_t tot = 0;
    for (int b = 0; b < c.B; ++b)
        tot += (c.p->y_off_host[b + 1] - c.p->y_off_host[b] + kSumChunk - 1) / kSumChunk;
    return tot;
}

size_t seq_sum_bytes(const Ctx &c, int nc)
{
    Carver cv{nullptr};
    cv.take<int64_t>(c.B + 1);
    cv.take<double>((size_t)nc * seq_chunks(c));
    return cv.used;
}

int launch_seq_sum(const Ctx &c, int nc, const double *terms, int64_t ld, double *out, void *ws)
{
    Carver cv{static_cast<char *>(ws)};
    int64_t *chunk_off = cv.take<int64_t>(c.B + 1);
    const int64_t nch = seq_chunks(c);
    double *partial = cv.take<double>((size_t)nc * nch);
    ScanShape sh;
    sh.L = 1;
    sh.T[0] = kSumChunk;
    sh.E[0] = 1;
    int rc = launch_plan(c, sh, 0, &chunk_off);
    if (rc)
        return rc;
    if (nc == 1) {
        hipLaunchKernelGGL(k_chunk_sum<1>, dim3((unsigned)nch), dim3(256), 0, c.s, c.p->y_off,
                           chunk_off, c.B, terms, ld, partial, nch);
        hipLaunchKernelGGL(k_seq_total<1>, dim3((c.B + 63) / 64), dim3(64), 0, c.s, chunk_off,
                           partial, nch, c.B, out);
    } else {
        hipLaunchKernelGGL(k_chunk_sum<3>, dim3((unsigned)nch), dim3(256), 0, c.s, c.p->y_off,
                           chunk_off, c.B, terms, ld, partial, nch);
        hipLaunchKernelGGL(k_seq_total<3>, dim3((c.B + 63) / 64), dim3(64), 0, c.s, chunk_off,
                           partial, nch, c.B, out);
    }
    return hip_check(hipGetLastError(), "sequence sum launch");
}

__global__ __launch_bounds__(256) void k_weighted_grad(const double *grad, const double *w, int B,
                                                       double *theta_bar)
{
    if (threadIdx.x < 3) {
        double s = 0.0;
        for (int b = 0; b < B; ++b)
            s += (w ? w[b] : 1.0) * grad[(int64_t)threadIdx.x * B + b];
        theta_bar[threadIdx.x] = s;
    }
}

// per-sequence non-finite check: one thread per state (or per sequence for
// the log-likelihood); a thread that sees a NaN or infinity ORs `bit` into
// its sequence's status word (a vector atomic; none in the common case)
template <typename T>
__global__ __launch_bounds__(256) void k_nan_status(const int64_t *y_off, int B, int64_t T_x,
                                                    const T *m, const T *N, int nx, int np,
                                                    const double *ll, int32_t bit_marg,
                                                    int32_t bit_ll, int32_t *status)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m && s < T_x) {
        bool bad = false;
        for (int c = 0; c < nx; ++c)
            bad |= !isfinite(m[c * T_x + s]);
        for (int c = 0; c < np; ++c)
            bad |= !isfinite(N[c * T_x + s]);
        if (bad)
            atomicOr(status + find_seq(y_off, B, s, 1), bit_marg);
    }
    if (ll && s < B && !isfinite(ll[s]))
        atomicOr(status + s, bit_ll);
}

int launch_nan_status(const Ctx &c, const void *m, const void *N, const double *ll, int bit_marg,
                      int bit_ll, int32_t *status)
{
    const int nx = c.p->nx, np = nx * (nx + 1) / 2;
    const int64_t work = m ? std::max<int64_t>(c.T_x, c.B) : c.B;
    const dim3 grid((unsigned)((work + 255) / 256));
    if (c.p->dtype == PSS_F64)
        hipLaunchKernelGGL(k_nan_status<double>, grid, dim3(256), 0, c.s, c.p->y_off, c.B, c.T_x,
                           static_cast<const double *>(m), static_cast<const double *>(N), nx, np,
                           ll, bit_marg, bit_ll, status);
    else
        hipLaunchKernelGGL(k_nan_status<float>, grid, dim3(256), 0, c.s, c.p->y_off, c.B, c.T_x,
                           static_cast<const float *>(m), static_cast<const float *>(N), nx, np,
                           ll, bit_marg, bit_ll, status);
    return hip_check(hipGetLastError(), "nan status launch");
}

int launch_weighted_grad(const Ctx &c, const double *grad, const double *w, double *theta_bar)
{
    hipLaunchKernelGGL(k_weighted_grad, dim3(1), dim3(64), 0, c.s, grad, w, c.B, theta_bar);
    return hip_check(hipGetLastError(), "weighted gradient launch");
}

// ---------------------------------------------------------------------------
// coordinated-turn constants: Q(theta) = q1 Qv + q2 Qw (integrated white-noise
// acceleration on each axis, random-walk turn rate); its lower factor splits
// into the q1 part L1 (per axis [[a, 0], [b, c]] on (p, v)) and the q2 part L2.
// ---------------------------------------------------------------------------
CTHost ct_host(const pss_problem *p)
{
    CTHost h{};
    h.dt = p->dt;
    h.q1 = exp(p->theta[0]);
    h.q2 = exp(p->theta[1]);
    h.sigma = exp(p->theta[2]);
    h.s1x = p->sensors[0];
    h.s1y = p->sensors[1];
    h.s2x = p->sensors[2];
    h.s2y = p->sensors[3];
    const double dt = h.dt;
    const double a = sqrt(h.q1 * dt * dt * dt / 3.0);
    const double b = (h.q1 * dt * dt / 2.0) / a;
    const double cc = 0.5 * sqrt(h.q1 * dt);
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 5; ++j)
            h.L1[i][j] = h.L2[i][j] = 0.0;
    h.L1[0][0] = h.L1[1][1] = a;
    h.L1[2][0] = h.L1[3][1] = b;
    h.L1[2][2] = h.L1[3][3] = cc;
    h.L2[4][4] = sqrt(h.q2 * dt);
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 5; ++j)
            h.LQ[i][j] = h.L1[i][j] + h.L2[i][j];
    return h;
}

RickerHost ricker_host(const pss_problem *p)
{
    RickerHost h;
    h.loga = p->theta[0];
    h.b = exp(p->theta[1]);
    h.sqQ = exp(0.5 * p->theta[2]);
    return h;
}

bool rule_host(const pss_problem *p, int nx, RuleHost &r)
{
    r = RuleHost{};
    switch (p->linearization) {
    case PSS_LIN_UNSCENTED: {
        const double k = p->ut_kappa;
        r.kind = 1;
        r.w0 = k / (nx + k);
        r.wi = 1.0 / (2.0 * (nx + k));
        r.spread = sqrt(nx + k);
        r.np = 2 * nx + (k > 0.0 ? 1 : 0);
        return true;
    }
    case PSS_LIN_GAUSS_HERMITE: {
        const int q = p->gh_order;
        if (q < 2 || q > kMaxGH) {
            set_error("gh_order must be in 2..20");
            return false;
        }
        int64_t np = 1;
        for (int j = 0; j < nx; ++j)
            np *= q;
        if (np > kMaxRulePoints) {
            set_error("Gauss-Hermite rule: gh_order^nx must not exceed 1024 points");
            return false;
        }
        r.kind = 2;
        r.p = q;
        r.np = (int)np;
        gauss_hermite_1d(q, r.gx, r.gw);
        return true;
    }
    default: // cubature
        r.kind = 0;
        r.w0 = 0.0;
        r.wi = 1.0 / (2.0 * nx);
        r.spread = sqrt((double)nx);
        r.np = 2 * nx;
        return true;
    }
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
template <typename T, int NX, int NY>
struct Tag {
    using I = Impl<T, NX, NY>;
};

template <typename T, class Fn>
static int dispatch_dims(const pss_problem *p, Fn &&fn)
{
#define PSS_CASE(a, b)                                                                           \
    if (p->nx == a && p->ny == b)                                                                \
        return fn(Tag<T, a, b>{});
    PSS_DIMS(PSS_CASE)
#undef PSS_CASE
    set_error("dimension pair (nx, ny) not built");
    return PSS_EUNSUPPORTED;
}

template <class Fn>
static int dispatch(const pss_problem *p, Fn &&fn)
{
    if (p->dtype == PSS_F64)
        return dispatch_dims<double>(p, fn);
    return dispatch_dims<float>(p, fn);
}

static bool dims_built(int nx, int ny)
{
#define PSS_CHK(a, b)                                                                            \
    if (nx == a && ny == b)                                                                      \
        return true;
    PSS_DIMS(PSS_CHK)
#undef PSS_CHK
    return false;
}

static int validate(const pss_problem *p)
{
    if (!p) {
        set_error("null problem");
        return PSS_EINVAL;
    }
    if (p->model != PSS_MODEL_LINEAR && p->model != PSS_MODEL_CT_BEARINGS &&
        p->model != PSS_MODEL_RICKER_POISSON) {
        set_error("unknown model");
        return PSS_EINVAL;
    }
    if (p->dtype != PSS_F32 && p->dtype != PSS_F64) {
        set_error("unknown dtype");
        return PSS_EINVAL;
    }
    if (p->nx < 1 || p->ny < 1 || p->nx > 8 || p->ny > 8) {
        set_error("nx and ny must be in 1..8");
        return PSS_EINVAL;
    }
    if (p->model == PSS_MODEL_CT_BEARINGS && (p->nx != 5 || p->ny != 2)) {
        set_error("the coordinated-turn model has nx = 5, ny = 2");
        return PSS_EINVAL;
    }
    if (p->model == PSS_MODEL_RICKER_POISSON && (p->nx != 1 || p->ny != 1)) {
        set_error("the Ricker-Poisson model has nx = ny = 1");
        return PSS_EINVAL;
    }
    if (!dims_built(p->nx, p->ny)) {
        set_error("dimension pair (nx, ny) not built");
        return PSS_EUNSUPPORTED;
    }
    if (p->B < 1) {
        set_error("B must be >= 1");
        return PSS_EINVAL;
    }
    if (!p->y_off || !p->y_off_host || !p->m0 || !p->N0) {
        set_error("null y_off, y_off_host, m0 or N0");
        return PSS_EINVAL;
    }
    if (p->y_off_host[0] != 0) {
        set_error("y_off[0] must be 0");
        return PSS_EINVAL;
    }
    for (int b = 0; b < p->B; ++b)
        if (p->y_off_host[b + 1] <= p->y_off_host[b]) {
            set_error("every sequence needs at least one measurement (y_off strictly rising)");
            return PSS_EINVAL;
        }
    if (p->scan_threads != 0 && p->scan_threads != 64 && p->scan_threads != 128 &&
        p->scan_threads != 256) {
        set_error("scan_threads must be 0, 64, 128 or 256");
        return PSS_EINVAL;
    }
    if (p->form != PSS_FORM_SQRT && p->form != PSS_FORM_COV) {
        set_error("form must be PSS_FORM_SQRT or PSS_FORM_COV");
        return PSS_EINVAL;
    }
    if (p->linearization < PSS_LIN_CUBATURE || p->linearization > PSS_LIN_GAUSS_HERMITE) {
        set_error("linearization must be one of the pss_linearization values");
        return PSS_EINVAL;
    }
    if (p->model != PSS_MODEL_LINEAR) {
        if (p->linearization == PSS_LIN_UNSCENTED &&
            !(isfinite(p->ut_kappa) && p->ut_kappa >= 0.0)) {
            set_error("the unscented rule needs a finite ut_kappa >= 0 (positive weights)");
            return PSS_EINVAL;
        }
        RuleHost r;
        if (p->linearization == PSS_LIN_GAUSS_HERMITE && !rule_host(p, p->nx, r))
            return PSS_EINVAL;
    }
    if (p->scan_elems < 0 || p->scan_elems > 256) {
        set_error("scan_elems must be in 0..256");
        return PSS_EINVAL;
    }
    if (p->model == PSS_MODEL_CT_BEARINGS) {
        if (!(p->dt > 0.0) || !isfinite(p->theta[0]) || !isfinite(p->theta[1]) ||
            !isfinite(p->theta[2])) {
            set_error("coordinated-turn model needs dt > 0 and a finite theta");
            return PSS_EINVAL;
        }
    }
    if (p->model == PSS_MODEL_RICKER_POISSON &&
        !(isfinite(p->theta[0]) && isfinite(p->theta[1]) && isfinite(p->theta[2]))) {
        set_error("Ricker-Poisson model needs a finite theta");
        return PSS_EINVAL;
    }
    return PSS_OK;
}

static Ctx make_ctx(const pss_problem *p, hipStream_t s)
{
    Ctx c;
    c.p = p;
    c.B = p->B;
    c.T_y = p->y_off_host[p->B];
    c.T_x = c.T_y + p->B;
    c.s = s;
    return c;
}

static bool gamma_ok(const pss_gamma *g)
{
    return g && g->F && g->c && g->SL && g->H && g->d && g->SO &&
           (g->stride == 0 || g->stride == 1);
}

static int check_ws(const Ctx &c, int op, const void *ws, size_t ws_bytes)
{
    size_t need = 0;
    dispatch(c.p, [&](auto tag) {
        using I = typename decltype(tag)::I;
        need = I::ws_size(c, op);
        return 0;
    });
    if (ws_bytes < need || (need > 0 && !ws)) {
        set_error("workspace too small: need " + std::to_string(need) + " bytes");
        return PSS_EWORKSPACE;
    }
    return PSS_OK;
}

// identity of a checkpoint: FNV-1a over what fixes the filter pass it
// stores (model, dimensions, dtype, batch offsets, model constants, the
// linearisation, launch shape, level)
static uint64_t ckpt_tag(const pss_problem *p, int32_t level)
{
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](const void *d, size_t n) {
        const unsigned char *b = static_cast<const unsigned char *>(d);
        for (size_t i = 0; i < n; ++i) {
            h ^= b[i];
            h *= 1099511628211ull;
        }
    };
    const int32_t ints[] = {p->model, p->dtype, p->nx, p->ny, p->B, p->scan_threads,
                            p->scan_elems, p->linearization, p->form, p->gh_order, level};
    mix(ints, sizeof ints);
    mix(p->y_off_host, sizeof(int64_t) * ((size_t)p->B + 1));
    const double dbl[] = {p->dt, p->theta[0], p->theta[1], p->theta[2], p->sensors[0],
                          p->sensors[1], p->sensors[2], p->sensors[3], p->ut_kappa};
    mix(dbl, sizeof dbl);
    return h;
}

static size_t ckpt_need(const Ctx &c, int level)
{
    size_t need = 0;
    dispatch(c.p, [&](auto tag) {
        using I = typename decltype(tag)::I;
        need = I::ckpt_bytes(c, level);
        return 0;
    });
    return need;
}

// a checkpoint about to be filled (for_fill) or consumed
static int check_ckpt(const Ctx &c, const pss_ckpt *ck, bool for_fill)
{
    if (!ck)
        return PSS_OK;
    if (c.p->form != PSS_FORM_SQRT) {
        set_error("checkpoints are defined for the square-root form only");
        return PSS_EUNSUPPORTED;
    }
    if (ck->level < 0 || !ck->buf) {
        set_error("checkpoint: negative level or null buffer");
        return PSS_EINVAL;
    }
    const size_t need = ckpt_need(c, ck->level);
    if (ck->bytes < need) {
        set_error("checkpoint buffer too small: need " + std::to_string(need) + " bytes");
        return PSS_EWORKSPACE;
    }
    if (!for_fill && ck->tag != ckpt_tag(c.p, ck->level)) {
        set_error("checkpoint was filled for another problem, level or launch shape");
        return PSS_EINVAL;
    }
    return PSS_OK;
}

} // namespace pss

using namespace pss;

// entry points of the square-root form only
static int need_sqrt(const pss_problem *p, const char *what)
{
    if (p->form != PSS_FORM_SQRT) {
        set_error(std::string(what) + " is defined for the square-root form only");
        return PSS_EUNSUPPORTED;
    }
    return PSS_OK;
}

#define PSS_GUARD(expr)                                                                          \
    do {                                                                                         \
        try {                                                                                    \
            return (expr);                                                                       \
        } catch (const std::exception &ex) {                                                     \
            set_error(ex.what());                                                                \
            return PSS_EINVAL;                                                                   \
        } catch (...) {                                                                          \
            set_error("unknown exception");                                                      \
            return PSS_EINVAL;                                                                   \
        }                                                                                        \
    } while (0)

extern "C" {

const char *pss_last_error(void) { return g_last_error.c_str(); }

const char *pss_version(void) { return "pss 0.1 (gfx950)"; }

int pss_kernel_timing(int32_t enable)
{
    g_kt_on.store(enable != 0);
    return PSS_OK;
}

int64_t pss_kernel_times(char *buf, size_t cap)
{
    try {
        // a NULL buffer only asks for the size: the records stay
        const bool take = buf != nullptr;
        std::vector<KRec> recs;
        {
            std::lock_guard<std::mutex> lk(g_kt_mu);
            if (take)
                recs.swap(g_kt_recs);
            else
                recs = g_kt_recs;
        }
        std::map<std::pair<std::string, int>, std::pair<int64_t, double>> acc;
        int rc = PSS_OK;
        for (const KRec &r : recs) {
            float ms = 0.f;
            if (rc == PSS_OK && (rc = hip_check(hipEventSynchronize(r.b), "kernel timing sync")) ==
                                    PSS_OK)
                rc = hip_check(hipEventElapsedTime(&ms, r.a, r.b), "kernel timing elapsed");
            auto &v = acc[{r.key, r.level}];
            v.first += 1;
            v.second += ms;
            if (take) {
                kt_release(r.a);
                kt_release(r.b);
            }
        }
        if (rc != PSS_OK)
            return rc;
        std::string out;
        char line[192];
        for (const auto &kv : acc) {
            snprintf(line, sizeof line, "%s %d %lld %.6f\n", kv.first.first.c_str(), kv.first.second,
                     (long long)kv.second.first, kv.second.second);
            out += line;
        }
        if (buf && cap > 0) {
            const size_t n = std::min(cap - 1, out.size());
            memcpy(buf, out.data(), n);
            buf[n] = 0;
        }
        return (int64_t)out.size() + 1;
    } catch (...) {
        set_error("exception in pss_kernel_times");
        return PSS_EINVAL;
    }
}

int pss_validate(const pss_problem *p)
{
    PSS_GUARD(validate(p));
}

size_t pss_workspace_size(const pss_problem *p, int32_t op)
{
    try {
        if (validate(p) != PSS_OK)
            return 0;
        if (op == PSS_OP_LOGLIK_GRAD_IFT)
            return p->model == PSS_MODEL_CT_BEARINGS ? ift_ws_size(p) : 0;
        const Ctx c = make_ctx(p, nullptr);
        size_t n = 0;
        dispatch(p, [&](auto tag) {
            using I = typename decltype(tag)::I;
            n = I::ws_size(c, op);
            return 0;
        });
        return n;
    } catch (...) {
        set_error("exception in pss_workspace_size");
        return 0;
    }
}

int pss_slr_linearize(const pss_problem *p, const void *m_nom, const void *N_nom, const void *y,
                      const pss_gamma *out, hipStream_t stream)
{
    PSS_GUARD(([&]() -> int {
        int rc = validate(p);
        if (rc)
            return rc;
        if (p->model == PSS_MODEL_LINEAR) {
            set_error("slr_linearize needs a nonlinear model");
            return PSS_EUNSUPPORTED;
        }
        if (!m_nom || !N_nom || !y || !gamma_ok(out) || out->stride != 1) {
            set_error("slr_linearize: null buffer or output stride != 1");
            return PSS_EINVAL;
        }
        const Ctx c = make_ctx(p, stream);
        return dispatch(p, [&](auto tag) {
            using I = typename decltype(tag)::I;
            return I::slr(c, m_nom, N_nom, y, out);
        });
    }()));
}

int pss_sqrt_filter_elements(const pss_problem *p, const pss_gamma *g, const void *y,
                             const pss_felem *out, hipStream_t stream)
{
    PSS_GUARD(([&]() -> int {
        int rc = validate(p);
        if (rc)
            return rc;
        if ((rc = need_sqrt(p, "sqrt_filter_elements")))
            return rc;
        if (!gamma_ok(g) || !y || !out || !out->A || !out->b || !out->U || !out->eta ||
            !out->Z) {
            set_error("sqrt_filter_elements: null buffer");
            return PSS_EINVAL;
        }
        const Ctx c = make_ctx(p, stream);
        return dispatch(p, [&](auto tag) {
            using I = typename decltype(tag)::I;
            return I::felem(c, g, y, out);
        });
    }()));
}

int pss_sqrt_filter_scan(const pss_problem *p, const pss_felem *el, void *m_f, void *N_f,
                         void *ws, size_t ws_bytes, hipStream_t stream)
{
    PSS_GUARD(([&]() -> int {
        int rc = validate(p);
        if (rc)
            return rc;
        if ((rc = need_sqrt(p, "sqrt_filter_scan")))
            return rc;
        if (!el || !el->A || !el->b || !el->U || !el->eta || !el->Z || !m_f || !N_f) {
            set_error("sqrt_filter_scan: null buffer");
            return PSS_EINVAL;
        }
        const Ctx c = make_ctx(p, stream);
        if ((rc = check_ws(c, PSS_OP_FILTER_SCAN, ws, ws_bytes)))
            return rc;
        return dispatch(p, [&](auto tag) {
            using I = typename decltype(tag)::I;
            return I::fscan(c, el, m_f, N_f, ws);
        });
    }()));
}

int pss_sqrt_smoother_scan(const pss_problem *p, const pss_gamma *g, const void *m_f,
                           const void *N_f, void *m_s, void *N_s, void *ws, size_t ws_bytes,
                           hipStream_t stream)
{
    PSS_GUARD(([&]() -> int {
        int rc = validate(p);
        if (rc)
            return rc;
        if ((rc = need_sqrt(p, "sqrt_smoother_scan")))
            return rc;
        if (!gamma_ok(g) || !m_f || !N_f || !m_s || !N_s) {
            set_error("sqrt_smoother_scan: null buffer");
            return PSS_EINVAL;
        }
        const Ctx c = make_ctx(p, stream);
        if ((rc = check_ws(c, PSS_OP_SMOOTHER_SCAN, ws, ws_bytes)))
            return rc;
        return dispatch(p, [&](auto tag) {
            using I = typename decltype(tag)::I;
            return I::sscan(c, g, m_f, N_f, m_s, N_s, ws);
        });
    }()));
}

int pss_ipls_iterate(const pss_problem *p, const pss_gamma *g, const void *y, int32_t n_iter,
                     void *m_nom, void *N_nom, void *m_f, void *N_f, void *ws, size_t ws_bytes,
                     hipStream_t stream)
{
    PSS_GUARD(([&]() -> int {
        int rc = validate(p);
        if (rc)
            return rc;
        if (!y || !m_nom || !N_nom || n_iter < 0 || ((m_f == nullptr) != (N_f == nullptr))) {
            set_error("ipls_iterate: null buffer or negative n_iter");
            return PSS_EINVAL;
        }
        if (p->model == PSS_MODEL_LINEAR ? !gamma_ok(g) : g != nullptr) {
            set_error("ipls_iterate: a linear model needs g, a nonlinear model takes g = NULL");
            return PSS_EINVAL;
        }
        const Ctx c = make_ctx(p, stream);
        if ((rc = check_ws(c, PSS_OP_IPLS, ws, ws_bytes)))
            return rc;
        return dispatch(p, [&](auto tag) {
            using I = typename decltype(tag)::I;
            return I::ipls(c, g, y, n_iter, m_nom, N_nom, m_f, N_f, ws);
        });
    }()));
}

size_t pss_ckpt_size(const pss_problem *p, int32_t level)
{
    try {
        if (validate(p) != PSS_OK)
            return 0;
        if (level < 0) {
            set_error("checkpoint level must be >= 0");
            return 0;
        }
        return ckpt_need(make_ctx(p, nullptr), level);
    } catch (...) {
        set_error("exception in pss_ckpt_size");
        return 0;
    }
}

int pss_loglik(const pss_problem *p, const pss_gamma *g, const void *m_nom, const void *N_nom,
               const void *y, double *ll, pss_ckpt *ckpt, void *ws, size_t ws_bytes,
               hipStream_t stream)
{
    PSS_GUARD(([&]() -> int {
        int rc = validate(p);
        if (rc)
            return rc;
        if (!y || !ll) {
            set_error("loglik: null buffer");
            return PSS_EINVAL;
        }
        if (p->model == PSS_MODEL_LINEAR ? !gamma_ok(g) : (!m_nom || !N_nom)) {
            set_error("loglik: a linear model needs g, a nonlinear model needs the nominal");
            return PSS_EINVAL;
        }
        const Ctx c = make_ctx(p, stream);
        if ((rc = check_ws(c, PSS_OP_LOGLIK, ws, ws_bytes)))
            return rc;
        if ((rc = check_ckpt(c, ckpt, true)))
            return rc;
        rc = dispatch(p, [&](auto tag) {
            using I = typename decltype(tag)::I;
            return I::loglik(c, g, m_nom, N_nom, y, ll, ckpt, ws);
        });
        if (rc == PSS_OK && ckpt)
            ckpt->tag = ckpt_tag(p, ckpt->level);
        return rc;
    }()));
}

int pss_loglik_grad(const pss_problem *p, const void *m_nom, const void *N_nom, const void *y,
                    const double *ll_bar, const pss_ckpt *ckpt, double *ll, double *grad,
                    double *theta_bar, void *ws, size_t ws_bytes, hipStream_t stream)
{
    PSS_GUARD(([&]() -> int {
        int rc = validate(p);
        if (rc)
            return rc;
        if ((rc = need_sqrt(p, "loglik_grad")))
            return rc;
        if (p->model != PSS_MODEL_CT_BEARINGS) {
            set_error("loglik_grad: theta is defined for the coordinated-turn model");
            return PSS_EUNSUPPORTED;
        }
        if (!m_nom || !N_nom || !y || !ll) {
            set_error("loglik_grad: null buffer");
            return PSS_EINVAL;
        }
        const Ctx c = make_ctx(p, stream);
        if ((rc = check_ws(c, PSS_OP_LOGLIK_GRAD, ws, ws_bytes)))
            return rc;
        if ((rc = check_ckpt(c, ckpt, false)))
            return rc;
        return dispatch(p, [&](auto tag) {
            using I = typename decltype(tag)::I;
            return I::loglik_grad(c, m_nom, N_nom, y, ll_bar, ckpt, ll, grad, theta_bar, ws);
        });
    }()));
}

int pss_loglik_vjp(const pss_problem *p, const pss_gamma *g, const void *m_nom,
                   const void *N_nom, const void *y, const double *ll_bar, const pss_ckpt *ckpt,
                   double *ll, const pss_gamma *g_bar, void *m0_bar, void *N0_bar, void *ws,
                   size_t ws_bytes, hipStream_t stream)
{
    PSS_GUARD(([&]() -> int {
        int rc = validate(p);
        if (rc)
            return rc;
        if ((rc = need_sqrt(p, "loglik_vjp")))
            return rc;
        if (!y || !ll || !gamma_ok(g_bar) || g_bar->stride != 1 ||
            ((m0_bar == nullptr) != (N0_bar == nullptr))) {
            set_error("loglik_vjp: null buffer, g_bar stride != 1, or only one of m0_bar, "
                      "N0_bar");
            return PSS_EINVAL;
        }
        if (p->model == PSS_MODEL_LINEAR ? !gamma_ok(g) : (!m_nom || !N_nom || g != nullptr)) {
            set_error("loglik_vjp: a linear model needs g, a nonlinear model the nominal and "
                      "g = NULL");
            return PSS_EINVAL;
        }
        const Ctx c = make_ctx(p, stream);
        if ((rc = check_ws(c, PSS_OP_LOGLIK_VJP, ws, ws_bytes)))
            return rc;
        if ((rc = check_ckpt(c, ckpt, false)))
            return rc;
        return dispatch(p, [&](auto tag) {
            using I = typename decltype(tag)::I;
            return I::loglik_vjp(c, g, m_nom, N_nom, y, ll_bar, ckpt, ll, g_bar, m0_bar, N0_bar,
                                 ws);
        });
    }()));
}

int pss_nan_status(const pss_problem *p, const void *m, const void *N, int32_t marg_bit,
                   const double *ll, int32_t ll_bit, int32_t *status, hipStream_t stream)
{
    PSS_GUARD(([&]() -> int {
        int rc = validate(p);
        if (rc)
            return rc;
        if (!status || ((m == nullptr) != (N == nullptr)) || (!m && !ll)) {
            set_error("nan_status: null status, only one of m, N, or nothing to check");
            return PSS_EINVAL;
        }
        const Ctx c = make_ctx(p, stream);
        return launch_nan_status(c, m, N, ll, marg_bit, ll_bit, status);
    }()));
}

int pss_score_fisher(const pss_problem *p, const void *m_nom, const void *N_nom, const void *y,
                     const double *ll_bar, double *ll, double *grad, double *theta_bar,
                     void *ws, size_t ws_bytes, hipStream_t stream)
{
    PSS_GUARD(([&]() -> int {
        int rc = validate(p);
        if (rc)
            return rc;
        if ((rc = need_sqrt(p, "score_fisher")))
            return rc;
        if (p->model != PSS_MODEL_CT_BEARINGS) {
            set_error("score_fisher: theta is defined for the coordinated-turn model");
            return PSS_EUNSUPPORTED;
        }
        if (!m_nom || !N_nom || !y || !ll) {
            set_error("score_fisher: null buffer");
            return PSS_EINVAL;
        }
        const Ctx c = make_ctx(p, stream);
        if ((rc = check_ws(c, PSS_OP_SCORE_FISHER, ws, ws_bytes)))
            return rc;
        return dispatch(p, [&](auto tag) {
            using I = typename decltype(tag)::I;
            return I::score_fisher(c, m_nom, N_nom, y, ll_bar, ll, grad, theta_bar, ws);
        });
    }()));
}

int pss_sequential_smoother(const pss_problem *p, const pss_gamma *g, const void *y,
                            int32_t n_iter, void *m_nom, void *N_nom, void *m_f, void *N_f,
                            void *ws, size_t ws_bytes, hipStream_t stream)
{
    PSS_GUARD(([&]() -> int {
        int rc = validate(p);
        if (rc)
            return rc;
        if (!y || !m_nom || !N_nom || n_iter < 0 || ((m_f == nullptr) != (N_f == nullptr))) {
            set_error("sequential_smoother: null buffer or negative n_iter");
            return PSS_EINVAL;
        }
        if (p->model == PSS_MODEL_LINEAR ? !gamma_ok(g) : g != nullptr) {
            set_error("sequential_smoother: a linear model needs g, a nonlinear model takes g = "
                      "NULL");
            return PSS_EINVAL;
        }
        const Ctx c = make_ctx(p, stream);
        if ((rc = check_ws(c, PSS_OP_SEQUENTIAL, ws, ws_bytes)))
            return rc;
        return dispatch(p, [&](auto tag) {
            using I = typename decltype(tag)::I;
            return I::sequential(c, g, y, n_iter, m_nom, N_nom, m_f, N_f, ws);
        });
    }()));
}

} // extern "C"
