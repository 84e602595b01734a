// Host side of the persistent batched IPLS pass and its autotuner.
#include <math.h>
#include <stdio.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "persistent.hpp"

namespace pss {

namespace {

struct Shape {
    int T = 0;   // block threads
    int E_f = 0; // filter elements per thread
    int E_s = 0; // smoother elements per thread
};

// ---- autotune cache (host, mutex-guarded) ---------------------------------
std::mutex g_tune_mu;
std::map<std::string, Shape> g_tune;
bool g_tune_loaded = false;

std::string sig_of(const pss_group *gs, int ng)
{
    std::string s = gs[0].p->dtype == PSS_F64 ? "f64" : "f32";
    for (int i = 0; i < ng; ++i) {
        const pss_problem *p = gs[i].p;
        const int64_t T_y = p->y_off_host[p->B];
        int lg = 0;
        while ((int64_t(1) << lg) < T_y)
            ++lg;
        s += "|" + std::to_string(p->model) + ":" + std::to_string(p->nx) + ":B" +
             std::to_string(p->B) + ":L" + std::to_string(lg);
    }
    return s;
}

void load_cache_file(const char *path)
{
    FILE *f = fopen(path, "r");
    if (!f)
        return;
    char key[512];
    int T, Ef, Es;
    // one entry per line: "key" T E_f E_s
    while (fscanf(f, " \"%511[^\"]\" %d %d %d", key, &T, &Ef, &Es) == 4) {
        Shape sh;
        sh.T = T;
        sh.E_f = Ef;
        sh.E_s = Es;
        g_tune[key] = sh;
    }
    fclose(f);
}

void save_cache_file(const char *path)
{
    FILE *f = fopen(path, "w");
    if (!f)
        return;
    for (auto &kv : g_tune)
        fprintf(f, "\"%s\" %d %d %d\n", kv.first.c_str(), kv.second.T, kv.second.E_f,
                kv.second.E_s);
    fclose(f);
}

bool lookup(const std::string &key, Shape &sh)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!g_tune_loaded) {
        g_tune_loaded = true;
        const char *env = getenv("PSS_TUNE_CACHE");
        if (env)
            load_cache_file(env);
    }
    auto it = g_tune.find(key);
    if (it == g_tune.end())
        return false;
    sh = it->second;
    return true;
}

int kind_of(const pss_problem *p)
{
    if (p->model == PSS_MODEL_CT_BEARINGS && p->nx == 5 && p->ny == 2)
        return kGroupCT;
    if (p->model == PSS_MODEL_LINEAR && p->nx == 4 && p->ny == 2)
        return kGroupLinear4;
    return 0;
}

int64_t tiles_of(const pss_problem *p, int64_t TS, int extra)
{
    int64_t t = 0;
    for (int b = 0; b < p->B; ++b)
        t += (p->y_off_host[b + 1] - p->y_off_host[b] + extra + TS - 1) / TS;
    return t;
}

template <typename T>
struct Layout {
    // per group
    int64_t *tile_f[kMaxGroups], *tile_s[kMaxGroups];
    T *nom2[kMaxGroups], *mf[kMaxGroups], *fstash[kMaxGroups], *gstash[kMaxGroups];
    T *sstash[kMaxGroups], *pre_f[kMaxGroups], *pre_s[kMaxGroups];
    int *flags;
    int64_t nflags;
    int *counter;
    int *error;
    int64_t ntf[kMaxGroups], nts[kMaxGroups];
};

template <typename T>
Layout<T> carve(Carver &cv, const pss_group *gs, int ng, const Shape &sh)
{
    Layout<T> L{};
    int64_t nflags = 0;
    for (int i = 0; i < ng; ++i) {
        const pss_problem *p = gs[i].p;
        const int nx = p->nx;
        const int64_t T_y = p->y_off_host[p->B], T_x = T_y + p->B;
        const int P = nx * (nx + 1) / 2;
        const int NEf = nx * nx + nx + P + nx + P, NEs = nx * nx + nx + P;
        L.ntf[i] = tiles_of(p, (int64_t)sh.T * sh.E_f, 0);
        L.nts[i] = tiles_of(p, (int64_t)sh.T * sh.E_s, 1);
        L.tile_f[i] = cv.take<int64_t>(p->B + 1);
        L.tile_s[i] = cv.take<int64_t>(p->B + 1);
        L.nom2[i] = cv.take<T>((size_t)(nx + P) * T_x);
        L.mf[i] = cv.take<T>((size_t)(nx + P) * T_x);
        L.fstash[i] = cv.take<T>((size_t)NEf * T_y);
        L.gstash[i] = kind_of(p) == kGroupCT ? cv.take<T>((size_t)(nx * nx + nx + P) * T_y)
                                             : nullptr;
        L.sstash[i] = cv.take<T>((size_t)NEs * T_x);
        L.pre_f[i] = cv.take<T>((size_t)(nx + P) * L.ntf[i]);
        L.pre_s[i] = cv.take<T>((size_t)(nx + P) * L.nts[i]);
        nflags += 2 * L.ntf[i] + L.nts[i];
    }
    L.nflags = nflags;
    L.flags = cv.take<int>((size_t)nflags + 2);
    L.counter = L.flags ? L.flags + nflags : nullptr;
    L.error = L.flags ? L.flags + nflags + 1 : nullptr;
    return L;
}

Shape default_shape(const pss_group *gs, int ng)
{
    Shape sh;
    const bool f64 = gs[0].p->dtype == PSS_F64;
    sh.T = gs[0].p->scan_threads > 0 ? gs[0].p->scan_threads : (f64 ? 128 : 256);
    sh.E_f = gs[0].p->scan_elems > 0 ? gs[0].p->scan_elems : 4;
    sh.E_s = sh.E_f;
    if (gs[0].p->scan_threads <= 0 && gs[0].p->scan_elems <= 0) {
        Shape tuned;
        if (lookup(sig_of(gs, ng), tuned))
            sh = tuned;
    }
    return sh;
}

int validate_groups(const pss_group *gs, int ng)
{
    if (!gs || ng < 1 || ng > kMaxGroups) {
        set_error("batched: need 1..4 groups");
        return PSS_EINVAL;
    }
    for (int i = 0; i < ng; ++i) {
        const int rc = pss_validate(gs[i].p);
        if (rc)
            return rc;
        const pss_problem *p = gs[i].p;
        if (!kind_of(p)) {
            set_error("batched: groups must be CT (nx 5, ny 2) or linear (nx 4, ny 2)");
            return PSS_EUNSUPPORTED;
        }
        if (p->form != PSS_FORM_SQRT) {
            set_error("batched: the persistent pass is defined for the square-root form only");
            return PSS_EUNSUPPORTED;
        }
        if (p->model != PSS_MODEL_LINEAR && p->linearization != PSS_LIN_CUBATURE &&
            p->linearization != PSS_LIN_TAYLOR) {
            set_error("batched: the persistent pass fuses the cubature or Taylor linearisation "
                      "only");
            return PSS_EUNSUPPORTED;
        }
        if (p->dtype != gs[0].p->dtype) {
            set_error("batched: all groups need the same dtype");
            return PSS_EINVAL;
        }
        if (p->scan_threads != gs[0].p->scan_threads || p->scan_elems != gs[0].p->scan_elems) {
            set_error("batched: all groups need the same launch shape overrides");
            return PSS_EINVAL;
        }
        if (!gs[i].y || !gs[i].m_nom || !gs[i].N_nom) {
            set_error("batched: null y or nominal");
            return PSS_EINVAL;
        }
        if (p->model == PSS_MODEL_LINEAR) {
            const pss_gamma *g = gs[i].g;
            if (!g || !g->F || !g->c || !g->SL || !g->H || !g->d || !g->SO ||
                (g->stride != 0 && g->stride != 1)) {
                set_error("batched: a linear group needs its parameters");
                return PSS_EINVAL;
            }
        } else if (gs[i].g) {
            set_error("batched: a CT group takes g = NULL");
            return PSS_EINVAL;
        }
    }
    return PSS_OK;
}

template <typename T>
size_t ws_bytes_for(const pss_group *gs, int ng, const Shape &sh)
{
    Carver cv{nullptr};
    carve<T>(cv, gs, ng, sh);
    return cv.used;
}

template <typename T>
int run(const pss_group *gs, int ng, int n_iter, int32_t *status, void *ws, size_t ws_bytes,
        hipStream_t s, const Shape &sh)
{
    if (ws_bytes < ws_bytes_for<T>(gs, ng, sh) || !ws) {
        set_error("batched: workspace too small");
        return PSS_EWORKSPACE;
    }
    if (sh.T != 64 && sh.T != 128 && sh.T != 256) {
        set_error("batched: block threads must be 64, 128 or 256");
        return PSS_EINVAL;
    }
    Carver cv{static_cast<char *>(ws)};
    Layout<T> L = carve<T>(cv, gs, ng, sh);
    PArgs<T> a{};
    a.n_groups = ng;
    a.counter = L.counter;
    a.error = status ? status : L.error;
    a.spin_limit = 1 << 24;
    int64_t item = 0, flag_pos = 0;
    int b_all = 0;
    for (int i = 0; i < ng; ++i) {
        const pss_problem *p = gs[i].p;
        Ctx c{p, p->B, p->y_off_host[p->B], p->y_off_host[p->B] + p->B, s};
        ScanShape plan;
        plan.L = 1;
        plan.T[0] = sh.T;
        plan.E[0] = sh.E_f;
        int rc = launch_plan(c, plan, 0, &L.tile_f[i]);
        if (rc)
            return rc;
        plan.E[0] = sh.E_s;
        if ((rc = launch_plan(c, plan, 1, &L.tile_s[i])))
            return rc;
        PGroup<T> &G = a.g[i];
        G.kind = kind_of(p);
        G.B = p->B;
        G.seq0 = b_all;
        b_all += p->B;
        G.E_f = sh.E_f;
        G.E_s = sh.E_s;
        G.taylor = p->linearization == PSS_LIN_TAYLOR ? 1 : 0;
        G.stage_f = scan_stage(65, 20, sh.T, sh.E_f, sizeof(T));
        G.stage_s = scan_stage(45, 20, sh.T, sh.E_s, sizeof(T));
        G.y_off = p->y_off;
        G.T_y = c.T_y;
        G.T_x = c.T_x;
        G.y = static_cast<const T *>(gs[i].y);
        G.m0 = static_cast<const T *>(p->m0);
        G.N0 = static_cast<const T *>(p->N0);
        G.mf = L.mf[i];
        G.Nf = L.mf[i] + (int64_t)p->nx * c.T_x;
        G.fstash = L.fstash[i];
        G.gstash = L.gstash[i];
        G.sstash = L.sstash[i];
        G.pre_f = L.pre_f[i];
        G.pre_s = L.pre_s[i];
        G.tile_f = L.tile_f[i];
        G.tile_s = L.tile_s[i];
        G.ntiles_f = L.ntf[i];
        G.ntiles_s = L.nts[i];
        G.item_f0 = item;
        item += L.ntf[i];
        G.flag_f = L.flags + flag_pos;
        G.done_f = L.flags + flag_pos + L.ntf[i];
        G.flag_s = L.flags + flag_pos + 2 * L.ntf[i];
        flag_pos += 2 * L.ntf[i] + L.nts[i];
        if (p->model == PSS_MODEL_LINEAR) {
            const pss_gamma *g = gs[i].g;
            G.gF = static_cast<const T *>(g->F);
            G.gc = static_cast<const T *>(g->c);
            G.gSL = static_cast<const T *>(g->SL);
            G.gH = static_cast<const T *>(g->H);
            G.gd = static_cast<const T *>(g->d);
            G.gSO = static_cast<const T *>(g->SO);
            G.gstride = g->stride;
        } else {
            const CTHost h = ct_host(p);
            G.ct.dt = (T)h.dt;
            G.ct.s1x = (T)h.s1x;
            G.ct.s1y = (T)h.s1y;
            G.ct.s2x = (T)h.s2x;
            G.ct.s2y = (T)h.s2y;
            G.ct.sigma = (T)h.sigma;
            for (int r = 0; r < 5; ++r)
                for (int q = 0; q < 5; ++q)
                    G.ct.LQ[r][q] = (T)h.LQ[r][q];
        }
    }
    for (int i = 0; i < ng; ++i) {
        a.g[i].item_s0 = item;
        item += L.nts[i];
    }
    a.total_items = item;
    // time-major order when at least a quarter of its (sequence, tile) slots
    // hold a tile
    {
        int64_t maxt_f = 0, maxt_s = 0, nt = 0;
        const int64_t TSf = (int64_t)sh.T * sh.E_f, TSs = (int64_t)sh.T * sh.E_s;
        for (int i = 0; i < ng; ++i) {
            const pss_problem *p = gs[i].p;
            for (int b = 0; b < p->B; ++b) {
                const int64_t n = p->y_off_host[b + 1] - p->y_off_host[b];
                maxt_f = std::max(maxt_f, (n + TSf - 1) / TSf);
                maxt_s = std::max(maxt_s, (n + 1 + TSs - 1) / TSs);
            }
        }
        nt = item;
        const int64_t slots = (maxt_f + maxt_s) * (int64_t)b_all;
        a.rr = b_all > 1 && slots <= 4 * nt;
        a.B_all = b_all;
        a.n_f_items = maxt_f * (int64_t)b_all;
        if (a.rr)
            a.total_items = slots;
    }

    auto kern = k_ipls_persistent<T>;
    // sized for the largest objects (coordinated-turn filter / smoother)
    size_t lds = scan_lds(65, 20, sh.T, sh.E_f, sizeof(T), scan_stage(65, 20, sh.T, sh.E_f, sizeof(T)));
    lds = std::max(lds, scan_lds(45, 20, sh.T, sh.E_s, sizeof(T),
                                 scan_stage(45, 20, sh.T, sh.E_s, sizeof(T))));
    int rc = hip_check(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
                       "hipFuncSetAttribute");
    if (rc)
        return rc;
    int dev = 0, ncu = 0, per_cu = 0;
    if ((rc = hip_check(hipGetDevice(&dev), "hipGetDevice")))
        return rc;
    if ((rc = hip_check(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev),
                        "hipDeviceGetAttribute")))
        return rc;
    if ((rc = hip_check(hipOccupancyMaxActiveBlocksPerMultiprocessor(
                            &per_cu, reinterpret_cast<const void *>(kern), sh.T, lds),
                        "hipOccupancyMaxActiveBlocksPerMultiprocessor")))
        return rc;
    int64_t grid = (int64_t)ncu * std::max(per_cu, 1);
    grid = std::min<int64_t>(grid, a.total_items);
    grid = std::max<int64_t>(grid, 1);

    if (status) {
        hipLaunchKernelGGL(k_clear_ints, dim3(1), dim3(64), 0, s, status, (int64_t)1);
    }
    for (int it = 0; it < n_iter; ++it) {
        // pass it reads buffer it % 2 and writes the other (buffer 0 is the caller's)
        for (int i = 0; i < ng; ++i) {
            const pss_problem *p = gs[i].p;
            const int64_t T_x = p->y_off_host[p->B] + p->B;
            T *m_a = static_cast<T *>(gs[i].m_nom), *N_a = static_cast<T *>(gs[i].N_nom);
            T *m_b = L.nom2[i], *N_b = L.nom2[i] + (int64_t)p->nx * T_x;
            const bool even = (it % 2) == 0;
            a.g[i].nom_in_m = even ? m_a : m_b;
            a.g[i].nom_in_N = even ? N_a : N_b;
            a.g[i].nom_out_m = even ? m_b : m_a;
            a.g[i].nom_out_N = even ? N_b : N_a;
        }
        const int64_t nclr = L.nflags + (status ? 1 : 2);
        hipLaunchKernelGGL(k_clear_ints, dim3((unsigned)std::min<int64_t>((nclr + 255) / 256, 1024)),
                           dim3(256), 0, s, L.flags, nclr);
        {
            KTime kt(s, "persistent_pass", "", 0);
            hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(sh.T), lds, s, a);
        }
        if ((rc = hip_check(hipGetLastError(), "persistent pass launch")))
            return rc;
    }
    if (n_iter % 2 == 1) {
        for (int i = 0; i < ng; ++i) {
            const pss_problem *p = gs[i].p;
            const int64_t T_x = p->y_off_host[p->B] + p->B;
            const int nx = p->nx;
            hipLaunchKernelGGL(k_copy<T>, dim3(256), dim3(256), 0, s, L.nom2[i],
                               static_cast<T *>(gs[i].m_nom), (int64_t)nx * T_x);
            hipLaunchKernelGGL(k_copy<T>, dim3(256), dim3(256), 0, s,
                               L.nom2[i] + (int64_t)nx * T_x, static_cast<T *>(gs[i].N_nom),
                               (int64_t)(nx * (nx + 1) / 2) * T_x);
        }
        if ((rc = hip_check(hipGetLastError(), "copy launch")))
            return rc;
    }
    return PSS_OK;
}

size_t max_ws(const pss_group *gs, int ng, const std::vector<Shape> &cands)
{
    size_t m = 0;
    for (const Shape &sh : cands)
        m = std::max(m, gs[0].p->dtype == PSS_F64 ? ws_bytes_for<double>(gs, ng, sh)
                                                  : ws_bytes_for<float>(gs, ng, sh));
    return m;
}

std::vector<Shape> candidates(bool f64)
{
    std::vector<Shape> c;
    const int Ts[3] = {64, 128, 256};
    const int Es[4] = {1, 2, 4, 8};
    for (int T : Ts) {
        if (f64 && T == 256)
            continue; // FP64 tiles of 256 threads exceed the LDS budget of two blocks per CU
        for (int Ef : Es)
            for (int Es_ : Es) {
                if (Es_ != Ef && Es_ != 2 * Ef && 2 * Es_ != Ef)
                    continue;
                Shape sh;
                sh.T = T;
                sh.E_f = Ef;
                sh.E_s = Es_;
                c.push_back(sh);
            }
    }
    return c;
}

} // namespace

} // namespace pss

using namespace pss;

extern "C" {

size_t pss_batched_workspace_size(const pss_group *groups, int32_t n_groups)
{
    try {
        if (validate_groups(groups, n_groups))
            return 0;
        const Shape sh = default_shape(groups, n_groups);
        return groups[0].p->dtype == PSS_F64 ? ws_bytes_for<double>(groups, n_groups, sh)
                                             : ws_bytes_for<float>(groups, n_groups, sh);
    } catch (...) {
        set_error("exception in pss_batched_workspace_size");
        return 0;
    }
}

int pss_ipls_batched(const pss_group *groups, int32_t n_groups, int32_t n_iter, int32_t *status,
                     void *ws, size_t ws_bytes, hipStream_t stream)
{
    try {
        int rc = validate_groups(groups, n_groups);
        if (rc)
            return rc;
        if (n_iter < 0) {
            set_error("batched: negative n_iter");
            return PSS_EINVAL;
        }
        const Shape sh = default_shape(groups, n_groups);
        if (groups[0].p->dtype == PSS_F64)
            return run<double>(groups, n_groups, n_iter, status, ws, ws_bytes, stream, sh);
        return run<float>(groups, n_groups, n_iter, status, ws, ws_bytes, stream, sh);
    } catch (...) {
        set_error("exception in pss_ipls_batched");
        return PSS_EINVAL;
    }
}

size_t pss_autotune_workspace_size(const pss_group *groups, int32_t n_groups)
{
    try {
        if (validate_groups(groups, n_groups))
            return 0;
        const bool f64 = groups[0].p->dtype == PSS_F64;
        size_t nom = 0;
        for (int i = 0; i < n_groups; ++i) {
            const pss_problem *p = groups[i].p;
            const int64_t T_x = p->y_off_host[p->B] + p->B;
            nom += align256((size_t)(p->nx + p->nx * (p->nx + 1) / 2) * T_x * (f64 ? 8 : 4));
        }
        return max_ws(groups, n_groups, candidates(f64)) + nom;
    } catch (...) {
        set_error("exception in pss_autotune_workspace_size");
        return 0;
    }
}

int pss_autotune(const pss_group *groups, int32_t n_groups, void *ws, size_t ws_bytes,
                 const char *cache_path_host, int32_t *best_host, hipStream_t stream)
{
    try {
        int rc = validate_groups(groups, n_groups);
        if (rc)
            return rc;
        const bool f64 = groups[0].p->dtype == PSS_F64;
        const std::vector<Shape> cands = candidates(f64);
        const size_t need = pss_autotune_workspace_size(groups, n_groups);
        if (!ws || ws_bytes < need) {
            set_error("autotune: workspace too small");
            return PSS_EWORKSPACE;
        }
        // scratch nominal copies after the largest pass workspace
        const size_t base = max_ws(groups, n_groups, cands);
        Carver cv{static_cast<char *>(ws) + base};
        std::vector<pss_group> tmp(groups, groups + n_groups);
        std::vector<pss_problem> probs(n_groups);
        for (int i = 0; i < n_groups; ++i) {
            probs[i] = *groups[i].p;
            tmp[i].p = &probs[i];
            const int64_t T_x = probs[i].y_off_host[probs[i].B] + probs[i].B;
            const int64_t cnt = (int64_t)(probs[i].nx + probs[i].nx * (probs[i].nx + 1) / 2) * T_x;
            char *buf = f64 ? (char *)cv.take<double>((size_t)cnt) : (char *)cv.take<float>((size_t)cnt);
            tmp[i].m_nom = buf;
            tmp[i].N_nom = buf + (size_t)probs[i].nx * T_x * (f64 ? 8 : 4);
        }
        hipEvent_t e0, e1;
        if ((rc = hip_check(hipEventCreate(&e0), "hipEventCreate")))
            return rc;
        if ((rc = hip_check(hipEventCreate(&e1), "hipEventCreate"))) {
            (void)hipEventDestroy(e0);
            return rc;
        }
        auto reset = [&]() {
            for (int i = 0; i < n_groups; ++i) {
                const pss_problem *p = groups[i].p;
                const int64_t T_x = p->y_off_host[p->B] + p->B;
                const int64_t nm = (int64_t)p->nx * T_x, nN = (int64_t)(p->nx * (p->nx + 1) / 2) * T_x;
                if (f64) {
                    hipLaunchKernelGGL(k_copy<double>, dim3(256), dim3(256), 0, stream,
                                       (const double *)groups[i].m_nom, (double *)tmp[i].m_nom, nm);
                    hipLaunchKernelGGL(k_copy<double>, dim3(256), dim3(256), 0, stream,
                                       (const double *)groups[i].N_nom, (double *)tmp[i].N_nom, nN);
                } else {
                    hipLaunchKernelGGL(k_copy<float>, dim3(256), dim3(256), 0, stream,
                                       (const float *)groups[i].m_nom, (float *)tmp[i].m_nom, nm);
                    hipLaunchKernelGGL(k_copy<float>, dim3(256), dim3(256), 0, stream,
                                       (const float *)groups[i].N_nom, (float *)tmp[i].N_nom, nN);
                }
            }
        };
        float best_ms = 1e30f;
        Shape best = cands[0];
        for (const Shape &sh : cands) {
            float ms = 0.f;
            for (int rep = 0; rep < 2 && rc == PSS_OK; ++rep) {
                reset();
                if (rep == 1)
                    rc = hip_check(hipEventRecord(e0, stream), "hipEventRecord");
                if (!rc)
                    rc = f64 ? run<double>(tmp.data(), n_groups, 1, nullptr, ws, base, stream, sh)
                             : run<float>(tmp.data(), n_groups, 1, nullptr, ws, base, stream, sh);
                if (rep == 1 && !rc) {
                    rc = hip_check(hipEventRecord(e1, stream), "hipEventRecord");
                    if (!rc)
                        rc = hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
                    if (!rc)
                        rc = hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
                }
            }
            if (rc)
                break;
            if (ms < best_ms) {
                best_ms = ms;
                best = sh;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (rc)
            return rc;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tune_loaded = true;
            g_tune[sig_of(groups, n_groups)] = best;
            if (cache_path_host)
                save_cache_file(cache_path_host);
        }
        if (best_host) {
            best_host[0] = best.T;
            best_host[1] = best.E_f;
            best_host[2] = best.E_s;
        }
        return PSS_OK;
    } catch (...) {
        set_error("exception in pss_autotune");
        return PSS_EINVAL;
    }
}

} // extern "C"
