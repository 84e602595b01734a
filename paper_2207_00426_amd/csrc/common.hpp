// Declarations shared by the C-ABI unit and the per-dimension units.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <string>

#include "../../include/pss.h"

namespace pss {

constexpr int kMaxLevels = 8;

void set_error(const std::string &msg);
int hip_check(hipError_t e, const char *what);

// Optional per-launch kernel timing: while enabled (and the stream is not
// being captured), a KTime scope records a HIP event on the launch stream
// when it opens and another when it closes; pss_kernel_times() reads them.
struct KTime {
    hipStream_t s;
    const char *name, *phase;
    int level;
    hipEvent_t a = nullptr;
    KTime(hipStream_t s_, const char *name_, const char *phase_, int level_);
    ~KTime();
    KTime(const KTime &) = delete;
    KTime &operator=(const KTime &) = delete;
};

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// LDS of a scan tile of T threads folding E elements each: the tree holds NE
// values per thread; staged outputs (see apply_phase) NP values per element.
// Outputs are staged when that fits in the tree's space or in 48 KiB.
inline bool scan_stage(int NE, int NP, int T, int E, size_t esz)
{
    const size_t tree = (size_t)NE * T * esz, st = (size_t)NP * T * E * esz;
    return st <= tree || st <= 48 * 1024;
}
inline size_t scan_lds(int NE, int NP, int T, int E, size_t esz, bool stage)
{
    const size_t tree = (size_t)NE * T * esz, st = stage ? (size_t)NP * T * E * esz : 0;
    return tree > st ? tree : st;
}

// bump allocator over the caller's workspace
struct Carver {
    char *base;
    size_t used = 0;
    template <typename X>
    X *take(size_t count)
    {
        X *p = base ? reinterpret_cast<X *>(base + used) : nullptr;
        used = align256(used + count * sizeof(X));
        return p;
    }
};

// resolved call context
struct Ctx {
    const pss_problem *p;
    int B;
    int64_t T_y, T_x;
    hipStream_t s;
    // inside the FP32 IPLS loop of the CT model: the filter and smoother run
    // in deviation coordinates relative to the nominal means dev_m ([NX][T_x]):
    // x~_k = x_k - r_k, so the transition offset of step k is
    // F r_k + c - r_{k+1}, the measurement offset d + H r_{k+1}, the prior
    // mean m0 - r_0, and the smoother adds r_k back to its output
    const void *dev_m = nullptr;
};

// shape of one scan (filter: n_b elements per sequence, smoother: n_b + 1).
// Level l has tiles of T[l] * E[l] elements, one block of T[l] threads each.
// A tree level hands one aggregate per tile to the level above; a flat level
// (flat[l], never the top) hands up every thread's aggregate and runs no
// in-tile tree.
struct ScanShape {
    int L = 0;
    int T[kMaxLevels] = {};
    int E[kMaxLevels] = {};
    int flat[kMaxLevels] = {};
    int64_t ntiles[kMaxLevels] = {};
    int64_t nelem[kMaxLevels] = {};
};

// level 0 takes (T0, E0), level 1 (Tup, E1), the levels above (Tup, Eup)
ScanShape plan_scan(const Ctx &c, int extra, int T0, int E0, int Tup, int E1, int Eup,
                    bool flat0);
// device tile offsets of every level and, where elem_off is given, the
// element offsets of every level >= 1 (both [B + 1] per level)
int launch_plan(const Ctx &c, const ScanShape &sh, int extra, int64_t *const *tile_off,
                int64_t *const *elem_off = nullptr);
// per-sequence sums of step terms (two deterministic stages); the workspace
// part (seq_sum_bytes) comes from the caller
size_t seq_sum_bytes(const Ctx &c, int nc);
int launch_seq_sum(const Ctx &c, int nc, const double *terms, int64_t ld, double *out, void *ws);
int launch_weighted_grad(const Ctx &c, const double *grad, const double *w, double *theta_bar);

// coordinated-turn constants from the problem (host, double precision)
struct CTHost {
    double dt, q1, q2, sigma, LQ[5][5], L1[5][5], L2[5][5];
    double s1x, s1y, s2x, s2y;
};
CTHost ct_host(const pss_problem *p);

// Ricker-Poisson constants (host, double precision)
struct RickerHost {
    double loga, b, sqQ;
};
RickerHost ricker_host(const pss_problem *p);

// positive-weight sigma-point rule of the problem's linearisation (host):
// cubature (kind 0), unscented (1) or tensor Gauss-Hermite (2), see pss.h
constexpr int kMaxGH = 20;
constexpr int kMaxRulePoints = 1024;
struct RuleHost {
    int kind = 0, np = 0, p = 0;
    double w0 = 0.0, wi = 0.0, spread = 0.0;
    double gx[kMaxGH] = {}, gw[kMaxGH] = {};
};
// builds the rule for dimension nx; returns false (with the error set) for
// an invalid order or too many points
bool rule_host(const pss_problem *p, int nx, RuleHost &r);

// workspace of pss_loglik_grad_ift (defined in ift.hip)
size_t ift_ws_size(const pss_problem *p);

// one implementation per (dtype, nx, ny); defined in impl.hpp, explicitly
// instantiated in inst.hip
template <typename T, int NX, int NY>
struct Impl {
    static size_t ws_size(const Ctx &c, int op);
    static int slr(const Ctx &c, const void *m, const void *N, const void *y,
                   const pss_gamma *out);
    static int felem(const Ctx &c, const pss_gamma *g, const void *y, const pss_felem *out);
    static int fscan(const Ctx &c, const pss_felem *el, void *mf, void *Nf, void *ws);
    static int sscan(const Ctx &c, const pss_gamma *g, const void *mf, const void *Nf, void *ms,
                     void *Ns, void *ws);
    static int ipls(const Ctx &c, const pss_gamma *g, const void *y, int n_iter, void *m_nom,
                    void *N_nom, void *mf_out, void *Nf_out, void *ws);
    static int loglik(const Ctx &c, const pss_gamma *g, const void *m_nom, const void *N_nom,
                      const void *y, double *ll, const pss_ckpt *ckpt, void *ws);
    static int loglik_grad(const Ctx &c, const void *m_nom, const void *N_nom, const void *y,
                           const double *ll_bar, const pss_ckpt *ckpt, double *ll, double *grad,
                           double *theta_bar, void *ws);
    static int loglik_vjp(const Ctx &c, const pss_gamma *g, const void *m_nom, const void *N_nom,
                          const void *y, const double *ll_bar, const pss_ckpt *ckpt, double *ll,
                          const pss_gamma *gbar, void *m0_bar, void *N0_bar, void *ws);
    static int score_fisher(const Ctx &c, const void *m_nom, const void *N_nom, const void *y,
                            const double *ll_bar, double *ll, double *grad, double *theta_bar,
                            void *ws);
    static size_t ckpt_bytes(const Ctx &c, int level);
    static int filter_levels(const Ctx &c);
    static int sequential(const Ctx &c, const pss_gamma *g, const void *y, int n_iter,
                          void *m_nom, void *N_nom, void *mf_out, void *Nf_out, void *ws);
};

#define PSS_DIMS(X) X(1, 1) X(2, 1) X(2, 3) X(3, 2) X(3, 3) X(4, 2) X(5, 2)

} // namespace pss
