// Shared pieces of the fixed-point gradient (ift.hip, ift_smoother.hip,
// ift_api.hip): the dual-number types of its passes, the workspace buffers of
// one call, and the per-precision entry points (S = double or float).
#pragma once

#include "dual.hpp"
#include "impl.hpp"

namespace pss {

// launch shapes of the dual-number scans: the tree at every level.  A dual
// scan kernel runs one tile per CU (4x the registers and LDS of its value
// type), so the extra level that a flat finest level brings costs more than
// the tree it saves at the sizes this gradient is used on (n = 1000: 196 ms
// per call flat, 177 ms with the tree).
template <typename S, int NX>
struct Defaults<Dual<S, 3>, NX> {
    static constexpr int T0 = 64;
    static constexpr int E0_filter = 4;
    static constexpr int E0_smoother = 2;
    static constexpr int Tup = 64;
    static constexpr int E1_filter = 2;
    static constexpr int E1_smoother = 2;
    static constexpr int Eup_filter = 2;
    static constexpr int Eup_smoother = 2;
    static constexpr bool flat_filter = false;
    static constexpr bool flat_smoother = false;
};

template <typename S>
using IftC = Core<Dual<S, 3>, 5, 2>;

template <typename S>
struct IftBufs {
    Dual<S, 3> *nm, *nP, *mf, *Pf, *yd, *m0d, *N0d;
    pss_gamma gam;
    FElemRef<Dual<S, 3>, 5> fel;
    double *ell;
    double *prev, *stat; // previous tangents [60][T_x]; per-state change [T_x]
    void *scan_ws;
    size_t used;
};

// covariance-form smoother scan of the dual pass (ift_smoother.hip): reads
// the dual linearisation and filter marginals, writes the dual nominal
template <typename S>
int run_sscan(const Ctx &c, const IftBufs<S> &w);

// workspace bytes and the whole computation (ift.hip); the problem has been
// validated by the caller (ift_api.hip)
template <typename S>
size_t ift_ws(const pss_problem *p);
template <typename S>
int ift_run(const pss_problem *p, const void *m_nom, const void *N_nom, const void *y,
            int32_t n_iter, double *ll, double *grad, double *delta, void *ws,
            hipStream_t stream);

} // namespace pss
