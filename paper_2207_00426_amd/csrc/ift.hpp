// Shared pieces of the fixed-point gradient (ift.hip, ift_smoother.hip): the
// dual-number type of its passes and the workspace buffers of one call.
#pragma once

#include "dual.hpp"
#include "impl.hpp"

namespace pss {

using D = Dual<double, 3>;
using C = Core<D, 5, 2>;
using FSC = FilterScanCov<D, 5>;
using SSC = SmootherScanCov<D, 5>;

struct IftBufs {
    D *nm, *nP, *mf, *Pf, *yd, *m0d, *N0d;
    pss_gamma gam;
    FElemRef<D, 5> fel;
    double *ell;
    double *prev, *stat; // previous tangents [60][T_x]; per-state change [T_x]
    void *scan_ws;
    size_t used;
};

// covariance-form smoother scan of the dual pass (ift_smoother.hip): reads
// the dual linearisation and filter marginals, writes the dual nominal
int run_sscan(const Ctx &c, const IftBufs &w);

} // namespace pss
