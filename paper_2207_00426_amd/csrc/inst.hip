// One explicit instantiation of the per-dimension implementation; the build
// compiles this file once per (dtype, nx, ny) with PSS_T, PSS_NX, PSS_NY set.
#include "impl.hpp"

#if !defined(PSS_T) || !defined(PSS_NX) || !defined(PSS_NY)
#error "compile with -DPSS_T=<float|double> -DPSS_NX=<n> -DPSS_NY=<n>"
#endif

template struct pss::Impl<PSS_T, PSS_NX, PSS_NY>;
