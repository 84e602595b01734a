// Covariance-form smoother scan of the fixed-point gradient's dual passes,
// compiled on its own once per precision (-DPSS_IFT_T=double|float; the
// dual-number scans are large).
#include "ift.hpp"

namespace pss {

template <typename S>
int run_sscan(const Ctx &c, const IftBufs<S> &w)
{
    using D = Dual<S, 3>;
    using C = IftC<S>;
    using SSC = SmootherScanCov<D, 5>;
    const ScanShape sh = C::smoother_shape(c);
    Carver cv{static_cast<char *>(w.scan_ws)};
    auto sw = C::template carve_scan<SSC>(cv, c, sh);
    D *stash = cv.take<D>((size_t)Sizes<5>::selem * c.T_x);
    SmootherSrc<D, 5, 2, true> src{C::gamma_ref(&w.gam, c.T_y), C::marg_ref2(w.mf, w.Pf, c.T_x),
                                   C::selem_ref(stash, c.T_x), c.p->y_off};
    SmoothDst<D, 5> dst{C::marg_ref2(w.nm, w.nP, c.T_x)};
    StartPre<D, 5> st{nullptr, nullptr};
    return C::template run_scan<SSC, C::kFlatS>(c, sh, sw, 1, src, dst, st, &C::selem_ref);
}

#if !defined(PSS_IFT_T)
#error "compile with -DPSS_IFT_T=<double|float>"
#endif
template int run_sscan<PSS_IFT_T>(const Ctx &c, const IftBufs<PSS_IFT_T> &w);

} // namespace pss
