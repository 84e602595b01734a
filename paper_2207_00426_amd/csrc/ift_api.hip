// C ABI of the fixed-point gradient (pss_loglik_grad_ift): validation and
// dispatch on the precision; the computation is in ift.hip.
#include <string>

#include "ift.hpp"

namespace pss {

static int ift_validate(const pss_problem *p)
{
    int rc = pss_validate(p);
    if (rc)
        return rc;
    if (p->model != PSS_MODEL_CT_BEARINGS) {
        set_error("loglik_grad_ift: theta is defined for the coordinated-turn model");
        return PSS_EUNSUPPORTED;
    }
    return PSS_OK;
}

size_t ift_ws_size(const pss_problem *p)
{
    return p->dtype == PSS_F64 ? ift_ws<double>(p) : ift_ws<float>(p);
}

} // namespace pss

using namespace pss;

extern "C" int pss_loglik_grad_ift(const pss_problem *p, const void *m_nom, const void *N_nom,
                                   const void *y, int32_t n_iter, double *ll, double *grad,
                                   double *delta, void *ws, size_t ws_bytes, hipStream_t stream)
{
    try {
        int rc = ift_validate(p);
        if (rc)
            return rc;
        if (!m_nom || !N_nom || !y || !ll || !grad || n_iter < 1) {
            set_error("loglik_grad_ift: null buffer or n_iter < 1");
            return PSS_EINVAL;
        }
        const size_t need = ift_ws_size(p);
        if (!ws || ws_bytes < need) {
            set_error("workspace too small: need " + std::to_string(need) + " bytes");
            return PSS_EWORKSPACE;
        }
        if (p->dtype == PSS_F64)
            return ift_run<double>(p, m_nom, N_nom, y, n_iter, ll, grad, delta, ws, stream);
        return ift_run<float>(p, m_nom, N_nom, y, n_iter, ll, grad, delta, ws, stream);
    } catch (const std::exception &ex) {
        set_error(ex.what());
        return PSS_EINVAL;
    } catch (...) {
        set_error("unknown exception in loglik_grad_ift");
        return PSS_EINVAL;
    }
}
