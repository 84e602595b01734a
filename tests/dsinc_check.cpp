// Host build of the library's sinc-difference helper (the transition SLR's
// cancellation-free sigma-point deviations) in FP32 and FP64.  Reads pairs
// "x d" from stdin and prints "dsinc_f32 dsinc_f64" per pair.  Test
// infrastructure: compiled and run by tests/test_dsinc_cpu.py.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>

// host stand-ins for the device builtins the shared headers name (only the
// host pass sees them; nothing here calls them)
#if !defined(__HIP_DEVICE_COMPILE__)
static inline int host_frexp_exp(double x)
{
    int e;
    std::frexp(x, &e);
    return e;
}
#define __builtin_amdgcn_rcpf(x) (1.0f / (x))
#define __builtin_amdgcn_rcp(x) (1.0 / (x))
#define __builtin_amdgcn_frexp_expf(x) host_frexp_exp((double)(x))
#define __builtin_amdgcn_frexp_exp(x) host_frexp_exp(x)
#define __builtin_amdgcn_ldexpf(x, e) std::ldexp((float)(x), e)
#define __builtin_amdgcn_ldexp(x, e) std::ldexp((double)(x), e)
#endif

#include "../paper_2207_00426_amd/csrc/device_ops.hpp"

int main()
{
    double x, d;
    while (std::scanf("%lf %lf", &x, &d) == 2) {
        const float f = pss::dsinc((float)x, (float)d);
        const double g = pss::dsinc(x, d);
        std::printf("%.9e %.17e\n", (double)f, g);
    }
    return 0;
}
