// Forward-mode derivatives: a number carrying K directional derivatives
// (tangents) beside its value.  Every arithmetic operation and every math
// helper of the device code has a Dual overload that applies the chain rule,
// so the templated kernels instantiated with T = Dual<double, K> compute the
// tangents of their outputs along with the values (Jacobian-vector products
// through the whole pass).  Comparisons and branch decisions look at the
// value only: the derivative is that of the branch taken.
#pragma once

#include <type_traits>

#include "device_math.hpp"
#include "device_ops.hpp"

namespace pss {

template <typename T, int K>
struct Dual {
    T v;
    T d[K];
    Dual() = default;
    // a constant (zero tangents) from any plain number
    template <typename U, typename = typename std::enable_if<std::is_arithmetic<U>::value>::type>
    PSS_INL Dual(U x) : v(T(x))
    {
#pragma unroll
        for (int k = 0; k < K; ++k)
            d[k] = T(0);
    }
    PSS_INL Dual &operator+=(const Dual &o)
    {
        v += o.v;
#pragma unroll
        for (int k = 0; k < K; ++k)
            d[k] += o.d[k];
        return *this;
    }
    PSS_INL Dual &operator-=(const Dual &o)
    {
        v -= o.v;
#pragma unroll
        for (int k = 0; k < K; ++k)
            d[k] -= o.d[k];
        return *this;
    }
    PSS_INL Dual &operator*=(const Dual &o)
    {
#pragma unroll
        for (int k = 0; k < K; ++k)
            d[k] = d[k] * o.v + v * o.d[k];
        v *= o.v;
        return *this;
    }
    PSS_INL Dual &operator/=(const Dual &o)
    {
        const T r = T(1) / o.v;
        const T q = v * r;
#pragma unroll
        for (int k = 0; k < K; ++k)
            d[k] = (d[k] - q * o.d[k]) * r;
        v = q;
        return *this;
    }
};

template <typename T, int K>
PSS_INL Dual<T, K> operator-(const Dual<T, K> &a)
{
    Dual<T, K> r;
    r.v = -a.v;
#pragma unroll
    for (int k = 0; k < K; ++k)
        r.d[k] = -a.d[k];
    return r;
}
template <typename T, int K>
PSS_INL Dual<T, K> operator+(Dual<T, K> a, const Dual<T, K> &b) { return a += b; }
template <typename T, int K>
PSS_INL Dual<T, K> operator-(Dual<T, K> a, const Dual<T, K> &b) { return a -= b; }
template <typename T, int K>
PSS_INL Dual<T, K> operator*(Dual<T, K> a, const Dual<T, K> &b) { return a *= b; }
template <typename T, int K>
PSS_INL Dual<T, K> operator/(Dual<T, K> a, const Dual<T, K> &b) { return a /= b; }

// mixed with a plain value
template <typename T, int K>
PSS_INL Dual<T, K> operator+(Dual<T, K> a, T b) { a.v += b; return a; }
template <typename T, int K>
PSS_INL Dual<T, K> operator+(T b, Dual<T, K> a) { a.v += b; return a; }
template <typename T, int K>
PSS_INL Dual<T, K> operator-(Dual<T, K> a, T b) { a.v -= b; return a; }
template <typename T, int K>
PSS_INL Dual<T, K> operator-(T b, const Dual<T, K> &a) { return Dual<T, K>(b) - a; }
template <typename T, int K>
PSS_INL Dual<T, K> operator*(Dual<T, K> a, T b)
{
    a.v *= b;
#pragma unroll
    for (int k = 0; k < K; ++k)
        a.d[k] *= b;
    return a;
}
template <typename T, int K>
PSS_INL Dual<T, K> operator*(T b, Dual<T, K> a) { return a * b; }
template <typename T, int K>
PSS_INL Dual<T, K> operator/(Dual<T, K> a, T b) { return a * (T(1) / b); }
template <typename T, int K>
PSS_INL Dual<T, K> operator/(T b, const Dual<T, K> &a) { return Dual<T, K>(b) / a; }

#define PSS_DUAL_CMP(op)                                                                         \
    template <typename T, int K>                                                                 \
    PSS_INL bool operator op(const Dual<T, K> &a, const Dual<T, K> &b) { return a.v op b.v; }    \
    template <typename T, int K>                                                                 \
    PSS_INL bool operator op(const Dual<T, K> &a, T b) { return a.v op b; }                      \
    template <typename T, int K>                                                                 \
    PSS_INL bool operator op(T a, const Dual<T, K> &b) { return a op b.v; }
PSS_DUAL_CMP(<)
PSS_DUAL_CMP(>)
PSS_DUAL_CMP(<=)
PSS_DUAL_CMP(>=)
PSS_DUAL_CMP(==)
PSS_DUAL_CMP(!=)
#undef PSS_DUAL_CMP

// f(a) with f' = g: value fv, derivative gv
template <typename T, int K>
PSS_INL Dual<T, K> dual_chain(const Dual<T, K> &a, T fv, T gv)
{
    Dual<T, K> r;
    r.v = fv;
#pragma unroll
    for (int k = 0; k < K; ++k)
        r.d[k] = gv * a.d[k];
    return r;
}

template <typename T, int K>
PSS_INL Dual<T, K> pfma(const Dual<T, K> &a, const Dual<T, K> &b, const Dual<T, K> &c)
{
    Dual<T, K> r;
    r.v = pfma(a.v, b.v, c.v);
#pragma unroll
    for (int k = 0; k < K; ++k)
        r.d[k] = pfma(a.d[k], b.v, pfma(a.v, b.d[k], c.d[k]));
    return r;
}
template <typename T, int K>
PSS_INL Dual<T, K> psqrt(const Dual<T, K> &a)
{
    const T s = psqrt(a.v);
    return dual_chain(a, s, T(0.5) / s);
}
template <typename T, int K>
PSS_INL Dual<T, K> prcp(const Dual<T, K> &a)
{
    const T r = prcp(a.v);
    return dual_chain(a, r, -r * r);
}
template <typename T, int K>
PSS_INL Dual<T, K> plog(const Dual<T, K> &a) { return dual_chain(a, plog(a.v), prcp(a.v)); }
template <typename T, int K>
PSS_INL Dual<T, K> vexp(const Dual<T, K> &a)
{
    const T e = vexp(a.v);
    return dual_chain(a, e, e);
}
template <typename T, int K>
PSS_INL Dual<T, K> vexpm1(const Dual<T, K> &a)
{
    return dual_chain(a, vexpm1(a.v), vexp(a.v));
}
template <typename T, int K>
PSS_INL Dual<T, K> psin(const Dual<T, K> &a) { return dual_chain(a, psin(a.v), pcos(a.v)); }
template <typename T, int K>
PSS_INL Dual<T, K> pcos(const Dual<T, K> &a) { return dual_chain(a, pcos(a.v), -psin(a.v)); }
template <typename T, int K>
PSS_INL Dual<T, K> pfloor(const Dual<T, K> &a) { return Dual<T, K>(pfloor(a.v)); }
// the plain overloads stay visible beside the dual one inside this namespace
using ::fabs;
template <typename T, int K>
PSS_INL Dual<T, K> fabs(const Dual<T, K> &a) { return a.v < T(0) ? -a : a; }
template <typename T, int K>
PSS_INL Dual<T, K> pabs(const Dual<T, K> &a) { return a.v < T(0) ? -a : a; }
template <typename T, int K>
PSS_INL Dual<T, K> patan2(const Dual<T, K> &y, const Dual<T, K> &x)
{
    Dual<T, K> r;
    r.v = patan2(y.v, x.v);
    const T q = prcp(x.v * x.v + y.v * y.v);
#pragma unroll
    for (int k = 0; k < K; ++k)
        r.d[k] = (x.v * y.d[k] - y.v * x.d[k]) * q;
    return r;
}

template <typename T, int K>
PSS_INL Dual<T, K> pldexp(const Dual<T, K> &a, int e)
{
    Dual<T, K> r;
    r.v = pldexp(a.v, e);
#pragma unroll
    for (int k = 0; k < K; ++k)
        r.d[k] = pldexp(a.d[k], e);
    return r;
}

template <typename T, int K>
struct Eps<Dual<T, K>> {
    static constexpr T v = Eps<T>::v;
};
template <typename T, int K>
struct TaylorSwitch<Dual<T, K>> {
    static constexpr T a = TaylorSwitch<T>::a;
};

} // namespace pss
