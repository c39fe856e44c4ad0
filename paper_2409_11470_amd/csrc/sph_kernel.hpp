// SPH smoothing kernels with support 2h, written W(r, h) = f(q)/(pi h^3),
// q = r/h, so that every sum carries f and its q-derivatives and the 1/pi
// and powers of h are applied once per target:
//   M4 cubic spline (paper appendix A, kernel table; h_fact 1.2 there)
//     f = 1 - 3/2 q^2 + 3/4 q^3 (q < 1),  1/4 (2 - q)^3 (1 <= q < 2)
//   Wendland C2 (the paper's example applications, Sec. 3: kernel radius 2h,
//   h_fact 1.3), normalised in 3D
//     f = 21/16 (1 - q/2)^4 (1 + 2 q)   (q < 2)
// Kern<K>::eval<T, D>(q, f, df, d2f) gives f and, for D >= 1 and D >= 2, f'
// and f'' (0 <= q <= 2; q slightly above 2 from rounding gives about 0).
// Kern<K>::f0 is f(0), the self term.
#pragma once

#include "common.hpp"

namespace apr {

constexpr int kM4 = APR_KERNEL_M4;
constexpr int kWC2 = APR_KERNEL_WC2;

template <int K>
struct Kern;

// M4, branch-free from t = 2 - q and u = max(1 - q, 0):
//   f = t^3/4 - u^3,  f' = 3 u^2 - 3/4 t^2,  f'' = 3/2 t - 6 u.
template <>
struct Kern<kM4> {
    static constexpr double f0 = 1.0;
    template <class T, int D>
    __device__ static inline void eval(T q, T &f, T &df, T &d2f)
    {
        T t = T(2) - q;
        T u = T(1) - q;
        u = u > T(0) ? u : T(0);
        T t2 = t * t, u2 = u * u;
        f = T(0.25) * t2 * t - u2 * u;
        if (D >= 1) df = T(3) * u2 - T(0.75) * t2;
        if (D >= 2) d2f = T(1.5) * t - T(6) * u;
    }
};

// Wendland C2 from u = max(1 - q/2, 0):
//   f = 21/16 u^4 (1 + 2 q),  f' = -105/16 q u^3,  f'' = -105/16 u^2 (1 - 2 q).
template <>
struct Kern<kWC2> {
    static constexpr double f0 = 21.0 / 16.0;
    template <class T, int D>
    __device__ static inline void eval(T q, T &f, T &df, T &d2f)
    {
        T u = T(1) - T(0.5) * q;
        u = u > T(0) ? u : T(0);
        T u2 = u * u, u3 = u2 * u;
        f = T(1.3125) * u3 * u * (T(1) + T(2) * q);
        if (D >= 1) df = T(-6.5625) * q * u3;
        if (D >= 2) d2f = T(-6.5625) * u2 * (T(1) - T(2) * q);
    }
};

}  // namespace apr
