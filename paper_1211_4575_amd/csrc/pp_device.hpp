// Device-side building blocks of the particle step: B-spline weights, the Vay and
// Boris momentum updates, periodic index helpers.  Templated on the arithmetic type
// (double for the FP64 form, float for the split-precision form).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pp {

__device__ __forceinline__ int wrap(int i, int n) {
    // i is at most a few periods away from [0, n)
    i %= n;
    return i < 0 ? i + n : i;
}

// The same for i within one period of [0, n) (a compare and an add; no division), falling
// back to the general form farther away (grids smaller than a tile's halo).
__device__ __forceinline__ int wrap_near(int i, int n) {
    const int j = i < 0 ? i + n : (i >= n ? i - n : i);
    return (j >= 0 && j < n) ? j : wrap(i, n);
}

// Weights of order O (Sec. II: TSC for O = 2, PCS for O = 3) of the O+1 nodes
// i0, i0+1, ..., i0+O nearest to coordinate y (node positions are integers).
//   O = 2: c = floor(y + 1/2), t = y - c in [-1/2, 1/2), i0 = c - 1,
//          w = (1/2 (1/2 - t)^2, 3/4 - t^2, 1/2 (1/2 + t)^2)
//   O = 3: f = floor(y), t = y - f in [0, 1), i0 = f - 1,
//          w = ((1-t)^3/6, (4 - 6t^2 + 3t^3)/6, (4 - 6(1-t)^2 + 3(1-t)^3)/6, t^3/6)
// These are the paper's piecewise W^O evaluated at delta = node - y on each node.
template <int O, typename T>
__device__ __forceinline__ void weights_frac(T t, T* w);

template <>
__device__ __forceinline__ void weights_frac<2, double>(double t, double* w) {
    double a = 0.5 - t, b = 0.5 + t;
    w[0] = 0.5 * a * a;
    w[1] = 0.75 - t * t;
    w[2] = 0.5 * b * b;
}
template <>
__device__ __forceinline__ void weights_frac<2, float>(float t, float* w) {
    float a = 0.5f - t, b = 0.5f + t;
    w[0] = 0.5f * a * a;
    w[1] = 0.75f - t * t;
    w[2] = 0.5f * b * b;
}
template <>
__device__ __forceinline__ void weights_frac<3, double>(double t, double* w) {
    double s = 1.0 - t;
    const double k6 = 1.0 / 6.0;
    w[0] = k6 * s * s * s;
    w[1] = k6 * (4.0 - 6.0 * t * t + 3.0 * t * t * t);
    w[2] = k6 * (4.0 - 6.0 * s * s + 3.0 * s * s * s);
    w[3] = k6 * t * t * t;
}
template <>
__device__ __forceinline__ void weights_frac<3, float>(float t, float* w) {
    // the same polynomials with the powers shared: (4 - 6t^2 + 3t^3)/6 = 2/3 + t^2 (t/2 - 1)
    const float s = 1.0f - t;
    const float t2 = t * t, s2 = s * s;
    const float k6 = 1.0f / 6.0f;
    w[0] = (k6 * s) * s2;
    w[1] = fmaf(t2, fmaf(0.5f, t, -1.0f), 2.0f / 3.0f);
    w[2] = fmaf(s2, fmaf(0.5f, s, -1.0f), 2.0f / 3.0f);
    w[3] = (k6 * t) * t2;
}

// First node and weights for an absolute coordinate y (FP64 form).
template <int O>
__device__ __forceinline__ int weights_abs(double y, double* w) {
    if (O == 2) {
        double c = floor(y + 0.5);
        weights_frac<2, double>(y - c, w);
        return (int)c - 1;
    } else {
        double f = floor(y);
        weights_frac<3, double>(y - f, w);
        return (int)f - 1;
    }
}

template <typename T>
struct V3 {
    T x, y, z;
};

template <typename T>
__device__ __forceinline__ T dot(const V3<T>& a, const V3<T>& b) {
    return a.x * b.x + a.y * b.y + a.z * b.z;
}
template <typename T>
__device__ __forceinline__ V3<T> cross(const V3<T>& a, const V3<T>& b) {
    return V3<T>{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

__device__ __forceinline__ double rsqrt_t(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float rsqrt_t(float x) { return 1.0f / sqrtf(x); }
__device__ __forceinline__ double sqrt_t(double x) { return sqrt(x); }
__device__ __forceinline__ float sqrt_t(float x) { return sqrtf(x); }

// Momentum update u^{n-1/2} -> u^{n+1/2} (Sec. III.A).  h = q dt / m, ic2 = 1/c^2.
// Vay (2008): the three-velocities of the old and new state are averaged in v x B;
// the new Lorentz factor is the positive root of a quadratic in gamma^2.
template <typename T>
__device__ __forceinline__ void push_vay(T h, T ic, const V3<T>& E, const V3<T>& B, V3<T>& u) {
    const T half = T(0.5);
    T ig0 = rsqrt_t(T(1) + dot(u, u) * ic * ic);
    V3<T> v{u.x * ig0, u.y * ig0, u.z * ig0};
    V3<T> vxB = cross(v, B);
    V3<T> up{u.x + h * (E.x + half * vxB.x), u.y + h * (E.y + half * vxB.y), u.z + h * (E.z + half * vxB.z)};
    V3<T> tau{half * h * B.x, half * h * B.y, half * h * B.z};
    T tau2 = dot(tau, tau);
    T ust = dot(up, tau) * ic;
    T sigma = T(1) + dot(up, up) * ic * ic - tau2;
    T g2 = half * (sigma + sqrt_t(sigma * sigma + T(4) * (tau2 + ust * ust)));
    T ig = rsqrt_t(g2);
    V3<T> t{tau.x * ig, tau.y * ig, tau.z * ig};
    T s = T(1) / (T(1) + dot(t, t));
    T upt = dot(up, t);
    V3<T> uxt = cross(up, t);
    u = V3<T>{s * (up.x + upt * t.x + uxt.x), s * (up.y + upt * t.y + uxt.y), s * (up.z + upt * t.z + uxt.z)};
}

// Boris (1970): half electric kick, rotation with the Lorentz factor of the half-kicked
// proper velocity, second half kick.
template <typename T>
__device__ __forceinline__ void push_boris(T h, T ic, const V3<T>& E, const V3<T>& B, V3<T>& u) {
    const T hh = T(0.5) * h;
    V3<T> um{u.x + hh * E.x, u.y + hh * E.y, u.z + hh * E.z};
    T ig = rsqrt_t(T(1) + dot(um, um) * ic * ic);
    V3<T> t{hh * B.x * ig, hh * B.y * ig, hh * B.z * ig};
    T f = T(2) / (T(1) + dot(t, t));
    V3<T> s{f * t.x, f * t.y, f * t.z};
    V3<T> umxt = cross(um, t);
    V3<T> upr{um.x + umxt.x, um.y + umxt.y, um.z + umxt.z};
    V3<T> c2 = cross(upr, s);
    u = V3<T>{um.x + c2.x + hh * E.x, um.y + c2.y + hh * E.y, um.z + c2.z + hh * E.z};
}

// Radiative cooling of one step (Sec. "Radiative cooling", eqs. "prad", "udot"): um is the
// proper velocity before the push, u the one after the electromagnetic push; with u0 their
// mean, gamma0 = sqrt(1 + u0^2/c^2) and a = (u - um)/dt the proper acceleration,
//   u -= k (gamma0 / u0^2) (|a|^2 + |a x u0|^2 / c^2) u0 dt,   k = rad_tau q^2 / m.
// Only proper velocities enter (no cancellation between gamma^2 and u^2 in FP32).
template <typename T>
__device__ __forceinline__ void rad_cool(T k, T dt, T ic, const V3<T>& um, V3<T>& u) {
    const V3<T> u0{(T)0.5 * (u.x + um.x), (T)0.5 * (u.y + um.y), (T)0.5 * (u.z + um.z)};
    const T idt = (T)1 / dt;
    const V3<T> a{(u.x - um.x) * idt, (u.y - um.y) * idt, (u.z - um.z) * idt};
    const T u02 = dot(u0, u0);
    if (!(u02 > (T)0)) return;
    const V3<T> x = cross(a, u0);
    const T g0 = sqrt((T)1 + u02 * ic * ic);
    const T f = -k * g0 / u02 * (dot(a, a) + dot(x, x) * ic * ic) * dt;
    u.x += f * u0.x;
    u.y += f * u0.y;
    u.z += f * u0.z;
}

__device__ __forceinline__ void atomic_add_f64(double* p, double v) { unsafeAtomicAdd(p, v); }

// Segment of a batched launch: the largest r in [0, n) with prefix[r] <= b < prefix[r + 1]
// (prefix has n + 1 non-decreasing entries), or -1 when b is beyond the last segment.
__device__ __forceinline__ int find_segment(const int64_t* __restrict__ prefix, int n, int64_t b) {
    if (n <= 0 || b < prefix[0] || b >= prefix[n]) return -1;
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}
__device__ __forceinline__ void atomic_or_flag(int32_t* p, int32_t v) { atomicOr(p, v); }

}  // namespace pp
