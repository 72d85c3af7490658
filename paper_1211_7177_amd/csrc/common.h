// Internal helpers shared by the library's HIP sources: complex arithmetic,
// error plumbing, and the special functions the expansions need.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/fmbem.h"

namespace fmb {

// ---------------------------------------------------------------------------
// error plumbing: every entry point returns a status, the message is kept
// per thread and handed out by fmb_last_error().
// ---------------------------------------------------------------------------
void set_error(const std::string &msg);

struct Status {
    int code;
    std::string msg;
};

#define FMB_CHECK_HIP(expr)                                                          \
    do {                                                                             \
        hipError_t _e = (expr);                                                      \
        if (_e != hipSuccess) {                                                      \
            throw ::fmb::Status{_e == hipErrorOutOfMemory ? FMB_ENOMEM : FMB_EDEVICE,  \
                                std::string(#expr) + ": " + hipGetErrorString(_e)};  \
        }                                                                            \
    } while (0)

#define FMB_REQUIRE(cond, msg)                                 \
    do {                                                       \
        if (!(cond)) throw ::fmb::Status{FMB_EINVAL, (msg)};   \
    } while (0)

#define FMB_LAUNCH_CHECK() FMB_CHECK_HIP(hipGetLastError())

template <typename F>
int guarded(F &&f) {
    try {
        f();
        return FMB_OK;
    } catch (const Status &s) {
        set_error(s.msg);
        return s.code;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return FMB_ENOMEM;
    } catch (const std::exception &e) {
        set_error(e.what());
        return FMB_EDEVICE;
    }
}

// device buffer owned by a plan / problem
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) {
            release();
            p = o.p;
            bytes = o.bytes;
            o.p = nullptr;
            o.bytes = 0;
        }
        return *this;
    }
    ~DevBuf() { release(); }
    void alloc(size_t b) {
        release();
        if (b == 0) b = 256;
        FMB_CHECK_HIP(hipMalloc(&p, b));
        bytes = b;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <typename T>
    T *as() const { return static_cast<T *>(p); }
};

// ---------------------------------------------------------------------------
// complex numbers
// ---------------------------------------------------------------------------
template <typename T>
struct cx {
    T re, im;
};

template <typename T>
__host__ __device__ inline cx<T> mk(T r, T i) { cx<T> z; z.re = r; z.im = i; return z; }
template <typename T>
__host__ __device__ inline cx<T> operator+(cx<T> a, cx<T> b) { return mk(a.re + b.re, a.im + b.im); }
template <typename T>
__host__ __device__ inline cx<T> operator-(cx<T> a, cx<T> b) { return mk(a.re - b.re, a.im - b.im); }
template <typename T>
__host__ __device__ inline cx<T> operator-(cx<T> a) { return mk(-a.re, -a.im); }
template <typename T>
__host__ __device__ inline cx<T> operator*(cx<T> a, cx<T> b) {
    return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T>
__host__ __device__ inline cx<T> operator*(T s, cx<T> a) { return mk(s * a.re, s * a.im); }
template <typename T>
__host__ __device__ inline cx<T> operator*(cx<T> a, T s) { return mk(s * a.re, s * a.im); }
template <typename T>
__host__ __device__ inline cx<T> &operator+=(cx<T> &a, cx<T> b) { a.re += b.re; a.im += b.im; return a; }
template <typename T>
__host__ __device__ inline cx<T> &operator-=(cx<T> &a, cx<T> b) { a.re -= b.re; a.im -= b.im; return a; }
template <typename T>
__host__ __device__ inline cx<T> conj(cx<T> a) { return mk(a.re, -a.im); }
template <typename T>
__host__ __device__ inline T abs2(cx<T> a) { return a.re * a.re + a.im * a.im; }
template <typename T>
__host__ __device__ inline cx<T> cdiv(cx<T> a, cx<T> b) {
    // scaled division (Smith's method) so that large/small moduli do not overflow
    if (fabs(b.re) >= fabs(b.im)) {
        T r = b.im / b.re, d = b.re + b.im * r;
        return mk((a.re + a.im * r) / d, (a.im - a.re * r) / d);
    } else {
        T r = b.re / b.im, d = b.re * r + b.im;
        return mk((a.re * r + a.im) / d, (a.im * r - a.re) / d);
    }
}
template <typename T>
__host__ __device__ inline cx<T> cexp_(cx<T> z) {
    T e = (T)exp(z.re);
    T s = (T)sin(z.im), c = (T)cos(z.im);
    return mk(e * c, e * s);
}
template <typename T>
__host__ __device__ inline cx<T> csin_(cx<T> z) {
    return mk((T)(sin(z.re) * cosh(z.im)), (T)(cos(z.re) * sinh(z.im)));
}

__device__ inline void sincos_t(double x, double *s, double *c) { sincos(x, s, c); }
__device__ inline void sincos_t(float x, float *s, float *c) { sincosf(x, s, c); }
// near-field kernel transcendentals: accurate FP64 library calls, hardware FP32 units
// (v_sin/v_cos/v_exp/v_rsq; used where the arguments stay within a few radians)
__device__ inline void fast_sincos(double x, double *s, double *c) { sincos(x, s, c); }
__device__ inline void fast_sincos(float x, float *s, float *c) { *s = __sinf(x); *c = __cosf(x); }
__device__ inline double fast_exp(double x) { return exp(x); }
__device__ inline float fast_exp(float x) { return __expf(x); }
__device__ inline double fast_rsqrt(double x) { return 1.0 / sqrt(x); }
__device__ inline float fast_rsqrt(float x) { return rsqrtf(x); }

// ---------------------------------------------------------------------------
// spherical Bessel functions of complex argument (FP64 or FP32)
// ---------------------------------------------------------------------------
//
// j_n(z), n = 0..N: Miller's method in ratio form.  r_n = j_n / j_{n-1}
// satisfies r_n = z / (2n + 1 - z r_{n+1}); started far above N with r = 0 it
// is stable for every z, including z -> 0 where r_n -> z/(2n+1).  Then
// j_0 = sin z / z (series for small |z|) and j_n = j_{n-1} r_n.
// z / den for the ratio recurrence (|den| >= 1 there, no scaling needed):
// FP32 uses the hardware reciprocal.
__device__ inline cx<double> cdiv_ratio(cx<double> a, cx<double> b) { return cdiv(a, b); }
__device__ inline cx<float> cdiv_ratio(cx<float> a, cx<float> b) {
    const float inv = __builtin_amdgcn_rcpf(b.re * b.re + b.im * b.im);
    return mk((a.re * b.re + a.im * b.im) * inv, (a.im * b.re - a.re * b.im) * inv);
}

template <typename T>
__device__ inline void sph_bessel_j(cx<T> z, int N, cx<T> *out) {
    const T az = (T)sqrt(abs2(z));
    if (az < T(1e-30)) {
        out[0] = mk(T(1), T(0));
        for (int n = 1; n <= N; ++n) out[n] = mk(T(0), T(0));
        return;
    }
    // FP32 needs fewer extra terms: the neglected tail scales like the product
    // of |z / (2n + 1)|^2 over the skipped degrees
    const int extra = sizeof(T) == sizeof(float) ? 8 + (int)(T(1.2) * az) : 16 + (int)az;
    const int start = N + extra;
    cx<T> r = mk(T(0), T(0));
    // walk down from `start`, store ratios for n <= N in out[] temporarily
    for (int n = start; n >= 1; --n) {
        cx<T> den = mk(T(2 * n + 1), T(0)) - z * r;
        r = cdiv_ratio(z, den);
        if (n <= N) out[n] = r;
    }
    cx<T> j0;
    if (az < T(1e-3)) {
        cx<T> z2 = z * z;
        j0 = mk(T(1), T(0)) - z2 * (T(1) / T(6)) + (z2 * z2) * (T(1) / T(120));
    } else {
        j0 = cdiv(csin_(z), z);
    }
    out[0] = j0;
    for (int n = 1; n <= N; ++n) out[n] = out[n - 1] * out[n];
}

// h_n^(1)(z), n = 0..N, by upward recurrence (h_n grows with n: stable).
template <typename T>
__host__ __device__ inline void sph_hankel_h1(cx<T> z, int N, cx<T> *out) {
    cx<T> e = cexp_(mk(-z.im, z.re));               // exp(i z)
    cx<T> iz = cdiv(mk(T(1), T(0)), z);
    out[0] = mk(T(0), T(-1)) * (e * iz);             // -i e^{iz}/z
    if (N >= 1) out[1] = -(e * (z + mk(T(0), T(1)))) * (iz * iz);   // -e^{iz}(z+i)/z^2
    for (int n = 1; n < N; ++n) out[n + 1] = T(2 * n + 1) * (iz * out[n]) - out[n - 1];
}

// ---------------------------------------------------------------------------
// spherical harmonics of eq. 2.15:
//   Y_n^m = (-1)^m sqrt((2n+1)/(4pi) (n-|m|)!/(n+|m|)!) P_n^|m|(cos th) e^{i m ph}
// with P_n^|m| carrying no Condon-Shortley phase.  Written as
//   Y_n^m = (-1)^m Q_n^|m|(cos th) (sin th e^{i ph})^m  (m >= 0),   Y_n^{-m} = conj(Y_n^m),
// where Q_n^m = Ntilde_n^m / sin^m th is a polynomial in cos th.
//   Q_0^0 = 1/sqrt(4pi),  Q_m^m = sqrt((2m+1)/(2m)) Q_{m-1}^{m-1},
//   Q_{m+1}^m = sqrt(2m+3) x Q_m^m,
//   Q_n^m = a_nm (x Q_{n-1}^m - b_nm Q_{n-2}^m),
//   a_nm = sqrt((4n^2-1)/(n^2-m^2)),  b_nm = sqrt(((n-1)^2-m^2)/(4(n-1)^2-1)).
// ---------------------------------------------------------------------------
__host__ __device__ inline int nm_index(int n, int m) { return n * n + n + m; }

}  // namespace fmb
