// Shared device/host helpers of the RSRR HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define RSRR_DEV __device__ __forceinline__

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

// Complex element type per real type: float -> float2 (c64), double -> double2 (c128).
template <typename R> struct cpx;
template <> struct cpx<float> { typedef float2 T; };
template <> struct cpx<double> { typedef double2 T; };

RSRR_DEV float2 mk(float a, float b) { return make_float2(a, b); }
RSRR_DEV double2 mk(double a, double b) { return make_double2(a, b); }

template <typename C> RSRR_DEV C cadd(C a, C b) { a.x += b.x; a.y += b.y; return a; }
template <typename C> RSRR_DEV C csub(C a, C b) { a.x -= b.x; a.y -= b.y; return a; }
template <typename C> RSRR_DEV C cmul(C a, C b) {
    C r; r.x = a.x * b.x - a.y * b.y; r.y = a.x * b.y + a.y * b.x; return r;
}
template <typename C> RSRR_DEV C cconj(C a) { a.y = -a.y; return a; }
// a - b*c
template <typename C> RSRR_DEV C cfms(C a, C b, C c) {
    a.x -= b.x * c.x - b.y * c.y; a.y -= b.x * c.y + b.y * c.x; return a;
}
// a + b*c
template <typename C> RSRR_DEV C cfma(C a, C b, C c) {
    a.x += b.x * c.x - b.y * c.y; a.y += b.x * c.y + b.y * c.x; return a;
}
// a + conj(b)*c
template <typename C> RSRR_DEV C cfma_cj(C a, C b, C c) {
    a.x += b.x * c.x + b.y * c.y; a.y += b.x * c.y - b.y * c.x; return a;
}
// Reciprocal by Smith's scaling (avoids overflow of |a|^2).
template <typename C> RSRR_DEV C crecip(C a) {
    C r;
    if (fabs(a.x) >= fabs(a.y)) {
        auto t = a.y / a.x; auto d = a.x + a.y * t;
        r.x = 1 / d; r.y = -t / d;
    } else {
        auto t = a.x / a.y; auto d = a.y + a.x * t;
        r.x = t / d; r.y = -1 / d;
    }
    return r;
}
// LAPACK's complex magnitude measure for pivoting: |Re| + |Im|.
template <typename C> RSRR_DEV auto cabs1(C a) -> decltype(a.x) { return fabs(a.x) + fabs(a.y); }

template <typename C> RSRR_DEV C czero() { C r; r.x = 0; r.y = 0; return r; }

// Real element types: the same helpers for real LU kernels (a real NEP sampled
// at real points).  Non-template overloads win over the complex templates.
RSRR_DEV float cadd(float a, float b) { return a + b; }
RSRR_DEV double cadd(double a, double b) { return a + b; }
RSRR_DEV float csub(float a, float b) { return a - b; }
RSRR_DEV double csub(double a, double b) { return a - b; }
RSRR_DEV float cmul(float a, float b) { return a * b; }
RSRR_DEV double cmul(double a, double b) { return a * b; }
RSRR_DEV float cconj(float a) { return a; }
RSRR_DEV double cconj(double a) { return a; }
RSRR_DEV float cfms(float a, float b, float c) { return a - b * c; }
RSRR_DEV double cfms(double a, double b, double c) { return a - b * c; }
RSRR_DEV float cfma(float a, float b, float c) { return a + b * c; }
RSRR_DEV double cfma(double a, double b, double c) { return a + b * c; }
RSRR_DEV float crecip(float a) { return 1.0f / a; }
RSRR_DEV double crecip(double a) { return 1.0 / a; }
RSRR_DEV float cabs1(float a) { return fabsf(a); }
RSRR_DEV double cabs1(double a) { return fabs(a); }
template <> RSRR_DEV float czero<float>() { return 0.0f; }
template <> RSRR_DEV double czero<double>() { return 0.0; }

// Element traits: the real type of an element, exact zero and finiteness tests,
// and an element holding a real value.
template <typename C> struct elem_traits;
template <> struct elem_traits<float2> { typedef float R; static constexpr bool complex = true; };
template <> struct elem_traits<double2> { typedef double R; static constexpr bool complex = true; };
template <> struct elem_traits<float> { typedef float R; static constexpr bool complex = false; };
template <> struct elem_traits<double> { typedef double R; static constexpr bool complex = false; };
template <typename C> using real_t = typename elem_traits<C>::R;

template <typename C> RSRR_DEV bool is_zero(C a) { return a.x == 0 && a.y == 0; }
RSRR_DEV bool is_zero(float a) { return a == 0.0f; }
RSRR_DEV bool is_zero(double a) { return a == 0.0; }
template <typename C> RSRR_DEV bool all_finite(C a) { return isfinite(a.x) && isfinite(a.y); }
RSRR_DEV bool all_finite(float a) { return isfinite(a); }
RSRR_DEV bool all_finite(double a) { return isfinite(a); }
template <typename C> RSRR_DEV C from_real(real_t<C> v)
{
    if constexpr (elem_traits<C>::complex) return mk(v, (real_t<C>)0);
    else return v;
}

// Round an interleaved c128 value to c64.
RSRR_DEV float2 to_c64(double2 a) { return make_float2((float)a.x, (float)a.y); }
RSRR_DEV double2 to_c128(float2 a) { return make_double2((double)a.x, (double)a.y); }

// Workgroups are dispatched round-robin over the 8 XCDs (blockIdx % 8 -> XCD).
// Remap a linear block id so that consecutive logical tiles land on the same
// XCD (and share its L2).  `total` must be a multiple of 8.
RSRR_DEV long xcd_remap(long g, long total) {
    long per = total >> 3;
    return (g & 7) * per + (g >> 3);
}

static inline long round_up_l(long x, long m) { return (x + m - 1) / m * m; }
