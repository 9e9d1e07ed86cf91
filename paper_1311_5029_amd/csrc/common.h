// Internal helpers shared by the HIP sources of libokinv (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/okinv.h"

namespace okinv {

// ---------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
int hip_fail(hipError_t e, const char* what, const char* file, int line);

#define OK_HIP(call)                                                          \
    do {                                                                      \
        hipError_t _e = (call);                                               \
        if (_e != hipSuccess) return okinv::hip_fail(_e, #call, __FILE__, __LINE__); \
    } while (0)

#define OK_LAUNCH_CHECK(name)                                                 \
    do {                                                                      \
        hipError_t _e = hipGetLastError();                                    \
        if (_e != hipSuccess) return okinv::hip_fail(_e, name, __FILE__, __LINE__); \
    } while (0)

// ---------------------------------------------------------------- geometry
struct Geo {
    int L[4];       // Lx, Ly, Lz, Lt
    int V;          // sites
    int Vs;         // site stride of W planes (V rounded up to 64)
};

int make_geo(const ok_geom* g, Geo* out);   // validates; returns ok_status
int check_ptr(const void* p, const char* name);

constexpr int kW = 27;           // blocks per site
constexpr int kWE = 144;         // complex entries per block

// Offsets d_k = (dx, dy, dz, dt) in storage order (see okinv.h).
__host__ __device__ constexpr int off_d(int k, int mu) {
    // rows: k, columns x y z t
    constexpr int T[27][4] = {
        {0, 0, 0, 0},
        {1, 0, 0, 0},  {0, 1, 0, 0},  {0, 0, 1, 0},  {0, 0, 0, 1},
        {-1, 0, 0, 0}, {0, -1, 0, 0}, {0, 0, -1, 0}, {0, 0, 0, -1},
        {2, 0, 0, 0},  {0, 2, 0, 0},  {0, 0, 2, 0},
        {-2, 0, 0, 0}, {0, -2, 0, 0}, {0, 0, -2, 0},
        {1, 1, 0, 0},  {1, 0, 1, 0},  {0, 1, 1, 0},
        {-1, -1, 0, 0}, {-1, 0, -1, 0}, {0, -1, -1, 0},
        {1, -1, 0, 0}, {1, 0, -1, 0}, {0, 1, -1, 0},
        {-1, 1, 0, 0}, {-1, 0, 1, 0}, {0, -1, 1, 0},
    };
    return T[k][mu];
}

__device__ __forceinline__ int wrap(int v, int L) {
    v += (v < 0) ? L : 0;
    v -= (v >= L) ? L : 0;
    return v;
}

__device__ __forceinline__ void site_coords(const Geo& g, int s, int& x, int& y, int& z, int& t) {
    x = s % g.L[0];
    int r = s / g.L[0];
    y = r % g.L[1];
    r /= g.L[1];
    z = r % g.L[2];
    t = r / g.L[2];
}

__device__ __forceinline__ int site_index(const Geo& g, int x, int y, int z, int t) {
    return x + g.L[0] * (y + g.L[1] * (z + g.L[2] * t));
}

__device__ __forceinline__ int neighbour(const Geo& g, int x, int y, int z, int t,
                                         int dx, int dy, int dz, int dt) {
    return site_index(g, wrap(x + dx, g.L[0]), wrap(y + dy, g.L[1]),
                      wrap(z + dz, g.L[2]), wrap(t + dt, g.L[3]));
}

// ---------------------------------------------------------------- complex
template <typename T>
struct cpx {
    T re, im;
};
using c64 = cpx<float>;
using c128 = cpx<double>;

template <typename T>
__host__ __device__ __forceinline__ cpx<T> cmk(T r, T i) { return cpx<T>{r, i}; }
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator-(cpx<T> a) { return {-a.re, -a.im}; }
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator*(cpx<T> a, cpx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator*(T s, cpx<T> a) { return {s * a.re, s * a.im}; }
template <typename T>
__host__ __device__ __forceinline__ cpx<T> conj(cpx<T> a) { return {a.re, -a.im}; }
// a += b * c
template <typename T>
__host__ __device__ __forceinline__ void cfma(cpx<T>& a, cpx<T> b, cpx<T> c) {
    a.re = fma(b.re, c.re, a.re);
    a.re = fma(-b.im, c.im, a.re);
    a.im = fma(b.re, c.im, a.im);
    a.im = fma(b.im, c.re, a.im);
}
// a += conj(b) * c
template <typename T>
__host__ __device__ __forceinline__ void cfma_conj(cpx<T>& a, cpx<T> b, cpx<T> c) {
    a.re = fma(b.re, c.re, a.re);
    a.re = fma(b.im, c.im, a.re);
    a.im = fma(b.re, c.im, a.im);
    a.im = fma(-b.im, c.re, a.im);
}

// ---------------------------------------------------------------- bf16
// Round-to-nearest-even FP32 -> BF16 (NaN kept quiet).
__host__ __device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__host__ __device__ __forceinline__ float bf16_to_f32(uint32_t h) {
    return __builtin_bit_cast(float, h << 16);
}

// ---------------------------------------------------------------- streaming loads
// W is read exactly once per application: load it non-temporally so that it
// does not evict the reused neighbour spinors from L2.
typedef unsigned nt_u4 __attribute__((ext_vector_type(4)));
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef float nt_f2 __attribute__((ext_vector_type(2)));
typedef double nt_d2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint4 ld_stream(const uint4* p) {
    const nt_u4 v = __builtin_nontemporal_load(reinterpret_cast<const nt_u4*>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ float4 ld_stream(const float4* p) {
    const nt_f4 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f4*>(p));
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ float2 ld_stream(const float2* p) {
    const nt_f2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f2*>(p));
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ double2 ld_stream(const double2* p) {
    const nt_d2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(p));
    return make_double2(v.x, v.y);
}

// ---------------------------------------------------------------- launches
// The hardware places workgroup b on XCD b % 8.  Hand each XCD a contiguous
// range of the n tiles so that neighbouring sites are served by the same L2.
__device__ __forceinline__ int xcd_tile(int b, int n) {
    const int x = b & 7, q = b >> 3;
    int start = 0;
    for (int y = 0; y < x; ++y) start += (n - y + 7) >> 3;
    return start + q;
}

inline unsigned grid_for(long n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace okinv
