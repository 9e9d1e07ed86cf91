// The 27-point operator (M psi)_x = mhat psi_x + sum_k W_{k,x} psi_{x+d_k}  (Eq. minFlopForm).
//
// HBM-bound: per site and application it streams the 27 dense W blocks
// (62,208 B FP64, 31,104 B FP32, 15,552 B BF16) and one spinor in and out;
// the 27 neighbour spinor reads hit L2/MALL.  TPS threads cooperate on a site,
// each owning 12/TPS output rows; lanes are grouped so that the TPS groups of a
// wavefront each read 64/TPS consecutive sites of one W plane (contiguous
// 16-byte cells).  Accumulation is FP64 for FP64 W and FP32 otherwise.
//
// An optional epilogue reduces per-block partial sums of the dot products the
// BiCGStab recurrence needs right after an application (see blas1.hip):
//   EPI_RV:  <aux, out>                  (r^ . v)
//   EPI_TS:  <out, aux or in>, <out, out>  (t . s, t . t; aux NULL: s is the input)
#include <algorithm>

#include "common.h"
#include "kernels.h"
#include "wlayout.h"

namespace okinv {
namespace {

template <int P> struct Arith { using T = float; };
template <> struct Arith<OK_F64> { using T = double; };

// Load 12 complex spinor components of site s.
template <typename T>
__device__ __forceinline__ void ld_spinor(const T* __restrict__ psi, int s, cpx<T> v[12]) {
    if constexpr (sizeof(T) == 8) {
        const double2* p = reinterpret_cast<const double2*>(psi) + (size_t)s * 12;
#pragma unroll
        for (int i = 0; i < 12; ++i) {
            double2 d = p[i];
            v[i] = cpx<T>{d.x, d.y};
        }
    } else {
        const float4* p = reinterpret_cast<const float4*>(psi) + (size_t)s * 6;
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            float4 f = p[i];
            v[2 * i] = cpx<T>{f.x, f.y};
            v[2 * i + 1] = cpx<T>{f.z, f.w};
        }
    }
}

// acc[q] += row (r0 + q) of W_k(s) . v  for q < RPT
template <int P, int RPT, typename T>
__device__ __forceinline__ void block_rows(const void* __restrict__ W, int Vs, int k, int r0, int s,
                                           const cpx<T> v[12], cpx<T> acc[RPT]) {
    constexpr int per = WL<P>::per, ch = WL<P>::chunks;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int row = r0 + q;
#pragma unroll
        for (int j = 0; j < 12 / per; ++j) {
            const size_t cell = ((size_t)(k * ch + row * (12 / per) + j)) * Vs + s;
            if constexpr (P == OK_F64) {
                double2 w = ld_stream(reinterpret_cast<const double2*>(W) + cell);
                cfma(acc[q], cpx<T>{w.x, w.y}, v[j]);
            } else if constexpr (P == OK_F32) {
                float4 w = ld_stream(reinterpret_cast<const float4*>(W) + cell);
                cfma(acc[q], cpx<T>{w.x, w.y}, v[2 * j]);
                cfma(acc[q], cpx<T>{w.z, w.w}, v[2 * j + 1]);
            } else {
                uint4 w = ld_stream(reinterpret_cast<const uint4*>(W) + cell);
                const uint32_t u[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    cpx<T> we{bf16_to_f32(u[e] & 0xffffu), bf16_to_f32(u[e] >> 16)};
                    cfma(acc[q], we, v[4 * j + e]);
                }
            }
        }
    }
}

template <int P, int TPS, int EPI>
__global__ void __launch_bounds__(256) k_apply(Geo g, const void* __restrict__ W,
                                               const typename Arith<P>::T* __restrict__ psi,
                                               typename Arith<P>::T* __restrict__ out,
                                               double mhat_d,
                                               const typename Arith<P>::T* __restrict__ aux,
                                               double2* __restrict__ partial) {
    using T = typename Arith<P>::T;
    constexpr int RPT = 12 / TPS;
    constexpr int SPW = 64 / TPS;            // sites per wavefront
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int grp = lane / SPW;              // row group of this lane
    // contiguous site ranges per XCD: neighbour spinors are shared within one L2
    const int s = (xcd_tile(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + wave) * SPW + (lane % SPW);
    const bool live = s < g.V;
    const int r0 = grp * RPT;
    const T mhat = (T)mhat_d;

    cpx<T> acc[RPT];
    double2 d1{0.0, 0.0}, d2{0.0, 0.0};
    if (live) {
        int x, y, z, t;
        site_coords(g, s, x, y, z, t);
        cpx<T> v[12];
        {
            const cpx<T>* c = reinterpret_cast<const cpx<T>*>(psi) + (size_t)s * 12 + r0;
#pragma unroll
            for (int q = 0; q < RPT; ++q) acc[q] = mhat * c[q];
        }
#pragma unroll 1
        for (int k = 0; k < kW; ++k) {
            const int n = neighbour(g, x, y, z, t, off_d(k, 0), off_d(k, 1), off_d(k, 2), off_d(k, 3));
            ld_spinor(psi, n, v);
            block_rows<P, RPT, T>(W, g.Vs, k, r0, s, v, acc);
        }
        // store rows r0 .. r0+RPT-1 of out_s
        if constexpr (sizeof(T) == 8) {
            double2* o = reinterpret_cast<double2*>(out) + (size_t)s * 12 + r0;
#pragma unroll
            for (int q = 0; q < RPT; ++q) o[q] = make_double2(acc[q].re, acc[q].im);
        } else {
            if constexpr (RPT % 2 == 0) {
                float4* o = reinterpret_cast<float4*>(out) + (size_t)s * 6 + r0 / 2;
#pragma unroll
                for (int q = 0; q < RPT / 2; ++q)
                    o[q] = make_float4(acc[2 * q].re, acc[2 * q].im, acc[2 * q + 1].re, acc[2 * q + 1].im);
            } else {
                float2* o = reinterpret_cast<float2*>(out) + (size_t)s * 12 + r0;
#pragma unroll
                for (int q = 0; q < RPT; ++q) o[q] = make_float2(acc[q].re, acc[q].im);
            }
        }
        if constexpr (EPI == EPI_RV) {
            const cpx<T>* a = reinterpret_cast<const cpx<T>*>(aux) + (size_t)s * 12 + r0;
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const cpx<T> av = a[q];
                d1.x += (double)av.re * acc[q].re + (double)av.im * acc[q].im;
                d1.y += (double)av.re * acc[q].im - (double)av.im * acc[q].re;
            }
        } else if constexpr (EPI == EPI_TS) {
            // <t, s>: s is aux when given (a preconditioned solve applies M to N s, not to s)
            const cpx<T>* a = reinterpret_cast<const cpx<T>*>(aux ? aux : psi) + (size_t)s * 12 + r0;
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const cpx<T> sv = a[q];
                d1.x += (double)acc[q].re * sv.re + (double)acc[q].im * sv.im;
                d1.y += (double)acc[q].re * sv.im - (double)acc[q].im * sv.re;
                d2.x += (double)acc[q].re * acc[q].re + (double)acc[q].im * acc[q].im;
            }
        }
    }
    if constexpr (EPI != EPI_NONE) block_reduce2_store(d1, d2, partial);
}

template <int P, int TPS>
int launch_apply_t(const Geo& g, const void* W, const void* psi, void* out, double mhat, int epi,
                   const void* aux, double2* partial, hipStream_t st) {
    using T = typename Arith<P>::T;
    constexpr int BS = 256;
    const unsigned nb = grid_for((long)g.V * TPS, BS);
    const T* in = reinterpret_cast<const T*>(psi);
    T* o = reinterpret_cast<T*>(out);
    const T* ax = reinterpret_cast<const T*>(aux);
    if (epi == EPI_NONE)
        k_apply<P, TPS, EPI_NONE><<<nb, BS, 0, st>>>(g, W, in, o, mhat, ax, partial);
    else if (epi == EPI_RV)
        k_apply<P, TPS, EPI_RV><<<nb, BS, 0, st>>>(g, W, in, o, mhat, ax, partial);
    else
        k_apply<P, TPS, EPI_TS><<<nb, BS, 0, st>>>(g, W, in, o, mhat, ax, partial);
    OK_LAUNCH_CHECK("k_apply");
    return OK_SUCCESS;
}

// Saved-set W (OK_LAYOUT_SAVED, 14 blocks per site): one thread per site owns all 12 output
// rows.  A forward offset reads its block at x; the backward offset -d reads the forward block
// X of +d at x - d (the site its spinor comes from) and applies gamma5 X^dag gamma5 on the fly.
// Walking X row by row (the rows are what the plane layout stores contiguously per chunk):
//   out_{(q+6)%12} += sg(p, q) conj(X[p][q]) v_{(p+6)%12},  sg = +1 if (p < 6) == (q < 6) else -1,
// which is entry ((q+6)%12, (p+6)%12) of gamma5 X^dag gamma5 (gamma5 swaps the upper and lower
// spin pairs, with a sign on the off-diagonal pair blocks).
template <int P, typename T>
__device__ __forceinline__ void saved_row_chunks(const void* __restrict__ W, int Vs, int ks, int row, int s,
                                                 cpx<T> w[12]) {
    constexpr int per = WL<P>::per, ch = WL<P>::chunks;
#pragma unroll
    for (int j = 0; j < 12 / per; ++j) {
        const size_t cell = ((size_t)(ks * ch + row * (12 / per) + j)) * Vs + s;
        if constexpr (P == OK_F64) {
            const double2 d = ld_stream(reinterpret_cast<const double2*>(W) + cell);
            w[j] = cpx<T>{d.x, d.y};
        } else if constexpr (P == OK_F32) {
            const float4 f = ld_stream(reinterpret_cast<const float4*>(W) + cell);
            w[2 * j] = cpx<T>{f.x, f.y};
            w[2 * j + 1] = cpx<T>{f.z, f.w};
        } else {
            const uint4 u4 = ld_stream(reinterpret_cast<const uint4*>(W) + cell);
            const uint32_t u[4] = {u4.x, u4.y, u4.z, u4.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) w[4 * j + e] = cpx<T>{bf16_to_f32(u[e] & 0xffffu), bf16_to_f32(u[e] >> 16)};
        }
    }
}

template <int P, int EPI>
__global__ void __launch_bounds__(256) k_apply_saved(Geo g, const void* __restrict__ W,
                                                     const typename Arith<P>::T* __restrict__ psi,
                                                     typename Arith<P>::T* __restrict__ out, double mhat_d,
                                                     const typename Arith<P>::T* __restrict__ aux,
                                                     double2* __restrict__ partial) {
    using T = typename Arith<P>::T;
    // contiguous site ranges per XCD: the forward blocks reread as backward blocks stay in L2
    const int s = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const bool live = s < g.V;
    double2 d1{0.0, 0.0}, d2{0.0, 0.0};
    if (live) {
        const T mhat = (T)mhat_d;
        int x, y, z, t;
        site_coords(g, s, x, y, z, t);
        cpx<T> acc[12], v[12], w[12];
        {
            const cpx<T>* c = reinterpret_cast<const cpx<T>*>(psi) + (size_t)s * 12;
#pragma unroll
            for (int q = 0; q < 12; ++q) acc[q] = mhat * c[q];
        }
#pragma unroll 1
        for (int ks = 0; ks < kSaved; ++ks) {   // forward offsets: W_k(x) psi(x + d_k)
            const int k = saved_k(ks);
            const int n = neighbour(g, x, y, z, t, off_d(k, 0), off_d(k, 1), off_d(k, 2), off_d(k, 3));
            ld_spinor(psi, n, v);
#pragma unroll
            for (int r = 0; r < 12; ++r) {
                saved_row_chunks<P, T>(W, g.Vs, ks, r, s, w);
#pragma unroll
                for (int q = 0; q < 12; ++q) cfma(acc[r], w[q], v[q]);
            }
        }
#pragma unroll 1
        for (int ks = 1; ks < kSaved; ++ks) {   // backward offsets: Gamma(W_{+d}(x - d)) psi(x - d)
            const int k = saved_k(ks);
            const int n = neighbour(g, x, y, z, t, -off_d(k, 0), -off_d(k, 1), -off_d(k, 2), -off_d(k, 3));
            ld_spinor(psi, n, v);
#pragma unroll
            for (int p = 0; p < 12; ++p) {
                saved_row_chunks<P, T>(W, g.Vs, ks, p, n, w);
                const cpx<T> vv = v[(p + 6) % 12];
#pragma unroll
                for (int q = 0; q < 12; ++q) {
                    const bool plus = (p < 6) == (q < 6);
                    const cpx<T> c = plus ? conj(w[q]) : -conj(w[q]);
                    cfma(acc[(q + 6) % 12], c, vv);
                }
            }
        }
        if constexpr (sizeof(T) == 8) {
            double2* o = reinterpret_cast<double2*>(out) + (size_t)s * 12;
#pragma unroll
            for (int q = 0; q < 12; ++q) o[q] = make_double2(acc[q].re, acc[q].im);
        } else {
            float4* o = reinterpret_cast<float4*>(out) + (size_t)s * 6;
#pragma unroll
            for (int q = 0; q < 6; ++q)
                o[q] = make_float4(acc[2 * q].re, acc[2 * q].im, acc[2 * q + 1].re, acc[2 * q + 1].im);
        }
        if constexpr (EPI == EPI_RV) {
            const cpx<T>* a = reinterpret_cast<const cpx<T>*>(aux) + (size_t)s * 12;
#pragma unroll
            for (int q = 0; q < 12; ++q) {
                const cpx<T> av = a[q];
                d1.x += (double)av.re * acc[q].re + (double)av.im * acc[q].im;
                d1.y += (double)av.re * acc[q].im - (double)av.im * acc[q].re;
            }
        } else if constexpr (EPI == EPI_TS) {
            const cpx<T>* a = reinterpret_cast<const cpx<T>*>(aux ? aux : psi) + (size_t)s * 12;
#pragma unroll
            for (int q = 0; q < 12; ++q) {
                const cpx<T> sv = a[q];
                d1.x += (double)acc[q].re * sv.re + (double)acc[q].im * sv.im;
                d1.y += (double)acc[q].re * sv.im - (double)acc[q].im * sv.re;
                d2.x += (double)acc[q].re * acc[q].re + (double)acc[q].im * acc[q].im;
            }
        }
    }
    if constexpr (EPI != EPI_NONE) block_reduce2_store(d1, d2, partial);
}

template <int P>
int launch_saved_t(const Geo& g, const void* W, const void* psi, void* out, double mhat, int epi, const void* aux,
                   double2* partial, hipStream_t st) {
    using T = typename Arith<P>::T;
    const unsigned nb = grid_for(g.V, 256);
    const T* in = reinterpret_cast<const T*>(psi);
    T* o = reinterpret_cast<T*>(out);
    const T* ax = reinterpret_cast<const T*>(aux);
    if (epi == EPI_NONE) k_apply_saved<P, EPI_NONE><<<nb, 256, 0, st>>>(g, W, in, o, mhat, ax, partial);
    else if (epi == EPI_RV) k_apply_saved<P, EPI_RV><<<nb, 256, 0, st>>>(g, W, in, o, mhat, ax, partial);
    else k_apply_saved<P, EPI_TS><<<nb, 256, 0, st>>>(g, W, in, o, mhat, ax, partial);
    OK_LAUNCH_CHECK("k_apply_saved");
    return OK_SUCCESS;
}

// FP64 W (plane layout) applied to NR right-hand sides in one pass, out_r = mhat in_r + sum_k W_k in_r(x+d_k):
// each W element is loaded once and multiplied into every right-hand side.  TPS threads per site
// (12/TPS output rows each); the right-hand sides are separate FP64 fields [V][12] named in `cols`.
struct Cols64 {
    const double* in[4];
    double* out[4];
};

template <int NR, int TPS>
__global__ void __launch_bounds__(256) k_apply_m64(Geo g, const void* __restrict__ W, Cols64 cols, double mhat) {
    constexpr int RPT = 12 / TPS, SPW = 64 / TPS;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int grp = lane / SPW;
    const int s = (xcd_tile(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + wave) * SPW + (lane % SPW);
    if (s >= g.V) return;
    const int r0 = grp * RPT;
    int x, y, z, t;
    site_coords(g, s, x, y, z, t);
    c128 acc[NR][RPT];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const double2* c = reinterpret_cast<const double2*>(cols.in[r]) + (size_t)s * 12 + r0;
#pragma unroll
        for (int q = 0; q < RPT; ++q) acc[r][q] = c128{mhat * c[q].x, mhat * c[q].y};
    }
    constexpr int ch = WL<OK_F64>::chunks;
#pragma unroll 1
    for (int k = 0; k < kW; ++k) {
        const int n = neighbour(g, x, y, z, t, off_d(k, 0), off_d(k, 1), off_d(k, 2), off_d(k, 3));
#pragma unroll 2
        for (int j = 0; j < 12; ++j) {
            c128 w[RPT];
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const double2 d = ld_stream(reinterpret_cast<const double2*>(W) +
                                            ((size_t)(k * ch + (r0 + q) * 12 + j)) * g.Vs + s);
                w[q] = c128{d.x, d.y};
            }
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const double2 v = reinterpret_cast<const double2*>(cols.in[r])[(size_t)n * 12 + j];
#pragma unroll
                for (int q = 0; q < RPT; ++q) cfma(acc[r][q], w[q], c128{v.x, v.y});
            }
        }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        double2* o = reinterpret_cast<double2*>(cols.out[r]) + (size_t)s * 12 + r0;
#pragma unroll
        for (int q = 0; q < RPT; ++q) o[q] = make_double2(acc[r][q].re, acc[r][q].im);
    }
}

#ifndef OKINV_M64_TPS
#define OKINV_M64_TPS 4
#endif
constexpr int M64_TPS = OKINV_M64_TPS;

}  // namespace

int launch_apply_m64(const Geo& g, const void* W, const double* const* in, double* const* out, int n, double mhat,
                     hipStream_t st) {
    for (int r0 = 0; r0 < n; r0 += 4) {
        const int nr = std::min(4, n - r0);
        Cols64 c{};
        for (int r = 0; r < nr; ++r) {
            c.in[r] = in[r0 + r];
            c.out[r] = out[r0 + r];
        }
        const unsigned nb = grid_for((long)g.V * M64_TPS, 256);
        switch (nr) {
            case 1: k_apply_m64<1, M64_TPS><<<nb, 256, 0, st>>>(g, W, c, mhat); break;
            case 2: k_apply_m64<2, M64_TPS><<<nb, 256, 0, st>>>(g, W, c, mhat); break;
            case 3: k_apply_m64<3, M64_TPS><<<nb, 256, 0, st>>>(g, W, c, mhat); break;
            default: k_apply_m64<4, M64_TPS><<<nb, 256, 0, st>>>(g, W, c, mhat); break;
        }
        OK_LAUNCH_CHECK("k_apply_m64");
    }
    return OK_SUCCESS;
}

int apply_blocks(const Geo& g, int tps) {
    return (int)grid_for((long)g.V * tps, 256);
}

// Wprec may carry OK_LAYOUT_SAVED or OK_LAYOUT_SIGMA (one thread per site; tps must then be 1)
int launch_apply(const Geo& g, const void* W, int Wprec, const void* psi, void* out, double mhat, int tps,
                 int epi, const void* aux, double2* partial, hipStream_t st) {
    if (Wprec & OK_LAYOUT_SIGMA) return launch_apply_sigma(g, W, Wprec, psi, out, mhat, epi, aux, partial, st);
    if (Wprec & OK_LAYOUT_SAVED) {
        switch (Wprec & 3) {
            case OK_F64: return launch_saved_t<OK_F64>(g, W, psi, out, mhat, epi, aux, partial, st);
            case OK_F32: return launch_saved_t<OK_F32>(g, W, psi, out, mhat, epi, aux, partial, st);
            default: return launch_saved_t<OK_BF16>(g, W, psi, out, mhat, epi, aux, partial, st);
        }
    }
#define OK_TPS_CASES(P)                                                                  \
    switch (tps) {                                                                       \
        case 1: return launch_apply_t<P, 1>(g, W, psi, out, mhat, epi, aux, partial, st); \
        case 2: return launch_apply_t<P, 2>(g, W, psi, out, mhat, epi, aux, partial, st); \
        default: return launch_apply_t<P, 4>(g, W, psi, out, mhat, epi, aux, partial, st); \
    }
    switch (Wprec) {
        case OK_F64: OK_TPS_CASES(OK_F64)
        case OK_F32: OK_TPS_CASES(OK_F32)
        default: OK_TPS_CASES(OK_BF16)
    }
#undef OK_TPS_CASES
}

}  // namespace okinv
