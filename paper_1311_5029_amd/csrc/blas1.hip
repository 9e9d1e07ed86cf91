// BiCGStab vector updates fused with the reductions the recurrence needs next.
//
// The scalars alpha, beta, omega, rho of every right-hand side live in device
// memory (struct Scal) and are produced by one-block "finish" kernels that
// reduce the per-block partial sums in a fixed order, so results are bitwise
// reproducible run to run.  Vector kernels read the scalars they need directly;
// the host only reads the residual norm once per iteration.
#include "common.h"
#include "kernels.h"

namespace okinv {
namespace {

constexpr int BS = 256;

template <typename T>
__device__ __forceinline__ cpx<T> ld(const T* f, size_t i) {
    return reinterpret_cast<const cpx<T>*>(f)[i];
}
template <typename T>
__device__ __forceinline__ void st(T* f, size_t i, cpx<T> v) {
    reinterpret_cast<cpx<T>*>(f)[i] = v;
}
template <typename T>
__device__ __forceinline__ cpx<T> cast(double2 d) {
    return cpx<T>{(T)d.x, (T)d.y};
}
__device__ __forceinline__ double2 cmul2(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cdiv2(double2 a, double2 b) {
    const double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
// accumulate conj(a) b
template <typename T>
__device__ __forceinline__ void dotacc(double2& d, cpx<T> a, cpx<T> b) {
    d.x += (double)a.re * b.re + (double)a.im * b.im;
    d.y += (double)a.re * b.im - (double)a.im * b.re;
}

// p = r + beta (p - omega v)
template <typename T>
__global__ void __launch_bounds__(BS) k_p_update(int n, T* p, const T* r, const T* v, const Scal* sc) {
    const int s = blockIdx.x * BS + threadIdx.x;
    if (s >= n) return;
    const cpx<T> beta = cast<T>(sc->beta), omega = cast<T>(sc->omega);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const size_t i = (size_t)s * 12 + c;
        cpx<T> pv = ld(p, i) - omega * ld(v, i);
        st(p, i, ld(r, i) + beta * pv);
    }
}

// s = r - alpha v
template <typename T>
__global__ void __launch_bounds__(BS) k_s_update(int n, T* s_, const T* r, const T* v, const Scal* sc) {
    const int s = blockIdx.x * BS + threadIdx.x;
    if (s >= n) return;
    const cpx<T> alpha = cast<T>(sc->alpha);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const size_t i = (size_t)s * 12 + c;
        st(s_, i, ld(r, i) - alpha * ld(v, i));
    }
}

// x += alpha p + omega s ; r = s - omega t ; partial <r^, r>, <r, r>
template <typename T>
__global__ void __launch_bounds__(BS) k_xr_update(int n, T* x, T* r, const T* p, const T* sx, const T* s_,
                                                  const T* t, const T* rhat, const Scal* sc, double2* partial) {
    const int s = blockIdx.x * BS + threadIdx.x;
    double2 d1{0, 0}, d2{0, 0};
    if (s < n) {
        const cpx<T> alpha = cast<T>(sc->alpha), omega = cast<T>(sc->omega);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const size_t i = (size_t)s * 12 + c;
            const cpx<T> sv = ld(s_, i);
            st(x, i, ld(x, i) + alpha * ld(p, i) + omega * ld(sx, i));
            const cpx<T> rv = sv - omega * ld(t, i);
            st(r, i, rv);
            dotacc(d1, ld(rhat, i), rv);
            dotacc(d2, rv, rv);
        }
    }
    block_reduce2_store(d1, d2, partial);
}

// partial <a, b>, <b, b>
template <typename T>
__global__ void __launch_bounds__(BS) k_dot(int n, const T* a, const T* b, double2* partial) {
    const int s = blockIdx.x * BS + threadIdx.x;
    double2 d1{0, 0}, d2{0, 0};
    if (s < n) {
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const size_t i = (size_t)s * 12 + c;
            const cpx<T> bv = ld(b, i);
            dotacc(d1, ld(a, i), bv);
            dotacc(d2, bv, bv);
        }
    }
    block_reduce2_store(d1, d2, partial);
}

// r64 = xi - t64 ; rlo = (float) r64 ; partial <r64, r64> (in the second slot)
__global__ void __launch_bounds__(BS) k_residual(int n, const double* xi, const double* t64, double* r64, float* rlo,
                                                 double2* partial) {
    const int s = blockIdx.x * BS + threadIdx.x;
    double2 d1{0, 0}, d2{0, 0};
    if (s < n) {
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const size_t i = (size_t)s * 12 + c;
            const c128 rv = ld(xi, i) - ld(t64, i);
            st(r64, i, rv);
            if (rlo) st(rlo, i, c64{(float)rv.re, (float)rv.im});
            dotacc(d2, rv, rv);
        }
    }
    block_reduce2_store(d1, d2, partial);
}

__global__ void __launch_bounds__(BS) k_accum_x(int n, double* x64, float* xlo) {
    const int s = blockIdx.x * BS + threadIdx.x;
    if (s >= n) return;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const size_t i = (size_t)s * 12 + c;
        const c64 l = ld(xlo, i);
        st(x64, i, ld(x64, i) + c128{(double)l.re, (double)l.im});
        st(xlo, i, c64{0.0f, 0.0f});
    }
}

template <typename T>
__global__ void __launch_bounds__(BS) k_copy(int n, T* dst, const T* src) {
    const int s = blockIdx.x * BS + threadIdx.x;
    if (s >= n) return;
#pragma unroll
    for (int c = 0; c < 12; ++c) st(dst, (size_t)s * 12 + c, ld(src, (size_t)s * 12 + c));
}

template <typename T>
__global__ void __launch_bounds__(BS) k_zero(int n, T* dst) {
    const int s = blockIdx.x * BS + threadIdx.x;
    if (s >= n) return;
#pragma unroll
    for (int c = 0; c < 12; ++c) st(dst, (size_t)s * 12 + c, cpx<T>{(T)0, (T)0});
}

// ---- CG on the normal equations M^dag M x = M^dag xi (M^dag = gamma5 M gamma5) ----------
// gamma5 = [[0, -i], [i, 0]] on the upper (spins 0, 1) and lower (spins 2, 3) spin pairs:
// (gamma5 psi)_u = -i psi_d, (gamma5 psi)_d = i psi_u.
__device__ __forceinline__ double2 g5_comp(const double2* f, size_t site, int c) {
    const double2 o = f[site * 12 + (c + 6) % 12];
    return c < 6 ? make_double2(o.y, -o.x) : make_double2(-o.y, o.x);   // -i o  |  i o
}

// g = gamma5 r ; partial (0, ||r||^2)
__global__ void __launch_bounds__(BS) k_cg_gamma5(int n, double2* g, const double2* r, double2* partial) {
    const int s = blockIdx.x * BS + threadIdx.x;
    double2 d{0, 0};
    if (s < n) {
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const double2 v = r[(size_t)s * 12 + c];
            d.x += v.x * v.x + v.y * v.y;
            g[(size_t)s * 12 + c] = g5_comp(r, s, c);
        }
    }
    block_reduce2_store(double2{0, 0}, d, partial);
}

// x += alpha p ; r -= alpha w ; g = gamma5 r ; partial (0, ||r||^2)   (alpha real)
__global__ void __launch_bounds__(BS) k_cg_xr(int n, double2* x, double2* r, const double2* p, const double2* w,
                                              double2* g, const Scal* sc, double2* partial) {
    const int s = blockIdx.x * BS + threadIdx.x;
    double2 d{0, 0};
    if (s < n) {
        const double a = sc->alpha.x;
        double2 rn[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const size_t i = (size_t)s * 12 + c;
            const double2 pv = p[i], wv = w[i], xv = x[i], rv = r[i];
            x[i] = make_double2(fma(a, pv.x, xv.x), fma(a, pv.y, xv.y));
            rn[c] = make_double2(fma(-a, wv.x, rv.x), fma(-a, wv.y, rv.y));
            r[i] = rn[c];
            d.x += rn[c].x * rn[c].x + rn[c].y * rn[c].y;
        }
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const double2 o = rn[(c + 6) % 12];
            g[(size_t)s * 12 + c] = c < 6 ? make_double2(o.y, -o.x) : make_double2(-o.y, o.x);
        }
    }
    block_reduce2_store(double2{0, 0}, d, partial);
}

// p = gamma5 z' + beta p   (beta real; z' = M gamma5 r, so gamma5 z' = M^dag r)
__global__ void __launch_bounds__(BS) k_cg_p(int n, double2* p, const double2* zp, const Scal* sc) {
    const int s = blockIdx.x * BS + threadIdx.x;
    if (s >= n) return;
    const double b = sc->beta.x;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const size_t i = (size_t)s * 12 + c;
        const double2 z = g5_comp(zp, s, c), pv = p[i];
        p[i] = make_double2(fma(b, pv.x, z.x), fma(b, pv.y, z.y));
    }
}

// One block: fixed-order reduction of nb partial pairs, then the scalar update.
__global__ void __launch_bounds__(BS) k_finish(int kind, int nb, const double2* partial, Scal* sc) {
    double2 d1{0, 0}, d2{0, 0};
    for (int i = threadIdx.x; i < nb; i += BS) {
        const double2 a = partial[2 * i], b = partial[2 * i + 1];
        d1.x += a.x;
        d1.y += a.y;
        d2.x += b.x;
        d2.y += b.y;
    }
    block_reduce2(d1, d2);
    if (threadIdx.x != 0) return;
    Scal& S = *sc;
    const double tiny = 1e-300;
    switch (kind) {
        case FIN_ALPHA: {
            S.rv = d1;
            const double m = d1.x * d1.x + d1.y * d1.y;
            if (!(m > tiny)) {
                S.flags |= 1;
                S.alpha = make_double2(0.0, 0.0);
            } else {
                S.alpha = cdiv2(S.rho, d1);
            }
            break;
        }
        case FIN_OMEGA: {
            S.ts = d1;
            S.tt = d2.x;
            if (!(d2.x > tiny)) {
                S.flags |= 1;
                S.omega = make_double2(0.0, 0.0);
            } else {
                S.omega = make_double2(d1.x / d2.x, d1.y / d2.x);
            }
            break;
        }
        case FIN_RHO:
        case FIN_RHO_REPLACE: {
            if (kind == FIN_RHO) S.rho_old = S.rho;
            S.rho = d1;
            S.rr = d2.x;
            const double mo = S.omega.x * S.omega.x + S.omega.y * S.omega.y;
            const double mr = S.rho_old.x * S.rho_old.x + S.rho_old.y * S.rho_old.y;
            const double mrho = d1.x * d1.x + d1.y * d1.y;
            if (!(mo > tiny) || !(mr > tiny) || !(mrho > 1e-60 * d2.x * d2.x)) {
                S.flags |= 1;
                S.beta = make_double2(0.0, 0.0);
            } else {
                S.beta = cmul2(cdiv2(S.rho, S.rho_old), cdiv2(S.alpha, S.omega));
            }
            break;
        }
        case FIN_INIT: {
            S.rho = d1;
            S.rr = d2.x;
            S.rho_old = make_double2(1.0, 0.0);
            S.alpha = make_double2(1.0, 0.0);
            S.omega = make_double2(1.0, 0.0);
            S.beta = make_double2(0.0, 0.0);
            S.flags = 0;
            break;
        }
        case FIN_CG_INIT: {   // d2.x = ||M^dag r||^2
            S.rho = make_double2(d2.x, 0.0);
            S.beta = make_double2(0.0, 0.0);
            S.flags = 0;
            break;
        }
        case FIN_CG_ALPHA: {   // d2.x = ||M p||^2
            S.tt = d2.x;
            if (!(d2.x > tiny)) {
                S.flags |= 1;
                S.alpha = make_double2(0.0, 0.0);
            } else {
                S.alpha = make_double2(S.rho.x / d2.x, 0.0);
            }
            break;
        }
        case FIN_CG_BETA: {   // d2.x = ||M^dag r||^2 of the new residual
            if (!(S.rho.x > tiny)) {
                S.flags |= 1;
                S.beta = make_double2(0.0, 0.0);
            } else {
                S.beta = make_double2(d2.x / S.rho.x, 0.0);
            }
            S.rho = make_double2(d2.x, 0.0);
            break;
        }
        case FIN_CG_RR: {
            S.rr = d2.x;
            break;
        }
        default: {   // FIN_TRUE
            S.rr_true = d2.x;
            break;
        }
    }
}

}  // namespace

int blas_blocks(const Geo& g) { return (int)grid_for(g.V, BS); }

template <typename T> static T* tp(void* p) { return reinterpret_cast<T*>(p); }
template <typename T> static const T* tp(const void* p) { return reinterpret_cast<const T*>(p); }

int launch_p_update(const Geo& g, bool f64, void* p, const void* r, const void* v, const Scal* sc, hipStream_t st) {
    if (f64) k_p_update<double><<<grid_for(g.V, BS), BS, 0, st>>>(g.V, tp<double>(p), tp<double>(r), tp<double>(v), sc);
    else k_p_update<float><<<grid_for(g.V, BS), BS, 0, st>>>(g.V, tp<float>(p), tp<float>(r), tp<float>(v), sc);
    OK_LAUNCH_CHECK("k_p_update");
    return OK_SUCCESS;
}

int launch_s_update(const Geo& g, bool f64, void* s, const void* r, const void* v, const Scal* sc, hipStream_t st) {
    if (f64) k_s_update<double><<<grid_for(g.V, BS), BS, 0, st>>>(g.V, tp<double>(s), tp<double>(r), tp<double>(v), sc);
    else k_s_update<float><<<grid_for(g.V, BS), BS, 0, st>>>(g.V, tp<float>(s), tp<float>(r), tp<float>(v), sc);
    OK_LAUNCH_CHECK("k_s_update");
    return OK_SUCCESS;
}

int launch_xr_update(const Geo& g, bool f64, void* x, void* r, const void* p, const void* sx, const void* s,
                     const void* t, const void* rhat, const Scal* sc, double2* partial, hipStream_t st) {
    if (f64)
        k_xr_update<double><<<grid_for(g.V, BS), BS, 0, st>>>(g.V, tp<double>(x), tp<double>(r), tp<double>(p),
                                                              tp<double>(sx), tp<double>(s), tp<double>(t),
                                                              tp<double>(rhat), sc, partial);
    else
        k_xr_update<float><<<grid_for(g.V, BS), BS, 0, st>>>(g.V, tp<float>(x), tp<float>(r), tp<float>(p),
                                                             tp<float>(sx), tp<float>(s), tp<float>(t),
                                                             tp<float>(rhat), sc, partial);
    OK_LAUNCH_CHECK("k_xr_update");
    return OK_SUCCESS;
}

int launch_dot_rr(const Geo& g, bool f64, const void* rhat, const void* r, double2* partial, hipStream_t st) {
    if (f64) k_dot<double><<<grid_for(g.V, BS), BS, 0, st>>>(g.V, tp<double>(rhat), tp<double>(r), partial);
    else k_dot<float><<<grid_for(g.V, BS), BS, 0, st>>>(g.V, tp<float>(rhat), tp<float>(r), partial);
    OK_LAUNCH_CHECK("k_dot");
    return OK_SUCCESS;
}

int launch_norm64(const Geo& g, const double* a, double2* partial, hipStream_t st) {
    k_dot<double><<<grid_for(g.V, BS), BS, 0, st>>>(g.V, a, a, partial);
    OK_LAUNCH_CHECK("k_dot");
    return OK_SUCCESS;
}

int launch_finish(int kind, int nblocks, const double2* partial, Scal* sc, hipStream_t st) {
    k_finish<<<1, BS, 0, st>>>(kind, nblocks, partial, sc);
    OK_LAUNCH_CHECK("k_finish");
    return OK_SUCCESS;
}

int launch_residual(const Geo& g, const double* xi, const double* t64, double* r64, float* rlo, double2* partial,
                    hipStream_t st) {
    k_residual<<<grid_for(g.V, BS), BS, 0, st>>>(g.V, xi, t64, r64, rlo, partial);
    OK_LAUNCH_CHECK("k_residual");
    return OK_SUCCESS;
}

int launch_accum_x(const Geo& g, double* x64, float* xlo, hipStream_t st) {
    k_accum_x<<<grid_for(g.V, BS), BS, 0, st>>>(g.V, x64, xlo);
    OK_LAUNCH_CHECK("k_accum_x");
    return OK_SUCCESS;
}

int launch_copy(const Geo& g, bool f64, void* dst, const void* src, hipStream_t st) {
    if (f64) k_copy<double><<<grid_for(g.V, BS), BS, 0, st>>>(g.V, tp<double>(dst), tp<double>(src));
    else k_copy<float><<<grid_for(g.V, BS), BS, 0, st>>>(g.V, tp<float>(dst), tp<float>(src));
    OK_LAUNCH_CHECK("k_copy");
    return OK_SUCCESS;
}

int launch_zero(const Geo& g, bool f64, void* dst, hipStream_t st) {
    if (f64) k_zero<double><<<grid_for(g.V, BS), BS, 0, st>>>(g.V, tp<double>(dst));
    else k_zero<float><<<grid_for(g.V, BS), BS, 0, st>>>(g.V, tp<float>(dst));
    OK_LAUNCH_CHECK("k_zero");
    return OK_SUCCESS;
}

int launch_cg_gamma5(const Geo& g, double* out, const double* r, double2* partial, hipStream_t st) {
    k_cg_gamma5<<<grid_for(g.V, BS), BS, 0, st>>>(g.V, reinterpret_cast<double2*>(out),
                                                   reinterpret_cast<const double2*>(r), partial);
    OK_LAUNCH_CHECK("k_cg_gamma5");
    return OK_SUCCESS;
}

int launch_cg_xr(const Geo& g, double* x, double* r, const double* p, const double* w, double* gr, const Scal* sc,
                 double2* partial, hipStream_t st) {
    k_cg_xr<<<grid_for(g.V, BS), BS, 0, st>>>(g.V, reinterpret_cast<double2*>(x), reinterpret_cast<double2*>(r),
                                               reinterpret_cast<const double2*>(p), reinterpret_cast<const double2*>(w),
                                               reinterpret_cast<double2*>(gr), sc, partial);
    OK_LAUNCH_CHECK("k_cg_xr");
    return OK_SUCCESS;
}

int launch_cg_p(const Geo& g, double* p, const double* zp, const Scal* sc, hipStream_t st) {
    k_cg_p<<<grid_for(g.V, BS), BS, 0, st>>>(g.V, reinterpret_cast<double2*>(p), reinterpret_cast<const double2*>(zp),
                                              sc);
    OK_LAUNCH_CHECK("k_cg_p");
    return OK_SUCCESS;
}

}  // namespace okinv
