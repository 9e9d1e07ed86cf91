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

// The vector kernels run one thread per complex component (ne = 12 V of them), so that
// consecutive lanes touch consecutive addresses.

// p = r + beta (p - omega v)
template <typename T>
__global__ void __launch_bounds__(BS) k_p_update(long ne, T* p, const T* r, const T* v, const Scal* sc) {
    const long i = (long)blockIdx.x * BS + threadIdx.x;
    if (i >= ne) return;
    const cpx<T> beta = cast<T>(sc->beta), omega = cast<T>(sc->omega);
    const cpx<T> pv = ld(p, i) - omega * ld(v, i);
    st(p, i, ld(r, i) + beta * pv);
}

// s = r - alpha v
template <typename T>
__global__ void __launch_bounds__(BS) k_s_update(long ne, T* s_, const T* r, const T* v, const Scal* sc) {
    const long i = (long)blockIdx.x * BS + threadIdx.x;
    if (i >= ne) return;
    const cpx<T> alpha = cast<T>(sc->alpha);
    st(s_, i, ld(r, i) - alpha * ld(v, i));
}

// x += alpha p + omega s ; r = s - omega t ; partial <r^, r>, <r, r>
template <typename T>
__global__ void __launch_bounds__(BS) k_xr_update(long ne, T* x, T* r, const T* p, const T* sx, const T* s_,
                                                  const T* t, const T* rhat, const Scal* sc, double2* partial) {
    const long i = (long)blockIdx.x * BS + threadIdx.x;
    double2 d1{0, 0}, d2{0, 0};
    if (i < ne) {
        const cpx<T> alpha = cast<T>(sc->alpha), omega = cast<T>(sc->omega);
        const cpx<T> sv = ld(s_, i);
        st(x, i, ld(x, i) + alpha * ld(p, i) + omega * ld(sx, i));
        const cpx<T> rv = sv - omega * ld(t, i);
        st(r, i, rv);
        dotacc(d1, ld(rhat, i), rv);
        dotacc(d2, rv, rv);
    }
    block_reduce2_store(d1, d2, partial);
}

// partial <a, b>, <b, b>
template <typename T>
__global__ void __launch_bounds__(BS) k_dot(long ne, const T* a, const T* b, double2* partial) {
    const long i = (long)blockIdx.x * BS + threadIdx.x;
    double2 d1{0, 0}, d2{0, 0};
    if (i < ne) {
        const cpx<T> bv = ld(b, i);
        dotacc(d1, ld(a, i), bv);
        dotacc(d2, bv, bv);
    }
    block_reduce2_store(d1, d2, partial);
}

// r64 = xi - t64 ; rlo = (float) r64 ; partial <r64, r64> (in the second slot)
__global__ void __launch_bounds__(BS) k_residual(long ne, const double* xi, const double* t64, double* r64, float* rlo,
                                                 double2* partial) {
    const long i = (long)blockIdx.x * BS + threadIdx.x;
    double2 d1{0, 0}, d2{0, 0};
    if (i < ne) {
        const c128 rv = ld(xi, i) - ld(t64, i);
        st(r64, i, rv);
        if (rlo) st(rlo, i, c64{(float)rv.re, (float)rv.im});
        dotacc(d2, rv, rv);
    }
    block_reduce2_store(d1, d2, partial);
}

__global__ void __launch_bounds__(BS) k_accum_x(long ne, double* x64, float* xlo) {
    const long i = (long)blockIdx.x * BS + threadIdx.x;
    if (i >= ne) return;
    const c64 l = ld(xlo, i);
    st(x64, i, ld(x64, i) + c128{(double)l.re, (double)l.im});
    st(xlo, i, c64{0.0f, 0.0f});
}

template <typename T>
__global__ void __launch_bounds__(BS) k_copy(long ne, T* dst, const T* src) {
    const long i = (long)blockIdx.x * BS + threadIdx.x;
    if (i < ne) st(dst, i, ld(src, i));
}

template <typename T>
__global__ void __launch_bounds__(BS) k_zero(long ne, T* dst) {
    const long i = (long)blockIdx.x * BS + threadIdx.x;
    if (i < ne) st(dst, i, cpx<T>{(T)0, (T)0});
}

// ---- CG on the normal equations M^dag M x = M^dag xi (M^dag = gamma5 M gamma5) ----------
// gamma5 = [[0, -i], [i, 0]] on the upper (spins 0, 1) and lower (spins 2, 3) spin pairs:
// (gamma5 psi)_u = -i psi_d, (gamma5 psi)_d = i psi_u.  Component c of a site pairs with
// component (c + 6) % 12 of the same site.
__device__ __forceinline__ long g5_partner(long i) {
    const int c = (int)(i % 12);
    return i - c + (c + 6) % 12;
}
// the entry at the partner of component i that gamma5 makes from the value o at i
__device__ __forceinline__ double2 g5_to_partner(long i, double2 o) {
    return (i % 12) < 6 ? make_double2(-o.y, o.x) : make_double2(o.y, -o.x);   // i o (lower)  |  -i o (upper)
}

// g = gamma5 r ; partial (0, ||r||^2)
__global__ void __launch_bounds__(BS) k_cg_gamma5(long ne, double2* g, const double2* r, double2* partial) {
    const long i = (long)blockIdx.x * BS + threadIdx.x;
    double2 d{0, 0};
    if (i < ne) {
        const double2 v = r[i];
        d.x = v.x * v.x + v.y * v.y;
        g[g5_partner(i)] = g5_to_partner(i, v);
    }
    block_reduce2_store(double2{0, 0}, d, partial);
}

// x += alpha p ; r -= alpha w ; g = gamma5 r ; partial (0, ||r||^2)   (alpha real).  Each thread
// writes the gamma5 entry its new r makes at the partner component, so no thread reads an r that
// another one updates.
__global__ void __launch_bounds__(BS) k_cg_xr(long ne, double2* x, double2* r, const double2* p, const double2* w,
                                              double2* g, const Scal* sc, double2* partial) {
    const long i = (long)blockIdx.x * BS + threadIdx.x;
    double2 d{0, 0};
    if (i < ne) {
        const double a = sc->alpha.x;
        const double2 pv = p[i], wv = w[i], xv = x[i], rv = r[i];
        x[i] = make_double2(fma(a, pv.x, xv.x), fma(a, pv.y, xv.y));
        const double2 rn = make_double2(fma(-a, wv.x, rv.x), fma(-a, wv.y, rv.y));
        r[i] = rn;
        d.x = rn.x * rn.x + rn.y * rn.y;
        g[g5_partner(i)] = g5_to_partner(i, rn);
    }
    block_reduce2_store(double2{0, 0}, d, partial);
}

// p = gamma5 z' + beta p   (beta real; z' = M gamma5 r, so gamma5 z' = M^dag r)
__global__ void __launch_bounds__(BS) k_cg_p(long ne, double2* p, const double2* zp, const Scal* sc) {
    const long i = (long)blockIdx.x * BS + threadIdx.x;
    if (i >= ne) return;
    const double b = sc->beta.x;
    const long j = g5_partner(i);
    const double2 z = g5_to_partner(j, zp[j]), pv = p[i];
    p[i] = make_double2(fma(b, pv.x, z.x), fma(b, pv.y, z.y));
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

int blas_blocks(const Geo& g) { return (int)grid_for(12L * g.V, BS); }

template <typename T> static T* tp(void* p) { return reinterpret_cast<T*>(p); }
template <typename T> static const T* tp(const void* p) { return reinterpret_cast<const T*>(p); }

int launch_p_update(const Geo& g, bool f64, void* p, const void* r, const void* v, const Scal* sc, hipStream_t st) {
    if (f64) k_p_update<double><<<grid_for(12L * g.V, BS), BS, 0, st>>>(12L * g.V, tp<double>(p), tp<double>(r), tp<double>(v), sc);
    else k_p_update<float><<<grid_for(12L * g.V, BS), BS, 0, st>>>(12L * g.V, tp<float>(p), tp<float>(r), tp<float>(v), sc);
    OK_LAUNCH_CHECK("k_p_update");
    return OK_SUCCESS;
}

int launch_s_update(const Geo& g, bool f64, void* s, const void* r, const void* v, const Scal* sc, hipStream_t st) {
    if (f64) k_s_update<double><<<grid_for(12L * g.V, BS), BS, 0, st>>>(12L * g.V, tp<double>(s), tp<double>(r), tp<double>(v), sc);
    else k_s_update<float><<<grid_for(12L * g.V, BS), BS, 0, st>>>(12L * g.V, tp<float>(s), tp<float>(r), tp<float>(v), sc);
    OK_LAUNCH_CHECK("k_s_update");
    return OK_SUCCESS;
}

int launch_xr_update(const Geo& g, bool f64, void* x, void* r, const void* p, const void* sx, const void* s,
                     const void* t, const void* rhat, const Scal* sc, double2* partial, hipStream_t st) {
    if (f64)
        k_xr_update<double><<<grid_for(12L * g.V, BS), BS, 0, st>>>(12L * g.V, tp<double>(x), tp<double>(r), tp<double>(p),
                                                              tp<double>(sx), tp<double>(s), tp<double>(t),
                                                              tp<double>(rhat), sc, partial);
    else
        k_xr_update<float><<<grid_for(12L * g.V, BS), BS, 0, st>>>(12L * g.V, tp<float>(x), tp<float>(r), tp<float>(p),
                                                             tp<float>(sx), tp<float>(s), tp<float>(t),
                                                             tp<float>(rhat), sc, partial);
    OK_LAUNCH_CHECK("k_xr_update");
    return OK_SUCCESS;
}

int launch_dot_rr(const Geo& g, bool f64, const void* rhat, const void* r, double2* partial, hipStream_t st) {
    if (f64) k_dot<double><<<grid_for(12L * g.V, BS), BS, 0, st>>>(12L * g.V, tp<double>(rhat), tp<double>(r), partial);
    else k_dot<float><<<grid_for(12L * g.V, BS), BS, 0, st>>>(12L * g.V, tp<float>(rhat), tp<float>(r), partial);
    OK_LAUNCH_CHECK("k_dot");
    return OK_SUCCESS;
}

int launch_norm64(const Geo& g, const double* a, double2* partial, hipStream_t st) {
    k_dot<double><<<grid_for(12L * g.V, BS), BS, 0, st>>>(12L * g.V, a, a, partial);
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
    k_residual<<<grid_for(12L * g.V, BS), BS, 0, st>>>(12L * g.V, xi, t64, r64, rlo, partial);
    OK_LAUNCH_CHECK("k_residual");
    return OK_SUCCESS;
}

int launch_accum_x(const Geo& g, double* x64, float* xlo, hipStream_t st) {
    k_accum_x<<<grid_for(12L * g.V, BS), BS, 0, st>>>(12L * g.V, x64, xlo);
    OK_LAUNCH_CHECK("k_accum_x");
    return OK_SUCCESS;
}

int launch_copy(const Geo& g, bool f64, void* dst, const void* src, hipStream_t st) {
    if (f64) k_copy<double><<<grid_for(12L * g.V, BS), BS, 0, st>>>(12L * g.V, tp<double>(dst), tp<double>(src));
    else k_copy<float><<<grid_for(12L * g.V, BS), BS, 0, st>>>(12L * g.V, tp<float>(dst), tp<float>(src));
    OK_LAUNCH_CHECK("k_copy");
    return OK_SUCCESS;
}

int launch_zero(const Geo& g, bool f64, void* dst, hipStream_t st) {
    if (f64) k_zero<double><<<grid_for(12L * g.V, BS), BS, 0, st>>>(12L * g.V, tp<double>(dst));
    else k_zero<float><<<grid_for(12L * g.V, BS), BS, 0, st>>>(12L * g.V, tp<float>(dst));
    OK_LAUNCH_CHECK("k_zero");
    return OK_SUCCESS;
}

int launch_cg_gamma5(const Geo& g, double* out, const double* r, double2* partial, hipStream_t st) {
    k_cg_gamma5<<<grid_for(12L * g.V, BS), BS, 0, st>>>(12L * g.V, reinterpret_cast<double2*>(out),
                                                   reinterpret_cast<const double2*>(r), partial);
    OK_LAUNCH_CHECK("k_cg_gamma5");
    return OK_SUCCESS;
}

int launch_cg_xr(const Geo& g, double* x, double* r, const double* p, const double* w, double* gr, const Scal* sc,
                 double2* partial, hipStream_t st) {
    k_cg_xr<<<grid_for(12L * g.V, BS), BS, 0, st>>>(12L * g.V, reinterpret_cast<double2*>(x), reinterpret_cast<double2*>(r),
                                               reinterpret_cast<const double2*>(p), reinterpret_cast<const double2*>(w),
                                               reinterpret_cast<double2*>(gr), sc, partial);
    OK_LAUNCH_CHECK("k_cg_xr");
    return OK_SUCCESS;
}

int launch_cg_p(const Geo& g, double* p, const double* zp, const Scal* sc, hipStream_t st) {
    k_cg_p<<<grid_for(12L * g.V, BS), BS, 0, st>>>(12L * g.V, reinterpret_cast<double2*>(p), reinterpret_cast<const double2*>(zp),
                                              sc);
    OK_LAUNCH_CHECK("k_cg_p");
    return OK_SUCCESS;
}

}  // namespace okinv
