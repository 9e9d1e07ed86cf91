// BiCGStab driver (Sec. 2.3: the general-purpose "bi-stabilized CG" inverter,
// with mixed precision "in single or double precision, as appropriate").
//
// Plain form: FP64 fields and FP64 W.  Per iteration (van der Vorst):
//   p = r + beta (p - omega v);  v = M p  [+ <r^, v>];  alpha = rho / <r^, v>;
//   s = r - alpha v;             t = M s  [+ <t, s>, <t, t>];  omega = <t,s>/<t,t>;
//   x += alpha p + omega s;  r = s - omega t  [+ <r^, r>, <r, r>];  beta = ...
// The bracketed reductions are fused into the kernel that produces the vector;
// the scalars stay on the device and the host reads only ||r||^2 per iteration.
//
// Mixed form: the same recurrence in FP32 fields with the FP32 (or BF16) W,
// plus reliable updates: when the iterated residual has fallen by delta below
// its maximum since the last update, x64 += x32, r = xi - M64 x64 in FP64 and
// the recurrence continues from that residual.  Convergence is always decided
// by the FP64 true residual ||xi - M64 x|| / ||xi||.
//
// Right preconditioning by the learned network N (low-precision solves only):
// the same recurrence on M N y = xi with x = N y carried directly, i.e.
//   p^ = N p, v = M p^, s^ = N s, t = M s^, x += alpha p^ + omega s^,
// so r stays the residual of M x = xi and the reliable updates and the
// stopping test are unchanged.  A breakdown, a stall or a non-finite value in
// the preconditioned recurrence hands the right-hand side to the
// unpreconditioned solve, which continues from the last FP64 iterate.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "common.h"
#include "kernels.h"
#include "wlayout.h"

namespace okinv {
namespace {

// internal outcome of a preconditioned solve: continue without the network
constexpr int kFallback = 100;

struct Work {
    Scal* sc;
    double2* partial;
    int npart;
    // FP64 fields (plain: r rhat p v s t ; mixed: r64 t64)
    double* f64[6];
    // FP32 fields (mixed: xlo r rhat p v s t ; with a network also p^ s^)
    float* f32[9];
    void* netw;   // network ping-pong fields
};

size_t align256(size_t n) { return (n + 255) / 256 * 256; }

size_t layout(const Geo& g, bool mixed, int net_layers, char* base, Work* w) {
    const int tps = std::max(stencil_tps(OK_F64), stencil_tps(OK_F32));
    const int npart = std::max({apply_blocks(g, 1), apply_blocks(g, 2), apply_blocks(g, 4), blas_blocks(g), tps});
    size_t off = 0;
    auto take = [&](size_t n) {
        char* p = base ? base + off : nullptr;
        off += align256(n);
        return p;
    };
    Work tmp;
    Work& W = w ? *w : tmp;
    W.sc = reinterpret_cast<Scal*>(take(sizeof(Scal)));
    W.partial = reinterpret_cast<double2*>(take((size_t)npart * 2 * sizeof(double2)));
    W.npart = npart;
    const size_t s64 = (size_t)g.V * 12 * 16, s32 = (size_t)g.V * 12 * 8;
    for (auto& f : W.f64) f = nullptr;
    for (auto& f : W.f32) f = nullptr;
    if (!mixed) {
        for (int i = 0; i < 6; ++i) W.f64[i] = reinterpret_cast<double*>(take(s64));
    } else {
        for (int i = 0; i < 2; ++i) W.f64[i] = reinterpret_cast<double*>(take(s64));
        for (int i = 0; i < (net_layers ? 9 : 7); ++i) W.f32[i] = reinterpret_cast<float*>(take(s32));
    }
    W.netw = net_layers ? take(net_apply_work_bytes(g, net_layers, 1)) : nullptr;
    return off;
}

#define OK_TRY(expr)                      \
    do {                                  \
        int _r = (expr);                  \
        if (_r != OK_SUCCESS) return _r;  \
    } while (0)

struct Ctx {
    Geo g;
    const ok_coeffs* c;
    const ok_solver_params* p;
    const void* W64;
    const void* Wlo;
    int Wlo_prec;
    const ok_net* net;   // the preconditioner of the current solve, or NULL
    hipStream_t st;
    Work w;
    int W64_prec;        // OK_F64 | the layout of W64
    int tps64, tpslo;
};

int apply_net(Ctx& C, const float* in, float* out, int nf, bool inner, void* work) {
    return net_apply(C.g, C.net->n_layers, C.net->d_params, C.net->d_T, in, out, nf, inner, work, C.st);
}

int read_scal(Ctx& C, Scal* h) {
    OK_HIP(hipMemcpyAsync(h, C.w.sc, sizeof(Scal), hipMemcpyDeviceToHost, C.st));
    OK_HIP(hipStreamSynchronize(C.st));
    return OK_SUCCESS;
}

// reduce the partial sums of the kernel that just ran (nblocks of them)
int fin(Ctx& C, int kind, int nblocks) { return launch_finish(kind, nblocks, C.w.partial, C.w.sc, C.st); }
int fin_blas(Ctx& C, int kind) { return fin(C, kind, blas_blocks(C.g)); }

// t = M64 x ; r64 = xi - t ; rlo = (float) r64 (if given) ; returns ||r64||^2 on the host
int true_residual(Ctx& C, const double* xi, const double* x, double* t, double* r64, float* rlo, double* rr,
                  ok_solver_stats* S) {
    OK_TRY(launch_apply(C.g, C.W64, C.W64_prec, x, t, C.c->mhat, C.tps64, EPI_NONE, nullptr, nullptr, C.st));
    S->matvec_hi++;
    OK_TRY(launch_residual(C.g, xi, t, r64, rlo, C.w.partial, C.st));
    OK_TRY(fin_blas(C, FIN_TRUE));
    Scal h;
    OK_TRY(read_scal(C, &h));
    *rr = h.rr_true;
    return OK_SUCCESS;
}

int source_norm(Ctx& C, const double* xi, double* xn) {
    OK_TRY(launch_norm64(C.g, xi, C.w.partial, C.st));
    OK_TRY(fin_blas(C, FIN_TRUE));
    Scal h;
    OK_TRY(read_scal(C, &h));
    *xn = std::sqrt(h.rr_true);
    return OK_SUCCESS;
}

// One BiCGStab iteration on fields of type T (f64 selects double) with operator (W, prec, tps).
// With C.net (FP32 fields only) p^ and s^ are C.w.f32[7] and [8].
int iterate(Ctx& C, bool f64, const void* W, int prec, int tps, void* x, void* r, void* rhat, void* p, void* v,
            void* s, void* t) {
    const Geo& g = C.g;
    void* ph = p;
    void* sh = s;
    if (C.net) {
        ph = C.w.f32[7];
        sh = C.w.f32[8];
    }
    OK_TRY(launch_p_update(g, f64, p, r, v, C.w.sc, C.st));
    if (C.net) OK_TRY(apply_net(C, static_cast<float*>(p), static_cast<float*>(ph), 1, false, C.w.netw));
    OK_TRY(launch_apply(g, W, prec, ph, v, C.c->mhat, tps, EPI_RV, rhat, C.w.partial, C.st));
    OK_TRY(fin(C, FIN_ALPHA, apply_blocks(g, tps)));
    OK_TRY(launch_s_update(g, f64, s, r, v, C.w.sc, C.st));
    if (C.net) OK_TRY(apply_net(C, static_cast<float*>(s), static_cast<float*>(sh), 1, false, C.w.netw));
    // omega = <t, s> / <t, t> with the unpreconditioned s (the operator's input is N s when preconditioned)
    OK_TRY(launch_apply(g, W, prec, sh, t, C.c->mhat, tps, EPI_TS, C.net ? s : nullptr, C.w.partial, C.st));
    OK_TRY(fin(C, FIN_OMEGA, apply_blocks(g, tps)));
    OK_TRY(launch_xr_update(g, f64, x, r, ph, sh, s, t, rhat, C.w.sc, C.w.partial, C.st));
    OK_TRY(fin_blas(C, FIN_RHO));
    return OK_SUCCESS;
}

// restart the Krylov recurrence from the current residual r: r^ = r, p = v = 0
int restart_from(Ctx& C, bool f64, void* r, void* rhat, void* p, void* v) {
    OK_TRY(launch_copy(C.g, f64, rhat, r, C.st));
    OK_TRY(launch_dot_rr(C.g, f64, rhat, r, C.w.partial, C.st));
    OK_TRY(fin_blas(C, FIN_INIT));
    OK_TRY(launch_zero(C.g, f64, p, C.st));
    OK_TRY(launch_zero(C.g, f64, v, C.st));
    return OK_SUCCESS;
}

int solve_plain(Ctx& C, const double* xi, double* x, ok_solver_stats* S) {
    const ok_solver_params& P = *C.p;
    double* r = C.w.f64[0];
    double* rhat = C.w.f64[1];
    double* p = C.w.f64[2];
    double* v = C.w.f64[3];
    double* s = C.w.f64[4];
    double* t = C.w.f64[5];
    double xn;
    OK_TRY(source_norm(C, xi, &xn));
    if (!std::isfinite(xn)) {
        set_error("source is not finite");
        return S->status = OK_ENONFINITE;
    }
    if (xn == 0.0) {
        OK_TRY(launch_zero(C.g, true, x, C.st));
        S->true_rel_resid = 0.0;
        return S->status = OK_SUCCESS;
    }
    double rr;
    if (P.zero_guess) {
        OK_TRY(launch_zero(C.g, true, x, C.st));
        OK_TRY(launch_copy(C.g, true, r, xi, C.st));
    } else {
        OK_TRY(true_residual(C, xi, x, t, r, nullptr, &rr, S));
    }
    OK_TRY(restart_from(C, true, r, rhat, p, v));
    Scal h;
    while (true) {
        if (S->iterations >= P.max_iter) {
            OK_TRY(true_residual(C, xi, x, t, r, nullptr, &rr, S));
            S->true_rel_resid = std::sqrt(rr) / xn;
            return S->status = (S->true_rel_resid <= P.tol) ? OK_SUCCESS : OK_NOT_CONVERGED;
        }
        OK_TRY(iterate(C, true, C.W64, C.W64_prec, C.tps64, x, r, rhat, p, v, s, t));
        S->matvec_hi += 2;
        S->iterations++;
        OK_TRY(read_scal(C, &h));
        const double rel = std::sqrt(h.rr) / xn;
        if (P.verbose) fprintf(stderr, "okinv bicgstab64 it %d |r|/|xi| %.3e\n", S->iterations, rel);
        if (!std::isfinite(rel)) {
            set_error("residual became non-finite at iteration %d", S->iterations);
            return S->status = OK_ENONFINITE;
        }
        const bool broke = h.flags & 1;
        if (rel <= P.tol || broke) {
            OK_TRY(true_residual(C, xi, x, t, r, nullptr, &rr, S));
            S->true_rel_resid = std::sqrt(rr) / xn;
            if (S->true_rel_resid <= P.tol) return S->status = OK_SUCCESS;
            if (S->restarts >= P.max_restarts) return S->status = broke ? OK_BREAKDOWN : OK_NOT_CONVERGED;
            S->restarts++;
            OK_TRY(restart_from(C, true, r, rhat, p, v));
        }
    }
}

// CG on the normal equations M^dag M x = M^dag xi with M^dag = gamma5 M gamma5 (Eq. conjugate makes M
// gamma5-hermitian), in the residual form that keeps r = xi - M x: with z = M^dag r,
//   alpha = |z|^2 / |M p|^2 ; x += alpha p ; r -= alpha M p ; beta = |z_new|^2 / |z|^2 ; p = z_new + beta p.
// z is formed as gamma5 (M (gamma5 r)); |z| = |M gamma5 r| since gamma5 is unitary.
// FP64 fields r p w g z' t = C.w.f64[0..5].
int cg_start(Ctx& C, double* r, double* p, double* g, double* zp) {
    OK_TRY(launch_cg_gamma5(C.g, g, r, C.w.partial, C.st));
    OK_TRY(fin_blas(C, FIN_CG_RR));
    OK_TRY(launch_apply(C.g, C.W64, C.W64_prec, g, zp, C.c->mhat, C.tps64, EPI_TS, nullptr, C.w.partial, C.st));
    OK_TRY(fin(C, FIN_CG_INIT, apply_blocks(C.g, C.tps64)));
    OK_TRY(launch_zero(C.g, true, p, C.st));
    return launch_cg_p(C.g, p, zp, C.w.sc, C.st);
}

int solve_cgnr(Ctx& C, const double* xi, double* x, ok_solver_stats* S) {
    const ok_solver_params& P = *C.p;
    double* r = C.w.f64[0];
    double* p = C.w.f64[1];
    double* w = C.w.f64[2];
    double* g = C.w.f64[3];
    double* zp = C.w.f64[4];
    double* t = C.w.f64[5];
    double xn;
    OK_TRY(source_norm(C, xi, &xn));
    if (!std::isfinite(xn)) {
        set_error("source is not finite");
        return S->status = OK_ENONFINITE;
    }
    if (xn == 0.0) {
        OK_TRY(launch_zero(C.g, true, x, C.st));
        S->true_rel_resid = 0.0;
        return S->status = OK_SUCCESS;
    }
    double rr;
    if (P.zero_guess) {
        OK_TRY(launch_zero(C.g, true, x, C.st));
        OK_TRY(launch_copy(C.g, true, r, xi, C.st));
    } else {
        OK_TRY(true_residual(C, xi, x, t, r, nullptr, &rr, S));
    }
    OK_TRY(cg_start(C, r, p, g, zp));
    S->matvec_hi++;
    Scal h;
    while (true) {
        if (S->iterations >= P.max_iter) {
            OK_TRY(true_residual(C, xi, x, t, r, nullptr, &rr, S));
            S->true_rel_resid = std::sqrt(rr) / xn;
            return S->status = (S->true_rel_resid <= P.tol) ? OK_SUCCESS : OK_NOT_CONVERGED;
        }
        OK_TRY(launch_apply(C.g, C.W64, C.W64_prec, p, w, C.c->mhat, C.tps64, EPI_TS, nullptr, C.w.partial, C.st));
        OK_TRY(fin(C, FIN_CG_ALPHA, apply_blocks(C.g, C.tps64)));
        OK_TRY(launch_cg_xr(C.g, x, r, p, w, g, C.w.sc, C.w.partial, C.st));
        OK_TRY(fin_blas(C, FIN_CG_RR));
        OK_TRY(launch_apply(C.g, C.W64, C.W64_prec, g, zp, C.c->mhat, C.tps64, EPI_TS, nullptr, C.w.partial, C.st));
        OK_TRY(fin(C, FIN_CG_BETA, apply_blocks(C.g, C.tps64)));
        OK_TRY(launch_cg_p(C.g, p, zp, C.w.sc, C.st));
        S->matvec_hi += 2;
        S->iterations++;
        OK_TRY(read_scal(C, &h));
        const double rel = std::sqrt(h.rr) / xn;
        if (P.verbose) fprintf(stderr, "okinv cgnr it %d |r|/|xi| %.3e\n", S->iterations, rel);
        if (!std::isfinite(rel)) {
            set_error("residual became non-finite at iteration %d", S->iterations);
            return S->status = OK_ENONFINITE;
        }
        const bool broke = h.flags & 1;
        if (rel <= P.tol || broke) {
            OK_TRY(true_residual(C, xi, x, t, r, nullptr, &rr, S));
            S->true_rel_resid = std::sqrt(rr) / xn;
            if (S->true_rel_resid <= P.tol) return S->status = OK_SUCCESS;
            if (S->restarts >= P.max_restarts) return S->status = broke ? OK_BREAKDOWN : OK_NOT_CONVERGED;
            S->restarts++;
            OK_TRY(cg_start(C, r, p, g, zp));
            S->matvec_hi++;
        }
    }
}

int solve_mixed(Ctx& C, const double* xi, double* x64, ok_solver_stats* S) {
    const ok_solver_params& P = *C.p;
    double* r64 = C.w.f64[0];
    double* t64 = C.w.f64[1];
    float* xlo = C.w.f32[0];
    float* r = C.w.f32[1];
    float* rhat = C.w.f32[2];
    float* p = C.w.f32[3];
    float* v = C.w.f32[4];
    float* s = C.w.f32[5];
    float* t = C.w.f32[6];
    double xn;
    OK_TRY(source_norm(C, xi, &xn));
    if (!std::isfinite(xn)) {
        set_error("source is not finite");
        return S->status = OK_ENONFINITE;
    }
    if (xn == 0.0) {
        OK_TRY(launch_zero(C.g, true, x64, C.st));
        S->true_rel_resid = 0.0;
        return S->status = OK_SUCCESS;
    }
    double rr;
    if (P.zero_guess) {
        OK_TRY(launch_zero(C.g, true, x64, C.st));
        OK_TRY(launch_zero(C.g, true, t64, C.st));
        OK_TRY(launch_residual(C.g, xi, t64, r64, r, C.w.partial, C.st));
        OK_TRY(fin_blas(C, FIN_TRUE));
        Scal h0;
        OK_TRY(read_scal(C, &h0));
        rr = h0.rr_true;
    } else {
        OK_TRY(true_residual(C, xi, x64, t64, r64, r, &rr, S));
    }
    S->true_rel_resid = std::sqrt(rr) / xn;
    if (S->true_rel_resid <= P.tol) return S->status = OK_SUCCESS;
    OK_TRY(launch_zero(C.g, false, xlo, C.st));
    OK_TRY(restart_from(C, false, r, rhat, p, v));
    double maxr = std::sqrt(rr);
    double best = maxr;
    int best_it = S->iterations;
    Scal h;
    while (true) {
        if (S->iterations >= P.max_iter) {
            OK_TRY(launch_accum_x(C.g, x64, xlo, C.st));
            OK_TRY(true_residual(C, xi, x64, t64, r64, r, &rr, S));
            S->true_rel_resid = std::sqrt(rr) / xn;
            return S->status = (S->true_rel_resid <= P.tol) ? OK_SUCCESS : OK_NOT_CONVERGED;
        }
        OK_TRY(iterate(C, false, C.Wlo, C.Wlo_prec, C.tpslo, xlo, r, rhat, p, v, s, t));
        S->matvec_lo += 2;
        if (C.net) S->net_applies += 2;
        S->iterations++;
        OK_TRY(read_scal(C, &h));
        const double rn = std::sqrt(h.rr);
        if (P.verbose) fprintf(stderr, "okinv bicgstab32 it %d |r|/|xi| %.3e\n", S->iterations, rn / xn);
        const bool broke = h.flags & 1;
        if (C.net) {
            // the network's recurrence failed: x64 holds the last reliable iterate
            if (rn < best) {
                best = rn;
                best_it = S->iterations;
            }
            const bool stalled = P.stall_window > 0 && S->iterations - best_it >= P.stall_window;
            if (!std::isfinite(rn) || broke || stalled) {
                if (P.verbose) fprintf(stderr, "okinv preconditioned solve %s at iteration %d: fallback\n",
                                       !std::isfinite(rn) ? "non-finite" : broke ? "broke down" : "stalled",
                                       S->iterations);
                if (std::isfinite(rn)) OK_TRY(launch_accum_x(C.g, x64, xlo, C.st));
                return kFallback;
            }
        }
        if (!std::isfinite(rn)) {
            set_error("low-precision residual became non-finite at iteration %d", S->iterations);
            return S->status = OK_ENONFINITE;
        }
        maxr = std::max(maxr, rn);
        if (rn < P.delta * maxr || rn / xn <= P.tol || broke) {
            // reliable update: fold x32 into x64 and recompute the residual in FP64
            OK_TRY(launch_accum_x(C.g, x64, xlo, C.st));
            OK_TRY(true_residual(C, xi, x64, t64, r64, r, &rr, S));
            S->reliable_updates++;
            const double rt = std::sqrt(rr);
            S->true_rel_resid = rt / xn;
            if (P.verbose) fprintf(stderr, "okinv reliable update %d true |r|/|xi| %.3e\n", S->reliable_updates, rt / xn);
            if (S->true_rel_resid <= P.tol) return S->status = OK_SUCCESS;
            maxr = rt;
            if (broke) {
                if (S->restarts >= P.max_restarts) return S->status = OK_BREAKDOWN;
                S->restarts++;
                OK_TRY(restart_from(C, false, r, rhat, p, v));
            } else {
                OK_TRY(launch_dot_rr(C.g, false, rhat, r, C.w.partial, C.st));
                OK_TRY(fin_blas(C, FIN_RHO_REPLACE));
            }
        }
    }
}

// ------------------------------------------------------------------ batched
// All right-hand sides (up to 16) iterate together: one MFMA application of the
// low-precision site-major W per BiCGStab step for the whole batch, FP32 fields
// with the right-hand side index fastest, per-right-hand-side scalars, and FP64
// reliable updates per right-hand side (column) when its residual has dropped
// by delta.  Converged right-hand sides stop updating; the operator still runs
// over every column.
struct WorkB {
    ScalB* sc;
    double2* partial;
    double* t64;
    float* f[9];   // x32 r rhat p v s t ; with a network also p^ s^
    void* netw;
};

size_t layout_batched(const Geo& g, int nrhs, int net_layers, char* base, WorkB* w) {
    size_t off = 0;
    auto take = [&](size_t n) {
        char* p = base ? base + off : nullptr;
        off += align256(n);
        return p;
    };
    WorkB tmp;
    WorkB& W = w ? *w : tmp;
    W.sc = reinterpret_cast<ScalB*>(take(sizeof(ScalB)));
    int nb = std::max(kGridB, col_blocks(g));
    for (int n = 1; n <= kMaxRhsB; ++n) nb = std::max(nb, sigma_mr_blocks(g, n));
    W.partial = reinterpret_cast<double2*>(take((size_t)nb * kMaxRhsB * 2 * sizeof(double2)));
    W.t64 = reinterpret_cast<double*>(take((size_t)4 * g.V * 12 * 16));   // four FP64 fields
    for (int i = 0; i < (net_layers ? 9 : 7); ++i) W.f[i] = reinterpret_cast<float*>(take((size_t)g.V * 12 * nrhs * 8));
    W.netw = net_layers ? take(net_apply_work_bytes(g, net_layers, nrhs)) : nullptr;
    return off;
}

int bfin(Ctx& C, WorkB& B, int kind, int nb, int j0, int nj) {
    return launch_bfinish(kind, nb, j0, nj, B.partial, B.sc, C.st);
}

int read_scalb(Ctx& C, WorkB& B, ScalB* h) {
    OK_HIP(hipMemcpyAsync(h, B.sc, sizeof(ScalB), hipMemcpyDeviceToHost, C.st));
    OK_HIP(hipStreamSynchronize(C.st));
    return OK_SUCCESS;
}

int write_active(Ctx& C, WorkB& B, const ScalB* h) {
    OK_HIP(hipMemcpyAsync(B.sc->active, h->active, sizeof(h->active), hipMemcpyHostToDevice, C.st));
    OK_HIP(hipStreamSynchronize(C.st));
    return OK_SUCCESS;
}

// The low-precision operator on nrhs right-hand-side-inner FP32 fields of the batched solve.
int apply_lo_batched(Ctx& C, const float* in, float* out, int nrhs) {
    if (C.Wlo_prec & OK_LAYOUT_SIGMA) return launch_apply_sigma_mr(C.g, C.Wlo, in, out, C.c->mhat, nrhs, C.st);
    return launch_apply_site(C.g, C.Wlo, C.Wlo_prec & ~OK_LAYOUT_SITE, in, out, C.c->mhat, nrhs, 1, C.st);
}

// For every column j in cols[0..n): x64_j += x32[:, j]; r[:, j] = xi_j - M64 x64_j;
// rr[j] = ||r_j||^2 in FP64.  xi and x are the bases of the [nrhs][V][12] FP64 fields.
// The FP64 operator runs on up to four columns per pass, reading W once per pass.
int batched_true_residuals(Ctx& C, WorkB& B, int nrhs, const int* cols, int n, const double* xi, double* x,
                           double* rr, ok_solver_stats* S) {
    const Geo& g = C.g;
    const size_t col = (size_t)g.V * 24;
    unsigned mask = 0;
    for (int i = 0; i < n; ++i) mask |= 1u << cols[i];
    OK_TRY(launch_cols_accum(g, nrhs, mask, x, B.f[0], C.st));
    for (int i0 = 0; i0 < n; i0 += 4) {
        const int m = std::min(4, n - i0);
        const double* in[4];
        double* out[4];
        for (int r = 0; r < m; ++r) {
            in[r] = x + cols[i0 + r] * col;
            out[r] = B.t64 + (size_t)r * col;
        }
        if (C.W64_prec == OK_F64) {
            OK_TRY(launch_apply_m64(g, C.W64, in, out, m, C.c->mhat, C.st));
        } else if (C.W64_prec & OK_LAYOUT_SIGMA) {
            OK_TRY(launch_apply_sigma_cols(g, C.W64, in, out, m, C.c->mhat, C.st));
        } else {   // saved layout: one single-right-hand-side application per column
            for (int r = 0; r < m; ++r)
                OK_TRY(launch_apply(g, C.W64, C.W64_prec, in[r], out[r], C.c->mhat, 1, EPI_NONE, nullptr, nullptr,
                                    C.st));
        }
        ColSlots sl;
        for (int j = 0; j < kMaxRhsB; ++j) sl.slot[j] = -1;
        for (int r = 0; r < m; ++r) sl.slot[cols[i0 + r]] = r;
        OK_TRY(launch_cols_residual(g, nrhs, sl, xi, B.t64, B.f[1], B.partial, C.st));
        for (int r = 0; r < m; ++r) {
            const int j = cols[i0 + r];
            S[j].matvec_hi++;
            OK_TRY(bfin(C, B, FIN_TRUE, kGridB, j, 1));
        }
    }
    ScalB h;
    OK_TRY(read_scalb(C, B, &h));
    for (int i = 0; i < n; ++i) rr[cols[i]] = h.rr_true[cols[i]];
    return OK_SUCCESS;
}

int batched_restart(Ctx& C, WorkB& B, int nrhs, int j) {
    const Geo& g = C.g;
    OK_TRY(launch_col_restart(g, nrhs, j, B.f[1], B.f[2], B.f[3], B.f[4], C.st));
    OK_TRY(launch_col_dot(g, nrhs, j, B.f[2], B.f[1], B.partial, C.st));
    return bfin(C, B, FIN_INIT, col_blocks(g), j, 1);
}

// xi, x: FP64 [nrhs][V][12]; S: nrhs stats.  Returns the first failing status.  With
// C.net, right-hand sides whose preconditioned recurrence fails get fallback[j] = 1
// (x64 holds their last reliable iterate) and take no part in the returned status.
int solve_batched(Ctx& C, WorkB& B, int nrhs, const double* xi, double* x, ok_solver_stats* S, int* fallback) {
    const ok_solver_params& P = *C.p;
    const Geo& g = C.g;
    const size_t fb = (size_t)g.V * 12 * nrhs * 8;
    const size_t col = (size_t)g.V * 24;   // doubles per right-hand side in the ABI layout
    float *x32 = B.f[0], *r = B.f[1], *rhat = B.f[2], *p = B.f[3], *v = B.f[4], *s = B.f[5], *t = B.f[6];
    OK_HIP(hipMemsetAsync(B.sc, 0, sizeof(ScalB), C.st));
    OK_HIP(hipMemsetAsync(x32, 0, fb, C.st));
    OK_HIP(hipMemsetAsync(p, 0, fb, C.st));
    OK_HIP(hipMemsetAsync(v, 0, fb, C.st));
    OK_HIP(hipMemsetAsync(r, 0, fb, C.st));
    OK_HIP(hipMemsetAsync(rhat, 0, fb, C.st));
    ScalB h;
    memset(&h, 0, sizeof(h));
    double xn[kMaxRhsB], maxr[kMaxRhsB], best[kMaxRhsB];
    int best_it[kMaxRhsB];
    int rc_all = OK_SUCCESS;
    for (int j = 0; j < nrhs; ++j) {
        OK_TRY(launch_col_norm64(g, j, xi + j * col, B.partial, C.st));
        OK_TRY(bfin(C, B, FIN_TRUE, col_blocks(g), j, 1));
        ScalB h0;
        OK_TRY(read_scalb(C, B, &h0));
        xn[j] = std::sqrt(h0.rr_true[j]);
        if (!std::isfinite(xn[j])) {
            set_error("source %d is not finite", j);
            S[j].status = OK_ENONFINITE;
            return OK_ENONFINITE;
        }
        if (xn[j] == 0.0) {
            OK_HIP(hipMemsetAsync(x + j * col, 0, col * 8, C.st));
            S[j].true_rel_resid = 0.0;
            S[j].status = OK_SUCCESS;
            continue;
        }
        double rr;
        if (P.zero_guess) {
            OK_HIP(hipMemsetAsync(x + j * col, 0, col * 8, C.st));
            OK_TRY(launch_col_load(g, nrhs, j, xi + j * col, r, C.st));
            rr = xn[j] * xn[j];
        } else {
            double rrv[kMaxRhsB];
            OK_TRY(batched_true_residuals(C, B, nrhs, &j, 1, xi, x, rrv, S));
            rr = rrv[j];
        }
        S[j].true_rel_resid = std::sqrt(rr) / xn[j];
        if (S[j].true_rel_resid <= P.tol) {
            S[j].status = OK_SUCCESS;
            continue;
        }
        h.active[j] = 1;
        OK_HIP(hipMemcpyAsync(&B.sc->active[j], &h.active[j], sizeof(int), hipMemcpyHostToDevice, C.st));
        OK_TRY(batched_restart(C, B, nrhs, j));
        maxr[j] = best[j] = std::sqrt(rr);
        best_it[j] = 0;
    }
    OK_TRY(write_active(C, B, &h));
    auto any_active = [&]() {
        for (int j = 0; j < nrhs; ++j)
            if (h.active[j]) return true;
        return false;
    };
    int it = 0;
    while (any_active()) {
        if (it >= P.max_iter) {
            int cols[kMaxRhsB], n = 0;
            double rrv[kMaxRhsB];
            for (int j = 0; j < nrhs; ++j)
                if (h.active[j]) cols[n++] = j;
            OK_TRY(batched_true_residuals(C, B, nrhs, cols, n, xi, x, rrv, S));
            for (int j = 0; j < nrhs; ++j) {
                if (!h.active[j]) continue;
                const double rr = rrv[j];
                S[j].true_rel_resid = std::sqrt(rr) / xn[j];
                S[j].status = S[j].true_rel_resid <= P.tol ? OK_SUCCESS : OK_NOT_CONVERGED;
                if (S[j].status != OK_SUCCESS && rc_all == OK_SUCCESS) rc_all = S[j].status;
                h.active[j] = 0;
            }
            break;
        }
        float* ph = C.net ? B.f[7] : p;
        float* sh = C.net ? B.f[8] : s;
        OK_TRY(launch_bp_update(g, nrhs, p, r, v, B.sc, C.st));
        if (C.net) OK_TRY(apply_net(C, p, ph, nrhs, true, B.netw));
        const bool sig = (C.Wlo_prec & OK_LAYOUT_SIGMA) != 0;   // its epilogue forms the dots
        if (sig) {
            OK_TRY(launch_apply_sigma_mr(g, C.Wlo, ph, v, C.c->mhat, nrhs, C.st, EPI_RV, rhat, B.partial));
            OK_TRY(bfin(C, B, FIN_ALPHA, sigma_mr_blocks(g, nrhs), 0, nrhs));
        } else {
            OK_TRY(apply_lo_batched(C, ph, v, nrhs));
            OK_TRY(launch_bdot(g, nrhs, rhat, v, B.sc, B.partial, C.st));
            OK_TRY(bfin(C, B, FIN_ALPHA, kGridB, 0, nrhs));
        }
        OK_TRY(launch_bs_update(g, nrhs, s, r, v, B.sc, C.st));
        if (C.net) OK_TRY(apply_net(C, s, sh, nrhs, true, B.netw));
        if (sig) {
            OK_TRY(launch_apply_sigma_mr(g, C.Wlo, sh, t, C.c->mhat, nrhs, C.st, EPI_TS, s, B.partial));
            OK_TRY(bfin(C, B, FIN_OMEGA, sigma_mr_blocks(g, nrhs), 0, nrhs));
        } else {
            OK_TRY(apply_lo_batched(C, sh, t, nrhs));
            OK_TRY(launch_bdot(g, nrhs, t, s, B.sc, B.partial, C.st));
            OK_TRY(bfin(C, B, FIN_OMEGA, kGridB, 0, nrhs));
        }
        OK_TRY(launch_bxr_update(g, nrhs, x32, r, ph, sh, s, t, rhat, B.sc, B.partial, C.st));
        OK_TRY(bfin(C, B, FIN_RHO, kGridB, 0, nrhs));
        ScalB hd;
        OK_TRY(read_scalb(C, B, &hd));
        ++it;
        bool changed = false;
        // pass 1: bookkeeping, failures, and which right-hand sides are due for a reliable update
        bool due[kMaxRhsB] = {false};
        double rnv[kMaxRhsB];
        bool any_due = false;
        for (int j = 0; j < nrhs; ++j) {
            if (!h.active[j]) continue;
            S[j].iterations++;
            S[j].matvec_lo += 2;
            if (C.net) S[j].net_applies += 2;
            const double rn = std::sqrt(hd.rr[j]);
            rnv[j] = rn;
            if (P.verbose) fprintf(stderr, "okinv batched it %d rhs %d |r|/|xi| %.3e\n", it, j, rn / xn[j]);
            if (C.net) {
                if (rn < best[j]) {
                    best[j] = rn;
                    best_it[j] = it;
                }
                const bool stalled = P.stall_window > 0 && it - best_it[j] >= P.stall_window;
                if (!std::isfinite(rn) || (hd.flags[j] & 1) || stalled) {
                    if (P.verbose) fprintf(stderr, "okinv batched rhs %d: preconditioned solve failed at %d\n", j, it);
                    if (std::isfinite(rn)) OK_TRY(launch_col_accum(g, nrhs, j, x + j * col, x32, C.st));
                    fallback[j] = 1;
                    h.active[j] = 0;
                    changed = true;
                    continue;
                }
            }
            if (!std::isfinite(rn)) {
                set_error("residual of right-hand side %d became non-finite at iteration %d", j, it);
                S[j].status = OK_ENONFINITE;
                return OK_ENONFINITE;
            }
            maxr[j] = std::max(maxr[j], rn);
            due[j] = rn < P.delta * maxr[j] || rn / xn[j] <= P.tol || (hd.flags[j] & 1);
            any_due |= due[j];
        }
        // pass 2: when any right-hand side is due, every one within sqrt(delta) of its maximum joins
        // the same FP64 pass (one W read per four of them)
        if (any_due) {
            int cols[kMaxRhsB], n = 0;
            const double dg = std::sqrt(P.delta);
            for (int j = 0; j < nrhs; ++j)
                if (h.active[j] && (due[j] || rnv[j] < dg * maxr[j])) cols[n++] = j;
            double rrv[kMaxRhsB];
            OK_TRY(batched_true_residuals(C, B, nrhs, cols, n, xi, x, rrv, S));
            unsigned replace = 0;   // columns that continue from the new residual: rho = <r^, r>
            for (int i = 0; i < n; ++i) {
                const int j = cols[i];
                const bool broke = hd.flags[j] & 1;
                S[j].reliable_updates++;
                const double rt = std::sqrt(rrv[j]);
                S[j].true_rel_resid = rt / xn[j];
                if (S[j].true_rel_resid <= P.tol) {
                    S[j].status = OK_SUCCESS;
                    h.active[j] = 0;
                    changed = true;
                    continue;
                }
                maxr[j] = rt;
                if (broke) {
                    if (S[j].restarts >= P.max_restarts) {
                        S[j].status = OK_BREAKDOWN;
                        if (rc_all == OK_SUCCESS) rc_all = OK_BREAKDOWN;
                        h.active[j] = 0;
                        changed = true;
                        continue;
                    }
                    S[j].restarts++;
                    OK_TRY(batched_restart(C, B, nrhs, j));
                } else {
                    replace |= 1u << j;
                }
            }
            if (replace) {   // a restart touches only its own column, so these dots can come after
                OK_TRY(launch_cols_dot(g, nrhs, replace, rhat, r, B.partial, C.st));
                for (int j = 0; j < nrhs; ++j)
                    if ((replace >> j) & 1u) OK_TRY(bfin(C, B, FIN_RHO_REPLACE, kGridB, j, 1));
            }
        }
        if (changed) OK_TRY(write_active(C, B, &h));
    }
    return rc_all;
}

}  // namespace
}  // namespace okinv

using namespace okinv;

extern "C" {

namespace {

// the right-hand sides iterate together: site-major W on the matrix cores, or FP32 sigma-layout W
// with right-hand-side-inner fields
bool is_batched(int wlo) {
    return wlo >= 0 && ((wlo & OK_LAYOUT_SITE) || ((wlo & OK_LAYOUT_SIGMA) && (wlo & OK_SPINOR_RHS_INNER)));
}

// low-precision operator of a mixed solve: F32 / BF16, at most one layout flag, sigma only in F32;
// F32 | OK_LAYOUT_SIGMA | OK_SPINOR_RHS_INNER selects the batched solve with the sigma layout
bool valid_wlo(int p) {
    if (p & OK_SPINOR_RHS_INNER) return (p & ~OK_SPINOR_RHS_INNER) == (OK_F32 | OK_LAYOUT_SIGMA);
    const int lay = p & (OK_LAYOUT_SITE | OK_LAYOUT_SAVED | OK_LAYOUT_SIGMA), b = p & ~lay;
    if (lay & (lay - 1)) return false;
    if (lay == OK_LAYOUT_SIGMA) return b == OK_F32;
    return b == OK_F32 || b == OK_BF16;
}

int check_solver_net(const ok_net* net, bool mixed) {
    if (!net) return OK_SUCCESS;
    if (!mixed) {
        set_error("the preconditioner network needs the low-precision solve (d_Wlo)");
        return OK_EINVAL;
    }
    if (net->n_layers < 1 || net->n_layers > OK_NET_MAX_LAYERS) {
        set_error("net->n_layers = %d outside [1, %d]", net->n_layers, OK_NET_MAX_LAYERS);
        return OK_EINVAL;
    }
    int rc = check_ptr(net->d_params, "net->d_params");
    return rc ? rc : check_ptr(net->d_T, "net->d_T");
}

size_t workspace(const Geo& G, int nrhs, int Wlo_prec, const ok_net* net) {
    const int nl = net ? net->n_layers : 0;
    if (is_batched(Wlo_prec)) return layout_batched(G, std::min(nrhs, kMaxRhsB), nl, nullptr, nullptr);
    return layout(G, Wlo_prec >= 0, nl, nullptr, nullptr);
}

}  // namespace

int ok_bicgstab_workspace_bytes(const ok_geom* g, int nrhs, int Wlo_prec, const ok_net* net, size_t* bytes) {
    Geo G;
    int rc = make_geo(g, &G);
    if (rc) return rc;
    if (nrhs < 1 || !bytes) {
        set_error("nrhs must be >= 1 and bytes non-NULL");
        return OK_EINVAL;
    }
    if (Wlo_prec >= 0 && !valid_wlo(Wlo_prec)) {
        set_error("Wlo_prec must be OK_F32 or OK_BF16 (optionally | OK_LAYOUT_SITE or OK_LAYOUT_SAVED), "
                  "OK_F32 | OK_LAYOUT_SIGMA (optionally | OK_SPINOR_RHS_INNER), or negative (plain FP64)");
        return OK_EINVAL;
    }
    if ((rc = check_solver_net(net, Wlo_prec >= 0))) return rc;
    *bytes = workspace(G, nrhs, Wlo_prec, net);
    return OK_SUCCESS;
}

namespace {

// Fixed workspace of ok_bicgstab_static: one copy per GPU, held until the process ends.  Host code
// never passes this array's name to a kernel or a copy: it takes the device address that
// hipGetSymbolAddress returns on each device (static_scratch below).
constexpr size_t kStaticWorkBytes = (size_t)64 << 20;
__device__ __align__(256) char scratch[kStaticWorkBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices];

// the current device's address of `scratch`, looked up on the first call on that device
int static_scratch(void** ptr) {
    int dev = -1;
    OK_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device %d outside the %d the static workspace table holds", dev, kMaxDevices);
        return OK_EDEVICE;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        OK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) {
            set_error("hipGetSymbolAddress returned no address for the static workspace");
            return OK_EDEVICE;
        }
        g_scratch[dev] = p;
    }
    *ptr = g_scratch[dev];
    return OK_SUCCESS;
}

// ok_bicgstab with the caller's workspace (use_static false) or with `scratch` (true)
int bicgstab_run(const ok_geom* g, const ok_coeffs* c, const ok_solver_params* p, const void* d_W64,
                 const void* d_Wlo, int Wlo_prec, const ok_net* net, const double* d_xi, double* d_psi, int nrhs,
                 void* d_work, size_t work_bytes, ok_solver_stats* stats, void* stream, bool use_static) {
    Ctx C;
    int rc = make_geo(g, &C.g);
    if (rc) return rc;
    if (!c || !p || !stats) {
        set_error("coefficients, params and stats must be non-NULL");
        return OK_EINVAL;
    }
    if (!std::isfinite(c->mhat) || !(c->u0 > 0)) {
        set_error("invalid coefficients");
        return OK_EINVAL;
    }
    if (!(p->tol > 0) || p->max_iter < 0 || p->max_restarts < 0 || !(p->delta > 0 && p->delta < 1) ||
        p->stall_window < 0) {
        set_error("invalid solver parameters (tol > 0, max_iter >= 0, 0 < delta < 1, stall_window >= 0)");
        return OK_EINVAL;
    }
    if (nrhs < 1 || nrhs > 4096) {
        set_error("nrhs = %d outside [1, 4096]", nrhs);
        return OK_EINVAL;
    }
    const bool mixed = d_Wlo != nullptr;
    const int wlb = Wlo_prec & 3;
    if (mixed && !valid_wlo(Wlo_prec)) {
        set_error("Wlo_prec must be OK_F32 or OK_BF16 (optionally | OK_LAYOUT_SITE or OK_LAYOUT_SAVED), or "
                  "OK_F32 | OK_LAYOUT_SIGMA (optionally | OK_SPINOR_RHS_INNER), when d_Wlo is given");
        return OK_EINVAL;
    }
    if (p->W64_layout != 0 && p->W64_layout != OK_LAYOUT_SAVED && p->W64_layout != OK_LAYOUT_SIGMA) {
        set_error("params->W64_layout must be 0, OK_LAYOUT_SAVED or OK_LAYOUT_SIGMA");
        return OK_EINVAL;
    }
    if ((rc = check_solver_net(net, mixed))) return rc;
    const bool batched = mixed && is_batched(Wlo_prec);
    if ((rc = check_ptr(d_W64, "d_W64")) || (mixed && (rc = check_ptr(d_Wlo, "d_Wlo"))) ||
        (rc = check_ptr(d_xi, "d_xi")) || (rc = check_ptr(d_psi, "d_psi")) ||
        (!use_static && (rc = check_ptr(d_work, "d_work"))))
        return rc;
    const size_t need = workspace(C.g, nrhs, mixed ? Wlo_prec : -1, net);
    if (use_static && need > kStaticWorkBytes) {
        set_error("this solve needs %zu bytes of workspace, more than the %zu of the static workspace of "
                  "ok_bicgstab_static (use ok_bicgstab with a workspace of that size)", need, kStaticWorkBytes);
        return OK_ESIZE;
    }
    if (!use_static && work_bytes < need) {
        set_error("workspace has %zu bytes, needs %zu", work_bytes, need);
        return OK_ESIZE;
    }
    const size_t sb = (size_t)C.g.V * 12 * 16 * nrhs;
    {
        auto a = reinterpret_cast<uintptr_t>(d_xi), b = reinterpret_cast<uintptr_t>(d_psi);
        if (a < b + sb && b < a + sb) {
            set_error("d_psi must not overlap d_xi");
            return OK_EINVAL;
        }
    }
    if (use_static) {
        if ((rc = static_scratch(&d_work))) return rc;
        work_bytes = kStaticWorkBytes;
    }
    const int nl = net ? net->n_layers : 0;
    WorkB B;
    if (batched)
        layout_batched(C.g, std::min(nrhs, kMaxRhsB), nl, reinterpret_cast<char*>(d_work), &B);
    else
        layout(C.g, mixed, nl, reinterpret_cast<char*>(d_work), &C.w);
    C.c = c;
    C.p = p;
    C.W64 = d_W64;
    C.Wlo = d_Wlo;
    C.Wlo_prec = Wlo_prec;
    C.net = net;
    C.st = reinterpret_cast<hipStream_t>(stream);
    C.W64_prec = OK_F64 | p->W64_layout;
    C.tps64 = p->W64_layout ? 1 : stencil_tps(OK_F64);
    C.tpslo = !mixed || (Wlo_prec & (OK_LAYOUT_SAVED | OK_LAYOUT_SIGMA)) ? 1 : stencil_tps(wlb);
    // the fallback continues from the iterate in d_psi
    ok_solver_params pf = *p;
    pf.zero_guess = 0;
    int first_bad = OK_SUCCESS;
    if (batched) {
        for (int k0 = 0; k0 < nrhs; k0 += kMaxRhsB) {
            const int nk = std::min(kMaxRhsB, nrhs - k0);
            const auto tk = std::chrono::steady_clock::now();
            for (int k = 0; k < nk; ++k) stats[k0 + k] = ok_solver_stats{};
            const size_t off = (size_t)k0 * C.g.V * 24;
            int fb[kMaxRhsB] = {0};
            C.net = net;
            C.p = p;
            rc = solve_batched(C, B, nk, d_xi + off, d_psi + off, stats + k0, fb);
            if (rc < 0) return rc;
            if (rc != OK_SUCCESS && first_bad == OK_SUCCESS) first_bad = rc;
            C.net = nullptr;
            C.p = &pf;
            for (int k = 0; k < nk; ++k) {
                if (!fb[k]) continue;
                const size_t o1 = (size_t)(k0 + k) * C.g.V * 24;
                stats[k0 + k].fallbacks = 1;
                int dummy = 0;
                rc = solve_batched(C, B, 1, d_xi + o1, d_psi + o1, stats + k0 + k, &dummy);
                if (rc < 0) return rc;
                if (rc != OK_SUCCESS && first_bad == OK_SUCCESS) first_bad = rc;
            }
            const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - tk).count();
            for (int k = 0; k < nk; ++k) stats[k0 + k].seconds = sec;
        }
        return first_bad;
    }
    for (int k = 0; k < nrhs; ++k) {
        const auto tk = std::chrono::steady_clock::now();
        ok_solver_stats& S = stats[k];
        S = ok_solver_stats{};
        const size_t off = (size_t)k * C.g.V * 24;
        C.net = net;
        C.p = p;
        rc = mixed ? solve_mixed(C, d_xi + off, d_psi + off, &S) : solve_plain(C, d_xi + off, d_psi + off, &S);
        if (rc == kFallback) {
            S.fallbacks = 1;
            C.net = nullptr;
            C.p = &pf;
            rc = solve_mixed(C, d_xi + off, d_psi + off, &S);
        }
        S.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - tk).count();
        if (rc < 0) {
            S.status = rc;
            return rc;
        }
        if (rc != OK_SUCCESS && first_bad == OK_SUCCESS) first_bad = rc;
    }
    return first_bad;
}

}  // namespace

int ok_bicgstab(const ok_geom* g, const ok_coeffs* c, const ok_solver_params* p, const void* d_W64,
                const void* d_Wlo, int Wlo_prec, const ok_net* net, const double* d_xi, double* d_psi, int nrhs,
                void* d_work, size_t work_bytes, ok_solver_stats* stats, void* stream) {
    return bicgstab_run(g, c, p, d_W64, d_Wlo, Wlo_prec, net, d_xi, d_psi, nrhs, d_work, work_bytes, stats, stream,
                        false);
}

int ok_bicgstab_static(const ok_geom* g, const ok_coeffs* c, const ok_solver_params* p, const void* d_W64,
                       const void* d_Wlo, int Wlo_prec, const ok_net* net, const double* d_xi, double* d_psi,
                       int nrhs, ok_solver_stats* stats, void* stream) {
    return bicgstab_run(g, c, p, d_W64, d_Wlo, Wlo_prec, net, d_xi, d_psi, nrhs, nullptr, 0, stats, stream, true);
}

size_t ok_bicgstab_static_max_bytes(void) { return kStaticWorkBytes; }

int ok_cgnr_workspace_bytes(const ok_geom* g, int nrhs, size_t* bytes) {
    Geo G;
    int rc = make_geo(g, &G);
    if (rc) return rc;
    if (nrhs < 1 || !bytes) {
        set_error("nrhs must be >= 1 and bytes non-NULL");
        return OK_EINVAL;
    }
    *bytes = layout(G, false, 0, nullptr, nullptr);
    return OK_SUCCESS;
}

int ok_cgnr(const ok_geom* g, const ok_coeffs* c, const ok_solver_params* p, const void* d_W64, const double* d_xi,
            double* d_psi, int nrhs, void* d_work, size_t work_bytes, ok_solver_stats* stats, void* stream) {
    Ctx C;
    int rc = make_geo(g, &C.g);
    if (rc) return rc;
    if (!c || !p || !stats) {
        set_error("coefficients, params and stats must be non-NULL");
        return OK_EINVAL;
    }
    if (!std::isfinite(c->mhat) || !(c->u0 > 0)) {
        set_error("invalid coefficients");
        return OK_EINVAL;
    }
    if (!(p->tol > 0) || p->max_iter < 0 || p->max_restarts < 0) {
        set_error("invalid solver parameters (tol > 0, max_iter >= 0, max_restarts >= 0)");
        return OK_EINVAL;
    }
    if (p->W64_layout != 0 && p->W64_layout != OK_LAYOUT_SAVED && p->W64_layout != OK_LAYOUT_SIGMA) {
        set_error("params->W64_layout must be 0, OK_LAYOUT_SAVED or OK_LAYOUT_SIGMA");
        return OK_EINVAL;
    }
    if (nrhs < 1 || nrhs > 4096) {
        set_error("nrhs = %d outside [1, 4096]", nrhs);
        return OK_EINVAL;
    }
    if ((rc = check_ptr(d_W64, "d_W64")) || (rc = check_ptr(d_xi, "d_xi")) || (rc = check_ptr(d_psi, "d_psi")) ||
        (rc = check_ptr(d_work, "d_work")))
        return rc;
    const size_t need = layout(C.g, false, 0, nullptr, nullptr);
    if (work_bytes < need) {
        set_error("workspace has %zu bytes, needs %zu", work_bytes, need);
        return OK_ESIZE;
    }
    const size_t sb = (size_t)C.g.V * 12 * 16 * nrhs;
    {
        auto a = reinterpret_cast<uintptr_t>(d_xi), b = reinterpret_cast<uintptr_t>(d_psi);
        if (a < b + sb && b < a + sb) {
            set_error("d_psi must not overlap d_xi");
            return OK_EINVAL;
        }
    }
    layout(C.g, false, 0, reinterpret_cast<char*>(d_work), &C.w);
    C.c = c;
    C.p = p;
    C.W64 = d_W64;
    C.Wlo = nullptr;
    C.Wlo_prec = -1;
    C.net = nullptr;
    C.st = reinterpret_cast<hipStream_t>(stream);
    C.W64_prec = OK_F64 | p->W64_layout;
    C.tps64 = p->W64_layout ? 1 : stencil_tps(OK_F64);
    C.tpslo = 1;
    int first_bad = OK_SUCCESS;
    for (int k = 0; k < nrhs; ++k) {
        const auto tk = std::chrono::steady_clock::now();
        ok_solver_stats& S = stats[k];
        S = ok_solver_stats{};
        const size_t off = (size_t)k * C.g.V * 24;
        rc = solve_cgnr(C, d_xi + off, d_psi + off, &S);
        S.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - tk).count();
        if (rc < 0) {
            S.status = rc;
            return rc;
        }
        if (rc != OK_SUCCESS && first_bad == OK_SUCCESS) first_bad = rc;
    }
    return first_bad;
}

}  // extern "C"
