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
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>

#include "common.h"
#include "kernels.h"
#include "wlayout.h"

namespace okinv {
namespace {

struct Work {
    Scal* sc;
    double2* partial;
    int npart;
    // FP64 fields (plain: r rhat p v s t ; mixed: r64 t64)
    double* f64[6];
    // FP32 fields (mixed: xlo r rhat p v s t)
    float* f32[7];
};

size_t align256(size_t n) { return (n + 255) / 256 * 256; }

size_t layout(const Geo& g, bool mixed, char* base, Work* w) {
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
        for (int i = 0; i < 7; ++i) W.f32[i] = reinterpret_cast<float*>(take(s32));
    }
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
    hipStream_t st;
    Work w;
    int tps64, tpslo;
};

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
    OK_TRY(launch_apply(C.g, C.W64, OK_F64, x, t, C.c->mhat, C.tps64, EPI_NONE, nullptr, nullptr, C.st));
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
int iterate(Ctx& C, bool f64, const void* W, int prec, int tps, void* x, void* r, void* rhat, void* p, void* v,
            void* s, void* t) {
    const Geo& g = C.g;
    OK_TRY(launch_p_update(g, f64, p, r, v, C.w.sc, C.st));
    OK_TRY(launch_apply(g, W, prec, p, v, C.c->mhat, tps, EPI_RV, rhat, C.w.partial, C.st));
    OK_TRY(fin(C, FIN_ALPHA, apply_blocks(g, tps)));
    OK_TRY(launch_s_update(g, f64, s, r, v, C.w.sc, C.st));
    OK_TRY(launch_apply(g, W, prec, s, t, C.c->mhat, tps, EPI_TS, nullptr, C.w.partial, C.st));
    OK_TRY(fin(C, FIN_OMEGA, apply_blocks(g, tps)));
    OK_TRY(launch_xr_update(g, f64, x, r, p, s, t, rhat, C.w.sc, C.w.partial, C.st));
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
        OK_TRY(iterate(C, true, C.W64, OK_F64, C.tps64, x, r, rhat, p, v, s, t));
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
        S->iterations++;
        OK_TRY(read_scal(C, &h));
        const double rn = std::sqrt(h.rr);
        if (P.verbose) fprintf(stderr, "okinv bicgstab32 it %d |r|/|xi| %.3e\n", S->iterations, rn / xn);
        if (!std::isfinite(rn)) {
            set_error("low-precision residual became non-finite at iteration %d", S->iterations);
            return S->status = OK_ENONFINITE;
        }
        const bool broke = h.flags & 1;
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

}  // namespace
}  // namespace okinv

using namespace okinv;

extern "C" {

int ok_bicgstab_workspace_bytes(const ok_geom* g, int nrhs, int Wlo_prec, size_t* bytes) {
    Geo G;
    int rc = make_geo(g, &G);
    if (rc) return rc;
    if (nrhs < 1 || !bytes) {
        set_error("nrhs must be >= 1 and bytes non-NULL");
        return OK_EINVAL;
    }
    if (Wlo_prec >= 0 && Wlo_prec != OK_F32 && Wlo_prec != OK_BF16) {
        set_error("Wlo_prec must be OK_F32, OK_BF16 or negative (plain FP64)");
        return OK_EINVAL;
    }
    *bytes = layout(G, Wlo_prec >= 0, nullptr, nullptr);
    return OK_SUCCESS;
}

int ok_bicgstab(const ok_geom* g, const ok_coeffs* c, const ok_solver_params* p, const void* d_W64,
                const void* d_Wlo, int Wlo_prec, const double* d_xi, double* d_psi, int nrhs, void* d_work,
                size_t work_bytes, ok_solver_stats* stats, void* stream) {
    const auto t0 = std::chrono::steady_clock::now();
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
    if (!(p->tol > 0) || p->max_iter < 0 || p->max_restarts < 0 || !(p->delta > 0 && p->delta < 1)) {
        set_error("invalid solver parameters (tol > 0, max_iter >= 0, 0 < delta < 1)");
        return OK_EINVAL;
    }
    if (nrhs < 1 || nrhs > 4096) {
        set_error("nrhs = %d outside [1, 4096]", nrhs);
        return OK_EINVAL;
    }
    const bool mixed = d_Wlo != nullptr;
    if (mixed && Wlo_prec != OK_F32 && Wlo_prec != OK_BF16) {
        set_error("Wlo_prec must be OK_F32 or OK_BF16 when d_Wlo is given");
        return OK_EINVAL;
    }
    if ((rc = check_ptr(d_W64, "d_W64")) || (mixed && (rc = check_ptr(d_Wlo, "d_Wlo"))) ||
        (rc = check_ptr(d_xi, "d_xi")) || (rc = check_ptr(d_psi, "d_psi")) || (rc = check_ptr(d_work, "d_work")))
        return rc;
    const size_t need = layout(C.g, mixed, nullptr, nullptr);
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
    layout(C.g, mixed, reinterpret_cast<char*>(d_work), &C.w);
    C.c = c;
    C.p = p;
    C.W64 = d_W64;
    C.Wlo = d_Wlo;
    C.Wlo_prec = Wlo_prec;
    C.st = reinterpret_cast<hipStream_t>(stream);
    C.tps64 = stencil_tps(OK_F64);
    C.tpslo = mixed ? stencil_tps(Wlo_prec) : 1;
    int first_bad = OK_SUCCESS;
    for (int k = 0; k < nrhs; ++k) {
        const auto tk = std::chrono::steady_clock::now();
        ok_solver_stats& S = stats[k];
        S = ok_solver_stats{};
        const size_t off = (size_t)k * C.g.V * 24;
        rc = mixed ? solve_mixed(C, d_xi + off, d_psi + off, &S) : solve_plain(C, d_xi + off, d_psi + off, &S);
        S.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - tk).count();
        if (rc < 0) {
            S.status = rc;
            return rc;
        }
        if (rc != OK_SUCCESS && first_bad == OK_SUCCESS) first_bad = rc;
    }
    (void)t0;
    return first_bad;
}

}  // extern "C"
