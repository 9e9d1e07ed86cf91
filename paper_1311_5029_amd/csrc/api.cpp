// C-ABI entry points of libokinv: validation, size queries, precompute, apply.
// Every argument is checked on the host before the first HIP call.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "common.h"
#include "kernels.h"
#include "wlayout.h"

namespace okinv {

static thread_local char g_err[1024] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int hip_fail(hipError_t e, const char* what, const char* file, int line) {
    set_error("HIP error %d (%s) in %s at %s:%d", (int)e, hipGetErrorString(e), what, file, line);
    return OK_EDEVICE;
}

int make_geo(const ok_geom* g, Geo* out) {
    if (!g) {
        set_error("geometry is NULL");
        return OK_EINVAL;
    }
    long v = 1;
    for (int mu = 0; mu < 4; ++mu) {
        if (g->L[mu] < 3 || g->L[mu] > 4096) {
            set_error("lattice extent L[%d] = %d outside [3, 4096]", mu, g->L[mu]);
            return OK_EINVAL;
        }
        v *= g->L[mu];
        if (v > (1L << 28)) {
            set_error("lattice volume exceeds 2^28 sites");
            return OK_EINVAL;
        }
    }
    for (int mu = 0; mu < 4; ++mu) out->L[mu] = g->L[mu];
    out->V = (int)v;
    out->Vs = (int)((v + 63) / 64 * 64);
    return OK_SUCCESS;
}

int check_ptr(const void* p, const char* name) {
    if (!p) {
        set_error("%s is NULL", name);
        return OK_EINVAL;
    }
    if (reinterpret_cast<uintptr_t>(p) % 16) {
        set_error("%s is not 16-byte aligned", name);
        return OK_EALIGN;
    }
    return OK_SUCCESS;
}

static int check_coeffs(const ok_coeffs* c) {
    if (!c) {
        set_error("coefficients are NULL");
        return OK_EINVAL;
    }
    const double* v = &c->mhat;
    for (int i = 0; i < 12; ++i)
        if (!std::isfinite(v[i])) {
            set_error("coefficient %d is not finite", i);
            return OK_EINVAL;
        }
    if (!(c->u0 > 0.0)) {
        set_error("u0 must be positive");
        return OK_EINVAL;
    }
    return OK_SUCCESS;
}

static bool valid_prec(int p) { return p == OK_F64 || p == OK_F32 || p == OK_BF16; }

// W precision with an optional layout flag: OK_LAYOUT_SITE (FP32 and BF16) or OK_LAYOUT_SAVED
static bool valid_wprec(int p) {
    const int lay = p & (OK_LAYOUT_SITE | OK_LAYOUT_SAVED | OK_LAYOUT_SIGMA);
    const int b = p & ~(OK_LAYOUT_SITE | OK_LAYOUT_SAVED | OK_LAYOUT_SIGMA);
    if (lay & (lay - 1)) return false;   // at most one layout flag
    if (lay == OK_LAYOUT_SITE) return b == OK_F32 || b == OK_BF16;
    if (lay == OK_LAYOUT_SIGMA) return b == OK_F64 || b == OK_F32;
    return valid_prec(b);
}

static size_t spinor_bytes(const Geo& g, int sprec) { return (size_t)g.V * 12 * (sprec == OK_F64 ? 16 : 8); }

static bool overlap(const void* a, size_t na, const void* b, size_t nb) {
    auto x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + nb && y < x + na;
}

#define OK_TRY(expr)                 \
    do {                             \
        int _r = (expr);             \
        if (_r != OK_SUCCESS) return _r; \
    } while (0)

}  // namespace okinv

using namespace okinv;

extern "C" {

int ok_abi_version(void) { return OKINV_ABI_VERSION; }

const char* ok_last_error(void) { return g_err; }

int ok_W_bytes(const ok_geom* g, int prec, size_t* bytes) {
    Geo G;
    OK_TRY(make_geo(g, &G));
    if (!valid_wprec(prec)) {
        set_error("unknown W precision/layout %d", prec);
        return OK_EINVAL;
    }
    if (!bytes) {
        set_error("bytes is NULL");
        return OK_EINVAL;
    }
    *bytes = w_bytes(prec & 3, G.Vs, layout_of(prec));
    return OK_SUCCESS;
}

int ok_precompute_scratch_bytes(const ok_geom* g, size_t* bytes) {
    Geo G;
    OK_TRY(make_geo(g, &G));
    if (!bytes) {
        set_error("bytes is NULL");
        return OK_EINVAL;
    }
    *bytes = (size_t)6 * 9 * 16 * G.Vs;
    return OK_SUCCESS;
}

int ok_precompute_W(const ok_geom* g, const ok_coeffs* c, const double* d_links, int prec, void* d_W,
                    size_t W_bytes, void* d_scratch, size_t scratch_bytes, void* stream) {
    Geo G;
    OK_TRY(make_geo(g, &G));
    OK_TRY(check_coeffs(c));
    if (!valid_wprec(prec)) {
        set_error("unknown W precision/layout %d", prec);
        return OK_EINVAL;
    }
    const size_t wb = w_bytes(prec & 3, G.Vs, layout_of(prec));
    OK_TRY(check_ptr(d_links, "d_links"));
    OK_TRY(check_ptr(d_W, "d_W"));
    OK_TRY(check_ptr(d_scratch, "d_scratch"));
    if (W_bytes < wb) {
        set_error("W buffer has %zu bytes, needs %zu", W_bytes, wb);
        return OK_ESIZE;
    }
    const size_t need = (size_t)6 * 9 * 16 * G.Vs;
    if (scratch_bytes < need) {
        set_error("scratch has %zu bytes, needs %zu", scratch_bytes, need);
        return OK_ESIZE;
    }
    const size_t lb = (size_t)G.V * 4 * 9 * 16;
    if (overlap(d_W, wb, d_links, lb) || overlap(d_scratch, need, d_links, lb) || overlap(d_W, wb, d_scratch, need)) {
        set_error("d_W, d_scratch and d_links must not overlap");
        return OK_EINVAL;
    }
    return launch_precompute(G, *c, d_links, prec, d_W, d_scratch, reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"

// Threads per site of the single right-hand-side stencil (1, 2 or 4); the
// environment variable OKINV_TPS overrides the default per precision.
int okinv::stencil_tps(int Wprec) {
    const char* e = getenv("OKINV_TPS");
    const int over = e ? atoi(e) : 0;
    if (over == 1 || over == 2 || over == 4) return over;
    return Wprec == OK_F32 ? 1 : 4;
}

// Multi-right-hand-side MFMA kernel for nrhs > 1 (OKINV_MRHS=0 selects one
// single-right-hand-side launch per right-hand side instead).
static bool use_mrhs() {
    const char* e = getenv("OKINV_MRHS");
    return !(e && e[0] == '0');
}

extern "C" {

int ok_apply_M(const ok_geom* g, const ok_coeffs* c, const void* d_W, int W_prec, const void* d_psi, void* d_out,
               int spinor_prec, int nrhs, void* stream) {
    Geo G;
    OK_TRY(make_geo(g, &G));
    OK_TRY(check_coeffs(c));
    if (!valid_wprec(W_prec)) {
        set_error("unknown W precision/layout %d", W_prec);
        return OK_EINVAL;
    }
    const int wbase = W_prec & 3;
    const bool site_major = (W_prec & OK_LAYOUT_SITE) != 0;
    const bool saved = (W_prec & (OK_LAYOUT_SAVED | OK_LAYOUT_SIGMA)) != 0;   // one thread per site
    const bool rhs_inner = (spinor_prec & OK_SPINOR_RHS_INNER) != 0;
    const bool sigma32 = (W_prec & OK_LAYOUT_SIGMA) && wbase == OK_F32;
    if (rhs_inner && (!(site_major || sigma32) || nrhs > 16)) {
        set_error("OK_SPINOR_RHS_INNER needs site-major W (OK_LAYOUT_SITE) or FP32 sigma-layout W, and nrhs <= 16");
        return OK_EINVAL;
    }
    spinor_prec &= ~OK_SPINOR_RHS_INNER;
    const bool ok_pair = (wbase == OK_F64 && spinor_prec == OK_F64) ||
                         (wbase != OK_F64 && spinor_prec == OK_F32);
    if (!ok_pair) {
        set_error("unsupported (W_prec, spinor_prec) = (%d, %d)", W_prec, spinor_prec);
        return OK_EINVAL;
    }
    if (nrhs < 1 || nrhs > 4096) {
        set_error("nrhs = %d outside [1, 4096]", nrhs);
        return OK_EINVAL;
    }
    OK_TRY(check_ptr(d_W, "d_W"));
    OK_TRY(check_ptr(d_psi, "d_psi"));
    OK_TRY(check_ptr(d_out, "d_out"));
    const size_t sb = spinor_bytes(G, spinor_prec);
    if (overlap(d_psi, sb * nrhs, d_out, sb * nrhs)) {
        set_error("d_out must not overlap d_psi");
        return OK_EINVAL;
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (rhs_inner && sigma32)
        return launch_apply_sigma_mr(G, d_W, reinterpret_cast<const float*>(d_psi), reinterpret_cast<float*>(d_out),
                                     c->mhat, nrhs, st);
    if (site_major)
        return launch_apply_site(G, d_W, wbase, reinterpret_cast<const float*>(d_psi),
                                 reinterpret_cast<float*>(d_out), c->mhat, nrhs, rhs_inner ? 1 : 0, st);
    if (nrhs > 1 && wbase != OK_F64 && !saved && use_mrhs())
        return launch_apply_mrhs(G, d_W, W_prec, reinterpret_cast<const float*>(d_psi),
                                 reinterpret_cast<float*>(d_out), c->mhat, nrhs, st);
    if ((W_prec & OK_LAYOUT_SIGMA) && wbase == OK_F64 && nrhs > 1) {   // W read once per four right-hand sides
        std::vector<const double*> in(nrhs);
        std::vector<double*> out(nrhs);
        for (int r = 0; r < nrhs; ++r) {
            in[r] = reinterpret_cast<const double*>(reinterpret_cast<const char*>(d_psi) + sb * r);
            out[r] = reinterpret_cast<double*>(reinterpret_cast<char*>(d_out) + sb * r);
        }
        return launch_apply_sigma_cols(G, d_W, in.data(), out.data(), nrhs, c->mhat, st);
    }
    const int tps = saved ? 1 : stencil_tps(W_prec);
    for (int r = 0; r < nrhs; ++r) {
        const char* in = reinterpret_cast<const char*>(d_psi) + sb * r;
        char* out = reinterpret_cast<char*>(d_out) + sb * r;
        OK_TRY(launch_apply(G, d_W, W_prec, in, out, c->mhat, tps, EPI_NONE, nullptr, nullptr, st));
    }
    return OK_SUCCESS;
}

int ok_W_to_dense(const ok_geom* g, const void* d_W, int prec, double* d_dense, void* stream) {
    Geo G;
    OK_TRY(make_geo(g, &G));
    if (!valid_wprec(prec)) {
        set_error("unknown W precision/layout %d", prec);
        return OK_EINVAL;
    }
    OK_TRY(check_ptr(d_W, "d_W"));
    OK_TRY(check_ptr(d_dense, "d_dense"));
    return launch_to_dense(G, d_W, prec, d_dense, reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"
