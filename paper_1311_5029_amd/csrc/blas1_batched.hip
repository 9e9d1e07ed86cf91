// BiCGStab vector kernels for a batch of right-hand sides that iterate together.
//
// Fields are FP32 with the right-hand side index fastest: element
// (row, j) = row * nrhs + j with row = 12 * site + component.  Every right-hand
// side has its own scalars (alpha, beta, omega, rho) and an "active" flag in
// device memory (struct ScalB); finished right-hand sides are left untouched.
// A block is 16 rows x 16 right-hand-side slots; the grid is fixed
// (kGridB blocks, grid-stride over rows), so every per-right-hand-side partial
// sum is reduced in the same order on every run.
#include "common.h"
#include "kernels.h"

namespace okinv {
namespace {

constexpr int BS = 256;

__device__ __forceinline__ c64 ldc(const float* f, size_t i) { return reinterpret_cast<const c64*>(f)[i]; }
__device__ __forceinline__ void stc(float* f, size_t i, c64 v) { reinterpret_cast<c64*>(f)[i] = v; }
__device__ __forceinline__ c64 f32c(double2 d) { return c64{(float)d.x, (float)d.y}; }
__device__ __forceinline__ void dacc(double2& d, c64 a, c64 b) {   // d += conj(a) b
    d.x += (double)a.re * b.re + (double)a.im * b.im;
    d.y += (double)a.re * b.im - (double)a.im * b.re;
}
__device__ __forceinline__ double2 cmul2(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cdiv2(double2 a, double2 b) {
    const double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

// Per block: sums over the 16 rows of each right-hand-side slot, in row order.
__device__ __forceinline__ void slot_reduce_store(double2 d1, double2 d2, double2* partial, int nrhs) {
    __shared__ double2 red[2][16][16];
    const int r = threadIdx.x >> 4, j = threadIdx.x & 15;
    red[0][r][j] = d1;
    red[1][r][j] = d2;
    __syncthreads();
    if (threadIdx.x < 16 && j < nrhs) {
        double2 a{0, 0}, b{0, 0};
        for (int q = 0; q < 16; ++q) {
            a.x += red[0][q][j].x;
            a.y += red[0][q][j].y;
            b.x += red[1][q][j].x;
            b.y += red[1][q][j].y;
        }
        double2* p = partial + ((size_t)blockIdx.x * kMaxRhsB + j) * 2;
        p[0] = a;
        p[1] = b;
    }
}

// p = r + beta (p - omega v)
__global__ void __launch_bounds__(BS) kb_p_update(int rows, int nrhs, float* p, const float* r, const float* v,
                                                  const ScalB* sc) {
    const int j = threadIdx.x & 15;
    if (j >= nrhs || !sc->active[j]) return;
    const c64 beta = f32c(sc->beta[j]), omega = f32c(sc->omega[j]);
    for (int row = blockIdx.x * 16 + (threadIdx.x >> 4); row < rows; row += gridDim.x * 16) {
        const size_t i = (size_t)row * nrhs + j;
        stc(p, i, ldc(r, i) + beta * (ldc(p, i) - omega * ldc(v, i)));
    }
}

// s = r - alpha v
__global__ void __launch_bounds__(BS) kb_s_update(int rows, int nrhs, float* s, const float* r, const float* v,
                                                  const ScalB* sc) {
    const int j = threadIdx.x & 15;
    if (j >= nrhs || !sc->active[j]) return;
    const c64 alpha = f32c(sc->alpha[j]);
    for (int row = blockIdx.x * 16 + (threadIdx.x >> 4); row < rows; row += gridDim.x * 16) {
        const size_t i = (size_t)row * nrhs + j;
        stc(s, i, ldc(r, i) - alpha * ldc(v, i));
    }
}

// x += alpha p + omega s ; r = s - omega t ; partial <r^, r>, <r, r>
__global__ void __launch_bounds__(BS) kb_xr_update(int rows, int nrhs, float* x, float* r, const float* p,
                                                   const float* sx, const float* s, const float* t,
                                                   const float* rhat, const ScalB* sc, double2* partial) {
    const int j = threadIdx.x & 15;
    double2 d1{0, 0}, d2{0, 0};
    if (j < nrhs && sc->active[j]) {
        const c64 alpha = f32c(sc->alpha[j]), omega = f32c(sc->omega[j]);
        for (int row = blockIdx.x * 16 + (threadIdx.x >> 4); row < rows; row += gridDim.x * 16) {
            const size_t i = (size_t)row * nrhs + j;
            const c64 sv = ldc(s, i);
            stc(x, i, ldc(x, i) + alpha * ldc(p, i) + omega * ldc(sx, i));
            const c64 rv = sv - omega * ldc(t, i);
            stc(r, i, rv);
            dacc(d1, ldc(rhat, i), rv);
            dacc(d2, rv, rv);
        }
    }
    slot_reduce_store(d1, d2, partial, nrhs);
}

// partial <a, b>, <a, a>
__global__ void __launch_bounds__(BS) kb_dot(int rows, int nrhs, const float* a, const float* b, const ScalB* sc,
                                             double2* partial) {
    const int j = threadIdx.x & 15;
    double2 d1{0, 0}, d2{0, 0};
    if (j < nrhs && sc->active[j]) {
        for (int row = blockIdx.x * 16 + (threadIdx.x >> 4); row < rows; row += gridDim.x * 16) {
            const size_t i = (size_t)row * nrhs + j;
            const c64 av = ldc(a, i);
            dacc(d1, av, ldc(b, i));
            dacc(d2, av, av);
        }
    }
    slot_reduce_store(d1, d2, partial, nrhs);
}

// One block per right-hand side j0, j0 + 1, ...: fixed-order reduction of the
// partials, then the scalar update.
__global__ void __launch_bounds__(BS) kb_finish(int kind, int nb, int j0, const double2* partial, ScalB* sc) {
    const int j = j0 + blockIdx.x;
    double2 d1{0, 0}, d2{0, 0};
    for (int b = threadIdx.x; b < nb; b += BS) {
        const double2* p = partial + ((size_t)b * kMaxRhsB + j) * 2;
        d1.x += p[0].x;
        d1.y += p[0].y;
        d2.x += p[1].x;
        d2.y += p[1].y;
    }
    block_reduce2(d1, d2);
    if (threadIdx.x != 0) return;
    ScalB& S = *sc;
    if (kind == FIN_TRUE) {
        S.rr_true[j] = d2.x;
        return;
    }
    if (kind != FIN_INIT && !S.active[j]) return;
    const double tiny = 1e-300;
    switch (kind) {
        case FIN_ALPHA: {
            const double m = d1.x * d1.x + d1.y * d1.y;
            if (!(m > tiny)) {
                S.flags[j] |= 1;
                S.alpha[j] = make_double2(0.0, 0.0);
            } else {
                S.alpha[j] = cdiv2(S.rho[j], d1);
            }
            break;
        }
        case FIN_OMEGA: {   // d1 = <t, s>, d2 = <t, t>
            if (!(d2.x > tiny)) {
                S.flags[j] |= 1;
                S.omega[j] = make_double2(0.0, 0.0);
            } else {
                S.omega[j] = make_double2(d1.x / d2.x, d1.y / d2.x);
            }
            break;
        }
        case FIN_RHO:
        case FIN_RHO_REPLACE: {
            if (kind == FIN_RHO) S.rho_old[j] = S.rho[j];
            S.rho[j] = d1;
            S.rr[j] = d2.x;
            const double2 om = S.omega[j], ro = S.rho_old[j];
            const double mo = om.x * om.x + om.y * om.y, mr = ro.x * ro.x + ro.y * ro.y;
            const double mrho = d1.x * d1.x + d1.y * d1.y;
            if (!(mo > tiny) || !(mr > tiny) || !(mrho > 1e-60 * d2.x * d2.x)) {
                S.flags[j] |= 1;
                S.beta[j] = make_double2(0.0, 0.0);
            } else {
                S.beta[j] = cmul2(cdiv2(S.rho[j], ro), cdiv2(S.alpha[j], om));
            }
            break;
        }
        default: {   // FIN_INIT: fresh recurrence from r (p = v = 0)
            S.rho[j] = d1;
            S.rr[j] = d2.x;
            S.rho_old[j] = make_double2(1.0, 0.0);
            S.alpha[j] = make_double2(1.0, 0.0);
            S.omega[j] = make_double2(1.0, 0.0);
            S.beta[j] = make_double2(0.0, 0.0);
            S.flags[j] = 0;
            break;
        }
    }
}

// ---- single right-hand-side columns of the batch, against FP64 fields in the ABI layout

// x64 += (double) x32[:, j]; x32[:, j] = 0
__global__ void __launch_bounds__(BS) kb_col_accum(int rows, int nrhs, int j, double* x64, float* x32) {
    const int row = blockIdx.x * BS + threadIdx.x;
    if (row >= rows) return;
    const size_t i = (size_t)row * nrhs + j;
    const c64 l = ldc(x32, i);
    c128* xp = reinterpret_cast<c128*>(x64) + row;
    *xp = *xp + c128{(double)l.re, (double)l.im};
    stc(x32, i, c64{0.f, 0.f});
}

__device__ __forceinline__ void col_slot_store(double2 d1, double2 d2, double2* partial, int j) {
    block_reduce2(d1, d2);
    if (threadIdx.x == 0) {
        double2* p = partial + ((size_t)blockIdx.x * kMaxRhsB + j) * 2;
        p[0] = d1;
        p[1] = d2;
    }
}

// r32[:, j] = (float)(xi - t64) ; partial (second slot) ||xi - t64||^2, slot j
__global__ void __launch_bounds__(BS) kb_col_residual(int rows, int nrhs, int j, const double* xi, const double* t64,
                                                      float* r32, double2* partial) {
    const int row = blockIdx.x * BS + threadIdx.x;
    double2 d1{0, 0}, d2{0, 0};
    if (row < rows) {
        const c128 v = reinterpret_cast<const c128*>(xi)[row] - reinterpret_cast<const c128*>(t64)[row];
        stc(r32, (size_t)row * nrhs + j, c64{(float)v.re, (float)v.im});
        d2.x = v.re * v.re + v.im * v.im;
    }
    col_slot_store(d1, d2, partial, j);
}

// partial (second slot) ||a||^2 of an FP64 field in the ABI layout, slot j
__global__ void __launch_bounds__(BS) kb_col_norm64(int rows, int j, const double* a, double2* partial) {
    const int row = blockIdx.x * BS + threadIdx.x;
    double2 d1{0, 0}, d2{0, 0};
    if (row < rows) {
        const c128 v = reinterpret_cast<const c128*>(a)[row];
        d2.x = v.re * v.re + v.im * v.im;
    }
    col_slot_store(d1, d2, partial, j);
}

// r32[:, j] = (float) a64 (the FP64 residual of a zero start)
__global__ void __launch_bounds__(BS) kb_col_load(int rows, int nrhs, int j, const double* a, float* r32) {
    const int row = blockIdx.x * BS + threadIdx.x;
    if (row >= rows) return;
    const c128 v = reinterpret_cast<const c128*>(a)[row];
    stc(r32, (size_t)row * nrhs + j, c64{(float)v.re, (float)v.im});
}

// column j: r^ = r, p = v = 0, x32 = 0 (if clear_x)
__global__ void __launch_bounds__(BS) kb_col_restart(int rows, int nrhs, int j, const float* r, float* rhat, float* p,
                                                     float* v) {
    const int row = blockIdx.x * BS + threadIdx.x;
    if (row >= rows) return;
    const size_t i = (size_t)row * nrhs + j;
    stc(rhat, i, ldc(r, i));
    stc(p, i, c64{0.f, 0.f});
    stc(v, i, c64{0.f, 0.f});
}

// partial <a[:, j], b[:, j]>, <b, b> into the batched partial slots of right-hand side j
__global__ void __launch_bounds__(BS) kb_col_dot(int rows, int nrhs, int j, const float* a, const float* b,
                                                 double2* partial) {
    const int row = blockIdx.x * BS + threadIdx.x;
    double2 d1{0, 0}, d2{0, 0};
    if (row < rows) {
        const size_t i = (size_t)row * nrhs + j;
        const c64 bv = ldc(b, i);
        dacc(d1, ldc(a, i), bv);
        dacc(d2, bv, bv);
    }
    col_slot_store(d1, d2, partial, j);
}

// ---- several columns at once (the grouped reliable updates): one thread per (row, slot) as above,
// working on the right-hand sides j whose bit is set in mask (or whose slot[j] >= 0); the FP64
// fields of column j are at base + j * col (col complex numbers per column).

// x64_j += x32[:, j] ; x32[:, j] = 0
__global__ void __launch_bounds__(BS) kb_cols_accum(int rows, int nrhs, unsigned mask, double* x64, size_t col,
                                                    float* x32) {
    const int j = threadIdx.x & 15;
    if (j >= nrhs || !((mask >> j) & 1u)) return;
    c128* xj = reinterpret_cast<c128*>(x64) + (size_t)j * col;
    for (int row = blockIdx.x * 16 + (threadIdx.x >> 4); row < rows; row += gridDim.x * 16) {
        const size_t i = (size_t)row * nrhs + j;
        const c64 l = ldc(x32, i);
        xj[row] = xj[row] + c128{(double)l.re, (double)l.im};
        stc(x32, i, c64{0.f, 0.f});
    }
}

// r32[:, j] = xi_j - t64[slot j] ; partial (0, |r_j|^2) for every j with slot j >= 0
__global__ void __launch_bounds__(BS) kb_cols_residual(int rows, int nrhs, ColSlots sl, const double* xi, size_t col,
                                                       const double* t64, float* r32, double2* partial) {
    const int j = threadIdx.x & 15;
    const int slot = j < nrhs ? sl.slot[j] : -1;
    double2 d1{0, 0}, d2{0, 0};
    if (slot >= 0) {
        const c128* x = reinterpret_cast<const c128*>(xi) + (size_t)j * col;
        const c128* t = reinterpret_cast<const c128*>(t64) + (size_t)slot * col;
        for (int row = blockIdx.x * 16 + (threadIdx.x >> 4); row < rows; row += gridDim.x * 16) {
            const c128 v = x[row] - t[row];
            stc(r32, (size_t)row * nrhs + j, c64{(float)v.re, (float)v.im});
            d2.x += v.re * v.re + v.im * v.im;
        }
    }
    slot_reduce_store(d1, d2, partial, nrhs);
}

// partial <a_j, b_j>, <b_j, b_j> for every j in mask
__global__ void __launch_bounds__(BS) kb_cols_dot(int rows, int nrhs, unsigned mask, const float* a, const float* b,
                                                  double2* partial) {
    const int j = threadIdx.x & 15;
    double2 d1{0, 0}, d2{0, 0};
    if (j < nrhs && ((mask >> j) & 1u)) {
        for (int row = blockIdx.x * 16 + (threadIdx.x >> 4); row < rows; row += gridDim.x * 16) {
            const size_t i = (size_t)row * nrhs + j;
            const c64 bv = ldc(b, i);
            dacc(d1, ldc(a, i), bv);
            dacc(d2, bv, bv);
        }
    }
    slot_reduce_store(d1, d2, partial, nrhs);
}

}  // namespace

int launch_cols_accum(const Geo& g, int nrhs, unsigned mask, double* x64, float* x32, hipStream_t st) {
    kb_cols_accum<<<kGridB, BS, 0, st>>>(batch_rows(g), nrhs, mask, x64, (size_t)g.V * 12, x32);
    OK_LAUNCH_CHECK("kb_cols_accum");
    return OK_SUCCESS;
}
int launch_cols_residual(const Geo& g, int nrhs, const ColSlots& sl, const double* xi, const double* t64, float* r32,
                         double2* partial, hipStream_t st) {
    kb_cols_residual<<<kGridB, BS, 0, st>>>(batch_rows(g), nrhs, sl, xi, (size_t)g.V * 12, t64, r32, partial);
    OK_LAUNCH_CHECK("kb_cols_residual");
    return OK_SUCCESS;
}
int launch_cols_dot(const Geo& g, int nrhs, unsigned mask, const float* a, const float* b, double2* partial,
                    hipStream_t st) {
    kb_cols_dot<<<kGridB, BS, 0, st>>>(batch_rows(g), nrhs, mask, a, b, partial);
    OK_LAUNCH_CHECK("kb_cols_dot");
    return OK_SUCCESS;
}

int batch_rows(const Geo& g) { return g.V * 12; }
int col_blocks(const Geo& g) { return (int)grid_for((long)g.V * 12, BS); }

int launch_bp_update(const Geo& g, int nrhs, float* p, const float* r, const float* v, const ScalB* sc,
                     hipStream_t st) {
    kb_p_update<<<kGridB, BS, 0, st>>>(batch_rows(g), nrhs, p, r, v, sc);
    OK_LAUNCH_CHECK("kb_p_update");
    return OK_SUCCESS;
}
int launch_bs_update(const Geo& g, int nrhs, float* s, const float* r, const float* v, const ScalB* sc,
                     hipStream_t st) {
    kb_s_update<<<kGridB, BS, 0, st>>>(batch_rows(g), nrhs, s, r, v, sc);
    OK_LAUNCH_CHECK("kb_s_update");
    return OK_SUCCESS;
}
int launch_bxr_update(const Geo& g, int nrhs, float* x, float* r, const float* p, const float* sx, const float* s,
                      const float* t, const float* rhat, const ScalB* sc, double2* partial, hipStream_t st) {
    kb_xr_update<<<kGridB, BS, 0, st>>>(batch_rows(g), nrhs, x, r, p, sx, s, t, rhat, sc, partial);
    OK_LAUNCH_CHECK("kb_xr_update");
    return OK_SUCCESS;
}
int launch_bdot(const Geo& g, int nrhs, const float* a, const float* b, const ScalB* sc, double2* partial,
                hipStream_t st) {
    kb_dot<<<kGridB, BS, 0, st>>>(batch_rows(g), nrhs, a, b, sc, partial);
    OK_LAUNCH_CHECK("kb_dot");
    return OK_SUCCESS;
}
int launch_bfinish(int kind, int nblocks, int j0, int nj, const double2* partial, ScalB* sc, hipStream_t st) {
    kb_finish<<<nj, BS, 0, st>>>(kind, nblocks, j0, partial, sc);
    OK_LAUNCH_CHECK("kb_finish");
    return OK_SUCCESS;
}
int launch_col_accum(const Geo& g, int nrhs, int j, double* x64, float* x32, hipStream_t st) {
    kb_col_accum<<<col_blocks(g), BS, 0, st>>>(batch_rows(g), nrhs, j, x64, x32);
    OK_LAUNCH_CHECK("kb_col_accum");
    return OK_SUCCESS;
}
int launch_col_residual(const Geo& g, int nrhs, int j, const double* xi, const double* t64, float* r32,
                        double2* partial, hipStream_t st) {
    kb_col_residual<<<col_blocks(g), BS, 0, st>>>(batch_rows(g), nrhs, j, xi, t64, r32, partial);
    OK_LAUNCH_CHECK("kb_col_residual");
    return OK_SUCCESS;
}
int launch_col_norm64(const Geo& g, int j, const double* a, double2* partial, hipStream_t st) {
    kb_col_norm64<<<col_blocks(g), BS, 0, st>>>(batch_rows(g), j, a, partial);
    OK_LAUNCH_CHECK("kb_col_norm64");
    return OK_SUCCESS;
}
int launch_col_load(const Geo& g, int nrhs, int j, const double* a, float* r32, hipStream_t st) {
    kb_col_load<<<col_blocks(g), BS, 0, st>>>(batch_rows(g), nrhs, j, a, r32);
    OK_LAUNCH_CHECK("kb_col_load");
    return OK_SUCCESS;
}
int launch_col_restart(const Geo& g, int nrhs, int j, const float* r, float* rhat, float* p, float* v,
                       hipStream_t st) {
    kb_col_restart<<<col_blocks(g), BS, 0, st>>>(batch_rows(g), nrhs, j, r, rhat, p, v);
    OK_LAUNCH_CHECK("kb_col_restart");
    return OK_SUCCESS;
}
int launch_col_dot(const Geo& g, int nrhs, int j, const float* a, const float* b, double2* partial,
                   hipStream_t st) {
    kb_col_dot<<<col_blocks(g), BS, 0, st>>>(batch_rows(g), nrhs, j, a, b, partial);
    OK_LAUNCH_CHECK("kb_col_dot");
    return OK_SUCCESS;
}

}  // namespace okinv
