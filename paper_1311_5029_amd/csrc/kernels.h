// Internal launchers of libokinv (not part of the ABI).
#pragma once

#include "common.h"

namespace okinv {

enum Epilogue { EPI_NONE = 0, EPI_RV = 1, EPI_TS = 2 };

// Deterministic block reduction of two complex values; thread 0 writes
// partial[2*blockIdx.x] = sum d1, partial[2*blockIdx.x + 1] = sum d2.
// Requires blockDim.x == 256 and that every thread of the block calls it.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sums d1, d2 over the block in a fixed order; the result is valid in thread 0.
__device__ __forceinline__ void block_reduce2(double2& d1, double2& d2) {
    __shared__ double red[4][4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double a = wave_sum(d1.x), b = wave_sum(d1.y), c = wave_sum(d2.x), d = wave_sum(d2.y);
    if (lane == 0) {
        red[wave][0] = a;
        red[wave][1] = b;
        red[wave][2] = c;
        red[wave][3] = d;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            s0 += red[w][0];
            s1 += red[w][1];
            s2 += red[w][2];
            s3 += red[w][3];
        }
        d1 = make_double2(s0, s1);
        d2 = make_double2(s2, s3);
    }
}

__device__ __forceinline__ void block_reduce2_store(double2 d1, double2 d2, double2* partial) {
    block_reduce2(d1, d2);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = d1;
        partial[2 * blockIdx.x + 1] = d2;
    }
}

// api.cpp
int stencil_tps(int Wprec);

// stencil.hip
int apply_blocks(const Geo& g, int tps);
int launch_apply(const Geo& g, const void* W, int Wprec, const void* psi, void* out, double mhat, int tps,
                 int epi, const void* aux, double2* partial, hipStream_t st);
// FP32 sigma-layout W on nrhs (<= 16) right-hand sides stored [V][12][nrhs]; with epi EPI_RV the
// per-right-hand-side partials <aux, out>, with EPI_TS <out, aux>, <out, out>, in
// partial[block][j][2] over sigma_mr_blocks blocks (the batched solver's layout)
int sigma_mr_blocks(const Geo& g, int nrhs);
int launch_apply_sigma_mr(const Geo& g, const void* W, const float* psi, float* out, double mhat, int nrhs,
                          hipStream_t st, int epi = EPI_NONE, const float* aux = nullptr,
                          double2* partial = nullptr);
// FP64 sigma-layout W on n separate [V][12] fields, up to four per pass (W read once per pass)
int launch_apply_sigma_cols(const Geo& g, const void* W, const double* const* in, double* const* out, int n,
                            double mhat, hipStream_t st);
// W in OK_LAYOUT_SIGMA (FP64 or FP32), one thread per site (stencil_sigma.hip)
int launch_apply_sigma(const Geo& g, const void* W, int Wprec, const void* psi, void* out, double mhat, int epi,
                       const void* aux, double2* partial, hipStream_t st);

// FP64 W on n separate FP64 right-hand sides (in[r] -> out[r]), W read once per four of them
int launch_apply_m64(const Geo& g, const void* W, const double* const* in, double* const* out, int n, double mhat,
                     hipStream_t st);

// stencil_mrhs.hip: up to 16 right-hand sides per pass on MFMA (FP32 or BF16 W, FP32 spinors)
int launch_apply_mrhs(const Geo& g, const void* W, int Wprec, const float* psi, float* out, double mhat,
                      int nrhs, hipStream_t st);

// the same for site-major W (OK_LAYOUT_SITE), any nrhs >= 1; rhs_inner selects
// spinors [V][12][nrhs] (nrhs <= 16) instead of [nrhs][V][12]
int launch_apply_site(const Geo& g, const void* W, int Wprec, const float* psi, float* out, double mhat,
                      int nrhs, int rhs_inner, hipStream_t st);

// precompute.hip
int launch_precompute(const Geo& g, const ok_coeffs& c, const double* links, int prec, void* W,
                      void* scratch, hipStream_t st);
int launch_to_dense(const Geo& g, const void* W, int prec, double* dense, hipStream_t st);

// blas1.hip -- per right-hand side BiCGStab scalars live in device memory
struct Scal {
    double2 rho, rho_old, alpha, omega, beta, rv, ts;
    double tt, rr, rr_true;
    int flags;      // bit 0: breakdown seen (rho, <r^,v> or <t,t> vanished)
    int pad;
};

int blas_blocks(const Geo& g);
// fields of 12 V complex of type T (double or float)
int launch_p_update(const Geo& g, bool f64, void* p, const void* r, const void* v, const Scal* sc, hipStream_t st);
int launch_s_update(const Geo& g, bool f64, void* s, const void* r, const void* v, const Scal* sc, hipStream_t st);
// x += alpha p + omega sx ; r = s - omega t ; partial <r^, r>, <r, r>  (sx = s unless preconditioned)
int launch_xr_update(const Geo& g, bool f64, void* x, void* r, const void* p, const void* sx, const void* s,
                     const void* t, const void* rhat, const Scal* sc, double2* partial, hipStream_t st);
int launch_dot_rr(const Geo& g, bool f64, const void* rhat, const void* r, double2* partial, hipStream_t st);
int launch_finish(int kind, int nblocks, const double2* partial, Scal* sc, hipStream_t st);
enum Finish { FIN_ALPHA = 0, FIN_OMEGA = 1, FIN_RHO = 2, FIN_RHO_REPLACE = 3, FIN_INIT = 4, FIN_TRUE = 5,
              FIN_CG_INIT = 6, FIN_CG_ALPHA = 7, FIN_CG_BETA = 8, FIN_CG_RR = 9 };
// CG on M^dag M (FP64 fields; M^dag = gamma5 M gamma5):
//   out = gamma5 r, partial ||r||^2
int launch_cg_gamma5(const Geo& g, double* out, const double* r, double2* partial, hipStream_t st);
//   x += alpha p ; r -= alpha w ; gr = gamma5 r ; partial ||r||^2
int launch_cg_xr(const Geo& g, double* x, double* r, const double* p, const double* w, double* gr, const Scal* sc,
                 double2* partial, hipStream_t st);
//   p = gamma5 zp + beta p
int launch_cg_p(const Geo& g, double* p, const double* zp, const Scal* sc, hipStream_t st);
// r64 = xi - t64; optionally rlo = (float) r64; partial <r64, r64>
int launch_residual(const Geo& g, const double* xi, const double* t64, double* r64, float* rlo,
                    double2* partial, hipStream_t st);
// x64 += (double) xlo; xlo = 0
int launch_accum_x(const Geo& g, double* x64, float* xlo, hipStream_t st);
int launch_copy(const Geo& g, bool f64, void* dst, const void* src, hipStream_t st);
int launch_zero(const Geo& g, bool f64, void* dst, hipStream_t st);
// partial <a, a> of an FP64 field (norm of the source)
int launch_norm64(const Geo& g, const double* a, double2* partial, hipStream_t st);

// blas1_batched.hip -- a batch of right-hand sides iterating together (FP32 fields, right-hand side
// index fastest: element (12 * site + component) * nrhs + j)
constexpr int kMaxRhsB = 16;
constexpr int kGridB = 1024;     // fixed grid of the batched vector kernels
struct ScalB {
    double2 rho[kMaxRhsB], rho_old[kMaxRhsB], alpha[kMaxRhsB], omega[kMaxRhsB], beta[kMaxRhsB];
    double rr[kMaxRhsB], rr_true[kMaxRhsB];
    int flags[kMaxRhsB], active[kMaxRhsB];
};
int batch_rows(const Geo& g);
int col_blocks(const Geo& g);
int launch_bp_update(const Geo& g, int nrhs, float* p, const float* r, const float* v, const ScalB* sc,
                     hipStream_t st);
int launch_bs_update(const Geo& g, int nrhs, float* s, const float* r, const float* v, const ScalB* sc,
                     hipStream_t st);
int launch_bxr_update(const Geo& g, int nrhs, float* x, float* r, const float* p, const float* sx, const float* s,
                      const float* t, const float* rhat, const ScalB* sc, double2* partial, hipStream_t st);
int launch_bdot(const Geo& g, int nrhs, const float* a, const float* b, const ScalB* sc, double2* partial,
                hipStream_t st);
int launch_bfinish(int kind, int nblocks, int j0, int nj, const double2* partial, ScalB* sc, hipStream_t st);
int launch_col_accum(const Geo& g, int nrhs, int j, double* x64, float* x32, hipStream_t st);
// several columns per kernel (fixed kGridB grid; partials as launch_bdot): x64 is the base of the
// [nrhs][V][12] FP64 fields, column j's FP64 residual input at t64 + slot[j] * 12 V
struct ColSlots {
    int slot[kMaxRhsB];   // -1: column not in this pass
};
int launch_cols_accum(const Geo& g, int nrhs, unsigned mask, double* x64, float* x32, hipStream_t st);
int launch_cols_residual(const Geo& g, int nrhs, const ColSlots& sl, const double* xi, const double* t64, float* r32,
                         double2* partial, hipStream_t st);
int launch_cols_dot(const Geo& g, int nrhs, unsigned mask, const float* a, const float* b, double2* partial,
                    hipStream_t st);
int launch_col_residual(const Geo& g, int nrhs, int j, const double* xi, const double* t64, float* r32,
                        double2* partial, hipStream_t st);
int launch_col_norm64(const Geo& g, int j, const double* a, double2* partial, hipStream_t st);
int launch_col_load(const Geo& g, int nrhs, int j, const double* a, float* r32, hipStream_t st);
int launch_col_restart(const Geo& g, int nrhs, int j, const float* r, float* rhat, float* p, float* v,
                       hipStream_t st);
int launch_col_dot(const Geo& g, int nrhs, int j, const float* a, const float* b, double2* partial,
                   hipStream_t st);

// net.hip -- the learned preconditioner (FP32 fields, [nf][V][12] or with inner [V][12][nf])
size_t net_T_bytes(const Geo& g);
int net_wgrad_chunks(const Geo& g, int nf);
size_t net_wgrad_partial_bytes(const Geo& g, int nf);
size_t net_loss_partial_bytes(int nf);
int launch_net_transports(const Geo& g, const double* links, float* T, hipStream_t st);
int launch_net_layer(const Geo& g, int nf, bool inner, bool adjoint, const float* A, const float* T,
                     const float* in, float* out, hipStream_t st);
// gA = weight gradient of one layer; partial holds net_wgrad_partial_bytes
int launch_net_wgrad(const Geo& g, int nf, bool inner, const float* T, const float* gout, const float* in,
                     float* partial, float* gA, hipStream_t st);
// loss and gout = dL/d(conj out); scratch holds net_loss_partial_bytes
int launch_net_loss_grad(const Geo& g, int nf, bool inner, const float* out, const float* psi, float* gout,
                         double* loss, void* scratch, hipStream_t st);
int launch_cast(long n, const double* in, float* out, hipStream_t st);
int launch_adam(long n, float* p, const float* g, float* m, float* v, const ok_adam_cfg& c, int step,
                hipStream_t st);

// net_api.cpp -- the whole network on nf fields (work: net_apply_work_bytes)
size_t net_apply_work_bytes(const Geo& g, int n_layers, int nf);
int net_apply(const Geo& g, int n_layers, const float* params, const float* T, const float* in, float* out, int nf,
              bool inner, void* work, hipStream_t st);

}  // namespace okinv
