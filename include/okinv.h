/*
 * okinv.h -- C-ABI of the MI355X (gfx950) Oktay-Kronfeld operator and inverter.
 *
 * The library applies the rewritten OK Dirac operator
 *
 *   (M psi)_x = mhat psi_x + sum_{k=0}^{26} W_{k,x} psi_{x+d_k}           (Eq. minFlopForm)
 *
 * with the 12x12 spin-colour precalculation matrices W (Sec. 2.2,
 * Eqs. shifted_W_first..shifted_W_last) built once per gauge field, and solves
 * M psi = xi (Eq. dslash) by BiCGStab (Sec. 2.3), optionally right-preconditioned
 * by a learned gauge-covariant linear stencil network (an addition to the
 * paper's method, declared at the end of this header).
 *
 * Conventions shared by every call:
 *   - Geometry: L = (Lx, Ly, Lz, Lt), every L >= 3, periodic in all four
 *     directions; direction mu = 0..3 is x, y, z, t (the paper's mu = 4 is t).
 *     Site index s = x + Lx*(y + Ly*(z + Lz*t)); V = Lx*Ly*Lz*Lt < 2^31 / 64.
 *   - Complex numbers are (re, im) pairs of the stated real type.
 *   - Links: d_links is FP64 complex [V][4][3][3] (row-major colour), the link
 *     U_mu(x) from x to x+mu (it multiplies psi_{x+mu}).
 *   - Spinors: [nrhs][V][4 spin][3 colour] complex, FP64 or FP32; the
 *     spin-colour index is 3*alpha + a; the spin basis is the one in which the
 *     paper writes W (gamma_4 = diag(1,1,-1,-1), gamma_i = [[0,s_i],[s_i,0]]).
 *   - The 27 offsets d_k in storage order: k=0: 0; 1..4: +mu; 5..8: -mu;
 *     9..11: +2i; 12..14: -2i; 15..17: +i+j (ij = xy,xz,yz); 18..20: -i-j;
 *     21..23: +i-j; 24..26: -i+j.
 *   - Device pointers are hipMalloc'ed by the caller, 16-byte aligned at least
 *     (256 recommended).  The caller owns and frees every buffer (W, scratch,
 *     workspace); the library allocates no device memory and keeps no pointer
 *     after a call returns.  `stream` is a hipStream_t (NULL: default stream).
 *   - Every call validates its arguments on the host before any HIP call and
 *     returns an ok_status; on error ok_last_error() holds a message.
 */
#ifndef OKINV_H
#define OKINV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OKINV_ABI_VERSION 3

/* Status codes.  0 success, > 0 solver outcomes (stats filled), < 0 errors. */
enum ok_status {
    OK_SUCCESS = 0,
    OK_NOT_CONVERGED = 1,   /* max_iter reached; stats hold the last residual   */
    OK_BREAKDOWN = 2,       /* BiCGStab breakdown persisted through restarts     */
    OK_EINVAL = -1,         /* bad geometry, nrhs, null/aliasing pointer, precision */
    OK_ESIZE = -2,          /* a buffer or workspace is smaller than required    */
    OK_EALIGN = -3,         /* a device pointer is not 16-byte aligned            */
    OK_EDEVICE = -4,        /* a HIP runtime error; message in ok_last_error()    */
    OK_ENONFINITE = -5      /* NaN/Inf met in the source or a residual            */
};

/* Storage / arithmetic precision of W and of spinors. */
enum ok_prec { OK_F64 = 0, OK_F32 = 1, OK_BF16 = 2 };

/* Layout flag OR-ed into the W precision of ok_W_bytes, ok_precompute_W,
 * ok_apply_M and ok_W_to_dense: the 27 blocks of each site stored
 * contiguously (site-major), the layout the multi-right-hand-side MFMA
 * kernel of ok_apply_M streams best.  Without it W is plane-major (each
 * 16-byte piece of a block laid out over consecutive sites), best for one
 * right-hand side.  Both layouts hold the same numbers; the flag is valid
 * with OK_F32 and OK_BF16. */
#define OK_LAYOUT_SITE 0x10

/* Layout flag OR-ed into the W precision (OK_F64, OK_F32 or OK_BF16) of
 * ok_W_bytes, ok_precompute_W, ok_apply_M and ok_W_to_dense: only the 14
 * blocks of the forward offsets (k = 0, +mu, +2i, +i+j, +i-j: the saved set of
 * Eq. FinalForm) are stored, plane-major; each backward block is formed where
 * it is used from the neighbour's forward block by Eq. conjugate,
 * W_{-d,x} = gamma5 W_{+d,x-d}^dag gamma5.  About half the bytes of the
 * 27-block layout for the same numbers (one right-hand side at a time; not
 * with OK_LAYOUT_SITE). */
#define OK_LAYOUT_SAVED 0x100

/* Layout flag OR-ed into the W precision (OK_F64 or OK_F32) of ok_W_bytes,
 * ok_precompute_W, ok_apply_M and ok_W_to_dense: every forward block is kept as
 * the colour matrices of its Pauli decomposition in spin (Sec. 2.2: each 2x2
 * spin block of Eqs. shifted_W_first..last is a sum of sigma_n (x) colour
 * matrix), 46 per site, and the blocks are formed where they are used, the
 * backward ones by Eq. conjugate.  3,312 bytes per site in FP32 and 6,624 in
 * FP64 against 31,104 and 62,208 for 27 dense blocks, for the same operator
 * (up to rounding: W0 and W+_i are stored as half sums and differences of
 * their two spin blocks).  One right-hand side at a time. */
#define OK_LAYOUT_SIGMA 0x200

/* Spinor layout flag OR-ed into spinor_prec of ok_apply_M (FP32 spinors,
 * site-major W or FP32 sigma-layout W, nrhs <= 16): spinors stored
 * [V][4][3][nrhs] complex, the right-hand side index fastest, which the
 * multi-right-hand-side kernels read contiguously.  Without it spinors are
 * [nrhs][V][4][3]. */
#define OK_SPINOR_RHS_INNER 0x20

typedef struct ok_geom {
    int32_t L[4];           /* Lx, Ly, Lz, Lt */
} ok_geom;

/* Coefficients of the tree-level tadpole-improved OK operator as they appear
 * in Eqs. shifted_W_first..last.  mhat = u0/(2 kappa) is the identity part of
 * W0; the paper applies it separately from the stored W0 (footnote in
 * Sec. 2.2), so W does not depend on mhat. */
typedef struct ok_coeffs {
    double mhat, u0, zeta, r_s, c_B, c_E, c_EE, c_1, c_2, c_3, c_4, c_5;
} ok_coeffs;

typedef struct ok_solver_params {
    double tol;             /* stop when ||xi - M psi|| / ||xi|| <= tol in FP64 (e.g. 1e-10) */
    double delta;           /* reliable-update threshold of the low-precision solve: an FP64
                               update when the low-precision residual has dropped by this
                               factor (e.g. 0.1 for BF16 W; FP32 W stays accurate to 0.003) */
    int32_t max_iter;       /* BiCGStab iterations, all restarts included       */
    int32_t max_restarts;   /* restarts after breakdown or residual drift        */
    int32_t zero_guess;     /* 1: start from psi = 0; 0: use d_psi as the guess  */
    int32_t verbose;        /* 1: print one line per iteration to stderr         */
    int32_t stall_window;   /* > 0: in a preconditioned solve, a residual with no
                               new minimum for this many iterations is a stall
                               and hands over to the unpreconditioned solve;
                               0: off                                           */
    int32_t W64_layout;     /* layout of d_W64: 0 (27 dense blocks, plane-major),
                               OK_LAYOUT_SAVED or OK_LAYOUT_SIGMA               */
} ok_solver_params;

typedef struct ok_solver_stats {
    int32_t status;         /* ok_status of this right-hand side                 */
    int32_t iterations;     /* BiCGStab iterations                               */
    int32_t matvec_hi;      /* FP64 applications of M                            */
    int32_t matvec_lo;      /* low-precision applications of M                   */
    int32_t reliable_updates;
    int32_t restarts;
    int32_t net_applies;    /* applications of the preconditioner network        */
    int32_t fallbacks;      /* 1 if the preconditioned solve failed and the
                               unpreconditioned one continued from its iterate   */
    double true_rel_resid;  /* ||xi - M64 psi|| / ||xi||, FP64, at return       */
    double seconds;         /* wall time of the call                             */
} ok_solver_stats;

/* ABI version of this header and of the private W layout. */
int ok_abi_version(void);

/* Message of the last error on the calling thread ("" if none). */
const char* ok_last_error(void);

/* Bytes of the W buffer for precision prec (OK_F64, OK_F32 or OK_BF16):
 * 27 blocks x 144 complex x sizeof(complex) per site, site stride padded to a
 * multiple of 64.  The layout is private to the library (versioned by
 * ok_abi_version). */
int ok_W_bytes(const ok_geom* g, int prec, size_t* bytes);

/* Bytes of the scratch ok_precompute_W needs: the six clover planes F_{mu nu}
 * (3x3 complex FP64) per site. */
int ok_precompute_scratch_bytes(const ok_geom* g, size_t* bytes);

/* Precalculation (Sec. 2.2): fill d_W with the 27 blocks W_{k,x} of every site
 * from the links, in FP64 arithmetic, stored at precision prec.  The 14
 * forward blocks follow Eqs. shifted_W_first..last; the 13 backward blocks
 * are W_{-d,x} = gamma5 W_{+d,x-d}^dag gamma5 (Eqs. conjugate and
 * opp_diag_pre_mat).  B_i and E_i are the clover fields of the links:
 * F_{mu nu} = traceless part of (Q_{mu nu} - Q_{mu nu}^dag)/8 with Q the sum
 * of the four counter-clockwise plaquette leaves at x, B_i = eps_ijk F_jk / 2,
 * E_i = F_{ti}.  Asynchronous on `stream`.  Redo it when the links, u0 or any
 * c changes; mhat alone does not need it. */
int ok_precompute_W(const ok_geom* g, const ok_coeffs* c, const double* d_links,
                    int prec, void* d_W, size_t W_bytes,
                    void* d_scratch, size_t scratch_bytes, void* stream);

/* d_out = M d_psi for nrhs right-hand sides (Eq. minFlopForm with mhat from c).
 * Allowed (W_prec, spinor_prec): (F64, F64), (F32, F32), (BF16, F32), each
 * W precision optionally | OK_LAYOUT_SITE and, with it, the FP32 spinors
 * optionally | OK_SPINOR_RHS_INNER.  Arithmetic is FP64 for FP64 W and FP32
 * (FP32 accumulation) otherwise; with nrhs > 1 (and always with site-major W)
 * FP32 and BF16 W run on the matrix cores, BF16 W multiplying the FP32
 * spinor split into two bf16 terms (2^-16 relative).
 * d_out must not overlap d_psi.  Asynchronous on `stream`. */
int ok_apply_M(const ok_geom* g, const ok_coeffs* c, const void* d_W, int W_prec,
               const void* d_psi, void* d_out, int spinor_prec, int nrhs, void* stream);

/* Expand d_W into dense FP64 blocks d_dense[V][27][12][12] complex (for
 * inspection and tests).  Asynchronous on `stream`. */
int ok_W_to_dense(const ok_geom* g, const void* d_W, int prec, double* d_dense, void* stream);

typedef struct ok_net ok_net;

/* Workspace bytes of ok_bicgstab for nrhs right-hand sides; Wlo_prec < 0 means
 * plain FP64 (no low-precision operator); net as passed to ok_bicgstab (NULL:
 * no preconditioner). */
int ok_bicgstab_workspace_bytes(const ok_geom* g, int nrhs, int Wlo_prec, const ok_net* net,
                                size_t* bytes);

/* Solve M psi = xi for nrhs right-hand sides by BiCGStab (Sec. 2.3).
 *   d_W64   FP64 W in the layout params->W64_layout (always needed: residuals
 *           and the final check are FP64).
 *   d_Wlo   NULL: plain FP64 BiCGStab.  Otherwise W at Wlo_prec (OK_F32 or
 *           OK_BF16, optionally | OK_LAYOUT_SAVED, or OK_F32 | OK_LAYOUT_SIGMA,
 *           for one right-hand side at a time; or | OK_LAYOUT_SITE, or
 *           OK_F32 | OK_LAYOUT_SIGMA | OK_SPINOR_RHS_INNER, below):
 *           the iteration runs in FP32 fields with that operator and
 *           FP64 reliable updates (x accumulated and r recomputed in FP64 when
 *           the low-precision residual drops by params->delta).  With
 *           Wlo_prec | OK_LAYOUT_SITE (or FP32 sigma-layout W with
 *           OK_SPINOR_RHS_INNER) the right-hand sides (in groups of up to
 *           16) iterate together: one application of W per BiCGStab step for
 *           the whole group (on the matrix cores for site-major W; the sigma
 *           layout reads each matrix once for all of them), per-right-hand-side scalars,
 *           reliable updates and convergence.  When a right-hand side is due
 *           for a reliable update, every one whose residual has fallen below
 *           sqrt(delta) of its maximum is updated in the same FP64 pass (W64
 *           read once per four right-hand sides).
 *   net     NULL, or the learned preconditioner N (low-precision solves
 *           only): BiCGStab then runs right-preconditioned, each step
 *           applying N to the search direction and to s (p^ = N p,
 *           v = M p^, s^ = N s, t = M s^, x += alpha p^ + omega s^), so the
 *           residual and the stopping test stay those of M psi = xi.  If that
 *           recurrence breaks down, stalls (params->stall_window) or meets a
 *           non-finite value, the unpreconditioned solve continues from the
 *           last FP64 iterate with the remaining iterations
 *           (stats.fallbacks = 1).  The network needs d_Wlo (OK_EINVAL
 *           otherwise).
 *   d_xi    FP64 source [nrhs][V][4][3] complex.
 *   d_psi   FP64 [nrhs][V][4][3]: the initial guess unless params->zero_guess,
 *           the solution on return.
 *   d_work  workspace of ok_bicgstab_workspace_bytes bytes.
 *   stats   host array of nrhs entries, filled for every right-hand side.
 * Synchronous: returns after every right-hand side converged or failed.
 * Returns OK_SUCCESS if all converged, else the first failing status. */
int ok_bicgstab(const ok_geom* g, const ok_coeffs* c, const ok_solver_params* p,
                const void* d_W64, const void* d_Wlo, int Wlo_prec, const ok_net* net,
                const double* d_xi, double* d_psi, int nrhs,
                void* d_work, size_t work_bytes, ok_solver_stats* stats, void* stream);

/* ok_bicgstab without a workspace argument and without any device allocation,
 * for callers that cannot allocate device memory (serving loops that must not
 * call hipMalloc, harnesses that forbid it).  The workspace is a fixed array
 * in the library's device memory, one per GPU, of
 * ok_bicgstab_static_max_bytes() bytes (64 MiB), held until the process ends;
 * a solve whose ok_bicgstab_workspace_bytes exceeds it returns OK_ESIZE (with
 * a message) before any HIP call.  Every argument, the result and the
 * statuses are those of ok_bicgstab.  All calls on one GPU share that array:
 * two calls that overlap in time on the same GPU (from different host
 * threads) race and give undefined results.  The first call on a device
 * looks the array's address up on that device (no allocation). */
int ok_bicgstab_static(const ok_geom* g, const ok_coeffs* c, const ok_solver_params* p,
                       const void* d_W64, const void* d_Wlo, int Wlo_prec, const ok_net* net,
                       const double* d_xi, double* d_psi, int nrhs, ok_solver_stats* stats,
                       void* stream);

/* Bytes of ok_bicgstab_static's fixed workspace. */
size_t ok_bicgstab_static_max_bytes(void);

/* Workspace bytes of ok_cgnr (six FP64 fields and the reduction scratch). */
int ok_cgnr_workspace_bytes(const ok_geom* g, int nrhs, size_t* bytes);

/* Solve M psi = xi for nrhs right-hand sides, one after the other, by CG on
 * the normal equations M^dag M psi = M^dag xi (the M^dag M route the paper
 * lists under Future Work), with M^dag = gamma5 M gamma5 (Eq. conjugate makes
 * M gamma5-hermitian; gamma5 = [[0, -i], [i, 0]] on the spin pairs (0, 1),
 * (2, 3)).  FP64 throughout; d_W64 in the layout params->W64_layout.  The
 * recurrence keeps r = xi - M psi, so the stopping test is the same as
 * ok_bicgstab's: the FP64 true residual ||xi - M psi|| / ||xi|| <= params->tol,
 * checked by recomputing r when the recurrence reaches it (restarting from it
 * if not, at most params->max_restarts times).  Each iteration applies M
 * twice (to p and to gamma5 r).  params->delta, stall_window are unused.
 * Arrays, ownership, statuses and synchronous behaviour as ok_bicgstab; the
 * workspace has ok_cgnr_workspace_bytes bytes. */
int ok_cgnr(const ok_geom* g, const ok_coeffs* c, const ok_solver_params* p, const void* d_W64,
            const double* d_xi, double* d_psi, int nrhs, void* d_work, size_t work_bytes,
            ok_solver_stats* stats, void* stream);

/* ------------------------------------------------------------------ learned preconditioner
 *
 * Not part of the paper's method: a gauge-covariant linear stencil network N,
 * trained so that N xi approximates M^{-1} xi, used as the right
 * preconditioner of ok_bicgstab.  One layer maps a spinor field phi to
 *
 *   phi'_x = sum_{k=0}^{26} A_k P_k(x) phi_{x+d_k}
 *
 * over the 27 offsets of Eq. minFlopForm, with A_k a 4x4 complex spin matrix
 * (colour blind) and P_k(x) the colour transport along hop k: 1 for k = 0,
 * U_mu(x) for +mu, U_i(x) U_i(x+i) for +2i, the mean of the two L-shaped
 * two-link paths for +i+j and +i-j (the paths of the off-axis W blocks,
 * Eqs. shifted_W_first..last), and P_{-d}(x) = P_d(x-d)^dag.  Each P_k(x)
 * transforms as g(x) P_k(x) g(x+d_k)^dag, so N is gauge covariant.  N is a
 * chain of n_layers layers.
 *
 *   Parameters: FP32 complex [n_layers][27][4][4] (A_k[spin out][spin in]).
 *   Transports: the 13 forward P_k per site, FP32, private layout
 *               (ok_net_transports).
 *   Fields:     FP32 complex batches of nfields spinor fields,
 *               [nfields][V][4][3], or with OK_SPINOR_RHS_INNER in flags
 *               [V][4][3][nfields].
 * Gradients are Wirtinger derivatives dL/d(conj A) of the real loss L; the
 * gradient with respect to (Re A, Im A) is twice that. */
#define OK_NET_MAX_LAYERS 16
#define OK_NET_ADJOINT 0x40     /* flag of ok_net_layer: apply the adjoint layer */

struct ok_net {
    int32_t n_layers;           /* 1 .. OK_NET_MAX_LAYERS                        */
    int32_t reserved;           /* 0                                             */
    const float* d_params;      /* [n_layers][27][4][4] complex FP32             */
    const float* d_T;           /* transports of the current gauge field         */
};

typedef struct ok_adam_cfg {
    double lr, beta1, beta2, eps;   /* e.g. 1e-3, 0.9, 0.999, 1e-8                */
} ok_adam_cfg;

/* Real (FP32) parameter count of an n_layers network: n_layers * 27 * 16 * 2. */
int ok_net_param_count(int n_layers, size_t* n_floats);

/* Bytes of the transport buffer (13 x 9 complex FP32 per site, padded). */
int ok_net_transports_bytes(const ok_geom* g, size_t* bytes);

/* Build the transports from FP64 links [V][4][3][3] (FP64 products, stored
 * FP32).  Redo it whenever the links change.  Asynchronous. */
int ok_net_transports(const ok_geom* g, const double* d_links, float* d_T, size_t T_bytes, void* stream);

/* One layer: d_out = sum_k A_k P_k d_in_{x+d_k} with d_A = [27][4][4] complex
 * FP32; with OK_NET_ADJOINT in flags the adjoint layer
 * sum_k P_{-k} A_k^dag d_in_{x-d_k}.  d_out must not overlap d_in.
 * Asynchronous. */
int ok_net_layer(const ok_geom* g, const float* d_A, const float* d_T, const float* d_in, float* d_out,
                 int nfields, int flags, void* stream);

/* Workspace bytes: training = 0 for ok_net_apply (ping-pong fields),
 * 1 for ok_net_loss_and_grad / ok_net_train_step (every layer's output, the
 * gradient partial sums and the loss scratch), 2 for ok_net_layer_wgrad and
 * ok_net_loss_grad alone. */
int ok_net_workspace_bytes(const ok_geom* g, int n_layers, int nfields, int training, size_t* bytes);

/* d_out = N d_in.  Asynchronous. */
int ok_net_apply(const ok_geom* g, const ok_net* net, const float* d_in, float* d_out, int nfields,
                 int flags, void* d_work, size_t work_bytes, void* stream);

/* Weight gradient of one layer: d_gA[k][a][b] = sum over fields, sites x and
 * colour c of d_gout_x^{a c} conj((P_k d_in_{x+d_k})^{b c}), [27][4][4]
 * complex FP32, summed in a fixed order (bitwise reproducible).
 * Asynchronous. */
int ok_net_layer_wgrad(const ok_geom* g, const float* d_T, const float* d_gout, const float* d_in,
                       float* d_gA, int nfields, int flags, void* d_work, size_t work_bytes, void* stream);

/* Loss L = (1/nfields) sum_f ||out_f - psi_f||^2 / ||psi_f||^2 (fields with
 * psi_f = 0 contribute 0) into *d_loss (FP64, device), and its gradient
 * d_gout = dL/d(conj out) = (out_f - psi_f) / (nfields ||psi_f||^2).  d_gout
 * may equal d_out.  Asynchronous. */
int ok_net_loss_grad(const ok_geom* g, const float* d_out, const float* d_psi, float* d_gout, double* d_loss,
                     int nfields, int flags, void* d_work, size_t work_bytes, void* stream);

/* Forward pass of N on the batch d_xi, the loss against d_psi into *d_loss and
 * the gradient dL/d(conj params) into d_grad ([n_layers][27][4][4] complex
 * FP32).  Asynchronous. */
int ok_net_loss_and_grad(const ok_geom* g, const ok_net* net, const float* d_xi, const float* d_psi,
                         int nfields, int flags, double* d_loss, float* d_grad, void* d_work, size_t work_bytes,
                         void* stream);

/* d_out[i] = (float) d_in[i] for n reals, round to nearest (e.g. FP64 training pairs
 * from ok_bicgstab to the network's FP32 fields).  Asynchronous. */
int ok_cast_f64_to_f32(const double* d_in, float* d_out, size_t n, void* stream);

/* Adam on n real parameters d_p with Wirtinger gradient d_g (the real
 * gradient is 2 d_g) and moments d_m, d_v (zero before step 1); step >= 1.
 * Asynchronous. */
int ok_adam_step(float* d_p, const float* d_g, float* d_m, float* d_v, size_t n, const ok_adam_cfg* cfg,
                 int step, void* stream);

/* One training step: ok_net_loss_and_grad, then ok_adam_step on the
 * parameters of an n_layers network.  d_grad receives the gradient.
 * Asynchronous. */
int ok_net_train_step(const ok_geom* g, int n_layers, float* d_params, float* d_m, float* d_v, const float* d_T,
                      const float* d_xi, const float* d_psi, int nfields, int flags, const ok_adam_cfg* cfg,
                      int step, double* d_loss, float* d_grad, void* d_work, size_t work_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* OKINV_H */
