// The 27-point operator (Eq. minFlopForm) with W kept as the colour matrices of its Pauli
// decomposition in spin (OK_LAYOUT_SIGMA, 46 matrices per site; wlayout.h lists them).
//
// Every spin block of Eqs. shifted_W_first..last is a sum over sigma_n (x) colour matrix, and
// the forward blocks come in four shapes:
//   [[A, B], [B, A]]   (W+_i, W++_ii):  out_u +- out_d = (A +- B)(psi_u +- psi_d)
//   [[A, B], [-B, A]]  (W0):            out_u +- i out_d = (A -+ i B)(psi_u +- i psi_d)
//   [[0, H], [H, N]]   (W+_4)
//   [[0, H], [H, 0]]   (W++_ij, W+-_ij, H = (sigma_i +- sigma_j) (x) T)
// (u, d: the upper and lower spin pairs).  A backward block W_{-d,x} = gamma5 W_{+d,x-d}^dag
// gamma5 (Eq. conjugate) is [[D^dag, -B^dag], [-C^dag, A^dag]] of the forward block
// [[A, B], [C, D]] at x - d; since the sigma_n are hermitian that only takes colour
// daggers: the [[A, B], [B, A]] shape maps to itself with (A + B, A - B) -> ((A - B)^dag,
// (A + B)^dag), the off-diagonal one to -H^dag, and [[0, H], [H, N]] to [[N^dag, -H^dag],
// [-H^dag, 0]].
//
// One thread per site, or several per site (right-hand-side-inner FP32 fields, two right-hand
// sides per thread when their number is even; or up to four separate FP64 fields, one per
// thread), the lanes of a site then sharing every matrix load.  Per site and right-hand side: 46 matrices
// (3,312 B FP32, 6,624 B FP64) read at the site and again as the backward blocks of its
// neighbours, one spinor out, and 27 neighbour spinors (L2 hits mostly); 232 colour
// matrix-vector products (2,088 complex multiply-adds, against 3,888 for 27 dense blocks).
#include <algorithm>

#include "common.h"
#include "kernels.h"
#include "wlayout.h"

namespace okinv {
namespace {

template <int P> struct SArith { using T = float; };
template <> struct SArith<OK_F64> { using T = double; };

// colour matrix mi of site s (row-major 3x3)
template <int P, typename T>
__device__ __forceinline__ void ld_mat(const void* __restrict__ W, int Vs, int mi, int s, cpx<T> M[9]) {
    const char* base = reinterpret_cast<const char*>(W);
    if constexpr (P == OK_F64) {
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            const double2 d = *reinterpret_cast<const double2*>(base + sigma_off<P>(Vs, mi, e, s));
            M[e] = cpx<T>{d.x, d.y};
        }
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float4 f = *reinterpret_cast<const float4*>(base + sigma_off<P>(Vs, mi, 2 * j, s));
            M[2 * j] = cpx<T>{f.x, f.y};
            M[2 * j + 1] = cpx<T>{f.z, f.w};
        }
        const float2 f = *reinterpret_cast<const float2*>(base + sigma_off<P>(Vs, mi, 8, s));
        M[8] = cpx<T>{f.x, f.y};
    }
}

// y[k] = M x[k] (DAG: y = M^dag x) for the two spins of a pair and the R right-hand sides of a
// lane (one matrix load serves all R)
template <int R, bool DAG, typename T>
__device__ __forceinline__ void mv2(const cpx<T> M[9], const cpx<T> x[R][2][3], cpx<T> y[R][2][3]) {
#pragma unroll
    for (int k = 0; k < R; ++k)
#pragma unroll
        for (int sp = 0; sp < 2; ++sp)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                cpx<T> acc{0, 0};
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    if constexpr (DAG) cfma_conj(acc, M[3 * b + a], x[k][sp][b]);
                    else cfma(acc, M[3 * a + b], x[k][sp][b]);
                }
                y[k][sp][a] = acc;
            }
}

// o += c * sigma_n y on a spin pair (n = 0..3, uniform across the wavefront), c = +1 or -1
template <typename T>
__device__ __forceinline__ void sig_acc1(int n, T c, const cpx<T> y[2][3], cpx<T> o[2][3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const cpx<T> y0 = c * y[0][a], y1 = c * y[1][a];
        switch (n) {
            case 0: o[0][a] = o[0][a] + y0; o[1][a] = o[1][a] + y1; break;
            case 1: o[0][a] = o[0][a] + y1; o[1][a] = o[1][a] + y0; break;
            case 2:   // sigma_2 = [[0, -i], [i, 0]]
                o[0][a] = o[0][a] + cpx<T>{y1.im, -y1.re};
                o[1][a] = o[1][a] + cpx<T>{-y0.im, y0.re};
                break;
            default: o[0][a] = o[0][a] + y0; o[1][a] = o[1][a] - y1; break;
        }
    }
}

template <int R, typename T>
__device__ __forceinline__ void sig_acc(int n, T c, const cpx<T> y[R][2][3], cpx<T> o[R][2][3]) {
#pragma unroll
    for (int k = 0; k < R; ++k) sig_acc1(n, c, y[k], o[k]);
}

template <int R, typename T>
__device__ __forceinline__ void zero2(cpx<T> o[R][2][3]) {
#pragma unroll
    for (int k = 0; k < R; ++k)
#pragma unroll
        for (int sp = 0; sp < 2; ++sp)
#pragma unroll
            for (int a = 0; a < 3; ++a) o[k][sp][a] = cpx<T>{0, 0};
}

// o += sum_{n in [n0, n0 + cnt)} sigma_n (M_{mi0 + n - n0}^(dag) x)
template <int P, int R, bool DAG, typename T>
__device__ __forceinline__ void pauli_sum(const void* __restrict__ W, int Vs, int s, int mi0, int n0, int cnt, T c,
                                          const cpx<T> x[R][2][3], cpx<T> o[R][2][3]) {
    // unrolled (cnt is a constant where this is inlined), so the next matrix's loads overlap
    // the current mat-vec: 4-8 % faster than a rolled loop
#pragma unroll
    for (int q = 0; q < cnt; ++q) {
        cpx<T> M[9], y[R][2][3];
        ld_mat<P, T>(W, Vs, mi0 + q, s, M);
        mv2<R, DAG, T>(M, x, y);
        sig_acc<R>(n0 + q, c, y, o);
    }
}

// acc[k][spin pair][spin][colour] += [[A, B], [B, A]] (u, d) with A + B = 2 sum_n sigma_n P_n,
// A - B = 2 sum_n sigma_n Q_n, P_n / Q_n at mi (P), mi + 4 (Q); the backward block swaps and
// daggers them.  Half h = 0: y = (A + B)(u + d) / 2 goes to both pairs; h = 1: y = (A - B)(u - d) / 2
// to the upper pair and, negated, to the lower one.
template <int P, int R, bool BWD, typename T>
__device__ __forceinline__ void hop_ds(const void* __restrict__ W, int Vs, int s, int mi, const cpx<T> v[R][12],
                                       cpx<T> acc[R][2][2][3]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        cpx<T> x[R][2][3], y[R][2][3];
#pragma unroll
        for (int k = 0; k < R; ++k)
#pragma unroll
            for (int sp = 0; sp < 2; ++sp)
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    x[k][sp][a] = h == 0 ? v[k][3 * sp + a] + v[k][6 + 3 * sp + a]
                                         : v[k][3 * sp + a] - v[k][6 + 3 * sp + a];
        zero2<R>(y);
        pauli_sum<P, R, BWD, T>(W, Vs, s, (h == 0) == BWD ? mi + 4 : mi, 0, 4, T(1), x, y);
#pragma unroll
        for (int k = 0; k < R; ++k)
#pragma unroll
            for (int sp = 0; sp < 2; ++sp)
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    acc[k][0][sp][a] = acc[k][0][sp][a] + y[k][sp][a];
                    acc[k][1][sp][a] = h == 0 ? acc[k][1][sp][a] + y[k][sp][a] : acc[k][1][sp][a] - y[k][sp][a];
                }
    }
}

// the upper (u) and lower (d) spin pairs of each right-hand side of a lane
template <int R, typename T>
__device__ __forceinline__ void pairs(const cpx<T> v[R][12], cpx<T> u[R][2][3], cpx<T> d[R][2][3]) {
#pragma unroll
    for (int k = 0; k < R; ++k)
#pragma unroll
        for (int sp = 0; sp < 2; ++sp)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                u[k][sp][a] = v[k][3 * sp + a];
                d[k][sp][a] = v[k][6 + 3 * sp + a];
            }
}

// per right-hand side k: o[k][h] += c sigma_n y[k] (h = 0: upper pair, 1: lower)
template <int R, typename T>
__device__ __forceinline__ void sig_acc_h(int n, T c, int h, const cpx<T> y[R][2][3], cpx<T> acc[R][2][2][3]) {
#pragma unroll
    for (int k = 0; k < R; ++k) sig_acc1(n, c, y[k], acc[k][h]);
}

// W++_ii: A = 1 (x) G0, B = sigma_i (x) G1 (G0 at mi, G1 at mi + 1); backward: G0^dag, -G1^dag
template <int P, int R, bool BWD, typename T>
__device__ __forceinline__ void hop_ii(const void* __restrict__ W, int Vs, int s, int mi, int i,
                                       const cpx<T> v[R][12], cpx<T> acc[R][2][2][3]) {
    cpx<T> u[R][2][3], d[R][2][3];
    pairs<R>(v, u, d);
    const T c1 = BWD ? T(-1) : T(1);
    cpx<T> M[9], y[R][2][3];
    ld_mat<P, T>(W, Vs, mi, s, M);
    mv2<R, BWD, T>(M, u, y);
    sig_acc_h<R>(0, T(1), 0, y, acc);
    mv2<R, BWD, T>(M, d, y);
    sig_acc_h<R>(0, T(1), 1, y, acc);
    ld_mat<P, T>(W, Vs, mi + 1, s, M);
    mv2<R, BWD, T>(M, d, y);
    sig_acc_h<R>(1 + i, c1, 0, y, acc);
    mv2<R, BWD, T>(M, u, y);
    sig_acc_h<R>(1 + i, c1, 1, y, acc);
}

// [[0, H], [H, 0]] with H = (sigma_{1+i} + sg sigma_{1+j}) (x) T (T at mi); backward: -H^dag
template <int P, int R, bool BWD, typename T>
__device__ __forceinline__ void hop_off(const void* __restrict__ W, int Vs, int s, int mi, int i, int j, T sg,
                                        const cpx<T> v[R][12], cpx<T> acc[R][2][2][3]) {
    cpx<T> u[R][2][3], d[R][2][3];
    pairs<R>(v, u, d);
    const T c = BWD ? T(-1) : T(1);
    cpx<T> M[9], y[R][2][3];
    ld_mat<P, T>(W, Vs, mi, s, M);
    mv2<R, BWD, T>(M, d, y);
    sig_acc_h<R>(1 + i, c, 0, y, acc);
    sig_acc_h<R>(1 + j, c * sg, 0, y, acc);
    mv2<R, BWD, T>(M, u, y);
    sig_acc_h<R>(1 + i, c, 1, y, acc);
    sig_acc_h<R>(1 + j, c * sg, 1, y, acc);
}

// W+_4 = [[0, H], [H, N]], H = sum_{m=1..3} sigma_m S_m (mi .. mi + 2), N at mi + 3;
// backward: [[N^dag, -H^dag], [-H^dag, 0]]
template <int P, int R, bool BWD, typename T>
__device__ __forceinline__ void hop_t(const void* __restrict__ W, int Vs, int s, int mi, const cpx<T> v[R][12],
                                      cpx<T> acc[R][2][2][3]) {
    cpx<T> u[R][2][3], d[R][2][3], o0[R][2][3], o1[R][2][3];
    pairs<R>(v, u, d);
#pragma unroll
    for (int k = 0; k < R; ++k)
#pragma unroll
        for (int sp = 0; sp < 2; ++sp)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                o0[k][sp][a] = acc[k][0][sp][a];
                o1[k][sp][a] = acc[k][1][sp][a];
            }
    const T c = BWD ? T(-1) : T(1);
    pauli_sum<P, R, BWD, T>(W, Vs, s, mi, 1, 3, c, d, o0);
    pauli_sum<P, R, BWD, T>(W, Vs, s, mi, 1, 3, c, u, o1);
    cpx<T> M[9], y[R][2][3];
    ld_mat<P, T>(W, Vs, mi + 3, s, M);
    if constexpr (BWD) {
        mv2<R, true, T>(M, u, y);
        sig_acc<R>(0, T(1), y, o0);
    } else {
        mv2<R, false, T>(M, d, y);
        sig_acc<R>(0, T(1), y, o1);
    }
#pragma unroll
    for (int k = 0; k < R; ++k)
#pragma unroll
        for (int sp = 0; sp < 2; ++sp)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                acc[k][0][sp][a] = o0[k][sp][a];
                acc[k][1][sp][a] = o1[k][sp][a];
            }
}

// W0 = [[A, B], [-B, A]]: out_u + i out_d = (A - iB)(u + i d), out_u - i out_d = (A + iB)(u - i d),
// (A -+ iB) = 2 sum_m sigma_m R-+_m with R-_m at mi + m - 1 and R+_m at mi + 2 + m.  Half h = 0:
// y = (A - iB)(u + i d) / 2 adds y to the upper pair and -i y to the lower; h = 1: y = (A + iB)(u - i d) / 2
// adds y and +i y.
template <int P, int R, typename T>
__device__ __forceinline__ void hop_w0(const void* __restrict__ W, int Vs, int s, int mi, const cpx<T> v[R][12],
                                       cpx<T> acc[R][2][2][3]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        cpx<T> x[R][2][3], y[R][2][3];
#pragma unroll
        for (int k = 0; k < R; ++k)
#pragma unroll
            for (int sp = 0; sp < 2; ++sp)
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const cpx<T> u = v[k][3 * sp + a], d = v[k][6 + 3 * sp + a];
                    const cpx<T> id{-d.im, d.re};
                    x[k][sp][a] = h == 0 ? u + id : u - id;
                }
        zero2<R>(y);
        pauli_sum<P, R, false, T>(W, Vs, s, mi + 3 * h, 1, 3, T(1), x, y);
#pragma unroll
        for (int k = 0; k < R; ++k)
#pragma unroll
            for (int sp = 0; sp < 2; ++sp)
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const cpx<T> w = y[k][sp][a];
                    acc[k][0][sp][a] = acc[k][0][sp][a] + w;
                    acc[k][1][sp][a] = acc[k][1][sp][a] + (h == 0 ? cpx<T>{w.im, -w.re} : cpx<T>{-w.im, w.re});
                }
    }
}

// spinor component q of site s: [V][12] (nr = 0), or right-hand sides r .. r + R - 1 of
// [V][12][nr] (nr > 0; with R = 2 and FP32 one 16-byte load per component)
template <int R, typename T>
__device__ __forceinline__ void ld_sp(const T* __restrict__ psi, int s, cpx<T> v[R][12], int nr = 0, int r = 0) {
    const cpx<T>* p = reinterpret_cast<const cpx<T>*>(psi);
#pragma unroll
    for (int q = 0; q < 12; ++q) {
        if constexpr (R == 2 && sizeof(T) == 4) {
            const float4 f = *reinterpret_cast<const float4*>(p + ((size_t)s * 12 + q) * nr + r);
            v[0][q] = cpx<T>{f.x, f.y};
            v[1][q] = cpx<T>{f.z, f.w};
        } else {
#pragma unroll
            for (int k = 0; k < R; ++k)
                v[k][q] = nr ? p[((size_t)s * 12 + q) * nr + r + k] : p[(size_t)s * 12 + q];
        }
    }
}

// Per right-hand side of a block of the MR == 1 kernel: the lanes holding right-hand side r (lane
// group g of slot k of wavefront w is lane 64 w + k (nr / R) + g, holding right-hand sides
// R g .. R g + R - 1) summed in a fixed order, stored as partial[block][r][2] (the layout of the
// batched solver's reductions).
template <int R>
__device__ __forceinline__ void rhs_reduce_store(const double2 d1[R], const double2 d2[R], double2* partial, int nr) {
    __shared__ double2 red[R][2][256];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        red[k][0][threadIdx.x] = d1[k];
        red[k][1][threadIdx.x] = d2[k];
    }
    __syncthreads();
    if ((int)threadIdx.x < nr) {
        const int r = threadIdx.x, L = nr / R, spw = 64 / L, g = r / R, k = r % R;
        double2 a{0.0, 0.0}, b{0.0, 0.0};
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w)
            for (int sl = 0; sl < spw; ++sl) {
                const int l = w * 64 + sl * L + g;
                a.x += red[k][0][l].x;
                a.y += red[k][0][l].y;
                b.x += red[k][1][l].x;
                b.y += red[k][1][l].y;
            }
        double2* p = partial + ((size_t)blockIdx.x * kMaxRhsB + r) * 2;
        p[0] = a;
        p[1] = b;
    }
}

// Up to four separate [V][12] fields (MR == 2).
template <typename T>
struct SCols {
    const T* in[4];
    T* out[4];
};

// MR = 0: one thread per site, spinors [V][12].  MR = 1: nr (<= 16) right-hand sides with the
// right-hand side fastest ([V][12][nr]), R of them per lane (R = 2 needs an even nr); MR = 2:
// nr (<= 4) separate [V][12] fields in cols.  With MR > 0 the lanes of a wavefront are split into
// site slots of nr / R lanes (MR = 1) or nr lanes (MR = 2), so the lanes of a site issue the same
// matrix addresses and each W byte is fetched once for all right-hand sides; with R = 2 every
// matrix a lane loads serves two right-hand sides.
// WPE: waves per SIMD the register allocation aims at (1: no constraint)
template <int P, int EPI, int MR, int WPE = 1, int R = 1>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) k_apply_sigma(Geo g, const void* __restrict__ W,
                                                     const typename SArith<P>::T* __restrict__ psi,
                                                     typename SArith<P>::T* __restrict__ out, double mhat_d,
                                                     const typename SArith<P>::T* __restrict__ aux,
                                                     double2* __restrict__ partial, int nr,
                                                     SCols<typename SArith<P>::T> cols) {
    using T = typename SArith<P>::T;
    static_assert(R == 1 || MR == 1, "two right-hand sides per lane only with right-hand-side-inner fields");
    // each XCD takes a contiguous range of sites, so that the matrices a site's neighbours
    // read again as their backward blocks are still in that XCD's L2
    int s, r = 0;
    bool live;
    if constexpr (MR) {
        const int L = MR == 1 ? nr / R : nr;   // lanes per site slot
        const int lane = threadIdx.x & 63, spw = 64 / L, slot = lane / L;
        r = (lane - slot * L) * (MR == 1 ? R : 1);
        s = (xcd_tile(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + (threadIdx.x >> 6)) * spw + slot;
        live = slot < spw && s < g.V;
        if constexpr (MR == 2) {   // this lane's field, addressed as one [V][12] spinor
            psi = r == 0 ? cols.in[0] : r == 1 ? cols.in[1] : r == 2 ? cols.in[2] : cols.in[3];
            out = r == 0 ? cols.out[0] : r == 1 ? cols.out[1] : r == 2 ? cols.out[2] : cols.out[3];
            nr = 0;
            r = 0;
        }
    } else {
        nr = 0;
        s = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
        live = s < g.V;
    }
    double2 d1[R], d2[R];
#pragma unroll
    for (int k = 0; k < R; ++k) d1[k] = d2[k] = double2{0.0, 0.0};
    if (live) {
        const int Vs = g.Vs;
        int x, y, z, t;
        site_coords(g, s, x, y, z, t);
        cpx<T> acc[R][2][2][3], v[R][12];
        ld_sp<R>(psi, s, v, nr, r);
#pragma unroll
        for (int k = 0; k < R; ++k)
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int sp = 0; sp < 2; ++sp)
#pragma unroll
                    for (int a = 0; a < 3; ++a) acc[k][h][sp][a] = T(mhat_d) * v[k][6 * h + 3 * sp + a];
        hop_w0<P, R, T>(W, Vs, s, SG_W0, v, acc);
#pragma unroll 1
        for (int i = 0; i < 3; ++i) {   // +-i: W+_i at x, Gamma(W+_i) at x - i
            int n = neighbour(g, x, y, z, t, off_d(1 + i, 0), off_d(1 + i, 1), off_d(1 + i, 2), 0);
            ld_sp<R>(psi, n, v, nr, r);
            hop_ds<P, R, false, T>(W, Vs, s, SG_WI + 8 * i, v, acc);
            n = neighbour(g, x, y, z, t, -off_d(1 + i, 0), -off_d(1 + i, 1), -off_d(1 + i, 2), 0);
            ld_sp<R>(psi, n, v, nr, r);
            hop_ds<P, R, true, T>(W, Vs, n, SG_WI + 8 * i, v, acc);
        }
        {   // +-t
            int n = neighbour(g, x, y, z, t, 0, 0, 0, 1);
            ld_sp<R>(psi, n, v, nr, r);
            hop_t<P, R, false, T>(W, Vs, s, SG_W4, v, acc);
            n = neighbour(g, x, y, z, t, 0, 0, 0, -1);
            ld_sp<R>(psi, n, v, nr, r);
            hop_t<P, R, true, T>(W, Vs, n, SG_W4, v, acc);
        }
#pragma unroll 1
        for (int i = 0; i < 3; ++i) {   // +-2i
            int n = neighbour(g, x, y, z, t, off_d(9 + i, 0), off_d(9 + i, 1), off_d(9 + i, 2), 0);
            ld_sp<R>(psi, n, v, nr, r);
            hop_ii<P, R, false, T>(W, Vs, s, SG_WII + 2 * i, i, v, acc);
            n = neighbour(g, x, y, z, t, -off_d(9 + i, 0), -off_d(9 + i, 1), -off_d(9 + i, 2), 0);
            ld_sp<R>(psi, n, v, nr, r);
            hop_ii<P, R, true, T>(W, Vs, n, SG_WII + 2 * i, i, v, acc);
        }
#pragma unroll 1
        for (int p = 0; p < 3; ++p) {   // +-(i+j) and +-(i-j)
            const int i = p < 2 ? 0 : 1, j = p == 0 ? 1 : 2;
            const int k1 = 15 + p, k2 = 21 + p;
            int n = neighbour(g, x, y, z, t, off_d(k1, 0), off_d(k1, 1), off_d(k1, 2), 0);
            ld_sp<R>(psi, n, v, nr, r);
            hop_off<P, R, false, T>(W, Vs, s, SG_WIJ + p, i, j, T(1), v, acc);
            n = neighbour(g, x, y, z, t, -off_d(k1, 0), -off_d(k1, 1), -off_d(k1, 2), 0);
            ld_sp<R>(psi, n, v, nr, r);
            hop_off<P, R, true, T>(W, Vs, n, SG_WIJ + p, i, j, T(1), v, acc);
            n = neighbour(g, x, y, z, t, off_d(k2, 0), off_d(k2, 1), off_d(k2, 2), 0);
            ld_sp<R>(psi, n, v, nr, r);
            hop_off<P, R, false, T>(W, Vs, s, SG_WIMJ + p, i, j, T(-1), v, acc);
            n = neighbour(g, x, y, z, t, -off_d(k2, 0), -off_d(k2, 1), -off_d(k2, 2), 0);
            ld_sp<R>(psi, n, v, nr, r);
            hop_off<P, R, true, T>(W, Vs, n, SG_WIMJ + p, i, j, T(-1), v, acc);
        }
        cpx<T>* o = reinterpret_cast<cpx<T>*>(out);
#pragma unroll
        for (int q = 0; q < 12; ++q) {
            if constexpr (R == 2 && sizeof(T) == 4) {
                const cpx<T> w0 = acc[0][q / 6][(q / 3) & 1][q % 3], w1 = acc[1][q / 6][(q / 3) & 1][q % 3];
                *reinterpret_cast<float4*>(o + ((size_t)s * 12 + q) * nr + r) = make_float4(w0.re, w0.im, w1.re, w1.im);
            } else {
#pragma unroll
                for (int k = 0; k < R; ++k)
                    o[MR == 1 ? ((size_t)s * 12 + q) * nr + r + k : (size_t)s * 12 + q] = acc[k][q / 6][(q / 3) & 1][q % 3];
            }
        }
        // epilogue dots; with MR == 1 over this lane's right-hand sides.  The second vector of
        // <t, s> is aux when given (the solver's s, which is not the operator's input when it is
        // preconditioned), else the input
        const cpx<T>* ax = reinterpret_cast<const cpx<T>*>(aux);
        const cpx<T>* ps = reinterpret_cast<const cpx<T>*>(psi);
        auto at = [&](const cpx<T>* f, int q, int k) __attribute__((always_inline)) {
            return MR == 1 ? f[((size_t)s * 12 + q) * nr + r + k] : f[(size_t)s * 12 + q];
        };
#pragma unroll
        for (int k = 0; k < R; ++k) {
            if constexpr (EPI == EPI_RV) {
#pragma unroll
                for (int q = 0; q < 12; ++q) {
                    const cpx<T> av = at(ax, q, k), w = acc[k][q / 6][(q / 3) & 1][q % 3];
                    d1[k].x += (double)av.re * w.re + (double)av.im * w.im;
                    d1[k].y += (double)av.re * w.im - (double)av.im * w.re;
                }
            } else if constexpr (EPI == EPI_TS) {
#pragma unroll
                for (int q = 0; q < 12; ++q) {
                    const cpx<T> sv = at(ax ? ax : ps, q, k), w = acc[k][q / 6][(q / 3) & 1][q % 3];
                    d1[k].x += (double)w.re * sv.re + (double)w.im * sv.im;
                    d1[k].y += (double)w.re * sv.im - (double)w.im * sv.re;
                    d2[k].x += (double)w.re * w.re + (double)w.im * w.im;
                }
            }
        }
    }
    if constexpr (EPI != EPI_NONE) {
        if constexpr (MR == 1) rhs_reduce_store<R>(d1, d2, partial, nr);
        else block_reduce2_store(d1[0], d2[0], partial);
    }
}

template <int P>
int launch_sigma_t(const Geo& g, const void* W, const void* psi, void* out, double mhat, int epi, const void* aux,
                   double2* partial, hipStream_t st) {
    using T = typename SArith<P>::T;
    const unsigned nb = grid_for(g.V, 256);
    const T* in = reinterpret_cast<const T*>(psi);
    T* o = reinterpret_cast<T*>(out);
    const T* ax = reinterpret_cast<const T*>(aux);
    const SCols<T> nc{};
    if (epi == EPI_NONE) k_apply_sigma<P, EPI_NONE, 0><<<nb, 256, 0, st>>>(g, W, in, o, mhat, ax, partial, 0, nc);
    else if (epi == EPI_RV) k_apply_sigma<P, EPI_RV, 0><<<nb, 256, 0, st>>>(g, W, in, o, mhat, ax, partial, 0, nc);
    else k_apply_sigma<P, EPI_TS, 0><<<nb, 256, 0, st>>>(g, W, in, o, mhat, ax, partial, 0, nc);
    OK_LAUNCH_CHECK("k_apply_sigma");
    return OK_SUCCESS;
}

}  // namespace

// right-hand sides per lane of the right-hand-side-inner kernel: two when nrhs is even
static int sigma_mr_rpl(int nrhs) { return nrhs % 2 == 0 ? 2 : 1; }

int sigma_mr_blocks(const Geo& g, int nrhs) {
    const int spw = 64 / (nrhs / sigma_mr_rpl(nrhs));
    const long waves = ((long)g.V + spw - 1) / spw;
    return (int)((waves + 3) / 4);
}

int launch_apply_sigma_mr(const Geo& g, const void* W, const float* psi, float* out, double mhat, int nrhs,
                          hipStream_t st, int epi, const float* aux, double2* partial) {
    if (nrhs < 1 || nrhs > 16) {
        set_error("right-hand-side-inner spinors support 1 to 16 right-hand sides");
        return OK_EINVAL;
    }
    const unsigned nb = (unsigned)sigma_mr_blocks(g, nrhs);
    const SCols<float> nc{};
    if (sigma_mr_rpl(nrhs) == 2) {
        if (epi == EPI_RV)
            k_apply_sigma<OK_F32, EPI_RV, 1, 1, 2><<<nb, 256, 0, st>>>(g, W, psi, out, mhat, aux, partial, nrhs, nc);
        else if (epi == EPI_TS)
            k_apply_sigma<OK_F32, EPI_TS, 1, 1, 2><<<nb, 256, 0, st>>>(g, W, psi, out, mhat, aux, partial, nrhs, nc);
        else
            k_apply_sigma<OK_F32, EPI_NONE, 1, 1, 2><<<nb, 256, 0, st>>>(g, W, psi, out, mhat, nullptr, nullptr,
                                                                         nrhs, nc);
    } else {
        if (epi == EPI_RV)
            k_apply_sigma<OK_F32, EPI_RV, 1><<<nb, 256, 0, st>>>(g, W, psi, out, mhat, aux, partial, nrhs, nc);
        else if (epi == EPI_TS)
            k_apply_sigma<OK_F32, EPI_TS, 1><<<nb, 256, 0, st>>>(g, W, psi, out, mhat, aux, partial, nrhs, nc);
        else
            k_apply_sigma<OK_F32, EPI_NONE, 1><<<nb, 256, 0, st>>>(g, W, psi, out, mhat, nullptr, nullptr, nrhs, nc);
    }
    OK_LAUNCH_CHECK("k_apply_sigma");
    return OK_SUCCESS;
}

int launch_apply_sigma_cols(const Geo& g, const void* W, const double* const* in, double* const* out, int n,
                            double mhat, hipStream_t st) {
    for (int c0 = 0; c0 < n; c0 += 4) {
        const int m = std::min(4, n - c0);
        SCols<double> cols{};
        for (int c = 0; c < m; ++c) {
            cols.in[c] = in[c0 + c];
            cols.out[c] = out[c0 + c];
        }
        const int spw = 64 / m;
        const long waves = ((long)g.V + spw - 1) / spw;
        const unsigned nb = (unsigned)((waves + 3) / 4);
        // two waves per SIMD (a few registers spill to scratch) measured 17 % faster here than one
        // wave without spills; the one-field kernels are faster with the default
        k_apply_sigma<OK_F64, EPI_NONE, 2, 2><<<nb, 256, 0, st>>>(g, W, nullptr, nullptr, mhat, nullptr, nullptr, m,
                                                                  cols);
        OK_LAUNCH_CHECK("k_apply_sigma");
    }
    return OK_SUCCESS;
}

int launch_apply_sigma(const Geo& g, const void* W, int Wprec, const void* psi, void* out, double mhat, int epi,
                       const void* aux, double2* partial, hipStream_t st) {
    if ((Wprec & 3) == OK_F64) return launch_sigma_t<OK_F64>(g, W, psi, out, mhat, epi, aux, partial, st);
    return launch_sigma_t<OK_F32>(g, W, psi, out, mhat, epi, aux, partial, st);
}

}  // namespace okinv
