// Precalculation of the 27 W blocks per site (Sec. 2.2, Eqs. shifted_W_first..last).
//
// Three kernels, all FP64 arithmetic:
//   k_clover    F_{mu nu}(x) for the six planes (clover of the links), into scratch;
//   k_forward   the 14 forward blocks from the printed formulas, one thread per
//               (site, block, colour row a): every 2x2 spin block of W is
//               accumulated in its Pauli decomposition sum_n sigma_n (x) X_n
//               (row a of each X_n), then expanded to the four dense rows
//               (alpha, a), alpha = 0..3, and stored at the storage precision;
//   k_backward  the 13 backward blocks W_{-d,x} = gamma5 W_{+d,x-d}^dag gamma5
//               (Eqs. conjugate, opp_diag_pre_mat), an exact transpose/conjugate/
//               sign gather of the stored forward block of site x - d.
#include "common.h"
#include "wlayout.h"

namespace okinv {
namespace {

struct m3 {
    c128 e[3][3];
};

__device__ __forceinline__ m3 ld_link(const double* links, int s, int mu) {
    const double2* p = reinterpret_cast<const double2*>(links) + ((size_t)s * 4 + mu) * 9;
    m3 m;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            double2 d = p[a * 3 + b];
            m.e[a][b] = c128{d.x, d.y};
        }
    return m;
}

__device__ __forceinline__ m3 dagm(const m3& A) {
    m3 m;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) m.e[a][b] = conj(A.e[b][a]);
    return m;
}

__device__ __forceinline__ m3 mul(const m3& A, const m3& B) {
    m3 m;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            c128 acc{0.0, 0.0};
#pragma unroll
            for (int c = 0; c < 3; ++c) cfma(acc, A.e[a][c], B.e[c][b]);
            m.e[a][b] = acc;
        }
    return m;
}

// Row a of U_mu(s), and row a of U_mu(s)^dag (= conjugated column a).
__device__ __forceinline__ void ld_link_row(const double* links, int s, int mu, int a, c128 r[3]) {
    const double2* p = reinterpret_cast<const double2*>(links) + ((size_t)s * 4 + mu) * 9;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        double2 d = p[a * 3 + b];
        r[b] = c128{d.x, d.y};
    }
}
__device__ __forceinline__ void ld_link_dag_row(const double* links, int s, int mu, int a, c128 r[3]) {
    const double2* p = reinterpret_cast<const double2*>(links) + ((size_t)s * 4 + mu) * 9;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        double2 d = p[b * 3 + a];
        r[b] = c128{d.x, -d.y};
    }
}

// r . M (row vector times matrix)
__device__ __forceinline__ void rowmul(const c128 r[3], const m3& M, c128 out[3]) {
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        c128 acc{0.0, 0.0};
#pragma unroll
        for (int c = 0; c < 3; ++c) cfma(acc, r[c], M.e[c][b]);
        out[b] = acc;
    }
}

// Clover planes p = 0..5: (mu, nu) = (x,y) (x,z) (x,t) (y,z) (y,t) (z,t).
__device__ __forceinline__ int plane_mu(int p) { return p < 3 ? 0 : (p < 5 ? 1 : 2); }
__device__ __forceinline__ int plane_nu(int p) { return p == 0 ? 1 : p == 1 ? 2 : p == 2 ? 3 : p == 3 ? 2 : 3; }

// B_m = eps_mjk F_jk / 2 and E_m = F_{t m} as (plane, sign): B_x = F_yz, B_y = -F_xz,
// B_z = F_xy; E_m = -F_{m t}.
__device__ __forceinline__ void b_plane(int m, int& p, double& sg) {
    p = m == 0 ? 3 : m == 1 ? 1 : 0;
    sg = m == 1 ? -1.0 : 1.0;
}
__device__ __forceinline__ void e_plane(int m, int& p, double& sg) {
    p = m == 0 ? 2 : m == 1 ? 4 : 5;
    sg = -1.0;
}

__device__ __forceinline__ m3 ld_F(const double2* F, int Vs, int p, double sg, int s) {
    m3 m;
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        double2 d = F[((size_t)p * 9 + e) * Vs + s];
        m.e[e / 3][e % 3] = c128{sg * d.x, sg * d.y};
    }
    return m;
}
__device__ __forceinline__ void ld_F_row(const double2* F, int Vs, int p, double sg, int s, int a, c128 r[3]) {
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        double2 d = F[((size_t)p * 9 + a * 3 + b) * Vs + s];
        r[b] = c128{sg * d.x, sg * d.y};
    }
}
__device__ __forceinline__ m3 ld_B(const double2* F, int Vs, int m, int s) {
    int p; double sg; b_plane(m, p, sg);
    return ld_F(F, Vs, p, sg, s);
}
__device__ __forceinline__ m3 ld_E(const double2* F, int Vs, int m, int s) {
    int p; double sg; e_plane(m, p, sg);
    return ld_F(F, Vs, p, sg, s);
}
__device__ __forceinline__ void ld_B_row(const double2* F, int Vs, int m, int s, int a, c128 r[3]) {
    int p; double sg; b_plane(m, p, sg);
    ld_F_row(F, Vs, p, sg, s, a, r);
}
__device__ __forceinline__ void ld_E_row(const double2* F, int Vs, int m, int s, int a, c128 r[3]) {
    int p; double sg; e_plane(m, p, sg);
    ld_F_row(F, Vs, p, sg, s, a, r);
}

// x + n mu-hat (+ m nu-hat); written with selects so that runtime directions stay in registers
__device__ __forceinline__ int nb2(const Geo& g, const int c[4], int mu, int n, int nu, int m) {
    const int dx = (mu == 0 ? n : 0) + (nu == 0 ? m : 0);
    const int dy = (mu == 1 ? n : 0) + (nu == 1 ? m : 0);
    const int dz = (mu == 2 ? n : 0) + (nu == 2 ? m : 0);
    const int dt = (mu == 3 ? n : 0) + (nu == 3 ? m : 0);
    return neighbour(g, c[0], c[1], c[2], c[3], dx, dy, dz, dt);
}
__device__ __forceinline__ int nb1(const Geo& g, const int c[4], int mu, int n) {
    return nb2(g, c, mu, n, mu, 0);
}

// ------------------------------------------------------------------ clover
__global__ void __launch_bounds__(256) k_clover(Geo g, const double* links, double2* F) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.V) return;
    const int p = blockIdx.y;
    const int mu = plane_mu(p), nu = plane_nu(p);
    int c[4];
    site_coords(g, s, c[0], c[1], c[2], c[3]);
    const int xpm = nb1(g, c, mu, 1), xpn = nb1(g, c, nu, 1);
    const int xmm = nb1(g, c, mu, -1), xmn = nb1(g, c, nu, -1);
    const int xmm_pn = nb2(g, c, mu, -1, nu, 1), xmm_mn = nb2(g, c, mu, -1, nu, -1);
    const int xmn_pm = nb2(g, c, nu, -1, mu, 1);

    const m3 Umu = ld_link(links, s, mu), Unu = ld_link(links, s, nu);
    // leaf 1: x -> x+mu -> x+mu+nu -> x+nu -> x
    m3 Q = mul(mul(mul(Umu, ld_link(links, xpm, nu)), dagm(ld_link(links, xpn, mu))), dagm(Unu));
    // leaf 2: x -> x+nu -> x+nu-mu -> x-mu -> x
    m3 L = mul(mul(mul(Unu, dagm(ld_link(links, xmm_pn, mu))), dagm(ld_link(links, xmm, nu))),
               ld_link(links, xmm, mu));
#pragma unroll
    for (int e = 0; e < 9; ++e) Q.e[e / 3][e % 3] = Q.e[e / 3][e % 3] + L.e[e / 3][e % 3];
    // leaf 3: x -> x-mu -> x-mu-nu -> x-nu -> x
    L = mul(mul(mul(dagm(ld_link(links, xmm, mu)), dagm(ld_link(links, xmm_mn, nu))),
                ld_link(links, xmm_mn, mu)), ld_link(links, xmn, nu));
#pragma unroll
    for (int e = 0; e < 9; ++e) Q.e[e / 3][e % 3] = Q.e[e / 3][e % 3] + L.e[e / 3][e % 3];
    // leaf 4: x -> x-nu -> x-nu+mu -> x+mu -> x
    L = mul(mul(mul(dagm(ld_link(links, xmn, nu)), ld_link(links, xmn, mu)), ld_link(links, xmn_pm, nu)),
            dagm(Umu));
#pragma unroll
    for (int e = 0; e < 9; ++e) Q.e[e / 3][e % 3] = Q.e[e / 3][e % 3] + L.e[e / 3][e % 3];

    // F = traceless part of (Q - Q^dag)/8
    m3 Fm;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) Fm.e[a][b] = 0.125 * (Q.e[a][b] - conj(Q.e[b][a]));
    const c128 tr = (1.0 / 3.0) * (Fm.e[0][0] + Fm.e[1][1] + Fm.e[2][2]);
#pragma unroll
    for (int a = 0; a < 3; ++a) Fm.e[a][a] = Fm.e[a][a] - tr;
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        c128 v = Fm.e[e / 3][e % 3];
        F[((size_t)p * 9 + e) * g.Vs + s] = make_double2(v.re, v.im);
    }
}

// ------------------------------------------------------------------ forward blocks
// One 2x2 spin block of W, row a of its colour part, in the Pauli decomposition
// sum_{n=0..3} sigma_n (x) X_n (sigma_0 = 1).
struct Half {
    c128 h[4][3];
};

__device__ __forceinline__ void hzero(Half& H) {
#pragma unroll
    for (int n = 0; n < 4; ++n)
#pragma unroll
        for (int b = 0; b < 3; ++b) H.h[n][b] = c128{0.0, 0.0};
}

// H += coef * sigma_n (x) r
__device__ __forceinline__ void hacc(Half& H, int n, c128 coef, const c128 r[3]) {
#pragma unroll
    for (int m = 0; m < 4; ++m)
        if (m == n) {
#pragma unroll
            for (int b = 0; b < 3; ++b) cfma(H.h[m][b], coef, r[b]);
        }
}

// sigma_n sigma_m = ph * sigma_idx for n, m in 1..3 (sigma_n^2 = 1, sigma_n sigma_m = i eps_nmk sigma_k).
__device__ __forceinline__ void pauli_prod(int n, int m, int& idx, c128& ph) {
    if (n == m) {
        idx = 0;
        ph = c128{1.0, 0.0};
        return;
    }
    idx = 6 - n - m;   // the third of {1, 2, 3}
    const bool cyc = (n == 1 && m == 2) || (n == 2 && m == 3) || (n == 3 && m == 1);
    ph = c128{0.0, cyc ? 1.0 : -1.0};
}

// Entry (s, t) of the 2x2 spin matrix sum_n sigma_n X_n at colour column b.
__device__ __forceinline__ c128 half_entry(const Half& H, int s, int t, int b) {
    const c128 h0 = H.h[0][b], h1 = H.h[1][b], h2 = H.h[2][b], h3 = H.h[3][b];
    if (s == 0 && t == 0) return h0 + h3;
    if (s == 0 && t == 1) return c128{h1.re + h2.im, h1.im - h2.re};   // h1 - i h2
    if (s == 1 && t == 0) return c128{h1.re - h2.im, h1.im + h2.re};   // h1 + i h2
    return h0 - h3;
}

// Arrangement of the two distinct spin blocks H1, H2 in W = [[A, B], [C, D]].
enum Shape { SH_DS = 0,    // [[H1, H2], [H2, H1]]   W+_i, W++_ii
             SH_W0 = 1,    // [[H1, H2], [-H2, H1]]  W0
             SH_T4 = 2,    // [[0, H1], [H1, H2]]    W+_4
             SH_OFF = 3 }; // [[0, H1], [H1, 0]]     W++_ij, W+-_ij

__device__ __forceinline__ void shape_weights(int shape, int hr, int hc, double& w1, double& w2) {
    const bool diag = hr == hc;
    switch (shape) {
        case SH_DS: w1 = diag ? 1.0 : 0.0; w2 = diag ? 0.0 : 1.0; break;
        case SH_W0: w1 = diag ? 1.0 : 0.0; w2 = diag ? 0.0 : (hr == 0 ? 1.0 : -1.0); break;
        case SH_T4: w1 = diag ? 0.0 : 1.0; w2 = (hr == 1 && hc == 1) ? 1.0 : 0.0; break;
        default: w1 = diag ? 0.0 : 1.0; w2 = 0.0; break;
    }
}

struct PreCoef {
    double cD0, cS0;        // W0: -(c_B zeta + 16 c5)/(2 u0^3), -c_E zeta/(2 u0^3)
    double cS4;             // W+_4: c_EE/(2 u0^4)
    double cSi, cC3;        // S+_i: (zeta - 2c1 - 12c2)/2, c3/(2 u0^4)
    double cDi, cEps, cC5;  // D+_i: -(r_s zeta + 8c4)/2, (c5/4)(u0^-2 - u0^-4), c5/u0^4
    double cDii, cSii;      // W++_ii: c4/u0, (c1 + 2c2)/(2u0)
    double cOff;            // W++_ij, W+-_ij: c2/(2u0)
};

constexpr int kPairI[3] = {0, 0, 1};
constexpr int kPairJ[3] = {1, 2, 2};

// ------------------------------------------------------------------ Pauli-decomposed storage
// Row a (three FP64 entries) of colour matrix mi of site s, stored at precision P (LAY_SIGMA).
template <int P>
__device__ __forceinline__ void sigma_store_row(void* W, int Vs, int mi, int a, int s, const c128 r[3]) {
    char* base = reinterpret_cast<char*>(W);
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const size_t off = sigma_off<P>(Vs, mi, 3 * a + b, s);
        if constexpr (P == OK_F64) *reinterpret_cast<double2*>(base + off) = make_double2(r[b].re, r[b].im);
        else *reinterpret_cast<float2*>(base + off) = make_float2((float)r[b].re, (float)r[b].im);
    }
}

template <int P>
__device__ __forceinline__ void sigma_load_row(const void* W, int Vs, int mi, int a, int s, c128 r[3]) {
    const char* base = reinterpret_cast<const char*>(W);
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const size_t off = sigma_off<P>(Vs, mi, 3 * a + b, s);
        if constexpr (P == OK_F64) {
            const double2 d = *reinterpret_cast<const double2*>(base + off);
            r[b] = c128{d.x, d.y};
        } else {
            const float2 f = *reinterpret_cast<const float2*>(base + off);
            r[b] = c128{(double)f.x, (double)f.y};
        }
    }
}

// Forward block f (0: W0, 1..3: W+_i, 4: W+_4, 5..7: W++_ii, 8..10: W++_ij, 11..13: W+-_ij),
// colour row a, from its two Pauli-decomposed spin blocks: store the matrices listed in wlayout.h.
template <int P>
__device__ void sigma_store_block(void* W, int Vs, int f, int a, int s, const Half& H1, const Half& H2) {
    c128 r[3];
    if (f == 0) {
#pragma unroll
        for (int m = 1; m <= 3; ++m) {
#pragma unroll
            for (int b = 0; b < 3; ++b)   // (X1 - i X2) / 2
                r[b] = c128{0.5 * (H1.h[m][b].re + H2.h[m][b].im), 0.5 * (H1.h[m][b].im - H2.h[m][b].re)};
            sigma_store_row<P>(W, Vs, SG_W0 + m - 1, a, s, r);
#pragma unroll
            for (int b = 0; b < 3; ++b)   // (X1 + i X2) / 2
                r[b] = c128{0.5 * (H1.h[m][b].re - H2.h[m][b].im), 0.5 * (H1.h[m][b].im + H2.h[m][b].re)};
            sigma_store_row<P>(W, Vs, SG_W0 + 2 + m, a, s, r);
        }
    } else if (f <= 3) {
        const int base = SG_WI + 8 * (f - 1);
#pragma unroll
        for (int n = 0; n < 4; ++n) {
#pragma unroll
            for (int b = 0; b < 3; ++b) r[b] = 0.5 * (H1.h[n][b] + H2.h[n][b]);
            sigma_store_row<P>(W, Vs, base + n, a, s, r);
#pragma unroll
            for (int b = 0; b < 3; ++b) r[b] = 0.5 * (H1.h[n][b] - H2.h[n][b]);
            sigma_store_row<P>(W, Vs, base + 4 + n, a, s, r);
        }
    } else if (f == 4) {
#pragma unroll
        for (int m = 1; m <= 3; ++m) sigma_store_row<P>(W, Vs, SG_W4 + m - 1, a, s, H1.h[m]);
        sigma_store_row<P>(W, Vs, SG_W4 + 3, a, s, H2.h[0]);
    } else if (f <= 7) {
        const int i = f - 5;
        sigma_store_row<P>(W, Vs, SG_WII + 2 * i, a, s, H1.h[0]);
        sigma_store_row<P>(W, Vs, SG_WII + 2 * i + 1, a, s, H2.h[1 + i]);
    } else if (f <= 10) {
        sigma_store_row<P>(W, Vs, SG_WIJ + f - 8, a, s, H1.h[1 + kPairI[f - 8]]);
    } else {
        sigma_store_row<P>(W, Vs, SG_WIMJ + f - 11, a, s, H1.h[1 + kPairI[f - 11]]);
    }
}

// Inverse of sigma_store_block: the two spin blocks (row a) and the shape of forward block f.
template <int P>
__device__ void sigma_load_block(const void* W, int Vs, int f, int a, int s, Half& H1, Half& H2, int& shape) {
    hzero(H1);
    hzero(H2);
    c128 r[3], q[3];
    if (f == 0) {
        shape = SH_W0;
#pragma unroll
        for (int m = 1; m <= 3; ++m) {
            sigma_load_row<P>(W, Vs, SG_W0 + m - 1, a, s, r);   // (X1 - i X2) / 2
            sigma_load_row<P>(W, Vs, SG_W0 + 2 + m, a, s, q);   // (X1 + i X2) / 2
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                H1.h[m][b] = r[b] + q[b];
                const c128 d = r[b] - q[b];                      // -i X2
                H2.h[m][b] = c128{-d.im, d.re};                  // i (-i X2)
            }
        }
    } else if (f <= 3) {
        shape = SH_DS;
        const int base = SG_WI + 8 * (f - 1);
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            sigma_load_row<P>(W, Vs, base + n, a, s, r);
            sigma_load_row<P>(W, Vs, base + 4 + n, a, s, q);
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                H1.h[n][b] = r[b] + q[b];
                H2.h[n][b] = r[b] - q[b];
            }
        }
    } else if (f == 4) {
        shape = SH_T4;
#pragma unroll
        for (int m = 1; m <= 3; ++m) sigma_load_row<P>(W, Vs, SG_W4 + m - 1, a, s, H1.h[m]);
        sigma_load_row<P>(W, Vs, SG_W4 + 3, a, s, H2.h[0]);
    } else if (f <= 7) {
        shape = SH_DS;
        const int i = f - 5;
        sigma_load_row<P>(W, Vs, SG_WII + 2 * i, a, s, H1.h[0]);
        sigma_load_row<P>(W, Vs, SG_WII + 2 * i + 1, a, s, H2.h[1 + i]);
    } else {
        shape = SH_OFF;
        const bool plus = f <= 10;
        const int p = plus ? f - 8 : f - 11;
        sigma_load_row<P>(W, Vs, (plus ? SG_WIJ : SG_WIMJ) + p, a, s, r);
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            H1.h[1 + kPairI[p]][b] = r[b];
            H1.h[1 + kPairJ[p]][b] = plus ? r[b] : -r[b];
        }
    }
}

// Row (alpha, a) of a block from its spin blocks: entry (beta, b) = sum of the spin blocks at (alpha/2, beta/2).
__device__ __forceinline__ void expand_row(int shape, int al, const Half& H1, const Half& H2, c128 v[12]) {
#pragma unroll
    for (int be = 0; be < 4; ++be) {
        double w1, w2;
        shape_weights(shape, al >> 1, be >> 1, w1, w2);
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            c128 e1 = half_entry(H1, al & 1, be & 1, b);
            c128 e2 = half_entry(H2, al & 1, be & 1, b);
            v[3 * be + b] = w1 * e1 + w2 * e2;
        }
    }
}

template <int P>
__global__ void __launch_bounds__(64) k_forward(Geo g, PreCoef q, const double* links, const double2* F,
                                                void* W, int layout) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.V) return;
    const int f = blockIdx.y;   // 0: W0, 1..3: W+_i, 4: W+_4, 5..7: W++_ii, 8..10: W++_ij, 11..13: W+-_ij
    const int a = blockIdx.z;   // colour row
    int c[4];
    site_coords(g, s, c[0], c[1], c[2], c[3]);
    const int Vs = g.Vs;

    Half H1, H2;
    hzero(H1);
    hzero(H2);
    int shape, k;
    c128 r[3], t1[3], t2[3];

    if (f == 0) {
        // W0 - mhat = [[D0, S0], [-S0, D0]], D0 = cD0 * i sum_m sigma_m B_m, S0 = cS0 * sum_m sigma_m E_m
        shape = SH_W0;
        k = 0;
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            ld_B_row(F, Vs, m, s, a, r);
            hacc(H1, 1 + m, c128{0.0, q.cD0}, r);
            ld_E_row(F, Vs, m, s, a, r);
            hacc(H2, 1 + m, c128{q.cS0, 0.0}, r);
        }
    } else if (f <= 3) {
        // W+_i = [[D_i, S_i], [S_i, D_i]]
        const int i = f - 1;
        shape = SH_DS;
        k = 1 + i;
        const int xpi = nb1(g, c, i, 1);
        const m3 Ui = ld_link(links, s, i);
        c128 ur[3];
        ld_link_row(links, s, i, a, ur);
        // S_i: (zeta - 2c1 - 12c2)/2 sigma_i U_i ;  D_i: -(r_s zeta + 8 c4)/2 U_i
        hacc(H2, 1 + i, c128{q.cSi, 0.0}, ur);
        hacc(H1, 0, c128{q.cDi, 0.0}, ur);
        // clover terms: with P_m = U_i B_m(x+i), Q_m = B_m(x) U_i,
        //   S_i += c3/(2u0^4) [ sum_m i sigma_i sigma_m (P_m - Q_m) + 2i B_i U_i ]
        //   D_i += c5/u0^4 [ sum_m i sigma_m (P_m + Q_m) - i sigma_i (P_i + Q_i) ]
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            rowmul(ur, ld_B(F, Vs, m, xpi), t1);     // row a of P_m
            ld_B_row(F, Vs, m, s, a, r);
            rowmul(r, Ui, t2);                        // row a of Q_m
            int idx;
            c128 ph;
            pauli_prod(1 + i, 1 + m, idx, ph);
            const c128 cs = c128{0.0, q.cC3} * ph;    // i * c3/(2u0^4) * phase
#pragma unroll
            for (int b = 0; b < 3; ++b) r[b] = t1[b] - t2[b];
            hacc(H2, idx, cs, r);
#pragma unroll
            for (int b = 0; b < 3; ++b) r[b] = t1[b] + t2[b];
            if (m != i) hacc(H1, 1 + m, c128{0.0, q.cC5}, r);
            if (m == i) hacc(H2, 0, c128{0.0, 2.0 * q.cC3}, t2);   // 2i c3/(2u0^4) B_i U_i
        }
        // staple term: i (c5/4)(u0^-2 - u0^-4) sum_{jk} eps_ijk sigma_j
        //   (U_k(x) U_i(x+k) U_k(x+i)^dag - U_k(x-k)^dag U_i(x-k) U_k(x-k+i))
        if (q.cEps != 0.0) {
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                if (j == i) continue;
                const int kk = 3 - i - j;
                const double eps = ((i == 0 && j == 1) || (i == 1 && j == 2) || (i == 2 && j == 0)) ? 1.0 : -1.0;
                const int xpk = nb1(g, c, kk, 1), xmk = nb1(g, c, kk, -1);
                const int xmk_pi = nb2(g, c, kk, -1, i, 1);
                ld_link_row(links, s, kk, a, r);
                rowmul(r, ld_link(links, xpk, i), t1);
                rowmul(t1, dagm(ld_link(links, xpi, kk)), t2);
                ld_link_dag_row(links, xmk, kk, a, r);
                rowmul(r, ld_link(links, xmk, i), t1);
                rowmul(t1, ld_link(links, xmk_pi, kk), r);
#pragma unroll
                for (int b = 0; b < 3; ++b) t2[b] = t2[b] - r[b];
                hacc(H1, 1 + j, c128{0.0, eps * q.cEps}, t2);
            }
        }
    } else if (f == 4) {
        // W+_4 = [[0, S4], [S4, -U_4]], S4 = c_EE/(2u0^4) (U_4 E^S_{x+4} - E^S_x U_4)
        shape = SH_T4;
        k = 4;
        const int xpt = nb1(g, c, 3, 1);
        const m3 U4 = ld_link(links, s, 3);
        c128 ur[3];
        ld_link_row(links, s, 3, a, ur);
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            rowmul(ur, ld_E(F, Vs, m, xpt), t1);
            ld_E_row(F, Vs, m, s, a, r);
            rowmul(r, U4, t2);
#pragma unroll
            for (int b = 0; b < 3; ++b) r[b] = t1[b] - t2[b];
            hacc(H1, 1 + m, c128{q.cS4, 0.0}, r);
        }
        hacc(H2, 0, c128{-1.0, 0.0}, ur);
    } else if (f <= 7) {
        // W++_ii = [[D, S], [S, D]], D = c4/u0 U_i(x) U_i(x+i), S = (c1 + 2c2)/(2u0) sigma_i U_i U_i
        const int i = f - 5;
        shape = SH_DS;
        k = 9 + i;
        ld_link_row(links, s, i, a, r);
        rowmul(r, ld_link(links, nb1(g, c, i, 1), i), t1);
        hacc(H1, 0, c128{q.cDii, 0.0}, t1);
        hacc(H2, 1 + i, c128{q.cSii, 0.0}, t1);
    } else if (f <= 10) {
        // W++_ij = [[0, S], [S, 0]], S = c2/(2u0) (sigma_i + sigma_j)(U_i(x) U_j(x+i) + U_j(x) U_i(x+j))
        const int p = f - 8, i = kPairI[p], j = kPairJ[p];
        shape = SH_OFF;
        k = 15 + p;
        ld_link_row(links, s, i, a, r);
        rowmul(r, ld_link(links, nb1(g, c, i, 1), j), t1);
        ld_link_row(links, s, j, a, r);
        rowmul(r, ld_link(links, nb1(g, c, j, 1), i), t2);
#pragma unroll
        for (int b = 0; b < 3; ++b) t1[b] = t1[b] + t2[b];
        hacc(H1, 1 + i, c128{q.cOff, 0.0}, t1);
        hacc(H1, 1 + j, c128{q.cOff, 0.0}, t1);
    } else {
        // W+-_ij = [[0, S'], [S', 0]], S' = c2/(2u0) (sigma_i - sigma_j)
        //          (U_i(x) U_j(x-j+i)^dag + U_j(x-j)^dag U_i(x-j))
        const int p = f - 11, i = kPairI[p], j = kPairJ[p];
        shape = SH_OFF;
        k = 21 + p;
        const int xmj = nb1(g, c, j, -1);
        ld_link_row(links, s, i, a, r);
        rowmul(r, dagm(ld_link(links, nb2(g, c, j, -1, i, 1), j)), t1);
        ld_link_dag_row(links, xmj, j, a, r);
        rowmul(r, ld_link(links, xmj, i), t2);
#pragma unroll
        for (int b = 0; b < 3; ++b) t1[b] = t1[b] + t2[b];
        hacc(H1, 1 + i, c128{q.cOff, 0.0}, t1);
        hacc(H1, 1 + j, c128{-q.cOff, 0.0}, t1);
    }

    if (layout == LAY_SIGMA) {
        if constexpr (P != OK_BF16) sigma_store_block<P>(W, Vs, f, a, s, H1, H2);
        return;
    }
    // expand: row (alpha, a) of W, entry (beta, b) = sum of the spin blocks at (alpha/2, beta/2)
#pragma unroll
    for (int al = 0; al < 4; ++al) {
        c128 v[12];
        expand_row(shape, al, H1, H2, v);
        w_store_row<P>(W, Vs, layout, k, 3 * al + a, s, v);
    }
}

// ------------------------------------------------------------------ backward blocks
constexpr int kBwd[13] = {5, 6, 7, 8, 12, 13, 14, 18, 19, 20, 24, 25, 26};
constexpr int kFwdOf[13] = {1, 2, 3, 4, 9, 10, 11, 15, 16, 17, 21, 22, 23};

template <int P>
__global__ void __launch_bounds__(64) k_backward(Geo g, void* W, int layout) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.V) return;
    const int kb = kBwd[blockIdx.y], kf = kFwdOf[blockIdx.y];
    const int row = blockIdx.z;
    int x, y, z, t;
    site_coords(g, s, x, y, z, t);
    const int src = neighbour(g, x, y, z, t, -off_d(kf, 0), -off_d(kf, 1), -off_d(kf, 2), -off_d(kf, 3));
    const int al = row / 3, a = row % 3, alp = al ^ 2;
    c128 v[12];
#pragma unroll
    for (int be = 0; be < 4; ++be) {
        const int bep = be ^ 2;
        const double sg = ((al < 2) == (be < 2)) ? 1.0 : -1.0;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            // Gamma(X)[(al,a),(be,b)] = sg * conj(X[(be^2, b), (al^2, a)])
            c128 xv = w_load_entry<P>(W, g.Vs, layout, kf, (3 * bep + b) * 12 + 3 * alp + a, src);
            v[3 * be + b] = c128{sg * xv.re, -sg * xv.im};
        }
    }
    w_store_row<P>(W, g.Vs, layout, kb, row, s, v);
}

// ------------------------------------------------------------------ dense expansion
template <int P>
__global__ void __launch_bounds__(64) k_to_dense(Geo g, const void* W, int layout, double2* dense) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.V) return;
    const int k = blockIdx.y, row = blockIdx.z;
    if constexpr (P != OK_BF16) {
        if (layout == LAY_SIGMA) {
            // forward block f of offset kf, expanded from its matrices; a backward offset takes
            // gamma5 (forward block at x - d)^dag gamma5 entry by entry
            const int ks = saved_index(k);
            int kf = k;
            if (ks < 0)
                for (int i = 0; i < 13; ++i)
                    if (kBwd[i] == k) kf = kFwdOf[i];
            const int f = kf == 0 ? 0 : kf <= 3 ? kf : kf == 4 ? 4 : kf <= 11 ? kf - 4 : kf <= 17 ? kf - 7 : kf - 10;
            int x, y, z, t;
            site_coords(g, s, x, y, z, t);
            const int src = ks >= 0 ? s : neighbour(g, x, y, z, t, -off_d(kf, 0), -off_d(kf, 1), -off_d(kf, 2), -off_d(kf, 3));
            const int al = row / 3, a = row % 3;
            Half H1, H2;
            int shape;
            c128 v[12];
            if (ks >= 0) {
                sigma_load_block<P>(W, g.Vs, f, a, src, H1, H2, shape);
                expand_row(shape, al, H1, H2, v);
                for (int col = 0; col < 12; ++col) dense[((size_t)s * kW + k) * kWE + row * 12 + col] = make_double2(v[col].re, v[col].im);
                return;
            }
            for (int be = 0; be < 4; ++be)
                for (int b = 0; b < 3; ++b) {
                    // Gamma(X)[(al,a),(be,b)] = sg * conj(X[(be^2, b), (al^2, a)])
                    sigma_load_block<P>(W, g.Vs, f, b, src, H1, H2, shape);
                    expand_row(shape, be ^ 2, H1, H2, v);
                    const c128 xv = v[3 * (al ^ 2) + a];
                    const double sg = ((al < 2) == (be < 2)) ? 1.0 : -1.0;
                    dense[((size_t)s * kW + k) * kWE + row * 12 + 3 * be + b] = make_double2(sg * xv.re, -sg * xv.im);
                }
            return;
        }
    }
    if (layout == LAY_SAVED && saved_index(k) < 0) {
        // backward block of the saved set: gamma5 (forward block at x - d)^dag gamma5
        int kf = 0;
        for (int i = 0; i < 13; ++i)
            if (kBwd[i] == k) kf = kFwdOf[i];
        int x, y, z, t;
        site_coords(g, s, x, y, z, t);
        const int src = neighbour(g, x, y, z, t, -off_d(kf, 0), -off_d(kf, 1), -off_d(kf, 2), -off_d(kf, 3));
        const int al = row / 3, a = row % 3, alp = al ^ 2;
        for (int be = 0; be < 4; ++be) {
            const double sg = ((al < 2) == (be < 2)) ? 1.0 : -1.0;
            for (int b = 0; b < 3; ++b) {
                const c128 xv = w_load_entry<P>(W, g.Vs, layout, kf, (3 * (be ^ 2) + b) * 12 + 3 * alp + a, src);
                dense[((size_t)s * kW + k) * kWE + row * 12 + 3 * be + b] = make_double2(sg * xv.re, -sg * xv.im);
            }
        }
        return;
    }
#pragma unroll
    for (int col = 0; col < 12; ++col) {
        c128 v = w_load_entry<P>(W, g.Vs, layout, k, row * 12 + col, s);
        dense[((size_t)s * kW + k) * kWE + row * 12 + col] = make_double2(v.re, v.im);
    }
}

template <int P>
int run_precompute(const Geo& g, const PreCoef& q, const double* links, void* W, int layout, double2* F,
                   hipStream_t st) {
    const unsigned nb = grid_for(g.V, 64);
    k_clover<<<dim3(grid_for(g.V, 256), 6), 256, 0, st>>>(g, links, F);
    OK_LAUNCH_CHECK("k_clover");
    k_forward<P><<<dim3(nb, 14, 3), 64, 0, st>>>(g, q, links, F, W, layout);
    OK_LAUNCH_CHECK("k_forward");
    if (layout != LAY_SAVED && layout != LAY_SIGMA) {   // these form their backward blocks where they are used
        k_backward<P><<<dim3(nb, 13, 12), 64, 0, st>>>(g, W, layout);
        OK_LAUNCH_CHECK("k_backward");
    }
    return OK_SUCCESS;
}

}  // namespace

int launch_precompute(const Geo& g, const ok_coeffs& c, const double* links, int prec, void* W,
                      void* scratch, hipStream_t st) {
    const double u0 = c.u0;
    const double u2 = 1.0 / (u0 * u0), u3 = u2 / u0, u4 = u2 * u2;
    PreCoef q;
    q.cD0 = -(c.c_B * c.zeta + 16.0 * c.c_5) * 0.5 * u3;
    q.cS0 = -(c.c_E * c.zeta) * 0.5 * u3;
    q.cS4 = c.c_EE * 0.5 * u4;
    q.cSi = 0.5 * (c.zeta - 2.0 * c.c_1 - 12.0 * c.c_2);
    q.cC3 = c.c_3 * 0.5 * u4;
    q.cDi = -0.5 * (c.r_s * c.zeta + 8.0 * c.c_4);
    q.cEps = 0.25 * c.c_5 * (u2 - u4);
    q.cC5 = c.c_5 * u4;
    q.cDii = c.c_4 / u0;
    q.cSii = (c.c_1 + 2.0 * c.c_2) * 0.5 / u0;
    q.cOff = c.c_2 * 0.5 / u0;
    double2* F = reinterpret_cast<double2*>(scratch);
    const int layout = layout_of(prec);
    switch (prec & 3) {
        case OK_F64: return run_precompute<OK_F64>(g, q, links, W, layout, F, st);
        case OK_F32: return run_precompute<OK_F32>(g, q, links, W, layout, F, st);
        default: return run_precompute<OK_BF16>(g, q, links, W, layout, F, st);
    }
}

int launch_to_dense(const Geo& g, const void* W, int prec, double* dense, hipStream_t st) {
    dim3 grid(grid_for(g.V, 64), kW, 12);
    double2* d = reinterpret_cast<double2*>(dense);
    const int layout = layout_of(prec);
    switch (prec & 3) {
        case OK_F64: k_to_dense<OK_F64><<<grid, 64, 0, st>>>(g, W, layout, d); break;
        case OK_F32: k_to_dense<OK_F32><<<grid, 64, 0, st>>>(g, W, layout, d); break;
        default: k_to_dense<OK_BF16><<<grid, 64, 0, st>>>(g, W, layout, d); break;
    }
    OK_LAUNCH_CHECK("k_to_dense");
    return OK_SUCCESS;
}

}  // namespace okinv
