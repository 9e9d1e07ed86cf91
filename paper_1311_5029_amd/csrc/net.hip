// Kernels of the learned right preconditioner: a chain of gauge-covariant
// linear stencil layers over the 27 offsets of Eq. minFlopForm,
//
//   phi'_x = sum_k A_k P_k(x) phi_{x+d_k},
//
// A_k a 4x4 complex spin matrix and P_k(x) the colour transport of hop k.
// Fields are FP32 complex, either [nf][V][12] ("outer") or [V][12][nf]
// ("inner", the layout of the batched solver).  Reductions (weight gradients,
// loss) run over a fixed grid and finish in FP64 in a fixed order, so every
// result is bitwise reproducible.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace okinv {
namespace {

constexpr int BS = 256;

// Transport planes: the 13 forward hops (k = 1..4, 9..11, 15..17, 21..23).
// plane_of(k) is the plane of hop k (forward or backward), is_fwd(k) whether
// hop k reads the plane at x (forward) or takes P_d(x - d)^dag (backward).
__host__ __device__ constexpr int plane_of(int k) {
    return k <= 4 ? k - 1 : k <= 8 ? k - 5 : k <= 11 ? k - 5 : k <= 14 ? k - 8
         : k <= 17 ? k - 8 : k <= 20 ? k - 11 : k <= 23 ? k - 11 : k - 14;
}
__host__ __device__ constexpr bool is_fwd(int k) {
    return (k >= 1 && k <= 4) || (k >= 9 && k <= 11) || (k >= 15 && k <= 17) || (k >= 21 && k <= 23);
}
// index of the hop -d_k
__host__ __device__ constexpr int neg_hop(int k) {
    return k == 0 ? 0 : k <= 4 ? k + 4 : k <= 8 ? k - 4 : k <= 11 ? k + 3 : k <= 14 ? k - 3
         : k <= 17 ? k + 3 : k <= 20 ? k - 3 : k <= 23 ? k + 3 : k - 3;
}
static_assert(plane_of(4) == 3 && plane_of(8) == 3 && plane_of(9) == 4 && plane_of(14) == 6, "planes");
static_assert(plane_of(15) == 7 && plane_of(20) == 9 && plane_of(21) == 10 && plane_of(26) == 12, "planes");
static_assert(neg_hop(neg_hop(17)) == 17 && neg_hop(1) == 5 && neg_hop(24) == 21, "neg");

// ------------------------------------------------------------------ transports
struct M3 {
    double2 e[9];
};
__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zmulc(double2 a, double2 b) {   // a * conj(b)
    return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ double2 zcmul(double2 a, double2 b) {   // conj(a) * b
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ M3 load_link(const double2* U, int s, int mu) {
    M3 m;
    const double2* p = U + ((size_t)s * 4 + mu) * 9;
#pragma unroll
    for (int e = 0; e < 9; ++e) m.e[e] = p[e];
    return m;
}
// a b, a b^dag, a^dag b
__device__ __forceinline__ M3 mm(const M3& a, const M3& b) {
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double2 v = make_double2(0, 0);
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                const double2 t = zmul(a.e[i * 3 + l], b.e[l * 3 + j]);
                v.x += t.x;
                v.y += t.y;
            }
            c.e[i * 3 + j] = v;
        }
    return c;
}
__device__ __forceinline__ M3 mmd(const M3& a, const M3& b) {
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double2 v = make_double2(0, 0);
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                const double2 t = zmulc(a.e[i * 3 + l], b.e[j * 3 + l]);
                v.x += t.x;
                v.y += t.y;
            }
            c.e[i * 3 + j] = v;
        }
    return c;
}
__device__ __forceinline__ M3 mdm(const M3& a, const M3& b) {
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double2 v = make_double2(0, 0);
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                const double2 t = zcmul(a.e[l * 3 + i], b.e[l * 3 + j]);
                v.x += t.x;
                v.y += t.y;
            }
            c.e[i * 3 + j] = v;
        }
    return c;
}
__device__ __forceinline__ void store_plane(float2* T, int Vs, int plane, int s, const M3& m, double f) {
#pragma unroll
    for (int e = 0; e < 9; ++e)
        T[((size_t)plane * 9 + e) * Vs + s] = make_float2((float)(f * m.e[e].x), (float)(f * m.e[e].y));
}
__device__ __forceinline__ M3 madd(const M3& a, const M3& b) {
    M3 c;
#pragma unroll
    for (int e = 0; e < 9; ++e) c.e[e] = make_double2(a.e[e].x + b.e[e].x, a.e[e].y + b.e[e].y);
    return c;
}

// The 13 forward transports of site s, computed in FP64 and stored FP32:
// planes 0..3: U_mu(x); 4..6: U_i(x) U_i(x+i); 7..9 (ij = xy, xz, yz):
// (U_i(x) U_j(x+i) + U_j(x) U_i(x+j)) / 2; 10..12: (U_i(x) U_j(x+i-j)^dag +
// U_j(x-j)^dag U_i(x-j)) / 2.
__global__ void __launch_bounds__(BS) k_transports(Geo g, const double2* __restrict__ U, float2* __restrict__ T) {
    const int s = blockIdx.x * BS + threadIdx.x;
    if (s >= g.V) return;
    int c[4];
    site_coords(g, s, c[0], c[1], c[2], c[3]);
    auto nb = [&](int mu, int a, int nu, int b) {
        int d[4] = {0, 0, 0, 0};
        d[mu] += a;
        d[nu] += b;
        return neighbour(g, c[0], c[1], c[2], c[3], d[0], d[1], d[2], d[3]);
    };
    for (int mu = 0; mu < 4; ++mu) store_plane(T, g.Vs, mu, s, load_link(U, s, mu), 1.0);
    for (int i = 0; i < 3; ++i)
        store_plane(T, g.Vs, 4 + i, s, mm(load_link(U, s, i), load_link(U, nb(i, 1, i, 0), i)), 1.0);
    const int PI[3] = {0, 0, 1}, PJ[3] = {1, 2, 2};
    for (int p = 0; p < 3; ++p) {
        const int i = PI[p], j = PJ[p];
        const M3 Ui = load_link(U, s, i), Uj = load_link(U, s, j);
        const M3 a = mm(Ui, load_link(U, nb(i, 1, j, 0), j));
        const M3 b = mm(Uj, load_link(U, nb(j, 1, i, 0), i));
        store_plane(T, g.Vs, 7 + p, s, madd(a, b), 0.5);
        const int smj = nb(j, -1, i, 0);
        const M3 c1 = mmd(Ui, load_link(U, nb(i, 1, j, -1), j));
        const M3 c2 = mdm(load_link(U, smj, j), load_link(U, smj, i));
        store_plane(T, g.Vs, 10 + p, s, madd(c1, c2), 0.5);
    }
}

// ------------------------------------------------------------------ fields
template <bool INNER>
__device__ __forceinline__ size_t fidx(int V, int nf, int s, int b, int c) {
    return INNER ? ((size_t)s * 12 + c) * nf + b : ((size_t)b * V + s) * 12 + c;
}
template <bool INNER>
__device__ __forceinline__ void item_of(const Geo& g, int nf, long t, int& s, int& b) {
    if (INNER) {
        s = (int)(t / nf);
        b = (int)(t - (long)s * nf);
    } else {
        b = (int)(t / g.V);
        s = (int)(t - (long)b * g.V);
    }
}
__device__ __forceinline__ float2 fmac(float2 acc, float2 a, float2 b) {   // acc + a b
    acc.x = fmaf(a.x, b.x, acc.x);
    acc.x = fmaf(-a.y, b.y, acc.x);
    acc.y = fmaf(a.x, b.y, acc.y);
    acc.y = fmaf(a.y, b.x, acc.y);
    return acc;
}
__device__ __forceinline__ float2 fmacc(float2 acc, float2 a, float2 b) {   // acc + conj(a) b
    acc.x = fmaf(a.x, b.x, acc.x);
    acc.x = fmaf(a.y, b.y, acc.x);
    acc.y = fmaf(a.x, b.y, acc.y);
    acc.y = fmaf(-a.y, b.x, acc.y);
    return acc;
}

// u = P_k(x) phi_{x+d_k} for the 12 components of item (s, b); k is a compile-time hop.
template <bool INNER, int K>
__device__ __forceinline__ void hop(const Geo& g, int nf, const float2* __restrict__ T,
                                    const float2* __restrict__ in, int s, int b, const int* c, float2* u) {
    const int sn = K == 0 ? s
                          : neighbour(g, c[0], c[1], c[2], c[3], off_d(K, 0), off_d(K, 1), off_d(K, 2), off_d(K, 3));
    float2 ph[12];
#pragma unroll
    for (int e = 0; e < 12; ++e) ph[e] = in[fidx<INNER>(g.V, nf, sn, b, e)];
    if (K == 0) {
#pragma unroll
        for (int e = 0; e < 12; ++e) u[e] = ph[e];
        return;
    }
    constexpr int pl = plane_of(K);
    const int st = is_fwd(K) ? s : sn;
    float2 P[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) P[e] = T[((size_t)pl * 9 + e) * g.Vs + st];
#pragma unroll
    for (int al = 0; al < 4; ++al)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float2 v = make_float2(0.f, 0.f);
#pragma unroll
            for (int bb = 0; bb < 3; ++bb)
                v = is_fwd(K) ? fmac(v, P[a * 3 + bb], ph[al * 3 + bb]) : fmacc(v, P[bb * 3 + a], ph[al * 3 + bb]);
            u[al * 3 + a] = v;
        }
}

template <int K, int N>
struct Unroll {
    template <typename F>
    __device__ __forceinline__ static void run(F&& f) {
        f(std::integral_constant<int, K>{});
        Unroll<K + 1, N>::run(f);
    }
};
template <int N>
struct Unroll<N, N> {
    template <typename F>
    __device__ __forceinline__ static void run(F&&) {}
};

// out = sum_k A'_k P_k phi_{x+d_k}; A'_k = A_k, or A_{-k}^dag for the adjoint layer.
template <bool INNER, bool ADJ>
__global__ void __launch_bounds__(BS) k_layer(Geo g, int nf, const float2* __restrict__ A,
                                              const float2* __restrict__ T, const float2* __restrict__ in,
                                              float2* __restrict__ out) {
    const long t = (long)xcd_tile(blockIdx.x, gridDim.x) * BS + threadIdx.x;
    if (t >= (long)g.V * nf) return;
    int s, b;
    item_of<INNER>(g, nf, t, s, b);
    int c[4];
    site_coords(g, s, c[0], c[1], c[2], c[3]);
    float2 acc[12];
#pragma unroll
    for (int e = 0; e < 12; ++e) acc[e] = make_float2(0.f, 0.f);
    Unroll<0, 27>::run([&](auto kc) {
        constexpr int K = decltype(kc)::value;
        float2 u[12];
        hop<INNER, K>(g, nf, T, in, s, b, c, u);
        const float2* Ak = A + (ADJ ? neg_hop(K) : K) * 16;
#pragma unroll
        for (int al = 0; al < 4; ++al)
#pragma unroll
            for (int be = 0; be < 4; ++be) {
                float2 w = ADJ ? Ak[be * 4 + al] : Ak[al * 4 + be];
                if (ADJ) w.y = -w.y;
#pragma unroll
                for (int a = 0; a < 3; ++a) acc[al * 3 + a] = fmac(acc[al * 3 + a], w, u[be * 3 + a]);
            }
    });
#pragma unroll
    for (int e = 0; e < 12; ++e) out[fidx<INNER>(g.V, nf, s, b, e)] = acc[e];
}

// Weight gradient, first pass.  Block (ch, k) handles hop k over the items
// ch*BS + tid + i*nch*BS and writes the block sum
// partial[ch][k][16] of  sum g^{alpha a} conj(u_k^{beta a}).
template <bool INNER, int K>
__device__ __forceinline__ void wgrad_hop(const Geo& g, int nf, int nch, int ch, const float2* __restrict__ T,
                                          const float2* __restrict__ gout, const float2* __restrict__ in,
                                          float2* acc) {
    const long n = (long)g.V * nf;
    for (long t = (long)ch * BS + threadIdx.x; t < n; t += (long)nch * BS) {
        int s, b;
        item_of<INNER>(g, nf, t, s, b);
        int c[4];
        site_coords(g, s, c[0], c[1], c[2], c[3]);
        float2 u[12];
        hop<INNER, K>(g, nf, T, in, s, b, c, u);
#pragma unroll
        for (int al = 0; al < 4; ++al) {
            float2 gv[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) gv[a] = gout[fidx<INNER>(g.V, nf, s, b, al * 3 + a)];
#pragma unroll
            for (int be = 0; be < 4; ++be)
#pragma unroll
                for (int a = 0; a < 3; ++a) acc[al * 4 + be] = fmacc(acc[al * 4 + be], u[be * 3 + a], gv[a]);
        }
    }
}

template <bool INNER>
__global__ void __launch_bounds__(BS) k_wgrad(Geo g, int nf, int nch, const float2* __restrict__ T,
                                              const float2* __restrict__ gout, const float2* __restrict__ in,
                                              float2* __restrict__ partial) {
    // the 27 blocks of one chunk run on one XCD and share its L2 for gout and in
    const int blk = xcd_tile(blockIdx.x, gridDim.x);
    const int ch = blk / 27, k = blk % 27;
    float2 acc[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[e] = make_float2(0.f, 0.f);
    Unroll<0, 27>::run([&](auto kc) {
        constexpr int K = decltype(kc)::value;
        if (k == K) wgrad_hop<INNER, K>(g, nf, nch, ch, T, gout, in, acc);
    });
    // block sum in a fixed order: waves by shuffles, then the four waves in order
    __shared__ float2 red[BS / 64][16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        float2 v = acc[e];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            v.x += __shfl_xor(v.x, o, 64);
            v.y += __shfl_xor(v.y, o, 64);
        }
        if (lane == 0) red[wave][e] = v;
    }
    __syncthreads();
    if (threadIdx.x < 16) {
        float2 v = red[0][threadIdx.x];
        for (int w = 1; w < BS / 64; ++w) {
            v.x += red[w][threadIdx.x].x;
            v.y += red[w][threadIdx.x].y;
        }
        partial[((size_t)ch * 27 + k) * 16 + threadIdx.x] = v;
    }
}

// Second pass: gA[i] = sum over ch of partial[ch][i] (i = 16 k + e), one wavefront per i:
// lane l sums the chunks l, l + 64, ... in FP64, then the lanes are combined by a fixed
// shuffle tree, so the result does not depend on timing.
__global__ void __launch_bounds__(BS) k_wgrad_finish(int nch, const float2* __restrict__ partial,
                                                     float2* __restrict__ gA) {
    const int i = blockIdx.x * (BS / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= 27 * 16) return;
    double x = 0.0, y = 0.0;
    for (int ch = lane; ch < nch; ch += 64) {
        const float2 v = partial[(size_t)ch * 27 * 16 + i];
        x += v.x;
        y += v.y;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        x += __shfl_xor(x, o, 64);
        y += __shfl_xor(y, o, 64);
    }
    if (lane == 0) gA[i] = make_float2((float)x, (float)y);
}

// ------------------------------------------------------------------ loss
constexpr int kLossBlocks = 64;
// partial[b][blk] = (sum |psi_b|^2, sum |out_b - psi_b|^2) over the sites of block blk
template <bool INNER>
__global__ void __launch_bounds__(BS) k_loss_norms(Geo g, int nf, const float2* __restrict__ out,
                                                   const float2* __restrict__ psi, double2* __restrict__ partial) {
    const int b = blockIdx.y;
    double pp = 0.0, dd = 0.0;
    for (int s = blockIdx.x * BS + threadIdx.x; s < g.V; s += gridDim.x * BS) {
#pragma unroll
        for (int e = 0; e < 12; ++e) {
            const size_t i = fidx<INNER>(g.V, nf, s, b, e);
            const float2 p = psi[i], o = out[i];
            const double dx = (double)o.x - p.x, dy = (double)o.y - p.y;
            pp += (double)p.x * p.x + (double)p.y * p.y;
            dd += dx * dx + dy * dy;
        }
    }
    double2 d1 = make_double2(pp, 0.0), d2 = make_double2(dd, 0.0);
    block_reduce2(d1, d2);
    if (threadIdx.x == 0) partial[(size_t)b * gridDim.x + blockIdx.x] = make_double2(d1.x, d2.x);
}

// scale[b] = 1 / (nf |psi_b|^2) (0 for a zero psi_b); loss = (1/nf) sum_b |out_b - psi_b|^2 / |psi_b|^2
__global__ void __launch_bounds__(BS) k_loss_finish(int nf, int nblk, const double2* __restrict__ partial,
                                                    double* __restrict__ scale, double* __restrict__ loss) {
    __shared__ double terms[BS];
    double acc = 0.0;
    for (int b0 = 0; b0 < nf; b0 += BS) {
        const int b = b0 + threadIdx.x;
        double term = 0.0;
        if (b < nf) {
            double pp = 0.0, dd = 0.0;
            for (int k = 0; k < nblk; ++k) {
                pp += partial[(size_t)b * nblk + k].x;
                dd += partial[(size_t)b * nblk + k].y;
            }
            scale[b] = pp > 0.0 ? 1.0 / ((double)nf * pp) : 0.0;
            term = pp > 0.0 ? dd / pp : 0.0;
        }
        terms[threadIdx.x] = term;
        __syncthreads();
        if (threadIdx.x == 0)
            for (int i = 0; i < BS; ++i) acc += terms[i];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss) *loss = acc / nf;
}

// gout = (out - psi) * scale[b]  (gout may be out)
template <bool INNER>
__global__ void __launch_bounds__(BS) k_loss_grad(Geo g, int nf, const float2* out, const float2* __restrict__ psi,
                                                  const double* __restrict__ scale, float2* gout) {
    const long t = (long)blockIdx.x * BS + threadIdx.x;
    if (t >= (long)g.V * nf) return;
    int s, b;
    item_of<INNER>(g, nf, t, s, b);
    const float f = (float)scale[b];
#pragma unroll
    for (int e = 0; e < 12; ++e) {
        const size_t i = fidx<INNER>(g.V, nf, s, b, e);
        const float2 o = out[i], p = psi[i];
        gout[i] = make_float2((o.x - p.x) * f, (o.y - p.y) * f);
    }
}

// ------------------------------------------------------------------ Adam
// Real parameters p (the re and im parts); the gradient of the real loss is
// twice the Wirtinger gradient g.  c1 = 1/(1-b1^t), c2 = 1/(1-b2^t).
__global__ void __launch_bounds__(BS) k_adam(long n, float* __restrict__ p, const float* __restrict__ g,
                                             float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                                             float b2, float eps, float c1, float c2) {
    const long i = (long)blockIdx.x * BS + threadIdx.x;
    if (i >= n) return;
    const float gr = 2.0f * g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gr;
    const float vi = b2 * v[i] + (1.0f - b2) * gr * gr;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

__global__ void __launch_bounds__(BS) k_cast(long n, const double* __restrict__ in, float* __restrict__ out) {
    const long i = (long)blockIdx.x * BS + threadIdx.x;
    if (i < n) out[i] = (float)in[i];
}

unsigned layer_grid(const Geo& g, int nf) { return grid_for((long)g.V * nf, BS); }

}  // namespace

size_t net_T_bytes(const Geo& g) { return (size_t)13 * 9 * g.Vs * sizeof(float2); }

int net_wgrad_chunks(const Geo& g, int nf) {
    const long n = (long)g.V * nf;
    return (int)std::min<long>(512, (n + BS - 1) / BS);
}
size_t net_wgrad_partial_bytes(const Geo& g, int nf) { return (size_t)net_wgrad_chunks(g, nf) * 27 * 16 * 8; }
size_t net_loss_partial_bytes(int nf) { return (size_t)nf * kLossBlocks * sizeof(double2) + (size_t)nf * 8; }

int launch_net_transports(const Geo& g, const double* links, float* T, hipStream_t st) {
    k_transports<<<grid_for(g.V, BS), BS, 0, st>>>(g, reinterpret_cast<const double2*>(links),
                                                   reinterpret_cast<float2*>(T));
    OK_LAUNCH_CHECK("k_transports");
    return OK_SUCCESS;
}

int launch_net_layer(const Geo& g, int nf, bool inner, bool adjoint, const float* A, const float* T,
                     const float* in, float* out, hipStream_t st) {
    const float2* a = reinterpret_cast<const float2*>(A);
    const float2* t = reinterpret_cast<const float2*>(T);
    const float2* i = reinterpret_cast<const float2*>(in);
    float2* o = reinterpret_cast<float2*>(out);
    const unsigned grid = layer_grid(g, nf);
    if (inner) {
        if (adjoint) k_layer<true, true><<<grid, BS, 0, st>>>(g, nf, a, t, i, o);
        else k_layer<true, false><<<grid, BS, 0, st>>>(g, nf, a, t, i, o);
    } else {
        if (adjoint) k_layer<false, true><<<grid, BS, 0, st>>>(g, nf, a, t, i, o);
        else k_layer<false, false><<<grid, BS, 0, st>>>(g, nf, a, t, i, o);
    }
    OK_LAUNCH_CHECK("k_layer");
    return OK_SUCCESS;
}

int launch_net_wgrad(const Geo& g, int nf, bool inner, const float* T, const float* gout, const float* in,
                     float* partial, float* gA, hipStream_t st) {
    const int nch = net_wgrad_chunks(g, nf);
    const float2* t = reinterpret_cast<const float2*>(T);
    const float2* go = reinterpret_cast<const float2*>(gout);
    const float2* i = reinterpret_cast<const float2*>(in);
    float2* p = reinterpret_cast<float2*>(partial);
    const unsigned grid = nch * 27;
    if (inner) k_wgrad<true><<<grid, BS, 0, st>>>(g, nf, nch, t, go, i, p);
    else k_wgrad<false><<<grid, BS, 0, st>>>(g, nf, nch, t, go, i, p);
    OK_LAUNCH_CHECK("k_wgrad");
    k_wgrad_finish<<<grid_for(27 * 16 * 64, BS), BS, 0, st>>>(nch, p, reinterpret_cast<float2*>(gA));
    OK_LAUNCH_CHECK("k_wgrad_finish");
    return OK_SUCCESS;
}

int launch_net_loss_grad(const Geo& g, int nf, bool inner, const float* out, const float* psi, float* gout,
                         double* loss, void* scratch, hipStream_t st) {
    double2* partial = reinterpret_cast<double2*>(scratch);
    double* scale = reinterpret_cast<double*>(partial + (size_t)nf * kLossBlocks);
    const float2* o = reinterpret_cast<const float2*>(out);
    const float2* p = reinterpret_cast<const float2*>(psi);
    const dim3 grid(kLossBlocks, nf);
    if (inner) k_loss_norms<true><<<grid, BS, 0, st>>>(g, nf, o, p, partial);
    else k_loss_norms<false><<<grid, BS, 0, st>>>(g, nf, o, p, partial);
    OK_LAUNCH_CHECK("k_loss_norms");
    k_loss_finish<<<1, BS, 0, st>>>(nf, kLossBlocks, partial, scale, loss);
    OK_LAUNCH_CHECK("k_loss_finish");
    float2* go = reinterpret_cast<float2*>(gout);
    if (inner) k_loss_grad<true><<<layer_grid(g, nf), BS, 0, st>>>(g, nf, o, p, scale, go);
    else k_loss_grad<false><<<layer_grid(g, nf), BS, 0, st>>>(g, nf, o, p, scale, go);
    OK_LAUNCH_CHECK("k_loss_grad");
    return OK_SUCCESS;
}

int launch_cast(long n, const double* in, float* out, hipStream_t st) {
    k_cast<<<grid_for(n, BS), BS, 0, st>>>(n, in, out);
    OK_LAUNCH_CHECK("k_cast");
    return OK_SUCCESS;
}

int launch_adam(long n, float* p, const float* g, float* m, float* v, const ok_adam_cfg& c, int step,
                hipStream_t st) {
    const double c1 = 1.0 / (1.0 - std::pow(c.beta1, step)), c2 = 1.0 / (1.0 - std::pow(c.beta2, step));
    k_adam<<<grid_for(n, BS), BS, 0, st>>>(n, p, g, m, v, (float)c.lr, (float)c.beta1, (float)c.beta2,
                                           (float)c.eps, (float)c1, (float)c2);
    OK_LAUNCH_CHECK("k_adam");
    return OK_SUCCESS;
}

}  // namespace okinv
