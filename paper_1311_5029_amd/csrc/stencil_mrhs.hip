// M applied to up to 16 right-hand sides at once on the matrix cores (MFMA).
//
// Per site and offset the 12x12 complex block W_{k,x} multiplies the 12x12
// complex matrix of neighbour spinors (12 components x 12 right-hand sides):
// a small complex GEMM whose W operand is streamed from HBM once for all
// right-hand sides.  A workgroup (4 wavefronts) owns a tile of 32 consecutive
// sites; for every offset k it copies the tile's W_k (32 x 1152 B FP32, 32 x
// 576 B BF16) from the plane layout into LDS (coalesced 512-byte runs, double
// buffered), and each wavefront runs the GEMMs of 8 sites with operands read
// from LDS (W) and L2 (neighbour spinors).
//
// FP32 W (v_mfma_f32_16x16x4f32, 12 instructions per site and offset; the site-major kernel
// below forms the complex product from three real ones, 9 instructions):
//   C_r += A_r B_r - A_i B_i,  C_i += A_r B_i + A_i B_r,
//   M index = output component (12 of 16), N = right-hand side (nrhs of 16),
//   K step q, lane group g  <->  input component 3g + q.
// BF16 W (v_mfma_f32_16x16x32_bf16, 4 instructions per site and offset):
//   real embedding with interleaved rows: output row 2c+p is the real (p = 0)
//   or imaginary (p = 1) part of component c; K index 8g + 2m + p' is part p'
//   of input component 4g + m.  The A operand is a BF16 chunk of W with its
//   imaginary halves negated (p = 0) or its halves swapped (p = 1); the FP32
//   spinors are split into bf16 hi + lo and both are multiplied, so the
//   result equals BF16 W times the FP32 spinor up to 2^-16 relative.
// Accumulation is FP32 in both cases.
#include "common.h"
#include "kernels.h"
#include "wlayout.h"

namespace okinv {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));

constexpr int TS = 32;          // sites per tile (workgroup)
constexpr int NWAVE = 4;
constexpr int SPW = TS / NWAVE;  // sites per wavefront
constexpr int BS = 64 * NWAVE;

template <int P> struct MR;
template <> struct MR<OK_F32> {
    static constexpr int CH = 72;    // 16-byte chunks per block
    static constexpr int CHP = 73;   // padded LDS stride per site (bank spread)
};
template <> struct MR<OK_BF16> {
    static constexpr int CH = 36;
    static constexpr int CHP = 37;
};

template <int P>
__global__ void __launch_bounds__(BS, 2) k_apply_mrhs(Geo g, const uint4* __restrict__ W,
                                                      const float* __restrict__ psi, float* __restrict__ out,
                                                      float mhat, int nrhs) {
    constexpr int CH = MR<P>::CH, CHP = MR<P>::CHP;
    constexpr int NCELL = TS * CH;
    constexpr int NPT = (NCELL + BS - 1) / BS;
    __shared__ uint4 sW[2][TS * CHP];

    const int ntiles = (g.V + TS - 1) / TS;
    const int tile = xcd_tile(blockIdx.x, ntiles);
    const int s0 = tile * TS;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l16 = lane & 15, grp = lane >> 4;

    // coordinates of this wavefront's sites
    int cx[SPW], cy[SPW], cz[SPW], ct[SPW];
#pragma unroll
    for (int u = 0; u < SPW; ++u) {
        const int s = min(s0 + wave * SPW + u, g.V - 1);
        site_coords(g, s, cx[u], cy[u], cz[u], ct[u]);
    }

    uint4 stage[NPT];
    auto fetch = [&](int k) {
#pragma unroll
        for (int n = 0; n < NPT; ++n) {
            const int cell = threadIdx.x + BS * n;
            const int ch = cell / TS, st = cell % TS;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (cell < NCELL && s0 + st < g.V) v = ld_stream(W + ((size_t)(k * CH + ch)) * g.Vs + s0 + st);
            stage[n] = v;
        }
    };
    auto commit = [&](int buf) {
#pragma unroll
        for (int n = 0; n < NPT; ++n) {
            const int cell = threadIdx.x + BS * n;
            if (cell < NCELL) sW[buf][(cell % TS) * CHP + cell / TS] = stage[n];
        }
    };

    v4f acc0[SPW], acc1[SPW];
#pragma unroll
    for (int u = 0; u < SPW; ++u) {
        acc0[u] = v4f{0.f, 0.f, 0.f, 0.f};
        acc1[u] = v4f{0.f, 0.f, 0.f, 0.f};
    }
    const bool jlive = l16 < nrhs;
    const size_t rstride = (size_t)g.V * 24;    // floats per right-hand side

    fetch(0);
    commit(0);
    __syncthreads();
#pragma unroll 1
    for (int k = 0; k < kW; ++k) {
        const int buf = k & 1;
        if (k + 1 < kW) fetch(k + 1);
        const int dx = off_d(k, 0), dy = off_d(k, 1), dz = off_d(k, 2), dt = off_d(k, 3);
        const uint4* wt = &sW[buf][wave * SPW * CHP];
#pragma unroll
        for (int u = 0; u < SPW; ++u) {
            const int nb = neighbour(g, cx[u], cy[u], cz[u], ct[u], dx, dy, dz, dt);
            const float* pn = psi + (size_t)l16 * rstride + (size_t)nb * 24;
            if constexpr (P == OK_F32) {
                // B: components 3g .. 3g+2 of right-hand side l16; A: row l16, columns 3g .. 3g+2
                float2 b[3], a[3];
                const float2* pb = reinterpret_cast<const float2*>(pn) + 3 * grp;
                const float2* pa = reinterpret_cast<const float2*>(wt + u * CHP) + l16 * 12 + 3 * grp;
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    b[q] = jlive ? pb[q] : make_float2(0.f, 0.f);
                    a[q] = l16 < 12 ? pa[q] : make_float2(0.f, 0.f);
                }
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    acc0[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[q].x, b[q].x, acc0[u], 0, 0, 0);
                    acc1[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[q].x, b[q].y, acc1[u], 0, 0, 0);
                    acc0[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(-a[q].y, b[q].y, acc0[u], 0, 0, 0);
                    acc1[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[q].y, b[q].x, acc1[u], 0, 0, 0);
                }
            } else {
                // B: (re, im) of components 4g .. 4g+3 of right-hand side l16, split into bf16 hi + lo
                v8bf bhi, blo;
                if (jlive && grp < 3) {
                    const float4* pb = reinterpret_cast<const float4*>(pn) + 2 * grp;
                    const float4 x0 = pb[0], x1 = pb[1];
                    const float xs[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const __bf16 h = (__bf16)xs[e];
                        bhi[e] = h;
                        blo[e] = (__bf16)(xs[e] - (float)h);
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        bhi[e] = (__bf16)0.0f;
                        blo[e] = (__bf16)0.0f;
                    }
                }
                // A: output row 2c + p; W chunk (row c, columns 4g .. 4g+3)
                const int p = l16 & 1;
                v4u w0 = v4u{0u, 0u, 0u, 0u}, w1 = v4u{0u, 0u, 0u, 0u};
                if (grp < 3) {
                    const uint4 c0 = wt[u * CHP + (l16 >> 1) * 3 + grp];
                    w0 = v4u{c0.x, c0.y, c0.z, c0.w};
                    if (l16 < 8) {
                        const uint4 c1 = wt[u * CHP + (8 + (l16 >> 1)) * 3 + grp];
                        w1 = v4u{c1.x, c1.y, c1.z, c1.w};
                    }
                }
                if (p == 0) {   // [re, -im]
                    w0 ^= 0x80000000u;
                    w1 ^= 0x80000000u;
                } else {        // [im, re]
                    w0 = (w0 >> 16) | (w0 << 16);
                    w1 = (w1 >> 16) | (w1 << 16);
                }
                if (grp == 3) {
                    w0 = v4u{0u, 0u, 0u, 0u};
                    w1 = v4u{0u, 0u, 0u, 0u};
                }
                if (l16 >= 8) w1 = v4u{0u, 0u, 0u, 0u};
                const v8bf a0 = __builtin_bit_cast(v8bf, w0), a1 = __builtin_bit_cast(v8bf, w1);
                acc0[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, bhi, acc0[u], 0, 0, 0);
                acc1[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bhi, acc1[u], 0, 0, 0);
                acc0[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, blo, acc0[u], 0, 0, 0);
                acc1[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, blo, acc1[u], 0, 0, 0);
            }
        }
        if (k + 1 < kW) {
            commit(buf ^ 1);
            __syncthreads();
        }
    }

    // epilogue: out = mhat psi + acc for the live right-hand side of this lane
    if (!jlive) return;
#pragma unroll
    for (int u = 0; u < SPW; ++u) {
        const int s = s0 + wave * SPW + u;
        if (s >= g.V) continue;
        const size_t base = (size_t)l16 * rstride + (size_t)s * 24;
        if constexpr (P == OK_F32) {
            if (grp < 3) {   // rows 4g .. 4g+3 = components 4g .. 4g+3
                const float4* pc = reinterpret_cast<const float4*>(psi + base) + 2 * grp;
                float4* po = reinterpret_cast<float4*>(out + base) + 2 * grp;
                const float4 c0 = pc[0], c1 = pc[1];
                po[0] = make_float4(mhat * c0.x + acc0[u][0], mhat * c0.y + acc1[u][0],
                                    mhat * c0.z + acc0[u][1], mhat * c0.w + acc1[u][1]);
                po[1] = make_float4(mhat * c1.x + acc0[u][2], mhat * c1.y + acc1[u][2],
                                    mhat * c1.z + acc0[u][3], mhat * c1.w + acc1[u][3]);
            }
        } else {
            // tile 0 rows 4g .. 4g+3 = components 2g, 2g+1 as (re, im); tile 1 rows 16 + 4g .. = components 8 + 2g ..
            {
                const float4 c0 = reinterpret_cast<const float4*>(psi + base)[grp];
                reinterpret_cast<float4*>(out + base)[grp] =
                    make_float4(mhat * c0.x + acc0[u][0], mhat * c0.y + acc0[u][1],
                                mhat * c0.z + acc0[u][2], mhat * c0.w + acc0[u][3]);
            }
            if (grp < 2) {
                const float4 c1 = reinterpret_cast<const float4*>(psi + base)[4 + grp];
                reinterpret_cast<float4*>(out + base)[4 + grp] =
                    make_float4(mhat * c1.x + acc1[u][0], mhat * c1.y + acc1[u][1],
                                mhat * c1.z + acc1[u][2], mhat * c1.w + acc1[u][3]);
            }
        }
    }
}

// Site-major W (OK_LAYOUT_SITE): every wavefront walks its own sites, and for
// each site the 27 blocks it streams are one contiguous 31 KB (FP32) or 15.5 KB
// (BF16) run, read straight into the MFMA operand registers (no LDS, no
// barriers).  The 27 offsets are unrolled so the loads of later offsets are
// issued while earlier ones are being multiplied.  In this kernel the K slot
// of lane group g in step q is input component 4q + g (FP32; the block is
// stored column-major so a step's A operand is one contiguous 384-byte run).
//
// Spinor layout SL = 0: [nrhs][V][12] complex (the ABI default);
// SL = 1 (OK_SPINOR_RHS_INNER): [V][12][nrhs] complex, so the 12 right-hand
// sides of one component are adjacent and a step's B operand is contiguous.
#ifndef OKINV_SITE_SPW
#define OKINV_SITE_SPW 2
#endif
constexpr int SPW_SITE = OKINV_SITE_SPW;     // sites per wavefront

template <int SL>
__device__ __forceinline__ size_t sp_index(int nrhs, size_t V, int j, int s, int c) {
    return SL ? ((size_t)s * 12 + c) * nrhs + j : ((size_t)j * V + s) * 12 + c;
}

// Operands of one (site, offset) step, loaded ahead of use.
template <int P> struct Ops;
template <> struct Ops<OK_F32> {
    float2 a[3], b[3];
};
template <> struct Ops<OK_BF16> {
    uint4 w0, w1;
    float2 x[4];
};

// Per-lane constant parts of the operand addresses.  Padding rows (i >= 12)
// and columns (j >= nrhs) only feed output rows/columns that are discarded, so
// their lanes read a valid in-block address instead of being zeroed.
template <int P, int SL> struct LaneOff {
    int a[3], a1, b[4];
    bool wl, bl;   // FP32: this lane's W row / right-hand side is live (otherwise its operand is zero)
};

template <int P, int SL>
__device__ __forceinline__ LaneOff<P, SL> lane_offsets(int l16, int grp, int nrhs, size_t V) {
    LaneOff<P, SL> o;
    const int j = l16 < nrhs ? l16 : nrhs - 1;
    o.wl = l16 < 12;
    o.bl = l16 < nrhs;
    if constexpr (P == OK_F32) {
        const int i = l16 < 12 ? l16 : l16 - 4;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int c = 4 * q + grp;
            o.a[q] = 12 * c + i;                                   // float2 index in the block
            o.b[q] = SL ? c * nrhs + j : (int)0;                   // float2 index in the site (SL = 1)
        }
        o.b[3] = 0;
        o.a1 = 0;
    } else {
        const int g3 = grp < 3 ? grp : 2;
        o.a[0] = (l16 >> 1) * 3 + g3;                              // uint4 index in the block
        o.a1 = (8 + ((l16 & 7) >> 1)) * 3 + g3;
        o.a[1] = o.a[2] = 0;
#pragma unroll
        for (int m = 0; m < 4; ++m) o.b[m] = SL ? (4 * g3 + m) * nrhs + j : 4 * g3 + m;
    }
    return o;
}

template <int P, int SL>
__device__ __forceinline__ void load_ops(Ops<P>& o, const uint4* __restrict__ wk, const float2* __restrict__ sp,
                                         const LaneOff<P, SL>& lo, int l16, int grp) {
    // wk: this block; sp: this neighbour's spinor (SL = 1: its [12][nrhs] run; SL = 0: its
    // 12 components of right-hand side l16)
    if constexpr (P == OK_F32) {
        const float2* pa = reinterpret_cast<const float2*>(wk);
#pragma unroll
        for (int q = 0; q < 3; ++q) {   // padding rows and columns load nothing
            o.a[q] = lo.wl ? ld_stream(pa + lo.a[q]) : make_float2(0.f, 0.f);
            o.b[q] = lo.bl ? (SL ? sp[lo.b[q]] : sp[4 * q + grp]) : make_float2(0.f, 0.f);
        }
    } else {
#pragma unroll
        for (int m = 0; m < 4; ++m) o.x[m] = sp[lo.b[m]];
        o.w0 = ld_stream(wk + lo.a[0]);
        o.w1 = ld_stream(wk + lo.a1);
    }
}

template <int P>
__device__ __forceinline__ void mma_ops(const Ops<P>& o, int l16, int grp, v4f& acc0, v4f& acc1, v4f& acc2) {
    if constexpr (P == OK_F32) {
        // three real products per complex product (Gauss): acc0 += Re a Re b, acc1 += Im a Im b,
        // acc2 += (Re a + Im a)(Re b + Im b); Re = acc0 - acc1, Im = acc2 - acc0 - acc1 at the end
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(o.a[q].x, o.b[q].x, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(o.a[q].y, o.b[q].y, acc1, 0, 0, 0);
            acc2 = __builtin_amdgcn_mfma_f32_16x16x4f32(o.a[q].x + o.a[q].y, o.b[q].x + o.b[q].y, acc2, 0, 0, 0);
        }
    } else {
        v8bf bhi, blo;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const float xs[2] = {o.x[m].x, o.x[m].y};
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                const __bf16 h = (__bf16)xs[p];
                bhi[2 * m + p] = h;
                blo[2 * m + p] = (__bf16)(xs[p] - (float)h);
            }
        }
        v4u w0 = v4u{o.w0.x, o.w0.y, o.w0.z, o.w0.w}, w1 = v4u{o.w1.x, o.w1.y, o.w1.z, o.w1.w};
        if ((l16 & 1) == 0) {   // output row 2c: [re, -im]
            w0 ^= 0x80000000u;
            w1 ^= 0x80000000u;
        } else {                // output row 2c + 1: [im, re]
            w0 = (w0 >> 16) | (w0 << 16);
            w1 = (w1 >> 16) | (w1 << 16);
        }
        // K slots 24..31 (lane group 3) are padding: zero one operand
        if (grp == 3) {
            w0 = v4u{0u, 0u, 0u, 0u};
            w1 = v4u{0u, 0u, 0u, 0u};
        }
        const v8bf a0 = __builtin_bit_cast(v8bf, w0), a1 = __builtin_bit_cast(v8bf, w1);
        acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, bhi, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bhi, acc1, 0, 0, 0);
        acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, blo, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, blo, acc1, 0, 0, 0);
    }
}

// Prefetch depth: operands of DEPTH offsets are in flight ahead of the MFMAs.
#ifndef OKINV_SITE_DEPTH
#define OKINV_SITE_DEPTH 4
#endif
constexpr int DEPTH = OKINV_SITE_DEPTH;

template <int P, int SL>
__global__ void __launch_bounds__(256) k_apply_site(Geo g, const uint4* __restrict__ W,
                                                    const float* __restrict__ psi, float* __restrict__ out,
                                                    float mhat, int nrhs) {
    constexpr int CH = MR<P>::CH;
    const int lane = threadIdx.x & 63;
    const int blk = xcd_tile(blockIdx.x, gridDim.x);
    // the wavefront index is uniform: keep it (and every site index derived from it) scalar
    const int wave = __builtin_amdgcn_readfirstlane(blk * 4 + (threadIdx.x >> 6));
    const int l16 = lane & 15, grp = lane >> 4;
    const bool jlive = l16 < nrhs;
    const float2* ps = reinterpret_cast<const float2*>(psi);
    float2* po = reinterpret_cast<float2*>(out);
    const size_t V = g.V;
    const LaneOff<P, SL> lo = lane_offsets<P, SL>(l16, grp, nrhs, V);
    const int jc = l16 < nrhs ? l16 : nrhs - 1;
    // spinor of site n as seen by this lane: SL = 1 the [12][nrhs] run, SL = 0 right-hand side jc
    auto spin = [&](int n) -> const float2* {
        return SL ? ps + (size_t)n * 12 * nrhs : ps + ((size_t)jc * V + n) * 12;
    };

#pragma unroll 1
    for (int u = 0; u < SPW_SITE; ++u) {
        const int s = wave * SPW_SITE + u;
        if (s >= g.V) return;
        int x, y, z, t;
        site_coords(g, s, x, y, z, t);
        const uint4* ws = W + (size_t)s * kW * CH;
        Ops<P> ring[DEPTH];
#pragma unroll
        for (int k = 0; k < DEPTH; ++k) {
            const int nb = neighbour(g, x, y, z, t, off_d(k, 0), off_d(k, 1), off_d(k, 2), off_d(k, 3));
            load_ops<P, SL>(ring[k], ws + k * CH, spin(nb), lo, l16, grp);
        }
        v4f acc0 = v4f{0.f, 0.f, 0.f, 0.f}, acc1 = v4f{0.f, 0.f, 0.f, 0.f}, acc2 = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < kW; ++k) {
            const Ops<P> cur = ring[k % DEPTH];
            if (k + DEPTH < kW) {
                const int kn = k + DEPTH;
                const int nb = neighbour(g, x, y, z, t, off_d(kn, 0), off_d(kn, 1), off_d(kn, 2), off_d(kn, 3));
                load_ops<P, SL>(ring[k % DEPTH], ws + kn * CH, spin(nb), lo, l16, grp);
            }
            mma_ops<P>(cur, l16, grp, acc0, acc1, acc2);
        }
        if (!jlive) continue;
        // out = mhat psi + acc
        if constexpr (P == OK_F32) {
            if (grp < 3) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const size_t i = sp_index<SL>(nrhs, V, l16, s, 4 * grp + r);
                    const float2 c = ps[i];
                    const float re = acc0[r] - acc1[r], im = acc2[r] - acc0[r] - acc1[r];
                    po[i] = make_float2(mhat * c.x + re, mhat * c.y + im);
                }
            }
        } else {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const size_t i = sp_index<SL>(nrhs, V, l16, s, 2 * grp + h);
                const float2 c = ps[i];
                po[i] = make_float2(mhat * c.x + acc0[2 * h], mhat * c.y + acc0[2 * h + 1]);
            }
            if (grp < 2) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const size_t i = sp_index<SL>(nrhs, V, l16, s, 8 + 2 * grp + h);
                    const float2 c = ps[i];
                    po[i] = make_float2(mhat * c.x + acc1[2 * h], mhat * c.y + acc1[2 * h + 1]);
                }
            }
        }
    }
}

}  // namespace

int launch_apply_site(const Geo& g, const void* W, int Wprec, const float* psi, float* out, double mhat,
                      int nrhs, int rhs_inner, hipStream_t st) {
    const int nblk = (g.V + 4 * SPW_SITE - 1) / (4 * SPW_SITE);
    const uint4* w = reinterpret_cast<const uint4*>(W);
    if (rhs_inner) {
        if (nrhs > 16) {
            set_error("right-hand-side-inner spinors support at most 16 right-hand sides");
            return OK_EINVAL;
        }
        if (Wprec == OK_F32)
            k_apply_site<OK_F32, 1><<<nblk, 256, 0, st>>>(g, w, psi, out, (float)mhat, nrhs);
        else
            k_apply_site<OK_BF16, 1><<<nblk, 256, 0, st>>>(g, w, psi, out, (float)mhat, nrhs);
        OK_LAUNCH_CHECK("k_apply_site");
        return OK_SUCCESS;
    }
    for (int r0 = 0; r0 < nrhs; r0 += 16) {
        const int nr = min(16, nrhs - r0);
        const float* in = psi + (size_t)r0 * g.V * 24;
        float* o = out + (size_t)r0 * g.V * 24;
        if (Wprec == OK_F32)
            k_apply_site<OK_F32, 0><<<nblk, 256, 0, st>>>(g, w, in, o, (float)mhat, nr);
        else
            k_apply_site<OK_BF16, 0><<<nblk, 256, 0, st>>>(g, w, in, o, (float)mhat, nr);
        OK_LAUNCH_CHECK("k_apply_site");
    }
    return OK_SUCCESS;
}

int launch_apply_mrhs(const Geo& g, const void* W, int Wprec, const float* psi, float* out, double mhat,
                      int nrhs, hipStream_t st) {
    const int ntiles = (g.V + TS - 1) / TS;
    for (int r0 = 0; r0 < nrhs; r0 += 16) {
        const int nr = min(16, nrhs - r0);
        const float* in = psi + (size_t)r0 * g.V * 24;
        float* o = out + (size_t)r0 * g.V * 24;
        if (Wprec == OK_F32)
            k_apply_mrhs<OK_F32><<<ntiles, BS, 0, st>>>(g, reinterpret_cast<const uint4*>(W), in, o, (float)mhat, nr);
        else
            k_apply_mrhs<OK_BF16><<<ntiles, BS, 0, st>>>(g, reinterpret_cast<const uint4*>(W), in, o, (float)mhat, nr);
        OK_LAUNCH_CHECK("k_apply_mrhs");
    }
    return OK_SUCCESS;
}

}  // namespace okinv
