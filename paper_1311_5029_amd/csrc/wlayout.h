// Private layout of the W buffer (versioned by OKINV_ABI_VERSION).
//
// Every block W_{k,x} (12x12 complex, row-major, entry e = 12*row + col) is cut
// into 16-byte chunks of consecutive entries: 1 complex in FP64, 2 in FP32,
// 4 in BF16 (each complex a (re, im) pair of bf16).  Chunk j of block k of
// every site forms one plane of Vs 16-byte cells, site-fastest:
//
//     cell(k, j, s) = base + ((k * chunks_per_block + j) * Vs + s) * 16 bytes
//
// so a wavefront of consecutive sites reads or writes 1 KiB contiguously
// (plane layout, the default: best for one right-hand side).
//
// With OK_LAYOUT_SITE the 27 blocks of a site are contiguous instead:
//
//     cell(k, j, s) = base + ((s * 27 + k) * chunks_per_block + j) * 16 bytes
//
// which the multi-right-hand-side MFMA kernel streams one block at a time; in
// that layout FP32 blocks are stored column-major (entry 12*col + row), the
// order in which the lanes of the FP32 MFMA read their A operands, and BF16
// blocks row-major (the BF16 MFMA reads 4 consecutive columns per lane).
#pragma once

#include "common.h"

namespace okinv {

template <int P> struct WL;
template <> struct WL<OK_F64> {
    static constexpr int per = 1;   // complex per 16-byte chunk
    static constexpr int chunks = 144;
    static constexpr int esize = 16;
};
template <> struct WL<OK_F32> {
    static constexpr int per = 2;
    static constexpr int chunks = 72;
    static constexpr int esize = 8;
};
template <> struct WL<OK_BF16> {
    static constexpr int per = 4;
    static constexpr int chunks = 36;
    static constexpr int esize = 4;
};

__host__ __device__ __forceinline__ size_t w_cell(int layout, int Vs, int ch, int k, int j, int s) {
    return layout ? ((size_t)s * kW + k) * ch + j : ((size_t)(k * ch + j)) * Vs + s;
}

inline size_t w_bytes(int prec, int Vs) {
    size_t es = prec == OK_F64 ? 16 : prec == OK_F32 ? 8 : 4;
    return (size_t)kW * kWE * es * (size_t)Vs;
}

// Store one row (12 complex, FP64 values) of block k at site s.
template <int P>
__device__ __forceinline__ void w_store_row(void* W, int Vs, int layout, int k, int row, int s, const c128 v[12]) {
    uint4* base = reinterpret_cast<uint4*>(W);
    constexpr int per = WL<P>::per, ch = WL<P>::chunks;
    if constexpr (P == OK_F32) {
        if (layout) {   // column-major block: entry (row, col) at 12*col + row
            float2* b = reinterpret_cast<float2*>(base + w_cell(layout, Vs, ch, k, 0, s));
#pragma unroll
            for (int c = 0; c < 12; ++c) b[12 * c + row] = make_float2((float)v[c].re, (float)v[c].im);
            return;
        }
    }
    const int j0 = row * 12 / per;
#pragma unroll
    for (int q = 0; q < 12 / per; ++q) {
        size_t cell = w_cell(layout, Vs, ch, k, j0 + q, s);
        if constexpr (P == OK_F64) {
            double2 d = make_double2(v[q].re, v[q].im);
            reinterpret_cast<double2*>(base)[cell] = d;
        } else if constexpr (P == OK_F32) {
            float4 f = make_float4((float)v[2 * q].re, (float)v[2 * q].im,
                                   (float)v[2 * q + 1].re, (float)v[2 * q + 1].im);
            reinterpret_cast<float4*>(base)[cell] = f;
        } else {
            uint32_t w[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                uint32_t lo = f32_to_bf16((float)v[4 * q + u].re);
                uint32_t hi = f32_to_bf16((float)v[4 * q + u].im);
                w[u] = lo | (hi << 16);
            }
            base[cell] = make_uint4(w[0], w[1], w[2], w[3]);
        }
    }
}

// Load entry e (0..143) of block k at site s as FP64 (exact for every storage type).
template <int P>
__device__ __forceinline__ c128 w_load_entry(const void* W, int Vs, int layout, int k, int e, int s) {
    constexpr int per = WL<P>::per, ch = WL<P>::chunks;
    if (P == OK_F32 && layout) e = 12 * (e % 12) + e / 12;   // column-major block
    size_t cell = w_cell(layout, Vs, ch, k, e / per, s);
    if constexpr (P == OK_F64) {
        double2 d = reinterpret_cast<const double2*>(W)[cell];
        return c128{d.x, d.y};
    } else if constexpr (P == OK_F32) {
        const float2* f = reinterpret_cast<const float2*>(reinterpret_cast<const float4*>(W) + cell);
        float2 v = f[e % 2];
        return c128{(double)v.x, (double)v.y};
    } else {
        const uint32_t* u = reinterpret_cast<const uint32_t*>(reinterpret_cast<const uint4*>(W) + cell);
        uint32_t w = u[e % 4];
        return c128{(double)bf16_to_f32(w & 0xffffu), (double)bf16_to_f32(w >> 16)};
    }
}

}  // namespace okinv
