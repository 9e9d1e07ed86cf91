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
//
// With OK_LAYOUT_SIGMA (FP64 or FP32) each forward block is kept as the colour matrices of
// its Pauli decomposition, 46 per site (listed below), and every block is formed where
// it is used.  Matrix mi of site s, entry e = 3a + b (row a, column b), is at
//
//     FP64:  double2 cell (mi * 9 + e) * Vs + s
//     FP32:  e < 8: half e % 2 of float4 cell (mi * 4 + e / 2) * Vs + s;
//            e = 8: float2 cell mi * Vs + s of a second region after the 46 * 4 float4 planes
//
// so that a wavefront of consecutive sites reads each piece of a matrix contiguously.
//
// With OK_LAYOUT_SAVED only the 14 blocks of the forward offsets (k = 0, +mu,
// +2i, +i+j, +i-j: the saved set of Eq. FinalForm) are stored, plane-major as
// above with the saved index ks in place of k; a backward block is formed
// where it is used from the forward block of the neighbour it points to,
// W_{-d,x} = gamma5 W_{+d,x-d}^dag gamma5 (Eq. conjugate).
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

// layout codes of the kernels: plane (27 blocks), site-major, saved set (14 blocks, plane)
constexpr int LAY_PLANE = 0, LAY_SITE = 1, LAY_SAVED = 2;
constexpr int kSaved = 14;
// forward offset of saved index ks, and saved index of offset k (-1 for a backward offset)
__host__ __device__ constexpr int saved_k(int ks) {
    return ks <= 4 ? ks : ks <= 7 ? ks + 4 : ks <= 10 ? ks + 7 : ks + 10;
}
__host__ __device__ constexpr int saved_index(int k) {
    return k <= 4 ? k : k <= 8 ? -1 : k <= 11 ? k - 4 : k <= 14 ? -1 : k <= 17 ? k - 7 : k <= 20 ? -1
         : k <= 23 ? k - 10 : -1;
}
static_assert(saved_k(13) == 23 && saved_index(23) == 13 && saved_index(9) == 5 && saved_index(15) == 8 &&
              saved_index(26) == -1 && saved_k(5) == 9, "saved set");

// Pauli-decomposed forward blocks (layout LAY_SIGMA): W = [[A, B], [C, D]] in 2x2 spin blocks,
// each a sum_n sigma_n (x) X_n over n = 0..3 (sigma_0 = 1).  Colour matrices kept per site:
//   W0      [[H1, H2], [-H2, H1]]:  (X1_m - i X2_m) / 2, then (X1_m + i X2_m) / 2, m = 1..3  (mi 0..5)
//   W+_i    [[H1, H2], [H2, H1]]:   P_n = (X1_n + X2_n) / 2, then Q_n = (X1_n - X2_n) / 2    (mi 6 + 8i ..)
//   W+_4    [[0, H1], [H1, H2]]:    X1_1..3, then X2_0 (= -U_4)                              (mi 30..33)
//   W++_ii  [[H1, H2], [H2, H1]]:   X1_0, X2_i                                               (mi 34 + 2i ..)
//   W++_ij  [[0, H1], [H1, 0]]:     X1_i (H1 = (sigma_i + sigma_j) X1_i)                     (mi 40 + p)
//   W+-_ij  [[0, H1], [H1, 0]]:     X1_i (H1 = (sigma_i - sigma_j) X1_i)                     (mi 43 + p)
// (X1, X2: the components of H1, H2; p = 0, 1, 2 for (i, j) = (x, y), (x, z), (y, z).)
constexpr int LAY_SIGMA = 3;
constexpr int kSigma = 46;
constexpr int SG_W0 = 0, SG_WI = 6, SG_W4 = 30, SG_WII = 34, SG_WIJ = 40, SG_WIMJ = 43;

inline int layout_of(int prec) {
    return (prec & OK_LAYOUT_SITE) ? LAY_SITE : (prec & OK_LAYOUT_SAVED) ? LAY_SAVED
         : (prec & OK_LAYOUT_SIGMA) ? LAY_SIGMA : LAY_PLANE;
}

// byte offset of entry e of colour matrix mi at site s (LAY_SIGMA; P = OK_F64 or OK_F32)
template <int P>
__host__ __device__ __forceinline__ size_t sigma_off(int Vs, int mi, int e, int s) {
    if constexpr (P == OK_F64) return ((size_t)(mi * 9 + e) * Vs + s) * 16;
    if (e < 8) return ((size_t)(mi * 4 + e / 2) * Vs + s) * 16 + (size_t)(e & 1) * 8;
    return (size_t)kSigma * 4 * Vs * 16 + ((size_t)mi * Vs + s) * 8;
}

__host__ __device__ __forceinline__ size_t w_cell(int layout, int Vs, int ch, int k, int j, int s) {
    if (layout == LAY_SITE) return ((size_t)s * kW + k) * ch + j;
    if (layout == LAY_SAVED) k = saved_index(k);
    return ((size_t)(k * ch + j)) * Vs + s;
}

inline size_t w_bytes(int prec, int Vs, int layout = LAY_PLANE) {
    size_t es = prec == OK_F64 ? 16 : prec == OK_F32 ? 8 : 4;
    if (layout == LAY_SIGMA) return (size_t)kSigma * 9 * es * (size_t)Vs;
    return (size_t)(layout == LAY_SAVED ? kSaved : kW) * kWE * es * (size_t)Vs;
}

// Store one row (12 complex, FP64 values) of block k at site s.
template <int P>
__device__ __forceinline__ void w_store_row(void* W, int Vs, int layout, int k, int row, int s, const c128 v[12]) {
    uint4* base = reinterpret_cast<uint4*>(W);
    constexpr int per = WL<P>::per, ch = WL<P>::chunks;
    if constexpr (P == OK_F32) {
        if (layout == LAY_SITE) {   // column-major block: entry (row, col) at 12*col + row
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
    if (P == OK_F32 && layout == LAY_SITE) e = 12 * (e % 12) + e / 12;   // column-major block
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
