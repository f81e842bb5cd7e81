// 16-point DFTs on the matrix cores (gfx950 MFMA) with split-BF16 operands.
//
// For 32 butterflies at a time, the complex 16-point DFT y = F a with
// F[k][n] = exp(S 2 pi i k n / 16) is the real 32 x 32 by 32 x 32 product
//   [Re y]   [ C  -S' ] [Re a]
//   [Im y] = [ S'  C  ] [Im a],   C = cos(2 pi k n/16), S' = S sin(2 pi k n/16),
// evaluated with v_mfma_f32_32x32x16_bf16 (FP32 accumulation).  BF16 keeps 8
// significant bits, so each FP32 operand x is split into NTERM BF16 terms
// x = t0 + t1 (+ t2) + residual, t_i = RNE(x - t0 - ... - t_{i-1}), and the
// product is the sum of the term products up to total order NTERM - 1
// (2 terms: t0 t0 + t0 t1 + t1 t0; 3 terms: adds t0 t2, t2 t0, t1 t1),
// smallest first.  Relative error per product about 2^-16 (2 terms) or
// 2^-24 (3 terms).
//
// Operand layout of v_mfma_f32_32x32x16_bf16 in a 64-lane wave (h = lane/32):
//   A (32 x 16): lane holds A[lane % 32][8h + j], j = 0..7
//   B (16 x 32): lane holds B[8h + j][lane % 32]
//   D (32 x 32): lane holds D[8 (v/4) + 4h + v%4][lane % 32], v = 0..15
// Here B columns are butterflies and the K = 32 inputs (Re a, Im a) take two
// instructions per term product.  Lane (h, n) therefore supplies inputs
// a[8h .. 8h+7] of butterfly n and receives outputs y[4h .. 4h+3] and
// y[8+4h .. 8+4h+3] (Re in D rows 0-15, Im in rows 16-31).
#pragma once

#include "cx.h"

namespace gfft {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Round to nearest even, FP32 -> BF16 (finite inputs).
__device__ __forceinline__ __bf16 bf16_rne(float x) {
    unsigned u = __builtin_bit_cast(unsigned, x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return __builtin_bit_cast(__bf16, static_cast<unsigned short>(u >> 16));
}
__device__ __forceinline__ float bf16_val(__bf16 h) {
    return __builtin_bit_cast(float, static_cast<unsigned>(__builtin_bit_cast(unsigned short, h)) << 16);
}

template <int NTERM>
struct split8 {
    bf16x8 t[NTERM];
};

template <int NTERM>
__device__ __forceinline__ split8<NTERM> split_bf16(const float (&v)[8]) {
    split8<NTERM> s;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        float r = v[j];
#pragma unroll
        for (int p = 0; p < NTERM; ++p) {
            const __bf16 h = bf16_rne(r);
            s.t[p][j] = h;
            r -= bf16_val(h);
        }
    }
    return s;
}

// cos and sin of 2 pi m / 16
__device__ __forceinline__ void unit16(int m, float& c, float& s) {
    const float c8 = k_<float>::c8, s8 = k_<float>::s8, r2 = k_<float>::r2;
    const float cs[16] = {1.f, c8, r2, s8, 0.f, -s8, -r2, -c8, -1.f, -c8, -r2, -s8, 0.f, s8, r2, c8};
    c = cs[m & 15];
    s = cs[(m + 12) & 15];  // sin t = cos(t - pi/2)
}

template <int S, int NTERM>
struct dft16_mfma {
    split8<NTERM> w[2];  // A operand for the Re-input and Im-input halves of K

    __device__ __forceinline__ void init(int lane) {
        const int i = lane & 31, h = lane >> 5;
#pragma unroll
        for (int sl = 0; sl < 2; ++sl) {
            float v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int k = sl * 16 + 8 * h + j;
                float c, s;
                unit16((i & 15) * (k & 15), c, s);
                const bool out_im = i >= 16, in_im = k >= 16;
                v[j] = out_im == in_im ? c : (out_im ? S * s : -S * s);
            }
            w[sl] = split_bf16<NTERM>(v);
        }
    }

    // in[j] = a[8h + j]; out[v] = y[8 (v/4) + 4h + v%4]
    __device__ __forceinline__ void run(const cx<float> (&in)[8], cx<float> (&out)[8]) const {
        float re[8], im[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            re[j] = in[j].x;
            im[j] = in[j].y;
        }
        const split8<NTERM> xs[2] = {split_bf16<NTERM>(re), split_bf16<NTERM>(im)};
        f32x16 acc = {};
        // term pairs (p, q) with p + q < NTERM, the smallest first
#pragma unroll
        for (int ord = NTERM - 1; ord >= 0; --ord) {
#pragma unroll
            for (int p = 0; p <= ord; ++p) {
                const int q = ord - p;
#pragma unroll
                for (int sl = 0; sl < 2; ++sl)
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w[sl].t[p], xs[sl].t[q], acc, 0, 0, 0);
            }
        }
#pragma unroll
        for (int v = 0; v < 8; ++v) out[v] = cx<float>{acc[v], acc[v + 8]};
    }
};

// Output slot v of lane half h holds y[out_index(h, v)].
__device__ __forceinline__ int dft16_out_index(int h, int v) { return 8 * (v >> 2) + 4 * h + (v & 3); }

}  // namespace gfft
