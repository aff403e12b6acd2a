// Building blocks of the GNN kernels: BF16 MFMA tiles (gfx950
// v_mfma_f32_32x32x16_bf16) over 32 rows (nodes or directed edges) per wave.
//
// Orientation.  Every Linear layer y = x W is computed transposed,
// D = W^T X^T, so that the rows (nodes/edges) are the 32 columns of the MFMA
// tile:
//   * B operand (X^T, K x 32): lane l holds row l%32 and 8 consecutive input
//     features 8*(l/32) + 0..7 of K-step s (16 features per step) -- exactly a
//     16-byte slice of the row in a row-major [rows x K] BF16 array;
//   * A operand (W^T, 32 x K per output tile mt): lane l holds output
//     feature mt*32 + l%32 and the same 8 input features;
//   * accumulator D (32 x 32 per output tile): value i of lane l is output
//     feature mt*32 + 8*(i/4) + 4*(l/32) + (i%4) of row l%32.
// A layer whose input is the previous layer's accumulator (the hidden layer
// of an MLP) takes its B operand straight from those registers; the K index
// then runs over features in accumulator order, which is absorbed by reading
// the weight rows in the same permuted order ("phi" order) when the A operand
// is staged.  No transpose through LDS is needed between the two Linear
// layers of an MLP.
//
// Weights are staged once per workgroup into LDS as BF16, already in operand
// order (lane-contiguous 16-byte slices), from the FP32 master parameters.
#pragma once

#include <hip/hip_runtime.h>

#include "device_util.h"

namespace lpcg {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMaxMp = 8;

// Offsets (in floats) of one MLP's tensors inside the flat parameter vector.
struct MlpOff {
    int W0, b0, W1, b1;
};
struct GnnOff {
    MlpOff node_enc, edge_enc, node[kMaxMp], edge[kMaxMp], dec;
    MlpOff xdec;  // node decoder of the initial-guess head (when present)
    int total;
};

// Feature index of accumulator value i of lane l in output tile mt.
__device__ __forceinline__ int acc_feat(int mt, int i, int lane) {
    return mt * 32 + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
}
// Input feature of B-operand slot j at K-step s for lane l.
//   natural order (input read from memory): s*16 + 8*(l/32) + j
//   phi order (input = previous accumulators): acc_feat(s/2, (s%2)*8 + j, l)
__device__ __forceinline__ int k_nat(int s, int j, int lane) { return s * 16 + 8 * (lane >> 5) + j; }
__device__ __forceinline__ int k_phi(int s, int j, int lane) {
    return acc_feat(s >> 1, ((s & 1) << 3) + j, lane);
}

// Stage W^T operands of a [K x M] FP32 row-major matrix W (row stride ldw,
// first row k0) into LDS: slot ((mt*S + s)*64 + lane)*8 + j holds
// W[k0 + korder(s, j, lane)][mt*32 + lane%32], S = K/16 steps, M/32 tiles.
template <bool PHI>
__device__ __forceinline__ void stage_weights(__bf16 *lds, const float *__restrict__ W, int ldw, int K,
                                              int M) {
    const int S = K / 16, MT = M / 32;
    const int total = MT * S * 64 * 8;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
        const int j = idx & 7;
        const int lane = (idx >> 3) & 63;
        const int ms = idx >> 9;
        const int s = ms % S, mt = ms / S;
        const int k = PHI ? k_phi(s, j, lane) : k_nat(s, j, lane);
        lds[idx] = (__bf16)W[(size_t)k * ldw + mt * 32 + (lane & 31)];
    }
}

// Stage W (untransposed) operands for a data-gradient product gx = g W^T,
// computed as gx^T = W g^T: the contraction runs over W's columns (fan_out,
// Kc of them) and the output over its rows (fan_in, Mo of them).  Slot
// ((mt*S + s)*64 + lane)*8 + j holds W[mt*32 + lane%32][korder(s, j, lane)].
template <bool PHI>
__device__ __forceinline__ void stage_weightsT(__bf16 *lds, const float *__restrict__ W, int ldw, int Kc,
                                               int Mo) {
    const int S = Kc / 16, MT = Mo / 32;
    const int total = MT * S * 64 * 8;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
        const int j = idx & 7;
        const int lane = (idx >> 3) & 63;
        const int ms = idx >> 9;
        const int s = ms % S, mt = ms / S;
        const int k = PHI ? k_phi(s, j, lane) : k_nat(s, j, lane);
        lds[idx] = (__bf16)W[(size_t)(mt * 32 + (lane & 31)) * ldw + k];
    }
}

__device__ __forceinline__ bf16x8 lds_op(const __bf16 *lds, int S, int mt, int s, int lane) {
    return *reinterpret_cast<const bf16x8 *>(lds + (((mt * S + s) << 6) + lane) * 8);
}

__device__ __forceinline__ f32x16 mfma(bf16x8 a, bf16x8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f32x16 zero16() {
    f32x16 z;
#pragma unroll
    for (int i = 0; i < 16; ++i) z[i] = 0.f;
    return z;
}

// B operand for K-step s from accumulator tiles (phi order).
template <int MT>
__device__ __forceinline__ bf16x8 acc_operand(const f32x16 (&acc)[MT], int s) {
    bf16x8 b;
    const f32x16 &t = acc[s >> 1];
    const int base = (s & 1) << 3;
#pragma unroll
    for (int j = 0; j < 8; ++j) b[j] = (__bf16)t[base + j];
    return b;
}

// Store the accumulator tiles of one row as FP32.
template <int MT>
__device__ __forceinline__ void store_acc_f32(float *row, const f32x16 (&acc)[MT], int lane) {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            f32x4 v;
#pragma unroll
            for (int r = 0; r < 4; ++r) v[r] = acc[mt][4 * q + r];
            *reinterpret_cast<f32x4 *>(row + acc_feat(mt, 4 * q, lane)) = v;
        }
}

// B operand for K-step s from a row-major FP32 row (natural order).
__device__ __forceinline__ bf16x8 load8f(const float *p) {
    const f32x4 a = *reinterpret_cast<const f32x4 *>(p);
    const f32x4 c = *reinterpret_cast<const f32x4 *>(p + 4);
    bf16x8 b;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        b[j] = (__bf16)a[j];
        b[4 + j] = (__bf16)c[j];
    }
    return b;
}

// 16-byte row slice load/store helpers (BF16 row-major arrays).
__device__ __forceinline__ bf16x8 load8(const __bf16 *p) { return *reinterpret_cast<const bf16x8 *>(p); }

// Store the accumulator tiles of one row (this lane's features) as BF16.
template <int MT>
__device__ __forceinline__ void store_acc_bf16(__bf16 *row, const f32x16 (&acc)[MT], int lane) {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            bf16x4 v;
#pragma unroll
            for (int r = 0; r < 4; ++r) v[r] = (__bf16)acc[mt][4 * q + r];
            *reinterpret_cast<bf16x4 *>(row + acc_feat(mt, 4 * q, lane)) = v;
        }
}

// Accumulator tile holding a bias vector (this lane's features), the
// starting value of a product that adds onto it.
// b must be 16-byte aligned: each group of four features is one 16-byte read.
__device__ __forceinline__ f32x16 bias16(const float *b, int lane) {
    f32x16 v;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const f32x4 t = *reinterpret_cast<const f32x4 *>(b + acc_feat(0, 4 * q, lane));
#pragma unroll
        for (int r = 0; r < 4; ++r) v[4 * q + r] = t[r];
    }
    return v;
}

// max(x, 0) for every non-NaN x as one integer max on the bit pattern
// (negative values and -0 have the sign bit set); unlike fmaxf it needs no
// canonicalisation of an MFMA result first.
__device__ __forceinline__ float relu_bits(float x) {
    return __builtin_bit_cast(float, max(__builtin_bit_cast(int, x), 0));
}

// Two 4-wide BF16 slices as one B-operand slot group.
__device__ __forceinline__ bf16x8 cat8(bf16x4 a, bf16x4 b) {
    return __builtin_shufflevector(a, b, 0, 1, 2, 3, 4, 5, 6, 7);
}

// Stage the identity as an A operand in phi order (32 x 32): a product with
// it copies a B operand given in phi order into the accumulator layout.
__device__ __forceinline__ void stage_identity(__bf16 *lds) {
    for (int idx = threadIdx.x; idx < 2 * 64 * 8; idx += blockDim.x) {
        const int j = idx & 7, lane = (idx >> 3) & 63, s = idx >> 9;
        lds[idx] = (__bf16)(k_phi(s, j, lane) == (lane & 31) ? 1.f : 0.f);
    }
}

// Add bias (FP32 params) to accumulator tiles.
template <int MT>
__device__ __forceinline__ void add_bias(f32x16 (&acc)[MT], const float *__restrict__ b, int lane,
                                         bool relu) {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            float v = acc[mt][i] + b[acc_feat(mt, i, lane)];
            acc[mt][i] = relu ? fmaxf(v, 0.f) : v;
        }
}

}  // namespace lpcg
