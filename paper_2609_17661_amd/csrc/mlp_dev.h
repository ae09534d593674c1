// Device-side evaluation of the RICS surrogate network on gfx950 MFMA.
//
// Network: 4 -> 128 -> 128 -> 128 -> 128 -> 3, SiLU after the hidden layers,
// linear output; 50,563 parameters, flat as [W1 (128x4 row-major), b1, W2, b2,
// W3, b3, W4, b4, W5 (3x128), b5].  Weights enter the matrix cores as bfloat16;
// every activation and back-propagated gradient enters as three bfloat16 terms
// hi + mid + lo (each the rounding of what the previous terms leave), so a
// product costs three v_mfma_f32_16x16x32_bf16 that share the weight operand
// and the network evaluates at float32 accuracy with float32 accumulation.
//
// One wavefront evaluates a group of 16 samples at a time as Z^T = W A^T: the
// 16 samples are the MFMA's N dimension, the neurons its M dimension.  With the
// 16x16x32 operand layout (lane l, g = l/16, r = l%16):
//   A (weights, 16 x 32):  lane holds A[r][8g + i], i = 0..7
//   B (activations, 32x16): lane holds B[8g + i][r]
//   D (16 x 16):           lane holds D[4g + j][r], j = 0..3
// the outputs of m-tiles 2K and 2K+1 already sit in the lanes that feed the
// B operand of k-step K, in the neuron order perm(K, g, i) = 32K + 4g + i
// (i < 4) and 32K + 16 + 4g + (i - 4) (i >= 4).  The weight tiles are stored
// pre-permuted in that order, so activations stay in registers between layers.
// Layers with 3 or 4 inputs (the input layer, and W5^T in the backward pass)
// pack the three split terms along K into one MFMA.
#pragma once

#include "pic1d_dev.h"

namespace pic1d {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

constexpr int MLP_IN = 4, MLP_OUT = 3, MLP_W = 128;
constexpr int MLP_NPARAM = 50563;
constexpr int MLP_OFF_W1 = 0, MLP_OFF_B1 = 512;
constexpr int MLP_OFF_W2 = 640, MLP_OFF_B2 = 17024;
constexpr int MLP_OFF_W3 = 17152, MLP_OFF_B3 = 33536;
constexpr int MLP_OFF_W4 = 33664, MLP_OFF_B4 = 50048;
constexpr int MLP_OFF_W5 = 50176, MLP_OFF_B5 = 50560;

// Tiles of 64 lanes x 8 bfloat16.  Forward: W1 (8 m-tiles), W2..W4 (8 m x 4 k
// tiles each, index T*4+K), W5 (4 k-tiles).  Backward: W2^T..W4^T (T*4+K, T the
// input-neuron tile), W5^T (8 tiles).
constexpr int FT_L1 = 0, FT_H0 = 8, FT_OUT = 104, FT_TOTAL = 108;
constexpr int BT_H0 = 0, BT_OUT = 96, BT_TOTAL = 104;
constexpr int MLP_BIAS = 4 * MLP_W + 4;      // b1..b4, b5 (3) + pad: float offsets 0,128,256,384,512

// input box of the network (log10 gamma, s/L, log10 b, kT/keV), mapped to [-1, 1]
__host__ __device__ constexpr float mlp_in_lo(int k) { return k == 0 ? 0.0f : k == 1 ? 0.0f : k == 2 ? -2.0f : 0.3f; }
__host__ __device__ constexpr float mlp_in_hi(int k) { return k == 0 ? 8.0f : k == 1 ? 1.0f : k == 2 ? 3.0f : 1.0f; }

__host__ __device__ inline int mlp_perm(int K, int g, int i) {
    return 32 * K + (i < 4 ? 4 * g + i : 16 + 4 * g + (i - 4));
}

struct Split3 {
    bf16x8 hi, mid, lo;
};

__device__ __forceinline__ void split3(const float (&v)[8], Split3& s) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const __bf16 h = (__bf16)v[i];
        const float r1 = v[i] - (float)h;
        const __bf16 m = (__bf16)r1;
        const float r2 = r1 - (float)m;
        s.hi[i] = h;
        s.mid[i] = m;
        s.lo[i] = (__bf16)r2;
    }
}

__device__ __forceinline__ f32x4 mfma(const bf16x8& a, const bf16x8& b, const f32x4& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float silu_f(float z) { return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }

__device__ __forceinline__ float silu_grad_f(float z) {
    const float s = __builtin_amdgcn_rcpf(1.0f + __expf(-z));
    return s * fmaf(z, 1.0f - s, 1.0f);
}

// B operand of the input layer for sample values x[0..3] (already normalised):
// positions 0..3 hi, 4..7 mid, 8..11 lo, zero beyond.  Lanes g = 0, 1 carry
// data; the caller provides each lane the inputs of sample r of its group.
__device__ __forceinline__ bf16x8 mlp_input_operand(const float (&x)[4], int g) {
    bf16x8 b;
#pragma unroll
    for (int i = 0; i < 8; ++i) b[i] = (__bf16)0.0f;
    if (g < 2) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const __bf16 h = (__bf16)x[k];
            const float r1 = x[k] - (float)h;
            const __bf16 m = (__bf16)r1;
            const __bf16 l = (__bf16)(r1 - (float)m);
            if (g == 0) { b[k] = h; b[4 + k] = m; }
            else b[k] = l;
        }
    }
    return b;
}

// Activations of m-tiles 2K, 2K+1 as the B operand of k-step K.
__device__ __forceinline__ void operand_from_tiles(const f32x4& t0, const f32x4& t1, Split3& s) {
    const float v[8] = {t0[0], t0[1], t0[2], t0[3], t1[0], t1[1], t1[2], t1[3]};
    split3(v, s);
}

// One 128 -> 128 layer on a 16-sample group: acc[T] = bias + sum_K W(T,K) B(K) over
// the three terms of B.  The loops run K, term, tile, so that consecutive MFMAs
// write eight different accumulators (independent chains); each tile still sums
// in the order K0 hi, K0 mid, K0 lo, K1 hi, ...  bias == nullptr starts from zero.
template <class WPtr>
__device__ __forceinline__ void hidden_layer(WPtr w, int base, const float* __restrict__ bias, const Split3 (&op)[4],
                                             f32x4 (&acc)[8]) {
    const int lane = threadIdx.x & 63, g = lane >> 4;
    f32x4 c[8];
#pragma unroll
    for (int T = 0; T < 8; ++T)
        c[T] = bias ? *reinterpret_cast<const f32x4*>(bias + 16 * T + 4 * g) : f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int K = 0; K < 4; ++K) {
        bf16x8 wt[8];
#pragma unroll
        for (int T = 0; T < 8; ++T) wt[T] = w[(base + T * 4 + K) * 64 + lane];
#pragma unroll
        for (int T = 0; T < 8; ++T) c[T] = mfma(wt[T], op[K].hi, c[T]);
#pragma unroll
        for (int T = 0; T < 8; ++T) c[T] = mfma(wt[T], op[K].mid, c[T]);
#pragma unroll
        for (int T = 0; T < 8; ++T) c[T] = mfma(wt[T], op[K].lo, c[T]);
    }
#pragma unroll
    for (int T = 0; T < 8; ++T) acc[T] = c[T];
}

// Forward pass of one 16-sample group.  `bin` is the input operand of this
// lane; returns D of the output layer (lanes g == 0: outputs 0..2 of sample r).
// With STORE, the pre-activations of the four hidden layers are written to
// zs + l*zlayer + row*128 (row = first sample of the group + r).
template <bool STORE, class WPtr>
__device__ __forceinline__ f32x4 mlp_group_forward(WPtr wf, const float* __restrict__ bias, const bf16x8& bin,
                                                   float* __restrict__ zs, int64_t zlayer, int64_t row) {
    const int lane = threadIdx.x & 63, g = lane >> 4;
    f32x4 acc[8];
#pragma unroll
    for (int T = 0; T < 8; ++T) {
        acc[T] = *reinterpret_cast<const f32x4*>(bias + 16 * T + 4 * g);
        acc[T] = mfma(wf[(FT_L1 + T) * 64 + lane], bin, acc[T]);
    }
#pragma unroll 1
    for (int h = 0; h < 3; ++h) {
        if (STORE) {
#pragma unroll
            for (int T = 0; T < 8; ++T)
                *reinterpret_cast<f32x4*>(zs + h * zlayer + row * MLP_W + 16 * T + 4 * g) = acc[T];
        }
        Split3 op[4];
#pragma unroll
        for (int K = 0; K < 4; ++K) {
            f32x4 a0, a1;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                a0[j] = silu_f(acc[2 * K][j]);
                a1[j] = silu_f(acc[2 * K + 1][j]);
            }
            operand_from_tiles(a0, a1, op[K]);
        }
        const float* bl = bias + MLP_W * (h + 1);
        const int base = FT_H0 + 32 * h;
        hidden_layer(wf, base, bl, op, acc);
    }
    if (STORE) {
#pragma unroll
        for (int T = 0; T < 8; ++T)
            *reinterpret_cast<f32x4*>(zs + 3 * zlayer + row * MLP_W + 16 * T + 4 * g) = acc[T];
    }
    Split3 op[4];
#pragma unroll
    for (int K = 0; K < 4; ++K) {
        f32x4 a0, a1;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            a0[j] = silu_f(acc[2 * K][j]);
            a1[j] = silu_f(acc[2 * K + 1][j]);
        }
        operand_from_tiles(a0, a1, op[K]);
    }
    // one output tile: three partial sums (one per term) keep three MFMA chains in flight
    f32x4 o_hi, o_mid = {0.0f, 0.0f, 0.0f, 0.0f}, o_lo = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int j = 0; j < 4; ++j) o_hi[j] = (g == 0 && j < 3) ? bias[4 * MLP_W + j] : 0.0f;
#pragma unroll
    for (int K = 0; K < 4; ++K) {
        const bf16x8 w = wf[(FT_OUT + K) * 64 + lane];
        o_hi = mfma(w, op[K].hi, o_hi);
        o_mid = mfma(w, op[K].mid, o_mid);
        o_lo = mfma(w, op[K].lo, o_lo);
    }
    f32x4 out;
#pragma unroll
    for (int j = 0; j < 4; ++j) out[j] = o_hi[j] + (o_mid[j] + o_lo[j]);
    return out;
}

// Backward pass of one 16-sample group: from dL/d(out) (lanes g == 0, sample r,
// components 0..2) to dL/dz of the four hidden layers, written to
// ds + l*zlayer + row*128; the stored pre-activations zs are read back.
template <class WPtr>
__device__ __forceinline__ void mlp_group_backward(WPtr wb, const f32x4& dout, const float* __restrict__ zs,
                                                   float* __restrict__ ds, int64_t zlayer, int64_t row) {
    const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
    // small-K operand of W5^T: positions 0..2 hi, 3..5 mid, 6..8 lo
    float d3[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) d3[j] = __shfl(dout[j], r, 64);
    __bf16 hi[3], mi[3], lo[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        hi[j] = (__bf16)d3[j];
        const float r1 = d3[j] - (float)hi[j];
        mi[j] = (__bf16)r1;
        lo[j] = (__bf16)(r1 - (float)mi[j]);
    }
    bf16x8 bdo;
#pragma unroll
    for (int i = 0; i < 8; ++i) bdo[i] = (__bf16)0.0f;
    if (g == 0) {
        bdo[0] = hi[0]; bdo[1] = hi[1]; bdo[2] = hi[2];
        bdo[3] = mi[0]; bdo[4] = mi[1]; bdo[5] = mi[2];
        bdo[6] = lo[0]; bdo[7] = lo[1];
    } else if (g == 1) {
        bdo[0] = lo[2];
    }
    f32x4 acc[8];
#pragma unroll
    for (int T = 0; T < 8; ++T) {
        acc[T] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        acc[T] = mfma(wb[(BT_OUT + T) * 64 + lane], bdo, acc[T]);
    }
#pragma unroll 1
    for (int h = 3; h >= 0; --h) {
        // acc holds dL/da of hidden layer h (0-based); times SiLU'(z) gives dL/dz
#pragma unroll
        for (int T = 0; T < 8; ++T) {
            const f32x4 z = *reinterpret_cast<const f32x4*>(zs + h * zlayer + row * MLP_W + 16 * T + 4 * g);
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[T][j] *= silu_grad_f(z[j]);
            *reinterpret_cast<f32x4*>(ds + h * zlayer + row * MLP_W + 16 * T + 4 * g) = acc[T];
        }
        if (h == 0) break;
        Split3 op[4];
#pragma unroll
        for (int K = 0; K < 4; ++K) operand_from_tiles(acc[2 * K], acc[2 * K + 1], op[K]);
        const int base = BT_H0 + 32 * (h - 1);          // W_{h+1}^T maps dL/dz_h to dL/da_{h-1}
        hidden_layer(wb, base, nullptr, op, acc);
    }
}

}  // namespace pic1d
