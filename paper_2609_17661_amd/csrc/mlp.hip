// RICS surrogate network: training samples, bfloat16-MFMA forward, backward and
// weight-gradient kernels, Adam, and the C ABI of the pic1d_mlp_* calls.
//
// The network and its operand layout are described in mlp_dev.h.  What it
// learns, for momenta u >= 0 on the R_max = 4 dipole line (Appendix B.2):
//   o1 = log10(|F_hat| / |gamma mu - u|) = log10(A_F g(y) / x^2)   (Eq. contdrag)
//   o2 = log10(Ndot_hat)                                           (Eq. scatteringNdot)
//   o3 = log10(eps), eps = gamma (1 - (1 + 2b)^-1/2)               (Appendix A.3)
// as functions of (log10 gamma, s/L, log10 b, kT), with b an independent field
// strength.  The training samples are computed here in float64 from those
// closed forms; the loss is the mean squared error of the normalised targets.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pic1d.h"
#include "mlp_dev.h"

namespace pic1d {

int set_global_error(int code, const std::string& msg);
inline int fail(void*, int code, const std::string& msg) { return set_global_error(code, msg); }

constexpr uint32_t STREAM_MLP_SAMPLE = 7, STREAM_MLP_INIT = 8, STREAM_MLP_BATCH = 9;
constexpr int MLP_MAX_ATTEMPTS = 64;
constexpr int MLP_CHUNK = 256;          // samples per weight-gradient block
constexpr int WGRAD_ZSPLIT = 4;         // blocks sharing one chunk of a 128 x 128 layer's tiles
constexpr int MLP_TPB = 256;
constexpr int ADAM_BLOCKS = (MLP_NPARAM + MLP_TPB - 1) / MLP_TPB;   // one parameter per thread

// float64 constants of the RICS prefactors (CODATA 2018; R* = 1e6 cm)
constexpr double kMlpRe = 2.8179403262e-13, kMlpLbar = 3.8615926796e-11, kMlpMeC2 = 510.99895, kMlpRstar = 1.0e6;

// ---------------------------------------------------------------------------
// training samples
// ---------------------------------------------------------------------------

// cos(theta) at arc-length fraction f of the line r = R sin^2(theta), s = 0 at the
// northern footpoint: P(v) = P(v0)(1 - 2f) with P(v) = v (1+3v^2)^1/2 + asinh(3^1/2 v)/3^1/2
// (Appendix B.2), by safeguarded Newton (P' = 2 (1 + 3 v^2)^1/2).
__device__ double mlp_cos_at(double R, double f) {
    const double v0 = sqrt(1.0 - 1.0 / R);
    auto P = [](double v) { return v * sqrt(1.0 + 3.0 * v * v) + asinh(1.7320508075688772 * v) / 1.7320508075688772; };
    const double target = P(v0) * (1.0 - 2.0 * f);
    double lo = -v0, hi = v0, v = v0 * (1.0 - 2.0 * f);
    for (int it = 0; it < 60; ++it) {
        const double e = P(v) - target;
        if (e > 0.0) hi = fmin(hi, v); else lo = fmax(lo, v);
        double vn = v - e / (2.0 * sqrt(1.0 + 3.0 * v * v));
        if (!(vn >= lo && vn <= hi)) vn = 0.5 * (lo + hi);
        if (fabs(vn - v) <= 1e-17 * (1.0 + fabs(v))) { v = vn; break; }
        v = vn;
    }
    return v;
}

// (o1, o2, o3, y) of one input point, float64
__device__ void mlp_targets(const float (&xin)[4], double R, double (&o)[3], double& y) {
    const double lg = xin[0], sl = xin[1], lb = xin[2], kT = xin[3];
    const double gam = exp10(lg);
    const double u = sqrt(fmax(gam * gam - 1.0, 0.0));
    const double b = exp10(lb);
    const double c = mlp_cos_at(R, sl);
    const double mu = 2.0 * c / sqrt(1.0 + 3.0 * c * c);
    const double x = R * (1.0 - c * c);
    const double th = kT / kMlpMeC2;
    y = b / (th * (gam - u * mu));
    const double base = kMlpRe * kMlpRstar / (4.0 * kMlpLbar * kMlpLbar);
    const double em1 = expm1(fmin(y, 700.0));
    o[0] = log10(base * th * th * th * y * y * y / em1 / (x * x));
    o[1] = log10(base * th * th * y * y / em1 / (x * x * gam));
    const double q = sqrt(1.0 + 2.0 * b);
    o[2] = log10(gam * (1.0 - 1.0 / q));
}

__global__ __launch_bounds__(MLP_TPB) void k_mlp_samples(uint32_t k0, uint32_t k1, int64_t first, int64_t n,
                                                         float R, float4* __restrict__ X, float4* __restrict__ O,
                                                         int* __restrict__ err) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t id = (uint64_t)(first + i);
        bool done = false;
        for (int a = 0; a < MLP_MAX_ATTEMPTS && !done; ++a) {
            const uint4 w = philox4x32_10(make_uint4((uint32_t)id, (uint32_t)(id >> 32), (uint32_t)a, STREAM_MLP_SAMPLE),
                                          k0, k1);
            const double u0 = (double)(w.x >> 8) * 0x1.0p-24, u1 = (double)(w.y >> 8) * 0x1.0p-24;
            const double u2 = (double)(w.z >> 8) * 0x1.0p-24, u3 = (double)(w.w >> 8) * 0x1.0p-24;
            const float xin[4] = {(float)(8.0 * u0), (float)u1, (float)(-2.0 + 5.0 * u2), (float)(0.3 + 0.7 * u3)};
            double o[3], y;
            mlp_targets(xin, (double)R, o, y);
            if (y <= (double)Y_CUT) {
                X[i] = make_float4(xin[0], xin[1], xin[2], xin[3]);
                O[i] = make_float4((float)o[0], (float)o[1], (float)o[2], 0.0f);
                done = true;
            }
        }
        if (!done) atomicExch(err, 1);
    }
}

// sums (pass 0) or sums of squared deviations from mean (pass 1) of the three
// target columns, one float64 partial per block and column
__global__ __launch_bounds__(MLP_TPB) void k_mlp_stats(const float4* __restrict__ O, int64_t n, int pass,
                                                       const double* __restrict__ mean, double* __restrict__ part) {
    __shared__ double sh[3][MLP_TPB];
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float4 o = O[i];
        const double v[3] = {o.x, o.y, o.z};
#pragma unroll
        for (int k = 0; k < 3; ++k) acc[k] += pass == 0 ? v[k] : (v[k] - mean[k]) * (v[k] - mean[k]);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) sh[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int s = MLP_TPB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
#pragma unroll
            for (int k = 0; k < 3; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 3) part[blockIdx.x * 3 + threadIdx.x] = sh[threadIdx.x][0];
}

// ---------------------------------------------------------------------------
// parameters -> bfloat16 MFMA tiles
// ---------------------------------------------------------------------------

__device__ __forceinline__ float mlp_w(const float* p, int layer, int o, int i) {
    switch (layer) {
        case 1: return p[MLP_OFF_W1 + o * 4 + i];
        case 2: return p[MLP_OFF_W2 + o * 128 + i];
        case 3: return p[MLP_OFF_W3 + o * 128 + i];
        case 4: return p[MLP_OFF_W4 + o * 128 + i];
        default: return p[MLP_OFF_W5 + o * 128 + i];
    }
}

__global__ __launch_bounds__(MLP_TPB) void k_mlp_pack(const float* __restrict__ p, bf16x8* __restrict__ ft,
                                                      bf16x8* __restrict__ bt, float* __restrict__ bias) {
    const int n_f = FT_TOTAL * 64, n_b = BT_TOTAL * 64;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n_f + n_b + MLP_BIAS; e += gridDim.x * blockDim.x) {
        if (e < n_f + n_b) {
            const bool fwd = e < n_f;
            const int t = fwd ? e / 64 : (e - n_f) / 64;
            const int lane = e & 63, g = lane >> 4, r = lane & 15;
            bf16x8 v;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                float w = 0.0f;
                const int pp = 8 * g + i;
                if (fwd) {
                    if (t < FT_H0) {
                        w = pp < 12 ? mlp_w(p, 1, 16 * t + r, pp & 3) : 0.0f;
                    } else if (t < FT_OUT) {
                        const int h = (t - FT_H0) / 32, idx = (t - FT_H0) % 32, T = idx / 4, K = idx % 4;
                        w = mlp_w(p, h + 2, 16 * T + r, mlp_perm(K, g, i));
                    } else {
                        const int K = t - FT_OUT;
                        w = r < 3 ? mlp_w(p, 5, r, mlp_perm(K, g, i)) : 0.0f;
                    }
                } else {
                    if (t < BT_OUT) {
                        const int h = t / 32, idx = t % 32, T = idx / 4, K = idx % 4;
                        w = mlp_w(p, h + 2, mlp_perm(K, g, i), 16 * T + r);
                    } else {
                        const int T = t - BT_OUT;
                        w = pp < 9 ? mlp_w(p, 5, pp % 3, 16 * T + r) : 0.0f;
                    }
                }
                v[i] = (__bf16)w;
            }
            (fwd ? ft[e] : bt[e - n_f]) = v;
        } else {
            const int k = e - n_f - n_b;
            float b = 0.0f;
            if (k < 128) b = p[MLP_OFF_B1 + k];
            else if (k < 256) b = p[MLP_OFF_B2 + k - 128];
            else if (k < 384) b = p[MLP_OFF_B3 + k - 256];
            else if (k < 512) b = p[MLP_OFF_B4 + k - 384];
            else if (k < 515) b = p[MLP_OFF_B5 + k - 512];
            bias[k] = b;
        }
    }
}

// Glorot-uniform weights from Philox (counter (p, 0, 0, STREAM_MLP_INIT)), zero biases
__global__ __launch_bounds__(MLP_TPB) void k_mlp_init(uint32_t k0, uint32_t k1, float* __restrict__ p) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < MLP_NPARAM; e += gridDim.x * blockDim.x) {
        int fin = 0, fout = 0;
        bool weight = true;
        if (e < MLP_OFF_B1) { fin = 4; fout = 128; }
        else if (e < MLP_OFF_W2) weight = false;
        else if (e < MLP_OFF_B2) { fin = 128; fout = 128; }
        else if (e < MLP_OFF_W3) weight = false;
        else if (e < MLP_OFF_B3) { fin = 128; fout = 128; }
        else if (e < MLP_OFF_W4) weight = false;
        else if (e < MLP_OFF_B4) { fin = 128; fout = 128; }
        else if (e < MLP_OFF_W5) weight = false;
        else if (e < MLP_OFF_B5) { fin = 128; fout = 3; }
        else weight = false;
        float v = 0.0f;
        if (weight) {
            const uint4 w = philox4x32_10(make_uint4((uint32_t)e, 0u, 0u, STREAM_MLP_INIT), k0, k1);
            v = sqrtf(6.0f / (float)(fin + fout)) * (2.0f * uniform24(w.x) - 1.0f);
        }
        p[e] = v;
    }
}

// ---------------------------------------------------------------------------
// forward / backward over a batch
// ---------------------------------------------------------------------------

__device__ __forceinline__ void mlp_normalise(const float4& x, float (&xn)[4]) {
    const float v[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) xn[k] = (v[k] - mlp_in_lo(k)) * (2.0f / (mlp_in_hi(k) - mlp_in_lo(k))) - 1.0f;
}

// Inference: raw inputs X (n x 4) -> network outputs out (n x 3, normalised targets).
__global__ __launch_bounds__(MLP_TPB) void k_mlp_forward(const bf16x8* __restrict__ ft, const float* __restrict__ bias,
                                                         const float4* __restrict__ X, int64_t n,
                                                         float* __restrict__ out) {
    const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t q = wave; q * 16 < n; q += nwave) {
        const int64_t row = q * 16 + r;
        float xn[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (row < n && g < 2) mlp_normalise(X[row], xn);
        const bf16x8 bin = mlp_input_operand(xn, g);
        const f32x4 o = mlp_group_forward<false>(ft, bias, bin, nullptr, 0, 0);
        if (g == 0 && row < n) {
            out[row * 3 + 0] = o[0];
            out[row * 3 + 1] = o[1];
            out[row * 3 + 2] = o[2];
        }
    }
}

struct TrainFwdArgs {
    const bf16x8* ft;
    const float* bias;
    const float4* X;          // inputs (raw)
    const float* T;           // explicit normalised targets (n x 3), or null
    const float4* O;          // sample targets (o1, o2, o3), used with norm when T is null
    const float* norm;        // mean[3], std[3]
    int64_t n_batch;          // samples in the batch
    int64_t n_pool;           // sample pool size; batch rows draw from it when > 0
    uint32_t step, k0, k1;
    float4* XN;               // normalised inputs of the batch rows
    float* Z;                 // pre-activations, 4 x rows x 128
    float4* DOUT;             // dL/d(out), rows x 4
    int64_t zlayer;
    double* loss_part;        // one partial sum of squared errors per block
};

__global__ __launch_bounds__(MLP_TPB) void k_mlp_train_fwd(TrainFwdArgs a) {
    __shared__ double sl[MLP_TPB / 64];
    const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t rows = a.zlayer / MLP_W;
    double lsum = 0.0;
    for (int64_t q = wave; q * 16 < rows; q += nwave) {
        const int64_t row = q * 16 + r;
        const bool valid = row < a.n_batch;
        float xn[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        float t[3] = {0.0f, 0.0f, 0.0f};
        if (valid && g < 2) {
            int64_t src = row;
            if (a.n_pool > 0) {
                const uint4 w = philox4x32_10(make_uint4(a.step, (uint32_t)row, (uint32_t)(row >> 32), STREAM_MLP_BATCH),
                                              a.k0, a.k1);
                const uint64_t h = ((uint64_t)w.x << 32) | w.y;
                src = (int64_t)__umul64hi(h, (uint64_t)a.n_pool);
            }
            mlp_normalise(a.X[src], xn);
            if (g == 0) {
                if (a.T) {
                    t[0] = a.T[src * 3]; t[1] = a.T[src * 3 + 1]; t[2] = a.T[src * 3 + 2];
                } else {
                    const float4 o = a.O[src];
                    t[0] = (o.x - a.norm[0]) / a.norm[3];
                    t[1] = (o.y - a.norm[1]) / a.norm[4];
                    t[2] = (o.z - a.norm[2]) / a.norm[5];
                }
            }
        }
        const bf16x8 bin = mlp_input_operand(xn, g);
        const f32x4 o = mlp_group_forward<true>(a.ft, a.bias, bin, a.Z, a.zlayer, row);
        if (g == 0) {
            const float c = 2.0f / (3.0f * (float)a.n_batch);
            float4 d = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (valid) {
                const float e0 = o[0] - t[0], e1 = o[1] - t[1], e2 = o[2] - t[2];
                d = make_float4(c * e0, c * e1, c * e2, 0.0f);
                lsum += (double)e0 * e0 + (double)e1 * e1 + (double)e2 * e2;
            }
            a.DOUT[row] = d;
            a.XN[row] = make_float4(xn[0], xn[1], xn[2], xn[3]);
        }
    }
    for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o, 64);
    if (lane == 0) sl[threadIdx.x >> 6] = lsum;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < MLP_TPB / 64; ++w) s += sl[w];
        a.loss_part[blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(MLP_TPB) void k_mlp_train_bwd(const bf16x8* __restrict__ bt, const float4* __restrict__ DOUT,
                                                           const float* __restrict__ Z, float* __restrict__ DS,
                                                           int64_t zlayer) {
    const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t rows = zlayer / MLP_W;
    for (int64_t q = wave; q * 16 < rows; q += nwave) {
        const int64_t row = q * 16 + r;
        f32x4 d = {0.0f, 0.0f, 0.0f, 0.0f};
        if (g == 0) {
            const float4 v = DOUT[row];
            d = f32x4{v.x, v.y, v.z, 0.0f};
        }
        mlp_group_backward(bt, d, Z, DS, zlayer, row);
    }
}

// Weight and bias gradients of one layer over one chunk of MLP_CHUNK rows:
// dW[o][i] = sum_s delta[s][o] a[s][i], db[o] = sum_s delta[s][o]; both operands
// enter as three bfloat16 terms (the six products above 2^-24 relative).
// grid = (chunks, 5 layers); partial[chunk][param] in the flat packing.
__global__ __launch_bounds__(MLP_TPB) void k_mlp_wgrad(const float4* __restrict__ XN, const float* __restrict__ Z,
                                                       const float* __restrict__ DS, const float4* __restrict__ DOUT,
                                                       int64_t zlayer, float* __restrict__ partial) {
    constexpr int LD = 36;
    __shared__ float sD[MLP_W][LD];
    __shared__ float sA[MLP_W][LD];
    const int layer = blockIdx.y + 1;
    const int M = layer == 5 ? 3 : MLP_W;
    const int N = layer == 1 ? 4 : MLP_W;
    const int offW = layer == 1 ? MLP_OFF_W1 : layer == 2 ? MLP_OFF_W2 : layer == 3 ? MLP_OFF_W3
                   : layer == 4 ? MLP_OFF_W4 : MLP_OFF_W5;
    const int offB = offW + M * N;
    const int nTo = (M + 15) / 16, nTi = (N + 15) / 16, ntile = nTo * nTi;
    // the 128 x 128 layers split their 64 tiles over the blocks of gridDim.z (more
    // blocks than CUs at training batches); the small layers take z = 0 alone
    const int zsplit = (M == MLP_W && N == MLP_W) ? (int)gridDim.z : 1;
    if ((int)blockIdx.z >= zsplit) return;
    const int t_first = (int)blockIdx.z * (ntile / zsplit), t_end = t_first + ntile / zsplit;
    const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
    const int w = threadIdx.x >> 6;
    const int64_t row0 = (int64_t)blockIdx.x * MLP_CHUNK;
    f32x4 acc[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    float db = 0.0f;
    for (int ks = 0; ks < MLP_CHUNK / 32; ++ks) {
        const int64_t s0 = row0 + 32 * ks;
        // stage delta^T and a^T for 32 rows (zero beyond M / N)
        for (int e = threadIdx.x; e < 32 * MLP_W; e += blockDim.x) {
            const int s = e / MLP_W, c = e % MLP_W;
            const int64_t row = s0 + s;
            float dv = 0.0f, av = 0.0f;
            // the deltas of the block's output rows (all rows in block z = 0, which also
            // sums the bias gradient)
            const bool dneed = blockIdx.z == 0 || (c >= 32 * (int)blockIdx.z && c < 32 * (int)blockIdx.z + 32);
            if (c < M && dneed) {
                if (layer == 5) {
                    const float4 v = DOUT[row];
                    dv = c == 0 ? v.x : c == 1 ? v.y : v.z;
                } else {
                    dv = DS[(layer - 1) * zlayer + row * MLP_W + c];
                }
            }
            if (c < N) {
                if (layer == 1) {
                    const float4 v = XN[row];
                    av = c == 0 ? v.x : c == 1 ? v.y : c == 2 ? v.z : v.w;
                } else {
                    av = silu_f(Z[(layer - 2) * zlayer + row * MLP_W + c]);
                }
            }
            sD[c][s] = dv;
            sA[c][s] = av;
        }
        __syncthreads();
        if (blockIdx.z == 0 && (int)threadIdx.x < M) {
            float s = 0.0f;
            for (int k = 0; k < 32; ++k) s += sD[threadIdx.x][k];
            db += s;
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int t = t_first + w + 4 * k;
            if (t < t_end) {
                const int To = t / nTi, Ti = t % nTi;
                float dv[8], av[8];
                const float4 d0 = *reinterpret_cast<const float4*>(&sD[16 * To + r][8 * g]);
                const float4 d1 = *reinterpret_cast<const float4*>(&sD[16 * To + r][8 * g + 4]);
                const float4 a0 = *reinterpret_cast<const float4*>(&sA[16 * Ti + r][8 * g]);
                const float4 a1 = *reinterpret_cast<const float4*>(&sA[16 * Ti + r][8 * g + 4]);
                dv[0] = d0.x; dv[1] = d0.y; dv[2] = d0.z; dv[3] = d0.w;
                dv[4] = d1.x; dv[5] = d1.y; dv[6] = d1.z; dv[7] = d1.w;
                av[0] = a0.x; av[1] = a0.y; av[2] = a0.z; av[3] = a0.w;
                av[4] = a1.x; av[5] = a1.y; av[6] = a1.z; av[7] = a1.w;
                Split3 A, B;
                split3(dv, A);
                split3(av, B);
                f32x4 c = acc[k];
                c = mfma(A.hi, B.hi, c);
                c = mfma(A.hi, B.mid, c);
                c = mfma(A.mid, B.hi, c);
                c = mfma(A.hi, B.lo, c);
                c = mfma(A.lo, B.hi, c);
                c = mfma(A.mid, B.mid, c);
                acc[k] = c;
            }
        }
        __syncthreads();
    }
    float* out = partial + (int64_t)blockIdx.x * MLP_NPARAM;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int t = t_first + w + 4 * k;
        if (t < t_end) {
            const int To = t / nTi, Ti = t % nTi;
            const int i = 16 * Ti + r;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int o = 16 * To + 4 * g + j;
                if (o < M && i < N) out[offW + o * N + i] = acc[k][j];
            }
        }
    }
    if (blockIdx.z == 0 && (int)threadIdx.x < M) out[offB + threadIdx.x] = db;
}

// Sum of the chunk partials (fixed order) and, if apply, one Adam step
// (Kingma & Ba 2015, Algorithm 1) with bias corrections bc1 = 1 - beta1^t, bc2 = 1 - beta2^t.
struct AdamArgs {
    float lr, beta1, omb1, beta2, omb2, eps, bc1, bc2;   // omb = 1 - beta, bc = 1 - beta^t (formed in float64)
};

__global__ __launch_bounds__(MLP_TPB) void k_mlp_adam(const float* __restrict__ partial, int nchunk,
                                                      float* __restrict__ p, float* __restrict__ m,
                                                      float* __restrict__ v, float* __restrict__ grad_out, int apply,
                                                      AdamArgs h) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < MLP_NPARAM; e += gridDim.x * blockDim.x) {
        float gsum = 0.0f;
#pragma unroll 8
        for (int c = 0; c < nchunk; ++c) gsum += partial[(int64_t)c * MLP_NPARAM + e];
        if (grad_out) grad_out[e] = gsum;
        if (apply) {
            const float mm = h.beta1 * m[e] + h.omb1 * gsum;
            const float vv = h.beta2 * v[e] + h.omb2 * gsum * gsum;
            m[e] = mm;
            v[e] = vv;
            p[e] -= h.lr * (mm / h.bc1) / (sqrtf(vv / h.bc2) + h.eps);
        }
    }
}

}  // namespace pic1d

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
using namespace pic1d;

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

AdamArgs adam_args(double lr, double beta1, double beta2, double eps, int64_t t) {
    AdamArgs h;
    h.lr = (float)lr;
    h.beta1 = (float)beta1;
    h.omb1 = (float)(1.0 - beta1);
    h.beta2 = (float)beta2;
    h.omb2 = (float)(1.0 - beta2);
    h.eps = (float)eps;
    h.bc1 = (float)(1.0 - std::pow(beta1, (double)t));
    h.bc2 = (float)(1.0 - std::pow(beta2, (double)t));
    return h;
}

struct MlpWork {
    bf16x8* ft = nullptr;
    bf16x8* bt = nullptr;
    float* bias = nullptr;
    float* master = nullptr;
    float* m = nullptr;
    float* v = nullptr;
    float* grad = nullptr;
    float* norm = nullptr;
    float4* X = nullptr;
    float4* O = nullptr;
    float4* XN = nullptr;
    float4* DOUT = nullptr;
    float* Z = nullptr;
    float* DS = nullptr;
    float* partial = nullptr;
    double* loss_part = nullptr;
    double* stat_part = nullptr;
    double* mean_dev = nullptr;
    int* err = nullptr;
    int64_t rows = 0;            // batch rows rounded up to MLP_CHUNK
    int nchunk = 0;
    size_t bytes = 0;
};

constexpr int FWD_BLOCKS = 1024;
constexpr int STAT_BLOCKS = 512;

// Carve the training workspace: tiles, parameters and Adam moments, the sample
// pool (n_pool rows of inputs and targets), the per-batch activations and the
// weight-gradient partials.  With base == nullptr only the size is computed.
MlpWork mlp_layout(char* base, int64_t batch, int64_t n_pool) {
    MlpWork w;
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        char* p = base ? base + off : nullptr;
        off = align256(off + bytes);
        return p;
    };
    w.rows = ((batch + MLP_CHUNK - 1) / MLP_CHUNK) * MLP_CHUNK;
    w.nchunk = (int)(w.rows / MLP_CHUNK);
    w.ft = reinterpret_cast<bf16x8*>(take(sizeof(bf16x8) * FT_TOTAL * 64));
    w.bt = reinterpret_cast<bf16x8*>(take(sizeof(bf16x8) * BT_TOTAL * 64));
    w.bias = reinterpret_cast<float*>(take(sizeof(float) * MLP_BIAS));
    w.master = reinterpret_cast<float*>(take(sizeof(float) * MLP_NPARAM));
    w.m = reinterpret_cast<float*>(take(sizeof(float) * MLP_NPARAM));
    w.v = reinterpret_cast<float*>(take(sizeof(float) * MLP_NPARAM));
    w.grad = reinterpret_cast<float*>(take(sizeof(float) * MLP_NPARAM));
    w.norm = reinterpret_cast<float*>(take(sizeof(float) * 8));
    w.X = reinterpret_cast<float4*>(take(sizeof(float4) * std::max<int64_t>(n_pool, 1)));
    w.O = reinterpret_cast<float4*>(take(sizeof(float4) * std::max<int64_t>(n_pool, 1)));
    w.XN = reinterpret_cast<float4*>(take(sizeof(float4) * w.rows));
    w.DOUT = reinterpret_cast<float4*>(take(sizeof(float4) * w.rows));
    w.Z = reinterpret_cast<float*>(take(sizeof(float) * 4 * w.rows * MLP_W));
    w.DS = reinterpret_cast<float*>(take(sizeof(float) * 4 * w.rows * MLP_W));
    w.partial = reinterpret_cast<float*>(take(sizeof(float) * (size_t)w.nchunk * MLP_NPARAM));
    w.loss_part = reinterpret_cast<double*>(take(sizeof(double) * FWD_BLOCKS));
    w.stat_part = reinterpret_cast<double*>(take(sizeof(double) * 3 * STAT_BLOCKS));
    w.mean_dev = reinterpret_cast<double*>(take(sizeof(double) * 4));
    w.err = reinterpret_cast<int*>(take(sizeof(int) * 4));
    w.bytes = off;
    return w;
}

#define MLP_TRY(expr)                                                                               \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess) return fail(nullptr, PIC1D_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

int check_workspace(void* ws, size_t have, size_t need) {
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) != 0 || have < need)
        return fail(nullptr, PIC1D_ENOMEM, "workspace missing, misaligned (256 B) or smaller than pic1d_mlp_workspace_size");
    return PIC1D_OK;
}

void split_seed(uint64_t seed, uint32_t& k0, uint32_t& k1) {
    k0 = (uint32_t)seed;
    k1 = (uint32_t)(seed >> 32);
}

// one forward + backward + weight-gradient pass over the batch rows already
// addressed by `fa`; leaves the chunk partials in w.partial
int run_grad(const MlpWork& w, TrainFwdArgs fa, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_train_fwd, dim3(std::min<int64_t>(FWD_BLOCKS, (w.rows / 16 + 3) / 4)), dim3(MLP_TPB), 0,
                       s, fa);
    hipLaunchKernelGGL(k_mlp_train_bwd, dim3(std::min<int64_t>(FWD_BLOCKS, (w.rows / 16 + 3) / 4)), dim3(MLP_TPB), 0,
                       s, w.bt, w.DOUT, w.Z, w.DS, (int64_t)(w.rows * MLP_W));
    hipLaunchKernelGGL(k_mlp_wgrad, dim3(w.nchunk, 5, WGRAD_ZSPLIT), dim3(MLP_TPB), 0, s, w.XN, w.Z, w.DS, w.DOUT,
                       (int64_t)(w.rows * MLP_W), w.partial);
    MLP_TRY(hipGetLastError());
    return PIC1D_OK;
}

double sum_loss(const MlpWork& w, int nblocks, hipStream_t s) {
    double h[FWD_BLOCKS];          // on the stack: the allocation-free entry point uses this too
    nblocks = std::min(nblocks, FWD_BLOCKS);
    if (hipMemcpyAsync(h, w.loss_part, sizeof(double) * nblocks, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return NAN;
    double t = 0.0;
    for (int b = 0; b < nblocks; ++b) t += h[b];
    return t;
}

// The loss and gradient of n samples on a carved workspace w (pic1d_mlp_loss_grad
// and its allocation-free variant).
int loss_grad_on(const MlpWork& w, const float* params, int64_t n, const float* x, const float* t, float* grad,
                 double* loss, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_pack, dim3(64), dim3(MLP_TPB), 0, s, params, w.ft, w.bt, w.bias);
    TrainFwdArgs fa{};
    fa.ft = w.ft; fa.bias = w.bias; fa.X = reinterpret_cast<const float4*>(x); fa.T = t;
    fa.n_batch = n; fa.n_pool = 0; fa.XN = w.XN; fa.Z = w.Z; fa.DOUT = w.DOUT;
    fa.zlayer = w.rows * MLP_W; fa.loss_part = w.loss_part;
    if (int rc = run_grad(w, fa, s)) return rc;
    hipLaunchKernelGGL(k_mlp_adam, dim3(ADAM_BLOCKS), dim3(MLP_TPB), 0, s, w.partial, w.nchunk, nullptr, nullptr, nullptr, grad,
                       0, adam_args(0.0, 0.0, 0.0, 1.0, 1));
    MLP_TRY(hipGetLastError());
    const double l = sum_loss(w, (int)std::min<int64_t>(FWD_BLOCKS, (w.rows / 16 + 3) / 4), s);
    if (loss) *loss = l / (3.0 * (double)n);
    return PIC1D_OK;
}

// ---------------------------------------------------------------------------
// Scratch of pic1d_mlp_loss_grad_static: the workspace of a batch of up to
// MLP_STATIC_MAX_ROWS samples as a file-scope device array, held by each GPU the
// library runs on until the process ends.  In host code `scratch` names a host
// stand-in, never the device memory: the device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
// ---------------------------------------------------------------------------
constexpr int64_t MLP_STATIC_MAX_ROWS = 2048;
constexpr size_t MLP_STATIC_BYTES = (size_t)12 << 20;
constexpr int MLP_STATIC_MAX_DEVICES = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[MLP_STATIC_BYTES];

namespace {

std::mutex g_scratch_mutex;
void* g_scratch_ptr[MLP_STATIC_MAX_DEVICES] = {};

int static_scratch(void** out) {
    int dev = -1;
    MLP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= MLP_STATIC_MAX_DEVICES)
        return fail(nullptr, PIC1D_EDEVICE, "device index beyond the static scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(nullptr, PIC1D_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PIC1D_OK;
}

}  // namespace

extern "C" {

int pic1d_mlp_param_count(void) { return MLP_NPARAM; }

int pic1d_mlp_workspace_size(int64_t batch, int64_t n_pool, size_t* bytes) {
    if (!bytes || batch <= 0 || n_pool < 0) return fail(nullptr, PIC1D_EINVAL, "bad arguments");
    *bytes = mlp_layout(nullptr, batch, n_pool).bytes;
    return PIC1D_OK;
}

int pic1d_mlp_samples(uint64_t seed, int64_t first, int64_t n, float* x, float* o, void* workspace,
                      size_t workspace_bytes, void* stream) {
    if (n < 0 || first < 0 || (n > 0 && (!x || !o)) || (reinterpret_cast<uintptr_t>(x) & 15) ||
        (reinterpret_cast<uintptr_t>(o) & 15))
        return fail(nullptr, PIC1D_EINVAL, "bad arguments (x, o: device, 16-byte aligned, n x 4 floats)");
    if (int rc = check_workspace(workspace, workspace_bytes, PIC1D_MLP_SAMPLES_WORKSPACE)) return rc;
    if (n == 0) return PIC1D_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int* err = static_cast<int*>(workspace);
    MLP_TRY(hipMemsetAsync(err, 0, sizeof(int), s));
    uint32_t k0, k1;
    split_seed(seed, k0, k1);
    const int blocks = (int)std::min<int64_t>((n + MLP_TPB - 1) / MLP_TPB, 65536);
    hipLaunchKernelGGL(k_mlp_samples, dim3(blocks), dim3(MLP_TPB), 0, s, k0, k1, first, n, 4.0f,
                       reinterpret_cast<float4*>(x), reinterpret_cast<float4*>(o), err);
    MLP_TRY(hipGetLastError());
    int h = 0;
    MLP_TRY(hipMemcpyAsync(&h, err, sizeof(int), hipMemcpyDeviceToHost, s));
    MLP_TRY(hipStreamSynchronize(s));
    if (h) return fail(nullptr, PIC1D_ENONFINITE, "sample stream exhausted its attempts");
    return PIC1D_OK;
}

int pic1d_mlp_forward(const float* params, int64_t n, const float* x, float* out, void* workspace,
                      size_t workspace_bytes, void* stream) {
    if (!params || n < 0 || (n > 0 && (!x || !out)) || (reinterpret_cast<uintptr_t>(x) & 15))
        return fail(nullptr, PIC1D_EINVAL, "bad arguments");
    const MlpWork need = mlp_layout(nullptr, 1, 0);
    if (int rc = check_workspace(workspace, workspace_bytes, need.bytes)) return rc;
    const MlpWork w = mlp_layout(static_cast<char*>(workspace), 1, 0);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_mlp_pack, dim3(64), dim3(MLP_TPB), 0, s, params, w.ft, w.bt, w.bias);
    if (n > 0) {
        const int blocks = (int)std::min<int64_t>(FWD_BLOCKS, (n + 63) / 64);
        hipLaunchKernelGGL(k_mlp_forward, dim3(blocks), dim3(MLP_TPB), 0, s, w.ft, w.bias,
                           reinterpret_cast<const float4*>(x), n, out);
    }
    MLP_TRY(hipGetLastError());
    MLP_TRY(hipStreamSynchronize(s));
    return PIC1D_OK;
}

int pic1d_mlp_loss_grad(const float* params, int64_t n, const float* x, const float* t, float* grad, double* loss,
                        void* workspace, size_t workspace_bytes, void* stream) {
    if (!params || n <= 0 || !x || !t || !grad || (reinterpret_cast<uintptr_t>(x) & 15))
        return fail(nullptr, PIC1D_EINVAL, "bad arguments");
    const MlpWork need = mlp_layout(nullptr, n, 0);
    if (int rc = check_workspace(workspace, workspace_bytes, need.bytes)) return rc;
    const MlpWork w = mlp_layout(static_cast<char*>(workspace), n, 0);
    return loss_grad_on(w, params, n, x, t, grad, loss, static_cast<hipStream_t>(stream));
}

int pic1d_mlp_loss_grad_static(const float* params, int64_t n, const float* x, const float* t, float* grad,
                               double* loss, void* stream) {
    if (!params || n <= 0 || !x || !t || !grad || (reinterpret_cast<uintptr_t>(x) & 15))
        return fail(nullptr, PIC1D_EINVAL, "bad arguments");
    if (n > MLP_STATIC_MAX_ROWS)
        return fail(nullptr, PIC1D_EINVAL,
                    "n exceeds the static scratch of pic1d_mlp_loss_grad_static (at most 2048 samples per call)");
    // every layout up to the maximum batch fits the array (checked, not assumed)
    if (mlp_layout(nullptr, MLP_STATIC_MAX_ROWS, 0).bytes > MLP_STATIC_BYTES)
        return fail(nullptr, PIC1D_ENOMEM, "static scratch smaller than the layout of its maximum batch");
    void* base = nullptr;
    if (int rc = static_scratch(&base)) return rc;
    const MlpWork w = mlp_layout(static_cast<char*>(base), n, 0);
    return loss_grad_on(w, params, n, x, t, grad, loss, static_cast<hipStream_t>(stream));
}

int pic1d_mlp_adam(float* params, float* m, float* v, const float* grad, int64_t t, double lr, double beta1,
                   double beta2, double eps, void* stream) {
    if (!params || !m || !v || !grad || t < 1 || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0))
        return fail(nullptr, PIC1D_EINVAL, "bad arguments");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_mlp_adam, dim3(ADAM_BLOCKS), dim3(MLP_TPB), 0, s, grad, 1, params, m, v, nullptr, 1,
                       adam_args(lr, beta1, beta2, eps, t));
    MLP_TRY(hipGetLastError());
    MLP_TRY(hipStreamSynchronize(s));
    return PIC1D_OK;
}

int pic1d_mlp_train(const pic1d_mlp_train_config* c, pic1d_mlp_train_result* res) {
    if (!c || !res || c->n_samples <= 0 || c->batch <= 0 || c->steps < 0 || !(c->lr > 0.0f) ||
        !(c->lr_final >= 0.0f) || !res->params || !res->norm)
        return fail(nullptr, PIC1D_EINVAL, "bad arguments");
    const MlpWork need = mlp_layout(nullptr, c->batch, c->n_samples);
    if (int rc = check_workspace(c->workspace, c->workspace_bytes, need.bytes)) return rc;
    const MlpWork w = mlp_layout(static_cast<char*>(c->workspace), c->batch, c->n_samples);
    hipStream_t s = static_cast<hipStream_t>(c->stream);
    const auto t0 = std::chrono::steady_clock::now();
    uint32_t k0, k1;
    split_seed(c->seed, k0, k1);

    // samples and their normalisation
    MLP_TRY(hipMemsetAsync(w.err, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_mlp_samples, dim3((int)std::min<int64_t>((c->n_samples + MLP_TPB - 1) / MLP_TPB, 65536)),
                       dim3(MLP_TPB), 0, s, k0, k1, (int64_t)0, c->n_samples, 4.0f, w.X, w.O, w.err);
    hipLaunchKernelGGL(k_mlp_stats, dim3(STAT_BLOCKS), dim3(MLP_TPB), 0, s, w.O, c->n_samples, 0, nullptr, w.stat_part);
    std::vector<double> part(3 * STAT_BLOCKS);
    MLP_TRY(hipMemcpyAsync(part.data(), w.stat_part, sizeof(double) * part.size(), hipMemcpyDeviceToHost, s));
    int herr = 0;
    MLP_TRY(hipMemcpyAsync(&herr, w.err, sizeof(int), hipMemcpyDeviceToHost, s));
    MLP_TRY(hipStreamSynchronize(s));
    if (herr) return fail(nullptr, PIC1D_ENONFINITE, "sample stream exhausted its attempts");
    double mean[4] = {0, 0, 0, 0}, var[3] = {0, 0, 0};
    for (int b = 0; b < STAT_BLOCKS; ++b)
        for (int k = 0; k < 3; ++k) mean[k] += part[b * 3 + k];
    for (int k = 0; k < 3; ++k) mean[k] /= (double)c->n_samples;
    MLP_TRY(hipMemcpyAsync(w.mean_dev, mean, sizeof(double) * 4, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_mlp_stats, dim3(STAT_BLOCKS), dim3(MLP_TPB), 0, s, w.O, c->n_samples, 1, w.mean_dev,
                       w.stat_part);
    MLP_TRY(hipMemcpyAsync(part.data(), w.stat_part, sizeof(double) * part.size(), hipMemcpyDeviceToHost, s));
    MLP_TRY(hipStreamSynchronize(s));
    for (int b = 0; b < STAT_BLOCKS; ++b)
        for (int k = 0; k < 3; ++k) var[k] += part[b * 3 + k];
    float norm[8] = {0};
    for (int k = 0; k < 3; ++k) {
        norm[k] = (float)mean[k];
        norm[3 + k] = (float)std::sqrt(var[k] / (double)c->n_samples);
        if (!(norm[3 + k] > 0.0f)) norm[3 + k] = 1.0f;
    }
    MLP_TRY(hipMemcpyAsync(w.norm, norm, sizeof(norm), hipMemcpyHostToDevice, s));

    // initial weights, zero moments
    if (c->init_params) {
        MLP_TRY(hipMemcpyAsync(w.master, c->init_params, sizeof(float) * MLP_NPARAM, hipMemcpyHostToDevice, s));
    } else {
        hipLaunchKernelGGL(k_mlp_init, dim3(64), dim3(MLP_TPB), 0, s, k0, k1, w.master);
    }
    MLP_TRY(hipMemsetAsync(w.m, 0, sizeof(float) * MLP_NPARAM, s));
    MLP_TRY(hipMemsetAsync(w.v, 0, sizeof(float) * MLP_NPARAM, s));
    MLP_TRY(hipMemsetAsync(w.XN, 0, sizeof(float4) * w.rows, s));

    const int fwd_blocks = (int)std::min<int64_t>(FWD_BLOCKS, (w.rows / 16 + 3) / 4);
    TrainFwdArgs fa{};
    fa.ft = w.ft; fa.bias = w.bias; fa.X = w.X; fa.T = nullptr; fa.O = w.O; fa.norm = w.norm;
    fa.n_batch = c->batch; fa.n_pool = c->n_samples; fa.k0 = k0; fa.k1 = k1;
    fa.XN = w.XN; fa.Z = w.Z; fa.DOUT = w.DOUT; fa.zlayer = w.rows * MLP_W; fa.loss_part = w.loss_part;
    const double b1 = c->beta1 > 0.0 ? c->beta1 : 0.9, b2 = c->beta2 > 0.0 ? c->beta2 : 0.999;
    const double eps = c->eps > 0.0 ? c->eps : 1e-8;
    const int nlog = std::max(0, std::min(res->n_loss, c->steps));
    int logged = 0;
    res->loss_first = NAN;
    for (int t = 1; t <= c->steps; ++t) {
        hipLaunchKernelGGL(k_mlp_pack, dim3(64), dim3(MLP_TPB), 0, s, w.master, w.ft, w.bt, w.bias);
        fa.step = (uint32_t)t;
        if (int rc = run_grad(w, fa, s)) return rc;
        const double lr = c->lr_final + 0.5 * (c->lr - c->lr_final) *
                                            (1.0 + std::cos(3.141592653589793 * (double)(t - 1) / (double)c->steps));
        hipLaunchKernelGGL(k_mlp_adam, dim3(ADAM_BLOCKS), dim3(MLP_TPB), 0, s, w.partial, w.nchunk, w.master, w.m, w.v,
                           nullptr, 1, adam_args(lr, b1, b2, eps, t));
        MLP_TRY(hipGetLastError());
        const bool first = t == 1;
        const bool log_now = nlog > 0 && res->loss && logged < nlog &&
                             (int64_t)(t - 1) * nlog / c->steps >= logged;
        if (first || log_now || t == c->steps) {
            const double l = sum_loss(w, fwd_blocks, s) / (3.0 * (double)c->batch);
            if (first) res->loss_first = l;
            if (log_now) res->loss[logged++] = l;
            if (t == c->steps) res->loss_last = l;
        }
    }
    MLP_TRY(hipMemcpyAsync(res->params, w.master, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToHost, s));
    MLP_TRY(hipStreamSynchronize(s));
    for (int k = 0; k < 6; ++k) res->norm[k] = norm[k];
    res->n_loss = logged;
    res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return PIC1D_OK;
}

}  // extern "C"
