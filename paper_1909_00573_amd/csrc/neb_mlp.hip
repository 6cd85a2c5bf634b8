// Learned density: a small MLP that maps a surface point and its normal to
// log(density of NEE vertices), trained on the octree's robust densities
// (Sec. 5 provides the targets; the model itself is not in the paper).
//
// Model: 80 encoded inputs (normalised point q, normal n, and sin/cos of
// 2^f pi c for the six coordinates c and octaves f = 0..5, two zero pads)
// -> 64 -> 64 -> 64 (ReLU) -> 1, output log rho = mu + sigma * y.
//
// gfx950 mapping.  The three 64-wide layers run on the matrix cores, bf16
// operands and FP32 accumulation: inference on v_mfma_f32_16x16x32_bf16
// (v_mfma_f32_16x16x16_bf16 for the last 16 inputs of layer 1), training
// on v_mfma_f32_16x16x16_bf16 (its loss came out wrong with the 16 x 16 x 32
// form in the training kernel under this toolchain, while inference with it
// matches the reference).  A wave
// evaluates 16 samples at a time with the transposed product
//     Z^T (64 x 16) = W^T (64 x K) . X^T (K x 16),
// so the weights are the A operand and the samples the B operand.  The
// accumulator of output block ob holds, in lane l, features 16 ob +
// 4 (l / 16) + i (i = 0..3) of sample l % 16 -- exactly the B-operand
// layout of the next layer's k-block ob, so layers chain in registers
// without any transpose.  The backward data pass uses A = W the same way.
// Weight gradients are K = batch GEMMs over feature-major bf16 stores of
// the activations and deltas.  Weights are kept as FP32 master copies
// (Adam) and re-packed after every step into bf16 operand fragments (each
// lane's four values contiguous), which the kernels stage in LDS.
#include <algorithm>

#include "neb_device.h"
#include "neb_mlp.h"

namespace neb {

typedef short bf16x4 __attribute__((ext_vector_type(4)));  // bf16 bit patterns
typedef short bf16x8b __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// round to nearest, ties to even.  (gfx950's v_cvt_pk_bf16_f32 rounds the
// same way, but with this toolchain its results fed to the 16 x 16 x 32
// product below gave wrong outputs, while each alone was right; the integer
// rounding is kept.)
__device__ __forceinline__ uint16_t to_bf16(float x) {
    uint32_t b = __float_as_uint(x);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16x4 pack4(float a, float b, float c, float d) {
    bf16x4 r;
    r[0] = (short)to_bf16(a);
    r[1] = (short)to_bf16(b);
    r[2] = (short)to_bf16(c);
    r[3] = (short)to_bf16(d);
    return r;
}

// 16 x 16 x 16 product (four k per lane)
__device__ __forceinline__ f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// 16 x 16 x 32 product of gfx950 (eight k per lane, twice the k of the
// instruction above in the same issue time).  The eight k of lane l are
// the four of the first 16 x 16 x 16 fragment pair (a0, b0) followed by the
// four of the second (a1, b1): the product sums the same terms as the two
// 16 x 16 x 16 products, the reduction only runs over a permuted k.
__device__ __forceinline__ f32x4 mfma2(bf16x4 a0, bf16x4 a1, bf16x4 b0, bf16x4 b1, f32x4 c) {
    const bf16x8b a = {a0[0], a0[1], a0[2], a0[3], a1[0], a1[1], a1[2], a1[3]};
    const bf16x8b b = {b0[0], b0[1], b0[2], b0[3], b1[0], b1[1], b1[2], b1[3]};
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
}

// Encoded input features f0 and f0 + 1 (f0 even) of (q, n): a raw pair,
// or the sine and cosine of the same 2^octave pi c, or the zero pads.
__device__ __forceinline__ void mlp_feature_pair(int f0, const float q[3], const float n[3], float& a, float& b) {
    if (f0 < 6) {
        a = f0 == 0 ? q[0] : (f0 == 2 ? q[2] : n[1]);
        b = f0 == 0 ? q[1] : (f0 == 2 ? n[0] : n[2]);
    } else if (f0 < kMlpEnc) {
        int c = (f0 - 6) / 12, oct = ((f0 - 6) % 12) >> 1;
        float x = c == 0 ? q[0] : c == 1 ? q[1] : c == 2 ? q[2] : c == 3 ? n[0] : c == 4 ? n[1] : n[2];
        sincospif((float)(1 << oct) * x, &a, &b);  // exact power-of-two scale
    } else {
        a = 0.f;
        b = 0.f;
    }
}

// fragment blob offsets (in bf16 elements)
constexpr int kFragF1 = 0;                              // W1^T: 4 ob x 5 ks x 64 lanes x 4
constexpr int kFragF2 = kFragF1 + 4 * 5 * 256;          // W2^T: 4 x 4 x 256
constexpr int kFragF3 = kFragF2 + 4 * 4 * 256;          // W3^T
constexpr int kFragB2 = kFragF3 + 4 * 4 * 256;          // W2 (backward): 4 kb x 4 nb x 256
constexpr int kFragB3 = kFragB2 + 4 * 4 * 256;          // W3 (backward)
constexpr int kFragFwd = kFragB2;                       // forward part
constexpr int kFragAll = kFragB3 + 4 * 4 * 256;         // 21504

// fragment index of W_l[k][n] in the forward (W^T as A) and backward (W as A) blobs
__device__ __forceinline__ int frag_fwd(int k, int n, int KS) {
    int ob = n >> 4, ks = k >> 4, lane = (n & 15) + 16 * ((k & 15) >> 2);
    return ((ob * KS + ks) * 64 + lane) * 4 + (k & 3);
}
__device__ __forceinline__ int frag_bwd(int k, int n) {
    int kb = k >> 4, nb = n >> 4, lane = (k & 15) + 16 * ((n & 15) >> 2);
    return ((kb * 4 + nb) * 64 + lane) * 4 + (n & 3);
}

// one parameter's bf16 copies into the blob (weights of layers 1..3 only)
__device__ __forceinline__ void pack_param(uint16_t* blob, int p, float w) {
    if (p < kMlpB1) {
        int k = p / kMlpWidth, n = p % kMlpWidth;
        blob[kFragF1 + frag_fwd(k, n, 5)] = to_bf16(w);
    } else if (p >= kMlpW2 && p < kMlpB2) {
        int e = p - kMlpW2, k = e / kMlpWidth, n = e % kMlpWidth;
        blob[kFragF2 + frag_fwd(k, n, 4)] = to_bf16(w);
        blob[kFragB2 + frag_bwd(k, n)] = to_bf16(w);
    } else if (p >= kMlpW3 && p < kMlpB3) {
        int e = p - kMlpW3, k = e / kMlpWidth, n = e % kMlpWidth;
        blob[kFragF3 + frag_fwd(k, n, 4)] = to_bf16(w);
        blob[kFragB3 + frag_bwd(k, n)] = to_bf16(w);
    }
}

__global__ void k_mlp_pack(const float* __restrict__ theta, uint16_t* __restrict__ blob) {
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < kMlpParams; p += gridDim.x * blockDim.x)
        pack_param(blob, p, theta[p]);
}

__device__ __forceinline__ void stage_blob(const uint16_t* __restrict__ blob, uint16_t* lds, int n) {
    const uint4* src = reinterpret_cast<const uint4*>(blob);
    uint4* dst = reinterpret_cast<uint4*>(lds);
    for (int i = threadIdx.x; i < n / 8; i += blockDim.x) dst[i] = src[i];
    __syncthreads();
}

__device__ __forceinline__ bf16x4 frag(const uint16_t* lds, int base, int idx, int lane) {
    return *reinterpret_cast<const bf16x4*>(lds + base + (idx * 64 + lane) * 4);
}

// Inputs of one sample.  Sources: float3 arrays of normalised points (or
// positions to normalise with an octree's box) and normals, with strides.
struct MlpInput {
    const float* pos;
    int pos_stride;
    const float* nrm;
    int nrm_stride;
    const int32_t* n_dev;  // item count in device memory (or null)
    int32_t n_host;        // capacity / count
    int normalize;         // 1: q = (pos - min_bound) * size_inv, clamped to [0, 1)
    float min_bound[3], size_inv[3];
};

__device__ __forceinline__ void load_input(const MlpInput& in, int i, float q[3], float n[3]) {
    const float* p = in.pos + (size_t)in.pos_stride * i;
    const float* m = in.nrm + (size_t)in.nrm_stride * i;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float v = p[c];
        if (in.normalize) {
            v = __fmul_rn(__fsub_rn(v, in.min_bound[c]), in.size_inv[c]);
            v = fminf(fmaxf(v, 0.f), 0.99999994f);
        }
        q[c] = v;
        n[c] = m[c];
    }
}

// Forward pass of one 16-sample tile.  Lane l works on sample l % 16 and
// holds features 16 ob + 4 g + i (g = l / 16) of every layer.  Outputs:
// z (pre-activations, FP32) of the three hidden layers and y.
struct TileFwd {
    f32x4 z1[4], z2[4], z3[4];
    bf16x4 x[5];  // encoded input, bf16
    float y;
};

// kK32: the layer products on the 16 x 16 x 32 instruction (inference);
// else on 16 x 16 x 16 (training: with the 16 x 16 x 32 form its loss came
// out wrong under this toolchain, see below)
template <bool kK32>
__device__ __forceinline__ void tile_forward(const uint16_t* lds, const float* __restrict__ theta, const float q[3],
                                             const float n[3], TileFwd& T) {
    const int lane = threadIdx.x & 63, g = lane >> 4;
#pragma unroll
    for (int ks = 0; ks < 5; ++ks) {
        int f = 16 * ks + 4 * g;
        float a0, a1, a2, a3;
        mlp_feature_pair(f, q, n, a0, a1);
        mlp_feature_pair(f + 2, q, n, a2, a3);
        T.x[ks] = pack4(a0, a1, a2, a3);
    }
    // layer 1
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        if (kK32) {
#pragma unroll
            for (int ks = 0; ks < 4; ks += 2)
                acc = mfma2(frag(lds, kFragF1, ob * 5 + ks, lane), frag(lds, kFragF1, ob * 5 + ks + 1, lane), T.x[ks],
                            T.x[ks + 1], acc);
            acc = mfma(frag(lds, kFragF1, ob * 5 + 4, lane), T.x[4], acc);
        } else {
#pragma unroll
            for (int ks = 0; ks < 5; ++ks) acc = mfma(frag(lds, kFragF1, ob * 5 + ks, lane), T.x[ks], acc);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i] += theta[kMlpB1 + 16 * ob + 4 * g + i];
        T.z1[ob] = acc;
    }
    bf16x4 h[4];
#pragma unroll
    for (int ob = 0; ob < 4; ++ob)
        h[ob] = pack4(fmaxf(T.z1[ob][0], 0.f), fmaxf(T.z1[ob][1], 0.f), fmaxf(T.z1[ob][2], 0.f),
                      fmaxf(T.z1[ob][3], 0.f));
    // layer 2
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 4; ks += kK32 ? 2 : 1)
            acc = kK32 ? mfma2(frag(lds, kFragF2, ob * 4 + ks, lane), frag(lds, kFragF2, ob * 4 + ks + 1, lane), h[ks],
                               h[ks + 1], acc)
                       : mfma(frag(lds, kFragF2, ob * 4 + ks, lane), h[ks], acc);
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i] += theta[kMlpB2 + 16 * ob + 4 * g + i];
        T.z2[ob] = acc;
    }
#pragma unroll
    for (int ob = 0; ob < 4; ++ob)
        h[ob] = pack4(fmaxf(T.z2[ob][0], 0.f), fmaxf(T.z2[ob][1], 0.f), fmaxf(T.z2[ob][2], 0.f),
                      fmaxf(T.z2[ob][3], 0.f));
    // layer 3 and the linear output (FP32 dot product over the lane's 16 features)
    float part = 0.f;
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 4; ks += kK32 ? 2 : 1)
            acc = kK32 ? mfma2(frag(lds, kFragF3, ob * 4 + ks, lane), frag(lds, kFragF3, ob * 4 + ks + 1, lane), h[ks],
                               h[ks + 1], acc)
                       : mfma(frag(lds, kFragF3, ob * 4 + ks, lane), h[ks], acc);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            acc[i] += theta[kMlpB3 + 16 * ob + 4 * g + i];
            part += theta[kMlpW4 + 16 * ob + 4 * g + i] * fmaxf(acc[i], 0.f);
        }
        T.z3[ob] = acc;
    }
    part += __shfl_xor(part, 16, 64);
    part += __shfl_xor(part, 32, 64);
    T.y = part + theta[kMlpB4];
}

// Inference: out[i] = log rho (mode 0) or rho = exp(log rho) (mode 1).
__global__ void __launch_bounds__(256) k_mlp_infer(const uint16_t* __restrict__ blob, const float* __restrict__ theta,
                                                   const MlpNorm* norm, MlpInput in, float* __restrict__ out,
                                                   int mode) {
    __shared__ __attribute__((aligned(16))) uint16_t lds[kFragFwd];
    stage_blob(blob, lds, kFragFwd);
    const int lane = threadIdx.x & 63, s = lane & 15;
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, n_waves = (gridDim.x * blockDim.x) >> 6;
    const int n = in.n_dev ? min(*in.n_dev, in.n_host) : in.n_host;
    const float mu = norm->mu, sigma = norm->sigma;
    for (int base = wave * 16; base < n; base += n_waves * 16) {
        int i = base + s;
        float q[3] = {0.f, 0.f, 0.f}, nn[3] = {0.f, 0.f, 1.f};
        if (i < n) load_input(in, i, q, nn);
        TileFwd T;
        tile_forward<true>(lds, theta, q, nn, T);
        if (lane < 16 && i < n) {
            float lr = mu + sigma * T.y;
            out[i] = mode ? __expf(lr) : lr;
        }
    }
}

// Training batch: items [0, n) of the given arrays, or n draws (with
// replacement, Philox) from a pool whose size is in device memory.
struct MlpBatch {
    MlpInput in;
    const float* target;       // log rho per item of in
    int32_t n;                 // batch size
    int32_t sample;            // 1: draw from the pool
    uint32_t k0, k1, step;     // Philox key and counter word for the draws
};

// per-wave partial sums of the small gradients: b1, b2, b3, w4 (64 each),
// b4, loss
constexpr int kPartStride = 4 * kMlpWidth + 2;
// Activations and deltas of a batch, tile-major: per 16-sample tile 400 rows
// of 16 bf16 (X rows 0..79, H1, H2, D1, D2, D3 64 rows each), so a wave
// writes whole cache lines and a 16 x 16 operand fragment is 8 contiguous
// bytes per lane.
constexpr int kRowsX = 0, kRowsH1 = kMlpIn, kRowsH2 = kRowsH1 + kMlpWidth, kRowsD1 = kRowsH2 + kMlpWidth,
              kRowsD2 = kRowsD1 + kMlpWidth, kRowsD3 = kRowsD2 + kMlpWidth, kRowsTile = kRowsD3 + kMlpWidth;

// Forward, output gradient, backward data pass, the wave's partial sums of
// the bias and output-layer gradients and of the loss (plain stores, summed
// by k_mlp_wgrad), and the tile-major bf16 stores the weight-gradient GEMMs
// read.
__global__ void __launch_bounds__(256) k_mlp_train_fb(const uint16_t* __restrict__ blob,
                                                      const float* __restrict__ theta, const MlpNorm* norm,
                                                      MlpBatch B, uint16_t* __restrict__ acts, int npad,
                                                      float* __restrict__ part) {
    __shared__ __attribute__((aligned(16))) uint16_t lds[kFragAll];
    stage_blob(blob, lds, kFragAll);
    const int lane = threadIdx.x & 63, s = lane & 15, g = lane >> 4;
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, n_waves = (gridDim.x * blockDim.x) >> 6;
    const float mu = norm->mu, inv_sigma = 1.0f / norm->sigma;
    const float inv_n = 2.0f / (float)B.n;
    float gb1[16], gb2[16], gb3[16], gw4[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) gb1[k] = gb2[k] = gb3[k] = gw4[k] = 0.f;
    float gb4 = 0.f, lsum = 0.f;
    int pool = B.sample ? (B.in.n_dev ? min(*B.in.n_dev, B.in.n_host) : B.in.n_host) : B.n;
    for (int base = wave * 16; base < npad; base += n_waves * 16) {
        int j = base + s;
        bool live = j < B.n && pool > 0;
        float q[3] = {0.f, 0.f, 0.f}, nn[3] = {0.f, 0.f, 1.f}, t = 0.f;
        if (live) {
            int item = j;
            if (B.sample) {
                uint4 r = philox10(make_uint4((uint32_t)j, B.step, 0u, kTagMlp), B.k0, B.k1);
                item = (int)(((uint64_t)r.x * (uint64_t)pool) >> 32);
            }
            load_input(B.in, item, q, nn);
            t = (B.target[item] - mu) * inv_sigma;
        }
        TileFwd T;
        tile_forward<false>(lds, theta, q, nn, T);
        float e = live ? T.y - t : 0.f;
        float dy = e * inv_n;
        if (g == 0) {
            lsum += e * e;
            gb4 += dy;
        }
        // output layer and delta 3
        bf16x4 d3b[4];
        f32x4 d3[4];
#pragma unroll
        for (int ob = 0; ob < 4; ++ob) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                int f = 16 * ob + 4 * g + i;
                float h3 = fmaxf(T.z3[ob][i], 0.f);
                gw4[4 * ob + i] += dy * h3;
                d3[ob][i] = T.z3[ob][i] > 0.f ? dy * theta[kMlpW4 + f] : 0.f;
                gb3[4 * ob + i] += d3[ob][i];
            }
            d3b[ob] = pack4(d3[ob][0], d3[ob][1], d3[ob][2], d3[ob][3]);
        }
        // delta 2 = (W3 d3) . [z2 > 0]
        bf16x4 d2b[4];
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) acc = mfma(frag(lds, kFragB3, kb * 4 + nb, lane), d3b[nb], acc);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                acc[i] = T.z2[kb][i] > 0.f ? acc[i] : 0.f;
                gb2[4 * kb + i] += acc[i];
            }
            d2b[kb] = pack4(acc[0], acc[1], acc[2], acc[3]);
        }
        // delta 1 = (W2 d2) . [z1 > 0]
        bf16x4 d1b[4];
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) acc = mfma(frag(lds, kFragB2, kb * 4 + nb, lane), d2b[nb], acc);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                acc[i] = T.z1[kb][i] > 0.f ? acc[i] : 0.f;
                gb1[4 * kb + i] += acc[i];
            }
            d1b[kb] = pack4(acc[0], acc[1], acc[2], acc[3]);
        }
        // tile-major stores for the weight gradients
        uint16_t* tile = acts + (size_t)(base >> 4) * (kRowsTile * 16) + s;
#pragma unroll
        for (int ks = 0; ks < 5; ++ks)
#pragma unroll
            for (int i = 0; i < 4; ++i) tile[(kRowsX + 16 * ks + 4 * g + i) * 16] = (uint16_t)T.x[ks][i];
#pragma unroll
        for (int ob = 0; ob < 4; ++ob)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int f = 16 * ob + 4 * g + i;
                tile[(kRowsH1 + f) * 16] = to_bf16(fmaxf(T.z1[ob][i], 0.f));
                tile[(kRowsH2 + f) * 16] = to_bf16(fmaxf(T.z2[ob][i], 0.f));
                tile[(kRowsD1 + f) * 16] = (uint16_t)d1b[ob][i];
                tile[(kRowsD2 + f) * 16] = (uint16_t)d2b[ob][i];
                tile[(kRowsD3 + f) * 16] = (uint16_t)d3b[ob][i];
            }
    }
    // sum the per-sample partials over the 16 sample lanes of each group
#pragma unroll
    for (int k = 0; k < 16; ++k) {
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) {
            gb1[k] += __shfl_xor(gb1[k], off, 64);
            gb2[k] += __shfl_xor(gb2[k], off, 64);
            gb3[k] += __shfl_xor(gb3[k], off, 64);
            gw4[k] += __shfl_xor(gw4[k], off, 64);
        }
    }
    for (int off = 1; off < 16; off <<= 1) {
        gb4 += __shfl_xor(gb4, off, 64);
        lsum += __shfl_xor(lsum, off, 64);
    }
    float* P = part + (size_t)wave * kPartStride;
    if (s == 0) {
#pragma unroll
        for (int ob = 0; ob < 4; ++ob)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                int f = 16 * ob + 4 * g + i;
                P[f] = gb1[4 * ob + i];
                P[kMlpWidth + f] = gb2[4 * ob + i];
                P[2 * kMlpWidth + f] = gb3[4 * ob + i];
                P[3 * kMlpWidth + f] = gw4[4 * ob + i];
            }
        if (g == 0) {
            P[4 * kMlpWidth] = gb4;
            P[4 * kMlpWidth + 1] = lsum;
        }
    }
}

// Weight gradients dW_l[k][n] = sum_s Hin[k][s] D[n][s] as K = batch GEMMs.
// Block (layer, slice) is one wave that reads each row of its slice of the
// batch once (per 16-sample tile: the layer's delta rows as A fragments,
// its input rows as B fragments) and accumulates every 16 x 16 tile of
// dW^T of that layer in registers, then stores them as its slice's part
// (k_mlp_wreduce sums the slices: per-lane atomics of every wave on the
// 13 312 weights took as long as the products).  Blocks past the three layers sum the
// training kernel's per-wave partials, each slice a share of the waves.
constexpr int kWgSlice = 512;
constexpr int kWgLayers = 3;
constexpr int kWgReduce = (kPartStride + 63) / 64;
// a slice's partial weight gradients: W1^T rows 0..79 (the input's two pads
// included, never read), then W2^T and W3^T, k-major (k * 64 + n)
constexpr int kWPartW2 = (kMlpEnc + 2) * kMlpWidth;
constexpr int kWPartW3 = kWPartW2 + kMlpWidth * kMlpWidth;
constexpr int kWPart = kWPartW3 + kMlpWidth * kMlpWidth;

template <int KB>
__device__ __forceinline__ void wgrad_layer(const uint16_t* __restrict__ acts, int t_begin, int t_end, int hrow,
                                            int drow, int kmax, float* __restrict__ wpart) {
    const int lane = threadIdx.x, g = lane >> 4, r = lane & 15;
    constexpr size_t kTile = (size_t)kRowsTile * 16;
    f32x4 acc[4][KB];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) acc[nb][kb] = f32x4{0.f, 0.f, 0.f, 0.f};
    const uint16_t* abase = acts + (drow + r) * 16 + 4 * g;
    const uint16_t* bbase = acts + (hrow + r) * 16 + 4 * g;
    // U tiles' fragments are loaded before any of them is used
    constexpr int U = 8;
    int t = t_begin;
    for (; t + U <= t_end; t += U) {
        bf16x4 a[U][4], b[U][KB];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const size_t off = (size_t)(t + u) * kTile;
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) a[u][nb] = *reinterpret_cast<const bf16x4*>(abase + off + 16 * 16 * nb);
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) b[u][kb] = *reinterpret_cast<const bf16x4*>(bbase + off + 16 * 16 * kb);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int nb = 0; nb < 4; ++nb)
#pragma unroll
                for (int kb = 0; kb < KB; ++kb) acc[nb][kb] = mfma(a[u][nb], b[u][kb], acc[nb][kb]);
    }
    for (; t < t_end; ++t) {
        const size_t off = (size_t)t * kTile;
        bf16x4 a[4], b[KB];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) a[nb] = *reinterpret_cast<const bf16x4*>(abase + off + 16 * 16 * nb);
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) b[kb] = *reinterpret_cast<const bf16x4*>(bbase + off + 16 * 16 * kb);
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) acc[nb][kb] = mfma(a[nb], b[kb], acc[nb][kb]);
    }
    // acc[nb][kb][i] = dW^T[16 nb + 4 g + i][16 kb + r]: this slice's part,
    // four consecutive n per store
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
        const int k = 16 * kb + r;
        if (k >= kmax) continue;  // the zero pads of the input carry no gradient
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
            *reinterpret_cast<f32x4*>(wpart + k * kMlpWidth + 16 * nb + 4 * g) = acc[nb][kb];
    }
}

__global__ void __launch_bounds__(64) k_mlp_wgrad(const uint16_t* __restrict__ acts, int npad,
                                                  float* __restrict__ grad, const float* __restrict__ part,
                                                  int n_waves, float* loss_sum, float* __restrict__ wpart) {
    const int lane = threadIdx.x;
    const int job = blockIdx.x;
    const int slice = blockIdx.y;
    if (job >= kWgLayers) {
        const int j = (job - kWgLayers) * 64 + lane;
        if (j >= kPartStride) return;
        const int share = (n_waves + gridDim.y - 1) / gridDim.y;
        const int w0 = slice * share, w1 = min(n_waves, w0 + share);
        if (w0 >= w1) return;
        float sum = 0.f;
        for (int w = w0; w < w1; ++w) sum += part[(size_t)w * kPartStride + j];
        if (j < 4 * kMlpWidth) {
            const int off = j < kMlpWidth ? kMlpB1 : (j < 2 * kMlpWidth ? kMlpB2 : (j < 3 * kMlpWidth ? kMlpB3 : kMlpW4));
            atomicAdd(grad + off + (j % kMlpWidth), sum);
        } else if (j == 4 * kMlpWidth) {
            atomicAdd(grad + kMlpB4, sum);
        } else {
            atomicAdd(loss_sum, sum);
        }
        return;
    }
    const int t_begin = (slice * kWgSlice) >> 4, t_end = min(npad, (slice + 1) * kWgSlice) >> 4;
    float* wp = wpart + (size_t)slice * kWPart;
    if (job == 0) wgrad_layer<5>(acts, t_begin, t_end, kRowsX, kRowsD1, kMlpEnc, wp);
    else if (job == 1) wgrad_layer<4>(acts, t_begin, t_end, kRowsH1, kRowsD2, kMlpWidth, wp + kWPartW2);
    else wgrad_layer<4>(acts, t_begin, t_end, kRowsH2, kRowsD3, kMlpWidth, wp + kWPartW3);
}

// The weight gradients: block (x, y) sums slices kWrGroup y .. + kWrGroup - 1
// of weights 256 x .. 256 x + 255 (one thread per weight, the slices' rows
// read coalesced, their loads in flight together) and adds the sum to grad.
constexpr int kWrGroup = 8;
__global__ void __launch_bounds__(256) k_mlp_wreduce(const float* __restrict__ wpart, int n_slices,
                                                     float* __restrict__ grad) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= kWPart) return;
    int dst;
    if (j < kWPartW2) {
        if (j >= kMlpEnc * kMlpWidth) return;  // the pads' rows
        dst = kMlpW1 + j;
    } else {
        dst = (j < kWPartW3 ? kMlpW2 + (j - kWPartW2) : kMlpW3 + (j - kWPartW3));
    }
    const int s0 = blockIdx.y * kWrGroup;
    float v[kWrGroup];
#pragma unroll
    for (int u = 0; u < kWrGroup; ++u) v[u] = s0 + u < n_slices ? wpart[(size_t)(s0 + u) * kWPart + j] : 0.f;
    float sum = 0.f;
#pragma unroll
    for (int u = 0; u < kWrGroup; ++u) sum += v[u];
    atomicAdd(grad + dst, sum);
}

// One Adam step on the FP32 master parameters; re-packs the bf16 operand
// fragments and clears the gradient for the next step.
__global__ void k_mlp_adam(float* __restrict__ theta, float* __restrict__ m, float* __restrict__ v,
                           float* __restrict__ grad, uint16_t* __restrict__ blob, MlpAdam A) {
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < kMlpParams; p += gridDim.x * blockDim.x) {
        float gr = grad[p];
        grad[p] = 0.f;
        float mm = A.beta1 * m[p] + (1.0f - A.beta1) * gr;
        float vv = A.beta2 * v[p] + (1.0f - A.beta2) * gr * gr;
        m[p] = mm;
        v[p] = vv;
        float mh = mm / A.bias1, vh = vv / A.bias2;
        float w = theta[p] - A.lr * mh / (sqrtf(vh) + A.eps);
        theta[p] = w;
        pack_param(blob, p, w);
    }
}

__global__ void k_mlp_set_norm(MlpNorm* norm, float mu, float sigma) {
    norm->mu = mu;
    norm->sigma = sigma;
}

// mean and standard deviation of the pool's targets (FP64 sums)
__global__ void k_mlp_moments(const float* __restrict__ t, const int32_t* n_dev, int32_t n_host, double* sums) {
    int n = n_dev ? min(*n_dev, n_host) : n_host;
    double a = 0.0, b = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double x = t[i];
        a += x;
        b += x * x;
    }
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off, 64);
        b += __shfl_xor(b, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(sums, a);
        atomicAdd(sums + 1, b);
    }
}

__global__ void k_mlp_norm_from_moments(const double* sums, const int32_t* n_dev, int32_t n_host, MlpNorm* norm) {
    int n = n_dev ? min(*n_dev, n_host) : n_host;
    if (n <= 0) {
        norm->mu = 0.f;
        norm->sigma = 1.f;
        return;
    }
    double mean = sums[0] / n;
    double var = fmax(sums[1] / n - mean * mean, 0.0);
    norm->mu = (float)mean;
    norm->sigma = (float)fmax(sqrt(var), 1e-3);
}

__global__ void k_mlp_zero_f64(double* p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0.0;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static int blocks_for(int64_t n, int per_block, int cap) {
    int64_t b = (n + per_block - 1) / per_block;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

hipError_t mlp_alloc(Mlp& m, int32_t max_batch) {
    m.max_batch = max_batch;
    m.npad = (max_batch + 15) & ~15;
    hipError_t e = hipMalloc(&m.theta, 4 * (size_t)kMlpParams);
    if (e == hipSuccess) e = hipMalloc(&m.m, 4 * (size_t)kMlpParams);
    if (e == hipSuccess) e = hipMalloc(&m.v, 4 * (size_t)kMlpParams);
    if (e == hipSuccess) e = hipMalloc(&m.grad, 4 * (size_t)kMlpParams);
    if (e == hipSuccess) e = hipMalloc(&m.blob, 2 * (size_t)kFragAll);
    if (e == hipSuccess) e = hipMalloc(&m.norm, sizeof(MlpNorm));
    if (e == hipSuccess) e = hipMalloc(&m.loss, sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&m.moments, 2 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&m.acts, 2 * (size_t)(kMlpIn + 5 * kMlpWidth) * m.npad);
    // one partial row per wave of the training kernel at its largest grid
    m.max_waves = 4 * std::max(1, std::min((m.npad / 16 + 15) / 16, 1 << 16));
    if (e == hipSuccess) e = hipMalloc(&m.part, 4 * (size_t)kPartStride * m.max_waves);
    m.max_slices = (m.npad + kWgSlice - 1) / kWgSlice;
    if (e == hipSuccess) e = hipMalloc(&m.wpart, 4 * (size_t)kWPart * m.max_slices);
    return e;
}

void mlp_free(Mlp& m) {
    void* ps[] = {m.theta, m.m, m.v, m.grad, m.blob, m.norm, m.loss, m.moments, m.acts, m.part, m.wpart};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    m = Mlp();
}

hipError_t mlp_set_weights(Mlp& m, const float* host_theta, hipStream_t s) {
    hipError_t e = hipMemcpyAsync(m.theta, host_theta, 4 * (size_t)kMlpParams, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    e = hipMemsetAsync(m.m, 0, 4 * (size_t)kMlpParams, s);
    if (e == hipSuccess) e = hipMemsetAsync(m.v, 0, 4 * (size_t)kMlpParams, s);
    if (e == hipSuccess) e = hipMemsetAsync(m.grad, 0, 4 * (size_t)kMlpParams, s);
    if (e == hipSuccess) e = hipMemsetAsync(m.blob, 0, 2 * (size_t)kFragAll, s);
    if (e == hipSuccess) e = hipMemsetAsync(m.loss, 0, sizeof(float), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_pack, dim3(blocks_for(kMlpParams, 256, 64)), dim3(256), 0, s, (const float*)m.theta,
                       m.blob);
    m.step = 0;
    return hipGetLastError();
}

hipError_t mlp_set_norm(Mlp& m, float mu, float sigma, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_set_norm, dim3(1), dim3(1), 0, s, m.norm, mu, sigma);
    return hipGetLastError();
}

hipError_t mlp_norm_from_pool(Mlp& m, const float* target, const int32_t* n_dev, int32_t n_host, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_zero_f64, dim3(1), dim3(64), 0, s, m.moments, 2);
    hipLaunchKernelGGL(k_mlp_moments, dim3(blocks_for(n_host, 256, 1024)), dim3(256), 0, s, target, n_dev, n_host,
                       m.moments);
    hipLaunchKernelGGL(k_mlp_norm_from_moments, dim3(1), dim3(1), 0, s, (const double*)m.moments, n_dev, n_host,
                       m.norm);
    return hipGetLastError();
}

static MlpInput make_input(const float* pos, int pos_stride, const float* nrm, int nrm_stride, const int32_t* n_dev,
                           int32_t n_host, const OctParams* box) {
    MlpInput in;
    in.pos = pos;
    in.pos_stride = pos_stride;
    in.nrm = nrm;
    in.nrm_stride = nrm_stride;
    in.n_dev = n_dev;
    in.n_host = n_host;
    in.normalize = box ? 1 : 0;
    for (int c = 0; c < 3; ++c) {
        in.min_bound[c] = box ? box->min_bound[c] : 0.f;
        in.size_inv[c] = box ? box->size_inv[c] : 1.f;
    }
    return in;
}

hipError_t mlp_infer(const Mlp& m, const float* pos, int pos_stride, const float* nrm, int nrm_stride,
                     const int32_t* n_dev, int32_t n_host, const OctParams* box, float* out, int mode,
                     hipStream_t s) {
    if (n_host <= 0) return hipSuccess;
    MlpInput in = make_input(pos, pos_stride, nrm, nrm_stride, n_dev, n_host, box);
    hipLaunchKernelGGL(k_mlp_infer, dim3(blocks_for((n_host + 15) / 16, 4, 2048)), dim3(256), 0, s,
                       (const uint16_t*)m.blob, (const float*)m.theta, (const MlpNorm*)m.norm, in, out, mode);
    return hipGetLastError();
}

// gradient of the mean loss over one batch into m.grad (accumulated; the
// Adam step clears it) and the loss sum into m.loss
hipError_t mlp_gradient(Mlp& m, const float* pos, int pos_stride, const float* nrm, int nrm_stride,
                        const float* target, const int32_t* pool_dev, int32_t pool_host, int32_t batch, int sample,
                        uint32_t k0, uint32_t k1, const OctParams* box, hipStream_t s) {
    if (batch <= 0 || batch > m.max_batch) return hipErrorInvalidValue;
    MlpBatch B;
    B.in = make_input(pos, pos_stride, nrm, nrm_stride, pool_dev, pool_host, box);
    B.target = target;
    B.n = batch;
    B.sample = sample;
    B.k0 = k0;
    B.k1 = k1;
    B.step = (uint32_t)m.step;
    const int npad = (batch + 15) & ~15;
    const int tiles = npad / 16;
    const int blocks = blocks_for(tiles, 16, 1 << 16);
    const int n_waves = 4 * blocks;
    if (n_waves > m.max_waves) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mlp_train_fb, dim3(blocks), dim3(256), 0, s, (const uint16_t*)m.blob, (const float*)m.theta,
                       (const MlpNorm*)m.norm, B, m.acts, npad, m.part);
    const int slices = (npad + kWgSlice - 1) / kWgSlice;
    if (slices > m.max_slices) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mlp_wgrad, dim3(kWgLayers + kWgReduce, slices), dim3(64), 0, s, (const uint16_t*)m.acts,
                       npad, m.grad, (const float*)m.part, n_waves, m.loss, m.wpart);
    hipLaunchKernelGGL(k_mlp_wreduce, dim3((kWPart + 255) / 256, (slices + kWrGroup - 1) / kWrGroup), dim3(256), 0, s,
                       (const float*)m.wpart, slices, m.grad);
    return hipGetLastError();
}

hipError_t mlp_adam(Mlp& m, float lr, float beta1, float beta2, float eps, hipStream_t s) {
    m.step += 1;
    MlpAdam A;
    A.lr = lr;
    A.beta1 = beta1;
    A.beta2 = beta2;
    A.eps = eps;
    A.bias1 = (float)(1.0 - std::pow((double)beta1, (double)m.step));
    A.bias2 = (float)(1.0 - std::pow((double)beta2, (double)m.step));
    hipLaunchKernelGGL(k_mlp_adam, dim3(blocks_for(kMlpParams, 256, 64)), dim3(256), 0, s, m.theta, m.m, m.v, m.grad,
                       m.blob, A);
    return hipGetLastError();
}

}  // namespace neb
