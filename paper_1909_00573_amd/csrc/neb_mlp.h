// Learned density model: constants, device state and host entry points
// (neb_mlp.hip).
#pragma once
#include "neb_internal.h"

namespace neb {

constexpr int kMlpIn = 80;     // encoded inputs (78 used, 2 zero pads)
constexpr int kMlpEnc = 78;
constexpr int kMlpWidth = 64;
// flat parameter layout: W1 (80 x 64, row k = input feature k), b1, W2
// (64 x 64), b2, W3, b3, w4 (64), b4
constexpr int kMlpW1 = 0;
constexpr int kMlpB1 = kMlpW1 + kMlpIn * kMlpWidth;
constexpr int kMlpW2 = kMlpB1 + kMlpWidth;
constexpr int kMlpB2 = kMlpW2 + kMlpWidth * kMlpWidth;
constexpr int kMlpW3 = kMlpB2 + kMlpWidth;
constexpr int kMlpB3 = kMlpW3 + kMlpWidth * kMlpWidth;
constexpr int kMlpW4 = kMlpB3 + kMlpWidth;
constexpr int kMlpB4 = kMlpW4 + kMlpWidth;
constexpr int kMlpParams = kMlpB4 + 1;  // 13569

struct MlpNorm {
    float mu, sigma;  // log rho = mu + sigma * y
};

struct MlpAdam {
    float lr, beta1, beta2, eps;
    float bias1, bias2;  // 1 - beta^t
};

// device state of one model
struct Mlp {
    float* theta = nullptr;    // FP32 master parameters
    float* m = nullptr;        // Adam moments
    float* v = nullptr;
    float* grad = nullptr;     // accumulated gradient (cleared by the Adam step)
    uint16_t* blob = nullptr;  // bf16 operand fragments of W1..W3
    MlpNorm* norm = nullptr;
    float* loss = nullptr;     // running sum of squared errors
    double* moments = nullptr;
    uint16_t* acts = nullptr;  // feature-major bf16 activations and deltas of one batch
    float* part = nullptr;     // per-wave partial sums of the small gradients and the loss
    float* wpart = nullptr;    // per-slice partial weight gradients of W1..W3 (summed by a second launch)
    int32_t max_batch = 0, npad = 0, max_waves = 0, max_slices = 0;
    int64_t step = 0;          // Adam steps taken
};

hipError_t mlp_alloc(Mlp& m, int32_t max_batch);
void mlp_free(Mlp& m);
hipError_t mlp_set_weights(Mlp& m, const float* host_theta, hipStream_t s);
hipError_t mlp_set_norm(Mlp& m, float mu, float sigma, hipStream_t s);
hipError_t mlp_norm_from_pool(Mlp& m, const float* target, const int32_t* n_dev, int32_t n_host, hipStream_t s);
// box == nullptr: pos holds normalised points; else positions normalised
// with the octree box.  mode 0 writes log rho, 1 writes rho.
hipError_t mlp_infer(const Mlp& m, const float* pos, int pos_stride, const float* nrm, int nrm_stride,
                     const int32_t* n_dev, int32_t n_host, const OctParams* box, float* out, int mode,
                     hipStream_t s);
hipError_t mlp_gradient(Mlp& m, const float* pos, int pos_stride, const float* nrm, int nrm_stride,
                        const float* target, const int32_t* pool_dev, int32_t pool_host, int32_t batch, int sample,
                        uint32_t k0, uint32_t k1, const OctParams* box, hipStream_t s);
hipError_t mlp_adam(Mlp& m, float lr, float beta1, float beta2, float eps, hipStream_t s);

}  // namespace neb
