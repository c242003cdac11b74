// Internal launch interface of the learned-shrinkage kernels (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace shear {

// One 3x3 layer launch. Every layer reads bfloat16 channel-last input: the
// packed z [b][y][x][shrink_cinp(K)] (launch_pack_z) for layer 0, hidden
// activations [b][y][x][32] for layers 1 and 2. Layers 0 and 1 write
// relu(conv + bias) as bfloat16 channel-last activations (out_bf); layer 2
// writes the shrunk FP32 coefficients out_f (coef kept where
// |coef * scale| >= softplus(conv + bias), plane `lowpass` kept whole) and,
// if non-null, the thresholds tau.
struct ConvArgs {
    const void* in;
    const unsigned short* W;  // packed bfloat16 weights [coutp][9][cinp]
    const float* bias;
    const float* scale;       // [B][K] 1 / (sigma_b RMS_k)
    const float* coef;        // layer 2: the coefficients (B x K x N x M)
    void* out_bf;
    float* out_f;
    float* tau;
    int N, M;
    int cin, cout;            // real channel counts (K for the coefficient side)
    int lowpass;
    // training
    const float* coef2;                // layer 2 training: coefficients of the clean images
    const unsigned short* mask_act;    // backward data: saved activation whose relu mask applies
    float* loss;                       // layer 2 training: sum of squared residuals (added)
    float loss_scale, temperature;
    int cus;  // compute units of the device (grid of the persistent first layer)
};

// Weight-gradient launch: dy bf16 channel-last with dy_ch channels; input x bf16 channel-last (the packed z
// for layer 0, else a hidden activation); per-block partials to part.
struct WgradArgs {
    const unsigned short* dy;
    int dy_ch;
    const unsigned short* xb;
    float* part;
    int batch, N, M;
};

// Byte offsets of the packed parameter block of a K-filter network.
struct ShrinkLayout {
    size_t w1, w2, w3, b1, b2, b3, bytes;
};

int shrink_cinp(int K);   // padded input channels of layer 0 (32 or 64)
int shrink_coutp(int K);  // padded output channels of layer 2 (multiple of 16)
bool shrink_supported(int K, int N, int M);
ShrinkLayout shrink_layout(int K);

// FP32 natural-layout parameters (device) -> packed block (device).
hipError_t launch_shrink_pack(int K, const float* W1, const float* b1, const float* W2, const float* b2,
                              const float* W3, const float* b3, void* packed, hipStream_t st);
hipError_t launch_inv_scale(const float* sigma, const float* rms, float* out, int B, int K, hipStream_t st);
// z = bf16(c x scale) as channel-last [b][y][x][shrink_cinp(K)], zero padded (M a multiple of 32)
hipError_t launch_pack_z(const float* c, const float* scale, unsigned short* z, int K, int N, int M, int batch,
                         hipStream_t st);
// layer 0, 1, 2: inference layers; 3: last layer with the training epilogue; 4: backward data from 32
// gradient channels; 5: backward data from shrink_cinp(K) gradient channels; 6: layer 0 with its input
// staged straight from the FP32 coefficients (coef, scale, cin = K) instead of the packed z.
hipError_t launch_conv(int layer, int K, const ConvArgs& a, int batch, hipStream_t st);
// weight gradients of layer 0, 1 or 2 (partials of `blocks` blocks of 32-pixel x 8-row tiles)
hipError_t launch_wgrad(int layer, int K, const WgradArgs& a, int blocks, hipStream_t st);
hipError_t launch_wgrad_reduce(const float* part, float* dW, float* db, int nblk, int cout, int cin, int coutp, int cinp,
                               hipStream_t st);
hipError_t launch_pack_weights_t(const float* W, unsigned short* out, int cout, int cin, int rows, int cols,
                                 hipStream_t st);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps,
                       int step, hipStream_t st);

}  // namespace shear
