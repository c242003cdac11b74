// gfx950 kernels of the learned shrinkage network (inference and training).
//
// Three 3x3 circular cross-correlations (K -> 32 -> 32 -> K channels) map the
// noise-normalised coefficients z_k = c_k / (sigma RMS_k) of a noisy image to
// per-coefficient thresholds tau = softplus(o); coefficients with |z| < tau are
// set to zero (the low-pass plane is kept). Every layer is an implicit GEMM on
// the matrix cores: pixels x (9 taps x input channels) times (9 taps x input
// channels) x output channels, bfloat16 operands, FP32 accumulation
// (v_mfma_f32_16x16x32_bf16).
//
// Lane layout of v_mfma_f32_16x16x32_bf16 (checked on the device): lane l
// holds A row l%16 and B column l%16 with k = 8(l/16) .. 8(l/16)+7, and D
// column l%16 with rows 4(l/16) .. 4(l/16)+3.
//
// A block computes a tile of TH x TW = 8 x 32 output pixels of one image for
// all output channels. Its input tile with a one-pixel halo (wrapped around
// the plane) is staged in LDS channel-last, one padded run of channels per
// pixel, so that a lane's 8 consecutive k of one tap are one 16-byte read.
// Hidden activations are stored channel-last in bfloat16: [b][y][x][32].
#include "shrink.h"

#include <hip/hip_runtime.h>

#include <algorithm>

namespace shear {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int TH = 8, TW = 32;                     // output tile (rows x cols)
constexpr int HH = TH + 2, HW = TW + 2;            // with halo
constexpr int THREADS = 256;                       // 4 wavefronts, 2 tile rows each

// round to nearest bfloat16, ties to even (finite inputs)
__device__ __forceinline__ unsigned short f2bf(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float(((unsigned)h) << 16); }

__device__ __forceinline__ float softplusf(float x) { return fmaxf(x, 0.0f) + log1pf(expf(-fabsf(x))); }

template <int CINP>
struct Pix {
    static constexpr int value = CINP + 8;  // bf16 per staged pixel: 16 bytes of padding against bank conflicts
};

template <int CINP>
constexpr size_t conv_lds_bytes() {
    return (size_t)HH * HW * Pix<CINP>::value * 2 + (size_t)TH * TW * 32 * 2;
}

// Stages the halo tile of one image: MODE 0 from FP32 channel-first coefficient
// planes (times scale[c], the noise normalisation), else from bfloat16
// channel-last activations with CINP channels.
template <int CINP, int MODE>
__device__ __forceinline__ void stage(const ConvArgs& a, unsigned short* s, int b, int y0, int x0) {
    constexpr int PIX = Pix<CINP>::value;
    const int N = a.N, M = a.M;
    if constexpr (MODE == 0) {
        const float* in = reinterpret_cast<const float*>(a.in);
        for (int i = threadIdx.x; i < CINP * HH * HW; i += THREADS) {
            const int xx = i % HW, r = i / HW, yy = r % HH, c = r / HH;
            float v = 0.0f;
            if (c < a.cin) {
                const int y = (y0 + yy - 1 + N) & (N - 1), x = (x0 + xx - 1 + M) & (M - 1);
                v = in[(((size_t)b * a.cin + c) * N + y) * M + x] * a.scale[b * a.cin + c];
            }
            s[(yy * HW + xx) * PIX + c] = f2bf(v);
        }
    } else {
        const uint4* in = reinterpret_cast<const uint4*>(a.in);
        constexpr int CH = CINP / 8;  // 16-byte chunks per pixel
        for (int i = threadIdx.x; i < HH * HW * CH; i += THREADS) {
            const int ch = i % CH, p = i / CH, xx = p % HW, yy = p / HW;
            const int y = (y0 + yy - 1 + N) & (N - 1), x = (x0 + xx - 1 + M) & (M - 1);
            const uint4 v = in[(((size_t)b * N + y) * M + x) * CH + ch];
            *reinterpret_cast<uint4*>(s + (yy * HW + xx) * PIX + ch * 8) = v;
        }
    }
}

// out[pixel][co] accumulators of a wavefront: 4 m-tiles (16 pixels of one row) x NT n-tiles.
template <int CINP, int COUTP>
__device__ __forceinline__ void mma(const ConvArgs& a, const unsigned short* s, f32x4 (&acc)[4][COUTP / 16]) {
    constexpr int PIX = Pix<CINP>::value, NT = COUTP / 16;
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    const int lr = l % 16, lk = 8 * (l / 16);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    const unsigned short* W = a.W;
#pragma unroll 1
    for (int tap = 0; tap < 9; ++tap) {
        const int dy = tap / 3, dx = tap % 3;
#pragma unroll
        for (int kc = 0; kc < CINP / 32; ++kc) {
            bf16x8 bfr[NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                bfr[nt] = *reinterpret_cast<const bf16x8*>(W + ((size_t)(nt * 16 + lr) * 9 + tap) * CINP + kc * 32 + lk);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                const int row = 2 * w + mt / 2, xs = (mt % 2) * 16;
                const bf16x8 afr =
                    *reinterpret_cast<const bf16x8*>(s + ((row + dy) * HW + xs + lr + dx) * PIX + kc * 32 + lk);
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr, bfr[nt], acc[mt][nt], 0, 0, 0);
            }
        }
    }
}

// MODE 0: z (FP32 coefficients x scale) -> relu -> bf16 activations; MODE 1: activations -> relu -> activations;
// MODE 2: activations -> o + b -> tau = softplus -> shrink of the coefficients.
template <int CINP, int COUTP, int MODE>
__global__ __launch_bounds__(THREADS) void k_conv3x3(ConvArgs a) {
    constexpr int NT = COUTP / 16;
    extern __shared__ unsigned short smem[];
    unsigned short* s_in = smem;
    unsigned short* s_out = smem + HH * HW * Pix<CINP>::value;
    const int tx = a.M / TW, ty = a.N / TH;
    const int bx = blockIdx.x % tx, by = (blockIdx.x / tx) % ty, b = blockIdx.x / (tx * ty);
    const int x0 = bx * TW, y0 = by * TH;
    stage<CINP, MODE>(a, s_in, b, y0, x0);
    __syncthreads();
    f32x4 acc[4][NT];
    mma<CINP, COUTP>(a, s_in, acc);
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    const int lr = l % 16, lm = 4 * (l / 16);
    if constexpr (MODE == 2) {
        const float* c = a.coef;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const int y = y0 + 2 * w + mt / 2, x = x0 + (mt % 2) * 16 + lm;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int k = nt * 16 + lr;
                if (k >= a.cout) continue;
                const size_t off = (((size_t)b * a.cout + k) * a.N + y) * a.M + x;
                const float4 cv = *reinterpret_cast<const float4*>(c + off);
                const float sc = a.scale[b * a.cout + k], bias = a.bias[k];
                float t[4], v[4] = {cv.x, cv.y, cv.z, cv.w}, o[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    t[i] = (k == a.lowpass) ? 0.0f : softplusf(acc[mt][nt][i] + bias);
                    o[i] = (fabsf(v[i] * sc) >= t[i]) ? v[i] : 0.0f;
                }
                *reinterpret_cast<float4*>(a.out_f + off) = make_float4(o[0], o[1], o[2], o[3]);
                if (a.tau) *reinterpret_cast<float4*>(a.tau + off) = make_float4(t[0], t[1], t[2], t[3]);
            }
        }
    } else {
        // relu(acc + bias) -> bf16 through LDS, then 16-byte channel-last stores
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const int prow = (2 * w + mt / 2) * TW + (mt % 2) * 16 + lm;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int co = nt * 16 + lr;
                const float bias = a.bias[co];
#pragma unroll
                for (int i = 0; i < 4; ++i) s_out[(prow + i) * 32 + co] = f2bf(fmaxf(acc[mt][nt][i] + bias, 0.0f));
            }
        }
        __syncthreads();
        uint4* out = reinterpret_cast<uint4*>(a.out_bf);
        for (int i = threadIdx.x; i < TH * TW * 4; i += THREADS) {
            const int ch = i % 4, p = i / 4, px = p % TW, py = p / TW;
            out[(((size_t)b * a.N + y0 + py) * a.M + x0 + px) * 4 + ch] = *reinterpret_cast<const uint4*>(s_out + p * 32 + ch * 8);
        }
    }
}

// inverse noise scale per (image, filter): 1 / (sigma_b RMS_k)
__global__ void k_inv_scale(const float* __restrict__ sigma, const float* __restrict__ rms, float* __restrict__ out,
                            int B, int K) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < B * K) out[i] = 1.0f / (sigma[i / K] * rms[i % K]);
}

// natural FP32 weights W[co][ci][3][3] -> bf16 [co][tap][ci] padded to COUTP x CINP (zeros)
__global__ void k_pack_weights(const float* __restrict__ W, unsigned short* __restrict__ out, int cout, int cin,
                               int coutp, int cinp) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= coutp * 9 * cinp) return;
    const int ci = i % cinp, tap = (i / cinp) % 9, co = i / (cinp * 9);
    out[i] = (co < cout && ci < cin) ? f2bf(W[((size_t)co * cin + ci) * 9 + tap]) : (unsigned short)0;
}

__global__ void k_pack_bias(const float* __restrict__ b, float* __restrict__ out, int n, int np) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < np) out[i] = i < n ? b[i] : 0.0f;
}

template <int CINP, int COUTP, int MODE>
hipError_t conv_t(const ConvArgs& a, int batch, hipStream_t st) {
    const void* fn = reinterpret_cast<const void*>(&k_conv3x3<CINP, COUTP, MODE>);
    const size_t lds = conv_lds_bytes<CINP>();
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const size_t blocks = (size_t)batch * (a.N / TH) * (a.M / TW);
    hipLaunchKernelGGL((k_conv3x3<CINP, COUTP, MODE>), dim3((unsigned)blocks), dim3(THREADS), lds, st, a);
    return hipGetLastError();
}

}  // namespace

int shrink_cinp(int K) { return K <= 32 ? 32 : 64; }
int shrink_coutp(int K) { return (K + 15) / 16 * 16; }
bool shrink_supported(int K, int N, int M) { return K >= 1 && K <= 64 && N >= TH && M >= TW && N % TH == 0 && M % TW == 0; }

ShrinkLayout shrink_layout(int K) {
    ShrinkLayout L;
    const int c1 = shrink_cinp(K), c3 = shrink_coutp(K);
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    size_t off = 0;
    L.w1 = off;
    off = al(off + (size_t)32 * 9 * c1 * 2);
    L.w2 = off;
    off = al(off + (size_t)32 * 9 * 32 * 2);
    L.w3 = off;
    off = al(off + (size_t)c3 * 9 * 32 * 2);
    L.b1 = off;
    off = al(off + 32 * 4);
    L.b2 = off;
    off = al(off + 32 * 4);
    L.b3 = off;
    off = al(off + (size_t)c3 * 4);
    L.bytes = off;
    return L;
}

hipError_t launch_shrink_pack(int K, const float* W1, const float* b1, const float* W2, const float* b2,
                              const float* W3, const float* b3, void* packed, hipStream_t st) {
    const ShrinkLayout L = shrink_layout(K);
    char* p = static_cast<char*>(packed);
    const int c1 = shrink_cinp(K), c3 = shrink_coutp(K);
    auto grid = [](int n) { return dim3((unsigned)((n + 255) / 256)); };
    hipLaunchKernelGGL(k_pack_weights, grid(32 * 9 * c1), dim3(256), 0, st, W1, (unsigned short*)(p + L.w1), 32, K, 32, c1);
    hipLaunchKernelGGL(k_pack_weights, grid(32 * 9 * 32), dim3(256), 0, st, W2, (unsigned short*)(p + L.w2), 32, 32, 32, 32);
    hipLaunchKernelGGL(k_pack_weights, grid(c3 * 9 * 32), dim3(256), 0, st, W3, (unsigned short*)(p + L.w3), K, 32, c3, 32);
    hipLaunchKernelGGL(k_pack_bias, grid(32), dim3(256), 0, st, b1, (float*)(p + L.b1), 32, 32);
    hipLaunchKernelGGL(k_pack_bias, grid(32), dim3(256), 0, st, b2, (float*)(p + L.b2), 32, 32);
    hipLaunchKernelGGL(k_pack_bias, grid(c3), dim3(256), 0, st, b3, (float*)(p + L.b3), K, c3);
    return hipGetLastError();
}

hipError_t launch_inv_scale(const float* sigma, const float* rms, float* out, int B, int K, hipStream_t st) {
    hipLaunchKernelGGL(k_inv_scale, dim3((unsigned)((B * K + 255) / 256)), dim3(256), 0, st, sigma, rms, out, B, K);
    return hipGetLastError();
}

hipError_t launch_conv(int layer, int K, const ConvArgs& a, int batch, hipStream_t st) {
    if (layer == 0) return shrink_cinp(K) == 32 ? conv_t<32, 32, 0>(a, batch, st) : conv_t<64, 32, 0>(a, batch, st);
    if (layer == 1) return conv_t<32, 32, 1>(a, batch, st);
    switch (shrink_coutp(K)) {
        case 16: return conv_t<32, 16, 2>(a, batch, st);
        case 32: return conv_t<32, 32, 2>(a, batch, st);
        case 48: return conv_t<32, 48, 2>(a, batch, st);
        case 64: return conv_t<32, 64, 2>(a, batch, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace shear
