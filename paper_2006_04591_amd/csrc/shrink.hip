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
#include <type_traits>

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

// softplus(x) = max(x, 0) + log1p(u), u = e^{-|x|} in (0, 1], from the hardware exponential and
// logarithm (relative error ~1e-6, far inside the threshold tolerance). log1p(u) is taken as
// log(w) u / (w - 1) with w = 1 + u rounded, which cancels the rounding of w (Goldberg, 1991,
// "What every computer scientist should know about floating-point arithmetic", Theorem 4);
// when w rounds to 1, log1p(u) = u to working precision.
__device__ __forceinline__ float softplusf(float x) {
    const float u = __expf(-fabsf(x));
    const float w = 1.0f + u;
    const float l = (w == 1.0f) ? u : __logf(w) * (u * __builtin_amdgcn_rcpf(w - 1.0f));
    return fmaxf(x, 0.0f) + l;
}

template <int CINP>
struct Pix {
    static constexpr int value = CINP + 8;  // bf16 per staged pixel: 16 bytes of padding against bank conflicts
};

// LDS of a conv block: the staged input tile; the bf16 output tile (the 32 hidden channels, or the
// padded gradient planes of layer 2's training epilogue) reuses it once the products are done.
// The shrink epilogue (MODE 2, 5) works from registers.
// Input channels are staged at most 32 at a time (a layer with 64 input channels stages and
// multiplies twice), which keeps the tile at 27 KB.
template <int CINP>
constexpr int staged_ch() {
    return CINP > 32 ? 32 : CINP;
}
template <int CINP, int OUTC, int MODE>
constexpr size_t conv_lds_bytes() {
    constexpr size_t in = (size_t)HH * HW * Pix<staged_ch<CINP>()>::value * 2, out = (size_t)TH * TW * OUTC * 2;
    return (MODE == 2 || MODE == 5 || in >= out) ? in : out;
}

__device__ __forceinline__ float sigmoidf(float x) { return 1.0f / (1.0f + expf(-x)); }

// Stages the halo tile of one image, channels cb .. cb + CS - 1, from bfloat16 channel-last
// activations with CIN channels per pixel.
template <int CIN, int CS>
__device__ __forceinline__ void stage(const ConvArgs& a, unsigned short* s, int b, int y0, int x0, int cb) {
    constexpr int PIX = Pix<CS>::value;
    const int N = a.N, M = a.M;
    const uint4* in = reinterpret_cast<const uint4*>(a.in);
    constexpr int CH = CS / 8, CHI = CIN / 8;  // 16-byte chunks per staged / input pixel
    constexpr int TOTAL = HH * HW * CH, NIT = (TOTAL + THREADS - 1) / THREADS;
    // all of a thread's loads are issued before its first LDS store, so that they are in flight
    // together (one load, wait and store at a time left each wavefront waiting on memory latency)
    uint4 v[NIT];
#pragma unroll
    for (int j = 0; j < NIT; ++j) {
        const int i = (int)threadIdx.x + j * THREADS;
        v[j] = make_uint4(0u, 0u, 0u, 0u);
        if (i < TOTAL) {
            const int ch = i % CH, p = i / CH, xx = p % HW, yy = p / HW;
            const int y = (y0 + yy - 1 + N) & (N - 1), x = (x0 + xx - 1 + M) & (M - 1);
            v[j] = in[(((size_t)b * N + y) * M + x) * CHI + cb / 8 + ch];
        }
    }
#pragma unroll
    for (int j = 0; j < NIT; ++j) {
        const int i = (int)threadIdx.x + j * THREADS;
        if (i < TOTAL) {
            const int ch = i % CH, p = i / CH, xx = p % HW, yy = p / HW;
            *reinterpret_cast<uint4*>(s + (yy * HW + xx) * PIX + ch * 8) = v[j];
        }
    }
}

// Four bfloat16 of 4 floats, rounded to nearest even (v_cvt_pk_bf16_f32), as one 8-byte word.
__device__ __forceinline__ uint2 pack_bf16x4(float a, float b, float c, float d) {
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    const bf16x2 lo = __builtin_convertvector((f32x2){a, b}, bf16x2);
    const bf16x2 hi = __builtin_convertvector((f32x2){c, d}, bf16x2);
    return make_uint2(__builtin_bit_cast(unsigned, lo), __builtin_bit_cast(unsigned, hi));
}

// z = bf16(coefficients x scale), channel-first FP32 -> channel-last bf16 [b][y][x][CINP] (zero padded):
// one block per ZW pixels of one row (512-byte runs of each plane), transposed through LDS.
constexpr int ZW = 128;

template <int CINP>
__global__ __launch_bounds__(THREADS) void k_pack_z(const float* __restrict__ c, const float* __restrict__ scale,
                                                 unsigned short* __restrict__ z, int K, int N, int M) {
    constexpr int PITCH = CINP + 8;
    __shared__ __attribute__((aligned(16))) unsigned short t[ZW * PITCH];
    const int xb = M / ZW;
    const int x0 = (blockIdx.x % xb) * ZW, y = (blockIdx.x / xb) % N, b = blockIdx.x / (xb * N);
    for (int i = threadIdx.x; i < CINP * ZW; i += THREADS) {
        const int px = i % ZW, k = i / ZW;
        float v = 0.0f;
        if (k < K) v = c[(((size_t)b * K + k) * N + y) * M + x0 + px] * scale[b * K + k];
        t[px * PITCH + k] = f2bf(v);
    }
    __syncthreads();
    uint4* out = reinterpret_cast<uint4*>(z + (((size_t)b * N + y) * M + x0) * CINP);
    for (int i = threadIdx.x; i < ZW * CINP / 8; i += THREADS) {
        const int ch = i % (CINP / 8), px = i / (CINP / 8);
        out[i] = *reinterpret_cast<const uint4*>(t + px * PITCH + ch * 8);
    }
}

template <int NT>
__device__ __forceinline__ void zero_acc(f32x4 (&acc)[4][NT]) {
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
}

// out[pixel][co] accumulators of a wavefront: 4 m-tiles (16 pixels of one row) x NT n-tiles, added
// to acc: output channels co0 .. co0 + COUTP - 1 of the packed weights (CINP input channels per
// tap), input channels cb .. cb + CS - 1 staged in s.
template <int CINP, int CS, int COUTP, int PD = 2>
__device__ __forceinline__ void mma(const ConvArgs& a, const unsigned short* s, f32x4 (&acc)[4][COUTP / 16], int co0,
                                    int cb) {
    constexpr int PIX = Pix<CS>::value, NT = COUTP / 16;
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    const int lr = l % 16, lk = 8 * (l / 16);
    const unsigned short* W = a.W;
    // steps (tap, 32-channel chunk kc) in order
    constexpr int KCN = CS / 32, STEPS = 9 * KCN;
    auto wfrag = [&](int it, int nt) {
        const int tap = it / KCN, kc = it % KCN;
        return *reinterpret_cast<const bf16x8*>(W + ((size_t)(co0 + nt * 16 + lr) * 9 + tap) * CINP + cb + kc * 32 +
                                                lk);
    };
    auto step = [&](int it, const bf16x8(&bf)[NT]) {
        const int tap = it / KCN, kc = it % KCN, dy = tap / 3, dx = tap % 3;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const int row = 2 * w + mt / 2, xs = (mt % 2) * 16;
            const bf16x8 afr =
                *reinterpret_cast<const bf16x8*>(s + ((row + dy) * HW + xs + lr + dx) * PIX + kc * 32 + lk);
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr, bf[nt], acc[mt][nt], 0, 0, 0);
        }
    };
    if constexpr (PD > 0) {
        // fully unrolled; the weight fragments are loaded PD steps ahead of their products, so that
        // their latency (an L2 hit, several times one step's products) overlaps PD steps of products
        // ((PD + 1) x NT x 4 VGPRs). A scheduling barrier after each step's loads keeps them there:
        // with a distance of one step and no barrier, the scheduler moved each load down to its use
        // and every step waited for L2.
        bf16x8 bq[STEPS][NT];
#pragma unroll
        for (int it = 0; it < PD && it < STEPS; ++it)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) bq[it][nt] = wfrag(it, nt);
#pragma unroll
        for (int it = 0; it < STEPS; ++it) {
            if (it + PD < STEPS) {
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) bq[it + PD][nt] = wfrag(it + PD, nt);
            }
            __builtin_amdgcn_sched_barrier(0);
            step(it, bq[it]);
        }
    } else {
        // one step at a time (the shrink layer: one step ahead measured no faster, 0.565 against
        // 0.572 ms, as its registers then hold it to 3 waves per SIMD instead of 4)
#pragma unroll 1
        for (int it = 0; it < STEPS; ++it) {
            bf16x8 bf[NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) bf[nt] = wfrag(it, nt);
            step(it, bf);
        }
    }
}

// Tile of a conv block. Hardware blocks go to the 8 XCDs in turn (block w on XCD w mod 8), each XCD
// with its own L2. Each XCD takes a contiguous range of the tile order (x fastest, then rows, then
// images), so that horizontally and vertically adjacent tiles, whose halos are each other's
// interiors, run on one XCD close in time and the halo re-reads hit its L2 (a tile's two halo
// columns of the channel-first coefficient planes are 4 bytes of a 128-byte line each: fetched
// from memory per tile, they tripled the first layer's traffic). A tail of fewer than 8 blocks
// keeps its order.
__device__ __forceinline__ int conv_tile() {
    const int w = (int)blockIdx.x, per = (int)gridDim.x / 8;
    if (w >= per * 8) return w;
    return (w % 8) * per + w / 8;
}

// MODE 1: bf16 activations (or the packed z) -> relu -> bf16 activations;
// MODE 2: activations -> o + b -> shrink of the coefficients where |c scale| >= tau = softplus(o);
// MODE 5: MODE 2 that also writes tau;
// MODE 3 (training, last layer): o -> smooth-gate loss (summed into *loss) and its gradient d o, stored as
//   bf16 channel-last planes [b][y][x][OUTC] (zero beyond K and on the low-pass plane);
// MODE 4 (training, backward data): gradient planes -> conv with flipped, transposed weights, times the relu
//   mask of the saved activation (mask_act > 0) -> bf16 gradient activations.
// Waves per SIMD a conv kernel's registers must allow, where its LDS allows them: the hidden layer
// holds 5 blocks per CU by its LDS (27 KB); the prefetched weight fragments would otherwise cost it
// a wave.
template <int CINP, int MODE>
constexpr int conv_min_waves() {
    return (MODE == 1 && CINP == 32) ? 5 : 1;
}

template <int CINP, int COUTP, int MODE, int OUTC = 32>
__global__ __launch_bounds__(THREADS, (conv_min_waves<CINP, MODE>())) void k_conv3x3(ConvArgs a) {
    constexpr int NT = COUTP / 16;
    extern __shared__ unsigned short smem[];
    unsigned short* s_in = smem;
    const int tx = a.M / TW, ty = a.N / TH, tile = conv_tile();
    const int bx = tile % tx, by = (tile / tx) % ty, b = tile / (tx * ty);
    const int x0 = bx * TW, y0 = by * TH;
    constexpr int CS = staged_ch<CINP>();
    static_assert((MODE != 2 && MODE != 5) || CS == CINP, "the shrink layer stages its whole input once");
    auto stage_part = [&](int cb) { stage<CINP, CS>(a, s_in, b, y0, x0, cb); };
    constexpr bool SHRINK = (MODE == 2 || MODE == 5);
    if constexpr (SHRINK) {
        stage_part(0);
        __syncthreads();
    }
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    const int lr = l % 16, lm = 4 * (l / 16);
    if constexpr (SHRINK) {
        // o = acc + bias, tau = softplus(o) (0 on the low-pass plane), keep |c scale| >= tau. A lane
        // holds 4 consecutive pixels of one channel, so it reads and writes the channel-first
        // coefficient planes directly as 16-byte vectors. At most 32 output channels per pass over
        // the staged tile, so that fewer accumulators leave room for more waves per SIMD.
        // (48 padded channels go in three passes of 16: a pass never reads weight rows past COUTP)
        // MODE 5 writes tau and decides with it. MODE 2 (no tau output) decides without forming
        // tau: with a = |c scale| >= 0, m = max(o, 0), u = e^-|o| in (0, 1] and d = a - m,
        // softplus(o) = m + log1p(u), so a >= softplus(o) <=> expm1(d) >= u. d is clamped to
        // [0, 0.75] (below 0, expm1 < 0 < u; above, expm1 > 1 >= u), where expm1 is its Taylor
        // polynomial of degree 9 (remainder < 2e-8 relative), and for o > 0, u is kept above 1e-30
        // (beyond o = 87 it underflows: then softplus(o) = o in FP32 and the test is d > 0). The
        // low-pass plane takes o = -inf: u = 0, every coefficient kept. One hardware exponential replaces
        // softplus's exponential, logarithm and reciprocal, with no branch, and the decision keeps
        // softplus's relative precision for small and large thresholds alike.
        constexpr int CG = COUTP <= 32 ? COUTP : (COUTP % 32 == 0 ? 32 : 16), NG = CG / 16;
        static_assert(COUTP % CG == 0, "the passes cover the padded output channels exactly");
        constexpr float L2E = 1.44269504088896341f;
        // offset of the lane's first vector in a plane: row y0 + 2 w, column x0 + lm; vector mt is
        // (mt / 2) rows and (mt % 2) 16 columns further
        const size_t pix0 = (size_t)(y0 + 2 * w) * a.M + x0 + lm;
#pragma unroll 1
        for (int c0 = 0; c0 < COUTP; c0 += CG) {
        // the pass's coefficient vectors, bias and scale are loaded before its products, so that
        // their latency overlaps the matrix work (loaded after the stores of the previous vector,
        // each load would also wait for those stores: one memory counter covers both)
        float4 cvs[NG][4];
        float biass[NG], scs[NG];
        size_t offs[NG];
#pragma unroll
        for (int nt = 0; nt < NG; ++nt) {
            const int k = c0 + nt * 16 + lr;
            biass[nt] = scs[nt] = 0.0f;
            offs[nt] = ((size_t)b * a.cout + k) * a.N * a.M + pix0;
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) cvs[nt][mt] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (k < a.cout) {
                biass[nt] = a.bias[k];
                scs[nt] = a.scale[b * a.cout + k];
                const float* cp = a.coef + offs[nt];
#pragma unroll
                for (int mt = 0; mt < 4; ++mt)
                    cvs[nt][mt] = *reinterpret_cast<const float4*>(cp + (mt / 2) * a.M + (mt % 2) * 16);
            }
        }
        f32x4 acc[4][NG];
        zero_acc(acc);
        mma<CINP, CS, CG, 0>(a, s_in, acc, c0, 0);
#pragma unroll
        for (int nt = 0; nt < NG; ++nt) {
            const int k = c0 + nt * 16 + lr;
            if (k >= a.cout) continue;
            const bool lowpass = (k == a.lowpass);
            const float bias = biass[nt];
            const float sc = scs[nt];
            float* op = a.out_f + offs[nt];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                const int vo = (mt / 2) * a.M + (mt % 2) * 16;
                const float4 cv = cvs[nt][mt];
                const float v[4] = {cv.x, cv.y, cv.z, cv.w};
                float t[4], r[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    if constexpr (MODE == 2) {
                        const float o = acc[mt][nt][i] + (lowpass ? -INFINITY : bias);
                        const float d = fminf(fmaxf(fabsf(v[i] * sc) - fmaxf(o, 0.0f), 0.0f), 0.75f);
                        const float u = fmaxf(__builtin_amdgcn_exp2f(-fabsf(o) * L2E), o > 0.0f ? 1e-30f : 0.0f);
                        float e = 1.0f / 362880.0f;
                        e = fmaf(e, d, 1.0f / 40320.0f);
                        e = fmaf(e, d, 1.0f / 5040.0f);
                        e = fmaf(e, d, 1.0f / 720.0f);
                        e = fmaf(e, d, 1.0f / 120.0f);
                        e = fmaf(e, d, 1.0f / 24.0f);
                        e = fmaf(e, d, 1.0f / 6.0f);
                        e = fmaf(e, d, 0.5f);
                        e = fmaf(e, d, 1.0f);
                        r[i] = (e * d >= u) ? v[i] : 0.0f;
                    } else {
                        t[i] = lowpass ? 0.0f : softplusf(acc[mt][nt][i] + bias);
                        r[i] = (fabsf(v[i] * sc) >= t[i]) ? v[i] : 0.0f;
                    }
                }
                *reinterpret_cast<float4*>(op + vo) = make_float4(r[0], r[1], r[2], r[3]);
                if constexpr (MODE == 5)
                    *reinterpret_cast<float4*>(a.tau + offs[nt] + vo) = make_float4(t[0], t[1], t[2], t[3]);
            }
        }
        }
    } else {
        f32x4 acc[4][NT];
        zero_acc(acc);
#pragma unroll 1
        for (int cb = 0; cb < CINP; cb += CS) {
            if (cb > 0) __syncthreads();  // every wave is done with the previous part
            stage_part(cb);
            __syncthreads();
            mma<CINP, CS, COUTP>(a, s_in, acc, 0, cb);
        }
        // bf16 results through LDS, then 16-byte channel-last stores of OUTC channels per pixel;
        // the output tile overwrites the staged input once every wave is done reading it
        unsigned short* s_out = smem;
        __syncthreads();
        float lsum = 0.0f;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const int prow = (2 * w + mt / 2) * TW + (mt % 2) * 16 + lm;
            const int y = y0 + 2 * w + mt / 2, x = x0 + (mt % 2) * 16 + lm;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int co = nt * 16 + lr;
                float v[4];
                if constexpr (MODE == 3) {
                    v[0] = v[1] = v[2] = v[3] = 0.0f;
                    if (co < a.cout && co != a.lowpass) {
                        const size_t off = (((size_t)b * a.cout + co) * a.N + y) * a.M + x;
                        const float4 cn = *reinterpret_cast<const float4*>(a.coef + off);
                        const float4 cc = *reinterpret_cast<const float4*>(a.coef2 + off);
                        const float sc = a.scale[b * a.cout + co], bias = a.bias[co];
                        const float n4[4] = {cn.x, cn.y, cn.z, cn.w}, c4[4] = {cc.x, cc.y, cc.z, cc.w};
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const float o = acc[mt][nt][i] + bias;
                            const float z = n4[i] * sc, zc = c4[i] * sc;
                            const float g = sigmoidf((fabsf(z) - softplusf(o)) / a.temperature);
                            const float r = z * g - zc;
                            lsum += r * r;
                            v[i] = 2.0f * a.loss_scale * r * z * g * (1.0f - g) * (-1.0f / a.temperature) * sigmoidf(o);
                        }
                    }
                } else if constexpr (MODE == 4) {
                    const unsigned short* h = a.mask_act + (((size_t)b * a.N + y) * a.M + x) * 32 + co;
#pragma unroll
                    for (int i = 0; i < 4; ++i) v[i] = (bf2f(h[(size_t)i * 32]) > 0.0f) ? acc[mt][nt][i] : 0.0f;
                } else {
                    const float bias = a.bias[co];
#pragma unroll
                    for (int i = 0; i < 4; ++i) v[i] = fmaxf(acc[mt][nt][i] + bias, 0.0f);
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) s_out[(prow + i) * OUTC + co] = f2bf(v[i]);
            }
        }
        if constexpr (OUTC > COUTP) {
            for (int i = threadIdx.x; i < TH * TW * (OUTC - COUTP); i += THREADS)
                s_out[(i / (OUTC - COUTP)) * OUTC + COUTP + i % (OUTC - COUTP)] = 0;
        }
        if constexpr (MODE == 3) {
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) lsum += __shfl_xor(lsum, off, 64);
            if (l == 0) atomicAdd(a.loss, lsum * a.loss_scale);
        }
        __syncthreads();
        constexpr int CH = OUTC / 8;
        uint4* out = reinterpret_cast<uint4*>(a.out_bf);
        for (int i = threadIdx.x; i < TH * TW * CH; i += THREADS) {
            const int ch = i % CH, p = i / CH, px = p % TW, py = p / TW;
            out[(((size_t)b * a.N + y0 + py) * a.M + x0 + px) * CH + ch] =
                *reinterpret_cast<const uint4*>(s_out + p * OUTC + ch * 8);
        }
    }
}

// ---------------------------------------------------------------- persistent first layer
// The first layer (coefficients -> 32 hidden channels) as a persistent kernel: one 512-thread block
// per CU keeps the layer's weights in LDS and walks a list of 8 x 64-pixel tiles, software
// pipelined: while the matrix cores work on tile t out of LDS, the FP32 loads of tile t + 1 are
// in flight in registers; then tile t's bf16 outputs leave through LDS (over the staged tile) and
// tile t + 1 is converted into the staging buffer. Only these loads and stores use the vector-memory
// counter, so waiting for the prefetched tile never waits for weight loads, and the stores of
// tile t (issued after the prefetch) are not waited for. A tile reads 256-byte runs of each
// coefficient plane (16 x 32-pixel tiles, 128-byte runs, measured 0.49 against 0.44 ms). The tiles
// of the batch are cut into 8 contiguous ranges, one per XCD (block w runs on XCD w mod 8), so
// that the halo re-reads of neighbouring tiles hit that XCD's L2. The hidden layer (32 bf16
// channels in, 32 out) runs in the same kernel with its own staging.
constexpr int PTH = 8, PHH = PTH + 2;     // tile rows, with halo
constexpr int PTW = 64, PHW = PTW + 2;    // tile columns, with halo
constexpr int PTHREADS = 512;             // 8 wavefronts, one tile row each

template <int CS>
struct PLds {
    static constexpr int PIX = Pix<CS>::value;
    static constexpr int WP = 9 * CS + 8;  // bf16 per output channel of the staged weights (padded)
    static constexpr size_t in = (size_t)PHH * PHW * PIX * 2, w = (size_t)32 * WP * 2;
    static constexpr size_t bytes = in + w;
    static_assert((size_t)PTH * PTW * 32 * 2 <= in, "the output tile fits over the staged tile");
};

// Staged rows R0 .. R0 + NR - 1 of a tile's FP32 inputs (staged row yy is image row y0 + yy - 1),
// held in registers between their loads and their conversion to LDS.
template <int CS, int NR>
struct CoefRegs {
    static constexpr int G = CS / 8, QW = PTW / 4;
    static constexpr int TOTAL = G * QW * NR, NIT = (TOTAL + PTHREADS - 1) / PTHREADS;
    static constexpr int HTOTAL = G * NR * 2, HNIT = (HTOTAL + PTHREADS - 1) / PTHREADS;
    float4 v[NIT][8];
    float h[HNIT][8];
    float sc[8];
};

// Loads staged rows R0 .. R0 + NR - 1 of tile (b, y0, x0) in units of 8 consecutive channels (one
// 16-byte run of a staged pixel) of 4 consecutive interior pixels of one row: 8 aligned 16-byte
// loads, one per channel plane. Lanes take the channel groups fastest: in each load instruction the
// lanes of one group read consecutive 16-byte pieces of a row of a plane. A lane's channel group is
// fixed (512 is a multiple of G), and so are its 8 scales within a tile. The two halo columns come
// one value per channel.
template <int CS, int NR>
__device__ __forceinline__ void coef_load(const ConvArgs& a, CoefRegs<CS, NR>& r, int b, int y0, int x0, int R0) {
    using R = CoefRegs<CS, NR>;
    const int N = a.N, M = a.M, K = a.cin;
    const int g = (int)threadIdx.x % R::G, k0 = 8 * g;
    const size_t plane = (size_t)N * M;
    const float* base = a.coef + ((size_t)b * K + k0) * plane;
#pragma unroll
    for (int c = 0; c < 8; ++c) r.sc[c] = (k0 + c < K) ? a.scale[b * K + k0 + c] : 0.0f;
#pragma unroll
    for (int j = 0; j < R::HNIT; ++j) {
        const int i = (int)threadIdx.x + j * PTHREADS;
        const int side = (i / R::G) % 2, yy = R0 + i / (2 * R::G);
        const int y = (y0 + yy - 1 + N) & (N - 1), x = side ? (x0 + PTW) & (M - 1) : (x0 - 1 + M) & (M - 1);
#pragma unroll
        for (int c = 0; c < 8; ++c)
            r.h[j][c] = (i < R::HTOTAL && k0 + c < K) ? base[c * plane + (size_t)y * M + x] : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < R::NIT; ++j) {
        const int i = (int)threadIdx.x + j * PTHREADS;
        const int q = (i / R::G) % R::QW, yy = R0 + i / (R::G * R::QW);
        const int y = (y0 + yy - 1 + N) & (N - 1);
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            r.v[j][c] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (i < R::TOTAL && k0 + c < K)
                r.v[j][c] = *reinterpret_cast<const float4*>(base + c * plane + (size_t)y * M + x0 + 4 * q);
        }
    }
}

// z = bf16(c scale) of the loaded rows -> the channel-last staging buffer (16-byte runs)
template <int CS, int NR>
__device__ __forceinline__ void coef_store(const CoefRegs<CS, NR>& r, unsigned short* s, int R0) {
    using R = CoefRegs<CS, NR>;
    constexpr int PIX = Pix<CS>::value;
    const int g = (int)threadIdx.x % R::G;
    const float* sc = r.sc;
#pragma unroll
    for (int j = 0; j < R::NIT; ++j) {
        const int i = (int)threadIdx.x + j * PTHREADS;
        if (i < R::TOTAL) {
            const int q = (i / R::G) % R::QW, yy = R0 + i / (R::G * R::QW);
            unsigned short* d = s + (yy * PHW + 1 + 4 * q) * PIX + 8 * g;
            const float4* w = r.v[j];
            const uint2 p0a = pack_bf16x4(w[0].x * sc[0], w[1].x * sc[1], w[2].x * sc[2], w[3].x * sc[3]);
            const uint2 p0b = pack_bf16x4(w[4].x * sc[4], w[5].x * sc[5], w[6].x * sc[6], w[7].x * sc[7]);
            const uint2 p1a = pack_bf16x4(w[0].y * sc[0], w[1].y * sc[1], w[2].y * sc[2], w[3].y * sc[3]);
            const uint2 p1b = pack_bf16x4(w[4].y * sc[4], w[5].y * sc[5], w[6].y * sc[6], w[7].y * sc[7]);
            const uint2 p2a = pack_bf16x4(w[0].z * sc[0], w[1].z * sc[1], w[2].z * sc[2], w[3].z * sc[3]);
            const uint2 p2b = pack_bf16x4(w[4].z * sc[4], w[5].z * sc[5], w[6].z * sc[6], w[7].z * sc[7]);
            const uint2 p3a = pack_bf16x4(w[0].w * sc[0], w[1].w * sc[1], w[2].w * sc[2], w[3].w * sc[3]);
            const uint2 p3b = pack_bf16x4(w[4].w * sc[4], w[5].w * sc[5], w[6].w * sc[6], w[7].w * sc[7]);
            *reinterpret_cast<uint4*>(d) = make_uint4(p0a.x, p0a.y, p0b.x, p0b.y);
            *reinterpret_cast<uint4*>(d + PIX) = make_uint4(p1a.x, p1a.y, p1b.x, p1b.y);
            *reinterpret_cast<uint4*>(d + 2 * PIX) = make_uint4(p2a.x, p2a.y, p2b.x, p2b.y);
            *reinterpret_cast<uint4*>(d + 3 * PIX) = make_uint4(p3a.x, p3a.y, p3b.x, p3b.y);
        }
    }
#pragma unroll
    for (int j = 0; j < R::HNIT; ++j) {
        const int i = (int)threadIdx.x + j * PTHREADS;
        if (i < R::HTOTAL) {
            const int side = (i / R::G) % 2, yy = R0 + i / (2 * R::G);
            const float* w = r.h[j];
            const uint2 pa = pack_bf16x4(w[0] * sc[0], w[1] * sc[1], w[2] * sc[2], w[3] * sc[3]);
            const uint2 pb = pack_bf16x4(w[4] * sc[4], w[5] * sc[5], w[6] * sc[6], w[7] * sc[7]);
            *reinterpret_cast<uint4*>(s + (yy * PHW + (side ? PHW - 1 : 0)) * PIX + 8 * g) =
                make_uint4(pa.x, pa.y, pb.x, pb.y);
        }
    }
}

// Staged rows R0 .. R0 + NR - 1 of a tile's hidden activations with the halo columns, [pixel][32
// channels] bf16, in 16-byte units.
template <int NR>
struct HidRegs {
    static constexpr int TOTAL = NR * PHW * 4, NIT = (TOTAL + PTHREADS - 1) / PTHREADS;
    uint4 v[NIT];
};

template <int NR>
__device__ __forceinline__ void hid_load(const ConvArgs& a, HidRegs<NR>& r, int b, int y0, int x0, int R0) {
    const int N = a.N, M = a.M;
    const uint4* in = reinterpret_cast<const uint4*>(a.in);
#pragma unroll
    for (int j = 0; j < HidRegs<NR>::NIT; ++j) {
        const int i = (int)threadIdx.x + j * PTHREADS;
        r.v[j] = make_uint4(0u, 0u, 0u, 0u);
        if (i < HidRegs<NR>::TOTAL) {
            const int ch = i % 4, p = i / 4, xx = p % PHW, yy = R0 + p / PHW;
            const int y = (y0 + yy - 1 + N) & (N - 1), x = (x0 + xx - 1 + M) & (M - 1);
            r.v[j] = in[(((size_t)b * N + y) * M + x) * 4 + ch];
        }
    }
}

template <int NR>
__device__ __forceinline__ void hid_store(const HidRegs<NR>& r, unsigned short* s, int R0) {
    constexpr int PIX = Pix<32>::value;
#pragma unroll
    for (int j = 0; j < HidRegs<NR>::NIT; ++j) {
        const int i = (int)threadIdx.x + j * PTHREADS;
        if (i < HidRegs<NR>::TOTAL) {
            const int ch = i % 4, p = i / 4;
            *reinterpret_cast<uint4*>(s + (R0 * PHW + p) * PIX + ch * 8) = r.v[j];
        }
    }
}

// The tiles of block w: t0 + j, t0 + j + per, ... < t1, where [t0, t1) is the (w mod 8)-th of 8
// contiguous ranges of the ntiles tiles, j = w / 8 and per = gridDim.x / 8 (the blocks on one XCD).
__device__ __forceinline__ void xcd_range(int ntiles, int& first, int& end, int& stride) {
    const int w = (int)blockIdx.x, per = (int)gridDim.x / 8, x = w % 8, j = w / 8;
    first = (int)(((long long)x * ntiles) / 8) + j;
    end = (int)(((long long)(x + 1) * ntiles) / 8);
    stride = per;
}

// The contiguous chunk [first, end) of tiles of block w: the j-th of per equal parts of the (w mod 8)-th
// of 8 contiguous ranges of the ntiles tiles (j = w / 8, per = gridDim.x / 8, the blocks on one XCD).
__device__ __forceinline__ void xcd_chunk(int ntiles, int& first, int& end) {
    const int w = (int)blockIdx.x, per = (int)gridDim.x / 8, x = w % 8, j = w / 8;
    const long long lo = ((long long)x * ntiles) / 8, hi = ((long long)(x + 1) * ntiles) / 8;
    first = (int)(lo + ((hi - lo) * j) / per);
    end = (int)(lo + ((hi - lo) * (j + 1)) / per);
}

// FROM_COEF: the first layer (input: the FP32 coefficient planes, normalised and rounded on staging);
// else the hidden layer (input: the bf16 activations of the first, CINP = 32).
// The first layer walks its block's chunk of tiles down vertical strips (tile index: rows of tiles
// fastest, then strips of 64 columns, then images), as a sliding window: the staged tile's last two
// rows (its bottom halo and last row) are the next tile's first two, so they move up in LDS and
// only 8 new rows are loaded per tile (10 at the top of a strip); neighbouring chunks of an XCD run
// down neighbouring strips together, so the halo columns hit that XCD's L2 (0.449 -> 0.406 ms).
// The hidden layer, whose tiles are a quarter of the bytes, takes its tiles interleaved over the
// XCD's blocks and loads all 10 rows (the sliding window's extra barrier and copy made it slower:
// 0.123 -> 0.138 ms).
template <int CINP, bool FROM_COEF>
__global__ __launch_bounds__(PTHREADS, FROM_COEF ? 2 : 4) void k_conv_relu(ConvArgs a, int ntiles) {
    constexpr int CS = CINP, PIX = Pix<CS>::value, WP = PLds<CS>::WP, KCN = CS / 32, STEPS = 9 * KCN;
    static_assert(FROM_COEF || CINP == 32, "the hidden layer has 32 input channels");
    constexpr bool SLIDE = FROM_COEF;
    constexpr int R0 = SLIDE ? 2 : 0, NR = PHH - R0;  // staged rows loaded per tile (the prefetch)
    using Regs8 = typename std::conditional<FROM_COEF, CoefRegs<CS, NR>, HidRegs<NR>>::type;
    using Regs2 = typename std::conditional<FROM_COEF, CoefRegs<CS, 2>, HidRegs<2>>::type;
    auto load8 = [&](Regs8& r, int b, int y0, int x0) {  // staged rows R0 .. 9
        if constexpr (FROM_COEF) {
            coef_load<CS, NR>(a, r, b, y0, x0, R0);
        } else {
            hid_load<NR>(a, r, b, y0, x0, R0);
        }
    };
    auto store8 = [&](const Regs8& r, unsigned short* s) {
        if constexpr (FROM_COEF) {
            coef_store<CS, NR>(r, s, R0);
        } else {
            hid_store<NR>(r, s, R0);
        }
    };
    auto stage_top = [&](unsigned short* s, int b, int y0, int x0) {  // staged rows 0, 1 straight from memory
        Regs2 r2;
        if constexpr (FROM_COEF) {
            coef_load<CS, 2>(a, r2, b, y0, x0, 0);
            coef_store<CS, 2>(r2, s, 0);
        } else {
            hid_load<2>(a, r2, b, y0, x0, 0);
            hid_store<2>(r2, s, 0);
        }
    };
    extern __shared__ unsigned short smem[];
    unsigned short* s_in = smem;
    unsigned short* s_out = smem;  // the output tile, over the staged tile's first rows once the products are done
    unsigned short* s_w = smem + PLds<CS>::in / 2;
    static_assert((size_t)PTH * PTW * 32 * 2 <= (size_t)(PHH - 2) * PHW * PIX * 2,
                  "the output tile leaves the staged tile's last two rows intact");
    const int tx = a.M / PTW, ty = a.N / PTH;
    int t, end, stride = 1;
    if constexpr (SLIDE) {
        xcd_chunk(ntiles, t, end);
    } else {
        xcd_range(ntiles, t, end, stride);
    }
    if (t >= end) return;  // the whole block: no tile
    auto tile_origin = [&](int tile, int& b, int& y0, int& x0) {
        if constexpr (SLIDE) {
            y0 = (tile % ty) * PTH;
            x0 = ((tile / ty) % tx) * PTW;
        } else {
            x0 = (tile % tx) * PTW;
            y0 = ((tile / tx) % ty) * PTH;
        }
        b = tile / (tx * ty);
    };
    // weights [co][tap][ci] -> LDS rows of WP bf16 (16-byte pieces)
    for (int i = (int)threadIdx.x; i < 32 * 9 * CS / 8; i += PTHREADS) {
        const int co = i / (9 * CS / 8), r = i % (9 * CS / 8);
        *reinterpret_cast<uint4*>(s_w + co * WP + 8 * r) = reinterpret_cast<const uint4*>(a.W)[i];
    }
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    const int lr = l % 16, lm = 4 * (l / 16), lk = 8 * (l / 16);
    float bias[2];
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) bias[nt] = a.bias[nt * 16 + lr];
    Regs8 r;
    int b, y0, x0;
    tile_origin(t, b, y0, x0);
    if constexpr (SLIDE) stage_top(s_in, b, y0, x0);
    load8(r, b, y0, x0);
    store8(r, s_in);
    if (t + stride < end) {
        int bn, yn, xn;
        tile_origin(t + stride, bn, yn, xn);
        load8(r, bn, yn, xn);
    }
    __syncthreads();
    for (;;) {
        // wave w: tile row w, 4 m-tiles of 16 pixels
        f32x4 acc[4][2];
        zero_acc(acc);
#pragma unroll 1
        for (int it = 0; it < STEPS; ++it) {
            const int tap = it / KCN, kc = it % KCN, dy = tap / 3, dx = tap % 3;
            bf16x8 bf[2];
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
                bf[nt] = *reinterpret_cast<const bf16x8*>(s_w + (nt * 16 + lr) * WP + tap * CS + kc * 32 + lk);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                const bf16x8 afr = *reinterpret_cast<const bf16x8*>(
                    s_in + ((w + dy) * PHW + 16 * mt + lr + dx) * PIX + kc * 32 + lk);
#pragma unroll
                for (int nt = 0; nt < 2; ++nt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr, bf[nt], acc[mt][nt], 0, 0, 0);
            }
        }
        __syncthreads();  // every wave is done reading the staged tile
        // relu(acc + bias) -> bf16 output tile [pixel][32 channels]
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const int prow = w * PTW + 16 * mt + lm;
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    s_out[(prow + i) * 32 + nt * 16 + lr] = f2bf(fmaxf(acc[mt][nt][i] + bias[nt], 0.0f));
        }
        __syncthreads();  // the output tile is written
        {
            uint4* out = reinterpret_cast<uint4*>(a.out_bf);
            for (int i = (int)threadIdx.x; i < PTH * PTW * 4; i += PTHREADS) {
                const int ch = i % 4, p = i / 4, px = p % PTW, py = p / PTW;
                out[(((size_t)b * a.N + y0 + py) * a.M + x0 + px) * 4 + ch] =
                    *reinterpret_cast<const uint4*>(s_out + p * 32 + ch * 8);
            }
        }
        if (t + stride >= end) break;
        const int tn = t + stride;
        int bn, yn, xn;
        tile_origin(tn, bn, yn, xn);
        __syncthreads();  // the output tile is read
        if (!SLIDE) {
            // every tile stages all its rows (below)
        } else if (yn != 0) {
            // the next tile continues the strip: its first two staged rows are this one's last two
            constexpr int U = 2 * PHW * PIX / 8;  // 16-byte units of two staged rows
            static_assert(U > PTHREADS && U <= 3 * PTHREADS, "two staged rows are 2 or 3 units per thread");
            const uint4* src = reinterpret_cast<const uint4*>(s_in + PTH * PHW * PIX);
            uint4* dst = reinterpret_cast<uint4*>(s_in);
            const int i0 = (int)threadIdx.x, i1 = i0 + PTHREADS, i2 = i0 + 2 * PTHREADS;
            const uint4 m0 = src[i0], m1 = src[min(i1, U - 1)], m2 = src[min(i2, U - 1)];
            __syncthreads();  // rows 8 and 9 are read before the new rows overwrite them
            dst[i0] = m0;
            if (i1 < U) dst[i1] = m1;
            if (i2 < U) dst[i2] = m2;
        } else {
            stage_top(s_in, bn, yn, xn);  // the top of a strip: its first two rows from memory
        }
        store8(r, s_in);  // staged rows R0 .. 9 of tile tn, loaded during this tile's products
        t = tn;
        b = bn;
        y0 = yn;
        x0 = xn;
        if (t + stride < end) {
            int bq, yq, xq;
            tile_origin(t + stride, bq, yq, xq);
            load8(r, bq, yq, xq);
        }
        __syncthreads();  // the next tile is staged
    }
}

// ---------------------------------------------------------------- persistent shrink layer
// The last layer with the shrink decision (no tau output) in the persistent form of k_conv_relu:
// one 512-thread block per CU keeps the layer's weights in LDS and walks its XCD's range of
// 8 x 64-pixel tiles. Per tile, the staged hidden activations serve CG output channels at a time;
// each pass's FP32 coefficients come into LDS as 256-byte row runs, are decided there in the matrix
// cores' lane layout (c kept or zeroed in place) and leave as 256-byte row runs. The next pass's
// coefficients, and during the first pass the next tile's activations, are in flight in registers
// while the matrix cores work.
template <int COUTP>
struct SLds {
    static constexpr int CG = COUTP <= 32 ? COUTP : (COUTP % 32 == 0 ? 32 : 16);  // channels per pass
    static constexpr int PIX = Pix<32>::value;
    static constexpr int WP = 9 * 32 + 8;            // bf16 per output channel of the staged weights
    static constexpr int CP = PTH * PTW + 4;         // floats per channel of the coefficient pass buffer
    static constexpr size_t h = (size_t)PHH * PHW * PIX * 2, w = (size_t)COUTP * WP * 2,
                            c = (size_t)CG * CP * 4;
    static constexpr size_t bytes = h + w + c;
};

// One pass's coefficients of tile (b, y0, x0): channels c0 .. c0 + CG - 1 (those below K), 8 rows of
// 64 pixels, as 16-byte units with 16 lanes per 256-byte row run.
template <int CG>
struct PassRegs {
    static constexpr int TOTAL = CG * PTH * (PTW / 4), NIT = (TOTAL + PTHREADS - 1) / PTHREADS;
    float4 v[NIT];
};

template <int CG>
__device__ __forceinline__ void pass_load(const ConvArgs& a, PassRegs<CG>& r, int b, int y0, int x0, int c0) {
#pragma unroll
    for (int j = 0; j < PassRegs<CG>::NIT; ++j) {
        const int i = (int)threadIdx.x + j * PTHREADS;
        const int q = i % (PTW / 4), yy = (i / (PTW / 4)) % PTH, kl = i / (PTH * PTW / 4), k = c0 + kl;
        r.v[j] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (i < PassRegs<CG>::TOTAL && k < a.cout)
            r.v[j] = *reinterpret_cast<const float4*>(a.coef + (((size_t)b * a.cout + k) * a.N + y0 + yy) * a.M + x0 + 4 * q);
    }
}

template <int COUTP>
__global__ __launch_bounds__(PTHREADS, 2) void k_conv_shrink(ConvArgs a, int ntiles) {
    using L = SLds<COUTP>;
    constexpr int CG = L::CG, NG = CG / 16, NP = COUTP / CG, PIX = L::PIX, WP = L::WP, CP = L::CP;
    static_assert(COUTP % CG == 0, "the passes cover the padded output channels exactly");
    constexpr float L2E = 1.44269504088896341f;
    extern __shared__ unsigned short smem[];
    unsigned short* s_h = smem;
    unsigned short* s_w = smem + L::h / 2;
    float* s_c = reinterpret_cast<float*>(smem + (L::h + L::w) / 2);
    const int tx = a.M / PTW, ty = a.N / PTH;
    int t, end, stride;
    xcd_range(ntiles, t, end, stride);
    if (t >= end) return;  // the whole block: no tile
    auto tile_origin = [&](int tile, int& b, int& y0, int& x0) {
        x0 = (tile % tx) * PTW;
        y0 = ((tile / tx) % ty) * PTH;
        b = tile / (tx * ty);
    };
    // weights [co][tap][ci] (COUTP rows, zero beyond K) -> LDS rows of WP bf16
    for (int i = (int)threadIdx.x; i < COUTP * 9 * 32 / 8; i += PTHREADS) {
        const int co = i / (9 * 32 / 8), r = i % (9 * 32 / 8);
        *reinterpret_cast<uint4*>(s_w + co * WP + 8 * r) = reinterpret_cast<const uint4*>(a.W)[i];
    }
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    const int lr = l % 16, lk = 8 * (l / 16), lm = 4 * (l / 16);
    HidRegs<PHH> hr;
    PassRegs<CG> pr;
    int b, y0, x0;
    tile_origin(t, b, y0, x0);
    hid_load<PHH>(a, hr, b, y0, x0, 0);
    pass_load<CG>(a, pr, b, y0, x0, 0);
    hid_store<PHH>(hr, s_h, 0);
    int tn = t + stride, bn = 0, yn = 0, xn = 0;
    if (tn < end) tile_origin(tn, bn, yn, xn);
    for (;;) {
#pragma unroll 1
        for (int p = 0; p < NP; ++p) {
            const int c0 = p * CG;
            // this pass's coefficients -> LDS [channel][row][pixel] (after the previous pass's copy-out
            // has read the buffer: the barrier at the end of each pass)
#pragma unroll
            for (int j = 0; j < PassRegs<CG>::NIT; ++j) {
                const int i = (int)threadIdx.x + j * PTHREADS;
                if (i < PassRegs<CG>::TOTAL) {
                    const int q = i % (PTW / 4), yy = (i / (PTW / 4)) % PTH, kl = i / (PTH * PTW / 4);
                    *reinterpret_cast<float4*>(s_c + kl * CP + yy * PTW + 4 * q) = pr.v[j];
                }
            }
            __syncthreads();  // coefficients (and, in the first pass, the activations) staged
            // next loads: the following pass's coefficients, or the next tile's first pass and activations
            if (p + 1 < NP) {
                pass_load<CG>(a, pr, b, y0, x0, c0 + CG);
            } else if (tn < end) {
                hid_load<PHH>(a, hr, bn, yn, xn, 0);
                pass_load<CG>(a, pr, bn, yn, xn, 0);
            }
            f32x4 acc[4][NG];
            zero_acc(acc);
#pragma unroll 1
            for (int tap = 0; tap < 9; ++tap) {
                const int dy = tap / 3, dx = tap % 3;
                bf16x8 bf[NG];
#pragma unroll
                for (int nt = 0; nt < NG; ++nt)
                    bf[nt] = *reinterpret_cast<const bf16x8*>(s_w + (c0 + nt * 16 + lr) * WP + tap * 32 + lk);
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) {
                    const bf16x8 afr = *reinterpret_cast<const bf16x8*>(s_h + ((w + dy) * PHW + 16 * mt + lr + dx) * PIX + lk);
#pragma unroll
                    for (int nt = 0; nt < NG; ++nt)
                        acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr, bf[nt], acc[mt][nt], 0, 0, 0);
                }
            }
            // the decision of k_conv3x3's MODE 2, on the staged coefficients, in place
#pragma unroll
            for (int nt = 0; nt < NG; ++nt) {
                const int kl = nt * 16 + lr, k = c0 + kl;
                if (k >= a.cout) continue;
                const bool lowpass = (k == a.lowpass);
                const float bias = lowpass ? -INFINITY : a.bias[k];
                const float sc = a.scale[b * a.cout + k];
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) {
                    float4* cp = reinterpret_cast<float4*>(s_c + kl * CP + w * PTW + 16 * mt + lm);
                    const float4 cv = *cp;
                    const float v[4] = {cv.x, cv.y, cv.z, cv.w};
                    float r[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const float o = acc[mt][nt][i] + bias;
                        const float d = fminf(fmaxf(fabsf(v[i] * sc) - fmaxf(o, 0.0f), 0.0f), 0.75f);
                        const float u = fmaxf(__builtin_amdgcn_exp2f(-fabsf(o) * L2E), o > 0.0f ? 1e-30f : 0.0f);
                        float e = 1.0f / 362880.0f;
                        e = fmaf(e, d, 1.0f / 40320.0f);
                        e = fmaf(e, d, 1.0f / 5040.0f);
                        e = fmaf(e, d, 1.0f / 720.0f);
                        e = fmaf(e, d, 1.0f / 120.0f);
                        e = fmaf(e, d, 1.0f / 24.0f);
                        e = fmaf(e, d, 1.0f / 6.0f);
                        e = fmaf(e, d, 0.5f);
                        e = fmaf(e, d, 1.0f);
                        r[i] = (e * d >= u) ? v[i] : 0.0f;
                    }
                    *cp = make_float4(r[0], r[1], r[2], r[3]);
                }
            }
            __syncthreads();  // the pass's shrunk coefficients are in LDS
#pragma unroll
            for (int j = 0; j < PassRegs<CG>::NIT; ++j) {
                const int i = (int)threadIdx.x + j * PTHREADS;
                const int q = i % (PTW / 4), yy = (i / (PTW / 4)) % PTH, kl = i / (PTH * PTW / 4), k = c0 + kl;
                if (i < PassRegs<CG>::TOTAL && k < a.cout)
                    *reinterpret_cast<float4*>(a.out_f + (((size_t)b * a.cout + k) * a.N + y0 + yy) * a.M + x0 + 4 * q) =
                        *reinterpret_cast<const float4*>(s_c + kl * CP + yy * PTW + 4 * q);
            }
            if (p + 1 < NP || tn < end) __syncthreads();  // the copy-out has read the buffer
        }
        if (tn >= end) break;
        hid_store<PHH>(hr, s_h, 0);  // the next tile's activations (every wave is past its products)
        t = tn;
        b = bn;
        y0 = yn;
        x0 = xn;
        tn = t + stride;
        if (tn < end) tile_origin(tn, bn, yn, xn);
    }
}

// ---------------------------------------------------------------- weight gradients
// dW[co][tap][ci] = sum over pixels p of dy[co](p) x[ci](p + tap offset): an MFMA GEMM with
// M = output channels, N = (tap, input channel), K = pixels (one 32-pixel tile row per step).
// A block loops over pixel tiles (stride gridDim.x) and writes its partial sums, and the bias
// gradient sum_p dy[co](p), to part[blockIdx.x]; k_wgrad_reduce adds the partials in block order.
// x: bf16 channel-last with CINP channels (the packed z, or a hidden activation).
// Rows of the staged input tile have a pitch of XP = 40 bf16 (80 bytes): 16-byte aligned, so a
// lane's 8 pixels at a tap's column offset come from two aligned 16-byte reads and a byte-align.
constexpr int XP = 40;

// bf16 elements off .. off + 7 (off in 0..2) of the 16 elements held in lo, hi
__device__ __forceinline__ bf16x8 shifted8(uint4 lo, uint4 hi, int off) {
    const unsigned d[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
    union {
        unsigned u[4];
        bf16x8 v;
    } r;
    if (off == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) r.u[j] = d[j];
    } else if (off == 2) {
#pragma unroll
        for (int j = 0; j < 4; ++j) r.u[j] = d[j + 1];
    } else {  // one element: each dword takes the high half of one and the low half of the next
#pragma unroll
        for (int j = 0; j < 4; ++j) r.u[j] = __builtin_amdgcn_alignbyte(d[j + 1], d[j], 2);
    }
    return r.v;
}

template <int CINP, int COUTP>
__global__ __launch_bounds__(THREADS) void k_wgrad(WgradArgs a) {
    constexpr int MT = COUTP / 16, NTT = 9 * CINP / 16, TT = MT * NTT, TPW = (TT + 3) / 4;
    extern __shared__ unsigned short smem[];
    unsigned short* s_dy = smem;                      // [COUTP][TH][TW]
    unsigned short* s_x = smem + COUTP * TH * TW;     // [CINP][HH][XP]
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    const int lr = l % 16, lk = 8 * (l / 16);
    const int N = a.N, M = a.M;
    const int tx = M / TW, ty = N / TH, ntiles = a.batch * tx * ty;
    f32x4 acc[TPW];
#pragma unroll
    for (int j = 0; j < TPW; ++j) acc[j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    float bsum = 0.0f;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int bx = tile % tx, by = (tile / tx) % ty, b = tile / (tx * ty);
        const int x0 = bx * TW, y0 = by * TH;
        __syncthreads();  // the previous tile's LDS reads are done
        // dy tile, channel-major
        for (int i = threadIdx.x; i < COUTP * TH * TW; i += THREADS) {
            const int px = i % TW, r = i / TW, py = r % TH, co = r / TH;
            s_dy[i] = a.dy[(((size_t)b * N + y0 + py) * M + x0 + px) * a.dy_ch + co];
        }
        // input tile with halo, channel-major
        for (int i = threadIdx.x; i < CINP * HH * HW; i += THREADS) {
            const int xx = i % HW, r = i / HW, yy = r % HH, ci = r / HH;
            const int y = (y0 + yy - 1 + N) & (N - 1), x = (x0 + xx - 1 + M) & (M - 1);
            s_x[(ci * HH + yy) * XP + xx] = a.xb[(((size_t)b * N + y) * M + x) * CINP + ci];
        }
        __syncthreads();
        if (threadIdx.x < COUTP) {
            const unsigned short* d = s_dy + threadIdx.x * TH * TW;
            for (int i = 0; i < TH * TW; ++i) bsum += bf2f(d[i]);
        }
#pragma unroll 1
        for (int r = 0; r < TH; ++r) {
#pragma unroll
            for (int j = 0; j < TPW; ++j) {
                const int t = w + 4 * j;
                if (t < TT) {
                    const int mt = t % MT, nt = t / MT;
                    const int tap = nt / (CINP / 16), cg = nt % (CINP / 16);
                    const int dy = tap / 3, dx = tap % 3;
                    const bf16x8 afr = *reinterpret_cast<const bf16x8*>(s_dy + ((mt * 16 + lr) * TH + r) * TW + lk);
                    const uint4* xp =
                        reinterpret_cast<const uint4*>(s_x + ((cg * 16 + lr) * HH + r + dy) * XP + lk);
                    const bf16x8 bfr = shifted8(xp[0], xp[1], dx);
                    acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr, bfr, acc[j], 0, 0, 0);
                }
            }
        }
    }
    // partial dW in [co][tap][ci] order, then the bias partial
    float* part = a.part + (size_t)blockIdx.x * (COUTP * 9 * CINP + COUTP);
#pragma unroll
    for (int j = 0; j < TPW; ++j) {
        const int t = w + 4 * j;
        if (t < TT) {
            const int mt = t % MT, nt = t / MT;
            const int tap = nt / (CINP / 16), ci = (nt % (CINP / 16)) * 16 + lr;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int co = mt * 16 + 4 * (l / 16) + i;
                part[((size_t)co * 9 + tap) * CINP + ci] = acc[j][i];
            }
        }
    }
    if (threadIdx.x < COUTP) part[COUTP * 9 * CINP + threadIdx.x] = bsum;
}

// grads in natural order: dW[co][ci][3][3] (co < cout, ci < cin), then db[co]; sums of nblk partials in order
__global__ void k_wgrad_reduce(const float* __restrict__ part, float* __restrict__ dW, float* __restrict__ db, int nblk,
                               int cout, int cin, int coutp, int cinp) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int nw = cout * cin * 9;
    if (i >= nw + cout) return;
    size_t src;
    if (i < nw) {
        const int tap = i % 9, ci = (i / 9) % cin, co = i / (9 * cin);
        src = ((size_t)co * 9 + tap) * cinp + ci;
    } else {
        src = (size_t)coutp * 9 * cinp + (i - nw);
    }
    const size_t stride = (size_t)coutp * 9 * cinp + coutp;
    float s = 0.0f;
    for (int b = 0; b < nblk; ++b) s += part[(size_t)b * stride + src];
    if (i < nw)
        dW[i] = s;
    else
        db[i - nw] = s;
}

// natural W[co][ci][3][3] -> flipped, transposed bf16 [ci][8 - tap][co], padded to cinp' x coutp'
// (the weights of the backward-data correlation)
__global__ void k_pack_weights_t(const float* __restrict__ W, unsigned short* __restrict__ out, int cout, int cin,
                                 int rows, int cols) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows * 9 * cols) return;
    const int co = i % cols, tap = (i / cols) % 9, ci = i / (cols * 9);
    out[i] = (ci < cin && co < cout) ? f2bf(W[((size_t)co * cin + ci) * 9 + (8 - tap)]) : (unsigned short)0;
}

// Adam (bias-corrected) on n FP32 parameters; step t >= 1
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       int n, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
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

template <int CINP, int COUTP, int MODE, int OUTC = 32>
hipError_t conv_t(const ConvArgs& a, int batch, hipStream_t st) {
    const void* fn = reinterpret_cast<const void*>(&k_conv3x3<CINP, COUTP, MODE, OUTC>);
    const size_t lds = conv_lds_bytes<CINP, OUTC, MODE>();
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const size_t blocks = (size_t)batch * (a.N / TH) * (a.M / TW);
    hipLaunchKernelGGL((k_conv3x3<CINP, COUTP, MODE, OUTC>), dim3((unsigned)blocks), dim3(THREADS), lds, st,
                       a);
    return hipGetLastError();
}

template <int CINP, bool FROM_COEF>
hipError_t conv_relu_t(const ConvArgs& a, int batch, hipStream_t st) {
    const void* fn = reinterpret_cast<const void*>(&k_conv_relu<CINP, FROM_COEF>);
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)PLds<CINP>::bytes);
    if (e != hipSuccess) return e;
    const int ntiles = batch * (a.N / PTH) * (a.M / PTW);
    // blocks per CU its registers and LDS allow (first layer: 187 VGPRs, 132 KB; hidden layer: 106
    // VGPRs, 72 KB), a multiple of the 8 XCDs
    const int blocks = (FROM_COEF ? 1 : 2) * std::max(8, a.cus / 8 * 8);
    hipLaunchKernelGGL((k_conv_relu<CINP, FROM_COEF>), dim3((unsigned)blocks), dim3(PTHREADS), PLds<CINP>::bytes, st,
                       a, ntiles);
    return hipGetLastError();
}

template <int COUTP>
hipError_t conv_shrink_t(const ConvArgs& a, int batch, hipStream_t st) {
    const void* fn = reinterpret_cast<const void*>(&k_conv_shrink<COUTP>);
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)SLds<COUTP>::bytes);
    if (e != hipSuccess) return e;
    const int ntiles = batch * (a.N / PTH) * (a.M / PTW);
    const int blocks = std::max(8, a.cus / 8 * 8);  // one per CU, a multiple of the 8 XCDs
    hipLaunchKernelGGL((k_conv_shrink<COUTP>), dim3((unsigned)blocks), dim3(PTHREADS), SLds<COUTP>::bytes, st, a, ntiles);
    return hipGetLastError();
}

template <int CINP, int COUTP>
hipError_t wgrad_t(const WgradArgs& a, int blocks, hipStream_t st) {
    const void* fn = reinterpret_cast<const void*>(&k_wgrad<CINP, COUTP>);
    const size_t lds = ((size_t)COUTP * TH * TW + (size_t)CINP * HH * XP) * 2;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_wgrad<CINP, COUTP>), dim3((unsigned)blocks), dim3(THREADS), lds, st, a);
    return hipGetLastError();
}

}  // namespace

int shrink_cinp(int K) { return K <= 32 ? 32 : 64; }
int shrink_coutp(int K) { return (K + 15) / 16 * 16; }
bool shrink_supported(int K, int N, int M) { return K >= 1 && K <= 64 && N >= TH && N % TH == 0 && M % ZW == 0; }

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
    if (layer == 0) return shrink_cinp(K) == 32 ? conv_t<32, 32, 1>(a, batch, st) : conv_t<64, 32, 1>(a, batch, st);
    if (layer == 1) return conv_relu_t<32, false>(a, batch, st);  // h1 -> h2 (persistent)
    if (layer == 6)  // layer 1 staged straight from the coefficients (a.coef, a.scale, a.cin = K)
        return shrink_cinp(K) == 32 ? conv_relu_t<32, true>(a, batch, st) : conv_relu_t<64, true>(a, batch, st);
    if (layer == 3) {  // training: last layer with the loss epilogue, gradient planes of shrink_cinp(K) channels
        if (shrink_cinp(K) == 32) {
            switch (shrink_coutp(K)) {
                case 16: return conv_t<32, 16, 3, 32>(a, batch, st);
                case 32: return conv_t<32, 32, 3, 32>(a, batch, st);
            }
        } else {
            switch (shrink_coutp(K)) {
                case 48: return conv_t<32, 48, 3, 64>(a, batch, st);
                case 64: return conv_t<32, 64, 3, 64>(a, batch, st);
            }
        }
        return hipErrorInvalidValue;
    }
    if (layer == 4) return conv_t<32, 32, 4>(a, batch, st);  // backward data from 32 gradient channels
    if (layer == 5) return shrink_cinp(K) == 32 ? conv_t<32, 32, 4>(a, batch, st) : conv_t<64, 32, 4>(a, batch, st);
    if (a.tau) {  // the shrink layer that also writes the thresholds
        switch (shrink_coutp(K)) {
            case 16: return conv_t<32, 16, 5>(a, batch, st);
            case 32: return conv_t<32, 32, 5>(a, batch, st);
            case 48: return conv_t<32, 48, 5>(a, batch, st);
            case 64: return conv_t<32, 64, 5>(a, batch, st);
        }
        return hipErrorInvalidValue;
    }
    switch (shrink_coutp(K)) {
        case 16: return conv_shrink_t<16>(a, batch, st);
        case 32: return conv_shrink_t<32>(a, batch, st);
        case 48: return conv_shrink_t<48>(a, batch, st);
        case 64: return conv_shrink_t<64>(a, batch, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace shear

namespace shear {

hipError_t launch_wgrad(int layer, int K, const WgradArgs& a, int blocks, hipStream_t st) {
    if (layer == 0) return shrink_cinp(K) == 32 ? wgrad_t<32, 32>(a, blocks, st) : wgrad_t<64, 32>(a, blocks, st);
    if (layer == 1) return wgrad_t<32, 32>(a, blocks, st);
    switch (shrink_coutp(K)) {
        case 16: return wgrad_t<32, 16>(a, blocks, st);
        case 32: return wgrad_t<32, 32>(a, blocks, st);
        case 48: return wgrad_t<32, 48>(a, blocks, st);
        case 64: return wgrad_t<32, 64>(a, blocks, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_wgrad_reduce(const float* part, float* dW, float* db, int nblk, int cout, int cin, int coutp, int cinp,
                               hipStream_t st) {
    const int n = cout * cin * 9 + cout;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, part, dW, db, nblk, cout, cin,
                       coutp, cinp);
    return hipGetLastError();
}

hipError_t launch_pack_weights_t(const float* W, unsigned short* out, int cout, int cin, int rows, int cols,
                                 hipStream_t st) {
    const int n = rows * 9 * cols;
    hipLaunchKernelGGL(k_pack_weights_t, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, W, out, cout, cin, rows,
                       cols);
    return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps,
                       int step, hipStream_t st) {
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, g, m, v, n, lr, b1, b2, eps, c1,
                       c2);
    return hipGetLastError();
}

}  // namespace shear

namespace shear {

hipError_t launch_pack_z(const float* c, const float* scale, unsigned short* z, int K, int N, int M, int batch,
                         hipStream_t st) {
    if (M % ZW != 0) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((size_t)batch * N * (M / ZW)));
    if (shrink_cinp(K) == 32)
        hipLaunchKernelGGL(k_pack_z<32>, grid, dim3(THREADS), 0, st, c, scale, z, K, N, M);
    else
        hipLaunchKernelGGL(k_pack_z<64>, grid, dim3(THREADS), 0, st, c, scale, z, K, N, M);
    return hipGetLastError();
}

}  // namespace shear
