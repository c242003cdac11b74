// gfx950 kernels of the FFT-domain shearlet filter bank.
//
// Data flow (Algorithm 1 / Algorithm 2 of Section 3.4.2 with the Fourier
// shifts folded into the stored filter order):
//   forward  x --rows r2c--> A --columns: FFT, x conj filter_k, IFFT--> T_k --rows c2r--> c_k
//   inverse  c_k --rows r2c--> U_k --columns: FFT, x dual filter_k, sum_k, IFFT--> V --rows c2r--> y
// A real row of M samples is transformed as M/2 complex samples plus a
// post-twiddle; the real DC and Nyquist bins of each row spectrum share one
// complex slot ("packed" column 0), so every intermediate plane is N x M/2
// complex, stored column-major so column passes read whole columns.
//
// FFTs are Stockham autosort passes (radix 2/4/8/16 butterflies in
// registers, LDS between passes). A thread of an FFT group of T = L/P threads
// holds P points: on input x[t + T q], on output X[t + T q], q < P.
#include "kernels.h"

namespace shear {
namespace {

// ---------------------------------------------------------------- complex helpers

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
// multiply by -i (forward sign) or +i (inverse sign)
template <bool INV>
__device__ __forceinline__ float2 mul_mi(float2 a) {
    return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// ---------------------------------------------------------------- butterflies
// In-register DFT of length R, natural order in and out, sign e^{-} (forward) or e^{+} (inverse).

template <bool INV>
__device__ __forceinline__ void dft2(float2& a, float2& b) {
    float2 s = cadd(a, b), d = csub(a, b);
    a = s;
    b = d;
}

template <bool INV>
__device__ __forceinline__ void dft4(float2& v0, float2& v1, float2& v2, float2& v3) {
    float2 s02 = cadd(v0, v2), d02 = csub(v0, v2), s13 = cadd(v1, v3), d13 = mul_mi<INV>(csub(v1, v3));
    v0 = cadd(s02, s13);
    v2 = csub(s02, s13);
    v1 = cadd(d02, d13);
    v3 = csub(d02, d13);
}

template <bool INV>
__device__ __forceinline__ float2 tw8_1(float2 a) {  // a * exp(-+ 2 pi i / 8)
    const float r = 0.70710678118654752440f;
    return INV ? make_float2((a.x - a.y) * r, (a.x + a.y) * r) : make_float2((a.x + a.y) * r, (a.y - a.x) * r);
}
template <bool INV>
__device__ __forceinline__ float2 tw8_3(float2 a) {  // a * exp(-+ 2 pi i 3 / 8)
    const float r = 0.70710678118654752440f;
    return INV ? make_float2((-a.x - a.y) * r, (a.x - a.y) * r) : make_float2((a.y - a.x) * r, (-a.x - a.y) * r);
}

template <bool INV>
__device__ __forceinline__ void dft8(float2* v) {
    float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<INV>(e0, e1, e2, e3);
    dft4<INV>(o0, o1, o2, o3);
    o1 = tw8_1<INV>(o1);
    o2 = mul_mi<INV>(o2);
    o3 = tw8_3<INV>(o3);
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1);
    v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2);
    v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3);
    v[7] = csub(e3, o3);
}

// 16 = 4 x 4: x[a + 4 b]; DFT4 over b, twiddle w16^{a kb}, DFT4 over a -> X[kb + 4 ka]
template <bool INV>
__device__ __forceinline__ void dft16(float2* v) {
    // cos / sin of 2 pi m / 16, m = 1, 2, 3
    const float c1 = 0.92387953251128675613f, s1 = 0.38268343236508977173f;
    const float c2 = 0.70710678118654752440f;
    float2 y[16];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        float2 p0 = v[a], p1 = v[a + 4], p2 = v[a + 8], p3 = v[a + 12];
        dft4<INV>(p0, p1, p2, p3);
        y[a * 4 + 0] = p0;
        y[a * 4 + 1] = p1;
        y[a * 4 + 2] = p2;
        y[a * 4 + 3] = p3;
    }
    const float sg = INV ? 1.0f : -1.0f;
    // a = 1: w^{0,1,2,3}; a = 2: w^{0,2,4,6}; a = 3: w^{0,3,6,9}
    y[5] = cmul(y[5], make_float2(c1, sg * s1));
    y[6] = cmul(y[6], make_float2(c2, sg * c2));
    y[7] = cmul(y[7], make_float2(s1, sg * c1));
    y[9] = cmul(y[9], make_float2(c2, sg * c2));
    y[10] = mul_mi<INV>(y[10]);
    y[11] = cmul(y[11], make_float2(-c2, sg * c2));
    y[13] = cmul(y[13], make_float2(s1, sg * c1));
    y[14] = cmul(y[14], make_float2(-c2, sg * c2));
    y[15] = cmul(y[15], make_float2(-c1, -sg * s1));
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
        float2 p0 = y[0 * 4 + kb], p1 = y[1 * 4 + kb], p2 = y[2 * 4 + kb], p3 = y[3 * 4 + kb];
        dft4<INV>(p0, p1, p2, p3);
        v[kb + 0] = p0;
        v[kb + 4] = p1;
        v[kb + 8] = p2;
        v[kb + 12] = p3;
    }
}

template <int R, bool INV>
__device__ __forceinline__ void dft(float2* v) {
    if constexpr (R == 2) {
        dft2<INV>(v[0], v[1]);
    } else if constexpr (R == 4) {
        dft4<INV>(v[0], v[1], v[2], v[3]);
    } else if constexpr (R == 8) {
        dft8<INV>(v);
    } else {
        static_assert(R == 16, "radix");
        dft16<INV>(v);
    }
}

// ---------------------------------------------------------------- Stockham FFT
// One pass with radix R = min(P, L/NS) over the L points of an FFT group.
// FIRST: inputs come from registers; LAST: outputs go to registers. Otherwise
// the pass reads the group's LDS scratch s (L float2), synchronises, and
// writes back. Every pass that reads LDS ends its read phase with a barrier,
// so a following pass (or a following FFT) may write s immediately.
template <int L, int P, bool INV, int NS, bool FIRST>
struct FFTPass {
    static __device__ __forceinline__ void run(float2 (&v)[P], float2* s, int t, const float2* __restrict__ tw) {
        constexpr int T = L / P;
        constexpr int R = (L / NS >= P) ? P : (L / NS);
        constexpr bool LAST = (NS * R == L);
        constexpr int BPT = P / R;
        float2 u[P];
        if constexpr (FIRST) {
#pragma unroll
            for (int q = 0; q < P; ++q) u[q] = v[q];
        } else {
            __syncthreads();
#pragma unroll
            for (int i = 0; i < BPT; ++i)
#pragma unroll
                for (int r = 0; r < R; ++r) u[i + BPT * r] = s[(t + T * i) + r * (L / R)];
            __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < BPT; ++i) {
            const int j = t + T * i;
            float2 w[R];
#pragma unroll
            for (int r = 0; r < R; ++r) w[r] = u[i + BPT * r];
            if constexpr (NS > 1) {
                const int kk = j & (NS - 1);
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    float2 tv = tw[r * kk * (L / (NS * R))];
                    if (INV) tv.y = -tv.y;
                    w[r] = cmul(w[r], tv);
                }
            }
            dft<R, INV>(w);
            if constexpr (LAST) {
#pragma unroll
                for (int r = 0; r < R; ++r) v[i + BPT * r] = w[r];
            } else {
                const int idxD = (j / NS) * NS * R + (j & (NS - 1));
#pragma unroll
                for (int r = 0; r < R; ++r) s[idxD + r * NS] = w[r];
            }
        }
        if constexpr (!LAST) FFTPass<L, P, INV, NS * R, false>::run(v, s, t, tw);
    }
};

template <int L, int P, bool INV>
__device__ __forceinline__ void fft(float2 (&v)[P], float2* s, int t, const float2* __restrict__ tw) {
    FFTPass<L, P, INV, 1, true>::run(v, s, t, tw);
}

// points per thread for an FFT of length L
template <int L>
struct Pts {
    static constexpr int value = (L >= 1024) ? 16 : (L == 256 ? 16 : 8);
};

constexpr int RB = 16;  // rows per block in the row passes

// ---------------------------------------------------------------- row passes

// TAG only separates launch roles into distinct symbols (0: images, 1: coefficient planes)
template <int M, int TAG>
__global__ __launch_bounds__(RB*(M / 2) / Pts<M / 2>::value) void k_rows_r2c(const float* __restrict__ in,
                                                                             float2* __restrict__ out, int N,
                                                                             const float2* __restrict__ twL,
                                                                             const float2* __restrict__ twM) {
    constexpr int L = M / 2, P = Pts<L>::value, T = L / P, PITCH = L + 1;
    extern __shared__ float2 lds[];
    const int tid = threadIdx.x;
    const int nrb = N / RB;
    const int plane = blockIdx.x / nrb;
    const int row0 = (blockIdx.x % nrb) * RB;
    const int t = tid % T, r = tid / T;
    float2* s = lds + r * PITCH;
    const float2* src = reinterpret_cast<const float2*>(in + ((size_t)plane * N + row0 + r) * M);
    float2 v[P];
#pragma unroll
    for (int q = 0; q < P; ++q) v[q] = src[t + T * q];
    fft<L, P, false>(v, s, t, twL);
#pragma unroll
    for (int q = 0; q < P; ++q) s[t + T * q] = v[q];
    __syncthreads();
    const int r2 = tid % RB, kk = tid / RB;
    const float2* s2 = lds + r2 * PITCH;
    float2* dst = out + (size_t)plane * L * N + row0 + r2;
#pragma unroll
    for (int i = 0; i < P; ++i) {
        const int k = kk + T * i;
        const float2 Z = s2[k];
        const float2 Zm = s2[(L - k) & (L - 1)];
        float2 X;
        if (k == 0) {
            X = make_float2(Z.x + Z.y, Z.x - Z.y);
        } else {
            const float2 E = make_float2(0.5f * (Z.x + Zm.x), 0.5f * (Z.y - Zm.y));
            const float2 D = make_float2(0.5f * (Z.x - Zm.x), 0.5f * (Z.y + Zm.y));
            const float2 O = make_float2(D.y, -D.x);  // (Z - conj Zm) / (2i)
            X = cadd(E, cmul(twM[k], O));
        }
        dst[(size_t)k * N] = X;
    }
}

template <int M, int TAG>
__global__ __launch_bounds__(RB*(M / 2) / Pts<M / 2>::value) void k_rows_c2r(const float2* __restrict__ in,
                                                                             float* __restrict__ out, int N,
                                                                             const float2* __restrict__ twL,
                                                                             const float2* __restrict__ twM,
                                                                             float scale) {
    constexpr int L = M / 2, P = Pts<L>::value, T = L / P, PITCH = L + 1;
    extern __shared__ float2 lds[];
    const int tid = threadIdx.x;
    const int nrb = N / RB;
    const int plane = blockIdx.x / nrb;
    const int row0 = (blockIdx.x % nrb) * RB;
    {
        const int r2 = tid % RB, kk = tid / RB;
        float2* s2 = lds + r2 * PITCH;
        const float2* src = in + (size_t)plane * L * N + row0 + r2;
#pragma unroll
        for (int i = 0; i < P; ++i) {
            const int k = kk + T * i;
            s2[k] = src[(size_t)k * N];
        }
    }
    __syncthreads();
    const int t = tid % T, r = tid / T;
    float2* s = lds + r * PITCH;
    float2 v[P];
    const float2 P0 = s[0];
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const int k = t + T * q;
        float2 X = s[k], Xm = s[(L - k) & (L - 1)];
        if (k == 0) {
            X = make_float2(P0.x, 0.0f);
            Xm = make_float2(P0.y, 0.0f);
        }
        const float2 A = make_float2(X.x + Xm.x, X.y - Xm.y);  // X + conj(Xm)
        const float2 D = make_float2(X.x - Xm.x, X.y + Xm.y);  // X - conj(Xm)
        const float2 B = cmul(D, cconj(twM[k]));
        v[q] = make_float2(A.x - B.y, A.y + B.x);  // A + i B
    }
    __syncthreads();
    fft<L, P, true>(v, s, t, twL);
    float2* dst = reinterpret_cast<float2*>(out + ((size_t)plane * N + row0 + r) * M);
#pragma unroll
    for (int q = 0; q < P; ++q) dst[t + T * q] = cscale(v[q], scale);
}

// ---------------------------------------------------------------- column passes

template <int N, int PW>
struct ColCfg {
    static constexpr int P = Pts<N>::value;
    static constexpr int T = N / P;
    static constexpr int THREADS = PW * T;
    static constexpr size_t LDS = (size_t)(PW + 1) * N * sizeof(float2);
};

template <bool REAL>
__device__ __forceinline__ float2 fmul(const void* __restrict__ f, size_t i, float2 a) {
    if constexpr (REAL) {
        return cscale(a, reinterpret_cast<const float*>(f)[i]);
    } else {
        return cmul(a, reinterpret_cast<const float2*>(f)[i]);
    }
}

template <int N, int PW, bool REAL>
__global__ __launch_bounds__((ColCfg<N, PW>::THREADS)) void k_cols_fwd(const float2* __restrict__ A,
                                                                    float2* __restrict__ Tout,
                                                                    const void* __restrict__ filt, int L, int K,
                                                                    int npan, const float2* __restrict__ twN,
                                                                    float scale) {
    using C = ColCfg<N, PW>;
    constexpr int P = C::P, T = C::T;
    extern __shared__ float2 lds[];
    const int tid = threadIdx.x;
    const int t = tid % T, c = tid / T;
    const int pan = blockIdx.x % npan, b = blockIdx.x / npan;
    const int col = pan * PW + c;
    float2* s = lds + c * N;
    float2* smir = lds + PW * N;
    const float2* a = A + ((size_t)b * L + col) * N;
    float2 xh[P];
#pragma unroll
    for (int q = 0; q < P; ++q) xh[q] = cscale(a[t + T * q], scale);
    fft<N, P, false>(xh, s, t, twN);
    if (col == 0) {
#pragma unroll
        for (int q = 0; q < P; ++q) smir[t + T * q] = xh[q];
    }
    __syncthreads();
    const size_t fstride = (size_t)(L + 1) * N;
    for (int k = 0; k < K; ++k) {
        const size_t fbase = (size_t)k * fstride + (size_t)col * N;
        float2 y[P];
#pragma unroll
        for (int q = 0; q < P; ++q) y[q] = fmul<REAL>(filt, fbase + t + T * q, xh[q]);
        if (col == 0) {
            const size_t bbase = (size_t)k * fstride + (size_t)L * N;
#pragma unroll
            for (int q = 0; q < P; ++q) {
                const int m = t + T * q;
                y[q] = cadd(y[q], fmul<REAL>(filt, bbase + m, cconj(smir[(N - m) & (N - 1)])));
            }
        }
        fft<N, P, true>(y, s, t, twN);
        float2* o = Tout + (((size_t)b * K + k) * L + col) * N;
#pragma unroll
        for (int q = 0; q < P; ++q) o[t + T * q] = y[q];
    }
}

template <int N, int PW, bool REAL>
__global__ __launch_bounds__((ColCfg<N, PW>::THREADS)) void k_cols_inv(const float2* __restrict__ U,
                                                                    float2* __restrict__ V,
                                                                    const void* __restrict__ filt, int L, int K,
                                                                    int npan, const float2* __restrict__ twN) {
    using C = ColCfg<N, PW>;
    constexpr int P = C::P, T = C::T;
    extern __shared__ float2 lds[];
    const int tid = threadIdx.x;
    const int t = tid % T, c = tid / T;
    const int pan = blockIdx.x % npan, b = blockIdx.x / npan;
    const int col = pan * PW + c;
    float2* s = lds + c * N;
    float2* smir = lds + PW * N;
    float2 acc[P], g[P];
#pragma unroll
    for (int q = 0; q < P; ++q) acc[q] = g[q] = make_float2(0.0f, 0.0f);
    const size_t fstride = (size_t)(L + 1) * N;
    for (int k = 0; k < K; ++k) {
        const float2* u = U + (((size_t)b * K + k) * L + col) * N;
        float2 x[P];
#pragma unroll
        for (int q = 0; q < P; ++q) x[q] = u[t + T * q];
        fft<N, P, false>(x, s, t, twN);
        const size_t fbase = (size_t)k * fstride + (size_t)col * N;
#pragma unroll
        for (int q = 0; q < P; ++q) acc[q] = cadd(acc[q], fmul<REAL>(filt, fbase + t + T * q, x[q]));
        if (col == 0) {
            const size_t gbase = (size_t)k * fstride + (size_t)L * N;
#pragma unroll
            for (int q = 0; q < P; ++q) g[q] = cadd(g[q], fmul<REAL>(filt, gbase + t + T * q, x[q]));
        }
    }
    if (col == 0) {
#pragma unroll
        for (int q = 0; q < P; ++q) smir[t + T * q] = g[q];
    }
    __syncthreads();
    if (col == 0) {
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const int m = t + T * q;
            acc[q] = cadd(acc[q], cconj(smir[(N - m) & (N - 1)]));
        }
    }
    fft<N, P, true>(acc, s, t, twN);
    float2* o = V + ((size_t)b * L + col) * N;
#pragma unroll
    for (int q = 0; q < P; ++q) o[t + T * q] = acc[q];
}

// ---------------------------------------------------------------- dispatch

template <typename F>
hipError_t set_lds(F* fn, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int M, int TAG>
hipError_t rows_r2c_t(const DevPlan& d, const float* in, float2* out, int planes, hipStream_t st) {
    constexpr int L = M / 2, P = Pts<L>::value, T = L / P;
    const size_t lds = (size_t)RB * (L + 1) * sizeof(float2);
    hipError_t e = set_lds(k_rows_r2c<M, TAG>, lds);
    if (e != hipSuccess) return e;
    const size_t blocks = (size_t)planes * (d.N / RB);
    hipLaunchKernelGGL((k_rows_r2c<M, TAG>), dim3((unsigned)blocks), dim3(RB * T), lds, st, in, out, d.N, d.twL, d.twM);
    return hipGetLastError();
}

template <int M, int TAG>
hipError_t rows_c2r_t(const DevPlan& d, const float2* in, float* out, int planes, float scale, hipStream_t st) {
    constexpr int L = M / 2, P = Pts<L>::value, T = L / P;
    const size_t lds = (size_t)RB * (L + 1) * sizeof(float2);
    hipError_t e = set_lds(k_rows_c2r<M, TAG>, lds);
    if (e != hipSuccess) return e;
    const size_t blocks = (size_t)planes * (d.N / RB);
    hipLaunchKernelGGL((k_rows_c2r<M, TAG>), dim3((unsigned)blocks), dim3(RB * T), lds, st, in, out, d.N, d.twL,
                       d.twM, scale);
    return hipGetLastError();
}

template <int N, int PW>
hipError_t cols_fwd_t(const DevPlan& d, const float2* A, float2* T, int nimg, const void* filt, float scale,
                      hipStream_t st) {
    using C = ColCfg<N, PW>;
    const int npan = d.L / PW;
    const size_t blocks = (size_t)npan * nimg;
    if (d.real) {
        hipError_t e = set_lds(k_cols_fwd<N, PW, true>, C::LDS);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_cols_fwd<N, PW, true>), dim3((unsigned)blocks), dim3(C::THREADS), C::LDS, st, A, T,
                           filt, d.L, d.K, npan, d.twN, scale);
    } else {
        hipError_t e = set_lds(k_cols_fwd<N, PW, false>, C::LDS);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_cols_fwd<N, PW, false>), dim3((unsigned)blocks), dim3(C::THREADS), C::LDS, st, A, T,
                           filt, d.L, d.K, npan, d.twN, scale);
    }
    return hipGetLastError();
}

template <int N, int PW>
hipError_t cols_inv_t(const DevPlan& d, const float2* U, float2* V, int nimg, const void* filt, hipStream_t st) {
    using C = ColCfg<N, PW>;
    const int npan = d.L / PW;
    const size_t blocks = (size_t)npan * nimg;
    if (d.real) {
        hipError_t e = set_lds(k_cols_inv<N, PW, true>, C::LDS);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_cols_inv<N, PW, true>), dim3((unsigned)blocks), dim3(C::THREADS), C::LDS, st, U, V,
                           filt, d.L, d.K, npan, d.twN);
    } else {
        hipError_t e = set_lds(k_cols_inv<N, PW, false>, C::LDS);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_cols_inv<N, PW, false>), dim3((unsigned)blocks), dim3(C::THREADS), C::LDS, st, U, V,
                           filt, d.L, d.K, npan, d.twN);
    }
    return hipGetLastError();
}

}  // namespace

bool size_supported(int n) { return n == 16 || n == 32 || n == 64 || n == 128 || n == 256 || n == 512 || n == 1024; }

template <int TAG>
hipError_t rows_r2c_sw(const DevPlan& d, const float* in, float2* out, int planes, hipStream_t st) {
    switch (d.M) {
        case 16: return rows_r2c_t<16, TAG>(d, in, out, planes, st);
        case 32: return rows_r2c_t<32, TAG>(d, in, out, planes, st);
        case 64: return rows_r2c_t<64, TAG>(d, in, out, planes, st);
        case 128: return rows_r2c_t<128, TAG>(d, in, out, planes, st);
        case 256: return rows_r2c_t<256, TAG>(d, in, out, planes, st);
        case 512: return rows_r2c_t<512, TAG>(d, in, out, planes, st);
        case 1024: return rows_r2c_t<1024, TAG>(d, in, out, planes, st);
    }
    return hipErrorInvalidValue;
}

template <int TAG>
hipError_t rows_c2r_sw(const DevPlan& d, const float2* in, float* out, int planes, float scale, hipStream_t st) {
    switch (d.M) {
        case 16: return rows_c2r_t<16, TAG>(d, in, out, planes, scale, st);
        case 32: return rows_c2r_t<32, TAG>(d, in, out, planes, scale, st);
        case 64: return rows_c2r_t<64, TAG>(d, in, out, planes, scale, st);
        case 128: return rows_c2r_t<128, TAG>(d, in, out, planes, scale, st);
        case 256: return rows_c2r_t<256, TAG>(d, in, out, planes, scale, st);
        case 512: return rows_c2r_t<512, TAG>(d, in, out, planes, scale, st);
        case 1024: return rows_c2r_t<1024, TAG>(d, in, out, planes, scale, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_rows_r2c(const DevPlan& d, const float* in, float2* out, int planes, bool coeff_planes,
                           hipStream_t st) {
    return coeff_planes ? rows_r2c_sw<1>(d, in, out, planes, st) : rows_r2c_sw<0>(d, in, out, planes, st);
}

hipError_t launch_rows_c2r(const DevPlan& d, const float2* in, float* out, int planes, float scale, bool coeff_planes,
                           hipStream_t st) {
    return coeff_planes ? rows_c2r_sw<1>(d, in, out, planes, scale, st) : rows_c2r_sw<0>(d, in, out, planes, scale, st);
}

#define SHEAR_COLS_SWITCH(FN, ...)                                                 \
    if (d.L >= 16) {                                                               \
        switch (d.N) {                                                             \
            case 16: return FN<16, 16>(__VA_ARGS__);                               \
            case 32: return FN<32, 16>(__VA_ARGS__);                               \
            case 64: return FN<64, 16>(__VA_ARGS__);                               \
            case 128: return FN<128, 16>(__VA_ARGS__);                             \
            case 256: return FN<256, 16>(__VA_ARGS__);                             \
            case 512: return FN<512, 16>(__VA_ARGS__);                             \
            case 1024: return FN<1024, 16>(__VA_ARGS__);                           \
        }                                                                          \
    } else if (d.L == 8) {                                                         \
        switch (d.N) {                                                             \
            case 16: return FN<16, 8>(__VA_ARGS__);                                \
            case 32: return FN<32, 8>(__VA_ARGS__);                                \
            case 64: return FN<64, 8>(__VA_ARGS__);                                \
            case 128: return FN<128, 8>(__VA_ARGS__);                              \
            case 256: return FN<256, 8>(__VA_ARGS__);                              \
            case 512: return FN<512, 8>(__VA_ARGS__);                              \
            case 1024: return FN<1024, 8>(__VA_ARGS__);                            \
        }                                                                          \
    }                                                                              \
    return hipErrorInvalidValue;

hipError_t launch_cols_fwd(const DevPlan& d, const float2* A, float2* T, int nimg, const void* filt, float scale,
                           hipStream_t st) {
    SHEAR_COLS_SWITCH(cols_fwd_t, d, A, T, nimg, filt, scale, st)
}

hipError_t launch_cols_inv(const DevPlan& d, const float2* U, float2* V, int nimg, const void* filt, hipStream_t st) {
    SHEAR_COLS_SWITCH(cols_inv_t, d, U, V, nimg, filt, st)
}

}  // namespace shear
