// Device-side FFT building blocks shared by the gfx950 kernels of the filter bank:
// complex helpers, streaming accesses, the panel layout of intermediate planes,
// in-register DFT butterflies and Stockham autosort passes staged in LDS.
//
// FFTs are Stockham autosort passes (radix 2/4/8/16 butterflies in
// registers, LDS between passes). A thread of an FFT group of T = L/P threads
// holds P points: on input x[t + T q], on output X[t + T q], q < P.
#pragma once

#include <hip/hip_runtime.h>

namespace shear {
namespace dev {

// ---------------------------------------------------------------- complex helpers

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// The fused multiply-adds are written out so that every kernel rounds a complex product the
// same way (left to the compiler, contraction can differ between kernels that inline it).
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
// multiply by -i (forward sign) or +i (inverse sign)
template <bool INV>
__device__ __forceinline__ float2 mul_mi(float2 a) {
    return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// Streaming global accesses (each byte touched once per launch): non-temporal hints.
typedef float v2f __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 ld_stream(const float2* p) {
    const v2f v = __builtin_nontemporal_load(reinterpret_cast<const v2f*>(p));
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ void st_stream(float2* p, float2 a) {
    const v2f v = {a.x, a.y};
    __builtin_nontemporal_store(v, reinterpret_cast<v2f*>(p));
}
// Accesses of exchange planes: non-temporal when the plane makes a round trip
// through HBM (NT), ordinary when it is meant to stay in the XCD's L2.
template <bool NT>
__device__ __forceinline__ float2 ld_x(const float2* p) {
    if constexpr (NT) {
        return ld_stream(p);
    } else {
        return *p;
    }
}
template <bool NT>
__device__ __forceinline__ void st_x(float2* p, float2 a) {
    if constexpr (NT) {
        st_stream(p, a);
    } else {
        *p = a;
    }
}

// Layout of an intermediate N x L packed plane (N a multiple of 16, L of 8):
// panels of 8 consecutive columns, each panel N x 8 float2 contiguous, made of
// tiles of 16 rows x 8 columns (128 float2, column-major inside the tile, so 16
// rows of one column are one 128-byte line), tile after tile down the panel.
// A column pass reads or writes whole panels as contiguous runs, as with a
// column-major plane; a row pass over 16 rows reads or writes one 1 KB run per
// panel instead of one 128-byte line per column.
__device__ __forceinline__ size_t xoff(int row, int col, int N) {
    return (size_t)(col >> 3) * ((size_t)N << 3) + (size_t)(((row >> 4) << 7) | ((col & 7) << 4) | (row & 15));
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

// ---------------------------------------------------------------- wave-level sync
// An FFT group of T = L/P <= 64 threads (aligned) lives inside one wavefront,
// and its LDS scratch is private to the group. LDS operations of a wavefront
// execute in issue order, so ordering the group's LDS writes before its reads
// needs only a compiler-level fence, not a workgroup barrier.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A group of more than 64 threads (the 2048-point column FFTs: 128 threads of 16 points) spans
// several wavefronts and synchronises with a workgroup barrier; every thread of such a block runs
// the same FFT calls, so all of them reach every barrier.
template <int T>
__device__ __forceinline__ void group_sync() {
    if constexpr (T <= 64) {
        wave_sync();
    } else {
        __syncthreads();
    }
}

// ---------------------------------------------------------------- Stockham FFT
// One pass with radix R = min(P, L/NS) over the L points of an FFT group.
// FIRST: inputs come from registers; LAST: outputs go to registers. Otherwise
// the pass reads the group's LDS scratch s (L float2), synchronises, and
// writes back. Every pass that reads LDS ends its read phase with a sync, so a
// following pass (or a following FFT) may write s immediately.
// LDS layout of one exchange between passes. A pass with stride NS and radix R
// writes runs of NS consecutive addresses spaced NS*R apart; inserting NS
// padding slots every NS*R slots puts consecutive runs on distinct banks.
// The next pass reads consecutive addresses, which the padding keeps
// consecutive within each 16-aligned lane group. Runs of 16 or more need no
// padding. Footprint: L + L/R slots.
template <int NS, int R>
__device__ __forceinline__ int xmap(int a) {
    if constexpr (NS >= 16) {
        return a;
    } else {
        return a + NS * (a / (NS * R));
    }
}

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
            group_sync<T>();
#pragma unroll
            for (int i = 0; i < BPT; ++i)
#pragma unroll
                for (int r = 0; r < R; ++r) u[i + BPT * r] = s[xmap<NS / P, P>((t + T * i) + r * (L / R))];
            group_sync<T>();
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
                for (int r = 0; r < R; ++r) s[xmap<NS, R>(idxD + r * NS)] = w[r];
            }
        }
        if constexpr (!LAST) FFTPass<L, P, INV, NS * R, false>::run(v, s, t, tw);
    }
};

template <int L, int P, bool INV>
__device__ __forceinline__ void fft(float2 (&v)[P], float2* s, int t, const float2* __restrict__ tw) {
    FFTPass<L, P, INV, 1, true>::run(v, s, t, tw);
}

template <bool REAL>
__device__ __forceinline__ float2 fmul(const void* __restrict__ f, size_t i, float2 a) {
    if constexpr (REAL) {
        return cscale(a, reinterpret_cast<const float*>(f)[i]);
    } else {
        return cmul(a, reinterpret_cast<const float2*>(f)[i]);
    }
}

}  // namespace dev
}  // namespace shear
