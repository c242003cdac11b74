// gfx950 kernels of the FFT-domain shearlet filter bank.
//
// Data flow (Algorithm 1 / Algorithm 2 of Section 3.4.2 with the Fourier
// shifts folded into the stored filter order):
//   forward  x --rows r2c--> A --columns: FFT, x conj filter_k, IFFT--> T_k --rows c2r--> c_k
//   inverse  c_k --rows r2c--> U_k --columns: FFT, x dual filter_k, sum_k, IFFT--> V --rows c2r--> y
// A real row of M samples is transformed as M/2 complex samples plus a
// post-twiddle; the real DC and Nyquist bins of each row spectrum share one
// complex slot ("packed" column 0), so every intermediate plane is N x M/2
// complex, stored in panels of 8 columns made of 16-row tiles (xoff below).
//
// FFTs are Stockham autosort passes (radix 2/4/8/16 butterflies in
// registers, LDS between passes). A thread of an FFT group of T = L/P threads
// holds P points: on input x[t + T q], on output X[t + T q], q < P.
#include "kernels.h"

#include <algorithm>

namespace shear {
namespace {

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
// Every FFT group (T = L/P <= 64 threads, aligned) lives inside one wavefront,
// and its LDS scratch is private to the group. LDS operations of a wavefront
// execute in issue order, so ordering the group's LDS writes before its reads
// needs only a compiler-level fence, not a workgroup barrier.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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
            static_assert(T <= 64, "an FFT group must fit in one wavefront");
            wave_sync();
#pragma unroll
            for (int i = 0; i < BPT; ++i)
#pragma unroll
                for (int r = 0; r < R; ++r) u[i + BPT * r] = s[xmap<NS / P, P>((t + T * i) + r * (L / R))];
            wave_sync();
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

// points per thread for an FFT of length L (standalone kernels)
template <int L>
struct Pts {
    static constexpr int value = (L >= 1024) ? 16 : (L == 256 ? 16 : 8);
};

// points per thread of the column FFTs (N-point): 8 up to N = 512 (256-point columns use two
// 32-thread groups per wavefront), 16 at N = 1024
template <int N>
struct ColPts {
    static constexpr int value = (N >= 1024) ? 16 : 8;
};

constexpr int RB = 16;  // rows per block in the standalone row passes (32 measured slower once the twiddle
                        // loads were off the tiles' critical path: 0.273 against 0.261 ms for the
                        // coefficient r2c pass at 512 x 512 x 49 x 16)

// rows per block of a standalone row pass: R, or fewer where that would exceed 512 threads (at
// M = 1024 a 1024-thread block of 16 rows filled its CU alone, so the phases of one block could
// not overlap another's)
template <int M, int R>
constexpr int cap_rows() {
    constexpr int T = (M / 2) / Pts<M / 2>::value;
    return (R * T <= 512) ? R : 512 / T;
}

// Logical block of a standalone row pass. Workgroups go to the 8 XCDs (each with its own L2) in
// turn, so hardware blocks b, b + 8, b + 16, ... share an XCD and start together. Where a block
// holds fewer than the 16 rows of a panel tile (S = 16 / ROWS blocks per tile), the S blocks of one
// tile get such a set of hardware blocks, so that each 128-byte line of the tile is read and
// written through one L2; a tail of fewer than 8 S blocks keeps its order.
template <int ROWS>
__device__ __forceinline__ int row_block() {
    static_assert(ROWS >= 16 || 16 % ROWS == 0, "rows per block must divide the 16-row tile");
    const int b = (int)blockIdx.x;
    if constexpr (ROWS >= 16) {
        return b;
    } else {
        constexpr int S = 16 / ROWS, G = 8 * S;
        if (b >= (int)(gridDim.x / G) * G) return b;
        const int w = b % G;
        return b - w + (w % 8) * S + w / 8;
    }
}

template <bool REAL>
__device__ __forceinline__ float2 fmul(const void* __restrict__ f, size_t i, float2 a) {
    if constexpr (REAL) {
        return cscale(a, reinterpret_cast<const float*>(f)[i]);
    } else {
        return cmul(a, reinterpret_cast<const float2*>(f)[i]);
    }
}

// ---------------------------------------------------------------- row tiles
// A tile is ROWS consecutive rows of one plane, handled by ROWS * (L/P) threads
// (thread t of row r is threadIdx.x = t + (L/P) r). lds holds ROWS * RowPitch<L, P>
// float2, plus L twiddles where a tile copies its FFT's twiddles there. The caller
// separates consecutive tiles that reuse lds with a barrier.

// real rows -> packed spectra, plane out in the panel layout (xoff)
// per-row LDS pitch of the row tiles: FFT scratch footprint plus one slot, so
// that column-wise accesses of consecutive rows fall on different banks
template <int L, int P>
struct RowPitch {
    static constexpr int value = L + L / P + 1;
};

// load(row, i) returns samples 2i and 2i+1 of a row of the plane.
// TWLDS: the FFT's twiddles twL are copied to LDS after the row scratches (L more float2)
// while the tile loads are in flight, one barrier before the FFT, which then reads them there.
template <int M, int P, int ROWS, bool XS, typename Load, bool TWLDS = false>
__device__ __forceinline__ void row_r2c_tile_ld(const Load& load, float2* __restrict__ out_plane, int N, int row0,
                                                float2* lds, const float2* __restrict__ twL,
                                                const float2* __restrict__ twM, const int tid) {
    constexpr int L = M / 2, T = L / P, PITCH = RowPitch<L, P>::value;
    constexpr int TWN = TWLDS ? (L + ROWS * T - 1) / (ROWS * T) : 0;  // twiddles copied per thread
    const int t = tid % T, r = tid / T;
    const int r2 = tid % ROWS, kk = tid / ROWS;
    float2* s = lds + r * PITCH;
    float2 twv[TWN > 0 ? TWN : 1];
#pragma unroll
    for (int j = 0; j < TWN; ++j) {
        const int i = tid + j * ROWS * T;
        if (i < L) twv[j] = twL[i];
    }
    float2 v[P];
#pragma unroll
    for (int q = 0; q < P; ++q) v[q] = load(row0 + r, t + T * q);
    // post-twiddle of column kk + T i as twM[kk] twM[T i]: one per-lane load, issued before any
    // store of the tile, and the wave-uniform twM[T i] (scalar loads)
    const float2 tw0 = twM[kk];
    const float2* twf = twL;
    if constexpr (TWLDS) {
        float2* stw = lds + ROWS * PITCH;
#pragma unroll
        for (int j = 0; j < TWN; ++j) {
            const int i = tid + j * ROWS * T;
            if (i < L) stw[i] = twv[j];
        }
        twf = stw;
        __syncthreads();
    }
    fft<L, P, false>(v, s, t, twf);
#pragma unroll
    for (int q = 0; q < P; ++q) s[t + T * q] = v[q];
    __syncthreads();
    const float2* s2 = lds + r2 * PITCH;
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
            X = cadd(E, cmul(i == 0 ? tw0 : cmul(tw0, twM[T * i]), O));
        }
        st_x<XS>(out_plane + xoff(row0 + r2, k, N), X);
    }
}

template <int M, int P, int ROWS, bool XS = true, bool TWLDS = false>
__device__ __forceinline__ void row_r2c_tile(const float* __restrict__ in_plane, float2* __restrict__ out_plane, int N,
                                             int row0, float2* lds, const float2* __restrict__ twL,
                                             const float2* __restrict__ twM, const int tid) {
    const float2* src = reinterpret_cast<const float2*>(in_plane);
    auto ld = [src](int row, int i) { return ld_stream(src + (size_t)row * (M / 2) + i); };
    row_r2c_tile_ld<M, P, ROWS, XS, decltype(ld), TWLDS>(
        ld, out_plane, N, row0, lds, twL, twM, tid);
}

// packed spectra (panel layout) -> real rows, out = scale * unnormalised inverse.
// TWLDS: the block copies the FFT's twiddles twL to LDS after the row scratches (L more
// float2) while its tile loads are in flight, and the FFT passes read them there instead of
// with vector-memory loads.
template <int M, int P, int ROWS, bool XS = true, bool TWLDS = false>
__device__ __forceinline__ void row_c2r_tile(const float2* __restrict__ in_plane, float* __restrict__ out_plane, int N,
                                             int row0, float2* lds, const float2* __restrict__ twL,
                                             const float2* __restrict__ twM, float scale, const int tid) {
    constexpr int L = M / 2, T = L / P, PITCH = RowPitch<L, P>::value;
    constexpr int TWN = TWLDS ? (L + ROWS * T - 1) / (ROWS * T) : 0;  // twiddles copied per thread
    const int t = tid % T, r = tid / T;
    // pre-twiddle of column t + T q as twM[t] twM[T q] (one per-lane load, issued with the tile's
    // loads; twM[T q] is wave-uniform)
    const float2 tw0 = twM[t];
    float2 twv[TWN > 0 ? TWN : 1];
#pragma unroll
    for (int j = 0; j < TWN; ++j) {
        const int i = tid + j * ROWS * T;
        if (i < L) twv[j] = twL[i];
    }
    {
        const int r2 = tid % ROWS, kk = tid / ROWS;
        float2* s2 = lds + r2 * PITCH;
#pragma unroll
        for (int i = 0; i < P; ++i) {
            const int k = kk + T * i;
            s2[k] = ld_x<XS>(in_plane + xoff(row0 + r2, k, N));
        }
    }
    const float2* twf = twL;
    if constexpr (TWLDS) {
        float2* stw = lds + ROWS * PITCH;
#pragma unroll
        for (int j = 0; j < TWN; ++j) {
            const int i = tid + j * ROWS * T;
            if (i < L) stw[i] = twv[j];
        }
        twf = stw;
    }
    __syncthreads();
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
        const float2 B = cmul(D, cconj(q == 0 ? tw0 : cmul(tw0, twM[T * q])));
        v[q] = make_float2(A.x - B.y, A.y + B.x);  // A + i B
    }
    __syncthreads();
    fft<L, P, true>(v, s, t, twf);
    float2* dst = reinterpret_cast<float2*>(out_plane + (size_t)(row0 + r) * M);
#pragma unroll
    for (int q = 0; q < P; ++q) st_stream(dst + t + T * q, cscale(v[q], scale));
}

// ---------------------------------------------------------------- column panels
// A panel is PW consecutive columns [col0, col0 + PW) of an N x L packed plane
// in the panel layout (element (row, col) at xoff(row, col, N)), handled by
// PW * (N/P) threads: thread t of panel column c is threadIdx.x = t + (N/P) c.
// lds holds PW FFT scratches of ColScratch<N, P> float2 plus the N-float2
// mirror buffer used by packed column 0.
template <int N, int P>
struct ColScratch {
    static constexpr int value = N + N / P;
};

// X = scale * colFFT(a panel); column 0's spectrum is also left in the mirror buffer.
template <int N, int P, int PW>
__device__ __forceinline__ void col_fwd_setup(const float2* __restrict__ a_img, int col0, float2 (&xh)[P], float2* lds,
                                              float scale, const float2* __restrict__ twN, const int tid) {
    constexpr int T = N / P;
    const int t = tid % T, c = tid / T;
    const int col = col0 + c;
    float2* s = lds + c * ColScratch<N, P>::value;
    float2* smir = lds + PW * ColScratch<N, P>::value;
#pragma unroll
    for (int q = 0; q < P; ++q) xh[q] = cscale(a_img[xoff(t + T * q, col, N)], scale);
    fft<N, P, false>(xh, s, t, twN);
    if (col == 0) {
#pragma unroll
        for (int q = 0; q < P; ++q) smir[t + T * q] = xh[q];
    }
    __syncthreads();
}

// out panel = colIFFT(filter_k (.) X); packed column 0 uses alpha X(m) + beta conj X(-m).
template <int N, int P, int PW, bool REAL, bool XS = true>
__device__ __forceinline__ void col_fwd_emit(const float2 (&xh)[P], const void* __restrict__ filt, int k, int L,
                                             int col0, float2* __restrict__ out_plane, float2* lds,
                                             const float2* __restrict__ twN, const int tid) {
    constexpr int T = N / P;
    const int t = tid % T, c = tid / T;
    const int col = col0 + c;
    float2* s = lds + c * ColScratch<N, P>::value;
    const float2* smir = lds + PW * ColScratch<N, P>::value;
    const size_t fstride = (size_t)(L + 1) * N;
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
#pragma unroll
    for (int q = 0; q < P; ++q) st_x<XS>(out_plane + xoff(t + T * q, col, N), y[q]);
}

// The mirrored-term accumulator g of packed column 0 lives in the panel's
// mirror buffer (N float2 of LDS after the FFT scratches), written only by the
// threads of column 0, each on its own entries: it costs no registers.
template <int N, int P, int PW>
__device__ __forceinline__ void col_inv_begin(int col0, float2* lds, const int tid) {
    constexpr int T = N / P;
    const int t = tid % T, c = tid / T;
    float2* smir = lds + PW * ColScratch<N, P>::value;
    if (col0 + c == 0) {
#pragma unroll
        for (int q = 0; q < P; ++q) smir[t + T * q] = make_float2(0.0f, 0.0f);
    }
}

// acc += filter_k (.) colFFT(u panel); packed column 0 also accumulates g for the mirrored term.
template <int N, int P, int PW, bool REAL, bool XS = true>
__device__ __forceinline__ void col_inv_accum(const float2* __restrict__ u_plane, const void* __restrict__ filt, int k,
                                              int L, int col0, float2 (&acc)[P], float2* lds,
                                              const float2* __restrict__ twN, const int tid) {
    constexpr int T = N / P;
    const int t = tid % T, c = tid / T;
    const int col = col0 + c;
    float2* s = lds + c * ColScratch<N, P>::value;
    float2 x[P];
#pragma unroll
    for (int q = 0; q < P; ++q) x[q] = ld_x<XS>(u_plane + xoff(t + T * q, col, N));
    fft<N, P, false>(x, s, t, twN);
    const size_t fstride = (size_t)(L + 1) * N;
    const size_t fbase = (size_t)k * fstride + (size_t)col * N;
#pragma unroll
    for (int q = 0; q < P; ++q) acc[q] = cadd(acc[q], fmul<REAL>(filt, fbase + t + T * q, x[q]));
    if (col == 0) {
        float2* g = lds + PW * ColScratch<N, P>::value;
        const size_t gbase = (size_t)k * fstride + (size_t)L * N;
#pragma unroll
        for (int q = 0; q < P; ++q) g[t + T * q] = cadd(g[t + T * q], fmul<REAL>(filt, gbase + t + T * q, x[q]));
    }
}

// v panel = colIFFT(acc + [column 0: conj g(-m)]), g in the mirror buffer
template <int N, int P, int PW>
__device__ __forceinline__ void col_inv_finish(float2 (&acc)[P], int col0, float2* __restrict__ v_img, float2* lds,
                                               const float2* __restrict__ twN, const int tid) {
    constexpr int T = N / P;
    const int t = tid % T, c = tid / T;
    const int col = col0 + c;
    float2* s = lds + c * ColScratch<N, P>::value;
    const float2* smir = lds + PW * ColScratch<N, P>::value;
    __syncthreads();  // every thread of column 0 has finished its entries of g
    if (col == 0) {
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const int m = t + T * q;
            acc[q] = cadd(acc[q], cconj(smir[(N - m) & (N - 1)]));
        }
    }
    fft<N, P, true>(acc, s, t, twN);
#pragma unroll
    for (int q = 0; q < P; ++q) v_img[xoff(t + T * q, col, N)] = acc[q];
}

// ---------------------------------------------------------------- standalone kernels

// TAG only separates launch roles into distinct symbols (0: images, 1: coefficient planes)
template <int M, int TAG, int ROWS>
__global__ __launch_bounds__(ROWS*(M / 2) / Pts<M / 2>::value) void k_rows_r2c(const float* __restrict__ in,
                                                                             float2* __restrict__ out, int N,
                                                                             const float2* __restrict__ twL,
                                                                             const float2* __restrict__ twM) {
    constexpr int L = M / 2;
    extern __shared__ float2 lds[];
    const int nrb = N / ROWS;
    const int blk = row_block<ROWS>();
    const int plane = blk / nrb;
    const int row0 = (blk % nrb) * ROWS;
    row_r2c_tile<M, Pts<L>::value, ROWS, true, true>(in + (size_t)plane * N * M, out + (size_t)plane * L * N, N, row0,
                                                     lds, twL, twM, (int)threadIdx.x);
}

// Row stage of one inpainting iteration (Algorithm 3): the rows of
// u = mask (f_masked - f) + f, formed while loading, -> packed spectra.
template <int M, int ROWS>
__global__ __launch_bounds__(ROWS*(M / 2) / Pts<M / 2>::value) void k_rows_r2c_mix(const float* __restrict__ fm,
                                                                                const float* __restrict__ mask,
                                                                                const float* __restrict__ f,
                                                                                float2* __restrict__ out, int N,
                                                                                const float2* __restrict__ twL,
                                                                                const float2* __restrict__ twM) {
    constexpr int L = M / 2;
    extern __shared__ float2 lds[];
    const int nrb = N / ROWS;
    const int blk = row_block<ROWS>();
    const int plane = blk / nrb;
    const int row0 = (blk % nrb) * ROWS;
    const size_t off = (size_t)plane * N * L;  // float2 units
    const float2* a = reinterpret_cast<const float2*>(fm) + off;
    const float2* m = reinterpret_cast<const float2*>(mask) + off;
    const float2* g = reinterpret_cast<const float2*>(f) + off;
    auto ld = [a, m, g](int row, int i) {
        const size_t j = (size_t)row * L + i;
        const float2 av = ld_stream(a + j), mv = ld_stream(m + j), gv = g[j];
        return make_float2(mv.x * (av.x - gv.x) + gv.x, mv.y * (av.y - gv.y) + gv.y);
    };
    row_r2c_tile_ld<M, Pts<L>::value, ROWS, true, decltype(ld), true>(ld, out + (size_t)plane * L * N, N, row0, lds,
                                                                      twL, twM, (int)threadIdx.x);
}

template <int M, int TAG, int ROWS>
__global__ __launch_bounds__(ROWS*(M / 2) / Pts<M / 2>::value) void k_rows_c2r(const float2* __restrict__ in,
                                                                             float* __restrict__ out, int N,
                                                                             const float2* __restrict__ twL,
                                                                             const float2* __restrict__ twM,
                                                                             float scale) {
    constexpr int L = M / 2, P = Pts<L>::value;
    extern __shared__ float2 lds[];
    const int nrb = N / ROWS;
    const int blk = row_block<ROWS>();
    const int plane = blk / nrb;
    const int row0 = (blk % nrb) * ROWS;
    row_c2r_tile<M, P, ROWS, true, true>(in + (size_t)plane * L * N, out + (size_t)plane * N * M, N, row0, lds, twL,
                                         twM, scale, (int)threadIdx.x);
}

// Forward row stage, hard threshold and inverse row stage of one tile of a
// coefficient plane, in place on its packed (panel layout) spectra: the rows
// become real coefficients c (as the forward transform writes them), every
// coefficient with |c| < thr is set to zero, and the thresholded rows are
// transformed back, so thresholded coefficients never leave the chip. The
// number of kept coefficients of the tile is added to *kept (when non-null).
template <int M, int P, int ROWS>
__device__ __forceinline__ void row_thresh_tile(float2* __restrict__ plane, int N, int row0, float2* lds,
                                                const float2* __restrict__ twL, const float2* __restrict__ twM,
                                                float thr, unsigned* __restrict__ kept, const int tid) {
    constexpr int L = M / 2, T = L / P, PITCH = RowPitch<L, P>::value;
    constexpr int TWN = (L + ROWS * T - 1) / (ROWS * T);  // FFT twiddles copied to LDS per thread
    const int r2 = tid % ROWS, kk = tid / ROWS;
    const int t = tid % T, r = tid / T;
    // Twiddles, all loaded with the tile: the FFTs' twL go to LDS after the row scratches
    // (L more float2); the pre- and post-twiddles of columns t + T q and kk + T i are a
    // per-lane base (twM[t], twM[kk]) times the wave-uniform twM[T q].
    float2 twv[TWN];
#pragma unroll
    for (int j = 0; j < TWN; ++j) {
        const int i = tid + j * ROWS * T;
        if (i < L) twv[j] = twL[i];
    }
    const float2 twa = twM[t], twb = twM[kk];
    {
        float2* s2 = lds + r2 * PITCH;
#pragma unroll
        for (int i = 0; i < P; ++i) {
            const int k = kk + T * i;
            s2[k] = ld_stream(plane + xoff(row0 + r2, k, N));
        }
    }
    float2* stw = lds + ROWS * PITCH;
#pragma unroll
    for (int j = 0; j < TWN; ++j) {
        const int i = tid + j * ROWS * T;
        if (i < L) stw[i] = twv[j];
    }
    __syncthreads();
    float2* s = lds + r * PITCH;
    float2 v[P];
    {
        const float2 P0 = s[0];
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const int k = t + T * q;
            float2 X = s[k], Xm = s[(L - k) & (L - 1)];
            if (k == 0) {
                X = make_float2(P0.x, 0.0f);
                Xm = make_float2(P0.y, 0.0f);
            }
            const float2 A = make_float2(X.x + Xm.x, X.y - Xm.y);
            const float2 D = make_float2(X.x - Xm.x, X.y + Xm.y);
            const float2 B = cmul(D, cconj(q == 0 ? twa : cmul(twa, twM[T * q])));
            v[q] = make_float2(A.x - B.y, A.y + B.x);
        }
    }
    __syncthreads();
    fft<L, P, true>(v, s, t, stw);
    // v[q] holds the coefficients at columns 2(t + T q) and 2(t + T q) + 1
    unsigned n = 0;
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const bool kx = fabsf(v[q].x) >= thr, ky = fabsf(v[q].y) >= thr;
        v[q] = make_float2(kx ? v[q].x : 0.0f, ky ? v[q].y : 0.0f);
        n += (kx ? 1u : 0u) + (ky ? 1u : 0u);
    }
    fft<L, P, false>(v, s, t, stw);
#pragma unroll
    for (int q = 0; q < P; ++q) s[t + T * q] = v[q];
    __syncthreads();
    {
        const float2* s2 = lds + r2 * PITCH;
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
                const float2 O = make_float2(D.y, -D.x);
                X = cadd(E, cmul(i == 0 ? twb : cmul(twb, twM[T * i]), O));
            }
            st_stream(plane + xoff(row0 + r2, k, N), X);
        }
    }
    if (kept != nullptr) {
        // sum over each wavefront (or the whole block, if smaller), then one atomic each
        constexpr int WV = (ROWS * T < 64) ? ROWS * T : 64;
#pragma unroll
        for (int off = WV / 2; off >= 1; off >>= 1) n += __shfl_xor(n, off, WV);
        if (tid % WV == 0) atomicAdd(kept, n);
    }
}

// planes[p] for p < gridDim.x / (N / ROWS): threshold thr[p], kept counts kept[p]
template <int M, int ROWS>
__global__ __launch_bounds__(ROWS*(M / 2) / Pts<M / 2>::value) void k_rows_thresh(float2* __restrict__ planes, int N,
                                                                              const float* __restrict__ thr,
                                                                              unsigned* __restrict__ kept,
                                                                              const float2* __restrict__ twL,
                                                                              const float2* __restrict__ twM) {
    constexpr int L = M / 2;
    extern __shared__ float2 lds[];
    const int nrb = N / ROWS;
    const int blk = row_block<ROWS>();
    const int plane = blk / nrb;
    const int row0 = (blk % nrb) * ROWS;
    row_thresh_tile<M, Pts<L>::value, ROWS>(planes + (size_t)plane * L * N, N, row0, lds, twL, twM, thr[plane],
                                          kept ? kept + plane : nullptr, (int)threadIdx.x);
}

template <int N, int PW>
struct ColCfg {
    static constexpr int P = ColPts<N>::value;
    static constexpr int T = N / P;
    static constexpr int THREADS = PW * T;
    static constexpr size_t LDS = ((size_t)PW * ColScratch<N, P>::value + N) * sizeof(float2);
};

// Filter groups: the K filters of a column panel may be split over kg blocks of kper
// consecutive filters (block index = pan + npan (g + kg b)), so that small batches still
// fill the device. The forward recomputes the panel's column FFT in each group; the
// inverse writes one partial sum per group and k_cols_inv_finish adds them in group order.
template <int N, int PW, bool REAL>
__global__ __launch_bounds__((ColCfg<N, PW>::THREADS)) void k_cols_fwd(const float2* __restrict__ A,
                                                                    float2* __restrict__ Tout,
                                                                    const void* __restrict__ filt, int L, int K,
                                                                    int npan, int kper, int kg,
                                                                    const float2* __restrict__ twN, float scale) {
    constexpr int P = ColCfg<N, PW>::P;
    extern __shared__ float2 lds[];
    const int pan = blockIdx.x % npan, g = (blockIdx.x / npan) % kg, b = blockIdx.x / (npan * kg);
    float2 xh[P];
    col_fwd_setup<N, P, PW>(A + (size_t)b * L * N, pan * PW, xh, lds, scale, twN, (int)threadIdx.x);
    const int k1 = min(K, (g + 1) * kper);
    for (int k = g * kper; k < k1; ++k)
        col_fwd_emit<N, P, PW, REAL>(xh, filt, k, L, pan * PW, Tout + ((size_t)b * K + k) * L * N, lds, twN,
                                     (int)threadIdx.x);
}

// kg == 1: V[b] = colIFFT(sum_k ...); kg > 1: part[b][g] (L x N column-major) and, for packed
// column 0, part0[b][g] (N) receive the group's sums.
template <int N, int PW, bool REAL>
__global__ __launch_bounds__((ColCfg<N, PW>::THREADS)) void k_cols_inv(const float2* __restrict__ U,
                                                                    float2* __restrict__ V,
                                                                    const void* __restrict__ filt, int L, int K,
                                                                    int npan, int kper, int kg,
                                                                    float2* __restrict__ part,
                                                                    float2* __restrict__ part0,
                                                                    const float2* __restrict__ twN) {
    constexpr int P = ColCfg<N, PW>::P, T = N / P;
    extern __shared__ float2 lds[];
    const int pan = blockIdx.x % npan, g = (blockIdx.x / npan) % kg, b = blockIdx.x / (npan * kg);
    const int tid = (int)threadIdx.x;
    float2 acc[P];
#pragma unroll
    for (int q = 0; q < P; ++q) acc[q] = make_float2(0.0f, 0.0f);
    col_inv_begin<N, P, PW>(pan * PW, lds, tid);
    const int k1 = min(K, (g + 1) * kper);
    for (int k = g * kper; k < k1; ++k)
        col_inv_accum<N, P, PW, REAL>(U + ((size_t)b * K + k) * L * N, filt, k, L, pan * PW, acc, lds, twN, tid);
    if (kg == 1) {
        col_inv_finish<N, P, PW>(acc, pan * PW, V + (size_t)b * L * N, lds, twN, tid);
        return;
    }
    const int t = tid % T, c = tid / T, col = pan * PW + c;
    float2* o = part + ((size_t)b * kg + g) * L * N + (size_t)col * N;
#pragma unroll
    for (int q = 0; q < P; ++q) o[t + T * q] = acc[q];
    if (col == 0) {
        // each thread of column 0 reads back the entries of the mirrored-term sum it accumulated
        const float2* sg = lds + PW * ColScratch<N, P>::value;
        float2* og = part0 + ((size_t)b * kg + g) * N;
#pragma unroll
        for (int q = 0; q < P; ++q) og[t + T * q] = sg[t + T * q];
    }
}

// V[b] panel = colIFFT(sum_g part[b][g] [+ conj of the mirrored column-0 partials]), g in order
template <int N, int PW>
__global__ __launch_bounds__((ColCfg<N, PW>::THREADS)) void k_cols_inv_finish(const float2* __restrict__ part,
                                                                           const float2* __restrict__ part0,
                                                                           float2* __restrict__ V, int L, int npan,
                                                                           int kg, const float2* __restrict__ twN) {
    constexpr int P = ColCfg<N, PW>::P, T = N / P;
    extern __shared__ float2 lds[];
    const int pan = blockIdx.x % npan, b = blockIdx.x / npan;
    const int tid = (int)threadIdx.x;
    const int t = tid % T, c = tid / T, col = pan * PW + c;
    float2 acc[P], gg[P];
#pragma unroll
    for (int q = 0; q < P; ++q) acc[q] = gg[q] = make_float2(0.0f, 0.0f);
    for (int g = 0; g < kg; ++g) {
        const float2* src = part + ((size_t)b * kg + g) * L * N + (size_t)col * N;
#pragma unroll
        for (int q = 0; q < P; ++q) acc[q] = cadd(acc[q], src[t + T * q]);
        if (col == 0) {
            const float2* sg = part0 + ((size_t)b * kg + g) * N;
#pragma unroll
            for (int q = 0; q < P; ++q) gg[q] = cadd(gg[q], sg[t + T * q]);
        }
    }
    if (col == 0) {
        float2* smir = lds + PW * ColScratch<N, P>::value;
#pragma unroll
        for (int q = 0; q < P; ++q) smir[t + T * q] = gg[q];
    }
    col_inv_finish<N, P, PW>(acc, pan * PW, V + (size_t)b * L * N, lds, twN, tid);
}

// ---------------------------------------------------------------- XCD-local persistent kernels
// One cooperative launch per transform direction fuses the column stage and
// the coefficient row stage, and hands each (image, filter) plane from one
// stage to the other through a small ring of exchange slots that stays in the
// L2 of one XCD. The L2 is the coherence point of the compute units of an XCD
// but not across XCDs, so every slot is produced and consumed by blocks of one
// XCD: each block reads the id of the XCD it runs on (hardware register
// XCC_ID), and takes work only from that XCD's queue.
//
// Start-up census: every block counts itself on its XCD and on a launch-wide
// arrival counter, then waits until all blocks of the (co-resident) grid have
// arrived. The XCDs that hold blocks, in id order, are the queues; image b goes
// to queue b mod Q.
//
// Tasks of a queue, in dequeue order, per group of GI images: the GI x npan
// column tasks (one panel of PW columns of one image, looping over all K
// filters), then the K x GI x nrb row tasks (ROWS rows of one plane), filter
// major. Image i of a group uses the slots i*S .. i*S+S-1 of its queue, filter
// k the slot k mod S; a slot's uses are numbered across the groups
// (generation), and each slot counts the column and the row tasks that have
// finished with it.
//
// Ordering within an XCD: a finishing task waits for its own loads and stores
// (stores are acknowledged by the L2), passes a block barrier, and one thread
// adds to the slot's counter with a relaxed atomic. A waiting task polls the
// counter with relaxed atomic loads, invalidates its compute unit's L1 with an
// acquire fence, and passes a block barrier. No L2 write-back is needed
// because producer and consumer share the L2; kernel boundaries order
// everything else (inputs, outputs, counters).
//
// Progress: a task waits only on tasks dequeued before it, except the column
// tasks of a group, which wait on the row tasks after them; their number
// (GI x npan) must stay below the blocks of the queue, which the census
// checks. Every wait is bounded: on timeout it raises an abort flag that makes
// every other wait give up, so the kernel always drains; the host reports the
// flag through shear_check.

constexpr int SPIN_LIMIT = 1 << 18;
constexpr int kMaxXcc = 16;  // XCC_ID values are taken modulo this

// counter words of a launch: census, arrival, abort flag, queue heads, then
// two counters (column side, row side) per slot
constexpr int CTR_CENSUS = 0;
constexpr int CTR_ARRIVED = kMaxXcc;
constexpr int CTR_ABORT = kMaxXcc + 1;
constexpr int CTR_HEADS = kMaxXcc + 2;
constexpr int CTR_DONE = 2 * kMaxXcc + 2;

__device__ __forceinline__ unsigned xcc_id() {
    // hardware register 20 (XCC_ID): bits [3:0] are the XCD of the wave
    return __builtin_amdgcn_s_getreg(20 | (0 << 6) | ((4 - 1) << 11)) & (kMaxXcc - 1);
}

__device__ __forceinline__ unsigned ld_relaxed(unsigned* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool spin_geq(unsigned* ctr, unsigned target, unsigned* abort_flag) {
    for (int it = 0; it < SPIN_LIMIT; ++it) {
        if (ld_relaxed(ctr) >= target) return true;
        if (ld_relaxed(abort_flag) != 0u) return false;
        __builtin_amdgcn_s_sleep(2);
    }
    __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return false;
}

// Block-wide wait until *ctr >= target (all threads call it); false on abort.
// Lines of the slot from an earlier generation may still sit in this compute
// unit's L1: after the counter is reached, an agent-scope acquire invalidates
// the L1 (the block's waves share it) before the barrier releases the block.
__device__ __forceinline__ bool block_wait(unsigned* ctr, unsigned target, unsigned* abort_flag, int* sh_ok) {
    if (threadIdx.x == 0) {
        const bool ok = spin_geq(ctr, target, abort_flag);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *sh_ok = ok ? 1 : 0;
    }
    __syncthreads();
    return *sh_ok != 0;
}

// Block-wide publish: every wave's loads and stores complete, then one relaxed increment.
__device__ __forceinline__ void block_signal(unsigned* ctr) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int N, int M, int PC, int PW, int PR>
struct FusedCfg {
    static constexpr int L = M / 2;
    static constexpr int TC = N / PC;
    static constexpr int THREADS = PW * TC;
    static constexpr int TR = L / PR;
    static constexpr int ROWS = THREADS / TR;
    static_assert(ROWS * TR == THREADS && ROWS >= 1, "row tile must use the whole block");
    static constexpr size_t LDS_COL = ((size_t)PW * ColScratch<N, PC>::value + N) * sizeof(float2);
    static constexpr size_t LDS_ROW = (size_t)ROWS * RowPitch<L, PR>::value * sizeof(float2);
    static constexpr size_t LDS = LDS_COL > LDS_ROW ? LDS_COL : LDS_ROW;
};

template <int N, int M, int PC, int PW, int PR, bool REAL, bool FWD>
__global__ __launch_bounds__((FusedCfg<N, M, PC, PW, PR>::THREADS), 4) void k_fused(FusedGeom g, FusedBufs bf) {
    using C = FusedCfg<N, M, PC, PW, PR>;
    constexpr int L = C::L, ROWS = C::ROWS;
    extern __shared__ float2 lds[];
    __shared__ int sh_task, sh_ok, sh_q, sh_nq;
    unsigned* ctr = bf.ctr;
    unsigned* abort_flag = ctr + CTR_ABORT;
    unsigned* heads = ctr + CTR_HEADS;
    unsigned* done = ctr + CTR_DONE;  // slot s: [2s] column side, [2s+1] row side

    // ---------------- census
    if (threadIdx.x == 0) {
        const unsigned x = xcc_id();
        __hip_atomic_fetch_add(ctr + CTR_CENSUS + x, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(ctr + CTR_ARRIVED, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int ok = spin_geq(ctr + CTR_ARRIVED, gridDim.x, abort_flag) ? 1 : 0;
        int rank = 0, nq = 0;
        unsigned mine = 0;
        for (unsigned y = 0; y < (unsigned)kMaxXcc; ++y) {
            const unsigned c = ld_relaxed(ctr + CTR_CENSUS + y);
            if (c != 0u) {
                rank += (y < x) ? 1 : 0;
                ++nq;
            }
            if (y == x) mine = c;
        }
        // the column tasks of a group must leave blocks for its row tasks; the slots exist for Qmax queues
        if (ok && (mine <= (unsigned)(g.GI * g.npan) || nq > g.Qmax)) {
            __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ok = 0;
        }
        sh_ok = ok;
        sh_q = rank;
        sh_nq = nq;
    }
    __syncthreads();
    if (!sh_ok) return;
    const int q = sh_q, Q = sh_nq;
    const int nimg = (q < g.B) ? (g.B - q + Q - 1) / Q : 0;  // images b = q + Q j of this queue
    const int per_img = g.npan + g.K * g.nrb;
    const int total = nimg * per_img;
    const int FG = g.GI * per_img;
    const size_t plane = (size_t)L * N;
    const size_t img = (size_t)N * M;
    float2* qslots = bf.slots + (size_t)q * g.GI * g.S * plane;
    unsigned* qdone = done + 2 * q * g.GI * g.S;

    for (;;) {
        __syncthreads();  // the previous task's LDS and shared reads are finished
        if (threadIdx.x == 0) sh_task = (int)__hip_atomic_fetch_add(&heads[q], 1u, __ATOMIC_RELAXED,
                                                                     __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int task = sh_task;
        if (task >= total) return;
        // an opaque copy of the thread index per task keeps the tiles' address
        // arithmetic inside the task instead of live across the task loop
        int tid = (int)threadIdx.x;
        asm volatile("" : "+v"(tid));
        const int grp = task / FG, rem = task % FG;
        const int gi = min(g.GI, nimg - grp * g.GI);
        if (rem < gi * g.npan) {
            // ---------------- column task: panel p of image i of the group, all K planes
            const int i = rem / g.npan, p = rem % g.npan;
            const int b = q + Q * (grp * g.GI + i);
            if constexpr (FWD) {
                float2 xh[PC];
                col_fwd_setup<N, PC, PW>(bf.A + (size_t)b * plane, p * PW, xh, lds, bf.scale, bf.twN, tid);
                for (int k = 0; k < g.K; ++k) {
                    const int s = k % g.S, sl = i * g.S + s;
                    const unsigned gen = (unsigned)(grp * ((g.K - s + g.S - 1) / g.S) + k / g.S);
                    // the slot's previous plane must have been read by all its row tasks
                    if (gen > 0 && !block_wait(&qdone[2 * sl + 1], gen * (unsigned)g.nrb, abort_flag, &sh_ok)) return;
                    col_fwd_emit<N, PC, PW, REAL, false>(xh, bf.filt, k, L, p * PW, qslots + (size_t)sl * plane, lds,
                                                         bf.twN, tid);
                    block_signal(&qdone[2 * sl]);
                }
            } else {
                float2 acc[PC];
#pragma unroll
                for (int qq = 0; qq < PC; ++qq) acc[qq] = make_float2(0.0f, 0.0f);
                col_inv_begin<N, PC, PW>(p * PW, lds, tid);
                for (int k = 0; k < g.K; ++k) {
                    const int s = k % g.S, sl = i * g.S + s;
                    const unsigned gen = (unsigned)(grp * ((g.K - s + g.S - 1) / g.S) + k / g.S);
                    // all row tasks of the plane must have written the slot
                    if (!block_wait(&qdone[2 * sl + 1], (gen + 1) * (unsigned)g.nrb, abort_flag, &sh_ok)) return;
                    col_inv_accum<N, PC, PW, REAL, false>(qslots + (size_t)sl * plane, bf.filt, k, L, p * PW, acc, lds,
                                                          bf.twN, tid);
                    block_signal(&qdone[2 * sl]);
                }
                col_inv_finish<N, PC, PW>(acc, p * PW, bf.V + (size_t)b * plane, lds, bf.twN, tid);
            }
        } else {
            // ---------------- row task: tile r of plane (i, k)
            const int r2 = rem - gi * g.npan;
            const int k = r2 / (gi * g.nrb);
            const int i = (r2 / g.nrb) % gi;
            const int r = r2 % g.nrb;
            const int b = q + Q * (grp * g.GI + i);
            const int s = k % g.S, sl = i * g.S + s;
            const unsigned gen = (unsigned)(grp * ((g.K - s + g.S - 1) / g.S) + k / g.S);
            if constexpr (FWD) {
                // all column tasks must have written the plane
                if (!block_wait(&qdone[2 * sl], (gen + 1) * (unsigned)g.npan, abort_flag, &sh_ok)) return;
                row_c2r_tile<M, PR, ROWS, false>(qslots + (size_t)sl * plane, bf.cout + ((size_t)b * g.K + k) * img, N,
                                                 r * ROWS, lds, bf.twL, bf.twM, 1.0f, tid);
            } else {
                // the slot's previous plane must have been read by all column tasks
                if (gen > 0 && !block_wait(&qdone[2 * sl], gen * (unsigned)g.npan, abort_flag, &sh_ok)) return;
                row_r2c_tile<M, PR, ROWS, false>(bf.cin + ((size_t)b * g.K + k) * img, qslots + (size_t)sl * plane, N,
                                                 r * ROWS, lds, bf.twL, bf.twM, tid);
            }
            block_signal(&qdone[2 * sl + 1]);
        }
    }
}

// ---------------------------------------------------------------- skewed pipeline kernels
// The batch is cut into chunks of images. Launch i of the forward transform
// runs the column stage of chunk i+1 and the coefficient row stage of chunk i
// as one grid (column blocks first), exchanging planes through two ping-pong
// buffers sized to stay in the on-package cache; kernel boundaries order the
// stages, so no block waits on another. The inverse runs the coefficient row
// stage of chunk i+1 with the column stage of chunk i, whose blocks each sum
// one group of filters into a partial spectrum; one more launch adds the
// partials in a fixed order and applies the column IFFT.

template <int N, int M, int PC, int PW, int PR, bool REAL>
__global__ __launch_bounds__((FusedCfg<N, M, PC, PW, PR>::THREADS)) void k_skew_fwd(SkewArgs a) {
    using C = FusedCfg<N, M, PC, PW, PR>;
    constexpr int L = C::L, ROWS = C::ROWS;
    extern __shared__ float2 lds[];
    const size_t plane = (size_t)L * N;
    const int ncol = a.col_nb * a.npan * a.kg;
    int task = blockIdx.x;
    if (task < ncol) {
        const int g = task % a.kg;
        const int p = (task / a.kg) % a.npan;
        const int i = task / (a.kg * a.npan);
        const int b = a.col_b0 + i;
        float2 xh[PC];
        col_fwd_setup<N, PC, PW>(a.A + (size_t)b * plane, p * PW, xh, lds, a.scale, a.twN, (int)threadIdx.x);
        const int k1 = min(a.K, (g + 1) * a.kper);
        for (int k = g * a.kper; k < k1; ++k)
            col_fwd_emit<N, PC, PW, REAL>(xh, a.filt, k, L, p * PW, a.bufC + ((size_t)i * a.K + k) * plane, lds, a.twN, (int)threadIdx.x);
        return;
    }
    task -= ncol;
    const int r = task % a.nrb;
    const int k = (task / a.nrb) % a.K;
    const int i = task / (a.nrb * a.K);
    const int b = a.row_b0 + i;
    row_c2r_tile<M, PR, ROWS>(a.bufR + ((size_t)i * a.K + k) * plane, a.cout + ((size_t)b * a.K + k) * N * M, N,
                              r * ROWS, lds, a.twL, a.twM, 1.0f, (int)threadIdx.x);
}

template <int N, int M, int PC, int PW, int PR, bool REAL>
__global__ __launch_bounds__((FusedCfg<N, M, PC, PW, PR>::THREADS)) void k_skew_inv(SkewArgs a) {
    using C = FusedCfg<N, M, PC, PW, PR>;
    constexpr int L = C::L, ROWS = C::ROWS, TC = C::TC;
    extern __shared__ float2 lds[];
    const size_t plane = (size_t)L * N;
    const int ncol = a.col_nb * a.npan * a.kg;
    int task = blockIdx.x;
    if (task < ncol) {
        const int g = task % a.kg;
        const int p = (task / a.kg) % a.npan;
        const int i = task / (a.kg * a.npan);
        const int b = a.col_b0 + i;
        float2 acc[PC];
#pragma unroll
        for (int q = 0; q < PC; ++q) acc[q] = make_float2(0.0f, 0.0f);
        col_inv_begin<N, PC, PW>(p * PW, lds, (int)threadIdx.x);
        const int k1 = min(a.K, (g + 1) * a.kper);
        for (int k = g * a.kper; k < k1; ++k)
            col_inv_accum<N, PC, PW, REAL>(a.bufC + ((size_t)i * a.K + k) * plane, a.filt, k, L, p * PW, acc, lds,
                                           a.twN, (int)threadIdx.x);
        // partial spectrum of filter group g (and, for packed column 0, its mirrored-term partial)
        const int t = threadIdx.x % TC, c = threadIdx.x / TC;
        const int col = p * PW + c;
        float2* o = a.part + ((size_t)b * a.kg + g) * plane + (size_t)col * N;
#pragma unroll
        for (int q = 0; q < PC; ++q) o[t + TC * q] = acc[q];
        if (col == 0) {
            // each thread of column 0 reads back the entries of g it accumulated
            const float2* sg = lds + PW * ColScratch<N, PC>::value;
            float2* og = a.part0 + ((size_t)b * a.kg + g) * N;
#pragma unroll
            for (int q = 0; q < PC; ++q) og[t + TC * q] = sg[t + TC * q];
        }
        return;
    }
    task -= ncol;
    const int r = task % a.nrb;
    const int k = (task / a.nrb) % a.K;
    const int i = task / (a.nrb * a.K);
    const int b = a.row_b0 + i;
    row_r2c_tile<M, PR, ROWS>(a.cin + ((size_t)b * a.K + k) * N * M, a.bufR + ((size_t)i * a.K + k) * plane, N,
                              r * ROWS, lds, a.twL, a.twM, (int)threadIdx.x);
}

// V[b] panel p = colIFFT( sum_g partial_g  [+ conj of the mirrored column-0 partials] ), g in order
template <int N, int M, int PC, int PW, int PR>
__global__ __launch_bounds__((FusedCfg<N, M, PC, PW, PR>::THREADS)) void k_skew_finish(SkewArgs a) {
    using C = FusedCfg<N, M, PC, PW, PR>;
    constexpr int L = C::L, TC = C::TC;
    extern __shared__ float2 lds[];
    const size_t plane = (size_t)L * N;
    const int p = blockIdx.x % a.npan, b = blockIdx.x / a.npan;
    const int t = threadIdx.x % TC, c = threadIdx.x / TC;
    const int col = p * PW + c;
    float2 acc[PC], gg[PC];
#pragma unroll
    for (int q = 0; q < PC; ++q) acc[q] = gg[q] = make_float2(0.0f, 0.0f);
    for (int g = 0; g < a.kg; ++g) {
        const float2* src = a.part + ((size_t)b * a.kg + g) * plane + (size_t)col * N;
#pragma unroll
        for (int q = 0; q < PC; ++q) acc[q] = cadd(acc[q], src[t + TC * q]);
        if (col == 0) {
            const float2* sg = a.part0 + ((size_t)b * a.kg + g) * N;
#pragma unroll
            for (int q = 0; q < PC; ++q) gg[q] = cadd(gg[q], sg[t + TC * q]);
        }
    }
    if (col == 0) {
        float2* smir = lds + PW * ColScratch<N, PC>::value;
#pragma unroll
        for (int q = 0; q < PC; ++q) smir[t + TC * q] = gg[q];
    }
    col_inv_finish<N, PC, PW>(acc, p * PW, a.V + (size_t)b * plane, lds, a.twN, (int)threadIdx.x);
}

__global__ void k_zero_u32(unsigned* p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

// ---------------------------------------------------------------- dispatch

template <typename F>
hipError_t set_lds(F* fn, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// rows per block: cap_rows<M, RB>; the block's LDS also holds the FFT's twiddles
template <int M, int TAG, int ROWS>
hipError_t rows_r2c_rt(const DevPlan& d, const float* in, float2* out, int planes, hipStream_t st) {
    constexpr int L = M / 2, P = Pts<L>::value, T = L / P;
    const size_t lds = ((size_t)ROWS * RowPitch<L, P>::value + L) * sizeof(float2);
    hipError_t e = set_lds(k_rows_r2c<M, TAG, ROWS>, lds);
    if (e != hipSuccess) return e;
    const size_t blocks = (size_t)planes * (d.N / ROWS);
    hipLaunchKernelGGL((k_rows_r2c<M, TAG, ROWS>), dim3((unsigned)blocks), dim3(ROWS * T), lds, st, in, out, d.N, d.twL,
                       d.twM);
    return hipGetLastError();
}

template <int M, int TAG>
hipError_t rows_r2c_t(const DevPlan& d, const float* in, float2* out, int planes, hipStream_t st) {
    return rows_r2c_rt<M, TAG, cap_rows<M, RB>()>(d, in, out, planes, st);
}

template <int M, int TAG, int ROWS>
hipError_t rows_c2r_rt(const DevPlan& d, const float2* in, float* out, int planes, float scale, hipStream_t st) {
    constexpr int L = M / 2, P = Pts<L>::value, T = L / P;
    const size_t lds = ((size_t)ROWS * RowPitch<L, P>::value + L) * sizeof(float2);
    hipError_t e = set_lds(k_rows_c2r<M, TAG, ROWS>, lds);
    if (e != hipSuccess) return e;
    const size_t blocks = (size_t)planes * (d.N / ROWS);
    hipLaunchKernelGGL((k_rows_c2r<M, TAG, ROWS>), dim3((unsigned)blocks), dim3(ROWS * T), lds, st, in, out, d.N, d.twL,
                       d.twM, scale);
    return hipGetLastError();
}

template <int M, int TAG>
hipError_t rows_c2r_t(const DevPlan& d, const float2* in, float* out, int planes, float scale, hipStream_t st) {
    return rows_c2r_rt<M, TAG, cap_rows<M, RB>()>(d, in, out, planes, scale, st);
}

template <int M>
hipError_t rows_r2c_mix_t(const DevPlan& d, const float* fm, const float* mask, const float* f, float2* out,
                          int planes, hipStream_t st) {
    constexpr int L = M / 2, P = Pts<L>::value, T = L / P, ROWS = cap_rows<M, RB>();
    const size_t lds = ((size_t)ROWS * RowPitch<L, P>::value + L) * sizeof(float2);  // + the FFT twiddles
    hipError_t e = set_lds(k_rows_r2c_mix<M, ROWS>, lds);
    if (e != hipSuccess) return e;
    const size_t blocks = (size_t)planes * (d.N / ROWS);
    hipLaunchKernelGGL((k_rows_r2c_mix<M, ROWS>), dim3((unsigned)blocks), dim3(ROWS * T), lds, st, fm, mask, f, out,
                       d.N, d.twL, d.twM);
    return hipGetLastError();
}

template <int M, int ROWS>
hipError_t rows_thresh_rt(const DevPlan& d, float2* planes, int nplanes, const float* thr, unsigned* kept,
                          hipStream_t st) {
    constexpr int L = M / 2, P = Pts<L>::value, T = L / P;
    const size_t lds = ((size_t)ROWS * RowPitch<L, P>::value + L) * sizeof(float2);  // + the FFT twiddles
    hipError_t e = set_lds(k_rows_thresh<M, ROWS>, lds);
    if (e != hipSuccess) return e;
    const size_t blocks = (size_t)nplanes * (d.N / ROWS);
    hipLaunchKernelGGL((k_rows_thresh<M, ROWS>), dim3((unsigned)blocks), dim3(ROWS * T), lds, st, planes, d.N, thr, kept,
                       d.twL, d.twM);
    return hipGetLastError();
}

template <int M>
hipError_t rows_thresh_t(const DevPlan& d, float2* planes, int nplanes, const float* thr, unsigned* kept,
                         hipStream_t st) {
    return rows_thresh_rt<M, cap_rows<M, RB>()>(d, planes, nplanes, thr, kept, st);
}

// filters per group for kg requested groups, and the groups that gives
inline void kgroups(int K, int kg_req, int& kper, int& kg) {
    kg_req = std::max(1, std::min(kg_req, K));
    kper = (K + kg_req - 1) / kg_req;
    kg = (K + kper - 1) / kper;
}

template <int N, int PW>
hipError_t cols_fwd_t(const DevPlan& d, const float2* A, float2* T, int nimg, const void* filt, float scale,
                      hipStream_t st) {
    using C = ColCfg<N, PW>;
    const int npan = d.L / PW;
    int kper, kg;
    kgroups(d.K, d.kg_fwd, kper, kg);
    const size_t blocks = (size_t)npan * kg * nimg;
    if (d.real) {
        hipError_t e = set_lds(k_cols_fwd<N, PW, true>, C::LDS);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_cols_fwd<N, PW, true>), dim3((unsigned)blocks), dim3(C::THREADS), C::LDS, st, A, T,
                           filt, d.L, d.K, npan, kper, kg, d.twN, scale);
    } else {
        hipError_t e = set_lds(k_cols_fwd<N, PW, false>, C::LDS);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_cols_fwd<N, PW, false>), dim3((unsigned)blocks), dim3(C::THREADS), C::LDS, st, A, T,
                           filt, d.L, d.K, npan, kper, kg, d.twN, scale);
    }
    return hipGetLastError();
}

template <int N, int PW>
hipError_t cols_inv_t(const DevPlan& d, const float2* U, float2* V, int nimg, const void* filt, float2* part,
                      hipStream_t st) {
    using C = ColCfg<N, PW>;
    const int npan = d.L / PW;
    int kper, kg;
    kgroups(d.K, d.kg_inv, kper, kg);
    if (kg > 1 && part == nullptr) return hipErrorInvalidValue;
    float2* part0 = kg > 1 ? part + (size_t)nimg * kg * d.L * d.N : nullptr;
    const size_t blocks = (size_t)npan * kg * nimg;
    if (d.real) {
        hipError_t e = set_lds(k_cols_inv<N, PW, true>, C::LDS);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_cols_inv<N, PW, true>), dim3((unsigned)blocks), dim3(C::THREADS), C::LDS, st, U, V,
                           filt, d.L, d.K, npan, kper, kg, part, part0, d.twN);
    } else {
        hipError_t e = set_lds(k_cols_inv<N, PW, false>, C::LDS);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_cols_inv<N, PW, false>), dim3((unsigned)blocks), dim3(C::THREADS), C::LDS, st, U, V,
                           filt, d.L, d.K, npan, kper, kg, part, part0, d.twN);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || kg == 1) return e;
    e = set_lds(k_cols_inv_finish<N, PW>, C::LDS);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_cols_inv_finish<N, PW>), dim3((unsigned)((size_t)npan * nimg)), dim3(C::THREADS), C::LDS, st,
                       part, part0, V, d.L, npan, kg, d.twN);
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

hipError_t launch_rows_r2c_mix(const DevPlan& d, const float* fm, const float* mask, const float* f, float2* out,
                               int planes, hipStream_t st) {
    switch (d.M) {
        case 16: return rows_r2c_mix_t<16>(d, fm, mask, f, out, planes, st);
        case 32: return rows_r2c_mix_t<32>(d, fm, mask, f, out, planes, st);
        case 64: return rows_r2c_mix_t<64>(d, fm, mask, f, out, planes, st);
        case 128: return rows_r2c_mix_t<128>(d, fm, mask, f, out, planes, st);
        case 256: return rows_r2c_mix_t<256>(d, fm, mask, f, out, planes, st);
        case 512: return rows_r2c_mix_t<512>(d, fm, mask, f, out, planes, st);
        case 1024: return rows_r2c_mix_t<1024>(d, fm, mask, f, out, planes, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_rows_thresh(const DevPlan& d, float2* planes, int nplanes, const float* thr, unsigned* kept,
                              hipStream_t st) {
    switch (d.M) {
        case 16: return rows_thresh_t<16>(d, planes, nplanes, thr, kept, st);
        case 32: return rows_thresh_t<32>(d, planes, nplanes, thr, kept, st);
        case 64: return rows_thresh_t<64>(d, planes, nplanes, thr, kept, st);
        case 128: return rows_thresh_t<128>(d, planes, nplanes, thr, kept, st);
        case 256: return rows_thresh_t<256>(d, planes, nplanes, thr, kept, st);
        case 512: return rows_thresh_t<512>(d, planes, nplanes, thr, kept, st);
        case 1024: return rows_thresh_t<1024>(d, planes, nplanes, thr, kept, st);
    }
    return hipErrorInvalidValue;
}

// PW8_1024: the block width that serves 8-column panels at N = 1024 (4 for the forward pass:
// two 256-thread blocks per CU instead of one of 512 at the same register-bound occupancy,
// 0.22 -> 0.20 ms in the uneven inpainting; the inverse stays at 8, which measured faster there)
#define SHEAR_COLS_SWITCH(PWSEL, PW8_1024, FN, ...)                                \
    if (d.L >= 16 && (PWSEL) == 16) {                                              \
        switch (d.N) {                                                             \
            case 16: return FN<16, 16>(__VA_ARGS__);                               \
            case 32: return FN<32, 16>(__VA_ARGS__);                               \
            case 64: return FN<64, 16>(__VA_ARGS__);                               \
            case 128: return FN<128, 16>(__VA_ARGS__);                             \
            case 256: return FN<256, 16>(__VA_ARGS__);                             \
            case 512: return FN<512, 16>(__VA_ARGS__);                             \
            case 1024: return FN<1024, 16>(__VA_ARGS__);                           \
        }                                                                          \
    } else if (d.L >= 8) {                                                         \
        switch (d.N) {                                                             \
            case 16: return FN<16, 8>(__VA_ARGS__);                                \
            case 32: return FN<32, 8>(__VA_ARGS__);                                \
            case 64: return FN<64, 8>(__VA_ARGS__);                                \
            case 128: return FN<128, 8>(__VA_ARGS__);                              \
            case 256: return FN<256, 8>(__VA_ARGS__);                              \
            case 512: return FN<512, 8>(__VA_ARGS__);                              \
            case 1024: return FN<1024, PW8_1024>(__VA_ARGS__);                     \
        }                                                                          \
    }                                                                              \
    return hipErrorInvalidValue;

hipError_t launch_cols_fwd(const DevPlan& d, const float2* A, float2* T, int nimg, const void* filt, float scale,
                           hipStream_t st) {
    SHEAR_COLS_SWITCH(d.pw_fwd, 4, cols_fwd_t, d, A, T, nimg, filt, scale, st)
}

hipError_t launch_cols_inv(const DevPlan& d, const float2* U, float2* V, int nimg, const void* filt, float2* part,
                           hipStream_t st) {
    SHEAR_COLS_SWITCH(d.pw_inv, 8, cols_inv_t, d, U, V, nimg, filt, part, st)
}

// ---------------------------------------------------------------- fused dispatch
namespace {

// Tile configuration of the fused kernels: 512 threads per block, and the same
// FFT decompositions as the standalone kernels, so both paths round identically.
template <int N, int M>
struct FusedPick {
    static constexpr int PC = ColPts<N>::value;
    static constexpr int PW = 512 / (N / PC);
    static constexpr int PR = Pts<M / 2>::value;
    using C = FusedCfg<N, M, PC, PW, PR>;
};

template <int N, int M, bool REAL, bool FWD>
const void* fused_fn() {
    using F = FusedPick<N, M>;
    return reinterpret_cast<const void*>(&k_fused<N, M, F::PC, F::PW, F::PR, REAL, FWD>);
}

template <int N, int M>
hipError_t fused_info_t(const DevPlan& d, bool fwd, FusedInfo& fi) {
    using F = FusedPick<N, M>;
    using C = typename F::C;
    fi.threads = C::THREADS;
    fi.lds = C::LDS;
    fi.npan = d.L / F::PW;
    fi.nrb = d.N / C::ROWS;
    fi.fn = d.real ? (fwd ? fused_fn<N, M, true, true>() : fused_fn<N, M, true, false>())
                   : (fwd ? fused_fn<N, M, false, true>() : fused_fn<N, M, false, false>());
    if (C::LDS > 65536) {
        hipError_t e = hipFuncSetAttribute(fi.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)C::LDS);
        if (e != hipSuccess) return e;
    }
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&fi.blocks_per_cu, fi.fn, C::THREADS, C::LDS);
}

template <int N>
hipError_t fused_info_m(const DevPlan& d, bool fwd, FusedInfo& fi) {
    switch (d.M) {
        case 128: return fused_info_t<N, 128>(d, fwd, fi);
        case 256: return fused_info_t<N, 256>(d, fwd, fi);
        case 512: return fused_info_t<N, 512>(d, fwd, fi);
        case 1024: return fused_info_t<N, 1024>(d, fwd, fi);
    }
    return hipErrorInvalidValue;
}

}  // namespace

bool fused_supported(int N, int M) {
    auto ok = [](int n) { return n == 128 || n == 256 || n == 512 || n == 1024; };
    return ok(N) && ok(M);
}

hipError_t fused_info(const DevPlan& d, bool fwd, FusedInfo& fi) {
    switch (d.N) {
        case 128: return fused_info_m<128>(d, fwd, fi);
        case 256: return fused_info_m<256>(d, fwd, fi);
        case 512: return fused_info_m<512>(d, fwd, fi);
        case 1024: return fused_info_m<1024>(d, fwd, fi);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_fused(const FusedInfo& fi, const FusedGeom& g, const FusedBufs& bf, int grid, hipStream_t st) {
    FusedGeom ga = g;
    FusedBufs ba = bf;
    void* args[] = {&ga, &ba};
    return hipLaunchCooperativeKernel(fi.fn, dim3((unsigned)grid), dim3((unsigned)fi.threads), args,
                                      (unsigned)fi.lds, st);
}

namespace {

template <int N, int M>
hipError_t skew_t(const DevPlan& d, int which, const SkewArgs& a, int blocks, hipStream_t st) {
    using F = FusedPick<N, M>;
    using C = typename F::C;
    const void* fn;
    if (which == 0)
        fn = d.real ? reinterpret_cast<const void*>(&k_skew_fwd<N, M, F::PC, F::PW, F::PR, true>)
                    : reinterpret_cast<const void*>(&k_skew_fwd<N, M, F::PC, F::PW, F::PR, false>);
    else if (which == 1)
        fn = d.real ? reinterpret_cast<const void*>(&k_skew_inv<N, M, F::PC, F::PW, F::PR, true>)
                    : reinterpret_cast<const void*>(&k_skew_inv<N, M, F::PC, F::PW, F::PR, false>);
    else
        fn = reinterpret_cast<const void*>(&k_skew_finish<N, M, F::PC, F::PW, F::PR>);
    if (C::LDS > 65536) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)C::LDS);
        if (e != hipSuccess) return e;
    }
    SkewArgs aa = a;
    void* args[] = {&aa};
    return hipLaunchKernel(fn, dim3((unsigned)blocks), dim3((unsigned)C::THREADS), args, C::LDS, st);
}

template <int N>
hipError_t skew_m(const DevPlan& d, int which, const SkewArgs& a, int blocks, hipStream_t st) {
    switch (d.M) {
        case 128: return skew_t<N, 128>(d, which, a, blocks, st);
        case 256: return skew_t<N, 256>(d, which, a, blocks, st);
        case 512: return skew_t<N, 512>(d, which, a, blocks, st);
        case 1024: return skew_t<N, 1024>(d, which, a, blocks, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace

namespace {
template <int N, int M>
SkewTiles tiles_t(const DevPlan& d) {
    using F = FusedPick<N, M>;
    SkewTiles t;
    t.ok = true;
    t.npan = d.L / F::PW;
    t.nrb = d.N / F::C::ROWS;
    return t;
}
template <int N>
SkewTiles tiles_m(const DevPlan& d) {
    switch (d.M) {
        case 128: return tiles_t<N, 128>(d);
        case 256: return tiles_t<N, 256>(d);
        case 512: return tiles_t<N, 512>(d);
        case 1024: return tiles_t<N, 1024>(d);
    }
    return SkewTiles{};
}
}  // namespace

SkewTiles skew_tiles(const DevPlan& d) {
    switch (d.N) {
        case 128: return tiles_m<128>(d);
        case 256: return tiles_m<256>(d);
        case 512: return tiles_m<512>(d);
        case 1024: return tiles_m<1024>(d);
    }
    return SkewTiles{};
}

hipError_t launch_skew(const DevPlan& d, int which, const SkewArgs& a, int blocks, hipStream_t st) {
    if (blocks <= 0) return hipSuccess;
    switch (d.N) {
        case 128: return skew_m<128>(d, which, a, blocks, st);
        case 256: return skew_m<256>(d, which, a, blocks, st);
        case 512: return skew_m<512>(d, which, a, blocks, st);
        case 1024: return skew_m<1024>(d, which, a, blocks, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_zero_u32(unsigned* p, int n, hipStream_t st) {
    const int threads = 256;
    const int blocks = std::max(1, std::min(1024, (n + threads - 1) / threads));
    hipLaunchKernelGGL(k_zero_u32, dim3(blocks), dim3(threads), 0, st, p, n);
    return hipGetLastError();
}

}  // namespace shear
