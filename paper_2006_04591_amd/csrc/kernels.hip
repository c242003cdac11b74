// gfx950 kernels of the FFT-domain shearlet filter bank.
//
// Data flow (Algorithm 1 / Algorithm 2 of Section 3.4.2 with the Fourier
// shifts folded into the stored filter order):
//   forward  x --rows r2c--> A --columns: FFT, x conj filter_k, IFFT--> T_k --rows c2r--> c_k
//   inverse  c_k --rows r2c--> U_k --columns: FFT, x dual filter_k, sum_k, IFFT--> V --rows c2r--> y
// A real row of M samples is transformed as M/2 complex samples plus a
// post-twiddle; the real DC and Nyquist bins of each row spectrum share one
// complex slot ("packed" column 0), so every intermediate plane is N x M/2
// complex, stored in panels of 8 columns made of 16-row tiles (xoff in fft_core.h).
#include "kernels.h"
#include "fft_core.h"

#include <algorithm>
#include <mutex>

namespace shear {
namespace {

using namespace dev;

// points per thread for an FFT of length L (standalone kernels)
template <int L>
struct Pts {
    static constexpr int value = (L >= 1024) ? 16 : (L == 256 ? 16 : 8);
};

// points per thread of the column FFTs (N-point): 8 up to N = 512 (256-point columns use two
// 32-thread groups per wavefront), 16 at N = 1024 and 2048 (a 2048-point group is 128 threads, two
// wavefronts that synchronise with workgroup barriers)
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

template <int N, int PW, int PP = ColPts<N>::value>
struct ColCfg {
    static constexpr int P = PP;
    static constexpr int T = N / P;
    static constexpr int THREADS = PW * T;
    static constexpr size_t LDS = ((size_t)PW * ColScratch<N, P>::value + N) * sizeof(float2);
};

// Filter groups: the K filters of a column panel may be split over kg blocks of kper
// consecutive filters (block index = pan + npan (g + kg b)), so that small batches still
// fill the device. The forward recomputes the panel's column FFT in each group; the
// inverse writes one partial sum per group and k_cols_inv_finish adds them in group order.
template <int N, int PW, bool REAL, int PP>
__global__ __launch_bounds__((ColCfg<N, PW, PP>::THREADS)) void k_cols_fwd(const float2* __restrict__ A,
                                                                    float2* __restrict__ Tout,
                                                                    const void* __restrict__ filt, int L, int K,
                                                                    int npan, int kper, int kg,
                                                                    const float2* __restrict__ twN, float scale) {
    constexpr int P = ColCfg<N, PW, PP>::P;
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
template <int N, int PW, bool REAL, int PP>
__global__ __launch_bounds__((ColCfg<N, PW, PP>::THREADS)) void k_cols_inv(const float2* __restrict__ U,
                                                                    float2* __restrict__ V,
                                                                    const void* __restrict__ filt, int L, int K,
                                                                    int npan, int kper, int kg,
                                                                    float2* __restrict__ part,
                                                                    float2* __restrict__ part0,
                                                                    const float2* __restrict__ twN) {
    constexpr int P = ColCfg<N, PW, PP>::P, T = N / P;
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
template <int N, int PW, int PP>
__global__ __launch_bounds__((ColCfg<N, PW, PP>::THREADS)) void k_cols_inv_finish(const float2* __restrict__ part,
                                                                           const float2* __restrict__ part0,
                                                                           float2* __restrict__ V, int L, int npan,
                                                                           int kg, const float2* __restrict__ twN) {
    constexpr int P = ColCfg<N, PW, PP>::P, T = N / P;
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

__global__ void k_zero_u32(unsigned* p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

// ---------------------------------------------------------------- whole-plane forward
// One workgroup per (image, filter) plane: the column IFFT of filter_k (.) X and the row c2r of
// the result both stay on chip, so the forward writes only the coefficients (no exchange planes).
// The N-point column IFFT runs as N = NA x NB (four steps): with xi = NB a + b and
// n = c + NA d, first an NA-point IDFT over a for each (column, b), then the twiddle
// e^{+2 pi i b c / N}, then an NB-point IDFT over b for each (column, c), which gives rows
// n = c + NA d, d < NB. After the first step the rows of each residue c depend only on that
// residue's values, so the plane is finished CR residues (CR NB rows) at a time in LDS while the
// first step's other residues wait in registers.
// The image spectra and the filters are read in a residue-major layout, element (b, a, j) of a
// plane at (b NA + a) L + j (b = xi mod NB, a = xi / NB, j the packed column), so that a
// wavefront of the first step (one b, 64 consecutive columns) loads whole 512-byte runs and its
// twiddles are wave-uniform.
template <int N, int M>
struct PlaneCfg {
    static constexpr int L = M / 2;
    static constexpr int NA = 16, NB = N / NA;
    static constexpr int CR = 8;                   // residues per round
    static constexpr int ROUNDS = NA / CR;
    static constexpr int ROWS = CR * NB;           // plane rows in LDS per round
    static constexpr int THREADS = ROWS / 2 * 16;  // rows: 16 threads per pair of rows
    static constexpr int PITCH = L + L / 16 + 1;   // a pair of rows holds an M-point FFT scratch (M + M/16)
    static constexpr int HALVES = L / 64;          // first step: 64 columns per wavefront, HALVES passes
    // + the row FFT's twiddles, packed column 0 of X and its mirrored-term filter
    static constexpr size_t LDS = ((size_t)ROWS * PITCH + M + N) * sizeof(float2) + N * sizeof(float);
    static_assert(NB == 16 && ROUNDS == 2, "four-step split");
    static_assert(THREADS == 64 * NB && CR * L == THREADS, "thread roles");
    static_assert(2 * PITCH >= M + M / 16, "row-pair FFT scratch");
};

// Xr[b] = scale * colFFT(A[b]) in the residue-major layout (N x L float2 per image); the panel's
// spectra pass through LDS so that each run of 16 columns is written whole.
template <int N, int PW, int PP>
__global__ __launch_bounds__((ColCfg<N, PW, PP>::THREADS)) void k_cols_spec(const float2* __restrict__ A,
                                                                      float2* __restrict__ Xr, int L, int npan,
                                                                      const float2* __restrict__ twN, float scale) {
    constexpr int P = ColCfg<N, PW, PP>::P, T = N / P, THR = ColCfg<N, PW, PP>::THREADS;
    constexpr int NA = 16, NB = N / NA, SP = PW + 1;
    static_assert((size_t)N * SP * sizeof(float2) <= ColCfg<N, PW, PP>::LDS, "staging fits the FFT scratch");
    extern __shared__ float2 lds[];
    const int pan = blockIdx.x % npan, b = blockIdx.x / npan;
    const int tid = (int)threadIdx.x;
    float2 xh[P];
    col_fwd_setup<N, P, PW>(A + (size_t)b * L * N, pan * PW, xh, lds, scale, twN, tid);
    const int t = tid % T, c = tid / T;
#pragma unroll
    for (int q = 0; q < P; ++q) lds[(t + T * q) * SP + c] = xh[q];
    __syncthreads();
    float2* o = Xr + (size_t)b * L * N + pan * PW;
#pragma unroll
    for (int i = 0; i < N * PW / THR; ++i) {
        const int e = tid + THR * i;
        const int cc = e % PW, ra = e / PW;  // ra = bb NA + a
        const int xi = NB * (ra % NA) + ra / NA;
        o[(size_t)ra * L + cc] = lds[xi * SP + cc];
    }
}

// Filters of one forward set in the residue-major layout: per filter N x L floats, then the N
// floats of packed column 0's mirrored-term filter (residue-major as well).
template <int N>
__global__ void k_plane_filters(const float* __restrict__ f, float* __restrict__ fr, int L, int K) {
    constexpr int NA = 16, NB = N / NA;
    const size_t per = (size_t)(L + 1) * N;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < per * K; i += (size_t)gridDim.x * blockDim.x) {
        const size_t k = i / per, r = i % per;
        int ra, j;
        if (r < (size_t)N * L) {
            ra = (int)(r / L);
            j = (int)(r % L);
        } else {
            ra = (int)(r - (size_t)N * L);
            j = L;
        }
        const int xi = NB * (ra % NA) + ra / NA;
        fr[i] = f[k * per + (size_t)j * N + xi];
    }
}

// out[b][k] (N x M real) = row c2r of colIFFT(filter_k (.) X[b]) for the gridDim.x = nimg K planes
// b K + k, from the residue-major spectra Xr and filters fr (real filter sets).
template <int N, int M>
__global__ __launch_bounds__((PlaneCfg<N, M>::THREADS)) void k_plane_fwd(const float2* __restrict__ Xr,
                                                                        const float* __restrict__ fr,
                                                                        float* __restrict__ out, int K,
                                                                        const float2* __restrict__ twN,
                                                                        const float2* __restrict__ twM) {
    using C = PlaneCfg<N, M>;
    constexpr int L = C::L, NA = C::NA, NB = C::NB, CR = C::CR, PITCH = C::PITCH;
    extern __shared__ float2 lds[];
    const int tid = (int)threadIdx.x;
    // Plane order: each XCD takes a contiguous run of the sequence, and the sequence walks the
    // images in groups of G, filter-major within a group, so that the blocks in flight on an XCD
    // share a few images' spectra and a few filters in its L2 (rather than one image and as many
    // filters as blocks).
    int plane;
    {
        constexpr int G = 4;
        int i = (int)blockIdx.x;
        const int per = (int)gridDim.x / 8;
        if (i < per * 8) i = (i % 8) * per + i / 8;
        const int nimg = (int)gridDim.x / K, g0 = i / (G * K) * G, gn = min(G, nimg - g0);
        const int r = i - g0 * K;
        plane = (g0 + r % gn) * K + r / gn;
    }
    const int b = plane / K, k = plane % K;
    const float2* xs = Xr + (size_t)b * L * N;
    const float* fa = fr + (size_t)k * (L + 1) * N;
    float2* stw = lds + C::ROWS * PITCH;  // the row FFT's twiddles exp(-2 pi i m / M), m < M
    float2* sx0 = stw + M;                // packed column 0 of X (N, residue-major)
    float* sbe = reinterpret_cast<float*>(sx0 + N);  // its mirrored-term filter (N, residue-major)
    // First step: wavefront bb (xi = NB a + bb), columns lane + 64 h; residues c < CR go to LDS row
    // c NB + bb, the rest wait in registers. The first half's inputs and the tables are loaded
    // before the block's first barrier, the other halves' right after it; packed column 0's
    // mirrored term beta(xi) conj X(-xi) takes X(-xi) from the wavefront that loaded it, through LDS.
    const int bb = __builtin_amdgcn_readfirstlane(tid / 64), lane = tid % 64;
    const float2* xb = xs + (size_t)bb * NA * L;
    const float* fb = fa + (size_t)bb * NA * L;
    float2 xv[C::HALVES][NA];
    float fv[C::HALVES][NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) {
        xv[0][a] = xb[(unsigned)(a * L + lane)];
        fv[0][a] = fb[(unsigned)(a * L + lane)];
    }
    float2 tm = make_float2(0.0f, 0.0f);
    float be = 0.0f;
    if (tid < M) tm = twM[tid];
    if (tid < N) be = fa[(size_t)N * L + tid];
    if (lane == 0) {
#pragma unroll
        for (int a = 0; a < NA; ++a) sx0[bb * NA + a] = xv[0][a];
    }
    if (tid < M) stw[tid] = tm;
    if (tid < N) sbe[tid] = be;
    __syncthreads();
#pragma unroll
    for (int h = 1; h < C::HALVES; ++h)
#pragma unroll
        for (int a = 0; a < NA; ++a) {
            const unsigned o = (unsigned)(a * L + lane + 64 * h);
            xv[h][a] = xb[o];
            fv[h][a] = fb[o];
        }
    float2 keep[C::HALVES][NA - CR];
#pragma unroll
    for (int h = 0; h < C::HALVES; ++h) {
        const int j = lane + 64 * h;
        float2 y[NA];
#pragma unroll
        for (int a = 0; a < NA; ++a) y[a] = cscale(xv[h][a], fv[h][a]);
        if (j == 0) {
#pragma unroll
            for (int a = 0; a < NA; ++a) {
                const int xm = (N - (NB * a + bb)) & (N - 1);
                y[a] = cadd(y[a], cscale(cconj(sx0[(xm % NB) * NA + xm / NB]), sbe[bb * NA + a]));
            }
        }
        dft16<true>(y);
#pragma unroll
        for (int c = 1; c < NA; ++c) y[c] = cmul(y[c], cconj(twN[bb * c]));
#pragma unroll
        for (int c = 0; c < CR; ++c) lds[(c * NB + bb) * PITCH + j] = y[c];
#pragma unroll
        for (int c = CR; c < NA; ++c) keep[h][c - CR] = y[c];
    }
    __syncthreads();
    // The rounds stay a loop: unrolled, the compiler keeps the LDS addresses of both rounds live
    // at once and spills.
#pragma unroll 1
    for (int R = 0; R < C::ROUNDS; ++R) {
        float2* ld = lds;
        if (R > 0) {
#pragma unroll
            for (int h = 0; h < C::HALVES; ++h)
#pragma unroll
                for (int c = 0; c < CR; ++c) ld[(c * NB + bb) * PITCH + lane + 64 * h] = keep[h][c];
            __syncthreads();
        }
        {
            // last step: thread (column j, residue cl + CR R) over its NB rows, in place
            const int j = tid % L, cl = tid / L;
            float2 z[NB];
#pragma unroll
            for (int x = 0; x < NB; ++x) z[x] = ld[(cl * NB + x) * PITCH + j];
            dft16<true>(z);
#pragma unroll
            for (int d = 0; d < NB; ++d) ld[(cl * NB + d) * PITCH + j] = z[d];
        }
        __syncthreads();
        {
            // Row c2r, two rows per FFT: with X1, X2 the Hermitian spectra of LDS rows 2p and 2p + 1
            // (plane rows cl + CR R + NA d, LDS row cl NB + d), the M-point IDFT of X1 + i X2 has
            // row 1 as its real part and row 2 as its imaginary part. 16 threads per pair, one
            // wavefront; the pair's two LDS rows are its FFT scratch.
            const int p2 = tid / 16, t16 = tid % 16;
            float2* s = ld + 2 * p2 * PITCH;
            const float2* s1 = s;
            const float2* s2 = s + PITCH;
            const float2* stw_r = ld + (stw - lds);
            float2 v[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int kk = t16 + 16 * q;
                if (q < 8) {  // kk < L: X1 + i X2; kk == 0: the real DC bins
                    float2 a1 = s1[kk], a2 = s2[kk];
                    if (kk == 0) {
                        a1 = make_float2(a1.x, 0.0f);
                        a2 = make_float2(a2.x, 0.0f);
                    }
                    v[q] = make_float2(a1.x - a2.y, a1.y + a2.x);
                } else {  // kk >= L: conj X1(M - kk) + i conj X2(M - kk); kk == L: the real Nyquist bins
                    const int m = (M - kk) & (L - 1);
                    float2 a1 = s1[m], a2 = s2[m];
                    if (m == 0) {
                        a1 = make_float2(a1.y, 0.0f);
                        a2 = make_float2(a2.y, 0.0f);
                    }
                    v[q] = make_float2(a1.x + a2.y, a2.x - a1.y);
                }
            }
            wave_sync();
            fft<M, 16, true>(v, s, t16, stw_r);
            const int ra = 2 * p2, rb = 2 * p2 + 1;
            float* d1 = out + ((size_t)plane * N + (ra / NB) + CR * R + NA * (ra % NB)) * M;
            float* d2 = out + ((size_t)plane * N + (rb / NB) + CR * R + NA * (rb % NB)) * M;
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                __builtin_nontemporal_store(v[q].x, d1 + t16 + 16 * q);
                __builtin_nontemporal_store(v[q].y, d2 + t16 + 16 * q);
            }
        }
        if (R + 1 < C::ROUNDS) __syncthreads();
    }
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

template <int N, int PW, int PP>
hipError_t cols_fwd_t(const DevPlan& d, const float2* A, float2* T, int nimg, const void* filt, float scale,
                      hipStream_t st) {
    using C = ColCfg<N, PW, PP>;
    const int npan = d.L / PW;
    int kper, kg;
    kgroups(d.K, d.kg_fwd, kper, kg);
    const size_t blocks = (size_t)npan * kg * nimg;
    if (d.real) {
        hipError_t e = set_lds(k_cols_fwd<N, PW, true, PP>, C::LDS);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_cols_fwd<N, PW, true, PP>), dim3((unsigned)blocks), dim3(C::THREADS), C::LDS, st, A, T,
                           filt, d.L, d.K, npan, kper, kg, d.twN, scale);
    } else {
        hipError_t e = set_lds(k_cols_fwd<N, PW, false, PP>, C::LDS);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_cols_fwd<N, PW, false, PP>), dim3((unsigned)blocks), dim3(C::THREADS), C::LDS, st, A, T,
                           filt, d.L, d.K, npan, kper, kg, d.twN, scale);
    }
    return hipGetLastError();
}

template <int N, int PW, int PP>
hipError_t cols_inv_t(const DevPlan& d, const float2* U, float2* V, int nimg, const void* filt, float2* part,
                      hipStream_t st) {
    using C = ColCfg<N, PW, PP>;
    const int npan = d.L / PW;
    int kper, kg;
    kgroups(d.K, d.kg_inv, kper, kg);
    if (kg > 1 && part == nullptr) return hipErrorInvalidValue;
    float2* part0 = kg > 1 ? part + (size_t)nimg * kg * d.L * d.N : nullptr;
    const size_t blocks = (size_t)npan * kg * nimg;
    if (d.real) {
        hipError_t e = set_lds(k_cols_inv<N, PW, true, PP>, C::LDS);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_cols_inv<N, PW, true, PP>), dim3((unsigned)blocks), dim3(C::THREADS), C::LDS, st, U, V,
                           filt, d.L, d.K, npan, kper, kg, part, part0, d.twN);
    } else {
        hipError_t e = set_lds(k_cols_inv<N, PW, false, PP>, C::LDS);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_cols_inv<N, PW, false, PP>), dim3((unsigned)blocks), dim3(C::THREADS), C::LDS, st, U, V,
                           filt, d.L, d.K, npan, kper, kg, part, part0, d.twN);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || kg == 1) return e;
    e = set_lds(k_cols_inv_finish<N, PW, PP>, C::LDS);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_cols_inv_finish<N, PW, PP>), dim3((unsigned)((size_t)npan * nimg)), dim3(C::THREADS), C::LDS, st,
                       part, part0, V, d.L, npan, kg, d.twN);
    return hipGetLastError();
}

// The alternative points per thread of an N-point column FFT (a different radix sequence), 0 where
// there is none: 16 at 256 and 512 points (two passes of 16 instead of 8 x 8 x 8 or 8 x 8 x 4),
// 8 at 1024 (8 x 8 x 8 x 2, a 128-thread group over two wavefronts with workgroup barriers).
template <int N>
constexpr int alt_col_pts() {
    return (N == 256 || N == 512) ? 16 : (N == 1024 ? 8 : 0);
}

// The column pass at the plan's points per thread: pc == the alternative (when the block stays
// within 1024 threads) or the default ColPts<N>.
template <int N, int PW>
hipError_t cols_fwd_pc(const DevPlan& d, const float2* A, float2* T, int nimg, const void* filt, float scale,
                       hipStream_t st) {
    constexpr int ALT = alt_col_pts<N>();
    if constexpr (ALT > 0 && PW * (N / ALT) <= 1024) {
        if (d.pc_fwd == ALT) return cols_fwd_t<N, PW, ALT>(d, A, T, nimg, filt, scale, st);
    }
    return cols_fwd_t<N, PW, ColPts<N>::value>(d, A, T, nimg, filt, scale, st);
}

template <int N, int PW>
hipError_t cols_inv_pc(const DevPlan& d, const float2* U, float2* V, int nimg, const void* filt, float2* part,
                       hipStream_t st) {
    constexpr int ALT = alt_col_pts<N>();
    if constexpr (ALT > 0 && PW * (N / ALT) <= 1024) {
        if (d.pc_inv == ALT) return cols_inv_t<N, PW, ALT>(d, U, V, nimg, filt, part, st);
    }
    return cols_inv_t<N, PW, ColPts<N>::value>(d, U, V, nimg, filt, part, st);
}

// whole-plane forward: column spectra of the images (residue-major), then one workgroup per plane
template <int N>
hipError_t cols_spec_t(const DevPlan& d, const float2* A, float2* Xr, int nimg, float scale, hipStream_t st) {
    constexpr int PW = 16, PP = ColPts<N>::value;
    using S = ColCfg<N, PW, PP>;
    const int npan = d.L / PW;
    hipError_t e = set_lds(k_cols_spec<N, PW, PP>, S::LDS);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_cols_spec<N, PW, PP>), dim3((unsigned)((size_t)npan * nimg)), dim3(S::THREADS), S::LDS, st, A,
                       Xr, d.L, npan, d.twN, scale);
    return hipGetLastError();
}

template <int N, int M>
hipError_t plane_fwd_t(const DevPlan& d, const float2* Xr, float* out, int nimg, const float* fr, hipStream_t st) {
    using C = PlaneCfg<N, M>;
    hipError_t e = set_lds(k_plane_fwd<N, M>, C::LDS);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_plane_fwd<N, M>), dim3((unsigned)((size_t)nimg * d.K)), dim3(C::THREADS), C::LDS, st, Xr, fr,
                       out, d.K, d.twN, d.twM);
    return hipGetLastError();
}

}  // namespace

int col_points_alternative(int N) {
    switch (N) {
        case 256: return alt_col_pts<256>();
        case 512: return alt_col_pts<512>();
        case 1024: return alt_col_pts<1024>();
    }
    return 0;
}

int col_points_default(int N) {
    switch (N) {
        case 16: return ColPts<16>::value;
        case 32: return ColPts<32>::value;
        case 64: return ColPts<64>::value;
        case 128: return ColPts<128>::value;
        case 256: return ColPts<256>::value;
        case 512: return ColPts<512>::value;
        case 1024: return ColPts<1024>::value;
        case 2048: return ColPts<2048>::value;
    }
    return 0;
}

bool size_supported(int n) {
    return n == 16 || n == 32 || n == 64 || n == 128 || n == 256 || n == 512 || n == 1024 || n == 2048;
}

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
        case 2048: return rows_r2c_t<2048, TAG>(d, in, out, planes, st);
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
        case 2048: return rows_c2r_t<2048, TAG>(d, in, out, planes, scale, st);
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
        case 2048: return rows_r2c_mix_t<2048>(d, fm, mask, f, out, planes, st);
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
        case 2048: return rows_thresh_t<2048>(d, planes, nplanes, thr, kept, st);
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
            case 2048: return FN<2048, 4>(__VA_ARGS__);                            \
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
            case 2048: return FN<2048, 4>(__VA_ARGS__);                            \
        }                                                                          \
    }                                                                              \
    return hipErrorInvalidValue;

hipError_t launch_cols_fwd(const DevPlan& d, const float2* A, float2* T, int nimg, const void* filt, float scale,
                           hipStream_t st) {
    SHEAR_COLS_SWITCH(d.pw_fwd, 4, cols_fwd_pc, d, A, T, nimg, filt, scale, st)
}

hipError_t launch_cols_inv(const DevPlan& d, const float2* U, float2* V, int nimg, const void* filt, float2* part,
                           hipStream_t st) {
    SHEAR_COLS_SWITCH(d.pw_inv, 8, cols_inv_pc, d, U, V, nimg, filt, part, st)
}

bool plane_fwd_supported(const DevPlan& d) { return d.real && d.N == 256 && d.M == 256; }

hipError_t launch_plane_filters(const DevPlan& d, const float* filt, float* fr, hipStream_t st) {
    if (!plane_fwd_supported(d)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_plane_filters<256>, dim3(1024), dim3(256), 0, st, filt, fr, d.L, d.K);
    return hipGetLastError();
}

hipError_t launch_cols_spec(const DevPlan& d, const float2* A, float2* Xr, int nimg, float scale, hipStream_t st) {
    if (!plane_fwd_supported(d)) return hipErrorInvalidValue;
    return cols_spec_t<256>(d, A, Xr, nimg, scale, st);
}

hipError_t launch_plane_fwd(const DevPlan& d, const float2* Xr, float* out, int nimg, const float* fr,
                            hipStream_t st) {
    if (!plane_fwd_supported(d)) return hipErrorInvalidValue;
    return plane_fwd_t<256, 256>(d, Xr, out, nimg, fr, st);
}

hipError_t launch_zero_u32(unsigned* p, int n, hipStream_t st) {
    const int threads = 256;
    const int blocks = std::max(1, std::min(1024, (n + threads - 1) / threads));
    hipLaunchKernelGGL(k_zero_u32, dim3(blocks), dim3(threads), 0, st, p, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------- fixed scratch (allocation-free forward)
// A file-scope device array, one copy per GPU the library runs on, held until the process ends. Host
// code never passes the array's name to a kernel: it is a host-side stand-in, not a device address.
// The device address comes from hipGetSymbolAddress, taken once per device with that device current.
namespace {
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch(void** ptr) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace shear
