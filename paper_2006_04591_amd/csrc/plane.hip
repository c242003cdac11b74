// gfx950 kernels of the on-chip ("plane") path of the forward transform.
//
// The separate-launch path (kernels.hip) passes every (image, filter) plane
// between its column and row stages through an intermediate plane in HBM: the
// 2-D inverse FFT of Algorithm 1 needs one transposition per plane. Here one
// workgroup computes a whole block of coefficient rows of one plane on chip,
// so only the coefficients themselves are written:
//   x --rows r2c--> A --column FFT--> Xh (image spectra, once per image)
//   task (b, k, r): Z = fold_r( Xh[b] (.) conj filter_k )       [registers]
//                   column IFFT of length N/D (each packed column) [registers, LDS scratch]
//                   rows through LDS, row c2r (length M)          [LDS]
//                   -> coefficient rows n1 = D m + r of c[b][k]
// D = 1 when an N x M/2 packed plane fits one workgroup (N x M/2 <= 32768
// complex values, 256 KB), else the column IFFT is decimated in frequency:
// with xi = u + (N/D) v and n1 = D m + r,
//   x[D m + r] = sum_u w_{N/D}^{+u m} [ w_N^{+u r} sum_v w_D^{+v r} Y[u + (N/D) v] ],
// so residue r of the output rows needs the D-fold sum (the "fold") of the
// filtered spectrum followed by an N/D-point IFFT. Each of the D tasks of a
// plane reads the whole image spectrum and filter (from L2) and writes only its
// own rows.
#include "fft_core.h"
#include "kernels.h"

namespace shear {
namespace {

using namespace dev;

// ---------------------------------------------------------------- image spectra

// Xh[b][col][row] = scale * colFFT(A[b]) for the packed columns col < L of each image (A in the
// panel layout of the row passes; Xh column-major, one contiguous run of N values per column).
template <int N, int P, int PW>
__global__ __launch_bounds__(PW*(N / P)) void k_image_spectra(const float2* __restrict__ A, float2* __restrict__ Xh,
                                                               int L, float scale, const float2* __restrict__ twN) {
    constexpr int T = N / P;
    extern __shared__ float2 lds[];
    const int npan = L / PW;
    const int pan = (int)blockIdx.x % npan, b = (int)blockIdx.x / npan;
    const int t = (int)threadIdx.x % T, c = (int)threadIdx.x / T;
    const int col = pan * PW + c;
    const float2* a = A + (size_t)b * L * N;
    float2 v[P];
#pragma unroll
    for (int q = 0; q < P; ++q) v[q] = cscale(a[xoff(t + T * q, col, N)], scale);
    fft<N, P, false>(v, lds + c * (N + N / P), t, twN);
    float2* o = Xh + ((size_t)b * L + col) * N;
#pragma unroll
    for (int q = 0; q < P; ++q) o[t + T * q] = v[q];
}

// ---------------------------------------------------------------- plane forward

// Geometry of one plane task: NR = N/D rows of L = M/2 packed columns.
//   phase 1: each packed column's NR-point IFFT by TC = NR/PC threads (PC points each), CPR
//            columns at a time, NCR rounds; results stay in registers (NCR * PC per thread);
//   phase 2: the rows go through LDS in H blocks of RPH rows (row pitch PITCH: the row FFT's
//            scratch footprint L + L/16 plus one slot against bank conflicts);
//   phase 3: each row's c2r by TR = L/PR threads, in place in its LDS row.
template <int N, int M, int D>
struct PlaneFwdCfg {
    static constexpr int L = M / 2, NR = N / D;
    static constexpr int PR = (L == 256) ? 8 : 16;  // row FFT points per thread
    static constexpr int PITCH0 = L + L / PR + 1;
    static constexpr int PC = (NR == 128 && L == 256) ? 8 : 16, TC = NR / PC;
    static constexpr int THREADS = (TC * L < 1024) ? TC * L : 1024;
    static constexpr int CPR = THREADS / TC, NCR = L / CPR;
    static constexpr int TR = L / PR, RPR = THREADS / TR;
    static constexpr int H = (NR * PITCH0 * 8 > 150 * 1024) ? 2 : 1, RPH = NR / H;
    static constexpr int PITCH = PITCH0;
    static constexpr int COLSCR = NR + NR / PC;
    static constexpr size_t LDS =
        (size_t)((CPR * COLSCR > RPH * PITCH) ? CPR * COLSCR : RPH * PITCH) * sizeof(float2);
    static_assert(NR == 128 || NR == 256, "column IFFT length");
    static_assert(L >= 64 && L <= 256, "row length");
    static_assert(NCR * CPR == L && RPH % RPR == 0 && TR <= 64 && TC <= 64, "plane task shape");
    static_assert(LDS <= 160 * 1024, "LDS of one plane task");
};

// Task of a block: images go to XCDs (hardware blocks i, i + 8, ... share one) so that the tasks
// of one image, which all read its spectrum, run through one L2; the D residues of a filter are
// consecutive, so a filter is fetched into that L2 once. Blocks past the work return.
__device__ __forceinline__ bool plane_task(int B, int K, int D, bool by_xcd, int& b, int& k, int& r) {
    int i = (int)blockIdx.x;
    if (by_xcd) {
        const int x = i % 8, j = i / 8, per = K * D;
        b = x + 8 * (j / per);
        i = j % per;
    } else {
        b = i / (K * D);
        i = i % (K * D);
    }
    k = i / D;
    r = i % D;
    return b < B;
}

template <int N, int M, int D, bool REAL>
__global__ __launch_bounds__((PlaneFwdCfg<N, M, D>::THREADS)) void k_plane_fwd(
    const float2* __restrict__ Xh, const void* __restrict__ filt, float* __restrict__ out, int B, int K, int by_xcd,
    const float2* __restrict__ twN, const float2* __restrict__ twL, const float2* __restrict__ twM) {
    using C = PlaneFwdCfg<N, M, D>;
    constexpr int L = C::L, NR = C::NR, PC = C::PC, TC = C::TC, PR = C::PR, TR = C::TR;
    constexpr int FG = 16 / D;  // fold points per load group
    extern __shared__ float2 lds[];
    int b, k, r;
    if (!plane_task(B, K, D, by_xcd != 0, b, k, r)) return;
    const int tid = (int)threadIdx.x;
    const float2* xb = Xh + (size_t)b * L * N;
    const size_t fbase = (size_t)k * (L + 1) * N;  // filter k: [col 0..L][row 0..N-1]

    // phase 1: filtered, folded spectrum and column IFFTs; wf[v] = w_D^{+v r} (block-uniform).
    // Offsets into the image spectrum and the filter are 32-bit, from block-uniform bases.
    float2 wf[D];
#pragma unroll
    for (int v = 0; v < D; ++v) wf[v] = cconj(twN[(v * r * (N / D)) & (N - 1)]);
    const char* fk = reinterpret_cast<const char*>(filt) + fbase * (REAL ? sizeof(float) : sizeof(float2));
    float2 res[C::NCR][PC];
    {
        const int t = tid % TC, c = tid / TC;
#pragma unroll
        for (int rho = 0; rho < C::NCR; ++rho) {
            const int col = rho * C::CPR + c;
            float2 z[PC];
#pragma unroll
            for (int q = 0; q < PC; ++q) {
                const unsigned o = (unsigned)(col * N + t + TC * q);
                float2 acc = fmul32<REAL>(fk, o, xb[o]);
#pragma unroll
                for (int v = 1; v < D; ++v) {
                    const unsigned ov = o + (unsigned)(NR * v);
                    acc = cadd(acc, cmul(fmul32<REAL>(fk, ov, xb[ov]), wf[v]));
                }
                z[q] = acc;
                // at most FG points' loads in flight: issuing all of them first would need more
                // registers than a thread of a 1024-thread block has
                if constexpr (D > 1)
                    if ((q + 1) % FG == 0) __builtin_amdgcn_sched_barrier(0);
            }
            if (col == 0) {
                // packed DC/Nyquist column: the beta term beta(xi) conj X(-xi) of the alpha/beta unpacking
#pragma unroll
                for (int q = 0; q < PC; ++q) {
#pragma unroll
                    for (int v = 0; v < D; ++v) {
                        const unsigned xi = (unsigned)(t + TC * q + NR * v);
                        const float2 y = fmul32<REAL>(fk, (unsigned)(L * N) + xi, cconj(xb[(N - xi) & (N - 1)]));
                        z[q] = cadd(z[q], v == 0 ? y : cmul(y, wf[v]));
                    }
                }
            }
            if constexpr (D > 1) {
#pragma unroll
                for (int q = 0; q < PC; ++q) z[q] = cmul(z[q], cconj(twN[((t + TC * q) * r) & (N - 1)]));
            }
            fft<NR, PC, true, D>(z, lds + c * C::COLSCR, t, twN);
#pragma unroll
            for (int q = 0; q < PC; ++q) res[rho][q] = z[q];
        }
    }

    // phases 2 and 3, one block of RPH rows at a time
    float* plane_out = out + ((size_t)b * K + k) * N * M;
#pragma unroll
    for (int h = 0; h < C::H; ++h) {
        __syncthreads();  // the column scratch, or the previous block's rows, is no longer read
        {
            const int t = tid % TC, c = tid / TC;
            constexpr int QH = PC / C::H;  // output rows t + TC q of block h: q in [h QH, (h + 1) QH)
#pragma unroll
            for (int rho = 0; rho < C::NCR; ++rho)
#pragma unroll
                for (int qq = 0; qq < QH; ++qq) {
                    const int q = h * QH + qq;
                    const int m = t + TC * q - h * C::RPH;
                    lds[m * C::PITCH + rho * C::CPR + c] = res[rho][q];
                }
        }
        __syncthreads();
#pragma unroll
        for (int rr = 0; rr < C::RPH / C::RPR; ++rr) {
            const int tr = tid % TR, mr = rr * C::RPR + tid / TR;
            float2* s = lds + mr * C::PITCH;
            float2 v[PR];
            const float2 P0 = s[0];
#pragma unroll
            for (int q = 0; q < PR; ++q) {
                const int kk = tr + TR * q;
                float2 X = s[kk], Xm = s[(L - kk) & (L - 1)];
                if (kk == 0) {
                    X = make_float2(P0.x, 0.0f);
                    Xm = make_float2(P0.y, 0.0f);
                }
                const float2 A = make_float2(X.x + Xm.x, X.y - Xm.y);   // X + conj(Xm)
                const float2 Dd = make_float2(X.x - Xm.x, X.y + Xm.y);  // X - conj(Xm)
                const float2 Bv = cmul(Dd, cconj(twM[kk]));
                v[q] = make_float2(A.x - Bv.y, A.y + Bv.x);  // A + i B
            }
            wave_sync();  // every lane of the row has read it before the FFT writes its scratch there
            fft<L, PR, true>(v, s, tr, twL);
            const int n1 = D * (h * C::RPH + mr) + r;
            float2* dst = reinterpret_cast<float2*>(plane_out + (size_t)n1 * M);
#pragma unroll
            for (int q = 0; q < PR; ++q) st_stream(dst + tr + TR * q, v[q]);
        }
    }
}

template <typename F>
hipError_t set_lds(F* fn, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int N>
hipError_t image_spectra_t(const DevPlan& d, const float2* A, float2* Xh, int nimg, float scale, hipStream_t st) {
    constexpr int P = (N >= 1024) ? 16 : 8, T = N / P;
    constexpr int PW = (512 / T >= 1) ? 512 / T : 1;
    const int pw = d.L < PW ? d.L : PW;
    if (d.L % pw != 0) return hipErrorInvalidValue;
    const size_t lds = (size_t)pw * (N + N / P) * sizeof(float2);
    if (pw == PW) {
        hipError_t e = set_lds(k_image_spectra<N, P, PW>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_image_spectra<N, P, PW>), dim3((unsigned)(nimg * (d.L / PW))), dim3(PW * T), lds, st, A,
                           Xh, d.L, scale, d.twN);
        return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

template <int N, int M>
constexpr int plane_d() {
    return (N * (M / 2) <= 32768) ? 1 : (N * (M / 2)) / 32768;
}

template <int N, int M>
hipError_t plane_fwd_t(const DevPlan& d, const float2* Xh, float* out, int nimg, const void* filt, hipStream_t st) {
    constexpr int D = plane_d<N, M>();
    using C = PlaneFwdCfg<N, M, D>;
    const bool by_xcd = nimg % 8 == 0;
    const size_t blocks = (size_t)nimg * d.K * D;
    if (d.real) {
        hipError_t e = set_lds(k_plane_fwd<N, M, D, true>, C::LDS);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_plane_fwd<N, M, D, true>), dim3((unsigned)blocks), dim3(C::THREADS), C::LDS, st, Xh, filt,
                           out, nimg, d.K, by_xcd ? 1 : 0, d.twN, d.twL, d.twM);
    } else {
        hipError_t e = set_lds(k_plane_fwd<N, M, D, false>, C::LDS);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_plane_fwd<N, M, D, false>), dim3((unsigned)blocks), dim3(C::THREADS), C::LDS, st, Xh,
                           filt, out, nimg, d.K, by_xcd ? 1 : 0, d.twN, d.twL, d.twM);
    }
    return hipGetLastError();
}

}  // namespace

// Sizes with a plane task shape: rows and columns in {128, 256, 512}, N/D in {128, 256}.
bool plane_fwd_supported(int N, int M) {
    auto ok = [](int n) { return n == 128 || n == 256 || n == 512; };
    return ok(N) && ok(M) && !(N == 512 && M == 128);
}

int plane_fwd_decimation(int N, int M) { return (N * (M / 2) <= 32768) ? 1 : (N * (M / 2)) / 32768; }

hipError_t launch_image_spectra(const DevPlan& d, const float2* A, float2* Xh, int nimg, float scale, hipStream_t st) {
    switch (d.N) {
        case 128: return image_spectra_t<128>(d, A, Xh, nimg, scale, st);
        case 256: return image_spectra_t<256>(d, A, Xh, nimg, scale, st);
        case 512: return image_spectra_t<512>(d, A, Xh, nimg, scale, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_plane_fwd(const DevPlan& d, const float2* Xh, float* out, int nimg, const void* filt,
                            hipStream_t st) {
    if (nimg <= 0) return hipSuccess;
    const int key = d.N * 4096 + d.M;
    switch (key) {
        case 128 * 4096 + 128: return plane_fwd_t<128, 128>(d, Xh, out, nimg, filt, st);
        case 128 * 4096 + 256: return plane_fwd_t<128, 256>(d, Xh, out, nimg, filt, st);
        case 128 * 4096 + 512: return plane_fwd_t<128, 512>(d, Xh, out, nimg, filt, st);
        case 256 * 4096 + 128: return plane_fwd_t<256, 128>(d, Xh, out, nimg, filt, st);
        case 256 * 4096 + 256: return plane_fwd_t<256, 256>(d, Xh, out, nimg, filt, st);
        case 256 * 4096 + 512: return plane_fwd_t<256, 512>(d, Xh, out, nimg, filt, st);
        case 512 * 4096 + 256: return plane_fwd_t<512, 256>(d, Xh, out, nimg, filt, st);
        case 512 * 4096 + 512: return plane_fwd_t<512, 512>(d, Xh, out, nimg, filt, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace shear
