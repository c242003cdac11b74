// Internal launch interface of the gfx950 kernels (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

namespace shear {

// Device-side description of a built system, passed to every launch.
struct DevPlan {
    int N = 0;                // rows (column FFT length)
    int M = 0;                // cols (real row length)
    int L = 0;                // M/2: packed half-spectrum columns
    int K = 0;                // filters
    bool real = false;        // filter sets stored as float (true) or float2
    const float2* twN = nullptr;  // exp(-2 pi i m / N), m < N
    const float2* twL = nullptr;  // exp(-2 pi i m / L), m < L
    const float2* twM = nullptr;  // exp(-2 pi i m / M), m < M
    int pw_fwd = 16;          // columns per block of the column passes (16 or 8; 8 when L < 16)
    int pw_inv = 16;
    int kg_fwd = 1;           // filter groups of the column passes (blocks per panel; capped at K)
    int kg_inv = 1;
    int pc_fwd = 0;           // points per thread of the column FFTs (0: col_points_default(N); else
    int pc_inv = 0;           // col_points_alternative(N), a different radix sequence)
    bool plane_fwd = false;   // shear_forward uses launch_plane_fwd (where plane_fwd_supported)
};

// Points per thread of the N-point column FFTs: the default, and the alternative the column-pass
// schedule may select instead (0 if there is none for this N).
int col_points_default(int N);
int col_points_alternative(int N);

// Partial-sum scratch of the inverse column pass for nimg images (float2 elements; 0 when kg_inv is 1).
inline size_t cols_inv_part_elems(const DevPlan& d, int nimg) {
    int kg = d.kg_inv < 1 ? 1 : (d.kg_inv > d.K ? d.K : d.kg_inv);
    if (kg <= 1) return 0;
    const int kper = (d.K + kg - 1) / kg;
    kg = (d.K + kper - 1) / kper;
    return kg <= 1 ? 0 : (size_t)nimg * kg * ((size_t)d.L * d.N + d.N);
}

// coeff_planes selects a separate kernel symbol for coefficient planes (same code).
// Rows (real, row-major planes x N x M) -> packed row spectra, planes of L x N
// float2 in the panel layout of kernels.hip (panels of 8 columns, 16-row tiles
// down each panel): element (r, k) = sum_c in[p][r][c] e^{-2 pi i k c / M},
// with element (r, 0) = X(0) + i X(M/2).
hipError_t launch_rows_r2c(const DevPlan& d, const float* in, float2* out, int planes, bool coeff_planes,
                           hipStream_t st);

// Inverse of the above up to scale: packed spectra (panel layout) -> real rows,
// out = scale * (unnormalised length-M inverse DFT of the Hermitian rows).
hipError_t launch_rows_c2r(const DevPlan& d, const float2* in, float* out, int planes, float scale, bool coeff_planes,
                           hipStream_t st);
// Row stage of an inpainting iteration: rows of u = mask (fm - f) + f (planes x N x M each) -> packed
// spectra in the panel layout, as launch_rows_r2c.
hipError_t launch_rows_r2c_mix(const DevPlan& d, const float* fm, const float* mask, const float* f, float2* out,
                               int planes, hipStream_t st);
// Coefficient row stages with a hard threshold between them, in place on
// nplanes packed planes; thr[p] and kept[p] (kept may be null) per plane.
hipError_t launch_rows_thresh(const DevPlan& d, float2* planes, int nplanes, const float* thr, unsigned* kept,
                              hipStream_t st);

// Forward transform, column stage, K-expanding: for each image of A (nimg x L x N),
// X = scale * colFFT(A); for each filter k: T[b][k] = colIFFT(filt_k (.) X)
// (DC/Nyquist packed column handled with the alpha/beta filter columns).
hipError_t launch_cols_fwd(const DevPlan& d, const float2* A, float2* T, int nimg, const void* filt, float scale,
                           hipStream_t st);

// Inverse / adjoint, column stage, K-reducing: V[b] = colIFFT( sum_k filt_k (.) colFFT(U[b][k]) ).
// part: cols_inv_part_elems(d, nimg) float2 of scratch (may be null when that is 0).
hipError_t launch_cols_inv(const DevPlan& d, const float2* U, float2* V, int nimg, const void* filt, float2* part,
                           hipStream_t st);

// Whole-plane forward (one workgroup per (image, filter) plane, its transposition on chip),
// available for 256 x 256 systems with real filter sets. Its operands are residue-major: element
// (xi, j) of an N x L packed plane at ((xi mod 16) (N / 16) + xi / 16) L + j.
// launch_plane_filters writes the forward filter set (K x (L + 1) x N floats, column-major, packed
// column 0's mirrored-term filter in column L) in that layout, per filter N x L floats and then the
// N mirrored-term floats (the same size); launch_cols_spec turns the packed row spectra A (as
// launch_cols_fwd takes them) into the column spectra Xr = scale * colFFT(A) (nimg x N x L float2);
// launch_plane_fwd then writes the coefficient planes out (nimg x K x N x M): the values of
// launch_cols_fwd followed by launch_rows_c2r (scale 1), up to rounding.
bool plane_fwd_supported(const DevPlan& d);
hipError_t launch_plane_filters(const DevPlan& d, const float* filt, float* fr, hipStream_t st);
hipError_t launch_cols_spec(const DevPlan& d, const float2* A, float2* Xr, int nimg, float scale, hipStream_t st);
hipError_t launch_plane_fwd(const DevPlan& d, const float2* Xr, float* out, int nimg, const float* fr,
                            hipStream_t st);

bool size_supported(int n);

// Fills n words with zero (a kernel, so that the fill can be captured in a graph).
hipError_t launch_zero_u32(unsigned* p, int n, hipStream_t st);

// Size of the fixed device scratch of the allocation-free forward (one copy per device).
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
// Device address of that scratch on the current device (looked up once per device).
hipError_t static_scratch(void** ptr);

}  // namespace shear
