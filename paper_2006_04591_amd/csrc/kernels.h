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
};

// coeff_planes selects a separate kernel symbol for coefficient planes (same code).
// Rows (real, row-major planes x N x M) -> packed row spectra, column-major
// (planes x L x N): out[p][k][r] = sum_c in[p][r][c] e^{-2 pi i k c / M}, with
// out[p][0][r] = X(0) + i X(M/2).
hipError_t launch_rows_r2c(const DevPlan& d, const float* in, float2* out, int planes, bool coeff_planes,
                           hipStream_t st);

// Inverse of the above up to scale: packed column-major spectra -> real rows,
// out = scale * (unnormalised length-M inverse DFT of the Hermitian rows).
hipError_t launch_rows_c2r(const DevPlan& d, const float2* in, float* out, int planes, float scale, bool coeff_planes,
                           hipStream_t st);

// Forward transform, column stage, K-expanding: for each image of A (nimg x L x N),
// X = scale * colFFT(A); for each filter k: T[b][k] = colIFFT(filt_k (.) X)
// (DC/Nyquist packed column handled with the alpha/beta filter columns).
hipError_t launch_cols_fwd(const DevPlan& d, const float2* A, float2* T, int nimg, const void* filt, float scale,
                           hipStream_t st);

// Inverse / adjoint, column stage, K-reducing: V[b] = colIFFT( sum_k filt_k (.) colFFT(U[b][k]) ).
hipError_t launch_cols_inv(const DevPlan& d, const float2* U, float2* V, int nimg, const void* filt, hipStream_t st);

bool size_supported(int n);

}  // namespace shear
