// Host-side (FP64) construction of the shearlet filter bank: Section 3.4.1
// (getshearletsystem2D) realised through the digital construction of Section 2.1.
#pragma once

#include <complex>
#include <string>
#include <vector>

#include "shear.h"

namespace shear {

using cd = std::complex<double>;

struct Design {
    int rows = 0, cols = 0, K = 0;
    std::vector<cd> spectra;  // K x rows x cols, natural DFT order (index 0 = zero frequency)
    std::vector<int> idx;     // K x 3: cone, scale, shear
    bool real = false;        // spectra are exactly real (symmetric filters)
};

// Builds the filter bank described by p (FP64). Returns SHEAR_OK or an error
// code with a message in err.
int design(const shear_build_params* p, Design& out, std::string& err);

// Validates p and returns the number of filters without building them.
int count_filters(const shear_build_params* p, int& K, std::string& err);

// In-place unnormalised 2-D DFT (forward: exp(-2 pi i ...)) of a rows x cols
// row-major array, both sizes powers of two.
void fft2_host(cd* a, int rows, int cols, bool inverse);

bool is_pow2(int n);

}  // namespace shear
