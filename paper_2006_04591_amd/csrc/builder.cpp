// FP64 host construction of the shearlet filter bank (Section 3.4.1, built on
// the digital construction of Section 2.1).
//
// Every filter is first built as a real spatial kernel and then transformed
// with a host FFT:
//   * low-pass h: 9-tap symmetric filter fixed by the design spec of
//     Section 3.4.1 (order 8, maximally flat, half power at half band), i.e.
//     hhat(0)=1, hhat''(0)=hhat''''(0)=0, hhat(pi)=0, hhat(pi/2)=1/sqrt(2);
//     mirror high-pass g[n] = (-1)^n h[n];
//   * a-trous chains (Section 2.1): h_(l) = h * (h up 2) * ... * (h up 2^(l-1)),
//     g_(l) = (g up 2^(l-1)) * h_(l-1);
//   * fan filter P: maximally flat diamond half-band filter (McClellan mapping
//     of the 1-D maxflat half-band polynomial of order 4), modulated by
//     (-1)^n1 into a fan passing |w2| < |w1|; expanded here as a polynomial of
//     the 3x3 mapping kernel by repeated 2-D convolution;
//   * wedge (shear level s, shear k, U = 2^s): narrow the fan by U along x2
//     (upsample x2, convolve with h_(s)), then the digital shear of
//     eqs. (2.5), (2.4): upsample x1 by U, convolve x1 with h_(s), shear
//     n -> (n1 + k n2, n2), convolve x1 with reversed h_(s), keep every U-th
//     x1 sample and scale by U;
//   * cone-1 shearlet = band-pass g_(J-j+1) along x1 convolved with the wedge
//     (Definition 2.3, eq. (2.6)); cone 2 = transpose; low-pass = h_(J) (x) h_(J).
// Axis 0 of the array is x1.
#include "builder.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace shear {

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

namespace {

// Centred real kernel with half-widths r0 (axis 0) and r1 (axis 1).
struct Ker {
    int r0 = 0, r1 = 0;
    std::vector<double> v;
    Ker() = default;
    Ker(int a, int b) : r0(a), r1(b), v((size_t)(2 * a + 1) * (2 * b + 1), 0.0) {}
    int w() const { return 2 * r1 + 1; }
    double& at(int i, int j) { return v[(size_t)(i + r0) * w() + (j + r1)]; }
    double at(int i, int j) const { return v[(size_t)(i + r0) * w() + (j + r1)]; }
};

using Taps = std::vector<double>;  // odd length, centred

Taps conv1(const Taps& a, const Taps& b) {
    Taps out(a.size() + b.size() - 1, 0.0);
    for (size_t i = 0; i < a.size(); ++i)
        for (size_t j = 0; j < b.size(); ++j) out[i + j] += a[i] * b[j];
    return out;
}

Taps up1(const Taps& a, int U) {
    int r = (int)a.size() / 2;
    Taps out((size_t)2 * r * U + 1, 0.0);
    for (int n = -r; n <= r; ++n) out[(size_t)(n * U + r * U)] = a[(size_t)(n + r)];
    return out;
}

Taps atrous_low(const Taps& h, int level) {
    Taps out{1.0};
    for (int i = 0; i < level; ++i) out = conv1(out, up1(h, 1 << i));
    return out;
}

Ker conv2(const Ker& a, const Ker& b) {
    Ker out(a.r0 + b.r0, a.r1 + b.r1);
    for (int i = -a.r0; i <= a.r0; ++i)
        for (int j = -a.r1; j <= a.r1; ++j) {
            double av = a.at(i, j);
            if (av == 0.0) continue;
            for (int p = -b.r0; p <= b.r0; ++p)
                for (int q = -b.r1; q <= b.r1; ++q) out.at(i + p, j + q) += av * b.at(p, q);
        }
    return out;
}

Ker conv_axis(const Ker& a, const Taps& t, int axis) {
    int rt = (int)t.size() / 2;
    Ker out(a.r0 + (axis == 0 ? rt : 0), a.r1 + (axis == 1 ? rt : 0));
    for (int i = -a.r0; i <= a.r0; ++i)
        for (int j = -a.r1; j <= a.r1; ++j) {
            double av = a.at(i, j);
            if (av == 0.0) continue;
            for (int n = -rt; n <= rt; ++n) {
                if (axis == 0)
                    out.at(i + n, j) += av * t[(size_t)(n + rt)];
                else
                    out.at(i, j + n) += av * t[(size_t)(n + rt)];
            }
        }
    return out;
}

Ker up_axis(const Ker& a, int U, int axis) {
    Ker out(axis == 0 ? a.r0 * U : a.r0, axis == 1 ? a.r1 * U : a.r1);
    for (int i = -a.r0; i <= a.r0; ++i)
        for (int j = -a.r1; j <= a.r1; ++j) {
            if (axis == 0)
                out.at(i * U, j) = a.at(i, j);
            else
                out.at(i, j * U) = a.at(i, j);
        }
    return out;
}

// n -> (n1 + k n2, n2): out(n1, n2) = in(n1 + k n2, n2)
Ker shear_x1(const Ker& a, int k) {
    Ker out(a.r0 + std::abs(k) * a.r1, a.r1);
    for (int i = -out.r0; i <= out.r0; ++i)
        for (int j = -a.r1; j <= a.r1; ++j) {
            int src = i + k * j;
            if (src >= -a.r0 && src <= a.r0) out.at(i, j) = a.at(src, j);
        }
    return out;
}

// keep every U-th sample along axis 0 (the centre is kept) and scale by U
Ker down_x1(const Ker& a, int U) {
    Ker out(a.r0 / U, a.r1);
    for (int i = -out.r0; i <= out.r0; ++i)
        for (int j = -a.r1; j <= a.r1; ++j) out.at(i, j) = U * a.at(i * U, j);
    return out;
}

Ker transpose(const Ker& a) {
    Ker out(a.r1, a.r0);
    for (int i = -a.r0; i <= a.r0; ++i)
        for (int j = -a.r1; j <= a.r1; ++j) out.at(j, i) = a.at(i, j);
    return out;
}

Ker scaled_sum(const Ker& a, double ca, const Ker& b, double cb) {
    Ker out(std::max(a.r0, b.r0), std::max(a.r1, b.r1));
    for (int i = -a.r0; i <= a.r0; ++i)
        for (int j = -a.r1; j <= a.r1; ++j) out.at(i, j) += ca * a.at(i, j);
    for (int i = -b.r0; i <= b.r0; ++i)
        for (int j = -b.r1; j <= b.r1; ++j) out.at(i, j) += cb * b.at(i, j);
    return out;
}

Ker delta() {
    Ker d(0, 0);
    d.at(0, 0) = 1.0;
    return d;
}

// Solves the 5 design conditions for a0..a4, hhat(w) = a0 + 2 sum a_n cos(n w).
Taps default_scaling() {
    double A[5][6] = {
        {1, 2, 2, 2, 2, 1.0},                    // hhat(0) = 1
        {0, 1, 4, 9, 16, 0.0},                   // sum n^2 a_n = 0
        {0, 1, 16, 81, 256, 0.0},                // sum n^4 a_n = 0
        {1, -2, 2, -2, 2, 0.0},                  // hhat(pi) = 0
        {1, 0, -2, 0, 2, 1.0 / std::sqrt(2.0)},  // hhat(pi/2) = 1/sqrt(2)
    };
    for (int c = 0; c < 5; ++c) {
        int piv = c;
        for (int r = c + 1; r < 5; ++r)
            if (std::fabs(A[r][c]) > std::fabs(A[piv][c])) piv = r;
        for (int j = 0; j < 6; ++j) std::swap(A[c][j], A[piv][j]);
        for (int r = 0; r < 5; ++r) {
            if (r == c) continue;
            double f = A[r][c] / A[c][c];
            for (int j = c; j < 6; ++j) A[r][j] -= f * A[c][j];
        }
    }
    double a[5];
    for (int i = 0; i < 5; ++i) a[i] = A[i][5] / A[i][i];
    Taps h(9);
    for (int n = -4; n <= 4; ++n) h[(size_t)(n + 4)] = a[std::abs(n)];
    return h;
}

Taps mirror(const Taps& h) {
    int r = (int)h.size() / 2;
    Taps g(h.size());
    for (int n = -r; n <= r; ++n) g[(size_t)(n + r)] = ((n % 2) == 0 ? 1.0 : -1.0) * h[(size_t)(n + r)];
    return g;
}

double binom(int n, int k) {
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

// P = H(y), y = (1 - t)/2, t = (cos w2 - cos w1)/2, H(y) = (1-y)^L sum_i C(L-1+i, i) y^i
Ker default_fan(int L) {
    Ker t(1, 1);
    t.at(1, 0) = t.at(-1, 0) = -0.25;
    t.at(0, 1) = t.at(0, -1) = 0.25;
    Ker y = scaled_sum(delta(), 0.5, t, -0.5);
    Ker omy = scaled_sum(delta(), 0.5, t, 0.5);  // 1 - y
    Ker omyL = delta();
    for (int i = 0; i < L; ++i) omyL = conv2(omyL, omy);
    Ker poly(0, 0), ypow = delta();
    for (int i = 0; i < L; ++i) {
        poly = scaled_sum(poly, 1.0, ypow, binom(L - 1 + i, i));
        ypow = conv2(ypow, y);
    }
    return conv2(omyL, poly);
}

bool symmetric_taps(const Taps& h) {
    for (size_t i = 0; i < h.size(); ++i)
        if (h[i] != h[h.size() - 1 - i]) return false;
    return true;
}

bool centro_symmetric(const Ker& k) {
    for (int i = -k.r0; i <= k.r0; ++i)
        for (int j = -k.r1; j <= k.r1; ++j)
            if (k.at(i, j) != k.at(-i, -j)) return false;
    return true;
}

// iterative radix-2 FFT of a contiguous array with a precomputed table
// tw[m] = exp(-+ 2 pi i m / n), m < n/2
void fft1(cd* a, int n, const std::vector<cd>& tw) {
    for (int i = 1, j = 0; i < n; ++i) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(a[i], a[j]);
    }
    for (int len = 2; len <= n; len <<= 1) {
        const int half = len / 2, step = n / len;
        for (int i = 0; i < n; i += len)
            for (int k = 0; k < half; ++k) {
                const cd u = a[i + k];
                const cd b = a[i + k + half], w = tw[(size_t)k * step];
                // explicit product: std::complex operator* takes the slow Annex-G path
                const cd v(b.real() * w.real() - b.imag() * w.imag(), b.real() * w.imag() + b.imag() * w.real());
                a[i + k] = u + v;
                a[i + k + half] = u - v;
            }
    }
}

std::vector<cd> fft_table(int n, bool inverse) {
    std::vector<cd> tw((size_t)std::max(1, n / 2));
    const double sgn = inverse ? 1.0 : -1.0;
    for (int m = 0; m < n / 2; ++m) {
        const double ang = sgn * 2.0 * M_PI * (double)m / (double)n;
        tw[(size_t)m] = cd(std::cos(ang), std::sin(ang));
    }
    return tw;
}

}  // namespace

void fft2_host(cd* a, int rows, int cols, bool inverse) {
    const std::vector<cd> twc = fft_table(cols, inverse), twr = fft_table(rows, inverse);
    for (int r = 0; r < rows; ++r) fft1(a + (size_t)r * cols, cols, twc);
    std::vector<cd> col((size_t)rows);
    for (int c = 0; c < cols; ++c) {
        for (int r = 0; r < rows; ++r) col[(size_t)r] = a[(size_t)r * cols + c];
        fft1(col.data(), rows, twr);
        for (int r = 0; r < rows; ++r) a[(size_t)r * cols + c] = col[(size_t)r];
    }
}

int count_filters(const shear_build_params* p, int& K, std::string& err) {
    if (!p) {
        err = "params is NULL";
        return SHEAR_E_INVALID;
    }
    if (p->n_scales < 1 || p->n_scales > 8) {
        err = "n_scales must be in [1, 8]";
        return SHEAR_E_INVALID;
    }
    K = 1;
    for (int j = 1; j <= p->n_scales; ++j) {
        const int s = p->shear_levels ? p->shear_levels[j - 1] : (j + 1) / 2;
        if (s < 0 || s > 4) {
            err = "shear levels must be in [0, 4]";
            return SHEAR_E_INVALID;
        }
        K += 4 << s;  // (2^{s+1} + 1) cone-1 shears + (2^{s+1} - 1) cone-2 shears
    }
    return SHEAR_OK;
}

int design(const shear_build_params* p, Design& out, std::string& err) {
    if (!p) {
        err = "params is NULL";
        return SHEAR_E_INVALID;
    }
    const int rows = p->rows, cols = p->cols, J = p->n_scales;
    if (J < 1 || J > 8) {
        err = "n_scales must be in [1, 8]";
        return SHEAR_E_INVALID;
    }
    if (!is_pow2(rows) || !is_pow2(cols) || rows < 4 || cols < 4 || rows > 4096 || cols > 4096) {
        err = "rows and cols must be powers of two in [4, 4096]";
        return SHEAR_E_SIZE;
    }
    std::vector<int> levels((size_t)J);
    for (int j = 1; j <= J; ++j) {
        levels[(size_t)(j - 1)] = p->shear_levels ? p->shear_levels[j - 1] : (j + 1) / 2;
        if (levels[(size_t)(j - 1)] < 0 || levels[(size_t)(j - 1)] > 4) {
            err = "shear levels must be in [0, 4]";
            return SHEAR_E_INVALID;
        }
    }
    Taps h;
    if (p->scaling_taps) {
        if (p->n_scaling < 1 || (p->n_scaling % 2) == 0) {
            err = "scaling_taps must have odd length";
            return SHEAR_E_INVALID;
        }
        h.assign(p->scaling_taps, p->scaling_taps + p->n_scaling);
    } else {
        h = default_scaling();
    }
    Ker fan;
    if (p->fan_taps) {
        if (p->fan_rows < 1 || p->fan_cols < 1 || (p->fan_rows % 2) == 0 || (p->fan_cols % 2) == 0) {
            err = "fan_taps must have odd sizes";
            return SHEAR_E_INVALID;
        }
        fan = Ker(p->fan_rows / 2, p->fan_cols / 2);
        std::memcpy(fan.v.data(), p->fan_taps, sizeof(double) * fan.v.size());
    } else {
        fan = default_fan(4);
    }
    const Taps g = mirror(h);

    std::vector<Ker> kers;
    std::vector<int> idx;
    for (int j = 1; j <= J; ++j) {
        const int s = levels[(size_t)(j - 1)], U = 1 << s, lvl = J - j + 1;
        const Taps hs = atrous_low(h, s);
        Taps hs_rev(hs.rbegin(), hs.rend());
        const Taps band = conv1(up1(g, 1 << (lvl - 1)), atrous_low(h, lvl - 1));
        // narrowed directional filter, then up-sampled and interpolated along x1 (eq. (2.5))
        const Ker q = conv_axis(up_axis(conv_axis(up_axis(fan, U, 1), hs, 1), U, 0), hs, 0);
        for (int cone = 1; cone <= 2; ++cone) {
            const int kmax = (cone == 1) ? U : U - 1;
            for (int k = -kmax; k <= kmax; ++k) {
                Ker wedge = down_x1(conv_axis(shear_x1(q, k), hs_rev, 0), U);  // eq. (2.4)
                Ker ker = conv_axis(wedge, band, 0);
                if (cone == 2) ker = transpose(ker);
                kers.push_back(std::move(ker));
                idx.insert(idx.end(), {cone, j, k});
            }
        }
    }
    {
        const Taps hl = atrous_low(h, J);
        int r = (int)hl.size() / 2;
        Ker low(r, r);
        for (int i = -r; i <= r; ++i)
            for (int j = -r; j <= r; ++j) low.at(i, j) = hl[(size_t)(i + r)] * hl[(size_t)(j + r)];
        kers.push_back(std::move(low));
        idx.insert(idx.end(), {0, 0, 0});
    }
    for (const Ker& k : kers) {
        if (2 * k.r0 + 1 > rows || 2 * k.r1 + 1 > cols) {
            err = "a constructed shearlet kernel (" + std::to_string(2 * k.r0 + 1) + "x" + std::to_string(2 * k.r1 + 1) +
                  ") does not fit in " + std::to_string(rows) + "x" + std::to_string(cols) + "; use fewer scales or larger images";
            return SHEAR_E_SIZE;
        }
    }
    const bool real = symmetric_taps(h) && centro_symmetric(fan);
    out.rows = rows;
    out.cols = cols;
    out.K = (int)kers.size();
    out.idx = idx;
    out.real = real;
    out.spectra.assign((size_t)out.K * rows * cols, cd(0, 0));
    for (int f = 0; f < out.K; ++f) {
        cd* a = out.spectra.data() + (size_t)f * rows * cols;
        const Ker& k = kers[(size_t)f];
        for (int i = -k.r0; i <= k.r0; ++i)
            for (int j = -k.r1; j <= k.r1; ++j)
                a[(size_t)((i + rows) % rows) * cols + (size_t)((j + cols) % cols)] += k.at(i, j);
        fft2_host(a, rows, cols, false);
        if (real)  // centro-symmetric real kernels have real spectra; drop the rounding residue
            for (size_t e = 0; e < (size_t)rows * cols; ++e) a[e] = cd(a[e].real(), 0.0);
    }
    return SHEAR_OK;
}

}  // namespace shear
