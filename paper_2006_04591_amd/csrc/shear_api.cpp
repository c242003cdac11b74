// C ABI of the shearlet filter-bank library (declared in include/shear.h).
//
// Host side of every call: argument checks, the FP64 -> FP32 preparation of
// the three device filter sets, workspace management and kernel launches.
// The device work itself is in kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "builder.h"
#include "kernels.h"
#include "shear.h"
#include "shrink.h"

using shear::cd;

struct shear_system {
    int device = -1;
    int rows = 0, cols = 0, K = 0;
    bool real = false;
    std::vector<cd> spectra;   // K x rows x cols, natural order
    std::vector<double> W;     // rows x cols, natural order
    std::vector<double> rms;   // K
    std::vector<int> idx;      // K x 3
    // device
    void* dev_block = nullptr;  // twiddles + three filter sets
    const void* filt_fwd = nullptr;
    const void* filt_inv = nullptr;
    const void* filt_adj = nullptr;
    const float* filt_plane = nullptr;  // forward set, residue-major (whole-plane forward), or null
    const float* rms_dev = nullptr;  // RMS_k as float (learned shrinkage)
    shear::DevPlan plan;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    size_t ws_cap = 0;
    // per-launch timing (shear_profile_enable / shear_profile_read)
    bool prof_on = false;
    std::vector<hipEvent_t> ev_free;
    struct Rec {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Rec> prof;
    int cus = 0;  // compute units of the device
    // inpainting: the whole iteration sequence of the last call shape, captured as one HIP graph
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    std::vector<const void*> graph_key;
    // shear_inpaint_groups led by this system: the branches of every group in one graph
    hipGraph_t ggraph = nullptr;
    hipGraphExec_t ggexec = nullptr;
    std::vector<const void*> ggraph_key;
    // learned shrinkage: scales and hidden activations
    void* ws2 = nullptr;
    size_t ws2_bytes = 0;
};

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(SHEAR_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

size_t centred_to_natural(size_t i, int n) { return (i + (size_t)n / 2) % (size_t)n; }

// Natural-order index (r, c) of the centred-layout element (rc, cc): the
// centred layout is fftshift(natural), so centred[rc] = natural[(rc + n/2) mod n]
// for even n (the only sizes accepted).
void centred_to_natural_spectra(const double* in, int K, int rows, int cols, std::vector<cd>& out) {
    out.assign((size_t)K * rows * cols, cd(0, 0));
    for (int k = 0; k < K; ++k)
        for (int r = 0; r < rows; ++r)
            for (int c = 0; c < cols; ++c) {
                const double* e = in + (((size_t)k * rows + r) * cols + c) * 2;
                out[((size_t)k * rows + centred_to_natural(r, rows)) * cols + centred_to_natural(c, cols)] = cd(e[0], e[1]);
            }
}

void natural_to_centred(const cd* in, int rows, int cols, double* out2 /* (re,im) */, double* outr /* real */) {
    for (int r = 0; r < rows; ++r)
        for (int c = 0; c < cols; ++c) {
            const cd v = in[(size_t)centred_to_natural(r, rows) * cols + centred_to_natural(c, cols)];
            const size_t o = (size_t)r * cols + c;
            if (out2) {
                out2[2 * o] = v.real();
                out2[2 * o + 1] = v.imag();
            }
            if (outr) outr[o] = v.real();
        }
}

// Device filter set layout: [k][col in 0..L][row in 0..N-1], float or float2.
//   columns 1..L-1 : the filter value at (row, col);
//   column 0       : (f(row, 0) + f(row, M/2)) / 2           -- acts on the packed DC/Nyquist column
//   column L       : forward: (f(row, 0) - f(row, M/2)) / 2,  multiplies conj(X(-row))
//                    inverse: conj of that at row -row,       accumulated then mirrored once
// where f = conj(Psi) (forward) or the dual / adjoint filter Psi * wgt (inverse side).
void pack_filter_set(const shear_system& s, bool forward, const std::vector<double>& wgt, std::vector<float>& out) {
    const int N = s.rows, M = s.cols, L = M / 2, K = s.K;
    const size_t per = (size_t)(L + 1) * N;
    const int comps = s.real ? 1 : 2;
    out.assign((size_t)K * per * comps, 0.0f);
    auto put = [&](int k, int col, int row, cd v) {
        const size_t i = (size_t)k * per + (size_t)col * N + row;
        if (s.real) {
            out[i] = (float)v.real();
        } else {
            out[2 * i] = (float)v.real();
            out[2 * i + 1] = (float)v.imag();
        }
    };
    for (int k = 0; k < K; ++k) {
        const cd* P = s.spectra.data() + (size_t)k * N * M;
        auto f = [&](int row, int col) -> cd {
            const cd v = P[(size_t)row * M + col];
            return forward ? std::conj(v) : v * wgt[(size_t)row * M + col];
        };
        for (int row = 0; row < N; ++row) {
            for (int col = 1; col < L; ++col) put(k, col, row, f(row, col));
            put(k, 0, row, 0.5 * (f(row, 0) + f(row, L)));
            if (forward) {
                put(k, L, row, 0.5 * (f(row, 0) - f(row, L)));
            } else {
                const int mr = (N - row) % N;
                put(k, L, row, std::conj(0.5 * (f(mr, 0) - f(mr, L))));
            }
        }
    }
}

int finish_system(shear_system* s, std::string& why) {
    const int N = s->rows, M = s->cols, K = s->K;
    const size_t NM = (size_t)N * M;
    s->W.assign(NM, 0.0);
    s->rms.assign((size_t)K, 0.0);
    for (int k = 0; k < K; ++k) {
        double e = 0.0;
        for (size_t i = 0; i < NM; ++i) {
            const double a = std::norm(s->spectra[(size_t)k * NM + i]);
            s->W[i] += a;
            e += a;
        }
        s->rms[(size_t)k] = std::sqrt(e / (double)NM);
    }
    const double wmin = *std::min_element(s->W.begin(), s->W.end());
    const double wmax = *std::max_element(s->W.begin(), s->W.end());
    if (!(wmin > 1e-10 * wmax)) {
        why = "dual-frame weight is (nearly) zero: min W = " + std::to_string(wmin) + ", max W = " + std::to_string(wmax);
        return SHEAR_E_FRAME;
    }
    // filter sets (FP64 -> FP32 once)
    std::vector<double> winv(NM), wadj(NM, 1.0 / (double)NM);
    for (size_t i = 0; i < NM; ++i) winv[i] = 1.0 / (s->W[i] * (double)NM);
    std::vector<float> ffwd, finv, fadj;
    pack_filter_set(*s, true, wadj, ffwd);
    pack_filter_set(*s, false, winv, finv);
    pack_filter_set(*s, false, wadj, fadj);
    // twiddles exp(-2 pi i m / n), computed in FP64 and rounded once
    const int L = M / 2;
    std::vector<float> tw;
    auto add_tw = [&](int n) {
        size_t off = tw.size();
        for (int m = 0; m < n; ++m) {
            const double a = -2.0 * M_PI * (double)m / (double)n;
            tw.push_back((float)std::cos(a));
            tw.push_back((float)std::sin(a));
        }
        return off;
    };
    const size_t oN = add_tw(N), oL = add_tw(L), oM = add_tw(M);
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t b_tw = al(tw.size() * sizeof(float));
    const size_t b_f = al(ffwd.size() * sizeof(float));
    std::vector<float> rms32(s->rms.begin(), s->rms.end());
    const size_t b_r = al((size_t)K * sizeof(float));
    // the forward filter set once more, residue-major, where the whole-plane forward is compiled
    // (the test of shear::plane_fwd_supported)
    const bool plane = s->real && N == 256 && M == 256;
    const size_t total = b_tw + 3 * b_f + b_r + (plane ? b_f : 0);
    hipError_t e = hipMalloc(&s->dev_block, total);
    if (e != hipSuccess) {
        s->dev_block = nullptr;
        why = std::string("hipMalloc of the filter bank failed: ") + hipGetErrorString(e);
        return SHEAR_E_NOMEM;
    }
    char* base = (char*)s->dev_block;
    if ((e = hipMemcpy(base, tw.data(), tw.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(base + b_tw, ffwd.data(), ffwd.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(base + b_tw + b_f, finv.data(), finv.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(base + b_tw + 2 * b_f, fadj.data(), fadj.size() * sizeof(float), hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (e = hipMemcpy(base + b_tw + 3 * b_f, rms32.data(), rms32.size() * sizeof(float), hipMemcpyHostToDevice)) !=
            hipSuccess) {
        why = std::string("hipMemcpy of the filter bank failed: ") + hipGetErrorString(e);
        return SHEAR_E_HIP;
    }
    const float2* twb = (const float2*)base;
    s->plan.N = N;
    s->plan.M = M;
    s->plan.L = L;
    s->plan.K = K;
    s->plan.real = s->real;
    s->plan.twN = twb + oN / 2;
    s->plan.twL = twb + oL / 2;
    s->plan.twM = twb + oM / 2;
    s->filt_fwd = base + b_tw;
    s->filt_inv = base + b_tw + b_f;
    s->filt_adj = base + b_tw + 2 * b_f;
    s->rms_dev = (const float*)(base + b_tw + 3 * b_f);
    if (plane) {
        float* fr = (float*)(base + b_tw + 3 * b_f + b_r);
        if ((e = shear::launch_plane_filters(s->plan, (const float*)s->filt_fwd, fr, nullptr)) != hipSuccess ||
            (e = hipStreamSynchronize(nullptr)) != hipSuccess) {
            why = std::string("reordering the forward filters failed: ") + hipGetErrorString(e);
            return SHEAR_E_HIP;
        }
        s->filt_plane = fr;
    }
    if ((e = hipDeviceGetAttribute(&s->cus, hipDeviceAttributeMultiprocessorCount, s->device)) != hipSuccess) {
        why = std::string("querying the compute-unit count failed: ") + hipGetErrorString(e);
        return SHEAR_E_HIP;
    }
    return SHEAR_OK;
}

void release(shear_system* s) {
    if (!s) return;
    for (auto& r : s->prof) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t e : s->ev_free) (void)hipEventDestroy(e);
    if (s->ggexec) (void)hipGraphExecDestroy(s->ggexec);
    if (s->ggraph) (void)hipGraphDestroy(s->ggraph);
    if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
    if (s->dev_block) (void)hipFree(s->dev_block);
    if (s->ws) (void)hipFree(s->ws);
    if (s->ws2) (void)hipFree(s->ws2);
    delete s;
}

int new_system(int rows, int cols, size_t cap, shear_system** out, shear_system*& s) {
    if (!out) return fail(SHEAR_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!shear::size_supported(rows) || !shear::size_supported(cols))
        return fail(SHEAR_E_SIZE, "GPU path needs rows and cols powers of two in [16, 2048], got " + std::to_string(rows) +
                                      "x" + std::to_string(cols));
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    s = new (std::nothrow) shear_system();
    if (!s) return fail(SHEAR_E_NOMEM, "host allocation failed");
    s->device = dev;
    s->rows = rows;
    s->cols = cols;
    s->ws_cap = cap ? cap : ((size_t)4 << 30);
    return SHEAR_OK;
}

size_t plane_bytes(const shear_system* s) { return (size_t)s->rows * (s->cols / 2) * sizeof(float2); }

// Separate-path workspace: [batch planes A or V][chunk x K exchange planes][inverse partial sums of chunk images].
size_t part_bytes(const shear_system* s, int chunk) { return shear::cols_inv_part_elems(s->plan, chunk) * sizeof(float2); }

// Images per chunk of the K-expanded intermediate, or 0 if even one does not fit.
int chunk_images(const shear_system* s, int batch) {
    const size_t pb = plane_bytes(s);
    const size_t fixed = (size_t)batch * pb;
    if (fixed >= s->ws_cap) return 0;
    const size_t per = (size_t)s->K * pb + part_bytes(s, 1);
    const size_t n = (s->ws_cap - fixed) / per;
    return (int)std::min<size_t>(n, (size_t)batch);
}

size_t ws_needed(const shear_system* s, int batch, int chunk) {
    return (size_t)batch * plane_bytes(s) + (size_t)chunk * s->K * plane_bytes(s) + part_bytes(s, chunk);
}

// The inverse partial-sum scratch after the exchange planes of a chunk.
float2* part_ptr(const shear_system* s, int batch, int chunk) {
    if (part_bytes(s, chunk) == 0) return nullptr;
    return (float2*)((char*)s->ws + (size_t)batch * plane_bytes(s) + (size_t)chunk * s->K * plane_bytes(s));
}

int ensure_ws(shear_system* s, size_t bytes) {
    if (bytes <= s->ws_bytes) return SHEAR_OK;
    if (s->ws) {
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize before workspace growth");
        (void)hipFree(s->ws);
        s->ws = nullptr;
        s->ws_bytes = 0;
    }
    hipError_t e = hipMalloc(&s->ws, bytes);
    if (e != hipSuccess) {
        s->ws = nullptr;
        return fail(SHEAR_E_NOMEM, std::string("workspace hipMalloc failed: ") + hipGetErrorString(e));
    }
    s->ws_bytes = bytes;
    return SHEAR_OK;
}

// check_call's result for an empty call (batch == 0 where allowed): the entry point returns
// SHEAR_OK without launching or reading anything else
constexpr int EMPTY_CALL = 1;

int check_call(shear_system* s, const void* a, const void* b, int batch, bool allow_empty = false) {
    if (!s) return fail(SHEAR_E_INVALID, "system is NULL");
    if (batch == 0 && allow_empty) return EMPTY_CALL;
    if (!a || !b) return fail(SHEAR_E_INVALID, "input or output pointer is NULL");
    if (batch <= 0) return fail(SHEAR_E_INVALID, "batch must be positive");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != s->device)
        return fail(SHEAR_E_DEVICE, "current device " + std::to_string(dev) + " is not the system's device " +
                                        std::to_string(s->device));
    return SHEAR_OK;
}

int prepare_ws(shear_system* s, int batch, int& chunk) {
    chunk = chunk_images(s, batch);
    if (chunk < 1)
        return fail(SHEAR_E_NOMEM, "workspace cap of " + std::to_string(s->ws_cap) + " bytes is below the " +
                                       std::to_string(ws_needed(s, batch, 1)) + " bytes one image needs");
    return ensure_ws(s, ws_needed(s, batch, chunk));
}

hipError_t take_event(shear_system* s, hipEvent_t& e) {
    if (!s->ev_free.empty()) {
        e = s->ev_free.back();
        s->ev_free.pop_back();
        return hipSuccess;
    }
    // timing-only events: no system-scope fence (cache write-back and invalidate) when recorded, so
    // that bracketing a launch does not slow the launches around it
    return hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
}

// Runs one launch; with profiling on, brackets it with two events on the same stream.
template <typename F>
hipError_t timed(shear_system* s, int kind, hipStream_t st, F&& launch) {
    if (!s->prof_on) return launch();
    hipEvent_t a, b;
    hipError_t e = take_event(s, a);
    if (e != hipSuccess) return e;
    if ((e = take_event(s, b)) != hipSuccess) return e;
    if ((e = hipEventRecord(a, st)) != hipSuccess) return e;
    if ((e = launch()) != hipSuccess) return e;
    if ((e = hipEventRecord(b, st)) != hipSuccess) return e;
    s->prof.push_back({kind, a, b});
    return hipSuccess;
}

int inverse_like(shear_system* s, const float* coeffs, float* x, int batch, void* stream, const void* filt) {
    int rc = check_call(s, coeffs, x, batch, true);
    if (rc == EMPTY_CALL) return SHEAR_OK;
    if (rc != SHEAR_OK) return rc;
    int chunk = 0;
    if ((rc = prepare_ws(s, batch, chunk)) != SHEAR_OK) return rc;
    const shear::DevPlan& d = s->plan;
    hipStream_t st = (hipStream_t)stream;
    const size_t pb = plane_bytes(s) / sizeof(float2);
    float2* V = (float2*)s->ws;
    float2* U = V + (size_t)batch * pb;
    const size_t img = (size_t)d.N * d.M;
    for (int b0 = 0; b0 < batch; b0 += chunk) {
        const int nb = std::min(chunk, batch - b0);
        hipError_t e = timed(s, SHEAR_KERNEL_ROWS_R2C_COEFFS, st, [&] {
            return shear::launch_rows_r2c(d, coeffs + (size_t)b0 * d.K * img, U, nb * d.K, true, st);
        });
        if (e != hipSuccess) return hip_fail(e, "row r2c launch");
        e = timed(s, SHEAR_KERNEL_COLS_INV, st, [&] {
            return shear::launch_cols_inv(d, U, V + (size_t)b0 * pb, nb, filt, part_ptr(s, batch, chunk), st);
        });
        if (e != hipSuccess) return hip_fail(e, "column pass launch");
    }
    hipError_t e = timed(s, SHEAR_KERNEL_ROWS_C2R_IMAGES, st,
                         [&] { return shear::launch_rows_c2r(d, V, x, batch, 1.0f, false, st); });
    if (e != hipSuccess) return hip_fail(e, "row c2r launch");
    return SHEAR_OK;
}

}  // namespace

extern "C" {

const char* shear_strerror(int code) {
    switch (code) {
        case SHEAR_OK: return "ok";
        case SHEAR_E_INVALID: return "invalid argument";
        case SHEAR_E_SIZE: return "unsupported size";
        case SHEAR_E_FRAME: return "not a usable frame (zero dual-frame weight or non-Hermitian spectra)";
        case SHEAR_E_NOMEM: return "out of memory";
        case SHEAR_E_HIP: return "HIP error";
        case SHEAR_E_DEVICE: return "wrong device";
    }
    return "unknown error";
}

const char* shear_last_error(void) { return g_err.c_str(); }

int shear_design_spectra(const shear_build_params* p, int* K, double* spectra_centred, int* idx) {
    try {
        if (!K) return fail(SHEAR_E_INVALID, "K is NULL");
        std::string why;
        if (!spectra_centred && !idx) {
            int rc = shear::count_filters(p, *K, why);
            return rc == SHEAR_OK ? SHEAR_OK : fail(rc, why);
        }
        shear::Design d;
        int rc = shear::design(p, d, why);
        if (rc != SHEAR_OK) return fail(rc, why);
        *K = d.K;
        if (spectra_centred)
            for (int k = 0; k < d.K; ++k)
                natural_to_centred(d.spectra.data() + (size_t)k * d.rows * d.cols, d.rows, d.cols,
                                   spectra_centred + (size_t)k * d.rows * d.cols * 2, nullptr);
        if (idx) std::memcpy(idx, d.idx.data(), sizeof(int) * d.idx.size());
        return SHEAR_OK;
    } catch (const std::bad_alloc&) {
        return fail(SHEAR_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(SHEAR_E_INVALID, "unexpected failure in shear_design_spectra");
    }
}

int shear_build_system(const shear_build_params* p, shear_system** out) {
    shear_system* s = nullptr;
    try {
        if (!p) return fail(SHEAR_E_INVALID, "params is NULL");
        int rc = new_system(p->rows, p->cols, p->max_workspace_bytes, out, s);
        if (rc != SHEAR_OK) return rc;
        shear::Design d;
        std::string why;
        rc = shear::design(p, d, why);
        if (rc != SHEAR_OK) {
            release(s);
            return fail(rc, why);
        }
        s->K = d.K;
        s->real = d.real;
        s->spectra = std::move(d.spectra);
        s->idx = std::move(d.idx);
        rc = finish_system(s, why);
        if (rc != SHEAR_OK) {
            release(s);
            return fail(rc, why);
        }
        *out = s;
        return SHEAR_OK;
    } catch (const std::bad_alloc&) {
        release(s);
        return fail(SHEAR_E_NOMEM, "host allocation failed");
    } catch (...) {
        release(s);
        return fail(SHEAR_E_INVALID, "unexpected failure in shear_build_system");
    }
}

int shear_system_from_spectra(int rows, int cols, int K, const double* spectra_centred, const int* idx,
                              size_t max_workspace_bytes, shear_system** out) {
    shear_system* s = nullptr;
    try {
        if (!spectra_centred) return fail(SHEAR_E_INVALID, "spectra is NULL");
        if (K <= 0) return fail(SHEAR_E_INVALID, "K must be positive");
        int rc = new_system(rows, cols, max_workspace_bytes, out, s);
        if (rc != SHEAR_OK) return rc;
        s->K = K;
        centred_to_natural_spectra(spectra_centred, K, rows, cols, s->spectra);
        const size_t NM = (size_t)rows * cols;
        double amax = 0.0, herm = 0.0, imax = 0.0;
        for (int k = 0; k < K; ++k) {
            const cd* P = s->spectra.data() + (size_t)k * NM;
            for (int r = 0; r < rows; ++r)
                for (int c = 0; c < cols; ++c) {
                    const cd v = P[(size_t)r * cols + c];
                    const cd m = P[(size_t)((rows - r) % rows) * cols + (size_t)((cols - c) % cols)];
                    amax = std::max(amax, std::abs(v));
                    imax = std::max(imax, std::fabs(v.imag()));
                    herm = std::max(herm, std::abs(v - std::conj(m)));
                }
        }
        if (herm > 1e-9 * amax) {
            release(s);
            return fail(SHEAR_E_FRAME, "spectra are not Hermitian (coefficients would not be real): deviation " +
                                           std::to_string(herm) + " vs max " + std::to_string(amax));
        }
        s->real = imax <= 1e-12 * amax;
        if (s->real)
            for (cd& v : s->spectra) v = cd(v.real(), 0.0);
        s->idx.assign((size_t)K * 3, 0);
        for (int k = 0; k < K; ++k) {
            if (idx) {
                for (int j = 0; j < 3; ++j) s->idx[(size_t)k * 3 + j] = idx[(size_t)k * 3 + j];
            } else {
                s->idx[(size_t)k * 3 + 2] = k;
            }
        }
        std::string why;
        rc = finish_system(s, why);
        if (rc != SHEAR_OK) {
            release(s);
            return fail(rc, why);
        }
        *out = s;
        return SHEAR_OK;
    } catch (const std::bad_alloc&) {
        release(s);
        return fail(SHEAR_E_NOMEM, "host allocation failed");
    } catch (...) {
        release(s);
        return fail(SHEAR_E_INVALID, "unexpected failure in shear_system_from_spectra");
    }
}

int shear_system_info(const shear_system* s, int* K, int* rows, int* cols, double* rms, int* idx) {
    if (!s) return fail(SHEAR_E_INVALID, "system is NULL");
    if (K) *K = s->K;
    if (rows) *rows = s->rows;
    if (cols) *cols = s->cols;
    if (rms) std::memcpy(rms, s->rms.data(), sizeof(double) * s->rms.size());
    if (idx) std::memcpy(idx, s->idx.data(), sizeof(int) * s->idx.size());
    return SHEAR_OK;
}

int shear_export_spectra(const shear_system* s, double* spectra_centred, double* W_centred) {
    if (!s) return fail(SHEAR_E_INVALID, "system is NULL");
    const size_t NM = (size_t)s->rows * s->cols;
    if (spectra_centred)
        for (int k = 0; k < s->K; ++k)
            natural_to_centred(s->spectra.data() + (size_t)k * NM, s->rows, s->cols, spectra_centred + (size_t)k * NM * 2,
                               nullptr);
    if (W_centred) {
        std::vector<cd> w(s->W.begin(), s->W.end());
        natural_to_centred(w.data(), s->rows, s->cols, nullptr, W_centred);
    }
    return SHEAR_OK;
}

int shear_workspace_bytes(const shear_system* s, int batch, size_t* bytes) {
    if (!s || !bytes) return fail(SHEAR_E_INVALID, "NULL argument");
    if (batch <= 0) return fail(SHEAR_E_INVALID, "batch must be positive");
    size_t need = 0;
    const int chunk = chunk_images(s, batch);
    if (chunk < 1) return fail(SHEAR_E_NOMEM, "workspace cap too small for one image");
    need = ws_needed(s, batch, chunk);
    *bytes = need;
    return SHEAR_OK;
}

int shear_reserve(shear_system* s, int batch) {
    size_t need = 0;
    int rc = shear_workspace_bytes(s, batch, &need);
    if (rc != SHEAR_OK) return rc;
    return ensure_ws(s, need);
}

int shear_forward(shear_system* s, const float* x, float* coeffs, int batch, void* stream) {
    int rc = check_call(s, x, coeffs, batch, true);
    if (rc == EMPTY_CALL) return SHEAR_OK;
    if (rc != SHEAR_OK) return rc;
    int chunk = 0;
    if ((rc = prepare_ws(s, batch, chunk)) != SHEAR_OK) return rc;
    const shear::DevPlan& d = s->plan;
    hipStream_t st = (hipStream_t)stream;
    const size_t pb = plane_bytes(s) / sizeof(float2);
    float2* A = (float2*)s->ws;
    float2* T = A + (size_t)batch * pb;
    const size_t img = (size_t)d.N * d.M;
    hipError_t e = timed(s, SHEAR_KERNEL_ROWS_R2C_IMAGES, st,
                         [&] { return shear::launch_rows_r2c(d, x, A, batch, false, st); });
    if (e != hipSuccess) return hip_fail(e, "row r2c launch");
    const float scale = (float)(1.0 / (double)img);  // 1/(N M): a power of two, exact
    const bool plane = d.plane_fwd && shear::plane_fwd_supported(d);
    for (int b0 = 0; b0 < batch; b0 += chunk) {
        const int nb = std::min(chunk, batch - b0);
        if (plane) {
            // the chunk's column spectra (nb planes) take the room of its K nb exchange planes
            e = timed(s, SHEAR_KERNEL_COLS_FWD, st,
                      [&] { return shear::launch_cols_spec(d, A + (size_t)b0 * pb, T, nb, scale, st); });
            if (e != hipSuccess) return hip_fail(e, "column spectra launch");
            e = timed(s, SHEAR_KERNEL_PLANE_FWD, st, [&] {
                return shear::launch_plane_fwd(d, T, coeffs + (size_t)b0 * d.K * img, nb, s->filt_plane, st);
            });
            if (e != hipSuccess) return hip_fail(e, "whole-plane forward launch");
            continue;
        }
        e = timed(s, SHEAR_KERNEL_COLS_FWD, st,
                  [&] { return shear::launch_cols_fwd(d, A + (size_t)b0 * pb, T, nb, s->filt_fwd, scale, st); });
        if (e != hipSuccess) return hip_fail(e, "column pass launch");
        e = timed(s, SHEAR_KERNEL_ROWS_C2R_COEFFS, st, [&] {
            return shear::launch_rows_c2r(d, T, coeffs + (size_t)b0 * d.K * img, nb * d.K, 1.0f, true, st);
        });
        if (e != hipSuccess) return hip_fail(e, "row c2r launch");
    }
    return SHEAR_OK;
}

int shear_forward_noalloc(shear_system* s, const float* x, float* coeffs, int batch, void* stream) {
    int rc = check_call(s, x, coeffs, batch, true);
    if (rc == EMPTY_CALL) return SHEAR_OK;
    if (rc != SHEAR_OK) return rc;
    const shear::DevPlan& d = s->plan;
    const size_t pb = plane_bytes(s);
    const size_t per_image = (size_t)(d.K + 1) * pb;  // row spectra of the image + its K exchange planes
    if (per_image > shear::kStaticScratchBytes)
        return fail(SHEAR_E_SIZE, "shear_forward_noalloc: one image needs " + std::to_string(per_image) +
                                      " bytes of scratch (K + 1 planes of " + std::to_string(pb) +
                                      " bytes), the fixed scratch holds " +
                                      std::to_string(shear::kStaticScratchBytes));
    void* base = nullptr;
    hipError_t e = shear::static_scratch(&base);
    if (e != hipSuccess) return hip_fail(e, "locating the fixed scratch");
    hipStream_t st = (hipStream_t)stream;
    const int chunk = (int)std::min<size_t>((size_t)batch, shear::kStaticScratchBytes / per_image);
    const size_t img = (size_t)d.N * d.M;
    const float scale = (float)(1.0 / (double)img);  // 1/(N M): a power of two, exact
    for (int b0 = 0; b0 < batch; b0 += chunk) {
        const int nb = std::min(chunk, batch - b0);
        float2* A = (float2*)base;
        float2* T = (float2*)((char*)base + (size_t)nb * pb);
        e = shear::launch_rows_r2c(d, x + (size_t)b0 * img, A, nb, false, st);
        if (e != hipSuccess) return hip_fail(e, "row r2c launch");
        e = shear::launch_cols_fwd(d, A, T, nb, s->filt_fwd, scale, st);
        if (e != hipSuccess) return hip_fail(e, "column pass launch");
        e = shear::launch_rows_c2r(d, T, coeffs + (size_t)b0 * d.K * img, nb * d.K, 1.0f, true, st);
        if (e != hipSuccess) return hip_fail(e, "row c2r launch");
    }
    return SHEAR_OK;
}

int shear_inverse(shear_system* s, const float* coeffs, float* x, int batch, void* stream) {
    return inverse_like(s, coeffs, x, batch, stream, s ? s->filt_inv : nullptr);
}

int shear_adjoint(shear_system* s, const float* coeffs, float* x, int batch, void* stream) {
    return inverse_like(s, coeffs, x, batch, stream, s ? s->filt_adj : nullptr);
}

int shear_denoise_thresholds(const shear_system* s, const double* sigma, int batch, const double* factors,
                             int n_factors, float* out) {
    if (!s || !sigma || !out) return fail(SHEAR_E_INVALID, "NULL argument");
    if (batch < 0) return fail(SHEAR_E_INVALID, "batch must not be negative");
    int J = 0;
    for (int k = 0; k < s->K; ++k) J = std::max(J, s->idx[(size_t)k * 3 + 1]);
    if (J < 1) return fail(SHEAR_E_INVALID, "the system's index triples name no scale");
    std::vector<double> f((size_t)J, 2.5);
    f[(size_t)J - 1] = 3.8;  // the paper's K_j: 2.5 on every scale but the finest
    if (factors) {
        if (n_factors != J)
            return fail(SHEAR_E_INVALID, "need " + std::to_string(J) + " scale factors, got " + std::to_string(n_factors));
        f.assign(factors, factors + J);
    }
    for (int b = 0; b < batch; ++b)
        for (int k = 0; k < s->K; ++k) {
            const int j = std::max(1, s->idx[(size_t)k * 3 + 1]);  // the low-pass (scale 0) takes K_1
            out[(size_t)b * s->K + k] = (float)(f[(size_t)j - 1] * sigma[b] * s->rms[(size_t)k]);
        }
    return SHEAR_OK;
}

int shear_inpaint_thresholds(const shear_system* s, const double* deltas, int iterations, int batch, float* out) {
    if (!s || !deltas || !out) return fail(SHEAR_E_INVALID, "NULL argument");
    if (iterations < 1 || batch < 0) return fail(SHEAR_E_INVALID, "iterations must be positive, batch not negative");
    for (int i = 0; i < iterations; ++i)
        for (int b = 0; b < batch; ++b)
            for (int k = 0; k < s->K; ++k)
                out[((size_t)i * batch + b) * s->K + k] = (float)(deltas[(size_t)i * batch + b] * s->rms[(size_t)k]);
    return SHEAR_OK;
}

int shear_delta_schedule(int kind, double delta_init, double delta_min, int iterations, double* out) {
    if (!out) return fail(SHEAR_E_INVALID, "out is NULL");
    if (iterations < 1) return fail(SHEAR_E_INVALID, "iterations must be positive");
    if (kind == SHEAR_DECAY_GEOMETRIC) {
        if (!(delta_init > 0.0) || !(delta_min > 0.0))
            return fail(SHEAR_E_INVALID, "the geometric decay needs delta_init > 0 and delta_min > 0");
        const double lam = iterations > 1 ? std::pow(delta_min / delta_init, 1.0 / (iterations - 1)) : 1.0;
        double d = delta_init;
        for (int i = 0; i < iterations; ++i) {
            out[i] = d;
            d *= lam;
        }
        return SHEAR_OK;
    }
    if (kind == SHEAR_DECAY_LINEAR) {
        for (int i = 0; i < iterations; ++i)
            out[i] = iterations > 1 ? delta_init * (1.0 - (double)i / (double)(iterations - 1)) : delta_init;
        return SHEAR_OK;
    }
    return fail(SHEAR_E_INVALID, "unknown decay kind " + std::to_string(kind));
}

int shear_denoise(shear_system* s, const float* x, float* y, int batch, const float* thresholds, unsigned* kept,
                  void* stream) {
    int rc = check_call(s, x, y, batch, true);
    if (rc == EMPTY_CALL) return SHEAR_OK;
    if (rc != SHEAR_OK) return rc;
    if (!thresholds) return fail(SHEAR_E_INVALID, "thresholds pointer is NULL");
    int chunk = 0;
    if ((rc = prepare_ws(s, batch, chunk)) != SHEAR_OK) return rc;
    const shear::DevPlan& d = s->plan;
    hipStream_t st = (hipStream_t)stream;
    const size_t pb = plane_bytes(s) / sizeof(float2);
    float2* A = (float2*)s->ws;  // row spectra of the images, then (image by image) the summed spectra
    float2* T = A + (size_t)batch * pb;
    const size_t img = (size_t)d.N * d.M;
    hipError_t e;
    if (kept) {
        e = shear::launch_zero_u32(kept, batch * d.K, st);
        if (e != hipSuccess) return hip_fail(e, "kept-count reset launch");
    }
    e = timed(s, SHEAR_KERNEL_ROWS_R2C_IMAGES, st, [&] { return shear::launch_rows_r2c(d, x, A, batch, false, st); });
    if (e != hipSuccess) return hip_fail(e, "row r2c launch");
    const float scale = (float)(1.0 / (double)img);  // 1/(N M): a power of two, exact
    for (int b0 = 0; b0 < batch; b0 += chunk) {
        const int nb = std::min(chunk, batch - b0);
        e = timed(s, SHEAR_KERNEL_COLS_FWD, st,
                  [&] { return shear::launch_cols_fwd(d, A + (size_t)b0 * pb, T, nb, s->filt_fwd, scale, st); });
        if (e != hipSuccess) return hip_fail(e, "column pass launch");
        e = timed(s, SHEAR_KERNEL_ROWS_THRESH, st, [&] {
            return shear::launch_rows_thresh(d, T, nb * d.K, thresholds + (size_t)b0 * d.K,
                                             kept ? kept + (size_t)b0 * d.K : nullptr, st);
        });
        if (e != hipSuccess) return hip_fail(e, "row threshold launch");
        // the images of this chunk no longer need their row spectra: the sums replace them
        e = timed(s, SHEAR_KERNEL_COLS_INV, st, [&] {
            return shear::launch_cols_inv(d, T, A + (size_t)b0 * pb, nb, s->filt_inv, part_ptr(s, batch, chunk), st);
        });
        if (e != hipSuccess) return hip_fail(e, "column pass launch");
    }
    e = timed(s, SHEAR_KERNEL_ROWS_C2R_IMAGES, st, [&] { return shear::launch_rows_c2r(d, A, y, batch, 1.0f, false, st); });
    if (e != hipSuccess) return hip_fail(e, "row c2r launch");
    return SHEAR_OK;
}

namespace {

// The launches of `iterations` inpainting iterations (Algorithm 3) on stream st.
hipError_t enqueue_inpaint(shear_system* s, const float* fm, const float* mask, float* f, int batch,
                           const float* thresholds, int iterations, int chunk, hipStream_t st) {
    const shear::DevPlan& d = s->plan;
    const size_t pb = plane_bytes(s) / sizeof(float2);
    float2* A = (float2*)s->ws;
    float2* T = A + (size_t)batch * pb;
    const size_t img = (size_t)d.N * d.M;
    const float scale = (float)(1.0 / (double)img);
    // f_inpainted := 0 (a fill kernel, so that the sequence can be captured)
    hipError_t e = shear::launch_zero_u32(reinterpret_cast<unsigned*>(f), (int)(batch * img), st);
    if (e != hipSuccess) return e;
    for (int it = 0; it < iterations; ++it) {
        e = timed(s, SHEAR_KERNEL_ROWS_R2C_IMAGES, st,
                  [&] { return shear::launch_rows_r2c_mix(d, fm, mask, f, A, batch, st); });
        if (e != hipSuccess) return e;
        const float* thr = thresholds + (size_t)it * batch * d.K;
        for (int b0 = 0; b0 < batch; b0 += chunk) {
            const int nb = std::min(chunk, batch - b0);
            e = timed(s, SHEAR_KERNEL_COLS_FWD, st,
                      [&] { return shear::launch_cols_fwd(d, A + (size_t)b0 * pb, T, nb, s->filt_fwd, scale, st); });
            if (e != hipSuccess) return e;
            e = timed(s, SHEAR_KERNEL_ROWS_THRESH, st, [&] {
                return shear::launch_rows_thresh(d, T, nb * d.K, thr + (size_t)b0 * d.K, nullptr, st);
            });
            if (e != hipSuccess) return e;
            e = timed(s, SHEAR_KERNEL_COLS_INV, st, [&] {
                return shear::launch_cols_inv(d, T, A + (size_t)b0 * pb, nb, s->filt_inv, part_ptr(s, batch, chunk), st);
            });
            if (e != hipSuccess) return e;
        }
        e = timed(s, SHEAR_KERNEL_ROWS_C2R_IMAGES, st,
                  [&] { return shear::launch_rows_c2r(d, A, f, batch, 1.0f, false, st); });
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

void drop_graph(shear_system* s) {
    if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    s->gexec = nullptr;
    s->graph = nullptr;
    s->graph_key.clear();
}

}  // namespace

int shear_inpaint(shear_system* s, const float* f_masked, const float* mask, float* f, int batch,
                  const float* thresholds, int iterations, void* stream) {
    int rc = check_call(s, f_masked, f, batch, true);
    if (rc == EMPTY_CALL) return SHEAR_OK;
    if (rc != SHEAR_OK) return rc;
    if (!mask || !thresholds) return fail(SHEAR_E_INVALID, "mask or thresholds pointer is NULL");
    if (iterations < 1) return fail(SHEAR_E_INVALID, "iterations must be positive");
    int chunk = 0;
    if ((rc = prepare_ws(s, batch, chunk)) != SHEAR_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    if (s->prof_on) {
        // per-launch timing needs the launches themselves
        e = enqueue_inpaint(s, f_masked, mask, f, batch, thresholds, iterations, chunk, st);
        return e == hipSuccess ? SHEAR_OK : hip_fail(e, "inpainting launch");
    }
    const std::vector<const void*> key = {f_masked, mask, f, thresholds, s->ws, (const void*)(intptr_t)batch,
                                          (const void*)(intptr_t)iterations, (const void*)(intptr_t)chunk};
    if (!s->gexec || key != s->graph_key) {
        drop_graph(s);
        if (!s->cap_stream && (e = hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking)) != hipSuccess)
            return hip_fail(e, "hipStreamCreateWithFlags");
        if ((e = hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeRelaxed)) != hipSuccess)
            return hip_fail(e, "hipStreamBeginCapture");
        const hipError_t el = enqueue_inpaint(s, f_masked, mask, f, batch, thresholds, iterations, chunk, s->cap_stream);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(s->cap_stream, &g);
        if (el != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return hip_fail(el, "inpainting launch under capture");
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        s->graph = g;
        if ((e = hipGraphInstantiate(&s->gexec, g, nullptr, nullptr, 0)) != hipSuccess) {
            drop_graph(s);
            return hip_fail(e, "hipGraphInstantiate");
        }
        s->graph_key = key;
    }
    if ((e = hipGraphLaunch(s->gexec, st)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return SHEAR_OK;
}

namespace {

void drop_group_graph(shear_system* s) {
    if (s->ggexec) (void)hipGraphExecDestroy(s->ggexec);
    if (s->ggraph) (void)hipGraphDestroy(s->ggraph);
    s->ggexec = nullptr;
    s->ggraph = nullptr;
    s->ggraph_key.clear();
}

// What a captured group sequence depends on, per group: the system, its filter bank, workspace and
// schedule, and the call's pointers and batch.
void group_key(shear_system* const* sys, int n, const float* const* fm, const float* const* mask, float* const* f,
               const int* batch, const float* const* thr, int iterations, const int* chunk,
               std::vector<const void*>& key) {
    auto v = [](long long x) { return (const void*)(intptr_t)x; };
    key.assign({v(n), v(iterations)});
    for (int g = 0; g < n; ++g) {
        const shear_system* s = sys[g];
        const shear::DevPlan& d = s->plan;
        key.insert(key.end(), {(const void*)s, s->dev_block, s->ws, v((long long)s->ws_bytes), v(s->rows), v(s->cols),
                               v(s->K), v(d.pw_fwd), v(d.pw_inv), v(d.kg_fwd), v(d.kg_inv), v(d.pc_fwd), v(d.pc_inv),
                               fm[g], mask[g], f[g], thr[g], v(batch[g]), v(chunk[g])});
    }
}

}  // namespace

int shear_inpaint_groups(shear_system* const* systems, int n_groups, const float* const* f_masked,
                         const float* const* mask, float* const* f, const int* batch, const float* const* thresholds,
                         int iterations, void* stream) {
    if (!systems || n_groups < 1 || !f_masked || !mask || !f || !batch || !thresholds)
        return fail(SHEAR_E_INVALID, "NULL array or no group");
    if (iterations < 1) return fail(SHEAR_E_INVALID, "iterations must be positive");
    std::vector<int> chunk((size_t)n_groups, 0);
    for (int g = 0; g < n_groups; ++g) {
        for (int h = 0; h < g; ++h)
            if (systems[h] == systems[g]) return fail(SHEAR_E_INVALID, "a system appears in two groups");
        int rc = check_call(systems[g], f_masked[g], f[g], batch[g]);
        if (rc != SHEAR_OK) return rc;
        if (!mask[g] || !thresholds[g]) return fail(SHEAR_E_INVALID, "mask or thresholds pointer is NULL");
        if ((rc = prepare_ws(systems[g], batch[g], chunk[(size_t)g])) != SHEAR_OK) return rc;
    }
    shear_system* lead = systems[0];
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    bool prof = false;
    for (int g = 0; g < n_groups; ++g) prof = prof || systems[g]->prof_on;
    if (prof) {
        // per-launch timing needs the launches themselves: the groups one after another
        for (int g = 0; g < n_groups; ++g) {
            e = enqueue_inpaint(systems[g], f_masked[g], mask[g], f[g], batch[g], thresholds[g], iterations,
                                chunk[(size_t)g], st);
            if (e != hipSuccess) return hip_fail(e, "inpainting launch");
        }
        return SHEAR_OK;
    }
    std::vector<const void*> key;
    group_key(systems, n_groups, f_masked, mask, f, batch, thresholds, iterations, chunk.data(), key);
    if (!lead->ggexec || key != lead->ggraph_key) {
        drop_group_graph(lead);
        for (int g = 0; g < n_groups; ++g)
            if (!systems[g]->cap_stream &&
                (e = hipStreamCreateWithFlags(&systems[g]->cap_stream, hipStreamNonBlocking)) != hipSuccess)
                return hip_fail(e, "hipStreamCreateWithFlags");
        std::vector<hipEvent_t> ev((size_t)n_groups, nullptr);  // [0] forks, [g > 0] joins
        for (auto& x : ev)
            if ((e = hipEventCreateWithFlags(&x, hipEventDisableTiming)) != hipSuccess) {
                for (auto y : ev)
                    if (y) (void)hipEventDestroy(y);
                return hip_fail(e, "hipEventCreate");
            }
        hipStream_t origin = lead->cap_stream;
        hipError_t el = hipStreamBeginCapture(origin, hipStreamCaptureModeRelaxed);
        if (el == hipSuccess) el = hipEventRecord(ev[0], origin);
        // group 0 on the origin stream, every other group on a branch forked from it and joined back
        for (int g = 1; g < n_groups && el == hipSuccess; ++g) {
            hipStream_t bs = systems[g]->cap_stream;
            if ((el = hipStreamWaitEvent(bs, ev[0], 0)) != hipSuccess) break;
            if ((el = enqueue_inpaint(systems[g], f_masked[g], mask[g], f[g], batch[g], thresholds[g], iterations,
                                      chunk[(size_t)g], bs)) != hipSuccess)
                break;
            if ((el = hipEventRecord(ev[(size_t)g], bs)) != hipSuccess) break;
        }
        if (el == hipSuccess)
            el = enqueue_inpaint(lead, f_masked[0], mask[0], f[0], batch[0], thresholds[0], iterations, chunk[0], origin);
        for (int g = 1; g < n_groups && el == hipSuccess; ++g) el = hipStreamWaitEvent(origin, ev[(size_t)g], 0);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(origin, &graph);
        for (auto y : ev) (void)hipEventDestroy(y);
        if (el != hipSuccess || e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return hip_fail(el != hipSuccess ? el : e, "capturing the grouped inpainting sequence");
        }
        lead->ggraph = graph;
        if ((e = hipGraphInstantiate(&lead->ggexec, graph, nullptr, nullptr, 0)) != hipSuccess) {
            drop_group_graph(lead);
            return hip_fail(e, "hipGraphInstantiate");
        }
        lead->ggraph_key = key;
    }
    if ((e = hipGraphLaunch(lead->ggexec, st)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return SHEAR_OK;
}

int shear_set_schedule(shear_system* s, int pw_fwd, int pw_inv, int kg_fwd, int kg_inv, int pc_fwd, int pc_inv) {
    if (!s) return fail(SHEAR_E_INVALID, "system is NULL");
    const int L = s->cols / 2;
    // pw_fwd == L: the whole plane per workgroup, where that forward is compiled
    const bool plane = shear::plane_fwd_supported(s->plan) && pw_fwd == L;
    for (int pw : {pw_fwd, pw_inv}) {
        if (pw == pw_fwd && plane) continue;
        if (pw != 0 && pw != 8 && pw != 16) return fail(SHEAR_E_INVALID, "panel width must be 0, 8 or 16");
        if (pw == 16 && L < 16) return fail(SHEAR_E_INVALID, "panel width 16 needs cols >= 32");
    }
    for (int kg : {kg_fwd, kg_inv})
        if (kg < 0 || kg > s->K) return fail(SHEAR_E_INVALID, "filter groups must be in [0, K]");
    const int pdef = shear::col_points_default(s->rows), palt = shear::col_points_alternative(s->rows);
    for (int pc : {pc_fwd, pc_inv})
        if (pc != 0 && pc != pdef && pc != palt)
            return fail(SHEAR_E_INVALID, "points per thread of the " + std::to_string(s->rows) + "-point column FFTs must be 0, " +
                                             std::to_string(pdef) + (palt ? " or " + std::to_string(palt) : std::string()));
    if (plane)
        s->plan.plane_fwd = true;
    else if (pw_fwd) {
        s->plan.pw_fwd = pw_fwd;
        s->plan.plane_fwd = false;
    }
    if (pw_inv) s->plan.pw_inv = pw_inv;
    if (kg_fwd) s->plan.kg_fwd = kg_fwd;
    if (kg_inv) s->plan.kg_inv = kg_inv;
    if (pc_fwd) s->plan.pc_fwd = pc_fwd;
    if (pc_inv) s->plan.pc_inv = pc_inv;
    drop_graph(s);  // a captured inpainting sequence holds the old schedule and workspace layout
    return SHEAR_OK;
}

int shear_autotune(shear_system* s, int batch, int* pw_fwd, int* pw_inv, int* kg_fwd, int* kg_inv, int* pc_fwd,
                   int* pc_inv) {
    int rc = check_call(s, s, s, batch);
    if (rc != SHEAR_OK) return rc;
    std::vector<int> pws = {8};
    if (s->cols / 2 >= 16) pws.insert(pws.begin(), 16);
    // points per thread of the column FFTs (the radix sequence): the default, and the alternative where
    // there is one
    std::vector<int> pcs = {shear::col_points_default(s->rows)};
    if (shear::col_points_alternative(s->rows)) pcs.push_back(shear::col_points_alternative(s->rows));
    // filter splits: up to 8 groups in the inverse (each group adds a partial-sum plane per image);
    // the forward, which needs no partial sums, also tries 16 and 32 when the batch's panels alone
    // (at 8 columns) would leave the device's compute units idle
    std::vector<int> kgs, kgs_fwd;
    for (int kg : {1, 2, 4, 8})
        if (kg <= s->K) kgs.push_back(kg);
    kgs_fwd = kgs;
    if ((long long)batch * (s->cols / 2 / 8) < (long long)s->cus)
        for (int kg : {16, 32})
            if (kg <= s->K) kgs_fwd.push_back(kg);
    // the workspace and chunk of the largest filter split (its partial sums need the most room)
    const shear::DevPlan saved = s->plan;
    s->plan.kg_inv = kgs.back();
    int chunk = 0;
    rc = prepare_ws(s, batch, chunk);
    s->plan = saved;
    if (rc != SHEAR_OK) return rc;
    drop_graph(s);  // a captured inpainting sequence holds the old schedule
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    // Candidates are timed inside whole forward + inverse steps on temporary images and coefficients:
    // a column pass's time depends on what the launches around it leave in the caches (at 16 x
    // 512 x 512 x 49 a forward split of 8 measured 0.165-0.18 ms between the inverse's passes against
    // 0.14 ms unsplit, while alone the two were within 3 %).
    const size_t img = (size_t)s->rows * s->cols;
    float* xt = nullptr;
    float* ct = nullptr;
    if ((e = hipMalloc(&xt, 2 * (size_t)batch * img * sizeof(float))) != hipSuccess)
        return fail(SHEAR_E_NOMEM, std::string("autotune: image buffers: ") + hipGetErrorString(e));
    if ((e = hipMalloc(&ct, (size_t)batch * s->K * img * sizeof(float))) != hipSuccess) {
        (void)hipFree(xt);
        return fail(SHEAR_E_NOMEM, std::string("autotune: coefficient buffer: ") + hipGetErrorString(e));
    }
    float* yt = xt + (size_t)batch * img;
    // defined, non-zero images: each a copy of the first N x M values of the forward filter table
    // (which holds K N (M/2 + 1) values, at least N x M from K = 2 on), else zeros
    const size_t filt_vals = (size_t)s->K * (s->cols / 2 + 1) * s->rows * (s->plan.real ? 1 : 2);
    e = shear::launch_zero_u32((unsigned*)xt, (int)std::min<size_t>(2 * (size_t)batch * img, (size_t)1 << 30), nullptr);
    for (int b = 0; b < batch && e == hipSuccess && filt_vals >= img; ++b)
        e = hipMemcpyAsync(xt + (size_t)b * img, s->filt_fwd, img * sizeof(float), hipMemcpyDeviceToDevice, nullptr);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (e == hipSuccess && (e = hipEventCreateWithFlags(&e0, hipEventDisableSystemFence)) == hipSuccess)
        e = hipEventCreateWithFlags(&e1, hipEventDisableSystemFence);
    const bool prof = s->prof_on;
    s->prof_on = false;  // the steps' launches are not part of the per-launch record
    int call_rc = SHEAR_OK;
    // each candidate is timed once per round, rounds interleaved (drifts of the device's clocks and
    // interference hit every candidate alike), and keeps the median of its rounds
    constexpr int kRounds = 5;
    for (int dir = 0; dir < 2 && e == hipSuccess && call_rc == SHEAR_OK; ++dir) {
        struct Cand {
            int pw, kg, pc;
            bool plane;
        };
        std::vector<Cand> cand;
        for (int pw : pws)
            for (int kg : (dir == 0 ? kgs_fwd : kgs))
                for (int pc : pcs) cand.push_back({pw, kg, pc, false});
        // the whole-plane forward, where it is compiled (last in the list)
        if (dir == 0 && shear::plane_fwd_supported(s->plan))
            cand.push_back({s->plan.pw_fwd, s->plan.kg_fwd, s->plan.pc_fwd, true});
        std::vector<std::vector<float>> times(cand.size());
        for (int round = 0; round <= kRounds && e == hipSuccess && call_rc == SHEAR_OK; ++round) {  // round 0 warms up
            for (size_t ci = 0; ci < cand.size() && e == hipSuccess && call_rc == SHEAR_OK; ++ci) {
                const shear::DevPlan keep = s->plan;
                (dir == 0 ? s->plan.pw_fwd : s->plan.pw_inv) = cand[ci].pw;
                (dir == 0 ? s->plan.kg_fwd : s->plan.kg_inv) = cand[ci].kg;
                (dir == 0 ? s->plan.pc_fwd : s->plan.pc_inv) = cand[ci].pc;
                if (dir == 0) s->plan.plane_fwd = cand[ci].plane;
                if ((e = hipEventRecord(e0, nullptr)) == hipSuccess &&
                    (call_rc = shear_forward(s, xt, ct, batch, nullptr)) == SHEAR_OK &&
                    (call_rc = shear_inverse(s, ct, yt, batch, nullptr)) == SHEAR_OK &&
                    (e = hipEventRecord(e1, nullptr)) == hipSuccess)
                    e = hipEventSynchronize(e1);
                s->plan = keep;
                float ms = 0.0f;
                if (e == hipSuccess && call_rc == SHEAR_OK && (e = hipEventElapsedTime(&ms, e0, e1)) == hipSuccess &&
                    round > 0)
                    times[ci].push_back(ms);
            }
        }
        if (e != hipSuccess || call_rc != SHEAR_OK) break;
        // The panel schedule is picked among the panel candidates (the denoising and inpainting
        // column passes use it whichever forward is chosen); the whole-plane forward replaces it
        // in shear_forward where its median step is faster.
        size_t n_panel = cand.size();
        while (n_panel > 0 && cand[n_panel - 1].plane) --n_panel;
        std::vector<float> med(cand.size(), -1.0f);
        float best = -1.0f;
        for (size_t ci = 0; ci < cand.size(); ++ci) {
            std::vector<float> t = times[ci];
            if (t.empty()) continue;
            std::nth_element(t.begin(), t.begin() + t.size() / 2, t.end());
            med[ci] = t[t.size() / 2];
            if (ci < n_panel && (best < 0.0f || med[ci] < best)) best = med[ci];
        }
        // a filter split adds work (the forward repeats a panel's column FFT per group, the inverse
        // writes and adds partial sums), so it is taken only where it is measurably faster: among
        // the candidates within 1 % of the fastest step, the fewest groups, then the fastest
        size_t pick_i = 0;
        for (size_t ci = 0; ci < n_panel; ++ci) {
            if (med[ci] < 0.0f || med[ci] > 1.01f * best) continue;
            if (med[pick_i] < 0.0f || med[pick_i] > 1.01f * best || cand[ci].kg < cand[pick_i].kg ||
                (cand[ci].kg == cand[pick_i].kg && med[ci] < med[pick_i]))
                pick_i = ci;
        }
        (dir == 0 ? s->plan.pw_fwd : s->plan.pw_inv) = cand[pick_i].pw;
        (dir == 0 ? s->plan.kg_fwd : s->plan.kg_inv) = cand[pick_i].kg;
        (dir == 0 ? s->plan.pc_fwd : s->plan.pc_inv) = cand[pick_i].pc;
        if (dir == 0)
            s->plan.plane_fwd = n_panel < cand.size() && med[n_panel] >= 0.0f && med[n_panel] < med[pick_i];
    }
    s->prof_on = prof;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    hipError_t es = hipDeviceSynchronize();
    (void)hipFree(ct);
    (void)hipFree(xt);
    if (call_rc != SHEAR_OK) return call_rc;
    if (e != hipSuccess) return hip_fail(e, "autotune launch");
    if (es != hipSuccess) return hip_fail(es, "hipDeviceSynchronize after autotune");
    if (pw_fwd) *pw_fwd = s->plan.plane_fwd ? s->cols / 2 : s->plan.pw_fwd;
    if (pw_inv) *pw_inv = s->plan.pw_inv;
    if (kg_fwd) *kg_fwd = s->plan.kg_fwd;
    if (kg_inv) *kg_inv = s->plan.kg_inv;
    if (pc_fwd) *pc_fwd = s->plan.pc_fwd ? s->plan.pc_fwd : shear::col_points_default(s->rows);
    if (pc_inv) *pc_inv = s->plan.pc_inv ? s->plan.pc_inv : shear::col_points_default(s->rows);
    return SHEAR_OK;
}

int shear_shrink_params_bytes(int K, size_t* bytes) {
    if (!bytes || K < 1 || K > 64) return fail(SHEAR_E_INVALID, "K must be in [1, 64] and bytes non-NULL");
    *bytes = shear::shrink_layout(K).bytes;
    return SHEAR_OK;
}

int shear_shrink_pack(shear_system* s, const float* W1, const float* b1, const float* W2, const float* b2,
                      const float* W3, const float* b3, void* packed, void* stream) {
    if (!s) return fail(SHEAR_E_INVALID, "system is NULL");
    if (!W1 || !b1 || !W2 || !b2 || !W3 || !b3 || !packed) return fail(SHEAR_E_INVALID, "NULL parameter pointer");
    if (s->K > 64) return fail(SHEAR_E_SIZE, "learned shrinkage supports at most 64 filters");
    hipError_t e = shear::launch_shrink_pack(s->K, W1, b1, W2, b2, W3, b3, packed, (hipStream_t)stream);
    return e == hipSuccess ? SHEAR_OK : hip_fail(e, "parameter packing launch");
}

namespace {

int ensure_ws2(shear_system* s, size_t need) {
    if (need <= s->ws2_bytes) return SHEAR_OK;
    if (s->ws2) {
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize before workspace growth");
        (void)hipFree(s->ws2);
        s->ws2 = nullptr;
        s->ws2_bytes = 0;
    }
    hipError_t e = hipMalloc(&s->ws2, need);
    if (e != hipSuccess) {
        s->ws2 = nullptr;
        return fail(SHEAR_E_NOMEM, std::string("shrinkage workspace hipMalloc failed: ") + hipGetErrorString(e));
    }
    s->ws2_bytes = need;
    return SHEAR_OK;
}

size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

int shear_shrink_param_count(int K) { return (K >= 1 && K <= 64) ? 577 * K + 9280 : SHEAR_E_INVALID; }

int shear_shrink_train_step(shear_system* s, const float* c_noisy, const float* c_clean, int batch, const float* sigma,
                            float* params, float* grads, float* adam_state, void* packed, int step, float lr,
                            float temperature, float* loss, void* stream) {
    int rc = check_call(s, c_noisy, c_clean, batch);
    if (rc != SHEAR_OK) return rc;
    if (!sigma || !params || !grads || !adam_state || !packed || !loss)
        return fail(SHEAR_E_INVALID, "NULL pointer argument");
    if (step < 1 || !(temperature > 0.0f) || !(lr >= 0.0f))
        return fail(SHEAR_E_INVALID, "step must be >= 1, temperature > 0 and lr >= 0");
    if (!shear::shrink_supported(s->K, s->rows, s->cols))
        return fail(SHEAR_E_SIZE, "learned shrinkage needs K <= 64, rows % 8 == 0 and cols % 128 == 0");
    const int K = s->K, N = s->rows, M = s->cols;
    const int cpo = shear::shrink_cinp(K), c3 = shear::shrink_coutp(K);
    const size_t pix = (size_t)batch * N * M;
    const int ntiles = (int)(pix / (8 * 32));
    const int G = std::max(1, std::min(ntiles, 2 * std::max(1, s->cus)));
    const size_t part_stride = (size_t)std::max({32 * 9 * cpo + 32, c3 * 9 * 32 + c3, 32 * 9 * 32 + 32});
    // workspace: scale | h1 | h2 | d o | dh2 | dh1 | transposed W3 | transposed W2 | partials
    size_t off = 0;
    const size_t o_sc = off;
    off = al256(off + (size_t)batch * K * 4);
    const size_t o_h1 = off;
    off = al256(off + pix * 64);
    const size_t o_h2 = off;
    off = al256(off + pix * 64);
    const size_t o_do = off;
    off = al256(off + pix * cpo * 2);
    const size_t o_dh2 = off;
    off = al256(off + pix * 64);
    const size_t o_dh1 = off;
    off = al256(off + pix * 64);
    const size_t o_z = off;
    off = al256(off + pix * cpo * 2);
    const size_t o_t3 = off;
    off = al256(off + (size_t)32 * 9 * cpo * 2);
    const size_t o_t2 = off;
    off = al256(off + (size_t)32 * 9 * 32 * 2);
    const size_t o_part = off;
    off = al256(off + (size_t)G * part_stride * 4);
    if ((rc = ensure_ws2(s, off)) != SHEAR_OK) return rc;
    char* w = (char*)s->ws2;
    float* scale = (float*)(w + o_sc);
    unsigned short* h1 = (unsigned short*)(w + o_h1);
    unsigned short* h2 = (unsigned short*)(w + o_h2);
    unsigned short* dO = (unsigned short*)(w + o_do);
    unsigned short* dh2 = (unsigned short*)(w + o_dh2);
    unsigned short* dh1 = (unsigned short*)(w + o_dh1);
    unsigned short* zp = (unsigned short*)(w + o_z);
    unsigned short* t3 = (unsigned short*)(w + o_t3);
    unsigned short* t2 = (unsigned short*)(w + o_t2);
    float* part = (float*)(w + o_part);
    // parameters, natural order, flat: W1 [32][K][3][3], b1 [32], W2 [32][32][3][3], b2 [32], W3 [K][32][3][3], b3 [K]
    const size_t pW1 = 0, pb1 = 288 * (size_t)K, pW2 = pb1 + 32, pb2 = pW2 + 9216, pW3 = pb2 + 32, pb3 = pW3 + 288 * (size_t)K;
    const int np = shear_shrink_param_count(K);
    hipStream_t st = (hipStream_t)stream;
    const shear::ShrinkLayout L = shear::shrink_layout(K);
    const char* pk = (const char*)packed;
    hipError_t e;
    if ((e = shear::launch_zero_u32((unsigned*)loss, 1, st)) != hipSuccess) return hip_fail(e, "loss reset");
    if ((e = shear::launch_inv_scale(sigma, s->rms_dev, scale, batch, K, st)) != hipSuccess) return hip_fail(e, "scale");
    if ((e = shear::launch_pack_z(c_noisy, scale, zp, K, N, M, batch, st)) != hipSuccess) return hip_fail(e, "z packing");
    // forward: h1, h2 (as in inference), then the loss epilogue of the last layer
    shear::ConvArgs a{};
    a.N = N;
    a.M = M;
    a.scale = scale;
    a.lowpass = K - 1;
    a.cus = s->cus;
    a.in = zp;
    a.W = (const unsigned short*)(pk + L.w1);
    a.bias = (const float*)(pk + L.b1);
    a.out_bf = h1;
    a.cin = K;
    a.cout = 32;
    if ((e = shear::launch_conv(0, K, a, batch, st)) != hipSuccess) return hip_fail(e, "layer 1");
    a.in = h1;
    a.W = (const unsigned short*)(pk + L.w2);
    a.bias = (const float*)(pk + L.b2);
    a.out_bf = h2;
    a.cin = 32;
    if ((e = shear::launch_conv(1, K, a, batch, st)) != hipSuccess) return hip_fail(e, "layer 2");
    a.in = h2;
    a.W = (const unsigned short*)(pk + L.w3);
    a.bias = (const float*)(pk + L.b3);
    a.out_bf = dO;
    a.coef = c_noisy;
    a.coef2 = c_clean;
    a.loss = loss;
    a.loss_scale = (float)(1.0 / ((double)batch * (K - 1 > 0 ? K - 1 : 1) * N * M));
    a.temperature = temperature;
    a.cout = K;
    if ((e = shear::launch_conv(3, K, a, batch, st)) != hipSuccess) return hip_fail(e, "layer 3 (loss)");
    // backward: dW3, dh2, dW2, dh1, dW1
    shear::WgradArgs g{};
    g.batch = batch;
    g.N = N;
    g.M = M;
    g.part = part;
    g.dy = dO;
    g.dy_ch = cpo;
    g.xb = h2;
    if ((e = shear::launch_wgrad(2, K, g, G, st)) != hipSuccess) return hip_fail(e, "dW3");
    if ((e = shear::launch_wgrad_reduce(part, grads + pW3, grads + pb3, G, K, 32, c3, 32, st)) != hipSuccess)
        return hip_fail(e, "dW3 reduce");
    if ((e = shear::launch_pack_weights_t(params + pW3, t3, K, 32, 32, cpo, st)) != hipSuccess) return hip_fail(e, "W3^T");
    shear::ConvArgs bd{};
    bd.N = N;
    bd.M = M;
    bd.in = dO;
    bd.W = t3;
    bd.mask_act = h2;
    bd.out_bf = dh2;
    if ((e = shear::launch_conv(5, K, bd, batch, st)) != hipSuccess) return hip_fail(e, "dh2");
    g.dy = dh2;
    g.dy_ch = 32;
    g.xb = h1;
    if ((e = shear::launch_wgrad(1, K, g, G, st)) != hipSuccess) return hip_fail(e, "dW2");
    if ((e = shear::launch_wgrad_reduce(part, grads + pW2, grads + pb2, G, 32, 32, 32, 32, st)) != hipSuccess)
        return hip_fail(e, "dW2 reduce");
    if ((e = shear::launch_pack_weights_t(params + pW2, t2, 32, 32, 32, 32, st)) != hipSuccess) return hip_fail(e, "W2^T");
    bd.in = dh2;
    bd.W = t2;
    bd.mask_act = h1;
    bd.out_bf = dh1;
    if ((e = shear::launch_conv(4, K, bd, batch, st)) != hipSuccess) return hip_fail(e, "dh1");
    g.dy = dh1;
    g.dy_ch = 32;
    g.xb = zp;
    if ((e = shear::launch_wgrad(0, K, g, G, st)) != hipSuccess) return hip_fail(e, "dW1");
    if ((e = shear::launch_wgrad_reduce(part, grads + pW1, grads + pb1, G, 32, K, 32, cpo, st)) != hipSuccess)
        return hip_fail(e, "dW1 reduce");
    // Adam on the FP32 parameters, then the bfloat16 block
    if ((e = shear::launch_adam(params, grads, adam_state, adam_state + np, np, lr, 0.9f, 0.999f, 1e-8f, step, st)) !=
        hipSuccess)
        return hip_fail(e, "Adam");
    if ((e = shear::launch_shrink_pack(K, params + pW1, params + pb1, params + pW2, params + pb2, params + pW3,
                                       params + pb3, packed, st)) != hipSuccess)
        return hip_fail(e, "parameter packing");
    return SHEAR_OK;
}

int shear_shrink_apply(shear_system* s, const float* coeffs, float* shrunk, float* tau, int batch, const float* sigma,
                       const void* packed, void* stream) {
    int rc = check_call(s, coeffs, shrunk, batch, true);
    if (rc == EMPTY_CALL) return SHEAR_OK;
    if (rc != SHEAR_OK) return rc;
    if (!sigma || !packed) return fail(SHEAR_E_INVALID, "sigma or parameter pointer is NULL");
    if (!shear::shrink_supported(s->K, s->rows, s->cols))
        return fail(SHEAR_E_SIZE, "learned shrinkage needs K <= 64, rows % 8 == 0 and cols % 128 == 0");
    const int K = s->K, N = s->rows, M = s->cols;
    const size_t act = (size_t)batch * N * M * 32 * 2;  // one bfloat16 activation tensor
    const size_t sc = ((size_t)batch * K * sizeof(float) + 255) & ~(size_t)255;
    if ((rc = ensure_ws2(s, sc + 2 * act)) != SHEAR_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    char* w = (char*)s->ws2;
    float* scale = (float*)w;
    void* h1 = w + sc;
    void* h2 = w + sc + act;
    const shear::ShrinkLayout L = shear::shrink_layout(K);
    const char* p = (const char*)packed;
    hipError_t e = shear::launch_inv_scale(sigma, s->rms_dev, scale, batch, K, st);
    if (e != hipSuccess) return hip_fail(e, "scale launch");
    shear::ConvArgs a{};
    a.N = N;
    a.M = M;
    a.scale = scale;
    a.lowpass = K - 1;
    a.cus = s->cus;
    // layer 1: z = bf16(c scale), staged from the coefficients inside the layer -> h1
    a.coef = coeffs;
    a.W = (const unsigned short*)(p + L.w1);
    a.bias = (const float*)(p + L.b1);
    a.out_bf = h1;
    a.cin = K;
    a.cout = 32;
    if ((e = shear::launch_conv(6, K, a, batch, st)) != hipSuccess) return hip_fail(e, "layer 1 launch");
    // layer 2: h1 -> h2
    a.in = h1;
    a.W = (const unsigned short*)(p + L.w2);
    a.bias = (const float*)(p + L.b2);
    a.out_bf = h2;
    a.cin = 32;
    if ((e = shear::launch_conv(1, K, a, batch, st)) != hipSuccess) return hip_fail(e, "layer 2 launch");
    // layer 3: h2 -> thresholds -> shrunk coefficients
    a.in = h2;
    a.W = (const unsigned short*)(p + L.w3);
    a.bias = (const float*)(p + L.b3);
    a.out_bf = nullptr;
    a.coef = coeffs;
    a.out_f = shrunk;
    a.tau = tau;
    a.cout = K;
    if ((e = shear::launch_conv(2, K, a, batch, st)) != hipSuccess) return hip_fail(e, "layer 3 launch");
    return SHEAR_OK;
}

int shear_profile_enable(shear_system* s, int on) {
    if (!s) return fail(SHEAR_E_INVALID, "system is NULL");
    s->prof_on = on != 0;
    return SHEAR_OK;
}

int shear_profile_read(shear_system* s, int* launches, double* total_ms) {
    if (!s || !launches || !total_ms) return fail(SHEAR_E_INVALID, "NULL argument");
    for (int k = 0; k < SHEAR_KERNEL_KINDS; ++k) {
        launches[k] = 0;
        total_ms[k] = 0.0;
    }
    int rc = SHEAR_OK;
    for (auto& r : s->prof) {
        float ms = 0.0f;
        hipError_t e = hipEventSynchronize(r.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess && rc == SHEAR_OK) rc = hip_fail(e, "reading launch events");
        launches[r.kind] += 1;
        total_ms[r.kind] += ms;
        s->ev_free.push_back(r.a);
        s->ev_free.push_back(r.b);
    }
    s->prof.clear();
    return rc;
}

void shear_destroy_system(shear_system* s) { release(s); }

}  // extern "C"
