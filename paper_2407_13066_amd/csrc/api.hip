// Host runtime behind the btoep C interface: operator objects, setup, workspace layout,
// the apply pipelines of F, F^T and H, and the refined CG solver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "btoep.h"
#include "blas1.h"
#include "internal.h"

using namespace btoep;

struct btoep_op_s {
    int device = 0;
    int64_t Nt = 0, Nd = 0, Nm = 0, N = 0, L = 0, nfreq = 0, ldF = 0, ldv = 0;
    btoep_dtype storage = BTOEP_F64;
    Stor stor = Stor::C128;
    Real vreal = Real::F64;
    void* fhat = nullptr;
    size_t fhat_bytes = 0;
    FftPlan plan{};
    void* tw64 = nullptr;  // exp(-2 pi i t / L), t < L, complex FP64
    void* tw32 = nullptr;  // same, complex FP32
    // four-step transforms (long series): N = lp1.N * lp2.N, sub-twiddle tables per type
    bool fft_long = false;
    FftPlan lp1{}, lp2{};
    void* ltw1_64 = nullptr;
    void* ltw2_64 = nullptr;
    void* ltw1_32 = nullptr;
    void* ltw2_32 = nullptr;
    bool gemm_enabled = true;  // MFMA kernels for several right-hand sides
    // per right-hand-side bucket (2..8, 9..16, 17..32, 33..64): matrix-core kernel variants and,
    // for FP32 storage, products on the BF16 matrix cores with the three-term split
    int gvar_n[4] = {0, 0, 0, 0};
    int gvar_c[4] = {0, 0, 0, 0};
    bool gsplit[4] = {false, false, false, false};
    int var_n = 3, var_c = 3;  // single-vector kernel variants (see sbgemv_variants)
    // the appendix (SOTI) form, kept for comparison: Fs[s][p][f] with rows of alt_ldf, the
    // matrix-sized product buffer, SOTI vector spectra and partial sums over parameter chunks
    bool alt_ready = false;
    void* alt_fs = nullptr;
    void* alt_q = nullptr;
    void* alt_v = nullptr;
    void* alt_d = nullptr;
    void* alt_part = nullptr;
    int64_t alt_ldf = 0;
    int alt_chunk = 0, alt_nchunk = 0;
    void* ws = nullptr;    // operator-owned workspace (used when the caller passes none)
    size_t ws_cap = 0;
    std::mutex mu;
    char err[512] = {0};
    // kernel timing (btoep_profile_*)
    struct Pending {
        int kid;
        hipEvent_t a, b;
    };
    bool prof = false;
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    int64_t prof_launches[16] = {0};
    double prof_ms[16] = {0};
};

namespace {

thread_local char g_err[512];

void set_err(btoep_op op, const char* what, hipError_t e) {
    char* dst = op ? op->err : g_err;
    snprintf(dst, 512, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

}  // namespace

void btoep::set_global_error(const char* what, hipError_t e) { set_err(nullptr, what, e); }

namespace {

#define BT_HIP(op, expr)                                  \
    do {                                                  \
        hipError_t e_ = (expr);                           \
        if (e_ != hipSuccess) {                           \
            set_err((op), #expr, e_);                     \
            return e_ == hipErrorOutOfMemory ? BTOEP_ERR_OUT_OF_MEMORY : BTOEP_ERR_HIP; \
        }                                                 \
    } while (0)

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
        else prev = -1;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

bool is_7smooth(int64_t n) {
    for (int p : {2, 3, 5, 7})
        while (n % p == 0) n /= p;
    return n == 1;
}

// Smallest 7-smooth N >= Nt: any padded length L = 2N >= 2Nt - 1 gives the exact linear
// convolution; 2N keeps the even/odd real-transform packing.
// Stored frequencies are a grid dimension of the product kernels (at most 65535), which bounds
// the series length: N + 1 <= 65535, i.e. Nt <= 64827 = 3^3 7^4 (the largest 7-smooth N
// below 65535).
constexpr int64_t kMaxFreq = 65535;

int64_t choose_N(int64_t Nt) {
    int64_t n = std::max<int64_t>(Nt, 1);
    while (!is_7smooth(n)) ++n;
    return n;
}

bool make_plan(int64_t N, FftPlan& pl) {
    pl = FftPlan{};
    pl.N = (int)N;
    int64_t n = N;
    auto take = [&](int r) {
        while (n % r == 0) {
            if (pl.npass >= kMaxPass) return false;
            pl.radix[pl.npass++] = r;
            n /= r;
        }
        return true;
    };
    if (!take(8) || !take(4) || !take(2) || !take(5) || !take(3) || !take(7)) return false;
    return n == 1;
}

size_t stor_bytes(Stor s) { return s == Stor::C128 ? 16 : (s == Stor::C64 ? 8 : 4); }
size_t vbytes(const btoep_op op) { return op->vreal == Real::F64 ? 8 : 4; }
size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
int64_t nspan_of(const btoep_op op) {
    const int cs = n_span_cols(op->stor, op->Nm, (int)op->nfreq);
    return (op->Nm + cs - 1) / cs;
}

// exp(-2 pi i t / (2 n)), t < 2n, in FP64 and FP32, uploaded to new device arrays.
hipError_t upload_twiddles(int64_t n, void*& t64, void*& t32) {
    std::vector<double> a(4 * n);
    std::vector<float> b(4 * n);
    for (int64_t t = 0; t < 2 * n; ++t) {
        const double ang = -M_PI * (double)t / (double)n;
        a[2 * t] = std::cos(ang);
        a[2 * t + 1] = std::sin(ang);
        b[2 * t] = (float)a[2 * t];
        b[2 * t + 1] = (float)a[2 * t + 1];
    }
    hipError_t e = hipMalloc(&t64, a.size() * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&t32, b.size() * sizeof(float));
    if (e == hipSuccess) e = hipMemcpy(t64, a.data(), a.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(t32, b.data(), b.size() * sizeof(float), hipMemcpyHostToDevice);
    return e;
}

// Four-step split N = N1 N2: N1 = n1 when given (must divide N), else the divisor nearest
// sqrt(N) from below for which both passes fit a column tile in FP64.
bool long_split(int64_t N, int64_t n1, FftPlan& p1, FftPlan& p2) {
    auto ok = [&](int64_t a) {
        return a > 1 && N % a == 0 && N / a > 1 && N / a <= 65535 && long_log_cols((int)a, (int)(N / a), Real::F64) >= 0 &&
               make_plan(a, p1) && make_plan(N / a, p2);
    };
    if (n1 > 0) return ok(n1);
    for (int64_t a = (int64_t)std::sqrt((double)N); a > 1; --a)
        if (ok(a)) return true;
    return false;
}

// Switch an operator to four-step transforms with first factor n1 (0: automatic), or back to
// single-pass transforms (n1 < 0).
btoep_status set_long(btoep_op op, int64_t n1) {
    for (void** q : {&op->ltw1_64, &op->ltw2_64, &op->ltw1_32, &op->ltw2_32}) {
        if (*q) (void)hipFree(*q);
        *q = nullptr;
    }
    op->fft_long = false;
    if (n1 < 0) return fft_log_cols((int)op->N, Real::F64) >= 0 ? BTOEP_OK : BTOEP_ERR_UNSUPPORTED;
    FftPlan p1, p2;
    if (!long_split(op->N, n1, p1, p2)) return n1 > 0 ? BTOEP_ERR_INVALID_ARG : BTOEP_ERR_UNSUPPORTED;
    BT_HIP(op, upload_twiddles(p1.N, op->ltw1_64, op->ltw1_32));
    BT_HIP(op, upload_twiddles(p2.N, op->ltw2_64, op->ltw2_32));
    op->lp1 = p1;
    op->lp2 = p2;
    op->fft_long = true;
    return BTOEP_OK;
}

// Workspace layout of one apply over nb right-hand sides (four-step transforms add a complex
// scratch of N rows, the data spectra summed over spans and, for H, the truncated data).
struct ApplyWs {
    size_t vh = 0, part = 0, dh = 0, tmp = 0, spec = 0, dtmp = 0, total = 0;
};
ApplyWs apply_layout(const btoep_op op, btoep_which which, int64_t nb) {
    const size_t c = 2 * vbytes(op);
    const size_t vh = align_up((size_t)nb * op->nfreq * op->ldv * c, 256);
    const size_t part = align_up((size_t)nb * op->nfreq * nspan_of(op) * op->Nd * c, 256);
    const size_t dh = align_up((size_t)nb * op->nfreq * op->Nd * c, 256);
    ApplyWs w;
    size_t off = 0;
    w.vh = off;
    off += vh;
    if (which == BTOEP_APPLY_F || which == BTOEP_APPLY_H) {
        w.part = off;
        off += part;
    }
    if (which == BTOEP_APPLY_FT || which == BTOEP_APPLY_H) {
        w.dh = off;
        off += dh;
    }
    if (op->fft_long) {
        w.tmp = off;
        off += align_up((size_t)nb * op->N * std::max<int64_t>(op->ldv, op->Nd) * c, 256);
        w.spec = off;
        off += align_up((size_t)nb * op->nfreq * op->Nd * c, 256);
        w.dtmp = off;
        off += align_up((size_t)nb * op->Nt * op->Nd * vbytes(op), 256);
    }
    w.total = off;
    return w;
}

// Workspace of a CG solve over nb right-hand sides.
struct CgWs {
    size_t sc = 0, tmp = 0, rhi = 0, r = 0, p = 0, Ap = 0, e = 0, apply = 0, total = 0;
};
CgWs cg_layout(const btoep_op lo, const btoep_op hi, int64_t nb) {
    const size_t n = (size_t)lo->Nt * lo->Nm;
    const size_t vl = vbytes(lo);
    CgWs w;
    size_t off = 0;
    auto put = [&](size_t& slot, size_t bytes) {
        slot = off;
        off += align_up(bytes, 256);
    };
    put(w.sc, (size_t)nb * kScal * sizeof(double));
    put(w.tmp, dot_tmp_doubles((int)nb) * sizeof(double));
    put(w.rhi, (size_t)nb * n * sizeof(double));
    put(w.r, (size_t)nb * n * vl);
    put(w.p, (size_t)nb * n * vl);
    put(w.Ap, (size_t)nb * n * vl);
    put(w.e, (size_t)nb * n * vl);
    const size_t a = std::max(apply_layout(lo, BTOEP_APPLY_H, nb).total,
                              hi ? apply_layout(hi, BTOEP_APPLY_H, nb).total : (size_t)0);
    put(w.apply, a);
    w.total = off;
    return w;
}

btoep_status get_ws(btoep_op op, size_t need, void*& ws, size_t& ws_bytes) {
    if (ws) return ws_bytes >= need ? BTOEP_OK : BTOEP_ERR_WORKSPACE_TOO_SMALL;
    std::lock_guard<std::mutex> lk(op->mu);
    if (op->ws_cap < need) {
        if (op->ws) (void)hipFree(op->ws);
        op->ws = nullptr;
        op->ws_cap = 0;
        BT_HIP(op, hipMalloc(&op->ws, need));
        op->ws_cap = need;
    }
    ws = op->ws;
    ws_bytes = op->ws_cap;
    return BTOEP_OK;
}

// Kernel identifiers for btoep_profile_read.
enum Kid { K_R2C_M = 0, K_SBGEMV_N, K_DSIDE_F, K_DSIDE_H, K_SBGEMV_C, K_C2R_M, K_R2C_D, K_COUNT };
const char* kid_name(int k) {
    static const char* names[K_COUNT] = {"fft_r2c_m", "sbgemv_n", "dside_f", "dside_h",
                                         "sbgemv_c", "fft_c2r_m", "fft_r2c_d"};
    return (k >= 0 && k < K_COUNT) ? names[k] : "?";
}

hipEvent_t pool_event(btoep_op op) {
    if (!op->pool.empty()) {
        hipEvent_t e = op->pool.back();
        op->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Set while this thread records launches into a graph: no timing events are recorded then.
thread_local bool g_capturing = false;

// Launch `fn` on `st`, bracketed by events when profiling is on.
template <typename Fn>
hipError_t timed(btoep_op op, int kid, hipStream_t st, Fn&& fn) {
    if (!op->prof || g_capturing) return fn();
    hipEvent_t a = pool_event(op), b = pool_event(op);
    if (!a || !b) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(a, st);
    if (e == hipSuccess) e = fn();
    if (e == hipSuccess) e = hipEventRecord(b, st);
    op->pending.push_back({kid, a, b});
    return e;
}

const void* tw_of(const btoep_op op) { return op->vreal == Real::F64 ? op->tw64 : op->tw32; }
Stor vstor(const btoep_op op) { return op->vreal == Real::F64 ? Stor::C128 : Stor::C64; }

// Per-frequency products: one vector per launch row (GEMV kernels) for a single right-hand
// side or FP64 storage; the MFMA kernels for nb >= 2 on FP32 / BF16 storage.
bool use_gemm(const btoep_op op, int nb) { return nb >= 2 && op->gemm_enabled; }
// Right-hand-side bucket of the matrix-core tuning: 2..8 -> 0, 9..16 -> 1, 17..32 -> 2, 33..64 -> 3.
int gemm_bucket(int nb) { return nb <= 8 ? 0 : (nb <= 16 ? 1 : (nb <= 32 ? 2 : 3)); }

hipError_t prod_n(btoep_op op, int nb, const void* vh, int64_t vh_b, void* part, int nspan, int64_t part_b,
                  hipStream_t st) {
    const int Nd = (int)op->Nd, Nm = (int)op->Nm, nf = (int)op->nfreq;
    if (use_gemm(op, nb)) {
        // groups of at most the variant's group size (FP64: kGemmNMax), balanced so that every
        // group keeps >= 2 and runs on the matrix cores
        const int bk = gemm_bucket(nb);
        const int var = op->gvar_n[bk];
        const int gmax = op->stor == Stor::C128 ? kGemmNMax : sbgemm_n_group(var);
        const int ng = (nb + gmax - 1) / gmax;
        const int g = (nb + ng - 1) / ng;
        const size_t cb = 2 * vbytes(op);  // bytes of a vector-side complex value
        for (int r0 = 0; r0 < nb; r0 += g) {
            const int n = std::min(g, nb - r0);
            const void* v = (const char*)vh + (size_t)r0 * vh_b * cb;
            void* pt = (char*)part + (size_t)r0 * part_b * cb;
            hipError_t e = op->stor == Stor::C128
                               ? launch_sbgemm_n64(op->fhat, op->ldF, nf, Nd, Nm, v, op->ldv, vh_b, n, pt, nspan,
                                                   part_b, st)
                               : launch_sbgemm_n(op->stor, op->fhat, op->ldF, nf, Nd, Nm, v, op->ldv, vh_b, n, pt,
                                                 nspan, part_b, st, op->gsplit[bk], var);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    return launch_sbgemv_n(op->stor, op->fhat, op->ldF, nf, Nd, Nm, vh, op->ldv, vh_b, nb, part, nspan, part_b, st,
                           op->var_n);
}

hipError_t prod_c(btoep_op op, int nb, const void* dh, int64_t dh_b, void* vh, int64_t vh_b, hipStream_t st) {
    const int Nd = (int)op->Nd, Nm = (int)op->Nm, nf = (int)op->nfreq;
    if (use_gemm(op, nb)) {
        // right-hand-side groups small enough for the staged data spectra
        const bool f64 = op->stor == Stor::C128;
        const size_t cb = 2 * vbytes(op);  // bytes of a vector-side complex value
        int g = f64 ? std::min(nb, kGemmNMax) : nb;
        const bool bf = op->stor == Stor::BF16 || op->gsplit[gemm_bucket(nb)];
        while (g > 1 && (f64 ? sbgemm_c64_lds(g, Nd) : sbgemm_c_lds(g, Nd, bf)) > 64 * 1024) g = (g + 1) / 2;
        for (int r0 = 0; r0 < nb; r0 += g) {
            const int n = std::min(g, nb - r0);
            const void* d = (const char*)dh + (size_t)r0 * dh_b * cb;
            void* o = (char*)vh + (size_t)r0 * vh_b * cb;
            hipError_t e;
            if (n < 2)
                e = launch_sbgemv_c(op->stor, op->fhat, op->ldF, nf, Nd, Nm, d, dh_b, n, o, op->ldv, vh_b, st,
                                    op->var_c);
            else if (f64)
                e = launch_sbgemm_c64(op->fhat, op->ldF, nf, Nd, Nm, d, dh_b, n, o, op->ldv, vh_b, st);
            else
                e = launch_sbgemm_c(op->stor, op->fhat, op->ldF, nf, Nd, Nm, d, dh_b, n, o, op->ldv, vh_b, st,
                                    op->gsplit[gemm_bucket(nb)], op->gvar_c[gemm_bucket(nb)]);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    return launch_sbgemv_c(op->stor, op->fhat, op->ldF, nf, Nd, Nm, dh, dh_b, nb, vh, op->ldv, vh_b, st, op->var_c);
}

// Vector-side transforms of nb right-hand sides: m [k][Nt][Nm] (row Nm) -> spectra
// vh[k][f][ldv], and back with out = inv_n x + add_scale * add; single-pass or four-step
// through tmp (N x ldv per right-hand side) by the operator's mode.
hipError_t vec_r2c(btoep_op op, int nb, const PtrBatch& in, void* vh, void* tmp, hipStream_t st) {
    const int64_t ldv = op->ldv, vh_b = op->nfreq * op->ldv;
    const Real vr = op->vreal;
    if (op->fft_long)
        return launch_long_r2c(vr, vr, vstor(op), in, 0, op->Nm, nb, (int)op->Nt, (int)op->Nm, tmp, ldv,
                               op->N * ldv, vh, ldv, vh_b, op->lp1, op->lp2,
                               vr == Real::F64 ? op->ltw1_64 : op->ltw1_32,
                               vr == Real::F64 ? op->ltw2_64 : op->ltw2_32, tw_of(op), st);
    return launch_fft_r2c(vr, vr, vstor(op), in, op->Nm, nb, vh, ldv, vh_b, (int)op->Nt, (int)op->Nm, op->plan,
                          tw_of(op), st);
}
hipError_t vec_c2r(btoep_op op, int nb, const void* vh, void* tmp, const PtrBatch& out, const PtrBatch& add,
                   double add_scale, hipStream_t st) {
    const int64_t ldv = op->ldv, vh_b = op->nfreq * op->ldv;
    const double inv_n = 1.0 / (double)op->N;
    const Real vr = op->vreal;
    if (op->fft_long)
        return launch_long_c2r(vr, vh, ldv, vh_b, nb, tmp, ldv, op->N * ldv, out, op->Nm, add, add_scale,
                               (int)op->Nt, (int)op->Nm, op->lp1, op->lp2, vr == Real::F64 ? op->ltw1_64 : op->ltw1_32,
                               vr == Real::F64 ? op->ltw2_64 : op->ltw2_32, tw_of(op), inv_n, st);
    return launch_fft_c2r(vr, vh, ldv, vh_b, nb, out, op->Nm, add, add_scale, (int)op->Nt, (int)op->Nm, op->plan,
                          tw_of(op), inv_n, st);
}

// One pipeline launch sequence over nb <= kMaxBatch right-hand sides.  Each transform step
// runs single-pass or, for operators switched to four-step transforms, as two passes through
// the scratch array of the workspace.
btoep_status run_apply(btoep_op op, btoep_which which, int nb, const PtrBatch& in, const PtrBatch& out,
                       double noise_prec, double prior_prec, char* ws, hipStream_t st) {
    const ApplyWs w = apply_layout(op, which, nb);
    void* vh = ws + w.vh;
    void* part = ws + w.part;
    void* dh = ws + w.dh;
    void* tmp = ws + w.tmp;
    void* spec = ws + w.spec;
    char* dtmp = ws + w.dtmp;
    const int Nt = (int)op->Nt, Nd = (int)op->Nd, nf = (int)op->nfreq;
    const int nspan = (int)nspan_of(op);
    const int64_t vh_b = op->nfreq * op->ldv, part_b = op->nfreq * nspan * op->Nd, dh_b = op->nfreq * op->Nd;
    const int64_t N = op->N;
    const double inv_n = 1.0 / (double)op->N;
    const void* tw = tw_of(op);
    const bool lg = op->fft_long;
    const void* tw1 = op->vreal == Real::F64 ? op->ltw1_64 : op->ltw1_32;
    const void* tw2 = op->vreal == Real::F64 ? op->ltw2_64 : op->ltw2_32;
    const Real vr = op->vreal;
    PtrBatch none{};

    // m side: [k][Nt][Nm] -> spectra vh[k][f][ldv], and back (with the prior term for H)
    auto r2c_m = [&]() { return vec_r2c(op, nb, in, vh, tmp, st); };
    auto c2r_m = [&](const PtrBatch& add, double add_scale) {
        return vec_c2r(op, nb, vh, tmp, out, add, add_scale, st);
    };
    // d side: [k][Nt][Nd] -> data spectra dh[k][f][Nd]
    auto r2c_d = [&](const PtrBatch& din) {
        return lg ? launch_long_r2c(vr, vr, vstor(op), din, 0, Nd, nb, Nt, Nd, tmp, Nd, N * Nd, dh, Nd, dh_b,
                                    op->lp1, op->lp2, tw1, tw2, tw, st)
                  : launch_fft_r2c(vr, vr, vstor(op), din, Nd, nb, dh, Nd, dh_b, Nt, Nd, op->plan, tw, st);
    };
    // partial sums -> d (F) or -> truncated, scaled and transformed again (H)
    auto dside = [&](bool hmode, double scale) -> hipError_t {
        if (!lg)
            return hmode ? launch_dside(vr, part, nspan, part_b, nb, nullptr, dh, dh_b, Nt, Nd, op->plan, tw, scale, st)
                         : launch_dside(vr, part, nspan, part_b, nb, &out, nullptr, 0, Nt, Nd, op->plan, tw, scale, st);
        hipError_t e = launch_sum_spans(vr, part, nspan, part_b, spec, (int64_t)nf * Nd, nf, Nd, nb, st);
        if (e != hipSuccess) return e;
        if (!hmode)
            return launch_long_c2r(vr, spec, Nd, (int64_t)nf * Nd, nb, tmp, Nd, N * Nd, out, Nd, none, 0.0, Nt, Nd,
                                   op->lp1, op->lp2, tw1, tw2, tw, scale, st);
        PtrBatch dt{};
        for (int b = 0; b < nb; ++b) dt.p[b] = dtmp + (size_t)b * Nt * Nd * vbytes(op);
        e = launch_long_c2r(vr, spec, Nd, (int64_t)nf * Nd, nb, tmp, Nd, N * Nd, dt, Nd, none, 0.0, Nt, Nd, op->lp1,
                            op->lp2, tw1, tw2, tw, scale, st);
        return e == hipSuccess ? r2c_d(dt) : e;
    };

    if (which == BTOEP_APPLY_F || which == BTOEP_APPLY_H) {
        BT_HIP(op, timed(op, K_R2C_M, st, r2c_m));
        BT_HIP(op, timed(op, K_SBGEMV_N, st, [&] {
            return prod_n(op, nb, vh, vh_b, part, nspan, part_b, st);
        }));
        if (which == BTOEP_APPLY_F) {
            BT_HIP(op, timed(op, K_DSIDE_F, st, [&] { return dside(false, inv_n); }));
            return BTOEP_OK;
        }
        BT_HIP(op, timed(op, K_DSIDE_H, st, [&] { return dside(true, noise_prec * inv_n); }));
        BT_HIP(op, timed(op, K_SBGEMV_C, st, [&] {
            return prod_c(op, nb, dh, dh_b, vh, vh_b, st);
        }));
        BT_HIP(op, timed(op, K_C2R_M, st, [&] { return c2r_m(in, prior_prec); }));
        return BTOEP_OK;
    }
    // F^T
    BT_HIP(op, timed(op, K_R2C_D, st, [&] { return r2c_d(in); }));
    BT_HIP(op, timed(op, K_SBGEMV_C, st, [&] {
        return prod_c(op, nb, dh, dh_b, vh, vh_b, st);
    }));
    BT_HIP(op, timed(op, K_C2R_M, st, [&] { return c2r_m(none, 0.0); }));
    return BTOEP_OK;
}

// An instantiated graph and the graph it came from.
struct GraphHolder {
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    GraphHolder() = default;
    GraphHolder(const GraphHolder&) = delete;
    GraphHolder& operator=(const GraphHolder&) = delete;
    ~GraphHolder() {
        if (x) (void)hipGraphExecDestroy(x);
        if (g) (void)hipGraphDestroy(g);
    }
};

// Records the launches `fn(stream)` makes on a private stream into a graph and instantiates
// it.  Nothing runs during the capture; the graph is launched later on any stream.
template <typename Fn>
btoep_status capture_graph(btoep_op op, GraphHolder& h, Fn&& fn) {
    hipStream_t cs = nullptr;
    BT_HIP(op, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    btoep_status s = BTOEP_OK;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        g_capturing = true;
        s = fn(cs);
        g_capturing = false;
        const hipError_t e2 = hipStreamEndCapture(cs, &h.g);
        if (e2 != hipSuccess) e = e2;
    }
    if (e == hipSuccess && s == BTOEP_OK) e = hipGraphInstantiate(&h.x, h.g, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (s != BTOEP_OK) return s;
    if (e != hipSuccess) {
        set_err(op, "graph capture", e);
        return BTOEP_ERR_HIP;
    }
    return BTOEP_OK;
}

btoep_status apply_contig(btoep_op op, btoep_which which, int64_t k, const void* in, void* out, double noise_prec,
                          double prior_prec, void* ws, size_t ws_bytes, void* stream) {
    if (!op) return BTOEP_ERR_INVALID_ARG;
    if (k < 0) return BTOEP_ERR_INVALID_ARG;
    if (k == 0) return BTOEP_OK;
    if (!in || !out) return BTOEP_ERR_INVALID_ARG;
    if (which == BTOEP_APPLY_H && in == out) return BTOEP_ERR_INVALID_ARG;
    const int64_t nb = std::min<int64_t>(k, kMaxBatch);
    btoep_status s = get_ws(op, apply_layout(op, which, nb).total, ws, ws_bytes);
    if (s != BTOEP_OK) return s;
    DeviceGuard g(op->device);
    const int64_t in_len = op->Nt * (which == BTOEP_APPLY_FT ? op->Nd : op->Nm);
    const int64_t out_len = op->Nt * (which == BTOEP_APPLY_F ? op->Nd : op->Nm);
    const size_t vb = vbytes(op);
    for (int64_t r0 = 0; r0 < k; r0 += nb) {
        const int n = (int)std::min<int64_t>(nb, k - r0);
        PtrBatch pi{}, po{};
        for (int r = 0; r < n; ++r) {
            pi.p[r] = (const char*)in + (size_t)(r0 + r) * in_len * vb;
            po.p[r] = (const char*)out + (size_t)(r0 + r) * out_len * vb;
        }
        s = run_apply(op, which, n, pi, po, noise_prec, prior_prec, (char*)ws, (hipStream_t)stream);
        if (s != BTOEP_OK) return s;
    }
    return BTOEP_OK;
}

// ---- setup ---------------------------------------------------------------------------
// Operator without its Fourier-space blocks: shapes, plans, twiddle tables and the storage of
// Fhat, zeroed when `zero` (otherwise only the alignment padding of each row is cleared).
btoep_status create_shell(int64_t Nt, int64_t Nd, int64_t Nm, btoep_dtype storage, bool zero, hipStream_t st,
                          btoep_op* out) {
    *out = nullptr;
    if (Nt < 1 || Nd < 1 || Nm < 1) return BTOEP_ERR_INVALID_ARG;
    if (storage != BTOEP_F64 && storage != BTOEP_F32 && storage != BTOEP_BF16) return BTOEP_ERR_INVALID_ARG;
    if (Nd > 65535 || Nm > ((int64_t)1 << 30) || Nt > kMaxFreq) return BTOEP_ERR_UNSUPPORTED;
    const int64_t N = choose_N(Nt);
    FftPlan plan;
    if (N + 1 > kMaxFreq || !make_plan(N, plan)) return BTOEP_ERR_UNSUPPORTED;

    btoep_op op = new (std::nothrow) btoep_op_s();
    if (!op) return BTOEP_ERR_OUT_OF_MEMORY;
    if (hipGetDevice(&op->device) != hipSuccess) {
        delete op;
        return BTOEP_ERR_HIP;
    }
    op->Nt = Nt;
    op->Nd = Nd;
    op->Nm = Nm;
    op->N = N;
    op->L = 2 * N;
    op->nfreq = N + 1;
    op->ldF = (int64_t)align_up((size_t)Nm, 8);
    op->ldv = op->ldF;
    op->storage = storage;
    op->stor = storage == BTOEP_F64 ? Stor::C128 : (storage == BTOEP_F32 ? Stor::C64 : Stor::BF16);
    op->vreal = storage == BTOEP_F64 ? Real::F64 : Real::F32;
    op->plan = plan;
    auto fail = [&](btoep_status s) {
        snprintf(g_err, sizeof g_err, "%s", op->err);
        btoep_destroy(op);
        return s;
    };
#define BT_SHELL(expr)                                                                      \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) {                                                             \
            set_err(op, #expr, e_);                                                         \
            return fail(e_ == hipErrorOutOfMemory ? BTOEP_ERR_OUT_OF_MEMORY : BTOEP_ERR_HIP); \
        }                                                                                   \
    } while (0)

    // twiddles exp(-2 pi i t / L), t < L, from FP64 cos / sin
    const int64_t L = op->L;
    std::vector<double> t64(2 * L);
    std::vector<float> t32(2 * L);
    for (int64_t t = 0; t < L; ++t) {
        const double a = -2.0 * M_PI * (double)t / (double)L;
        t64[2 * t] = std::cos(a);
        t64[2 * t + 1] = std::sin(a);
        t32[2 * t] = (float)t64[2 * t];
        t32[2 * t + 1] = (float)t64[2 * t + 1];
    }
    BT_SHELL(hipMalloc(&op->tw64, t64.size() * sizeof(double)));
    BT_SHELL(hipMalloc(&op->tw32, t32.size() * sizeof(float)));
    BT_SHELL(hipMemcpy(op->tw64, t64.data(), t64.size() * sizeof(double), hipMemcpyHostToDevice));
    BT_SHELL(hipMemcpy(op->tw32, t32.data(), t32.size() * sizeof(float), hipMemcpyHostToDevice));

    op->fhat_bytes = (size_t)op->nfreq * Nd * op->ldF * stor_bytes(op->stor);
    BT_SHELL(hipMalloc(&op->fhat, op->fhat_bytes));
    if (zero || op->ldF != Nm) BT_SHELL(hipMemsetAsync(op->fhat, 0, op->fhat_bytes, st));
    BT_SHELL(hipStreamSynchronize(st));
#undef BT_SHELL

    // series too long for one workgroup: four-step transforms throughout
    if (fft_log_cols((int)N, Real::F64) < 0) {
        const btoep_status ls = set_long(op, 0);
        if (ls != BTOEP_OK) return fail(ls);
    }
    *out = op;
    return BTOEP_OK;
}

// Transforms the series of sensors [s0, s0+ns) x parameters [p0, p0+np) and stores them in
// Fhat[f][s][p0 ..].  Element (t, s, p) of the input is src[t*ld_time + (s-s0)*ld_sensor +
// (p-p0)], read for t = 0 .. Nt-1 as F_t (block column) or as F_{Nt-1-t} (last block row);
// the kernels read the latter from its last time row with a negative row stride.  Host input
// is staged through device memory in groups of sensors of at most ~1 GiB.  Returns after the
// work has completed.
btoep_status fill_tile(btoep_op op, int64_t s0, int64_t ns, int64_t p0, int64_t np, const double* src,
                       int64_t ld_time, int64_t ld_sensor, btoep_block_order order, btoep_memory where,
                       hipStream_t st) {
    const int64_t Nt = op->Nt, N = op->N;
    const size_t sb = stor_bytes(op->stor);
    const int64_t out_row = op->Nd * op->ldF;
    const bool rev = order == BTOEP_LAST_BLOCK_ROW;
    void* ltmp = nullptr;
    int64_t ltmp_sensors = 0;
    struct Free {
        void*& p;
        ~Free() {
            if (p) (void)hipFree(p);
        }
    } free_ltmp{ltmp};
    if (op->fft_long) {
        // complex FP64 scratch of N rows for up to ~1 GiB of sensors at a time
        const size_t per = (size_t)N * np * 16;
        ltmp_sensors = std::max<int64_t>(1, std::min<int64_t>(ns, (int64_t)((1ull << 30) / per)));
        BT_HIP(op, hipMalloc(&ltmp, (size_t)ltmp_sensors * per));
    }
    // sensors [s, s+n) whose time row 0 (in block-column order) starts at `first`
    auto run = [&](const double* first, int64_t in_row, int64_t in_batch, int64_t s, int64_t n) -> hipError_t {
        char* dst = (char*)op->fhat + ((size_t)s * op->ldF + (size_t)p0) * sb;
        if (!op->fft_long)
            return launch_fft_r2c_strided(op->stor, first, in_row, in_batch, (int)n, dst, out_row, op->ldF, (int)Nt,
                                          (int)np, op->plan, op->tw64, st);
        for (int64_t a = 0; a < n; a += ltmp_sensors) {
            const int64_t c = std::min<int64_t>(ltmp_sensors, n - a);
            PtrBatch pb{};
            pb.p[0] = first + a * in_batch;
            const hipError_t e = launch_long_r2c(Real::F64, Real::F64, op->stor, pb, in_batch, in_row, (int)c,
                                                 (int)Nt, (int)np, ltmp, np, N * np, dst + (size_t)a * op->ldF * sb,
                                                 out_row, op->ldF, op->lp1, op->lp2, op->ltw1_64, op->ltw2_64,
                                                 op->tw64, st);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    if (where == BTOEP_DEVICE) {
        const double* first = rev ? src + (Nt - 1) * ld_time : src;
        BT_HIP(op, run(first, rev ? -ld_time : ld_time, ld_sensor, s0, ns));
        BT_HIP(op, hipStreamSynchronize(st));
        return BTOEP_OK;
    }
    // host: groups of sensors copied as [Nt][sc][np] FP64
    const size_t per_s = (size_t)Nt * np * sizeof(double);
    const int64_t sc = std::max<int64_t>(1, std::min<int64_t>(ns, (int64_t)((1ull << 30) / per_s)));
    double* stage = nullptr;
    BT_HIP(op, hipMalloc((void**)&stage, (size_t)sc * per_s));
    struct FreeStage {
        double*& p;
        ~FreeStage() { (void)hipFree(p); }
    } free_stage{stage};
    for (int64_t a = 0; a < ns; a += sc) {
        const int64_t n = std::min<int64_t>(sc, ns - a);
        const size_t dpitch = (size_t)n * np * sizeof(double), spitch = (size_t)ld_time * sizeof(double);
        if (ld_sensor == np) {
            BT_HIP(op, hipMemcpy2DAsync(stage, dpitch, src + a * ld_sensor, spitch, dpitch, (size_t)Nt,
                                        hipMemcpyHostToDevice, st));
        } else {
            for (int64_t i = 0; i < n; ++i)
                BT_HIP(op, hipMemcpy2DAsync(stage + i * np, dpitch, src + (a + i) * ld_sensor, spitch,
                                            (size_t)np * sizeof(double), (size_t)Nt, hipMemcpyHostToDevice, st));
        }
        const int64_t row = n * np;
        BT_HIP(op, run(rev ? stage + (Nt - 1) * row : stage, rev ? -row : row, np, s0 + a, n));
        BT_HIP(op, hipStreamSynchronize(st));
    }
    return BTOEP_OK;
}

// ---- persistence of the Fourier-space operator ----------------------------------------
// File: a 64-byte little-endian header, then Fhat[f][s][p] (f <= N, s < Nd, p < Nm) in the
// storage format (interleaved re, im).
struct FileHeader {
    char magic[8];  // "BTOEPFH\n"
    uint32_t version, storage;
    int64_t Nt, Nd, Nm, L;
    uint64_t payload;
    uint64_t reserved;
};
static_assert(sizeof(FileHeader) == 64, "operator file header is 64 bytes");
constexpr char kMagic[8] = {'B', 'T', 'O', 'E', 'P', 'F', 'H', '\n'};
constexpr size_t kFileChunk = (size_t)64 << 20;

struct File {
    FILE* f = nullptr;
    ~File() {
        if (f) fclose(f);
    }
};
struct Pinned {
    void* p = nullptr;
    ~Pinned() {
        if (p) (void)hipHostFree(p);
    }
};

btoep_status io_err(btoep_op op, const char* what, const char* path) {
    snprintf(op ? op->err : g_err, 512, "%s: %s", what, path);
    return BTOEP_ERR_IO;
}

btoep_status save_fhat(btoep_op op, const char* path, hipStream_t st) {
    const size_t sb = stor_bytes(op->stor), row = (size_t)op->Nm * sb;
    const int64_t rows = op->nfreq * op->Nd;
    FileHeader h{};
    memcpy(h.magic, kMagic, 8);
    h.version = 1;
    h.storage = (uint32_t)op->storage;
    h.Nt = op->Nt;
    h.Nd = op->Nd;
    h.Nm = op->Nm;
    h.L = op->L;
    h.payload = (uint64_t)rows * row;
    File fl;
    fl.f = fopen(path, "wb");
    if (!fl.f) return io_err(op, "cannot open for writing", path);
    if (fwrite(&h, sizeof h, 1, fl.f) != 1) return io_err(op, "write failed", path);
    const int64_t per = std::max<int64_t>(1, (int64_t)(kFileChunk / row));
    Pinned buf;
    BT_HIP(op, hipHostMalloc(&buf.p, (size_t)std::min<int64_t>(per, rows) * row, hipHostMallocDefault));
    for (int64_t r0 = 0; r0 < rows; r0 += per) {
        const int64_t n = std::min<int64_t>(per, rows - r0);
        BT_HIP(op, hipMemcpy2DAsync(buf.p, row, (const char*)op->fhat + (size_t)r0 * op->ldF * sb, (size_t)op->ldF * sb,
                                    row, (size_t)n, hipMemcpyDeviceToHost, st));
        BT_HIP(op, hipStreamSynchronize(st));
        if (fwrite(buf.p, row, (size_t)n, fl.f) != (size_t)n) return io_err(op, "write failed", path);
    }
    if (fflush(fl.f) != 0) return io_err(op, "write failed", path);
    return BTOEP_OK;
}

// The header is checked against the file before any device work: magic, version, storage
// code, sizes within the library's limits, the transform length the library derives from Nt,
// and a payload of exactly the stated size.
btoep_status load_fhat(const char* path, hipStream_t st, btoep_op* out) {
    File fl;
    fl.f = fopen(path, "rb");
    if (!fl.f) return io_err(nullptr, "cannot open for reading", path);
    FileHeader h{};
    if (fread(&h, sizeof h, 1, fl.f) != 1) return io_err(nullptr, "truncated header", path);
    if (memcmp(h.magic, kMagic, 8) != 0 || h.version != 1) return io_err(nullptr, "not an operator file", path);
    if (h.storage > (uint32_t)BTOEP_BF16 || h.Nt < 1 || h.Nd < 1 || h.Nm < 1 || h.Nd > 65535 ||
        h.Nm > ((int64_t)1 << 30) || h.Nt > kMaxFreq || h.L != 2 * choose_N(h.Nt) || h.L / 2 + 1 > kMaxFreq)
        return io_err(nullptr, "malformed operator header", path);
    const size_t sb = h.storage == BTOEP_F64 ? 16 : (h.storage == BTOEP_F32 ? 8 : 4);
    const size_t row = (size_t)h.Nm * sb;
    const int64_t rows = (h.L / 2 + 1) * h.Nd;
    if (h.payload != (uint64_t)rows * row) return io_err(nullptr, "malformed operator header", path);
    if (fseeko(fl.f, 0, SEEK_END) != 0 || ftello(fl.f) != (off_t)(sizeof h + h.payload) ||
        fseeko(fl.f, (off_t)sizeof h, SEEK_SET) != 0)
        return io_err(nullptr, "file size does not match its header", path);

    btoep_op op = nullptr;
    btoep_status s = create_shell(h.Nt, h.Nd, h.Nm, (btoep_dtype)h.storage, false, st, &op);
    if (s != BTOEP_OK) return s;
    auto fail = [&](btoep_status e) {
        snprintf(g_err, sizeof g_err, "%s", op->err);
        btoep_destroy(op);
        return e;
    };
    const int64_t per = std::max<int64_t>(1, (int64_t)(kFileChunk / row));
    Pinned buf;
    hipError_t e = hipHostMalloc(&buf.p, (size_t)std::min<int64_t>(per, rows) * row, hipHostMallocDefault);
    for (int64_t r0 = 0; e == hipSuccess && r0 < rows; r0 += per) {
        const int64_t n = std::min<int64_t>(per, rows - r0);
        if (fread(buf.p, row, (size_t)n, fl.f) != (size_t)n) return fail(io_err(op, "read failed", path));
        e = hipMemcpy2DAsync((char*)op->fhat + (size_t)r0 * op->ldF * sb, (size_t)op->ldF * sb, buf.p, row, row,
                             (size_t)n, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
    }
    if (e != hipSuccess) {
        set_err(op, "operator load", e);
        return fail(e == hipErrorOutOfMemory ? BTOEP_ERR_OUT_OF_MEMORY : BTOEP_ERR_HIP);
    }
    *out = op;
    return BTOEP_OK;
}

}  // namespace

extern "C" {

const char* btoep_status_string(btoep_status s) {
    switch (s) {
        case BTOEP_OK: return "ok";
        case BTOEP_ERR_INVALID_ARG: return "invalid argument";
        case BTOEP_ERR_OUT_OF_MEMORY: return "out of device memory";
        case BTOEP_ERR_HIP: return "HIP runtime error";
        case BTOEP_ERR_UNSUPPORTED: return "unsupported shape or option";
        case BTOEP_ERR_NOT_CONVERGED: return "CG did not converge";
        case BTOEP_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
        case BTOEP_ERR_IO: return "file I/O error or malformed operator file";
    }
    return "unknown status";
}

const char* btoep_last_error(btoep_op op) { return op ? op->err : g_err; }

btoep_status btoep_create(int64_t Nt, int64_t Nd, int64_t Nm, const double* blocks, btoep_memory where,
                          btoep_dtype storage, void* stream, btoep_op* out) {
    if (!out) return BTOEP_ERR_INVALID_ARG;
    *out = nullptr;
    if (!blocks) return BTOEP_ERR_INVALID_ARG;
    if (where != BTOEP_HOST && where != BTOEP_DEVICE) return BTOEP_ERR_INVALID_ARG;
    btoep_op op = nullptr;
    btoep_status s = create_shell(Nt, Nd, Nm, storage, false, (hipStream_t)stream, &op);
    if (s != BTOEP_OK) return s;
    s = fill_tile(op, 0, Nd, 0, Nm, blocks, Nd * Nm, Nm, BTOEP_BLOCK_COLUMN, where, (hipStream_t)stream);
    if (s != BTOEP_OK) {
        snprintf(g_err, sizeof g_err, "%s", op->err);
        btoep_destroy(op);
        return s;
    }
    *out = op;
    return BTOEP_OK;
}

btoep_status btoep_create_empty(int64_t Nt, int64_t Nd, int64_t Nm, btoep_dtype storage, void* stream,
                                btoep_op* out) {
    if (!out) return BTOEP_ERR_INVALID_ARG;
    *out = nullptr;
    return create_shell(Nt, Nd, Nm, storage, true, (hipStream_t)stream, out);
}

btoep_status btoep_set_blocks(btoep_op op, int64_t s0, int64_t ns, int64_t p0, int64_t np, const double* src,
                              int64_t ld_time, int64_t ld_sensor, btoep_block_order order, btoep_memory where,
                              void* stream) {
    if (!op || !src) return BTOEP_ERR_INVALID_ARG;
    if (order != BTOEP_BLOCK_COLUMN && order != BTOEP_LAST_BLOCK_ROW) return BTOEP_ERR_INVALID_ARG;
    if (where != BTOEP_HOST && where != BTOEP_DEVICE) return BTOEP_ERR_INVALID_ARG;
    if (s0 < 0 || ns < 1 || s0 + ns > op->Nd || p0 < 0 || np < 1 || p0 + np > op->Nm) return BTOEP_ERR_INVALID_ARG;
    if (ld_sensor < np || (ns > 1 && ld_time < (ns - 1) * ld_sensor + np) || (ns == 1 && ld_time < np))
        return BTOEP_ERR_INVALID_ARG;
    DeviceGuard g(op->device);
    return fill_tile(op, s0, ns, p0, np, src, ld_time, ld_sensor, order, where, (hipStream_t)stream);
}

btoep_status btoep_save(btoep_op op, const char* path, void* stream) {
    if (!op || !path) return BTOEP_ERR_INVALID_ARG;
    DeviceGuard g(op->device);
    return save_fhat(op, path, (hipStream_t)stream);
}

btoep_status btoep_load(const char* path, void* stream, btoep_op* out) {
    if (!out) return BTOEP_ERR_INVALID_ARG;
    *out = nullptr;
    if (!path) return BTOEP_ERR_INVALID_ARG;
    return load_fhat(path, (hipStream_t)stream, out);
}

btoep_status btoep_destroy(btoep_op op) {
    if (!op) return BTOEP_ERR_INVALID_ARG;
    DeviceGuard g(op->device);
    (void)hipDeviceSynchronize();
    if (op->fhat) (void)hipFree(op->fhat);
    if (op->tw64) (void)hipFree(op->tw64);
    if (op->tw32) (void)hipFree(op->tw32);
    for (void* q : {op->ltw1_64, op->ltw2_64, op->ltw1_32, op->ltw2_32, op->alt_fs, op->alt_q, op->alt_v, op->alt_d,
                    op->alt_part})
        if (q) (void)hipFree(q);
    if (op->ws) (void)hipFree(op->ws);
    for (auto& p : op->pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (hipEvent_t e : op->pool) (void)hipEventDestroy(e);
    delete op;
    return BTOEP_OK;
}

btoep_status btoep_query(btoep_op op, btoep_info* info) {
    if (!op || !info) return BTOEP_ERR_INVALID_ARG;
    info->Nt = op->Nt;
    info->Nd = op->Nd;
    info->Nm = op->Nm;
    info->L = op->L;
    info->nfreq = op->nfreq;
    info->ldF = op->ldF;
    info->storage = op->storage;
    info->vector = op->vreal == Real::F64 ? BTOEP_F64 : BTOEP_F32;
    info->fhat_bytes = op->fhat_bytes;
    info->device = op->device;
    return BTOEP_OK;
}

btoep_status btoep_workspace_size(btoep_op op, btoep_which which, int64_t k, size_t* bytes) {
    if (!op || !bytes || k < 0) return BTOEP_ERR_INVALID_ARG;
    const int64_t nb = std::max<int64_t>(1, std::min<int64_t>(k, kMaxBatch));
    switch (which) {
        case BTOEP_APPLY_F:
        case BTOEP_APPLY_FT:
        case BTOEP_APPLY_H: *bytes = apply_layout(op, which, nb).total; return BTOEP_OK;
        case BTOEP_CG: *bytes = cg_layout(op, nullptr, nb).total; return BTOEP_OK;
    }
    return BTOEP_ERR_INVALID_ARG;
}

btoep_status btoep_apply_F(btoep_op op, int64_t k, const void* m, void* d, void* ws, size_t ws_bytes, void* stream) {
    return apply_contig(op, BTOEP_APPLY_F, k, m, d, 0.0, 0.0, ws, ws_bytes, stream);
}

btoep_status btoep_apply_FT(btoep_op op, int64_t k, const void* d, void* m, void* ws, size_t ws_bytes, void* stream) {
    return apply_contig(op, BTOEP_APPLY_FT, k, d, m, 0.0, 0.0, ws, ws_bytes, stream);
}

btoep_status btoep_apply_H(btoep_op op, int64_t k, double noise_prec, double prior_prec, const void* m, void* Hm,
                           void* ws, size_t ws_bytes, void* stream) {
    return apply_contig(op, BTOEP_APPLY_H, k, m, Hm, noise_prec, prior_prec, ws, ws_bytes, stream);
}

}  // extern "C"

// ---- applies without allocation --------------------------------------------------------
// The workspace of btoep_apply_static: one array per device, alive until the process ends.
// Host code never passes `scratch` itself to a kernel: its device address, per device, comes
// from hipGetSymbolAddress on the first call on that device.
static __device__ __align__(256) char scratch[BTOEP_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {nullptr};

// Device address of this device's scratch array (looked up once per device, with it current).
btoep_status scratch_ptr(btoep_op op, void** out) {
    if (op->device < 0 || op->device >= kMaxDevices) return BTOEP_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[op->device]) {
        DeviceGuard g(op->device);
        void* p = nullptr;
        BT_HIP(op, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_ptr[op->device] = p;
    }
    *out = g_scratch_ptr[op->device];
    return BTOEP_OK;
}

}  // namespace

extern "C" {

btoep_status btoep_apply_static(btoep_op op, btoep_which which, int64_t k, double noise_prec, double prior_prec,
                                const void* in, void* out, void* stream) {
    if (!op || k < 0) return BTOEP_ERR_INVALID_ARG;
    if (which != BTOEP_APPLY_F && which != BTOEP_APPLY_FT && which != BTOEP_APPLY_H) return BTOEP_ERR_INVALID_ARG;
    if (k == 0) return BTOEP_OK;
    if (!in || !out || (which == BTOEP_APPLY_H && in == out)) return BTOEP_ERR_INVALID_ARG;
    const size_t need = apply_layout(op, which, std::min<int64_t>(k, kMaxBatch)).total;
    if (need > (size_t)BTOEP_STATIC_SCRATCH_BYTES) {
        snprintf(op->err, sizeof(op->err),
                 "btoep_apply_static: this apply needs %zu bytes of workspace, the static scratch holds %zu "
                 "(use fewer right-hand sides or pass a workspace to btoep_apply_*)",
                 need, (size_t)BTOEP_STATIC_SCRATCH_BYTES);
        return BTOEP_ERR_WORKSPACE_TOO_SMALL;
    }
    void* ws = nullptr;
    const btoep_status s = scratch_ptr(op, &ws);
    if (s != BTOEP_OK) return s;
    return apply_contig(op, which, k, in, out, noise_prec, prior_prec, ws, (size_t)BTOEP_STATIC_SCRATCH_BYTES,
                        stream);
}

btoep_status btoep_apply_batched(btoep_op op, btoep_which which, int64_t k, const void* const* in, void* const* out,
                                 double noise_prec, double prior_prec, void* ws, size_t ws_bytes, void* stream) {
    if (!op || k < 0 || k > kMaxBatch) return BTOEP_ERR_INVALID_ARG;
    if (which != BTOEP_APPLY_F && which != BTOEP_APPLY_FT && which != BTOEP_APPLY_H) return BTOEP_ERR_INVALID_ARG;
    if (k == 0) return BTOEP_OK;
    if (!in || !out) return BTOEP_ERR_INVALID_ARG;
    PtrBatch pi{}, po{};
    for (int64_t r = 0; r < k; ++r) {
        if (!in[r] || !out[r]) return BTOEP_ERR_INVALID_ARG;
        if (which == BTOEP_APPLY_H && in[r] == out[r]) return BTOEP_ERR_INVALID_ARG;
        pi.p[r] = in[r];
        po.p[r] = out[r];
    }
    btoep_status s = get_ws(op, apply_layout(op, which, k).total, ws, ws_bytes);
    if (s != BTOEP_OK) return s;
    DeviceGuard g(op->device);
    return run_apply(op, which, (int)k, pi, po, noise_prec, prior_prec, (char*)ws, (hipStream_t)stream);
}

}  // extern "C"

struct btoep_graph_s {
    btoep_op op = nullptr;
    int k = 0;
    const void** table = nullptr;  // device: k input addresses, then k output addresses
    bool table_set = false;        // a launch has written the table
    GraphHolder h;
    ~btoep_graph_s() {
        if (table) (void)hipFree(table);
    }
};

namespace {

// Writes a replay's addresses into the graph's table (one lane per right-hand side).
__global__ void k_write_table(PtrBatch in, PtrBatch out, int k, const void** table) {
    const int r = threadIdx.x;
    if (r < k) {
        table[r] = in.p[r];
        table[k + r] = out.p[r];
    }
}

}  // namespace

extern "C" {

btoep_status btoep_graph_create(btoep_op op, btoep_which which, int64_t k, double noise_prec, double prior_prec,
                                void* ws, size_t ws_bytes, btoep_graph* out) {
    if (!out) return BTOEP_ERR_INVALID_ARG;
    *out = nullptr;
    if (!op || k < 1 || k > kMaxBatch || !ws) return BTOEP_ERR_INVALID_ARG;
    if (which != BTOEP_APPLY_F && which != BTOEP_APPLY_FT && which != BTOEP_APPLY_H) return BTOEP_ERR_INVALID_ARG;
    if (ws_bytes < apply_layout(op, which, k).total) return BTOEP_ERR_WORKSPACE_TOO_SMALL;
    btoep_graph gr = new (std::nothrow) btoep_graph_s();
    if (!gr) return BTOEP_ERR_OUT_OF_MEMORY;
    gr->op = op;
    gr->k = (int)k;
    DeviceGuard g(op->device);
    hipError_t e = hipMalloc((void**)&gr->table, 2 * (size_t)k * sizeof(void*));
    if (e != hipSuccess) {
        set_err(op, "graph table", e);
        delete gr;
        return e == hipErrorOutOfMemory ? BTOEP_ERR_OUT_OF_MEMORY : BTOEP_ERR_HIP;
    }
    PtrBatch pi{}, po{};
    pi.dev = gr->table;
    po.dev = gr->table + k;
    const btoep_status s = capture_graph(op, gr->h, [&](hipStream_t cs) {
        return run_apply(op, which, (int)k, pi, po, noise_prec, prior_prec, (char*)ws, cs);
    });
    if (s != BTOEP_OK) {
        delete gr;
        return s;
    }
    *out = gr;
    return BTOEP_OK;
}

btoep_status btoep_graph_launch(btoep_graph gr, const void* const* in, void* const* out, void* stream) {
    if (!gr || (!in) != (!out)) return BTOEP_ERR_INVALID_ARG;
    if (!in && !gr->table_set) return BTOEP_ERR_INVALID_ARG;  // no vectors to replay on yet
    hipStream_t st = (hipStream_t)stream;
    DeviceGuard g(gr->op->device);
    if (in) {
        PtrBatch pi{}, po{};
        for (int r = 0; r < gr->k; ++r) {
            if (!in[r] || !out[r]) return BTOEP_ERR_INVALID_ARG;
            pi.p[r] = in[r];
            po.p[r] = out[r];
        }
        k_write_table<<<1, kMaxBatch, 0, st>>>(pi, po, gr->k, gr->table);
        BT_HIP(gr->op, hipGetLastError());
        gr->table_set = true;
    }
    BT_HIP(gr->op, hipGraphLaunch(gr->h.x, st));
    return BTOEP_OK;
}

btoep_status btoep_graph_destroy(btoep_graph gr) {
    if (!gr) return BTOEP_ERR_INVALID_ARG;
    DeviceGuard g(gr->op->device);
    (void)hipDeviceSynchronize();  // no replay may still be running
    delete gr;
    return BTOEP_OK;
}

btoep_status btoep_cg_solve(btoep_op lo, btoep_op hi, int64_t k, double noise_prec, double prior_prec,
                            const double* b, double* x, const btoep_cg_opts* opts, btoep_cg_result* results, void* ws,
                            size_t ws_bytes, void* stream) {
    if (!lo || k < 0) return BTOEP_ERR_INVALID_ARG;
    if (k == 0) return BTOEP_OK;
    if (!b || !x) return BTOEP_ERR_INVALID_ARG;
    if (!hi && lo->storage != BTOEP_F64) return BTOEP_ERR_INVALID_ARG;
    if (hi && (hi->storage != BTOEP_F64 || hi->Nt != lo->Nt || hi->Nd != lo->Nd || hi->Nm != lo->Nm ||
               hi->device != lo->device))
        return BTOEP_ERR_INVALID_ARG;
    btoep_cg_opts o{1e-8, 10, 1000, 1e-4, 4, 1};
    if (opts) o = *opts;
    if (!(o.rtol > 0) || o.max_outer < 1 || o.max_inner < 1 || !(o.inner_rtol > 0) || o.check_every < 1)
        return BTOEP_ERR_INVALID_ARG;
    if (k > kMaxBatch) return BTOEP_ERR_UNSUPPORTED;
    btoep_op H = hi ? hi : lo;
    const int nb = (int)k;
    const CgWs w = cg_layout(lo, hi, nb);
    btoep_status s = get_ws(lo, w.total, ws, ws_bytes);
    if (s != BTOEP_OK) return s;
    DeviceGuard g(lo->device);
    hipStream_t st = (hipStream_t)stream;
    char* base = (char*)ws;
    double* sc = (double*)(base + w.sc);
    double* tmp = (double*)(base + w.tmp);
    double* rhi = (double*)(base + w.rhi);
    void* r = base + w.r;
    void* p = base + w.p;
    void* Ap = base + w.Ap;
    void* e = base + w.e;
    char* aws = base + w.apply;
    const size_t aws_bytes = w.total - w.apply;
    const int64_t n = lo->Nt * lo->Nm;
    const Real rl = lo->vreal;

    double* hsc = nullptr;
    BT_HIP(lo, hipHostMalloc((void**)&hsc, (size_t)nb * kScal * sizeof(double), hipHostMallocDefault));
    struct HostFree {
        double* p;
        ~HostFree() {
            if (p) (void)hipHostFree(p);
        }
    } hf{hsc};

    std::vector<double> zeros((size_t)nb * kScal, 0.0);
    BT_HIP(lo, hipMemcpyAsync(sc, zeros.data(), zeros.size() * sizeof(double), hipMemcpyHostToDevice, st));
    BT_HIP(lo, launch_dot(Real::F64, b, b, n, nb, n, sc, kScBB, 0, tmp, st));

    // One inner CG iteration: Ap = H_lo p, then the FP64 scalar recurrences and vector
    // updates.  With opts.use_graph it is captured once per call and replayed.
    auto inner_step = [&](hipStream_t s1) -> btoep_status {
        const btoep_status q = apply_contig(lo, BTOEP_APPLY_H, k, p, Ap, noise_prec, prior_prec, aws, aws_bytes, s1);
        if (q != BTOEP_OK) return q;
        BT_HIP(lo, launch_dot(rl, p, Ap, n, nb, n, sc, kScPAP, kScPAP, tmp, s1));
        BT_HIP(lo, launch_cg_xr(rl, rl, e, r, p, Ap, n, nb, n, sc, s1));
        BT_HIP(lo, launch_dot(rl, r, r, n, nb, n, sc, kScRRN, kScRRN, tmp, s1));
        BT_HIP(lo, launch_cg_p(rl, p, r, n, nb, n, sc, s1));
        return BTOEP_OK;
    };
    GraphHolder step;

    int outer = 0, inner_total = 0, matvecs = 0;
    const double rtol2 = o.rtol * o.rtol;
    bool all_conv = false;
    for (;;) {
        // true residual in FP64 with the refinement operator: rhi = b - H x
        s = apply_contig(H, BTOEP_APPLY_H, k, x, rhi, noise_prec, prior_prec, aws, aws_bytes, stream);
        if (s != BTOEP_OK) return s;
        ++matvecs;
        BT_HIP(lo, launch_axpbz(Real::F64, rhi, -1.0, Real::F64, rhi, 1.0, Real::F64, b, n, nb, n, st));
        BT_HIP(lo, launch_dot(Real::F64, rhi, rhi, n, nb, n, sc, kScRH, 0, tmp, st));
        BT_HIP(lo, hipMemcpyAsync(hsc, sc, (size_t)nb * kScal * sizeof(double), hipMemcpyDeviceToHost, st));
        BT_HIP(lo, hipStreamSynchronize(st));
        all_conv = true;
        for (int i = 0; i < nb; ++i)
            if (hsc[i * kScal + kScRH] > rtol2 * hsc[i * kScal + kScBB]) all_conv = false;
        if (all_conv || outer >= o.max_outer) break;
        ++outer;
        // inner CG on H_lo e = r, e0 = 0, vectors in the low operator's type
        BT_HIP(lo, launch_axpbz(rl, r, 1.0, Real::F64, rhi, 0.0, Real::F64, nullptr, n, nb, n, st));
        BT_HIP(lo, launch_axpbz(rl, e, 0.0, rl, r, 0.0, rl, nullptr, n, nb, n, st));
        BT_HIP(lo, launch_axpbz(rl, p, 1.0, rl, r, 0.0, rl, nullptr, n, nb, n, st));
        BT_HIP(lo, launch_dot(rl, r, r, n, nb, n, sc, kScRR, 0, tmp, st));
        BT_HIP(lo, launch_cg_init_scalars(sc, nb, o.inner_rtol * o.inner_rtol, rtol2, 0.0, st));
        if (o.use_graph && !step.x) {
            s = capture_graph(lo, step, inner_step);
            if (s != BTOEP_OK) return s;
        }
        for (int it = 0; it < o.max_inner; ++it) {
            if (step.x) {
                BT_HIP(lo, hipGraphLaunch(step.x, st));
            } else {
                s = inner_step(st);
                if (s != BTOEP_OK) return s;
            }
            ++matvecs;
            ++inner_total;
            if ((it + 1) % o.check_every == 0) {
                BT_HIP(lo, hipMemcpyAsync(hsc, sc, (size_t)nb * kScal * sizeof(double), hipMemcpyDeviceToHost, st));
                BT_HIP(lo, hipStreamSynchronize(st));
                bool any = false;
                for (int i = 0; i < nb; ++i) any |= hsc[i * kScal + kScACT] != 0.0;
                if (!any) break;
            }
        }
        BT_HIP(lo, launch_axpbz(Real::F64, x, 1.0, Real::F64, x, 1.0, rl, e, n, nb, n, st));
    }
    if (results) {
        for (int i = 0; i < nb; ++i) {
            const double bb = hsc[i * kScal + kScBB], rh = hsc[i * kScal + kScRH];
            results[i].inner_iters = (int)hsc[i * kScal + kScIT];
            results[i].outer_iters = outer;
            results[i].matvecs = matvecs;
            results[i].rel_residual = bb > 0 ? std::sqrt(rh / bb) : std::sqrt(rh);
            results[i].converged = rh <= rtol2 * bb ? 1 : 0;
        }
    }
    (void)inner_total;
    return all_conv ? BTOEP_OK : BTOEP_ERR_NOT_CONVERGED;
}

}  // extern "C"

namespace {

// Transform mode: when a series fits one workgroup and a four-step split exists, time the
// vector-side forward and inverse transforms of one right-hand side in each mode and keep the
// faster.
btoep_status tune_fft_mode(btoep_op op, int reps, hipStream_t st, btoep_tune_result* out) {
    out->fft_four_step = op->fft_long ? 1 : 0;
    out->ms_fft[0] = out->ms_fft[1] = 0.0;
    FftPlan q1, q2;
    if (fft_log_cols((int)op->N, Real::F64) < 0 || !long_split(op->N, 0, q1, q2)) return BTOEP_OK;
    const size_t vb = (size_t)op->Nt * op->Nm * vbytes(op);
    void* vec = nullptr;
    BT_HIP(op, hipMalloc(&vec, 2 * vb));
    struct Free {
        void* p;
        ~Free() {
            if (p) (void)hipFree(p);
        }
    } free_vec{vec};
    BT_HIP(op, hipMemsetAsync(vec, 0, 2 * vb, st));
    PtrBatch pin{}, pout{};
    pin.p[0] = vec;
    pout.p[0] = (char*)vec + vb;
    hipEvent_t a = nullptr, b = nullptr;
    BT_HIP(op, hipEventCreate(&a));
    BT_HIP(op, hipEventCreate(&b));
    hipError_t e = hipSuccess;
    btoep_status s = BTOEP_OK;
    for (int mode = 0; mode < 2 && e == hipSuccess && s == BTOEP_OK; ++mode) {
        (void)hipStreamSynchronize(st);
        s = set_long(op, mode ? 0 : -1);
        if (s != BTOEP_OK) break;
        void* ws = nullptr;
        size_t ws_bytes = 0;
        s = get_ws(op, apply_layout(op, BTOEP_APPLY_H, 1).total, ws, ws_bytes);
        if (s != BTOEP_OK) break;
        const ApplyWs w = apply_layout(op, BTOEP_APPLY_H, 1);
        char* base = (char*)ws;
        auto pair = [&]() {
            hipError_t r = vec_r2c(op, 1, pin, base + w.vh, base + w.tmp, st);
            if (r == hipSuccess) r = vec_c2r(op, 1, base + w.vh, base + w.tmp, pout, pin, 1.0, st);
            return r;
        };
        e = pair();
        if (e == hipSuccess) e = hipEventRecord(a, st);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = pair();
        if (e == hipSuccess) e = hipEventRecord(b, st);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        out->ms_fft[mode] = (double)ms / reps;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipStreamSynchronize(st);
    const bool four = e == hipSuccess && s == BTOEP_OK && out->ms_fft[1] < out->ms_fft[0];
    const btoep_status s2 = set_long(op, four ? 0 : -1);
    out->fft_four_step = op->fft_long ? 1 : 0;
    if (e != hipSuccess) {
        set_err(op, "autotune transforms", e);
        return BTOEP_ERR_HIP;
    }
    return s != BTOEP_OK ? s : s2;
}

}  // namespace

extern "C" {

btoep_status btoep_autotune(btoep_op op, int reps, void* stream, btoep_tune_result* out) {
    if (!op || reps < 1 || !out) return BTOEP_ERR_INVALID_ARG;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    btoep_status s = get_ws(op, apply_layout(op, BTOEP_APPLY_H, 1).total, ws, ws_bytes);
    if (s != BTOEP_OK) return s;
    DeviceGuard g(op->device);
    hipStream_t st = (hipStream_t)stream;
    const ApplyWs w = apply_layout(op, BTOEP_APPLY_H, 1);
    char* base = (char*)ws;
    const int Nd = (int)op->Nd, Nm = (int)op->Nm, nf = (int)op->nfreq, nspan = (int)nspan_of(op);
    const int64_t vh_b = op->nfreq * op->ldv, part_b = op->nfreq * nspan * op->Nd, dh_b = op->nfreq * op->Nd;
    // defined inputs for the timing runs
    BT_HIP(op, hipMemsetAsync(base, 0, w.total, st));
    hipEvent_t a = nullptr, b = nullptr;
    BT_HIP(op, hipEventCreate(&a));
    BT_HIP(op, hipEventCreate(&b));
    const int nvar = std::min(sbgemv_variants(), 8);
    memset(out, 0, sizeof(*out));
    out->nvar = nvar;
    double best_n = 1e30, best_c = 1e30;
    hipError_t e = hipSuccess;
    for (int dir = 0; dir < 2 && e == hipSuccess; ++dir) {
        for (int v = 0; v < nvar && e == hipSuccess; ++v) {
            auto launch = [&]() {
                return dir == 0 ? launch_sbgemv_n(op->stor, op->fhat, op->ldF, nf, Nd, Nm, base + w.vh, op->ldv, vh_b,
                                                  1, base + w.part, nspan, part_b, st, v)
                                : launch_sbgemv_c(op->stor, op->fhat, op->ldF, nf, Nd, Nm, base + w.dh, dh_b, 1,
                                                  base + w.vh, op->ldv, vh_b, st, v);
            };
            e = launch();
            if (e == hipSuccess) e = hipEventRecord(a, st);
            for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
            if (e == hipSuccess) e = hipEventRecord(b, st);
            if (e == hipSuccess) e = hipEventSynchronize(b);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
            const double per = (double)ms / reps;
            if (dir == 0) {
                out->ms_n[v] = per;
                if (per < best_n) best_n = per, out->var_n = v;
            } else {
                out->ms_c[v] = per;
                if (per < best_c) best_c = per, out->var_c = v;
            }
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (e != hipSuccess) {
        set_err(op, "autotune", e);
        return BTOEP_ERR_HIP;
    }
    op->var_n = out->var_n;
    op->var_c = out->var_c;
    return tune_fft_mode(op, reps, st, out);
}

btoep_status btoep_set_fft(btoep_op op, int64_t n1) {
    if (!op) return BTOEP_ERR_INVALID_ARG;
    DeviceGuard g(op->device);
    (void)hipDeviceSynchronize();  // no apply may still use the tables being replaced
    const btoep_status s = set_long(op, n1 == 0 ? (fft_log_cols((int)op->N, Real::F64) < 0 ? 0 : -1) : n1);
    if (s != BTOEP_OK && n1 != 0) (void)set_long(op, fft_log_cols((int)op->N, Real::F64) < 0 ? 0 : -1);
    return s;
}

btoep_status btoep_alt_prepare(btoep_op op, int mode, void* stream) {
    if (!op || (mode != 0 && mode != 1)) return BTOEP_ERR_INVALID_ARG;
    const int64_t nf = op->nfreq, Nd = op->Nd, Nm = op->Nm;
    if (nf > 65535LL * 32 || Nm > 65535LL * 32 || Nd * Nm > 2147483647LL) return BTOEP_ERR_UNSUPPORTED;
    DeviceGuard g(op->device);
    hipStream_t st = (hipStream_t)stream;
    const size_t sb = stor_bytes(op->stor), vc = 2 * vbytes(op);
    if (!op->alt_ready) {
        const int64_t ldf = (int64_t)align_up((size_t)nf, 8);
        // parameter chunks of the sums over p: enough (chunk, frequency block, sensor)
        // workgroups to fill the chip
        const int64_t fb = (nf + 255) / 256;
        int64_t nchunk = std::min<int64_t>(std::min<int64_t>(Nm, 65535), std::max<int64_t>(1, 4096 / (fb * Nd)));
        const int64_t chunk = (Nm + nchunk - 1) / nchunk;
        nchunk = (Nm + chunk - 1) / chunk;
        if (!op->alt_fs) BT_HIP(op, hipMalloc(&op->alt_fs, (size_t)Nd * Nm * ldf * sb));
        if (!op->alt_v) BT_HIP(op, hipMalloc(&op->alt_v, (size_t)Nm * ldf * vc));
        if (!op->alt_d) BT_HIP(op, hipMalloc(&op->alt_d, (size_t)Nd * ldf * vc));
        if (!op->alt_part) BT_HIP(op, hipMalloc(&op->alt_part, (size_t)Nd * nf * nchunk * vc));
        op->alt_ldf = ldf;
        op->alt_chunk = (int)chunk;
        op->alt_nchunk = (int)nchunk;
        // Fhat[f][s][p] -> Fs[s][p][f], one sensor per batch
        BT_HIP(op, launch_transpose(sb, op->fhat, Nd * op->ldF, op->ldF, op->alt_fs, ldf, Nm * ldf, (int)nf, (int)Nm,
                                    (int)Nd, st));
        BT_HIP(op, hipStreamSynchronize(st));
        op->alt_ready = true;
    }
    if (mode == 0 && !op->alt_q) BT_HIP(op, hipMalloc(&op->alt_q, (size_t)Nd * Nm * op->alt_ldf * vc));
    return BTOEP_OK;
}

btoep_status btoep_alt_apply(btoep_op op, btoep_which which, int mode, const void* in, void* out, void* stream) {
    if (!op || !in || !out || (which != BTOEP_APPLY_F && which != BTOEP_APPLY_FT) || (mode != 0 && mode != 1))
        return BTOEP_ERR_INVALID_ARG;
    if (!op->alt_ready || (mode == 0 && !op->alt_q)) return BTOEP_ERR_INVALID_ARG;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    const ApplyWs w = apply_layout(op, BTOEP_APPLY_H, 1);
    btoep_status s = get_ws(op, w.total, ws, ws_bytes);
    if (s != BTOEP_OK) return s;
    DeviceGuard g(op->device);
    hipStream_t st = (hipStream_t)stream;
    char* base = (char*)ws;
    void* vh = base + w.vh;
    void* dh = base + w.dh;
    void* tmp = base + w.tmp;
    void* spec = base + w.spec;
    const int Nt = (int)op->Nt, Nd = (int)op->Nd, Nm = (int)op->Nm, nf = (int)op->nfreq;
    const int64_t N = op->N, ldf = op->alt_ldf;
    const size_t vc = 2 * vbytes(op);
    const Real vr = op->vreal;
    const void* tw = tw_of(op);
    const void* tw1 = vr == Real::F64 ? op->ltw1_64 : op->ltw1_32;
    const void* tw2 = vr == Real::F64 ? op->ltw2_64 : op->ltw2_32;
    const bool fused = mode == 1;
    PtrBatch pi{}, po{}, none{};
    pi.p[0] = in;
    po.p[0] = out;
    if (which == BTOEP_APPLY_F) {
        BT_HIP(op, vec_r2c(op, 1, pi, vh, tmp, st));
        BT_HIP(op, launch_transpose(vc, vh, op->ldv, 0, op->alt_v, ldf, 0, nf, Nm, 1, st));
        BT_HIP(op, launch_alt_product(op->stor, vr, false, fused, op->alt_fs, op->alt_v, op->alt_part, op->alt_q, Nd,
                                      Nm, nf, ldf, op->alt_chunk, op->alt_nchunk, st));
        const double inv_n = 1.0 / (double)N;
        if (!op->fft_long) {
            BT_HIP(op, launch_dside(vr, op->alt_part, op->alt_nchunk, 0, 1, &po, nullptr, 0, Nt, Nd, op->plan, tw, inv_n,
                                    st));
        } else {
            BT_HIP(op, launch_sum_spans(vr, op->alt_part, op->alt_nchunk, 0, spec, (int64_t)nf * Nd, nf, Nd, 1, st));
            BT_HIP(op, launch_long_c2r(vr, spec, Nd, (int64_t)nf * Nd, 1, tmp, Nd, N * Nd, po, Nd, none, 0.0, Nt, Nd,
                                       op->lp1, op->lp2, tw1, tw2, tw, inv_n, st));
        }
        return BTOEP_OK;
    }
    BT_HIP(op, op->fft_long ? launch_long_r2c(vr, vr, vstor(op), pi, 0, Nd, 1, Nt, Nd, tmp, Nd, N * Nd, dh, Nd,
                                              (int64_t)nf * Nd, op->lp1, op->lp2, tw1, tw2, tw, st)
                            : launch_fft_r2c(vr, vr, vstor(op), pi, Nd, 1, dh, Nd, (int64_t)nf * Nd, Nt, Nd, op->plan,
                                             tw, st));
    BT_HIP(op, launch_transpose(vc, dh, Nd, 0, op->alt_d, ldf, 0, nf, Nd, 1, st));
    BT_HIP(op, launch_alt_product(op->stor, vr, true, fused, op->alt_fs, op->alt_d, op->alt_v, op->alt_q, Nd, Nm, nf,
                                  ldf, op->alt_chunk, op->alt_nchunk, st));
    BT_HIP(op, launch_transpose(vc, op->alt_v, ldf, 0, vh, op->ldv, 0, Nm, nf, 1, st));
    BT_HIP(op, vec_c2r(op, 1, vh, tmp, po, none, 0.0, st));
    return BTOEP_OK;
}

btoep_status btoep_set_gemm(btoep_op op, int mode) {
    if (!op || mode < 0 || mode > 1 || (mode == 1 && op->storage != BTOEP_F32)) return BTOEP_ERR_INVALID_ARG;
    for (bool& b : op->gsplit) b = mode == 1;
    return BTOEP_OK;
}

btoep_status btoep_set_gemm_variants(btoep_op op, int64_t k, int var_n, int var_c) {
    if (!op || k < 2 || k > kMaxBatch || op->storage == BTOEP_F64) return BTOEP_ERR_INVALID_ARG;
    if (var_n < 0 || var_n >= sbgemm_n_variants() || var_c < 0 || var_c >= sbgemm_c_variants())
        return BTOEP_ERR_INVALID_ARG;
    op->gvar_n[gemm_bucket((int)k)] = var_n;
    op->gvar_c[gemm_bucket((int)k)] = var_c;
    return BTOEP_OK;
}

btoep_status btoep_autotune_gemm(btoep_op op, int64_t k, int allow_split, int reps, void* stream,
                                 btoep_gemm_tune_result* out) {
    if (!op || !out || k < 2 || k > kMaxBatch || reps < 1) return BTOEP_ERR_INVALID_ARG;
    if (op->storage == BTOEP_F64 || !op->gemm_enabled) return BTOEP_ERR_UNSUPPORTED;
    const int nb = (int)k, bk = gemm_bucket(nb);
    const ApplyWs w = apply_layout(op, BTOEP_APPLY_H, nb);
    void* ws = nullptr;
    size_t ws_bytes = 0;
    btoep_status s = get_ws(op, w.total, ws, ws_bytes);
    if (s != BTOEP_OK) return s;
    DeviceGuard g(op->device);
    hipStream_t st = (hipStream_t)stream;
    char* base = (char*)ws;
    const int nspan = (int)nspan_of(op);
    const int64_t vh_b = op->nfreq * op->ldv, part_b = op->nfreq * nspan * op->Nd, dh_b = op->nfreq * op->Nd;
    // defined (zero) inputs for the timing runs, written by a kernel
    BT_HIP(op, launch_zero(Real::F32, base, (int64_t)(w.total / 4), st));
    hipEvent_t a = nullptr, b = nullptr;
    BT_HIP(op, hipEventCreate(&a));
    BT_HIP(op, hipEventCreate(&b));
    memset(out, 0, sizeof(*out));
    out->k = nb;
    out->nvar_n = std::min(sbgemm_n_variants(), 8);
    out->nvar_c = std::min(sbgemm_c_variants(), 8);
    const int nmode = (op->storage == BTOEP_F32 && allow_split) ? 2 : 1;
    const int saved_n = op->gvar_n[bk], saved_c = op->gvar_c[bk];
    const bool saved_split = op->gsplit[bk];
    double best_n[2] = {1e30, 1e30}, best_c[2] = {1e30, 1e30};
    int arg_n[2] = {0, 0}, arg_c[2] = {0, 0};
    hipError_t e = hipSuccess;
    // modes timed: both when allowed, else the bucket's current one
    for (int mi = 0; mi < nmode && e == hipSuccess; ++mi) {
        const int mode = nmode == 2 ? mi : (saved_split ? 1 : 0);
        op->gsplit[bk] = mode == 1;
        for (int dir = 0; dir < 2 && e == hipSuccess; ++dir) {
            const int nv = dir == 0 ? out->nvar_n : out->nvar_c;
            for (int v = 0; v < nv && e == hipSuccess; ++v) {
                if (dir == 0)
                    op->gvar_n[bk] = v;
                else
                    op->gvar_c[bk] = v;
                auto launch = [&]() {
                    return dir == 0 ? prod_n(op, nb, base + w.vh, vh_b, base + w.part, nspan, part_b, st)
                                    : prod_c(op, nb, base + w.dh, dh_b, base + w.vh, vh_b, st);
                };
                e = launch();
                if (e == hipSuccess) e = hipEventRecord(a, st);
                for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
                if (e == hipSuccess) e = hipEventRecord(b, st);
                if (e == hipSuccess) e = hipEventSynchronize(b);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
                const double per = (double)ms / reps;
                if (dir == 0) {
                    out->ms_n[mode][v] = per;
                    if (per < best_n[mode]) best_n[mode] = per, arg_n[mode] = v;
                } else {
                    out->ms_c[mode][v] = per;
                    if (per < best_c[mode]) best_c[mode] = per, arg_c[mode] = v;
                }
            }
            if (dir == 0)
                op->gvar_n[bk] = saved_n;
            else
                op->gvar_c[bk] = saved_c;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    op->gsplit[bk] = saved_split;
    if (e != hipSuccess) {
        set_err(op, "autotune_gemm", e);
        return BTOEP_ERR_HIP;
    }
    const int m = nmode == 2 ? (best_n[1] + best_c[1] < best_n[0] + best_c[0] ? 1 : 0) : (saved_split ? 1 : 0);
    out->split = m;
    out->var_n = arg_n[m];
    out->var_c = arg_c[m];
    op->gsplit[bk] = m == 1;
    op->gvar_n[bk] = out->var_n;
    op->gvar_c[bk] = out->var_c;
    return BTOEP_OK;
}

btoep_status btoep_set_tuning(btoep_op op, int var_n, int var_c, int use_mfma) {
    if (!op || var_n < 0 || var_c < 0 || var_n >= sbgemv_variants() || var_c >= sbgemv_variants())
        return BTOEP_ERR_INVALID_ARG;
    op->var_n = var_n;
    op->var_c = var_c;
    op->gemm_enabled = use_mfma != 0;
    return BTOEP_OK;
}

}  // extern "C"

// ---- stepwise CG ----------------------------------------------------------------------
// State of one stepwise solve.  The caller applies H_lo p (and, with a refinement operator,
// H_hi x); the state holds the CG vectors in the inner operator's vector type, the FP64
// scalars and, when refined, the FP64 array that receives H_hi x and becomes the residual.
struct btoep_cg_s {
    btoep_op op = nullptr;  // inner operator
    btoep_op hi = nullptr;  // FP64 refinement operator, or null
    int64_t k = 0, n = 0;
    const void* b = nullptr;
    void* x = nullptr;
    void* r = nullptr;
    void* p = nullptr;
    void* Ap = nullptr;
    double* hx = nullptr;
    double* sc = nullptr;
    double* tmp = nullptr;
    double* host = nullptr;  // pinned copy of the scalars
    void* owned_dev = nullptr;  // memory allocated by btoep_cg_start (null for btoep_cg_begin)
    bool owned_host = false;
    hipEvent_t ev = nullptr;
    bool polled = false;
    double rtol2 = 0.0, inner_rtol2 = 0.0;
    int outer = 0, updates = 0;           // refinement steps and updates enqueued so far
    int seen_outer = 0, seen_updates = 0;  // the same, as of the last poll
};

namespace {

// Offsets of the state's arrays in its device memory.
struct CgStateLayout {
    size_t sc = 0, tmp = 0, r = 0, p = 0, Ap = 0, hx = 0, total = 0, host = 0;
};
CgStateLayout cg_state_layout(const btoep_op lo, const btoep_op hi, int64_t k) {
    const size_t n = (size_t)lo->Nt * lo->Nm, vl = vbytes(lo);
    CgStateLayout w;
    size_t off = 0;
    auto put = [&](size_t& slot, size_t bytes) {
        slot = off;
        off += align_up(bytes, 256);
    };
    put(w.sc, (size_t)k * kScal * sizeof(double));
    put(w.tmp, dot_tmp_doubles((int)k) * sizeof(double));
    put(w.r, (size_t)k * n * vl);
    put(w.p, (size_t)k * n * vl);
    put(w.Ap, (size_t)k * n * vl);
    if (hi) put(w.hx, (size_t)k * n * sizeof(double));
    w.total = off;
    w.host = (size_t)k * kScal * sizeof(double);
    return w;
}

bool cg_pair_ok(const btoep_op lo, const btoep_op hi) {
    return !hi || (hi->storage == BTOEP_F64 && hi->Nt == lo->Nt && hi->Nd == lo->Nd && hi->Nm == lo->Nm &&
                   hi->device == lo->device);
}

// Restart of the inner iteration from the residual held in `res` (type rres): r = res,
// p = r, RR = <r, r>, thresholds and active flags.
hipError_t cg_restart(btoep_cg cg, const void* res, Real rres, double outer_rtol2, double floor2, hipStream_t st) {
    const Real rv = cg->op->vreal;
    const int nb = (int)cg->k;
    const int64_t n = cg->n;
    hipError_t e = launch_axpbz(rv, cg->r, 1.0, rres, res, 0.0, rres, nullptr, n, nb, n, st);
    if (e == hipSuccess) e = launch_axpbz(rv, cg->p, 1.0, rv, cg->r, 0.0, rv, nullptr, n, nb, n, st);
    if (e == hipSuccess) e = launch_dot(rv, cg->r, cg->r, n, nb, n, cg->sc, kScRR, 0, cg->tmp, st);
    if (e == hipSuccess) e = launch_cg_init_scalars(cg->sc, nb, cg->inner_rtol2, outer_rtol2, floor2, st);
    return e;
}

// Initial state: x = 0, so the true residual is b itself.  Refined: BB = RH = <b, b> in FP64,
// inner iteration on r = b rounded to the inner type.  Plain: the recurrence residual is the
// only one and the inner threshold is rtol itself.
hipError_t cg_init(btoep_cg cg, hipStream_t st) {
    const btoep_op op = cg->op;
    const int nb = (int)cg->k;
    const int64_t n = cg->n;
    const Real rb = cg->hi ? Real::F64 : op->vreal;  // type of b and x
    hipError_t e = launch_zero(Real::F64, cg->sc, (int64_t)nb * kScal, st);
    if (e == hipSuccess) e = launch_zero(rb, cg->x, (int64_t)nb * n, st);
    if (e == hipSuccess) e = launch_dot(rb, cg->b, cg->b, n, nb, n, cg->sc, kScBB, 0, cg->tmp, st);
    if (e == hipSuccess) e = launch_dot(rb, cg->b, cg->b, n, nb, n, cg->sc, kScRH, 0, cg->tmp, st);
    if (e != hipSuccess) return e;
    if (cg->hi) return cg_restart(cg, cg->b, Real::F64, cg->rtol2, 0.25 * cg->rtol2, st);
    // plain: stop on ||r||^2 <= rtol^2 ||b||^2; outer test 0 keeps every nonzero column active
    cg->inner_rtol2 = cg->rtol2;
    return cg_restart(cg, cg->b, rb, 0.0, 0.0, st);
}

void cg_free(btoep_cg cg) {
    if (cg->ev) (void)hipEventDestroy(cg->ev);
    if (cg->owned_dev) (void)hipFree(cg->owned_dev);
    if (cg->owned_host && cg->host) (void)hipHostFree(cg->host);
    delete cg;
}

btoep_status cg_err(btoep_op op, const char* what, hipError_t e) {
    set_err(op, what, e);
    return e == hipErrorOutOfMemory ? BTOEP_ERR_OUT_OF_MEMORY : BTOEP_ERR_HIP;
}

// Points the state's arrays into `dev` (laid out by cg_state_layout) and `host`.
void cg_bind(btoep_cg cg, const CgStateLayout& w, char* dev, double* host) {
    cg->sc = (double*)(dev + w.sc);
    cg->tmp = (double*)(dev + w.tmp);
    cg->r = dev + w.r;
    cg->p = dev + w.p;
    cg->Ap = dev + w.Ap;
    cg->hx = cg->hi ? (double*)(dev + w.hx) : nullptr;
    cg->host = host;
}

}  // namespace

extern "C" {

btoep_status btoep_cg_workspace_size(btoep_op op_lo, btoep_op op_hi, int64_t k, size_t* bytes) {
    if (!op_lo || !bytes || k < 0 || !cg_pair_ok(op_lo, op_hi)) return BTOEP_ERR_INVALID_ARG;
    const int64_t nb = std::max<int64_t>(1, std::min<int64_t>(k, kMaxBatch));
    *bytes = cg_layout(op_lo, op_hi, nb).total;
    return BTOEP_OK;
}

btoep_status btoep_cg_state_size(btoep_op op_lo, btoep_op op_hi, int64_t k, size_t* dev_bytes,
                                 size_t* host_bytes) {
    if (!op_lo || !dev_bytes || !host_bytes || k < 1 || k > kMaxBatch || !cg_pair_ok(op_lo, op_hi))
        return BTOEP_ERR_INVALID_ARG;
    const CgStateLayout w = cg_state_layout(op_lo, op_hi, k);
    *dev_bytes = w.total;
    *host_bytes = w.host;
    return BTOEP_OK;
}

btoep_status btoep_cg_begin(btoep_op op_lo, btoep_op op_hi, int64_t k, const void* b, void* x, double rtol,
                            double inner_rtol, void* dev_mem, size_t dev_bytes, void* host_mem, size_t host_bytes,
                            void* stream, btoep_cg* out) {
    if (!out) return BTOEP_ERR_INVALID_ARG;
    *out = nullptr;
    if (!op_lo || !b || !x || k < 1 || k > kMaxBatch || !(rtol > 0.0) || !dev_mem || !host_mem)
        return BTOEP_ERR_INVALID_ARG;
    if (!cg_pair_ok(op_lo, op_hi) || (op_hi && !(inner_rtol > 0.0 && inner_rtol < 1.0)))
        return BTOEP_ERR_INVALID_ARG;
    if ((uintptr_t)dev_mem % 256 != 0 || (uintptr_t)host_mem % alignof(double) != 0) return BTOEP_ERR_INVALID_ARG;
    const CgStateLayout w = cg_state_layout(op_lo, op_hi, k);
    if (dev_bytes < w.total || host_bytes < w.host) return BTOEP_ERR_WORKSPACE_TOO_SMALL;
    btoep_cg cg = new (std::nothrow) btoep_cg_s();
    if (!cg) return BTOEP_ERR_OUT_OF_MEMORY;
    cg->op = op_lo;
    cg->hi = op_hi;
    cg->k = k;
    cg->n = op_lo->Nt * op_lo->Nm;
    cg->b = b;
    cg->x = x;
    cg->rtol2 = rtol * rtol;
    cg->inner_rtol2 = inner_rtol * inner_rtol;
    cg_bind(cg, w, (char*)dev_mem, (double*)host_mem);
    DeviceGuard g(op_lo->device);
    hipError_t e = hipEventCreateWithFlags(&cg->ev, hipEventDisableTiming);
    if (e == hipSuccess) e = cg_init(cg, (hipStream_t)stream);
    if (e != hipSuccess) {
        const btoep_status s = cg_err(op_lo, "cg_begin", e);
        cg_free(cg);
        return s;
    }
    *out = cg;
    return BTOEP_OK;
}

btoep_status btoep_cg_start(btoep_op op, int64_t k, double noise_prec, double prior_prec, const void* b, void* x,
                            double rtol, void* stream, btoep_cg* out) {
    (void)noise_prec;
    (void)prior_prec;
    if (!out) return BTOEP_ERR_INVALID_ARG;
    *out = nullptr;
    if (!op || !b || !x || k < 1 || k > kMaxBatch || !(rtol > 0.0)) return BTOEP_ERR_INVALID_ARG;
    btoep_cg cg = new (std::nothrow) btoep_cg_s();
    if (!cg) return BTOEP_ERR_OUT_OF_MEMORY;
    cg->op = op;
    cg->k = k;
    cg->n = op->Nt * op->Nm;
    cg->b = b;
    cg->x = x;
    cg->rtol2 = rtol * rtol;
    const CgStateLayout w = cg_state_layout(op, nullptr, k);
    DeviceGuard g(op->device);
    double* host = nullptr;
    hipError_t e = hipMalloc(&cg->owned_dev, w.total);
    if (e == hipSuccess) e = hipHostMalloc((void**)&host, w.host, hipHostMallocDefault);
    if (e == hipSuccess) {
        cg->owned_host = true;
        cg_bind(cg, w, (char*)cg->owned_dev, host);
        e = hipEventCreateWithFlags(&cg->ev, hipEventDisableTiming);
    }
    if (e == hipSuccess) e = cg_init(cg, (hipStream_t)stream);
    if (e != hipSuccess) {
        const btoep_status s = cg_err(op, "cg_start", e);
        if (host && !cg->owned_host) (void)hipHostFree(host);
        (void)hipDeviceSynchronize();
        cg_free(cg);
        return s;
    }
    *out = cg;
    return BTOEP_OK;
}

btoep_status btoep_cg_end(btoep_cg cg) {
    if (!cg) return BTOEP_ERR_INVALID_ARG;
    DeviceGuard g(cg->op->device);
    if (cg->owned_dev) (void)hipDeviceSynchronize();  // the state's own memory is freed below
    cg_free(cg);
    return BTOEP_OK;
}

btoep_status btoep_cg_vectors(btoep_cg cg, void** p, void** Ap) {
    if (!cg || !p || !Ap) return BTOEP_ERR_INVALID_ARG;
    *p = cg->p;
    *Ap = cg->Ap;
    return BTOEP_OK;
}

btoep_status btoep_cg_residual_vectors(btoep_cg cg, void** x, void** Hx) {
    if (!cg || !x || !Hx || !cg->hi) return BTOEP_ERR_INVALID_ARG;
    *x = cg->x;
    *Hx = cg->hx;
    return BTOEP_OK;
}

btoep_status btoep_cg_update(btoep_cg cg, void* stream) {
    if (!cg) return BTOEP_ERR_INVALID_ARG;
    btoep_op op = cg->op;
    DeviceGuard g(op->device);
    hipStream_t st = (hipStream_t)stream;
    const Real rv = op->vreal, rx = cg->hi ? Real::F64 : rv;
    const int nb = (int)cg->k;
    const int64_t n = cg->n;
    BT_HIP(op, launch_dot(rv, cg->p, cg->Ap, n, nb, n, cg->sc, kScPAP, kScPAP, cg->tmp, st));
    BT_HIP(op, launch_cg_xr(rv, rx, cg->x, cg->r, cg->p, cg->Ap, n, nb, n, cg->sc, st));
    BT_HIP(op, launch_dot(rv, cg->r, cg->r, n, nb, n, cg->sc, kScRRN, kScRRN, cg->tmp, st));
    BT_HIP(op, launch_cg_p(rv, cg->p, cg->r, n, nb, n, cg->sc, st));
    ++cg->updates;
    return BTOEP_OK;
}

btoep_status btoep_cg_refine(btoep_cg cg, void* stream) {
    if (!cg || !cg->hi) return BTOEP_ERR_INVALID_ARG;
    btoep_op op = cg->op;
    DeviceGuard g(op->device);
    hipStream_t st = (hipStream_t)stream;
    const int nb = (int)cg->k;
    const int64_t n = cg->n;
    // true residual in FP64: hx = b - H_hi x, RH = <hx, hx>
    BT_HIP(op, launch_axpbz(Real::F64, cg->hx, -1.0, Real::F64, cg->hx, 1.0, Real::F64, cg->b, n, nb, n, st));
    BT_HIP(op, launch_dot(Real::F64, cg->hx, cg->hx, n, nb, n, cg->sc, kScRH, 0, cg->tmp, st));
    BT_HIP(op, cg_restart(cg, cg->hx, Real::F64, cg->rtol2, 0.25 * cg->rtol2, st));
    ++cg->outer;
    return BTOEP_OK;
}

btoep_status btoep_cg_poll(btoep_cg cg, void* stream) {
    if (!cg) return BTOEP_ERR_INVALID_ARG;
    btoep_op op = cg->op;
    DeviceGuard g(op->device);
    hipStream_t st = (hipStream_t)stream;
    BT_HIP(op, hipMemcpyAsync(cg->host, cg->sc, (size_t)cg->k * kScal * sizeof(double), hipMemcpyDeviceToHost, st));
    BT_HIP(op, hipEventRecord(cg->ev, st));
    cg->polled = true;
    cg->seen_outer = cg->outer;
    cg->seen_updates = cg->updates;
    return BTOEP_OK;
}

}  // extern "C"

namespace {

// 1 when the last poll has landed, 0 while it is in flight or none was made, <0 on error.
int cg_landed(btoep_cg cg) {
    if (!cg->polled) return 0;
    DeviceGuard g(cg->op->device);
    const hipError_t q = hipEventQuery(cg->ev);
    if (q == hipErrorNotReady) return 0;
    if (q != hipSuccess) {
        set_err(cg->op, "cg poll", q);
        return -1;
    }
    return 1;
}

}  // namespace

extern "C" {

btoep_status btoep_cg_status(btoep_cg cg, int* ready, int* active, int* iters, double* rel_res) {
    if (!cg || !ready) return BTOEP_ERR_INVALID_ARG;
    *ready = 0;
    const int l = cg_landed(cg);
    if (l < 0) return BTOEP_ERR_HIP;
    if (l == 0) return BTOEP_OK;
    *ready = 1;
    int act = 0, it = 0;
    for (int64_t i = 0; i < cg->k; ++i) {
        const double* h = cg->host + i * kScal;
        act += h[kScACT] != 0.0;
        it = std::max(it, (int)h[kScIT]);
        if (rel_res) rel_res[i] = h[kScBB] > 0 ? std::sqrt(h[kScRR] / h[kScBB]) : 0.0;
    }
    if (active) *active = act;
    if (iters) *iters = it;
    return BTOEP_OK;
}

btoep_status btoep_cg_report(btoep_cg cg, int* ready, btoep_cg_result* results) {
    if (!cg || !ready || !results) return BTOEP_ERR_INVALID_ARG;
    *ready = 0;
    const int l = cg_landed(cg);
    if (l < 0) return BTOEP_ERR_HIP;
    if (l == 0) return BTOEP_OK;
    *ready = 1;
    for (int64_t i = 0; i < cg->k; ++i) {
        const double* h = cg->host + i * kScal;
        const double bb = h[kScBB], res2 = cg->hi ? h[kScRH] : h[kScRR];
        results[i].inner_iters = (int)h[kScIT];
        results[i].outer_iters = cg->seen_outer;
        results[i].matvecs = cg->seen_updates + cg->seen_outer;
        results[i].converged = res2 <= cg->rtol2 * bb ? 1 : 0;
        results[i].rel_residual = bb > 0 ? std::sqrt(res2 / bb) : std::sqrt(res2);
    }
    return BTOEP_OK;
}

btoep_status btoep_profile_enable(btoep_op op, int enable) {
    if (!op) return BTOEP_ERR_INVALID_ARG;
    DeviceGuard g(op->device);
    for (auto& p : op->pending) {
        (void)hipEventSynchronize(p.b);
        op->pool.push_back(p.a);
        op->pool.push_back(p.b);
    }
    op->pending.clear();
    for (int i = 0; i < 16; ++i) {
        op->prof_launches[i] = 0;
        op->prof_ms[i] = 0.0;
    }
    op->prof = enable != 0;
    return BTOEP_OK;
}

btoep_status btoep_profile_read(btoep_op op, btoep_kernel_time* out, int max, int* count) {
    if (!op || !count || max < 0 || (max > 0 && !out)) return BTOEP_ERR_INVALID_ARG;
    DeviceGuard g(op->device);
    for (auto& p : op->pending) {
        BT_HIP(op, hipEventSynchronize(p.b));
        float ms = 0.f;
        BT_HIP(op, hipEventElapsedTime(&ms, p.a, p.b));
        op->prof_launches[p.kid] += 1;
        op->prof_ms[p.kid] += ms;
        op->pool.push_back(p.a);
        op->pool.push_back(p.b);
    }
    op->pending.clear();
    int n = 0;
    for (int k = 0; k < K_COUNT; ++k) {
        if (op->prof_launches[k] == 0) continue;
        if (n < max) {
            snprintf(out[n].name, sizeof(out[n].name), "%s", kid_name(k));
            out[n].launches = op->prof_launches[k];
            out[n].total_ms = op->prof_ms[k];
        }
        ++n;
    }
    *count = std::min(n, max);
    return BTOEP_OK;
}

}  // extern "C"
