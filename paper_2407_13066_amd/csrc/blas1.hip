// Vector kernels for conjugate gradients on H (paper section 2.2): inner products
// accumulated in FP64 with a deterministic two-stage reduction, and the CG vector updates
// driven by per-right-hand-side scalars that stay in device memory (no host round trip per
// iteration).
//
// Scalars per right-hand side b, sc[b * kScal + .]:
//   RR   current <r, r>          PAP  <p, H p>        RRN  new <r, r>
//   TH   stopping threshold on <r, r>                 ACT  1.0 while iterating, else 0.0
//   AL   alpha = RR / PAP        BE   beta = RRN / RR
#include "blas1.h"
#include "common.h"

namespace btoep {

constexpr int kDotThreads = 256;
constexpr int kDotBlocks = 512;  // first-stage blocks per right-hand side

size_t dot_tmp_doubles(int nb) { return (size_t)nb * kDotBlocks; }

template <typename T>
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double red[kDotThreads / kWave];
    v = wave_sum(v);
    const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
    if (l == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kDotThreads / kWave; ++i) s += red[i];
    return s;  // valid in thread 0
}

template <typename T>
__global__ __launch_bounds__(kDotThreads) void k_dot_partial(const T* __restrict__ x, const T* __restrict__ y,
                                                             int64_t n, int64_t stride, double* __restrict__ tmp) {
    const int b = blockIdx.y;
    x += (int64_t)b * stride;
    y += (int64_t)b * stride;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kDotThreads + threadIdx.x; i < n; i += (int64_t)kDotBlocks * kDotThreads)
        acc = fma((double)x[i], (double)y[i], acc);
    const double s = block_sum<T>(acc);
    if (threadIdx.x == 0) tmp[(int64_t)b * kDotBlocks + blockIdx.x] = s;
}

// mode 0: sc[slot] = dot.  mode PAP: also AL = ACT ? RR / PAP : 0.
// mode RRN: also BE = RRN / RR, RR = RRN, ACT = (RRN > TH) when ACT was set.
__global__ __launch_bounds__(kDotThreads) void k_dot_final(const double* __restrict__ tmp, double* __restrict__ sc,
                                                           int slot, int mode) {
    const int b = blockIdx.x;
    double acc = 0.0;
    for (int i = threadIdx.x; i < kDotBlocks; i += kDotThreads) acc += tmp[(int64_t)b * kDotBlocks + i];
    const double s = block_sum<double>(acc);
    if (threadIdx.x != 0) return;
    double* q = sc + (int64_t)b * kScal;
    q[slot] = s;
    if (mode == kScPAP) {
        q[kScAL] = (q[kScACT] != 0.0 && s > 0.0) ? q[kScRR] / s : 0.0;
    } else if (mode == kScRRN) {
        if (q[kScACT] != 0.0) {
            q[kScIT] += 1.0;
            q[kScBE] = (q[kScRR] > 0.0) ? s / q[kScRR] : 0.0;
            q[kScRR] = s;
            q[kScACT] = (s > q[kScTH]) ? 1.0 : 0.0;
        } else {
            q[kScBE] = 0.0;
        }
    }
}

hipError_t launch_dot(Real r, const void* x, const void* y, int64_t n, int nb, int64_t stride, double* sc, int slot,
                      int mode, double* tmp, hipStream_t s) {
    dim3 g1(kDotBlocks, nb);
    if (r == Real::F64)
        k_dot_partial<double><<<g1, kDotThreads, 0, s>>>((const double*)x, (const double*)y, n, stride, tmp);
    else
        k_dot_partial<float><<<g1, kDotThreads, 0, s>>>((const float*)x, (const float*)y, n, stride, tmp);
    k_dot_final<<<nb, kDotThreads, 0, s>>>(tmp, sc, slot, mode);
    return hipGetLastError();
}

constexpr int kVecThreads = 256;
static inline dim3 vgrid(int64_t n, int nb) {
    int64_t g = (n + kVecThreads - 1) / kVecThreads;
    if (g > 4096) g = 4096;
    return dim3((unsigned)g, nb);
}

// x += AL p ; r -= AL Ap   (x may be wider than the other vectors)
template <typename T, typename TX>
__global__ void k_cg_xr(TX* __restrict__ x, T* __restrict__ r, const T* __restrict__ p, const T* __restrict__ Ap,
                        int64_t n, int64_t stride, const double* __restrict__ sc) {
    const int b = blockIdx.y;
    const double al = sc[(int64_t)b * kScal + kScAL];
    if (al == 0.0) return;
    const int64_t o = (int64_t)b * stride;
    for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVecThreads) {
        x[o + i] = (TX)fma(al, (double)p[o + i], (double)x[o + i]);
        r[o + i] = (T)fma(-al, (double)Ap[o + i], (double)r[o + i]);
    }
}

// p = r + BE p  (right-hand sides that stopped keep p)
template <typename T>
__global__ void k_cg_p(T* __restrict__ p, const T* __restrict__ r, int64_t n, int64_t stride,
                       const double* __restrict__ sc) {
    const int b = blockIdx.y;
    const double* q = sc + (int64_t)b * kScal;
    if (q[kScACT] == 0.0) return;
    const double be = q[kScBE];
    const int64_t o = (int64_t)b * stride;
    for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVecThreads)
        p[o + i] = (T)fma(be, (double)p[o + i], (double)r[o + i]);
}

// y = a x + c z  elementwise with conversion (types may differ); z may be null.
template <typename TY, typename TA, typename TB>
__global__ void k_axpbz(TY* __restrict__ y, double a, const TA* __restrict__ x, double c, const TB* __restrict__ z,
                        int64_t n, int64_t stride) {
    const int64_t o = (int64_t)blockIdx.y * stride;
    for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVecThreads) {
        double v = a * (double)x[o + i];
        if (z) v = fma(c, (double)z[o + i], v);
        y[o + i] = (TY)v;
    }
}

hipError_t launch_cg_xr(Real rv, Real rx, void* x, void* r, const void* p, const void* Ap, int64_t n, int nb,
                        int64_t stride, const double* sc, hipStream_t s) {
    dim3 g = vgrid(n, nb);
    if (rv == Real::F64 && rx == Real::F64)
        k_cg_xr<double, double><<<g, kVecThreads, 0, s>>>((double*)x, (double*)r, (const double*)p,
                                                           (const double*)Ap, n, stride, sc);
    else if (rv == Real::F32 && rx == Real::F32)
        k_cg_xr<float, float><<<g, kVecThreads, 0, s>>>((float*)x, (float*)r, (const float*)p, (const float*)Ap, n,
                                                         stride, sc);
    else if (rv == Real::F32 && rx == Real::F64)
        k_cg_xr<float, double><<<g, kVecThreads, 0, s>>>((double*)x, (float*)r, (const float*)p, (const float*)Ap,
                                                          n, stride, sc);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_cg_p(Real rv, void* p, const void* r, int64_t n, int nb, int64_t stride, const double* sc,
                       hipStream_t s) {
    dim3 g = vgrid(n, nb);
    if (rv == Real::F64)
        k_cg_p<double><<<g, kVecThreads, 0, s>>>((double*)p, (const double*)r, n, stride, sc);
    else
        k_cg_p<float><<<g, kVecThreads, 0, s>>>((float*)p, (const float*)r, n, stride, sc);
    return hipGetLastError();
}

hipError_t launch_axpbz(Real ry, void* y, double a, Real rx, const void* x, double c, Real rz, const void* z,
                        int64_t n, int nb, int64_t stride, hipStream_t s) {
    dim3 g = vgrid(n, nb);
#define BT_AXPBZ(TY, TA, TB) \
    k_axpbz<TY, TA, TB><<<g, kVecThreads, 0, s>>>((TY*)y, a, (const TA*)x, c, (const TB*)z, n, stride)
    if (ry == Real::F64 && rx == Real::F64 && rz == Real::F64) BT_AXPBZ(double, double, double);
    else if (ry == Real::F64 && rx == Real::F64 && rz == Real::F32) BT_AXPBZ(double, double, float);
    else if (ry == Real::F64 && rx == Real::F32 && rz == Real::F64) BT_AXPBZ(double, float, double);
    else if (ry == Real::F32 && rx == Real::F64 && rz == Real::F64) BT_AXPBZ(float, double, double);
    else if (ry == Real::F32 && rx == Real::F32 && rz == Real::F32) BT_AXPBZ(float, float, float);
    else if (ry == Real::F32 && rx == Real::F64 && rz == Real::F32) BT_AXPBZ(float, double, float);
    else return hipErrorInvalidValue;
#undef BT_AXPBZ
    return hipGetLastError();
}

__global__ void k_cg_init_scalars(double* sc, int nb, double inner_rtol2, double outer_rtol2, double floor2) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    double* q = sc + (int64_t)b * kScal;
    q[kScTH] = fmax(inner_rtol2 * q[kScRR], floor2 * q[kScBB]);
    const bool outer = q[kScRH] > outer_rtol2 * q[kScBB];
    q[kScACT] = (outer && q[kScRR] > q[kScTH] && q[kScRR] > 0.0) ? 1.0 : 0.0;
    q[kScAL] = 0.0;
    q[kScBE] = 0.0;
}

hipError_t launch_cg_init_scalars(double* sc, int nb, double inner_rtol2, double outer_rtol2, double floor2,
                                  hipStream_t s) {
    k_cg_init_scalars<<<(nb + 63) / 64, 64, 0, s>>>(sc, nb, inner_rtol2, outer_rtol2, floor2);
    return hipGetLastError();
}

template <typename T>
__global__ void k_zero(T* __restrict__ y, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVecThreads)
        y[i] = T(0);
}

hipError_t launch_zero(Real r, void* y, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const dim3 g = vgrid(n, 1);
    if (r == Real::F64)
        k_zero<double><<<g, kVecThreads, 0, s>>>((double*)y, n);
    else
        k_zero<float><<<g, kVecThreads, 0, s>>>((float*)y, n);
    return hipGetLastError();
}

}  // namespace btoep
