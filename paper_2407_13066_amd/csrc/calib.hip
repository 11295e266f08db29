// Measurement support: the rate at which one kernel can stream a large array out of HBM
// (non-temporal 16-byte loads, every lane keeping several loads in flight), the ceiling the
// operator-streaming product kernels are read against, and the rate at which one kernel can
// write one (non-temporal 8- or 16-byte stores), the ceiling of the result-writing ones.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>

#include "btoep.h"
#include "internal.h"

namespace {

constexpr int kThreads = 256;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kThreads) void k_fill(u32x4* __restrict__ p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kThreads)
        p[i] = u32x4{(uint32_t)i, (uint32_t)(i >> 32), 1u, 2u};
}

// Reads n 16-byte words, U loads in flight per lane; the xor of everything read goes to
// out[0] only if it matches a value the fill never produces, which keeps the loads without a
// store per lane.
template <int U>
__global__ __launch_bounds__(kThreads) void k_stream_read(const u32x4* __restrict__ p, size_t n,
                                                          uint32_t* __restrict__ out) {
    uint32_t acc = 0;
    const size_t stride = (size_t)gridDim.x * kThreads;
    size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x;
    for (; i + (U - 1) * stride < n; i += U * stride) {
        u32x4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = __builtin_nontemporal_load(p + i + u * stride);
#pragma unroll
        for (int u = 0; u < U; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    }
    for (; i < n; i += stride) {
        const u32x4 v = __builtin_nontemporal_load(p + i);
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    if (acc == 0xdeadbeefu) out[0] = acc;
}

// Writes n words of type V (8 or 16 bytes), U stores per lane and loop step.
template <typename V, int U>
__global__ __launch_bounds__(kThreads) void k_stream_write(V* __restrict__ p, size_t n) {
    const size_t stride = (size_t)gridDim.x * kThreads;
    size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x;
    V v;
    for (int k = 0; k < (int)(sizeof(V) / 4); ++k) v[k] = (uint32_t)(i + k);
    for (; i + (U - 1) * stride < n; i += U * stride) {
#pragma unroll
        for (int u = 0; u < U; ++u) __builtin_nontemporal_store(v, p + i + u * stride);
    }
    for (; i < n; i += stride) __builtin_nontemporal_store(v, p + i);
}
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

void launch_write(int width, unsigned grid, void* p, size_t bytes, hipStream_t st) {
    if (width == 8)
        k_stream_write<u32x2, 4><<<grid, kThreads, 0, st>>>(static_cast<u32x2*>(p), bytes / 8);
    else
        k_stream_write<u32x4, 4><<<grid, kThreads, 0, st>>>(static_cast<u32x4*>(p), bytes / 16);
}

void launch_read(int unroll, unsigned grid, const u32x4* p, size_t n, uint32_t* out, hipStream_t st) {
    if (unroll == 8)
        k_stream_read<8><<<grid, kThreads, 0, st>>>(p, n, out);
    else
        k_stream_read<4><<<grid, kThreads, 0, st>>>(p, n, out);
}

}  // namespace

extern "C" {

btoep_status btoep_read_bandwidth(size_t bytes, int reps, void* stream, double* best_ms, double* best_gbs,
                                  double* mean_gbs) {
    if (bytes < (1u << 20) || reps < 1 || !best_ms || !best_gbs || !mean_gbs) return BTOEP_ERR_INVALID_ARG;
    (void)hipGetLastError();  // an error left by an earlier call must not be taken for a launch failure
    hipStream_t st = (hipStream_t)stream;
    const size_t n = bytes / 16;
    u32x4* p = nullptr;
    uint32_t* out = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipMalloc(&p, n * 16);
    if (e == hipSuccess) e = hipMalloc(&out, 64);
    if (e == hipSuccess) e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    // launch shapes tried: 4 or 8 loads in flight per lane, 4, 8 or 16 workgroups per CU; the
    // best shape's times are reported
    double best = 1e30, sum = 0.0;
    if (e == hipSuccess) {
        const unsigned grid0 = (unsigned)std::max(1, cus);
        k_fill<<<grid0 * 8, kThreads, 0, st>>>(p, n);
        double best_shape_sum = 1e30;
        for (int unroll : {4, 8}) {
            for (unsigned per_cu : {4u, 8u, 16u}) {
                const unsigned grid = grid0 * per_cu;
                launch_read(unroll, grid, p, n, out, st);  // warm-up
                double b_min = 1e30, b_sum = 0.0;
                for (int r = 0; r < reps && e == hipSuccess; ++r) {
                    e = hipEventRecord(a, st);
                    launch_read(unroll, grid, p, n, out, st);
                    if (e == hipSuccess) e = hipEventRecord(b, st);
                    if (e == hipSuccess) e = hipEventSynchronize(b);
                    float ms = 0.f;
                    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
                    b_min = std::min(b_min, (double)ms);
                    b_sum += ms;
                }
                if (b_sum < best_shape_sum) {
                    best_shape_sum = b_sum;
                    best = b_min;
                    sum = b_sum;
                }
            }
        }
        if (e == hipSuccess) e = hipGetLastError();
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (p) (void)hipFree(p);
    if (out) (void)hipFree(out);
    if (e != hipSuccess) {
        btoep::set_global_error("btoep_read_bandwidth", e);
        return e == hipErrorOutOfMemory ? BTOEP_ERR_OUT_OF_MEMORY : BTOEP_ERR_HIP;
    }
    const double nb = (double)n * 16.0;
    *best_ms = best;
    *best_gbs = nb / (best * 1e-3) / 1e9;
    *mean_gbs = nb / (sum / reps * 1e-3) / 1e9;
    return BTOEP_OK;
}

btoep_status btoep_write_bandwidth(size_t bytes, int reps, void* stream, double* best_ms, double* best_gbs,
                                   double* mean_gbs) {
    if (bytes < (1u << 20) || reps < 1 || !best_ms || !best_gbs || !mean_gbs) return BTOEP_ERR_INVALID_ARG;
    (void)hipGetLastError();  // an error left by an earlier call must not be taken for a launch failure
    hipStream_t st = (hipStream_t)stream;
    const size_t nb = bytes / 16 * 16;
    void* p = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipMalloc(&p, nb);
    if (e == hipSuccess) e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    // launch shapes tried: 8- or 16-byte stores, 4, 8 or 16 workgroups per CU
    double best = 1e30, sum = 0.0;
    if (e == hipSuccess) {
        const unsigned grid0 = (unsigned)std::max(1, cus);
        double best_shape_sum = 1e30;
        for (int width : {8, 16}) {
            for (unsigned per_cu : {4u, 8u, 16u}) {
                const unsigned grid = grid0 * per_cu;
                launch_write(width, grid, p, nb, st);  // warm-up
                double b_min = 1e30, b_sum = 0.0;
                for (int r = 0; r < reps && e == hipSuccess; ++r) {
                    e = hipEventRecord(a, st);
                    launch_write(width, grid, p, nb, st);
                    if (e == hipSuccess) e = hipEventRecord(b, st);
                    if (e == hipSuccess) e = hipEventSynchronize(b);
                    float ms = 0.f;
                    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
                    b_min = std::min(b_min, (double)ms);
                    b_sum += ms;
                }
                if (b_sum < best_shape_sum) {
                    best_shape_sum = b_sum;
                    best = b_min;
                    sum = b_sum;
                }
            }
        }
        if (e == hipSuccess) e = hipGetLastError();
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (p) (void)hipFree(p);
    if (e != hipSuccess) {
        btoep::set_global_error("btoep_write_bandwidth", e);
        return e == hipErrorOutOfMemory ? BTOEP_ERR_OUT_OF_MEMORY : BTOEP_ERR_HIP;
    }
    *best_ms = best;
    *best_gbs = (double)nb / (best * 1e-3) / 1e9;
    *mean_gbs = (double)nb / (sum / reps * 1e-3) / 1e9;
    return BTOEP_OK;
}

}  // extern "C"
