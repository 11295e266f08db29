// Per-frequency complex matrix-vector products with the stored operator (paper section 3.3,
// the "apply_matrix" step of its Algorithms 2 and 3, which the paper maps to a strided
// batched GEMV).  For every frequency f the operator block Fh_f is Nd x Nm complex, stored
// row-major as Fh[f][s][p] with a padded row stride ldF (a multiple of 8 elements, zero
// padded), so both directions stream it with coalesced 32-byte-per-lane loads:
//
//   N (for F):   dh_f[s]  = sum_p Fh_f[s][p] mh_f[p]
//                Lanes walk p; each workgroup owns one frequency and a span of CS columns
//                (its slice of mh_f staged in LDS) and every wave reduces RB rows at a time
//                across its 64 lanes.  The per-span results are written as partial sums
//                part[f][span][s]; the data-side kernel adds them in a fixed order, so the
//                result is deterministic (no floating-point atomics).
//   C (for F^T): mo_f[p] = sum_s conj(Fh_f[s][p]) dh_f[s]   (paper section 3.4, eq. AdjointFFTMatvec)
//                Lanes own p and loop over s with dh_f broadcast from LDS: no reduction.
//
// Storage formats: complex FP64 (accumulate FP64), complex FP32 and complex BF16 (both
// accumulate FP32).  The operator is read with non-temporal loads: it is streamed once per
// application and should not evict the vectors from the caches.
#include "common.h"
#include "internal.h"

namespace btoep {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <typename S>
struct StorT;
template <>
struct StorT<cx<double>> {
    typedef double A;  // accumulation / vector real type
    static constexpr int VEC = 2;
    __device__ static cx<double> get(const u32x4* w, int v) {
        return cx<double>{__hiloint2double(w[v][1], w[v][0]), __hiloint2double(w[v][3], w[v][2])};
    }
};
template <>
struct StorT<cx<float>> {
    typedef float A;
    static constexpr int VEC = 4;
    __device__ static cx<float> get(const u32x4* w, int v) {
        const u32x4 q = w[v >> 1];
        return (v & 1) ? cx<float>{__uint_as_float(q[2]), __uint_as_float(q[3])}
                       : cx<float>{__uint_as_float(q[0]), __uint_as_float(q[1])};
    }
};
template <>
struct StorT<bf16c> {
    typedef float A;
    static constexpr int VEC = 8;
    __device__ static cx<float> get(const u32x4* w, int v) {
        const uint32_t u = w[v >> 2][v & 3];
        return cx<float>{bf16_lo(u), bf16_hi(u)};
    }
};

// 32 bytes of the operator (VEC complex entries), two non-temporal 16-byte loads.
__device__ __forceinline__ void load32_nt(const void* p, u32x4* w) {
    const u32x4* q = reinterpret_cast<const u32x4*>(p);
    w[0] = __builtin_nontemporal_load(q);
    w[1] = __builtin_nontemporal_load(q + 1);
}

constexpr int kGemvThreads = 256;
constexpr int kGemvWaves = kGemvThreads / kWave;

// ---- N direction ----------------------------------------------------------------------
template <typename S, int RB>
__global__ __launch_bounds__(kGemvThreads) void k_sbgemv_n(const S* __restrict__ Fh, int64_t ldF, int Nd, int Nm,
                                                           const cx<typename StorT<S>::A>* __restrict__ mh,
                                                           int64_t ldv, int64_t mh_batch,
                                                           cx<typename StorT<S>::A>* __restrict__ part,
                                                           int CS, int nspan, int64_t part_batch) {
    typedef typename StorT<S>::A A;
    constexpr int VEC = StorT<S>::VEC;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<A>* msh = reinterpret_cast<cx<A>*>(smem_raw);

    const int span = blockIdx.x, f = blockIdx.y, b = blockIdx.z;
    const int col0 = span * CS;
    const int ncol = min(CS, Nm - col0);
    const cx<A>* __restrict__ mrow = mh + (int64_t)b * mh_batch + (int64_t)f * ldv + col0;
    for (int i = threadIdx.x; i < CS; i += kGemvThreads) msh[i] = (i < ncol) ? mrow[i] : cx<A>{0, 0};
    __syncthreads();

    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const S* __restrict__ Ff = Fh + (int64_t)f * Nd * ldF + col0;
    cx<A>* __restrict__ pout = part + (int64_t)b * part_batch + ((int64_t)f * nspan + span) * Nd;

    for (int s0 = wave * RB; s0 < Nd; s0 += kGemvWaves * RB) {
        cx<A> acc[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) acc[r] = cx<A>{0, 0};
#pragma unroll 2
        for (int t = lane * VEC; t < ncol; t += kWave * VEC) {
            u32x4 w[RB][2];
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int s = min(s0 + r, Nd - 1);  // rows past Nd repeat the last one; discarded below
                load32_nt(Ff + (int64_t)s * ldF + t, w[r]);
            }
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                const cx<A> mv = msh[t + v];
#pragma unroll
                for (int r = 0; r < RB; ++r) cfma(acc[r], StorT<S>::get(w[r], v), mv);
            }
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            acc[r].re = wave_sum(acc[r].re);
            acc[r].im = wave_sum(acc[r].im);
        }
        if (lane == 0) {
#pragma unroll
            for (int r = 0; r < RB; ++r)
                if (s0 + r < Nd) pout[s0 + r] = acc[r];
        }
    }
}

// ---- C direction ----------------------------------------------------------------------
constexpr int kDChunk = 1024;

template <typename S, int RB>
__global__ __launch_bounds__(kGemvThreads) void k_sbgemv_c(const S* __restrict__ Fh, int64_t ldF, int Nd, int Nm,
                                                           const cx<typename StorT<S>::A>* __restrict__ dh,
                                                           int64_t dh_batch,
                                                           cx<typename StorT<S>::A>* __restrict__ mo, int64_t ldv,
                                                           int64_t mo_batch) {
    typedef typename StorT<S>::A A;
    constexpr int VEC = StorT<S>::VEC;
    __shared__ cx<A> dsh[kDChunk];
    const int f = blockIdx.y, b = blockIdx.z;
    const int col = (blockIdx.x * kGemvThreads + threadIdx.x) * VEC;
    const bool active = col < Nm;
    const S* __restrict__ Ff = Fh + (int64_t)f * Nd * ldF + col;
    const cx<A>* __restrict__ dv = dh + (int64_t)b * dh_batch + (int64_t)f * Nd;
    cx<A> acc[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[v] = cx<A>{0, 0};

    for (int c0 = 0; c0 < Nd; c0 += kDChunk) {
        const int ns = min(kDChunk, Nd - c0);
        __syncthreads();
        for (int i = threadIdx.x; i < ns; i += kGemvThreads) dsh[i] = dv[c0 + i];
        __syncthreads();
        if (active) {
            int s = 0;
            for (; s + RB <= ns; s += RB) {
                u32x4 w[RB][2];
#pragma unroll
                for (int r = 0; r < RB; ++r) load32_nt(Ff + (int64_t)(c0 + s + r) * ldF, w[r]);
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    const cx<A> d = dsh[s + r];
#pragma unroll
                    for (int v = 0; v < VEC; ++v) cfmac(acc[v], StorT<S>::get(w[r], v), d);
                }
            }
            for (; s < ns; ++s) {
                u32x4 w[2];
                load32_nt(Ff + (int64_t)(c0 + s) * ldF, w);
                const cx<A> d = dsh[s];
#pragma unroll
                for (int v = 0; v < VEC; ++v) cfmac(acc[v], StorT<S>::get(w, v), d);
            }
        }
    }
    if (active) {
        cx<A>* __restrict__ o = mo + (int64_t)b * mo_batch + (int64_t)f * ldv + col;
#pragma unroll
        for (int v = 0; v < VEC; ++v) o[v] = acc[v];
    }
}

// ----------------------------------------------------------------------------------------
static int stor_vec(Stor st) { return st == Stor::C128 ? 2 : (st == Stor::C64 ? 4 : 8); }

int sbgemv_n_span(Stor st, int64_t Nm) {
    // 4096 columns per span (2048 for FP64), i.e. a 32 KB slice of mh staged in LDS; narrow
    // operators use one span rounded up to whole 64-lane tiles.
    const int tile = kWave * stor_vec(st);
    int64_t cs = (st == Stor::C128) ? 2048 : 4096;
    const int64_t need = ((Nm + tile - 1) / tile) * tile;
    return (int)(cs < need ? cs : need);
}

hipError_t launch_sbgemv_n(Stor st, const void* Fh, int64_t ldF, int nfreq, int Nd, int Nm, const void* mh,
                           int64_t ldv, int64_t mh_batch, int nb, void* part, int nspan, int64_t part_batch,
                           hipStream_t s) {
    const int CS = sbgemv_n_span(st, Nm);
    if (nspan != (Nm + CS - 1) / CS) return hipErrorInvalidValue;
    dim3 grid(nspan, nfreq, nb), block(kGemvThreads);
    constexpr int RB = 4;
    switch (st) {
        case Stor::C128:
            k_sbgemv_n<cx<double>, RB><<<grid, block, CS * sizeof(cx<double>), s>>>(
                (const cx<double>*)Fh, ldF, Nd, Nm, (const cx<double>*)mh, ldv, mh_batch, (cx<double>*)part, CS,
                nspan, part_batch);
            break;
        case Stor::C64:
            k_sbgemv_n<cx<float>, RB><<<grid, block, CS * sizeof(cx<float>), s>>>(
                (const cx<float>*)Fh, ldF, Nd, Nm, (const cx<float>*)mh, ldv, mh_batch, (cx<float>*)part, CS,
                nspan, part_batch);
            break;
        case Stor::BF16:
            k_sbgemv_n<bf16c, RB><<<grid, block, CS * sizeof(cx<float>), s>>>(
                (const bf16c*)Fh, ldF, Nd, Nm, (const cx<float>*)mh, ldv, mh_batch, (cx<float>*)part, CS, nspan,
                part_batch);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_sbgemv_c(Stor st, const void* Fh, int64_t ldF, int nfreq, int Nd, int Nm, const void* dh,
                           int64_t dh_batch, int nb, void* mo, int64_t ldv, int64_t mo_batch, hipStream_t s) {
    const int per = kGemvThreads * stor_vec(st);
    dim3 grid((unsigned)((Nm + per - 1) / per), nfreq, nb), block(kGemvThreads);
    constexpr int RB = 8;
    switch (st) {
        case Stor::C128:
            k_sbgemv_c<cx<double>, RB><<<grid, block, 0, s>>>((const cx<double>*)Fh, ldF, Nd, Nm,
                                                              (const cx<double>*)dh, dh_batch, (cx<double>*)mo,
                                                              ldv, mo_batch);
            break;
        case Stor::C64:
            k_sbgemv_c<cx<float>, RB><<<grid, block, 0, s>>>((const cx<float>*)Fh, ldF, Nd, Nm, (const cx<float>*)dh,
                                                             dh_batch, (cx<float>*)mo, ldv, mo_batch);
            break;
        case Stor::BF16:
            k_sbgemv_c<bf16c, RB><<<grid, block, 0, s>>>((const bf16c*)Fh, ldF, Nd, Nm, (const cx<float>*)dh,
                                                         dh_batch, (cx<float>*)mo, ldv, mo_batch);
            break;
    }
    return hipGetLastError();
}

}  // namespace btoep
