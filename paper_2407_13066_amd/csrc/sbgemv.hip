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
//                part[b][s][f][span]; the data-side kernel adds them in a fixed order, so the
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

// 16 bytes of the operator; non-temporal when NTL.
template <bool NTL>
__device__ __forceinline__ u32x4 load16(const void* p) {
    const u32x4* q = reinterpret_cast<const u32x4*>(p);
    return NTL ? __builtin_nontemporal_load(q) : *q;
}

constexpr int kGemvThreads = 256;
constexpr int kGemvWaves = kGemvThreads / kWave;

// Lane data layout.  A wave covers a tile of 64 x VEC columns (2 KB of one operator row) as
// two 1 KB chunks; in chunk h lane l owns the CPL = 16 / sizeof(S) columns starting at
// h * 64 * CPL + l * CPL, so every load instruction reads one fully contiguous 1 KB run.
// Element v of a lane (v = h * CPL + e) is StorT<S>::get(w, v) with w[h] the chunk's load.
template <typename S>
struct Lanes {
    static constexpr int CPL = 16 / (int)sizeof(S);
    static constexpr int VEC = StorT<S>::VEC;
    static constexpr int NCH = VEC / CPL;  // 2
    __device__ static int col(int lane, int v) { return (v / CPL) * kWave * CPL + lane * CPL + (v % CPL); }
    __device__ static int chunk(int lane, int h) { return h * kWave * CPL + lane * CPL; }
};

// ---- N direction ----------------------------------------------------------------------
// Wave w owns row blocks s0 = RB (w + 4 j); for each it walks the span in tiles of 64 lanes x
// VEC columns.  The (row block, tile) iterations are flattened and software-pipelined: the
// loads of iteration i+1 are in flight while iteration i is consumed, so the wave never
// waits for an empty memory pipe (also not across the cross-lane reduction that ends a row
// block).  Partial sums go to part[b][s][f][span].
template <typename S, int RB, bool NTL>
__global__ __launch_bounds__(kGemvThreads) void k_sbgemv_n(const S* __restrict__ Fh, int64_t ldF, int Nd, int Nm,
                                                           const cx<typename StorT<S>::A>* __restrict__ mh,
                                                           int64_t ldv, int64_t mh_batch,
                                                           cx<typename StorT<S>::A>* __restrict__ part,
                                                           int CS, int nspan, int nfreq, int64_t part_batch) {
    typedef typename StorT<S>::A A;
    typedef Lanes<S> LN;
    constexpr int VEC = LN::VEC, CPL = LN::CPL, NCH = LN::NCH;
    constexpr int TILE = kWave * VEC;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<A>* msh = reinterpret_cast<cx<A>*>(smem_raw);

    const int span = blockIdx.x, f = blockIdx.y, b = blockIdx.z;
    const int col0 = span * CS;
    const int ncol = min(CS, Nm - col0);
    const cx<A>* __restrict__ mrow = mh + (int64_t)b * mh_batch + (int64_t)f * ldv + col0;
#pragma unroll 4
    for (int i = threadIdx.x; i < CS; i += kGemvThreads) msh[i] = (i < ncol) ? mrow[i] : cx<A>{0, 0};
    __syncthreads();

    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int ntile = (ncol + TILE - 1) / TILE;
    const int first = wave * RB;
    const int nrb = (first < Nd) ? (Nd - first + kGemvWaves * RB - 1) / (kGemvWaves * RB) : 0;
    const int total = nrb * ntile;
    if (total == 0) return;
    // last chunk start inside the row (chunks past ncol are clamped to it; the staged vector
    // is zero past ncol, so their products add nothing)
    const int last_chunk = ((ncol - 1) / CPL) * CPL;
    const S* __restrict__ Ff = Fh + (int64_t)f * Nd * ldF + col0;
    cx<A>* __restrict__ pout = part + (int64_t)b * part_batch + (int64_t)f * nspan + span;
    const int64_t pstride = (int64_t)nfreq * nspan;

    u32x4 wa[RB][NCH], wb[RB][NCH];
    int ij = 0, it = 0;  // issue pointer (row block, tile)
    auto issue = [&](u32x4(&w)[RB][NCH]) {
        const int s0 = first + ij * kGemvWaves * RB;
        const int base = it * TILE;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const S* row = Ff + (int64_t)min(s0 + r, Nd - 1) * ldF;
#pragma unroll
            for (int h = 0; h < NCH; ++h) w[r][h] = load16<NTL>(row + min(base + LN::chunk(lane, h), last_chunk));
        }
        if (++it == ntile) {
            it = 0;
            ++ij;
        }
    };
    cx<A> acc[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) acc[r] = cx<A>{0, 0};
    int cj = 0, ct = 0;  // consume pointer
    auto consume = [&](const u32x4(&w)[RB][NCH]) {
        const int base = ct * TILE;
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            const cx<A> mv = msh[base + LN::col(lane, v)];
#pragma unroll
            for (int r = 0; r < RB; ++r) cfma(acc[r], StorT<S>::get(w[r], v), mv);
        }
        if (++ct == ntile) {
            const int s0 = first + cj * kGemvWaves * RB;
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const A re = wave_sum(acc[r].re), im = wave_sum(acc[r].im);
                if (lane == 0 && s0 + r < Nd) pout[(int64_t)(s0 + r) * pstride] = cx<A>{re, im};
                acc[r] = cx<A>{0, 0};
            }
            ct = 0;
            ++cj;
        }
    };
    issue(wa);
    for (int i = 0; i < total; i += 2) {
        if (i + 1 < total) issue(wb);
        consume(wa);
        if (i + 1 < total) {
            if (i + 2 < total) issue(wa);
            consume(wb);
        }
    }
}

// ---- C direction ----------------------------------------------------------------------
// Each wave owns a tile of 64 x VEC columns; rows are consumed RB at a time with the next RB
// rows' loads already in flight.  dh_f is staged in LDS zero-padded to a multiple of 2 RB
// rows (rows past Nd load row Nd-1 and are multiplied by zero).
constexpr int kDChunk = 1024;

template <typename S, int RB, bool NTL>
__global__ __launch_bounds__(kGemvThreads) void k_sbgemv_c(const S* __restrict__ Fh, int64_t ldF, int Nd, int Nm,
                                                           const cx<typename StorT<S>::A>* __restrict__ dh,
                                                           int64_t dh_batch,
                                                           cx<typename StorT<S>::A>* __restrict__ mo, int64_t ldv,
                                                           int64_t mo_batch) {
    typedef typename StorT<S>::A A;
    typedef Lanes<S> LN;
    constexpr int VEC = LN::VEC, CPL = LN::CPL, NCH = LN::NCH;
    __shared__ cx<A> dsh[kDChunk];
    const int f = blockIdx.y, b = blockIdx.z;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int tile0 = (blockIdx.x * kGemvWaves + wave) * kWave * VEC;
    const int last_chunk = ((Nm - 1) / CPL) * CPL;
    int cofs[NCH];
    bool valid[NCH];
#pragma unroll
    for (int h = 0; h < NCH; ++h) {
        const int c = tile0 + LN::chunk(lane, h);
        valid[h] = c < Nm;
        cofs[h] = min(c, last_chunk);
    }
    const S* __restrict__ Ff = Fh + (int64_t)f * Nd * ldF;
    const cx<A>* __restrict__ dv = dh + (int64_t)b * dh_batch + (int64_t)f * Nd;
    cx<A> acc[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[v] = cx<A>{0, 0};

    for (int c0 = 0; c0 < Nd; c0 += kDChunk) {
        const int ns = min(kDChunk, Nd - c0);
        const int nsp = (ns + 2 * RB - 1) / (2 * RB) * (2 * RB);  // <= kDChunk: kDChunk is a multiple of 2 RB
        __syncthreads();
        for (int i = threadIdx.x; i < nsp; i += kGemvThreads) dsh[i] = (i < ns) ? dv[c0 + i] : cx<A>{0, 0};
        __syncthreads();
        u32x4 wa[RB][NCH], wb[RB][NCH];
        auto issue = [&](int s, u32x4(&w)[RB][NCH]) {
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const S* row = Ff + (int64_t)min(c0 + s + r, Nd - 1) * ldF;
#pragma unroll
                for (int h = 0; h < NCH; ++h) w[r][h] = load16<NTL>(row + cofs[h]);
            }
        };
        auto consume = [&](int s, const u32x4(&w)[RB][NCH]) {
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const cx<A> d = dsh[s + r];
#pragma unroll
                for (int v = 0; v < VEC; ++v) cfmac(acc[v], StorT<S>::get(w[r], v), d);
            }
        };
        issue(0, wa);
        for (int s = 0; s < nsp; s += 2 * RB) {
            issue(s + RB, wb);
            consume(s, wa);
            if (s + 2 * RB < nsp) issue(s + 2 * RB, wa);
            consume(s + RB, wb);
        }
    }
    // The result spectra are not read again by this launch: 16-byte non-temporal stores (a
    // chunk's CPL values are 16-byte aligned; a chunk that starts before Nm may reach into the
    // zero padding of the row, which stays inside ldv).
    cx<A>* __restrict__ o = mo + (int64_t)b * mo_batch + (int64_t)f * ldv;
#pragma unroll
    for (int h = 0; h < NCH; ++h) {
        if (!valid[h]) continue;
        u32x4* dst = reinterpret_cast<u32x4*>(o + tile0 + LN::chunk(lane, h));
        if constexpr (sizeof(A) == 4) {
#pragma unroll
            for (int q = 0; q < CPL / 2; ++q) {
                const cx<A> x0 = acc[h * CPL + 2 * q], x1 = acc[h * CPL + 2 * q + 1];
                const u32x4 w = {__float_as_uint(x0.re), __float_as_uint(x0.im), __float_as_uint(x1.re),
                                 __float_as_uint(x1.im)};
                __builtin_nontemporal_store(w, dst + q);
            }
        } else {
#pragma unroll
            for (int q = 0; q < CPL; ++q) {
                const cx<A> x = acc[h * CPL + q];
                const u32x4 w = {(unsigned)__double2loint(x.re), (unsigned)__double2hiint(x.re),
                                 (unsigned)__double2loint(x.im), (unsigned)__double2hiint(x.im)};
                __builtin_nontemporal_store(w, dst + q);
            }
        }
    }
}

// ----------------------------------------------------------------------------------------
static int stor_vec(Stor st) { return st == Stor::C128 ? 2 : (st == Stor::C64 ? 4 : 8); }

int n_span_cols(Stor st, int64_t Nm, int nfreq) {
    // 4096 columns per span (2048 for FP64), i.e. a 32 KB slice of mh staged in LDS, halved
    // (down to 512) while a launch would have fewer than 2048 (span, frequency) workgroups, so
    // that small operators still spread over the chip; an operator narrower than one span uses
    // one span rounded up to whole 64-lane tiles.
    const int tile = kWave * stor_vec(st);
    int64_t cs = (st == Stor::C128) ? 2048 : 4096;
    while (cs > 512 && ((Nm + cs - 1) / cs) * nfreq < 2048) cs /= 2;
    const int64_t need = ((Nm + tile - 1) / tile) * tile;
    return (int)(cs < need ? cs : need);
}

// Variant ids: bit 0 = non-temporal operator loads; bits 1.. = row-block index (N: RB 2/4/8,
// C: RB 4/8/16).  The default is what the autotuner measured best on MI355X.
int sbgemv_variants() { return 6; }

template <typename S, typename A>
static hipError_t run_n(int var, dim3 grid, size_t lds, hipStream_t s, const void* Fh, int64_t ldF, int Nd, int Nm,
                        const void* mh, int64_t ldv, int64_t mh_batch, void* part, int CS, int nspan, int nfreq,
                        int64_t part_batch) {
#define BT_N(RBV, NTV)                                                                                         \
    k_sbgemv_n<S, RBV, NTV><<<grid, kGemvThreads, lds, s>>>((const S*)Fh, ldF, Nd, Nm, (const cx<A>*)mh, ldv, \
                                                            mh_batch, (cx<A>*)part, CS, nspan, nfreq, part_batch)
    switch (var) {
        case 0: BT_N(2, false); break;
        case 1: BT_N(2, true); break;
        case 2: BT_N(4, false); break;
        case 3: BT_N(4, true); break;
        case 4: BT_N(8, false); break;
        default: BT_N(8, true); break;
    }
#undef BT_N
    return hipGetLastError();
}

template <typename S, typename A>
static hipError_t run_c(int var, dim3 grid, hipStream_t s, const void* Fh, int64_t ldF, int Nd, int Nm, const void* dh,
                        int64_t dh_batch, void* mo, int64_t ldv, int64_t mo_batch) {
#define BT_C(RBV, NTV)                                                                                          \
    k_sbgemv_c<S, RBV, NTV><<<grid, kGemvThreads, 0, s>>>((const S*)Fh, ldF, Nd, Nm, (const cx<A>*)dh, dh_batch, \
                                                          (cx<A>*)mo, ldv, mo_batch)
    switch (var) {
        case 0: BT_C(4, false); break;
        case 1: BT_C(4, true); break;
        case 2: BT_C(8, false); break;
        case 3: BT_C(8, true); break;
        case 4: BT_C(16, false); break;
        default: BT_C(16, true); break;
    }
#undef BT_C
    return hipGetLastError();
}

hipError_t launch_sbgemv_n(Stor st, const void* Fh, int64_t ldF, int nfreq, int Nd, int Nm, const void* mh,
                           int64_t ldv, int64_t mh_batch, int nb, void* part, int nspan, int64_t part_batch,
                           hipStream_t s, int var) {
    const int CS = n_span_cols(st, Nm, nfreq);
    if (nspan != (Nm + CS - 1) / CS || var < 0 || var >= sbgemv_variants()) return hipErrorInvalidValue;
    dim3 grid(nspan, nfreq, nb);
    switch (st) {
        case Stor::C128:
            return run_n<cx<double>, double>(var, grid, CS * sizeof(cx<double>), s, Fh, ldF, Nd, Nm, mh, ldv,
                                             mh_batch, part, CS, nspan, nfreq, part_batch);
        case Stor::C64:
            return run_n<cx<float>, float>(var, grid, CS * sizeof(cx<float>), s, Fh, ldF, Nd, Nm, mh, ldv, mh_batch,
                                           part, CS, nspan, nfreq, part_batch);
        case Stor::BF16:
            return run_n<bf16c, float>(var, grid, CS * sizeof(cx<float>), s, Fh, ldF, Nd, Nm, mh, ldv, mh_batch,
                                       part, CS, nspan, nfreq, part_batch);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_sbgemv_c(Stor st, const void* Fh, int64_t ldF, int nfreq, int Nd, int Nm, const void* dh,
                           int64_t dh_batch, int nb, void* mo, int64_t ldv, int64_t mo_batch, hipStream_t s, int var) {
    if (var < 0 || var >= sbgemv_variants()) return hipErrorInvalidValue;
    const int per = kGemvThreads * stor_vec(st);
    dim3 grid((unsigned)((Nm + per - 1) / per), nfreq, nb);
    switch (st) {
        case Stor::C128:
            return run_c<cx<double>, double>(var, grid, s, Fh, ldF, Nd, Nm, dh, dh_batch, mo, ldv, mo_batch);
        case Stor::C64:
            return run_c<cx<float>, float>(var, grid, s, Fh, ldF, Nd, Nm, dh, dh_batch, mo, ldv, mo_batch);
        case Stor::BF16:
            return run_c<bf16c, float>(var, grid, s, Fh, ldF, Nd, Nm, dh, dh_batch, mo, ldv, mo_batch);
    }
    return hipErrorInvalidValue;
}

}  // namespace btoep
