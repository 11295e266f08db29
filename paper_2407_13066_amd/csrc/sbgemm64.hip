// Multi-right-hand-side per-frequency products for the complex FP64 operator, on the FP64
// matrix cores (v_mfma_f64_16x16x4_f64).  Same decomposition as the FP32 kernels of
// sbgemm.hip -- the complex product as one real GEMM with the vector side expanded to
//      [ Re m  Im m ]        (adjoint: [ Re d   Im d ])
//      [-Im m  Re m ]                  [ Im d  -Re d ]
// -- with FP64 operands and FP64 accumulation throughout, so the result keeps the accuracy
// of the single-vector FP64 path while the operator is streamed once for all k vectors.
//
// MFMA 16x16x4 FP64 operand layout (lane l of 64, g = l / 16, i = l % 16):
//   A (16 x 4): lane holds row i, K index g;  B (4 x 16): lane holds column i, K index g;
//   C (16 x 16): lane holds C[g + 4 v][i], v = 0..3 (rows interleaved across the lane groups,
//   unlike the FP32 instruction's C[4 g + v][i]; measured with a probe of the instruction).
#include "common.h"
#include "internal.h"

namespace btoep {

typedef double d4v __attribute__((ext_vector_type(4)));

namespace {

constexpr int kThreads64 = 256;

__device__ __forceinline__ d4v mfma_f64(double a, double b, d4v c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Complex columns of the vector side staged per LDS chunk: two buffers of NT * 8 rows of
// (chunk + 1) 16-byte entries stay within 34 KB.
template <int NT>
struct Chunk64 {
    static constexpr int value = NT >= 4 ? 32 : 64;
};
size_t lds_n64(int NT) {
    const int ch = NT >= 4 ? 32 : 64;
    return (size_t)2 * NT * 8 * (ch + 1) * 16;
}

// N direction.  Grid (nspan, nfreq); 4 waves; wave w owns row tiles 2w, 2w+1 of each group of
// 128 rows; NT tiles of 16 real result columns (8 right-hand sides each).
template <int NT, int kChunk>
__global__ __launch_bounds__(kThreads64) void k_sbgemm_n64(const cx<double>* __restrict__ Fh, int64_t ldF, int Nd,
                                                           int Nm, const cx<double>* __restrict__ mh, int64_t ldv,
                                                           int64_t mh_batch, int nb, cx<double>* __restrict__ part,
                                                           int CS, int nspan, int nfreq, int64_t part_batch) {
    constexpr int LDR = kChunk + 1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<double>* buf = reinterpret_cast<cx<double>*>(smem_raw);  // [2][NT*8][LDR]
    const int span = blockIdx.x, f = blockIdx.y;
    const int col0 = span * CS;
    const int ncol = min(CS, Nm - col0);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int nchunk = (ncol + kChunk - 1) / kChunk;
    constexpr int rows_per_buf = NT * 8;

    typedef double d2v __attribute__((ext_vector_type(2)));
    // Staging of a chunk of the vector side in two halves: with four tiles (where it costs no
    // occupancy) the global loads of chunk c + 1 are issued into registers before chunk c is
    // multiplied and written to LDS after it, so neither their latency nor a wait for them
    // stalls the chunk's MFMAs; narrower tiles store them at once.
    constexpr bool kSplit = NT >= 4;
    constexpr int kPer = rows_per_buf * kChunk / kThreads64;  // staged entries per thread
    static_assert(kPer * kThreads64 == rows_per_buf * kChunk, "chunk entries split evenly over the threads");
    auto stage_load = [&](int c, d2v* v) {
        const int cbase = col0 + c * kChunk;
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int e = threadIdx.x + i * kThreads64;
            const int r = e / kChunk, q = e % kChunk;
            const bool ok = r < nb && cbase + q < col0 + ncol;
            const d2v* src = reinterpret_cast<const d2v*>(mh + (int64_t)min(r, nb - 1) * mh_batch + (int64_t)f * ldv +
                                                          min(cbase + q, col0 + ncol - 1));
            const d2v x = *src;
            v[i] = ok ? x : d2v{0.0, 0.0};
        }
    };
    auto stage = [&](int c, int which) {  // both halves at once, one entry at a time
        d2v* dst = reinterpret_cast<d2v*>(buf + (size_t)which * rows_per_buf * LDR);
        const int cbase = col0 + c * kChunk;
        for (int e = threadIdx.x; e < rows_per_buf * kChunk; e += kThreads64) {
            const int r = e / kChunk, q = e % kChunk;
            const bool ok = r < nb && cbase + q < col0 + ncol;
            const d2v* src = reinterpret_cast<const d2v*>(mh + (int64_t)min(r, nb - 1) * mh_batch + (int64_t)f * ldv +
                                                          min(cbase + q, col0 + ncol - 1));
            const d2v v = *src;
            dst[r * LDR + q] = ok ? v : d2v{0.0, 0.0};
        }
    };
    auto stage_store = [&](int which, const d2v* v) {
        d2v* dst = reinterpret_cast<d2v*>(buf + (size_t)which * rows_per_buf * LDR);
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int e = threadIdx.x + i * kThreads64;
            dst[(e / kChunk) * LDR + e % kChunk] = v[i];
        }
    };
    // Operator values of one K step (16 complex columns) for the wave's two row tiles: lane
    // group lg takes columns 4 q + lg, q = 0..3, so each load instruction reads a 64-byte run
    // of 16 rows.  Columns past the span end read as zero.
    constexpr int KS = kChunk / 16;  // K steps per chunk (even)
    static_assert(KS % 2 == 0, "double-buffered K steps");
    cx<double> A0[2][4], A1[2][4];
    auto loadA = [&](const cx<double>* F0, const cx<double>* F1, int c, int ks, int bsel) {
        const int64_t base = (int64_t)col0 + c * kChunk + ks * 16 + lg;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t col = base + 4 * q;
            const bool in = col < col0 + ncol;
            A0[bsel][q] = in ? F0[col] : cx<double>{0.0, 0.0};
            A1[bsel][q] = in ? F1[col] : cx<double>{0.0, 0.0};
        }
    };

    for (int rg = 0; rg < Nd; rg += 128) {
        const int rt0 = rg + wave * 32;  // first row of this wave's two 16-row tiles
        const bool t0 = rt0 < Nd, t1 = rt0 + 16 < Nd;
        const int s0 = min(rt0 + li, Nd - 1), s1 = min(rt0 + 16 + li, Nd - 1);
        const cx<double>* F0 = Fh + ((int64_t)f * Nd + s0) * ldF;
        const cx<double>* F1 = Fh + ((int64_t)f * Nd + s1) * ldF;
        d4v acc[2][NT];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int n = 0; n < NT; ++n) acc[a][n] = d4v{0.0, 0.0, 0.0, 0.0};

        d2v sv[kSplit ? kPer : 1];
        __syncthreads();
        stage(0, 0);
        // the next K step's operator loads are issued before the current step's MFMAs, also
        // across chunk boundaries (they do not depend on the staged vectors)
        if (t0) loadA(F0, F1, 0, 0, 0);
        for (int c = 0; c < nchunk; ++c) {
            // buffer c & 1 is complete, and every wave is done with buffer (c + 1) & 1
            __syncthreads();
            if (c + 1 < nchunk) {
                if constexpr (kSplit)
                    stage_load(c + 1, sv);
                else
                    stage(c + 1, (c + 1) & 1);
            }
            const cx<double>* B = buf + (size_t)(c & 1) * rows_per_buf * LDR;
            if (t0) {
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) {
                    const int cur = ks & 1;
                    if (ks + 1 < KS)
                        loadA(F0, F1, c, ks + 1, cur ^ 1);
                    else if (c + 1 < nchunk)
                        loadA(F0, F1, c + 1, 0, cur ^ 1);
#pragma unroll
                    for (int n = 0; n < NT; ++n) {
                        const int r = n * 8 + (li >> 1);
                        const bool imcol = li & 1;
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            // K = (column 4 q + lg, part): pairs with Re F and with Im F
                            const cx<double> mv = B[r * LDR + ks * 16 + 4 * q + lg];
                            const double b0 = imcol ? mv.im : mv.re;
                            const double b1 = imcol ? mv.re : -mv.im;
                            acc[0][n] = mfma_f64(A0[cur][q].re, b0, acc[0][n]);
                            acc[0][n] = mfma_f64(A0[cur][q].im, b1, acc[0][n]);
                            if (t1) {
                                acc[1][n] = mfma_f64(A1[cur][q].re, b0, acc[1][n]);
                                acc[1][n] = mfma_f64(A1[cur][q].im, b1, acc[1][n]);
                            }
                        }
                    }
                }
            }
            if constexpr (kSplit)
                if (c + 1 < nchunk) stage_store((c + 1) & 1, sv);
        }
        // C[lg + 4 v][li]: row s = rt0 + 16 a + lg + 4 v, column li -> rhs n*8 + li/2, part li&1
#pragma unroll
        for (int a = 0; a < 2; ++a) {
#pragma unroll
            for (int n = 0; n < NT; ++n) {
                const int r = n * 8 + (li >> 1);
                if (r >= nb) continue;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int s = rt0 + 16 * a + lg + 4 * v;
                    if (s < Nd) {
                        double* o = reinterpret_cast<double*>(part + (int64_t)r * part_batch +
                                                              ((int64_t)s * nfreq + f) * nspan + span);
                        o[li & 1] = acc[a][n][v];
                    }
                }
            }
        }
    }
}

// C direction.  Grid (ceil(Nm / 128), nfreq); 4 waves; wave w owns result columns
// p0 = 128 blockIdx.x + 32 w + [0, 32) as two 16-column tiles; NT row tiles of 16 real
// result rows (8 right-hand sides).  The data spectra of this frequency are staged in LDS.
template <int NT>
__global__ __launch_bounds__(kThreads64) void k_sbgemm_c64(const cx<double>* __restrict__ Fh, int64_t ldF, int Nd,
                                                           int Nm, const cx<double>* __restrict__ dh,
                                                           int64_t dh_batch, int nb, cx<double>* __restrict__ mo,
                                                           int64_t ldv, int64_t mo_batch) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<double>* dsh = reinterpret_cast<cx<double>*>(smem_raw);  // [NT*8][Ndp]
    const int Ndp = (Nd + 3) & ~3;
    const int f = blockIdx.y;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    for (int e = threadIdx.x; e < NT * 8 * Ndp; e += kThreads64) {
        const int r = e / Ndp, s = e % Ndp;
        dsh[e] = (r < nb && s < Nd) ? dh[(int64_t)r * dh_batch + (int64_t)f * Nd + s] : cx<double>{0.0, 0.0};
    }
    __syncthreads();

    const int pbase = blockIdx.x * 128 + wave * 32;
    if (pbase >= Nm) return;
    const int pc[2] = {min(pbase + li, Nm - 1), min(pbase + 16 + li, Nm - 1)};
    const bool tile1 = pbase + 16 < Nm;
    d4v acc[2][NT];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[a][n] = d4v{0.0, 0.0, 0.0, 0.0};

    const int64_t frow = (int64_t)f * Nd;
    // K step: 4 sensor rows (one per lane group) x (re, im): two MFMAs.  The operator loads of
    // the next kPre steps are in flight while a step runs: four with four tiles (9 % faster at
    // k = 32), one with fewer (deeper prefetch measured 3 % slower at k = 8 and 16).
    typedef double d2v __attribute__((ext_vector_type(2)));
    constexpr int kPre = NT >= 4 ? 4 : 1;
    d2v ring[kPre][2];
    auto loadB = [&](int s0, d2v(&dst)[2]) {
        const int sc = min(s0 + lg, Nd - 1);
#pragma unroll
        for (int a = 0; a < 2; ++a)
            dst[a] = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(Fh + (frow + sc) * ldF + pc[a]));
    };
#pragma unroll
    for (int j = 0; j < kPre; ++j)
        if (4 * j < Nd) loadB(4 * j, ring[j]);
    for (int sb = 0; sb < Nd; sb += 4 * kPre) {
#pragma unroll
        for (int j = 0; j < kPre; ++j) {
            const int s0 = sb + 4 * j;
            if (s0 >= Nd) break;
            const bool sv = s0 + lg < Nd;
            cx<double> b[2];
#pragma unroll
            for (int a = 0; a < 2; ++a)
                b[a] = sv ? cx<double>{ring[j][a][0], ring[j][a][1]} : cx<double>{0.0, 0.0};
            if (s0 + 4 * kPre < Nd) loadB(s0 + 4 * kPre, ring[j]);
#pragma unroll
            for (int n = 0; n < NT; ++n) {
                // A row li: rhs n*8 + li/2, part li&1 of the result; K = (s, part of F)
                const cx<double> dv = dsh[(n * 8 + (li >> 1)) * Ndp + s0 + lg];  // zero past Nd
                const bool imrow = li & 1;
                const double a0 = imrow ? dv.im : dv.re;   // pairs with Re F
                const double a1 = imrow ? -dv.re : dv.im;  // pairs with Im F
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    acc[a][n] = mfma_f64(a0, b[a].re, acc[a][n]);
                    acc[a][n] = mfma_f64(a1, b[a].im, acc[a][n]);
                }
            }
        }
    }
    // C[lg + 4 v][li]: result row lg + 4 v -> rhs n*8 + lg/2 + 2 v, part lg&1; column p = tile + li.
    // Lane groups 2 h and 2 h + 1 hold the real and imaginary parts of the same right-hand
    // sides, so each store instruction still covers whole 16-byte values.
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const int p = pbase + 16 * a + li;
        if (p >= Nm || (a == 1 && !tile1)) continue;
#pragma unroll
        for (int n = 0; n < NT; ++n) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = n * 8 + (lg >> 1) + 2 * v;
                if (r < nb) {
                    double* o = reinterpret_cast<double*>(mo + (int64_t)r * mo_batch + (int64_t)f * ldv + p);
                    __builtin_nontemporal_store(acc[a][n][v], o + (lg & 1));
                }
            }
        }
    }
}

int nt64_of(int nb) { return nb <= 8 ? 1 : (nb <= 16 ? 2 : 4); }

}  // namespace

size_t sbgemm_c64_lds(int nb, int Nd) { return (size_t)nt64_of(nb) * 8 * ((Nd + 3) & ~3) * 16; }

hipError_t launch_sbgemm_n64(const void* Fh, int64_t ldF, int nfreq, int Nd, int Nm, const void* mh, int64_t ldv,
                             int64_t mh_batch, int nb, void* part, int nspan, int64_t part_batch, hipStream_t s) {
    if (nb < 1 || nb > kGemmNMax) return hipErrorInvalidValue;
    const int CS = n_span_cols(Stor::C128, Nm, nfreq);  // the single-vector kernel's spans
    if (nspan != (Nm + CS - 1) / CS) return hipErrorInvalidValue;
    const int NT = nt64_of(nb);
    dim3 grid(nspan, nfreq), block(kThreads64);
    const size_t lds = lds_n64(NT);
    const cx<double>* F = (const cx<double>*)Fh;
    const cx<double>* m = (const cx<double>*)mh;
    cx<double>* p = (cx<double>*)part;
    switch (NT) {
        case 1:
            k_sbgemm_n64<1, Chunk64<1>::value><<<grid, block, lds, s>>>(F, ldF, Nd, Nm, m, ldv, mh_batch, nb, p, CS,
                                                                       nspan, nfreq, part_batch);
            break;
        case 2:
            k_sbgemm_n64<2, Chunk64<2>::value><<<grid, block, lds, s>>>(F, ldF, Nd, Nm, m, ldv, mh_batch, nb, p, CS,
                                                                       nspan, nfreq, part_batch);
            break;
        default:
            k_sbgemm_n64<4, Chunk64<4>::value><<<grid, block, lds, s>>>(F, ldF, Nd, Nm, m, ldv, mh_batch, nb, p, CS,
                                                                       nspan, nfreq, part_batch);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_sbgemm_c64(const void* Fh, int64_t ldF, int nfreq, int Nd, int Nm, const void* dh,
                             int64_t dh_batch, int nb, void* mo, int64_t ldv, int64_t mo_batch, hipStream_t s) {
    if (nb < 1 || nb > kGemmNMax) return hipErrorInvalidValue;
    const size_t lds = sbgemm_c64_lds(nb, Nd);
    if (lds > 64 * 1024) return hipErrorInvalidValue;
    const int NT = nt64_of(nb);
    dim3 grid((unsigned)((Nm + 127) / 128), nfreq), block(kThreads64);
    const cx<double>* F = (const cx<double>*)Fh;
    const cx<double>* d = (const cx<double>*)dh;
    cx<double>* o = (cx<double>*)mo;
    switch (NT) {
        case 1: k_sbgemm_c64<1><<<grid, block, lds, s>>>(F, ldF, Nd, Nm, d, dh_batch, nb, o, ldv, mo_batch); break;
        case 2: k_sbgemm_c64<2><<<grid, block, lds, s>>>(F, ldF, Nd, Nm, d, dh_batch, nb, o, ldv, mo_batch); break;
        default: k_sbgemm_c64<4><<<grid, block, lds, s>>>(F, ldF, Nd, Nm, d, dh_batch, nb, o, ldv, mo_batch); break;
    }
    return hipGetLastError();
}

}  // namespace btoep
