// Multi-right-hand-side per-frequency products on the matrix cores (MFMA).
//
// With k right-hand sides stacked, the per-frequency matrix-vector product of the paper's
// "apply_matrix" step (section 3.3) becomes a matrix-matrix product per frequency, so the
// stored operator is streamed once for all k vectors instead of k times.  A complex
// product is run as one real GEMM: with the operator row read as interleaved (re, im)
// pairs along K, the vector side is expanded on the fly to
//      [ Re m  Im m ]                      (rows: re / im part of the operator entry,
//      [-Im m  Re m ]                       columns: re / im part of the result)
// so that a real MFMA accumulates Re(F m) and Im(F m) directly.  The adjoint uses the
// conjugate-transposed pattern [[Re d, Im d], [Im d, -Re d]] (eq. AdjointFFTMatvec).
//
//   N (for F):  C_f (Nd x 2k) += Fh_f (Nd x 2Nm) B_f (2Nm x 2k), split over column spans
//               (partial sums part[r][s][f][span], summed in order by the data-side kernel).
//               A workgroup keeps the whole Nd x 2k accumulator of its span in registers
//               and streams the right-hand sides through LDS in chunks (256 or 64 columns
//               for one tile of 8 right-hand sides; 128 / NT columns of ready-made operand
//               patterns for NT = 2, 4 or 8 tiles).  Up to 64 right-hand sides per launch.
//   C (for F^T): O_f^T (2k x Nm) = D_f^T (2k x 2Nd) Fh_f (2Nd x Nm): the operator is the
//               B operand, lanes own output columns p, so each result row of 16 p values
//               is stored as one contiguous run; no reduction across workgroups.  The data
//               spectra of the frequency are staged in LDS as ready-made A operands.
//
// Three product modes (template parameter MODE):
//   kF32   FP32 storage on v_mfma_f32_16x16x4_f32 (FP32 operands);
//   kBF16  BF16 storage on v_mfma_f32_16x16x32_bf16, with the FP32 vector operand split into a
//          BF16 high part and a BF16 remainder (two MFMAs), so the vector keeps ~16 significant
//          bits and the result error is dominated by the BF16 rounding of the stored operator;
//   kSplit FP32 storage on the BF16 matrix cores: the FP32 operator is split the same way as
//          it is loaded (hardware round-to-nearest-even conversions), and the product keeps
//          the three terms hi*hi + hi*lo + lo*hi (three MFMAs, each ~16x the FP32 MFMA rate);
//          the dropped lo*lo term and the remainders' rounding leave a relative error of
//          about 2^-17 per product, averaging to a few 1e-6 over the sums.
// Accumulation is FP32 in all three.
//
// MFMA 16x16 operand layout used (lane l of 64, g = l / 16, i = l % 16):
//   A (16 x K): lane holds row i, K group g;  B (K x 16): lane holds column i, K group g;
//   C (16 x 16): lane holds C[4 g + v][i], v = 0..3.
// Any fixed assignment of K indices to (group, item) is valid as long as A and B agree.
#include <algorithm>

#include "common.h"
#include "internal.h"

namespace btoep {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef __bf16 bf2v __attribute__((ext_vector_type(2)));
typedef float f2v_t __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kF32 = 0, kBF16 = 1, kSplit = 2;

constexpr int kGemmThreads = 256;
// Complex columns of the vector side staged per LDS chunk (N direction).  On wide launches the
// narrow tiles take 2 KB of every operator row per chunk (long runs per DRAM page), halved with
// each doubling of the tile so that two chunk buffers stay within 33 KB of LDS; narrow launches
// keep 64 columns (17 KB or less, so more workgroups fit a CU).
template <int NT, bool WIDE>
struct Chunk {
    static constexpr int value = NT >= 2 ? 128 / NT : (WIDE ? 256 : 64);
};
// With several tiles the vector side is staged as ready-made B-operand patterns (twice the
// bytes of the plain entries, see k_sbgemm_n), so the chunk holds 128 / NT columns.
static constexpr bool pat_of(int NT, int ch) { return NT >= 2 && ch * NT <= 128; }
// BF16 / split staging of operand patterns ("slot layout"): for a tile n of 8 right-hand sides
// and a group g of 4 K columns (or sensors), a 256-byte block of 16 slots, slot i holding the
// 4 pattern words that lane li = i ^ swizzle(g) needs for its MFMA operand: one block per
// (n, g) for the high parts and, a plane further on, one for the remainders.  The 16 lanes of a
// lane group read one block (256 contiguous bytes: no bank conflicts in any lane grouping);
// the swizzle moves the group's two low bits into slot bits 0 and 2 so that the scattered
// 4-byte writes of the staging hit distinct banks across 32 lanes.
__device__ __forceinline__ int pat_slot(int i, int g) { return i ^ ((g & 1) | ((g & 2) << 1)); }
// Bytes of one staged plane for NT tiles and G groups; a buffer holds two planes.
static constexpr int pat_plane_bytes(int NT, int G) { return NT * G * 256; }
static constexpr int chunk_of(int NT, bool wide) { return NT >= 2 ? 128 / NT : (wide ? 256 : 64); }
static_assert(Chunk<1, true>::value == chunk_of(1, true) && Chunk<1, false>::value == chunk_of(1, false) &&
                  Chunk<2, true>::value == chunk_of(2, true) && Chunk<4, false>::value == chunk_of(4, false) &&
                  Chunk<8, true>::value == chunk_of(8, true),
              "host and kernel chunk sizes");
static size_t sbgemm_n_lds(int NT, int ch, bool bf) {
    if (pat_of(NT, ch)) return bf ? (size_t)2 * 2 * pat_plane_bytes(NT, ch / 4) : (size_t)2 * NT * 8 * (ch + 1) * 16;
    return (size_t)2 * NT * 8 * (ch + 2) * 8;
}
// Launches with fewer (span, frequency) workgroups than this keep 64-column chunks, whose
// smaller LDS footprint lets more workgroups share a CU.
constexpr int64_t kWideGrid = 4096;
// Waves per workgroup of the C kernel: the staged data spectra (NT * 8 rows) are shared by
// 8 waves once they are large.
template <int NT>
struct CWaves {
    static constexpr int value = NT >= 4 ? 8 : 4;
};

// Operator loads of the adjoint kernel: streamed once per application, so non-temporal (they
// should not evict the staged data spectra from the caches).  The N kernel measured faster
// with ordinary loads.
__device__ __forceinline__ uint2 ld_nt8(const void* p) {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    const u32x2 v = __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(p));
    return uint2{v[0], v[1]};
}
__device__ __forceinline__ uint32_t ld_nt4(const void* p) {
    return __builtin_nontemporal_load(reinterpret_cast<const uint32_t*>(p));
}

__device__ __forceinline__ f4v mfma_f32(float a, float b, f4v c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4v mfma_bf16(u32x4 a, u32x4 b, f4v c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8v, a), __builtin_bit_cast(bf8v, b), c, 0,
                                                   0, 0);
}

// (re, im) of an FP32 complex value (raw bits) as packed bf16 high parts and remainders
// (re | im << 16), with the packed round-to-nearest-even conversion of gfx950; the remainder
// re - hi is exact in FP32.  Returns (hi, lo).
__device__ __forceinline__ uint2 split_bf16_hw(uint32_t re_bits, uint32_t im_bits) {
    const f2v_t x = {__uint_as_float(re_bits), __uint_as_float(im_bits)};
    const uint32_t hi = __builtin_bit_cast(uint32_t, __builtin_convertvector(x, bf2v));
    const f2v_t r = {x[0] - __uint_as_float(hi << 16), x[1] - __uint_as_float(hi & 0xffff0000u)};
    return uint2{hi, __builtin_bit_cast(uint32_t, __builtin_convertvector(r, bf2v))};
}

// From a packed bf16 pair (re | im << 16): (re, -im) and (im, re).
__device__ __forceinline__ uint32_t bf_re_negim(uint32_t x) { return x ^ 0x80000000u; }
__device__ __forceinline__ uint32_t bf_im_re(uint32_t x) { return (x >> 16) | (x << 16); }
// (im, -re) for the adjoint pattern.
__device__ __forceinline__ uint32_t bf_im_negre(uint32_t x) { return ((x >> 16) | (x << 16)) ^ 0x80000000u; }

// =========================================================================================
// N direction.  Grid (nspan, nfreq); 4 waves; wave w owns row tiles 2w, 2w+1 of each group
// of 128 rows; NT tiles of 16 real result columns (8 right-hand sides each).
// LDS: two chunk buffers of nb x kChunk vector entries.  An entry is the column's value as
// staged (8 bytes: float complex, or (hi, lo) packed bf16 pairs; row stride kChunk + 2) or,
// with PAT, both B-operand patterns a lane can need: FP32 mode 16 bytes per column (row stride
// kChunk + 1), lanes of even result column (real part) taking the first 8 bytes, lanes of odd
// column the second; BF16 and split modes (GP) the slot layout (pat_slot): a lane's B operands
// are two aligned 16-byte LDS reads, and the inner loop has no pattern arithmetic.
template <int MODE, int NT, int kChunk, int OCC>
__global__ __launch_bounds__(kGemmThreads) __attribute__((amdgpu_waves_per_eu(OCC))) void k_sbgemm_n(const void* __restrict__ Fh_, int64_t ldF, int Nd, int Nm,
                                                           const cx<float>* __restrict__ mh, int64_t ldv,
                                                           int64_t mh_batch, int nb, cx<float>* __restrict__ part,
                                                           int CS, int nspan, int nfreq, int64_t part_batch) {
    constexpr bool PAT = pat_of(NT, kChunk);
    constexpr bool BF = MODE != kF32;                 // vector side staged as bf16 (hi, lo)
    constexpr bool GP = PAT && BF;                    // slot layout of ready-made patterns
    constexpr int SB = MODE == kBF16 ? 4 : 8;         // bytes of a stored operator entry
    constexpr int LDR = PAT ? kChunk + 1 : kChunk + 2;  // row stride (entries) of a staged chunk
    constexpr int GPL = pat_plane_bytes(NT, kChunk / 4);  // bytes of a GP plane
    extern __shared__ __align__(16) unsigned char smem_raw[];
    uint2* buf = reinterpret_cast<uint2*>(smem_raw);   // [2][NT*8][LDR] 8-byte entries
    uint4* buf4 = reinterpret_cast<uint4*>(smem_raw);  // [2][NT*8][LDR] 16-byte entries (PAT)
    const int span = blockIdx.x, f = blockIdx.y;
    const int col0 = span * CS;
    const int ncol = min(CS, Nm - col0);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: scalar branches
    const int li = lane & 15, lg = lane >> 4;
    const int nchunk = (ncol + kChunk - 1) / kChunk;
    const int rows_per_buf = NT * 8;

    // Staging of a chunk of the vector side in two halves: the global loads of chunk c + 1 are
    // issued into registers before chunk c is multiplied and written to LDS after it, so their
    // latency is hidden behind the chunk's MFMAs.
    constexpr int kPer = NT * 8 * kChunk / kGemmThreads;  // staged entries per thread
    static_assert(kPer * kGemmThreads == NT * 8 * kChunk, "chunk entries split evenly over the threads");
    auto stage_load = [&](int c, cx<float>* v) {
        const int cbase = col0 + c * kChunk;
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int e = threadIdx.x + i * kGemmThreads;
            const int r = e / kChunk, q = e % kChunk;
            v[i] = cx<float>{0.f, 0.f};
            if (r < nb && cbase + q < col0 + ncol) v[i] = mh[(int64_t)r * mh_batch + (int64_t)f * ldv + cbase + q];
        }
    };
    auto stage_store = [&](int which, const cx<float>* v) {
        if constexpr (GP) {
            // entry (r, q) -> word q % 4 of the slots of lanes 2 (r % 8) (real-part column) and
            // 2 (r % 8) + 1 (imaginary-part column) in block (r / 8, q / 4); the loads above stay
            // lane-contiguous (coalesced), the scatter happens in the LDS writes
#pragma unroll
            for (int i = 0; i < kPer; ++i) {
                const int e = threadIdx.x + i * kGemmThreads;
                const int r = e / kChunk, q = e % kChunk;
                const int g = q >> 2;
                const uint2 h = split_bf16_hw(__float_as_uint(v[i].re), __float_as_uint(v[i].im));
                unsigned char* blk = smem_raw + (size_t)which * 2 * GPL + ((r >> 3) * (kChunk / 4) + g) * 256 + (q & 3) * 4;
                // (Re m, -Im m) pairs with (Re F, Im F) for a real-part column, (Im m, Re m) for
                // an imaginary-part column
                uint32_t* d0 = reinterpret_cast<uint32_t*>(blk + pat_slot(2 * (r & 7), g) * 16);
                uint32_t* d1 = reinterpret_cast<uint32_t*>(blk + pat_slot(2 * (r & 7) + 1, g) * 16);
                d0[0] = bf_re_negim(h.x);
                d0[GPL / 4] = bf_re_negim(h.y);
                d1[0] = bf_im_re(h.x);
                d1[GPL / 4] = bf_im_re(h.y);
            }
            return;
        }
        uint2* dst = buf + (size_t)which * rows_per_buf * LDR;
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int e = threadIdx.x + i * kGemmThreads;
            const int r = e / kChunk, q = e % kChunk;
            const float re = v[i].re, im = v[i].im;
            if constexpr (PAT) {
                // (pairs with Re F, pairs with Im F) for a real-part column, then for an
                // imaginary-part column: (Re m, -Im m), (Im m, Re m)
                uint4 out;
                if (BF) {
                    const uint2 h = split_bf16_hw(__float_as_uint(re), __float_as_uint(im));
                    out = uint4{bf_re_negim(h.x), bf_re_negim(h.y), bf_im_re(h.x), bf_im_re(h.y)};
                } else {
                    out = uint4{__float_as_uint(re), __float_as_uint(-im), __float_as_uint(im), __float_as_uint(re)};
                }
                buf4[(size_t)which * rows_per_buf * LDR + r * LDR + q] = out;
            } else {
                uint2 out;
                if (BF) {
                    out = split_bf16_hw(__float_as_uint(re), __float_as_uint(im));
                } else {
                    out.x = __float_as_uint(re);
                    out.y = __float_as_uint(im);
                }
                dst[r * LDR + q] = out;
            }
        }
    };

    for (int rg = 0; rg < Nd; rg += 128) {
        const int rt0 = rg + wave * 32;  // first row of this wave's two 16-row tiles
        const bool t0 = rt0 < Nd;
        const int s0 = min(rt0 + li, Nd - 1), s1 = min(rt0 + 16 + li, Nd - 1);
        const char* F0 = (const char*)Fh_ + ((int64_t)f * Nd + s0) * ldF * SB;
        const char* F1 = (const char*)Fh_ + ((int64_t)f * Nd + s1) * ldF * SB;
        f4v acc[2][NT];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int n = 0; n < NT; ++n) acc[a][n] = f4v{0.f, 0.f, 0.f, 0.f};

        // BF16 / split modes: the raw operator words of a K step (16-byte groups of 4 columns,
        // rows s0 and s1), loaded one K step ahead -- across chunk boundaries too -- so their
        // latency overlaps the current step's matrix-core work.
        constexpr int WPA = MODE == kSplit ? 2 : 1;  // 16-byte words per row and K step
        // (row s0 words 0 / 1, row s1 words 0 / 1); the second words are used in split mode only
        u32x4 c00, c01, c10, c11, n00, n01, n10, n11;
        auto loadA = [&](int c, int ks, u32x4& w00, u32x4& w01, u32x4& w10, u32x4& w11) {
            const int64_t col = col0 + c * kChunk + ks * 16 + lg * 4;
            const u32x4 z = {0u, 0u, 0u, 0u};
            const bool in = col < col0 + ncol;
            const u32x4* p0 = reinterpret_cast<const u32x4*>(F0 + col * SB);
            const u32x4* p1 = reinterpret_cast<const u32x4*>(F1 + col * SB);
            w00 = in ? p0[0] : z;
            w10 = in ? p1[0] : z;
            if constexpr (WPA == 2) {
                w01 = in ? p0[1] : z;
                w11 = in ? p1[1] : z;
            }
        };
        if constexpr (BF)
            if (t0) loadA(0, 0, c00, c01, c10, c11);

        cx<float> sv[kPer];
        __syncthreads();
        stage_load(0, sv);
        stage_store(0, sv);
        for (int c = 0; c < nchunk; ++c) {
            // buffer c & 1 is complete, and every wave is done with buffer (c + 1) & 1
            __syncthreads();
            if (c + 1 < nchunk) stage_load(c + 1, sv);
            const uint2* B = buf + (size_t)(c & 1) * rows_per_buf * LDR;
            const uint4* B4 = buf4 + (size_t)(c & 1) * rows_per_buf * LDR;
            const int cb = col0 + c * kChunk;  // first complex column of the chunk
            if (t0) {
                // K step = 16 complex columns; lane group lg covers columns 4 lg .. 4 lg + 3
#pragma unroll
                for (int ks = 0; ks < kChunk / 16; ++ks) {
                    const int q0 = ks * 16 + lg * 4;       // column within the chunk
                    const int64_t col = cb + q0;           // operator column
                    const bool in = (col < col0 + ncol);   // whole 4-column group lies past the end otherwise
                    if constexpr (!BF) {
                        float a0[8], a1[8];
                        if (in) {
                            const u32x4* p0 = (const u32x4*)(F0 + col * 8);
                            const u32x4 w0 = p0[0], w1 = p0[1];
                            const u32x4* p1 = (const u32x4*)(F1 + col * 8);
                            const u32x4 x0 = p1[0], x1 = p1[1];
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                a0[e] = __uint_as_float(w0[e]);
                                a0[4 + e] = __uint_as_float(w1[e]);
                                a1[e] = __uint_as_float(x0[e]);
                                a1[4 + e] = __uint_as_float(x1[e]);
                            }
                        } else {
#pragma unroll
                            for (int e = 0; e < 8; ++e) a0[e] = a1[e] = 0.f;
                        }
#pragma unroll
                        for (int n = 0; n < NT; ++n) {
                            const int r = n * 8 + (li >> 1);
                            const bool imcol = li & 1;
#pragma unroll
                            for (int q = 0; q < 4; ++q) {
                                // K = (column q, part c): c = 0 real, c = 1 imaginary part of F
                                float b0, b1;  // pair with Re F, with Im F
                                if constexpr (PAT) {
                                    const uint2 pv = reinterpret_cast<const uint2*>(B4 + r * LDR + q0 + q)[imcol];
                                    b0 = __uint_as_float(pv.x);
                                    b1 = __uint_as_float(pv.y);
                                } else {
                                    const uint2 mv = B[r * LDR + q0 + q];
                                    const float mre = __uint_as_float(mv.x), mim = __uint_as_float(mv.y);
                                    b0 = imcol ? mim : mre;
                                    b1 = imcol ? mre : -mim;
                                }
                                // the second tile is computed even past Nd (rows clamped to a
                                // valid one, results not stored): no divergent accumulators
                                acc[0][n] = mfma_f32(a0[2 * q], b0, acc[0][n]);
                                acc[0][n] = mfma_f32(a0[2 * q + 1], b1, acc[0][n]);
                                acc[1][n] = mfma_f32(a1[2 * q], b0, acc[1][n]);
                                acc[1][n] = mfma_f32(a1[2 * q + 1], b1, acc[1][n]);
                            }
                        }
                    } else {
                        // A operand: 4 complex operator entries of this lane group's columns,
                        // K order (column q, re / im); kSplit also keeps the remainders.  The
                        // next step's operator words are requested first.
                        if (ks + 1 < kChunk / 16)
                            loadA(c, ks + 1, n00, n01, n10, n11);
                        else if (c + 1 < nchunk)
                            loadA(c + 1, 0, n00, n01, n10, n11);
                        u32x4 a0, a1, a0l = {0u, 0u, 0u, 0u}, a1l = {0u, 0u, 0u, 0u};
                        if constexpr (MODE == kBF16) {
                            a0 = c00;
                            a1 = c10;
                        } else {
#pragma unroll
                            for (int e = 0; e < 2; ++e) {
                                uint2 h = split_bf16_hw(c00[2 * e], c00[2 * e + 1]);
                                a0[e] = h.x;
                                a0l[e] = h.y;
                                h = split_bf16_hw(c01[2 * e], c01[2 * e + 1]);
                                a0[2 + e] = h.x;
                                a0l[2 + e] = h.y;
                                h = split_bf16_hw(c10[2 * e], c10[2 * e + 1]);
                                a1[e] = h.x;
                                a1l[e] = h.y;
                                h = split_bf16_hw(c11[2 * e], c11[2 * e + 1]);
                                a1[2 + e] = h.x;
                                a1l[2 + e] = h.y;
                            }
                        }
#pragma unroll
                        for (int n = 0; n < NT; ++n) {
                            const int r = n * 8 + (li >> 1);
                            const bool imcol = li & 1;
                            u32x4 bh, bl;
                            if constexpr (GP) {
                                const int g = q0 >> 2;
                                const u32x4* pb = reinterpret_cast<const u32x4*>(
                                    smem_raw + (size_t)(c & 1) * 2 * GPL + (n * (kChunk / 4) + g) * 256 + pat_slot(li, g) * 16);
                                bh = pb[0];
                                bl = pb[GPL / 16];
                            } else {
#pragma unroll
                                for (int q = 0; q < 4; ++q) {
                                    const uint2 mv = B[r * LDR + q0 + q];
                                    bh[q] = imcol ? bf_im_re(mv.x) : bf_re_negim(mv.x);
                                    bl[q] = imcol ? bf_im_re(mv.y) : bf_re_negim(mv.y);
                                }
                            }
                            acc[0][n] = mfma_bf16(a0, bh, acc[0][n]);
                            acc[0][n] = mfma_bf16(a0, bl, acc[0][n]);
                            if constexpr (MODE == kSplit) acc[0][n] = mfma_bf16(a0l, bh, acc[0][n]);
                            acc[1][n] = mfma_bf16(a1, bh, acc[1][n]);
                            acc[1][n] = mfma_bf16(a1, bl, acc[1][n]);
                            if constexpr (MODE == kSplit) acc[1][n] = mfma_bf16(a1l, bh, acc[1][n]);
                        }
                        c00 = n00;
                        c10 = n10;
                        if constexpr (WPA == 2) {
                            c01 = n01;
                            c11 = n11;
                        }
                    }
                }
            }
            if (c + 1 < nchunk) stage_store((c + 1) & 1, sv);
        }
        // C[4 lg + v][li]: row s = rt0 + 16 a + 4 lg + v, column li -> rhs n*8 + li/2, part li&1
#pragma unroll
        for (int a = 0; a < 2; ++a) {
#pragma unroll
            for (int n = 0; n < NT; ++n) {
                const int r = n * 8 + (li >> 1);
                if (r >= nb) continue;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int s = rt0 + 16 * a + 4 * lg + v;
                    if (s < Nd) {
                        float* o = reinterpret_cast<float*>(part + (int64_t)r * part_batch +
                                                            ((int64_t)s * nfreq + f) * nspan + span);
                        o[li & 1] = acc[a][n][v];
                    }
                }
            }
        }
    }
}

// =========================================================================================
// C direction.  Grid (ceil(Nm / (32 W)), nfreq); W waves; wave w owns result columns
// p0 = 32 W blockIdx.x + 32 w + [0, 32) as two 16-column tiles; NT row tiles of 16 real
// result rows (8 right-hand sides).  The data spectra dh[r][f][s] of this frequency are staged
// in LDS (as the A operand's source), kStageUnroll loads per thread in flight at a time.
//   FP32 mode: all Nd sensors at once, one 8-byte entry per (r, s); a lane forms the
//     imaginary-row pattern itself.
//   BF16 / split modes: both A-operand patterns ready-made in the slot layout (pat_slot; the
//     rows of a tile are (right-hand side, real / imaginary part) as the lanes li), so a lane's
//     A operands are two aligned 16-byte LDS reads and the inner loop has no pattern
//     arithmetic; staged c_phase_sensors(NT) sensors at a time (the LDS bound), with a barrier
//     between phases.
// PF (BF16 and split modes): 1 issues the operator loads of the next K step before the current
// step's matrix-core work, so one more step of the operator stream is in flight per wave; the
// first step's loads are then issued before the staging.
constexpr int kStageUnroll = 8;
static constexpr int c_phase_sensors(int NT) {
    // largest multiple of 16 with two planes of NT tiles x KH / 4 groups within 64 KB
    return (65536 / (2 * NT * 256)) * 4 / 16 * 16;
}

template <int MODE, int NT, int W, int PF>
__global__ __launch_bounds__(64 * W) void k_sbgemm_c(const void* __restrict__ Fh_, int64_t ldF, int Nd, int Nm,
                                                           const cx<float>* __restrict__ dh, int64_t dh_batch, int nb,
                                                           cx<float>* __restrict__ mo, int64_t ldv, int64_t mo_batch) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int Ndp = (Nd + 15) & ~15;
    const int f = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: scalar branches
    const int li = lane & 15, lg = lane >> 4;
    const int64_t frow = (int64_t)f * Nd;
    const int pbase = blockIdx.x * (32 * W) + wave * 32;
    // the two operator columns this lane reads (clamped: always a valid address)
    const int pc[2] = {min(pbase + li, Nm - 1), min(pbase + 16 + li, Nm - 1)};
    const bool tile1 = pbase + 16 < Nm;
    const bool live = pbase < Nm;
    f4v acc[2][NT];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[a][n] = f4v{0.f, 0.f, 0.f, 0.f};

    if constexpr (MODE == kF32) {
        uint2* dsh = reinterpret_cast<uint2*>(smem_raw);  // [NT*8][Ndp] float complex
        const int total = NT * 8 * Ndp;
        for (int e0 = threadIdx.x; e0 < total; e0 += kStageUnroll * 64 * W) {
            cx<float> v[kStageUnroll];
#pragma unroll
            for (int u = 0; u < kStageUnroll; ++u) {
                const int e = e0 + u * 64 * W;
                const int r = e / Ndp, s = e % Ndp;
                v[u] = cx<float>{0.f, 0.f};
                if (e < total && r < nb && s < Nd) v[u] = dh[(int64_t)r * dh_batch + (int64_t)f * Nd + s];
            }
#pragma unroll
            for (int u = 0; u < kStageUnroll; ++u) {
                const int e = e0 + u * 64 * W;
                if (e < total) dsh[e] = uint2{__float_as_uint(v[u].re), __float_as_uint(v[u].im)};
            }
        }
        __syncthreads();
        if (!live) return;
        const cx<float>* Fh = (const cx<float>*)Fh_;
        // K step: 4 sensor rows (one per lane group) x (re, im): two MFMAs.  The operator loads
        // of the next kPre steps are in flight while a step runs.
        constexpr int kPre = NT >= 4 ? 4 : 1;
        uint2 ring[kPre][2];
        auto loadB = [&](int s0, uint2(&dst)[2]) {
            const int sc = min(s0 + lg, Nd - 1);
#pragma unroll
            for (int a = 0; a < 2; ++a) dst[a] = ld_nt8(Fh + (frow + sc) * ldF + pc[a]);
        };
#pragma unroll
        for (int j = 0; j < kPre; ++j)
            if (4 * j < Nd) loadB(4 * j, ring[j]);
        for (int sb = 0; sb < Nd; sb += 4 * kPre) {
#pragma unroll
            for (int j = 0; j < kPre; ++j) {
                const int s0 = sb + 4 * j;
                if (s0 >= Nd) break;
                const int s = s0 + lg;
                const bool sv = s < Nd;
                cx<float> b[2];
#pragma unroll
                for (int a = 0; a < 2; ++a)
                    b[a] = sv ? cx<float>{__uint_as_float(ring[j][a].x), __uint_as_float(ring[j][a].y)}
                              : cx<float>{0.f, 0.f};
                if (s0 + 4 * kPre < Nd) loadB(s0 + 4 * kPre, ring[j]);
#pragma unroll
                for (int n = 0; n < NT; ++n) {
                    // A row li: rhs n*8 + li/2, part li&1 of the result; K = (s, c)
                    const uint2 dv = dsh[(n * 8 + (li >> 1)) * Ndp + (sv ? s : 0)];
                    const float dre = sv ? __uint_as_float(dv.x) : 0.f, dim = sv ? __uint_as_float(dv.y) : 0.f;
                    const bool imrow = li & 1;
                    const float a0 = imrow ? dim : dre;   // pairs with Re F
                    const float a1 = imrow ? -dre : dim;  // pairs with Im F
#pragma unroll
                    for (int a = 0; a < 2; ++a) {
                        acc[a][n] = mfma_f32(a0, b[a].re, acc[a][n]);
                        acc[a][n] = mfma_f32(a1, b[a].im, acc[a][n]);
                    }
                }
            }
        }
    } else {
        static_assert(c_phase_sensors(NT) >= 16 && 2 * pat_plane_bytes(NT, c_phase_sensors(NT) / 4) <= 65536,
                      "phase staging fits 64 KB");
        const int KH = min(c_phase_sensors(NT), Ndp);  // sensors staged per phase
        const int GPL = NT * (KH / 4) * 256;           // bytes of a staged plane
        // K step: 16 sensor rows; lane group lg holds rows 4 lg .. 4 lg + 3, items (re, im).
        // Raw operator words of one step: a bf16 pair, or the FP32 (re, im) (split when used).
        constexpr int WPE = MODE == kSplit ? 2 : 1;
        struct Raw {
            uint32_t w[2][4][WPE];
        };
        auto load_step = [&](int s0, Raw& raw) {
            const uint32_t* Fh = (const uint32_t*)Fh_;
            const cx<float>* Fh32 = (const cx<float>*)Fh_;
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int s = s0 + 4 * lg + k;
                    if constexpr (MODE == kBF16) {
                        raw.w[a][k][0] = (s < Nd) ? ld_nt4(Fh + (frow + s) * ldF + pc[a]) : 0u;
                    } else {
                        const uint2 w = (s < Nd) ? ld_nt8(Fh32 + (frow + s) * ldF + pc[a]) : uint2{0u, 0u};
                        raw.w[a][k][0] = w.x;
                        raw.w[a][k][WPE - 1] = w.y;
                    }
                }
        };
        Raw cur, nxt;
        if constexpr (PF > 0)
            if (live) load_step(0, cur);
        constexpr int kGU = 2;  // staged groups per thread in flight
        for (int sb = 0; sb < Nd; sb += KH) {
            const int ng = min(KH, Ndp - sb) >> 2;  // groups of 4 sensors in this phase
            const int total = NT * 8 * ng;
            if (sb > 0) __syncthreads();  // every wave is done with the previous phase
            for (int e0 = threadIdx.x; e0 < total; e0 += kGU * 64 * W) {
                cx<float> v[kGU][4];
#pragma unroll
                for (int u = 0; u < kGU; ++u) {
                    const int e = e0 + u * 64 * W;
                    const int r = e / ng, s = sb + 4 * (e % ng);
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        v[u][i] = cx<float>{0.f, 0.f};
                        if (e < total && r < nb && s + i < Nd)
                            v[u][i] = dh[(int64_t)r * dh_batch + (int64_t)f * Nd + s + i];
                    }
                }
#pragma unroll
                for (int u = 0; u < kGU; ++u) {
                    const int e = e0 + u * 64 * W;
                    if (e < total) {
                        const int r = e / ng, g = e % ng;
                        u32x4 p[4];  // real-row hi, lo; imaginary-row hi, lo
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const uint2 h = split_bf16_hw(__float_as_uint(v[u][i].re), __float_as_uint(v[u][i].im));
                            // K items (re F, im F) pair with (Re d, Im d) for the real row, (Im d,
                            // -Re d) for the imaginary row
                            p[0][i] = h.x;
                            p[1][i] = h.y;
                            p[2][i] = bf_im_negre(h.x);
                            p[3][i] = bf_im_negre(h.y);
                        }
                        unsigned char* blk = smem_raw + ((r >> 3) * (KH / 4) + g) * 256;
                        u32x4* d0 = reinterpret_cast<u32x4*>(blk + pat_slot(2 * (r & 7), g) * 16);
                        u32x4* d1 = reinterpret_cast<u32x4*>(blk + pat_slot(2 * (r & 7) + 1, g) * 16);
                        d0[0] = p[0];
                        d0[GPL / 16] = p[1];
                        d1[0] = p[2];
                        d1[GPL / 16] = p[3];
                    }
                }
            }
            __syncthreads();
            if (!live) continue;
            const int send = min(sb + KH, Nd);
            for (int s0 = sb; s0 < send; s0 += 16) {
                if constexpr (PF > 0) {
                    if (s0 + 16 < Nd) load_step(s0 + 16, nxt);
                } else {
                    load_step(s0, cur);
                }
                u32x4 b[2], bl[2];
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        if constexpr (MODE == kBF16) {
                            b[a][k] = cur.w[a][k][0];
                        } else {
                            const uint2 h = split_bf16_hw(cur.w[a][k][0], cur.w[a][k][WPE - 1]);
                            b[a][k] = h.x;
                            bl[a][k] = h.y;
                        }
                    }
                const int gq = ((s0 - sb) >> 2) + lg;  // this lane group's sensor group in the phase
#pragma unroll
                for (int n = 0; n < NT; ++n) {
                    const u32x4* pa =
                        reinterpret_cast<const u32x4*>(smem_raw + (n * (KH / 4) + gq) * 256 + pat_slot(li, gq) * 16);
                    const u32x4 ah = pa[0], al = pa[GPL / 16];
#pragma unroll
                    for (int a = 0; a < 2; ++a) {
                        acc[a][n] = mfma_bf16(ah, b[a], acc[a][n]);
                        acc[a][n] = mfma_bf16(al, b[a], acc[a][n]);
                        if constexpr (MODE == kSplit) acc[a][n] = mfma_bf16(ah, bl[a], acc[a][n]);
                    }
                }
                if constexpr (PF > 0) cur = nxt;
            }
        }
        if (!live) return;
    }
    // C[4 lg + v][li]: result row 4 lg + v -> rhs n*8 + 2 lg + v/2, part v&1; column p = tile + li
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const int p = pbase + 16 * a + li;
        if (p >= Nm || (a == 1 && !tile1)) continue;
#pragma unroll
        for (int n = 0; n < NT; ++n) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int r = n * 8 + 2 * lg + h;
                if (r < nb) {
                    // not read again by this launch: non-temporal store
                    typedef float f2v __attribute__((ext_vector_type(2)));
                    const f2v w = {acc[a][n][2 * h], acc[a][n][2 * h + 1]};
                    __builtin_nontemporal_store(w, reinterpret_cast<f2v*>(mo + (int64_t)r * mo_batch + (int64_t)f * ldv + p));
                }
            }
        }
    }
}

// =========================================================================================
size_t sbgemm_c_lds(int nb, int Nd, bool bf) {
    const int NT = nb <= 8 ? 1 : (nb <= 16 ? 2 : (nb <= 32 ? 4 : 8));
    if (bf) return (size_t)2 * pat_plane_bytes(NT, std::min(c_phase_sensors(NT), (Nd + 15) & ~15) / 4);
    return (size_t)NT * 8 * ((Nd + 15) & ~15) * 8;
}

static int nt_of(int nb) { return nb <= 8 ? 1 : (nb <= 16 ? 2 : (nb <= 32 ? 4 : 8)); }

// Variants of the N kernel: 0 the default rule (wide chunks on launches of >= kWideGrid
// workgroups; more than kGemmNMax right-hand sides in one eight-tile pass, with the two-wave
// register budget in the BF16 and split modes -- the fastest choices measured at 64), 1 groups
// of up to 64 (one pass over the operator for up to 64 right-hand sides, eight-tile kernel),
// 2 / 3 narrow / wide chunks on every launch, in groups of at most kGemmNMax, 4 as 1 with the
// register budget of two waves per SIMD instead of four (four or more tiles, whose accumulators
// and operator prefetch spill at four; below that it equals 1).
int sbgemm_n_variants() { return 5; }
int sbgemm_n_group(int var) { return (var == 2 || var == 3) ? kGemmNMax : kMaxBatch; }

hipError_t launch_sbgemm_n(Stor st, const void* Fh, int64_t ldF, int nfreq, int Nd, int Nm, const void* mh,
                           int64_t ldv, int64_t mh_batch, int nb, void* part, int nspan, int64_t part_batch,
                           hipStream_t s, bool split, int var) {
    if (st == Stor::C128 || nb < 1 || nb > sbgemm_n_group(var)) return hipErrorInvalidValue;
    const int CS = n_span_cols(st, Nm, nfreq);  // the single-vector kernel's spans (multiples of 256 columns)
    if (nspan != (Nm + CS - 1) / CS) return hipErrorInvalidValue;
    const int NT = nt_of(nb);
    const int mode = st == Stor::BF16 ? kBF16 : (split ? kSplit : kF32);
    const bool occ2 = (var == 4 || (var == 0 && nb > kGemmNMax && mode != kF32)) && NT >= 4;
    const bool wide = occ2 || (var == 2 ? false : (var == 3 ? true : (int64_t)nspan * nfreq >= kWideGrid));
    const size_t lds = sbgemm_n_lds(NT, chunk_of(NT, wide), mode != kF32);
    dim3 grid(nspan, nfreq), block(kGemmThreads);
    const cx<float>* m = (const cx<float>*)mh;
    cx<float>* p = (cx<float>*)part;
#define BT_GN_K(BFV, NTV, CHV, OCCV)                                                                       \
    k_sbgemm_n<BFV, NTV, CHV, OCCV><<<grid, block, lds, s>>>(Fh, ldF, Nd, Nm, m, ldv, mh_batch, nb, p, CS, nspan, \
                                                           nfreq, part_batch)
#define BT_GN(BFV, NTV)                                                            \
    do {                                                                           \
        if (occ2 && NTV >= 4)                                                      \
            BT_GN_K(BFV, NTV, (Chunk<NTV, true>::value), (NTV >= 4 ? 2 : 4));      \
        else if (wide)                                                             \
            BT_GN_K(BFV, NTV, (Chunk<NTV, true>::value), 4);                       \
        else                                                                       \
            BT_GN_K(BFV, NTV, (Chunk<NTV, false>::value), 4);                      \
    } while (0)
#define BT_GN_MODE(NTV)                     \
    do {                                    \
        if (mode == kBF16) BT_GN(kBF16, NTV);   \
        else if (mode == kSplit) BT_GN(kSplit, NTV); \
        else BT_GN(kF32, NTV);              \
    } while (0)
    switch (NT) {
        case 1: BT_GN_MODE(1); break;
        case 2: BT_GN_MODE(2); break;
        case 4: BT_GN_MODE(4); break;
        default: BT_GN_MODE(8); break;
    }
#undef BT_GN_MODE
#undef BT_GN
#undef BT_GN_K
    return hipGetLastError();
}

// Variants of the C kernel (waves per workgroup, steps of operator loads in flight): 0 is the
// default rule (4 waves below four tiles, 8 from four on; no extra step), 1..4 fix (W, PF).
static void c_variant(int var, int NT, int& W, int& PF) {
    static const int tab[5][2] = {{0, 0}, {4, 0}, {8, 0}, {4, 1}, {8, 1}};
    const int v = (var >= 0 && var < 5) ? var : 0;
    W = tab[v][0] ? tab[v][0] : (NT >= 4 ? CWaves<4>::value : CWaves<1>::value);
    PF = tab[v][1];
}
int sbgemm_c_variants() { return 5; }

hipError_t launch_sbgemm_c(Stor st, const void* Fh, int64_t ldF, int nfreq, int Nd, int Nm, const void* dh,
                           int64_t dh_batch, int nb, void* mo, int64_t ldv, int64_t mo_batch, hipStream_t s,
                           bool split, int var) {
    if (st == Stor::C128 || nb < 1 || nb > kMaxBatch) return hipErrorInvalidValue;
    const int NT = nt_of(nb);
    const size_t lds = sbgemm_c_lds(nb, Nd, st == Stor::BF16 || split);
    if (lds > 64 * 1024) return hipErrorInvalidValue;
    int W, PF;
    c_variant(var, NT, W, PF);
    dim3 grid((unsigned)((Nm + 32 * W - 1) / (32 * W)), nfreq), block(64 * W);
    const cx<float>* d = (const cx<float>*)dh;
    cx<float>* o = (cx<float>*)mo;
#define BT_GC_K(BFV, NTV, WV, PFV) \
    k_sbgemm_c<BFV, NTV, WV, PFV><<<grid, block, lds, s>>>(Fh, ldF, Nd, Nm, d, dh_batch, nb, o, ldv, mo_batch)
#define BT_GC(BFV, NTV)                      \
    do {                                     \
        if (W == 4 && PF == 0)               \
            BT_GC_K(BFV, NTV, 4, 0);         \
        else if (W == 4)                     \
            BT_GC_K(BFV, NTV, 4, 1);         \
        else if (PF == 0)                    \
            BT_GC_K(BFV, NTV, 8, 0);         \
        else                                 \
            BT_GC_K(BFV, NTV, 8, 1);         \
    } while (0)
    const int mode = st == Stor::BF16 ? kBF16 : (split ? kSplit : kF32);
#define BT_GC_MODE(NTV)                     \
    do {                                    \
        if (mode == kBF16) BT_GC(kBF16, NTV);   \
        else if (mode == kSplit) BT_GC(kSplit, NTV); \
        else BT_GC(kF32, NTV);              \
    } while (0)
    switch (NT) {
        case 1: BT_GC_MODE(1); break;
        case 2: BT_GC_MODE(2); break;
        case 4: BT_GC_MODE(4); break;
        default: BT_GC_MODE(8); break;
    }
#undef BT_GC_MODE
#undef BT_GC
#undef BT_GC_K
    return hipGetLastError();
}

}  // namespace btoep
