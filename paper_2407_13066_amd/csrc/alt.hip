// The paper's alternate local matvec (appendix): the transformed operator in SOTI order,
// Fs[s][p][f] (each sensor-parameter series contiguous over frequency), applied by
// elementwise products with the vector spectrum in SOTI order and sums over the block rows
// (F) or block columns (F^T).  Kept as an ablation beside the frequency-outer products.
#include <hip/hip_runtime.h>

#include "common.h"
#include "internal.h"

namespace btoep {

namespace {

// A stored complex value in the compute type T.
template <typename T>
__device__ __forceinline__ cx<T> ld_el(const cx<double>* p) {
    const cx<double> v = *p;
    return cx<T>{(T)v.re, (T)v.im};
}
template <typename T>
__device__ __forceinline__ cx<T> ld_el(const cx<float>* p) {
    const cx<float> v = *p;
    return cx<T>{(T)v.re, (T)v.im};
}
template <typename T>
__device__ __forceinline__ cx<T> ld_el(const bf16c* p) {
    const uint32_t u = p->bits;
    return cx<T>{(T)bf16_lo(u), (T)bf16_hi(u)};
}

constexpr int kTile = 32;

// out[b][c][r] = in[b][r][c] for r < rows, c < cols: 32 x 32 tiles through LDS (one padding
// column against bank conflicts), 256 threads, four elements each.
template <typename E>
__global__ __launch_bounds__(256) void k_transpose(const E* __restrict__ in, int64_t in_ld, int64_t in_batch,
                                                   E* __restrict__ out, int64_t out_ld, int64_t out_batch, int rows,
                                                   int cols) {
    __shared__ E t[kTile][kTile + 1];
    const int c0 = blockIdx.x * kTile, r0 = blockIdx.y * kTile;
    const E* __restrict__ ib = in + (int64_t)blockIdx.z * in_batch;
    E* __restrict__ ob = out + (int64_t)blockIdx.z * out_batch;
    const int tx = threadIdx.x & (kTile - 1), ty = threadIdx.x / kTile;  // ty < 8
#pragma unroll
    for (int i = 0; i < kTile; i += 8) {
        const int r = r0 + ty + i, c = c0 + tx;
        if (r < rows && c < cols) t[ty + i][tx] = ib[(int64_t)r * in_ld + c];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kTile; i += 8) {
        const int c = c0 + ty + i, r = r0 + tx;
        if (r < rows && c < cols) ob[(int64_t)c * out_ld + r] = t[tx][ty + i];
    }
}

// Appendix form, step 1 (F): Q[s][p][f] = Fs[s][p][f] * mh[p][f]; one series (s, p) per
// workgroup.  F^T: Q[s][p][f] = conj(Fs[s][p][f]) * dh[s][f].
template <typename S, typename T, bool ADJ>
__global__ __launch_bounds__(256) void k_ewp(const S* __restrict__ Fs, const cx<T>* __restrict__ v,
                                             cx<T>* __restrict__ Q, int Nm, int nf, int64_t ldf) {
    const int64_t row = blockIdx.x;  // s * Nm + p
    const int64_t s = row / Nm, p = row - s * Nm;
    const S* __restrict__ a = Fs + row * ldf;
    const cx<T>* __restrict__ x = v + (ADJ ? s : p) * ldf;
    cx<T>* __restrict__ q = Q + row * ldf;
    for (int f = threadIdx.x; f < nf; f += 256) q[f] = ADJ ? cmulc(ld_el<T>(a + f), x[f]) : cmul(ld_el<T>(a + f), x[f]);
}

// Appendix form, step 2 (F): part[s][f][c] = sum over p in chunk c of Q[s][p][f] (the partial
// sums the data-side kernel reduces); a workgroup per (frequency block, chunk, s).  With
// FUSED the products are formed on the fly from Fs and mh instead of read from Q.
template <typename S, typename T, bool FUSED>
__global__ __launch_bounds__(256) void k_sum_rows(const cx<T>* __restrict__ Q, const S* __restrict__ Fs,
                                                  const cx<T>* __restrict__ mh, cx<T>* __restrict__ part, int Nm,
                                                  int nf, int64_t ldf, int chunk, int nchunk) {
    const int f = blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y, s = blockIdx.z;
    if (f >= nf) return;
    const int p0 = c * chunk, p1 = min(Nm, p0 + chunk);
    cx<T> acc = cx<T>{0, 0};
    const int64_t base = (int64_t)s * Nm * ldf + f;
#pragma unroll 4
    for (int p = p0; p < p1; ++p) {
        if (FUSED)
            cfma(acc, ld_el<T>(Fs + base + (int64_t)p * ldf), mh[(int64_t)p * ldf + f]);
        else
            acc = cadd(acc, Q[base + (int64_t)p * ldf]);
    }
    part[((int64_t)s * nf + f) * nchunk + c] = acc;
}

// F^T, step 2: mh'[p][f] = sum over s of Q[s][p][f] (or, FUSED, of conj(Fs[s][p][f]) dh[s][f]);
// a workgroup per (p, frequency block).
template <typename S, typename T, bool FUSED>
__global__ __launch_bounds__(256) void k_sum_cols(const cx<T>* __restrict__ Q, const S* __restrict__ Fs,
                                                  const cx<T>* __restrict__ dh, cx<T>* __restrict__ mh, int Nd,
                                                  int Nm, int nf, int64_t ldf) {
    const int f = blockIdx.y * 256 + threadIdx.x;
    const int64_t p = blockIdx.x;
    if (f >= nf) return;
    cx<T> acc = cx<T>{0, 0};
    for (int s = 0; s < Nd; ++s) {
        const int64_t i = ((int64_t)s * Nm + p) * ldf + f;
        if (FUSED)
            cfmac(acc, ld_el<T>(Fs + i), dh[(int64_t)s * ldf + f]);
        else
            acc = cadd(acc, Q[i]);
    }
    mh[p * ldf + f] = acc;
}

template <typename S, typename T>
hipError_t alt_product(bool adj, bool fused, const void* Fs, const void* vin, void* vout, void* Q, int Nd, int Nm,
                       int nf, int64_t ldf, int chunk, int nchunk, hipStream_t st) {
    const S* a = (const S*)Fs;
    const cx<T>* x = (const cx<T>*)vin;
    cx<T>* y = (cx<T>*)vout;
    cx<T>* q = (cx<T>*)Q;
    const unsigned fb = (unsigned)((nf + 255) / 256);
    if (!adj) {
        if (!fused) k_ewp<S, T, false><<<dim3((unsigned)((int64_t)Nd * Nm)), 256, 0, st>>>(a, x, q, Nm, nf, ldf);
        dim3 g(fb, (unsigned)nchunk, (unsigned)Nd);
        if (fused)
            k_sum_rows<S, T, true><<<g, 256, 0, st>>>(q, a, x, y, Nm, nf, ldf, chunk, nchunk);
        else
            k_sum_rows<S, T, false><<<g, 256, 0, st>>>(q, a, x, y, Nm, nf, ldf, chunk, nchunk);
    } else {
        if (!fused) k_ewp<S, T, true><<<dim3((unsigned)((int64_t)Nd * Nm)), 256, 0, st>>>(a, x, q, Nm, nf, ldf);
        dim3 g((unsigned)Nm, fb);
        if (fused)
            k_sum_cols<S, T, true><<<g, 256, 0, st>>>(q, a, x, y, Nd, Nm, nf, ldf);
        else
            k_sum_cols<S, T, false><<<g, 256, 0, st>>>(q, a, x, y, Nd, Nm, nf, ldf);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_transpose(size_t elem, const void* in, int64_t in_ld, int64_t in_batch, void* out, int64_t out_ld,
                            int64_t out_batch, int rows, int cols, int nb, hipStream_t st) {
    if (rows <= 0 || cols <= 0 || nb <= 0 || nb > 65535) return hipErrorInvalidValue;
    const int64_t gy = (rows + kTile - 1) / kTile;
    if (gy > 65535) return hipErrorInvalidValue;
    dim3 g((unsigned)((cols + kTile - 1) / kTile), (unsigned)gy, (unsigned)nb);
    switch (elem) {
        case 16:
            k_transpose<cx<double>><<<g, 256, 0, st>>>((const cx<double>*)in, in_ld, in_batch, (cx<double>*)out,
                                                       out_ld, out_batch, rows, cols);
            break;
        case 8:
            k_transpose<cx<float>><<<g, 256, 0, st>>>((const cx<float>*)in, in_ld, in_batch, (cx<float>*)out,
                                                      out_ld, out_batch, rows, cols);
            break;
        case 4:
            k_transpose<bf16c><<<g, 256, 0, st>>>((const bf16c*)in, in_ld, in_batch, (bf16c*)out, out_ld, out_batch,
                                                  rows, cols);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_alt_product(Stor os, Real r, bool adj, bool fused, const void* Fs, const void* vin, void* vout,
                              void* Q, int Nd, int Nm, int nf, int64_t ldf, int chunk, int nchunk, hipStream_t st) {
    if (Nd <= 0 || Nm <= 0 || nf <= 0 || nf > 65535 * 256 || (!fused && !Q) || nchunk < 1 || nchunk > 65535 ||
        Nd > 65535 || (int64_t)Nd * Nm > 2147483647 || (!adj && (int64_t)chunk * nchunk < Nm))
        return hipErrorInvalidValue;
    if (r == Real::F64) {
        if (os != Stor::C128) return hipErrorInvalidValue;
        return alt_product<cx<double>, double>(adj, fused, Fs, vin, vout, Q, Nd, Nm, nf, ldf, chunk, nchunk, st);
    }
    switch (os) {
        case Stor::C64:
            return alt_product<cx<float>, float>(adj, fused, Fs, vin, vout, Q, Nd, Nm, nf, ldf, chunk, nchunk, st);
        case Stor::BF16:
            return alt_product<bf16c, float>(adj, fused, Fs, vin, vout, Q, Nd, Nm, nf, ldf, chunk, nchunk, st);
        default:
            return hipErrorInvalidValue;
    }
}

}  // namespace btoep
