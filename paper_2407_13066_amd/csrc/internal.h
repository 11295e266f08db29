// Host-side declarations shared by the btoep translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace btoep {

// Mixed-radix factorisation of the half-length complex transform N (radices 2,3,4,5,7,8).
constexpr int kMaxPass = 16;
struct FftPlan {
    int N;
    int npass;
    int radix[kMaxPass];
};

// Up to kMaxBatch right-hand-side base pointers, passed by value as a kernel argument, or,
// when `dev` is set, read by the kernels from that device array (so that a captured graph
// can be replayed on other vectors by rewriting the array).
constexpr int kMaxBatch = 64;
struct PtrBatch {
    const void* p[kMaxBatch];
    const void* const* dev = nullptr;
    __host__ __device__ const void* at(int b) const { return dev ? dev[b] : p[b]; }
};

enum class Real { F32, F64 };

// Records a failed HIP call as the thread's last error (btoep_last_error(NULL)).
void set_global_error(const char* what, hipError_t e);
enum class Stor { C128 = 0, C64 = 1, BF16 = 2 };

// Threads per workgroup of every FFT kernel.
constexpr int kFftThreads = 512;

// Columns per FFT workgroup (power of two, log2) for a transform of half-length N in
// real type `r`; 0 columns (returns -1) when N does not fit one workgroup.
int fft_log_cols(int N, Real r);
size_t fft_lds_bytes(int N, int logP, Real r);

// ---- launchers (fft.hip) ------------------------------------------------------------
// Forward real-to-complex transform of zero-padded columns.
//   in  : batch b (b < nb) base in.at(b); element (j, c) at [j * in_row + c], j < Nt, c < ncols
//   out : complex, element (f, c) at out + b*out_batch + f*out_row + c, f <= N
// Storage of `out` follows `os`; the compute precision is `r`.  Inputs of type `ir`.
hipError_t launch_fft_r2c(Real r, Real ir, Stor os, const PtrBatch& in, int64_t in_row, int nb,
                          void* out, int64_t out_row, int64_t out_batch, int Nt, int ncols,
                          const FftPlan& plan, const void* tw, hipStream_t st);
// Setup form: batch over sensor rows s with explicit strides (block column input).
hipError_t launch_fft_r2c_strided(Stor os, const double* in, int64_t in_row, int64_t in_batch, int nb,
                                  void* out, int64_t out_row, int64_t out_batch, int Nt, int ncols,
                                  const FftPlan& plan, const void* tw64, hipStream_t st);
// Inverse complex-to-real transform; keeps samples j < Nt:
//   out[b][j][c] = out_scale * x_j  (+ add_scale * add[b][j][c] when `add` is present)
hipError_t launch_fft_c2r(Real r, const void* in, int64_t in_row, int64_t in_batch, int nb,
                          const PtrBatch& out, int64_t out_row, const PtrBatch& add, double add_scale,
                          int Nt, int ncols, const FftPlan& plan, const void* tw, double out_scale,
                          hipStream_t st);
// Data side of F and H: sums split partial sums part[b][s][f][span] over spans, inverse
// transforms along f, keeps j < Nt and scales by `scale`.  With `dout` given, writes the data
// vector d[b][j][s]; otherwise (H) zero-pads and forward transforms again into dh[b][f][s].
hipError_t launch_dside(Real r, const void* part, int nspan, int64_t part_batch, int nb,
                        const PtrBatch* dout, void* dh, int64_t dh_batch, int Nt, int Nd,
                        const FftPlan& plan, const void* tw, double scale, hipStream_t st);

// ---- launchers (sbgemm64.hip): the same for the complex FP64 operator ------------------
// FP64 operands and accumulation on the FP64 matrix cores; at most kGemmNMax right-hand
// sides per launch; sbgemm_c64 needs sbgemm_c64_lds(nb, Nd) <= 64 KB.
size_t sbgemm_c64_lds(int nb, int Nd);
hipError_t launch_sbgemm_n64(const void* Fh, int64_t ldF, int nfreq, int Nd, int Nm, const void* mh, int64_t ldv,
                             int64_t mh_batch, int nb, void* part, int nspan, int64_t part_batch, hipStream_t s);
hipError_t launch_sbgemm_c64(const void* Fh, int64_t ldF, int nfreq, int Nd, int Nm, const void* dh,
                             int64_t dh_batch, int nb, void* mo, int64_t ldv, int64_t mo_batch, hipStream_t s);

// ---- the appendix (SOTI) form of the frequency-domain step (alt.hip) --------------------
// out[b][c][r] = in[b][r][c] (r < rows, c < cols) for elements of `elem` bytes (16, 8 or 4).
hipError_t launch_transpose(size_t elem, const void* in, int64_t in_ld, int64_t in_batch, void* out, int64_t out_ld,
                            int64_t out_batch, int rows, int cols, int nb, hipStream_t st);
// F (adj false): vout = part[s][f][c], the sums over parameter chunk c (chunk columns each) of
// Fs[s][p][f] * vin[p][f]; F^T (adj true): vout[p][f] = sum_s conj(Fs[s][p][f]) vin[s][f].
// Rows of Fs, vin and vout (SOTI) have stride ldf.  Unfused, the products go through the
// matrix-sized buffer Q[s][p][f] first.  Compute precision r, operator storage os.
hipError_t launch_alt_product(Stor os, Real r, bool adj, bool fused, const void* Fs, const void* vin, void* vout,
                              void* Q, int Nd, int Nm, int nf, int64_t ldf, int chunk, int nchunk, hipStream_t st);

// ---- four-step transforms for long series (fft.hip) ------------------------------------
// N = N1 N2 (plans p1, p2; sub-twiddle tables tw1, tw2 of exp(-2 pi i t / (2 Nsub)), t < 2 Nsub;
// twN the operator's table).  Same inputs and outputs as launch_fft_r2c / launch_fft_c2r plus
// a complex scratch tmp[b][N][tmp_row] (tmp_row >= ncols).  The forward input of batch b is
// in.at(b), or in.at(0) + b * in_batch when in_batch != 0 (setup: sensors of a block column).
int long_log_cols(int N1, int N2, Real r);
hipError_t launch_long_r2c(Real r, Real ir, Stor os, const PtrBatch& in, int64_t in_batch, int64_t in_row, int nb,
                           int Nt, int ncols, void* tmp, int64_t tmp_row, int64_t tmp_batch, void* out,
                           int64_t out_row, int64_t out_batch, const FftPlan& p1, const FftPlan& p2, const void* tw1,
                           const void* tw2, const void* twN, hipStream_t st);
hipError_t launch_long_c2r(Real r, const void* in, int64_t in_row, int64_t in_batch, int nb, void* tmp,
                           int64_t tmp_row, int64_t tmp_batch, const PtrBatch& out, int64_t out_row,
                           const PtrBatch& add, double add_scale, int Nt, int ncols, const FftPlan& p1,
                           const FftPlan& p2, const void* tw1, const void* tw2, const void* twN, double out_scale,
                           hipStream_t st);
// Partial sums part[b][s][f][span] summed over spans into spec[b][f][s].
hipError_t launch_sum_spans(Real r, const void* part, int nspan, int64_t part_batch, void* spec, int64_t spec_batch,
                            int nfreq, int Nd, int nb, hipStream_t st);

// ---- launchers (sbgemv.hip) ---------------------------------------------------------
// Per-frequency products with the stored operator Fh[f][s][p] (row stride ldF, frequency
// stride Nd*ldF).  N: part[b][s][f][span] = sum_{p in span} Fh[f][s][p] mh[b][f][p].
// C: mo[b][f][p] = sum_s conj(Fh[f][s][p]) dh[b][f][s].
// Partial sums are laid out part[b][s][f][span] (part_batch = Nd * nfreq * nspan).
// `var` selects a tuning variant (0 .. sbgemv_variants()-1).
int n_span_cols(Stor st, int64_t Nm, int nfreq);  // columns per span of the N-direction products
int sbgemv_variants();
hipError_t launch_sbgemv_n(Stor st, const void* Fh, int64_t ldF, int nfreq, int Nd, int Nm,
                           const void* mh, int64_t ldv, int64_t mh_batch, int nb, void* part,
                           int nspan, int64_t part_batch, hipStream_t s, int var);
hipError_t launch_sbgemv_c(Stor st, const void* Fh, int64_t ldF, int nfreq, int Nd, int Nm,
                           const void* dh, int64_t dh_batch, int nb, void* mo, int64_t ldv,
                           int64_t mo_batch, hipStream_t s, int var);

// ---- launchers (sbgemm.hip): k >= 2 right-hand sides on the matrix cores ----------------
// Same operands and outputs as the single-vector launchers above, for nb right-hand sides in
// one launch (FP32 or BF16 storage only).  sbgemm_c needs sbgemm_c_lds(nb, Nd, bf) <= 64 KB
// (bf: BF16 storage or the split mode, whose staging is phased and fits any Nd).
size_t sbgemm_c_lds(int nb, int Nd, bool bf);
// Right-hand sides per N launch in the narrow/wide-chunk variants and in the FP64 kernels
// (four 16-column result tiles); the other FP32 / BF16 variants take up to kMaxBatch in one
// eight-tile pass (sbgemm_n_group); callers group larger batches.
constexpr int kGemmNMax = 32;
// `split` (FP32 storage only): run the products on the BF16 matrix cores with the operator and
// the vectors split into BF16 high parts and remainders (three MFMAs per product).
// `var` selects a tuning variant of each kernel (0 .. sbgemm_n_variants() - 1 and
// 0 .. sbgemm_c_variants() - 1; 0 is the default rule); the N launcher takes at most
// sbgemm_n_group(var) right-hand sides.
int sbgemm_n_variants();
int sbgemm_c_variants();
int sbgemm_n_group(int var);
hipError_t launch_sbgemm_n(Stor st, const void* Fh, int64_t ldF, int nfreq, int Nd, int Nm,
                           const void* mh, int64_t ldv, int64_t mh_batch, int nb, void* part,
                           int nspan, int64_t part_batch, hipStream_t s, bool split = false, int var = 0);
hipError_t launch_sbgemm_c(Stor st, const void* Fh, int64_t ldF, int nfreq, int Nd, int Nm,
                           const void* dh, int64_t dh_batch, int nb, void* mo, int64_t ldv,
                           int64_t mo_batch, hipStream_t s, bool split = false, int var = 0);

}  // namespace btoep
