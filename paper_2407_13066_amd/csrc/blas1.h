// Conjugate-gradient vector kernels (blas1.hip): declarations and the per-right-hand-side
// scalar slots kept in device memory.
#pragma once

#include "internal.h"

namespace btoep {

constexpr int kScal = 12;  // doubles per right-hand side
constexpr int kScRR = 0, kScPAP = 1, kScRRN = 2, kScTH = 3, kScACT = 4, kScAL = 5, kScBE = 6;
// BB = <b, b>, RH = <r, r> of the true (refinement) residual, IT = CG iterations taken.
constexpr int kScBB = 7, kScRH = 8, kScIT = 9;

// Doubles of scratch needed by launch_dot for nb right-hand sides.
size_t dot_tmp_doubles(int nb);
// sc[b*kScal + slot] = sum_i x[b][i] y[b][i] in FP64; mode kScPAP / kScRRN also updates the
// CG scalars (alpha, or beta / RR / ACT); any other mode only stores.
hipError_t launch_dot(Real r, const void* x, const void* y, int64_t n, int nb, int64_t stride, double* sc, int slot,
                      int mode, double* tmp, hipStream_t s);
// x += alpha p, r -= alpha Ap with alpha = sc[AL]; rv = type of r, p, Ap; rx = type of x.
hipError_t launch_cg_xr(Real rv, Real rx, void* x, void* r, const void* p, const void* Ap, int64_t n, int nb,
                        int64_t stride, const double* sc, hipStream_t s);
// p = r + beta p for right-hand sides still iterating.
hipError_t launch_cg_p(Real rv, void* p, const void* r, int64_t n, int nb, int64_t stride, const double* sc,
                       hipStream_t s);
// y = a x + c z (z may be null), elementwise with type conversion.
hipError_t launch_axpbz(Real ry, void* y, double a, Real rx, const void* x, double c, Real rz, const void* z,
                        int64_t n, int nb, int64_t stride, hipStream_t s);
// Start of an inner CG solve: TH = max(inner_rtol2 * RR, floor2 * BB), AL = BE = 0, and
// ACT = 1 only where RR > TH and the true residual has not yet met the outer test
// RH > outer_rtol2 * BB.
hipError_t launch_cg_init_scalars(double* sc, int nb, double inner_rtol2, double outer_rtol2, double floor2,
                                  hipStream_t s);
// y[i] = 0 for i < n (a kernel, so that it may be captured into a graph).
hipError_t launch_zero(Real r, void* y, int64_t n, hipStream_t s);

}  // namespace btoep
