// Batched FFTs along the time axis of block-Toeplitz vectors and block columns.
//
// The method (paper section 2.4, section 3.3) zero-pads every length-Nt time series to
// L = 2N (N >= Nt), transforms it, and after the per-frequency product transforms back and
// keeps the first Nt samples.  Here a length-L real transform is one complex transform of
// half length N on z[n] = x[2n] + i x[2n+1] (even/odd packing), followed by the usual
// split into the L/2 + 1 = N + 1 non-redundant bins.  The complex transform is a
// mixed-radix Stockham autosort FFT (radices 2, 3, 4, 5, 7, 8) run entirely in LDS: a
// workgroup owns P consecutive columns (the contiguous axis of the time-outer layout), so
// every global load and store is a run of P consecutive elements of one time row (or one
// frequency row) and the time-outer <-> frequency-outer reordering of the paper's
// SOTI/TOSI steps costs nothing extra.  Layout in LDS: element (n, c) at n*P + c.
#include "common.h"
#include "internal.h"

namespace btoep {

// ----------------------------------------------------------------------------------------
// Small DFTs in registers:  y_t = sum_q x_q exp(DIR * 2 pi i q t / R), DIR = -1 forward.
template <int R, int DIR, typename T>
struct Dft;

template <int DIR, typename T>
struct Dft<2, DIR, T> {
    __device__ static void run(cx<T>* v) {
        cx<T> a = v[0];
        v[0] = cadd(a, v[1]);
        v[1] = csub(a, v[1]);
    }
};

template <int DIR, typename T>
struct Dft<4, DIR, T> {
    __device__ static void run(cx<T>* v) {
        cx<T> a0 = cadd(v[0], v[2]), a1 = cadd(v[1], v[3]);
        cx<T> b0 = csub(v[0], v[2]), b1 = cmul_i<DIR>(csub(v[1], v[3]));
        v[0] = cadd(a0, a1);
        v[2] = csub(a0, a1);
        v[1] = cadd(b0, b1);
        v[3] = csub(b0, b1);
    }
    // the same with v[2] = v[3] = 0 (the zero padding of a transform's first pass)
    __device__ static void run_hz(cx<T>* v) {
        const cx<T> a0 = v[0], a1 = v[1], b1 = cmul_i<DIR>(v[1]);
        v[0] = cadd(a0, a1);
        v[2] = csub(a0, a1);
        v[1] = cadd(a0, b1);
        v[3] = csub(a0, b1);
    }
};

template <int DIR, typename T>
struct Dft<8, DIR, T> {
    __device__ static void run(cx<T>* v) {
        const T h = (T)0.70710678118654752440;  // 1/sqrt(2)
        cx<T> a[4], b[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            a[q] = cadd(v[q], v[q + 4]);
            b[q] = csub(v[q], v[q + 4]);
        }
        // b_q *= exp(DIR * 2 pi i q / 8)
        b[1] = cx<T>{h * (b[1].re - DIR * b[1].im), h * (b[1].im + DIR * b[1].re)};
        b[2] = cmul_i<DIR>(b[2]);
        b[3] = cx<T>{h * (-b[3].re - DIR * b[3].im), h * (-b[3].im + DIR * b[3].re)};
        Dft<4, DIR, T>::run(a);
        Dft<4, DIR, T>::run(b);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            v[2 * u] = a[u];
            v[2 * u + 1] = b[u];
        }
    }
    // the same with v[4..7] = 0
    __device__ static void run_hz(cx<T>* v) {
        const T h = (T)0.70710678118654752440;
        cx<T> a[4], b[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) a[q] = b[q] = v[q];
        b[1] = cx<T>{h * (b[1].re - DIR * b[1].im), h * (b[1].im + DIR * b[1].re)};
        b[2] = cmul_i<DIR>(b[2]);
        b[3] = cx<T>{h * (-b[3].re - DIR * b[3].im), h * (-b[3].im + DIR * b[3].re)};
        Dft<4, DIR, T>::run(a);
        Dft<4, DIR, T>::run(b);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            v[2 * u] = a[u];
            v[2 * u + 1] = b[u];
        }
    }
};

// cos / sin of 2 pi n / R for the odd radices.
template <int R>
struct OddConst;
template <>
struct OddConst<3> {
    __device__ static double c(int n) {
        constexpr double t[3] = {1.0, -0.5, -0.5};
        return t[n];
    }
    __device__ static double s(int n) {
        constexpr double t[3] = {0.0, 0.8660254037844386, -0.8660254037844386};
        return t[n];
    }
};
template <>
struct OddConst<5> {
    __device__ static double c(int n) {
        constexpr double t[5] = {1.0, 0.30901699437494745, -0.8090169943749475, -0.8090169943749475,
                                 0.30901699437494745};
        return t[n];
    }
    __device__ static double s(int n) {
        constexpr double t[5] = {0.0, 0.9510565162951535, 0.5877852522924731, -0.5877852522924731,
                                 -0.9510565162951535};
        return t[n];
    }
};
template <>
struct OddConst<7> {
    __device__ static double c(int n) {
        constexpr double t[7] = {1.0, 0.6234898018587335, -0.2225209339563144, -0.9009688679024191,
                                 -0.9009688679024191, -0.2225209339563144, 0.6234898018587335};
        return t[n];
    }
    __device__ static double s(int n) {
        constexpr double t[7] = {0.0, 0.7818314824680298, 0.9749279121818236, 0.4338837391175581,
                                 -0.4338837391175581, -0.9749279121818236, -0.7818314824680298};
        return t[n];
    }
};

// Odd prime R: pair inputs q and R-q, a_q = x_q + x_{R-q}, b_q = x_q - x_{R-q};
//   y_t     = x_0 + sum_q cos(2pi qt/R) a_q + DIR i sum_q sin(2pi qt/R) b_q
//   y_{R-t} = x_0 + sum_q cos(2pi qt/R) a_q - DIR i sum_q sin(2pi qt/R) b_q
template <int R, int DIR, typename T>
struct DftOdd {
    __device__ static void run(cx<T>* v) {
        constexpr int H = (R - 1) / 2;
        cx<T> a[H + 1], b[H + 1];
        cx<T> y0 = v[0];
#pragma unroll
        for (int q = 1; q <= H; ++q) {
            a[q] = cadd(v[q], v[R - q]);
            b[q] = csub(v[q], v[R - q]);
            y0 = cadd(y0, a[q]);
        }
        cx<T> out[R];
        out[0] = y0;
#pragma unroll
        for (int t = 1; t <= H; ++t) {
            cx<T> sc = v[0], ss = cx<T>{0, 0};
#pragma unroll
            for (int q = 1; q <= H; ++q) {
                const T c = (T)OddConst<R>::c((q * t) % R);
                const T s = (T)OddConst<R>::s((q * t) % R);
                sc = cx<T>{fma(c, a[q].re, sc.re), fma(c, a[q].im, sc.im)};
                ss = cx<T>{fma(s, b[q].re, ss.re), fma(s, b[q].im, ss.im)};
            }
            cx<T> iss = cmul_i<DIR>(ss);
            out[t] = cadd(sc, iss);
            out[R - t] = csub(sc, iss);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = out[r];
    }
};
template <int DIR, typename T>
struct Dft<3, DIR, T> : DftOdd<3, DIR, T> {};
template <int DIR, typename T>
struct Dft<5, DIR, T> : DftOdd<5, DIR, T> {};
template <int DIR, typename T>
struct Dft<7, DIR, T> : DftOdd<7, DIR, T> {};

// cos / sin of 2 pi m / N (m < N) for the twiddles inside the composite radices.
template <int N>
struct RootTable;
template <>
struct RootTable<12> {
    __device__ static double c(int m) {
        constexpr double h = 0.86602540378443865;  // sqrt(3) / 2
        constexpr double t[12] = {1, h, 0.5, 0, -0.5, -h, -1, -h, -0.5, 0, 0.5, h};
        return t[m];
    }
    __device__ static double s(int m) {
        constexpr double h = 0.86602540378443865;
        constexpr double t[12] = {0, 0.5, h, 1, h, 0.5, 0, -0.5, -h, -1, -h, -0.5};
        return t[m];
    }
};
template <>
struct RootTable<16> {
    __device__ static double c(int m) {
        constexpr double t[16] = {1, 0.92387953251128674, 0.70710678118654757, 0.38268343236508984, 0, -0.38268343236508973,
                                   -0.70710678118654746, -0.92387953251128674, -1, -0.92387953251128685, -0.70710678118654768,
                                   -0.38268343236509034, 0, 0.38268343236509, 0.70710678118654735, 0.92387953251128652};
        return t[m];
    }
    __device__ static double s(int m) {
        constexpr double t[16] = {0, 0.38268343236508978, 0.70710678118654746, 0.92387953251128674, 1, 0.92387953251128674,
                                   0.70710678118654757, 0.38268343236508989, 0, -0.38268343236508967, -0.70710678118654746,
                                   -0.92387953251128652, -1, -0.92387953251128663, -0.70710678118654768, -0.38268343236509039};
        return t[m];
    }
};
template <>
struct RootTable<20> {
    __device__ static double c(int m) {
        constexpr double t[20] = {1, 0.95105651629515353, 0.80901699437494745, 0.58778525229247314, 0.30901699437494745, 0,
                                   -0.30901699437494734, -0.58778525229247303, -0.80901699437494734, -0.95105651629515353, -1,
                                   -0.95105651629515375, -0.80901699437494756, -0.58778525229247325, -0.30901699437494756, 0,
                                   0.30901699437494723, 0.58778525229247292, 0.80901699437494734, 0.95105651629515353};
        return t[m];
    }
    __device__ static double s(int m) {
        constexpr double t[20] = {0, 0.3090169943749474, 0.58778525229247314, 0.80901699437494745, 0.95105651629515353, 1,
                                   0.95105651629515364, 0.80901699437494745, 0.58778525229247325, 0.30901699437494751, 0,
                                   -0.3090169943749469, -0.58778525229247303, -0.80901699437494734, -0.95105651629515353, -1,
                                   -0.95105651629515364, -0.80901699437494756, -0.58778525229247336, -0.30901699437494762};
        return t[m];
    }
};
template <>
struct RootTable<21> {
    __device__ static double c(int m) {
        constexpr double t[21] = {1, 0.95557280578614068, 0.82623877431599491, 0.62348980185873359, 0.36534102436639498,
                                   0.074730093586424393, -0.22252093395631434, -0.49999999999999978, -0.73305187182982634,
                                   -0.90096886790241903, -0.98883082622512852, -0.98883082622512863, -0.90096886790241915,
                                   -0.73305187182982623, -0.50000000000000044, -0.22252093395631459, 0.074730093586424365,
                                   0.36534102436639537, 0.62348980185873337, 0.82623877431599446, 0.95557280578614057};
        return t[m];
    }
    __device__ static double s(int m) {
        constexpr double t[21] = {0, 0.29475517441090421, 0.56332005806362206, 0.7818314824680298, 0.93087374864420425,
                                   0.99720379718118013, 0.97492791218182362, 0.86602540378443871, 0.68017273777091936,
                                   0.43388373911755823, 0.14904226617617472, -0.14904226617617403, -0.43388373911755801,
                                   -0.68017273777091947, -0.86602540378443837, -0.97492791218182362, -0.99720379718118013,
                                   -0.93087374864420414, -0.78183148246802991, -0.56332005806362273, -0.29475517441090471};
        return t[m];
    }
};

// Composite radix N = N1 N2 in registers (Cooley-Tukey): with n = N2 n1 + n2 and
// k = k1 + N1 k2,  X[k] = sum_{n2} W_N^{n2 k1} W_{N2}^{n2 k2} sum_{n1} x[n] W_{N1}^{n1 k1},
// W_M = exp(DIR 2 pi i / M): N2 DFTs of size N1, the twiddles, then N1 DFTs of size N2.
template <int N1, int N2, int DIR, typename T>
struct DftComp {
    __device__ static void run(cx<T>* v) { run_t<false>(v); }
    // the same with the upper half v[N/2 ..] = 0 (N1 even: the inputs with n1 >= N1/2)
    __device__ static void run_hz(cx<T>* v) { run_t<true>(v); }
    template <bool HZ>
    __device__ static void run_t(cx<T>* v) {
        constexpr int N = N1 * N2;
        static_assert(!HZ || N1 % 2 == 0, "zero upper half needs an even first factor");
        cx<T> y[N2][N1];
#pragma unroll
        for (int n2 = 0; n2 < N2; ++n2) {
#pragma unroll
            for (int n1 = 0; n1 < N1; ++n1) y[n2][n1] = v[N2 * n1 + n2];
            if constexpr (HZ)
                Dft<N1, DIR, T>::run_hz(y[n2]);
            else
                Dft<N1, DIR, T>::run(y[n2]);
#pragma unroll
            for (int k1 = 1; k1 < N1; ++k1) {
                if (n2 == 0) continue;
                const int m = n2 * k1;  // < N
                const cx<T> w = cx<T>{(T)RootTable<N>::c(m), (T)(DIR * RootTable<N>::s(m))};
                y[n2][k1] = cmul(y[n2][k1], w);
            }
        }
#pragma unroll
        for (int k1 = 0; k1 < N1; ++k1) {
            cx<T> b[N2];
#pragma unroll
            for (int n2 = 0; n2 < N2; ++n2) b[n2] = y[n2][k1];
            Dft<N2, DIR, T>::run(b);
#pragma unroll
            for (int k2 = 0; k2 < N2; ++k2) v[k1 + N1 * k2] = b[k2];
        }
    }
};
template <int DIR, typename T>
struct Dft<12, DIR, T> : DftComp<4, 3, DIR, T> {};
template <int DIR, typename T>
struct Dft<16, DIR, T> : DftComp<4, 4, DIR, T> {};
template <int DIR, typename T>
struct Dft<20, DIR, T> : DftComp<4, 5, DIR, T> {};
template <int DIR, typename T>
struct Dft<21, DIR, T> : DftComp<3, 7, DIR, T> {};

// ----------------------------------------------------------------------------------------
// One Stockham pass of radix R over all P columns held in LDS.  Ns = product of the radices
// already applied.  Butterfly j (< N/R) of column c reads elements j + r N/R, multiplies by
// W_{Ns R}^{k r} (k = j mod Ns) and writes its outputs to (j - k) R + k + r Ns.  The
// twiddle table holds exp(-2 pi i t / (2N)), t < 2N, so W_{Ns R}^{k r} is entry
// 2 k r N / (Ns R).  Each thread keeps its butterflies in registers across the barrier,
// which lets the pass run in place.  The read/compute phase has no branches (threads past
// the last butterfly redo the last one and do not store), so all of a thread's LDS and
// twiddle reads can be in flight together.
// Dynamic LDS of every FFT kernel: data (N+1) x P complex, then (when staged) the twiddles.
// The kernels ask for four waves per SIMD (two 512-thread workgroups per CU): measured faster
// than full-register single-workgroup occupancy although the passes then keep some state in
// scratch.
extern __shared__ __align__(16) unsigned char fft_smem[];

// Each pass is its own (non-inlined) function so that register allocation is per radix;
// it addresses the data through the kernel's dynamic LDS symbol so accesses stay LDS ops.
template <typename T, int R, int DIR, int CMAX, bool TWL>
__device__ __noinline__ void stockham_pass(int N, int logP, int Ns, size_t tw_off, const cx<T>* __restrict__ twg) {
    cx<T>* sh = reinterpret_cast<cx<T>*>(fft_smem);
    const cx<T>* tw = TWL ? reinterpret_cast<const cx<T>*>(fft_smem + tw_off) : twg;
    constexpr int MAXB = (CMAX + R - 1) / R;
    const int NR = N / R;
    const int nbf = NR << logP;
    const int stride = NR / Ns;
    const int P1 = (1 << logP) - 1;
    const int tid = threadIdx.x;
    cx<T> v[MAXB][R];
#pragma unroll
    for (int bb = 0; bb < MAXB; ++bb) {
        const int g = min(tid + bb * kFftThreads, nbf - 1);
        const int c = g & P1, j = g >> logP;
        const int k = j % Ns;
#pragma unroll
        for (int r = 0; r < R; ++r) v[bb][r] = sh[((j + r * NR) << logP) + c];
#pragma unroll
        for (int r = 1; r < R; ++r) {
            cx<T> w = tw[2 * (k * r * stride)];  // k = 0 (first pass) reads W = 1
            if (DIR > 0) w.im = -w.im;
            v[bb][r] = cmul(v[bb][r], w);
        }
        Dft<R, DIR, T>::run(v[bb]);
    }
    __syncthreads();
#pragma unroll
    for (int bb = 0; bb < MAXB; ++bb) {
        const int g = tid + bb * kFftThreads;
        if (g < nbf) {
            const int c = g & P1, j = g >> logP;
            const int k = j % Ns;
            const int base = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) sh[((base + r * Ns) << logP) + c] = v[bb][r];
        }
    }
    __syncthreads();
}

template <typename T, int DIR, int CMAX, bool TWL>
__device__ void fft_passes(const FftPlan& plan, int logP, size_t tw_off, const cx<T>* __restrict__ twg) {
    int Ns = 1;
    for (int ip = 0; ip < plan.npass; ++ip) {
        const int R = plan.radix[ip];
        switch (R) {
            case 2: stockham_pass<T, 2, DIR, CMAX, TWL>(plan.N, logP, Ns, tw_off, twg); break;
            case 3: stockham_pass<T, 3, DIR, CMAX, TWL>(plan.N, logP, Ns, tw_off, twg); break;
            case 4: stockham_pass<T, 4, DIR, CMAX, TWL>(plan.N, logP, Ns, tw_off, twg); break;
            case 5: stockham_pass<T, 5, DIR, CMAX, TWL>(plan.N, logP, Ns, tw_off, twg); break;
            case 7: stockham_pass<T, 7, DIR, CMAX, TWL>(plan.N, logP, Ns, tw_off, twg); break;
            default: stockham_pass<T, 8, DIR, CMAX, TWL>(plan.N, logP, Ns, tw_off, twg); break;
        }
        Ns *= R;
    }
}

// All passes of one transform over the P columns in LDS.
template <typename T, int DIR, int CMAX>
__device__ __forceinline__ void fft_lds(const FftPlan& plan, int logP, bool twl, size_t tw_off,
                                        const cx<T>* __restrict__ twg) {
    if (twl)
        fft_passes<T, DIR, CMAX, true>(plan, logP, tw_off, twg);
    else
        fft_passes<T, DIR, CMAX, false>(plan, logP, tw_off, twg);
}

// ---- compile-time plans ---------------------------------------------------------------
// For the transform lengths of the common workloads the passes are instantiated with N, Ns
// and R as constants and inlined: no per-pass calls, constant strides and modulo, twiddles
// read from LDS.  Any other length runs the runtime plan above.
struct RuntimePlan {
    static constexpr bool kStatic = false;
};
template <int... Rs>
struct CtPlan {
    static constexpr bool kStatic = true;
    static constexpr int N = (Rs * ... * 1);
};

// HALF: only outputs r < (R+1)/2 of every butterfly are written -- for the last pass of an
// inverse transform whose consumer reads only z_m, m < N/2 (there m = j + r Ns).
template <typename T, int R, int DIR, int CMAX, int N, int Ns, bool TWL, bool HALF = false>
__device__ __forceinline__ void ct_pass(int logP, size_t tw_off, const cx<T>* __restrict__ twg) {
    cx<T>* sh = reinterpret_cast<cx<T>*>(fft_smem);
    const cx<T>* tw = TWL ? reinterpret_cast<const cx<T>*>(fft_smem + tw_off) : twg;
    constexpr int MAXB = (CMAX + R - 1) / R;
    constexpr int NR = N / R;
    constexpr int stride = NR / Ns;
    const int nbf = NR << logP;
    const int P1 = (1 << logP) - 1;
    const int tid = threadIdx.x;
    cx<T> v[MAXB][R];
#pragma unroll
    for (int bb = 0; bb < MAXB; ++bb) {
        const int g = min(tid + bb * kFftThreads, nbf - 1);
        const int c = g & P1, j = g >> logP;
        const int k = j % Ns;
#pragma unroll
        for (int r = 0; r < R; ++r) v[bb][r] = sh[((j + r * NR) << logP) + c];
        if (Ns > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                cx<T> w = tw[2 * (k * r * stride)];
                if (DIR > 0) w.im = -w.im;
                v[bb][r] = cmul(v[bb][r], w);
            }
        }
        Dft<R, DIR, T>::run(v[bb]);
    }
    __syncthreads();
#pragma unroll
    for (int bb = 0; bb < MAXB; ++bb) {
        const int g = tid + bb * kFftThreads;
        if (g < nbf) {
            const int c = g & P1, j = g >> logP;
            const int k = j % Ns;
            const int base = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < (HALF ? (R + 1) / 2 : R); ++r) sh[((base + r * Ns) << logP) + c] = v[bb][r];
        }
    }
    __syncthreads();
}

template <typename T, int DIR, int CMAX, bool TWL, bool HALF_LAST, int N, int Ns, int R, int... Rest>
__device__ __forceinline__ void ct_passes_h(int logP, size_t tw_off, const cx<T>* __restrict__ twg) {
    if constexpr (sizeof...(Rest) > 0) {
        ct_pass<T, R, DIR, CMAX, N, Ns, TWL>(logP, tw_off, twg);
        ct_passes_h<T, DIR, CMAX, TWL, HALF_LAST, N, Ns * R, Rest...>(logP, tw_off, twg);
    } else {
        ct_pass<T, R, DIR, CMAX, N, Ns, TWL, HALF_LAST>(logP, tw_off, twg);
    }
}
template <typename T, int DIR, int CMAX, bool TWL, int N, int Ns, int R, int... Rest>
__device__ __forceinline__ void ct_passes(int logP, size_t tw_off, const cx<T>* __restrict__ twg) {
    ct_passes_h<T, DIR, CMAX, TWL, false, N, Ns, R, Rest...>(logP, tw_off, twg);
}

template <typename T, int DIR, int CMAX, bool TWL, bool HALF_LAST = false, int... Rs>
__device__ __forceinline__ void ct_run(CtPlan<Rs...>, int logP, size_t tw_off, const cx<T>* __restrict__ twg) {
    ct_passes_h<T, DIR, CMAX, TWL, HALF_LAST, CtPlan<Rs...>::N, 1, Rs...>(logP, tw_off, twg);
}

template <typename T>
struct FftCfg;
template <>
struct FftCfg<float> {
    static constexpr int CMAX = 16;  // complex values per thread held across a pass
};
template <>
struct FftCfg<double> {
    static constexpr int CMAX = 8;
};

constexpr int kLoadUnroll = 8;  // global loads each thread keeps in flight when staging

// ---- storing a complex value in each output format ----------------------------------
template <typename T>
__device__ __forceinline__ void put(cx<double>* p, cx<T> v) { *p = cx<double>{(double)v.re, (double)v.im}; }
template <typename T>
__device__ __forceinline__ void put(cx<float>* p, cx<T> v) { *p = cx<float>{(float)v.re, (float)v.im}; }
template <typename T>
__device__ __forceinline__ void put(bf16c* p, cx<T> v) {
    *p = Store<bf16c>::from(cx<double>{(double)v.re, (double)v.im});
}


// Vector-side outputs are written with non-temporal stores when a workgroup's run of P values
// per row spans at least 64 bytes: left as dirty lines in the caches they would be written back
// while the next kernel streams the operator.  Shorter runs (long series, narrow tiles) use
// ordinary stores, which measured up to twice as fast for such partial lines.
template <typename T>
__device__ __forceinline__ void put_nt(cx<float>* p, cx<T> v) {
    typedef float f2v __attribute__((ext_vector_type(2)));
    const f2v w = {(float)v.re, (float)v.im};
    __builtin_nontemporal_store(w, reinterpret_cast<f2v*>(p));
}
template <typename T>
__device__ __forceinline__ void put_nt(cx<double>* p, cx<T> v) { put(p, v); }
template <typename T>
__device__ __forceinline__ void put_nt(bf16c* p, cx<T> v) { put(p, v); }

// Bins f = 0..N of the length-2N real transform from the half-length transform Z held in
// LDS:  X_f = (Z_f + conj Z_{N-f}) / 2 + W_{2N}^f (Z_f - conj Z_{N-f}) / (2i).
template <typename T>
__device__ __forceinline__ cx<T> r2c_bin(const cx<T>* sh, int N, int logP, int f, int c, const cx<T>* tw) {
    const int fa = (f == N) ? 0 : f;
    const int fb = (f == 0) ? 0 : N - f;
    cx<T> Z = sh[(fa << logP) + c];
    cx<T> Zc = cconj(sh[(fb << logP) + c]);
    cx<T> E = cscale(cadd(Z, Zc), (T)0.5);
    cx<T> O = cmul_i<-1>(cscale(csub(Z, Zc), (T)0.5));
    return cadd(E, cmul(tw[f], O));
}

// Inverse split, in place on LDS rows f and N-f: from bins Y_0..Y_N of a real signal build
// Z_f = E_f + i O_f with E_f = (Y_f + conj Y_{N-f}) / 2 and O_f = (Y_f - conj Y_{N-f}) / 2 *
// W_{2N}^{-f}; then the inverse half-length transform of Z gives x_{2n} + i x_{2n+1} (times N).
template <typename T>
__device__ __forceinline__ void c2r_split(cx<T>* sh, int N, int logP, const cx<T>* tw) {
    const int P = 1 << logP;
    const int npair = (N / 2 + 1) << logP;
    for (int e = threadIdx.x; e < npair; e += kFftThreads) {
        const int c = e & (P - 1), f = e >> logP;
        const int g = N - f;
        if (g < f) continue;  // only when N is odd: f = (N+1)/2 has no partner of its own
        cx<T> Yf = sh[(f << logP) + c];
        cx<T> Yg = sh[(g << logP) + c];
        {
            cx<T> b = cconj(Yg);
            cx<T> E = cscale(cadd(Yf, b), (T)0.5);
            cx<T> O = cmul(cscale(csub(Yf, b), (T)0.5), cconj(tw[f]));
            sh[(f << logP) + c] = cadd(E, cmul_i<1>(O));
        }
        if (f != 0 && g != f) {
            cx<T> b = cconj(Yf);
            cx<T> E = cscale(cadd(Yg, b), (T)0.5);
            cx<T> O = cmul(cscale(csub(Yg, b), (T)0.5), cconj(tw[g]));
            sh[(g << logP) + c] = cadd(E, cmul_i<1>(O));
        }
    }
}

// Twiddle table e^{-2 pi i t / L}, t < L = 2N: copied into LDS behind the data when `twl`,
// otherwise read from global memory (it stays in the caches).
template <typename T>
__device__ __forceinline__ const cx<T>* stage_twiddles(size_t data_bytes, bool twl, int N,
                                                       const cx<T>* __restrict__ twg) {
    if (!twl) return twg;
    cx<T>* t = reinterpret_cast<cx<T>*>(fft_smem + data_bytes);
#pragma unroll 4
    for (int i = threadIdx.x; i < 2 * N; i += kFftThreads) t[i] = twg[i];
    return t;
}

// LDS a workgroup may use for one column tile plus the twiddle table.
static constexpr size_t kFftLdsBudget = 64 * 1024;

// Widest column tile (log2) of a length-N transform with elements of `elem` bytes, with or
// without the twiddle table in LDS (-1 when not even one column fits).
constexpr int tile_log_cols(int N, size_t elem, int cmax, bool twl) {
    for (int lp = 6; lp >= 0; --lp) {
        const size_t P = (size_t)1 << lp;
        if ((size_t)(N + 1) * P * elem + (twl ? (size_t)2 * N * elem : 0) <= kFftLdsBudget &&
            (size_t)N * P <= (size_t)cmax * kFftThreads)
            return lp;
    }
    return -1;
}
// Twiddles live in LDS when they fit without narrowing the column tile: every global access
// of a tile is a run of P consecutive columns, and runs shorter than a cache line cost more
// than twiddle reads from the caches.
constexpr bool tile_twl(int N, size_t elem, int cmax) {
    const int with = tile_log_cols(N, elem, cmax, true);
    return with >= 0 && with >= tile_log_cols(N, elem, cmax, false);
}
// The same rules for a compile-time plan of length N: where its twiddles live, the widest tile
// the launchers pick, and the global loads per thread that then cover one tile of N+1 rows.
template <typename T>
constexpr bool ct_twl(int N) {
    return tile_twl(N, sizeof(cx<T>), FftCfg<T>::CMAX);
}
template <typename T>
constexpr int ct_log_cols(int N) {
    const int lp = tile_log_cols(N, sizeof(cx<T>), FftCfg<T>::CMAX, ct_twl<T>(N));
    return lp < 0 ? 0 : lp;
}

template <typename T, int DIR, int CMAX, typename PL>
__device__ __forceinline__ void run_fft(const FftPlan& plan, int logP, bool twl, size_t tw_off,
                                        const cx<T>* __restrict__ twg) {
    if constexpr (PL::kStatic)
        ct_run<T, DIR, CMAX, ct_twl<T>(PL::N)>(PL{}, logP, tw_off, twg);
    else
        fft_lds<T, DIR, CMAX>(plan, logP, twl, tw_off, twg);
}
template <typename T, typename PL, bool STATIC = PL::kStatic>
struct LoadSlots {
    static constexpr int value = FftCfg<T>::CMAX;
};
template <typename T, typename PL>
struct LoadSlots<T, PL, true> {
    static constexpr int value = (((PL::N + 1) << ct_log_cols<T>(PL::N)) + kFftThreads - 1) / kFftThreads;
};

// Real input rows j < Nt of one column tile (P columns) in the packed LDS layout
// z[n] = x[2n] + i x[2n+1], zero rows j in [Nt, 2N).  `load` issues every global load of the
// tile at once (NL per thread cover the Nt P elements: the launchers check it), with clamped
// addresses, before anything waits for them; `commit` writes them.
template <typename T, typename Tin, int NL>
struct RealTile {
    T v[NL];
    __device__ __forceinline__ void load(const Tin* __restrict__ x, int64_t in_row, int total, int logP, int col0,
                                         int ncols) {
        const int P1 = (1 << logP) - 1;
#pragma unroll
        for (int u = 0; u < NL; ++u) {
            const int e = min(u * kFftThreads + (int)threadIdx.x, total - 1);
            const int c = e & P1, j = e >> logP;
            v[u] = (T)x[(int64_t)j * in_row + min(col0 + c, ncols - 1)];
        }
    }
    __device__ __forceinline__ void commit(T* shr, int Nt, int N, int logP, int col0, int ncols) const {
        const int P1 = (1 << logP) - 1;
        const int total = Nt << logP;
        for (int e = total + threadIdx.x; e < (2 * N) << logP; e += kFftThreads) {
            const int c = e & P1, j = e >> logP;
            shr[2 * (((j >> 1) << logP) + c) + (j & 1)] = (T)0;
        }
#pragma unroll
        for (int u = 0; u < NL; ++u) {
            const int e = u * kFftThreads + (int)threadIdx.x;
            if (e < total) {
                const int c = e & P1, j = e >> logP;
                shr[2 * (((j >> 1) << logP) + c) + (j & 1)] = (col0 + c < ncols) ? v[u] : (T)0;
            }
        }
    }
};

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2).  When the
// column-block count divides by 8, XCD x is given the contiguous range of column blocks
// [x nbx/8, (x+1) nbx/8) in order, so neighbouring column blocks -- which share 128-byte lines
// of every time and frequency row -- meet in the same L2.
__device__ __forceinline__ int column_block() {
    const int nbx = gridDim.x, bx = blockIdx.x;
    return (nbx & 7) ? bx : (bx & 7) * (nbx >> 3) + (bx >> 3);
}

// ----------------------------------------------------------------------------------------
// Forward: x (real, Nt rows) -> X (N+1 complex rows).
template <typename T, typename Tin, typename So, typename PL>
__global__ __launch_bounds__(kFftThreads) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_fft_r2c(PtrBatch in, int64_t in_row, So* __restrict__ out,
                                                         int64_t out_row, int64_t out_batch, int Nt, int ncols,
                                                         FftPlan plan, int logP, const cx<T>* __restrict__ twg,
                                                         int twl, int ntw) {
    cx<T>* sh = reinterpret_cast<cx<T>*>(fft_smem);
    const int N = plan.N, P = 1 << logP;
    const int col0 = column_block() << logP;
    const size_t tw_off = (size_t)(N + 1) * P * sizeof(cx<T>);
    const Tin* __restrict__ x = static_cast<const Tin*>(in.at(blockIdx.y));
    So* __restrict__ y = out + (int64_t)blockIdx.y * out_batch;
    // all input loads in flight before the twiddle copy waits for its own
    RealTile<T, Tin, LoadSlots<T, PL>::value> tile;
    tile.load(x, in_row, Nt << logP, logP, col0, ncols);
    const cx<T>* tw = stage_twiddles<T>(tw_off, twl, N, twg);
    tile.commit(reinterpret_cast<T*>(fft_smem), Nt, N, logP, col0, ncols);
    __syncthreads();
    run_fft<T, -1, FftCfg<T>::CMAX, PL>(plan, logP, twl, tw_off, twg);
#pragma unroll 4
    for (int e = threadIdx.x; e < (N + 1) << logP; e += kFftThreads) {
        const int c = e & (P - 1), f = e >> logP;
        if (col0 + c < ncols) {
            So* q = &y[(int64_t)f * out_row + col0 + c];
            if (ntw)
                put_nt(q, r2c_bin(sh, N, logP, f, c, tw));
            else
                put(q, r2c_bin(sh, N, logP, f, c, tw));
        }
    }
}

// Setup form (operator block column, FP64 in, batch over rows s with explicit strides).
template <typename So, typename PL>
__global__ __launch_bounds__(kFftThreads) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_fft_r2c_strided(const double* __restrict__ in, int64_t in_row,
                                                                 int64_t in_batch, So* __restrict__ out,
                                                                 int64_t out_row, int64_t out_batch, int Nt,
                                                                 int ncols, FftPlan plan, int logP,
                                                                 const cx<double>* __restrict__ twg, int twl) {
    cx<double>* sh = reinterpret_cast<cx<double>*>(fft_smem);
    const int N = plan.N, P = 1 << logP;
    const int col0 = column_block() << logP;
    const size_t tw_off = (size_t)(N + 1) * P * sizeof(cx<double>);
    const double* __restrict__ x = in + (int64_t)blockIdx.y * in_batch;
    So* __restrict__ y = out + (int64_t)blockIdx.y * out_batch;
    RealTile<double, double, LoadSlots<double, PL>::value> tile;
    tile.load(x, in_row, Nt << logP, logP, col0, ncols);
    const cx<double>* tw = stage_twiddles<double>(tw_off, twl, N, twg);
    tile.commit(reinterpret_cast<double*>(fft_smem), Nt, N, logP, col0, ncols);
    __syncthreads();
    run_fft<double, -1, FftCfg<double>::CMAX, PL>(plan, logP, twl, tw_off, twg);
    for (int e = threadIdx.x; e < (N + 1) << logP; e += kFftThreads) {
        const int c = e & (P - 1), f = e >> logP;
        if (col0 + c < ncols) put(&y[(int64_t)f * out_row + col0 + c], r2c_bin(sh, N, logP, f, c, tw));
    }
}

// Inverse: X (N+1 complex rows) -> x_j for j < Nt, times out_scale, plus add_scale * addend.
template <typename T, typename PL>
__global__ __launch_bounds__(kFftThreads) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_fft_c2r(const cx<T>* __restrict__ in, int64_t in_row,
                                                         int64_t in_batch, PtrBatch out, int64_t out_row,
                                                         PtrBatch add, T add_scale, int Nt, int ncols,
                                                         FftPlan plan, int logP, const cx<T>* __restrict__ twg,
                                                         int twl, T out_scale, int ntw) {
    cx<T>* sh = reinterpret_cast<cx<T>*>(fft_smem);
    const T* shr = reinterpret_cast<const T*>(fft_smem);
    const int N = plan.N, P = 1 << logP, P1 = P - 1;
    const int col0 = column_block() << logP;
    const size_t tw_off = (size_t)(N + 1) * P * sizeof(cx<T>);
    const cx<T>* __restrict__ y = in + (int64_t)blockIdx.y * in_batch;
    T* __restrict__ x = static_cast<T*>(const_cast<void*>(out.at(blockIdx.y)));
    const T* __restrict__ a = static_cast<const T*>(add.at(blockIdx.y));

    // every spectrum load of the tile in flight (one batch: the launcher checks that
    // (N+1) P <= CMAX threads) before the twiddle copy waits for its own
    constexpr int K = LoadSlots<T, PL>::value;
    const int total = (N + 1) << logP;
    cx<T> val[K];
#pragma unroll
    for (int u = 0; u < K; ++u) {
        const int e = min(u * kFftThreads + (int)threadIdx.x, total - 1);
        const int c = e & P1, f = e >> logP;
        val[u] = y[(int64_t)f * in_row + min(col0 + c, ncols - 1)];
    }
    const cx<T>* tw = stage_twiddles<T>(tw_off, twl, N, twg);
#pragma unroll
    for (int u = 0; u < K; ++u) {
        const int e = u * kFftThreads + (int)threadIdx.x;
        if (e < total) sh[e] = (col0 + (e & P1) < ncols) ? val[u] : cx<T>{0, 0};
    }
    __syncthreads();
    c2r_split<T>(sh, N, logP, tw);
    __syncthreads();
    run_fft<T, 1, FftCfg<T>::CMAX, PL>(plan, logP, twl, tw_off, twg);
    const int nout = Nt << logP;
    for (int e0 = 0; e0 < nout; e0 += kLoadUnroll * kFftThreads) {
        T av[kLoadUnroll];
#pragma unroll
        for (int u = 0; u < kLoadUnroll; ++u) {
            const int e = min(e0 + u * kFftThreads + (int)threadIdx.x, nout - 1);
            const int c = e & P1, j = e >> logP;
            av[u] = a ? a[(int64_t)j * out_row + min(col0 + c, ncols - 1)] : (T)0;
        }
#pragma unroll
        for (int u = 0; u < kLoadUnroll; ++u) {
            const int e = e0 + u * kFftThreads + (int)threadIdx.x;
            const int c = e & P1, j = e >> logP;
            if (e < nout && col0 + c < ncols) {
                const T v = out_scale * shr[2 * (((j >> 1) << logP) + c) + (j & 1)];
                T* q = &x[(int64_t)j * out_row + col0 + c];
                const T w = a ? fma(add_scale, av[u], v) : v;
                if (ntw)
                    __builtin_nontemporal_store(w, q);
                else
                    *q = w;
            }
        }
    }
}

// ---- vector-side transforms with fixed column tiles (FP32 / FP64, compile-time plans) -----
// The same transforms as k_fft_r2c / k_fft_c2r at their widest tile, with the tile width
// 2^LOGP a compile-time constant (every index is then shifts and masks) and the two ends of
// each transform fused with its global memory accesses; the arithmetic counts, not the
// memory traffic, bounded the general kernels:
//  - forward: every thread of the first pass loads its butterflies' inputs straight from the
//    real rows (z_n = x_{2n} + i x_{2n+1}; the upper half n >= N/2 is the zero padding and is
//    neither loaded nor added), so the input never passes through LDS; the output bins are
//    formed in pairs f, N-f, which share both spectrum reads and the twiddle product:
//    X_f = E + T, X_{N-f} = conj(E - T) with E = (Z_f + conj Z_{N-f}) / 2 and T = W_{2N}^f O;
//  - inverse: the spectrum rows f and N-f are loaded into registers and split into Z_f, Z_{N-f}
//    before the first LDS write (one LDS round trip and one barrier fewer).
template <typename PL>
struct FirstRadix;
template <int R0, int... Rs>
struct FirstRadix<CtPlan<R0, Rs...>> {
    static constexpr int value = R0;
};
// The passes of a plan after its first one.
template <typename T, int DIR, int CMAX, bool TWL, typename PL>
struct RestPasses;
template <typename T, int DIR, int CMAX, bool TWL, int R0, int... Rs>
struct RestPasses<T, DIR, CMAX, TWL, CtPlan<R0, Rs...>> {
    __device__ static void run(int logP, size_t tw_off, const cx<T>* __restrict__ twg) {
        if constexpr (sizeof...(Rs) > 0)
            ct_passes<T, DIR, CMAX, TWL, CtPlan<R0, Rs...>::N, R0, Rs...>(logP, tw_off, twg);
    }
};

// Global pointers (address space 1), so that the accesses compile to global rather than flat
// memory instructions.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;

// A complex value stored to a vector-side spectrum row: FP32 runs of >= 64 bytes per row go
// non-temporal (see put_nt); FP64 values use ordinary 16-byte stores, as the general kernels do.
template <typename T, int LOGP>
__device__ __forceinline__ void put_vec(gptr<cx<T>> q, cx<T> v) {
    if constexpr (sizeof(T) == 4 && (8 << LOGP) >= 64) {
        typedef float f2v __attribute__((ext_vector_type(2)));
        __builtin_nontemporal_store(f2v{v.re, v.im}, (gptr<f2v>)q);
    } else {
        q->re = v.re;
        q->im = v.im;
    }
}

template <typename T, typename PL, int LOGP>
__global__ __launch_bounds__(kFftThreads) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_vr2c(
    PtrBatch in, int64_t in_row, cx<T>* __restrict__ out, int64_t out_row, int64_t out_batch, int Nt, int ncols,
    const cx<T>* __restrict__ twg) {
    constexpr int N = PL::N, P = 1 << LOGP, R = FirstRadix<PL>::value, NR = N / R;
    constexpr int RSTEP = kFftThreads >> LOGP;  // rows a thread advances per loop step
    constexpr int NB = (NR * P + kFftThreads - 1) / kFftThreads;  // first-pass butterflies per thread
    constexpr bool TWL = ct_twl<T>(N);
    static_assert(R % 2 == 0, "the zero padding is the upper half of each first-pass butterfly");
    cx<T>* sh = reinterpret_cast<cx<T>*>(fft_smem);
    const size_t tw_off = (size_t)(N + 1) * P * sizeof(cx<T>);
    const int col0 = column_block() << LOGP;
    const int tid = threadIdx.x;
    const int c = tid & (P - 1), j = tid >> LOGP;  // column; first-pass butterfly / first bin pair
    const bool live = col0 + c < ncols;
    const gptr<const T> xc = (gptr<const T>)static_cast<const T*>(in.at(blockIdx.y)) + min(col0 + c, ncols - 1);
    // first pass (Ns = 1), butterflies jb = j + b RSTEP < NR: inputs n = jb + r NR for r < R/2,
    // loaded from rows 2n, 2n+1 (every load of the thread in flight before the first DFT)
    cx<T> v[NB][R];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int jb = j + b * RSTEP;
        if (jb < NR) {
#pragma unroll
            for (int r = 0; r < R / 2; ++r) {
                const int n = jb + r * NR;
                v[b][r].re = (2 * n < Nt && live) ? xc[(int64_t)(2 * n) * in_row] : (T)0;
                v[b][r].im = (2 * n + 1 < Nt && live) ? xc[(int64_t)(2 * n + 1) * in_row] : (T)0;
            }
        }
    }
    const cx<T>* tw = stage_twiddles<T>(tw_off, TWL, N, twg);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int jb = j + b * RSTEP;
        if (jb < NR) {
            Dft<R, -1, T>::run_hz(v[b]);
#pragma unroll
            for (int r = 0; r < R; ++r) sh[((jb * R + r) << LOGP) + c] = v[b][r];
        }
    }
    __syncthreads();
    RestPasses<T, -1, FftCfg<T>::CMAX, TWL, PL>::run(LOGP, tw_off, twg);
    // bins in pairs (f, N - f), f = j, j + RSTEP, ... <= N/2; this thread keeps column c
    if (!live) return;
    const gptr<cx<T>> yc = (gptr<cx<T>>)(out + (int64_t)blockIdx.y * out_batch + col0 + c);
    gptr<cx<T>> q0 = yc + (int64_t)j * out_row;
    gptr<cx<T>> q1 = yc + (int64_t)(N - j) * out_row;
    const int64_t qstep = (int64_t)RSTEP * out_row;
    for (int f = j; f <= N / 2; f += RSTEP, q0 += qstep, q1 -= qstep) {
        const int g = f == 0 ? 0 : N - f;
        const cx<T> Z = sh[(f << LOGP) + c];
        const cx<T> Zc = cconj(sh[(g << LOGP) + c]);
        const cx<T> E = cscale(cadd(Z, Zc), (T)0.5);
        const cx<T> O = cmul_i<-1>(cscale(csub(Z, Zc), (T)0.5));
        const cx<T> Tw = cmul(tw[f], O);
        put_vec<T, LOGP>(q0, cadd(E, Tw));
        if (2 * f != N) put_vec<T, LOGP>(q1, cconj(csub(E, Tw)));
    }
}

template <typename T, typename PL, int LOGP>
__global__ __launch_bounds__(kFftThreads) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_vc2r(
    const cx<T>* __restrict__ in, int64_t in_row, int64_t in_batch, PtrBatch out, int64_t out_row, PtrBatch add,
    T add_scale, int Nt, int ncols, const cx<T>* __restrict__ twg, T out_scale) {
    constexpr int N = PL::N, P = 1 << LOGP;
    constexpr int RSTEP = kFftThreads >> LOGP;
    constexpr bool TWL = ct_twl<T>(N);
    constexpr int K = (N / 2 + 1 + RSTEP - 1) / RSTEP;  // bin pairs per thread (upper bound)
    cx<T>* sh = reinterpret_cast<cx<T>*>(fft_smem);
    const T* shr = reinterpret_cast<const T*>(fft_smem);
    const size_t tw_off = (size_t)(N + 1) * P * sizeof(cx<T>);
    const int col0 = column_block() << LOGP;
    const int tid = threadIdx.x;
    const int c = tid & (P - 1), j0 = tid >> LOGP;
    const bool live = col0 + c < ncols;
    const int cc = min(col0 + c, ncols - 1);
    const gptr<const cx<T>> yc = (gptr<const cx<T>>)(in + (int64_t)blockIdx.y * in_batch + cc);
    // rows f and N - f of every pair f = j0 + u RSTEP <= N/2, all loads in flight together
    cx<T> yf[K], yg[K];
#pragma unroll
    for (int u = 0; u < K; ++u) {
        const int f = min(j0 + u * RSTEP, N / 2);
        const gptr<const cx<T>> pf = yc + (int64_t)f * in_row;
        const gptr<const cx<T>> pg = yc + (int64_t)(N - f) * in_row;
        yf[u] = cx<T>{pf->re, pf->im};
        yg[u] = cx<T>{pg->re, pg->im};
    }
    // the addend (the prior term of H) of every output row this thread writes, loaded now so
    // that its latency hides behind the transform
    constexpr int NJ = (N + RSTEP - 1) / RSTEP;  // rows per thread, upper bound (Nt <= N)
    const T* ab = static_cast<const T*>(add.at(blockIdx.y));
    T av[NJ];
    {
        const gptr<const T> acol = (gptr<const T>)ab + cc;
#pragma unroll
        for (int u = 0; u < NJ; ++u) {
            const int jr = min(j0 + u * RSTEP, Nt - 1);
            av[u] = ab ? acol[(int64_t)jr * out_row] : (T)0;
        }
    }
    const cx<T>* tw = stage_twiddles<T>(tw_off, TWL, N, twg);
    if (TWL) __syncthreads();  // the twiddles staged in LDS
    // inverse split (as c2r_split): Z_f = E + i O, E = (Y_f + conj Y_g) / 2,
    // O = (Y_f - conj Y_g) / 2 * conj(W_{2N}^f), and likewise Z_g for g = N - f (f != 0, g != f)
#pragma unroll
    for (int u = 0; u < K; ++u) {
        const int f = j0 + u * RSTEP, g = N - f;
        if (f > N / 2) break;
        const cx<T> Yf = live ? yf[u] : cx<T>{0, 0}, Yg = live ? yg[u] : cx<T>{0, 0};
        {
            const cx<T> b = cconj(Yg);
            const cx<T> E = cscale(cadd(Yf, b), (T)0.5);
            const cx<T> O = cmul(cscale(csub(Yf, b), (T)0.5), cconj(tw[f]));
            sh[(f << LOGP) + c] = cadd(E, cmul_i<1>(O));
        }
        if (f != 0 && g != f) {
            const cx<T> b = cconj(Yf);
            const cx<T> E = cscale(cadd(Yg, b), (T)0.5);
            const cx<T> O = cmul(cscale(csub(Yg, b), (T)0.5), cconj(tw[g]));
            sh[(g << LOGP) + c] = cadd(E, cmul_i<1>(O));
        }
    }
    __syncthreads();
    // the last pass writes only z_m, m < N/2: rows j < Nt <= N of x come from those
    ct_run<T, 1, FftCfg<T>::CMAX, TWL, true>(PL{}, LOGP, tw_off, twg);
    // x_j = out_scale z (j even: real part, odd: imaginary part of z_{j/2}) + add_scale a_j for
    // rows j = j0, j0 + RSTEP, ... < Nt of column c
    if (!live) return;
    const gptr<T> xcol = (gptr<T>)static_cast<T*>(const_cast<void*>(out.at(blockIdx.y))) + col0 + c;
#pragma unroll
    for (int u = 0; u < NJ; ++u) {
        const int jr = j0 + u * RSTEP;
        if (jr < Nt) {
            const T v = out_scale * shr[2 * (((jr >> 1) << LOGP) + c) + (jr & 1)];
            const T w = ab ? fma(add_scale, av[u], v) : v;
            const gptr<T> q = xcol + (int64_t)jr * out_row;
            if constexpr ((sizeof(T) << LOGP) >= 64)
                __builtin_nontemporal_store(w, q);
            else
                *q = w;
        }
    }
}

// Plans the fused kernels take at the widest tile, as measured against the general kernels
// (FP64 N = 420 with the plan 4, 5, 3, 7, then both kernels moved to 12, 5, 7).
// Forward: an even first radix, in FP32 one first-pass butterfly per thread, in FP64 a tile of
// at least four columns (FP64 N = 420 and 1000: 12-20 % faster; N = 2000, two columns, where
// the first-pass loads sit in half the waves: 5 % slower).  Inverse: every FP32 plan; in FP64
// tiles of at most four columns (N = 1000 and 2000: 5-7 % faster) and wider ones for several
// vectors (N = 420, eight columns: 6-10 % faster for 8-64 vectors, 5 % slower for one).
template <typename T, typename PL>
constexpr bool vec_fused_r2c() {
    constexpr int lp = ct_log_cols<T>(PL::N);
    return FirstRadix<PL>::value % 2 == 0 &&
           (sizeof(T) == 8 ? lp >= 2 : (PL::N / FirstRadix<PL>::value) << lp <= kFftThreads);
}
template <typename T, typename PL>
constexpr bool vec_fused_c2r(int nb) {
    return sizeof(T) == 4 || ct_log_cols<T>(PL::N) <= 2 || nb > 1;
}

// Data side: reduce split partial sums over spans, inverse transform, keep j < Nt, scale;
// then either store d (F) or zero-pad, forward transform and store the bins (H).  One
// sensor (column) per workgroup, whose partial sums part[b][s][f][span] are contiguous.
template <typename T, bool HMODE, typename PL>
__global__ __launch_bounds__(kFftThreads) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_dside(const cx<T>* __restrict__ part, int nspan, int64_t part_batch,
                                                       PtrBatch dout, cx<T>* __restrict__ dh, int64_t dh_batch,
                                                       int Nt, int Nd, FftPlan plan, const cx<T>* __restrict__ twg,
                                                       int twl, T scale) {
    cx<T>* sh = reinterpret_cast<cx<T>*>(fft_smem);
    T* shr = reinterpret_cast<T*>(fft_smem);
    constexpr int logP = 0;
    const int N = plan.N;
    const int s = blockIdx.x;
    const size_t tw_off = (size_t)(N + 1) * sizeof(cx<T>);
    const cx<T>* tw = stage_twiddles<T>(tw_off, twl, N, twg);
    const cx<T>* __restrict__ pb = part + (int64_t)blockIdx.y * part_batch + (int64_t)s * (N + 1) * nspan;

    for (int f = threadIdx.x; f <= N; f += kFftThreads) {
        const cx<T>* q = pb + (int64_t)f * nspan;
        cx<T> acc = cx<T>{0, 0};
#pragma unroll 8
        for (int sp = 0; sp < nspan; ++sp) acc = cadd(acc, q[sp]);
        sh[f] = acc;
    }
    __syncthreads();
    c2r_split<T>(sh, N, logP, tw);
    __syncthreads();
    run_fft<T, 1, FftCfg<T>::CMAX, PL>(plan, logP, twl, tw_off, twg);
    if (!HMODE) {
        T* __restrict__ d = static_cast<T*>(const_cast<void*>(dout.at(blockIdx.y)));
        for (int j = threadIdx.x; j < Nt; j += kFftThreads) d[(int64_t)j * Nd + s] = scale * shr[j];
        return;
    }
    // keep samples j < Nt (scaled), zero the padding, transform forward again
    for (int j = threadIdx.x; j < 2 * N; j += kFftThreads) shr[j] = (j < Nt) ? scale * shr[j] : (T)0;
    __syncthreads();
    run_fft<T, -1, FftCfg<T>::CMAX, PL>(plan, logP, twl, tw_off, twg);
    cx<T>* __restrict__ o = dh + (int64_t)blockIdx.y * dh_batch;
    for (int f = threadIdx.x; f <= N; f += kFftThreads) o[(int64_t)f * Nd + s] = r2c_bin(sh, N, logP, f, 0, tw);
}

// ----------------------------------------------------------------------------------------
static size_t elem_of(Real r) { return r == Real::F64 ? 16 : 8; }
static int cmax_of(Real r) { return r == Real::F64 ? FftCfg<double>::CMAX : FftCfg<float>::CMAX; }

static bool twl_of(int N, Real r) { return tile_twl(N, elem_of(r), cmax_of(r)); }

int fft_log_cols(int N, Real r) { return tile_log_cols(N, elem_of(r), cmax_of(r), twl_of(N, r)); }

size_t fft_lds_bytes(int N, int logP, Real r) {
    const size_t elem = elem_of(r);
    return (size_t)(N + 1) * ((size_t)1 << logP) * elem + (twl_of(N, r) ? (size_t)2 * N * elem : 0);
}

static inline unsigned nblk(int n, int logP) { return (unsigned)((n + (1 << logP) - 1) >> logP); }

// One batch of CMAX loads per thread covers a whole input tile (Nt P <= (N+1) P elements).
static bool one_batch(int N, int logP, Real r) {
    return ((int64_t)(N + 1) << logP) <= (int64_t)cmax_of(r) * kFftThreads;
}

// Narrow batches (the data side: Nd columns) get fewer columns per workgroup so that the
// launch still spreads over the chip; wide ones keep the largest tile that fits.
static int pick_log_cols(int N, Real r, int ncols, int nb) {
    int lp = fft_log_cols(N, r);
    while (lp > 0 && (int64_t)nblk(ncols, lp) * nb < 512) --lp;
    return lp;
}

// Vector-side transforms (many columns per workgroup) use two-pass plans where a composite
// radix (16 = 4 x 4, 20 = 4 x 5, 21 = 3 x 7) fits in registers: every pass costs a trip through
// LDS and a workgroup barrier.  The data-side kernel transforms one column per workgroup and
// keeps the finer plans, which give more threads work per pass.
typedef CtPlan<8, 4> Plan32;
typedef CtPlan<8, 8> Plan64;
typedef CtPlan<8, 16> Plan128;
typedef CtPlan<16, 16> Plan256;
typedef CtPlan<20, 21> Plan420;
typedef CtPlan<8, 8, 8> Plan512;
typedef CtPlan<8, 5, 5, 5> Plan1000d;
typedef CtPlan<16, 5, 5, 5> Plan2000d;
typedef CtPlan<16, 5, 5, 5, 2> Plan4000d;
typedef CtPlan<20, 20, 5> Plan2000;
typedef CtPlan<20, 20, 5, 2> Plan4000;
#define BT_STATIC_PLANS(X) \
    X(0, Plan32)           \
    X(1, Plan64)           \
    X(2, Plan128)          \
    X(3, Plan256)          \
    X(4, Plan420)          \
    X(5, Plan512)          \
    X(6, Plan1000d)        \
    X(7, Plan2000)         \
    X(8, Plan4000)
typedef CtPlan<8, 8, 2> Plan128f;
typedef CtPlan<8, 8, 4> Plan256f;
typedef CtPlan<4, 5, 3, 7> Plan420f;
typedef CtPlan<12, 5, 7> Plan420d;
#define BT_STATIC_PLANS_FINE(X) \
    X(0, Plan32)                \
    X(1, Plan64)                \
    X(2, Plan128f)              \
    X(3, Plan256f)              \
    X(4, Plan420f)              \
    X(5, Plan512)               \
    X(6, Plan1000d)             \
    X(7, Plan2000d)             \
    X(8, Plan4000d)

// FP64 data-side kernel (two transforms in one kernel): radices of at most 8.
typedef CtPlan<8, 5, 5, 5, 2> Plan2000df;
typedef CtPlan<8, 5, 5, 5, 4> Plan4000df;
#define BT_STATIC_PLANS64_FINE(X) \
    X(0, Plan420f)                \
    X(1, Plan1000d)               \
    X(2, Plan2000df)              \
    X(3, Plan4000df)              \
    X(4, Plan32)                  \
    X(5, Plan64)                  \
    X(6, Plan128f)                \
    X(7, Plan256f)                \
    X(8, Plan512)

// FP64 transforms (double registers: plans of radix at most 16 where they do not spill), for the
// benchmarked lengths N = 32 .. 512, 420, 1000, 2000 and 4000; 420 in three passes (12 = 4 x 3
// in registers): 5-8 % faster vector transforms and setup than the four passes 4, 5, 3, 7.
#define BT_STATIC_PLANS64(X) \
    X(0, Plan420d)           \
    X(1, Plan1000d)          \
    X(2, Plan2000d)          \
    X(3, Plan4000d)          \
    X(4, Plan32)             \
    X(5, Plan64)             \
    X(6, Plan128f)           \
    X(7, Plan256f)           \
    X(8, Plan512)

// Index of the compile-time plan of `plan`'s length in the table of its precision, or -1; for
// FP32 the same index selects the plan of that length in the vector-side or the fine table.
static int static_plan_id(const FftPlan& p, Real r) {
    // the kernels size their load slots for the widest tile fft_log_cols allows
    static_assert(ct_log_cols<float>(420) == 4 && LoadSlots<float, Plan420>::value == 14, "tile rule");
    static_assert(ct_log_cols<double>(420) == 3 && !ct_twl<double>(420) && LoadSlots<double, Plan420f>::value == 7,
                  "tile rule");
    static_assert(ct_log_cols<double>(2000) == 1 && LoadSlots<double, Plan2000d>::value == 8 &&
                      ct_log_cols<double>(4000) == 0 && LoadSlots<double, Plan4000d>::value == 8,
                  "tile rule");
    static_assert(ct_log_cols<float>(1000) == 3 && LoadSlots<float, Plan1000d>::value == 16 &&
                      ct_log_cols<float>(2000) == 2 && LoadSlots<float, Plan2000>::value == 16 &&
                      ct_log_cols<float>(4000) == 1 && LoadSlots<float, Plan4000>::value == 16,
                  "tile rule");
    // a compile-time plan applies to any transform of its length (its own radices replace
    // the runtime factorisation; the twiddle table depends on N only)
#define BT_MATCH(ID, PLAN) \
    if (p.N == PLAN::N) return ID;
    if (r == Real::F32) {
        BT_STATIC_PLANS(BT_MATCH)
    } else {
        BT_STATIC_PLANS64(BT_MATCH)
    }
#undef BT_MATCH
    return -1;
}

hipError_t launch_fft_r2c(Real r, Real ir, Stor os, const PtrBatch& in, int64_t in_row, int nb, void* out,
                          int64_t out_row, int64_t out_batch, int Nt, int ncols, const FftPlan& plan,
                          const void* tw, hipStream_t st) {
    if (fft_log_cols(plan.N, r) < 0 || nb <= 0 || nb > kMaxBatch) return hipErrorInvalidValue;
    const int lp = pick_log_cols(plan.N, r, ncols, nb);
    if (!one_batch(plan.N, lp, r)) return hipErrorInvalidValue;
    const int twl = twl_of(plan.N, r);
    dim3 grid(nblk(ncols, lp), nb), block(kFftThreads);
    const size_t lds = fft_lds_bytes(plan.N, lp, r);
    if (r == Real::F32 && ir == Real::F32 && os == Stor::C64) {
#define BT_R2C(PLAN)                                                                                       \
    k_fft_r2c<float, float, cx<float>, PLAN><<<grid, block, lds, st>>>(in, in_row, (cx<float>*)out, out_row, \
                                                                       out_batch, Nt, ncols, plan, lp,      \
                                                                       (const cx<float>*)tw, twl, (8 << lp) >= 64)
        // compile-time plans at their widest tile: the fused fixed-tile kernel
#define BT_R2C_V(PLAN)                                                                                    \
    do {                                                                                                  \
        if constexpr (vec_fused_r2c<float, PLAN>()) {                                                     \
            if (lp == ct_log_cols<float>(PLAN::N)) {                                                      \
                k_vr2c<float, PLAN, ct_log_cols<float>(PLAN::N)><<<grid, block, lds, st>>>(               \
                    in, in_row, (cx<float>*)out, out_row, out_batch, Nt, ncols, (const cx<float>*)tw);    \
                break;                                                                                    \
            }                                                                                             \
        }                                                                                                 \
        BT_R2C(PLAN);                                                                                     \
    } while (0)
        switch (static_plan_id(plan, r)) {
#define BT_CASE(ID, PLAN) \
    case ID: BT_R2C_V(PLAN); break;
            BT_STATIC_PLANS(BT_CASE)
#undef BT_CASE
            default: BT_R2C(RuntimePlan); break;
        }
#undef BT_R2C_V
#undef BT_R2C
    } else if (r == Real::F64 && ir == Real::F64 && os == Stor::C128) {
#define BT_R2C64(PLAN)                                                                                   \
    k_fft_r2c<double, double, cx<double>, PLAN><<<grid, block, lds, st>>>(                               \
        in, in_row, (cx<double>*)out, out_row, out_batch, Nt, ncols, plan, lp, (const cx<double>*)tw, twl, 0)
#define BT_R2C64_V(PLAN)                                                                                  \
    do {                                                                                                  \
        if constexpr (vec_fused_r2c<double, PLAN>()) {                                                    \
            if (lp == ct_log_cols<double>(PLAN::N)) {                                                     \
                k_vr2c<double, PLAN, ct_log_cols<double>(PLAN::N)><<<grid, block, lds, st>>>(             \
                    in, in_row, (cx<double>*)out, out_row, out_batch, Nt, ncols, (const cx<double>*)tw);  \
                break;                                                                                    \
            }                                                                                             \
        }                                                                                                 \
        BT_R2C64(PLAN);                                                                                   \
    } while (0)
        switch (static_plan_id(plan, r)) {
#define BT_CASE(ID, PLAN) \
    case ID: BT_R2C64_V(PLAN); break;
            BT_STATIC_PLANS64(BT_CASE)
#undef BT_CASE
            default: BT_R2C64(RuntimePlan); break;
        }
#undef BT_R2C64_V
#undef BT_R2C64
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fft_r2c_strided(Stor os, const double* in, int64_t in_row, int64_t in_batch, int nb, void* out,
                                  int64_t out_row, int64_t out_batch, int Nt, int ncols, const FftPlan& plan,
                                  const void* tw64, hipStream_t st) {
    if (fft_log_cols(plan.N, Real::F64) < 0 || nb <= 0) return hipErrorInvalidValue;
    const int lp = pick_log_cols(plan.N, Real::F64, ncols, nb);
    if (!one_batch(plan.N, lp, Real::F64)) return hipErrorInvalidValue;
    const int twl = twl_of(plan.N, Real::F64);
    dim3 grid(nblk(ncols, lp), nb), block(kFftThreads);
    const size_t lds = fft_lds_bytes(plan.N, lp, Real::F64);
    const cx<double>* tw = (const cx<double>*)tw64;
    const int pid = static_plan_id(plan, Real::F64);
#define BT_STR(SO, PLAN)                                                                                \
    k_fft_r2c_strided<SO, PLAN><<<grid, block, lds, st>>>(in, in_row, in_batch, (SO*)out, out_row, out_batch, \
                                                          Nt, ncols, plan, lp, tw, twl)
#define BT_STR_PLAN(SO)                    \
    switch (pid) {                         \
        BT_STATIC_PLANS64(BT_CASE)         \
        default: BT_STR(SO, RuntimePlan); break; \
    }
    switch (os) {
        case Stor::C128:
#define BT_CASE(ID, PLAN) \
    case ID: BT_STR(cx<double>, PLAN); break;
            BT_STR_PLAN(cx<double>)
#undef BT_CASE
            break;
        case Stor::C64:
#define BT_CASE(ID, PLAN) \
    case ID: BT_STR(cx<float>, PLAN); break;
            BT_STR_PLAN(cx<float>)
#undef BT_CASE
            break;
        case Stor::BF16:
#define BT_CASE(ID, PLAN) \
    case ID: BT_STR(bf16c, PLAN); break;
            BT_STR_PLAN(bf16c)
#undef BT_CASE
            break;
    }
#undef BT_STR_PLAN
#undef BT_STR
    return hipGetLastError();
}

hipError_t launch_fft_c2r(Real r, const void* in, int64_t in_row, int64_t in_batch, int nb, const PtrBatch& out,
                          int64_t out_row, const PtrBatch& add, double add_scale, int Nt, int ncols,
                          const FftPlan& plan, const void* tw, double out_scale, hipStream_t st) {
    if (fft_log_cols(plan.N, r) < 0 || nb <= 0 || nb > kMaxBatch) return hipErrorInvalidValue;
    const int lp = pick_log_cols(plan.N, r, ncols, nb);
    if (!one_batch(plan.N, lp, r)) return hipErrorInvalidValue;
    const int twl = twl_of(plan.N, r);
    dim3 grid(nblk(ncols, lp), nb), block(kFftThreads);
    const size_t lds = fft_lds_bytes(plan.N, lp, r);
    if (r == Real::F32) {
#define BT_C2R(PLAN)                                                                                            \
    k_fft_c2r<float, PLAN><<<grid, block, lds, st>>>((const cx<float>*)in, in_row, in_batch, out, out_row, add, \
                                                     (float)add_scale, Nt, ncols, plan, lp, (const cx<float>*)tw, \
                                                     twl, (float)out_scale, (4 << lp) >= 64)
#define BT_C2R_V(PLAN)                                                                                     \
    do {                                                                                                   \
        if (lp == ct_log_cols<float>(PLAN::N) && vec_fused_c2r<float, PLAN>(nb)) {                         \
            k_vc2r<float, PLAN, ct_log_cols<float>(PLAN::N)><<<grid, block, lds, st>>>(                    \
                (const cx<float>*)in, in_row, in_batch, out, out_row, add, (float)add_scale, Nt, ncols,     \
                (const cx<float>*)tw, (float)out_scale);                                                   \
            break;                                                                                         \
        }                                                                                                  \
        BT_C2R(PLAN);                                                                                      \
    } while (0)
        switch (static_plan_id(plan, r)) {
#define BT_CASE(ID, PLAN) \
    case ID: BT_C2R_V(PLAN); break;
            BT_STATIC_PLANS(BT_CASE)
#undef BT_CASE
            default: BT_C2R(RuntimePlan); break;
        }
#undef BT_C2R_V
#undef BT_C2R
    } else {
#define BT_C2R64(PLAN)                                                                                          \
    k_fft_c2r<double, PLAN><<<grid, block, lds, st>>>((const cx<double>*)in, in_row, in_batch, out, out_row, add, \
                                                      add_scale, Nt, ncols, plan, lp, (const cx<double>*)tw, twl, \
                                                      out_scale, (8 << lp) >= 64)
#define BT_C2R64_V(PLAN)                                                                                    \
    do {                                                                                                    \
        if (lp == ct_log_cols<double>(PLAN::N) && vec_fused_c2r<double, PLAN>(nb)) {                         \
            k_vc2r<double, PLAN, ct_log_cols<double>(PLAN::N)><<<grid, block, lds, st>>>(                   \
                (const cx<double>*)in, in_row, in_batch, out, out_row, add, add_scale, Nt, ncols,           \
                (const cx<double>*)tw, out_scale);                                                          \
            break;                                                                                          \
        }                                                                                                   \
        BT_C2R64(PLAN);                                                                                     \
    } while (0)
        switch (static_plan_id(plan, r)) {
#define BT_CASE(ID, PLAN) \
    case ID: BT_C2R64_V(PLAN); break;
            BT_STATIC_PLANS64(BT_CASE)
#undef BT_CASE
            default: BT_C2R64(RuntimePlan); break;
        }
#undef BT_C2R64_V
#undef BT_C2R64
    }
    return hipGetLastError();
}

hipError_t launch_dside(Real r, const void* part, int nspan, int64_t part_batch, int nb, const PtrBatch* dout,
                        void* dh, int64_t dh_batch, int Nt, int Nd, const FftPlan& plan, const void* tw,
                        double scale, hipStream_t st) {
    if (fft_log_cols(plan.N, r) < 0 || nb <= 0 || nb > kMaxBatch) return hipErrorInvalidValue;
    const int twl = twl_of(plan.N, r);
    dim3 grid(Nd, nb), block(kFftThreads);  // one sensor per workgroup
    const size_t lds = fft_lds_bytes(plan.N, 0, r);
    PtrBatch none{};
    const PtrBatch& d = dout ? *dout : none;
    if (r == Real::F32) {
#define BT_DS(MODE, PLAN)                                                                                     \
    k_dside<float, MODE, PLAN><<<grid, block, lds, st>>>((const cx<float>*)part, nspan, part_batch, d,        \
                                                         (cx<float>*)dh, dh_batch, Nt, Nd, plan, (const cx<float>*)tw, \
                                                         twl, (float)scale)
        switch (static_plan_id(plan, r)) {
#define BT_CASE(ID, PLAN)       \
    case ID:                    \
        if (dout)               \
            BT_DS(false, PLAN); \
        else                    \
            BT_DS(true, PLAN);  \
        break;
            BT_STATIC_PLANS_FINE(BT_CASE)
#undef BT_CASE
            default:
                if (dout)
                    BT_DS(false, RuntimePlan);
                else
                    BT_DS(true, RuntimePlan);
                break;
        }
#undef BT_DS
    } else {
#define BT_DS64(MODE, PLAN)                                                                                   \
    k_dside<double, MODE, PLAN><<<grid, block, lds, st>>>((const cx<double>*)part, nspan, part_batch, d,      \
                                                          (cx<double>*)dh, dh_batch, Nt, Nd, plan,            \
                                                          (const cx<double>*)tw, twl, scale)
        switch (static_plan_id(plan, r)) {
#define BT_CASE(ID, PLAN)         \
    case ID:                      \
        if (dout)                 \
            BT_DS64(false, PLAN); \
        else                      \
            BT_DS64(true, PLAN);  \
        break;
            BT_STATIC_PLANS64_FINE(BT_CASE)
#undef BT_CASE
            default:
                if (dout)
                    BT_DS64(false, RuntimePlan);
                else
                    BT_DS64(true, RuntimePlan);
                break;
        }
#undef BT_DS64
    }
    return hipGetLastError();
}


// ========================================================================================
// Four-step transforms for long series (N = N1 N2): when a length-N column does not fit one
// workgroup's LDS with a useful column tile, the half-length complex transform is split
// (paper section 2.4 computes one length-2N DFT per series; only the order of the arithmetic
// changes).  With n = N2 n1 + n2 and k = k1 + N1 k2,
//   Z[k1 + N1 k2] = sum_{n2} W_{N2}^{n2 k2} W_N^{n2 k1} sum_{n1} z[N2 n1 + n2] W_{N1}^{n1 k1},
// so pass A runs N1-point transforms (one per n2, over rows N2 n1 + n2) and applies W_N^{n2 k1},
// pass B runs N2-point transforms (one per k1, over the contiguous rows k1 N2 + n2).  Pass B
// transforms k1 and N1 - k1 side by side (as 2P columns), which puts every bin f next to its
// partner N - f, so the real-to-complex split into the N + 1 bins is its epilogue.  The
// inverse mirrors this: pass C splits, runs the N2-point inverse transforms and applies
// W_N^{-n2 k1}; pass D runs the N1-point inverse transforms and unpacks x[2n], x[2n+1].
// Every global access is a run of P consecutive columns of one row.  The sub-transforms use
// the runtime plans with their own twiddle tables exp(-2 pi i t / (2 Nsub)); twN is the
// operator's table exp(-2 pi i t / (2N)).

// Sub-transforms of the four-step passes: a compile-time plan when one exists for the length
// (twiddles read through the caches: these kernels keep no table in LDS), else the runtime plan.
template <typename T, int DIR, typename PL>
__device__ __forceinline__ void sub_fft(const FftPlan& p, int logP, const cx<T>* __restrict__ tw) {
    if constexpr (PL::kStatic)
        ct_run<T, DIR, FftCfg<T>::CMAX, false>(PL{}, logP, 0, tw);
    else
        fft_lds<T, DIR, FftCfg<T>::CMAX>(p, logP, false, 0, tw);
}

// Input base of batch b: in.at(b), or in.at(0) + b * in_batch when in_batch != 0.
template <typename T>
__device__ __forceinline__ const T* batch_base(const PtrBatch& in, int64_t in_batch, int b) {
    return in_batch ? static_cast<const T*>(in.at(0)) + (int64_t)b * in_batch : static_cast<const T*>(in.at(b));
}

// A: z[n] = x[2n] + i x[2n+1] (zero for rows >= Nt) at n = N2 n1 + n2 for one n2 (blockIdx.y);
// forward N1-point transform over n1; times W_N^{n2 k1}; y[b][k1 N2 + n2][c].
template <typename T, typename Tin, typename PL>
__global__ __launch_bounds__(kFftThreads) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_long_a(
    PtrBatch in, int64_t in_batch, int64_t in_row, int Nt, int ncols, cx<T>* __restrict__ y, int64_t y_row,
    int64_t y_batch, FftPlan p1, int N2, int logP, const cx<T>* __restrict__ tw1, const cx<T>* __restrict__ twN) {
    cx<T>* sh = reinterpret_cast<cx<T>*>(fft_smem);
    const int N1 = p1.N, P1 = (1 << logP) - 1;
    const int col0 = blockIdx.x << logP, n2 = blockIdx.y, b = blockIdx.z;
    const Tin* __restrict__ x = batch_base<Tin>(in, in_batch, b);
    const int total = N1 << logP;
    // every load of the tile in flight at once (the launcher keeps N1 P <= CMAX threads)
    constexpr int K = FftCfg<T>::CMAX;
    T vre[K], vim[K];
#pragma unroll
    for (int u = 0; u < K; ++u) {
        const int e = min(threadIdx.x + u * kFftThreads, total - 1);
        const int c = e & P1, n1 = e >> logP;
        const int64_t j = 2 * ((int64_t)N2 * n1 + n2);
        const int col = min(col0 + c, ncols - 1);
        vre[u] = (T)x[min(j, (int64_t)Nt - 1) * in_row + col];
        vim[u] = (T)x[min(j + 1, (int64_t)Nt - 1) * in_row + col];
    }
#pragma unroll
    for (int u = 0; u < K; ++u) {
        const int e = threadIdx.x + u * kFftThreads;
        if (e < total) {
            const int c = e & P1, n1 = e >> logP;
            const int64_t j = 2 * ((int64_t)N2 * n1 + n2);
            const bool ok = col0 + c < ncols;
            sh[e] = cx<T>{(ok && j < Nt) ? vre[u] : (T)0, (ok && j + 1 < Nt) ? vim[u] : (T)0};
        }
    }
    __syncthreads();
    sub_fft<T, -1, PL>(p1, logP, tw1);
    cx<T>* __restrict__ yb = y + (int64_t)b * y_batch;
#pragma unroll
    for (int u = 0; u < K; ++u) {
        const int e = threadIdx.x + u * kFftThreads;
        if (e < total) {
            const int c = e & P1, k1 = e >> logP;
            if (col0 + c < ncols) yb[((int64_t)k1 * N2 + n2) * y_row + col0 + c] = cmul(sh[e], twN[2 * n2 * k1]);
        }
    }
}

// Blocks of the paired passes: column cc < 2P of LDS holds k1 = a (block 0) or N1 - a
// (block 1) for a = blockIdx.y; when a has no distinct partner (a == 0, 2a == N1) block 1
// repeats block 0 and is not stored.
__device__ __forceinline__ int pair_k1(int a, int blk, int N1) { return blk ? (N1 - a) % N1 : a; }

// B: forward N2-point transforms of rows k1 N2 + n2 for k1 = a and N1 - a, then the split into
// bins X_f = (Z_f + conj Z_{N-f}) / 2 + W_{2N}^f (Z_f - conj Z_{N-f}) / (2i), f = k1 + N1 k2.
template <typename T, typename So, typename PL>
__global__ __launch_bounds__(kFftThreads) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_long_b(
    const cx<T>* __restrict__ y, int64_t y_row, int64_t y_batch, So* __restrict__ out, int64_t out_row,
    int64_t out_batch, int ncols, FftPlan p2, int N1, int logP, const cx<T>* __restrict__ tw2,
    const cx<T>* __restrict__ twN) {
    cx<T>* sh = reinterpret_cast<cx<T>*>(fft_smem);
    const int N2 = p2.N, N = N1 * N2, P = 1 << logP, P1 = P - 1, lq = logP + 1;
    const int col0 = blockIdx.x << logP, a = blockIdx.y, b = blockIdx.z;
    const bool paired = a != 0 && 2 * a != N1;
    const cx<T>* __restrict__ yb = y + (int64_t)b * y_batch;
    const int total = N2 << lq;
    constexpr int K = FftCfg<T>::CMAX;  // the launcher keeps N2 x 2P <= CMAX threads
    {
        cx<T> v[K];
#pragma unroll
        for (int u = 0; u < K; ++u) {
            const int e = min(threadIdx.x + u * kFftThreads, total - 1);
            const int cc = e & (2 * P - 1), n2 = e >> lq;
            const int c = cc & P1, k1 = pair_k1(a, cc >> logP, N1);
            v[u] = yb[((int64_t)k1 * N2 + n2) * y_row + min(col0 + c, ncols - 1)];
        }
#pragma unroll
        for (int u = 0; u < K; ++u) {
            const int e = threadIdx.x + u * kFftThreads;
            if (e < total) sh[e] = v[u];
        }
    }
    __syncthreads();
    sub_fft<T, -1, PL>(p2, lq, tw2);
    So* __restrict__ ob = out + (int64_t)b * out_batch;
#pragma unroll
    for (int u = 0; u < K; ++u) {
        const int e = threadIdx.x + u * kFftThreads;
        if (e >= total) continue;
        const int cc = e & (2 * P - 1), k2 = e >> lq;
        const int blk = cc >> logP, c = cc & P1;
        if (col0 + c >= ncols) continue;
        const int k1 = pair_k1(a, blk, N1);
        int f = k1 + N1 * k2;
        if (blk == 1 && !paired) {
            if (a != 0 || k2 != 0) continue;  // a repeated block stores nothing, except bin N
            f = N;
        }
        // partner of Z_f: Z_{N-f} (Z_0 for f = 0 and f = N)
        int prow, pblk;
        if (k1 == 0) {
            prow = (f == N) ? 0 : (N2 - k2) % N2;
            pblk = blk;
        } else {
            prow = N2 - 1 - k2;
            pblk = (N1 - k1 == a) ? 0 : 1;
        }
        const cx<T> Z = sh[((f == N ? 0 : k2) << lq) + cc];
        const cx<T> Zc = cconj(sh[(prow << lq) + (pblk << logP) + c]);
        const cx<T> E = cscale(cadd(Z, Zc), (T)0.5);
        const cx<T> O = cmul_i<-1>(cscale(csub(Z, Zc), (T)0.5));
        put_nt(&ob[(int64_t)f * out_row + col0 + c], cadd(E, cmul(twN[f], O)));
    }
}

// C: split of the bins Y_f (f = k1 + N1 k2 for k1 = a, N1 - a; Y_N in block 1, row 0 when
// a == 0) into Z_f = E_f + i O_f, E_f = (Y_f + conj Y_{N-f}) / 2,
// O_f = (Y_f - conj Y_{N-f}) / 2 W_{2N}^{-f}; inverse N2-point transforms over k2; times
// W_N^{-n2 k1}; u[b][k1 N2 + n2][c].
template <typename T, typename PL>
__global__ __launch_bounds__(kFftThreads) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_long_c(
    const cx<T>* __restrict__ bins, int64_t b_row, int64_t b_batch, cx<T>* __restrict__ u, int64_t u_row,
    int64_t u_batch, int ncols, FftPlan p2, int N1, int logP, const cx<T>* __restrict__ tw2,
    const cx<T>* __restrict__ twN) {
    cx<T>* sh = reinterpret_cast<cx<T>*>(fft_smem);
    const int N2 = p2.N, N = N1 * N2, P = 1 << logP, P1 = P - 1, lq = logP + 1;
    const int col0 = blockIdx.x << logP, a = blockIdx.y, b = blockIdx.z;
    const bool paired = a != 0 && 2 * a != N1;
    const cx<T>* __restrict__ bb = bins + (int64_t)b * b_batch;
    const int total = N2 << lq;
    // the launcher keeps N2 x 2P <= CMAX threads, so K slots per thread hold the whole tile
    constexpr int K = FftCfg<T>::CMAX;
    {
        cx<T> v[K];
#pragma unroll
        for (int u = 0; u < K; ++u) {
            const int e = min(threadIdx.x + u * kFftThreads, total - 1);
            const int cc = e & (2 * P - 1), k2 = e >> lq;
            const int blk = cc >> logP, c = cc & P1, k1 = pair_k1(a, blk, N1);
            int f = k1 + N1 * k2;
            if (a == 0 && blk == 1 && k2 == 0) f = N;  // Y_N, the partner of Y_0
            v[u] = bb[(int64_t)f * b_row + min(col0 + c, ncols - 1)];
        }
#pragma unroll
        for (int u = 0; u < K; ++u) {
            const int e = threadIdx.x + u * kFftThreads;
            if (e < total) sh[e] = v[u];
        }
    }
    __syncthreads();
    // split: every element reads itself and its partner, then all write
    cx<T> zf[K];
#pragma unroll
    for (int u2 = 0; u2 < K; ++u2) {
        const int e = threadIdx.x + u2 * kFftThreads;
        if (e < total) {
            const int cc = e & (2 * P - 1), k2 = e >> lq;
            const int blk = cc >> logP, c = cc & P1, k1 = pair_k1(a, blk, N1);
            const int f = k1 + N1 * k2;
            int prow, pblk;
            if (k1 == 0) {
                // partner of f = N1 k2 is N - f = N1 (N2 - k2); of f = 0 it is Y_N (block 1, row 0)
                prow = (k2 == 0) ? 0 : N2 - k2;
                pblk = (k2 == 0) ? 1 : blk;
            } else {
                prow = N2 - 1 - k2;
                pblk = (N1 - k1 == a) ? 0 : 1;
            }
            const cx<T> Yf = sh[e];
            const cx<T> Yg = cconj(sh[(prow << lq) + (pblk << logP) + c]);
            const cx<T> E = cscale(cadd(Yf, Yg), (T)0.5);
            const cx<T> O = cmul(cscale(csub(Yf, Yg), (T)0.5), cconj(twN[f]));
            zf[u2] = cadd(E, cmul_i<1>(O));
        }
    }
    __syncthreads();
#pragma unroll
    for (int u2 = 0; u2 < K; ++u2) {
        const int e = threadIdx.x + u2 * kFftThreads;
        if (e < total) sh[e] = zf[u2];
    }
    __syncthreads();
    sub_fft<T, 1, PL>(p2, lq, tw2);
    cx<T>* __restrict__ ub = u + (int64_t)b * u_batch;
#pragma unroll
    for (int u2 = 0; u2 < K; ++u2) {
        const int e = threadIdx.x + u2 * kFftThreads;
        if (e >= total) continue;
        const int cc = e & (2 * P - 1), n2 = e >> lq;
        const int blk = cc >> logP, c = cc & P1;
        if (col0 + c >= ncols || (blk == 1 && !paired)) continue;
        const int k1 = pair_k1(a, blk, N1);
        ub[((int64_t)k1 * N2 + n2) * u_row + col0 + c] = cmul(sh[e], cconj(twN[2 * n2 * k1]));
    }
}

// D: inverse N1-point transforms over k1 of rows k1 N2 + n2 for one n2 (blockIdx.y), giving
// z[N2 n1 + n2]; out rows 2n and 2n + 1 (< Nt) = out_scale * (Re, Im) (+ add_scale * addend).
template <typename T, typename PL>
__global__ __launch_bounds__(kFftThreads) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_long_d(
    const cx<T>* __restrict__ u, int64_t u_row, int64_t u_batch, PtrBatch out, int64_t out_row, PtrBatch add,
    T add_scale, int Nt, int ncols, FftPlan p1, int N2, int logP, const cx<T>* __restrict__ tw1, T out_scale) {
    cx<T>* sh = reinterpret_cast<cx<T>*>(fft_smem);
    const int N1 = p1.N, P1 = (1 << logP) - 1;
    const int col0 = blockIdx.x << logP, n2 = blockIdx.y, b = blockIdx.z;
    const cx<T>* __restrict__ ub = u + (int64_t)b * u_batch;
    const int total = N1 << logP;
    constexpr int K = FftCfg<T>::CMAX;  // the launcher keeps N1 P <= CMAX threads
    {
        cx<T> v[K];
#pragma unroll
        for (int u = 0; u < K; ++u) {
            const int e = min(threadIdx.x + u * kFftThreads, total - 1);
            const int c = e & P1, k1 = e >> logP;
            v[u] = ub[((int64_t)k1 * N2 + n2) * u_row + min(col0 + c, ncols - 1)];
        }
#pragma unroll
        for (int u = 0; u < K; ++u) {
            const int e = threadIdx.x + u * kFftThreads;
            if (e < total) sh[e] = v[u];
        }
    }
    __syncthreads();
    sub_fft<T, 1, PL>(p1, logP, tw1);
    T* __restrict__ x = static_cast<T*>(const_cast<void*>(out.at(b)));
    const T* __restrict__ ad = static_cast<const T*>(add.at(b));
#pragma unroll
    for (int u = 0; u < K; ++u) {
        const int e = threadIdx.x + u * kFftThreads;
        if (e >= total) continue;
        const int c = e & P1, n1 = e >> logP;
        if (col0 + c >= ncols) continue;
        const int64_t j = 2 * ((int64_t)N2 * n1 + n2);
        const cx<T> z = sh[e];
        if (j < Nt) {
            const T v = out_scale * z.re;
            const int64_t o = j * out_row + col0 + c;
            x[o] = ad ? fma(add_scale, ad[o], v) : v;
        }
        if (j + 1 < Nt) {
            const T v = out_scale * z.im;
            const int64_t o = (j + 1) * out_row + col0 + c;
            x[o] = ad ? fma(add_scale, ad[o], v) : v;
        }
    }
}

// Data side of the long path: part[b][s][f][span] summed over spans into spec[b][f][s].
template <typename T>
__global__ __launch_bounds__(256) void k_sum_spans(const cx<T>* __restrict__ part, int nspan, int64_t part_batch,
                                                   cx<T>* __restrict__ spec, int64_t spec_batch, int nfreq, int Nd) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)nfreq * Nd) return;
    const int f = (int)(e / Nd), s = (int)(e % Nd);
    const cx<T>* q = part + (int64_t)blockIdx.y * part_batch + ((int64_t)s * nfreq + f) * nspan;
    cx<T> acc = cx<T>{0, 0};
    for (int sp = 0; sp < nspan; ++sp) acc = cadd(acc, q[sp]);
    spec[(int64_t)blockIdx.y * spec_batch + e] = acc;
}


// ---- four-step launchers -------------------------------------------------------------------
// Widest column tile (log2) for the passes of N = N1 N2: N1 x P (passes A, D) and N2 x 2P
// (passes B, C) complex values in LDS and per CMAX threads; -1 when not even one column fits.
int long_log_cols(int N1, int N2, Real r) {
    const size_t elem = elem_of(r);
    for (int lp = 6; lp >= 0; --lp) {
        const size_t P = (size_t)1 << lp;
        const size_t a = (size_t)N1 * P, b = (size_t)N2 * 2 * P;
        if (a * elem <= kFftLdsBudget && b * elem <= kFftLdsBudget && a <= (size_t)cmax_of(r) * kFftThreads &&
            b <= (size_t)cmax_of(r) * kFftThreads)
            return lp;
    }
    return -1;
}

static int long_pick_cols(int N1, int N2, Real r, int ncols, int nb) {
    int lp = long_log_cols(N1, N2, r);
    while (lp > 0 && (int64_t)nblk(ncols, lp) * nb * N2 < 2048) --lp;
    return lp;
}

// Compile-time plans of the four-step sub-lengths (N = 10000 = 100 x 100 and 5000 = 50 x 100).
typedef CtPlan<4, 5, 5> Sub100d;
typedef CtPlan<20, 5> Sub100f;
typedef CtPlan<2, 5, 5> Sub50;
// Calls fn(plan tag) with the sub-plan of length N for precision T (RuntimePlan when none).
template <typename T, typename Fn>
static void with_sub_plan(int N, Fn&& fn) {
    if (N == 100) {
        if constexpr (sizeof(T) == 8)
            fn(Sub100d{});
        else
            fn(Sub100f{});
    } else if (N == 50) {
        if constexpr (sizeof(T) == 8)
            fn(Sub50{});
        else
            fn(RuntimePlan{});  // FP32: radix-2 passes with 16 values per thread spill
    } else {
        fn(RuntimePlan{});
    }
}

hipError_t launch_long_r2c(Real r, Real ir, Stor os, const PtrBatch& in, int64_t in_batch, int64_t in_row, int nb,
                           int Nt, int ncols, void* tmp, int64_t tmp_row, int64_t tmp_batch, void* out,
                           int64_t out_row, int64_t out_batch, const FftPlan& p1, const FftPlan& p2, const void* tw1,
                           const void* tw2, const void* twN, hipStream_t st) {
    const int N1 = p1.N, N2 = p2.N;
    const int lp = long_pick_cols(N1, N2, r, ncols, nb);
    if (lp < 0 || nb <= 0 || nb > 65535 || N2 > 65535 || tmp_row < ncols) return hipErrorInvalidValue;
    const unsigned nt = nblk(ncols, lp);
    const size_t elem = elem_of(r);
    const size_t lds_a = ((size_t)N1 << lp) * elem, lds_b = ((size_t)N2 << (lp + 1)) * elem;
    dim3 ga(nt, N2, nb), gb(nt, N1 / 2 + 1, nb), block(kFftThreads);
    if (r == Real::F32 && ir == Real::F32 && os == Stor::C64) {
        with_sub_plan<float>(N1, [&](auto pl) {
            k_long_a<float, float, decltype(pl)><<<ga, block, lds_a, st>>>(
                in, in_batch, in_row, Nt, ncols, (cx<float>*)tmp, tmp_row, tmp_batch, p1, N2, lp,
                (const cx<float>*)tw1, (const cx<float>*)twN);
        });
        with_sub_plan<float>(N2, [&](auto pl) {
            k_long_b<float, cx<float>, decltype(pl)><<<gb, block, lds_b, st>>>(
                (const cx<float>*)tmp, tmp_row, tmp_batch, (cx<float>*)out, out_row, out_batch, ncols, p2, N1, lp,
                (const cx<float>*)tw2, (const cx<float>*)twN);
        });
    } else if (r == Real::F64 && ir == Real::F64) {
        with_sub_plan<double>(N1, [&](auto pl) {
            k_long_a<double, double, decltype(pl)><<<ga, block, lds_a, st>>>(
                in, in_batch, in_row, Nt, ncols, (cx<double>*)tmp, tmp_row, tmp_batch, p1, N2, lp,
                (const cx<double>*)tw1, (const cx<double>*)twN);
        });
        const cx<double>* t = (const cx<double>*)tmp;
        const cx<double>* w2 = (const cx<double>*)tw2;
        const cx<double>* wN = (const cx<double>*)twN;
        with_sub_plan<double>(N2, [&](auto pl) {
            using PL = decltype(pl);
            switch (os) {
                case Stor::C128:
                    k_long_b<double, cx<double>, PL><<<gb, block, lds_b, st>>>(
                        t, tmp_row, tmp_batch, (cx<double>*)out, out_row, out_batch, ncols, p2, N1, lp, w2, wN);
                    break;
                case Stor::C64:
                    k_long_b<double, cx<float>, PL><<<gb, block, lds_b, st>>>(
                        t, tmp_row, tmp_batch, (cx<float>*)out, out_row, out_batch, ncols, p2, N1, lp, w2, wN);
                    break;
                case Stor::BF16:
                    k_long_b<double, bf16c, PL><<<gb, block, lds_b, st>>>(
                        t, tmp_row, tmp_batch, (bf16c*)out, out_row, out_batch, ncols, p2, N1, lp, w2, wN);
                    break;
            }
        });
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_long_c2r(Real r, const void* in, int64_t in_row, int64_t in_batch, int nb, void* tmp,
                           int64_t tmp_row, int64_t tmp_batch, const PtrBatch& out, int64_t out_row,
                           const PtrBatch& add, double add_scale, int Nt, int ncols, const FftPlan& p1,
                           const FftPlan& p2, const void* tw1, const void* tw2, const void* twN, double out_scale,
                           hipStream_t st) {
    const int N1 = p1.N, N2 = p2.N;
    const int lp = long_pick_cols(N1, N2, r, ncols, nb);
    if (lp < 0 || nb <= 0 || nb > 65535 || N2 > 65535 || tmp_row < ncols) return hipErrorInvalidValue;
    const unsigned nt = nblk(ncols, lp);
    const size_t elem = elem_of(r);
    const size_t lds_d = ((size_t)N1 << lp) * elem, lds_c = ((size_t)N2 << (lp + 1)) * elem;
    dim3 gc(nt, N1 / 2 + 1, nb), gd(nt, N2, nb), block(kFftThreads);
    if (r == Real::F32) {
        with_sub_plan<float>(N2, [&](auto pl) {
            k_long_c<float, decltype(pl)><<<gc, block, lds_c, st>>>(
                (const cx<float>*)in, in_row, in_batch, (cx<float>*)tmp, tmp_row, tmp_batch, ncols, p2, N1, lp,
                (const cx<float>*)tw2, (const cx<float>*)twN);
        });
        with_sub_plan<float>(N1, [&](auto pl) {
            k_long_d<float, decltype(pl)><<<gd, block, lds_d, st>>>(
                (const cx<float>*)tmp, tmp_row, tmp_batch, out, out_row, add, (float)add_scale, Nt, ncols, p1, N2,
                lp, (const cx<float>*)tw1, (float)out_scale);
        });
    } else {
        with_sub_plan<double>(N2, [&](auto pl) {
            k_long_c<double, decltype(pl)><<<gc, block, lds_c, st>>>(
                (const cx<double>*)in, in_row, in_batch, (cx<double>*)tmp, tmp_row, tmp_batch, ncols, p2, N1, lp,
                (const cx<double>*)tw2, (const cx<double>*)twN);
        });
        with_sub_plan<double>(N1, [&](auto pl) {
            k_long_d<double, decltype(pl)><<<gd, block, lds_d, st>>>(
                (const cx<double>*)tmp, tmp_row, tmp_batch, out, out_row, add, add_scale, Nt, ncols, p1, N2, lp,
                (const cx<double>*)tw1, out_scale);
        });
    }
    return hipGetLastError();
}

hipError_t launch_sum_spans(Real r, const void* part, int nspan, int64_t part_batch, void* spec, int64_t spec_batch,
                            int nfreq, int Nd, int nb, hipStream_t st) {
    if (nb <= 0 || nb > 65535) return hipErrorInvalidValue;
    dim3 grid((unsigned)(((int64_t)nfreq * Nd + 255) / 256), nb);
    if (r == Real::F32)
        k_sum_spans<float><<<grid, 256, 0, st>>>((const cx<float>*)part, nspan, part_batch, (cx<float>*)spec,
                                                 spec_batch, nfreq, Nd);
    else
        k_sum_spans<double><<<grid, 256, 0, st>>>((const cx<double>*)part, nspan, part_batch, (cx<double>*)spec,
                                                  spec_batch, nfreq, Nd);
    return hipGetLastError();
}

}  // namespace btoep
