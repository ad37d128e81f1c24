// APP kernel (eqs. 1-3).
#include "device_common.h"

#include <climits>

namespace mapdec {

// ---------------------------------------------------------------------------
// APP (eqs. 1-3).  One wave per (frame, i); lanes stride over m'.
//   U_i(D) = sum_{m', delta} alpha_i(m') R(n i + m', D, delta) beta_{i+1}(m' + delta)
//   S_i(D) = prior_i(D) U_i(D),  Z_i = sum_D S_i(D),  APP = S / Z,
//   d log P / d prior_i(D) = U_i(D) / Z_i.
// The row products alpha beta are formed from mantissas and exponent sums
// and scaled by 2^-E_i, E_i the largest exponent sum of the symbol: the
// two rows can peak at opposite ends of the drift range, with their product
// at the posterior's drifts below the FP64 range.

constexpr int kAppChunk = 16;

template <typename T>
__global__ __launch_bounds__(kAppThreads) void k_app(const FrameDesc *__restrict__ fd,
                                                     const Work *__restrict__ tab) {
    // accumulates in FP64 (the rows are FP64); R and the outputs are T
    const Work w = tab[blockIdx.x];
    const FrameDesc &f = fd[w.frame];
    const int i = f.i0 + w.item;
    if (*f.status != kStatusOk) return;
    extern __shared__ __align__(16) unsigned char smem[];
    const int Mt = f.Mt, mn = f.mn, M = f.M, Mn = f.Mn, q = f.q, n = f.n, rho = f.rho;
    const int s0 = f.s0;
    double *al = (double *)smem;
    double *be = al + Mt;            // Mt + 2 mn, padded
    double *U = be + Mt + 2 * mn;    // q
    const int tid = threadIdx.x;
    const double *A = f.alpha + (size_t)(i - f.i0) * Mt;
    const double *B = f.beta + (size_t)(i + 1 - f.i0) * Mt;
    for (int j = tid; j < Mt; j += kAppThreads) {
        al[j] = A[j];
        be[mn + j] = B[j];
    }
    for (int j = tid; j < mn; j += kAppThreads) {
        be[j] = 0.0;
        be[mn + Mt + j] = 0.0;
    }
    __syncthreads();
    // E_i = max over m', delta of the exponent sum of alpha(m') beta(m' + delta)
    int emax = INT_MIN / 2;
    for (int mi = tid; mi < Mt; mi += kAppThreads) {
        if (!(al[mi] > 0.0)) continue;
        int eb = INT_MIN / 2;
        for (int k = 0; k < Mn; ++k)
            if (be[mi + k] > 0.0) eb = max(eb, ilogb(be[mi + k]));
        if (eb > INT_MIN / 2) emax = max(emax, ilogb(al[mi]) + eb);
    }
    for (int off = 32; off >= 1; off >>= 1) emax = max(emax, __shfl_xor(emax, off, 64));

    const T *R = (const T *)f.R;
    const size_t sp = (size_t)f.sp;
    for (int dc = 0; dc < q; dc += kAppChunk) {
        double acc[kAppChunk];
#pragma unroll
        for (int e = 0; e < kAppChunk; ++e) acc[e] = 0.0;
        for (int mi = tid; mi < Mt; mi += kAppThreads) {
            const int s = n * i + mi - M;
            if (s < 0 || s > rho) continue;
            // R's column: the start index's, or (a codebook per symbol) the
            // symbol's and drift state's
            const int col = f.percol ? (i - f.i0) * Mt + mi : s - s0;
            const double av = al[mi];
            if (!(av > 0.0)) continue;
            // 2^-E alpha(m') beta(m' + delta), delta = k - mn
            double ab[2 * kMaxMn + 1];
            const int ea = ilogb(av);
            const double fa = scalbn(av, -ea);
            for (int k = 0; k < Mn; ++k) {
                const double b = be[mi + k];
                ab[k] = b > 0.0 ? scalbn(fa * scalbn(b, -ilogb(b)), ea + ilogb(b) - emax) : 0.0;
            }
#pragma unroll
            for (int e = 0; e < kAppChunk; ++e) {
                if (dc + e < q) {
                    const T *Rp = R + (size_t)(dc + e) * Mn * sp + col;
                    double t = 0.0;
                    for (int k = 0; k < Mn; ++k) t += (double)Rp[(size_t)k * sp] * ab[k];
                    acc[e] += t;
                }
            }
        }
#pragma unroll
        for (int e = 0; e < kAppChunk; ++e) {
            const double v = wave_sum(acc[e]);
            if (tid == 0 && dc + e < q) U[dc + e] = v;
        }
    }
    __syncthreads();
    const double u = (tid < q) ? U[tid] : 0.0;
    double p = 0.0;
    if (tid < q) p = f.uniform ? 1.0 / q : (double)((const T *)f.prior)[(size_t)i * q + tid];
    const double S = p * u;
    const double Z = wave_sum(S);
    if (tid < q) {
        if (f.app) ((T *)f.app)[(size_t)i * q + tid] = (T)(S / Z);
        if (f.dprior) ((T *)f.dprior)[(size_t)i * q + tid] = (T)(u / Z);
    }
    if (f.Zinv && tid == 0) {
        f.Zinv[i] = 1.0 / Z;
        f.Zexp[i] = emax;
    }
}

// ---------------------------------------------------------------------------
// launcher

hipError_t launch_app(int fp64, const FrameDesc *fd, const Work *tab, int nblocks,
                      size_t lds_bytes, hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    if (fp64)
        hipLaunchKernelGGL(k_app<double>, dim3(nblocks), dim3(kAppThreads), lds_bytes, st, fd,
                           tab);
    else
        hipLaunchKernelGGL(k_app<float>, dim3(nblocks), dim3(kAppThreads), lds_bytes, st, fd,
                           tab);
    return hipGetLastError();
}


// One object per precision built from k_app_tile.hip.
hipError_t app_tile_f32(int td, int mn, int nwaves, const FrameDesc *fd, const Work *tab,
                        int nblocks, size_t lds, hipStream_t st);
hipError_t app_tile_f64(int td, int mn, int nwaves, const FrameDesc *fd, const Work *tab,
                        int nblocks, size_t lds, hipStream_t st);

hipError_t launch_app_tile(int fp64, int td, int mn, int nwaves, const FrameDesc *fd,
                           const Work *tab, int nblocks, size_t lds_bytes, hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    return fp64 ? app_tile_f64(td, mn, nwaves, fd, tab, nblocks, lds_bytes, st)
                : app_tile_f32(td, mn, nwaves, fd, tab, nblocks, lds_bytes, st);
}

}  // namespace mapdec
