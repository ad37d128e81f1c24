// APP kernel (eqs. 1-3).
#include "device_common.h"

namespace mapdec {

// ---------------------------------------------------------------------------
// APP (eqs. 1-3).  One wave per (frame, i); lanes stride over m'.
//   U_i(D) = sum_{m', delta} alpha_i(m') R(n i + m', D, delta) beta_{i+1}(m' + delta)
//   S_i(D) = prior_i(D) U_i(D),  Z_i = sum_D S_i(D),  APP = S / Z,
//   d log P / d prior_i(D) = U_i(D) / Z_i.

constexpr int kAppChunk = 16;

template <typename T>
__global__ __launch_bounds__(kAppThreads) void k_app(const FrameDesc *__restrict__ fd,
                                                     const Work *__restrict__ tab) {
    const Work w = tab[blockIdx.x];
    const FrameDesc &f = fd[w.frame];
    const int i = w.item;
    if (*f.status != kStatusOk) return;
    extern __shared__ __align__(16) unsigned char smem[];
    const int Mt = f.Mt, mn = f.mn, M = f.M, Mn = f.Mn, q = f.q, n = f.n, rho = f.rho;
    T *al = (T *)smem;
    T *be = al + Mt;            // Mt + 2 mn, padded
    T *U = be + Mt + 2 * mn;    // q
    const int tid = threadIdx.x;
    const T *A = (const T *)f.alpha + (size_t)i * Mt;
    const T *B = (const T *)f.beta + (size_t)(i + 1) * Mt;
    for (int j = tid; j < Mt; j += kAppThreads) {
        al[j] = A[j];
        be[mn + j] = B[j];
    }
    for (int j = tid; j < mn; j += kAppThreads) {
        be[j] = T(0);
        be[mn + Mt + j] = T(0);
    }
    __syncthreads();

    const T *R = (const T *)f.R;
    const size_t sp = (size_t)f.sp;
    for (int dc = 0; dc < q; dc += kAppChunk) {
        T acc[kAppChunk];
#pragma unroll
        for (int e = 0; e < kAppChunk; ++e) acc[e] = T(0);
        for (int mi = tid; mi < Mt; mi += kAppThreads) {
            const int s = n * i + mi - M;
            if (s < 0 || s > rho) continue;
            const T av = al[mi];
            if (av == T(0)) continue;
#pragma unroll
            for (int e = 0; e < kAppChunk; ++e) {
                if (dc + e < q) {
                    const T *Rp = R + (size_t)(dc + e) * Mn * sp + s;
                    T t = T(0);
                    for (int k = 0; k < Mn; ++k) t += Rp[(size_t)k * sp] * be[mi + k];
                    acc[e] += av * t;
                }
            }
        }
#pragma unroll
        for (int e = 0; e < kAppChunk; ++e) {
            const T v = wave_sum(acc[e]);
            if (tid == 0 && dc + e < q) U[dc + e] = v;
        }
    }
    __syncthreads();
    const T u = (tid < q) ? U[tid] : T(0);
    T p = T(0);
    if (tid < q) p = f.uniform ? T(1) / T(q) : ((const T *)f.prior)[(size_t)i * q + tid];
    const T S = p * u;
    const T Z = wave_sum(S);
    if (tid < q) {
        if (f.app) ((T *)f.app)[(size_t)i * q + tid] = S / Z;
        if (f.dprior) ((T *)f.dprior)[(size_t)i * q + tid] = u / Z;
    }
    if (f.Zinv && tid == 0) f.Zinv[i] = 1.0 / (double)Z;
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
