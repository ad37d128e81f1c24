// Tiled APP kernel (eqs. 1-3).  Compiled once per precision: build with
// -DAPP_T=float|double -DAPP_FN=<launcher name>.
//
// One workgroup per (frame, TI = 8 consecutive symbols i); wave w owns the
// symbol values D in [w TD, w TD + TD).  The 64 lanes of a wave walk
// consecutive start indices s of the block's window, so every R load is a
// coalesced row segment, and each loaded R(s, D, delta) feeds the TI
// symbols whose drift band covers s:
//   U_i(D) += alpha_i(s - n i) beta_{i+1}(s - n i + delta) R(s, D, delta).
// FP64 alpha and beta rows are staged in LDS with zero padding wide enough that
// no lane branches on the band edges (states outside the band, and start
// indices outside [0, rho], have zero metrics).  The R values of the next
// 64 start indices are loaded while the current ones are used.  The TI x TD
// accumulators are summed across lanes by a butterfly reduce-scatter, then
//   S_i(D) = prior_i(D) U_i(D),  Z_i = sum_D S_i(D),  APP = S / Z,
//   d log P / d prior_i(D) = U_i(D) / Z_i.
#include "device_common.h"

#if !defined(APP_T) || !defined(APP_FN)
#error "compile with -DAPP_T and -DAPP_FN"
#endif

namespace mapdec {

template <typename T, int CNT, int H>
struct ReduceScatter {
    // After run(), v[0] of lane l holds the sum over the wave of the value
    // each lane had at index l >> (6 - log2 CNT0), CNT0 the initial count.
    static __device__ __forceinline__ void run(T *v, int lane) {
        if constexpr (H >= 1) {
            if constexpr (CNT > 1) {
                const bool upper = (lane & H) != 0;
#pragma unroll
                for (int k = 0; k < CNT / 2; ++k) {
                    const T send = upper ? v[k] : v[k + CNT / 2];
                    const T keep = upper ? v[k + CNT / 2] : v[k];
                    v[k] = keep + __shfl_xor(send, H, 64);
                }
                ReduceScatter<T, CNT / 2, H / 2>::run(v, lane);
            } else {
                v[0] += __shfl_xor(v[0], H, 64);
                ReduceScatter<T, 1, H / 2>::run(v, lane);
            }
        }
    }
};

template <int V>
constexpr int log2_of() { return V <= 1 ? 0 : 1 + log2_of<V / 2>(); }

template <typename T, int TD, int MN>
__global__ __launch_bounds__(512) void k_app_tile(const FrameDesc *__restrict__ fd,
                                                   const Work *__restrict__ tab) {
    constexpr int TI = kAppTI;
    constexpr int V = TI * TD;
    constexpr int Mn = 2 * MN + 1;
    const Work w = tab[blockIdx.x];
    const FrameDesc &f = fd[w.frame];
    if (*f.status != kStatusOk) return;
    extern __shared__ __align__(16) unsigned char smem[];
    const int Mt = f.Mt, M = f.M, q = f.q, n = f.n, rho = f.rho, N = f.N;
    const int i0 = w.item * TI;
    const int PAD = app_tile_pad(n);
    const int WA = Mt + 2 * PAD, WB = Mt + 2 * (PAD + MN);
    double *ar = (double *)smem;   // [TI][WA]  sc_i alpha_i(m) at m + M + PAD
    double *br = ar + TI * WA;     // [TI][WB]  beta_{i+1}(m) at m + M + PAD + mn
    double *Zsh = br + TI * WB;    // [TI]
    unsigned long long *smax = (unsigned long long *)(Zsh + TI);   // [TI]
    T *Ush = (T *)(smax + TI);     // [TI][q]
    const int tid = threadIdx.x, nth = blockDim.x, lane = tid & 63, wv = tid >> 6;
    const gptr<const double> A = to_global((const double *)f.alpha);
    const gptr<const double> B = to_global((const double *)f.beta);
    if (tid < TI) smax[tid] = 0ull;
    for (int j = tid; j < TI * WA; j += nth) {
        const int ii = j / WA, m = j - ii * WA - PAD, i = i0 + ii;
        ar[j] = (i < N && m >= 0 && m < Mt) ? A[(size_t)i * Mt + m] : 0.0;
    }
    for (int j = tid; j < TI * WB; j += nth) {
        const int ii = j / WB, m = j - ii * WB - PAD - MN, i = i0 + ii;
        br[j] = (i < N && m >= 0 && m < Mt) ? B[(size_t)(i + 1) * Mt + m] : 0.0;
    }
    __syncthreads();
    // Two-slice scale: the rows' product alpha_i(m') beta_{i+1}(m'+delta)
    // spans far less than either row, so dividing it by its maximum brings
    // it into the FP32 range; the scale is folded into the staged alpha row.
    // (Max of non-negative doubles through their bit patterns.)
    for (int j = tid; j < TI * Mt; j += nth) {
        const int ii = j / Mt, m = j - ii * Mt;
        double bm = 0.0;
#pragma unroll
        for (int k = 0; k < Mn; ++k) bm = fmax(bm, br[ii * WB + PAD + m + k]);
        const double v = ar[ii * WA + PAD + m] * bm;
        if (v > 0.0) atomicMax(&smax[ii], (unsigned long long)__double_as_longlong(v));
    }
    __syncthreads();
    for (int j = tid; j < TI * WA; j += nth) {
        const int ii = j / WA;
        const double mx = __longlong_as_double((long long)smax[ii]);
        ar[j] = mx > 0.0 ? ar[j] / mx : 0.0;
    }

    const gptr<const T> R = to_global((const T *)f.R);
    const size_t sp = (size_t)f.sp;
    const int s_lo = n * i0 - M;
    const int span = n * (TI - 1) + Mt;   // s in [s_lo, s_lo + span)
    const int iters = (span + 63) / 64;
    const int nwaves = nth >> 6;
    __syncthreads();
    // wave wv handles the symbol-value tiles wv, wv + nwaves, ...
    for (int d0 = wv * TD; d0 < q; d0 += nwaves * TD) {
        size_t rrow[TD];
#pragma unroll
        for (int d = 0; d < TD; ++d) rrow[d] = (size_t)min(d0 + d, q - 1) * Mn * sp;
        auto load_r = [&](T (&r)[Mn][TD], int c) {
            const int sc = min(max(s_lo + c, 0), rho);
#pragma unroll
            for (int k = 0; k < Mn; ++k)
#pragma unroll
                for (int d = 0; d < TD; ++d) r[k][d] = R[rrow[d] + (size_t)k * sp + sc];
        };
        T rc[Mn][TD], rn[Mn][TD];
        load_r(rc, lane);
        T acc[V];
#pragma unroll
        for (int v = 0; v < V; ++v) acc[v] = T(0);
        for (int it = 0; it < iters; ++it) {
            const int c = lane + 64 * it;
            if (it + 1 < iters) load_r(rn, c + 64);
            const int cc = min(c, span - 1);
            const T live = c < span ? T(1) : T(0);
            double a[TI];
#pragma unroll
            for (int ii = 0; ii < TI; ++ii)
                a[ii] = (double)live * ar[ii * WA + PAD + cc - n * ii];
            const double *bb = br + PAD + cc;
#pragma unroll
            for (int k = 0; k < Mn; ++k) {
#pragma unroll
                for (int ii = 0; ii < TI; ++ii) {
                    const T kv = (T)(a[ii] * bb[ii * (WB - n) + k]);
#pragma unroll
                    for (int d = 0; d < TD; ++d) acc[ii * TD + d] += kv * rc[k][d];
                }
            }
#pragma unroll
            for (int k = 0; k < Mn; ++k)
#pragma unroll
                for (int d = 0; d < TD; ++d) rc[k][d] = rn[k][d];
        }
        ReduceScatter<T, V, 32>::run(acc, lane);
        constexpr int SH = 6 - log2_of<V>();
        const int idx = lane >> SH, ii = idx / TD, d = idx - ii * TD;
        if ((lane & ((1 << SH) - 1)) == 0 && d0 + d < q) Ush[ii * q + d0 + d] = acc[0];
    }
    __syncthreads();
    const T up = T(1) / T(q);
    if (tid < TI && i0 + tid < N) {
        double Z = 0.0;
        const T *pr = f.uniform ? nullptr : (const T *)f.prior + (size_t)(i0 + tid) * q;
        for (int D = 0; D < q; ++D) Z += (double)((pr ? pr[D] : up) * Ush[tid * q + D]);
        Zsh[tid] = Z;
        // 1/Z_i in the units of the unscaled FP64 rows
        const double mx = __longlong_as_double((long long)smax[tid]);
        if (f.Zinv) f.Zinv[i0 + tid] = Z > 0.0 ? 1.0 / (Z * mx) : 0.0;
    }
    __syncthreads();
    for (int j = tid; j < TI * q; j += nth) {
        const int ii = j / q, D = j - ii * q, i = i0 + ii;
        if (i >= N) continue;
        const T u = Ush[j];
        const T p = f.uniform ? up : ((const T *)f.prior)[(size_t)i * q + D];
        const T Zi = (T)Zsh[ii];
        if (f.app) ((T *)f.app)[(size_t)i * q + D] = p * u / Zi;
        if (f.dprior) ((T *)f.dprior)[(size_t)i * q + D] = u / Zi;
    }
}

template <int TD, int MN>
static hipError_t tile_launch(int nwaves, const FrameDesc *fd, const Work *tab, int nblocks,
                              size_t lds, hipStream_t st) {
    auto kern = k_app_tile<APP_T, TD, MN>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)kern,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(64 * nwaves), lds, st, fd, tab);
    return hipGetLastError();
}

template <int TD>
static hipError_t tile_td(int mn, int nwaves, const FrameDesc *fd, const Work *tab, int nblocks,
                          size_t lds, hipStream_t st) {
    switch (mn) {
        case 0: return tile_launch<TD, 0>(nwaves, fd, tab, nblocks, lds, st);
        case 1: return tile_launch<TD, 1>(nwaves, fd, tab, nblocks, lds, st);
        case 2: return tile_launch<TD, 2>(nwaves, fd, tab, nblocks, lds, st);
        case 3: return tile_launch<TD, 3>(nwaves, fd, tab, nblocks, lds, st);
        case 4: return tile_launch<TD, 4>(nwaves, fd, tab, nblocks, lds, st);
        case 5: return tile_launch<TD, 5>(nwaves, fd, tab, nblocks, lds, st);
        case 6: return tile_launch<TD, 6>(nwaves, fd, tab, nblocks, lds, st);
        case 7: return tile_launch<TD, 7>(nwaves, fd, tab, nblocks, lds, st);
        case 8: return tile_launch<TD, 8>(nwaves, fd, tab, nblocks, lds, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t APP_FN(int td, int mn, int nwaves, const FrameDesc *fd, const Work *tab, int nblocks,
                  size_t lds, hipStream_t st) {
    switch (td) {
        case 2: return tile_td<2>(mn, nwaves, fd, tab, nblocks, lds, st);
        case 4: return tile_td<4>(mn, nwaves, fd, tab, nblocks, lds, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace mapdec
