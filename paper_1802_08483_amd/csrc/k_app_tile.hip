// Tiled APP kernel (eqs. 1-3).  Compiled once per precision: build with
// -DAPP_T=float|double -DAPP_FN=<launcher name>.
//
// One workgroup per (frame, TI = kAppTI consecutive symbols i).  With
// s_lo = n i0 - M the start indices the block needs are s = s_lo + c,
// c in [0, span), span = n (TI - 1) + 2M + 1, in chunks of 64, and the
// symbol values D in tiles of TD.  The nw waves of the workgroup form G
// tile groups of nw / G waves (G the largest divisor of nw that is at most
// the number of tiles): in round r the waves of group g take tile g + r G,
// each over its own share of the chunks, so a wave sums its accumulators
// across lanes once per round.  The 64 lanes of a wave walk consecutive s,
// so every R load is a coalesced row segment.  A lane accumulates, for the
// TD symbol values of its tile and every symbol of the block,
//   U_i(D) += K_i(s, k) R(s, D, k),
//   K_i(s, k) = alpha_i(s - n i) beta_{i+1}(s - n i + k - mn),
// streaming over k: per k the TI products K_i are formed once (FP64, then
// the batch precision) and each of the TD loaded R values feeds TI fused
// multiply-adds.  The FP64 alpha and beta rows are staged in LDS as
// (mantissa, exponent) pairs with zero padding wide enough that no lane
// branches on the band edges (states outside the band, and start indices
// outside [0, rho], have zero metrics).  R is read through a buffer
// descriptor with the D row offset in a scalar register and the lane's
// start index plus the k row offset in a vector one (one add per k), so the
// loads cost almost no vector instructions; every index is clamped into the
// table (the host keeps the table below 2^31 bytes).  The TI x TD accumulators are summed
// across lanes by a butterfly reduce-scatter and across the waves of a tile
// group through LDS, then
//   S_i(D) = prior_i(D) U_i(D),  Z_i = sum_D S_i(D),  APP = S / Z,
//   d log P / d prior_i(D) = U_i(D) / Z_i.
#include "device_common.h"

#if !defined(APP_T) || !defined(APP_FN)
#error "compile with -DAPP_T and -DAPP_FN"
#endif

namespace mapdec {

template <typename T, int CNT, int H>
struct ReduceScatter {
    // Butterfly over the wave.  With CNT0 = m 64 (m >= 1) initial values,
    // afterwards v[j] (j < m) of lane l holds the wave sum of index m l + j;
    // with CNT0 < 64, v[0] of lane l holds the sum of index
    // l >> (6 - log2 CNT0).
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

// A metric value as mantissa (in [1/2, 1), batch precision) and binary
// exponent.  The two normalised rows of a symbol can peak at opposite ends
// of the drift range, so that their product at the drifts carrying the
// posterior lies below even the FP64 range while each factor is well
// inside it; products are therefore formed from mantissas and exponent
// sums, scaled by the symbol's largest exponent sum.
template <typename T>
struct alignas(2 * sizeof(T) > 8 ? 16 : 8) ME {
    T m;
    int e;
};
constexpr int kZeroExp = -(1 << 20);   // exponent of a zero metric
template <typename T>
__device__ __forceinline__ ME<T> to_me(double v) {
    ME<T> r;
    if (v > 0.0) {
        int e;
        r.m = (T)frexp(v, &e);
        r.e = e;
    } else {
        r.m = T(0);
        r.e = kZeroExp;
    }
    return r;
}
__device__ __forceinline__ float scale2(float x, int e) { return ldexpf(x, e); }
__device__ __forceinline__ double scale2(double x, int e) { return ldexp(x, e); }

template <typename T>
__device__ __forceinline__ T rload(__amdgpu_buffer_rsrc_t rs, int voff, int soff) {
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, voff, soff, 0));
    } else {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 0));
    }
}

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
    const int Mt = f.Mt, M = f.M, q = f.q, n = f.n, s0 = f.s0, s1 = f.s1;
    const int N = f.i1;                  // symbols of the segment end here
    const int i0 = f.i0 + w.item * TI;   // first symbol of the block
    const int ib = f.i0;                 // row index base of alpha / beta
    const int PAD = app_tile_pad(n);
    const int WA = Mt + 2 * PAD, WB = Mt + 2 * (PAD + MN);
    const int tid = threadIdx.x, nth = blockDim.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform
    const int nwaves = nth >> 6;
    ME<T> *ar = (ME<T> *)smem;     // [TI][WA]  alpha_i(m) at m + M + PAD
    ME<T> *br = ar + TI * WA;      // [TI][WB]  beta_{i+1}(m) at m + M + PAD + mn
    double *Zsh = (double *)(br + TI * WB);   // [TI]
    T *Ush = (T *)(Zsh + TI);      // [TI][q]
    T *part = Ush + TI * q;        // [nwaves][V] per-wave sums
    int *emax = (int *)(part + nwaves * V);   // [TI]
    const gptr<const double> A = to_global((const double *)f.alpha);
    const gptr<const double> B = to_global((const double *)f.beta);
    if (tid < TI) emax[tid] = 2 * kZeroExp;
    // (ii, x) = divmod(j, W) of a flat loop j = tid, tid + nth, ..
    auto step = [&](int &ii, int &x, int W) {
        x += nth;
        while (x >= W) {
            x -= W;
            ++ii;
        }
    };
    {
        int ii = tid / WA, x = tid - ii * WA;
        for (int j = tid; j < TI * WA; j += nth, step(ii, x, WA)) {
            const int m = x - PAD, i = i0 + ii;
            ar[j] = to_me<T>((i < N && m >= 0 && m < Mt) ? A[(size_t)(i - ib) * Mt + m] : 0.0);
        }
    }
    {
        int ii = tid / WB, x = tid - ii * WB;
        for (int j = tid; j < TI * WB; j += nth, step(ii, x, WB)) {
            const int m = x - PAD - MN, i = i0 + ii;
            br[j] = to_me<T>((i < N && m >= 0 && m < Mt) ? B[(size_t)(i + 1 - ib) * Mt + m] : 0.0);
        }
    }
    __syncthreads();
    // Two-slice scale: the product alpha_i(m') beta_{i+1}(m'+delta) spans
    // far less than either row; E_i = max over m', delta of the exponent
    // sum, and every product is taken as 2^-E_i times its true value.
    {
        int ii = tid / Mt, m = tid - ii * Mt;
        for (int j = tid; j < TI * Mt; j += nth, step(ii, m, Mt)) {
            const ME<T> a = ar[ii * WA + PAD + m];
            if (a.m == T(0)) continue;
            int eb = 2 * kZeroExp;
#pragma unroll
            for (int k = 0; k < Mn; ++k) {
                const ME<T> b = br[ii * WB + PAD + m + k];
                if (b.m != T(0)) eb = max(eb, b.e);
            }
            if (eb > 2 * kZeroExp) atomicMax(&emax[ii], a.e + eb);
        }
    }
    __syncthreads();

    // R(s, D, k) lives at ((D Mn + k) sp + s - s0) in the frame's table
    const int sp = f.sp;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        f.R, (short)0, (int)((size_t)q * Mn * sp * sizeof(T)), 0x00020000);
    const int s_lo = n * i0 - M;
    const int span = n * (TI - 1) + Mt;   // s in [s_lo, s_lo + span)
    const int nchunks = (span + 63) / 64;
    const int ntiles = (q + TD - 1) / TD;
    int G = min(ntiles, nwaves);
    while (nwaves % G != 0) --G;
    const int CG = nwaves / G, tg = wv % G, cg = wv / G;
    // chunks of this wave (at least one step, so that every wave reaches
    // the same barriers; a chunk past the span is dead)
    const int nmy = max(1, (nchunks - cg + CG - 1) / CG);
    const int nrounds = (ntiles + G - 1) / G;
    const int total = nrounds * nmy;
    // One flat sequence of (round, chunk) steps per wave, k unrolled
    // inside; the R loads run PF steps ahead, across chunk and round
    // boundaries.
    constexpr int PF = 2;
    T r[PF + 1][TD];
    auto voff_at = [&](int jc) {
        const int ch = cg + jc * CG;
        return (min(max(s_lo + 64 * ch + lane, s0), s1) - s0) * (int)sizeof(T);
    };
    const int spb = sp * (int)sizeof(T);   // bytes per (D, k) row of R
    // byte offsets of the rows (D, 0) of a tile starting at d0
    auto rows_of = [&](int(&ro)[TD], int d0) {
#pragma unroll
        for (int d = 0; d < TD; ++d) ro[d] = min(d0 + d, q - 1) * Mn * spb;
    };
    auto load_k = [&](T(&dst)[TD], int vo, const int(&ro)[TD], int k) {
#pragma unroll
        for (int d = 0; d < TD; ++d) dst[d] = rload<T>(rs, vo + k * spb, ro[d]);
    };
    int jr = 0, jc = 0;   // round and chunk index of step j
    {
        int ro[TD];
        rows_of(ro, tg * TD);
#pragma unroll
        for (int e = 0; e < PF; ++e) load_k(r[e], voff_at(0), ro, e);
    }
    T acc[V];
#pragma unroll
    for (int v = 0; v < V; ++v) acc[v] = T(0);
    for (int j = 0; j < total; ++j) {
        const int c = 64 * (cg + jc * CG) + lane;
        const int cc = min(c, span - 1);
        const bool live = c < span;
        T am[TI];
        int ae[TI];
#pragma unroll
        for (int ii = 0; ii < TI; ++ii) {
            const ME<T> x = ar[ii * WA + PAD + cc - n * ii];
            am[ii] = live ? x.m : T(0);
            ae[ii] = x.e - emax[ii];
        }
        const ME<T> *bb = br + PAD + cc;
        // a chunk where no symbol of the block has a forward metric (states
        // the path thresholds dropped, or none reachable) adds nothing: the
        // wave skips its products (the R loads still run, they feed the
        // prefetch of the next step)
        bool anz = false;
#pragma unroll
        for (int ii = 0; ii < TI; ++ii) anz |= am[ii] != T(0);
        const bool act = __ballot(anz) != 0;
        // the next step (a repeated load past the end is harmless)
        const bool last_chunk = jc + 1 == nmy;
        const int jcn = last_chunk ? 0 : jc + 1;
        const int jrn = last_chunk ? min(jr + 1, nrounds - 1) : jr;
        const int vo = voff_at(jc), von = voff_at(jcn);
        int ro[TD], ron[TD];
        rows_of(ro, (tg + jr * G) * TD);
        rows_of(ron, (tg + jrn * G) * TD);
#pragma unroll
        for (int k = 0; k < Mn; ++k) {
            // issue the loads of step (j, k + PF), or of the next step's first k
            if (k + PF < Mn)
                load_k(r[(k + PF) % (PF + 1)], vo, ro, k + PF);
            else
                load_k(r[(k + PF) % (PF + 1)], von, ron, k + PF - Mn);
            if (act) {
                T kv[TI];
#pragma unroll
                for (int ii = 0; ii < TI; ++ii) {
                    const ME<T> b = bb[ii * (WB - n) + k];
                    kv[ii] = scale2(am[ii] * b.m, ae[ii] + b.e);
                }
#pragma unroll
                for (int ii = 0; ii < TI; ++ii)
#pragma unroll
                    for (int d = 0; d < TD; ++d)
                        acc[ii * TD + d] += kv[ii] * r[k % (PF + 1)][d];
            }
        }
        // the ring position of step (j + 1, 0) must be slot 0
        if constexpr (Mn % (PF + 1) != 0) {
            T tmp[PF + 1][TD];
#pragma unroll
            for (int e = 0; e <= PF; ++e)
#pragma unroll
                for (int d = 0; d < TD; ++d) tmp[e][d] = r[(e + Mn) % (PF + 1)][d];
#pragma unroll
            for (int e = 0; e <= PF; ++e)
#pragma unroll
                for (int d = 0; d < TD; ++d) r[e][d] = tmp[e][d];
        }
        if (last_chunk) {
            // round jr complete: sum over lanes, then over the waves of
            // each tile group
            ReduceScatter<T, V, 32>::run(acc, lane);
            if constexpr (V >= 64) {
                constexpr int m = V / 64;
#pragma unroll
                for (int x = 0; x < m; ++x) part[wv * V + m * lane + x] = acc[x];
            } else {
                constexpr int SH = 6 - log2_of<V>();
                if ((lane & ((1 << SH) - 1)) == 0) part[wv * V + (lane >> SH)] = acc[0];
            }
            __syncthreads();
            for (int x = tid; x < G * V; x += nth) {
                const int g = x / V, xv = x - g * V;
                const int ii = xv / TD, D = (g + jr * G) * TD + (xv - ii * TD);
                if (D >= q) continue;
                T u = T(0);
                for (int y = 0; y < CG; ++y) u += part[(y * G + g) * V + xv];
                Ush[ii * q + D] = u;
            }
            __syncthreads();
#pragma unroll
            for (int v = 0; v < V; ++v) acc[v] = T(0);
        }
        jc = jcn;
        jr = last_chunk ? jr + 1 : jr;
    }
    const T up = T(1) / T(q);
    if (tid < TI && i0 + tid < N) {
        double Z = 0.0;
        const T *pr = f.uniform ? nullptr : (const T *)f.prior + (size_t)(i0 + tid) * q;
        for (int D = 0; D < q; ++D) Z += (double)((pr ? pr[D] : up) * Ush[tid * q + D]);
        Zsh[tid] = Z;
        // the rows' Z_i is 2^E_i Z: keep 1/Z and E_i
        if (f.Zinv) {
            f.Zinv[i0 + tid] = Z > 0.0 ? 1.0 / Z : 0.0;
            f.Zexp[i0 + tid] = emax[tid];
        }
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
    if (nwaves < 1 || nwaves > kAppMaxWaves) return hipErrorInvalidValue;
    switch (td) {
        case 2: return tile_td<2>(mn, nwaves, fd, tab, nblocks, lds, st);
        case 4: return tile_td<4>(mn, nwaves, fd, tab, nblocks, lds, st);
        case 8:
            if constexpr (sizeof(APP_T) == 4) return tile_td<8>(mn, nwaves, fd, tab, nblocks, lds, st);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

}  // namespace mapdec
