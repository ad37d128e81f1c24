// gfx950 kernels of the MAP forward-backward decoder (Sec. II-C).
//
// Data flow per frame (one workspace region per frame, see FrameDesc):
//   k_pack     received bytes -> 32-bit words of bits
//   k_lattice  receiver metric R(s, D, delta) of eqs. 7-10 for every start
//              index s and symbol D (one lattice per (s, D) serves every
//              (i, m') with n i + m' = s, since the codebook is fixed), plus
//              Gamma(s, delta) = sum_D R / q when the priors are uniform
//   k_gamma    Gamma_i(m', delta) = sum_D prior_i(D) R(n i + m', D, delta)
//              for general priors (eq. 6 summed over D)
//   k_chain    normalised alpha (eqs. 4, 11, 12) and beta (eq. 5) chains,
//              one workgroup per frame and direction, log-normalisers in FP64
//   k_app      APP of eqs. 1-3: S_i(D) = prior_i(D) sum_{m', delta}
//              alpha_i(m') R(n i + m', D, delta) beta_{i+1}(m' + delta),
//              each row divided by its own sum
#include <math.h>

#include "kernels.h"

namespace mapdec {

// ---------------------------------------------------------------------------
// small helpers

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum of one double per thread over the workgroup; every thread gets the
// same value (same summation order everywhere).  red: one double per wave.
__device__ __forceinline__ double block_sum(double v, double *red) {
    v = wave_sum(v);
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double tot = 0.0;
    const int nw = blockDim.x >> 6;
    for (int w = 0; w < nw; ++w) tot += red[w];
    __syncthreads();
    return tot;
}

// ---------------------------------------------------------------------------
// per-call initialisation of the per-frame results

__global__ void k_init(const FrameDesc *__restrict__ fd, int nframes) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nframes) return;
    *fd[f].status = kStatusOk;
    *fd[f].logp = 0.0;
}

// ---------------------------------------------------------------------------
// received bytes -> packed bits: one wave packs 64 consecutive bits with a
// ballot; a 256-thread workgroup writes kPackWords words.

__global__ __launch_bounds__(256) void k_pack(const FrameDesc *__restrict__ fd,
                                              const Work *__restrict__ tab) {
    const Work w = tab[blockIdx.x];
    const FrameDesc &f = fd[w.frame];
    const int word0 = w.item;
    const int p = word0 * 32 + (int)threadIdx.x;
    const bool bit = (p < f.rho) && (f.y[p] != 0);
    const unsigned long long m = __ballot(bit);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int wd = word0 + 2 * wv;
    if (lane == 0 && wd < f.nwords) f.ybits[wd] = (uint32_t)m;
    if (lane == 1 && wd + 1 < f.nwords) f.ybits[wd + 1] = (uint32_t)(m >> 32);
}

// ---------------------------------------------------------------------------
// Receiver-metric lattice (eqs. 7-10), corridor form.
//
// A lane owns one start index s and walks all q codewords; the wave's lanes
// hold 64 consecutive s, so the codeword (and each of its bits) is uniform
// across the wave.  Row r of the lattice is kept in registers in corridor
// coordinates k = j - r + MN (j = received bits consumed), k in [0, 2 MN]:
//   G_r[k] = d F_{r-1}[k+1] + Q(y[s + r + k - MN - 1] | x_r) F_{r-1}[k]
//   F_r[k] = G_r[k] + sum_{t=1..min(IM,k)} a_t G_r[k-t]     (r < n)
//   F_n[k] = G_n[k]                                          (last row)
// with a_t = a^t for t <= I and 0 beyond (at most I insertions in a row).
// The two possible values of Q for each received position are prepared once
// per lane (qx0 for a 0 codeword bit, qx1 for a 1), so a node costs one
// multiply and 1 + IM fused multiply-adds.

template <typename T, int MN, int NB>
__device__ __forceinline__ void lattice_row_in(T (&G)[2 * MN + 1], const T (&F)[2 * MN + 1],
                                               const T (&qx)[NB], T d, int r) {
#pragma unroll
    for (int k = 0; k < 2 * MN + 1; ++k) {
        T v = (k + 1 < 2 * MN + 1) ? d * F[k + 1] : T(0);
        const int b = r + k - MN - 1;
        if (b >= 0) v += qx[b] * F[k];
        G[k] = v;
    }
}

template <typename T, int MN, int IM>
__global__ __launch_bounds__(kLatticeLanes) void k_lattice(const FrameDesc *__restrict__ fd,
                                                           const Work *__restrict__ tab) {
    constexpr int KW = 2 * MN + 1;
    constexpr int NB = kMaxN + MN;   // received positions a lattice can read
    const Work w = tab[blockIdx.x];
    const FrameDesc &f = fd[w.frame];
    const int s = w.item + (int)threadIdx.x;
    if (s > f.rho) return;
    const int n = f.n, q = f.q, rho = f.rho;
    const T d = (T)f.d, t1 = (T)f.t1, t0 = (T)f.t0;

    T apow[IM + 1];
    {
        T p = T(1);
        apow[0] = T(1);
#pragma unroll
        for (int t = 1; t <= IM; ++t) {
            p *= (T)f.a;
            apow[t] = (t <= f.I) ? p : T(0);
        }
    }

    // received bits y[s .. s+32) of this lane
    const int wi = s >> 5, sh = s & 31;
    const uint32_t lo = f.ybits[wi], hi = f.ybits[wi + 1];
    const uint32_t win = sh ? ((lo >> sh) | (hi << (32 - sh))) : lo;
    T qx0[NB], qx1[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const bool one = (win >> b) & 1u;
        qx0[b] = one ? t0 : t1;
        qx1[b] = one ? t1 : t0;
    }

    T gsum[KW];
#pragma unroll
    for (int k = 0; k < KW; ++k) gsum[k] = T(0);

    T *R = (T *)f.R;
    const size_t sp = (size_t)f.sp;
    for (int D = 0; D < q; ++D) {
        const uint32_t cw = f.cw[D];
        T F[KW];
#pragma unroll
        for (int k = 0; k < KW; ++k) {
            const int dl = k - MN;   // row 0: dl insertions before the first bit
            F[k] = (dl >= 0 && dl <= IM) ? apow[dl] : T(0);
        }
#pragma unroll
        for (int r = 1; r <= kMaxN; ++r) {
            if (r > n) break;
            T G[KW];
            if ((cw >> (n - r)) & 1u)
                lattice_row_in<T, MN, NB>(G, F, qx1, d, r);
            else
                lattice_row_in<T, MN, NB>(G, F, qx0, d, r);
            if (r < n) {
#pragma unroll
                for (int k = 0; k < KW; ++k) {
                    T v = G[k];
#pragma unroll
                    for (int t = 1; t <= IM; ++t)
                        if (t <= k) v += apow[t] * G[k - t];
                    F[k] = v;
                }
            } else {
#pragma unroll
                for (int k = 0; k < KW; ++k) F[k] = G[k];
            }
        }
#pragma unroll
        for (int k = 0; k < KW; ++k) {
            const int len = n + k - MN;   // segment length n + delta
            const T v = (len >= 0 && s + len <= rho) ? F[k] : T(0);
            R[((size_t)D * KW + k) * sp + s] = v;
            gsum[k] += v;
        }
    }
    if (f.uniform) {
        T *G = (T *)f.G;
        const T invq = T(1) / T(q);
#pragma unroll
        for (int k = 0; k < KW; ++k) G[(size_t)k * sp + s] = gsum[k] * invq;
    }
}

// ---------------------------------------------------------------------------
// Gamma_i(m', delta) = sum_D prior_i(D) R(n i + m', D, delta) for general
// priors; one lane per drift state m', lanes read consecutive s.

template <typename T>
__global__ __launch_bounds__(kGammaLanes) void k_gamma(const FrameDesc *__restrict__ fd,
                                                       const Work *__restrict__ tab) {
    const Work w = tab[blockIdx.x];
    const FrameDesc &f = fd[w.frame];
    const int per_i = (f.Mt + kGammaLanes - 1) / kGammaLanes;
    const int i = w.item / per_i;
    const int mi = (w.item % per_i) * kGammaLanes + (int)threadIdx.x;
    if (mi >= f.Mt) return;
    const int Mn = f.Mn, Mt = f.Mt, q = f.q;
    const int s = f.n * i + mi - f.M;
    T *G = (T *)f.G + (size_t)i * Mn * Mt + mi;
    if (s < 0 || s > f.rho) {
        for (int k = 0; k < Mn; ++k) G[(size_t)k * Mt] = T(0);
        return;
    }
    const T *pr = (const T *)f.prior + (size_t)i * q;
    const T *R = (const T *)f.R + s;
    const size_t sp = (size_t)f.sp;
    for (int k = 0; k < Mn; ++k) {
        T acc = T(0);
        for (int D = 0; D < q; ++D) acc += pr[D] * R[((size_t)D * Mn + k) * sp];
        G[(size_t)k * Mt] = acc;
    }
}

// ---------------------------------------------------------------------------
// alpha / beta chains.  Workgroup 2c runs the forward chain of frame
// frames[c], workgroup 2c+1 the backward chain.  Rows live in LDS with mn
// zero entries of padding on each side (states outside [-M, M] are 0).

template <typename T>
__device__ __forceinline__ T gamma_at(const FrameDesc &f, const T *G, int i, int mp, int k) {
    if (mp < -f.M || mp > f.M) return T(0);
    if (f.uniform) {
        const int s = f.n * i + mp;
        return (s >= 0 && s <= f.rho) ? G[(size_t)k * f.sp + s] : T(0);
    }
    return G[((size_t)i * f.Mn + k) * f.Mt + (mp + f.M)];
}

template <typename T>
__global__ __launch_bounds__(kChainThreads) void k_chain(const FrameDesc *__restrict__ fd,
                                                         const int *__restrict__ frames) {
    const int fi = frames[blockIdx.x >> 1];
    const int dir = blockIdx.x & 1;
    const FrameDesc &f = fd[fi];
    extern __shared__ __align__(16) unsigned char smem[];
    const int Mt = f.Mt, mn = f.mn, M = f.M, N = f.N, Mn = f.Mn;
    const int W = Mt + 2 * mn;
    T *buf0 = (T *)smem;
    T *buf1 = buf0 + W;
    double *red = (double *)(smem + (((size_t)2 * W * sizeof(T) + 15) & ~(size_t)15));
    const int tid = threadIdx.x, nth = blockDim.x;

    for (int j = tid; j < 2 * W; j += nth) buf0[j] = T(0);
    __syncthreads();
    const int m0 = dir == 0 ? 0 : f.rho - f.tau;
    T *out = (T *)(dir == 0 ? f.alpha : f.beta);
    double *logX = dir == 0 ? f.logA : f.logB;
    const int row0 = dir == 0 ? 0 : N;
    if (tid == 0) {
        buf0[mn + m0 + M] = T(1);
        logX[row0] = 0.0;
    }
    for (int mi = tid; mi < Mt; mi += nth)
        out[(size_t)row0 * Mt + mi] = (mi == m0 + M) ? T(1) : T(0);
    __syncthreads();

    const T *G = (const T *)f.G;
    double lsum = 0.0;
    T *cur = buf0, *nxt = buf1;
    bool dead = false;
    for (int step = 0; step < N; ++step) {
        const int i = dir == 0 ? step : N - 1 - step;
        double part = 0.0;
        for (int mi = tid; mi < Mt; mi += nth) {
            const int m = mi - M;
            T acc = T(0);
            if (dir == 0) {
                // alpha'_{i+1}(m) = sum_delta alpha_i(m - delta) Gamma_i(m - delta, delta)
                for (int k = 0; k < Mn; ++k) {
                    const int dl = k - mn;
                    acc += cur[mn + mi - dl] * gamma_at(f, G, i, m - dl, k);
                }
            } else {
                // beta'_i(m) = sum_delta Gamma_i(m, delta) beta_{i+1}(m + delta)
                for (int k = 0; k < Mn; ++k) {
                    const int dl = k - mn;
                    acc += gamma_at(f, G, i, m, k) * cur[mn + mi + dl];
                }
            }
            nxt[mn + mi] = acc;
            part += (double)acc;
        }
        const double c = block_sum(part, red);
        if (!(c > 0.0) || !isfinite(c)) {
            dead = true;
            break;
        }
        const T inv = (T)(1.0 / c);
        const int row = dir == 0 ? i + 1 : i;
        for (int mi = tid; mi < Mt; mi += nth) {
            const T v = nxt[mn + mi] * inv;
            nxt[mn + mi] = v;
            out[(size_t)row * Mt + mi] = v;
        }
        lsum += log(c);
        if (tid == 0) logX[row] = lsum;
        T *t = cur;
        cur = nxt;
        nxt = t;
        __syncthreads();
    }
    if (tid != 0) return;
    if (dead) {
        atomicOr(f.status, kStatusNoPath);
        if (dir == 0) *f.logp = -INFINITY;
        return;
    }
    if (dir == 0) {
        // P(y) = alpha_N(rho - tau) in unnormalised terms
        const T aN = cur[mn + (f.rho - f.tau) + M];
        if (!(aN > T(0))) {
            atomicOr(f.status, kStatusNoPath);
            *f.logp = -INFINITY;
        } else {
            *f.logp = lsum + log((double)aN);
        }
    }
}

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
// launchers

hipError_t launch_init(const FrameDesc *fd, int nframes, hipStream_t st) {
    hipLaunchKernelGGL(k_init, dim3((nframes + 255) / 256), dim3(256), 0, st, fd, nframes);
    return hipGetLastError();
}

hipError_t launch_pack(const FrameDesc *fd, const Work *tab, int nblocks, hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack, dim3(nblocks), dim3(256), 0, st, fd, tab);
    return hipGetLastError();
}

template <typename T, int MN>
static void lattice_mn(int imode, const FrameDesc *fd, const Work *tab, int nblocks,
                       hipStream_t st) {
    constexpr int IM2 = (2 < 2 * MN) ? 2 : 2 * MN;
    if (imode == 0)
        hipLaunchKernelGGL((k_lattice<T, MN, IM2>), dim3(nblocks), dim3(kLatticeLanes), 0, st,
                           fd, tab);
    else
        hipLaunchKernelGGL((k_lattice<T, MN, 2 * MN>), dim3(nblocks), dim3(kLatticeLanes), 0,
                           st, fd, tab);
}

template <typename T>
static hipError_t lattice_t(int mn, int imode, const FrameDesc *fd, const Work *tab,
                            int nblocks, hipStream_t st) {
    switch (mn) {
        case 0: lattice_mn<T, 0>(imode, fd, tab, nblocks, st); break;
        case 1: lattice_mn<T, 1>(imode, fd, tab, nblocks, st); break;
        case 2: lattice_mn<T, 2>(imode, fd, tab, nblocks, st); break;
        case 3: lattice_mn<T, 3>(imode, fd, tab, nblocks, st); break;
        case 4: lattice_mn<T, 4>(imode, fd, tab, nblocks, st); break;
        case 5: lattice_mn<T, 5>(imode, fd, tab, nblocks, st); break;
        case 6: lattice_mn<T, 6>(imode, fd, tab, nblocks, st); break;
        case 7: lattice_mn<T, 7>(imode, fd, tab, nblocks, st); break;
        case 8: lattice_mn<T, 8>(imode, fd, tab, nblocks, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_lattice(int fp64, int mn, int imode, const FrameDesc *fd, const Work *tab,
                          int nblocks, hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    return fp64 ? lattice_t<double>(mn, imode, fd, tab, nblocks, st)
                : lattice_t<float>(mn, imode, fd, tab, nblocks, st);
}

hipError_t launch_gamma(int fp64, const FrameDesc *fd, const Work *tab, int nblocks,
                        hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    if (fp64)
        hipLaunchKernelGGL(k_gamma<double>, dim3(nblocks), dim3(kGammaLanes), 0, st, fd, tab);
    else
        hipLaunchKernelGGL(k_gamma<float>, dim3(nblocks), dim3(kGammaLanes), 0, st, fd, tab);
    return hipGetLastError();
}

hipError_t launch_chain(int fp64, const FrameDesc *fd, const int *frames, int nchains,
                        size_t lds_bytes, hipStream_t st) {
    if (nchains == 0) return hipSuccess;
    if (fp64)
        hipLaunchKernelGGL(k_chain<double>, dim3(2 * nchains), dim3(kChainThreads), lds_bytes,
                           st, fd, frames);
    else
        hipLaunchKernelGGL(k_chain<float>, dim3(2 * nchains), dim3(kChainThreads), lds_bytes,
                           st, fd, frames);
    return hipGetLastError();
}

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

}  // namespace mapdec
