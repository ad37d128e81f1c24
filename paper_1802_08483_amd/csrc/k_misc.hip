// Per-call initialisation, bit packing and Gamma assembly for general priors.
#include "device_common.h"

namespace mapdec {

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
// Gamma_i(m', delta) = sum_D prior_i(D) R(n i + m', D, delta) for general
// priors; one lane per drift state m', lanes read consecutive s.

template <typename T>
__global__ __launch_bounds__(kGammaLanes) void k_gamma(const FrameDesc *__restrict__ fd,
                                                       const Work *__restrict__ tab) {
    const Work w = tab[blockIdx.x];
    const FrameDesc &f = fd[w.frame];
    const int per_i = (f.Mt + kGammaLanes - 1) / kGammaLanes;
    const int i = f.i0 + w.item / per_i;
    const int mi = (w.item % per_i) * kGammaLanes + (int)threadIdx.x;
    if (mi >= f.Mt) return;
    const int Mn = f.Mn, Mt = f.Mt, q = f.q;
    const int s = f.n * i + mi - f.M;
    T *G = (T *)f.G + (size_t)(i - f.i0) * Mn * Mt + mi;
    if (s < 0 || s > f.rho) {
        for (int k = 0; k < Mn; ++k) G[(size_t)k * Mt] = T(0);
        return;
    }
    const T *pr = (const T *)f.prior + (size_t)i * q;
    const T *R = (const T *)f.R + (s - f.s0);   // s in [s0, s1] for the segment's symbols
    const size_t sp = (size_t)f.sp;
    for (int k = 0; k < Mn; ++k) {
        T acc = T(0);
        for (int D = 0; D < q; ++D) acc += pr[D] * R[((size_t)D * Mn + k) * sp];
        G[(size_t)k * Mt] = acc;
    }
}

// ---------------------------------------------------------------------------
// Per frame: sum the lattice workgroups' partials and apply the chain rule
//   d/dPi = g_a / 2 - (1 - Ps) g_t1 - Ps g_t0
//   d/dPd = g_d     - (1 - Ps) g_t1 - Ps g_t0
//   d/dPs = -Pt g_t1 + Pt g_t0

__global__ void k_dparams(const FrameDesc *__restrict__ fd, int nframes) {
    const int fi = blockIdx.x * blockDim.x + threadIdx.x;
    if (fi >= nframes) return;
    const FrameDesc &f = fd[fi];
    if (!f.dparams) return;
    if (*f.status != kStatusOk) {
        f.dparams[0] = f.dparams[1] = f.dparams[2] = NAN;
        return;
    }
    double g[4] = {0, 0, 0, 0};
    for (int b = 0; b < f.gacc_n; ++b)
        for (int t = 0; t < 4; ++t) g[t] += f.gacc_all[(size_t)b * 4 + t];
    // without the d/da sweep: a g_a - d g_d = rho - tau (every path inserts
    // rho - tau more bits than it deletes)
    if (!f.adj_da) g[0] = ((double)(f.rho - f.tau) + f.d * g[1]) / f.a;
    const double Ps = f.Ps, Pt = 1.0 - f.Pi - f.Pd;
    f.dparams[0] = 0.5 * g[0] - (1.0 - Ps) * g[2] - Ps * g[3];
    f.dparams[1] = g[1] - (1.0 - Ps) * g[2] - Ps * g[3];
    f.dparams[2] = -Pt * g[2] + Pt * g[3];
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

hipError_t launch_gamma(int fp64, const FrameDesc *fd, const Work *tab, int nblocks,
                        hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    if (fp64)
        hipLaunchKernelGGL(k_gamma<double>, dim3(nblocks), dim3(kGammaLanes), 0, st, fd, tab);
    else
        hipLaunchKernelGGL(k_gamma<float>, dim3(nblocks), dim3(kGammaLanes), 0, st, fd, tab);
    return hipGetLastError();
}

hipError_t launch_dparams(const FrameDesc *fd, int nframes, hipStream_t st) {
    hipLaunchKernelGGL(k_dparams, dim3((nframes + 63) / 64), dim3(64), 0, st, fd, nframes);
    return hipGetLastError();
}

}  // namespace mapdec
