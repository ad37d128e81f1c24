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
// priors, stored by delta with the states of consecutive symbols in one row
// (column (i - i0) Mt + m' + M).  One 64-lane workgroup per (symbol i, 64 drift states m'): lanes
// read consecutive start indices s = n i + m' (coalesced), the priors of
// symbol i are wave-uniform (scalar loads), and the loads of kGammaDC
// symbol values (every delta) are issued together: addresses are clamped
// into the table and out-of-range values multiplied by 0, so no load waits
// on a branch.

constexpr int kGammaDC = 4;

template <typename T, int MN>
__global__ __launch_bounds__(kGammaLanes) void k_gamma(const FrameDesc *__restrict__ fd,
                                                       const Work *__restrict__ tab) {
    constexpr int KW = 2 * MN + 1;
    const Work w = tab[blockIdx.x];
    const FrameDesc &f = fd[w.frame];
    const int Mt = f.Mt, q = f.q;
    const int per_i = (Mt + kGammaLanes - 1) / kGammaLanes;
    const int i = f.i0 + w.item / per_i;
    const int mi = (w.item % per_i) * kGammaLanes + (int)threadIdx.x;
    const int s = f.n * i + mi - f.M;
    const bool valid = mi < Mt && s >= 0 && s <= f.rho;
    const T vf = valid ? T(1) : T(0);
    // column in the segment's R table: the start index's, or (a codebook
    // per symbol) the symbol's and drift state's
    const int sc = f.percol ? (i - f.i0) * Mt + min(mi, Mt - 1)
                            : min(max(s, f.s0), f.s1) - f.s0;
    const gptr<const T> R = to_global((const T *)f.R);
    const T *pr = (const T *)f.prior + (size_t)i * q;
    const size_t sp = (size_t)f.sp;
    T acc[KW];
#pragma unroll
    for (int k = 0; k < KW; ++k) acc[k] = T(0);
    for (int D0 = 0; D0 < q; D0 += kGammaDC) {
        T r[kGammaDC][KW];
        T p[kGammaDC];
#pragma unroll
        for (int c = 0; c < kGammaDC; ++c) {
            const int D = min(D0 + c, q - 1);
            p[c] = (D0 + c < q) ? pr[D] : T(0);
#pragma unroll
            for (int k = 0; k < KW; ++k) r[c][k] = R[((size_t)D * KW + k) * sp + sc];
        }
#pragma unroll
        for (int c = 0; c < kGammaDC; ++c)
#pragma unroll
            for (int k = 0; k < KW; ++k) acc[k] += p[c] * r[c][k];
    }
    if (mi >= Mt) return;
    T *G = (T *)f.G + (size_t)(i - f.i0) * Mt + mi;   // [delta][(i - i0) Mt + m' + M]
#pragma unroll
    for (int k = 0; k < KW; ++k) G[(size_t)k * f.gsp] = acc[k] * vf;
}

// ---------------------------------------------------------------------------
// Per frame: sum the lattice workgroups' partials and apply the chain rule
//   d/dPi = g_a / 2 - (1 - Ps) g_t1 - Ps g_t0
//   d/dPd = g_d     - (1 - Ps) g_t1 - Ps g_t0
//   d/dPs = -Pt g_t1 + Pt g_t0

// One workgroup per frame: strided FP64 sums over the partials, then a
// fixed-order reduction across the workgroup.
__global__ __launch_bounds__(256) void k_dparams(const FrameDesc *__restrict__ fd) {
    __shared__ double red[4];
    const FrameDesc &f = fd[blockIdx.x];
    if (!f.dparams) return;
    if (*f.status != kStatusOk) {
        if (threadIdx.x == 0) f.dparams[0] = f.dparams[1] = f.dparams[2] = NAN;
        return;
    }
    double g[4] = {0, 0, 0, 0};
    for (int b = threadIdx.x; b < f.gacc_n; b += blockDim.x)
        for (int t = 0; t < 4; ++t) g[t] += f.gacc_all[(size_t)b * 4 + t];
    for (int t = 0; t < 4; ++t) g[t] = block_sum(g[t], red);
    if (threadIdx.x != 0) return;
    // without the d/da sweep: a path from start drift m0 to end drift mN
    // inserts mN - m0 more bits than it deletes, so a g_a - d g_d is the
    // posterior mean of mN - m0: rho - tau for known boundaries, else the
    // means the chains left after the partials
    if (!f.adj_da) {
        const double *mom = f.gacc_all + 4 * (size_t)f.gacc_n;
        const double net = (f.end_prior ? mom[0] : (double)(f.rho - f.tau)) -
                           (f.start_prior ? mom[1] : 0.0);
        g[0] = (net + f.d * g[1]) / f.a;
    }
    const double Ps = f.Ps, Pt = 1.0 - f.Pi - f.Pd;
    f.dparams[0] = 0.5 * g[0] - (1.0 - Ps) * g[2] - Ps * g[3];
    f.dparams[1] = g[1] - (1.0 - Ps) * g[2] - Ps * g[3];
    f.dparams[2] = -Pt * g[2] + Pt * g[3];
}

// Gamma(s, delta) = sum_D R(s, D, delta) / q for uniform priors whose
// lattice items are split over codeword chunks (the lattice kernel writes it
// itself otherwise): the sum of the chunks' partial sums, which the lattice
// items leave in f.Gpart ([dsplit][Mn][sp]).  Lane = start index s; every
// read is a coalesced row segment.
template <typename T, int MN>
__global__ __launch_bounds__(64) void k_gsum(const FrameDesc *__restrict__ fd,
                                             const Work *__restrict__ tab) {
    constexpr int KW = 2 * MN + 1;
    const Work w = tab[blockIdx.x];
    const FrameDesc &f = fd[w.frame];
    const int s = f.s0 + w.item + (int)threadIdx.x;
    if (s > f.s1) return;
    const size_t sp = (size_t)f.sp, c = (size_t)(s - f.s0);
    const gptr<const T> P = to_global((const T *)f.Gpart);
    T acc[KW];
#pragma unroll
    for (int k = 0; k < KW; ++k) acc[k] = T(0);
    for (int x = 0; x < f.dsplit; ++x)
#pragma unroll
        for (int k = 0; k < KW; ++k) acc[k] += P[((size_t)x * KW + k) * sp + c];
    T *G = (T *)f.G;
    const T invq = T(1) / T(f.q);
#pragma unroll
    for (int k = 0; k < KW; ++k) G[(size_t)k * f.gsp + c] = acc[k] * invq;
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

template <typename T>
static hipError_t gamma_t(int mn, const FrameDesc *fd, const Work *tab, int nblocks,
                          hipStream_t st) {
    switch (mn) {
#define MAPDEC_GAMMA_CASE(K)                                                                \
    case K:                                                                                 \
        hipLaunchKernelGGL((k_gamma<T, K>), dim3(nblocks), dim3(kGammaLanes), 0, st, fd, tab); \
        break;
        MAPDEC_GAMMA_CASE(0) MAPDEC_GAMMA_CASE(1) MAPDEC_GAMMA_CASE(2) MAPDEC_GAMMA_CASE(3)
        MAPDEC_GAMMA_CASE(4) MAPDEC_GAMMA_CASE(5) MAPDEC_GAMMA_CASE(6) MAPDEC_GAMMA_CASE(7)
        MAPDEC_GAMMA_CASE(8)
#undef MAPDEC_GAMMA_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_gamma(int fp64, int mn, const FrameDesc *fd, const Work *tab, int nblocks,
                        hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    return fp64 ? gamma_t<double>(mn, fd, tab, nblocks, st)
                : gamma_t<float>(mn, fd, tab, nblocks, st);
}

template <typename T>
static hipError_t gsum_t(int mn, const FrameDesc *fd, const Work *tab, int nblocks,
                         hipStream_t st) {
    switch (mn) {
#define MAPDEC_GSUM_CASE(K)                                                                \
    case K:                                                                                \
        hipLaunchKernelGGL((k_gsum<T, K>), dim3(nblocks), dim3(64), 0, st, fd, tab);       \
        break;
        MAPDEC_GSUM_CASE(0) MAPDEC_GSUM_CASE(1) MAPDEC_GSUM_CASE(2) MAPDEC_GSUM_CASE(3)
        MAPDEC_GSUM_CASE(4) MAPDEC_GSUM_CASE(5) MAPDEC_GSUM_CASE(6) MAPDEC_GSUM_CASE(7)
        MAPDEC_GSUM_CASE(8)
#undef MAPDEC_GSUM_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_gsum(int fp64, int mn, const FrameDesc *fd, const Work *tab, int nblocks,
                       hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    return fp64 ? gsum_t<double>(mn, fd, tab, nblocks, st)
                : gsum_t<float>(mn, fd, tab, nblocks, st);
}

hipError_t launch_dparams(const FrameDesc *fd, int nframes, hipStream_t st) {
    hipLaunchKernelGGL(k_dparams, dim3(nframes), dim3(256), 0, st, fd);
    return hipGetLastError();
}

}  // namespace mapdec
