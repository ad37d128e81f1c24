// Forward/backward recursions (eqs. 4, 5, 11, 12).
#include "device_common.h"

namespace mapdec {

// ---------------------------------------------------------------------------
// alpha / beta chains over the symbols [i0, i1) of a segment.  With both
// directions, workgroup 2c runs the forward chain of frame frames[c] and
// workgroup 2c+1 the backward chain; with one direction, workgroup c runs
// that chain.  Rows live in LDS with mn zero entries of padding on each side
// (states outside [-M, M] are 0).  A chain starts from the row given by the
// descriptor (a_init / b_init) or from the known boundary state, stores the
// rows it computes, optionally copies its last row out (a_fin / b_fin), and
// continues the cumulative log of its normalisers (logA / logB).

template <typename T>
__device__ __forceinline__ T gamma_at(const FrameDesc &f, const T *G, int i, int mp, int k) {
    if (mp < -f.M || mp > f.M) return T(0);
    if (f.uniform && !f.percol) {
        const int s = f.n * i + mp;
        return (s >= 0 && s <= f.rho) ? G[(size_t)k * f.gsp + (s - f.s0)] : T(0);
    }
    return G[(size_t)k * f.gsp + (size_t)(i - f.i0) * f.Mt + (mp + f.M)];
}

template <typename T>
__global__ __launch_bounds__(kChainThreads) void k_chain(const FrameDesc *__restrict__ fd,
                                                         const int *__restrict__ frames,
                                                         int dirs) {
    const int nd = dirs == 3 ? 2 : 1;
    const int fi = frames[blockIdx.x / nd];
    const int dir = nd == 2 ? (int)(blockIdx.x & 1) : (dirs == 1 ? 0 : 1);
    const FrameDesc &f = fd[fi];
    if (*f.status != kStatusOk) return;
    extern __shared__ __align__(16) unsigned char smem[];
    const int Mt = f.Mt, mn = f.mn, M = f.M, N = f.N, Mn = f.Mn, i0 = f.i0, i1 = f.i1;
    const int W = Mt + 2 * mn;
    double *buf0 = (double *)smem;   // rows in FP64 whatever the precision
    double *buf1 = buf0 + W;
    double *red = buf1 + W;
    const int tid = threadIdx.x, nth = blockDim.x;

    for (int j = tid; j < 2 * W; j += nth) buf0[j] = 0.0;
    __syncthreads();
    const int m0 = dir == 0 ? 0 : f.rho - f.tau;
    double *out = dir == 0 ? f.alpha : f.beta;
    double *logX = dir == 0 ? f.logA : f.logB;
    const double *init = dir == 0 ? f.a_init : f.b_init;
    const int row0 = dir == 0 ? i0 : i1;
    // where row r goes (sweep: checkpoints only), whether the starting row
    // is stored, and whether the cumulative logs are written
    const int mode = f.chain_mode, cks = f.ck_stride;
    auto stored = [&](int r) { return mode != kChainSweep || r % cks == 0; };
    auto slot = [&](int r) { return (size_t)(mode == kChainSweep ? r / cks : r - i0) * Mt; };
    // a sweep part after the first starts from the checkpoint (and its log)
    // the previous part wrote, which main passes may be reading already
    const bool resumed = mode == kChainSweep && (dir == 0 ? i0 > 0 : i1 < N);
    const bool put_init = mode == kChainSub ? ((f.wr_init >> dir) & 1) != 0
                                            : stored(row0) && !resumed;
    const bool logs = mode != kChainSub;
    const double lbase = (logs && (dir == 0 ? i0 > 0 : i1 < N)) ? logX[row0] : 0.0;
    // a boundary prior's entries whose received position (m at the start,
    // tau + m at the end) lies outside [0, rho] carry no path: zero, so that
    // no later kernel pairs them with a clamped start index
    const bool prior_row = init && (dir == 0 ? i0 == 0 : i1 == N);
    const int pos0 = dir == 0 ? 0 : f.tau;
    // drift states kept (asymmetric limits): indices [lo_i, hi_i]
    const int lo_i = f.lim_lo + M, hi_i = f.lim_hi + M;
    // path thresholds: the forward chain over the frame decides which
    // states are kept, every other chain applies its decisions
    const bool pr = f.theta > 0.0;
    const bool decide = pr && dir == 0 && mode != kChainSub;
    uint8_t *kept = f.kept;
    double s0 = 0.0;
    for (int mi = tid; mi < Mt; mi += nth) {
        double v = init ? init[mi] : ((mi == m0 + M) ? 1.0 : 0.0);
        if (prior_row && (pos0 + mi - M < 0 || pos0 + mi - M > f.rho)) v = 0.0;
        if (mi < lo_i || mi > hi_i) v = 0.0;
        if (pr && !decide && !kept[(size_t)row0 * Mt + mi]) v = 0.0;
        buf0[mn + mi] = v;
        s0 += v;
    }
    if (decide) {   // the start row against its own sum
        const double cut = f.theta * block_sum(s0, red);
        for (int mi = tid; mi < Mt; mi += nth) {
            const double v = buf0[mn + mi];
            const bool k = v > 0.0 && !(v < cut);
            buf0[mn + mi] = k ? v : 0.0;
            kept[(size_t)row0 * Mt + mi] = k ? 1 : 0;
        }
    }
    if (put_init)
        for (int mi = tid; mi < Mt; mi += nth) out[slot(row0) + mi] = buf0[mn + mi];
    if (tid == 0 && logs && !resumed) logX[row0] = lbase;
    __syncthreads();

    const T *G = (const T *)f.G;
    double lsum = lbase;
    double *cur = buf0, *nxt = buf1;
    bool dead = false;
    for (int step = 0; step < i1 - i0; ++step) {
        const int i = dir == 0 ? i0 + step : i1 - 1 - step;
        double part = 0.0;
        for (int mi = tid; mi < Mt; mi += nth) {
            const int m = mi - M;
            double acc = 0.0;
            if (dir == 0) {
                // alpha'_{i+1}(m) = sum_delta alpha_i(m - delta) Gamma_i(m - delta, delta)
                for (int k = 0; k < Mn; ++k) {
                    const int dl = k - mn;
                    acc += cur[mn + mi - dl] * (double)gamma_at(f, G, i, m - dl, k);
                }
            } else {
                // beta'_i(m) = sum_delta Gamma_i(m, delta) beta_{i+1}(m + delta)
                for (int k = 0; k < Mn; ++k) {
                    const int dl = k - mn;
                    acc += (double)gamma_at(f, G, i, m, k) * cur[mn + mi + dl];
                }
            }
            if (mi < lo_i || mi > hi_i) acc = 0.0;
            nxt[mn + mi] = acc;
            part += acc;
        }
        const double c = block_sum(part, red);
        if (!(c > 0.0) || !isfinite(c)) {
            dead = true;
            break;
        }
        const double inv = 1.0 / c;
        const int row = dir == 0 ? i + 1 : i;
        const bool st_row = stored(row);
        const size_t ro = slot(row);
        for (int mi = tid; mi < Mt; mi += nth) {
            double v = nxt[mn + mi] * inv;
            if (decide) {   // not pursued: a normalised metric below theta
                const bool k = v > 0.0 && !(v < f.theta);
                v = k ? v : 0.0;
                kept[(size_t)row * Mt + mi] = k ? 1 : 0;
            } else if (pr && !kept[(size_t)row * Mt + mi]) {
                v = 0.0;
            }
            nxt[mn + mi] = v;
            if (st_row) out[ro + mi] = v;
        }
        lsum += log(c);
        if (tid == 0 && logs && st_row) logX[row] = lsum;
        double *t = cur;
        cur = nxt;
        nxt = t;
        __syncthreads();
    }
    if (dead) {
        if (tid == 0) {
            atomicOr(f.status, kStatusNoPath);
            if (dir == 0) *f.logp = -INFINITY;
        }
        return;
    }
    double *fin = dir == 0 ? f.a_fin : f.b_fin;
    if (fin)
        for (int mi = tid; mi < Mt; mi += nth) fin[mi] = cur[mn + mi];
    if (tid != 0 || !logs) return;
    if (dir == 1 && i0 == 0 && f.grad && f.start_prior) {
        // posterior mean of the start drift (prior entries outside [0, rho]
        // carry no path), for the path-count identity of the adjoint
        double b0 = 0.0, b0m = 0.0;
        for (int mi = 0; mi < Mt; ++mi) {
            if (mi - M < 0 || mi - M > f.rho) continue;
            const double v = cur[mn + mi] * f.start_prior[mi];
            b0 += v;
            b0m += v * (double)(mi - M);
        }
        // written on every run, so that no earlier run's value is read
        f.gacc_all[4 * (size_t)f.gacc_n + 1] = b0 > 0.0 ? b0m / b0 : 0.0;
    }
    if (dir == 0 && i1 == N) {
        // P(y) = alpha_N(rho - tau), or sum_m alpha_N(m) end_prior(m), in
        // unnormalised terms
        double aN = 0.0, aNm = 0.0;
        if (f.end_prior) {
            for (int mi = 0; mi < Mt; ++mi) {
                const double v = cur[mn + mi] * f.end_prior[mi];
                aN += v;
                aNm += v * (double)(mi - M);
            }
            // posterior mean of the end drift, for the path-count identity
            // of the adjoint
            if (f.grad) f.gacc_all[4 * (size_t)f.gacc_n] = aN > 0.0 ? aNm / aN : 0.0;
        } else {
            aN = cur[mn + (f.rho - f.tau) + M];
        }
        if (!(aN > 0.0)) {
            atomicOr(f.status, kStatusNoPath);
            *f.logp = -INFINITY;
        } else {
            *f.logp = lsum + log(aN);
        }
    }
}

// ---------------------------------------------------------------------------
// launchers

hipError_t launch_chain(int fp64, const FrameDesc *fd, const int *frames, int nchains,
                        int dirs, size_t lds_bytes, hipStream_t st) {
    if (nchains == 0) return hipSuccess;
    if (dirs < 1 || dirs > 3) return hipErrorInvalidValue;
    const int nb = nchains * (dirs == 3 ? 2 : 1);
    if (fp64)
        hipLaunchKernelGGL(k_chain<double>, dim3(nb), dim3(kChainThreads), lds_bytes, st, fd,
                           frames, dirs);
    else
        hipLaunchKernelGGL(k_chain<float>, dim3(nb), dim3(kChainThreads), lds_bytes, st, fd,
                           frames, dirs);
    return hipGetLastError();
}

}  // namespace mapdec

namespace mapdec {

// One object per (precision, shape) built from k_chain_ring.hip.
#define MAPDEC_RING_DECL(name)                                                            \
    hipError_t name(int mn, int waves, int nchains, int dirs, size_t lds, hipStream_t st,  \
                    const FrameDesc *fd, const int *frames);
MAPDEC_RING_DECL(chain_ring_f32_0)
MAPDEC_RING_DECL(chain_ring_f32_1)
MAPDEC_RING_DECL(chain_ring_f32_2)
MAPDEC_RING_DECL(chain_ring_f32_3)
MAPDEC_RING_DECL(chain_ring_f32_4)
MAPDEC_RING_DECL(chain_ring_f32_5)
MAPDEC_RING_DECL(chain_ring_f32_6)
MAPDEC_RING_DECL(chain_ring_f64_0)
MAPDEC_RING_DECL(chain_ring_f64_1)
MAPDEC_RING_DECL(chain_ring_f64_2)
MAPDEC_RING_DECL(chain_ring_f64_3)
MAPDEC_RING_DECL(chain_ring_f64_4)
MAPDEC_RING_DECL(chain_ring_f64_5)
MAPDEC_RING_DECL(chain_ring_f64_6)
#undef MAPDEC_RING_DECL

hipError_t launch_chain_ring(int fp64, int shape, int mn, int waves, const FrameDesc *fd,
                             const int *frames, int nchains, int dirs, size_t lds,
                             hipStream_t st) {
    if (nchains == 0) return hipSuccess;
    if (dirs < 1 || dirs > 3) return hipErrorInvalidValue;
    using Fn = hipError_t (*)(int, int, int, int, size_t, hipStream_t, const FrameDesc *,
                              const int *);
    static const Fn f32[kNumRingShapes] = {chain_ring_f32_0, chain_ring_f32_1, chain_ring_f32_2,
                                           chain_ring_f32_3, chain_ring_f32_4, chain_ring_f32_5,
                                           chain_ring_f32_6};
    static const Fn f64[kNumRingShapes] = {chain_ring_f64_0, chain_ring_f64_1, chain_ring_f64_2,
                                           chain_ring_f64_3, chain_ring_f64_4, chain_ring_f64_5,
                                           chain_ring_f64_6};
    if (shape < 0 || shape >= kNumRingShapes) return hipErrorInvalidValue;
    if (waves < 1 || waves > kRingShapes[shape].nw) return hipErrorInvalidValue;
    return (fp64 ? f64 : f32)[shape](mn, waves, nchains, dirs, lds, st, fd, frames);
}

}  // namespace mapdec
