// Adjoint of log P(y) with respect to the channel parameters.
// Compiled once per precision: build with -DADJ_T=float|double
// -DADJ_FN=<launcher prefix>.
//
// log P(y) depends on (Pi, Pd, Ps) only through the receiver metric, and
//   d log P / d theta = sum_i (1/Z_i) sum_{m', delta, D}
//       alpha_i(m') prior_i(D) dR(n i + m', D, delta)/d theta beta_{i+1}(m' + delta)
// for any per-row scaling of alpha and beta (Z_i = sum_D S_i(D) is computed
// from the same rows, eqs. 1-3).  In reverse mode this is
//   W(s, D, delta) = sum_{i : |s - n i| <= M} prior_i(D) alpha_i(s - n i)
//                    beta_{i+1}(s - n i + delta) / Z_i                 (k_wadj)
// followed by one backward sweep through every lattice of eqs. 7-10 seeded
// with the output adjoints W, accumulating d/d(a, d, t1, t0) of the
// lattice weights a = Pi/2, d = Pd, t1 = Pt(1-Ps), t0 = Pt Ps (k_adjoint),
// and the chain rule to (Pi, Pd, Ps) with Pt = 1 - Pi - Pd (k_dparams, in
// k_misc.hip).
// Per-lattice sums are single-pass in T; every sum across lattices is FP64.
#include "device_common.h"

#if !defined(ADJ_T) || !defined(ADJ_FN)
#error "compile with -DADJ_T and -DADJ_FN"
#endif

namespace mapdec {

// ---------------------------------------------------------------------------
// W(s, D, delta): lane = start index s.  Uniform priors give W independent
// of D (one [Mn][sp] table, written over Gamma); general priors give
// [q][Mn][sp] (written over R, which the APP no longer needs).

template <typename T>
__global__ __launch_bounds__(64) void k_wadj(const FrameDesc *__restrict__ fd,
                                             const Work *__restrict__ tab) {
    const Work w = tab[blockIdx.x];
    const FrameDesc &f = fd[w.frame];
    if (*f.status != kStatusOk) return;
    const int s = w.item + (int)threadIdx.x;
    if (s > f.rho) return;
    const int n = f.n, M = f.M, Mt = f.Mt, Mn = f.Mn, mn = f.mn, N = f.N, q = f.q;
    const gptr<const double> A = to_global((const double *)f.alpha);
    const gptr<const double> B = to_global((const double *)f.beta);
    const size_t sp = (size_t)f.sp;
    // symbols whose drift band [n i - M, n i + M] contains s
    const int ilo = max(0, (s - M + n - 1) / n), ihi = min(N - 1, (s + M) / n);
    if (f.uniform) {
        const gptr<T> W = to_global((T *)f.G);
        for (int k = 0; k < Mn; ++k) {
            double acc = 0.0;
            for (int i = ilo; i <= ihi; ++i) {
                const int mp = s - n * i, m = mp + k - mn;
                if (m < -M || m > M) continue;
                acc += A[(size_t)i * Mt + mp + M] * B[(size_t)(i + 1) * Mt + m + M] * f.Zinv[i];
            }
            W[(size_t)k * sp + s] = (T)(acc / q);
        }
    } else {
        const gptr<T> W = to_global((T *)f.R);
        const T *pr = (const T *)f.prior;
        for (int D = 0; D < q; ++D) {
            for (int k = 0; k < Mn; ++k) {
                double acc = 0.0;
                for (int i = ilo; i <= ihi; ++i) {
                    const int mp = s - n * i, m = mp + k - mn;
                    if (m < -M || m > M) continue;
                    acc += (double)pr[(size_t)i * q + D] * A[(size_t)i * Mt + mp + M] *
                           B[(size_t)(i + 1) * Mt + m + M] * f.Zinv[i];
                }
                W[((size_t)D * Mn + k) * sp + s] = (T)acc;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Backward sweep through the lattices.  Lane = start index s, loop over D
// (codeword bits are wave-uniform).  Forward rows F_0 .. F_{n-1} are parked
// in LDS ([row][k][lane], conflict-free); the sweep then runs from the last
// row up, with corridor coordinates k = j - r + MN as in the lattice kernel:
//   Gbar_n = Fbar_n = W
//   Gbar_r[k] = Fbar_r[k] + sum_t a_t Fbar_r[k + t]        (r < n)
//   abar += Fbar_r[k] sum_t (t a^(t-1)) G_r[k - t]         (r < n, t <= I)
//   dbar += Gbar_r[k] F_{r-1}[k + 1]
//   t1bar / t0bar += Gbar_r[k] F_{r-1}[k] (bit received equal / flipped)
//   Fbar_{r-1}[k] = Q_r[k] Gbar_r[k] + d Gbar_r[k - 1]
// and row 0, F_0[k] = a^(k - MN), adds its own term to abar.

template <typename T, int MN, int NB>
__device__ __forceinline__ void adj_row_in(T (&G)[2 * MN + 1], const T (&F)[2 * MN + 1],
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
__global__ __launch_bounds__(64) void k_adjoint(const FrameDesc *__restrict__ fd,
                                                const Work *__restrict__ tab) {
    constexpr int KW = 2 * MN + 1;
    constexpr int NB = kMaxN + MN;
    extern __shared__ __align__(16) unsigned char smem[];
    const Work w = tab[blockIdx.x];
    const FrameDesc &f = fd[w.frame];
    if (*f.status != kStatusOk) return;
    const int lane = threadIdx.x;
    const int s = w.item + lane;
    const bool live = s <= f.rho;
    const int n = f.n, q = f.q, rho = f.rho;
    const T d = (T)f.d, t1 = (T)f.t1, t0 = (T)f.t0;
    T *rows = (T *)smem;   // [n][KW][64]

    T apow[IM + 1], dapow[IM + 1];
    {
        T p = T(1);
        apow[0] = T(1);
        dapow[0] = T(0);
#pragma unroll
        for (int t = 1; t <= IM; ++t) {
            dapow[t] = (t <= f.I) ? T(t) * p : T(0);   // d(a^t)/da = t a^(t-1)
            p *= (T)f.a;
            apow[t] = (t <= f.I) ? p : T(0);
        }
    }
    const int sl = live ? s : 0;
    const int wi = sl >> 5, sh = sl & 31;
    const uint32_t lo = f.ybits[wi], hi = f.ybits[wi + 1];
    const uint32_t win = sh ? ((lo >> sh) | (hi << (32 - sh))) : lo;
    // Q values for a 0 / 1 codeword bit, and the received bit as 0/1 weights
    // (exact) to split the transmission adjoint into equal / flipped bits
    T qx0[NB], qx1[NB], ym[NB], yn[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const bool one = (win >> b) & 1u;
        qx0[b] = one ? t0 : t1;
        qx1[b] = one ? t1 : t0;
        ym[b] = one ? T(1) : T(0);
        yn[b] = one ? T(0) : T(1);
    }
    const gptr<const T> Wt = to_global((const T *)(f.uniform ? f.G : f.R));
    const size_t sp = (size_t)f.sp;
    double ga = 0.0, gd = 0.0, g1 = 0.0, g0 = 0.0;

    for (int D = 0; D < q; ++D) {
        const uint32_t cw = f.cw[D];
        // output adjoints of this lattice (zero for invalid segments)
        T Fb[KW];
        const size_t wbase = (size_t)(f.uniform ? 0 : D) * KW * sp;
#pragma unroll
        for (int k = 0; k < KW; ++k) {
            const int len = n + k - MN;
            Fb[k] = (live && len >= 0 && s + len <= rho) ? Wt[wbase + (size_t)k * sp + sl] : T(0);
        }
        // forward rows F_0 .. F_{n-1} to LDS
        T F[KW];
#pragma unroll
        for (int k = 0; k < KW; ++k) {
            const int dl = k - MN;
            F[k] = (dl >= 0 && dl <= IM) ? apow[dl] : T(0);
        }
#pragma unroll
        for (int r = 1; r <= kMaxN; ++r) {
            if (r > n - 1) break;
#pragma unroll
            for (int k = 0; k < KW; ++k) rows[((r - 1) * KW + k) * 64 + lane] = F[k];
            T G[KW];
            if ((cw >> (n - r)) & 1u)
                adj_row_in<T, MN, NB>(G, F, qx1, d, r);
            else
                adj_row_in<T, MN, NB>(G, F, qx0, d, r);
#pragma unroll
            for (int k = 0; k < KW; ++k) {
                T v = G[k];
#pragma unroll
                for (int t = 1; t <= IM; ++t)
                    if (t <= k) v += apow[t] * G[k - t];
                F[k] = v;
            }
        }
#pragma unroll
        for (int k = 0; k < KW; ++k) rows[((n - 1) * KW + k) * 64 + lane] = F[k];
        // backward sweep, rows n .. 1
        T sa = T(0), sd = T(0), s1 = T(0), s0 = T(0);
#pragma unroll
        for (int rr = kMaxN; rr >= 1; --rr) {
            if (rr > n) continue;
            const int r = rr;
            T Fp[KW];
#pragma unroll
            for (int k = 0; k < KW; ++k) Fp[k] = rows[((r - 1) * KW + k) * 64 + lane];
            const bool xb = (cw >> (n - r)) & 1u;
            T Gb[KW];
            if (r == n) {
#pragma unroll
                for (int k = 0; k < KW; ++k) Gb[k] = Fb[k];
            } else {
                // G_r recomputed from F_{r-1} for the insertion-weight term
                T G[KW];
                if (xb)
                    adj_row_in<T, MN, NB>(G, Fp, qx1, d, r);
                else
                    adj_row_in<T, MN, NB>(G, Fp, qx0, d, r);
#pragma unroll
                for (int k = 0; k < KW; ++k) {
                    T v = Fb[k];
#pragma unroll
                    for (int t = 1; t <= IM; ++t)
                        if (k + t < KW) v += apow[t] * Fb[k + t];
                    Gb[k] = v;
                    T u = T(0);
#pragma unroll
                    for (int t = 1; t <= IM; ++t)
                        if (t <= k) u += dapow[t] * G[k - t];
                    sa += Fb[k] * u;
                }
            }
            // diagonal and vertical moves into row r; yeq / yne are the 0/1
            // weights of "received bit equal to / different from x_r"
            auto back = [&](const T(&qx)[NB], const T(&yeq)[NB], const T(&yne)[NB]) {
#pragma unroll
                for (int k = 0; k < KW; ++k) {
                    if (k + 1 < KW) sd += Gb[k] * Fp[k + 1];
                    const int b = r + k - MN - 1;
                    if (b >= 0) {
                        const T prod = Gb[k] * Fp[k];
                        s1 += prod * yeq[b];
                        s0 += prod * yne[b];
                    }
                }
#pragma unroll
                for (int k = 0; k < KW; ++k) {
                    const int b = r + k - MN - 1;
                    T v = (b >= 0) ? qx[b] * Gb[k] : T(0);
                    if (k >= 1) v += d * Gb[k - 1];
                    Fb[k] = v;
                }
            };
            if (xb)
                back(qx1, ym, yn);
            else
                back(qx0, yn, ym);
        }
        // row 0: F_0[k] = a^(k - MN) for 1 <= k - MN <= I
#pragma unroll
        for (int k = 0; k < KW; ++k) {
            const int dl = k - MN;
            if (dl >= 1 && dl <= IM) sa += Fb[k] * dapow[dl];
        }
        ga += (double)sa;
        gd += (double)sd;
        g1 += (double)s1;
        g0 += (double)s0;
    }
    ga = wave_sum(ga);
    gd = wave_sum(gd);
    g1 = wave_sum(g1);
    g0 = wave_sum(g0);
    if (lane == 0) {
        double *o = f.gacc + (size_t)(w.item / 64) * 4;
        o[0] = ga;
        o[1] = gd;
        o[2] = g1;
        o[3] = g0;
    }
}

// ---------------------------------------------------------------------------
// launchers

#define ADJ_CAT2(a, b) a##b
#define ADJ_CAT(a, b) ADJ_CAT2(a, b)

hipError_t ADJ_CAT(ADJ_FN, _w)(const FrameDesc *fd, const Work *tab, int nblocks,
                               hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_wadj<ADJ_T>, dim3(nblocks), dim3(64), 0, st, fd, tab);
    return hipGetLastError();
}

template <int MN>
static hipError_t adj_mn(int imode, const FrameDesc *fd, const Work *tab, int nblocks,
                         size_t lds, hipStream_t st) {
    constexpr int IM2 = (2 < 2 * MN) ? 2 : 2 * MN;
    if (imode == 0)
        hipLaunchKernelGGL((k_adjoint<ADJ_T, MN, IM2>), dim3(nblocks), dim3(64), lds, st, fd,
                           tab);
    else
        hipLaunchKernelGGL((k_adjoint<ADJ_T, MN, 2 * MN>), dim3(nblocks), dim3(64), lds, st, fd,
                           tab);
    return hipGetLastError();
}

hipError_t ADJ_CAT(ADJ_FN, _lattice)(int mn, int imode, const FrameDesc *fd, const Work *tab,
                                     int nblocks, size_t lds, hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    switch (mn) {
        case 0: return adj_mn<0>(imode, fd, tab, nblocks, lds, st);
        case 1: return adj_mn<1>(imode, fd, tab, nblocks, lds, st);
        case 2: return adj_mn<2>(imode, fd, tab, nblocks, lds, st);
        case 3: return adj_mn<3>(imode, fd, tab, nblocks, lds, st);
        case 4: return adj_mn<4>(imode, fd, tab, nblocks, lds, st);
        case 5: return adj_mn<5>(imode, fd, tab, nblocks, lds, st);
        case 6: return adj_mn<6>(imode, fd, tab, nblocks, lds, st);
        case 7: return adj_mn<7>(imode, fd, tab, nblocks, lds, st);
        case 8: return adj_mn<8>(imode, fd, tab, nblocks, lds, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace mapdec
