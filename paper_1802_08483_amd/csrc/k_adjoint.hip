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
// with the output adjoints W (k_adjoint), which accumulates the partials
// g_d, g_1, g_0 of log P with respect to the lattice weights d = Pd,
// t1 = Pt(1-Ps), t0 = Pt Ps, and, where needed, g_a for a = Pi/2.
//
// Every path through the frame's lattices inserts rho - tau more bits than it
// deletes, so a g_a - d g_d = rho - tau exactly; k_dparams (k_misc.hip) uses
// that to obtain g_a from g_d, except when Pi is zero or small against Pd
// (a g_a would then be a small difference of larger terms), where the sweep
// accumulates g_a itself.  k_dparams then applies the chain rule to
// (Pi, Pd, Ps) with Pt = 1 - Pi - Pd.
// Per-lattice sums are single-pass in T; every sum across lattices is FP64.
#include "device_common.h"

#if !defined(ADJ_T) || !defined(ADJ_FN)
#error "compile with -DADJ_T and -DADJ_FN"
#endif

namespace mapdec {

// ---------------------------------------------------------------------------
// W(s, D, delta): lane = start index s; the 64 lanes of a workgroup take
// consecutive s, so the symbols i whose drift band reaches the wave form one
// wave-uniform range and every alpha / beta load is a coalesced row segment.
// Products and sums are FP64 (the metric rows are FP64), each product
// alpha_i beta_{i+1} / Z_i formed from mantissas and exponent sums with the
// APP's per-symbol scale 2^-Zexp[i], which keeps it inside the FP64 range
// where the plain product of the two rows would not be; W is stored in T.
// Uniform priors give W independent of D (one [Mn][sp] table, written over
// Gamma); general priors give [q][Mn][sp] (written over R, which the APP no
// longer needs), computed in chunks of kWadjDC symbol values.

constexpr int kWadjDC = 4;

// UNI: every frame of the launch has uniform priors (else none has).
template <typename T, int MN, bool UNI>
__global__ __launch_bounds__(64) void k_wadj(const FrameDesc *__restrict__ fd,
                                             const Work *__restrict__ tab) {
    constexpr int KW = 2 * MN + 1;
    const Work w = tab[blockIdx.x];
    const FrameDesc &f = fd[w.frame];
    if (*f.status != kStatusOk) return;
    const int sa = f.s0 + w.item, s = sa + (int)threadIdx.x;   // column s - s0
    const int n = f.n, M = f.M, Mt = f.Mt, q = f.q, ib = f.i0;
    const bool live = s <= f.s1;
    const gptr<const double> A = to_global((const double *)f.alpha);
    const gptr<const double> B = to_global((const double *)f.beta);
    const gptr<const double> Zi = to_global((const double *)f.Zinv);
    const gptr<const int> Ze = to_global((const int *)f.Zexp);
    const size_t sp = (size_t)f.sp;
    // symbols of the segment whose band [n i - M, n i + M] meets [sa, sa + 63]
    const int ilo = max(f.i0, sa - M <= 0 ? 0 : (sa - M + n - 1) / n);
    const int ihi = min(f.i1 - 1, (sa + 63 + M) / n);
    // one term of the sum over i: the lane's alpha_i(m') / Z_i and beta_{i+1}(m' + delta).
    // Every load is issued (addresses clamped into the row, out-of-band values
    // multiplied by 0), so the compiler cannot turn them into one branch and
    // one wait per load.
    // term = ldexp(av bv[k], ae + be[k]) with av, bv[k] mantissas
    auto term = [&](int i, double &av, int &ae, double (&bv)[KW], int (&be)[KW]) {
        const int mp = s - n * i;
        const double in = (live && mp >= -M && mp <= M) ? 1.0 : 0.0;
        const int mc = min(max(mp, -M), M);
        int ea;
        av = frexp(A[(size_t)(i - ib) * Mt + mc + M], &ea) * Zi[i] * in;
        ae = ea - Ze[i];
#pragma unroll
        for (int k = 0; k < KW; ++k) {
            const int m = mp + k - MN;
            const int cm = min(max(m, -M), M);
            int eb;
            const double b = frexp(B[(size_t)(i + 1 - ib) * Mt + cm + M], &eb);
            bv[k] = b * ((m >= -M && m <= M) ? 1.0 : 0.0);
            be[k] = eb;
        }
    };
    if constexpr (UNI) {
        // beta_{i+1} over the wave's window (drifts sa - n i - mn ..
        // sa + 63 - n i + mn), split into (mantissa, exponent) once per value
        // and staged in LDS, where each lane reads its 2 mn + 1 neighbours
        // (one wave: LDS operations stay in program order).  The loads of
        // symbol i + 1 (its window, alpha, 1/Z) are issued before symbol i's
        // products, so their latency overlaps them.
        constexpr int WIN = 64 + 2 * MN;
        static_assert(WIN <= 128, "two window values per lane");
        __shared__ double bm[2][WIN];
        __shared__ int bx[2][WIN];
        const int lane = threadIdx.x;
        double acc[KW];
#pragma unroll
        for (int k = 0; k < KW; ++k) acc[k] = 0.0;
        // raw values of one symbol: window slots lane and lane + 64, alpha
        // of the lane's drift state (addresses clamped into the rows)
        double rb0 = 0.0, rb1 = 0.0, ra = 0.0, rz = 0.0;
        int rze = 0;
        auto fetch = [&](int i) {
            const size_t rb = (size_t)(i + 1 - ib) * Mt + M;
            const int base = sa - n * i - MN;
            rb0 = B[rb + min(max(base + lane, -M), M)];
            if (lane + 64 < WIN) rb1 = B[rb + min(max(base + lane + 64, -M), M)];
            ra = A[(size_t)(i - ib) * Mt + M + min(max(s - n * i, -M), M)];
            rz = Zi[i];
            rze = Ze[i];
        };
        if (ilo <= ihi) fetch(ilo);
        for (int i = ilo; i <= ihi; ++i) {
            const int buf = (i - ilo) & 1;
            const int base = sa - n * i - MN;   // drift of window slot 0
            {
                int e;
                const int m = base + lane;
                const double v = frexp(rb0, &e);
                bm[buf][lane] = (m >= -M && m <= M) ? v : 0.0;
                bx[buf][lane] = e;
            }
            if (lane + 64 < WIN) {
                int e;
                const int m = base + lane + 64;
                const double v = frexp(rb1, &e);
                bm[buf][lane + 64] = (m >= -M && m <= M) ? v : 0.0;
                bx[buf][lane + 64] = e;
            }
            const int mp = s - n * i;
            const double in = (live && mp >= -M && mp <= M) ? 1.0 : 0.0;
            int ea;
            double av = frexp(ra, &ea) * rz * in;
            int ae = ea - rze;
            // this symbol's loads are used up before the next ones are issued
            // (load counters drain in order: a later use of an older load
            // would wait for the newer loads too)
            asm volatile("" : "+v"(av), "+v"(ae) : : "memory");
            if (i < ihi) fetch(i + 1);
            lds_wave_sync();
#pragma unroll
            for (int k = 0; k < KW; ++k)
                acc[k] += ldexp(av * bm[buf][lane + k], ae + bx[buf][lane + k]);
        }
        if (!live) return;
        const gptr<T> W = to_global((T *)f.G);
        const double invq = 1.0 / q;
#pragma unroll
        for (int k = 0; k < KW; ++k) W[(size_t)k * sp + (s - f.s0)] = (T)(acc[k] * invq);
    } else {
        const gptr<T> W = to_global((T *)f.R);
        const T *pr = (const T *)f.prior;
        for (int D0 = 0; D0 < q; D0 += kWadjDC) {
            double acc[kWadjDC][KW];
#pragma unroll
            for (int c = 0; c < kWadjDC; ++c)
#pragma unroll
                for (int k = 0; k < KW; ++k) acc[c][k] = 0.0;
            for (int i = ilo; i <= ihi; ++i) {
                double av, bv[KW];
                int ae, be[KW];
                term(i, av, ae, bv, be);
                double pb[KW];
#pragma unroll
                for (int k = 0; k < KW; ++k) pb[k] = ldexp(av * bv[k], ae + be[k]);
#pragma unroll
                for (int c = 0; c < kWadjDC; ++c) {
                    const int D = min(D0 + c, q - 1);
                    const double pa = (double)pr[(size_t)i * q + D];
#pragma unroll
                    for (int k = 0; k < KW; ++k) acc[c][k] += pa * pb[k];
                }
            }
            if (!live) continue;
#pragma unroll
            for (int c = 0; c < kWadjDC; ++c) {
                if (D0 + c >= q) break;
#pragma unroll
                for (int k = 0; k < KW; ++k)
                    W[((size_t)(D0 + c) * KW + k) * sp + (s - f.s0)] = (T)acc[c][k];
            }
        }
    }
}

// W with a codebook per symbol position: R has one column per (symbol i,
// drift state m') (column c = (i - i0) Mt + m' + M), so each column meets
// one symbol only and W needs no sum over i:
//   W(c, D, delta) = prior_i(D) alpha_i(m') beta_{i+1}(m' + delta) / Z_i,
// formed from mantissas and exponent sums as above.  Lane = column.
template <typename T, int MN, bool UNI>
__global__ __launch_bounds__(64) void k_wadj_col(const FrameDesc *__restrict__ fd,
                                                 const Work *__restrict__ tab) {
    constexpr int KW = 2 * MN + 1;
    const Work w = tab[blockIdx.x];
    const FrameDesc &f = fd[w.frame];
    if (*f.status != kStatusOk) return;
    const int c = w.item + (int)threadIdx.x;
    const int Mt = f.Mt, M = f.M, q = f.q, ib = f.i0;
    if (c >= (f.i1 - f.i0) * Mt) return;
    const int di = c / Mt, i = ib + di, mi = c - di * Mt, mp = mi - M;
    const gptr<const double> A = to_global((const double *)f.alpha);
    const gptr<const double> B = to_global((const double *)f.beta);
    int ea;
    const double av = frexp(A[(size_t)di * Mt + mi], &ea) * f.Zinv[i];
    const int ae = ea - f.Zexp[i];
    double pb[KW];
#pragma unroll
    for (int k = 0; k < KW; ++k) {
        const int m = mp + k - MN;
        const int cm = min(max(m, -M), M);
        int eb;
        const double b = frexp(B[(size_t)(di + 1) * Mt + cm + M], &eb);
        pb[k] = (m >= -M && m <= M) ? ldexp(av * b, ae + eb) : 0.0;
    }
    const size_t sp = (size_t)f.sp;
    if constexpr (UNI) {
        const gptr<T> W = to_global((T *)f.G);
        const double invq = 1.0 / q;
#pragma unroll
        for (int k = 0; k < KW; ++k) W[(size_t)k * sp + c] = (T)(pb[k] * invq);
    } else {
        const gptr<T> W = to_global((T *)f.R);
        const T *pr = (const T *)f.prior + (size_t)i * q;
        for (int D = 0; D < q; ++D) {
            const double pa = (double)pr[D];
#pragma unroll
            for (int k = 0; k < KW; ++k) W[((size_t)D * KW + k) * sp + c] = (T)(pa * pb[k]);
        }
    }
}

// ---------------------------------------------------------------------------
// Backward sweep through the lattices.  Lane = start index s, loop over D
// (codeword bits are wave-uniform).  The even forward rows F_2, F_4, .. below
// row n are parked in LDS with no padding: 16-byte slots [slot][lane] of
// 16 / sizeof(T) corridor coordinates each, then the last coordinates one
// by one, [value][lane]; a slot wholly below mn - r is not stored (a node
// there would have consumed fewer than 0 received bits: always zero).  Each
// odd row is recomputed from the even row under it
// when the sweep needs it (half the LDS, so twice the waves per SIMD, for
// one extra forward row per two rows); the sweep then
// runs from the last row up, with corridor coordinates k = j - r + MN as in
// the lattice kernel:
//   Gbar_n = Fbar_n = W
//   Gbar_r[k] = Fbar_r[k] + sum_t a_t Fbar_r[k + t]        (r < n)
//   dbar += Gbar_r[k] F_{r-1}[k + 1]
//   P_x[b] += Gbar_r[k] F_{r-1}[k]     (x = codeword bit x_r, b = received
//                                       position of the diagonal move)
//   Fbar_{r-1}[k] = Q_r[k] Gbar_r[k] + d Gbar_r[k - 1]
// After each lattice, t1bar = sum_b P_{y_b}[b] (received bit equal to the
// codeword bit) and t0bar = sum_b P_{1 - y_b}[b].  With SA the sweep also
// accumulates
//   abar += Fbar_r[k] sum_t (t a^(t-1)) G_r[k - t]         (r < n, t <= I)
// and row 0, F_0[k] = a^(k - MN), adds its own term.

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

template <typename T>
struct alignas(16) Slot {
    static constexpr int E = 16 / sizeof(T);
    T v[E];
};

// Zeroes corridor coordinates outside the frame's corridor (asymmetric
// limits: the lattice zeroed those nodes, so their adjoints are zero too);
// frames with the full corridor skip it on one scalar compare.
template <typename T, int KW>
__device__ __forceinline__ void adj_mask(T (&F)[KW], uint32_t cmask) {
    if (cmask != (1u << KW) - 1u) {
#pragma unroll
        for (int k = 0; k < KW; ++k) F[k] = ((cmask >> k) & 1u) ? F[k] : T(0);
    }
}

// GEN: the general scheme's instance (a codebook per symbol or a narrower
// corridor).  With f.percol, lane = column (symbol i, drift state m') with
// codeword C_i(D), as in the lattice kernel; else lane = start index s.
template <typename T, int MN, int IM, bool SA, bool GEN>
__global__ __launch_bounds__(64) void k_adjoint(const FrameDesc *__restrict__ fd,
                                                const Work *__restrict__ tab) {
    constexpr int KW = 2 * MN + 1;
    constexpr int NB = kMaxN + MN;
    constexpr int VE = Slot<T>::E;
    extern __shared__ __align__(16) unsigned char smem[];
    const Work w = tab[blockIdx.x];
    const FrameDesc &f = fd[w.frame];
    if (*f.status != kStatusOk) return;
    const int lane = threadIdx.x;
    const int chunk = w.item & 63;   // codewords [chunk dq, (chunk + 1) dq)
    const int col = (w.item & ~63) + lane;   // column of W
    const int n = f.n, q = f.q, rho = f.rho;
    const bool PERCOL = GEN && f.percol;
    int s, sym = 0;
    bool live;
    if (PERCOL) {
        const bool in = col < (f.i1 - f.i0) * f.Mt;
        const int cc = in ? col : 0;
        const int di = cc / f.Mt;
        sym = f.i0 + di;
        s = n * sym + (cc - di * f.Mt) - f.M;
        live = in && s >= 0 && s <= rho;
    } else {
        s = f.s0 + col;
        live = s <= f.s1;
    }
    const uint32_t cmask = GEN ? f.cmask : 0xffffffffu;
    const T d = (T)f.d, t1 = (T)f.t1, t0 = (T)f.t0;
    // parked row F_r (r even): park_values(MN, r, VE) values of 64 lanes from
    // value park_offset<MN>(r, VE) of the region (64 sizeof(T) bytes per
    // value: every row starts on a 16-byte boundary)
    auto row_at = [&](int r) {
        return smem + (size_t)park_offset<MN>(r, VE) * 64 * sizeof(T);
    };

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
    T F0[KW];
#pragma unroll
    for (int k = 0; k < KW; ++k) {
        const int dl = k - MN;   // row 0: dl insertions before the first bit
        F0[k] = (dl >= 0 && dl <= IM) ? apow[dl] : T(0);
    }
    if (GEN) adj_mask<T, KW>(F0, cmask);
    const int sl = live ? s : (PERCOL ? 0 : f.s0);
    const int wc = PERCOL ? (live ? col : 0) : sl - f.s0;   // W column
    const int wi = sl >> 5, sh = sl & 31;
    const uint32_t lo = f.ybits[wi], hi = f.ybits[wi + 1];
    const uint32_t win = sh ? ((lo >> sh) | (hi << (32 - sh))) : lo;
    // Q values for a 0 / 1 codeword bit
    T qx0[NB], qx1[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const bool one = (win >> b) & 1u;
        qx0[b] = one ? t0 : t1;
        qx1[b] = one ? t1 : t0;
    }
    const gptr<const T> Wt = to_global((const T *)(f.uniform ? f.G : f.R));
    const size_t sp = (size_t)f.sp;
    double ga = 0.0, gd = 0.0, g1 = 0.0, g0 = 0.0;

    // (r is a constant in every call: the row loops are unrolled)
    constexpr int KV = KW / VE;        // 16-byte slots of a row, then KT values
    constexpr int KT = KW - KV * VE;
    auto park = [&](int r, const T(&F)[KW]) {
        const int c0 = park_first<MN>(r) / VE;   // slots below c0 hold zeros only
        Slot<T> *sl = (Slot<T> *)row_at(r) - c0 * 64;
        T *tl = (T *)(sl + KV * 64);
#pragma unroll
        for (int c = 0; c < KV; ++c) {
            if (c < c0) continue;
            Slot<T> sv;
#pragma unroll
            for (int e = 0; e < VE; ++e) sv.v[e] = F[c * VE + e];
            sl[c * 64 + lane] = sv;
        }
#pragma unroll
        for (int t = 0; t < KT; ++t) tl[t * 64 + lane] = F[KV * VE + t];
    };
    auto unpark = [&](int r, T(&F)[KW]) {
        const int c0 = park_first<MN>(r) / VE;
        const Slot<T> *sl = (const Slot<T> *)row_at(r) - c0 * 64;
        const T *tl = (const T *)(sl + KV * 64);
#pragma unroll
        for (int c = 0; c < KV; ++c) {
            if (c < c0) {
#pragma unroll
                for (int e = 0; e < VE; ++e) F[c * VE + e] = T(0);
                continue;
            }
            const Slot<T> sv = sl[c * 64 + lane];
#pragma unroll
            for (int e = 0; e < VE; ++e) F[c * VE + e] = sv.v[e];
        }
#pragma unroll
        for (int t = 0; t < KT; ++t) F[KV * VE + t] = tl[t * 64 + lane];
    };

    const int Dlo = chunk * f.dq, Dhi = min(q, Dlo + f.dq);
    for (int D = Dlo; D < Dhi; ++D) {
        // wave-uniform with one codebook, the lane's symbol's otherwise
        const uint32_t cw = GEN ? f.cw[(size_t)sym * f.cwi + D]
                                : __builtin_amdgcn_readfirstlane(f.cw[D]);
        // output adjoints of this lattice (zero for invalid segments)
        T Fb[KW];
        const size_t wbase = (size_t)(f.uniform ? 0 : D) * KW * sp;
        bool nz = false;
#pragma unroll
        for (int k = 0; k < KW; ++k) {
            const int len = n + k - MN;
            Fb[k] = (live && len >= 0 && s + len <= rho) ? Wt[wbase + (size_t)k * sp + wc] : T(0);
            nz |= Fb[k] != T(0);
        }
        // lattices whose output adjoints are all zero (no path through
        // them: metric rows zero there, e.g. states the path thresholds
        // dropped) contribute nothing: the wave skips them together
        if (__ballot(nz) == 0) continue;
        // forward rows F_1 .. F_{n-1}; the even ones to LDS
        {
            T F[KW];
#pragma unroll
            for (int k = 0; k < KW; ++k) F[k] = F0[k];
#pragma unroll
            for (int r = 1; r <= kMaxN; ++r) {
                if (r > n - 1) continue;   // constant trip count: the loop unrolls
                T G[KW];
                if ((cw >> (n - r)) & 1u) {
                    adj_row_in<T, MN, NB>(G, F, qx1, d, r);
                    keep_branch();
                } else {
                    adj_row_in<T, MN, NB>(G, F, qx0, d, r);
                }
                if (GEN) adj_mask<T, KW>(G, cmask);
#pragma unroll
                for (int k = 0; k < KW; ++k) {
                    T v = G[k];
#pragma unroll
                    for (int t = 1; t <= IM; ++t)
                        if (t <= k) v += apow[t] * G[k - t];
                    F[k] = v;
                }
                if (GEN) adj_mask<T, KW>(F, cmask);
                if ((r & 1) == 0) park(r, F);
            }
        }
        // backward sweep, rows n .. 1
        T P0[NB], P1[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) P0[b] = P1[b] = T(0);
        T sa = T(0), sd = T(0);
#pragma unroll
        for (int rr = kMaxN; rr >= 1; --rr) {
            if (rr > n) continue;
            const int r = rr;
            // F_{r-1}: parked (even), row 0, or recomputed from F_{r-2} (odd)
            T Fp[KW];
            if (r == 1) {
#pragma unroll
                for (int k = 0; k < KW; ++k) Fp[k] = F0[k];
            } else if (((r - 1) & 1) == 0) {
                unpark(r - 1, Fp);
            } else {
                T E[KW];
                if (r == 2) {
#pragma unroll
                    for (int k = 0; k < KW; ++k) E[k] = F0[k];
                } else {
                    unpark(r - 2, E);
                }
                T G[KW];
                if ((cw >> (n - (r - 1))) & 1u) {
                    adj_row_in<T, MN, NB>(G, E, qx1, d, r - 1);
                    keep_branch();
                } else {
                    adj_row_in<T, MN, NB>(G, E, qx0, d, r - 1);
                }
                if (GEN) adj_mask<T, KW>(G, cmask);
#pragma unroll
                for (int k = 0; k < KW; ++k) {
                    T v = G[k];
#pragma unroll
                    for (int t = 1; t <= IM; ++t)
                        if (t <= k) v += apow[t] * G[k - t];
                    Fp[k] = v;
                }
                if (GEN) adj_mask<T, KW>(Fp, cmask);
            }
            const bool xb = (cw >> (n - r)) & 1u;
            // the adjoint of the row before its corridor mask
            if (GEN) adj_mask<T, KW>(Fb, cmask);
            T Gb[KW];
            if (r == n) {
#pragma unroll
                for (int k = 0; k < KW; ++k) Gb[k] = Fb[k];
            } else {
#pragma unroll
                for (int k = 0; k < KW; ++k) {
                    T v = Fb[k];
#pragma unroll
                    for (int t = 1; t <= IM; ++t)
                        if (k + t < KW) v += apow[t] * Fb[k + t];
                    Gb[k] = v;
                }
                // G_r was masked before its insertion runs
                if (GEN) adj_mask<T, KW>(Gb, cmask);
                if constexpr (SA) {
                    // G_r recomputed from F_{r-1} for the insertion-weight term
                    T G[KW];
                    if (xb) {
                        adj_row_in<T, MN, NB>(G, Fp, qx1, d, r);
                        keep_branch();
                    } else {
                        adj_row_in<T, MN, NB>(G, Fp, qx0, d, r);
                    }
                    if (GEN) adj_mask<T, KW>(G, cmask);
#pragma unroll
                    for (int k = 0; k < KW; ++k) {
                        T u = T(0);
#pragma unroll
                        for (int t = 1; t <= IM; ++t)
                            if (t <= k) u += dapow[t] * G[k - t];
                        sa += Fb[k] * u;
                    }
                }
            }
#pragma unroll
            for (int k = 0; k + 1 < KW; ++k) sd += Gb[k] * Fp[k + 1];
            // diagonal moves into row r and the adjoint of F_{r-1}
            auto back = [&](const T(&qx)[NB], T(&P)[NB]) {
#pragma unroll
                for (int k = 0; k < KW; ++k) {
                    const int b = r + k - MN - 1;
                    if (b >= 0) P[b] += Gb[k] * Fp[k];
                }
#pragma unroll
                for (int k = 0; k < KW; ++k) {
                    const int b = r + k - MN - 1;
                    T v = (b >= 0) ? qx[b] * Gb[k] : T(0);
                    if (k >= 1) v += d * Gb[k - 1];
                    Fb[k] = v;
                }
            };
            if (xb) {
                back(qx1, P1);
                keep_branch();
            } else {
                back(qx0, P0);
            }
        }
        if constexpr (SA) {
            // row 0: F_0[k] = a^(k - MN) for 1 <= k - MN <= I
            if (GEN) adj_mask<T, KW>(Fb, cmask);
#pragma unroll
            for (int k = 0; k < KW; ++k) {
                const int dl = k - MN;
                if (dl >= 1 && dl <= IM) sa += Fb[k] * dapow[dl];
            }
            ga += (double)sa;
        }
        // received bit equal to / different from the codeword bit
        T se = T(0), sn = T(0);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const bool one = (win >> b) & 1u;
            se += one ? P1[b] : P0[b];
            sn += one ? P0[b] : P1[b];
        }
        gd += (double)sd;
        g1 += (double)se;
        g0 += (double)sn;
    }
    ga = wave_sum(ga);
    gd = wave_sum(gd);
    g1 = wave_sum(g1);
    g0 = wave_sum(g0);
    if (lane == 0) {
        double *o = f.gacc + ((size_t)(w.item >> 6) * f.dsplit + chunk) * 4;
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

template <int MN>
static hipError_t wadj_mn(int uniform, int percol, const FrameDesc *fd, const Work *tab,
                          int nblocks, hipStream_t st) {
    if (percol) {
        if (uniform)
            hipLaunchKernelGGL((k_wadj_col<ADJ_T, MN, true>), dim3(nblocks), dim3(64), 0, st, fd,
                               tab);
        else
            hipLaunchKernelGGL((k_wadj_col<ADJ_T, MN, false>), dim3(nblocks), dim3(64), 0, st,
                               fd, tab);
    } else if (uniform) {
        hipLaunchKernelGGL((k_wadj<ADJ_T, MN, true>), dim3(nblocks), dim3(64), 0, st, fd, tab);
    } else {
        hipLaunchKernelGGL((k_wadj<ADJ_T, MN, false>), dim3(nblocks), dim3(64), 0, st, fd, tab);
    }
    return hipGetLastError();
}

hipError_t ADJ_CAT(ADJ_FN, _w)(int mn, int uniform, int percol, const FrameDesc *fd,
                               const Work *tab, int nblocks, hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    switch (mn) {
        case 0: return wadj_mn<0>(uniform, percol, fd, tab, nblocks, st);
        case 1: return wadj_mn<1>(uniform, percol, fd, tab, nblocks, st);
        case 2: return wadj_mn<2>(uniform, percol, fd, tab, nblocks, st);
        case 3: return wadj_mn<3>(uniform, percol, fd, tab, nblocks, st);
        case 4: return wadj_mn<4>(uniform, percol, fd, tab, nblocks, st);
        case 5: return wadj_mn<5>(uniform, percol, fd, tab, nblocks, st);
        case 6: return wadj_mn<6>(uniform, percol, fd, tab, nblocks, st);
        case 7: return wadj_mn<7>(uniform, percol, fd, tab, nblocks, st);
        case 8: return wadj_mn<8>(uniform, percol, fd, tab, nblocks, st);
        default: return hipErrorInvalidValue;
    }
}

template <int MN, int IM, bool SA, bool PC>
static hipError_t adj_launch(const FrameDesc *fd, const Work *tab, int nblocks, size_t lds,
                             hipStream_t st) {
    auto kern = k_adjoint<ADJ_T, MN, IM, SA, PC>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)kern,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(64), lds, st, fd, tab);
    return hipGetLastError();
}

template <int MN, bool PC>
static hipError_t adj_mn(int imode, int sa, const FrameDesc *fd, const Work *tab, int nblocks,
                         size_t lds, hipStream_t st) {
    constexpr int IM2 = (2 < 2 * MN) ? 2 : 2 * MN;
    if (imode == 0)
        return sa ? adj_launch<MN, IM2, true, PC>(fd, tab, nblocks, lds, st)
                  : adj_launch<MN, IM2, false, PC>(fd, tab, nblocks, lds, st);
    return sa ? adj_launch<MN, 2 * MN, true, PC>(fd, tab, nblocks, lds, st)
              : adj_launch<MN, 2 * MN, false, PC>(fd, tab, nblocks, lds, st);
}

template <bool PC>
static hipError_t adj_pc(int mn, int imode, int sa, const FrameDesc *fd, const Work *tab,
                         int nblocks, size_t lds, hipStream_t st) {
    switch (mn) {
        case 0: return adj_mn<0, PC>(imode, sa, fd, tab, nblocks, lds, st);
        case 1: return adj_mn<1, PC>(imode, sa, fd, tab, nblocks, lds, st);
        case 2: return adj_mn<2, PC>(imode, sa, fd, tab, nblocks, lds, st);
        case 3: return adj_mn<3, PC>(imode, sa, fd, tab, nblocks, lds, st);
        case 4: return adj_mn<4, PC>(imode, sa, fd, tab, nblocks, lds, st);
        case 5: return adj_mn<5, PC>(imode, sa, fd, tab, nblocks, lds, st);
        case 6: return adj_mn<6, PC>(imode, sa, fd, tab, nblocks, lds, st);
        case 7: return adj_mn<7, PC>(imode, sa, fd, tab, nblocks, lds, st);
        case 8: return adj_mn<8, PC>(imode, sa, fd, tab, nblocks, lds, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t ADJ_CAT(ADJ_FN, _lattice)(int mn, int imode, int sa, int gen, const FrameDesc *fd,
                                     const Work *tab, int nblocks, size_t lds, hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    return gen ? adj_pc<true>(mn, imode, sa, fd, tab, nblocks, lds, st)
                  : adj_pc<false>(mn, imode, sa, fd, tab, nblocks, lds, st);
}

}  // namespace mapdec
