// Forward/backward recursions for uniform priors (eqs. 4, 5, 11, 12), where
// Gamma depends on the start index s = n i + m' only.
//
// This file is compiled once per (precision, waves, states per thread):
// build with -DCHAIN_T=float|double -DCHAIN_NW=<waves> -DCHAIN_SPL=<states>
// -DCHAIN_FN=<launcher name>.
//
// One workgroup of nt = 64 nw threads runs one chain, nw the waves the
// state space needs (at most the compiled NW, NT = 64 NW): a step's issue
// time grows with the waves that share a SIMD, so none are launched only to
// hold zeros.  Thread t owns drift-state index t (SPL = 1) or SPL of them:
// the adjacent indices SPL t .. SPL t + SPL - 1 (FP32 Gamma) or t, t + nt,
// .. (FP64).  Rows are padded to NT SPL states (zero beyond 2M+1) plus mn
// zeros on each side, so no thread branches on its state.  One workgroup
// barrier per step.
//
// Rows are FP64 at every precision (their spread within a row can exceed
// the FP32 range); Gamma stays in the batch precision.  Each step scales its
// new row by a power of two, 2^-e, so that the rows' sums stay near
// 2^kRowExp (far above 1: the entries that matter on long noisy frames can
// lie a thousand binary orders below a row's largest, and the FP64 range
// below the row then holds them; the largest entries keep a margin of
// hundreds of orders below the FP64 maximum): the
// normalisation of eqs. 11-12 up to a scale factor, which every consumer of
// the rows (APP, adjoint) is invariant to, applied exactly (no rounding) and
// accounted exactly: log P(y) = (sum of the e) ln 2 + log alpha_N(rho - tau)
// for the stored (scaled) last row.  The sum of the input row is not known
// when the step starts: only the binary exponent m of the sum of the row
// before it is (every thread adds that sum's wave partials; the partials of
// the input row, whose values each thread still holds from writing them,
// are reduced with DPP moves during the step, so no reduction and no
// division sits on the path from one barrier to the next).  The step
// predicts the input row's exponent from m, the exponents it applied to the
// last two rows and the growth measured between the two rows before, and
// takes e = prediction + that growth - kRowExp: the stored rows' exponents
// then stay within the step-to-step change of the growth (a sum of two such
// differences) of kRowExp, however long the chain; feeding m back alone
// would let them drift without bound.  beta is handled the same way from the other
// end.  A zero sum (no path) leaves the rows zero and is reported after the
// chain.
// A chain covers the symbols [i0, i1) of its frame's segment: it starts from
// the row the descriptor gives (a checkpoint) or from the boundary state,
// continues the cumulative log of the normalisers, and can copy its last
// row out (the next checkpoint).
//
// With general priors Gamma_i(m', delta) depends on the symbol too; its
// table holds the states of consecutive symbols one after the other, so
// "column" Mt i + m' + M plays the part of s and step i reads the Mt columns
// from Mt i on: the same ring, with Mt columns per step instead of n.
//
// Gamma(s, delta) for the start indices a chunk of C steps reads sits in an
// LDS ring of RING (a power of two) slots of Mn values each, slot-major
// (threads read with a stride of Mn words, which is odd: no bank conflicts).
// For small state spaces the slots near both ends are duplicated past the
// ends, so one step's reads never wrap and every read is a base register
// plus a compile-time offset; large state spaces mask one base slot per
// state and step and repeat the ring's first 2 mn slots past its end, so
// their reads are a base plus compile-time offsets too.
// The n C columns the next chunk adds are loaded into registers one chunk
// ahead and written to the ring when that chunk starts, so global-memory
// latency overlaps a whole chunk of steps.
#include "device_common.h"

#if !defined(CHAIN_T) || !defined(CHAIN_NW) || !defined(CHAIN_SPL) || !defined(CHAIN_FN)
#error "compile with -DCHAIN_T, -DCHAIN_NW, -DCHAIN_SPL and -DCHAIN_FN"
#endif
// CHAIN_ONEROW=1: one metric row in LDS, read and then overwritten in place
// (a second barrier per step), for state spaces whose two rows and ring
// would not fit in LDS together.
#ifndef CHAIN_ONEROW
#define CHAIN_ONEROW 0
#endif

namespace mapdec {

constexpr int kRowExp = 640;   // binary exponent the stored rows' sums are held near

// ONE (one metric row) is a template parameter, not only a macro, so the
// one-row and two-row objects built from this file never define the same
// kernel symbol.
template <typename T, int NW, int SPL, int MN, int DIR, bool ONE>
__device__ __forceinline__ void chain_ring_body(const FrameDesc &f, unsigned char *smem) {
    constexpr int NT = 64 * NW;
    constexpr int Mn = 2 * MN + 1;
    constexpr int ROWW = NT * SPL + 2 * MN;            // padded row
    constexpr bool DUP = ring_duplicates(NT * SPL);
    constexpr int PF = ring_prefetch_regs(NW, sizeof(T));
    const int Mt = f.Mt, M = f.M, N = f.N;
    const int i0 = f.i0, i1 = f.i1, NS = i1 - i0;
    // column of state m at step i: n i + m (uniform priors: the start index)
    // or Mt i + m + M (general priors); the table holds columns [s0, s1]
    const bool uni = f.uniform != 0 && !f.percol;
    const int n = uni ? f.n : Mt;
    const int MC = uni ? M : 0;
    const int s0 = uni ? f.s0 : Mt * i0;
    const int s1 = uni ? f.s1 : Mt * i1 - 1;
    // columns the chain's rows read (its chunks load up to C - 1 steps
    // more): loads outside them take 0, so a chain never depends on table
    // columns beyond its own rows (a sweep part runs beside the pre-pass
    // rounds that write the later columns)
    const int ld_lo = min(max(s0, n * i0 - MC), s1);
    const int ld_hi = max(min(s1, n * (i1 - 1) - MC + Mt - 1), ld_lo);
    const int C = f.ring_chunk, RING = f.ring_cols, mask = RING - 1;
    const int RPHYS = DUP ? RING + NT * SPL + 2 * MN : RING + 2 * MN;
    using R = double;                                  // metric rows: FP64 always
    R *row0 = (R *)smem;
    R *row1 = ONE ? row0 : row0 + ROWW;
    R *part = row1 + ROWW;                             // [2][NW] wave partial sums
    R *red = part + 2 * NW;                            // [NW] partial sums of a new row
    T *ring = (T *)(part + 3 * NW);                    // [RPHYS][Mn], batch precision
    // the launch's threads: nt = 64 nw <= NT (as many waves as the state
    // space needs)
    const int tid = threadIdx.x, wv = tid >> 6, nt = blockDim.x, nw = nt >> 6;
    // drift-state index of the thread's j-th state: with several states per
    // thread (FP32 Gamma) they are adjacent (SPL tid + j), so the row windows
    // of a thread's states overlap and pair up in LDS reads; FP64 Gamma keeps
    // them nt apart (fewer live registers)
    constexpr bool ADJ = SPL > 1 && sizeof(T) == 4;
    auto state = [&](int j) { return ADJ ? SPL * tid + j : tid + nt * j; };
    const gptr<const T> G = to_global((const T *)f.G);   // [Mn][gsp]
    const size_t sp = (size_t)f.gsp;

    for (int j = tid; j < (ONE ? 1 : 2) * ROWW + 3 * NW; j += nt) row0[j] = R(0);
    for (int j = tid; j < RPHYS * Mn; j += nt) ring[j] = T(0);
    __syncthreads();
    const int m0 = DIR == 0 ? 0 : f.rho - f.tau;
    const double *init = DIR == 0 ? f.a_init : f.b_init;
    const gptr<R> out = to_global(DIR == 0 ? f.alpha : f.beta);
    const int rowA = DIR == 0 ? i0 : i1;
    // a boundary prior's entries whose received position (m at the start,
    // tau + m at the end) lies outside [0, rho] carry no path: zero, so that
    // no later kernel pairs them with a clamped start index
    const bool prior_row = init && (DIR == 0 ? i0 == 0 : i1 == N);
    const int pos0 = DIR == 0 ? 0 : f.tau;
    // where row r goes (sweep: checkpoints only), and whether the starting
    // row is stored
    const int mode = f.chain_mode, cks = f.ck_stride;
    auto stored = [&](int r) { return mode != kChainSweep || r % cks == 0; };
    auto slot = [&](int r) { return (size_t)(mode == kChainSweep ? r / cks : r - i0) * Mt; };
    // a sweep part after the first starts from the checkpoint the previous
    // part wrote, which main passes may be reading already: not rewritten
    const bool resumed = mode == kChainSweep && (DIR == 0 ? i0 > 0 : i1 < N);
    const bool put_init = mode == kChainSub ? ((f.wr_init >> DIR) & 1) != 0
                                            : stored(rowA) && !resumed;
    // drift states kept (asymmetric limits): indices [lo_i, hi_i]
    const int lo_i = f.lim_lo + M, hi_i = f.lim_hi + M;
    // path thresholds: the forward chain over the frame decides which
    // states are kept (decide), every other chain applies its decisions
    const bool pr = f.theta > 0.0;
    const bool decide = pr && DIR == 0 && mode != kChainSub;
    const gptr<uint8_t> kept = to_global(f.kept);
    for (int mi = tid; mi < Mt; mi += nt) {
        R v = init ? (R)init[mi] : ((mi == m0 + M) ? R(1) : R(0));
        if (prior_row && (pos0 + mi - M < 0 || pos0 + mi - M > f.rho)) v = R(0);
        if (mi < lo_i || mi > hi_i) v = R(0);
        if (pr && !decide && !kept[(size_t)rowA * Mt + mi]) v = R(0);
        row0[MN + mi] = v;
    }
    if (decide) {   // the start row against its own sum
        __syncthreads();
        R t = R(0);
        for (int mi = tid; mi < Mt; mi += nt) t += row0[MN + mi];
        t = wave_sum_dpp(t);
        if ((tid & 63) == 0) red[wv] = t;
        __syncthreads();
        R sum = R(0);
        for (int w = 0; w < nw; ++w) sum += red[w];
        const R cut = (R)f.theta * sum;
        for (int mi = tid; mi < Mt; mi += nt) {
            const R v = row0[MN + mi];
            const bool k = v > R(0) && !(v < cut);
            row0[MN + mi] = k ? v : R(0);
            kept[(size_t)rowA * Mt + mi] = k ? 1 : 0;
        }
    }
    if (put_init)
        for (int mi = tid; mi < Mt; mi += nt) out[slot(rowA) + mi] = row0[MN + mi];
    double *logX = DIR == 0 ? f.logA : f.logB;
    // A sweep in parts carries its row-scale predictor from part to part
    // (f.sweep_state, per direction: the stale sum the next step reads, the
    // predictor's three exponents and the exponent total), so the parts
    // apply the scales the sweep in one launch would, and their logs are the
    // same bits.
    double *sst = mode == kChainSweep && f.sweep_state ? f.sweep_state + 8 * DIR : nullptr;
    const bool resume = sst && resumed;
    const bool suspend = sst && (DIR == 0 ? i1 < N : i0 > 0);
    const double lbase =
        (!resume && mode != kChainSub && (DIR == 0 ? i0 > 0 : i1 < N)) ? logX[rowA] : 0.0;

    // chunk k covers steps i0+kC .. i0+kC+C-1 (forward) or i1-1-kC down to
    // i1-C-kC (backward), which read s in [n i_lo - M, n i_hi + M]
    auto chunk_lo_s = [&](int k) { return n * (DIR == 0 ? i0 + k * C : i1 - C - k * C) - MC; };
    auto chunk_hi_s = [&](int k) {
        return n * (DIR == 0 ? i0 + k * C + C - 1 : i1 - 1 - k * C) - MC + Mt - 1;
    };
    auto new_base = [&](int k) { return DIR == 0 ? chunk_hi_s(k - 1) + 1 : chunk_lo_s(k); };

    auto put = [&](int s, int kk, T v) {
        const int L = s & mask;
        if (DUP) {
            ring[(L + MN) * Mn + kk] = v;
            if (L < NT * SPL + MN) ring[(L + RING + MN) * Mn + kk] = v;
            if (L >= RING - MN) ring[(L - RING + MN) * Mn + kk] = v;
        } else {
            ring[L * Mn + kk] = v;
            if (L < 2 * MN) ring[(L + RING) * Mn + kk] = v;
        }
    };

    // Prefetch registers: element p = tid + nt r is column base + (p mod nC)
    // of drift change p / nC.  (kk, col) advance by (nt / nC, nt mod nC)
    // per register with one carry test; loads are unconditional (clamped
    // address) so all of them stay in flight, validity kept as a bit mask.
    const int nC = n * C;
    const int dq = nt / nC, dr = nt - dq * nC;
    T pre[PF];
    uint32_t pvalid = 0;
    auto issue = [&](int base) {
        int kk = tid / nC, col = tid - kk * nC;
        pvalid = 0;
#pragma unroll
        for (int r = 0; r < PF; ++r) {
            const int s = base + col;
            const int sc = min(max(s, ld_lo), ld_hi);   // inside the table [s0, s1]
            const int kc = min(kk, Mn - 1);
            pre[r] = G[(size_t)kc * sp + (sc - s0)];
            pvalid |= (s == sc) ? (1u << r) : 0u;
            col += dr;
            kk += dq;
            const bool carry = col >= nC;
            col -= carry ? nC : 0;
            kk += carry ? 1 : 0;
        }
    };
    auto commit = [&](int base, int lo, int hi) {   // columns in [lo, hi] only
        int kk = tid / nC, col = tid - kk * nC;
#pragma unroll
        for (int r = 0; r < PF; ++r) {
            const int s = base + col;
            if (kk < Mn && s >= lo && s <= hi) put(s, kk, ((pvalid >> r) & 1u) ? pre[r] : T(0));
            col += dr;
            kk += dq;
            const bool carry = col >= nC;
            col -= carry ? nC : 0;
            kk += carry ? 1 : 0;
        }
    };
    {   // chunk 0's window, nC columns at a time
        const int lo = chunk_lo_s(0), hi = chunk_hi_s(0);
        for (int base = lo; base <= hi; base += nC) {
            issue(base);
            commit(base, lo, hi);
        }
    }
    const int nchunks = (NS + C - 1) / C;
    if (nchunks > 1) issue(new_base(1));

    R *cur = row0, *nxt = row1;
    R own[SPL];
    __syncthreads();
    {
        R p = R(0);
#pragma unroll
        for (int j = 0; j < SPL; ++j) {
            own[j] = cur[MN + state(j)];
            p += own[j];
        }
        p = wave_sum_dpp(p);
        if ((tid & 63) == 0) part[wv] = p;   // stands in for the row before the first
    }
    __syncthreads();
    int pp = 0;      // partial-sum buffer read this step (the row before the input row)
    long long lexp = 0;   // sum of the scale exponents applied so far
    // exponent of the previous step's measured sum, exponents applied one and
    // two steps ago; first: the step has no earlier measurement
    int m2 = 0, u1 = 0, u2 = 0;
    bool first = true;
    if (resume) {   // where the previous part stopped
        m2 = (int)sst[1];
        u1 = (int)sst[2];
        u2 = (int)sst[3];
        lexp = (long long)sst[4];
        first = false;
        // the stale sum as the first step's partials (plus exact zeros)
        if (tid < NW) part[tid] = tid == 0 ? sst[0] : R(0);
        __syncthreads();
    }
    bool dead = false;
    // applied decisions of the rows KPF steps ahead, loaded that early so
    // that their latency stays off the step (kq[0] is this step's row)
    constexpr int KPF = 4;
    uint32_t kq[KPF][SPL];
    auto krow = [&](int g) { return DIR == 0 ? i0 + g + 1 : i1 - 1 - g; };   // row of step g
    auto kload = [&](uint32_t(&dst)[SPL], int g) {
        const int r = krow(g);
        const bool in = g < NS;
#pragma unroll
        for (int j = 0; j < SPL; ++j) {
            const int mi = min(state(j), Mt - 1);
            dst[j] = in ? kept[(size_t)(in ? r : 0) * Mt + mi] : 0u;
        }
    };
    if (pr && !decide) {
#pragma unroll
        for (int d = 0; d < KPF; ++d) kload(kq[d], d);
    }
    int gs = 0;   // steps done
    for (int k = 0; k < nchunks && !dead; ++k) {
        if (k >= 1) {
            const int b = new_base(k);
            commit(b, b, b + nC - 1);
            if (k + 1 < nchunks) issue(new_base(k + 1));
            __syncthreads();
        }
        const int steps = min(C, NS - k * C);
        for (int t = 0; t < steps; ++t) {
            const int i = DIR == 0 ? i0 + k * C + t : i1 - 1 - k * C - t;
            R csum = R(0);
#pragma unroll
            // (partials of waves not launched stay 0 from the start: the
            // loop keeps its compile-time trip count and its loads issue
            // together)
            for (int w = 0; w < NW; ++w) csum += part[pp * NW + w];
            dead |= !(csum > R(0));
            int m1;
            (void)frexp(csum, &m1);   // binary exponent of the sum of the row before the input
            if (first) m2 = m1;
            first = false;
            const int g = m1 - m2 + u2;         // growth measured between those two rows
            const int rin = m1 + g - u1;        // predicted exponent of the input row's sum
            // a zero (dead) or denormal sum keeps the scale finite
            const int e = min(max(rin + g - kRowExp, -1000), 1000);
            m2 = m1;
            u2 = u1;
            u1 = e;
            const R scl = ldexp(R(1), -e);
            lexp += e;
            const int sb = (n * i - MC) & mask;
            const R *cb = cur + MN;
            // ring slot of the thread's state j at drift change x - MN: forward
            // (column sb + state - x + MN) gb[j] + 2 mn - x, backward (column
            // sb + state) gb[j]; without the duplicated ring the base is
            // masked once per state and the first 2 mn slots are repeated past
            // the end, so every read is the base plus a compile-time offset
            int gb[SPL];
#pragma unroll
            for (int j = 0; j < SPL; ++j)
                gb[j] = DUP ? 0 : (sb + state(j) - (DIR == 0 ? MN : 0)) & mask;
            // Gamma(column, delta) for the thread's state j and drift change x - MN
            auto gam = [&](int j, int x) -> R {
                if (DUP) {
                    const int c = DIR == 0 ? sb + state(j) - (x - MN) : sb + state(j);
                    return (R)ring[(c + MN) * Mn + x];
                }
                return (R)ring[(gb[j] + (DIR == 0 ? 2 * MN - x : 0)) * Mn + x];
            };
            // the row value that meets it
            auto rowv = [&](int j, int x) -> R {
                return DIR == 0 ? cb[state(j) - (x - MN)] : cb[state(j) + x - MN];
            };
            auto partial = [&]() {   // partial sum of the input row, for the next step
                R p = R(0);
#pragma unroll
                for (int j = 0; j < SPL; ++j) p += own[j];
                p = wave_sum_dpp(p);
                if ((tid & 63) == 0) part[(pp ^ 1) * NW + wv] = p;
            };
            // alpha'_{i+1}(m) = sum_delta alpha_i(m - delta) Gamma(n i + m - delta, delta)
            // beta'_i(m) = sum_delta Gamma(n i + m, delta) beta_{i+1}(m + delta)
            // (two partial sums over delta halve the dependent FMA chain)
            R acc[SPL];
            if constexpr (SPL == 1) {
                // operands loaded first, so the partial sum's reduction (a
                // block of its own: one lane writes) overlaps their latency
                R rv[Mn], gv[Mn];
#pragma unroll
                for (int x = 0; x < Mn; ++x) {
                    rv[x] = rowv(0, x);
                    gv[x] = gam(0, x);
                }
                partial();
                R a0 = R(0), a1 = R(0);
#pragma unroll
                for (int x = 0; x < Mn; ++x) {
                    if (x & 1) a1 += rv[x] * gv[x]; else a0 += rv[x] * gv[x];
                }
                acc[0] = a0 + a1;
            } else {
                partial();
#pragma unroll
                for (int j = 0; j < SPL; ++j) {
                    R a0 = R(0), a1 = R(0);
#pragma unroll
                    for (int x = 0; x < Mn; ++x) {
                        if (x & 1) a1 += rowv(j, x) * gam(j, x); else a0 += rowv(j, x) * gam(j, x);
                    }
                    acc[j] = a0 + a1;
                }
            }
            const int row = DIR == 0 ? i + 1 : i;
            if (decide) {
                // the new row's sum (its scale is that of acc), then the
                // states below theta times it are not pursued
                R t = R(0);
#pragma unroll
                for (int j = 0; j < SPL; ++j) {
                    const int mi = state(j);
                    t += (mi >= lo_i && mi <= hi_i) ? acc[j] : R(0);
                }
                t = wave_sum_dpp(t);
                if ((tid & 63) == 0) red[wv] = t;
                __syncthreads();
                R sum = R(0);
#pragma unroll
                for (int w = 0; w < NW; ++w) sum += red[w];
                const R cut = (R)f.theta * sum;
#pragma unroll
                for (int j = 0; j < SPL; ++j) {
                    const int mi = state(j);
                    const bool k = mi >= lo_i && mi <= hi_i && acc[j] > R(0) && !(acc[j] < cut);
                    acc[j] = k ? acc[j] : R(0);
                    if (mi < Mt) kept[(size_t)row * Mt + mi] = k ? 1 : 0;
                }
            } else if (pr) {
#pragma unroll
                for (int j = 0; j < SPL; ++j) acc[j] = kq[0][j] ? acc[j] : R(0);
#pragma unroll
                for (int d = 0; d + 1 < KPF; ++d)
#pragma unroll
                    for (int j = 0; j < SPL; ++j) kq[d][j] = kq[d + 1][j];
                kload(kq[KPF - 1], gs + KPF);
            }
            ++gs;
            if (ONE) __syncthreads();   // every read of the row is done
            R *nb = nxt + MN;
            const bool st_row = stored(row);
            const size_t ro = slot(row);
#pragma unroll
            for (int j = 0; j < SPL; ++j) {
                const int mi = state(j);
                const R v = (mi >= lo_i && mi <= hi_i) ? acc[j] * scl : R(0);
                own[j] = v;
                nb[mi] = v;
                if (mi < Mt && st_row) out[ro + mi] = v;
            }
            // the sweep keeps each checkpoint's cumulative log for the
            // recomputations that start from it
            if (mode == kChainSweep && st_row && tid == 0)
                logX[row] = lbase + (double)lexp * 0.69314718055994530942;
            pp ^= 1;
            R *tmp = cur;
            cur = nxt;
            nxt = tmp;
            __syncthreads();
        }
    }
    const double lsum = lbase + (double)lexp * 0.69314718055994530942;
    if (suspend && !dead && tid == 0) {
        R c = R(0);   // the sum the next step would read, summed as it would
        for (int w = 0; w < NW; ++w) c += part[pp * NW + w];
        sst[0] = c;
        sst[1] = m2;
        sst[2] = u1;
        sst[3] = u2;
        sst[4] = (double)lexp;
    }
    if (dead) {
        if (tid == 0) {
            atomicOr(f.status, kStatusNoPath);
            if (DIR == 0) *f.logp = -INFINITY;
        }
        return;
    }
    double *fin = DIR == 0 ? f.a_fin : f.b_fin;
    if (fin)
        for (int mi = tid; mi < Mt; mi += nt) fin[mi] = cur[MN + mi];
    if (tid != 0 || mode == kChainSub) return;
    logX[DIR == 0 ? i1 : i0] = lsum;
    if (DIR == 1 && i0 == 0 && f.grad && f.start_prior) {
        // posterior mean of the start drift (prior entries outside [0, rho]
        // carry no path), for the path-count identity of the adjoint
        R b0 = R(0), b0m = R(0);
        for (int mi = 0; mi < Mt; ++mi) {
            if (mi - M < 0 || mi - M > f.rho) continue;
            const R v = cur[MN + mi] * (R)f.start_prior[mi];
            b0 += v;
            b0m += v * (R)(mi - M);
        }
        // written on every run, so that no earlier run's value is read
        f.gacc_all[4 * (size_t)f.gacc_n + 1] = b0 > R(0) ? b0m / b0 : R(0);
    }
    if (DIR == 0 && i1 == N) {
        // P(y) = alpha_N(rho - tau), or sum_m alpha_N(m) end_prior(m), in
        // the row's scale
        R aN = R(0), aNm = R(0);
        if (f.end_prior) {
            for (int mi = 0; mi < Mt; ++mi) {
                const R v = cur[MN + mi] * (R)f.end_prior[mi];
                aN += v;
                aNm += v * (R)(mi - M);
            }
            // posterior mean of the end drift, for the path-count identity
            // of the adjoint
            if (f.grad) f.gacc_all[4 * (size_t)f.gacc_n] = aN > R(0) ? aNm / aN : R(0);
        } else {
            aN = cur[MN + (f.rho - f.tau) + M];
        }
        if (!(aN > R(0))) {
            atomicOr(f.status, kStatusNoPath);
            *f.logp = -INFINITY;
        } else {
            *f.logp = lsum + log(aN);
        }
    }
}

// dirs: 1 forward only, 2 backward only, 3 both (workgroups 2c, 2c+1)
template <typename T, int NW, int SPL, int MN, bool ONE>
__global__ __launch_bounds__(64 * NW) void k_chain_ring(const FrameDesc *__restrict__ fd,
                                                        const int *__restrict__ frames,
                                                        int dirs) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int nd = dirs == 3 ? 2 : 1;
    const FrameDesc &f = fd[frames[blockIdx.x / nd]];
    if (*f.status != kStatusOk) return;
    const int dir = nd == 2 ? (int)(blockIdx.x & 1) : (dirs == 1 ? 0 : 1);
    if (dir)
        chain_ring_body<T, NW, SPL, MN, 1, ONE>(f, smem);
    else
        chain_ring_body<T, NW, SPL, MN, 0, ONE>(f, smem);
}

template <int MN>
static hipError_t ring_launch(int waves, int nchains, int dirs, size_t lds, hipStream_t st,
                              const FrameDesc *fd, const int *frames) {
    auto kern = k_chain_ring<CHAIN_T, CHAIN_NW, CHAIN_SPL, MN, CHAIN_ONEROW != 0>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)kern,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(nchains * (dirs == 3 ? 2 : 1)), dim3(64 * waves), lds, st,
                       fd, frames, dirs);
    return hipGetLastError();
}

hipError_t CHAIN_FN(int mn, int waves, int nchains, int dirs, size_t lds, hipStream_t st,
                    const FrameDesc *fd, const int *frames) {
    switch (mn) {
        case 0: return ring_launch<0>(waves, nchains, dirs, lds, st, fd, frames);
        case 1: return ring_launch<1>(waves, nchains, dirs, lds, st, fd, frames);
        case 2: return ring_launch<2>(waves, nchains, dirs, lds, st, fd, frames);
        case 3: return ring_launch<3>(waves, nchains, dirs, lds, st, fd, frames);
        case 4: return ring_launch<4>(waves, nchains, dirs, lds, st, fd, frames);
        case 5: return ring_launch<5>(waves, nchains, dirs, lds, st, fd, frames);
        case 6: return ring_launch<6>(waves, nchains, dirs, lds, st, fd, frames);
        case 7: return ring_launch<7>(waves, nchains, dirs, lds, st, fd, frames);
        case 8: return ring_launch<8>(waves, nchains, dirs, lds, st, fd, frames);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace mapdec
