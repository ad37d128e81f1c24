// Receiver-metric lattice kernel (eqs. 7-10).
#include "device_common.h"

namespace mapdec {

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
// per lane (qx0 for a 0 codeword bit, qx1 for a 1), so a node costs a select,
// one multiply and 1 + IM fused multiply-adds.

// G_r from F_{r-1}.  The codeword bit xb is wave-uniform; each node takes its
// Q by a select on it (one copy of the row code: two copies behind a branch
// cost a register merge of the whole row at every join).
template <typename T, int MN, int NB>
__device__ __forceinline__ void lattice_row_in(T (&G)[2 * MN + 1], const T (&F)[2 * MN + 1],
                                               const T (&qx0)[NB], const T (&qx1)[NB], bool xb,
                                               T d, int r) {
#pragma unroll
    for (int k = 0; k < 2 * MN + 1; ++k) {
        T v = (k + 1 < 2 * MN + 1) ? d * F[k + 1] : T(0);
        const int b = r + k - MN - 1;
        if (b >= 0) v += blend(xb, qx1[b], qx0[b]) * F[k];
        G[k] = v;
    }
}

// Zeroes the corridor coordinates outside the frame's corridor (asymmetric
// limits), before a row's insertion runs and after them; cmask is
// wave-uniform, so frames with the full corridor skip it on one scalar
// compare.
template <typename T, int KW>
__device__ __forceinline__ void corridor_mask(T (&F)[KW], uint32_t cmask) {
    if (cmask != (1u << KW) - 1u) {
#pragma unroll
        for (int k = 0; k < KW; ++k) F[k] = ((cmask >> k) & 1u) ? F[k] : T(0);
    }
}

// GEN: the general scheme's instance (frames with a codebook per symbol
// or a narrower corridor); the fixed-code instance has neither.  With
// f.percol, one lattice per (symbol i, drift state m', D) with codeword
// C_i(D) (a codebook per symbol position); the lane's column c = (i - i0)
// Mt + m' + M, start index s = n i + m'.  Else one per (s, D), column
// s - s0.
template <typename T, int MN, int IM, bool GEN>
__global__ __launch_bounds__(kLatticeLanes) void k_lattice(const FrameDesc *__restrict__ fd,
                                                           const Work *__restrict__ tab) {
    constexpr int KW = 2 * MN + 1;
    constexpr int NB = kMaxN + MN;   // received positions a lattice can read
    const Work w = tab[blockIdx.x];
    const FrameDesc &f = fd[w.frame];
    const int chunk = w.item & 63;   // codewords [chunk dq, (chunk + 1) dq)
    const int col = (w.item & ~63) + (int)threadIdx.x;   // column of the tables
    const bool PERCOL = GEN && f.percol;
    int s, sym = 0;
    if (PERCOL) {
        if (col >= (f.i1 - f.i0) * f.Mt) return;
        const int di = col / f.Mt;
        sym = f.i0 + di;
        s = f.n * sym + (col - di * f.Mt) - f.M;
    } else {
        s = f.s0 + col;
        if (s > f.s1) return;
    }
    const int n = f.n, q = f.q, rho = f.rho;
    const uint32_t cmask = GEN ? f.cmask : 0xffffffffu;
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

    // received bits y[s .. s+32) of this lane (start indices outside
    // [0, rho] have no valid segment: their R is 0 whatever is read here)
    const bool sok = !PERCOL || (s >= 0 && s <= rho);
    const int sr = PERCOL ? min(max(s, 0), rho) : s;
    const int wi = sr >> 5, sh = sr & 31;
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

    T *R = (T *)f.R;   // NULL: only Gamma is wanted (uniform priors)
    const size_t sp = (size_t)f.sp;
    const int Dlo = chunk * f.dq, Dhi = min(q, Dlo + f.dq);
    for (int D = Dlo; D < Dhi; ++D) {
        // the codeword: wave-uniform with one codebook, the lane's symbol's
        // otherwise
        const uint32_t cw = GEN ? f.cw[(size_t)sym * f.cwi + D]
                                : __builtin_amdgcn_readfirstlane(f.cw[D]);
        T F[KW];
#pragma unroll
        for (int k = 0; k < KW; ++k) {
            const int dl = k - MN;   // row 0: dl insertions before the first bit
            F[k] = (dl >= 0 && dl <= IM) ? apow[dl] : T(0);
        }
        if (GEN) corridor_mask<T, KW>(F, cmask);
#pragma unroll
        for (int r = 1; r <= kMaxN; ++r) {
            if (r > n) continue;   // constant trip count: the loop unrolls
            T G[KW];
            lattice_row_in<T, MN, NB>(G, F, qx0, qx1, (cw >> (n - r)) & 1u, d, r);
            // a node outside the corridor does not exist: no insertion run
            // may start from it (a deletion can reach one below the corridor)
            if (GEN) corridor_mask<T, KW>(G, cmask);
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
            if (GEN) corridor_mask<T, KW>(F, cmask);
        }
        const int rc = PERCOL ? col : s - f.s0;
#pragma unroll
        for (int k = 0; k < KW; ++k) {
            const int len = n + k - MN;   // segment length n + delta
            const T v = (sok && len >= 0 && s + len <= rho) ? F[k] : T(0);
            if (R) R[((size_t)D * KW + k) * sp + rc] = v;
            gsum[k] += v;
        }
    }
    const int gc = PERCOL ? col : s - f.s0;
    if (f.uniform) {
        if (f.dsplit == 1) {
            T *G = (T *)f.G;
            const T invq = T(1) / T(q);
#pragma unroll
            for (int k = 0; k < KW; ++k) G[(size_t)k * f.gsp + gc] = gsum[k] * invq;
        } else {   // this chunk's partial sums; k_gsum adds the chunks
            T *P = (T *)f.Gpart;
#pragma unroll
            for (int k = 0; k < KW; ++k) P[((size_t)chunk * KW + k) * sp + gc] = gsum[k];
        }
    }
}

// ---------------------------------------------------------------------------
// launcher

template <typename T, int MN, bool PC>
static void lattice_mn(int imode, const FrameDesc *fd, const Work *tab, int nblocks,
                       hipStream_t st) {
    constexpr int IM2 = (2 < 2 * MN) ? 2 : 2 * MN;
    if (imode == 0)
        hipLaunchKernelGGL((k_lattice<T, MN, IM2, PC>), dim3(nblocks), dim3(kLatticeLanes), 0,
                           st, fd, tab);
    else
        hipLaunchKernelGGL((k_lattice<T, MN, 2 * MN, PC>), dim3(nblocks), dim3(kLatticeLanes),
                           0, st, fd, tab);
}

template <typename T, bool PC>
static hipError_t lattice_t(int mn, int imode, const FrameDesc *fd, const Work *tab,
                            int nblocks, hipStream_t st) {
    switch (mn) {
        case 0: lattice_mn<T, 0, PC>(imode, fd, tab, nblocks, st); break;
        case 1: lattice_mn<T, 1, PC>(imode, fd, tab, nblocks, st); break;
        case 2: lattice_mn<T, 2, PC>(imode, fd, tab, nblocks, st); break;
        case 3: lattice_mn<T, 3, PC>(imode, fd, tab, nblocks, st); break;
        case 4: lattice_mn<T, 4, PC>(imode, fd, tab, nblocks, st); break;
        case 5: lattice_mn<T, 5, PC>(imode, fd, tab, nblocks, st); break;
        case 6: lattice_mn<T, 6, PC>(imode, fd, tab, nblocks, st); break;
        case 7: lattice_mn<T, 7, PC>(imode, fd, tab, nblocks, st); break;
        case 8: lattice_mn<T, 8, PC>(imode, fd, tab, nblocks, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_lattice(int fp64, int mn, int imode, int gen, const FrameDesc *fd,
                          const Work *tab, int nblocks, hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    if (gen)
        return fp64 ? lattice_t<double, true>(mn, imode, fd, tab, nblocks, st)
                    : lattice_t<float, true>(mn, imode, fd, tab, nblocks, st);
    return fp64 ? lattice_t<double, false>(mn, imode, fd, tab, nblocks, st)
                : lattice_t<float, false>(mn, imode, fd, tab, nblocks, st);
}

}  // namespace mapdec
