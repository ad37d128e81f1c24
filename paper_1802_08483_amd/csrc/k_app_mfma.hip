// APP (eqs. 1-3) as matrix products on the MFMA units, FP32 batches with one
// codebook.
//
// For a block of TB = 64 consecutive symbols i0 .. i0+63 of a frame, the
// start indices they reach are s = s_lo + c, c in [0, span), s_lo = n i0 -
// M, span = n (TB - 1) + Mt.  With the pair index (c, k) (k = delta + mn),
//   U_i(D) = sum_{c, k} K_i(c, k) R(s_lo + c, D, k),
//   K_i(c, k) = alpha_i(m') beta_{i+1}(m' + k - mn) 2^-E_i,  m' = s - n i,
// zero where m' or m' + k - mn leaves [-M, M]: a product of the TB x (span
// Mn) matrix K with the (span Mn) x q matrix R, which v_mfma_f32_32x32x2f32
// accumulates 32 symbols (a row tile) x 32 symbol values (a D tile) at a
// time, two (c, k) pairs per instruction.  Row tile t of the block only
// reaches the columns [32 n t, 32 n t + 31 n + Mt); its products elsewhere
// are skipped.
//
// The span goes in chunks of CS = 32 columns, each chunk in Mn steps, one
// per k; when a pass has too few blocks to fill the device, the chunks of a
// block are split into parts, one workgroup each, whose partial sums U
// k_app_fin adds.  Per chunk the workgroup stages in LDS the windows of alpha and
// beta of its 64 symbols as (mantissa, exponent) pairs; per step it stages
// R(s, D, k) of the chunk's columns for every D (full 128-byte row segments
// of the table), double-buffered, and issues the next step's loads into
// registers before the products, so their latency hides behind them.  Wave
// w takes row tile w / 2 and half the chunk's columns (w % 2), two per
// instruction (one per half-wave, the instruction's two contraction slots),
// and every D tile.  Each lane forms its own K operand, alpha beta 2^-E from
// the two pairs (the rows can peak at opposite ends of the drift range, so
// the product is formed from mantissas and exponent sums, E_i being the
// symbol's largest exponent sum over its band, from k_app_scale), and feeds
// it to the D tiles' instructions.  LDS rows have odd strides, so the 32
// lanes of a half-wave hit 32 banks.  The two waves of a row tile add their
// tiles through LDS at the end, into the part's U tile.
#include "device_common.h"

namespace mapdec {

namespace {

typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int kTB = kMfmaTB;   // symbols per workgroup: two row tiles of 32
constexpr int kCS = kMfmaCS;   // start-index columns per chunk
constexpr int kWaves = 4;

struct MEf {
    float m;
    int e;
};
constexpr int kZeroExpM = -(1 << 20);

__device__ __forceinline__ MEf split(double v) {
    MEf r;
    if (v > 0.0) {
        int e;
        r.m = (float)frexp(v, &e);
        r.e = e;
    } else {
        r.m = 0.f;
        r.e = kZeroExpM;
    }
    return r;
}

}  // namespace

// E_i = max over m' (alpha_i(m') > 0) of the binary exponent of alpha_i(m')
// plus the largest exponent of beta_{i+1} over m' + delta, delta in
// [-mn, mn] (beta > 0): the scale 2^-E_i that keeps the symbol's products
// alpha beta inside the FP32 range.  One wave per symbol; written to Zexp.
template <int MN>
__global__ __launch_bounds__(64) void k_app_scale(const FrameDesc *__restrict__ fd,
                                                  const Work *__restrict__ tab) {
    const Work w = tab[blockIdx.x];
    const FrameDesc &f = fd[w.frame];
    if (*f.status != kStatusOk) return;
    const int i = f.i0 + w.item, Mt = f.Mt, lane = threadIdx.x;
    __shared__ int eb[2048 + 2 * kMaxMn];
    const gptr<const double> A = to_global((const double *)f.alpha + (size_t)(i - f.i0) * Mt);
    const gptr<const double> B = to_global((const double *)f.beta + (size_t)(i + 1 - f.i0) * Mt);
    for (int j = lane; j < Mt + 2 * MN; j += 64) {
        const int m = j - MN;
        const double b = (m >= 0 && m < Mt) ? B[m] : 0.0;
        int e = kZeroExpM;
        if (b > 0.0) (void)frexp(b, &e);
        eb[j] = e;
    }
    lds_wave_sync();
    int best = 2 * kZeroExpM;
    for (int mi = lane; mi < Mt; mi += 64) {
        const double a = A[mi];
        if (!(a > 0.0)) continue;
        int ea;
        (void)frexp(a, &ea);
        int m = kZeroExpM;
#pragma unroll
        for (int k = 0; k < 2 * MN + 1; ++k) m = max(m, eb[mi + k]);
        if (m > kZeroExpM) best = max(best, ea + m);
    }
    for (int off = 32; off >= 1; off >>= 1) best = max(best, __shfl_xor(best, off, 64));
    if (lane == 0) f.Zexp[i] = best;
}

template <int MN, int QT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_app_mfma(const FrameDesc *__restrict__ fd,
                                                  const Work *__restrict__ tab) {
    constexpr int Mn = 2 * MN + 1;
    constexpr int RSC = kCS + 1;              // LDS row stride of a staged D row of R
    constexpr int APL = kCS + 1;              // alpha window row stride
    constexpr int BW = kCS + 2 * MN;          // beta window per symbol
    constexpr int BWP = BW | 1;
    constexpr int RPT = 32 * QT * kCS / 256;  // R values staged per thread and step
    constexpr int APT = kTB * kCS / 256;      // alpha values per thread and chunk
    constexpr int BPT = (kTB * BW + 255) / 256;
    constexpr int TPW = kCS / 4;              // instruction slots (column pairs) per wave
    static_assert(kCS == 32, "staging maps one column per lane of a half-wave");
    const Work w = tab[blockIdx.x];
    const FrameDesc &f = fd[w.frame];
    if (*f.status != kStatusOk) return;
    extern __shared__ __align__(16) unsigned char smem[];
    float *Rb = (float *)smem;                  // [2][32 QT][RSC]
    float *alm = Rb + 2 * 32 * QT * RSC;        // [kTB][APL] alpha mantissas
    int *ale = (int *)(alm + kTB * APL);        //            their exponents minus E_i
    float *blm = (float *)(ale + kTB * APL);    // [kTB][BWP] beta mantissas
    int *ble = (int *)(blm + kTB * BWP);        //            their exponents
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int rt = wv >> 1, cg = wv & 1;
    const int Mt = f.Mt, M = f.M, q = f.q, n = f.n, s0 = f.s0, s1 = f.s1;
    const int parts = f.app_parts, blk = w.item / parts, part = w.item - blk * parts;
    const int i0 = f.i0 + blk * kTB;
    const int nsym = min(kTB, f.i1 - i0);
    const int ib = f.i0;
    const int s_lo = n * i0 - M;
    const int span = n * (nsym - 1) + Mt;
    const int nch = (span + kCS - 1) / kCS;
    // this part's chunks
    const int ch_lo = part * nch / parts, ch_hi = (part + 1) * nch / parts;
    const gptr<const double> A = to_global((const double *)f.alpha);
    const gptr<const double> B = to_global((const double *)f.beta);
    const gptr<const float> R = to_global((const float *)f.R);
    const size_t sp = (size_t)f.sp;
    // the columns this wave's row tile reaches
    const int rt_lo = 32 * n * rt;
    const int rt_hi = 32 * rt < nsym ? rt_lo + n * (min(32, nsym - 32 * rt) - 1) + Mt : 0;

    // staging slots: R column rc of rows D = rd0 + 8 j; alpha / beta windows
    // at tid + 256 u
    const int rc = tid & 31, rd0 = tid >> 5;
    int aE[APT];
#pragma unroll
    for (int u = 0; u < APT; ++u) {
        const int j = (tid + 256 * u) / kCS;
        aE[u] = j < nsym ? f.Zexp[i0 + j] : 0;
    }
    // Raw values of the next loads: every load is issued unconditionally
    // from a clamped address and masked only when it is written to LDS, so
    // that no wait for it sits before the products it hides behind.
    float rv_[RPT];
    double av_[APT], bv_[BPT];
    auto col_ok = [&](int c0) {
        const int s = s_lo + c0 + rc;
        return s >= s0 && s <= s1;
    };
    auto fetch_r = [&](int c0, int k) {
        const int s = min(max(s_lo + c0 + rc, s0), s1);
        const size_t col = (size_t)(s - s0);
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            const int D = min(rd0 + 8 * j, q - 1);
            rv_[j] = R[(size_t)(D * Mn + k) * sp + col];
        }
    };
    // alpha_i(m') of slot u at chunk c0 (mp_of), beta_{i+1}(m' + delta)
    auto a_mp = [&](int c0, int u) {
        const int x = tid + 256 * u, j = x / kCS, cc = x % kCS;
        return s_lo + c0 + cc - n * (i0 + j);
    };
    auto b_m = [&](int c0, int u) {
        const int x = tid + 256 * u, j = x / BW, cc = x % BW;
        return s_lo + c0 + cc - MN - n * (i0 + j);
    };
    auto fetch_ab = [&](int c0) {
#pragma unroll
        for (int u = 0; u < APT; ++u) {
            const int j = min((tid + 256 * u) / kCS, nsym - 1);
            const int mc = min(max(a_mp(c0, u), -M), M);
            av_[u] = A[(size_t)(i0 + j - ib) * Mt + mc + M];
        }
#pragma unroll
        for (int u = 0; u < BPT; ++u) {
            const int j = min((tid + 256 * u) / BW, nsym - 1);
            const int mc = min(max(b_m(c0, u), -M), M);
            bv_[u] = B[(size_t)(i0 + j + 1 - ib) * Mt + mc + M];
        }
    };
    auto stage_ab = [&](int c0) {
#pragma unroll
        for (int u = 0; u < APT; ++u) {
            const int x = tid + 256 * u, j = x / kCS, cc = x % kCS;
            const int mp = a_mp(c0, u);
            const bool ok = j < nsym && mp >= -M && mp <= M;
            const MEf a = split(ok ? av_[u] : 0.0);
            alm[j * APL + cc] = a.m;
            ale[j * APL + cc] = a.e - aE[u];
        }
#pragma unroll
        for (int u = 0; u < BPT; ++u) {
            const int x = tid + 256 * u;
            if (x < kTB * BW) {
                const int j = x / BW, cc = x % BW;
                const int m = b_m(c0, u);
                const bool ok = j < nsym && m >= -M && m <= M;
                const MEf b = split(ok ? bv_[u] : 0.0);
                blm[j * BWP + cc] = b.m;
                ble[j * BWP + cc] = b.e;
            }
        }
    };

    v16f acc[QT];
#pragma unroll
    for (int t = 0; t < QT; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[t][r] = 0.f;

    // this lane's operands: symbol row ii of the row tile; columns
    // cc = 2 (TPW cg + t) + half
    const int ii = lane & 31, half = lane >> 5;
    const int row = 32 * rt + ii;
    fetch_ab(ch_lo * kCS);
    fetch_r(ch_lo * kCS, 0);
    int g = 0;   // step counter: R buffer g & 1
    for (int ch = ch_lo; ch < ch_hi; ++ch) {
        const int c0 = ch * kCS;
        if (ch > ch_lo) __syncthreads();   // the previous chunk's windows are read
        stage_ab(c0);
        fetch_ab(min(c0 + kCS, (ch_hi - 1) * kCS));   // in flight over the whole chunk
        const bool act = c0 < rt_hi && c0 + kCS > rt_lo;
        const bool rok = col_ok(c0);
        float am[TPW];
        int ae[TPW];
#pragma nounroll
        for (int k = 0; k < Mn; ++k, ++g) {
            float *Rs = Rb + (g & 1) * 32 * QT * RSC;
#pragma unroll
            for (int j = 0; j < RPT; ++j)
                Rs[(rd0 + 8 * j) * RSC + rc] = (rok && rd0 + 8 * j < q) ? rv_[j] : 0.f;
            __syncthreads();
            // the next step's R (past the last step: a repeat of it, unused)
            const bool last_k = k + 1 == Mn;
            fetch_r(last_k ? min(c0 + kCS, (ch_hi - 1) * kCS) : c0, last_k ? 0 : k + 1);
            if (!act) continue;
            if (k == 0) {
#pragma unroll
                for (int t = 0; t < TPW; ++t) {
                    const int cc = 2 * (TPW * cg + t) + half;
                    am[t] = alm[row * APL + cc];
                    ae[t] = ale[row * APL + cc];
                }
            }
#pragma unroll
            for (int t = 0; t < TPW; ++t) {
                const int cc = 2 * (TPW * cg + t) + half;
                // a zero mantissa carries exponent kZeroExpM: the product is 0
                const float kv = ldexpf(am[t] * blm[row * BWP + cc + k],
                                        ae[t] + ble[row * BWP + cc + k]);
#pragma unroll
                for (int qt = 0; qt < QT; ++qt) {
                    const float r = Rs[(qt * 32 + ii) * RSC + cc];
                    acc[qt] = __builtin_amdgcn_mfma_f32_32x32x2f32(kv, r, acc[qt], 0, 0, 0);
                }
            }
        }
    }
    __syncthreads();

    // the waves' tiles through LDS: Cw[wave][row][col D]; the two column
    // halves of each row tile added into this part's U tile
    float *Cw = (float *)smem;
#pragma unroll
    for (int qt = 0; qt < QT; ++qt)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int rr = 8 * (r / 4) + 4 * half + (r % 4);
            Cw[(wv * 32 + rr) * (32 * QT) + qt * 32 + ii] = acc[qt][r];
        }
    __syncthreads();
    float *Up = f.Up + (size_t)w.item * kTB * 32 * QT;
    for (int x = tid; x < kTB * 32 * QT; x += 256) {
        const int j = x / (32 * QT), d = x % (32 * QT);
        const int t = j >> 5, jr = j & 31;
        Up[x] = Cw[((2 * t) * 32 + jr) * (32 * QT) + d] + Cw[((2 * t + 1) * 32 + jr) * (32 * QT) + d];
    }
}

// The parts of a block added, then S_i(D) = prior_i(D) U_i(D), Z_i = sum_D
// S_i(D) (FP64), APP = S / Z, d log P / d prior = U / Z.  One workgroup per
// block of kTB symbols.
template <int QT>
__global__ __launch_bounds__(256) void k_app_fin(const FrameDesc *__restrict__ fd,
                                                 const Work *__restrict__ tab) {
    const Work w = tab[blockIdx.x];
    const FrameDesc &f = fd[w.frame];
    if (*f.status != kStatusOk) return;
    constexpr int US = 32 * QT + 1;   // odd row stride: a symbol per lane without bank conflicts
    __shared__ float Ush[kTB * US];
    __shared__ double Zsh[kTB];
    const int tid = threadIdx.x, q = f.q, parts = f.app_parts;
    const int i0 = f.i0 + w.item * kTB;
    const int nsym = min(kTB, f.i1 - i0);
    const float *Up = f.Up + (size_t)w.item * parts * kTB * 32 * QT;
    for (int x = tid; x < kTB * 32 * QT; x += 256) {
        float u = 0.f;
        for (int p = 0; p < parts; ++p) u += Up[(size_t)p * kTB * 32 * QT + x];
        Ush[(x / (32 * QT)) * US + x % (32 * QT)] = u;
    }
    __syncthreads();
    const float up = 1.f / (float)q;
    if (tid < nsym) {
        const int i = i0 + tid;
        const float *pr = f.uniform ? nullptr : (const float *)f.prior + (size_t)i * q;
        double Z = 0.0;
        for (int D = 0; D < q; ++D) Z += (double)((pr ? pr[D] : up) * Ush[tid * US + D]);
        Zsh[tid] = Z;
        if (f.Zinv) f.Zinv[i] = Z > 0.0 ? 1.0 / Z : 0.0;
    }
    __syncthreads();
    for (int x = tid; x < nsym * q; x += 256) {
        const int j = x / q, D = x - j * q, i = i0 + j;
        const float u = Ush[j * US + D];
        const float p = f.uniform ? up : ((const float *)f.prior)[(size_t)i * q + D];
        const float Zi = (float)Zsh[j];
        if (f.app) ((float *)f.app)[(size_t)i * q + D] = p * u / Zi;
        if (f.dprior) ((float *)f.dprior)[(size_t)i * q + D] = u / Zi;
    }
}

// LDS bytes of one k_app_mfma workgroup (staging; the epilogue reuses it)
size_t app_mfma_lds(int mn, int q) {
    const int QT = (q + 31) / 32;
    const size_t stage = (size_t)2 * 32 * QT * (kCS + 1) * sizeof(float) +
                         (size_t)kTB * (kCS + 1) * 8 + (size_t)kTB * ((kCS + 2 * mn) | 1) * 8;
    const size_t epi = (size_t)kWaves * 32 * 32 * QT * sizeof(float);
    return stage > epi ? stage : epi;
}

hipError_t launch_app_fin(int qt, const FrameDesc *fd, const Work *tab, int nblocks,
                          hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    if (qt == 1)
        hipLaunchKernelGGL(k_app_fin<1>, dim3(nblocks), dim3(256), 0, st, fd, tab);
    else if (qt == 2)
        hipLaunchKernelGGL(k_app_fin<2>, dim3(nblocks), dim3(256), 0, st, fd, tab);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <int MN>
static hipError_t mfma_mn(int qt, const FrameDesc *fd, const Work *tab, int nblocks,
                          size_t lds, hipStream_t st) {
    auto k1 = k_app_mfma<MN, 1>;
    auto k2 = k_app_mfma<MN, 2>;
    const void *kern = qt == 1 ? (const void *)k1 : (const void *)k2;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds);
        if (e != hipSuccess) return e;
    }
    if (qt == 1)
        hipLaunchKernelGGL(k1, dim3(nblocks), dim3(256), lds, st, fd, tab);
    else
        hipLaunchKernelGGL(k2, dim3(nblocks), dim3(256), lds, st, fd, tab);
    return hipGetLastError();
}

template <int MN>
static hipError_t scale_mn(const FrameDesc *fd, const Work *tab, int nitems, hipStream_t st) {
    hipLaunchKernelGGL(k_app_scale<MN>, dim3(nitems), dim3(64), 0, st, fd, tab);
    return hipGetLastError();
}

hipError_t launch_app_scale(int mn, const FrameDesc *fd, const Work *tab, int nitems,
                            hipStream_t st) {
    if (nitems == 0) return hipSuccess;
    switch (mn) {
        case 0: return scale_mn<0>(fd, tab, nitems, st);
        case 1: return scale_mn<1>(fd, tab, nitems, st);
        case 2: return scale_mn<2>(fd, tab, nitems, st);
        case 3: return scale_mn<3>(fd, tab, nitems, st);
        case 4: return scale_mn<4>(fd, tab, nitems, st);
        case 5: return scale_mn<5>(fd, tab, nitems, st);
        case 6: return scale_mn<6>(fd, tab, nitems, st);
        case 7: return scale_mn<7>(fd, tab, nitems, st);
        case 8: return scale_mn<8>(fd, tab, nitems, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_app_mfma(int mn, int qt, const FrameDesc *fd, const Work *tab, int nblocks,
                           size_t lds, hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    if (qt < 1 || qt > 2) return hipErrorInvalidValue;
    switch (mn) {
        case 0: return mfma_mn<0>(qt, fd, tab, nblocks, lds, st);
        case 1: return mfma_mn<1>(qt, fd, tab, nblocks, lds, st);
        case 2: return mfma_mn<2>(qt, fd, tab, nblocks, lds, st);
        case 3: return mfma_mn<3>(qt, fd, tab, nblocks, lds, st);
        case 4: return mfma_mn<4>(qt, fd, tab, nblocks, lds, st);
        case 5: return mfma_mn<5>(qt, fd, tab, nblocks, lds, st);
        case 6: return mfma_mn<6>(qt, fd, tab, nblocks, lds, st);
        case 7: return mfma_mn<7>(qt, fd, tab, nblocks, lds, st);
        case 8: return mfma_mn<8>(qt, fd, tab, nblocks, lds, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace mapdec
