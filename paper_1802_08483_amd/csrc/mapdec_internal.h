// Internal definitions shared by the host library and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace mapdec {

constexpr int kMaxN = 16;   // longest codeword the lattice kernel unrolls
constexpr int kMaxMn = 8;   // widest per-codeword drift limit instantiated
constexpr int kMaxQ = 64;   // largest alphabet (one APP row per wave)

// Everything a kernel needs to know about one frame.  Lives in device
// memory (the head of the workspace); kernels read it with scalar loads.
struct FrameDesc {
    int q, n, N, rho;
    int M, mn, I, tau;
    int Mt, Mn;         // 2M+1 drift states, 2mn+1 drift changes
    int sp;             // column stride (>= rho+1) of the R and uniform-Gamma tables
    int uniform;        // prior == NULL: every prior entry is 1/q
    int nwords;         // 32-bit words of packed received bits (with padding)
    int imode;          // 0: I <= 2 (two-term insertion runs); 1: any I
    int grad;           // the adjoint pass runs for this frame
    int ck;             // checkpoint spacing of the forward metric (0 = all rows)
    int ring_chunk;     // chain steps per prefetch chunk (single-wave chains)
    int ring_cols;      // LDS ring columns (power of two) for Gamma(s, .)
    double a, d, t1, t0;  // lattice weights: Pi/2, Pd, Pt(1-Ps), Pt Ps
    double Pi, Pd, Ps;    // channel parameters (for the gradient's chain rule)
    // caller buffers (device)
    const uint8_t *y;
    const void *prior;    // [N][q] or NULL
    void *app;            // [N][q] or NULL
    void *dprior;         // [N][q] or NULL
    double *logp;         // 1
    int *status;          // 1
    double *dparams;      // 3 or NULL
    // workspace (device)
    uint32_t *cw;         // [q] codewords; bit (n-1-r) holds C(D)[r]
    uint32_t *ybits;      // [nwords] bit b of word w = y[32w + b]
    void *R;              // [q][Mn][sp] receiver metric R(s, D, delta), or NULL
                          // (a pass that only wants Gamma, uniform priors)
    void *G;              // uniform: [Mn][gsp] sum_D R / q at column s - s0; general
                          // priors: [Mn][gsp] Gamma_i(m', .) at column (i - i0) Mt + m' + M
    int gsp;              // column stride of G
    double *alpha;        // [N+1][Mt] forward metric rows (FP64 at every precision)
    double *beta;         // [N+1][Mt] backward metric rows (FP64 at every precision)
    double *logA;         // [N+1] log of the product of forward normalisers
    double *logB;         // [N+1] log of the product of backward normalisers
    double *Zinv;         // [N] 1 / Z_i' with Z_i = 2^Zexp[i] Z_i' (gradient passes)
    int *Zexp;            // [N] binary exponent of the APP's row-product scale
    float *Up;            // APP on the MFMA units: [blocks][parts][64][32 D-tiles]
                          // partial sums U of each part of a block's span
    int app_parts;        // parts per block of that APP (1 .. kMfmaPartsMax)
    double *sweep_state;  // sweep in parts: [2 directions][8] ring-chain scale
                          // predictor carried from part to part, or NULL
    double *gacc;         // [lattice workgroups of this segment][4] partial
                          // d log P / d(a, d, t1, t0)
    double *gacc_all;     // every segment's partials of the frame, contiguous,
                          // then [4] more: the posterior means of the end and
                          // start drift (boundary priors, gradient passes)
    int gacc_n;           // number of [4] partials at gacc_all
    int adj_da;           // the adjoint sweep accumulates d/da (else from the
                          // path-count identity)
    // Codewords per lattice / adjoint workgroup: dq = q unless a pass has too
    // few workgroups to fill the device, when each (start-index block) item
    // is split into dsplit items of dq codewords; the chunk index rides in
    // the low 6 bits of Work::item (start offsets are multiples of 64).
    int dq, dsplit;
    void *Gpart;          // [dsplit][Mn][sp] per-chunk sums of R (uniform priors, dsplit > 1)
    // Segment of the frame that this descriptor's launches cover (the whole
    // frame unless the forward metric is checkpointed): symbols [i0, i1),
    // start indices [s0, s1].  Column c of R and of the uniform Gamma holds
    // start index s0 + c; row r of alpha / beta (and Gamma_i for general
    // priors) sits at index r - i0.
    int i0, i1, s0, s1;
    const double *a_init; // alpha row i0 ([Mt]) or NULL: the start state (i0 = 0)
    double *a_fin;        // receives alpha row i1, or NULL
    const double *b_init; // beta row i1 or NULL: the end state (i1 = N)
    double *b_fin;        // receives beta row i0, or NULL
    // How a chain over this descriptor stores its results:
    //   kChainRows  every row of [i0, i1] at index row - i0, the cumulative
    //               logs at i0 / i1, log P at i1 = N;
    //   kChainSweep only rows at multiples of ck_stride, at index
    //               row / ck_stride, with the cumulative log of each such row
    //               (the checkpoints of both directions), log P at i1 = N;
    //   kChainSub   a recomputation from checkpoints: rows of [i0, i1] at
    //               index row - i0 except the starting row unless wr_init
    //               asks for it (bit 0 forward, bit 1 backward), and no logs,
    //               log P or drift means (the sweep wrote them).
    int chain_mode, ck_stride, wr_init;
    // The general scheme (Sec. II-A: a codebook C_i per symbol position;
    // Sec. III-B: asymmetric limits).  percol: R holds one column per
    // (symbol i, drift state m'), column (i - i0) Mt + m' + M, computed with
    // codeword cw[i cwi + D]; else column s - s0 of the start index (one
    // codebook: R depends on s only).  Drift states outside [lim_lo, lim_hi]
    // (within [-M, M]) are zero in every metric row; a lattice keeps node
    // (r, j) only if bit j - r + mn of cmask is set (the corridor
    // [m_n^-, m_n^+] inside [-mn, mn]).
    int percol, cwi, lim_lo, lim_hi;
    uint32_t cmask;
    // Path thresholds (theta > 0): the forward chain over the frame drops
    // every state whose metric is below theta times its row's sum and
    // records which states it kept in kept ([N+1][Mt] bytes, frame rows);
    // backward chains and recomputations zero the states it dropped.
    double theta;
    uint8_t *kept;
    const double *start_prior;  // [Mt] prior of the frame's start drift, or NULL
    const double *end_prior;  // [Mt] prior of the frame's end drift, or NULL
                              // (known end drift rho - tau): log P(y) takes
                              // sum_m alpha_N(m) end_prior[m] at i1 = N
};

// Work-table entry: which frame a workgroup serves and where in it.  For
// lattice and adjoint items, item = start offset (a multiple of 64) plus the
// codeword chunk index.
struct Work {
    int frame;
    int item;
};

enum : int { kStatusOk = 0, kStatusNoPath = 3 };
enum : int { kChainRows = 0, kChainSweep = 1, kChainSub = 2 };

// Outer code of iterative decoding on the device (see k_outer.hip): H in
// compressed rows (edge e = row entry), the edges of every symbol, and the
// multiplication and inverse tables of GF(q).
constexpr int kOuterMaxDeg = 32;
struct OuterDev {
    int q, N, m, E;
    const int *row_ptr;     // [m+1]
    const int *col;         // [E]
    const uint8_t *coef;    // [E]
    const int *var_ptr;     // [N+1]
    const int *var_edge;    // [E] edges of symbol j at var_ptr[j] ..
    const uint8_t *mul;     // [q][q]
    const uint8_t *inv;     // [q]
};

// Records a failed call's status for mapdec_last_error; returns it.
int record_error(int st);

}  // namespace mapdec
