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
    void *R;              // [q][Mn][sp] receiver metric R(s, D, delta)
    void *G;              // uniform: [Mn][sp] sum_D R / q; else [N][Mn][Mt]
    double *alpha;        // [N+1][Mt] forward metric rows (FP64 at every precision)
    double *beta;         // [N+1][Mt] backward metric rows (FP64 at every precision)
    double *logA;         // [N+1] log of the product of forward normalisers
    double *logB;         // [N+1] log of the product of backward normalisers
    double *Zinv;         // [N] 1 / sum_D S_i(D)  (gradient passes)
    double *gacc;         // [lat_blocks][4] partial d log P / d(a, d, t1, t0)
    int lat_blocks;       // lattice workgroups of this frame
    int adj_da;           // the adjoint sweep accumulates d/da (else from rho - tau)
};

// Work-table entry: which frame a workgroup serves and where in it.
struct Work {
    int frame;
    int item;
};

enum : int { kStatusOk = 0, kStatusNoPath = 3 };

}  // namespace mapdec
