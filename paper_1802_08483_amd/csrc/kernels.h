// Launchers for the gfx950 kernels of the MAP forward-backward decoder
// (Sec. II-C), implemented in k_misc.hip, k_lattice.hip, k_chain.hip and
// k_app.hip.
//
// Data flow per frame (one workspace region per frame, see FrameDesc):
//   k_pack     received bytes -> 32-bit words of bits
//   k_lattice  receiver metric R(s, D, delta) of eqs. 7-10 for every start
//              index s and symbol D (one lattice per (s, D) serves every
//              (i, m') with n i + m' = s, since the codebook is fixed), plus
//              Gamma(s, delta) = sum_D R / q when the priors are uniform
//   k_gamma    Gamma_i(m', delta) = sum_D prior_i(D) R(n i + m', D, delta)
//              for general priors (eq. 6 summed over D)
//   k_chain    normalised alpha (eqs. 4, 11, 12) and beta (eq. 5) chains,
//              one workgroup per frame and direction, log-normalisers in FP64
//   k_app      APP of eqs. 1-3: S_i(D) = prior_i(D) sum_{m', delta}
//              alpha_i(m') R(n i + m', D, delta) beta_{i+1}(m' + delta),
//              each row divided by its own sum
#pragma once

#include "mapdec_internal.h"

namespace mapdec {

// fp64 != 0 selects the double-precision instantiation of each kernel.
hipError_t launch_init(const FrameDesc *fd, int nframes, hipStream_t st);
hipError_t launch_pack(const FrameDesc *fd, const Work *tab, int nblocks, hipStream_t st);
// gen: the general-scheme instance (frames with a codebook per symbol or a
// corridor narrower than [-mn, mn]); else every frame has neither
hipError_t launch_lattice(int fp64, int mn, int imode, int gen, const FrameDesc *fd,
                          const Work *tab, int nblocks, hipStream_t st);
// Gamma_i for general priors; every frame of the launch has drift limit mn.
hipError_t launch_gamma(int fp64, int mn, const FrameDesc *fd, const Work *tab, int nblocks,
                        hipStream_t st);
// Gamma(s, .) = sum_D R / q for uniform-prior frames whose lattice items are
// split over codeword chunks (items: start-offset blocks of 64).
hipError_t launch_gsum(int fp64, int mn, const FrameDesc *fd, const Work *tab, int nblocks,
                       hipStream_t st);
// Chains over each frame's segment; dirs: 1 forward (alpha) only, 2 backward
// (beta) only, 3 both (one workgroup per chain).
constexpr int kDirFwd = 1, kDirBwd = 2, kDirBoth = 3;
hipError_t launch_chain(int fp64, const FrameDesc *fd, const int *frames, int nchains,
                        int dirs, size_t lds_bytes, hipStream_t st);
// Chains for uniform priors with Gamma in an LDS ring (k_chain_ring.hip):
// shape = index into kRingShapes; every frame of the launch has drift
// limit mn; waves (1 .. the shape's nw) per workgroup, at least
// ring_waves(shape, 2M+1) of every frame of the launch.
hipError_t launch_chain_ring(int fp64, int shape, int mn, int waves, const FrameDesc *fd,
                             const int *frames, int nchains, int dirs, size_t lds_bytes,
                             hipStream_t st);

// Workgroup shapes of the ring chain kernel: waves per chain, drift states
// per thread, and one metric row in LDS instead of two; a frame takes the
// first shape with 64 nw spl >= 2M+1 whose LDS fits.
struct RingShape {
    int nw, spl, one_row;
};
constexpr RingShape kRingShapes[] = {{1, 1, 0}, {2, 1, 0}, {4, 1, 0}, {4, 2, 0},
                                     {8, 2, 0}, {16, 2, 0}, {16, 2, 1}};
constexpr int kNumRingShapes = 7;
// Rings of at most this many padded states duplicate their edge slots.
constexpr bool ring_duplicates(int slots) { return slots <= 512; }
// Waves a chain of Mt drift states needs in a shape: enough for Mt states
// at spl per thread (the shape's nw at most).
constexpr int ring_waves(int shape, int Mt) {
    const int per = 64 * kRingShapes[shape].spl;
    const int w = (Mt + per - 1) / per;
    return w < 1 ? 1 : (w > kRingShapes[shape].nw ? kRingShapes[shape].nw : w);
}
// Waves a chain is launched with: ring_waves for uniform priors; the whole
// shape for general priors, whose steps each prefetch Mt columns (the
// prefetch registers of every thread are needed).
constexpr int chain_waves(int shape, int Mt, bool uniform) {
    return uniform ? ring_waves(shape, Mt) : kRingShapes[shape].nw;
}
hipError_t launch_app(int fp64, const FrameDesc *fd, const Work *tab, int nblocks,
                      size_t lds_bytes, hipStream_t st);
// Tiled APP (k_app_tile.hip): td symbol values per D tile (2, 4 or 8; at
// most 4 in FP64), nwaves waves splitting the block's start indices,
// kAppTI symbols per workgroup; every frame of the launch has drift limit mn.
hipError_t launch_app_tile(int fp64, int td, int mn, int nwaves, const FrameDesc *fd,
                           const Work *tab, int nblocks, size_t lds_bytes, hipStream_t st);

// Adjoint (k_adjoint.hip, one object per precision): output adjoints W
// (per mn group), the backward lattice sweep (per (mn, imode, sa) group, sa =
// the sweep accumulates d/da itself; LDS from adjoint_lds), and the
// per-frame reduction with the chain rule (k_misc.hip).
// uniform: every frame of the W launch has uniform priors (else none has)
// W: percol, the launch's frames have a codebook per symbol (R by symbol
// and drift state), else every one has one codebook; the sweep: gen as for
// the lattice
hipError_t adj_f32_w(int mn, int uniform, int percol, const FrameDesc *fd, const Work *tab,
                     int nblocks, hipStream_t st);
hipError_t adj_f64_w(int mn, int uniform, int percol, const FrameDesc *fd, const Work *tab,
                     int nblocks, hipStream_t st);
hipError_t adj_f32_lattice(int mn, int imode, int sa, int gen, const FrameDesc *fd,
                           const Work *tab, int nblocks, size_t lds, hipStream_t st);
hipError_t adj_f64_lattice(int mn, int imode, int sa, int gen, const FrameDesc *fd,
                           const Work *tab, int nblocks, size_t lds, hipStream_t st);
// The adjoint parks the even forward rows F_2, F_4, .. below row n of its
// 64 lattices in LDS, each in 16-byte slots of E = 16 / sizeof(T) corridor
// coordinates, then the last 2 mn + 1 - E floor((2 mn + 1) / E) one by one;
// row r leaves out the first park_first(r) / E slots (coordinates below
// mn - r: a node there would have consumed fewer than 0 received bits, so
// it is zero).  park_values(r) values of 64 lanes per row, park_offset(r)
// before row r.
template <int MN>
__host__ __device__ constexpr int park_first(int r) { return MN > r ? MN - r : 0; }
__host__ __device__ constexpr int park_values(int mn, int r, int e) {
    return 2 * mn + 1 - (mn > r ? mn - r : 0) / e * e;
}
template <int MN>
__host__ __device__ constexpr int park_offset(int r, int e) {
    int o = 0;
    for (int p = 2; p < r; p += 2) o += park_values(MN, p, e);
    return o;
}
// LDS bytes of one adjoint workgroup for codewords of up to nmax bits
constexpr size_t adjoint_lds(int nmax, int mn, size_t tsize) {
    size_t v = 0;
    for (int r = 2; r <= nmax - 1; r += 2) v += (size_t)park_values(mn, r, (int)(16 / tsize));
    return v * 64 * tsize;
}
// The sweep accumulates d/da itself when a g_a = rho - tau + d g_d would be
// a small difference of larger terms (Pi zero or below Pd / 4).
inline bool adjoint_needs_da(double Pi, double Pd) { return !(Pi > 0.0) || 4.0 * Pi < Pd; }
hipError_t launch_dparams(const FrameDesc *fd, int nframes, hipStream_t st);

// APP on the MFMA units (k_app_mfma.hip; FP32, one codebook, q <= 64):
// k_app_scale (one item per symbol: the exponent scale E_i into Zexp), then
// k_app_mfma (item b * parts + p: part p of the span of the block b of
// kMfmaTB symbols; qt = D tiles of 32) writing partial sums to Up, then
// k_app_fin (item b: adds the parts, then eqs. 2-3).
constexpr int kMfmaTB = 64;
constexpr int kMfmaPartsMax = 8;
constexpr int kMfmaCS = 32;         // start-index columns per chunk of a block's span
constexpr int kMfmaMinChunks = 8;   // fewest chunks a part covers
hipError_t launch_app_scale(int mn, const FrameDesc *fd, const Work *tab, int nitems,
                            hipStream_t st);
hipError_t launch_app_mfma(int mn, int qt, const FrameDesc *fd, const Work *tab, int nitems,
                           size_t lds, hipStream_t st);
hipError_t launch_app_fin(int qt, const FrameDesc *fd, const Work *tab, int nblocks,
                          hipStream_t st);
size_t app_mfma_lds(int mn, int q);

// Belief propagation of the outer code (k_outer.hip): iters iterations on
// nframes words; v2c, c2v: [nframes][E][q] message buffers.
hipError_t launch_outer(int fp64, const OuterDev &c, int nframes, const void *chan, void *extr,
                        void *post, int iters, void *v2c, void *c2v, hipStream_t st);

// The fixed device array of the allocation-free decode (scratch.hip): its
// size, and its address on the current device (taken once per device).
size_t scratch_bytes();
hipError_t scratch_address(void **out);

// Block sizes the host uses to build work tables.
constexpr int kPackWords = 8;      // packed words per pack workgroup (256 threads)
constexpr int kLatticeLanes = 64;  // start indices per lattice workgroup
// Codeword chunks of lattice / adjoint items: a pass whose lattice has fewer
// than kLatticeTarget workgroups splits each into up to kLatticeSplitMax
// items of at least kLatticeMinDq codewords.
constexpr long long kLatticeTarget = 4096;
constexpr int kLatticeSplitMax = 16;
constexpr int kLatticeMinDq = 4;
constexpr int kGammaLanes = 64;    // drift states per Gamma workgroup
constexpr int kChainThreads = 256;
constexpr int kAppThreads = 64;
constexpr int kAppTI = 4;   // consecutive symbols per tiled-APP workgroup
// zero padding (states) on each side of the rows staged by the tiled APP
__host__ __device__ constexpr int app_tile_pad(int n) { return (kAppTI - 1) * n; }
constexpr int kAppMaxWaves = 8;
// symbol values per D tile of the tiled APP: the next power of two >= q,
// between 2 and 8 (4 in FP64)
constexpr int app_tile_td(int q, size_t tsize) {
    const int cap = tsize == 8 ? 4 : 8;
    int td = 2;
    while (td < q && td < cap) td *= 2;
    return td;
}
// waves of a tiled-APP workgroup: one per 64 of the span of start indices
// n (kAppTI - 1) + Mt, at most kAppMaxWaves
constexpr int app_tile_waves(int Mt, int n) {
    const int chunks = ((kAppTI - 1) * n + Mt + 63) / 64;
    return chunks < kAppMaxWaves ? chunks : kAppMaxWaves;
}
// LDS bytes of one tiled-APP workgroup of nwaves waves and D tiles of td:
// the rows as (mantissa, exponent) pairs (8 bytes in FP32, 16 in FP64), Z
// and the exponent scale per symbol, the U tile and the per-wave partial
// sums in the batch precision
constexpr size_t app_tile_lds(int Mt, int mn, int n, int q, size_t tsize, int td, int nwaves) {
    return (size_t)kAppTI * ((size_t)(Mt + 2 * app_tile_pad(n)) +
                             (size_t)(Mt + 2 * (app_tile_pad(n) + mn))) * (tsize == 8 ? 16 : 8) +
           (size_t)kAppTI * (sizeof(double) + sizeof(int)) + (size_t)kAppTI * q * tsize +
           (size_t)nwaves * kAppTI * td * tsize;
}
// prefetch registers per thread in k_chain_ring (fewer in the 16-wave shapes,
// whose threads have 128 VGPRs, and fewer still for 8-byte Gamma there)
__host__ __device__ constexpr int ring_prefetch_regs(int nw, size_t tsize) {
    return nw >= 16 ? (tsize == 8 ? 4 : 6) : 16;
}

}  // namespace mapdec
