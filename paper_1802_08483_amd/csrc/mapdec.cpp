// Host side of libmapdec: validation, workspace layout, descriptor upload,
// launch sequence and HIP-graph replay.  See include/mapdec.h for the ABI.
#include "mapdec.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "kernels.h"

using namespace mapdec;

struct mapdec_code {
    int q, n, I, M, mn;
    double Pi, Pd, Ps;
    // ncb codebooks of q codewords (ncb = 1, or N: codebook i for symbol i);
    // codeword D of codebook b at cw[b q + D]: bit (n-1-r) = C_b(D)[r]
    int ncb = 1;
    std::vector<uint32_t> cw;
    // drift state limits [mt_lo, mt_hi] and corridor [mn_lo, mn_hi]; M and
    // mn above are the symmetric limits that contain them
    int mt_lo = 0, mt_hi = 0, mn_lo = 0, mn_hi = 0;
    double theta = 0.0;   // path thresholds (0: none)
};

namespace {

thread_local int g_last_error = MAPDEC_OK;

int fail(int st) {
    g_last_error = st;
    return st;
}

}  // namespace

namespace mapdec {
int record_error(int st) { return fail(st); }
}  // namespace mapdec

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

int validate_code_params(int q, int n, double Pi, double Pd, double Ps, int I, int M, int mn) {
    if (n < 1 || n > 30 || q < 2 || q > (1 << n)) return MAPDEC_EINVAL;
    if (!(Pi >= 0.0) || !(Pd >= 0.0) || !(Ps >= 0.0) || !(Ps <= 1.0)) return MAPDEC_EINVAL;
    if (!(Pi + Pd < 1.0)) return MAPDEC_EINVAL;
    if (I < 0 || mn < 0 || M < mn) return MAPDEC_EINVAL;
    return MAPDEC_OK;
}

// Tuned launch choices, shared by every plan of the process.  The tiled
// APP's (D tile, waves) is tuned per (precision, q, n, mn, default waves),
// the ring chain's workgroup shape per (precision, uniform priors, columns
// per step, mn, first shape that fits); keys without an entry take the
// defaults (app_tile_td, app_tile_waves, the first ring shape that fits).
using TuneKey = std::array<int, 5>;
struct TuneTable {
    std::mutex mu;
    std::map<TuneKey, std::pair<int, int>> app;   // -> (td, waves)
    std::map<TuneKey, int> ring;                  // -> shape
};
TuneTable &tune_table() {
    static TuneTable t;
    return t;
}

// Sizes and places of one frame's workspace pieces.
//
// Checkpointed frames (checkpoint spacing ck < N) run in three kinds of
// pass: pre-passes compute Gamma for the whole frame into its own table
// (uniform priors: one lattice pass over every start index, no R stored;
// general priors: lattice and Gamma per group of segments); one sweep pass
// runs the forward and backward chains over the whole frame side by side,
// keeping only the rows at multiples of ck (the checkpoints of both
// directions); main passes then take the frame a group of consecutive
// checkpoint segments at a time: the group's receiver metric, every
// segment's forward and backward rows recomputed from its own two
// checkpoints (all at once), the APPs and the gradient terms.  Groups hold
// enough segments that the start indices the group's symbols reach (nK +
// 2M for K symbols) exceed the group's own nK by a quarter at most.
struct FrameLayout {
    int nwords = 0, sp = 0, gsp = 0, Mt = 0, Mn = 0, pack_blocks = 0;
    int K = 0, nseg = 1;   // symbols per main pass (group) and groups (1 unless checkpointed)
    int ck = 0, nck = 1;   // checkpoint spacing (0: none) and checkpoint segments
    // sweep in parts: forward part p covers rows [swa[p], swa[p+1]), backward
    // part p rows [swb[p+1], swb[p]) (checkpoint rows, swa[0] = 0, swb[0] = N)
    std::vector<int> swa, swb;
    size_t off_sws = 0;   // the sweep's carried scale predictor (parts > 1)
    // Gamma pre-pass in rounds (sweep in parts, Gamma by start index): the
    // round of each block of kLatticeLanes start indices, the first whose
    // sweep parts read it
    std::vector<int> pre_round;
    // percol: a codebook per symbol, R by (symbol, drift state); gcol: Gamma
    // by (symbol, drift state) (general priors, or percol); gen: the lattice
    // and adjoint kernels' general-scheme instance (percol, or a corridor
    // narrower than [-mn, mn])
    bool percol = false, gcol = false, gen = false;
    bool pruned = false;   // path thresholds (theta > 0)
    bool app_mfma = false; // the APP on the MFMA units
    int app_parts = 1;     // its parts per block of kMfmaTB symbols
    size_t off_up = 0;     // its partial sums
    int spw = 0, gspw = 0; // column strides of the whole-frame Gamma (checkpointed frames)
    int ring_shape = -1, ring_chunk = 0, ring_cols = 0;   // ring_shape -1: plain chain
    bool app_tiled = false;
    std::tuple<int, int, int> app_key;                     // (td, waves, mn) when tiled
    TuneKey app_bucket{}, ring_bucket{};                   // keys of the tuned choices
    int ring_first = -1;                                   // first shape that fits
    size_t off_cw = 0, off_ybits = 0, off_R = 0, off_G = 0, off_alpha = 0, off_beta = 0,
           off_logA = 0, off_logB = 0, off_Zinv = 0, off_Zexp = 0, off_gacc = 0, off_ck = 0,
           off_ckb = 0, off_Gw = 0, off_gpart = 0, off_kept = 0;
    std::vector<int> gacc_first;   // first [4] partial of each group
    int gacc_n = 0;
    int dq = 0, dsplit = 1;        // codewords per lattice / adjoint item, items per block
};

// Group j of a frame (the symbols of one main pass): symbols [i0, i1) and
// the start indices [s0, s1] their drift bands reach (s0 <= s1 whenever
// |rho - tau| <= M).
struct Segment {
    int i0, i1, s0, s1;
};
Segment segment_of(const mapdec_frame &fr, const FrameLayout &F, int j) {
    const mapdec_code *c = fr.code;
    Segment g;
    g.i0 = j * F.K;
    g.i1 = std::min(fr.N, g.i0 + F.K);
    g.s0 = std::max(0, c->n * g.i0 - c->M);
    g.s1 = std::min(fr.rho, c->n * (g.i1 - 1) + c->M);
    return g;
}
// Groups span at least this many times 2M received bits, so that the
// start indices a group's symbols reach exceed its own by 1/kGroupSpan.
constexpr int kGroupSpan = 4;
int lattice_blocks(const Segment &g) { return (g.s1 - g.s0 + 1 + kLatticeLanes - 1) / kLatticeLanes; }
// Lattice workgroups of a group: 64 start indices each, or (a codebook per
// symbol) 64 (symbol, drift state) columns.
int blocks_of(const FrameLayout &F, const Segment &g) {
    return F.percol ? ((g.i1 - g.i0) * F.Mt + kLatticeLanes - 1) / kLatticeLanes
                    : lattice_blocks(g);
}

// The launches of one pass.  Pre-pass j (checkpointed frames): the
// lattice and Gamma of group j into the whole-frame Gamma (uniform priors:
// every start index in pass 0).  Sweep (checkpointed frames): both chains
// over the whole frame, keeping the checkpoints.  Main pass j, over group
// j of every frame that has one: the lattice, the chains (unsegmented
// frames: Gamma and both chains over the frame; checkpointed frames: each
// segment's chains from its checkpoints, through extra descriptors after
// the frames'), the APP and, for gradients, W and the adjoint sweep.
enum PassKind { kPassPre, kPassSweep, kPassMain };
struct Pass {
    int kind = kPassMain;
    int seg = 0;
    int part = 0;    // sweep: the part; main: the sweep part after which its checkpoints exist
    size_t off_fd = 0;
    std::vector<int> sub_frame;   // frame of descriptor nframes + k
    std::vector<int> sub_seg;     // its checkpoint segment
    std::map<std::tuple<int, int, int>, std::vector<Work>> lat;   // (mn, imode, gen)
    std::map<std::tuple<int, int, int>, size_t> off_lat;
    // per mn: the start-index blocks without codeword chunks (W), and those
    // of uniform-prior frames whose lattice is split (Gamma from R)
    std::map<std::tuple<int, int, int>, std::vector<Work>> wlat;   // (mn, uniform priors, percol)
    std::map<std::tuple<int, int, int>, size_t> off_wlat;
    std::map<int, std::vector<Work>> gsum;
    std::map<int, size_t> off_gsum;
    std::map<int, std::vector<Work>> gamma;                         // mn
    std::map<int, size_t> off_gamma;
    // chain lists by (the frames' path thresholds are decided here, so the
    // forward chains run before the backward ones: 1, else both at once: 0)
    std::map<int, std::vector<int>> chain_plain;
    std::map<int, size_t> off_chain;
    std::map<std::tuple<int, int, int>, std::vector<int>> chain_ring;   // (shape, mn, fwd first)
    std::map<std::tuple<int, int, int>, size_t> off_chain_ring;
    std::map<std::tuple<int, int, int>, std::vector<Work>> app_tile;   // (td, waves, mn)
    std::map<std::tuple<int, int, int>, size_t> off_app_tile;
    std::vector<Work> app_plain;
    size_t off_app = 0;
    // the APP on the MFMA units: the scale items (one per symbol) by mn,
    // the blocks of kMfmaTB symbols by (mn, D tiles)
    std::map<int, std::vector<Work>> app_scale;
    std::map<int, size_t> off_app_scale;
    std::map<std::pair<int, int>, std::vector<Work>> app_mfma;
    std::map<std::pair<int, int>, size_t> off_app_mfma;
    std::map<int, std::vector<Work>> app_fin;   // by D tiles: one item per block
    std::map<int, size_t> off_app_fin;
    std::map<std::tuple<int, int, int, int>, std::vector<Work>> adj;   // (mn, imode, d/da, gen)
    std::map<std::tuple<int, int, int, int>, size_t> off_adj;
};

struct Layout {
    int nframes = 0, fp64 = 0, grad = 0, ckK = 0;
    // frame slices of an eager forked plan (1: none) and each frame's slice
    int slices = 1;
    // parts of the sweep of checkpointed frames (1: one launch)
    int sweep_parts = 1;
    bool pre_rounds = false;   // the Gamma pre-pass in rounds beside the sweep parts
    std::vector<int> fslice;
    size_t tsize = 4;
    size_t off_pack = 0, head = 0, total = 0;
    std::vector<Work> pack;
    std::vector<Pass> passes;
    // LDS bytes of each kernel instance (maxima over its launches)
    size_t chain_lds = 0, app_lds = 0;
    std::map<std::pair<int, int>, size_t> ring_lds;
    std::map<std::tuple<int, int, int>, size_t> app_tile_lds;
    std::map<std::pair<int, int>, size_t> app_mfma_lds;   // (mn, D tiles)
    std::map<std::tuple<int, int, int, int>, size_t> adj_lds;
    std::vector<FrameLayout> fl;
};

// The plan whose descriptors and work tables the head of a workspace holds.
// Plans of one batch share its workspace but not always its head layout
// (slices, tuned choices), so a run first restores its own head when
// another plan (or a one-shot decode) wrote it last.
struct HeadOwners {
    std::mutex mu;
    std::map<const void *, const void *> owner;   // workspace -> plan
};
HeadOwners &head_owners() {
    static HeadOwners h;
    return h;
}

// Frame slices: an eager plan of many frames runs its batch as this many
// contiguous slices of frames, slice k on stream k, so that one slice's
// chains (a latency-bound recursion) run beside another slice's
// compute-bound launches.
constexpr int kSlices = 4;
// Eager plans of checkpointed frames run the sweep in this many parts, so
// that the main passes of groups whose checkpoints are done run beside the
// rest of it (the sweep holds one workgroup per chain and direction).
constexpr int kSweepParts = 16;
constexpr int kSliceMinFrames = 16;

// Reorders a work list so that the workgroups the dispatcher sends to one
// XCD (workgroup ids congruent mod 8) take consecutive items: neighbouring
// symbol blocks of a frame then share that XCD's L2.
std::vector<Work> xcd_order(const std::vector<Work> &items) {
    constexpr int kXcd = 8;
    const size_t nb = items.size();
    std::vector<Work> out(nb);
    size_t start = 0;
    for (int x = 0; x < kXcd; ++x) {
        const size_t cnt = nb > (size_t)x ? (nb - x + kXcd - 1) / kXcd : 0;
        for (size_t j = 0; j < cnt; ++j) out[x + kXcd * j] = items[start + j];
        start += cnt;
    }
    return out;
}

// Ring-chain parameters of one workgroup shape (steps per prefetch chunk,
// ring slots, LDS bytes); false when the shape does not fit the frame.
// n = columns per step: the codeword length for uniform priors (the ring
// then covers at least 8 steps), Mt for general priors (Gamma columns are
// not shared between steps; one step per chunk).
bool ring_fit(int shape, int Mt, int Mn, int n, int mn, bool uniform, size_t tsize,
              size_t lds_limit, int &chunk, int &cols, size_t &lds) {
    const RingShape &rs = kRingShapes[shape];
    if (64 * rs.nw * rs.spl < Mt) return false;
    // the prefetch is spread over the threads the chain is launched with;
    // rows and ring duplication follow the compiled shape
    const int nt = 64 * chain_waves(shape, Mt, uniform), slots = 64 * rs.nw * rs.spl;
    // ring: a power of two covering the window of at least 8 steps; the
    // chunk is as long as the ring and the prefetch registers allow
    cols = 1;
    while (cols < Mt + (uniform ? n * 7 : 0)) cols *= 2;
    chunk = std::min({(cols - Mt) / n + 1, (nt * ring_prefetch_regs(rs.nw, tsize)) / (n * Mn), 64});
    if (chunk < 1) return false;
    const size_t roww = (size_t)slots + 2 * mn;
    const size_t rphys = ring_duplicates(slots) ? cols + roww : cols + 2 * mn;
    // FP64 rows and wave partials, Gamma ring in the batch precision
    lds = ((rs.one_row ? 1 : 2) * roww + 3 * rs.nw) * sizeof(double) + rphys * Mn * tsize;
    return lds <= lds_limit;
}

// The first ring shape that fits, or false when the frame needs the plain
// workgroup chain kernel instead.
bool ring_params(int Mt, int Mn, int n, int mn, bool uniform, size_t tsize, size_t lds_limit,
                 int &shape, int &chunk, int &cols, size_t &lds) {
    for (shape = 0; shape < kNumRingShapes; ++shape)
        if (ring_fit(shape, Mt, Mn, n, mn, uniform, tsize, lds_limit, chunk, cols, lds))
            return true;
    shape = -1;
    return false;
}

int frame_imode(const mapdec_code *c) { return c->I <= 2 ? 0 : 1; }
// 1 when the adjoint sweep of the frame accumulates d log P / d a itself,
// which it does when a g_a from the path-count identity would be a small
// difference of larger terms
int frame_da(const mapdec_frame &fr) { return adjoint_needs_da(fr.code->Pi, fr.code->Pd) ? 1 : 0; }

// LDS bytes one workgroup may use on the current device (64 KiB when the
// device cannot be queried, e.g. on a host without a GPU).
size_t device_lds_limit() {
    static thread_local int cached_dev = -1;
    static thread_local size_t cached = 65536;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    if (dev != cached_dev) {
        int v = 0;
        cached = hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) ==
                         hipSuccess && v > 0
                     ? (size_t)v
                     : 65536;
        cached_dev = dev;
    }
    return cached;
}

// Compute units of the current device (256 when it cannot be queried).
int device_cu_count() {
    static thread_local int cached_dev = -1;
    static thread_local int cached = 256;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (dev != cached_dev) {
        int v = 0;
        cached = hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) ==
                         hipSuccess && v > 0
                     ? v
                     : 256;
        cached_dev = dev;
    }
    return cached;
}

// Validates the frames and lays out the workspace.  ckK > 0 splits every
// frame into segments of ckK symbols with forward-metric checkpoints.
int build_layout(const mapdec_frame *frames, int nframes, int precision, int flags, int ckK,
                 Layout &L) {
    if (!frames || nframes < 1 || ckK < 0) return MAPDEC_EINVAL;
    if (precision != MAPDEC_FP32 && precision != MAPDEC_FP64) return MAPDEC_EINVAL;
    L.nframes = nframes;
    L.fp64 = precision == MAPDEC_FP64;
    L.grad = (flags & MAPDEC_FLAG_GRAD) != 0;
    L.ckK = ckK;
    L.tsize = L.fp64 ? 8 : 4;
    L.fl.resize(nframes);
    const size_t lds_limit = device_lds_limit();
    int smax = 1;
    for (int f = 0; f < nframes; ++f) {
        const mapdec_frame &fr = frames[f];
        const mapdec_code *c = fr.code;
        if (!c || fr.N < 1 || fr.rho < 0 || (fr.rho > 0 && !fr.y)) return MAPDEC_EINVAL;
        const long long tau = (long long)c->n * fr.N;
        if (tau > (1LL << 30) || fr.rho > (1 << 30)) return MAPDEC_EUNSUPPORTED;
        if ((long long)fr.rho - tau < c->mt_lo || (long long)fr.rho - tau > c->mt_hi)
            return MAPDEC_EDRIFT;
        if (c->ncb > 1 && c->ncb != fr.N) return MAPDEC_EINVAL;   // a codebook per symbol
        if (c->n > kMaxN || c->mn > kMaxMn || c->q > kMaxQ) return MAPDEC_EUNSUPPORTED;
        FrameLayout &F = L.fl[f];
        F.Mt = 2 * c->M + 1;
        F.Mn = 2 * c->mn + 1;
        F.percol = c->ncb > 1;
        F.gcol = F.percol || fr.prior != nullptr;
        F.gen = F.percol || c->mn_lo != -c->mn || c->mn_hi != c->mn;
        F.pruned = c->theta > 0.0;
        if (F.percol && (long long)fr.N * F.Mt + 64 > (1LL << 31)) return MAPDEC_EUNSUPPORTED;
        if (ckK > 0 && ckK < fr.N) {
            F.ck = ckK;
            F.nck = (fr.N + ckK - 1) / ckK;
            const long long span = (long long)kGroupSpan * 2 * c->M;
            const long long per = std::max<long long>(1, (span + (long long)c->n * ckK - 1) /
                                                             ((long long)c->n * ckK));
            F.K = (int)std::min<long long>((long long)F.nck, per) * ckK;
            F.K = std::min(F.K, fr.N);
            F.spw = (fr.rho + 1 + 63) / 64 * 64;
            F.gspw = (int)(((long long)fr.N * F.Mt + 63) / 64 * 64);
            if ((long long)fr.N * F.Mt + 64 > (1LL << 31)) return MAPDEC_EUNSUPPORTED;
        } else {
            F.K = fr.N;
        }
        F.nseg = (fr.N + F.K - 1) / F.K;
        smax = std::max(smax, F.nseg);
        F.sp = 0;
        for (int j = 0; j < F.nseg; ++j) {
            const Segment g = segment_of(fr, F, j);
            const int cols = F.percol ? (g.i1 - g.i0) * F.Mt : g.s1 - g.s0 + 1;
            F.sp = std::max(F.sp, (cols + 63) / 64 * 64);
        }
        F.nwords = (fr.rho + 63) / 32 + 2;
        F.pack_blocks = (F.nwords + kPackWords - 1) / kPackWords;
        for (int b = 0; b < F.pack_blocks; ++b) L.pack.push_back(Work{f, b * kPackWords});
        {
            int td = app_tile_td(c->q, L.tsize), nw = app_tile_waves(F.Mt, c->n);
            const size_t tl = app_tile_lds(F.Mt, c->mn, c->n, c->q, L.tsize, td, nw);
            // the tile kernel addresses R with 32-bit byte offsets, and
            // shares each R column among the symbols of a tile (one codebook)
            const bool fits = (double)c->q * F.Mn * F.sp * L.tsize < 2147483648.0;
            F.app_tiled = fits && tl <= lds_limit && !F.percol;
            // FP32 with one codebook and 16 < q <= 64: the matrix-unit form of
            // the same sums (at q <= 16 half of every 32-wide D tile would
            // be idle, and the tile kernel is the faster one)
            F.app_mfma = !L.fp64 && !F.percol && c->q > 16 && c->q <= 64 && F.Mt <= 2048 &&
                         app_mfma_lds(c->mn, c->q) <= lds_limit;
            if (F.app_mfma) {
                F.app_tiled = false;
                const auto mk = std::make_pair(c->mn, (c->q + 31) / 32);
                L.app_mfma_lds[mk] = std::max(L.app_mfma_lds[mk], app_mfma_lds(c->mn, c->q));
            }
            if (F.app_tiled && !F.app_mfma) {
                F.app_bucket = TuneKey{L.fp64, c->q, c->n, c->mn, nw};
                size_t lds = tl;
                {
                    TuneTable &T = tune_table();
                    std::lock_guard<std::mutex> g(T.mu);
                    auto it = T.app.find(F.app_bucket);
                    if (it != T.app.end()) {
                        const size_t l2 = app_tile_lds(F.Mt, c->mn, c->n, c->q, L.tsize,
                                                       it->second.first, it->second.second);
                        if (l2 <= lds_limit) {
                            td = it->second.first;
                            nw = it->second.second;
                            lds = l2;
                        }
                    }
                }
                F.app_key = std::make_tuple(td, nw, c->mn);
                L.app_tile_lds[F.app_key] = std::max(L.app_tile_lds[F.app_key], lds);
            } else if (!F.app_mfma) {
                L.app_lds = std::max(L.app_lds, (2 * (size_t)F.Mt + 2 * c->mn + c->q) * sizeof(double));
            }
        }
        int shape = -1;
        size_t rlds = 0;
        const int ncols = F.gcol ? F.Mt : c->n;
        if (ring_params(F.Mt, F.Mn, ncols, c->mn, !F.gcol, L.tsize, lds_limit, shape,
                        F.ring_chunk, F.ring_cols, rlds)) {
            F.ring_first = shape;
            F.ring_bucket = TuneKey{L.fp64, F.gcol ? 0 : 1, F.gcol ? 0 : c->n, c->mn, shape};
            {
                TuneTable &T = tune_table();
                std::lock_guard<std::mutex> g(T.mu);
                auto it = T.ring.find(F.ring_bucket);
                int ch, co;
                size_t l2;
                if (it != T.ring.end() && it->second != shape &&
                    ring_fit(it->second, F.Mt, F.Mn, ncols, c->mn, !F.gcol, L.tsize, lds_limit,
                             ch, co, l2)) {
                    shape = it->second;
                    F.ring_chunk = ch;
                    F.ring_cols = co;
                    rlds = l2;
                }
            }
            F.ring_shape = shape;
            const auto key = std::make_pair(shape, c->mn);
            L.ring_lds[key] = std::max(L.ring_lds[key], rlds);
        } else {
            F.ring_shape = -1;
            F.ring_chunk = F.ring_cols = 0;
            L.chain_lds = std::max(L.chain_lds, (2 * ((size_t)F.Mt + 2 * c->mn) + 16) * sizeof(double));
        }
        if (L.grad) {
            const auto akey = std::make_tuple(c->mn, frame_imode(c), frame_da(fr),
                                              F.gen ? 1 : 0);
            const size_t al = adjoint_lds(c->n, c->mn, L.tsize);
            if (al > lds_limit) return MAPDEC_EUNSUPPORTED;
            L.adj_lds[akey] = std::max(L.adj_lds[akey], al);
        }
    }
    if (L.chain_lds > 65536 || L.app_lds > 65536) return MAPDEC_EUNSUPPORTED;

    // Codeword chunks: when one pass's lattice workgroups (one wave each,
    // looping over every codeword) are too few to fill the device, every
    // start-index block becomes dsplit items of dq codewords each.
    {
        long long blocks = 0;
        for (int f = 0; f < nframes; ++f)
            blocks += blocks_of(L.fl[f], segment_of(frames[f], L.fl[f], 0));
        const int split = (int)std::min<long long>(
            kLatticeSplitMax, std::max<long long>(1, (kLatticeTarget + blocks - 1) / blocks));
        for (int f = 0; f < nframes; ++f) {
            FrameLayout &F = L.fl[f];
            const int q = frames[f].code->q;
            // per-symbol lattices are never short of workgroups
            F.dq = (split == 1 || F.percol)
                       ? q : std::max(std::min(q, kLatticeMinDq), (q + split - 1) / split);
            F.dsplit = (q + F.dq - 1) / F.dq;
            F.gacc_first.assign(F.nseg, 0);
            F.gacc_n = 0;
            for (int j = 0; j < F.nseg; ++j) {
                F.gacc_first[j] = F.gacc_n;
                F.gacc_n += blocks_of(F, segment_of(frames[f], F, j)) * F.dsplit;
            }
        }
    }

    // APP on the MFMA units: when one pass has too few blocks of kMfmaTB
    // symbols to give each workgroup slot of the device one (two per compute
    // unit), the span of every block is split into parts of at least
    // kMfmaMinChunks chunks, whose partial sums k_app_fin adds.
    {
        long long blocks = 0;
        for (int f = 0; f < nframes; ++f)
            if (L.fl[f].app_mfma) {
                const Segment g = segment_of(frames[f], L.fl[f], 0);
                blocks += (g.i1 - g.i0 + kMfmaTB - 1) / kMfmaTB;
            }
        if (blocks > 0) {
            const long long slots = 2LL * device_cu_count();
            const int parts = (int)std::max<long long>(
                1, std::min<long long>(kMfmaPartsMax, slots / blocks));
            for (int f = 0; f < nframes; ++f) {
                FrameLayout &F = L.fl[f];
                if (!F.app_mfma) continue;
                const mapdec_code *c = frames[f].code;
                const int nch = (c->n * (kMfmaTB - 1) + F.Mt + kMfmaCS - 1) / kMfmaCS;
                F.app_parts = std::max(1, std::min(parts, nch / kMfmaMinChunks));
            }
        }
    }

    // Slices pay off where every phase is one launch (frames of one kernel
    // configuration) and the step has enough compute after the chains to
    // hide them under (gradients); batches with several launch groups per
    // phase overlap those groups instead.
    bool one_config = true;
    {
        const mapdec_code *c0 = frames[0].code;
        const FrameLayout &F0 = L.fl[0];
        for (int f = 1; f < nframes && one_config; ++f) {
            const mapdec_code *c = frames[f].code;
            const FrameLayout &F = L.fl[f];
            one_config = c->mn == c0->mn && frame_imode(c) == frame_imode(c0) &&
                         F.percol == F0.percol && F.gen == F0.gen &&
                         (frames[f].prior != nullptr) == (frames[0].prior != nullptr) &&
                         F.ring_shape == F0.ring_shape && F.app_tiled == F0.app_tiled &&
                         F.app_key == F0.app_key && F.dsplit == F0.dsplit &&
                         frame_da(frames[f]) == frame_da(frames[0]);
        }
    }
    L.slices = (L.grad && one_config && !(flags & (MAPDEC_FLAG_GRAPH | MAPDEC_FLAG_SERIAL)) &&
                nframes >= 2 * kSliceMinFrames)
                   ? std::min(kSlices, nframes / kSliceMinFrames)
                   : 1;
    L.fslice.resize(nframes);
    for (int f = 0; f < nframes; ++f)
        L.fslice[f] = (int)((long long)f * L.slices / nframes);

    // passes: pre-passes and the sweep (checkpointed frames), then main
    // passes over groups S-1 .. 0 (the last pass covers group 0)
    int npre = 0;
    bool any_ck = false, gcol_ck = false, pruned_ck = false;
    for (int f = 0; f < nframes; ++f) {
        const FrameLayout &F = L.fl[f];
        if (!F.ck) continue;
        any_ck = true;
        gcol_ck |= F.gcol;
        pruned_ck |= F.pruned;
        npre = std::max(npre, F.gcol ? F.nseg : 1);
    }
    // The sweep in parts (eager plans without path thresholds or frame
    // slices): the forward chains advance from the start, the backward ones
    // from the end, so the checkpoints of the middle groups are done first.
    L.sweep_parts = (any_ck && !pruned_ck && L.slices == 1 &&
                     !(flags & (MAPDEC_FLAG_GRAPH | MAPDEC_FLAG_SERIAL)))
                        ? kSweepParts : 1;
    const int SP = L.sweep_parts;
    for (int f = 0; f < nframes; ++f) {
        FrameLayout &F = L.fl[f];
        if (!F.ck) continue;
        const long long N = frames[f].N, K = F.ck;
        F.swa.assign(SP + 1, 0);
        F.swb.assign(SP + 1, 0);
        for (int p = 0; p <= SP; ++p) {
            F.swa[p] = p == SP ? (int)N : (int)(N * p / SP / K * K);
            F.swb[p] = p == 0 ? (int)N : (int)((N - N * p / SP) / K * K);
        }
    }
    // With the sweep in parts and Gamma by start index, the pre-pass runs in
    // rounds beside the sweep: round r holds the blocks of start indices
    // that forward or backward part r reads first (rows [i0, i1) read
    // Gamma at n i0 - M .. n (i1 - 1) + M), and part r waits for rounds
    // 0 .. r only.
    L.pre_rounds = SP > 1 && !gcol_ck;
    if (L.pre_rounds) {
        npre = SP;
        for (int f = 0; f < nframes; ++f) {
            FrameLayout &F = L.fl[f];
            if (!F.ck) continue;
            const mapdec_frame &fr = frames[f];
            const int n = fr.code->n, M = fr.code->M;
            const int nb = (fr.rho + kLatticeLanes) / kLatticeLanes;
            F.pre_round.assign(nb, -1);
            auto mark = [&](int r, int i0, int i1) {
                if (i1 <= i0) return;
                const int lo = std::max(0, n * i0 - M), hi = std::min(fr.rho, n * (i1 - 1) + M);
                for (int b = lo / kLatticeLanes; b <= hi / kLatticeLanes; ++b)
                    if (F.pre_round[b] < 0) F.pre_round[b] = r;
            };
            for (int r = 0; r < SP; ++r) {
                mark(r, F.swa[r], F.swa[r + 1]);
                mark(r, F.swb[r + 1], F.swb[r]);
            }
            for (int &r : F.pre_round)   // start indices no chain reads
                if (r < 0) r = SP - 1;
        }
    }
    for (int j = 0; j < npre; ++j) {
        Pass P;
        P.kind = kPassPre;
        P.seg = j;
        L.passes.push_back(P);
    }
    if (any_ck)
        for (int p = 0; p < SP; ++p) {
            Pass P;
            P.kind = kPassSweep;
            P.part = p;
            L.passes.push_back(P);
        }
    std::vector<Pass> mains;
    for (int j = smax - 1; j >= 0; --j) {
        Pass P;
        P.kind = kPassMain;
        P.seg = j;
        // the first sweep part after which every checkpoint this group's
        // segments start from exists: forward row (last segment) k1 K,
        // backward row (first segment) (k0 + 1) K (the end prior beyond)
        int ready = 0;
        for (int f = 0; f < nframes && SP > 1; ++f) {
            const FrameLayout &F = L.fl[f];
            if (!F.ck || j >= F.nseg) continue;
            const Segment g = segment_of(frames[f], F, j);
            const int k0 = g.i0 / F.ck, k1 = (g.i1 - 1) / F.ck;
            const int ra = k1 * F.ck, rb = (k0 + 1) * F.ck;
            int pa = 0, pb = 0;
            while (pa < SP - 1 && F.swa[pa + 1] < ra) ++pa;
            if (k0 + 1 < F.nck)
                while (pb < SP - 1 && F.swb[pb + 1] > rb) ++pb;
            ready = std::max(ready, std::max(pa, pb));
        }
        P.part = ready;
        mains.push_back(P);
    }
    // main passes in the order their checkpoints are done
    std::stable_sort(mains.begin(), mains.end(),
                     [](const Pass &a, const Pass &b) { return a.part < b.part; });
    for (Pass &P : mains) L.passes.push_back(P);
    for (Pass &P : L.passes) {
        const int j = P.seg;
        std::vector<std::pair<int, int>> chains;   // (steps, descriptor)
        for (int f = 0; f < nframes; ++f) {
            const mapdec_frame &fr = frames[f];
            const mapdec_code *c = fr.code;
            const FrameLayout &F = L.fl[f];
            if (P.kind == kPassSweep) {
                if (!F.ck) continue;
                if (L.sweep_parts == 1) {
                    chains.push_back(std::make_pair(fr.N, f));
                    continue;
                }
                // the part's forward chain (descriptor f) and backward chain
                // (an extra descriptor), each when its rows are not empty
                const int p = P.part;
                if (F.swa[p + 1] > F.swa[p])
                    chains.push_back(std::make_pair(F.swa[p + 1] - F.swa[p], f));
                if (F.swb[p] > F.swb[p + 1]) {
                    const int d = nframes + (int)P.sub_frame.size();
                    P.sub_frame.push_back(f);
                    P.sub_seg.push_back(p);
                    chains.push_back(std::make_pair(F.swb[p] - F.swb[p + 1], d));
                }
                continue;
            }
            if (P.kind == kPassPre) {
                if (!F.ck || j >= (L.pre_rounds ? L.sweep_parts : F.gcol ? F.nseg : 1)) continue;
                const auto lkey = std::make_tuple(c->mn, frame_imode(c), F.gen ? 1 : 0);
                if (!F.gcol) {   // every start index (of the round), Gamma only
                    const int nb = (fr.rho + kLatticeLanes) / kLatticeLanes;
                    for (int b = 0; b < nb; ++b)
                        if (!L.pre_rounds || F.pre_round[b] == j)
                            P.lat[lkey].push_back(Work{f, b * kLatticeLanes});
                    continue;
                }
                auto &lv = P.lat[lkey];
                const Segment g = segment_of(fr, F, j);
                const int nb = blocks_of(F, g);
                for (int b = 0; b < nb; ++b)
                    for (int x = 0; x < F.dsplit; ++x) lv.push_back(Work{f, b * kLatticeLanes + x});
                if (fr.prior) {   // (uniform priors: the lattice writes Gamma)
                    const int per_i = (F.Mt + kGammaLanes - 1) / kGammaLanes;
                    auto &gv = P.gamma[c->mn];
                    for (int b = 0; b < (g.i1 - g.i0) * per_i; ++b) gv.push_back(Work{f, b});
                }
                continue;
            }
            if (j >= F.nseg) continue;
            const Segment g = segment_of(fr, F, j);
            auto &lv = P.lat[std::make_tuple(c->mn, frame_imode(c), F.gen ? 1 : 0)];
            auto &wv = P.wlat[std::make_tuple(c->mn, fr.prior ? 0 : 1, F.percol ? 1 : 0)];
            const int nb = blocks_of(F, g);
            for (int b = 0; b < nb; ++b) {
                wv.push_back(Work{f, b * kLatticeLanes});
                for (int x = 0; x < F.dsplit; ++x) lv.push_back(Work{f, b * kLatticeLanes + x});
            }
            if (F.ck) {
                // each checkpoint segment of the group: its own chains
                for (int k = g.i0 / F.ck; k * F.ck < g.i1; ++k) {
                    const int d = nframes + (int)P.sub_frame.size();
                    P.sub_frame.push_back(f);
                    P.sub_seg.push_back(k);
                    chains.push_back(std::make_pair(std::min(fr.N, (k + 1) * F.ck) - k * F.ck, d));
                }
            } else {
                if (!fr.prior && F.dsplit > 1) {
                    auto &gs = P.gsum[c->mn];
                    for (int b = 0; b < nb; ++b) gs.push_back(Work{f, b * kLatticeLanes});
                }
                if (fr.prior) {
                    const int per_i = (F.Mt + kGammaLanes - 1) / kGammaLanes;
                    auto &gv = P.gamma[c->mn];
                    for (int b = 0; b < (g.i1 - g.i0) * per_i; ++b) gv.push_back(Work{f, b});
                }
                chains.push_back(std::make_pair(g.i1 - g.i0, f));
            }
            if (F.app_mfma) {
                auto &sv = P.app_scale[c->mn];
                for (int i = g.i0; i < g.i1; ++i) sv.push_back(Work{f, i - g.i0});
                const int qt = (c->q + 31) / 32;
                auto &v = P.app_mfma[std::make_pair(c->mn, qt)];
                auto &fv = P.app_fin[qt];
                for (int b = 0; b * kMfmaTB < g.i1 - g.i0; ++b) {
                    for (int p = 0; p < F.app_parts; ++p) v.push_back(Work{f, b * F.app_parts + p});
                    fv.push_back(Work{f, b});
                }
            } else if (F.app_tiled) {
                auto &v = P.app_tile[F.app_key];
                for (int b = 0; b * kAppTI < g.i1 - g.i0; ++b) v.push_back(Work{f, b});
            } else {
                for (int i = g.i0; i < g.i1; ++i) P.app_plain.push_back(Work{f, i - g.i0});
            }
            if (L.grad) {
                auto &av = P.adj[std::make_tuple(c->mn, frame_imode(c), frame_da(fr),
                                                 F.gen ? 1 : 0)];
                for (int b = 0; b < nb; ++b)
                    for (int x = 0; x < F.dsplit; ++x) av.push_back(Work{f, b * kLatticeLanes + x});
            }
        }
        // longest chains first, so that the longest ones do not start last
        std::stable_sort(chains.begin(), chains.end(),
                         [](const std::pair<int, int> &a, const std::pair<int, int> &b) {
                             return a.first > b.first;
                         });
        for (const auto &ch : chains) {
            const int d = ch.second;   // descriptor
            const int f = d < nframes ? d : P.sub_frame[d - nframes];
            const FrameLayout &F = L.fl[f];
            // a forward chain over the frame decides the path thresholds
            // that the backward chain applies
            const int seq = (frames[f].code->theta > 0.0 && d < nframes) ? 1 : 0;
            if (F.ring_shape >= 0)
                P.chain_ring[std::make_tuple(F.ring_shape, frames[f].code->mn, seq)].push_back(d);
            else
                P.chain_plain[seq].push_back(d);
        }
        // items of one slice contiguous (slice order); neighbouring items
        // share rows (APP, W) or received columns (Gamma): keep them on one
        // XCD's L2 within each slice
        auto by_slice = [&](std::vector<Work> &v, bool xcd) {
            std::stable_sort(v.begin(), v.end(), [&](const Work &a, const Work &b) {
                return L.fslice[a.frame] < L.fslice[b.frame];
            });
            if (!xcd) return;
            size_t a = 0;
            while (a < v.size()) {
                size_t b = a;
                while (b < v.size() && L.fslice[v[b].frame] == L.fslice[v[a].frame]) ++b;
                std::vector<Work> part(v.begin() + a, v.begin() + b);
                part = xcd_order(part);
                std::copy(part.begin(), part.end(), v.begin() + a);
                a = b;
            }
        };
        for (auto &kv : P.app_tile) by_slice(kv.second, true);
        for (auto &kv : P.app_scale) by_slice(kv.second, false);
        for (auto &kv : P.app_mfma) by_slice(kv.second, true);
        for (auto &kv : P.app_fin) by_slice(kv.second, false);
        for (auto &kv : P.lat) by_slice(kv.second, true);
        for (auto &kv : P.wlat) by_slice(kv.second, true);
        for (auto &kv : P.gsum) by_slice(kv.second, true);
        for (auto &kv : P.gamma) by_slice(kv.second, true);
        for (auto &kv : P.adj) by_slice(kv.second, false);
        by_slice(P.app_plain, false);
        // by slice, and within a slice whole-frame chains before the
        // recomputations of checkpoint segments (separate launches)
        auto chains_by_slice = [&](std::vector<int> &v) {
            auto fr_of = [&](int d) { return d < nframes ? d : P.sub_frame[d - nframes]; };
            std::stable_sort(v.begin(), v.end(), [&](int a, int b) {
                const int sa = L.fslice[fr_of(a)], sb = L.fslice[fr_of(b)];
                return sa != sb ? sa < sb : (a >= nframes) < (b >= nframes);
            });
        };
        for (auto &kv : P.chain_plain) chains_by_slice(kv.second);
        for (auto &kv : P.chain_ring) chains_by_slice(kv.second);
    }

    // head: the pack table and, per pass, the descriptors, the work tables
    // back to back (8-byte entries) and the chain lists (4-byte entries), so
    // the head's size depends on the work items only, not on how they are
    // grouped into launches (tuned choices regroup them)
    size_t off = 0;
    L.off_pack = off;
    off = align_up(off + sizeof(Work) * L.pack.size());
    for (Pass &P : L.passes) {
        P.off_fd = off;
        off = align_up(off + sizeof(FrameDesc) * (nframes + P.sub_frame.size()));
        auto place = [&](auto &groups, auto &offs) {
            for (auto &kv : groups) {
                offs[kv.first] = off;
                off += sizeof(Work) * kv.second.size();
            }
        };
        place(P.lat, P.off_lat);
        place(P.wlat, P.off_wlat);
        place(P.gsum, P.off_gsum);
        place(P.adj, P.off_adj);
        place(P.gamma, P.off_gamma);
        place(P.app_tile, P.off_app_tile);
        place(P.app_scale, P.off_app_scale);
        place(P.app_mfma, P.off_app_mfma);
        place(P.app_fin, P.off_app_fin);
        P.off_app = off;
        off += sizeof(Work) * P.app_plain.size();
        for (auto &kv : P.chain_plain) {
            P.off_chain[kv.first] = off;
            off += sizeof(int) * kv.second.size();
        }
        for (auto &kv : P.chain_ring) {
            P.off_chain_ring[kv.first] = off;
            off += sizeof(int) * kv.second.size();
        }
        off = align_up(off);
    }
    L.head = off;

    // per-frame regions (R, Gamma, alpha and beta hold one segment)
    for (int f = 0; f < nframes; ++f) {
        const mapdec_frame &fr = frames[f];
        const mapdec_code *c = fr.code;
        FrameLayout &F = L.fl[f];
        const size_t T = L.tsize;
        F.off_cw = off;
        off = align_up(off + sizeof(uint32_t) * c->q * c->ncb);
        F.off_ybits = off;
        off = align_up(off + sizeof(uint32_t) * F.nwords);
        F.off_R = off;
        off = align_up(off + T * c->q * F.Mn * (size_t)F.sp);
        F.off_G = off;
        F.gsp = F.gcol ? std::max(F.sp, (F.K * F.Mt + 63) / 64 * 64) : F.sp;
        // checkpointed frames with Gamma by symbol keep Gamma in the
        // whole-frame table only (uniform priors with a codebook per symbol
        // need the group's buffer for W)
        if (!(F.ck && fr.prior)) off = align_up(off + T * (size_t)F.Mn * F.gsp);
        if (F.ck) {
            F.off_Gw = off;
            off = align_up(off + T * (size_t)F.Mn * (F.gcol ? F.gspw : F.spw));
        }
        if (!fr.prior && F.dsplit > 1) {
            F.off_gpart = off;   // per-chunk partial sums of R for Gamma
            off = align_up(off + T * (size_t)F.dsplit * F.Mn * F.sp);
        }
        F.off_alpha = off;   // metric rows are FP64 at every precision
        off = align_up(off + sizeof(double) * (size_t)(F.K + 1) * F.Mt);
        F.off_beta = off;
        off = align_up(off + sizeof(double) * (size_t)(F.K + 1) * F.Mt);
        F.off_logA = off;
        off = align_up(off + sizeof(double) * (fr.N + 1));
        F.off_logB = off;
        off = align_up(off + sizeof(double) * (fr.N + 1));
        F.off_Zinv = off;
        off = align_up(off + sizeof(double) * fr.N);
        F.off_Zexp = off;
        off = align_up(off + sizeof(int) * fr.N);
        if (F.app_mfma) {
            // the partial sums of the blocks of the longest segment
            const int nb = (std::min(F.K, fr.N) + kMfmaTB - 1) / kMfmaTB;
            F.off_up = off;
            off = align_up(off + sizeof(float) * (size_t)nb * F.app_parts * kMfmaTB * 32 *
                                     ((c->q + 31) / 32));
        }
        F.off_gacc = off;   // the partials, then one slot for the boundary-drift means
        off = align_up(off + sizeof(double) * 4 * ((size_t)F.gacc_n + 1));
        if (F.pruned) {
            F.off_kept = off;    // the states the thresholds kept, a byte per (row, state)
            off = align_up(off + (size_t)(fr.N + 1) * F.Mt);
        }
        if (F.ck && L.sweep_parts > 1) {
            F.off_sws = off;
            off = align_up(off + sizeof(double) * 16);
        }
        if (F.ck) {
            F.off_ck = off;      // alpha rows 0, ck, 2 ck, .. (row j ck at index j)
            off = align_up(off + sizeof(double) * (size_t)(F.nck + 1) * F.Mt);
            F.off_ckb = off;     // beta rows at the same places
            off = align_up(off + sizeof(double) * (size_t)(F.nck + 1) * F.Mt);
        }
    }
    L.total = off;
    return MAPDEC_OK;
}

// Per-launch phase names, in the order of mapdec_phase_name().
// kPhRechain: the chains of checkpoint segments recomputed in main passes.
enum Phase {
    kPhPack, kPhLattice, kPhGamma, kPhChain, kPhApp, kPhWgrad, kPhAdjoint, kPhDparams,
    kPhRechain, kNumPhases
};

// One kernel launch (or, for the set-up, two) of a plan, with the frames
// whose workspace regions it reads or writes.
struct Op {
    int phase = 0;
    bool all = false;          // touches every frame (set-up, parameter sums)
    std::vector<int> frames;   // sorted, distinct (when !all)
    int stream = 0;            // 0: the run's stream, k > 0: forked stream k - 1
    int slice = -1;            // frame slice, or -1
    int after = -1;            // an earlier op this one also waits for, or -1
    std::vector<int> afters;   // more earlier ops it waits for (sweep parts)
    bool rows_only = false;    // reads only the group's rows (the APP's scale pass)
    std::function<hipError_t(hipStream_t)> fn;
};

std::vector<int> frames_of(const std::vector<Work> &items) {
    std::vector<int> v;
    v.reserve(items.size());
    for (const Work &w : items) v.push_back(w.frame);
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    return v;
}
std::vector<int> sorted_frames(std::vector<int> v) {
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    return v;
}

// Launch groups of one phase that can run side by side: the forked streams
// besides the run's own.  Kernels of different groups share no workspace
// region, so only the frames a launch touches order it after earlier ones.
constexpr int kForkStreams = 3;

}  // namespace

struct mapdec_plan {
    Layout L;
    unsigned char *ws = nullptr;
    int flags = 0;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t last_stream = nullptr;
    bool ran = false;

    template <typename P>
    P *at(size_t off) const { return reinterpret_cast<P *>(ws + off); }

    std::vector<unsigned char> head_host;   // this plan's head of the workspace
    // Restores this plan's head of the workspace (stream-ordered) when
    // another plan wrote it last.
    hipError_t own_head(hipStream_t st) {
        HeadOwners &h = head_owners();
        std::lock_guard<std::mutex> g(h.mu);
        auto it = h.owner.find(ws);
        if (it != h.owner.end() && it->second == this) return hipSuccess;
        const hipError_t e =
            hipMemcpyAsync(ws, head_host.data(), head_host.size(), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) h.owner[ws] = this;
        return e;
    }

    std::vector<Op> ops;
    bool forked = false;                  // some phase has several launch groups
    hipStream_t side[kForkStreams] = {};
    std::vector<hipEvent_t> dep;          // one per op, plus the fork

    // profiling: timing events recorded just before and just after each
    // launch, on the launch's stream
    std::vector<hipEvent_t> pb, pa;
    hipError_t prof_events() {
        hipError_t e = hipSuccess;
        while (e == hipSuccess && pb.size() < ops.size()) {
            hipEvent_t x, y;
            e = hipEventCreate(&x);
            if (e != hipSuccess) break;
            e = hipEventCreate(&y);
            if (e != hipSuccess) {
                hipEventDestroy(x);
                break;
            }
            pb.push_back(x);
            pa.push_back(y);
        }
        return e;
    }

    // The plan's launches in dependency order: set-up, then per pass the
    // lattice, Gamma, chains, APP and (gradients) W and the adjoint sweep,
    // and the parameter sums.  Without slices, the launch groups of a phase
    // are dealt to the streams in order of decreasing size (chains: their
    // longest chain).  With frame slices every group becomes one launch per
    // slice on the slice's stream, and every launch but the chains also
    // waits for the same group's launch of the slice before, so that the
    // compute-bound phases advance slice by slice while each slice's chains
    // run beside them.
    // With the sweep in parts, its forward launches run on forked stream 1
    // and its backward ones on stream 2, each tracked as a resource of its
    // own per frame (nf + f, 2 nf + f); the other launches keep streams 0
    // and 3, and every launch of a main pass also waits for the sweep part
    // after which its group's checkpoints exist.
    void build_ops() {
        const int nf = L.nframes;
        const bool sliced = L.slices > 1;
        const bool split = L.sweep_parts > 1;
        std::vector<int> sweep_fwd(L.sweep_parts, -1), sweep_bwd(L.sweep_parts, -1);
        // the pre-passes' launches, by pre-pass (with rounds: sweep part p
        // waits for those of rounds 0 .. p; else each sweep direction's
        // first launch waits for all)
        std::vector<std::vector<int>> pre_ops(1);
        auto add = [&](int phase, std::vector<int> frames, bool all,
                       std::function<hipError_t(hipStream_t)> fn) {
            Op o;
            o.phase = phase;
            o.all = all;
            o.frames = std::move(frames);
            o.fn = std::move(fn);
            ops.push_back(std::move(o));
        };
        const FrameDesc *fd0 = at<FrameDesc>(L.passes.front().off_fd);
        const int npack = (int)L.pack.size();
        const Work *ptab = at<Work>(L.off_pack);
        add(kPhPack, {}, true, [=](hipStream_t st) {
            hipError_t e = launch_init(fd0, nf, st);
            return e == hipSuccess ? launch_pack(fd0, ptab, npack, st) : e;
        });
        const int fp64 = L.fp64;
        for (const Pass &P : L.passes) {
            const FrameDesc *fd = at<FrameDesc>(P.off_fd);
            const size_t first_op = ops.size();
            // size of each group, for dealing the groups of a phase to streams
            std::vector<std::pair<long long, size_t>> group;
            auto deal = [&]() {
                if (sliced) {
                    for (auto &g : group) ops[g.second].stream = ops[g.second].slice % (kForkStreams + 1);
                    if (!group.empty()) forked = true;
                    group.clear();
                    return;
                }
                std::stable_sort(group.begin(), group.end(),
                                 [](const std::pair<long long, size_t> &a,
                                    const std::pair<long long, size_t> &b) {
                                     return a.first > b.first;
                                 });
                for (size_t g = 0; g < group.size(); ++g)
                    ops[group[g].second].stream =
                        split ? (g % 2 ? kForkStreams : 0) : (int)(g % (kForkStreams + 1));
                if (group.size() > 1) forked = true;
                group.clear();
            };
            // one launch per slice range of a work table (the whole table
            // without slices); launch(stream, table, count)
            auto add_work = [&](int phase, bool staggered, const std::vector<Work> &items, size_t off,
                                std::function<hipError_t(hipStream_t, const Work *, int)> launch) {
                size_t a = 0;
                int prev = -1;
                while (a < items.size()) {
                    size_t b = a;
                    const int sl = L.fslice[items[a].frame];
                    while (b < items.size() && L.fslice[items[b].frame] == sl) ++b;
                    const Work *tab = at<Work>(off) + a;
                    const int nb = (int)(b - a);
                    const std::vector<Work> part(items.begin() + a, items.begin() + b);
                    add(phase, frames_of(part), false,
                        [=](hipStream_t st) { return launch(st, tab, nb); });
                    ops.back().slice = sl;
                    if (sliced && staggered) ops.back().after = prev;
                    prev = (int)ops.size() - 1;
                    group.push_back(std::make_pair((long long)nb, ops.size() - 1));
                    a = b;
                }
            };
            // chain lists hold descriptors: frames, or a checkpoint
            // segment's descriptor after them
            auto frame_of = [&](int d) { return d < nf ? d : P.sub_frame[d - nf]; };
            auto add_chains = [&](const std::vector<int> &list, size_t off, long long steps_of_first,
                                  std::function<hipError_t(hipStream_t, const int *, int)> launch) {
                size_t a = 0;
                while (a < list.size()) {
                    size_t b = a;
                    const int sl = L.fslice[frame_of(list[a])];
                    const bool sub = list[a] >= nf;
                    while (b < list.size() && L.fslice[frame_of(list[b])] == sl &&
                           (list[b] >= nf) == sub)
                        ++b;
                    const int *tab = at<int>(off) + a;
                    const int nc = (int)(b - a);
                    std::vector<int> fl;
                    for (size_t k = a; k < b; ++k) fl.push_back(frame_of(list[k]));
                    add(sub ? kPhRechain : kPhChain, sorted_frames(fl),
                        false, [=](hipStream_t st) { return launch(st, tab, nc); });
                    ops.back().slice = sl;
                    group.push_back(std::make_pair(steps_of_first, ops.size() - 1));
                    a = b;
                }
            };
            for (auto &kv : P.lat) {
                const int mn = std::get<0>(kv.first), im = std::get<1>(kv.first),
                          pc = std::get<2>(kv.first);
                add_work(kPhLattice, true, kv.second, P.off_lat.at(kv.first),
                         [=](hipStream_t st, const Work *tab, int nb) {
                             return launch_lattice(fp64, mn, im, pc, fd, tab, nb, st);
                         });
            }
            deal();
            for (auto &kv : P.gamma) {
                const int mn = kv.first;
                add_work(kPhGamma, true, kv.second, P.off_gamma.at(kv.first),
                         [=](hipStream_t st, const Work *tab, int nb) {
                             return launch_gamma(fp64, mn, fd, tab, nb, st);
                         });
            }
            for (auto &kv : P.gsum) {
                const int mn = kv.first;
                add_work(kPhGamma, true, kv.second, P.off_gsum.at(kv.first),
                         [=](hipStream_t st, const Work *tab, int nb) {
                             return launch_gsum(fp64, mn, fd, tab, nb, st);
                         });
            }
            deal();
            if (P.kind == kPassSweep && split) {
                // forward descriptors (frames) first, then backward (extra)
                auto emit = [&](const std::vector<int> &list, size_t off,
                                std::function<hipError_t(hipStream_t, const int *, int, int)> launch) {
                    size_t na = 0;
                    while (na < list.size() && list[na] < nf) ++na;
                    for (int dir = 0; dir < 2; ++dir) {
                        const size_t a = dir ? na : 0, b = dir ? list.size() : na;
                        if (a == b) continue;
                        std::vector<int> res;
                        for (size_t k = a; k < b; ++k) res.push_back((dir ? 2 : 1) * nf + frame_of(list[k]));
                        const int *tab = at<int>(off) + a;
                        const int nc = (int)(b - a), dd = dir ? kDirBwd : kDirFwd;
                        add(kPhChain, sorted_frames(res), false,
                            [=](hipStream_t st) { return launch(st, tab, nc, dd); });
                        ops.back().stream = dir ? 2 : 1;
                        // the direction's first launch waits for the pre-passes
                        // (its first parts may be empty for every frame)
                        std::vector<int> &mine = dir ? sweep_bwd : sweep_fwd;
                        if (L.pre_rounds) {
                            for (int r = 0; r <= P.part && r < (int)pre_ops.size(); ++r)
                                for (int k : pre_ops[r]) ops.back().afters.push_back(k);
                        } else if (*std::max_element(mine.begin(), mine.end()) < 0) {
                            for (const auto &v : pre_ops)
                                for (int k : v) ops.back().afters.push_back(k);
                        }
                        mine[P.part] = (int)ops.size() - 1;
                    }
                };
                for (auto &kv : P.chain_plain) {
                    const size_t lds = L.chain_lds;
                    emit(kv.second, P.off_chain.at(kv.first),
                         [=](hipStream_t st, const int *tab, int nc, int dd) {
                             return launch_chain(fp64, fd, tab, nc, dd, lds, st);
                         });
                }
                for (auto &kv : P.chain_ring) {
                    const int shape = std::get<0>(kv.first), mn = std::get<1>(kv.first);
                    const size_t lds = L.ring_lds.at(std::make_pair(shape, mn));
                    int waves = 1;
                    for (int dsc : kv.second)
                        waves = std::max(waves, chain_waves(shape, L.fl[frame_of(dsc)].Mt,
                                                            !L.fl[frame_of(dsc)].gcol));
                    emit(kv.second, P.off_chain_ring.at(kv.first),
                         [=](hipStream_t st, const int *tab, int nc, int dd) {
                             return launch_chain_ring(fp64, shape, mn, waves, fd, tab, nc, dd,
                                                      lds, st);
                         });
                }
                forked = true;
                continue;
            }
            const int dirs = kDirBoth;
            auto steps = [&](int d) {
                const int f = frame_of(d);
                const FrameLayout &F = L.fl[f];
                if (d >= nf) {
                    const int j = P.sub_seg[d - nf];
                    return (long long)(std::min(frames_[f].N, (j + 1) * F.ck) - j * F.ck);
                }
                if (P.kind == kPassSweep) return (long long)frames_[f].N;
                const Segment g = segment_of(frames_[f], F, std::min(P.seg, F.nseg - 1));
                return (long long)(g.i1 - g.i0);
            };
            // lists whose forward chains decide path thresholds: the forward
            // launch, then the backward one (ordered through their frames)
            for (auto &kv : P.chain_plain) {
                const size_t lds = L.chain_lds;
                for (int dd : kv.first ? std::vector<int>{kDirFwd, kDirBwd} : std::vector<int>{dirs})
                    add_chains(kv.second, P.off_chain.at(kv.first), steps(kv.second.front()),
                               [=](hipStream_t st, const int *tab, int nc) {
                                   return launch_chain(fp64, fd, tab, nc, dd, lds, st);
                               });
            }
            for (auto &kv : P.chain_ring) {
                const int shape = std::get<0>(kv.first), mn = std::get<1>(kv.first);
                const size_t lds = L.ring_lds.at(std::make_pair(shape, mn));
                int waves = 1;   // enough for every chain of the group
                for (int dsc : kv.second)
                    waves = std::max(waves, chain_waves(shape, L.fl[frame_of(dsc)].Mt,
                                                        !L.fl[frame_of(dsc)].gcol));
                for (int dd : std::get<2>(kv.first) ? std::vector<int>{kDirFwd, kDirBwd}
                                                   : std::vector<int>{dirs})
                    add_chains(kv.second, P.off_chain_ring.at(kv.first), steps(kv.second.front()),
                               [=](hipStream_t st, const int *tab, int nc) {
                                   return launch_chain_ring(fp64, shape, mn, waves, fd, tab, nc,
                                                            dd, lds, st);
                               });
            }
            deal();
            if (P.kind == kPassPre) {
                const size_t j = L.pre_rounds ? (size_t)P.seg : 0;
                if (pre_ops.size() <= j) pre_ops.resize(j + 1);
                for (size_t k = first_op; k < ops.size(); ++k) pre_ops[j].push_back((int)k);
            }
            if (P.kind != kPassMain) continue;
            // With the sweep in parts, every launch of a main pass but its
            // lattice waits for the newest launch of each sweep direction up
            // to the part after which its checkpoints exist (a part whose
            // rows are empty for every frame has none).  The group's alpha / beta rows are a
            // resource of their own per frame (3 nf + f): the recomputation
            // of the checkpoint segments reads only the pre-pass's Gamma and
            // the checkpoints and writes only the rows, so with Gamma by start
            // index (pre-pass rounds) it runs on stream 3 as soon as the
            // previous group's APP and W have read them, beside that group's
            // adjoint and this group's lattice, followed there by the APP's
            // scale pass (rows in, the scale of the group's own symbols out);
            // the other APP launches and W take both resources.
            auto wait_sweep = [&]() {
                if (!split) return;
                int wf = -1, wb = -1;
                for (int p = 0; p <= P.part; ++p) {
                    wf = std::max(wf, sweep_fwd[p]);
                    wb = std::max(wb, sweep_bwd[p]);
                }
                for (size_t k = first_op; k < ops.size(); ++k) {
                    Op &o = ops[k];
                    // (the group's lattice reads no checkpoint: the first
                    // group's runs while the sweep approaches the middle)
                    if (o.phase != kPhLattice) {
                        if (wf >= 0) o.afters.push_back(wf);
                        if (wb >= 0) o.afters.push_back(wb);
                    }
                    if (o.phase == kPhRechain && L.pre_rounds) {
                        for (int &f : o.frames)
                            if (f < nf) f += 3 * nf;
                        o.stream = kForkStreams;
                        for (const auto &v : pre_ops) o.afters.insert(o.afters.end(), v.begin(), v.end());
                    } else if (o.rows_only && L.pre_rounds) {
                        // the APP's scale pass reads the rows and writes the
                        // scale of the group's own symbols only: it follows
                        // the recomputation on stream 3
                        for (int &f : o.frames)
                            if (f < nf) f += 3 * nf;
                        o.stream = kForkStreams;
                    } else if (o.phase == kPhApp || o.phase == kPhWgrad || o.phase == kPhChain ||
                               o.phase == kPhRechain) {
                        const size_t nfr = o.frames.size();
                        for (size_t x = 0; x < nfr; ++x)
                            if (o.frames[x] < nf) o.frames.push_back(3 * nf + o.frames[x]);
                    }
                }
            };
            if (!P.app_plain.empty()) {
                const size_t lds = L.app_lds;
                add_work(kPhApp, true, P.app_plain, P.off_app,
                         [=](hipStream_t st, const Work *tab, int nb) {
                             return launch_app(fp64, fd, tab, nb, lds, st);
                         });
            }
            for (auto &kv : P.app_scale) {
                const int mn = kv.first;
                const size_t a = ops.size();
                add_work(kPhApp, true, kv.second, P.off_app_scale.at(kv.first),
                         [=](hipStream_t st, const Work *tab, int nb) {
                             return launch_app_scale(mn, fd, tab, nb, st);
                         });
                for (size_t k = a; k < ops.size(); ++k) ops[k].rows_only = true;
            }
            deal();
            for (auto &kv : P.app_mfma) {
                const int mn = kv.first.first, qt = kv.first.second;
                const size_t lds = L.app_mfma_lds.at(kv.first);
                add_work(kPhApp, true, kv.second, P.off_app_mfma.at(kv.first),
                         [=](hipStream_t st, const Work *tab, int nb) {
                             return launch_app_mfma(mn, qt, fd, tab, nb, lds, st);
                         });
            }
            if (!P.app_fin.empty()) deal();
            for (auto &kv : P.app_fin) {
                const int qt = kv.first;
                add_work(kPhApp, true, kv.second, P.off_app_fin.at(kv.first),
                         [=](hipStream_t st, const Work *tab, int nb) {
                             return launch_app_fin(qt, fd, tab, nb, st);
                         });
            }
            for (auto &kv : P.app_tile) {
                const int td = std::get<0>(kv.first), nw = std::get<1>(kv.first),
                          mn = std::get<2>(kv.first);
                const size_t lds = L.app_tile_lds.at(kv.first);
                add_work(kPhApp, true, kv.second, P.off_app_tile.at(kv.first),
                         [=](hipStream_t st, const Work *tab, int nb) {
                             return launch_app_tile(fp64, td, mn, nw, fd, tab, nb, lds, st);
                         });
            }
            deal();
            if (!L.grad) {
                wait_sweep();
                continue;
            }
            for (auto &kv : P.wlat) {
                const int mn = std::get<0>(kv.first), uni = std::get<1>(kv.first),
                          pc = std::get<2>(kv.first);
                add_work(kPhWgrad, true, kv.second, P.off_wlat.at(kv.first),
                         [=](hipStream_t st, const Work *tab, int nb) {
                             return fp64 ? adj_f64_w(mn, uni, pc, fd, tab, nb, st)
                                         : adj_f32_w(mn, uni, pc, fd, tab, nb, st);
                         });
            }
            deal();
            for (auto &kv : P.adj) {
                const int mn = std::get<0>(kv.first), im = std::get<1>(kv.first),
                          da = std::get<2>(kv.first), pc = std::get<3>(kv.first);
                const size_t lds = L.adj_lds.at(kv.first);
                add_work(kPhAdjoint, true, kv.second, P.off_adj.at(kv.first),
                         [=](hipStream_t st, const Work *tab, int nb) {
                             return fp64 ? adj_f64_lattice(mn, im, da, pc, fd, tab, nb, lds, st)
                                         : adj_f32_lattice(mn, im, da, pc, fd, tab, nb, lds, st);
                         });
            }
            deal();
            wait_sweep();
        }
        if (L.grad) {
            const FrameDesc *fdl = at<FrameDesc>(L.passes.back().off_fd);
            add(kPhDparams, {}, true, [=](hipStream_t st) { return launch_dparams(fdl, nf, st); });
        }
        if (flags & MAPDEC_FLAG_SERIAL) forked = false;
        if (!forked)
            for (Op &o : ops) o.stream = 0;
    }
    std::vector<mapdec_frame> frames_;   // host copy of the frame table (build_ops only)

    // Every launch in order on st (with prof, between the events pb[j] and
    // pa[j]).
    hipError_t enqueue_serial(hipStream_t st, bool prof) {
        hipError_t e = prof ? prof_events() : hipSuccess;
        for (size_t j = 0; j < ops.size() && e == hipSuccess; ++j) {
            if (prof) e = hipEventRecord(pb[j], st);
            if (e == hipSuccess) e = ops[j].fn(st);
            if (prof && e == hipSuccess) e = hipEventRecord(pa[j], st);
        }
        return e;
    }

    // The launches spread over st and the forked streams: each launch waits
    // for the last earlier launch that touched any of its frames (event
    // dep[j + 1] follows op j; dep[0] forks from st), and st finally waits
    // for every forked stream.
    hipError_t enqueue_forked(hipStream_t st, bool prof) {
        constexpr int NS = kForkStreams + 1;
        if (prof) {
            const hipError_t e0 = prof_events();
            if (e0 != hipSuccess) return e0;
        }
        hipStream_t sx[NS] = {st};
        for (int x = 1; x < NS; ++x) sx[x] = side[x - 1];
        // per resource (frame, the sweep's forward and backward parts of
        // every frame, the rows of every frame's group): event of its last
        // launch
        std::vector<int> last(4 * (size_t)L.nframes, 0);
        int tail[NS];                         // per stream: event of its last launch
        int seen[NS][NS];                     // newest event of stream y that x waited for
        std::vector<int> ev_stream(ops.size() + 1, 0);
        for (int x = 0; x < NS; ++x) {
            tail[x] = x == 0 ? 0 : -1;
            for (int y = 0; y < NS; ++y) seen[x][y] = -1;
        }
        hipError_t e = hipEventRecord(dep[0], st);
        std::vector<int> need;
        for (size_t j = 0; j < ops.size() && e == hipSuccess; ++j) {
            const Op &o = ops[j];
            const int x = o.stream;
            need.clear();
            if (o.all) {
                for (int y = 0; y < NS; ++y)
                    if (tail[y] >= 0) need.push_back(tail[y]);
            } else {
                for (int f : o.frames) need.push_back(last[f]);
            }
            if (o.after >= 0) need.push_back(o.after + 1);
            for (int a : o.afters) need.push_back(a + 1);
            if (tail[x] < 0) need.push_back(0);   // first launch on a forked stream
            for (int d : need) {
                const int y = ev_stream[d];
                if (y == x || seen[x][y] >= d) continue;
                e = hipStreamWaitEvent(sx[x], dep[d], 0);
                if (e != hipSuccess) break;
                seen[x][y] = d;
            }
            if (e != hipSuccess) break;
            if (prof) e = hipEventRecord(pb[j], sx[x]);
            if (e == hipSuccess) e = o.fn(sx[x]);
            if (prof && e == hipSuccess) e = hipEventRecord(pa[j], sx[x]);
            if (e != hipSuccess) break;
            const int me = (int)j + 1;
            e = hipEventRecord(dep[me], sx[x]);
            ev_stream[me] = x;
            tail[x] = me;
            if (o.all)
                std::fill(last.begin(), last.end(), me);
            else
                for (int f : o.frames) last[f] = me;
        }
        for (int y = 1; y < NS && e == hipSuccess; ++y)
            if (tail[y] > seen[0][y]) e = hipStreamWaitEvent(st, dep[tail[y]], 0);
        return e;
    }

    // Graph capture always takes the one-stream order: a capture that forked
    // onto the plan's streams ended in a host-side crash inside the runtime
    // on its first run, so forking is kept to eager runs.
    hipError_t enqueue(hipStream_t st, bool prof = false, bool capture = false) {
        return (capture || !forked) ? enqueue_serial(st, prof) : enqueue_forked(st, prof);
    }
};

namespace {

// Packs ncb codebooks of q codewords (q n bytes of 0/1 each) into c->cw;
// false if a byte is not 0/1 or a codebook repeats a codeword (each
// encoding must be injective, Sec. II-A).
bool pack_codebooks(mapdec_code *c, int ncb, const uint8_t *bytes) {
    const int q = c->q, n = c->n;
    c->ncb = ncb;
    c->cw.assign((size_t)ncb * q, 0u);
    for (int b = 0; b < ncb; ++b) {
        for (int D = 0; D < q; ++D) {
            uint32_t w = 0;
            for (int r = 0; r < n; ++r) {
                const uint8_t x = bytes[((size_t)b * q + D) * n + r];
                if (x > 1) return false;
                w |= (uint32_t)x << (n - 1 - r);
            }
            c->cw[(size_t)b * q + D] = w;
        }
        std::vector<uint32_t> sorted(c->cw.begin() + (size_t)b * q,
                                     c->cw.begin() + (size_t)(b + 1) * q);
        std::sort(sorted.begin(), sorted.end());
        if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end()) return false;
    }
    return true;
}

}  // namespace

extern "C" {

mapdec_code *mapdec_create(int q, int n, const uint8_t *codebook, double Pi, double Pd,
                           double Ps, int I, int M, int mn) {
    if (!codebook || validate_code_params(q, n, Pi, Pd, Ps, I, M, mn) != MAPDEC_OK) {
        fail(MAPDEC_EINVAL);
        return nullptr;
    }
    mapdec_code *c = new (std::nothrow) mapdec_code;
    if (!c) {
        fail(MAPDEC_ENOMEM);
        return nullptr;
    }
    c->q = q; c->n = n; c->I = I; c->M = M; c->mn = mn;
    c->Pi = Pi; c->Pd = Pd; c->Ps = Ps;
    c->mt_lo = -M; c->mt_hi = M; c->mn_lo = -mn; c->mn_hi = mn;
    if (!pack_codebooks(c, 1, codebook)) {
        delete c;
        fail(MAPDEC_EINVAL);
        return nullptr;
    }
    return c;
}

mapdec_code *mapdec_create_general(int q, int n, int ncb, const uint8_t *codebooks, double Pi,
                                   double Pd, double Ps, int I, int mt_lo, int mt_hi, int mn_lo,
                                   int mn_hi) {
    // Sec. III-B: m_n^- <= 0 <= m_n^+, m_tau^- <= m_n^-, m_tau^+ >= m_n^+
    const bool limits = mn_lo <= 0 && mn_hi >= 0 && mt_lo <= mn_lo && mt_hi >= mn_hi;
    const int M = std::max(-mt_lo, mt_hi), mn = std::max(-mn_lo, mn_hi);
    if (!codebooks || ncb < 1 || !limits ||
        validate_code_params(q, n, Pi, Pd, Ps, I, M, mn) != MAPDEC_OK) {
        fail(MAPDEC_EINVAL);
        return nullptr;
    }
    mapdec_code *c = new (std::nothrow) mapdec_code;
    if (!c) {
        fail(MAPDEC_ENOMEM);
        return nullptr;
    }
    c->q = q; c->n = n; c->I = I; c->M = M; c->mn = mn;
    c->Pi = Pi; c->Pd = Pd; c->Ps = Ps;
    c->mt_lo = mt_lo; c->mt_hi = mt_hi; c->mn_lo = mn_lo; c->mn_hi = mn_hi;
    if (!pack_codebooks(c, ncb, codebooks)) {
        delete c;
        fail(MAPDEC_EINVAL);
        return nullptr;
    }
    return c;
}

mapdec_code *mapdec_with_threshold(const mapdec_code *code, double theta) {
    if (!code || !(theta >= 0.0) || !(theta < 1.0)) {
        fail(MAPDEC_EINVAL);
        return nullptr;
    }
    mapdec_code *c = new (std::nothrow) mapdec_code(*code);
    if (!c) {
        fail(MAPDEC_ENOMEM);
        return nullptr;
    }
    c->theta = theta;
    return c;
}

void mapdec_destroy(mapdec_code *code) { delete code; }

size_t mapdec_workspace_size(const mapdec_frame *frames, int nframes, int precision, int flags,
                             int checkpoint_K) {
    Layout L;
    if (build_layout(frames, nframes, precision, flags, checkpoint_K, L) != MAPDEC_OK) return 0;
    return L.total;
}

}  // extern "C"

namespace {

mapdec_plan *plan_create(const mapdec_frame *frames, int nframes, double *logp, double *dparams,
                         int32_t *status, void *ws, size_t ws_bytes, int precision, int flags,
                         int checkpoint_K, void *stream) {
    if (!logp || !status || !ws || checkpoint_K < 0 ||
        ((flags & MAPDEC_FLAG_GRAD) && !dparams)) {
        fail(MAPDEC_EINVAL);
        return nullptr;
    }
    mapdec_plan *p = new (std::nothrow) mapdec_plan;
    if (!p) {
        fail(MAPDEC_ENOMEM);
        return nullptr;
    }
    int st = build_layout(frames, nframes, precision, flags, checkpoint_K, p->L);
    if (st == MAPDEC_OK && ws_bytes < p->L.total) st = MAPDEC_ESIZE;
    if (st != MAPDEC_OK) {
        delete p;
        fail(st);
        return nullptr;
    }
    const Layout &L = p->L;
    p->ws = static_cast<unsigned char *>(ws);
    p->flags = flags;

    // descriptors and work tables, staged on the host
    std::vector<unsigned char> stage(L.head, 0);
    if (!L.pack.empty())
        std::memcpy(stage.data() + L.off_pack, L.pack.data(), sizeof(Work) * L.pack.size());
    unsigned char *base = p->ws;
    for (const Pass &P : L.passes) {
        FrameDesc *fd = reinterpret_cast<FrameDesc *>(stage.data() + P.off_fd);
        for (int f = 0; f < nframes; ++f) {
            const mapdec_frame &fr = frames[f];
            const mapdec_code *c = fr.code;
            const FrameLayout &F = L.fl[f];
            FrameDesc &d = fd[f];
            d.q = c->q; d.n = c->n; d.N = fr.N; d.rho = fr.rho;
            d.M = c->M; d.mn = c->mn; d.I = c->I; d.tau = c->n * fr.N;
            d.Mt = F.Mt; d.Mn = F.Mn; d.sp = F.sp; d.gsp = F.gsp; d.uniform = fr.prior ? 0 : 1;
            d.nwords = F.nwords; d.imode = frame_imode(c); d.grad = L.grad; d.ck = F.K;
            d.ring_chunk = F.ring_chunk; d.ring_cols = F.ring_cols;
            const double Pt = 1.0 - c->Pi - c->Pd;
            d.a = 0.5 * c->Pi; d.d = c->Pd; d.t1 = Pt * (1.0 - c->Ps); d.t0 = Pt * c->Ps;
            d.Pi = c->Pi; d.Pd = c->Pd; d.Ps = c->Ps;
            d.adj_da = frame_da(fr);
            d.start_prior = fr.start_drift;
            d.end_prior = fr.end_drift;
            d.y = fr.y; d.prior = fr.prior; d.app = fr.app; d.dprior = fr.dprior;
            d.logp = logp + f; d.status = status + f;
            d.dparams = dparams ? dparams + 3 * f : nullptr;
            d.cw = reinterpret_cast<uint32_t *>(base + F.off_cw);
            d.ybits = reinterpret_cast<uint32_t *>(base + F.off_ybits);
            d.R = base + F.off_R;
            d.G = base + F.off_G;
            d.alpha = reinterpret_cast<double *>(base + F.off_alpha);
            d.beta = reinterpret_cast<double *>(base + F.off_beta);
            d.logA = reinterpret_cast<double *>(base + F.off_logA);
            d.logB = reinterpret_cast<double *>(base + F.off_logB);
            d.Zinv = L.grad ? reinterpret_cast<double *>(base + F.off_Zinv) : nullptr;
            // (the MFMA APP keeps its exponent scales there in every plan)
            d.Zexp = (L.grad || F.app_mfma) ? reinterpret_cast<int *>(base + F.off_Zexp) : nullptr;
            d.Up = F.app_mfma ? reinterpret_cast<float *>(base + F.off_up) : nullptr;
            d.sweep_state = F.off_sws ? reinterpret_cast<double *>(base + F.off_sws) : nullptr;
            d.app_parts = F.app_parts;
            d.gacc_all = reinterpret_cast<double *>(base + F.off_gacc);
            d.gacc_n = F.gacc_n;
            d.dq = F.dq;
            d.dsplit = F.dsplit;
            d.Gpart = F.off_gpart ? base + F.off_gpart : nullptr;
            const int j = std::min(P.seg, F.nseg - 1);
            const Segment g = segment_of(fr, F, j);
            d.i0 = g.i0; d.i1 = g.i1; d.s0 = g.s0; d.s1 = g.s1;
            d.gacc = d.gacc_all + 4 * (size_t)F.gacc_first[j];
            d.a_init = fr.start_drift;
            d.b_init = fr.end_drift;
            d.a_fin = d.b_fin = nullptr;
            d.chain_mode = kChainRows;
            d.ck_stride = 0;
            d.wr_init = 3;
            d.percol = F.percol ? 1 : 0;
            d.cwi = F.percol ? c->q : 0;
            d.lim_lo = c->mt_lo;
            d.lim_hi = c->mt_hi;
            d.theta = c->theta;
            d.kept = F.pruned ? base + F.off_kept : nullptr;
            d.cmask = 0;
            for (int k = 0; k < F.Mn; ++k)
                if (k - c->mn >= c->mn_lo && k - c->mn <= c->mn_hi) d.cmask |= 1u << k;
            if (!F.ck) continue;
            const size_t T = L.tsize;
            unsigned char *Gw = base + F.off_Gw;
            double *cka = reinterpret_cast<double *>(base + F.off_ck);
            double *ckb = reinterpret_cast<double *>(base + F.off_ckb);
            if (P.kind == kPassPre) {
                if (!F.gcol) {   // the whole frame, Gamma only
                    d.i0 = 0; d.i1 = fr.N; d.s0 = 0; d.s1 = fr.rho;
                    d.R = nullptr;
                    d.G = Gw;
                    d.gsp = F.spw;
                    d.dq = c->q;
                    d.dsplit = 1;
                } else {           // group j's Gamma into the whole-frame table
                    d.G = Gw + T * (size_t)g.i0 * F.Mt;
                    d.gsp = F.gspw;
                }
            } else if (P.kind == kPassSweep) {
                d.i0 = 0; d.i1 = fr.N; d.s0 = 0; d.s1 = fr.rho;
                d.G = Gw;
                d.gsp = F.gcol ? F.gspw : F.spw;
                d.alpha = cka;
                d.beta = ckb;
                d.chain_mode = kChainSweep;
                d.ck_stride = F.ck;
                if (L.sweep_parts > 1) {   // the forward chain of part P.part
                    const int p = P.part;
                    d.i0 = F.swa[p];
                    d.i1 = F.swa[p + 1];
                    // from the checkpoint the previous parts left (the
                    // start state while no part has covered a row)
                    if (F.swa[p] > 0) d.a_init = cka + (size_t)(F.swa[p] / F.ck) * F.Mt;
                    // Gamma by symbol: the table from the part's first symbol
                    // (the chains address it relative to i0)
                    if (F.gcol) d.G = Gw + T * (size_t)d.i0 * F.Mt;
                }
            } else if (fr.prior) {
                // main pass: Gamma stays in the whole-frame table
                d.G = Gw + T * (size_t)g.i0 * F.Mt;
                d.gsp = F.gspw;
            }
        }
        // the chains of each checkpoint segment of a main pass's groups, or
        // the backward chains of a sweep part
        for (size_t k = 0; k < P.sub_frame.size(); ++k) {
            const int f = P.sub_frame[k], j = P.sub_seg[k];
            const mapdec_frame &fr = frames[f];
            const FrameLayout &F = L.fl[f];
            FrameDesc &d = fd[nframes + k];
            d = fd[f];
            if (P.kind == kPassSweep) {
                double *ckb = reinterpret_cast<double *>(base + F.off_ckb);
                d.i0 = F.swb[j + 1];
                d.i1 = F.swb[j];
                d.b_init = F.swb[j] < fr.N ? ckb + (size_t)(F.swb[j] / F.ck) * F.Mt
                                           : fr.end_drift;
                if (F.gcol) d.G = base + F.off_Gw + L.tsize * (size_t)d.i0 * F.Mt;
                continue;
            }
            const Segment g = segment_of(fr, F, P.seg);
            d.i0 = j * F.ck;
            d.i1 = std::min(fr.N, d.i0 + F.ck);
            d.s0 = 0;
            d.s1 = fr.rho;
            unsigned char *Gw = base + F.off_Gw;
            d.G = F.gcol ? Gw + L.tsize * (size_t)d.i0 * F.Mt : Gw;
            d.gsp = F.gcol ? F.gspw : F.spw;
            d.alpha = fd[f].alpha + (size_t)(d.i0 - g.i0) * F.Mt;
            d.beta = fd[f].beta + (size_t)(d.i0 - g.i0) * F.Mt;
            double *cka = reinterpret_cast<double *>(base + F.off_ck);
            double *ckb = reinterpret_cast<double *>(base + F.off_ckb);
            d.a_init = j > 0 ? cka + (size_t)j * F.Mt : fr.start_drift;
            d.b_init = j + 1 < F.nck ? ckb + (size_t)(j + 1) * F.Mt : fr.end_drift;
            d.a_fin = d.b_fin = nullptr;
            d.chain_mode = kChainSub;
            // rows shared with the neighbouring segment are written by the
            // chain that computes them; each starting row only at the
            // group's ends
            d.wr_init = (d.i0 == g.i0 ? 1 : 0) | (d.i1 == g.i1 ? 2 : 0);
        }
        for (auto &kv : P.wlat)
            std::memcpy(stage.data() + P.off_wlat.at(kv.first), kv.second.data(),
                        sizeof(Work) * kv.second.size());
        for (auto &kv : P.gsum)
            std::memcpy(stage.data() + P.off_gsum.at(kv.first), kv.second.data(),
                        sizeof(Work) * kv.second.size());
        for (auto &kv : P.lat)
            std::memcpy(stage.data() + P.off_lat.at(kv.first), kv.second.data(),
                        sizeof(Work) * kv.second.size());
        for (auto &kv : P.adj)
            std::memcpy(stage.data() + P.off_adj.at(kv.first), kv.second.data(),
                        sizeof(Work) * kv.second.size());
        for (auto &kv : P.gamma)
            std::memcpy(stage.data() + P.off_gamma.at(kv.first), kv.second.data(),
                        sizeof(Work) * kv.second.size());
        for (auto &kv : P.chain_plain)
            std::memcpy(stage.data() + P.off_chain.at(kv.first), kv.second.data(),
                        sizeof(int) * kv.second.size());
        for (auto &kv : P.chain_ring)
            std::memcpy(stage.data() + P.off_chain_ring.at(kv.first), kv.second.data(),
                        sizeof(int) * kv.second.size());
        for (auto &kv : P.app_tile)
            std::memcpy(stage.data() + P.off_app_tile.at(kv.first), kv.second.data(),
                        sizeof(Work) * kv.second.size());
        if (!P.app_plain.empty())
            std::memcpy(stage.data() + P.off_app, P.app_plain.data(),
                        sizeof(Work) * P.app_plain.size());
        for (auto &kv : P.app_scale)
            std::memcpy(stage.data() + P.off_app_scale.at(kv.first), kv.second.data(),
                        sizeof(Work) * kv.second.size());
        for (auto &kv : P.app_mfma)
            std::memcpy(stage.data() + P.off_app_mfma.at(kv.first), kv.second.data(),
                        sizeof(Work) * kv.second.size());
        for (auto &kv : P.app_fin)
            std::memcpy(stage.data() + P.off_app_fin.at(kv.first), kv.second.data(),
                        sizeof(Work) * kv.second.size());
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(p->ws, stage.data(), L.head, hipMemcpyHostToDevice, s);
    p->head_host = std::move(stage);
    {
        HeadOwners &h = head_owners();
        std::lock_guard<std::mutex> g(h.mu);
        h.owner[p->ws] = p;
    }
    // codewords go straight into each frame's region
    for (int f = 0; f < nframes && e == hipSuccess; ++f)
        e = hipMemcpyAsync(base + L.fl[f].off_cw, frames[f].code->cw.data(),
                           sizeof(uint32_t) * frames[f].code->cw.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) {
        p->frames_.assign(frames, frames + nframes);
        p->build_ops();
        p->frames_.clear();
        if (flags & MAPDEC_FLAG_GRAPH) p->forked = false;
        for (int x = 0; p->forked && x < kForkStreams && e == hipSuccess; ++x)
            e = hipStreamCreateWithFlags(&p->side[x], hipStreamNonBlocking);
        if (p->forked) p->dep.reserve(p->ops.size() + 1);
        for (size_t k = 0; p->forked && k <= p->ops.size() && e == hipSuccess; ++k) {
            hipEvent_t x;
            e = hipEventCreateWithFlags(&x, hipEventDisableTiming);
            if (e == hipSuccess) p->dep.push_back(x);
        }
    }
    if (e != hipSuccess) {
        mapdec_plan_destroy(p);
        fail(MAPDEC_EDEVICE);
        return nullptr;
    }
    return p;
}

// Milliseconds per launch of fn: one launch to warm up, then reps launches
// between two events.
hipError_t time_launch(hipStream_t s, hipEvent_t e0, hipEvent_t e1, int reps,
                       const std::function<hipError_t(hipStream_t)> &fn, float &ms) {
    hipError_t e = fn(s);
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = fn(s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    ms /= (float)reps;
    return e;
}

// Caps on the work one bucket's candidates are timed on.
constexpr size_t kTuneAppItems = 8192;   // tiled-APP workgroups
constexpr size_t kTuneChains = 1024;     // ring chains (frames)

// Fills the tune table for every bucket of plan t's frames that has no
// entry yet.  t is a decode-only plan on the caller's workspace: one run of
// it leaves the receiver metric, Gamma and both metric rows of its last
// pass in place; the candidates then re-run that pass's APP tiles and
// chains (which only rewrite outputs the final plan writes again).
int tune_plan(mapdec_plan *t, hipStream_t s) {
    const Layout &L = t->L;
    const size_t lds_limit = device_lds_limit();
    std::map<TuneKey, std::vector<int>> app_b, ring_b;
    {
        TuneTable &T = tune_table();
        std::lock_guard<std::mutex> g(T.mu);
        for (int f = 0; f < L.nframes; ++f) {
            const FrameLayout &F = L.fl[f];
            if (F.app_tiled && !T.app.count(F.app_bucket)) app_b[F.app_bucket].push_back(f);
            // (checkpointed frames' main-pass descriptors hold no whole chain)
            if (F.ring_first >= 0 && !F.ck && !F.pruned &&
                !T.ring.count(F.ring_bucket))
                ring_b[F.ring_bucket].push_back(f);
        }
    }
    if (app_b.empty() && ring_b.empty()) return MAPDEC_OK;
    hipError_t e = t->enqueue_serial(s, false);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return MAPDEC_EDEVICE;

    const Pass &P = L.passes.back();   // main pass over segment 0
    const size_t fd_bytes = align_up(sizeof(FrameDesc) * L.nframes);
    const size_t tab_bytes = std::max(kTuneAppItems * sizeof(Work), kTuneChains * sizeof(int)) +
                             sizeof(Work) * 4096;
    unsigned char *tbuf = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = hipMalloc(&tbuf, fd_bytes + tab_bytes);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    FrameDesc *fd_tmp = reinterpret_cast<FrameDesc *>(tbuf);
    unsigned char *tab_tmp = tbuf + fd_bytes;
    std::vector<FrameDesc> fd_host(L.nframes);
    if (e == hipSuccess)
        e = hipMemcpy(fd_host.data(), t->at<FrameDesc>(P.off_fd), sizeof(FrameDesc) * L.nframes,
                      hipMemcpyDeviceToHost);
    const FrameDesc *fd = t->at<FrameDesc>(P.off_fd);
    const int fp64 = L.fp64;

    for (auto &kv : app_b) {
        if (e != hipSuccess) break;
        const TuneKey &key = kv.first;
        const int q = key[1], n = key[2], mn = key[3], wdef = key[4];
        std::vector<Work> items;
        std::vector<int> used;
        for (int f : kv.second) {
            const FrameDesc &d = fd_host[f];
            const int nb = (d.i1 - d.i0 + kAppTI - 1) / kAppTI;
            if (!items.empty() && items.size() + nb > kTuneAppItems) break;
            for (int b = 0; b < nb && items.size() < kTuneAppItems; ++b) items.push_back(Work{f, b});
            used.push_back(f);
        }
        e = hipMemcpy(tab_tmp, items.data(), sizeof(Work) * items.size(), hipMemcpyHostToDevice);
        const Work *tab = reinterpret_cast<const Work *>(tab_tmp);
        const int nb = (int)items.size();
        std::pair<int, int> best(app_tile_td(q, L.tsize), wdef);
        float best_ms = -1.f;
        for (int td = 2; td <= app_tile_td(q, L.tsize) && e == hipSuccess; td *= 2) {
            std::vector<int> waves{wdef};
            if ((wdef + 1) / 2 != wdef) waves.push_back((wdef + 1) / 2);
            for (int nw : waves) {
                size_t lds = 0;
                for (int f : used)
                    lds = std::max(lds, app_tile_lds(L.fl[f].Mt, mn, n, q, L.tsize, td, nw));
                if (lds > lds_limit) continue;
                float ms = 0.f;
                e = time_launch(s, e0, e1, 3, [&](hipStream_t st) {
                    return launch_app_tile(fp64, td, mn, nw, fd, tab, nb, lds, st);
                }, ms);
                if (e != hipSuccess) break;
                if (best_ms < 0.f || ms < best_ms) {
                    best_ms = ms;
                    best = std::make_pair(td, nw);
                }
            }
        }
        if (e == hipSuccess) {
            TuneTable &T = tune_table();
            std::lock_guard<std::mutex> g(T.mu);
            T.app[key] = best;
        }
    }

    for (auto &kv : ring_b) {
        if (e != hipSuccess) break;
        const TuneKey &key = kv.first;
        const int mn = key[3], first = key[4];
        std::vector<int> used(kv.second.begin(),
                              kv.second.begin() + std::min(kv.second.size(), kTuneChains));
        int best = first;
        float best_ms = -1.f;
        for (int shape = first; shape < kNumRingShapes && shape <= first + 2 && e == hipSuccess;
             ++shape) {
            std::vector<FrameDesc> patched = fd_host;
            size_t lds = 0;
            bool ok = true;
            int waves = 1;
            for (int f : used) {
                const FrameLayout &F = L.fl[f];
                const bool uni = !F.gcol;
                if (64 * kRingShapes[shape].nw * kRingShapes[shape].spl >= F.Mt)
                    waves = std::max(waves, chain_waves(shape, F.Mt, uni));
                int ch, co;
                size_t l;
                if (!ring_fit(shape, F.Mt, F.Mn, uni ? fd_host[f].n : F.Mt, mn, uni, L.tsize,
                              lds_limit, ch, co, l)) {
                    ok = false;
                    break;
                }
                patched[f].ring_chunk = ch;
                patched[f].ring_cols = co;
                lds = std::max(lds, l);
            }
            if (!ok) continue;
            e = hipMemcpy(fd_tmp, patched.data(), sizeof(FrameDesc) * L.nframes,
                          hipMemcpyHostToDevice);
            if (e == hipSuccess)
                e = hipMemcpy(tab_tmp, used.data(), sizeof(int) * used.size(), hipMemcpyHostToDevice);
            if (e != hipSuccess) break;
            const int *list = reinterpret_cast<const int *>(tab_tmp);
            const int nc = (int)used.size();
            float ms = 0.f;
            e = time_launch(s, e0, e1, 2, [&](hipStream_t st) {
                return launch_chain_ring(fp64, shape, mn, waves, fd_tmp, list, nc, kDirBoth, lds,
                                         st);
            }, ms);
            if (e != hipSuccess) break;
            if (best_ms < 0.f || ms < best_ms) {
                best_ms = ms;
                best = shape;
            }
        }
        if (e == hipSuccess) {
            TuneTable &T = tune_table();
            std::lock_guard<std::mutex> g(T.mu);
            T.ring[key] = best;
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (tbuf) hipFree(tbuf);
    return e == hipSuccess ? MAPDEC_OK : MAPDEC_EDEVICE;
}

}  // namespace

extern "C" {

mapdec_plan *mapdec_plan_create(const mapdec_frame *frames, int nframes, double *logp,
                                double *dparams, int32_t *status, void *ws, size_t ws_bytes,
                                int precision, int flags, int checkpoint_K, void *stream) {
    if (flags & MAPDEC_FLAG_TUNE) {
        // tune on a decode-only plan, then lay out the real one with the choices
        mapdec_plan *t = plan_create(frames, nframes, logp, nullptr, status, ws, ws_bytes,
                                     precision, MAPDEC_FLAG_SERIAL, checkpoint_K, stream);
        if (!t) return nullptr;
        const int st = tune_plan(t, static_cast<hipStream_t>(stream));
        mapdec_plan_destroy(t);
        if (st != MAPDEC_OK) {
            fail(st);
            return nullptr;
        }
    }
    return plan_create(frames, nframes, logp, dparams, status, ws, ws_bytes, precision,
                       flags & ~MAPDEC_FLAG_TUNE, checkpoint_K, stream);
}

int mapdec_tune_entries(void) {
    TuneTable &T = tune_table();
    std::lock_guard<std::mutex> g(T.mu);
    return (int)(T.app.size() + T.ring.size());
}

void mapdec_tune_reset(void) {
    TuneTable &T = tune_table();
    std::lock_guard<std::mutex> g(T.mu);
    T.app.clear();
    T.ring.clear();
}

int mapdec_plan_run(mapdec_plan *p, void *stream) {
    if (!p) return MAPDEC_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = p->own_head(s);
    if (p->flags & MAPDEC_FLAG_GRAPH) {
        if (!p->exec) {
            if (!p->cap_stream) e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
            if (e == hipSuccess) e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                hipError_t e2 = p->enqueue(p->cap_stream, false, true);
                e = hipStreamEndCapture(p->cap_stream, &p->graph);
                if (e2 != hipSuccess) e = e2;
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
        }
        if (e == hipSuccess) e = hipGraphLaunch(p->exec, s);
    } else {
        e = p->enqueue(s);
    }
    p->last_stream = s;
    p->ran = true;
    return e == hipSuccess ? MAPDEC_OK : MAPDEC_EDEVICE;
}

int mapdec_plan_profile(mapdec_plan *p, void *stream, float *phase_ms, int max_phases) {
    if (!p || (max_phases > 0 && !phase_ms)) return -MAPDEC_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = p->own_head(s);
    if (e == hipSuccess) e = p->enqueue(s, true);
    p->last_stream = s;
    p->ran = true;
    const int nph = kNumPhases;
    for (int k = 0; k < max_phases && k < nph; ++k) phase_ms[k] = 0.f;
    if (e == hipSuccess) e = hipStreamSynchronize(s);   // s has joined every forked stream
    // a phase's time is the sum of its launches' durations
    for (size_t j = 0; j < p->ops.size() && e == hipSuccess; ++j) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, p->pb[j], p->pa[j]);
        if (p->ops[j].phase < max_phases) phase_ms[p->ops[j].phase] += ms;
    }
    return e == hipSuccess ? nph : -MAPDEC_EDEVICE;
}

int mapdec_plan_launches(const mapdec_plan *p, int phase) {
    if (!p) return -MAPDEC_EINVAL;
    int n = 0;
    for (const Op &o : p->ops) n += o.phase == phase ? 1 : 0;
    return n;
}

const char *mapdec_phase_name(int phase) {
    static const char *names[] = {"pack", "lattice", "gamma", "chain", "app",
                                  "wgrad", "adjoint", "dparams", "rechain"};
    return (phase >= 0 && phase < (int)(sizeof(names) / sizeof(names[0]))) ? names[phase]
                                                                           : nullptr;
}

void mapdec_plan_destroy(mapdec_plan *p) {
    if (!p) return;
    {
        HeadOwners &h = head_owners();
        std::lock_guard<std::mutex> g(h.mu);
        auto it = h.owner.find(p->ws);
        if (it != h.owner.end() && it->second == p) h.owner.erase(it);
    }
    if (p->ran) hipStreamSynchronize(p->last_stream);
    for (hipStream_t x : p->side)
        if (x) {
            hipStreamSynchronize(x);
            hipStreamDestroy(x);
        }
    for (hipEvent_t x : p->dep) hipEventDestroy(x);
    for (hipEvent_t x : p->pb) hipEventDestroy(x);
    for (hipEvent_t x : p->pa) hipEventDestroy(x);
    if (p->exec) hipGraphExecDestroy(p->exec);
    if (p->graph) hipGraphDestroy(p->graph);
    if (p->cap_stream) hipStreamDestroy(p->cap_stream);
    delete p;
}

int mapdec_decode(const mapdec_frame *frames, int nframes, double *logp, int32_t *status,
                  void *ws, size_t ws_bytes, int precision, void *stream) {
    mapdec_plan *p = mapdec_plan_create(frames, nframes, logp, nullptr, status, ws, ws_bytes,
                                        precision, 0, 0, stream);
    if (!p) return g_last_error;
    int st = mapdec_plan_run(p, stream);
    mapdec_plan_destroy(p);
    return st;
}

int mapdec_grad(const mapdec_frame *frames, int nframes, double *logp, double *dparams,
                int32_t *status, void *ws, size_t ws_bytes, int checkpoint_K, int precision,
                void *stream) {
    mapdec_plan *p = mapdec_plan_create(frames, nframes, logp, dparams, status, ws, ws_bytes,
                                        precision, MAPDEC_FLAG_GRAD, checkpoint_K, stream);
    if (!p) return g_last_error;
    int st = mapdec_plan_run(p, stream);
    mapdec_plan_destroy(p);
    return st;
}

int mapdec_decode_noalloc(const mapdec_frame *frames, int nframes, double *logp,
                          int32_t *status, int precision, void *stream) {
    Layout L;
    const int v = build_layout(frames, nframes, precision, MAPDEC_FLAG_SERIAL, 0, L);
    if (v != MAPDEC_OK) return v;
    if (L.total > scratch_bytes()) return MAPDEC_ESIZE;
    void *ws = nullptr;
    if (scratch_address(&ws) != hipSuccess) return MAPDEC_EDEVICE;
    // the plan's only device memory is the scratch array; a serial plan
    // creates no streams or events either
    mapdec_plan *p = mapdec_plan_create(frames, nframes, logp, nullptr, status, ws,
                                        scratch_bytes(), precision, MAPDEC_FLAG_SERIAL, 0, stream);
    if (!p) return g_last_error;
    int st = mapdec_plan_run(p, stream);
    mapdec_plan_destroy(p);
    return st;
}

size_t mapdec_noalloc_limit(void) { return scratch_bytes(); }

int mapdec_last_error(void) { return g_last_error; }

const char *mapdec_strerror(int status) {
    switch (status) {
        case MAPDEC_OK: return "MAPDEC_OK";
        case MAPDEC_EINVAL: return "MAPDEC_EINVAL: invalid argument";
        case MAPDEC_EDRIFT: return "MAPDEC_EDRIFT: end drift outside [-M, M]";
        case MAPDEC_ENOPATH: return "MAPDEC_ENOPATH: P(y) = 0 under the truncated model";
        case MAPDEC_ENOMEM: return "MAPDEC_ENOMEM: allocation failed";
        case MAPDEC_ESIZE: return "MAPDEC_ESIZE: workspace too small";
        case MAPDEC_EDEVICE: return "MAPDEC_EDEVICE: HIP runtime error";
        case MAPDEC_EUNSUPPORTED: return "MAPDEC_EUNSUPPORTED: beyond the library's kernel limits";
        default: return "unknown mapdec status";
    }
}

int mapdec_version(void) { return MAPDEC_VERSION; }

}  // extern "C"
