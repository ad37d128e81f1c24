// Host side of libmapdec: validation, workspace layout, descriptor upload,
// launch sequence and HIP-graph replay.  See include/mapdec.h for the ABI.
#include "mapdec.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "kernels.h"

using namespace mapdec;

struct mapdec_code {
    int q, n, I, M, mn;
    double Pi, Pd, Ps;
    std::vector<uint32_t> cw;   // codeword D: bit (n-1-r) = C(D)[r]
};

namespace {

thread_local int g_last_error = MAPDEC_OK;

int fail(int st) {
    g_last_error = st;
    return st;
}

constexpr size_t kAlign = 256;
constexpr int kMaxPhases = 8;
size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

int validate_code_params(int q, int n, double Pi, double Pd, double Ps, int I, int M, int mn) {
    if (n < 1 || n > 30 || q < 2 || q > (1 << n)) return MAPDEC_EINVAL;
    if (!(Pi >= 0.0) || !(Pd >= 0.0) || !(Ps >= 0.0) || !(Ps <= 1.0)) return MAPDEC_EINVAL;
    if (!(Pi + Pd < 1.0)) return MAPDEC_EINVAL;
    if (I < 0 || mn < 0 || M < mn) return MAPDEC_EINVAL;
    return MAPDEC_OK;
}

// Sizes of one frame's workspace pieces.
struct FrameLayout {
    int nwords, sp, Mt, Mn, lat_blocks, pack_blocks, gamma_blocks;
    int ring_chunk = 0, ring_cols = 0;
    size_t off_cw, off_ybits, off_R, off_G, off_alpha, off_beta, off_logA, off_logB, off_Zinv,
        off_gacc, end;
};

struct Layout {
    int nframes = 0, fp64 = 0, grad = 0;
    size_t tsize = 4;
    size_t off_fd = 0, off_pack = 0, off_gamma = 0, off_chain = 0, off_app = 0, head = 0, total = 0;
    int n_pack = 0, n_gamma = 0;
    // lattice work grouped by template instance (mn, imode)
    std::map<std::pair<int, int>, std::vector<Work>> lat;
    std::map<std::pair<int, int>, size_t> off_lat;
    std::map<std::pair<int, int>, int> lat_nmax;   // longest codeword per group
    // adjoint sweep work grouped by (mn, imode, accumulates d/da)
    std::map<std::tuple<int, int, int>, std::vector<Work>> adj;
    std::map<std::tuple<int, int, int>, size_t> off_adj, adj_lds;
    size_t chain_lds = 0, app_lds = 0;
    // chains: single-wave ring kernel grouped by states per lane, else the
    // workgroup kernel
    std::vector<int> chain_plain;
    // keyed by (states per lane, mn)
    std::map<std::pair<int, int>, std::vector<int>> chain_ring;
    std::map<std::pair<int, int>, size_t> off_chain_ring, ring_lds;
    // tiled APP work grouped by (symbols per wave, waves per workgroup, mn);
    // frames whose rows do not fit in LDS use the one-wave APP kernel
    std::map<std::tuple<int, int, int>, std::vector<Work>> app_tile;
    std::map<std::tuple<int, int, int>, size_t> off_app_tile, app_tile_lds;
    std::vector<Work> app_plain;
    std::vector<FrameLayout> fl;
};

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

// Ring-chain parameters for a uniform-prior frame (workgroup shape, steps
// per prefetch chunk, ring slots, LDS bytes); false when the frame needs
// the plain workgroup chain kernel instead.
bool ring_params(int Mt, int Mn, int n, int mn, size_t tsize, size_t lds_limit, int &shape,
                 int &chunk, int &cols, size_t &lds) {
    shape = -1;
    for (int k = 0; k < kNumRingShapes; ++k)
        if (64 * kRingShapes[k].nw * kRingShapes[k].spl >= Mt) {
            shape = k;
            break;
        }
    if (shape < 0) return false;
    const int nt = 64 * kRingShapes[shape].nw, slots = nt * kRingShapes[shape].spl;
    // ring: a power of two covering the window of at least 8 steps; the
    // chunk is as long as the ring and the prefetch registers allow
    cols = 1;
    while (cols < Mt + n * 7) cols *= 2;
    chunk = std::min({(cols - Mt) / n + 1, (nt * kRingPrefetchRegs) / (n * Mn), 64});
    if (chunk < 1) return false;
    const size_t roww = (size_t)slots + 2 * mn;
    const size_t rphys = ring_duplicates(slots) ? cols + roww : cols;
    // FP64 rows and wave partials, Gamma ring in the batch precision
    lds = (2 * roww + 2 * kRingShapes[shape].nw) * sizeof(double) + rphys * Mn * tsize;
    return lds <= lds_limit;
}

int frame_imode(const mapdec_code *c) { return c->I <= 2 ? 0 : 1; }

// LDS bytes one workgroup may use on the current device (64 KiB when the
// device cannot be queried, e.g. on a host without a GPU).
size_t device_lds_limit() {
    static thread_local int cached_dev = -1;
    static thread_local size_t cached = 65536;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    if (dev != cached_dev) {
        int v = 0;
        cached = (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) ==
                      hipSuccess && v > 0)
                     ? (size_t)v
                     : 65536;
        cached_dev = dev;
    }
    return cached;
}

// Validates the frames and lays out the workspace.
int build_layout(const mapdec_frame *frames, int nframes, int precision, int flags, Layout &L) {
    if (!frames || nframes < 1) return MAPDEC_EINVAL;
    if (precision != MAPDEC_FP32 && precision != MAPDEC_FP64) return MAPDEC_EINVAL;
    L.nframes = nframes;
    L.fp64 = precision == MAPDEC_FP64;
    L.grad = (flags & MAPDEC_FLAG_GRAD) != 0;
    L.tsize = L.fp64 ? 8 : 4;
    L.fl.resize(nframes);
    size_t max_chain = 0, max_app = 0;
    for (int f = 0; f < nframes; ++f) {
        const mapdec_frame &fr = frames[f];
        const mapdec_code *c = fr.code;
        if (!c || fr.N < 1 || fr.rho < 0 || (fr.rho > 0 && !fr.y)) return MAPDEC_EINVAL;
        const long long tau = (long long)c->n * fr.N;
        if (tau > (1LL << 30) || fr.rho > (1 << 30)) return MAPDEC_EUNSUPPORTED;
        if (std::llabs((long long)fr.rho - tau) > c->M) return MAPDEC_EDRIFT;
        if (c->n > kMaxN || c->mn > kMaxMn || c->q > kMaxQ) return MAPDEC_EUNSUPPORTED;
        FrameLayout &F = L.fl[f];
        F.Mt = 2 * c->M + 1;
        F.Mn = 2 * c->mn + 1;
        F.sp = (int)(((size_t)fr.rho + 1 + 63) / 64 * 64);
        F.nwords = (fr.rho + 63) / 32 + 2;
        F.pack_blocks = (F.nwords + kPackWords - 1) / kPackWords;
        F.lat_blocks = (fr.rho + 1 + kLatticeLanes - 1) / kLatticeLanes;
        F.gamma_blocks = fr.prior ? fr.N * ((F.Mt + kGammaLanes - 1) / kGammaLanes) : 0;
        L.n_pack += F.pack_blocks;
        L.n_gamma += F.gamma_blocks;
        {
            const size_t tl = app_tile_lds(F.Mt, c->mn, c->n, c->q, L.tsize);
            // the tile kernel addresses R with 32-bit byte offsets
            const bool fits = (double)c->q * F.Mn * F.sp * L.tsize < 2147483648.0;
            if (fits && tl <= device_lds_limit()) {
                const int td = app_tile_td(c->q, L.tsize);
                const auto key = std::make_tuple(td, app_tile_waves(F.Mt, c->n), c->mn);
                auto &v = L.app_tile[key];
                for (int b = 0; b * kAppTI < fr.N; ++b) v.push_back(Work{f, b});
                L.app_tile_lds[key] = std::max(L.app_tile_lds[key], tl);
            } else {
                for (int i = 0; i < fr.N; ++i) L.app_plain.push_back(Work{f, i});
                max_app = std::max(max_app, (2 * (size_t)F.Mt + 2 * c->mn + c->q) * sizeof(double));
            }
        }
        const size_t W = (size_t)F.Mt + 2 * c->mn;
        int spl = 0;
        size_t rlds = 0;
        if (!fr.prior && ring_params(F.Mt, F.Mn, c->n, c->mn, L.tsize, device_lds_limit(),
                                     spl, F.ring_chunk, F.ring_cols, rlds)) {
            const auto key = std::make_pair(spl, c->mn);
            L.chain_ring[key].push_back(f);
            L.ring_lds[key] = std::max(L.ring_lds[key], rlds);
        } else {
            F.ring_chunk = F.ring_cols = 0;
            L.chain_plain.push_back(f);
            max_chain = std::max(max_chain, (2 * W + 16) * sizeof(double));
        }
        auto key = std::make_pair(c->mn, frame_imode(c));
        L.lat_nmax[key] = std::max(L.lat_nmax[key], c->n);
        auto &v = L.lat[key];
        for (int b = 0; b < F.lat_blocks; ++b) v.push_back(Work{f, b * kLatticeLanes});
        if (L.grad) {
            const auto akey = std::make_tuple(c->mn, frame_imode(c),
                                              adjoint_needs_da(c->Pi, c->Pd) ? 1 : 0);
            auto &av = L.adj[akey];
            for (int b = 0; b < F.lat_blocks; ++b) av.push_back(Work{f, b * kLatticeLanes});
            const size_t al = adjoint_lds(c->n, c->mn, L.tsize);
            if (al > device_lds_limit()) return MAPDEC_EUNSUPPORTED;
            L.adj_lds[akey] = std::max(L.adj_lds[akey], al);
        }
    }
    if (max_chain > 65536 || max_app > 65536) return MAPDEC_EUNSUPPORTED;
    L.chain_lds = max_chain;
    L.app_lds = max_app;

    // head: descriptors and work tables
    size_t off = 0;
    L.off_fd = off;
    off = align_up(off + sizeof(FrameDesc) * nframes);
    L.off_pack = off;
    off = align_up(off + sizeof(Work) * L.n_pack);
    for (auto &kv : L.lat) {
        L.off_lat[kv.first] = off;
        off = align_up(off + sizeof(Work) * kv.second.size());
    }
    for (auto &kv : L.adj) {
        L.off_adj[kv.first] = off;
        off = align_up(off + sizeof(Work) * kv.second.size());
    }
    L.off_gamma = off;
    off = align_up(off + sizeof(Work) * L.n_gamma);
    L.off_chain = off;
    off = align_up(off + sizeof(int) * L.chain_plain.size());
    for (auto &kv : L.chain_ring) {
        L.off_chain_ring[kv.first] = off;
        off = align_up(off + sizeof(int) * kv.second.size());
    }
    for (auto &kv : L.app_tile) {
        kv.second = xcd_order(kv.second);
        L.off_app_tile[kv.first] = off;
        off = align_up(off + sizeof(Work) * kv.second.size());
    }
    L.off_app = off;
    off = align_up(off + sizeof(Work) * L.app_plain.size());
    L.head = off;

    // per-frame regions
    for (int f = 0; f < nframes; ++f) {
        const mapdec_frame &fr = frames[f];
        const mapdec_code *c = fr.code;
        FrameLayout &F = L.fl[f];
        const size_t T = L.tsize;
        F.off_cw = off;
        off = align_up(off + sizeof(uint32_t) * c->q);
        F.off_ybits = off;
        off = align_up(off + sizeof(uint32_t) * F.nwords);
        F.off_R = off;
        off = align_up(off + T * c->q * F.Mn * (size_t)F.sp);
        F.off_G = off;
        off = align_up(off + T * (fr.prior ? (size_t)fr.N * F.Mn * F.Mt : (size_t)F.Mn * F.sp));
        F.off_alpha = off;   // metric rows are FP64 at every precision
        off = align_up(off + sizeof(double) * (size_t)(fr.N + 1) * F.Mt);
        F.off_beta = off;
        off = align_up(off + sizeof(double) * (size_t)(fr.N + 1) * F.Mt);
        F.off_logA = off;
        off = align_up(off + sizeof(double) * (fr.N + 1));
        F.off_logB = off;
        off = align_up(off + sizeof(double) * (fr.N + 1));
        F.off_Zinv = off;
        off = align_up(off + sizeof(double) * fr.N);
        F.off_gacc = off;
        off = align_up(off + sizeof(double) * 4 * F.lat_blocks);
        F.end = off;
    }
    L.total = off;
    return MAPDEC_OK;
}

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

    hipEvent_t ev[kMaxPhases + 1] = {};
    bool have_events = false;

    // Enqueues every launch of one run.  With ev != nullptr an event is
    // recorded before the first phase and after each phase.
    hipError_t enqueue(hipStream_t st, hipEvent_t *ev = nullptr, int *nphases = nullptr) const {
        const FrameDesc *fd = at<FrameDesc>(L.off_fd);
        hipError_t e = hipSuccess;
        int k = 0;
        auto mark = [&]() {
            if (ev && e == hipSuccess) e = hipEventRecord(ev[k], st);
            ++k;
        };
        mark();
        e = launch_init(fd, L.nframes, st);   // phase "pack"
        if (e == hipSuccess) e = launch_pack(fd, at<Work>(L.off_pack), L.n_pack, st);
        mark();
        for (auto &kv : L.lat) {               // phase "lattice"
            if (e != hipSuccess) break;
            e = launch_lattice(L.fp64, kv.first.first, kv.first.second, fd,
                               at<Work>(L.off_lat.at(kv.first)), (int)kv.second.size(), st);
        }
        mark();
        if (e == hipSuccess)                   // phase "gamma"
            e = launch_gamma(L.fp64, fd, at<Work>(L.off_gamma), L.n_gamma, st);
        mark();
        if (e == hipSuccess)                   // phase "chain"
            e = launch_chain(L.fp64, fd, at<int>(L.off_chain), (int)L.chain_plain.size(),
                             L.chain_lds, st);
        for (auto &kv : L.chain_ring) {
            if (e != hipSuccess) break;
            e = launch_chain_ring(L.fp64, kv.first.first, kv.first.second, fd,
                                  at<int>(L.off_chain_ring.at(kv.first)),
                                  (int)kv.second.size(), L.ring_lds.at(kv.first), st);
        }
        mark();
        if (e == hipSuccess)                   // phase "app"
            e = launch_app(L.fp64, fd, at<Work>(L.off_app), (int)L.app_plain.size(), L.app_lds,
                           st);
        for (auto &kv : L.app_tile) {
            if (e != hipSuccess) break;
            e = launch_app_tile(L.fp64, std::get<0>(kv.first), std::get<2>(kv.first),
                                std::get<1>(kv.first), fd, at<Work>(L.off_app_tile.at(kv.first)),
                                (int)kv.second.size(), L.app_tile_lds.at(kv.first), st);
        }
        mark();
        if (L.grad) {
            for (auto &kv : L.lat) {           // phase "wgrad"
                if (e != hipSuccess) break;
                const Work *tab = at<Work>(L.off_lat.at(kv.first));
                const int mn = kv.first.first;
                e = L.fp64 ? adj_f64_w(mn, fd, tab, (int)kv.second.size(), st)
                           : adj_f32_w(mn, fd, tab, (int)kv.second.size(), st);
            }
            mark();
            for (auto &kv : L.adj) {           // phase "adjoint"
                if (e != hipSuccess) break;
                const Work *tab = at<Work>(L.off_adj.at(kv.first));
                const int mn = std::get<0>(kv.first), imode = std::get<1>(kv.first),
                          da = std::get<2>(kv.first);
                const size_t lds = L.adj_lds.at(kv.first);
                const int nb = (int)kv.second.size();
                e = L.fp64 ? adj_f64_lattice(mn, imode, da, fd, tab, nb, lds, st)
                           : adj_f32_lattice(mn, imode, da, fd, tab, nb, lds, st);
            }
            mark();
            if (e == hipSuccess) e = launch_dparams(fd, L.nframes, st);   // phase "dparams"
            mark();
        }
        if (nphases) *nphases = k - 1;
        return e;
    }
};

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
    c->cw.resize(q);
    for (int D = 0; D < q; ++D) {
        uint32_t w = 0;
        for (int r = 0; r < n; ++r) {
            const uint8_t b = codebook[(size_t)D * n + r];
            if (b > 1) {
                delete c;
                fail(MAPDEC_EINVAL);
                return nullptr;
            }
            w |= (uint32_t)b << (n - 1 - r);
        }
        c->cw[D] = w;
    }
    std::vector<uint32_t> sorted = c->cw;
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end()) {
        delete c;
        fail(MAPDEC_EINVAL);   // the encoding must be injective
        return nullptr;
    }
    return c;
}

void mapdec_destroy(mapdec_code *code) { delete code; }

size_t mapdec_workspace_size(const mapdec_frame *frames, int nframes, int precision, int flags) {
    Layout L;
    if (build_layout(frames, nframes, precision, flags, L) != MAPDEC_OK) return 0;
    return L.total;
}

mapdec_plan *mapdec_plan_create(const mapdec_frame *frames, int nframes, double *logp,
                                double *dparams, int32_t *status, void *ws, size_t ws_bytes,
                                int precision, int flags, int checkpoint_K, void *stream) {
    if (!logp || !status || !ws || checkpoint_K < 0 ||
        ((flags & MAPDEC_FLAG_GRAD) && !dparams)) {
        fail(MAPDEC_EINVAL);
        return nullptr;
    }
    if (checkpoint_K > 0) {   // checkpointed forward metric: not part of this build yet
        fail(MAPDEC_EUNSUPPORTED);
        return nullptr;
    }
    mapdec_plan *p = new (std::nothrow) mapdec_plan;
    if (!p) {
        fail(MAPDEC_ENOMEM);
        return nullptr;
    }
    int st = build_layout(frames, nframes, precision, flags, p->L);
    if (st == MAPDEC_OK && ws_bytes < p->L.total) st = MAPDEC_ESIZE;
    if (st != MAPDEC_OK) {
        delete p;
        fail(st);
        return nullptr;
    }
    const Layout &L = p->L;
    p->ws = static_cast<unsigned char *>(ws);
    p->flags = flags;

    // descriptors, work tables and codewords, staged on the host
    std::vector<unsigned char> stage(L.head, 0);
    FrameDesc *fd = reinterpret_cast<FrameDesc *>(stage.data() + L.off_fd);
    Work *pack = reinterpret_cast<Work *>(stage.data() + L.off_pack);
    Work *gam = reinterpret_cast<Work *>(stage.data() + L.off_gamma);
    int *chain = reinterpret_cast<int *>(stage.data() + L.off_chain);
    Work *app = reinterpret_cast<Work *>(stage.data() + L.off_app);
    int ip = 0, ig = 0;
    unsigned char *base = p->ws;
    for (int f = 0; f < nframes; ++f) {
        const mapdec_frame &fr = frames[f];
        const mapdec_code *c = fr.code;
        const FrameLayout &F = L.fl[f];
        FrameDesc &d = fd[f];
        d.q = c->q; d.n = c->n; d.N = fr.N; d.rho = fr.rho;
        d.M = c->M; d.mn = c->mn; d.I = c->I; d.tau = c->n * fr.N;
        d.Mt = F.Mt; d.Mn = F.Mn; d.sp = F.sp; d.uniform = fr.prior ? 0 : 1;
        d.nwords = F.nwords; d.imode = frame_imode(c); d.grad = L.grad; d.ck = 0;
        d.ring_chunk = F.ring_chunk; d.ring_cols = F.ring_cols;
        const double Pt = 1.0 - c->Pi - c->Pd;
        d.a = 0.5 * c->Pi; d.d = c->Pd; d.t1 = Pt * (1.0 - c->Ps); d.t0 = Pt * c->Ps;
        d.Pi = c->Pi; d.Pd = c->Pd; d.Ps = c->Ps;
        d.lat_blocks = F.lat_blocks;
        d.adj_da = adjoint_needs_da(c->Pi, c->Pd) ? 1 : 0;
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
        d.gacc = reinterpret_cast<double *>(base + F.off_gacc);
        for (int b = 0; b < F.pack_blocks; ++b) pack[ip++] = Work{f, b * kPackWords};
        for (int b = 0; b < F.gamma_blocks; ++b) gam[ig++] = Work{f, b};


    }
    for (auto &kv : L.lat)
        std::memcpy(stage.data() + L.off_lat.at(kv.first), kv.second.data(),
                    sizeof(Work) * kv.second.size());
    for (auto &kv : L.adj)
        std::memcpy(stage.data() + L.off_adj.at(kv.first), kv.second.data(),
                    sizeof(Work) * kv.second.size());
    if (!L.app_plain.empty())
        std::memcpy(app, L.app_plain.data(), sizeof(Work) * L.app_plain.size());
    for (auto &kv : L.app_tile)
        std::memcpy(stage.data() + L.off_app_tile.at(kv.first), kv.second.data(),
                    sizeof(Work) * kv.second.size());
    if (!L.chain_plain.empty())
        std::memcpy(chain, L.chain_plain.data(), sizeof(int) * L.chain_plain.size());
    for (auto &kv : L.chain_ring)
        std::memcpy(stage.data() + L.off_chain_ring.at(kv.first), kv.second.data(),
                    sizeof(int) * kv.second.size());
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(p->ws, stage.data(), L.head, hipMemcpyHostToDevice, s);
    // codewords go straight into each frame's region
    for (int f = 0; f < nframes && e == hipSuccess; ++f)
        e = hipMemcpyAsync(base + L.fl[f].off_cw, frames[f].code->cw.data(),
                           sizeof(uint32_t) * frames[f].code->q, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        delete p;
        fail(MAPDEC_EDEVICE);
        return nullptr;
    }
    return p;
}

int mapdec_plan_run(mapdec_plan *p, void *stream) {
    if (!p) return MAPDEC_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
    if (p->flags & MAPDEC_FLAG_GRAPH) {
        if (!p->exec) {
            if (!p->cap_stream) e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
            if (e == hipSuccess) e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                hipError_t e2 = p->enqueue(p->cap_stream);
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
    hipError_t e = hipSuccess;
    if (!p->have_events) {
        for (int k = 0; k <= kMaxPhases && e == hipSuccess; ++k) e = hipEventCreate(&p->ev[k]);
        if (e != hipSuccess) return -MAPDEC_EDEVICE;
        p->have_events = true;
    }
    int nph = 0;
    e = p->enqueue(s, p->ev, &nph);
    p->last_stream = s;
    if (e == hipSuccess) e = hipEventSynchronize(p->ev[nph]);
    for (int k = 0; k < nph && k < max_phases && e == hipSuccess; ++k)
        e = hipEventElapsedTime(&phase_ms[k], p->ev[k], p->ev[k + 1]);
    return e == hipSuccess ? nph : -MAPDEC_EDEVICE;
}

const char *mapdec_phase_name(int phase) {
    static const char *names[] = {"pack", "lattice", "gamma", "chain", "app",
                                  "wgrad", "adjoint", "dparams"};
    return (phase >= 0 && phase < (int)(sizeof(names) / sizeof(names[0]))) ? names[phase]
                                                                           : nullptr;
}

void mapdec_plan_destroy(mapdec_plan *p) {
    if (!p) return;
    if (p->have_events) {
        hipStreamSynchronize(p->last_stream);
        for (int k = 0; k <= kMaxPhases; ++k) hipEventDestroy(p->ev[k]);
    }
    if (p->exec) {
        hipStreamSynchronize(p->last_stream);
        hipGraphExecDestroy(p->exec);
    }
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
        case MAPDEC_EUNSUPPORTED: return "MAPDEC_EUNSUPPORTED: beyond this build's kernel limits";
        default: return "unknown mapdec status";
    }
}

int mapdec_version(void) { return MAPDEC_VERSION; }

}  // extern "C"
