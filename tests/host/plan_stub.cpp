// Host-only stand-ins for the HIP runtime calls and kernel launchers that
// libmapdec's host code (mapdec.cpp) uses, so its plan logic runs on a CPU
// under AddressSanitizer.  The "device" workspace is host memory; descriptor
// and work-table uploads are real copies, and every launch reads its work
// table to learn which frames it touches.
//
// Ordering is checked with vector clocks: each stream carries a clock, an
// event records a copy, a wait merges it, and a launch ticks its stream.  A
// launch must be ordered after the previous launch of every frame it
// touches (same stream, or through waited events), and when the caller's
// stream is synchronised it must be ordered after every launch so far.
// The sweep of checkpointed frames is tracked apart: its forward and
// backward chains own the frame's forward and backward checkpoint rows (a
// sweep launch must follow every earlier launch of the frame other than the
// pre-passes that write Gamma by start index, the writer of every block of
// start indices its rows read, and the previous sweep launch of its
// direction), and a chain that starts from checkpoints must follow the
// sweep launches that wrote those rows.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <set>
#include <vector>

#include "kernels.h"
#include "mapdec_internal.h"

namespace {
constexpr int kMaxStreams = 256;
struct Clock {
    int t[kMaxStreams] = {};
};
struct SStream {
    int id;
    Clock vc;
};
struct SEvent {
    bool recorded = false;
    Clock vc;
};
struct SGraph {
    Clock vc;   // what the captured launches were ordered after, and themselves
};
std::set<void *> g_streams, g_events;
std::map<unsigned char *, size_t> g_allocs;
SStream g_null{0, {}};   // the legacy stream (handle 0)
int g_nstreams = 1;
long g_launches = 0, g_waits = 0;
unsigned char *g_ws = nullptr;
size_t g_ws_bytes = 0, g_ws_alloc = 0;
int g_nframes = 0;
struct Last {
    int stream = -1, tick = 0;
};
// Per frame: the stream and tick of its last launch touching the buffers
// other than the group's alpha / beta rows (g_last), and the rows (g_rows).
constexpr int kBufMain = 1, kBufRows = 2;
std::vector<Last> g_last, g_rows;
std::vector<Last> g_lastx;  // per frame: its last launch other than a Gamma-only pre-pass
// writers of the blocks of start indices of each whole-frame Gamma table
// (Gamma-only pre-pass lattices), by table
std::map<const void *, std::map<int, Last>> g_gblock;
// per frame: the writer of each symbol's APP scale (Zexp), which the APP's
// scale pass writes for its group's symbols and the APP and W read
std::vector<std::map<int, Last>> g_zexp;
Last g_any[kMaxStreams];    // per stream: its last launch
// per frame and direction: the last sweep launch, and the writer of every
// checkpoint row
std::vector<Last> g_sweep[2];
std::vector<std::map<int, Last>> g_ckrow[2];

[[noreturn]] void die(const char *what) {
    fprintf(stderr, "plan_stub: %s\n", what);
    abort();
}
SStream *S(hipStream_t s) {
    if (!s) return &g_null;
    if (!g_streams.count((void *)s)) die("unknown stream");
    return (SStream *)s;
}
bool in_range(const void *p, size_t n) {
    const unsigned char *c = (const unsigned char *)p;
    if (c >= g_ws && c + n <= g_ws + g_ws_bytes) return true;
    for (auto &kv : g_allocs)
        if (c >= kv.first && c + n <= kv.first + kv.second) return true;
    return false;
}
bool readable(const void *p, size_t n) {
    const unsigned char *c = (const unsigned char *)p;
    if (c >= g_ws && c + n <= g_ws + g_ws_alloc) return true;
    for (auto &kv : g_allocs)
        if (c >= kv.first && c + n <= kv.first + kv.second) return true;
    return false;
}
bool happened(const Last &l, const Clock &now) { return l.stream < 0 || now.t[l.stream] >= l.tick; }

// One launch on st touching buffers bufs of frames (all frames and buffers
// when all is set); returns its stream and tick.
Last launch(hipStream_t st, const std::vector<int> &frames, bool all, bool gamma_only = false,
            int bufs = kBufMain) {
    SStream *x = S(st);
    for (int f : frames)
        if (f < 0 || f >= g_nframes) die("work item names a frame out of range");
    const Clock &now = x->vc;
    if (all) {
        for (int y = 0; y < g_nstreams; ++y)
            if (!happened(g_any[y], now)) die("launch over all frames not ordered after every launch");
    } else {
        for (int f : frames) {
            if ((bufs & kBufMain) && !happened(g_last[f], now))
                die("launch not ordered after the last launch of its frame");
            if ((bufs & kBufRows) && !happened(g_rows[f], now))
                die("launch not ordered after the last launch on its frame's rows");
        }
    }
    x->vc.t[x->id] += 1;
    const Last me{x->id, x->vc.t[x->id]};
    if (all) {
        for (Last &l : g_last) l = me;
        for (Last &l : g_rows) l = me;
        for (Last &l : g_lastx) l = me;
    } else {
        for (int f : frames) {
            if (bufs & kBufMain) g_last[f] = me;
            if (bufs & kBufRows) g_rows[f] = me;
            if (!gamma_only) g_lastx[f] = me;
        }
    }
    g_any[x->id] = me;
    ++g_launches;
    return me;
}
std::vector<int> work_frames(const mapdec::Work *t, int n) {
    if (n && !in_range(t, sizeof(mapdec::Work) * n)) die("work table outside the workspace");
    std::vector<int> v;
    if (n && !readable(t, sizeof(mapdec::Work) * n)) return v;   // not materialised
    for (int i = 0; i < n; ++i) v.push_back(t[i].frame);
    return v;
}
std::vector<int> list_frames(const int *t, int n) {
    if (n && !in_range(t, sizeof(int) * n)) die("chain list outside the workspace");
    std::vector<int> v;
    if (n && !readable(t, sizeof(int) * n)) return v;
    for (int i = 0; i < n; ++i) v.push_back(t[i]);
    return v;
}
void check_fd(const mapdec::FrameDesc *fd) {
    if (!in_range(fd, sizeof(mapdec::FrameDesc))) die("descriptor table outside the workspace");
}
// Chain lists name descriptors: a frame's own, or (checkpoint segments)
// one after the frames' whose status pointer gives its frame.
std::vector<int> chain_frames(const mapdec::FrameDesc *fd, const int *t, int n) {
    std::vector<int> v = list_frames(t, n);
    for (int &d : v) {
        if (d < g_nframes) continue;
        if (!in_range(fd + d, sizeof(mapdec::FrameDesc))) die("chain descriptor outside the workspace");
        if (!readable(fd + d, sizeof(mapdec::FrameDesc)) || !readable(fd, sizeof(mapdec::FrameDesc)))
            die("chain descriptor not materialised");
        d = (int)(fd[d].status - fd[0].status);
    }
    return v;
}
}  // namespace

// test driver hooks
void stub_set_workspace(void *p, size_t bytes, size_t alloc, int nframes) {
    g_ws = (unsigned char *)p;
    g_ws_bytes = bytes;
    g_ws_alloc = alloc;
    g_nframes = nframes;
    g_last.assign(nframes, Last{});
    g_rows.assign(nframes, Last{});
    g_lastx.assign(nframes, Last{});
    g_gblock.clear();
    g_zexp.assign(nframes, {});
    for (int dir = 0; dir < 2; ++dir) {
        g_sweep[dir].assign(nframes, Last{});
        g_ckrow[dir].assign(nframes, {});
    }
    for (Last &l : g_any) l = Last{};
}
long stub_launches() { return g_launches; }
long stub_waits() { return g_waits; }
int stub_live_objects() { return (int)(g_streams.size() + g_events.size() + g_allocs.size()); }

extern "C" {
hipError_t hipGetDevice(int *d) {
    *d = 0;
    return hipSuccess;
}
hipError_t hipDeviceGetAttribute(int *v, hipDeviceAttribute_t a, int) {
    *v = a == hipDeviceAttributeMultiprocessorCount ? 256 : 160 * 1024;
    return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t *e) {
    SEvent *x = new SEvent;
    g_events.insert(x);
    *e = (hipEvent_t)x;
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
    if (!g_events.erase((void *)e)) die("destroying an unknown event");
    delete (SEvent *)e;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
    if (!g_events.count((void *)e)) die("recording an unknown event");
    SEvent *x = (SEvent *)e;
    x->recorded = true;
    x->vc = S(s)->vc;
    return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
    if (!g_events.count((void *)e)) die("unknown event");
    return hipSuccess;
}
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b) {
    if (!g_events.count((void *)a) || !g_events.count((void *)b)) die("unknown event");
    *ms = 1.f;
    return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) {
    if (g_nstreams >= kMaxStreams) die("too many streams");
    SStream *x = new SStream{g_nstreams++, {}};
    g_streams.insert(x);
    *s = (hipStream_t)x;
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
    if (!g_streams.erase((void *)s)) die("destroying an unknown stream");
    delete (SStream *)s;
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
    SStream *x = S(s);
    if (x == &g_null)   // the caller's stream: everything enqueued so far is done
        for (int y = 0; y < g_nstreams; ++y)
            if (!happened(g_any[y], x->vc)) die("caller's stream not joined with a forked stream");
    return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) {
    if (!g_events.count((void *)e)) die("waiting on an unknown event");
    SEvent *ev = (SEvent *)e;
    if (!ev->recorded) die("waiting on an event never recorded");
    SStream *x = S(s);
    for (int y = 0; y < kMaxStreams; ++y) x->vc.t[y] = std::max(x->vc.t[y], ev->vc.t[y]);
    ++g_waits;
    return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
    S(s);
    return hipSuccess;
}
// Launches enqueued during a capture are checked as they are enqueued; a
// replay orders the capturing stream's clock into the replay stream.
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g) {
    SGraph *x = new SGraph;
    x->vc = S(s)->vc;
    *g = (hipGraph_t)x;
    return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t *x, hipGraph_t g, hipGraphNode_t *, char *, size_t) {
    SGraph *y = new SGraph(*(SGraph *)g);
    *x = (hipGraphExec_t)y;
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t g, hipStream_t s) {
    SStream *x = S(s);
    const SGraph *y = (const SGraph *)g;
    for (int k = 0; k < kMaxStreams; ++k) x->vc.t[k] = std::max(x->vc.t[k], y->vc.t[k]);
    return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t x) {
    delete (SGraph *)x;
    return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
    delete (SGraph *)g;
    return hipSuccess;
}
hipError_t hipMalloc(void **p, size_t n) {
    *p = malloc(n);
    g_allocs[(unsigned char *)*p] = n;
    return hipSuccess;
}
hipError_t hipFree(void *p) {
    if (!g_allocs.erase((unsigned char *)p)) die("freeing an unknown pointer");
    free(p);
    return hipSuccess;
}
hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind k) {
    if (k == hipMemcpyHostToDevice) {
        if (!in_range(d, n)) die("upload outside device memory");
        if (readable(d, n)) memcpy(d, s, n);
    } else {
        if (!in_range(s, n)) die("download outside device memory");
        if (readable(s, n)) memcpy(d, s, n);
        else memset(d, 0, n);
    }
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind k, hipStream_t st) {
    S(st);
    return hipMemcpy(d, s, n, k);
}
}  // extern "C"

namespace mapdec {
hipError_t launch_init(const FrameDesc *fd, int nf, hipStream_t st) {
    check_fd(fd);
    launch(st, {}, true);
    return hipSuccess;
}
hipError_t launch_pack(const FrameDesc *fd, const Work *t, int nb, hipStream_t st) {
    check_fd(fd);
    launch(st, work_frames(t, nb), true);
    return hipSuccess;
}
hipError_t launch_lattice(int, int, int, int, const FrameDesc *fd, const Work *t, int nb,
                          hipStream_t st) {
    check_fd(fd);
    const std::vector<int> frames = work_frames(t, nb);
    // a pre-pass writing only the whole-frame Gamma table (no R)
    bool gamma_only = !frames.empty() && readable(fd, sizeof(FrameDesc));
    for (int f : frames)
        if (gamma_only && (!readable(fd + f, sizeof(FrameDesc)) || fd[f].R != nullptr))
            gamma_only = false;
    const Last me = launch(st, frames, false, gamma_only);
    if (gamma_only)
        for (int i = 0; i < nb; ++i) g_gblock[fd[t[i].frame].G][t[i].item / kLatticeLanes] = me;
    return hipSuccess;
}
hipError_t launch_gsum(int, int, const FrameDesc *fd, const Work *t, int nb, hipStream_t st) {
    check_fd(fd);
    launch(st, work_frames(t, nb), false);
    return hipSuccess;
}
hipError_t launch_gamma(int, int, const FrameDesc *fd, const Work *t, int nb, hipStream_t st) {
    check_fd(fd);
    launch(st, work_frames(t, nb), false);
    return hipSuccess;
}
namespace {
// Launches that read the APP scale of their group's symbols ([i0, i1) of
// each work item's frame descriptor) follow its writers.
void zexp_read(hipStream_t st, const FrameDesc *fd, const Work *t, int nb) {
    if (!nb || !readable(t, sizeof(Work) * nb)) return;
    const Clock &now = S(st)->vc;
    std::set<int> seen;
    for (int k = 0; k < nb; ++k) {
        const int f = t[k].frame;
        if (!seen.insert(f).second) continue;
        for (int i = fd[f].i0; i < fd[f].i1; ++i) {
            auto w = g_zexp[f].find(i);
            if (w != g_zexp[f].end() && !happened(w->second, now))
                die("launch reads an APP scale not written before it");
        }
    }
}
// Whether Gamma by start index is tracked for d's table; if so, every block
// that rows [i0, i1) read (n i0 - M .. n (i1 - 1) + M) must have been
// written before now.
bool gamma_blocks_checked(const FrameDesc &d, int f, const Clock &now, const char *who) {
    auto gt = g_gblock.find(d.G);
    if (gt == g_gblock.end()) return false;
    if (d.i1 <= d.i0) return true;
    const int lo = std::max(0, d.n * d.i0 - d.M);
    const int hi = std::min(d.rho, d.n * (d.i1 - 1) + d.M);
    for (int b = lo / kLatticeLanes; b <= hi / kLatticeLanes; ++b) {
        auto w = gt->second.find(b);
        if (w == gt->second.end() || !happened(w->second, now)) {
            fprintf(stderr, "plan_stub: frame %d rows [%d, %d): Gamma block %d %s\n", f, d.i0, d.i1,
                    b, w == gt->second.end() ? "never written" : "written later");
            die(who);
        }
    }
    return true;
}
// A chain launch: sweep chains (checkpoint rows) apart from the rest.
void chain_launch(hipStream_t st, const FrameDesc *fd, const int *fr, int nc, int dirs) {
    const std::vector<int> frames = chain_frames(fd, fr, nc);
    const std::vector<int> descs = list_frames(fr, nc);
    if (frames.size() != descs.size() || frames.empty()) {   // not materialised
        launch(st, frames, false, false, kBufMain | kBufRows);
        return;
    }
    bool sweep = false;
    for (int d : descs) sweep |= fd[d].chain_mode == kChainSweep;
    if (!sweep) {
        SStream *x = S(st);
        // segment recomputations (every descriptor of the launch, or none)
        // write only the rows; with Gamma by start index tracked they need
        // not follow the frame's other launches, only the writers of the
        // Gamma blocks they read
        bool sub = true, blocks = true;
        for (size_t k = 0; k < descs.size(); ++k) {
            const FrameDesc &d = fd[descs[k]];
            if (d.chain_mode != kChainSub) {
                sub = blocks = false;
                continue;
            }
            const int f = frames[k];
            blocks &= gamma_blocks_checked(d, f, x->vc,
                                           "segment chain reads Gamma not written before it");
            // forward row i0 and backward row i1 come from checkpoints
            if (d.i0 > 0) {
                auto it = g_ckrow[0][f].find(d.i0);
                if (it == g_ckrow[0][f].end() || !happened(it->second, x->vc)) {
                    fprintf(stderr, "plan_stub: frame %d rows [%d, %d) of %d: row %d %s\n", f, d.i0,
                            d.i1, d.N, d.i0,
                            it == g_ckrow[0][f].end() ? "never written" : "written later");
                    die("segment chain not ordered after its forward checkpoint");
                }
            }
            if (d.i1 < d.N) {
                auto it = g_ckrow[1][f].find(d.i1);
                if (it == g_ckrow[1][f].end() || !happened(it->second, x->vc))
                    die("segment chain not ordered after its backward checkpoint");
            }
        }
        launch(st, frames, false, false, sub && blocks ? kBufRows : kBufMain | kBufRows);
        return;
    }
    SStream *x = S(st);
    for (size_t k = 0; k < descs.size(); ++k) {
        const FrameDesc &d = fd[descs[k]];
        if (d.chain_mode != kChainSweep) die("sweep and other chains in one launch");
        const int f = frames[k];
        if (!happened(g_lastx[f], x->vc)) die("sweep not ordered after the frame's earlier launches");
        gamma_blocks_checked(d, f, x->vc, "sweep part reads Gamma not written before it");
        for (int dir = 0; dir < 2; ++dir)
            if (dirs & (1 << dir))
                if (!happened(g_sweep[dir][f], x->vc)) die("sweep part not ordered after the previous one");
        // a part that starts from a checkpoint row: written before it
        const double *ck[2] = {d.alpha, d.beta};
        const double *init[2] = {d.a_init, d.b_init};
        const int row[2] = {d.i0, d.i1};
        for (int dir = 0; dir < 2; ++dir) {
            if (!(dirs & (1 << dir)) || !init[dir]) continue;
            const bool from_ck = init[dir] >= ck[dir] &&
                                 init[dir] <= ck[dir] + (size_t)(d.N / d.ck_stride + 1) * d.Mt;
            if (!from_ck) continue;
            if (init[dir] != ck[dir] + (size_t)(row[dir] / d.ck_stride) * d.Mt)
                die("sweep part starts from another checkpoint row than its first");
            auto it = g_ckrow[dir][f].find(row[dir]);
            if (it == g_ckrow[dir][f].end() || !happened(it->second, x->vc))
                die("sweep part starts from a checkpoint row not written before it");
        }
    }
    x->vc.t[x->id] += 1;
    const Last me{x->id, x->vc.t[x->id]};
    for (size_t k = 0; k < descs.size(); ++k) {
        const FrameDesc &d = fd[descs[k]];
        const int f = frames[k];
        for (int dir = 0; dir < 2; ++dir) {
            if (!(dirs & (1 << dir))) continue;
            g_sweep[dir][f] = me;
            // the rows the chain computes, and its starting row unless it
            // resumes from a checkpoint (not rewritten)
            const bool resumed = dir == 0 ? d.i0 > 0 : d.i1 < d.N;
            const int lo = dir == 0 && resumed ? d.i0 + 1 : d.i0;
            const int hi = dir == 1 && resumed ? d.i1 - 1 : d.i1;
            for (int r = lo; r <= hi; ++r)
                if (r % d.ck_stride == 0) g_ckrow[dir][f][r] = me;
        }
    }
    g_any[x->id] = me;
    ++g_launches;
}
}  // namespace

hipError_t launch_chain(int, const FrameDesc *fd, const int *fr, int nc, int dirs, size_t,
                        hipStream_t st) {
    check_fd(fd);
    chain_launch(st, fd, fr, nc, dirs);
    return hipSuccess;
}
hipError_t launch_chain_ring(int, int shape, int, int waves, const FrameDesc *fd, const int *fr,
                             int nc, int dirs, size_t lds, hipStream_t st) {
    check_fd(fd);
    if (shape < 0 || shape >= kNumRingShapes || lds > 160 * 1024) die("bad ring launch");
    if (waves < 1 || waves > kRingShapes[shape].nw) die("bad ring wave count");
    chain_launch(st, fd, fr, nc, dirs);
    return hipSuccess;
}
hipError_t launch_app(int, const FrameDesc *fd, const Work *t, int nb, size_t, hipStream_t st) {
    check_fd(fd);
    launch(st, work_frames(t, nb), false, false, kBufMain | kBufRows);
    return hipSuccess;
}
hipError_t launch_app_tile(int fp64, int td, int, int nw, const FrameDesc *fd, const Work *t,
                           int nb, size_t lds, hipStream_t st) {
    check_fd(fd);
    if (td != 2 && td != 4 && td != 8) die("bad D tile");
    if (fp64 && td > 4) die("FP64 D tile above 4");
    if (nw < 1 || nw > kAppMaxWaves || lds > 160 * 1024) die("bad tiled-APP launch");
    launch(st, work_frames(t, nb), false, false, kBufMain | kBufRows);
    return hipSuccess;
}
hipError_t launch_app_scale(int mn, const FrameDesc *fd, const Work *t, int nb, hipStream_t st) {
    check_fd(fd);
    if (mn < 0 || mn > kMaxMn) die("bad APP-scale launch");
    // reads the group's rows, writes the scale of the group's symbols
    const Last me = launch(st, work_frames(t, nb), false, false, kBufRows);
    if (nb && readable(t, sizeof(Work) * nb))
        for (int k = 0; k < nb; ++k) g_zexp[t[k].frame][fd[t[k].frame].i0 + t[k].item] = me;
    return hipSuccess;
}
hipError_t launch_app_mfma(int mn, int qt, const FrameDesc *fd, const Work *t, int nb,
                           size_t lds, hipStream_t st) {
    check_fd(fd);
    if (mn < 0 || mn > kMaxMn || qt < 1 || qt > 2 || lds > 160 * 1024)
        die("bad MFMA-APP launch");
    zexp_read(st, fd, t, nb);
    launch(st, work_frames(t, nb), false, false, kBufMain | kBufRows);
    return hipSuccess;
}
hipError_t launch_app_fin(int qt, const FrameDesc *fd, const Work *t, int nb, hipStream_t st) {
    check_fd(fd);
    if (qt < 1 || qt > 2) die("bad APP-finish launch");
    zexp_read(st, fd, t, nb);
    launch(st, work_frames(t, nb), false, false, kBufMain | kBufRows);
    return hipSuccess;
}
size_t app_mfma_lds(int mn, int q) {
    const int QT = (q + 31) / 32;
    const size_t stage = (size_t)2 * 32 * QT * 33 * 4 + 64 * 33 * 8 + 64 * ((32 + 2 * mn) | 1) * 8;
    const size_t epi = (size_t)4 * 32 * 32 * QT * 4;
    return stage > epi ? stage : epi;
}
hipError_t adj_f32_w(int, int, int, const FrameDesc *fd, const Work *t, int nb, hipStream_t st) {
    check_fd(fd);
    zexp_read(st, fd, t, nb);
    launch(st, work_frames(t, nb), false, false, kBufMain | kBufRows);
    return hipSuccess;
}
hipError_t adj_f64_w(int, int, int, const FrameDesc *fd, const Work *t, int nb, hipStream_t st) {
    check_fd(fd);
    zexp_read(st, fd, t, nb);
    launch(st, work_frames(t, nb), false, false, kBufMain | kBufRows);
    return hipSuccess;
}
hipError_t adj_f32_lattice(int, int, int, int, const FrameDesc *fd, const Work *t, int nb, size_t,
                           hipStream_t st) {
    check_fd(fd);
    launch(st, work_frames(t, nb), false);
    return hipSuccess;
}
hipError_t adj_f64_lattice(int, int, int, int, const FrameDesc *fd, const Work *t, int nb, size_t,
                           hipStream_t st) {
    check_fd(fd);
    launch(st, work_frames(t, nb), false);
    return hipSuccess;
}
hipError_t launch_dparams(const FrameDesc *fd, int nf, hipStream_t st) {
    check_fd(fd);
    launch(st, {}, true);
    return hipSuccess;
}
// the allocation-free decode's array: host memory here (no kernel runs)
size_t scratch_bytes() { return (size_t)64 << 20; }
hipError_t scratch_address(void **out) {
    static std::vector<unsigned char> buf(scratch_bytes());
    *out = buf.data();
    return hipSuccess;
}
}  // namespace mapdec
