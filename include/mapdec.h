/*
 * mapdec.h -- MAP forward-backward decoder for a fixed inner codebook on the
 * binary substitution / insertion / deletion (BSID) channel, on AMD gfx950.
 *
 * The decoder computes, for a received frame y of rho bits that carried N
 * q-ary symbols D_0..D_{N-1} each encoded as an n-bit codeword C(D)
 * (Sec. II-A), the a-posteriori probabilities L_i(D) = P(D_i = D | y) of
 * eqs. 1-3 and log P(y), by the forward/backward recursions of eqs. 4-5 over
 * the frame drift m in [-M, M], with the state-transition metric of eq. 6
 * and the receiver metric of the corridor-constrained bit lattice of
 * eqs. 7-10 (per-codeword drift change in [-mn, mn]), normalised per step as
 * in eqs. 11-12.  An insertion cap I limits the number of consecutive
 * insertions at one channel time step.  mapdec_grad also returns the
 * gradient of log P(y) with respect to (Pi, Pd, Ps) and to the priors.
 *
 * Conventions for every call:
 *   - All functions are plain C and never throw.  Status codes are the
 *     MAPDEC_* values below; mapdec_strerror() names them.
 *   - Pointers documented as "device" are HIP device pointers (e.g. from
 *     hipMalloc or a torch tensor on the GPU) owned by the caller.  Pointers
 *     documented as "host" are ordinary host memory owned by the caller.
 *   - "stream" arguments are hipStream_t values passed as void* (NULL = the
 *     default stream).  Work is enqueued asynchronously on that stream.
 *   - precision: MAPDEC_FP64 computes everything in double precision (the
 *     plain decoder); MAPDEC_FP32 computes the bulk arithmetic in single
 *     precision with per-step normalisation, and keeps log-normalisers and
 *     gradient reductions in double precision.
 */
#ifndef MAPDEC_H
#define MAPDEC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MAPDEC_VERSION 107

enum {
    MAPDEC_OK = 0,
    MAPDEC_EINVAL = 1,       /* invalid argument or code/channel parameters       */
    MAPDEC_EDRIFT = 2,       /* a frame's end drift rho - n N lies outside [-M, M] */
    MAPDEC_ENOPATH = 3,      /* P(y) = 0 under the truncated channel model         */
    MAPDEC_ENOMEM = 4,       /* host or device allocation failed                   */
    MAPDEC_ESIZE = 5,        /* workspace smaller than mapdec_workspace_size()     */
    MAPDEC_EDEVICE = 6,      /* a HIP runtime call failed                          */
    MAPDEC_EUNSUPPORTED = 7  /* parameters beyond the library's kernel limits     */
};

enum { MAPDEC_FP32 = 0, MAPDEC_FP64 = 1 };

/* Flags for mapdec_workspace_size / mapdec_plan_create. */
enum {
    MAPDEC_FLAG_GRAD = 1,    /* the plan will also compute gradients        */
    MAPDEC_FLAG_GRAPH = 2,   /* replay the plan's launches as a HIP graph    */
    MAPDEC_FLAG_SERIAL = 4,  /* every launch in order on the run's stream    */
    MAPDEC_FLAG_TUNE = 8     /* time launch choices first (plan creation)    */
};

/* Kernel limits of the library: n <= MAPDEC_MAX_N, mn <= MAPDEC_MAX_MN,
 * q <= MAPDEC_MAX_Q; beyond them decode calls return MAPDEC_EUNSUPPORTED. */
#define MAPDEC_MAX_N 16
#define MAPDEC_MAX_MN 8
#define MAPDEC_MAX_Q 64

typedef struct mapdec_code mapdec_code;

/*
 * mapdec_create -- an immutable code + channel + state-space description.
 *
 * q, n       alphabet size and codeword length (Sec. II-A): 2 <= q <= 2^n.
 * codebook   host, q*n bytes of 0/1; row D (bytes D*n .. D*n+n-1) is the
 *            codeword C(D) in transmission order.  Codewords must be
 *            distinct (the encoding is injective).  The bytes are copied.
 * Pi, Pd, Ps insertion, deletion and substitution probabilities of the BSID
 *            channel (Sec. II-B): Pi, Pd, Ps >= 0, Pi + Pd < 1, Ps <= 1.
 *            The lattice weights are Pi/2 per inserted bit, Pd per deleted
 *            bit, Pt(1-Ps) / Pt Ps per transmitted bit received equal /
 *            flipped, Pt = 1 - Pi - Pd (eqs. 7-10).
 * I          maximum number of consecutive insertions at one channel time
 *            step, I >= 0.  (For I >= 2 mn the cap never binds.)
 * M          frame drift limit: drift states m in [-M, M] at codeword
 *            boundaries (Sec. II-C, m_tau^- = -M, m_tau^+ = M).
 * mn         per-codeword drift limit: every lattice node stays within
 *            [-mn, mn] of the codeword's start drift (the corridor of
 *            Sec. II-C, m_n^- = -mn, m_n^+ = mn); 0 <= mn <= M.
 * Returns NULL on failure; mapdec_last_error() then gives MAPDEC_EINVAL or
 * MAPDEC_ENOMEM.  Host-only: no device memory is touched.  A handle may be
 * shared by any number of frames, plans and threads.
 */
mapdec_code *mapdec_create(int q, int n, const uint8_t *codebook, double Pi, double Pd,
                           double Ps, int I, int M, int mn);

/*
 * mapdec_create_general -- the general scheme (Sec. II-A: a constituent
 * encoding C_i for every symbol position; Sec. III-B: arbitrary state-space
 * limits m_n^- <= 0 <= m_n^+, m_tau^- <= m_n^-, m_tau^+ >= m_n^+).
 * ncb        1 (one codebook for every position, as mapdec_create) or the
 *            number of symbols N of every frame that uses the handle
 *            (codebook i encodes symbol i).
 * codebooks  host, ncb*q*n bytes of 0/1; codebook i occupies bytes
 *            [i q n, (i+1) q n), row D of it is C_i(D).  Each codebook must
 *            be injective.  The bytes are copied.
 * mt_lo, mt_hi  frame drift limits m_tau^-, m_tau^+: drift states at
 *            codeword boundaries lie in [mt_lo, mt_hi].
 * mn_lo, mn_hi  per-codeword drift change limits m_n^-, m_n^+: every
 *            lattice node (r, j) keeps j - r in [mn_lo, mn_hi].
 * Other arguments as mapdec_create.  Frames of such a code give their
 * boundary drift priors (if any) as 2M+1 entries [m + M] with M =
 * max(-mt_lo, mt_hi); entries outside [mt_lo, mt_hi] are ignored.  A frame
 * reports MAPDEC_EDRIFT unless mt_lo <= rho - tau <= mt_hi, and
 * MAPDEC_EINVAL if ncb > 1 and its N differs from ncb.  The kernel limits
 * apply to max(-mn_lo, mn_hi).  Returns NULL on failure (mapdec_last_error()
 * gives MAPDEC_EINVAL or MAPDEC_ENOMEM).  With ncb > 1 the receiver metric
 * is computed per (symbol, drift state) instead of being shared by the
 * start index (the lattices of Sec. IV-A): about M_tau / n times the work.
 */
mapdec_code *mapdec_create_general(int q, int n, int ncb, const uint8_t *codebooks, double Pi,
                                   double Pd, double Ps, int I, int mt_lo, int mt_hi, int mn_lo,
                                   int mn_hi);

/*
 * mapdec_with_threshold -- a new handle: code with path thresholds (the
 * flexibility list of Sec. III-B: thresholds that avoid pursuing
 * low-probability trellis paths).  After every forward step (and at the
 * start row) a drift state whose forward metric is below theta times the
 * sum of its row is not pursued (its metric becomes zero); the backward
 * recursion runs on the states the forward recursion kept.  log P(y), the
 * APPs and the gradient are then those of the kept paths (with the kept
 * states held fixed); MAPDEC_ENOPATH when the thresholds drop every path.
 * 0 <= theta < 1 (theta = 0: the exact decoder).  The forward chain of a
 * frame then runs before its backward chain, and the workspace holds a byte
 * per (symbol boundary, drift state).  code is not changed; the new handle
 * is destroyed with mapdec_destroy.  NULL on failure (MAPDEC_EINVAL for a
 * theta outside [0, 1), MAPDEC_ENOMEM).
 */
mapdec_code *mapdec_with_threshold(const mapdec_code *code, double theta);

/* Frees a handle.  NULL is a no-op.  Plans that use it must be destroyed first. */
void mapdec_destroy(mapdec_code *code);

/*
 * One frame of a batch.  Frames of one batch may use different codes.
 *   code   the frame's code handle.
 *   N      number of symbols, N >= 1 (frame length tau = n N bits).
 *   rho    number of received bits, rho >= 0, |rho - tau| <= M.
 *   y      device, rho bytes of 0/1 (received bits in order).
 *   prior  device, N*q prior probabilities P(D_i = D) row-major [i][D]
 *          (float for MAPDEC_FP32, double for MAPDEC_FP64), used as given;
 *          NULL means 1/q for every entry (eq. 6).
 *   app    device, N*q output APPs [i][D] in the same type as prior, or NULL.
 *   dprior device, N*q output d log P(y) / d prior[i][D] = U_i(D) / Z_i
 *          (decode and gradient calls; the inner decoder's extrinsic
 *          output for iterative decoding), same type, or NULL.
 *   start_drift, end_drift
 *          device, 2M+1 doubles each, entry [m + M] the prior probability
 *          that the frame's first codeword starts at received bit m (start)
 *          or that its last codeword ends at received bit tau + m (end),
 *          used as given; NULL means the known boundary (start drift 0, end
 *          drift rho - tau).  These are the priors of the frame boundaries
 *          that start the forward and backward metrics (Sec. II-C): alpha_0
 *          = start, beta_N = end, and P(y) = sum_m alpha_N(m) end[m + M].
 *          Received bits before the start or after the end are not scored;
 *          entries whose position (m, or tau + m) lies outside [0, rho]
 *          carry no path and contribute nothing.  The priors are inputs
 *          only: gradients cover (Pi, Pd, Ps) and the symbol priors, not
 *          these.  Zero-initialise both when they are not used.
 */
typedef struct {
    const mapdec_code *code;
    int32_t N;
    int32_t rho;
    const uint8_t *y;
    const void *prior;
    void *app;
    void *dprior;
    const double *start_drift;
    const double *end_drift;
} mapdec_frame;

/*
 * mapdec_workspace_size -- bytes of device workspace that a decode (or,
 * with MAPDEC_FLAG_GRAD, a gradient) of these frames needs with forward
 * checkpoints every checkpoint_K symbols (0: none; see mapdec_grad).
 * frames: host array of nframes entries.  Returns 0 if the frames are
 * invalid or checkpoint_K < 0.
 */
size_t mapdec_workspace_size(const mapdec_frame *frames, int nframes, int precision,
                             int flags, int checkpoint_K);

/*
 * mapdec_decode -- APPs and log P(y) of every frame (eqs. 1-12).
 *   frames   host array of nframes frame descriptions.
 *   logp     device, nframes doubles: natural log of P(y) per frame.
 *   status   device, nframes int32: MAPDEC_OK, or MAPDEC_ENOPATH when
 *            P(y) = 0 (then that frame's logp is -inf and its APP row
 *            contents are unspecified).
 *   ws       device workspace of ws_bytes >= mapdec_workspace_size(...).
 * The return value reports host-side validation (MAPDEC_EINVAL,
 * MAPDEC_EDRIFT, MAPDEC_ESIZE, MAPDEC_EUNSUPPORTED) or a launch failure
 * (MAPDEC_EDEVICE); per-frame results come through status.  Nothing is
 * enqueued unless the return value is MAPDEC_OK.
 */
int mapdec_decode(const mapdec_frame *frames, int nframes, double *logp, int32_t *status,
                  void *ws, size_t ws_bytes, int precision, void *stream);

/*
 * mapdec_grad -- everything mapdec_decode computes, plus the gradient of
 * log P(y) with M, mn and I held fixed and Pt = 1 - Pi - Pd:
 *   dparams  device, 3*nframes doubles: d log P / d(Pi, Pd, Ps) per frame.
 *   frames[f].dprior receives d log P / d prior[i][D] when non-NULL.
 * checkpoint_K: 0 keeps the receiver metric, Gamma and every forward and
 * backward metric row of the whole frame in the workspace.  K > 0 (K < N)
 * keeps the forward and backward rows only at every K-th symbol (the
 * checkpoints) and recomputes the receiver metric: a first pass computes
 * Gamma for the whole frame (2 mn + 1 values per received bit) and runs the
 * forward and backward recursions over the whole frame side by side,
 * storing the checkpoints of both; main passes then take consecutive
 * segments of K symbols a group at a time (enough segments that the
 * received bits a group reaches exceed its own by a quarter at most): the
 * group's receiver metric is recomputed, every segment's forward and
 * backward rows are recomputed from its two checkpoints (all segments at
 * once), then the APPs and gradient terms of the group follow.  The
 * workspace then holds one group's tables plus O(N) checkpoints and Gamma
 * instead of O(N) rows and receiver metric; K = ceil(sqrt(N)) balances the
 * two.  Results equal those of K = 0 up to rounding.
 * Workspace from mapdec_workspace_size(..., flags | MAPDEC_FLAG_GRAD,
 * checkpoint_K).
 */
int mapdec_grad(const mapdec_frame *frames, int nframes, double *logp, double *dparams,
                int32_t *status, void *ws, size_t ws_bytes, int checkpoint_K, int precision,
                void *stream);

/*
 * Plans: the same work as mapdec_decode / mapdec_grad, with validation,
 * workspace layout and descriptor upload done once at creation and every
 * later run replaying the same launches (as one HIP graph with
 * MAPDEC_FLAG_GRAPH).  A plan keeps pointers to the caller's buffers (y,
 * prior, app, dprior, logp, status, dparams, ws): they must stay valid
 * until mapdec_plan_destroy; their contents may change between runs.
 * dparams is used only with MAPDEC_FLAG_GRAD (may be NULL otherwise).
 * checkpoint_K as for mapdec_grad (it applies to decode-only plans too);
 * ws_bytes >= mapdec_workspace_size(frames, nframes, precision, flags,
 * checkpoint_K).  Returns NULL on failure (see mapdec_last_error()).  The
 * descriptor upload is enqueued on stream.
 *
 * Forked runs use 4 streams at once; a process has a limited number of
 * hardware queues (4 by default), and streams beyond them share one, which
 * serialises what they share.
 *
 * Batches whose frames differ in shape (q, n, M, mn, priors) need several
 * launches per phase, one per kernel instance.  A plan without
 * MAPDEC_FLAG_GRAPH or MAPDEC_FLAG_SERIAL then deals those launches to
 * three streams of its own (created at plan creation, default priority)
 * besides the run's stream: each launch waits only for earlier launches
 * that touched one of its frames, and the run's stream waits for all of
 * them at the end, so a run is still ordered on the caller's stream as a
 * whole.  Gradient plans of at least 32 frames that need one launch per
 * phase run eagerly as min(4, nframes / 16) contiguous slices of frames
 * instead (2 slices for 32-47 frames, 3 for 48-63, 4 from 64), slice k on
 * stream k, every launch other than the chains also waiting for the same
 * launch of the slice before: the compute-bound phases then advance slice
 * by slice while each slice's chains (a latency-bound recursion) run
 * beside them.  With checkpointed frames (checkpoint_K > 0, no path
 * thresholds, no frame slices) such a plan also runs the sweep that writes
 * the checkpoints in 16 parts, its forward chains on one of those streams
 * and its backward chains on another, while the groups of segments whose
 * checkpoints exist already run on the others (the middle of the frames
 * first); with Gamma by start index the pre-pass that computes it for the
 * sweep runs in 16 rounds beside the parts.  Graph plans record every
 * launch in order on one stream.  Results do not depend on the order: the
 * parts carry the row-scale predictor from one to the next, so every
 * schedule gives the same bits.
 */
typedef struct mapdec_plan mapdec_plan;

mapdec_plan *mapdec_plan_create(const mapdec_frame *frames, int nframes, double *logp,
                                double *dparams, int32_t *status, void *ws, size_t ws_bytes,
                                int precision, int flags, int checkpoint_K, void *stream);
int mapdec_plan_run(mapdec_plan *plan, void *stream);

/*
 * Empirical tuning (the run-time choice of kernel configurations, Sec. V,
 * made by measurement).  With MAPDEC_FLAG_TUNE, mapdec_plan_create first
 * builds a decode-only plan of the same frames on ws, runs it once, and
 * times the alternatives of two launch choices on its metric tables:
 *   - the tiled APP kernel's D tile (2, 4 or 8 symbol values; at most 4 in
 *     FP64, at most the default for q) and waves per workgroup (the default
 *     one per 64 start indices, or half of it), per bucket (precision, q, n,
 *     mn, default waves), on up to 8192 workgroups of the bucket's frames;
 *   - the ring chain's workgroup shape (the first shape that fits and the
 *     next two), per bucket (precision, uniform priors, codeword length,
 *     mn, first shape), on up to 1024 of the bucket's frames.
 * The fastest choice of each bucket goes into a table shared by every
 * later plan of the process (buckets already in it are not timed again),
 * then the plan is laid out with it.  The workspace size does not depend
 * on these choices.  Tuning writes the frames' outputs (they are written
 * again by every run) and blocks until its timing runs have finished; it
 * allocates a small device scratch buffer for the duration.
 */
/* Number of buckets in the process's tuned table. */
int mapdec_tune_entries(void);
/* Empties the process's tuned table (later plans take the defaults). */
void mapdec_tune_reset(void);
/* Waits for the plan's pending work and frees it.  NULL is a no-op. */
void mapdec_plan_destroy(mapdec_plan *plan);

/*
 * mapdec_plan_profile -- per-phase time split of one run (the decoder's
 * time per metric, Sec. VI).  Runs the plan's launches once, eagerly, in
 * the plan's own eager schedule (forked streams and frame slices as for a
 * run without MAPDEC_FLAG_GRAPH; one stream for graph and serial plans),
 * with a timing event recorded on each launch's stream just before and just
 * after it; waits for them and writes into phase_ms[k] (k < max_phases)
 * the sum of the durations of phase k's launches (with checkpoints or
 * slices a phase has several).  Launches that overlap each count in full.
 * Returns the number of phases, or a negative MAPDEC_* status.  Results
 * land in the plan's outputs as after mapdec_plan_run.
 */
int mapdec_plan_profile(mapdec_plan *plan, void *stream, float *phase_ms, int max_phases);
/* Number of launches of profile phase k in one run of the plan (a negative
 * MAPDEC_* status for a NULL plan). */
int mapdec_plan_launches(const mapdec_plan *plan, int phase);
/* Static name of profile phase k ("pack", "lattice", "gamma", "chain",
 * "app", "wgrad", "adjoint", "dparams", "rechain": the forward and backward
 * rows recomputed from checkpoints), or NULL past the last phase. */
const char *mapdec_phase_name(int phase);

/*
 * mapdec_decode_noalloc -- mapdec_decode for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid allocation).  Same frames, outputs, status codes and
 * asynchronous semantics as mapdec_decode, with no workspace argument: the
 * workspace is a fixed device array of mapdec_noalloc_limit() bytes
 * (64 MiB) inside the library, one per device, held until the process
 * ends.  Returns MAPDEC_ESIZE when mapdec_workspace_size(frames, nframes,
 * precision, 0, 0) exceeds that limit.  No hipMalloc / hipFree or other
 * device allocation, no stream or event creation; the frame descriptors are
 * copied from host memory into the array's head on stream.  Every call on a
 * device shares that device's array, which keeps the last call's contents:
 * calls that overlap on one device (other streams, other threads, before
 * the previous call's work has finished on a different stream) race and
 * give undefined results.  Calls in order on one stream are safe.
 */
int mapdec_decode_noalloc(const mapdec_frame *frames, int nframes, double *logp,
                          int32_t *status, int precision, void *stream);
/* Bytes of the device array behind mapdec_decode_noalloc. */
size_t mapdec_noalloc_limit(void);

/*
 * Iterative decoding with an outer code (Sec. II-A: the inner code serially
 * concatenated with an outer code; Sec. II-C: in iterative decoding the
 * inner decoder's symbol priors P(D_i = D) come from the outer decoder's
 * extrinsic information of the previous pass).  A pass is mapdec_decode (or
 * a plan) with the frames' priors set to the last pass's extrinsic output
 * (1/q at first) and their dprior set to the buffer that
 * mapdec_outer_decode then reads as its channel: d log P / d prior_i(D) =
 * U_i(D) / Z_i is the inner APP with the symbol's own prior divided out
 * (eqs. 1-3), up to a factor per symbol.
 *
 * The outer code is linear over GF(q), q = 2^p, 1 <= p <= 6 (q equals the
 * inner alphabet): a word x of N symbols is a codeword when
 * sum_j H[c][j] x_j = 0 for every row c of the parity-check matrix H.
 * Field elements are the integers 0 .. q-1 read as polynomials over GF(2)
 * (bit k the coefficient of z^k): addition is bitwise XOR, multiplication
 * the polynomial product reduced modulo the primitive polynomial
 * z+1 (p = 1), z^2+z+1, z^3+z+1, z^4+z+1, z^5+z^2+1, z^6+z+1 (p = 6).
 */
typedef struct mapdec_outer mapdec_outer;

/* Largest number of entries in one row, and of rows holding one symbol. */
#define MAPDEC_OUTER_MAX_DEG 32

/*
 * mapdec_outer_create -- H in compressed rows, host arrays: row_ptr (m+1
 * int32, row_ptr[0] = 0, nondecreasing), col (row_ptr[m] int32 in [0, N),
 * no column twice in a row), coef (row_ptr[m] bytes in [1, q-1]).  Every
 * row and every column has at most MAPDEC_OUTER_MAX_DEG entries.  Copies
 * the code to the current device.  NULL on failure (mapdec_last_error():
 * MAPDEC_EINVAL, MAPDEC_EUNSUPPORTED for a degree above the limit,
 * MAPDEC_ENOMEM, MAPDEC_EDEVICE).
 */
mapdec_outer *mapdec_outer_create(int q, int N, int m, const int32_t *row_ptr,
                                  const int32_t *col, const uint8_t *coef);
void mapdec_outer_destroy(mapdec_outer *code);
/* Device workspace bytes of mapdec_outer_decode for nframes frames. */
size_t mapdec_outer_workspace_size(const mapdec_outer *code, int nframes, int precision);

/*
 * mapdec_outer_decode -- iters >= 1 iterations of belief propagation
 * (sum-product, flooding schedule: every check, then every symbol) on
 * nframes words of the outer code (nframes <= 65535).
 *   chan  device, [nframes][N][q] in the precision's type: the channel
 *         distribution of every symbol (each row is divided by its sum, so
 *         the inner decoder's dprior serves as it is; a row summing to 0
 *         counts as uniform).
 *   extr  device, [nframes][N][q] output: the extrinsic distributions,
 *         proportional to the product of the symbol's incoming check
 *         messages (the next pass's priors).
 *   post  device, [nframes][N][q] output (posteriors, proportional to the
 *         channel times that product), or NULL.
 * Messages from a check to symbol j are the distribution of
 * H[c][j]^-1 sum_{k != j} H[c][k] x_k under the symbols' incoming
 * messages; every message is normalised to sum 1 (a vector summing to 0
 * becomes uniform).  ws: ws_bytes >= mapdec_outer_workspace_size(...).
 * Returns MAPDEC_OK, MAPDEC_EINVAL, MAPDEC_ESIZE or MAPDEC_EDEVICE; work is
 * enqueued on stream.
 */
int mapdec_outer_decode(const mapdec_outer *code, int nframes, const void *chan, void *extr,
                        void *post, int iters, void *ws, size_t ws_bytes, int precision,
                        void *stream);

/* Status of the calling thread's last failed mapdec_create / plan_create /
 * mapdec_outer_create. */
int mapdec_last_error(void);
/* Static string naming a status code. */
const char *mapdec_strerror(int status);
/* MAPDEC_VERSION of the library. */
int mapdec_version(void);

#ifdef __cplusplus
}
#endif
#endif
