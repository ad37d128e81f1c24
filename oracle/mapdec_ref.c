/*
 * mapdec_ref.c -- plain FP64 CPU oracle for the MAP forward-backward decoder
 * for a fixed inner codebook on the binary substitution / insertion /
 * deletion (BSID) channel.  J. A. Briffa, "GPU Implementation and
 * Optimization of a Flexible MAP Decoder for Synchronization Correction".
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg call this code.  It shares nothing with the
 * GPU library: no headers, helpers or tables.
 *
 * The code follows the decoder's steps in the paper's order and notation,
 * with no blocking or fusion:
 *   1. channel weights (Sec. II-B; the lattice weights of Sec. II-C);
 *   2. receiver metric R by the corridor-constrained lattice (eqs. 7-10);
 *   3. gamma = prior * R (eq. 6) with the state-space limits of Sec. II-C;
 *   4. normalised forward recursion alpha (eqs. 4, 11, 12);
 *   5. normalised backward recursion beta (eq. 5 and its normalisation);
 *   6. log P(y) from the product of alpha normalisers;
 *   7. APP by eqs. 1-3, each row normalised by its own sum;
 *   8. gradient of log P(y) by forward-mode tangents through the lattice.
 *
 * Every quantity is FP64 except the products of a forward and a backward
 * metric row in steps 7-8 and their sums, which are long double: on long
 * frames with uninformative priors the normalised alpha_i and beta_{i+1}
 * rows peak at opposite ends of the drift range, and their product at the
 * drifts that carry the posterior can lie below the FP64 range (about
 * 1e-420 on 120 000-bit frames at Pi = Pd = 0.1), although each factor is
 * representable.  The extended exponent range keeps those products exact
 * to FP64 precision.
 *
 * Readings where the paper is silent (each one is listed with the design
 * notes):
 *   - I caps the number of consecutive insertions at one channel time step,
 *     i.e. horizontal moves within one lattice row (the channel stays at the
 *     same time after an insertion, Sec. II-B); kept paths are not
 *     renormalised.
 *   - The corridor holds every lattice node (r, j) to m_n^- <= j - r <=
 *     m_n^+ ([-mn, mn] for the symmetric limits of a fixed code).
 *   - Frame drift limits [m_tau^-, m_tau^+] ([-M, M]) hold at codeword
 *     boundaries only.
 *   - Segments that start before 0 or end after rho have gamma = 0.
 *   - Frame boundaries are known, alpha_0 = delta(m) and beta_N = delta(m -
 *     (rho - tau)), unless drift priors are given: Sec. II-C makes alpha_0
 *     and beta_N the prior probabilities of the frame boundaries, so a start
 *     prior phi_0 and an end prior phi_N over [-M, M] are used as those rows
 *     (as given, not renormalised), and P(y) = sum_m alpha_N(m) phi_N(m) in
 *     unnormalised terms.  Received bits before the frame's start or after
 *     its end are not scored.
 *   - With per-step normalisation the APP row is divided by its own sum Z_i
 *     instead of lambda_N(rho - tau) (equal in exact arithmetic).
 *   - Priors are used as given.
 */
#include "mapdec_ref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---- step 1: channel weights -------------------------------------------- */

typedef struct {
    double a;   /* insertion of a given bit: Pi / 2   (horizontal move)     */
    double d;   /* deletion: Pd                        (vertical move)       */
    double t1;  /* transmission, bit unchanged: Pt (1 - Ps)  (diagonal)      */
    double t0;  /* transmission, bit flipped:   Pt Ps       (diagonal)       */
} weights;

static weights channel_weights(const ref_code *c)
{
    weights w;
    double Pt = 1.0 - c->Pi - c->Pd;
    w.a = 0.5 * c->Pi;
    w.d = c->Pd;
    w.t1 = Pt * (1.0 - c->Ps);
    w.t0 = Pt * c->Ps;
    return w;
}

/* The fixed-code, symmetric-limit parameters as an instance of the general
 * scheme: one codebook, m_tau^-/+ = -/+M, m_n^-/+ = -/+mn. */
static ref_gcode as_general(const ref_code *c)
{
    ref_gcode g;
    g.q = c->q; g.n = c->n; g.ncb = 1; g.codebooks = c->codebook;
    g.Pi = c->Pi; g.Pd = c->Pd; g.Ps = c->Ps; g.I = c->I;
    g.mt_lo = -c->M; g.mt_hi = c->M; g.mn_lo = -c->mn; g.mn_hi = c->mn;
    return g;
}

static int check_codebook(const uint8_t *cb, int q, int n)
{
    /* the encoding must be injective (Sec. II-A) */
    for (int D = 0; D < q; D++) {
        for (int r = 0; r < n; r++)
            if (cb[D * n + r] > 1) return REF_EINVAL;
        for (int E = 0; E < D; E++)
            if (memcmp(cb + D * n, cb + E * n, (size_t)n) == 0) return REF_EINVAL;
    }
    return REF_OK;
}

int mapdec_ref_gcheck(const ref_gcode *c, int N)
{
    if (!c || !c->codebooks || N < 1) return REF_EINVAL;
    if (c->n < 1 || c->n > 30 || c->q < 2 || c->q > (1 << c->n)) return REF_EINVAL;
    if (!(c->Pi >= 0.0) || !(c->Pd >= 0.0) || !(c->Ps >= 0.0) || !(c->Ps <= 1.0))
        return REF_EINVAL;
    if (!(c->Pi + c->Pd < 1.0)) return REF_EINVAL;
    if (c->I < 0) return REF_EINVAL;
    /* Sec. III-B: m_n^- <= 0 <= m_n^+, m_tau^- <= m_n^-, m_tau^+ >= m_n^+ */
    if (c->mn_lo > 0 || c->mn_hi < 0 || c->mt_lo > c->mn_lo || c->mt_hi < c->mn_hi)
        return REF_EINVAL;
    if (c->ncb != 1 && c->ncb != N) return REF_EINVAL;
    for (int i = 0; i < c->ncb; i++) {
        int st = check_codebook(c->codebooks + (size_t)i * c->q * c->n, c->q, c->n);
        if (st) return st;
    }
    return REF_OK;
}

int mapdec_ref_check(const ref_code *c)
{
    if (!c || !c->codebook) return REF_EINVAL;
    if (c->mn < 0 || c->M < c->mn) return REF_EINVAL;
    ref_gcode g = as_general(c);
    return mapdec_ref_gcheck(&g, 1);
}

/* ---- step 2: receiver metric lattice (eqs. 7-10) -------------------------- *
 *
 * Rows r = 0..n (bits of x consumed), columns j = 0..mu (bits of the
 * segment consumed).  Entering row r from row r-1 is a deletion of x_r
 * (vertical) or a transmission of x_r received as ydot_j (diagonal);
 * moving along a row is an insertion of ydot_j (horizontal), at most I in a
 * row, none along the last row.  Node (r, j) exists iff j - r lies in the
 * corridor [m_n^-, m_n^+].
 *
 * G[r][j] collects the paths that enter node (r, j) from row r-1, and
 * F[r][j] adds the up-to-I insertions along row r:
 *   G[0][j] = [j == 0]
 *   G[r][j] = d F[r-1][j] + Q(ydot_j | x_r) F[r-1][j-1]          (r >= 1)
 *   F[r][j] = sum_{k=0..min(I,j)} a^k G[r][j-k]                   (r <  n)
 *   F[n][j] = G[n][j]                                             (eq. 10)
 * With I unbounded this is eq. (7): F[r][j] = a F[r][j-1] + G[r][j].
 * Tangents (when dF != NULL) carry d/d(a, d, t1, t0) along every node.
 */

typedef struct {
    int n, mu, I, lo, hi;  /* corridor: lo <= j - r <= hi */
    const uint8_t *ydot;   /* segment, 1-based access ydot[j-1] */
    const uint8_t *x;      /* codeword, 1-based access x[r-1]   */
    weights w;
} lattice_job;

static int in_corridor(const lattice_job *L, int j, int r)
{
    return j - r >= L->lo && j - r <= L->hi;
}

static double Qdot(const weights *w, uint8_t y, uint8_t x)
{
    return (y != x) ? w->t0 : w->t1;
}

/* Runs the lattice for a segment of length mu; writes F[n][j], j = 0..mu,
 * into Fn (and its 4 tangents per j into dFn when requested). */
static int run_lattice(const lattice_job *L, double *Fn, double *dFn)
{
    const int n = L->n, mu = L->mu, W = mu + 1;
    const weights *w = &L->w;
    double *F = calloc((size_t)(n + 1) * W, sizeof(double));
    double *G = calloc((size_t)(n + 1) * W, sizeof(double));
    double *dF = NULL, *dG = NULL;
    if (!F || !G) { free(F); free(G); return REF_ENOMEM; }
    if (dFn) {
        dF = calloc((size_t)(n + 1) * W * 4, sizeof(double));
        dG = calloc((size_t)(n + 1) * W * 4, sizeof(double));
        if (!dF || !dG) { free(F); free(G); free(dF); free(dG); return REF_ENOMEM; }
    }
#define AT(A, r, j) A[(size_t)(r) * W + (j)]
#define DAT(A, r, j, t) A[((size_t)(r) * W + (j)) * 4 + (t)]
    for (int r = 0; r <= n; r++) {
        /* vertical and diagonal moves into row r */
        for (int j = 0; j <= mu; j++) {
            if (!in_corridor(L, j, r)) continue;      /* outside the corridor */
            if (r == 0) {
                AT(G, 0, j) = (j == 0) ? 1.0 : 0.0;
                continue;
            }
            double v = w->d * AT(F, r - 1, j);
            if (dF) {
                for (int t = 0; t < 4; t++) DAT(dG, r, j, t) = w->d * DAT(dF, r - 1, j, t);
                DAT(dG, r, j, 1) += AT(F, r - 1, j);
            }
            if (j >= 1) {
                uint8_t yj = L->ydot[j - 1], xr = L->x[r - 1];
                double Q = Qdot(w, yj, xr);
                v += Q * AT(F, r - 1, j - 1);
                if (dF) {
                    for (int t = 0; t < 4; t++) DAT(dG, r, j, t) += Q * DAT(dF, r - 1, j - 1, t);
                    DAT(dG, r, j, (yj != xr) ? 3 : 2) += AT(F, r - 1, j - 1);
                }
            }
            AT(G, r, j) = v;
        }
        /* horizontal moves along row r: at most I consecutive insertions,
         * none along the last row */
        for (int j = 0; j <= mu; j++) {
            if (!in_corridor(L, j, r)) continue;
            if (r == n) {
                AT(F, r, j) = AT(G, r, j);
                if (dF) for (int t = 0; t < 4; t++) DAT(dF, r, j, t) = DAT(dG, r, j, t);
                continue;
            }
            double v = 0.0, ak = 1.0;
            double dv[4] = {0, 0, 0, 0};
            for (int k = 0; k <= L->I && k <= j; k++) {
                if (in_corridor(L, j - k, r)) {      /* every node on the run */
                    v += ak * AT(G, r, j - k);
                    if (dF) {
                        for (int t = 0; t < 4; t++) dv[t] += ak * DAT(dG, r, j - k, t);
                        /* d(a^k)/da = k a^(k-1) */
                        if (k >= 1) dv[0] += (double)k * pow(w->a, k - 1) * AT(G, r, j - k);
                    }
                } else {
                    break;
                }
                ak *= w->a;
            }
            AT(F, r, j) = v;
            if (dF) for (int t = 0; t < 4; t++) DAT(dF, r, j, t) = dv[t];
        }
    }
    for (int j = 0; j <= mu; j++) {
        Fn[j] = AT(F, n, j);
        if (dFn) for (int t = 0; t < 4; t++) dFn[(size_t)j * 4 + t] = DAT(dF, n, j, t);
    }
#undef AT
#undef DAT
    free(F); free(G); free(dF); free(dG);
    return REF_OK;
}

/* Codeword C_i(D) of the general scheme. */
static const uint8_t *codeword(const ref_gcode *c, int i, int D)
{
    const int b = c->ncb == 1 ? 0 : i;
    return c->codebooks + ((size_t)b * c->q + D) * c->n;
}

/* R(Y[s, s+n+delta) | x) for all delta in [m_n^-, m_n^+]: one lattice over
 * the longest segment that is needed (Sec. II-C: the last row holds all
 * drift changes).  The segment is extracted from y first (ydot of eq. 6).
 * Invalid segments (s < 0, n + delta < 0, s + n + delta > rho) get 0.
 * R[delta - m_n^-]; dR[t][delta - m_n^-] with M_n columns per tangent. */
static int receiver_metric(const ref_gcode *c, const weights *w, int rho, const uint8_t *y,
                           int s, const uint8_t *x, double *R, double *dR)
{
    const int n = c->n, lo = c->mn_lo, hi = c->mn_hi, Mn = hi - lo + 1;
    for (int k = 0; k < Mn; k++) {
        R[k] = 0.0;
        if (dR) for (int t = 0; t < 4; t++) dR[t * Mn + k] = 0.0;
    }
    if (s < 0 || s > rho) return REF_OK;
    int mu = n + hi;
    if (s + mu > rho) mu = rho - s;                 /* longest valid segment */
    if (mu < 0) return REF_OK;
    uint8_t *ydot = malloc((size_t)mu + 1);
    double *Fn = malloc(sizeof(double) * (size_t)(mu + 1));
    double *dFn = dR ? malloc(sizeof(double) * 4 * (size_t)(mu + 1)) : NULL;
    if (!ydot || !Fn || (dR && !dFn)) { free(ydot); free(Fn); free(dFn); return REF_ENOMEM; }
    memcpy(ydot, y + s, (size_t)mu);
    lattice_job L = { n, mu, c->I, lo, hi, ydot, x, *w };
    int st = run_lattice(&L, Fn, dFn);
    if (st == REF_OK) {
        for (int delta = lo; delta <= hi; delta++) {
            int len = n + delta;
            if (len < 0 || len > mu) continue;
            R[delta - lo] = Fn[len];
            if (dR) for (int t = 0; t < 4; t++) dR[t * Mn + delta - lo] = dFn[(size_t)len * 4 + t];
        }
    }
    free(ydot); free(Fn); free(dFn);
    return st;
}

static weights channel_weights_g(const ref_gcode *c)
{
    ref_code k = {0};
    k.Pi = c->Pi; k.Pd = c->Pd; k.Ps = c->Ps;
    return channel_weights(&k);
}

int mapdec_ref_glattice(const ref_gcode *c, int N, int rho, const uint8_t *y, int i, int s,
                        int D, double *R, double *dR)
{
    int st = mapdec_ref_gcheck(c, N);
    if (st) return st;
    if (D < 0 || D >= c->q || rho < 0 || i < 0 || i >= N) return REF_EINVAL;
    weights w = channel_weights_g(c);
    return receiver_metric(c, &w, rho, y, s, codeword(c, i, D), R, dR);
}

int mapdec_ref_lattice(const ref_code *c, int rho, const uint8_t *y, int s, int D,
                       double *R, double *dR)
{
    int st = mapdec_ref_check(c);
    if (st) return st;
    ref_gcode g = as_general(c);
    return mapdec_ref_glattice(&g, 1, rho, y, 0, s, D, R, dR);
}

/* ---- steps 3-8 ------------------------------------------------------------ */

typedef struct {
    const ref_gcode *c;
    weights w;
    int N, rho, literal, tangents;
    const uint8_t *y;
    const double *prior;
    /* memo (one codebook): R for every start s in [0, rho], [s][D][k] with
     * k = delta - m_n^- */
    double *Rtab, *dRtab;
    double *Rbuf, *dRbuf;   /* literal mode scratch */
    int status;
} decoder;

/* Receiver metric row R(s, C_i(D), .) (and tangents [w][k]) -- memoised
 * per s (one codebook) or recomputed for this (i, m', D).  Returns NULL for
 * s outside [0, rho]. */
static const double *R_row(decoder *dc, int i, int s, int D, const double **dRrow)
{
    const int Mn = dc->c->mn_hi - dc->c->mn_lo + 1, q = dc->c->q;
    if (s < 0 || s > dc->rho) return NULL;
    if (!dc->literal) {
        if (dRrow) *dRrow = dc->dRtab ? dc->dRtab + ((size_t)s * q + D) * 4 * Mn : NULL;
        return dc->Rtab + ((size_t)s * q + D) * Mn;
    }
    int st = receiver_metric(dc->c, &dc->w, dc->rho, dc->y, s, codeword(dc->c, i, D),
                             dc->Rbuf, dc->tangents ? dc->dRbuf : NULL);
    if (st) dc->status = st;
    if (dRrow) *dRrow = dc->tangents ? dc->dRbuf : NULL;
    return dc->Rbuf;
}

static double prior_of(const decoder *dc, int i, int D)
{
    return dc->prior ? dc->prior[(size_t)i * dc->c->q + D] : 1.0 / dc->c->q;
}

int mapdec_ref_run(const ref_code *c, int N, int rho, const uint8_t *y,
                   const double *prior, int literal, ref_out *out)
{
    return mapdec_ref_run_drift(c, N, rho, y, prior, NULL, NULL, literal, out);
}

int mapdec_ref_run_drift(const ref_code *c, int N, int rho, const uint8_t *y,
                         const double *prior, const double *start, const double *end,
                         int literal, ref_out *out)
{
    int st = mapdec_ref_check(c);
    if (st) return st;
    ref_gcode g = as_general(c);
    return mapdec_ref_run_general(&g, N, rho, y, prior, start, end, literal, out);
}

static int run_core(const ref_gcode *c, int N, int rho, const uint8_t *y,
                    const double *prior, const double *start, const double *end,
                    int literal, double theta, ref_out *out);

int mapdec_ref_run_general(const ref_gcode *c, int N, int rho, const uint8_t *y,
                           const double *prior, const double *start, const double *end,
                           int literal, ref_out *out)
{
    return run_core(c, N, rho, y, prior, start, end, literal, 0.0, out);
}

int mapdec_ref_run_pruned(const ref_gcode *c, int N, int rho, const uint8_t *y,
                          const double *prior, const double *start, const double *end,
                          double theta, ref_out *out)
{
    if (!(theta >= 0.0) || !(theta < 1.0)) return REF_EINVAL;
    return run_core(c, N, rho, y, prior, start, end, 0, theta, out);
}

/* The decoder's steps (Sec. II-C) under the general scheme.  theta > 0
 * adds path thresholds (the flexibility list of Sec. III-B): a state whose
 * normalised forward metric is below theta is not pursued (its metric is
 * set to zero), and the backward recursion runs on the states the forward
 * recursion kept, so every result is that of the kept paths. */
static int run_core(const ref_gcode *c, int N, int rho, const uint8_t *y,
                    const double *prior, const double *start, const double *end,
                    int literal, double theta, ref_out *out)
{
    int st = mapdec_ref_gcheck(c, N);
    if (st) return st;
    if (rho < 0 || (!y && rho > 0)) return REF_EINVAL;
    const int n = c->n, q = c->q;
    const int mlo = c->mt_lo, mhi = c->mt_hi, dlo = c->mn_lo, dhi = c->mn_hi;
    const int Mt = mhi - mlo + 1, Mn = dhi - dlo + 1;
    const int tau = n * N;
    if (rho - tau < mlo || rho - tau > mhi) return REF_EDRIFT;   /* end drift out of range */
    ref_out none = {0};
    if (!out) out = &none;
    const int tangents = out->dparams != NULL;
    if (c->ncb > 1) literal = 1;   /* R depends on i as well as on s */

    decoder dc = {0};
    dc.c = c; dc.w = channel_weights_g(c); dc.N = N; dc.rho = rho; dc.literal = literal;
    dc.tangents = tangents; dc.y = y; dc.prior = prior;

    double *alpha = calloc((size_t)(N + 1) * Mt, sizeof(double));
    double *beta = calloc((size_t)(N + 1) * Mt, sizeof(double));
    double *logA = calloc((size_t)N + 1, sizeof(double));
    double *logB = calloc((size_t)N + 1, sizeof(double));
    long double *S = calloc((size_t)q, sizeof(long double));
    long double *U = calloc((size_t)q, sizeof(long double));
    double *acc = calloc((size_t)Mt, sizeof(double));
    if (!alpha || !beta || !logA || !logB || !S || !U || !acc) { st = REF_ENOMEM; goto done; }

    /* step 2, memoised: one lattice per start s (with one codebook R
     * depends on s and D only) */
    if (!literal) {
        dc.Rtab = malloc(sizeof(double) * (size_t)(rho + 1) * q * Mn);
        if (!dc.Rtab) { st = REF_ENOMEM; goto done; }
        if (tangents) {
            dc.dRtab = malloc(sizeof(double) * (size_t)(rho + 1) * q * 4 * Mn);
            if (!dc.dRtab) { st = REF_ENOMEM; goto done; }
        }
        for (int s = 0; s <= rho; s++)
            for (int D = 0; D < q; D++) {
                st = receiver_metric(c, &dc.w, rho, y, s, codeword(c, 0, D),
                                     dc.Rtab + ((size_t)s * q + D) * Mn,
                                     tangents ? dc.dRtab + ((size_t)s * q + D) * 4 * Mn : NULL);
                if (st) goto done;
            }
    } else {
        dc.Rbuf = malloc(sizeof(double) * Mn);
        dc.dRbuf = malloc(sizeof(double) * 4 * Mn);
        if (!dc.Rbuf || !dc.dRbuf) { st = REF_ENOMEM; goto done; }
    }

#define ALPHA(i, m) alpha[(size_t)(i) * Mt + (m) - mlo]
#define BETA(i, m) beta[(size_t)(i) * Mt + (m) - mlo]

    /* step 4: alpha_0 = delta(m) or the start prior; alpha'_{i+1}(m) =
     * sum_{m',D} alpha_i(m') gamma_i(m', m, D); alpha_{i+1} = alpha' / sum
     * alpha'.  gamma_i(m', m, D) = prior_i(D) R(Y[ni+m', n(i+1)+m) |
     * C_i(D)) (eq. 6), defined for m - m' in [m_n^-, m_n^+] and m, m' in
     * [m_tau^-, m_tau^+]. */
    if (start) {
        for (int m = mlo; m <= mhi; m++) ALPHA(0, m) = start[m - mlo];
    } else {
        ALPHA(0, 0) = 1.0;
    }
    logA[0] = 0.0;
    /* thresholds: row 0 like every other row, against its own sum */
    if (theta > 0.0) {
        double s0 = 0.0;
        for (int m = mlo; m <= mhi; m++) s0 += ALPHA(0, m);
        for (int m = mlo; m <= mhi; m++)
            if (ALPHA(0, m) < theta * s0) ALPHA(0, m) = 0.0;
    }
    for (int i = 0; i < N; i++) {
        for (int m = mlo; m <= mhi; m++) acc[m - mlo] = 0.0;
        for (int mp = mlo; mp <= mhi; mp++) {
            for (int D = 0; D < q; D++) {
                const double *R = R_row(&dc, i, n * i + mp, D, NULL);
                if (dc.status) { st = dc.status; goto done; }
                if (!R) continue;
                for (int delta = dlo; delta <= dhi; delta++) {
                    int m = mp + delta;
                    if (m < mlo || m > mhi) continue;
                    double gamma = prior_of(&dc, i, D) * R[delta - dlo];
                    acc[m - mlo] += ALPHA(i, mp) * gamma;
                }
            }
        }
        double csum = 0.0;
        for (int m = mlo; m <= mhi; m++) csum += acc[m - mlo];
        if (!(csum > 0.0)) { st = REF_ENOPATH; goto done; }
        for (int m = mlo; m <= mhi; m++) {
            /* not pursued: a normalised metric below theta */
            const double v = acc[m - mlo] / csum;
            ALPHA(i + 1, m) = v < theta ? 0.0 : v;
        }
        logA[i + 1] = logA[i] + log(csum);
    }

    /* step 5: beta_N = delta(m - (rho - tau)) or the end prior; beta'_i(m')
     * = sum_{m,D} gamma_i(m', m, D) beta_{i+1}(m); beta_i = beta' / sum
     * beta'. */
    if (end) {
        for (int m = mlo; m <= mhi; m++) BETA(N, m) = end[m - mlo];
    } else {
        BETA(N, rho - tau) = 1.0;
    }
    /* with thresholds, only the states the forward recursion kept */
    if (theta > 0.0)
        for (int m = mlo; m <= mhi; m++)
            if (!(ALPHA(N, m) > 0.0)) BETA(N, m) = 0.0;
    logB[N] = 0.0;
    for (int i = N - 1; i >= 0; i--) {
        for (int mp = mlo; mp <= mhi; mp++) {
            double v = 0.0;
            for (int D = 0; D < q; D++) {
                const double *R = R_row(&dc, i, n * i + mp, D, NULL);
                if (dc.status) { st = dc.status; goto done; }
                if (!R) continue;
                for (int delta = dlo; delta <= dhi; delta++) {
                    int m = mp + delta;
                    if (m < mlo || m > mhi) continue;
                    double gamma = prior_of(&dc, i, D) * R[delta - dlo];
                    v += gamma * BETA(i + 1, m);
                }
            }
            acc[mp - mlo] = (theta > 0.0 && !(ALPHA(i, mp) > 0.0)) ? 0.0 : v;
        }
        double esum = 0.0;
        for (int m = mlo; m <= mhi; m++) esum += acc[m - mlo];
        if (!(esum > 0.0)) { st = REF_ENOPATH; goto done; }
        for (int m = mlo; m <= mhi; m++) BETA(i, m) = acc[m - mlo] / esum;
        logB[i] = logB[i + 1] + log(esum);
    }

    /* step 6: P(y) = alpha_N(rho - tau) in unnormalised terms (eq. 1), or
     * sum_m alpha_N(m) phi_N(m) with an end prior */
    {
        double aN = 0.0;
        if (end) {
            for (int m = mlo; m <= mhi; m++) aN += ALPHA(N, m) * end[m - mlo];
        } else {
            aN = ALPHA(N, rho - tau);
        }
        if (!(aN > 0.0)) { st = REF_ENOPATH; goto done; }
        if (out->logp) *out->logp = logA[N] + log(aN);
    }

    /* steps 7-8: sigma_i(m', m, D) = alpha_i(m') gamma_i(m', m, D)
     * beta_{i+1}(m) (eq. 3); S_i(D) = sum sigma; APP_i(D) = S_i(D) / Z_i.
     * d log P / d prior_i(D) = sum alpha R beta / Z_i;
     * d log P / d w = sum_i sum alpha prior dR/dw beta / Z_i. */
    {
        long double g[4] = {0, 0, 0, 0};
        for (int i = 0; i < N; i++) {
            long double gi[4] = {0, 0, 0, 0};
            for (int D = 0; D < q; D++) { S[D] = 0.0; U[D] = 0.0; }
            for (int mp = mlo; mp <= mhi; mp++) {
                for (int D = 0; D < q; D++) {
                    const double *dR = NULL;
                    const double *R = R_row(&dc, i, n * i + mp, D, tangents ? &dR : NULL);
                    if (dc.status) { st = dc.status; goto done; }
                    if (!R) continue;
                    for (int delta = dlo; delta <= dhi; delta++) {
                        int m = mp + delta;
                        if (m < mlo || m > mhi) continue;
                        long double ab = (long double)ALPHA(i, mp) * BETA(i + 1, m);
                        double gamma = prior_of(&dc, i, D) * R[delta - dlo];
                        S[D] += ab * gamma;
                        U[D] += ab * R[delta - dlo];
                        if (tangents)
                            for (int t = 0; t < 4; t++)
                                gi[t] += ab * prior_of(&dc, i, D) * dR[t * Mn + delta - dlo];
                    }
                }
            }
            long double Zi = 0.0L;
            for (int D = 0; D < q; D++) Zi += S[D];
            if (!(Zi > 0.0L)) { st = REF_ENOPATH; goto done; }
            if (out->logZ) out->logZ[i] = (double)logl(Zi);
            for (int D = 0; D < q; D++) {
                if (out->app) out->app[(size_t)i * q + D] = (double)(S[D] / Zi);
                if (out->dprior) out->dprior[(size_t)i * q + D] = (double)(U[D] / Zi);
            }
            for (int t = 0; t < 4; t++) g[t] += gi[t] / Zi;
        }
        if (out->dparams) {
            /* chain rule: a = Pi/2, d = Pd, t1 = (1-Pi-Pd)(1-Ps), t0 = (1-Pi-Pd)Ps */
            double Ps = c->Ps, Pt = 1.0 - c->Pi - c->Pd;
            out->dparams[0] = (double)(0.5L * g[0] - (1.0L - Ps) * g[2] - Ps * g[3]);
            out->dparams[1] = (double)(g[1] - (1.0L - Ps) * g[2] - Ps * g[3]);
            out->dparams[2] = (double)(-Pt * g[2] + Pt * g[3]);
        }
    }
    if (out->alpha) memcpy(out->alpha, alpha, sizeof(double) * (size_t)(N + 1) * Mt);
    if (out->beta) memcpy(out->beta, beta, sizeof(double) * (size_t)(N + 1) * Mt);
    if (out->logA) memcpy(out->logA, logA, sizeof(double) * (size_t)(N + 1));
    if (out->logB) memcpy(out->logB, logB, sizeof(double) * (size_t)(N + 1));
    st = REF_OK;
#undef ALPHA
#undef BETA
done:
    free(alpha); free(beta); free(logA); free(logB); free(S); free(U); free(acc);
    free(dc.Rtab); free(dc.dRtab); free(dc.Rbuf); free(dc.dRbuf);
    return st;
}
