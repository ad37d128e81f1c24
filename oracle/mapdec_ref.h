/*
 * mapdec_ref.h -- plain FP64 CPU oracle for the MAP forward-backward decoder
 * of J. A. Briffa, "GPU Implementation and Optimization of a Flexible MAP
 * Decoder for Synchronization Correction" (Sec. II-C, eqs. 1-12).
 *
 * TEST INFRASTRUCTURE.  This library exists only to check the GPU decoder.
 * It is called from the test suite, from the smoke check and from the
 * benchmark's CPU-baseline leg, never from the product path.  It shares no
 * source with the GPU library.
 *
 * All pointers are host pointers.  Everything is computed in IEEE double.
 */
#ifndef MAPDEC_REF_H
#define MAPDEC_REF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    REF_OK = 0,
    REF_EINVAL = 1,   /* bad code / channel / state-space parameters       */
    REF_EDRIFT = 2,   /* |rho - tau| > M: end drift outside the state space */
    REF_ENOPATH = 3,  /* P(y) = 0 under the truncated channel model         */
    REF_ENOMEM = 4
};

/* Code, channel and state-space parameters (Sec. II-A, II-B, II-C). */
typedef struct {
    int q;                    /* alphabet size, 2 <= q <= 2^n               */
    int n;                    /* codeword length in bits                     */
    const uint8_t *codebook;  /* q*n bytes of 0/1; row D is C(D)             */
    double Pi, Pd, Ps;        /* insertion, deletion, substitution probs     */
    int I;                    /* max consecutive insertions per time step    */
    int M;                    /* frame drift limit: states m in [-M, M]      */
    int mn;                   /* per-codeword drift change limit [-mn, mn]   */
} ref_code;

/*
 * The general scheme (Sec. II-A: a constituent encoding C_i per symbol
 * position; Sec. III-B: arbitrary state-space limits m_n^- <= 0 <= m_n^+,
 * m_tau^- <= m_n^-, m_tau^+ >= m_n^+).  Drift states m at codeword
 * boundaries lie in [mt_lo, mt_hi] (M_tau = mt_hi - mt_lo + 1 of them);
 * every lattice node (r, j) keeps j - r in [mn_lo, mn_hi] (the corridor,
 * M_n = mn_hi - mn_lo + 1 drift changes).  ncb = 1: one codebook for every
 * position; ncb = N: codebook i serves symbol i.  Codebook i occupies bytes
 * [i q n, (i+1) q n), row D of it is C_i(D).
 */
typedef struct {
    int q, n;
    int ncb;                   /* 1 or N                                      */
    const uint8_t *codebooks;  /* ncb*q*n bytes of 0/1                        */
    double Pi, Pd, Ps;
    int I;
    int mt_lo, mt_hi;          /* frame drift limits m_tau^-, m_tau^+         */
    int mn_lo, mn_hi;          /* per-codeword drift change limits m_n^-, m_n^+ */
} ref_gcode;

/* Requested outputs; any pointer may be NULL.  With a ref_gcode the rows
 * alpha/beta (and the drift priors) have M_tau entries, [i][m - mt_lo]. */
typedef struct {
    double *app;      /* N*q   APP L_i(D), row-major [i][D]                  */
    double *logp;     /* 1     natural log of P(y)                           */
    double *dparams;  /* 3     d log P(y) / d(Pi, Pd, Ps)  (forward mode)     */
    double *dprior;   /* N*q   d log P(y) / d prior[i][D]                     */
    double *alpha;    /* (N+1)*(2M+1) normalised forward metric  [i][m+M]    */
    double *beta;     /* (N+1)*(2M+1) normalised backward metric [i][m+M]    */
    double *logA;     /* N+1   log of the product of alpha normalisers        */
    double *logB;     /* N+1   log of the product of beta normalisers         */
    double *logZ;     /* N     log of the sum over D of the unnormalised APP
                       *       row alpha_i gamma_i beta_{i+1} (normalised rows)  */
} ref_out;

/* Check code parameters; returns REF_OK or REF_EINVAL. */
int mapdec_ref_check(const ref_code *c);

/*
 * Decode one frame.  y: rho bytes of 0/1.  prior: N*q probabilities
 * [i][D] used as given, or NULL for 1/q.  literal != 0 recomputes every
 * receiver-metric lattice once per (i, m', D) on the extracted segment (the
 * decoder as written); literal == 0 memoises the lattice per start index
 * s = n*i + m'.  Returns a REF_* status.
 */
int mapdec_ref_run(const ref_code *c, int N, int rho, const uint8_t *y,
                   const double *prior, int literal, ref_out *out);

/*
 * As mapdec_ref_run with priors of the frame boundaries (Sec. II-C: alpha_0
 * and beta_N are those priors).  start, end: 2M+1 entries each, [m + M] for
 * drift m, used as given, or NULL for the known boundary (start drift 0,
 * end drift rho - tau).  P(y) = sum_m alpha_N(m) end[m + M] in
 * unnormalised terms; received bits outside the frame are not scored.
 */
int mapdec_ref_run_drift(const ref_code *c, int N, int rho, const uint8_t *y,
                         const double *prior, const double *start, const double *end,
                         int literal, ref_out *out);

/* Check general-scheme parameters for frames of N symbols; REF_OK or
 * REF_EINVAL (ncb must be 1 or N, every C_i injective, limits ordered as
 * above). */
int mapdec_ref_gcheck(const ref_gcode *c, int N);

/*
 * Decode one frame under the general scheme.  As mapdec_ref_run_drift,
 * with start / end of M_tau entries ([m - mt_lo]) or NULL for the known
 * boundary; REF_EDRIFT unless mt_lo <= rho - tau <= mt_hi.  With ncb = N
 * every lattice is recomputed per (i, m', D) (literal is then implied).
 */
int mapdec_ref_run_general(const ref_gcode *c, int N, int rho, const uint8_t *y,
                           const double *prior, const double *start, const double *end,
                           int literal, ref_out *out);

/*
 * mapdec_ref_run_general with path thresholds (Sec. III-B, flexibility
 * item h): after every forward step (and at the start row) a drift state
 * whose forward metric, normalised to sum 1 over the row, is below theta is
 * not pursued (set to zero); the backward recursion is computed on the
 * states the forward recursion kept (beta_i(m) = 0 where alpha_i(m) = 0).
 * log P(y), APPs and gradients are then those of the kept paths (the kept
 * states held fixed).  theta = 0 gives mapdec_ref_run_general.  0 <= theta
 * < 1, else REF_EINVAL.  Every lattice is memoised per start index (ncb = 1)
 * or recomputed per (i, m', D).
 */
int mapdec_ref_run_pruned(const ref_gcode *c, int N, int rho, const uint8_t *y,
                          const double *prior, const double *start, const double *end,
                          double theta, ref_out *out);

/*
 * Receiver metric R(y[s .. s+n+delta) | C_i(D)) for delta in [mn_lo,
 * mn_hi] (R[delta - mn_lo]) under the general scheme; dR as below with
 * M_n columns per tangent.
 */
int mapdec_ref_glattice(const ref_gcode *c, int N, int rho, const uint8_t *y, int i, int s,
                        int D, double *R, double *dR);

/*
 * Receiver metric of one lattice: R[k] = R(y[s .. s+n+k) | C(D)) for
 * k = delta + mn, delta in [-mn, mn] (0 where the segment is invalid).
 * dR (may be NULL): 4*(2mn+1) forward-mode tangents, [w][k] for
 * w = (a, d, t1, t0) with a = Pi/2, d = Pd, t1 = Pt(1-Ps), t0 = Pt Ps.
 */
int mapdec_ref_lattice(const ref_code *c, int rho, const uint8_t *y, int s, int D,
                       double *R, double *dR);

#ifdef __cplusplus
}
#endif
#endif
