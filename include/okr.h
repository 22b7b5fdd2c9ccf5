/*
 * okr.h -- C ABI of the MI355X (gfx950) segment-exhaustive Kron-reduction
 * search ("Opti-KRON" exhaustive aggregation search, arXiv 2510.19608).
 *
 * What the library computes (Section IV of the paper, generalised from single
 * edge moves to every subset of a segment's eligible nodes):
 *
 *   for each segment g (increasing id), against the cumulative state left by
 *   the segments before it:
 *     for every mask m in [0, 2^k):  reduce the nodes whose bit is set
 *       - assignment: each reduced node moves its (aggregated) injection to
 *         its nearest kept ancestor (Section II.C, eq. i_agg; Algorithm 1
 *         current aggregation);
 *       - Kron reduction of the network (eq. Y_kron, Schur complement with
 *         the pseudo-inverse on present phases) and the fixed-current solve
 *         of the reduced network over every load snapshot (Algorithm 1
 *         "solve I^c = Y V^c", which gives the same super-node voltages);
 *       - reduced nodes take their super-node's voltage (Algorithm 1);
 *       - error e = max over snapshots, nodes, phases of ||V^| - |V^c||
 *         (eq. iter_obj) and the margins: e <= e_bar (eq. v_abs, inclusive)
 *         and v_min <= |V^c| <= v_max on every kept node-phase;
 *     select the feasible mask with the most reduced nodes, then the smallest
 *     error over the nodes the segment can affect, then the lowest mask
 *     (errors within tie_tol of the minimum tie).
 *   The scenario library (V^, I^) comes from an AC load flow of the full
 *   network with constant-PQ wye loads (Section III, library L), unless the
 *   caller passes V^.
 *
 * Conventions.
 *   Complex numbers are interleaved double pairs (re, im).  3x3 blocks are
 *   row-major, phase order a, b, c.  Values are per unit on a per-phase
 *   line-to-neutral base.  Node 0 is the slack, parent[0] = -1.
 *   Mask bit j of segment g is the j-th node of g in DFS preorder, children
 *   visited in increasing node id.
 *
 * Memory.  The library allocates no device memory: the caller passes one
 * device workspace of the size okr_plan() reports.  Pointers marked DEVICE
 * must be device memory; pointers marked HOST host memory.  Nothing is
 * retained after a call returns.  Calls on one handle must not overlap.
 *
 * Errors.  Every function returns 0 on success, a negative OKR_E_* code on
 * failure (okr_last_error() gives a message) or a positive OKR_W_* warning.
 * No exception or abort crosses the ABI.
 */
#ifndef OKR_H
#define OKR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OKR_OK 0
#define OKR_E_ARG (-1)         /* bad argument, size or pointer */
#define OKR_E_NOT_TREE (-2)    /* parent[] is not a tree rooted at node 0 */
#define OKR_E_PHASE (-3)       /* child phases not a subset of the parent's, or
                                  nonzero entries on absent phases */
#define OKR_E_SINGULAR (-4)    /* a present-phase branch block is singular */
#define OKR_E_PF_DIVERGED (-5) /* load flow did not converge */
#define OKR_E_WORKSPACE (-6)   /* workspace missing or smaller than planned */
#define OKR_E_HIP (-7)         /* a HIP runtime call failed */
#define OKR_E_UNSUPPORTED (-8) /* shunts / asymmetric blocks, or a segment with
                                  more than 24 eligible nodes, or an eligible
                                  node that is the slack or has two children */
#define OKR_W_BASE_OUT_OF_BAND 1 /* the full network violates the band: nothing
                                    is reduced (Algorithm 1 stops at once) */

#define OKR_PRECISION_FP64 0   /* complex128 everywhere */
#define OKR_PRECISION_MIXED 1  /* FP32 difference-form sweep, FP64 refine */
#define OKR_PRECISION_FP64_FACTORED 2 /* complex128; every mask's score assembled
                                  from per-chain pattern tables (a chain's
                                  terms depend only on its own and its nesting
                                  path's mask bits; max and min are exact), so
                                  the scores equal OKR_PRECISION_FP64's bit for
                                  bit */

#define OKR_SECONDARY_MAXERR 0 /* key: the largest error over the affected
                                  nodes (eq. iter_obj) */
#define OKR_SECONDARY_SMICE 1  /* key: SMICE, Algorithm 1's selection: per
                                  snapshot, each cluster's largest member
                                  error over members and phases (MICE,
                                  Section II.C), summed over clusters and
                                  snapshots */

#define OKR_FLAG_TIMING 1u     /* record per-kernel HIP-event timings */
#define OKR_FLAG_VHAT_GIVEN 2u /* loads->Vhat holds the scenario voltages */
#define OKR_FLAG_DUMP_SCORES 4u /* keep every segment's per-mask (e, slack) for
                                   okr_dump_scores() */
#define OKR_FLAG_AUTOTUNE 16u  /* before this call's search, run the search
                                  once per candidate shape of the FP64
                                  scoring launch (snapshots per pass 1, 2 or
                                  4; waves per 64 masks 1, 2 or 4; snapshot
                                  groups 1, 2, 4, ... 32 within the planned
                                  workspace) and keep the fastest per segment
                                  size and chunk width in the handle for this
                                  and later calls */
#define OKR_FLAG_GRAPH 8u      /* capture the whole search (load flow, every
                                  segment, final outputs) as one hipGraph on
                                  the first call and replay it afterwards;
                                  ignored with TIMING, DUMP_SCORES or a
                                  features dump; needs a non-null stream */

typedef struct okr_handle okr_handle;

/* Topology (HOST).  eligible[i] = 1 marks a node the search may reduce: it
 * must not be the slack and must have at most one child (so reductions never
 * create meshes, Section V).  segment[i] is the segment id of an eligible
 * node, -1 otherwise; ids run from 0 without gaps. */
typedef struct {
    int32_t n;
    const int32_t *parent;   /* [n] */
    const uint8_t *phase;    /* [n] bit0 = a, bit1 = b, bit2 = c */
    const uint8_t *eligible; /* [n] */
    const int32_t *segment;  /* [n] */
} okr_topology;

/* Nodal admittance blocks (DEVICE, complex128 [n][3][3]).
 * Y_off[i] = Y_{i,parent(i)} for i >= 1 (Y_off[0] ignored); Y_diag[i] = Y_ii.
 * Blocks must be symmetric, zero on absent phases, and without shunts
 * (Y_ii = -sum of the incident off-diagonal blocks, 1e-9 relative). */
typedef struct {
    const double *Y_diag;
    const double *Y_off;
} okr_yblocks;

/* Loads.  S_load (DEVICE, complex128 [S][n][3]) is the consumed power P + jQ
 * per node-phase and snapshot; V0 (HOST, complex128 [3]) the slack voltage;
 * Vhat (DEVICE, complex128 [S][n][3], optional) the scenario voltages, used
 * instead of the load flow when OKR_FLAG_VHAT_GIVEN is set. */
typedef struct {
    int32_t S;
    const double *S_load;
    const double *V0;
    const double *Vhat;
} okr_loads;

typedef struct {
    double e_bar;     /* voltage-magnitude error bound (p.u.), e.g. 0.003 */
    double v_min;     /* band, inclusive, e.g. 0.95 */
    double v_max;     /* e.g. 1.05 */
    double tie_tol;   /* errors within tie_tol of the minimum tie (1e-11) */
    double amb_tol;   /* near-boundary window for the ambiguity flag (1e-13) */
    double pf_tol;    /* load-flow stop: max |dV| <= pf_tol (1e-13) */
    int32_t pf_maxit; /* load-flow iteration cap (100) */
    int32_t precision;/* OKR_PRECISION_* */
    uint32_t flags;   /* OKR_FLAG_* */
    int32_t top_k;    /* > 0 with `surrogate`: rescore only the top_k masks the
                         surrogate ranks first (full enumeration as fallback) */
    const float *surrogate; /* DEVICE FP32 parameters of the surrogate MLP
                               (layout in okr_train_surrogate), or NULL */
    int32_t lanes;    /* segments per launch chunk (0 = 8, at most 8): each
                         search step is launched once over a chunk of
                         mutually independent segments (no shared affected
                         region or chain head), conflicting segments keep
                         their order; read by okr_plan (each chunk position
                         has its own scratch block) */
    float surrogate_margin; /* with `surrogate`: a mask counts as predicted
                               feasible while its predicted ln error is at
                               most ln(e_bar) + surrogate_margin (the
                               calibrated over-prediction of the network, so
                               that feasible masks are not ranked out) */
    double mixed_delta;     /* MIXED: the bound assumed on |e32 - e64| and
                               |slack32 - slack64| (0 = 1e-8, above the proven
                               2e-9); a segment whose measured deviation over
                               its rescored masks exceeds it is scored again in
                               FP64 over every mask */
    int32_t secondary;      /* key among the feasible masks of the most
                               reducing level: OKR_SECONDARY_MAXERR (0) or
                               OKR_SECONDARY_SMICE, the latter with
                               OKR_PRECISION_FP64 or FP64_FACTORED and no
                               surrogate (OKR_E_UNSUPPORTED otherwise); read by
                               okr_plan too, which sizes the SMICE buffers */
    double smice_tol;       /* SMICE: masks within smice_tol of the smallest
                               SMICE tie, the lowest mask wins (0 = 1e-9); a
                               candidate within smice_tol / 100 of that window's
                               edge flags the segment ambiguous */
} okr_margins;

/* Sizes okr_plan() reports. */
typedef struct {
    int32_t n_segments;
    int32_t k_max;        /* largest segment */
    int64_t n_candidates; /* sum over segments of 2^k */
} okr_sizes;

/* Per-segment outcome. */
typedef struct {
    int32_t segment, k;
    uint32_t mask;      /* chosen aggregation of the segment */
    int32_t popcount;
    double e_loc;       /* error of the chosen mask over the affected nodes */
    double e_min;       /* smallest error at the chosen level */
    int32_t ambiguous;  /* a candidate lay within amb_tol of a decision boundary */
    int32_t n_scored;   /* masks scored exactly */
    double flops;       /* algorithmic flops of scoring the segment's 2^k
                           candidates (the method's own work per candidate and
                           snapshot, see okr_result.algorithmic_flops; 0 with
                           OKR_PRECISION_FP64_FACTORED) */
    float score_ms;     /* scoring-kernel time of the segment's chunk divided
                           by the chunk's segments (OKR_FLAG_TIMING) */
    int32_t n_refined;  /* MIXED: masks rescored in FP64 (shortlists A + B) */
    double fp32_dev;    /* MIXED: max |e32 - e64| over rescored masks with e64 <= 2 e_bar */
    int32_t score_groups;   /* FP64 scoring launch shape: snapshot groups, ... */
    int32_t score_mpl;      /* ... snapshots per pass, ... */
    int32_t chunk;          /* index of the launch chunk the segment ran in */
    double kernel_flops;    /* flops the per-mask scoring kernel itself performs
                               (shared tables replace the per-candidate
                               voltage-change products; 0 with FACTORED) */
    int32_t score_waves;    /* ... and waves sharing each 64 masks' chains (default rule or autotuned) */
    double key_gap;         /* margin of the decision: the smallest key (e_loc, or SMICE with
                               OKR_SECONDARY_SMICE) of a feasible mask of the chosen level outside the tie
                               window, minus the smallest (+inf if none).  Exact for FP64 and FP64_FACTORED;
                               MIXED and top_k take it over their FP64-rescored masks, which can only
                               overstate it */
    double smice_rise;      /* OKR_SECONDARY_SMICE: SMICE of the chosen mask minus SMICE of mask 0 (the
                               error the segment's reduction adds, summed over clusters and snapshots);
                               NaN with OKR_SECONDARY_MAXERR */
} okr_segment_result;

/* Outputs (HOST buffers owned by the caller). */
typedef struct {
    int32_t *super;          /* [n] aggregation map: super[i] = i when kept */
    int32_t *kept_parent;    /* [n] reduced-network parent of each kept node, -1 otherwise */
    double *Yk_diag;         /* [n][3][3] complex128: Y_Kron(i,i), zero rows for reduced nodes */
    double *Yk_off;          /* [n][3][3] complex128: Y_Kron(i, kept_parent[i]) */
    double *err_per_snapshot;/* [S] max error over all nodes of the final reduction */
    double *Vhat;            /* [S][n][3] complex128 scenario voltages, or NULL */
    okr_segment_result *seg; /* [n_segments] */
    float *features;         /* DEVICE [n_candidates][32] or NULL: per-mask surrogate
                                features of every segment, in segment then mask order */
    float *targets;          /* DEVICE [n_candidates] or NULL: ln(e_loc + 1e-12) of
                                every mask (FP64 scores); needs precision FP64 or FP64_FACTORED */
    int32_t n_kept;
    int32_t warnings;        /* OKR_W_* bits seen */
    double max_err;
    /* wall-clock phase times (ms) and summed kernel times (OKR_FLAG_TIMING) */
    double t_setup_ms, t_pf_ms, t_search_ms, t_final_ms;
    /* algorithmic_flops: per candidate and snapshot, 2|phi_r| per reduced
       node and hop to its super-node (moved current), 8|phi_e|^2 + 2|phi_e|
       per edge carrying it (voltage change), 2|phi| per segment node (shift),
       10 per node-phase of the affected region (magnitude, error, margins);
       plus 18 per reduced node per candidate (series sums); averaged exactly
       over the masks.  kernel_form_flops: what the scoring kernel computes. */
    double score_kernel_ms, algorithmic_flops;
    int32_t pf_iterations, n_score_launches; /* scoring launches: one per chunk */
    double kernel_form_flops;
} okr_result;

/* One handle per HIP stream (hip_stream may be NULL for the null stream).
 * The handle holds only host metadata (no paper passage: bookkeeping). */
int okr_create(okr_handle **h, void *hip_stream);

/* Validate the topology of the three-phase radial network (Section II.A: a
 * tree rooted at the slack, phase sets shrinking from parent to child, the
 * eligible nodes the reduction may remove) and the segments (the candidate
 * set of Section IV's search taken per segment: every subset of a segment's
 * eligible nodes), group independent segments into launch chunks, and report
 * the device workspace size for S snapshots plus the output sizes.  HOST
 * only; OKR_E_NOT_TREE / OKR_E_PHASE / OKR_E_UNSUPPORTED / OKR_E_ARG on
 * invalid input. */
int okr_plan(okr_handle *h, const okr_topology *topo, const okr_margins *mg,
             int32_t S, size_t *workspace_bytes, okr_sizes *sizes);

/* The search (Section IV, Algorithm 1 generalised to every subset of each
 * segment's eligible nodes): the scenario library by AC load flow (Section
 * III, library L) unless V^ is given; per segment and mask, the assignment
 * and current aggregation (Section II.C, eq. i_agg), the Kron-reduced
 * network (Section II.B, eq. Y_kron) and its fixed-current solve with
 * reduced nodes copying their super-node's voltage (Algorithm 1), the error
 * (eq. iter_obj) and margins (eq. v_abs and the voltage band), the
 * lexicographic arg-min; after the last segment the reduced network's
 * blocks (eq. Y_kron) and per-snapshot errors.  topo must be the planned
 * topology; d_workspace (DEVICE) must hold workspace_bytes >= the planned
 * size (OKR_E_WORKSPACE otherwise).  Synchronous on the handle's stream:
 * outputs are complete in `out` on return. */
int okr_reduce_feeder(okr_handle *h, const okr_yblocks *Y, const okr_topology *topo,
                      const okr_loads *loads, const okr_margins *mg,
                      void *d_workspace, size_t workspace_bytes, okr_result *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * search as okr_reduce_feeder, with the workspace taken from a scratch array
 * the library holds on each GPU it runs on (OKR_NOALLOC_SCRATCH_BYTES, held
 * until the process ends; its address is looked up once per device, on the
 * first call with that device current).  It calls no hipMalloc, hipFree or
 * other allocating routine.  The caller passes inputs and outputs as for
 * okr_reduce_feeder and must have the handle stream's device current.
 * Returns OKR_E_WORKSPACE when the planned workspace exceeds the array (for
 * example the 1000-node, 24-snapshot workload fits with margins.lanes = 1)
 * and OKR_E_ARG for OKR_FLAG_TIMING, OKR_FLAG_GRAPH, OKR_FLAG_AUTOTUNE or
 * OKR_FLAG_DUMP_SCORES (each would allocate events, graphs or host copies).
 * Every call on a GPU shares that GPU's array, which keeps the last call's
 * contents (the search initialises what it reads): calls that overlap on one
 * GPU, from any handle or stream, race and must be serialised by the caller. */
#define OKR_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int okr_reduce_feeder_noalloc(okr_handle *h, const okr_yblocks *Y, const okr_topology *topo,
                              const okr_loads *loads, const okr_margins *mg, okr_result *out);

/* With OKR_FLAG_DUMP_SCORES: copy segment `segment`'s per-mask error over
 * the affected nodes (eq. iter_obj) and band slack from the last call (HOST
 * double[2^k] each) and return k through *k. */
int okr_dump_scores(okr_handle *h, int32_t segment, double *e, double *slack, int32_t *k);

/* Surrogate MLP (learned pruning; not in the paper, which scores every
 * candidate: a ranking that lets okr_reduce_feeder rescore only the top_k
 * masks exactly, full enumeration as fallback).  Parameters are one FP32 buffer in
 * [out][in] layout: W1[256][32] b1[256] W2[256][256] b2[256] w3[256] b3[1]
 * (OKR_SURR_PARAMS floats).  The network maps 32 per-mask features (from
 * okr_result.features) through two GELU layers to y = ln(e_loc + 1e-12); its
 * GEMMs run on MFMA with BF16 operands and FP32 accumulation. */
#define OKR_SURR_FEATURES 32
#define OKR_SURR_PARAMS (256 * 32 + 256 + 256 * 256 + 256 + 256 + 1)

/* Device workspace bytes for okr_train_surrogate / okr_surrogate_grad /
 * okr_surrogate_forward with batches of `batch` rows (a multiple of 64). */
int okr_surrogate_workspace(int32_t batch, size_t *bytes);

/* Train in place (DEVICE params, Adam, mean-squared error) on n rows of
 * features X (DEVICE float [n][32]) and targets t (DEVICE float [n]) for
 * `epochs` passes of whole batches in an order drawn from `seed`; writes the
 * mean loss of each epoch to loss (HOST float [epochs]).  Synchronous. */
int okr_train_surrogate(const float *X, const float *t, int64_t n, int32_t epochs, int32_t batch, float lr,
                        uint64_t seed, float *params, void *work, size_t work_bytes, void *hip_stream,
                        float *loss);

/* Loss gradient of one batch (B rows, a multiple of 64) into grads (DEVICE
 * float [OKR_SURR_PARAMS]); the batch loss to *loss (HOST).  Synchronous. */
int okr_surrogate_grad(const float *params, const float *X, const float *t, int32_t B, float *grads,
                       float *loss, void *work, size_t work_bytes, void *hip_stream);

/* Predictions y (DEVICE float [n]) for features X (DEVICE float [n][32]),
 * n a multiple of 64 (at most the workspace batch).  Synchronous. */
int okr_surrogate_forward(const float *params, const float *X, int64_t n, float *y, void *work,
                          size_t work_bytes, void *hip_stream);

/* Self-test of the square root the FP64 scoring kernels use for voltage
 * magnitudes: y[i] = sqrt(x[i]) for n DEVICE doubles.  Synchronous on
 * hip_stream.  For tests of its rounding; not part of the search. */
int okr_selftest_sqrt(const double *x, double *y, int32_t n, void *hip_stream);

int okr_destroy(okr_handle *h);
const char *okr_last_error(const okr_handle *h);

#ifdef __cplusplus
}
#endif
#endif /* OKR_H */
