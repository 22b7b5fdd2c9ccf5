/*
 * okr_greedy.h -- C ABI of the greedy single-move reduction search
 * (Algorithm 1 of arXiv 2510.19608, Section IV), of the evaluation of a
 * fixed reduction over many loading scenarios (the robustness study of
 * Section VI) and of the three-phase radialization of a reduction
 * (Section V), on MI355X (gfx950).
 *
 * Algorithm 1, as computed here:
 *   state: every node's super-node (initially itself) and the aggregated load
 *   currents I = A I^ (a super-node carries its cluster's currents);
 *   repeat:
 *     candidates: every ordered pair (s, r) of super-nodes whose clusters are
 *       joined by an edge of the network (adjacency after contraction) with
 *       the phases of r a subset of those of s; both directions of an edge
 *       are candidates; the slack's cluster never moves;
 *     each candidate, independently: r's cluster current moves to s, the full
 *       network is solved with the currents fixed and the slack at V0, every
 *       reduced node takes its super-node's voltage, e = ||V^| - |V^c|| per
 *       node, phase and scenario; feasible when max e <= e_bar; SMICE = sum
 *       over scenarios and clusters of the cluster's largest member error;
 *     the feasible candidate with the smallest SMICE is applied (clusters
 *       merge, currents aggregate); stop when no candidate is feasible.
 *   Candidate ids: the edge (x, parent(x)) joining two clusters gives id 2x
 *   (the child-side cluster moves up) and 2x + 1 (the parent-side cluster
 *   moves down).  SMICE values within tie_tol of the minimum tie; the lowest
 *   id wins.
 *
 * Types okr_yblocks and okr_loads and the error codes are those of okr.h.
 * The library allocates no device memory: the caller passes a device
 * workspace of the size okr_greedy_plan() reports.  Calls on one handle must
 * not overlap.
 */
#ifndef OKR_GREEDY_H
#define OKR_GREEDY_H

#include "okr.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct okr_greedy okr_greedy;

/* okr_greedy_params.flags: score candidates incrementally (only the clusters
 * whose super-node lies under lca(r, s) towards r or s, and the merged
 * cluster) even where every node of every candidate could be scored.  The
 * incremental form is used anyway when S * n exceeds 6144; it needs
 * n <= 12288.  Both forms give the same moves. */
#define OKR_GREEDY_INCREMENTAL 0x100u

typedef struct {
  double e_bar;      /* error bound of Algorithm 1 (p.u.), inclusive */
  double tie_tol;    /* SMICE tie tolerance (1e-11 if 0) */
  double amb_tol;    /* ambiguity margin of the step flags (1e-13 if 0) */
  int32_t max_iter;  /* stop after this many moves (0: until none is feasible) */
  uint32_t flags;    /* OKR_FLAG_VHAT_GIVEN: loads->Vhat holds V^ (no load flow);
                        OKR_FLAG_TIMING: time the candidate-scoring launches;
                        OKR_GREEDY_INCREMENTAL (below) */
  double pf_tol;     /* load-flow stopping rule (1e-13 if 0) */
  int32_t pf_maxit;  /* load-flow iteration cap (100 if 0) */
  int32_t pad;
} okr_greedy_params;

/* One applied move. */
typedef struct {
  int32_t cand;        /* candidate id (see above) */
  int32_t s, r;        /* super-node that absorbs, super-node that moves */
  int32_t ambiguous;   /* a feasible SMICE within amb_tol of the tie threshold,
                          or an active candidate's error within amb_tol of e_bar */
  int32_t n_cand;      /* candidates of this iteration */
  int32_t n_feasible;  /* feasible candidates of this iteration */
  double smice;        /* SMICE of the applied move */
  double emax;         /* its largest error over nodes, phases and scenarios */
} okr_greedy_step;

typedef struct {
  int32_t* super;            /* HOST [n]: final super-node of every node */
  okr_greedy_step* steps;    /* HOST [n]: the applied moves, in order */
  double* err_per_snapshot;  /* HOST [S]: final largest error per scenario */
  int32_t n_steps;           /* moves applied */
  int32_t n_kept;            /* super-nodes left */
  double max_err;            /* max of err_per_snapshot */
  double t_pf_ms;            /* load flow and set-up, HIP events */
  double t_search_ms;        /* the iterations, HIP events */
  int32_t pf_iterations;     /* largest load-flow iteration count (0 when V^ given) */
  int32_t n_score_launches;  /* candidate-scoring launches that ran */
  double t_score_ms;         /* with OKR_FLAG_TIMING: summed duration of the
                                candidate-scoring launches (HIP events on the
                                handle's stream), else 0 */
  int64_t n_scored;          /* candidates scored in the iterations that applied
                                a move */
  int32_t incremental;       /* 1 when only the clusters a move can change were
                                scored again (see OKR_GREEDY_INCREMENTAL) */
  int32_t pad2;
} okr_greedy_result;

/* Handle on a HIP stream (NULL = the null stream).  Returns OKR_E_ARG on a
 * null out pointer. */
int okr_greedy_create(okr_greedy** g, void* hip_stream);

/* Validates the tree (parent[0] = -1, every node reachable from node 0) and
 * the phases (1..7, each node's phases within its parent's), HOST arrays of n
 * entries, and reports the device workspace needed for S scenarios.  The
 * search (okr_greedy_run) additionally needs S <= 64 (the moved currents are
 * staged in LDS) and, when S * n > 6144, n <= 12288; okr_greedy_evaluate has
 * no such limits.
 * Errors: OKR_E_ARG, OKR_E_NOT_TREE, OKR_E_PHASE. */
int okr_greedy_plan(okr_greedy* g, int32_t n, const int32_t* parent, const uint8_t* phase, int32_t S,
                    size_t* workspace_bytes);

/* Runs Algorithm 1.  Y (DEVICE, okr.h layout) and loads (S_load and Vhat
 * DEVICE, V0 HOST, loads->S must equal the planned S); d_workspace DEVICE of
 * at least the planned size; out's arrays HOST, caller-owned.  Synchronous
 * on the handle's stream.  Errors: OKR_E_ARG, OKR_E_WORKSPACE,
 * OKR_E_UNSUPPORTED (S or n above the limits, or shunts / asymmetric blocks),
 * OKR_E_SINGULAR, OKR_E_PHASE, OKR_E_PF_DIVERGED, OKR_E_HIP. */
int okr_greedy_run(okr_greedy* g, const okr_yblocks* Y, const okr_loads* loads, const okr_greedy_params* p,
                   void* d_workspace, okr_greedy_result* out);

/* Scores a fixed assignment (super[n], HOST; every cluster connected, every
 * node's phases within its super-node's) over loads->S scenarios (the
 * planned S): load flow, aggregated currents, fixed-current solve, largest
 * error per scenario into err_per_snapshot (HOST [S]) and their max into
 * *max_err (HOST, may be NULL).  Synchronous.  Errors as okr_greedy_run, and
 * OKR_E_ARG for an invalid assignment. */
int okr_greedy_evaluate(okr_greedy* g, const okr_yblocks* Y, const okr_loads* loads, const int32_t* super,
                        const okr_greedy_params* p, void* d_workspace, double* err_per_snapshot, double* max_err);

/* Three-phase radialization (Section V) of a fixed assignment (super[n],
 * HOST, as for okr_greedy_evaluate).  The Kron-reduced network of the
 * super-nodes is an edge-disjoint union of cliques, one per connected group
 * of reduced nodes, over the kept nodes bordering it (Lemma 2: the pattern
 * is that of the single-phase network); a clique of three or more kept nodes
 * is a mesh.  Its critical nodes, the nodes of degree 3 or more in the
 * sub-tree of the feeder spanning the clique, are kept again (with no
 * injection of their own), which makes the reduced network radial.
 * Outputs (HOST): kept_radial[n] (1 for super-nodes and critical nodes),
 * kept_parent[n] (each node's nearest kept proper ancestor in the radialized
 * set, -1 at the slack: the edges of the radial reduced network),
 * *n_critical, and the voltage checks over the first min(loads->S, 4)
 * scenarios (the check costs n^2 per scenario; may be NULL):
 * *dv_radial, the largest distance between the kept nodes' voltages of the
 * radial network built on kept_parent (series impedances, aggregated
 * currents) and those of the full network (about 1e-15 when radialization
 * succeeded), and *dv_meshed, the same for the network built on the kept
 * parents of the super-nodes alone (nonzero when the reduction meshes).
 * Synchronous.  Errors as okr_greedy_evaluate. */
int okr_greedy_radialize(okr_greedy* g, const okr_yblocks* Y, const okr_loads* loads, const int32_t* super,
                         const okr_greedy_params* p, void* d_workspace, uint8_t* kept_radial, int32_t* kept_parent,
                         int32_t* n_critical, double* dv_radial, double* dv_meshed);

int okr_greedy_destroy(okr_greedy* g);
const char* okr_greedy_last_error(const okr_greedy* g);

#ifdef __cplusplus
}
#endif

#endif /* OKR_GREEDY_H */
