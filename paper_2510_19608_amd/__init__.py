"""MI355X (gfx950) segment-exhaustive Kron-reduction search (Opti-KRON).

The compute path is the HIP library ``libokr.so`` behind the C ABI declared in
``include/okr.h`` (and ``include/okr_greedy.h`` for the single-move greedy
search of Algorithm 1); ``binding`` marshals arguments into it.  There is no CPU
fallback: without the built library or a GPU the calls raise.
"""
from .binding import (OKR, SURR_FEATURES, SURR_PARAMS, OkrError, Reducer, lib, okr_create, okr_destroy,
                      okr_dump_scores, okr_last_error, okr_plan, okr_reduce_feeder, okr_surrogate_forward,
                      okr_surrogate_grad, okr_surrogate_workspace, okr_train_surrogate, reduce_feeder,
                      Greedy, greedy, evaluate_assignment, okr_greedy_create, okr_greedy_destroy,
                      okr_greedy_evaluate, okr_greedy_last_error, okr_greedy_plan, okr_greedy_radialize,
                      okr_greedy_run)

__all__ = ["OKR", "SURR_FEATURES", "SURR_PARAMS", "OkrError", "Reducer", "lib", "okr_create", "okr_destroy",
           "okr_dump_scores", "okr_last_error", "okr_plan", "okr_reduce_feeder", "okr_surrogate_forward",
           "okr_surrogate_grad", "okr_surrogate_workspace", "okr_train_surrogate", "reduce_feeder",
           "Greedy", "greedy", "evaluate_assignment", "okr_greedy_create", "okr_greedy_destroy",
           "okr_greedy_evaluate", "okr_greedy_last_error", "okr_greedy_plan", "okr_greedy_radialize",
           "okr_greedy_run"]
