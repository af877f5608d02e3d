/* Prints "struct field offset size" for every field of the ABI structs and
 * "struct - sizeof" lines, compiled as plain C against include/liblogdet.h. */
#include <stddef.h>
#include <stdio.h>
#include "liblogdet.h"

#define F(S, f) printf(#S " " #f " %zu %zu\n", offsetof(S, f), sizeof(((S*)0)->f))
#define Z(S) printf(#S " - %zu 0\n", sizeof(S))

int main(void) {
  F(ld_ctx_opts, device); F(ld_ctx_opts, max_slots); F(ld_ctx_opts, hbm_budget_bytes);
  F(ld_ctx_opts, hip_stream); F(ld_ctx_opts, default_method); F(ld_ctx_opts, default_precision);
  Z(ld_ctx_opts);
  F(ld_params, method); F(ld_params, precision); F(ld_params, n_probes); F(ld_params, sketch_rank);
  F(ld_params, krylov_steps); F(ld_params, iop_window); F(ld_params, seed); F(ld_params, tol);
  F(ld_params, probe_dist); F(ld_params, subspace_rank); F(ld_params, adapt_tol);
  F(ld_params, adapt_every); F(ld_params, sketch_passes);
  Z(ld_params);
  F(ld_result, logdet); F(ld_result, tr_sketch); F(ld_result, tr_resid); F(ld_result, shift_c);
  F(ld_result, lambda_lo); F(ld_result, lambda_hi); F(ld_result, scale); F(ld_result, probe_steps);
  F(ld_result, matvecs); F(ld_result, min_steps); F(ld_result, n_breakdowns);
  F(ld_result, device_ms); F(ld_result, latency_ms); F(ld_result, basis_rank);
  Z(ld_result);
  F(ld_detail, probe_K); F(ld_detail, probe_norm2); F(ld_detail, probe_steps);
  F(ld_detail, tri_alpha); F(ld_detail, tri_beta); F(ld_detail, sketch_basis);
  Z(ld_detail);
  F(ld_tune_result, spmm_lanes); F(ld_tune_result, spmm_chunks); F(ld_tune_result, update_lanes);
  F(ld_tune_result, update_chunks); F(ld_tune_result, spmm_ms); F(ld_tune_result, spmm_default_ms);
  F(ld_tune_result, update_ms); F(ld_tune_result, update_default_ms);
  F(ld_tune_result, candidates); F(ld_tune_result, spmm_entry_split);
  F(ld_tune_result, spmm_interleave); F(ld_tune_result, spmm_row_stride);
  F(ld_tune_result, step_presub); F(ld_tune_result, step_presub_ms);
  F(ld_tune_result, step_plain_ms); F(ld_tune_result, spmm_row_groups);
  Z(ld_tune_result);
  F(ld_serving_stats, submitted); F(ld_serving_stats, completed); F(ld_serving_stats, ticks);
  F(ld_serving_stats, batched_steps); F(ld_serving_stats, batched_launches);
  F(ld_serving_stats, held_bytes); F(ld_serving_stats, peak_held_bytes);
  F(ld_serving_stats, budget_bytes); F(ld_serving_stats, buffer_allocs);
  F(ld_serving_stats, buffer_frees); F(ld_serving_stats, peak_active);
  F(ld_serving_stats, max_slots);
  Z(ld_serving_stats);
  F(ld_graph_stats, captures); F(ld_graph_stats, replays); F(ld_graph_stats, eager);
  F(ld_graph_stats, cached); F(ld_graph_stats, mode); F(ld_graph_stats, capture_failed);
  Z(ld_graph_stats);
  return 0;
}
