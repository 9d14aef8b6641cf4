/* Prints the layout of the structs in hmle.h (name, field, offset, size and
 * the struct's total size) and the checkpoint size constant, read by
 * tests/test_abi_layout.py to check the Python binding's ctypes structures and
 * constants against the C compiler's view. */
#include <stddef.h>
#include <stdio.h>

#include "../../include/hmle.h"

#define F(S, f) printf("%s %s %zu %zu\n", #S, #f, offsetof(S, f), sizeof(((S*)0)->f))
#define T(S) printf("%s _size %zu %zu\n", #S, sizeof(S), (size_t)0)

int main(void) {
  F(hmle_theta, sigma2); F(hmle_theta, range); F(hmle_theta, nu); F(hmle_theta, tau2); T(hmle_theta);
  F(hmle_opts, leaf_size); F(hmle_opts, eta); F(hmle_opts, aca_tol); F(hmle_opts, max_rank);
  F(hmle_opts, precision); F(hmle_opts, pair_chunk); F(hmle_opts, sketch_group); F(hmle_opts, spd_margin);
  F(hmle_opts, seg_entries); F(hmle_opts, gseg_rows); F(hmle_opts, sum_kc); T(hmle_opts);
  F(hmle_tune_entry, opts); F(hmle_tune_entry, ms); T(hmle_tune_entry);
  F(hmle_fit_opts, max_iter); F(hmle_fit_opts, tol); F(hmle_fit_opts, step); F(hmle_fit_opts, use_backoff);
  F(hmle_fit_opts, report_every); F(hmle_fit_opts, profile_variance); T(hmle_fit_opts);
  F(hmle_fit_report, evals); F(hmle_fit_report, iters); F(hmle_fit_report, failed_evals);
  F(hmle_fit_report, converged); F(hmle_fit_report, logL); F(hmle_fit_report, wall_s); T(hmle_fit_report);
  printf("const FIT_STATE_BYTES %d 0\n", HMLE_FIT_STATE_BYTES);
  return 0;
}
