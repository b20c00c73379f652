// Host-side helpers of the engine shared with the batch engine.
#pragma once

#include "nmf.h"
#include "nmf_internal.h"

#include <string>

namespace nmf {
namespace host {
// The message returned by nmf_last_error(NULL) on this thread.
void set_error(const std::string &msg);
nmf_status check_params(const nmf_params *p);
nmf_status check_matrix(const nmf_matrix *X);
// check_matrix without the scan of the dense values (shape, pointers, CSR).
nmf_status check_matrix_shape(const nmf_matrix *X);
// Copies cnt floats from src to dst in one pass, checking them on the way:
// returns the index of the first non-finite value (dst then partly written)
// or -1, and sets *nonzero when any value is nonzero.
int64_t copy_checked(const float *src, float *dst, int64_t cnt, bool *nonzero);
int round_rank(int r);
int64_t round_up(int64_t v, int64_t q);
// Split-K plan of one product; target_wg = 0 takes the single-problem default.
void plan_product(ProdArgs &a, int kernel, int64_t rows, int64_t rows_pad, int64_t K, int64_t ld,
                  int64_t target_wg);
}  // namespace host
}  // namespace nmf
