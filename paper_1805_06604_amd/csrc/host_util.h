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
int round_rank(int r);
int64_t round_up(int64_t v, int64_t q);
// Split-K plan of one product; target_wg = 0 takes the single-problem default.
void plan_product(ProdArgs &a, int kernel, int64_t rows, int64_t rows_pad, int64_t K, int64_t ld,
                  int64_t target_wg);
}  // namespace host
}  // namespace nmf
