// Internal helpers shared by the fit entry points (not part of the C ABI).
#pragma once
#include <cstdint>

#include "../../include/hmle.h"

namespace hmle {

// A batch built from identical copies of one point set (the candidate batch of
// hmle_fit_batch): its copy count and the size of one copy. HMLE_E_INVALID
// (with the problem's error message set) when the problems differ in size,
// ordering or coordinates.
hmle_status candidate_layout(hmle_problem p, int32_t* count, int64_t* n1);

// A device buffer of the batch's total point count owned by the problem
// (allocated on first use, kept until hmle_destroy), filled with `count`
// copies of the n1 values z (device) on the problem's stream.
hmle_status candidate_data(hmle_problem p, const double* z, int32_t count, int64_t n1, double** out);

}  // namespace hmle
