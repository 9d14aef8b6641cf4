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

// 32-bit FNV-1a fingerprint of what a fit checkpoint depends on besides the
// problem size: the data z (device, the problem's n values) and the options
// that define the objective (leaf size, eta, accuracy, rank cap, precision and
// the resolved definiteness floor).
hmle_status fit_fingerprint(hmle_problem p, const double* z, uint32_t* out);

}  // namespace hmle
