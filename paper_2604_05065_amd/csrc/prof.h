// Event timing of the blocked product kernel (prof.cpp).
#pragma once

#include <hip/hip_runtime.h>

namespace aplicur {

// Kinds of timed launch: A X and A^T X with FP64 accumulation (0, 1), FP32
// products (2, 3), BF16 products (4, 5).
constexpr int kProfKinds = 6;

// While timing is on (aplicur_prof_products), hands out an event pair for
// one launch of the given kind and returns true; false (no events) when
// timing is off, on another device, or the record is full.
bool prof_take(int kind, hipEvent_t* e0, hipEvent_t* e1);

}  // namespace aplicur
