// All-pairs force kernels (the force function as stated, no cutoff): their
// launch, called by the C entry point pmd_allpairs_forces.
#pragma once

#include <hip/hip_runtime.h>

namespace pmd {

hipError_t launch_allpairs(int precision, int n, const double* x, const double box[3], double eps,
                           double sigma, double* f, double* u, double* e, hipStream_t s);

}  // namespace pmd
