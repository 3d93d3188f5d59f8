// Split (two-pass streaming) operator application (device code in split.hip).
#pragma once

#include "batch.h"

namespace sgdg {

// y = A u for every problem and vector of the call: v-stencil stage into C.Z,
// then x-stencils and upper-partner terms into C.y (the scans must have run).
// bc: vectors per thread (1, 2 or 4 for d <= 2; 1 for d = 3)
template <class T>
void split_apply(const SplitCall<T>& C, int d, int R, int bc, hipStream_t s);
int split_points_per_item();
int split_default_bc(int d);

}  // namespace sgdg
