// Split (multi-pass streaming) operator application (device code in split.hip).
#pragma once

#include "batch.h"

namespace sgdg {

// One pass of y = A u for every problem and vector of the call (the scans must
// have run): stage 0 writes the v-stage W into C.Z, stage 1 writes the
// upper-partner part into C.y, stage 2 adds the x-stencils of W to C.y.
// bc: vectors per thread (1, 2 or 4 for d <= 2; 1 for d = 3)
template <class T>
void split_stage(const SplitCall<T>& C, int d, int R, int bc, int stage, hipStream_t s);
int split_points_per_item();
// x-stencil tile (edge t, v-run vb) for a grid with mx nodes per x-axis and nv v-nodes
void split_tile_shape(int d, int mx, int nv, int& t, int& vb);
int split_default_bc(int d);
bool split_vmajor();
int split_xcd();

}  // namespace sgdg
