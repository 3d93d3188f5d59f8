// Fused box-tiled operator application (device code in fused.hip).
#pragma once

#include "batch.h"

namespace sgdg {

// one step of both partner-sum scans over every problem of the batch, the
// factor groups split over `chunks` blocks per item
template <class T>
void fused_scan_step(const FusedCall<T>& C, int nsitems, int d, int R, int chunks, hipStream_t s);
// the box-tiled accumulation over all grids of all problems (one launch)
template <class T>
void fused_tiles(const FusedCall<T>& C, int d, int R, hipStream_t s);
int fused_rows_per_thread();
int fused_threads();

}  // namespace sgdg
