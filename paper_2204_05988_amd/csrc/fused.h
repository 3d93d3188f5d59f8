// Fused box-tiled operator application (device code in fused.hip).
#pragma once

#include "kernels.h"

namespace sgdg {

// One work item: a box of x-nodes times a box of v-nodes of one grid.
struct FusedItem {
  int grid;
  int xb[3], xs[3];  // x-box start and size (lattice coordinates)
  int vb[3], vs[3];  // v-box start and size
};

template <class T>
struct FusedArgs {
  DevGrids G;        // upper grids (R = op.Rin slices)
  DevGrids Gl;       // lower grids holding the scan arrays (same R)
  GridPts P;         // point offsets of the upper grids
  DevDomain DX, DV;
  DevOp op;
  int mx[kMaxLevels], mv[kMaxLevels];  // nodes per axis by level
  int xper, vper;                      // periodic domains
  int off[kMaxS][3];                   // Kuhn stencil offsets (same for both domains)
  const FusedItem* items;
  int nitems;
  int max_stage;                       // LDS elements needed by the largest item
  int max_tab;                         // LDS ints of the per-block index tables
  int diag_only;                       // 1: only the diagonal blocks A_{l,l}
  int B;
  const T* u;
  T* y;
  T* Pt;   // [nvg][B][lower total]
  T* Qt;   // [nxg][B][lower total]
};

// level scans of both partner sums (n-1 launches on the lower diagonal)
template <class T>
void fused_scans(const FusedArgs<T>& A, int d, hipStream_t s);
// the box-tiled accumulation over all grids (one launch)
template <class T>
void fused_tiles(const FusedArgs<T>& A, int d, hipStream_t s);
int fused_points_per_block();
int fused_rows_per_thread();
int fused_threads();

}  // namespace sgdg
