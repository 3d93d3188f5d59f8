// Multi-problem device descriptors and work tables.
//
// Every device launch of the library works on a *batch* of independent strip
// problems (one problem is a batch of one).  Vectors of a batch are the
// concatenation of the problems' vectors; static per-problem descriptors live
// in device memory and carry the problem's offsets into the concatenated
// layouts, and every launch is driven by a work table that maps a block to
// (problem, grid, tile) or (segment, chunk).
#pragma once

#include "sgdg_internal.h"

namespace sgdg {

// Static description of one problem's grid set for the operator kernels.
struct ProbDesc {
  DevGrids G;          // grid set (upper diagonal, or upper+lower for the grid problems)
  DevGrids Gl;         // lower diagonal (scan arrays), same R
  int64_t poff[kMaxGrids + 1];  // point offsets (nx*nv) of G
  DevDomain DX, DV;
  DevOp op;
  int mx[kMaxLevels], mv[kMaxLevels];  // nodes per axis by level
  int xper, vper;
  int off[kMaxS][3];   // Kuhn stencil offsets
  int diag_only;       // 1: diagonal blocks only (no scans, no partner sums)
  int64_t u_off;       // start of this problem's vector in the concatenated layout
  int64_t y_off;       // start of its output vector
  int64_t pt_off, qt_off;  // start of its scan arrays
  int64_t z_off;           // start of its staged v-stage arrays (split application)
  // partner-scan recursion through restricted scan arrays:
  //   Rv_t = (I (x) E^vT) Pt on lower grid t-1, shape nx(low t-1) x nv(low t), feeds lower target t
  //   Rx_l = (E^xT (x) I) Qt on lower grid l+1, shape nx(low l) x nv(low l+1), feeds upper target l
  int64_t rv_off, rx_off;              // start of this problem's arrays (per factor group stride rv_len/rx_len)
  int64_t rv_len, rx_len;              // elements per factor group (all slices, all targets)
  int64_t rvo[kMaxGrids], rxo[kMaxGrids];  // start of target t's block within one group
};

// A box of x-nodes times a box of v-nodes of one grid of one problem.
struct FusedItem {
  int prob, grid;
  int xb[3], xs[3];
  int vb[3], vs[3];
};

// One block of a scan step: target lower grid of one problem, one side.
struct ScanItem {
  int prob, side;      // side 0: lower partners (Pt), 1: upper partners (Qt)
  int lg;              // target lower grid
  int grp;             // 0: scan step (base + recursion), 2: restriction feeding the next step
  int64_t start;       // first element of the block in the target
};

template <class T>
struct FusedCall {
  const ProbDesc* descs;
  const FusedItem* items;
  const ScanItem* sitems;
  int nitems;
  int max_u, max_stage, max_tab;  // LDS elements (u halo box, group stage) / ints per block
  int B;                   // vectors per problem
  int64_t u_bstride, y_bstride, pt_bstride, qt_bstride;  // batch strides
  const T* u;
  T* y;
  T* Pt;                   // [b][problem: V-group j][lower grids: nx][nv][R]
  T* Qt;                   // [b][problem: X-group m][lower grids: nx][nv][R]
  int64_t rv_bstride, rx_bstride;
  T* Rv;                   // restrictions of the previous scan step, same slice order
  T* Rx;
  // 1: the scans fill the partner arrays only where the split passes read
  // them (the op's xpt_mask / xqt_mask); 0: everywhere (the box-tiled kernel)
  int sparse_partners;
};

// Split application: one block of points of one grid of one problem.
struct SplitItem {
  int prob, grid;
  int64_t p0;  // first point (x * nv + v) of the block
  // upper-partner pass: bit m, Qt^m can be nonzero on one of the block's
  // x-rows (groups >= 64: always)
  uint64_t gmask;
  // upper-partner pass (d <= 2): the in-lattice prolongation slots of the
  // block's points, as x * nvl + coarse node on the lower grid, lie in
  // [q0, q0 + qn); qn = 0 when the grid has no upper partner
  int64_t q0;
  int qn;
};

// A tile of the x-stencil pass: t^d x-nodes from x0 (lattice coordinates)
// times vb v-nodes from v0, staged in LDS with a one-node x-halo.
struct TileItem {
  int prob, grid;
  int x0[3];
  int v0, t, vb;
  uint64_t gmask;  // bit m: X-group m has a nonzero row among the tile's x-nodes (groups >= 64: always)
};

template <class T>
struct SplitCall {
  const ProbDesc* descs;
  const SplitItem* items;
  int nitems;
  int B;                   // vectors per problem
  int64_t u_bstride, y_bstride, pt_bstride, qt_bstride, z_bstride;
  const T* u;
  T* y;
  const T* Pt;
  const T* Qt;
  T* Z;                    // [b][problem: X-group m][grid: nx][nv][R] staged v-stage W^m
  int max_qn;              // largest SplitItem::qn (LDS of the upper-partner pass)
  int x_assign;            // 1: no upper-partner pass ran (block-diagonal kinds), pass 3 writes y
  const TileItem* tiles;   // x-stencil pass on LDS tiles (ntiles = 0: per-point items)
  int ntiles;
  int max_tile;            // largest (t + 2)^d vb of a tile
  int xcd;                 // 1: each XCD takes a contiguous range of (vector group, item) blocks
};

// A contiguous segment of a concatenated vector: one component grid of one
// problem (grid problems of the combination technique) or one whole problem
// (strip FGMRES).  The CT fields describe the transfers.
struct SegInfo {
  int prob, lx, lv, nx, nv, R;
  int64_t off;          // start in the segment layout
  int64_t len;          // elements
  int chunk0, nchunk;   // reduction chunks owned by the segment
  // combination technique (lower segments: restriction source; upper: combination partner)
  int kind;             // 0 upper grid, 1 lower grid, 2 whole problem
  int64_t src_off;      // upper: start of the grid in the residual (upper-diagonal) layout;
                        // lower: start of its source upper grid (lx+1, lv) there
  int64_t low_off;      // upper with lx > lmin: start of the lower grid (lx-1, lv) in the CT layout, else -1
  int nx_src;           // lower: nx of the source upper grid; upper: nx of the lower partner
  int S;                // stencil size of the x-domain
  const int32_t* xchi;  // x children table of level lx (lower segments)
  const double* xchiw;
  const int32_t* xpar;  // x parent table of level lx (upper segments)
  const double* xparw;
  const double* mxd;    // x mass factor rows of level lx ([nx][Sx], slot 0 = diagonal)
  const double* mvd;    // v mass factor rows of level lv ([nv][Sv])
  int Sx, Sv;
  double pinv[kMaxR * kMaxR];
  // exact or polynomial mass inverses of the grid-problem preconditioner
  const int32_t* xnbr;  // x stencil neighbours of level lx ([nx][Sx], self outside the box)
  const int32_t* vnbr;  // v stencil neighbours of level lv ([nv][Sv])
  int xper, vper;       // periodic domains
  int sm, sp;           // d = 1: stencil slots of the offsets -1 and +1
};

struct BlockRef {  // one block of a segmented launch
  int seg, chunk;
};

constexpr int kChunk = 512;  // elements per block in segmented launches

}  // namespace sgdg
