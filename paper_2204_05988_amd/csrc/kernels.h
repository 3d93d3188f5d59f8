// Kernel launchers of libsgdg (device code in kernels.hip).
#pragma once

#include "batch.h"

namespace sgdg {

// A segment layout on the device: SegInfo per segment and the block table of
// a segmented launch (chunks of kChunk elements).
struct SegTable {
  const SegInfo* segs = nullptr;
  const BlockRef* blk = nullptr;
  int nseg = 0, nblk = 0, nchunks = 0;
};

template <class T>
struct KernelsT {
  // partial[(chunk0 + c) * nvec + k] = <V_k, w> over chunk c of each segment
  static void seg_dots(const SegTable& S, const T* V, int64_t vstride, int nvec, const T* w, double* partial,
                       hipStream_t s);
  // w += sign * sum_k coef[seg][k] V_k; optional partial norms of the result
  static void seg_axpy(const SegTable& S, const T* V, int64_t vstride, int nvec, const double* coef, int cstride,
                       T* w, double sign, double* partial_norm, hipStream_t s);
  // w -= sum_k coef[seg][k] V_k, then partial as seg_dots of the new w (one
  // Gram-Schmidt pass and the next pass's projections in one launch)
  static void seg_axpy_dots(const SegTable& S, const T* V, int64_t vstride, int nvec, const double* coef,
                            int cstride, T* w, double* partial, hipStream_t s);
  static void seg_scale(const SegTable& S, const T* w, const double* scal, T* out, hipStream_t s);
  static void seg_norm2(const SegTable& S, const T* w, double* partial, hipStream_t s);
  // combination technique on the CT segment table (upper grids then lower grids per problem)
  static void ct_gather(const SegTable& S, const T* r, T* b, hipStream_t s);
  static void ct_combine(const SegTable& S, const T* ct, T* z, hipStream_t s);
  static void minv(const SegTable& S, const T* x, T* y, hipStream_t s);
  // y = (Tt + delta Ct + Gt)^-1 x per point (time blocks only, no mass factor)
  static void tinv(const SegTable& S, const T* x, T* y, hipStream_t s);
  // one Chebyshev step of the Jacobi-preconditioned mass solve M_axis z = b
  // along axis 0 (x) or 1 (v) of every segment (see mass_cheb_coefs):
  //   d_out = cd * d + cr * D^-1 (b - M x),  x_out = x + d_out
  // first = 1: x = d = 0 (not read).  tinv = 1: x_out is mapped by the time
  // blocks (Tt + delta Ct + Gt)^-1 before it is stored.
  static void mass_cheb(const SegTable& S, int axis, double cd, double cr, int first, int tinv, const T* b,
                        const T* x, const T* d, T* x_out, T* d_out, hipStream_t s);
  // exact tridiagonal (d = 1) mass solve along axis 0 or 1 of every segment,
  // one thread per grid line (Thomas; cyclic lines by Sherman-Morrison).
  // y may equal b; cbuf, zbuf: scratch of the segment layout's size.
  static void mass_thomas(const SegTable& S, int axis, int max_lines, const T* b, T* y, T* cbuf, T* zbuf,
                          hipStream_t s);
  static void axpby(int64_t n, T a, const T* x, T b, T* y, hipStream_t s);
  static void copy(int64_t n, const T* x, T* y, hipStream_t s);
  static void fill(int64_t n, T v, T* y, hipStream_t s);
};

void convert_f64_to_f32(int64_t n, const double* x, float* y, hipStream_t s);
void convert_f32_to_f64(int64_t n, const float* x, double* y, hipStream_t s);

// GMRES bookkeeping for a batch of independent segments (one thread per segment).
struct GmresState {
  double* H;      // [seg][(m+1)*m]  column-major: H[j*(m+1) + i]
  double* cs;     // [seg][m]
  double* sn;     // [seg][m]
  double* g;      // [seg][m+1]
  double* bnorm;  // [seg]
  double* beta;   // [seg] current residual estimate
  int* active;    // [seg] 1 iterating, 0 converged/stopped, -1 non-finite
  int* kused;     // [seg]
  double* hcol;   // [seg][m+1] projection coefficients of the current column
  double* inv;    // [seg] 1/h_{j+1,j} for the next basis vector (0 when stopped)
  double* y;      // [seg][m]
  int m;
};
void gmres_start(int nseg, const GmresState& st, const SegInfo* segs, const double* partial, double tol, int first,
                 hipStream_t s);
void gmres_add_proj(int nseg, const GmresState& st, const SegInfo* segs, const double* partial, int j, hipStream_t s);
void gmres_givens(int nseg, const GmresState& st, const SegInfo* segs, const double* partial, int j, double tol,
                  hipStream_t s);
void gmres_lsq(int nseg, const GmresState& st, hipStream_t s);

// Data functionals: slice projection of nodal samples at Gauss points in time.
void project_time(int64_t n, int nq, int R, const double* wts, const double* samples, double* out, hipStream_t s);
// Jump term on the per-grid segment table of one problem (src_off = point offset of the grid):
// trace = sum_s u_s (Legendre values 1 at the right end); b[g][s] = (-1)^s (M trace)[g].
void trace_sum(const SegTable& S, int Rprev, const double* u, double* out, hipStream_t s);
void spread_left(const SegTable& S, const double* m, double* b, hipStream_t s);

}  // namespace sgdg
