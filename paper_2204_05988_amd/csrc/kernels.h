// Kernel launchers of libsgdg (device code in kernels.hip).
#pragma once

#include "sgdg_internal.h"

namespace sgdg {

// Contiguous segments of a vector (one per component grid, or one in total).
struct Segs {
  int n = 0;
  int64_t off[kMaxGrids + 1] = {};
};

// Point offsets (nx*nv per grid, no time slices) for a grid set.
struct GridPts {
  int64_t poff[kMaxGrids + 1] = {};
};

template <class T>
struct KernelsT {
  // lower grid g (lx, lv) = (I (x) E^x_{lx+1,lx}^T (x) I) upper grid g+1 (lx+1, lv)
  static void restrict_x(const DevGrids& Gout, const DevGrids& Gin, const DevDomain& DX, const T* in, T* out,
                         hipStream_t s);
  // out_up(lx,lv) = a_up(lx,lv) - (E^x (x) I) a_low(lx-1,lv)
  static void combine(const DevGrids& Gup, const DevGrids& Glow, int lmin, const DevDomain& DX, const T* up,
                      const T* low, T* out, int R, hipStream_t s);
  // y = (Pinv (x) Mx^-1 (x) Mv^-1) x  approximately (Jacobi + Chebyshev)
  static void minv(const DevGrids& G, const GridPts& P, const DevDomain& DX, const DevDomain& DV,
                   const double* pinv, int sweeps, const T* x, T* y, T* tmp1, T* tmp2, hipStream_t s);
  // Krylov primitives over segments (FP64 accumulation)
  static void seg_dots(const Segs& S, const T* V, int64_t vstride, int nvec, const T* w, double* partial,
                       int nchunks, hipStream_t s);
  static void seg_axpy_multi(const Segs& S, const T* V, int64_t vstride, int nvec, const double* coef,
                             int cstride, T* w, double sign, double* partial_norm, int nchunks,
                             hipStream_t s);
  static void seg_scale(const Segs& S, const T* w, const double* scal, T* out, hipStream_t s);
  static void seg_norm2(const Segs& S, const T* w, double* partial, int nchunks, hipStream_t s);
  static void axpby(int64_t n, T a, const T* x, T b, T* y, hipStream_t s);
  static void copy(int64_t n, const T* x, T* y, hipStream_t s);
  static void fill(int64_t n, T v, T* y, hipStream_t s);
};

void convert_f64_to_f32(int64_t n, const double* x, float* y, hipStream_t s);
void convert_f32_to_f64(int64_t n, const float* x, double* y, hipStream_t s);
void add_f32_to_f64(int64_t n, const float* x, double* y, hipStream_t s);

// partial[seg][chunk][k] -> out[seg][k]  (deterministic order)
void finish_dots(int nseg, int nvec, int nchunks, const double* partial, double* out, hipStream_t s);

// GMRES bookkeeping for a batch of independent segments (one thread per segment).
struct GmresState {
  double* H;      // [seg][(m+1)*m]  column-major: H[j*(m+1) + i]
  double* cs;     // [seg][m]
  double* sn;     // [seg][m]
  double* g;      // [seg][m+1]
  double* bnorm;  // [seg]
  double* beta;   // [seg]
  int* active;    // [seg]
  int* kused;     // [seg]
  double* hcol;   // [seg][m+1] scratch: dots of the current column
  double* inv;    // [seg] 1/h_{j+1,j} for the next basis vector (0 when stopped)
  double* y;      // [seg][m]
  int m;
};
// Start of a cycle: beta from partial norms, g = beta e1, inv = 1/beta (0 if converged/zero).
void gmres_start(int nseg, const GmresState& st, const double* partial, int nchunks, double tol, int first,
                 hipStream_t s);
// Accumulate one projection pass: H[:, j] += hcol (from partials).
void gmres_add_proj(int nseg, const GmresState& st, const double* partial, int nchunks, int j, hipStream_t s);
// Norm of w, Givens rotation of column j, convergence bookkeeping.
void gmres_givens(int nseg, const GmresState& st, const double* partial, int nchunks, int j, double tol,
                  hipStream_t s);
// Back substitution y = H^-1 g over kused columns.
void gmres_lsq(int nseg, const GmresState& st, hipStream_t s);

// Data functionals: slice projection of nodal samples at Gauss points in time.
void project_time(int64_t n, int nq, int R, const double* wts, const double* samples, double* out,
                  hipStream_t s);
// Jump term: trace = sum_s u_s (Legendre values 1 at the right end);
// b[g][s] = (-1)^s (M trace)[g]  (Legendre values at the left end).
void trace_sum(const DevGrids& G, const double* u, double* out, hipStream_t s);
void spread_left(const DevGrids& G, int R, const double* m, double* b, hipStream_t s);

}  // namespace sgdg
