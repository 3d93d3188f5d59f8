// Device kernels of libsgdg for gfx950 (wave64), all driven by segment tables:
//  * Krylov primitives over segments (one component grid of one problem, or
//    one whole problem): dot products of a block of basis vectors, fused
//    multi-axpy with the norm of the result, per-segment scaling.  Reductions
//    run in FP64 and in a fixed order (per-chunk partial sums, then per
//    segment), so results are reproducible run to run.
//  * GMRES bookkeeping, one thread per segment (Givens rotations, residual
//    estimates, convergence and breakdown flags, back substitution).
//  * The transfers of the combination technique (Algorithm 1): restriction of
//    the residual in x to the lower diagonal, the combination step, and the
//    preconditioner of the grid problems (Sect. 4.3), the inverse of
//    (Tt + delta Ct + Gt) (x) M^x (x) M^v: the mass matrices replaced by their
//    diagonals, inverted by fixed-degree Chebyshev-Jacobi steps along each
//    axis, or (d = 1) inverted exactly by a tridiagonal solve per grid line.
//  * Right-hand-side helpers of one strip.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace sgdg {

constexpr int kBlock = 256;
constexpr int kPer = kChunk / kBlock;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// block-wide sum, valid in thread 0
__device__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < int(blockDim.x >> 6); ++i) r += sh[i];
  return r;
}

// ------------------------------------------------------------ segments ----
constexpr int kDotWaves = kBlock / 64;
constexpr int kDotMaxVec = 72;

// partial[(chunk0 + chunk) * nvec + k] = sum over the block's chunk of V_k * wl
// (wl: the thread's kPer elements of w, 0 past the segment): wave sums per
// vector in LDS, one barrier, then thread k adds the waves of vector k
template <class T>
__device__ __forceinline__ void chunk_dots(const SegInfo& S, const BlockRef& br, const T* __restrict__ V,
                                           int64_t vstride, int nvec, const double (&wl)[kPer],
                                           double* __restrict__ partial, double (*sh)[kDotMaxVec]) {
  constexpr int kWaves = kDotWaves;
  constexpr int kMaxVec = kDotMaxVec;
  const int64_t beg = S.off + int64_t(br.chunk) * kChunk;
  const int64_t end = S.off + S.len;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double* out = partial + int64_t(S.chunk0 + br.chunk) * nvec;
  for (int k0 = 0; k0 < nvec; k0 += kMaxVec) {
    const int nk = nvec - k0 < kMaxVec ? nvec - k0 : kMaxVec;
    // four vectors at a time: their loads and wave reductions overlap
    int k = 0;
    for (; k + 4 <= nk; k += 4) {
      double acc[4] = {0, 0, 0, 0};
#pragma unroll
      for (int t = 0; t < kPer; ++t) {
        const int64_t i = beg + int64_t(t) * kBlock + threadIdx.x;
        if (i < end) {
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[q] += double(V[int64_t(k0 + k + q) * vstride + i]) * wl[t];
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = wave_sum(acc[q]);
      if (lane == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) sh[wv][k + q] = acc[q];
      }
    }
    for (; k < nk; ++k) {
      const T* vk = V + int64_t(k0 + k) * vstride;
      double acc = 0;
#pragma unroll
      for (int t = 0; t < kPer; ++t) {
        const int64_t i = beg + int64_t(t) * kBlock + threadIdx.x;
        if (i < end) acc += double(vk[i]) * wl[t];
      }
      acc = wave_sum(acc);
      if (lane == 0) sh[wv][k] = acc;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nk; k += kBlock) {
      double a = 0;
#pragma unroll
      for (int q = 0; q < kWaves; ++q) a += sh[q][k];
      out[k0 + k] = a;
    }
    __syncthreads();
  }
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_seg_dots(const SegInfo* __restrict__ segs, const BlockRef* __restrict__ blk,
                                                     const T* __restrict__ V, int64_t vstride, int nvec,
                                                     const T* __restrict__ w, double* __restrict__ partial) {
  __shared__ double sh[kDotWaves][kDotMaxVec];
  const BlockRef br = blk[blockIdx.x];
  const SegInfo& S = segs[br.seg];
  const int64_t beg = S.off + int64_t(br.chunk) * kChunk;
  const int64_t end = S.off + S.len;
  double wl[kPer];
#pragma unroll
  for (int t = 0; t < kPer; ++t) {
    const int64_t i = beg + int64_t(t) * kBlock + threadIdx.x;
    wl[t] = i < end ? double(w[i]) : 0.0;
  }
  chunk_dots<T>(S, br, V, vstride, nvec, wl, partial, sh);
}

// One classical Gram-Schmidt pass followed by the next pass's projections:
// w -= sum_k coef[seg][k] V_k (the arithmetic of k_seg_axpy with sign -1),
// then partial = <V_k, w> as k_seg_dots computes it.  The block's chunk of
// every V_k is read from memory once; the second read comes from the cache.
template <class T>
__global__ void __launch_bounds__(kBlock) k_seg_axpy_dots(const SegInfo* __restrict__ segs,
                                                          const BlockRef* __restrict__ blk, const T* __restrict__ V,
                                                          int64_t vstride, int nvec, const double* __restrict__ coef,
                                                          int cstride, T* __restrict__ w, double* __restrict__ partial) {
  __shared__ double sh[kDotWaves][kDotMaxVec];
  const BlockRef br = blk[blockIdx.x];
  const SegInfo& S = segs[br.seg];
  const int64_t beg = S.off + int64_t(br.chunk) * kChunk;
  const int64_t end = S.off + S.len;
  const double* c = coef + int64_t(br.seg) * cstride;
  const double sign = -1.0;
  double wl[kPer];
#pragma unroll
  for (int t = 0; t < kPer; ++t) {
    const int64_t i = beg + int64_t(t) * kBlock + threadIdx.x;
    wl[t] = 0.0;
    if (i < end) {
      double a = double(w[i]);
      int k = 0;
      for (; k + 4 <= nvec; k += 4) {
        double v4[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) v4[q] = double(V[int64_t(k + q) * vstride + i]);
#pragma unroll
        for (int q = 0; q < 4; ++q) a += sign * c[k + q] * v4[q];
      }
      for (; k < nvec; ++k) a += sign * c[k] * double(V[int64_t(k) * vstride + i]);
      const T r = T(a);
      w[i] = r;
      wl[t] = double(r);
    }
  }
  chunk_dots<T>(S, br, V, vstride, nvec, wl, partial, sh);
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_seg_axpy(const SegInfo* __restrict__ segs, const BlockRef* __restrict__ blk,
                                                     const T* __restrict__ V, int64_t vstride, int nvec,
                                                     const double* __restrict__ coef, int cstride, T* __restrict__ w,
                                                     double sign, double* __restrict__ partial) {
  __shared__ double sh[kBlock / 64];
  const BlockRef br = blk[blockIdx.x];
  const SegInfo& S = segs[br.seg];
  const int64_t beg = S.off + int64_t(br.chunk) * kChunk;
  const int64_t end = S.off + S.len;
  const double* c = coef + int64_t(br.seg) * cstride;
  double nrm = 0;
#pragma unroll
  for (int t = 0; t < kPer; ++t) {
    const int64_t i = beg + int64_t(t) * kBlock + threadIdx.x;
    if (i < end) {
      double a = double(w[i]);
      // four independent loads in flight per step; the sum keeps the order k = 0, 1, ...
      int k = 0;
      for (; k + 4 <= nvec; k += 4) {
        double v4[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) v4[q] = double(V[int64_t(k + q) * vstride + i]);
#pragma unroll
        for (int q = 0; q < 4; ++q) a += sign * c[k + q] * v4[q];
      }
      for (; k < nvec; ++k) a += sign * c[k] * double(V[int64_t(k) * vstride + i]);
      const T r = T(a);
      w[i] = r;
      nrm += double(r) * double(r);
    }
  }
  if (partial) {
    nrm = block_sum(nrm, sh);
    if (threadIdx.x == 0) partial[S.chunk0 + br.chunk] = nrm;
  }
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_seg_scale(const SegInfo* __restrict__ segs, const BlockRef* __restrict__ blk,
                                                      const T* __restrict__ w, const double* __restrict__ scal,
                                                      T* __restrict__ out) {
  const BlockRef br = blk[blockIdx.x];
  const SegInfo& S = segs[br.seg];
  const int64_t beg = S.off + int64_t(br.chunk) * kChunk;
  const int64_t end = S.off + S.len;
  const double sc = scal[br.seg];
#pragma unroll
  for (int t = 0; t < kPer; ++t) {
    const int64_t i = beg + int64_t(t) * kBlock + threadIdx.x;
    if (i < end) out[i] = T(double(w[i]) * sc);
  }
}

template <class T>
__global__ void k_axpby(int64_t n, T a, const T* __restrict__ x, T b, T* __restrict__ y) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i] + b * y[i];
}
template <class T>
__global__ void k_copy(int64_t n, const T* __restrict__ x, T* __restrict__ y) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i];
}
template <class T>
__global__ void k_fill(int64_t n, T v, T* __restrict__ y) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = v;
}
__global__ void k_d2f(int64_t n, const double* __restrict__ x, float* __restrict__ y) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = float(x[i]);
}
__global__ void k_f2d(int64_t n, const float* __restrict__ x, double* __restrict__ y) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = double(x[i]);
}

// ------------------------------------------------------ GMRES bookkeeping --
__device__ __forceinline__ bool finite(double x) { return x == x && x - x == 0.0; }

// Sum of partial[(chunk0 + c) * stride + idx] over the segment's chunks with the
// whole block (fixed order per thread, then a fixed tree): valid in thread 0.
__device__ double seg_chunk_sum(const SegInfo& S, const double* __restrict__ partial, int stride, int idx,
                                double* sh) {
  double a = 0;
  for (int c = threadIdx.x; c < S.nchunk; c += kBlock) a += partial[int64_t(S.chunk0 + c) * stride + idx];
  return block_sum(a, sh);
}

// one block per segment
__global__ void __launch_bounds__(kBlock) k_gmres_start(int nseg, GmresState st, const SegInfo* __restrict__ segs,
                                                        const double* __restrict__ partial, double tol, int first) {
  __shared__ double sh[kBlock / 64];
  const int g = blockIdx.x;
  const int m = st.m;
  const double s = seg_chunk_sum(segs[g], partial, 1, 0, sh);
  for (int i = threadIdx.x; i < (m + 1) * m; i += kBlock) st.H[int64_t(g) * (m + 1) * m + i] = 0.0;
  for (int i = threadIdx.x; i <= m; i += kBlock) st.g[int64_t(g) * (m + 1) + i] = 0.0;
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double beta = sqrt(s);
  if (first) st.bnorm[g] = beta;
  st.beta[g] = beta;
  st.g[int64_t(g) * (m + 1)] = beta;
  const bool act = finite(beta) && beta > 0.0 && beta > tol * st.bnorm[g];
  st.active[g] = act ? 1 : (finite(beta) ? 0 : -1);
  st.kused[g] = 0;
  st.inv[g] = act ? 1.0 / beta : 0.0;
}

// one block per (segment, projection coefficient i): the block's threads
// stride over the segment's chunk partials, then a fixed-order block sum
__global__ void __launch_bounds__(kBlock) k_gmres_proj(int nseg, GmresState st, const SegInfo* __restrict__ segs,
                                                       const double* __restrict__ partial, int j) {
  __shared__ double sh[kBlock / 64];
  const int g = blockIdx.x, i = blockIdx.y;
  const int m = st.m;
  const double a = seg_chunk_sum(segs[g], partial, j + 1, i, sh);
  if (threadIdx.x != 0) return;
  const double t = st.active[g] == 1 ? a : 0.0;
  st.hcol[int64_t(g) * (m + 1) + i] = t;
  st.H[int64_t(g) * (m + 1) * m + int64_t(j) * (m + 1) + i] += t;
}

// one block per segment: the norm of the new direction from the chunk
// partials, then the Givens rotations in thread 0
__global__ void __launch_bounds__(kBlock) k_gmres_givens(int nseg, GmresState st, const SegInfo* __restrict__ segs,
                                                         const double* __restrict__ partial, int j, double tol) {
  __shared__ double sh[kBlock / 64];
  const int g = blockIdx.x;
  const int m = st.m;
  const double s = seg_chunk_sum(segs[g], partial, 1, 0, sh);
  if (threadIdx.x != 0) return;
  if (st.active[g] != 1) {
    st.inv[g] = 0.0;
    return;
  }
  const double hn = sqrt(s);
  double* H = st.H + int64_t(g) * (m + 1) * m + int64_t(j) * (m + 1);
  double* cs = st.cs + int64_t(g) * m;
  double* sn = st.sn + int64_t(g) * m;
  double* gv = st.g + int64_t(g) * (m + 1);
  H[j + 1] = hn;
  for (int i = 0; i < j; ++i) {
    const double t = cs[i] * H[i] + sn[i] * H[i + 1];
    H[i + 1] = -sn[i] * H[i] + cs[i] * H[i + 1];
    H[i] = t;
  }
  const double den = sqrt(H[j] * H[j] + H[j + 1] * H[j + 1]);
  if (!finite(den) || !finite(hn)) {
    st.active[g] = -1;
    st.inv[g] = 0.0;
    return;
  }
  cs[j] = den > 0 ? H[j] / den : 1.0;
  sn[j] = den > 0 ? H[j + 1] / den : 0.0;
  H[j] = den;
  H[j + 1] = 0.0;
  gv[j + 1] = -sn[j] * gv[j];
  gv[j] = cs[j] * gv[j];
  st.kused[g] = j + 1;
  const double res = fabs(gv[j + 1]);
  const bool stop = res <= tol * st.bnorm[g] || hn == 0.0 || den == 0.0;
  st.beta[g] = res;
  st.active[g] = stop ? 0 : 1;
  st.inv[g] = stop ? 0.0 : 1.0 / hn;
}

__global__ void k_gmres_lsq(int nseg, GmresState st) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nseg) return;
  const int m = st.m;
  const int k = st.kused[g];
  const double* H = st.H + int64_t(g) * (m + 1) * m;
  const double* gv = st.g + int64_t(g) * (m + 1);
  double* y = st.y + int64_t(g) * m;
  for (int i = 0; i < m; ++i) y[i] = 0.0;
  for (int i = k - 1; i >= 0; --i) {
    double a = gv[i];
    for (int c = i + 1; c < k; ++c) a -= H[int64_t(c) * (m + 1) + i] * y[c];
    const double d = H[int64_t(i) * (m + 1) + i];
    y[i] = d != 0.0 ? a / d : 0.0;
  }
}

// ---------------------------------------------- combination technique ----
__device__ __forceinline__ void decode(const SegInfo& S, int64_t loc, int& s, int& x, int& v) {
  const int64_t plane = int64_t(S.nx) * S.nv;
  s = int(loc / plane);
  const int64_t rem = loc - int64_t(s) * plane;
  x = int(rem / S.nv);
  v = int(rem - int64_t(x) * S.nv);
}

// CT layout <- residual layout: upper grids copied, lower grids restricted in x
template <class T>
__global__ void __launch_bounds__(kBlock) k_ct_gather(const SegInfo* __restrict__ segs, const BlockRef* __restrict__ blk,
                                                      const T* __restrict__ r, T* __restrict__ b) {
  const BlockRef br = blk[blockIdx.x];
  const SegInfo& S = segs[br.seg];
  for (int t = 0; t < kPer; ++t) {
    const int64_t loc = int64_t(br.chunk) * kChunk + int64_t(t) * kBlock + threadIdx.x;
    if (loc >= S.len) return;
    if (S.kind == 0) {
      b[S.off + loc] = r[S.src_off + loc];
    } else {
      int s, x, v;
      decode(S, loc, s, x, v);
      const T* src = r + S.src_off + int64_t(s) * S.nx_src * S.nv + v;
      const int32_t* c = S.xchi + int64_t(x) * S.Sx;
      const double* cw = S.xchiw + int64_t(x) * S.Sx;
      T acc = 0;
      for (int e = 0; e < S.Sx; ++e) acc += T(cw[e]) * src[int64_t(c[e]) * S.nv];
      b[S.off + loc] = acc;
    }
  }
}

// residual layout <- combination of the CT solution: dU_up - (E^x (x) I) dU_low
template <class T>
__global__ void __launch_bounds__(kBlock) k_ct_combine(const SegInfo* __restrict__ segs, const BlockRef* __restrict__ blk,
                                                       const T* __restrict__ ct, T* __restrict__ z) {
  const BlockRef br = blk[blockIdx.x];
  const SegInfo& S = segs[br.seg];
  if (S.kind != 0) return;
  for (int t = 0; t < kPer; ++t) {
    const int64_t loc = int64_t(br.chunk) * kChunk + int64_t(t) * kBlock + threadIdx.x;
    if (loc >= S.len) return;
    T val = ct[S.off + loc];
    if (S.low_off >= 0) {
      int s, x, v;
      decode(S, loc, s, x, v);
      const T* src = ct + S.low_off + int64_t(s) * S.nx_src * S.nv + v;
      const int32_t* p = S.xpar + 2 * int64_t(x);
      const double* pw = S.xparw + 2 * int64_t(x);
      val -= T(pw[0]) * src[int64_t(p[0]) * S.nv] + T(pw[1]) * src[int64_t(p[1]) * S.nv];
    }
    z[S.src_off + loc] = val;
  }
}

// y = (Pinv (x) diag(M^x)^-1 (x) diag(M^v)^-1) x on every grid segment
template <class T>
__global__ void __launch_bounds__(kBlock) k_minv(const SegInfo* __restrict__ segs, const BlockRef* __restrict__ blk,
                                                 const T* __restrict__ x, T* __restrict__ y) {
  const BlockRef br = blk[blockIdx.x];
  const SegInfo& S = segs[br.seg];
  const int64_t plane = int64_t(S.nx) * S.nv;
  for (int t = 0; t < kPer; ++t) {
    const int64_t p = int64_t(br.chunk) * kChunk + int64_t(t) * kBlock + threadIdx.x;
    if (p >= plane) return;
    const int xi = int(p / S.nv), vi = int(p - int64_t(p / S.nv) * S.nv);
    const T sc = T(1.0 / (S.mxd[int64_t(xi) * S.Sx] * S.mvd[int64_t(vi) * S.Sv]));
    T in[kMaxR];
    for (int s = 0; s < S.R; ++s) in[s] = x[S.off + s * plane + p];
    for (int s = 0; s < S.R; ++s) {
      T a = 0;
      for (int s2 = 0; s2 < S.R; ++s2) a += T(S.pinv[s * S.R + s2]) * in[s2];
      y[S.off + s * plane + p] = a * sc;
    }
  }
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_tinv(const SegInfo* __restrict__ segs, const BlockRef* __restrict__ blk,
                                                 const T* __restrict__ x, T* __restrict__ y) {
  const BlockRef br = blk[blockIdx.x];
  const SegInfo& S = segs[br.seg];
  const int64_t plane = int64_t(S.nx) * S.nv;
  for (int t = 0; t < kPer; ++t) {
    const int64_t p = int64_t(br.chunk) * kChunk + int64_t(t) * kBlock + threadIdx.x;
    if (p >= plane) return;
    T in[kMaxR];
    for (int s = 0; s < S.R; ++s) in[s] = x[S.off + s * plane + p];
    for (int s = 0; s < S.R; ++s) {
      T a = 0;
      for (int s2 = 0; s2 < S.R; ++s2) a += T(S.pinv[s * S.R + s2]) * in[s2];
      y[S.off + s * plane + p] = a;
    }
  }
}

// One step of the Chebyshev semi-iteration for M z = b with the Jacobi
// splitting D = diag(M), along one axis of a segment's [R][nx][nv] block (the
// mass matrix of that axis acts on every line of the other axis and every
// slice).  The diagonal is the true one: the sum of the stencil slots that
// land on the row's own node (periodic lattices of 1 or 2 nodes wrap onto it).
template <class T>
__global__ void __launch_bounds__(kBlock) k_mass_cheb(const SegInfo* __restrict__ segs,
                                                      const BlockRef* __restrict__ blk, int axis, double cd,
                                                      double cr, int first, int tinv, const T* __restrict__ b,
                                                      const T* __restrict__ x, const T* __restrict__ d,
                                                      T* __restrict__ x_out, T* __restrict__ d_out) {
  const BlockRef br = blk[blockIdx.x];
  const SegInfo& S = segs[br.seg];
  const int64_t plane = int64_t(S.nx) * S.nv;
  const int Sn = axis == 0 ? S.Sx : S.Sv;
  const double* rows = axis == 0 ? S.mxd : S.mvd;
  const int32_t* nbr = axis == 0 ? S.xnbr : S.vnbr;
  for (int t = 0; t < kPer; ++t) {
    const int64_t p = int64_t(br.chunk) * kChunk + int64_t(t) * kBlock + threadIdx.x;
    if (p >= plane) return;
    const int xi = int(p / S.nv), vi = int(p - int64_t(xi) * S.nv);
    const int row = axis == 0 ? xi : vi;
    double diag = 0;
    for (int e = 0; e < Sn; ++e)
      if (nbr[int64_t(row) * Sn + e] == row) diag += rows[int64_t(row) * Sn + e];
    const double rdiag = 1.0 / diag;
    T xn[kMaxR];
    for (int s = 0; s < S.R; ++s) {
      const int64_t base = S.off + s * plane;
      const int64_t i = base + p;
      double res = double(b[i]);
      double dn;
      if (first) {
        dn = cr * rdiag * res;
        xn[s] = T(dn);
      } else {
        for (int e = 0; e < Sn; ++e) {
          const int64_t c = nbr[int64_t(row) * Sn + e];
          const int64_t q = axis == 0 ? c * S.nv + vi : int64_t(xi) * S.nv + c;
          res -= rows[int64_t(row) * Sn + e] * double(x[base + q]);
        }
        dn = cd * double(d[i]) + cr * rdiag * res;
        xn[s] = T(double(x[i]) + dn);
      }
      if (d_out) d_out[i] = T(dn);
    }
    for (int s = 0; s < S.R; ++s) {
      T a = xn[s];
      if (tinv) {
        a = 0;
        for (int s2 = 0; s2 < S.R; ++s2) a += T(S.pinv[s * S.R + s2]) * xn[s2];
      }
      x_out[S.off + s * plane + p] = a;
    }
  }
}

// Exact solve of the 1D mass matrix along one axis, one thread per line of a
// segment.  A line of n nodes carries the tridiagonal rows (lo_i, di_i, up_i)
// of the stencil (offsets -1, 0, +1).  A periodic line of n >= 3 nodes is
// cyclic: its corner entries are split off as a rank-one term u v^T and the
// Sherman-Morrison formula combines two tridiagonal solves (right-hand side
// and u); a periodic line of 2 nodes couples both slots to the other node, one
// of 1 node to itself.
template <class T>
__global__ void __launch_bounds__(kBlock) k_mass_thomas(const SegInfo* __restrict__ segs, int axis,
                                                        const T* __restrict__ b, T* __restrict__ y,
                                                        T* __restrict__ cbuf, T* __restrict__ zbuf) {
  const SegInfo& S = segs[blockIdx.y];
  const int64_t line = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const int n = axis == 0 ? S.nx : S.nv;
  const int other = axis == 0 ? S.nv : S.nx;
  if (line >= int64_t(S.R) * other) return;
  const int s = int(line / other), k = int(line - int64_t(s) * other);
  const int64_t plane = int64_t(S.nx) * S.nv;
  const int64_t base = S.off + s * plane + (axis == 0 ? k : int64_t(k) * S.nv);
  const int64_t stride = axis == 0 ? S.nv : 1;
  const int Sn = axis == 0 ? S.Sx : S.Sv;
  const double* rows = axis == 0 ? S.mxd : S.mvd;
  const int32_t* nbr = axis == 0 ? S.xnbr : S.vnbr;
  const bool per = (axis == 0 ? S.xper : S.vper) != 0;
  auto coef = [&](int i, double& lo, double& di, double& up) {
    lo = di = up = 0;
    for (int e = 0; e < Sn; ++e) {
      const int c = nbr[int64_t(i) * Sn + e];
      const double v = rows[int64_t(i) * Sn + e];
      if (c == i) di += v;
      else if (e == S.sm) lo += v;
      else if (e == S.sp) up += v;
    }
  };
  if (n == 1 || (per && n == 2)) {  // every slot lands on the line's own nodes: a dense 1x1 or 2x2 solve
    double l0, d0, u0;
    coef(0, l0, d0, u0);
    if (n == 1) {
      y[base] = T(double(b[base]) / d0);
      return;
    }
    double l1, d1, u1;
    coef(1, l1, d1, u1);
    const double a01 = l0 + u0, a10 = l1 + u1, det = d0 * d1 - a01 * a10;
    const double b0 = double(b[base]), b1 = double(b[base + stride]);
    y[base] = T((d1 * b0 - a01 * b1) / det);
    y[base + stride] = T((d0 * b1 - a10 * b0) / det);
    return;
  }
  // A = T' + u v^T with u = (g, 0.., 0, alpha), v = (1, 0.., 0, beta / g) for a cyclic line
  double lo0, di0, up0;
  coef(0, lo0, di0, up0);
  double loN, diN, upN;
  coef(n - 1, loN, diN, upN);
  const double beta = per ? lo0 : 0.0;   // row 0, column n-1
  const double alpha = per ? upN : 0.0;  // row n-1, column 0
  const double g = -di0;
  // forward elimination of T' y = b and T' z = u (c' kept in cbuf, z's in zbuf)
  double cprev = 0, dprev = 0, zprev = 0;
  for (int i = 0; i < n; ++i) {
    double lo, di, up;
    coef(i, lo, di, up);
    if (i == 0) lo = 0;
    if (i == n - 1) up = 0;
    if (per && i == 0) di -= g;
    if (per && i == n - 1) di -= alpha * beta / g;
    const double den = di - lo * cprev;
    const double c = up / den;
    const double dd = (double(b[base + i * stride]) - lo * dprev) / den;
    const double ui = per ? (i == 0 ? g : (i == n - 1 ? alpha : 0.0)) : 0.0;
    const double zz = (ui - lo * zprev) / den;
    cbuf[base + i * stride] = T(c);
    y[base + i * stride] = T(dd);
    if (per) zbuf[base + i * stride] = T(zz);
    cprev = c;
    dprev = dd;
    zprev = zz;
  }
  // back substitution
  double ynext = 0, znext = 0;
  for (int i = n - 1; i >= 0; --i) {
    const double c = double(cbuf[base + i * stride]);
    const double yi = double(y[base + i * stride]) - c * ynext;
    y[base + i * stride] = T(yi);
    ynext = yi;
    if (per) {
      const double zi = double(zbuf[base + i * stride]) - c * znext;
      zbuf[base + i * stride] = T(zi);
      znext = zi;
    }
  }
  if (!per) return;
  const double y0 = double(y[base]), yN = double(y[base + (n - 1) * stride]);
  const double z0 = double(zbuf[base]), zN = double(zbuf[base + (n - 1) * stride]);
  const double f = (y0 + beta / g * yN) / (1.0 + z0 + beta / g * zN);
  for (int i = 0; i < n; ++i) y[base + i * stride] = T(double(y[base + i * stride]) - f * double(zbuf[base + i * stride]));
}

// ------------------------------------------------------------- data / rhs --
__global__ void k_project(int64_t n, int nq, int R, const double* __restrict__ wts, const double* __restrict__ samples,
                          double* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int s = 0; s < R; ++s) {
    double a = 0;
    for (int q = 0; q < nq; ++q) a += wts[s * nq + q] * samples[int64_t(q) * n + i];
    out[int64_t(s) * n + i] = a;
  }
}

// trace of a previous solution with Rprev slices: out[poff + p] = sum_s u[Rprev poff + s plane + p]
__global__ void k_trace(const SegInfo* __restrict__ segs, const BlockRef* __restrict__ blk, int Rprev,
                        const double* __restrict__ u, double* __restrict__ out) {
  const BlockRef br = blk[blockIdx.x];
  const SegInfo& S = segs[br.seg];
  const int64_t plane = int64_t(S.nx) * S.nv;
  for (int t = 0; t < kPer; ++t) {
    const int64_t p = int64_t(br.chunk) * kChunk + int64_t(t) * kBlock + threadIdx.x;
    if (p >= plane) return;
    double a = 0;
    for (int s = 0; s < Rprev; ++s) a += u[S.src_off * Rprev + s * plane + p];
    out[S.src_off + p] = a;
  }
}

// b[off + s plane + p] = (-1)^s m[poff + p]
__global__ void k_spread(const SegInfo* __restrict__ segs, const BlockRef* __restrict__ blk,
                         const double* __restrict__ m, double* __restrict__ b) {
  const BlockRef br = blk[blockIdx.x];
  const SegInfo& S = segs[br.seg];
  const int64_t plane = int64_t(S.nx) * S.nv;
  for (int t = 0; t < kPer; ++t) {
    const int64_t p = int64_t(br.chunk) * kChunk + int64_t(t) * kBlock + threadIdx.x;
    if (p >= plane) return;
    const double val = m[S.src_off + p];
    for (int s = 0; s < S.R; ++s) b[S.off + s * plane + p] = (s & 1) ? -val : val;
  }
}

// ================================================================ launchers =
static inline unsigned nblk(int64_t n) { return unsigned((n + kBlock - 1) / kBlock); }
#define LAUNCH_CHECK() SGDG_CHECK_HIP(hipGetLastError())

template <class T>
void KernelsT<T>::seg_dots(const SegTable& S, const T* V, int64_t vstride, int nvec, const T* w, double* partial,
                           hipStream_t s) {
  if (S.nblk == 0) return;
  hipLaunchKernelGGL(k_seg_dots<T>, dim3(S.nblk), dim3(kBlock), 0, s, S.segs, S.blk, V, vstride, nvec, w, partial);
  LAUNCH_CHECK();
}
template <class T>
void KernelsT<T>::seg_axpy(const SegTable& S, const T* V, int64_t vstride, int nvec, const double* coef, int cstride,
                           T* w, double sign, double* partial_norm, hipStream_t s) {
  if (S.nblk == 0) return;
  hipLaunchKernelGGL(k_seg_axpy<T>, dim3(S.nblk), dim3(kBlock), 0, s, S.segs, S.blk, V, vstride, nvec, coef, cstride,
                     w, sign, partial_norm);
  LAUNCH_CHECK();
}
template <class T>
void KernelsT<T>::seg_axpy_dots(const SegTable& S, const T* V, int64_t vstride, int nvec, const double* coef,
                                int cstride, T* w, double* partial, hipStream_t s) {
  if (S.nblk == 0) return;
  hipLaunchKernelGGL(k_seg_axpy_dots<T>, dim3(S.nblk), dim3(kBlock), 0, s, S.segs, S.blk, V, vstride, nvec, coef,
                     cstride, w, partial);
  LAUNCH_CHECK();
}
template <class T>
void KernelsT<T>::seg_scale(const SegTable& S, const T* w, const double* scal, T* out, hipStream_t s) {
  if (S.nblk == 0) return;
  hipLaunchKernelGGL(k_seg_scale<T>, dim3(S.nblk), dim3(kBlock), 0, s, S.segs, S.blk, w, scal, out);
  LAUNCH_CHECK();
}
template <class T>
void KernelsT<T>::seg_norm2(const SegTable& S, const T* w, double* partial, hipStream_t s) {
  seg_dots(S, w, 0, 1, w, partial, s);
}
template <class T>
void KernelsT<T>::ct_gather(const SegTable& S, const T* r, T* b, hipStream_t s) {
  if (S.nblk == 0) return;
  hipLaunchKernelGGL(k_ct_gather<T>, dim3(S.nblk), dim3(kBlock), 0, s, S.segs, S.blk, r, b);
  LAUNCH_CHECK();
}
template <class T>
void KernelsT<T>::ct_combine(const SegTable& S, const T* ct, T* z, hipStream_t s) {
  if (S.nblk == 0) return;
  hipLaunchKernelGGL(k_ct_combine<T>, dim3(S.nblk), dim3(kBlock), 0, s, S.segs, S.blk, ct, z);
  LAUNCH_CHECK();
}
template <class T>
void KernelsT<T>::minv(const SegTable& S, const T* x, T* y, hipStream_t s) {
  if (S.nblk == 0) return;
  hipLaunchKernelGGL(k_minv<T>, dim3(S.nblk), dim3(kBlock), 0, s, S.segs, S.blk, x, y);
  LAUNCH_CHECK();
}
template <class T>
void KernelsT<T>::tinv(const SegTable& S, const T* x, T* y, hipStream_t s) {
  if (S.nblk == 0) return;
  hipLaunchKernelGGL(k_tinv<T>, dim3(S.nblk), dim3(kBlock), 0, s, S.segs, S.blk, x, y);
  LAUNCH_CHECK();
}
template <class T>
void KernelsT<T>::mass_cheb(const SegTable& S, int axis, double cd, double cr, int first, int tinv, const T* b,
                            const T* x, const T* d, T* x_out, T* d_out, hipStream_t s) {
  if (S.nblk == 0) return;
  hipLaunchKernelGGL(k_mass_cheb<T>, dim3(S.nblk), dim3(kBlock), 0, s, S.segs, S.blk, axis, cd, cr, first, tinv, b,
                     x, d, x_out, d_out);
  LAUNCH_CHECK();
}
template <class T>
void KernelsT<T>::mass_thomas(const SegTable& S, int axis, int max_lines, const T* b, T* y, T* cbuf, T* zbuf,
                              hipStream_t s) {
  if (S.nseg == 0 || max_lines <= 0) return;
  hipLaunchKernelGGL(k_mass_thomas<T>, dim3(unsigned((max_lines + kBlock - 1) / kBlock), unsigned(S.nseg)),
                     dim3(kBlock), 0, s, S.segs, axis, b, y, cbuf, zbuf);
  LAUNCH_CHECK();
}
template <class T>
void KernelsT<T>::axpby(int64_t n, T a, const T* x, T b, T* y, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_axpby<T>, dim3(nblk(n)), dim3(kBlock), 0, s, n, a, x, b, y);
  LAUNCH_CHECK();
}
template <class T>
void KernelsT<T>::copy(int64_t n, const T* x, T* y, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_copy<T>, dim3(nblk(n)), dim3(kBlock), 0, s, n, x, y);
  LAUNCH_CHECK();
}
template <class T>
void KernelsT<T>::fill(int64_t n, T v, T* y, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_fill<T>, dim3(nblk(n)), dim3(kBlock), 0, s, n, v, y);
  LAUNCH_CHECK();
}

template struct KernelsT<double>;
template struct KernelsT<float>;

void convert_f64_to_f32(int64_t n, const double* x, float* y, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_d2f, dim3(nblk(n)), dim3(kBlock), 0, s, n, x, y);
  LAUNCH_CHECK();
}
void convert_f32_to_f64(int64_t n, const float* x, double* y, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_f2d, dim3(nblk(n)), dim3(kBlock), 0, s, n, x, y);
  LAUNCH_CHECK();
}
void gmres_start(int nseg, const GmresState& st, const SegInfo* segs, const double* partial, double tol, int first,
                 hipStream_t s) {
  if (nseg == 0) return;
  hipLaunchKernelGGL(k_gmres_start, dim3(nseg), dim3(kBlock), 0, s, nseg, st, segs, partial, tol, first);
  LAUNCH_CHECK();
}
void gmres_add_proj(int nseg, const GmresState& st, const SegInfo* segs, const double* partial, int j, hipStream_t s) {
  if (nseg == 0) return;
  hipLaunchKernelGGL(k_gmres_proj, dim3(nseg, j + 1), dim3(kBlock), 0, s, nseg, st, segs, partial, j);
  LAUNCH_CHECK();
}
void gmres_givens(int nseg, const GmresState& st, const SegInfo* segs, const double* partial, int j, double tol,
                  hipStream_t s) {
  if (nseg == 0) return;
  hipLaunchKernelGGL(k_gmres_givens, dim3(nseg), dim3(kBlock), 0, s, nseg, st, segs, partial, j, tol);
  LAUNCH_CHECK();
}
void gmres_lsq(int nseg, const GmresState& st, hipStream_t s) {
  hipLaunchKernelGGL(k_gmres_lsq, dim3(nblk(nseg)), dim3(kBlock), 0, s, nseg, st);
  LAUNCH_CHECK();
}
void project_time(int64_t n, int nq, int R, const double* wts, const double* samples, double* out, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_project, dim3(nblk(n)), dim3(kBlock), 0, s, n, nq, R, wts, samples, out);
  LAUNCH_CHECK();
}
void trace_sum(const SegTable& S, int Rprev, const double* u, double* out, hipStream_t s) {
  if (S.nblk == 0) return;
  hipLaunchKernelGGL(k_trace, dim3(S.nblk), dim3(kBlock), 0, s, S.segs, S.blk, Rprev, u, out);
  LAUNCH_CHECK();
}
void spread_left(const SegTable& S, const double* m, double* b, hipStream_t s) {
  if (S.nblk == 0) return;
  hipLaunchKernelGGL(k_spread, dim3(S.nblk), dim3(kBlock), 0, s, S.segs, S.blk, m, b);
  LAUNCH_CHECK();
}

}  // namespace sgdg
