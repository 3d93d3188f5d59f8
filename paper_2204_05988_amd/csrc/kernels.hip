// Device kernels of libsgdg for gfx950 (wave64).
//
// Operator application (Sect. 4.2).  A block of the strip matrix is
//   A_{l,l'} = sum_k Tm_k (x) X_k(lx,lx') (x) V_k(lv,lv').
// On the upper diagonal lx + lv is constant, so lx' < lx implies lv' > lv and
//   X_k(lx,lx') = X_k(lx) E^x_{lx<-lx'},   V_k(lv,lv') = E^v_{lv'<-lv}^T V_k(lv')
// (both from X_{l,l'} = E_{L,l}^T X_L E_{L,l'}).  The sum over all lower
// partners l' of grid i is therefore a prefix scan along the chain of grids,
//   Z_i = W_i + (E^x (x) E^vT) Z_{i-1},     W_i = (I (x) V) u_i,
// one array per distinct v-factor V, after which y_i = sum_k Tm_k (X_k (x) I) Z_i.
// The upper partners give the mirror scan over distinct x-factors X,
//   Q_i = (E^xT (x) E^v)(Q_{i+1} + (X (x) I) u_{i+1}),  y_i += sum_k Tm_k (I (x) V_k) Q_i.
// Each step reads a grid once per stencil entry and is streamed from HBM;
// factor values are per-level [n][S] tables shared by all rows (L2 resident).
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace sgdg {

constexpr int kBlock = 256;
constexpr int kChunk = 4096;  // elements per block in segment reductions

template <class T> __device__ __forceinline__ const T* fvals(const DevDomain& D);
template <> __device__ __forceinline__ const double* fvals<double>(const DevDomain& D) { return D.vals; }
template <> __device__ __forceinline__ const float* fvals<float>(const DevDomain& D) { return D.vals32; }
template <class T> __device__ __forceinline__ const T* tmats(const DevOp& op);
template <> __device__ __forceinline__ const double* tmats<double>(const DevOp& op) { return op.term_tm; }
template <> __device__ __forceinline__ const float* tmats<float>(const DevOp& op) { return op.term_tm32; }

__device__ __forceinline__ int locate(const DevGrids& G, int64_t idx) {
  int g = 0;
  while (g + 1 < G.n && idx >= G.off[g + 1]) ++g;
  return g;
}

// ---------------------------------------------------------------- sweeps --
template <class T>
__global__ void __launch_bounds__(kBlock) k_sweeps(DevGrids G, DevDomain DX, DevDomain DV, DevOp op,
                                                   const T* __restrict__ u, T* __restrict__ W,
                                                   T* __restrict__ Rr, int B) {
  const int64_t total = G.off[G.n];
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (idx >= total) return;
  const int g = locate(G, idx);
  const int nx = G.nx[g], nv = G.nv[g];
  const int64_t loc = idx - G.off[g];
  const int64_t plane = int64_t(nx) * nv;
  const int s = int(loc / plane);
  const int64_t rem = loc - int64_t(s) * plane;
  const int x = int(rem / nv), v = int(rem - int64_t(x) * nv);
  const T* ub = u + int64_t(b) * total + G.off[g] + int64_t(s) * plane;
  {
    const int Sv = DV.S;
    const int64_t lo = DV.lev_off[G.lv[g] - DV.lmin] + int64_t(v) * Sv;
    const int32_t* nb = DV.nbr + lo;
    T un[kMaxS];
#pragma unroll
    for (int e = 0; e < kMaxS; ++e) un[e] = e < Sv ? ub[int64_t(x) * nv + nb[e]] : T(0);
    const T* vals = fvals<T>(DV);
    for (int j = 0; j < op.nvg; ++j) {
      const T* fv = vals + int64_t(op.vg_fac[j]) * DV.fac_stride + lo;
      T acc = 0;
#pragma unroll
      for (int e = 0; e < kMaxS; ++e)
        if (e < Sv) acc += fv[e] * un[e];
      W[(int64_t(j) * B + b) * total + idx] = acc;
    }
  }
  if (Rr) {
    const int Sx = DX.S;
    const int64_t lo = DX.lev_off[G.lx[g] - DX.lmin] + int64_t(x) * Sx;
    const int32_t* nb = DX.nbr + lo;
    T un[kMaxS];
#pragma unroll
    for (int e = 0; e < kMaxS; ++e) un[e] = e < Sx ? ub[int64_t(nb[e]) * nv + v] : T(0);
    const T* vals = fvals<T>(DX);
    for (int m = 0; m < op.nxg; ++m) {
      const T* fx = vals + int64_t(op.xg_fac[m]) * DX.fac_stride + lo;
      T acc = 0;
#pragma unroll
      for (int e = 0; e < kMaxS; ++e)
        if (e < Sx) acc += fx[e] * un[e];
      Rr[(int64_t(m) * B + b) * total + idx] = acc;
    }
  }
}

// One step of both scans.  blockIdx.z = 0: lower scan into grid `step`;
// blockIdx.z = 1: upper scan into grid n-1-step.  blockIdx.y = group*B + b.
template <class T>
__global__ void __launch_bounds__(kBlock) k_scan(DevGrids G, DevDomain DX, DevDomain DV, int ngroups_lo,
                                                 int ngroups_up, T* __restrict__ Z, T* __restrict__ Q,
                                                 const T* __restrict__ Rr, int step, int B) {
  const int64_t total = G.off[G.n];
  const bool lower = blockIdx.z == 0;
  const int gb = blockIdx.y;
  if (lower && gb >= ngroups_lo * B) return;
  if (!lower && gb >= ngroups_up * B) return;
  const int i = lower ? step : G.n - 1 - step;
  const int src = lower ? i - 1 : i + 1;
  const int nx = G.nx[i], nv = G.nv[i];
  const int64_t plane = int64_t(nx) * nv;
  const int64_t loc = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (loc >= int64_t(G.R) * plane) return;
  const int s = int(loc / plane);
  const int64_t rem = loc - int64_t(s) * plane;
  const int x = int(rem / nv), v = int(rem - int64_t(x) * nv);
  const int nvs = G.nv[src];
  const int64_t splane = int64_t(G.nx[src]) * nvs;
  if (lower) {
    // out(lx, lv) += sum_parents(x) w sum_children(v) w Z(lx-1, lv+1)
    const T* in = Z + int64_t(gb) * total + G.off[src] + int64_t(s) * splane;
    const int64_t po = DX.par_off[G.lx[i] - DX.lmin] + 2 * int64_t(x);
    const int Sv = DV.S;
    const int64_t co = DV.lev_off[G.lv[i] - DV.lmin] + int64_t(v) * Sv;
    T acc = 0;
    for (int k = 0; k < 2; ++k) {
      const double wx = DX.parw[po + k];
      if (wx == 0.0) continue;
      const T* row = in + int64_t(DX.par[po + k]) * nvs;
      T a = 0;
      for (int e = 0; e < Sv; ++e) a += T(DV.chiw[co + e]) * row[DV.chi[co + e]];
      acc += T(wx) * a;
    }
    Z[int64_t(gb) * total + G.off[i] + loc] += acc;
  } else {
    // out(lx, lv) = sum_children(x) w sum_parents(v) w (Q + Rr)(lx+1, lv-1)
    // the last grid has no upper partners: its Q is zero and never stored
    const bool top = src == G.n - 1;
    const T* q = Q + int64_t(gb) * total + G.off[src] + int64_t(s) * splane;
    const T* r = Rr + int64_t(gb) * total + G.off[src] + int64_t(s) * splane;
    const int Sx = DX.S;
    const int64_t co = DX.lev_off[G.lx[i] - DX.lmin] + int64_t(x) * Sx;
    const int64_t po = DV.par_off[G.lv[i] - DV.lmin] + 2 * int64_t(v);
    const int32_t p0 = DV.par[po], p1 = DV.par[po + 1];
    const T w0 = T(DV.parw[po]), w1 = T(DV.parw[po + 1]);
    T acc = 0;
    for (int e = 0; e < Sx; ++e) {
      const double wx = DX.chiw[co + e];
      if (wx == 0.0) continue;
      const int64_t rowo = int64_t(DX.chi[co + e]) * nvs;
      T a0 = r[rowo + p0], a1 = r[rowo + p1];
      if (!top) {
        a0 += q[rowo + p0];
        a1 += q[rowo + p1];
      }
      acc += T(wx) * (w0 * a0 + w1 * a1);
    }
    Q[int64_t(gb) * total + G.off[i] + loc] = acc;
  }
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_final(DevGrids G, GridPts P, DevDomain DX, DevDomain DV, DevOp op,
                                                  const T* __restrict__ Z, const T* __restrict__ Q,
                                                  T* __restrict__ y, int B) {
  const int64_t npts = P.poff[G.n];
  const int64_t pidx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (pidx >= npts) return;
  int g = 0;
  while (g + 1 < G.n && pidx >= P.poff[g + 1]) ++g;
  const int nx = G.nx[g], nv = G.nv[g];
  const int64_t p = pidx - P.poff[g];
  const int x = int(p / nv), v = int(p - int64_t(x) * nv);
  const int64_t plane = int64_t(nx) * nv;
  const int64_t total = G.off[G.n];
  const int Rin = op.Rin, Rout = op.Rout;
  T acc[kMaxR];
#pragma unroll
  for (int s = 0; s < kMaxR; ++s) acc[s] = 0;
  const T* tm = tmats<T>(op);
  {
    const int Sx = DX.S;
    const int64_t lo = DX.lev_off[G.lx[g] - DX.lmin] + int64_t(x) * Sx;
    int32_t nb[kMaxS];
#pragma unroll
    for (int e = 0; e < kMaxS; ++e) nb[e] = e < Sx ? DX.nbr[lo + e] : 0;
    const T* vals = fvals<T>(DX);
    for (int k = 0; k < op.nterms; ++k) {
      const T* fx = vals + int64_t(op.term_xf[k]) * DX.fac_stride + lo;
      const T* zb = Z + (int64_t(op.term_vg[k]) * B + b) * total + G.off[g] + v;
      for (int s2 = 0; s2 < Rin; ++s2) {
        T t = 0;
#pragma unroll
        for (int e = 0; e < kMaxS; ++e)
          if (e < Sx) t += fx[e] * zb[int64_t(s2) * plane + int64_t(nb[e]) * nv];
        for (int s = 0; s < Rout; ++s) acc[s] += tm[(int64_t(k) * Rout + s) * Rin + s2] * t;
      }
    }
  }
  if (Q && g + 1 < G.n) {  // the last grid has no upper partners
    const int Sv = DV.S;
    const int64_t lo = DV.lev_off[G.lv[g] - DV.lmin] + int64_t(v) * Sv;
    int32_t nb[kMaxS];
#pragma unroll
    for (int e = 0; e < kMaxS; ++e) nb[e] = e < Sv ? DV.nbr[lo + e] : 0;
    const T* vals = fvals<T>(DV);
    for (int k = 0; k < op.nterms; ++k) {
      const T* fv = vals + int64_t(op.term_vf[k]) * DV.fac_stride + lo;
      const T* qb = Q + (int64_t(op.term_xg[k]) * B + b) * total + G.off[g] + int64_t(x) * nv;
      for (int s2 = 0; s2 < Rin; ++s2) {
        T t = 0;
#pragma unroll
        for (int e = 0; e < kMaxS; ++e)
          if (e < Sv) t += fv[e] * qb[int64_t(s2) * plane + nb[e]];
        for (int s = 0; s < Rout; ++s) acc[s] += tm[(int64_t(k) * Rout + s) * Rin + s2] * t;
      }
    }
  }
  T* yb = y + int64_t(b) * (int64_t(Rout) * npts) + int64_t(Rout) * P.poff[g] + p;
  for (int s = 0; s < Rout; ++s) yb[int64_t(s) * plane] = acc[s];
}

// ------------------------------------------------------------- transfers --
// lower grid g (lx, lv) <- upper grid g+1 (lx+1, lv)
template <class T>
__global__ void k_restrict_x(DevGrids Go, DevGrids Gi, DevDomain DX, const T* __restrict__ in, T* __restrict__ out) {
  const int64_t total = Go.off[Go.n];
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int g = locate(Go, idx);
  const int gi = g + 1;
  const int nx = Go.nx[g], nv = Go.nv[g];
  const int64_t loc = idx - Go.off[g];
  const int64_t plane = int64_t(nx) * nv;
  const int s = int(loc / plane);
  const int64_t rem = loc - int64_t(s) * plane;
  const int x = int(rem / nv), v = int(rem - int64_t(x) * nv);
  const int S = DX.S;
  const int64_t co = DX.lev_off[Go.lx[g] - DX.lmin] + int64_t(x) * S;
  const T* src = in + Gi.off[gi] + int64_t(s) * int64_t(Gi.nx[gi]) * nv;
  T acc = 0;
  for (int e = 0; e < S; ++e) acc += T(DX.chiw[co + e]) * src[int64_t(DX.chi[co + e]) * nv + v];
  out[idx] = acc;
}

template <class T>
__global__ void k_combine(DevGrids Gu, DevGrids Gl, int lmin, DevDomain DX, const T* __restrict__ up,
                          const T* __restrict__ low, T* __restrict__ out) {
  const int64_t total = Gu.off[Gu.n];
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int g = locate(Gu, idx);
  T val = up[idx];
  if (Gu.lx[g] > lmin) {
    const int gl = g - 1;  // lower grid (lx-1, lv) has index g-1 on the lower diagonal
    const int nx = Gu.nx[g], nv = Gu.nv[g];
    const int64_t loc = idx - Gu.off[g];
    const int64_t plane = int64_t(nx) * nv;
    const int s = int(loc / plane);
    const int64_t rem = loc - int64_t(s) * plane;
    const int x = int(rem / nv), v = int(rem - int64_t(x) * nv);
    const int64_t po = DX.par_off[Gu.lx[g] - DX.lmin] + 2 * int64_t(x);
    const T* src = low + Gl.off[gl] + int64_t(s) * int64_t(Gl.nx[gl]) * nv;
    val -= T(DX.parw[po]) * src[int64_t(DX.par[po]) * nv + v] + T(DX.parw[po + 1]) * src[int64_t(DX.par[po + 1]) * nv + v];
  }
  out[idx] = val;
}

// Jacobi approximation of (Pinv (x) Mx^-1 (x) Mv^-1): y[s] = sum_s' Pinv[s][s'] x[s'] / (Dx Dv)
template <class T>
__global__ void k_minv_jacobi(DevGrids G, GridPts P, DevDomain DX, DevDomain DV, const double* __restrict__ pinv,
                              const T* __restrict__ x, T* __restrict__ y) {
  const int64_t npts = P.poff[G.n];
  const int64_t pidx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (pidx >= npts) return;
  int g = 0;
  while (g + 1 < G.n && pidx >= P.poff[g + 1]) ++g;
  const int nx = G.nx[g], nv = G.nv[g];
  const int64_t p = pidx - P.poff[g];
  const int xi = int(p / nv), vi = int(p - int64_t(xi) * nv);
  const int64_t plane = int64_t(nx) * nv;
  const int R = G.R;
  const T dx = T(fvals<T>(DX)[int64_t(DX.mass_fac) * DX.fac_stride + DX.lev_off[G.lx[g] - DX.lmin] + int64_t(xi) * DX.S]);
  const T dv = T(fvals<T>(DV)[int64_t(DV.mass_fac) * DV.fac_stride + DV.lev_off[G.lv[g] - DV.lmin] + int64_t(vi) * DV.S]);
  const T sc = T(1) / (dx * dv);
  const int64_t base = G.off[g] + p;
  T in[kMaxR];
  for (int s = 0; s < R; ++s) in[s] = x[base + s * plane];
  for (int s = 0; s < R; ++s) {
    T a = 0;
    for (int s2 = 0; s2 < R; ++s2) a += T(pinv[s * R + s2]) * in[s2];
    y[base + s * plane] = a * sc;
  }
}

// ------------------------------------------------------- reductions -------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

__device__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < int(blockDim.x >> 6); ++i) r += sh[i];
  return r;  // valid in thread 0
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_seg_dots(Segs S, const T* __restrict__ V, int64_t vstride, int nvec,
                                                     const T* __restrict__ w, double* __restrict__ partial,
                                                     int nchunks) {
  __shared__ double sh[kBlock / 64];
  const int seg = blockIdx.y, chunk = blockIdx.x;
  const int64_t beg = S.off[seg] + int64_t(chunk) * kChunk;
  const int64_t end = S.off[seg + 1];
  constexpr int kPer = kChunk / kBlock;
  double wl[kPer];
#pragma unroll
  for (int t = 0; t < kPer; ++t) {
    const int64_t i = beg + int64_t(t) * kBlock + threadIdx.x;
    wl[t] = i < end ? double(w[i]) : 0.0;
  }
  for (int k = 0; k < nvec; ++k) {
    const T* vk = V + int64_t(k) * vstride;
    double acc = 0;
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
      const int64_t i = beg + int64_t(t) * kBlock + threadIdx.x;
      if (i < end) acc += double(vk[i]) * wl[t];
    }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[(int64_t(seg) * nchunks + chunk) * nvec + k] = acc;
  }
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_seg_axpy(Segs S, const T* __restrict__ V, int64_t vstride, int nvec,
                                                     const double* __restrict__ coef, int cstride, T* __restrict__ w,
                                                     double sign, double* __restrict__ partial, int nchunks) {
  __shared__ double sh[kBlock / 64];
  const int seg = blockIdx.y, chunk = blockIdx.x;
  const int64_t beg = S.off[seg] + int64_t(chunk) * kChunk;
  const int64_t end = S.off[seg + 1];
  constexpr int kPer = kChunk / kBlock;
  double nrm = 0;
  const double* c = coef + int64_t(seg) * cstride;
#pragma unroll
  for (int t = 0; t < kPer; ++t) {
    const int64_t i = beg + int64_t(t) * kBlock + threadIdx.x;
    if (i < end) {
      double a = double(w[i]);
      for (int k = 0; k < nvec; ++k) a += sign * c[k] * double(V[int64_t(k) * vstride + i]);
      const T r = T(a);
      w[i] = r;
      nrm += double(r) * double(r);
    }
  }
  if (partial) {
    nrm = block_sum(nrm, sh);
    if (threadIdx.x == 0) partial[int64_t(seg) * nchunks + chunk] = nrm;
  }
}

template <class T>
__global__ void k_seg_scale(Segs S, const T* __restrict__ w, const double* __restrict__ scal, T* __restrict__ out) {
  const int seg = blockIdx.y;
  const int64_t i = S.off[seg] + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= S.off[seg + 1]) return;
  out[i] = T(double(w[i]) * scal[seg]);
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
__global__ void k_addf2d(int64_t n, const float* __restrict__ x, double* __restrict__ y) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] += double(x[i]);
}

__global__ void k_finish(int nseg, int nvec, int nchunks, const double* __restrict__ partial, double* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nseg * nvec) return;
  const int seg = t / nvec, k = t - seg * nvec;
  double a = 0;
  for (int c = 0; c < nchunks; ++c) a += partial[(int64_t(seg) * nchunks + c) * nvec + k];
  out[t] = a;
}

// ------------------------------------------------------ GMRES bookkeeping --
__device__ __forceinline__ bool finite(double x) { return x == x && x - x == 0.0; }

__global__ void k_gmres_start(int nseg, GmresState st, const double* __restrict__ partial, int nchunks, double tol,
                              int first) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nseg) return;
  const int m = st.m;
  double s = 0;
  for (int c = 0; c < nchunks; ++c) s += partial[int64_t(g) * nchunks + c];
  const double beta = sqrt(s);
  if (first) st.bnorm[g] = beta;
  st.beta[g] = beta;
  for (int i = 0; i < (m + 1) * m; ++i) st.H[int64_t(g) * (m + 1) * m + i] = 0.0;
  for (int i = 0; i <= m; ++i) st.g[int64_t(g) * (m + 1) + i] = 0.0;
  st.g[int64_t(g) * (m + 1)] = beta;
  const bool act = finite(beta) && beta > 0.0 && beta > tol * st.bnorm[g];
  st.active[g] = act ? 1 : (finite(beta) ? 0 : -1);
  st.kused[g] = 0;
  st.inv[g] = act ? 1.0 / beta : 0.0;
}

__global__ void k_gmres_proj(int nseg, GmresState st, const double* __restrict__ partial, int nchunks, int j) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int nv = j + 1;
  if (t >= nseg * nv) return;
  const int g = t / nv, i = t - g * nv;
  const int m = st.m;
  double a = 0;
  for (int c = 0; c < nchunks; ++c) a += partial[(int64_t(g) * nchunks + c) * nv + i];
  if (st.active[g] != 1) a = 0.0;
  st.hcol[int64_t(g) * (m + 1) + i] = a;
  st.H[int64_t(g) * (m + 1) * m + int64_t(j) * (m + 1) + i] += a;
}

__global__ void k_gmres_givens(int nseg, GmresState st, const double* __restrict__ partial, int nchunks, int j,
                               double tol) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nseg) return;
  const int m = st.m;
  if (st.active[g] != 1) {
    st.inv[g] = 0.0;
    return;
  }
  double s = 0;
  for (int c = 0; c < nchunks; ++c) s += partial[int64_t(g) * nchunks + c];
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

__global__ void k_trace(DevGrids G, const double* __restrict__ u, double* __restrict__ out, int64_t npts_total) {
  // out is one-slice [grid][nx][nv]; u is G (R slices)
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= npts_total) return;
  int g = 0;
  int64_t acc = 0;
  while (g + 1 < G.n && idx >= acc + int64_t(G.nx[g]) * G.nv[g]) {
    acc += int64_t(G.nx[g]) * G.nv[g];
    ++g;
  }
  const int64_t p = idx - acc;
  const int64_t plane = int64_t(G.nx[g]) * G.nv[g];
  double a = 0;
  for (int s = 0; s < G.R; ++s) a += u[G.off[g] + s * plane + p];
  out[idx] = a;
}

__global__ void k_spread(DevGrids G, int R, const double* __restrict__ m, double* __restrict__ b,
                         int64_t npts_total) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= npts_total) return;
  int g = 0;
  int64_t acc = 0;
  while (g + 1 < G.n && idx >= acc + int64_t(G.nx[g]) * G.nv[g]) {
    acc += int64_t(G.nx[g]) * G.nv[g];
    ++g;
  }
  const int64_t p = idx - acc;
  const int64_t plane = int64_t(G.nx[g]) * G.nv[g];
  const double val = m[idx];
  for (int s = 0; s < R; ++s) b[int64_t(R) * acc + s * plane + p] = (s & 1) ? -val : val;
}

// ================================================================ launchers =
static inline unsigned nblk(int64_t n) { return unsigned((n + kBlock - 1) / kBlock); }
#define LAUNCH_CHECK() SGDG_CHECK_HIP(hipGetLastError())

template <class T>
void KernelsT<T>::sweeps(const DevGrids& G, const DevDomain& DX, const DevDomain& DV, const DevOp& op, const T* u,
                         T* W, T* Rr, int B, hipStream_t s) {
  const int64_t total = G.off[G.n];
  if (total == 0) return;
  hipLaunchKernelGGL(k_sweeps<T>, dim3(nblk(total), B), dim3(kBlock), 0, s, G, DX, DV, op, u, W, Rr, B);
  LAUNCH_CHECK();
}

template <class T>
void KernelsT<T>::scan_step(const DevGrids& G, const DevDomain& DX, const DevDomain& DV, const DevOp& op, T* Z, T* Q,
                            const T* Rr, int step, int B, hipStream_t s) {
  const int i_lo = step, i_up = G.n - 1 - step;
  const int64_t n_lo = int64_t(G.R) * G.nx[i_lo] * G.nv[i_lo];
  const int64_t n_up = int64_t(G.R) * G.nx[i_up] * G.nv[i_up];
  const int64_t n = n_lo > n_up ? n_lo : n_up;
  const int gy = (op.nvg > op.nxg ? op.nvg : op.nxg) * B;
  hipLaunchKernelGGL(k_scan<T>, dim3(nblk(n), gy, Q ? 2 : 1), dim3(kBlock), 0, s, G, DX, DV, op.nvg, op.nxg, Z, Q,
                     Rr, step, B);
  LAUNCH_CHECK();
}

template <class T>
void KernelsT<T>::final_(const DevGrids& G, const GridPts& P, const DevDomain& DX, const DevDomain& DV,
                         const DevOp& op, const T* Z, const T* Q, T* y, int B, hipStream_t s) {
  const int64_t npts = P.poff[G.n];
  if (npts == 0) return;
  hipLaunchKernelGGL(k_final<T>, dim3(nblk(npts), B), dim3(kBlock), 0, s, G, P, DX, DV, op, Z, Q, y, B);
  LAUNCH_CHECK();
}

template <class T>
void KernelsT<T>::restrict_x(const DevGrids& Go, const DevGrids& Gi, const DevDomain& DX, const T* in, T* out,
                             hipStream_t s) {
  const int64_t total = Go.off[Go.n];
  if (total == 0) return;
  hipLaunchKernelGGL(k_restrict_x<T>, dim3(nblk(total)), dim3(kBlock), 0, s, Go, Gi, DX, in, out);
  LAUNCH_CHECK();
}

template <class T>
void KernelsT<T>::combine(const DevGrids& Gu, const DevGrids& Gl, int lmin, const DevDomain& DX, const T* up,
                          const T* low, T* out, int R, hipStream_t s) {
  (void)R;
  const int64_t total = Gu.off[Gu.n];
  hipLaunchKernelGGL(k_combine<T>, dim3(nblk(total)), dim3(kBlock), 0, s, Gu, Gl, lmin, DX, up, low, out);
  LAUNCH_CHECK();
}

template <class T>
void KernelsT<T>::minv(const DevGrids& G, const GridPts& P, const DevDomain& DX, const DevDomain& DV,
                       const double* pinv, int sweeps, const T* x, T* y, T* tmp1, T* tmp2, hipStream_t s) {
  (void)sweeps;
  (void)tmp1;
  (void)tmp2;
  const int64_t npts = P.poff[G.n];
  hipLaunchKernelGGL(k_minv_jacobi<T>, dim3(nblk(npts)), dim3(kBlock), 0, s, G, P, DX, DV, pinv, x, y);
  LAUNCH_CHECK();
}

template <class T>
void KernelsT<T>::seg_dots(const Segs& S, const T* V, int64_t vstride, int nvec, const T* w, double* partial,
                           int nchunks, hipStream_t s) {
  hipLaunchKernelGGL(k_seg_dots<T>, dim3(nchunks, S.n), dim3(kBlock), 0, s, S, V, vstride, nvec, w, partial, nchunks);
  LAUNCH_CHECK();
}

template <class T>
void KernelsT<T>::seg_axpy_multi(const Segs& S, const T* V, int64_t vstride, int nvec, const double* coef, int cstride,
                                 T* w, double sign, double* partial_norm, int nchunks, hipStream_t s) {
  hipLaunchKernelGGL(k_seg_axpy<T>, dim3(nchunks, S.n), dim3(kBlock), 0, s, S, V, vstride, nvec, coef, cstride, w,
                     sign, partial_norm, nchunks);
  LAUNCH_CHECK();
}

template <class T>
void KernelsT<T>::seg_scale(const Segs& S, const T* w, const double* scal, T* out, hipStream_t s) {
  int64_t mx = 0;
  for (int i = 0; i < S.n; ++i) mx = mx > S.off[i + 1] - S.off[i] ? mx : S.off[i + 1] - S.off[i];
  if (mx == 0) return;
  hipLaunchKernelGGL(k_seg_scale<T>, dim3(nblk(mx), S.n), dim3(kBlock), 0, s, S, w, scal, out);
  LAUNCH_CHECK();
}

template <class T>
void KernelsT<T>::seg_norm2(const Segs& S, const T* w, double* partial, int nchunks, hipStream_t s) {
  hipLaunchKernelGGL(k_seg_dots<T>, dim3(nchunks, S.n), dim3(kBlock), 0, s, S, w, int64_t(0), 1, w, partial, nchunks);
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
void add_f32_to_f64(int64_t n, const float* x, double* y, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_addf2d, dim3(nblk(n)), dim3(kBlock), 0, s, n, x, y);
  LAUNCH_CHECK();
}
void finish_dots(int nseg, int nvec, int nchunks, const double* partial, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_finish, dim3(nblk(int64_t(nseg) * nvec)), dim3(kBlock), 0, s, nseg, nvec, nchunks, partial, out);
  LAUNCH_CHECK();
}
void gmres_start(int nseg, const GmresState& st, const double* partial, int nchunks, double tol, int first,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_gmres_start, dim3(nblk(nseg)), dim3(kBlock), 0, s, nseg, st, partial, nchunks, tol, first);
  LAUNCH_CHECK();
}
void gmres_add_proj(int nseg, const GmresState& st, const double* partial, int nchunks, int j, hipStream_t s) {
  hipLaunchKernelGGL(k_gmres_proj, dim3(nblk(int64_t(nseg) * (j + 1))), dim3(kBlock), 0, s, nseg, st, partial, nchunks,
                     j);
  LAUNCH_CHECK();
}
void gmres_givens(int nseg, const GmresState& st, const double* partial, int nchunks, int j, double tol,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_gmres_givens, dim3(nblk(nseg)), dim3(kBlock), 0, s, nseg, st, partial, nchunks, j, tol);
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
void trace_sum(const DevGrids& G, const double* u, double* out, hipStream_t s) {
  int64_t np = 0;
  for (int g = 0; g < G.n; ++g) np += int64_t(G.nx[g]) * G.nv[g];
  hipLaunchKernelGGL(k_trace, dim3(nblk(np)), dim3(kBlock), 0, s, G, u, out, np);
  LAUNCH_CHECK();
}
void spread_left(const DevGrids& G, int R, const double* m, double* b, hipStream_t s) {
  int64_t np = 0;
  for (int g = 0; g < G.n; ++g) np += int64_t(G.nx[g]) * G.nv[g];
  hipLaunchKernelGGL(k_spread, dim3(nblk(np)), dim3(kBlock), 0, s, G, R, m, b, np);
  LAUNCH_CHECK();
}

}  // namespace sgdg
