// Device kernels of libsgdg for gfx950 (wave64): transfers between component
// grids (embedding E and its transpose), the combination step, the inner
// preconditioner, Krylov primitives (segmented dot products / updates with
// FP64 accumulation, deterministic two-pass reductions), GMRES bookkeeping and
// right-hand-side helpers.  The operator itself is applied by fused.hip.
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
