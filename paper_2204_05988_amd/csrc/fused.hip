// Fused operator application for gfx950 (wave64, LDS-staged box tiles).
//
// For upper grid i (levels (lx, lv)), with V-groups j (terms sharing a v-factor)
// and X-groups m (terms sharing an x-factor), the block row of the strip
// operator is (Sect. 4.2, blockwise application with the embedding identities
// X_{l,l'} = X_l E_{l<-l'} for l' < l and E_{l'<-l}^T X_{l'} for l' > l):
//
//   y_i = sum_k Tm_k (X_k (x) I) [ (I (x) V_k) u_i + (E^x (x) I) Pt_i^{j(k)} ]      diagonal + lower partners
//       + sum_k Tm_k (I (x) V_k) (I (x) E^v) Qt_i^{m(k)}                          upper partners
//
// where the partner sums are carried by two scans whose arrays live on the
// lower diagonal (2^d times smaller than the upper grids):
//   Pt_{i+1} = (I (x) E^vT) [ (I (x) V) u_i + (E^x (x) I) Pt_i ]      on (lx_i,   lv_i - 1)
//   Qt_i     = (E^xT (x) I) [ (X (x) I) u_{i+1} + (I (x) E^v) Qt_{i+1} ] on (lx_i, lv_i - 1)
//
// The fused kernel works on a box of x-nodes times a box of v-nodes of one
// grid: phase 1 stages Z = V u + E^x Pt on the x-box plus a one-node halo in
// LDS, phase 2 applies every x-factor of the group from LDS; the upper part
// stages E^v Qt on the v-box plus halo and applies the v-factors.  Halo nodes
// are addressed by unwrapped box coordinates, so periodic wrap only appears
// when the staged values are fetched.
//
// The partner arrays Pt, Qt and their restrictions Rv, Rx keep the R slices
// of a node contiguous ([group][lower grid: n_x][n_v][R]).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fused.h"

namespace sgdg {

constexpr int kFB = 256;   // threads per block
constexpr int kRows = 4;   // box rows per thread: nxb <= kRows * (kFB / nvb)

template <class T> __device__ __forceinline__ const T* fv(const DevDomain& D);
template <> __device__ __forceinline__ const double* fv<double>(const DevDomain& D) { return D.vals; }
template <> __device__ __forceinline__ const float* fv<float>(const DevDomain& D) { return D.vals32; }
template <class T> __device__ __forceinline__ const T* tmx(const DevOp& op);
template <> __device__ __forceinline__ const double* tmx<double>(const DevOp& op) { return op.term_tm; }
template <> __device__ __forceinline__ const float* tmx<float>(const DevOp& op) { return op.term_tm32; }

// lattice helpers ------------------------------------------------------------
template <int D>
__device__ __forceinline__ void unflat(int p, const int* dims, int* c) {
#pragma unroll
  for (int a = D - 1; a >= 0; --a) {
    c[a] = p % dims[a];
    p /= dims[a];
  }
}
// node index of lattice coordinates (m nodes per axis); -1 if outside a non-periodic lattice
template <int D>
__device__ __forceinline__ int node_of(const int* c, int m, int periodic_cells) {
  int p = 0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    int x = c[a];
    if (periodic_cells > 0) {
      x %= periodic_cells;
      if (x < 0) x += periodic_cells;
    } else if (x < 0 || x >= m) {
      return -1;
    }
    p = p * m + x;
  }
  return p;
}

// LDS of a block: U (the item's u values on the x-halo box times the v-halo
// box, all slices) | the group stage | index tables.
// Per-block index tables live in LDS after the staging area:
//   xh_node[nxh]  x node of each halo row (-1 outside a non-periodic lattice)
//   xb_halo[nxb]  halo row of each box row;  xb_node[nxb] x node of each box row
//   vb_node[nvb]  v node of each box column; vb_halo[nvb] halo column of each box column
//   vh_node[nvh]  v node of each halo column (-1 outside)
// Threads own one box column (col = tid % nvb) and a strided set of rows, so
// stencil indices and v-factor values are loaded once per column and group.
template <class T, int D, int R>
__global__ void __launch_bounds__(kFB) k_fused(FusedCall<T> C) {
  constexpr int SS = D == 1 ? 3 : (D == 2 ? 7 : 15);  // Kuhn stencil size
  extern __shared__ unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  const FusedItem it = C.items[blockIdx.x];
  const int b = blockIdx.y;
  const ProbDesc& A = C.descs[it.prob];
  const DevGrids& G = A.G;
  const int g = it.grid;
  const int lx = G.lx[g], lv = G.lv[g];
  const int nx = G.nx[g], nv = G.nv[g];
  const int mx = A.mx[lx], mv = A.mv[lv];
  const int pcx = A.xper ? (1 << lx) : 0, pcv = A.vper ? (1 << lv) : 0;
  const DevOp& op = A.op;
  constexpr int Rin = R, Rout = R;
  const int64_t plane = int64_t(nx) * nv;
  const int64_t total = G.off[G.n];
  const T* ug = C.u + int64_t(b) * C.u_bstride + A.u_off + G.off[g];
  constexpr int SX = SS, SV = SS;
  (void)total;

  int xs[3] = {1, 1, 1}, vs[3] = {1, 1, 1}, xh[3] = {1, 1, 1}, vh[3] = {1, 1, 1};
  int nxb = 1, nvb = 1, nxh = 1, nvh = 1;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    xs[a] = it.xs[a];
    vs[a] = it.vs[a];
    xh[a] = xs[a] + 2;
    vh[a] = vs[a] + 2;
    nxb *= xs[a];
    nvb *= vs[a];
    nxh *= xh[a];
    nvh *= vh[a];
  }
  const bool has_p = !A.diag_only && g > 0;
  const bool has_q = !A.diag_only && g + 1 < G.n;
  T* U = lds;                    // [R][nxh][nvh]
  T* stg = lds + C.max_u;        // group stage
  // index tables
  int* tab = reinterpret_cast<int*>(lds + C.max_u + C.max_stage);
  int* xh_node = tab;
  int* xb_halo = xh_node + nxh;
  int* xb_node = xb_halo + nxb;
  int* vb_node = xb_node + nxb;
  int* vb_halo = vb_node + nvb;
  int* vh_node = vb_halo + nvb;
  for (int i = threadIdx.x; i < nxh; i += kFB) {
    int c[3];
    unflat<D>(i, xh, c);
#pragma unroll
    for (int a = 0; a < D; ++a) c[a] += it.xb[a] - 1;
    xh_node[i] = node_of<D>(c, mx, pcx);
  }
  for (int i = threadIdx.x; i < nxb; i += kFB) {
    int c[3];
    unflat<D>(i, xs, c);
    int h = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      h = h * xh[a] + c[a] + 1;
      c[a] += it.xb[a];
    }
    xb_halo[i] = h;
    xb_node[i] = node_of<D>(c, mx, 0);
  }
  for (int i = threadIdx.x; i < nvb; i += kFB) {
    int c[3];
    unflat<D>(i, vs, c);
    int h = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      h = h * vh[a] + c[a] + 1;
      c[a] += it.vb[a];
    }
    vb_halo[i] = h;
    vb_node[i] = node_of<D>(c, mv, 0);
  }
  for (int i = threadIdx.x; i < nvh; i += kFB) {
    int c[3];
    unflat<D>(i, vh, c);
#pragma unroll
    for (int a = 0; a < D; ++a) c[a] += it.vb[a] - 1;
    vh_node[i] = node_of<D>(c, mv, pcv);
  }
  // halo offsets of the stencil slots
  int dxh[SS], dvh[SS];
#pragma unroll
  for (int e = 0; e < SS; ++e) {
    int ox = 0, ov = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      ox = ox * xh[a] + A.off[e][a];
      ov = ov * vh[a] + A.off[e][a];
    }
    dxh[e] = ox;
    dvh[e] = ov;
  }
  __syncthreads();
  // stage u on the halo boxes once (zero outside the lattices)
  {
    const int nhh = nxh * nvh;
    for (int i = threadIdx.x; i < R * nhh; i += kFB) {
      const int s = i / nhh, rem = i - s * nhh;
      const int r = rem / nvh, c = rem - r * nvh;
      const int xn = xh_node[r], vn = vh_node[c];
      U[i] = (xn >= 0 && vn >= 0) ? ug[int64_t(s) * plane + int64_t(xn) * nv + vn] : T(0);
    }
  }
  __syncthreads();

  const int nrg = kFB / nvb;            // row groups (nvb <= kFB)
  const int col = threadIdx.x % nvb;
  const int rg = threadIdx.x / nvb;
  const bool active = rg < nrg;
  const int vi = active ? vb_node[col] : 0;
  const int vhc = active ? vb_halo[col] : 0;
  const T* xvals = fv<T>(A.DX);
  const T* vvals = fv<T>(A.DV);
  const T* tm = tmx<T>(op);
  const int64_t xlo = A.DX.lev_off[lx - A.DX.lmin];
  const int64_t vlo = A.DV.lev_off[lv - A.DV.lmin];

  T acc[kRows][R];
#pragma unroll
  for (int r = 0; r < kRows; ++r)
#pragma unroll
    for (int s = 0; s < R; ++s) acc[r][s] = T(0);

  // ---------------- diagonal + lower partners, one V-group at a time -------
  const int gl = g - 1;  // lower grid holding Pt_g: (lx-1, lv)
  const int64_t ltotal = A.Gl.off[A.Gl.n];
  const int64_t po = has_p ? A.DX.par_off[lx - A.DX.lmin] : 0;
  for (int j = 0; j < op.nvg; ++j) {
    if (active) {
      const T* vf = vvals + int64_t(op.vg_fac[j]) * A.DV.fac_stride + vlo + int64_t(vi) * SV;
      T fvv[SS];
#pragma unroll
      for (int e = 0; e < SS; ++e) fvv[e] = vf[e];
      const T* pt = has_p ? C.Pt + int64_t(b) * C.pt_bstride + A.pt_off + int64_t(j) * ltotal + A.Gl.off[gl] +
                                int64_t(vi) * R
                          : nullptr;
      for (int r = rg; r < nxh; r += nrg) {
        const int xi = xh_node[r];
#pragma unroll
        for (int s = 0; s < R; ++s) {
          T z = T(0);
          if (xi >= 0) {
            const T* urow = U + (s * nxh + r) * nvh + vhc;
#pragma unroll
            for (int e = 0; e < SS; ++e) z += fvv[e] * urow[dvh[e]];
            if (has_p) {
              const int64_t pp = po + 2 * int64_t(xi);
              const T* pr = pt + s;
              z += T(A.DX.parw[pp]) * pr[int64_t(A.DX.par[pp]) * nv * R] +
                   T(A.DX.parw[pp + 1]) * pr[int64_t(A.DX.par[pp + 1]) * nv * R];
            }
          }
          stg[(s * nxh + r) * nvb + col] = z;
        }
      }
    }
    __syncthreads();
    if (active) {
      const int k0 = op.vg_start[j], k1 = op.vg_start[j + 1];
#pragma unroll
      for (int q = 0; q < kRows; ++q) {
        const int r = rg + q * nrg;
        if (r >= nxb) break;
        const int hb = xb_halo[r];
        const int64_t xo = xlo + int64_t(xb_node[r]) * SX;
#pragma unroll
        for (int s2 = 0; s2 < R; ++s2) {
          // staged values of the x-neighbourhood, shared by every term of the group
          const T* l = stg + (s2 * nxh + hb) * nvb + col;
          T z[SS];
#pragma unroll
          for (int e = 0; e < SS; ++e) z[e] = l[dxh[e] * nvb];
          for (int kk = k0; kk < k1; ++kk) {
            const int k = op.vg_terms[kk];
            const T* fr = xvals + int64_t(op.term_xf[k]) * A.DX.fac_stride + xo;
            const T* tk = tm + int64_t(k) * R * R;
            T t = T(0);
#pragma unroll
            for (int e = 0; e < SS; ++e) t += fr[e] * z[e];
#pragma unroll
            for (int s = 0; s < R; ++s) acc[q][s] += tk[s * R + s2] * t;
          }
        }
      }
    }
    __syncthreads();
  }

  // ---------------- upper partners, one X-group at a time ------------------
  if (has_q) {
    const int nvl = A.Gl.nv[g];  // lower grid g: (lx, lv-1)
    const int64_t vpo = A.DV.par_off[lv - A.DV.lmin];
    const int nst = nxb * nvh;
    for (int m = 0; m < op.nxg; ++m) {
      const T* qt = C.Qt + int64_t(b) * C.qt_bstride + A.qt_off + int64_t(m) * ltotal + A.Gl.off[g];
      for (int h = threadIdx.x; h < nst; h += kFB) {
        const int r = h / nvh, c = h - (h / nvh) * nvh;
        const int vn = vh_node[c];
        const int xi = xb_node[r];
#pragma unroll
        for (int s = 0; s < R; ++s) {
          T z = T(0);
          if (vn >= 0) {
            const int64_t pp = vpo + 2 * int64_t(vn);
            const T* qr = qt + int64_t(xi) * nvl * R + s;
            z = T(A.DV.parw[pp]) * qr[int64_t(A.DV.par[pp]) * R] + T(A.DV.parw[pp + 1]) * qr[int64_t(A.DV.par[pp + 1]) * R];
          }
          stg[(s * nxb + r) * nvh + c] = z;
        }
      }
      __syncthreads();
      if (active) {
        for (int kk = op.xg_start[m]; kk < op.xg_start[m + 1]; ++kk) {
          const int k = op.xg_terms[kk];
          const T* vfk = vvals + int64_t(op.term_vf[k]) * A.DV.fac_stride + vlo + int64_t(vi) * SV;
          T fvv[SS];
#pragma unroll
          for (int e = 0; e < SS; ++e) fvv[e] = vfk[e];
          const T* tk = tm + int64_t(k) * Rout * Rin;
#pragma unroll
          for (int q = 0; q < kRows; ++q) {
            const int r = rg + q * nrg;
            if (r >= nxb) break;
#pragma unroll
            for (int s2 = 0; s2 < R; ++s2) {
              const T* l = stg + (s2 * nxb + r) * nvh + vhc;
              T t = T(0);
#pragma unroll
              for (int e = 0; e < SS; ++e) t += fvv[e] * l[dvh[e]];
#pragma unroll
              for (int s = 0; s < R; ++s) acc[q][s] += tk[s * R + s2] * t;
            }
          }
        }
      }
      __syncthreads();
    }
  }

  // ---------------- store -------------------------------------------------
  if (active) {
    T* yg = C.y + int64_t(b) * C.y_bstride + A.y_off + int64_t(Rout) * A.poff[g] + vi;
#pragma unroll
    for (int q = 0; q < kRows; ++q) {
      const int r = rg + q * nrg;
      if (r >= nxb) break;
      const int64_t p = int64_t(xb_node[r]) * nv;
#pragma unroll
      for (int s = 0; s < R; ++s) yg[int64_t(s) * plane + p] = acc[q][s];
    }
  }
}

// Scan step on the lower diagonal, the factor groups of a chunk per thread.
// Each item is one side: Pt_{t+1} on lower grid t, or Qt on lower grid
// nlow-1-t (both sides of a step in one launch).  The restricted stencils E^T V (resp. E^T X) of width W couple a
// coarse node with the fine nodes 2P + o; the u values at those nodes are
// loaded once and reused by every group.
// slot-major restricted stencils: entry o of the coarse nodes of one level is contiguous
template <class T> __device__ __forceinline__ const T* rv(const DevDomain& D);
template <> __device__ __forceinline__ const double* rv<double>(const DevDomain& D) { return D.trvals; }
template <> __device__ __forceinline__ const float* rv<float>(const DevDomain& D) { return D.trvals32; }
// slot-pair copies ([W/2][n][2] per level): slots 2p and 2p+1 of a coarse node
// adjacent, the pair read with one 2-wide load
template <class T> __device__ __forceinline__ const T* qrv(const DevDomain& D);
template <> __device__ __forceinline__ const double* qrv<double>(const DevDomain& D) { return D.qrvals; }
template <> __device__ __forceinline__ const float* qrv<float>(const DevDomain& D) { return D.qrvals32; }
// the R slices of one node, adjacent in memory: 2-wide loads
template <class T, int R>
__device__ __forceinline__ void load_slices_f(const T* p, T (&v)[R]) {
  typedef T T2 __attribute__((ext_vector_type(2)));
  int s = 0;
#pragma unroll
  for (; s + 2 <= R; s += 2) {
    const T2 a = *reinterpret_cast<const T2*>(p + s);
    v[s] = a.x;
    v[s + 1] = a.y;
  }
  if (s < R) v[s] = p[s];
}
// FP64 reads the pairs (fewer load instructions); FP32 single slots measured faster
template <class T> constexpr bool kScanPairs = sizeof(T) == 8;
template <class T, int S>
__device__ __forceinline__ void load_rpairs(const T* q, int64_t n, int64_t node, T (&f)[S]) {
  typedef T T2 __attribute__((ext_vector_type(2)));
#pragma unroll
  for (int p = 0; p < (S + 1) / 2; ++p) {
    const T2 a = *reinterpret_cast<const T2*>(q + (int64_t(p) * n + node) * 2);
    f[2 * p] = a.x;
    if (2 * p + 1 < S) f[2 * p + 1] = a.y;
  }
}

// One launch of the partner scans.  Mode 0 (a step): the restricted-stencil
// part from u plus the recursion term, which acts on the previous step's array
// through its restriction (E^x and E^vT act on different axes and commute):
//   Pt_{t}   = (I (x) E^vT V) u_t + (E^x (x) I) Rv_t,   Rv_t = (I (x) E^vT) Pt_{t-1}
//   Qt_l     = (E^xT X (x) I) u_{l+1} + (I (x) E^v) Rx_l, Rx_l = (E^xT (x) I) Qt_{l+1}
// Mode 2 computes Rv_t and Rx_l from the arrays the previous step finished.
template <class T, int D, int R>
__global__ void __launch_bounds__(kFB) k_scan2(FusedCall<T> C) {
  constexpr int W = D == 1 ? 5 : (D == 2 ? 19 : 65);
  constexpr int SS = D == 1 ? 3 : (D == 2 ? 7 : 15);
  constexpr int RS = R * W <= 48 ? R : 1;  // slices gathered per pass (registers)
  // vector-fastest block order: the blocks of one item for all vectors are
  // dispatched together, so the item's stencil tables are read from L2 by
  // every vector instead of being fetched again per vector (4% faster scans
  // at 64 vectors, measured; an XCD-contiguous order measured slower)
  const int lin = int(blockIdx.y) * int(gridDim.x) + int(blockIdx.x);
  const int bx = lin / int(gridDim.y), b = lin - bx * int(gridDim.y);
  const ScanItem si = C.sitems[bx];
  const ProbDesc& A = C.descs[si.prob];
  const DevGrids& G = A.G;
  const DevGrids& L = A.Gl;
  const bool lower = si.side == 0;
  const DevOp& op = A.op;
  // blockIdx.z: this block's share of the factor groups (shorter dependent
  // chains per thread, more blocks for the small steps)
  const int ng = lower ? op.nvg : op.nxg;
  const int g0 = int(blockIdx.z) * ng / int(gridDim.z), g1 = int(blockIdx.z + 1) * ng / int(gridDim.z);
  const int lg = si.lg;
  const int64_t ltotal = L.off[L.n];
  T* Ptb = C.Pt + int64_t(b) * C.pt_bstride + A.pt_off;
  T* Qtb = C.Qt + int64_t(b) * C.qt_bstride + A.qt_off;
  T* Rvb = C.Rv + int64_t(b) * C.rv_bstride + A.rv_off;
  T* Rxb = C.Rx + int64_t(b) * C.rx_bstride + A.rx_off;
  if (si.grp == 2) {
    if (lower) {
      // Rv_t[xc][vc] = sum_c chiw_c(vc) Pt_{t-1}[xc][chi_c(vc)], vc on the target's v-level
      const int nxs = L.nx[lg - 1], nvs = L.nv[lg - 1], nvt = L.nv[lg];
      const int64_t n = int64_t(nxs) * nvt;
      const int64_t e = si.start + threadIdx.x;
      if (e >= n) return;
      const int xc = int(e / nvt), vc = int(e - int64_t(e / nvt) * nvt);
      const int lvc = G.lv[lg] - 1 - A.DV.lmin;
      const int64_t co = A.DV.lev_off[lvc] + vc;
      // Pt_{t-1} holds values only on the rows where it is read
      const uint64_t need = C.sparse_partners ? op.xpt_mask[A.DX.node_off[G.lx[lg - 1] - A.DX.lmin] + xc] : ~uint64_t(0);
      int32_t ch[SS];
      T cw[SS];
#pragma unroll
      for (int c = 0; c < SS; ++c) {
        ch[c] = A.DV.tchi[co + int64_t(c) * nvt];
        cw[c] = T(A.DV.tchiw[co + int64_t(c) * nvt]);
      }
      for (int j = g0; j < g1; ++j) {
        if (j < 64 && !((need >> j) & 1)) continue;
        // the R slices of a child with one 2-wide load
        const T* row = Ptb + int64_t(j) * ltotal + L.off[lg - 1] + int64_t(xc) * nvs * R;
        T acc[R];
#pragma unroll
        for (int s = 0; s < R; ++s) acc[s] = T(0);
#pragma unroll
        for (int c = 0; c < SS; ++c) {
          T a[R];
          load_slices_f<T, R>(row + int64_t(ch[c]) * R, a);
#pragma unroll
          for (int s = 0; s < R; ++s) acc[s] += cw[c] * a[s];
        }
#pragma unroll
        for (int s = 0; s < R; ++s) Rvb[int64_t(j) * A.rv_len + A.rvo[lg] + e * R + s] = acc[s];
      }
    } else {
      // Rx_l[xc][vq] = sum_c chiw_c(xc) Qt_{l+1}[chi_c(xc)][vq], xc on the target's x-level
      const int nxt = L.nx[lg], nvs = L.nv[lg + 1];
      const int64_t n = int64_t(nxt) * nvs;
      const int64_t e = si.start + threadIdx.x;
      if (e >= n) return;
      const int xc = int(e / nvs), vq = int(e - int64_t(e / nvs) * nvs);
      const int lxc = G.lx[lg] - A.DX.lmin;  // target x-level (= lower grid lg's)
      const int64_t co = A.DX.lev_off[lxc] + xc;
      int32_t ch[SS];
      T cw[SS];
#pragma unroll
      for (int c = 0; c < SS; ++c) {
        ch[c] = A.DX.tchi[co + int64_t(c) * nxt];
        cw[c] = T(A.DX.tchiw[co + int64_t(c) * nxt]);
      }
      for (int m = g0; m < g1; ++m) {
        const T* col = Qtb + int64_t(m) * ltotal + L.off[lg + 1] + int64_t(vq) * R;
        T acc[R];
#pragma unroll
        for (int s = 0; s < R; ++s) acc[s] = T(0);
#pragma unroll
        for (int c = 0; c < SS; ++c) {
          T a[R];
          load_slices_f<T, R>(col + int64_t(ch[c]) * nvs * R, a);
#pragma unroll
          for (int s = 0; s < R; ++s) acc[s] += cw[c] * a[s];
        }
#pragma unroll
        for (int s = 0; s < R; ++s) Rxb[int64_t(m) * A.rx_len + A.rxo[lg] + e * R + s] = acc[s];
      }
    }
    return;
  }
  const int nxl = L.nx[lg], nvl = L.nv[lg];
  const int64_t lplane = int64_t(nxl) * nvl;
  const int64_t pt = si.start + threadIdx.x;  // target point x * nvl + v
  if (pt >= lplane) return;
  const int x = int(pt / nvl), v = int(pt - int64_t(pt / nvl) * nvl);
  const T* ub = C.u + int64_t(b) * C.u_bstride + A.u_off;
  if (lower) {
    // source grid t (lx, lv); target (lx, lv-1); recursion from Rv_t (x-level lx-1)
    const int src = lg;
    const int nv = G.nv[src];
    const int lvc = G.lv[src] - 1 - A.DV.lmin;  // level of v (coarse) = the target's
    const int64_t splane = int64_t(G.nx[src]) * nv;
    int32_t wi[W];
#pragma unroll
    for (int o = 0; o < W; ++o) wi[o] = A.DV.twide[A.DV.wlev_off[lvc] + int64_t(o) * nvl + v];
    const bool has_p = src > 0;
    // Pt^j is computed only where it is read (v-groups of face terms: near the x-faces)
    const uint64_t need = C.sparse_partners ? op.xpt_mask[A.DX.node_off[G.lx[src] - A.DX.lmin] + x] : ~uint64_t(0);
    int32_t p0 = 0, p1 = 0;
    T w0 = 0, w1 = 0;
    if (has_p) {
      const int64_t po = A.DX.par_off[G.lx[src] - A.DX.lmin] + 2 * int64_t(x);
      p0 = A.DX.par[po];
      p1 = A.DX.par[po + 1];
      w0 = T(A.DX.parw[po]);
      w1 = T(A.DX.parw[po + 1]);
    }
    for (int s0 = 0; s0 < R; s0 += RS) {
      T un[RS][W];
#pragma unroll
      for (int q = 0; q < RS; ++q) {
        const T* us = ub + G.off[src] + int64_t(s0 + q) * splane + int64_t(x) * nv;
#pragma unroll
        for (int o = 0; o < W; ++o) un[q][o] = us[wi[o]];
      }
      for (int j = g0; j < g1; ++j) {
        if (j < 64 && !((need >> j) & 1)) continue;
        T rr[W];
        if constexpr (kScanPairs<T>) {
          load_rpairs<T, W>(qrv<T>(A.DV) + int64_t(op.vg_fac[j]) * A.DV.qrstride + A.DV.qrlev_off[lvc], nvl, v, rr);
        } else {
          const T* r = rv<T>(A.DV) + int64_t(op.vg_fac[j]) * A.DV.rstride + A.DV.wlev_off[lvc] + v;
#pragma unroll
          for (int o = 0; o < W; ++o) rr[o] = r[int64_t(o) * nvl];
        }
        // the two x-parents' restricted values, all RS slices per 2-wide load
        T ra[RS], rb[RS];
        if (has_p) {
          const T* rvp = Rvb + int64_t(j) * A.rv_len + A.rvo[lg] + int64_t(v) * R + s0;
          load_slices_f<T, RS>(rvp + int64_t(p0) * nvl * R, ra);
          load_slices_f<T, RS>(rvp + int64_t(p1) * nvl * R, rb);
        }
#pragma unroll
        for (int q = 0; q < RS; ++q) {
          const int s = s0 + q;
          T acc = T(0);
#pragma unroll
          for (int o = 0; o < W; ++o) acc += rr[o] * un[q][o];
          if (has_p) acc += w0 * ra[q] + w1 * rb[q];
          Ptb[int64_t(j) * ltotal + L.off[lg] + pt * R + s] = acc;
        }
      }
    }
  } else {
    // source grid lg+1 (lx+1, lv-1); target lower lg (lx, lv-1); recursion from Rx_lg (v-level lv-2)
    const int src = lg + 1;
    const int nv = G.nv[src];
    const int lxc = G.lx[src] - 1 - A.DX.lmin;  // level of x (coarse) = the target's
    const int64_t splane = int64_t(G.nx[src]) * nv;
    int32_t wi[W];
#pragma unroll
    for (int o = 0; o < W; ++o) wi[o] = A.DX.twide[A.DX.wlev_off[lxc] + int64_t(o) * nxl + x];
    const bool has_q = src + 1 < G.n;
    // Qt^m is computed only where it can be nonzero (face terms: near the
    // x-faces); elsewhere it is exactly zero and stored as such, for the
    // restriction of the next step reads every child
    const uint64_t need = C.sparse_partners ? op.xqt_mask[A.DX.node_off[G.lx[lg] - A.DX.lmin] + x] : ~uint64_t(0);
    int32_t p0 = 0, p1 = 0;
    T w0 = 0, w1 = 0;
    int nvq = 0;
    if (has_q) {
      const int64_t po = A.DV.par_off[G.lv[src] - A.DV.lmin] + 2 * int64_t(v);
      p0 = A.DV.par[po];
      p1 = A.DV.par[po + 1];
      w0 = T(A.DV.parw[po]);
      w1 = T(A.DV.parw[po + 1]);
      nvq = L.nv[src];
    }
    for (int s0 = 0; s0 < R; s0 += RS) {
      T un[RS][W];
#pragma unroll
      for (int q = 0; q < RS; ++q) {
        const T* us = ub + G.off[src] + int64_t(s0 + q) * splane + v;
#pragma unroll
        for (int o = 0; o < W; ++o) un[q][o] = us[int64_t(wi[o]) * nv];
      }
      for (int m = g0; m < g1; ++m) {
        if (m < 64 && !((need >> m) & 1)) {
#pragma unroll
          for (int q = 0; q < RS; ++q) Qtb[int64_t(m) * ltotal + L.off[lg] + pt * R + s0 + q] = T(0);
          continue;
        }
        T rr[W];
        if constexpr (kScanPairs<T>) {
          load_rpairs<T, W>(qrv<T>(A.DX) + int64_t(op.xg_fac[m]) * A.DX.qrstride + A.DX.qrlev_off[lxc], nxl, x, rr);
        } else {
          const T* r = rv<T>(A.DX) + int64_t(op.xg_fac[m]) * A.DX.rstride + A.DX.wlev_off[lxc] + x;
#pragma unroll
          for (int o = 0; o < W; ++o) rr[o] = r[int64_t(o) * nxl];
        }
        // the two v-parents' restricted values, all RS slices per 2-wide load
        T ra[RS], rb[RS];
        if (has_q) {
          const T* rxp = Rxb + int64_t(m) * A.rx_len + A.rxo[lg] + int64_t(x) * nvq * R + s0;
          load_slices_f<T, RS>(rxp + int64_t(p0) * R, ra);
          load_slices_f<T, RS>(rxp + int64_t(p1) * R, rb);
        }
#pragma unroll
        for (int q = 0; q < RS; ++q) {
          const int s = s0 + q;
          T acc = T(0);
#pragma unroll
          for (int o = 0; o < W; ++o) acc += rr[o] * un[q][o];
          if (has_q) acc += w0 * ra[q] + w1 * rb[q];
          Qtb[int64_t(m) * ltotal + L.off[lg] + pt * R + s] = acc;
        }
      }
    }
  }
}

// ------------------------------------------------------------- launchers --
template <class T>
void fused_scan_step(const FusedCall<T>& C, int nsitems, int d, int R, int chunks, hipStream_t s) {
  if (nsitems == 0) return;
  dim3 grid(unsigned(nsitems), C.B, unsigned(std::max(1, chunks)));
#define SGDG_SCAN_CASE(DD, RR) \
  if (d == DD && R == RR) hipLaunchKernelGGL((k_scan2<T, DD, RR>), grid, dim3(kFB), 0, s, C);
  SGDG_SCAN_CASE(1, 1) SGDG_SCAN_CASE(1, 2) SGDG_SCAN_CASE(1, 3)
  SGDG_SCAN_CASE(2, 1) SGDG_SCAN_CASE(2, 2) SGDG_SCAN_CASE(2, 3)
  SGDG_SCAN_CASE(3, 1) SGDG_SCAN_CASE(3, 2) SGDG_SCAN_CASE(3, 3)
#undef SGDG_SCAN_CASE
  SGDG_CHECK_HIP(hipGetLastError());
}

template <class T>
void fused_tiles(const FusedCall<T>& C, int d, int R, hipStream_t s) {
  const size_t sm = size_t(C.max_u + C.max_stage) * sizeof(T) + size_t(C.max_tab) * sizeof(int);
  if (sm > 64 * 1024) throw Error{SGDG_E_ARG, "box tiles exceed the LDS budget"};
  dim3 grid(unsigned(C.nitems), C.B);
#define SGDG_FUSED_CASE(DD, RR) \
  if (d == DD && R == RR) hipLaunchKernelGGL((k_fused<T, DD, RR>), grid, dim3(kFB), sm, s, C);
  SGDG_FUSED_CASE(1, 1) SGDG_FUSED_CASE(1, 2) SGDG_FUSED_CASE(1, 3)
  SGDG_FUSED_CASE(2, 1) SGDG_FUSED_CASE(2, 2) SGDG_FUSED_CASE(2, 3)
  SGDG_FUSED_CASE(3, 1) SGDG_FUSED_CASE(3, 2) SGDG_FUSED_CASE(3, 3)
#undef SGDG_FUSED_CASE
  SGDG_CHECK_HIP(hipGetLastError());
}

template void fused_scan_step<double>(const FusedCall<double>&, int, int, int, int, hipStream_t);
template void fused_scan_step<float>(const FusedCall<float>&, int, int, int, int, hipStream_t);
template void fused_tiles<double>(const FusedCall<double>&, int, int, hipStream_t);
template void fused_tiles<float>(const FusedCall<float>&, int, int, hipStream_t);

int fused_rows_per_thread() { return kRows; }
int fused_threads() { return kFB; }

}  // namespace sgdg
