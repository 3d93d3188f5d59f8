// Split operator application for gfx950: three streaming passes over the
// points of every upper grid, with a v-stage kept in HBM between them.
//
// With X-groups m (terms sharing an x-factor X_m) and the V-group j(k) of each
// term, the block row of upper grid i is (Sect. 4.2, with the embedding
// identities X_{l,l'} = X_l E_{l<-l'} below and E_{l'<-l}^T X_{l'} above):
//
//   y_i = sum_m (X_m (x) I) W_i^m + sum_k Tm_k (I (x) V_k) (I (x) E^v) Qt_i^{m(k)}
//   W_i^m = sum_{k in m} Tm_k [ (I (x) V_k) u_i + (E^x (x) I) Pt_i^{j(k)} ]
//
// Pass 1 (k_vstage) computes W for every X-group: the v-stencils of u (v is
// the fastest axis, so the neighbour gathers stay in L1/L2), the x-prolonged
// lower-partner scan arrays and the time-block mixing.  Pass 1b (k_ustage)
// writes the upper-partner part into y with the prolongated stencils V_k E^v.
// Pass 2 (k_xstage per point, k_xtile on LDS tiles) adds one x-stencil per
// X-group applied to W.  Grouping by x-factor makes the number of staged
// arrays and of x-stencil passes the number of distinct x-factors.  One
// thread owns one point and BC vectors of the batch; the stencil indices,
// parent tables and factor values of its point are loaded once and reused
// across them.  What bounds these passes is the vector-memory instruction
// rate of a CU, so the layouts below let one load move two values and the
// tiled forms serve reused values from LDS.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>

#include "split.h"

namespace sgdg {

namespace {

constexpr int kSB = 256;  // threads (points) per block
constexpr int kQlIters = 2;  // staged coarse range of an item: at most kQlIters * kSB nodes
constexpr int kTileIters = 4;  // staged x-stencil tile: at most kTileIters * kSB values per slab
constexpr int kTileFacIters = 2;  // staged x-factors of a tile: at most kTileFacIters * kSB values
// slot-major factor tables: entry e of the nodes of one level is contiguous
template <class T> __device__ __forceinline__ const T* vals(const DevDomain& D);
template <> __device__ __forceinline__ const double* vals<double>(const DevDomain& D) { return D.tvals; }
template <> __device__ __forceinline__ const float* vals<float>(const DevDomain& D) { return D.tvals32; }
template <class T> __device__ __forceinline__ const T* pvals(const DevDomain& D);
template <> __device__ __forceinline__ const double* pvals<double>(const DevDomain& D) { return D.pvals; }
template <> __device__ __forceinline__ const float* pvals<float>(const DevDomain& D) { return D.pvals32; }
template <class T> __device__ __forceinline__ const T* tmat(const DevOp& op);
template <> __device__ __forceinline__ const double* tmat<double>(const DevOp& op) { return op.term_tm; }
template <> __device__ __forceinline__ const float* tmat<float>(const DevOp& op) { return op.term_tm32; }

// The staged W keeps the R slices of a point contiguous ([grid][x][v][R]), so
// the x-stage reads a pair of slices with one 2-wide load (half the memory
// instructions).
// slot-pair factor tables ([S/2][n][2] per level): slots 2p, 2p+1 of a node
// are adjacent and read with one 2-wide load
template <class T> __device__ __forceinline__ const T* qvals(const DevDomain& D);
template <> __device__ __forceinline__ const double* qvals<double>(const DevDomain& D) { return D.qvals; }
template <> __device__ __forceinline__ const float* qvals<float>(const DevDomain& D) { return D.qvals32; }
template <class T> __device__ __forceinline__ const T* qpvals(const DevDomain& D);
template <> __device__ __forceinline__ const double* qpvals<double>(const DevDomain& D) { return D.qpvals; }
template <> __device__ __forceinline__ const float* qpvals<float>(const DevDomain& D) { return D.qpvals32; }
template <class T, int S>
__device__ __forceinline__ void load_slot_pairs(const T* q, int64_t n, int64_t node, T (&f)[S]) {
  typedef T T2 __attribute__((ext_vector_type(2)));
#pragma unroll
  for (int p = 0; p < (S + 1) / 2; ++p) {
    const T2 a = *reinterpret_cast<const T2*>(q + (int64_t(p) * n + node) * 2);
    f[2 * p] = a.x;
    if (2 * p + 1 < S) f[2 * p + 1] = a.y;
  }
}

template <class T, int R>
__device__ __forceinline__ void load_slices(const T* p, T (&v)[R]) {
  typedef T T2 __attribute__((ext_vector_type(2)));
  int s = 0;
#pragma unroll
  for (; s + 2 <= R; s += 2) {
    const T2 a = *reinterpret_cast<const T2*>(p + s);
    v[s] = a.x;
    v[s + 1] = a.y;
  }
  if constexpr (R % 2 == 1) v[R - 1] = p[R - 1];
}

// Item and vector group of this block.  With C.xcd the linear block id is
// remapped so that XCD k (blocks are dealt to the 8 XCDs round-robin) runs one
// contiguous range of (vector group, item) pairs and its L2 sees neighbouring
// items together.
template <class T>
__device__ __forceinline__ void block_coords(const SplitCall<T>& C, int& item, int& vg) {
  int L = int(blockIdx.y) * int(gridDim.x) + int(blockIdx.x);
  if (C.xcd) {
    const int total = int(gridDim.x) * int(gridDim.y);
    const int per = total >> 3, rem = total & 7, k = L & 7;
    L = k * per + min(k, rem) + (L >> 3);
  }
  vg = L / int(gridDim.x);
  item = L - vg * int(gridDim.x);
}

// X-groups whose factor's stencil rows with a nonzero read x-node x of level
// lx (read_needs), or whose factor has a nonzero in row x (row_needs); bit m
// for group m < 64 (groups beyond are always taken)
__device__ __forceinline__ uint64_t read_needs(const DevDomain& DX, const DevOp& op, int lx, int x) {
  return op.xread_mask[DX.node_off[lx - DX.lmin] + x];
}
__device__ __forceinline__ uint64_t row_needs(const DevDomain& DX, const DevOp& op, int lx, int x) {
  return op.xrow_mask[DX.node_off[lx - DX.lmin] + x];
}

template <class T, int D, int R, int BC>
__global__ void __launch_bounds__(kSB) k_vstage(SplitCall<T> C) {
  constexpr int SS = D == 1 ? 3 : (D == 2 ? 7 : 15);
  int ii, vg;
  block_coords(C, ii, vg);
  const SplitItem it = C.items[ii];
  const int b0 = vg * BC;
  const ProbDesc& A = C.descs[it.prob];
  const int g = it.grid;
  const int nx = A.G.nx[g], nv = A.G.nv[g];
  const int64_t plane = int64_t(nx) * nv;
  const int64_t p = it.p0 + threadIdx.x;
  if (p >= plane) return;
  const int x = int(p / nv), v = int(p - int64_t(p / nv) * nv);
  const int lx = A.G.lx[g], lv = A.G.lv[g];
  const int64_t vlo = A.DV.lev_off[lv - A.DV.lmin];
  const DevOp& op = A.op;
  int32_t nbv[SS];
#pragma unroll
  for (int e = 0; e < SS; ++e) nbv[e] = A.DV.tnbr[vlo + int64_t(e) * nv + v];
  const bool has_p = !A.diag_only && g > 0;
  int32_t px0 = 0, px1 = 0;
  T wx0 = 0, wx1 = 0;
  int64_t lo = 0;
  if (has_p) {
    const int64_t pp = A.DX.par_off[lx - A.DX.lmin] + 2 * int64_t(x);
    px0 = A.DX.par[pp];
    px1 = A.DX.par[pp + 1];
    wx0 = T(A.DX.parw[pp]);
    wx1 = T(A.DX.parw[pp + 1]);
    lo = A.Gl.off[g - 1];
  }
  const int64_t total = A.G.off[A.G.n];
  const int64_t ltotal = A.Gl.off[A.Gl.n];
  const T* tm = tmat<T>(op);
  // W^m is read only by the x-stencils of the rows where X-group m's factor
  // has a nonzero: a face term's W is needed on its face's x-nodes and their
  // stencil neighbours alone; elsewhere its terms are skipped and nothing is
  // stored (the x-stage skips the rows that would read it there)
  // (not for d <= 2 with one vector per thread: there the branches cost more
  // than the skipped terms save, measured, and W is staged everywhere)
  constexpr bool kSkip = D == 3 || BC > 1;
  const uint64_t need = kSkip ? read_needs(A.DX, op, lx, x) : ~uint64_t(0);
  auto needs = [&](int m) { return !kSkip || m >= 64 || ((need >> m) & 1); };
  T un[BC][R][SS];
#pragma unroll
  for (int q = 0; q < BC; ++q) {
    const int b = b0 + q < C.B ? b0 + q : b0;
    const T* ub = C.u + int64_t(b) * C.u_bstride + A.u_off + A.G.off[g] + int64_t(x) * nv;
#pragma unroll
    for (int s = 0; s < R; ++s)
#pragma unroll
      for (int e = 0; e < SS; ++e) un[q][s][e] = ub[int64_t(s) * plane + nbv[e]];
  }
  // Terms in X-group order, software-pipelined for d <= 2 and BC > 1: the v-factors and
  // the lower-partner values of term kk + 1 are loaded while term kk is
  // computed; W^m is stored when its group's last term is done (empty groups
  // store 0).
  const int nt = op.xg_start[op.nxg];
  auto load = [&](int kk, T (&f)[SS], T (&pv)[BC][R][2]) {
    if (!needs(op.xg_of[kk])) {
#pragma unroll
      for (int e = 0; e < SS; ++e) f[e] = T(0);
#pragma unroll
      for (int q = 0; q < BC; ++q)
#pragma unroll
        for (int s2 = 0; s2 < R; ++s2) pv[q][s2][0] = pv[q][s2][1] = T(0);
      return;
    }
    const int k = op.xg_terms[kk];
    load_slot_pairs<T, SS>(qvals<T>(A.DV) + int64_t(op.term_vf[k]) * A.DV.qfac_stride + A.DV.qlev_off[lv - A.DV.lmin],
                           nv, v, f);
    const int j = op.term_vg[k];
#pragma unroll
    for (int q = 0; q < BC; ++q) {
      const int b = b0 + q < C.B ? b0 + q : b0;
      const T* pt = C.Pt + int64_t(b) * C.pt_bstride + A.pt_off + int64_t(j) * ltotal + lo + int64_t(v) * R;
      T a0[R], a1[R];
      if (has_p) {
        load_slices<T, R>(pt + int64_t(px0) * nv * R, a0);
        // an x-node that coincides with a coarse node has one parent (the
        // second weight is zero); a wavefront within one x-row skips the load
        if (wx1 != T(0)) {
          load_slices<T, R>(pt + int64_t(px1) * nv * R, a1);
        } else {
#pragma unroll
          for (int s2 = 0; s2 < R; ++s2) a1[s2] = T(0);
        }
      } else {
#pragma unroll
        for (int s2 = 0; s2 < R; ++s2) a0[s2] = a1[s2] = T(0);
      }
#pragma unroll
      for (int s2 = 0; s2 < R; ++s2) {
        pv[q][s2][0] = a0[s2];
        pv[q][s2][1] = a1[s2];
      }
    }
  };
  T w[BC][R];
#pragma unroll
  for (int q = 0; q < BC; ++q)
#pragma unroll
    for (int s = 0; s < R; ++s) w[q][s] = T(0);
  auto store = [&](int m) {
    const bool nm = needs(m);
#pragma unroll
    for (int q = 0; q < BC; ++q) {
      const int b = b0 + q;
      if (b < C.B && nm) {
        // W is read once, by the x-stage pass: stream it past the caches (a
        // 2-wide store of the slice pair measured slower than two scalar ones)
        T* zb = C.Z + int64_t(b) * C.z_bstride + A.z_off + int64_t(m) * total + A.G.off[g] + p * R;
#pragma unroll
        for (int s = 0; s < R; ++s) __builtin_nontemporal_store(w[q][s], zb + s);
      }
#pragma unroll
      for (int s = 0; s < R; ++s) w[q][s] = T(0);
    }
  };
  // for d = 3, and for one vector per thread, the extra registers cost more
  // occupancy than the pipelining hides (measured)
  constexpr bool kPipe = D <= 2 && BC > 1;
  T fn[SS], pn[BC][R][2];
  if (kPipe && nt > 0) load(0, fn, pn);
  int m = 0;
  for (int kk = 0; kk < nt; ++kk) {
    T fc[SS], pc[BC][R][2];
    if constexpr (kPipe) {
#pragma unroll
      for (int e = 0; e < SS; ++e) fc[e] = fn[e];
#pragma unroll
      for (int q = 0; q < BC; ++q)
#pragma unroll
        for (int s2 = 0; s2 < R; ++s2) {
          pc[q][s2][0] = pn[q][s2][0];
          pc[q][s2][1] = pn[q][s2][1];
        }
      if (kk + 1 < nt) load(kk + 1, fn, pn);
    } else {
      load(kk, fc, pc);
    }
    while (kk >= op.xg_start[m + 1]) store(m++);  // empty groups before this term's
    if (!needs(m)) {
      if (kk + 1 == op.xg_start[m + 1]) store(m++);
      continue;
    }
    const T* tk = tm + int64_t(op.xg_terms[kk]) * R * R;
    T tkv[R * R];
#pragma unroll
    for (int i = 0; i < R * R; ++i) tkv[i] = tk[i];
#pragma unroll
    for (int q = 0; q < BC; ++q)
#pragma unroll
      for (int s2 = 0; s2 < R; ++s2) {
        T z = wx0 * pc[q][s2][0] + wx1 * pc[q][s2][1];
#pragma unroll
        for (int e = 0; e < SS; ++e) z += fc[e] * un[q][s2][e];
#pragma unroll
        for (int s = 0; s < R; ++s) w[q][s] += tkv[s * R + s2] * z;
      }
    if (kk + 1 == op.xg_start[m + 1]) store(m++);
  }
  while (m < op.nxg) store(m++);
}

// Pass 1b: y = upper-partner part sum_k Tm_k (I (x) V_k E^v) Qt^{m(k)}, with the
// prolongated stencils V_k E^v (fine node -> 3^d coarse nodes around floor(v/2))
// precomputed per level; zero for grids without an upper partner.  Pass 2 then
// adds the x-stencils.  For d <= 2 the coarse range an item touches (host
// computed) is staged in LDS once per X-group, so the 3^d slot reads of every
// point come from LDS instead of the vector L1 (QL); without staging (a range
// too long for LDS) the slots are read from memory.  The 3^d-slot gathers are
// what bounds this pass: served by the vector L1 they run at a fraction of
// the LDS read rate.
template <class T, int D, int R, int BC, bool QL>
__global__ void __launch_bounds__(kSB) k_ustage(SplitCall<T> C) {
  extern __shared__ unsigned char split_smem[];
  T* sq = reinterpret_cast<T*>(split_smem);  // two buffers [BC][R][qn]
  int ii, vg;
  block_coords(C, ii, vg);
  const SplitItem it = C.items[ii];
  const int b0 = vg * BC;
  const ProbDesc& A = C.descs[it.prob];
  const int g = it.grid;
  const int nx = A.G.nx[g], nv = A.G.nv[g];
  const int64_t plane = int64_t(nx) * nv;
  const int64_t p = it.p0 + threadIdx.x;
  const bool act = p < plane;
  const int x = act ? int(p / nv) : 0;
  const int v = act ? int(p - int64_t(x) * nv) : 0;
  const int lv = A.G.lv[g];
  const DevOp& op = A.op;
  const T* tm = tmat<T>(op);
  T acc[BC][R];
#pragma unroll
  for (int q = 0; q < BC; ++q)
#pragma unroll
    for (int s = 0; s < R; ++s) acc[q][s] = T(0);
  const bool has_q = !A.diag_only && g + 1 < A.G.n;
  if (has_q) {
    const int nvl = A.Gl.nv[g];  // lower grid g: (lx, lv - 1)
    const int64_t ltotal = A.Gl.off[A.Gl.n];
    // Either the prolongated stencils V_k E^v on 3^d coarse slots (d <= 2), or,
    // for d = 3 where 27 slots cost more than 2 parents of 15 neighbours,
    // the v-stencil of Qt prolonged on the fly.
    constexpr bool kPro = D <= 2;
    constexpr int NS = kPro ? (D == 1 ? 3 : 9) : 15;  // slots per point
    constexpr bool ql = kPro && QL;
    int32_t i0[NS], i1[NS];
    T w0[NS], w1[NS];
    int64_t fbase;
    int64_t fstride;
    const T* fvals;
    if constexpr (kPro) {
      const int64_t plo = A.DV.plev_off[lv - A.DV.lmin];
#pragma unroll
      for (int sl = 0; sl < NS; ++sl) {
        i0[sl] = A.DV.pidx[plo + int64_t(sl) * nv + v];
        i1[sl] = 0;
        w0[sl] = T(1);
        w1[sl] = T(0);
      }
      fvals = pvals<T>(A.DV);
      fbase = plo + v;
      fstride = A.DV.pstride;
    } else {
      const int64_t vlo = A.DV.lev_off[lv - A.DV.lmin];
      const int64_t vpo = A.DV.par_off[lv - A.DV.lmin];
#pragma unroll
      for (int e = 0; e < NS; ++e) {
        const int32_t vn = A.DV.tnbr[vlo + int64_t(e) * nv + v];
        i0[e] = A.DV.par[vpo + 2 * int64_t(vn)];
        i1[e] = A.DV.par[vpo + 2 * int64_t(vn) + 1];
        w0[e] = T(A.DV.parw[vpo + 2 * int64_t(vn)]);
        w1[e] = T(A.DV.parw[vpo + 2 * int64_t(vn) + 1]);
      }
      fvals = vals<T>(A.DV);
      fbase = vlo + v;
      fstride = A.DV.fac_stride;
    }
    // one term of X-group m: acc += Tm_k (slots of V_k) . qv
    auto term = [&](int k, const T (&vf)[NS], const T (&qv)[BC][R][NS]) {
      const T* tk = tm + int64_t(k) * R * R;
      T tkv[R * R];
#pragma unroll
      for (int i = 0; i < R * R; ++i) tkv[i] = tk[i];
#pragma unroll
      for (int q = 0; q < BC; ++q)
#pragma unroll
        for (int s2 = 0; s2 < R; ++s2) {
          T t = T(0);
#pragma unroll
          for (int e = 0; e < NS; ++e) t += vf[e] * qv[q][s2][e];
#pragma unroll
          for (int s = 0; s < R; ++s) acc[q][s] += tkv[s * R + s2] * t;
        }
    };
    auto factors = [&](int k, T (&vf)[NS]) {
      if constexpr (kPro) {
        load_slot_pairs<T, NS>(qpvals<T>(A.DV) + int64_t(op.term_vf[k]) * A.DV.qpstride +
                                   A.DV.qplev_off[lv - A.DV.lmin],
                               nv, v, vf);
      } else {
        const T* f = fvals + int64_t(op.term_vf[k]) * fstride + fbase;
#pragma unroll
        for (int e = 0; e < NS; ++e) vf[e] = f[int64_t(e) * nv];
      }
    };
    if constexpr (ql) {
      // Software pipeline over the X-groups with two LDS buffers: the coarse
      // range of group m + 1 is fetched into registers while group m is
      // computed, so one barrier per group and no exposed fetch latency.
      const int qn = it.qn;
      T pre[BC][R * kQlIters];
      // the range is qn R contiguous values per vector (slices fastest)
      const int qnr = qn * R;
      auto fetch = [&](int m) {
        const T* qm = C.Qt + A.qt_off + int64_t(m) * ltotal + A.Gl.off[g] + it.q0 * R;
#pragma unroll
        for (int q = 0; q < BC; ++q) {
          const int b = b0 + q < C.B ? b0 + q : b0;
#pragma unroll
          for (int j = 0; j < R * kQlIters; ++j) {
            const int i = int(threadIdx.x) + j * kSB;
            if (i < qnr) pre[q][j] = qm[int64_t(b) * C.qt_bstride + i];
          }
        }
      };
      // only the X-groups whose Qt^m can be nonzero on the block's rows
      // (it.gmask), and per thread on its own row (face terms off the face)
      const uint64_t rneed = act ? op.xqt_mask[A.DX.node_off[A.G.lx[g] - A.DX.lmin] + x] : 0;
      auto gnext = [&](int m) {
        ++m;
        while (m < op.nxg && m < 64 && !((it.gmask >> m) & 1)) ++m;
        return m;
      };
      int m = gnext(-1);
      if (m < op.nxg) fetch(m);
      const int qo = int(int64_t(x) * nvl - it.q0);  // every slot of the item lies in the range (host)
      for (int n = 0; m < op.nxg; ++n) {
        const int mn = gnext(m);
        T* cur = sq + (n & 1) * (BC * qnr);
#pragma unroll
        for (int q = 0; q < BC; ++q)
#pragma unroll
          for (int j = 0; j < R * kQlIters; ++j) {
            const int i = int(threadIdx.x) + j * kSB;
            if (i < qnr) cur[q * qnr + i] = pre[q][j];
          }
        const int ka = op.xg_start[m], kb = op.xg_start[m + 1];
        const bool use = act && ka < kb && (m >= 64 || ((rneed >> m) & 1));
        T vf[NS];
        if (use) factors(op.xg_terms[ka], vf);
        if (mn < op.nxg) fetch(mn);
        __syncthreads();  // cur is complete; the buffer written next was last read before this barrier
        if (use) {
          T qv[BC][R][NS];
#pragma unroll
          for (int q = 0; q < BC; ++q)
#pragma unroll
            for (int e = 0; e < NS; ++e) {
              T a[R];
              load_slices<T, R>(cur + q * qnr + (qo + i0[e]) * R, a);
#pragma unroll
              for (int s = 0; s < R; ++s) qv[q][s][e] = a[s];
            }
          term(op.xg_terms[ka], vf, qv);
          for (int kk = ka + 1; kk < kb; ++kk) {
            factors(op.xg_terms[kk], vf);
            term(op.xg_terms[kk], vf, qv);
          }
        }
        m = mn;
      }
    } else {
      const uint64_t rneed = act ? op.xqt_mask[A.DX.node_off[A.G.lx[g] - A.DX.lmin] + x] : 0;
      for (int m = 0; m < op.nxg; ++m) {
        if (!act || (m < 64 && !((rneed >> m) & 1))) continue;
        const T* qm = C.Qt + A.qt_off + int64_t(m) * ltotal + A.Gl.off[g];
        T qv[BC][R][NS];
#pragma unroll
        for (int q = 0; q < BC; ++q) {
          const int b = b0 + q < C.B ? b0 + q : b0;
          const T* qb = qm + int64_t(b) * C.qt_bstride + int64_t(x) * nvl * R;
#pragma unroll
          for (int e = 0; e < NS; ++e) {
            T a0[R], a1[R];
            load_slices<T, R>(qb + int64_t(i0[e]) * R, a0);
            if (!kPro) load_slices<T, R>(qb + int64_t(i1[e]) * R, a1);
#pragma unroll
            for (int s = 0; s < R; ++s) qv[q][s][e] = kPro ? a0[s] : w0[e] * a0[s] + w1[e] * a1[s];
          }
        }
        for (int kk = op.xg_start[m]; kk < op.xg_start[m + 1]; ++kk) {
          T vf[NS];
          factors(op.xg_terms[kk], vf);
          term(op.xg_terms[kk], vf, qv);
        }
      }
    }
  }
  if (!act) return;
#pragma unroll
  for (int q = 0; q < BC; ++q) {
    const int b = b0 + q;
    if (b >= C.B) break;
    T* yb = C.y + int64_t(b) * C.y_bstride + A.y_off + int64_t(R) * A.poff[g] + p;
#pragma unroll
    for (int s = 0; s < R; ++s) yb[int64_t(s) * plane] = acc[q][s];
  }
}

template <class T, int D, int R, int BC>
__global__ void __launch_bounds__(kSB) k_xstage(SplitCall<T> C) {
  constexpr int SS = D == 1 ? 3 : (D == 2 ? 7 : 15);
  int ii, vg;
  block_coords(C, ii, vg);
  const SplitItem it = C.items[ii];
  const int b0 = vg * BC;
  const ProbDesc& A = C.descs[it.prob];
  const int g = it.grid;
  const int nx = A.G.nx[g], nv = A.G.nv[g];
  const int64_t plane = int64_t(nx) * nv;
  const int64_t p = it.p0 + threadIdx.x;
  if (p >= plane) return;
  const int x = int(p / nv), v = int(p - int64_t(p / nv) * nv);
  const int lx = A.G.lx[g];
  const int64_t xlo = A.DX.lev_off[lx - A.DX.lmin];
  const DevOp& op = A.op;
  const int64_t total = A.G.off[A.G.n];
  int32_t nbx[SS];
#pragma unroll
  for (int e = 0; e < SS; ++e) nbx[e] = A.DX.tnbr[xlo + int64_t(e) * nx + x];
  T acc[BC][R];
#pragma unroll
  for (int q = 0; q < BC; ++q)
#pragma unroll
    for (int s = 0; s < R; ++s) acc[q][s] = T(0);
  // diagonal + lower partners: one x-stencil per X-group on the staged W.
  // A group whose factor row is zero here is skipped (its W^m is staged only
  // around the rows with a nonzero, which covers every slot of such a row).
  const uint64_t need = row_needs(A.DX, op, lx, x);
  for (int m = 0; m < op.nxg; ++m) {
    if (m < 64 && !((need >> m) & 1)) continue;
    T xf[SS];
    load_slot_pairs<T, SS>(qvals<T>(A.DX) + int64_t(op.xg_fac[m]) * A.DX.qfac_stride + A.DX.qlev_off[lx - A.DX.lmin],
                           nx, x, xf);
#pragma unroll
    for (int q = 0; q < BC; ++q) {
      const int b = b0 + q < C.B ? b0 + q : b0;
      const T* zb = C.Z + int64_t(b) * C.z_bstride + A.z_off + int64_t(m) * total + A.G.off[g] + int64_t(v) * R;
      T t[R];
#pragma unroll
      for (int s = 0; s < R; ++s) t[s] = T(0);
#pragma unroll
      for (int e = 0; e < SS; ++e) {
        T zz[R];
        load_slices<T, R>(zb + int64_t(nbx[e]) * nv * R, zz);
#pragma unroll
        for (int s = 0; s < R; ++s) t[s] += xf[e] * zz[s];
      }
#pragma unroll
      for (int s = 0; s < R; ++s) acc[q][s] += t[s];
    }
  }
#pragma unroll
  for (int q = 0; q < BC; ++q) {
    const int b = b0 + q;
    if (b >= C.B) break;
    T* yb = C.y + int64_t(b) * C.y_bstride + A.y_off + int64_t(R) * A.poff[g] + p;
#pragma unroll
    for (int s = 0; s < R; ++s) {
      if (C.x_assign) yb[int64_t(s) * plane] = acc[q][s];  // no upper-partner pass ran
      else yb[int64_t(s) * plane] += acc[q][s];            // after the upper-partner pass
    }
  }
}


// Pass 2 on tiles: a block owns t^d x-nodes times vb v-nodes and stages W^m
// on the tile plus a one-node x-halo in LDS (zero outside a non-periodic
// lattice), so each point's x-stencil reads come from LDS; the next group's
// halo is fetched into registers while the current one is computed.  Thread
// (xl, vl) = (tid / vb, tid % vb).  The stencil slots follow the lattice
// offsets of the Kuhn stencil, like the factor tables.
template <class T, int D, int R, int BC>
__global__ void __launch_bounds__(kSB) k_xtile(SplitCall<T> C) {
  constexpr int SS = D == 1 ? 3 : (D == 2 ? 7 : 15);
  constexpr int KS = kTileIters;
  extern __shared__ unsigned char split_smem[];
  T* sz = reinterpret_cast<T*>(split_smem);  // [BC][R][halo nodes][vb]
  int ii, vg;
  block_coords(C, ii, vg);
  const TileItem it = C.tiles[ii];
  const int b0 = vg * BC;
  const ProbDesc& A = C.descs[it.prob];
  const int g = it.grid;
  const int nx = A.G.nx[g], nv = A.G.nv[g];
  const int lx = A.G.lx[g];
  const int mx = A.mx[lx];
  const bool xper = A.xper != 0;
  const int64_t plane = int64_t(nx) * nv;
  const int64_t total = A.G.off[A.G.n];
  const int t = it.t, vb = it.vb, hw = t + 2;
  int hn = 1, tn = 1;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    hn *= hw;
    tn *= t;
  }
  const int hsz = hn * vb;  // staged values per (vector, slice)
  // this thread's output point
  const int xl = int(threadIdx.x) / vb, vl = int(threadIdx.x) - xl * vb;
  bool act = xl < tn && it.v0 + vl < nv;
  int x = 0, hb = 0;
  {
    int r = xl, lc[3] = {0, 0, 0};
#pragma unroll
    for (int a = D - 1; a >= 0; --a) {
      lc[a] = r % t;
      r /= t;
    }
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int c = it.x0[a] + lc[a];
      act = act && c < mx;
      x = x * mx + c;
      hb = hb * hw + lc[a] + 1;
    }
  }
  if (!act) x = 0;
  const int v = act ? it.v0 + vl : 0;
  int hoff[SS];
#pragma unroll
  for (int e = 0; e < SS; ++e) {
    int o = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) o = o * hw + A.off[e][a];
    hoff[e] = (hb + o) * vb + vl;
  }
  // staging: element w = h vb + wv of a (vector, slice) slab <- plane offset
  // node(h) nv + v0 + wv, or -1 (zero) outside the lattice
  int32_t goff[KS];
#pragma unroll
  for (int j = 0; j < KS; ++j) {
    const int w = int(threadIdx.x) + j * kSB;
    goff[j] = -1;
    if (w < hsz) {
      const int h = w / vb, vv = it.v0 + (w - h * vb);
      bool ok = vv < nv;
      int node = 0, r = h, c[3] = {0, 0, 0};
#pragma unroll
      for (int a = D - 1; a >= 0; --a) {
        c[a] = r % hw + it.x0[a] - 1;
        r /= hw;
      }
#pragma unroll
      for (int a = 0; a < D; ++a) {
        int cc = c[a];
        if (xper) cc = cc < 0 ? cc + mx : (cc >= mx ? cc - mx : cc);
        ok = ok && cc >= 0 && cc < mx;
        node = node * mx + cc;
      }
      if (ok) goff[j] = node * nv + vv;
    }
  }
  const int64_t xlo = A.DX.lev_off[lx - A.DX.lmin];
  const T* xv = vals<T>(A.DX);
  const DevOp& op = A.op;
  T pre[BC * R][KS];
  auto fetch = [&](int m) {
#pragma unroll
    for (int q = 0; q < BC; ++q) {
      const int b = b0 + q < C.B ? b0 + q : b0;
      const T* zb = C.Z + int64_t(b) * C.z_bstride + A.z_off + int64_t(m) * total + A.G.off[g];
#pragma unroll
      for (int j = 0; j < KS; ++j) {
        T zz[R];
        if (goff[j] >= 0) {
          load_slices<T, R>(zb + int64_t(goff[j]) * R, zz);
        } else {
#pragma unroll
          for (int s = 0; s < R; ++s) zz[s] = T(0);
        }
#pragma unroll
        for (int s = 0; s < R; ++s) pre[q * R + s][j] = zz[s];
      }
    }
  };
  // The group's x-factor values: for d = 3 (15 slots) the tile's nodes are
  // staged after the halo (element f = e tn + xi, slot e of tile node xi; -1
  // outside the lattice) and read from LDS; for d <= 2 each thread loads its
  // node's slots directly, which measured faster there.
  constexpr bool kFacLds = D == 3;
  T* sf = sz + BC * R * hsz;
  const int nf = SS * tn;
  int32_t fidx[kTileFacIters];
#pragma unroll
  for (int j = 0; j < kTileFacIters; ++j) {
    const int f = int(threadIdx.x) + j * kSB;
    fidx[j] = -1;
    if (kFacLds && f < nf) {
      const int e = f / tn, xi = f - e * tn;
      int r = xi, node = 0, lc[3] = {0, 0, 0};
      bool ok = true;
#pragma unroll
      for (int a = D - 1; a >= 0; --a) {
        lc[a] = r % t;
        r /= t;
      }
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const int c = it.x0[a] + lc[a];
        ok = ok && c < mx;
        node = node * mx + c;
      }
      if (ok) fidx[j] = e * nx + node;
    }
  }
  T fpre[kFacLds ? kTileFacIters : SS];
  auto ffetch = [&](int m) {
    const T* fp = xv + int64_t(op.xg_fac[m]) * A.DX.fac_stride + xlo;
    if constexpr (kFacLds) {
#pragma unroll
      for (int j = 0; j < kTileFacIters; ++j) fpre[j] = fidx[j] >= 0 ? fp[fidx[j]] : T(0);
    } else {  // slot-major direct loads: the pair loads measured slower here (one wave less per SIMD)
#pragma unroll
      for (int e = 0; e < SS; ++e) fpre[e] = fp[int64_t(e) * nx + x];
    }
  };
  T acc[BC][R];
#pragma unroll
  for (int q = 0; q < BC; ++q)
#pragma unroll
    for (int s = 0; s < R; ++s) acc[q][s] = T(0);
  // the tile's groups (it.gmask: groups with a nonzero factor row on the
  // tile); within one, a thread whose row of the factor is zero adds nothing
  // (the staged W^m of a partial group is valid only around its nonzero rows)
  const uint64_t rneed = act ? row_needs(A.DX, op, lx, x) : 0;
  auto gnext = [&](int m) {
    ++m;
    while (m < op.nxg && m < 64 && !((it.gmask >> m) & 1)) ++m;
    return m;
  };
  int m = gnext(-1);
  if (m < op.nxg) {
    fetch(m);
    ffetch(m);
  }
  while (m < op.nxg) {
    const int mn = gnext(m);
    __syncthreads();  // the previous group's reads are done
#pragma unroll
    for (int i = 0; i < BC * R; ++i)
#pragma unroll
      for (int j = 0; j < KS; ++j) {
        const int w = int(threadIdx.x) + j * kSB;
        if (w < hsz) sz[i * hsz + w] = pre[i][j];
      }
    T xc[SS];
    if constexpr (kFacLds) {
#pragma unroll
      for (int j = 0; j < kTileFacIters; ++j) {
        const int f = int(threadIdx.x) + j * kSB;
        if (f < nf) sf[f] = fpre[j];
      }
    } else {
#pragma unroll
      for (int e = 0; e < SS; ++e) xc[e] = fpre[e];
    }
    if (mn < op.nxg) {
      fetch(mn);
      ffetch(mn);
    }
    __syncthreads();
    if (act && (m >= 64 || ((rneed >> m) & 1))) {
      if constexpr (kFacLds) {
#pragma unroll
        for (int e = 0; e < SS; ++e) xc[e] = sf[e * tn + xl];
      }
#pragma unroll
      for (int q = 0; q < BC; ++q)
#pragma unroll
        for (int s = 0; s < R; ++s) {
          const T* l = sz + (q * R + s) * hsz;
          T a = T(0);
#pragma unroll
          for (int e = 0; e < SS; ++e) a += xc[e] * l[hoff[e]];
          acc[q][s] += a;
        }
    }
    m = mn;
  }
  if (!act) return;
  const int64_t p = int64_t(x) * nv + v;
#pragma unroll
  for (int q = 0; q < BC; ++q) {
    const int b = b0 + q;
    if (b >= C.B) break;
    T* yb = C.y + int64_t(b) * C.y_bstride + A.y_off + int64_t(R) * A.poff[g] + p;
#pragma unroll
    for (int s = 0; s < R; ++s) {
      if (C.x_assign) yb[int64_t(s) * plane] = acc[q][s];  // no upper-partner pass ran
      else yb[int64_t(s) * plane] += acc[q][s];            // after the upper-partner pass
    }
  }
}

}  // namespace

int split_points_per_item() { return kSB; }
int split_default_bc(int d) { return d == 3 ? 1 : 2; }
// Tile edge t (x-nodes per axis) and v-run vb: every thread owns one point
// (t^d vb <= kSB), the halo box fits the staging registers ((t+2)^d vb <=
// kTileIters kSB), and among those the shape with the fewest thread slots plus
// staged in-lattice values wins.
void split_tile_shape(int d, int mx, int nv, int& t_out, int& vb_out) {
  auto inlat = [&](int t) {  // in-lattice halo coordinates over the tiles of one axis
    int64_t s = 0;
    for (int x0 = 0; x0 < mx; x0 += t) s += std::min(x0 + t + 1, mx) - std::max(x0 - 1, 0);
    return s;
  };
  double best = -1;
  t_out = 1;
  vb_out = std::min(nv, kSB);
  const int cand[] = {8, 16, 32, 64, nv};
  for (int t = 1; t <= std::min(mx, 16); ++t) {
    int64_t td = 1, hd = 1, il = 1;
    for (int a = 0; a < d; ++a) {
      td *= t;
      hd *= t + 2;
      il *= inlat(t);
    }
    for (int vb : cand) {
      const int ss = d == 1 ? 3 : (d == 2 ? 7 : 15);
      if (vb > nv || (vb == nv && nv > 64) || td * vb > kSB || hd * vb > int64_t(kTileIters) * kSB ||
          td * ss > int64_t(kTileFacIters) * kSB)
        continue;
      int64_t ntx = (mx + t - 1) / t, nt = (nv + vb - 1) / vb;
      for (int a = 0; a < d; ++a) nt *= ntx;
      const double cost = double(nt) * kSB + double(il) * nv;
      if (best < 0 || cost < best) {
        best = cost;
        t_out = t;
        vb_out = vb;
      }
    }
  }
}
bool split_vmajor() {
  const char* v = getenv("SGDG_SPLIT_ORDER");
  return v && atoi(v) == 1;
}
int split_xcd() {
  const char* v = getenv("SGDG_SPLIT_XCD");
  return v && atoi(v) == 1 ? 1 : 0;
}

// LDS budgets of the upper-partner staging and of the x-stencil tiles (about a
// quarter of a CU's LDS, so several blocks share a CU); beyond them the
// per-point kernels read from memory
constexpr size_t kQLdsMax = 32 * 1024;
constexpr size_t kTileLdsMax = 40 * 1024;

template <class T>
void split_stage(const SplitCall<T>& C, int d, int R, int bc, int stage, hipStream_t s) {
  if (C.nitems == 0) return;
  if (d == 3 || (bc != 1 && bc != 2 && bc != 4)) bc = d == 3 ? 1 : 2;
  size_t lds = 2 * size_t(C.max_qn) * R * bc * sizeof(T);  // two buffers
  const bool ql = stage == 1 && d <= 2 && C.max_qn > 0 && C.max_qn <= kQlIters * kSB && lds <= kQLdsMax;
  if (!ql) lds = 0;
  const size_t tlds = (size_t(C.max_tile) * R * bc + (d == 3 ? size_t(kTileFacIters) * kSB : 0)) * sizeof(T);
  const bool tiles = stage == 2 && C.ntiles > 0 && bc <= 2 && C.max_tile <= kTileIters * kSB && tlds <= kTileLdsMax;
  if (tiles) {
    const dim3 tgrid(unsigned(C.ntiles), unsigned((C.B + bc - 1) / bc));
#define SGDG_TILE_CASE(DD, RR, BB)                                                                 \
    if (d == DD && R == RR && bc == BB) {                                                          \
      hipLaunchKernelGGL((k_xtile<T, DD, RR, BB>), tgrid, dim3(kSB), tlds, s, C);                  \
      SGDG_CHECK_HIP(hipGetLastError());                                                           \
      return;                                                                                      \
    }
#define SGDG_TILE_R(DD, BB) SGDG_TILE_CASE(DD, 1, BB) SGDG_TILE_CASE(DD, 2, BB) SGDG_TILE_CASE(DD, 3, BB)
    SGDG_TILE_R(1, 1) SGDG_TILE_R(1, 2) SGDG_TILE_R(2, 1) SGDG_TILE_R(2, 2) SGDG_TILE_R(3, 1)
#undef SGDG_TILE_R
#undef SGDG_TILE_CASE
  }
  dim3 grid(unsigned(C.nitems), unsigned((C.B + bc - 1) / bc));
#define SGDG_SPLIT_CASE(DD, RR, BB)                                                                 \
  if (d == DD && R == RR && bc == BB) {                                                             \
    if (stage == 0) hipLaunchKernelGGL((k_vstage<T, DD, RR, BB>), grid, dim3(kSB), 0, s, C);        \
    else if (stage == 1 && ql) hipLaunchKernelGGL((k_ustage<T, DD, RR, BB, true>), grid, dim3(kSB), lds, s, C); \
    else if (stage == 1) hipLaunchKernelGGL((k_ustage<T, DD, RR, BB, false>), grid, dim3(kSB), 0, s, C);   \
    else hipLaunchKernelGGL((k_xstage<T, DD, RR, BB>), grid, dim3(kSB), 0, s, C);                   \
    SGDG_CHECK_HIP(hipGetLastError());                                                              \
    return;                                                                                         \
  }
#define SGDG_SPLIT_R(DD, BB) SGDG_SPLIT_CASE(DD, 1, BB) SGDG_SPLIT_CASE(DD, 2, BB) SGDG_SPLIT_CASE(DD, 3, BB)
  SGDG_SPLIT_R(1, 1) SGDG_SPLIT_R(1, 2) SGDG_SPLIT_R(1, 4)
  SGDG_SPLIT_R(2, 1) SGDG_SPLIT_R(2, 2) SGDG_SPLIT_R(2, 4)
  SGDG_SPLIT_R(3, 1)
#undef SGDG_SPLIT_R
#undef SGDG_SPLIT_CASE
  throw Error{SGDG_E_ARG, "unsupported dimension or time degree"};
}

template void split_stage<double>(const SplitCall<double>&, int, int, int, int, hipStream_t);
template void split_stage<float>(const SplitCall<float>&, int, int, int, int, hipStream_t);

}  // namespace sgdg
