// The C ABI of libsgdg: layout, assembly/upload, operator application, the
// combination-technique preconditioner (Algorithm 1's body, Sect. 4.3), the
// strip right-hand side (eq:weak_form_j) and the flexible-GMRES strip solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <stdexcept>

#include "ops_internal.h"

using namespace sgdg;

// ------------------------------------------------------------------ errors --
namespace sgdg {
static thread_local std::string g_err = "no error";
void set_error(const std::string& m) { g_err = m; }

static std::atomic<uint64_t> g_alloc_epoch{0};
uint64_t alloc_epoch() { return g_alloc_epoch.load(); }

DevBuf::~DevBuf() {
  if (p) {
    (void)hipFree(p);
    ++g_alloc_epoch;
  }
}
void DevBuf::alloc(size_t b) {
  ++g_alloc_epoch;
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
  if (b == 0) return;
  if (hipMalloc(&p, b) != hipSuccess) {
    p = nullptr;
    throw Error{SGDG_E_ALLOC, "hipMalloc of " + std::to_string(b) + " bytes failed"};
  }
  bytes = b;
}
void DevBuf::ensure(size_t b) {
  if (b > bytes) {
    // work queued earlier may still use the old allocation
    if (p) SGDG_CHECK_HIP(hipDeviceSynchronize());
    alloc(b);
  }
}
}  // namespace sgdg

extern "C" const char* sgdg_last_error(void) { return g_err.c_str(); }

// -------------------------------------------------------------------- grid --
extern "C" sgdg_status sgdg_build_sparse_grid(const sgdg_domain* x, const sgdg_domain* v, int level_min,
                                              int level_max, int time_degree, sgdg_grid* out) {
  API_BEGIN
  require(x && v && out, "null argument");
  require(x->dim == v->dim && x->dim >= 1 && x->dim <= 3, "domains must share dim in 1..3");
  require(level_min >= 0 && level_min <= level_max && level_max <= 12, "levels must satisfy 0 <= min <= max <= 12");
  require(time_degree >= 0 && time_degree <= 2, "time degree must be 0..2");
  const int n_up = level_max - level_min + 1;
  require(n_up <= kMaxGrids / 2, "too many component grids");
  auto* g = new sgdg_grid_s;
  for (int side = 0; side < 2; ++side) {
    const sgdg_domain* s = side == 0 ? x : v;
    Dom& D = side == 0 ? g->x : g->v;
    D.d = s->dim;
    D.periodic = s->periodic != 0;
    for (int a = 0; a < 3; ++a) {
      D.lo[a] = s->lo[a];
      D.hi[a] = s->hi[a];
      if (a < s->dim && !(s->hi[a] > s->lo[a])) {
        delete g;
        throw Error{SGDG_E_ARG, "domain must have lo < hi on every axis"};
      }
    }
  }
  g->lmin = level_min;
  g->lmax = level_max;
  g->r = time_degree;
  g->R = time_degree + 1;
  const int S = level_max + level_min;
  for (int lx = level_min; lx <= level_max; ++lx) g->up.push_back({lx, S - lx, g->x.nodes(lx), g->v.nodes(S - lx)});
  for (int lx = level_min; lx < level_max; ++lx)
    g->low.push_back({lx, S - 1 - lx, g->x.nodes(lx), g->v.nodes(S - 1 - lx)});
  for (auto& d : g->up) g->up_pts += d.nx * d.nv;
  for (auto& d : g->low) g->low_pts += d.nx * d.nv;
  *out = g;
  API_END
}

extern "C" sgdg_status sgdg_grid_info(sgdg_grid g, int which, int* n_comp, int64_t* n_dof, int* lx, int* lv,
                                      int64_t* nx, int64_t* nv, int64_t* offset) {
  API_BEGIN
  require(g != nullptr, "null grid");
  require(which == 0 || which == 1, "which must be 0 (upper) or 1 (lower)");
  const auto& gs = which == 0 ? g->up : g->low;
  if (n_comp) *n_comp = int(gs.size());
  if (n_dof) *n_dof = which == 0 ? g->R * g->up_pts : g->low_pts;
  int64_t o = 0;
  for (size_t i = 0; i < gs.size(); ++i) {
    if (lx) lx[i] = gs[i].lx;
    if (lv) lv[i] = gs[i].lv;
    if (nx) nx[i] = gs[i].nx;
    if (nv) nv[i] = gs[i].nv;
    if (offset) offset[i] = o;
    o += gs[i].nx * gs[i].nv;
  }
  API_END
}

extern "C" void sgdg_grid_destroy(sgdg_grid g) { delete g; }

// --------------------------------------------------------------------- ops --
static void upload_domain(DomainData& D, DomDev& dd) {
  const int S = D.st.S;
  std::vector<int32_t> nbr, par, chi;
  std::vector<double> parw, chiw;
  DevDomain& d = dd.d;
  d.S = S;
  d.lmin = D.lmin;
  d.lmax = D.lmax;
  int64_t o = 0, po = 0;
  for (int l = D.lmin; l <= D.lmax; ++l) {
    const LevelTables& T = D.L(l);
    d.lev_off[l - D.lmin] = o;
    d.par_off[l - D.lmin] = po;
    nbr.insert(nbr.end(), T.nbr.begin(), T.nbr.end());
    if (l < D.lmax) {
      chi.insert(chi.end(), T.chi.begin(), T.chi.end());
      chiw.insert(chiw.end(), T.chiw.begin(), T.chiw.end());
    } else {
      chi.insert(chi.end(), size_t(T.n) * S, 0);
      chiw.insert(chiw.end(), size_t(T.n) * S, 0.0);
    }
    if (l > D.lmin) {
      par.insert(par.end(), T.par.begin(), T.par.end());
      parw.insert(parw.end(), T.parw.begin(), T.parw.end());
    } else {
      par.insert(par.end(), size_t(T.n) * 2, 0);
      parw.insert(parw.end(), size_t(T.n) * 2, 0.0);
    }
    d.lev_n[l - D.lmin] = T.n;
    o += T.n * S;
    po += T.n * 2;
  }
  d.nbr = upload(dd.nbr, nbr);
  // slot-major copies: entry e of consecutive nodes is contiguous.  off(l) is
  // the start of level l in a block of `stride` elements; K entries per node.
  // (the host loops below run on all cores: a field refresh repeats them per
  // fixed-point iteration)
  auto slot_major = [&](auto& dst, const auto& src, size_t nblocks, int64_t stride, int K, auto off) {
    dst.resize(src.size());
    for (size_t bk = 0; bk < nblocks; ++bk)
      for (int l = D.lmin; l <= D.lmax; ++l) {
        const int64_t n = D.L(l).n, base = int64_t(bk) * stride + off(l);
#pragma omp parallel for if (n >= 4096)
        for (int64_t i = 0; i < n; ++i)
          for (int e = 0; e < K; ++e) dst[base + int64_t(e) * n + i] = src[base + i * K + e];
      }
  };
  auto to_f32 = [](const std::vector<double>& a, std::vector<float>& b) {
    b.resize(a.size());
    const int64_t n = int64_t(a.size());
#pragma omp parallel for if (n >= 65536)
    for (int64_t i = 0; i < n; ++i) b[size_t(i)] = float(a[size_t(i)]);
  };
  auto loff = [&](int l) { return d.lev_off[l - D.lmin]; };
  {
    std::vector<int32_t> t;
    slot_major(t, nbr, 1, o, S, loff);
    d.tnbr = upload(dd.tnbr, t);
    std::vector<int32_t> tc;
    slot_major(tc, chi, 1, o, S, loff);
    d.tchi = upload(dd.tchi, tc);
    std::vector<double> tw;
    slot_major(tw, chiw, 1, o, S, loff);
    d.tchiw = upload(dd.tchiw, tw);
  }
  d.chi = upload(dd.chi, chi);
  d.chiw = upload(dd.chiw, chiw);
  d.par = upload(dd.par, par);
  d.parw = upload(dd.parw, parw);
  d.fac_stride = o;
  const size_t nf = D.factors.size();
  std::vector<double> vals(nf * o);
  std::vector<float> v32(nf * o);
  for (size_t f = 0; f < nf; ++f)
    for (int l = D.lmin; l <= D.lmax; ++l) {
      const auto& src = D.values[f][l - D.lmin];
      std::copy(src.begin(), src.end(), vals.begin() + f * o + d.lev_off[l - D.lmin]);
    }
  to_f32(vals, v32);
  d.vals = upload(dd.vals, vals);
  d.vals32 = upload(dd.vals32, v32);
  {
    int64_t no = 0;
    for (int l = D.lmin; l <= D.lmax; ++l) {
      d.node_off[l - D.lmin] = no;
      no += D.L(l).n;
    }
    d.node_stride = no;
    dd.hsup.assign(nf * size_t(no), 0);
    dd.hpartial.assign(nf, 0);
#pragma omp parallel for schedule(dynamic)
    for (size_t f = 0; f < nf; ++f) {
      uint8_t* sf = dd.hsup.data() + f * no;
      for (int l = D.lmin; l <= D.lmax; ++l) {
        const LevelTables& T = D.L(l);
        const auto& val = D.values[f][l - D.lmin];
        uint8_t* sl = sf + d.node_off[l - D.lmin];
        for (int64_t i = 0; i < T.n; ++i)
          for (int e = 0; e < S; ++e)
            if (val[size_t(i) * S + e] != 0.0) {
              sl[i] |= 1;
              sl[T.nbr[size_t(i) * S + e]] |= 2;
            }
      }
      // bit 2: the node is a stencil neighbour of a nonzero row (read by
      // the x-stencil of a row that has a nonzero)
      for (int l = D.lmin; l <= D.lmax; ++l) {
        const LevelTables& T = D.L(l);
        uint8_t* sl = sf + d.node_off[l - D.lmin];
        for (int64_t i = 0; i < T.n; ++i)
          if (sl[i] & 1)
            for (int e = 0; e < S; ++e) sl[T.nbr[size_t(i) * S + e]] |= 4;
      }
      for (int64_t i = 0; i < no; ++i)
        if ((sf[i] & 3) != 3) dd.hpartial[f] = 1;
    }
    d.sup = upload(dd.sup, dd.hsup);
    d.fpartial = upload(dd.fpartial, dd.hpartial);
  }
  {
    std::vector<double> t;
    slot_major(t, vals, nf, o, S, loff);
    std::vector<float> t32;
    to_f32(t, t32);
    d.tvals = upload(dd.tvals, t);
    d.tvals32 = upload(dd.tvals32, t32);
  }
  // restricted stencils
  const int W = int(D.woff.size());
  d.W = W;
  std::vector<int32_t> wide;
  int64_t wo = 0;
  for (int l = D.lmin; l <= D.lmax; ++l) {
    d.wlev_off[l - D.lmin] = wo;
    const int64_t n = D.L(l).n;
    if (l < D.lmax) wide.insert(wide.end(), D.wide_idx[l - D.lmin].begin(), D.wide_idx[l - D.lmin].end());
    else wide.insert(wide.end(), size_t(n) * W, 0);
    wo += n * W;
  }
  d.wide = upload(dd.wide, wide);
  d.rstride = wo;
  std::vector<double> rv(nf * wo, 0.0);
  for (size_t f = 0; f < nf; ++f)
    for (int l = D.lmin; l < D.lmax; ++l) {
      const auto& src = D.rvalues[f][l - D.lmin];
      std::copy(src.begin(), src.end(), rv.begin() + f * wo + d.wlev_off[l - D.lmin]);
    }
  std::vector<float> rv32;
  to_f32(rv, rv32);
  d.rvals = upload(dd.rvals, rv);
  d.rvals32 = upload(dd.rvals32, rv32);
  auto woff = [&](int l) { return d.wlev_off[l - D.lmin]; };
  std::vector<int32_t> tw;
  slot_major(tw, wide, 1, wo, W, woff);
  d.twide = upload(dd.twide, tw);
  std::vector<double> trv;
  slot_major(trv, rv, nf, wo, W, woff);
  std::vector<float> trv32;
  to_f32(trv, trv32);
  d.trvals = upload(dd.trvals, trv);
  d.trvals32 = upload(dd.trvals32, trv32);
  // prolongated stencils (already slot-major per level)
  int PW = 1;
  for (int a = 0; a < D.dom.d; ++a) PW *= 3;
  d.PW = PW;
  std::vector<int32_t> pidx;
  int64_t pof = 0;
  for (int l = D.lmin; l <= D.lmax; ++l) {
    d.plev_off[l - D.lmin] = pof;
    const int64_t n = D.L(l).n;
    if (l > D.lmin) pidx.insert(pidx.end(), D.pro_idx[l - D.lmin].begin(), D.pro_idx[l - D.lmin].end());
    else pidx.insert(pidx.end(), size_t(n) * PW, 0);
    pof += n * PW;
  }
  d.pidx = upload(dd.pidx, pidx);
  d.pstride = pof;
  std::vector<double> pv(nf * pof, 0.0);
  for (size_t f = 0; f < nf; ++f)
    for (int l = D.lmin + 1; l <= D.lmax; ++l) {
      const auto& src = D.pvalues[f][l - D.lmin];
      std::copy(src.begin(), src.end(), pv.begin() + f * pof + d.plev_off[l - D.lmin]);
    }
  std::vector<float> pv32;
  to_f32(pv, pv32);
  d.pvals = upload(dd.pvals, pv);
  d.pvals32 = upload(dd.pvals32, pv32);
  // slot-pair copies of the slot-major factor tables: [K/2][n][2] per level
  auto pair_major = [&](const std::vector<double>& src, size_t nblocks, int64_t stride, int K, const int64_t* off,
                        int64_t* qoff, int64_t& qstride, std::vector<double>& dst, std::vector<float>& dst32) {
    const int K2 = K + (K & 1);
    int64_t q = 0;
    for (int l = D.lmin; l <= D.lmax; ++l) {
      qoff[l - D.lmin] = q;
      q += D.L(l).n * K2;
    }
    qstride = q;
    dst.assign(nblocks * size_t(q), 0.0);
    for (size_t bk = 0; bk < nblocks; ++bk)
      for (int l = D.lmin; l <= D.lmax; ++l) {
        const int64_t n = D.L(l).n, sb = int64_t(bk) * stride + off[l - D.lmin];
        const int64_t qb = int64_t(bk) * q + qoff[l - D.lmin];
#pragma omp parallel for if (n >= 4096)
        for (int64_t i = 0; i < n; ++i)
          for (int e = 0; e < K; ++e) dst[qb + ((e >> 1) * n + i) * 2 + (e & 1)] = src[sb + int64_t(e) * n + i];
      }
    to_f32(dst, dst32);
  };
  {
    std::vector<double> tq;
    std::vector<float> tq32;
    std::vector<double> t(nf * o);
    slot_major(t, vals, nf, o, S, loff);
    pair_major(t, nf, o, S, d.lev_off, d.qlev_off, d.qfac_stride, tq, tq32);
    d.qvals = upload(dd.qvals, tq);
    d.qvals32 = upload(dd.qvals32, tq32);
    std::vector<double> pq;
    std::vector<float> pq32;
    pair_major(pv, nf, pof, PW, d.plev_off, d.qplev_off, d.qpstride, pq, pq32);
    d.qpvals = upload(dd.qpvals, pq);
    d.qpvals32 = upload(dd.qpvals32, pq32);
    std::vector<double> rq;
    std::vector<float> rq32;
    pair_major(trv, nf, wo, W, d.wlev_off, d.qrlev_off, d.qrstride, rq, rq32);
    d.qrvals = upload(dd.qrvals, rq);
    d.qrvals32 = upload(dd.qrvals32, rq32);
  }
}

static void upload_op(OpDev& od, const DomainData& X, const DomDev& dx) {
  const TermList& L = od.host;
  std::vector<int> xf, vf, vg, xg, vgf, xgf;
  std::vector<double> tm;
  std::vector<float> tm32;
  for (const Term& t : L.terms) {
    xf.push_back(t.xf);
    vf.push_back(t.vf);
    auto iv = std::find(vgf.begin(), vgf.end(), t.vf);
    if (iv == vgf.end()) {
      vgf.push_back(t.vf);
      iv = vgf.end() - 1;
    }
    vg.push_back(int(iv - vgf.begin()));
    auto ix = std::find(xgf.begin(), xgf.end(), t.xf);
    if (ix == xgf.end()) {
      xgf.push_back(t.xf);
      ix = xgf.end() - 1;
    }
    xg.push_back(int(ix - xgf.begin()));
    for (int i = 0; i < L.Rout * L.Rin; ++i) {
      tm.push_back(t.tm[i]);
      tm32.push_back(float(t.tm[i]));
    }
  }
  std::vector<int> vgt, vgs(vgf.size() + 1, 0), xgt, xgs(xgf.size() + 1, 0);
  for (size_t j = 0; j < vgf.size(); ++j) {
    vgs[j] = int(vgt.size());
    for (size_t k = 0; k < vg.size(); ++k)
      if (vg[k] == int(j)) vgt.push_back(int(k));
  }
  vgs[vgf.size()] = int(vgt.size());
  for (size_t m = 0; m < xgf.size(); ++m) {
    xgs[m] = int(xgt.size());
    for (size_t k = 0; k < xg.size(); ++k)
      if (xg[k] == int(m)) xgt.push_back(int(k));
  }
  xgs[xgf.size()] = int(xgt.size());
  std::vector<int> xgk(xgt.size());  // X-group of the term at each position of the X-group order
  for (size_t m = 0; m < xgf.size(); ++m)
    for (int kk = xgs[m]; kk < xgs[m + 1]; ++kk) xgk[size_t(kk)] = int(m);
  DevOp& op = od.op;
  op.xg_of = upload(od.xgk, xgk);
  op.vg_terms = upload(od.vgt, vgt);
  op.vg_start = upload(od.vgs, vgs);
  op.xg_terms = upload(od.xgt, xgt);
  op.xg_start = upload(od.xgs, xgs);
  op.Rin = L.Rin;
  op.Rout = L.Rout;
  op.nterms = int(L.terms.size());
  op.nvg = int(vgf.size());
  op.nxg = int(xgf.size());
  op.term_xf = upload(od.xf, xf);
  op.term_vf = upload(od.vf, vf);
  op.term_vg = upload(od.vg, vg);
  op.term_xg = upload(od.xg, xg);
  op.term_tm = upload(od.tm, tm);
  op.term_tm32 = upload(od.tm32, tm32);
  op.vg_fac = upload(od.vgf, vgf);
  op.xg_fac = upload(od.xgf, xgf);
  od.hxgf = xgf;
  // per x-node masks of the X-groups (bit m for m < 64): the node's row of
  // the group's factor has a nonzero; the x-stencil of such a row reads the node
  const int64_t no = dx.d.node_stride;
  std::vector<uint64_t> rowm(size_t(no), 0), readm(size_t(no), 0);
  for (size_t m = 0; m < xgf.size() && m < 64; ++m) {
    const size_t f = size_t(xgf[m]);
    const uint64_t bit = uint64_t(1) << m;
    for (int64_t i = 0; i < no; ++i) {
      const uint8_t sp = dx.hsup[f * size_t(no) + size_t(i)];
      if (!dx.hpartial[f] || (sp & 1)) rowm[size_t(i)] |= bit;
      if (!dx.hpartial[f] || (sp & 4)) readm[size_t(i)] |= bit;
    }
  }
  // the upper-partner arrays Qt^m at x-level l restrict the level-(l+1)
  // product X_m u and Qt^m of level l + 1: they can be nonzero only at the
  // embedding parents of the level-(l+1) nodes where either can be
  std::vector<uint64_t> qm(size_t(no), 0);
  for (int l = X.lmax - 1; l >= X.lmin; --l) {
    const LevelTables& F = X.L(l + 1);
    const int64_t fo = dx.d.node_off[l + 1 - X.lmin], co = dx.d.node_off[l - X.lmin];
    for (int64_t f = 0; f < F.n; ++f) {
      const uint64_t src = rowm[size_t(fo + f)] | qm[size_t(fo + f)];
      for (int j = 0; j < 2; ++j)
        if (F.parw[size_t(f) * 2 + j] != 0.0) qm[size_t(co + F.par[size_t(f) * 2 + j])] |= src;
    }
  }
  // the lower-partner arrays Pt^j at x-level l are read by the v-stage at the
  // embedding parents of the level-(l+1) rows that stage a term of v-group j,
  // and by the next scan step at the parents of its own rows: they are needed
  // only at the parents of the nodes where either holds
  std::vector<uint64_t> rj(size_t(no), 0), pm(size_t(no), 0);
  for (size_t k = 0; k < vg.size(); ++k) {
    if (vg[k] >= 64) continue;
    const uint64_t bj = uint64_t(1) << vg[k];
    for (int64_t i = 0; i < no; ++i)
      if (xg[k] >= 64 || ((readm[size_t(i)] >> xg[k]) & 1)) rj[size_t(i)] |= bj;
  }
  for (int l = X.lmax - 1; l >= X.lmin; --l) {
    const LevelTables& F = X.L(l + 1);
    const int64_t fo = dx.d.node_off[l + 1 - X.lmin], co = dx.d.node_off[l - X.lmin];
    for (int64_t f = 0; f < F.n; ++f) {
      // both parent slots, a zero-weight one included: the readers load both
      const uint64_t src = rj[size_t(fo + f)] | pm[size_t(fo + f)];
      for (int j = 0; j < 2; ++j) pm[size_t(co + F.par[size_t(f) * 2 + j])] |= src;
    }
  }
  op.xrow_mask = upload(od.xrowm, rowm);
  op.xread_mask = upload(od.xreadm, readm);
  op.xqt_mask = upload(od.xqtm, qm);
  op.xpt_mask = upload(od.xptm, pm);
  od.hxrowm = rowm;
  od.hxreadm = readm;
  od.hxqtm = qm;
  od.hxgs = xgs;
}

static void invert_small(int R, const double* A, double* inv) {
  double a[9], b[9];
  std::memcpy(a, A, sizeof(double) * R * R);
  for (int i = 0; i < R * R; ++i) b[i] = 0;
  for (int i = 0; i < R; ++i) b[i * R + i] = 1;
  for (int c = 0; c < R; ++c) {
    int piv = c;
    for (int i = c + 1; i < R; ++i)
      if (std::fabs(a[i * R + c]) > std::fabs(a[piv * R + c])) piv = i;
    for (int k = 0; k < R; ++k) {
      std::swap(a[c * R + k], a[piv * R + k]);
      std::swap(b[c * R + k], b[piv * R + k]);
    }
    const double d = a[c * R + c];
    if (d == 0.0) throw Error{SGDG_E_STATE, "singular time block"};
    for (int k = 0; k < R; ++k) {
      a[c * R + k] /= d;
      b[c * R + k] /= d;
    }
    for (int i = 0; i < R; ++i)
      if (i != c) {
        const double f = a[i * R + c];
        for (int k = 0; k < R; ++k) {
          a[i * R + k] -= f * a[c * R + k];
          b[i * R + k] -= f * b[c * R + k];
        }
      }
  }
  std::memcpy(inv, b, sizeof(double) * R * R);
}

static void check_problem(const sgdg_grid g, const sgdg_problem* p) {
  require(p->dt > 0 && p->delta >= 0, "dt must be > 0 and delta >= 0");
  const int d = g->x.d;
  for (int c = 0; c < 2 * d; ++c)
    if (p->beta[c]) {
      require(p->beta[c]->n_xf >= 0 && p->beta[c]->n_vf >= 0 && p->beta[c]->n_xf <= 2 && p->beta[c]->n_vf <= 2,
              "each beta component may carry at most two field factors per domain");
      for (int i = 0; i < p->beta[c]->n_xf; ++i) require(p->beta[c]->xf[i] != nullptr, "null field");
      for (int i = 0; i < p->beta[c]->n_vf; ++i) require(p->beta[c]->vf[i] != nullptr, "null field");
    }
  require(p->n_sigma >= 0 && p->n_sigma <= 8, "n_sigma must be 0..8");
  for (int t = 0; t < p->n_sigma; ++t)
    require(p->sigma[t].n_xf >= 0 && p->sigma[t].n_vf >= 0 && p->sigma[t].n_xf <= 2 && p->sigma[t].n_vf <= 2,
            "each sigma term may carry at most two field factors per domain");
}

// Factor tables, term lists and uploads of one strip operator; `terms` fills
// the four term lists (registering the factors it uses).
template <class F>
static sgdg_ops assemble_ops(sgdg_grid g, double dt, double delta, F&& terms) {
  std::unique_ptr<sgdg_ops_s> o(new sgdg_ops_s);
  o->grid = g;
  SGDG_CHECK_HIP(hipGetDevice(&o->device));
  for (int side = 0; side < 2; ++side) {
    DomainData& D = side == 0 ? o->X : o->V;
    D.dom = side == 0 ? g->x : g->v;
    D.lmin = g->lmin;
    D.lmax = g->lmax;
    build_domain_tables(D);
  }
  TermList tl[4];
  terms(o->X, o->V, tl);
  // the plain mass factor drives the inner preconditioner
  FactorKey mk;
  mk.kind = kMass;
  o->dx.d.mass_fac = o->X.factor_id(mk);
  o->dv.d.mass_fac = o->V.factor_id(mk);
  assemble_all(o->X);
  assemble_all(o->V);
  const int mfx = o->dx.d.mass_fac, mfv = o->dv.d.mass_fac;
  upload_domain(o->X, o->dx);
  upload_domain(o->V, o->dv);
  o->dx.d.mass_fac = mfx;
  o->dv.d.mass_fac = mfv;
  for (int k = 0; k < 4; ++k) {
    o->ops[k].host = tl[k];
    upload_op(o->ops[k], o->X, o->dx);
  }
  // inner preconditioner time block (Tt + delta Ct + Gt)^-1
  const int R = g->R;
  double Mt[9], Tt[9], Ct[9], Gt[9], P[9];
  time_matrices(g->r, dt, Mt, Tt, Ct, Gt);
  for (int i = 0; i < R * R; ++i) P[i] = Tt[i] + delta * Ct[i] + Gt[i];
  invert_small(R, P, o->pinv);
  return o.release();
}

thread_local bool g_upload_inplace = false;

static bool same_terms(const TermList& a, const TermList& b) {
  if (a.Rin != b.Rin || a.Rout != b.Rout || a.terms.size() != b.terms.size()) return false;
  for (size_t i = 0; i < a.terms.size(); ++i) {
    const Term &s = a.terms[i], &t = b.terms[i];
    if (s.xf != t.xf || s.vf != t.vf) return false;
    for (int k = 0; k < kMaxR * kMaxR; ++k)
      if (s.tm[k] != t.tm[k]) return false;
  }
  return true;
}

bool refresh_fields(sgdg_ops o, const sgdg_problem& p) {
  check_problem(o->grid, &p);
  DomainData &X = o->X, &V = o->V;
  const size_t nfx = X.factors.size(), nfv = V.factors.size();
  bool vchanged = false;
  for (size_t i = 0; i < X.fields.size(); ++i)
    std::copy(X.field_src[i], X.field_src[i] + X.fields[i].size(), X.fields[i].begin());
  for (size_t i = 0; i < V.fields.size(); ++i) {
    const double* src = V.field_src[i];
    vchanged = vchanged || !std::equal(V.fields[i].begin(), V.fields[i].end(), src);
    std::copy(src, src + V.fields[i].size(), V.fields[i].begin());
  }
  // the term lists of the new values (a term whose kinked weight vanishes for
  // these fields is left out, which changes the structure)
  TermList tl[4];
  build_terms(X, V, p, o->grid->r, tl);
  if (X.factors.size() != nfx || V.factors.size() != nfv) return false;
  for (int k = 0; k < 4; ++k)
    if (!same_terms(tl[k], o->ops[k].host)) return false;
  assemble_all(X);
  if (vchanged) assemble_all(V);
  // the host-side masks that launch tables and cached batches are built from
  const auto masks = [&]() {
    std::vector<std::vector<uint64_t>> m;
    std::vector<uint64_t> s(o->dx.hsup.begin(), o->dx.hsup.end());
    s.insert(s.end(), o->dv.hsup.begin(), o->dv.hsup.end());
    m.push_back(s);
    for (int k = 0; k < 4; ++k) {
      const OpDev& od = o->ops[k];
      m.push_back(od.hxrowm);
      m.push_back(od.hxreadm);
      m.push_back(od.hxqtm);
    }
    return m;
  };
  const auto before = masks();
  const uint64_t epoch = alloc_epoch();
  {
    g_upload_inplace = true;
    struct Reset {
      ~Reset() { g_upload_inplace = false; }
    } reset;
    const int mfx = o->dx.d.mass_fac, mfv = o->dv.d.mass_fac;
    upload_domain(o->X, o->dx);
    if (vchanged) upload_domain(o->V, o->dv);
    o->dx.d.mass_fac = mfx;
    o->dv.d.mass_fac = mfv;
    for (int k = 0; k < 4; ++k) upload_op(o->ops[k], o->X, o->dx);
  }
  if (alloc_epoch() != epoch || masks() != before) {
    o->self.reset();
    o->replicas.clear();
  }
  return true;
}

extern "C" sgdg_status sgdg_assemble_1d_factors(sgdg_grid g, const sgdg_problem* p, sgdg_ops* out) {
  API_BEGIN
  require(g && p && out, "null argument");
  check_problem(g, p);
  *out = assemble_ops(g, p->dt, p->delta,
                      [&](DomainData& X, DomainData& V, TermList* tl) { build_terms(X, V, *p, g->r, tl); });
  API_END
}

extern "C" sgdg_status sgdg_assemble_factors_t(sgdg_grid g, const sgdg_problem_t* p, sgdg_ops* out) {
  API_BEGIN
  require(g && p && out && p->tau && p->weight && p->at, "null argument");
  require(p->m >= 1 && p->m <= 8, "m must be 1..8");
  double wsum = 0;
  for (int mu = 0; mu < p->m; ++mu) {
    require(p->tau[mu] >= -1.0 && p->tau[mu] <= 1.0, "quadrature points must lie in [-1, 1]");
    check_problem(g, &p->at[mu]);
    require(p->at[mu].dt == p->at[0].dt && p->at[mu].delta == p->at[0].delta,
            "dt and delta must agree at every quadrature point");
    wsum += p->weight[mu];
  }
  require(std::fabs(wsum - 2.0) <= 1e-12, "quadrature weights must sum to 2 (the reference interval [-1, 1])");
  *out = assemble_ops(g, p->at[0].dt, p->at[0].delta, [&](DomainData& X, DomainData& V, TermList* tl) {
    build_terms_t(X, V, p->at, p->tau, p->weight, p->m, g->r, tl);
  });
  API_END
}

extern "C" void sgdg_ops_destroy(sgdg_ops o) {
  if (!o) return;
  for (sgdg_net n : o->nets) net_detach(n);  // networks outliving their problem become unusable, not dangling
  delete o;
}

