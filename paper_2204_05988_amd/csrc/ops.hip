// The C ABI of libsgdg: layout, assembly/upload, operator application, the
// combination-technique preconditioner (Algorithm 1's body, Sect. 4.3), the
// strip right-hand side (eq:weak_form_j) and the flexible-GMRES strip solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <stdexcept>

#include "fused.h"
#include "kernels.h"
#include "sgdg_internal.h"

using namespace sgdg;

// ------------------------------------------------------------------ errors --
namespace sgdg {
static thread_local std::string g_err = "no error";
void set_error(const std::string& m) { g_err = m; }

DevBuf::~DevBuf() {
  if (p) (void)hipFree(p);
}
void DevBuf::alloc(size_t b) {
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

#define API_BEGIN try {
#define API_END                                          \
  }                                                      \
  catch (const Error& e) {                               \
    set_error(e.msg);                                    \
    return e.code;                                       \
  }                                                      \
  catch (const std::bad_alloc&) {                        \
    set_error("host allocation failed");                 \
    return SGDG_E_ALLOC;                                 \
  }                                                      \
  catch (const std::exception& e) {                      \
    set_error(e.what());                                 \
    return SGDG_E_STATE;                                 \
  }                                                      \
  return SGDG_OK;

static void require(bool ok, const std::string& msg) {
  if (!ok) throw Error{SGDG_E_ARG, msg};
}

template <class T>
static T* ptr(const DevBuf& b) {
  return static_cast<T*>(b.p);
}

template <class T>
static T* upload(DevBuf& b, const std::vector<T>& h) {
  b.alloc(h.size() * sizeof(T));
  if (!h.empty()) SGDG_CHECK_HIP(hipMemcpy(b.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return ptr<T>(b);
}

// -------------------------------------------------------------------- grid --
struct GridDesc {
  int lx, lv;
  int64_t nx, nv;
};

struct sgdg_grid_s {
  Dom x, v;
  int lmin = 0, lmax = 0, r = 0, R = 1;
  std::vector<GridDesc> up, low;
  int64_t up_pts = 0, low_pts = 0;

  DevGrids make(const std::vector<GridDesc>& gs, int R_, int first = 0, int count = -1) const {
    DevGrids G;
    if (count < 0) count = int(gs.size()) - first;
    G.n = count;
    G.R = R_;
    int64_t o = 0;
    for (int i = 0; i < count; ++i) {
      const GridDesc& d = gs[first + i];
      G.lx[i] = d.lx;
      G.lv[i] = d.lv;
      G.nx[i] = int(d.nx);
      G.nv[i] = int(d.nv);
      G.off[i] = o;
      o += int64_t(R_) * d.nx * d.nv;
    }
    G.off[count] = o;
    return G;
  }
  // upper then lower grids in one set (the combination-technique grid problems)
  DevGrids make_ct(int R_) const {
    std::vector<GridDesc> all = up;
    all.insert(all.end(), low.begin(), low.end());
    return make(all, R_);
  }
};

static GridPts points_of(const DevGrids& G) {
  GridPts P;
  int64_t o = 0;
  for (int g = 0; g < G.n; ++g) {
    P.poff[g] = o;
    o += int64_t(G.nx[g]) * G.nv[g];
  }
  P.poff[G.n] = o;
  return P;
}

static Segs segs_of(const DevGrids& G) {
  Segs S;
  S.n = G.n;
  for (int g = 0; g <= G.n; ++g) S.off[g] = G.off[g];
  return S;
}

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
struct DomDev {
  DevBuf nbr, par, parw, chi, chiw, vals, vals32, wide, rvals, rvals32;
  DevDomain d;
};

struct OpDev {
  TermList host;
  DevBuf xf, vf, vg, xg, tm, tm32, vgf, xgf, vgt, vgs, xgt, xgs;
  DevOp op;
};

// Box tiling of a grid set for the fused kernel (cached per set and precision).
struct ItemTable {
  DevBuf buf;
  int n = 0;
  int max_stage = 0;
  int max_tab = 0;
};

template <class T>
struct Work {  // scratch of one precision
  DevBuf Pt, Qt;              // partner-sum scans on the lower diagonal
  DevBuf ctb, ctx, ctw, cttmp, ctV, ctin;  // CT inner solves
  DevBuf r32, z32, a32, b32;  // conversions
};

struct sgdg_ops_s {
  sgdg_grid grid = nullptr;
  DomainData X, V;
  DomDev dx, dv;
  OpDev ops[4];
  double pinv[kMaxR * kMaxR] = {};
  DevBuf pinv_dev;
  int device = 0;
  Work<double> w64;
  Work<float> w32;
  // GMRES state buffers: [0] grid problems (inner), [1] strip FGMRES (outer), [2] norms
  struct GBufs {
    DevBuf H, cs, sn, g, bn, beta, act, k, hc, inv, y, partial;
  } gb[3];
  // outer FGMRES
  DevBuf fV, fZ, fw, fr, fe, fb, ftmp;
  // rhs
  DevBuf rhs_a, rhs_b, rhs_c, rhs_d, rhs_w;
  int64_t inner_iters = 0;
  std::map<std::string, std::unique_ptr<ItemTable>> items;
  // event timing of the operator kernels: slot 0 level scans, 1 fused tiles, 2 unused
  bool prof = false;
  struct Ev {
    hipEvent_t a, b;
    int slot;
  };
  std::vector<Ev> events;
  double prof_ms[3] = {0, 0, 0};
  int64_t prof_n[3] = {0, 0, 0};
  ~sgdg_ops_s() {
    for (auto& e : events) {
      (void)hipEventDestroy(e.a);
      (void)hipEventDestroy(e.b);
    }
  }
};

// Records an event pair around `launch` when profiling is on.
template <class F>
static void timed(sgdg_ops o, int slot, hipStream_t s, F&& launch) {
  if (!o->prof) {
    launch();
    return;
  }
  sgdg_ops_s::Ev e;
  e.slot = slot;
  SGDG_CHECK_HIP(hipEventCreate(&e.a));
  SGDG_CHECK_HIP(hipEventCreate(&e.b));
  SGDG_CHECK_HIP(hipEventRecord(e.a, s));
  launch();
  SGDG_CHECK_HIP(hipEventRecord(e.b, s));
  o->events.push_back(e);
}

static void drain_events(sgdg_ops o) {
  for (auto& e : o->events) {
    SGDG_CHECK_HIP(hipEventSynchronize(e.b));
    float ms = 0;
    SGDG_CHECK_HIP(hipEventElapsedTime(&ms, e.a, e.b));
    o->prof_ms[e.slot] += ms;
    o->prof_n[e.slot] += 1;
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  o->events.clear();
}

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
    o += T.n * S;
    po += T.n * 2;
  }
  d.nbr = upload(dd.nbr, nbr);
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
  for (size_t i = 0; i < vals.size(); ++i) v32[i] = float(vals[i]);
  d.vals = upload(dd.vals, vals);
  d.vals32 = upload(dd.vals32, v32);
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
  std::vector<float> rv32(rv.size());
  for (size_t i = 0; i < rv.size(); ++i) rv32[i] = float(rv[i]);
  d.rvals = upload(dd.rvals, rv);
  d.rvals32 = upload(dd.rvals32, rv32);
}

static void upload_op(OpDev& od) {
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
  DevOp& op = od.op;
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

extern "C" sgdg_status sgdg_assemble_1d_factors(sgdg_grid g, const sgdg_problem* p, sgdg_ops* out) {
  API_BEGIN
  require(g && p && out, "null argument");
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
  build_terms(o->X, o->V, *p, g->r, tl);
  // the plain mass factor drives the inner preconditioner
  FactorKey mk;
  mk.kind = kMass;
  o->dx.d.mass_fac = o->X.factor_id(mk);
  o->dv.d.mass_fac = o->V.factor_id(mk);
  for (int side = 0; side < 2; ++side) {
    DomainData& D = side == 0 ? o->X : o->V;
    D.values.assign(D.factors.size(), {});
    D.rvalues.assign(D.factors.size(), {});
    build_wide_tables(D);
#pragma omp parallel for schedule(dynamic)
    for (int f = 0; f < int(D.factors.size()); ++f) {
      assemble_factor(D, f);
      restrict_factor(D, f);
    }
  }
  const int mfx = o->dx.d.mass_fac, mfv = o->dv.d.mass_fac;
  upload_domain(o->X, o->dx);
  upload_domain(o->V, o->dv);
  o->dx.d.mass_fac = mfx;
  o->dv.d.mass_fac = mfv;
  for (int k = 0; k < 4; ++k) {
    o->ops[k].host = tl[k];
    upload_op(o->ops[k]);
  }
  // inner preconditioner time block (Tt + delta Ct + Gt)^-1
  const int R = g->R;
  double Mt[9], Tt[9], Ct[9], Gt[9], P[9];
  time_matrices(g->r, p->dt, Mt, Tt, Ct, Gt);
  for (int i = 0; i < R * R; ++i) P[i] = Tt[i] + p->delta * Ct[i] + Gt[i];
  invert_small(R, P, o->pinv);
  std::vector<double> pv(o->pinv, o->pinv + R * R);
  upload(o->pinv_dev, pv);
  *out = o.release();
  API_END
}

extern "C" void sgdg_ops_destroy(sgdg_ops o) { delete o; }

// ------------------------------------------------------------- apply ------
template <class T>
static Work<T>& work(sgdg_ops o);
template <>
Work<double>& work<double>(sgdg_ops o) { return o->w64; }
template <>
Work<float>& work<float>(sgdg_ops o) { return o->w32; }

// Box shape of one grid for the fused kernel: x-box and v-box sizes per axis,
// at most fused_points_per_block() outputs and a bounded LDS stage.
static void choose_boxes(int d, int mx, int mv, int R, int elem, int* xs, int* vs) {
  const int nthr = fused_threads(), rows = fused_rows_per_thread();
  const int bx = d == 1 ? 32 : (d == 2 ? 8 : 4);
  const size_t lds_cap = 60 * 1024;
  for (int a = 0; a < 3; ++a) {
    xs[a] = a < d ? std::min(bx, mx) : 1;
    vs[a] = 1;
  }
  auto fits = [&](const int* v) {
    size_t nvb = 1, nvh = 1, nxh = 1, nx = 1;
    for (int a = 0; a < d; ++a) {
      nvb *= v[a];
      nvh *= v[a] + 2;
      nxh *= xs[a] + 2;
      nx *= xs[a];
    }
    if (nvb > size_t(nthr)) return false;
    if (nx > size_t(rows) * (nthr / nvb)) return false;
    const size_t st = std::max(nxh * nvb, nx * nvh) * size_t(R) * elem;
    const size_t tab = (nxh + 2 * nx + 2 * nvb + nvh) * sizeof(int);
    return st + tab <= lds_cap;
  };
  // grow the v-box, fastest axis first, by doubling
  bool grew = true;
  while (grew) {
    grew = false;
    for (int a = d - 1; a >= 0; --a) {
      if (vs[a] >= mv) continue;
      int t[3] = {vs[0], vs[1], vs[2]};
      t[a] = std::min(mv, vs[a] * 2);
      if (fits(t)) {
        vs[a] = t[a];
        grew = true;
      }
    }
  }
}

static ItemTable& item_table(sgdg_ops o, const std::string& key, const DevGrids& G, int elem) {
  auto it = o->items.find(key);
  if (it != o->items.end()) return *it->second;
  auto tab = std::make_unique<ItemTable>();
  std::vector<FusedItem> items;
  const int d = o->X.dom.d;
  int max_stage = 1, max_tab = 1;
  for (int g = 0; g < G.n; ++g) {
    const int mx = o->X.dom.axis_nodes(G.lx[g]), mv = o->V.dom.axis_nodes(G.lv[g]);
    int xs[3], vs[3];
    choose_boxes(d, mx, mv, G.R, elem, xs, vs);
    int nbx[3] = {1, 1, 1}, nbv[3] = {1, 1, 1};
    int64_t nx_h = 1, nv_b = 1, nx_b = 1, nv_h = 1;
    for (int a = 0; a < d; ++a) {
      nbx[a] = (mx + xs[a] - 1) / xs[a];
      nbv[a] = (mv + vs[a] - 1) / vs[a];
      nx_h *= xs[a] + 2;
      nx_b *= xs[a];
      nv_b *= vs[a];
      nv_h *= vs[a] + 2;
    }
    max_stage = std::max<int64_t>(max_stage, std::max(nx_h * nv_b, nx_b * nv_h) * G.R);
    max_tab = std::max<int64_t>(max_tab, nx_h + 2 * nx_b + 2 * nv_b + nv_h);
    for (int i0 = 0; i0 < nbx[0]; ++i0)
      for (int i1 = 0; i1 < nbx[1]; ++i1)
        for (int i2 = 0; i2 < nbx[2]; ++i2)
          for (int j0 = 0; j0 < nbv[0]; ++j0)
            for (int j1 = 0; j1 < nbv[1]; ++j1)
              for (int j2 = 0; j2 < nbv[2]; ++j2) {
                FusedItem f{};
                f.grid = g;
                const int ix[3] = {i0, i1, i2}, iv[3] = {j0, j1, j2};
                for (int a = 0; a < 3; ++a) {
                  f.xb[a] = a < d ? ix[a] * xs[a] : 0;
                  f.xs[a] = a < d ? std::min(xs[a], mx - f.xb[a]) : 1;
                  f.vb[a] = a < d ? iv[a] * vs[a] : 0;
                  f.vs[a] = a < d ? std::min(vs[a], mv - f.vb[a]) : 1;
                }
                items.push_back(f);
              }
  }
  upload(tab->buf, items);
  tab->n = int(items.size());
  tab->max_stage = max_stage;
  tab->max_tab = max_tab;
  ItemTable& ref = *tab;
  o->items[key] = std::move(tab);
  return ref;
}

// y = Op u on grid set G (G.R == op.Rin).  With full coupling the partner sums
// of the lower diagonal Gl are scanned first; diag_only applies the blocks A_{l,l}.
template <class T>
static void apply_on(sgdg_ops o, const DevOp& op, const DevGrids& G, bool diag_only, const T* u, T* y, int B,
                     hipStream_t s, const char* set_name = "up") {
  Work<T>& w = work<T>(o);
  sgdg_grid g = o->grid;
  FusedArgs<T> A{};
  A.G = G;
  A.P = points_of(G);
  A.DX = o->dx.d;
  A.DV = o->dv.d;
  A.op = op;
  for (int l = 0; l < kMaxLevels; ++l) {
    A.mx[l] = g->x.axis_nodes(l);
    A.mv[l] = g->v.axis_nodes(l);
  }
  A.xper = g->x.periodic;
  A.vper = g->v.periodic;
  for (int e = 0; e < kMaxS; ++e)
    for (int a = 0; a < 3; ++a) A.off[e][a] = e < o->X.st.S ? o->X.st.off[e][a] : 0;
  const bool full = !diag_only && G.n > 1;
  A.diag_only = full ? 0 : 1;
  A.B = B;
  A.u = u;
  A.y = y;
  if (full) {
    A.Gl = g->make(g->low, G.R);
    const int64_t lt = A.Gl.off[A.Gl.n];
    w.Pt.ensure(sizeof(T) * std::max(1, op.nvg) * size_t(B) * lt);
    w.Qt.ensure(sizeof(T) * std::max(1, op.nxg) * size_t(B) * lt);
    A.Pt = ptr<T>(w.Pt);
    A.Qt = ptr<T>(w.Qt);
  }
  const std::string key = std::string(set_name) + "/R" + std::to_string(G.R) + "/e" + std::to_string(sizeof(T));
  ItemTable& tab = item_table(o, key, G, int(sizeof(T)));
  A.items = ptr<FusedItem>(tab.buf);
  A.nitems = tab.n;
  A.max_stage = tab.max_stage;
  A.max_tab = tab.max_tab;
  if (full) timed(o, 0, s, [&] { fused_scans<T>(A, o->X.dom.d, s); });
  timed(o, 1, s, [&] { fused_tiles<T>(A, o->X.dom.d, s); });
}

extern "C" sgdg_status sgdg_apply_operator(sgdg_ops o, int kind, const void* u_dev, void* y_dev, sgdg_dtype t,
                                           int batch, hipStream_t s) {
  API_BEGIN
  require(o != nullptr, "null ops");
  require(kind >= SGDG_OP_FULL && kind <= SGDG_OP_DATA_G, "unknown operator kind");
  require(u_dev && y_dev && u_dev != y_dev, "u and y must be distinct non-null device buffers");
  require(batch >= 1, "batch must be >= 1");
  require(t == SGDG_F64 || t == SGDG_F32, "dtype must be F64 or F32");
  const int idx = kind == SGDG_OP_FULL || kind == SGDG_OP_BLOCKDIAG ? 0 : kind - 1;
  const DevOp& op = o->ops[idx].op;
  const DevGrids G = o->grid->make(o->grid->up, op.Rin);
  const bool diag = kind == SGDG_OP_BLOCKDIAG;
  if (t == SGDG_F64)
    apply_on<double>(o, op, G, diag, static_cast<const double*>(u_dev), static_cast<double*>(y_dev), batch, s);
  else
    apply_on<float>(o, op, G, diag, static_cast<const float*>(u_dev), static_cast<float*>(y_dev), batch, s);
  API_END
}

// ------------------------------------------------------ batched GMRES -----
static int nchunks_of(const Segs& S) {
  int64_t mx = 1;
  for (int i = 0; i < S.n; ++i) mx = std::max<int64_t>(mx, S.off[i + 1] - S.off[i]);
  return int((mx + 4095) / 4096);
}

static GmresState gmres_state(sgdg_ops_s::GBufs& b, int nseg, int m) {
  b.H.ensure(sizeof(double) * nseg * (m + 1) * m);
  b.cs.ensure(sizeof(double) * nseg * m);
  b.sn.ensure(sizeof(double) * nseg * m);
  b.g.ensure(sizeof(double) * nseg * (m + 1));
  b.bn.ensure(sizeof(double) * nseg);
  b.beta.ensure(sizeof(double) * nseg);
  b.act.ensure(sizeof(int) * nseg);
  b.k.ensure(sizeof(int) * nseg);
  b.hc.ensure(sizeof(double) * nseg * (m + 1));
  b.inv.ensure(sizeof(double) * nseg);
  b.y.ensure(sizeof(double) * nseg * m);
  GmresState st;
  st.H = b.H.as<double>();
  st.cs = b.cs.as<double>();
  st.sn = b.sn.as<double>();
  st.g = b.g.as<double>();
  st.bnorm = b.bn.as<double>();
  st.beta = b.beta.as<double>();
  st.active = b.act.as<int>();
  st.kused = b.k.as<int>();
  st.hcol = b.hc.as<double>();
  st.inv = b.inv.as<double>();
  st.y = b.y.as<double>();
  st.m = m;
  return st;
}

// Right-preconditioned restarted GMRES on independent segments (the grid
// problems A_{l,l} dU_l = r_l), preconditioner x -> Minv(x) fixed and linear.
// Returns iterations; sets *nan if a segment produced a non-finite norm.
template <class T>
static int batched_gmres(sgdg_ops o, const Segs& S, std::function<void(const T*, T*)> A,
                         std::function<void(const T*, T*)> Minv, const T* b, T* x, T* V, T* w, T* tmp, int m,
                         int maxit, double tol, hipStream_t s, bool* nan) {
  const int nseg = S.n;
  const int64_t total = S.off[S.n];
  const int nch = nchunks_of(S);
  auto& gbuf = o->gb[0];
  gbuf.partial.ensure(sizeof(double) * nseg * nch * (m + 1));
  double* part = gbuf.partial.as<double>();
  GmresState st = gmres_state(gbuf, nseg, m);
  KernelsT<T>::fill(total, T(0), x, s);
  int it = 0;
  std::vector<int> act(nseg);
  *nan = false;
  for (int cycle = 0; it < maxit; ++cycle) {
    T* V0 = V;
    if (cycle == 0) {
      KernelsT<T>::copy(total, b, V0, s);
    } else {
      A(x, w);
      KernelsT<T>::copy(total, b, V0, s);
      KernelsT<T>::axpby(total, T(-1), w, T(1), V0, s);
    }
    KernelsT<T>::seg_norm2(S, V0, part, nch, s);
    gmres_start(nseg, st, part, nch, tol, cycle == 0, s);
    KernelsT<T>::seg_scale(S, V0, st.inv, V0, s);
    SGDG_CHECK_HIP(hipMemcpyAsync(act.data(), st.active, sizeof(int) * nseg, hipMemcpyDeviceToHost, s));
    SGDG_CHECK_HIP(hipStreamSynchronize(s));
    bool any = false;
    for (int a : act) {
      any = any || a == 1;
      *nan = *nan || a == -1;
    }
    if (!any) break;
    const int mm = std::min(m, maxit - it);
    int j = 0;
    for (; j < mm; ++j) {
      T* Vj = V + int64_t(j) * total;
      Minv(Vj, tmp);
      A(tmp, w);
      for (int pass = 0; pass < 2; ++pass) {
        KernelsT<T>::seg_dots(S, V, total, j + 1, w, part, nch, s);
        gmres_add_proj(nseg, st, part, nch, j, s);
        KernelsT<T>::seg_axpy_multi(S, V, total, j + 1, st.hcol, m + 1, w, -1.0, pass == 1 ? part : nullptr, nch, s);
      }
      gmres_givens(nseg, st, part, nch, j, tol, s);
      KernelsT<T>::seg_scale(S, w, st.inv, V + int64_t(j + 1) * total, s);
      if ((j + 1) % 8 == 0 && j + 1 < mm) {
        SGDG_CHECK_HIP(hipMemcpyAsync(act.data(), st.active, sizeof(int) * nseg, hipMemcpyDeviceToHost, s));
        SGDG_CHECK_HIP(hipStreamSynchronize(s));
        bool a1 = false;
        for (int a : act) a1 = a1 || a == 1;
        if (!a1) {
          ++j;
          break;
        }
      }
    }
    it += j;
    gmres_lsq(nseg, st, s);
    KernelsT<T>::fill(total, T(0), w, s);
    KernelsT<T>::seg_axpy_multi(S, V, total, j, st.y, m, w, 1.0, nullptr, nch, s);
    Minv(w, tmp);
    KernelsT<T>::axpby(total, T(1), tmp, T(1), x, s);
  }
  return it;
}

// --------------------------------------------------- CT preconditioner ----
template <class T>
static void ct_apply(sgdg_ops o, const T* r, T* z, const sgdg_precond_opts& po, hipStream_t s, bool* nan) {
  sgdg_grid g = o->grid;
  const int R = g->R;
  const DevGrids Gup = g->make(g->up, R);
  const DevGrids Glow = g->make(g->low, R);
  const DevGrids Gct = g->make_ct(R);
  const GridPts Pct = points_of(Gct);
  const int64_t nup = Gup.off[Gup.n], nlow = Glow.off[Glow.n], nct = Gct.off[Gct.n];
  Work<T>& w = work<T>(o);
  const int m = std::max(1, std::min(po.inner_restart, 64));
  w.ctb.ensure(sizeof(T) * nct);
  w.ctx.ensure(sizeof(T) * nct);
  w.ctw.ensure(sizeof(T) * nct);
  w.cttmp.ensure(sizeof(T) * nct);
  w.ctV.ensure(sizeof(T) * nct * (m + 1));
  T* b = ptr<T>(w.ctb);
  // residual on the upper grids, restricted in x to the lower grids (Algorithm 1)
  KernelsT<T>::copy(nup, r, b, s);
  KernelsT<T>::restrict_x(Glow, Gup, o->dx.d, r, b + nup, s);
  const DevOp& op = o->ops[0].op;
  auto A = [&](const T* in, T* out) { apply_on<T>(o, op, Gct, true, in, out, 1, s, "ct"); };
  auto M = [&](const T* in, T* out) {
    KernelsT<T>::minv(Gct, Pct, o->dx.d, o->dv.d, o->pinv_dev.as<double>(), po.mass_sweeps, in, out, nullptr,
                      nullptr, s);
  };
  const Segs S = segs_of(Gct);
  o->inner_iters += batched_gmres<T>(o, S, A, M, b, ptr<T>(w.ctx), ptr<T>(w.ctV), ptr<T>(w.ctw), ptr<T>(w.cttmp), m,
                                     po.inner_maxit, po.inner_rtol, s, nan);
  // combination step
  KernelsT<T>::combine(Gup, Glow, g->lmin, o->dx.d, ptr<T>(w.ctx), ptr<T>(w.ctx) + nup, z, R, s);
  (void)nlow;
}

static sgdg_precond_opts default_pc() {
  sgdg_precond_opts p;
  p.kind = 0;
  p.inner_rtol = 1e-8;
  p.inner_maxit = 200;
  p.inner_restart = 30;
  p.mass_sweeps = 0;
  return p;
}

extern "C" sgdg_status sgdg_precondition(sgdg_ops o, const void* r_dev, void* z_dev, sgdg_dtype t, int batch,
                                         const sgdg_precond_opts* po_in, hipStream_t s) {
  API_BEGIN
  require(o && r_dev && z_dev && r_dev != z_dev, "null or aliased argument");
  require(batch == 1, "precondition supports batch == 1");
  const sgdg_precond_opts po = po_in ? *po_in : default_pc();
  require(po.kind == 0, "only the combination-technique preconditioner (kind 0) is available");
  require(po.inner_rtol > 0 && po.inner_maxit >= 1 && po.inner_restart >= 1, "invalid inner solver options");
  bool nan = false;
  if (t == SGDG_F64) ct_apply<double>(o, static_cast<const double*>(r_dev), static_cast<double*>(z_dev), po, s, &nan);
  else ct_apply<float>(o, static_cast<const float*>(r_dev), static_cast<float*>(z_dev), po, s, &nan);
  if (nan) throw Error{SGDG_E_NAN, "non-finite residual in a grid problem"};
  API_END
}

// --------------------------------------------------------------- data -----
static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0);
  w.assign(n, 0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      const double pn = n == 0 ? 1 : (n == 1 ? z : p1);
      const double pm = n == 1 ? 1 : p0;
      const double dp = n * (z * pn - pm) / (z * z - 1);
      const double dz = pn / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1, p1 = z;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    const double pn = n == 1 ? z : p1, pm = n == 1 ? 1 : p0;
    const double dp = n * (z * pn - pm) / (z * z - 1);
    x[i] = z;
    w[i] = 2.0 / ((1 - z * z) * dp * dp);
  }
  // ascending order
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return x[a] < x[b]; });
  std::vector<double> xs(n), ws(n);
  for (int i = 0; i < n; ++i) {
    xs[i] = x[idx[i]];
    ws[i] = w[idx[i]];
  }
  x = xs;
  w = ws;
}

static double legendre(int s, double z) {
  if (s == 0) return 1;
  double p0 = 1, p1 = z;
  for (int k = 2; k <= s; ++k) {
    const double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

// nodal [nq][up nodes + low nodes] -> projected blocks [grid][R][nx][nv] on both diagonals -> combined
static void nodal_to_coef(sgdg_ops o, const double* samples, int nq, const double* wts_host, int R, double* coef,
                          hipStream_t s) {
  sgdg_grid g = o->grid;
  const int64_t nall = g->up_pts + g->low_pts;
  o->rhs_w.ensure(sizeof(double) * R * nq);
  SGDG_CHECK_HIP(hipStreamSynchronize(s));  // rhs_w may still be read by earlier work
  SGDG_CHECK_HIP(hipMemcpy(o->rhs_w.p, wts_host, sizeof(double) * R * nq, hipMemcpyHostToDevice));
  o->rhs_a.ensure(sizeof(double) * R * nall);
  o->rhs_b.ensure(sizeof(double) * R * nall);
  double* proj = o->rhs_a.as<double>();   // [R][all nodes]
  double* blk = o->rhs_b.as<double>();    // [up blocks R][low blocks R]
  project_time(nall, nq, R, o->rhs_w.as<double>(), samples, proj, s);
  // reorder [R][nodes] -> per grid [R][nodes]
  const DevGrids Gup = g->make(g->up, R), Glow = g->make(g->low, R);
  int64_t node = 0;
  for (int part = 0; part < 2; ++part) {
    const DevGrids& G = part == 0 ? Gup : Glow;
    const int64_t base = part == 0 ? 0 : Gup.off[Gup.n];
    for (int gi = 0; gi < G.n; ++gi) {
      const int64_t np = int64_t(G.nx[gi]) * G.nv[gi];
      for (int sl = 0; sl < R; ++sl)
        SGDG_CHECK_HIP(hipMemcpyAsync(blk + base + G.off[gi] + sl * np, proj + int64_t(sl) * nall + node,
                                      sizeof(double) * np, hipMemcpyDeviceToDevice, s));
      node += np;
    }
  }
  KernelsT<double>::combine(Gup, Glow, g->lmin, o->dx.d, blk, blk + Gup.off[Gup.n], coef, R, s);
}

extern "C" sgdg_status sgdg_combine(sgdg_ops o, const double* nodal_dev, double* coef_dev, int nslices, hipStream_t s) {
  API_BEGIN
  require(o && nodal_dev && coef_dev, "null argument");
  require(nslices >= 1 && nslices <= kMaxR, "nslices must be 1..3");
  std::vector<double> wts(nslices * nslices, 0.0);
  for (int i = 0; i < nslices; ++i) wts[i * nslices + i] = 1.0;
  nodal_to_coef(o, nodal_dev, nslices, wts.data(), nslices, coef_dev, s);
  API_END
}

extern "C" sgdg_status sgdg_rhs(sgdg_ops o, const double* u_prev_dev, int prev_slices, const double* f_nodal_dev,
                                const double* g_nodal_dev, double* b_dev, hipStream_t s) {
  API_BEGIN
  require(o && u_prev_dev && b_dev, "null argument");
  require(prev_slices >= 1 && prev_slices <= kMaxR, "prev_slices must be 1..3");
  sgdg_grid g = o->grid;
  const int R = g->R;
  const int64_t npts = g->up_pts;
  // jump term
  o->rhs_c.ensure(sizeof(double) * 2 * npts);
  double* tr = o->rhs_c.as<double>();
  double* mtr = tr + npts;
  trace_sum(g->make(g->up, prev_slices), u_prev_dev, tr, s);
  apply_on<double>(o, o->ops[1].op, g->make(g->up, 1), false, tr, mtr, 1, s);
  spread_left(g->make(g->up, 1), R, mtr, b_dev, s);  // w(t_{j-1}^+) = eta_s(-1) = (-1)^s
  // data functionals
  if (f_nodal_dev || g_nodal_dev) {
    const int nq = g->r + 2;
    std::vector<double> xg, wg;
    gauss_legendre(nq, xg, wg);
    std::vector<double> wts(R * nq);
    // c_s = (2s+1)/dt int f eta_s = (2s+1)/2 sum_q wg_q P_s(xg_q) f_q
    for (int k = 0; k < R; ++k)
      for (int q = 0; q < nq; ++q) wts[k * nq + q] = 0.5 * (2 * k + 1) * wg[q] * legendre(k, xg[q]);
    const int64_t ndof = int64_t(R) * npts;
    o->rhs_d.ensure(sizeof(double) * 2 * ndof);
    double* coef = o->rhs_d.as<double>();
    double* out = coef + ndof;
    const DevGrids G = g->make(g->up, R);
    for (int which = 0; which < 2; ++which) {
      const double* smp = which == 0 ? f_nodal_dev : g_nodal_dev;
      if (!smp) continue;
      const DevOp& op = o->ops[which == 0 ? 2 : 3].op;
      if (op.nterms == 0) continue;
      nodal_to_coef(o, smp, nq, wts.data(), R, coef, s);
      apply_on<double>(o, op, G, false, coef, out, 1, s);
      KernelsT<double>::axpby(ndof, 1.0, out, 1.0, b_dev, s);
    }
  }
  API_END
}

// ------------------------------------------------------------- FGMRES -----
struct FgmresResult {
  int iters = 0;
  double rel = 0;
  bool nan = false;
};

// Flexible GMRES on the full vector (one segment) in FP64.  A and P act on FP64 vectors.
static FgmresResult fgmres(sgdg_ops o, int64_t n, std::function<void(const double*, double*)> A,
                           std::function<void(const double*, double*)> P, const double* b, double* x, double tol,
                           int m, int maxit, hipStream_t s) {
  Segs S;
  S.n = 1;
  S.off[0] = 0;
  S.off[1] = n;
  const int nch = nchunks_of(S);
  o->fV.ensure(sizeof(double) * n * (m + 1));
  o->fZ.ensure(sizeof(double) * n * m);
  o->fw.ensure(sizeof(double) * n);
  double* V = o->fV.as<double>();
  double* Z = o->fZ.as<double>();
  double* w = o->fw.as<double>();
  auto& gbuf = o->gb[1];
  gbuf.partial.ensure(sizeof(double) * nch * (m + 1));
  double* part = gbuf.partial.as<double>();
  GmresState st = gmres_state(gbuf, 1, m);
  FgmresResult res;
  const bool verbose = getenv("SGDG_VERBOSE") != nullptr;
  double bn2 = 0;
  KernelsT<double>::seg_norm2(S, b, part, nch, s);
  {
    std::vector<double> h(nch);
    SGDG_CHECK_HIP(hipMemcpyAsync(h.data(), part, sizeof(double) * nch, hipMemcpyDeviceToHost, s));
    SGDG_CHECK_HIP(hipStreamSynchronize(s));
    for (double v : h) bn2 += v;
  }
  const double bnorm = std::sqrt(bn2);
  if (!std::isfinite(bnorm)) {
    res.nan = true;
    return res;
  }
  if (bnorm == 0.0) {
    KernelsT<double>::fill(n, 0.0, x, s);
    return res;
  }
  for (;;) {
    // r = b - A x
    A(x, w);
    KernelsT<double>::copy(n, b, V, s);
    KernelsT<double>::axpby(n, -1.0, w, 1.0, V, s);
    KernelsT<double>::seg_norm2(S, V, part, nch, s);
    std::vector<double> h(nch);
    SGDG_CHECK_HIP(hipMemcpyAsync(h.data(), part, sizeof(double) * nch, hipMemcpyDeviceToHost, s));
    SGDG_CHECK_HIP(hipStreamSynchronize(s));
    double r2 = 0;
    for (double v : h) r2 += v;
    res.rel = std::sqrt(r2) / bnorm;
    if (verbose) fprintf(stderr, "[sgdg fgmres] true residual %.3e after %d\n", res.rel, res.iters);
    if (!std::isfinite(res.rel)) {
      res.nan = true;
      return res;
    }
    if (res.rel <= tol || res.iters >= maxit) return res;
    // start the cycle with the same tolerance measured against ||b||
    gmres_start(1, st, part, nch, 0.0, 1, s);
    // bnorm in the state is ||r0||; convergence is tested against tol*||b|| below on the host
    KernelsT<double>::seg_scale(S, V, st.inv, V, s);
    const int mm = std::min(m, maxit - res.iters);
    int j = 0;
    double est = res.rel;
    for (; j < mm; ++j) {
      P(V + int64_t(j) * n, Z + int64_t(j) * n);
      A(Z + int64_t(j) * n, w);
      for (int pass = 0; pass < 2; ++pass) {
        KernelsT<double>::seg_dots(S, V, n, j + 1, w, part, nch, s);
        gmres_add_proj(1, st, part, nch, j, s);
        KernelsT<double>::seg_axpy_multi(S, V, n, j + 1, st.hcol, m + 1, w, -1.0, pass == 1 ? part : nullptr, nch, s);
      }
      gmres_givens(1, st, part, nch, j, 0.0, s);
      KernelsT<double>::seg_scale(S, w, st.inv, V + int64_t(j + 1) * n, s);
      double beta = 0;
      int act = 0;
      SGDG_CHECK_HIP(hipMemcpyAsync(&beta, st.beta, sizeof(double), hipMemcpyDeviceToHost, s));
      SGDG_CHECK_HIP(hipMemcpyAsync(&act, st.active, sizeof(int), hipMemcpyDeviceToHost, s));
      SGDG_CHECK_HIP(hipStreamSynchronize(s));
      est = beta / bnorm;
      if (verbose) fprintf(stderr, "[sgdg fgmres] it %d  est %.3e\n", res.iters + j + 1, est);
      if (act == -1 || !std::isfinite(est)) {
        res.nan = true;
        return res;
      }
      if (est <= tol * 0.5 || act == 0) {
        ++j;
        break;
      }
    }
    res.iters += j;
    gmres_lsq(1, st, s);
    KernelsT<double>::seg_axpy_multi(S, Z, n, j, st.y, m, x, 1.0, nullptr, nch, s);
  }
}

extern "C" sgdg_status sgdg_solve_strip(sgdg_ops o, const double* b_dev, double* u_dev, const sgdg_solve_opts* so,
                                        sgdg_solve_stats* st, hipStream_t s) {
  API_BEGIN
  require(o && b_dev && u_dev && so, "null argument");
  require(so->rtol > 0 && so->restart >= 1 && so->restart <= 64 && so->maxit >= 1, "invalid solver options");
  const auto t0 = std::chrono::steady_clock::now();
  sgdg_grid g = o->grid;
  const int R = g->R;
  const DevGrids G = g->make(g->up, R);
  const int64_t n = G.off[G.n];
  const DevOp& op = o->ops[0].op;
  sgdg_precond_opts pc = so->pc;
  if (pc.inner_restart <= 0) pc = default_pc();
  o->inner_iters = 0;
  bool nan = false;
  auto A64 = [&](const double* in, double* out) { apply_on<double>(o, op, G, false, in, out, 1, s); };
  auto P64 = [&](const double* in, double* out) { ct_apply<double>(o, in, out, pc, s, &nan); };
  sgdg_solve_stats stats{};
  FgmresResult r;
  if (!so->mixed_precision) {
    r = fgmres(o, n, A64, P64, b_dev, u_dev, so->rtol, so->restart, so->maxit, s);
    stats.outer_iters = r.iters;
    stats.rel_residual = r.rel;
  } else {
    // FP64 iterative refinement; each correction solved by FGMRES with FP32
    // operator applications and an FP32 combination-technique preconditioner.
    Work<float>& w = o->w32;
    w.a32.ensure(sizeof(float) * n);
    w.b32.ensure(sizeof(float) * n);
    o->fr.ensure(sizeof(double) * n);
    o->fe.ensure(sizeof(double) * n);
    o->ftmp.ensure(sizeof(double) * n);
    float* a32 = w.a32.as<float>();
    float* b32 = w.b32.as<float>();
    auto A32 = [&](const double* in, double* out) {
      convert_f64_to_f32(n, in, a32, s);
      apply_on<float>(o, op, G, false, a32, b32, 1, s);
      convert_f32_to_f64(n, b32, out, s);
    };
    // FP32 grid problems cannot reach FP64 tolerances: solve them to >= 1e-5
    sgdg_precond_opts pc32 = pc;
    pc32.inner_rtol = std::max(pc.inner_rtol, 1e-5);
    auto P32 = [&](const double* in, double* out) {
      convert_f64_to_f32(n, in, a32, s);
      ct_apply<float>(o, a32, b32, pc32, s, &nan);
      convert_f32_to_f64(n, b32, out, s);
    };
    double* rr = o->fr.as<double>();
    double* e = o->fe.as<double>();
    double* tmp = o->ftmp.as<double>();
    const double inner_tol = so->inner_outer_rtol > 0 ? so->inner_outer_rtol : 1e-4;
    int total = 0, steps = 0;
    double rel = 1;
    Segs S1;
    S1.n = 1;
    S1.off[1] = n;
    const int nch = nchunks_of(S1);
    o->gb[2].partial.ensure(sizeof(double) * nch);
    std::vector<double> hp(nch);
    auto norm = [&](const double* v) {
      KernelsT<double>::seg_norm2(S1, v, o->gb[2].partial.as<double>(), nch, s);
      SGDG_CHECK_HIP(hipMemcpyAsync(hp.data(), o->gb[2].partial.p, sizeof(double) * nch, hipMemcpyDeviceToHost, s));
      SGDG_CHECK_HIP(hipStreamSynchronize(s));
      double a = 0;
      for (double v2 : hp) a += v2;
      return std::sqrt(a);
    };
    const double bnorm = norm(b_dev);
    for (;;) {
      A64(u_dev, tmp);
      KernelsT<double>::copy(n, b_dev, rr, s);
      KernelsT<double>::axpby(n, -1.0, tmp, 1.0, rr, s);
      rel = bnorm > 0 ? norm(rr) / bnorm : 0.0;
      if (!std::isfinite(rel)) {
        nan = true;
        break;
      }
      if (rel <= so->rtol || total >= so->maxit || steps >= 20) break;
      KernelsT<double>::fill(n, 0.0, e, s);
      FgmresResult ri = fgmres(o, n, A32, P32, rr, e, inner_tol, so->restart, so->maxit - total, s);
      total += std::max(ri.iters, 1);
      ++steps;
      if (ri.nan) {
        nan = true;
        break;
      }
      KernelsT<double>::axpby(n, 1.0, e, 1.0, u_dev, s);
    }
    stats.outer_iters = total;
    stats.refinement_steps = steps;
    stats.rel_residual = rel;
    r.rel = rel;
    r.nan = nan;
  }
  SGDG_CHECK_HIP(hipStreamSynchronize(s));
  stats.inner_iters_total = int(o->inner_iters);
  stats.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (st) *st = stats;
  if (nan || r.nan) throw Error{SGDG_E_NAN, "non-finite residual norm"};
  if (stats.rel_residual > so->rtol) throw Error{SGDG_E_NOCONV, "iteration limit reached before the tolerance"};
  API_END
}

// ---------------------------------------------------------- diagnostics ---
extern "C" sgdg_status sgdg_profile(sgdg_ops o, int mode) {
  API_BEGIN
  require(o != nullptr, "null ops");
  drain_events(o);
  if (mode == 1) {
    for (int i = 0; i < 3; ++i) {
      o->prof_ms[i] = 0;
      o->prof_n[i] = 0;
    }
  }
  o->prof = mode == 1;
  API_END
}

extern "C" sgdg_status sgdg_profile_read(sgdg_ops o, int slot, double* ms, int64_t* launches) {
  API_BEGIN
  require(o != nullptr && slot >= 0 && slot < 3, "bad slot");
  drain_events(o);
  if (ms) *ms = o->prof_ms[slot];
  if (launches) *launches = o->prof_n[slot];
  API_END
}

extern "C" sgdg_status sgdg_op_info(sgdg_ops o, int kind, int* nterms, int* nvg, int* nxg, int* Sx, int* Sv,
                                    int* Rin, int* Rout) {
  API_BEGIN
  require(o != nullptr && kind >= SGDG_OP_FULL && kind <= SGDG_OP_DATA_G, "bad arguments");
  const int idx = kind == SGDG_OP_FULL || kind == SGDG_OP_BLOCKDIAG ? 0 : kind - 1;
  const DevOp& op = o->ops[idx].op;
  if (nterms) *nterms = op.nterms;
  if (nvg) *nvg = op.nvg;
  if (nxg) *nxg = op.nxg;
  if (Sx) *Sx = o->dx.d.S;
  if (Sv) *Sv = o->dv.d.S;
  if (Rin) *Rin = op.Rin;
  if (Rout) *Rout = op.Rout;
  API_END
}
