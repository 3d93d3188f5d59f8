// Batched operator application, the combination-technique preconditioner
// (Algorithm 1's body, Sect. 4.3), the strip right-hand side
// (eq:weak_form_j) and the flexible-GMRES strip solves, for a batch of
// independent problems.  The single-problem entry points use a batch of one.
#include <sys/stat.h>

#include <chrono>
#include <mutex>
#include <fstream>
#include <limits>
#include <sstream>
#include <type_traits>

#include <complex>

#include "fourier.h"
#include "ops_internal.h"
#include "split.h"

// ----------------------------------------------------------------- batch ---
namespace {

enum Kind { K_FULL = 0, K_DIAG = 1, K_MASS = 2, K_DATAF = 3, K_DATAG = 4, K_CT = 5, K_COUNT = 6 };

struct GBufs {
  DevBuf H, cs, sn, g, bn, beta, act, k, hc, inv, y, partial;
};

struct SegTab {
  DevBuf segs, blk;
  std::vector<SegInfo> host;
  SegTable t;
  // x-transport preconditioner of the segments (periodic x), built on first use
  DevBuf fsegs, flines, fpinv;
  FourierTab ftab;
  bool fourier = false;
};

struct Items {
  DevBuf items, sitems;
  int n = 0, max_u = 0, max_stage = 0, max_tab = 0;
  std::vector<int> step_first, step_count;
  bool built = false;
};

struct KindData {
  DevBuf desc;
  std::vector<ProbDesc> host;
  int64_t pt_bstride = 0, qt_bstride = 0, z_bstride = 0, rv_bstride = 0, rx_bstride = 0, total = 0;
  int R = 1;
  bool any_scan = false;
  Items it[2];  // FP64, FP32
  DevBuf split_items;
  int n_split = 0;
  int max_qn = 0;  // largest coarse range of an item in the upper-partner pass
  DevBuf tile_items;
  int n_tile = 0;
  int max_tile = 0;  // largest staged tile of the x-stencil pass
};

template <class T>
struct BWork {
  DevBuf Pt, Qt, Rv, Rx, Z, ctb, ctx, ctw, cttmp, ctV, cvt_in, cvt_out;
  DevBuf mU, mX0, mX1, mD0, mD1;  // mass-inverse stages of the grid-problem preconditioner
};

// Pinned host copies of the per-segment GMRES flags and residual estimates of
// two consecutive iterations, each with the event that marks its copy done.
struct FlagRing {
  int* act[2] = {nullptr, nullptr};
  double* beta[2] = {nullptr, nullptr};
  hipEvent_t ev[2] = {nullptr, nullptr};
  int cap = 0;
  void release() {
    for (int i = 0; i < 2; ++i) {
      if (act[i]) (void)hipHostFree(act[i]);
      if (beta[i]) (void)hipHostFree(beta[i]);
      if (ev[i]) (void)hipEventDestroy(ev[i]);
      act[i] = nullptr;
      beta[i] = nullptr;
      ev[i] = nullptr;
    }
    cap = 0;
  }
  ~FlagRing() { release(); }
};


}  // namespace

struct sgdg_batch_s {
  std::vector<sgdg_ops> P;
  int d = 1, R = 1;
  KindData kinds[K_COUNT];
  std::map<int, std::unique_ptr<SegTab>> ct_tabs, prob_tabs;
  std::unique_ptr<SegTab> pts;
  GBufs gb[3];  // grid problems, strip FGMRES, norms
  BWork<double> w64;
  BWork<float> w32;
  DevBuf fV, fZ, fw, fr, fe, ftmp, a32, b32;
  DevBuf rhs_a, rhs_b, rhs_c, rhs_d, rhs_w;
  int64_t inner_iters = 0;
  bool owned_by_ops = false;
  std::unique_ptr<FlagRing> flags;  // pinned flag copies of the strip FGMRES
  std::vector<sgdg_net> nets;  // learned preconditioner of each problem (sgdg_batch_set_networks)
  DevBuf fourier_c;            // complex scratch of the x-transport preconditioner
  // box-shape choice of the fused kernel per element size (tuned or default)
  int xbox[2] = {0, 0};
  // operator application variant: 0 split (streaming passes), 1 fused box
  // tiles, 2 split with the x-stage on LDS tiles
  int variant = 0;
  int split_bc = 0;  // vectors per thread of the split passes (0: default for d)
  int split_xcd = 0;  // 1: XCD-contiguous block order in the split passes
  // blocks sharing the factor groups of a scan item; 0: chosen per launch so
  // that a step has about kScanBlocks blocks (small steps and single vectors
  // split their groups; large batched steps keep one block per item)
  int scan_chunks = 1;
  // graphs of grid-problem GMRES cycles, valid while alloc_epoch() equals
  // graph_epoch (a reallocated work buffer or rebuilt table empties the cache)
  std::map<std::string, hipGraphExec_t> graphs;
  uint64_t graph_epoch = 0;
  hipStream_t cap_stream = nullptr;
  void clear_graphs() {
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.second);
    graphs.clear();
  }
  // event timing: slot 0 level scans, 1 fused tiles, 2 grid-problem cycles,
  // 3/4/5 split v-stage, upper-partner and x-stage passes
  static constexpr int kSlots = 6;
  bool prof = false;
  struct Ev {
    hipEvent_t a, b;
    int slot;
  };
  std::vector<Ev> events;
  double prof_ms[kSlots] = {};
  int64_t prof_n[kSlots] = {};
  ~sgdg_batch_s() {
    for (auto& e : events) {
      (void)hipEventDestroy(e.a);
      (void)hipEventDestroy(e.b);
    }
    clear_graphs();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
  }
};

void destroy_batch(Batch* b) { delete b; }

Batch& self_batch(sgdg_ops o) {
  if (!o->self) {
    Batch* b = new Batch;
    b->P = {o};
    b->d = o->X.dom.d;
    b->R = o->grid->R;
    b->owned_by_ops = true;
    if (const char* v = getenv("SGDG_APPLY_VARIANT"))
      b->variant = std::string(v) == "fused" ? 1 : (std::string(v) == "split_tiled" ? 2 : 0);
    if (const char* v = getenv("SGDG_SPLIT_BC")) b->split_bc = atoi(v);
    b->split_xcd = split_xcd();
    if (const char* v = getenv("SGDG_SCAN_CHUNKS")) b->scan_chunks = std::max(0, atoi(v));
    o->self.reset(b);
  }
  return *o->self;
}

Batch& replica_batch(sgdg_ops o, int n) {
  if (n == 1) return self_batch(o);
  auto it = o->replicas.find(n);
  if (it != o->replicas.end()) return *it->second;
  const Batch& S = self_batch(o);
  Batch* b = new Batch;
  b->P.assign(size_t(n), o);
  b->d = S.d;
  b->R = S.R;
  b->variant = S.variant;
  b->split_bc = S.split_bc;
  b->split_xcd = S.split_xcd;
  b->scan_chunks = S.scan_chunks;
  o->replicas[n].reset(b);
  return *b;
}

template <class T>
static BWork<T>& work(Batch& B);
template <>
BWork<double>& work<double>(Batch& B) { return B.w64; }
template <>
BWork<float>& work<float>(Batch& B) { return B.w32; }

template <class F>
static void timed(Batch& B, int slot, hipStream_t s, F&& launch) {
  if (!B.prof) {
    launch();
    return;
  }
  Batch::Ev e;
  e.slot = slot;
  SGDG_CHECK_HIP(hipEventCreate(&e.a));
  SGDG_CHECK_HIP(hipEventCreate(&e.b));
  SGDG_CHECK_HIP(hipEventRecord(e.a, s));
  launch();
  SGDG_CHECK_HIP(hipEventRecord(e.b, s));
  B.events.push_back(e);
}

static void drain_events(Batch& B) {
  for (auto& e : B.events) {
    SGDG_CHECK_HIP(hipEventSynchronize(e.b));
    float ms = 0;
    SGDG_CHECK_HIP(hipEventElapsedTime(&ms, e.a, e.b));
    B.prof_ms[e.slot] += ms;
    B.prof_n[e.slot] += 1;
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  B.events.clear();
}

// ------------------------------------------------------- descriptors -----
static int64_t up_pts(sgdg_ops o) { return o->grid->up_pts; }

// longest coarse range an item of the upper-partner pass stages in LDS; with a
// longer one anywhere in the batch the pass reads the slots from memory
constexpr int64_t kMaxItemRange = 512;

static KindData& kind(Batch& B, int k) {
  KindData& K = B.kinds[k];
  if (!K.host.empty()) return K;
  const bool ct = k == K_CT;
  const int opidx = (k == K_FULL || k == K_DIAG || k == K_CT) ? 0 : (k == K_MASS ? 1 : (k == K_DATAF ? 2 : 3));
  const int R = B.P[0]->ops[opidx].op.Rin;
  K.R = R;
  int64_t off = 0, pt = 0, qt = 0, zo = 0, rvb = 0, rxb = 0;
  std::vector<SplitItem> sitems;
  std::vector<TileItem> titems;
  const bool vmajor = split_vmajor();
  bool tiles_ok = true;  // tiles address a grid plane with 32-bit offsets
  for (size_t p = 0; p < B.P.size(); ++p) {
    sgdg_ops o = B.P[p];
    sgdg_grid g = o->grid;
    ProbDesc D{};
    require(o->ops[opidx].op.Rin == R && o->ops[opidx].op.Rout == R, "operator slices differ within the batch");
    require(int(g->up.size() + (ct ? g->low.size() : 0)) <= kMaxGrids, "too many component grids");
    D.G = ct ? g->make_ct(R) : g->make(g->up, R);
    D.Gl = g->make(g->low, R);
    int64_t po = 0;
    for (int i = 0; i < D.G.n; ++i) {
      D.poff[i] = po;
      po += int64_t(D.G.nx[i]) * D.G.nv[i];
    }
    D.poff[D.G.n] = po;
    D.DX = o->dx.d;
    D.DV = o->dv.d;
    D.op = o->ops[opidx].op;
    for (int l = 0; l < kMaxLevels; ++l) {
      D.mx[l] = g->x.axis_nodes(l);
      D.mv[l] = g->v.axis_nodes(l);
    }
    D.xper = g->x.periodic;
    D.vper = g->v.periodic;
    for (int e = 0; e < kMaxS; ++e)
      for (int a = 0; a < 3; ++a) D.off[e][a] = e < o->X.st.S ? o->X.st.off[e][a] : 0;
    D.diag_only = (k == K_DIAG || ct || D.G.n == 1) ? 1 : 0;
    D.u_off = D.y_off = off;
    off += D.G.off[D.G.n];
    D.pt_off = pt;
    D.qt_off = qt;
    D.z_off = zo;
    zo += int64_t(std::max(1, D.op.nxg)) * D.G.off[D.G.n];  // one staged array per X-group
    for (int gi = 0; gi < D.G.n; ++gi) {
      // blocks in Morton order of their x-node (then v): x-rows that share
      // parents or stencil neighbours run close together in time
      const int64_t nvg = D.G.nv[gi];
      const int64_t plane = int64_t(D.G.nx[gi]) * nvg;
      const int mxg = g->x.axis_nodes(D.G.lx[gi]);
      std::vector<std::pair<uint64_t, int64_t>> keyed;
      for (int64_t p0 = 0; p0 < plane; p0 += split_points_per_item()) {
        int64_t xn = p0 / nvg;
        int c[3] = {0, 0, 0};
        for (int a = B.d - 1; a >= 0; --a) {
          c[a] = int(xn % mxg);
          xn /= mxg;
        }
        uint64_t key = 0;
        for (int bit = 0; bit < 16; ++bit)
          for (int a = 0; a < B.d; ++a) key |= uint64_t((c[a] >> bit) & 1) << (bit * B.d + a);
        const uint64_t vb = uint64_t((p0 % nvg) / split_points_per_item());
        keyed.push_back({vmajor ? (vb << 40) | key : (key << 24) | vb, p0});
      }
      std::stable_sort(keyed.begin(), keyed.end());
      const bool upper = !D.diag_only && gi + 1 < D.G.n && B.d <= 2;
      for (const auto& kp : keyed) {
        SplitItem it{};
        it.prob = int(p);
        it.grid = gi;
        it.p0 = kp.second;
        it.gmask = ~uint64_t(0);
        if (upper) {
          // X-groups whose Qt can be nonzero on the block's x-rows
          const std::vector<uint64_t>& qm = o->ops[opidx].hxqtm;
          const int64_t noff = o->dx.d.node_off[D.G.lx[gi] - o->dx.d.lmin];
          const int64_t pend = std::min<int64_t>(kp.second + split_points_per_item(), plane);
          it.gmask = 0;
          for (int64_t xr = kp.second / nvg; xr <= (pend - 1) / nvg; ++xr) it.gmask |= qm[size_t(noff + xr)];
        }
        if (upper) {
          // the prolongation slots of every point, from the level's slot table
          const std::vector<int32_t>& ptab = o->V.pro_idx[D.G.lv[gi] - o->V.lmin];
          const int npw = int(ptab.size() / size_t(nvg));
          const int64_t nvl = D.Gl.nv[gi];
          int64_t lo = std::numeric_limits<int64_t>::max(), hi = -1;
          const int64_t pend = std::min<int64_t>(kp.second + split_points_per_item(), plane);
          for (int64_t pp = kp.second; pp < pend; ++pp) {
            const int64_t xn = pp / nvg, vn = pp % nvg;
            for (int sl = 0; sl < npw; ++sl) {
              const int64_t f = xn * nvl + ptab[size_t(sl) * nvg + vn];
              lo = std::min(lo, f);
              hi = std::max(hi, f);
            }
          }
          it.q0 = lo;
          it.qn = int(std::min<int64_t>(hi - lo + 1, kMaxItemRange + 1));
          K.max_qn = std::max(K.max_qn, it.qn);
        }
        sitems.push_back(it);
      }
      // x-stencil tiles: t^d x-nodes times vb v-nodes
      if (plane >= (int64_t(1) << 31)) tiles_ok = false;
      {
        const int mxg2 = g->x.axis_nodes(D.G.lx[gi]);
        int t = 1, vb = 1;
        split_tile_shape(B.d, mxg2, int(nvg), t, vb);
        const int ntx = (mxg2 + t - 1) / t;
        int ntt = 1;
        for (int a = 0; a < B.d; ++a) ntt *= ntx;
        for (int tt = 0; tt < ntt; ++tt) {
          TileItem ti{};
          ti.prob = int(p);
          ti.grid = gi;
          int r = tt;
          for (int a = B.d - 1; a >= 0; --a) {
            ti.x0[a] = (r % ntx) * t;
            r /= ntx;
          }
          ti.t = t;
          ti.vb = vb;
          // X-groups whose factor has a nonzero row on the tile (a face term
          // only on tiles that touch its face)
          {
            const DomDev& dx = o->dx;
            const std::vector<int>& xgf = o->ops[opidx].hxgf;
            const int lxg = D.G.lx[gi];
            const int64_t noff = dx.d.node_off[lxg - dx.d.lmin];
            ti.gmask = 0;
            for (size_t m = 0; m < xgf.size() && m < 64; ++m) {
              bool need = dx.hpartial[size_t(xgf[m])] == 0;
              const uint8_t* sp = dx.hsup.data() + size_t(xgf[m]) * size_t(dx.d.node_stride) + noff;
              int nt = 1;
              for (int a = 0; a < B.d; ++a) nt *= t;
              for (int xi = 0; xi < nt && !need; ++xi) {
                int rr = xi, node = 0;
                bool in = true;
                int c[3] = {0, 0, 0};
                for (int a = B.d - 1; a >= 0; --a) {
                  c[a] = ti.x0[a] + rr % t;
                  rr /= t;
                }
                for (int a = 0; a < B.d; ++a) {
                  in = in && c[a] < mxg2;
                  node = node * mxg2 + c[a];
                }
                need = in && (sp[node] & 1);
              }
              if (need) ti.gmask |= uint64_t(1) << m;
            }
          }
          int halo = 1;
          for (int a = 0; a < B.d; ++a) halo *= t + 2;
          K.max_tile = std::max(K.max_tile, halo * vb);
          for (int v0 = 0; v0 < nvg; v0 += vb) {
            ti.v0 = v0;
            titems.push_back(ti);
          }
        }
      }
    }
    D.rv_off = rvb;
    D.rx_off = rxb;
    D.rv_len = D.rx_len = 0;
    if (!D.diag_only) {
      K.any_scan = true;
      const int64_t lt = D.Gl.off[D.Gl.n];
      pt += int64_t(std::max(1, D.op.nvg)) * lt;
      qt += int64_t(std::max(1, D.op.nxg)) * lt;
      const int nlow = D.Gl.n;
      for (int t = 0; t < nlow; ++t) {
        D.rvo[t] = D.rv_len;
        if (t >= 1) D.rv_len += int64_t(R) * D.Gl.nx[t - 1] * D.Gl.nv[t];
        D.rxo[t] = D.rx_len;
        if (t + 1 < nlow) D.rx_len += int64_t(R) * D.Gl.nx[t] * D.Gl.nv[t + 1];
      }
      rvb += int64_t(std::max(1, D.op.nvg)) * std::max<int64_t>(1, D.rv_len);
      rxb += int64_t(std::max(1, D.op.nxg)) * std::max<int64_t>(1, D.rx_len);
    }
    K.host.push_back(D);
  }
  if (K.max_qn > kMaxItemRange) K.max_qn = 0;  // some range too long: every item reads from memory
  K.total = off;
  K.pt_bstride = pt;
  K.qt_bstride = qt;
  K.z_bstride = zo;
  K.rv_bstride = rvb;
  K.rx_bstride = rxb;
  upload(K.desc, K.host);
  upload(K.split_items, sitems);
  upload(K.tile_items, titems);
  K.n_tile = tiles_ok ? int(titems.size()) : 0;
  K.n_split = int(sitems.size());
  return K;
}

// Box shape of one grid for the fused kernel: x-box and v-box sizes per axis
// under the per-thread row limit and a bounded LDS stage.
static void choose_boxes(int d, int bx, int mx, int mv, int R, int elem, int* xs, int* vs) {
  const int nthr = fused_threads(), rows = fused_rows_per_thread();
  const size_t lds_cap = 56 * 1024;  // per item; the launch sizes for the largest stage and halo over all items
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
    const size_t uh = nxh * nvh * size_t(R) * elem;  // u on the halo boxes
    const size_t tab = (nxh + 2 * nx + 2 * nvb + nvh) * sizeof(int);
    return uh + st + tab <= lds_cap;
  };
  const int one[3] = {1, 1, 1};
  while (!fits(one)) {  // shrink the x-box until the smallest v-box fits
    int a = 0;
    for (int c = 1; c < d; ++c)
      if (xs[c] > xs[a]) a = c;
    if (xs[a] <= 1) throw Error{SGDG_E_ARG, "no box shape fits the LDS budget"};
    xs[a] = (xs[a] + 1) / 2;
  }
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

static int default_xbox(int d) { return d == 1 ? 32 : (d == 2 ? 8 : 4); }

static Items& items(Batch& B, int k, int elem) {
  KindData& K = kind(B, k);
  Items& I = K.it[elem == 8 ? 0 : 1];
  if (I.built) return I;
  const int bx = B.xbox[elem == 8 ? 0 : 1] > 0 ? B.xbox[elem == 8 ? 0 : 1] : default_xbox(B.d);
  std::vector<FusedItem> its;
  int64_t max_stage = 1, max_tab = 1, max_u = 1;
  int maxn = 0;
  for (size_t p = 0; p < B.P.size(); ++p) {
    const ProbDesc& D = K.host[p];
    sgdg_grid g = B.P[p]->grid;
    maxn = std::max(maxn, D.G.n);
    for (int gi = 0; gi < D.G.n; ++gi) {
      const int mx = g->x.axis_nodes(D.G.lx[gi]), mv = g->v.axis_nodes(D.G.lv[gi]);
      int xs[3], vs[3];
      choose_boxes(B.d, bx, mx, mv, K.R, elem, xs, vs);
      int nbx[3] = {1, 1, 1}, nbv[3] = {1, 1, 1};
      int64_t nx_h = 1, nv_b = 1, nx_b = 1, nv_h = 1;
      for (int a = 0; a < B.d; ++a) {
        nbx[a] = (mx + xs[a] - 1) / xs[a];
        nbv[a] = (mv + vs[a] - 1) / vs[a];
        nx_h *= xs[a] + 2;
        nx_b *= xs[a];
        nv_b *= vs[a];
        nv_h *= vs[a] + 2;
      }
      max_stage = std::max<int64_t>(max_stage, std::max(nx_h * nv_b, nx_b * nv_h) * K.R);
      max_u = std::max<int64_t>(max_u, nx_h * nv_h * K.R);
      max_tab = std::max<int64_t>(max_tab, nx_h + 2 * nx_b + 2 * nv_b + nv_h);
      for (int i0 = 0; i0 < nbx[0]; ++i0)
        for (int i1 = 0; i1 < nbx[1]; ++i1)
          for (int i2 = 0; i2 < nbx[2]; ++i2)
            for (int j0 = 0; j0 < nbv[0]; ++j0)
              for (int j1 = 0; j1 < nbv[1]; ++j1)
                for (int j2 = 0; j2 < nbv[2]; ++j2) {
                  FusedItem f{};
                  f.prob = int(p);
                  f.grid = gi;
                  const int ix[3] = {i0, i1, i2}, iv[3] = {j0, j1, j2};
                  for (int a = 0; a < 3; ++a) {
                    f.xb[a] = a < B.d ? ix[a] * xs[a] : 0;
                    f.xs[a] = a < B.d ? std::min(xs[a], mx - f.xb[a]) : 1;
                    f.vb[a] = a < B.d ? iv[a] * vs[a] : 0;
                    f.vs[a] = a < B.d ? std::min(vs[a], mv - f.vb[a]) : 1;
                  }
                  its.push_back(f);
                }
    }
  }
  upload(I.items, its);
  I.n = int(its.size());
  I.max_stage = int(max_stage);
  I.max_u = int(max_u);
  I.max_tab = int(max_tab);
  // scan work: launch 2t is step t (base + recursion from the restricted
  // arrays), launch 2t-1 restricts the arrays step t - 1 finished (t >= 1)
  std::vector<ScanItem> sits;
  I.step_first.clear();
  I.step_count.clear();
  if (K.any_scan) {
    for (int t = 0; t + 1 < maxn; ++t) {
      for (int phase = (t == 0 ? 1 : 0); phase < 2; ++phase) {
        I.step_first.push_back(int(sits.size()));
        for (size_t p = 0; p < B.P.size(); ++p) {
          const ProbDesc& D = K.host[p];
          if (D.diag_only || t + 1 >= D.G.n) continue;
          const int nlow = D.Gl.n;
          for (int side = 0; side < 2; ++side) {
            const int lg = side == 0 ? t : nlow - 1 - t;
            int64_t len;
            if (phase == 1) {
              len = int64_t(D.Gl.nx[lg]) * D.Gl.nv[lg];  // target points; slices loop in the kernel
            } else {
              len = side == 0 ? int64_t(D.Gl.nx[lg - 1]) * D.Gl.nv[lg] : int64_t(D.Gl.nx[lg]) * D.Gl.nv[lg + 1];
            }
            for (int64_t st = 0; st < len; st += fused_threads())
              sits.push_back(ScanItem{int(p), side, lg, phase == 1 ? 0 : 2, st});
          }
        }
        I.step_count.push_back(int(sits.size()) - I.step_first.back());
      }
    }
  }
  upload(I.sitems, sits);
  I.built = true;
  return I;
}

// target block count of a level-scan launch when the group split is automatic
constexpr int64_t kScanBlocks = 2048;

// Caller-provided scratch for the allocation-free application: the work
// arrays of one call are carved from it in turn (256-byte aligned pieces).
struct Carve {
  unsigned char* base = nullptr;
  size_t bytes = 0, used = 0;
  template <class T>
  T* take(size_t n) {
    const size_t b = (sizeof(T) * n + 255) & ~size_t(255);
    if (used + b > bytes) throw Error{SGDG_E_ARG, "scratch too small"};
    T* p = reinterpret_cast<T*>(base + used);
    used += b;
    return p;
  }
};

// Scratch bytes one application of kind k needs for nb vectors of T (the
// launch tables must exist).
template <class T>
static size_t apply_scratch_bytes(Batch& B, int k, int nb) {
  const KindData& K = B.kinds[k];
  auto r = [](size_t b) { return (b + 255) & ~size_t(255); };
  size_t need = 0;
  if (K.any_scan)
    need += r(sizeof(T) * size_t(K.pt_bstride) * nb) + r(sizeof(T) * size_t(K.qt_bstride) * nb) +
            r(sizeof(T) * size_t(K.rv_bstride) * nb) + r(sizeof(T) * size_t(K.rx_bstride) * nb);
  if (B.variant != 1) need += r(sizeof(T) * size_t(K.z_bstride) * nb);
  return need;
}

// ws == nullptr: work arrays from the handle's workspaces (grown on demand);
// otherwise every work array comes from *ws, the tables must already exist and
// nothing is allocated or timed.
template <class T>
static void apply(Batch& B, int k, const T* u, T* y, int nb, hipStream_t s, Carve* ws = nullptr) {
  if (ws) require_state(!B.kinds[k].host.empty() && B.kinds[k].it[sizeof(T) == 8 ? 0 : 1].built,
                        "launch tables of this operator kind and dtype are not built yet: apply it once with "
                        "sgdg_apply_operator first");
  KindData& K = kind(B, k);
  Items& I = items(B, k, int(sizeof(T)));
  BWork<T>& w = work<T>(B);
  auto buf = [&](DevBuf& d, size_t n) -> T* {
    if (ws) return ws->take<T>(n);
    d.ensure(sizeof(T) * n);
    return ptr<T>(d);
  };
  auto run = [&](int slot, auto&& launch) {
    if (ws) launch();
    else timed(B, slot, s, launch);
  };
  FusedCall<T> C{};
  C.descs = ptr<ProbDesc>(K.desc);
  C.items = ptr<FusedItem>(I.items);
  C.sitems = ptr<ScanItem>(I.sitems);
  C.nitems = I.n;
  C.max_stage = I.max_stage;
  C.max_u = I.max_u;
  C.max_tab = I.max_tab;
  C.B = nb;
  C.u_bstride = C.y_bstride = K.total;
  C.u = u;
  C.y = y;
  C.sparse_partners = B.variant == 1 ? 0 : 1;
  if (K.any_scan) {
    C.Pt = buf(w.Pt, size_t(K.pt_bstride) * nb);
    C.Qt = buf(w.Qt, size_t(K.qt_bstride) * nb);
    C.pt_bstride = K.pt_bstride;
    C.qt_bstride = K.qt_bstride;
    C.Rv = buf(w.Rv, size_t(K.rv_bstride) * nb);
    C.Rx = buf(w.Rx, size_t(K.rx_bstride) * nb);
    C.rv_bstride = K.rv_bstride;
    C.rx_bstride = K.rx_bstride;
    run(0, [&] {
      for (size_t t = 0; t < I.step_first.size(); ++t) {
        FusedCall<T> Cs = C;
        Cs.sitems = C.sitems + I.step_first[t];
        int chunks = B.scan_chunks;
        if (chunks == 0) {
          int ng = 1;
          for (const ProbDesc& D : K.host) ng = std::max(ng, std::max(D.op.nvg, D.op.nxg));
          const int64_t blocks = int64_t(std::max(1, I.step_count[t])) * nb;
          chunks = int(std::min<int64_t>(ng, std::max<int64_t>(1, (kScanBlocks + blocks - 1) / blocks)));
        }
        fused_scan_step<T>(Cs, I.step_count[t], B.d, K.R, chunks, s);
      }
    });
  }
  if (B.variant == 1) {
    run(1, [&] { fused_tiles<T>(C, B.d, K.R, s); });
    return;
  }
  SplitCall<T> S{};
  S.descs = C.descs;
  S.items = ptr<SplitItem>(K.split_items);
  S.nitems = K.n_split;
  S.B = nb;
  S.u_bstride = S.y_bstride = K.total;
  S.pt_bstride = K.pt_bstride;
  S.qt_bstride = K.qt_bstride;
  S.z_bstride = K.z_bstride;
  S.u = u;
  S.y = y;
  S.Pt = C.Pt;
  S.Qt = C.Qt;
  S.Z = buf(w.Z, size_t(K.z_bstride) * nb);
  S.max_qn = K.max_qn;
  S.tiles = ptr<TileItem>(K.tile_items);
  S.ntiles = B.variant == 2 ? K.n_tile : 0;
  S.max_tile = K.max_tile;
  S.xcd = B.split_xcd;
  // one vector per thread for single vectors (the solvers); tuned otherwise
  const int bc = nb == 1 ? 1 : (B.split_bc > 0 ? B.split_bc : split_default_bc(B.d));
  // without any partner coupling (block-diagonal kinds) the upper-partner pass
  // would only zero y: pass 3 writes y instead
  S.x_assign = K.any_scan ? 0 : 1;
  for (int stage = 0; stage < 3; ++stage) {
    if (stage == 1 && S.x_assign) continue;
    run(3 + stage, [&] { split_stage<T>(S, B.d, K.R, bc, stage, s); });
  }
}

// ---------------------------------------------------------- segments -----
static void finish_tab(SegTab& T) {
  std::vector<BlockRef> blk;
  int chunk = 0;
  for (size_t i = 0; i < T.host.size(); ++i) {
    SegInfo& S = T.host[i];
    S.chunk0 = chunk;
    S.nchunk = int(std::max<int64_t>(1, (S.len + kChunk - 1) / kChunk));
    for (int c = 0; c < S.nchunk; ++c) blk.push_back(BlockRef{int(i), c});
    chunk += S.nchunk;
  }
  T.t.segs = upload(T.segs, T.host);
  T.t.blk = upload(T.blk, blk);
  T.t.nseg = int(T.host.size());
  T.t.nblk = int(blk.size());
  T.t.nchunks = chunk;
}

static void fill_domain_ptrs(sgdg_ops o, SegInfo& S) {
  const DevDomain& X = o->dx.d;
  const DevDomain& V = o->dv.d;
  S.Sx = X.S;
  S.Sv = V.S;
  S.S = X.S;
  S.mxd = X.vals + int64_t(X.mass_fac) * X.fac_stride + X.lev_off[S.lx - X.lmin];
  S.mvd = V.vals + int64_t(V.mass_fac) * V.fac_stride + V.lev_off[S.lv - V.lmin];
  S.xchi = X.chi + X.lev_off[S.lx - X.lmin];
  S.xchiw = X.chiw + X.lev_off[S.lx - X.lmin];
  S.xpar = X.par + X.par_off[S.lx - X.lmin];
  S.xparw = X.parw + X.par_off[S.lx - X.lmin];
  for (int i = 0; i < kMaxR * kMaxR; ++i) S.pinv[i] = o->pinv[i];
  S.xnbr = X.nbr + X.lev_off[S.lx - X.lmin];
  S.vnbr = V.nbr + V.lev_off[S.lv - V.lmin];
  S.xper = o->grid->x.periodic ? 1 : 0;
  S.vper = o->grid->v.periodic ? 1 : 0;
  S.sm = S.sp = -1;
  if (o->X.dom.d == 1) {
    const int om[3] = {-1, 0, 0}, op[3] = {1, 0, 0};
    S.sm = o->X.st.slot(om);
    S.sp = o->X.st.slot(op);
  }
}

// grid problems of the combination technique: upper then lower grids of each problem
static SegTab& ct_tab(Batch& B, int Rs) {
  auto it = B.ct_tabs.find(Rs);
  if (it != B.ct_tabs.end()) return *it->second;
  auto T = std::make_unique<SegTab>();
  int64_t ct = 0, up = 0;
  for (size_t p = 0; p < B.P.size(); ++p) {
    sgdg_ops o = B.P[p];
    sgdg_grid g = o->grid;
    std::vector<int64_t> up_start, low_start;
    int64_t c = ct;
    for (auto& gd : g->up) {
      up_start.push_back(c);
      c += int64_t(Rs) * gd.nx * gd.nv;
    }
    for (auto& gd : g->low) {
      low_start.push_back(c);
      c += int64_t(Rs) * gd.nx * gd.nv;
    }
    int64_t u = up;
    std::vector<int64_t> up_res;
    for (auto& gd : g->up) {
      up_res.push_back(u);
      u += int64_t(Rs) * gd.nx * gd.nv;
    }
    for (size_t i = 0; i < g->up.size(); ++i) {
      SegInfo S{};
      S.prob = int(p);
      S.kind = 0;
      S.lx = g->up[i].lx;
      S.lv = g->up[i].lv;
      S.nx = int(g->up[i].nx);
      S.nv = int(g->up[i].nv);
      S.R = Rs;
      S.off = up_start[i];
      S.len = int64_t(Rs) * S.nx * S.nv;
      S.src_off = up_res[i];
      S.low_off = i > 0 ? low_start[i - 1] : -1;
      S.nx_src = i > 0 ? int(g->low[i - 1].nx) : 0;
      fill_domain_ptrs(o, S);
      T->host.push_back(S);
    }
    for (size_t i = 0; i < g->low.size(); ++i) {
      SegInfo S{};
      S.prob = int(p);
      S.kind = 1;
      S.lx = g->low[i].lx;
      S.lv = g->low[i].lv;
      S.nx = int(g->low[i].nx);
      S.nv = int(g->low[i].nv);
      S.R = Rs;
      S.off = low_start[i];
      S.len = int64_t(Rs) * S.nx * S.nv;
      S.src_off = up_res[i + 1];
      S.low_off = -1;
      S.nx_src = int(g->up[i + 1].nx);
      fill_domain_ptrs(o, S);
      T->host.push_back(S);
    }
    ct = c;
    up = u;
  }
  finish_tab(*T);
  SegTab& ref = *T;
  B.ct_tabs[Rs] = std::move(T);
  return ref;
}

// one segment per problem over the upper-diagonal layout with Rs slices
static SegTab& prob_tab(Batch& B, int Rs) {
  auto it = B.prob_tabs.find(Rs);
  if (it != B.prob_tabs.end()) return *it->second;
  auto T = std::make_unique<SegTab>();
  int64_t off = 0;
  for (size_t p = 0; p < B.P.size(); ++p) {
    SegInfo S{};
    S.prob = int(p);
    S.kind = 2;
    S.R = Rs;
    S.off = off;
    S.len = int64_t(Rs) * up_pts(B.P[p]);
    S.low_off = -1;
    off += S.len;
    T->host.push_back(S);
  }
  finish_tab(*T);
  SegTab& ref = *T;
  B.prob_tabs[Rs] = std::move(T);
  return ref;
}

// single problem: one segment per upper grid over points (jump term)
static SegTab& pts_tab(Batch& B) {
  if (B.pts) return *B.pts;
  auto T = std::make_unique<SegTab>();
  sgdg_grid g = B.P[0]->grid;
  int64_t po = 0;
  for (auto& gd : g->up) {
    SegInfo S{};
    S.kind = 0;
    S.lx = gd.lx;
    S.lv = gd.lv;
    S.nx = int(gd.nx);
    S.nv = int(gd.nv);
    S.R = B.R;
    S.off = int64_t(B.R) * po;
    S.src_off = po;
    S.len = gd.nx * gd.nv;
    S.low_off = -1;
    po += gd.nx * gd.nv;
    T->host.push_back(S);
  }
  finish_tab(*T);
  B.pts = std::move(T);
  return *B.pts;
}

// ------------------------------------------------------ batched GMRES -----
static GmresState gstate(GBufs& b, int nseg, int m) {
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
  st.H = ptr<double>(b.H);
  st.cs = ptr<double>(b.cs);
  st.sn = ptr<double>(b.sn);
  st.g = ptr<double>(b.g);
  st.bnorm = ptr<double>(b.bn);
  st.beta = ptr<double>(b.beta);
  st.active = ptr<int>(b.act);
  st.kused = ptr<int>(b.k);
  st.hcol = ptr<double>(b.hc);
  st.inv = ptr<double>(b.inv);
  st.y = ptr<double>(b.y);
  st.m = m;
  return st;
}

// Right-preconditioned restarted GMRES on the independent grid problems
// A_{l,l} dU_l = r_l (one segment each), preconditioner M fixed and linear.
// A cycle of m iterations needs no host synchronisation.  The host polls the
// convergence flags every kPoll iterations; with use_graph each chunk of kPoll
// iterations is captured once (per buffer set and chunk) and replayed, with
// the same polls between chunks, so graph and eager solves run the same
// iterations; converged segments idle until the next poll.
constexpr int kPoll = 8;

template <class T>
static int batched_gmres(Batch& B, const SegTab& ST, const std::function<void(const T*, T*, hipStream_t)>& A,
                         const std::function<void(const T*, T*, hipStream_t)>& M, const T* b, T* x, T* V, T* w, T* tmp, int m,
                         int maxit, double tol, bool use_graph, hipStream_t s, bool* nan) {
  const SegTable& S = ST.t;
  const int nseg = S.nseg;
  const int64_t total = ST.host.back().off + ST.host.back().len;
  GBufs& gb = B.gb[0];
  gb.partial.ensure(sizeof(double) * size_t(S.nchunks) * (m + 1));
  double* part = ptr<double>(gb.partial);
  GmresState st = gstate(gb, nseg, m);
  KernelsT<T>::fill(total, T(0), x, s);
  std::vector<int> act(nseg);
  bool bad = false;
  int it = 0;
  auto step = [&](int j, hipStream_t q) {
    M(V + int64_t(j) * total, tmp, q);
    A(tmp, w, q);
    // CGS2: two projection passes; the first pass's update and the second
    // pass's projections share one read of the basis
    KernelsT<T>::seg_dots(S, V, total, j + 1, w, part, q);
    gmres_add_proj(nseg, st, S.segs, part, j, q);
    KernelsT<T>::seg_axpy_dots(S, V, total, j + 1, st.hcol, m + 1, w, part, q);
    gmres_add_proj(nseg, st, S.segs, part, j, q);
    KernelsT<T>::seg_axpy(S, V, total, j + 1, st.hcol, m + 1, w, -1.0, part, q);
    gmres_givens(nseg, st, S.segs, part, j, tol, q);
    KernelsT<T>::seg_scale(S, w, st.inv, V + int64_t(j + 1) * total, q);
  };
  auto any_active = [&]() {
    SGDG_CHECK_HIP(hipMemcpyAsync(act.data(), st.active, sizeof(int) * nseg, hipMemcpyDeviceToHost, s));
    SGDG_CHECK_HIP(hipStreamSynchronize(s));
    bool any = false;
    for (int a : act) {
      any = any || a == 1;
      bad = bad || a == -1;
    }
    return any;
  };
  for (int cycle = 0; it < maxit; ++cycle) {
    KernelsT<T>::copy(total, b, V, s);
    if (cycle > 0) {
      A(x, w, s);
      KernelsT<T>::axpby(total, T(-1), w, T(1), V, s);
    }
    KernelsT<T>::seg_norm2(S, V, part, s);
    gmres_start(nseg, st, S.segs, part, tol, cycle == 0, s);
    KernelsT<T>::seg_scale(S, V, st.inv, V, s);
    if (!any_active()) break;
    const int mm = std::min(m, maxit - it);
    int j = 0;
    if (use_graph && mm == m) {
      // a graph replays the device addresses it was captured with: any
      // buffer or table reallocated since then invalidates every graph
      if (B.graph_epoch != alloc_epoch()) {
        SGDG_CHECK_HIP(hipStreamSynchronize(s));
        B.clear_graphs();
        B.graph_epoch = alloc_epoch();
      }
      // the cycle in chunks of kPoll iterations, one graph per chunk, with the
      // same convergence polls between chunks as the eager loop below
      std::ostringstream base;
      base << sizeof(T) << '/' << m << '/' << total << '/' << (const void*)V << '/' << (const void*)w << '/'
           << (const void*)tmp << '/' << (const void*)part << '/' << (const void*)st.H << '/' << (const void*)b
           << '/' << B.variant << '/' << B.split_bc << '/' << B.split_xcd << '/' << B.scan_chunks;
      bool warmed = false;
      while (j < mm) {
        const int j1 = std::min(mm, j + kPoll);
        std::ostringstream key;
        key << base.str() << '/' << j << '-' << j1;
        auto g = B.graphs.find(key.str());
        if (g == B.graphs.end()) {
          if (!warmed) {
            // One eager application of M and A first: workspaces and item tables
            // are created on first use, and allocation and table uploads cannot be
            // captured.  Its result is overwritten by the cycle.
            M(V + int64_t(j) * total, tmp, s);
            A(tmp, w, s);
            SGDG_CHECK_HIP(hipStreamSynchronize(s));
            if (B.graph_epoch != alloc_epoch()) {  // the warm-up allocated: older graphs may be stale
              B.clear_graphs();
              B.graph_epoch = alloc_epoch();
            }
            warmed = true;
          }
          // capture on a private stream (the caller's may be the null stream, which cannot be captured)
          if (!B.cap_stream) SGDG_CHECK_HIP(hipStreamCreate(&B.cap_stream));
          const bool prof = B.prof;
          B.prof = false;
          hipGraph_t graph = nullptr;
          SGDG_CHECK_HIP(hipStreamBeginCapture(B.cap_stream, hipStreamCaptureModeThreadLocal));
          try {
            for (int jj = j; jj < j1; ++jj) step(jj, B.cap_stream);
          } catch (...) {
            (void)hipStreamEndCapture(B.cap_stream, &graph);
            if (graph) (void)hipGraphDestroy(graph);
            B.prof = prof;
            throw;
          }
          B.prof = prof;
          SGDG_CHECK_HIP(hipStreamEndCapture(B.cap_stream, &graph));
          hipGraphExec_t exec = nullptr;
          const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
          (void)hipGraphDestroy(graph);
          SGDG_CHECK_HIP(e);
          g = B.graphs.emplace(key.str(), exec).first;
          // instantiation allocates no DevBuf: the epoch still matches the capture
          require(B.graph_epoch == alloc_epoch(), "work buffers changed during graph capture");
        }
        timed(B, 2, s, [&] { SGDG_CHECK_HIP(hipGraphLaunch(g->second, s)); });
        j = j1;
        if (j < mm && !any_active()) break;
      }
    } else {
      timed(B, 2, s, [&] {
        for (; j < mm; ++j) {
          step(j, s);
          if ((j + 1) % kPoll == 0 && j + 1 < mm && !any_active()) {
            ++j;
            break;
          }
        }
      });
    }
    it += j;
    gmres_lsq(nseg, st, s);
    KernelsT<T>::fill(total, T(0), w, s);
    KernelsT<T>::seg_axpy(S, V, total, j, st.y, m, w, 1.0, nullptr, s);
    M(w, tmp, s);
    KernelsT<T>::axpby(total, T(1), tmp, T(1), x, s);
  }
  *nan = *nan || bad;
  return it;
}

// ------------------------------------- x-transport preconditioner tables ---
// For every grid-problem segment: the terms of the strip operator whose
// x-factor is translation invariant (no x-field weight, not a face) and whose
// v-factor is a mass matrix, the v-factor lumped to its row sums.  On a
// periodic x-lattice these form, for every v-node q, a circulant operator in
// x; its action on the Fourier mode theta is the R x R matrix
//   sum_terms Tm_k * xhat_k(theta) * lambda_k(q),
//   xhat_k(theta) = sum_slots c_e exp(i theta . o_e)  (the stencil of any row),
//   lambda_k(q) = sum_e V_k[q, e],
// which the tables hold inverted, one per (mode, v-node).
static FourierTab& fourier_tab(Batch& B, SegTab& ST) {
  if (ST.fourier) return ST.ftab;
  using cd = std::complex<double>;
  std::vector<FourierSeg> fs;
  std::vector<int2> lines;
  std::vector<double> pinv;
  const int d = B.d;
  for (size_t gi = 0; gi < ST.host.size(); ++gi) {
    const SegInfo& S = ST.host[gi];
    sgdg_ops o = B.P[size_t(S.prob)];
    const DomainData& X = o->X;
    const DomainData& V = o->V;
    require(X.dom.periodic, "the x-transport preconditioner needs a periodic x-domain");
    const int n1 = X.dom.axis_nodes(S.lx);
    require(n1 <= 1024, "the x-transport preconditioner takes at most 1024 nodes per x-axis");
    const int R = S.R;
    FourierSeg F{};
    F.off = S.off;
    F.poff = int64_t(pinv.size() / 2);
    F.nx = S.nx;
    F.nv = S.nv;
    F.R = R;
    F.n1 = n1;
    F.d = d;
    fs.push_back(F);
    const int Sx = X.st.S, Sv = V.st.S;
    const int lxi = S.lx - X.lmin, lvi = S.lv - V.lmin;
    const LevelTables& VL = V.L(S.lv);
    struct Sel {
      const Term* t;
      std::vector<cd> sym;
      std::vector<double> lam;
    };
    std::vector<Sel> sel;
    for (const Term& t : o->ops[0].host.terms) {
      const FactorKey& kx = X.factors[size_t(t.xf)];
      const FactorKey& kv = V.factors[size_t(t.vf)];
      if (kx.kind == kFace || !factor_plain(X, t.xf) || kv.kind != kMass) continue;
      const std::vector<double>& xv = X.values[size_t(t.xf)][size_t(lxi)];
      // translation invariance: every row repeats row 0
      for (int64_t r = 0; r < S.nx; ++r)
        for (int e = 0; e < Sx; ++e)
          require(std::fabs(xv[size_t(r * Sx + e)] - xv[size_t(e)]) <= 1e-12 * (1.0 + std::fabs(xv[size_t(e)])),
                  "an x-factor of the x-transport part is not translation invariant");
      Sel z;
      z.t = &t;
      z.sym.resize(size_t(S.nx));
      for (int64_t m = 0; m < S.nx; ++m) {
        int64_t rem = m;
        double th[3] = {0, 0, 0};
        for (int a = d - 1; a >= 0; --a) {
          th[a] = 2.0 * M_PI * double(rem % n1) / double(n1);
          rem /= n1;
        }
        cd acc = 0;
        for (int e = 0; e < Sx; ++e) {
          double ph = 0;
          for (int a = 0; a < d; ++a) ph += th[a] * X.st.off[e][a];
          acc += xv[size_t(e)] * cd(std::cos(ph), std::sin(ph));
        }
        z.sym[size_t(m)] = acc;
      }
      const std::vector<double>& vv = V.values[size_t(t.vf)][size_t(lvi)];
      z.lam.assign(size_t(S.nv), 0.0);
      for (int64_t q = 0; q < S.nv; ++q)
        for (int e = 0; e < Sv; ++e)
          if (VL.valid[size_t(q * Sv + e)]) z.lam[size_t(q)] += vv[size_t(q * Sv + e)];
      sel.push_back(std::move(z));
    }
    require(!sel.empty(), "no translation-invariant terms for the x-transport preconditioner");
    std::vector<cd> P(size_t(R * R)), Inv(size_t(R * R));
    for (int64_t m = 0; m < S.nx; ++m)
      for (int64_t q = 0; q < S.nv; ++q) {
        std::fill(P.begin(), P.end(), cd(0));
        for (const Sel& z : sel) {
          const cd f = z.sym[size_t(m)] * z.lam[size_t(q)];
          for (int i = 0; i < R * R; ++i) P[size_t(i)] += z.t->tm[i] * f;
        }
        // Gauss-Jordan with partial pivoting
        std::vector<cd> A = P;
        for (int i = 0; i < R * R; ++i) Inv[size_t(i)] = (i / R == i % R) ? cd(1) : cd(0);
        for (int c = 0; c < R; ++c) {
          int pr = c;
          for (int r = c + 1; r < R; ++r)
            if (std::abs(A[size_t(r * R + c)]) > std::abs(A[size_t(pr * R + c)])) pr = r;
          require(std::abs(A[size_t(pr * R + c)]) > 1e-300, "singular mode of the x-transport preconditioner");
          if (pr != c)
            for (int k = 0; k < R; ++k) {
              std::swap(A[size_t(c * R + k)], A[size_t(pr * R + k)]);
              std::swap(Inv[size_t(c * R + k)], Inv[size_t(pr * R + k)]);
            }
          const cd piv = A[size_t(c * R + c)];
          for (int k = 0; k < R; ++k) {
            A[size_t(c * R + k)] /= piv;
            Inv[size_t(c * R + k)] /= piv;
          }
          for (int r = 0; r < R; ++r) {
            if (r == c) continue;
            const cd f = A[size_t(r * R + c)];
            for (int k = 0; k < R; ++k) {
              A[size_t(r * R + k)] -= f * A[size_t(c * R + k)];
              Inv[size_t(r * R + k)] -= f * Inv[size_t(c * R + k)];
            }
          }
        }
        for (int i = 0; i < R * R; ++i) {
          pinv.push_back(Inv[size_t(i)].real());
          pinv.push_back(Inv[size_t(i)].imag());
        }
      }
    int64_t other = 1;
    for (int a = 0; a < d - 1; ++a) other *= n1;
    const int64_t nl = int64_t(R) * S.nv * other;
    for (int64_t l = 0; l < nl; ++l) lines.push_back(int2{int(gi), int(l)});
  }
  upload(ST.fsegs, fs);
  upload(ST.flines, lines);
  upload(ST.fpinv, pinv);
  ST.ftab.d = d;
  ST.ftab.nlines = int(lines.size());
  ST.ftab.segs = ptr<FourierSeg>(ST.fsegs);
  ST.ftab.lines = ptr<int2>(ST.flines);
  ST.ftab.pinv = ptr<double>(ST.fpinv);
  ST.fourier = true;
  return ST.ftab;
}

static int64_t seg_total(const SegTab& ST) {
  return ST.host.empty() ? 0 : ST.host.back().off + ST.host.back().len;
}

// ------------------------------------------- grid-problem preconditioner ---
// Chebyshev semi-iteration coefficients for M z = b with the Jacobi splitting:
// the eigenvalues of D^-1 M of the P1 mass matrix on Kuhn simplices lie in
// [1/2, 1 + d/2] (element by element, the Jacobi-scaled element mass matrix
// of a d-simplex has the eigenvalues 1/2 and 1 + d/2), so after k steps the
// error is reduced by the Chebyshev factor of that interval.  Step 0 is
// z_1 = D^-1 b / theta; step k >= 1 is d_k = rho_k rho_{k-1} d_{k-1} +
// (2 rho_k / delta) D^-1 (b - M z_k), z_{k+1} = z_k + d_k, with
// rho_k = 1 / (2 sigma - rho_{k-1}), rho_0 = 1 / sigma (Chebyshev
// acceleration of a splitting, e.g. Saad's Iterative Methods, Sect. 12.3).
static void mass_cheb_coefs(int d, int k, double* cd, double* cr) {
  const double lmin = 0.5, lmax = 1.0 + 0.5 * d;
  const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin), sigma = theta / delta;
  double rho_prev = 1.0 / sigma;
  if (k == 0) {
    *cd = 0;
    *cr = 1.0 / theta;
    return;
  }
  double rho = rho_prev;
  for (int i = 1; i <= k; ++i) {
    rho = 1.0 / (2 * sigma - rho_prev);
    if (i < k) rho_prev = rho;
  }
  *cd = rho * rho_prev;
  *cr = 2 * rho / delta;
}

static void check_mass(const sgdg_precond_opts& po, int d) {
  require(po.mass_sweeps >= -2 && po.mass_sweeps <= 64, "mass_sweeps must be -2..64");
  require(po.mass_sweeps != -1 || d == 1, "mass_sweeps = -1 (exact tridiagonal mass solves) needs d = 1");
}

// The preconditioner of the grid problems (Sect. 4.3): the inverse of
// (Tt + delta Ct + Gt) (x) M^x (x) M^v on every segment.  sweeps 0: the mass
// matrices replaced by their diagonals; k > 0: k Chebyshev-Jacobi steps per
// mass factor (a fixed polynomial, so a fixed linear map); -1 (d = 1): the
// mass factors inverted exactly, one tridiagonal solve per grid line.  The
// mass factors act on different axes and commute with the time block, so the
// x-solve, the v-solve and the time block run one after the other.
template <class T>
static void mass_precond(Batch& B, const SegTab& ST, int sweeps, const T* in, T* out, hipStream_t q) {
  const SegTable& S = ST.t;
  BWork<T>& w = work<T>(B);
  if (sweeps == 0) {
    KernelsT<T>::minv(S, in, out, q);
    return;
  }
  if (sweeps == -2) {
    const int64_t total = seg_total(ST);
    B.fourier_c.ensure(sizeof(double) * 2 * size_t(total));
    fourier_precond_n<T>(fourier_tab(B, const_cast<SegTab&>(ST)), S, total, in, out, ptr<double>(B.fourier_c), q);
    return;
  }
  if (sweeps < 0) {
    int lx = 0, lv = 0;
    for (const SegInfo& g : ST.host) {
      lx = std::max(lx, g.R * g.nv);
      lv = std::max(lv, g.R * g.nx);
    }
    T* c = ptr<T>(w.mX0);
    T* z = ptr<T>(w.mX1);
    KernelsT<T>::mass_thomas(S, 0, lx, in, out, c, z, q);
    KernelsT<T>::mass_thomas(S, 1, lv, out, out, c, z, q);
    KernelsT<T>::tinv(S, out, out, q);
    return;
  }
  T* xs[2] = {ptr<T>(w.mX0), ptr<T>(w.mX1)};
  T* ds[2] = {ptr<T>(w.mD0), ptr<T>(w.mD1)};
  for (int axis = 0; axis < 2; ++axis) {
    const T* b = axis == 0 ? in : ptr<T>(w.mU);
    T* dst = axis == 0 ? ptr<T>(w.mU) : out;
    for (int k = 0; k < sweeps; ++k) {
      double cd, cr;
      mass_cheb_coefs(B.d, k, &cd, &cr);
      const bool last = k + 1 == sweeps;
      T* xo = last ? dst : xs[k & 1];
      T* dout = last ? nullptr : ds[k & 1];
      KernelsT<T>::mass_cheb(S, axis, cd, cr, k == 0 ? 1 : 0, (last && axis == 1) ? 1 : 0, b,
                             k == 0 ? nullptr : xs[(k - 1) & 1], k == 0 ? nullptr : ds[(k - 1) & 1], xo, dout, q);
    }
  }
}

// --------------------------------------------------- CT preconditioner ----
template <class T>
static void ct_apply(Batch& B, const T* r, T* z, const sgdg_precond_opts& po, bool use_graph, hipStream_t s,
                     bool* nan) {
  SegTab& ST = ct_tab(B, B.R);
  const int64_t nct = kind(B, K_CT).total;
  BWork<T>& w = work<T>(B);
  const int m = std::max(1, std::min(po.inner_restart, 64));
  w.ctb.ensure(sizeof(T) * nct);
  w.ctx.ensure(sizeof(T) * nct);
  w.ctw.ensure(sizeof(T) * nct);
  w.cttmp.ensure(sizeof(T) * nct);
  w.ctV.ensure(sizeof(T) * nct * (m + 1));
  if (po.mass_sweeps != 0) {
    w.mU.ensure(sizeof(T) * nct);
    w.mX0.ensure(sizeof(T) * nct);
    w.mX1.ensure(sizeof(T) * nct);
    w.mD0.ensure(sizeof(T) * nct);
    w.mD1.ensure(sizeof(T) * nct);
  }
  T* b = ptr<T>(w.ctb);
  KernelsT<T>::ct_gather(ST.t, r, b, s);
  items(B, K_CT, int(sizeof(T)));  // tables exist before any capture
  if (po.mass_sweeps == -2) {
    fourier_tab(B, ST);
    B.fourier_c.ensure(sizeof(double) * 2 * size_t(nct));
  }
  const int sweeps = po.mass_sweeps;
  auto A = [&](const T* in, T* out, hipStream_t q) { apply<T>(B, K_CT, in, out, 1, q); };
  auto M = [&](const T* in, T* out, hipStream_t q) { mass_precond<T>(B, ST, sweeps, in, out, q); };
  B.inner_iters += batched_gmres<T>(B, ST, A, M, b, ptr<T>(w.ctx), ptr<T>(w.ctV), ptr<T>(w.ctw), ptr<T>(w.cttmp), m,
                                    po.inner_maxit, po.inner_rtol, use_graph, s, nan);
  KernelsT<T>::ct_combine(ST.t, ptr<T>(w.ctx), z, s);
}

static sgdg_precond_opts default_pc() {
  sgdg_precond_opts p{};
  p.kind = 0;
  p.inner_rtol = 1e-8;
  p.inner_maxit = 200;
  p.inner_restart = 30;
  p.mass_sweeps = 0;
  return p;
}

// ------------------------------------------------------------- FGMRES -----
struct FgmresResult {
  int iters = 0;
  double rel = 0;  // largest relative residual over the problems
  bool nan = false;
};

static std::vector<double> seg_norms(Batch& B, const SegTab& ST, const double* v, hipStream_t s) {
  GBufs& gb = B.gb[2];
  gb.partial.ensure(sizeof(double) * ST.t.nchunks);
  KernelsT<double>::seg_norm2(ST.t, v, ptr<double>(gb.partial), s);
  std::vector<double> h(ST.t.nchunks);
  SGDG_CHECK_HIP(hipMemcpyAsync(h.data(), gb.partial.p, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
  SGDG_CHECK_HIP(hipStreamSynchronize(s));
  std::vector<double> out(ST.host.size(), 0.0);
  for (size_t i = 0; i < ST.host.size(); ++i) {
    double a = 0;
    for (int c = 0; c < ST.host[i].nchunk; ++c) a += h[ST.host[i].chunk0 + c];
    out[i] = std::sqrt(a);
  }
  return out;
}

// Flexible GMRES on every problem of the batch in lockstep (one segment per
// problem, FP64 Arnoldi), stopping per problem at ||b - A u|| <= tol ||b||.
// monitor(iterations, largest relative residual estimate, largest relative residual at entry)
// called after every FGMRES iteration with (iteration, residual estimate, residual at
// entry); true ends the current cycle (restart from the true residual)
using Monitor = std::function<bool(int, double, double)>;

static FlagRing& flag_ring(Batch& B, int nseg) {
  if (!B.flags) B.flags.reset(new FlagRing);
  FlagRing& f = *B.flags;
  if (f.cap >= nseg) return f;
  f.release();
  for (int i = 0; i < 2; ++i) {
    SGDG_CHECK_HIP(hipHostMalloc(reinterpret_cast<void**>(&f.act[i]), sizeof(int) * nseg, hipHostMallocDefault));
    SGDG_CHECK_HIP(hipHostMalloc(reinterpret_cast<void**>(&f.beta[i]), sizeof(double) * nseg, hipHostMallocDefault));
    SGDG_CHECK_HIP(hipEventCreateWithFlags(&f.ev[i], hipEventDisableTiming));
  }
  f.cap = nseg;
  return f;
}
static FgmresResult fgmres(Batch& B, const std::function<void(const double*, double*)>& A,
                           const std::function<void(const double*, double*)>& P, const double* b, double* x,
                           double tol, int m, int maxit, hipStream_t s, const Monitor* monitor = nullptr,
                           const bool* pipelined = nullptr) {
  SegTab& ST = prob_tab(B, B.R);
  const SegTable& S = ST.t;
  const int nseg = S.nseg;
  const int64_t n = kind(B, K_FULL).total;
  B.fV.ensure(sizeof(double) * n * (m + 1));
  B.fZ.ensure(sizeof(double) * n * m);
  B.fw.ensure(sizeof(double) * n);
  double* V = ptr<double>(B.fV);
  double* Z = ptr<double>(B.fZ);
  double* w = ptr<double>(B.fw);
  GBufs& gb = B.gb[1];
  gb.partial.ensure(sizeof(double) * size_t(S.nchunks) * (m + 1));
  double* part = ptr<double>(gb.partial);
  GmresState st = gstate(gb, nseg, m);
  const bool verbose = getenv("SGDG_VERBOSE") != nullptr;
  FgmresResult res;
  // ||b|| per problem into st.bnorm
  KernelsT<double>::seg_norm2(S, b, part, s);
  gmres_start(nseg, st, S.segs, part, 0.0, 1, s);
  const std::vector<double> bn = seg_norms(B, ST, b, s);
  for (double v : bn)
    if (!std::isfinite(v)) {
      res.nan = true;
      return res;
    }
  for (int i = 0; i < nseg; ++i)  // b = 0 has the solution 0
    if (bn[i] == 0.0) KernelsT<double>::fill(ST.host[i].len, 0.0, x + ST.host[i].off, s);
  double rel0 = -1;
  for (;;) {
    A(x, w);
    KernelsT<double>::copy(n, b, V, s);
    KernelsT<double>::axpby(n, -1.0, w, 1.0, V, s);
    const std::vector<double> rn = seg_norms(B, ST, V, s);
    res.rel = 0;
    bool nanr = false;
    for (int i = 0; i < nseg; ++i) {
      const double rel = bn[i] > 0 ? rn[i] / bn[i] : 0.0;
      nanr = nanr || !std::isfinite(rel);
      res.rel = std::max(res.rel, rel);
    }
    if (verbose) fprintf(stderr, "[sgdg fgmres] true residual %.3e after %d\n", res.rel, res.iters);
    if (nanr) {
      res.nan = true;
      return res;
    }
    if (rel0 < 0) rel0 = res.rel;
    if (res.rel <= tol || res.iters >= maxit) return res;
    KernelsT<double>::seg_norm2(S, V, part, s);
    gmres_start(nseg, st, S.segs, part, tol, 0, s);  // converged problems start inactive
    KernelsT<double>::seg_scale(S, V, st.inv, V, s);
    const int mm = std::min(m, maxit - res.iters);
    // The flags and residual estimates of iteration j are copied to pinned host
    // memory behind its launches.  While the preconditioner runs on the device
    // alone (*pipelined: the learned map), they are read one iteration late,
    // after the launches of iteration j + 1 are queued, so the device does not
    // wait for the host between iterations; an iteration run past a segment's
    // convergence leaves that segment untouched (inactive segments take no
    // rotation and count no iteration), so stopping one iteration late changes
    // no result.  Otherwise (the combination technique, which synchronises
    // inside) they are read at once, so no preconditioner application is
    // spent after convergence.
    FlagRing& fr = flag_ring(B, nseg);
    enum { GO, CONVERGED, RESTART, BAD };
    auto evaluate = [&](int e) {
      const int* a = fr.act[e & 1];
      const double* be = fr.beta[e & 1];
      SGDG_CHECK_HIP(hipEventSynchronize(fr.ev[e & 1]));
      bool any = false, bad = false;
      double est = 0;
      for (int i = 0; i < nseg; ++i) {
        any = any || a[i] == 1;
        bad = bad || a[i] == -1;
        if (bn[i] > 0) est = std::max(est, be[i] / bn[i]);
      }
      if (verbose) fprintf(stderr, "[sgdg fgmres] it %d  est %.3e\n", res.iters + e + 1, est);
      const bool restart = monitor && (*monitor)(res.iters + e + 1, est, rel0);
      if (bad) return int(BAD);
      if (!any) return int(CONVERGED);
      return restart ? int(RESTART) : int(GO);
    };
    int j = 0, pending = -1, used = -1, ran = 0;
    for (; j < mm; ++j) {
      ran = j + 1;  // iterations queued (their directions Z_0..Z_j enter the update)
      P(V + int64_t(j) * n, Z + int64_t(j) * n);
      A(Z + int64_t(j) * n, w);
      // CGS2, the first update fused with the second projections
      KernelsT<double>::seg_dots(S, V, n, j + 1, w, part, s);
      gmres_add_proj(nseg, st, S.segs, part, j, s);
      KernelsT<double>::seg_axpy_dots(S, V, n, j + 1, st.hcol, m + 1, w, part, s);
      gmres_add_proj(nseg, st, S.segs, part, j, s);
      KernelsT<double>::seg_axpy(S, V, n, j + 1, st.hcol, m + 1, w, -1.0, part, s);
      gmres_givens(nseg, st, S.segs, part, j, tol * 0.5, s);
      KernelsT<double>::seg_scale(S, w, st.inv, V + int64_t(j + 1) * n, s);
      SGDG_CHECK_HIP(hipMemcpyAsync(fr.act[j & 1], st.active, sizeof(int) * nseg, hipMemcpyDeviceToHost, s));
      SGDG_CHECK_HIP(hipMemcpyAsync(fr.beta[j & 1], st.beta, sizeof(double) * nseg, hipMemcpyDeviceToHost, s));
      SGDG_CHECK_HIP(hipEventRecord(fr.ev[j & 1], s));
      const bool lag = pipelined && *pipelined;
      int v = GO, e = -1;
      if (pending >= 0) {
        e = pending;
        v = evaluate(e);
      }
      pending = j;
      if (v == GO && !lag) {
        e = j;
        v = evaluate(e);
        pending = -1;
      }
      if (v != GO) {
        if (v == BAD) {
          res.nan = true;
          return res;
        }
        // converged at iteration e: the iterations after it did nothing
        used = v == CONVERGED ? e + 1 : j + 1;
        break;
      }
    }
    if (used < 0) {
      used = j;
      if (pending >= 0 && evaluate(pending) == BAD) {  // the cycle's last iteration
        res.nan = true;
        return res;
      }
    }
    res.iters += used;
    gmres_lsq(nseg, st, s);
    // y has kused entries per segment (zeros beyond): every queued direction may enter
    KernelsT<double>::seg_axpy(S, Z, n, ran, st.y, m, x, 1.0, nullptr, s);
  }
}

// The learned preconditioner's fallback rule: over any `iters` consecutive
// learned FGMRES iterations of one FGMRES call the residual estimate must drop
// by the factor `drop`.  Estimates are relative to that call's right-hand side
// (in mixed precision each refinement step solves for its own residual), so the
// history restarts with every call.
struct FallbackMonitor {
  int iters;
  double drop;
  std::vector<double> hist;  // estimate at entry, then after each learned iteration
  FallbackMonitor(int it, double dr) : iters(it), drop(dr) {}
  void begin() { hist.clear(); }
  // true: switch to the combination technique now
  bool step(double est, double rel0) {
    if (hist.empty()) hist.push_back(rel0);
    hist.push_back(est);
    const size_t k = hist.size() - 1;
    return k >= size_t(iters) && est > hist[k - size_t(iters)] / drop;
  }
};

static sgdg_solve_stats solve_batch(Batch& B, const double* b, double* u, const sgdg_solve_opts& so, hipStream_t s,
                                    bool* nan) {
  const auto t0 = std::chrono::steady_clock::now();
  const int64_t n = kind(B, K_FULL).total;
  sgdg_precond_opts pc = so.pc;
  if (pc.inner_restart <= 0) {  // unset inner options: defaults, keeping the kind and network
    const sgdg_precond_opts d = default_pc();
    pc.inner_rtol = d.inner_rtol;
    pc.inner_maxit = d.inner_maxit;
    pc.inner_restart = d.inner_restart;
  }
  const bool graph = so.use_graph != 0;
  B.inner_iters = 0;
  // preconditioner: combination technique, or the learned network until it
  // fails to reduce the residual estimate by fallback_drop within fallback_iters
  // iterations (FGMRES admits a change of preconditioner between iterations)
  const bool learned = pc.kind == 1;
  bool use_ct = !learned, fell_back = false;
  int pc_apps = 0;
  const int fb_iters = pc.fallback_iters > 0 ? pc.fallback_iters : 10;
  const double fb_drop = pc.fallback_drop > 1 ? pc.fallback_drop : 10.0;
  sgdg_net rec = B.owned_by_ops ? B.P[0]->recorder : nullptr;
  FallbackMonitor fb(fb_iters, fb_drop);
  // At the switch the cycle ends: the combination technique then starts a
  // fresh Krylov space from the true residual instead of extending the basis
  // the network built.
  // the learned map runs on the device alone: FGMRES may read its flags late
  bool device_only_pc = !use_ct;
  const Monitor monitor = [&](int it, double est, double rel0) {
    (void)it;
    if (use_ct) return false;
    if (fb.step(est, rel0)) {
      use_ct = true;
      device_only_pc = false;
      fell_back = true;
      return true;
    }
    return false;
  };
  auto A64 = [&](const double* in, double* out) { apply<double>(B, K_FULL, in, out, 1, s); };
  // the learned map: one network per problem, each on its problem's slice
  auto learned_apply = [&](const double* in, double* out) {
    if (B.nets.empty()) {
      net_apply_dev(pc.net, in, out, s);
      return;
    }
    int64_t off = 0;
    for (size_t i = 0; i < B.P.size(); ++i) {
      net_apply_dev(B.nets[i], in + off, out + off, s);
      off += int64_t(B.R) * B.P[i]->grid->up_pts;
    }
  };
  auto P64 = [&](const double* in, double* out) {
    ++pc_apps;
    if (!use_ct) {
      learned_apply(in, out);
      return;
    }
    ct_apply<double>(B, in, out, pc, graph, s, nan);
    if (rec) net_record_pair(rec, in, out, s);
  };
  sgdg_solve_stats st{};
  if (!so.mixed_precision) {
    FgmresResult r =
        fgmres(B, A64, P64, b, u, so.rtol, so.restart, so.maxit, s, learned ? &monitor : nullptr, &device_only_pc);
    st.outer_iters = r.iters;
    st.rel_residual = r.rel;
    *nan = *nan || r.nan;
  } else {
    // FP64 iterative refinement; each correction solved by FGMRES with FP32
    // operator applications and an FP32 combination-technique preconditioner.
    B.a32.ensure(sizeof(float) * n);
    B.b32.ensure(sizeof(float) * n);
    B.fr.ensure(sizeof(double) * n);
    B.fe.ensure(sizeof(double) * n);
    B.ftmp.ensure(sizeof(double) * n);
    float* a32 = ptr<float>(B.a32);
    float* b32 = ptr<float>(B.b32);
    sgdg_precond_opts pc32 = pc;
    pc32.inner_rtol = std::max(pc.inner_rtol, 1e-5);  // FP32 grid problems cannot reach FP64 tolerances
    auto A32 = [&](const double* in, double* out) {
      convert_f64_to_f32(n, in, a32, s);
      apply<float>(B, K_FULL, a32, b32, 1, s);
      convert_f32_to_f64(n, b32, out, s);
    };
    auto P32 = [&](const double* in, double* out) {
      ++pc_apps;
      if (!use_ct) {
        learned_apply(in, out);
        return;
      }
      convert_f64_to_f32(n, in, a32, s);
      ct_apply<float>(B, a32, b32, pc32, graph, s, nan);
      convert_f32_to_f64(n, b32, out, s);
      if (rec) net_record_pair(rec, in, out, s);
    };
    double* rr = ptr<double>(B.fr);
    double* e = ptr<double>(B.fe);
    double* tmp = ptr<double>(B.ftmp);
    const double inner_tol = so.inner_outer_rtol > 0 ? so.inner_outer_rtol : 1e-4;
    SegTab& ST = prob_tab(B, B.R);
    const std::vector<double> bn = seg_norms(B, ST, b, s);
    int total = 0, steps = 0;
    double rel = 1;
    for (;;) {
      A64(u, tmp);
      KernelsT<double>::copy(n, b, rr, s);
      KernelsT<double>::axpby(n, -1.0, tmp, 1.0, rr, s);
      const std::vector<double> rn = seg_norms(B, ST, rr, s);
      rel = 0;
      for (size_t i = 0; i < rn.size(); ++i) rel = std::max(rel, bn[i] > 0 ? rn[i] / bn[i] : 0.0);
      if (!std::isfinite(rel)) {
        *nan = true;
        break;
      }
      if (rel <= so.rtol || total >= so.maxit || steps >= 20) break;
      KernelsT<double>::fill(n, 0.0, e, s);
      fb.begin();  // estimates of this correction solve are relative to its own right-hand side
      FgmresResult ri = fgmres(B, A32, P32, rr, e, inner_tol, so.restart, so.maxit - total, s,
                               learned ? &monitor : nullptr, &device_only_pc);
      total += std::max(ri.iters, 1);
      ++steps;
      if (ri.nan) {
        *nan = true;
        break;
      }
      KernelsT<double>::axpby(n, 1.0, e, 1.0, u, s);
    }
    st.outer_iters = total;
    st.refinement_steps = steps;
    st.rel_residual = rel;
  }
  SGDG_CHECK_HIP(hipStreamSynchronize(s));
  st.fallback_used = fell_back ? 1 : 0;
  st.pc_applications = pc_apps;
  st.inner_iters_total = int(B.inner_iters);
  st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return st;
}

// ------------------------------------------------------------------ data --
static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0);
  w.assign(n, 0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      const double pn = n == 1 ? z : p1, pm = n == 1 ? 1 : p0;
      dp = n * (z * pn - pm) / (z * z - 1);
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
    dp = n * (z * pn - pm) / (z * z - 1);
    x[i] = z;
    w[i] = 2.0 / ((1 - z * z) * dp * dp);
  }
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

// nodal [nq][up nodes + low nodes] -> slices (projection weights) in the CT
// layout [upper grids][lower grids] -> combination into spanning coefficients
static void nodal_to_coef(Batch& B, const double* samples, int nq, const double* wts_host, int Rs, double* coef,
                          hipStream_t s) {
  sgdg_grid g = B.P[0]->grid;
  const int64_t nall = g->up_pts + g->low_pts;
  B.rhs_w.ensure(sizeof(double) * Rs * nq);
  SGDG_CHECK_HIP(hipStreamSynchronize(s));  // rhs_w may still be read by earlier work
  SGDG_CHECK_HIP(hipMemcpy(B.rhs_w.p, wts_host, sizeof(double) * Rs * nq, hipMemcpyHostToDevice));
  B.rhs_a.ensure(sizeof(double) * Rs * nall);
  B.rhs_b.ensure(sizeof(double) * Rs * nall);
  double* proj = ptr<double>(B.rhs_a);
  double* blk = ptr<double>(B.rhs_b);
  project_time(nall, nq, Rs, ptr<double>(B.rhs_w), samples, proj, s);
  int64_t node = 0, out = 0;
  for (int part = 0; part < 2; ++part) {
    const auto& gs = part == 0 ? g->up : g->low;
    for (const auto& gd : gs) {
      const int64_t np = gd.nx * gd.nv;
      for (int sl = 0; sl < Rs; ++sl)
        SGDG_CHECK_HIP(hipMemcpyAsync(blk + out + sl * np, proj + int64_t(sl) * nall + node, sizeof(double) * np,
                                      hipMemcpyDeviceToDevice, s));
      node += np;
      out += int64_t(Rs) * np;
    }
  }
  KernelsT<double>::ct_combine(ct_tab(B, Rs).t, blk, coef, s);
}

// ------------------------------------------------------------ autotuner --
struct TuneCfg {
  int variant, bc, xbox, xcd;
  int chunks = 1;  // blocks sharing a scan item's factor groups
};

static std::vector<TuneCfg> tune_candidates(int d) {
  std::vector<TuneCfg> c;
  for (int variant : {0, 2})
    for (int bc : {1, 2, 4})
      for (int xcd : {0, 1})
        if (bc == 1 || (d < 3 && (variant == 0 || bc == 2))) c.push_back({variant, bc, 0, xcd});
  const int base = d == 1 ? 32 : (d == 2 ? 8 : 4);
  for (int xb : {base / 2, base, base * 2}) c.push_back({1, 0, xb, 0});
  return c;
}

static std::string tune_key(const Batch& B, int elem, int nb) {
  std::ostringstream k;
  k << "v3_d" << B.d << "_R" << B.R << "_e" << elem << "_b" << nb << "_p" << B.P.size() << "_g";
  for (sgdg_ops o : B.P) {
    for (const auto& gd : o->grid->up) k << gd.lx << "." << gd.lv << ",";
    k << (o->grid->x.periodic ? "P" : "N") << (o->grid->v.periodic ? "P" : "N") << ";";
  }
  return k.str();
}

static std::string tune_cache_path() {
  if (const char* p = getenv("SGDG_TUNE_CACHE")) return p;
  const char* h = getenv("HOME");
  return std::string(h ? h : ".") + "/.cache/sgdg_tune.txt";
}

static bool tune_lookup(const std::string& key, TuneCfg& cfg, double& ms) {
  std::ifstream f(tune_cache_path());
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {  // last entry of a key wins
    std::istringstream in(line);
    std::string k;
    TuneCfg c{};
    double t = 0;
    if (in >> k >> c.variant >> c.bc >> c.xbox >> c.xcd >> c.chunks >> t && k == key) {
      cfg = c;
      ms = t;
      found = true;
    }
  }
  return found;
}

static void tune_store(const std::string& key, const TuneCfg& c, double ms) {
  const std::string path = tune_cache_path();
  const size_t slash = path.find_last_of('/');
  if (slash != std::string::npos) (void)::mkdir(path.substr(0, slash).c_str(), 0755);  // one level, best effort
  std::ofstream f(path, std::ios::app);
  if (f) f << key << " " << c.variant << " " << c.bc << " " << c.xbox << " " << c.xcd << " " << c.chunks << " " << ms
           << "\n";
}

static void set_cfg(Batch& B, const TuneCfg& c) {
  B.scan_chunks = std::max(0, c.chunks);
  B.variant = c.variant;
  B.split_bc = c.bc;
  B.split_xcd = c.xcd;
  if (c.variant == 1 && (B.xbox[0] != c.xbox || B.xbox[1] != c.xbox)) {
    SGDG_CHECK_HIP(hipDeviceSynchronize());
    B.xbox[0] = B.xbox[1] = c.xbox;
    for (auto& K : B.kinds)
      for (auto& I : K.it) I.built = false;  // box tables follow the new shape
  }
}

template <class T>
static double time_apply(Batch& B, const T* u, T* y, int nb, int reps, hipStream_t s) {
  hipEvent_t a, b;
  SGDG_CHECK_HIP(hipEventCreate(&a));
  SGDG_CHECK_HIP(hipEventCreate(&b));
  apply<T>(B, K_FULL, u, y, nb, s);
  SGDG_CHECK_HIP(hipEventRecord(a, s));
  for (int r = 0; r < reps; ++r) apply<T>(B, K_FULL, u, y, nb, s);
  SGDG_CHECK_HIP(hipEventRecord(b, s));
  SGDG_CHECK_HIP(hipEventSynchronize(b));
  float ms = 0;
  SGDG_CHECK_HIP(hipEventElapsedTime(&ms, a, b));
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return double(ms) / reps;
}

template <class T>
static sgdg_tune_result tune(Batch& B, int nb, int reps, bool force, hipStream_t s) {
  sgdg_tune_result r{};
  const std::string key = tune_key(B, int(sizeof(T)), nb);
  TuneCfg best{};
  double best_ms = 0;
  if (!force && tune_lookup(key, best, best_ms)) {
    set_cfg(B, best);
    r = {best.variant, best.bc, best.xbox, best.xcd, best_ms, 1, best.chunks};
    return r;
  }
  const int64_t n = kind(B, K_FULL).total * nb;
  DevBuf u, y;
  u.alloc(sizeof(T) * n);
  y.alloc(sizeof(T) * n);
  KernelsT<T>::fill(n, T(1), ptr<T>(u), s);
  const bool prof = B.prof;
  B.prof = false;
  best_ms = 1e300;
  for (const TuneCfg& c : tune_candidates(B.d)) {
    set_cfg(B, c);
    double ms = 0;
    try {
      ms = time_apply<T>(B, ptr<T>(u), ptr<T>(y), nb, std::max(1, reps), s);
    } catch (const Error& e) {
      if (e.code != SGDG_E_ARG) throw;
      continue;  // configuration not available for these grids (e.g. beyond the LDS budget)
    }
    if (ms < best_ms) {
      best_ms = ms;
      best = c;
    }
  }
  if (best_ms >= 1e300) {
    B.prof = prof;
    throw Error{SGDG_E_STATE, "no launch configuration could run"};
  }
  // few vectors leave the level scans short of blocks: split each item's
  // factor groups over several blocks (more parallel, the u gathers repeated)
  if (nb <= 4) {
    int ng = 1;
    for (const ProbDesc& D : kind(B, K_FULL).host) ng = std::max(ng, std::max(D.op.nvg, D.op.nxg));
    const TuneCfg base = best;
    for (int ch : {2, 4, 8}) {
      if (ch > ng) break;
      TuneCfg c = base;
      c.chunks = ch;
      set_cfg(B, c);
      const double ms = time_apply<T>(B, ptr<T>(u), ptr<T>(y), nb, std::max(1, reps), s);
      if (ms < best_ms) {
        best_ms = ms;
        best = c;
      }
    }
  }
  B.prof = prof;
  set_cfg(B, best);
  SGDG_CHECK_HIP(hipStreamSynchronize(s));
  tune_store(key, best, best_ms);
  r = {best.variant, best.bc, best.xbox, best.xcd, best_ms, 0, best.chunks};
  return r;
}

// ================================================================== ABI ===
extern "C" sgdg_status sgdg_apply_operator(sgdg_ops o, int kind_, const void* u_dev, void* y_dev, sgdg_dtype t,
                                           int batch, hipStream_t s) {
  API_BEGIN
  require(o != nullptr, "null ops");
  require(kind_ >= SGDG_OP_FULL && kind_ <= SGDG_OP_DATA_G, "unknown operator kind");
  require(u_dev && y_dev && u_dev != y_dev, "u and y must be distinct non-null device buffers");
  require(batch >= 1, "batch must be >= 1");
  require(t == SGDG_F64 || t == SGDG_F32, "dtype must be F64 or F32");
  static const int map[5] = {K_FULL, K_DIAG, K_MASS, K_DATAF, K_DATAG};
  Batch& B = self_batch(o);
  if (t == SGDG_F64) apply<double>(B, map[kind_], static_cast<const double*>(u_dev), static_cast<double*>(y_dev), batch, s);
  else apply<float>(B, map[kind_], static_cast<const float*>(u_dev), static_cast<float*>(y_dev), batch, s);
  API_END
}

// ------------------------------------------------ allocation-free apply ---
// Device scratch of sgdg_apply_operator_noalloc.  Host code never uses this
// name as an address (on the host it is only a stand-in for the symbol): the
// device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[SGDG_NOALLOC_SCRATCH_BYTES];

static unsigned char* scratch_ptr() {
  static std::mutex mu;
  static std::map<int, unsigned char*> ptrs;
  int dev = -1;
  SGDG_CHECK_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  auto it = ptrs.find(dev);
  if (it != ptrs.end()) return it->second;
  void* p = nullptr;
  SGDG_CHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  require(p != nullptr, "no device address for the scratch array");
  ptrs[dev] = static_cast<unsigned char*>(p);
  return static_cast<unsigned char*>(p);
}

extern "C" sgdg_status sgdg_apply_operator_noalloc(sgdg_ops o, int kind_, const void* u_dev, void* y_dev,
                                                   sgdg_dtype t, int batch, hipStream_t s) {
  API_BEGIN
  require(o != nullptr, "null ops");
  require(kind_ >= SGDG_OP_FULL && kind_ <= SGDG_OP_DATA_G, "unknown operator kind");
  require(u_dev && y_dev && u_dev != y_dev, "u and y must be distinct non-null device buffers");
  require(batch >= 1, "batch must be >= 1");
  require(t == SGDG_F64 || t == SGDG_F32, "dtype must be F64 or F32");
  int dev = -1;
  SGDG_CHECK_HIP(hipGetDevice(&dev));
  require(dev == o->device, "the current device is not the device of the ops handle");
  static const int map[5] = {K_FULL, K_DIAG, K_MASS, K_DATAF, K_DATAG};
  require_state(o->self != nullptr, "the ops handle has no launch tables yet: apply it once with sgdg_apply_operator first");
  Batch& B = *o->self;
  const int k = map[kind_];
  const int e = t == SGDG_F64 ? 0 : 1;
  require_state(!B.kinds[k].host.empty() && B.kinds[k].it[e].built,
                "launch tables of this operator kind and dtype are not built yet: apply it once with "
                "sgdg_apply_operator first");
  const size_t need = t == SGDG_F64 ? apply_scratch_bytes<double>(B, k, batch) : apply_scratch_bytes<float>(B, k, batch);
  if (need > SGDG_NOALLOC_SCRATCH_BYTES) {
    std::ostringstream m;
    m << "the application needs " << need << " bytes of scratch; the allocation-free entry point holds "
      << size_t(SGDG_NOALLOC_SCRATCH_BYTES) << " (use a smaller batch or sgdg_apply_operator)";
    throw Error{SGDG_E_ARG, m.str()};
  }
  Carve c{scratch_ptr(), size_t(SGDG_NOALLOC_SCRATCH_BYTES), 0};
  if (t == SGDG_F64) apply<double>(B, k, static_cast<const double*>(u_dev), static_cast<double*>(y_dev), batch, s, &c);
  else apply<float>(B, k, static_cast<const float*>(u_dev), static_cast<float*>(y_dev), batch, s, &c);
  API_END
}

extern "C" sgdg_status sgdg_precondition(sgdg_ops o, const void* r_dev, void* z_dev, sgdg_dtype t, int batch,
                                         const sgdg_precond_opts* po_in, hipStream_t s) {
  API_BEGIN
  require(o && r_dev && z_dev && r_dev != z_dev, "null or aliased argument");
  require(batch >= 1 && batch <= 4096, "batch must be 1..4096");
  const sgdg_precond_opts po = po_in ? *po_in : default_pc();
  require(po.kind == 0, "sgdg_precondition applies the combination technique (kind 0); see sgdg_net_apply");
  require(po.inner_rtol > 0 && po.inner_maxit >= 1 && po.inner_restart >= 1, "invalid inner solver options");
  check_mass(po, o->X.dom.d);
  // batch vectors [B][n_dof] are the layout of the problem replicated B times:
  // every grid problem of every vector iterates in the same launches
  Batch& B = replica_batch(o, batch);
  bool nan = false;
  if (t == SGDG_F64)
    ct_apply<double>(B, static_cast<const double*>(r_dev), static_cast<double*>(z_dev), po, false, s, &nan);
  else
    ct_apply<float>(B, static_cast<const float*>(r_dev), static_cast<float*>(z_dev), po, false, s, &nan);
  if (nan) throw Error{SGDG_E_NAN, "non-finite residual in a grid problem"};
  API_END
}

extern "C" sgdg_status sgdg_debug_grid_precond(sgdg_ops o, int sweeps, const void* in_dev, void* out_dev,
                                               sgdg_dtype t, hipStream_t s) {
  API_BEGIN
  require(o && in_dev && out_dev && in_dev != out_dev, "null or aliased argument");
  require(t == SGDG_F64 || t == SGDG_F32, "dtype must be F64 or F32");
  sgdg_precond_opts po = default_pc();
  po.mass_sweeps = sweeps;
  check_mass(po, o->X.dom.d);
  Batch& B = self_batch(o);
  SegTab& ST = ct_tab(B, B.R);
  const int64_t nct = kind(B, K_CT).total;
  auto run = [&](auto* tag) {
    using T = std::remove_pointer_t<decltype(tag)>;
    BWork<T>& w = work<T>(B);
    for (DevBuf* b : {&w.mU, &w.mX0, &w.mX1, &w.mD0, &w.mD1}) b->ensure(sizeof(T) * nct);
    mass_precond<T>(B, ST, sweeps, static_cast<const T*>(in_dev), static_cast<T*>(out_dev), s);
  };
  if (t == SGDG_F64) run(static_cast<double*>(nullptr));
  else run(static_cast<float*>(nullptr));
  API_END
}

extern "C" sgdg_status sgdg_combine(sgdg_ops o, const double* nodal_dev, double* coef_dev, int nslices, hipStream_t s) {
  API_BEGIN
  require(o && nodal_dev && coef_dev, "null argument");
  require(nslices >= 1 && nslices <= kMaxR, "nslices must be 1..3");
  std::vector<double> wts(nslices * nslices, 0.0);
  for (int i = 0; i < nslices; ++i) wts[i * nslices + i] = 1.0;
  nodal_to_coef(self_batch(o), nodal_dev, nslices, wts.data(), nslices, coef_dev, s);
  API_END
}

extern "C" sgdg_status sgdg_rhs(sgdg_ops o, const double* u_prev_dev, int prev_slices, const double* f_nodal_dev,
                                const double* g_nodal_dev, double* b_dev, hipStream_t s) {
  API_BEGIN
  require(o && u_prev_dev && b_dev, "null argument");
  require(prev_slices >= 1 && prev_slices <= kMaxR, "prev_slices must be 1..3");
  Batch& B = self_batch(o);
  sgdg_grid g = o->grid;
  const int R = g->R;
  const int64_t npts = g->up_pts;
  // jump term (U_{j-1}^-, w_{j-1}^+)
  B.rhs_c.ensure(sizeof(double) * 2 * npts);
  double* tr = ptr<double>(B.rhs_c);
  double* mtr = tr + npts;
  SegTab& PT = pts_tab(B);
  trace_sum(PT.t, prev_slices, u_prev_dev, tr, s);
  apply<double>(B, K_MASS, tr, mtr, 1, s);
  spread_left(PT.t, mtr, b_dev, s);
  // data functionals of f and g
  if (f_nodal_dev || g_nodal_dev) {
    const int nq = g->r + 2;
    std::vector<double> xg, wg;
    gauss_legendre(nq, xg, wg);
    std::vector<double> wts(R * nq);
    // c_s = (2s+1)/dt int f eta_s = (2s+1)/2 sum_q wg_q P_s(xg_q) f_q
    for (int k = 0; k < R; ++k)
      for (int q = 0; q < nq; ++q) wts[k * nq + q] = 0.5 * (2 * k + 1) * wg[q] * legendre(k, xg[q]);
    const int64_t ndof = int64_t(R) * npts;
    B.rhs_d.ensure(sizeof(double) * 2 * ndof);
    double* coef = ptr<double>(B.rhs_d);
    double* out = coef + ndof;
    for (int which = 0; which < 2; ++which) {
      const double* smp = which == 0 ? f_nodal_dev : g_nodal_dev;
      if (!smp) continue;
      if (o->ops[which == 0 ? 2 : 3].op.nterms == 0) continue;
      nodal_to_coef(B, smp, nq, wts.data(), R, coef, s);
      apply<double>(B, which == 0 ? K_DATAF : K_DATAG, coef, out, 1, s);
      KernelsT<double>::axpby(ndof, 1.0, out, 1.0, b_dev, s);
    }
  }
  API_END
}

static void check_solve_opts(const sgdg_solve_opts* so, const Batch& B) {
  require(so != nullptr, "null solver options");
  require(so->rtol > 0 && so->restart >= 1 && so->restart <= 64 && so->maxit >= 1, "invalid solver options");
  require(so->pc.kind == 0 || so->pc.kind == 1, "unknown preconditioner kind");
  check_mass(so->pc, B.d);
  if (so->pc.kind == 1) {
    if (B.owned_by_ops)
      require(so->pc.net != nullptr && net_problem(so->pc.net) == B.P[0],
              "the learned preconditioner needs the network of this problem");
    else
      require(B.nets.size() == B.P.size(),
              "the learned preconditioner of a batch needs one network per problem (sgdg_batch_set_networks)");
  }
}

extern "C" sgdg_status sgdg_solve_strip(sgdg_ops o, const double* b_dev, double* u_dev, const sgdg_solve_opts* so,
                                        sgdg_solve_stats* st, hipStream_t s) {
  API_BEGIN
  require(o && b_dev && u_dev, "null argument");
  check_solve_opts(so, self_batch(o));
  bool nan = false;
  const sgdg_solve_stats stats = solve_batch(self_batch(o), b_dev, u_dev, *so, s, &nan);
  if (st) *st = stats;
  if (nan) throw Error{SGDG_E_NAN, "non-finite residual norm"};
  if (stats.rel_residual > so->rtol) throw Error{SGDG_E_NOCONV, "iteration limit reached before the tolerance"};
  API_END
}

// ------------------------------------------------------------ batch ABI ---
extern "C" sgdg_status sgdg_batch_create(const sgdg_ops* ops, int n, sgdg_batch* out) {
  API_BEGIN
  require(ops && out && n >= 1, "need n >= 1 ops handles");
  for (int i = 0; i < n; ++i) require(ops[i] != nullptr, "null ops handle");
  const int d = ops[0]->X.dom.d, r = ops[0]->grid->r, dev = ops[0]->device;
  for (int i = 1; i < n; ++i) {
    require(ops[i]->X.dom.d == d, "all problems of a batch must share the dimension");
    require(ops[i]->grid->r == r, "all problems of a batch must share the time degree");
    require(ops[i]->device == dev, "all problems of a batch must live on one device");
  }
  auto* b = new Batch;
  b->P.assign(ops, ops + n);
  b->d = d;
  b->R = r + 1;
  if (const char* v = getenv("SGDG_APPLY_VARIANT"))
    b->variant = std::string(v) == "fused" ? 1 : (std::string(v) == "split_tiled" ? 2 : 0);
  if (const char* v = getenv("SGDG_SPLIT_BC")) b->split_bc = atoi(v);
  b->split_xcd = split_xcd();
  if (const char* v = getenv("SGDG_SCAN_CHUNKS")) b->scan_chunks = std::max(0, atoi(v));
  *out = b;
  API_END
}

extern "C" sgdg_status sgdg_batch_layout(sgdg_batch b, int64_t* offsets) {
  API_BEGIN
  require(b && offsets, "null argument");
  int64_t off = 0;
  for (size_t i = 0; i < b->P.size(); ++i) {
    offsets[i] = off;
    off += int64_t(b->R) * b->P[i]->grid->up_pts;
  }
  offsets[b->P.size()] = off;
  API_END
}

extern "C" sgdg_status sgdg_batch_apply(sgdg_batch b, const void* u_dev, void* y_dev, sgdg_dtype t, hipStream_t s) {
  API_BEGIN
  require(b && u_dev && y_dev && u_dev != y_dev, "null or aliased argument");
  if (t == SGDG_F64) apply<double>(*b, K_FULL, static_cast<const double*>(u_dev), static_cast<double*>(y_dev), 1, s);
  else apply<float>(*b, K_FULL, static_cast<const float*>(u_dev), static_cast<float*>(y_dev), 1, s);
  API_END
}

extern "C" sgdg_status sgdg_batch_solve(sgdg_batch b, const double* b_dev, double* u_dev, const sgdg_solve_opts* so,
                                        sgdg_solve_stats* st, hipStream_t s) {
  API_BEGIN
  require(b && b_dev && u_dev, "null argument");
  check_solve_opts(so, *b);
  bool nan = false;
  const sgdg_solve_stats stats = solve_batch(*b, b_dev, u_dev, *so, s, &nan);
  if (st) *st = stats;
  if (nan) throw Error{SGDG_E_NAN, "non-finite residual norm"};
  if (stats.rel_residual > so->rtol) throw Error{SGDG_E_NOCONV, "iteration limit reached before the tolerance"};
  API_END
}

extern "C" sgdg_status sgdg_batch_set_networks(sgdg_batch b, const sgdg_net* nets, int n) {
  API_BEGIN
  require(b != nullptr, "null batch");
  require(n == 0 || (nets != nullptr && n == int(b->P.size())), "need one network per problem of the batch (or n = 0)");
  for (int i = 0; i < n; ++i)
    require(nets[i] != nullptr && net_problem(nets[i]) == b->P[size_t(i)],
            "network " + std::to_string(i) + " does not belong to problem " + std::to_string(i) + " of the batch");
  b->nets.assign(nets, nets + n);
  API_END
}

extern "C" void sgdg_batch_destroy(sgdg_batch b) { delete b; }

// ---------------------------------------------------------- diagnostics ---
extern "C" sgdg_status sgdg_profile(sgdg_ops o, int mode) {
  API_BEGIN
  require(o != nullptr, "null ops");
  Batch& B = self_batch(o);
  drain_events(B);
  if (mode == 1)
    for (int i = 0; i < Batch::kSlots; ++i) {
      B.prof_ms[i] = 0;
      B.prof_n[i] = 0;
    }
  B.prof = mode == 1;
  API_END
}

extern "C" sgdg_status sgdg_profile_read(sgdg_ops o, int slot, double* ms, int64_t* launches) {
  API_BEGIN
  require(o != nullptr && slot >= 0 && slot < Batch::kSlots, "bad slot");
  Batch& B = self_batch(o);
  drain_events(B);
  if (ms) *ms = B.prof_ms[slot];
  if (launches) *launches = B.prof_n[slot];
  API_END
}

extern "C" sgdg_status sgdg_debug_fallback(int iters, double drop, int n, const int* call, const double* rel0,
                                           const double* est, int* switch_at) {
  API_BEGIN
  require(iters >= 1 && drop > 1 && n >= 0 && (n == 0 || (call && rel0 && est)) && switch_at, "bad arguments");
  FallbackMonitor fb(iters, drop);
  *switch_at = -1;
  for (int i = 0; i < n; ++i) {
    if (i == 0 || call[i] != call[i - 1]) fb.begin();
    if (fb.step(est[i], rel0[i])) {
      *switch_at = i;
      break;
    }
  }
  API_END
}

extern "C" sgdg_status sgdg_graph_cache_size(sgdg_ops o, int* count) {
  API_BEGIN
  require(o != nullptr && count != nullptr, "null argument");
  Batch& B = self_batch(o);
  // a stale cache is emptied on the next graph solve; report what would survive it
  *count = B.graph_epoch == alloc_epoch() ? int(B.graphs.size()) : 0;
  API_END
}

extern "C" sgdg_status sgdg_op_info(sgdg_ops o, int kind_, int* nterms, int* nvg, int* nxg, int* Sx, int* Sv,
                                    int* Rin, int* Rout) {
  API_BEGIN
  require(o != nullptr && kind_ >= SGDG_OP_FULL && kind_ <= SGDG_OP_DATA_G, "bad arguments");
  const int idx = kind_ == SGDG_OP_FULL || kind_ == SGDG_OP_BLOCKDIAG ? 0 : kind_ - 1;
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

extern "C" sgdg_status sgdg_op_support(sgdg_ops o, int kind_, int lx, int64_t* counts) {
  API_BEGIN
  require(o != nullptr && counts != nullptr && kind_ >= SGDG_OP_FULL && kind_ <= SGDG_OP_DATA_G, "bad arguments");
  const DevDomain& dx = o->dx.d;
  require(lx >= dx.lmin && lx <= dx.lmax, "x-level outside the hierarchy");
  const int idx = kind_ == SGDG_OP_FULL || kind_ == SGDG_OP_BLOCKDIAG ? 0 : kind_ - 1;
  const OpDev& od = o->ops[idx];
  const int nxg = od.op.nxg;
  const int64_t n = dx.lev_n[lx - dx.lmin], no = dx.node_off[lx - dx.lmin];
  for (int i = 0; i < 6; ++i) counts[i] = 0;
  counts[0] = n;
  for (int64_t x = 0; x < n; ++x)
    for (int m = 0; m < nxg; ++m) {
      const int64_t nt = od.hxgs[size_t(m) + 1] - od.hxgs[size_t(m)];
      const bool all = m >= 64;
      const uint64_t bit = all ? 0 : uint64_t(1) << m;
      if (all || (od.hxreadm[size_t(no + x)] & bit)) {
        counts[1] += 1;
        counts[2] += nt;
      }
      if (all || (od.hxrowm[size_t(no + x)] & bit)) counts[3] += 1;
      if (all || (od.hxqtm[size_t(no + x)] & bit)) {
        counts[4] += 1;
        counts[5] += nt;
      }
    }
  API_END
}

extern "C" sgdg_status sgdg_tune(sgdg_ops o, sgdg_dtype t, int batch, int reps, int force, sgdg_tune_result* out,
                                 hipStream_t s) {
  API_BEGIN
  require(o != nullptr && batch >= 1 && reps >= 1, "bad arguments");
  require(t == SGDG_F64 || t == SGDG_F32, "dtype must be F64 or F32");
  Batch& B = self_batch(o);
  const sgdg_tune_result r = t == SGDG_F64 ? tune<double>(B, batch, reps, force != 0, s)
                                           : tune<float>(B, batch, reps, force != 0, s);
  if (out) *out = r;
  API_END
}

extern "C" sgdg_status sgdg_batch_tune(sgdg_batch b, sgdg_dtype t, int reps, int force, sgdg_tune_result* out,
                                       hipStream_t s) {
  API_BEGIN
  require(b != nullptr && reps >= 1, "bad arguments");
  require(t == SGDG_F64 || t == SGDG_F32, "dtype must be F64 or F32");
  const sgdg_tune_result r = t == SGDG_F64 ? tune<double>(*b, 1, reps, force != 0, s)
                                           : tune<float>(*b, 1, reps, force != 0, s);
  if (out) *out = r;
  API_END
}

extern "C" sgdg_status sgdg_set_launch(sgdg_ops o, const sgdg_tune_result* cfg) {
  API_BEGIN
  require(o != nullptr && cfg != nullptr, "null argument");
  require(cfg->variant >= 0 && cfg->variant <= 2, "variant must be 0 (split), 1 (fused) or 2 (split, tiled x-stage)");
  Batch& B = self_batch(o);
  if (cfg->variant != 1)
    require(cfg->vectors_per_thread == 1 || (B.d < 3 && (cfg->vectors_per_thread == 2 || cfg->vectors_per_thread == 4)),
            "vectors_per_thread must be 1, 2 or 4 (1 for d = 3)");
  else
    require(cfg->xbox >= 1 && cfg->xbox <= 256, "xbox must be 1..256");
  require(cfg->block_map == 0 || cfg->block_map == 1, "block_map must be 0 or 1");
  require(cfg->scan_chunks >= 0 && cfg->scan_chunks <= 64, "scan_chunks must be 0..64");
  set_cfg(B, TuneCfg{cfg->variant, cfg->variant != 1 ? cfg->vectors_per_thread : 0,
                     cfg->variant == 1 ? cfg->xbox : B.xbox[0], cfg->variant != 1 ? cfg->block_map : 0,
                     cfg->scan_chunks > 0 ? cfg->scan_chunks : B.scan_chunks});
  API_END
}
