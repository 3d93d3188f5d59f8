// Internal structures shared by problem.hip (layout, assembly, upload) and
// solver.hip (operator application, preconditioners, solvers).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "fused.h"
#include "kernels.h"
#include "sgdg_internal.h"

using namespace sgdg;

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

static inline void require(bool ok, const std::string& msg) {
  if (!ok) throw Error{SGDG_E_ARG, msg};
}

static inline void require_state(bool ok, const std::string& msg) {
  if (!ok) throw Error{SGDG_E_STATE, msg};
}

template <class T>
static inline T* ptr(const DevBuf& b) {
  return static_cast<T*>(b.p);
}

// While set (refresh_fields), an upload of the size a buffer already has
// rewrites that allocation in place; otherwise every upload allocates anew.
extern thread_local bool g_upload_inplace;

template <class T>
static inline T* upload(DevBuf& b, const std::vector<T>& h) {
  const size_t nb = h.size() * sizeof(T);
  if (!(g_upload_inplace && b.bytes == nb && (b.p != nullptr || nb == 0))) b.alloc(nb);
  if (nb) SGDG_CHECK_HIP(hipMemcpy(b.p, h.data(), nb, hipMemcpyHostToDevice));
  return ptr<T>(b);
}

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

struct DomDev {
  DevBuf nbr, tnbr, par, parw, chi, chiw, tchi, tchiw, vals, vals32, tvals, tvals32, wide, rvals, rvals32, twide,
      trvals, trvals32, pidx, pvals, pvals32, qvals, qvals32, qpvals, qpvals32, qrvals, qrvals32, sup, fpartial;
  DevDomain d;
  std::vector<uint8_t> hsup, hpartial;  // host copies of d.sup, d.fpartial
};

struct OpDev {
  TermList host;
  DevBuf xf, vf, vg, xg, tm, tm32, vgf, xgf, vgt, vgs, xgt, xgs, xrowm, xreadm, xqtm, xptm, xgk;
  DevOp op;
  std::vector<int> hxgf, hxgs;                 // host copies of op.xg_fac, op.xg_start
  std::vector<uint64_t> hxrowm, hxreadm, hxqtm;  // host copies of the per-node group masks
};

// A batch of independent strip problems sharing dimension and time degree
// (the C type sgdg_batch); a single problem is used as a batch of one.
using Batch = sgdg_batch_s;
void destroy_batch(Batch* b);
struct BatchDeleter {
  void operator()(Batch* b) const { destroy_batch(b); }
};

struct sgdg_ops_s {
  sgdg_grid grid = nullptr;
  DomainData X, V;
  DomDev dx, dv;
  OpDev ops[4];  // FULL, MASS, DATA_F, DATA_G term lists
  double pinv[kMaxR * kMaxR] = {};  // (Tt + delta Ct + Gt)^-1
  int device = 0;
  std::unique_ptr<Batch, BatchDeleter> self;  // this problem as a batch of one
  // this problem replicated n times (n independent vectors in one lockstep
  // preconditioner application), keyed by n
  std::map<int, std::unique_ptr<Batch, BatchDeleter>> replicas;
  sgdg_net recorder = nullptr;                 // network recording (r, P_CT r) pairs of this problem
  std::vector<sgdg_net> nets;                  // networks created for this problem
};

// Re-assembles the operator of o for new values of the coefficient fields the
// problem registered (read again through the same pointers, which must still be
// valid): the term lists are rebuilt from p, and if they and the factor
// registries come out unchanged, the factor tables are recomputed and written
// into the existing device buffers, so work buffers, launch tables and captured
// graphs stay valid; cached batches are dropped only if a support mask
// changed.  Returns false if the structure differs: o is then no longer
// consistent and must be replaced by a newly assembled handle.
bool refresh_fields(sgdg_ops o, const sgdg_problem& p);

// The learned preconditioner (net.hip) as seen by the strip solver.
void net_apply_dev(sgdg_net n, const double* r, double* z, hipStream_t s);
sgdg_ops net_problem(sgdg_net n);
void net_record_pair(sgdg_net n, const double* r, const double* z, hipStream_t s);
void net_detach(sgdg_net n);  // the problem is being destroyed

// the problem as a batch of one (created on first use)
Batch& self_batch(sgdg_ops o);
// the problem replicated n times (created on first use, kept with the handle)
Batch& replica_batch(sgdg_ops o, int n);
