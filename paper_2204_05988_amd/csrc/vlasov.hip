// Vlasov-Poisson coupling (Sect. 5.3): the density rho = int f dv of a
// sparse-grid function, the Poisson problem -Laplace phi = 1 - rho on the
// finest x-lattice with P1 elements, the field E = -grad phi (its L2
// projection onto P1), and the per-strip fixed point that alternates the
// linear transport (eq:E_f) with beta = (v, -E) and the field (eq:poisson).
//
// The density of component grid l is a P1 function on x-level lx,
// c_l[kx] = sum_kv f_l[kx, kv] int phi_kv dv; the upper grids have distinct
// x-levels, so the finest-level density is one prolongation chain
// acc_lx = E acc_{lx-1} + c_lx from the coarsest x-level up.  The field
// problems are small (at most 2^16 nodes): one workgroup runs the whole
// conjugate-gradient solve (stiffness, then one mass solve per axis) in a
// single launch, so the solve costs no host round trips.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <vector>

#include "ops_internal.h"

using namespace sgdg;

namespace {

constexpr int kVB = 1024;  // threads of the single-workgroup kernels
constexpr int kMB = 256;   // threads of the moment kernel

__device__ double vp_block_sum(double a, double* sh) {
  for (int o = 32; o > 0; o >>= 1) a += __shfl_down(a, o, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wv] = a;
  __syncthreads();
  double t = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < int(blockDim.x >> 6); ++i) t += sh[i];
  __syncthreads();
  if (threadIdx.x == 0) sh[0] = t;
  __syncthreads();
  const double r = sh[0];
  __syncthreads();
  return r;
}

__device__ double vp_block_max(double a, double* sh) {
  for (int o = 32; o > 0; o >>= 1) a = fmax(a, __shfl_down(a, o, 64));
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wv] = a;
  __syncthreads();
  double t = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < int(blockDim.x >> 6); ++i) t = fmax(t, sh[i]);
  __syncthreads();
  if (threadIdx.x == 0) sh[0] = t;
  __syncthreads();
  const double r = sh[0];
  __syncthreads();
  return r;
}

struct VpGrids {
  int n = 0, R = 1, S = 1;
  int lx[kMaxGrids] = {};
  int nx[kMaxGrids] = {}, nv[kMaxGrids] = {};
  int64_t off[kMaxGrids] = {};   // start of grid g's [R][nx][nv] block in f
  int64_t coff[kMaxGrids] = {};  // start of grid g's x-level density in the moment buffer
  int64_t woff[kMaxGrids] = {};  // start of grid g's v weights (level lv)
  double tw[kMaxR] = {};         // Legendre values of the slices at the evaluation time
};

// c_g[kx] = sum_kv (sum_s tw_s f[s][kx][kv]) w_g[kv]; one block per (grid, x-node)
__global__ void __launch_bounds__(kMB) k_vp_moment(VpGrids G, const int* __restrict__ item_grid,
                                                   const int* __restrict__ item_x, const double* __restrict__ f,
                                                   const double* __restrict__ vw, double* __restrict__ c) {
  __shared__ double sh[kMB / 64];
  const int g = item_grid[blockIdx.x], x = item_x[blockIdx.x];
  const int nv = G.nv[g];
  const int64_t plane = int64_t(G.nx[g]) * nv;
  const double* fb = f + G.off[g] + int64_t(x) * nv;
  const double* w = vw + G.woff[g];
  double a = 0;
  for (int v = threadIdx.x; v < nv; v += kMB) {
    double s = 0;
    for (int q = 0; q < G.R; ++q) s += G.tw[q] * fb[int64_t(q) * plane + v];
    a += s * w[v];
  }
  a = vp_block_sum(a, sh);
  if (threadIdx.x == 0) c[G.coff[g] + x] = a;
}

// rho on the finest x-level: acc = c_lmin; acc_l = E acc_{l-1} + c_l (one workgroup)
__global__ void __launch_bounds__(kVB) k_vp_chain(int nlev, const int64_t* __restrict__ lev_n,
                                                  const int64_t* __restrict__ lev_c, const int64_t* __restrict__ lev_p,
                                                  const int32_t* __restrict__ par, const double* __restrict__ parw,
                                                  const double* __restrict__ c, double* __restrict__ a0,
                                                  double* __restrict__ a1, double* __restrict__ rho) {
  double* cur = a0;
  double* nxt = a1;
  for (int64_t i = threadIdx.x; i < lev_n[0]; i += kVB) cur[i] = c[lev_c[0] + i];
  __syncthreads();
  for (int l = 1; l < nlev; ++l) {
    const int32_t* p = par + lev_p[l];
    const double* pw = parw + lev_p[l];
    double* out = l + 1 == nlev ? rho : nxt;
    for (int64_t i = threadIdx.x; i < lev_n[l]; i += kVB)
      out[i] = pw[2 * i] * cur[p[2 * i]] + pw[2 * i + 1] * cur[p[2 * i + 1]] + c[lev_c[l] + i];
    __syncthreads();
    double* t = cur;
    cur = nxt;
    nxt = t;
  }
  if (nlev == 1)
    for (int64_t i = threadIdx.x; i < lev_n[0]; i += kVB) rho[i] = cur[i];
}

struct Ell {
  int64_t n = 0;
  int S = 0;
  const int32_t* nbr = nullptr;  // [n][S]
};

__device__ void ell_apply(const Ell& E, const double* __restrict__ val, const double* __restrict__ x,
                          double* __restrict__ y, double scale) {
  for (int64_t i = threadIdx.x; i < E.n; i += kVB) {
    double a = 0;
    for (int e = 0; e < E.S; ++e) a += val[i * E.S + e] * x[E.nbr[i * E.S + e]];
    y[i] = scale * a;
  }
}

// conjugate gradients for A x = b in one workgroup (A = val on E), x0 = 0;
// mean_zero: A is singular with the constants as kernel, b has mean zero and
// the iterates are kept of mean zero.  Returns the iterations.
__device__ int block_cg(const Ell& E, const double* val, const double* b, double* x, double* r, double* p,
                        double* q, double tol, int maxit, bool mean_zero, double* sh) {
  const int64_t n = E.n;
  double bb = 0;
  for (int64_t i = threadIdx.x; i < n; i += kVB) {
    x[i] = 0;
    r[i] = b[i];
    p[i] = b[i];
    bb += b[i] * b[i];
  }
  bb = vp_block_sum(bb, sh);
  double rr = bb;
  const double stop = tol * tol * bb;
  int it = 0;
  while (it < maxit && rr > stop && rr > 0) {
    ell_apply(E, val, p, q, 1.0);
    __syncthreads();
    double pq = 0;
    for (int64_t i = threadIdx.x; i < n; i += kVB) pq += p[i] * q[i];
    pq = vp_block_sum(pq, sh);
    const double al = rr / pq;
    double rn = 0, rs = 0;
    for (int64_t i = threadIdx.x; i < n; i += kVB) {
      x[i] += al * p[i];
      r[i] -= al * q[i];
      rs += r[i];
    }
    if (mean_zero) {
      rs = vp_block_sum(rs, sh) / double(n);
      for (int64_t i = threadIdx.x; i < n; i += kVB) r[i] -= rs;
    }
    for (int64_t i = threadIdx.x; i < n; i += kVB) rn += r[i] * r[i];
    rn = vp_block_sum(rn, sh);
    const double be = rn / rr;
    for (int64_t i = threadIdx.x; i < n; i += kVB) p[i] = r[i] + be * p[i];
    __syncthreads();
    rr = rn;
    ++it;
  }
  return it;
}

// phi from K phi = M (1 - rho) (mean zero), E_i from M E_i = -D_i phi, and the
// electric energy 1/2 sum_i E_i^T M E_i.  out[0] energy, out[1] Poisson CG
// iterations, out[2] largest mass-solve iterations.  w: 6 n scratch.
__global__ void __launch_bounds__(kVB) k_vp_field(Ell E, int d, const double* __restrict__ K,
                                                  const double* __restrict__ M, const double* __restrict__ D,
                                                  const double* __restrict__ rho, double* __restrict__ field,
                                                  double* __restrict__ phi, double* __restrict__ w, double tol,
                                                  int maxit, double* __restrict__ out) {
  __shared__ double sh[kVB / 64];
  const int64_t n = E.n;
  double* b = w;
  double* r = w + n;
  double* p = w + 2 * n;
  double* q = w + 3 * n;
  double* t = w + 4 * n;
  for (int64_t i = threadIdx.x; i < n; i += kVB) t[i] = 1.0 - rho[i];
  __syncthreads();
  ell_apply(E, M, t, b, 1.0);
  __syncthreads();
  double s = 0;
  for (int64_t i = threadIdx.x; i < n; i += kVB) s += b[i];
  s = vp_block_sum(s, sh) / double(n);
  for (int64_t i = threadIdx.x; i < n; i += kVB) b[i] -= s;
  __syncthreads();
  const int itp = block_cg(E, K, b, phi, r, p, q, tol, maxit, true, sh);
  double m = 0;
  for (int64_t i = threadIdx.x; i < n; i += kVB) m += phi[i];
  m = vp_block_sum(m, sh) / double(n);
  for (int64_t i = threadIdx.x; i < n; i += kVB) phi[i] -= m;
  __syncthreads();
  int itm = 0;
  double en = 0;
  for (int a = 0; a < d; ++a) {
    ell_apply(E, D + int64_t(a) * n * E.S, phi, b, -1.0);
    __syncthreads();
    double* Ea = field + int64_t(a) * n;
    itm = max(itm, block_cg(E, M, b, Ea, r, p, q, tol, maxit, false, sh));
    __syncthreads();
    ell_apply(E, M, Ea, t, 1.0);
    __syncthreads();
    double e = 0;
    for (int64_t i = threadIdx.x; i < n; i += kVB) e += Ea[i] * t[i];
    en += 0.5 * vp_block_sum(e, sh);
  }
  if (threadIdx.x == 0) {
    out[0] = en;
    out[1] = itp;
    out[2] = itm;
  }
}

// out[0] = max |a - b|, out[1] = sum a * b (one workgroup)
__global__ void __launch_bounds__(kVB) k_vp_diffdot(int64_t n, const double* __restrict__ a,
                                                    const double* __restrict__ b, const double* __restrict__ c,
                                                    const double* __restrict__ e, double* __restrict__ out) {
  __shared__ double sh[kVB / 64];
  double mx = 0, dt = 0;
  for (int64_t i = threadIdx.x; i < n; i += kVB) mx = fmax(mx, fabs(a[i] - b[i]));
  mx = vp_block_max(mx, sh);
  for (int64_t i = threadIdx.x; i < n; i += kVB) dt += c[i] * e[i];
  dt = vp_block_sum(dt, sh);
  if (threadIdx.x == 0) {
    out[0] = mx;
    out[1] = dt;
  }
}

// y = sum_s tw_s (x1 - x0)[s] per grid block (one slice out)
__global__ void k_vp_slice_diff(VpGrids G, int64_t npts, const double* __restrict__ x1, const double* __restrict__ x0,
                                double* __restrict__ y) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= npts) return;
  int g = 0;
  int64_t base = 0;
  while (g + 1 < G.n && i >= base + int64_t(G.nx[g]) * G.nv[g]) {
    base += int64_t(G.nx[g]) * G.nv[g];
    ++g;
  }
  const int64_t plane = int64_t(G.nx[g]) * G.nv[g];
  const int64_t k = i - base;
  double a = 0;
  for (int s = 0; s < G.R; ++s) a += G.tw[s] * (x1[G.off[g] + s * plane + k] - (x0 ? x0[G.off[g] + s * plane + k] : 0.0));
  y[i] = a;
}

double legendre_at(int s, double z) {
  double p0 = 1, p1 = z;
  if (s == 0) return p0;
  for (int k = 1; k < s; ++k) {
    const double p2 = ((2 * k + 1) * z * p1 - k * p0) / (k + 1);
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

}  // namespace

struct sgdg_vp_s {
  sgdg_grid g = nullptr;
  double dt = 0, delta = 0;
  int d = 1, L = 0, lmin = 0, R = 1, S = 1;
  int64_t nfine = 0;
  DomainData X, V;
  DevBuf nbr, Kv, Mv, Dv, vw, par, parw, lev_n, lev_c, lev_p, items_g, items_x, cbuf, acc0, acc1, fw, out, phi,
      slice, mslice, fprev_it;
  std::vector<int64_t> h_lev_n, h_lev_c, h_lev_p, h_vwoff;
  int nitems = 0;
  VpGrids G;
  std::vector<std::vector<double>> vcoord;  // finest v-lattice coordinates per axis (the fields v_i)
  sgdg_ops ops = nullptr;                   // transport operator of the current field
  std::vector<double> Ehost;
  double assemble_s = 0;
  ~sgdg_vp_s() {
    if (ops) sgdg_ops_destroy(ops);
  }
};

namespace {

void vp_grids(sgdg_vp p, double tau) {
  VpGrids& G = p->G;
  const sgdg_grid g = p->g;
  G.n = int(g->up.size());
  G.R = g->R;
  G.S = p->S;
  int64_t off = 0, coff = 0;
  for (int i = 0; i < G.n; ++i) {
    G.lx[i] = g->up[i].lx;
    G.nx[i] = int(g->up[i].nx);
    G.nv[i] = int(g->up[i].nv);
    G.off[i] = off;
    off += int64_t(G.R) * g->up[i].nx * g->up[i].nv;
    G.coff[i] = coff;
    coff += g->up[i].nx;
    G.woff[i] = p->h_vwoff[g->up[i].lv - p->lmin];
  }
  for (int s = 0; s < kMaxR; ++s) G.tw[s] = s < G.R ? legendre_at(s, tau) : 0.0;
}

void vp_density(sgdg_vp p, const double* f, int nslices, double tau, double* rho, hipStream_t s) {
  vp_grids(p, tau);
  VpGrids G = p->G;
  if (nslices != G.R) {  // a one-slice function (a trace): its only slice at weight 1
    require(nslices == 1, "nslices must be 1 or the number of time slices");
    int64_t off = 0;
    for (int i = 0; i < G.n; ++i) {
      G.off[i] = off;
      off += int64_t(G.nx[i]) * G.nv[i];
    }
    G.R = 1;
    G.tw[0] = 1.0;
  }
  hipLaunchKernelGGL(k_vp_moment, dim3(unsigned(p->nitems)), dim3(kMB), 0, s, G, ptr<int>(p->items_g),
                     ptr<int>(p->items_x), f, ptr<double>(p->vw), ptr<double>(p->cbuf));
  SGDG_CHECK_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_vp_chain, dim3(1), dim3(kVB), 0, s, int(p->h_lev_n.size()), ptr<int64_t>(p->lev_n),
                     ptr<int64_t>(p->lev_c), ptr<int64_t>(p->lev_p), ptr<int32_t>(p->par), ptr<double>(p->parw),
                     ptr<double>(p->cbuf), ptr<double>(p->acc0), ptr<double>(p->acc1), rho);
  SGDG_CHECK_HIP(hipGetLastError());
}

void vp_field(sgdg_vp p, const double* rho, double* E, double tol, int maxit, hipStream_t s) {
  Ell e;
  e.n = p->nfine;
  e.S = p->S;
  e.nbr = ptr<int32_t>(p->nbr);
  hipLaunchKernelGGL(k_vp_field, dim3(1), dim3(kVB), 0, s, e, p->d, ptr<double>(p->Kv), ptr<double>(p->Mv),
                     ptr<double>(p->Dv), rho, E, ptr<double>(p->phi), ptr<double>(p->fw), tol, maxit,
                     ptr<double>(p->out));
  SGDG_CHECK_HIP(hipGetLastError());
}

// the transport operator of field E (host copy p->Ehost, [d][nfine]): beta = (v, -E)
void vp_assemble(sgdg_vp p) {
  const auto t0 = std::chrono::steady_clock::now();
  const int d = p->d;
  std::vector<const double*> vf(d), xf(d);
  std::vector<sgdg_separable> sep(2 * d);
  for (int i = 0; i < d; ++i) {
    vf[i] = p->vcoord[i].data();
    sep[i] = sgdg_separable{1.0, 0, nullptr, 1, &vf[i]};
    xf[i] = p->Ehost.data() + int64_t(i) * p->nfine;
    sep[d + i] = sgdg_separable{-1.0, 1, &xf[i], 0, nullptr};
  }
  sgdg_problem pr{};
  for (int c = 0; c < 2 * d; ++c) pr.beta[c] = &sep[c];
  pr.n_sigma = 0;
  pr.sigma = nullptr;
  pr.dt = p->dt;
  pr.delta = p->delta;
  // the field changes only the values of the E-weighted x-factors: rewrite the
  // existing operator's tables in place (its work buffers, launch tables and
  // graphs stay); a new operator only if the term structure changed
  if (p->ops) {
    bool done = false;
    try {
      done = refresh_fields(p->ops, pr);
    } catch (...) {
      sgdg_ops_destroy(p->ops);  // possibly half rewritten
      p->ops = nullptr;
      throw;
    }
    if (done) {
      p->assemble_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      return;
    }
    sgdg_ops_destroy(p->ops);  // no longer consistent
    p->ops = nullptr;
  }
  sgdg_ops o = nullptr;
  const sgdg_status st = sgdg_assemble_1d_factors(p->g, &pr, &o);
  if (st != SGDG_OK) throw Error{st, std::string("assembling the transport operator: ") + sgdg_last_error()};
  if (p->ops) sgdg_ops_destroy(p->ops);
  p->ops = o;
  p->assemble_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

extern "C" sgdg_status sgdg_vp_create(sgdg_grid g, double dt, double delta, sgdg_vp* out) {
  API_BEGIN
  require(g && out, "null argument");
  require(g->x.periodic, "the Vlasov-Poisson coupling needs a periodic x-domain");
  require(g->x.d <= 2, "the Vlasov-Poisson coupling is built for d = 1 and 2");
  require(dt > 0 && delta >= 0, "dt must be > 0 and delta >= 0");
  std::unique_ptr<sgdg_vp_s> p(new sgdg_vp_s);
  p->g = g;
  p->dt = dt;
  p->delta = delta;
  p->d = g->x.d;
  p->L = g->lmax;
  p->lmin = g->lmin;
  p->R = g->R;
  require(int(g->up.size()) <= kMaxGrids, "too many component grids");
  // host factor tables: x mass, stiffness, derivatives (finest level), v masses (all levels)
  for (int side = 0; side < 2; ++side) {
    DomainData& D = side == 0 ? p->X : p->V;
    D.dom = side == 0 ? g->x : g->v;
    D.lmin = g->lmin;
    D.lmax = g->lmax;
    build_domain_tables(D);
  }
  FactorKey mk;
  mk.kind = kMass;
  const int xm = p->X.factor_id(mk), vm = p->V.factor_id(mk);
  std::vector<int> xs(p->d), xd(p->d);
  for (int a = 0; a < p->d; ++a) {
    FactorKey k;
    k.kind = kStiff;
    k.a = a;
    k.b = a;
    xs[a] = p->X.factor_id(k);
    FactorKey q;
    q.kind = kDeriv;
    q.a = a;
    xd[a] = p->X.factor_id(q);
  }
  p->X.values.assign(p->X.factors.size(), {});
  p->V.values.assign(p->V.factors.size(), {});
  for (int f = 0; f < int(p->X.factors.size()); ++f) assemble_factor(p->X, f);
  assemble_factor(p->V, vm);
  const LevelTables& LT = p->X.L(p->L);
  p->S = p->X.st.S;
  p->nfine = LT.n;
  require(p->nfine <= (int64_t(1) << 20), "x-lattice too large for the single-workgroup field solve");
  const int64_t nS = p->nfine * p->S;
  const std::vector<double>& Mx = p->X.values[xm][p->L - p->lmin];
  std::vector<double> K(nS, 0.0), Dall(int64_t(p->d) * nS);
  for (int a = 0; a < p->d; ++a) {
    const std::vector<double>& Sa = p->X.values[xs[a]][p->L - p->lmin];
    for (int64_t i = 0; i < nS; ++i) K[i] += Sa[i];
    const std::vector<double>& Da = p->X.values[xd[a]][p->L - p->lmin];
    std::copy(Da.begin(), Da.end(), Dall.begin() + int64_t(a) * nS);
  }
  upload(p->nbr, LT.nbr);
  upload(p->Kv, K);
  upload(p->Mv, Mx);
  upload(p->Dv, Dall);
  // v weights int phi_kv dv = row sums of the v mass matrix of each level
  std::vector<double> vw;
  for (int l = g->lmin; l <= g->lmax; ++l) {
    const LevelTables& VL = p->V.L(l);
    const std::vector<double>& Mv = p->V.values[vm][l - p->lmin];
    p->h_vwoff.push_back(int64_t(vw.size()));
    for (int64_t k = 0; k < VL.n; ++k) {
      double s = 0;
      for (int e = 0; e < p->V.st.S; ++e)
        if (VL.valid[k * p->V.st.S + e]) s += Mv[k * p->V.st.S + e];
      vw.push_back(s);
    }
  }
  upload(p->vw, vw);
  // the prolongation chain over the upper grids' x-levels (lmin .. L, one grid each)
  std::vector<int32_t> par;
  std::vector<double> parw;
  std::vector<int64_t> cofs(g->lmax + 1, -1);
  int64_t coff = 0;
  for (const GridDesc& gd : g->up) {
    cofs[gd.lx] = coff;
    coff += gd.nx;
  }
  for (int l = g->lmin; l <= g->lmax; ++l) {
    require(cofs[l] >= 0, "every x-level must carry one upper grid");
    const LevelTables& XL = p->X.L(l);
    p->h_lev_n.push_back(XL.n);
    p->h_lev_c.push_back(cofs[l]);
    p->h_lev_p.push_back(int64_t(par.size()));
    if (l > g->lmin) {
      par.insert(par.end(), XL.par.begin(), XL.par.end());
      parw.insert(parw.end(), XL.parw.begin(), XL.parw.end());
    }
  }
  if (par.empty()) {
    par.push_back(0);
    parw.push_back(0.0);
  }
  upload(p->par, par);
  upload(p->parw, parw);
  upload(p->lev_n, p->h_lev_n);
  upload(p->lev_c, p->h_lev_c);
  upload(p->lev_p, p->h_lev_p);
  std::vector<int> ig, ix;
  for (int i = 0; i < int(g->up.size()); ++i)
    for (int64_t x = 0; x < g->up[i].nx; ++x) {
      ig.push_back(i);
      ix.push_back(int(x));
    }
  p->nitems = int(ig.size());
  upload(p->items_g, ig);
  upload(p->items_x, ix);
  p->cbuf.alloc(sizeof(double) * coff);
  p->acc0.alloc(sizeof(double) * p->nfine);
  p->acc1.alloc(sizeof(double) * p->nfine);
  p->fw.alloc(sizeof(double) * 6 * p->nfine);
  p->phi.alloc(sizeof(double) * p->nfine);
  p->out.alloc(sizeof(double) * 8);
  p->slice.alloc(sizeof(double) * g->up_pts);
  p->mslice.alloc(sizeof(double) * g->up_pts);
  p->fprev_it.alloc(sizeof(double) * g->R * g->up_pts);
  // the v fields v_i at the finest v-lattice nodes
  const Dom& vd = g->v;
  const int mv = vd.axis_nodes(g->lmax);
  const int64_t nvf = vd.nodes(g->lmax);
  p->vcoord.assign(p->d, std::vector<double>(nvf));
  for (int64_t k = 0; k < nvf; ++k) {
    int64_t r = k;
    for (int a = vd.d - 1; a >= 0; --a) {
      const int ia = int(r % mv);
      r /= mv;
      p->vcoord[a][k] = vd.lo[a] + ia * vd.h(g->lmax, a);
    }
  }
  p->Ehost.assign(size_t(p->d) * p->nfine, 0.0);
  *out = p.release();
  API_END
}

extern "C" void sgdg_vp_destroy(sgdg_vp p) { delete p; }

extern "C" sgdg_status sgdg_vp_info(sgdg_vp p, int64_t* n_fine, int* d) {
  API_BEGIN
  require(p != nullptr, "null handle");
  if (n_fine) *n_fine = p->nfine;
  if (d) *d = p->d;
  API_END
}

extern "C" sgdg_status sgdg_vp_density(sgdg_vp p, const double* f_dev, int nslices, double tau, double* rho_dev,
                                       hipStream_t s) {
  API_BEGIN
  require(p && f_dev && rho_dev, "null argument");
  require(tau >= -1.0 && tau <= 1.0, "tau must lie in [-1, 1]");
  vp_density(p, f_dev, nslices, tau, rho_dev, s);
  API_END
}

extern "C" sgdg_status sgdg_vp_field(sgdg_vp p, const double* rho_dev, double* E_dev, double* energy,
                                     hipStream_t s) {
  API_BEGIN
  require(p && rho_dev && E_dev, "null argument");
  vp_field(p, rho_dev, E_dev, 1e-14, 50000, s);
  if (energy) {
    double h[3];
    SGDG_CHECK_HIP(hipMemcpyAsync(h, p->out.p, sizeof(h), hipMemcpyDeviceToHost, s));
    SGDG_CHECK_HIP(hipStreamSynchronize(s));
    *energy = h[0];
  }
  API_END
}

extern "C" sgdg_status sgdg_vp_strip(sgdg_vp p, const double* f_prev_dev, int prev_slices, const double* E0_dev,
                                     double* f_dev, double* E_dev, const sgdg_vp_opts* vo, sgdg_vp_stats* st,
                                     hipStream_t s) {
  API_BEGIN
  require(p && f_prev_dev && E0_dev && f_dev && E_dev && vo, "null argument");
  require(prev_slices == 1 || prev_slices == p->R, "prev_slices must be 1 or the number of time slices");
  require(vo->max_fp >= 1 && vo->fp_tol > 0, "max_fp must be >= 1 and fp_tol > 0");
  require(vo->solve.pc.kind == 0, "the fixed point uses the combination-technique preconditioner");
  const auto t0 = std::chrono::steady_clock::now();
  p->assemble_s = 0;
  sgdg_vp_stats out{};
  const int64_t nd = int64_t(p->R) * p->g->up_pts;
  const int64_t ne = int64_t(p->d) * p->nfine;
  DevBuf b, Enew, rho;
  b.alloc(sizeof(double) * nd);
  Enew.alloc(sizeof(double) * ne);
  rho.alloc(sizeof(double) * p->nfine);
  SGDG_CHECK_HIP(hipMemcpyAsync(E_dev, E0_dev, sizeof(double) * ne, hipMemcpyDeviceToDevice, s));
  SGDG_CHECK_HIP(hipMemsetAsync(f_dev, 0, sizeof(double) * nd, s));
  double* fold = ptr<double>(p->fprev_it);
  for (int it = 1; it <= vo->max_fp; ++it) {
    // transport with the current field (a new operator: the field enters the factors)
    SGDG_CHECK_HIP(hipMemcpyAsync(p->Ehost.data(), E_dev, sizeof(double) * ne, hipMemcpyDeviceToHost, s));
    SGDG_CHECK_HIP(hipStreamSynchronize(s));
    vp_assemble(p);
    sgdg_status r = sgdg_rhs(p->ops, f_prev_dev, prev_slices, nullptr, nullptr, ptr<double>(b), s);
    if (r != SGDG_OK) throw Error{r, sgdg_last_error()};
    SGDG_CHECK_HIP(hipMemcpyAsync(fold, f_dev, sizeof(double) * nd, hipMemcpyDeviceToDevice, s));
    sgdg_solve_stats ss{};
    r = sgdg_solve_strip(p->ops, ptr<double>(b), f_dev, &vo->solve, &ss, s);
    if (r != SGDG_OK && r != SGDG_E_NOCONV) throw Error{r, sgdg_last_error()};
    out.outer_iters += ss.outer_iters;
    out.inner_iters += ss.inner_iters_total;
    out.rel_residual = ss.rel_residual;
    // the new field from the density at the strip's midpoint
    vp_density(p, f_dev, p->R, 0.0, ptr<double>(rho), s);
    vp_field(p, ptr<double>(rho), ptr<double>(Enew), 1e-14, 50000, s);
    // changes: max |E_new - E| and the L2 norm of the midpoint slice of f - f_old
    vp_grids(p, 0.0);
    const int64_t npts = p->g->up_pts;
    hipLaunchKernelGGL(k_vp_slice_diff, dim3(unsigned((npts + 255) / 256)), dim3(256), 0, s, p->G, npts, f_dev,
                       it == 1 ? nullptr : fold, ptr<double>(p->slice));
    SGDG_CHECK_HIP(hipGetLastError());
    r = sgdg_apply_operator(p->ops, SGDG_OP_MASS, p->slice.p, p->mslice.p, SGDG_F64, 1, s);
    if (r != SGDG_OK) throw Error{r, sgdg_last_error()};
    hipLaunchKernelGGL(k_vp_diffdot, dim3(1), dim3(kVB), 0, s, ne, ptr<double>(Enew), E_dev, ptr<double>(p->slice),
                       ptr<double>(p->mslice), ptr<double>(p->out) + 4);
    SGDG_CHECK_HIP(hipGetLastError());
    SGDG_CHECK_HIP(hipMemcpyAsync(E_dev, Enew.p, sizeof(double) * ne, hipMemcpyDeviceToDevice, s));
    double h[6];
    SGDG_CHECK_HIP(hipMemcpyAsync(h, p->out.p, sizeof(h), hipMemcpyDeviceToHost, s));
    SGDG_CHECK_HIP(hipStreamSynchronize(s));
    out.fp_iters = it;
    out.energy = h[0];
    out.dE = h[4];
    out.df = it == 1 ? INFINITY : std::sqrt(std::fabs(h[5]));
    if (!std::isfinite(h[4])) throw Error{SGDG_E_NAN, "non-finite field"};
    if (out.dE + out.df < vo->fp_tol) break;
  }
  out.assemble_seconds = p->assemble_s;
  out.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (st) *st = out;
  if (out.dE + out.df >= vo->fp_tol) throw Error{SGDG_E_NOCONV, "fixed point not converged within max_fp"};
  API_END
}
