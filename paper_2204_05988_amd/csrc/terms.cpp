// Kronecker term lists of the strip operator (Sect. 4.2).
//
// For time-independent separable coefficients the block formula reads
//   A = (Tt + delta Ct + Gt) (x) M  +  delta Tt (x) T^T  +  delta Tt^T (x) (T + K)
//       + Mt (x) (T + delta C + K + delta K~ - G),
// with the K~ term carrying delta (expanding (sigma v, delta d_beta w) from the
// weak form (eq:weak_form_j)).  Spatial matrices (row = test phi, column =
// trial phi'):
//   M  = (phi', phi)                      -> M^x (x) M^v
//   T  = (beta.grad phi', phi)            -> per component c: D_c[a] (x) M[b] or M[a] (x) D_c[b]
//   C  = (beta.grad phi', beta.grad phi)  -> per pair (c, c'): stiffness / derivative products
//   K  = (sigma phi', phi)                -> M[p] (x) M[q]
//   K~ = (sigma phi', beta.grad phi)      -> transposed derivative factors
//   -G = inflow integral of |beta.n| phi' phi; on a face with normal velocity
//        s a(x) b(v):  (s a)^+ b^- + (s a)^- b^+ (each a P1 interpolant of kinked values).
// Time blocks on a strip of length dt in the Legendre basis (closed forms):
//   Mt = diag(dt/(2s+1)),  Tt[s][s'] = 2 if s' > s and s + s' odd,
//   Ct[s][s'] = (2/dt) min(s,s')(min(s,s')+1) if s + s' even,  Gt[s][s'] = (-1)^(s+s').
// The data functionals use  (f, w + delta(d_t w + d_beta w)) -> (Mt + delta Tt^T) (x) M + delta Mt (x) T^T
// and  inflow |beta.n| g w -> Mt (x) (-G).
#include <algorithm>
#include <cmath>
#include <map>
#include <stdexcept>

#include "sgdg_internal.h"

namespace sgdg {

void time_matrices(int r, double dt, double Mt[], double Tt[], double Ct[], double Gt[]) {
  const int R = r + 1;
  for (int s = 0; s < R; ++s)
    for (int q = 0; q < R; ++q) {
      const int i = s * R + q;
      Mt[i] = s == q ? dt / (2 * s + 1) : 0.0;
      Tt[i] = (q > s && ((s + q) & 1)) ? 2.0 : 0.0;
      const int mn = std::min(s, q);
      Ct[i] = ((s + q) & 1) ? 0.0 : (2.0 / dt) * mn * (mn + 1);
      Gt[i] = ((s + q) & 1) ? -1.0 : 1.0;
    }
}

namespace {

struct KTerm {  // coef * X (x) V
  double c;
  FactorKey X, V;
};

Weight plain(DomainData& D, const sgdg_separable* sep, bool xside, int64_t n) {
  Weight w;
  w.scale = 1.0;
  const int nf = xside ? sep->n_xf : sep->n_vf;
  const double* const* f = xside ? sep->xf : sep->vf;
  for (int i = 0; i < nf; ++i) w.fields.push_back(D.field_id(f[i], n));
  std::sort(w.fields.begin(), w.fields.end());
  return w;
}

Weight concat(const Weight& a, const Weight& b) {
  Weight w;
  w.scale = a.scale * b.scale;
  w.fields = a.fields;
  w.fields.insert(w.fields.end(), b.fields.begin(), b.fields.end());
  std::sort(w.fields.begin(), w.fields.end());
  return w;
}

FactorKey key(int kind, const Weight& w, int a = -1, int b = -1, int axis = -1, int side = -1) {
  FactorKey k;
  k.kind = kind;
  k.w = w;
  k.a = a;
  k.b = b;
  k.axis = axis;
  k.side = side;
  return k;
}

FactorKey tr(FactorKey k) {
  // a transposed symmetric factor is the factor itself
  if (k.kind == kMass || k.kind == kFace) return k;
  if (k.kind == kStiff) {
    std::swap(k.a, k.b);
    return k;
  }
  k.trans = !k.trans;
  return k;
}

bool weight_zero(const DomainData& D, const Weight& w) {
  if (w.kink == 0) return w.scale == 0.0;
  const int64_t n = D.L(D.lmax).n;
  for (int64_t p = 0; p < n; ++p) {
    double v = w.scale;
    for (int f : w.fields) v *= D.fields[f][p];
    if ((w.kink == 1 && v > 0) || (w.kink == 2 && v < 0)) return false;
  }
  return true;
}

}  // namespace

namespace {

// The spatial operators of one coefficient set as Kronecker lists.
struct Spatial {
  std::vector<KTerm> M, T, C, K, Kt, Gm;
};

Spatial spatial_terms(DomainData& X, DomainData& V, const sgdg_problem& p) {
  const int d = X.dom.d;
  const int64_t nx = X.L(X.lmax).n, nv = V.L(V.lmax).n;
  Spatial S;
  const Weight one;
  S.M.push_back({1.0, key(kMass, one), key(kMass, one)});

  std::vector<Weight> A(2 * d), B(2 * d);
  std::vector<double> sc(2 * d, 0.0);
  std::vector<bool> has(2 * d, false);
  for (int c = 0; c < 2 * d; ++c) {
    if (!p.beta[c]) continue;
    has[c] = true;
    sc[c] = p.beta[c]->scale;
    A[c] = plain(X, p.beta[c], true, nx);
    B[c] = plain(V, p.beta[c], false, nv);
  }
  for (int c = 0; c < 2 * d; ++c) {
    if (!has[c]) continue;
    if (c < d) S.T.push_back({sc[c], key(kDeriv, A[c], c), key(kMass, B[c])});
    else S.T.push_back({sc[c], key(kMass, A[c]), key(kDeriv, B[c], c - d)});
  }
  for (int c = 0; c < 2 * d; ++c)
    for (int c2 = 0; c2 < 2 * d; ++c2) {
      if (!has[c] || !has[c2]) continue;
      const Weight wa = concat(A[c], A[c2]), wb = concat(B[c], B[c2]);
      // (beta_c d_c phi', beta_c2 d_c2 phi)
      FactorKey fx, fv;
      if (c < d && c2 < d) {
        fx = key(kStiff, wa, c, c2);
        fv = key(kMass, wb);
      } else if (c < d) {
        fx = key(kDeriv, wa, c);
        fv = tr(key(kDeriv, wb, c2 - d));
      } else if (c2 < d) {
        fx = tr(key(kDeriv, wa, c2));
        fv = key(kDeriv, wb, c - d);
      } else {
        fx = key(kMass, wa);
        fv = key(kStiff, wb, c - d, c2 - d);
      }
      S.C.push_back({sc[c] * sc[c2], fx, fv});
    }
  for (int t = 0; t < p.n_sigma; ++t) {
    const sgdg_separable* s = &p.sigma[t];
    const Weight P = plain(X, s, true, nx), Q = plain(V, s, false, nv);
    S.K.push_back({s->scale, key(kMass, P), key(kMass, Q)});
    for (int c = 0; c < 2 * d; ++c) {
      if (!has[c]) continue;
      const Weight wa = concat(P, A[c]), wb = concat(Q, B[c]);
      // (sigma phi', beta_c d_c phi)
      if (c < d) S.Kt.push_back({s->scale * sc[c], tr(key(kDeriv, wa, c)), key(kMass, wb)});
      else S.Kt.push_back({s->scale * sc[c], key(kMass, wa), tr(key(kDeriv, wb, c - d))});
    }
  }
  for (int side_dom = 0; side_dom < 2; ++side_dom) {  // 0: faces of Omega_x, 1: faces of Omega_v
    DomainData& D = side_dom == 0 ? X : V;
    if (D.dom.periodic) continue;
    for (int axis = 0; axis < d; ++axis) {
      const int c = side_dom == 0 ? axis : d + axis;
      if (!has[c]) continue;
      for (int side = 0; side < 2; ++side) {
        const double sgn = side == 0 ? -1.0 : 1.0;
        for (int pass = 0; pass < 2; ++pass) {
          Weight wa = A[c], wb = B[c];
          wa.scale = sgn * sc[c];
          wa.kink = pass == 0 ? 1 : 2;  // (s a)^+ with b^-, then (s a)^- with b^+
          wb.scale = 1.0;
          wb.kink = pass == 0 ? 2 : 1;
          if (weight_zero(X, wa) || weight_zero(V, wb)) continue;
          if (side_dom == 0) S.Gm.push_back({1.0, key(kFace, wa, -1, -1, axis, side), key(kMass, wb)});
          else S.Gm.push_back({1.0, key(kMass, wa), key(kFace, wb, -1, -1, axis, side)});
        }
      }
    }
  }
  return S;
}

// Appends scale * tm (x) ops to L (terms with the same factor pair merge).
void add_terms(DomainData& X, DomainData& V, TermList& L, const double* tm, double scale,
               const std::vector<KTerm>& ops, bool transpose) {
  bool nz = false;
  for (int i = 0; i < L.Rout * L.Rin; ++i) nz = nz || tm[i] != 0.0;
  if (!nz || scale == 0.0) return;
  for (const KTerm& k : ops) {
    Term t;
    const FactorKey fx = transpose ? tr(k.X) : k.X;
    const FactorKey fv = transpose ? tr(k.V) : k.V;
    t.xf = X.factor_id(fx);
    t.vf = V.factor_id(fv);
    for (int i = 0; i < L.Rout * L.Rin; ++i) t.tm[i] = scale * k.c * tm[i];
    bool merged = false;
    for (Term& e : L.terms)
      if (e.xf == t.xf && e.vf == t.vf) {
        for (int i = 0; i < L.Rout * L.Rin; ++i) e.tm[i] += t.tm[i];
        merged = true;
        break;
      }
    if (!merged) L.terms.push_back(t);
  }
}

double legendre_val(int s, double z, double* deriv) {
  // P_s(z) and P_s'(z) by the three-term recurrence
  double p0 = 1, p1 = z, d0 = 0, d1 = 1;
  if (s == 0) {
    *deriv = 0;
    return 1;
  }
  for (int k = 1; k < s; ++k) {
    const double p2 = ((2 * k + 1) * z * p1 - k * p0) / (k + 1);
    const double d2 = ((2 * k + 1) * (p1 + z * d1) - k * d0) / (k + 1);
    p0 = p1;
    p1 = p2;
    d0 = d1;
    d1 = d2;
  }
  *deriv = d1;
  return p1;
}

// tm_j = a tm_i (to rounding), a returned
bool proportional(const double* ti, const double* tj, int n, double* a) {
  int p = 0;
  double mi = 0.0, mj = 0.0;
  for (int k = 0; k < n; ++k) {
    if (std::fabs(ti[k]) > mi) {
      mi = std::fabs(ti[k]);
      p = k;
    }
    mj = std::max(mj, std::fabs(tj[k]));
  }
  if (mi == 0.0 || mj == 0.0) return false;
  const double r = tj[p] / ti[p];
  for (int k = 0; k < n; ++k)
    if (std::fabs(tj[k] - r * ti[k]) > 1e-14 * mj) return false;
  *a = r;
  return true;
}

// The factor c_i F_i + c_j F_j (F_i, F_j of one kind), registered as a
// combination; -1 if the parts cancel.
int combine(DomainData& D, int fi, double ci, int fj, double cj) {
  std::map<int, double> acc;
  auto add = [&](int f, double c) {
    const FactorKey& k = D.factors[size_t(f)];
    if (k.parts.empty()) {
      acc[f] += c;
      return;
    }
    for (const auto& p : k.parts) acc[p.second] += c * p.first;
  };
  add(fi, ci);
  add(fj, cj);
  FactorKey key;
  key.kind = D.factors[size_t(fi)].kind;
  for (const auto& e : acc)
    if (e.second != 0.0) key.parts.push_back({e.second, e.first});
  if (key.parts.empty()) return -1;
  if (key.parts.size() == 1 && key.parts[0].first == 1.0) return key.parts[0].second;
  return D.factor_id(key);
}

// Terms that share one factor and whose time blocks are proportional,
// tm (x) X (x) V_i + a tm (x) X (x) V_j = tm (x) X (x) (V_i + a V_j) (and the
// same with the roles of x and v swapped), become one term with a combined
// factor of the same kind: the passes then run fewer stencils, staged arrays
// and partner scans.  Repeated until no pair is left.
void merge_terms(DomainData& X, DomainData& V, TermList& L) {
  const int n = L.Rout * L.Rin;
  for (bool changed = true; changed;) {
    changed = false;
    for (size_t i = 0; i < L.terms.size() && !changed; ++i)
      for (size_t j = i + 1; j < L.terms.size() && !changed; ++j) {
        Term& a = L.terms[i];
        const Term& b = L.terms[j];
        double r;
        if (a.xf == b.xf && a.vf == b.vf) {  // a pair made equal by an earlier merge
          for (int k = 0; k < n; ++k) a.tm[k] += b.tm[k];
        } else if (!proportional(a.tm, b.tm, n, &r)) {
          continue;
        } else if (a.xf == b.xf && V.factors[size_t(a.vf)].kind == V.factors[size_t(b.vf)].kind) {
          a.vf = combine(V, a.vf, 1.0, b.vf, r);
        } else if (a.vf == b.vf && X.factors[size_t(a.xf)].kind == X.factors[size_t(b.xf)].kind) {
          a.xf = combine(X, a.xf, 1.0, b.xf, r);
        } else {
          continue;
        }
        L.terms.erase(L.terms.begin() + std::ptrdiff_t(j));
        bool zero = a.xf < 0 || a.vf < 0;  // the pair cancels
        if (!zero) {
          zero = true;
          for (int k = 0; k < n; ++k) zero = zero && a.tm[k] == 0.0;
        }
        if (zero) L.terms.erase(L.terms.begin() + std::ptrdiff_t(i));
        changed = true;
      }
  }
}

void init_lists(TermList out[4], int R) {
  out[0].Rin = out[0].Rout = R;
  out[1].Rin = out[1].Rout = 1;
  out[2].Rin = out[2].Rout = R;
  out[3].Rin = out[3].Rout = R;
  for (int k = 0; k < 4; ++k) out[k].terms.clear();
}

}  // namespace

void build_terms(DomainData& X, DomainData& V, const sgdg_problem& p, int r, TermList out[4]) {
  const int R = r + 1;
  const double dl = p.delta;
  const Spatial S = spatial_terms(X, V, p);
  double Mt[9], Tt[9], Ct[9], Gt[9], TtT[9];
  time_matrices(r, p.dt, Mt, Tt, Ct, Gt);
  for (int s = 0; s < R; ++s)
    for (int q = 0; q < R; ++q) TtT[s * R + q] = Tt[q * R + s];
  init_lists(out, R);
  // FULL
  TermList& F = out[0];
  double P0[9];
  for (int i = 0; i < R * R; ++i) P0[i] = Tt[i] + dl * Ct[i] + Gt[i];
  add_terms(X, V, F, P0, 1.0, S.M, false);
  add_terms(X, V, F, Tt, dl, S.T, true);
  add_terms(X, V, F, TtT, dl, S.T, false);
  add_terms(X, V, F, TtT, dl, S.K, false);
  add_terms(X, V, F, Mt, 1.0, S.T, false);
  add_terms(X, V, F, Mt, dl, S.C, false);
  add_terms(X, V, F, Mt, 1.0, S.K, false);
  add_terms(X, V, F, Mt, dl, S.Kt, false);
  add_terms(X, V, F, Mt, 1.0, S.Gm, false);
  // MASS
  const double one1[1] = {1.0};
  add_terms(X, V, out[1], one1, 1.0, S.M, false);
  // DATA_F
  double P1[9];
  for (int i = 0; i < R * R; ++i) P1[i] = Mt[i] + dl * TtT[i];
  add_terms(X, V, out[2], P1, 1.0, S.M, false);
  add_terms(X, V, out[2], Mt, dl, S.T, true);
  // DATA_G
  add_terms(X, V, out[3], Mt, 1.0, S.Gm, false);
  for (int k = 0; k < 4; ++k) merge_terms(X, V, out[k]);
}

// Coefficients that depend on time (Sect. 4.2, the block formula with an
// m-point time quadrature): per point mu the spatial factors of the
// coefficients at tau_mu and the time matrices w_mu eta_s'(tau_mu) eta_s(tau_mu)
// (M_mu), w_mu eta'_s'(tau_mu) eta_s(tau_mu) (T_mu), w_mu eta'_s' eta'_s (C_mu):
//   A = G^t (x) M + sum_mu [ (T_mu + delta C_mu) (x) M + delta T_mu (x) T_mu^T
//       + delta T_mu^T (x) (T_mu + K_mu) + M_mu (x) (T_mu + delta C_mu + K_mu + delta K~_mu - G_mu) ],
// and the data functionals (M^t + delta T^t^T) (x) M + sum_mu delta M_mu (x) T_mu^T
// and sum_mu M_mu (x) (-G_mu).
void build_terms_t(DomainData& X, DomainData& V, const sgdg_problem* at, const double* tau, const double* wref, int m,
                   int r, TermList out[4]) {
  const int R = r + 1;
  const double dt = at[0].dt, dl = at[0].delta;
  double Mt[9], Tt[9], Ct[9], Gt[9], TtT[9];
  time_matrices(r, dt, Mt, Tt, Ct, Gt);
  for (int s = 0; s < R; ++s)
    for (int q = 0; q < R; ++q) TtT[s * R + q] = Tt[q * R + s];
  init_lists(out, R);
  const Spatial S0 = spatial_terms(X, V, at[0]);
  add_terms(X, V, out[0], Gt, 1.0, S0.M, false);
  const double one1[1] = {1.0};
  add_terms(X, V, out[1], one1, 1.0, S0.M, false);
  double P1[9];
  for (int i = 0; i < R * R; ++i) P1[i] = Mt[i] + dl * TtT[i];
  add_terms(X, V, out[2], P1, 1.0, S0.M, false);
  for (int mu = 0; mu < m; ++mu) {
    const Spatial S = spatial_terms(X, V, at[mu]);
    double e[kMaxR], de[kMaxR];
    for (int s = 0; s < R; ++s) {
      double dp;
      e[s] = legendre_val(s, tau[mu], &dp);
      de[s] = dp * 2.0 / dt;
    }
    const double w = wref[mu] * dt / 2.0;
    double Mm[9], Tm[9], Cm[9], TmT[9], P0[9];
    for (int s = 0; s < R; ++s)
      for (int q = 0; q < R; ++q) {
        Mm[s * R + q] = w * e[q] * e[s];
        Tm[s * R + q] = w * de[q] * e[s];
        Cm[s * R + q] = w * de[q] * de[s];
        TmT[s * R + q] = w * de[s] * e[q];
      }
    for (int i = 0; i < R * R; ++i) P0[i] = Tm[i] + dl * Cm[i];
    TermList& F = out[0];
    add_terms(X, V, F, P0, 1.0, S.M, false);
    add_terms(X, V, F, Tm, dl, S.T, true);
    add_terms(X, V, F, TmT, dl, S.T, false);
    add_terms(X, V, F, TmT, dl, S.K, false);
    add_terms(X, V, F, Mm, 1.0, S.T, false);
    add_terms(X, V, F, Mm, dl, S.C, false);
    add_terms(X, V, F, Mm, 1.0, S.K, false);
    add_terms(X, V, F, Mm, dl, S.Kt, false);
    add_terms(X, V, F, Mm, 1.0, S.Gm, false);
    add_terms(X, V, out[2], Mm, dl, S.T, true);
    add_terms(X, V, out[3], Mm, 1.0, S.Gm, false);
  }
  for (int k = 0; k < 4; ++k) merge_terms(X, V, out[k]);
}

}  // namespace sgdg
