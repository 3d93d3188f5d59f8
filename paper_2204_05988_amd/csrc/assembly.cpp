// Factor matrices of the strip operator (Sect. 4.2, (eq:matrices)).
//
// Every factor is a bilinear form on the P1 space of one domain, weighted by
// a product of P1 fields:
//   mass    (w phi_k', phi_k)            deriv(a)   (w d_a phi_k', phi_k)
//   stiff(a,b) (w d_a phi_k', d_b phi_k)  face(f)    int_f w phi_k' phi_k
// (row k = test, column k' = trial).  On the finest level each simplex
// contributes exactly: with lambda the barycentric coordinates,
//   int_K prod lambda^alpha = |K| dim! prod alpha_i! / (dim + |alpha|)!,
// and a Kuhn simplex of the chain c, c+e_p0, c+e_p0+e_p1, ... has constant
// gradients grad lambda_0 = -e_p0/h, grad lambda_k = e_p(k-1)/h - e_pk/h,
// grad lambda_d = e_p(d-1)/h and volume prod h / d!.  Coarser levels follow
// by the Galerkin identity X_l = E_{l+1,l}^T X_{l+1} E_{l+1,l} (Sect. 4.2).
// Values are stored per row in the Kuhn stencil slots ([n][S]); a slot is the
// unwrapped lattice offset of the element edge, so periodic lattices with
// coinciding neighbours stay exact.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <stdexcept>

#include "sgdg_internal.h"

namespace sgdg {

static double factorial(int n) {
  double r = 1;
  for (int i = 2; i <= n; ++i) r *= i;
  return r;
}

// exponent tuples of a product of m linear fields on a simplex with nv vertices
struct TupleTable {
  int m = 0, nv = 0, ntup = 0;
  std::vector<int> tup;  // [ntup][m]
  void init(int m_, int nv_) {
    m = m_;
    nv = nv_;
    ntup = 1;
    for (int i = 0; i < m; ++i) ntup *= nv;
    tup.assign(size_t(ntup) * std::max(m, 1), 0);
    for (int t = 0; t < ntup; ++t) {
      int x = t;
      for (int i = 0; i < m; ++i) {
        tup[t * m + i] = x % nv;
        x /= nv;
      }
    }
  }
  // coefficient of tuple t for extra vertices (e1, e2; -1 = none): dim! prod a! / (dim+|a|)!
  double coef(int t, int e1, int e2, int dim) const {
    int alpha[4] = {0, 0, 0, 0};
    for (int i = 0; i < m; ++i) alpha[tup[t * m + i]]++;
    if (e1 >= 0) alpha[e1]++;
    if (e2 >= 0) alpha[e2]++;
    double num = 1;
    int tot = 0;
    for (int v = 0; v < nv; ++v) {
      num *= factorial(alpha[v]);
      tot += alpha[v];
    }
    return factorial(dim) * num / factorial(dim + tot);
  }
};

static inline void unflat(int64_t p, int d, int m, int* i) {
  for (int a = d - 1; a >= 0; --a) {
    i[a] = int(p % m);
    p /= m;
  }
}

static inline int64_t flat_wrap(const int* i, int d, int m, bool periodic, int ncell) {
  int64_t p = 0;
  for (int a = 0; a < d; ++a) {
    int x = i[a];
    if (periodic) x = ((x % ncell) + ncell) % ncell;
    p = p * m + x;
  }
  return p;
}

// nodal values of the weight's factors on the finest level: either the plain
// fields (product expanded exactly) or one kinked field.
static void weight_fields(const DomainData& D, const Weight& w, std::vector<std::vector<double>>& out,
                          double& scale) {
  out.clear();
  if (w.kink == 0) {
    scale = w.scale;
    for (int f : w.fields) out.push_back(D.fields[f]);
    return;
  }
  const int64_t n = D.L(D.lmax).n;
  std::vector<double> k(n, w.scale);
  for (int f : w.fields)
    for (int64_t p = 0; p < n; ++p) k[p] *= D.fields[f][p];
  for (int64_t p = 0; p < n; ++p) k[p] = w.kink == 1 ? std::max(k[p], 0.0) : std::max(-k[p], 0.0);
  out.push_back(std::move(k));
  scale = 1.0;
}

static void assemble_finest(const DomainData& D, const FactorKey& key, std::vector<double>& val) {
  const Dom& dom = D.dom;
  const int d = dom.d, S = D.st.S, L = D.lmax, ncell = 1 << L;
  const LevelTables& T = D.L(L);
  val.assign(T.n * S, 0.0);
  std::vector<std::vector<double>> wf;
  double scale = 1;
  weight_fields(D, key.w, wf, scale);
  const int m = int(wf.size());
  double hvec[3] = {dom.h(L, 0), d > 1 ? dom.h(L, 1) : 1, d > 2 ? dom.h(L, 2) : 1};

  const bool face = key.kind == kFace;
  const int nv = face ? d : d + 1;     // vertices of the integration simplex
  const int dim = face ? d - 1 : d;
  TupleTable tt;
  tt.init(m, nv);
  // precomputed coefficient tables
  std::vector<double> c2(size_t(tt.ntup) * nv * nv), c1(size_t(tt.ntup) * nv), c0(tt.ntup);
  for (int t = 0; t < tt.ntup; ++t) {
    c0[t] = tt.coef(t, -1, -1, dim);
    for (int a = 0; a < nv; ++a) {
      c1[t * nv + a] = tt.coef(t, a, -1, dim);
      for (int b = 0; b < nv; ++b) c2[(t * nv + a) * nv + b] = tt.coef(t, a, b, dim);
    }
  }
  std::vector<int> perm(d);
  std::iota(perm.begin(), perm.end(), 0);
  std::vector<std::vector<int>> perms;
  do perms.push_back(perm);
  while (std::next_permutation(perm.begin(), perm.end()));

  double vol = 1;
  for (int a = 0; a < d; ++a) vol *= hvec[a];
  vol /= factorial(d);
  double fmeas = 1;
  if (face) {
    for (int a = 0; a < d; ++a)
      if (a != key.axis) fmeas *= hvec[a];
    fmeas /= factorial(d - 1);
  }

  int64_t ncells = 1;
  for (int a = 0; a < d; ++a) ncells *= ncell;
  std::vector<double> prods(tt.ntup);
  int cell[3], vert[4][3], fv[4][3];
  int64_t vidx[4], fidx[4];
  double grad[4][3];
  for (int64_t c = 0; c < ncells; ++c) {
    unflat(c, d, ncell, cell);
    if (face) {
      const int want = key.side == 0 ? 0 : ncell - 1;
      if (cell[key.axis] != want) continue;
    }
    for (const auto& pm : perms) {
      for (int a = 0; a < d; ++a) vert[0][a] = cell[a];
      for (int k = 1; k <= d; ++k) {
        for (int a = 0; a < d; ++a) vert[k][a] = vert[k - 1][a];
        vert[k][pm[k - 1]] += 1;
      }
      for (int k = 0; k <= d; ++k) vidx[k] = flat_wrap(vert[k], d, T.m, dom.periodic, ncell);
      int nvk = d + 1;
      const int(*V)[3] = vert;
      const int64_t* VI = vidx;
      if (face) {  // keep the vertices on the face; need exactly d of them
        const int target = key.side == 0 ? 0 : ncell;
        int cnt = 0;
        for (int k = 0; k <= d; ++k)
          if (vert[k][key.axis] == target) {
            for (int a = 0; a < d; ++a) fv[cnt][a] = vert[k][a];
            fidx[cnt++] = vidx[k];
          }
        if (cnt != d) continue;
        nvk = d;
        V = fv;
        VI = fidx;
      } else {
        for (int k = 0; k <= d; ++k)
          for (int a = 0; a < 3; ++a) grad[k][a] = 0;
        grad[0][pm[0]] = -1.0 / hvec[pm[0]];
        for (int k = 1; k < d; ++k) {
          grad[k][pm[k - 1]] += 1.0 / hvec[pm[k - 1]];
          grad[k][pm[k]] -= 1.0 / hvec[pm[k]];
        }
        grad[d][pm[d - 1]] += 1.0 / hvec[pm[d - 1]];
      }
      for (int t = 0; t < tt.ntup; ++t) {
        double pr = 1;
        for (int i = 0; i < m; ++i) pr *= wf[i][VI[tt.tup[t * m + i]]];
        prods[t] = pr;
      }
      const double meas = face ? fmeas : vol;
      for (int a = 0; a < nvk; ++a) {      // test vertex
        for (int b = 0; b < nvk; ++b) {    // trial vertex
          double I = 0;
          switch (key.kind) {
            case kMass:
            case kFace:
              for (int t = 0; t < tt.ntup; ++t) I += prods[t] * c2[(t * nv + a) * nv + b];
              break;
            case kDeriv:
              for (int t = 0; t < tt.ntup; ++t) I += prods[t] * c1[t * nv + a];
              I *= grad[b][key.a];
              break;
            case kStiff:
              for (int t = 0; t < tt.ntup; ++t) I += prods[t] * c0[t];
              I *= grad[b][key.a] * grad[a][key.b];
              break;
          }
          I *= meas * scale;
          int o[3] = {0, 0, 0};
          for (int x = 0; x < d; ++x) o[x] = V[b][x] - V[a][x];
          const int e = D.st.slot(o);
          if (e < 0) throw Error{SGDG_E_STATE, "assembly: element edge is not a Kuhn offset"};
          val[VI[a] * S + e] += I;
        }
      }
    }
  }
}

// X_l = E^T X_{l+1} E, stencil form
static void restrict_galerkin(const DomainData& D, int l, const std::vector<double>& fine,
                              std::vector<double>& coarse) {
  const Dom& dom = D.dom;
  const int d = dom.d, S = D.st.S;
  const LevelTables& C = D.L(l);
  const LevelTables& F = D.L(l + 1);
  coarse.assign(C.n * S, 0.0);
  int iP[3], q[3];
  for (int64_t P = 0; P < C.n; ++P) {
    unflat(P, d, C.m, iP);
    for (int c = 0; c < S; ++c) {
      const double wc = C.chiw[P * S + c];
      if (wc == 0.0) continue;
      const int64_t p = C.chi[P * S + c];
      for (int e = 0; e < S; ++e) {
        const double x = fine[p * S + e];
        if (x == 0.0) continue;
        int odd[3] = {0, 0, 0};
        bool any = false;
        for (int a = 0; a < d; ++a) {
          q[a] = 2 * iP[a] + D.st.off[c][a] + D.st.off[e][a];
          odd[a] = ((q[a] % 2) + 2) % 2;
          any = any || odd[a];
        }
        for (int k = 0; k < (any ? 2 : 1); ++k) {
          int O[3] = {0, 0, 0};
          for (int a = 0; a < d; ++a) {
            const int Q = (k == 0 ? (q[a] - odd[a]) : (q[a] + odd[a])) / 2;
            O[a] = Q - iP[a];
          }
          const int s = D.st.slot(O);
          if (s < 0) throw Error{SGDG_E_STATE, "restriction: coarse coupling outside the Kuhn stencil"};
          coarse[P * S + s] += wc * x * (any ? 0.5 : 1.0);
        }
      }
    }
  }
}

static void transpose_level(const DomainData& D, int l, const std::vector<double>& X, std::vector<double>& T) {
  const int S = D.st.S;
  const LevelTables& Lt = D.L(l);
  T.assign(Lt.n * S, 0.0);
  for (int64_t p = 0; p < Lt.n; ++p)
    for (int e = 0; e < S; ++e)
      if (Lt.valid[p * S + e]) T[p * S + e] = X[int64_t(Lt.nbr[p * S + e]) * S + D.st.neg(e)];
}

void build_wide_tables(DomainData& D) {
  const Dom& dom = D.dom;
  const int d = dom.d, S = D.st.S;
  D.woff.clear();
  for (int a = 0; a < S; ++a)
    for (int b = 0; b < S; ++b) {
      std::array<int, 3> o{0, 0, 0};
      for (int x = 0; x < d; ++x) o[x] = D.st.off[a][x] + D.st.off[b][x];
      if (std::find(D.woff.begin(), D.woff.end(), o) == D.woff.end()) D.woff.push_back(o);
    }
  std::sort(D.woff.begin(), D.woff.end());
  const int W = int(D.woff.size());
  D.wide_idx.assign(D.lmax - D.lmin + 1, {});
  int iP[3], q[3];
  for (int l = D.lmin; l < D.lmax; ++l) {
    const LevelTables& C = D.L(l);
    const int mf = dom.axis_nodes(l + 1), nf = 1 << (l + 1);
    auto& tab = D.wide_idx[l - D.lmin];
    tab.assign(C.n * W, 0);
    for (int64_t P = 0; P < C.n; ++P) {
      unflat(P, d, C.m, iP);
      for (int w = 0; w < W; ++w) {
        bool ok = true;
        for (int a = 0; a < d; ++a) {
          q[a] = 2 * iP[a] + D.woff[w][a];
          if (dom.periodic) q[a] = ((q[a] % nf) + nf) % nf;
          else if (q[a] < 0 || q[a] >= mf) ok = false;
        }
        if (!ok)
          for (int a = 0; a < d; ++a) q[a] = dom.periodic ? ((2 * iP[a]) % nf) : 2 * iP[a];
        int64_t f = 0;
        for (int a = 0; a < d; ++a) f = f * mf + q[a];
        tab[P * W + w] = int32_t(f);
      }
    }
  }
}

void restrict_factor(DomainData& D, int fid) {
  const int S = D.st.S, W = int(D.woff.size()), d = D.dom.d;
  // slot of off_c + off_e in woff
  std::vector<int> pair(S * S);
  for (int c = 0; c < S; ++c)
    for (int e = 0; e < S; ++e) {
      std::array<int, 3> o{0, 0, 0};
      for (int x = 0; x < d; ++x) o[x] = D.st.off[c][x] + D.st.off[e][x];
      pair[c * S + e] = int(std::find(D.woff.begin(), D.woff.end(), o) - D.woff.begin());
    }
  auto& out = D.rvalues[fid];
  out.assign(D.lmax - D.lmin + 1, {});
  for (int l = D.lmin; l < D.lmax; ++l) {
    const LevelTables& C = D.L(l);
    const auto& fine = D.values[fid][l + 1 - D.lmin];
    auto& r = out[l - D.lmin];
    r.assign(C.n * W, 0.0);
    for (int64_t P = 0; P < C.n; ++P)
      for (int c = 0; c < S; ++c) {
        const double wc = C.chiw[P * S + c];
        if (wc == 0.0) continue;
        const int64_t fc = C.chi[P * S + c];
        for (int e = 0; e < S; ++e) r[P * W + pair[c * S + e]] += wc * fine[fc * S + e];
      }
  }
}

// Kuhn refinement: a fine node 2a + b (b in {0,1}^d) is the midpoint of the
// coarse edge a -> a + b, so its parents are floor(q/2) and ceil(q/2) with
// weights 1/2 each, or the single node q/2 when q is even.
static int pro_slot(const int* q, const int* base, int d) {
  int s = 0;
  for (int a = d - 1; a >= 0; --a) s = s * 3 + (q[a] - base[a] + 1);
  return s;
}

void build_prolong_tables(DomainData& D) {
  const Dom& dom = D.dom;
  const int d = dom.d;
  int PW = 1;
  for (int a = 0; a < d; ++a) PW *= 3;
  D.pro_idx.assign(D.lmax - D.lmin + 1, {});
  int q[3], base[3], c[3];
  for (int l = D.lmin + 1; l <= D.lmax; ++l) {
    const LevelTables& F = D.L(l);
    const int mc = dom.axis_nodes(l - 1), nc = 1 << (l - 1);
    auto& tab = D.pro_idx[l - D.lmin];
    tab.assign(size_t(F.n) * PW, 0);
    for (int64_t P = 0; P < F.n; ++P) {
      unflat(P, d, F.m, q);
      for (int a = 0; a < d; ++a) base[a] = q[a] >> 1;
      // a slot outside a non-periodic lattice carries weight 0; it points at the
      // nearest lattice node so that every slot of a node stays next to its base
      for (int sl = 0; sl < PW; ++sl) {
        int t = sl;
        for (int a = 0; a < d; ++a) {
          c[a] = base[a] + (t % 3) - 1;
          t /= 3;
          if (!dom.periodic) c[a] = std::min(std::max(c[a], 0), mc - 1);
        }
        tab[size_t(sl) * F.n + P] = int32_t(flat_wrap(c, d, mc, dom.periodic, nc));
      }
    }
  }
}

void prolong_factor(DomainData& D, int fid) {
  const Dom& dom = D.dom;
  const int d = dom.d, S = D.st.S;
  int PW = 1;
  for (int a = 0; a < d; ++a) PW *= 3;
  auto& out = D.pvalues[fid];
  out.assign(D.lmax - D.lmin + 1, {});
  int q[3], base[3], f[3], lo[3], hi[3];
  for (int l = D.lmin + 1; l <= D.lmax; ++l) {
    const LevelTables& F = D.L(l);
    const auto& X = D.values[fid][l - D.lmin];
    auto& r = out[l - D.lmin];
    r.assign(size_t(F.n) * PW, 0.0);
    for (int64_t P = 0; P < F.n; ++P) {
      unflat(P, d, F.m, q);
      for (int a = 0; a < d; ++a) base[a] = q[a] >> 1;
      for (int e = 0; e < S; ++e) {
        if (!F.valid[P * S + e]) continue;
        const double xv = X[P * S + e];
        if (xv == 0.0) continue;
        bool even = true;
        for (int a = 0; a < d; ++a) {
          f[a] = q[a] + D.st.off[e][a];  // unwrapped fine neighbour
          lo[a] = f[a] >> 1;             // arithmetic shift: floor for -1 too
          hi[a] = (f[a] + 1) >> 1;
          even = even && lo[a] == hi[a];
        }
        if (even) {
          r[size_t(pro_slot(lo, base, d)) * F.n + P] += xv;
        } else {
          r[size_t(pro_slot(lo, base, d)) * F.n + P] += 0.5 * xv;
          r[size_t(pro_slot(hi, base, d)) * F.n + P] += 0.5 * xv;
        }
      }
    }
  }
}

void assemble_factor(DomainData& D, int fid) {
  FactorKey key = D.factors[fid];
  const int nlev = D.lmax - D.lmin + 1;
  std::vector<std::vector<double>> vals(nlev);
  if (!key.parts.empty()) {
    // a combination: the same linear combination of its parts on every level
    // (the Galerkin restriction and the transposition are linear)
    for (int l = 0; l < nlev; ++l) {
      const size_t n = D.values[size_t(key.parts[0].second)][size_t(l)].size();
      vals[size_t(l)].assign(n, 0.0);
      for (const auto& p : key.parts) {
        const auto& src = D.values[size_t(p.second)][size_t(l)];
        if (src.size() != n) throw std::logic_error("combination of factors assembled before its parts");
        for (size_t i = 0; i < n; ++i) vals[size_t(l)][i] += p.first * src[i];
      }
    }
    D.values[fid] = std::move(vals);
    return;
  }
  FactorKey base = key;
  base.trans = false;
  assemble_finest(D, base, vals[nlev - 1]);
  for (int l = D.lmax - 1; l >= D.lmin; --l) restrict_galerkin(D, l, vals[l + 1 - D.lmin], vals[l - D.lmin]);
  if (key.trans) {
    for (int l = D.lmin; l <= D.lmax; ++l) {
      std::vector<double> t;
      transpose_level(D, l, vals[l - D.lmin], t);
      vals[l - D.lmin].swap(t);
    }
  }
  D.values[fid] = std::move(vals);
}

void assemble_all(DomainData& D) {
  D.values.assign(D.factors.size(), {});
  D.rvalues.assign(D.factors.size(), {});
  D.pvalues.assign(D.factors.size(), {});
  build_wide_tables(D);
  build_prolong_tables(D);
  for (int phase = 0; phase < 2; ++phase) {
    // assembled factors first, then the combinations of them
#pragma omp parallel for schedule(dynamic)
    for (int f = 0; f < int(D.factors.size()); ++f) {
      if (D.factors[size_t(f)].parts.empty() != (phase == 0)) continue;
      assemble_factor(D, f);
      restrict_factor(D, f);
      prolong_factor(D, f);
    }
  }
}

}  // namespace sgdg
