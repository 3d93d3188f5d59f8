// Lattice tables of the nested Kuhn meshes (Sect. 2: nested spaces by uniform refinement).
//
// Level l of a box has 2^l cells per axis; each cell is split into d! Kuhn
// simplices along its main diagonal.  The P1 stiffness pattern of such a mesh
// couples a node with the nodes at offsets +-b, b a non-zero 0/1 vector (the
// Kuhn edge directions): 3, 7 and 15 entries per row for d = 1, 2, 3.
//
// Embedding E_{l+1,l} (Sect. 4.2): a fine node with all lattice coordinates
// even is a coarse node (weight 1); otherwise, with S the set of odd
// coordinates, it is the midpoint of the coarse Kuhn edge from (q - 1_S)/2 to
// (q + 1_S)/2 (weights 1/2, 1/2).  The transpose gathers, for a coarse node P,
// the fine nodes 2P + off (weight 1 at the centre, 1/2 elsewhere).
#include <algorithm>
#include <cstring>
#include <stdexcept>

#include "sgdg_internal.h"

namespace sgdg {

void Stencil::init(int dim) {
  d = dim;
  S = 1;
  for (int a = 0; a < 3; ++a) off[0][a] = 0;
  for (int mask = 1; mask < (1 << d); ++mask) {
    for (int sgn = 1; sgn >= -1; sgn -= 2) {
      for (int a = 0; a < 3; ++a) off[S][a] = (a < d && (mask >> a) & 1) ? sgn : 0;
      ++S;
    }
  }
}

int Stencil::slot(const int* o) const {
  for (int e = 0; e < S; ++e) {
    bool eq = true;
    for (int a = 0; a < d; ++a) eq = eq && off[e][a] == o[a];
    if (eq) return e;
  }
  return -1;
}

int Stencil::neg(int e) const {
  int o[3] = {-off[e][0], -off[e][1], -off[e][2]};
  return slot(o);
}

static inline void unflatten(int64_t p, int d, int m, int* i) {
  for (int a = d - 1; a >= 0; --a) {
    i[a] = int(p % m);
    p /= m;
  }
}

static inline int64_t flatten(const int* i, int d, int m) {
  int64_t p = 0;
  for (int a = 0; a < d; ++a) p = p * m + i[a];
  return p;
}

static inline int wrap(int x, int m) {
  int r = x % m;
  return r < 0 ? r + m : r;
}

void build_domain_tables(DomainData& D) {
  const Dom& dom = D.dom;
  D.st.init(dom.d);
  const int S = D.st.S, d = dom.d;
  D.lev.clear();
  for (int l = D.lmin; l <= D.lmax; ++l) {
    LevelTables T;
    T.level = l;
    T.m = dom.axis_nodes(l);
    T.n = dom.nodes(l);
    T.nbr.assign(T.n * S, 0);
    T.valid.assign(T.n * S, 0);
    const int ncell = 1 << l;
    int i[3], j[3];
    for (int64_t p = 0; p < T.n; ++p) {
      unflatten(p, d, T.m, i);
      for (int e = 0; e < S; ++e) {
        bool ok = true;
        for (int a = 0; a < d; ++a) {
          j[a] = i[a] + D.st.off[e][a];
          if (dom.periodic) j[a] = wrap(j[a], ncell);
          else if (j[a] < 0 || j[a] >= T.m) ok = false;
        }
        T.nbr[p * S + e] = ok ? int32_t(flatten(j, d, T.m)) : int32_t(p);
        T.valid[p * S + e] = ok;
      }
    }
    if (l > D.lmin) {  // parents on level l-1
      const int mc = dom.axis_nodes(l - 1), nc = 1 << (l - 1);
      T.par.assign(T.n * 2, 0);
      T.parw.assign(T.n * 2, 0.0);
      for (int64_t p = 0; p < T.n; ++p) {
        unflatten(p, d, T.m, i);
        bool odd = false;
        for (int a = 0; a < d; ++a) odd = odd || (i[a] & 1);
        int q1[3], q2[3];
        for (int a = 0; a < d; ++a) {
          const int s = i[a] & 1;
          q1[a] = (i[a] - s) / 2;
          q2[a] = (i[a] + s) / 2;
          if (dom.periodic) {
            q1[a] = wrap(q1[a], nc);
            q2[a] = wrap(q2[a], nc);
          }
        }
        T.par[2 * p] = int32_t(flatten(q1, d, mc));
        T.par[2 * p + 1] = int32_t(flatten(q2, d, mc));
        T.parw[2 * p] = odd ? 0.5 : 1.0;
        T.parw[2 * p + 1] = odd ? 0.5 : 0.0;
      }
    }
    if (l < D.lmax) {  // children on level l+1
      const int mf = dom.axis_nodes(l + 1), nf = 1 << (l + 1);
      T.chi.assign(T.n * S, 0);
      T.chiw.assign(T.n * S, 0.0);
      for (int64_t p = 0; p < T.n; ++p) {
        unflatten(p, d, T.m, i);
        for (int e = 0; e < S; ++e) {
          bool ok = true;
          for (int a = 0; a < d; ++a) {
            j[a] = 2 * i[a] + D.st.off[e][a];
            if (dom.periodic) j[a] = wrap(j[a], nf);
            else if (j[a] < 0 || j[a] >= mf) ok = false;
          }
          if (!ok)
            for (int a = 0; a < d; ++a) j[a] = dom.periodic ? wrap(2 * i[a], nf) : 2 * i[a];
          T.chi[p * S + e] = int32_t(flatten(j, d, mf));
          T.chiw[p * S + e] = ok ? (e == 0 ? 1.0 : 0.5) : 0.0;
        }
      }
    }
    D.lev.push_back(std::move(T));
  }
}

bool Weight::operator<(const Weight& o) const {
  if (scale != o.scale) return scale < o.scale;
  if (kink != o.kink) return kink < o.kink;
  return fields < o.fields;
}

bool FactorKey::operator<(const FactorKey& o) const {
  if (kind != o.kind) return kind < o.kind;
  if (a != o.a) return a < o.a;
  if (b != o.b) return b < o.b;
  if (axis != o.axis) return axis < o.axis;
  if (side != o.side) return side < o.side;
  if (trans != o.trans) return trans < o.trans;
  if (w < o.w) return true;
  if (o.w < w) return false;
  return parts < o.parts;
}

bool factor_plain(const DomainData& D, int fid) {
  const FactorKey& k = D.factors[size_t(fid)];
  if (k.parts.empty()) return k.w.fields.empty() && k.w.kink == 0;
  for (const auto& p : k.parts)
    if (!factor_plain(D, p.second)) return false;
  return true;
}

int DomainData::field_id(const double* src, int64_t n) {
  for (size_t i = 0; i < field_src.size(); ++i)
    if (field_src[i] == src) return int(i);
  field_src.push_back(src);
  fields.emplace_back(src, src + n);
  return int(fields.size()) - 1;
}

int DomainData::factor_id(const FactorKey& k) {
  for (size_t i = 0; i < factors.size(); ++i)
    if (!(factors[i] < k) && !(k < factors[i])) return int(i);
  factors.push_back(k);
  return int(factors.size()) - 1;
}

}  // namespace sgdg
