// Host-only diagnostics: dense blocks of the strip operators built from the
// host-assembled factor tables, for checking the assembly on small grids.
// Not used by any device path.
#include <cstring>
#include <vector>

#include "sgdg_internal.h"

using namespace sgdg;

namespace {

using Dense = std::vector<double>;  // row-major

Dense stencil_dense(const DomainData& D, int fid, int l) {
  const LevelTables& T = D.L(l);
  const int S = D.st.S;
  Dense M(size_t(T.n) * T.n, 0.0);
  const auto& v = D.values[fid][l - D.lmin];
  for (int64_t p = 0; p < T.n; ++p)
    for (int e = 0; e < S; ++e)
      if (T.valid[p * S + e]) M[p * T.n + T.nbr[p * S + e]] += v[p * S + e];
  return M;
}

// E_{l <- l-1} dense (n_l x n_{l-1}) from the parent tables
Dense prolong_dense(const DomainData& D, int l) {
  const LevelTables& F = D.L(l);
  const LevelTables& C = D.L(l - 1);
  Dense E(size_t(F.n) * C.n, 0.0);
  for (int64_t p = 0; p < F.n; ++p)
    for (int k = 0; k < 2; ++k) E[p * C.n + F.par[2 * p + k]] += F.parw[2 * p + k];
  return E;
}

Dense matmul(const Dense& A, const Dense& B, int64_t n, int64_t k, int64_t m) {
  Dense C(size_t(n) * m, 0.0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t t = 0; t < k; ++t) {
      const double a = A[i * k + t];
      if (a == 0.0) continue;
      for (int64_t j = 0; j < m; ++j) C[i * m + j] += a * B[t * m + j];
    }
  return C;
}

Dense transpose(const Dense& A, int64_t n, int64_t m) {
  Dense T(size_t(n) * m);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < m; ++j) T[j * n + i] = A[i * m + j];
  return T;
}

// E_{lf <- lc}
Dense chain(const DomainData& D, int lf, int lc) {
  int64_t nc = D.L(lc).n;
  Dense E(size_t(nc) * nc, 0.0);
  for (int64_t i = 0; i < nc; ++i) E[i * nc + i] = 1.0;
  int64_t rows = nc;
  for (int l = lc + 1; l <= lf; ++l) {
    Dense P = prolong_dense(D, l);
    E = matmul(P, E, D.L(l).n, rows, nc);
    rows = D.L(l).n;
  }
  return E;
}

// X_{l,l'} = E_{L,l}^T X_L E_{L,l'} expressed through the coarser of the two levels
Dense coupling(const DomainData& D, int fid, int l, int l2) {
  const int64_t n = D.L(l).n, n2 = D.L(l2).n;
  if (l == l2) return stencil_dense(D, fid, l);
  if (l2 < l) {  // X_l E_{l <- l2}
    Dense X = stencil_dense(D, fid, l);
    return matmul(X, chain(D, l, l2), n, n, n2);
  }
  Dense X = stencil_dense(D, fid, l2);  // E_{l2 <- l}^T X_{l2}
  Dense Et = transpose(chain(D, l2, l), n2, n);
  return matmul(Et, X, n, n2, n2);
}

}  // namespace

extern "C" sgdg_status sgdg_debug_dense_block(const sgdg_domain* x, const sgdg_domain* v, int level_min,
                                              int level_max, int time_degree, const sgdg_problem* p, int kind,
                                              int row_grid, int col_grid, double* out) {
  try {
    if (!x || !v || !p || !out || x->dim != v->dim) throw Error{SGDG_E_ARG, "bad arguments"};
    DomainData X, V;
    for (int side = 0; side < 2; ++side) {
      const sgdg_domain* s = side == 0 ? x : v;
      DomainData& D = side == 0 ? X : V;
      D.dom.d = s->dim;
      D.dom.periodic = s->periodic != 0;
      for (int a = 0; a < 3; ++a) {
        D.dom.lo[a] = s->lo[a];
        D.dom.hi[a] = s->hi[a];
      }
      D.lmin = level_min;
      D.lmax = level_max;
      build_domain_tables(D);
    }
    TermList tl[4];
    build_terms(X, V, *p, time_degree, tl);
    for (int side = 0; side < 2; ++side) {
      DomainData& D = side == 0 ? X : V;
      D.values.assign(D.factors.size(), {});
      for (int f = 0; f < int(D.factors.size()); ++f) assemble_factor(D, f);
    }
    const int idx = kind == SGDG_OP_FULL ? 0 : kind - 1;
    if (kind < 0 || kind > SGDG_OP_DATA_G || kind == SGDG_OP_BLOCKDIAG) throw Error{SGDG_E_ARG, "bad kind"};
    const TermList& L = tl[idx];
    const int S = level_max + level_min;
    const int lx = level_min + row_grid, lv = S - lx, lx2 = level_min + col_grid, lv2 = S - lx2;
    if (lx > level_max || lx2 > level_max || row_grid < 0 || col_grid < 0) throw Error{SGDG_E_ARG, "bad grid"};
    const int64_t nx = X.L(lx).n, nv = V.L(lv).n, nx2 = X.L(lx2).n, nv2 = V.L(lv2).n;
    const int64_t rows = L.Rout * nx * nv, cols = L.Rin * nx2 * nv2;
    std::memset(out, 0, sizeof(double) * rows * cols);
    for (const Term& t : L.terms) {
      Dense Xc = coupling(X, t.xf, lx, lx2);
      Dense Vc = coupling(V, t.vf, lv, lv2);
      for (int s = 0; s < L.Rout; ++s)
        for (int s2 = 0; s2 < L.Rin; ++s2) {
          const double c = t.tm[s * L.Rin + s2];
          if (c == 0.0) continue;
          for (int64_t a = 0; a < nx; ++a)
            for (int64_t a2 = 0; a2 < nx2; ++a2) {
              const double xv = Xc[a * nx2 + a2];
              if (xv == 0.0) continue;
              for (int64_t b = 0; b < nv; ++b)
                for (int64_t b2 = 0; b2 < nv2; ++b2) {
                  const double vv = Vc[b * nv2 + b2];
                  if (vv == 0.0) continue;
                  out[((s * nx + a) * nv + b) * cols + (s2 * nx2 + a2) * nv2 + b2] += c * xv * vv;
                }
            }
        }
    }
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::exception& e) {
    set_error(e.what());
    return SGDG_E_STATE;
  }
  return SGDG_OK;
}
