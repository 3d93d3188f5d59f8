// Internal declarations of libsgdg (host structures, device descriptors, kernel launchers).
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/sgdg.h"

namespace sgdg {

constexpr int kMaxS = 15;       // Kuhn stencil: 1 + 2 (2^d - 1) for d <= 3
constexpr int kMaxR = 3;        // time slices (r <= 2)
constexpr int kMaxGrids = 32;   // component grids in one launch
constexpr int kMaxLevels = 13;  // levels 0..12

// ------------------------------------------------------------------ errors --
void set_error(const std::string& msg);
struct Error {
  sgdg_status code;
  std::string msg;
};
#define SGDG_CHECK_HIP(call)                                                            \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      throw ::sgdg::Error{SGDG_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

// ---------------------------------------------------------------- domains --
struct Dom {
  int d = 1;
  double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
  bool periodic = false;
  int axis_nodes(int l) const { return periodic ? (1 << l) : (1 << l) + 1; }
  int64_t nodes(int l) const {
    int64_t r = 1;
    for (int a = 0; a < d; ++a) r *= axis_nodes(l);
    return r;
  }
  double h(int l, int a) const { return (hi[a] - lo[a]) / double(1 << l); }
};

// Kuhn neighbourhood: offset 0 and +-b for every non-zero 0/1 vector b.
struct Stencil {
  int d = 0, S = 0;
  int off[kMaxS][3] = {};
  void init(int dim);
  int slot(const int* o) const;  // -1 if o is not a stencil offset
  int neg(int e) const;          // slot of -off[e]
};

// Index tables of one level of one domain (host copies).
struct LevelTables {
  int level = 0;
  int m = 0;        // nodes per axis
  int64_t n = 0;    // nodes
  std::vector<int32_t> nbr;   // [n][S] neighbour node index (self if outside a non-periodic box)
  std::vector<uint8_t> valid; // [n][S] 1 if the neighbour exists
  std::vector<int32_t> par;   // [n][2] parents on level-1 (coarse node of the embedding E)
  std::vector<double> parw;   // [n][2] weights (1,0) or (1/2,1/2)
  std::vector<int32_t> chi;   // [n][S] children on level+1
  std::vector<double> chiw;   // [n][S] weights (1 centre, 1/2 edge midpoints, 0 outside)
};

// A weight: scale * prod fields, optionally kinked (1: max(.,0), 2: max(-.,0)).
struct Weight {
  double scale = 1.0;
  std::vector<int> fields;  // indices into the domain's field registry
  int kink = 0;
  bool operator<(const Weight& o) const;
};

enum FactorKind { kMass = 0, kDeriv = 1, kStiff = 2, kFace = 3 };

struct DomainData;

struct FactorKey {
  int kind = kMass;
  int a = -1, b = -1;        // derivative directions
  int axis = -1, side = -1;  // face
  Weight w;
  bool trans = false;
  // a linear combination sum_i c_i F_i of registered factors of one kind
  // (ids ascending, none itself a combination); empty for an assembled factor
  std::vector<std::pair<double, int>> parts;
  bool operator<(const FactorKey& o) const;
};
// true if the factor (every part of a combination) has a constant weight and no kink
bool factor_plain(const DomainData& D, int fid);

struct DomainData {
  Dom dom;
  Stencil st;
  int lmin = 0, lmax = 0;
  std::vector<LevelTables> lev;            // index level - lmin
  std::vector<std::vector<double>> fields; // registry of nodal fields on the finest level
  std::vector<const double*> field_src;    // caller pointers (identity for de-duplication)
  std::vector<FactorKey> factors;          // registry of factors
  std::vector<std::vector<std::vector<double>>> values;  // [factor][level-lmin][n*S]
  // restricted stencils E_{l+1,l}^T X_{l+1}: coarse node P couples to the fine
  // nodes 2P + o, o in woff (sums of two Kuhn offsets); levels lmin..lmax-1
  std::vector<std::array<int, 3>> woff;
  std::vector<std::vector<int32_t>> wide_idx;             // [level-lmin][n*W] fine node index
  std::vector<std::vector<std::vector<double>>> rvalues;  // [factor][level-lmin][n*W]
  // prolongated stencils X_l E_{l<-l-1}: fine node P of level l couples to the
  // coarse nodes floor(P/2) + o, o in {-1,0,1}^d (3^d slots, slot-major per level);
  // levels lmin+1..lmax
  std::vector<std::vector<int32_t>> pro_idx;              // [level-lmin][slot*n + P] coarse node (0 if unused)
  std::vector<std::vector<std::vector<double>>> pvalues;  // [factor][level-lmin][slot*n + P]
  int field_id(const double* src, int64_t n);
  int factor_id(const FactorKey& k);
  const LevelTables& L(int l) const { return lev[l - lmin]; }
};

// One Kronecker term  Tm (x) X (x) V  (Tm: Rout x Rin, row-major).
struct Term {
  double tm[kMaxR * kMaxR] = {};
  int xf = -1, vf = -1;
};

struct TermList {
  int Rin = 1, Rout = 1;
  std::vector<Term> terms;
};

// Host-side construction (mesh.cpp, assembly.cpp, terms.cpp).
void build_domain_tables(DomainData& D);
void assemble_factor(DomainData& D, int fid);  // all levels of one factor
// every factor of D: values, restricted and prolongated stencils (combinations after their parts)
void assemble_all(DomainData& D);
void build_wide_tables(DomainData& D);          // woff and wide_idx
void restrict_factor(DomainData& D, int fid);   // rvalues of one factor
void build_prolong_tables(DomainData& D);       // pro_idx
void prolong_factor(DomainData& D, int fid);    // pvalues of one factor
struct ProblemIn {
  const sgdg_problem* p;
  int d, r;
};
// Builds the operator term lists: 0 FULL, 1 MASS, 2 DATA_F, 3 DATA_G. Registers factors.
void build_terms(DomainData& X, DomainData& V, const sgdg_problem& p, int r, TermList out[4]);
// The same for coefficients given at m time-quadrature points tau (reference
// interval [-1, 1], weights wref summing to 2): at[mu] holds beta and sigma at
// tau[mu]; dt and delta from at[0].
void build_terms_t(DomainData& X, DomainData& V, const sgdg_problem* at, const double* tau, const double* wref, int m,
                   int r, TermList out[4]);
void time_matrices(int r, double dt, double Mt[], double Tt[], double Ct[], double Gt[]);

// ------------------------------------------------------ device descriptors --
struct DevDomain {
  int S = 0, lmin = 0, lmax = 0;
  int64_t lev_off[kMaxLevels] = {};   // start of level l in the [n][S] tables (l - lmin)
  int64_t par_off[kMaxLevels] = {};   // start of level l in the [n][2] parent tables
  int64_t lev_n[kMaxLevels] = {};     // nodes of level l (l - lmin)
  const int32_t* nbr = nullptr;       // [n][S] per level
  const int32_t* tnbr = nullptr;      // the same, slot-major [S][n] per level (coalesced by node)
  const int32_t* par = nullptr;
  const double* parw = nullptr;
  const int32_t* chi = nullptr;
  const double* chiw = nullptr;
  const double* vals = nullptr;       // [factor][level-major [n][S]] FP64
  const float* vals32 = nullptr;      // same, FP32
  const double* tvals = nullptr;      // [factor][level-major [S][n]] FP64 (slot-major)
  const float* tvals32 = nullptr;     // same, FP32
  int64_t fac_stride = 0;             // elements per factor
  int mass_fac = -1;                  // plain mass factor (Jacobi / Chebyshev preconditioner)
  int W = 0;                          // restricted-stencil width
  int64_t wlev_off[kMaxLevels] = {};  // start of level l in the [n][W] tables
  const int32_t* wide = nullptr;      // fine node of each restricted slot
  const double* rvals = nullptr;      // [factor][levels [n][W]] FP64
  const float* rvals32 = nullptr;
  const int32_t* twide = nullptr;     // slot-major copies [W][n] per level (coalesced by node)
  const double* trvals = nullptr;
  const float* trvals32 = nullptr;
  const int32_t* tchi = nullptr;      // slot-major children [S][n] per level
  const double* tchiw = nullptr;
  int PW = 0;                         // prolongated-stencil slots (3^d)
  int64_t plev_off[kMaxLevels] = {};  // start of level l in the [PW][n] tables
  const int32_t* pidx = nullptr;      // coarse node of each slot
  const double* pvals = nullptr;      // [factor][levels [PW][n]] FP64
  const float* pvals32 = nullptr;
  int64_t pstride = 0;                // elements per factor
  int64_t rstride = 0;                // elements per factor
  // slot-pair copies: slots 2p and 2p+1 of a node are adjacent ([S/2][n][2]
  // per level, an odd last slot padded with 0), read with one 2-wide load
  int64_t qlev_off[kMaxLevels] = {};  // start of level l in the pair stencil tables
  const double* qvals = nullptr;      // [factor][levels [S/2][n][2]]
  const float* qvals32 = nullptr;
  int64_t qfac_stride = 0;            // elements per factor
  int64_t qplev_off[kMaxLevels] = {}; // start of level l in the pair prolongated tables
  const double* qpvals = nullptr;     // [factor][levels [PW/2][n][2]]
  const float* qpvals32 = nullptr;
  int64_t qpstride = 0;               // elements per factor
  int64_t qrlev_off[kMaxLevels] = {}; // start of level l in the pair restricted tables
  const double* qrvals = nullptr;     // [factor][levels [W/2][n][2]] (slot pairs of trvals)
  const float* qrvals32 = nullptr;
  int64_t qrstride = 0;               // elements per factor
  // support of each factor matrix per node: bit 0 its row has a nonzero,
  // bit 1 it is the column of a nonzero, bit 2 it is a stencil neighbour of a
  // row with a nonzero; a factor is partial when some node lacks bit 0 or 1
  // (face masses: only the face's nodes)
  int64_t node_off[kMaxLevels] = {};  // first node of level l in the per-node tables
  int64_t node_stride = 0;            // nodes of all levels (per factor)
  const uint8_t* sup = nullptr;       // [factor][nodes]
  const uint8_t* fpartial = nullptr;  // [factor]
};

struct DevGrids {
  int n = 0, R = 1;
  int lx[kMaxGrids] = {}, lv[kMaxGrids] = {};
  int nx[kMaxGrids] = {}, nv[kMaxGrids] = {};
  int64_t off[kMaxGrids + 1] = {};    // start of grid g's [R][nx][nv] block; off[n] = total
};

struct DevOp {
  int Rin = 1, Rout = 1, nterms = 0, nvg = 0, nxg = 0;
  const int* term_xf = nullptr;
  const int* term_vf = nullptr;
  const int* term_vg = nullptr;
  const int* term_xg = nullptr;
  const double* term_tm = nullptr;   // [nterms][Rout][Rin]
  const float* term_tm32 = nullptr;
  const int* vg_fac = nullptr;       // v factor of each V group
  const int* xg_fac = nullptr;       // x factor of each X group
  const int* vg_terms = nullptr;     // term indices ordered by V group
  const int* vg_start = nullptr;     // [nvg + 1]
  const int* xg_terms = nullptr;     // term indices ordered by X group
  const int* xg_start = nullptr;     // [nxg + 1]
  const int* xg_of = nullptr;        // X-group of position kk of xg_terms
  // per x-node (the x-domain's node_off layout), bit m for X-group m < 64:
  // row of the group's factor has a nonzero / read by the x-stencil of such a row
  const uint64_t* xrow_mask = nullptr;
  const uint64_t* xread_mask = nullptr;
  // per x-node, bit m: the upper-partner array Qt^m can be nonzero there
  const uint64_t* xqt_mask = nullptr;
  // per x-node, bit j of V-group j < 64: the lower-partner array Pt^j is read there
  const uint64_t* xpt_mask = nullptr;
};

// Number of device allocations and frees made through DevBuf so far.  A
// captured hipGraph bakes in device addresses; it stays valid only while
// this count is unchanged since its capture.
uint64_t alloc_epoch();

// Device buffer helper.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf();
  void alloc(size_t b);
  void ensure(size_t b);  // grow-only
  template <class T> T* as() const { return static_cast<T*>(p); }
};

}  // namespace sgdg
