// Learned correction of the preconditioner: per-upper-grid convolution
// networks standing in for the combination technique's per-grid map
// r_l -> z_l (Algorithm 1's body), with their own forward, backward and Adam
// kernels.  Convolutions run on the matrix cores (bf16 16x16x32 MFMA, FP32
// accumulation); activations are channels-last bf16 [points][32].
//
// Convolution as an MFMA product: for one tap t the output tile of 32
// channels x 16 points is W_t (32 x 32) times the gathered inputs
// (32 channels x 16 points), i.e. A = W_t rows (out channels) by K = input
// channels, B = 8 consecutive channels of one neighbour point per lane (one
// 16-byte load), and the 9 taps accumulate into the same tile.  Each wave
// keeps its 9 x 2 weight fragments in registers for all its tiles.
#include "ops_internal.h"

#include <chrono>
#include <random>

namespace {

constexpr int NC = 32;
constexpr int NCONV = 8;
constexpr int NTAP = 9;
constexpr int CONV_PARAMS = NTAP * NC * NC + NC;  // weights then bias
constexpr int WFRAG = NTAP * 2 * 64;              // bf16x8 fragments per convolution
constexpr int kConvWaves = 4, kConvThreads = 64 * kConvWaves;  // k_conv block

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct NetGrid {
  int mx, mv;       // nodes per axis of the x- and v-lattices (2D each)
  int64_t poff;     // first point of the grid in the concatenated point order
  int64_t np;       // points mx^2 mv^2 (below 2^24)
  float rmx, rmv, rnv;  // 1/mx, 1/mv, 1/mv^2 (FP32, for qdiv)
};

struct NetGeom {
  int G = 0, R = 1, xper = 0, vper = 0;
  int64_t Ptot = 0, ndof = 0;
  NetGrid g[kMaxGrids];
};

struct ConvItem {
  int s, g;
  int64_t p0;  // first point within the grid
  int np;      // points of the item
};

__device__ __forceinline__ bool nbr_ok(int& n, int m, int per) {
  if (per) {
    if (n < 0) n += m;
    else if (n >= m) n -= m;
    return true;
  }
  return n >= 0 && n < m;
}

// floor(n / m) for 0 <= n < 2^24, m >= 1, rm = 1/m in FP32: the FP32 product is
// within one of the quotient there (relative error below 2^-22 on a quotient
// below 2^23, exact for m = 1), and one correction each way makes it exact.
__device__ __forceinline__ int qdiv(int n, int m, float rm) {
  int q = int(float(n) * rm);
  q -= int(q * m > n);
  q += int((q + 1) * m <= n);
  return q;
}

// Neighbour point of p for tap (a, b) in the x-plane (plane 0) or v-plane (1); -1 outside.
// 32-bit index arithmetic: points of a grid number below 2^24.
__device__ __forceinline__ int neighbour(int p, int a, int b, int plane, const NetGrid& G, int xper, int vper) {
  const int nv = G.mv * G.mv;
  const int xi = qdiv(p, nv, G.rnv);
  const int vi = p - xi * nv;
  if (plane == 0) {
    int x1 = qdiv(xi, G.mx, G.rmx), x2 = xi - x1 * G.mx;
    x1 += a;
    x2 += b;
    if (!nbr_ok(x1, G.mx, xper) || !nbr_ok(x2, G.mx, xper)) return -1;
    return (x1 * G.mx + x2) * nv + vi;
  }
  int v1 = qdiv(vi, G.mv, G.rmv), v2 = vi - v1 * G.mv;
  v1 += a;
  v2 += b;
  if (!nbr_ok(v1, G.mv, vper) || !nbr_ok(v2, G.mv, vper)) return -1;
  return xi * nv + v1 * G.mv + v2;
}

__device__ __forceinline__ bf16x8 zero8() {
  bf16x8 z;
#pragma unroll
  for (int e = 0; e < 8; ++e) z[e] = __bf16(0.0f);
  return z;
}

// out = act(bias + sum_t W_t in[nbr(p, sign * t)]) on a tile of points, one item per block.
// sign = -1 with the transposed fragments computes the adjoint convolution.
// mask (optional): out *= (mask > 0) (the ReLU derivative of the layer below).
template <bool OUT_F32>
__global__ void __launch_bounds__(kConvThreads) k_conv(const ConvItem* __restrict__ items, NetGeom geo,
                                                       const bf16x8* __restrict__ W, int64_t wstride,
                                                       const float* __restrict__ bias, int64_t bstride, int plane,
                                                       int sign, int relu, const __bf16* __restrict__ in,
                                                       void* __restrict__ out, const __bf16* __restrict__ mask) {
  // the item's weight fragments, shared by the block's waves
  __shared__ bf16x8 wl[NTAP * 2 * 64];
  const ConvItem it = items[blockIdx.x];
  const NetGrid G = geo.g[it.g];
  const int lane = int(threadIdx.x) & 63, wave = int(threadIdx.x) >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const bf16x8* Wg = W + int64_t(it.g) * wstride;
  for (int i = int(threadIdx.x); i < NTAP * 2 * 64; i += kConvThreads) wl[i] = Wg[i];
  float bv[2][4];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int j = 0; j < 4; ++j) bv[h][j] = bias ? bias[int64_t(it.g) * bstride + h * 16 + kq * 4 + j] : 0.0f;
  const int64_t base = (int64_t(it.s) * geo.Ptot + G.poff) * NC;
  const int steps = (it.np + 15) / 16;
  // the 9 neighbour fragments of step st; the wave's next step is in flight
  // while the current step's products run
  auto gather = [&](int st, bf16x8 (&f)[NTAP]) {
    const int loc = st * 16 + col;
    const bool valid = loc < it.np;
    const int p = int(it.p0) + loc;
#pragma unroll
    for (int t = 0; t < NTAP; ++t) {
      const int a = (t / 3 - 1) * sign, b = (t % 3 - 1) * sign;
      const int q = valid ? neighbour(p, a, b, plane, G, geo.xper, geo.vper) : -1;
      f[t] = q >= 0 ? *reinterpret_cast<const bf16x8*>(in + base + int64_t(q) * NC + kq * 8) : zero8();
    }
  };
  bf16x8 bn[NTAP];
  if (wave < steps) gather(wave, bn);
  __syncthreads();  // wl complete
  // the block's waves take the item's 16-point steps in turn
  for (int st = wave; st < steps; st += kConvWaves) {
    const int loc = st * 16 + col;
    const bool valid = loc < it.np;
    const int64_t p = it.p0 + loc;
    bf16x8 bo[NTAP];
#pragma unroll
    for (int t = 0; t < NTAP; ++t) bo[t] = bn[t];
    if (st + kConvWaves < steps) gather(st + kConvWaves, bn);
    // weight fragments are read from LDS at each use (not held in registers)
    __asm__ volatile("" ::: "memory");
    f32x4 acc[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) acc[h] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < NTAP; ++t)
#pragma unroll
      for (int h = 0; h < 2; ++h)
        acc[h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wl[(t * 2 + h) * 64 + lane], bo[t], acc[h], 0, 0, 0);
    if (!valid) continue;
    const int64_t o = base + p * NC;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int c0 = h * 16 + kq * 4;
      float v[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        v[j] = acc[h][j] + bv[h][j];
        if (relu) v[j] = fmaxf(v[j], 0.0f);
      }
      if (mask) {
        const bf16x4 m = *reinterpret_cast<const bf16x4*>(mask + o + c0);
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (!(float(m[j]) > 0.0f)) v[j] = 0.0f;
      }
      if (OUT_F32) {
        *reinterpret_cast<f32x4*>(static_cast<float*>(out) + o + c0) = f32x4{v[0], v[1], v[2], v[3]};
      } else {
        bf16x4 w;
#pragma unroll
        for (int j = 0; j < 4; ++j) w[j] = __bf16(v[j]);
        *reinterpret_cast<bf16x4*>(static_cast<__bf16*>(out) + o + c0) = w;
      }
    }
  }
}

// Partial weight and bias gradients of one item:
//   dW[t][co][ci] = sum_p dz[p][co] x[nbr(p, t)][ci],  db[co] = sum_p dz[p][co].
// Chunks of 32 points are staged channel-major in LDS so that each lane reads
// 8 consecutive points of one channel as an MFMA operand (K = points).
constexpr int kLdsRow = 40;  // 32 points + pad (bf16)
__global__ void __launch_bounds__(64) k_wgrad(const ConvItem* __restrict__ items, NetGeom geo, int plane,
                                              const __bf16* __restrict__ x, const __bf16* __restrict__ dz,
                                              float* __restrict__ partial) {
  __shared__ __bf16 xT[NC * kLdsRow];
  __shared__ __bf16 dT[NC * kLdsRow];
  const ConvItem it = items[blockIdx.x];
  const NetGrid G = geo.g[it.g];
  const int lane = threadIdx.x;
  const int col = lane & 15, kq = lane >> 4;
  const int64_t base = (int64_t(it.s) * geo.Ptot + G.poff) * NC;
  f32x4 acc[NTAP][2][2];
#pragma unroll
  for (int t = 0; t < NTAP; ++t)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[t][a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  float db = 0.0f;
  const int chunks = (it.np + 31) / 32;
  for (int ch = 0; ch < chunks; ++ch) {
    // stage dz: 32 points x 32 channels, two 16-byte loads per lane
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int idx = r * 64 + lane, pt = idx >> 2, q4 = idx & 3;
      const int loc = ch * 32 + pt;
      bf16x8 v = zero8();
      if (loc < it.np) v = *reinterpret_cast<const bf16x8*>(dz + base + (it.p0 + loc) * NC + q4 * 8);
#pragma unroll
      for (int e = 0; e < 8; ++e) dT[(q4 * 8 + e) * kLdsRow + pt] = v[e];
    }
    __syncthreads();
    if (lane < NC) {
#pragma unroll 8
      for (int pt = 0; pt < 32; ++pt) db += float(dT[lane * kLdsRow + pt]);
    }
    bf16x8 bop[2];
#pragma unroll
    for (int hn = 0; hn < 2; ++hn) bop[hn] = *reinterpret_cast<const bf16x8*>(&dT[(hn * 16 + col) * kLdsRow + kq * 8]);
#pragma unroll
    for (int t = 0; t < NTAP; ++t) {
      const int a = t / 3 - 1, b = t % 3 - 1;
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const int idx = r * 64 + lane, pt = idx >> 2, q4 = idx & 3;
        const int loc = ch * 32 + pt;
        bf16x8 v = zero8();
        if (loc < it.np) {
          const int q = neighbour(int(it.p0) + loc, a, b, plane, G, geo.xper, geo.vper);
          if (q >= 0) v = *reinterpret_cast<const bf16x8*>(x + base + int64_t(q) * NC + q4 * 8);
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) xT[(q4 * 8 + e) * kLdsRow + pt] = v[e];
      }
      __syncthreads();
      bf16x8 aop[2];
#pragma unroll
      for (int hm = 0; hm < 2; ++hm)
        aop[hm] = *reinterpret_cast<const bf16x8*>(&xT[(hm * 16 + col) * kLdsRow + kq * 8]);
#pragma unroll
      for (int hm = 0; hm < 2; ++hm)
#pragma unroll
        for (int hn = 0; hn < 2; ++hn)
          acc[t][hm][hn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop[hm], bop[hn], acc[t][hm][hn], 0, 0, 0);
      __syncthreads();
    }
  }
  // C[ci][co]: lane holds ci = hm*16 + kq*4 + j, co = hn*16 + col
  float* out = partial + int64_t(blockIdx.x) * CONV_PARAMS;
#pragma unroll
  for (int t = 0; t < NTAP; ++t)
#pragma unroll
    for (int hm = 0; hm < 2; ++hm)
#pragma unroll
      for (int hn = 0; hn < 2; ++hn)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int ci = hm * 16 + kq * 4 + j, co = hn * 16 + col;
          out[(t * NC + co) * NC + ci] = acc[t][hm][hn][j];
        }
  if (lane < NC) out[NTAP * NC * NC + lane] = db;
}

// grad[g][j] = sum of the partials of grid g's items (contiguous, fixed order)
__global__ void k_wreduce(int G, const int* __restrict__ istart, const int* __restrict__ icount,
                          const float* __restrict__ partial, float* __restrict__ grad, int64_t gstride) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(G) * CONV_PARAMS) return;
  const int g = int(t / CONV_PARAMS), j = int(t - int64_t(g) * CONV_PARAMS);
  float a = 0.0f;
  for (int i = 0; i < icount[g]; ++i) a += partial[int64_t(istart[g] + i) * CONV_PARAMS + j];
  grad[int64_t(g) * gstride + j] = a;
}

__global__ void k_adam(int64_t n, float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float c1, float c2) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

// bf16 MFMA fragments of every convolution: forward (A = W_t[co][ci]) and
// adjoint (A = W_t^T[ci][co]); lane l of half h holds row h*16 + l%16, K = (l/16)*8 + e.
__global__ void k_pack(int64_t nconv, const float* __restrict__ th, bf16x8* __restrict__ wf,
                       bf16x8* __restrict__ wt) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;  // fragment index
  if (i >= nconv * WFRAG) return;
  const int64_t c = i / WFRAG;
  const int f = int(i - c * WFRAG);
  const int t = f / 128, h = (f / 64) & 1, l = f & 63;
  const float* W = th + c * CONV_PARAMS + int64_t(t) * NC * NC;
  const int row = h * 16 + (l & 15), k0 = (l >> 4) * 8;
  bf16x8 a, b;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    a[e] = __bf16(W[row * NC + k0 + e]);      // W[co=row][ci=k]
    b[e] = __bf16(W[(k0 + e) * NC + row]);    // W[co=k][ci=row]
  }
  wf[i] = a;
  wt[i] = b;
}

// point index -> grid (G <= 32)
__device__ __forceinline__ int grid_of(const NetGeom& geo, int64_t p) {
  int g = 0;
  while (g + 1 < geo.G && p >= geo.g[g + 1].poff) ++g;
  return g;
}

// x[s][p][c] = r_s[grid block][c][p_local] * inv[s][g] (c < R), 0 otherwise; bf16
template <class T>
__global__ void k_pack_in(NetGeom geo, int S, const T* __restrict__ r, int64_t rstride,
                          const float* __restrict__ inv, __bf16* __restrict__ x) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(S) * geo.Ptot) return;
  const int s = int(i / geo.Ptot);
  const int64_t p = i - int64_t(s) * geo.Ptot;
  const int g = grid_of(geo, p);
  const int64_t pl = p - geo.g[g].poff;
  const float sc = inv ? inv[s * geo.G + g] : 1.0f;
  bf16x8 out[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) out[q] = zero8();
  for (int c = 0; c < geo.R; ++c)
    out[0][c] = __bf16(float(r[int64_t(s) * rstride + geo.R * geo.g[g].poff + c * geo.g[g].np + pl]) * sc);
  bf16x8* dst = reinterpret_cast<bf16x8*>(x + i * NC);
#pragma unroll
  for (int q = 0; q < 4; ++q) dst[q] = out[q];
}

// z[grid block][c][p_local] = fac[g] * y[p][c] (c < R)
template <class T>
__global__ void k_unpack(NetGeom geo, const float* __restrict__ y, const float* __restrict__ fac, T* __restrict__ z) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= geo.Ptot) return;
  const int g = grid_of(geo, p);
  const int64_t pl = p - geo.g[g].poff;
  const float f = fac ? fac[g] : 1.0f;
  for (int c = 0; c < geo.R; ++c) z[geo.R * geo.g[g].poff + c * geo.g[g].np + pl] = T(f * y[p * NC + c]);
}

// raw tensors [p][R] <-> [p][32]
// one point per thread: R channels, zero padding, four 16-byte stores (R <= 8)
__global__ void k_raw_in(int64_t P, int R, const float* __restrict__ x, __bf16* __restrict__ h) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= P) return;
  bf16x8 out[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) out[q] = zero8();
  for (int c = 0; c < R; ++c) out[0][c] = __bf16(x[p * R + c]);
  bf16x8* dst = reinterpret_cast<bf16x8*>(h + p * NC);
#pragma unroll
  for (int q = 0; q < 4; ++q) dst[q] = out[q];
}
__global__ void k_raw_out(int64_t P, int R, const float* __restrict__ y, float* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= P * R) return;
  const int64_t p = i / R;
  out[i] = y[p * NC + (i - p * R)];
}

// Mean-squared-error gradient of the normalised outputs:
//   t = z_s[block][c][p] * tfac[s][g],  dy = 2 (y - t) / (S P_g R)  (c < R; 0 otherwise)
__global__ void __launch_bounds__(256) k_loss(NetGeom geo, int S, const float* __restrict__ y,
                                              const float* __restrict__ z, int64_t zstride,
                                              const float* __restrict__ tfac, __bf16* __restrict__ dy,
                                              double* __restrict__ partial) {
  __shared__ double sh[4];
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  double l = 0.0;
  if (i < int64_t(S) * geo.Ptot) {
    const int s = int(i / geo.Ptot);
    const int64_t p = i - int64_t(s) * geo.Ptot;
    const int g = grid_of(geo, p);
    const int64_t pl = p - geo.g[g].poff;
    const float w = 1.0f / (float(S) * float(geo.g[g].np) * float(geo.R));
    bf16x8 out[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) out[q] = zero8();
    for (int c = 0; c < geo.R; ++c) {
      const float t = z[int64_t(s) * zstride + geo.R * geo.g[g].poff + c * geo.g[g].np + pl] * tfac[s * geo.G + g];
      const float d = y[i * NC + c] - t;
      l += double(d) * d * w;
      out[0][c] = __bf16(2.0f * d * w);
    }
    bf16x8* dst = reinterpret_cast<bf16x8*>(dy + i * NC);
#pragma unroll
    for (int q = 0; q < 4; ++q) dst[q] = out[q];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) l += __shfl_down(l, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = l;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// per-segment sums of squares -> rms (and its inverse), segments of equal role
__global__ void k_seg_rms(int nseg, const SegInfo* __restrict__ segs, const double* __restrict__ partial,
                          float* __restrict__ rms, float* __restrict__ inv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nseg) return;
  double a = 0;
  for (int c = 0; c < segs[i].nchunk; ++c) a += partial[segs[i].chunk0 + c];
  const double r = sqrt(a / double(segs[i].len));
  rms[i] = float(r);
  inv[i] = r > 0 ? float(1.0 / r) : 0.0f;
}

// samples_s = sum_k coef[s][k] base_k (elementwise), S <= 32
__global__ void k_mix(int64_t n, int K, int S, const float* __restrict__ coef, const float* __restrict__ base,
                      float* __restrict__ out) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= n) return;
  float acc[32];
  for (int s = 0; s < S; ++s) acc[s] = 0.0f;
  for (int k = 0; k < K; ++k) {
    const float b = base[int64_t(k) * n + e];
    for (int s = 0; s < S; ++s) acc[s] += coef[s * K + k] * b;
  }
  for (int s = 0; s < S; ++s) out[int64_t(s) * n + e] = acc[s];
}

// fac[i] = a[i] * b[i % G]  or  a[i] / b[i % G]
__global__ void k_fac(int n, int G, const float* __restrict__ a, const float* __restrict__ b, int divide,
                      float* __restrict__ fac) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float bg = b[i % G];
  fac[i] = divide ? (bg > 0.0f ? a[i] / bg : 0.0f) : a[i] * bg;
}

__global__ void k_d2f_off(int64_t n, const double* __restrict__ x, float* __restrict__ y) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = float(x[i]);
}

inline unsigned nb(int64_t n, int b = 256) { return unsigned((n + b - 1) / b); }
#define NET_CHECK() SGDG_CHECK_HIP(hipGetLastError())

}  // namespace

// ------------------------------------------------------------------ host ---
struct sgdg_net_s {
  sgdg_ops o = nullptr;
  NetGeom geo;
  int64_t nparams = 0;
  DevBuf theta, m, v, grad, wf, wt;
  std::vector<double> scales;
  DevBuf scales_f;  // per grid FP32
  int64_t adam_step = 0;
  // training pairs (FP32 [K][ndof])
  DevBuf pr, pz;
  int npairs = 0, capacity = 0, record_cap = 0;
  // work
  struct Tab {
    DevBuf items, istart, icount;
    int n = 0;
    std::vector<int> hstart, hcount;
  };
  std::map<std::pair<int, int>, std::unique_ptr<Tab>> tabs;  // (S, points per item)
  DevBuf act, Y, D0, D1, partial, lossp;
  DevBuf seg_segs, seg_blk, seg_part, rms, inv, tfac, samp_r, samp_z, coef;
  int seg_S = -1;
  SegTable segt;
};

namespace {

using Net = sgdg_net_s;

Net::Tab& conv_tab(Net& N, int S, int per) {
  auto key = std::make_pair(S, per);
  auto f = N.tabs.find(key);
  if (f != N.tabs.end()) return *f->second;
  auto T = std::make_unique<Net::Tab>();
  std::vector<ConvItem> its;
  // grid-major, then sample, then chunk: the items of one grid are contiguous
  for (int g = 0; g < N.geo.G; ++g) {
    T->hstart.push_back(int(its.size()));
    for (int s = 0; s < S; ++s)
      for (int64_t p0 = 0; p0 < N.geo.g[g].np; p0 += per)
        its.push_back(ConvItem{s, g, p0, int(std::min<int64_t>(per, N.geo.g[g].np - p0))});
    T->hcount.push_back(int(its.size()) - T->hstart.back());
  }
  upload(T->items, its);
  upload(T->istart, T->hstart);
  upload(T->icount, T->hcount);
  T->n = int(its.size());
  Net::Tab& r = *T;
  N.tabs[key] = std::move(T);
  return r;
}

// points per item: enough items to fill the chip, at least 64 points
// (one input: 1024 items measured fastest, 0.184 ms for the 218 197-point
// forward against 0.202 ms at 2048 and 0.235 ms at 512 items)
constexpr int kInferItems = 1024;
int per_item(const Net& N, int S, int target_items) {
  int64_t per = (int64_t(S) * N.geo.Ptot) / std::max(1, target_items);
  per = std::max<int64_t>(64, std::min<int64_t>(1024, (per + 15) / 16 * 16));
  return int(per);
}

const bf16x8* wfrag(const Net& N, const DevBuf& b, int c) {
  return ptr<bf16x8>(b) + int64_t(c) * WFRAG;
}

void conv(Net& N, const Net::Tab& T, int c, bool transposed, int relu, const __bf16* in, void* out, bool out_f32,
          const __bf16* mask, hipStream_t s) {
  const int plane = c & 1;
  const bf16x8* W = wfrag(N, transposed ? N.wt : N.wf, c);
  const int64_t wstride = int64_t(NCONV) * WFRAG;
  const float* bias = transposed ? nullptr : ptr<float>(N.theta) + int64_t(c) * CONV_PARAMS + NTAP * NC * NC;
  const int64_t bstride = int64_t(NCONV) * CONV_PARAMS;
  const int sign = transposed ? -1 : 1;
  if (out_f32)
    hipLaunchKernelGGL(k_conv<true>, dim3(T.n), dim3(kConvThreads), 0, s, ptr<ConvItem>(T.items), N.geo, W, wstride, bias,
                       bstride, plane, sign, relu, in, out, mask);
  else
    hipLaunchKernelGGL(k_conv<false>, dim3(T.n), dim3(kConvThreads), 0, s, ptr<ConvItem>(T.items), N.geo, W, wstride, bias,
                       bstride, plane, sign, relu, in, out, mask);
  NET_CHECK();
}

void wgrad(Net& N, const Net::Tab& T, int c, const __bf16* x, const __bf16* dz, hipStream_t s) {
  N.partial.ensure(sizeof(float) * size_t(T.n) * CONV_PARAMS);
  hipLaunchKernelGGL(k_wgrad, dim3(T.n), dim3(64), 0, s, ptr<ConvItem>(T.items), N.geo, c & 1, x, dz,
                     ptr<float>(N.partial));
  NET_CHECK();
  const int64_t tot = int64_t(N.geo.G) * CONV_PARAMS;
  hipLaunchKernelGGL(k_wreduce, dim3(nb(tot)), dim3(256), 0, s, N.geo.G, ptr<int>(T.istart), ptr<int>(T.icount),
                     ptr<float>(N.partial), ptr<float>(N.grad) + int64_t(c) * CONV_PARAMS,
                     int64_t(NCONV) * CONV_PARAMS);
  NET_CHECK();
}

size_t act_elems(const Net& N, int S) { return size_t(S) * N.geo.Ptot * NC; }
__bf16* actbuf(Net& N, int S, int i) { return ptr<__bf16>(N.act) + act_elems(N, S) * i; }

// forward of S packed inputs (act slot 0); saves h_k in slots 2k, t_k in 2k+1; output Y (FP32)
void forward(Net& N, const Net::Tab& T, int S, hipStream_t s) {
  N.Y.ensure(sizeof(float) * act_elems(N, S));
  for (int k = 0; k < 4; ++k) {
    conv(N, T, 2 * k, false, 0, actbuf(N, S, 2 * k), actbuf(N, S, 2 * k + 1), false, nullptr, s);
    if (k < 3) conv(N, T, 2 * k + 1, false, 1, actbuf(N, S, 2 * k + 1), actbuf(N, S, 2 * k + 2), false, nullptr, s);
    else conv(N, T, 2 * k + 1, false, 0, actbuf(N, S, 2 * k + 1), ptr<float>(N.Y), true, nullptr, s);
  }
}

// backward from dY (bf16 in D0): all parameter gradients into N.grad
void backward(Net& N, const Net::Tab& T, int S, hipStream_t s) {
  __bf16* D0 = ptr<__bf16>(N.D0);
  __bf16* D1 = ptr<__bf16>(N.D1);
  for (int k = 3; k >= 0; --k) {
    // D0 = dL/dz of the v-conv of layer k (masked)
    wgrad(N, T, 2 * k + 1, actbuf(N, S, 2 * k + 1), D0, s);
    conv(N, T, 2 * k + 1, true, 0, D0, D1, false, nullptr, s);
    wgrad(N, T, 2 * k, actbuf(N, S, 2 * k), D1, s);
    if (k > 0) conv(N, T, 2 * k, true, 0, D1, D0, false, actbuf(N, S, 2 * k), s);
  }
}

void ensure_act(Net& N, int S) {
  N.act.ensure(sizeof(__bf16) * act_elems(N, S) * 8);
  N.D0.ensure(sizeof(__bf16) * act_elems(N, S));
  N.D1.ensure(sizeof(__bf16) * act_elems(N, S));
}

void pack_weights(Net& N, hipStream_t s) {
  const int64_t nconv = int64_t(N.geo.G) * NCONV;
  hipLaunchKernelGGL(k_pack, dim3(nb(nconv * WFRAG)), dim3(256), 0, s, nconv, ptr<float>(N.theta),
                     ptr<bf16x8>(N.wf), ptr<bf16x8>(N.wt));
  NET_CHECK();
}

// segment table over (sample, grid) blocks of [S][ndof] vectors
void seg_table(Net& N, int S) {
  if (N.seg_S == S) return;
  std::vector<SegInfo> segs;
  std::vector<BlockRef> blk;
  int chunk = 0;
  for (int sa = 0; sa < S; ++sa)
    for (int g = 0; g < N.geo.G; ++g) {
      SegInfo I{};
      I.kind = 2;
      I.off = int64_t(sa) * N.geo.ndof + int64_t(N.geo.R) * N.geo.g[g].poff;
      I.len = int64_t(N.geo.R) * N.geo.g[g].np;
      I.low_off = -1;
      I.chunk0 = chunk;
      I.nchunk = int(std::max<int64_t>(1, (I.len + kChunk - 1) / kChunk));
      for (int c = 0; c < I.nchunk; ++c) blk.push_back(BlockRef{int(segs.size()), c});
      chunk += I.nchunk;
      segs.push_back(I);
    }
  N.segt.segs = upload(N.seg_segs, segs);
  N.segt.blk = upload(N.seg_blk, blk);
  N.segt.nseg = int(segs.size());
  N.segt.nblk = int(blk.size());
  N.segt.nchunks = chunk;
  N.seg_part.ensure(sizeof(double) * chunk);
  N.rms.ensure(sizeof(float) * segs.size());
  N.inv.ensure(sizeof(float) * segs.size());
  N.seg_S = S;
}

template <class T>
void seg_rms(Net& N, int S, const T* v, hipStream_t s) {
  seg_table(N, S);
  KernelsT<T>::seg_norm2(N.segt, v, ptr<double>(N.seg_part), s);
  hipLaunchKernelGGL(k_seg_rms, dim3(nb(N.segt.nseg)), dim3(256), 0, s, N.segt.nseg, N.segt.segs,
                     ptr<double>(N.seg_part), ptr<float>(N.rms), ptr<float>(N.inv));
  NET_CHECK();
}

void upload_scales(Net& N) {
  std::vector<float> f(N.scales.begin(), N.scales.end());
  upload(N.scales_f, f);
}

}  // namespace

// learned preconditioner as seen by the strip solver
void net_apply_dev(sgdg_net n, const double* r, double* z, hipStream_t s) {
  Net& N = *n;
  const int S = 1;
  const Net::Tab& T = conv_tab(N, S, per_item(N, S, kInferItems));
  ensure_act(N, S);
  seg_rms<double>(N, S, r, s);
  hipLaunchKernelGGL(k_pack_in<double>, dim3(nb(N.geo.Ptot)), dim3(256), 0, s, N.geo, S, r, N.geo.ndof,
                     ptr<float>(N.inv), actbuf(N, S, 0));
  NET_CHECK();
  forward(N, T, S, s);
  // z = s_g * rms_g * y
  N.tfac.ensure(sizeof(float) * N.geo.G);
  hipLaunchKernelGGL(k_fac, dim3(1), dim3(64), 0, s, N.geo.G, N.geo.G, ptr<float>(N.rms), ptr<float>(N.scales_f),
                     0, ptr<float>(N.tfac));
  NET_CHECK();
  hipLaunchKernelGGL(k_unpack<double>, dim3(nb(N.geo.Ptot)), dim3(256), 0, s, N.geo, ptr<float>(N.Y),
                     ptr<float>(N.tfac), z);
  NET_CHECK();
}

sgdg_ops net_problem(sgdg_net n) { return n->o; }

void net_detach(sgdg_net n) { n->o = nullptr; }

static Net& live(sgdg_net n) {
  require(n != nullptr, "null net");
  require(n->o != nullptr, "the network's problem has been destroyed");
  return *n;
}

void net_record_pair(sgdg_net n, const double* r, const double* z, hipStream_t s) {
  Net& N = *n;
  if (N.npairs >= N.record_cap || N.npairs >= N.capacity) return;
  const int64_t nd = N.geo.ndof;
  hipLaunchKernelGGL(k_d2f_off, dim3(nb(nd)), dim3(256), 0, s, nd, r, ptr<float>(N.pr) + int64_t(N.npairs) * nd);
  NET_CHECK();
  hipLaunchKernelGGL(k_d2f_off, dim3(nb(nd)), dim3(256), 0, s, nd, z, ptr<float>(N.pz) + int64_t(N.npairs) * nd);
  NET_CHECK();
  ++N.npairs;
}

// ================================================================== ABI ===
extern "C" sgdg_status sgdg_net_create(sgdg_ops o, uint64_t seed, sgdg_net* out) {
  API_BEGIN
  require(o && out, "null argument");
  require(o->X.dom.d == 2, "the learned preconditioner is defined for d = 2 (4D phase space)");
  sgdg_grid g = o->grid;
  require(int(g->up.size()) <= kMaxGrids, "too many component grids");
  auto N = std::make_unique<Net>();
  N->o = o;
  NetGeom& geo = N->geo;
  geo.G = int(g->up.size());
  geo.R = g->R;
  geo.xper = g->x.periodic;
  geo.vper = g->v.periodic;
  int64_t po = 0;
  for (int i = 0; i < geo.G; ++i) {
    NetGrid& G = geo.g[i];
    G.mx = g->x.axis_nodes(g->up[i].lx);
    G.mv = g->v.axis_nodes(g->up[i].lv);
    G.np = int64_t(G.mx) * G.mx * G.mv * G.mv;
    require(G.np == g->up[i].nx * g->up[i].nv, "grid lattice mismatch");
    require(G.np < (int64_t(1) << 24), "a component grid of the learned preconditioner exceeds 2^24 points");
    G.rmx = 1.0f / float(G.mx);
    G.rmv = 1.0f / float(G.mv);
    G.rnv = 1.0f / float(int64_t(G.mv) * G.mv);
    G.poff = po;
    po += G.np;
  }
  geo.Ptot = po;
  geo.ndof = po * geo.R;
  N->nparams = int64_t(geo.G) * NCONV * CONV_PARAMS;
  // weights: scaled normal draws, zero biases and padding channels
  std::vector<float> th(N->nparams, 0.0f);
  for (int gi = 0; gi < geo.G; ++gi) {
    std::mt19937_64 rng(seed * 1000003ULL + uint64_t(gi));
    std::normal_distribution<double> nd(0.0, 1.0);
    for (int c = 0; c < NCONV; ++c) {
      float* W = th.data() + (int64_t(gi) * NCONV + c) * CONV_PARAMS;
      const int cin = c == 0 ? geo.R : NC, cout = c == NCONV - 1 ? geo.R : NC;
      const double sd = (c & 1) ? std::sqrt(2.0 / (9.0 * cin)) : std::sqrt(1.0 / (9.0 * cin));
      for (int t = 0; t < NTAP; ++t)
        for (int co = 0; co < NC; ++co)
          for (int ci = 0; ci < NC; ++ci) {
            const double r = nd(rng);
            if (co < cout && ci < cin) W[(t * NC + co) * NC + ci] = float(sd * r);
          }
    }
  }
  upload(N->theta, th);
  std::vector<float> zero(N->nparams, 0.0f);
  upload(N->m, zero);
  upload(N->v, zero);
  upload(N->grad, zero);
  N->wf.alloc(sizeof(bf16x8) * size_t(geo.G) * NCONV * WFRAG);
  N->wt.alloc(sizeof(bf16x8) * size_t(geo.G) * NCONV * WFRAG);
  N->scales.assign(geo.G, 1.0);
  upload_scales(*N);
  pack_weights(*N, nullptr);
  SGDG_CHECK_HIP(hipDeviceSynchronize());
  o->nets.push_back(N.get());
  *out = N.release();
  API_END
}

extern "C" sgdg_status sgdg_net_shape(sgdg_net n, int64_t* n_params, int* n_grids) {
  API_BEGIN
  require(n != nullptr, "null net");
  if (n_params) *n_params = n->nparams;
  if (n_grids) *n_grids = n->geo.G;
  API_END
}

extern "C" sgdg_status sgdg_net_get_params(sgdg_net n, float* params, double* scales) {
  API_BEGIN
  require(n != nullptr, "null net");
  SGDG_CHECK_HIP(hipDeviceSynchronize());
  if (params) SGDG_CHECK_HIP(hipMemcpy(params, n->theta.p, sizeof(float) * n->nparams, hipMemcpyDeviceToHost));
  if (scales) std::copy(n->scales.begin(), n->scales.end(), scales);
  API_END
}

extern "C" sgdg_status sgdg_net_set_params(sgdg_net n, const float* params, const double* scales) {
  API_BEGIN
  require(n != nullptr, "null net");
  SGDG_CHECK_HIP(hipDeviceSynchronize());
  if (params) {
    SGDG_CHECK_HIP(hipMemcpy(n->theta.p, params, sizeof(float) * n->nparams, hipMemcpyHostToDevice));
    pack_weights(*n, nullptr);
  }
  if (scales) {
    n->scales.assign(scales, scales + n->geo.G);
    upload_scales(*n);
  }
  SGDG_CHECK_HIP(hipDeviceSynchronize());
  API_END
}

static void ensure_pairs(Net& N, int cap) {
  if (cap <= N.capacity) return;
  // grow keeping the stored pairs
  const size_t bytes = sizeof(float) * size_t(cap) * N.geo.ndof;
  DevBuf nr, nz;
  nr.alloc(bytes);
  nz.alloc(bytes);
  if (N.npairs > 0) {
    const size_t used = sizeof(float) * size_t(N.npairs) * N.geo.ndof;
    SGDG_CHECK_HIP(hipDeviceSynchronize());
    SGDG_CHECK_HIP(hipMemcpy(nr.p, N.pr.p, used, hipMemcpyDeviceToDevice));
    SGDG_CHECK_HIP(hipMemcpy(nz.p, N.pz.p, used, hipMemcpyDeviceToDevice));
  }
  std::swap(N.pr.p, nr.p);
  std::swap(N.pr.bytes, nr.bytes);
  std::swap(N.pz.p, nz.p);
  std::swap(N.pz.bytes, nz.bytes);
  N.capacity = cap;
}

extern "C" sgdg_status sgdg_net_add_pairs(sgdg_net n, const double* r_dev, const double* z_dev, int count,
                                          hipStream_t s) {
  API_BEGIN
  live(n);
  require(r_dev && z_dev && count >= 0, "bad arguments");
  require(count <= 1 << 20, "too many pairs");
  ensure_pairs(*n, n->npairs + count);
  const int64_t nd = n->geo.ndof;
  for (int k = 0; k < count; ++k) {
    hipLaunchKernelGGL(k_d2f_off, dim3(nb(nd)), dim3(256), 0, s, nd, r_dev + int64_t(k) * nd,
                       ptr<float>(n->pr) + int64_t(n->npairs) * nd);
    NET_CHECK();
    hipLaunchKernelGGL(k_d2f_off, dim3(nb(nd)), dim3(256), 0, s, nd, z_dev + int64_t(k) * nd,
                       ptr<float>(n->pz) + int64_t(n->npairs) * nd);
    NET_CHECK();
    ++n->npairs;
  }
  API_END
}

extern "C" sgdg_status sgdg_net_record(sgdg_net n, int capacity) {
  API_BEGIN
  live(n);
  require(capacity >= 0 && capacity <= 1 << 20, "bad arguments");
  if (capacity > 0) {
    ensure_pairs(*n, capacity);
    n->record_cap = capacity;
    n->o->recorder = n;
  } else {
    n->record_cap = 0;
    if (n->o->recorder == n) n->o->recorder = nullptr;
  }
  API_END
}

extern "C" sgdg_status sgdg_net_pair_count(sgdg_net n, int* count) {
  API_BEGIN
  require(n && count, "null argument");
  *count = n->npairs;
  API_END
}

extern "C" sgdg_status sgdg_net_train(sgdg_net n, const sgdg_train_opts* to, sgdg_train_stats* st, hipStream_t s) {
  API_BEGIN
  live(n);
  require(to != nullptr, "null argument");
  require(to->steps >= 0 && to->batch >= 1 && to->batch <= 32 && to->lr > 0, "bad training options");
  require(n->npairs >= 1, "no training pairs stored");
  Net& N = *n;
  const auto t0 = std::chrono::steady_clock::now();
  const int K = N.npairs, G = N.geo.G, S = to->batch;
  const int64_t nd = N.geo.ndof;
  // output scales from the stored pairs: mean over pairs of rms(z_l) / rms(r_l)
  {
    std::vector<float> rr(size_t(K) * G), rz(size_t(K) * G);
    seg_rms<float>(N, K, ptr<float>(N.pr), s);
    SGDG_CHECK_HIP(hipMemcpyAsync(rr.data(), N.rms.p, sizeof(float) * rr.size(), hipMemcpyDeviceToHost, s));
    SGDG_CHECK_HIP(hipStreamSynchronize(s));
    seg_rms<float>(N, K, ptr<float>(N.pz), s);
    SGDG_CHECK_HIP(hipMemcpyAsync(rz.data(), N.rms.p, sizeof(float) * rz.size(), hipMemcpyDeviceToHost, s));
    SGDG_CHECK_HIP(hipStreamSynchronize(s));
    for (int g = 0; g < G; ++g) {
      double a = 0;
      int c = 0;
      for (int k = 0; k < K; ++k)
        if (rr[size_t(k) * G + g] > 0) {
          a += double(rz[size_t(k) * G + g]) / rr[size_t(k) * G + g];
          ++c;
        }
      N.scales[g] = c > 0 && a > 0 ? a / c : 1.0;
    }
    upload_scales(N);
  }
  const Net::Tab& T = conv_tab(N, S, per_item(N, S, 4096));
  ensure_act(N, S);
  N.samp_r.ensure(sizeof(float) * size_t(S) * nd);
  N.samp_z.ensure(sizeof(float) * size_t(S) * nd);
  N.tfac.ensure(sizeof(float) * size_t(S) * G);
  const int64_t nl = int64_t(S) * N.geo.Ptot;
  N.lossp.ensure(sizeof(double) * nb(nl));
  std::vector<double> lp(nb(nl));
  std::mt19937_64 rng(to->seed);
  std::normal_distribution<double> nd01(0.0, 1.0);
  std::vector<float> coef(size_t(S) * K);
  std::vector<double> losses;
  for (int step = 0; step < to->steps; ++step) {
    for (int sa = 0; sa < S; ++sa)
      for (int k = 0; k < K; ++k) {
        if (to->mix) coef[size_t(sa) * K + k] = float(nd01(rng) / std::sqrt(double(K)));
        else coef[size_t(sa) * K + k] = (int64_t(step) * S + sa) % K == k ? 1.0f : 0.0f;
      }
    SGDG_CHECK_HIP(hipStreamSynchronize(s));  // the previous step's coefficients are no longer read
    upload(N.coef, coef);
    hipLaunchKernelGGL(k_mix, dim3(nb(nd)), dim3(256), 0, s, nd, K, S, ptr<float>(N.coef), ptr<float>(N.pr),
                       ptr<float>(N.samp_r));
    NET_CHECK();
    hipLaunchKernelGGL(k_mix, dim3(nb(nd)), dim3(256), 0, s, nd, K, S, ptr<float>(N.coef), ptr<float>(N.pz),
                       ptr<float>(N.samp_z));
    NET_CHECK();
    seg_rms<float>(N, S, ptr<float>(N.samp_r), s);
    hipLaunchKernelGGL(k_fac, dim3(nb(S * G)), dim3(256), 0, s, S * G, G, ptr<float>(N.inv), ptr<float>(N.scales_f),
                       1, ptr<float>(N.tfac));
    NET_CHECK();
    hipLaunchKernelGGL(k_pack_in<float>, dim3(nb(nl)), dim3(256), 0, s, N.geo, S, ptr<float>(N.samp_r), nd,
                       ptr<float>(N.inv), actbuf(N, S, 0));
    NET_CHECK();
    forward(N, T, S, s);
    hipLaunchKernelGGL(k_loss, dim3(nb(nl)), dim3(256), 0, s, N.geo, S, ptr<float>(N.Y), ptr<float>(N.samp_z), nd,
                       ptr<float>(N.tfac), ptr<__bf16>(N.D0), ptr<double>(N.lossp));
    NET_CHECK();
    backward(N, T, S, s);
    ++N.adam_step;
    const float c1 = float(1.0 - std::pow(0.9, double(N.adam_step)));
    const float c2 = float(1.0 - std::pow(0.999, double(N.adam_step)));
    hipLaunchKernelGGL(k_adam, dim3(nb(N.nparams)), dim3(256), 0, s, N.nparams, ptr<float>(N.theta),
                       ptr<float>(N.grad), ptr<float>(N.m), ptr<float>(N.v), float(to->lr), c1, c2);
    NET_CHECK();
    pack_weights(N, s);
    SGDG_CHECK_HIP(hipMemcpyAsync(lp.data(), N.lossp.p, sizeof(double) * lp.size(), hipMemcpyDeviceToHost, s));
    SGDG_CHECK_HIP(hipStreamSynchronize(s));
    double l = 0;
    for (double v : lp) l += v;
    if (!std::isfinite(l)) throw Error{SGDG_E_NAN, "non-finite training loss"};
    losses.push_back(l);
  }
  SGDG_CHECK_HIP(hipStreamSynchronize(s));
  if (st) {
    const int w = std::min<int>(10, int(losses.size()));
    double a = 0, b = 0;
    for (int i = 0; i < w; ++i) {
      a += losses[i];
      b += losses[losses.size() - 1 - i];
    }
    st->loss_first = w ? a / w : 0.0;
    st->loss_last = w ? b / w : 0.0;
    st->steps = int(losses.size());
    st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  API_END
}

extern "C" sgdg_status sgdg_net_apply(sgdg_net n, const double* r_dev, double* z_dev, hipStream_t s) {
  API_BEGIN
  live(n);
  require(r_dev && z_dev && r_dev != z_dev, "null or aliased argument");
  net_apply_dev(n, r_dev, z_dev, s);
  API_END
}

extern "C" sgdg_status sgdg_net_forward(sgdg_net n, const float* x_dev, float* y_dev, hipStream_t s) {
  API_BEGIN
  live(n);
  require(x_dev && y_dev, "null argument");
  Net& N = *n;
  const Net::Tab& T = conv_tab(N, 1, per_item(N, 1, kInferItems));
  ensure_act(N, 1);
  hipLaunchKernelGGL(k_raw_in, dim3(nb(N.geo.Ptot)), dim3(256), 0, s, N.geo.Ptot, N.geo.R, x_dev,
                     actbuf(N, 1, 0));
  NET_CHECK();
  forward(N, T, 1, s);
  hipLaunchKernelGGL(k_raw_out, dim3(nb(N.geo.Ptot * N.geo.R)), dim3(256), 0, s, N.geo.Ptot, N.geo.R,
                     ptr<float>(N.Y), y_dev);
  NET_CHECK();
  API_END
}

extern "C" sgdg_status sgdg_net_backward(sgdg_net n, const float* x_dev, const float* dy_dev, float* grad_dev,
                                         hipStream_t s) {
  API_BEGIN
  live(n);
  require(x_dev && dy_dev && grad_dev, "null argument");
  Net& N = *n;
  const Net::Tab& T = conv_tab(N, 1, per_item(N, 1, kInferItems));
  ensure_act(N, 1);
  hipLaunchKernelGGL(k_raw_in, dim3(nb(N.geo.Ptot)), dim3(256), 0, s, N.geo.Ptot, N.geo.R, x_dev,
                     actbuf(N, 1, 0));
  NET_CHECK();
  forward(N, T, 1, s);
  hipLaunchKernelGGL(k_raw_in, dim3(nb(N.geo.Ptot)), dim3(256), 0, s, N.geo.Ptot, N.geo.R, dy_dev,
                     ptr<__bf16>(N.D0));
  NET_CHECK();
  backward(N, T, 1, s);
  SGDG_CHECK_HIP(hipMemcpyAsync(grad_dev, N.grad.p, sizeof(float) * N.nparams, hipMemcpyDeviceToDevice, s));
  API_END
}

extern "C" void sgdg_net_destroy(sgdg_net n) {
  if (!n) return;
  if (n->o) {
    if (n->o->recorder == n) n->o->recorder = nullptr;
    auto& v = n->o->nets;
    v.erase(std::remove(v.begin(), v.end(), n), v.end());
  }
  (void)hipDeviceSynchronize();
  delete n;
}
