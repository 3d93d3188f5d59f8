// Discrete Fourier transforms over periodic x-lattices and the mode-wise
// inverse of the x-transport preconditioner (see fourier.h).
//
// Convention: the forward transform is u^(theta) = sum_p u_p exp(-i theta.p),
// theta_a = 2 pi m_a / n1, unnormalised; the inverse carries the factor
// 1 / n1 per axis.  A stencil y_p = sum_o c_o u_{p+o} then acts on mode theta
// as the multiplication by sum_o c_o exp(i theta.o), which the host uses to
// build the mode inverses.  Each FFT line (n1 <= 1024 nodes along one x-axis
// at fixed slice, v-node and other x-coordinates) is one workgroup: radix-2
// butterflies in LDS after a bit-reversed load.
#include <hip/hip_runtime.h>

#include "fourier.h"

namespace sgdg {

namespace {

constexpr int kFB = 128;     // threads per FFT line
constexpr int kMaxN = 1024;  // longest line
constexpr int kSolveBlock = 256;

__device__ __forceinline__ int bitrev(int j, int logn) { return int(__brev(unsigned(j)) >> (32 - logn)); }

// in-place complex FFT along x-axis `axis` of every line; sign -1 forward, +1
// inverse (scaled by 1/n1)
__global__ void __launch_bounds__(kFB) k_fft_lines(const FourierSeg* __restrict__ segs, const int2* __restrict__ lines,
                                                   int axis, double sign, double* __restrict__ c) {
  __shared__ double re[kMaxN], im[kMaxN];
  const int2 L = lines[blockIdx.x];
  const FourierSeg S = segs[L.x];
  const int n = S.n1;
  if (n == 1) return;
  int logn = 0;
  while ((1 << logn) < n) ++logn;
  // decode the line: v-node q, slice s and the coordinates of the other axes
  int64_t l = L.y;
  const int q = int(l % S.nv);
  l /= S.nv;
  int64_t other = 1;
  for (int a = 0; a < S.d - 1; ++a) other *= n;
  const int64_t oth = l % other;
  const int s = int(l / other);
  int64_t xbase = 0, stride = 1, rem = oth, w = 1;
  for (int a = S.d - 1; a >= 0; --a) {  // axis a has x-stride n^(d-1-a)
    if (a == axis) {
      stride = w;
    } else {
      xbase += (rem % n) * w;
      rem /= n;
    }
    w *= n;
  }
  const int64_t base = S.off + int64_t(s) * S.nx * S.nv + xbase * S.nv + q;
  const int64_t st = stride * S.nv;
  for (int j = threadIdx.x; j < n; j += kFB) {
    const int64_t e = base + int64_t(j) * st;
    const int b = bitrev(j, logn);
    re[b] = c[2 * e];
    im[b] = c[2 * e + 1];
  }
  __syncthreads();
  for (int len = 2; len <= n; len <<= 1) {
    const int half = len >> 1;
    for (int k = threadIdx.x; k < n / 2; k += kFB) {
      const int grp = k / half, pos = k - grp * half;
      const int i = grp * len + pos, j = i + half;
      double sn, cs;
      sincospi(sign * 2.0 * double(pos) / double(len), &sn, &cs);
      const double tr = cs * re[j] - sn * im[j];
      const double ti = cs * im[j] + sn * re[j];
      re[j] = re[i] - tr;
      im[j] = im[i] - ti;
      re[i] += tr;
      im[i] += ti;
    }
    __syncthreads();
  }
  const double sc = sign > 0 ? 1.0 / double(n) : 1.0;
  for (int j = threadIdx.x; j < n; j += kFB) {
    const int64_t e = base + int64_t(j) * st;
    c[2 * e] = re[j] * sc;
    c[2 * e + 1] = im[j] * sc;
  }
}

template <class T>
__global__ void k_to_complex(int64_t n, const T* __restrict__ x, double* __restrict__ c) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  c[2 * i] = double(x[i]);
  c[2 * i + 1] = 0.0;
}

template <class T>
__global__ void k_to_real(int64_t n, const double* __restrict__ c, T* __restrict__ y) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  y[i] = T(c[2 * i]);
}

// z^(theta, q) = Pinv(theta, q) r^(theta, q) over the R slices, in place
__global__ void __launch_bounds__(kSolveBlock) k_mode_solve(const BlockRef* __restrict__ blk,
                                                            const FourierSeg* __restrict__ fsegs,
                                                            const double* __restrict__ pinv, double* __restrict__ c) {
  const BlockRef br = blk[blockIdx.x];
  const FourierSeg F = fsegs[br.seg];
  const int64_t plane = int64_t(F.nx) * F.nv;
  const int R = F.R;
  for (int t = 0; t < kChunk / kSolveBlock; ++t) {
    const int64_t p = int64_t(br.chunk) * kChunk + int64_t(t) * kSolveBlock + threadIdx.x;
    if (p >= plane) return;
    double xr[kMaxR], xi[kMaxR];
    for (int s = 0; s < R; ++s) {
      const int64_t e = F.off + s * plane + p;
      xr[s] = c[2 * e];
      xi[s] = c[2 * e + 1];
    }
    const double* P = pinv + 2 * (F.poff + p * R * R);
    for (int s = 0; s < R; ++s) {
      double ar = 0, ai = 0;
      for (int s2 = 0; s2 < R; ++s2) {
        const double pr = P[2 * (s * R + s2)], pi = P[2 * (s * R + s2) + 1];
        ar += pr * xr[s2] - pi * xi[s2];
        ai += pr * xi[s2] + pi * xr[s2];
      }
      const int64_t e = F.off + s * plane + p;
      c[2 * e] = ar;
      c[2 * e + 1] = ai;
    }
  }
}

}  // namespace

template <class T>
void fourier_precond_n(const FourierTab& F, const SegTable& S, int64_t total, const T* in, T* out, double* cbuf,
                       hipStream_t s) {
  const unsigned nb = unsigned((total + 255) / 256);
  hipLaunchKernelGGL(k_to_complex<T>, dim3(nb), dim3(256), 0, s, total, in, cbuf);
  SGDG_CHECK_HIP(hipGetLastError());
  for (int a = 0; a < F.d; ++a) {
    hipLaunchKernelGGL(k_fft_lines, dim3(unsigned(F.nlines)), dim3(kFB), 0, s, F.segs, F.lines, a, -1.0, cbuf);
    SGDG_CHECK_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_mode_solve, dim3(unsigned(S.nblk)), dim3(kSolveBlock), 0, s, S.blk, F.segs, F.pinv, cbuf);
  SGDG_CHECK_HIP(hipGetLastError());
  for (int a = 0; a < F.d; ++a) {
    hipLaunchKernelGGL(k_fft_lines, dim3(unsigned(F.nlines)), dim3(kFB), 0, s, F.segs, F.lines, a, 1.0, cbuf);
    SGDG_CHECK_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_to_real<T>, dim3(nb), dim3(256), 0, s, total, cbuf, out);
  SGDG_CHECK_HIP(hipGetLastError());
}

template void fourier_precond_n<double>(const FourierTab&, const SegTable&, int64_t, const double*, double*, double*,
                                        hipStream_t);
template void fourier_precond_n<float>(const FourierTab&, const SegTable&, int64_t, const float*, float*, double*,
                                       hipStream_t);

}  // namespace sgdg
