// x-transport preconditioner of the grid problems on periodic x-lattices (an
// extension of the grid-problem preconditioner of Sect. 4.3): the part of
// A_{l,l} whose x-factors are translation invariant, with the v-factors
// lumped to their row sums, is block-circulant in x for every v-node, so it is
// inverted mode by mode after a discrete Fourier transform over x.
#pragma once

#include "kernels.h"

namespace sgdg {

struct FourierSeg {
  int64_t off;     // start of the segment in the grid-problem layout ([R][nx][nv])
  int64_t poff;    // start of its mode inverses ([nx (modes)][nv][R][R] complex)
  int nx, nv, R;
  int n1;          // x-lattice nodes per axis (a power of two)
  int d;           // x dimension
};

struct FourierTab {
  int d = 1;
  int nlines = 0;                 // FFT lines per axis (every segment, slice, v-node, other axes)
  const FourierSeg* segs = nullptr;
  const int2* lines = nullptr;    // (segment, line within the segment)
  const double* pinv = nullptr;   // mode inverses, complex interleaved
};

// out = P^-1 in on the grid-problem layout of `total` elements (S: its
// segments); cbuf: 2 * total doubles of scratch.  in and out may alias.
template <class T>
void fourier_precond_n(const FourierTab& F, const SegTable& S, int64_t total, const T* in, T* out, double* cbuf,
                       hipStream_t s);

}  // namespace sgdg
