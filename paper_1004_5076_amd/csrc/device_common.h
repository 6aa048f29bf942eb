// Device helpers shared by the HIP kernels: complex arithmetic, Lagrange
// stencils and an in-LDS radix-2 Stockham FFT.
#pragma once
#include <hip/hip_runtime.h>

#include "internal.h"

namespace scabs {

template <typename T> __host__ __device__ inline cx<T> mk(T a, T b) { return cx<T>{a, b}; }
template <typename T> __device__ inline cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T> __device__ inline cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T> __device__ inline cx<T> operator-(cx<T> a) { return {-a.x, -a.y}; }
template <typename T> __device__ inline cx<T> operator*(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T> __device__ inline cx<T> operator*(T s, cx<T> a) { return {s * a.x, s * a.y}; }
template <typename T> __device__ inline cx<T> operator*(cx<T> a, T s) { return {s * a.x, s * a.y}; }
template <typename T> __device__ inline cx<T> &operator+=(cx<T> &a, cx<T> b) {
  a.x += b.x;
  a.y += b.y;
  return a;
}
template <typename T> __device__ inline cx<T> &operator-=(cx<T> &a, cx<T> b) {
  a.x -= b.x;
  a.y -= b.y;
  return a;
}
template <typename T> __device__ inline cx<T> czero() { return {T(0), T(0)}; }
template <typename T> __device__ inline cx<T> mul_j(cx<T> a) { return {-a.y, a.x}; }   // j * a
template <typename T> __device__ inline cx<T> conjc(cx<T> a) { return {a.x, -a.y}; }
// a += s * b (s real)
template <typename T> __device__ inline void axpy(cx<T> &a, T s, cx<T> b) {
  a.x += s * b.x;
  a.y += s * b.y;
}

// 3-point Lagrange weights on nodes -1, 0, +1 at offset u in [-1/2, 1/2] and
// their derivatives d/du.
template <typename T> __device__ inline void lagr3(T u, T *L, T *dL) {
  L[0] = T(0.5) * u * (u - T(1));
  L[1] = T(1) - u * u;
  L[2] = T(0.5) * u * (u + T(1));
  dL[0] = u - T(0.5);
  dL[1] = T(-2) * u;
  dL[2] = u + T(0.5);
}

__device__ inline void unpack_anchor(int a, int &x, int &y, int &z) {
  x = a & 0x3fff;
  y = (a >> 14) & 0x1ff;
  z = (a >> 23) & 0x1ff;
}

// Radix-2 Stockham FFTs of `nlines` lines of length L (power of two) held in
// LDS: element e of line l at buf[l * lstride + e * estride].  tw holds
// exp(-2 pi i j / twL), j < twL / 2, twL >= L.  MAXB bounds the butterflies
// per thread per stage (nlines * L / 2 <= MAXB * blockDim.x).  All threads of
// the block must call it.
template <typename T, int MAXB>
__device__ void lds_fft(cx<T> *buf, int L, int nlines, int lstride, int estride, const cx<T> *tw, int twL,
                        bool inverse) {
  const int half = L >> 1;
  const int nb = nlines * half;
  int lgh = 0;
  while ((1 << lgh) < half) lgh++;
  for (int Ns = 1; Ns < L; Ns <<= 1) {
    cx<T> ra[MAXB], rb[MAXB];
    int ro[MAXB];
#pragma unroll
    for (int c = 0; c < MAXB; c++) {
      int t = threadIdx.x + c * blockDim.x;
      if (t < nb) {
        int line = t >> lgh, j = t & (half - 1);
        cx<T> *base = buf + line * lstride;
        cx<T> a = base[j * estride], b = base[(j + half) * estride];
        int k = j & (Ns - 1);
        cx<T> w = tw[k * (twL / (2 * Ns))];
        if (inverse) w.y = -w.y;
        b = b * w;
        ra[c] = a + b;
        rb[c] = a - b;
        ro[c] = line * lstride + ((j - k) * 2 + k) * estride;
      }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < MAXB; c++) {
      int t = threadIdx.x + c * blockDim.x;
      if (t < nb) {
        buf[ro[c]] = ra[c];
        buf[ro[c] + Ns * estride] = rb[c];
      }
    }
    __syncthreads();
  }
}

}  // namespace scabs
