// Device helpers shared by the HIP kernels: complex arithmetic, Lagrange
// stencils and an in-LDS radix-2 Stockham FFT.
#pragma once
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "internal.h"

namespace scabs {

template <typename T> __host__ __device__ inline cx<T> mk(T a, T b) { return cx<T>{a, b}; }
template <typename T> __host__ __device__ inline cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T> __host__ __device__ inline cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T> __host__ __device__ inline cx<T> operator-(cx<T> a) { return {-a.x, -a.y}; }
template <typename T> __host__ __device__ inline cx<T> operator*(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T> __host__ __device__ inline cx<T> operator*(T s, cx<T> a) { return {s * a.x, s * a.y}; }
template <typename T> __host__ __device__ inline cx<T> operator*(cx<T> a, T s) { return {s * a.x, s * a.y}; }
template <typename T> __host__ __device__ inline cx<T> &operator+=(cx<T> &a, cx<T> b) {
  a.x += b.x;
  a.y += b.y;
  return a;
}
template <typename T> __host__ __device__ inline cx<T> &operator-=(cx<T> &a, cx<T> b) {
  a.x -= b.x;
  a.y -= b.y;
  return a;
}
template <typename T> __host__ __device__ inline cx<T> czero() { return {T(0), T(0)}; }
template <typename T> __host__ __device__ inline cx<T> mul_j(cx<T> a) { return {-a.y, a.x}; }   // j * a
template <typename T> __host__ __device__ inline cx<T> conjc(cx<T> a) { return {a.x, -a.y}; }
// acc += a * b in four FMAs (complex multiply-accumulate; written out so the
// accumulation fuses instead of a product followed by an add)
template <typename T> __host__ __device__ inline void cmac(cx<T> &acc, cx<T> a, cx<T> b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}
// a += s * b (s real)
template <typename T> __host__ __device__ inline void axpy(cx<T> &a, T s, cx<T> b) {
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

// the same weights for a node at offset o (-1, 0, 1) from the anchor:
// (1 - u^2) at o = 0, u (u + o) / 2 otherwise; and d/du of it
template <typename T> __device__ __forceinline__ T lag_w(int o, T u) {
  return o == 0 ? T(1) - u * u : T(0.5) * u * (u + T(o));
}
template <typename T> __device__ __forceinline__ T lag_d(int o, T u) { return o == 0 ? T(-2) * u : u + T(0.5) * T(o); }

__device__ inline void unpack_anchor(int a, int &x, int &y, int &z) {
  x = a & 0x3fff;
  y = (a >> 14) & 0x1ff;
  z = (a >> 23) & 0x1ff;
}

// ---------------------------------------------------------------------------
// Mixed-radix (8, 4, 2, 3) Stockham FFTs of lines held in LDS.
// Line l (0 <= l < nlines) starts at logical index (l / nin) * lso + (l % nin) * lsi;
// element e of a line is at + e * es; logical index a lives at buf[lpad(a)].  tw holds exp(-2 pi i j / twL) for
// 0 <= j < twL, twL a multiple of L.  Stage with radix R and input stride
// Ns: v_r = x[j + r L/R], v_r *= w^(r k), k = j mod Ns, w = exp(-+2 pi i/(Ns R)),
// V = DFT_R(v), y[(j - k) R + k + r Ns] = V_r.  ELEMS bounds the elements per
// thread (nlines * L <= ELEMS * blockDim.x).  All threads must call it.
// ---------------------------------------------------------------------------
template <typename T, int R> __host__ __device__ inline void dft_small(cx<T> *v, bool inv) {
  if (R == 2) {
    cx<T> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
  } else if (R == 3) {
    const T h = T(0.86602540378443864676);   // sqrt(3)/2
    cx<T> a = v[0], b = v[1], c = v[2];
    cx<T> s = b + c, d = b - c;
    cx<T> m = {a.x - T(0.5) * s.x, a.y - T(0.5) * s.y};
    // i * (sign) * h * d ; forward sign -1
    cx<T> rot = inv ? cx<T>{-h * d.y, h * d.x} : cx<T>{h * d.y, -h * d.x};
    v[0] = a + s;
    v[1] = m + rot;
    v[2] = m - rot;
  } else if (R == 4) {
    cx<T> t0 = v[0] + v[2], t1 = v[0] - v[2], t2 = v[1] + v[3], t3 = v[1] - v[3];
    // forward: X1 = t1 - i t3, X3 = t1 + i t3
    cx<T> it3 = inv ? cx<T>{-t3.y, t3.x} : cx<T>{t3.y, -t3.x};
    v[0] = t0 + t2;
    v[2] = t0 - t2;
    v[1] = t1 + it3;
    v[3] = t1 - it3;
  } else if (R == 8) {
    const T c = T(0.70710678118654752440);
    cx<T> e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
    dft_small<T, 4>(e, inv);
    dft_small<T, 4>(o, inv);
    // twiddles W^m, W = exp(-+ 2 pi i / 8)
    cx<T> w1 = inv ? cx<T>{c * (o[1].x - o[1].y), c * (o[1].x + o[1].y)}
                   : cx<T>{c * (o[1].x + o[1].y), c * (o[1].y - o[1].x)};
    cx<T> w2 = inv ? cx<T>{-o[2].y, o[2].x} : cx<T>{o[2].y, -o[2].x};
    cx<T> w3 = inv ? cx<T>{-c * (o[3].x + o[3].y), c * (o[3].x - o[3].y)}
                   : cx<T>{c * (o[3].y - o[3].x), -c * (o[3].x + o[3].y)};
    v[0] = e[0] + o[0];
    v[4] = e[0] - o[0];
    v[1] = e[1] + w1;
    v[5] = e[1] - w1;
    v[2] = e[2] + w2;
    v[6] = e[2] - w2;
    v[3] = e[3] + w3;
    v[7] = e[3] - w3;
  }
}

// complex coefficient stored as two FP16 halves (real in the low 16 bits)
__device__ inline cx<float> unpack_h2(uint32_t v) {
  return {__half2float(__ushort_as_half((unsigned short)(v & 0xffffu))),
          __half2float(__ushort_as_half((unsigned short)(v >> 16)))};
}
__device__ inline uint32_t pack_h2(float re, float im) {
  return (uint32_t)__half_as_ushort(__float2half_rn(re)) | ((uint32_t)__half_as_ushort(__float2half_rn(im)) << 16);
}

// XCD-aware work-group order.  Work-groups are dealt round-robin to the 8
// XCDs (each with its own L2) in linear order, so ids lin and lin + 8 run on
// the same XCD at about the same time.  Renumbering so that every XCD takes a
// contiguous range of logical ids gives those two neighbouring logical ids:
// work that shares lines with its neighbour (the next column block, the next
// lattice plane) then finds them in the same L2.  A bijection of [0, total).
__device__ inline int xcd_remap(int lin, int total) {
  const int q = total >> 3, rem = total & 7, i = lin & 7, k = lin >> 3;
  return i * q + min(i, rem) + k;
}

// One halving exchange of a per-lane array (any arithmetic type): lanes whose
// bit (lane & MASK) is set keep the upper HALF values, the others the lower
// HALF; each adds its partner's copy of the kept values (partner = lane ^
// MASK).  Kept values move to v[0, HALF).
template <typename T, int HALF, int MASK> __device__ inline void halve_exchange_t(T *v, int lane) {
  const bool up = (lane & MASK) != 0;
#pragma unroll
  for (int k = 0; k < HALF; k++) {
    const T send = up ? v[k] : v[k + HALF];
    const T keep = up ? v[k + HALF] : v[k];
    v[k] = keep + __shfl_xor(send, MASK, 64);
  }
}

// One halving exchange: lanes whose bit (lane & MASK) is set keep the upper
// HALF values, the others the lower HALF; each adds its partner's copy of the
// kept values (partner = lane ^ MASK).  Kept values move to v[0, HALF).
template <int HALF, int MASK> __device__ inline void halve_exchange(double *v, int lane) {
  const bool up = (lane & MASK) != 0;
#pragma unroll
  for (int k = 0; k < HALF; k++) {
    const double send = up ? v[k] : v[k + HALF];
    const double keep = up ? v[k + HALF] : v[k];
    v[k] = keep + __shfl_xor(send, MASK, 64);
  }
}

// Sum over the 64 lanes of 16 values at once: four halving exchanges leave
// lane L with a 16-lane partial of value (L >> 2) & 15, two more exchanges
// finish it.  Returns, on every lane, the full sum of value (L >> 2) & 15.
__device__ inline double wsum16_scatter(double v[16]) {
  const int lane = threadIdx.x & 63;
  halve_exchange<8, 32>(v, lane);
  halve_exchange<4, 16>(v, lane);
  halve_exchange<2, 8>(v, lane);
  halve_exchange<1, 4>(v, lane);
  double t = v[0];
  t += __shfl_xor(t, 2, 64);
  t += __shfl_xor(t, 1, 64);
  return t;
}

// Division by a work-group-uniform divisor d >= 1 through a multiply-high
// (round-up method of Granlund and Montgomery): for 0 <= n < 2^31,
// n / d = (umulhi(n, m) + n) >> s with s = ceil(log2 d),
// m = floor(2^32 (2^s - d) / d) + 1.
struct FastDiv {
  unsigned m, s, d;
};
__host__ __device__ inline FastDiv make_fastdiv(unsigned d) {
  unsigned s = 0;
  while ((1u << s) < d) s++;
  const unsigned long long two32 = 1ull << 32;
  const unsigned m = (unsigned)((two32 * ((1ull << s) - d)) / d + 1);
  return {m, s, d};
}
__device__ inline int fdiv(int n, FastDiv f) { return (int)((__umulhi((unsigned)n, f.m) + (unsigned)n) >> f.s); }

// LDS address swizzle for the FFT buffers: one pad element every 16 breaks
// the power-of-two strides of Stockham writes (outputs of a radix-R stage
// land R elements apart) and of strided lines.
template <typename T> __device__ inline int lpad(int a) { return a + (a >> 4); }
template <typename T> __host__ __device__ inline int lpad_size(int n) { return n + (n >> 4) + 1; }

template <typename T, int R, int NB>
__device__ inline void stockham_stage(cx<T> *buf, int L, int nlines, int nin, int lso, int lsi, int es, int Ns,
                                      const cx<T> *tw, int twL, bool inv) {
  const int LR = L / R;
  const int nb = nlines * LR;
  const FastDiv dLR = make_fastdiv(LR), dnin = make_fastdiv(nin), dNs = make_fastdiv(Ns);
  const int tstep = twL / (Ns * R);
  cx<T> v[NB][R];
  int ob[NB];
#pragma unroll
  for (int c = 0; c < NB; c++) {
    const int b = threadIdx.x + c * blockDim.x;
    if (b < nb) {
      const int line = fdiv(b, dLR), j = b - line * LR;
      const int lo = fdiv(line, dnin);
      const int base = lo * lso + (line - lo * nin) * lsi;
      const int k = j - fdiv(j, dNs) * Ns;
#pragma unroll
      for (int r = 0; r < R; r++) v[c][r] = buf[lpad<T>(base + (j + r * LR) * es)];
      if (k) {
        const int step = tstep * k;
#pragma unroll
        for (int r = 1; r < R; r++) {
          cx<T> w = tw[r * step];
          if (inv) w.y = -w.y;
          v[c][r] = v[c][r] * w;
        }
      }
      dft_small<T, R>(v[c], inv);
      ob[c] = base + ((j - k) * R + k) * es;
    }
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NB; c++) {
    const int b = threadIdx.x + c * blockDim.x;
    if (b < nb) {
#pragma unroll
      for (int r = 0; r < R; r++) buf[lpad<T>(ob[c] + r * Ns * es)] = v[c][r];
    }
  }
  __syncthreads();
}

template <typename T, int ELEMS>
__device__ void lds_fft_mr(cx<T> *buf, int L, int nlines, int nin, int lso, int lsi, int es, const cx<T> *tw, int twL,
                           bool inv) {
  int m = L, Ns = 1;
  while (m > 1) {
    if (m % 8 == 0) {
      stockham_stage<T, 8, (ELEMS + 7) / 8>(buf, L, nlines, nin, lso, lsi, es, Ns, tw, twL, inv);
      m /= 8;
      Ns *= 8;
    } else if (m % 4 == 0) {
      stockham_stage<T, 4, (ELEMS + 3) / 4>(buf, L, nlines, nin, lso, lsi, es, Ns, tw, twL, inv);
      m /= 4;
      Ns *= 4;
    } else if (m % 2 == 0) {
      stockham_stage<T, 2, (ELEMS + 1) / 2>(buf, L, nlines, nin, lso, lsi, es, Ns, tw, twL, inv);
      m /= 2;
      Ns *= 2;
    } else {
      stockham_stage<T, 3, (ELEMS + 2) / 3>(buf, L, nlines, nin, lso, lsi, es, Ns, tw, twL, inv);
      m /= 3;
      Ns *= 3;
    }
  }
}

// Wave-owned variant: the lines [0, nlines) are split into contiguous groups,
// one per wave of the work-group; each wave runs every stage on its own group
// with only wave-level ordering between stages (no work-group barrier).  The
// caller synchronises the work-group before (data loaded) and after (data
// consumed by other waves).  Requires ceil(nlines / waves) * L <= ELEMS * 64.
__device__ inline void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T, int R, int NB>
__device__ inline void stockham_stage_w(cx<T> *buf, int L, int l0, int l1, int nin, int lso, int lsi, int es, int Ns,
                                        const cx<T> *tw, int twL, bool inv, int lane) {
  const int LR = L / R;
  const int nb = (l1 - l0) * LR;
  const FastDiv dLR = make_fastdiv(LR), dnin = make_fastdiv(nin), dNs = make_fastdiv(Ns);
  const int tstep = twL / (Ns * R);
  cx<T> v[NB][R];
  int ob[NB];
#pragma unroll
  for (int c = 0; c < NB; c++) {
    const int b = lane + c * 64;
    if (b < nb) {
      const int lr = fdiv(b, dLR), j = b - lr * LR;
      const int line = l0 + lr;
      const int lo = fdiv(line, dnin);
      const int base = lo * lso + (line - lo * nin) * lsi;
      const int k = j - fdiv(j, dNs) * Ns;
#pragma unroll
      for (int r = 0; r < R; r++) v[c][r] = buf[lpad<T>(base + (j + r * LR) * es)];
      if (k) {
        const int step = tstep * k;
#pragma unroll
        for (int r = 1; r < R; r++) {
          cx<T> w = tw[r * step];
          if (inv) w.y = -w.y;
          v[c][r] = v[c][r] * w;
        }
      }
      dft_small<T, R>(v[c], inv);
      ob[c] = base + ((j - k) * R + k) * es;
    }
  }
  wave_lds_fence();
#pragma unroll
  for (int c = 0; c < NB; c++) {
    const int b = lane + c * 64;
    if (b < nb) {
#pragma unroll
      for (int r = 0; r < R; r++) buf[lpad<T>(ob[c] + r * Ns * es)] = v[c][r];
    }
  }
  wave_lds_fence();
}

template <typename T, int ELEMS>
__device__ void lds_fft_wave(cx<T> *buf, int L, int nlines, int nin, int lso, int lsi, int es, const cx<T> *tw,
                             int twL, bool inv) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int G = (nlines + nw - 1) / nw;
  const int l0 = min(nlines, wave * G), l1 = min(nlines, l0 + G);
  int m = L, Ns = 1;
  while (m > 1) {
    if (m % 8 == 0) {
      stockham_stage_w<T, 8, (ELEMS + 7) / 8>(buf, L, l0, l1, nin, lso, lsi, es, Ns, tw, twL, inv, lane);
      m /= 8;
      Ns *= 8;
    } else if (m % 4 == 0) {
      stockham_stage_w<T, 4, (ELEMS + 3) / 4>(buf, L, l0, l1, nin, lso, lsi, es, Ns, tw, twL, inv, lane);
      m /= 4;
      Ns *= 4;
    } else if (m % 2 == 0) {
      stockham_stage_w<T, 2, (ELEMS + 1) / 2>(buf, L, l0, l1, nin, lso, lsi, es, Ns, tw, twL, inv, lane);
      m /= 2;
      Ns *= 2;
    } else {
      stockham_stage_w<T, 3, (ELEMS + 2) / 3>(buf, L, l0, l1, nin, lso, lsi, es, Ns, tw, twL, inv, lane);
      m /= 3;
      Ns *= 3;
    }
  }
}

// Transforms of nlines lines: wave-owned (WAVE, the caller guarantees a
// wave's share fits EW elements per lane) or work-group-wide; the data is
// visible to the whole work-group on return.
template <typename T, int ELEMS, int EW, bool WAVE>
__device__ inline void lds_fft(cx<T> *buf, int L, int nlines, int nin, int lso, int lsi, int es, const cx<T> *tw,
                               int twL, bool inv) {
  if (WAVE) {
    lds_fft_wave<T, EW>(buf, L, nlines, nin, lso, lsi, es, tw, twL, inv);
    __syncthreads();
  } else {
    lds_fft_mr<T, ELEMS>(buf, L, nlines, nin, lso, lsi, es, tw, twL, inv);
  }
}
// whether nlines lines of length L split over nw waves fit EW elements per lane
__host__ __device__ inline bool wave_fits(int L, int nlines, int nw, int EW) {
  return ((nlines + nw - 1) / nw) * L <= EW * 64;
}

}  // namespace scabs
