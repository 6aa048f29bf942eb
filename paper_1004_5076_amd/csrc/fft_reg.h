// In-register DFTs of compile-time length (a lane transforms a whole short
// line held in its registers) and the pieces of a wave-wide 1024-point
// transform: roots of unity evaluated at compile time, a recursive
// mixed-radix (4, 2, 3) decimation in time, and a 4-point DFT across the four
// lanes of a quad through DPP lane permutations.
#pragma once
#include "device_common.h"

namespace scabs {

struct CosSin {
  double c, s;
};
// cos x and sin x for 0 <= x <= pi/4 by their Taylor series (14 terms: below
// double rounding on that interval)
constexpr CosSin cs_series(double x) {
  double x2 = x * x, s = x, ts = x, c = 1.0, tc = 1.0;
  for (int k = 1; k <= 14; k++) {
    ts *= -x2 / ((2.0 * k) * (2.0 * k + 1.0));
    tc *= -x2 / ((2.0 * k - 1.0) * (2.0 * k));
    s += ts;
    c += tc;
  }
  return {c, s};
}
// cos and sin of 2 pi j / n: exact reduction to an octant in integer
// arithmetic, then the series and the octant's symmetry
constexpr CosSin cs_2pi(long j, long n) {
  j %= n;
  if (j < 0) j += n;
  const long m = 8 * j, o = m / n, r = m - o * n;
  const double q = 0.78539816339744830962;   // pi / 4
  double c = 0, s = 0;
  if (o & 1) {
    const CosSin t = cs_series(q * double(n - r) / double(n));
    c = t.s;
    s = t.c;
  } else {
    const CosSin t = cs_series(q * double(r) / double(n));
    c = t.c;
    s = t.s;
  }
  switch ((o >> 1) & 3) {
    case 1: {
      const double t = c;
      c = -s;
      s = t;
      break;
    }
    case 2:
      c = -c;
      s = -s;
      break;
    case 3: {
      const double t = c;
      c = s;
      s = -t;
      break;
    }
    default:
      break;
  }
  return {c, s};
}
// cos and sin of 2 pi j / N for j < N
template <int N> struct RootTable {
  double c[N], s[N];
  constexpr RootTable() : c(), s() {
    for (int j = 0; j < N; j++) {
      const CosSin t = cs_2pi(j, N);
      c[j] = t.c;
      s[j] = t.s;
    }
  }
};

// v * exp(-+ 2 pi i e / N) given cos and sin of 2 pi e / N (forward: minus)
template <typename T, bool INV> __host__ __device__ __forceinline__ cx<T> rot(cx<T> v, T c, T s) {
  return INV ? cx<T>{v.x * c - v.y * s, v.y * c + v.x * s} : cx<T>{v.x * c + v.y * s, v.y * c - v.x * s};
}
// v * w for a tabulated root w = exp(-2 pi i e / N); conj(w) for INV
template <typename T, bool INV> __host__ __device__ __forceinline__ cx<T> twm(cx<T> v, cx<T> w) {
  return INV ? cx<T>{v.x * w.x + v.y * w.y, v.y * w.x - v.x * w.y} : v * w;
}

template <int N> struct FirstRadix {
  static constexpr int value = (N % 4 == 0) ? 4 : ((N % 2 == 0) ? 2 : 3);
};

// X[k] = sum_n v[n] exp(-+ 2 pi i n k / N) in place (natural order in and
// out).  N = R M: the M-point transforms of the R decimated sequences
// v[R m + r], the twiddles exp(-+ 2 pi i r k / N), then R-point transforms
// across them (X[k + M k2]).
template <typename T, int N, bool INV> __host__ __device__ __forceinline__ void rdft(cx<T> *v) {
  if constexpr (N == 1) {
    return;
  } else if constexpr (N == 2 || N == 3 || N == 4 || N == 8) {
    dft_small<T, N>(v, INV);
  } else {
    constexpr int R = FirstRadix<N>::value, M = N / R;
    constexpr RootTable<N> W{};
    cx<T> sub[R][M];
#pragma unroll
    for (int r = 0; r < R; r++) {
#pragma unroll
      for (int m = 0; m < M; m++) sub[r][m] = v[R * m + r];
      rdft<T, M, INV>(sub[r]);
      if (r) {
#pragma unroll
        for (int k = 1; k < M; k++) {
          const int e = (r * k) % N;
          sub[r][k] = rot<T, INV>(sub[r][k], (T)W.c[e], (T)W.s[e]);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < M; k++) {
      cx<T> t[R];
#pragma unroll
      for (int r = 0; r < R; r++) t[r] = sub[r][k];
      dft_small<T, R>(t, INV);
#pragma unroll
      for (int r = 0; r < R; r++) v[k + M * r] = t[r];
    }
  }
}

// ---- quad-lane 4-point DFT -------------------------------------------------
// DPP quad permutations: lane p of each quad reads lane p ^ 1 / p ^ 2.
constexpr int DPP_XOR1 = 0xB1, DPP_XOR2 = 0x4E;
template <int CTRL> __device__ __forceinline__ float dpp_mov(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, false));
}
template <int CTRL> __device__ __forceinline__ double dpp_mov(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL, typename T> __device__ __forceinline__ cx<T> dpp_mov(cx<T> v) {
  return {dpp_mov<CTRL>(v.x), dpp_mov<CTRL>(v.y)};
}
// (this lane, partner) -> partner + sgn * this: the sum on the lower lane of
// the pair (sgn = 1), partner - this on the upper (sgn = -1); one exact FMA
template <int CTRL, typename T> __device__ __forceinline__ cx<T> quad_bfly(cx<T> v, T sgn) {
  const cx<T> o = dpp_mov<CTRL>(v);
  return {fma(sgn, v.x, o.x), fma(sgn, v.y, o.y)};
}
// Lane signs of the two butterflies for lane p of a quad
template <typename T> struct QuadSigns {
  T s1, s2;   // -1 on the upper lane of the xor-1 / xor-2 pairs
  __device__ explicit QuadSigns(int p) : s1((p & 1) ? T(-1) : T(1)), s2((p >= 2) ? T(-1) : T(1)) {}
};
// Forward: lane p (= lane & 3) holds z_p; afterwards lane p holds Z_{d(p)}
// with d(p) = 2 (p & 1) + (p >> 1), Z_d = sum_p z_p exp(-2 pi i p d / 4).
// Inverse (INV): the adjoint, from that order back to natural order with
// exp(+2 pi i p d / 4).  Every lane of the wave must take part.
template <typename T, bool INV> __device__ __forceinline__ cx<T> quad_dft4(cx<T> v, int p, const QuadSigns<T> &q) {
  if (!INV) {
    v = quad_bfly<DPP_XOR2>(v, q.s2);
    if (p == 3) v = cx<T>{v.y, -v.x};   // * (-i)
    return quad_bfly<DPP_XOR1>(v, q.s1);
  }
  v = quad_bfly<DPP_XOR1>(v, q.s1);
  if (p == 3) v = cx<T>{-v.y, v.x};     // * (+i)
  return quad_bfly<DPP_XOR2>(v, q.s2);
}

}  // namespace scabs
