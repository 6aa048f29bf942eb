// 3-D FFT convolution with the Helmholtz grid kernel (precorrected-FFT far
// field).  Zero-padded, pruned: forward y-z transforms of the physical x
// planes, then per (k_y, k_z) column an x transform, the product with the
// kernel spectrum and the inverse x transform in one LDS pass, then inverse
// y-z transforms back onto the physical planes.
#include <algorithm>

#include "device_common.h"
#include "fft_reg.h"
#include "kernels.h"

namespace scabs {

constexpr size_t LDS_BUDGET = 64 * 1024;
// threads per work-group, elements per thread held in registers by one
// work-group-wide Stockham stage, elements per lane of a wave-owned pass,
// minimum waves per SIMD (occupancy), and whether wave-owned passes are used
// (measured: wave-owned at 4 waves per SIMD for FP32, work-group-wide for FP64)
template <typename T> struct FftCfg {
  static constexpr int threads = 512, elems = 16, wave_elems = 16, min_waves = 4;
  static constexpr bool wave = true;
};
template <> struct FftCfg<double> {
  static constexpr int threads = 512, elems = 8, wave_elems = 16, min_waves = 4;
  static constexpr bool wave = false;
};

// P consecutive x planes of one field per work-group: y-z transforms.
// Forward: physical n1 x n2 plane -> zero-padded N1 x N2 spectrum (z lines
// with data first, then every y line).  Inverse: the reverse, keeping n1 x n2.
template <typename T, bool WAVE>
__global__ void __launch_bounds__(FftCfg<T>::threads, FftCfg<T>::min_waves)
plane_fwd_kernel(const cx<T> *__restrict__ phys, cx<T> *__restrict__ spec, int n0, int n1, int n2, int N1, int N2,
                 int P, const cx<T> *__restrict__ tw, int twL) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T> *buf = reinterpret_cast<cx<T> *>(smem_raw);
  const int f = blockIdx.y, x0 = blockIdx.x * P;
  const int np = min(P, n0 - x0);
  const int M = N1 * N2;
  const cx<T> *src = phys + ((size_t)f * n0 + x0) * n1 * n2;
  const FastDiv dM = make_fastdiv(M), dN2 = make_fastdiv(N2);
  for (int i = threadIdx.x; i < np * M; i += blockDim.x) {
    const int pl = fdiv(i, dM), r = i - pl * M, y = fdiv(r, dN2), z = r - y * N2;
    buf[lpad<T>(i)] = (y < n1 && z < n2) ? src[(size_t)pl * n1 * n2 + y * n2 + z] : czero<T>();
  }
  __syncthreads();
  lds_fft<T, FftCfg<T>::elems, FftCfg<T>::wave_elems, WAVE>(buf, N2, np * n1, n1, M, N2, 1, tw, twL, false);   // z lines with data
  lds_fft<T, FftCfg<T>::elems, FftCfg<T>::wave_elems, WAVE>(buf, N1, np * N2, N2, M, 1, N2, tw, twL, false);   // y lines
  cx<T> *dst = spec + ((size_t)f * n0 + x0) * M;
  for (int i = threadIdx.x; i < np * M; i += blockDim.x) dst[i] = buf[lpad<T>(i)];
}

template <typename T, bool WAVE>
__global__ void __launch_bounds__(FftCfg<T>::threads, FftCfg<T>::min_waves)
plane_inv_kernel(const cx<T> *__restrict__ spec, cx<T> *__restrict__ phys, int n0, int n1, int n2, int N1, int N2,
                 int P, const cx<T> *__restrict__ tw, int twL) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T> *buf = reinterpret_cast<cx<T> *>(smem_raw);
  const int f = blockIdx.y, x0 = blockIdx.x * P;
  const int np = min(P, n0 - x0);
  const int M = N1 * N2;
  const cx<T> *src = spec + ((size_t)f * n0 + x0) * M;
  for (int i = threadIdx.x; i < np * M; i += blockDim.x) buf[lpad<T>(i)] = src[i];
  __syncthreads();
  lds_fft<T, FftCfg<T>::elems, FftCfg<T>::wave_elems, WAVE>(buf, N1, np * N2, N2, M, 1, N2, tw, twL, true);    // y lines
  lds_fft<T, FftCfg<T>::elems, FftCfg<T>::wave_elems, WAVE>(buf, N2, np * n1, n1, M, N2, 1, tw, twL, true);    // z lines that are kept
  cx<T> *dst = phys + ((size_t)f * n0 + x0) * n1 * n2;
  const FastDiv dP = make_fastdiv(n1 * n2), dn2 = make_fastdiv(n2);
  for (int i = threadIdx.x; i < np * n1 * n2; i += blockDim.x) {
    const int pl = fdiv(i, dP), r = i - pl * n1 * n2, y = fdiv(r, dn2), z = r - y * n2;
    dst[i] = buf[lpad<T>(pl * M + y * N2 + z)];
  }
}

// mode 0: forward x FFT, product with ghat, inverse; x < n0 kept.
// mode 1: forward x FFT only over the full length (n0 == N0).
template <typename T, bool WAVE>
__global__ void __launch_bounds__(FftCfg<T>::threads, FftCfg<T>::min_waves)
xline_kernel(cx<T> *__restrict__ spec, int n0, int N0, int N1, int N2, int C, const cx<T> *__restrict__ ghat,
             const cx<T> *__restrict__ tw, int twL, int mode) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T> *buf = reinterpret_cast<cx<T> *>(smem_raw);   // [c][x]
  const int f = blockIdx.y, b0 = blockIdx.x * C;
  const int M = N1 * N2;
  const int nl = min(C, M - b0);
  cx<T> *base = spec + (size_t)f * n0 * M;
  const int LS = N0 + 1;   // odd line stride: the staging loop writes across lines
  const FastDiv dnl = make_fastdiv(nl), dN0 = make_fastdiv(N0), dN2 = make_fastdiv(N2);
  for (int i = threadIdx.x; i < nl * N0; i += blockDim.x) {
    const int x = fdiv(i, dnl), c = i - x * nl;
    buf[lpad<T>(c * LS + x)] = x < n0 ? base[(size_t)x * M + b0 + c] : czero<T>();
  }
  __syncthreads();
  lds_fft<T, FftCfg<T>::elems, FftCfg<T>::wave_elems, WAVE>(buf, N0, nl, 1, LS, 0, 1, tw, twL, false);
  if (mode == 0) {
    const int h1 = N1 / 2 + 1, h2 = N2 / 2 + 1;
    for (int i = threadIdx.x; i < nl * N0; i += blockDim.x) {
      const int c = fdiv(i, dN0), kx = i - c * N0;
      const int b = b0 + c;
      const int ky = fdiv(b, dN2), kz = b - ky * N2;
      const int ax = min(kx, N0 - kx), ay = min(ky, N1 - ky), az = min(kz, N2 - kz);
      const int a = lpad<T>(c * LS + kx);
      buf[a] = buf[a] * ghat[((size_t)ax * h1 + ay) * h2 + az];
    }
    __syncthreads();
    lds_fft<T, FftCfg<T>::elems, FftCfg<T>::wave_elems, WAVE>(buf, N0, nl, 1, LS, 0, 1, tw, twL, true);
  }
  for (int i = threadIdx.x; i < nl * n0; i += blockDim.x) {
    const int x = fdiv(i, dnl), c = i - x * nl;
    base[(size_t)x * M + b0 + c] = buf[lpad<T>(c * LS + x)];
  }
}

// ---- register-resident transforms ---------------------------------------------
// y-z planes: a lane holds one whole z line, then one whole y line, in its
// registers and transforms it there (lengths in reg_line_ok); the planes of
// a work-group meet in LDS between the two directions.
__host__ __device__ constexpr bool reg_line_ok(int n) {
  return n == 4 || n == 6 || n == 8 || n == 12 || n == 16 || n == 24 || n == 32 || n == 48;
}

// out[i os] = (DFT of in[0..nin) zero-padded to NN)[i] for i < nout.  The
// embedding has NN >= 2 n - 1, so a forward line's input (HALF_IN) and an
// inverse line's kept output (HALF_OUT) lie in the lower half: the upper
// half is known zero, or not computed back.
template <typename T, int NN, bool INV, bool HALF_IN, bool HALF_OUT>
__device__ __forceinline__ void line_dft(const cx<T> *in, int is, int nin, cx<T> *out, int os, int nout) {
  cx<T> v[NN];
#pragma unroll
  for (int i = 0; i < NN; i++) v[i] = (HALF_IN && i >= NN / 2) || i >= nin ? czero<T>() : in[i * is];
  rdft<T, NN, INV>(v);
#pragma unroll
  for (int i = 0; i < NN; i++)
    if ((!HALF_OUT || i < NN / 2) && i < nout) out[i * os] = v[i];
}
template <typename T, bool INV, bool HALF_IN, bool HALF_OUT>
__device__ __forceinline__ void line_dft_n(int NN, const cx<T> *in, int is, int nin, cx<T> *out, int os, int nout) {
  switch (NN) {
    case 4: line_dft<T, 4, INV, HALF_IN, HALF_OUT>(in, is, nin, out, os, nout); break;
    case 6: line_dft<T, 6, INV, HALF_IN, HALF_OUT>(in, is, nin, out, os, nout); break;
    case 8: line_dft<T, 8, INV, HALF_IN, HALF_OUT>(in, is, nin, out, os, nout); break;
    case 12: line_dft<T, 12, INV, HALF_IN, HALF_OUT>(in, is, nin, out, os, nout); break;
    case 16: line_dft<T, 16, INV, HALF_IN, HALF_OUT>(in, is, nin, out, os, nout); break;
    case 24: line_dft<T, 24, INV, HALF_IN, HALF_OUT>(in, is, nin, out, os, nout); break;
    case 32: line_dft<T, 32, INV, HALF_IN, HALF_OUT>(in, is, nin, out, os, nout); break;
    default: line_dft<T, 48, INV, HALF_IN, HALF_OUT>(in, is, nin, out, os, nout); break;
  }
}

constexpr int PLANE_REG_THREADS = 256;
// Forward: z lines y < n1 of P physical planes (zero-padded n2 -> N2) into LDS
// rows of stride N2 + 1, then every y line (n1 -> N1) out to the spectrum.
template <typename T>
__global__ void __launch_bounds__(PLANE_REG_THREADS)
plane_fwd_reg_kernel(const cx<T> *__restrict__ phys, cx<T> *__restrict__ spec, int n0, int n1, int n2, int N1,
                     int N2, int P) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T> *buf = reinterpret_cast<cx<T> *>(smem_raw);
  const int f = blockIdx.y, x0 = blockIdx.x * P;
  const int np = min(P, n0 - x0), S = N2 + 1;
  const cx<T> *src = phys + ((size_t)f * n0 + x0) * n1 * n2;
  for (int i = threadIdx.x; i < np * n1; i += blockDim.x)
    line_dft_n<T, false, true, false>(N2, src + (size_t)i * n2, 1, n2, buf + i * S, 1, N2);
  __syncthreads();
  cx<T> *dst = spec + ((size_t)f * n0 + x0) * N1 * N2;
  for (int i = threadIdx.x; i < np * N2; i += blockDim.x) {
    const int pl = i / N2, kz = i - pl * N2;
    line_dft_n<T, false, true, false>(N1, buf + pl * n1 * S + kz, S, n1, dst + (size_t)pl * N1 * N2 + kz, N2, N1);
  }
}
// Inverse: every y line (N1, kept y < n1) into LDS, then the z lines (kept z < n2).
template <typename T>
__global__ void __launch_bounds__(PLANE_REG_THREADS)
plane_inv_reg_kernel(const cx<T> *__restrict__ spec, cx<T> *__restrict__ phys, int n0, int n1, int n2, int N1,
                     int N2, int P) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T> *buf = reinterpret_cast<cx<T> *>(smem_raw);
  const int f = blockIdx.y, x0 = blockIdx.x * P;
  const int np = min(P, n0 - x0), S = N2 + 1;
  const cx<T> *src = spec + ((size_t)f * n0 + x0) * N1 * N2;
  for (int i = threadIdx.x; i < np * N2; i += blockDim.x) {
    const int pl = i / N2, kz = i - pl * N2;
    line_dft_n<T, true, false, true>(N1, src + (size_t)pl * N1 * N2 + kz, N2, N1, buf + pl * n1 * S + kz, S, n1);
  }
  __syncthreads();
  cx<T> *dst = phys + ((size_t)f * n0 + x0) * n1 * n2;
  for (int i = threadIdx.x; i < np * n1; i += blockDim.x)
    line_dft_n<T, true, false, true>(N2, buf + i * S, 1, N2, dst + (size_t)i * n2, 1, n2);
}
static int reg_planes(int n1, int N2) { return std::max(1, PLANE_REG_THREADS / std::max(n1, N2)); }

// x lines of length 1024: one wave per (k_y, k_z) column, 16 elements per
// lane.  1024 = 16 x 64: a 16-point transform in each lane's registers over
// x = l + 64 r, twiddles exp(-2 pi i l a / 1024), an exchange through LDS to
// lane 4 a + p holding l = p + 4 s, a 16-point transform over s, twiddles
// exp(-2 pi i p c / 64) and a 4-point transform across the lane quad: lane
// 4 a + p then holds k_x = a + 16 c + 256 d(p) in register c.  The product
// with the kernel spectrum is taken there, and the inverse runs the adjoint
// steps in reverse order back to x = l + 64 r.  The columns of a work-group
// are staged through LDS (row-major global rows, one LDS line per column);
// the exchange reuses the wave's own line.
// minimum waves per SIMD the register budget is sized for (LDS allows two
// work-groups per CU: 4 waves per SIMD in FP32)
template <typename T> struct XRegCfg {
  static constexpr int threads = 512, min_waves = 4;
  static constexpr bool lds_twiddles = true;   // twiddle table copied to LDS (fits beside two work-groups)
};
template <> struct XRegCfg<double> {
  static constexpr int threads = 256, min_waves = 2;
  static constexpr bool lds_twiddles = false;
};
constexpr int XR_TW = XLINE_REG_LEN + 64;   // twiddle table entries
constexpr int XR_LS = 1096;   // LDS line stride: >= 16 x 68 exchange slots, = 8 (mod 64)
constexpr int XR_XS = 68;     // exchange row stride

template <typename T>
__global__ void __launch_bounds__(XRegCfg<T>::threads, XRegCfg<T>::min_waves)
xline_reg_kernel(cx<T> *__restrict__ spec, int n0, int N1, int N2, const cx<T> *__restrict__ ghx,
                 const cx<T> *__restrict__ twx) {
  constexpr int C = XRegCfg<T>::threads / 64;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T> *buf = reinterpret_cast<cx<T> *>(smem_raw);
  // XCD-aware order: neighbouring column blocks, whose 64-byte row segments
  // share 128-byte lines, run on one XCD at about the same time
  const int nbx = gridDim.x;
  const int lb = xcd_remap(blockIdx.y * nbx + blockIdx.x, nbx * gridDim.y);
  const int f = lb / nbx, b0 = (lb - f * nbx) * C;
  const int M = N1 * N2;
  const int nl = min(C, M - b0);
  cx<T> *base = spec + (size_t)f * n0 * M + b0;
  const cx<T> *tw = twx;
  if (XRegCfg<T>::lds_twiddles) {
    cx<T> *tw_s = buf + C * XR_LS;
    for (int i = threadIdx.x; i < XR_TW; i += blockDim.x) tw_s[i] = twx[i];
    tw = tw_s;
  }
  {
    const int c = threadIdx.x % C, xr = threadIdx.x / C;   // 64 rows per pass
    for (int xb = 0; xb < n0; xb += 8 * 64) {
      cx<T> t[8];
#pragma unroll
      for (int k = 0; k < 8; k++) {
        const int x = xb + xr + 64 * k;
        t[k] = (x < n0 && c < nl) ? base[(size_t)x * M + c] : czero<T>();
      }
#pragma unroll
      for (int k = 0; k < 8; k++) {
        const int x = xb + xr + 64 * k;
        if (x < n0) buf[c * XR_LS + x] = t[k];
      }
    }
  }
  __syncthreads();
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (w < nl) {   // wave-uniform: every lane of the wave takes part below
    cx<T> *ln = buf + w * XR_LS;
    // n0 <= 512 (launch condition): elements 8..15 of every lane are the
    // zero padding, known zero here so the first 16-point transform folds them
    cx<T> v[16];
#pragma unroll
    for (int r = 0; r < 8; r++) {
      const int x = lane + 64 * r;
      v[r] = x < n0 ? ln[x] : czero<T>();
    }
#pragma unroll
    for (int r = 8; r < 16; r++) v[r] = czero<T>();
    rdft<T, 16, false>(v);
#pragma unroll
    for (int a = 1; a < 16; a++) v[a] = v[a] * tw[a * 64 + lane];
    wave_lds_fence();
#pragma unroll
    for (int a = 0; a < 16; a++) ln[a * XR_XS + lane] = v[a];
    wave_lds_fence();
    const int qa = lane >> 2, p = lane & 3;
    const QuadSigns<T> qs(p);
#pragma unroll
    for (int s = 0; s < 16; s++) v[s] = ln[qa * XR_XS + p + 4 * s];
    rdft<T, 16, false>(v);
#pragma unroll
    for (int c = 1; c < 16; c++) v[c] = v[c] * tw[XLINE_REG_LEN + c * 4 + p];
#pragma unroll
    for (int c = 0; c < 16; c++) v[c] = quad_dft4<T, false>(v[c], p, qs);
    // product with the kernel spectrum (octant storage with k_x fastest,
    // mirrored indices: the 16 lanes of one d read 16 neighbouring entries)
    const int b = b0 + w, ky = b / N2, kz = b - ky * N2;
    const int h2 = N2 / 2 + 1, h0 = XLINE_REG_LEN / 2 + 1;
    const cx<T> *gl = ghx + ((size_t)min(ky, N1 - ky) * h2 + min(kz, N2 - kz)) * h0;
    const int d = 2 * (p & 1) + (p >> 1);
#pragma unroll
    for (int c = 0; c < 16; c++) {
      const int kx = qa + 16 * c + 256 * d;
      v[c] = v[c] * gl[min(kx, XLINE_REG_LEN - kx)];
    }
#pragma unroll
    for (int c = 0; c < 16; c++) v[c] = quad_dft4<T, true>(v[c], p, qs);
#pragma unroll
    for (int c = 1; c < 16; c++) v[c] = twm<T, true>(v[c], tw[XLINE_REG_LEN + c * 4 + p]);
    rdft<T, 16, true>(v);
    wave_lds_fence();
#pragma unroll
    for (int s = 0; s < 16; s++) ln[qa * XR_XS + p + 4 * s] = v[s];
    wave_lds_fence();
#pragma unroll
    for (int a = 0; a < 16; a++) v[a] = ln[a * XR_XS + lane];
#pragma unroll
    for (int a = 1; a < 16; a++) v[a] = twm<T, true>(v[a], tw[a * 64 + lane]);
    rdft<T, 16, true>(v);
    wave_lds_fence();
    // only the physical range x < n0 <= 512 is kept: elements 0..7
#pragma unroll
    for (int r = 0; r < 8; r++) {
      const int x = lane + 64 * r;
      if (x < n0) ln[x] = v[r];
    }
  }
  __syncthreads();
  {
    const int c = threadIdx.x % C, xr = threadIdx.x / C;
    if (c < nl)
      for (int xb = 0; xb < n0; xb += 8 * 64) {
        cx<T> t[8];
#pragma unroll
        for (int k = 0; k < 8; k++) {
          const int x = xb + xr + 64 * k;
          t[k] = x < n0 ? buf[c * XR_LS + x] : czero<T>();
        }
#pragma unroll
        for (int k = 0; k < 8; k++) {
          const int x = xb + xr + 64 * k;
          if (x < n0) base[(size_t)x * M + c] = t[k];
        }
      }
  }
}

template <typename T> static int xline_lines(int N0) {
  int C = (int)std::min<size_t>(LDS_BUDGET / (sizeof(cx<T>) * (size_t)lpad_size<T>(N0 + 1)),
                                (size_t)FftCfg<T>::elems * FftCfg<T>::threads / N0);
  return std::max(1, std::min(C, 16));
}
template <typename T> static size_t xline_lds(int N0, int C) { return sizeof(cx<T>) * (size_t)lpad_size<T>(C * (N0 + 1)); }
template <typename T> static int planes_per_group(int N1, int N2) {
  int P = (int)std::min<size_t>(LDS_BUDGET / 2 / (sizeof(cx<T>) * (size_t)lpad_size<T>(N1 * N2)),
                                (size_t)FftCfg<T>::elems * FftCfg<T>::threads / ((size_t)N1 * N2));
  return std::max(1, P);
}

template <typename T> void launch_conv(const DevGrid<T> &g, hipStream_t s, int nb, int parts) {
  const int n0 = g.n[0], n1 = g.n[1], n2 = g.n[2];
  const int N0 = g.N[0], N1 = g.N[1], N2 = g.N[2];
  const int P = planes_per_group<T>(N1, N2);
  const size_t plane_lds = sizeof(cx<T>) * (size_t)lpad_size<T>(P * N1 * N2);
  const int npg = (n0 + P - 1) / P;
  const int nw = FftCfg<T>::threads / 64, EW = FftCfg<T>::wave_elems;
  // wave-owned passes measured faster in FP32 only (FP64 needs too many registers)
  const bool pw = FftCfg<T>::wave && wave_fits(N2, P * n1, nw, EW) && wave_fits(N1, P * N2, nw, EW);
  // register-resident y-z transforms where both lengths are supported
  const int Pr = std::min(reg_planes(n1, N2), (int)(LDS_BUDGET / (sizeof(cx<T>) * (size_t)n1 * (N2 + 1))));
  // (the register kernels assume the physical lengths fill at most half of
  // the transform lengths, which the embedding size guarantees)
  const bool preg = reg_line_ok(N1) && reg_line_ok(N2) && Pr >= 1 && 2 * n1 <= N1 && 2 * n2 <= N2;
  const size_t preg_lds = sizeof(cx<T>) * (size_t)Pr * n1 * (N2 + 1);
  const int npr = (n0 + Pr - 1) / Pr;
  if (!(parts & CONV_PLANES_FWD)) {
  } else if (preg)
    hipLaunchKernelGGL(plane_fwd_reg_kernel<T>, dim3(npr, 8 * nb), dim3(PLANE_REG_THREADS), preg_lds, s, g.phys,
                       g.spec, n0, n1, n2, N1, N2, Pr);
  else if (pw)
    hipLaunchKernelGGL((plane_fwd_kernel<T, true>), dim3(npg, 8 * nb), dim3(FftCfg<T>::threads), plane_lds, s, g.phys,
                       g.spec, n0, n1, n2, N1, N2, P, g.tw, g.twL);
  else
    hipLaunchKernelGGL((plane_fwd_kernel<T, false>), dim3(npg, 8 * nb), dim3(FftCfg<T>::threads), plane_lds, s, g.phys,
                       g.spec, n0, n1, n2, N1, N2, P, g.tw, g.twL);
  const int C = xline_lines<T>(N0);
  const int nlb = (N1 * N2 + C - 1) / C;
  constexpr int CR = XRegCfg<T>::threads / 64;
  if (!(parts & CONV_XLINES)) {
  } else if (g.twx && g.ghx && N0 == XLINE_REG_LEN && n0 <= XLINE_REG_LEN / 2)
    hipLaunchKernelGGL(xline_reg_kernel<T>, dim3((N1 * N2 + CR - 1) / CR, 8 * nb), dim3(XRegCfg<T>::threads),
                       sizeof(cx<T>) * ((size_t)CR * XR_LS + (XRegCfg<T>::lds_twiddles ? XR_TW : 0)), s, g.spec,
                       n0, N1, N2, g.ghx, g.twx);
  else if (FftCfg<T>::wave && wave_fits(N0, C, nw, EW))
    hipLaunchKernelGGL((xline_kernel<T, true>), dim3(nlb, 8 * nb), dim3(FftCfg<T>::threads), xline_lds<T>(N0, C), s,
                       g.spec, n0, N0, N1, N2, C, g.ghat, g.tw, g.twL, 0);
  else
    hipLaunchKernelGGL((xline_kernel<T, false>), dim3(nlb, 8 * nb), dim3(FftCfg<T>::threads), xline_lds<T>(N0, C), s,
                       g.spec, n0, N0, N1, N2, C, g.ghat, g.tw, g.twL, 0);
  if (!(parts & CONV_PLANES_INV)) {
  } else if (preg)
    hipLaunchKernelGGL(plane_inv_reg_kernel<T>, dim3(npr, 8 * nb), dim3(PLANE_REG_THREADS), preg_lds, s, g.spec,
                       g.phys, n0, n1, n2, N1, N2, Pr);
  else if (pw)
    hipLaunchKernelGGL((plane_inv_kernel<T, true>), dim3(npg, 8 * nb), dim3(FftCfg<T>::threads), plane_lds, s, g.spec,
                       g.phys, n0, n1, n2, N1, N2, P, g.tw, g.twL);
  else
    hipLaunchKernelGGL((plane_inv_kernel<T, false>), dim3(npg, 8 * nb), dim3(FftCfg<T>::threads), plane_lds, s, g.spec,
                       g.phys, n0, n1, n2, N1, N2, P, g.tw, g.twL);
}
template void launch_conv<float>(const DevGrid<float> &, hipStream_t, int, int);
template void launch_conv<double>(const DevGrid<double> &, hipStream_t, int, int);

template <typename T>
__global__ void ghat_xfast_kernel(const cx<T> *__restrict__ ghat, cx<T> *__restrict__ ghx, int h0, int h1, int h2) {
  const size_t total = (size_t)h0 * h1 * h2;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const int x = (int)(i % h0);
    const size_t yz = i / h0;
    const int z = (int)(yz % h2), y = (int)(yz / h2);
    ghx[i] = ghat[((size_t)x * h1 + y) * h2 + z];
  }
}
template <typename T> void launch_ghat_xfast(const cx<T> *ghat, cx<T> *ghx, int h0, int h1, int h2, hipStream_t s) {
  hipLaunchKernelGGL(ghat_xfast_kernel<T>, dim3(256), dim3(256), 0, s, ghat, ghx, h0, h1, h2);
}
template void launch_ghat_xfast<float>(const cx<float> *, cx<float> *, int, int, int, hipStream_t);
template void launch_ghat_xfast<double>(const cx<double> *, cx<double> *, int, int, int, hipStream_t);

// ---- kernel spectrum -----------------------------------------------------------
// circulant embedding of H(d) = G(h |d|) (H(0) = 0) on N0 x N1 x N2, offsets
// |d_a| <= n_a - 1 (the rest of the embedding is zero)
__global__ void sample_kernel(cx<double> *out, int N0, int N1, int N2, int n0, int n1, int n2, double h, double k) {
  size_t total = (size_t)N0 * N1 * N2;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    int z = (int)(i % N2), y = (int)((i / N2) % N1), x = (int)(i / ((size_t)N1 * N2));
    int dx = x <= N0 / 2 ? x : x - N0, dy = y <= N1 / 2 ? y : y - N1, dz = z <= N2 / 2 ? z : z - N2;
    cx<double> v = {0.0, 0.0};
    if (abs(dx) <= n0 - 1 && abs(dy) <= n1 - 1 && abs(dz) <= n2 - 1 && (dx || dy || dz)) {
      double R = h * sqrt((double)dx * dx + (double)dy * dy + (double)dz * dz);
      double sn, cs;
      sincos(k * R, &sn, &cs);
      double s = 1.0 / (4.0 * PI * R);
      v = {cs * s, -sn * s};
    }
    out[i] = v;
  }
}

__global__ void extract_octant(const cx<double> *full, cx<double> *g64, cx<float> *g32, int N0, int N1, int N2) {
  int h0 = N0 / 2 + 1, h1 = N1 / 2 + 1, h2 = N2 / 2 + 1;
  size_t total = (size_t)h0 * h1 * h2;
  double scale = 1.0 / ((double)N0 * N1 * N2);
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    int z = (int)(i % h2), y = (int)((i / h2) % h1), x = (int)(i / ((size_t)h1 * h2));
    cx<double> v = full[((size_t)x * N1 + y) * N2 + z];
    v.x *= scale;
    v.y *= scale;
    g64[i] = v;
    g32[i] = {(float)v.x, (float)v.y};
  }
}

hipError_t build_ghat(const GridDesc &d, double h, const cx<double> *tw64, int twL, cx<double> *ghat64,
                      cx<float> *ghat32, hipStream_t s) {
  const int N0 = d.N[0], N1 = d.N[1], N2 = d.N[2];
  size_t total = (size_t)N0 * N1 * N2;
  cx<double> *full = nullptr, *spec = nullptr;
  hipError_t e = hipMalloc(&full, total * sizeof(cx<double>));
  if (e != hipSuccess) return e;
  e = hipMalloc(&spec, total * sizeof(cx<double>));
  if (e != hipSuccess) {
    hipFree(full);
    return e;
  }
  hipLaunchKernelGGL(sample_kernel, dim3(1024), dim3(256), 0, s, full, N0, N1, N2, d.n[0], d.n[1], d.n[2], h, d.k);
  // forward 3-D FFT: y-z planes (full), then x lines (full length); one field
  const int P = planes_per_group<double>(N1, N2);
  const size_t plane_lds = sizeof(cx<double>) * (size_t)lpad_size<double>(P * N1 * N2);
  hipLaunchKernelGGL((plane_fwd_kernel<double, false>), dim3((N0 + P - 1) / P, 1), dim3(FftCfg<double>::threads), plane_lds, s, full, spec,
                     N0, N1, N2, N1, N2, P, tw64, twL);
  int C = xline_lines<double>(N0);
  int nb = (N1 * N2 + C - 1) / C;
  hipLaunchKernelGGL((xline_kernel<double, false>), dim3(nb, 1), dim3(FftCfg<double>::threads), xline_lds<double>(N0, C), s, spec, N0, N0, N1,
                     N2, C, (const cx<double> *)nullptr, tw64, twL, 1);
  hipLaunchKernelGGL(extract_octant, dim3(256), dim3(256), 0, s, spec, ghat64, ghat32, N0, N1, N2);
  e = hipGetLastError();
  hipError_t e2 = hipStreamSynchronize(s);
  hipFree(full);
  hipFree(spec);
  return e != hipSuccess ? e : e2;
}

}  // namespace scabs
