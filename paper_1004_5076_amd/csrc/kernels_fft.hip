// 3-D FFT convolution with the Helmholtz grid kernel (precorrected-FFT far
// field).  Zero-padded, pruned: forward y-z transforms of the physical x
// planes, then per (k_y, k_z) column an x transform, the product with the
// kernel spectrum and the inverse x transform in one LDS pass, then inverse
// y-z transforms back onto the physical planes.
#include <algorithm>

#include "device_common.h"
#include "kernels.h"

namespace scabs {

constexpr int FFT_THREADS = 256;
constexpr size_t LDS_BUDGET = 64 * 1024;
// butterflies per thread per stage held in registers by the x-line kernel
template <typename T> struct XStage { static constexpr int value = 16; };
template <> struct XStage<double> { static constexpr int value = 8; };

template <typename T>
__global__ void __launch_bounds__(FFT_THREADS)
plane_fwd_kernel(const cx<T> *__restrict__ phys, cx<T> *__restrict__ spec, int n0, int n1, int n2, int N1, int N2,
                 const cx<T> *__restrict__ tw, int twL) {
  extern __shared__ unsigned char smem_raw[];
  cx<T> *buf = reinterpret_cast<cx<T> *>(smem_raw);
  const int x = blockIdx.x, f = blockIdx.y;
  const int M = N1 * N2;
  const cx<T> *src = phys + ((size_t)f * n0 + x) * n1 * n2;
  for (int i = threadIdx.x; i < M; i += blockDim.x) {
    int y = i / N2, z = i - y * N2;
    buf[i] = (y < n1 && z < n2) ? src[y * n2 + z] : czero<T>();
  }
  __syncthreads();
  lds_fft<T, 8>(buf, N2, n1, N2, 1, tw, twL, false);   // z lines with data
  lds_fft<T, 8>(buf, N1, N2, 1, N2, tw, twL, false);   // y lines
  cx<T> *dst = spec + ((size_t)f * n0 + x) * M;
  for (int i = threadIdx.x; i < M; i += blockDim.x) dst[i] = buf[i];
}

template <typename T>
__global__ void __launch_bounds__(FFT_THREADS)
plane_inv_kernel(const cx<T> *__restrict__ spec, cx<T> *__restrict__ phys, int n0, int n1, int n2, int N1, int N2,
                 const cx<T> *__restrict__ tw, int twL) {
  extern __shared__ unsigned char smem_raw[];
  cx<T> *buf = reinterpret_cast<cx<T> *>(smem_raw);
  const int x = blockIdx.x, f = blockIdx.y;
  const int M = N1 * N2;
  const cx<T> *src = spec + ((size_t)f * n0 + x) * M;
  for (int i = threadIdx.x; i < M; i += blockDim.x) buf[i] = src[i];
  __syncthreads();
  lds_fft<T, 8>(buf, N1, N2, 1, N2, tw, twL, true);    // y lines
  lds_fft<T, 8>(buf, N2, n1, N2, 1, tw, twL, true);    // z lines that are kept
  cx<T> *dst = phys + ((size_t)f * n0 + x) * n1 * n2;
  for (int i = threadIdx.x; i < n1 * n2; i += blockDim.x) {
    int y = i / n2, z = i - y * n2;
    dst[i] = buf[y * N2 + z];
  }
}

// mode 0: forward x FFT, product with ghat, inverse; x < n0 kept.
// mode 1: forward x FFT only over the full length (n0 == N0).
template <typename T>
__global__ void __launch_bounds__(FFT_THREADS)
xline_kernel(cx<T> *__restrict__ spec, int n0, int N0, int N1, int N2, int C, const cx<T> *__restrict__ ghat,
             const cx<T> *__restrict__ tw, int twL, int mode) {
  extern __shared__ unsigned char smem_raw[];
  cx<T> *buf = reinterpret_cast<cx<T> *>(smem_raw);   // [c][x]
  const int f = blockIdx.y, b0 = blockIdx.x * C;
  const int M = N1 * N2;
  cx<T> *base = spec + (size_t)f * n0 * M;
  for (int i = threadIdx.x; i < C * N0; i += blockDim.x) {
    int x = i / C, c = i - x * C;
    cx<T> v = czero<T>();
    if (x < n0 && b0 + c < M) v = base[(size_t)x * M + b0 + c];
    buf[c * N0 + x] = v;
  }
  __syncthreads();
  lds_fft<T, XStage<T>::value>(buf, N0, C, N0, 1, tw, twL, false);
  if (mode == 0) {
    const int h1 = N1 / 2 + 1, h2 = N2 / 2 + 1;
    for (int i = threadIdx.x; i < C * N0; i += blockDim.x) {
      int c = i / N0, kx = i - c * N0;
      int b = b0 + c;
      if (b >= M) continue;
      int ky = b / N2, kz = b - ky * N2;
      int ax = min(kx, N0 - kx), ay = min(ky, N1 - ky), az = min(kz, N2 - kz);
      buf[i] = buf[i] * ghat[((size_t)ax * h1 + ay) * h2 + az];
    }
    __syncthreads();
    lds_fft<T, XStage<T>::value>(buf, N0, C, N0, 1, tw, twL, true);
  }
  for (int i = threadIdx.x; i < C * n0; i += blockDim.x) {
    int x = i / C, c = i - x * C;
    if (b0 + c < M) base[(size_t)x * M + b0 + c] = buf[c * N0 + x];
  }
}

template <typename T> static int xline_lines(int N0) {
  int C = (int)(LDS_BUDGET / (sizeof(cx<T>) * (size_t)N0));
  C = std::max(1, std::min(C, 16));
  // butterflies per thread per stage must fit the register staging
  while (C > 1 && (size_t)C * N0 / 2 > (size_t)XStage<T>::value * FFT_THREADS) C /= 2;
  return C;
}

template <typename T> void launch_conv(const DevGrid<T> &g, hipStream_t s) {
  const int n0 = g.n[0], n1 = g.n[1], n2 = g.n[2];
  const int N0 = g.N[0], N1 = g.N[1], N2 = g.N[2];
  size_t plane_lds = sizeof(cx<T>) * (size_t)N1 * N2;
  hipLaunchKernelGGL(plane_fwd_kernel<T>, dim3(n0, 8), dim3(FFT_THREADS), plane_lds, s, g.phys, g.spec, n0, n1, n2, N1,
                     N2, g.tw, g.twL);
  int C = xline_lines<T>(N0);
  int nb = (N1 * N2 + C - 1) / C;
  hipLaunchKernelGGL(xline_kernel<T>, dim3(nb, 8), dim3(FFT_THREADS), sizeof(cx<T>) * (size_t)C * N0, s, g.spec, n0,
                     N0, N1, N2, C, g.ghat, g.tw, g.twL, 0);
  hipLaunchKernelGGL(plane_inv_kernel<T>, dim3(n0, 8), dim3(FFT_THREADS), plane_lds, s, g.spec, g.phys, n0, n1, n2, N1,
                     N2, g.tw, g.twL);
}
template void launch_conv<float>(const DevGrid<float> &, hipStream_t);
template void launch_conv<double>(const DevGrid<double> &, hipStream_t);

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
  size_t plane_lds = sizeof(cx<double>) * (size_t)N1 * N2;
  hipLaunchKernelGGL(plane_fwd_kernel<double>, dim3(N0, 1), dim3(FFT_THREADS), plane_lds, s, full, spec, N0, N1, N2, N1,
                     N2, tw64, twL);
  int C = xline_lines<double>(N0);
  int nb = (N1 * N2 + C - 1) / C;
  hipLaunchKernelGGL(xline_kernel<double>, dim3(nb, 1), dim3(FFT_THREADS), sizeof(cx<double>) * (size_t)C * N0, s, spec,
                     N0, N0, N1, N2, C, (const cx<double> *)nullptr, tw64, twL, 1);
  hipLaunchKernelGGL(extract_octant, dim3(256), dim3(256), 0, s, spec, ghat64, ghat32, N0, N1, N2);
  e = hipGetLastError();
  hipError_t e2 = hipStreamSynchronize(s);
  hipFree(full);
  hipFree(spec);
  return e != hipSuccess ? e : e2;
}

}  // namespace scabs
