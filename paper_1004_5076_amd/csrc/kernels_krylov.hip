// FP64 reductions and vector updates of the GMRES solver (complex vectors,
// interleaved): multi-vector conjugate dots, basis updates, norms.
#include "device_common.h"

namespace scabs {

constexpr int KR_THREADS = 256;

__device__ inline double block_sum(double v, double *sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); i++) r += sh[i];
  __syncthreads();
  return r;
}

// part[j * nb + b] = sum over rows of chunk b of conj(V_j) w (V in FP64, or
// FP32 for the basis of the single-precision inner solves; FP64 sums)
template <typename VT>
__global__ void __launch_bounds__(KR_THREADS)
dots_partial(const cx<VT> *__restrict__ V, int64_t ldv, const cx<double> *__restrict__ w, int64_t N,
             cx<double> *__restrict__ part) {
  __shared__ double sh[2][KR_THREADS / 64];
  const int j = blockIdx.y, nb = gridDim.x;
  const cx<VT> *v = V + (size_t)j * ldv;
  double re = 0, im = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)nb * blockDim.x) {
    const cx<VT> a = v[i];
    const cx<double> b = w[i];
    re += (double)a.x * b.x + (double)a.y * b.y;
    im += (double)a.x * b.y - (double)a.y * b.x;
  }
  re = block_sum(re, sh[0]);
  im = block_sum(im, sh[1]);
  if (threadIdx.x == 0) part[(size_t)j * nb + blockIdx.x] = {re, im};
}

// out[j] (+)= sum_b part[j * nb + b]
__global__ void reduce_parts(const cx<double> *__restrict__ part, int nb, int jn, cx<double> *out, int accumulate) {
  __shared__ double sh[2][KR_THREADS / 64];
  const int j = blockIdx.x;
  if (j >= jn) return;
  double re = 0, im = 0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    re += part[(size_t)j * nb + b].x;
    im += part[(size_t)j * nb + b].y;
  }
  re = block_sum(re, sh[0]);
  im = block_sum(im, sh[1]);
  if (threadIdx.x == 0) {
    if (accumulate) {
      out[j].x += re;
      out[j].y += im;
    } else {
      out[j] = {re, im};
    }
  }
}

// w += sgn * sum_{j < jn} V_j c_j
template <typename VT>
__global__ void __launch_bounds__(KR_THREADS)
basis_update(cx<double> *__restrict__ w, const cx<VT> *__restrict__ V, int64_t ldv, int jn,
             const cx<double> *__restrict__ c, int64_t N, double sgn) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    cx<double> acc = w[i];
    for (int j = 0; j < jn; j++) {
      const cx<VT> v = V[(size_t)j * ldv + i];
      const cx<double> t = cx<double>{(double)v.x, (double)v.y} * c[j];
      acc.x += sgn * t.x;
      acc.y += sgn * t.y;
    }
    w[i] = acc;
  }
}

__global__ void __launch_bounds__(KR_THREADS)
norm2_partial(const cx<double> *__restrict__ w, int64_t N, double *__restrict__ part) {
  __shared__ double sh[KR_THREADS / 64];
  double s = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    cx<double> a = w[i];
    s += a.x * a.x + a.y * a.y;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void reduce_norm(const double *__restrict__ part, int nb, double *out) {
  __shared__ double sh[KR_THREADS / 64];
  double s = 0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) s += part[b];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) *out = sqrt(s);
}

// dst = src / *nrm (nrm > 0), else dst = 0; dst in FP64 or FP32
template <typename VT>
__global__ void scale_by_inv(cx<VT> *__restrict__ dst, const cx<double> *__restrict__ src, const double *nrm,
                             int64_t N) {
  const double n = *nrm;
  const double s = n > 0 ? 1.0 / n : 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = {(VT)(src[i].x * s), (VT)(src[i].y * s)};
}

// FP32 basis vectors -> FP64 operator input
__global__ void widen_kernel(const cx<float> *__restrict__ src, cx<double> *__restrict__ dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = {(double)src[i].x, (double)src[i].y};
}

// r = b - r (in place on r, which holds A x)
__global__ void residual_kernel(const cx<double> *__restrict__ b, cx<double> *__restrict__ r, int64_t N) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
    r[i] = b[i] - r[i];
}

__global__ void axpy_kernel(cx<double> *__restrict__ x, const cx<double> *__restrict__ d, int64_t N) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
    x[i] += d[i];
}

__global__ void finite_check(const double *__restrict__ v, int64_t n, int *bad) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (!isfinite(v[i])) *bad = 1;
}

// ---------------------------------------------------------------------------
static int reduce_blocks(int64_t N) {
  int64_t b = (N + KR_THREADS - 1) / KR_THREADS;
  return (int)(b < 1024 ? (b < 1 ? 1 : b) : 1024);
}

template <typename VT>
void kr_dots(const cx<VT> *V, int64_t ldv, int jn, const cx<double> *w, int64_t N, cx<double> *part,
             cx<double> *out, int accumulate, hipStream_t s) {
  int nb = reduce_blocks(N);
  if (nb > 256) nb = 256;
  hipLaunchKernelGGL(dots_partial<VT>, dim3(nb, jn), dim3(KR_THREADS), 0, s, V, ldv, w, N, part);
  hipLaunchKernelGGL(reduce_parts, dim3(jn), dim3(KR_THREADS), 0, s, part, nb, jn, out, accumulate);
}
template <typename VT>
void kr_update(cx<double> *w, const cx<VT> *V, int64_t ldv, int jn, const cx<double> *c, int64_t N, double sgn,
               hipStream_t s) {
  hipLaunchKernelGGL(basis_update<VT>, dim3(reduce_blocks(N)), dim3(KR_THREADS), 0, s, w, V, ldv, jn, c, N, sgn);
}
template <typename VT> void kr_scale(cx<VT> *dst, const cx<double> *src, const double *nrm, int64_t N, hipStream_t s) {
  hipLaunchKernelGGL(scale_by_inv<VT>, dim3(reduce_blocks(N)), dim3(KR_THREADS), 0, s, dst, src, nrm, N);
}
template void kr_dots<double>(const cx<double> *, int64_t, int, const cx<double> *, int64_t, cx<double> *,
                              cx<double> *, int, hipStream_t);
template void kr_dots<float>(const cx<float> *, int64_t, int, const cx<double> *, int64_t, cx<double> *,
                             cx<double> *, int, hipStream_t);
template void kr_update<double>(cx<double> *, const cx<double> *, int64_t, int, const cx<double> *, int64_t, double,
                                hipStream_t);
template void kr_update<float>(cx<double> *, const cx<float> *, int64_t, int, const cx<double> *, int64_t, double,
                               hipStream_t);
template void kr_scale<double>(cx<double> *, const cx<double> *, const double *, int64_t, hipStream_t);
template void kr_scale<float>(cx<float> *, const cx<double> *, const double *, int64_t, hipStream_t);
void kr_widen(const cx<float> *src, cx<double> *dst, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(widen_kernel, dim3(reduce_blocks(n)), dim3(KR_THREADS), 0, s, src, dst, n);
}
void kr_norm(const cx<double> *w, int64_t N, double *part, double *out, hipStream_t s) {
  int nb = reduce_blocks(N);
  hipLaunchKernelGGL(norm2_partial, dim3(nb), dim3(KR_THREADS), 0, s, w, N, part);
  hipLaunchKernelGGL(reduce_norm, dim3(1), dim3(KR_THREADS), 0, s, part, nb, out);
}
void kr_residual(const cx<double> *b, cx<double> *r, int64_t N, hipStream_t s) {
  hipLaunchKernelGGL(residual_kernel, dim3(reduce_blocks(N)), dim3(KR_THREADS), 0, s, b, r, N);
}
void kr_axpy(cx<double> *x, const cx<double> *d, int64_t N, hipStream_t s) {
  hipLaunchKernelGGL(axpy_kernel, dim3(reduce_blocks(N)), dim3(KR_THREADS), 0, s, x, d, N);
}
void kr_finite(const double *v, int64_t n, int *bad, hipStream_t s) {
  hipLaunchKernelGGL(finite_check, dim3(reduce_blocks(n)), dim3(KR_THREADS), 0, s, v, n, bad);
}

}  // namespace scabs
