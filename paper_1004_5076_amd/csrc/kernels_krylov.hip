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
// FP32 for the basis of the single-precision inner solves; FP64 sums).  Each
// work-group takes KD_J consecutive columns, so w is read once per KD_J.
constexpr int KD_J = 8;
template <typename VT>
__global__ void __launch_bounds__(KR_THREADS)
dots_partial(const cx<VT> *__restrict__ V, int64_t ldv, int jn, const cx<double> *__restrict__ w, int64_t N,
             cx<double> *__restrict__ part) {
  __shared__ double sh[2 * KD_J][KR_THREADS / 64];
  const int j0 = blockIdx.y * KD_J, nb = gridDim.x;
  const int nj = min(KD_J, jn - j0);
  double re[KD_J], im[KD_J];
#pragma unroll
  for (int q = 0; q < KD_J; q++) re[q] = im[q] = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)nb * blockDim.x) {
    const cx<double> b = w[i];
#pragma unroll
    for (int q = 0; q < KD_J; q++) {
      if (q < nj) {
        const cx<VT> a = V[(size_t)(j0 + q) * ldv + i];
        re[q] += (double)a.x * b.x + (double)a.y * b.y;
        im[q] += (double)a.x * b.y - (double)a.y * b.x;
      }
    }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < KD_J; q++) {
    for (int o = 32; o > 0; o >>= 1) {
      re[q] += __shfl_xor(re[q], o, 64);
      im[q] += __shfl_xor(im[q], o, 64);
    }
    if (lane == 0) {
      sh[2 * q][wid] = re[q];
      sh[2 * q + 1][wid] = im[q];
    }
  }
  __syncthreads();
  if (threadIdx.x < nj) {
    const int q = threadIdx.x;
    double r = 0, m = 0;
    for (int k = 0; k < (int)(blockDim.x >> 6); k++) {
      r += sh[2 * q][k];
      m += sh[2 * q + 1][k];
    }
    part[(size_t)(j0 + q) * nb + blockIdx.x] = {r, m};
  }
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
// One Gram-Schmidt pass for the systems of a batch in three launches (the
// systems in blockIdx.z), system b's vectors at offset b N:
//   (1) per row chunk and group of KD_J columns: conj(V_j) w partial sums,
//       and (first pass) ||w||^2 partials;
//   (2) the partials summed in a fixed order into h_j (and ||w||);
//   (3) w -= sum_j V_j h_j with ||w||^2 partials of the result, summed by (4).
// ---------------------------------------------------------------------------
constexpr int OG_BLOCKS = 64;   // row chunks of the dot pass (several rows per thread)
static_assert(KD_J == 8, "the wave reduction of og_dots is written for 8 columns (16 values)");
template <typename VT>
__global__ void __launch_bounds__(KR_THREADS)
og_dots(const cx<VT> *__restrict__ V, int64_t ldv, int jn, const cx<double> *__restrict__ w, int64_t N, KrRun run,
        int with_norm, cx<double> *__restrict__ part) {
  __shared__ double sh[2 * KD_J + 1][KR_THREADS / 64];
  const int b = run.b[blockIdx.z];
  const int jg = blockIdx.y, j0 = jg * KD_J, nblk = gridDim.x;
  const int nj = min(KD_J, jn - j0);
  const cx<VT> *Vb = V + (size_t)b * N;
  const cx<double> *wb = w + (size_t)b * N;
  // columns past the group's last one repeat it (their sums are never stored),
  // so the loop has no per-column branches
  const cx<VT> *Vq[KD_J];
#pragma unroll
  for (int q = 0; q < KD_J; q++) Vq[q] = Vb + (size_t)(j0 + min(q, nj - 1)) * ldv;
  double v[2 * KD_J], nn = 0;
#pragma unroll
  for (int q = 0; q < 2 * KD_J; q++) v[q] = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)nblk * blockDim.x) {
    const cx<double> x = wb[i];
    nn = fma(x.x, x.x, nn);
    nn = fma(x.y, x.y, nn);
#pragma unroll
    for (int q = 0; q < KD_J; q++) {
      const cx<VT> a = Vq[q][i];
      v[2 * q] = fma((double)a.x, x.x, v[2 * q]);
      v[2 * q] = fma((double)a.y, x.y, v[2 * q]);
      v[2 * q + 1] = fma((double)a.x, x.y, v[2 * q + 1]);
      v[2 * q + 1] = fma(-(double)a.y, x.x, v[2 * q + 1]);
    }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  // lane L ends with the wave sum of value (L >> 2) & 15
  const double t = wsum16_scatter(v);
  if ((lane & 3) == 0) sh[(lane >> 2) & 15][wid] = t;
  for (int o = 32; o > 0; o >>= 1) nn += __shfl_xor(nn, o, 64);
  if (lane == 0) sh[2 * KD_J][wid] = nn;
  __syncthreads();
  // part[(z (jn + 1) + j) nblk + blk]; column jn holds ||w||^2
  cx<double> *pz = part + (size_t)blockIdx.z * (jn + 1) * nblk;
  if (threadIdx.x < nj) {
    const int q = threadIdx.x;
    double r = 0, m = 0;
    for (int k = 0; k < (int)(blockDim.x >> 6); k++) {
      r += sh[2 * q][k];
      m += sh[2 * q + 1][k];
    }
    pz[(size_t)(j0 + q) * nblk + blockIdx.x] = {r, m};
  }
  if (with_norm && jg == 0 && threadIdx.x == 64) {
    double r = 0;
    for (int k = 0; k < (int)(blockDim.x >> 6); k++) r += sh[2 * KD_J][k];
    pz[(size_t)jn * nblk + blockIdx.x] = {r, 0.0};
  }
}

// h[b][j] (j < jn) into hcol + b hstride + hoff, and ||w_b|| into nrm_before[b]
__global__ void og_reduce(const cx<double> *__restrict__ part, int nblk, int jn, KrRun run, int with_norm,
                          cx<double> *hcol, int64_t hstride, int64_t hoff, double *nrm_before) {
  __shared__ double sh[2][KR_THREADS / 64];
  const int j = blockIdx.x, b = run.b[blockIdx.y];
  if (j == jn && !with_norm) return;
  const cx<double> *pz = part + ((size_t)blockIdx.y * (jn + 1) + j) * nblk;
  double re = 0, im = 0;
  for (int k = threadIdx.x; k < nblk; k += blockDim.x) {
    re += pz[k].x;
    im += pz[k].y;
  }
  re = block_sum(re, sh[0]);
  im = block_sum(im, sh[1]);
  if (threadIdx.x == 0) {
    if (j < jn)
      hcol[b * hstride + hoff + j] = {re, im};
    else
      nrm_before[b] = sqrt(re);
  }
}

// w_b -= sum_{j < jn} V_j h_j, and per block the sum of |w_b|^2 of the result
template <typename VT>
__global__ void __launch_bounds__(KR_THREADS)
og_update(cx<double> *__restrict__ w, const cx<VT> *__restrict__ V, int64_t ldv, int jn,
          const cx<double> *__restrict__ hcol, int64_t hstride, int64_t hoff, int64_t N, KrRun run,
          double *__restrict__ npart) {
  __shared__ double sh[KR_THREADS / 64];
  const int b = run.b[blockIdx.y];
  const cx<VT> *Vb = V + (size_t)b * N;
  cx<double> *wb = w + (size_t)b * N;
  const cx<double> *h = hcol + b * hstride + hoff;
  double nn = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    cx<double> acc = wb[i];
    int j = 0;
    for (; j + 4 <= jn; j += 4) {   // four basis loads in flight
      cx<VT> v[4];
#pragma unroll
      for (int u = 0; u < 4; u++) v[u] = Vb[(size_t)(j + u) * ldv + i];
#pragma unroll
      for (int u = 0; u < 4; u++) acc -= cx<double>{(double)v[u].x, (double)v[u].y} * h[j + u];
    }
    for (; j < jn; j++) {
      const cx<VT> v = Vb[(size_t)j * ldv + i];
      acc -= cx<double>{(double)v.x, (double)v.y} * h[j];
    }
    wb[i] = acc;
    nn += acc.x * acc.x + acc.y * acc.y;
  }
  nn = block_sum(nn, sh);
  if (threadIdx.x == 0) npart[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = nn;
}

__global__ void og_norm(const double *__restrict__ npart, int nblk, KrRun run, double *nrm) {
  __shared__ double sh[KR_THREADS / 64];
  double s = 0;
  for (int k = threadIdx.x; k < nblk; k += blockDim.x) s += npart[(size_t)blockIdx.x * nblk + k];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) nrm[run.b[blockIdx.x]] = sqrt(s);
}

// V_dst[b] = w_b / nrm[b] for the systems of the run
template <typename VT>
__global__ void og_scale(cx<VT> *__restrict__ Vdst, const cx<double> *__restrict__ w, const double *nrm, int64_t N,
                         KrRun run) {
  const int b = run.b[blockIdx.y];
  const double n = nrm[b];
  const double sc = n > 0 ? 1.0 / n : 0.0;
  cx<VT> *d = Vdst + (size_t)b * N;
  const cx<double> *src = w + (size_t)b * N;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
    d[i] = {(VT)(src[i].x * sc), (VT)(src[i].y * sc)};
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
  hipLaunchKernelGGL(dots_partial<VT>, dim3(nb, (jn + KD_J - 1) / KD_J), dim3(KR_THREADS), 0, s, V, ldv, jn, w, N,
                     part);
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
template <typename VT>
void kr_ortho_pass(const cx<VT> *V, int64_t ldv, int jn, cx<double> *w, int64_t N, const KrRun &run, int with_norm,
                   cx<double> *part, double *npart, cx<double> *hcol, int64_t hstride, int64_t hoff,
                   double *nrm_before, double *nrm_after, hipStream_t s) {
  if (run.n == 0) return;
  const int ub = reduce_blocks(N);
  hipLaunchKernelGGL(og_dots<VT>, dim3(OG_BLOCKS, (jn + KD_J - 1) / KD_J, run.n), dim3(KR_THREADS), 0, s, V, ldv, jn,
                     (const cx<double> *)w, N, run, with_norm, part);
  hipLaunchKernelGGL(og_reduce, dim3(jn + 1, run.n), dim3(KR_THREADS), 0, s, (const cx<double> *)part, OG_BLOCKS, jn,
                     run, with_norm, hcol, hstride, hoff, nrm_before);
  hipLaunchKernelGGL(og_update<VT>, dim3(ub, run.n), dim3(KR_THREADS), 0, s, w, V, ldv, jn,
                     (const cx<double> *)hcol, hstride, hoff, N, run, npart);
  hipLaunchKernelGGL(og_norm, dim3(run.n), dim3(KR_THREADS), 0, s, (const double *)npart, ub, run, nrm_after);
}
template <typename VT>
void kr_scale_run(cx<VT> *Vdst, const cx<double> *w, const double *nrm, int64_t N, const KrRun &run, hipStream_t s) {
  if (run.n == 0) return;
  hipLaunchKernelGGL(og_scale<VT>, dim3(reduce_blocks(N), run.n), dim3(KR_THREADS), 0, s, Vdst, w, nrm, N, run);
}
// Read-back of one Arnoldi step into mapped, coherent host memory: the norm
// entries [0, nnrm) and, per column block k < ncol (stride entries apart,
// after the norms), its first rows entries; then, once every thread's stores
// are visible system-wide, flag = seq.  One work-group.
__global__ void kr_publish_kernel(const cx<double> *__restrict__ src, cx<double> *dst, int nnrm, int ncol,
                                  int stride, int rows, unsigned *flag, unsigned seq) {
  for (int t = threadIdx.x; t < nnrm; t += blockDim.x) dst[t] = src[t];
  const int total = ncol * rows;
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int k = t / rows, i = t - k * rows;
    const size_t at = (size_t)nnrm + (size_t)k * stride + i;
    dst[at] = src[at];
  }
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(flag, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}
void kr_publish(const cx<double> *src, cx<double> *dst, int nnrm, int ncol, int stride, int rows, unsigned *flag,
                unsigned seq, hipStream_t s) {
  hipLaunchKernelGGL(kr_publish_kernel, dim3(1), dim3(256), 0, s, src, dst, nnrm, ncol, stride, rows, flag, seq);
}

size_t kr_ortho_part_entries(int jn_max, int nsys) { return (size_t)OG_BLOCKS * (jn_max + 1) * nsys; }
size_t kr_ortho_npart_entries(int64_t N, int nsys) { return (size_t)reduce_blocks(N) * nsys; }
template void kr_ortho_pass<float>(const cx<float> *, int64_t, int, cx<double> *, int64_t, const KrRun &, int,
                                   cx<double> *, double *, cx<double> *, int64_t, int64_t, double *, double *,
                                   hipStream_t);
template void kr_ortho_pass<double>(const cx<double> *, int64_t, int, cx<double> *, int64_t, const KrRun &, int,
                                    cx<double> *, double *, cx<double> *, int64_t, int64_t, double *, double *,
                                    hipStream_t);
template void kr_scale_run<float>(cx<float> *, const cx<double> *, const double *, int64_t, const KrRun &,
                                  hipStream_t);
template void kr_scale_run<double>(cx<double> *, const cx<double> *, const double *, int64_t, const KrRun &,
                                   hipStream_t);

// zero fill by a kernel (unlike a memset node it may sit in a captured graph)
__global__ void zero_kernel(uint32_t *__restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}
void kr_zero(void *p, size_t bytes, hipStream_t s) {
  const int64_t n = (int64_t)(bytes / sizeof(uint32_t));
  if (n > 0) hipLaunchKernelGGL(zero_kernel, dim3(reduce_blocks(n)), dim3(KR_THREADS), 0, s, (uint32_t *)p, n);
}
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
