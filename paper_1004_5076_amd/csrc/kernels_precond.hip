// Restricted additive Schwarz preconditioner built from the exact near-field
// matrix: for every box cluster the dense near-field block on its extended
// (overlapping) unknown set is assembled in FP64, inverted by Gauss-Jordan
// elimination with partial pivoting, and the rows of its core unknowns are
// kept (FP32).  Applying it is one dense block product per cluster.
#include "device_common.h"
#include "kernels.h"

namespace scabs {

// exact values per CSR entry: L_e, K_e, L_i, K_i, Lrot_e, Krot_e, Lsig_i, Ksig_i
__global__ void exact_assemble_kernel(int64_t nnz, const int64_t *__restrict__ cptr, const int *__restrict__ cpair,
                                      const uint8_t *__restrict__ cij, const cx<double> *__restrict__ blocks,
                                      cx<double> *__restrict__ X8) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
    cx<double> acc[8];
    for (int t = 0; t < 8; t++) acc[t] = {0.0, 0.0};
    for (int64_t c = cptr[e]; c < cptr[e + 1]; c++) {
      const cx<double> *b = blocks + (size_t)cpair[c] * 72 + cij[c];
      for (int t = 0; t < 8; t++) acc[t] += b[t * 9];
    }
    for (int t = 0; t < 8; t++) X8[8 * e + t] = acc[t];
  }
}

void launch_exact_assemble(int64_t nnz, const int64_t *cptr, const int *cpair, const uint8_t *cij,
                           const cx<double> *blocks, cx<double> *X8, hipStream_t s) {
  hipLaunchKernelGGL(exact_assemble_kernel, dim3(2048), dim3(256), 0, s, nnz, cptr, cpair, cij, blocks, X8);
}

// Near-field matrix entry (row slot a, column slot b).  Rows: E (eq1/eq3),
// H (eq2/eq13), eq14; per-edge currents J_e, J_i, M with J_i = -J_e on L edges.
__device__ cx<double> near_entry(const PrecondArgs &p, int a, int b) {
  const int n = p.slot_edge[a], r = p.slot_kind[a];
  const int m = p.slot_edge[b], cc = p.slot_kind[b];
  cx<double> X[8];
  for (int t = 0; t < 8; t++) X[t] = {0.0, 0.0};
  {
    int64_t lo = p.rowptr[n], hi = p.rowptr[n + 1];
    while (lo < hi) {
      int64_t mid = (lo + hi) >> 1;
      if (p.col[mid] < m) lo = mid + 1;
      else hi = mid;
    }
    if (lo < p.rowptr[n + 1] && p.col[lo] == m)
      for (int t = 0; t < 8; t++) X[t] = p.X8[8 * lo + t];
  }
  double gram = 0, nx = 0, srot = 0, snx = 0;
  for (int64_t k = p.lptr[n]; k < p.lptr[n + 1]; k++)
    if (p.lcol[k] == m) {
      gram = p.lval[4 * k];
      nx = p.lval[4 * k + 1];
      srot = p.lval[4 * k + 2];
      snx = p.lval[4 * k + 3];
    }
  const double Ze = p.Ze, Zi = p.Zi;
  cx<double> cJe, cJi, cM;
  if (r == 0) {
    cJe = X[0] * (-Ze);
    cJi = X[2] * Zi;
    cM = X[1] + X[3];
  } else if (r == 1) {
    cJe = -X[1] - cx<double>{0.5 * nx, 0.0};
    cJi = X[3] - cx<double>{0.5 * nx, 0.0};
    cM = -(X[0] * (1.0 / Ze) + X[2] * (1.0 / Zi));
    if (p.isR[n]) {
      cJe -= X[4] * Ze;
      cM += X[5] + cx<double>{0.5 * srot, 0.0};
    }
  } else {
    cJe = {gram, 0.0};
    cJi = X[6] * Zi + cx<double>{gram, 0.0};
    cM = X[7] - cx<double>{0.5 * snx, 0.0};
  }
  if (p.isR[m]) return cc == 0 ? cJe : (cc == 2 ? cJi : cM);
  return cc == 0 ? cJe - cJi : cM;
}

// Dense cluster blocks, assembled in FP64 and stored in FP32 for the
// inversion (the preconditioner only needs an approximate inverse; its rows
// are kept in FP32 anyway).
__global__ void block_assemble_kernel(PrecondArgs p) {
  const int c = blockIdx.y;
  const int64_t e0 = p.ext_ptr[c];
  const int ne = (int)(p.ext_ptr[c + 1] - e0);
  cx<float> *A = p.A + p.a_off[c];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (int64_t)ne * ne;
       i += (int64_t)gridDim.x * blockDim.x) {
    int a = (int)(i / ne), b = (int)(i - (int64_t)a * ne);
    const cx<double> v = near_entry(p, p.ext_slot[e0 + a], p.ext_slot[e0 + b]);
    A[i] = {(float)v.x, (float)v.y};
  }
}

// In-place inverse of each cluster block (row-major n x n, FP32) by
// Gauss-Jordan elimination with partial pivoting; the row interchanges are
// undone as column interchanges at the end.  One work-group per cluster.
constexpr int GJ_THREADS = 1024;
constexpr int GJ_MAXN = 4096;   // largest cluster (extended set) the inversion handles

__global__ void __launch_bounds__(GJ_THREADS) gauss_jordan_kernel(cx<float> *Ablocks, const int64_t *a_off,
                                                                  const int64_t *ext_ptr, int *piv_all, int *status) {
  const int c = blockIdx.x;
  const int n = (int)(ext_ptr[c + 1] - ext_ptr[c]);
  cx<float> *A = Ablocks + a_off[c];
  int *piv = piv_all + ext_ptr[c];
  __shared__ cx<float> rowk[GJ_MAXN];
  __shared__ cx<float> colk[GJ_MAXN];
  __shared__ float red_v[GJ_THREADS / 64];
  __shared__ int red_i[GJ_THREADS / 64];
  __shared__ int s_p;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = GJ_THREADS / 64;
  for (int k = 0; k < n; k++) {
    // pivot: largest |A[i][k]|, i >= k
    float best = -1.0f;
    int bi = k;
    for (int i = k + tid; i < n; i += blockDim.x) {
      cx<float> v = A[(size_t)i * n + k];
      float m = v.x * v.x + v.y * v.y;
      if (m > best) {
        best = m;
        bi = i;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      float ov = __shfl_xor(best, o, 64);
      int oi = __shfl_xor(bi, o, 64);
      if (ov > best || (ov == best && oi < bi)) {
        best = ov;
        bi = oi;
      }
    }
    if (lane == 0) {
      red_v[wid] = best;
      red_i[wid] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      float bv = red_v[0];
      int bb = red_i[0];
      for (int w = 1; w < nw; w++)
        if (red_v[w] > bv || (red_v[w] == bv && red_i[w] < bb)) {
          bv = red_v[w];
          bb = red_i[w];
        }
      s_p = bb;
      piv[k] = bb;
      if (!(bv > 0)) *status = 1;   // singular block
    }
    __syncthreads();
    const int pr = s_p;
    if (pr != k)
      for (int j = tid; j < n; j += blockDim.x) {
        cx<float> t = A[(size_t)k * n + j];
        A[(size_t)k * n + j] = A[(size_t)pr * n + j];
        A[(size_t)pr * n + j] = t;
      }
    __syncthreads();
    // pivot row scaled by 1/d, pivot column saved
    const cx<float> d = A[(size_t)k * n + k];
    const float dn = d.x * d.x + d.y * d.y;
    const cx<float> inv = dn > 0 ? cx<float>{d.x / dn, -d.y / dn} : cx<float>{0.0f, 0.0f};
    for (int j = tid; j < n; j += blockDim.x) {
      cx<float> v = j == k ? cx<float>{1.0f, 0.0f} : A[(size_t)k * n + j];
      rowk[j] = v * inv;
      colk[j] = A[(size_t)j * n + k];
    }
    __syncthreads();
    for (int j = tid; j < n; j += blockDim.x) A[(size_t)k * n + j] = rowk[j];
    // every other row: one wave per row, lanes along the (contiguous) columns
    for (int i = wid; i < n; i += nw) {
      if (i == k) continue;
      const cx<float> f = colk[i];
      cx<float> *Ai = A + (size_t)i * n;
      for (int j = lane; j < n; j += 64) {
        if (j == k)
          Ai[j] = -(f * inv);
        else
          Ai[j] -= f * rowk[j];
      }
    }
    __syncthreads();
  }
  // undo row interchanges as column interchanges, last first
  for (int k = n - 1; k >= 0; k--) {
    const int pr = piv[k];
    if (pr != k)
      for (int i = tid; i < n; i += blockDim.x) {
        cx<float> t = A[(size_t)i * n + k];
        A[(size_t)i * n + k] = A[(size_t)i * n + pr];
        A[(size_t)i * n + pr] = t;
      }
    __syncthreads();
  }
}

// Stored rows: for ext column j of cluster c, Rt[j][i] = inverse[core_pos[i]][j]
// over the core rows i (column-major, column stride rt_stride(nc)), as FP16
// halves divided by the column's scale Rs = max |re|, |im| (1 for a zero
// column).  One wave per column: the maximum, then the scaled entries.
__global__ void __launch_bounds__(256)
extract_kernel(const cx<float> *Ablocks, const int64_t *a_off, const int64_t *ext_ptr, const int64_t *core_ptr,
               const int *core_pos, const int64_t *r_off, int nclust, uint32_t *Rt, float *Rs) {
  const int64_t col = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (col >= ext_ptr[nclust]) return;
  int lo = 0, hi = nclust;   // owning cluster: ext_ptr[c] <= col < ext_ptr[c + 1]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (ext_ptr[mid] <= col) lo = mid;
    else hi = mid;
  }
  const int c = lo;
  const int ne = (int)(ext_ptr[c + 1] - ext_ptr[c]);
  const int nc = (int)(core_ptr[c + 1] - core_ptr[c]);
  const int j = (int)(col - ext_ptr[c]);
  const cx<float> *A = Ablocks + a_off[c];
  const int *cp = core_pos + core_ptr[c];
  float m = 0;
  for (int i = lane; i < nc; i += 64) {
    const cx<float> v = A[(size_t)cp[i] * ne + j];
    m = fmaxf(m, fmaxf(fabsf(v.x), fabsf(v.y)));
  }
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  const float sc = m > 0 ? m : 1.0f, inv = 1.0f / sc;
  uint32_t *R = Rt + r_off[c] + (int64_t)j * rt_stride(nc);
  for (int i = lane; i < nc; i += 64) {
    const cx<float> v = A[(size_t)cp[i] * ne + j];
    R[i] = pack_h2(v.x * inv, v.y * inv);
  }
  if (lane == 0) Rs[col] = sc;
}

void launch_precond_build(const PrecondArgs &p, int max_ext, const int64_t *core_ptr, const int *core_pos,
                          const int64_t *r_off, uint32_t *Rt, float *Rs, int *piv, int *status, hipStream_t s) {
  (void)max_ext;
  hipLaunchKernelGGL(block_assemble_kernel, dim3(64, p.nc), dim3(256), 0, s, p);
  hipLaunchKernelGGL(gauss_jordan_kernel, dim3(p.nc), dim3(GJ_THREADS), 0, s, p.A, p.a_off, p.ext_ptr, piv, status);
  hipLaunchKernelGGL(extract_kernel, dim3((unsigned)((p.n_ext * 64 + 255) / 256)), dim3(256), 0, s,
                     (const cx<float> *)p.A, p.a_off, p.ext_ptr, core_ptr, core_pos, r_off, p.nc, Rt, Rs);
}
// y[core] = R_c x[ext] for every cluster; each unknown is in exactly one core.
// One work-group per item (cluster c, PA_ROWS core rows from row0): the ext
// columns split in PA_Q contiguous parts (coalesced reads of the
// column-major block), partial sums reduced in LDS in a fixed order.
constexpr int PA_ROWS = 64;
constexpr int PA_Q = 4;
constexpr int PA_THREADS = PA_ROWS * PA_Q;
constexpr int PA_CW = 512;   // ext columns staged per pass
__global__ void __launch_bounds__(PA_THREADS)
precond_apply_kernel(const int *__restrict__ items, const int64_t *__restrict__ ext_ptr,
                     const int *__restrict__ ext_slot, const int64_t *__restrict__ core_ptr,
                     const int *__restrict__ core_slot, const int64_t *__restrict__ r_off, PcStore pc,
                     const cx<double> *__restrict__ x, cx<double> *__restrict__ y) {
  __shared__ cx<double> xs[PA_CW];
  __shared__ cx<double> red[PA_Q][PA_ROWS];
  const int c = items[2 * blockIdx.x], i0 = items[2 * blockIdx.x + 1];
  const int64_t e0 = ext_ptr[c];
  const int ne = (int)(ext_ptr[c + 1] - e0);
  const int nc = (int)(core_ptr[c + 1] - core_ptr[c]);
  const uint32_t *R = pc.R + r_off[c];
  const int64_t ncp = rt_stride(nc);
  const int q = threadIdx.x / PA_ROWS, il = threadIdx.x - q * PA_ROWS;
  const int i = i0 + il;
  // four independent partial sums keep several loads in flight
  double pr[4] = {0, 0, 0, 0}, pi[4] = {0, 0, 0, 0};
  for (int cb = 0; cb < ne; cb += PA_CW) {
    const int cw = min(PA_CW, ne - cb);
    __syncthreads();   // the previous pass is done with xs
    // the column scales fold into the staged inputs
    for (int jj = threadIdx.x; jj < cw; jj += blockDim.x)
      xs[jj] = x[ext_slot[e0 + cb + jj]] * (double)pc.scale[e0 + cb + jj];
    __syncthreads();
    const int jb = (cw * q) / PA_Q, je = (cw * (q + 1)) / PA_Q;
    if (i < nc) {
      const uint32_t *Rc = R + (int64_t)cb * ncp + i;
      int j = jb;
      for (; j + 4 <= je; j += 4) {
#pragma unroll
        for (int u = 0; u < 4; u++) {
          const cx<float> rv = unpack_h2(Rc[(j + u) * ncp]);
          const cx<double> xv = xs[j + u];
          pr[u] += (double)rv.x * xv.x - (double)rv.y * xv.y;
          pi[u] += (double)rv.x * xv.y + (double)rv.y * xv.x;
        }
      }
      for (; j < je; j++) {
        const cx<float> rv = unpack_h2(Rc[j * ncp]);
        const cx<double> xv = xs[j];
        pr[0] += (double)rv.x * xv.x - (double)rv.y * xv.y;
        pi[0] += (double)rv.x * xv.y + (double)rv.y * xv.x;
      }
    }
  }
  red[q][il] = {(pr[0] + pr[1]) + (pr[2] + pr[3]), (pi[0] + pi[1]) + (pi[2] + pi[3])};
  __syncthreads();
  if (q == 0 && i < nc) {
    cx<double> t = red[0][il];
    for (int k = 1; k < PA_Q; k++) t += red[k][il];
    y[core_slot[core_ptr[c] + i]] = t;
  }
}

int precond_rows_per_item() { return PA_ROWS; }

void launch_precond_apply(int n_items, const int *items, const int64_t *ext_ptr, const int *ext_slot,
                          const int64_t *core_ptr, const int *core_slot, const int64_t *r_off, PcStore pc,
                          const cx<double> *x, cx<double> *y, int max_ext, hipStream_t s) {
  (void)max_ext;
  hipLaunchKernelGGL(precond_apply_kernel, dim3(n_items), dim3(PA_THREADS), 0, s, items, ext_ptr, ext_slot, core_ptr,
                     core_slot, r_off, pc, x, y);
}

// Batched apply in single precision for the FP32 inner solves: nb <= 8
// vectors per launch, their ext entries staged in LDS as FP32 (all lanes of a
// wave read the same column: broadcast), each coefficient read once for all
// of them, FP32 accumulation.  Inner solves stop at relative residuals of
// 1e-5 or more and an FP64 refinement follows, so the rounding of x and of
// the sums only perturbs the preconditioner, not the solution.
constexpr int PA32_Q = 8;
constexpr int PA32_THREADS = PA_ROWS * PA32_Q;
constexpr int PA32_CW = 512;   // ext columns staged per pass
template <int NB>
__global__ void __launch_bounds__(PA32_THREADS)
precond_apply32_kernel(const int *__restrict__ items, const int64_t *__restrict__ ext_ptr,
                       const int *__restrict__ ext_slot, const int64_t *__restrict__ core_ptr,
                       const int *__restrict__ core_slot, const int64_t *__restrict__ r_off, PcStore pc,
                       const cx<double> *__restrict__ x, cx<double> *__restrict__ y, int64_t N, int nb) {
  // the column staging and, after the last pass, the partial sums share LDS
  static_assert(PA32_Q * PA_ROWS <= PA32_CW, "partial sums must fit the staging buffer");
  __shared__ cx<float> xs[NB][PA32_CW];
  cx<float>(*red)[PA_ROWS][NB] = reinterpret_cast<cx<float>(*)[PA_ROWS][NB]>(&xs[0][0]);
  const int c = items[2 * blockIdx.x], i0 = items[2 * blockIdx.x + 1];
  const int64_t e0 = ext_ptr[c];
  const int ne = (int)(ext_ptr[c + 1] - e0);
  const int nc = (int)(core_ptr[c + 1] - core_ptr[c]);
  const uint32_t *R = pc.R + r_off[c];
  const int64_t ncp = rt_stride(nc);
  const int q = threadIdx.x / PA_ROWS, il = threadIdx.x - q * PA_ROWS;
  const int i = i0 + il;
  cx<float> acc[NB];
#pragma unroll
  for (int b = 0; b < NB; b++) acc[b] = czero<float>();
  for (int cb = 0; cb < ne; cb += PA32_CW) {
    const int cw = min(PA32_CW, ne - cb);
    __syncthreads();   // the previous pass is done with xs
    for (int t = threadIdx.x; t < nb * cw; t += blockDim.x) {
      const int b = t / cw, jj = t - b * cw;
      const cx<double> v = x[(size_t)b * N + ext_slot[e0 + cb + jj]];
      const float sc = pc.scale[e0 + cb + jj];   // the column scale folds into the staged input
      xs[b][jj] = {(float)v.x * sc, (float)v.y * sc};
    }
    __syncthreads();
    const int jb = (cw * q) / PA32_Q, je = (cw * (q + 1)) / PA32_Q;
    if (i < nc) {
      // eight coefficient loads in flight per thread
      const uint32_t *Rc = R + (int64_t)cb * ncp + i;
      int j = jb;
      for (; j + 8 <= je; j += 8) {
        cx<float> rv[8];
#pragma unroll
        for (int u = 0; u < 8; u++) rv[u] = unpack_h2(Rc[(j + u) * ncp]);
#pragma unroll
        for (int u = 0; u < 8; u++)
#pragma unroll
          for (int b = 0; b < NB; b++)
            if (b < nb) acc[b] += rv[u] * xs[b][j + u];
      }
      for (; j < je; j++) {
        const cx<float> rv = unpack_h2(Rc[j * ncp]);
#pragma unroll
        for (int b = 0; b < NB; b++)
          if (b < nb) acc[b] += rv * xs[b][j];
      }
    }
  }
  __syncthreads();   // every wave is done with xs
#pragma unroll
  for (int b = 0; b < NB; b++) red[q][il][b] = acc[b];
  __syncthreads();
  if (q == 0 && i < nc) {
    const int slot = core_slot[core_ptr[c] + i];
#pragma unroll
    for (int b = 0; b < NB; b++) {
      if (b >= nb) break;
      cx<float> t = red[0][il][b];
      for (int k = 1; k < PA32_Q; k++) t += red[k][il][b];
      y[(size_t)b * N + slot] = {(double)t.x, (double)t.y};
    }
  }
}

int precond_apply32_max_batch() { return 8; }

// m <= precond_apply32_max_batch() vectors; max_ext (largest extended set)
// sizes the LDS staging
void launch_precond_apply32(int n_items, const int *items, const int64_t *ext_ptr, const int *ext_slot,
                            const int64_t *core_ptr, const int *core_slot, const int64_t *r_off, PcStore pc,
                            const cx<double> *x, cx<double> *y, int64_t N, int m, int max_ext, hipStream_t s) {
  const size_t lds = 0;
  (void)max_ext;
  if (m == 1)
    hipLaunchKernelGGL((precond_apply32_kernel<1>), dim3(n_items), dim3(PA32_THREADS), lds, s, items, ext_ptr, ext_slot,
                       core_ptr, core_slot, r_off, pc, x, y, N, m);
  else if (m == 2)
    hipLaunchKernelGGL((precond_apply32_kernel<2>), dim3(n_items), dim3(PA32_THREADS), lds, s, items, ext_ptr, ext_slot,
                       core_ptr, core_slot, r_off, pc, x, y, N, m);
  else if (m <= 4)
    hipLaunchKernelGGL((precond_apply32_kernel<4>), dim3(n_items), dim3(PA32_THREADS), lds, s, items, ext_ptr, ext_slot,
                       core_ptr, core_slot, r_off, pc, x, y, N, m);
  else
    hipLaunchKernelGGL((precond_apply32_kernel<8>), dim3(n_items), dim3(PA32_THREADS), lds, s, items, ext_ptr, ext_slot,
                       core_ptr, core_slot, r_off, pc, x, y, N, m);
}

}  // namespace scabs
