// Restricted additive Schwarz preconditioner built from the exact near-field
// matrix: for every box cluster the dense near-field block on its extended
// (overlapping) unknown set is assembled in FP64, inverted by Gauss-Jordan
// elimination with partial pivoting, and the rows of its core unknowns are
// kept (FP32).  Applying it is one dense block product per cluster.
#include <algorithm>
#include <vector>

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

// In-place inverse of each cluster block (row-major n x n, FP32) by blocked
// Gauss-Jordan elimination with partial pivoting.  Panels of GJ_B columns:
// the panel kernel (one work-group per cluster) runs the GJ_B elimination
// steps on the panel columns of every row only (pivot search, full-row
// interchange, panel update); the b steps compose to T = I + (P - E) E^T
// with P the panel columns afterwards and E the pivot rows' unit vectors, so
// every other column v becomes v + (P - E) v_E: a rank-GJ_B update of the
// remaining columns (update kernel, 64 x 64 tiles of all clusters) from a
// snapshot of the pivot rows.  The row interchanges are undone as column
// interchanges at the end.
constexpr int GJ_THREADS = 1024;
constexpr int GJ_MAXN = PC_MAX_EXT;   // largest cluster (extended set) the inversion handles
constexpr int GJ_B = 32;        // panel width
constexpr int GJ_TILE = 64;     // update tile (rows x columns)

__global__ void __launch_bounds__(GJ_THREADS)
gj_panel_kernel(cx<float> *Ablocks, const int64_t *a_off, const int64_t *ext_ptr, int *piv_all, int *status,
                int k0) {
  const int c = blockIdx.x;
  const int n = (int)(ext_ptr[c + 1] - ext_ptr[c]);
  if (n <= k0) return;
  cx<float> *A = Ablocks + a_off[c];
  int *piv = piv_all + ext_ptr[c];
  const int kb = min(k0 + GJ_B, n), bw = kb - k0;
  __shared__ cx<float> colk[GJ_MAXN];
  __shared__ cx<float> rowp[GJ_B];
  __shared__ float red_v[GJ_THREADS / 64];
  __shared__ int red_i[GJ_THREADS / 64];
  __shared__ int s_p;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = GJ_THREADS / 64;
  const FastDiv dbw = make_fastdiv(bw);
  for (int k = k0; k < kb; k++) {
    // pivot: largest |A[i][k]|, i >= k
    float best = -1.0f;
    int bi = k;
    for (int i = k + tid; i < n; i += blockDim.x) {
      const cx<float> v = A[(size_t)i * n + k];
      const float m = v.x * v.x + v.y * v.y;
      if (m > best) {
        best = m;
        bi = i;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const float ov = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
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
    if (pr != k)   // whole rows: the deferred update reads the pivot rows
      for (int j = tid; j < n; j += blockDim.x) {
        const cx<float> t = A[(size_t)k * n + j];
        A[(size_t)k * n + j] = A[(size_t)pr * n + j];
        A[(size_t)pr * n + j] = t;
      }
    __syncthreads();
    const cx<float> d = A[(size_t)k * n + k];
    const float dn = d.x * d.x + d.y * d.y;
    const cx<float> inv = dn > 0 ? cx<float>{d.x / dn, -d.y / dn} : cx<float>{0.0f, 0.0f};
    for (int q = tid; q < bw; q += blockDim.x)
      rowp[q] = (k0 + q == k ? cx<float>{1.0f, 0.0f} : A[(size_t)k * n + k0 + q]) * inv;
    for (int i = tid; i < n; i += blockDim.x) colk[i] = A[(size_t)i * n + k];
    __syncthreads();
    // panel columns of every row (the pivot row takes the scaled row)
    for (int idx = tid; idx < n * bw; idx += blockDim.x) {
      const int i = fdiv(idx, dbw), q = idx - i * bw, j = k0 + q;
      cx<float> *a = A + (size_t)i * n + j;
      if (i == k)
        *a = rowp[q];
      else
        *a = (j == k ? czero<float>() : *a) - colk[i] * rowp[q];
    }
    __syncthreads();
  }
}

// snapshot of the panel's pivot rows: tmp[q][j] = A[k0 + q][j]
__global__ void gj_pivot_rows_kernel(const cx<float> *Ablocks, const int64_t *a_off, const int64_t *ext_ptr,
                                     cx<float> *tmp_all, int k0) {
  const int c = blockIdx.y;
  const int n = (int)(ext_ptr[c + 1] - ext_ptr[c]);
  if (n <= k0) return;
  const int bw = min(GJ_B, n - k0);
  const cx<float> *A = Ablocks + a_off[c] + (size_t)k0 * n;
  cx<float> *tmp = tmp_all + (size_t)GJ_B * ext_ptr[c];
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < (int64_t)bw * n;
       idx += (int64_t)gridDim.x * blockDim.x)
    tmp[idx] = A[idx];
}

// A[i][j] += sum_q (P - E)[i][q] tmp[q][j] for every j outside the panel;
// work-group = (cluster, 64 x 64 tile) from the per-panel tile prefix sums
__global__ void __launch_bounds__(256)
gj_update_kernel(cx<float> *Ablocks, const int64_t *a_off, const int64_t *ext_ptr, const cx<float> *tmp_all,
                 const int *tiles, int nclust, int k0) {
  __shared__ cx<float> sP[GJ_TILE][GJ_B + 1];
  __shared__ cx<float> sT[GJ_B][GJ_TILE + 1];
  const int t = blockIdx.x;
  int lo = 0, hi = nclust;   // tiles[c] <= t < tiles[c + 1]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (tiles[mid] <= t) lo = mid;
    else hi = mid;
  }
  const int c = lo;
  const int n = (int)(ext_ptr[c + 1] - ext_ptr[c]);
  const int bw = min(GJ_B, n - k0);
  const int nt = (n + GJ_TILE - 1) / GJ_TILE, tl = t - tiles[c];
  const int i0 = (tl / nt) * GJ_TILE, j0 = (tl % nt) * GJ_TILE;
  cx<float> *A = Ablocks + a_off[c];
  const cx<float> *tmp = tmp_all + (size_t)GJ_B * ext_ptr[c];
  for (int e = threadIdx.x; e < GJ_TILE * GJ_B; e += blockDim.x) {
    const int r = e / GJ_B, q = e - r * GJ_B, i = i0 + r;
    cx<float> v = czero<float>();
    if (i < n && q < bw) {
      v = A[(size_t)i * n + k0 + q];
      if (i == k0 + q) v.x -= 1.0f;
    }
    sP[r][q] = v;
  }
  for (int e = threadIdx.x; e < GJ_B * GJ_TILE; e += blockDim.x) {
    const int q = e / GJ_TILE, cc = e - q * GJ_TILE, j = j0 + cc;
    sT[q][cc] = (q < bw && j < n) ? tmp[(size_t)q * n + j] : czero<float>();
  }
  __syncthreads();
  const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;
  cx<float> acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; a++)
#pragma unroll
    for (int b = 0; b < 4; b++) acc[a][b] = czero<float>();
  for (int q = 0; q < bw; q++) {
    cx<float> pv[4], tv[4];
#pragma unroll
    for (int a = 0; a < 4; a++) pv[a] = sP[tr + 16 * a][q];
#pragma unroll
    for (int b = 0; b < 4; b++) tv[b] = sT[q][tc + 16 * b];
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
      for (int b = 0; b < 4; b++) cmac(acc[a][b], pv[a], tv[b]);
  }
#pragma unroll
  for (int a = 0; a < 4; a++) {
    const int i = i0 + tr + 16 * a;
    if (i >= n) continue;
#pragma unroll
    for (int b = 0; b < 4; b++) {
      const int j = j0 + tc + 16 * b;
      if (j < n && (j < k0 || j >= k0 + bw)) A[(size_t)i * n + j] += acc[a][b];
    }
  }
}

// undo the row interchanges as column interchanges, last first
__global__ void __launch_bounds__(GJ_THREADS)
gj_unswap_kernel(cx<float> *Ablocks, const int64_t *a_off, const int64_t *ext_ptr, const int *piv_all) {
  const int c = blockIdx.x;
  const int n = (int)(ext_ptr[c + 1] - ext_ptr[c]);
  cx<float> *A = Ablocks + a_off[c];
  const int *piv = piv_all + ext_ptr[c];
  for (int k = n - 1; k >= 0; k--) {
    const int pr = piv[k];
    if (pr != k)
      for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const cx<float> t = A[(size_t)i * n + k];
        A[(size_t)i * n + k] = A[(size_t)i * n + pr];
        A[(size_t)i * n + pr] = t;
      }
    __syncthreads();
  }
}

std::vector<int> gj_tile_table(const std::vector<int64_t> &ext_ptr, int &npanels) {
  const int nc = (int)ext_ptr.size() - 1;
  int64_t maxn = 0;
  for (int c = 0; c < nc; c++) maxn = std::max(maxn, ext_ptr[c + 1] - ext_ptr[c]);
  npanels = (int)((maxn + GJ_B - 1) / GJ_B);
  std::vector<int> t((size_t)npanels * (nc + 1), 0);
  for (int p = 0; p < npanels; p++)
    for (int c = 0; c < nc; c++) {
      const int64_t n = ext_ptr[c + 1] - ext_ptr[c];
      const int64_t nt = n > (int64_t)p * GJ_B ? (n + GJ_TILE - 1) / GJ_TILE : 0;
      t[(size_t)p * (nc + 1) + c + 1] = t[(size_t)p * (nc + 1) + c] + (int)(nt * nt);
    }
  return t;
}
size_t gj_scratch_entries(const std::vector<int64_t> &ext_ptr) { return (size_t)GJ_B * ext_ptr.back(); }

// Stored rows: for ext column j of cluster c, entry (i, j) = inverse[core_pos[i]][j]
// over the core rows i (8-column row-major blocks, rt_index), as FP16
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
  uint32_t *R = Rt + r_off[c];
  const int64_t ncp = rt_stride(nc);
  for (int i = lane; i < nc; i += 64) {
    const cx<float> v = A[(size_t)cp[i] * ne + j];
    R[rt_index(i, j, ncp)] = pack_h2(v.x * inv, v.y * inv);
  }
  if (lane == 0) Rs[col] = sc;
}

void launch_precond_build(const PrecondArgs &p, const std::vector<int64_t> &ext_ptr_h, const int *tiles_dev,
                          const std::vector<int> &tiles_h, int npanels, cx<float> *gj_tmp, const int64_t *core_ptr,
                          const int *core_pos, const int64_t *r_off, uint32_t *Rt, float *Rs, int *piv, int *status,
                          hipStream_t s) {
  (void)ext_ptr_h;
  hipLaunchKernelGGL(block_assemble_kernel, dim3(64, p.nc), dim3(256), 0, s, p);
  for (int pn = 0; pn < npanels; pn++) {
    const int k0 = pn * GJ_B;
    hipLaunchKernelGGL(gj_panel_kernel, dim3(p.nc), dim3(GJ_THREADS), 0, s, p.A, p.a_off, p.ext_ptr, piv, status, k0);
    hipLaunchKernelGGL(gj_pivot_rows_kernel, dim3(16, p.nc), dim3(256), 0, s, (const cx<float> *)p.A, p.a_off,
                       p.ext_ptr, gj_tmp, k0);
    const int ntiles = tiles_h[(size_t)pn * (p.nc + 1) + p.nc];
    if (ntiles > 0)
      hipLaunchKernelGGL(gj_update_kernel, dim3(ntiles), dim3(256), 0, s, p.A, p.a_off, p.ext_ptr,
                         (const cx<float> *)gj_tmp, tiles_dev + (size_t)pn * (p.nc + 1), p.nc, k0);
  }
  hipLaunchKernelGGL(gj_unswap_kernel, dim3(p.nc), dim3(GJ_THREADS), 0, s, p.A, p.a_off, p.ext_ptr, piv);
  hipLaunchKernelGGL(extract_kernel, dim3((unsigned)((p.n_ext * 64 + 255) / 256)), dim3(256), 0, s,
                     (const cx<float> *)p.A, p.a_off, p.ext_ptr, core_ptr, core_pos, r_off, p.nc, Rt, Rs);
}

// y[core] = R_c x[ext] for every cluster; each unknown is in exactly one core.
// One work-group per item (cluster c, PA_ROWS core rows from row0): the ext
// columns are staged in LDS per pass and their 8-column stored blocks split
// in PA_Q contiguous parts (each lane reads its row's 8 coefficients of a
// block at once), partial sums reduced in LDS in a fixed order.
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
  static_assert(PA_CW % RT_CB == 0, "passes start on a stored column block");
  for (int cb = 0; cb < ne; cb += PA_CW) {
    const int cw = min(PA_CW, ne - cb);
    const int cwp = (int)rt_cols(cw);
    __syncthreads();   // the previous pass is done with xs
    // the column scales fold into the staged inputs; padding columns get 0
    for (int jj = threadIdx.x; jj < cwp; jj += blockDim.x)
      xs[jj] = jj < cw ? x[ext_slot[e0 + cb + jj]] * (double)pc.scale[e0 + cb + jj] : cx<double>{0.0, 0.0};
    __syncthreads();
    // this quarter's 8-column blocks; each lane reads its row's 8 coefficients
    const int nbk = cwp / RT_CB, kb = (nbk * q) / PA_Q, ke = (nbk * (q + 1)) / PA_Q;
    if (i < nc) {
      for (int k = kb; k < ke; k++) {
        const uint4 *Rb = reinterpret_cast<const uint4 *>(R + rt_index(i, cb + k * RT_CB, ncp));
        const uint4 c0 = Rb[0], c1 = Rb[1];
        const uint32_t wd[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
#pragma unroll
        for (int u = 0; u < 8; u++) {
          const cx<float> rv = unpack_h2(wd[u]);
          const cx<double> xv = xs[k * RT_CB + u];
          pr[u & 3] += (double)rv.x * xv.x - (double)rv.y * xv.y;
          pi[u & 3] += (double)rv.x * xv.y + (double)rv.y * xv.x;
        }
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

// Batched apply in single precision for the FP32 inner solves: NB <= 8
// vectors per launch (a compile-time count, so the inner loop has no
// per-vector branches).  The inputs are first gathered once into an
// ext-ordered FP32 copy with the column scale folded in (NB values per
// column, contiguous).  Work-group = PA_ROWS core rows of one cluster, its
// PA32_Q waves split the cluster's 8-column stored blocks; per block each lane
// reads its row's 8 coefficients (32 contiguous bytes), every lane needs the
// same columns' NB inputs, so these are wave-uniform (scalar) loads fed
// straight into the FMAs, and each coefficient is read once for all vectors;
// FP32 sums, combined across the waves in LDS at the end.  This vector-ALU
// form serves 1 to 7 vectors; 8 vectors take the matrix-core form below
// (the same work split, a quarter of the issue slots per coefficient).  Inner solves stop
// at relative residuals of 1e-5 or more and an FP64 refinement follows, so
// the rounding of x and of the sums only perturbs the preconditioner, not
// the solution.
constexpr int PA32_Q = 8;
constexpr int PA32_THREADS = PA_ROWS * PA32_Q;

// inputs in FP64, or in FP32 straight from the inner solves' basis (the same
// values: FP32 to FP64 is exact)
template <typename TI>
__global__ void precond_gather32_kernel(int64_t n_ext, int m, const int *__restrict__ ext_slot,
                                        const float *__restrict__ scale, const cx<TI> *__restrict__ x, int64_t N,
                                        cx<float> *__restrict__ xe) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_ext * m) return;
  const int64_t e = t / m;
  const int b = (int)(t - e * m);
  const cx<TI> v = x[(size_t)b * N + ext_slot[e]];
  const float sc = scale[e];
  xe[t] = {(float)v.x * sc, (float)v.y * sc};
}

template <int NB>
__global__ void __launch_bounds__(PA32_THREADS)
precond_apply32_kernel(const int *__restrict__ items, const int64_t *__restrict__ ext_ptr,
                       const int64_t *__restrict__ core_ptr, const int *__restrict__ core_slot,
                       const int64_t *__restrict__ r_off, const uint32_t *__restrict__ Rst,
                       const cx<float> *__restrict__ xe, cx<double> *__restrict__ y, int64_t N) {
  __shared__ cx<float> red[PA32_Q][PA_ROWS][NB];
  // items are listed in dispatch order (see launch_precond_apply32)
  const int item = blockIdx.x;
  const int c = items[2 * item], i0 = items[2 * item + 1];
  if (c < 0) return;   // padding entry: the whole work-group leaves
  const int64_t e0 = ext_ptr[c];
  const int ne = (int)(ext_ptr[c + 1] - e0);
  const int nc = (int)(core_ptr[c + 1] - core_ptr[c]);
  const uint32_t *R = Rst + r_off[c];
  const int64_t ncp = rt_stride(nc);
  // q is uniform within a wave (PA_ROWS is the wave size); saying so lets the
  // column loads below be scalar loads
  static_assert(PA_ROWS == 64, "one wave per row block");
  const int q = __builtin_amdgcn_readfirstlane(threadIdx.x / PA_ROWS);
  const int il = threadIdx.x - q * PA_ROWS;
  const int i = i0 + il;
  cx<float> acc[NB];
#pragma unroll
  for (int b = 0; b < NB; b++) acc[b] = czero<float>();
  // the wave's share of the cluster's 8-column blocks; per block each lane
  // reads its row's 8 coefficients (32 contiguous bytes; the wave: 2 KB).
  // Padding columns hold zero coefficients and their inputs are finite (the
  // next cluster's, or the zeroed tail of the gathered copy): they add nothing.
  const int nblk = (int)(rt_cols(ne) / RT_CB);
  const int kb = (nblk * q) / PA32_Q, ke = (nblk * (q + 1)) / PA32_Q;
  if (i < nc && kb < ke) {
    const int64_t bstride = ncp * RT_CB / 4;   // uint4 per block
    const uint4 *Rb = reinterpret_cast<const uint4 *>(R + (int64_t)i * RT_CB);
    const cx<float> *xc = xe + e0 * NB;
    // the next block's loads are issued before this block's products
    uint4 c0 = Rb[kb * bstride], c1 = Rb[kb * bstride + 1];
    for (int k = kb; k < ke; k++) {
      const int kn = k + 1 < ke ? k + 1 : k;
      const uint4 n0 = Rb[kn * bstride], n1 = Rb[kn * bstride + 1];
      const uint32_t wd[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
      const cx<float> *xk = xc + (int64_t)k * RT_CB * NB;
#pragma unroll
      for (int u = 0; u < 8; u++) {
        const cx<float> rv = unpack_h2(wd[u]);
#pragma unroll
        for (int b = 0; b < NB; b++) cmac(acc[b], rv, xk[u * NB + b]);
      }
      c0 = n0;
      c1 = n1;
    }
  }
#pragma unroll
  for (int b = 0; b < NB; b++) red[q][il][b] = acc[b];
  __syncthreads();
  if (q == 0 && i < nc) {
    const int slot = core_slot[core_ptr[c] + i];
#pragma unroll
    for (int b = 0; b < NB; b++) {
      cx<float> t = red[0][il][b];
      for (int k = 1; k < PA32_Q; k++) t += red[k][il][b];
      y[(size_t)b * N + slot] = {(double)t.x, (double)t.y};
    }
  }
}

// The 8-vector apply on the matrix cores.  Per stored 8-column block the
// product Y[rows, 8 vectors] += R[rows, 8 columns] X[8 columns, 8 vectors] is
// taken in real form: K = 16 (column, re/im of R) and N = 16 (vector, re/im
// of the result), with B[(u, re)][(b, .)] = (Re x, Im x) and
// B[(u, im)][(b, .)] = (-Im x, Re x), so that D = Re(R x), Im(R x) side by
// side; four 16x16x4 FP32 steps per block and 16-row tile.  Lane (m, kq),
// m = lane % 16, kq = lane / 16, supplies in step s the (column 2 kq + s / 2,
// part s % 2) entries: of row m of the tile for A (one 8-byte read of two
// coefficients per tile) and of vector m / 2 for B (two gathered inputs, the
// component picked by m % 2).  A wave covers 64 rows as four tiles that share
// B; the waves split the blocks as in the vector-ALU form above.
typedef float mf4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(PA32_THREADS)
precond_apply32_mfma_kernel(const int *__restrict__ items, const int64_t *__restrict__ ext_ptr,
                            const int64_t *__restrict__ core_ptr, const int *__restrict__ core_slot,
                            const int64_t *__restrict__ r_off, const uint32_t *__restrict__ Rst,
                            const cx<float> *__restrict__ xe, cx<double> *__restrict__ y, int64_t N) {
  constexpr int NB = 8;
  __shared__ float red[PA32_Q][PA_ROWS][2 * NB];
  const int item = blockIdx.x;
  const int c = items[2 * item], i0 = items[2 * item + 1];
  if (c < 0) return;   // padding entry: the whole work-group leaves
  const int64_t e0 = ext_ptr[c];
  const int ne = (int)(ext_ptr[c + 1] - e0);
  const int nc = (int)(core_ptr[c + 1] - core_ptr[c]);
  const uint32_t *R = Rst + r_off[c];
  const int64_t ncp = rt_stride(nc);
  const int q = __builtin_amdgcn_readfirstlane(threadIdx.x / PA_ROWS);
  const int lane = threadIdx.x - q * PA_ROWS;
  const int m = lane & 15, kq = lane >> 4;
  const bool odd = (m & 1) != 0;
  mf4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; t++) acc[t] = mf4{0.f, 0.f, 0.f, 0.f};
  const int nblk = (int)(rt_cols(ne) / RT_CB);
  const int kb = (nblk * q) / PA32_Q, ke = (nblk * (q + 1)) / PA32_Q;
  if (kb < ke) {   // wave-uniform
    // row i0 + 16 t + m of the tiles; rows past the core read as zero
    bool live[4];
    const uint2 *Ra[4];
#pragma unroll
    for (int t = 0; t < 4; t++) {
      const int i = i0 + 16 * t + m;
      live[t] = i < nc;
      Ra[t] = reinterpret_cast<const uint2 *>(R + (int64_t)(live[t] ? i : 0) * RT_CB + 2 * kq);
    }
    const int64_t bstride = ncp * RT_CB / 2;   // uint2 per block
    // inputs of columns 2 kq, 2 kq + 1 of block k for vector m / 2
    const cx<float> *xl = xe + e0 * NB + (2 * kq) * NB + (m >> 1);
    auto load = [&](int k, uint2 *a, cx<float> *xv) {
#pragma unroll
      for (int t = 0; t < 4; t++) a[t] = live[t] ? Ra[t][k * bstride] : make_uint2(0u, 0u);
      xv[0] = xl[(int64_t)k * RT_CB * NB];
      xv[1] = xl[(int64_t)k * RT_CB * NB + NB];
    };
    uint2 a[4], an[4];
    cx<float> xv[2], xn[2];
    load(kb, a, xv);
    for (int k = kb; k < ke; k++) {
      load(k + 1 < ke ? k + 1 : k, an, xn);
      float b[4];
#pragma unroll
      for (int u = 0; u < 2; u++) {
        b[2 * u] = odd ? xv[u].y : xv[u].x;
        b[2 * u + 1] = odd ? xv[u].x : -xv[u].y;
      }
#pragma unroll
      for (int t = 0; t < 4; t++) {
        const cx<float> r0 = unpack_h2(a[t].x), r1 = unpack_h2(a[t].y);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(r0.x, b[0], acc[t], 0, 0, 0);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(r0.y, b[1], acc[t], 0, 0, 0);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(r1.x, b[2], acc[t], 0, 0, 0);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(r1.y, b[3], acc[t], 0, 0, 0);
      }
#pragma unroll
      for (int t = 0; t < 4; t++) a[t] = an[t];
      xv[0] = xn[0];
      xv[1] = xn[1];
    }
  }
  // lane (m, kq) holds D[4 kq + r][m] of each tile: row 16 t + 4 kq + r,
  // vector m / 2, real part for even m
#pragma unroll
  for (int t = 0; t < 4; t++)
#pragma unroll
    for (int r = 0; r < 4; r++) red[q][16 * t + 4 * kq + r][m] = acc[t][r];
  __syncthreads();
  const int i = i0 + lane;
  if (q == 0 && i < nc) {
    const int slot = core_slot[core_ptr[c] + i];
#pragma unroll
    for (int b = 0; b < NB; b++) {
      float tr = red[0][lane][2 * b], ti = red[0][lane][2 * b + 1];
      for (int k = 1; k < PA32_Q; k++) {
        tr += red[k][lane][2 * b];
        ti += red[k][lane][2 * b + 1];
      }
      y[(size_t)b * N + slot] = {(double)tr, (double)ti};
    }
  }
}

int precond_apply32_max_batch() { return 8; }

template <typename TI>
void launch_precond_gather32(int64_t n_ext, const int *ext_slot, const float *scale, const cx<TI> *x, int64_t N,
                             int m, cx<float> *xe, hipStream_t s) {
  const int64_t total = n_ext * m;
  if (total == 0) return;
  const int threads = 256;
  hipLaunchKernelGGL(precond_gather32_kernel<TI>, dim3((unsigned)((total + threads - 1) / threads)), dim3(threads), 0,
                     s, n_ext, m, ext_slot, scale, x, N, xe);
}
template void launch_precond_gather32<double>(int64_t, const int *, const float *, const cx<double> *, int64_t, int,
                                              cx<float> *, hipStream_t);
template void launch_precond_gather32<float>(int64_t, const int *, const float *, const cx<float> *, int64_t, int,
                                             cx<float> *, hipStream_t);

template <int NB>
static void apply32_launch(int n_items, const int *items, const int64_t *ext_ptr, const int64_t *core_ptr,
                           const int *core_slot, const int64_t *r_off, const uint32_t *R, const cx<float> *xe,
                           cx<double> *y, int64_t N, hipStream_t s) {
  hipLaunchKernelGGL((precond_apply32_kernel<NB>), dim3(n_items), dim3(PA32_THREADS), 0, s, items, ext_ptr, core_ptr,
                     core_slot, r_off, R, xe, y, N);
}

// m <= precond_apply32_max_batch() vectors (one kernel instance per count);
// xe as written by launch_precond_gather32 with the same m.  items: n_items
// (cluster, first core row) pairs, one work-group each in list order, so the
// list fixes which XCD runs what (work-group i goes to XCD i mod 8); entries
// with cluster -1 are empty.
void launch_precond_apply32(int n_items, const int *items, const int64_t *ext_ptr, const int64_t *core_ptr,
                            const int *core_slot, const int64_t *r_off, const uint32_t *R, const cx<float> *xe,
                            cx<double> *y, int64_t N, int m, hipStream_t s) {
  if (n_items == 0) return;
#define SCABS_APPLY32(NB) apply32_launch<NB>(n_items, items, ext_ptr, core_ptr, core_slot, r_off, R, xe, y, N, s)
  switch (m) {
    case 1: SCABS_APPLY32(1); break;
    case 2: SCABS_APPLY32(2); break;
    case 3: SCABS_APPLY32(3); break;
    case 4: SCABS_APPLY32(4); break;
    case 5: SCABS_APPLY32(5); break;
    case 6: SCABS_APPLY32(6); break;
    case 7: SCABS_APPLY32(7); break;
    default:
      hipLaunchKernelGGL(precond_apply32_mfma_kernel, dim3(n_items), dim3(PA32_THREADS), 0, s, items, ext_ptr,
                         core_ptr, core_slot, r_off, R, xe, y, N);
      break;
  }
#undef SCABS_APPLY32
}

}  // namespace scabs
