// Matrix-vector product kernels of the precorrected-FFT operator.
//
// Row conventions (paper Sec. II / Appendix A, one row triple per edge):
//   E row  <X_n, E_e(J_e, M_e) - E_i(J_i, M_i)>                     (eq1 / eq3)
//   H row  <X_n, H_e^+ - H_i^->  + sum_q w sigma (X_n x n).E_e^+(q)   (eq2 / eq13,
//          tested after rotating eq4 by n x)
//   eq14   <X_n, J_e + J_i> - sum_q w sigma X_n.E_i^-(q)
// with per-edge currents J_e, J_i, M_e = M, M_i = -M (eq10-eq12) and one-sided
// limits E^+/- = PV +/- 1/2 n x M, H^+/- = PV -/+ 1/2 n x J.
#include <algorithm>

#include "device_common.h"
#include "kernels.h"

namespace scabs {

// ---------------------------------------------------------------------------
// unknown vector -> per-edge currents (J_e, J_i, M)
// ---------------------------------------------------------------------------
// batch index blockIdx.y: x + b * 2N, src + b * 3 ne; with srcI (nb > 1) the
// same currents also edge-major, srcI[(e nb + b) 3 + j]
template <typename T>
__global__ void unpack_kernel(const EdgeRec *__restrict__ edges, int ne, int N, const double *__restrict__ x,
                              cx<T> *__restrict__ src, cx<T> *__restrict__ srcI, int nb) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const int bb = blockIdx.y;
  x += (size_t)bb * 2 * N;
  src += (size_t)bb * 3 * ne;
  EdgeRec r = edges[e];
  const cx<T> a = {(T)x[2 * r.col[0]], (T)x[2 * r.col[0] + 1]};
  const cx<T> b = {(T)x[2 * r.col[1]], (T)x[2 * r.col[1] + 1]};
  cx<T> v[3];
  if (!r.isR) {
    v[0] = a;
    v[1] = -a;
    v[2] = b;
  } else {
    v[0] = a;
    v[1] = b;
    v[2] = cx<T>{(T)x[2 * r.col[2]], (T)x[2 * r.col[2] + 1]};
  }
#pragma unroll
  for (int j = 0; j < 3; j++) src[3 * e + j] = v[j];
  if (srcI) {
    cx<T> *o = srcI + ((size_t)e * nb + bb) * 3;
#pragma unroll
    for (int j = 0; j < 3; j++) o[j] = v[j];
  }
}

template <typename T> void launch_unpack(const DevOperator<T> &op, const double *x, hipStream_t s, int nb) {
  hipLaunchKernelGGL(unpack_kernel<T>, dim3((op.ne + 255) / 256, nb), dim3(256), 0, s, op.edges, op.ne, op.N, x,
                     op.src, nb > 1 ? op.srcI : (cx<T> *)nullptr, nb);
}
template void launch_unpack<float>(const DevOperator<float> &, const double *, hipStream_t, int);
template void launch_unpack<double>(const DevOperator<double> &, const double *, hipStream_t, int);

// ---------------------------------------------------------------------------
// projection: every quadrature point spreads w_q (J, div J, M, div M) of its
// medium onto the 27 nodes around its anchor with tensor Lagrange weights.
// Gather form: (1) per point the 8 weighted source values, written in the
// grid's cell-sorted order; (2) one thread per node sums the points of the 27
// cells around it.  No atomics; the summation order is fixed.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
point_sources_kernel(const PointRec<T> *__restrict__ pts, const TriRec<T> *__restrict__ tris,
                     const cx<T> *__restrict__ esrc, const cx<T> *__restrict__ esrcI, GatherGrid<T> g, int interior,
                     int ne, int nb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.np) return;
  // the point's records once for all vectors of the batch; batch currents
  // edge-major ([e][b][3]) when there are several
  const PointRec<T> P = pts[g.perm[i]];
  const TriRec<T> tr = tris[P.tri];
  for (int b = 0; b < nb; b++) {
    cx<T> s[8];
#pragma unroll
    for (int f = 0; f < 8; f++) s[f] = czero<T>();
#pragma unroll
    for (int j = 0; j < 3; j++) {
      const int e = tr.edge[j];
      const cx<T> *c = nb > 1 ? esrcI + ((size_t)e * nb + b) * 3 : esrc + (size_t)3 * e;
      const cx<T> J = interior ? c[1] : c[0];
      const cx<T> M = interior ? -c[2] : c[2];
#pragma unroll
      for (int a = 0; a < 3; a++) {
        axpy(s[a], P.f[3 * j + a], J);
        axpy(s[4 + a], P.f[3 * j + a], M);
      }
      axpy(s[3], tr.div[j], J);
      axpy(s[7], tr.div[j], M);
    }
    cx<T> *o = g.src + (size_t)8 * g.np * b + (size_t)8 * i;
#pragma unroll
    for (int f = 0; f < 8; f++) o[f] = s[f] * P.w;
  }
}

// One work-group per x plane of a grid (and vector of the batch), in chunks
// of the cells that hold points among the planes x-1..x+1 (listed per plane
// at setup).  Phase A, work item (cell, y offset oy) (FP32; (cell, (oy, oz))
// otherwise): the cell's points, in sorted order, summed into the
// contributions to the nodes of plane x at offsets (oy, -1..1) (the x offset
// is fixed by the cell's plane); the lanes of a cell share its loop length,
// and empty cells cost nothing.  Phase B, work item (node, x offset): the
// contributions of the 9 cells around the node in that offset's plane, read
// through a cell -> slot map in LDS; the three x partials of a node sit in
// neighbouring lanes and are added by shuffles.  No atomics; the summation
// order is fixed.
// cells per pass: FP32 64 (measured best of 48-160 for batches: less LDS,
// more resident work-groups), FP64 48; the same for every batch size, so a
// batch gives each vector the sums of its own product
template <typename T> struct CellChunk { static constexpr int value = 64; };
template <> struct CellChunk<double> { static constexpr int value = 48; };
template <typename T, int MAXI>
__global__ void __launch_bounds__(1024) gather_kernel(DevGrid<T> dg, GatherGrid<T> g) {
  constexpr int SC = CellChunk<T>::value, SQ = 9 * SC;
  static_assert(8 * SQ >= 3 * 1024, "the final reduction reuses s_q for 3 planes of at most 1024 nodes");
  __shared__ cx<T> s_q[8][SQ];
  extern __shared__ __align__(16) int s_map[];   // (plane - xl) * plane + yz -> slot, or -1
  const int n0 = dg.n[0], n1 = dg.n[1], n2 = dg.n[2];
  const int plane = n1 * n2;
  // XCD-aware order: neighbouring planes (which read the same points) on one XCD
  const int lb = xcd_remap(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  const int bb = lb / gridDim.x, x = lb - bb * gridDim.x;   // batch index, plane
  const cx<T> *gsrc = g.src + (size_t)8 * g.np * bb;
  cx<T> *phys = dg.phys + (size_t)8 * g.ncell * bb;
  const int xl = max(x - 1, 0), xh = min(x + 1, n0 - 1);
  const int K0 = g.nz_ptr[xl], K = g.nz_ptr[xh + 1] - K0;
  const int B1 = g.nz_ptr[min(xl + 1, xh + 1)] - K0, B2 = g.nz_ptr[min(xl + 2, xh + 1)] - K0;
  for (int t = threadIdx.x; t < (xh - xl + 1) * plane; t += blockDim.x) s_map[t] = -1;
  __syncthreads();
  for (int k = threadIdx.x; k < K; k += blockDim.x) s_map[((k >= B1) + (k >= B2)) * plane + g.nz_yz[K0 + k]] = k;
  __syncthreads();
  const FastDiv dn2 = make_fastdiv(n2), dpl = make_fastdiv(plane), d9 = make_fastdiv(9), d3 = make_fastdiv(3);
  cx<T> acc[MAXI][8];
#pragma unroll
  for (int m = 0; m < MAXI; m++)
#pragma unroll
    for (int f = 0; f < 8; f++) acc[m][f] = czero<T>();
  for (int c0 = 0; c0 < K; c0 += SC) {
    const int cn = min(SC, K - c0);
    if constexpr (sizeof(T) == 4 && MAXI == 1) {
      // FP32, at most one node per thread: one item per (cell, y offset)
      // producing the three z offsets, so a point's loads and its x-y weight
      // serve three node sums (same products and order as one item per
      // offset; with more nodes per thread, or in FP64, the registers of the
      // three sums would spill)
      for (int it = threadIdx.x; it < 3 * cn; it += blockDim.x) {
        const int kk = fdiv(it, d3), oyi = it - 3 * kk;
        const int k = c0 + kk;
        const int cxo = (k >= B1) + (k >= B2);
        const int yz = g.nz_yz[K0 + k];
        const int cy = fdiv(yz, dn2);
        const int ox = x - (xl + cxo), oy = oyi - 1;
        cx<T> a[3][8];
#pragma unroll
        for (int r = 0; r < 3; r++)
#pragma unroll
          for (int f = 0; f < 8; f++) a[r][f] = czero<T>();
        if (cy + oy >= 0 && cy + oy < n1) {
          const int64_t cell = (int64_t)(xl + cxo) * plane + yz;
          const int64_t p1 = g.cellptr[cell + 1];
          int64_t p = g.cellptr[cell];
          for (; p + 2 <= p1; p += 2) {
            cx<T> s0[8], s1[8];
#pragma unroll
            for (int f = 0; f < 8; f++) {
              s0[f] = gsrc[8 * p + f];
              s1[f] = gsrc[8 * p + 8 + f];
            }
            const T w0 = lag_w(ox, g.u[3 * p]) * lag_w(oy, g.u[3 * p + 1]);
            const T w1 = lag_w(ox, g.u[3 * p + 3]) * lag_w(oy, g.u[3 * p + 4]);
            const T uz0 = g.u[3 * p + 2], uz1 = g.u[3 * p + 5];
#pragma unroll
            for (int r = 0; r < 3; r++) {
              const T wr0 = w0 * lag_w(r - 1, uz0), wr1 = w1 * lag_w(r - 1, uz1);
#pragma unroll
              for (int f = 0; f < 8; f++) axpy(a[r][f], wr0, s0[f]);
#pragma unroll
              for (int f = 0; f < 8; f++) axpy(a[r][f], wr1, s1[f]);
            }
          }
          for (; p < p1; p++) {
            const T w = lag_w(ox, g.u[3 * p]) * lag_w(oy, g.u[3 * p + 1]);
            const T uz = g.u[3 * p + 2];
            cx<T> s0[8];
#pragma unroll
            for (int f = 0; f < 8; f++) s0[f] = gsrc[8 * p + f];
#pragma unroll
            for (int r = 0; r < 3; r++) {
              const T wr = w * lag_w(r - 1, uz);
#pragma unroll
              for (int f = 0; f < 8; f++) axpy(a[r][f], wr, s0[f]);
            }
          }
        }
        // z offsets whose node lies outside the lattice are never read back
#pragma unroll
        for (int r = 0; r < 3; r++)
#pragma unroll
          for (int f = 0; f < 8; f++) s_q[f][9 * kk + 3 * oyi + r] = a[r][f];
      }
    } else {
      for (int it = threadIdx.x; it < 9 * cn; it += blockDim.x) {
        const int kk = fdiv(it, d9), off = it - 9 * kk;
        const int k = c0 + kk;
        const int cxo = (k >= B1) + (k >= B2);
        const int yz = g.nz_yz[K0 + k];
        const int cy = fdiv(yz, dn2), cz = yz - cy * n2;
        const int oyi = fdiv(off, d3);
        const int ox = x - (xl + cxo), oy = oyi - 1, oz = off - 3 * oyi - 1;
        cx<T> a[8];
#pragma unroll
        for (int f = 0; f < 8; f++) a[f] = czero<T>();
        if (cy + oy >= 0 && cy + oy < n1 && cz + oz >= 0 && cz + oz < n2) {
          const int64_t cell = (int64_t)(xl + cxo) * plane + yz;
          const int64_t p1 = g.cellptr[cell + 1];
          int64_t p = g.cellptr[cell];
          for (; p < p1; p++) {
            const T w = lag_w(ox, g.u[3 * p]) * lag_w(oy, g.u[3 * p + 1]) * lag_w(oz, g.u[3 * p + 2]);
#pragma unroll
            for (int f = 0; f < 8; f++) axpy(a[f], w, gsrc[8 * p + f]);
          }
        }
#pragma unroll
        for (int f = 0; f < 8; f++) s_q[f][it] = a[f];
      }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < MAXI; m++) {
      int it = threadIdx.x + m * blockDim.x, oxi, nd;
      if constexpr (MAXI == 1) {
        // 21 nodes per wave, their three x offsets in neighbouring lanes
        const int ln = threadIdx.x & 63;
        oxi = ln % 3;
        nd = (threadIdx.x >> 6) * GB_NODES_PER_WAVE + ln / 3;
        if (ln >= 3 * GB_NODES_PER_WAVE || nd >= plane) continue;
      } else {
        if (it >= 3 * plane) continue;
        oxi = fdiv(it, dpl);
        nd = it - oxi * plane;
      }
      const int cxp = x - (oxi - 1);   // the cells' plane: node offset oxi - 1 from their anchors
      if (cxp < xl || cxp > xh) continue;
      const int y = fdiv(nd, dn2), z = nd - y * n2;
      const int *mp = s_map + (cxp - xl) * plane;
#pragma unroll
      for (int oy = -1; oy <= 1; oy++) {
        const int cy = y - oy;
        if (cy < 0 || cy >= n1) continue;
#pragma unroll
        for (int oz = -1; oz <= 1; oz++) {
          const int cz = z - oz;
          if (cz < 0 || cz >= n2) continue;
          const int k = mp[cy * n2 + cz] - c0;
          if ((unsigned)k < (unsigned)cn) {
            const int q = 9 * k + 3 * (oy + 1) + oz + 1;
#pragma unroll
            for (int f = 0; f < 8; f++) acc[m][f] += s_q[f][q];
          }
        }
      }
    }
    __syncthreads();
  }
  const size_t G = (size_t)g.ncell;
  if constexpr (MAXI == 1) {
    // the three x-offset sums of a node meet across neighbouring lanes
    const int ln = threadIdx.x & 63;
    const int nd = (threadIdx.x >> 6) * GB_NODES_PER_WAVE + ln / 3;
    const bool own = ln < 3 * GB_NODES_PER_WAVE && ln % 3 == 0 && nd < plane;
#pragma unroll
    for (int f = 0; f < 8; f++) {
      const cx<T> v = acc[0][f];
      const cx<T> v1 = {__shfl_down(v.x, 1, 64), __shfl_down(v.y, 1, 64)};
      const cx<T> v2 = {__shfl_down(v.x, 2, 64), __shfl_down(v.y, 2, 64)};
      if (own) phys[f * G + (size_t)x * plane + nd] = v + v1 + v2;
    }
    return;
  }
  cx<T> *s_red = &s_q[0][0];   // 3 * plane <= 8 * SQ
  for (int f = 0; f < 8; f++) {
#pragma unroll
    for (int m = 0; m < MAXI; m++) {
      const int it = threadIdx.x + m * blockDim.x;
      if (it < 3 * plane) s_red[it] = acc[m][f];
    }
    __syncthreads();
    for (int nd = threadIdx.x; nd < plane; nd += blockDim.x)
      phys[f * G + (size_t)x * plane + nd] = s_red[nd] + s_red[plane + nd] + s_red[2 * plane + nd];
    __syncthreads();
  }
}

template <typename T>
void launch_project(const DevOperator<T> &op, const std::vector<DevGrid<T>> &grids,
                    const std::vector<GatherGrid<T>> &gg, hipStream_t s, int nb, int part) {
  if (part < 0)   // -1: sources and gathers; -2: sources only
    for (size_t k = 0; k < grids.size(); k++) {
      const GatherGrid<T> &g = gg[k];
      hipLaunchKernelGGL(point_sources_kernel<T>, dim3((g.np + 255) / 256), dim3(256), 0, s, op.pts, op.tris,
                         op.src, op.srcI, g, grids[k].which >= 0 ? 1 : 0, op.ne, nb);
    }
  for (size_t k = 0; k < grids.size(); k++) {
    if (part == -2 || (part >= 0 && (int)k != part)) continue;
    const GatherGrid<T> &g = gg[k];
    const int plane = grids[k].n[1] * grids[k].n[2];
    const int items = 3 * plane;
    int threads = std::min(1024, (items + 63) / 64 * 64);
    int maxi = (items + threads - 1) / threads;
    // one pass over the nodes: waves of 21 nodes (their 3 x offsets in lane
    // triples), when they fit one work-group
    const int triple_threads = (plane + GB_NODES_PER_WAVE - 1) / GB_NODES_PER_WAVE * 64;
    if (maxi == 1) {
      if (triple_threads <= 1024) {
        threads = std::max(threads, triple_threads);
      } else {
        threads = 1024;
        maxi = 2;
      }
    }
    const size_t lds = sizeof(int) * (size_t)items;   // cell -> slot map of three planes
    const dim3 grid(grids[k].n[0], nb);
    if (maxi == 1)
      hipLaunchKernelGGL((gather_kernel<T, 1>), grid, dim3(threads), lds, s, grids[k], g);
    else if (maxi == 2)
      hipLaunchKernelGGL((gather_kernel<T, 2>), grid, dim3(threads), lds, s, grids[k], g);
    else
      hipLaunchKernelGGL((gather_kernel<T, 3>), grid, dim3(threads), lds, s, grids[k], g);
  }
}
template void launch_project<float>(const DevOperator<float> &, const std::vector<DevGrid<float>> &,
                                    const std::vector<GatherGrid<float>> &, hipStream_t, int, int);
template void launch_project<double>(const DevOperator<double> &, const std::vector<DevGrid<double>> &,
                                     const std::vector<GatherGrid<double>> &, hipStream_t, int, int);

// ---------------------------------------------------------------------------
// interpolation at test points + row contributions + local terms, reduced to
// per-triangle half-edge partials.  One thread per point, 32 triangles per
// work-group.
// ---------------------------------------------------------------------------
constexpr int IT_TRIS = 32;
constexpr int IT_THREADS = IT_TRIS * NQ;

template <typename T> struct Pot {
  cx<T> val[8];
  cx<T> grad[8][3];
};

template <typename T>
__device__ inline void gather_direct(const DevGrid<T> &g, int ax, int ay, int az, const T *Lx, const T *Ly, const T *Lz,
                              const T *dLx, const T *dLy, const T *dLz, T inv_h, Pot<T> &p, int b) {
#pragma unroll
  for (int f = 0; f < 8; f++) {
    p.val[f] = czero<T>();
    p.grad[f][0] = p.grad[f][1] = p.grad[f][2] = czero<T>();
  }
  const int n1 = g.n[1], n2 = g.n[2];
  const size_t G = (size_t)g.n[0] * n1 * n2;
  const cx<T> *phys = g.phys + (size_t)8 * G * b;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      const size_t row = ((size_t)(ax + i - 1) * n1 + (ay + j - 1)) * n2 + (az - 1);
      const T wxy = Lx[i] * Ly[j], dxy = dLx[i] * Ly[j], xdy = Lx[i] * dLy[j];
#pragma unroll
      for (int k = 0; k < 3; k++) {
        const T w = wxy * Lz[k], gx = dxy * Lz[k] * inv_h, gy = xdy * Lz[k] * inv_h, gz = wxy * dLz[k] * inv_h;
#pragma unroll
        for (int f = 0; f < 8; f++) {
          const cx<T> v = phys[f * G + row + k];
          axpy(p.val[f], w, v);
          axpy(p.grad[f][0], gx, v);
          axpy(p.grad[f][1], gy, v);
          axpy(p.grad[f][2], gz, v);
        }
      }
    }
}

// Potentials and gradients of the 8 fields at a point from its 27 nodes,
// contracted one axis at a time (the weights are a tensor product): per
// field, z first (values and z-derivative weights), then y, then x; one
// field at a time (its 27 loads in flight).
template <typename T>
__device__ inline void gather_separable(const DevGrid<T> &g, int ax, int ay, int az, const T *Lx, const T *Ly, const T *Lz,
                              const T *dLx, const T *dLy, const T *dLz, T inv_h, Pot<T> &p, int b) {
  const int n1 = g.n[1], n2 = g.n[2];
  const size_t G = (size_t)g.n[0] * n1 * n2;
  const cx<T> *phys = g.phys + (size_t)8 * G * b + ((size_t)(ax - 1) * n1 + (ay - 1)) * n2 + (az - 1);
#pragma unroll 1
  for (int f = 0; f < 8; f++) {
    const cx<T> *pf = phys + f * G;
    cx<T> val = czero<T>(), gx = czero<T>(), gy = czero<T>(), gz = czero<T>();
#pragma unroll
    for (int i = 0; i < 3; i++) {
      cx<T> C = czero<T>(), D = czero<T>(), E = czero<T>();
#pragma unroll
      for (int j = 0; j < 3; j++) {
        const cx<T> *r = pf + ((size_t)i * n1 + j) * n2;
        const cx<T> v0 = r[0], v1 = r[1], v2 = r[2];
        cx<T> A = v0 * Lz[0], B = v0 * dLz[0];
        axpy(A, Lz[1], v1);
        axpy(A, Lz[2], v2);
        axpy(B, dLz[1], v1);
        axpy(B, dLz[2], v2);
        axpy(C, Ly[j], A);
        axpy(D, dLy[j], A);
        axpy(E, Ly[j], B);
      }
      axpy(val, Lx[i], C);
      axpy(gx, dLx[i], C);
      axpy(gy, Lx[i], D);
      axpy(gz, Lx[i], E);
    }
    p.val[f] = val;
    p.grad[f][0] = gx * inv_h;
    p.grad[f][1] = gy * inv_h;
    p.grad[f][2] = gz * inv_h;
  }
}

// FP32: the direct sum (all loads of the 27 nodes in flight; 213 VGPRs, no
// spill); FP64: the separable form with one field at a time (the direct sum
// needs more than the 256 VGPRs there; measured 240 -> 178 us per product)
template <typename T>
__device__ inline void gather(const DevGrid<T> &g, int ax, int ay, int az, const T *Lx, const T *Ly, const T *Lz,
                              const T *dLx, const T *dLy, const T *dLz, T inv_h, Pot<T> &p, int b) {
  if constexpr (sizeof(T) == 8)
    gather_separable(g, ax, ay, az, Lx, Ly, Lz, dLx, dLy, dLz, inv_h, p, b);
  else
    gather_direct(g, ax, ay, az, Lx, Ly, Lz, dLx, dLy, dLz, inv_h, p, b);
}

template <typename T> __device__ inline cx<T> rdot(const T *a, const cx<T> *b) {
  cx<T> r = a[0] * b[0];
  axpy(r, a[1], b[1]);
  axpy(r, a[2], b[2]);
  return r;
}

template <typename T>
__global__ void __launch_bounds__(IT_THREADS)
interp_test_kernel(DevOperator<T> op, DevGrid<T> ext, const DevGrid<T> *__restrict__ ints, T inv_h) {
  __shared__ cx<T> part[IT_THREADS][9];
  const int lt = threadIdx.x / NQ, q = threadIdx.x - lt * NQ;
  const int tri = blockIdx.x * IT_TRIS + lt;
  const int bb = blockIdx.y;   // batch index
  const cx<T> *esrc = op.src + (size_t)3 * op.ne * bb;
  cx<T> out[9];
#pragma unroll
  for (int r = 0; r < 9; r++) out[r] = czero<T>();
  if (tri < op.nt) {
    const PointRec<T> P = op.pts[tri * NQ + q];
    const TriRec<T> tr = op.tris[tri];
    const T n[3] = {tr.nrm[0], tr.nrm[1], tr.nrm[2]};
    // local currents at the point
    cx<T> Jsum[3], Mq[3];
    for (int a = 0; a < 3; a++) Jsum[a] = Mq[a] = czero<T>();
    for (int j = 0; j < 3; j++) {
      const int e = tr.edge[j];
      const cx<T> Je = esrc[3 * e], Ji = esrc[3 * e + 1], M = esrc[3 * e + 2];
      for (int a = 0; a < 3; a++) {
        axpy(Jsum[a], P.f[3 * j + a], Je + Ji);
        axpy(Mq[a], P.f[3 * j + a], M);
      }
    }
    // 1/2 n x M (residue of the one-sided E limits) and n x (J_e + J_i)
    cx<T> hnM[3], nJ[3];
    hnM[0] = T(0.5) * (n[1] * Mq[2] - n[2] * Mq[1]);
    hnM[1] = T(0.5) * (n[2] * Mq[0] - n[0] * Mq[2]);
    hnM[2] = T(0.5) * (n[0] * Mq[1] - n[1] * Mq[0]);
    nJ[0] = n[1] * Jsum[2] - n[2] * Jsum[1];
    nJ[1] = n[2] * Jsum[0] - n[0] * Jsum[2];
    nJ[2] = n[0] * Jsum[1] - n[1] * Jsum[0];
    T Lx[3], Ly[3], Lz[3], dLx[3], dLy[3], dLz[3];
    lagr3(P.u[0], Lx, dLx);
    lagr3(P.u[1], Ly, dLy);
    lagr3(P.u[2], Lz, dLz);
    int ax, ay, az;
    unpack_anchor(P.anc, ax, ay, az);
    const T w = P.w, ws = P.w * P.sigma;
    Pot<T> pot;
    for (int med = 0; med < 2; med++) {
      const DevGrid<T> &g = med == 0 ? ext : ints[tr.body];
      gather(g, ax - g.off[0], ay - g.off[1], az - g.off[2], Lx, Ly, Lz, dLx, dLy, dLz, inv_h, pot, bb);
      const T k = g.k, Z = g.Z, ik2 = T(1) / (k * k);
      const T sgn = med == 0 ? T(1) : T(-1);
      cx<T> aJ[3] = {pot.val[0], pot.val[1], pot.val[2]};
      cx<T> aM[3] = {pot.val[4], pot.val[5], pot.val[6]};
      cx<T> cJ[3] = {pot.grad[2][1] - pot.grad[1][2], pot.grad[0][2] - pot.grad[2][0], pot.grad[1][0] - pot.grad[0][1]};
      cx<T> cM[3] = {pot.grad[6][1] - pot.grad[5][2], pot.grad[4][2] - pot.grad[6][0], pot.grad[5][0] - pot.grad[4][1]};
      // pointwise one-sided field: E = -Z jk (a_J + k^-2 grad phi_J) - curl a_M + 1/2 n x M
      cx<T> Ep[3];
      for (int a = 0; a < 3; a++) {
        cx<T> t = aJ[a];
        axpy(t, ik2, pot.grad[3][a]);
        Ep[a] = mul_j(t) * (-Z * k) - cM[a] + hnM[a];
      }
      const cx<T> phJ = pot.val[3], phM = pot.val[7];
      for (int i = 0; i < 3; i++) {
        const T gi[3] = {P.f[3 * i], P.f[3 * i + 1], P.f[3 * i + 2]};
        const T dg = tr.div[i];
        // <g, E> = -Z jk (g.a_J - k^-2 div g phi_J) - g.curl a_M
        cx<T> t1 = rdot(gi, aJ);
        axpy(t1, -dg * ik2, phJ);
        cx<T> e = mul_j(t1) * (-Z * k) - rdot(gi, cM);
        // <g, H> = g.curl a_J - (jk/Z)(g.a_M - k^-2 div g phi_M)
        cx<T> t2 = rdot(gi, aM);
        axpy(t2, -dg * ik2, phM);
        cx<T> h = rdot(gi, cJ) - mul_j(t2) * (k / Z);
        axpy(out[3 * i], sgn * w, e);
        axpy(out[3 * i + 1], sgn * w, h);
        if (ws != T(0)) {
          if (med == 0) {
            const T gxn[3] = {gi[1] * n[2] - gi[2] * n[1], gi[2] * n[0] - gi[0] * n[2], gi[0] * n[1] - gi[1] * n[0]};
            axpy(out[3 * i + 1], ws, rdot(gxn, Ep));
          } else {
            axpy(out[3 * i + 2], -ws, rdot(gi, Ep));
          }
        }
      }
    }
    // local terms: H residue -1/2 <g, n x (J_e + J_i)>, Gram <g, J_e + J_i>
    for (int i = 0; i < 3; i++) {
      const T gi[3] = {P.f[3 * i], P.f[3 * i + 1], P.f[3 * i + 2]};
      axpy(out[3 * i + 1], T(-0.5) * w, rdot(gi, nJ));
      axpy(out[3 * i + 2], w, rdot(gi, Jsum));
    }
  }
#pragma unroll
  for (int r = 0; r < 9; r++) part[threadIdx.x][r] = out[r];
  __syncthreads();
  for (int it = threadIdx.x; it < IT_TRIS * 9; it += blockDim.x) {
    const int l = it / 9, r = it - l * 9;
    const int t2 = blockIdx.x * IT_TRIS + l;
    if (t2 < op.nt) {
      cx<T> s = czero<T>();
      for (int qq = 0; qq < NQ; qq++) s += part[l * NQ + qq][r];
      op.tri_out[(size_t)9 * op.nt * bb + (size_t)t2 * 9 + r] = s;
    }
  }
}

template <typename T>
void launch_interp_test(const DevOperator<T> &op, const DevGrid<T> &ext, const DevGrid<T> *ints_dev, T inv_h,
                        hipStream_t s, int nb) {
  hipLaunchKernelGGL(interp_test_kernel<T>, dim3((op.nt + IT_TRIS - 1) / IT_TRIS, nb), dim3(IT_THREADS), 0, s, op, ext,
                     ints_dev, inv_h);
}
template void launch_interp_test<float>(const DevOperator<float> &, const DevGrid<float> &, const DevGrid<float> *,
                                        float, hipStream_t, int);
template void launch_interp_test<double>(const DevOperator<double> &, const DevGrid<double> &,
                                         const DevGrid<double> *, double, hipStream_t, int);

// ---------------------------------------------------------------------------
// near correction (exact - grid) rows, plus the two triangle halves of every
// edge's grid/local rows; writes the FP64 output rows.  One wave per edge.
// ---------------------------------------------------------------------------
template <typename T> __device__ inline T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Up to NR_MAXB vectors per launch, NRB = their count (no per-vector
// branches): every CSR entry's values are read once, combined into the
// coefficients of J_i, J_e and M of each output row, and applied to all
// vectors, whose currents at the column edge are contiguous (edge-major
// batch copy); the 6 NRB sums are reduced across the wave together.
constexpr int NR_MAXB = 8;
template <typename T, int NRB>
__global__ void __launch_bounds__(256) near_rows_kernel(DevOperator<T> op, double *__restrict__ y) {
  const int n = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (n >= op.ne) return;   // wave-uniform
  const EdgeRec r = op.edges[n];
  const T Ze = op.Z_e, Zi = op.Z_i, iZe = T(1) / op.Z_e, iZi = T(1) / op.Z_i;
  const cx<T> *cur = NRB > 1 ? op.srcI : op.src;   // [m][b][3]
  // v[6 b + (0, 1 | 2, 3 | 4, 5)] = (E | H | eq14 row) of vector b, re and im
  T v[6 * NRB];
#pragma unroll
  for (int q = 0; q < 6 * NRB; q++) v[q] = T(0);
  const int64_t kb = op.rowptr[n], ke = op.rowptr[n + 1];
  // the column indices of this lane's first NR_PRE entries are loaded up
  // front, so only the first entry waits for its index before its currents
  constexpr int NR_PRE = 4;
  int mpre[NR_PRE];
#pragma unroll
  for (int u = 0; u < NR_PRE; u++) mpre[u] = kb + lane + 64 * u < ke ? op.col[kb + lane + 64 * u] : 0;
  int u = 0;
  for (int64_t k = kb + lane; k < ke; k += 64, u++) {
    const int m = u == 0 ? mpre[0] : u == 1 ? mpre[1] : u == 2 ? mpre[2] : u == 3 ? mpre[3] : op.col[k];
    static_assert(NR_PRE == 4, "the selection above names the four prefetched indices");
    const cx<T> Le = op.V4[4 * k], Ke = op.V4[4 * k + 1], Li = op.V4[4 * k + 2], Ki = op.V4[4 * k + 3];
    //   E += Zi Li Ji - Ze Le Je + (Ke + Ki) M
    //   H += Ki Ji - (Ke + Ze Lr) Je + (Kr - Le / Ze - Li / Zi) M
    //   R += Zi Ls Ji + Ks M          (Lr, Kr, Ls, Ks on absorber rows only)
    cx<T> eJi = Li * Zi, eJe = Le * (-Ze), eM = Ke + Ki;
    cx<T> hJi = Ki, hJe = -Ke, hM = Le * (-iZe) - Li * iZi;
    cx<T> rJi = czero<T>(), rM = czero<T>();
    if (r.isR) {
      const cx<T> Lr = op.S4[4 * k], Kr = op.S4[4 * k + 1], Ls = op.S4[4 * k + 2], Ks = op.S4[4 * k + 3];
      hJe = hJe - Lr * Ze;
      hM = hM + Kr;
      rJi = Ls * Zi;
      rM = Ks;
    }
    const cx<T> *cm = cur + (size_t)m * NRB * 3;
#pragma unroll
    for (int b = 0; b < NRB; b++) {
      const cx<T> Je = cm[3 * b], Ji = cm[3 * b + 1], M = cm[3 * b + 2];
      cx<T> e = {v[6 * b], v[6 * b + 1]}, h = {v[6 * b + 2], v[6 * b + 3]}, q = {v[6 * b + 4], v[6 * b + 5]};
      cmac(e, eJi, Ji);
      cmac(e, eJe, Je);
      cmac(e, eM, M);
      cmac(h, hJi, Ji);
      cmac(h, hJe, Je);
      cmac(h, hM, M);
      cmac(q, rJi, Ji);
      cmac(q, rM, M);
      v[6 * b] = e.x;
      v[6 * b + 1] = e.y;
      v[6 * b + 2] = h.x;
      v[6 * b + 3] = h.y;
      v[6 * b + 4] = q.x;
      v[6 * b + 5] = q.y;
    }
  }
  // lane b (b < NRB) ends with the 6 sums of vector b
  T s6[6];
  if constexpr (NRB == 8) {
    // halving exchanges: 48 values -> 3 per lane (values 3 ((L >> 2) & 15) + t
    // summed over the 16 lanes that share L & 3), then the last two lane bits
    halve_exchange_t<T, 24, 32>(v, lane);
    halve_exchange_t<T, 12, 16>(v, lane);
    halve_exchange_t<T, 6, 8>(v, lane);
    halve_exchange_t<T, 3, 4>(v, lane);
#pragma unroll
    for (int t = 0; t < 3; t++) {
      v[t] += __shfl_xor(v[t], 2, 64);
      v[t] += __shfl_xor(v[t], 1, 64);
    }
    // lane 8 b holds values 6 b .. 6 b + 2, lane 8 b + 4 values 6 b + 3 .. 6 b + 5
    const int src_lane = 8 * lane;
#pragma unroll
    for (int t = 0; t < 3; t++) {
      s6[t] = __shfl(v[t], src_lane, 64);
      s6[3 + t] = __shfl(v[t], src_lane + 4, 64);
    }
  } else {
#pragma unroll
    for (int q = 0; q < 6 * NRB; q++) v[q] = wave_sum(v[q]);
#pragma unroll
    for (int t = 0; t < 6; t++) {
      T sel = v[t];
#pragma unroll
      for (int b = 1; b < NRB; b++)
        if (lane == b) sel = v[6 * b + t];
      s6[t] = sel;
    }
  }
  if (lane < NRB) {
    const int b = lane;
    cx<T> e = {s6[0], s6[1]}, h = {s6[2], s6[3]}, rr = {s6[4], s6[5]};
    const cx<T> *to = op.tri_out + (size_t)9 * op.nt * b;
    const cx<T> *p0 = to + ((size_t)r.tri[0] * 3 + r.loc[0]) * 3;
    const cx<T> *p1 = to + ((size_t)r.tri[1] * 3 + r.loc[1]) * 3;
    e += p0[0] + p1[0];
    h += p0[1] + p1[1];
    rr += p0[2] + p1[2];
    if (op.edge_out) {
      const cx<T> *eo = op.edge_out + ((size_t)b * op.ne + n) * 2;
      e += eo[0];
      h += eo[1];
    }
    double *yb = y + (size_t)2 * op.N * b;
    yb[2 * r.row[0]] = e.x;
    yb[2 * r.row[0] + 1] = e.y;
    yb[2 * r.row[1]] = h.x;
    yb[2 * r.row[1] + 1] = h.y;
    if (r.isR) {
      yb[2 * r.row[2]] = rr.x;
      yb[2 * r.row[2] + 1] = rr.y;
    }
  }
}

int near_rows_max_batch() { return NR_MAXB; }

template <typename T> void launch_near_rows(const DevOperator<T> &op, double *y, hipStream_t s, int nb) {
  const int blocks = (int)(((int64_t)op.ne * 64 + 255) / 256);
#define SCABS_NEAR_ROWS(NB) \
  hipLaunchKernelGGL((near_rows_kernel<T, NB>), dim3(blocks), dim3(256), 0, s, op, y)
  switch (nb) {
    case 1: SCABS_NEAR_ROWS(1); break;
    case 2: SCABS_NEAR_ROWS(2); break;
    case 3: SCABS_NEAR_ROWS(3); break;
    case 4: SCABS_NEAR_ROWS(4); break;
    case 5: SCABS_NEAR_ROWS(5); break;
    case 6: SCABS_NEAR_ROWS(6); break;
    case 7: SCABS_NEAR_ROWS(7); break;
    default: SCABS_NEAR_ROWS(8); break;
  }
#undef SCABS_NEAR_ROWS
}
template void launch_near_rows<float>(const DevOperator<float> &, double *, hipStream_t, int);
template void launch_near_rows<double>(const DevOperator<double> &, double *, hipStream_t, int);

// ---------------------------------------------------------------------------
// right-hand side of an electric dipole in the interior medium of one body
// ---------------------------------------------------------------------------
__device__ inline void dipole_fields(double k, double Z, const double *r0, const cx<double> *p, const double *r,
                                     cx<double> *E, cx<double> *H) {
  double d[3] = {r[0] - r0[0], r[1] - r0[1], r[2] - r0[2]};
  double R = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  double u[3] = {d[0] / R, d[1] / R, d[2] / R};
  double sn, cs;
  sincos(k * R, &sn, &cs);
  cx<double> ph = {cs, -sn};                                   // exp(-jkR)
  double c4 = 1.0 / (4.0 * PI);
  cx<double> G = ph * (c4 / R);
  cx<double> G1 = (cx<double>{1.0, k * R} * ph) * (-c4 / (R * R));                       // dG/dR
  cx<double> G2 = (cx<double>{2.0 - k * k * R * R, 2.0 * k * R} * ph) * (c4 / (R * R * R));  // d2G/dR2
  cx<double> up = u[0] * p[0] + u[1] * p[1] + u[2] * p[2];
  // H = grad G x p ; E = -jkZ [p G + k^-2 (G'' (u.p) u + (G'/R)(p - (u.p) u))]
  H[0] = G1 * (u[1] * p[2] - u[2] * p[1]);
  H[1] = G1 * (u[2] * p[0] - u[0] * p[2]);
  H[2] = G1 * (u[0] * p[1] - u[1] * p[0]);
  for (int a = 0; a < 3; a++) {
    cx<double> hp = (G2 * up) * u[a] + (G1 * (1.0 / R)) * (p[a] - up * u[a]);
    cx<double> t = p[a] * G + hp * (1.0 / (k * k));
    E[a] = mul_j(t) * (-k * Z);
  }
}

// complex quotient and principal square root (Re >= 0, cut on the negative axis)
__device__ inline cx<double> cdivd(cx<double> a, cx<double> b) {
  const double den = b.x * b.x + b.y * b.y;
  return {(a.x * b.x + a.y * b.y) / den, (a.y * b.x - a.x * b.y) / den};
}
__device__ inline cx<double> csqrtd(cx<double> z) {
  const double r = hypot(z.x, z.y);
  const double re = sqrt(0.5 * (r + z.x)), im = sqrt(0.5 * fmax(r - z.x, 0.0));
  return {re, z.y < 0 ? -im : im};
}

// Fields of a source (SourceDev) in the medium (k, Z): b = 0 the point
// dipole above; b > 0 the same closed form continued to the complex source
// position r0 - j b dir (a complex-source-point beam along +dir with its
// waist at r0): complex distance R = sqrt(d.d), d = r - r0 + j b dir,
// principal branch, complex unit vector u = d / R, all times exp(-k b) so
// that the beam's on-axis amplitude stays of order one.
__device__ inline void source_fields(const SourceDev &S, double k, double Z, const double *r, cx<double> *E,
                                     cx<double> *H) {
  if (S.b == 0.0) {
    dipole_fields(k, Z, S.r0, S.p, r, E, H);
    return;
  }
  const cx<double> d[3] = {{r[0] - S.r0[0], S.bd[0]}, {r[1] - S.r0[1], S.bd[1]}, {r[2] - S.r0[2], S.bd[2]}};
  const cx<double> R = csqrtd(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  const cx<double> u[3] = {cdivd(d[0], R), cdivd(d[1], R), cdivd(d[2], R)};
  // exp(-jkR - kb)
  const double mag = exp(k * R.y - k * S.b);
  double sn, cs;
  sincos(-k * R.x, &sn, &cs);
  const cx<double> ph = {mag * cs, mag * sn};
  const double c4 = 1.0 / (4.0 * PI);
  const cx<double> kR = R * k, R2 = R * R, R3 = R2 * R;
  const cx<double> G = cdivd(ph * c4, R);
  const cx<double> G1 = cdivd((cx<double>{1.0, 0.0} + mul_j(kR)) * ph, R2) * (-c4);
  const cx<double> G2 = cdivd((cx<double>{2.0, 0.0} + mul_j(kR) * 2.0 - kR * kR) * ph, R3) * c4;
  const cx<double> up = u[0] * S.p[0] + u[1] * S.p[1] + u[2] * S.p[2];
  H[0] = G1 * (u[1] * S.p[2] - u[2] * S.p[1]);
  H[1] = G1 * (u[2] * S.p[0] - u[0] * S.p[2]);
  H[2] = G1 * (u[0] * S.p[1] - u[1] * S.p[0]);
  const cx<double> G1R = cdivd(G1, R);
  for (int a = 0; a < 3; a++) {
    const cx<double> hp = G2 * up * u[a] + G1R * (S.p[a] - up * u[a]);
    const cx<double> t = S.p[a] * G + hp * (1.0 / (k * k));
    E[a] = mul_j(t) * (-k * Z);
  }
}

__global__ void rhs_dipole_kernel(int nt, const int *__restrict__ body, const TriRec<double> *__restrict__ tris,
                                  const PointRec<double> *__restrict__ pts, const double *__restrict__ qp,
                                  const EdgeRec *__restrict__ edges, double k, double Z, SourceDev S, int bodyid,
                                  double *b) {
  int T = blockIdx.x * blockDim.x + threadIdx.x;
  if (T >= nt || body[T] != bodyid) return;
  cx<double> acc[3][3];
  for (int i = 0; i < 3; i++) acc[i][0] = acc[i][1] = acc[i][2] = czero<double>();
  for (int q = 0; q < NQ; q++) {
    const PointRec<double> &P = pts[T * NQ + q];
    cx<double> E[3], H[3];
    source_fields(S, k, Z, qp + 3 * ((size_t)T * NQ + q), E, H);
    for (int i = 0; i < 3; i++) {
      const double *gi = P.f + 3 * i;
      cx<double> ge = rdot(gi, E), gh = rdot(gi, H);
      axpy(acc[i][0], P.w, ge);
      axpy(acc[i][1], P.w, gh);
      axpy(acc[i][2], P.w * P.sigma, ge);
    }
  }
  const TriRec<double> tr = tris[T];
  for (int i = 0; i < 3; i++) {
    const EdgeRec r = edges[tr.edge[i]];
    for (int s = 0; s < 3; s++) {
      if (r.row[s] < 0) continue;
      atomicAdd(&b[2 * r.row[s]], acc[i][s].x);
      atomicAdd(&b[2 * r.row[s] + 1], acc[i][s].y);
    }
  }
}

// incident field of the source at every quadrature point of its body (zero on
// the other bodies)
__global__ void incident_points_kernel(int np, const int *__restrict__ body, const PointRec<double> *__restrict__ pts,
                                       const double *__restrict__ qp, double k, double Z, SourceDev S, int bodyid,
                                       cx<double> *__restrict__ E) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  cx<double> e[3] = {{0, 0}, {0, 0}, {0, 0}}, h[3];
  if (body[pts[p].tri] == bodyid) source_fields(S, k, Z, qp + 3 * (size_t)p, e, h);
  for (int a = 0; a < 3; a++) E[3 * (size_t)p + a] = e[a];
}

void launch_incident_points(int np, const int *body, const PointRec<double> *pts, const double *qp, double k, double Z,
                            const SourceDev &S, int bodyid, cx<double> *E, hipStream_t s) {
  hipLaunchKernelGGL(incident_points_kernel, dim3((np + 255) / 256), dim3(256), 0, s, np, body, pts, qp, k, Z, S,
                     bodyid, E);
}

// the source's fields (interior medium) at arbitrary points, 3 complex per point
__global__ void dipole_points_kernel(int npts, const double *__restrict__ pts, double k, double Z, SourceDev S,
                                     cx<double> *__restrict__ E, cx<double> *__restrict__ H) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npts) return;
  cx<double> e[3], h[3];
  source_fields(S, k, Z, pts + 3 * (size_t)p, e, h);
  for (int a = 0; a < 3; a++) {
    E[3 * (size_t)p + a] = e[a];
    H[3 * (size_t)p + a] = h[a];
  }
}

void launch_dipole_points(int npts, const double *pts, double k, double Z, const SourceDev &S, cx<double> *E,
                          cx<double> *H, hipStream_t s) {
  hipLaunchKernelGGL(dipole_points_kernel, dim3((npts + 255) / 256), dim3(256), 0, s, npts, pts, k, Z, S, E, H);
}

void launch_rhs_dipole(int nt, const double *qp, const int *body, const TriRec<double> *tris,
                       const PointRec<double> *pts, const EdgeRec *edges, double k, double Z, const SourceDev &S,
                       int bodyid, double *b, hipStream_t s) {
  hipLaunchKernelGGL(rhs_dipole_kernel, dim3((nt + 127) / 128), dim3(128), 0, s, nt, body, tris, pts, qp, edges, k, Z,
                     S, bodyid, b);
}

}  // namespace scabs
