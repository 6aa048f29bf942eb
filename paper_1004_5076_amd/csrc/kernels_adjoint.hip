// Transposed product y = A~^T z of the precorrected-FFT operator, the
// transposed Schwarz preconditioner, and the pointwise one-sided fields and
// sigma derivative used by the adjoint gradient.
//
// A~ = (test) G (source) + (near correction) + (local terms).  The lattice
// convolution G is symmetric (the sampled kernel is even), so
//   A~^T z = source^T G test^T z + near^T z + local^T z,
// where test^T turns the row weights z at every test point into lattice
// sources with both value weights W and derivative weights grad W (the
// forward testing reads potentials through both), and source^T reads the
// convolved lattice with W at the source points and hands the result back to
// the half-RWG currents.  The near transpose walks the same edge-pair CSR
// (the near list is symmetric) reading the entry of the mirrored pair.
#include <algorithm>

#include "device_common.h"
#include "kernels.h"
#include "near_math.h"

namespace scabs {

// ---------------------------------------------------------------------------
// row-space vector -> per-edge row weights (z_E, z_H, z_14); z_14 = 0 on
// sigma-free edges
// ---------------------------------------------------------------------------
template <typename T>
__global__ void unpack_rows_kernel(const EdgeRec *__restrict__ edges, int ne, const double *__restrict__ z,
                                   cx<T> *__restrict__ dst) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const EdgeRec r = edges[e];
  dst[3 * e] = {(T)z[2 * r.row[0]], (T)z[2 * r.row[0] + 1]};
  dst[3 * e + 1] = {(T)z[2 * r.row[1]], (T)z[2 * r.row[1] + 1]};
  dst[3 * e + 2] = r.isR ? cx<T>{(T)z[2 * r.row[2]], (T)z[2 * r.row[2] + 1]} : czero<T>();
}

template <typename T> void launch_unpack_rows(const DevOperator<T> &op, const double *z, hipStream_t s) {
  hipLaunchKernelGGL(unpack_rows_kernel<T>, dim3((op.ne + 255) / 256), dim3(256), 0, s, op.edges, op.ne, z, op.src);
}
template void launch_unpack_rows<float>(const DevOperator<float> &, const double *, hipStream_t);
template void launch_unpack_rows<double>(const DevOperator<double> &, const double *, hipStream_t);

// ---------------------------------------------------------------------------
// test^T, step 1: per point (in the grid's cell-sorted order) the coefficients
// that the forward rows give to each potential field's value and gradient.
// With t_E = sum z_E f, t_H = sum z_H f, d_E = sum z_E div f, d_H = sum z_H div f
// and the sigma vector s (exterior: w sigma sum z_H (f x n); interior:
// -w sigma sum z_14 f), the rows read
//   a_J: -Z jk (sgn w t_E + s)      phi_J: sgn w Z jk d_E / k^2
//   a_M: -(jk/Z) sgn w t_H          phi_M: (jk/Z) sgn w d_H / k^2
//   curl a_J . (sgn w t_H)           curl a_M . (-(sgn w t_E + s))
//   grad phi_J . (-Z jk s / k^2)
// and the gradient coefficient of component c inside v . curl a is e_c x v.
// Output per point (ADJ_COEF): the 8 value coefficients, then vJ, vM and the
// gradient vector of phi_J; the lattice node at weight W then receives
// W c + (grad W) . (gradient coefficients), i.e. -(grad W x vJ) on a_J,
// grad W . gp on phi_J and -(grad W x vM) on a_M.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
adj_sources_kernel(const PointRec<T> *__restrict__ pts, const TriRec<T> *__restrict__ tris,
                   const cx<T> *__restrict__ zr, GatherGrid<T> g, cx<T> *__restrict__ out, T k, T Z, int interior) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.np) return;
  const PointRec<T> P = pts[g.perm[i]];
  const TriRec<T> tr = tris[P.tri];
  const T n[3] = {tr.nrm[0], tr.nrm[1], tr.nrm[2]};
  const T w = P.w, ws = P.w * P.sigma, sgn = interior ? T(-1) : T(1);
  cx<T> tE[3], tH[3], sv[3], dE = czero<T>(), dH = czero<T>();
#pragma unroll
  for (int a = 0; a < 3; a++) tE[a] = tH[a] = sv[a] = czero<T>();
#pragma unroll
  for (int j = 0; j < 3; j++) {
    const int e = tr.edge[j];
    const cx<T> zE = zr[3 * e], zH = zr[3 * e + 1], z14 = zr[3 * e + 2];
    const T f[3] = {P.f[3 * j], P.f[3 * j + 1], P.f[3 * j + 2]};
    const T fxn[3] = {f[1] * n[2] - f[2] * n[1], f[2] * n[0] - f[0] * n[2], f[0] * n[1] - f[1] * n[0]};
#pragma unroll
    for (int a = 0; a < 3; a++) {
      axpy(tE[a], f[a], zE);
      axpy(tH[a], f[a], zH);
      if (interior)
        axpy(sv[a], -ws * f[a], z14);
      else
        axpy(sv[a], ws * fxn[a], zH);
    }
    axpy(dE, tr.div[j], zE);
    axpy(dH, tr.div[j], zH);
  }
  cx<T> cv[8], vJ[3], vM[3], gp[3];
#pragma unroll
  for (int a = 0; a < 3; a++) {
    cx<T> te = sgn * w * tE[a] + sv[a];
    cv[a] = mul_j(te) * (-Z * k);
    cv[4 + a] = mul_j(tH[a]) * (-(k / Z) * sgn * w);
    vJ[a] = (sgn * w) * tH[a];
    vM[a] = -te;
    gp[a] = mul_j(sv[a]) * (-Z / k);
  }
  cv[3] = mul_j(dE) * (sgn * w * Z / k);
  cv[7] = mul_j(dH) * (sgn * w / (Z * k));
  cx<T> *o = out + (size_t)ADJ_COEF * i;
#pragma unroll
  for (int f = 0; f < 8; f++) o[f] = cv[f];
#pragma unroll
  for (int a = 0; a < 3; a++) {
    o[8 + a] = vJ[a];
    o[11 + a] = vM[a];
    o[14 + a] = gp[a];
  }
}

// test^T, step 2: every node sums, over the points of its 27 neighbouring
// cells, W c_value + grad W . (gradient coefficients) per field.  Same
// organisation as the forward projection: per x plane, phase A over (cell,
// node offset) items of the nonempty cells of planes x-1..x+1, phase B over
// (node, x offset) items through the cell -> slot map, x partials added last.
template <typename T> struct CellChunkT { static constexpr int value = 96; };
template <> struct CellChunkT<double> { static constexpr int value = 48; };

// one point's contribution to the node at offset (ox, oy, oz) from its anchor:
// W c_value, -(grad W x vJ) on a_J, grad W . gp on phi_J, -(grad W x vM) on a_M
template <typename T>
__device__ __forceinline__ void adj_point(cx<T> *a, const cx<T> *c, const T *u, int ox, int oy, int oz, T inv_h) {
  const T ux = u[0], uy = u[1], uz = u[2];
  const T Lx = lag_w(ox, ux), Ly = lag_w(oy, uy), Lz = lag_w(oz, uz);
  const T W = Lx * Ly * Lz, Wx = lag_d(ox, ux) * Ly * Lz * inv_h, Wy = Lx * lag_d(oy, uy) * Lz * inv_h,
          Wz = Lx * Ly * lag_d(oz, uz) * inv_h;
#pragma unroll
  for (int f = 0; f < 8; f++) axpy(a[f], W, c[f]);
  axpy(a[0], -Wy, c[10]);
  axpy(a[0], Wz, c[9]);
  axpy(a[1], -Wz, c[8]);
  axpy(a[1], Wx, c[10]);
  axpy(a[2], -Wx, c[9]);
  axpy(a[2], Wy, c[8]);
  axpy(a[4], -Wy, c[13]);
  axpy(a[4], Wz, c[12]);
  axpy(a[5], -Wz, c[11]);
  axpy(a[5], Wx, c[13]);
  axpy(a[6], -Wx, c[12]);
  axpy(a[6], Wy, c[11]);
  axpy(a[3], Wx, c[14]);
  axpy(a[3], Wy, c[15]);
  axpy(a[3], Wz, c[16]);
}

template <typename T, int MAXI>
__global__ void __launch_bounds__(1024)
gather_adj_kernel(DevGrid<T> dg, GatherGrid<T> g, const cx<T> *__restrict__ src4, T inv_h) {
  constexpr int SC = CellChunkT<T>::value, SQ = 9 * SC;
  static_assert(8 * SQ >= 3 * 1024, "the final reduction reuses s_q for 3 planes of at most 1024 nodes");
  __shared__ cx<T> s_q[8][SQ];
  extern __shared__ __align__(16) int s_map[];
  const int n0 = dg.n[0], n1 = dg.n[1], n2 = dg.n[2];
  const int plane = n1 * n2;
  const int x = xcd_remap(blockIdx.x, gridDim.x);   // neighbouring planes on one XCD
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
        // two points' loads in flight (FP32; FP64 would spill)
        for (; sizeof(T) == 4 && p + 2 <= p1; p += 2) {
          cx<T> c0[ADJ_COEF], c1[ADJ_COEF];
#pragma unroll
          for (int f = 0; f < ADJ_COEF; f++) {
            c0[f] = src4[(size_t)ADJ_COEF * p + f];
            c1[f] = src4[(size_t)ADJ_COEF * (p + 1) + f];
          }
          adj_point(a, c0, g.u + 3 * p, ox, oy, oz, inv_h);
          adj_point(a, c1, g.u + 3 * p + 3, ox, oy, oz, inv_h);
        }
        for (; p < p1; p++) adj_point(a, src4 + (size_t)ADJ_COEF * p, g.u + 3 * p, ox, oy, oz, inv_h);
      }
#pragma unroll
      for (int f = 0; f < 8; f++) s_q[f][it] = a[f];
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < MAXI; m++) {
      int oxi, nd;
      if constexpr (MAXI == 1) {
        // 21 nodes per wave, their three x offsets in neighbouring lanes
        const int ln = threadIdx.x & 63;
        oxi = ln % 3;
        nd = (threadIdx.x >> 6) * GB_NODES_PER_WAVE + ln / 3;
        if (ln >= 3 * GB_NODES_PER_WAVE || nd >= plane) continue;
      } else {
        const int it = threadIdx.x + m * blockDim.x;
        if (it >= 3 * plane) continue;
        oxi = fdiv(it, dpl);
        nd = it - oxi * plane;
      }
      const int cxp = x - (oxi - 1);
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
      if (own) dg.phys[f * G + (size_t)x * plane + nd] = v + v1 + v2;
    }
    return;
  }
  cx<T> *s_red = &s_q[0][0];
  for (int f = 0; f < 8; f++) {
#pragma unroll
    for (int m = 0; m < MAXI; m++) {
      const int it = threadIdx.x + m * blockDim.x;
      if (it < 3 * plane) s_red[it] = acc[m][f];
    }
    __syncthreads();
    for (int nd = threadIdx.x; nd < plane; nd += blockDim.x)
      dg.phys[f * G + (size_t)x * plane + nd] = s_red[nd] + s_red[plane + nd] + s_red[2 * plane + nd];
    __syncthreads();
  }
}

template <typename T>
void launch_test_t(const DevOperator<T> &op, const std::vector<DevGrid<T>> &grids, const std::vector<GatherGrid<T>> &gg,
                   const std::vector<cx<T> *> &src4, T inv_h, hipStream_t s) {
  for (size_t k = 0; k < grids.size(); k++) {
    const GatherGrid<T> &g = gg[k];
    hipLaunchKernelGGL(adj_sources_kernel<T>, dim3((g.np + 255) / 256), dim3(256), 0, s, op.pts, op.tris, op.src, g,
                       src4[k], grids[k].k, grids[k].Z, grids[k].which >= 0 ? 1 : 0);
  }
  for (size_t k = 0; k < grids.size(); k++) {
    const int plane = grids[k].n[1] * grids[k].n[2];
    const int items = 3 * plane;
    int threads = std::min(1024, (items + 63) / 64 * 64);
    int maxi = (items + threads - 1) / threads;
    // one pass over the nodes in lane triples when they fit one work-group
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
    if (maxi == 1)
      hipLaunchKernelGGL((gather_adj_kernel<T, 1>), dim3(grids[k].n[0]), dim3(threads), lds, s, grids[k], gg[k],
                         src4[k], inv_h);
    else if (maxi == 2)
      hipLaunchKernelGGL((gather_adj_kernel<T, 2>), dim3(grids[k].n[0]), dim3(threads), lds, s, grids[k], gg[k],
                         src4[k], inv_h);
    else
      hipLaunchKernelGGL((gather_adj_kernel<T, 3>), dim3(grids[k].n[0]), dim3(threads), lds, s, grids[k], gg[k],
                         src4[k], inv_h);
  }
}
template void launch_test_t<float>(const DevOperator<float> &, const std::vector<DevGrid<float>> &,
                                   const std::vector<GatherGrid<float>> &, const std::vector<cx<float> *> &, float,
                                   hipStream_t);
template void launch_test_t<double>(const DevOperator<double> &, const std::vector<DevGrid<double>> &,
                                    const std::vector<GatherGrid<double>> &, const std::vector<cx<double> *> &, double,
                                    hipStream_t);

// ---------------------------------------------------------------------------
// source^T and local^T: at every point the convolved lattice values of the
// exterior grid and of the point's own interior grid (W only), handed to the
// three half-RWG currents (J_e, J_i, M) of its triangle, plus the transposed
// point-local terms:  H residue -1/2 <f, n x (J_e + J_i)>, Gram <f, J_e + J_i>
// on eq14 rows, and the 1/2 n x M residue inside the sigma-weighted tests.
// Per-triangle half-edge partials (3 currents per half-edge) in tri_out.
// ---------------------------------------------------------------------------
constexpr int IA_TRIS = 32;
constexpr int IA_THREADS = IA_TRIS * NQ;

template <typename T>
__device__ inline void gather_vals(const DevGrid<T> &g, int ax, int ay, int az, const T *Lx, const T *Ly, const T *Lz,
                                   cx<T> *val) {
#pragma unroll
  for (int f = 0; f < 8; f++) val[f] = czero<T>();
  const int n1 = g.n[1], n2 = g.n[2];
  const size_t G = (size_t)g.n[0] * n1 * n2;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      const size_t row = ((size_t)(ax + i - 1) * n1 + (ay + j - 1)) * n2 + (az - 1);
      const T wxy = Lx[i] * Ly[j];
#pragma unroll
      for (int k = 0; k < 3; k++) {
        const T w = wxy * Lz[k];
#pragma unroll
        for (int f = 0; f < 8; f++) axpy(val[f], w, g.phys[f * G + row + k]);
      }
    }
}

template <typename T>
__global__ void __launch_bounds__(IA_THREADS)
interp_adj_kernel(DevOperator<T> op, DevGrid<T> ext, const DevGrid<T> *__restrict__ ints) {
  __shared__ cx<T> part[IA_THREADS][9];
  const int lt = threadIdx.x / NQ, q = threadIdx.x - lt * NQ;
  const int tri = blockIdx.x * IA_TRIS + lt;
  cx<T> out[9];
#pragma unroll
  for (int r = 0; r < 9; r++) out[r] = czero<T>();
  if (tri < op.nt) {
    const PointRec<T> P = op.pts[tri * NQ + q];
    const TriRec<T> tr = op.tris[tri];
    const T n[3] = {tr.nrm[0], tr.nrm[1], tr.nrm[2]};
    const T w = P.w, ws = P.w * P.sigma;
    cx<T> tH[3], tR[3];
    for (int a = 0; a < 3; a++) tH[a] = tR[a] = czero<T>();
    for (int j = 0; j < 3; j++) {
      const int e = tr.edge[j];
      const cx<T> zH = op.src[3 * e + 1], z14 = op.src[3 * e + 2];
      for (int a = 0; a < 3; a++) {
        axpy(tH[a], P.f[3 * j + a], zH);
        axpy(tR[a], P.f[3 * j + a], z14);
      }
    }
    // coefficient vectors of J_e + J_i and of M at the point
    cx<T> hxn[3], rxn[3], aJs[3], aMq[3];
    hxn[0] = tH[1] * n[2] - tH[2] * n[1];
    hxn[1] = tH[2] * n[0] - tH[0] * n[2];
    hxn[2] = tH[0] * n[1] - tH[1] * n[0];
    rxn[0] = tR[1] * n[2] - tR[2] * n[1];
    rxn[1] = tR[2] * n[0] - tR[0] * n[2];
    rxn[2] = tR[0] * n[1] - tR[1] * n[0];
    const cx<T> hxnxn[3] = {hxn[1] * n[2] - hxn[2] * n[1], hxn[2] * n[0] - hxn[0] * n[2],
                            hxn[0] * n[1] - hxn[1] * n[0]};
    for (int a = 0; a < 3; a++) {
      aJs[a] = (T(-0.5) * w) * hxn[a] + w * tR[a];
      aMq[a] = (T(0.5) * ws) * (hxnxn[a] - rxn[a]);
    }
    T Lx[3], Ly[3], Lz[3], dLx[3], dLy[3], dLz[3];
    lagr3(P.u[0], Lx, dLx);
    lagr3(P.u[1], Ly, dLy);
    lagr3(P.u[2], Lz, dLz);
    int ax, ay, az;
    unpack_anchor(P.anc, ax, ay, az);
    cx<T> ve[8], vi[8];
    gather_vals(ext, ax - ext.off[0], ay - ext.off[1], az - ext.off[2], Lx, Ly, Lz, ve);
    const DevGrid<T> &gi = ints[tr.body];
    gather_vals(gi, ax - gi.off[0], ay - gi.off[1], az - gi.off[2], Lx, Ly, Lz, vi);
    for (int j = 0; j < 3; j++) {
      const T f[3] = {P.f[3 * j], P.f[3 * j + 1], P.f[3 * j + 2]};
      const T dv = tr.div[j];
      cx<T> fl = f[0] * aJs[0];
      axpy(fl, f[1], aJs[1]);
      axpy(fl, f[2], aJs[2]);
      cx<T> fm = f[0] * aMq[0];
      axpy(fm, f[1], aMq[1]);
      axpy(fm, f[2], aMq[2]);
      cx<T> je = dv * ve[3], ji = dv * vi[3], me = dv * ve[7], mi = dv * vi[7];
      for (int a = 0; a < 3; a++) {
        axpy(je, f[a], ve[a]);
        axpy(ji, f[a], vi[a]);
        axpy(me, f[a], ve[4 + a]);
        axpy(mi, f[a], vi[4 + a]);
      }
      out[3 * j] = w * je + fl;
      out[3 * j + 1] = w * ji + fl;
      out[3 * j + 2] = w * (me - mi) + fm;
    }
  }
#pragma unroll
  for (int r = 0; r < 9; r++) part[threadIdx.x][r] = out[r];
  __syncthreads();
  for (int it = threadIdx.x; it < IA_TRIS * 9; it += blockDim.x) {
    const int l = it / 9, r = it - l * 9;
    const int t2 = blockIdx.x * IA_TRIS + l;
    if (t2 < op.nt) {
      cx<T> s = czero<T>();
      for (int qq = 0; qq < NQ; qq++) s += part[l * NQ + qq][r];
      op.tri_out[(size_t)t2 * 9 + r] = s;
    }
  }
}

template <typename T>
void launch_interp_adj(const DevOperator<T> &op, const DevGrid<T> &ext, const DevGrid<T> *ints_dev, hipStream_t s) {
  hipLaunchKernelGGL(interp_adj_kernel<T>, dim3((op.nt + IA_TRIS - 1) / IA_TRIS), dim3(IA_THREADS), 0, s, op, ext,
                     ints_dev);
}
template void launch_interp_adj<float>(const DevOperator<float> &, const DevGrid<float> &, const DevGrid<float> *,
                                       hipStream_t);
template void launch_interp_adj<double>(const DevOperator<double> &, const DevGrid<double> &,
                                        const DevGrid<double> *, hipStream_t);

// ---------------------------------------------------------------------------
// near^T: one wave per column edge m.  Row n of the forward correction adds
//   E_n += Z_i L_i J_i - Z_e L_e J_e + (K_e + K_i) M
//   H_n += K_i J_i - K_e J_e - (L_e/Z_e + L_i/Z_i) M + K_r M - Z_e L_r J_e
//   14_n += Z_i L_s J_i + K_s M
// (the last four values vanish on sigma-free rows), so m's currents collect
// the same coefficients against (z_E, z_H, z_14) of every row n near m, read
// at the mirrored CSR entry tpos.  Adds the two triangle halves of m and maps
// (J_e, J_i, M) to m's unknowns (sigma-free: J_e = J, J_i = -J).
// ---------------------------------------------------------------------------
template <typename T> __device__ inline T wsum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename T>
__global__ void __launch_bounds__(256)
near_rows_t_kernel(DevOperator<T> op, const int64_t *__restrict__ tpos, double *__restrict__ y) {
  const int m = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (m >= op.ne) return;
  const EdgeRec r = op.edges[m];
  const T Ze = op.Z_e, Zi = op.Z_i, iZe = T(1) / op.Z_e, iZi = T(1) / op.Z_i;
  cx<T> aJe = czero<T>(), aJi = czero<T>(), aM = czero<T>();
  const int64_t b = op.rowptr[m], e = op.rowptr[m + 1];
  // mirrored values: row-ordered copies where they exist, else through tpos
  const bool mirrored = op.V4T != nullptr;
  const cx<T> *V4 = mirrored ? op.V4T : op.V4, *S4 = mirrored ? op.S4T : op.S4;
  // the column indices of this lane's first four entries are loaded up front
  int npre[4];
#pragma unroll
  for (int u = 0; u < 4; u++) npre[u] = b + lane + 64 * u < e ? op.col[b + lane + 64 * u] : 0;
  int u = 0;
  for (int64_t k = b + lane; k < e; k += 64, u++) {
    const int n = u == 0 ? npre[0] : u == 1 ? npre[1] : u == 2 ? npre[2] : u == 3 ? npre[3] : op.col[k];
    const int64_t t = mirrored ? k : tpos[k];
    const cx<T> zE = op.src[3 * n], zH = op.src[3 * n + 1], z14 = op.src[3 * n + 2];
    const cx<T> Le = V4[4 * t], Ke = V4[4 * t + 1], Li = V4[4 * t + 2], Ki = V4[4 * t + 3];
    const cx<T> Lr = S4[4 * t], Kr = S4[4 * t + 1], Ls = S4[4 * t + 2], Ks = S4[4 * t + 3];
    aJe -= (Le * zE) * Ze + Ke * zH + (Lr * zH) * Ze;
    aJi += (Li * zE) * Zi + Ki * zH + (Ls * z14) * Zi;
    aM += (Ke + Ki) * zE - (Le * zH) * iZe - (Li * zH) * iZi + Kr * zH + Ks * z14;
  }
  aJe.x = wsum(aJe.x);
  aJe.y = wsum(aJe.y);
  aJi.x = wsum(aJi.x);
  aJi.y = wsum(aJi.y);
  aM.x = wsum(aM.x);
  aM.y = wsum(aM.y);
  if (lane == 0) {
    const cx<T> *p0 = op.tri_out + ((size_t)r.tri[0] * 3 + r.loc[0]) * 3;
    const cx<T> *p1 = op.tri_out + ((size_t)r.tri[1] * 3 + r.loc[1]) * 3;
    aJe += p0[0] + p1[0];
    aJi += p0[1] + p1[1];
    aM += p0[2] + p1[2];
    if (!r.isR) {
      const cx<T> j = aJe - aJi;
      y[2 * r.col[0]] = j.x;
      y[2 * r.col[0] + 1] = j.y;
      y[2 * r.col[1]] = aM.x;
      y[2 * r.col[1] + 1] = aM.y;
    } else {
      y[2 * r.col[0]] = aJe.x;
      y[2 * r.col[0] + 1] = aJe.y;
      y[2 * r.col[1]] = aJi.x;
      y[2 * r.col[1] + 1] = aJi.y;
      y[2 * r.col[2]] = aM.x;
      y[2 * r.col[2] + 1] = aM.y;
    }
  }
}

template <typename T>
void launch_near_rows_t(const DevOperator<T> &op, const int64_t *tpos, double *y, hipStream_t s) {
  int blocks = (int)(((int64_t)op.ne * 64 + 255) / 256);
  hipLaunchKernelGGL(near_rows_t_kernel<T>, dim3(blocks), dim3(256), 0, s, op, tpos, y);
}
template void launch_near_rows_t<float>(const DevOperator<float> &, const int64_t *, double *, hipStream_t);

__global__ void mirror4_kernel(int64_t nnz, const int64_t *__restrict__ tpos, const cx<float> *__restrict__ src,
                               cx<float> *__restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 4 * nnz) return;
  const int64_t k = i >> 2;
  dst[i] = src[4 * tpos[k] + (i & 3)];
}

void launch_mirror4(int64_t nnz, const int64_t *tpos, const cx<float> *src, cx<float> *dst, hipStream_t s) {
  if (nnz == 0) return;
  hipLaunchKernelGGL(mirror4_kernel, dim3((unsigned)((4 * nnz + 255) / 256)), dim3(256), 0, s, nnz, tpos, src, dst);
}
template void launch_near_rows_t<double>(const DevOperator<double> &, const int64_t *, double *, hipStream_t);

// ---------------------------------------------------------------------------
// transposed Schwarz preconditioner: y = sum_c R_ext^T B_c^T P_core x with
// B_c the stored core rows of cluster c's inverse.  Step 1: x is copied into
// core order (the cores partition the unknowns, so this is a permutation).
// Step 2: one work-group per (cluster, block of PT_COLS ext columns); each
// wave forms dot(B_c[:, j], x[core_c]) for PT_WCOLS columns j at once, lanes
// over rows (every stored column read once, contiguously, PT_WCOLS loads in
// flight per row block, the core-ordered x read from L2), then reduces the
// 2 PT_WCOLS partial sums across the wave in one halving exchange.  Step 3:
// every unknown sums its entries over the clusters whose ext set holds it
// (fixed order, no atomics).
// ---------------------------------------------------------------------------
constexpr int PT_COLS = 64;
constexpr int PT_THREADS = 512;
constexpr int PT_WCOLS = PT_COLS / (PT_THREADS / 64);   // columns per wave
static_assert(PT_WCOLS == 8, "the wave reduction below is written for 8 columns (16 values)");
int precond_t_cols_per_item() { return PT_COLS; }

// x in FP64, or in FP32 straight from the inner solves' basis (widened here)
template <typename TI>
__global__ void precond_t_gather_kernel(int64_t n, const int *__restrict__ core_slot, const cx<TI> *__restrict__ x,
                                        cx<double> *__restrict__ xc) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) {
    const cx<TI> v = x[core_slot[p]];
    xc[p] = {(double)v.x, (double)v.y};
  }
}

// at most 64 VGPRs (8 waves per SIMD, more coefficient loads in flight): 4%
// faster than the 90 the compiler picks unbounded, with no spills
__global__ void __launch_bounds__(PT_THREADS, 8)
precond_t_dots_kernel(const int *__restrict__ items, const int64_t *__restrict__ ext_ptr,
                      const int64_t *__restrict__ core_ptr, const int64_t *__restrict__ r_off, PcStore pc,
                      const cx<double> *__restrict__ xc, cx<double> *__restrict__ tmp) {
  // items are listed in dispatch order: the host keeps a cluster's items on
  // one XCD (its L2 then serves the cluster's core-ordered x to all of them)
  const int item = blockIdx.x;
  const int c = items[2 * item], j0 = items[2 * item + 1];
  if (c < 0) return;   // padding entry
  const int64_t e0 = ext_ptr[c];
  const int ne = (int)(ext_ptr[c + 1] - e0);
  const int ncore = (int)(core_ptr[c + 1] - core_ptr[c]);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int jw = j0 + w * PT_WCOLS;
  const int nj = min(PT_WCOLS, ne - jw);   // wave-uniform
  if (nj <= 0) return;
  const int64_t ncp = rt_stride(ncore);
  const cx<double> *xcc = xc + core_ptr[c];
  // the wave's 8 columns are one stored block (jw is a multiple of 8): each
  // lane reads its row's 8 coefficients, 32 contiguous bytes (padding columns
  // past the last hold zeros and are never written)
  static_assert(PT_WCOLS == RT_CB, "one stored column block per wave");
  const uint4 *Rb = reinterpret_cast<const uint4 *>(pc.R + r_off[c] + (int64_t)(jw / RT_CB) * (ncp * RT_CB));
  double v[2 * PT_WCOLS];
#pragma unroll
  for (int k = 0; k < 2 * PT_WCOLS; k++) v[k] = 0.0;
  auto row = [&](const uint4 c0, const uint4 c1, const cx<double> xv) {
    const uint32_t wd[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
#pragma unroll
    for (int u = 0; u < PT_WCOLS; u++) {
      const cx<float> rv = unpack_h2(wd[u]);
      v[2 * u] = fma((double)rv.x, xv.x, v[2 * u]);
      v[2 * u] = fma(-(double)rv.y, xv.y, v[2 * u]);
      v[2 * u + 1] = fma((double)rv.x, xv.y, v[2 * u + 1]);
      v[2 * u + 1] = fma((double)rv.y, xv.x, v[2 * u + 1]);
    }
  };
  // two row blocks per step: 64 bytes of coefficients in flight per lane
  int i = lane;
  for (; i + 64 < ncore; i += 128) {
    const uint4 a0 = Rb[2 * i], a1 = Rb[2 * i + 1], b0 = Rb[2 * (i + 64)], b1 = Rb[2 * (i + 64) + 1];
    const cx<double> xa = xcc[i], xb = xcc[i + 64];
    row(a0, a1, xa);
    row(b0, b1, xb);
  }
  if (i < ncore) row(Rb[2 * i], Rb[2 * i + 1], xcc[i]);
  const double t = wsum16_scatter(v);
  const int k = (lane >> 2) & 15, u = k >> 1;
  // lanes 0, 8, 16, ... hold the real parts, lanes 4, 12, ... the imaginary parts
  const double other = __shfl_down(t, 4, 64);
  if ((lane & 7) == 0 && u < nj) {
    const double sc = pc.scale[e0 + jw + u];
    tmp[e0 + jw + u] = {t * sc, other * sc};
  }
}

__global__ void precond_t_sum_kernel(int64_t N, const int64_t *__restrict__ inv_ptr, const int64_t *__restrict__ inv_pos,
                                     const cx<double> *__restrict__ tmp, cx<double> *__restrict__ y) {
  for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < N; u += (int64_t)gridDim.x * blockDim.x) {
    cx<double> s = {0.0, 0.0};
    for (int64_t p = inv_ptr[u]; p < inv_ptr[u + 1]; p++) s += tmp[inv_pos[p]];
    y[u] = s;
  }
}

// xc: n_core entries of work space (x in core order; n_core = N when the
// cores cover every unknown, fewer when the clusters cover a subset); y: all
// N rows written (zero outside the cores)
template <typename TI>
void launch_precond_apply_t(int n_items, const int *items, int64_t N, int64_t n_core, const int64_t *ext_ptr,
                            const int64_t *core_ptr, const int *core_slot, const int64_t *r_off, PcStore pc,
                            const int64_t *inv_ptr, const int64_t *inv_pos, cx<double> *tmp, cx<double> *xc,
                            const cx<TI> *x, cx<double> *y, hipStream_t s) {
  if (N == 0) return;
  if (n_core > 0)
    hipLaunchKernelGGL(precond_t_gather_kernel<TI>, dim3((unsigned)((n_core + 255) / 256)), dim3(256), 0, s, n_core,
                       core_slot, x, xc);
  if (n_items > 0)
    hipLaunchKernelGGL(precond_t_dots_kernel, dim3(n_items), dim3(PT_THREADS), 0, s, items, ext_ptr, core_ptr, r_off,
                       pc, (const cx<double> *)xc, tmp);
  hipLaunchKernelGGL(precond_t_sum_kernel, dim3(1024), dim3(256), 0, s, N, inv_ptr, inv_pos, (const cx<double> *)tmp,
                     y);
}
#define SCABS_APPLY_T(TI)                                                                                         \
  template void launch_precond_apply_t<TI>(int, const int *, int64_t, int64_t, const int64_t *, const int64_t *,    \
                                           const int *,                                                             \
                                           const int64_t *, PcStore, const int64_t *, const int64_t *, cx<double> *,  \
                                           cx<double> *, const cx<TI> *, cx<double> *, hipStream_t);
SCABS_APPLY_T(double)
SCABS_APPLY_T(float)
#undef SCABS_APPLY_T

// ---------------------------------------------------------------------------
// pointwise one-sided fields of the grid part (FP64) at every test point:
//   E_e^+ = -Z_e jk_e (a_J + k_e^-2 grad phi_J) - curl a_M + 1/2 n x M
//   E_i^- = the same with the interior potentials (J_i, -M) + 1/2 n x M
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
point_fields_kernel(DevOperator<double> op, DevGrid<double> ext, const DevGrid<double> *__restrict__ ints,
                    double inv_h, cx<double> *__restrict__ Ee, cx<double> *__restrict__ Ei) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= op.np) return;
  const PointRec<double> P = op.pts[p];
  const TriRec<double> tr = op.tris[P.tri];
  const double *n = tr.nrm;
  cx<double> Mq[3] = {{0, 0}, {0, 0}, {0, 0}};
  for (int j = 0; j < 3; j++) {
    const cx<double> M = op.src[3 * tr.edge[j] + 2];
    for (int a = 0; a < 3; a++) axpy(Mq[a], P.f[3 * j + a], M);
  }
  cx<double> hnM[3];
  hnM[0] = 0.5 * (n[1] * Mq[2] - n[2] * Mq[1]);
  hnM[1] = 0.5 * (n[2] * Mq[0] - n[0] * Mq[2]);
  hnM[2] = 0.5 * (n[0] * Mq[1] - n[1] * Mq[0]);
  double L[3][3], dL[3][3];
  for (int a = 0; a < 3; a++) lagr3(P.u[a], L[a], dL[a]);
  int ax, ay, az;
  unpack_anchor(P.anc, ax, ay, az);
  for (int med = 0; med < 2; med++) {
    const DevGrid<double> &g = med == 0 ? ext : ints[tr.body];
    const int bx = ax - g.off[0], by = ay - g.off[1], bz = az - g.off[2];
    const int n1 = g.n[1], n2 = g.n[2];
    const size_t G = (size_t)g.n[0] * n1 * n2;
    // values of a_J (0..2) and grad of phi_J (3) and of a_M (4..6)
    cx<double> aJ[3] = {{0, 0}, {0, 0}, {0, 0}}, gphi[3] = {{0, 0}, {0, 0}, {0, 0}};
    cx<double> gM[3][3] = {{{0, 0}, {0, 0}, {0, 0}}, {{0, 0}, {0, 0}, {0, 0}}, {{0, 0}, {0, 0}, {0, 0}}};
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++)
        for (int k = 0; k < 3; k++) {
          const size_t node = ((size_t)(bx + i - 1) * n1 + (by + j - 1)) * n2 + (bz + k - 1);
          const double w = L[0][i] * L[1][j] * L[2][k];
          const double gw[3] = {dL[0][i] * L[1][j] * L[2][k] * inv_h, L[0][i] * dL[1][j] * L[2][k] * inv_h,
                                L[0][i] * L[1][j] * dL[2][k] * inv_h};
          for (int a = 0; a < 3; a++) axpy(aJ[a], w, g.phys[a * G + node]);
          const cx<double> ph = g.phys[3 * G + node];
          for (int a = 0; a < 3; a++) axpy(gphi[a], gw[a], ph);
          for (int c = 0; c < 3; c++) {
            const cx<double> v = g.phys[(4 + c) * G + node];
            for (int a = 0; a < 3; a++) axpy(gM[c][a], gw[a], v);
          }
        }
    const cx<double> cM[3] = {gM[2][1] - gM[1][2], gM[0][2] - gM[2][0], gM[1][0] - gM[0][1]};
    const double k = g.k, Z = g.Z;
    cx<double> *dst = (med == 0 ? Ee : Ei) + 3 * (size_t)p;
    for (int a = 0; a < 3; a++) {
      cx<double> t = aJ[a];
      axpy(t, 1.0 / (k * k), gphi[a]);
      dst[a] = mul_j(t) * (-Z * k) - cM[a] + hnM[a];
    }
  }
}

void launch_point_fields(const DevOperator<double> &op, const DevGrid<double> &ext, const DevGrid<double> *ints_dev,
                         double inv_h, cx<double> *Ee, cx<double> *Ei, hipStream_t s) {
  hipLaunchKernelGGL(point_fields_kernel, dim3((op.np + 255) / 256), dim3(256), 0, s, op, ext, ints_dev, inv_h, Ee, Ei);
}

// ---------------------------------------------------------------------------
// d f / d sigma_q = 2 Re{ w_q [ t_14 . (E_inc + E_i^-) - (t_H x n) . E_e^+ ] }
// with t_H = sum lam_H f, t_14 = sum lam_14 f over the absorber edges of the
// point's triangle (lam unpacked into op.src as row weights): the sigma-
// weighted tests of eq13 (rotated by n x) and eq14 and the eq14 right-hand
// side are the only places sigma enters (Appendix A).
// ---------------------------------------------------------------------------
__global__ void sigma_grad_kernel(DevOperator<double> op, const cx<double> *__restrict__ Ee,
                                  const cx<double> *__restrict__ Ei, const cx<double> *__restrict__ Einc,
                                  double *__restrict__ dfds) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= op.np) return;
  const PointRec<double> P = op.pts[p];
  const TriRec<double> tr = op.tris[P.tri];
  const double *n = tr.nrm;
  cx<double> tH[3] = {{0, 0}, {0, 0}, {0, 0}}, t14[3] = {{0, 0}, {0, 0}, {0, 0}};
  for (int j = 0; j < 3; j++) {
    const int e = tr.edge[j];
    if (!op.edges[e].isR) continue;
    const cx<double> lH = op.src[3 * e + 1], l14 = op.src[3 * e + 2];
    for (int a = 0; a < 3; a++) {
      axpy(tH[a], P.f[3 * j + a], lH);
      axpy(t14[a], P.f[3 * j + a], l14);
    }
  }
  const cx<double> hxn[3] = {tH[1] * n[2] - tH[2] * n[1], tH[2] * n[0] - tH[0] * n[2], tH[0] * n[1] - tH[1] * n[0]};
  cx<double> v = {0.0, 0.0};
  for (int a = 0; a < 3; a++) {
    cx<double> et = Ei[3 * (size_t)p + a];
    if (Einc) et += Einc[3 * (size_t)p + a];
    v += t14[a] * et - hxn[a] * Ee[3 * (size_t)p + a];
  }
  dfds[p] = 2.0 * P.w * v.x;
}

void launch_sigma_grad(const DevOperator<double> &op, const cx<double> *Ee, const cx<double> *Ei,
                       const cx<double> *Einc, double *dfds, hipStream_t s) {
  hipLaunchKernelGGL(sigma_grad_kernel, dim3((op.np + 255) / 256), dim3(256), 0, s, op, Ee, Ei, Einc, dfds);
}

// ---------------------------------------------------------------------------
// fields at off-surface points (plain 7-point rule over every source point;
// targets must stay well away from the surface).  region < 0: exterior
// medium, currents (J_e, M); region = b: interior medium of body b, currents
// (J_i, -M) of its triangles.  E = -Z L(J) + K(M), H = -K(J) - L(M)/Z with
// L(X) = jk [int X G + k^-2 int grad G div X], K(X) = -int grad G x X.
// One work-group per target point.
// ---------------------------------------------------------------------------
constexpr int EF_THREADS = 256;
__device__ inline void green_grad(double k, const double *r, const double *s, cx<double> &G, cx<double> *g) {
  const double d[3] = {r[0] - s[0], r[1] - s[1], r[2] - s[2]};
  const double R = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  double sn, cs;
  sincos(k * R, &sn, &cs);
  const cx<double> e = {cs, -sn};
  G = e * (1.0 / (4.0 * PI * R));
  const cx<double> dG = (cx<double>{1.0, k * R} * e) * (-1.0 / (4.0 * PI * R * R));
  for (int a = 0; a < 3; a++) g[a] = dG * (d[a] / R);
}

__global__ void __launch_bounds__(EF_THREADS)
eval_field_kernel(DevOperator<double> op, const double *__restrict__ qp, const double *__restrict__ pts, int region,
                  double k, double Z, cx<double> *__restrict__ E, cx<double> *__restrict__ H) {
  const int t = blockIdx.x;
  const double r[3] = {pts[3 * t], pts[3 * t + 1], pts[3 * t + 2]};
  cx<double> e[3] = {{0, 0}, {0, 0}, {0, 0}}, h[3] = {{0, 0}, {0, 0}, {0, 0}};
  for (int p = threadIdx.x; p < op.np; p += blockDim.x) {
    const PointRec<double> P = op.pts[p];
    const TriRec<double> tr = op.tris[P.tri];
    if (region >= 0 && tr.body != region) continue;
    cx<double> Jq[3] = {{0, 0}, {0, 0}, {0, 0}}, Mq[3] = {{0, 0}, {0, 0}, {0, 0}}, rJ = {0, 0}, rM = {0, 0};
    for (int j = 0; j < 3; j++) {
      const int m = tr.edge[j];
      const cx<double> J = op.src[3 * m + (region < 0 ? 0 : 1)];
      const cx<double> M = region < 0 ? op.src[3 * m + 2] : -op.src[3 * m + 2];
      for (int a = 0; a < 3; a++) {
        axpy(Jq[a], P.f[3 * j + a], J);
        axpy(Mq[a], P.f[3 * j + a], M);
      }
      axpy(rJ, tr.div[j], J);
      axpy(rM, tr.div[j], M);
    }
    cx<double> G, g[3];
    green_grad(k, r, qp + 3 * (size_t)p, G, g);
    const cx<double> gJ[3] = {g[1] * Jq[2] - g[2] * Jq[1], g[2] * Jq[0] - g[0] * Jq[2], g[0] * Jq[1] - g[1] * Jq[0]};
    const cx<double> gM[3] = {g[1] * Mq[2] - g[2] * Mq[1], g[2] * Mq[0] - g[0] * Mq[2], g[0] * Mq[1] - g[1] * Mq[0]};
    for (int a = 0; a < 3; a++) {
      const cx<double> LJ = mul_j(Jq[a] * G + g[a] * rJ * (1.0 / (k * k))) * k;
      const cx<double> LM = mul_j(Mq[a] * G + g[a] * rM * (1.0 / (k * k))) * k;
      e[a] += (LJ * (-Z) - gM[a]) * P.w;
      h[a] += (gJ[a] - LM * (1.0 / Z)) * P.w;
    }
  }
  __shared__ cx<double> red[EF_THREADS / 64][6];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int a = 0; a < 3; a++) {
    e[a].x = wsum(e[a].x);
    e[a].y = wsum(e[a].y);
    h[a].x = wsum(h[a].x);
    h[a].y = wsum(h[a].y);
  }
  if (lane == 0)
    for (int a = 0; a < 3; a++) {
      red[wv][a] = e[a];
      red[wv][3 + a] = h[a];
    }
  __syncthreads();
  if (threadIdx.x < 6) {
    cx<double> s = {0, 0};
    for (int w = 0; w < EF_THREADS / 64; w++) s += red[w][threadIdx.x];
    if (threadIdx.x < 3)
      E[3 * t + threadIdx.x] = s;
    else
      H[3 * t + threadIdx.x - 3] = s;
  }
}

void launch_eval_field(const DevOperator<double> &op, const double *qp, const double *pts, int npts, int region,
                       double k, double Z, cx<double> *E, cx<double> *H, hipStream_t s) {
  hipLaunchKernelGGL(eval_field_kernel, dim3(npts), dim3(EF_THREADS), 0, s, op, qp, pts, region, k, Z, E, H);
}

// The same fields, accurate close to the surface: per source triangle the
// inner integrals of its three half-RWG functions (inner_j), with the static
// part 1/(4 pi R) integrated analytically and the 7-point rule on the smooth
// remainder when the point lies within SCABS_NEAR_FIELD_RADIUS triangle radii
// of the centroid, the plain rule otherwise.  Threads over triangles, one
// work-group per point.
__global__ void __launch_bounds__(EF_THREADS)
eval_field_exact_kernel(DevOperator<double> op, const TriD *__restrict__ tri, const double *__restrict__ pts,
                        int region, double k, double Z, cx<double> *__restrict__ E, cx<double> *__restrict__ H) {
  const int t = blockIdx.x;
  const D3 r = {pts[3 * t], pts[3 * t + 1], pts[3 * t + 2]};
  const double ik2 = 1.0 / (k * k);
  cx<double> e[3] = {{0, 0}, {0, 0}, {0, 0}}, h[3] = {{0, 0}, {0, 0}, {0, 0}};
  for (int T = threadIdx.x; T < op.nt; T += blockDim.x) {
    const TriRec<double> tr = op.tris[T];
    if (region >= 0 && tr.body != region) continue;
    const TriD *B = tri + T;
    const D3 dc = r - D3{B->cen[0], B->cen[1], B->cen[2]};
    const double thr = SCABS_NEAR_FIELD_RADIUS * B->rho;
    const bool near = dotd(dc, dc) < thr * thr;
    StaticJ st = {0, {0, 0, 0}, {0, 0, 0}};
    if (near) st = static_of(r, B, 0.0);
    for (int j = 0; j < 3; j++) {
      const int m = tr.edge[j];
      const cx<double> J = op.src[3 * m + (region < 0 ? 0 : 1)];
      const cx<double> M = region < 0 ? op.src[3 * m + 2] : -op.src[3 * m + 2];
      InnerJ in;
      inner_j(r, B, 0.0, j, near, st, k, in);
      // L(f) = jk (a + k^-2 gphi), K(f) = -c; E = -Z L(J) + K(M), H = -K(J) - L(M) / Z
      const cx<double> Lf[3] = {mul_j(in.a.x + in.gphi.x * ik2) * k, mul_j(in.a.y + in.gphi.y * ik2) * k,
                                mul_j(in.a.z + in.gphi.z * ik2) * k};
      const cx<double> cf[3] = {in.c.x, in.c.y, in.c.z};
      for (int a = 0; a < 3; a++) {
        e[a] += Lf[a] * J * (-Z) - cf[a] * M;
        h[a] += cf[a] * J - Lf[a] * M * (1.0 / Z);
      }
    }
  }
  __shared__ cx<double> red[EF_THREADS / 64][6];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int a = 0; a < 3; a++) {
    e[a].x = wsum(e[a].x);
    e[a].y = wsum(e[a].y);
    h[a].x = wsum(h[a].x);
    h[a].y = wsum(h[a].y);
  }
  if (lane == 0)
    for (int a = 0; a < 3; a++) {
      red[wv][a] = e[a];
      red[wv][3 + a] = h[a];
    }
  __syncthreads();
  if (threadIdx.x < 6) {
    cx<double> s = {0, 0};
    for (int w = 0; w < EF_THREADS / 64; w++) s += red[w][threadIdx.x];
    if (threadIdx.x < 3)
      E[3 * t + threadIdx.x] = s;
    else
      H[3 * t + threadIdx.x - 3] = s;
  }
}

void launch_eval_field_exact(const DevOperator<double> &op, const TriD *tri, const double *pts, int npts, int region,
                             double k, double Z, cx<double> *E, cx<double> *H, hipStream_t s) {
  hipLaunchKernelGGL(eval_field_exact_kernel, dim3(npts), dim3(EF_THREADS), 0, s, op, tri, pts, region, k, Z, E, H);
}

// ---------------------------------------------------------------------------
// One-sided fields of the discrete Galerkin operator itself (Appendix A) at
// the quadrature points of listed triangles, by direct summation over every
// source triangle with the inner integrals the dense tests use: singular pairs
// (centroid distance below kappa (rho_T + rho_B)) take the static part of G
// analytically and the seven-point rule on the smooth remainder, all others
// the seven-point rule on G.  Adds the residue 1/2 n x M of the point's own
// triangle (exterior limit of the exterior field, interior limit of the
// interior field with M_i = -M).
// ---------------------------------------------------------------------------
// E at r of J = sum_j J_j f_j, M = sum_j M_j f_j on source triangle B in
// medium (k, Z), f_j = coef_j (r' - v_j):
//   E = -Z jk (sum_j a_j J_j + k^-2 sum_j gphi_j J_j) - sum_j c_j M_j
// with the weighted currents Jw = sum coef_j J_j, Jv = sum coef_j J_j v_j:
//   sum a_j J_j    = Jw S1 + S0 (Jw r - Jv)       S0 = int G, S1 = int G (r' - r)
//   sum gphi_j J_j = 2 Jw Sg                      Sg = int grad G
//   sum c_j M_j    = Mw Cg - Sg x Mv              Cg = int grad G x r'
// so each source point's kernel value is computed once for all three halves.
__device__ inline Z3 zcross3(Z3 a, Z3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ inline void tri_field(D3 r, const TriD *B, const cx<double> J[3], const cx<double> M[3], bool sing,
                                 const StaticJ &st, double k, double Z, cx<double> E[3]) {
  cx<double> Jw = {0, 0}, Mw = {0, 0};
  Z3 Jv = {{0, 0}, {0, 0}, {0, 0}}, Mv = Jv;
  for (int j = 0; j < 3; j++) {
    const double cf = B->coef[j];
    const D3 vj = tri_vertex(B, j, 0.0);
    const cx<double> cj = J[j] * cf, cm = M[j] * cf;
    Jw += cj;
    Mw += cm;
    Jv = zadd(Jv, zscale(cj, vj));
    Mv = zadd(Mv, zscale(cm, vj));
  }
  cx<double> S0 = {0, 0};
  Z3 S1 = {{0, 0}, {0, 0}, {0, 0}}, Sg = S1, Cg = S1;
  for (int s = 0; s < NQ; s++) {
    const D3 sp = tri_point(B, s, 0.0);
    const double w = B->qw[s];
    const D3 dv = r - sp;
    const double R = sqrt(dotd(dv, dv));
    cx<double> G = {0, 0}, dG = {0, 0};
    if (R > 0 || sing) kernel_val(k, R, sing, G, dG);
    Z3 grw = {{0, 0}, {0, 0}, {0, 0}};
    if (R > 1e-14) grw = zscale(dG * (w / R), dv);
    S0 += G * w;
    S1 = zadd(S1, zscale(G * w, sp - r));
    Sg = zadd(Sg, grw);
    Cg = zadd(Cg, zcross(grw, sp));
  }
  // sum_j c_j M_j from the rule; the static part adds c4 Jg x (Mw r - Mv)
  Z3 C = zadd({Cg.x * Mw, Cg.y * Mw, Cg.z * Mw}, zcross3(Mv, Sg));
  if (sing) {
    const double c4 = 1.0 / (4.0 * PI);
    S0.x += c4 * st.J0;
    S1.x.x += c4 * st.J1.x;
    S1.y.x += c4 * st.J1.y;
    S1.z.x += c4 * st.J1.z;
    Sg.x.x += c4 * st.Jg.x;
    Sg.y.x += c4 * st.Jg.y;
    Sg.z.x += c4 * st.Jg.z;
    const Z3 mr = {Mw * r.x - Mv.x, Mw * r.y - Mv.y, Mw * r.z - Mv.z};
    const Z3 cs = zcross3({{st.Jg.x, 0}, {st.Jg.y, 0}, {st.Jg.z, 0}}, mr);
    C = zadd(C, {cs.x * c4, cs.y * c4, cs.z * c4});
  }
  const Z3 Jr = {Jw * r.x - Jv.x, Jw * r.y - Jv.y, Jw * r.z - Jv.z};
  const cx<double> ga[3] = {S1.x * Jw + S0 * Jr.x, S1.y * Jw + S0 * Jr.y, S1.z * Jw + S0 * Jr.z};
  const cx<double> gs[3] = {Sg.x * Jw, Sg.y * Jw, Sg.z * Jw};
  const cx<double> cc[3] = {C.x, C.y, C.z};
  const double ik2 = 2.0 / (k * k);
  for (int a = 0; a < 3; a++) {
    cx<double> t = ga[a];
    axpy(t, ik2, gs[a]);
    E[a] = mul_j(t) * (-Z * k) - cc[a];
  }
}

__global__ void __launch_bounds__(EF_THREADS)
point_fields_exact_kernel(DevOperator<double> op, const TriD *__restrict__ tri, const int *__restrict__ list,
                          double k_e, double Z_e, double k_i, double Z_i, double kappa, cx<double> *__restrict__ Ee,
                          cx<double> *__restrict__ Ei) {
  const int T = list[blockIdx.x / NQ], q = blockIdx.x % NQ;
  const TriD *A = tri + T;
  const D3 r = tri_point(A, q, 0.0);
  const int body = op.tris[T].body;
  cx<double> e[3] = {{0, 0}, {0, 0}, {0, 0}}, ii[3] = {{0, 0}, {0, 0}, {0, 0}};
  for (int S = threadIdx.x; S < op.nt; S += blockDim.x) {
    const TriRec<double> tr = op.tris[S];
    const TriD *B = tri + S;
    const bool sing = singular_pair(A, 0.0, B, 0.0, kappa);
    StaticJ st = {0, {0, 0, 0}, {0, 0, 0}};
    if (sing) st = static_of(r, B, 0.0);
    cx<double> Je[3], Ji[3], M[3], Mi[3], f[3];
    for (int j = 0; j < 3; j++) {
      const cx<double> *src = op.src + 3 * (size_t)tr.edge[j];
      Je[j] = src[0];
      Ji[j] = src[1];
      M[j] = src[2];
      Mi[j] = -src[2];
    }
    tri_field(r, B, Je, M, sing, st, k_e, Z_e, f);
    for (int a = 0; a < 3; a++) e[a] += f[a];
    if (tr.body == body) {
      tri_field(r, B, Ji, Mi, sing, st, k_i, Z_i, f);
      for (int a = 0; a < 3; a++) ii[a] += f[a];
    }
  }
  __shared__ cx<double> red[EF_THREADS / 64][6];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int a = 0; a < 3; a++) {
    e[a].x = wsum(e[a].x);
    e[a].y = wsum(e[a].y);
    ii[a].x = wsum(ii[a].x);
    ii[a].y = wsum(ii[a].y);
  }
  if (lane == 0)
    for (int a = 0; a < 3; a++) {
      red[wv][a] = e[a];
      red[wv][3 + a] = ii[a];
    }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int p = T * NQ + q;
    const PointRec<double> P = op.pts[p];
    const TriRec<double> tr = op.tris[T];
    cx<double> Mq[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (int j = 0; j < 3; j++) {
      const cx<double> Mj = op.src[3 * (size_t)tr.edge[j] + 2];
      for (int a = 0; a < 3; a++) axpy(Mq[a], P.f[3 * j + a], Mj);
    }
    const double *n = tr.nrm;
    const cx<double> hnM[3] = {(n[1] * Mq[2] - n[2] * Mq[1]) * 0.5, (n[2] * Mq[0] - n[0] * Mq[2]) * 0.5,
                               (n[0] * Mq[1] - n[1] * Mq[0]) * 0.5};
    const int a = threadIdx.x % 3;
    cx<double> sum = {0, 0};
    for (int w = 0; w < EF_THREADS / 64; w++) sum += red[w][threadIdx.x];
    (threadIdx.x < 3 ? Ee : Ei)[3 * (size_t)p + a] = sum + hnM[a];
  }
}

void launch_point_fields_exact(const DevOperator<double> &op, const TriD *tri, const int *list, int nlist,
                               double k_e, double Z_e, double k_i, double Z_i, double kappa, cx<double> *Ee,
                               cx<double> *Ei, hipStream_t s) {
  if (nlist <= 0) return;
  hipLaunchKernelGGL(point_fields_exact_kernel, dim3(nlist * NQ), dim3(EF_THREADS), 0, s, op, tri, list, k_e, Z_e,
                     k_i, Z_i, kappa, Ee, Ei);
}

// Block-Toeplitz contexts, points of periodic absorber triangles: the
// product's own point lines hold the tangential principal-value fields of
// every periodic edge's currents there (pf, template tangents t1, t2); the
// half functions of the non-periodic edges (listed per triangle with a mask of
// their local halves) are summed directly with the same inner integrals, and
// the residue 1/2 n x M is added.  The point lines carry the two in-plane
// components only (all the sigma tests read); the normal component of what
// Ee / Ei hold is kept.  One wave per point.
__global__ void __launch_bounds__(64)
toe_point_fields_kernel(DevOperator<double> op, ToeDev<double> d, const TriD *__restrict__ tri,
                        const int *__restrict__ list, const int *__restrict__ np_tri, const int *__restrict__ np_mask,
                        int nnp, double k_e, double Z_e, double k_i, double Z_i, double kappa,
                        cx<double> *__restrict__ Ee, cx<double> *__restrict__ Ei) {
  const int T = list[blockIdx.x / NQ], q = blockIdx.x % NQ;
  const TriD *A = tri + T;
  const D3 r = tri_point(A, q, 0.0);
  const int body = op.tris[T].body;
  cx<double> e[3] = {{0, 0}, {0, 0}, {0, 0}}, ii[3] = {{0, 0}, {0, 0}, {0, 0}};
  for (int i = threadIdx.x; i < nnp; i += 64) {
    const int S = np_tri[i], mask = np_mask[i];
    const TriRec<double> tr = op.tris[S];
    const TriD *B = tri + S;
    const bool sing = singular_pair(A, 0.0, B, 0.0, kappa);
    StaticJ st = {0, {0, 0, 0}, {0, 0, 0}};
    if (sing) st = static_of(r, B, 0.0);
    cx<double> Je[3], Ji[3], M[3], Mi[3], f[3];
    for (int j = 0; j < 3; j++) {
      const cx<double> *src = op.src + 3 * (size_t)tr.edge[j];
      const bool on = (mask >> j) & 1;
      Je[j] = on ? src[0] : cx<double>{0, 0};
      Ji[j] = on ? src[1] : cx<double>{0, 0};
      M[j] = on ? src[2] : cx<double>{0, 0};
      Mi[j] = -M[j];
    }
    tri_field(r, B, Je, M, sing, st, k_e, Z_e, f);
    for (int a = 0; a < 3; a++) e[a] += f[a];
    if (tr.body == body) {
      tri_field(r, B, Ji, Mi, sing, st, k_i, Z_i, f);
      for (int a = 0; a < 3; a++) ii[a] += f[a];
    }
  }
  for (int a = 0; a < 3; a++) {
    e[a].x = wsum(e[a].x);
    e[a].y = wsum(e[a].y);
    ii[a].x = wsum(ii[a].x);
    ii[a].y = wsum(ii[a].y);
  }
  if (threadIdx.x != 0) return;
  const int p = T * NQ + q;
  const PointRec<double> P = op.pts[p];
  const TriRec<double> tr = op.tris[T];
  cx<double> Mq[3] = {{0, 0}, {0, 0}, {0, 0}};
  for (int j = 0; j < 3; j++) {
    const cx<double> Mj = op.src[3 * (size_t)tr.edge[j] + 2];
    for (int a = 0; a < 3; a++) axpy(Mq[a], P.f[3 * j + a], Mj);
  }
  const double *n = tr.nrm;
  const cx<double> hnM[3] = {(n[1] * Mq[2] - n[2] * Mq[1]) * 0.5, (n[2] * Mq[0] - n[0] * Mq[2]) * 0.5,
                             (n[0] * Mq[1] - n[1] * Mq[0]) * 0.5};
  const int lt = d.tri_loc[T], j = d.tri_ring[T], nr = d.nr;
  const size_t R2 = 2 * (size_t)NQ * d.nt_r, row = 2 * ((size_t)lt * NQ + q);
  const cx<double> *pe = d.pf + row * nr + j, *pi = pe + R2 * nr;
  const double *t1 = d.t1 + 3 * (size_t)lt, *t2 = d.t2 + 3 * (size_t)lt;
  for (int side = 0; side < 2; side++) {
    const cx<double> *pv = side == 0 ? pe : pi;
    const cx<double> *dir = side == 0 ? e : ii;
    cx<double> *dst = (side == 0 ? Ee : Ei) + 3 * (size_t)p;
    cx<double> dn = dir[0] * n[0], ln = dst[0] * n[0];
    axpy(dn, n[1], dir[1]);
    axpy(dn, n[2], dir[2]);
    axpy(ln, n[1], dst[1]);
    axpy(ln, n[2], dst[2]);
    cx<double> out[3];
    for (int a = 0; a < 3; a++) {
      cx<double> v = pv[0] * t1[a] + pv[nr] * t2[a] + hnM[a] + dir[a];
      axpy(v, -n[a], dn);    // tangential part of the direct sum
      axpy(v, n[a], ln);     // normal component kept
      out[a] = v;
    }
    for (int a = 0; a < 3; a++) dst[a] = out[a];
  }
}

void launch_toe_point_fields(const DevOperator<double> &op, const ToeDev<double> &d, const TriD *tri, const int *list,
                             int nlist, const int *np_tri, const int *np_mask, int nnp, double k_e, double Z_e,
                             double k_i, double Z_i, double kappa, cx<double> *Ee, cx<double> *Ei, hipStream_t s) {
  if (nlist <= 0) return;
  hipLaunchKernelGGL(toe_point_fields_kernel, dim3(nlist * NQ), dim3(64), 0, s, op, d, tri, list, np_tri, np_mask, nnp,
                     k_e, Z_e, k_i, Z_i, kappa, Ee, Ei);
}

// Transpose of the E part: for weights wE (npts x 3) the per-point
// coefficients of the half-RWG currents,
//   J_j: w_p sum_t wE_t . (-Z jk (f_j G + k^-2 grad G div f_j))
//   M_j: -w_p sum_t f_j . (wE_t x grad G)
// summed over each triangle's points into tri_out (J_e or J_i, M slots).
constexpr int ET_TRIS = 32;
__global__ void __launch_bounds__(ET_TRIS * NQ)
eval_field_t_kernel(DevOperator<double> op, const double *__restrict__ qp, const double *__restrict__ pts, int npts,
                    int region, double k, double Z, const cx<double> *__restrict__ wE) {
  __shared__ cx<double> part[ET_TRIS * NQ][9];
  const int lt = threadIdx.x / NQ, q = threadIdx.x - lt * NQ;
  const int tri = blockIdx.x * ET_TRIS + lt;
  cx<double> out[9];
  for (int r = 0; r < 9; r++) out[r] = {0, 0};
  if (tri < op.nt && (region < 0 || op.tris[tri].body == region)) {
    const int p = tri * NQ + q;
    const PointRec<double> P = op.pts[p];
    const TriRec<double> tr = op.tris[tri];
    cx<double> sG[3] = {{0, 0}, {0, 0}, {0, 0}}, sg = {0, 0}, cr[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (int t = 0; t < npts; t++) {
      cx<double> G, g[3];
      green_grad(k, pts + 3 * t, qp + 3 * (size_t)p, G, g);
      const cx<double> *w = wE + 3 * t;
      for (int a = 0; a < 3; a++) sG[a] += w[a] * G;          // sum_t wE G
      sg += w[0] * g[0] + w[1] * g[1] + w[2] * g[2];          // sum_t wE . grad G
      cr[0] += w[1] * g[2] - w[2] * g[1];                     // sum_t wE x grad G
      cr[1] += w[2] * g[0] - w[0] * g[2];
      cr[2] += w[0] * g[1] - w[1] * g[0];
    }
    for (int j = 0; j < 3; j++) {
      const double *f = P.f + 3 * j;
      cx<double> fv = f[0] * sG[0];
      axpy(fv, f[1], sG[1]);
      axpy(fv, f[2], sG[2]);
      axpy(fv, tr.div[j] / (k * k), sg);
      const cx<double> aj = mul_j(fv) * (-Z * k * P.w);
      cx<double> am = f[0] * cr[0];
      axpy(am, f[1], cr[1]);
      axpy(am, f[2], cr[2]);
      am = am * (-P.w);
      if (region < 0) {
        out[3 * j] = aj;
        out[3 * j + 2] = am;
      } else {
        out[3 * j + 1] = aj;
        out[3 * j + 2] = -am;
      }
    }
  }
  for (int r = 0; r < 9; r++) part[threadIdx.x][r] = out[r];
  __syncthreads();
  for (int it = threadIdx.x; it < ET_TRIS * 9; it += blockDim.x) {
    const int l = it / 9, r = it - l * 9;
    const int t2 = blockIdx.x * ET_TRIS + l;
    if (t2 < op.nt) {
      cx<double> s = {0, 0};
      for (int qq = 0; qq < NQ; qq++) s += part[l * NQ + qq][r];
      op.tri_out[(size_t)t2 * 9 + r] = s;
    }
  }
}

// per edge: sum of its two triangle halves of (J_e, J_i, M) adjoints mapped to
// its unknowns (sigma-free edges: J_e = J, J_i = -J)
__global__ void edge_collect_kernel(DevOperator<double> op, double *__restrict__ y) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= op.ne) return;
  const EdgeRec r = op.edges[m];
  const cx<double> *p0 = op.tri_out + ((size_t)r.tri[0] * 3 + r.loc[0]) * 3;
  const cx<double> *p1 = op.tri_out + ((size_t)r.tri[1] * 3 + r.loc[1]) * 3;
  const cx<double> aJe = p0[0] + p1[0], aJi = p0[1] + p1[1], aM = p0[2] + p1[2];
  if (!r.isR) {
    const cx<double> j = aJe - aJi;
    y[2 * r.col[0]] = j.x;
    y[2 * r.col[0] + 1] = j.y;
    y[2 * r.col[1]] = aM.x;
    y[2 * r.col[1] + 1] = aM.y;
  } else {
    y[2 * r.col[0]] = aJe.x;
    y[2 * r.col[0] + 1] = aJe.y;
    y[2 * r.col[1]] = aJi.x;
    y[2 * r.col[1] + 1] = aJi.y;
    y[2 * r.col[2]] = aM.x;
    y[2 * r.col[2] + 1] = aM.y;
  }
}

void launch_eval_field_t(const DevOperator<double> &op, const double *qp, const double *pts, int npts, int region,
                         double k, double Z, const cx<double> *wE, double *y, hipStream_t s) {
  hipLaunchKernelGGL(eval_field_t_kernel, dim3((op.nt + ET_TRIS - 1) / ET_TRIS), dim3(ET_TRIS * NQ), 0, s, op, qp, pts,
                     npts, region, k, Z, wE);
  hipLaunchKernelGGL(edge_collect_kernel, dim3((op.ne + 255) / 256), dim3(256), 0, s, op, y);
}

}  // namespace scabs
