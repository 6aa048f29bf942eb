// Transposed block-Toeplitz product y = A^T z (the adjoint solves of the
// gradient), exact like the forward product.  Every stage of the forward
// product is transposed:
//  * the circulant block products: with the forward tables T(f) (row a,
//    column b), the transposed circulant takes T_ab(-f) contracted over the
//    row index a, so the row weights are transformed forward along the rings,
//    multiplied per frequency by the tables at P - f, and transformed back
//    onto the column slots (J_e, M, J_i, M_i = -M) of the periodic edges;
//  * the sigma tests of the periodic test halves against the periodic point
//    fields: per point the tangential weights that the tests give to the
//    exterior and interior fields (the point rows of the circulant);
//  * the local terms (residues, Gram block, the 1/2 n x M part of the sigma
//    tests) per triangle;
//  * the stored entries of the non-periodic pairs: the short part (periodic
//    rows, non-periodic columns) summed per non-periodic column, the long
//    part (non-periodic rows, every column) summed per column.
// Up to 8 vectors per call: each vector's rows, point weights, local terms
// and column outputs in a slice of its own; the transform lines and spectra
// carry the vector index fastest (line = row nb + v), so the block products
// and the stored entries are read once for all of them.
#include <algorithm>
#include <cmath>

#include "device_common.h"
#include "kernels.h"

namespace scabs {

constexpr int TT_THREADS = 512;
constexpr int TT_ELEMS = 16;
static_assert(TT_THREADS * TT_ELEMS >= 8192, "a work-group must hold one line of the longest circulant the build accepts");

// LDS of a group of G transform lines: padded lines, then P twiddles
template <typename T> inline size_t tt_tw_offset(int P, int G) {
  return ((size_t)lpad_size<T>(G * P) * sizeof(cx<T>) + 15) / 16 * 16;
}
template <typename T> inline size_t tt_lds(int P, int G) { return tt_tw_offset<T>(P, G) + (size_t)P * sizeof(cx<T>); }
template <typename T>
__device__ inline const cx<T> *tt_twiddles(unsigned char *smem, const cx<T> *tw, int P, int G) {
  cx<T> *t = reinterpret_cast<cx<T> *>(smem + ((size_t)lpad_size<T>(G * P) * sizeof(cx<T>) + 15) / 16 * 16);
  for (int i = threadIdx.x; i < P; i += blockDim.x) t[i] = tw[i];
  return t;
}
// lines per transform work-group of the transposed product: at most 8,
// within the Stockham stages' elements per thread (a hard limit of the
// transform) and with the padded lines within 64 KiB of LDS
template <typename T> inline int tt_lines(int P) {
  int g = TT_ELEMS * TT_THREADS / P;
  if (g > 8) g = 8;
  while (g > 1 && (size_t)lpad_size<T>(g * P) * sizeof(cx<T>) > 65536) g--;
  return g < 1 ? 1 : g;
}
int toe_t_max_lines(int P, bool fp32) { return fp32 ? tt_lines<float>(P) : tt_lines<double>(P); }
template <typename K> size_t tt_launch_lds(K kernel, size_t lds) {
  if (lds > 65536)
    (void)hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  return lds;
}

// ---------------------------------------------------------------------------
// local terms and sigma tests, transposed, per triangle.  rows[e] = (z_E,
// z_H, z_14) of edge e (op.src after the row unpack).  Per test half i the
// forward H and eq14 rows read, at every point q (w the weight, ws = w sigma,
// Jsum = sum_j f_j (J_e + J_i)_j, Mq = sum_j f_j M_j):
//   h_i   += -1/2 w g_i.(n x Jsum) + ws (g_i x n).(1/2 n x Mq + E_e^PV)
//   r14_i += w g_i.Jsum - ws g_i.(1/2 n x Mq + E_i^PV)
// (PV fields only for periodic test halves of periodic triangles).  The
// transpose collects per point Jsum' = sum_i [-1/2 w z_H (g_i x n) + w z_14
// g_i], Mq' = sum_i [1/2 ws z_H ((g_i x n) x n) - 1/2 ws z_14 (g_i x n)], and
// the field weights E_e' = sum_i ws z_H (g_i x n), E_i' = -sum_i ws z_14 g_i,
// projected on the point's tangents into the point-row weights pw (ring-major
// like the forward point fields).  Per half j of the triangle the columns
// receive (J_e', J_i', M') = (f_j.Jsum', f_j.Jsum', f_j.Mq').
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) toe_t_local_kernel(DevOperator<T> op, ToeDev<T> d) {
  const int T_ = blockIdx.x * blockDim.x + threadIdx.x, v = blockIdx.y;
  if (T_ >= op.nt) return;
  const cx<T> *rows = op.src + (size_t)3 * op.ne * v;
  const TriRec<T> tr = op.tris[T_];
  const bool per = d.tri_loc[T_] >= 0;
  const T n[3] = {tr.nrm[0], tr.nrm[1], tr.nrm[2]};
  cx<T> zH[3], zQ[3];
  bool eper[3];
  for (int i = 0; i < 3; i++) {
    const int e = tr.edge[i];
    zH[i] = rows[3 * e + 1];
    zQ[i] = rows[3 * e + 2];
    eper[i] = d.edge_sgn[e] != 0;
  }
  cx<T> out[9];
  for (int k = 0; k < 9; k++) out[k] = czero<T>();
  for (int q = 0; q < NQ; q++) {
    const PointRec<T> P = op.pts[(size_t)T_ * NQ + q];
    const T w = P.w, ws = P.w * P.sigma;
    cx<T> Js[3], Ms[3], Ee[3], Ei[3];
    for (int a = 0; a < 3; a++) Js[a] = Ms[a] = Ee[a] = Ei[a] = czero<T>();
    for (int i = 0; i < 3; i++) {
      const T g[3] = {P.f[3 * i], P.f[3 * i + 1], P.f[3 * i + 2]};
      const T gxn[3] = {g[1] * n[2] - g[2] * n[1], g[2] * n[0] - g[0] * n[2], g[0] * n[1] - g[1] * n[0]};
      const T gxnxn[3] = {gxn[1] * n[2] - gxn[2] * n[1], gxn[2] * n[0] - gxn[0] * n[2],
                          gxn[0] * n[1] - gxn[1] * n[0]};
      for (int a = 0; a < 3; a++) {
        axpy(Js[a], T(-0.5) * w * gxn[a], zH[i]);
        axpy(Js[a], w * g[a], zQ[i]);
      }
      if (ws != T(0)) {
        for (int a = 0; a < 3; a++) {
          axpy(Ms[a], T(0.5) * ws * gxnxn[a], zH[i]);
          axpy(Ms[a], T(-0.5) * ws * gxn[a], zQ[i]);
        }
        if (per && eper[i])
          for (int a = 0; a < 3; a++) {
            axpy(Ee[a], ws * gxn[a], zH[i]);
            axpy(Ei[a], -ws * g[a], zQ[i]);
          }
      }
    }
    for (int j = 0; j < 3; j++) {
      cx<T> fj = czero<T>(), fm = czero<T>();
      for (int a = 0; a < 3; a++) {
        axpy(fj, P.f[3 * j + a], Js[a]);
        axpy(fm, P.f[3 * j + a], Ms[a]);
      }
      out[3 * j] += fj;
      out[3 * j + 1] += fj;
      out[3 * j + 2] += fm;
    }
    if (per) {
      const int lt = d.tri_loc[T_], jr = d.tri_ring[T_], nr = d.nr;
      const size_t R2 = 2 * (size_t)NQ * d.nt_r, r = 2 * ((size_t)lt * NQ + q);
      const T *t1 = d.t1 + 3 * (size_t)lt, *t2 = d.t2 + 3 * (size_t)lt;
      cx<T> e1 = czero<T>(), e2 = czero<T>(), i1 = czero<T>(), i2 = czero<T>();
      for (int a = 0; a < 3; a++) {
        axpy(e1, t1[a], Ee[a]);
        axpy(e2, t2[a], Ee[a]);
        axpy(i1, t1[a], Ei[a]);
        axpy(i2, t2[a], Ei[a]);
      }
      cx<T> *pw = d.pf + (size_t)v * 2 * R2 * nr + r * nr + jr;
      pw[0] = e1;
      pw[nr] = e2;
      pw[R2 * nr] = i1;
      pw[(R2 + 1) * nr] = i2;
    }
  }
  cx<T> *to = op.tri_out + (size_t)9 * op.nt * v + (size_t)T_ * 9;
  for (int k = 0; k < 9; k++) to[k] = out[k];
}

// ---------------------------------------------------------------------------
// row lines (forward transform), line l = s nb + v: row s < 2 ne_r: rows
// E (s even) and H of template edge s / 2 at the periodic edges of the rings
// (template orientation); row 2 ne_r + rr: point-row weights pw[rr][j]; zero
// beyond the rings; spectra to Y[f][line]
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(TT_THREADS) toe_t_fwd_kernel(DevOperator<T> op, ToeDev<T> d, int nb) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T> *buf = reinterpret_cast<cx<T> *>(smem_raw);
  const int P = d.P, nr = d.nr, G = d.lines, ne_r = d.ne_r;
  const int R2 = 2 * NQ * d.nt_r, nlines = (2 * ne_r + 2 * R2) * nb;
  const int l0 = blockIdx.x * G, nl = min(G, nlines - l0);
  const cx<T> *tws = tt_twiddles<T>(smem_raw, d.tw, P, G);
  for (int i = threadIdx.x; i < nl * P; i += blockDim.x) {
    const int li = i / P, j = i - li * P, l = l0 + li;
    const int row = l / nb, v = l - row * nb;
    cx<T> val = czero<T>();
    if (j < nr) {
      if (row < 2 * ne_r) {
        const int e = d.ringmap[(size_t)(row >> 1) * nr + j];
        if (e >= 0) val = op.src[(size_t)3 * op.ne * v + 3 * e + (row & 1)] * (T)d.edge_sgn[e];
      } else {
        val = d.pf[((size_t)v * 2 * R2 + row - 2 * ne_r) * nr + j];
      }
    }
    buf[lpad<T>(i)] = val;
  }
  __syncthreads();
  lds_fft_mr<T, TT_ELEMS>(buf, P, nl, 1, P, 0, 1, tws, P, false);
  for (int i = threadIdx.x; i < nl * P; i += blockDim.x) {
    const int f = i / nl, li = i - f * nl;
    d.Y[(size_t)f * nlines + l0 + li] = buf[lpad<T>(li * P + f)];
  }
}

// ---------------------------------------------------------------------------
// per frequency f, one wave per template edge b (column): the four column
// slots from the row spectra with the tables at P - f, rows contracted
//   J_e' = sum_a (-Z_e L E - K H) + sum_r PJ_e W_e     (exterior)
//   M'   = sum_a (K E - L H / Z_e) + sum_r PM_e W_e
//   J_i' = sum_a (Z_i L E + K H)   + sum_r PJ_i W_i     (interior, b's body)
//   M_i' = sum_a (-K E + L H / Z_i) + sum_r PM_i W_i
// written to X[f][slot ne_r + b] (slots J_e, M, J_i, M_i)
// ---------------------------------------------------------------------------
constexpr int TT_NB = 8;   // vectors per call
// NBM: the most vectors the instance handles (1 keeps the single-vector
// kernel's registers low)
template <typename T, int NBM>
__global__ void __launch_bounds__(256) toe_t_apply_kernel(ToeDev<T> d, int nb) {
  int part, f;
  toe_xcd_order(part, f);
  const int b = part * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (b >= d.ne_r) return;   // wave-uniform
  const int ne_r = d.ne_r, R2 = 2 * NQ * d.nt_r, nout = 2 * ne_r + 2 * R2, P = d.P;
  const int fr = f == 0 ? 0 : P - f;
  const cx<T> *Yf = d.Y + (size_t)f * nout * nb;   // [row][v]
  const int bd = d.ebody[b], e0 = d.body_e0[bd], neb = d.body_e0[bd + 1] - e0;
  const int r0 = 2 * NQ * d.body_t0[bd], R2b = 2 * NQ * (d.body_t0[bd + 1] - d.body_t0[bd]);
  const T Ze = d.Z_e, Zi = d.Z_i, iZe = T(1) / Ze, iZi = T(1) / Zi;
  cx<T> je[NBM], me[NBM], ji[NBM], mi[NBM];
#pragma unroll
  for (int v = 0; v < NBM; v++) je[v] = me[v] = ji[v] = mi[v] = czero<T>();
  const cx<T> *G = d.GE + ((size_t)fr * ne_r * ne_r + (size_t)b * ne_r) * 2;
  for (int a = lane; a < ne_r; a += 64) {
    const cx<T> L = G[2 * a], K = G[2 * a + 1];
    const cx<T> *Ea = Yf + (size_t)(2 * a) * nb, *Ha = Ea + nb;
#pragma unroll
    for (int v = 0; v < NBM; v++)
      if (v < nb) {
        const cx<T> E = Ea[v], H = Ha[v];
        je[v] += (L * E) * (-Ze) - K * H;
        me[v] += K * E - (L * H) * iZe;
      }
  }
  const cx<T> *GI = d.GI + ((size_t)fr * d.gi_per_f + d.ibase[bd] + (size_t)(b - e0) * neb) * 2;
  for (int a = lane; a < neb; a += 64) {
    const cx<T> L = GI[2 * a], K = GI[2 * a + 1];
    const cx<T> *Ea = Yf + (size_t)(2 * (e0 + a)) * nb, *Ha = Ea + nb;
#pragma unroll
    for (int v = 0; v < NBM; v++)
      if (v < nb) {
        const cx<T> E = Ea[v], H = Ha[v];
        ji[v] += (L * E) * Zi + K * H;
        mi[v] += (L * H) * iZi - K * E;
      }
  }
  const cx<T> *PE = d.PE + ((size_t)fr * ne_r * R2 + (size_t)b * R2) * 2;
  for (int r = lane; r < R2; r += 64) {
    const cx<T> pj = PE[2 * r], pm = PE[2 * r + 1];
    const cx<T> *W = Yf + (size_t)(2 * ne_r + r) * nb;
#pragma unroll
    for (int v = 0; v < NBM; v++)
      if (v < nb) {
        je[v] += pj * W[v];
        me[v] += pm * W[v];
      }
  }
  const cx<T> *PI = d.PI + ((size_t)fr * d.pi_per_f + d.pbase[bd] + (size_t)(b - e0) * R2b) * 2;
  for (int r = lane; r < R2b; r += 64) {
    const cx<T> pj = PI[2 * r], pm = PI[2 * r + 1];
    const cx<T> *W = Yf + (size_t)(2 * ne_r + R2 + r0 + r) * nb;
#pragma unroll
    for (int v = 0; v < NBM; v++)
      if (v < nb) {
        ji[v] += pj * W[v];
        mi[v] += pm * W[v];
      }
  }
  cx<T> *Xf = d.X + (size_t)f * 4 * ne_r * nb;   // [slot ne_r + b][v]
#pragma unroll
  for (int v = 0; v < NBM; v++) {
    if (v >= nb) break;
    T sv[8] = {je[v].x, je[v].y, me[v].x, me[v].y, ji[v].x, ji[v].y, mi[v].x, mi[v].y};
#pragma unroll
    for (int k = 0; k < 8; k++)
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) sv[k] += __shfl_xor(sv[k], o, 64);
    if (lane == 0) {
      Xf[(size_t)b * nb + v] = {sv[0], sv[1]};
      Xf[(size_t)(ne_r + b) * nb + v] = {sv[2], sv[3]};
      Xf[(size_t)(2 * ne_r + b) * nb + v] = {sv[4], sv[5]};
      Xf[(size_t)(3 * ne_r + b) * nb + v] = {sv[6], sv[7]};
    }
  }
}

// column lines (inverse transform): slot c of template edge b over the
// rings; tcol[e][c] at the periodic edges (template orientation back to the
// edge's; slot 3 carries -M, so its value enters M with the opposite sign)
template <typename T>
__global__ void __launch_bounds__(TT_THREADS) toe_t_inv_kernel(ToeDev<T> d, cx<T> *__restrict__ tcol, int ne, int nb) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T> *buf = reinterpret_cast<cx<T> *>(smem_raw);
  const int P = d.P, nr = d.nr, G = d.lines, ne_r = d.ne_r;
  const int nlines = 4 * ne_r * nb;
  const int l0 = blockIdx.x * G, nl = min(G, nlines - l0);
  const cx<T> *tws = tt_twiddles<T>(smem_raw, d.tw, P, G);
  for (int i = threadIdx.x; i < nl * P; i += blockDim.x) {
    const int f = i / nl, li = i - f * nl;
    buf[lpad<T>(li * P + f)] = d.X[(size_t)f * nlines + l0 + li];
  }
  __syncthreads();
  lds_fft_mr<T, TT_ELEMS>(buf, P, nl, 1, P, 0, 1, tws, P, true);
  for (int i = threadIdx.x; i < nl * nr; i += blockDim.x) {
    const int li = i / nr, j = i - li * nr, l = l0 + li;
    const int cb = l / nb, v = l - cb * nb;
    const int c = cb / ne_r, b = cb - c * ne_r;
    const int e = d.ringmap[(size_t)b * nr + j];
    if (e < 0) continue;
    const T sg = (T)d.edge_sgn[e] * (c == 3 ? T(-1) : T(1));
    tcol[((size_t)v * ne + e) * 4 + c] = buf[lpad<T>(li * P + j)] * sg;
  }
}

// transposed entry of a stored pair: the column currents' weights from the
// row weights (z_E, z_H, z_14) of the pair's row edge
template <typename T> struct ColAcc {
  cx<T> je, ji, m;
};
template <typename T>
__device__ inline void col_mac(const RowCoef<T> &c, cx<T> zE, cx<T> zH, cx<T> zQ, ColAcc<T> &o) {
  cmac(o.je, c.eJe, zE);
  cmac(o.je, c.hJe, zH);
  cmac(o.ji, c.eJi, zE);
  cmac(o.ji, c.hJi, zH);
  cmac(o.ji, c.rJi, zQ);
  cmac(o.m, c.eM, zE);
  cmac(o.m, c.hM, zH);
  cmac(o.m, c.rM, zQ);
}

// short part transposed: work-group (non-periodic column j, row chunk s),
// threads over the chunk's periodic rows n; the chunk's partial (J_e', J_i',
// M') goes to scol[j][s], summed in a fixed order by the combine kernel
template <typename T>
__global__ void __launch_bounds__(256) toe_t_short_kernel(DevOperator<T> op, ToeRows<T> R, cx<T> *__restrict__ scol) {
  const int j = blockIdx.x, sp = blockIdx.y;
  const int chunk = (op.ne + TOE_T_SHORT_SPLIT - 1) / TOE_T_SHORT_SPLIT;
  const int n0 = sp * chunk, n1 = min(op.ne, n0 + chunk);
  const T Ze = op.Z_e, Zi = op.Z_i;
  ColAcc<T> o = {czero<T>(), czero<T>(), czero<T>()};
  for (int n = n0 + threadIdx.x; n < n1; n += blockDim.x) {
    const int fl = R.eflag[n];
    if (!(fl & 1)) continue;   // non-periodic rows are in the long part
    const size_t k = ((size_t)j * op.ne + n) * 4;
    const RowCoef<T> c = row_coef(R.V4S + k, R.S4S + k, (fl & 2) != 0, Ze, Zi);
    col_mac(c, op.src[3 * n], op.src[3 * n + 1], op.src[3 * n + 2], o);
  }
  __shared__ T red[6][4];
  T v[6] = {o.je.x, o.je.y, o.ji.x, o.ji.y, o.m.x, o.m.y};
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 6; k++) {
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) v[k] += __shfl_xor(v[k], s, 64);
    if (lane == 0) red[k][w] = v[k];
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    T t = 0;
    for (int q = 0; q < (int)(blockDim.x >> 6); q++) t += red[threadIdx.x][q];
    reinterpret_cast<T *>(scol + ((size_t)j * TOE_T_SHORT_SPLIT + sp) * 3)[threadIdx.x] = t;
  }
}

// short part transposed for several vectors: work-group (non-periodic
// column j, row chunk s), threads over the chunk's periodic rows, each record
// read once for all vectors; scol[v][j][s] as the single-vector kernel
template <typename T>
__global__ void __launch_bounds__(256) toe_t_short_nb_kernel(DevOperator<T> op, ToeRows<T> R, cx<T> *__restrict__ scol,
                                                             int nb) {
  const int j = blockIdx.x, sp = blockIdx.y;
  const int chunk = (op.ne + TOE_T_SHORT_SPLIT - 1) / TOE_T_SHORT_SPLIT;
  const int n0 = sp * chunk, n1 = min(op.ne, n0 + chunk);
  const T Ze = op.Z_e, Zi = op.Z_i;
  ColAcc<T> o[TT_NB];
#pragma unroll
  for (int v = 0; v < TT_NB; v++) o[v] = {czero<T>(), czero<T>(), czero<T>()};
  for (int n = n0 + threadIdx.x; n < n1; n += blockDim.x) {
    const int fl = R.eflag[n];
    if (!(fl & 1)) continue;   // non-periodic rows are in the long part
    const size_t k = ((size_t)j * op.ne + n) * 4;
    const RowCoef<T> c = row_coef(R.V4S + k, R.S4S + k, (fl & 2) != 0, Ze, Zi);
#pragma unroll
    for (int v = 0; v < TT_NB; v++)
      if (v < nb) {
        const cx<T> *z = op.src + (size_t)3 * op.ne * v + 3 * n;
        col_mac(c, z[0], z[1], z[2], o[v]);
      }
  }
  __shared__ T red[6 * TT_NB][4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int v = 0; v < TT_NB; v++) {
    if (v >= nb) break;
    T sv[6] = {o[v].je.x, o[v].je.y, o[v].ji.x, o[v].ji.y, o[v].m.x, o[v].m.y};
#pragma unroll
    for (int k = 0; k < 6; k++) {
#pragma unroll
      for (int s = 32; s > 0; s >>= 1) sv[k] += __shfl_xor(sv[k], s, 64);
      if (lane == 0) red[6 * v + k][w] = sv[k];
    }
  }
  __syncthreads();
  if (threadIdx.x < 6 * nb) {
    const int v = threadIdx.x / 6, k = threadIdx.x - 6 * v;
    T t = 0;
    for (int q = 0; q < (int)(blockDim.x >> 6); q++) t += red[threadIdx.x][q];
    reinterpret_cast<T *>(scol + (((size_t)v * R.ncap + j) * TOE_T_SHORT_SPLIT + sp) * 3)[k] = t;
  }
}

// long part transposed: one wave per column m, lanes over the non-periodic
// rows (a column's records are contiguous), each record read once for all
// vectors, then wave sums; lcol[v][m]
template <typename T, int NBM>
__global__ void __launch_bounds__(256) toe_t_long_kernel(DevOperator<T> op, ToeRows<T> R, cx<T> *__restrict__ lcol,
                                                         int nb) {
  const int m = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (m >= op.ne) return;   // wave-uniform
  const T Ze = op.Z_e, Zi = op.Z_i;
  ColAcc<T> o[NBM];
#pragma unroll
  for (int v = 0; v < NBM; v++) o[v] = {czero<T>(), czero<T>(), czero<T>()};
  for (int i = lane; i < R.nlong; i += 64) {
    const int n = R.capcol[i];
    const size_t k = ((size_t)m * R.nlong + i) * 4;
    const RowCoef<T> c = row_coef(R.V4L + k, R.S4L + k, (R.eflag[n] & 2) != 0, Ze, Zi);
#pragma unroll
    for (int v = 0; v < NBM; v++)
      if (v < nb) {
        const cx<T> *z = op.src + (size_t)3 * op.ne * v + 3 * n;
        col_mac(c, z[0], z[1], z[2], o[v]);
      }
  }
#pragma unroll
  for (int v = 0; v < NBM; v++) {
    if (v >= nb) break;
    T sv[6] = {o[v].je.x, o[v].je.y, o[v].ji.x, o[v].ji.y, o[v].m.x, o[v].m.y};
#pragma unroll
    for (int k = 0; k < 6; k++)
#pragma unroll
      for (int s = 32; s > 0; s >>= 1) sv[k] += __shfl_xor(sv[k], s, 64);
    if (lane < 6) reinterpret_cast<T *>(lcol + ((size_t)v * op.ne + m) * 3)[lane] = sv[lane];
  }
}

// per edge: the circulant columns (periodic edges), the long and short parts
// and the local terms of its two halves, onto the unknowns (J^L = J_e - J_i
// and M^L on sigma-free edges; J_e, J_i, M on absorber edges)
template <typename T>
__global__ void __launch_bounds__(256)
toe_t_combine_kernel(DevOperator<T> op, ToeRows<T> R, const cx<T> *__restrict__ tcol, const cx<T> *__restrict__ lcol,
                     const cx<T> *__restrict__ scol, const int *__restrict__ capidx, double *__restrict__ y) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x, v = blockIdx.y;
  if (e >= op.ne) return;
  tcol += (size_t)4 * op.ne * v;
  lcol += (size_t)3 * op.ne * v;
  scol += (size_t)3 * TOE_T_SHORT_SPLIT * R.ncap * v;
  y += (size_t)2 * op.N * v;
  const EdgeRec r = op.edges[e];
  cx<T> je = lcol[(size_t)e * 3], ji = lcol[(size_t)e * 3 + 1], m = lcol[(size_t)e * 3 + 2];
  if (R.edge_sgn[e] != 0) {
    je += tcol[(size_t)e * 4];
    m += tcol[(size_t)e * 4 + 1] + tcol[(size_t)e * 4 + 3];
    ji += tcol[(size_t)e * 4 + 2];
  }
  const int ci = capidx[e];
  if (ci >= 0)
    for (int sp = 0; sp < TOE_T_SHORT_SPLIT; sp++) {
      const cx<T> *sc = scol + ((size_t)ci * TOE_T_SHORT_SPLIT + sp) * 3;
      je += sc[0];
      ji += sc[1];
      m += sc[2];
    }
  for (int s = 0; s < 2; s++) {
    const cx<T> *h = op.tri_out + (size_t)9 * op.nt * v + ((size_t)r.tri[s] * 3 + r.loc[s]) * 3;
    je += h[0];
    ji += h[1];
    m += h[2];
  }
  auto put = [&](int slot, cx<T> v) {
    y[2 * (size_t)slot] = (double)v.x;
    y[2 * (size_t)slot + 1] = (double)v.y;
  };
  if (!r.isR) {
    put(r.col[0], je - ji);
    put(r.col[1], m);
  } else {
    put(r.col[0], je);
    put(r.col[1], ji);
    put(r.col[2], m);
  }
}

template <typename T>
void launch_toe_product_t(const DevOperator<T> &op, const ToeDev<T> &d, const ToeRows<T> &R, cx<T> *tcol,
                          cx<T> *lcol, cx<T> *scol, const int *capidx, double *y, hipStream_t s, int parts, int nb) {
  const int G = d.lines;
  const int nrow = (2 * d.ne_r + 4 * NQ * d.nt_r) * nb, ncol = 4 * d.ne_r * nb;
  if (parts & TOE_FWD) {
    hipLaunchKernelGGL(toe_t_local_kernel<T>, dim3((op.nt + 255) / 256, nb), dim3(256), 0, s, op, d);
    hipLaunchKernelGGL(toe_t_fwd_kernel<T>, dim3((nrow + G - 1) / G), dim3(TT_THREADS),
                       tt_launch_lds(toe_t_fwd_kernel<T>, tt_lds<T>(d.P, G)), s, op, d, nb);
  }
  if (parts & TOE_APPLY) {
    if (nb == 1)
      hipLaunchKernelGGL((toe_t_apply_kernel<T, 1>), dim3((d.ne_r + 3) / 4, d.P), dim3(256), 0, s, d, nb);
    else
      hipLaunchKernelGGL((toe_t_apply_kernel<T, TT_NB>), dim3((d.ne_r + 3) / 4, d.P), dim3(256), 0, s, d, nb);
  }
  if (parts & TOE_INV)
    hipLaunchKernelGGL(toe_t_inv_kernel<T>, dim3((ncol + G - 1) / G), dim3(TT_THREADS),
                       tt_launch_lds(toe_t_inv_kernel<T>, tt_lds<T>(d.P, G)), s, d, tcol, op.ne, nb);
  if ((parts & TOE_SHORT) && R.ncap > 0) {
    if (nb == 1)
      hipLaunchKernelGGL(toe_t_short_kernel<T>, dim3(R.ncap, TOE_T_SHORT_SPLIT), dim3(256), 0, s, op, R, scol);
    else
      hipLaunchKernelGGL(toe_t_short_nb_kernel<T>, dim3(R.ncap, TOE_T_SHORT_SPLIT), dim3(256), 0, s, op, R, scol,
                         nb);
  }
  if (parts & TOE_LONG) {
    if (nb == 1)
      hipLaunchKernelGGL((toe_t_long_kernel<T, 1>), dim3((op.ne + 3) / 4), dim3(256), 0, s, op, R, lcol, nb);
    else
      hipLaunchKernelGGL((toe_t_long_kernel<T, TT_NB>), dim3((op.ne + 3) / 4), dim3(256), 0, s, op, R, lcol, nb);
  }
  if (parts & TOE_SUM)
    hipLaunchKernelGGL(toe_t_combine_kernel<T>, dim3((op.ne + 255) / 256, nb), dim3(256), 0, s, op, R,
                       (const cx<T> *)tcol, (const cx<T> *)lcol, (const cx<T> *)scol, capidx, y);
}
template void launch_toe_product_t<float>(const DevOperator<float> &, const ToeDev<float> &, const ToeRows<float> &,
                                          cx<float> *, cx<float> *, cx<float> *, const int *, double *, hipStream_t,
                                          int, int);
template void launch_toe_product_t<double>(const DevOperator<double> &, const ToeDev<double> &,
                                           const ToeRows<double> &, cx<double> *, cx<double> *, cx<double> *,
                                           const int *, double *, hipStream_t, int, int);

}  // namespace scabs
