// Block-Toeplitz product of the sigma-modified PMCHW system (fast-solver
// appendix): on a mesh that repeats along x with pitch dx, the tested
// Galerkin operators between periodic RWG edges depend only on the ring
// offset of the two edges, so their block Toeplitz matrices are embedded in
// circulants of length P >= 2 nr - 1 and applied by FFTs along the ring axis
// with one dense block product per frequency.  The sigma-weighted rows of
// eq13 and eq14 take the one-sided fields at the quadrature (target) points,
// which are Toeplitz in the same way (potential operators at target points),
// before the points' Gauss weights and conductivities are applied.  Entries
// that involve a non-periodic edge (end caps and the edges touching them)
// are computed exactly and applied as sparse rows.  Everything here is exact
// for the discrete Galerkin system: the same quadrature and singularity
// treatment as the near-pair setup, no lattice approximation.
#include <algorithm>
#include <cmath>

#include "device_common.h"
#include "kernels.h"
#include "near_math.h"

namespace scabs {

// ---------------------------------------------------------------------------
// exact inner integrals and tested values (FP64)
// ---------------------------------------------------------------------------
// Tested interactions of half function i of target triangle A (shift sa)
// with half function j of source triangle B (shift sb):
//   out[0..3] = L_e, K_e, L_i, K_i  (Galerkin; L tested by parts)
//   out[4..7] = Lrot_e, Krot_e, Lsig_i, Ksig_i at A's points with conductivity
//               sig[q] (sig null: not computed)
// interior values only when inner != 0.  Added into out.
__device__ void tested_pair(const TriD *A, double sa, int i, const TriD *B, double sb, int j, double ke, double ki,
                            double kappa, bool inner, const double *sig, cx<double> *out) {
  const bool sing = singular_pair(A, sa, B, sb, kappa);
  const D3 vi = tri_vertex(A, i, sa);
  const D3 n = {A->nrm[0], A->nrm[1], A->nrm[2]};
  const double ci = A->coef[i], di = 2.0 * ci;
  for (int q = 0; q < NQ; q++) {
    const D3 r = tri_point(A, q, sa);
    const double w = A->qw[q];
    const D3 g = ci * (r - vi);
    StaticJ st = {0, {0, 0, 0}, {0, 0, 0}};
    if (sing) st = static_of(r, B, sb);
    const double sg = sig ? sig[q] : 0.0;
    for (int med = 0; med < (inner ? 2 : 1); med++) {
      const double k = med ? ki : ke, ik2 = 1.0 / (k * k);
      InnerJ in;
      inner_j(r, B, sb, j, sing, st, k, in);
      cx<double> tl = zdot(g, in.a);
      axpy(tl, -di * ik2, in.phi);
      out[med ? 2 : 0] += mul_j(tl) * (k * w);
      const Z3 Kv = {-in.c.x, -in.c.y, -in.c.z};
      out[med ? 3 : 1] += zdot(g, Kv) * w;
      if (sg != 0.0) {
        Z3 Lv;
        Lv.x = mul_j(in.a.x + in.gphi.x * ik2) * k;
        Lv.y = mul_j(in.a.y + in.gphi.y * ik2) * k;
        Lv.z = mul_j(in.a.z + in.gphi.z * ik2) * k;
        if (med == 0) {
          const D3 gxn = crossd(g, n);
          out[4] += zdot(gxn, Lv) * (w * sg);
          out[5] += zdot(gxn, Kv) * (w * sg);
        } else {
          out[6] += zdot(g, Lv) * (w * sg);
          out[7] += zdot(g, Kv) * (w * sg);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// setup: spatial ring blocks (series over the circulant index m in [0, P))
// ---------------------------------------------------------------------------
__device__ inline bool circ_offset(int m, int nr, int P, int &delta) {
  if (m < nr) {
    delta = m;
    return true;
  }
  if (m > P - nr) {
    delta = m - P;
    return true;
  }
  return false;
}

// Galerkin ring blocks: target local edge a at ring delta, source local edge
// b at ring 0.  Series (a, b) over m; ext: sLe/sKe[(a ne_r + b) P + m]; int
// (same body only): sLi/sKi[(ibase_bd + (a - e0) ne_b + (b - e0)) P + m].
__global__ void __launch_bounds__(64) toe_galerkin_kernel(ToeSetupArgs s) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)s.ne_r * s.ne_r * s.P;
  if (gid >= total) return;
  const int m = (int)(gid % s.P);
  const int64_t ab = gid / s.P;
  const int a = (int)(ab / s.ne_r), b = (int)(ab % s.ne_r);
  const int ba = s.ebody[a], bb = s.ebody[b];
  const bool same = ba == bb;
  cx<double> out[8];
  for (int t = 0; t < 8; t++) out[t] = {0, 0};
  int delta;
  if (circ_offset(m, s.nr, s.P, delta)) {
    for (int sa_ = 0; sa_ < 2; sa_++) {
      const TriD *A = s.tri + s.e_tri[2 * a + sa_];
      const double xa = (delta + s.e_off[2 * a + sa_]) * s.dx;
      for (int sb_ = 0; sb_ < 2; sb_++) {
        const TriD *B = s.tri + s.e_tri[2 * b + sb_];
        const double xb = s.e_off[2 * b + sb_] * s.dx;
        tested_pair(A, xa, s.e_k[2 * a + sa_], B, xb, s.e_k[2 * b + sb_], s.k_e, s.k_i, s.kappa, same, nullptr, out);
      }
    }
  }
  s.sLe[ab * s.P + m] = out[0];
  s.sKe[ab * s.P + m] = out[1];
  if (same) {
    const int e0 = s.body_e0[ba], neb = s.body_e0[ba + 1] - e0;
    const int64_t ser = s.ibase[ba] + (int64_t)(a - e0) * neb + (b - e0);
    s.sLi[ser * s.P + m] = out[2];
    s.sKi[ser * s.P + m] = out[3];
  }
}

// One-sided principal-value fields at the target points: local point p
// (triangle p / 7 at ring delta, point p % 7), tangential components along
// t1, t2 of its triangle, of unit J and unit M on source local edge b at ring
// 0: E(J) = -Z L(f), E(M) = K(f).  Row r = 2 p + c.  ext: sPeJ/sPeM[(r ne_r + b) P + m];
// int (same body): sPiJ/sPiM[(pbase_bd + (r - r0) ne_b + (b - e0)) P + m].
__global__ void __launch_bounds__(64) toe_points_kernel(ToeSetupArgs s) {
  const int np_r = NQ * s.nt_r;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)np_r * s.ne_r * s.P;
  if (gid >= total) return;
  const int m = (int)(gid % s.P);
  const int64_t pb = gid / s.P;
  const int p = (int)(pb / s.ne_r), b = (int)(pb % s.ne_r);
  const int lt = p / NQ, q = p - lt * NQ;
  const TriD *A = s.tri + lt;
  const int bd = A->body, bb = s.ebody[b];
  const bool same = bd == bb;
  cx<double> e[8];
  for (int t = 0; t < 8; t++) e[t] = {0, 0};
  int delta;
  if (circ_offset(m, s.nr, s.P, delta)) {
    const double xa = delta * s.dx;
    const D3 r = tri_point(A, q, xa);
    const D3 t1 = {A->t1[0], A->t1[1], A->t1[2]}, t2 = {A->t2[0], A->t2[1], A->t2[2]};
    for (int sb_ = 0; sb_ < 2; sb_++) {
      const TriD *B = s.tri + s.e_tri[2 * b + sb_];
      const double xb = s.e_off[2 * b + sb_] * s.dx;
      const int j = s.e_k[2 * b + sb_];
      // the point's own triangle: the rule's coincident points are handled as
      // in the Galerkin blocks (remainder gradient 0 at R = 0)
      const bool sing = singular_pair(A, xa, B, xb, s.kappa);
      StaticJ st = {0, {0, 0, 0}, {0, 0, 0}};
      if (sing) st = static_of(r, B, xb);
      for (int med = 0; med < (same ? 2 : 1); med++) {
        const double k = med ? s.k_i : s.k_e, Z = med ? s.Z_i : s.Z_e, ik2 = 1.0 / (k * k);
        InnerJ in;
        inner_j(r, B, xb, j, sing, st, k, in);
        Z3 Lv;
        Lv.x = mul_j(in.a.x + in.gphi.x * ik2) * k;
        Lv.y = mul_j(in.a.y + in.gphi.y * ik2) * k;
        Lv.z = mul_j(in.a.z + in.gphi.z * ik2) * k;
        const Z3 EJ = {Lv.x * (-Z), Lv.y * (-Z), Lv.z * (-Z)};
        const Z3 EM = {-in.c.x, -in.c.y, -in.c.z};
        cx<double> *o = e + 4 * med;
        o[0] += zdot(t1, EJ);
        o[1] += zdot(t2, EJ);
        o[2] += zdot(t1, EM);
        o[3] += zdot(t2, EM);
      }
    }
  }
  for (int c = 0; c < 2; c++) {
    const int64_t row = 2 * (int64_t)p + c;
    s.sPeJ[(row * s.ne_r + b) * s.P + m] = e[c];
    s.sPeM[(row * s.ne_r + b) * s.P + m] = e[2 + c];
    if (same) {
      const int e0 = s.body_e0[bd], neb = s.body_e0[bd + 1] - e0;
      const int64_t r0 = 2 * (int64_t)NQ * s.body_t0[bd];
      const int64_t ser = s.pbase[bd] + (row - r0) * neb + (b - e0);
      s.sPiJ[ser * s.P + m] = e[4 + c];
      s.sPiM[ser * s.P + m] = e[6 + c];
    }
  }
}

// Sparse rows of every edge pair with a non-periodic edge: exact tested values
// (8 types, summed over the 2 x 2 triangle pairs of the two edges) per CSR
// entry, in FP64 and FP32.
__global__ void __launch_bounds__(64) toe_cap_entries_kernel(ToeCapArgs c) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= c.nnz) return;
  const int n = c.row[k], m = c.col[k];
  cx<double> out[8];
  for (int t = 0; t < 8; t++) out[t] = {0, 0};
  for (int sa_ = 0; sa_ < 2; sa_++) {
    const int T = c.et[2 * n + sa_];
    int i = 0;
    for (int kk = 0; kk < 3; kk++)
      if (c.tedge[3 * T + kk] == n) i = kk;
    const double *sig = c.sigma + (size_t)T * NQ;
    bool any = false;
    for (int q = 0; q < NQ; q++) any |= sig[q] != 0.0;
    for (int sb_ = 0; sb_ < 2; sb_++) {
      const int U = c.et[2 * m + sb_];
      int j = 0;
      for (int kk = 0; kk < 3; kk++)
        if (c.tedge[3 * U + kk] == m) j = kk;
      tested_pair(c.tri + T, 0.0, i, c.tri + U, 0.0, j, c.k_e, c.k_i, c.kappa, c.tri[T].body == c.tri[U].body,
                  any ? sig : nullptr, out);
    }
  }
  for (int t = 0; t < 4; t++) {
    c.V4[4 * k + t] = out[t];
    c.S4[4 * k + t] = out[4 + t];
    c.V4f[4 * k + t] = {(float)out[t].x, (float)out[t].y};
    c.S4f[4 * k + t] = {(float)out[4 + t].x, (float)out[4 + t].y};
  }
}

void launch_toe_setup(const ToeSetupArgs &s, hipStream_t st) {
  const int64_t ng = (int64_t)s.ne_r * s.ne_r * s.P;
  hipLaunchKernelGGL(toe_galerkin_kernel, dim3((unsigned)((ng + 63) / 64)), dim3(64), 0, st, s);
  const int64_t npn = (int64_t)NQ * s.nt_r * s.ne_r * s.P;
  hipLaunchKernelGGL(toe_points_kernel, dim3((unsigned)((npn + 63) / 64)), dim3(64), 0, st, s);
}
void launch_toe_cap_entries(const ToeCapArgs &c, hipStream_t st) {
  if (c.nnz == 0) return;
  hipLaunchKernelGGL(toe_cap_entries_kernel, dim3((unsigned)((c.nnz + 63) / 64)), dim3(64), 0, st, c);
}

// ---------------------------------------------------------------------------
// FFTs along the ring axis: groups of TOE_LINES lines of length P in LDS
// ---------------------------------------------------------------------------
constexpr int TOE_FFT_THREADS = 512;
constexpr int TOE_GATHER = 8;   // global loads issued together per thread
// waves per SIMD asked of the product's transforms: two work-groups per CU
// in FP32 (registers capped at 128), one in FP64
template <typename T> constexpr int toe_fft_waves() { return sizeof(T) == sizeof(float) ? 4 : 2; }
constexpr int TOE_FFT_ELEMS = 16;
// lines per work-group: at most 8, within the Stockham stage's elements per
// thread and within 64 KiB of LDS (padded addressing); the product's
// transforms take d.lines <= this (tuned)
template <typename T> __host__ __device__ inline int toe_lines_per_group(int P) {
  int g = TOE_FFT_ELEMS * TOE_FFT_THREADS / P;
  if (g > 8) g = 8;
  while (g > 1 && (size_t)lpad_size<T>(g * P) * sizeof(cx<T>) > 65536) g--;
  return g < 1 ? 1 : g;
}
int toe_max_lines(int P, bool fp32) { return fp32 ? toe_lines_per_group<float>(P) : toe_lines_per_group<double>(P); }
// LDS of a group of G lines: the padded lines, then the P twiddles
template <typename T> __host__ __device__ inline size_t toe_tw_offset(int P, int G) {
  return ((size_t)lpad_size<T>(G * P) * sizeof(cx<T>) + 15) / 16 * 16;
}
template <typename T> size_t toe_fft_lds(int P, int G) { return toe_tw_offset<T>(P, G) + (size_t)P * sizeof(cx<T>); }
// dynamic LDS of a transform launch (attribute raised past 64 KiB)
template <typename K> size_t toe_fft_launch_lds(K kernel, size_t lds) {
  if (lds > 65536)
    (void)hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  return lds;
}
// twiddles copied to LDS (read by every Stockham stage)
template <typename T>
__device__ inline const cx<T> *toe_stage_twiddles(unsigned char *smem, const cx<T> *tw, int P, int G) {
  cx<T> *t = reinterpret_cast<cx<T> *>(smem + toe_tw_offset<T>(P, G));
  for (int i = threadIdx.x; i < P; i += blockDim.x) t[i] = tw[i];
  return t;
}

// setup: lines stored contiguously (series of length P), transformed in
// place with the factor 1/P of the inverse folded in
__global__ void __launch_bounds__(TOE_FFT_THREADS) toe_series_fft_kernel(cx<double> *data, int64_t nlines, int P,
                                                                         const cx<double> *tw) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<double> *buf = reinterpret_cast<cx<double> *>(smem_raw);
  const int G = toe_lines_per_group<double>(P);
  const int64_t l0 = (int64_t)blockIdx.x * G;
  const int nl = (int)(nlines - l0 < G ? nlines - l0 : G);
  const cx<double> *tws = toe_stage_twiddles<double>(smem_raw, tw, P, G);
  for (int i = threadIdx.x; i < nl * P; i += blockDim.x) buf[lpad<double>(i)] = data[l0 * P + i];
  __syncthreads();
  lds_fft_mr<double, TOE_FFT_ELEMS>(buf, P, nl, 1, P, 0, 1, tws, P, false);
  const double sc = 1.0 / P;
  for (int i = threadIdx.x; i < nl * P; i += blockDim.x) data[l0 * P + i] = buf[lpad<double>(i)] * sc;
}

void launch_toe_series_fft(cx<double> *data, int64_t nlines, int P, const cx<double> *tw, hipStream_t s) {
  if (nlines == 0) return;
  const int G = toe_lines_per_group<double>(P);
  hipLaunchKernelGGL(toe_series_fft_kernel, dim3((unsigned)((nlines + G - 1) / G)), dim3(TOE_FFT_THREADS),
                     toe_fft_launch_lds(toe_series_fft_kernel, toe_fft_lds<double>(P, G)), s, data, nlines, P, tw);
}

// series-major (FFT'd) -> per-frequency layouts of the block products, FP64
// and FP32.  Pair tables: two series (X, Y) become one record {X, Y} at
// dst[f * per_f + d] for destination d, whose source series index is given
// by the map kind.
//   kind 0 (Galerkin ext): d = b ne_r + a          <- series a ne_r + b
//   kind 1 (Galerkin int): d = ibase + (b-e0) neb + (a-e0) <- ibase + (a-e0) neb + (b-e0)
//   kind 2 (points ext):   d = b R2 + r            <- r ne_r + b
//   kind 3 (points int):   d = pbase + (b-e0) R2b + (r-r0) <- pbase + (r-r0) neb + (b-e0)
__device__ inline int64_t toe_src_series(const ToeSetupArgs &s, int kind, int64_t d) {
  if (kind == 0) {
    const int64_t b = d / s.ne_r, a = d % s.ne_r;
    return a * s.ne_r + b;
  }
  if (kind == 2) {
    const int64_t R2 = 2 * (int64_t)NQ * s.nt_r;
    const int64_t b = d / R2, r = d % R2;
    return r * s.ne_r + b;
  }
  // per-body blocks: find the body
  for (int bd = 0; bd < s.nbody; bd++) {
    const int64_t base = kind == 1 ? s.ibase[bd] : s.pbase[bd];
    const int64_t next = kind == 1 ? s.ibase[bd + 1] : s.pbase[bd + 1];
    if (d < base || d >= next) continue;
    const int64_t neb = s.body_e0[bd + 1] - s.body_e0[bd];
    const int64_t rows = kind == 1 ? neb : 2 * (int64_t)NQ * (s.body_t0[bd + 1] - s.body_t0[bd]);
    const int64_t off = d - base, col = off / rows, row = off % rows;
    return base + row * neb + col;
  }
  return 0;
}

__global__ void toe_layout_kernel(ToeSetupArgs s, int kind, const cx<double> *X, const cx<double> *Y, int64_t per_f,
                                  cx<double> *dst64, cx<float> *dst32) {
  const int64_t total = per_f * s.P;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t f = i / per_f, d = i % per_f;
    const int64_t ser = toe_src_series(s, kind, d);
    const cx<double> x = X[ser * s.P + f], y = Y[ser * s.P + f];
    dst64[2 * i] = x;
    dst64[2 * i + 1] = y;
    dst32[2 * i] = {(float)x.x, (float)x.y};
    dst32[2 * i + 1] = {(float)y.x, (float)y.y};
  }
}

void launch_toe_layout(const ToeSetupArgs &s, int kind, const cx<double> *X, const cx<double> *Y, int64_t per_f,
                       cx<double> *dst64, cx<float> *dst32, hipStream_t st) {
  if (per_f == 0) return;
  hipLaunchKernelGGL(toe_layout_kernel, dim3(4096), dim3(256), 0, st, s, kind, X, Y, per_f, dst64, dst32);
}

// ---------------------------------------------------------------------------
// product
// ---------------------------------------------------------------------------
// forward: line l = slot * nb + v (slot = c ne_r + a; c: 0 J_e, 1 M (exterior
// sources), 2 J_i, 3 M_i = -M (interior sources)); values over rings j < nr
// gathered from the per-edge currents (template orientation), zero beyond,
// transformed; spectrum written to X[f][l].
template <typename T>
__global__ void __launch_bounds__(TOE_FFT_THREADS) __attribute__((amdgpu_waves_per_eu(toe_fft_waves<T>())))
toe_fwd_kernel(ToeDev<T> d, const cx<T> *__restrict__ src,
                                                                  const cx<T> *__restrict__ srcI, int ne, int nb) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T> *buf = reinterpret_cast<cx<T> *>(smem_raw);
  const int P = d.P, nr = d.nr;
  const int G = d.lines;
  const int nlines = 4 * d.ne_r * nb;
  const int l0 = blockIdx.x * G;
  const int nl = min(G, nlines - l0);
  // gathers in batches of TOE_GATHER per thread, every load in bounds
  // (indices clamped, results masked) so that a batch's loads overlap
  const cx<T> *tws = toe_stage_twiddles<T>(smem_raw, d.tw, P, G);
  const int n = nl * P;
  for (int i0 = threadIdx.x; i0 < n; i0 += TOE_GATHER * blockDim.x) {
    int rm[TOE_GATHER];
#pragma unroll
    for (int u = 0; u < TOE_GATHER; u++) {
      const int i = min(i0 + u * (int)blockDim.x, n - 1);
      const int li = i / P, j = min(i - li * P, nr - 1);
      const int slot = (l0 + li) / nb, a = slot % d.ne_r;
      rm[u] = d.ringmap[(size_t)a * nr + j];
    }
    cx<T> x[TOE_GATHER];
    int sg[TOE_GATHER];
#pragma unroll
    for (int u = 0; u < TOE_GATHER; u++) {
      const int i = min(i0 + u * (int)blockDim.x, n - 1);
      const int l = l0 + i / P, slot = l / nb, v = l - slot * nb, c = slot / d.ne_r;
      const int cc = c == 0 ? 0 : c == 2 ? 1 : 2;
      const int e = rm[u] >= 0 ? rm[u] : 0;
      x[u] = nb > 1 ? srcI[((size_t)e * nb + v) * 3 + cc] : src[(size_t)e * 3 + cc];
      sg[u] = d.edge_sgn[e];
    }
#pragma unroll
    for (int u = 0; u < TOE_GATHER; u++) {
      const int i = i0 + u * (int)blockDim.x;
      if (i < n) {
        const int li = i / P, j = i - li * P;
        const int c = ((l0 + li) / nb) / d.ne_r;
        const T s = (T)sg[u] * (c == 3 ? T(-1) : T(1));
        buf[lpad<T>(i)] = (j < nr && rm[u] >= 0) ? x[u] * s : czero<T>();
      }
    }
  }
  __syncthreads();
  if (wave_fits(P, nl, blockDim.x >> 6, TOE_FFT_ELEMS))
    lds_fft<T, TOE_FFT_ELEMS, TOE_FFT_ELEMS, true>(buf, P, nl, 1, P, 0, 1, tws, P, false);
  else
    lds_fft_mr<T, TOE_FFT_ELEMS>(buf, P, nl, 1, P, 0, 1, tws, P, false);
  for (int i = threadIdx.x; i < nl * P; i += blockDim.x) {
    const int f = i / nl, li = i - f * nl;
    d.X[(size_t)f * nlines + l0 + li] = buf[lpad<T>(li * P + f)];
  }
}

// per frequency: rows [0, ne_r) Galerkin (E and H rows of the local edge,
// exterior minus interior), rows [ne_r, ne_r + R2) point fields (exterior and
// interior tangential components).  Output slots: 2 a + (0: E, 1: H); 2 ne_r + r
// (exterior point row r); 2 ne_r + R2 + r (interior).  Y[f][slot * nb + v].
template <typename T, int NB>
__global__ void __launch_bounds__(256) toe_apply_kernel(ToeDev<T> d) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T> *xs = reinterpret_cast<cx<T> *>(smem_raw);   // [slot][v]
  int part, f;
  toe_xcd_order(part, f);
  const int ne_r = d.ne_r, R2 = 2 * NQ * d.nt_r;
  const int nin = 4 * ne_r * NB;
  const cx<T> *Xf = d.X + (size_t)f * nin;
  for (int i = threadIdx.x; i < nin; i += blockDim.x) xs[i] = Xf[i];
  __syncthreads();
  const int row = part * blockDim.x + threadIdx.x;
  const int nout = 2 * ne_r + 2 * R2;
  cx<T> *Yf = d.Y + (size_t)f * nout * NB;
  if (row < ne_r) {
    const int a = row;
    const int bd = d.ebody[a], e0 = d.body_e0[bd], neb = d.body_e0[bd + 1] - e0;
    cx<T> out_e[NB], out_h[NB];
    for (int med = 0; med < 2; med++) {
      cx<T> LJ[NB], LM[NB], KJ[NB], KM[NB];
#pragma unroll
      for (int v = 0; v < NB; v++) LJ[v] = LM[v] = KJ[v] = KM[v] = czero<T>();
      const int b0 = med ? e0 : 0, b1 = med ? e0 + neb : ne_r;
      const cx<T> *G = med ? d.GI + ((size_t)f * d.gi_per_f + d.ibase[bd] + (size_t)(a - e0)) * 2
                           : d.GE + ((size_t)f * ne_r * ne_r + a) * 2;
      const size_t cstride = (size_t)(med ? neb : ne_r) * 2;
      const cx<T> *xJ = xs + (size_t)(med ? 2 : 0) * ne_r * NB, *xM = xs + (size_t)(med ? 3 : 1) * ne_r * NB;
      constexpr int DEP = NB == 1 ? 8 : 2;   // column pairs in flight
      int b = b0;
      for (; b + DEP <= b1; b += DEP) {
        cx<T> Lp[DEP], Kp[DEP];
#pragma unroll
        for (int u = 0; u < DEP; u++) {
          const cx<T> *g = G + (size_t)(b + u - b0) * cstride;
          Lp[u] = g[0];
          Kp[u] = g[1];
        }
#pragma unroll
        for (int u = 0; u < DEP; u++)
#pragma unroll
          for (int v = 0; v < NB; v++) {
            const cx<T> J = xJ[(b + u) * NB + v], M = xM[(b + u) * NB + v];
            cmac(LJ[v], Lp[u], J);
            cmac(LM[v], Lp[u], M);
            cmac(KJ[v], Kp[u], J);
            cmac(KM[v], Kp[u], M);
          }
      }
      for (; b < b1; b++) {
        const cx<T> *g = G + (size_t)(b - b0) * cstride;
        const cx<T> L = g[0], K = g[1];
#pragma unroll
        for (int v = 0; v < NB; v++) {
          const cx<T> J = xJ[b * NB + v], M = xM[b * NB + v];
          cmac(LJ[v], L, J);
          cmac(LM[v], L, M);
          cmac(KJ[v], K, J);
          cmac(KM[v], K, M);
        }
      }
      const T Z = med ? d.Z_i : d.Z_e, iZ = T(1) / Z, sgn = med ? T(-1) : T(1);
#pragma unroll
      for (int v = 0; v < NB; v++) {
        const cx<T> E = KM[v] - LJ[v] * Z, H = -KJ[v] - LM[v] * iZ;
        if (med == 0) {
          out_e[v] = E;
          out_h[v] = H;
        } else {
          out_e[v] += E * sgn;
          out_h[v] += H * sgn;
        }
      }
    }
#pragma unroll
    for (int v = 0; v < NB; v++) {
      Yf[(size_t)(2 * a) * NB + v] = out_e[v];
      Yf[(size_t)(2 * a + 1) * NB + v] = out_h[v];
    }
  } else if (row < ne_r + R2) {
    const int r = row - ne_r, lt = r / (2 * NQ);
    const int bd = d.tbody[lt], e0 = d.body_e0[bd], neb = d.body_e0[bd + 1] - e0;
    const int r0 = 2 * NQ * d.body_t0[bd], R2b = 2 * NQ * (d.body_t0[bd + 1] - d.body_t0[bd]);
    for (int med = 0; med < 2; med++) {
      cx<T> acc[NB];
#pragma unroll
      for (int v = 0; v < NB; v++) acc[v] = czero<T>();
      const int b0 = med ? e0 : 0, b1 = med ? e0 + neb : ne_r;
      const cx<T> *G = med ? d.PI + ((size_t)f * d.pi_per_f + d.pbase[bd] + (size_t)(r - r0)) * 2
                           : d.PE + ((size_t)f * ne_r * R2 + r) * 2;
      const size_t cstride = (size_t)(med ? R2b : R2) * 2;
      const cx<T> *xJ = xs + (size_t)(med ? 2 : 0) * ne_r * NB, *xM = xs + (size_t)(med ? 3 : 1) * ne_r * NB;
      constexpr int DEP = NB == 1 ? 8 : 2;
      int b = b0;
      for (; b + DEP <= b1; b += DEP) {
        cx<T> Pj[DEP], Pm[DEP];
#pragma unroll
        for (int u = 0; u < DEP; u++) {
          const cx<T> *g = G + (size_t)(b + u - b0) * cstride;
          Pj[u] = g[0];
          Pm[u] = g[1];
        }
#pragma unroll
        for (int u = 0; u < DEP; u++)
#pragma unroll
          for (int v = 0; v < NB; v++) {
            cmac(acc[v], Pj[u], xJ[(b + u) * NB + v]);
            cmac(acc[v], Pm[u], xM[(b + u) * NB + v]);
          }
      }
      for (; b < b1; b++) {
        const cx<T> *g = G + (size_t)(b - b0) * cstride;
        const cx<T> PJ = g[0], PM = g[1];
#pragma unroll
        for (int v = 0; v < NB; v++) {
          cmac(acc[v], PJ, xJ[b * NB + v]);
          cmac(acc[v], PM, xM[b * NB + v]);
        }
      }
#pragma unroll
      for (int v = 0; v < NB; v++) Yf[(size_t)(2 * ne_r + med * R2 + r) * NB + v] = acc[v];
    }
  }
}

// The same products for 8 vectors on the matrix cores
// (v_mfma_f32_16x16x4_f32, complex arithmetic in real form).  One wave per
// 16-row tile of one frequency, 16 tiles per work-group sharing the input
// spectra in LDS.  A tile row's table record for source column c is four
// floats ({L re, L im, K re, K im} or {PJ re, PJ im, PM re, PM im}); lane
// (i, kq) loads the whole record of row i, column 4 g + kq (one 16-byte load
// per lane per group g of four columns) and MFMA step j of the group takes
// slot j of it: A[i][kq] = record j of column 4 g + kq, B[kq][n] = the
// real-form entry of that column for output column n (vector n / 2, real
// part for even n).  Slot j reads the source (J for j < 2, M otherwise, or
// the reverse) and forms (x_re, x_im) for j even, (-x_im, x_re) for odd.
// Galerkin rows run two products sharing the loads: E with slots (J, M) and
// coefficients (-Z L, K), H with slots (M, J) and (-L / Z, -K); the interior
// medium's enter with the opposite sign.  Lane (n, kq) ends with rows
// 4 kq + r of column n.
typedef float tf4 __attribute__((ext_vector_type(4)));
constexpr int TOE_MF_WAVES = 16;
constexpr int TOE_MF_DEPTH = 4;   // 16-byte table loads per lane per chunk (two chunks in flight)

// real-form B entry of slot j for a lane of output column n (odd: imaginary)
__device__ inline float mf_form(cx<float> x, int j, bool odd) {
  return (j & 1) == 0 ? (odd ? x.y : x.x) : (odd ? x.x : -x.y);
}

// chunk of TOE_MF_DEPTH column groups starting at group q0 of row records
// Arow[c * stride] (zero where !live or c >= n; groups past the last are
// skipped and left zero); the address is clamped so every load is in bounds
__device__ inline void mf_load(const float *Arow, size_t stride, int n, bool live, int kq, int q0,
                               tf4 (&v)[TOE_MF_DEPTH]) {
  const int nq = (n + 3) >> 2;
#pragma unroll
  for (int u = 0; u < TOE_MF_DEPTH; u++) {
    v[u] = tf4{0.f, 0.f, 0.f, 0.f};
    if (q0 + u < nq) {   // uniform
      const int c = 4 * (q0 + u) + kq;
      const tf4 t = *reinterpret_cast<const tf4 *>(Arow + (size_t)(c < n ? c : n - 1) * stride);
      if (live && c < n) v[u] = t;
    }
  }
}

// acc[k] += sum over source columns c < n of the row records (see mf_load)
// against the B-entries bf(c, bv) fills for c; v holds the first chunk,
// loaded by the caller; each chunk's successor is loaded before its MFMAs.
// Lanes past the last column take column 0's (finite) B-entries against a
// zero record.
template <int NACC, typename BF>
__device__ inline void mf_quads(const float *Arow, size_t stride, int n, bool live, int kq, BF bf, tf4 (&acc)[NACC],
                                tf4 (&v)[TOE_MF_DEPTH]) {
  const int nq = (n + 3) >> 2;
  for (int q0 = 0; q0 < nq; q0 += TOE_MF_DEPTH) {
    tf4 w[TOE_MF_DEPTH];
    mf_load(Arow, stride, n, live, kq, q0 + TOE_MF_DEPTH, w);
#pragma unroll
    for (int u = 0; u < TOE_MF_DEPTH; u++) {
      if (q0 + u >= nq) break;   // uniform
      const int c = 4 * (q0 + u) + kq;
      float bv[NACC][4];
      bf(c < n ? c : 0, bv);
#pragma unroll
      for (int j = 0; j < 4; j++)
#pragma unroll
        for (int k = 0; k < NACC; k++) acc[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(v[u][j], bv[k][j], acc[k], 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < TOE_MF_DEPTH; u++) v[u] = w[u];
  }
}

// Galerkin E/H B-entries of column c from sources xJ, xM with E scales
// (sJ, sJ, sM, sM) and H scales (hM, hM, hJ, hJ)
struct MfGalerkinB {
  const cx<float> *xJ, *xM;
  float sJ, sM, hM, hJ;
  int cv;
  bool odd;
  __device__ void operator()(int c, float (&bv)[2][4]) const {
    const cx<float> x = xJ[c * 8 + cv], y = xM[c * 8 + cv];
#pragma unroll
    for (int j = 0; j < 2; j++) {
      bv[0][j] = sJ * mf_form(x, j, odd);
      bv[0][j + 2] = sM * mf_form(y, j, odd);
      bv[1][j] = hM * mf_form(y, j, odd);
      bv[1][j + 2] = hJ * mf_form(x, j, odd);
    }
  }
};
// point-field B-entries: slots (J, J, M, M) of column c
struct MfPointB {
  const cx<float> *xJ, *xM;
  int cv;
  bool odd;
  __device__ void operator()(int c, float (&bv)[1][4]) const {
    const cx<float> x = xJ[c * 8 + cv], y = xM[c * 8 + cv];
#pragma unroll
    for (int j = 0; j < 2; j++) {
      bv[0][j] = mf_form(x, j, odd);
      bv[0][j + 2] = mf_form(y, j, odd);
    }
  }
};

__global__ void __launch_bounds__(64 * TOE_MF_WAVES) toe_apply_mfma_kernel(ToeDev<float> d) {
  constexpr int NB = 8;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<float> *xs = reinterpret_cast<cx<float> *>(smem_raw);   // [slot][column][v]
  int part, f;
  toe_xcd_order(part, f);
  const int ne_r = d.ne_r, R2 = 2 * NQ * d.nt_r;
  const int gt = (ne_r + 15) / 16, pt = (R2 + 15) / 16;
  const int t = part * TOE_MF_WAVES + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63, m = lane & 15, kq = lane >> 4;
  // the exterior table rows of this wave's tile, first chunk loaded before
  // the spectra are staged (it does not depend on them)
  const bool gal = t < gt;
  const int row = gal ? 16 * t + m : 16 * (t - gt) + m;
  const bool live = t < gt + pt && row < (gal ? ne_r : R2);
  const float *Aext =
      gal ? reinterpret_cast<const float *>(d.GE + (size_t)f * ne_r * ne_r * 2) + (size_t)(live ? row : 0) * 4
          : reinterpret_cast<const float *>(d.PE + (size_t)f * ne_r * R2 * 2) + (size_t)(live ? row : 0) * 4;
  const size_t sext = (size_t)(gal ? ne_r : R2) * 4;
  tf4 v[TOE_MF_DEPTH];
  mf_load(Aext, sext, ne_r, live, kq, 0, v);
  const int nin = 4 * ne_r * NB;
  const cx<float> *Xf = d.X + (size_t)f * nin;
  for (int i = threadIdx.x; i < nin; i += blockDim.x) xs[i] = Xf[i];
  __syncthreads();
  if (t >= gt + pt) return;
  const int cv = m >> 1;
  const bool odd = (m & 1) != 0;
  const int nout = 2 * ne_r + 2 * R2;
  float *Yf = reinterpret_cast<float *>(d.Y + (size_t)f * nout * NB);
  const cx<float> *xJe = xs, *xMe = xs + ne_r * NB, *xJi = xs + 2 * ne_r * NB, *xMi = xs + 3 * ne_r * NB;
  if (gal) {
    tf4 acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
    {
      const float Z = (float)d.Z_e;
      mf_quads<2>(Aext, sext, ne_r, live, kq, MfGalerkinB{xJe, xMe, -Z, 1.f, -1.f / Z, -1.f, cv, odd}, acc, v);
    }
    const float Z = (float)d.Z_i;
    const int bd_lo = d.ebody[min(16 * t, ne_r - 1)], bd_hi = d.ebody[min(16 * t + 15, ne_r - 1)];
    for (int bd = bd_lo; bd <= bd_hi; bd++) {
      const int e0 = d.body_e0[bd], neb = d.body_e0[bd + 1] - e0;
      const bool in = live && row >= e0 && row < e0 + neb;
      const float *A = reinterpret_cast<const float *>(d.GI + ((size_t)f * d.gi_per_f + d.ibase[bd]) * 2) +
                       (size_t)(in ? row - e0 : 0) * 4;
      mf_load(A, (size_t)neb * 4, neb, in, kq, 0, v);
      mf_quads<2>(A, (size_t)neb * 4, neb, in, kq,
                  MfGalerkinB{xJi + e0 * NB, xMi + e0 * NB, Z, -1.f, 1.f / Z, 1.f, cv, odd}, acc, v);
    }
#pragma unroll
    for (int r = 0; r < 4; r++) {
      const int a = 16 * t + 4 * kq + r;
      if (a < ne_r) {
        Yf[((size_t)(2 * a) * NB + cv) * 2 + (odd ? 1 : 0)] = acc[0][r];
        Yf[((size_t)(2 * a + 1) * NB + cv) * 2 + (odd ? 1 : 0)] = acc[1][r];
      }
    }
    return;
  }
  const int pt0 = 16 * (t - gt);
  tf4 accE[1] = {{0.f, 0.f, 0.f, 0.f}}, accI[1] = {{0.f, 0.f, 0.f, 0.f}};
  mf_quads<1>(Aext, sext, ne_r, live, kq, MfPointB{xJe, xMe, cv, odd}, accE, v);
  {
    const int lt_lo = min(pt0, R2 - 1) / (2 * NQ), lt_hi = min(pt0 + 15, R2 - 1) / (2 * NQ);
    const int bd_lo = d.tbody[lt_lo], bd_hi = d.tbody[lt_hi];
    for (int bd = bd_lo; bd <= bd_hi; bd++) {
      const int e0 = d.body_e0[bd], neb = d.body_e0[bd + 1] - e0;
      const int r0 = 2 * NQ * d.body_t0[bd], R2b = 2 * NQ * (d.body_t0[bd + 1] - d.body_t0[bd]);
      const bool in = live && row >= r0 && row < r0 + R2b;
      const float *A = reinterpret_cast<const float *>(d.PI + ((size_t)f * d.pi_per_f + d.pbase[bd]) * 2) +
                       (size_t)(in ? row - r0 : 0) * 4;
      mf_load(A, (size_t)R2b * 4, neb, in, kq, 0, v);
      mf_quads<1>(A, (size_t)R2b * 4, neb, in, kq, MfPointB{xJi + e0 * NB, xMi + e0 * NB, cv, odd}, accI, v);
    }
  }
#pragma unroll
  for (int q = 0; q < 4; q++) {
    const int rr = pt0 + 4 * kq + q;
    if (rr < R2) {
      Yf[((size_t)(2 * ne_r + rr) * NB + cv) * 2 + (odd ? 1 : 0)] = accE[0][q];
      Yf[((size_t)(2 * ne_r + R2 + rr) * NB + cv) * 2 + (odd ? 1 : 0)] = accI[0][q];
    }
  }
}

// stores of the transformed lines [w0, w1) of a group starting at line l0
// (rings j < nr): Galerkin slots scattered to the edges of their ring
// positions, point slots contiguous.  By the calling wave alone (its lanes
// over j) or by the whole work-group (threads over line and ring).
template <typename T>
__device__ inline void toe_inv_store_lines(const ToeDev<T> &d, const cx<T> *buf, int ne, int nb, int l0, int w0, int w1,
                                           bool by_wave) {
  const int P = d.P, nr = d.nr, ne_r = d.ne_r, R2 = 2 * NQ * d.nt_r;
  if (!by_wave) {
    for (int i = threadIdx.x; i < (w1 - w0) * nr; i += blockDim.x) {
      const int li = w0 + i / nr, j = i % nr;
      const int l = l0 + li, slot = l / nb, v = l - slot * nb;
      const cx<T> val = buf[lpad<T>(li * P + j)];
      if (slot < 2 * ne_r) {
        const int e = d.ringmap[(size_t)(slot >> 1) * nr + j];
        if (e >= 0) d.edge_out[((size_t)v * ne + e) * 2 + (slot & 1)] = val * (T)d.edge_sgn[e];
      } else {
        d.pf[((size_t)v * 2 * R2 + slot - 2 * ne_r) * nr + j] = val;
      }
    }
    return;
  }
  const int t0 = threadIdx.x & 63, dt = 64;
  for (int li = w0; li < w1; li++) {
    const int l = l0 + li, slot = l / nb, v = l - slot * nb;   // uniform over the wave
    const cx<T> *line = buf;
    if (slot >= 2 * ne_r) {
      cx<T> *dst = d.pf + ((size_t)v * 2 * R2 + slot - 2 * ne_r) * nr;
      for (int j = t0; j < nr; j += dt) dst[j] = line[lpad<T>(li * P + j)];
      continue;
    }
    const int *rmap = d.ringmap + (size_t)(slot >> 1) * nr;
    cx<T> *dst = d.edge_out + (size_t)v * ne * 2 + (slot & 1);
    for (int j0 = t0; j0 < nr; j0 += TOE_GATHER * dt) {
      int rm[TOE_GATHER], sg[TOE_GATHER];
#pragma unroll
      for (int u = 0; u < TOE_GATHER; u++) rm[u] = rmap[min(j0 + u * dt, nr - 1)];
#pragma unroll
      for (int u = 0; u < TOE_GATHER; u++) sg[u] = d.edge_sgn[rm[u] >= 0 ? rm[u] : 0];
#pragma unroll
      for (int u = 0; u < TOE_GATHER; u++) {
        const int j = j0 + u * dt;
        if (j < nr && rm[u] >= 0) dst[(size_t)rm[u] * 2] = line[lpad<T>(li * P + j)] * (T)sg[u];
      }
    }
  }
}

// inverse: line l = slot * nb + v over f, inverse transform, rings i < nr
// scattered: Galerkin slots to edge_out[v][e][2] (E, H rows; template
// orientation back to the edge's), point slots to pf[v][point][4]
// (exterior t1, t2, interior t1, t2).
template <typename T>
__global__ void __launch_bounds__(TOE_FFT_THREADS) __attribute__((amdgpu_waves_per_eu(toe_fft_waves<T>())))
toe_inv_kernel(ToeDev<T> d, int ne, int np, int nb) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T> *buf = reinterpret_cast<cx<T> *>(smem_raw);
  const int P = d.P;
  const int G = d.lines;
  const int nlines = (2 * d.ne_r + 4 * NQ * d.nt_r) * nb;
  const int l0 = blockIdx.x * G;
  const int nl = min(G, nlines - l0);
  const cx<T> *tws = toe_stage_twiddles<T>(smem_raw, d.tw, P, G);
  const int n = nl * P;
  for (int i0 = threadIdx.x; i0 < n; i0 += TOE_GATHER * blockDim.x) {
    cx<T> y[TOE_GATHER];
#pragma unroll
    for (int u = 0; u < TOE_GATHER; u++) {
      const int i = min(i0 + u * (int)blockDim.x, n - 1);
      const int f = i / nl, li = i - f * nl;
      y[u] = d.Y[(size_t)f * nlines + l0 + li];
    }
#pragma unroll
    for (int u = 0; u < TOE_GATHER; u++) {
      const int i = i0 + u * (int)blockDim.x;
      if (i < n) {
        const int f = i / nl, li = i - f * nl;
        buf[lpad<T>(li * P + f)] = y[u];
      }
    }
  }
  __syncthreads();
  const int nwv = blockDim.x >> 6;
  if (!wave_fits(P, nl, nwv, TOE_FFT_ELEMS)) {
    lds_fft_mr<T, TOE_FFT_ELEMS>(buf, P, nl, 1, P, 0, 1, tws, P, true);
    toe_inv_store_lines(d, buf, ne, nb, l0, 0, nl, false);
    return;
  }
  // each wave transforms its own lines and stores them: no work-group barrier
  lds_fft_wave<T, TOE_FFT_ELEMS>(buf, P, nl, 1, P, 0, 1, tws, P, true);
  const int gw = (nl + nwv - 1) / nwv, wave = threadIdx.x >> 6;   // the wave's lines, as in lds_fft_wave
  const int w0 = min(nl, wave * gw), w1 = min(nl, w0 + gw);
  toe_inv_store_lines(d, buf, ne, nb, l0, w0, w1, true);
}

// local terms and the sigma tests of the point fields, per triangle (like
// the lattice path's testing step, without a lattice): H-row residue
// -1/2 <g, n x (J_e + J_i)>, eq14 Gram <g, J_e + J_i>, and on absorber points
// w sigma (g x n).(E_e^PV + 1/2 n x M) into the H row and
// -w sigma g.(E_i^PV + 1/2 n x M) into the eq14 row, where the PV fields
// come from the periodic sources (their half functions of periodic edges
// only: every other pair is in the sparse rows).  tri_out[v][T][3 half][3 row].
template <typename T>
__global__ void __launch_bounds__(256) toe_local_kernel(DevOperator<T> op, ToeDev<T> d, int nb) {
  const int T_ = blockIdx.x * blockDim.x + threadIdx.x;
  const int v = blockIdx.y;
  if (T_ >= op.nt) return;
  const cx<T> *esrc = op.src + (size_t)3 * op.ne * v;
  const TriRec<T> tr = op.tris[T_];
  const bool per = d.tri_loc[T_] >= 0;
  const T n[3] = {tr.nrm[0], tr.nrm[1], tr.nrm[2]};
  cx<T> out[9];
  for (int k = 0; k < 9; k++) out[k] = czero<T>();
  bool eper[3];
  for (int i = 0; i < 3; i++) eper[i] = d.edge_sgn[tr.edge[i]] != 0;
  for (int q = 0; q < NQ; q++) {
    const PointRec<T> P = op.pts[(size_t)T_ * NQ + q];
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
    cx<T> hnM[3], nJ[3];
    hnM[0] = T(0.5) * (n[1] * Mq[2] - n[2] * Mq[1]);
    hnM[1] = T(0.5) * (n[2] * Mq[0] - n[0] * Mq[2]);
    hnM[2] = T(0.5) * (n[0] * Mq[1] - n[1] * Mq[0]);
    nJ[0] = n[1] * Jsum[2] - n[2] * Jsum[1];
    nJ[1] = n[2] * Jsum[0] - n[0] * Jsum[2];
    nJ[2] = n[0] * Jsum[1] - n[1] * Jsum[0];
    const T w = P.w, ws = P.w * P.sigma;
    cx<T> Ee[3], Ei[3];
    for (int a = 0; a < 3; a++) Ee[a] = Ei[a] = czero<T>();
    if (per && ws != T(0)) {
      const int lt = d.tri_loc[T_], j = d.tri_ring[T_], nr = d.nr;
      const size_t R2 = 2 * (size_t)NQ * d.nt_r, r = 2 * ((size_t)lt * NQ + q);
      const cx<T> *pe = d.pf + ((size_t)v * 2 * R2 + r) * nr + j, *pi = pe + R2 * nr;
      const T *t1 = d.t1 + 3 * (size_t)lt, *t2 = d.t2 + 3 * (size_t)lt;
      for (int a = 0; a < 3; a++) {
        Ee[a] = pe[0] * t1[a] + pe[nr] * t2[a];
        Ei[a] = pi[0] * t1[a] + pi[nr] * t2[a];
      }
    }
    for (int i = 0; i < 3; i++) {
      const T gi[3] = {P.f[3 * i], P.f[3 * i + 1], P.f[3 * i + 2]};
      cx<T> h = czero<T>(), r14 = czero<T>();
      for (int a = 0; a < 3; a++) {
        axpy(h, T(-0.5) * w * gi[a], nJ[a]);
        axpy(r14, w * gi[a], Jsum[a]);
      }
      if (ws != T(0)) {
        const T gxn[3] = {gi[1] * n[2] - gi[2] * n[1], gi[2] * n[0] - gi[0] * n[2], gi[0] * n[1] - gi[1] * n[0]};
        const bool pv = per && eper[i];
        for (int a = 0; a < 3; a++) {
          axpy(h, ws * gxn[a], hnM[a] + (pv ? Ee[a] : czero<T>()));
          axpy(r14, -ws * gi[a], hnM[a] + (pv ? Ei[a] : czero<T>()));
        }
      }
      out[3 * i + 1] += h;
      out[3 * i + 2] += r14;
    }
  }
  cx<T> *to = op.tri_out + (size_t)9 * op.nt * v + (size_t)T_ * 9;
  for (int k = 0; k < 9; k++) to[k] = out[k];
}

// ---------------------------------------------------------------------------
// rows: the periodic sums (edge_out), the local terms (tri_out) and the exact
// entries of every pair with a non-periodic edge, stored column-major so that
// lanes walk rows: short part [j][n] (every row n against non-periodic
// column j; used by periodic rows), long part [m][i] (non-periodic row i
// against every column m)
// ---------------------------------------------------------------------------
template <typename T> __device__ inline T wsum64(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename T>
__device__ inline void row_mac(const RowCoef<T> &c, const cx<T> *cm, cx<T> &e, cx<T> &h, cx<T> &q) {
  const cx<T> Je = cm[0], Ji = cm[1], M = cm[2];
  cmac(e, c.eJi, Ji);
  cmac(e, c.eJe, Je);
  cmac(e, c.eM, M);
  cmac(h, c.hJi, Ji);
  cmac(h, c.hJe, Je);
  cmac(h, c.hM, M);
  cmac(q, c.rJi, Ji);
  cmac(q, c.rM, M);
}

// periodic rows against the non-periodic columns, in R.groups column groups
// (one thread per (row, group)): partial sums rpart[g][b][k][n]
constexpr int TOE_RG_MAX = 16;
template <typename T, int NRB>
__global__ void __launch_bounds__(256) toe_rows_part_kernel(DevOperator<T> op, ToeRows<T> R) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x, g = blockIdx.y;
  if (n >= op.ne) return;
  const EdgeRec r = op.edges[n];
  const T Ze = op.Z_e, Zi = op.Z_i;
  const cx<T> *cur = NRB > 1 ? op.srcI : op.src;   // [m][b][3]
  cx<T> e[NRB], h[NRB], q[NRB];
#pragma unroll
  for (int b = 0; b < NRB; b++) e[b] = h[b] = q[b] = czero<T>();
  const int j0 = (R.ncap * g) / R.groups, j1 = (R.ncap * (g + 1)) / R.groups;
  if (R.edge_sgn[n] != 0) {
    constexpr int DEP = 4;
    int j = j0;
    for (; j + DEP <= j1; j += DEP) {
      cx<T> V[DEP][4], S[DEP][4];
#pragma unroll
      for (int u = 0; u < DEP; u++) {
        const size_t k = ((size_t)(j + u) * op.ne + n) * 4;
#pragma unroll
        for (int t = 0; t < 4; t++) {
          V[u][t] = R.V4S[k + t];
          S[u][t] = r.isR ? R.S4S[k + t] : czero<T>();
        }
      }
#pragma unroll
      for (int u = 0; u < DEP; u++) {
        const RowCoef<T> c = row_coef(V[u], S[u], r.isR != 0, Ze, Zi);
        const cx<T> *cm = cur + (size_t)R.capcol[j + u] * NRB * 3;
#pragma unroll
        for (int b = 0; b < NRB; b++) row_mac(c, cm + 3 * b, e[b], h[b], q[b]);
      }
    }
    for (; j < j1; j++) {
      const size_t k = ((size_t)j * op.ne + n) * 4;
      const RowCoef<T> c = row_coef(R.V4S + k, R.S4S + k, r.isR != 0, Ze, Zi);
      const cx<T> *cm = cur + (size_t)R.capcol[j] * NRB * 3;
#pragma unroll
      for (int b = 0; b < NRB; b++) row_mac(c, cm + 3 * b, e[b], h[b], q[b]);
    }
  }
#pragma unroll
  for (int b = 0; b < NRB; b++) {
    T *p = R.rpart + ((size_t)(g * NRB + b) * 6) * op.ne + n;
    p[0] = e[b].x;
    p[(size_t)op.ne] = e[b].y;
    p[2 * (size_t)op.ne] = h[b].x;
    p[3 * (size_t)op.ne] = h[b].y;
    p[4 * (size_t)op.ne] = q[b].x;
    p[5 * (size_t)op.ne] = q[b].y;
  }
}

// one thread per (edge row, vector): the groups' partial sums, the local
// terms of its two halves and the periodic sums; writes the rows
template <typename T>
__global__ void __launch_bounds__(256) toe_rows_kernel(DevOperator<T> op, ToeRows<T> R, double *__restrict__ y, int nb) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x, b = blockIdx.y;
  if (n >= op.ne) return;
  const EdgeRec r = op.edges[n];
  {
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int g = 0; g < R.groups; g++) {
      const T *p = R.rpart + ((size_t)(g * nb + b) * 6) * op.ne + n;
      for (int k = 0; k < 6; k++) v[k] += (double)p[(size_t)k * op.ne];
    }
    const cx<T> *to = op.tri_out + (size_t)9 * op.nt * b;
    const cx<T> *p0 = to + ((size_t)r.tri[0] * 3 + r.loc[0]) * 3;
    const cx<T> *p1 = to + ((size_t)r.tri[1] * 3 + r.loc[1]) * 3;
    const cx<T> *eo = op.edge_out + ((size_t)b * op.ne + n) * 2;
    const cx<T> E = p0[0] + p1[0] + eo[0], H = p0[1] + p1[1] + eo[1], Q = p0[2] + p1[2];
    double *yb = y + (size_t)2 * op.N * b;
    yb[2 * r.row[0]] = v[0] + E.x;
    yb[2 * r.row[0] + 1] = v[1] + E.y;
    yb[2 * r.row[1]] = v[2] + H.x;
    yb[2 * r.row[1] + 1] = v[3] + H.y;
    if (r.isR) {
      yb[2 * r.row[2]] = v[4] + Q.x;
      yb[2 * r.row[2] + 1] = v[5] + Q.y;
    }
  }
}

// long rows: one work-group per chunk of TOE_LCH columns; the chunk's
// currents in LDS; lane i walks long row i over the chunk; partial sums per
// (chunk, row, vector)
constexpr int TOE_LCH = 64;
template <typename T, int NRB>
__global__ void __launch_bounds__(256) toe_long_kernel(DevOperator<T> op, ToeRows<T> R) {
  __shared__ cx<T> xs[TOE_LCH * NRB * 3];
  const int ch = blockIdx.x, c0 = ch * TOE_LCH, nc = min(TOE_LCH, op.ne - c0);
  const cx<T> *cur = NRB > 1 ? op.srcI : op.src;
  for (int i = threadIdx.x; i < nc * NRB * 3; i += blockDim.x) xs[i] = cur[(size_t)c0 * NRB * 3 + i];
  __syncthreads();
  const T Ze = op.Z_e, Zi = op.Z_i;
  for (int i = threadIdx.x; i < R.nlong; i += blockDim.x) {
    const EdgeRec r = op.edges[R.capcol[i]];
    cx<T> e[NRB], h[NRB], q[NRB];
#pragma unroll
    for (int b = 0; b < NRB; b++) e[b] = h[b] = q[b] = czero<T>();
    constexpr int DEP = 4;
    int m = 0;
    for (; m + DEP <= nc; m += DEP) {
      cx<T> V[DEP][4], S[DEP][4];
#pragma unroll
      for (int u = 0; u < DEP; u++) {
        const size_t k = ((size_t)(c0 + m + u) * R.nlong + i) * 4;
#pragma unroll
        for (int t = 0; t < 4; t++) {
          V[u][t] = R.V4L[k + t];
          S[u][t] = r.isR ? R.S4L[k + t] : czero<T>();
        }
      }
#pragma unroll
      for (int u = 0; u < DEP; u++) {
        const RowCoef<T> c = row_coef(V[u], S[u], r.isR != 0, Ze, Zi);
        const cx<T> *cm = xs + (size_t)(m + u) * NRB * 3;
#pragma unroll
        for (int b = 0; b < NRB; b++) row_mac(c, cm + 3 * b, e[b], h[b], q[b]);
      }
    }
    for (; m < nc; m++) {
      const size_t k = ((size_t)(c0 + m) * R.nlong + i) * 4;
      const RowCoef<T> c = row_coef(R.V4L + k, R.S4L + k, r.isR != 0, Ze, Zi);
      const cx<T> *cm = xs + (size_t)m * NRB * 3;
#pragma unroll
      for (int b = 0; b < NRB; b++) row_mac(c, cm + 3 * b, e[b], h[b], q[b]);
    }
    T *p = R.part + ((size_t)ch * R.nlong + i) * NRB * 6;
#pragma unroll
    for (int b = 0; b < NRB; b++) {
      p[6 * b] = e[b].x;
      p[6 * b + 1] = e[b].y;
      p[6 * b + 2] = h[b].x;
      p[6 * b + 3] = h[b].y;
      p[6 * b + 4] = q[b].x;
      p[6 * b + 5] = q[b].y;
    }
  }
}

// ---------------------------------------------------------------------------
// Sparse rows of 8 FP32 vectors on the matrix cores.  A stored pair holds
// two 16-byte records {L_e, K_e}, {L_i, K_i} (on absorber rows two more, the
// sigma tests' {L_r, K_r}, {L_s, K_s}); with the column's currents the row
// sums (the coefficients of row_coef) are
//   E = L_e (-Z_e J_e) + K_e M + L_i (Z_i J_i) + K_i M
//   H = L_e (-M / Z_e) + K_e (-J_e) + L_i (-M / Z_i) + K_i J_i
//       [+ L_r (-Z_e J_e) + K_r M]
//   Q = [L_s (Z_i J_i) + K_s M]
// As in the block products, lane (i, kq) loads the records of row i, column
// 4 g + kq, MFMA step j takes slot j of a record and the B entries are the
// real forms of the scaled currents (output column n: vector n / 2, real
// part for even n); lane (n, kq) ends with rows 4 kq + r of column n.
// ---------------------------------------------------------------------------
struct SpForms {
  float e1[4], h1[4], e2[4], h2[4], h3[4], q4[4];
};
__device__ inline void sp_forms(const cx<float> *cm, float Ze, float Zi, bool odd, SpForms &b) {
  const cx<float> Je = cm[0], Ji = cm[1], M = cm[2];
  const cx<float> a = Je * (-Ze), mz = M * (-1.f / Ze), ci = Ji * Zi, mi = M * (-1.f / Zi), nJe = -Je;
#pragma unroll
  for (int j = 0; j < 2; j++) {
    b.e1[j] = mf_form(a, j, odd);
    b.e1[j + 2] = mf_form(M, j, odd);
    b.h1[j] = mf_form(mz, j, odd);
    b.h1[j + 2] = mf_form(nJe, j, odd);
    b.e2[j] = mf_form(ci, j, odd);
    b.e2[j + 2] = mf_form(M, j, odd);
    b.h2[j] = mf_form(mi, j, odd);
    b.h2[j + 2] = mf_form(Ji, j, odd);
    b.h3[j] = b.e1[j];
    b.h3[j + 2] = b.e1[j + 2];
    b.q4[j] = b.e2[j];
    b.q4[j + 2] = b.e2[j + 2];
  }
}
// one 16-row tile's records of one column: r[0..1] always, r[2..3] on absorber rows
struct SpRec {
  tf4 r[4];
};
__device__ inline void sp_load(const cx<float> *V4, const cx<float> *S4, size_t k, bool live, bool isR, bool withR,
                               SpRec &o) {
  const tf4 z = {0.f, 0.f, 0.f, 0.f};
  o.r[0] = live ? *reinterpret_cast<const tf4 *>(V4 + k) : z;
  o.r[1] = live ? *reinterpret_cast<const tf4 *>(V4 + k + 2) : z;
  if (withR) {   // wave-uniform
    o.r[2] = isR ? *reinterpret_cast<const tf4 *>(S4 + k) : z;
    o.r[3] = isR ? *reinterpret_cast<const tf4 *>(S4 + k + 2) : z;
  }
}
__device__ inline void sp_mfma(const SpRec &a, const SpForms &b, bool withR, tf4 &E, tf4 &H, tf4 &Q) {
#pragma unroll
  for (int j = 0; j < 4; j++) {
    E = __builtin_amdgcn_mfma_f32_16x16x4f32(a.r[0][j], b.e1[j], E, 0, 0, 0);
    H = __builtin_amdgcn_mfma_f32_16x16x4f32(a.r[0][j], b.h1[j], H, 0, 0, 0);
    E = __builtin_amdgcn_mfma_f32_16x16x4f32(a.r[1][j], b.e2[j], E, 0, 0, 0);
    H = __builtin_amdgcn_mfma_f32_16x16x4f32(a.r[1][j], b.h2[j], H, 0, 0, 0);
  }
  if (withR) {
#pragma unroll
    for (int j = 0; j < 4; j++) {
      H = __builtin_amdgcn_mfma_f32_16x16x4f32(a.r[2][j], b.h3[j], H, 0, 0, 0);
      Q = __builtin_amdgcn_mfma_f32_16x16x4f32(a.r[3][j], b.q4[j], Q, 0, 0, 0);
    }
  }
}

// periodic rows against the non-periodic columns of group g: one wave per
// 16-row tile, the group's column currents in LDS (dynamic, [column][v][3]);
// partial sums rpart[g][v][6][row] as toe_rows_part_kernel writes them
__global__ void __launch_bounds__(256) toe_rows_part_mfma_kernel(DevOperator<float> op, ToeRows<float> R) {
  constexpr int NB = 8;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<float> *xs = reinterpret_cast<cx<float> *>(smem_raw);
  const int g = blockIdx.y;
  const int j0 = (R.ncap * g) / R.groups, j1 = (R.ncap * (g + 1)) / R.groups, nj = j1 - j0;
  for (int i = threadIdx.x; i < nj * NB * 3; i += blockDim.x) {
    const int jj = i / (NB * 3);
    xs[i] = op.srcI[(size_t)R.capcol[j0 + jj] * NB * 3 + (i - jj * NB * 3)];
  }
  __syncthreads();
  const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (16 * tile >= op.ne) return;   // wave-uniform
  const int lane = threadIdx.x & 63, m = lane & 15, kq = lane >> 4;
  const int n = 16 * tile + m;
  const int fl = n < op.ne ? R.eflag[n] : 0;
  const bool live = (fl & 1) != 0, isR = live && (fl & 2) != 0;
  const bool withR = __ballot(isR) != 0;
  const float Ze = op.Z_e, Zi = op.Z_i;
  const int cv = m >> 1;
  const bool odd = (m & 1) != 0;
  tf4 E = {0.f, 0.f, 0.f, 0.f}, H = E, Q = E;
  const int nq = (nj + 3) >> 2;
  const size_t rowk = (size_t)(live ? n : 0) * 4;
  SpRec cur{}, nxt{};
  {
    const bool cok = kq < nj;
    sp_load(R.V4S, R.S4S, (size_t)(j0 + (cok ? kq : 0)) * op.ne * 4 + rowk, live && cok, isR && cok, withR, cur);
  }
  for (int q = 0; q < nq; q++) {
    const int jj = 4 * q + kq;
    if (q + 1 < nq) {   // next column group's records first
      const int jn = jj + 4;
      const bool cok = jn < nj;
      sp_load(R.V4S, R.S4S, (size_t)(j0 + (cok ? jn : 0)) * op.ne * 4 + rowk, live && cok, isR && cok, withR, nxt);
    }
    SpForms b;
    sp_forms(xs + ((size_t)(jj < nj ? jj : 0) * NB + cv) * 3, Ze, Zi, odd, b);
    sp_mfma(cur, b, withR, E, H, Q);
    cur = nxt;
  }
  float *p = R.rpart + (size_t)((g * NB + cv) * 6 + (odd ? 1 : 0)) * op.ne;
#pragma unroll
  for (int r = 0; r < 4; r++) {
    const int nr = 16 * tile + 4 * kq + r;
    if (nr < op.ne) {
      p[nr] = E[r];
      p[2 * (size_t)op.ne + nr] = H[r];
      p[4 * (size_t)op.ne + nr] = Q[r];
    }
  }
}

// long rows: one work-group per chunk of TOE_LCH columns (their currents in
// LDS); each wave takes TOE_SP_TILES row tiles at a time and walks the
// chunk's column groups, the next group's records loaded before the current
// group's products, the B entries shared by its tiles; partial sums per
// (chunk, row, vector) as toe_long_kernel writes them
constexpr int TOE_SP_TILES = 2;
__global__ void __launch_bounds__(256) toe_long_mfma_kernel(DevOperator<float> op, ToeRows<float> R) {
  constexpr int NB = 8;
  __shared__ cx<float> xs[TOE_LCH * NB * 3];
  const int ch = blockIdx.x, c0 = ch * TOE_LCH, nc = min(TOE_LCH, op.ne - c0);
  for (int i = threadIdx.x; i < nc * NB * 3; i += blockDim.x) xs[i] = op.srcI[(size_t)c0 * NB * 3 + i];
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, m = lane & 15, kq = lane >> 4;
  const int cv = m >> 1;
  const bool odd = (m & 1) != 0;
  const float Ze = op.Z_e, Zi = op.Z_i;
  const int ntile = (R.nlong + 15) / 16, nq = (nc + 3) >> 2;
  for (int t0 = wave * TOE_SP_TILES; t0 < ntile; t0 += 4 * TOE_SP_TILES) {
    bool live[TOE_SP_TILES], isR[TOE_SP_TILES], withR[TOE_SP_TILES];
    size_t rowk[TOE_SP_TILES];
    tf4 E[TOE_SP_TILES], H[TOE_SP_TILES], Q[TOE_SP_TILES];
#pragma unroll
    for (int u = 0; u < TOE_SP_TILES; u++) {
      const int i = 16 * (t0 + u) + m;
      live[u] = t0 + u < ntile && i < R.nlong;
      isR[u] = live[u] && (R.eflag[R.capcol[live[u] ? i : 0]] & 2) != 0;
      withR[u] = __ballot(isR[u]) != 0;
      rowk[u] = (size_t)(live[u] ? i : 0) * 4;
      E[u] = tf4{0.f, 0.f, 0.f, 0.f};
      H[u] = E[u];
      Q[u] = E[u];
    }
    SpRec a[TOE_SP_TILES], an[TOE_SP_TILES];
    {
      const bool cok = kq < nc;
      const size_t ck = (size_t)(c0 + (cok ? kq : 0)) * R.nlong * 4;
#pragma unroll
      for (int u = 0; u < TOE_SP_TILES; u++)
        sp_load(R.V4L, R.S4L, ck + rowk[u], live[u] && cok, isR[u] && cok, withR[u], a[u]);
    }
    for (int q = 0; q < nq; q++) {
      const int col = 4 * q + kq;
      if (q + 1 < nq) {
        const bool cok = col + 4 < nc;
        const size_t ck = (size_t)(c0 + (cok ? col + 4 : 0)) * R.nlong * 4;
#pragma unroll
        for (int u = 0; u < TOE_SP_TILES; u++)
          sp_load(R.V4L, R.S4L, ck + rowk[u], live[u] && cok, isR[u] && cok, withR[u], an[u]);
      }
      SpForms b;
      sp_forms(xs + ((size_t)(col < nc ? col : 0) * NB + cv) * 3, Ze, Zi, odd, b);
#pragma unroll
      for (int u = 0; u < TOE_SP_TILES; u++) {
        sp_mfma(a[u], b, withR[u], E[u], H[u], Q[u]);
        a[u] = an[u];
      }
    }
#pragma unroll
    for (int u = 0; u < TOE_SP_TILES; u++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int i = 16 * (t0 + u) + 4 * kq + r;
        if (t0 + u < ntile && i < R.nlong) {
          float *p = R.part + (((size_t)ch * R.nlong + i) * NB + cv) * 6 + (odd ? 1 : 0);
          p[0] = E[u][r];
          p[2] = H[u][r];
          p[4] = Q[u][r];
        }
      }
  }
}

// long rows += sum over chunks: one wave per (row, vector), lanes over chunks
template <typename T>
__global__ void toe_long_reduce_kernel(DevOperator<T> op, ToeRows<T> R, double *y, int nb) {
  const int w = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, lane = threadIdx.x & 63;
  if (w >= R.nlong * nb) return;   // wave-uniform
  const int i = w / nb, b = w - i * nb;
  const EdgeRec r = op.edges[R.capcol[i]];
  double s6[6] = {0, 0, 0, 0, 0, 0};
  for (int ch = lane; ch < R.nchunk; ch += 64) {
    const T *p = R.part + (((size_t)ch * R.nlong + i) * nb + b) * 6;
    for (int k = 0; k < 6; k++) s6[k] += (double)p[k];
  }
  for (int k = 0; k < 6; k++) s6[k] = wsum64(s6[k]);
  if (lane != 0) return;
  double *yb = y + (size_t)2 * op.N * b;
  yb[2 * r.row[0]] += s6[0];
  yb[2 * r.row[0] + 1] += s6[1];
  yb[2 * r.row[1]] += s6[2];
  yb[2 * r.row[1] + 1] += s6[3];
  if (r.isR) {
    yb[2 * r.row[2]] += s6[4];
    yb[2 * r.row[2] + 1] += s6[5];
  }
}

template <typename T>
void launch_toe_rows(const DevOperator<T> &op, const ToeRows<T> &R, double *y, hipStream_t s, int nb, int parts) {
  const int nchunk = (op.ne + TOE_LCH - 1) / TOE_LCH;
  const bool lng = (parts & TOE_LONG) && R.nlong > 0, sht = (parts & TOE_SHORT) != 0;
  // 8 FP32 vectors: both sparse parts on the matrix cores (the group's column
  // currents must fit the LDS)
  const size_t sp_lds = sizeof(cx<float>) * 8 * 3 * (size_t)((R.ncap + R.groups - 1) / R.groups + 1);
  if (sizeof(T) == sizeof(float) && nb == 8 && R.sparse_form == 0 && sp_lds <= 65536) {
    const DevOperator<float> &of = *reinterpret_cast<const DevOperator<float> *>(&op);
    const ToeRows<float> &rf = *reinterpret_cast<const ToeRows<float> *>(&R);
    if (lng) hipLaunchKernelGGL(toe_long_mfma_kernel, dim3(nchunk), dim3(256), 0, s, of, rf);
    if (sht)
      hipLaunchKernelGGL(toe_rows_part_mfma_kernel, dim3((op.ne + 63) / 64, R.groups), dim3(256), sp_lds, s, of, rf);
  } else {
#define SCABS_TOE_ROWS(NB)                                                                                           \
  do {                                                                                                               \
    if (lng) hipLaunchKernelGGL((toe_long_kernel<T, NB>), dim3(nchunk), dim3(256), 0, s, op, R);                      \
    if (sht)                                                                                                         \
      hipLaunchKernelGGL((toe_rows_part_kernel<T, NB>), dim3((op.ne + 255) / 256, R.groups), dim3(256), 0, s, op, R);   \
  } while (0)
    switch (nb) {
      case 1: SCABS_TOE_ROWS(1); break;
      case 2: SCABS_TOE_ROWS(2); break;
      case 3: SCABS_TOE_ROWS(3); break;
      case 4: SCABS_TOE_ROWS(4); break;
      case 5: SCABS_TOE_ROWS(5); break;
      case 6: SCABS_TOE_ROWS(6); break;
      case 7: SCABS_TOE_ROWS(7); break;
      default: SCABS_TOE_ROWS(8); break;
    }
#undef SCABS_TOE_ROWS
  }
  if (!(parts & TOE_SUM)) return;
  hipLaunchKernelGGL(toe_rows_kernel<T>, dim3((op.ne + 255) / 256, nb), dim3(256), 0, s, op, R, y, nb);
  if (R.nlong > 0)
    hipLaunchKernelGGL(toe_long_reduce_kernel<T>, dim3((R.nlong * nb * 64 + 255) / 256), dim3(256), 0, s, op, R, y, nb);
}
template void launch_toe_rows<float>(const DevOperator<float> &, const ToeRows<float> &, double *, hipStream_t, int,
                                     int);
template void launch_toe_rows<double>(const DevOperator<double> &, const ToeRows<double> &, double *, hipStream_t,
                                      int, int);
int toe_long_chunk() { return TOE_LCH; }
int toe_row_groups() { return TOE_RG_MAX; }

template <typename T>
void launch_toe_product(const DevOperator<T> &op, const ToeDev<T> &d, hipStream_t s, int nb, int parts) {
  const int G = d.lines;
  const int nin = 4 * d.ne_r * nb;
  if (parts & TOE_FWD)
    hipLaunchKernelGGL(toe_fwd_kernel<T>, dim3((nin + G - 1) / G), dim3(TOE_FFT_THREADS),
                       toe_fft_launch_lds(toe_fwd_kernel<T>, toe_fft_lds<T>(d.P, G)), s, d, op.src, op.srcI, op.ne, nb);
  if (!(parts & TOE_APPLY)) goto inverse;
  {
  const int R2 = 2 * NQ * d.nt_r;
  const int rows = d.ne_r + R2;
#define SCABS_TOE_APPLY(NBV)                                                                                         \
  do {                                                                                                               \
    const size_t lds = sizeof(cx<T>) * 4 * d.ne_r * (NBV);                                                           \
    if (lds > 65536)                                                                                                 \
      (void)hipFuncSetAttribute((const void *)toe_apply_kernel<T, NBV>, hipFuncAttributeMaxDynamicSharedMemorySize,   \
                                (int)lds);                                                                           \
    hipLaunchKernelGGL((toe_apply_kernel<T, NBV>), dim3((rows + 255) / 256, d.P), dim3(256), lds, s, d);              \
  } while (0)
  switch (nb) {
    case 1: SCABS_TOE_APPLY(1); break;
    case 2: SCABS_TOE_APPLY(2); break;
    case 3: SCABS_TOE_APPLY(3); break;
    case 4: SCABS_TOE_APPLY(4); break;
    case 5: SCABS_TOE_APPLY(5); break;
    case 6: SCABS_TOE_APPLY(6); break;
    case 7: SCABS_TOE_APPLY(7); break;
    default:
      if (sizeof(T) == sizeof(float) && d.apply_form == 0) {
        // eight vectors: the matrix-core form
        const int tiles = (d.ne_r + 15) / 16 + (R2 + 15) / 16;
        const size_t lds = sizeof(cx<float>) * 4 * d.ne_r * 8;
        if (lds > 65536)
          (void)hipFuncSetAttribute((const void *)toe_apply_mfma_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)lds);
        hipLaunchKernelGGL(toe_apply_mfma_kernel, dim3((tiles + TOE_MF_WAVES - 1) / TOE_MF_WAVES, d.P),
                           dim3(64 * TOE_MF_WAVES), lds, s, *reinterpret_cast<const ToeDev<float> *>(&d));
      } else {
        SCABS_TOE_APPLY(8);
      }
      break;
  }
#undef SCABS_TOE_APPLY
  }
inverse:
  if (parts & TOE_INV) {
    const int R2 = 2 * NQ * d.nt_r;
    const int nout = (2 * d.ne_r + 2 * R2) * nb;
    hipLaunchKernelGGL(toe_inv_kernel<T>, dim3((nout + G - 1) / G), dim3(TOE_FFT_THREADS),
                       toe_fft_launch_lds(toe_inv_kernel<T>, toe_fft_lds<T>(d.P, G)), s, d, op.ne, op.np, nb);
    hipLaunchKernelGGL(toe_local_kernel<T>, dim3((op.nt + 255) / 256, nb), dim3(256), 0, s, op, d, nb);
  }
}
template void launch_toe_product<float>(const DevOperator<float> &, const ToeDev<float> &, hipStream_t, int, int);
template void launch_toe_product<double>(const DevOperator<double> &, const ToeDev<double> &, hipStream_t, int, int);

size_t toe_apply_lds_bytes(int ne_r, int nb, size_t elem) { return elem * 4 * (size_t)ne_r * nb; }

// ---------------------------------------------------------------------------
// circulant preconditioner of the lossless guide block A_LL (fast-solver
// appendix): on the unknowns J, M of the sigma-free periodic edges A_LL is
// block Toeplitz over the rings with the blocks of the E and H rows
//   E = -(Z_e L_e + Z_i L_i) J + (K_e + K_i) M
//   H = -(K_e + K_i) J - (L_e / Z_e + L_i / Z_i) M        (J_i = -J, M_i = -M)
// embedded in its circulant of length P (the product's); the inverse of the
// circulant is the per-frequency inverse of the symbol.  Frequency vectors
// are ordered (J_0, M_0, J_1, M_1, ...) over the template edges.
// ---------------------------------------------------------------------------
// symbol at frequency blockIdx.y, 2 ne_r square, row-major (rows E_a, H_a)
__global__ void pc_circ_symbol_kernel(ToeDev<double> d, cx<double> *__restrict__ S) {
  const int f = blockIdx.y, ne_r = d.ne_r, n = 2 * ne_r;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)ne_r * ne_r) return;
  const int b = (int)(idx / ne_r), a = (int)(idx % ne_r);
  const cx<double> *ge = d.GE + ((size_t)f * ne_r * ne_r + (size_t)b * ne_r + a) * 2;
  cx<double> Le = ge[0], Ke = ge[1], Li = {0, 0}, Ki = {0, 0};
  const int bd = d.ebody[a];
  if (d.ebody[b] == bd) {
    const int e0 = d.body_e0[bd], neb = d.body_e0[bd + 1] - e0;
    const cx<double> *gi = d.GI + ((size_t)f * d.gi_per_f + d.ibase[bd] + (size_t)(b - e0) * neb + (a - e0)) * 2;
    Li = gi[0];
    Ki = gi[1];
  }
  const double P = d.P, Ze = d.Z_e, Zi = d.Z_i;   // the tables hold the symbol / P
  cx<double> *r0 = S + ((size_t)f * n + 2 * a) * n, *r1 = r0 + n;
  r0[2 * b] = (Le * Ze + Li * Zi) * (-P);
  r0[2 * b + 1] = (Ke + Ki) * P;
  r1[2 * b] = (Ke + Ki) * (-P);
  r1[2 * b + 1] = (Le * (1.0 / Ze) + Li * (1.0 / Zi)) * (-P);
}

// batched inverse by Gauss-Jordan elimination with partial pivoting (FP64):
// A (n x n row-major, destroyed) -> B = A^-1, one work-group per matrix,
// n <= PC_GJ_MAX; a zero pivot leaves B's matrix filled with NaN
constexpr int PC_GJ_THREADS = 1024, PC_GJ_MAX = 1024;
__global__ void __launch_bounds__(PC_GJ_THREADS) gj_inverse_kernel(cx<double> *A, cx<double> *B, int n) {
  A += (size_t)blockIdx.x * n * n;
  B += (size_t)blockIdx.x * n * n;
  __shared__ double rv[PC_GJ_THREADS];
  __shared__ int ri[PC_GJ_THREADS];
  __shared__ cx<double> m[PC_GJ_MAX];
  __shared__ cx<double> piv;
  const int t = threadIdx.x, nt = blockDim.x;
  for (int i = t; i < n * n; i += nt) B[i] = (i / n == i % n) ? cx<double>{1.0, 0.0} : cx<double>{0.0, 0.0};
  for (int k = 0; k < n; k++) {
    __syncthreads();
    double best = -1.0;
    int bi = k;
    for (int i = k + t; i < n; i += nt) {
      const cx<double> v = A[(size_t)i * n + k];
      const double a = v.x * v.x + v.y * v.y;
      if (a > best) {
        best = a;
        bi = i;
      }
    }
    rv[t] = best;
    ri[t] = bi;
    __syncthreads();
    for (int w = nt / 2; w > 0; w >>= 1) {
      if (t < w && (rv[t + w] > rv[t] || (rv[t + w] == rv[t] && ri[t + w] < ri[t]))) {
        rv[t] = rv[t + w];
        ri[t] = ri[t + w];
      }
      __syncthreads();
    }
    const int p = ri[0];
    if (p != k)
      for (int j = t; j < n; j += nt) {
        const cx<double> a0 = A[(size_t)k * n + j], b0 = B[(size_t)k * n + j];
        A[(size_t)k * n + j] = A[(size_t)p * n + j];
        B[(size_t)k * n + j] = B[(size_t)p * n + j];
        A[(size_t)p * n + j] = a0;
        B[(size_t)p * n + j] = b0;
      }
    __syncthreads();
    if (t == 0) {
      const cx<double> v = A[(size_t)k * n + k];
      const double den = v.x * v.x + v.y * v.y;
      piv = den > 0 ? cx<double>{v.x / den, -v.y / den} : cx<double>{NAN, NAN};
    }
    __syncthreads();
    for (int j = t; j < n; j += nt) {
      A[(size_t)k * n + j] = A[(size_t)k * n + j] * piv;
      B[(size_t)k * n + j] = B[(size_t)k * n + j] * piv;
    }
    for (int i = t; i < n; i += nt) m[i] = i == k ? cx<double>{0.0, 0.0} : A[(size_t)i * n + k];
    __syncthreads();
    for (int64_t q = t; q < (int64_t)n * 2 * n; q += nt) {
      const int i = (int)(q / (2 * n)), j = (int)(q % (2 * n));
      if (i == k) continue;
      if (j < n)
        A[(size_t)i * n + j] -= m[i] * A[(size_t)k * n + j];
      else
        B[(size_t)i * n + j - n] -= m[i] * B[(size_t)k * n + j - n];
    }
  }
}

// inverse tables Tinv[f][j][i] = (S(f)^-1)[i][j] / P in both precisions
__global__ void pc_circ_store_kernel(const cx<double> *__restrict__ B, int n, int64_t total, double invP,
                                     cx<double> *__restrict__ T64, cx<float> *__restrict__ T32) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t f = q / ((int64_t)n * n), r = q % ((int64_t)n * n);
    const int j = (int)(r / n), i = (int)(r % n);
    const cx<double> v = B[(size_t)f * n * n + (size_t)i * n + j] * invP;
    T64[q] = v;
    T32[q] = {(float)v.x, (float)v.y};
  }
}

void launch_pc_circ_setup(const ToeDev<double> &d, cx<double> *S, cx<double> *B, cx<double> *T64, cx<float> *T32,
                          hipStream_t s) {
  const int n = 2 * d.ne_r;
  const int64_t ab = (int64_t)d.ne_r * d.ne_r;
  hipLaunchKernelGGL(pc_circ_symbol_kernel, dim3((unsigned)((ab + 255) / 256), d.P), dim3(256), 0, s, d, S);
  hipLaunchKernelGGL(gj_inverse_kernel, dim3(d.P), dim3(PC_GJ_THREADS), 0, s, S, B, n);
  const int64_t total = (int64_t)d.P * n * n;
  hipLaunchKernelGGL(pc_circ_store_kernel, dim3(4096), dim3(256), 0, s, (const cx<double> *)B, n, total,
                     1.0 / d.P, T64, T32);
}
int pc_circ_max_order() { return PC_GJ_MAX; }

// forward: lines l = (2 a + s) nb + v (s = 0 J, 1 M of template edge a,
// vector v): the L unknowns of the periodic edges at rings j < nr (template
// orientation), zero for absorber edges and beyond; transformed; X[f][l]
template <typename TI, typename T>
__global__ void __launch_bounds__(TOE_FFT_THREADS) __attribute__((amdgpu_waves_per_eu(toe_fft_waves<T>())))
pc_circ_fwd_kernel(ToeDev<T> d, const EdgeRec *__restrict__ edges, const cx<TI> *__restrict__ x, int64_t N, int nb,
                   cx<T> *__restrict__ X) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T> *buf = reinterpret_cast<cx<T> *>(smem_raw);
  const int P = d.P, nr = d.nr, G = d.lines;
  const int nlines = 2 * d.ne_r * nb;
  const int l0 = blockIdx.x * G, nl = min(G, nlines - l0);
  const cx<T> *tws = toe_stage_twiddles<T>(smem_raw, d.tw, P, G);
  const int n = nl * P;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int li = i / P, j = i - li * P;
    const int l = l0 + li, q = l / nb, v = l - q * nb, a = q >> 1, sl = q & 1;
    cx<T> val = czero<T>();
    if (j < nr) {
      const int e = d.ringmap[(size_t)a * nr + j];
      if (e >= 0) {
        const EdgeRec r = edges[e];
        if (!r.isR) {
          const cx<TI> u = x[(size_t)v * N + r.col[sl]];
          val = cx<T>{(T)u.x, (T)u.y} * (T)d.edge_sgn[e];
        }
      }
    }
    buf[lpad<T>(i)] = val;
  }
  __syncthreads();
  if (wave_fits(P, nl, blockDim.x >> 6, TOE_FFT_ELEMS))
    lds_fft<T, TOE_FFT_ELEMS, TOE_FFT_ELEMS, true>(buf, P, nl, 1, P, 0, 1, tws, P, false);
  else
    lds_fft_mr<T, TOE_FFT_ELEMS>(buf, P, nl, 1, P, 0, 1, tws, P, false);
  for (int i = threadIdx.x; i < nl * P; i += blockDim.x) {
    const int f = i / nl, li = i - f * nl;
    X[(size_t)f * nlines + l0 + li] = buf[lpad<T>(li * P + f)];
  }
}

// per frequency: Y[f][i][v] = sum_j Tinv[f][j][i] X[f][j][v]; transposed:
// the symbol's inverse at -f, transposed
template <typename T, int NB>
__global__ void __launch_bounds__(256) pc_circ_apply_kernel(const cx<T> *__restrict__ Tinv, const cx<T> *__restrict__ X,
                                                             cx<T> *__restrict__ Y, int n, int P, int trans) {
  const int f = blockIdx.y, i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int fs = trans ? (P - f) % P : f;
  const cx<T> *Xf = X + (size_t)f * n * NB;
  cx<T> acc[NB];
#pragma unroll
  for (int v = 0; v < NB; v++) acc[v] = czero<T>();
  for (int j = 0; j < n; j++) {
    const cx<T> c = trans ? Tinv[((size_t)fs * n + i) * n + j] : Tinv[((size_t)fs * n + j) * n + i];
#pragma unroll
    for (int v = 0; v < NB; v++) acc[v] += c * Xf[(size_t)j * NB + v];
  }
#pragma unroll
  for (int v = 0; v < NB; v++) Y[((size_t)f * n + i) * NB + v] = acc[v];
}

// inverse transform of the lines; rings j < nr of L periodic edges written
// to y (template orientation back to the edge's)
template <typename T>
__global__ void __launch_bounds__(TOE_FFT_THREADS) __attribute__((amdgpu_waves_per_eu(toe_fft_waves<T>())))
pc_circ_inv_kernel(ToeDev<T> d, const EdgeRec *__restrict__ edges, const cx<T> *__restrict__ Y, int64_t N, int nb,
                   cx<double> *__restrict__ y) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T> *buf = reinterpret_cast<cx<T> *>(smem_raw);
  const int P = d.P, nr = d.nr, G = d.lines;
  const int nlines = 2 * d.ne_r * nb;
  const int l0 = blockIdx.x * G, nl = min(G, nlines - l0);
  const cx<T> *tws = toe_stage_twiddles<T>(smem_raw, d.tw, P, G);
  for (int i = threadIdx.x; i < nl * P; i += blockDim.x) {
    const int f = i / nl, li = i - f * nl;
    buf[lpad<T>(li * P + f)] = Y[(size_t)f * nlines + l0 + li];
  }
  __syncthreads();
  lds_fft_mr<T, TOE_FFT_ELEMS>(buf, P, nl, 1, P, 0, 1, tws, P, true);
  for (int i = threadIdx.x; i < nl * nr; i += blockDim.x) {
    const int li = i / nr, j = i - li * nr;
    const int l = l0 + li, q = l / nb, v = l - q * nb, a = q >> 1, sl = q & 1;
    const int e = d.ringmap[(size_t)a * nr + j];
    if (e < 0) continue;
    const EdgeRec r = edges[e];
    if (r.isR) continue;
    const cx<T> val = buf[lpad<T>(li * P + j)] * (T)d.edge_sgn[e];
    y[(size_t)v * N + r.col[sl]] = {(double)val.x, (double)val.y};
  }
}

// L unknowns of non-periodic edges pass through (no block of A_LL covers them)
template <typename TI>
__global__ void pc_identity_kernel(const EdgeRec *__restrict__ edges, const int *__restrict__ edge_sgn, int ne,
                                   const cx<TI> *__restrict__ x, int64_t N, int nb, cx<double> *__restrict__ y) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x, v = blockIdx.y;
  if (e >= ne || v >= nb) return;
  const EdgeRec r = edges[e];
  if (r.isR || edge_sgn[e] != 0) return;
  for (int s = 0; s < 2; s++) {
    const cx<TI> u = x[(size_t)v * N + r.col[s]];
    y[(size_t)v * N + r.col[s]] = {(double)u.x, (double)u.y};
  }
}

template <typename TI, typename T>
void launch_pc_circ_apply(const ToeDev<T> &d, const EdgeRec *edges, const cx<T> *Tinv, const cx<TI> *x, int64_t N,
                          int nb, bool trans, cx<T> *X, cx<T> *Y, cx<double> *y, int ne, hipStream_t s) {
  const int G = d.lines, n = 2 * d.ne_r;
  const int nlines = n * nb;
  hipLaunchKernelGGL((pc_circ_fwd_kernel<TI, T>), dim3((nlines + G - 1) / G), dim3(TOE_FFT_THREADS),
                     toe_fft_launch_lds((pc_circ_fwd_kernel<TI, T>), toe_fft_lds<T>(d.P, G)), s, d, edges, x, N, nb,
                     X);
#define SCABS_PC_APPLY(NBV)                                                                                          \
  hipLaunchKernelGGL((pc_circ_apply_kernel<T, NBV>), dim3((n + 255) / 256, d.P), dim3(256), 0, s, (const cx<T> *)Tinv, \
                     (const cx<T> *)X, Y, n, d.P, trans ? 1 : 0)
  switch (nb) {
    case 1: SCABS_PC_APPLY(1); break;
    case 2: SCABS_PC_APPLY(2); break;
    case 3: SCABS_PC_APPLY(3); break;
    case 4: SCABS_PC_APPLY(4); break;
    case 5: SCABS_PC_APPLY(5); break;
    case 6: SCABS_PC_APPLY(6); break;
    case 7: SCABS_PC_APPLY(7); break;
    default: SCABS_PC_APPLY(8); break;
  }
#undef SCABS_PC_APPLY
  hipLaunchKernelGGL(pc_circ_inv_kernel<T>, dim3((nlines + G - 1) / G), dim3(TOE_FFT_THREADS),
                     toe_fft_launch_lds(pc_circ_inv_kernel<T>, toe_fft_lds<T>(d.P, G)), s, d, edges,
                     (const cx<T> *)Y, N, nb, y);
  hipLaunchKernelGGL(pc_identity_kernel<TI>, dim3((ne + 255) / 256, nb), dim3(256), 0, s, edges, d.edge_sgn, ne, x,
                     N, nb, y);
}
template void launch_pc_circ_apply<double, double>(const ToeDev<double> &, const EdgeRec *, const cx<double> *,
                                                   const cx<double> *, int64_t, int, bool, cx<double> *, cx<double> *,
                                                   cx<double> *, int, hipStream_t);
template void launch_pc_circ_apply<float, float>(const ToeDev<float> &, const EdgeRec *, const cx<float> *,
                                                 const cx<float> *, int64_t, int, bool, cx<float> *, cx<float> *,
                                                 cx<double> *, int, hipStream_t);
template void launch_pc_circ_apply<double, float>(const ToeDev<float> &, const EdgeRec *, const cx<float> *,
                                                  const cx<double> *, int64_t, int, bool, cx<float> *, cx<float> *,
                                                  cx<double> *, int, hipStream_t);
template void launch_pc_circ_apply<float, double>(const ToeDev<double> &, const EdgeRec *, const cx<double> *,
                                                  const cx<float> *, int64_t, int, bool, cx<double> *, cx<double> *,
                                                  cx<double> *, int, hipStream_t);

}  // namespace scabs
