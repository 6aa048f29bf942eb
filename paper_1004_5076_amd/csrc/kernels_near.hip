// Near-pair setup (FP64): for every near (test T, source T') triangle pair the
// tested interactions of their half-RWG functions computed exactly (Galerkin
// with singularity subtraction) minus the same interactions as the grid
// (projection -> sampled kernel -> interpolation) reproduces them.
//
// Exact rule: static part of G integrated analytically over T' (potential
// integrals of a flat triangle, Wilton et al. 1984 / Graglia 1993) plus the
// 7-point rule on the smooth remainder G - 1/(4 pi R), for pairs with centroid
// distance < kappa_s (rho_T + rho_T'); plain 7-point rule on G otherwise.
// Test side: 7-point rule, L tested by parts (div on the test function).
#include <cmath>

#include "device_common.h"
#include "kernels.h"
#include "near_math.h"

namespace scabs {

constexpr int NS_THREADS = 64;
constexpr int MAXBOX = 343;
constexpr int NTYPES = 8;   // L_e, K_e, L_i, K_i, Lrot_e, Krot_e, Lsig_i, Ksig_i

// MODE 0: tested blocks of every near pair (exact - grid, and exact alone).
// MODE 1: pointwise (exact - grid) one-sided fields at the test points of the
//         masked triangles from the currents a.cur, added into a.Ee / a.Ei.
template <int MODE> __global__ void __launch_bounds__(NS_THREADS) near_setup_kernel(NearSetupArgs a) {
  const int T = blockIdx.x;
  const int tid = threadIdx.x;
  if (MODE == 1 && !a.tmask[T]) return;   // uniform over the work-group
  cx<double> fe[3] = {{0, 0}, {0, 0}, {0, 0}}, fi[3] = {{0, 0}, {0, 0}, {0, 0}};
  __shared__ double s_tp[NQ][3], s_tw[NQ], s_tsig[NQ];
  __shared__ double s_tg[NQ][3][3];
  __shared__ double s_tdiv[3], s_n[3];
  __shared__ int s_tanc[NQ][3];
  __shared__ double s_Iw[NQ][27][4];
  __shared__ int s_blo[3], s_bn[3];
  __shared__ double s_sp[NQ][3], s_sw[NQ];
  __shared__ int s_sanc[NQ][3];
  __shared__ double s_Pw[NQ][27];
  __shared__ double s_sv[3][3], s_scoef[3], s_sdiv[3];
  __shared__ cx<double> s_Phi[NQ][MAXBOX];
  __shared__ cx<double> s_D[NQ][NQ][8];   // exact (value, grad), grid (value, grad)
  __shared__ cx<double> s_part[2][NQ][NTYPES * 9];   // [exact - grid, exact]

  // ---- test triangle -------------------------------------------------------
  if (tid < NQ) {
    const int q = tid, ip = T * NQ + q;
    for (int c = 0; c < 3; c++) {
      s_tp[q][c] = a.qp[3 * ip + c];
      s_tanc[q][c] = a.anchor[3 * ip + c];
    }
    s_tw[q] = a.qw[ip];
    s_tsig[q] = a.sigma[ip];
    double L[3][3], dL[3][3];
    for (int c = 0; c < 3; c++) lagr3(a.u[3 * ip + c], L[c], dL[c]);
    const double ih = 1.0 / a.h;
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++)
        for (int k = 0; k < 3; k++) {
          int d = i * 9 + j * 3 + k;
          s_Iw[q][d][0] = L[0][i] * L[1][j] * L[2][k];
          s_Iw[q][d][1] = dL[0][i] * L[1][j] * L[2][k] * ih;
          s_Iw[q][d][2] = L[0][i] * dL[1][j] * L[2][k] * ih;
          s_Iw[q][d][3] = L[0][i] * L[1][j] * dL[2][k] * ih;
        }
    for (int i = 0; i < 3; i++) {
      int e = a.tedge[3 * T + i];
      double cf = a.tsign[3 * T + i] * a.elen[e] / (2.0 * a.area[T]);
      const double *vk = a.v + 3 * a.t[3 * T + i];
      for (int c = 0; c < 3; c++) s_tg[q][i][c] = cf * (s_tp[q][c] - vk[c]);
    }
  }
  if (tid < 3) {
    int e = a.tedge[3 * T + tid];
    s_tdiv[tid] = a.tsign[3 * T + tid] * a.elen[e] / a.area[T];
    s_n[tid] = a.nrm[3 * T + tid];
  }
  __syncthreads();
  if (tid < 3) {
    int lo = s_tanc[0][tid], hi = lo;
    for (int q = 1; q < NQ; q++) {
      lo = min(lo, s_tanc[q][tid]);
      hi = max(hi, s_tanc[q][tid]);
    }
    s_blo[tid] = lo - 1;
    s_bn[tid] = hi - lo + 3;
  }
  __syncthreads();
  const int bn0 = s_bn[0], bn1 = s_bn[1], bn2 = s_bn[2], boxN = bn0 * bn1 * bn2;
  bool tsig_any = false;
  for (int q = 0; q < NQ; q++) tsig_any |= s_tsig[q] != 0.0;
  const D3 nT = {s_n[0], s_n[1], s_n[2]};

  for (int64_t p = a.tptr[T]; p < a.tptr[T + 1]; p++) {
    const int Tp = a.src[p];
    const bool sing = a.sing[p] != 0;
    const bool same = a.body[T] == a.body[Tp];
    // ---- source triangle ----------------------------------------------------
    if (tid < NQ) {
      const int q = tid, ip = Tp * NQ + q;
      for (int c = 0; c < 3; c++) {
        s_sp[q][c] = a.qp[3 * ip + c];
        s_sanc[q][c] = a.anchor[3 * ip + c];
      }
      s_sw[q] = a.qw[ip];
      double L[3][3], dL[3][3];
      for (int c = 0; c < 3; c++) lagr3(a.u[3 * ip + c], L[c], dL[c]);
      for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
          for (int k = 0; k < 3; k++) s_Pw[q][i * 9 + j * 3 + k] = L[0][i] * L[1][j] * L[2][k];
    }
    if (tid < 3) {
      int e = a.tedge[3 * Tp + tid];
      s_scoef[tid] = a.tsign[3 * Tp + tid] * a.elen[e] / (2.0 * a.area[Tp]);
      s_sdiv[tid] = 2.0 * s_scoef[tid];
      for (int c = 0; c < 3; c++) s_sv[tid][c] = a.v[3 * a.t[3 * Tp + tid] + c];
    }
    if (MODE == 0)
      for (int i = tid; i < 2 * NQ * NTYPES * 9; i += NS_THREADS) (&s_part[0][0][0])[i] = cx<double>{0.0, 0.0};
    __syncthreads();

    for (int med = 0; med < (same ? 2 : 1); med++) {
      const double k = med ? a.k_i : a.k_e;
      const cx<double> *tab = med ? a.htab_i : a.htab_e;
      // grid potential of each projected source point on the test box
      for (int it = tid; it < NQ * boxN; it += NS_THREADS) {
        const int s = it / boxN, gb = it - s * boxN;
        const int bx = gb / (bn1 * bn2), by = (gb / bn2) % bn1, bz = gb % bn2;
        const int gx = s_blo[0] + bx, gy = s_blo[1] + by, gz = s_blo[2] + bz;
        cx<double> acc = {0.0, 0.0};
        int d = 0;
        for (int i = -1; i <= 1; i++)
          for (int j = -1; j <= 1; j++)
            for (int kk = -1; kk <= 1; kk++, d++) {
              int dx = abs(gx - s_sanc[s][0] - i), dy = abs(gy - s_sanc[s][1] - j), dz = abs(gz - s_sanc[s][2] - kk);
              if (dx | dy | dz) axpy(acc, s_Pw[s][d], tab[((size_t)dx * (a.D + 1) + dy) * (a.D + 1) + dz]);
            }
        s_Phi[s][gb] = acc;
      }
      __syncthreads();
      // per (test, source) point pair: w_s (exact kernel - grid kernel), value and gradient
      if (tid < NQ * NQ) {
        const int t = tid / NQ, s = tid - t * NQ;
        cx<double> Hv = {0, 0}, Hg[3] = {{0, 0}, {0, 0}, {0, 0}};
        int d = 0;
        for (int i = -1; i <= 1; i++)
          for (int j = -1; j <= 1; j++)
            for (int kk = -1; kk <= 1; kk++, d++) {
              int bx = s_tanc[t][0] + i - s_blo[0], by = s_tanc[t][1] + j - s_blo[1], bz = s_tanc[t][2] + kk - s_blo[2];
              cx<double> ph = s_Phi[s][(bx * bn1 + by) * bn2 + bz];
              axpy(Hv, s_Iw[t][d][0], ph);
              axpy(Hg[0], s_Iw[t][d][1], ph);
              axpy(Hg[1], s_Iw[t][d][2], ph);
              axpy(Hg[2], s_Iw[t][d][3], ph);
            }
        D3 dv = d3(s_tp[t]) - d3(s_sp[s]);
        double R = sqrt(dotd(dv, dv));
        cx<double> G = {0, 0}, dG = {0, 0};
        if (R > 0 || sing) kernel_val(k, R, sing, G, dG);
        cx<double> gr[3] = {{0, 0}, {0, 0}, {0, 0}};
        if (R > 1e-14) {
          gr[0] = dG * (dv.x / R);
          gr[1] = dG * (dv.y / R);
          gr[2] = dG * (dv.z / R);
        }
        const double ws = s_sw[s];
        s_D[t][s][0] = G * ws;
        s_D[t][s][4] = Hv * ws;
        for (int c = 0; c < 3; c++) {
          s_D[t][s][1 + c] = gr[c] * ws;
          s_D[t][s][5 + c] = Hg[c] * ws;
        }
      }
      __syncthreads();
      // per test point: inner integrals, then its share of the tested blocks,
      // once for exact - grid (variant 0) and once for exact alone (variant 1)
      if (tid < (MODE == 0 ? 2 : 1) * NQ) {
        const int t = tid % NQ, var = tid / NQ;
        const D3 r = d3(s_tp[t]);
        cx<double> S0 = {0, 0};
        Z3 S1 = {{0, 0}, {0, 0}, {0, 0}}, Sg = S1, Sc[3] = {S1, S1, S1};
        for (int s = 0; s < NQ; s++) {
          const D3 sp = d3(s_sp[s]);
          cx<double> g0 = s_D[t][s][0];
          Z3 gv = {s_D[t][s][1], s_D[t][s][2], s_D[t][s][3]};
          if (var == 0) {
            g0 -= s_D[t][s][4];
            gv.x -= s_D[t][s][5];
            gv.y -= s_D[t][s][6];
            gv.z -= s_D[t][s][7];
          }
          S0 += g0;
          S1 = zadd(S1, zscale(g0, sp - r));
          Sg = zadd(Sg, gv);
          for (int j = 0; j < 3; j++) Sc[j] = zadd(Sc[j], zcross(gv, sp - d3(s_sv[j])));
        }
        if (sing) {
          double J0;
          D3 J1, Jg;
          tri_potentials(r, d3(a.v + 3 * a.t[3 * Tp]), d3(a.v + 3 * a.t[3 * Tp + 1]), d3(a.v + 3 * a.t[3 * Tp + 2]), J0,
                         J1, Jg);
          const double c4 = 1.0 / (4.0 * PI);
          S0.x += c4 * J0;
          S1.x.x += c4 * J1.x;
          S1.y.x += c4 * J1.y;
          S1.z.x += c4 * J1.z;
          Sg.x.x += c4 * Jg.x;
          Sg.y.x += c4 * Jg.y;
          Sg.z.x += c4 * Jg.z;
          for (int j = 0; j < 3; j++) {
            D3 cr = crossd(Jg, r - d3(s_sv[j]));
            Sc[j].x.x += c4 * cr.x;
            Sc[j].y.x += c4 * cr.y;
            Sc[j].z.x += c4 * cr.z;
          }
        }
        cx<double> *part = s_part[var][t];
        const double w = s_tw[t], sg = s_tsig[t], ik2 = 1.0 / (k * k);
        const double Zm = med ? a.Z_i : a.Z_e;
        for (int j = 0; j < 3; j++) {
          const D3 rv = r - d3(s_sv[j]);
          // a_j = coef_j (S1 + (r - v_j) S0); phi_j = div_j S0; grad phi_j = div_j Sg; c_j = coef_j Sc_j
          Z3 aj = zadd(S1, zscale(S0, rv));
          aj = {aj.x * s_scoef[j], aj.y * s_scoef[j], aj.z * s_scoef[j]};
          const cx<double> phj = S0 * s_sdiv[j];
          const Z3 gpj = {Sg.x * s_sdiv[j], Sg.y * s_sdiv[j], Sg.z * s_sdiv[j]};
          const Z3 cj = {Sc[j].x * s_scoef[j], Sc[j].y * s_scoef[j], Sc[j].z * s_scoef[j]};
          // pointwise L(f_j) = jk (a_j + k^-2 grad phi_j), K(f_j) = -c_j
          Z3 Lv;
          Lv.x = mul_j(aj.x + gpj.x * ik2) * k;
          Lv.y = mul_j(aj.y + gpj.y * ik2) * k;
          Lv.z = mul_j(aj.z + gpj.z * ik2) * k;
          const Z3 Kv = {-cj.x, -cj.y, -cj.z};
          if (MODE == 1) {
            // E_e += -Z_e L(f_j) J_e + K(f_j) M ;  E_i += -Z_i L(f_j) J_i - K(f_j) M  (M_i = -M)
            const int m = a.tedge[3 * Tp + j];
            const cx<double> J = a.cur[3 * m + (med ? 1 : 0)], M = a.cur[3 * m + 2];
            cx<double> *f = med ? fi : fe;
            const double sm = med ? -1.0 : 1.0;
            f[0] += (Lv.x * J) * (-Zm) + (Kv.x * M) * sm;
            f[1] += (Lv.y * J) * (-Zm) + (Kv.y * M) * sm;
            f[2] += (Lv.z * J) * (-Zm) + (Kv.z * M) * sm;
            continue;
          }
          for (int i = 0; i < 3; i++) {
            const D3 gi = d3(s_tg[t][i]);
            cx<double> tl = zdot(gi, aj);
            axpy(tl, -s_tdiv[i] * ik2, phj);
            const int ij = i * 3 + j;
            part[(med ? 2 : 0) * 9 + ij] = mul_j(tl) * (k * w);
            part[(med ? 3 : 1) * 9 + ij] = zdot(gi, Kv) * w;
            if (sg != 0.0) {
              if (med == 0) {
                const D3 gxn = crossd(gi, nT);
                part[4 * 9 + ij] = zdot(gxn, Lv) * (w * sg);
                part[5 * 9 + ij] = zdot(gxn, Kv) * (w * sg);
              } else {
                part[6 * 9 + ij] = zdot(gi, Lv) * (w * sg);
                part[7 * 9 + ij] = zdot(gi, Kv) * (w * sg);
              }
            }
          }
        }
      }
      __syncthreads();
    }
    if (MODE == 0)
      for (int e = tid; e < 2 * NTYPES * 9; e += NS_THREADS) {
        const int var = e / (NTYPES * 9), ee = e - var * NTYPES * 9;
        cx<double> s = {0, 0};
        for (int t = 0; t < NQ; t++) s += s_part[var][t][ee];
        (var ? a.blocks_exact : a.blocks)[(size_t)p * NTYPES * 9 + ee] = s;
      }
    __syncthreads();
  }
  if (MODE == 1 && tid < NQ) {
    const size_t ip = (size_t)T * NQ + tid;
    for (int c = 0; c < 3; c++) {
      a.Ee[3 * ip + c] += fe[c];
      a.Ei[3 * ip + c] += fi[c];
    }
  }
  (void)tsig_any;
}

void launch_near_setup(const NearSetupArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(near_setup_kernel<0>, dim3(a.nt), dim3(NS_THREADS), 0, s, a);
}
void launch_near_point_fields(const NearSetupArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(near_setup_kernel<1>, dim3(a.nt), dim3(NS_THREADS), 0, s, a);
}

__global__ void htab_kernel(double k, double h, int D, cx<double> *tab) {
  int n = (D + 1) * (D + 1) * (D + 1);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    int dz = i % (D + 1), dy = (i / (D + 1)) % (D + 1), dx = i / ((D + 1) * (D + 1));
    cx<double> v = {0.0, 0.0};
    if (dx | dy | dz) {
      double R = h * sqrt((double)dx * dx + (double)dy * dy + (double)dz * dz);
      double sn, cs;
      sincos(k * R, &sn, &cs);
      double sc = 1.0 / (4.0 * PI * R);
      v = {cs * sc, -sn * sc};
    }
    tab[i] = v;
  }
}
void build_htab(double k, double h, int D, cx<double> *tab, hipStream_t s) {
  hipLaunchKernelGGL(htab_kernel, dim3(64), dim3(256), 0, s, k, h, D, tab);
}

__global__ void near_assemble_kernel(int64_t nnz, const int64_t *__restrict__ cptr, const int *__restrict__ cpair,
                                     const uint8_t *__restrict__ cij, const cx<double> *__restrict__ blocks,
                                     cx<double> *V4, cx<double> *S4, cx<float> *V4f, cx<float> *S4f) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
    cx<double> acc[NTYPES];
    for (int t = 0; t < NTYPES; t++) acc[t] = {0.0, 0.0};
    for (int64_t c = cptr[e]; c < cptr[e + 1]; c++) {
      const cx<double> *b = blocks + (size_t)cpair[c] * NTYPES * 9 + cij[c];
      for (int t = 0; t < NTYPES; t++) acc[t] += b[t * 9];
    }
    for (int t = 0; t < 4; t++) {
      V4[4 * e + t] = acc[t];
      S4[4 * e + t] = acc[4 + t];
      V4f[4 * e + t] = {(float)acc[t].x, (float)acc[t].y};
      S4f[4 * e + t] = {(float)acc[4 + t].x, (float)acc[4 + t].y};
    }
  }
}
void launch_near_assemble(int64_t nnz, const int64_t *cptr, const int *cpair, const uint8_t *cij,
                          const cx<double> *blocks, cx<double> *V4, cx<double> *S4, cx<float> *V4f, cx<float> *S4f,
                          hipStream_t s) {
  hipLaunchKernelGGL(near_assemble_kernel, dim3(2048), dim3(256), 0, s, nnz, cptr, cpair, cij, blocks, V4, S4, V4f, S4f);
}

}  // namespace scabs
