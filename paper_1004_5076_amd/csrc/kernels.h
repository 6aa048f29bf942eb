// Launch interfaces of the HIP kernels.
#pragma once
#include <vector>

#include "internal.h"

namespace scabs {

// One lattice box on the device, in precision T.  Potential/source fields are
// stored [field][x][y][z] (z fastest), 8 fields:
// J_x, J_y, J_z, div J, M_x, M_y, M_z, div M (each weighted by w_q).
template <typename T> struct DevGrid {
  int which;
  int n[3], N[3];
  int off[3];        // origin minus the exterior grid's origin (lattice units)
  int twL;
  T k, Z;
  cx<T> *phys;       // 8 * n0 n1 n2
  cx<T> *spec;       // 8 * n0 N1 N2 (y-z transformed planes)
  const cx<T> *ghat; // (N0/2+1)(N1/2+1)(N2/2+1): FFT of the embedded kernel / (N0 N1 N2)
  const cx<T> *tw;   // exp(-2 pi i j / twL), j < twL
  // x lines of length 1024 only (else null): exp(-2 pi i a l / 1024) at
  // [a * 64 + l] (a < 16, l < 64), then exp(-2 pi i p c / 64) at [1024 + c * 4 + p]
  const cx<T> *twx;
  // with twx: the kernel spectrum octant again, x fastest:
  // [(k_y' (N2/2+1) + k_z') (N0/2+1) + k_x'] (null otherwise)
  const cx<T> *ghx;
};

// Per-grid point lists for the gather projection: the grid's points sorted by
// anchor cell (x, y, z), cell ranges, and per sorted point its offset from
// the anchor (grid units).
template <typename T> struct GatherGrid {
  int np;                  // points in this grid
  int64_t ncell;           // n0 n1 n2
  const int *perm;         // sorted index -> point id
  const int64_t *cellptr;  // ncell + 1
  const T *u;              // 3 per sorted point
  cx<T> *src;              // 8 per sorted point (written each product)
  const int *nz_ptr;       // n0 + 1: cells holding points, listed plane by plane
  const int *nz_yz;        // their (y, z) index y n2 + z within the plane
};
// coefficients per point of the transposed testing (lattice sources of test^T):
// 8 value coefficients, then the three vectors whose curls and gradient enter
constexpr int ADJ_COEF = 17;

template <typename T> struct DevOperator {
  int np, nt, ne, N;
  T k_e, Z_e, k_i, Z_i;
  const PointRec<T> *pts;
  const TriRec<T> *tris;
  const EdgeRec *edges;
  // near correction CSR (edge rows)
  const int64_t *rowptr;
  const int *col;
  const cx<T> *V4;   // per entry: L_e, K_e, L_i, K_i   (exact - grid)
  const cx<T> *S4;   // per entry: Lrot_e, Krot_e, Lsig_i, Ksig_i (R rows only)
  // the same values at the mirrored entry: V4T[4 k + j] = V4[4 tpos[k] + j]
  // (row-ordered reads for the transposed product; null: read through tpos)
  const cx<T> *V4T, *S4T;
  // work buffers
  cx<T> *src;        // ne * 3: J_e, J_i, M
  // batches of nb > 1 vectors: the same currents per edge for all vectors,
  // [e][b][3] (written by the unpack step; null until a batch is used)
  cx<T> *srcI;
  cx<T> *tri_out;    // nt * 3 (half-edge) * 3 (E, H, eq14 rows)
  // block-Toeplitz product: per vector and edge the (E, H) row sums of the
  // periodic part, added by the row kernel ([v][e][2]; null: none)
  const cx<T> *edge_out;
};

// ---- FFT convolution -------------------------------------------------------
// nb vectors: phys/spec hold nb consecutive 8-field blocks
constexpr int XLINE_REG_LEN = 1024;   // x length with the wave-per-line register transform
// parts of the convolution (bit flags): forward y-z transforms, x lines with
// the kernel product, inverse y-z transforms
enum ConvPart { CONV_PLANES_FWD = 1, CONV_XLINES = 2, CONV_PLANES_INV = 4, CONV_ALL = 7 };
template <typename T> void launch_conv(const DevGrid<T> &g, hipStream_t s, int nb = 1, int parts = CONV_ALL);
// ghx[(y h2 + z) h0 + x] = ghat[(x h1 + y) h2 + z]
template <typename T> void launch_ghat_xfast(const cx<T> *ghat, cx<T> *ghx, int h0, int h1, int h2, hipStream_t s);
// FFT of the circulant-embedded grid kernel; writes the scaled octant in both precisions
hipError_t build_ghat(const GridDesc &d, double h, const cx<double> *tw64, int twL, cx<double> *ghat64,
                      cx<float> *ghat32, hipStream_t s);

// ---- matvec steps ------------------------------------------------------------
// lattice gathers (projection and transposed testing): phase-B layout with one
// node per lane triple (its three x offsets), 21 nodes (63 lanes) per wave
constexpr int GB_NODES_PER_WAVE = 21;
// Batched steps: nb vectors at once; every per-vector buffer (x, y, op.src,
// op.tri_out, gather sources, grid fields) holds nb consecutive copies.
template <typename T> void launch_unpack(const DevOperator<T> &op, const double *x, hipStream_t s, int nb = 1);
// part < 0: point sources and gathers of every grid; part = k: grid k's gather only
template <typename T>
void launch_project(const DevOperator<T> &op, const std::vector<DevGrid<T>> &grids,
                    const std::vector<GatherGrid<T>> &gg, hipStream_t s, int nb = 1, int part = -1);
template <typename T>
void launch_interp_test(const DevOperator<T> &op, const DevGrid<T> &ext, const DevGrid<T> *ints_dev, T inv_h,
                        hipStream_t s, int nb = 1);
// nb <= near_rows_max_batch()
template <typename T> void launch_near_rows(const DevOperator<T> &op, double *y, hipStream_t s, int nb = 1);
int near_rows_max_batch();

// ---- setup (FP64) ------------------------------------------------------------
struct NearSetupArgs {
  int nt;
  double h, k_e, k_i;
  const double *v;           // vertices
  const int *t;              // triangles
  const int *body;
  const int *tedge;
  const int *tsign;
  const double *elen, *area, *nrm;
  const double *qp, *qw, *sigma;
  const int *anchor;         // absolute lattice anchors, np*3
  const double *u;           // np*3
  const int64_t *tptr;
  const int *src;
  const uint8_t *sing;
  int D;                     // kernel table extent
  const cx<double> *htab_e, *htab_i;   // (D+1)^3 each
  cx<double> *blocks;        // npairs * 8 * 9: exact - grid
  cx<double> *blocks_exact;  // npairs * 8 * 9: exact
  // pointwise-field mode
  double Z_e, Z_i;
  const uint8_t *tmask;      // triangles whose test points are needed
  const cx<double> *cur;     // per edge: J_e, J_i, M
  cx<double> *Ee, *Ei;       // np * 3 each (added into)
};
void launch_near_setup(const NearSetupArgs &a, hipStream_t s);
// (exact - grid) near-pair part of the one-sided pointwise fields, added
void launch_near_point_fields(const NearSetupArgs &a, hipStream_t s);
void build_htab(double k, double h, int D, cx<double> *tab, hipStream_t s);
void launch_near_assemble(int64_t nnz, const int64_t *cptr, const int *cpair, const uint8_t *cij,
                          const cx<double> *blocks, cx<double> *V4, cx<double> *S4, cx<float> *V4f, cx<float> *S4f,
                          hipStream_t s);

// ---- preconditioner (restricted additive Schwarz on the exact near field) -----
struct PrecondArgs {
  int nc;
  double Ze, Zi;
  const int64_t *rowptr;
  const int *col;
  const cx<double> *X8;      // exact near values per CSR entry (8 operator types)
  const int64_t *lptr;       // local-term CSR
  const int *lcol;
  const double *lval;
  const int *slot_edge;      // unknown slot -> edge
  const int8_t *slot_kind;   // 0: J / J_e / E row, 1: M / H row, 2: J_i / eq14 row
  const int *isR;            // per edge
  const int64_t *ext_ptr;
  const int *ext_slot;
  const int64_t *a_off;
  int64_t n_ext;             // ext entries of all clusters
  cx<float> *A;              // dense cluster blocks (FP32)
};
void launch_exact_assemble(int64_t nnz, const int64_t *cptr, const int *cpair, const uint8_t *cij,
                           const cx<double> *blocks, cx<double> *X8, hipStream_t s);
// Stored Schwarz rows: per cluster the core rows x ext columns of the block
// inverse in 8-column row-major blocks (rt_index), each complex entry as two
// FP16 halves (real in the low 16 bits) divided by its column's scale (the
// largest |re|, |im| of the column, FP32, one per ext entry).
struct PcStore {
  const uint32_t *R;
  const float *scale;
};
// blocked Gauss-Jordan: per panel the prefix sums over clusters of their
// update tiles (npanels x (nclusters + 1)), and the pivot-row scratch size
std::vector<int> gj_tile_table(const std::vector<int64_t> &ext_ptr, int &npanels);
size_t gj_scratch_entries(const std::vector<int64_t> &ext_ptr);
void launch_precond_build(const PrecondArgs &p, const std::vector<int64_t> &ext_ptr_h, const int *tiles_dev,
                          const std::vector<int> &tiles_h, int npanels, cx<float> *gj_tmp, const int64_t *core_ptr,
                          const int *core_pos, const int64_t *r_off, uint32_t *Rt, float *Rs, int *piv, int *status,
                          hipStream_t s);
// rows of one cluster's core handled by one work-group of the apply kernel
int precond_rows_per_item();
// items: n_items pairs (cluster, first core row), rows per item as above
void launch_precond_apply(int n_items, const int *items, const int64_t *ext_ptr, const int *ext_slot,
                          const int64_t *core_ptr, const int *core_slot, const int64_t *r_off, PcStore pc,
                          const cx<double> *x, cx<double> *y, int max_ext, hipStream_t s);

// FP32 batched apply (inner solves of the mixed mode): m vectors of N,
// m <= precond_apply32_max_batch().  First the inputs are gathered into an
// ext-ordered copy xe[e m + b] = scale_e x_b[ext_slot_e] (FP32, n_ext m
// entries), then every work-group reads its cluster's part of xe.  items:
// (cluster, first core row) pairs in dispatch order (work-group i runs entry
// i; cluster -1 marks an empty entry).
int precond_apply32_max_batch();
template <typename TI>   // double or float inputs
void launch_precond_gather32(int64_t n_ext, const int *ext_slot, const float *scale, const cx<TI> *x, int64_t N,
                             int m, cx<float> *xe, hipStream_t s);
void launch_precond_apply32(int n_items, const int *items, const int64_t *ext_ptr, const int64_t *core_ptr,
                            const int *core_slot, const int64_t *r_off, const uint32_t *R, const cx<float> *xe,
                            cx<double> *y, int64_t N, int m, hipStream_t s);

// ---- transposed product, adjoint gradient --------------------------------------
template <typename T> void launch_unpack_rows(const DevOperator<T> &op, const double *z, hipStream_t s);
// dst[4 k + j] = src[4 tpos[k] + j] for k < nnz (mirrored-entry copy)
void launch_mirror4(int64_t nnz, const int64_t *tpos, const cx<float> *src, cx<float> *dst, hipStream_t s);
// src4[k]: ADJ_COEF coefficients per sorted point of grid k (work buffer)
template <typename T>
void launch_test_t(const DevOperator<T> &op, const std::vector<DevGrid<T>> &grids, const std::vector<GatherGrid<T>> &gg,
                   const std::vector<cx<T> *> &src4, T inv_h, hipStream_t s);
template <typename T>
void launch_interp_adj(const DevOperator<T> &op, const DevGrid<T> &ext, const DevGrid<T> *ints_dev, hipStream_t s);
template <typename T>
void launch_near_rows_t(const DevOperator<T> &op, const int64_t *tpos, double *y, hipStream_t s);
// items: (cluster, first ext column) per work-group, precond_t_cols_per_item() columns each, in
// dispatch order (work-group i runs entry i; cluster -1 marks an empty entry)
int precond_t_cols_per_item();
template <typename TI>   // double or float inputs x
void launch_precond_apply_t(int n_items, const int *items, int64_t N, int64_t n_core, const int64_t *ext_ptr,
                            const int64_t *core_ptr, const int *core_slot, const int64_t *r_off, PcStore pc,
                            const int64_t *inv_ptr, const int64_t *inv_pos, cx<double> *tmp, cx<double> *xc,
                            const cx<TI> *x, cx<double> *y, hipStream_t s);
void launch_point_fields(const DevOperator<double> &op, const DevGrid<double> &ext, const DevGrid<double> *ints_dev,
                         double inv_h, cx<double> *Ee, cx<double> *Ei, hipStream_t s);
void launch_sigma_grad(const DevOperator<double> &op, const cx<double> *Ee, const cx<double> *Ei,
                       const cx<double> *Einc, double *dfds, hipStream_t s);
// fields at points near or on either side of the surface: per triangle the
// static part analytic within SCABS_NEAR_FIELD_RADIUS triangle radii
// one-sided fields of the discrete Galerkin operator at the quadrature points
// of the listed triangles, by direct summation (overwrites those points)
void launch_point_fields_exact(const DevOperator<double> &op, const TriD *tri, const int *list, int nlist,
                               double k_e, double Z_e, double k_i, double Z_i, double kappa, cx<double> *Ee,
                               cx<double> *Ei, hipStream_t s);
void launch_eval_field_exact(const DevOperator<double> &op, const TriD *tri, const double *pts, int npts, int region,
                             double k, double Z, cx<double> *E, cx<double> *H, hipStream_t s);
// an incident source in the interior medium: a point dipole (b = 0) at r0 or
// the complex-source-point beam at r0 - j b dir (bd = b dir); moment p
struct SourceDev {
  double r0[3], bd[3], b;
  cx<double> p[3];
};
void launch_dipole_points(int npts, const double *pts, double k, double Z, const SourceDev &S, cx<double> *E,
                          cx<double> *H, hipStream_t s);
void launch_incident_points(int np, const int *body, const PointRec<double> *pts, const double *qp, double k, double Z,
                            const SourceDev &S, int bodyid, cx<double> *E, hipStream_t s);

// fields at off-surface points (currents from op.src) and the transpose of
// their E part (adjoint currents collected into y, unknown space)
void launch_eval_field(const DevOperator<double> &op, const double *qp, const double *pts, int npts, int region,
                       double k, double Z, cx<double> *E, cx<double> *H, hipStream_t s);
void launch_eval_field_t(const DevOperator<double> &op, const double *qp, const double *pts, int npts, int region,
                         double k, double Z, const cx<double> *wE, double *y, hipStream_t s);

// ---- block-Toeplitz product (periodic guides) ----------------------------------
struct ToeSetupArgs {
  int nr, P, ne_r, nt_r, nbody;
  double dx, k_e, k_i, Z_e, Z_i, kappa;
  const TriD *tri;                 // nt_r template triangles (ring 0)
  const int *e_tri, *e_k, *e_off;  // ne_r * 2
  const int *ebody;                // ne_r
  const int *body_e0, *body_t0;    // nbody + 1
  const int64_t *ibase, *pbase;    // nbody + 1: interior Galerkin / interior point series offsets
  cx<double> *sLe, *sKe, *sLi, *sKi, *sPeJ, *sPeM, *sPiJ, *sPiM;   // spatial series, P each
};
struct ToeCapArgs {
  int64_t nnz;
  const int *row, *col;            // per entry: row edge, column edge
  const int *et, *tedge;
  const TriD *tri;                 // every triangle of the mesh
  const double *sigma;             // per quadrature point
  double k_e, k_i, kappa;
  cx<double> *V4, *S4;
  cx<float> *V4f, *S4f;
};
template <typename T> struct ToeDev {
  int nr, P, ne_r, nt_r;
  T Z_e, Z_i;
  const int *ringmap, *pmap, *edge_sgn, *tri_loc, *tri_ring, *ebody, *tbody, *body_e0, *body_t0;
  const int64_t *ibase, *pbase;
  int64_t gi_per_f, pi_per_f;
  const cx<T> *GE, *GI, *PE, *PI;  // per-frequency pair tables (see kernels_toeplitz.hip)
  const cx<T> *tw;                 // exp(-2 pi i j / P), j < P
  const T *t1, *t2;                // per local triangle: in-plane basis of its point fields
  cx<T> *X, *Y;                    // spectra of a product
  cx<T> *edge_out;                 // [v][e][2]
  cx<T> *pf;                       // [v][point row r < 2 R2][ring]: exterior rows r < R2, interior after
  int lines;                       // ring-axis lines per transform work-group (<= toe_max_lines)
  int apply_form;                  // 8 FP32 vectors: 0 matrix cores, 1 vector ALUs
};

// block-Toeplitz contexts: tangential fields at points of periodic absorber
// triangles from the product's point lines (pf of the last FP64 product of
// x) plus the non-periodic edges' halves summed directly and the residue
void launch_toe_point_fields(const DevOperator<double> &op, const ToeDev<double> &d, const TriD *tri, const int *list,
                             int nlist, const int *np_tri, const int *np_mask, int nnp, double k_e, double Z_e,
                             double k_i, double Z_i, double kappa, cx<double> *Ee, cx<double> *Ei, hipStream_t s);
// exact entries of the pairs with a non-periodic edge, column-major: short
// part V4S/S4S[(j ne + n) 4 + t] (row n, non-periodic column capcol[j]),
// long part V4L/S4L[(m nlong + i) 4 + t] (non-periodic row capcol[i],
// column m); 4 sigma-free values (L_e, K_e, L_i, K_i) and 4 sigma values
// (Lrot_e, Krot_e, Lsig_i, Ksig_i) per entry
template <typename T> struct ToeRows {
  int ncap, nlong, nchunk;
  const int *capcol;      // the non-periodic edges
  const int *edge_sgn;    // per edge: 0 for non-periodic edges
  const unsigned char *eflag;   // per edge: bit 0 periodic, bit 1 absorber (R) edge
  const cx<T> *V4S, *S4S, *V4L, *S4L;
  T *part;                // [chunk][row][vector][6] partial sums of the long rows
  T *rpart;               // [group][vector][6][edge] partial sums of the periodic rows
  int groups;             // column groups of the periodic rows (<= toe_row_groups())
  int sparse_form;        // 8 FP32 vectors: 0 matrix cores, 1 vector ALUs
};
// coefficients of (J_i, J_e, M) in the E, H and eq14 rows from one entry's
// 8 tested values (sigma values on absorber rows only)
template <typename T> struct RowCoef {
  cx<T> eJi, eJe, eM, hJi, hJe, hM, rJi, rM;
};
template <typename T>
__device__ inline RowCoef<T> row_coef(const cx<T> *V4, const cx<T> *S4, bool isR, T Ze, T Zi) {
  RowCoef<T> c;
  const cx<T> Le = V4[0], Ke = V4[1], Li = V4[2], Ki = V4[3];
  c.eJi = Li * Zi;
  c.eJe = Le * (-Ze);
  c.eM = Ke + Ki;
  c.hJi = Ki;
  c.hJe = -Ke;
  c.hM = Le * (T(-1) / Ze) - Li * (T(1) / Zi);
  c.rJi = czero<T>();
  c.rM = czero<T>();
  if (isR) {
    const cx<T> Lr = S4[0], Kr = S4[1], Ls = S4[2], Ks = S4[3];
    c.hJe = c.hJe - Lr * Ze;
    c.hM = c.hM + Kr;
    c.rJi = Ls * Zi;
    c.rM = Ks;
  }
  return c;
}
// transposed block-Toeplitz product of nb <= 8 vectors (rows z unpacked
// into op.src, one slice of 3 ne per vector): circulant columns
// tcol[v][e][4], long-part columns lcol[v][e][3], short-part partial columns
// scol[v][j][TOE_T_SHORT_SPLIT][3] (capidx: edge -> non-periodic index or -1)
constexpr int TOE_T_SHORT_SPLIT = 16;
int toe_t_max_lines(int P, bool fp32);   // transform lines per work-group of the transposed product
// Work-groups are dispatched round-robin over the chip's 8 XCDs, each with
// its own L2.  A launch of gridDim.x work-groups per frequency over
// gridDim.y = P frequencies takes its (part, frequency) so that the parts of
// one frequency run on one XCD, one after another: that XCD's L2 then serves
// the frequency's spectra to all of them.  A permutation of the grid (the
// identity when P is not a multiple of 8).
__device__ inline void toe_xcd_order(int &part, int &f) {
  const int gx = gridDim.x, P = gridDim.y;
  if ((P & 7) != 0) {
    part = blockIdx.x;
    f = blockIdx.y;
    return;
  }
  const int L = blockIdx.y * gx + blockIdx.x, k = L >> 3, q = k / gx;
  f = q * 8 + (L & 7);
  part = k - q * gx;
}
// parts of the product, launched separately so that the sparse parts can run
// on a second stream beside the transforms: ring-axis forward transforms
// (with the transposed product's local terms), per-frequency block products,
// inverse transforms (with the forward product's local and sigma terms), the
// stored entries' short part (periodic rows x non-periodic columns) and long
// part (non-periodic rows x every column), and the final sums into y
enum ToePart { TOE_FWD = 1, TOE_APPLY = 2, TOE_INV = 4, TOE_SHORT = 8, TOE_LONG = 16, TOE_SUM = 32, TOE_ALL = 63 };
template <typename T>
void launch_toe_product_t(const DevOperator<T> &op, const ToeDev<T> &d, const ToeRows<T> &R, cx<T> *tcol,
                          cx<T> *lcol, cx<T> *scol, const int *capidx, double *y, hipStream_t s, int parts, int nb);
// the forward product's stored entries: parts TOE_SHORT, TOE_LONG, TOE_SUM
template <typename T>
void launch_toe_rows(const DevOperator<T> &op, const ToeRows<T> &R, double *y, hipStream_t s, int nb,
                     int parts = TOE_ALL);
int toe_long_chunk();
int toe_row_groups();   // the largest number of column groups
int toe_max_lines(int P, bool fp32);   // the largest transform line group for circulant length P
// circulant preconditioner of A_LL: symbol S and its inverse B (workspaces of
// P (2 ne_r)^2), inverse tables T64/T32[f][j][i]; apply to nb vectors x
// (rows of L periodic edges written to y, non-periodic L rows copied)
void launch_pc_circ_setup(const ToeDev<double> &d, cx<double> *S, cx<double> *B, cx<double> *T64, cx<float> *T32,
                          hipStream_t s);
int pc_circ_max_order();
template <typename TI, typename T>
void launch_pc_circ_apply(const ToeDev<T> &d, const EdgeRec *edges, const cx<T> *Tinv, const cx<TI> *x, int64_t N,
                          int nb, bool trans, cx<T> *X, cx<T> *Y, cx<double> *y, int ne, hipStream_t s);
void launch_toe_setup(const ToeSetupArgs &s, hipStream_t st);
void launch_toe_cap_entries(const ToeCapArgs &c, hipStream_t st);
void launch_toe_series_fft(cx<double> *data, int64_t nlines, int P, const cx<double> *tw, hipStream_t s);
void launch_toe_layout(const ToeSetupArgs &s, int kind, const cx<double> *X, const cx<double> *Y, int64_t per_f,
                       cx<double> *dst64, cx<float> *dst32, hipStream_t st);
template <typename T>
void launch_toe_product(const DevOperator<T> &op, const ToeDev<T> &d, hipStream_t s, int nb, int parts = TOE_ALL);

// ---- misc --------------------------------------------------------------------
void launch_rhs_dipole(int nt, const double *qp, const int *body, const TriRec<double> *tris,
                       const PointRec<double> *pts, const EdgeRec *edges, double k, double Z, const SourceDev &S,
                       int bodyid, double *b, hipStream_t s);

}  // namespace scabs
