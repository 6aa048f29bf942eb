// Internal data layouts of the scabs library (host and device).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <complex>
#include <vector>

#include "../../include/scabs.h"

namespace scabs {

constexpr int NQ = 7;           // quadrature points per triangle (degree-5 rule)
constexpr double PI = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// host-side geometry and layout (setup.cpp)
// ---------------------------------------------------------------------------
struct Geometry {
  int nv = 0, nt = 0, ne = 0, nbody = 0;
  std::vector<double> v;          // nv*3
  std::vector<int> t, body;       // nt*3, nt
  std::vector<double> area, nrm, cen, rho;   // per triangle
  std::vector<double> qp, qw;     // nt*NQ*3, nt*NQ
  std::vector<int> tedge, tsign;  // nt*3: edge opposite local vertex k; +1 on T+
  std::vector<int> ev, et;        // ne*2 (sorted vertex pair; T+ < T-)
  std::vector<double> elen;
};

struct SigmaEnd {
  int axis, dir, degree;
  double x0, length, sigma0;
  std::vector<double> ctrl;       // piecewise-linear control values (empty: monomial)
  std::vector<double> pts;        // raw values per quadrature point (non-empty: neither profile)
};

struct Layout {
  int NL = 0, NR = 0, N = 0;
  std::vector<int> isR, eidx;     // per edge
  std::vector<double> sigma;      // per quadrature point
};

// One lattice box: nodes h*(o + i), i in [0, n); FFT sizes N >= 2n - 1.
struct GridDesc {
  int which;                      // -1 exterior (all bodies), b >= 0 interior of body b
  int o[3], n[3], N[3];
  double k;
};

struct NearList {
  std::vector<int64_t> tptr;      // nt+1: pairs of test triangle T
  std::vector<int> src;           // source triangle of each pair
  std::vector<uint8_t> sing;      // singular-subtraction flag per pair
  // edge-pair CSR of the correction
  std::vector<int64_t> rowptr;    // ne+1
  std::vector<int> col;           // nnz
  std::vector<int64_t> cptr;      // nnz+1: contributions (pair, i, j) of each entry
  std::vector<int> cpair;         // pair index
  std::vector<uint8_t> cij;       // i*3 + j
};

// Column stride of a cluster's stored core rows: a multiple of 16 FP32
// complex values (128 bytes), so every column segment starts on a cache line.
__host__ __device__ inline int64_t rt_stride(int64_t nc) { return (nc + 15) / 16 * 16; }
// Stored Schwarz rows of a cluster (nc core rows, ne ext columns): the columns
// in blocks of RT_CB, each block row-major (RT_CB consecutive entries per core
// row), rows padded to ncp = rt_stride(nc), columns to rt_cols(ne) (padding
// zero); entry (i, j) at rt_index(i, j, ncp).  A wave reading RT_CB columns of
// 64 rows reads one contiguous 2 KB run.
constexpr int RT_CB = 8;
__host__ __device__ inline int64_t rt_cols(int64_t ne) { return (ne + RT_CB - 1) / RT_CB * RT_CB; }
__host__ __device__ inline int64_t rt_index(int64_t i, int64_t j, int64_t ncp) {
  return (j / RT_CB) * (ncp * RT_CB) + i * RT_CB + (j % RT_CB);
}

// Overlapping box clusters of edges (restricted additive Schwarz on the
// near-field matrix): core = edges whose midpoint lies in a cubic cell,
// ext = edges whose midpoint lies in the cell grown by the overlap.
struct Clusters {
  int nc = 0;
  std::vector<int64_t> ext_ptr, core_ptr, a_off, r_off;   // nc + 1 each
  std::vector<int> ext_slot;    // unknown slots of the extended set (sorted)
  std::vector<int> core_pos;    // position of each core unknown in its ext list
  std::vector<int> core_slot;   // its unknown slot
};

// Same-triangle (local) interactions per edge pair, 4 values each:
// Gram <g, f>, <g, n x f>, sum w sigma (g x n).(n x f), sum w sigma g.(n x f)
struct LocalTerms {
  std::vector<int64_t> ptr;     // ne + 1
  std::vector<int> col;
  std::vector<double> val;      // 4 per entry
};

std::string build_geometry(const std::vector<double> &v, const std::vector<int> &t, const std::vector<int> &body,
                           Geometry &g);
void eval_sigma(const Geometry &g, const std::vector<SigmaEnd> &ends, std::vector<double> &sigma);
// conductivity at a point r of triangle T: profile ends evaluated at r, raw
// per-point values taken at T's nearest quadrature point
double sigma_at(const Geometry &g, const std::vector<SigmaEnd> &ends, const double *r, int T);
// post-processing helpers
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w);
int locate_surface_point(const Geometry &g, const double *r, int body, double tol);
void surface_currents_at(const Geometry &g, const Layout &L, const double *x, int T, const double *r, bool interior,
                         std::complex<double> J[3], std::complex<double> M[3]);
void build_layout(const Geometry &g, Layout &L);
void sigma_param_jacobian(const Geometry &g, const std::vector<SigmaEnd> &ends, std::vector<int64_t> &ptr,
                          std::vector<int> &idx, std::vector<double> &val, int64_t *npar);
std::string build_grids(const Geometry &g, double h, double k_e, double k_i, std::vector<GridDesc> &grids,
                        std::vector<int> &anchor /* np*3 absolute */, std::vector<double> &u /* np*3 */);
std::string build_near(const Geometry &g, double r_near, double kappa_s, NearList &nl);
// Largest preconditioner cluster: extended set (the block the Gauss-Jordan
// kernels invert) and core (staged whole in LDS by the transposed apply).
constexpr int PC_MAX_EXT = 8192;
constexpr int PC_MAX_CORE = 4096;
// Box clusters of side `cell` grown by `overlap`; sets *too_large when a
// grown box holds more than PC_MAX_EXT unknowns or its core more than
// PC_MAX_CORE.
std::string build_clusters(const Geometry &g, const Layout &L, double cell, double overlap, Clusters &cl,
                           bool *too_large,
                           const std::vector<int> *mask = nullptr);
void build_local_terms(const Geometry &g, const Layout &L, LocalTerms &lt);
void edge_slots(const Layout &L, int e, int *slots, int *nslots);

// ---------------------------------------------------------------------------
// block-Toeplitz product (fast-solver appendix): the mesh's periodic unit
// ---------------------------------------------------------------------------
// FP64 triangle record for exact interactions: vertices, quadrature points
// and weights, normal, centroid, in-plane basis (t1 along the first edge,
// t2 = n x t1), largest centroid-vertex distance, and per half function
// k (edge opposite vertex k) its signed coefficient s l / (2A)
struct TriD {
  double v[9], qp[21], qw[7], nrm[3], cen[3], t1[3], t2[3];
  double rho, coef[3];
  int body, pad;
};

// Rings along x: every periodic triangle is one of nt_r local triangles at
// ring r = 0..nr-1, translated by r dx; every periodic edge (both triangles
// periodic) one of ne_r local edges, whose two halves lie on local triangles
// at ring offsets 0 or -1 from the edge's ring.  Local triangles and edges
// are ordered by body.  Everything else (end caps and the edges touching
// them) is non-periodic.
struct RingTemplate {
  int nr = 0, P = 0, nt_r = 0, ne_r = 0, nbody = 0;
  double dx = 0;
  std::vector<TriD> tri;              // nt_r template triangles at ring 0
  std::vector<int> e_tri, e_k, e_off; // ne_r * 2: per side (0: +, 1: -) local tri, half index, ring offset
  std::vector<int> body_e0, body_t0;  // nbody + 1: local edge / triangle ranges of each body
  std::vector<int> ringmap;           // ne_r * nr: actual edge of local edge a at ring j (-1: none)
  std::vector<int> pmap;              // nt_r * nr: actual triangle of local triangle t at ring j
  std::vector<int> edge_loc, edge_ring, edge_sgn;   // per actual edge (-1 / 0 when non-periodic)
  std::vector<int> tri_loc;           // per actual triangle (-1 when non-periodic)
  std::vector<int> tri_ring;          // per actual triangle: its ring (-1 when non-periodic)
};

// Detects the periodic unit along x (period = smallest vertex x spacing),
// fills rt; an error string when fewer than 3 rings or no periodic part exist.
std::string build_rings(const Geometry &g, RingTemplate &rt);
// FP64 records of every triangle of the mesh
void make_tri_records(const Geometry &g, std::vector<TriD> &out);
// circulant length: smallest 2^a 3^b >= n
int smooth_length(int n);

// ---------------------------------------------------------------------------
// device-side records
// ---------------------------------------------------------------------------
// aligned to its size, so that LDS and global accesses of one value are single
// 8-byte (FP32) or 16-byte (FP64) instructions
template <typename T> struct alignas(2 * sizeof(T)) cx { T x, y; };

// per quadrature point (also a test point: the rule is shared)
template <typename T> struct PointRec {
  T f[9];        // the three half-RWG vectors f_j(q) of its triangle (j-major, unweighted)
  T w;           // quadrature weight (area included)
  T sigma;       // surface conductivity at q
  T u[3];        // position relative to its anchor node, in grid units (|u| <= 1/2)
  int anc;       // anchor node relative to the exterior grid origin, packed x | y << 14 | z << 23
  int tri;
};

template <typename T> struct TriRec {
  T nrm[3];
  T div[3];      // div f_j (constant on the triangle)
  int edge[3];
  int body;
  int flags;     // bit0: triangle carries sigma > 0
  int pad;
};

// per edge: row and unknown slots
struct EdgeRec {
  int tri[2];    // T+, T-
  int loc[2];    // local index of the edge in T+, T-
  int row[3];    // E row, H row, eq14 row (-1 on L edges)
  int col[3];    // L: (J, M, -1); R: (Je, Ji, M)
  int isR;
  int pad;
};

inline int pack_anchor(int x, int y, int z) { return x | (y << 14) | (z << 23); }

// the systems of a GMRES batch taking part in one step (kernel argument)
constexpr int KR_MAX_SYSTEMS = 8;
struct KrRun {
  int n;
  int b[KR_MAX_SYSTEMS];
};

}  // namespace scabs
