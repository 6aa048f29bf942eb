/*
 * scabs -- surface-conductive-absorber PMCHW solver for MI355X (gfx950).
 *
 * C ABI of the library.  The operation it implements is the Galerkin system
 * A x = b of the paper's Appendix A (eq19): RWG currents x = [J^L, M^L,
 * J_e^R, J_i^R, M^R] on closed dielectric surfaces, rows eq1/eq2 on edges
 * without surface conductivity and eq3/eq13/eq14 on absorber edges (Sec. II),
 * with the sigma-weighted terms tested at quadrature (target) points as in the
 * fast-solver appendix.  The matrix is never formed: its product is applied
 * with a precorrected FFT (grid projection, 3-D FFT convolution with the
 * Helmholtz kernel of each medium, interpolation, near-pair corrections).
 *
 * Conventions
 *  - exp(+j w t) time dependence, G = exp(-j k R) / (4 pi R) (Appendix A).
 *  - eps0 = mu0 = 1; lengths in the caller's unit (the paper uses the
 *    wavelength inside the guide).  k_l = omega sqrt(eps_l), Z_l = 1/sqrt(eps_l).
 *  - Complex vectors are interleaved (re, im) doubles, length 2N.
 *  - Every function returns SCABS_OK (0) or a negative SCABS_E_* code; no
 *    exception crosses the ABI.  scabs_last_error() gives the message.
 *  - Ownership: setters copy their inputs; the caller owns every buffer it
 *    passes.  Vector arguments of scabs_rhs_dipole, scabs_matvec,
 *    scabs_solve and scabs_gradient are DEVICE pointers on the context's
 *    device; work is queued on the context's stream and completes before the
 *    call returns.
 *  - Not thread safe per context: calls on one context must not overlap.
 */
#ifndef SCABS_H
#define SCABS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SCABS_OK 0
#define SCABS_E_ARG (-1)      /* invalid argument (null pointer, size, range) */
#define SCABS_E_MESH (-2)     /* mesh is not a closed, outward, 2-manifold surface */
#define SCABS_E_STATE (-3)    /* call out of order (e.g. matvec before build) */
#define SCABS_E_HIP (-4)      /* HIP runtime error */
#define SCABS_E_OOM (-5)      /* device allocation failed */
#define SCABS_E_NOCONV (-6)   /* iterative solve did not reach the tolerance */
#define SCABS_E_NAN (-7)      /* non-finite value in an input vector */

#define SCABS_FP64 0          /* every step in complex FP64 */
#define SCABS_FP32 1          /* projection, FFT convolution, near field in complex FP32 */
#define SCABS_MIXED 2         /* solve: FP32 inner GMRES inside FP64 iterative refinement */

typedef struct scabs_ctx scabs_ctx;

typedef struct {
  double h;        /* projection-grid spacing (> 0) */
  double r_near;   /* triangle pairs whose centroids are closer than r_near are
                      corrected to the exact Galerkin interaction; must exceed
                      the singular-pair radius (kappa_s * (rho_T + rho_T')) */
  double kappa_s;  /* singularity subtraction is used for pairs with centroid
                      distance < kappa_s * (rho_T + rho_T'), rho = largest
                      centroid-vertex distance; <= 0 selects 1.37 */
  int device;      /* HIP device ordinal */
  void *stream;    /* hipStream_t; NULL = a stream created by the library */
  int precond;     /* 2 (SCABS_PRECOND_PAPER, block-Toeplitz contexts only): the
                      preconditioners of the fast-solver appendix, the inverse
                      of the circulant that embeds the block-Toeplitz A_LL
                      (sigma-free periodic edges; applied by FFTs along the
                      rings, per-frequency inverse symbols computed once in
                      FP64 by Gauss-Jordan) and the block-diagonal inverse of
                      A_RR (absorber unknowns grouped in boxes of side
                      pc_cell, no overlap, exact near-field blocks as below);
                      L unknowns of non-periodic edges are passed through.
                      3 (SCABS_PRECOND_CIRC_SCHWARZ): the same circulant
                      inverse on A_LL with the restricted additive Schwarz
                      preconditioner below (with its overlap) on A_RR.
                      1: restricted additive Schwarz preconditioner on the exact
                      near-field matrix (boxes of side pc_cell grown by
                      pc_overlap); 0: none.  Where a grown box would hold
                      more than 8192 unknowns (or its core more than 4096),
                      cell and overlap are scaled down together (factor
                      0.85 per try) until all fit.
                      The block inverses (FP32 Gauss-Jordan) are stored as
                      FP16 pairs scaled per column; the preconditioner only
                      steers convergence, not the solution's accuracy */
  double pc_cell;     /* <= 0 selects 2 r_near */
  double pc_overlap;  /* < 0 selects 1.5 r_near; must not exceed pc_cell */
  int product;        /* SCABS_PRODUCT_PFFT (0): precorrected FFT on a lattice
                         (any mesh, approximate far field);
                         SCABS_PRODUCT_TOEPLITZ (1): the fast-solver appendix's
                         block-Toeplitz product on a mesh that repeats along x
                         (exact: the discrete Galerkin operator itself).  The
                         forward product of scabs_matvec and of the solves uses
                         it; the transposed product, the pointwise fields and
                         the gradient use the lattice operator either way */
} scabs_opts;

#define SCABS_PRECOND_NONE 0
#define SCABS_PRECOND_SCHWARZ 1
#define SCABS_PRECOND_PAPER 2
#define SCABS_PRECOND_CIRC_SCHWARZ 3
#define SCABS_PRODUCT_PFFT 0
#define SCABS_PRODUCT_TOEPLITZ 1

typedef struct {
  int64_t N, NL, NR;       /* unknowns: N = 2 NL + 3 NR (Appendix A) */
  int64_t n_edges, n_tris, n_points, n_bodies;
  int64_t n_near_pairs;    /* triangle pairs in the near list */
  int64_t nnz_near;        /* edge pairs in the near correction */
  int64_t grid_phys[3];    /* exterior grid, physical node counts */
  int64_t grid_fft[3];     /* exterior grid, FFT sizes */
  int64_t nnz_near_r;      /* of which on absorber (R) rows */
  int64_t n_clusters;      /* preconditioner clusters (0 without) */
  int64_t precond_entries; /* stored preconditioner coefficients */
  int64_t device_bytes;    /* device memory held by the context */
  int64_t precond_ext_entries; /* sum over clusters of their extended sets */
  int64_t product;         /* SCABS_PRODUCT_* of the built context */
  int64_t rings, circulant_length, ring_edges, ring_triangles;  /* block-Toeplitz: periodic
                              rings along x, circulant length P (2^a 3^b >= 2 rings - 1),
                              local edges and triangles of one ring (0 for the lattice) */
  int64_t nnz_nonperiodic; /* block-Toeplitz: entries of the sparse rows of
                              pairs with a non-periodic edge */
  int64_t toeplitz_table_bytes; /* block-Toeplitz: FP32 spectrum tables read per product */
} scabs_info_t;

typedef struct {
  int status;              /* SCABS_OK or SCABS_E_NOCONV */
  int outer_iters;         /* refinement steps (MIXED) or restart cycles (FP64) */
  int inner_iters;         /* total Arnoldi steps */
  int matvecs64, matvecs32; /* operator products this system's iteration used (the
                              batched launches compute every vector of the batch,
                              including systems that have already converged) */
  double rel_residual;     /* final ||b - A x|| / ||b|| with the FP64 operator */
} scabs_solve_info;

/* Create a context on opts->device.  *out receives the handle. */
int scabs_create(scabs_ctx **out, const scabs_opts *opts);

/* Surface triangulation (host arrays, copied): verts[3 nv], tris[3 nt]
 * (counter-clockwise seen from outside, so normals point into the exterior
 * medium, eq6-eq9), body[nt] (0-based body index; interior operators couple
 * triangles of the same body only).  Validated at scabs_build. */
int scabs_set_mesh(scabs_ctx *c, const double *verts, int64_t nv, const int32_t *tris, int64_t nt,
                   const int32_t *body);

/* Media: angular frequency omega and relative permittivities of the exterior
 * and of every body's interior (mu = 1). */
int scabs_set_media(scabs_ctx *c, double omega, double eps_out, double eps_in);

/* Surface conductivity (Sec. IV, eq60): sigma = sum over absorbers of
 * sigma0 * u(s), s = dir * (x_axis - x0) / length, u = 0 for s < 0, s held at
 * 1 beyond the absorber end.  Monomial: u = s^degree.  Piecewise linear: u is
 * the hat-function interpolant of ctrl[0..n-1] at s_k = k / (n - 1).
 * sigma is in units of 1/Z0.  An edge is an absorber (R) edge when sigma > 0
 * at a quadrature point of either of its triangles. */
int scabs_sigma_clear(scabs_ctx *c);
int scabs_sigma_add_monomial(scabs_ctx *c, int axis, double x0, double length, int dir, int degree,
                             double sigma0);
int scabs_sigma_add_pwl(scabs_ctx *c, int axis, double x0, double length, int dir, int n, const double *ctrl);
/* Raw conductivity at every quadrature point (host array, copied): nq must be
 * 7 n_tris of the mesh set before (points triangle by triangle, in the order
 * of the seven-point rule: centroid, then the two orbits of three), values
 * >= 0, added to the profile ends.  A later call replaces the earlier values;
 * scabs_sigma_clear removes them.  For scabs_sigma_gradient the nq values are
 * nq parameters, placed in the order the call was made among the ends. */
int scabs_set_sigma_points(scabs_ctx *c, const double *sigma_q, int64_t nq);

/* Build everything the products need: RWG edges, quadrature points, unknown
 * layout, grids, near list, exact and grid near-pair interactions (FP64 on the
 * device).  Must be called again after any setter. */
int scabs_build(scabs_ctx *c);

int scabs_info(const scabs_ctx *c, scabs_info_t *info);

/* Host copies of the layout: is_r[n_edges] (1 for absorber edges), idx[n_edges]
 * (index of the edge within its L or R block).  Either pointer may be NULL. */
int scabs_layout(const scabs_ctx *c, int32_t *is_r, int32_t *idx);

/* Right-hand side of an electric dipole (current moment p = I l, complex
 * moment[6] = re/im pairs) at pos inside body `body`; the incident field is
 * that of the dipole in the interior medium and vanishes on other bodies
 * (Sec. II).  b: device, 2N doubles. */
int scabs_rhs_dipole(scabs_ctx *c, const double pos[3], const double moment[6], int body, double *b);

/* y = A x for nrhs vectors stored one after another (device, 2N doubles
 * each).  prec: SCABS_FP64 or SCABS_FP32 (inputs and outputs stay FP64). */
int scabs_matvec(scabs_ctx *c, const double *x, double *y, int nrhs, int prec);

/* Solve A x = b (device vectors, nrhs of them).  x holds the initial guess
 * on entry.  mode: SCABS_FP64 (restarted GMRES on the FP64 operator) or
 * SCABS_MIXED (FP64 refinement around FP32-operator GMRES).  Orthogonalisation
 * (classical Gram-Schmidt, repeated where the first pass lost more than
 * 1 - 1/sqrt(2) of the norm) and the Hessenberg least squares are FP64 (the
 * basis of the FP32 inner solves is stored in FP32); the preconditioner (if
 * enabled) is applied on the right.
 * tol: relative residual with the FP64 operator.  info may be NULL.
 * Returns SCABS_E_NOCONV (x holds the last iterate) if max_iter Arnoldi
 * steps do not reach tol. */
int scabs_solve(scabs_ctx *c, const double *b, double *x, int nrhs, double tol, int max_iter, int restart,
                int mode, scabs_solve_info *info);

/* Transposed system (adjoint method).  y = A^T x, same argument rules as
 * scabs_matvec (block-Toeplitz contexts apply up to 8 vectors per pass, the
 * lattice product one at a time).  Precorrected-FFT
 * context: the lattice convolution is symmetric, so the transpose runs the
 * testing and projection steps in reverse (test-side sources with value and
 * derivative stencil weights, convolution, values read at the source points)
 * and the near correction through the mirrored pair entries.  Block-Toeplitz
 * context (fast-solver appendix): the exact transpose of the Galerkin matrix,
 * the ring-circulant blocks taken at frequency -f and contracted over the
 * row index, the local and sigma-point terms transposed per triangle, and
 * the stored entries of non-periodic edges read by column. */
int scabs_matvec_transpose(scabs_ctx *c, const double *x, double *y, int nrhs, int prec);

/* Solve A^T x = b; arguments and precision modes as scabs_solve (the right
 * preconditioner is the transposed Schwarz operator). */
int scabs_solve_transpose(scabs_ctx *c, const double *b, double *x, int nrhs, double tol, int max_iter, int restart,
                          int mode, scabs_solve_info *info);

/* HIP graphs in the Krylov solves (on by default).  Every Arnoldi step
 * launches the same sequence (preconditioner, then product, on nb vectors):
 * the first step of a shape (vectors, precision, transpose) runs it as usual
 * and captures it into a graph, later steps copy the step's basis vectors
 * into a staging buffer the graph reads and replay it (one launch instead of
 * one per kernel).  Results are the same bit for bit either way.  Graphs are
 * dropped whenever a buffer they read is reallocated (larger batches, a new
 * restart length), at scabs_build and at tuning changes; a shape whose capture
 * the runtime refuses keeps the ordinary launches.  Not used while stage
 * profiling is on.  on = 0 turns them off and frees them. */
int scabs_set_graphs(scabs_ctx *c, int on);

/* Autotuner of the block-Toeplitz product (contexts built with
 * SCABS_PRODUCT_TOEPLITZ; SCABS_E_STATE otherwise).  Launch choices, kept
 * per context separately for products of fewer than 8 vectors (class 0) and
 * of 8 vectors (class 1): the apply form of the per-frequency block
 * products (0: matrix cores for 8 FP32 vectors, vector ALUs otherwise; 1:
 * vector ALUs), the number of column groups of the periodic rows' sparse
 * part (1-16), the ring-axis lines per transform work-group (0: the
 * largest that fits 64 KiB of LDS) and the overlap of the stored entries'
 * sparse parts (1: on a second stream of the context, the short part beside
 * the forward transforms and the long part beside the inverse transforms,
 * the block products alone on the chip; 0: after the transforms, on the
 * context stream).  The transposed products follow their class's overlap.
 * Every choice computes the same product (only the order of sums over
 * column groups changes).
 * scabs_autotune times every candidate (forms {0, 1} for class 1, groups
 * {4, 8, 16}, lines {4, largest}, overlap {0, 1}) on FP32 products of this context, reps
 * products each after one warm-up, with HIP events on the context stream,
 * and keeps the fastest per class; rec (max_rec entries, may be NULL when
 * max_rec is 0) receives one record per candidate and *n_rec (may be NULL)
 * their number.  scabs_set_tune sets one class's choices directly
 * (SCABS_E_ARG for values out of range). */
typedef struct {
  int32_t nrhs;        /* 1 (class 0) or 8 (class 1) */
  int32_t apply_form;
  int32_t groups;
  int32_t lines;
  double us;           /* mean product time */
  int32_t chosen;      /* 1 for the kept candidate of its class */
  int32_t overlap;
} scabs_tune_record;
int scabs_autotune(scabs_ctx *c, int reps, scabs_tune_record *rec, int max_rec, int *n_rec);
int scabs_set_tune(scabs_ctx *c, int nrhs_class, int form, int groups, int lines, int overlap);

/* Several contexts' systems at once (batching across operators of uneven N:
 * absorber lengths, wavelengths, geometries).  Context i solves nrhs[i]
 * systems b[i] -> x[i] (device, its own N) as scabs_solve with the shared
 * tol, max_iter, restart and mode; info[i] (NULL, or info itself NULL) gets
 * nrhs[i] records.  The contexts run concurrently, each on its own stream
 * driven by its own host thread, so their launches interleave on the GPU;
 * results equal those of scabs_solve per context.  The contexts must be
 * distinct (SCABS_E_ARG otherwise) and not used elsewhere during the call.
 * Returns SCABS_OK, else an error of some context (preferred over
 * SCABS_E_NOCONV); per-context messages via scabs_last_error. */
int scabs_solve_batched(scabs_ctx *const *ctxs, int nctx, const double *const *b, double *const *x, const int *nrhs,
                        double tol, int max_iter, int restart, int mode, scabs_solve_info *const *info);

/* The right preconditioner of the solves on its own: y = M x (transpose = 0)
 * or y = M^T x (transpose = 1), M the restricted additive Schwarz operator
 * (the stored core rows of each cluster's inverted exact near-field block,
 * see scabs_opts.precond), for nrhs device vectors of 2N doubles stored one
 * after another (x and y must not overlap).  prec: SCABS_FP64, or SCABS_FP32
 * for the arithmetic of the FP32 inner solves (vectors stay FP64; the
 * transposed apply is FP64 either way).  SCABS_E_STATE when the context was
 * built without a preconditioner. */
int scabs_precond_apply(scabs_ctx *c, const double *x, double *y, int nrhs, int prec, int transpose);

/* An incident source in the interior medium of one body (Sec. II).  b = 0:
 * the electric dipole of scabs_rhs_dipole (current moment p = I l at pos).
 * b > 0: the Gaussian beam of Sec. II, generated by the same dipole placed at
 * the complex position pos - j b dir (a complex-source-point beam): it
 * propagates along +dir, with its waist at pos, Rayleigh distance b and waist
 * radius sqrt(2 b / k_i); its fields are the dipole's closed form continued
 * to the complex distance R = sqrt(d.d), d = r - pos + j b dir (principal
 * branch, cut on the disc of radius b around pos normal to dir), multiplied
 * by exp(-k_i b) so that the on-axis amplitude stays of order one.  dir must
 * be a unit vector when b > 0 (ignored otherwise). */
typedef struct {
  double pos[3];
  double dir[3];
  double b;
  double moment[6]; /* p, re/im pairs */
  int32_t body;
  int32_t pad;
} scabs_source;

/* Right-hand side of a source (as scabs_rhs_dipole for b = 0).  b: device,
 * N complex.  SCABS_E_ARG for a body out of range, b < 0 or a non-unit
 * direction. */
int scabs_rhs_source(scabs_ctx *c, const scabs_source *src, double *b);
/* Incident field of a source at every quadrature point (as
 * scabs_incident_dipole_points). */
int scabs_incident_source_points(scabs_ctx *c, const scabs_source *src, double *E);
/* Fields of a source at points of a region (as scabs_dipole_field). */
int scabs_source_field(scabs_ctx *c, const scabs_source *src, const double *pts, int npts, int region, double *E,
                       double *H);

/* Incident field of an electric dipole (as scabs_rhs_dipole) at every
 * quadrature point (zero on other bodies).  E: device, n_points * 3 complex
 * (6 n_points doubles), point-major. */
int scabs_incident_dipole_points(scabs_ctx *c, const double pos[3], const double moment[6], int body, double *E);

/* One-sided pointwise fields of the discrete operator at every quadrature
 * point for currents x (device, 2N doubles): Ee = E_e^+ (exterior limit of the
 * exterior-medium field of J_e, M_e) and Ei = E_i^- (interior limit of the
 * interior-medium field of J_i, M_i, without the incident field), each
 * n_points * 3 complex on the device.  These are the fields the sigma-weighted
 * tests of eq13 (rotated by n x) and eq14 integrate (Appendix A), for the
 * context's operator.  Precorrected-FFT context: the lattice operator's,
 * exact at the points of triangles carrying an absorber edge (elsewhere the
 * near-pair correction is omitted).  Block-Toeplitz context: the Galerkin
 * matrix's own at the points of triangles carrying an absorber edge -- on
 * periodic triangles the two in-plane components (the ones the sigma tests
 * read; normal component 0), on the others full vectors by direct summation
 * over every source triangle -- and 0 at all other points. */
int scabs_point_fields(scabs_ctx *c, const double *x, double *Ee, double *Ei);

/* Scattered fields at off-surface points pts (host, npts * 3) from currents x
 * (device): region < 0 the exterior medium's field of (J_e, M); region = b the
 * interior field of body b's currents (J_i, -M), without the incident field.
 * E, H: device, npts * 3 complex.  Plain 7-point rule on every triangle, so
 * the points must lie well away from the surface (several edge lengths). */
int scabs_eval_field(scabs_ctx *c, const double *x, const double *pts, int npts, int region, double *E, double *H);

/* Scattered fields as scabs_eval_field (same arguments, layouts and
 * results), accurate close to the surface as well: for every source triangle
 * whose centroid lies within SCABS_NEAR_FIELD_RADIUS times its radius (largest
 * centroid-vertex distance) of the point, the static part 1/(4 pi R) of the
 * kernel is integrated analytically over the triangle (the potential
 * integrals of the singular-pair treatment, Appendix A) and the smooth
 * remainder by the 7-point rule; farther triangles take the 7-point rule.
 * Points may lie at any distance from the surface on the side of the chosen
 * region (the field on the surface itself is not defined). */
#define SCABS_NEAR_FIELD_RADIUS 5.0
int scabs_eval_field_exact(scabs_ctx *c, const double *x, const double *pts, int npts, int region, double *E,
                           double *H);

/* Field post-processing (Sec. I, Table I; Sec. III).  Host arrays; E holds
 * n complex samples (re/im pairs) of one field component.
 * scabs_swr: the standing-wave ratio max|E| / min|E| over the samples
 * (out[0]) and the reflection coefficient (SWR - 1) / (SWR + 1) of a
 * transmission line (out[1]).
 * scabs_standing_wave_fit: least-squares fit of E(x) = a exp(-j beta x) +
 * c exp(+j beta x) at the positions xs; beta fixed (beta_lo == beta_hi) or
 * chosen in [beta_lo, beta_hi] by the smallest residual (scan of 401 values,
 * golden-section refinement).  out: beta, |c| / |a|, relative residual, |a|,
 * |c|, arg(c / a).
 * scabs_decay_fit: least-squares fit of ln|E| = c0 - alpha x and of the
 * unwrapped phase = p0 - beta x.  out: alpha, beta, relative residual of the
 * log fit, c0.
 * All three return SCABS_E_ARG for null pointers, too few samples or zero
 * magnitudes. */
int scabs_swr(const double *E, int n, double out[2]);
int scabs_standing_wave_fit(const double *xs, const double *E, int n, double beta_lo, double beta_hi, double out[6]);
int scabs_decay_fit(const double *xs, const double *E, int n, double out[4]);

/* Decay rate of the guided wave from Poynting's theorem (Sec. III,
 * eq_alpha_power): on the cross-section plane x = xpos, with the guide's
 * rectangle guide = {y0, y1, z0, z1} (its surface belongs to body `body`)
 * inside the box A = {Y0, Y1, Z0, Z1},
 *   alpha = [int_{L'} sigma |E_tan|^2 dl + Re int_L (E x H*).n dl]
 *           / [2 Re int_A (E x H*).x dS],
 * L' the guide's perimeter (E_tan from the magnetic current, |E_tan| = |M|;
 * sigma of the profile at the point), L the box boundary (outward normals).
 * Fields are totals (scabs_eval_field_exact plus the source's incident field
 * in its body, src may be NULL): interior on the guide rectangle, exterior on
 * the eight rectangles around it and on L; Gauss-Legendre rules of nq x nq
 * points per rectangle and 2 nq per segment.  x: device, the solution.
 * out: alpha, the perimeter integral, the boundary flux, the flux through A.
 * SCABS_E_ARG when the box does not contain the guide strictly, nq is not in
 * [2, 64] or a perimeter point is not on the body's surface. */
int scabs_poynting_decay(scabs_ctx *c, const double *x, const scabs_source *src, int body, double xpos,
                         const double guide[4], const double box[4], int nq, double out[4]);

/* Fields of an electric dipole (as scabs_rhs_dipole: current moment p = I l,
 * moment[6] re/im pairs, at pos inside body `body`) at points pts (host,
 * npts * 3) of region `region` (< 0 exterior, b >= 0 interior of body b):
 * the closed-form dipole fields of the interior medium (Sec. II; the
 * incident field of the rows) when region == body, zero otherwise.  E, H:
 * device, npts * 3 complex.  Added to scabs_eval_field's scattered fields
 * this gives the total field at monitor points. */
int scabs_dipole_field(scabs_ctx *c, const double pos[3], const double moment[6], int body, const double *pts,
                       int npts, int region, double *E, double *H);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * fields as scabs_eval_field, with the same arguments and results, but the
 * device copy of the points goes into a fixed scratch array of the library
 * (a static device array of 3 * SCABS_NOALLOC_MAX_POINTS doubles, 96 KiB,
 * one per GPU, held until the process ends) instead of a per-call
 * allocation; the call allocates nothing.  npts above
 * SCABS_NOALLOC_MAX_POINTS returns SCABS_E_ARG.  Every call on one GPU
 * shares that GPU's array, whatever its context: calls that overlap on one
 * GPU (other threads, other contexts' streams) race.  The context's own
 * buffers were allocated by scabs_build. */
#define SCABS_NOALLOC_MAX_POINTS 4096
int scabs_eval_field_noalloc(scabs_ctx *c, const double *x, const double *pts, int npts, int region, double *E,
                             double *H);

/* Transpose of the E part of scabs_eval_field: y = Q^T wE where E = Q x;
 * wE: device, npts * 3 complex; y: device, 2N doubles (overwritten). */
int scabs_eval_field_transpose(scabs_ctx *c, const double *pts, int npts, int region, const double *wE, double *y);

/* Number of profile parameters: per absorber in the order added, 1 (sigma0)
 * for a monomial profile, n for a piecewise-linear one (its control values). */
int scabs_sigma_params(const scabs_ctx *c, int64_t *n);

/* Gradient of a real objective f(x), x = A^-1 b, with respect to sigma by the
 * adjoint method: given x and lam solving A^T lam = g, g = df/dx in the sense
 * df = 2 Re(g^T dx), returns
 *   dfdsigma[q] = 2 Re[lam^T (db/dsigma_q - dA/dsigma_q x)]  (device, n_points;
 *                 may be NULL)
 *   dfdparam[k] = sum_q dsigma_q/dp_k dfdsigma[q]            (host,
 *                 scabs_sigma_params entries; may be NULL)
 * sigma enters A only through the sigma-weighted tests of eq13 and eq14 and b
 * through eq14's incident-field term; einc (device, n_points * 3 complex, from
 * scabs_incident_dipole_points; NULL for no incident field on the absorber)
 * supplies the latter.  The layout (which edges are absorber edges) is held
 * fixed. */
int scabs_sigma_gradient(scabs_ctx *c, const double *x, const double *lam, const double *einc, double *dfdsigma,
                         double *dfdparam);

/* One-call gradient: solves A^T lam = g (device, 2N doubles; g = df/dx as in
 * scabs_sigma_gradient) with scabs_solve_transpose's rules (tol, max_iter,
 * restart, mode; info may be NULL), then returns scabs_sigma_gradient(x, lam,
 * einc, dfdsigma, dfdparam).  SCABS_E_NOCONV if the adjoint solve misses tol
 * (no gradient is written then). */
int scabs_gradient(scabs_ctx *c, const double *x, const double *g, const double *einc, double tol, int max_iter,
                   int restart, int mode, double *dfdsigma, double *dfdparam, scabs_solve_info *info);

/* Stage timing (tracing): between scabs_profile_begin and scabs_profile_end
 * every stage of every product and solve is bracketed by HIP events on the
 * context stream.  scabs_profile_end synchronises the stream and returns, per
 * stage, the summed duration in milliseconds and the number of kernel launches
 * (one per record, or the launch count of a record that spans several)
 * (arrays of SCABS_NSTAGES entries; either may be NULL). */
#define SCABS_STAGE_UNPACK 0     /* unknowns -> per-edge currents */
#define SCABS_STAGE_PROJECT 1    /* sources -> grid */
#define SCABS_STAGE_FFT 2        /* grid convolution (all grids) */
#define SCABS_STAGE_INTERP 3     /* grid -> tested rows + local terms */
#define SCABS_STAGE_NEAR 4       /* near correction rows */
#define SCABS_STAGE_FP32_OFFSET 5  /* add to stages 0-4 for the FP32 product */
#define SCABS_STAGE_PRECOND 10   /* preconditioner application */
#define SCABS_STAGE_ORTHO 11     /* Gram-Schmidt, norms (FP64) */
#define SCABS_STAGE_PRECOND_T 12 /* transposed preconditioner application */
#define SCABS_STAGE_XLINE32 13   /* x-line transforms and kernel product of the FP32
                                    convolution: one record per product over the
                                    grids' back-to-back launches, counted as one
                                    launch per grid (inside stage SCABS_STAGE_FFT +
                                    SCABS_STAGE_FP32_OFFSET) */
#define SCABS_STAGE_GATHER32 14  /* lattice gather of the FP32 projection, recorded
                                    as SCABS_STAGE_XLINE32 (inside stage
                                    SCABS_STAGE_PROJECT + SCABS_STAGE_FP32_OFFSET) */
#define SCABS_STAGE_PCGATHER32 15 /* FP32 inner solves: the inputs of the Schwarz
                                     blocks gathered once per application into an
                                     ext-ordered FP32 copy (before each
                                     SCABS_STAGE_PRECOND record) */
#define SCABS_STAGE_TOEAPPLY32 16 /* block-Toeplitz product, FP32: the per-frequency block
                                     products (the ring-axis transforms are recorded
                                     as SCABS_STAGE_FFT + SCABS_STAGE_FP32_OFFSET, the
                                     sparse rows of the non-periodic pairs as
                                     SCABS_STAGE_NEAR + SCABS_STAGE_FP32_OFFSET) */
#define SCABS_STAGE_TOEAPPLY64 17 /* the same in FP64 */
#define SCABS_STAGE_TOEPRODUCT32 18 /* the whole block-Toeplitz product, FP32 (spans the
                                       records of its parts) */
#define SCABS_STAGE_TOEPRODUCT64 19 /* the same in FP64 */
#define SCABS_STAGE_TOEAPPLYT32 20 /* transposed block-Toeplitz product, FP32: the
                                      per-frequency transposed block products (its
                                      transforms are recorded as those of the forward
                                      product) */
#define SCABS_STAGE_TOEAPPLYT64 21 /* the same in FP64 */
#define SCABS_NSTAGES 22
int scabs_profile_begin(scabs_ctx *c);
int scabs_profile_end(scabs_ctx *c, double *ms, int64_t *count);
/* Restrict the stages that profiling sessions record to those whose bit
 * (1u << stage) is set in mask (0: every stage, the default); unrecorded
 * stages add no events to the stream.  SCABS_E_ARG for bits beyond
 * SCABS_NSTAGES. */
int scabs_profile_mask(scabs_ctx *c, uint32_t mask);
/* Algorithmic HBM bytes of the records of each stage of the last finished
 * profiling session (SCABS_NSTAGES entries, written to the caller's host
 * array; 0 for stages that do not define them).  SCABS_STAGE_XLINE32: the
 * physical x range of every transformed line read and written once;
 * SCABS_STAGE_GATHER32: the 8 weighted sources of every point read once and
 * the 8 fields of every lattice node written once;
 * SCABS_STAGE_PRECOND (FP32 inner solves): every stored coefficient once (4
 * bytes), per extended-set entry the FP32 gathered inputs of the vectors
 * applied, per unknown its index and FP64 outputs;
 * SCABS_STAGE_PCGATHER32: per extended-set entry its index, its column scale,
 * the FP64 inputs read and the FP32 copies written;
 * SCABS_STAGE_TOEAPPLY32/64 and SCABS_STAGE_TOEAPPLYT32/64: every entry of
 * the spectrum tables read once, the input spectra read and the output
 * spectra written once;
 * SCABS_STAGE_TOEPRODUCT32/64: the spectrum tables and the stored entries of
 * the non-periodic pairs that the product uses read once (the absorber test
 * records only on absorber rows), the input and output vectors read and
 * written once, and the ring-axis spectra written and read back once.
 * Returns SCABS_E_ARG for null arguments. */
int scabs_profile_bytes(const scabs_ctx *c, double *bytes);

const char *scabs_last_error(const scabs_ctx *c);
void scabs_destroy(scabs_ctx *c);

#ifdef __cplusplus
}
#endif
#endif
