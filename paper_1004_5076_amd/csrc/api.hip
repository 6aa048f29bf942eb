// C ABI of the library: context, setup orchestration, products and solves.
#include <algorithm>
#include <atomic>
#include <complex>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <thread>
#include <numeric>
#include <string>
#include <type_traits>
#include <vector>

#include "kernels.h"

namespace scabs {
template <typename VT>
void kr_dots(const cx<VT> *V, int64_t ldv, int jn, const cx<double> *w, int64_t N, cx<double> *part,
             cx<double> *out, int accumulate, hipStream_t s);
template <typename VT>
void kr_update(cx<double> *w, const cx<VT> *V, int64_t ldv, int jn, const cx<double> *c, int64_t N, double sgn,
               hipStream_t s);
void kr_norm(const cx<double> *w, int64_t N, double *part, double *out, hipStream_t s);
template <typename VT> void kr_scale(cx<VT> *dst, const cx<double> *src, const double *nrm, int64_t N, hipStream_t s);
void kr_widen(const cx<float> *src, cx<double> *dst, int64_t n, hipStream_t s);
void kr_zero(void *p, size_t bytes, hipStream_t s);
template <typename VT>
void kr_ortho_pass(const cx<VT> *V, int64_t ldv, int jn, cx<double> *w, int64_t N, const KrRun &run, int with_norm,
                   cx<double> *part, double *npart, cx<double> *hcol, int64_t hstride, int64_t hoff,
                   double *nrm_before, double *nrm_after, hipStream_t s);
template <typename VT>
void kr_scale_run(cx<VT> *Vdst, const cx<double> *w, const double *nrm, int64_t N, const KrRun &run, hipStream_t s);
size_t kr_ortho_part_entries(int jn_max, int nsys);
size_t kr_ortho_npart_entries(int64_t N, int nsys);
void kr_publish(const cx<double> *src, cx<double> *dst, int nnrm, int ncol, int stride, int rows, unsigned *flag,
                unsigned seq, hipStream_t s);
void kr_residual(const cx<double> *b, cx<double> *r, int64_t N, hipStream_t s);
void kr_axpy(cx<double> *x, const cx<double> *d, int64_t N, hipStream_t s);
void kr_finite(const double *v, int64_t n, int *bad, hipStream_t s);
}  // namespace scabs

using namespace scabs;

namespace {

struct HipError {
  hipError_t e;
  const char *what;
};
#define HIPCHK(x)                                   \
  do {                                              \
    hipError_t _e = (x);                            \
    if (_e != hipSuccess) throw HipError{_e, #x};   \
  } while (0)

// owned device allocation list
struct DevMem {
  std::vector<void *> ptrs;
  size_t bytes = 0;
  template <typename T> T *alloc(size_t n) {
    void *p = nullptr;
    if (n == 0) n = 1;
    hipError_t e = hipMalloc(&p, n * sizeof(T));
    if (e != hipSuccess) throw HipError{e, "hipMalloc"};
    ptrs.push_back(p);
    bytes += n * sizeof(T);
    return (T *)p;
  }
  template <typename T> T *upload(const std::vector<T> &v) {
    T *p = alloc<T>(v.size());
    if (!v.empty()) HIPCHK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return p;
  }
  void release() {
    for (void *p : ptrs) hipFree(p);
    ptrs.clear();
    bytes = 0;
  }
  void free_one(void *p) {
    for (size_t i = 0; i < ptrs.size(); i++)
      if (ptrs[i] == p) {
        hipFree(p);
        ptrs.erase(ptrs.begin() + i);
        return;
      }
  }
};

template <typename T> struct PrecState {
  PointRec<T> *pts = nullptr;
  TriRec<T> *tris = nullptr;
  cx<T> *V4 = nullptr, *S4 = nullptr;
  cx<T> *src = nullptr, *tri_out = nullptr;
  cx<T> *srcI = nullptr;           // edge-major currents of a batch (nb > 1)
  std::vector<DevGrid<T>> grids;   // host copies holding device pointers
  DevGrid<T> *grids_dev = nullptr;
  std::vector<GatherGrid<T>> gather;
  std::vector<cx<T> *> src4;       // per grid: ADJ_COEF adjoint-source coefficients per sorted point
  int bcap = 1;                    // vectors the per-vector buffers hold
  DevOperator<T> op;
  T inv_h = 0;
};

}  // namespace

struct scabs_ctx {
  scabs_opts opts{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // second stream of the block-Toeplitz products (the stored entries' sparse
  // parts beside the transforms), default priority; fork/join events
  hipStream_t side = nullptr;
  hipEvent_t ev_side[4] = {nullptr, nullptr, nullptr, nullptr};
  std::string err;
  // inputs
  std::vector<double> verts;
  std::vector<int> tris, body;
  double omega = 0, eps_out = 1, eps_in = 1;
  std::vector<SigmaEnd> ends;
  bool built = false;
  // host state
  Geometry geo;
  Layout lay;
  std::vector<GridDesc> grids;
  std::vector<int> anchor;
  std::vector<double> u;
  NearList near;
  double k_e = 0, k_i = 0, Z_e = 1, Z_i = 1;
  // device state
  DevMem mem;
  EdgeRec *edges = nullptr;
  int64_t *rowptr = nullptr;
  int *col = nullptr;
  int64_t nnz = 0;
  double *qp64 = nullptr;
  const TriD *trid = nullptr;   // per-triangle geometry records (near-surface fields)
  int *body_dev = nullptr;
  int64_t *tpos = nullptr;     // per near CSR entry (n, m): index of the entry (m, n)
  NearSetupArgs nsa{};         // near-pair tables kept for the pointwise-field pass
  uint8_t *tmask = nullptr;    // triangles with an absorber edge
  PrecState<float> p32;
  PrecState<double> p64;
  // preconditioner
  bool has_pc = false;
  bool pc_schwarz = false;   // the Schwarz (or, paper mode, block-diagonal A_RR) part
  int64_t pc_n_core = 0;     // unknowns in the cluster cores (N, or 3 N_R in paper mode)
  bool pc_circ = false;      // the circulant A_LL part (paper mode)
  cx<double> *pc_T64 = nullptr, *pc_cX64 = nullptr, *pc_cY64 = nullptr;
  cx<float> *pc_T32 = nullptr, *pc_cX32 = nullptr, *pc_cY32 = nullptr;
  Clusters cl;
  int64_t nnzR = 0;
  int64_t *pc_ext_ptr = nullptr, *pc_core_ptr = nullptr, *pc_r_off = nullptr;
  int *pc_ext_slot = nullptr, *pc_core_slot = nullptr;
  int *pc_items = nullptr;   // (cluster, first core row) per apply work-group
  int pc_n_items = 0;
  int *pc_items32 = nullptr;   // the same work-groups in the FP32 apply's dispatch order (cluster -1: empty)
  int pc_n_items32 = 0;
  int pc_max_ext = 0;        // largest extended set
  uint32_t *pc_Rt = nullptr;   // stored rows (FP16 pairs), see PcStore
  float *pc_Rs = nullptr;      // column scales, one per ext entry
  cx<float> *pc_xe = nullptr;  // FP32 ext-ordered inputs of the batched apply (n_ext x max batch)
  // transposed apply: cluster of every ext entry, and per unknown its ext entries
  int64_t pc_n_ext = 0;
  int64_t pc_coef = 0;   // stored preconditioner coefficients (core rows x ext columns, unpadded)
  int *pc_t_items = nullptr;   // (cluster, first ext column) per transposed-apply work-group
  int pc_n_t_items = 0;
  int64_t *pc_inv_ptr = nullptr, *pc_inv_pos = nullptr;
  cx<double> *pc_tmp = nullptr;
  cx<double> *pc_xc = nullptr;   // x in core order (N entries)
  // solver workspace (grown on demand)
  DevMem work;
  int work_restart = -1, work_nb = 0;
  int64_t work_N = -1;
  cx<double> *w = nullptr, *r = nullptr, *d = nullptr, *hcol = nullptr, *part = nullptr;
  cx<double> *z = nullptr, *t = nullptr;
  // HIP graphs of an Arnoldi step's preconditioner + product launches, one
  // per (vectors, precision, basis precision, transpose), captured on first
  // use and replayed every step; the step's basis vector is copied into
  // gstage first (the graph reads fixed addresses).  Dropped whenever a
  // buffer they read is reallocated, at a rebuild and at a tuning change.
  struct StepGraph {
    hipGraphExec_t exec;
    int nb, prec, vt, trans;
  };
  std::vector<StepGraph> step_graphs;
  bool graphs_on = true;
  cx<double> *gstage = nullptr;
  // Krylov bases: FP64 for FP64 solves, FP32 for the single-precision inner
  // solves of the mixed mode (each grown on demand)
  DevMem workV64, workV32;
  int64_t cap_V64 = 0, cap_V32 = 0;   // complex entries
  cx<double> *V64 = nullptr;
  cx<float> *V32 = nullptr;
  // stage timing with HIP events on the context stream
  bool prof_on = false;
  uint32_t prof_mask = ~0u;   // stages recorded by profiling sessions (bit k: stage k)
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  struct ProfRec {
    int stage;
    hipEvent_t e0, e1;
    double bytes;   // algorithmic HBM bytes of the bracketed work (0: not defined)
    int launches;   // kernel launches of the stage inside the record
  };
  std::vector<ProfRec> prof_recs;
  double prof_bytes[SCABS_NSTAGES] = {};   // per stage, last finished session
  double *nrm = nullptr, *nrm_part = nullptr, *npart = nullptr;
  // nrm (KR_NRM entries) followed by hcol in one device block, mirrored in
  // mapped, coherent host memory that a kernel writes at the end of each
  // Arnoldi step, followed by a sequence number the host waits for
  cx<double> *hblock = nullptr;
  cx<double> *hpin = nullptr, *hpin_dev = nullptr;
  size_t hpin_entries = 0;
  unsigned *hflag = nullptr, *hflag_dev = nullptr;
  unsigned hseq = 0;
  int *flag = nullptr;
  double *noalloc_pts = nullptr;   // this device's copy of the no-allocation scratch array
  // block-Toeplitz product (scabs_opts.product == SCABS_PRODUCT_TOEPLITZ)
  bool toe = false;
  RingTemplate rt;
  ToeDev<double> t64{};
  ToeDev<float> t32{};
  int toe_bcap = 0;
  int64_t toe_nnz = 0;
  cx<double> *toe_V4 = nullptr, *toe_S4 = nullptr;   // column-major entries: short part, then long part
  cx<float> *toe_V4f = nullptr, *toe_S4f = nullptr;
  int64_t toe_nshort = 0;
  const int *toe_capcol = nullptr, *toe_esgn = nullptr;
  const unsigned char *toe_eflag = nullptr;   // per edge: bit 0 periodic, bit 1 absorber
  cx<double> *toe_tri64 = nullptr;
  cx<float> *toe_tri32 = nullptr;
  // transposed product: circulant, long and short column parts per precision
  cx<float> *toe_tcol32 = nullptr, *toe_lcol32 = nullptr, *toe_scol32 = nullptr;
  cx<double> *toe_tcol64 = nullptr, *toe_lcol64 = nullptr, *toe_scol64 = nullptr;
  int *toe_capidx = nullptr;   // per edge its non-periodic index, -1 for periodic edges
  // exact point fields: triangles carrying an absorber edge (periodic ones,
  // the others) and the triangles of non-periodic edge halves (mask of halves)
  int *toe_abs_per = nullptr, *toe_abs_np = nullptr, *toe_np_tri = nullptr, *toe_np_mask = nullptr;
  int toe_nabs_per = 0, toe_nabs_np = 0, toe_nnp = 0;
  double toe_table_bytes[2] = {0, 0};   // per-frequency tables of one product (FP64, FP32)
  double toe_sparse_bytes[2] = {0, 0};  // stored non-periodic entries one product reads (FP64, FP32)
  // launch choices of the product for fewer than 8 and for 8 vectors:
  // {apply form (0 matrix cores at 8 FP32 vectors, 1 vector ALUs), column
  // groups of the periodic rows, transform lines per work-group (0: largest),
  // sparse parts on the second stream beside the transforms (1) or after
  // them (0)}
  int toe_tune[2][4] = {{0, 8, 0, 0}, {0, 8, 0, 0}};
  int toe_ncap = 0;
  double *toe_part64 = nullptr, *toe_rpart64 = nullptr;
  float *toe_part32 = nullptr, *toe_rpart32 = nullptr;
};

// drop the captured Arnoldi-step graphs (before any buffer they read goes)
// waits for a stream that is not capturing itself (every synchronisation of
// the library goes through here); while another thread of a batched solve
// captures its graph the runtime may refuse the wait, which is then asked
// again
static hipError_t sync_stream(hipStream_t s) {
  for (;;) {
    const hipError_t e = hipStreamSynchronize(s);
    if (e != hipErrorStreamCaptureUnsupported && e != hipErrorStreamCaptureImplicit) return e;
    (void)hipGetLastError();
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess || st != hipStreamCaptureStatusNone) return e;
    std::this_thread::yield();
  }
}

static void clear_graphs(scabs_ctx *c) {
  if (c->step_graphs.empty()) return;
  (void)sync_stream(c->stream);   // none of them may still be running
  for (auto &g : c->step_graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  c->step_graphs.clear();
}

// RAII stage timer: records a start/end event pair on the context stream
struct StageTimer {
  scabs_ctx *c;
  int stage;
  double bytes;
  int launches;
  hipEvent_t e0 = nullptr;
  hipStream_t strm;
  StageTimer(scabs_ctx *cc, int st, double b = 0, int n = 1, hipStream_t on = nullptr);
  ~StageTimer();
};

static hipEvent_t next_event(scabs_ctx *c) {
  if (c->ev_used == c->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->ev_pool.push_back(e);
  }
  return c->ev_pool[c->ev_used++];
}
StageTimer::StageTimer(scabs_ctx *cc, int st, double b, int n, hipStream_t on)
    : c(cc), stage(st), bytes(b), launches(n), strm(on ? on : cc->stream) {
  if (c->prof_on && ((c->prof_mask >> st) & 1u) && (e0 = next_event(c))) hipEventRecord(e0, strm);
}
StageTimer::~StageTimer() {
  if (!e0) return;
  hipEvent_t e1 = next_event(c);
  if (!e1) return;
  hipEventRecord(e1, strm);
  c->prof_recs.push_back({stage, e0, e1, bytes, launches});
}

static int fail(scabs_ctx *c, int code, const std::string &m) {
  if (c) c->err = m;
  return code;
}

static int hip_fail(scabs_ctx *c, const HipError &e) {
  return fail(c, SCABS_E_HIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
}

// every exception a call can raise becomes a status code: none crosses the ABI
#define SCABS_CATCH(c)                                                             \
  catch (const HipError &e) {                                                      \
    if (e.e == hipErrorOutOfMemory) return fail(c, SCABS_E_OOM, "device allocation failed"); \
    return hip_fail(c, e);                                                         \
  }                                                                                \
  catch (const std::bad_alloc &) {                                                 \
    return fail(c, SCABS_E_OOM, "host allocation failed");                         \
  }                                                                                \
  catch (const std::exception &e) {                                                \
    return fail(c, SCABS_E_HIP, e.what());                                         \
  }                                                                                \
  catch (const std::string &m) {                                                   \
    return fail(c, SCABS_E_STATE, m);                                              \
  }                                                                                \
  catch (...) {                                                                    \
    return fail(c, SCABS_E_HIP, "unexpected exception");                           \
  }

// ---------------------------------------------------------------------------
// scratch of scabs_eval_field_noalloc: a file-scope device array (each device
// holds its own copy until the process ends).  Host code never passes the
// array's name to a kernel or copy: it uses the address hipGetSymbolAddress
// returns with the device current, looked up once per device.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[3 * SCABS_NOALLOC_MAX_POINTS];

static std::mutex g_scratch_mu;
static std::vector<double *> g_scratch_ptr;   // per device ordinal (null: not looked up yet)

// the device's scratch address; the device must be current
static hipError_t scratch_address(int device, double **out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (device < 0) return hipErrorInvalidDevice;
  if ((size_t)device >= g_scratch_ptr.size()) g_scratch_ptr.resize(device + 1, nullptr);
  if (!g_scratch_ptr[device]) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = (double *)p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// build
// ---------------------------------------------------------------------------
// twiddle table length: a common multiple of the grid's FFT sizes (2^a or 3 2^a)
static int twiddle_length(const GridDesc &d) {
  int p2 = 1, three = 1;
  for (int a = 0; a < 3; a++) {
    int m = d.N[a];
    if (m % 3 == 0) {
      three = 3;
      m /= 3;
    }
    p2 = std::max(p2, m);
  }
  return p2 * three;
}
template <typename T>
static void build_precision(scabs_ctx *c, PrecState<T> &P, const std::vector<cx<double>> &tw_host,
                            const std::vector<int> &tw_off, const std::vector<cx<double> *> &ghat64,
                            const std::vector<cx<float> *> &ghat32, cx<T> *V4, cx<T> *S4, const cx<T> *V4T,
                            const cx<T> *S4T) {
  const Geometry &g = c->geo;
  const Layout &L = c->lay;
  const size_t np = (size_t)g.nt * NQ;
  // points
  std::vector<PointRec<T>> pts(np);
  const GridDesc &ext = c->grids[0];
  for (int Tt = 0; Tt < g.nt; Tt++) {
    const double A = g.area[Tt];
    for (int q = 0; q < NQ; q++) {
      size_t ip = (size_t)Tt * NQ + q;
      PointRec<T> &P0 = pts[ip];
      for (int j = 0; j < 3; j++) {
        int e = g.tedge[3 * Tt + j];
        double cf = g.tsign[3 * Tt + j] * g.elen[e] / (2.0 * A);
        const double *vj = &g.v[3 * g.t[3 * Tt + j]];
        for (int a = 0; a < 3; a++) P0.f[3 * j + a] = (T)(cf * (g.qp[3 * ip + a] - vj[a]));
      }
      P0.w = (T)g.qw[ip];
      P0.sigma = (T)L.sigma[ip];
      for (int a = 0; a < 3; a++) P0.u[a] = (T)c->u[3 * ip + a];
      P0.anc = pack_anchor(c->anchor[3 * ip] - ext.o[0], c->anchor[3 * ip + 1] - ext.o[1], c->anchor[3 * ip + 2] - ext.o[2]);
      P0.tri = Tt;
    }
  }
  P.pts = c->mem.upload(pts);
  std::vector<TriRec<T>> tr(g.nt);
  for (int Tt = 0; Tt < g.nt; Tt++) {
    TriRec<T> &r = tr[Tt];
    for (int a = 0; a < 3; a++) r.nrm[a] = (T)g.nrm[3 * Tt + a];
    int sig = 0;
    for (int j = 0; j < 3; j++) {
      int e = g.tedge[3 * Tt + j];
      r.div[j] = (T)(g.tsign[3 * Tt + j] * g.elen[e] / g.area[Tt]);
      r.edge[j] = e;
    }
    for (int q = 0; q < NQ; q++) sig |= L.sigma[(size_t)Tt * NQ + q] > 0;
    r.body = g.body[Tt];
    r.flags = sig;
    r.pad = 0;
  }
  P.tris = c->mem.upload(tr);
  P.src = c->mem.alloc<cx<T>>((size_t)g.ne * 3);
  P.srcI = nullptr;
  P.tri_out = c->mem.alloc<cx<T>>((size_t)g.nt * 9);
  P.V4 = V4;
  P.S4 = S4;
  // grids
  P.grids.clear();
  P.gather.clear();
  P.src4.clear();
  for (size_t gi = 0; gi < c->grids.size(); gi++) {
    const GridDesc &d = c->grids[gi];
    DevGrid<T> G{};
    G.which = d.which;
    for (int a = 0; a < 3; a++) {
      G.n[a] = d.n[a];
      G.N[a] = d.N[a];
      G.off[a] = d.o[a] - ext.o[a];
    }
    G.k = (T)d.k;
    G.Z = (T)(d.which < 0 ? c->Z_e : c->Z_i);
    size_t nphys = (size_t)d.n[0] * d.n[1] * d.n[2];
    G.phys = c->mem.alloc<cx<T>>(8 * nphys);
    G.spec = c->mem.alloc<cx<T>>(8 * (size_t)d.n[0] * d.N[1] * d.N[2]);
    int twL = twiddle_length(d);
    G.twL = twL;
    std::vector<cx<T>> tw(twL);
    for (int j = 0; j < twL; j++) tw[j] = {(T)tw_host[tw_off[gi] + j].x, (T)tw_host[tw_off[gi] + j].y};
    G.tw = c->mem.upload(tw);
    G.twx = nullptr;
    if (d.N[0] == XLINE_REG_LEN) {
      std::vector<cx<T>> tx(XLINE_REG_LEN + 64);
      auto root = [](long e, long n) {
        const double a = -2.0 * PI * (double)(e % n) / (double)n;
        return cx<double>{std::cos(a), std::sin(a)};
      };
      for (int a = 0; a < 16; a++)
        for (int l = 0; l < 64; l++) {
          const cx<double> w = root((long)a * l, XLINE_REG_LEN);
          tx[a * 64 + l] = {(T)w.x, (T)w.y};
        }
      for (int cc = 0; cc < 16; cc++)
        for (int p = 0; p < 4; p++) {
          const cx<double> w = root((long)p * cc, 64);
          tx[XLINE_REG_LEN + cc * 4 + p] = {(T)w.x, (T)w.y};
        }
      G.twx = c->mem.upload(tx);
    }
    if (sizeof(T) == sizeof(double))
      G.ghat = (const cx<T> *)ghat64[gi];
    else
      G.ghat = (const cx<T> *)ghat32[gi];
    G.ghx = nullptr;
    if (G.twx) {
      const int h0 = d.N[0] / 2 + 1, h1 = d.N[1] / 2 + 1, h2 = d.N[2] / 2 + 1;
      cx<T> *ghx = c->mem.alloc<cx<T>>((size_t)h0 * h1 * h2);
      launch_ghat_xfast<T>(G.ghat, ghx, h0, h1, h2, c->stream);
      G.ghx = ghx;
    }
    P.grids.push_back(G);
    // gather projection: the grid's points sorted by anchor cell
    std::vector<std::pair<int64_t, int>> key;
    for (int Tt = 0; Tt < g.nt; Tt++) {
      if (d.which >= 0 && g.body[Tt] != d.which) continue;
      for (int q = 0; q < NQ; q++) {
        size_t ip = (size_t)Tt * NQ + q;
        int ax = c->anchor[3 * ip] - d.o[0], ay = c->anchor[3 * ip + 1] - d.o[1], az = c->anchor[3 * ip + 2] - d.o[2];
        key.push_back({((int64_t)ax * d.n[1] + ay) * d.n[2] + az, (int)ip});
      }
    }
    std::sort(key.begin(), key.end());
    std::vector<int> perm(key.size());
    std::vector<int64_t> cellptr(nphys + 1, 0);
    std::vector<T> uu(3 * key.size());
    for (size_t i = 0; i < key.size(); i++) {
      perm[i] = key[i].second;
      cellptr[key[i].first + 1]++;
      for (int a = 0; a < 3; a++) uu[3 * i + a] = (T)c->u[3 * (size_t)key[i].second + a];
    }
    for (size_t k = 0; k < nphys; k++) cellptr[k + 1] += cellptr[k];
    GatherGrid<T> GG{};
    GG.np = (int)key.size();
    GG.ncell = (int64_t)nphys;
    GG.perm = c->mem.upload(perm);
    GG.cellptr = c->mem.upload(cellptr);
    GG.u = c->mem.upload(uu);
    GG.src = c->mem.alloc<cx<T>>(8 * key.size());
    std::vector<int> nz_ptr(d.n[0] + 1, 0), nz_yz;
    const size_t plane = (size_t)d.n[1] * d.n[2];
    for (int xx = 0; xx < d.n[0]; xx++) {
      for (size_t yz = 0; yz < plane; yz++)
        if (cellptr[xx * plane + yz + 1] > cellptr[xx * plane + yz]) nz_yz.push_back((int)yz);
      nz_ptr[xx + 1] = (int)nz_yz.size();
    }
    if (nz_yz.empty()) nz_yz.push_back(0);
    GG.nz_ptr = c->mem.upload(nz_ptr);
    GG.nz_yz = c->mem.upload(nz_yz);
    P.gather.push_back(GG);
    P.src4.push_back(c->mem.alloc<cx<T>>((size_t)ADJ_COEF * key.size()));
  }
  P.grids_dev = c->mem.upload(P.grids);
  P.inv_h = (T)(1.0 / c->opts.h);
  DevOperator<T> &op = P.op;
  op.np = (int)np;
  op.nt = g.nt;
  op.ne = g.ne;
  op.N = L.N;
  op.k_e = (T)c->k_e;
  op.k_i = (T)c->k_i;
  op.Z_e = (T)c->Z_e;
  op.Z_i = (T)c->Z_i;
  op.pts = P.pts;
  op.tris = P.tris;
  op.edges = c->edges;
  op.rowptr = c->rowptr;
  op.col = c->col;
  op.V4 = P.V4;
  op.S4 = P.S4;
  op.V4T = V4T;
  op.S4T = S4T;
  op.src = P.src;
  op.srcI = nullptr;
  op.tri_out = P.tri_out;
  op.edge_out = nullptr;
}

// Dispatch order of per-cluster work-groups: items holds (cluster, offset)
// pairs, a cluster's consecutive; len[k] is the run time of one of cluster
// k's work-groups (any unit).  Work-groups go to the eight XCDs in turn (work-
// group i to XCD i mod 8), so the returned list is read as eight interleaved
// lists: whole clusters go to the XCDs longest total first, each to the least
// loaded (longest-processing-time rule; a cluster's shared inputs then stay
// in one L2), and each XCD takes its work-groups longest first, so that the
// short ones fill the gaps at the end.  Shorter lists are padded with empty
// entries (cluster -1), which the kernels skip.
static std::vector<int> xcd_dispatch_order(const std::vector<int> &items, const std::vector<double> &len) {
  constexpr int NXCD = 8;
  const int nc = (int)len.size();
  std::vector<std::vector<int>> offs(nc);
  for (size_t i = 0; i + 1 < items.size(); i += 2) offs[items[i]].push_back(items[i + 1]);
  std::vector<double> work(nc);
  for (int k = 0; k < nc; k++) work[k] = len[k] * (double)offs[k].size();
  std::vector<int> by_work(nc);
  std::iota(by_work.begin(), by_work.end(), 0);
  std::stable_sort(by_work.begin(), by_work.end(), [&](int a, int b) { return work[a] > work[b]; });
  std::vector<double> load(NXCD, 0.0);
  std::vector<std::vector<int>> xcd(NXCD);
  for (int k : by_work) {
    if (offs[k].empty()) continue;
    const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    load[x] += work[k];
    xcd[x].push_back(k);
  }
  size_t n = 0;
  for (int x = 0; x < NXCD; x++) {
    std::stable_sort(xcd[x].begin(), xcd[x].end(), [&](int a, int b) { return len[a] > len[b]; });
    size_t cnt = 0;
    for (int k : xcd[x]) cnt += offs[k].size();
    n = std::max(n, cnt);
  }
  std::vector<int> out(2 * NXCD * n, -1);
  for (int x = 0; x < NXCD; x++) {
    size_t j = 0;
    for (int k : xcd[x])
      for (int o : offs[k]) {
        out[2 * (j * NXCD + x)] = k;
        out[2 * (j * NXCD + x) + 1] = o;
        j++;
      }
  }
  return out;
}

// Restricted additive Schwarz preconditioner from the exact near-field values
static void build_preconditioner(scabs_ctx *c, const cx<double> *X8, DevMem &tmp) {
  const Geometry &g = c->geo;
  const Layout &L = c->lay;
  hipStream_t s = c->stream;
  double cell = c->opts.pc_cell > 0 ? c->opts.pc_cell : 2.0 * c->opts.r_near;
  double ov = c->opts.pc_overlap >= 0 ? c->opts.pc_overlap : 1.5 * c->opts.r_near;
  // paper mode: block diagonal on the absorber unknowns only (no overlap);
  // the hybrid keeps the overlap (restricted additive Schwarz on A_RR)
  const bool paper = c->opts.precond == SCABS_PRECOND_PAPER || c->opts.precond == SCABS_PRECOND_CIRC_SCHWARZ;
  if (c->opts.precond == SCABS_PRECOND_PAPER) ov = 0.0;
  const std::vector<int> *mask = paper ? &L.isR : nullptr;
  // boxes that would hold more unknowns than one work-group inverts shrink
  // the cell and overlap together until every cluster fits
  std::string e;
  bool too_large = false;
  for (int attempt = 0;; attempt++) {
    too_large = false;
    e = build_clusters(g, L, cell, ov, c->cl, &too_large, mask);
    if (!too_large || attempt == 30) break;
    cell *= 0.85;
    ov *= 0.85;
  }
  if (!e.empty()) throw e;
  if (too_large) throw std::string("preconditioner clusters above the largest invertible block remain");
  // the cores must partition the unknowns (the applies write every unknown
  // once and the transposed apply permutes x into core order)
  const int64_t covered = paper ? 3 * (int64_t)L.NR : (int64_t)L.N;
  if (c->cl.core_ptr[c->cl.nc] != covered)
    throw std::string("preconditioner cores do not cover every unknown once");
  LocalTerms lt;
  build_local_terms(g, L, lt);
  const Clusters &cl = c->cl;
  std::vector<int> slot_edge(L.N);
  std::vector<int8_t> slot_kind(L.N);
  for (int ed = 0; ed < g.ne; ed++) {
    int sl[3], ns;
    edge_slots(L, ed, sl, &ns);
    for (int k = 0; k < ns; k++) {
      slot_edge[sl[k]] = ed;
      slot_kind[sl[k]] = (int8_t)(ns == 2 ? k : (k == 0 ? 0 : (k == 1 ? 2 : 1)));
    }
  }
  PrecondArgs p{};
  p.nc = cl.nc;
  p.Ze = c->Z_e;
  p.Zi = c->Z_i;
  p.rowptr = c->rowptr;
  p.col = c->col;
  p.X8 = X8;
  p.lptr = tmp.upload(lt.ptr);
  p.lcol = tmp.upload(lt.col);
  p.lval = tmp.upload(lt.val);
  p.slot_edge = tmp.upload(slot_edge);
  p.slot_kind = tmp.upload(slot_kind);
  p.isR = tmp.upload(L.isR);
  c->pc_ext_ptr = c->mem.upload(cl.ext_ptr);
  c->pc_ext_slot = c->mem.upload(cl.ext_slot);
  c->pc_core_ptr = c->mem.upload(cl.core_ptr);
  c->pc_core_slot = c->mem.upload(cl.core_slot);
  c->pc_r_off = c->mem.upload(cl.r_off);
  {
    // transposed apply: (cluster, first ext column) per work-group; per
    // unknown the ext entries that hold it (cluster order)
    const int64_t n_ext = cl.ext_ptr[cl.nc];
    std::vector<int> t_items;
    std::vector<int64_t> inv_ptr(L.N + 1, 0), inv_pos(n_ext);
    const int tcols = precond_t_cols_per_item();
    for (int k = 0; k < cl.nc; k++) {
      for (int64_t j0 = 0; j0 < cl.ext_ptr[k + 1] - cl.ext_ptr[k]; j0 += tcols) {
        t_items.push_back(k);
        t_items.push_back((int)j0);
      }
      for (int64_t q = cl.ext_ptr[k]; q < cl.ext_ptr[k + 1]; q++) inv_ptr[cl.ext_slot[q] + 1]++;
    }
    for (int64_t u = 0; u < L.N; u++) inv_ptr[u + 1] += inv_ptr[u];
    std::vector<int64_t> fill(inv_ptr.begin(), inv_ptr.end() - 1);
    for (int64_t q = 0; q < n_ext; q++) inv_pos[fill[cl.ext_slot[q]]++] = q;
    c->pc_n_ext = n_ext;
    c->pc_coef = 0;
    for (int k = 0; k < cl.nc; k++)
      c->pc_coef += (cl.ext_ptr[k + 1] - cl.ext_ptr[k]) * (cl.core_ptr[k + 1] - cl.core_ptr[k]);
    // the transposed apply's work-groups take time in proportion to their
    // cluster's core size (a fivefold range)
    std::vector<double> len_t(cl.nc);
    for (int k = 0; k < cl.nc; k++) len_t[k] = (double)(cl.core_ptr[k + 1] - cl.core_ptr[k]);
    t_items = xcd_dispatch_order(t_items, len_t);
    c->pc_n_t_items = (int)(t_items.size() / 2);
    c->pc_t_items = c->mem.upload(t_items);
    c->pc_inv_ptr = c->mem.upload(inv_ptr);
    c->pc_inv_pos = c->mem.upload(inv_pos);
    c->pc_tmp = c->mem.alloc<cx<double>>(n_ext);
    c->pc_xc = c->mem.alloc<cx<double>>((size_t)L.N);
  }
  {
    const int rows = precond_rows_per_item();
    std::vector<int> items;
    for (int k = 0; k < cl.nc; k++)
      for (int64_t r0 = 0; r0 < cl.core_ptr[k + 1] - cl.core_ptr[k]; r0 += rows) {
        items.push_back(k);
        items.push_back((int)r0);
      }
    c->pc_n_items = (int)(items.size() / 2);
    c->pc_items = c->mem.upload(items);
    // the FP32 batched apply's work-groups run in one and a half waves of
    // residency and differ up to threefold in length (a work-group's time
    // follows its cluster's column count)
    std::vector<double> len32(cl.nc);
    for (int k = 0; k < cl.nc; k++) len32[k] = (double)((cl.ext_ptr[k + 1] - cl.ext_ptr[k] + RT_CB - 1) / RT_CB);
    const std::vector<int> items32 = xcd_dispatch_order(items, len32);
    c->pc_n_items32 = (int)(items32.size() / 2);
    c->pc_items32 = c->mem.upload(items32);
  }
  p.ext_ptr = c->pc_ext_ptr;
  p.ext_slot = c->pc_ext_slot;
  p.a_off = tmp.upload(cl.a_off);
  p.A = tmp.alloc<cx<float>>((size_t)cl.a_off[cl.nc]);
  int *core_pos = tmp.upload(cl.core_pos);
  int *piv = tmp.alloc<int>((size_t)cl.ext_ptr[cl.nc]);
  int *status = tmp.alloc<int>(1);
  HIPCHK(hipMemsetAsync(status, 0, sizeof(int), s));
  c->pc_Rt = c->mem.alloc<uint32_t>((size_t)cl.r_off[cl.nc]);
  HIPCHK(hipMemsetAsync(c->pc_Rt, 0, sizeof(uint32_t) * (size_t)cl.r_off[cl.nc], s));   // padding stays zero
  c->pc_Rs = c->mem.alloc<float>((size_t)cl.ext_ptr[cl.nc]);
  // gathered inputs of the batched apply, with a zeroed tail for the padding
  // columns of the last cluster
  const size_t xe_n = ((size_t)cl.ext_ptr[cl.nc] + RT_CB) * precond_apply32_max_batch();
  c->pc_xe = c->mem.alloc<cx<float>>(xe_n);
  HIPCHK(hipMemsetAsync(c->pc_xe, 0, sizeof(cx<float>) * xe_n, s));
  p.n_ext = cl.ext_ptr[cl.nc];
  int max_ext = 0;
  for (int k = 0; k < cl.nc; k++) max_ext = std::max(max_ext, (int)(cl.ext_ptr[k + 1] - cl.ext_ptr[k]));
  c->pc_max_ext = max_ext;
  int npanels = 0;
  const std::vector<int> tiles = gj_tile_table(cl.ext_ptr, npanels);
  const int *tiles_dev = tmp.upload(tiles);
  cx<float> *gj_tmp = tmp.alloc<cx<float>>(gj_scratch_entries(cl.ext_ptr));
  launch_precond_build(p, cl.ext_ptr, tiles_dev, tiles, npanels, gj_tmp, c->pc_core_ptr, core_pos, c->pc_r_off,
                       c->pc_Rt, c->pc_Rs, piv, status, s);
  HIPCHK(hipGetLastError());
  int st = 0;
  HIPCHK(hipMemcpyAsync(&st, status, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(sync_stream(s));
  if (st) throw std::string("a preconditioner block is singular");
  c->pc_n_core = cl.core_ptr[cl.nc];
  c->has_pc = true;
  c->pc_schwarz = true;
}

// circulant part of the paper-mode preconditioner: the inverse symbol of
// A_LL at every frequency of the block-Toeplitz product, both precisions
static void build_circulant(scabs_ctx *c) {
  const ToeDev<double> &d = c->t64;
  const int n = 2 * d.ne_r;
  if (n > pc_circ_max_order()) throw std::string("ring too large for the circulant preconditioner");
  const size_t mat = (size_t)d.P * n * n;
  DevMem tmp;
  cx<double> *S = tmp.alloc<cx<double>>(mat), *B = tmp.alloc<cx<double>>(mat);
  c->pc_T64 = c->mem.alloc<cx<double>>(mat);
  c->pc_T32 = c->mem.alloc<cx<float>>(mat);
  HIPCHK(hipMemsetAsync(S, 0, sizeof(cx<double>) * mat, c->stream));
  launch_pc_circ_setup(d, S, B, c->pc_T64, c->pc_T32, c->stream);
  HIPCHK(hipGetLastError());
  const size_t spec = (size_t)d.P * n * 8;   // up to 8 vectors per apply
  c->pc_cX64 = c->mem.alloc<cx<double>>(spec);
  c->pc_cY64 = c->mem.alloc<cx<double>>(spec);
  c->pc_cX32 = c->mem.alloc<cx<float>>(spec);
  c->pc_cY32 = c->mem.alloc<cx<float>>(spec);
  // a singular symbol leaves NaN in its inverse
  std::vector<cx<double>> probe(std::min(mat, (size_t)4096));
  HIPCHK(hipMemcpyAsync(probe.data(), c->pc_T64, sizeof(cx<double>) * probe.size(), hipMemcpyDeviceToHost,
                        c->stream));
  HIPCHK(sync_stream(c->stream));
  for (const cx<double> &v : probe)
    if (!std::isfinite(v.x) || !std::isfinite(v.y)) throw std::string("the circulant symbol of A_LL is singular");
  c->pc_circ = true;
  c->has_pc = true;
}

static void apply_precond(scabs_ctx *c, const cx<double> *x, cx<double> *y, bool trans) {
  StageTimer tm(c, trans ? SCABS_STAGE_PRECOND_T : SCABS_STAGE_PRECOND);
  if (!trans)
    launch_precond_apply(c->pc_n_items, c->pc_items, c->pc_ext_ptr, c->pc_ext_slot, c->pc_core_ptr, c->pc_core_slot,
                         c->pc_r_off, PcStore{c->pc_Rt, c->pc_Rs}, x, y, c->pc_max_ext, c->stream);
  else
    launch_precond_apply_t<double>(c->pc_n_t_items, c->pc_t_items, c->lay.N, c->pc_n_core, c->pc_ext_ptr, c->pc_core_ptr, c->pc_core_slot,
                           c->pc_r_off, PcStore{c->pc_Rt, c->pc_Rs}, c->pc_inv_ptr, c->pc_inv_pos, c->pc_tmp, c->pc_xc, x, y,
                           c->stream);
}

// ---------------------------------------------------------------------------
// block-Toeplitz product: rings, exact ring blocks, their spectra, the sparse
// rows of the non-periodic edges
// ---------------------------------------------------------------------------
template <typename T>
static void toe_common(scabs_ctx *c, ToeDev<T> &d, const RingTemplate &rt, const int *ringmap, const int *pmap,
                       const int *esgn, const int *tloc, const int *tring, const int *ebody, const int *tbody, const int *be0,
                       const int *bt0, const int64_t *ibase, const int64_t *pbase, int64_t gi_per_f,
                       int64_t pi_per_f, const std::vector<double> &t1, const std::vector<double> &t2) {
  d.nr = rt.nr;
  d.P = rt.P;
  d.ne_r = rt.ne_r;
  d.nt_r = rt.nt_r;
  d.lines = toe_max_lines(rt.P, sizeof(T) == sizeof(float));
  d.apply_form = 0;
  d.Z_e = (T)c->Z_e;
  d.Z_i = (T)c->Z_i;
  d.ringmap = ringmap;
  d.pmap = pmap;
  d.edge_sgn = esgn;
  d.tri_loc = tloc;
  d.tri_ring = tring;
  d.ebody = ebody;
  d.tbody = tbody;
  d.body_e0 = be0;
  d.body_t0 = bt0;
  d.ibase = ibase;
  d.pbase = pbase;
  d.gi_per_f = gi_per_f;
  d.pi_per_f = pi_per_f;
  std::vector<cx<T>> tw(rt.P);
  for (int j = 0; j < rt.P; j++) {
    const double a = -2.0 * PI * j / rt.P;
    tw[j] = {(T)std::cos(a), (T)std::sin(a)};
  }
  d.tw = c->mem.upload(tw);
  std::vector<T> a1(t1.begin(), t1.end()), a2(t2.begin(), t2.end());
  d.t1 = c->mem.upload(a1);
  d.t2 = c->mem.upload(a2);
}

static std::string build_toeplitz(scabs_ctx *c) {
  const Geometry &g = c->geo;
  RingTemplate &rt = c->rt;
  std::string e = build_rings(g, rt);
  if (!e.empty()) return e;
  if (rt.P > 8192) return "too many periodic rings for the ring-axis transforms (more than 4096)";
  if ((size_t)4 * rt.ne_r * 8 * sizeof(cx<double>) > 160 * 1024)
    return "too many edges in one ring for the per-frequency block product (more than 320)";
  hipStream_t s = c->stream;
  const int nb = g.nbody, ne_r = rt.ne_r, nt_r = rt.nt_r, P = rt.P;
  const int64_t R2 = 2 * (int64_t)NQ * nt_r;
  std::vector<int> ebody(ne_r), tbody(nt_r);
  for (int a = 0; a < ne_r; a++) ebody[a] = rt.tri[rt.e_tri[2 * a]].body;
  for (int t = 0; t < nt_r; t++) tbody[t] = rt.tri[t].body;
  std::vector<int64_t> ibase(nb + 1, 0), pbase(nb + 1, 0);
  for (int b = 0; b < nb; b++) {
    const int64_t neb = rt.body_e0[b + 1] - rt.body_e0[b], ntb = rt.body_t0[b + 1] - rt.body_t0[b];
    ibase[b + 1] = ibase[b] + neb * neb;
    pbase[b + 1] = pbase[b] + 2 * NQ * ntb * neb;
  }
  ToeSetupArgs a{};
  a.nr = rt.nr;
  a.P = P;
  a.ne_r = ne_r;
  a.nt_r = nt_r;
  a.nbody = nb;
  a.dx = rt.dx;
  a.k_e = c->k_e;
  a.k_i = c->k_i;
  a.Z_e = c->Z_e;
  a.Z_i = c->Z_i;
  a.kappa = c->opts.kappa_s;
  a.tri = c->mem.upload(rt.tri);
  a.e_tri = c->mem.upload(rt.e_tri);
  a.e_k = c->mem.upload(rt.e_k);
  a.e_off = c->mem.upload(rt.e_off);
  a.ebody = c->mem.upload(ebody);
  a.body_e0 = c->mem.upload(rt.body_e0);
  a.body_t0 = c->mem.upload(rt.body_t0);
  a.ibase = c->mem.upload(ibase);
  a.pbase = c->mem.upload(pbase);
  {
    DevMem tmp;
    const size_t nLe = (size_t)ne_r * ne_r, nLi = (size_t)ibase[nb], nPe = (size_t)R2 * ne_r, nPi = (size_t)pbase[nb];
    a.sLe = tmp.alloc<cx<double>>(nLe * P);
    a.sKe = tmp.alloc<cx<double>>(nLe * P);
    a.sLi = tmp.alloc<cx<double>>(nLi * P);
    a.sKi = tmp.alloc<cx<double>>(nLi * P);
    a.sPeJ = tmp.alloc<cx<double>>(nPe * P);
    a.sPeM = tmp.alloc<cx<double>>(nPe * P);
    a.sPiJ = tmp.alloc<cx<double>>(nPi * P);
    a.sPiM = tmp.alloc<cx<double>>(nPi * P);
    std::vector<cx<double>> tw(P);
    for (int j = 0; j < P; j++) tw[j] = {std::cos(-2.0 * PI * j / P), std::sin(-2.0 * PI * j / P)};
    cx<double> *tw64 = tmp.upload(tw);
    launch_toe_setup(a, s);
    HIPCHK(hipGetLastError());
    launch_toe_series_fft(a.sLe, (int64_t)nLe, P, tw64, s);
    launch_toe_series_fft(a.sKe, (int64_t)nLe, P, tw64, s);
    launch_toe_series_fft(a.sLi, (int64_t)nLi, P, tw64, s);
    launch_toe_series_fft(a.sKi, (int64_t)nLi, P, tw64, s);
    launch_toe_series_fft(a.sPeJ, (int64_t)nPe, P, tw64, s);
    launch_toe_series_fft(a.sPeM, (int64_t)nPe, P, tw64, s);
    launch_toe_series_fft(a.sPiJ, (int64_t)nPi, P, tw64, s);
    launch_toe_series_fft(a.sPiM, (int64_t)nPi, P, tw64, s);
    HIPCHK(hipGetLastError());
    cx<double> *GE64 = c->mem.alloc<cx<double>>(2 * nLe * P), *GI64 = c->mem.alloc<cx<double>>(2 * nLi * P);
    cx<double> *PE64 = c->mem.alloc<cx<double>>(2 * nPe * P), *PI64 = c->mem.alloc<cx<double>>(2 * nPi * P);
    cx<float> *GE32 = c->mem.alloc<cx<float>>(2 * nLe * P), *GI32 = c->mem.alloc<cx<float>>(2 * nLi * P);
    cx<float> *PE32 = c->mem.alloc<cx<float>>(2 * nPe * P), *PI32 = c->mem.alloc<cx<float>>(2 * nPi * P);
    launch_toe_layout(a, 0, a.sLe, a.sKe, (int64_t)nLe, GE64, GE32, s);
    launch_toe_layout(a, 1, a.sLi, a.sKi, (int64_t)nLi, GI64, GI32, s);
    launch_toe_layout(a, 2, a.sPeJ, a.sPeM, (int64_t)nPe, PE64, PE32, s);
    launch_toe_layout(a, 3, a.sPiJ, a.sPiM, (int64_t)nPi, PI64, PI32, s);
    HIPCHK(hipGetLastError());
    HIPCHK(sync_stream(s));
    tmp.release();
    c->t64.GE = GE64;
    c->t64.GI = GI64;
    c->t64.PE = PE64;
    c->t64.PI = PI64;
    c->t32.GE = GE32;
    c->t32.GI = GI32;
    c->t32.PE = PE32;
    c->t32.PI = PI32;
    const double ent = 2.0 * P * (double)(nLe + nLi + nPe + nPi);
    c->toe_table_bytes[0] = ent * sizeof(cx<double>);
    c->toe_table_bytes[1] = ent * sizeof(cx<float>);
  }
  // maps and per-local-triangle bases
  std::vector<double> t1(3 * (size_t)nt_r), t2(3 * (size_t)nt_r);
  for (int t = 0; t < nt_r; t++)
    for (int k = 0; k < 3; k++) {
      t1[3 * t + k] = rt.tri[t].t1[k];
      t2[3 * t + k] = rt.tri[t].t2[k];
    }
  const int *ringmap = c->mem.upload(rt.ringmap), *pmap = c->mem.upload(rt.pmap);
  const int *esgn = c->mem.upload(rt.edge_sgn), *tloc = c->mem.upload(rt.tri_loc);
  const int *esgn_dev = esgn;
  const int *tring = c->mem.upload(rt.tri_ring);
  toe_common(c, c->t64, rt, ringmap, pmap, esgn, tloc, tring, a.ebody, c->mem.upload(tbody), a.body_e0, a.body_t0, a.ibase,
             a.pbase, ibase[nb], pbase[nb], t1, t2);
  toe_common(c, c->t32, rt, ringmap, pmap, esgn, tloc, tring, a.ebody, c->t64.tbody, a.body_e0, a.body_t0, a.ibase, a.pbase,
             ibase[nb], pbase[nb], t1, t2);
  // exact entries of the pairs with a non-periodic edge, column-major: the
  // short part (every row against each non-periodic column; read by the
  // periodic rows), then the long part (each non-periodic row against every
  // column)
  std::vector<int> nonper;
  for (int n = 0; n < g.ne; n++)
    if (rt.edge_loc[n] < 0) nonper.push_back(n);
  const int64_t ncap = (int64_t)nonper.size();
  const int64_t nshort = ncap * g.ne;
  const int64_t nnz = 2 * nshort;
  std::vector<int> rows(nnz), cols(nnz);
  for (int64_t j = 0; j < ncap; j++)
    for (int n = 0; n < g.ne; n++) {
      rows[j * g.ne + n] = n;
      cols[j * g.ne + n] = nonper[j];
    }
  for (int m = 0; m < g.ne; m++)
    for (int64_t i = 0; i < ncap; i++) {
      rows[nshort + (int64_t)m * ncap + i] = nonper[i];
      cols[nshort + (int64_t)m * ncap + i] = m;
    }
  {
    // entries the row kernels read: the short part on periodic rows, the
    // long part on non-periodic rows; absorber test records on absorber rows
    int64_t nR = 0, nRcap = 0;
    for (int n = 0; n < g.ne; n++) nR += c->lay.isR[n] != 0;
    for (int n : nonper) nRcap += c->lay.isR[n] != 0;
    const double recs = 4.0 * ((double)(g.ne - ncap) * ncap + (double)ncap * g.ne) +
                        4.0 * ((double)(nR - nRcap) * ncap + (double)nRcap * g.ne);
    c->toe_sparse_bytes[0] = recs * sizeof(cx<double>);
    c->toe_sparse_bytes[1] = recs * sizeof(cx<float>);
  }
  c->toe_ncap = (int)ncap;
  c->toe_nshort = nshort;
  c->toe_capcol = c->mem.upload(nonper);
  {
    std::vector<int> capidx(g.ne, -1);
    for (size_t j = 0; j < nonper.size(); j++) capidx[nonper[j]] = (int)j;
    c->toe_capidx = c->mem.upload(capidx);
    std::vector<int> abs_per, abs_np, np_tri, np_mask;
    for (int T = 0; T < g.nt; T++) {
      const int *te = g.tedge.data() + 3 * T;
      if (c->lay.isR[te[0]] || c->lay.isR[te[1]] || c->lay.isR[te[2]])
        (rt.tri_loc[T] >= 0 ? abs_per : abs_np).push_back(T);
      int mask = 0;
      for (int k = 0; k < 3; k++) mask |= (rt.edge_loc[te[k]] < 0) << k;
      if (mask) {
        np_tri.push_back(T);
        np_mask.push_back(mask);
      }
    }
    c->toe_nabs_per = (int)abs_per.size();
    c->toe_nabs_np = (int)abs_np.size();
    c->toe_nnp = (int)np_tri.size();
    c->toe_abs_per = abs_per.empty() ? nullptr : c->mem.upload(abs_per);
    c->toe_abs_np = abs_np.empty() ? nullptr : c->mem.upload(abs_np);
    c->toe_np_tri = np_tri.empty() ? nullptr : c->mem.upload(np_tri);
    c->toe_np_mask = np_mask.empty() ? nullptr : c->mem.upload(np_mask);
    const size_t nc = std::max<size_t>(1, nonper.size());
    // column outputs of the transposed product for up to 8 vectors
    const size_t V = 8;
    c->toe_tcol32 = c->mem.alloc<cx<float>>(4 * (size_t)g.ne * V);
    c->toe_lcol32 = c->mem.alloc<cx<float>>(3 * (size_t)g.ne * V);
    c->toe_scol32 = c->mem.alloc<cx<float>>(3 * nc * TOE_T_SHORT_SPLIT * V);
    c->toe_tcol64 = c->mem.alloc<cx<double>>(4 * (size_t)g.ne * V);
    c->toe_lcol64 = c->mem.alloc<cx<double>>(3 * (size_t)g.ne * V);
    c->toe_scol64 = c->mem.alloc<cx<double>>(3 * nc * TOE_T_SHORT_SPLIT * V);
    std::vector<unsigned char> ef(g.ne);
    for (int n = 0; n < g.ne; n++) ef[n] = (unsigned char)((rt.edge_sgn[n] != 0) | ((c->lay.isR[n] != 0) << 1));
    c->toe_eflag = c->mem.upload(ef);
  }
  c->toe_esgn = esgn_dev;
  c->toe_nnz = nnz;
  c->toe_V4 = c->mem.alloc<cx<double>>(4 * (size_t)nnz);
  c->toe_S4 = c->mem.alloc<cx<double>>(4 * (size_t)nnz);
  c->toe_V4f = c->mem.alloc<cx<float>>(4 * (size_t)nnz);
  c->toe_S4f = c->mem.alloc<cx<float>>(4 * (size_t)nnz);
  {
    DevMem tmp;
    std::vector<TriD> all;
    make_tri_records(g, all);
    ToeCapArgs ca{};
    ca.nnz = nnz;
    ca.row = tmp.upload(rows);
    ca.col = tmp.upload(cols);
    ca.et = tmp.upload(g.et);
    ca.tedge = tmp.upload(g.tedge);
    ca.tri = tmp.upload(all);
    ca.sigma = tmp.upload(c->lay.sigma);
    ca.k_e = c->k_e;
    ca.k_i = c->k_i;
    ca.kappa = c->opts.kappa_s;
    ca.V4 = c->toe_V4;
    ca.S4 = c->toe_S4;
    ca.V4f = c->toe_V4f;
    ca.S4f = c->toe_S4f;
    launch_toe_cap_entries(ca, s);
    HIPCHK(hipGetLastError());
    HIPCHK(sync_stream(s));
  }
  c->toe_bcap = 0;
  return "";
}

// grow the per-vector buffers of the block-Toeplitz product to nb vectors
template <typename T> static void toe_ensure(scabs_ctx *c, ToeDev<T> &d, cx<T> *&tri_out, int nb) {
  const int cap = sizeof(T) == sizeof(float) ? (c->toe_bcap & 0xffff) : (c->toe_bcap >> 16);
  if (nb <= cap) return;
  clear_graphs(c);
  const Geometry &g = c->geo;
  if (d.X) {
    c->mem.free_one(d.X);
    c->mem.free_one(d.Y);
    c->mem.free_one(d.edge_out);
    c->mem.free_one(d.pf);
    c->mem.free_one(tri_out);
  }
  const size_t R2 = 2 * (size_t)NQ * d.nt_r;
  d.X = c->mem.alloc<cx<T>>((size_t)d.P * 4 * d.ne_r * nb);
  d.Y = c->mem.alloc<cx<T>>((size_t)d.P * (2 * d.ne_r + 2 * R2) * nb);
  d.edge_out = c->mem.alloc<cx<T>>((size_t)nb * g.ne * 2);
  d.pf = c->mem.alloc<cx<T>>((size_t)nb * 2 * R2 * d.nr);
  tri_out = c->mem.alloc<cx<T>>((size_t)nb * g.nt * 9);
  const size_t npart = (size_t)std::max(1, c->toe_ncap * ((g.ne + toe_long_chunk() - 1) / toe_long_chunk())) * 6 * nb;
  const size_t nrpart = (size_t)toe_row_groups() * nb * 6 * g.ne;
  if (sizeof(T) == sizeof(float)) {
    if (c->toe_part32) c->mem.free_one(c->toe_part32);
    if (c->toe_rpart32) c->mem.free_one(c->toe_rpart32);
    c->toe_part32 = c->mem.alloc<float>(npart);
    c->toe_rpart32 = c->mem.alloc<float>(nrpart);
  } else {
    if (c->toe_part64) c->mem.free_one(c->toe_part64);
    if (c->toe_rpart64) c->mem.free_one(c->toe_rpart64);
    c->toe_part64 = c->mem.alloc<double>(npart);
    c->toe_rpart64 = c->mem.alloc<double>(nrpart);
  }
  // rows of non-periodic edges are never written by the transforms
  HIPCHK(hipMemsetAsync(d.edge_out, 0, sizeof(cx<T>) * nb * g.ne * 2, c->stream));
  HIPCHK(hipMemsetAsync(d.pf, 0, sizeof(cx<T>) * (size_t)nb * 2 * R2 * d.nr, c->stream));
  if (sizeof(T) == sizeof(float))
    c->toe_bcap = (c->toe_bcap & ~0xffff) | nb;
  else
    c->toe_bcap = (c->toe_bcap & 0xffff) | (nb << 16);
}

static int do_build(scabs_ctx *c) {
  c->built = false;
  c->has_pc = false;
  c->pc_schwarz = false;
  c->pc_circ = false;
  if (c->opts.precond >= SCABS_PRECOND_PAPER && c->opts.product != SCABS_PRODUCT_TOEPLITZ)
    return fail(c, SCABS_E_ARG, "the circulant preconditioner needs the block-Toeplitz product");
  if (c->opts.precond < 0 || c->opts.precond > SCABS_PRECOND_CIRC_SCHWARZ) return fail(c, SCABS_E_ARG, "unknown precond");
  clear_graphs(c);
  c->mem.release();
  // every device buffer of the last build is gone: forget the per-vector
  // buffers the products grow on demand, so that growing them never frees an
  // address the new build has been handed again
  c->t64 = ToeDev<double>{};
  c->t32 = ToeDev<float>{};
  c->toe_bcap = 0;
  c->toe_tri64 = nullptr;
  c->toe_tri32 = nullptr;
  c->toe_part64 = c->toe_rpart64 = nullptr;
  c->toe_part32 = c->toe_rpart32 = nullptr;
  c->p64.srcI = nullptr;
  c->p32.srcI = nullptr;
  c->work.release();
  c->work_restart = -1;
  c->work_N = -1;
  c->work_nb = 0;
  c->p32.bcap = c->p64.bcap = 1;
  if (c->verts.empty() || c->tris.empty()) return fail(c, SCABS_E_STATE, "mesh not set");
  if (!(c->omega > 0)) return fail(c, SCABS_E_STATE, "media not set");
  std::string e = build_geometry(c->verts, c->tris, c->body, c->geo);
  if (!e.empty()) return fail(c, SCABS_E_MESH, e);
  Geometry &g = c->geo;
  eval_sigma(g, c->ends, c->lay.sigma);
  build_layout(g, c->lay);
  c->k_e = c->omega * std::sqrt(c->eps_out);
  c->k_i = c->omega * std::sqrt(c->eps_in);
  c->Z_e = 1.0 / std::sqrt(c->eps_out);
  c->Z_i = 1.0 / std::sqrt(c->eps_in);
  e = build_grids(g, c->opts.h, c->k_e, c->k_i, c->grids, c->anchor, c->u);
  if (!e.empty()) return fail(c, SCABS_E_ARG, e);
  e = build_near(g, c->opts.r_near, c->opts.kappa_s, c->near);
  if (!e.empty()) return fail(c, SCABS_E_ARG, e);
  const size_t np = (size_t)g.nt * NQ;
  // test boxes must fit the setup kernel's LDS tile; kernel-table extent
  std::vector<int> alo(3 * g.nt), ahi(3 * g.nt);
  for (int T = 0; T < g.nt; T++)
    for (int a = 0; a < 3; a++) {
      int lo = 1 << 30, hi = -(1 << 30);
      for (int q = 0; q < NQ; q++) {
        int v = c->anchor[3 * ((size_t)T * NQ + q) + a];
        lo = std::min(lo, v);
        hi = std::max(hi, v);
      }
      alo[3 * T + a] = lo;
      ahi[3 * T + a] = hi;
      if (hi - lo + 3 > 7) return fail(c, SCABS_E_ARG, "grid spacing too fine for the triangle size (stencil box > 7)");
    }
  int D = 0;
  for (int T = 0; T < g.nt; T++)
    for (int64_t p = c->near.tptr[T]; p < c->near.tptr[T + 1]; p++) {
      int Tp = c->near.src[p];
      for (int a = 0; a < 3; a++)
        D = std::max(D, std::max(ahi[3 * T + a] - alo[3 * Tp + a], ahi[3 * Tp + a] - alo[3 * T + a]) + 2);
    }
  hipStream_t s = c->stream;
  // ---- edges -----------------------------------------------------------------
  const Layout &L = c->lay;
  std::vector<EdgeRec> er(g.ne);
  for (int n = 0; n < g.ne; n++) {
    EdgeRec &r = er[n];
    for (int sd = 0; sd < 2; sd++) {
      int T = g.et[2 * n + sd];
      r.tri[sd] = T;
      r.loc[sd] = g.tedge[3 * T] == n ? 0 : (g.tedge[3 * T + 1] == n ? 1 : 2);
    }
    int id = L.eidx[n];
    r.isR = L.isR[n];
    if (!r.isR) {
      r.row[0] = r.col[0] = id;
      r.row[1] = r.col[1] = L.NL + id;
      r.row[2] = r.col[2] = -1;
    } else {
      int b0 = 2 * L.NL;
      r.row[0] = r.col[0] = b0 + id;
      r.row[1] = r.col[1] = b0 + L.NR + id;
      r.row[2] = r.col[2] = b0 + 2 * L.NR + id;
    }
    r.pad = 0;
  }
  c->edges = c->mem.upload(er);
  c->rowptr = c->mem.upload(c->near.rowptr);
  c->col = c->mem.upload(c->near.col);
  c->nnz = c->near.rowptr[g.ne];
  {
    // mirrored entry of every near pair (the near list is symmetric)
    std::vector<int64_t> tp(c->nnz);
    const std::vector<int64_t> &rp = c->near.rowptr;
    const std::vector<int> &cl = c->near.col;
    for (int n = 0; n < g.ne; n++)
      for (int64_t k = rp[n]; k < rp[n + 1]; k++) {
        const int m = cl[k];
        auto b = cl.begin() + rp[m], e = cl.begin() + rp[m + 1];
        auto it = std::lower_bound(b, e, n);
        if (it == e || *it != n) return fail(c, SCABS_E_ARG, "near list is not symmetric");
        tp[k] = it - cl.begin();
      }
    c->tpos = c->mem.upload(tp);
    std::vector<uint8_t> tm(g.nt, 0);
    for (int T = 0; T < g.nt; T++)
      for (int j = 0; j < 3; j++) tm[T] |= (uint8_t)(L.isR[g.tedge[3 * T + j]] != 0);
    c->tmask = c->mem.upload(tm);
  }
  c->nnzR = 0;
  for (int n = 0; n < g.ne; n++)
    if (L.isR[n]) c->nnzR += c->near.rowptr[n + 1] - c->near.rowptr[n];
  c->qp64 = c->mem.upload(g.qp);
  {
    std::vector<TriD> all;
    make_tri_records(g, all);
    c->trid = c->mem.upload(all);
  }
  c->body_dev = c->mem.upload(g.body);
  // ---- twiddles and kernel spectra ---------------------------------------------
  std::vector<cx<double>> tw_all;
  std::vector<int> tw_off;
  std::vector<cx<double> *> ghat64;
  std::vector<cx<float> *> ghat32;
  for (const GridDesc &d : c->grids) {
    int twL = twiddle_length(d);
    tw_off.push_back((int)tw_all.size());
    for (int j = 0; j < twL; j++) {
      double a = -2.0 * PI * j / twL;
      tw_all.push_back({std::cos(a), std::sin(a)});
    }
  }
  for (size_t gi = 0; gi < c->grids.size(); gi++) {
    const GridDesc &d = c->grids[gi];
    int twL = twiddle_length(d);
    std::vector<cx<double>> tw(tw_all.begin() + tw_off[gi], tw_all.begin() + tw_off[gi] + twL);
    cx<double> *tw64 = c->mem.upload(tw);
    size_t oct = (size_t)(d.N[0] / 2 + 1) * (d.N[1] / 2 + 1) * (d.N[2] / 2 + 1);
    cx<double> *g64 = c->mem.alloc<cx<double>>(oct);
    cx<float> *g32 = c->mem.alloc<cx<float>>(oct);
    HIPCHK(build_ghat(d, c->opts.h, tw64, twL, g64, g32, s));
    ghat64.push_back(g64);
    ghat32.push_back(g32);
  }
  // ---- near-pair blocks (FP64) and the edge-pair correction --------------------
  {
    DevMem tmp;
    int64_t npairs = c->near.tptr[g.nt];
    NearSetupArgs a{};
    a.nt = g.nt;
    a.h = c->opts.h;
    a.k_e = c->k_e;
    a.k_i = c->k_i;
    a.Z_e = c->Z_e;
    a.Z_i = c->Z_i;
    a.v = c->mem.upload(g.v);
    a.t = c->mem.upload(g.t);
    a.body = c->body_dev;
    a.tedge = c->mem.upload(g.tedge);
    a.tsign = c->mem.upload(g.tsign);
    a.elen = c->mem.upload(g.elen);
    a.area = c->mem.upload(g.area);
    a.nrm = c->mem.upload(g.nrm);
    a.qp = c->qp64;
    a.qw = c->mem.upload(g.qw);
    a.sigma = c->mem.upload(L.sigma);
    a.anchor = c->mem.upload(c->anchor);
    a.u = c->mem.upload(c->u);
    a.tptr = c->mem.upload(c->near.tptr);
    a.src = c->mem.upload(c->near.src);
    a.sing = c->mem.upload(c->near.sing);
    a.D = D;
    a.tmask = c->tmask;
    cx<double> *he = c->mem.alloc<cx<double>>((size_t)(D + 1) * (D + 1) * (D + 1));
    cx<double> *hi = c->mem.alloc<cx<double>>((size_t)(D + 1) * (D + 1) * (D + 1));
    build_htab(c->k_e, c->opts.h, D, he, s);
    build_htab(c->k_i, c->opts.h, D, hi, s);
    a.htab_e = he;
    a.htab_i = hi;
    a.blocks = tmp.alloc<cx<double>>((size_t)npairs * 72);
    a.blocks_exact = tmp.alloc<cx<double>>((size_t)npairs * 72);
    launch_near_setup(a, s);
    HIPCHK(hipGetLastError());
    c->nsa = a;
    c->nsa.blocks = c->nsa.blocks_exact = nullptr;
    cx<double> *V4 = c->mem.alloc<cx<double>>(4 * (size_t)c->nnz);
    cx<double> *S4 = c->mem.alloc<cx<double>>(4 * (size_t)c->nnz);
    cx<float> *V4f = c->mem.alloc<cx<float>>(4 * (size_t)c->nnz);
    cx<float> *S4f = c->mem.alloc<cx<float>>(4 * (size_t)c->nnz);
    int64_t *cptr = tmp.upload(c->near.cptr);
    int *cpair = tmp.upload(c->near.cpair);
    uint8_t *cij = tmp.upload(c->near.cij);
    launch_near_assemble(c->nnz, cptr, cpair, cij, a.blocks, V4, S4, V4f, S4f, s);
    HIPCHK(hipGetLastError());
    if (c->opts.precond && !(c->opts.precond >= SCABS_PRECOND_PAPER && c->lay.NR == 0)) {
      cx<double> *X8 = tmp.alloc<cx<double>>(8 * (size_t)c->nnz);
      launch_exact_assemble(c->nnz, cptr, cpair, cij, a.blocks_exact, X8, s);
      HIPCHK(hipGetLastError());
      HIPCHK(sync_stream(s));
      tmp.free_one(a.blocks);
      tmp.free_one(a.blocks_exact);
      build_preconditioner(c, X8, tmp);
    }
    HIPCHK(sync_stream(s));
    tmp.release();
    // FP32 transposed product: mirrored copies of the near values, read in row order
    cx<float> *V4fT = c->mem.alloc<cx<float>>(4 * (size_t)c->nnz);
    cx<float> *S4fT = c->mem.alloc<cx<float>>(4 * (size_t)c->nnz);
    launch_mirror4(c->nnz, c->tpos, V4f, V4fT, s);
    launch_mirror4(c->nnz, c->tpos, S4f, S4fT, s);
    HIPCHK(hipGetLastError());
    build_precision<double>(c, c->p64, tw_all, tw_off, ghat64, ghat32, V4, S4, nullptr, nullptr);
    build_precision<float>(c, c->p32, tw_all, tw_off, ghat64, ghat32, V4f, S4f, V4fT, S4fT);
  }
  HIPCHK(sync_stream(s));
  c->toe = false;
  if (c->opts.product == SCABS_PRODUCT_TOEPLITZ) {
    e = build_toeplitz(c);
    if (!e.empty()) return fail(c, SCABS_E_MESH, e);
    c->toe = true;
    if (c->opts.precond >= SCABS_PRECOND_PAPER) build_circulant(c);
  }
  c->built = true;
  return SCABS_OK;
}

// ---------------------------------------------------------------------------
// products
// ---------------------------------------------------------------------------
// Grow the per-vector buffers of one precision to hold nb vectors.
template <typename T> static void ensure_batch(scabs_ctx *c, PrecState<T> &P, int nb) {
  if (nb <= P.bcap) return;
  clear_graphs(c);
  const Geometry &g = c->geo;
  c->mem.free_one(P.src);
  c->mem.free_one(P.tri_out);
  if (P.srcI) c->mem.free_one(P.srcI);
  P.src = c->mem.alloc<cx<T>>((size_t)g.ne * 3 * nb);
  P.srcI = c->mem.alloc<cx<T>>((size_t)g.ne * 3 * nb);
  P.tri_out = c->mem.alloc<cx<T>>((size_t)g.nt * 9 * nb);
  for (size_t k = 0; k < P.grids.size(); k++) {
    DevGrid<T> &G = P.grids[k];
    c->mem.free_one(G.phys);
    c->mem.free_one(G.spec);
    c->mem.free_one(P.gather[k].src);
    G.phys = c->mem.alloc<cx<T>>(8 * (size_t)G.n[0] * G.n[1] * G.n[2] * nb);
    G.spec = c->mem.alloc<cx<T>>(8 * (size_t)G.n[0] * G.N[1] * G.N[2] * nb);
    P.gather[k].src = c->mem.alloc<cx<T>>(8 * (size_t)P.gather[k].np * nb);
  }
  c->mem.free_one(P.grids_dev);
  P.grids_dev = c->mem.upload(P.grids);
  P.op.src = P.src;
  P.op.srcI = P.srcI;
  P.op.tri_out = P.tri_out;
  P.bcap = nb;
}

// lattice convolutions of all grids; in FP32 the x-line transforms of each
// grid also get a record of their own (algorithmic bytes: the physical x range
// of every transformed line read and written once)
template <typename T> static void conv_timed(scabs_ctx *c, PrecState<T> &P, int nb) {
  hipStream_t s = c->stream;
  const int off = sizeof(T) == sizeof(float) ? SCABS_STAGE_FP32_OFFSET : 0;
  StageTimer t(c, SCABS_STAGE_FFT + off);
  for (const DevGrid<T> &g : P.grids) launch_conv(g, s, nb, CONV_PLANES_FWD);
  if (sizeof(T) == sizeof(float)) {
    // one record over the grids' back-to-back launches (events between them
    // would stall the stream), counted as one launch per grid
    double bytes = 0;
    for (const DevGrid<T> &g : P.grids) bytes += 2.0 * sizeof(cx<T>) * g.n[0] * (8.0 * nb * g.N[1] * g.N[2]);
    StageTimer tx(c, SCABS_STAGE_XLINE32, bytes, (int)P.grids.size());
    for (const DevGrid<T> &g : P.grids) launch_conv(g, s, nb, CONV_XLINES);
  } else {
    for (const DevGrid<T> &g : P.grids) launch_conv(g, s, nb, CONV_XLINES);
  }
  for (const DevGrid<T> &g : P.grids) launch_conv(g, s, nb, CONV_PLANES_INV);
}

// y = A x for nb vectors (nb <= near_rows_max_batch(), within the capacity)
template <typename T> static void apply(scabs_ctx *c, PrecState<T> &P, const double *x, double *y, int nb) {
  hipStream_t s = c->stream;
  const int off = sizeof(T) == sizeof(float) ? SCABS_STAGE_FP32_OFFSET : 0;
  {
    StageTimer t(c, SCABS_STAGE_UNPACK + off);
    launch_unpack(P.op, x, s, nb);
  }
  {
    StageTimer t(c, SCABS_STAGE_PROJECT + off);
    if (sizeof(T) == sizeof(float)) {
      // point sources of every grid, then each grid's gather with a record of
      // its own (algorithmic bytes: the 8 sources of every point read once,
      // the 8 fields of every node written once)
      launch_project(P.op, P.grids, P.gather, s, nb, -2);
      double bytes = 0;
      for (size_t k = 0; k < P.grids.size(); k++) {
        const DevGrid<T> &g = P.grids[k];
        bytes += 8.0 * sizeof(cx<T>) * nb * ((double)P.gather[k].np + (double)g.n[0] * g.n[1] * g.n[2]);
      }
      StageTimer tg(c, SCABS_STAGE_GATHER32, bytes, (int)P.grids.size());
      for (size_t k = 0; k < P.grids.size(); k++) launch_project(P.op, P.grids, P.gather, s, nb, (int)k);
    } else {
      launch_project(P.op, P.grids, P.gather, s, nb);
    }
  }
  conv_timed(c, P, nb);
  {
    StageTimer t(c, SCABS_STAGE_INTERP + off);
    launch_interp_test(P.op, P.grids[0], P.grids_dev + 1, P.inv_h, s, nb);
  }
  {
    StageTimer t(c, SCABS_STAGE_NEAR + off);
    launch_near_rows(P.op, y, s, nb);
  }
}

// y = A~^T z: row weights -> lattice sources (value and gradient weights),
// the same convolution, transposed projection, then transposed near rows
template <typename T> static void apply_t(scabs_ctx *c, PrecState<T> &P, const double *z, double *y) {
  hipStream_t s = c->stream;
  const int off = sizeof(T) == sizeof(float) ? SCABS_STAGE_FP32_OFFSET : 0;
  {
    StageTimer t(c, SCABS_STAGE_UNPACK + off);
    launch_unpack_rows(P.op, z, s);
  }
  {
    StageTimer t(c, SCABS_STAGE_PROJECT + off);
    launch_test_t(P.op, P.grids, P.gather, P.src4, P.inv_h, s);
  }
  conv_timed(c, P, 1);
  {
    StageTimer t(c, SCABS_STAGE_INTERP + off);
    launch_interp_adj(P.op, P.grids[0], P.grids_dev + 1, s);
  }
  {
    StageTimer t(c, SCABS_STAGE_NEAR + off);
    launch_near_rows_t(P.op, c->tpos, y, s);
  }
}

static float *toe_part(scabs_ctx *c, float *) { return c->toe_part32; }
static double *toe_part(scabs_ctx *c, double *) { return c->toe_part64; }
static float *toe_rpart(scabs_ctx *c, float *) { return c->toe_rpart32; }
static double *toe_rpart(scabs_ctx *c, double *) { return c->toe_rpart64; }

// y = A x by the block-Toeplitz product for nb vectors: currents per edge,
// ring-axis transforms, per-frequency block products, inverse transforms,
// local and sigma terms, then the rows (sparse rows of the non-periodic
// pairs plus the periodic sums)
// the stored entries of the non-periodic pairs in the product's precision
template <typename T> static ToeRows<T> toe_rows_of(scabs_ctx *c) {
  const bool f32 = sizeof(T) == sizeof(float);
  const cx<T> *V4 = f32 ? (const cx<T> *)c->toe_V4f : (const cx<T> *)c->toe_V4;
  const cx<T> *S4 = f32 ? (const cx<T> *)c->toe_S4f : (const cx<T> *)c->toe_S4;
  ToeRows<T> R;
  R.ncap = R.nlong = c->toe_ncap;
  R.nchunk = (c->geo.ne + toe_long_chunk() - 1) / toe_long_chunk();
  R.capcol = c->toe_capcol;
  R.edge_sgn = c->toe_esgn;
  R.eflag = c->toe_eflag;
  R.V4S = V4;
  R.S4S = S4;
  R.V4L = V4 + 4 * (size_t)c->toe_nshort;
  R.S4L = S4 + 4 * (size_t)c->toe_nshort;
  R.part = toe_part(c, (T *)nullptr);
  R.rpart = toe_rpart(c, (T *)nullptr);
  R.groups = 8;
  R.sparse_form = 0;
  return R;
}

// the second stream and its events, made when a tuning first asks for the
// overlap (outside any graph capture)
static void ensure_side(scabs_ctx *c) {
  if (c->side) return;   // the stream is set last: it implies the events
  for (hipEvent_t &e : c->ev_side)
    if (!e) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  HIPCHK(hipStreamCreate(&c->side));
}

// ordering between the context stream and its second stream: 'to' waits for
// the work enqueued so far on 'from' (event k of the product's four)
static void stream_after(scabs_ctx *c, hipStream_t to, hipStream_t from, int k) {
  HIPCHK(hipEventRecord(c->ev_side[k], from));
  HIPCHK(hipStreamWaitEvent(to, c->ev_side[k], 0));
}

// y = A^T z for nb <= 8 vectors (one after another, 2N doubles each) with
// the transposed block-Toeplitz product
template <typename T>
static void apply_toe_t(scabs_ctx *c, PrecState<T> &P, ToeDev<T> &d, cx<T> *&tri_out, const double *z, double *y,
                        int nb) {
  hipStream_t s = c->stream;
  const int off = sizeof(T) == sizeof(float) ? SCABS_STAGE_FP32_OFFSET : 0;
  ensure_batch(c, P, nb);
  toe_ensure(c, d, tri_out, nb);
  DevOperator<T> op = P.op;
  op.tri_out = tri_out;
  const bool f32 = sizeof(T) == sizeof(float);
  ToeRows<T> R = toe_rows_of<T>(c);
  d.lines = toe_t_max_lines(d.P, f32);
  cx<T> *tcol = f32 ? (cx<T> *)c->toe_tcol32 : (cx<T> *)c->toe_tcol64;
  cx<T> *lcol = f32 ? (cx<T> *)c->toe_lcol32 : (cx<T> *)c->toe_lcol64;
  cx<T> *scol = f32 ? (cx<T> *)c->toe_scol32 : (cx<T> *)c->toe_scol64;
  const size_t stride = 2 * (size_t)c->lay.N;
  const bool side = c->toe_tune[nb >= 8 ? 1 : 0][3] != 0 && c->side;
  auto parts = [&](hipStream_t on, int which) {
    launch_toe_product_t(op, d, R, tcol, lcol, scol, c->toe_capidx, y, on, which, nb);
  };
  {
    StageTimer t(c, SCABS_STAGE_UNPACK + off);
    for (int v = 0; v < nb; v++) {
      DevOperator<T> ov = op;
      ov.src = op.src + (size_t)3 * op.ne * v;
      launch_unpack_rows(ov, z + v * stride, s);
    }
    // point weights are written only at periodic triangles' points (a fill
    // kernel: this sequence may be captured into a graph)
    kr_zero(d.pf, sizeof(cx<T>) * 2 * 2 * (size_t)NQ * d.nt_r * d.nr * nb, s);
  }
  // with the second stream: the short part beside the local terms and
  // forward transforms, the long part beside the inverse transforms; the
  // block products run alone
  if (side) {
    stream_after(c, c->side, s, 0);
    StageTimer t(c, SCABS_STAGE_NEAR + off, 0, 1, c->side);
    parts(c->side, TOE_SHORT);
  }
  {
    StageTimer t(c, SCABS_STAGE_FFT + off);
    parts(s, TOE_FWD);
  }
  if (side) stream_after(c, s, c->side, 1);
  {
    // every spectrum table entry read once, the row spectra (2 ne_r + 4 NQ
    // nt_r lines per vector) read and the column spectra (4 ne_r lines per
    // vector) written once
    const double spectra = (double)sizeof(cx<T>) * d.P * nb * (6.0 * d.ne_r + 4.0 * NQ * d.nt_r);
    StageTimer t(c, f32 ? SCABS_STAGE_TOEAPPLYT32 : SCABS_STAGE_TOEAPPLYT64,
                 c->toe_table_bytes[f32 ? 1 : 0] + spectra);
    parts(s, TOE_APPLY);
  }
  if (side) {
    stream_after(c, c->side, s, 2);
    {
      StageTimer t(c, SCABS_STAGE_NEAR + off, 0, 1, c->side);
      parts(c->side, TOE_LONG);
    }
    {
      StageTimer t(c, SCABS_STAGE_FFT + off);
      parts(s, TOE_INV);
    }
    stream_after(c, s, c->side, 3);
    StageTimer t(c, SCABS_STAGE_NEAR + off);
    parts(s, TOE_SUM);
  } else {
    {
      StageTimer t(c, SCABS_STAGE_FFT + off);
      parts(s, TOE_INV);
    }
    StageTimer t(c, SCABS_STAGE_NEAR + off);
    parts(s, TOE_SHORT | TOE_LONG | TOE_SUM);
  }
}

template <typename T>
static void apply_toe(scabs_ctx *c, PrecState<T> &P, ToeDev<T> &d, cx<T> *&tri_out, const double *x, double *y,
                      int nb) {
  hipStream_t s = c->stream;
  const int off = sizeof(T) == sizeof(float) ? SCABS_STAGE_FP32_OFFSET : 0;
  toe_ensure(c, d, tri_out, nb);
  DevOperator<T> op = P.op;
  op.tri_out = tri_out;
  op.edge_out = d.edge_out;
  const bool f32 = sizeof(T) == sizeof(float);
  ToeRows<T> R = toe_rows_of<T>(c);
  bool side = false;
  {
    const int *tn = c->toe_tune[nb >= 8 ? 1 : 0];
    const int lmax = toe_max_lines(d.P, f32);
    side = tn[3] != 0 && c->side;
    d.apply_form = tn[0];
    R.groups = std::max(1, std::min(tn[1], toe_row_groups()));
    R.sparse_form = tn[0];   // the 8-vector sparse rows follow the block products' form
    d.lines = tn[2] > 0 ? std::min(tn[2], lmax) : lmax;
  }
  // algorithmic bytes: per-frequency tables, stored sparse entries, the
  // spectra (input 4 ne_r, output 2 ne_r + 4 NQ nt_r lines per vector)
  const double el = sizeof(cx<T>);
  const double spectra = el * d.P * nb * (4.0 * d.ne_r + 2.0 * d.ne_r + 4.0 * NQ * d.nt_r);
  const double tables = c->toe_table_bytes[f32 ? 1 : 0], sparse = c->toe_sparse_bytes[f32 ? 1 : 0];
  const double vectors = 2.0 * 16.0 * c->lay.N * nb;
  StageTimer whole(c, f32 ? SCABS_STAGE_TOEPRODUCT32 : SCABS_STAGE_TOEPRODUCT64, tables + sparse + vectors + 2 * spectra);
  {
    StageTimer t(c, SCABS_STAGE_UNPACK + off);
    launch_unpack(op, x, s, nb);
  }
  // with the second stream: the stored entries' short part beside the
  // forward transforms, the long part beside the inverse transforms and the
  // local terms; the block products run alone
  if (side) {
    stream_after(c, c->side, s, 0);
    StageTimer t(c, SCABS_STAGE_NEAR + off, 0, 1, c->side);
    launch_toe_rows(op, R, y, c->side, nb, TOE_SHORT);
  }
  {
    StageTimer t(c, SCABS_STAGE_FFT + off);
    launch_toe_product(op, d, s, nb, TOE_FWD);
  }
  if (side) stream_after(c, s, c->side, 1);
  {
    // the per-frequency block products: every spectrum table entry read
    // once, the input spectra read and the output spectra written once
    StageTimer ta(c, f32 ? SCABS_STAGE_TOEAPPLY32 : SCABS_STAGE_TOEAPPLY64, tables + spectra);
    launch_toe_product(op, d, s, nb, TOE_APPLY);
  }
  if (side) {
    stream_after(c, c->side, s, 2);
    StageTimer t(c, SCABS_STAGE_NEAR + off, 0, 1, c->side);
    launch_toe_rows(op, R, y, c->side, nb, TOE_LONG);
  }
  {
    StageTimer t(c, SCABS_STAGE_FFT + off);
    launch_toe_product(op, d, s, nb, TOE_INV);
  }
  if (side) stream_after(c, s, c->side, 3);
  {
    StageTimer t(c, SCABS_STAGE_NEAR + off);
    launch_toe_rows(op, R, y, s, nb, side ? TOE_SUM : TOE_ALL);
  }
}

// nb products (vectors stored one after another, 2N doubles each)
static void matvec_n(scabs_ctx *c, const double *x, double *y, int nb, int prec, bool trans = false) {
  const size_t stride = 2 * (size_t)c->lay.N;
  if (trans && c->toe) {
    for (int k0 = 0; k0 < nb; k0 += 8) {
      const int m = std::min(8, nb - k0);
      if (prec == SCABS_FP32)
        apply_toe_t(c, c->p32, c->t32, c->toe_tri32, x + k0 * stride, y + k0 * stride, m);
      else
        apply_toe_t(c, c->p64, c->t64, c->toe_tri64, x + k0 * stride, y + k0 * stride, m);
    }
    return;
  }
  if (trans) {
    for (int k = 0; k < nb; k++) {
      if (prec == SCABS_FP32) {
        apply_t(c, c->p32, x + k * stride, y + k * stride);
      } else {
        apply_t(c, c->p64, x + k * stride, y + k * stride);
      }
    }
    return;
  }
  const int B = near_rows_max_batch();
  for (int k0 = 0; k0 < nb; k0 += B) {
    const int m = std::min(B, nb - k0);
    if (c->toe) {
      if (prec == SCABS_FP32) {
        ensure_batch(c, c->p32, m);
        apply_toe(c, c->p32, c->t32, c->toe_tri32, x + k0 * stride, y + k0 * stride, m);
      } else {
        ensure_batch(c, c->p64, m);
        apply_toe(c, c->p64, c->t64, c->toe_tri64, x + k0 * stride, y + k0 * stride, m);
      }
      continue;
    }
    if (prec == SCABS_FP32) {
      ensure_batch(c, c->p32, m);
      apply(c, c->p32, x + k0 * stride, y + k0 * stride, m);
    } else {
      ensure_batch(c, c->p64, m);
      apply(c, c->p64, x + k0 * stride, y + k0 * stride, m);
    }
  }
}

// prec: precision of the products the preconditioner feeds (FP32 inner solves
// use the batched single-precision apply)
// x: nb vectors of N, FP64, or FP32 (the inner solves' basis, read directly
// by the gathers of the FP32 apply and of the transposed apply)
template <typename TI>
static void apply_schwarz_n(scabs_ctx *c, const cx<TI> *x, cx<double> *y, int nb, bool trans, int prec);

// paper mode, A_LL part: rows of the sigma-free periodic edges from the
// inverse circulant (FP32 tables for the FP32 inner solves), the other L rows
// copied; written after the block-diagonal part, which leaves them alone
// (forward) or zero (transposed)
template <typename TI>
static void apply_circ_n(scabs_ctx *c, const cx<TI> *x, cx<double> *y, int nb, bool trans, int prec) {
  const int64_t N = c->lay.N;
  StageTimer tm(c, trans ? SCABS_STAGE_PRECOND_T : SCABS_STAGE_PRECOND);
  for (int b0 = 0; b0 < nb; b0 += 8) {
    const int m = std::min(8, nb - b0);
    if (prec == SCABS_FP32)
      launch_pc_circ_apply<TI, float>(c->t32, c->edges, c->pc_T32, x + b0 * N, N, m, trans, c->pc_cX32, c->pc_cY32,
                                      y + b0 * N, c->geo.ne, c->stream);
    else
      launch_pc_circ_apply<TI, double>(c->t64, c->edges, c->pc_T64, x + b0 * N, N, m, trans, c->pc_cX64,
                                       c->pc_cY64, y + b0 * N, c->geo.ne, c->stream);
  }
}

template <typename TI>
static void apply_precond_n(scabs_ctx *c, const cx<TI> *x, cx<double> *y, int nb, bool trans, int prec) {
  if (c->pc_schwarz) apply_schwarz_n(c, x, y, nb, trans, prec);
  if (c->pc_circ) apply_circ_n(c, x, y, nb, trans, prec);
}

template <typename TI>
static void apply_schwarz_n(scabs_ctx *c, const cx<TI> *x, cx<double> *y, int nb, bool trans, int prec) {
  const size_t N = (size_t)c->lay.N;
  if (!trans && prec == SCABS_FP32) {
    const int B = precond_apply32_max_batch();
    for (int b0 = 0; b0 < nb; b0 += B) {
      const int m = std::min(B, nb - b0);
      {
        // per ext entry its index and column scale, m inputs read and m FP32
        // copies written
        StageTimer tm(c, SCABS_STAGE_PCGATHER32, (8.0 + (2.0 * sizeof(TI) + 8.0) * m) * (double)c->pc_n_ext);
        launch_precond_gather32(c->pc_n_ext, c->pc_ext_slot, c->pc_Rs, x + b0 * N, (int64_t)N, m, c->pc_xe,
                                c->stream);
      }
      // coefficients once (4 B); per ext entry the m FP32 gathered inputs;
      // per unknown its index and m FP64 outputs
      const double bytes =
          4.0 * (double)c->pc_coef + 8.0 * m * (double)c->pc_n_ext + (4.0 + 16.0 * m) * (double)c->lay.N;
      StageTimer tm(c, SCABS_STAGE_PRECOND, bytes);
      launch_precond_apply32(c->pc_n_items32, c->pc_items32, c->pc_ext_ptr, c->pc_core_ptr, c->pc_core_slot, c->pc_r_off,
                             c->pc_Rt, c->pc_xe, y + b0 * N, (int64_t)N, m, c->stream);
    }
    return;
  }
  if constexpr (std::is_same<TI, double>::value) {
    for (int k = 0; k < nb; k++) apply_precond(c, x + k * N, y + k * N, trans);
  } else {
    if (!trans) throw std::string("the FP64 Schwarz apply takes FP64 inputs");
    for (int k = 0; k < nb; k++) {
      StageTimer tm(c, SCABS_STAGE_PRECOND_T);
      launch_precond_apply_t<TI>(c->pc_n_t_items, c->pc_t_items, c->lay.N, c->pc_n_core, c->pc_ext_ptr, c->pc_core_ptr,
                                 c->pc_core_slot, c->pc_r_off, PcStore{c->pc_Rt, c->pc_Rs}, c->pc_inv_ptr,
                                 c->pc_inv_pos, c->pc_tmp, c->pc_xc, x + k * N, y + k * N, c->stream);
    }
  }
}

// Read back the norms and the first `rows` entries of every Hessenberg column
// block (2 nb blocks of `stride` entries) into the mapped host copy and wait
// for them: the publishing kernel sets the host flag to a new sequence
// number after its stores.  The host spins on the flag; nothing is enqueued
// behind the publishing kernel before the flag is seen, so an idle stream
// without the flag (or a stream error) ends the wait with an error.
static void read_back(scabs_ctx *c, hipStream_t s, size_t nnrm, int nb, int stride, int rows) {
  const unsigned seq = ++c->hseq;
  kr_publish(c->hblock, c->hpin_dev, (int)nnrm, 2 * nb, stride, rows, c->hflag_dev, seq, s);
  const volatile unsigned *f = c->hflag;
  for (unsigned spin = 1;; spin++) {
    if (*f == seq) break;
    if ((spin & 16383) == 0) {
      // a liveness check only: while another thread of a batched solve
      // captures its graph the runtime may refuse the query, which is asked
      // again later
      const hipError_t e = hipStreamQuery(s);
      if (e == hipSuccess) {
        if (*f == seq) break;
        throw HipError{hipErrorLaunchFailure, "Arnoldi read-back: the stream finished without setting the host flag"};
      }
      if (e == hipErrorStreamCaptureUnsupported || e == hipErrorStreamCaptureImplicit) {
        (void)hipGetLastError();
        hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s, &st) != hipSuccess || st != hipStreamCaptureStatusNone)
          throw HipError{e, "Arnoldi read-back on a capturing stream"};
        continue;
      }
      if (e != hipErrorNotReady) throw HipError{e, "hipStreamQuery"};
    }
  }
  std::atomic_thread_fence(std::memory_order_acquire);
}

// complex entries in front of the Hessenberg columns that hold the norms
// (2 nb + 4 doubles for nb <= KR_MAX_SYSTEMS)
constexpr size_t KR_NRM = KR_MAX_SYSTEMS + 2;
static void ensure_work(scabs_ctx *c, int restart, int nb) {
  int64_t N = c->lay.N;
  if (c->work_restart >= restart && c->work_N == N && c->work_nb >= nb) return;
  clear_graphs(c);
  c->work.release();
  c->w = c->work.alloc<cx<double>>(N * nb);
  c->r = c->work.alloc<cx<double>>(N * nb);
  c->d = c->work.alloc<cx<double>>(N * nb);
  c->z = c->work.alloc<cx<double>>(N * nb);
  c->t = c->work.alloc<cx<double>>(N * nb);
  c->gstage = c->work.alloc<cx<double>>(N * nb);
  const size_t hentries = KR_NRM + 2 * (size_t)(restart + 2) * nb;
  c->hblock = c->work.alloc<cx<double>>(hentries);
  c->nrm = reinterpret_cast<double *>(c->hblock);
  c->hcol = c->hblock + KR_NRM;
  if (c->hpin) HIPCHK(hipHostFree(c->hpin));
  c->hpin = nullptr;
  HIPCHK(hipHostMalloc((void **)&c->hpin, sizeof(cx<double>) * hentries, hipHostMallocMapped | hipHostMallocCoherent));
  HIPCHK(hipHostGetDevicePointer((void **)&c->hpin_dev, c->hpin, 0));
  c->hpin_entries = hentries;
  if (!c->hflag) {
    HIPCHK(hipHostMalloc((void **)&c->hflag, 64, hipHostMallocMapped | hipHostMallocCoherent));
    HIPCHK(hipHostGetDevicePointer((void **)&c->hflag_dev, c->hflag, 0));
    *(volatile unsigned *)c->hflag = 0;
    c->hseq = 0;
  }
  c->part = c->work.alloc<cx<double>>(std::max((size_t)256 * (restart + 2), kr_ortho_part_entries(restart + 1, nb)));
  c->npart = c->work.alloc<double>(kr_ortho_npart_entries(N, nb));
  c->nrm_part = c->work.alloc<double>(1024);
  c->flag = c->work.alloc<int>(1);
  c->work_restart = restart;
  c->work_N = N;
  c->work_nb = nb;
}

// norms of nb vectors (one synchronisation)
static void dev_norms(scabs_ctx *c, const cx<double> *v, int nb, double *out) {
  const int64_t N = c->lay.N;
  for (int b = 0; b < nb; b++) kr_norm(v + b * N, N, c->nrm_part, c->nrm + b, c->stream);
  HIPCHK(hipMemcpyAsync(out, c->nrm, sizeof(double) * nb, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(sync_stream(c->stream));
}

struct GmresResult {
  int iters = 0;
  double rel = 1.0;      // true relative residual w.r.t. the operator used
  bool converged = false;
};

// Solve A sol_b = rhs_b (b < nb, vectors one after another) from sol = 0 to
// ||rhs_b - A sol_b|| <= tol[b] ||rhs_b||.
// the Krylov basis of restart + 1 vectors for nb systems, in FP64 or FP32
static cx<double> *basis(scabs_ctx *c, int restart, int nb, cx<double> *) {
  const int64_t need = (int64_t)(restart + 1) * c->lay.N * nb;
  if (c->cap_V64 < need) {
    c->workV64.release();
    c->V64 = c->workV64.alloc<cx<double>>((size_t)need);
    c->cap_V64 = need;
  }
  return c->V64;
}
static cx<float> *basis(scabs_ctx *c, int restart, int nb, cx<float> *) {
  const int64_t need = (int64_t)(restart + 1) * c->lay.N * nb;
  if (c->cap_V32 < need) {
    c->workV32.release();
    c->V32 = c->workV32.alloc<cx<float>>((size_t)need);
    c->cap_V32 = need;
  }
  return c->V32;
}
// FP64 view of nb basis vectors for the operator (FP32 ones widened into t)
static const cx<double> *operator_input(scabs_ctx *c, const cx<double> *v, int64_t n) {
  (void)c;
  (void)n;
  return v;
}
static const cx<double> *operator_input(scabs_ctx *c, const cx<float> *v, int64_t n) {
  kr_widen(v, c->t, n, c->stream);
  return c->t;
}

// w = A M v for the nb basis vectors at v (the launches of one Arnoldi step
// between its host synchronisations)
template <typename VT>
static void step_sequence(scabs_ctx *c, const cx<VT> *v, int nb, int prec, bool trans) {
  if (c->has_pc) {
    // the preconditioner's gathers read the basis vectors in their own
    // precision (no widened copy)
    apply_precond_n(c, v, c->z, nb, trans, prec);
    matvec_n(c, (const double *)c->z, (double *)c->w, nb, prec, trans);
  } else {
    const cx<double> *vj = operator_input(c, v, (int64_t)c->lay.N * nb);
    matvec_n(c, (const double *)vj, (double *)c->w, nb, prec, trans);
  }
}

// The step sequence from a HIP graph: the basis vectors are copied into the
// staging buffer the graph reads, then the graph replays the launches.  The
// first use of a shape runs the sequence eagerly (it grows any per-vector
// buffers), then captures it (thread-local mode: other threads of a batched
// solve keep launching).  Not while stage profiling records events.
template <typename VT>
static void step_product(scabs_ctx *c, const cx<VT> *v, int nb, int prec, bool trans) {
  if (!c->graphs_on || c->prof_on) {
    step_sequence(c, v, nb, prec, trans);
    return;
  }
  hipStream_t s = c->stream;
  const int vt = sizeof(VT) == sizeof(float);
  const scabs_ctx::StepGraph *hit = nullptr;
  for (const auto &g : c->step_graphs)
    if (g.nb == nb && g.prec == prec && g.vt == vt && g.trans == (int)trans) hit = &g;
  if (hit && !hit->exec) {   // this shape could not be captured: launches as usual
    step_sequence(c, v, nb, prec, trans);
    return;
  }
  cx<VT> *stage = reinterpret_cast<cx<VT> *>(c->gstage);
  HIPCHK(hipMemcpyAsync(stage, v, sizeof(cx<VT>) * (size_t)c->lay.N * nb, hipMemcpyDeviceToDevice, s));
  if (hit) {
    HIPCHK(hipGraphLaunch(hit->exec, s));
    return;
  }
  step_sequence(c, (const cx<VT> *)stage, nb, prec, trans);   // this step's product, eagerly
  // capture: nothing runs while the stream records, so a failure here can
  // only be the capture's; the shape then keeps the ordinary launches
  hipGraphExec_t exec = nullptr;
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess) {
    bool ok = true;
    try {
      step_sequence(c, (const cx<VT> *)stage, nb, prec, trans);
    } catch (...) {
      ok = false;
    }
    hipGraph_t graph = nullptr;
    ok = hipStreamEndCapture(s, &graph) == hipSuccess && ok && graph;
    if (ok && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) exec = nullptr;
    if (graph) (void)hipGraphDestroy(graph);
  }
  if (!exec) (void)hipGetLastError();
  c->step_graphs.push_back({exec, nb, prec, vt, (int)trans});
}

// ---------------------------------------------------------------------------
// GMRES on a batch of right-hand sides (restarted; classical Gram-Schmidt
// with a second pass where the first lost more than 1 - 1/sqrt(2) of the
// vector's norm, Givens rotations; sums and rotations in FP64, the basis
// stored in FP64, or in FP32 for the single-precision inner solves, whose
// tolerance is 1e-5 or looser and whose correction an FP64 residual checks).  The nb systems step
// together: one batched preconditioner + product per Arnoldi step,
// per-system orthogonalisation, one host synchronisation per step for all of
// them (two when a system needs the second pass).
template <typename VT>
static void gmres_batch(scabs_ctx *c, int nb, const cx<double> *rhs, cx<double> *sol, int prec, const double *tol,
                        int max_iter, int restart, std::vector<int> &nmv, bool trans, std::vector<GmresResult> &res) {
  typedef std::complex<double> zd;
  hipStream_t s = c->stream;
  const int64_t N = c->lay.N;
  const int m = restart;
  cx<VT> *const V = basis(c, restart, nb, (cx<VT> *)nullptr);
  const int64_t ldv = N * nb;   // V[j][b] at V + (j nb + b) N
  res.assign(nb, GmresResult());
  nmv.assign(nb, 0);
  HIPCHK(hipMemsetAsync(sol, 0, sizeof(cx<double>) * N * nb, s));
  HIPCHK(hipMemcpyAsync(c->r, rhs, sizeof(cx<double>) * N * nb, hipMemcpyDeviceToDevice, s));
  std::vector<double> bn(nb), beta(nb), hn(2 * nb);
  std::vector<int> reo2(nb, 0);
  dev_norms(c, rhs, nb, bn.data());
  beta = bn;
  std::vector<std::vector<zd>> H(nb, std::vector<zd>((size_t)(m + 1) * m)), g(nb, std::vector<zd>(m + 1)),
      cs(nb, std::vector<zd>(m)), sn(nb, std::vector<zd>(m));
  std::vector<int> jb(nb);
  // Hessenberg columns of the running step (both passes), read in place in
  // the mapped host copy of the device block: system b's at hb + 2 (m + 2) b
  const cx<double> *const hb = c->hpin + KR_NRM;
  while (true) {
    std::vector<int> act;
    for (int b = 0; b < nb; b++) {
      res[b].rel = bn[b] > 0 ? beta[b] / bn[b] : 0.0;
      if (res[b].rel <= tol[b]) {
        res[b].converged = true;
        continue;
      }
      if (res[b].iters < max_iter) act.push_back(b);
    }
    if (act.empty()) break;
    for (int b : act) {
      kr_norm(c->r + b * N, N, c->nrm_part, c->nrm + b, s);
      kr_scale(V + b * N, c->r + b * N, c->nrm + b, N, s);
      std::fill(g[b].begin(), g[b].end(), zd(0));
      g[b][0] = beta[b];
      jb[b] = 0;
    }
    std::vector<int> run = act;
    int j = 0;
    // w = A M v_j for every vector of the batch (the batched stages take all
    // nb vectors; only the orthogonalisation is restricted to running systems)
    auto enqueue_product = [&](int jj) { step_product(c, V + (size_t)jj * ldv, nb, prec, trans); };
    // the product of step j is already in the stream (enqueued during step
    // j - 1, before the host's Givens update; unused if the cycle ends there)
    bool pending = false;
    while (j < m && !run.empty()) {
      if (!pending) enqueue_product(j);
      pending = false;
      for (int b : run) nmv[b]++;
      // classical Gram-Schmidt, repeated only where it lost too much of w
      // (Daniel-Gragg-Kaufman-Stewart test ||w1|| < ||w|| / sqrt(2)); one
      // set of launches for all running systems
      const int64_t hstride = 2 * (int64_t)(m + 2);
      auto to_run = [](const std::vector<int> &v) {
        KrRun r{};
        r.n = (int)v.size();
        for (size_t i = 0; i < v.size(); i++) r.b[i] = v[i];
        return r;
      };
      {
        StageTimer tm(c, SCABS_STAGE_ORTHO);
        kr_ortho_pass(V, ldv, j + 1, c->w, N, to_run(run), 1, c->part, c->npart, c->hcol, hstride, 0, c->nrm + nb,
                      c->nrm, s);
      }
      // v_{j+1} = w / ||w|| before the read-back (redone below for systems
      // that take a second pass)
      kr_scale_run(V + (size_t)(j + 1) * ldv, c->w, c->nrm, N, to_run(run), s);
      // norms and Hessenberg columns written into mapped host memory by one
      // kernel, waited for by spinning on its flag (a blocking wait wakes the
      // host up later, a copy adds a blit and its own latency)
      read_back(c, s, KR_NRM, nb, m + 2, j + 1);
      std::copy((const double *)c->hpin, (const double *)c->hpin + 2 * nb, hn.begin());
      std::vector<int> reo;
      for (int b : run) {
        reo2[b] = 0;
        if (hn[b] < 0.7071067811865476 * hn[nb + b]) reo.push_back(b);
      }
      if (!reo.empty()) {
        {
          StageTimer tm(c, SCABS_STAGE_ORTHO);
          kr_ortho_pass(V, ldv, j + 1, c->w, N, to_run(reo), 0, c->part, c->npart, c->hcol, hstride, m + 2,
                        c->nrm + nb, c->nrm, s);
        }
        for (int b : reo) reo2[b] = 1;
        // the block again: the second pass's columns beside the unchanged first ones
        read_back(c, s, KR_NRM, nb, m + 2, j + 1);
        std::copy((const double *)c->hpin, (const double *)c->hpin + nb, hn.begin());
        kr_scale_run(V + (size_t)(j + 1) * ldv, c->w, c->nrm, N, to_run(reo), s);
      }
      // the next step's product goes into the stream now, so the GPU works
      // while the host updates the rotations
      if (j + 1 < m) {
        enqueue_product(j + 1);
        pending = true;
      }
      std::vector<int> next;
      for (int b : run) {
        const cx<double> *h1 = hb + 2 * (size_t)(m + 2) * b, *h2 = h1 + (m + 2);
        zd *col = &H[b][(size_t)j * (m + 1)];
        for (int i = 0; i <= j; i++)
          col[i] = reo2[b] ? zd(h1[i].x + h2[i].x, h1[i].y + h2[i].y) : zd(h1[i].x, h1[i].y);
        col[j + 1] = hn[b];
        for (int i = 0; i < j; i++) {
          zd a = col[i], bb = col[i + 1];
          col[i] = cs[b][i] * a + sn[b][i] * bb;
          col[i + 1] = -std::conj(sn[b][i]) * a + cs[b][i] * bb;
        }
        double an = std::abs(col[j]), bnrm = std::abs(col[j + 1]);
        if (bnrm == 0) {
          cs[b][j] = 1;
          sn[b][j] = 0;
        } else if (an == 0) {
          cs[b][j] = 0;
          sn[b][j] = std::conj(col[j + 1]) / bnrm;
        } else {
          double t = std::hypot(an, bnrm);
          cs[b][j] = an / t;
          sn[b][j] = (col[j] / an) * std::conj(col[j + 1]) / t;
        }
        col[j] = cs[b][j] * col[j] + sn[b][j] * col[j + 1];
        col[j + 1] = 0;
        g[b][j + 1] = -std::conj(sn[b][j]) * g[b][j];
        g[b][j] = cs[b][j] * g[b][j];
        jb[b] = j + 1;
        res[b].iters++;
        const bool done = std::abs(g[b][j + 1]) <= tol[b] * bn[b] || hn[b] == 0 || res[b].iters >= max_iter;
        if (!done) next.push_back(b);
      }
      run.swap(next);
      j++;
    }
    // y = H^-1 g (upper triangular); sol += M (V y)
    HIPCHK(hipMemsetAsync(c->t, 0, sizeof(cx<double>) * N * nb, s));
    for (int b : act) {
      const int jj = jb[b];
      std::vector<zd> y(jj);
      for (int i = jj - 1; i >= 0; i--) {
        zd acc = g[b][i];
        for (int k = i + 1; k < jj; k++) acc -= H[b][(size_t)k * (m + 1) + i] * y[k];
        y[i] = acc / H[b][(size_t)i * (m + 1) + i];
      }
      std::vector<cx<double>> yb(jj);
      for (int i = 0; i < jj; i++) yb[i] = {y[i].real(), y[i].imag()};
      cx<double> *h1 = c->hcol + 2 * (size_t)(m + 2) * b;
      HIPCHK(hipMemcpyAsync(h1, yb.data(), sizeof(cx<double>) * jj, hipMemcpyHostToDevice, s));
      kr_update(c->t + b * N, V + b * N, ldv, jj, h1, N, +1.0, s);
      // the host vector yb must outlive the copy
      HIPCHK(sync_stream(s));
    }
    if (c->has_pc) {
      apply_precond_n(c, c->t, c->z, nb, trans, prec);
      for (int b : act) kr_axpy(sol + b * N, c->z + b * N, N, s);
    } else {
      for (int b : act) kr_axpy(sol + b * N, c->t + b * N, N, s);
    }
    // true residuals
    matvec_n(c, (const double *)sol, (double *)c->w, nb, prec, trans);
    for (int b : act) nmv[b]++;
    for (int b : act) {
      HIPCHK(hipMemcpyAsync(c->r + b * N, rhs + b * N, sizeof(cx<double>) * N, hipMemcpyDeviceToDevice, s));
      kr_residual((const cx<double> *)(c->r + b * N), c->w + b * N, N, s);   // w = rhs - A sol
      HIPCHK(hipMemcpyAsync(c->r + b * N, c->w + b * N, sizeof(cx<double>) * N, hipMemcpyDeviceToDevice, s));
    }
    std::vector<double> nr(nb);
    dev_norms(c, c->r, nb, nr.data());
    for (int b : act) beta[b] = nr[b];
  }
}

// FP64 iterative refinement around batched GMRES on the operator of the inner
// precision; nb right-hand sides (vectors one after another).
static int solve_batch(scabs_ctx *c, int nb, const cx<double> *b, cx<double> *x, double tol, int max_iter,
                       int restart, int mode, scabs_solve_info *info, bool trans) {
  hipStream_t s = c->stream;
  const int64_t N = c->lay.N;
  ensure_work(c, restart, nb);
  std::vector<scabs_solve_info> loc(nb);
  const int inner_prec = mode == SCABS_MIXED ? SCABS_FP32 : SCABS_FP64;
  const double floor_tol = mode == SCABS_MIXED ? 1e-5 : 1e-14;
  std::vector<double> bn(nb), rn(nb), rel(nb, 1.0);
  dev_norms(c, b, nb, bn.data());
  DevMem tmp;
  cx<double> *rr = tmp.alloc<cx<double>>(N * nb);     // residuals
  cx<double> *rhs = tmp.alloc<cx<double>>(N * nb);    // compacted residuals of the active systems
  cx<double> *corr = tmp.alloc<cx<double>>(N * nb);
  std::vector<int> status(nb, SCABS_E_NOCONV), stalled(nb, 0);
  for (int outer = 0; outer < 50; outer++) {
    matvec_n(c, (const double *)x, (double *)rr, nb, SCABS_FP64, trans);
    for (int k = 0; k < nb; k++) kr_residual(b + k * N, rr + k * N, N, s);   // rr = b - A x
    dev_norms(c, rr, nb, rn.data());
    std::vector<int> act;
    for (int k = 0; k < nb; k++) {
      loc[k].matvecs64 += status[k] == SCABS_E_NOCONV && !stalled[k] ? 1 : 0;
      if (status[k] == SCABS_OK || stalled[k]) continue;
      rel[k] = bn[k] > 0 ? rn[k] / bn[k] : 0.0;
      if (rel[k] <= tol) {
        status[k] = SCABS_OK;
        continue;
      }
      if (loc[k].inner_iters >= max_iter) continue;
      act.push_back(k);
    }
    if (act.empty()) break;
    const int na = (int)act.size();
    std::vector<double> tin(na);
    int min_left = max_iter;
    for (int a = 0; a < na; a++) {
      const int k = act[a];
      tin[a] = std::max(0.5 * tol / rel[k], floor_tol);
      min_left = std::min(min_left, max_iter - loc[k].inner_iters);
      HIPCHK(hipMemcpyAsync(rhs + a * N, rr + k * N, sizeof(cx<double>) * N, hipMemcpyDeviceToDevice, s));
    }
    std::vector<int> nmv;
    std::vector<GmresResult> g;
    if (inner_prec == SCABS_FP32)
      gmres_batch<float>(c, na, rhs, corr, inner_prec, tin.data(), min_left, restart, nmv, trans, g);
    else
      gmres_batch<double>(c, na, rhs, corr, inner_prec, tin.data(), min_left, restart, nmv, trans, g);
    for (int a = 0; a < na; a++) {
      const int k = act[a];
      if (inner_prec == SCABS_FP32)
        loc[k].matvecs32 += nmv[a];
      else
        loc[k].matvecs64 += nmv[a];
      loc[k].inner_iters += g[a].iters;
      loc[k].outer_iters++;
      kr_axpy(x + k * N, corr + a * N, N, s);
      if (g[a].iters == 0 && !g[a].converged) stalled[k] = 1;
    }
  }
  HIPCHK(sync_stream(s));
  tmp.release();
  int worst = SCABS_OK;
  for (int k = 0; k < nb; k++) {
    loc[k].rel_residual = rel[k];
    loc[k].status = status[k];
    if (info) info[k] = loc[k];
    if (status[k] != SCABS_OK) worst = status[k];
  }
  return worst;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int scabs_create(scabs_ctx **out, const scabs_opts *o) {
  if (!out || !o) return SCABS_E_ARG;
  *out = nullptr;
  if (!(o->h > 0) || !(o->r_near > 0)) return SCABS_E_ARG;
  std::unique_ptr<scabs_ctx> c(new scabs_ctx());
  c->opts = *o;
  if (!(c->opts.kappa_s > 0)) c->opts.kappa_s = 1.37;
  if (hipSetDevice(o->device) != hipSuccess) return SCABS_E_HIP;
  if (scratch_address(o->device, &c->noalloc_pts) != hipSuccess) return SCABS_E_HIP;
  if (o->stream) {
    c->stream = (hipStream_t)o->stream;
  } else {
    if (hipStreamCreate(&c->stream) != hipSuccess) return SCABS_E_HIP;
    c->own_stream = true;
  }
  *out = c.release();
  return SCABS_OK;
}

int scabs_set_mesh(scabs_ctx *c, const double *verts, int64_t nv, const int32_t *tris, int64_t nt,
                   const int32_t *body) {
  if (!c) return SCABS_E_ARG;
  if (!verts || !tris || nv <= 0 || nt <= 0 || nt > (1 << 27)) return fail(c, SCABS_E_ARG, "bad mesh arguments");
  c->verts.assign(verts, verts + 3 * nv);
  c->tris.assign(tris, tris + 3 * nt);
  if (body)
    c->body.assign(body, body + nt);
  else
    c->body.assign(nt, 0);
  c->built = false;
  return SCABS_OK;
}

int scabs_set_media(scabs_ctx *c, double omega, double eps_out, double eps_in) {
  if (!c) return SCABS_E_ARG;
  if (!(omega > 0) || !(eps_out > 0) || !(eps_in > 0)) return fail(c, SCABS_E_ARG, "media must be positive");
  c->omega = omega;
  c->eps_out = eps_out;
  c->eps_in = eps_in;
  c->built = false;
  return SCABS_OK;
}

int scabs_sigma_clear(scabs_ctx *c) {
  if (!c) return SCABS_E_ARG;
  c->ends.clear();
  c->built = false;
  return SCABS_OK;
}

int scabs_sigma_add_monomial(scabs_ctx *c, int axis, double x0, double length, int dir, int degree,
                             double sigma0) {
  if (!c) return SCABS_E_ARG;
  if (axis < 0 || axis > 2 || !(length > 0) || (dir != 1 && dir != -1) || degree < 0 || !(sigma0 >= 0))
    return fail(c, SCABS_E_ARG, "bad absorber profile");
  SigmaEnd e{axis, dir, degree, x0, length, sigma0, {}};
  c->ends.push_back(e);
  c->built = false;
  return SCABS_OK;
}

int scabs_sigma_add_pwl(scabs_ctx *c, int axis, double x0, double length, int dir, int n, const double *ctrl) {
  if (!c) return SCABS_E_ARG;
  if (axis < 0 || axis > 2 || !(length > 0) || (dir != 1 && dir != -1) || n < 2 || !ctrl)
    return fail(c, SCABS_E_ARG, "bad absorber profile");
  for (int k = 0; k < n; k++)
    if (!(ctrl[k] >= 0)) return fail(c, SCABS_E_ARG, "conductivity control values must be >= 0");
  SigmaEnd e{axis, dir, 1, x0, length, 1.0, std::vector<double>(ctrl, ctrl + n)};
  c->ends.push_back(e);
  c->built = false;
  return SCABS_OK;
}

int scabs_set_sigma_points(scabs_ctx *c, const double *sigma_q, int64_t nq) {
  if (!c) return SCABS_E_ARG;
  if (!sigma_q || nq != (int64_t)(c->tris.size() / 3) * NQ)
    return fail(c, SCABS_E_ARG, "scabs_set_sigma_points needs 7 values per triangle of the mesh set before");
  for (int64_t i = 0; i < nq; i++)
    if (!(sigma_q[i] >= 0)) return fail(c, SCABS_E_ARG, "conductivity values must be >= 0");
  for (size_t k = 0; k < c->ends.size(); k++)
    if (!c->ends[k].pts.empty()) {
      c->ends.erase(c->ends.begin() + k);
      break;
    }
  SigmaEnd e{0, 1, 0, 0.0, 1.0, 0.0, {}, std::vector<double>(sigma_q, sigma_q + nq)};
  c->ends.push_back(e);
  c->built = false;
  return SCABS_OK;
}

int scabs_build(scabs_ctx *c) {
  if (!c) return SCABS_E_ARG;
  try {
    HIPCHK(hipSetDevice(c->opts.device));
    return do_build(c);
  } catch (const HipError &e) {
    c->mem.release();
    if (e.e == hipErrorOutOfMemory) return fail(c, SCABS_E_OOM, "device allocation failed");
    return hip_fail(c, e);
  } catch (const std::string &m) {
    c->mem.release();
    return fail(c, SCABS_E_ARG, m);
  } catch (const std::bad_alloc &) {
    c->mem.release();
    return fail(c, SCABS_E_OOM, "host allocation failed");
  }
}

int scabs_info(const scabs_ctx *c, scabs_info_t *info) {
  if (!c || !info) return SCABS_E_ARG;
  if (!c->built) return SCABS_E_STATE;
  memset(info, 0, sizeof(*info));
  info->N = c->lay.N;
  info->NL = c->lay.NL;
  info->NR = c->lay.NR;
  info->n_edges = c->geo.ne;
  info->n_tris = c->geo.nt;
  info->n_points = (int64_t)c->geo.nt * NQ;
  info->n_bodies = c->geo.nbody;
  info->n_near_pairs = c->near.tptr[c->geo.nt];
  info->nnz_near = c->nnz;
  for (int a = 0; a < 3; a++) {
    info->grid_phys[a] = c->grids[0].n[a];
    info->grid_fft[a] = c->grids[0].N[a];
  }
  info->nnz_near_r = c->nnzR;
  info->n_clusters = c->pc_schwarz ? c->cl.nc : 0;
  info->precond_entries = 0;
  if (c->pc_schwarz)
    for (int k = 0; k < c->cl.nc; k++)
      info->precond_entries += (c->cl.ext_ptr[k + 1] - c->cl.ext_ptr[k]) * (c->cl.core_ptr[k + 1] - c->cl.core_ptr[k]);
  info->device_bytes = (int64_t)(c->mem.bytes + c->work.bytes);
  info->precond_ext_entries = c->pc_schwarz ? c->cl.ext_ptr[c->cl.nc] : 0;
  info->product = c->toe ? SCABS_PRODUCT_TOEPLITZ : SCABS_PRODUCT_PFFT;
  if (c->toe) {
    info->rings = c->rt.nr;
    info->circulant_length = c->rt.P;
    info->ring_edges = c->rt.ne_r;
    info->ring_triangles = c->rt.nt_r;
    info->nnz_nonperiodic = c->toe_nnz;
    info->toeplitz_table_bytes = (int64_t)c->toe_table_bytes[1];
  }
  return SCABS_OK;
}

int scabs_layout(const scabs_ctx *c, int32_t *is_r, int32_t *idx) {
  if (!c) return SCABS_E_ARG;
  if (!c->built) return SCABS_E_STATE;
  for (int e = 0; e < c->geo.ne; e++) {
    if (is_r) is_r[e] = c->lay.isR[e];
    if (idx) idx[e] = c->lay.eidx[e];
  }
  return SCABS_OK;
}

// device form of a point dipole (b = 0) or of a complex-source-point beam
static SourceDev source_dev(const double pos[3], const double moment[6], const double *dir, double b) {
  SourceDev S{};
  for (int a = 0; a < 3; a++) {
    S.r0[a] = pos[a];
    S.bd[a] = b > 0 ? b * dir[a] : 0.0;
    S.p[a] = {moment[2 * a], moment[2 * a + 1]};
  }
  S.b = b > 0 ? b : 0.0;
  return S;
}
// checks of a source descriptor: body in range, b >= 0, unit direction when b > 0
static int check_source(scabs_ctx *c, const scabs_source *src) {
  if (!src) return SCABS_E_ARG;
  if (src->body < 0 || src->body >= c->geo.nbody) return fail(c, SCABS_E_ARG, "source body out of range");
  if (!(src->b >= 0)) return fail(c, SCABS_E_ARG, "source b must be >= 0");
  if (src->b > 0) {
    const double n = std::sqrt(src->dir[0] * src->dir[0] + src->dir[1] * src->dir[1] + src->dir[2] * src->dir[2]);
    if (std::fabs(n - 1.0) > 1e-9) return fail(c, SCABS_E_ARG, "beam direction must be a unit vector");
  }
  return SCABS_OK;
}

static void rhs_source(scabs_ctx *c, const SourceDev &S, int body, double *b) {
  HIPCHK(hipMemsetAsync(b, 0, sizeof(double) * 2 * c->lay.N, c->stream));
  launch_rhs_dipole(c->geo.nt, c->qp64, c->body_dev, c->p64.tris, c->p64.pts, c->edges, c->k_i, c->Z_i, S, body, b,
                    c->stream);
}

int scabs_rhs_source(scabs_ctx *c, const scabs_source *src, double *b) {
  if (!c || !src || !b) return SCABS_E_ARG;
  if (!c->built) return fail(c, SCABS_E_STATE, "scabs_build has not succeeded");
  if (int st = check_source(c, src)) return st;
  try {
    rhs_source(c, source_dev(src->pos, src->moment, src->dir, src->b), src->body, b);
    HIPCHK(hipGetLastError());
    HIPCHK(sync_stream(c->stream));
  }
  SCABS_CATCH(c)
  return SCABS_OK;
}

int scabs_rhs_dipole(scabs_ctx *c, const double pos[3], const double moment[6], int body, double *b) {
  if (!c || !pos || !moment || !b) return SCABS_E_ARG;
  if (!c->built) return fail(c, SCABS_E_STATE, "scabs_build has not succeeded");
  if (body < 0 || body >= c->geo.nbody) return fail(c, SCABS_E_ARG, "body index out of range");
  try {
    rhs_source(c, source_dev(pos, moment, nullptr, 0.0), body, b);
    HIPCHK(hipGetLastError());
    HIPCHK(sync_stream(c->stream));
  }
  SCABS_CATCH(c)
  return SCABS_OK;
}

static int do_matvec(scabs_ctx *c, const double *x, double *y, int nrhs, int prec, bool trans) {
  if (!c || !x || !y || nrhs < 1) return SCABS_E_ARG;
  if (!c->built) return fail(c, SCABS_E_STATE, "scabs_build has not succeeded");
  if (prec != SCABS_FP32 && prec != SCABS_FP64) return fail(c, SCABS_E_ARG, "prec must be SCABS_FP32 or SCABS_FP64");
  try {
    matvec_n(c, x, y, nrhs, prec, trans);
    HIPCHK(hipGetLastError());
    HIPCHK(sync_stream(c->stream));
  }
  SCABS_CATCH(c)
  return SCABS_OK;
}

int scabs_matvec(scabs_ctx *c, const double *x, double *y, int nrhs, int prec) {
  return do_matvec(c, x, y, nrhs, prec, false);
}

int scabs_matvec_transpose(scabs_ctx *c, const double *x, double *y, int nrhs, int prec) {
  return do_matvec(c, x, y, nrhs, prec, true);
}

int scabs_precond_apply(scabs_ctx *c, const double *x, double *y, int nrhs, int prec, int transpose) {
  if (!c || !x || !y || nrhs < 1) return SCABS_E_ARG;
  if (!c->built) return fail(c, SCABS_E_STATE, "scabs_build has not succeeded");
  if (!c->has_pc) return fail(c, SCABS_E_STATE, "the context was built without a preconditioner");
  if (prec != SCABS_FP32 && prec != SCABS_FP64) return fail(c, SCABS_E_ARG, "prec must be SCABS_FP32 or SCABS_FP64");
  if (transpose != 0 && transpose != 1) return fail(c, SCABS_E_ARG, "transpose must be 0 or 1");
  try {
    apply_precond_n(c, (const cx<double> *)x, (cx<double> *)y, nrhs, transpose != 0, prec);
    HIPCHK(hipGetLastError());
    HIPCHK(sync_stream(c->stream));
  }
  SCABS_CATCH(c)
  return SCABS_OK;
}

static int do_solve(scabs_ctx *c, const double *b, double *x, int nrhs, double tol, int max_iter, int restart,
                    int mode, scabs_solve_info *info, bool trans) {
  if (!c || !b || !x || nrhs < 1 || !(tol > 0) || max_iter < 1 || restart < 1) return SCABS_E_ARG;
  if (!c->built) return fail(c, SCABS_E_STATE, "scabs_build has not succeeded");
  if (mode != SCABS_FP64 && mode != SCABS_MIXED) return fail(c, SCABS_E_ARG, "mode must be SCABS_FP64 or SCABS_MIXED");
  try {
    const size_t stride = 2 * (size_t)c->lay.N;
    const int B = std::min(nrhs, near_rows_max_batch());
    ensure_work(c, restart, B);
    HIPCHK(hipMemsetAsync(c->flag, 0, sizeof(int), c->stream));
    kr_finite(b, (int64_t)stride * nrhs, c->flag, c->stream);
    kr_finite(x, (int64_t)stride * nrhs, c->flag, c->stream);
    int bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(sync_stream(c->stream));
    if (bad) return fail(c, SCABS_E_NAN, "non-finite value in b or x");
    int worst = SCABS_OK;
    for (int k0 = 0; k0 < nrhs; k0 += B) {
      const int m = std::min(B, nrhs - k0);
      int st = solve_batch(c, m, (const cx<double> *)(b + k0 * stride), (cx<double> *)(x + k0 * stride), tol,
                           max_iter, restart, mode, info ? info + k0 : nullptr, trans);
      if (st != SCABS_OK) worst = st;
    }
    if (worst != SCABS_OK) c->err = "GMRES did not reach the tolerance within max_iter";
    return worst;
  }
  SCABS_CATCH(c)
}

int scabs_solve(scabs_ctx *c, const double *b, double *x, int nrhs, double tol, int max_iter, int restart, int mode,
                scabs_solve_info *info) {
  return do_solve(c, b, x, nrhs, tol, max_iter, restart, mode, info, false);
}

int scabs_solve_transpose(scabs_ctx *c, const double *b, double *x, int nrhs, double tol, int max_iter, int restart,
                          int mode, scabs_solve_info *info) {
  return do_solve(c, b, x, nrhs, tol, max_iter, restart, mode, info, true);
}

// launch choices of the block-Toeplitz product, checked against the kernels'
// limits: form 0/1, groups 1..toe_row_groups(), lines 0 (largest) or
// 1..toe_max_lines
static int check_tune(scabs_ctx *c, int form, int groups, int lines, int overlap) {
  if (form != 0 && form != 1) return fail(c, SCABS_E_ARG, "apply form must be 0 or 1");
  if (overlap != 0 && overlap != 1) return fail(c, SCABS_E_ARG, "overlap must be 0 or 1");
  if (groups < 1 || groups > toe_row_groups()) return fail(c, SCABS_E_ARG, "column groups out of range");
  if (lines < 0 || lines > toe_max_lines(c->rt.P, true)) return fail(c, SCABS_E_ARG, "transform lines out of range");
  return SCABS_OK;
}

int scabs_set_graphs(scabs_ctx *c, int on) {
  if (!c) return SCABS_E_ARG;
  try {
    HIPCHK(hipSetDevice(c->opts.device));
    clear_graphs(c);
    c->graphs_on = on != 0;
  }
  SCABS_CATCH(c)
  return SCABS_OK;
}

int scabs_set_tune(scabs_ctx *c, int nrhs_class, int form, int groups, int lines, int overlap) {
  if (!c) return SCABS_E_ARG;
  if (!c->built || !c->toe) return fail(c, SCABS_E_STATE, "needs a built block-Toeplitz context");
  if (nrhs_class != 0 && nrhs_class != 1) return fail(c, SCABS_E_ARG, "nrhs_class must be 0 (< 8) or 1 (8)");
  if (int st = check_tune(c, form, groups, lines, overlap)) return st;
  try {
    if (overlap) {
      HIPCHK(hipSetDevice(c->opts.device));
      ensure_side(c);
    }
  }
  SCABS_CATCH(c)
  clear_graphs(c);
  c->toe_tune[nrhs_class][0] = form;
  c->toe_tune[nrhs_class][1] = groups;
  c->toe_tune[nrhs_class][2] = lines;
  c->toe_tune[nrhs_class][3] = overlap;
  return SCABS_OK;
}

int scabs_autotune(scabs_ctx *c, int reps, scabs_tune_record *rec, int max_rec, int *n_rec) {
  if (!c || reps < 1 || max_rec < 0 || (max_rec > 0 && !rec)) return SCABS_E_ARG;
  if (!c->built || !c->toe) return fail(c, SCABS_E_STATE, "autotuning applies to a built block-Toeplitz context");
  clear_graphs(c);
  try {
    HIPCHK(hipSetDevice(c->opts.device));
    const size_t stride = 2 * (size_t)c->lay.N;
    DevMem tmp;
    double *x = tmp.alloc<double>(stride * 8), *y = tmp.alloc<double>(stride * 8);
    HIPCHK(hipMemsetAsync(x, 0, sizeof(double) * stride * 8, c->stream));
    ensure_side(c);
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    const int lmax = toe_max_lines(c->rt.P, true);
    int nr = 0;
    for (int cls = 0; cls < 2; cls++) {
      const int nb = cls ? 8 : 1;
      double best = 1e300;
      int bestc[4] = {0, 8, 0, 0}, first = nr;
      std::vector<int> line_cands = {lmax};
      if (lmax > 4) line_cands.insert(line_cands.begin(), 4);
      for (int form = 0; form < (cls ? 2 : 1); form++)
        for (int groups : {4, 8, 16})
          for (int lines : line_cands)
            for (int overlap = 0; overlap < 2; overlap++) {
              c->toe_tune[cls][0] = form;
              c->toe_tune[cls][1] = groups;
              c->toe_tune[cls][2] = lines;
              c->toe_tune[cls][3] = overlap;
              matvec_n(c, x, y, nb, SCABS_FP32);   // warm
              HIPCHK(hipEventRecord(e0, c->stream));
              for (int r = 0; r < reps; r++) matvec_n(c, x, y, nb, SCABS_FP32);
              HIPCHK(hipEventRecord(e1, c->stream));
              HIPCHK(hipEventSynchronize(e1));
              float ms = 0;
              HIPCHK(hipEventElapsedTime(&ms, e0, e1));
              const double us = 1e3 * ms / reps;
              if (nr < max_rec) rec[nr] = scabs_tune_record{nb, form, groups, lines, us, 0, overlap};
              nr++;
              if (us < best) {
                best = us;
                bestc[0] = form;
                bestc[1] = groups;
                bestc[2] = lines;
                bestc[3] = overlap;
              }
            }
      for (int k = 0; k < 4; k++) c->toe_tune[cls][k] = bestc[k];
      for (int i = first; i < std::min(nr, max_rec); i++)
        rec[i].chosen = rec[i].apply_form == bestc[0] && rec[i].groups == bestc[1] && rec[i].lines == bestc[2] &&
                        rec[i].overlap == bestc[3];
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (n_rec) *n_rec = nr;
  }
  SCABS_CATCH(c)
  return SCABS_OK;
}

int scabs_solve_batched(scabs_ctx *const *ctxs, int nctx, const double *const *b, double *const *x, const int *nrhs,
                        double tol, int max_iter, int restart, int mode, scabs_solve_info *const *info) {
  if (!ctxs || nctx < 1 || !b || !x || !nrhs) return SCABS_E_ARG;
  for (int i = 0; i < nctx; i++) {
    if (!ctxs[i] || !b[i] || !x[i] || nrhs[i] < 1) return SCABS_E_ARG;
    for (int j = 0; j < i; j++)
      if (ctxs[j] == ctxs[i]) return fail(ctxs[i], SCABS_E_ARG, "a context appears twice in scabs_solve_batched");
    if (!ctxs[i]->built) return fail(ctxs[i], SCABS_E_STATE, "scabs_build has not succeeded");
  }
  // every context's restarted GMRES on its own stream, driven by its own
  // host thread: the systems' launches interleave on the GPU while each
  // host thread waits on its own Arnoldi read-backs
  std::vector<int> st(nctx, SCABS_OK);
  std::vector<std::thread> th;
  th.reserve(nctx);
  for (int i = 0; i < nctx; i++)
    th.emplace_back([&, i] {
      if (hipSetDevice(ctxs[i]->opts.device) != hipSuccess) {
        st[i] = fail(ctxs[i], SCABS_E_HIP, "hipSetDevice failed");
        return;
      }
      st[i] = do_solve(ctxs[i], b[i], x[i], nrhs[i], tol, max_iter, restart, mode, info ? info[i] : nullptr, false);
    });
  for (auto &t : th) t.join();
  int worst = SCABS_OK;
  for (int i = 0; i < nctx; i++)
    if (st[i] != SCABS_OK && (worst == SCABS_OK || worst == SCABS_E_NOCONV)) worst = st[i];
  return worst;
}

int scabs_incident_dipole_points(scabs_ctx *c, const double pos[3], const double moment[6], int body, double *E) {
  if (!c || !pos || !moment || !E) return SCABS_E_ARG;
  if (!c->built) return fail(c, SCABS_E_STATE, "scabs_build has not succeeded");
  if (body < 0 || body >= c->geo.nbody) return fail(c, SCABS_E_ARG, "body index out of range");
  try {
    launch_incident_points(c->p64.op.np, c->body_dev, c->p64.pts, c->qp64, c->k_i, c->Z_i,
                           source_dev(pos, moment, nullptr, 0.0), body, (cx<double> *)E, c->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(sync_stream(c->stream));
  }
  SCABS_CATCH(c)
  return SCABS_OK;
}

int scabs_incident_source_points(scabs_ctx *c, const scabs_source *src, double *E) {
  if (!c || !src || !E) return SCABS_E_ARG;
  if (!c->built) return fail(c, SCABS_E_STATE, "scabs_build has not succeeded");
  if (int st = check_source(c, src)) return st;
  try {
    launch_incident_points(c->p64.op.np, c->body_dev, c->p64.pts, c->qp64, c->k_i, c->Z_i,
                           source_dev(src->pos, src->moment, src->dir, src->b), src->body, (cx<double> *)E,
                           c->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(sync_stream(c->stream));
  }
  SCABS_CATCH(c)
  return SCABS_OK;
}

// one-sided pointwise fields of the operator (FP64) at every quadrature point:
// grid part, near-pair (exact - grid) part on triangles with absorber edges,
// and the 1/2 n x M residue
static void point_fields(scabs_ctx *c, const double *x, cx<double> *Ee, cx<double> *Ei) {
  PrecState<double> &P = c->p64;
  hipStream_t s = c->stream;
  if (c->toe) {
    // the block-Toeplitz operator is the Galerkin matrix itself, and its sigma
    // tests read the exact fields at the absorber triangles' points: on
    // periodic triangles the tangential fields of the product's own point
    // lines (periodic sources) plus the non-periodic edges' halves, on the
    // others a direct sum over every source triangle; zero elsewhere
    const size_t np = (size_t)P.op.np;
    HIPCHK(hipMemsetAsync(Ee, 0, 3 * np * sizeof(cx<double>), s));
    HIPCHK(hipMemsetAsync(Ei, 0, 3 * np * sizeof(cx<double>), s));
    DevMem tmp;
    double *y = tmp.alloc<double>(2 * (size_t)c->lay.N);
    apply_toe(c, c->p64, c->t64, c->toe_tri64, x, y, 1);
    launch_toe_point_fields(P.op, c->t64, c->trid, c->toe_abs_per, c->toe_nabs_per, c->toe_np_tri, c->toe_np_mask,
                            c->toe_nnp, c->k_e, c->Z_e, c->k_i, c->Z_i, c->opts.kappa_s, Ee, Ei, s);
    launch_point_fields_exact(P.op, c->trid, c->toe_abs_np, c->toe_nabs_np, c->k_e, c->Z_e, c->k_i, c->Z_i,
                              c->opts.kappa_s, Ee, Ei, s);
    HIPCHK(hipGetLastError());
    HIPCHK(sync_stream(s));
    tmp.release();
    return;
  }
  launch_unpack(P.op, x, s);
  launch_project(P.op, P.grids, P.gather, s);
  for (const DevGrid<double> &g : P.grids) launch_conv(g, s);
  launch_point_fields(P.op, P.grids[0], P.grids_dev + 1, P.inv_h, Ee, Ei, s);
  NearSetupArgs a = c->nsa;
  a.cur = P.src;
  a.Ee = Ee;
  a.Ei = Ei;
  launch_near_point_fields(a, s);
  HIPCHK(hipGetLastError());
}

int scabs_point_fields(scabs_ctx *c, const double *x, double *Ee, double *Ei) {
  if (!c || !x || !Ee || !Ei) return SCABS_E_ARG;
  if (!c->built) return fail(c, SCABS_E_STATE, "scabs_build has not succeeded");
  try {
    point_fields(c, x, (cx<double> *)Ee, (cx<double> *)Ei);
    HIPCHK(sync_stream(c->stream));
  }
  SCABS_CATCH(c)
  return SCABS_OK;
}

int scabs_eval_field(scabs_ctx *c, const double *x, const double *pts, int npts, int region, double *E, double *H) {
  if (!c || !x || !pts || npts < 1 || !E || !H) return SCABS_E_ARG;
  if (!c->built) return fail(c, SCABS_E_STATE, "scabs_build has not succeeded");
  if (region >= c->geo.nbody) return fail(c, SCABS_E_ARG, "region out of range");
  try {
    DevMem tmp;
    double *p = tmp.alloc<double>(3 * (size_t)npts);
    HIPCHK(hipMemcpyAsync(p, pts, sizeof(double) * 3 * npts, hipMemcpyHostToDevice, c->stream));
    launch_unpack(c->p64.op, x, c->stream);
    const double k = region < 0 ? c->k_e : c->k_i, Z = region < 0 ? c->Z_e : c->Z_i;
    launch_eval_field(c->p64.op, c->qp64, p, npts, region, k, Z, (cx<double> *)E, (cx<double> *)H, c->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(sync_stream(c->stream));
  }
  SCABS_CATCH(c)
  return SCABS_OK;
}

int scabs_eval_field_exact(scabs_ctx *c, const double *x, const double *pts, int npts, int region, double *E,
                           double *H) {
  if (!c || !x || !pts || npts < 1 || !E || !H) return SCABS_E_ARG;
  if (!c->built) return fail(c, SCABS_E_STATE, "scabs_build has not succeeded");
  if (region >= c->geo.nbody) return fail(c, SCABS_E_ARG, "region out of range");
  try {
    DevMem tmp;
    double *p = tmp.alloc<double>(3 * (size_t)npts);
    HIPCHK(hipMemcpyAsync(p, pts, sizeof(double) * 3 * npts, hipMemcpyHostToDevice, c->stream));
    launch_unpack(c->p64.op, x, c->stream);
    const double k = region < 0 ? c->k_e : c->k_i, Z = region < 0 ? c->Z_e : c->Z_i;
    launch_eval_field_exact(c->p64.op, c->trid, p, npts, region, k, Z, (cx<double> *)E, (cx<double> *)H, c->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(sync_stream(c->stream));
  }
  SCABS_CATCH(c)
  return SCABS_OK;
}

// incident fields of a source at points of one region: the closed form in
// the interior medium of its body, zero elsewhere
static void source_field(scabs_ctx *c, const SourceDev &S, int body, const double *pts, int npts, int region,
                         double *E, double *H) {
  if (region != body) {
    HIPCHK(hipMemsetAsync(E, 0, sizeof(cx<double>) * 3 * (size_t)npts, c->stream));
    HIPCHK(hipMemsetAsync(H, 0, sizeof(cx<double>) * 3 * (size_t)npts, c->stream));
    HIPCHK(sync_stream(c->stream));
    return;
  }
  DevMem tmp;
  double *p = tmp.alloc<double>(3 * (size_t)npts);
  HIPCHK(hipMemcpyAsync(p, pts, sizeof(double) * 3 * npts, hipMemcpyHostToDevice, c->stream));
  launch_dipole_points(npts, p, c->k_i, c->Z_i, S, (cx<double> *)E, (cx<double> *)H, c->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(sync_stream(c->stream));
}

int scabs_dipole_field(scabs_ctx *c, const double pos[3], const double moment[6], int body, const double *pts,
                       int npts, int region, double *E, double *H) {
  if (!c || !pos || !moment || !pts || npts < 1 || !E || !H) return SCABS_E_ARG;
  if (!c->built) return fail(c, SCABS_E_STATE, "scabs_build has not succeeded");
  if (body < 0 || body >= c->geo.nbody || region >= c->geo.nbody)
    return fail(c, SCABS_E_ARG, "body or region out of range");
  try {
    source_field(c, source_dev(pos, moment, nullptr, 0.0), body, pts, npts, region, E, H);
  }
  SCABS_CATCH(c)
  return SCABS_OK;
}

int scabs_source_field(scabs_ctx *c, const scabs_source *src, const double *pts, int npts, int region, double *E,
                       double *H) {
  if (!c || !src || !pts || npts < 1 || !E || !H) return SCABS_E_ARG;
  if (!c->built) return fail(c, SCABS_E_STATE, "scabs_build has not succeeded");
  if (int st = check_source(c, src)) return st;
  if (region >= c->geo.nbody) return fail(c, SCABS_E_ARG, "region out of range");
  try {
    source_field(c, source_dev(src->pos, src->moment, src->dir, src->b), src->body, pts, npts, region, E, H);
  }
  SCABS_CATCH(c)
  return SCABS_OK;
}

// total fields at points of one region on the host: scattered (near-surface
// accurate) plus the source's incident field where it lives
static void total_fields_host(scabs_ctx *c, const double *x, const scabs_source *src, const std::vector<double> &pts,
                              int region, std::vector<std::complex<double>> &E, std::vector<std::complex<double>> &H) {
  const int n = (int)(pts.size() / 3);
  E.assign(3 * (size_t)n, 0.0);
  H.assign(3 * (size_t)n, 0.0);
  if (n == 0) return;
  DevMem tmp;
  double *p = tmp.upload(pts);
  cx<double> *Ed = tmp.alloc<cx<double>>(3 * (size_t)n), *Hd = tmp.alloc<cx<double>>(3 * (size_t)n);
  launch_unpack(c->p64.op, x, c->stream);
  const double k = region < 0 ? c->k_e : c->k_i, Z = region < 0 ? c->Z_e : c->Z_i;
  launch_eval_field_exact(c->p64.op, c->trid, p, n, region, k, Z, Ed, Hd, c->stream);
  HIPCHK(hipGetLastError());
  std::vector<cx<double>> e(3 * (size_t)n), h(3 * (size_t)n), ei, hi;
  HIPCHK(hipMemcpyAsync(e.data(), Ed, sizeof(cx<double>) * e.size(), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(h.data(), Hd, sizeof(cx<double>) * h.size(), hipMemcpyDeviceToHost, c->stream));
  if (src && src->body == region) {
    ei.resize(e.size());
    hi.resize(h.size());
    launch_dipole_points(n, p, c->k_i, c->Z_i, source_dev(src->pos, src->moment, src->dir, src->b), Ed, Hd, c->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(ei.data(), Ed, sizeof(cx<double>) * e.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(hi.data(), Hd, sizeof(cx<double>) * h.size(), hipMemcpyDeviceToHost, c->stream));
  }
  HIPCHK(sync_stream(c->stream));
  for (size_t i = 0; i < e.size(); i++) {
    E[i] = {e[i].x, e[i].y};
    H[i] = {h[i].x, h[i].y};
    if (!ei.empty()) {
      E[i] += std::complex<double>(ei[i].x, ei[i].y);
      H[i] += std::complex<double>(hi[i].x, hi[i].y);
    }
  }
}

int scabs_poynting_decay(scabs_ctx *c, const double *x, const scabs_source *src, int body, double xpos,
                         const double guide[4], const double box[4], int nq, double out[4]) {
  if (!c || !x || !guide || !box || !out) return SCABS_E_ARG;
  if (!c->built) return fail(c, SCABS_E_STATE, "scabs_build has not succeeded");
  if (body < 0 || body >= c->geo.nbody) return fail(c, SCABS_E_ARG, "body out of range");
  if (src)
    if (int st = check_source(c, src)) return st;
  if (nq < 2 || nq > 64) return fail(c, SCABS_E_ARG, "nq must be in [2, 64]");
  if (!(box[0] < guide[0] && guide[0] < guide[1] && guide[1] < box[1] && box[2] < guide[2] && guide[2] < guide[3] &&
        guide[3] < box[3]))
    return fail(c, SCABS_E_ARG, "the box must contain the guide rectangle strictly");
  try {
    const Geometry &g = c->geo;
    std::vector<double> gx, gw;
    gauss_legendre(nq, gx, gw);
    // rectangles of A: the guide's (interior) and the eight around it (exterior)
    const double ys[4] = {box[0], guide[0], guide[1], box[1]}, zs[4] = {box[2], guide[2], guide[3], box[3]};
    std::vector<double> pin, win, pex, wex;
    for (int iy = 0; iy < 3; iy++)
      for (int iz = 0; iz < 3; iz++) {
        const bool inside = iy == 1 && iz == 1;
        std::vector<double> &P = inside ? pin : pex, &W = inside ? win : wex;
        const double hy = 0.5 * (ys[iy + 1] - ys[iy]), hz = 0.5 * (zs[iz + 1] - zs[iz]);
        const double cy = 0.5 * (ys[iy + 1] + ys[iy]), cz = 0.5 * (zs[iz + 1] + zs[iz]);
        for (int a = 0; a < nq; a++)
          for (int b = 0; b < nq; b++) {
            P.insert(P.end(), {xpos, cy + hy * gx[a], cz + hz * gx[b]});
            W.push_back(hy * hz * gw[a] * gw[b]);
          }
      }
    // boundary L of A (exterior medium): 2 nq points per side, outward normals
    std::vector<double> pl, wl, nl;
    for (int sd = 0; sd < 4; sd++) {
      const bool yside = sd < 2;   // sides y = box[0], box[1], then z = box[2], box[3]
      const double lo = yside ? box[2] : box[0], hi = yside ? box[3] : box[1];
      std::vector<double> lx, lw;
      gauss_legendre(2 * nq, lx, lw);
      for (int a = 0; a < 2 * nq; a++) {
        const double t = 0.5 * (lo + hi) + 0.5 * (hi - lo) * lx[a];
        if (yside)
          pl.insert(pl.end(), {xpos, box[sd], t});
        else
          pl.insert(pl.end(), {xpos, t, box[sd]});
        wl.push_back(0.5 * (hi - lo) * lw[a]);
        const double sgn = (sd % 2 == 0) ? -1.0 : 1.0;
        nl.insert(nl.end(), {0.0, yside ? sgn : 0.0, yside ? 0.0 : sgn});
      }
    }
    std::vector<std::complex<double>> Ei, Hi, Ee, He, El, Hl;
    total_fields_host(c, x, src, pin, body, Ei, Hi);
    total_fields_host(c, x, src, pex, -1, Ee, He);
    total_fields_host(c, x, src, pl, -1, El, Hl);
    auto sx = [](const std::complex<double> *E, const std::complex<double> *H) {   // (E x H*) . x
      return (E[1] * std::conj(H[2]) - E[2] * std::conj(H[1])).real();
    };
    double fluxA = 0, fluxL = 0, perim = 0;
    for (size_t i = 0; i < win.size(); i++) fluxA += win[i] * sx(&Ei[3 * i], &Hi[3 * i]);
    for (size_t i = 0; i < wex.size(); i++) fluxA += wex[i] * sx(&Ee[3 * i], &He[3 * i]);
    for (size_t i = 0; i < wl.size(); i++) {
      const std::complex<double> *E = &El[3 * i], *H = &Hl[3 * i];
      const std::complex<double> S[3] = {E[1] * std::conj(H[2]) - E[2] * std::conj(H[1]),
                                         E[2] * std::conj(H[0]) - E[0] * std::conj(H[2]),
                                         E[0] * std::conj(H[1]) - E[1] * std::conj(H[0])};
      fluxL += wl[i] * (S[1].real() * nl[3 * i + 1] + S[2].real() * nl[3 * i + 2]);
    }
    // the guide's perimeter at xpos: sigma |E_tan|^2 = sigma |M|^2 (M = E x n)
    std::vector<double> xh(2 * (size_t)c->lay.N);
    HIPCHK(hipMemcpy(xh.data(), x, sizeof(double) * xh.size(), hipMemcpyDeviceToHost));
    double ext = 0;
    for (int i = 0; i < 4; i++) ext = std::max(ext, std::fabs(box[i]));
    const double tol = 1e-7 * std::max(ext, std::fabs(xpos) + 1.0);
    std::vector<double> lx, lw;
    gauss_legendre(2 * nq, lx, lw);
    for (int sd = 0; sd < 4; sd++) {
      const bool yside = sd < 2;
      const double lo = yside ? guide[2] : guide[0], hi = yside ? guide[3] : guide[1];
      for (int a = 0; a < 2 * nq; a++) {
        const double t = 0.5 * (lo + hi) + 0.5 * (hi - lo) * lx[a];
        const double r[3] = {xpos, yside ? guide[sd] : t, yside ? t : guide[sd]};
        const int T = locate_surface_point(g, r, body, tol);
        if (T < 0) return fail(c, SCABS_E_ARG, "a point of the guide rectangle is not on the body's surface");
        std::complex<double> J[3], M[3];
        surface_currents_at(g, c->lay, xh.data(), T, r, false, J, M);
        const double m2 = std::norm(M[0]) + std::norm(M[1]) + std::norm(M[2]);
        perim += 0.5 * (hi - lo) * lw[a] * sigma_at(g, c->ends, r, T) * m2;
      }
    }
    out[0] = (perim + fluxL) / (2.0 * fluxA);
    out[1] = perim;
    out[2] = fluxL;
    out[3] = fluxA;
  }
  SCABS_CATCH(c)
  return SCABS_OK;
}

int scabs_eval_field_noalloc(scabs_ctx *c, const double *x, const double *pts, int npts, int region, double *E,
                             double *H) {
  if (!c || !x || !pts || npts < 1 || !E || !H) return SCABS_E_ARG;
  if (npts > SCABS_NOALLOC_MAX_POINTS)
    return fail(c, SCABS_E_ARG, "npts exceeds SCABS_NOALLOC_MAX_POINTS (the scratch array's capacity)");
  if (!c->built) return fail(c, SCABS_E_STATE, "scabs_build has not succeeded");
  if (region >= c->geo.nbody) return fail(c, SCABS_E_ARG, "region out of range");
  try {
    // the points go into this device's scratch array (its looked-up address)
    HIPCHK(hipMemcpyAsync(c->noalloc_pts, pts, sizeof(double) * 3 * npts, hipMemcpyHostToDevice, c->stream));
    launch_unpack(c->p64.op, x, c->stream);
    const double k = region < 0 ? c->k_e : c->k_i, Z = region < 0 ? c->Z_e : c->Z_i;
    launch_eval_field(c->p64.op, c->qp64, c->noalloc_pts, npts, region, k, Z, (cx<double> *)E, (cx<double> *)H,
                      c->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(sync_stream(c->stream));
  }
  SCABS_CATCH(c)
  return SCABS_OK;
}

int scabs_eval_field_transpose(scabs_ctx *c, const double *pts, int npts, int region, const double *wE, double *y) {
  if (!c || !pts || npts < 1 || !wE || !y) return SCABS_E_ARG;
  if (!c->built) return fail(c, SCABS_E_STATE, "scabs_build has not succeeded");
  if (region >= c->geo.nbody) return fail(c, SCABS_E_ARG, "region out of range");
  try {
    DevMem tmp;
    double *p = tmp.alloc<double>(3 * (size_t)npts);
    HIPCHK(hipMemcpyAsync(p, pts, sizeof(double) * 3 * npts, hipMemcpyHostToDevice, c->stream));
    const double k = region < 0 ? c->k_e : c->k_i, Z = region < 0 ? c->Z_e : c->Z_i;
    launch_eval_field_t(c->p64.op, c->qp64, p, npts, region, k, Z, (const cx<double> *)wE, y, c->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(sync_stream(c->stream));
  }
  SCABS_CATCH(c)
  return SCABS_OK;
}

int scabs_sigma_params(const scabs_ctx *c, int64_t *n) {
  if (!c || !n) return SCABS_E_ARG;
  int64_t k = 0;
  for (const SigmaEnd &e : c->ends) k += !e.pts.empty() ? (int64_t)e.pts.size() : e.ctrl.empty() ? 1 : (int64_t)e.ctrl.size();
  *n = k;
  return SCABS_OK;
}

int scabs_sigma_gradient(scabs_ctx *c, const double *x, const double *lam, const double *einc, double *dfdsigma,
                         double *dfdparam) {
  if (!c || !x || !lam) return SCABS_E_ARG;
  if (!c->built) return fail(c, SCABS_E_STATE, "scabs_build has not succeeded");
  try {
    const size_t np = (size_t)c->p64.op.np;
    DevMem tmp;
    cx<double> *Ee = tmp.alloc<cx<double>>(3 * np), *Ei = tmp.alloc<cx<double>>(3 * np);
    double *dfds = dfdsigma ? dfdsigma : tmp.alloc<double>(np);
    point_fields(c, x, Ee, Ei);
    launch_unpack_rows(c->p64.op, lam, c->stream);
    launch_sigma_grad(c->p64.op, Ee, Ei, (const cx<double> *)einc, dfds, c->stream);
    HIPCHK(hipGetLastError());
    std::vector<double> h(dfdparam ? np : 0);
    if (dfdparam) HIPCHK(hipMemcpyAsync(h.data(), dfds, np * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(sync_stream(c->stream));
    tmp.release();
    if (dfdparam) {
      // chain rule through the profile: d sigma_q / d p for every end's parameters
      std::vector<int64_t> jp;
      std::vector<int> jk;
      std::vector<double> jv;
      int64_t npar = 0;
      sigma_param_jacobian(c->geo, c->ends, jp, jk, jv, &npar);
      std::vector<double> g(npar, 0.0);
      for (size_t q = 0; q < np; q++)
        for (int64_t t = jp[q]; t < jp[q + 1]; t++) g[jk[t]] += jv[t] * h[q];
      std::memcpy(dfdparam, g.data(), npar * sizeof(double));
    }
  }
  SCABS_CATCH(c)
  return SCABS_OK;
}

int scabs_gradient(scabs_ctx *c, const double *x, const double *g, const double *einc, double tol, int max_iter,
                   int restart, int mode, double *dfdsigma, double *dfdparam, scabs_solve_info *info) {
  if (!c || !x || !g) return SCABS_E_ARG;
  if (!c->built) return fail(c, SCABS_E_STATE, "scabs_build has not succeeded");
  try {
    DevMem tmp;
    double *lam = tmp.alloc<double>(2 * (size_t)c->lay.N);
    HIPCHK(hipMemsetAsync(lam, 0, sizeof(double) * 2 * (size_t)c->lay.N, c->stream));
    const int st = do_solve(c, g, lam, 1, tol, max_iter, restart, mode, info, true);
    if (st != SCABS_OK) return st;
    return scabs_sigma_gradient(c, x, lam, einc, dfdsigma, dfdparam);
  }
  SCABS_CATCH(c)
}

int scabs_profile_begin(scabs_ctx *c) {
  if (!c) return SCABS_E_ARG;
  c->prof_recs.clear();
  c->ev_used = 0;
  c->prof_on = true;
  return SCABS_OK;
}

int scabs_profile_mask(scabs_ctx *c, uint32_t mask) {
  if (!c) return SCABS_E_ARG;
  if (mask >> SCABS_NSTAGES) return fail(c, SCABS_E_ARG, "mask names a stage that does not exist");
  c->prof_mask = mask ? mask : ~0u;
  return SCABS_OK;
}

int scabs_profile_end(scabs_ctx *c, double *ms, int64_t *count) {
  if (!c) return SCABS_E_ARG;
  c->prof_on = false;
  if (sync_stream(c->stream) != hipSuccess) return fail(c, SCABS_E_HIP, "stream synchronisation failed");
  for (int k = 0; k < SCABS_NSTAGES; k++) {
    if (ms) ms[k] = 0;
    if (count) count[k] = 0;
    c->prof_bytes[k] = 0;
  }
  for (auto &r : c->prof_recs) {
    float t = 0;
    if (hipEventElapsedTime(&t, r.e0, r.e1) != hipSuccess) continue;
    if (r.stage >= 0 && r.stage < SCABS_NSTAGES) {
      if (ms) ms[r.stage] += t;
      if (count) count[r.stage] += r.launches;
      c->prof_bytes[r.stage] += r.bytes;
    }
  }
  c->prof_recs.clear();
  c->ev_used = 0;
  return SCABS_OK;
}

int scabs_profile_bytes(const scabs_ctx *c, double *bytes) {
  if (!c || !bytes) return SCABS_E_ARG;
  for (int k = 0; k < SCABS_NSTAGES; k++) bytes[k] = c->prof_bytes[k];
  return SCABS_OK;
}

const char *scabs_last_error(const scabs_ctx *c) { return c ? c->err.c_str() : "null context"; }

void scabs_destroy(scabs_ctx *c) {
  if (!c) return;
  hipSetDevice(c->opts.device);
  if (c->stream) (void)sync_stream(c->stream);
  clear_graphs(c);
  c->work.release();
  c->workV64.release();
  c->workV32.release();
  c->mem.release();
  if (c->hpin) hipHostFree(c->hpin);
  if (c->hflag) hipHostFree(c->hflag);
  for (hipEvent_t e : c->ev_pool) hipEventDestroy(e);
  if (c->side) (void)sync_stream(c->side);
  for (hipEvent_t e : c->ev_side)
    if (e) hipEventDestroy(e);
  if (c->side) hipStreamDestroy(c->side);
  if (c->own_stream && c->stream) hipStreamDestroy(c->stream);
  delete c;
}

}  // extern "C"
