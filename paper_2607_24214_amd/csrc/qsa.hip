// Host runtime and C ABI of the QSA slice sweep (see include/qsa.h).
//
// The context carves every device array out of the caller's workspace, keeps
// the host-side state (loaded particle counts, error state) and enqueues the
// kernels of qsa_kernels.h on the caller's stream.  One sweep is
// 4 + 4 + 4K + 1 dependent launches per xi slice.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/qsa.h"
#include "qsa_kernels.h"

using namespace qsa;

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxN = 512;
constexpr int kSortEvery = 8;   // plasma counting sort every kSortEvery slices

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// Byte offsets of every device array inside the workspace.
struct Layout {
  size_t twx, twy, kx2, kdx, ky2, kdy;
  size_t tmpl[4], pl[4], pl2[4];
  size_t cell_of, count, bsum, prow, ppart;
  size_t rowoff[QSA_MAX_SPECIES], scan64, bpart, strays, ctl;
  int64_t stray_cap;
  size_t beam[QSA_MAX_SPECIES][7];  // x, y, ux, uy, uz, w (real), xi (double)
  size_t src, fields, dep, rowspec, colout, jring, jz, bring, ode, err, emit, lane;
  size_t total;
};

struct Carver {
  size_t off = 0;
  size_t take(size_t bytes) {
    size_t o = off;
    off += (bytes + kAlign - 1) / kAlign * kAlign;
    return o;
  }
};

Layout make_layout(const qsa_params& p) {
  const size_t rs = (p.precision == QSA_FP32) ? 4 : 8;
  const size_t cs = 2 * rs;
  const size_t nperp = (size_t)p.nx * p.ny;
  const size_t nxh = (size_t)p.nx / 2 + 1;
  const size_t spec = (size_t)p.ny * nxh * cs;
  Layout L;
  Carver c;
  L.twx = c.take(p.nx * cs);
  L.twy = c.take(p.ny * cs);
  L.kx2 = c.take(nxh * rs);
  L.kdx = c.take(nxh * rs);
  L.ky2 = c.take(p.ny * rs);
  L.kdy = c.take(p.ny * rs);
  for (int i = 0; i < 4; ++i) L.tmpl[i] = c.take(p.n_plasma * rs);
  for (int i = 0; i < 4; ++i) L.pl[i] = c.take(p.n_plasma * rs);
  for (int i = 0; i < 4; ++i) L.pl2[i] = c.take(p.n_plasma * rs);
  L.cell_of = c.take(p.n_plasma * sizeof(int));
  L.count = c.take(nperp * sizeof(int));
  L.bsum = c.take(256 * sizeof(int));
  L.prow = c.take((p.ny + 1) * sizeof(int));
  L.ppart = c.take((size_t)p.ny * 4 * 3 * p.nx * rs);
  const size_t nrows = (size_t)p.nxi * p.ny;
  int64_t total = 0;
  for (int s = 0; s < QSA_MAX_SPECIES; ++s) {
    L.rowoff[s] = c.take((nrows + 2) * sizeof(int64_t));
    if (s < p.n_species) total += p.beam_capacity[s];
  }
  L.scan64 = c.take(((nrows + 2) / 1024 + 8) * 2 * sizeof(int64_t));
  L.bpart = c.take(nrows * 2 * 4 * 4 * (size_t)p.nx * rs);   // up to 4 node rows per block
  L.stray_cap = std::min<int64_t>(total, std::max<int64_t>((int64_t)1 << 20, total / 8));
  L.strays = c.take((size_t)std::max<int64_t>(L.stray_cap, 1) * sizeof(int64_t));
  L.ctl = c.take(4 * sizeof(int));
  for (int s = 0; s < QSA_MAX_SPECIES; ++s) {
    const size_t cap = (s < p.n_species) ? (size_t)p.beam_capacity[s] : 0;
    for (int k = 0; k < 6; ++k) L.beam[s][k] = c.take(cap * rs);
    L.beam[s][6] = c.take(cap * 8);
  }
  L.src = c.take(4 * (size_t)p.nxi * nperp * rs);
  L.fields = c.take((size_t)N_STORED * p.nxi * nperp * rs);
  L.dep = c.take(3 * nperp * rs);
  L.rowspec = c.take(4 * spec);
  L.colout = c.take(4 * spec);
  L.jring = c.take(4 * spec);
  L.jz = c.take(spec);
  L.bring = c.take(6 * spec);
  L.ode = c.take(2 * sizeof(double));
  L.err = c.take(sizeof(int));
  L.emit = c.take(nperp * sizeof(double));
  L.lane = c.take(sizeof(Lane<double>));
  L.total = c.off;
  return L;
}

const char* validate(const qsa_params* p) {
  if (!p) return "null parameters";
  if (p->precision != QSA_FP64 && p->precision != QSA_FP32) return "precision must be QSA_FP64 or QSA_FP32";
  if (!pow2(p->nx) || p->nx < 8 || p->nx > kMaxN) return "nx must be a power of two in [8, 512]";
  if (!(p->ny == 1 || (pow2(p->ny) && p->ny >= 8 && p->ny <= kMaxN)))
    return "ny must be 1 (slab) or a power of two in [8, 512]";
  if (p->nxi < 2) return "nxi must be >= 2";
  if (!(p->dx > 0) || !(p->dy > 0) || !(p->dxi > 0)) return "cell sizes must be > 0";
  if (!(p->dt > 0) || !std::isfinite(p->dt)) return "dt must be finite and > 0";
  if (p->n_corr < 0 || p->n_corr > 64) return "n_corr must be in [0, 64]";
  if (!(p->kappa2 > 0)) return "kappa2 must be > 0";
  if (p->n_plasma <= 0 || p->n_plasma > (int64_t)1 << 30) return "n_plasma must be in [1, 2^30]";
  if (!(p->plasma_w > 0)) return "plasma_w must be > 0";
  if (p->n_species < 1 || p->n_species > QSA_MAX_SPECIES) return "n_species must be in [1, 4]";
  for (int s = 0; s < p->n_species; ++s) {
    if (p->beam_capacity[s] < 0) return "beam capacity must be >= 0";
    if (!(p->species[s].M > 0)) return "species mass must be > 0";
  }
  return nullptr;
}

}  // namespace

struct qsa_ctx {
  qsa_params p;
  Layout L;
  char* ws = nullptr;
  hipStream_t user = nullptr;     // the caller's stream
  hipStream_t stream = nullptr;   // the library's work stream (ordered after `user` per call)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipGraphExec_t gx_step = nullptr, gx_sweep = nullptr;   // captured beam step / sweep
  bool use_graphs = true;
  int bnl = 2;   // node rows per beam partial block along y (4 = one margin row each side)
  int64_t beam_n[QSA_MAX_SPECIES] = {0, 0, 0, 0};
  bool plasma_loaded = false;
  bool swept = false;
  qsa_status sticky = QSA_OK;
  std::string err;
  // launch timing (qsa_timing_begin/end)
  int timing_class = -1;
  std::vector<hipEvent_t> events;
  size_t ev_used = 0;
  template <typename T>
  T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
  void tstart(int k) {
    if (k != timing_class) return;
    if (ev_used + 2 > events.size()) {
      if (events.size() >= (size_t)2 << 17) return;
      hipEvent_t a, b;
      if (hipEventCreate(&a) != hipSuccess) return;
      if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return;
      }
      events.push_back(a);
      events.push_back(b);
    }
    (void)hipEventRecord(events[ev_used], stream);
  }
  void tstop(int k) {
    if (k != timing_class || ev_used + 2 > events.size()) return;
    (void)hipEventRecord(events[ev_used + 1], stream);
    ev_used += 2;
  }
  void drop_graphs() {
    if (gx_step) (void)hipGraphExecDestroy(gx_step);
    if (gx_sweep) (void)hipGraphExecDestroy(gx_sweep);
    gx_step = gx_sweep = nullptr;
  }
  ~qsa_ctx() {
    drop_graphs();
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (stream) (void)hipStreamDestroy(stream);
  }
};

// A batch: the slice loops of several contexts run as lanes of the same
// launches; beam deposits and pushes run per context on the batch's stream.
struct qsa_batch {
  std::vector<qsa_ctx*> ctxs;
  int precision = QSA_FP64;
  char* ws = nullptr;     // lane table
  hipStream_t user = nullptr, stream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipGraphExec_t gx_step = nullptr, gx_sweep = nullptr;
  bool use_graphs = true;
  ~qsa_batch() {
    if (gx_step) (void)hipGraphExecDestroy(gx_step);
    if (gx_sweep) (void)hipGraphExecDestroy(gx_sweep);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (stream) (void)hipStreamDestroy(stream);
  }
};

static qsa_status fail(qsa_ctx* c, qsa_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

#define HIP_OK(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) {                                                            \
      c->sticky = QSA_E_DEVICE;                                                        \
      return fail(c, QSA_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    }                                                                                  \
  } while (0)

namespace {

template <typename R>
struct Engine {
  static Geo<R> geo(const qsa_params& p) {
    Geo<R> g;
    g.nx = p.nx;
    g.ny = p.ny;
    g.nxi = p.nxi;
    g.nxh = p.nx / 2 + 1;
    g.nperp = p.nx * p.ny;
    g.lgx = ilog2(p.nx);
    g.lgy = ilog2(p.ny);
    g.dx = (R)p.dx;
    g.dy = (R)p.dy;
    g.dxi = (R)p.dxi;
    g.inv_dx = (R)(1.0 / p.dx);
    g.inv_dy = (R)(1.0 / p.dy);
    g.lx = (R)(p.nx * p.dx);
    g.ly = (R)(p.ny * p.dy);
    g.inv_lx = (R)(1.0 / (p.nx * p.dx));
    g.inv_ly = (R)(1.0 / (p.ny * p.dy));
    return g;
  }

  // transform and wavenumber tables, computed in long double on the host
  static void tables(const qsa_params& p, std::vector<char>& twx, std::vector<char>& twy,
                     std::vector<char>& kx2, std::vector<char>& kdx, std::vector<char>& ky2,
                     std::vector<char>& kdy) {
    auto tw = [](int n, std::vector<char>& out) {
      out.resize(n * sizeof(C2<R>));
      C2<R>* t = reinterpret_cast<C2<R>*>(out.data());
      const long double pi = 3.141592653589793238462643383279502884L;
      for (int m = 0; m < n; ++m) {
        long double a = 2.0L * pi * (long double)m / (long double)n;
        t[m].x = (R)cosl(a);
        t[m].y = (R)(-sinl(a));
      }
    };
    tw(p.nx, twx);
    tw(p.ny, twy);
    const int nxh = p.nx / 2 + 1;
    kx2.resize(nxh * sizeof(R));
    kdx.resize(nxh * sizeof(R));
    ky2.resize(p.ny * sizeof(R));
    kdy.resize(p.ny * sizeof(R));
    R* a = reinterpret_cast<R*>(kx2.data());
    R* b = reinterpret_cast<R*>(kdx.data());
    const double twopi = 6.283185307179586;
    for (int m = 0; m < nxh; ++m) {
      const int ms = (m == p.nx / 2) ? -m : m;  // Nyquist index is m = -nx/2
      const double k = 2.0 * M_PI * ms / (p.nx * p.dx);
      a[m] = (R)(k * k);
      b[m] = (m == p.nx / 2) ? R(0) : (R)k;
    }
    (void)twopi;
    R* cc = reinterpret_cast<R*>(ky2.data());
    R* d = reinterpret_cast<R*>(kdy.data());
    for (int m = 0; m < p.ny; ++m) {
      const int ms = (m < (p.ny + 1) / 2) ? m : m - p.ny;
      const double k = 2.0 * M_PI * ms / (p.ny * p.dy);
      cc[m] = (R)(k * k);
      d[m] = (p.ny > 1 && m == p.ny / 2) ? R(0) : (R)k;
    }
  }

  static int fill_blocks(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (int)b;
  }

  static qsa_status fill(qsa_ctx* c, R* p, int64_t n, R v) {
    if (n <= 0) return QSA_OK;
    hipLaunchKernelGGL(k_fill<R>, dim3(fill_blocks(n)), dim3(256), 0, c->stream, p, n, v);
    HIP_OK(hipGetLastError());
    return QSA_OK;
  }

  static BeamDepArgs<R> beam_dep_args(qsa_ctx* c) {
    const qsa_params& p = c->p;
    BeamDepArgs<R> a;
    std::memset(&a, 0, sizeof(a));
    a.ns = p.n_species;
    for (int s = 0; s < p.n_species; ++s) {
      a.x[s] = c->at<R>(c->L.beam[s][0]);
      a.y[s] = c->at<R>(c->L.beam[s][1]);
      a.ux[s] = c->at<R>(c->L.beam[s][2]);
      a.uy[s] = c->at<R>(c->L.beam[s][3]);
      a.uz[s] = c->at<R>(c->L.beam[s][4]);
      a.w[s] = c->at<R>(c->L.beam[s][5]);
      a.xi[s] = c->at<double>(c->L.beam[s][6]);
      a.rowoff[s] = c->at<int64_t>(c->L.rowoff[s]);
      a.zq[s] = (R)(p.species[s].Z / (p.dx * p.dy * p.dxi));
    }
    a.bpart = c->at<R>(c->L.bpart);
    a.strays = c->at<int64_t>(c->L.strays);
    a.stray_cap = c->L.stray_cap;
    a.ctl = c->at<int>(c->L.ctl);
    a.inv_dxi = 1.0 / p.dxi;
    a.nl = c->bnl;
    return a;
  }

  // Exclusive scan of n int64 values in place (multi-level, workspace temp).
  static qsa_status scan64(qsa_ctx* c, int64_t* v, int64_t n, int64_t* tmp) {
    const int64_t nb = (n + 1023) / 1024;
    hipLaunchKernelGGL(k_scan64_local, dim3((unsigned)nb), dim3(256), 0, c->stream, v, n, tmp);
    HIP_OK(hipGetLastError());
    if (nb > 1) {
      qsa_status st = scan64(c, tmp, nb, tmp + nb);
      if (st != QSA_OK) return st;
      hipLaunchKernelGGL(k_scan64_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, v, n,
                         (const int64_t*)tmp);
      HIP_OK(hipGetLastError());
    }
    return QSA_OK;
  }

  // Cell-row offsets of beam species s (after a load).
  static qsa_status beam_rows(qsa_ctx* c, int s) {
    const qsa_params& p = c->p;
    const Geo<R> g = geo(p);
    const int64_t nrows = (int64_t)p.nxi * p.ny;
    int64_t* off = c->at<int64_t>(c->L.rowoff[s]);
    hipLaunchKernelGGL(k_fill<int64_t>, dim3(fill_blocks(nrows + 2)), dim3(256), 0, c->stream, off,
                       nrows + 2, (int64_t)0);
    const int64_t n = c->beam_n[s];
    if (n > 0) {
      BeamDepArgs<R> a = beam_dep_args(c);
      hipLaunchKernelGGL(k_beam_rowcount<R>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, g,
                         a, s, n, off);
    }
    HIP_OK(hipGetLastError());
    return scan64(c, off, nrows + 2, c->at<int64_t>(c->L.scan64));
  }

  // Beam sources as block-private partial rows (+ atomics for strays).
  static qsa_status beam_deposit_all(qsa_ctx* c, const Geo<R>& g) {
    const qsa_params& p = c->p;
    hipLaunchKernelGGL(k_fill<int>, dim3(1), dim3(64), 0, c->stream, c->at<int>(c->L.ctl), (int64_t)4, 0);
    BeamDepArgs<R> a = beam_dep_args(c);
    const int nrows = p.nxi * p.ny;
    c->tstart(QSA_K_BEAM_DEPOSIT);
    hipLaunchKernelGGL(k_beam_rows<R>, dim3(nrows), dim3(256), 2 * a.nl * 4 * g.nx * sizeof(R), c->stream, g,
                       a);
    c->tstop(QSA_K_BEAM_DEPOSIT);
    hipLaunchKernelGGL(k_beam_strays<R>, dim3(std::min(nrows, 2048)), dim3(256), 0, c->stream, g, a);
    const int64_t plane = (int64_t)p.nxi * g.nperp;
    hipLaunchKernelGGL(k_beam_reduce<R>, dim3((unsigned)((plane + 255) / 256)), dim3(256), 0, c->stream, g,
                       (const R*)a.bpart, a.nl, c->at<R>(c->L.src));
    HIP_OK(hipGetLastError());
    return QSA_OK;
  }

  static BeamArgs<R> beam_args(qsa_ctx* c, const Geo<R>& g, int s) {
    const qsa_params& p = c->p;
    BeamArgs<R> a;
    a.x = c->at<R>(c->L.beam[s][0]);
    a.y = c->at<R>(c->L.beam[s][1]);
    a.ux = c->at<R>(c->L.beam[s][2]);
    a.uy = c->at<R>(c->L.beam[s][3]);
    a.uz = c->at<R>(c->L.beam[s][4]);
    a.w = c->at<R>(c->L.beam[s][5]);
    a.xi = c->at<double>(c->L.beam[s][6]);
    a.n = c->beam_n[s];
    a.fields = c->at<R>(c->L.fields);
    a.zq = (R)(p.species[s].Z / (p.dx * p.dy * p.dxi));
    a.qmh = (R)((double)p.species[s].Z / p.species[s].M * 0.5 * p.dt);
    a.dt = (R)p.dt;
    a.inv_dxi = 1.0 / p.dxi;
    a.xi_max = (double)(p.nxi - 1) * p.dxi;
    return a;
  }

  // ---- lanes ---------------------------------------------------------------
  // Device-pointer descriptor of this context's box for the per-slice kernels.
  static Lane<R> make_lane(qsa_ctx* c) {
    const qsa_params& p = c->p;
    const Layout& L = c->L;
    Lane<R> a;
    std::memset(&a, 0, sizeof(a));
    a.g = geo(p);
    a.np = (int)p.n_plasma;
    a.q = (R)(-p.plasma_w / (p.dx * p.dy));
    a.h = (R)p.dxi;
    a.kappa2 = (R)p.kappa2;
    a.fields = c->at<R>(L.fields);
    a.src = c->at<R>(L.src);
    for (int i = 0; i < 4; ++i) {
      a.tmpl[i] = c->at<R>(L.tmpl[i]);
      a.pl[0][i] = c->at<R>(L.pl[i]);
      a.pl[1][i] = c->at<R>(L.pl2[i]);
    }
    a.twx = c->at<C2<R>>(L.twx);
    a.twy = c->at<C2<R>>(L.twy);
    a.kx2 = c->at<R>(L.kx2);
    a.kdx = c->at<R>(L.kdx);
    a.ky2 = c->at<R>(L.ky2);
    a.kdy = c->at<R>(L.kdy);
    a.err = c->at<int>(L.err);
    a.cell_of = c->at<int>(L.cell_of);
    a.count = c->at<int>(L.count);
    a.bsum = c->at<int>(L.bsum);
    a.prow = c->at<int>(L.prow);
    a.ppart = c->at<R>(L.ppart);
    a.dep = c->at<R>(L.dep);
    a.rowspec = c->at<C2<R>>(L.rowspec);
    a.colout = c->at<C2<R>>(L.colout);
    a.jring = c->at<C2<R>>(L.jring);
    a.jz = c->at<C2<R>>(L.jz);
    a.bring = c->at<C2<R>>(L.bring);
    a.ode = c->at<double>(L.ode);
    return a;
  }

  // Launch shapes of a set of lanes (maxima over the boxes).
  struct Dims {
    int n = 0, nx = 0, ny = 0, nxi = 0, nxh = 0, np = 0, per_row = 0, n_corr = 0;
    int rows_r2c = 0, rt_rows = 64;   // row-pass grid and block size
    int cols[3] = {0, 0, 0};          // column-pass grid per mode
    size_t smem_col[3] = {0, 0, 0};
    int64_t clear = 0;
  };
  static void add_dims(Dims& d, const qsa_params& p) {
    d.n += 1;
    d.nx = std::max(d.nx, p.nx);
    d.ny = std::max(d.ny, p.ny);
    d.nxi = std::max(d.nxi, p.nxi);
    d.nxh = std::max(d.nxh, p.nx / 2 + 1);
    d.np = std::max(d.np, (int)p.n_plasma);
    d.per_row = std::max(d.per_row, (int)((p.n_plasma + p.ny - 1) / p.ny));
    d.n_corr = std::max(d.n_corr, p.n_corr);
    const int64_t spec = (int64_t)p.ny * (p.nx / 2 + 1);
    d.clear = std::max<int64_t>(d.clear, std::max<int64_t>(6 * spec, 3 * (int64_t)p.nx * p.ny));
  }
  static void finish_dims(Dims& d, const qsa_params* const* ps, int n) {
    d.rt_rows = std::max(64, d.nx / 4);
    d.rows_r2c = 0;
    for (int m = 0; m < 3; ++m) {
      d.cols[m] = 0;
      d.smem_col[m] = 0;
    }
    const int G[3] = {ColShape<COL_PSI>::G, ColShape<COL_J>::G, ColShape<COL_B>::G};
    for (int i = 0; i < n; ++i) {
      const qsa_params& p = *ps[i];
      const int ppw = d.rt_rows / (p.nx / 4);
      d.rows_r2c = std::max(d.rows_r2c, ((p.ny + 1) / 2 + ppw - 1) / ppw);
      const int tpt = col_tpt(p.ny);
      const int cpw = 64 / tpt;
      for (int m = 0; m < 3; ++m) {
        d.cols[m] = std::max(d.cols[m], (p.nx / 2 + 1 + cpw - 1) / cpw);
        d.smem_col[m] = std::max(d.smem_col[m], ((size_t)cpw * 2 * G[m] + 1) * p.ny * sizeof(C2<R>));
      }
    }
  }

  // The slice loop of every lane: one launch per phase per slice, blockIdx.z
  // = lane.  `tc` receives the kernel-class timing marks.
  static qsa_status slices(qsa_ctx* tc, hipStream_t st, const Lane<R>* lanes, const Dims& d) {
    const int n = d.n;
    const int pb = (d.np + 255) / 256;
    const size_t smem_rows = ((size_t)d.nx + 8 * (size_t)d.rt_rows) * sizeof(C2<R>);
    int nt = (d.per_row + 63) / 64 * 64;
    nt = std::max(64, std::min(256, nt));
    {
      const int blocks = (int)std::min<int64_t>(1024, (d.clear + 255) / 256);
      hipLaunchKernelGGL((k_lane_clear<R, 0>), dim3(blocks, 1, n), dim3(256), 0, st, lanes, 0);
    }
    for (int j = 0; j < d.nxi; ++j) {
      if (j % QSA_SORT_EVERY == 0) {
        hipLaunchKernelGGL((k_lane_clear<R, 1>), dim3((d.nx * d.ny + 255) / 256, 1, n), dim3(256), 0, st, lanes,
                           j);
        hipLaunchKernelGGL(k_sort_count<R>, dim3(pb, 1, n), dim3(256), 0, st, lanes, j);
        hipLaunchKernelGGL(k_scan_local<R>, dim3((d.nx * d.ny + 1023) / 1024, 1, n), dim3(256), 0, st, lanes, j);
        hipLaunchKernelGGL(k_scan_blocks<R>, dim3(1, 1, n), dim3(256), 0, st, lanes, j);
        hipLaunchKernelGGL(k_row_offsets<R>, dim3((d.ny + 1 + 255) / 256, 1, n), dim3(256), 0, st, lanes, j);
        hipLaunchKernelGGL(k_sort_scatter<R>, dim3(pb, 1, n), dim3(256), 0, st, lanes, j);
      }
      const dim3 rgrid_psi(d.rows_r2c, 1, n), rgrid_j(d.rows_r2c, 3, n), rgrid_b(d.rows_r2c, 2, n);
      const dim3 rblock(d.rt_rows);
      // ---- psi stage
      tc->tstart(QSA_K_DEP_S);
      hipLaunchKernelGGL((k_plasma_rows<R, PL_DEP_S>), dim3(d.ny, 1, n), dim3(nt),
                         4 * 1 * (size_t)d.nx * sizeof(R), st, lanes, j);
      tc->tstop(QSA_K_DEP_S);
      tc->tstart(QSA_K_ROW_R2C);
      hipLaunchKernelGGL(k_row_r2c<R>, rgrid_psi, rblock, smem_rows, st, lanes, j, (int)ST_PSI);
      tc->tstop(QSA_K_ROW_R2C);
      tc->tstart(QSA_K_COL);
      hipLaunchKernelGGL((k_col<R, COL_PSI>), dim3(d.cols[0], 1, n), dim3(64 * ColShape<COL_PSI>::G),
                         d.smem_col[0], st, lanes, j);
      tc->tstop(QSA_K_COL);
      tc->tstart(QSA_K_ROW_C2R);
      hipLaunchKernelGGL(k_row_c2r<R>, dim3(d.rows_r2c, 3, n), rblock, smem_rows, st, lanes, j, (int)ST_PSI);
      tc->tstop(QSA_K_ROW_C2R);
      // ---- J stage
      tc->tstart(QSA_K_DEP_J);
      hipLaunchKernelGGL((k_plasma_rows<R, PL_DEP_J>), dim3(d.ny, 1, n), dim3(nt),
                         4 * 3 * (size_t)d.nx * sizeof(R), st, lanes, j);
      tc->tstop(QSA_K_DEP_J);
      tc->tstart(QSA_K_ROW_R2C);
      hipLaunchKernelGGL(k_row_r2c<R>, rgrid_j, rblock, smem_rows, st, lanes, j, (int)ST_J);
      tc->tstop(QSA_K_ROW_R2C);
      tc->tstart(QSA_K_COL);
      hipLaunchKernelGGL((k_col<R, COL_J>), dim3(d.cols[1], 1, n), dim3(64 * ColShape<COL_J>::G),
                         d.smem_col[1], st, lanes, j);
      tc->tstop(QSA_K_COL);
      tc->tstart(QSA_K_ROW_C2R);
      hipLaunchKernelGGL(k_row_c2r<R>, dim3(d.rows_r2c, 4, n), rblock, smem_rows, st, lanes, j, (int)ST_J);
      tc->tstop(QSA_K_ROW_C2R);
      // ---- B_perp predictor-corrector
      for (int k = 0; k < d.n_corr; ++k) {
        tc->tstart(QSA_K_PUSH_PRED);
        hipLaunchKernelGGL((k_plasma_rows<R, PL_PRED>), dim3(d.ny, 1, n), dim3(nt),
                           4 * 2 * (size_t)d.nx * sizeof(R), st, lanes, j);
        tc->tstop(QSA_K_PUSH_PRED);
        tc->tstart(QSA_K_ROW_R2C);
        hipLaunchKernelGGL(k_row_r2c<R>, rgrid_b, rblock, smem_rows, st, lanes, j, (int)ST_B);
        tc->tstop(QSA_K_ROW_R2C);
        tc->tstart(QSA_K_COL);
        hipLaunchKernelGGL((k_col<R, COL_B>), dim3(d.cols[2], 1, n), dim3(64 * ColShape<COL_B>::G),
                           d.smem_col[2], st, lanes, j);
        tc->tstop(QSA_K_COL);
        tc->tstart(QSA_K_ROW_C2R);
        hipLaunchKernelGGL(k_row_c2r<R>, rgrid_b, rblock, smem_rows, st, lanes, j, (int)ST_B);
        tc->tstop(QSA_K_ROW_C2R);
      }
      // ---- advance the plasma to slice j+1
      tc->tstart(QSA_K_PUSH_FINAL);
      hipLaunchKernelGGL(k_push_final<R>, dim3(pb, 1, n), dim3(256), 0, st, lanes, j);
      tc->tstop(QSA_K_PUSH_FINAL);
    }
    return QSA_OK;
  }

  static Dims dims_of(qsa_ctx* c) {
    Dims d;
    add_dims(d, c->p);
    const qsa_params* ps[1] = {&c->p};
    finish_dims(d, ps, 1);
    return d;
  }

  static qsa_status sweep(qsa_ctx* c) {
    const Geo<R> g = geo(c->p);
    qsa_status st = beam_deposit_all(c, g);
    if (st != QSA_OK) return st;
    if ((st = slices(c, c->stream, c->at<Lane<R>>(c->L.lane), dims_of(c))) != QSA_OK) return st;
    HIP_OK(hipGetLastError());
    c->swept = true;
    return QSA_OK;
  }

  static qsa_status push(qsa_ctx* c) {
    const Geo<R> g = geo(c->p);
    for (int s = 0; s < c->p.n_species; ++s) {
      if (c->beam_n[s] == 0) continue;
      BeamArgs<R> a = beam_args(c, g, s);
      const int64_t blocks = (a.n + 255) / 256;
      c->tstart(QSA_K_BEAM_PUSH);
      hipLaunchKernelGGL(k_beam_push<R>, dim3((unsigned)blocks), dim3(256), 0, c->stream, g, a);
      c->tstop(QSA_K_BEAM_PUSH);
    }
    HIP_OK(hipGetLastError());
    return QSA_OK;
  }

  // device float64 -> working precision; host float64 goes through a chunked
  // staging copy
  static qsa_status upload(qsa_ctx* c, const double* src, void* dst, int64_t n, int on_device,
                           bool keep_f64) {
    if (n == 0) return QSA_OK;
    if (keep_f64 || sizeof(R) == 8) {
      HIP_OK(hipMemcpyAsync(dst, src, n * 8, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                            c->stream));
      if (!on_device) HIP_OK(hipStreamSynchronize(c->stream));
      return QSA_OK;
    }
    if (on_device) {
      hipLaunchKernelGGL(k_from_f64<R>, dim3(fill_blocks(n)), dim3(256), 0, c->stream, src,
                         reinterpret_cast<R*>(dst), n);
      HIP_OK(hipGetLastError());
      return QSA_OK;
    }
    const int64_t chunk = 1 << 22;
    std::vector<R> tmp((size_t)std::min<int64_t>(n, chunk));
    for (int64_t o = 0; o < n; o += chunk) {
      const int64_t m = std::min<int64_t>(chunk, n - o);
      for (int64_t i = 0; i < m; ++i) tmp[i] = (R)src[o + i];
      HIP_OK(hipMemcpyAsync(reinterpret_cast<R*>(dst) + o, tmp.data(), m * sizeof(R),
                            hipMemcpyHostToDevice, c->stream));
      HIP_OK(hipStreamSynchronize(c->stream));
    }
    return QSA_OK;
  }

  static qsa_status download(qsa_ctx* c, const void* src, double* dst, int64_t n, int on_device,
                             bool is_f64) {
    if (n == 0) return QSA_OK;
    if (is_f64 || sizeof(R) == 8) {
      HIP_OK(hipMemcpyAsync(dst, src, n * 8, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                            c->stream));
      if (!on_device) HIP_OK(hipStreamSynchronize(c->stream));
      return QSA_OK;
    }
    if (on_device) {
      hipLaunchKernelGGL(k_to_f64<R>, dim3(fill_blocks(n)), dim3(256), 0, c->stream,
                         reinterpret_cast<const R*>(src), dst, n);
      HIP_OK(hipGetLastError());
      return QSA_OK;
    }
    const int64_t chunk = 1 << 22;
    std::vector<R> tmp((size_t)std::min<int64_t>(n, chunk));
    for (int64_t o = 0; o < n; o += chunk) {
      const int64_t m = std::min<int64_t>(chunk, n - o);
      HIP_OK(hipMemcpyAsync(tmp.data(), reinterpret_cast<const R*>(src) + o, m * sizeof(R),
                            hipMemcpyDeviceToHost, c->stream));
      HIP_OK(hipStreamSynchronize(c->stream));
      for (int64_t i = 0; i < m; ++i) dst[o + i] = (double)tmp[i];
    }
    return QSA_OK;
  }

  static qsa_status fields(qsa_ctx* c, int field, int xi0, int xi1, double* dst, int on_device) {
    const qsa_params& p = c->p;
    const int64_t nperp = (int64_t)p.nx * p.ny;
    const int64_t plane = (int64_t)p.nxi * nperp;
    const R* F = c->at<R>(c->L.fields);
    double* emit = c->at<double>(c->L.emit);
    for (int j = xi0; j < xi1; ++j) {
      double* out = on_device ? dst + (int64_t)(j - xi0) * nperp : emit;
      const R* A = nullptr;
      const R* B = nullptr;
      R a = 1, b = 0;
      const int64_t o = (int64_t)j * nperp;
      switch (field) {
        case QSA_PSI: A = F + F_PSI * plane + o; break;
        case QSA_EX: A = F + F_DXPSI * plane + o; a = -1; B = F + F_BY * plane + o; b = 1; break;
        case QSA_EY: A = F + F_DYPSI * plane + o; a = -1; B = F + F_BX * plane + o; b = -1; break;
        case QSA_EZ: A = F + F_EZ * plane + o; break;
        case QSA_BX: A = F + F_BX * plane + o; break;
        case QSA_BY: A = F + F_BY * plane + o; break;
        case QSA_BZ: A = F + F_BZ * plane + o; break;
        case QSA_DXPSI: A = F + F_DXPSI * plane + o; break;
        case QSA_DYPSI: A = F + F_DYPSI * plane + o; break;
        default: A = c->at<R>(c->L.src) + (field - QSA_SRC_S) * plane + o; break;
      }
      hipLaunchKernelGGL(k_emit<R>, dim3(fill_blocks(nperp)), dim3(256), 0, c->stream, A, a, B, b,
                         out, nperp);
      HIP_OK(hipGetLastError());
      if (!on_device)
        HIP_OK(hipMemcpyAsync(dst + (int64_t)(j - xi0) * nperp, emit, nperp * 8, hipMemcpyDeviceToHost,
                              c->stream));
    }
    HIP_OK(hipStreamSynchronize(c->stream));
    return QSA_OK;
  }

  // Beam partial blocks carry one margin row on each side (so particles that
  // drifted to a neighbouring cell row stay on the LDS path) when the tile
  // 2*4*4*nx values plus the block's stray list fit the device's LDS.
  static qsa_status choose_beam_tile(qsa_ctx* c) {
    int dev = 0, optin = 0, plain = 0;
    HIP_OK(hipGetDevice(&dev));
    if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess) optin = 0;
    HIP_OK(hipDeviceGetAttribute(&plain, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const int limit = std::max(optin, plain);
    const int need = 2 * 4 * 4 * c->p.nx * (int)sizeof(R);
    const int stat = 4096;   // block stray list and counters
    c->bnl = 2;
    if (c->p.ny > 1 && need + stat <= limit) {
      if (need + stat > 65536)
        HIP_OK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_beam_rows<R>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, need));
      c->bnl = 4;
    }
    // column transforms: (2G + 1) columns of ny complex values per block
    const int colj = (2 * ColShape<COL_J>::G + 1) * c->p.ny * (int)sizeof(C2<R>);
    if (colj > limit) return fail(c, QSA_E_INVALID, "ny too large for the device's LDS");
    if (colj > 65536) {
      HIP_OK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_col<R, COL_PSI>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, colj));
      HIP_OK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_col<R, COL_J>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, colj));
      HIP_OK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_col<R, COL_B>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, colj));
    }
    return QSA_OK;
  }

  static qsa_status upload_tables(qsa_ctx* c) {
    qsa_status st0 = choose_beam_tile(c);
    if (st0 != QSA_OK) return st0;
    std::vector<char> twx, twy, kx2, kdx, ky2, kdy;
    tables(c->p, twx, twy, kx2, kdx, ky2, kdy);
    HIP_OK(hipMemcpyAsync(c->ws + c->L.twx, twx.data(), twx.size(), hipMemcpyHostToDevice, c->stream));
    HIP_OK(hipMemcpyAsync(c->ws + c->L.twy, twy.data(), twy.size(), hipMemcpyHostToDevice, c->stream));
    HIP_OK(hipMemcpyAsync(c->ws + c->L.kx2, kx2.data(), kx2.size(), hipMemcpyHostToDevice, c->stream));
    HIP_OK(hipMemcpyAsync(c->ws + c->L.kdx, kdx.data(), kdx.size(), hipMemcpyHostToDevice, c->stream));
    HIP_OK(hipMemcpyAsync(c->ws + c->L.ky2, ky2.data(), ky2.size(), hipMemcpyHostToDevice, c->stream));
    HIP_OK(hipMemcpyAsync(c->ws + c->L.kdy, kdy.data(), kdy.size(), hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(k_fill<int>, dim3(1), dim3(64), 0, c->stream, c->at<int>(c->L.err), (int64_t)1, 0);
    {
      const Lane<R> lane = make_lane(c);
      HIP_OK(hipMemcpyAsync(c->ws + c->L.lane, &lane, sizeof(lane), hipMemcpyHostToDevice, c->stream));
    }
    // no beam loaded yet: every species has empty cell rows
    const int64_t nrows = (int64_t)c->p.nxi * c->p.ny;
    for (int s = 0; s < QSA_MAX_SPECIES; ++s)
      hipLaunchKernelGGL(k_fill<int64_t>, dim3(fill_blocks(nrows + 2)), dim3(256), 0, c->stream,
                         c->at<int64_t>(c->L.rowoff[s]), nrows + 2, (int64_t)0);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(c->stream));
    return QSA_OK;
  }
};

// Pending device error -> status (synchronizing).
qsa_status check_device(qsa_ctx* c) {
  HIP_OK(hipStreamSynchronize(c->stream));
  int e = 0;
  HIP_OK(hipMemcpy(&e, c->ws + c->L.err, sizeof(int), hipMemcpyDeviceToHost));
  if (e & ERR_BREAKDOWN) {
    c->sticky = QSA_E_BREAKDOWN;
    return fail(c, QSA_E_BREAKDOWN, "quasistatic breakdown: 1 + psi <= 1e-3 or non-finite at a plasma particle");
  }
  return QSA_OK;
}

template <typename F64, typename F32>
qsa_status dispatch(qsa_ctx* c, F64 f64, F32 f32) {
  return c->p.precision == QSA_FP32 ? f32() : f64();
}

// Order the work stream after what the caller has enqueued so far, and the
// caller's stream after the work a call enqueued.
qsa_status enter(qsa_ctx* c) {
  HIP_OK(hipEventRecord(c->ev_in, c->user));
  HIP_OK(hipStreamWaitEvent(c->stream, c->ev_in, 0));
  return QSA_OK;
}
qsa_status leave(qsa_ctx* c) {
  HIP_OK(hipEventRecord(c->ev_out, c->stream));
  HIP_OK(hipStreamWaitEvent(c->user, c->ev_out, 0));
  return QSA_OK;
}

// Capture the launches `body` enqueues into an executable graph (once).  If
// the runtime refuses the capture, graphs are switched off for the context
// and the caller enqueues the launches directly (*gx stays null).
template <typename Fn>
qsa_status capture(qsa_ctx* c, hipGraphExec_t* gx, Fn body) {
  if (*gx) return QSA_OK;
  if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    c->use_graphs = false;
    return QSA_OK;
  }
  const qsa_status st = body();
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(c->stream, &graph);
  hipError_t ei = hipErrorUnknown;
  if (st == QSA_OK && e == hipSuccess) ei = hipGraphInstantiate(gx, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  if (st != QSA_OK) return st;
  if (e != hipSuccess || ei != hipSuccess) {
    (void)hipGetLastError();
    *gx = nullptr;
    c->use_graphs = false;
  }
  return QSA_OK;
}

qsa_status run_sweep(qsa_ctx* c) {
  return dispatch(c, [&] { return Engine<double>::sweep(c); }, [&] { return Engine<float>::sweep(c); });
}
qsa_status run_step(qsa_ctx* c) {
  qsa_status st = run_sweep(c);
  if (st != QSA_OK) return st;
  return dispatch(c, [&] { return Engine<double>::push(c); }, [&] { return Engine<float>::push(c); });
}

// Batched sweep (and push): every context's beam deposit on the batch's
// stream, then one slice loop over all lanes.
template <typename R>
qsa_status batch_run(qsa_batch* b, bool push) {
  qsa_ctx* c0 = b->ctxs[0];
  typename Engine<R>::Dims d;
  std::vector<const qsa_params*> ps;
  for (qsa_ctx* c : b->ctxs) {
    Engine<R>::add_dims(d, c->p);
    ps.push_back(&c->p);
  }
  Engine<R>::finish_dims(d, ps.data(), (int)ps.size());
  for (qsa_ctx* c : b->ctxs) {
    hipStream_t own = c->stream;
    c->stream = b->stream;
    const qsa_status st = Engine<R>::beam_deposit_all(c, Engine<R>::geo(c->p));
    c->stream = own;
    if (st != QSA_OK) return st;
  }
  qsa_status st = Engine<R>::slices(c0, b->stream, reinterpret_cast<const Lane<R>*>(b->ws), d);
  if (st != QSA_OK) return st;
  for (qsa_ctx* c : b->ctxs) {
    c->swept = true;
    if (!push) continue;
    hipStream_t own = c->stream;
    c->stream = b->stream;
    st = Engine<R>::push(c);
    c->stream = own;
    if (st != QSA_OK) return st;
  }
  return QSA_OK;
}

}  // namespace

extern "C" {

size_t qsa_workspace_bytes(const qsa_params* p) {
  if (validate(p)) return 0;
  return make_layout(*p).total;
}

qsa_status qsa_create(const qsa_params* p, void* dev_ws, size_t ws_bytes, void* hip_stream,
                      qsa_ctx** out) {
  if (!out) return QSA_E_INVALID;
  *out = nullptr;
  if (validate(p)) return QSA_E_INVALID;
  const Layout L = make_layout(*p);
  if (!dev_ws || ((uintptr_t)dev_ws % kAlign) != 0) return QSA_E_INVALID;
  if (ws_bytes < L.total) return QSA_E_NOMEM;
  qsa_ctx* c = new qsa_ctx();
  c->p = *p;
  c->L = L;
  c->ws = reinterpret_cast<char*>(dev_ws);
  c->user = reinterpret_cast<hipStream_t>(hip_stream);
  if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming) != hipSuccess) {
    delete c;
    return QSA_E_DEVICE;
  }
  qsa_status st = enter(c);
  if (st == QSA_OK)
    st = (p->precision == QSA_FP32) ? Engine<float>::upload_tables(c) : Engine<double>::upload_tables(c);
  if (st != QSA_OK) {
    delete c;
    return st;
  }
  *out = c;
  return QSA_OK;
}

static bool all_finite(const double* a, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

qsa_status qsa_load_plasma(qsa_ctx* c, const double* x, const double* y, const double* ux,
                           const double* uy, int64_t n, int32_t on_device) {
  if (!c) return QSA_E_INVALID;
  if (c->sticky != QSA_OK) return c->sticky;
  if (n != c->p.n_plasma) return fail(c, QSA_E_INVALID, "plasma count differs from n_plasma");
  if (!x || !y || !ux || !uy) return fail(c, QSA_E_INVALID, "null plasma array");
  const double* arr[4] = {x, y, ux, uy};
  if (!on_device)
    for (int i = 0; i < 4; ++i)
      if (!all_finite(arr[i], n)) return fail(c, QSA_E_NONFINITE, "non-finite plasma value");
  qsa_status st0 = enter(c);
  if (st0 != QSA_OK) return st0;
  for (int i = 0; i < 4; ++i) {
    qsa_status st = dispatch(
        c, [&] { return Engine<double>::upload(c, arr[i], c->ws + c->L.tmpl[i], n, on_device, false); },
        [&] { return Engine<float>::upload(c, arr[i], c->ws + c->L.tmpl[i], n, on_device, false); });
    if (st != QSA_OK) return st;
  }
  c->plasma_loaded = true;
  c->drop_graphs();
  return leave(c);
}

qsa_status qsa_load_beam(qsa_ctx* c, int32_t s, const double* x, const double* y, const double* xi,
                         const double* ux, const double* uy, const double* uz, const double* w,
                         int64_t n, int32_t on_device) {
  if (!c) return QSA_E_INVALID;
  if (c->sticky != QSA_OK) return c->sticky;
  if (s < 0 || s >= c->p.n_species) return fail(c, QSA_E_INVALID, "species index out of range");
  if (n < 0 || n > c->p.beam_capacity[s]) return fail(c, QSA_E_INVALID, "beam count exceeds capacity");
  const double* arr[7] = {x, y, ux, uy, uz, w, xi};
  for (int i = 0; i < 7; ++i)
    if (n > 0 && !arr[i]) return fail(c, QSA_E_INVALID, "null beam array");
  if (!on_device)
    for (int i = 0; i < 7; ++i)
      if (!all_finite(arr[i], n)) return fail(c, QSA_E_NONFINITE, "non-finite beam value");
  qsa_status st0 = enter(c);
  if (st0 != QSA_OK) return st0;
  for (int i = 0; i < 7; ++i) {
    const bool f64 = (i == 6);
    qsa_status st = dispatch(
        c, [&] { return Engine<double>::upload(c, arr[i], c->ws + c->L.beam[s][i], n, on_device, f64); },
        [&] { return Engine<float>::upload(c, arr[i], c->ws + c->L.beam[s][i], n, on_device, f64); });
    if (st != QSA_OK) return st;
  }
  c->beam_n[s] = n;
  c->drop_graphs();
  qsa_status st = dispatch(c, [&] { return Engine<double>::beam_rows(c, s); },
                           [&] { return Engine<float>::beam_rows(c, s); });
  if (st != QSA_OK) return st;
  return leave(c);
}

qsa_status qsa_read_beam(qsa_ctx* c, int32_t s, double* x, double* y, double* xi, double* ux,
                         double* uy, double* uz, double* w, int64_t cap, int64_t* n,
                         int32_t on_device) {
  if (!c || !n) return QSA_E_INVALID;
  if (c->sticky != QSA_OK) return c->sticky;
  if (s < 0 || s >= c->p.n_species) return fail(c, QSA_E_INVALID, "species index out of range");
  const int64_t m = c->beam_n[s];
  *n = m;
  if (cap < m) return fail(c, QSA_E_INVALID, "destination too small");
  double* arr[7] = {x, y, ux, uy, uz, w, xi};
  for (int i = 0; i < 7; ++i)
    if (m > 0 && !arr[i]) return fail(c, QSA_E_INVALID, "null destination array");
  qsa_status st0 = enter(c);
  if (st0 != QSA_OK) return st0;
  for (int i = 0; i < 7; ++i) {
    const bool f64 = (i == 6);
    qsa_status st = dispatch(
        c, [&] { return Engine<double>::download(c, c->ws + c->L.beam[s][i], arr[i], m, on_device, f64); },
        [&] { return Engine<float>::download(c, c->ws + c->L.beam[s][i], arr[i], m, on_device, f64); });
    if (st != QSA_OK) return st;
  }
  if ((st0 = leave(c)) != QSA_OK) return st0;
  return check_device(c);
}

qsa_status qsa_slice_sweep(qsa_ctx* c) {
  if (!c) return QSA_E_INVALID;
  if (c->sticky != QSA_OK) return c->sticky;
  if (!c->plasma_loaded) return fail(c, QSA_E_STATE, "no plasma template loaded");
  qsa_status st = enter(c);
  if (st != QSA_OK) return st;
  const bool graphs = c->use_graphs && c->timing_class < 0;
  if (graphs && (st = capture(c, &c->gx_sweep, [&] { return run_sweep(c); })) != QSA_OK) return st;
  if (graphs && c->gx_sweep) {
    HIP_OK(hipGraphLaunch(c->gx_sweep, c->stream));
    c->swept = true;
  } else if ((st = run_sweep(c)) != QSA_OK) {
    return st;
  }
  return leave(c);
}

qsa_status qsa_beam_step(qsa_ctx* c, int32_t n_steps) {
  if (!c) return QSA_E_INVALID;
  if (c->sticky != QSA_OK) return c->sticky;
  if (n_steps < 0) return fail(c, QSA_E_INVALID, "n_steps must be >= 0");
  if (!c->plasma_loaded) return fail(c, QSA_E_STATE, "no plasma template loaded");
  if (n_steps == 0) return QSA_OK;
  qsa_status st = enter(c);
  if (st != QSA_OK) return st;
  const bool graphs = c->use_graphs && c->timing_class < 0;
  if (graphs && (st = capture(c, &c->gx_step, [&] { return run_step(c); })) != QSA_OK) return st;
  for (int i = 0; i < n_steps; ++i) {
    if (graphs && c->gx_step) {
      HIP_OK(hipGraphLaunch(c->gx_step, c->stream));
      c->swept = true;
    } else if ((st = run_step(c)) != QSA_OK) {
      return st;
    }
  }
  return leave(c);
}

qsa_status qsa_set_option(qsa_ctx* c, int32_t option, int64_t value) {
  if (!c) return QSA_E_INVALID;
  if (option == QSA_OPT_GRAPHS) {
    c->use_graphs = value != 0;
    return QSA_OK;
  }
  return fail(c, QSA_E_INVALID, "unknown option");
}

qsa_status qsa_fields(qsa_ctx* c, int32_t field, int32_t xi0, int32_t xi1, double* dst, size_t count,
                      int32_t dst_on_device) {
  if (!c) return QSA_E_INVALID;
  if (c->sticky != QSA_OK) return c->sticky;
  if (!c->swept) return fail(c, QSA_E_STATE, "no sweep has run");
  if (field < QSA_PSI || field > QSA_SRC_JZ) return fail(c, QSA_E_INVALID, "unknown field");
  if (xi0 < 0 || xi1 > c->p.nxi || xi0 > xi1) return fail(c, QSA_E_INVALID, "slice range out of bounds");
  const size_t need = (size_t)(xi1 - xi0) * c->p.nx * c->p.ny;
  if (!dst || count < need) return fail(c, QSA_E_INVALID, "destination too small");
  qsa_status st = enter(c);
  if (st != QSA_OK) return st;
  st = dispatch(c, [&] { return Engine<double>::fields(c, field, xi0, xi1, dst, dst_on_device); },
                           [&] { return Engine<float>::fields(c, field, xi0, xi1, dst, dst_on_device); });
  if (st != QSA_OK) return st;
  if ((st = leave(c)) != QSA_OK) return st;
  return check_device(c);
}

qsa_status qsa_sync(qsa_ctx* c) {
  if (!c) return QSA_E_INVALID;
  if (c->sticky != QSA_OK) return c->sticky;
  return check_device(c);
}

qsa_status qsa_timing_begin(qsa_ctx* c, int32_t kernel_class) {
  if (!c) return QSA_E_INVALID;
  if (kernel_class < 0 || kernel_class >= QSA_K_COUNT) return fail(c, QSA_E_INVALID, "unknown kernel class");
  c->timing_class = kernel_class;
  c->ev_used = 0;
  return QSA_OK;
}

qsa_status qsa_timing_end(qsa_ctx* c, double* total_ms, int64_t* launches) {
  if (!c || !total_ms || !launches) return QSA_E_INVALID;
  HIP_OK(hipStreamSynchronize(c->stream));
  double tot = 0.0;
  bool ok = true;
  for (size_t i = 0; i + 1 < c->ev_used; i += 2) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->events[i], c->events[i + 1]) != hipSuccess) {
      ok = false;
      break;
    }
    tot += ms;
  }
  *total_ms = tot;
  *launches = (int64_t)(c->ev_used / 2);
  c->timing_class = -1;
  c->ev_used = 0;
  if (!ok) {
    (void)hipGetLastError();
    return fail(c, QSA_E_DEVICE, "hipEventElapsedTime failed");
  }
  return QSA_OK;
}

size_t qsa_batch_workspace_bytes(int32_t n_ctx) {
  if (n_ctx < 1) return 0;
  return ((size_t)n_ctx * sizeof(Lane<double>) + kAlign - 1) / kAlign * kAlign;
}

qsa_status qsa_batch_create(qsa_ctx* const* ctxs, int32_t n_ctx, void* dev_ws, size_t ws_bytes,
                            void* hip_stream, qsa_batch** out) {
  if (!out || !ctxs || n_ctx < 1) return QSA_E_INVALID;
  *out = nullptr;
  if (!dev_ws || ((uintptr_t)dev_ws % kAlign) != 0) return QSA_E_INVALID;
  if (ws_bytes < qsa_batch_workspace_bytes(n_ctx)) return QSA_E_NOMEM;
  for (int i = 0; i < n_ctx; ++i) {
    qsa_ctx* c = ctxs[i];
    if (!c) return QSA_E_INVALID;
    if (c->p.precision != ctxs[0]->p.precision || c->p.n_corr != ctxs[0]->p.n_corr) return QSA_E_INVALID;
    if (!c->plasma_loaded) return QSA_E_STATE;
    for (int k = 0; k < i; ++k)
      if (ctxs[k] == c) return QSA_E_INVALID;
  }
  qsa_batch* b = new qsa_batch();
  b->ctxs.assign(ctxs, ctxs + n_ctx);
  b->precision = ctxs[0]->p.precision;
  b->ws = reinterpret_cast<char*>(dev_ws);
  b->user = reinterpret_cast<hipStream_t>(hip_stream);
  if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess) {
    delete b;
    return QSA_E_DEVICE;
  }
  // lane table: one descriptor per context
  std::vector<char> host(qsa_batch_workspace_bytes(n_ctx), 0);
  for (int i = 0; i < n_ctx; ++i) {
    if (b->precision == QSA_FP32) {
      const Lane<float> l = Engine<float>::make_lane(ctxs[i]);
      std::memcpy(host.data() + i * sizeof(Lane<float>), &l, sizeof(l));
    } else {
      const Lane<double> l = Engine<double>::make_lane(ctxs[i]);
      std::memcpy(host.data() + i * sizeof(Lane<double>), &l, sizeof(l));
    }
  }
  if (hipMemcpyAsync(b->ws, host.data(), host.size(), hipMemcpyHostToDevice, b->stream) != hipSuccess ||
      hipStreamSynchronize(b->stream) != hipSuccess) {
    delete b;
    return QSA_E_DEVICE;
  }
  *out = b;
  return QSA_OK;
}

static qsa_status batch_call(qsa_batch* b, int32_t n_steps, bool push) {
  qsa_ctx* c = b->ctxs[0];   // error reporting
  for (qsa_ctx* m : b->ctxs)
    if (m->sticky != QSA_OK) return m->sticky;
  HIP_OK(hipEventRecord(b->ev_in, b->user));
  HIP_OK(hipStreamWaitEvent(b->stream, b->ev_in, 0));
  hipGraphExec_t* gx = push ? &b->gx_step : &b->gx_sweep;
  auto body = [&] { return b->precision == QSA_FP32 ? batch_run<float>(b, push) : batch_run<double>(b, push); };
  const bool graphs = b->use_graphs && c->timing_class < 0;
  if (graphs && !*gx) {
    if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) == hipSuccess) {
      const qsa_status st = body();
      hipGraph_t graph = nullptr;
      const hipError_t e = hipStreamEndCapture(b->stream, &graph);
      hipError_t ei = hipErrorUnknown;
      if (st == QSA_OK && e == hipSuccess) ei = hipGraphInstantiate(gx, graph, nullptr, nullptr, 0);
      if (graph) (void)hipGraphDestroy(graph);
      if (st != QSA_OK) return st;
      if (e != hipSuccess || ei != hipSuccess) {
        (void)hipGetLastError();
        *gx = nullptr;
        b->use_graphs = false;
      }
    } else {
      (void)hipGetLastError();
      b->use_graphs = false;
    }
  }
  for (int i = 0; i < n_steps; ++i) {
    if (graphs && *gx) {
      HIP_OK(hipGraphLaunch(*gx, b->stream));
      for (qsa_ctx* m : b->ctxs) m->swept = true;
    } else {
      const qsa_status st = body();
      if (st != QSA_OK) return st;
    }
  }
  HIP_OK(hipEventRecord(b->ev_out, b->stream));
  HIP_OK(hipStreamWaitEvent(b->user, b->ev_out, 0));
  return QSA_OK;
}

qsa_status qsa_batch_sweep(qsa_batch* b) {
  if (!b) return QSA_E_INVALID;
  return batch_call(b, 1, false);
}

qsa_status qsa_batch_step(qsa_batch* b, int32_t n_steps) {
  if (!b || n_steps < 0) return QSA_E_INVALID;
  if (n_steps == 0) return QSA_OK;
  return batch_call(b, n_steps, true);
}

qsa_status qsa_batch_sync(qsa_batch* b) {
  if (!b) return QSA_E_INVALID;
  {
    qsa_ctx* c = b->ctxs[0];
    HIP_OK(hipStreamSynchronize(b->stream));
  }
  for (qsa_ctx* c : b->ctxs) {
    const qsa_status st = qsa_sync(c);
    if (st != QSA_OK) return st;
  }
  return QSA_OK;
}

qsa_status qsa_batch_destroy(qsa_batch* b) {
  delete b;
  return QSA_OK;
}

qsa_status qsa_destroy(qsa_ctx* c) {
  delete c;
  return QSA_OK;
}

const char* qsa_status_string(qsa_status s) {
  switch (s) {
    case QSA_OK: return "ok";
    case QSA_E_INVALID: return "invalid argument";
    case QSA_E_NOMEM: return "workspace too small";
    case QSA_E_DEVICE: return "HIP runtime error";
    case QSA_E_BREAKDOWN: return "quasistatic breakdown (1 + psi <= 1e-3) or non-finite plasma state";
    case QSA_E_NONFINITE: return "non-finite input value";
    case QSA_E_STATE: return "call out of order";
  }
  return "unknown status";
}

const char* qsa_last_error(const qsa_ctx* c) { return c ? c->err.c_str() : "null context"; }

}  // extern "C"
