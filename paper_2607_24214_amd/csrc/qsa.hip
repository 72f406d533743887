// Host runtime and C ABI of the QSA slice sweep (see include/qsa.h).
//
// The context carves every device array out of the caller's workspace, keeps
// the host-side state (loaded particle counts, error state) and enqueues the
// kernels of qsa_kernels.h on the caller's stream.  One sweep is
// 4 + 4 + 4K + 1 dependent launches per xi slice.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/qsa.h"
#include "qsa_kernels.h"
#include "qsa_linear.h"
#include "qsa_dirichlet.h"
#include "qsa_adjoint.h"

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

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Adjoint grid scratch indices (each [ny][nx]).
enum {
  AG_S = 0,              // forward: rho - J_z of the slice
  AG_JF0,                // forward J (x, y, z) of slice j: AG_JF0 + 3 (j & 1) + c
  AG_JT = AG_JF0 + 6,    // predictor J_perp (x, y)
  AG_PSIT = AG_JT + 2,   // psi extrapolated to j + 1
  AG_ZERO,               // zeros (fields before slice 0)
  AG_SINK,               // 7 write-only grids: adjoints of fields before slice 0
  AA_JZ = AG_SINK + 7,   // reverse: J_z adjoint of the slice
  AA_PSIT,               // adjoint of the extrapolated psi
  AA_JB0,                // J_perp adjoint (x, y) of slice j: AA_JB0 + 2 (j & 1) + c
  AA_DB = AA_JB0 + 4,    // adjoint of the predictor's current difference (x, y)
  AA_BP0 = AA_DB + 2,    // two pairs of B_perp iterate adjoints (x, y)
  AA_S = AA_BP0 + 4,     // adjoint of rho - J_z
  AG_COUNT
};

struct AdjLayout {
  int steps = 0, nseg = 0, ck_len = 0;
  size_t state[QSA_MAX_SPECIES] = {};   // per species: bytes of one beam state in the tape
  size_t beam[QSA_MAX_SPECIES] = {};    // tape base per species
  size_t bin[QSA_MAX_SPECIES] = {}, w0[QSA_MAX_SPECIES] = {}, bb[QSA_MAX_SPECIES][7] = {};
  size_t fields = 0, biter = 0, src = 0, srcb = 0, fb = 0;
  size_t ck = 0, ck_bytes = 0;
  size_t segY = 0, segYt = 0, Y[2] = {}, Yb[2] = {};
  size_t grids = 0, work = 0, ktab = 0, sc = 0, sums = 0, part = 0, grad = 0, amps = 0;
};


// Carve the adjoint arrays after the forward workspace.
void adjoint_layout(const qsa_params& p, size_t& off, AdjLayout& A) {
  const size_t rs = (p.precision == QSA_FP32) ? 4 : 8;
  const size_t nperp = (size_t)p.nx * p.ny;
  const size_t np = (size_t)p.n_plasma;
  const size_t plane = (size_t)p.nxi * nperp;
  const int K = std::max(p.n_corr, 0);
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes);
    return o;
  };
  A.steps = p.adjoint_steps;
  if (A.steps <= 0) return;
  A.ck_len = (p.ckpt_every > 0) ? p.ckpt_every : QSA_ADJ_CKPT;
  A.nseg = (p.nxi + A.ck_len - 1) / A.ck_len;
  for (int s = 0; s < p.n_species; ++s) {
    const size_t cap = (size_t)p.beam_capacity[s];
    A.state[s] = 6 * align_up(cap * rs) + align_up(cap * 8);
    A.beam[s] = take(A.state[s] * (size_t)(A.steps + 1));
    A.bin[s] = take(cap * sizeof(int));
    A.w0[s] = take(cap * rs);
    for (int k = 0; k < 7; ++k) A.bb[s][k] = take(cap * rs);
  }
  A.fields = take((size_t)(A.steps + 1) * N_STORED * plane * rs);
  A.biter = take((size_t)(A.steps + 1) * std::max(K, 1) * 2 * plane * rs);
  A.src = take(4 * plane * rs);
  A.srcb = take(4 * plane * rs);
  A.fb = take(N_STORED * plane * rs);
  A.ck_bytes = align_up(4 * np * rs);
  A.ck = take((size_t)(A.steps + 1) * A.nseg * A.ck_bytes);
  A.segY = take((size_t)A.ck_len * 4 * np * rs);
  A.segYt = take((size_t)A.ck_len * std::max(K, 1) * 4 * np * rs);
  for (int i = 0; i < 2; ++i) {
    A.Y[i] = take(4 * np * rs);
    A.Yb[i] = take(4 * np * rs);
  }
  A.grids = take((size_t)AG_COUNT * nperp * rs);
  A.work = take((size_t)SPEC_IN * nperp * 2 * rs);
  A.ktab = take((size_t)(p.nx / 2 + 1) * p.ny * 4 * sizeof(double));
  A.sc = take(64 * sizeof(double));
  A.sums = take(2 * (size_t)p.nxi * sizeof(double));
  A.part = take(((np + 255) / 256 + (size_t)p.ny) * sizeof(double));   // per-block / per-row partial sums
  A.grad = take(4096 * sizeof(double));
  A.amps = take(4096 * sizeof(double));
}

// Byte offsets of one sweep's working set: plasma state, sources, fields and
// the spectral rings.  Set 0 is the only set without pipelining; with beam
// steps in flight, lane k of a group works in set k.
struct SetLayout {
  size_t pl[4], pl2[4];
  size_t qw[2];   // plasma relative weights of the two buffer sets (plasma_weights)
  size_t cell_of, count, bsum, prow, ppart;
  size_t src, fields, half, dep, rowspec, colout, jring, jz, bring, ode;
  size_t ring;   // slab ring of the deposits this set receives from the lane before it
  size_t fpack;  // packed fields of the beam push
  int pack_ring;  // slices fpack holds
  size_t hist;   // new-row count matrix of this set's slab pushes, and row starts
  size_t base;
  size_t rk2c;   // RK2 cache of the slice's plasma particles (8 values each)
};

// Byte offsets of every device array inside the workspace.
struct Layout {
  size_t twx, twy, kx2, kdx, ky2, kdy;
  size_t tmpl[4];
  size_t tmpl_qw;                   // template relative weights (plasma_weights)
  size_t ion;                       // ion density at the nodes (plasma_weights)
  int nset;                         // working sets (beam steps in flight)
  bool lean;                        // steps in flight without a second copy of the beam
  SetLayout set[QSA_MAX_PIPELINE];
  size_t rowoff[QSA_MAX_SPECIES];   // slab partition of the sorted beam (pipelining)
  size_t doff[QSA_MAX_SPECIES];     // sort-key offsets into perm of the current deposit
  size_t cnt_next[QSA_MAX_SPECIES]; // key counts of the beam's current positions (see keys())
  size_t key[QSA_MAX_SPECIES], perm[QSA_MAX_SPECIES];
  size_t cursor, scan64;
  size_t beam[QSA_MAX_SPECIES][8];  // x, y, ux, uy, uz, w (real), xi (double), id (int64, pipelining)
  size_t snap[QSA_MAX_SPECIES][8];  // sort target and the beam at the start of a pipelined group
  size_t err, emit, lane, pipe;
  size_t kvalid;                    // int: cnt_next holds the key counts of the beam as it stands
  size_t diag;                      // diagnostics: 7 doubles per slice
  AdjLayout adj;                    // adjoint tapes and arrays (adjoint_steps > 0)
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

// Blocks of the key, permutation and gather passes over n beam particles.
unsigned beam_blocks(int64_t n) { return (unsigned)((n + 256 * QSA_BEAM_UNROLL - 1) / (256 * QSA_BEAM_UNROLL)); }

int pipeline_depth(const qsa_params& p) { return std::max(1, (int)p.pipeline); }

// bytes of one node's packed beam-push fields (element size rs)
size_t pack_stride_bytes(size_t rs) { return rs == 8 ? 6 * 8 : 8 * 4; }

Layout make_layout(const qsa_params& p) {
  const size_t rs = (p.precision == QSA_FP32) ? 4 : 8;
  const size_t cs = 2 * rs;
  const size_t nperp = (size_t)p.nx * p.ny;
  const size_t nxh = (size_t)p.nx / 2 + 1;
  const size_t spec = (size_t)p.ny * nxh * cs;
  Layout L{};
  Carver c;
  L.twx = c.take(p.nx * cs);
  L.twy = c.take(p.ny * cs);
  L.kx2 = c.take(nxh * rs);
  L.kdx = c.take(nxh * rs);
  L.ky2 = c.take(p.ny * rs);
  L.kdy = c.take(p.ny * rs);
  // plasma x, y in float64 for either precision; u_x, u_y in R
  for (int i = 0; i < 4; ++i) L.tmpl[i] = c.take(p.n_plasma * (i < 2 ? 8 : rs));
  L.tmpl_qw = p.plasma_weights ? c.take(p.n_plasma * rs) : 0;
  L.ion = p.plasma_weights ? c.take(nperp * rs) : 0;
  L.nset = pipeline_depth(p);
  L.lean = L.nset > 1 && p.lean_pipeline;
  for (int k = 0; k < L.nset; ++k) {
    SetLayout& S = L.set[k];
    for (int i = 0; i < 4; ++i) S.pl[i] = c.take(p.n_plasma * (i < 2 ? 8 : rs));
    for (int i = 0; i < 4; ++i) S.pl2[i] = c.take(p.n_plasma * (i < 2 ? 8 : rs));
    for (int i = 0; i < 2; ++i) S.qw[i] = p.plasma_weights ? c.take(p.n_plasma * rs) : 0;
    S.cell_of = c.take(p.n_plasma * sizeof(int));
    S.count = c.take(nperp * sizeof(int));
    S.bsum = c.take(256 * sizeof(int));
    S.prow = c.take((p.ny + 1) * sizeof(int));
    S.ppart = c.take((size_t)p.ny * 4 * 3 * p.nx * rs);
    S.src = c.take(4 * (size_t)p.nxi * nperp * rs);
    S.fields = c.take((size_t)N_STORED * p.nxi * nperp * rs);
    S.half = c.take((size_t)N_HALF * nperp * rs);
    S.dep = c.take(3 * nperp * rs);
    S.rowspec = c.take(4 * spec);
    S.colout = c.take(4 * spec);
    S.jring = c.take(4 * spec);
    S.jz = c.take(spec);
    S.bring = c.take(6 * spec);
    S.ode = c.take(2 * sizeof(double));
    // two slabs x ny cell rows x (2 node slices x 2 node rows x 4 sources x nx)
    S.ring = (k > 0) ? c.take(2 * (size_t)p.ny * 2 * 2 * 4 * p.nx * rs) : 0;
    S.hist = (L.nset > 1) ? c.take((size_t)QSA_MAX_SPECIES * p.ny * p.ny * sizeof(int)) : 0;
    // packed push fields: a ring of slices with steps in flight, every slice
    // without (the beam push then reads them after the sweep)
    S.pack_ring = (L.nset > 1) ? QSA_PACK_RING : (p.no_field_pack ? 0 : p.nxi);
    S.fpack = S.pack_ring ? c.take((size_t)S.pack_ring * nperp * pack_stride_bytes(rs)) : 0;
    S.base = (L.nset > 1) ? c.take((size_t)QSA_MAX_SPECIES * (p.ny + 1) * sizeof(int)) : 0;
    S.rk2c = c.take(p.n_plasma * 8 * rs);
  }
  const size_t nrows = (size_t)p.nxi * p.ny;
  const size_t nkeys = nrows * (nx_chunks_of(p.nx)) + 1;   // sort keys, the last for inert particles
  for (int s = 0; s < QSA_MAX_SPECIES; ++s) {
    const size_t cap = (s < p.n_species) ? (size_t)p.beam_capacity[s] : 0;
    const bool used = s < p.n_species;
    L.rowoff[s] = c.take((nrows + 2) * sizeof(int64_t));
    L.doff[s] = used ? c.take((nkeys + 2) * sizeof(int64_t)) : 0;
    // key counts of the next deposit, made by the pushes beside the slice loop
    L.cnt_next[s] = (used && L.nset == 1) ? c.take((nkeys + 2) * sizeof(int64_t)) : 0;
    L.key[s] = (L.nset > 1) ? c.take(cap * sizeof(int)) : 0;   // kept only for steps in flight
    L.perm[s] = c.take(cap * sizeof(int));
  }
  L.cursor = c.take((nkeys + 2) * sizeof(int64_t));
  L.scan64 = c.take(((nkeys + 2) / 1024 + 64) * 2 * sizeof(int64_t));
  for (int s = 0; s < QSA_MAX_SPECIES; ++s) {
    const size_t cap = (s < p.n_species) ? (size_t)p.beam_capacity[s] : 0;
    for (int k = 0; k < 6; ++k) L.beam[s][k] = c.take(cap * rs);
    L.beam[s][6] = c.take(cap * 8);
    if (L.nset > 1 && !L.lean) {
      L.beam[s][7] = c.take(cap * 8);
      for (int k = 0; k < 6; ++k) L.snap[s][k] = c.take(cap * rs);
      L.snap[s][6] = c.take(cap * 8);
      L.snap[s][7] = c.take(cap * 8);
    }
  }
  L.err = c.take(sizeof(int));
  L.kvalid = c.take(sizeof(int));
  L.emit = c.take(nperp * sizeof(double));
  L.diag = c.take(7 * (size_t)p.nxi * sizeof(double));
  L.lane = c.take(L.nset * sizeof(Lane<double>));
  L.pipe = c.take(L.nset * sizeof(PipeBeam<double>));
  adjoint_layout(p, c.off, L.adj);
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
  if ((int64_t)p->nxi * p->ny * (nx_chunks_of(p->nx)) > ((int64_t)1 << 30))
    return "nxi * ny * nx / 8 must be <= 2^30";
  if (p->pipeline < 0 || p->pipeline > QSA_MAX_PIPELINE) return "pipeline must be in [0, 16]";
  if (p->adjoint_steps < 0 || p->adjoint_steps > 1024) return "adjoint_steps must be in [0, 1024]";
  if (p->ckpt_every < 0 || p->ckpt_every > p->nxi) return "ckpt_every must be in [0, nxi]";
  if (p->no_field_pack != 0 && p->no_field_pack != 1) return "no_field_pack must be 0 or 1";
  if (p->plasma_weights != 0 && p->plasma_weights != 1) return "plasma_weights must be 0 or 1";
  if (p->lean_pipeline != 0 && p->lean_pipeline != 1) return "lean_pipeline must be 0 or 1";
  if (!std::isfinite(p->b0z)) return "b0z must be finite";
  if (p->b0z != 0.0 && p->adjoint_steps > 0) return "b0z must be 0 with adjoint_steps > 0 (the adjoint takes no external field)";
  if (!(p->ion_m >= 0.0) || !std::isfinite(p->ion_m)) return "ion_m must be finite and >= 0";
  if (p->ion_m > 0.0 && !p->plasma_weights) return "mobile ions (ion_m > 0) need plasma_weights = 1";
  if (p->ion_m > 0.0 && (p->ion_z < 1 || p->ion_z > 64)) return "ion_z must be in [1, 64]";
  if (p->lean_pipeline && p->pipeline > 1 && p->adjoint_steps > 0)
    return "lean_pipeline: the adjoint's bins follow the load order, which a lean pipeline does not keep";
  if (p->lean_pipeline && p->pipeline > 1) {
    // the group's sort gathers every beam array through the sources and
    // stored fields of working set 0
    const size_t rs = (p->precision == QSA_FP32) ? 4 : 8;
    const size_t scratch = (size_t)(4 + N_STORED) * p->nxi * p->ny * p->nx * rs;
    for (int s = 0; s < p->n_species; ++s)
      if ((size_t)std::max<int64_t>(p->beam_capacity[s], 0) * 8 > scratch)
        return "lean_pipeline: a beam capacity times 8 bytes exceeds the sources and fields of one working set";
  }
  for (int s = 0; s < p->n_species; ++s) {
    if (p->beam_capacity[s] < 0 || p->beam_capacity[s] > INT32_MAX) return "beam capacity must be in [0, 2^31)";
    if (!(p->species[s].M > 0)) return "species mass must be > 0";
  }
  return nullptr;
}

}  // namespace

#define QSA_GEV 4   // events per ring between the slice loop and the beam stream
#define QSA_BEAM_CHUNK 8    // slabs per beam deposit and push beside the slice loop
#define QSA_BEAM_AHEAD 2    // chunks deposited ahead of the slice loop
#define QSA_PUSH_BLOCKS 2048   // grid of a key-range push
// Host-side bound on the work enqueued ahead of the device: a slice loop
// enqueues about QSA_TICK_LAUNCHES launches per tick, and the host waits
// (spinning on an event) before it runs more than 2 QSA_THROTTLE_TICKS
// ticks ahead.  A full hardware queue otherwise parks the enqueuing thread
// in a blocking wait that was measured to resume only at whole seconds
// (a 512x512x2048 step: exactly 1.000 s however fast the kernels got).
// Graph replays cannot be throttled, so slice loops longer than
// QSA_GRAPH_MAX_LAUNCHES launches are enqueued directly.
#define QSA_THROTTLE_TICKS 16
#define QSA_TEV 4
#define QSA_TICK_LAUNCHES 26
#define QSA_GRAPH_MAX_LAUNCHES 4096

struct qsa_ctx {
  qsa_params p;
  Layout L;
  char* ws = nullptr;
  hipStream_t user = nullptr;     // the caller's stream
  hipStream_t stream = nullptr;   // the library's work stream (ordered after `user` per call)
  hipStream_t bstream = nullptr;  // beam work of steps in flight, overlapping the slice loop
  int beside_blocks = 0;          // workgroups per beam launch beside the slice loop (0: the work's)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipEvent_t gfork[QSA_GEV] = {}, gdone[QSA_GEV] = {};   // slice loop -> beam work -> slice loop
  hipEvent_t tev[QSA_TEV] = {};   // enqueue throttle (see QSA_THROTTLE_TICKS)
  hipGraphExec_t gx_step = nullptr, gx_sweep = nullptr;   // captured beam step / sweep
  bool use_graphs = true;
  bool beam_beside = false;   // one step at a time: the beam work beside the slice loop
  int64_t resort_every = 0;   // one step at a time: the beam storage reordered by deposit key every n steps
  int64_t beam_steps = 0;     // beam steps since the last beam load (the re-sort's clock)
  bool resort_pending = false;   // the next deposit re-sorts the storage (direct launches only)
  bool pipe_ok = true;   // off after a drift violation, until the next beam load
  int pipe_max = 1;      // beam steps in flight when pipelining (<= L.nset)
  int tune_nt = 0;       // threads per plasma-row block (0: from the particles per row)
  int tune_rt = 0;       // threads per row-transform block (0: min(256, max(64, nx/2)))
  int tune_ct = 0;       // threads per column transform (0: QSA_COL_TPT)
  int col_lds_max = 0;   // LDS the column passes may take (opted in)
  int cur_set = 0;       // working set holding the last sweep's sources and fields
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
  bool event_pair() {
    if (ev_used + 2 <= events.size()) return true;
    if (events.size() >= (size_t)2 << 17) return false;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return false;
    if (hipEventCreate(&b) != hipSuccess) {
      (void)hipEventDestroy(a);
      return false;
    }
    events.push_back(a);
    events.push_back(b);
    return true;
  }
  void tstart(int k) {
    if (k != timing_class || !event_pair()) return;
    (void)hipEventRecord(events[ev_used], stream);
  }
  // Events for one launch of class k when that class is timed: the launch
  // records them at the kernel's own start and end.
  bool timing_pair(int k, hipEvent_t* a, hipEvent_t* b) {
    if (k != timing_class || !event_pair()) return false;
    *a = events[ev_used];
    *b = events[ev_used + 1];
    ev_used += 2;
    return true;
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
    // finish all work (and the graphs' use of the workspace) before the
    // graphs and streams go, so that the caller can free the workspace
    if (bstream) (void)hipStreamSynchronize(bstream);
    if (stream) (void)hipStreamSynchronize(stream);
    drop_graphs();
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    for (int i = 0; i < QSA_GEV; ++i) {
      if (gfork[i]) (void)hipEventDestroy(gfork[i]);
      if (gdone[i]) (void)hipEventDestroy(gdone[i]);
    }
    for (int i = 0; i < QSA_TEV; ++i)
      if (tev[i]) (void)hipEventDestroy(tev[i]);
    if (bstream) (void)hipStreamDestroy(bstream);
    if (stream) (void)hipStreamDestroy(stream);
  }
};


// Slice loops short enough to be replayed from a graph (see
// QSA_GRAPH_MAX_LAUNCHES).
static bool graph_fits(int nxi) { return (int64_t)nxi * QSA_TICK_LAUNCHES <= QSA_GRAPH_MAX_LAUNCHES; }

// The key counts the pushes made (cnt_next) no longer describe the beam
// (something else moved or reloaded it), or they do again: a flag on the
// device, written in stream order (also from captured graphs).
static void invalidate_counts(qsa_ctx* c) {
  hipLaunchKernelGGL(k_set_flag, dim3(1), dim3(64), 0, c->stream, reinterpret_cast<int*>(c->ws + c->L.kvalid), 0);
}
static void counts_made(qsa_ctx* c) {
  bool all = c->p.n_species > 0;
  for (int s = 0; s < c->p.n_species; ++s) all = all && c->L.cnt_next[s] != 0;
  hipLaunchKernelGGL(k_set_flag, dim3(1), dim3(64), 0, c->stream, reinterpret_cast<int*>(c->ws + c->L.kvalid),
                     all ? 1 : 0);
}

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
    // finish the batch's work before its graphs and stream go
    if (stream) (void)hipStreamSynchronize(stream);
    if (gx_step) (void)hipGraphExecDestroy(gx_step);
    if (gx_sweep) (void)hipGraphExecDestroy(gx_sweep);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (stream) (void)hipStreamDestroy(stream);
  }
};

// Launch a kernel; when its class is being timed, with events recorded at
// the kernel's own start and end.
#define QSA_LAUNCH(ctx, cls, kern, grid, block, shmem, st, ...)                      \
  do {                                                                               \
    hipEvent_t qe0_ = nullptr, qe1_ = nullptr;                                       \
    if ((ctx)->timing_pair((cls), &qe0_, &qe1_))                                     \
      hipExtLaunchKernelGGL(kern, grid, block, shmem, st, qe0_, qe1_, 0, __VA_ARGS__); \
    else                                                                             \
      hipLaunchKernelGGL(kern, grid, block, shmem, st, __VA_ARGS__);                 \
  } while (0)

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
    g.inv_dxd = 1.0 / p.dx;
    g.inv_dyd = 1.0 / p.dy;
    g.lxd = p.nx * p.dx;
    g.lyd = p.ny * p.dy;
    g.inv_lxd = 1.0 / (p.nx * p.dx);
    g.inv_lyd = 1.0 / (p.ny * p.dy);
    g.b0z = (R)p.b0z;
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
      a.key[s] = c->L.key[s] ? c->at<int>(c->L.key[s]) : nullptr;
      a.perm[s] = c->at<int>(c->L.perm[s]);
      a.doff[s] = c->at<int64_t>(c->L.doff[s]);
      a.zq[s] = (R)(p.species[s].Z / (p.dx * p.dy * p.dxi));
    }
    a.inv_dxi = 1.0 / p.dxi;
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

  // Sort keys of species s and their exclusive offsets in doff[s];
  // cursor <- doff[s].
  static qsa_status keys(qsa_ctx* c, int s) {
    const qsa_params& p = c->p;
    const Geo<R> g = geo(p);
    const int64_t nkeys = (int64_t)p.nxi * p.ny * (nx_chunks_of(p.nx)) + 1;
    int64_t* off = c->at<int64_t>(c->L.doff[s]);
    const int64_t n = c->beam_n[s];
    if (c->L.cnt_next[s]) {
      // the counts the last pushes made when they are valid (nothing has
      // moved the beam since; a flag on the device, so that a captured graph
      // decides at each replay), else counted here
      const int* valid = c->at<int>(c->L.kvalid);
      hipLaunchKernelGGL(k_counts_or_zero, dim3(fill_blocks(nkeys + 1)), dim3(256), 0, c->stream, valid,
                         (const int64_t*)c->at<int64_t>(c->L.cnt_next[s]), off, nkeys + 1);
      if (n > 0)
        hipLaunchKernelGGL(k_beam_keys<R>, dim3(beam_blocks(n)), dim3(256), 0, c->stream, g,
                           beam_dep_args(c), s, n, off, valid);
    } else {
      hipLaunchKernelGGL(k_fill<int64_t>, dim3(fill_blocks(nkeys + 1)), dim3(256), 0, c->stream, off, nkeys + 1,
                         (int64_t)0);
      if (n > 0)
        hipLaunchKernelGGL(k_beam_keys<R>, dim3(beam_blocks(n)), dim3(256), 0, c->stream, g,
                           beam_dep_args(c), s, n, off, (const int*)nullptr);
    }
    HIP_OK(hipGetLastError());
    qsa_status st = scan64(c, off, nkeys + 1, c->at<int64_t>(c->L.scan64));
    if (st != QSA_OK) return st;
    HIP_OK(hipMemcpyAsync(c->ws + c->L.cursor, off, (nkeys + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice,
                          c->stream));
    return QSA_OK;
  }

  // Reorder the particles of species s by cell row (pipelining only): the
  // slab partition rowoff[s] then holds every slab's index range.
  static qsa_status sort_species(qsa_ctx* c, int s) {
    const qsa_params& p = c->p;
    const Layout& L = c->L;
    const int64_t nrows = (int64_t)p.nxi * p.ny;
    const int64_t n = c->beam_n[s];
    qsa_status st = keys(c, s);
    if (st != QSA_OK) return st;
    hipLaunchKernelGGL(k_row_starts<R>, dim3((unsigned)((nrows + 2 + 255) / 256)), dim3(256), 0, c->stream,
                       geo(p), (const int64_t*)c->at<int64_t>(L.doff[s]), c->at<int64_t>(L.rowoff[s]));
    HIP_OK(hipGetLastError());
    if (n == 0) return QSA_OK;
    if (L.lean) {
      // no second copy of the beam: the permutation to key order, then
      // every array gathered through it in place (via set 0's scratch)
      hipLaunchKernelGGL(k_beam_perm<R>, dim3(beam_blocks(n)), dim3(256), 0, c->stream, geo(p), beam_dep_args(c), s,
                         n, c->at<int64_t>(L.cursor));
      HIP_OK(hipGetLastError());
      return resort_species(c, s);
    }
    BeamMove<R> m;
    for (int k = 0; k < 6; ++k) {
      m.src[k] = c->at<R>(L.beam[s][k]);
      m.dst[k] = c->at<R>(L.snap[s][k]);
    }
    m.sxi = c->at<double>(L.beam[s][6]);
    m.dxi = c->at<double>(L.snap[s][6]);
    m.sid = c->at<int64_t>(L.beam[s][7]);
    m.did = c->at<int64_t>(L.snap[s][7]);
    m.key = c->at<int>(L.key[s]);
    m.cur = c->at<int64_t>(L.cursor);
    m.n = n;
    hipLaunchKernelGGL(k_beam_sort<R>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, m);
    HIP_OK(hipGetLastError());
    for (int k = 0; k < 8; ++k)
      HIP_OK(hipMemcpyAsync(c->ws + L.beam[s][k], c->ws + L.snap[s][k], (size_t)n * (k < 6 ? sizeof(R) : 8),
                            hipMemcpyDeviceToDevice, c->stream));
    return QSA_OK;
  }

  // After a load: identities, and the sort by cell row when pipelining.
  static qsa_status loaded(qsa_ctx* c, int s) {
    if (c->L.nset < 2) return QSA_OK;
    const int64_t n = c->beam_n[s];
    if (n > 0 && !c->L.lean) {
      hipLaunchKernelGGL(k_iota64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream,
                         c->at<int64_t>(c->L.beam[s][7]), n);
      HIP_OK(hipGetLastError());
    }
    return sort_species(c, s);
  }

  static qsa_status sort_all(qsa_ctx* c) {
    for (int s = 0; s < c->p.n_species; ++s) {
      const qsa_status st = sort_species(c, s);
      if (st != QSA_OK) return st;
    }
    return QSA_OK;
  }

  // Beam sources: particles grouped by cell row (keys, their offsets and a
  // permutation), each row deposited by one block into the dense sources
  // (four launches by the parity of the row, see k_beam_rows).
  // sorted: the storage is in key order already, with the identity in perm
  // and the key offsets in doff (a lean group's sort has just made them).
  static qsa_status beam_perm_all(qsa_ctx* c, const Geo<R>& g, bool sorted = false) {
    const qsa_params& p = c->p;
    const bool resort = c->resort_pending;   // set by a single step that is due for it
    c->resort_pending = false;
    for (int s = 0; s < p.n_species && !sorted; ++s) {
      qsa_status st = keys(c, s);
      if (st != QSA_OK) return st;
      const int64_t n = c->beam_n[s];
      if (n > 0)
        hipLaunchKernelGGL(k_beam_perm<R>, dim3(beam_blocks(n)), dim3(256), 0, c->stream, g,
                           beam_dep_args(c), s, n, c->at<int64_t>(c->L.cursor));
      if (resort && (st = resort_species(c, s)) != QSA_OK) return st;
    }
    // consumed: the next push counts afresh
    const int64_t nkeys = (int64_t)p.nxi * p.ny * (nx_chunks_of(p.nx)) + 1;
    for (int s = 0; s < p.n_species; ++s)
      if (c->L.cnt_next[s])
        hipLaunchKernelGGL(k_fill<int64_t>, dim3(fill_blocks(nkeys + 1)), dim3(256), 0, c->stream,
                           c->at<int64_t>(c->L.cnt_next[s]), nkeys + 1, (int64_t)0);
    invalidate_counts(c);
    HIP_OK(hipGetLastError());
    return QSA_OK;
  }

  // Bytes of the step's sources and stored fields (adjacent in the workspace):
  // the scratch of the storage re-sort, which runs before a step's deposit
  // overwrites both.
  static size_t resort_scratch(const qsa_ctx* c) {
    const qsa_params& p = c->p;
    const size_t plane = (size_t)p.nxi * p.nx * p.ny * sizeof(R);
    const SetLayout& S = c->L.set[0];
    return S.fields + N_STORED * plane - S.src;
  }

  // The storage of species s reordered by deposit key (one step at a time),
  // right after the step's permutation to key order is made: as particles
  // drift across cells their storage order departs from the order the
  // deposit gathers them in, and the gathers (and the push's field reads)
  // lose coalescing.  Every beam array is gathered through the permutation
  // into the scratch (two float arrays per pass where it holds two) and
  // copied back; the permutation becomes the identity.  The key offsets
  // and counts stay valid (no particle moves).
  static qsa_status resort_species(qsa_ctx* c, int s) {
    const int64_t n = c->beam_n[s];
    if (n == 0) return QSA_OK;
    char* tmp = c->ws + c->L.set[0].src;
    const int64_t npad = (n + 63) / 64 * 64;   // the second plane 256-byte aligned
    const bool two = 2 * (size_t)npad * sizeof(R) <= resort_scratch(c);
    const dim3 grid(beam_blocks(n));
    int* perm = c->at<int>(c->L.perm[s]);
    auto copy_back = [&](char* dst, const char* src, int64_t bytes) {
      const int64_t blocks = std::min<int64_t>(std::max<int64_t>(((bytes >> 4) + 255) / 256, 1), 1 << 18);
      hipLaunchKernelGGL(k_copy_bytes, dim3((unsigned)blocks), dim3(256), 0, c->stream,
                         (const unsigned char*)src, (unsigned char*)dst, bytes);
    };
    R* t0 = reinterpret_cast<R*>(tmp);
    R* t1 = t0 + npad;
    for (int k = 0; k < 6; k += two ? 2 : 1) {
      R* a0 = c->at<R>(c->L.beam[s][k]);
      R* a1 = two ? c->at<R>(c->L.beam[s][k + 1]) : nullptr;
      hipLaunchKernelGGL(k_gather_perm<R>, grid, dim3(256), 0, c->stream, (const R*)a0, (const R*)a1, t0, t1,
                         (const int*)perm, n);
      copy_back((char*)a0, (const char*)t0, n * (int64_t)sizeof(R));
      if (two) copy_back((char*)a1, (const char*)t1, n * (int64_t)sizeof(R));
    }
    double* xi = c->at<double>(c->L.beam[s][6]);
    hipLaunchKernelGGL(k_gather_perm<double>, grid, dim3(256), 0, c->stream, (const double*)xi,
                       (const double*)nullptr, (double*)tmp, (double*)nullptr, (const int*)perm, n);
    copy_back((char*)xi, (const char*)tmp, n * (int64_t)sizeof(double));
    hipLaunchKernelGGL(k_iota32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, perm, n);
    HIP_OK(hipGetLastError());
    return QSA_OK;
  }

  // Deposit the slabs [jlo, jhi) into src (on stream st), with at most
  // max_blocks workgroups per launch (0: one per cell row).
  static qsa_status deposit_slabs(qsa_ctx* c, const Geo<R>& g, hipStream_t st, R* src, int jlo, int jhi,
                                  int max_blocks = 0) {
    const BeamDepArgs<R> a = beam_dep_args(c);
    for (int colour = 0; colour < 4; ++colour) {
      const int nb = beam_colour_rows(jlo, jhi, c->p.ny, colour);
      const int grid = (max_blocks > 0) ? std::min(nb, max_blocks) : nb;
      if (nb > 0)
        QSA_LAUNCH(c, QSA_K_BEAM_DEPOSIT, k_beam_rows<R>, dim3(grid), dim3(BeamRowBlock<R>::THREADS),
                   2 * 2 * 4 * g.nx * sizeof(double), st, g, a, src, colour, jlo, jhi);
    }
    HIP_OK(hipGetLastError());
    return QSA_OK;
  }

  static qsa_status beam_deposit_all(qsa_ctx* c, const Geo<R>& g, bool sorted = false) {
    qsa_status st = beam_perm_all(c, g, sorted);
    if (st != QSA_OK) return st;
    R* src = c->at<R>(c->L.set[0].src);
    if ((st = fill(c, src, 4 * (int64_t)c->p.nxi * g.nperp, R(0))) != QSA_OK) return st;
    return deposit_slabs(c, g, c->stream, src, 0, c->p.nxi);
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
    a.fields = c->at<R>(c->L.set[0].fields);
    // every slice's packed fields (contexts without steps in flight), else
    // gathers from the stored planes
    const SetLayout& S0 = c->L.set[0];
    a.fpack = (S0.fpack && S0.pack_ring >= p.nxi) ? c->at<R>(S0.fpack) : nullptr;
    a.ring = S0.pack_ring;
    a.zq = (R)(p.species[s].Z / (p.dx * p.dy * p.dxi));
    a.qmh = (R)((double)p.species[s].Z / p.species[s].M * 0.5 * p.dt);
    a.dt = (R)p.dt;
    a.inv_dxi = 1.0 / p.dxi;
    a.xi_max = (double)(p.nxi - 1) * p.dxi;
    return a;
  }

  // ---- lanes ---------------------------------------------------------------
  // Device-pointer descriptor of this context's box for the per-slice kernels,
  // working in set k with a lag of k * QSA_PIPE_LAG slices.
  static Lane<R> make_lane(qsa_ctx* c, int k = 0) {
    const qsa_params& p = c->p;
    const Layout& L = c->L;
    const SetLayout& S = L.set[k];
    Lane<R> a;
    std::memset(&a, 0, sizeof(a));
    a.g = geo(p);
    a.lag = k * QSA_PIPE_LAG;
    a.np = (int)p.n_plasma;
    a.q = (R)(-p.plasma_w / (p.dx * p.dy));
    a.h = (R)p.dxi;
    a.kappa2 = (R)p.kappa2;
    a.fields = c->at<R>(S.fields);
    a.half = c->at<R>(S.half);
    a.src = c->at<R>(S.src);
    for (int i = 0; i < 2; ++i) {
      a.tpos[i] = c->at<double>(L.tmpl[i]);
      a.tmom[i] = c->at<R>(L.tmpl[2 + i]);
      a.pos[0][i] = c->at<double>(S.pl[i]);
      a.pos[1][i] = c->at<double>(S.pl2[i]);
      a.mom[0][i] = c->at<R>(S.pl[2 + i]);
      a.mom[1][i] = c->at<R>(S.pl2[2 + i]);
      a.qw[i] = p.plasma_weights ? c->at<R>(S.qw[i]) : nullptr;
    }
    a.tqw = p.plasma_weights ? c->at<R>(L.tmpl_qw) : nullptr;
    a.ion = p.plasma_weights ? c->at<R>(L.ion) : nullptr;
    a.ion_s = p.ion_m > 0.0 ? (R)(-(double)p.ion_z / p.ion_m) : R(0);
    a.twx = c->at<C2<R>>(L.twx);
    a.twy = c->at<C2<R>>(L.twy);
    a.kx2 = c->at<R>(L.kx2);
    a.kdx = c->at<R>(L.kdx);
    a.ky2 = c->at<R>(L.ky2);
    a.kdy = c->at<R>(L.kdy);
    a.err = c->at<int>(L.err);
    a.cell_of = c->at<int>(S.cell_of);
    a.count = c->at<int>(S.count);
    a.bsum = c->at<int>(S.bsum);
    a.prow = c->at<int>(S.prow);
    a.ppart = c->at<R>(S.ppart);
    a.dep = c->at<R>(S.dep);
    a.rowspec = c->at<C2<R>>(S.rowspec);
    a.colout = c->at<C2<R>>(S.colout);
    a.jring = c->at<C2<R>>(S.jring);
    a.jz = c->at<C2<R>>(S.jz);
    a.bring = c->at<C2<R>>(S.bring);
    a.ode = c->at<double>(S.ode);
    a.fpack = S.fpack ? c->at<R>(S.fpack) : nullptr;
    a.pack_ring = S.pack_ring;
    a.rk2c = c->at<R>(S.rk2c);
    return a;
  }

  // Beam push and hand-over of lane k of a pipelined group.
  static PipeBeam<R> make_pipe(qsa_ctx* c, int k) {
    const qsa_params& p = c->p;
    const Layout& L = c->L;
    PipeBeam<R> a;
    std::memset(&a, 0, sizeof(a));
    a.g = geo(p);
    a.lag = k * QSA_PIPE_LAG;
    a.ns = p.n_species;
    for (int s = 0; s < p.n_species; ++s) {
      a.x[s] = c->at<R>(L.beam[s][0]);
      a.y[s] = c->at<R>(L.beam[s][1]);
      a.ux[s] = c->at<R>(L.beam[s][2]);
      a.uy[s] = c->at<R>(L.beam[s][3]);
      a.uz[s] = c->at<R>(L.beam[s][4]);
      a.w[s] = c->at<R>(L.beam[s][5]);
      a.xi[s] = c->at<double>(L.beam[s][6]);
      a.rowoff[s] = c->at<int64_t>(L.rowoff[s]);
      a.tag[s] = L.key[s] ? c->at<int>(L.key[s]) : nullptr;
      a.perm[s] = c->at<int>(L.perm[s]);
      a.qmh[s] = (R)((double)p.species[s].Z / p.species[s].M * 0.5 * p.dt);
      a.zq[s] = (R)(p.species[s].Z / (p.dx * p.dy * p.dxi));
    }
    a.dt = (R)p.dt;
    a.inv_dxi = 1.0 / p.dxi;
    a.xi_max = (double)(p.nxi - 1) * p.dxi;
    a.fields = c->at<R>(L.set[k].fields);
    a.fpack = L.set[k].fpack ? c->at<R>(L.set[k].fpack) : nullptr;
    a.hist = L.set[k].hist ? c->at<int>(L.set[k].hist) : nullptr;
    a.base = L.set[k].base ? c->at<int>(L.set[k].base) : nullptr;
    if (k + 1 < L.nset) {
      a.ring_next = c->at<R>(L.set[k + 1].ring);
      a.src_next = c->at<R>(L.set[k + 1].src);
    }
    a.err = c->at<int>(L.err);
    return a;
  }

  // Launch shapes of a set of lanes (maxima over the boxes).
  struct Dims {
    int n = 0, nx = 0, ny = 0, nxi = 0, nxh = 0, np = 0, per_row = 0, n_corr = 0;
    int nt = 64;                      // plasma-row block size
    int rows_r2c = 0, rt_rows = 64;   // row-pass grid and block size
    int ctpt = 0;                     // threads per column transform (0: default)
    int cols[3] = {0, 0, 0};          // column-pass grid per mode
    size_t smem_col[3] = {0, 0, 0};
    size_t smem_rows = 0;             // row-pass LDS
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
  static void finish_dims(Dims& d, const qsa_params* const* ps, int n, int nt = 0, int rt = 0, int ct = 0) {
    d.ctpt = (ct == 16 || ct == 32 || ct == 64) ? ct : 0;
    d.rt_rows = std::min(256, std::max(64, d.nx / 2));   // two row pairs per block from nx = 256
    if (rt >= row_tpt(d.nx) && rt % row_tpt(d.nx) == 0 && rt <= 256) d.rt_rows = rt;
    d.nt = std::max(64, std::min(PlasmaBlock<R>::MAX, (d.per_row + 63) / 64 * 64));
    if (nt == 64 || nt == 128 || nt == 256 || (nt == 512 && PlasmaBlock<R>::MAX >= 512)) d.nt = nt;
    d.rows_r2c = 0;
    d.smem_rows = 0;
    for (int m = 0; m < 3; ++m) {
      d.cols[m] = 0;
      d.smem_col[m] = 0;
    }
    const int G[3] = {ColShape<COL_PSI>::G, ColShape<COL_J>::G, ColShape<COL_B>::G};
    for (int i = 0; i < n; ++i) {
      const qsa_params& p = *ps[i];
      const int ppw = d.rt_rows / row_tpt(p.nx);
      d.rows_r2c = std::max(d.rows_r2c, ((p.ny + 1) / 2 + ppw - 1) / ppw);
      // twiddles and two FFT buffers per row pair, ppw pairs per block
      d.smem_rows = std::max(d.smem_rows, ((size_t)p.nx + 2 * (size_t)fft_cap(p.nx) * ppw) * sizeof(C2<R>));
      const int tpt = col_tpt(p.ny, d.ctpt);
      const int cpw = 64 / tpt;
      for (int m = 0; m < 3; ++m) {
        d.cols[m] = std::max(d.cols[m], (p.nx / 2 + 1 + cpw - 1) / cpw);
        d.smem_col[m] = std::max(d.smem_col[m],
                                 ((size_t)p.ny + (size_t)cpw * 2 * G[m] * fft_cap(p.ny)) * sizeof(C2<R>));
      }
    }
  }

  // One tick of the slice loops of every lane: one launch per phase, blockIdx.z
  // = lane, lane l working on slice t - lag(l).  `tc` receives the
  // kernel-class timing marks.
  // before_final (may be null): an event the final advance waits for.
  static qsa_status tick(qsa_ctx* tc, hipStream_t st, const Lane<R>* lanes, const Dims& d, int t,
                         hipEvent_t before_final = nullptr) {
    const int n = d.n;
    const int pb = (d.np + 255) / 256;
    const size_t smem_rows = d.smem_rows;
    const int nt = d.nt;
    const int j = t;   // every lag is a multiple of QSA_SORT_EVERY
    {
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
      QSA_LAUNCH(tc, QSA_K_DEP_S, (k_plasma_rows<R, PL_DEP_S>), dim3(d.ny, 1, n), dim3(nt),
                         4 * 1 * (size_t)d.nx * sizeof(double), st, lanes, j, 0);
      QSA_LAUNCH(tc, QSA_K_ROW_R2C, k_row_r2c<R>, rgrid_psi, rblock, smem_rows, st, lanes, j, (int)ST_PSI);
      QSA_LAUNCH(tc, QSA_K_COL, (k_col<R, COL_PSI>), dim3(d.cols[0], 1, n), dim3(64 * ColShape<COL_PSI>::G),
                         d.smem_col[0], st, lanes, j, d.ctpt);
      QSA_LAUNCH(tc, QSA_K_ROW_C2R, k_row_c2r<R>, dim3(d.rows_r2c, 3, n), rblock, smem_rows, st, lanes, j,
                 (int)ST_PSI);
      // ---- J stage
      QSA_LAUNCH(tc, QSA_K_DEP_J, (k_plasma_rows<R, PL_DEP_J>), dim3(d.ny, 1, n), dim3(nt),
                         4 * 3 * (size_t)d.nx * sizeof(double), st, lanes, j, 0);
      QSA_LAUNCH(tc, QSA_K_ROW_R2C, k_row_r2c<R>, rgrid_j, rblock, smem_rows, st, lanes, j, (int)ST_J);
      QSA_LAUNCH(tc, QSA_K_COL, (k_col<R, COL_J>), dim3(d.cols[1], 1, n), dim3(64 * ColShape<COL_J>::G),
                         d.smem_col[1], st, lanes, j, d.ctpt);
      QSA_LAUNCH(tc, QSA_K_ROW_C2R, k_row_c2r<R>, dim3(d.rows_r2c, 4, n), rblock, smem_rows, st, lanes, j, (int)ST_J);
      // ---- B_perp predictor-corrector
      for (int k = 0; k < d.n_corr; ++k) {
        QSA_LAUNCH(tc, QSA_K_PUSH_PRED, (k_plasma_rows<R, PL_PRED>), dim3(d.ny, 1, n), dim3(nt),
                           4 * 2 * (size_t)d.nx * sizeof(double), st, lanes, j, k);
        QSA_LAUNCH(tc, QSA_K_ROW_R2C, k_row_r2c<R>, rgrid_b, rblock, smem_rows, st, lanes, j, (int)ST_B);
        QSA_LAUNCH(tc, QSA_K_COL, (k_col<R, COL_B>), dim3(d.cols[2], 1, n), dim3(64 * ColShape<COL_B>::G),
                           d.smem_col[2], st, lanes, j, d.ctpt);
        QSA_LAUNCH(tc, QSA_K_ROW_C2R, k_row_c2r<R>, rgrid_b, rblock, smem_rows, st, lanes, j, (int)ST_B);
      }
      // ---- advance the plasma to slice j+1
      if (before_final) {
        const hipError_t e = hipStreamWaitEvent(st, before_final, 0);
        if (e != hipSuccess) {
          tc->sticky = QSA_E_DEVICE;
          return fail(tc, QSA_E_DEVICE, std::string("hipStreamWaitEvent: ") + hipGetErrorString(e));
        }
      }
      QSA_LAUNCH(tc, QSA_K_PUSH_FINAL, k_push_final<R>, dim3(pb, 1, n), dim3(256), 0, st, lanes, j,
                 d.n_corr > 0 ? 1 : 0);
    }
    return QSA_OK;
  }

  static void clear_lanes(hipStream_t st, const Lane<R>* lanes, const Dims& d, int t) {
    const int blocks = (int)std::min<int64_t>(1024, (d.clear + 255) / 256);
    hipLaunchKernelGGL((k_lane_clear<R, 0>), dim3(blocks, 1, d.n), dim3(256), 0, st, lanes, t);
  }

  // Before the launches of tick t on stream st: every QSA_THROTTLE_TICKS
  // ticks, wait (spinning) until the device has reached the mark of two
  // periods back, then set a new mark.  Nothing while st is being captured.
  static qsa_status throttle(qsa_ctx* c, hipStream_t st, int t) {
    if (t % QSA_THROTTLE_TICKS != 0) return QSA_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_OK(hipStreamIsCapturing(st, &cs));
    if (cs != hipStreamCaptureStatusNone) return QSA_OK;
    const int k = t / QSA_THROTTLE_TICKS;
    if (k >= 2) {
      hipError_t e;
      while ((e = hipEventQuery(c->tev[(k - 2) % QSA_TEV])) == hipErrorNotReady) {
      }
      HIP_OK(e);
    }
    HIP_OK(hipEventRecord(c->tev[k % QSA_TEV], st));
    return QSA_OK;
  }

  // The slice loop of every lane (all with lag 0).
  static qsa_status slices(qsa_ctx* tc, hipStream_t st, const Lane<R>* lanes, const Dims& d) {
    qsa_ctx* c = tc;   // error reporting (HIP_OK)
    clear_lanes(st, lanes, d, 0);
    for (int t = 0; t < d.nxi; ++t) {
      qsa_status s = throttle(tc, st, t);
      if (s == QSA_OK) s = tick(tc, st, lanes, d, t);
      if (s != QSA_OK) return s;
    }
    HIP_OK(hipGetLastError());
    return QSA_OK;
  }

  static Dims dims_of(qsa_ctx* c) {
    Dims d;
    add_dims(d, c->p);
    const qsa_params* ps[1] = {&c->p};
    finish_dims(d, ps, 1, c->tune_nt, c->tune_rt, c->tune_ct);
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

  // Push the particles of every species whose deposit keys lie in [k0, k1)
  // (on stream st).
  static qsa_status push_keys(qsa_ctx* c, const Geo<R>& g, hipStream_t st, int64_t k0, int64_t k1) {
    const BeamDepArgs<R> da = beam_dep_args(c);
    for (int s = 0; s < c->p.n_species; ++s) {
      if (c->beam_n[s] == 0) continue;
      const BeamArgs<R> a = beam_args(c, g, s);
      const int grid = (c->beside_blocks > 0) ? c->beside_blocks : QSA_PUSH_BLOCKS;
      const int blocks = (int)std::min<int64_t>(grid, (a.n + 255) / 256);
      int64_t* cnt = c->L.cnt_next[s] ? c->at<int64_t>(c->L.cnt_next[s]) : nullptr;
      QSA_LAUNCH(c, QSA_K_BEAM_PUSH, k_beam_push_keys<R>, dim3(blocks), dim3(256), 0, st, g, a,
                 (const int*)da.perm[s], da.doff[s], k0, k1, cnt);
    }
    HIP_OK(hipGetLastError());
    return QSA_OK;
  }

  // One beam step with the beam work beside the slice loop (one step in
  // flight).  The keys and permutation of the step's start order the beam
  // by slab; a second stream deposits the sources QSA_BEAM_CHUNK slabs at a
  // time, QSA_BEAM_AHEAD chunks ahead of the slice loop (tick j waits for
  // the chunk holding slab j, whose deposit completes node slice j), and
  // pushes each chunk once the slice loop has finished the slice after its
  // last slab (a slab-j particle gathers slices j and j + 1; the fields of
  // every slice are stored, so no later tick overwrites what it reads).  The
  // particles of a chunk are those its keys held at the step's start, so no
  // drift can take one out of the slices its push waits for.  Equal to
  // sweep() + push() up to the order of the deposit's additions.
  static qsa_status step_beside(qsa_ctx* c) {
    hipStream_t bs = c->bstream;
    const qsa_status st = step_beside_body(c, bs);
    if (st != QSA_OK) {
      // an early exit: no later call may overlap the beam work enqueued
      (void)hipStreamSynchronize(bs);
      if (c->sticky == QSA_OK) c->sticky = st;
    }
    return st;
  }

  static qsa_status step_beside_body(qsa_ctx* c, hipStream_t bs) {
    const qsa_params& p = c->p;
    const Geo<R> g = geo(p);
    static_assert(QSA_BEAM_AHEAD >= 2, "a chunk's deposit waits for the push of the chunk AHEAD before it");
    static_assert(QSA_BEAM_AHEAD + 1 < QSA_GEV, "event ring too short");
    qsa_status st = beam_perm_all(c, g);
    if (st != QSA_OK) return st;
    R* src = c->at<R>(c->L.set[0].src);
    if ((st = fill(c, src, 4 * (int64_t)p.nxi * g.nperp, R(0))) != QSA_OK) return st;
    const Lane<R>* lanes = c->at<Lane<R>>(c->L.lane);
    const Dims d = dims_of(c);
    const int C = QSA_BEAM_CHUNK, nch = (p.nxi + C - 1) / C;
    const int64_t keys_per_slab = (int64_t)p.ny * (nx_chunks_of(p.nx));
    const int64_t key_end = (int64_t)p.nxi * keys_per_slab + 1;   // past the left-the-box key
    auto chunk_end = [&](int ch) { return std::min(p.nxi, (ch + 1) * C); };
    auto deposit = [&](int ch) -> qsa_status {
      qsa_status s = deposit_slabs(c, g, bs, src, ch * C, chunk_end(ch), c->beside_blocks);
      if (s != QSA_OK) return s;
      HIP_OK(hipEventRecord(c->gdone[ch % QSA_GEV], bs));
      return QSA_OK;
    };
    auto fork = [&](int slot) -> qsa_status {
      HIP_OK(hipEventRecord(c->gfork[slot % QSA_GEV], c->stream));
      HIP_OK(hipStreamWaitEvent(bs, c->gfork[slot % QSA_GEV], 0));
      return QSA_OK;
    };
    if ((st = fork(0)) != QSA_OK) return st;
    for (int ch = 0; ch < std::min(QSA_BEAM_AHEAD, nch); ++ch)
      if ((st = deposit(ch)) != QSA_OK) return st;
    clear_lanes(c->stream, lanes, d, 0);
    int pushed = 0;   // chunks pushed so far
    for (int t = 0; t < p.nxi; ++t) {
      if ((st = throttle(c, c->stream, t)) != QSA_OK) return st;
      if (t % C == 0) HIP_OK(hipStreamWaitEvent(c->stream, c->gdone[(t / C) % QSA_GEV], 0));
      if ((st = tick(c, c->stream, lanes, d, t)) != QSA_OK) return st;
      if (t + 1 < p.nxi && t == chunk_end(pushed)) {
        // slices <= t are final: chunk `pushed` goes, then the deposit of
        // the chunk QSA_BEAM_AHEAD after it
        if ((st = fork(pushed)) != QSA_OK) return st;
        if ((st = push_keys(c, g, bs, (int64_t)pushed * C * keys_per_slab,
                            (int64_t)chunk_end(pushed) * keys_per_slab)) != QSA_OK)
          return st;
        if (pushed + QSA_BEAM_AHEAD < nch && (st = deposit(pushed + QSA_BEAM_AHEAD)) != QSA_OK) return st;
        ++pushed;
      }
    }
    // the chunks left, and the particles outside the box, after the last
    // slice (every chunk's deposit was enqueued before the tick that waits
    // for it: chunk k after the push of chunk k - QSA_BEAM_AHEAD)
    if ((st = fork(pushed)) != QSA_OK) return st;
    if ((st = push_keys(c, g, bs, (int64_t)pushed * C * keys_per_slab, key_end)) != QSA_OK) return st;
    HIP_OK(hipEventRecord(c->gdone[0], bs));
    HIP_OK(hipStreamWaitEvent(c->stream, c->gdone[0], 0));   // join
    counts_made(c);
    HIP_OK(hipGetLastError());
    c->swept = true;
    return QSA_OK;
  }

  // Every particle pushed; the pushes count the next deposit's keys where
  // the context keeps the counts (cnt_next was zeroed by this step's deposit).
  static qsa_status push(qsa_ctx* c) {
    const Geo<R> g = geo(c->p);
    for (int s = 0; s < c->p.n_species; ++s) {
      if (c->beam_n[s] == 0) continue;
      BeamArgs<R> a = beam_args(c, g, s);
      const int64_t blocks = (a.n + 255) / 256;
      int64_t* cnt = c->L.cnt_next[s] ? c->at<int64_t>(c->L.cnt_next[s]) : nullptr;
      QSA_LAUNCH(c, QSA_K_BEAM_PUSH, k_beam_push<R>, dim3((unsigned)blocks), dim3(256), 0, c->stream, g, a, cnt);
    }
    counts_made(c);
    HIP_OK(hipGetLastError());
    return QSA_OK;
  }

  // n beam steps in flight (n <= nset): lane k sweeps step n0 + k in set k,
  // QSA_PIPE_LAG slices behind lane k - 1, pushes each beam slab as soon as
  // its fields are final there and deposits it as lane k + 1's sources.
  static qsa_status group(qsa_ctx* c, int n) {
    invalidate_counts(c);
    int last = -1;
    const qsa_status st = group_body(c, n, last);
    if (st != QSA_OK && last >= 0) {
      // an early exit: order the work stream after the beam work already
      // enqueued, so that no later call overlaps it
      if (hipStreamWaitEvent(c->stream, c->gdone[last % QSA_GEV], 0) != hipSuccess)
        (void)hipStreamSynchronize(c->bstream);
    }
    if (st != QSA_OK && c->sticky == QSA_OK) c->sticky = st;
    return st;
  }

  // The body of group(); `last` receives the last tick whose beam work was
  // enqueued on the beam stream (-1: none).
  static qsa_status group_body(qsa_ctx* c, int n, int& last) {
    const qsa_params& p = c->p;
    const Layout& L = c->L;
    const Geo<R> g = geo(p);
    // the beam sorted by cell row; the sort buffer keeps a copy of it (a
    // lean sort instead leaves the storage in key order with the identity
    // permutation, which the first deposit then uses as it stands)
    qsa_status st = sort_all(c);
    if (st != QSA_OK) return st;
    if ((st = beam_deposit_all(c, g, L.lean)) != QSA_OK) return st;   // lane 0's sources
    for (int k = 1; k < n; ++k)
      if ((st = fill(c, c->at<R>(L.set[k].src), 4 * (int64_t)p.nxi * g.nperp, R(0))) != QSA_OK) return st;
    Dims d = dims_of(c);
    d.n = n;
    const Lane<R>* lanes = c->at<Lane<R>>(L.lane);
    const PipeBeam<R>* pipes = c->at<PipeBeam<R>>(L.pipe);
    const size_t tile = (size_t)2 * 2 * 4 * g.nx * sizeof(double);
    const int nperp_blocks = (g.nperp + 255) / 256;
    const int T = p.nxi + 2 + (n - 1) * QSA_PIPE_LAG;
    // The beam work of tick t (push, row sort, deposit of the slabs behind
    // every lane) runs on a stream of its own, after the slice loop's tick t
    // and alongside its next ticks; the final advance of tick
    // t + QSA_RING_WAIT waits for it (the constraints are in qsa_kernels.h).
    static_assert(QSA_RING_WAIT < QSA_GEV, "event ring too short");
    for (int t = 0; t < T; ++t) {
      if ((st = throttle(c, c->stream, t)) != QSA_OK) return st;
      if (t % QSA_PIPE_LAG == 0 && t < n * QSA_PIPE_LAG) clear_lanes(c->stream, lanes, d, t);
      const int tw = t - QSA_RING_WAIT;
      hipEvent_t wait = (tw >= QSA_PUSH_LAG) ? c->gdone[tw % QSA_GEV] : nullptr;
      if ((st = tick(c, c->stream, lanes, d, t, wait)) != QSA_OK) return st;
      if (t < QSA_PUSH_LAG) continue;
      hipStream_t bs = c->bstream;
      HIP_OK(hipEventRecord(c->gfork[t % QSA_GEV], c->stream));
      HIP_OK(hipStreamWaitEvent(bs, c->gfork[t % QSA_GEV], 0));
      QSA_LAUNCH(c, QSA_K_BEAM_PUSH, k_pipe_push<R>, dim3(g.ny, 1, n), dim3(256), 0, bs, pipes, t, n);
      hipLaunchKernelGGL(k_pipe_scan<R>, dim3(g.ny, 1, n - 1), dim3(256), 0, bs, pipes, t, n);
      hipLaunchKernelGGL(k_pipe_place<R>, dim3(g.ny, 1, n - 1), dim3(256), 0, bs, pipes, t, n);
      QSA_LAUNCH(c, QSA_K_BEAM_DEPOSIT, k_pipe_deposit<R>, dim3(g.ny, 1, n - 1), dim3(BeamRowBlock<R>::THREADS),
                 tile + (g.ny + 1 + 16) * sizeof(int), bs, pipes, t, n);
      hipLaunchKernelGGL(k_pipe_reduce<R>, dim3(nperp_blocks, 1, n - 1), dim3(256), 0, bs, pipes, t, n);
      HIP_OK(hipEventRecord(c->gdone[t % QSA_GEV], bs));
      last = t;
    }
    if (last >= 0) HIP_OK(hipStreamWaitEvent(c->stream, c->gdone[last % QSA_GEV], 0));   // join
    HIP_OK(hipGetLastError());
    c->swept = true;
    return QSA_OK;
  }

  // Copy every beam array (with identities) of every species.
  static qsa_status copy_beam(qsa_ctx* c, const size_t (&dst)[QSA_MAX_SPECIES][8],
                              const size_t (&src)[QSA_MAX_SPECIES][8]) {
    for (int s = 0; s < c->p.n_species; ++s) {
      const int64_t m = c->beam_n[s];
      for (int k = 0; k < 8 && m > 0; ++k)
        HIP_OK(hipMemcpyAsync(c->ws + dst[s][k], c->ws + src[s][k], (size_t)m * (k < 6 ? sizeof(R) : 8),
                              hipMemcpyDeviceToDevice, c->stream));
    }
    return QSA_OK;
  }

  // Put back the beam of the group's start, with clear device flags.
  static qsa_status restore(qsa_ctx* c) {
    invalidate_counts(c);
    qsa_status st = copy_beam(c, c->L.beam, c->L.snap);
    if (st != QSA_OK) return st;
    hipLaunchKernelGGL(k_fill<int>, dim3(1), dim3(64), 0, c->stream, c->at<int>(c->L.err), (int64_t)1, 0);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(c->stream));
    return QSA_OK;
  }

  // One autotuning trial on the work stream: n > 1 steps in flight (the beam
  // is put back afterwards) or one sweep; *ms = wall time per step or sweep.
  static qsa_status trial(qsa_ctx* c, int n, hipEvent_t e0, hipEvent_t e1, float* ms) {
    HIP_OK(hipEventRecord(e0, c->stream));
    qsa_status st = (n > 1) ? group(c, n) : sweep(c);
    if (st != QSA_OK) return st;
    HIP_OK(hipEventRecord(e1, c->stream));
    HIP_OK(hipEventSynchronize(e1));
    float t = 0.f;
    HIP_OK(hipEventElapsedTime(&t, e0, e1));
    *ms = t / (float)n;
    if (n > 1) return restore(c);
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

  // float64 values times `scale` -> working precision at workspace offset off
  static qsa_status scale_negative(qsa_ctx* c, size_t off, int64_t n, double z) {
    if (n == 0) return QSA_OK;
    hipLaunchKernelGGL(k_scale_negative<R>, dim3(fill_blocks(n)), dim3(256), 0, c->stream, c->at<R>(off), n, (R)z);
    HIP_OK(hipGetLastError());
    return QSA_OK;
  }

  static qsa_status upload_scaled(qsa_ctx* c, const double* src, size_t off, int64_t n, int on_device,
                                  double scale) {
    if (n == 0) return QSA_OK;
    R* dst = c->at<R>(off);
    if (on_device) {
      hipLaunchKernelGGL(k_scaled_from_f64<R>, dim3(fill_blocks(n)), dim3(256), 0, c->stream, src, dst, scale, n);
      HIP_OK(hipGetLastError());
      return QSA_OK;
    }
    const int64_t chunk = 1 << 22;
    std::vector<R> tmp((size_t)std::min<int64_t>(n, chunk));
    for (int64_t o = 0; o < n; o += chunk) {
      const int64_t m = std::min<int64_t>(chunk, n - o);
      for (int64_t i = 0; i < m; ++i) tmp[i] = (R)(src[o + i] * scale);
      HIP_OK(hipMemcpyAsync(dst + o, tmp.data(), m * sizeof(R), hipMemcpyHostToDevice, c->stream));
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

  // Beam array k of species s in load order (the pipelined path keeps the
  // particles sorted by cell row, with their load index): scattered by
  // identity straight into a device destination, or through the sort buffer
  // for a host one.
  static qsa_status read_beam_array(qsa_ctx* c, int s, int k, double* dst, int64_t n, int on_device) {
    if (c->L.nset < 2 || c->L.lean) return download(c, c->ws + c->L.beam[s][k], dst, n, on_device, k == 6);
    if (n == 0) return QSA_OK;
    double* out = on_device ? dst : c->at<double>(c->L.snap[s][6]);
    const int64_t* id = c->at<int64_t>(c->L.beam[s][7]);
    const dim3 grid((unsigned)((n + 255) / 256));
    if (k == 6)
      hipLaunchKernelGGL(k_unpermute<double>, grid, dim3(256), 0, c->stream, c->at<double>(c->L.beam[s][6]), id,
                         out, n);
    else
      hipLaunchKernelGGL(k_unpermute<R>, grid, dim3(256), 0, c->stream, c->at<R>(c->L.beam[s][k]), id, out, n);
    HIP_OK(hipGetLastError());
    if (!on_device) {
      HIP_OK(hipMemcpyAsync(dst, out, n * 8, hipMemcpyDeviceToHost, c->stream));
      HIP_OK(hipStreamSynchronize(c->stream));
    }
    return QSA_OK;
  }

  static qsa_status fields(qsa_ctx* c, int field, int xi0, int xi1, double* dst, int on_device) {
    const qsa_params& p = c->p;
    const int64_t nperp = (int64_t)p.nx * p.ny;
    const int64_t plane = (int64_t)p.nxi * nperp;
    const SetLayout& S = c->L.set[c->cur_set];
    const R* F = c->at<R>(S.fields);
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
        default: A = c->at<R>(S.src) + (field - QSA_SRC_S) * plane + o; break;
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

  // Diagnostics: per-window field mean squares of the last sweep, beam
  // moments of species s (k_field_moments, k_beam_moments).
  static qsa_status moments_out(qsa_ctx* c, double* out, double* dst, int64_t n, int on_device) {
    if (!on_device)
      HIP_OK(hipMemcpyAsync(dst, out, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    return QSA_OK;
  }

  static qsa_status field_moments(qsa_ctx* c, int ws, double* dst, int on_device) {
    const qsa_params& p = c->p;
    const Geo<R> g = geo(p);
    const int64_t n = 6 * (int64_t)((p.nxi + ws - 1) / ws);
    double* out = on_device ? dst : c->at<double>(c->L.diag);
    hipLaunchKernelGGL(k_fill<double>, dim3(fill_blocks(n)), dim3(256), 0, c->stream, out, n, 0.0);
    hipLaunchKernelGGL(k_field_moments<R>, dim3(p.nxi), dim3(256), 0, c->stream, g,
                       (const R*)c->at<R>(c->L.set[c->cur_set].fields), ws, out);
    HIP_OK(hipGetLastError());
    return moments_out(c, out, dst, n, on_device);
  }

  static qsa_status beam_moments(qsa_ctx* c, int s, int ws, double* dst, int on_device) {
    const qsa_params& p = c->p;
    const int64_t n = 7 * (int64_t)((p.nxi + ws - 1) / ws);
    double* out = on_device ? dst : c->at<double>(c->L.diag);
    hipLaunchKernelGGL(k_fill<double>, dim3(fill_blocks(n)), dim3(256), 0, c->stream, out, n, 0.0);
    const int64_t np = c->beam_n[s];
    if (np > 0) {
      const Layout& L = c->L;
      hipLaunchKernelGGL(k_beam_moments<R>, dim3((unsigned)((np + QSA_DIAG_CHUNK - 1) / QSA_DIAG_CHUNK)),
                         dim3(256), 0, c->stream, (const double*)c->at<double>(L.beam[s][6]),
                         (const R*)c->at<R>(L.beam[s][2]), (const R*)c->at<R>(L.beam[s][3]),
                         (const R*)c->at<R>(L.beam[s][4]), (const R*)c->at<R>(L.beam[s][5]), np, 1.0 / p.dxi,
                         p.nxi, ws, out);
      HIP_OK(hipGetLastError());
    }
    return moments_out(c, out, dst, n, on_device);
  }

  // Launch limits on LDS: beam tiles (2 node slices x 2 node rows x 4
  // sources x nx) stay within 64 KiB for nx <= 512; the column transforms of
  // tall grids opt in to more.
  // LDS of the widest column pass (COL_J) with ct threads per transform
  static int col_lds(int ny, int ct) {
    const int cpw = 64 / col_tpt(ny, ct);
    return (ny + cpw * 2 * ColShape<COL_J>::G * fft_cap(ny)) * (int)sizeof(C2<R>);
  }

  static qsa_status set_lds_limits(qsa_ctx* c) {
    int dev = 0, optin = 0, plain = 0;
    HIP_OK(hipGetDevice(&dev));
    if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess) optin = 0;
    HIP_OK(hipDeviceGetAttribute(&plain, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const int limit = std::max(optin, plain);
    static_assert(2 * 2 * 4 * 512 * 8 <= 65536, "beam tile");
    // beam deposits: the tile; the pipelined one also row starts and scan
    // scratch
    const int rows = 2 * 2 * 4 * c->p.nx * (int)sizeof(double);
    const int pipe = rows + (c->p.ny + 1 + 16) * (int)sizeof(int);
    if (pipe > limit) return fail(c, QSA_E_INVALID, "nx too large for the device's LDS");
    if (rows > 65536)
      HIP_OK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_beam_rows<R>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, rows));
    if (pipe > 65536)
      HIP_OK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pipe_deposit<R>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, pipe));
    // column transforms: twiddles and 2 G cpw FFT buffers per block, cpw =
    // 64 / threads per transform; the largest that fits
    int colj = col_lds(c->p.ny, 64);
    if (colj > limit) return fail(c, QSA_E_INVALID, "ny too large for the device's LDS");
    for (int ct = 32; ct >= 16; ct /= 2)
      if (col_lds(c->p.ny, ct) <= limit) colj = std::max(colj, col_lds(c->p.ny, ct));
    c->col_lds_max = colj;
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
    qsa_status st0 = set_lds_limits(c);
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
    hipLaunchKernelGGL(k_set_flag, dim3(1), dim3(64), 0, c->stream, c->at<int>(c->L.kvalid), 0);
    {
      std::vector<Lane<R>> lanes;
      std::vector<PipeBeam<R>> pipes;
      for (int k = 0; k < c->L.nset; ++k) {
        lanes.push_back(make_lane(c, k));
        pipes.push_back(make_pipe(c, k));
      }
      HIP_OK(hipMemcpyAsync(c->ws + c->L.lane, lanes.data(), lanes.size() * sizeof(Lane<R>),
                            hipMemcpyHostToDevice, c->stream));
      HIP_OK(hipMemcpyAsync(c->ws + c->L.pipe, pipes.data(), pipes.size() * sizeof(PipeBeam<R>),
                            hipMemcpyHostToDevice, c->stream));
      HIP_OK(hipStreamSynchronize(c->stream));
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

}  // namespace

#include "qsa_adjoint_host.h"

namespace {

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
qsa_status run_step_beside(qsa_ctx* c) {
  return dispatch(c, [&] { return Engine<double>::step_beside(c); },
                  [&] { return Engine<float>::step_beside(c); });
}
qsa_status run_group(qsa_ctx* c, int n) {
  return dispatch(c, [&] { return Engine<double>::group(c, n); }, [&] { return Engine<float>::group(c, n); });
}

// One beam step at a time: the beam work beside the slice loop on two
// streams (enqueued directly), else graph replay unless timing or graphs
// are off.
qsa_status step_one(qsa_ctx* c, bool graphs) {
  qsa_status st = QSA_OK;
  // a step due for the storage re-sort is enqueued directly (a captured
  // step replays without it)
  const bool resort = c->L.nset == 1 && c->resort_every > 0 && c->beam_steps % c->resort_every == 0;
  ++c->beam_steps;
  if (resort) {
    c->resort_pending = true;
    graphs = false;
  }
  if (c->beam_beside && c->L.nset == 1) {
    st = run_step_beside(c);
    c->resort_pending = false;
    if (st != QSA_OK) return st;
    c->cur_set = 0;
    return QSA_OK;
  }
  if (graphs && (st = capture(c, &c->gx_step, [&] { return run_step(c); })) != QSA_OK) return st;
  if (graphs && c->gx_step) {
    HIP_OK(hipGraphLaunch(c->gx_step, c->stream));
    c->swept = true;
  } else {
    st = run_step(c);
    c->resort_pending = false;
    if (st != QSA_OK) return st;
  }
  c->cur_set = 0;
  return QSA_OK;
}

// n > 1 beam steps in flight; false in *done when the group broke the
// schedule (the beam is then back at the group's start and pipelining off:
// the group sorted the beam first, so its drift within a group is too large).
qsa_status step_group(qsa_ctx* c, int n, bool graphs, bool* done) {
  *done = false;
  qsa_status st = check_device(c);   // the group starts with clear device flags
  if (st != QSA_OK) return st;
  // Enqueued directly, not replayed from a graph: the group runs on two
  // streams (the beam work alongside the slice loop), and measured faster
  // that way (75.8 against 76.9 ms per step); a graph captured across the
  // two streams also kept the workspace allocated after the context was
  // destroyed.
  (void)graphs;
  if ((st = run_group(c, n)) != QSA_OK) return st;
  HIP_OK(hipStreamSynchronize(c->stream));
  int e = 0;
  HIP_OK(hipMemcpy(&e, c->ws + c->L.err, sizeof(int), hipMemcpyDeviceToHost));
  if ((e & ERR_DRIFT) && c->L.lean) {
    c->sticky = QSA_E_STATE;
    return fail(c, QSA_E_STATE,
                "beam particles drifted beyond the steps-in-flight schedule, and a lean pipeline keeps no copy "
                "of the beam to repeat the group from");
  }
  if (e & ERR_DRIFT) {
    st = dispatch(c, [&] { return Engine<double>::restore(c); }, [&] { return Engine<float>::restore(c); });
    if (st != QSA_OK) return st;
    c->pipe_ok = false;
    return QSA_OK;
  }
  c->cur_set = n - 1;
  *done = true;
  return QSA_OK;
}

// Batched sweep (and push) of the member contexts ctxs[0 .. n): every
// context's beam deposit on stream st, then one slice loop over all lanes,
// whose descriptors are in `lanes` (device memory, one per member, in order).
// No allocation.
template <typename R>
qsa_status batch_run(qsa_ctx* const* ctxs, int n, hipStream_t st, const void* lanes, bool push) {
  qsa_ctx* c0 = ctxs[0];
  typename Engine<R>::Dims d;
  const qsa_params* ps[QSA_STATIC_MAX_CTX > 1024 ? QSA_STATIC_MAX_CTX : 1024];
  if (n > 1024) return fail(c0, QSA_E_INVALID, "a batch holds at most 1024 contexts");
  for (int i = 0; i < n; ++i) {
    Engine<R>::add_dims(d, ctxs[i]->p);
    ps[i] = &ctxs[i]->p;
  }
  Engine<R>::finish_dims(d, ps, n);
  for (int i = 0; i < n; ++i) {
    qsa_ctx* c = ctxs[i];
    hipStream_t own = c->stream;
    c->stream = st;
    const qsa_status s = Engine<R>::beam_deposit_all(c, Engine<R>::geo(c->p));
    c->stream = own;
    if (s != QSA_OK) return s;
  }
  qsa_status s = Engine<R>::slices(c0, st, reinterpret_cast<const Lane<R>*>(lanes), d);
  if (s != QSA_OK) return s;
  for (int i = 0; i < n; ++i) {
    qsa_ctx* c = ctxs[i];
    c->swept = true;
    c->cur_set = 0;
    if (!push) continue;
    hipStream_t own = c->stream;
    c->stream = st;
    s = Engine<R>::push(c);
    c->stream = own;
    if (s != QSA_OK) return s;
  }
  return QSA_OK;
}

template <typename R>
qsa_status batch_run(qsa_batch* b, bool push) {
  return batch_run<R>(b->ctxs.data(), (int)b->ctxs.size(), b->stream, b->ws, push);
}

// ---- the sweep of a batch with its lane table in static device memory ----
// The batch calls keep their lane table (one descriptor per member) in the
// workspace the caller passes to qsa_batch_create.  qsa_batch_sweep_static
// keeps it instead in `scratch`, a file-scope device array of
// QSA_STATIC_MAX_CTX descriptors that every call on a device shares.  Its
// device address is looked up once per device (hipGetSymbolAddress, with
// that device current) and kept in g_scratch: host code passes only that
// address to kernels, never the array's name.
constexpr size_t kLaneBytes = sizeof(Lane<double>) > sizeof(Lane<float>) ? sizeof(Lane<double>) : sizeof(Lane<float>);
static __device__ __align__(256) unsigned char scratch[QSA_STATIC_MAX_CTX * kLaneBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call for that device); null with a message on failure.
void* scratch_on_current_device(std::string& why) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    why = "no current HIP device (or more than 64 devices)";
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      why = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return nullptr;
    }
    g_scratch[dev] = ptr;
  }
  return g_scratch[dev];
}

// Copy one lane descriptor (passed by value) into the lane table.
template <typename R>
__global__ void k_put_lane(Lane<R>* __restrict__ dst, Lane<R> lane) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = lane;
}

template <typename R>
qsa_status static_sweep(qsa_ctx* const* ctxs, int n, hipStream_t st, void* table) {
  qsa_ctx* c = ctxs[0];   // error reporting (HIP_OK)
  Lane<R>* lanes = reinterpret_cast<Lane<R>*>(table);
  for (int i = 0; i < n; ++i)
    hipLaunchKernelGGL(k_put_lane<R>, dim3(1), dim3(64), 0, st, lanes + i, Engine<R>::make_lane(ctxs[i]));
  HIP_OK(hipGetLastError());
  return batch_run<R>(ctxs, n, st, table, false);
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
  c->pipe_max = L.nset;
  c->ws = reinterpret_cast<char*>(dev_ws);
  c->user = reinterpret_cast<hipStream_t>(hip_stream);
  bool made = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) == hipSuccess &&
              hipStreamCreateWithFlags(&c->bstream, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming) == hipSuccess;
  for (int i = 0; i < QSA_GEV && made; ++i)
    made = hipEventCreateWithFlags(&c->gfork[i], hipEventDisableTiming) == hipSuccess &&
           hipEventCreateWithFlags(&c->gdone[i], hipEventDisableTiming) == hipSuccess;
  for (int i = 0; i < QSA_TEV && made; ++i)
    made = hipEventCreateWithFlags(&c->tev[i], hipEventDisableTiming) == hipSuccess;
  if (!made) {
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
        c, [&] { return Engine<double>::upload(c, arr[i], c->ws + c->L.tmpl[i], n, on_device, i < 2); },
        [&] { return Engine<float>::upload(c, arr[i], c->ws + c->L.tmpl[i], n, on_device, i < 2); });
    if (st != QSA_OK) return st;
  }
  if (c->p.plasma_weights) {
    // uniform until qsa_load_plasma_weights
    qsa_status st = dispatch(
        c, [&] { return Engine<double>::fill(c, c->at<double>(c->L.tmpl_qw), n, 1.0); },
        [&] { return Engine<float>::fill(c, c->at<float>(c->L.tmpl_qw), n, 1.0f); });
    if (st != QSA_OK) return st;
    // uniform ions until qsa_load_ions
    const int64_t np = (int64_t)c->p.nx * c->p.ny;
    st = dispatch(c, [&] { return Engine<double>::fill(c, c->at<double>(c->L.ion), np, 1.0); },
                  [&] { return Engine<float>::fill(c, c->at<float>(c->L.ion), np, 1.0f); });
    if (st != QSA_OK) return st;
  }
  c->plasma_loaded = true;
  c->drop_graphs();
  return leave(c);
}

qsa_status qsa_load_plasma_weights(qsa_ctx* c, const double* w, int64_t n, int32_t on_device) {
  if (!c) return QSA_E_INVALID;
  if (c->sticky != QSA_OK) return c->sticky;
  if (!c->p.plasma_weights) return fail(c, QSA_E_STATE, "the context keeps no plasma weights (plasma_weights = 0)");
  if (!c->plasma_loaded) return fail(c, QSA_E_STATE, "no plasma template loaded");
  if (n != c->p.n_plasma) return fail(c, QSA_E_INVALID, "weight count differs from n_plasma");
  if (!w) return fail(c, QSA_E_INVALID, "null weight array");
  const bool mobile = c->p.ion_m > 0.0;
  if (!on_device)
    for (int64_t i = 0; i < n; ++i)
      if (!std::isfinite(w[i]) || (w[i] < 0 && !mobile))
        return fail(c, QSA_E_NONFINITE, "plasma weights must be finite and >= 0");
  qsa_status st0 = enter(c);
  if (st0 != QSA_OK) return st0;
  const double scale = 1.0 / c->p.plasma_w;
  qsa_status st = dispatch(c, [&] { return Engine<double>::upload_scaled(c, w, c->L.tmpl_qw, n, on_device, scale); },
                           [&] { return Engine<float>::upload_scaled(c, w, c->L.tmpl_qw, n, on_device, scale); });
  if (st != QSA_OK) return st;
  if (mobile && c->p.ion_z != 1) {
    // an ion's relative weight carries its charge: -Z |w|/plasma_w
    st = dispatch(c, [&] { return Engine<double>::scale_negative(c, c->L.tmpl_qw, n, (double)c->p.ion_z); },
                  [&] { return Engine<float>::scale_negative(c, c->L.tmpl_qw, n, (double)c->p.ion_z); });
    if (st != QSA_OK) return st;
  }
  c->drop_graphs();
  return leave(c);
}

qsa_status qsa_load_ions(qsa_ctx* c, const double* n_i, int64_t n, int32_t on_device) {
  if (!c) return QSA_E_INVALID;
  if (c->sticky != QSA_OK) return c->sticky;
  if (!c->p.plasma_weights) return fail(c, QSA_E_STATE, "the context keeps no ion profile (plasma_weights = 0)");
  if (!c->plasma_loaded) return fail(c, QSA_E_STATE, "no plasma template loaded");
  if (n != (int64_t)c->p.nx * c->p.ny) return fail(c, QSA_E_INVALID, "ion density count differs from nx * ny");
  if (!n_i) return fail(c, QSA_E_INVALID, "null ion density array");
  if (!on_device)
    for (int64_t i = 0; i < n; ++i)
      if (!std::isfinite(n_i[i]) || n_i[i] < 0) return fail(c, QSA_E_NONFINITE, "ion densities must be finite and >= 0");
  qsa_status st0 = enter(c);
  if (st0 != QSA_OK) return st0;
  qsa_status st = dispatch(c, [&] { return Engine<double>::upload_scaled(c, n_i, c->L.ion, n, on_device, 1.0); },
                           [&] { return Engine<float>::upload_scaled(c, n_i, c->L.ion, n, on_device, 1.0); });
  if (st != QSA_OK) return st;
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
  invalidate_counts(c);
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
  c->pipe_ok = true;
  c->beam_steps = 0;   // a loaded beam is re-sorted by the next step
  c->drop_graphs();
  qsa_status st = dispatch(c, [&] { return Engine<double>::loaded(c, s); },
                           [&] { return Engine<float>::loaded(c, s); });
  if (st != QSA_OK) return st;
  return leave(c);
}

qsa_status qsa_load_beam_range(qsa_ctx* c, int32_t s, int64_t first, const double* x, const double* y,
                               const double* xi, const double* ux, const double* uy, const double* uz,
                               const double* w, int64_t n, int32_t on_device) {
  if (!c) return QSA_E_INVALID;
  if (c->sticky != QSA_OK) return c->sticky;
  if (s < 0 || s >= c->p.n_species) return fail(c, QSA_E_INVALID, "species index out of range");
  invalidate_counts(c);
  if (first != 0 && first != c->beam_n[s])
    return fail(c, QSA_E_INVALID, "first must be 0 or the species' current particle count");
  if (n < 0 || first + n > c->p.beam_capacity[s]) return fail(c, QSA_E_INVALID, "beam count exceeds capacity");
  const double* arr[7] = {x, y, ux, uy, uz, w, xi};
  for (int i = 0; i < 7; ++i)
    if (n > 0 && !arr[i]) return fail(c, QSA_E_INVALID, "null beam array");
  if (!on_device)
    for (int i = 0; i < 7; ++i)
      if (!all_finite(arr[i], n)) return fail(c, QSA_E_NONFINITE, "non-finite beam value");
  qsa_status st0 = enter(c);
  if (st0 != QSA_OK) return st0;
  const size_t rs = (c->p.precision == QSA_FP32) ? 4 : 8;
  for (int i = 0; i < 7; ++i) {
    const bool f64 = (i == 6);
    char* dst = c->ws + c->L.beam[s][i] + (size_t)first * (f64 ? 8 : rs);
    qsa_status st = dispatch(c, [&] { return Engine<double>::upload(c, arr[i], dst, n, on_device, f64); },
                             [&] { return Engine<float>::upload(c, arr[i], dst, n, on_device, f64); });
    if (st != QSA_OK) return st;
  }
  c->beam_n[s] = first + n;
  c->pipe_ok = true;
  c->beam_steps = 0;   // a loaded beam is re-sorted by the next step
  c->drop_graphs();
  if (c->L.nset > 1 && !c->L.lean && n > 0) {
    // load indices of the new particles; the sort by cell row waits for the
    // next group of steps in flight, which starts with it
    hipLaunchKernelGGL(k_iota64_from, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream,
                       c->at<int64_t>(c->L.beam[s][7]) + first, first, n);
    HIP_OK(hipGetLastError());
  }
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
    qsa_status st = dispatch(c, [&] { return Engine<double>::read_beam_array(c, s, i, arr[i], m, on_device); },
                             [&] { return Engine<float>::read_beam_array(c, s, i, arr[i], m, on_device); });
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
  const bool graphs = c->use_graphs && c->timing_class < 0 && graph_fits(c->p.nxi);
  if (graphs && (st = capture(c, &c->gx_sweep, [&] { return run_sweep(c); })) != QSA_OK) return st;
  if (graphs && c->gx_sweep) {
    HIP_OK(hipGraphLaunch(c->gx_sweep, c->stream));
    c->swept = true;
  } else if ((st = run_sweep(c)) != QSA_OK) {
    return st;
  }
  c->cur_set = 0;
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
  const bool graphs = c->use_graphs && c->timing_class < 0 && graph_fits(c->p.nxi);
  for (int i = 0; i < n_steps;) {
    const int n = c->pipe_ok ? std::min(c->pipe_max, n_steps - i) : 1;
    if (n == 1) {
      if ((st = step_one(c, graphs && c->use_graphs)) != QSA_OK) return st;
      i += 1;
      continue;
    }
    bool done = false;
    if ((st = step_group(c, n, graphs && c->use_graphs, &done)) != QSA_OK) return st;
    if (done) i += n;   // else: repeated one step at a time
  }
  return leave(c);
}

qsa_status qsa_set_option(qsa_ctx* c, int32_t option, int64_t value) {
  if (!c) return QSA_E_INVALID;
  if (option == QSA_OPT_GRAPHS) {
    c->use_graphs = value != 0;
    return QSA_OK;
  }
  if (option == QSA_OPT_PIPELINE) {
    if (value < 1) return fail(c, QSA_E_INVALID, "pipeline depth must be >= 1");
    c->pipe_max = (int)std::min<int64_t>(value, c->L.nset);
    c->pipe_ok = true;
    return QSA_OK;
  }
  if (option == QSA_OPT_PLASMA_THREADS) {
    const bool f32 = c->p.precision == QSA_FP32;
    if (value != 0 && value != 64 && value != 128 && value != 256 && !(f32 && value == 512))
      return fail(c, QSA_E_INVALID, "plasma threads must be 0, 64, 128, 256 (or 512 in float32)");
    c->tune_nt = (int)value;
    c->drop_graphs();
    return QSA_OK;
  }
  if (option == QSA_OPT_ROW_THREADS) {
    const int tpt = row_tpt(c->p.nx);
    if (value != 0 && !((value == 64 || value == 128 || value == 256) && value >= tpt && value % tpt == 0))
      return fail(c, QSA_E_INVALID, "row threads must be 0 or 64, 128, 256 (a multiple of nx/4)");
    c->tune_rt = (int)value;
    c->drop_graphs();
    return QSA_OK;
  }
  if (option == QSA_OPT_BEAM_BESIDE) {
    if (value != 0 && value != 1) return fail(c, QSA_E_INVALID, "beam beside: 0 or 1");
    c->beam_beside = value != 0;
    return QSA_OK;
  }
  if (option == QSA_OPT_BESIDE_BLOCKS) {
    if (value < 0 || value > 65536) return fail(c, QSA_E_INVALID, "beside blocks: 0 .. 65536");
    c->beside_blocks = (int)value;
    return QSA_OK;
  }
  if (option == QSA_OPT_RESORT_EVERY) {
    if (value < 0) return fail(c, QSA_E_INVALID, "re-sort period must be >= 0");
    if (value > 0 && c->L.nset > 1)
      return fail(c, QSA_E_INVALID, "contexts with steps in flight sort their beam by cell row already");
    if (value > 0) {
      int64_t cap = 0;
      for (int s = 0; s < c->p.n_species; ++s) cap = std::max<int64_t>(cap, c->p.beam_capacity[s]);
      const size_t have = (c->p.precision == QSA_FP32) ? Engine<float>::resort_scratch(c)
                                                       : Engine<double>::resort_scratch(c);
      if ((size_t)cap * 8 > have)
        return fail(c, QSA_E_INVALID,
                    "re-sort: the largest beam capacity times 8 bytes exceeds the sources and fields it "
                    "reuses as scratch (" + std::to_string(have) + " bytes)");
    }
    c->resort_every = value;
    return QSA_OK;
  }
  if (option == QSA_OPT_COL_THREADS) {
    if (value != 0 && value != 16 && value != 32 && value != 64)
      return fail(c, QSA_E_INVALID, "column threads must be 0, 16, 32 or 64");
    const int need = (c->p.precision == QSA_FP32) ? Engine<float>::col_lds(c->p.ny, (int)value)
                                                   : Engine<double>::col_lds(c->p.ny, (int)value);
    if (need > c->col_lds_max)
      return fail(c, QSA_E_INVALID, "column threads: the column pass would not fit the device's LDS");
    c->tune_ct = (int)value;
    c->drop_graphs();
    return QSA_OK;
  }
  return fail(c, QSA_E_INVALID, "unknown option");
}

qsa_status qsa_autotune(qsa_ctx* c, double* ms_per_step) {
  if (!c) return QSA_E_INVALID;
  if (c->sticky != QSA_OK) return c->sticky;
  if (!c->plasma_loaded) return fail(c, QSA_E_STATE, "no plasma template loaded");
  if (c->timing_class >= 0) return fail(c, QSA_E_STATE, "kernel timing is active");
  invalidate_counts(c);
  qsa_status st = enter(c);
  if (st != QSA_OK) return st;
  if ((st = check_device(c)) != QSA_OK) return st;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_OK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(c, QSA_E_DEVICE, "hipEventCreate failed");
  }
  // (trials with steps in flight put the beam back from its copy: none in a
  // lean pipeline)
  const int depth0 = (c->L.nset > 1 && c->pipe_ok && !c->L.lean) ? c->L.nset : 1;
  auto run = [&](int n, float* ms) {
    return dispatch(c, [&] { return Engine<double>::trial(c, n, e0, e1, ms); },
                    [&] { return Engine<float>::trial(c, n, e0, e1, ms); });
  };
  float best = 0.f, t = 0.f;
  st = run(depth0, &best);   // warm-up: first launches of every kernel
  if (st == QSA_OK) st = run(depth0, &best);
  // threads per plasma-row block
  const int nts[4] = {64, 128, 256, 512};
  const int n_nt = (c->p.precision == QSA_FP32) ? 4 : 3;
  int best_nt = c->tune_nt;
  for (int k = 0; k < n_nt && st == QSA_OK; ++k) {
    c->tune_nt = nts[k];
    if ((st = run(depth0, &t)) == QSA_OK && t < best) {
      best = t;
      best_nt = nts[k];
    }
  }
  c->tune_nt = best_nt;
  // threads per row-transform block
  const int tpt = row_tpt(c->p.nx);
  int best_rt = c->tune_rt;
  for (int rt = 64; rt <= 256 && st == QSA_OK; rt *= 2) {
    if (rt < tpt || rt % tpt) continue;
    c->tune_rt = rt;
    if ((st = run(depth0, &t)) == QSA_OK && t < best) {
      best = t;
      best_rt = rt;
    }
  }
  c->tune_rt = best_rt;
  // threads per column transform
  int best_ct = c->tune_ct;
  for (int ct = 64; ct >= 16 && st == QSA_OK; ct /= 2) {
    const int need = (c->p.precision == QSA_FP32) ? Engine<float>::col_lds(c->p.ny, ct)
                                                   : Engine<double>::col_lds(c->p.ny, ct);
    if (need > c->col_lds_max) continue;
    c->tune_ct = ct;
    if ((st = run(depth0, &t)) == QSA_OK && t < best) {
      best = t;
      best_ct = ct;
    }
  }
  c->tune_ct = best_ct;
  // beam steps in flight (per step)
  int best_depth = c->pipe_max;
  if (depth0 > 1) {
    best_depth = depth0;
    for (int n = 2; n < depth0 && st == QSA_OK; n *= 2) {
      if ((st = run(n, &t)) == QSA_OK && t < best) {
        best = t;
        best_depth = n;
      }
    }
    c->pipe_max = best_depth;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != QSA_OK) return st;
  c->drop_graphs();
  c->swept = false;   // the trials' fields are not a sweep of the current beam
  c->cur_set = 0;
  if (ms_per_step) *ms_per_step = best;
  return leave(c);
}

qsa_status qsa_adjoint_sweep(qsa_ctx* c, int32_t n_steps, int32_t n_bins, const double* amps,
                             const int32_t* const* bins, double* loss, double* grad) {
  if (!c) return QSA_E_INVALID;
  if (c->sticky != QSA_OK) return c->sticky;
  if (!c->plasma_loaded) return fail(c, QSA_E_STATE, "no plasma template loaded");
  invalidate_counts(c);
  if (c->p.plasma_weights)
    return fail(c, QSA_E_INVALID, "the adjoint sweep takes a plasma of one weight (plasma_weights = 0)");
  const AdjLayout& A = c->L.adj;
  if (A.steps <= 0 || n_steps < 0 || n_steps > A.steps)
    return fail(c, QSA_E_INVALID, "n_steps exceeds the adjoint_steps the context was created with");
  if (n_bins < 1 || n_bins > 4096 || !amps || !bins || !loss || !grad)
    return fail(c, QSA_E_INVALID, "bad bins, amplitudes or outputs");
  for (int s = 0; s < c->p.n_species; ++s)
    if (c->beam_n[s] > 0 && !bins[s]) return fail(c, QSA_E_INVALID, "null bin array");
  for (int b = 0; b < n_bins; ++b)
    if (!std::isfinite(amps[b])) return fail(c, QSA_E_NONFINITE, "non-finite amplitude");
  qsa_status st = enter(c);
  if (st != QSA_OK) return st;
  if ((st = check_device(c)) != QSA_OK) return st;
  HIP_OK(hipMemcpy(c->ws + A.amps, amps, n_bins * sizeof(double), hipMemcpyHostToDevice));
  for (int s = 0; s < c->p.n_species; ++s) {
    const int64_t n = c->beam_n[s];
    if (n == 0) continue;
    int* dst = c->at<int>(A.bin[s]);
    if (c->L.nset > 1 && !c->L.lean) {
      // the library keeps this beam sorted: bins follow each particle's load index
      int* tmp = c->at<int>(A.bb[s][0]);
      HIP_OK(hipMemcpy(tmp, bins[s], n * sizeof(int), hipMemcpyHostToDevice));
      hipLaunchKernelGGL(k_gather_bins, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream,
                         (const int*)tmp, (const int64_t*)c->at<int64_t>(c->L.beam[s][7]), dst, n);
      HIP_OK(hipGetLastError());
    } else {
      HIP_OK(hipMemcpy(dst, bins[s], n * sizeof(int), hipMemcpyHostToDevice));
    }
  }
  st = dispatch(c, [&] { return Adj<double>(c, A).run(n_steps, n_bins, loss, grad); },
                [&] { return Adj<float>(c, A).run(n_steps, n_bins, loss, grad); });
  invalidate_counts(c);   // whatever the adjoint's own steps left in the counts
  if (st != QSA_OK) return st;
  if ((st = leave(c)) != QSA_OK) return st;
  return check_device(c);
}

qsa_status qsa_get_option(const qsa_ctx* c, int32_t option, int64_t* value) {
  if (!c || !value) return QSA_E_INVALID;
  if (option == QSA_OPT_GRAPHS) {
    *value = c->use_graphs ? 1 : 0;
    return QSA_OK;
  }
  if (option == QSA_OPT_PIPELINE) {
    *value = c->pipe_ok ? c->pipe_max : 1;
    return QSA_OK;
  }
  if (option == QSA_OPT_BEAM_BESIDE) {
    *value = c->beam_beside ? 1 : 0;
    return QSA_OK;
  }
  if (option == QSA_OPT_BESIDE_BLOCKS) {
    *value = c->beside_blocks;
    return QSA_OK;
  }
  if (option == QSA_OPT_RESORT_EVERY) {
    *value = c->resort_every;
    return QSA_OK;
  }
  if (option == QSA_OPT_PLASMA_THREADS || option == QSA_OPT_ROW_THREADS || option == QSA_OPT_COL_THREADS) {
    const qsa_params* ps[1] = {&c->p};
    int nt = 0, rt = 0, ctpt = 0;
    if (c->p.precision == QSA_FP32) {
      typename Engine<float>::Dims d;
      Engine<float>::add_dims(d, c->p);
      Engine<float>::finish_dims(d, ps, 1, c->tune_nt, c->tune_rt, c->tune_ct);
      nt = d.nt, rt = d.rt_rows, ctpt = d.ctpt;
    } else {
      typename Engine<double>::Dims d;
      Engine<double>::add_dims(d, c->p);
      Engine<double>::finish_dims(d, ps, 1, c->tune_nt, c->tune_rt, c->tune_ct);
      nt = d.nt, rt = d.rt_rows, ctpt = d.ctpt;
    }
    *value = (option == QSA_OPT_PLASMA_THREADS) ? nt : (option == QSA_OPT_ROW_THREADS) ? rt : col_tpt(c->p.ny, ctpt);
    return QSA_OK;
  }
  return QSA_E_INVALID;
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

qsa_status qsa_field_moments(qsa_ctx* c, int32_t window, double* dst, size_t count, int32_t dst_on_device) {
  if (!c) return QSA_E_INVALID;
  if (c->sticky != QSA_OK) return c->sticky;
  if (!c->swept) return fail(c, QSA_E_STATE, "no sweep has run");
  if (window < 1) return fail(c, QSA_E_INVALID, "window must be at least one slice");
  const size_t need = 6 * (size_t)((c->p.nxi + window - 1) / window);
  if (!dst || count < need) return fail(c, QSA_E_INVALID, "destination too small");
  qsa_status st = enter(c);
  if (st != QSA_OK) return st;
  st = dispatch(c, [&] { return Engine<double>::field_moments(c, window, dst, dst_on_device); },
                [&] { return Engine<float>::field_moments(c, window, dst, dst_on_device); });
  if (st != QSA_OK) return st;
  if ((st = leave(c)) != QSA_OK) return st;
  return check_device(c);
}

qsa_status qsa_beam_moments(qsa_ctx* c, int32_t species, int32_t window, double* dst, size_t count,
                            int32_t dst_on_device) {
  if (!c) return QSA_E_INVALID;
  if (c->sticky != QSA_OK) return c->sticky;
  if (species < 0 || species >= c->p.n_species) return fail(c, QSA_E_INVALID, "unknown species");
  if (window < 1) return fail(c, QSA_E_INVALID, "window must be at least one slice");
  const size_t need = 7 * (size_t)((c->p.nxi + window - 1) / window);
  if (!dst || count < need) return fail(c, QSA_E_INVALID, "destination too small");
  qsa_status st = enter(c);
  if (st != QSA_OK) return st;
  st = dispatch(c, [&] { return Engine<double>::beam_moments(c, species, window, dst, dst_on_device); },
                [&] { return Engine<float>::beam_moments(c, species, window, dst, dst_on_device); });
  if (st != QSA_OK) return st;
  if ((st = leave(c)) != QSA_OK) return st;
  return check_device(c);
}

qsa_status qsa_linear_model(int32_t n_inst, int32_t nxi, double dxi, double dtau, const double* gamma,
                            int32_t gamma_per_point, const double* n0, int32_t n_tau, const double* taus, double* n_out, double* psi_out,
                            void* hip_stream) {
  if (n_inst < 1 || nxi < 1 || nxi > QSA_LIN_THREADS * QSA_LIN_SEG) return QSA_E_INVALID;
  if (!(dxi > 0.0) || !std::isfinite(dxi) || !(dtau > 0.0) || !std::isfinite(dtau)) return QSA_E_INVALID;
  if (n_tau < 1 || n_tau > QSA_LIN_MAX_OUT) return QSA_E_INVALID;
  if (gamma_per_point != 0 && gamma_per_point != 1) return QSA_E_INVALID;
  if (!gamma || !n0 || !taus || !n_out || !psi_out) return QSA_E_INVALID;
  LinOut out{};
  out.n = n_tau;
  double t = 0.0;
  int64_t acc = 0;
  for (int m = 0; m < n_tau; ++m) {
    if (!std::isfinite(taus[m])) return QSA_E_INVALID;
    // steps to the next output time, rounded to the nearest (ties to even)
    const double k = std::nearbyint((taus[m] - t) / dtau);
    if (k < 0.0 || k > 1e9) return QSA_E_INVALID;
    acc += (int64_t)k;
    t += k * dtau;
    out.steps[m] = acc;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  hipLaunchKernelGGL(k_linear_model, dim3(n_inst), dim3(QSA_LIN_THREADS), 0, st, nxi, dxi, dtau, gamma, (int)gamma_per_point,
                     n0, out,
                     n_out, psi_out);
  return hipGetLastError() == hipSuccess ? QSA_OK : QSA_E_DEVICE;
}

}  // extern "C"

namespace {

template <typename R>
qsa_status dirichlet_launch(int n_grid, int nx, int ny, double dx, double dy, double kappa2, const void* f,
                            void* u, hipStream_t st) {
  const int Mx = 2 * (nx + 1);
  const int lgx = ilog2(Mx);
  const double inv_lx = 1.0 / ((nx + 1) * dx);
  const int64_t nrows = (int64_t)n_grid * ny;
  const int64_t bx = ((nrows + 1) / 2 + 256 / dst_tpt(Mx) - 1) / (256 / dst_tpt(Mx));
  if (ny == 1) {
    hipLaunchKernelGGL(k_dst_rows<R>, dim3((unsigned)bx), dim3(256), dst_lds<R>(Mx), st, nrows, nx, lgx,
                       (const R*)f, (R*)u, 2.0 / (nx + 1), 1, inv_lx, kappa2);
    return hipGetLastError() == hipSuccess ? QSA_OK : QSA_E_DEVICE;
  }
  const int My = 2 * (ny + 1);
  const int64_t tr = (int64_t)n_grid * ((nx + 1) / 2);
  const int64_t by = (tr + 256 / dst_tpt(My) - 1) / (256 / dst_tpt(My));
  hipLaunchKernelGGL(k_dst_rows<R>, dim3((unsigned)bx), dim3(256), dst_lds<R>(Mx), st, nrows, nx, lgx,
                     (const R*)f, (R*)u, 1.0, 0, inv_lx, kappa2);
  hipLaunchKernelGGL(k_dst_cols<R>, dim3((unsigned)by), dim3(256), dst_lds<R>(My), st, n_grid, nx, ny, ilog2(My),
                     (R*)u, inv_lx, 1.0 / ((ny + 1) * dy), kappa2, 2.0 / (ny + 1));
  hipLaunchKernelGGL(k_dst_rows<R>, dim3((unsigned)bx), dim3(256), dst_lds<R>(Mx), st, nrows, nx, lgx,
                     (const R*)u, (R*)u, 2.0 / (nx + 1), 0, inv_lx, kappa2);
  return hipGetLastError() == hipSuccess ? QSA_OK : QSA_E_DEVICE;
}

}  // namespace

extern "C" {

qsa_status qsa_dirichlet_solve(int32_t precision, int32_t n_grid, int32_t nx, int32_t ny, double dx, double dy,
                               double kappa2, const void* f, void* u, void* hip_stream) {
  if (precision != QSA_FP64 && precision != QSA_FP32) return QSA_E_INVALID;
  if (n_grid < 0 || !pow2(nx + 1) || nx + 1 < 2 || nx + 1 > kMaxN) return QSA_E_INVALID;
  if (!(ny == 1 || (pow2(ny + 1) && ny + 1 >= 2 && ny + 1 <= kMaxN))) return QSA_E_INVALID;
  if (!(dx > 0.0) || !std::isfinite(dx) || !(dy > 0.0) || !std::isfinite(dy)) return QSA_E_INVALID;
  if (!(kappa2 >= 0.0) || !std::isfinite(kappa2)) return QSA_E_INVALID;
  if ((int64_t)n_grid * ny * nx > ((int64_t)1 << 34)) return QSA_E_INVALID;
  if (n_grid == 0) return QSA_OK;
  if (!f || !u) return QSA_E_INVALID;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  return precision == QSA_FP64 ? dirichlet_launch<double>(n_grid, nx, ny, dx, dy, kappa2, f, u, st)
                               : dirichlet_launch<float>(n_grid, nx, ny, dx, dy, kappa2, f, u, st);
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
  int nxi_max = 0;
  for (qsa_ctx* m : b->ctxs) nxi_max = std::max(nxi_max, m->p.nxi);
  const bool graphs = b->use_graphs && c->timing_class < 0 && graph_fits(nxi_max);
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
      for (qsa_ctx* m : b->ctxs) {
        m->swept = true;
        m->cur_set = 0;
      }
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

qsa_status qsa_batch_sweep_static(qsa_ctx* const* ctxs, int32_t n_ctx, void* hip_stream) {
  if (!ctxs || n_ctx < 1) return QSA_E_INVALID;
  qsa_ctx* c = ctxs[0];
  for (int i = 0; i < n_ctx; ++i)
    if (!ctxs[i]) return QSA_E_INVALID;
  if (n_ctx > QSA_STATIC_MAX_CTX)
    return fail(c, QSA_E_INVALID,
                "qsa_batch_sweep_static: " + std::to_string(n_ctx) + " contexts, more than the " +
                    std::to_string(QSA_STATIC_MAX_CTX) + " its static lane table holds");
  for (int i = 0; i < n_ctx; ++i) {
    qsa_ctx* m = ctxs[i];
    if (m->sticky != QSA_OK) return m->sticky;
    if (m->p.precision != c->p.precision || m->p.n_corr != c->p.n_corr)
      return fail(c, QSA_E_INVALID, "qsa_batch_sweep_static: members differ in precision or n_corr");
    if (!m->plasma_loaded) return fail(c, QSA_E_STATE, "qsa_batch_sweep_static: a member has no plasma loaded");
    if (m->timing_class >= 0) return fail(c, QSA_E_STATE, "qsa_batch_sweep_static: kernel timing is active");
    for (int k = 0; k < i; ++k)
      if (ctxs[k] == m) return fail(c, QSA_E_INVALID, "qsa_batch_sweep_static: a context appears twice");
  }
  std::string why;
  void* table = scratch_on_current_device(why);
  if (!table) {
    c->sticky = QSA_E_DEVICE;
    return fail(c, QSA_E_DEVICE, "qsa_batch_sweep_static: " + why);
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  return c->p.precision == QSA_FP32 ? static_sweep<float>(ctxs, n_ctx, st, table)
                                    : static_sweep<double>(ctxs, n_ctx, st, table);
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
