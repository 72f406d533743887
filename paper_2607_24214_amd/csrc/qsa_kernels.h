// HIP kernels of the QSA slice sweep and beam push (gfx950).
//
// Per xi slice j the host enqueues, in order:
//   k_dep_S      plasma rho - J_z deposit                     -> dep[0]
//   k_row_r2c    real rows -> half spectra (+ ions + beam)    -> rowspec
//   k_col<PSI>   y transforms, psi, d_x psi, d_y psi          -> colout
//   k_row_c2r    half spectra -> real rows                    -> fields[j]
//   k_dep_J      gather psi, deposit J_x, J_y, J_z            -> dep[0..2]
//   k_row_r2c / k_col<J> / k_row_c2r                          -> B_z, E_z, B_perp^(0)
//   K x { k_push<pred> (predicted J_perp at j+1) / k_row_r2c / k_col<B> / k_row_c2r }
//   k_push<final>  advance the plasma to slice j+1
// The spectral state that links slices (J_perp of slice j-1, J_z, the B_perp
// iterate and its two predecessors, the transverse-mean wake) lives in the
// workspace and is touched only by the k_col kernels.
#pragma once

#include "qsa_device.h"

namespace qsa {

enum { COL_PSI = 0, COL_J = 1, COL_B = 2 };
// stored field slots
enum { F_PSI = 0, F_DXPSI = 1, F_DYPSI = 2, F_EZ = 3, F_BX = 4, F_BY = 5, F_BZ = 6, N_STORED = 7 };
// grids of the current slice the plasma pushes gather: the six pushed
// fields at j + 1/2, (3 F^j - F^{j-1})/2 (H_PSI .. H_BZ, in the order of
// PlasmaArgs::F0), and psi extrapolated to j + 1, 3 psi^j - 3 psi^{j-1} +
// psi^{j-2} (H_PSIT); written by the inverse row transforms with the fields
enum { H_PSI = 0, H_DXPSI, H_DYPSI, H_BX, H_BY, H_BZ, H_PSIT, N_HALF };
enum { ERR_BREAKDOWN = 1, ERR_DRIFT = 2 };

#define QSA_GMIN 1.0e-3
#define QSA_SORT_EVERY 8   // the plasma is counting-sorted by cell every this many slices
#define QSA_PIPE_LAG 8     // slices between successive beam steps in flight
#define QSA_PUSH_LAG 3     // a lane pushes beam slab j once it has finished slice j + 3
// A pushed particle of slab j must sit in cells [j - QSA_DRIFT_BACK,
// j + QSA_PUSH_LAG): its fields are final up to node slice j + QSA_PUSH_LAG,
// and its deposit (node slices down to j - QSA_DRIFT_BACK) must precede the
// next lane's first use of them.  Particles only drift to larger xi, so a
// particle of slab j never sits behind cell j; the guard flags anything else.
#define QSA_DRIFT_BACK 1
static_assert(QSA_PIPE_LAG % QSA_SORT_EVERY == 0 && QSA_PIPE_LAG > QSA_PUSH_LAG + QSA_DRIFT_BACK + 2, "pipeline lag");

// One box's slice loop: geometry, constants and every array the per-slice
// kernels touch.  The per-slice kernels take an array of lanes and a tick t;
// blockIdx.z selects the lane, which works on slice j = t - lag, so one
// launch advances many slice loops by one slice: independent boxes of a
// batched scan (lag 0), or successive beam steps of one box in flight at
// once (lag = k * QSA_PIPE_LAG).  A lane with j outside [0, nxi) returns.
template <typename R>
struct Lane {
  Geo<R> g;
  int lag;              // the lane works on slice j = t - lag at tick t
  int np;               // plasma macro-particles per slice
  R q;                  // -w/(dx dy): plasma rho - J_z per particle per unit area
  R h;                  // dxi
  R kappa2;             // Helmholtz shift of the B_perp iteration
  R* fields;            // [7][nxi][ny][nx]
  R* half;              // [N_HALF][ny][nx] of the slice being swept
  const R* src;         // beam sources [4][nxi][ny][nx]
  const double* tpos[2];  // plasma template x, y (float64 in either precision)
  const R* tmom[2];       // and u_x, u_y
  const R* tqw;           // and its weights relative to plasma_w (null: all 1)
  const R* ion;           // immobile ions' density at the nodes [ny][nx] (null: all 1)
  R ion_s;                // -Z/M of the mobile ions (particles with a negative relative weight)
  const C2<R>* twx;     // transform tables
  const C2<R>* twy;
  const R* kx2;
  const R* kdx;
  const R* ky2;
  const R* kdy;
  int* err;             // sticky device error flags
  double* pos[2][2];    // plasma x, y (float64), two buffer sets (sorts ping-pong)
  R* mom[2][2];         // plasma u_x, u_y, the same two sets
  R* qw[2];             // plasma relative weights, the same two sets (or null)
  int* cell_of;         // sort scratch
  int* count;
  int* bsum;
  int* prow;            // [ny + 1] first particle of each cell row
  R* ppart;             // plasma partial node rows [ny][4][3][nx]
  R* dep;               // out-of-row plasma deposits [3][nperp]
  C2<R>* rowspec;       // row-pass half spectra [4][ny][nxh]
  C2<R>* colout;        // column-pass outputs [4][ny][nxh]
  C2<R>* jring;         // J_perp spectra, ring of 2 slices [2][2][nxh][ny]
                        // (this and jz, bring: column-major, [kx][ky], as only the
                        // column pass touches them)
  C2<R>* jz;            // J_z spectrum [nxh][ny]
  C2<R>* bring;         // B_perp spectra, ring of 3 slices [3][2][nxh][ny]
  double* ode;          // [<E_z> at j-1/2, <psi> at j]
  R* fpack;             // the beam push's fields, packed per node (or null):
                        // [pack_ring][ny][nx][pack_stride<R>()], slice j in slot
                        // j % pack_ring
  int pack_ring;        // QSA_PACK_RING (steps in flight) or nxi (every slice)
  R* rk2c;              // RK2 cache of the slice, one record of 8 values per
                        // plasma particle (see rk2_full): the midpoint x, y
                        // (float64), or in float32 its offset from x, y (formed
                        // in float32, so x + offset is the midpoint exactly),
                        // then the parts of its RK2 step that B_perp does not
                        // enter (see rk2_full), written by the first predictor
                        // pass of a slice, read by the later ones and the final
                        // advance
};

// Fields of the beam push packed per node for aligned vector gathers:
// (d_x psi, d_y psi, E_z, B_x, B_y, B_z) in 48 bytes (float64) or in 32
// bytes with two unused (float32), in a ring of QSA_PACK_RING slices (slot
// j % QSA_PACK_RING).  The push of a lane's tick t reads node slices
// t - lag - QSA_PUSH_LAG - QSA_DRIFT_BACK .. t - lag (up to four back).
#define QSA_PACK_RING 8
// The beam work of tick t runs beside the slice loop's next ticks; the final
// advance of tick t + QSA_RING_WAIT (which packs a slice into the ring) waits
// for it.  That final advance must come before the ring slot of the lowest
// slice the push reads is overwritten, and before the next lane first reads
// the lowest source slice the deposit writes (at tick
// t + QSA_PIPE_LAG - QSA_PUSH_LAG - QSA_DRIFT_BACK - 1, for the predictor's
// J_perp one slice ahead).
#define QSA_RING_WAIT 2
static_assert(QSA_RING_WAIT >= 1, "the beam work of tick t starts after tick t");
static_assert(QSA_RING_WAIT <= QSA_PACK_RING - QSA_PUSH_LAG - QSA_DRIFT_BACK, "packed ring overwritten too early");
static_assert(QSA_RING_WAIT <= QSA_PIPE_LAG - QSA_PUSH_LAG - QSA_DRIFT_BACK - 2, "sources read too early");
template <typename R>
__host__ __device__ constexpr int pack_stride() {
  return sizeof(R) == 8 ? 6 : 8;
}

// plasma buffer set that holds the state at slice j
__device__ __forceinline__ int plasma_set(int j) { return (j / QSA_SORT_EVERY) & 1; }

enum { ST_PSI = 0, ST_J = 1, ST_B = 2 };   // the three solve stages of a slice

// ----------------------------------------------------------------- utility
template <typename R>
__global__ void k_fill(R* __restrict__ p, int64_t n, R v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t s = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += s) p[i] = v;
}

template <typename R>
__global__ void k_from_f64(const double* __restrict__ src, R* __restrict__ dst, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t s = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += s) dst[i] = (R)src[i];
}

template <typename R>
__global__ void k_scaled_from_f64(const double* __restrict__ src, R* __restrict__ dst, double scale, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t s = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += s) dst[i] = (R)(src[i] * scale);
}

// Multiply the negative entries by z (a mobile ion's relative weight
// becomes -Z times its weight).
template <typename R>
__global__ void k_scale_negative(R* __restrict__ p, int64_t n, R z) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (p[i] < R(0)) p[i] *= z;
}

template <typename R>
__global__ void k_to_f64(const R* __restrict__ src, double* __restrict__ dst, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t s = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += s) dst[i] = (double)src[i];
}

// dst = a*A + b*B (B may be null) as float64, n values
template <typename R>
__global__ void k_emit(const R* __restrict__ A, R a, const R* __restrict__ B, R b,
                       double* __restrict__ dst, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t s = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += s) {
    R v = a * A[i];
    if (B) v += b * B[i];
    dst[i] = (double)v;
  }
}

template <typename R>
__global__ void k_copy4(const R* __restrict__ a0, const R* __restrict__ a1,
                        const R* __restrict__ a2, const R* __restrict__ a3, R* __restrict__ b0,
                        R* __restrict__ b1, R* __restrict__ b2, R* __restrict__ b3, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    b0[i] = a0[i];
    b1[i] = a1[i];
    b2[i] = a2[i];
    b3[i] = a3[i];
  }
}

// Per-lane clears: WHAT = 0 zeroes the sweep state (J and B rings, the
// out-of-row grids, the transverse-mean wake), WHAT = 1 the sort counts.
template <typename R, int WHAT>
__global__ void k_lane_clear(const Lane<R>* __restrict__ lanes, int tick) {
  const Lane<R>& L = lanes[blockIdx.z];
  const int j = tick - L.lag;
  const Geo<R>& g = L.g;
  if (j < 0 || j >= g.nxi) return;
  const int64_t spec = (int64_t)g.ny * g.nxh;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  if (WHAT == 1) {
    if (j % QSA_SORT_EVERY != 0) return;
    for (int64_t i = i0; i < g.nperp; i += st) L.count[i] = 0;
    return;
  }
  if (j != 0) return;
  const C2<R> z{R(0), R(0)};
  for (int64_t i = i0; i < 4 * spec; i += st) L.jring[i] = z;
  for (int64_t i = i0; i < 6 * spec; i += st) L.bring[i] = z;
  for (int64_t i = i0; i < 3 * (int64_t)g.nperp; i += st) L.dep[i] = R(0);
  if (i0 < 2) L.ode[i0] = 0.0;
}

// ------------------------------------------- block-private partial node rows
// Deposits are owned: the block of plasma cell row r accumulates its
// particles in LDS and writes node rows r-1 .. r+2 (k = 0..3) with plain
// stores, ppart[((r*4 + k)*NC + c)*nx + i]; the block of beam cell row
// (j, l) writes node rows (j + dj, l - m .. l + 1 + m) of the 4 beam sources
// (layout below).  A grid value is the sum of the partial rows that cover
// it: the plasma's is formed by the row transform that consumes it, the
// beam's by one reduction pass before the sweep.  Particles that drifted
// further than the margin go through atomics instead (the plasma into the
// dep grids, the beam into the owning partial after all blocks have written).

template <typename R>
__device__ __forceinline__ R plasma_partial(const R* __restrict__ pp, int nc, int ny, int nx, int c,
                                           int L, int i) {
  R s = R(0);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    int r = L + 1 - k;
    if (ny == 1) {
      r = 0;
    } else {
      r += (r < 0) ? ny : 0;
      r -= (r >= ny) ? ny : 0;
    }
    s += pp[((size_t)(r * 4 + k) * nc + c) * nx + i];
  }
  return s;
}

// ------------------------------------------------------------ row transforms
// Row-pass inputs of field f of a stage at slice j: the plasma partial rows
// (for rho - J_z with the ion background folded in) and out-of-row grid of
// the stage's deposit, and the beam source (of slice j+1 for the predicted
// J_perp).
template <typename R>
struct RowIn {
  R* dep;             // out-of-row deposits of this field: read, then cleared
  const R* pp;        // plasma partial rows, component offset applied
  int pnc;            // components per plasma partial row block
  const R* add;       // beam source slice or null
  C2<R>* out;         // half spectra [ny][nxh]
};

template <typename R>
__device__ __forceinline__ int stage_fields_in(int stage) {
  return (stage == ST_PSI) ? 1 : (stage == ST_J ? 3 : 2);
}

template <typename R>
__device__ __forceinline__ RowIn<R> row_in(const Lane<R>& L, int j, int stage, int f) {
  const Geo<R>& g = L.g;
  const int64_t plane = (int64_t)g.nxi * g.nperp;
  RowIn<R> a;
  a.pnc = stage_fields_in<R>(stage);
  a.dep = L.dep + f * g.nperp;
  a.pp = L.ppart + (size_t)f * g.nx;
  a.out = L.rowspec + (size_t)f * g.ny * g.nxh;
  if (stage == ST_PSI) a.add = L.src + (int64_t)j * g.nperp;
  else if (stage == ST_J) a.add = L.src + (1 + f) * plane + (int64_t)j * g.nperp;
  else a.add = (j + 1 < g.nxi) ? L.src + (1 + f) * plane + (int64_t)(j + 1) * g.nperp : nullptr;
  return a;
}

template <typename R>
__device__ __forceinline__ R row_value(const Geo<R>& g, const RowIn<R>& a, int r, int i) {
  const int o = r * g.nx + i;
  R v = a.dep[o];
  a.dep[o] = R(0);
  // partial rows: block rr covers node rows rr-1 .. rr+2 (k = 0..3)
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    int rr = r + 1 - k;
    if (g.ny == 1) {
      rr = 0;
    } else {
      rr += (rr < 0) ? g.ny : 0;
      rr -= (rr >= g.ny) ? g.ny : 0;
    }
    v += a.pp[((size_t)(rr * 4 + k) * a.pnc) * g.nx + i];
  }
  if (a.add) v += a.add[o];
  return v;
}

// Real rows -> half spectra along x.  Rows 2p and 2p+1 are packed as the
// real and imaginary parts of one complex transform and separated after it.
// Block indices of a launch of gridDim.x x gridDim.y blocks per lane and
// gridDim.z lanes, remapped so that each XCD (workgroups go round-robin to
// the 8 XCDs in linear order) takes a contiguous range of the (lane, y, x)
// order: the same lanes as the particle kernels' remapping, so each lane's
// grids are written and read by one XCD and stay in its L2.
__device__ __forceinline__ void lane_block3(int& lane, int& by, int& bx) {
  const int nbx = gridDim.x, nby = gridDim.y;
  const int lg = xcd_block(blockIdx.x + nbx * (blockIdx.y + nby * blockIdx.z), nbx * nby * gridDim.z);
  bx = lg % nbx;
  const int r = lg / nbx;
  by = r % nby;
  lane = r / nby;
}

template <typename R>
__global__ void __launch_bounds__(256) k_row_r2c(const Lane<R>* __restrict__ lanes, int tick, int stage) {
  int lane, f, bx;
  lane_block3(lane, f, bx);
  const Lane<R>& L = lanes[lane];
  const int j = tick - L.lag;
  const Geo<R> g = L.g;
  if (j < 0 || j >= g.nxi || f >= stage_fields_in<R>(stage)) return;
  const RowIn<R> a = row_in(L, j, stage, f);
  const C2<R>* __restrict__ twx = L.twx;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C2<R>* sm = reinterpret_cast<C2<R>*>(smem_raw);
  const int tpt = row_tpt(g.nx);
  const int ppw = blockDim.x / tpt;
  if (bx * ppw >= ((g.ny + 1) >> 1)) return;
  const int slot = threadIdx.x / tpt, t = threadIdx.x - slot * tpt;
  const int npairs = (g.ny + 1) >> 1;
  const int pair = bx * ppw + slot;
  const bool v0 = pair < npairs;
  const int r0 = 2 * pair, r1 = 2 * pair + 1;
  const bool v1 = v0 && r1 < g.ny;
  C2<R>* tw = sm;                       // twiddles, staged once per block
  for (int i = threadIdx.x; i < g.nx; i += blockDim.x) tw[i] = twx[i];
  C2<R>* A = sm + g.nx + (size_t)slot * 2 * fft_cap(g.nx);
  C2<R>* B = A + fft_cap(g.nx);
  for (int i = t; i < g.nx; i += tpt) {
    const R va = v0 ? row_value(g, a, r0, i) : R(0);
    const R vb = v1 ? row_value(g, a, r1, i) : R(0);
    A[i] = C2<R>{va, vb};
  }
  __syncthreads();
  C2<R>* res = fft_lds<R, false>(A, B, g.nx, g.lgx, t, tpt, tw);
  if (v0) {
    C2<R>* out = a.out;
    for (int k = t; k < g.nxh; k += tpt) {
      const C2<R> z = res[k];
      const C2<R> zc = cconj(res[(g.nx - k) & (g.nx - 1)]);
      const C2<R> s = cadd(z, zc), d = csub(z, zc);
      out[r0 * g.nxh + k] = C2<R>{R(0.5) * s.x, R(0.5) * s.y};
      if (v1) out[r1 * g.nxh + k] = C2<R>{R(0.5) * d.y, R(-0.5) * d.x};
    }
  }
}

// Half spectra -> real rows (unnormalized inverse; the 1/(nx ny) factor is
// applied in the column pass).  Two rows are packed as A + iB.
// Row-pass output slot of field f of a stage: psi, d_x psi, d_y psi; or
// B_z, E_z and B_perp^(0); or the B_perp iterate.
__device__ __forceinline__ int stage_fields_out(int stage) {
  return (stage == ST_PSI) ? 3 : (stage == ST_J ? 4 : 2);
}
__device__ __forceinline__ int stage_slot(int stage, int f) {
  if (stage == ST_PSI) return f == 0 ? F_PSI : (f == 1 ? F_DXPSI : F_DYPSI);
  if (stage == ST_J) return f == 0 ? F_BZ : (f == 1 ? F_EZ : (f == 2 ? F_BX : F_BY));
  return f == 0 ? F_BX : F_BY;
}

// slot in Lane::half of a stored field (-1: E_z, not pushed with)
__device__ __forceinline__ int half_slot(int so) {
  switch (so) {
    case F_PSI: return H_PSI;
    case F_DXPSI: return H_DXPSI;
    case F_DYPSI: return H_DYPSI;
    case F_BX: return H_BX;
    case F_BY: return H_BY;
    case F_BZ: return H_BZ;
    default: return -1;
  }
}

template <typename R>
__global__ void __launch_bounds__(256) k_row_c2r(const Lane<R>* __restrict__ lanes, int tick, int stage) {
  int lane, f, bx;
  lane_block3(lane, f, bx);
  const Lane<R>& L = lanes[lane];
  const int j = tick - L.lag;
  const Geo<R> g = L.g;
  if (j < 0 || j >= g.nxi || f >= stage_fields_out(stage)) return;
  const C2<R>* __restrict__ in = L.colout + (size_t)f * g.ny * g.nxh;
  R* __restrict__ outp = L.fields + (int64_t)stage_slot(stage, f) * g.nxi * g.nperp + (int64_t)j * g.nperp;
  const C2<R>* __restrict__ twx = L.twx;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C2<R>* sm = reinterpret_cast<C2<R>*>(smem_raw);
  const int tpt = row_tpt(g.nx);
  const int ppw = blockDim.x / tpt;
  if (bx * ppw >= ((g.ny + 1) >> 1)) return;
  const int slot = threadIdx.x / tpt, t = threadIdx.x - slot * tpt;
  const int npairs = (g.ny + 1) >> 1;
  const int pair = bx * ppw + slot;
  const bool v0 = pair < npairs;
  const int r0 = 2 * pair, r1 = 2 * pair + 1;
  const bool v1 = v0 && r1 < g.ny;
  C2<R>* tw = sm;                       // twiddles, staged once per block
  for (int i = threadIdx.x; i < g.nx; i += blockDim.x) tw[i] = twx[i];
  C2<R>* A = sm + g.nx + (size_t)slot * 2 * fft_cap(g.nx);
  C2<R>* B = A + fft_cap(g.nx);
  const int half = g.nx >> 1;
  for (int i = t; i < g.nx; i += tpt) {
    C2<R> av{0, 0}, bv{0, 0};
    if (v0) {
      if (i <= half) {
        av = in[r0 * g.nxh + i];
        if (v1) bv = in[r1 * g.nxh + i];
      } else {
        const int kk = g.nx - i;
        av = cconj(in[r0 * g.nxh + kk]);
        if (v1) bv = cconj(in[r1 * g.nxh + kk]);
      }
      if (i == 0 || i == half) {
        av.y = 0;
        bv.y = 0;
      }
    }
    A[i] = C2<R>{av.x - bv.y, av.y + bv.x};
  }
  __syncthreads();
  C2<R>* res = fft_lds<R, true>(A, B, g.nx, g.lgx, t, tpt, tw);
  if (v0) {
    R* out = outp;
    for (int i = t; i < g.nx; i += tpt) {
      const C2<R> z = res[i];
      out[r0 * g.nx + i] = z.x;
      if (v1) out[r1 * g.nx + i] = z.y;
    }
    // the pushed fields at j + 1/2 (and psi extrapolated to j + 1)
    const int so = stage_slot(stage, f);
    const int hs = half_slot(so);
    if (hs >= 0) {
      R* hp = L.half + (size_t)hs * g.nperp;
      const R* m1 = (j >= 1) ? outp - g.nperp : nullptr;
      const R* m2 = (j >= 2) ? outp - 2 * g.nperp : nullptr;
      R* pt = L.half + (size_t)H_PSIT * g.nperp;
      for (int i = t; i < g.nx; i += tpt) {
        const C2<R> z = res[i];
        for (int k = 0; k < 2; ++k) {
          if (k == 1 && !v1) break;
          const int o = (k ? r1 : r0) * g.nx + i;
          const R v = k ? z.y : z.x;
          const R a = m1 ? m1[o] : R(0);
          hp[o] = R(1.5) * v - R(0.5) * a;
          if (so == F_PSI) pt[o] = R(3) * v - R(3) * a + (m2 ? m2[o] : R(0));
        }
      }
    }
  }
}

// ---------------------------------------------------------- column transforms
template <typename R>
struct ColArgs {
  C2<R>* jr_w[2];         // COL_J: spectra of J_x, J_y at slice j (ring slot j%2)
  const C2<R>* jr_r[2];   // COL_B: spectra of J_x, J_y at slice j-1
  C2<R>* jz;              // spectrum of J_z at slice j
  C2<R>* b_cur[2];        // B_x, B_y iterate at slice j (ring slot j%3)
  const C2<R>* b_m1[2];   // converged B_perp at j-1
  const C2<R>* b_m2[2];   // converged B_perp at j-2
  double* ode;            // [0] <E_z> at j-1/2, [1] <psi> at j
  const R* kx2;           // kx^2 on the half spectrum [nxh]
  const R* kdx;           // derivative multiplier kx (0 at Nyquist) [nxh]
  const R* ky2;           // ky^2 [ny]
  const R* kdy;           // derivative multiplier ky (0 at Nyquist) [ny]
  R inv_n;                // 1/(nx ny)
  R n_perp;               // nx ny
  R h;                    // dxi
  R kappa2;               // Helmholtz shift
};

template <int MODE>
struct ColShape {
  static constexpr int NIN = (MODE == COL_PSI) ? 1 : (MODE == COL_J ? 3 : 2);
  static constexpr int NOUT = (MODE == COL_PSI) ? 3 : (MODE == COL_J ? 4 : 2);
  static constexpr int G = NIN > NOUT ? NIN : NOUT;   // thread groups per column
};

// Threads per column transform for ny rows (loops cover the rest): want
// (16, 32 or 64; 0 = QSA_COL_TPT) capped at ny/4.  A wavefront takes
// 64 / threads adjacent columns, so fewer threads per transform read and
// write longer runs of each spectral row.
#define QSA_COL_TPT 64
__host__ __device__ __forceinline__ int col_tpt(int ny, int want = 0) {
  const int w = want > 0 ? want : QSA_COL_TPT;
  const int t = ny >> 2;
  return t < 1 ? 1 : (t > w ? w : t);
}

// Forward transform along y of each input column, the spectral solve of the
// mode, inverse transform along y of each output.  Each column is worked by
// G groups of tpt threads, one group per field transform, so the transforms
// of one column run side by side; cpw columns per block.
// Column-pass arguments at slice j (ring slots follow j).
template <typename R>
__device__ __forceinline__ ColArgs<R> col_args(const Lane<R>& L, int j) {
  const Geo<R>& g = L.g;
  const size_t spec = (size_t)g.ny * g.nxh;
  ColArgs<R> a;
  const int s2 = j & 1, s2m = (j + 1) & 1;                       // J ring: j % 2, (j - 1) % 2
  const int s3 = j % 3, s3m1 = (j + 2) % 3, s3m2 = (j + 1) % 3;  // B ring: j, j - 1, j - 2
  for (int q = 0; q < 2; ++q) {
    a.jr_w[q] = L.jring + (2 * s2 + q) * spec;
    a.jr_r[q] = L.jring + (2 * s2m + q) * spec;
    a.b_cur[q] = L.bring + (2 * s3 + q) * spec;
    a.b_m1[q] = L.bring + (2 * s3m1 + q) * spec;
    a.b_m2[q] = L.bring + (2 * s3m2 + q) * spec;
  }
  a.jz = L.jz;
  a.ode = L.ode;
  a.kx2 = L.kx2;
  a.kdx = L.kdx;
  a.ky2 = L.ky2;
  a.kdy = L.kdy;
  a.inv_n = R(1) / (R)g.nperp;
  a.n_perp = (R)g.nperp;
  a.h = L.h;
  a.kappa2 = L.kappa2;
  return a;
}

template <typename R, int MODE>
__global__ void __launch_bounds__(256) k_col(const Lane<R>* __restrict__ lanes, int tick, int ctpt) {
  using S = ColShape<MODE>;
  constexpr int G = S::G;
  int lane, by, bx;
  lane_block3(lane, by, bx);
  const Lane<R>& L = lanes[lane];
  const int j = tick - L.lag;
  const Geo<R> g = L.g;
  if (j < 0 || j >= g.nxi) return;
  const ColArgs<R> a = col_args(L, j);
  const C2<R>* __restrict__ twy = L.twy;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C2<R>* sm = reinterpret_cast<C2<R>*>(smem_raw);
  const int ny = g.ny;
  const int tpt = col_tpt(ny, ctpt);
  const int per_col = G * tpt;
  const int cpw = blockDim.x / per_col;
  if (bx * cpw >= g.nxh) return;
  const int c = threadIdx.x / per_col;
  const int r = threadIdx.x - c * per_col;
  const int grp = r / tpt, t = r - grp * tpt;
  const int kx = bx * cpw + c;
  const bool valid = kx < g.nxh;
  C2<R>* tw = sm;                          // twiddles, staged once per block
  for (int i = threadIdx.x; i < ny; i += blockDim.x) tw[i] = twy[i];
  const int cs = fft_cap(ny);               // column stride in LDS
  C2<R>* D = sm + ny + (size_t)c * 2 * G * cs;   // G data columns
  C2<R>* Sx = D + G * cs;                   // G scratch columns
  C2<R>* mine = D + grp * cs;
  for (int y = t; y < ny; y += tpt)
    mine[y] = (valid && grp < S::NIN) ? L.rowspec[(size_t)grp * g.ny * g.nxh + y * g.nxh + kx] : C2<R>{0, 0};
  __syncthreads();
  // every group's transform ends in the same one of its two buffers (same
  // pass count): the multipliers work there, with no copy back
  C2<R>* const Rb = (fft_lds<R, false>(mine, Sx + grp * cs, ny, g.lgy, t, tpt, tw) == mine) ? D : Sx;

  for (int y = r; y < ny; y += per_col) {
    C2<R> o[S::NOUT];
#pragma unroll
    for (int q = 0; q < S::NOUT; ++q) o[q] = C2<R>{0, 0};
    if (valid) {
      const int e = kx * ny + y;   // the spectral ring state is column-major
      const R kdx = a.kdx[kx], kdy = a.kdy[y];
      const R ksq = a.kx2[kx] + a.ky2[y];
      const bool k0 = (kx == 0 && y == 0);
      const R iks = k0 ? R(0) : R(1) / ksq;
      if (MODE == COL_PSI) {
        // -lap psi = rho - J_z; the k = 0 value is the transverse-mean wake
        C2<R> ph = cscale(Rb[y], iks);
        if (k0) ph = C2<R>{(R)a.ode[1] * a.n_perp, R(0)};
        o[0] = cscale(ph, a.inv_n);
        o[1] = cscale(cmul_ik(ph, kdx), a.inv_n);
        o[2] = cscale(cmul_ik(ph, kdy), a.inv_n);
      } else if (MODE == COL_J) {
        const C2<R> jx = Rb[y], jy = Rb[cs + y], jzv = Rb[2 * cs + y];
        a.jr_w[0][e] = jx;
        a.jr_w[1][e] = jy;
        a.jz[e] = jzv;
        // lap B_z = d_y J_x - d_x J_y ; lap E_z = div J_perp
        C2<R> bz = cscale(csub(cmul_ik(jx, kdy), cmul_ik(jy, kdx)), -iks);
        C2<R> ez = cscale(cadd(cmul_ik(jx, kdx), cmul_ik(jy, kdy)), -iks);
        if (k0) {
          // transverse mean: d_xi <E_z> = -<J_z>, d_xi <psi> = <E_z> (leapfrog)
          const double jzm = (double)jzv.x / (double)a.n_perp;
          const double eh = a.ode[0];
          const double en = eh - (double)a.h * jzm;
          const double ez0 = 0.5 * (eh + en);
          a.ode[0] = en;
          a.ode[1] = a.ode[1] + (double)a.h * en;
          ez = C2<R>{(R)ez0 * a.n_perp, R(0)};
          bz = C2<R>{0, 0};
        }
        // B_perp^(0) = 2 B_perp^{j-1} - B_perp^{j-2}
        const C2<R> bx0 = csub(cscale(a.b_m1[0][e], R(2)), a.b_m2[0][e]);
        const C2<R> by0 = csub(cscale(a.b_m1[1][e], R(2)), a.b_m2[1][e]);
        a.b_cur[0][e] = bx0;
        a.b_cur[1][e] = by0;
        o[0] = cscale(bz, a.inv_n);
        o[1] = cscale(ez, a.inv_n);
        o[2] = cscale(bx0, a.inv_n);
        o[3] = cscale(by0, a.inv_n);
      } else {
        // D = d_xi J_perp ~ (J~_perp^{j+1} - J_perp^{j-1})/(2h)
        const R i2h = R(0.5) / a.h;
        const C2<R> dx = cscale(csub(Rb[y], a.jr_r[0][e]), i2h);
        const C2<R> dy = cscale(csub(Rb[cs + y], a.jr_r[1][e]), i2h);
        const C2<R> jzv = a.jz[e];
        const C2<R> bxo = a.b_cur[0][e], byo = a.b_cur[1][e];
        const R iden = R(1) / (-ksq - a.kappa2);
        // (-|k|^2 - kappa^2) B_x' = -i ky J_z - D_y - kappa^2 B_x
        const C2<R> bxn = cscale(csub(csub(cscale(cmul_ik(jzv, kdy), R(-1)), dy), cscale(bxo, a.kappa2)), iden);
        // (-|k|^2 - kappa^2) B_y' =  i kx J_z + D_x - kappa^2 B_y
        const C2<R> byn = cscale(csub(cadd(cmul_ik(jzv, kdx), dx), cscale(byo, a.kappa2)), iden);
        a.b_cur[0][e] = bxn;
        a.b_cur[1][e] = byn;
        o[0] = cscale(bxn, a.inv_n);
        o[1] = cscale(byn, a.inv_n);
      }
    }
    // every thread of the column has read its inputs at row y before any
    // output at row y is written: rows are owned by exactly one thread here
#pragma unroll
    for (int q = 0; q < S::NOUT; ++q) Rb[q * cs + y] = o[q];
  }
  __syncthreads();
  const C2<R>* res = fft_lds<R, true>(Rb + grp * cs, ((Rb == D) ? Sx : D) + grp * cs, ny, g.lgy, t, tpt, tw);
  if (valid && grp < S::NOUT)
    for (int y = t; y < ny; y += tpt) L.colout[(size_t)grp * g.ny * g.nxh + y * g.nxh + kx] = res[y];
}

// ---------------------------------------------------------- plasma particles
template <typename R>
struct PlasmaArgs {
  double* x;          // positions in float64 for either precision
  double* y;
  R* ux;
  R* uy;
  int np;
  R q;                // -w/(dx dy): rho - J_z per particle per unit area
  const R* qw;        // per particle: its weight relative to w (null: all 1);
                      // negative for a mobile ion (-Z times its weight)
  R ion_s;            // -Z/M of the mobile ions
  R* dep0;
  R* dep1;
  R* dep2;
  const R* F0[6];     // psi, d_x psi, d_y psi, B_x, B_y, B_z at slice j
  const R* H[6];      // the six at j + 1/2: (3 F^j - F^{j-1})/2
  const R* psit;      // psi extrapolated to j + 1
  int* err;
  R h;
  const int* prow;    // [ny + 1] first particle of each cell row (state sorted by cell)
  R* ppart;           // partial node rows [ny][4][NC][nx]
  R* rk2c;            // RK2 cache of the slice, 8 values per particle (see rk2_full)
};

template <typename R>
__device__ __forceinline__ PlasmaArgs<R> plasma_args(const Lane<R>& L, int j) {
  const Geo<R>& g = L.g;
  const int64_t plane = (int64_t)g.nxi * g.nperp;
  PlasmaArgs<R> a;
  const int set = plasma_set(j);
  a.x = L.pos[set][0];
  a.y = L.pos[set][1];
  a.ux = L.mom[set][0];
  a.uy = L.mom[set][1];
  a.np = L.np;
  a.q = L.q;
  a.qw = L.qw[set];
  a.ion_s = L.ion_s;
  a.dep0 = L.dep;
  a.dep1 = L.dep + g.nperp;
  a.dep2 = L.dep + 2 * g.nperp;
  const int fs[6] = {F_PSI, F_DXPSI, F_DYPSI, F_BX, F_BY, F_BZ};
  for (int q = 0; q < 6; ++q) a.F0[q] = L.fields + fs[q] * plane + (int64_t)j * g.nperp;
  for (int q = 0; q < 6; ++q) a.H[q] = L.half + (size_t)q * g.nperp;
  a.psit = L.half + (size_t)H_PSIT * g.nperp;
  a.err = L.err;
  a.h = L.h;
  a.prow = L.prow;
  a.ppart = L.ppart;
  a.rk2c = L.rk2c;
  return a;
}

// Lane and block within it for a launch of gridDim.x blocks per lane and
// gridDim.z lanes: workgroups go round-robin to the 8 XCDs in linear order,
// so the linear index is remapped for each XCD to take consecutive blocks of
// as few lanes as possible, keeping the fields its blocks gather in its L2.
__device__ __forceinline__ void lane_block(int& lane, int& b) {
  const int per = gridDim.x;
  const int lg = xcd_block(blockIdx.x + blockIdx.z * per, per * gridDim.z);
  lane = lg / per;
  b = lg - lane * per;
}

// RK2 (midpoint) push from slice j with F^j and F^{j+1/2} = (3F^j - F^{j-1})/2
// (the latter gathered from its grids), F = (psi, d_x psi, d_y psi, B_x, B_y,
// B_z).  With G = 1 + psi and gamma = (1 + |u_perp|^2 + G^2)/(2G) at the
// stage position,
//   dx_perp/dxi = u_perp/G,
//   du_x/dxi = a_x - B_y,  a_x = gamma d_x psi/G - u_y B_z/G,
//   du_y/dxi = a_y + B_x,  a_y = gamma d_y psi/G + u_x B_z/G,
// B_z being the wake's plus the uniform guide field g.b0z.  A mobile ion
// (charge Z, mass M) has G = 1 - (Z/M) psi and both accelerations scaled by
// s = -Z/M (s = 1 for an electron); species_scale gives s.
// B_perp enters only through the last terms, and the midpoint position only
// through u_perp/G: so the stage-1 a_x, a_y, the midpoint (x_s, y_s) and
// G, d_x psi, d_y psi, B_z at the midpoint are the same in every predictor
// pass of a slice and in its final advance.  rk2_full gathers all twelve
// values (and stores those eight when `store`); rk2_cached reloads them and
// gathers only B_x, B_y at both stages.

// A particle's RK2 cache record (8 values, 32 bytes in float32 and 64 in
// float64, records aligned to their size): 16-byte vector stores and loads,
// so that a wavefront moves its 64 consecutive records in 2 (or 4)
// instructions instead of 8.
template <typename R>
__device__ __forceinline__ void rec8_store(R* __restrict__ r, const R (&v)[8]) {
  if constexpr (sizeof(R) == 4) {
    typedef float F4 __attribute__((ext_vector_type(4)));
    F4* q = reinterpret_cast<F4*>(r);
    q[0] = F4{v[0], v[1], v[2], v[3]};
    q[1] = F4{v[4], v[5], v[6], v[7]};
  } else {
    typedef double D2 __attribute__((ext_vector_type(2)));
    D2* q = reinterpret_cast<D2*>(r);
#pragma unroll
    for (int k = 0; k < 4; ++k) q[k] = D2{v[2 * k], v[2 * k + 1]};
  }
}
template <typename R>
__device__ __forceinline__ void rec8_load(const R* __restrict__ r, R (&v)[8]) {
  if constexpr (sizeof(R) == 4) {
    typedef float F4 __attribute__((ext_vector_type(4)));
    const F4* q = reinterpret_cast<const F4*>(r);
    const F4 a = q[0], b = q[1];
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  } else {
    typedef double D2 __attribute__((ext_vector_type(2)));
    const D2* q = reinterpret_cast<const D2*>(r);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const D2 t = q[k];
      v[2 * k] = t.x;
      v[2 * k + 1] = t.y;
    }
  }
}

template <typename R>
__device__ __forceinline__ R species_scale(const PlasmaArgs<R>& a, int p) {
  return (a.qw && a.qw[p] < R(0)) ? a.ion_s : R(1);
}

// The step from the cached parts and the four B_perp values (sp: the
// species' acceleration scale).
template <typename R>
__device__ __forceinline__ void rk2_finish(R hh, R sp, double x, double y, R ux, R uy, R ax, R ay, R bx1, R by1,
                                           R gs, R pxs, R pys, R bzs, R bxh, R byh, double& xn, double& yn,
                                           R& uxn, R& uyn) {
  const R hs = hh * sp;
  const R uxs = ux + R(0.5) * hs * (ax - by1);
  const R uys = uy + R(0.5) * hs * (ay + bx1);
  const R iGs = R(1) / gs;
  const R gams = (R(1) + uxs * uxs + uys * uys + gs * gs) * R(0.5) * iGs;
  // positions advance in float64 by increments formed in R
  xn = x + (double)(hh * (uxs * iGs));
  yn = y + (double)(hh * (uys * iGs));
  uxn = ux + hs * ((gams * pxs * iGs - uys * bzs * iGs) - byh);
  uyn = uy + hs * ((gams * pys * iGs + uxs * bzs * iGs) + bxh);
}

template <typename R>
__device__ __forceinline__ void rk2_full(const Geo<R>& g, const PlasmaArgs<R>& a, int p, bool store, double x,
                                         double y, R ux, R uy, double& xn, double& yn, R& uxn, R& uyn) {
  const R hh = a.h;
  const R sp = species_scale(a, p);
  R ax, ay, bx1, by1, dxs, dys;
  double xs, ys;
  {
    const Stencil<R> s = stencil2(g, x, y);
    const R G = R(1) + sp * gather(a.F0[0], s);
    if (!(G > R(QSA_GMIN))) atomicOr(a.err, ERR_BREAKDOWN);
    const R iG = R(1) / G;
    const R gam = (R(1) + ux * ux + uy * uy + G * G) * R(0.5) * iG;
    const R bz = gather(a.F0[5], s) + g.b0z;
    ax = gam * gather(a.F0[1], s) * iG - uy * bz * iG;
    ay = gam * gather(a.F0[2], s) * iG + ux * bz * iG;
    bx1 = gather(a.F0[3], s);
    by1 = gather(a.F0[4], s);
    dxs = R(0.5) * hh * (ux * iG);
    dys = R(0.5) * hh * (uy * iG);
    xs = x + (double)dxs;
    ys = y + (double)dys;
  }
  const Stencil<R> s = stencil2(g, xs, ys);
  const R gs = R(1) + sp * gather(a.H[0], s);
  if (!(gs > R(QSA_GMIN))) atomicOr(a.err, ERR_BREAKDOWN);
  const R pxs = gather(a.H[1], s), pys = gather(a.H[2], s), bzs = gather(a.H[5], s) + g.b0z;
  const R bxh = gather(a.H[3], s), byh = gather(a.H[4], s);
  if (store) {
    R rec[8];
    if constexpr (sizeof(R) == 4) {
      rec[0] = dxs;
      rec[1] = dys;
    } else {
      rec[0] = xs;
      rec[1] = ys;
    }
    rec[2] = ax;
    rec[3] = ay;
    rec[4] = gs;
    rec[5] = pxs;
    rec[6] = pys;
    rec[7] = bzs;
    rec8_store(a.rk2c + (size_t)p * 8, rec);
  }
  rk2_finish(hh, sp, x, y, ux, uy, ax, ay, bx1, by1, gs, pxs, pys, bzs, bxh, byh, xn, yn, uxn, uyn);
}

template <typename R>
__device__ __forceinline__ void rk2_cached(const Geo<R>& g, const PlasmaArgs<R>& a, int p, double x, double y,
                                           R ux, R uy, double& xn, double& yn, R& uxn, R& uyn) {
  R rec[8];
  rec8_load(a.rk2c + (size_t)p * 8, rec);
  double xs, ys;
  if constexpr (sizeof(R) == 4) {
    xs = x + (double)rec[0];
    ys = y + (double)rec[1];
  } else {
    xs = rec[0];
    ys = rec[1];
  }
  const R ax = rec[2], ay = rec[3], gs = rec[4];
  const R pxs = rec[5], pys = rec[6], bzs = rec[7];
  const Stencil<R> s1 = stencil2(g, x, y);
  const R bx1 = gather(a.F0[3], s1), by1 = gather(a.F0[4], s1);
  const Stencil<R> s2 = stencil2(g, xs, ys);
  const R bxh = gather(a.H[3], s2), byh = gather(a.H[4], s2);
  rk2_finish(a.h, species_scale(a, p), x, y, ux, uy, ax, ay, bx1, by1, gs, pxs, pys, bzs, bxh, byh, xn, yn, uxn,
             uyn);
}

// Value of lane i - N of the wavefront within its row of 16 lanes (DPP
// row_shr); only read where lane i - N lies in lane i's row.
template <int N>
__device__ __forceinline__ int lane_back(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x110 + N, 0xF, 0xF, false);
}
template <int N>
__device__ __forceinline__ float lane_back(float v) {
  return __int_as_float(lane_back<N>(__float_as_int(v)));
}
template <int N>
__device__ __forceinline__ double lane_back(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = lane_back<N>((int)(b & 0xffffffffll));
  const int hi = lane_back<N>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Segmented sums over consecutive lanes with equal keys: runs of equal keys
// are cut at every row of 16 lanes and into segments of at most 4 lanes;
// the last lane of each segment ends up with the segment's sum of the NV
// values acc and is the one that returns true (when act).  Every lane of the
// wavefront calls this together; an inactive lane passes a key no other
// lane has.
template <typename R, int NV>
__device__ __forceinline__ bool wave_segment_sum(int key, bool act, R* acc) {
  const int lane = threadIdx.x & 63;
  const int kprev = lane_back<1>(key);
  const bool head = ((lane & 15) == 0) || kprev != key;
  const unsigned long long heads = __ballot(head);
  const unsigned long long upto = (lane == 63) ? heads : (heads & ((2ull << lane) - 1ull));
  const int rs = 63 - __clzll((long long)upto);          // first lane of the run
  const int ss = rs + ((lane - rs) & ~3);                 // first lane of the segment
  const bool a1 = lane - 1 >= ss, a2 = lane - 2 >= ss;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    R v = acc[q];
    const R v1 = lane_back<1>(v);
    if (a1) v += v1;
    const R v2 = lane_back<2>(v);
    if (a2) v += v2;
    acc[q] = v;
  }
  const bool next_head = (lane == 63) || ((heads >> (lane + 1)) & 1ull);
  return act && (next_head || ((lane + 1 - rs) & 3) == 0);
}

enum { PL_DEP_S = 0, PL_DEP_J = 1, PL_PRED = 2 };

template <int MODE>
struct PlasmaNC {
  static constexpr int NC = (MODE == PL_DEP_S) ? 1 : (MODE == PL_DEP_J ? 3 : 2);
};

// Add the four-node contribution acc (nodes 00, 10, 01, 11) of cell
// (i0, l0) to the tile of block row r (node rows r-1 .. r+2), or, when the
// cell is more than one row away, to the stray grids with atomics.
template <typename R, int NC>
__device__ __forceinline__ void row_tile_add(const Geo<R>& g, double* tile, int r, int i0, int l0,
                                             const R (&acc)[4][NC], R* const* stray) {
  int d = l0 - r;
  if (g.ny == 1) {
    d = 0;
  } else {
    if (d > (g.ny >> 1)) d -= g.ny;
    if (d < -(g.ny >> 1)) d += g.ny;
  }
  const int i1 = (i0 + 1 == g.nx) ? 0 : i0 + 1;
  if (d >= -1 && d <= 1) {
    const int k0 = d + 1;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double* t0 = tile + (k0 * NC + c) * g.nx;
      double* t1 = tile + ((k0 + 1) * NC + c) * g.nx;
      atomicAdd(t0 + i0, (double)acc[0][c]);
      atomicAdd(t0 + i1, (double)acc[1][c]);
      atomicAdd(t1 + i0, (double)acc[2][c]);
      atomicAdd(t1 + i1, (double)acc[3][c]);
    }
  } else {
    const int l1 = (l0 + 1 == g.ny) ? 0 : l0 + 1;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      atomic_add(stray[c] + l0 * g.nx + i0, acc[0][c]);
      atomic_add(stray[c] + l0 * g.nx + i1, acc[1][c]);
      atomic_add(stray[c] + l1 * g.nx + i0, acc[2][c]);
      atomic_add(stray[c] + l1 * g.nx + i1, acc[3][c]);
    }
  }
}

// One plasma particle p of the row kernels: its deposit position and the
// NC values it deposits there.
//   PL_DEP_S: rho - J_z at slice j (positions only)
//   PL_DEP_J: J_x, J_y, J_z at slice j (gathers psi^j for 1 + psi)
//   PL_PRED : predictor push to j+1 and J~_perp at j+1 with 1 + psi~^{j+1},
//             psi~^{j+1} = 3 psi^j - 3 psi^{j-1} + psi^{j-2}; predictor pass
//             `pass` of the slice (the first gathers every field and caches
//             the parts of the step B_perp does not enter)
// Threads per plasma cell-row block at most: the float32 kernels fit 512
// (two wavefronts per SIMD from one block per CU, within 128 VGPRs); the
// float64 predictor needs more registers than 512 threads allow.
template <typename R>
struct PlasmaBlock {
  static constexpr int MAX = sizeof(R) == 4 ? 512 : 256;
};

template <typename R, int MODE>
__device__ __forceinline__ void plasma_particle(const Geo<R>& g, const PlasmaArgs<R>& a, int p, int pass,
                                                double& px, double& py, R (&v)[PlasmaNC<MODE>::NC]) {
  constexpr int NC = PlasmaNC<MODE>::NC;
  const R q = a.qw ? a.q * a.qw[p] : a.q;
  if constexpr (MODE == PL_DEP_S) {
    px = a.x[p];
    py = a.y[p];
    v[0] = q;
  } else if constexpr (MODE == PL_DEP_J) {
    px = a.x[p];
    py = a.y[p];
    const R ux = a.ux[p], uy = a.uy[p];
    const Stencil<R> s = stencil2(g, px, py);
    const R G = R(1) + species_scale(a, p) * gather(a.F0[0], s);
    if (!(G > R(QSA_GMIN))) atomicOr(a.err, ERR_BREAKDOWN);
    const R gam = (R(1) + ux * ux + uy * uy + G * G) / (R(2) * G);
    const R qg = q / G;
    v[0] = qg * ux;
    v[1] = qg * uy;
    v[(NC > 2) ? 2 : 0] = qg * (gam - G);
  } else {
    R uxn, uyn;
    if (pass == 0)
      rk2_full(g, a, p, true, a.x[p], a.y[p], a.ux[p], a.uy[p], px, py, uxn, uyn);
    else
      rk2_cached(g, a, p, a.x[p], a.y[p], a.ux[p], a.uy[p], px, py, uxn, uyn);
    const Stencil<R> s = stencil2(g, px, py);
    const R G = R(1) + species_scale(a, p) * gather(a.psit, s);
    if (!(G > R(QSA_GMIN))) atomicOr(a.err, ERR_BREAKDOWN);
    const R qg = q / G;
    v[0] = qg * uxn;
    v[(NC > 1) ? 1 : 0] = qg * uyn;
  }
}

// Plasma deposits owned by cell rows: block r takes the particles of cell
// row r (state sorted by cell) and adds them to its LDS tile of node rows
// r-1 .. r+2 with LDS atomics; the tile is written out as partial rows.
template <typename R, int MODE>
__global__ void __launch_bounds__(PlasmaBlock<R>::MAX) k_plasma_rows(const Lane<R>* __restrict__ lanes, int tick,
                                                                     int pass) {
  constexpr int NC = PlasmaNC<MODE>::NC;
  int lane, r;
  lane_block(lane, r);
  const Lane<R>& L = lanes[lane];
  const int j = tick - L.lag;
  const Geo<R> g = L.g;
  if (j < 0 || j >= g.nxi || r >= g.ny) return;
  const PlasmaArgs<R> a = plasma_args(L, j);
  // the LDS tile accumulates in float64 for either precision (LDS float32
  // atomic adds are about three times slower per instruction here)
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* tile = reinterpret_cast<double*>(smem_raw);
  const int nt = blockDim.x, tid = threadIdx.x;
  const int tn = 4 * NC * g.nx;
  // rho - J_z: the block's tile starts from half the ion density on node
  // rows r and r + 1 (k = 1, 2), so that every node row gets its ions once,
  // from blocks r and r - 1, and the stored partial rows hold the small
  // difference of ions and plasma instead of the plasma density (float32
  // partial rows then round that difference, not O(1) values).  The ions
  // are uniform (density 1) or follow a density profile at the nodes.
  for (int t = tid; t < tn; t += nt) {
    const int k = t / g.nx;
    double v = 0.0;
    if (MODE == PL_DEP_S && (k == 1 || k == 2)) {
      if (L.ion) {
        int row = r + k - 1;
        if (row >= g.ny) row -= g.ny;
        v = 0.5 * (double)L.ion[row * g.nx + (t - k * g.nx)];
      } else {
        v = 0.5;
      }
    }
    tile[t] = v;
  }
  __syncthreads();
  const int p0 = a.prow[r], p1 = a.prow[r + 1];
  R* stray[NC];
  stray[0] = a.dep0;
  if constexpr (NC > 1) stray[1] = a.dep1;
  if constexpr (NC > 2) stray[2] = a.dep2;
  if constexpr (MODE == PL_PRED) {
    // consecutive lanes take consecutive particles (coalesced loads of the
    // state and of the slice's RK2 cache); the row keeps its particles in
    // cell order, so the particles of a cell sit on neighbouring lanes: they
    // are summed across lanes (segmented sums) before the tile's LDS
    // atomics.  The trip count is uniform over the block, so every lane
    // reaches the sums.
    for (int base = p0; base < p1; base += nt) {
      const int p = base + tid;
      const bool act = p < p1;
      R acc[4][NC];
#pragma unroll
      for (int n = 0; n < 4; ++n)
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[n][c] = R(0);
      int i0 = 0, l0 = 0;
      if (act) {
        double px, py;
        R v[NC];
        plasma_particle<R, MODE>(g, a, p, pass, px, py, v);
        R fx, fy;
        cell2(g, px, py, i0, l0, fx, fy);
        const R ax = R(1) - fx, ay = R(1) - fy;
        const R w[4] = {ax * ay, fx * ay, ax * fy, fx * fy};
#pragma unroll
        for (int n = 0; n < 4; ++n)
#pragma unroll
          for (int c = 0; c < NC; ++c) acc[n][c] = v[c] * w[n];
      }
      const int key = act ? (l0 * g.nx + i0) : -1 - (tid & 63);
      if (wave_segment_sum<R, 4 * NC>(key, act, &acc[0][0])) row_tile_add<R, NC>(g, tile, r, i0, l0, acc, stray);
    }
  } else {
    // the deposits: each thread a contiguous run of the row's particles;
    // consecutive particles of one cell (the state is sorted by cell) add
    // up in registers and the sum goes to the tile when the cell changes
    const int run = (p1 - p0 + nt - 1) / nt;
    const int q0 = p0 + tid * run;
    const int q1 = min(q0 + run, p1);
    R acc[4][NC];
    int ci = -1, cl = -1;
    for (int p = q0; p < q1; ++p) {
      double px, py;
      R v[NC];
      plasma_particle<R, MODE>(g, a, p, pass, px, py, v);
      int i0, l0;
      R fx, fy;
      cell2(g, px, py, i0, l0, fx, fy);
      if (i0 != ci || l0 != cl) {
        if (ci >= 0) row_tile_add<R, NC>(g, tile, r, ci, cl, acc, stray);
        ci = i0;
        cl = l0;
#pragma unroll
        for (int n = 0; n < 4; ++n)
#pragma unroll
          for (int c = 0; c < NC; ++c) acc[n][c] = R(0);
      }
      const R ax = R(1) - fx, ay = R(1) - fy;
      const R w[4] = {ax * ay, fx * ay, ax * fy, fx * fy};
#pragma unroll
      for (int n = 0; n < 4; ++n)
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[n][c] += v[c] * w[n];
    }
    if (ci >= 0) row_tile_add<R, NC>(g, tile, r, ci, cl, acc, stray);
  }
  __syncthreads();
  R* out = a.ppart + (size_t)r * tn;
  for (int t = tid; t < tn; t += nt) out[t] = (R)tile[t];
}

// First particle of each cell row from the scanned cell counts (cell c
// starts at count[c] + bsum[c / 1024]); prow[ny] = np.
template <typename R>
__global__ void k_row_offsets(const Lane<R>* __restrict__ lanes, int tick) {
  const Lane<R>& L = lanes[blockIdx.z];
  const int j = tick - L.lag;
  if (j < 0 || j >= L.g.nxi) return;
  if (j % QSA_SORT_EVERY != 0) return;
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int nx = L.g.nx, ny = L.g.ny;
  if (r > ny) return;
  if (r == ny) {
    L.prow[r] = L.np;
  } else {
    const int c = r * nx;
    L.prow[r] = L.count[c] + L.bsum[c >> 10];
  }
}

// Final advance: Y^{j+1} with the converged fields, positions wrapped.
template <typename R>
__global__ void __launch_bounds__(256) k_push_final(const Lane<R>* __restrict__ lanes, int tick, int cached) {
  int lane, b;
  lane_block(lane, b);
  const Lane<R>& L = lanes[lane];
  const int j = tick - L.lag;
  const Geo<R> g = L.g;
  if (j < 0 || j >= g.nxi) return;
  const int p = b * blockDim.x + threadIdx.x;
  if (L.fpack) {
    // slice j is final: pack the beam push's fields
    const int64_t plane = (int64_t)g.nxi * g.nperp;
    const R* f = L.fields + (int64_t)j * g.nperp;
    R* dst = L.fpack + (int64_t)(j % L.pack_ring) * g.nperp * pack_stride<R>();
    const int slot[6] = {F_DXPSI, F_DYPSI, F_EZ, F_BX, F_BY, F_BZ};
    for (int o = p; o < g.nperp; o += gridDim.x * blockDim.x) {
      R v[pack_stride<R>()];
#pragma unroll
      for (int q = 0; q < 6; ++q) v[q] = f[slot[q] * plane + o];
#pragma unroll
      for (int q = 6; q < pack_stride<R>(); ++q) v[q] = R(0);
      // the record in 16-byte stores (records are 16-byte aligned)
      R* r = dst + (int64_t)o * pack_stride<R>();
      if constexpr (sizeof(R) == 8) {
        typedef double D2 __attribute__((ext_vector_type(2)));
        D2* q = reinterpret_cast<D2*>(r);
        q[0] = D2{v[0], v[1]};
        q[1] = D2{v[2], v[3]};
        q[2] = D2{v[4], v[5]};
      } else {
        typedef float F4 __attribute__((ext_vector_type(4)));
        F4* q = reinterpret_cast<F4*>(r);
        q[0] = F4{v[0], v[1], v[2], v[3]};
        q[1] = F4{v[4], v[5], v[6], v[7]};
      }
    }
  }
  if (p >= L.np) return;
  const PlasmaArgs<R> a = plasma_args(L, j);
  double xn, yn;
  R uxn, uyn;
  // with predictor passes the slice's RK2 cache holds the B_perp-free parts
  if (cached)
    rk2_cached(g, a, p, a.x[p], a.y[p], a.ux[p], a.uy[p], xn, yn, uxn, uyn);
  else
    rk2_full(g, a, p, false, a.x[p], a.y[p], a.ux[p], a.uy[p], xn, yn, uxn, uyn);
  a.x[p] = wrap_pos(xn, g.lxd, g.inv_lxd);
  a.y[p] = wrap_pos(yn, g.lyd, g.inv_lyd);
  a.ux[p] = uxn;
  a.uy[p] = uyn;
}

// Counting sort of the plasma by cell (keeps the particles of a block close
// together, which is what makes the tiled deposits pay).
// Sort at slice j (a multiple of QSA_SORT_EVERY): source buffers (the
// template at j = 0) and destination buffers.
template <typename R>
struct PlasmaSrc {
  const double* x;
  const double* y;
  const R* ux;
  const R* uy;
  const R* qw;   // relative weights (null: none kept)
};
template <typename R>
struct PlasmaDst {
  double* x;
  double* y;
  R* ux;
  R* uy;
  R* qw;
};
template <typename R>
__device__ __forceinline__ void sort_buffers(const Lane<R>& L, int j, PlasmaSrc<R>& A, PlasmaDst<R>& B) {
  const int m = j / QSA_SORT_EVERY;
  if (m == 0) {
    A = PlasmaSrc<R>{L.tpos[0], L.tpos[1], L.tmom[0], L.tmom[1], L.tqw};
  } else {
    const int a = (m - 1) & 1;
    A = PlasmaSrc<R>{L.pos[a][0], L.pos[a][1], L.mom[a][0], L.mom[a][1], L.qw[a]};
  }
  const int b = m & 1;
  B = PlasmaDst<R>{L.pos[b][0], L.pos[b][1], L.mom[b][0], L.mom[b][1], L.qw[b]};
}

template <typename R>
__global__ void __launch_bounds__(256) k_sort_count(const Lane<R>* __restrict__ lanes, int tick) {
  const Lane<R>& L = lanes[blockIdx.z];
  const int j = tick - L.lag;
  const Geo<R> g = L.g;
  if (j < 0 || j >= g.nxi) return;
  if (j % QSA_SORT_EVERY != 0) return;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= L.np) return;
  PlasmaSrc<R> A;
  PlasmaDst<R> B;
  sort_buffers(L, j, A, B);
  const double* __restrict__ x = A.x;
  const double* __restrict__ y = A.y;
  int* __restrict__ cell_of = L.cell_of;
  int* __restrict__ count = L.count;
  int i0, l0;
  R fx, fy;
  cell2(g, x[p], y[p], i0, l0, fx, fy);
  const int c = l0 * g.nx + i0;
  cell_of[p] = c;
  atomicAdd(&count[c], 1);
}

// Exclusive scan of v[0, n) in blocks of 1024: offsets within the block in
// place, block totals in bsum[block].
template <typename R>
__global__ void __launch_bounds__(256) k_scan_local(const Lane<R>* __restrict__ lanes, int tick) {
  const Lane<R>& L = lanes[blockIdx.z];
  const int j = tick - L.lag;
  if (j < 0 || j >= L.g.nxi) return;
  if (j % QSA_SORT_EVERY != 0) return;
  int* __restrict__ v = L.count;
  int* __restrict__ bsum = L.bsum;
  const int n = L.g.nperp;
  if ((int)blockIdx.x * 1024 >= n) return;
  __shared__ int s[256];
  const int t = threadIdx.x;
  const int base = blockIdx.x * 1024 + t * 4;
  int x[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) x[k] = (base + k < n) ? v[base + k] : 0;
  const int tsum = x[0] + x[1] + x[2] + x[3];
  s[t] = tsum;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int add = (t >= off) ? s[t - off] : 0;
    __syncthreads();
    s[t] += add;
    __syncthreads();
  }
  int run = s[t] - tsum;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (base + k < n) v[base + k] = run;
    run += x[k];
  }
  if (t == 255) bsum[blockIdx.x] = s[255];
}

// Exclusive scan of the (at most 256) block totals, one block.
template <typename R>
__global__ void __launch_bounds__(256) k_scan_blocks(const Lane<R>* __restrict__ lanes, int tick) {
  const Lane<R>& L = lanes[blockIdx.z];
  const int j = tick - L.lag;
  if (j < 0 || j >= L.g.nxi) return;
  if (j % QSA_SORT_EVERY != 0) return;
  int* __restrict__ bsum = L.bsum;
  const int nb = (L.g.nperp + 1023) / 1024;
  __shared__ int s[256];
  const int t = threadIdx.x;
  const int x = (t < nb) ? bsum[t] : 0;
  s[t] = x;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int add = (t >= off) ? s[t - off] : 0;
    __syncthreads();
    s[t] += add;
    __syncthreads();
  }
  if (t < nb) bsum[t] = s[t] - x;
}

// cursor[c] + bsum[c / 1024] is the first free slot of cell c.
template <typename R>
__global__ void __launch_bounds__(256) k_sort_scatter(const Lane<R>* __restrict__ lanes, int tick) {
  const Lane<R>& L = lanes[blockIdx.z];
  const int j = tick - L.lag;
  if (j < 0 || j >= L.g.nxi) return;
  if (j % QSA_SORT_EVERY != 0) return;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= L.np) return;
  PlasmaSrc<R> A;
  PlasmaDst<R> B;
  sort_buffers(L, j, A, B);
  const int* __restrict__ cell_of = L.cell_of;
  int* __restrict__ cursor = L.count;
  const int* __restrict__ bsum = L.bsum;
  const double* __restrict__ x = A.x;
  const double* __restrict__ y = A.y;
  const R* __restrict__ ux = A.ux;
  const R* __restrict__ uy = A.uy;
  double* __restrict__ x2 = B.x;
  double* __restrict__ y2 = B.y;
  R* __restrict__ ux2 = B.ux;
  R* __restrict__ uy2 = B.uy;
  const int c = cell_of[p];
  const int d = atomicAdd(&cursor[c], 1) + bsum[c >> 10];
  x2[d] = x[p];
  y2[d] = y[p];
  ux2[d] = ux[p];
  uy2[d] = uy[p];
  if (B.qw) B.qw[d] = A.qw[p];
}

// -------------------------------------------------------------------- beam
template <typename R>
struct BeamArgs {
  R* x;
  R* y;
  double* xi;
  R* ux;
  R* uy;
  R* uz;
  R* w;
  int64_t n;
  const R* fields;    // [7][nxi][nperp]
  const R* fpack;     // the same fields packed per node for every slice (or null)
  int ring;           // slots of fpack (>= nxi when set)
  R zq;               // Z/(dx dy dxi)
  R qmh;              // (Z/M) dt/2
  R dt;
  double inv_dxi;
  double xi_max;      // (nxi - 1) dxi: particles at or beyond it leave the box
};

// ------------------------------------------------------------- diagnostics
// Field moments of a sweep: block j reduces slice j of the stored fields to
// the transverse means of E_x^2, E_y^2, E_z^2, B_x^2, B_y^2, B_z^2 (E_x =
// -d_x psi + B_y, E_y = -d_y psi - B_x) in float64 and adds mean/cnt to the
// six sums of its window of ws slices (cnt = the window's slice count);
// out[(j/ws)*6 + f] must start at zero.
template <typename R>
__global__ void __launch_bounds__(256) k_field_moments(Geo<R> g, const R* __restrict__ fields, int ws,
                                                       double* __restrict__ out) {
  const int j = blockIdx.x;
  if (j >= g.nxi) return;
  const int64_t plane = (int64_t)g.nxi * g.nperp;
  const R* f = fields + (int64_t)j * g.nperp;
  double s[6] = {0, 0, 0, 0, 0, 0};
  for (int o = threadIdx.x; o < g.nperp; o += blockDim.x) {
    const double dx = f[F_DXPSI * plane + o], dy = f[F_DYPSI * plane + o], ez = f[F_EZ * plane + o];
    const double bx = f[F_BX * plane + o], by = f[F_BY * plane + o], bz = f[F_BZ * plane + o];
    const double ex = -dx + by, ey = -dy - bx;
    s[0] += ex * ex;
    s[1] += ey * ey;
    s[2] += ez * ez;
    s[3] += bx * bx;
    s[4] += by * by;
    s[5] += bz * bz;
  }
  __shared__ double red[4][6];
#pragma unroll
  for (int q = 0; q < 6; ++q)
    for (int off = 32; off >= 1; off >>= 1) s[q] += __shfl_xor(s[q], off);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int q = 0; q < 6; ++q) red[threadIdx.x >> 6][q] = s[q];
  __syncthreads();
  if (threadIdx.x < 6) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w][threadIdx.x];
    const int win = j / ws;
    const int cnt = min(ws, g.nxi - win * ws);
    atomicAdd(out + (int64_t)win * 6 + threadIdx.x, t / ((double)g.nperp * cnt));
  }
}

// Beam moments of one species: for the particles with w != 0 and slice j =
// floor(xi/dxi) in [0, nxi), the sums of (w, w u_x, w u_y, w u_z, w u_x^2,
// w u_y^2, w u_z^2) over each window of ws slices, into out[(j/ws)*7 + k]
// (zeroed before).  Block b takes particles [b CH, (b+1) CH); a thread sums
// in registers while its window stays the same (beam particles come sorted
// by slice) and folds the sums into an LDS window of QSA_DIAG_WIN windows
// from the block's first particle on, or straight into out outside it.
#define QSA_DIAG_WIN 32
#define QSA_DIAG_CHUNK 4096
template <typename R>
__global__ void __launch_bounds__(256) k_beam_moments(const double* __restrict__ xi, const R* __restrict__ ux,
                                                      const R* __restrict__ uy, const R* __restrict__ uz,
                                                      const R* __restrict__ w, int64_t n, double inv_dxi, int nxi,
                                                      int ws, double* __restrict__ out) {
  __shared__ double bins[QSA_DIAG_WIN][7];
  __shared__ int wb_s;
  const int64_t c0 = (int64_t)blockIdx.x * QSA_DIAG_CHUNK;
  for (int t = threadIdx.x; t < QSA_DIAG_WIN * 7; t += blockDim.x) (&bins[0][0])[t] = 0.0;
  if (threadIdx.x == 0) {
    const double gz = (c0 < n) ? floor(xi[c0] * inv_dxi) : 0.0;
    wb_s = (gz >= 0.0 && gz < (double)nxi) ? (int)gz / ws : 0;
  }
  __syncthreads();
  const int wb = wb_s, nwin = (nxi + ws - 1) / ws;
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  int cur = -1;
  auto flush = [&]() {
    if (cur < 0) return;
    const int k = cur - wb;
    if (k >= 0 && k < QSA_DIAG_WIN) {
#pragma unroll
      for (int q = 0; q < 7; ++q) atomicAdd(&bins[k][q], acc[q]);
    } else {
#pragma unroll
      for (int q = 0; q < 7; ++q) atomicAdd(out + (int64_t)cur * 7 + q, acc[q]);
    }
  };
  const int64_t c1 = min(n, c0 + (int64_t)QSA_DIAG_CHUNK);
  for (int64_t p = c0 + threadIdx.x; p < c1; p += blockDim.x) {
    const double wp = (double)w[p];
    const double gz = floor(xi[p] * inv_dxi);
    if (wp == 0.0 || !(gz >= 0.0 && gz < (double)nxi)) continue;
    const int win = (int)gz / ws;
    if (win != cur) {
      flush();
      cur = win;
#pragma unroll
      for (int q = 0; q < 7; ++q) acc[q] = 0.0;
    }
    const double u[3] = {(double)ux[p], (double)uy[p], (double)uz[p]};
    acc[0] += wp;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      acc[1 + a] += wp * u[a];
      acc[4 + a] += wp * u[a] * u[a];
    }
  }
  flush();
  __syncthreads();
  for (int t = threadIdx.x; t < QSA_DIAG_WIN * 7; t += blockDim.x) {
    const int k = t / 7, q = t - k * 7;
    const double v = bins[k][q];
    if (v != 0.0 && wb + k < nwin) atomicAdd(out + (int64_t)(wb + k) * 7 + q, v);
  }
}

// ------------------------------------------------------- beam source deposit
// Run-aggregated counter increments: every active lane of a wavefront takes
// the next slot of counter cnt[key]; consecutive lanes with equal keys (the
// usual case, as beam particles come nearly sorted) share one atomic.
// Returns the lane's slot.  All 64 lanes of the wavefront must call it.
__device__ __forceinline__ int lane_atomic_add(int* p, int v) { return atomicAdd(p, v); }
__device__ __forceinline__ int64_t lane_atomic_add(int64_t* p, int64_t v) {
  return (int64_t)atomicAdd(reinterpret_cast<unsigned long long*>(p), (unsigned long long)v);
}
template <typename T>
__device__ __forceinline__ T wave_run_add(T* cnt, int key, bool active) {
  const int lane = threadIdx.x & 63;
  const int k = active ? key : -1;
  const int prev = __shfl_up(k, 1);
  const bool brk = (lane == 0) || (prev != k);
  const unsigned long long b = __ballot(brk);
  const unsigned long long above = (lane == 63) ? 0ull : (b >> (lane + 1)) << (lane + 1);
  const int next = above ? __ffsll((long long)above) - 1 : 64;
  const unsigned long long upto = (lane == 63) ? b : (b & ((2ull << lane) - 1ull));
  const int head = 63 - __clzll((long long)upto);
  T base = 0;
  if (active && brk) base = lane_atomic_add(cnt + key, (T)(next - lane));
  base = __shfl(base, head);
  return base + (T)(lane - head);
}

// U independent wave_run_add's (U groups of 64 particles per wavefront),
// their atomics issued back to back before any result is waited for: one
// wavefront then keeps U round trips to the counters in flight.
template <typename T, int U>
__device__ __forceinline__ void wave_run_add_u(T* cnt, const int (&key)[U], const bool (&active)[U],
                                               T (&out)[U]) {
  const int lane = threadIdx.x & 63;
  int head[U];
  T base[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int k = active[u] ? key[u] : -1;
    const int prev = __shfl_up(k, 1);
    const bool brk = (lane == 0) || (prev != k);
    const unsigned long long b = __ballot(brk);
    const unsigned long long above = (lane == 63) ? 0ull : (b >> (lane + 1)) << (lane + 1);
    const int next = above ? __ffsll((long long)above) - 1 : 64;
    const unsigned long long upto = (lane == 63) ? b : (b & ((2ull << lane) - 1ull));
    head[u] = 63 - __clzll((long long)upto);
    base[u] = 0;
    if (active[u] && brk) base[u] = lane_atomic_add(cnt + key[u], (T)(next - lane));
  }
#pragma unroll
  for (int u = 0; u < U; ++u) out[u] = __shfl(base[u], head[u]) + (T)(lane - head[u]);
}

// Particles per thread of the key, permutation and gather passes over the
// beam (consecutive blocks of 256 per unroll step: coalesced, and U loads and
// counter round trips in flight per wavefront instead of one).
#define QSA_BEAM_UNROLL 4

// Sort key of a beam particle: cell row (j, l), j = floor(xi/dxi), then the
// chunk of QSA_BEAM_XCHUNK cells along x holding its cell, so that a
// wavefront of sorted particles gathers and deposits around a few cells.  A
// particle with j = -1 (node slice 0 only) counts as row (0, l); nxi*ny*nxc
// for a particle without a node in the grid or with nothing to deposit.
#define QSA_BEAM_XCHUNK 8
__host__ __device__ __forceinline__ int nx_chunks_of(int nx) { return nx >= QSA_BEAM_XCHUNK ? nx / QSA_BEAM_XCHUNK : 1; }
template <typename R>
__device__ __forceinline__ int nx_chunks(const Geo<R>& g) { return nx_chunks_of(g.nx); }
template <typename R>
__device__ __forceinline__ int beam_key(const Geo<R>& g, R x, R y, double xi, R w, double inv_dxi) {
  const int nxc = nx_chunks(g);
  const double gz = xi * inv_dxi;
  if (w == R(0) || !(gz > -1.0 && gz < (double)g.nxi)) return g.nxi * g.ny * nxc;
  int j = (int)floor(gz);
  j = j < 0 ? 0 : j;
  int i, l;
  R fx, fy;
  cell2(g, x, y, i, l, fx, fy);
  return (j * g.ny + l) * nxc + i / QSA_BEAM_XCHUNK;
}

// Start of every cell row among the chunk offsets: rowoff[b] = off[b*nxc]
// for b <= nrows, and the particle count after them.
template <typename R>
__global__ void __launch_bounds__(256) k_row_starts(Geo<R> g, const int64_t* __restrict__ off,
                                                    int64_t* __restrict__ rowoff) {
  const int64_t nrows = (int64_t)g.nxi * g.ny;
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int nxc = nx_chunks(g);
  if (b <= nrows) rowoff[b] = off[b * nxc];
  if (b == nrows + 1) rowoff[b] = off[nrows * nxc + 1];
}

template <typename R>
struct BeamDepArgs {
  int ns;                     // species
  const R* x[4];
  const R* y[4];
  const double* xi[4];
  const R* ux[4];
  const R* uy[4];
  const R* uz[4];
  const R* w[4];
  int* key[4];                // per particle: cell-row key (null: recomputed where needed)
  int* perm[4];               // particles of each cell row, row after row
  const int64_t* doff[4];     // chunk offsets [nxi*ny*nxc + 2]: row b's particles are
                              // perm[doff[b*nxc] .. doff[(b+1)*nxc])
  R zq[4];                    // Z/(dx dy dxi)
  double inv_dxi;
};

// Keys of species s and their counts per row (cnt zeroed by the caller);
// nothing when *skip is set (the counts are already there).  Block b takes
// particles [b, b + 1) * 256 * QSA_BEAM_UNROLL.
template <typename R>
__global__ void __launch_bounds__(256) k_beam_keys(Geo<R> g, BeamDepArgs<R> a, int s, int64_t n,
                                                   int64_t* __restrict__ cnt, const int* __restrict__ skip) {
  if (skip && *skip) return;
  constexpr int U = QSA_BEAM_UNROLL;
  const int64_t p0 = (int64_t)blockIdx.x * (256 * U) + threadIdx.x;
  int key[U];
  bool act[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t p = p0 + 256 * u;
    act[u] = p < n;
    key[u] = act[u] ? beam_key(g, a.x[s][p], a.y[s][p], a.xi[s][p], a.w[s][p], a.inv_dxi) : 0;
    if (act[u] && a.key[s]) a.key[s][p] = key[u];
  }
#pragma unroll
  for (int u = 0; u < U; ++u) (void)wave_run_add(cnt, key[u], act[u]);
}

// Particle indices grouped by key: cur holds the exclusive offsets on entry.
// Block b takes particles [b, b + 1) * 256 * QSA_BEAM_UNROLL.
template <typename R>
__global__ void __launch_bounds__(256) k_beam_perm(Geo<R> g, BeamDepArgs<R> a, int s, int64_t n,
                                                   int64_t* __restrict__ cur) {
  constexpr int U = QSA_BEAM_UNROLL;
  const int64_t p0 = (int64_t)blockIdx.x * (256 * U) + threadIdx.x;
  int key[U];
  bool act[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t p = p0 + 256 * u;
    act[u] = p < n;
    // the key kept by k_beam_keys, or the same key again (contexts without
    // steps in flight keep no key array)
    key[u] = act[u] ? (a.key[s] ? a.key[s][p] : beam_key(g, a.x[s][p], a.y[s][p], a.xi[s][p], a.w[s][p], a.inv_dxi))
                    : 0;
  }
  int64_t slot[U];
  wave_run_add_u<int64_t, U>(cur, key, act, slot);
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (act[u]) a.perm[s][slot[u]] = (int)(p0 + 256 * u);
}

// Storage re-sort of the beam by deposit key: d0[i] = s0[perm[i]] (and
// d1[i] = s1[perm[i]] when s1 is given), i < n, two beam arrays per pass of
// the permutation; then perm can become the identity.  Block b takes
// elements [b, b + 1) * 256 * QSA_BEAM_UNROLL.
template <typename T>
__global__ void __launch_bounds__(256) k_gather_perm(const T* __restrict__ s0, const T* __restrict__ s1,
                                                     T* __restrict__ d0, T* __restrict__ d1,
                                                     const int* __restrict__ perm, int64_t n) {
  constexpr int U = QSA_BEAM_UNROLL;
  const int64_t i0 = (int64_t)blockIdx.x * (256 * U) + threadIdx.x;
  int q[U];
#pragma unroll
  for (int u = 0; u < U; ++u) q[u] = (i0 + 256 * u < n) ? perm[i0 + 256 * u] : -1;
  T v0[U], v1[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    v0[u] = (q[u] >= 0) ? s0[q[u]] : T(0);
    v1[u] = (q[u] >= 0 && s1) ? s1[q[u]] : T(0);
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (q[u] < 0) continue;
    d0[i0 + 256 * u] = v0[u];
    if (s1) d1[i0 + 256 * u] = v1[u];
  }
}

// dst[0, bytes) = src[0, bytes): 16-byte vectors (both 16-byte aligned),
// the tail byte by byte.
__global__ void __launch_bounds__(256) k_copy_bytes(const unsigned char* __restrict__ src,
                                                    unsigned char* __restrict__ dst, int64_t bytes) {
  typedef unsigned int U4 __attribute__((ext_vector_type(4)));
  const int64_t nv = bytes >> 4;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += stride)
    reinterpret_cast<U4*>(dst)[i] = reinterpret_cast<const U4*>(src)[i];
  const int64_t t = (nv << 4) + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < bytes) dst[t] = src[t];
}

__global__ void __launch_bounds__(256) k_iota32(int* __restrict__ v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = (int)i;
}

// Sources of one beam particle: (rho - J_z, J_x, J_y, J_z) times Z w/dV, its
// cell and offsets.
template <typename R>
__device__ __forceinline__ void beam_sources_of(const Geo<R>& g, R x, R y, double xi, R ux, R uy, R uz, R qw,
                                                double inv_dxi, int& jc, int& i, int& l, R& fz, R& fy, R& fx,
                                                R (&v)[4]) {
  const double gz = xi * inv_dxi;
  const double fz0 = floor(gz);
  jc = (int)fz0;
  fz = (R)(gz - fz0);
  cell2(g, x, y, i, l, fx, fy);
  const R up2 = ux * ux + uy * uy;
  const R gam = sqrt(R(1) + up2 + uz * uz);
  v[0] = qw * ((R(1) + up2) / (gam * (gam + uz)));   // 1 - v_z without cancellation
  v[1] = qw * ux / gam;
  v[2] = qw * uy / gam;
  v[3] = qw * uz / gam;
}

// Add the accumulated nodes of one cell (node slices t0, t0+1 of the tile,
// t0 = the cell's slice minus the tile's first; node rows l, l+1; columns
// i, i+1; 4 sources) to a tile as tile_add lays it out.
template <typename R>
__device__ __forceinline__ void tile_add_cell(double* __restrict__ tile, int nx, int t0, int i,
                                              const R (&acc)[2][2][2][4]) {
  const int i1 = (i + 1 == nx) ? 0 : i + 1;
#pragma unroll
  for (int d = 0; d < 2; ++d) {
    if (t0 + d < 0) continue;   // node slice -1 of a particle in front of the grid
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      double* tt = tile + (((t0 + d) * 2 + e) * 4) * nx;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        atomicAdd(tt + c * nx + i, (double)acc[d][e][0][c]);
        atomicAdd(tt + c * nx + i1, (double)acc[d][e][1][c]);
      }
    }
  }
}

// Deposit of a cell row's n particles into the row's tile (src(k, ...) gives
// the row's k-th particle's cell, offsets and sources; t0 = the cell's slice
// minus the tile's first, -1 or 0): thread t takes particles 2t and 2t + 1 of
// each chunk of 2 x blockDim straight from memory (a wavefront still covers
// 128 consecutive particles, so the loads stay within a few cache lines) and
// sums them in registers when they share a cell; the lanes then sum runs of
// equal cells across the wavefront (a row keeps its particles in cell order,
// so a cell's particles sit on neighbouring lanes) before the LDS atomics,
// which same-address conflicts would otherwise serialize.
template <typename R, typename Src>
__device__ __forceinline__ void deposit_pairs(double* __restrict__ tile, int nx, int64_t n, Src src) {
  const int t = threadIdx.x;
  for (int64_t base = 0; base < n; base += 2 * (int64_t)blockDim.x) {
    // a uniform trip count: every lane reaches the cross-lane sums
    const int64_t c0 = base + 2 * (int64_t)t;
    const int m = (c0 + 1 < n) ? 2 : (c0 < n ? 1 : 0);
    int t0[2], i[2];
    R fz[2], fy[2], fx[2], v[2][4];
#pragma unroll
    for (int k = 0; k < 2; ++k)
      if (k < m) src(c0 + k, t0[k], i[k], fz[k], fy[k], fx[k], v[k]);
    R acc[2][2][2][4];
#pragma unroll
    for (int d = 0; d < 2; ++d)
#pragma unroll
      for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int c = 0; c < 4; ++c) acc[d][e][x][c] = R(0);
    int ck = -1, ct0 = 0;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if (k >= m) break;
      if (i[k] != ck || t0[k] != ct0) {
        if (ck >= 0) {
          tile_add_cell(tile, nx, ct0, ck, acc);
#pragma unroll
          for (int d = 0; d < 2; ++d)
#pragma unroll
            for (int e = 0; e < 2; ++e)
#pragma unroll
              for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[d][e][x][c] = R(0);
        }
        ck = i[k];
        ct0 = t0[k];
      }
      const R wz[2] = {R(1) - fz[k], fz[k]}, wy[2] = {R(1) - fy[k], fy[k]}, wx[2] = {R(1) - fx[k], fx[k]};
#pragma unroll
      for (int d = 0; d < 2; ++d)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const R wc = wz[d] * wy[e];
#pragma unroll
          for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[d][e][x][c] += v[k][c] * wc * wx[x];
        }
    }
    // the lane's last cell, summed with its neighbours' equal cells
    const int key = (ck >= 0) ? (((ct0 + 1) << 16) | ck) : -1 - (t & 63);
    if (wave_segment_sum<R, 32>(key, ck >= 0, &acc[0][0][0][0])) tile_add_cell(tile, nx, ct0, ck, acc);
  }
}

// Beam deposit owned by cell rows b = (j, l): the block takes exactly the
// particles of its row (through the permutation) and adds them to an LDS
// tile of node slices (j, j+1) x node rows (l, l+1) with LDS atomics.  The
// rows go in four launches by the parity of (j, l) (colour = 2 (j & 1) +
// (l & 1); in a slab only the parity of j): the blocks of one launch cover
// disjoint nodes, so each adds its tile to the dense sources [4][nxi][ny][nx]
// in place, with plain loads and stores (the sources are zeroed before the
// first launch).  A launch may cover the slabs [jlo, jhi) only; launches of
// neighbouring slab ranges share a node slice and must not overlap in time.
__host__ __device__ __forceinline__ int beam_colour_first(int jlo, int colour) {
  return jlo + ((jlo ^ (colour >> 1)) & 1);   // first slab of the colour's parity
}
__host__ __device__ __forceinline__ int beam_colour_rows(int jlo, int jhi, int ny, int colour) {
  const int cl = colour & 1;
  const int nyc = (ny == 1) ? (cl ? 0 : 1) : (ny >> 1);
  const int j0 = beam_colour_first(jlo, colour);
  return (j0 < jhi) ? ((jhi - j0 + 1) >> 1) * nyc : 0;
}

// One cell row (jb, lb) of a colour pass: tile, particles, store.
template <typename R>
__device__ __forceinline__ void beam_row(const Geo<R>& g, const BeamDepArgs<R>& a, R* __restrict__ src,
                                         double* tile, int jb, int lb);

// Threads per colour-pass block: the 2 x 2 x 4 x nx float64 tile (64 KB at
// nx = 512) allows two blocks per CU, so the float32 kernel (within 128
// VGPRs) takes 512 threads to keep four wavefronts per SIMD in flight.
template <typename R>
struct BeamRowBlock {
  static constexpr int THREADS = sizeof(R) == 4 ? 512 : 256;
};

// Block k of a launch of gridDim.x blocks takes the colour's rows k,
// k + gridDim.x, ... (one row per block when the grid covers them all).
template <typename R>
__global__ void __launch_bounds__(BeamRowBlock<R>::THREADS) k_beam_rows(Geo<R> g, BeamDepArgs<R> a, R* __restrict__ src, int colour,
                                                   int jlo, int jhi) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* tile = reinterpret_cast<double*>(smem_raw);   // float64 for either precision
  const int cl = colour & 1;
  const int nyc = (g.ny == 1) ? 1 : (g.ny >> 1);
  const int nb = beam_colour_rows(jlo, jhi, g.ny, colour);
  for (int k = blockIdx.x; k < nb; k += gridDim.x) {
    const int jj = k / nyc, ll = k - jj * nyc;
    const int jb = beam_colour_first(jlo, colour) + 2 * jj;
    const int lb = (g.ny == 1) ? 0 : 2 * ll + cl;
    if (jb >= jhi || jb >= g.nxi) continue;   // uniform over the block
    beam_row<R>(g, a, src, tile, jb, lb);
    __syncthreads();   // the tile is reused by the next row
  }
}

template <typename R>
__device__ __forceinline__ void beam_row(const Geo<R>& g, const BeamDepArgs<R>& a, R* __restrict__ src,
                                         double* tile, int jb, int lb) {
  const int b = jb * g.ny + lb;
  const int tn = 2 * 2 * 4 * g.nx;
  for (int t = threadIdx.x; t < tn; t += blockDim.x) tile[t] = 0.0;
  __syncthreads();
  for (int s = 0; s < a.ns; ++s) {
    const int nxc = nx_chunks(g);
    const int64_t q0 = a.doff[s][(int64_t)b * nxc], q1 = a.doff[s][(int64_t)(b + 1) * nxc];
    deposit_pairs<R>(tile, g.nx, q1 - q0, [&](int64_t k, int& t0, int& i, R& fz, R& fy, R& fx, R (&v)[4]) {
      const int p = a.perm[s][q0 + k];
      int jc, l;
      beam_sources_of(g, a.x[s][p], a.y[s][p], a.xi[s][p], a.ux[s][p], a.uy[s][p], a.uz[s][p],
                      a.zq[s] * a.w[s][p], a.inv_dxi, jc, i, l, fz, fy, fx, v);
      t0 = jc - jb;
    });
  }
  __syncthreads();
  // tile layout (tile_add_cell): [node slice d][node row e][source c][x]
  const int64_t plane = (int64_t)g.nxi * g.nperp;
  for (int t = threadIdx.x; t < 2 * 4 * g.nx; t += blockDim.x) {
    const int i = t % g.nx, rest = t / g.nx, c = rest & 3, d = rest >> 2;
    const int J = jb + d;
    if (J >= g.nxi) continue;
    const double v0 = tile[((d * 2 + 0) * 4 + c) * g.nx + i];
    const double v1 = tile[((d * 2 + 1) * 4 + c) * g.nx + i];
    R* base = src + c * plane + (int64_t)J * g.nperp + i;
    if (g.ny == 1) {
      // both node rows of a slab cell are row 0
      base[0] += (R)(v0 + v1);
    } else {
      const int L1 = (lb + 1 == g.ny) ? 0 : lb + 1;
      base[(int64_t)lb * g.nx] += (R)v0;
      base[(int64_t)L1 * g.nx] += (R)v1;
    }
  }
}

// Beam particles reordered by cell row (a stable-in-runs counting sort):
// particle p moves from the src arrays to slot cur[key[p]]++ of the dst
// arrays, with its identity (index at load).
template <typename R>
struct BeamMove {
  const R* src[6];        // x, y, ux, uy, uz, w
  const double* sxi;
  const int64_t* sid;
  R* dst[6];
  double* dxi;
  int64_t* did;
  const int* key;
  int64_t* cur;
  int64_t n;
};

template <typename R>
__global__ void __launch_bounds__(256) k_beam_sort(BeamMove<R> m) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = p < m.n;
  const int key = act ? m.key[p] : 0;
  const int64_t slot = wave_run_add(m.cur, key, act);
  if (!act) return;
#pragma unroll
  for (int k = 0; k < 6; ++k) m.dst[k][slot] = m.src[k][p];
  m.dxi[slot] = m.sxi[p];
  m.did[slot] = m.sid[p];
}

__global__ void __launch_bounds__(256) k_iota64(int64_t* __restrict__ v, int64_t n) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) v[p] = p;
}

// v[i] = first + i, i < n
__global__ void __launch_bounds__(256) k_iota64_from(int64_t* __restrict__ v, int64_t first, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = first + i;
}

// Back to load order as float64: dst[id[p]] = src[p].
template <typename T>
__global__ void __launch_bounds__(256) k_unpermute(const T* __restrict__ src, const int64_t* __restrict__ id,
                                                   double* __restrict__ dst, int64_t n) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) dst[id[p]] = (double)src[p];
}

// Exclusive scan of int64 values in blocks of 1024 (in place), block totals
// to bsum; k_scan64_add adds the scanned totals back.
__global__ void __launch_bounds__(256) k_scan64_local(int64_t* __restrict__ v, int64_t n,
                                                      int64_t* __restrict__ bsum) {
  __shared__ int64_t sh[256];
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * 1024 + t * 4;
  int64_t x[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) x[k] = (base + k < n) ? v[base + k] : 0;
  const int64_t tsum = x[0] + x[1] + x[2] + x[3];
  sh[t] = tsum;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int64_t add = (t >= off) ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  int64_t acc = sh[t] - tsum;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (base + k < n) v[base + k] = acc;
    acc += x[k];
  }
  if (t == 255) bsum[blockIdx.x] = sh[255];
}

__global__ void __launch_bounds__(256) k_scan64_add(int64_t* __restrict__ v, int64_t n,
                                                    const int64_t* __restrict__ bsum) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] += bsum[i >> 10];
}



// Boris push of one beam particle by dt in the stored fields, E = (-d_x psi
// + B_y, -d_y psi - B_x, E_z), B = (B_x, B_y, B_z), 3D linear shape, zero
// outside the xi grid.  Positions use the new momentum; dxi/dtau = 1 - v_z.
// A particle reaching xi >= (nxi - 1) dxi leaves the box (weight 0).
// State of a beam particle after its push (as stored), with gamma and
// u_perp^2 at the new momentum.
template <typename R>
struct BeamNew {
  R x, y, ux, uy, uz, gam, up2;
  double xi;
  bool lost;
};

// The six fields (d_x psi, d_y psi, E_z, B_x, B_y, B_z) at a beam particle:
// 3D linear shape, zero outside the xi grid; from the stored fields
// [7][nxi][ny][nx], or (packed set) from the packed ring of a pipelined lane.
template <typename R>
__device__ __forceinline__ void packed_node(const R* __restrict__ rec, R (&v)[6]) {
  if constexpr (sizeof(R) == 8) {
    typedef double D2 __attribute__((ext_vector_type(2)));
    const D2* q = reinterpret_cast<const D2*>(rec);
    const D2 a = q[0], b = q[1], c = q[2];
    v[0] = a.x;
    v[1] = a.y;
    v[2] = b.x;
    v[3] = b.y;
    v[4] = c.x;
    v[5] = c.y;
  } else {
    typedef float F4 __attribute__((ext_vector_type(4)));
    const F4* q = reinterpret_cast<const F4*>(rec);
    const F4 a = q[0], b = q[1];
    v[0] = a.x;
    v[1] = a.y;
    v[2] = a.z;
    v[3] = a.w;
    v[4] = b.x;
    v[5] = b.y;
  }
}

template <typename R>
__device__ __forceinline__ void beam_fields(const Geo<R>& g, const R* __restrict__ fields, const R* __restrict__ fpack, int ring,
                                            double inv_dxi, R x, R y, double xi, R (&fd)[6]) {
#pragma unroll
  for (int q = 0; q < 6; ++q) fd[q] = R(0);
  const double gz = xi * inv_dxi;
  if (!(gz > -1.0 && gz < (double)g.nxi)) return;
  const double fz0 = floor(gz);
  const int j0 = (int)fz0;
  const R fz = (R)(gz - fz0);
  const Stencil<R> s = stencil2(g, x, y);
  const int64_t plane = (int64_t)g.nxi * g.nperp;
  const int slot[6] = {F_DXPSI, F_DYPSI, F_EZ, F_BX, F_BY, F_BZ};
#pragma unroll
  for (int dj = 0; dj < 2; ++dj) {
    const int jj = j0 + dj;
    if (jj < 0 || jj >= g.nxi) continue;
    const R wz = dj ? fz : R(1) - fz;
    if (fpack) {
      const R* rec = fpack + (int64_t)(jj % ring) * g.nperp * pack_stride<R>();
      R a[6], b[6], c[6], d[6];
      packed_node(rec + (int64_t)s.n00 * pack_stride<R>(), a);
      packed_node(rec + (int64_t)s.n10 * pack_stride<R>(), b);
      packed_node(rec + (int64_t)s.n01 * pack_stride<R>(), c);
      packed_node(rec + (int64_t)s.n11 * pack_stride<R>(), d);
#pragma unroll
      for (int q = 0; q < 6; ++q) fd[q] += wz * (a[q] * s.w00 + b[q] * s.w10 + c[q] * s.w01 + d[q] * s.w11);
    } else {
#pragma unroll
      for (int q = 0; q < 6; ++q) fd[q] += wz * gather(fields + slot[q] * plane + (int64_t)jj * g.nperp, s);
    }
  }
}

// A beam particle's state before the push (loaded ahead of its use).
template <typename R>
struct BeamOld {
  R x, y, ux, uy, uz, w;
  double xi;
};

template <typename R>
__device__ __forceinline__ BeamOld<R> beam_old(const R* __restrict__ px, const R* __restrict__ py,
                                               const double* __restrict__ pxi, const R* __restrict__ pux,
                                               const R* __restrict__ puy, const R* __restrict__ puz,
                                               const R* __restrict__ pw, int64_t p) {
  BeamOld<R> o;
  o.x = px[p];
  o.y = py[p];
  o.xi = pxi[p];
  o.ux = pux[p];
  o.uy = puy[p];
  o.uz = puz[p];
  o.w = pw[p];
  return o;
}

// Boris push of particle p from its loaded state b; stores the new state.
template <typename R>
__device__ __forceinline__ BeamNew<R> boris_state(const Geo<R>& g, const R* __restrict__ fields,
                                                  const R* __restrict__ fpack, int ring, R qh, R dt, double inv_dxi,
                                                  double xi_max, const BeamOld<R>& b, R* __restrict__ px,
                                                  R* __restrict__ py, double* __restrict__ pxi,
                                                  R* __restrict__ pux, R* __restrict__ puy, R* __restrict__ puz,
                                                  R* __restrict__ pw, int64_t p) {
  const R x = b.x, y = b.y;
  const double xi = b.xi;
  R ux = b.ux, uy = b.uy, uz = b.uz;
  R fd[6];   // d_x psi, d_y psi, E_z, B_x, B_y, B_z
  beam_fields(g, fields, fpack, ring, inv_dxi, x, y, xi, fd);
  const R ex = -fd[0] + fd[4];
  const R ey = -fd[1] - fd[3];
  const R ez = fd[2];
  const R bx = fd[3], by = fd[4], bz = fd[5] + g.b0z;   // wake B_z plus the guide field
  // half electric kick
  const R umx = ux + qh * ex, umy = uy + qh * ey, umz = uz + qh * ez;
  const R gm = sqrt(R(1) + umx * umx + umy * umy + umz * umz);
  const R tx = qh * bx / gm, ty = qh * by / gm, tz = qh * bz / gm;
  const R sf = R(2) / (R(1) + tx * tx + ty * ty + tz * tz);
  const R sx = sf * tx, sy = sf * ty, sz = sf * tz;
  // magnetic rotation
  const R upx = umx + (umy * tz - umz * ty);
  const R upy = umy + (umz * tx - umx * tz);
  const R upz = umz + (umx * ty - umy * tx);
  const R uqx = umx + (upy * sz - upz * sy);
  const R uqy = umy + (upz * sx - upx * sz);
  const R uqz = umz + (upx * sy - upy * sx);
  // second half kick
  ux = uqx + qh * ex;
  uy = uqy + qh * ey;
  uz = uqz + qh * ez;
  const R up2 = ux * ux + uy * uy;
  const R gam = sqrt(R(1) + up2 + uz * uz);
  BeamNew<R> o;
  o.x = wrap_pos(x + dt * ux / gam, g.lx, g.inv_lx);
  o.y = wrap_pos(y + dt * uy / gam, g.ly, g.inv_ly);
  o.xi = xi + (double)(dt * (R(1) + up2) / (gam * (gam + uz)));
  o.ux = ux;
  o.uy = uy;
  o.uz = uz;
  o.gam = gam;
  o.up2 = up2;
  o.lost = o.xi >= xi_max;
  px[p] = o.x;
  py[p] = o.y;
  pxi[p] = o.xi;
  pux[p] = ux;
  puy[p] = uy;
  puz[p] = uz;
  if (o.lost) pw[p] = R(0);
  return o;
}

template <typename R>
__device__ __forceinline__ BeamNew<R> boris_one(const Geo<R>& g, const R* __restrict__ fields,
                                                const R* __restrict__ fpack, int ring, R qh, R dt, double inv_dxi,
                                                double xi_max, R* __restrict__ px, R* __restrict__ py,
                                                double* __restrict__ pxi, R* __restrict__ pux, R* __restrict__ puy,
                                                R* __restrict__ puz, R* __restrict__ pw, int64_t p) {
  const BeamOld<R> b = beam_old<R>(px, py, pxi, pux, puy, puz, pw, p);
  return boris_state(g, fields, fpack, ring, qh, dt, inv_dxi, xi_max, b, px, py, pxi, pux, puy, puz, pw, p);
}

// Counts of deposit keys: dst = *valid ? src : 0 (the counts a push made, or
// a fresh start for k_beam_keys).
__global__ void __launch_bounds__(256) k_counts_or_zero(const int* __restrict__ valid,
                                                        const int64_t* __restrict__ src,
                                                        int64_t* __restrict__ dst, int64_t n) {
  const bool ok = *valid != 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = ok ? src[i] : 0;
}

__global__ void k_set_flag(int* __restrict__ f, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *f = v;
}

// Every particle of a species pushed once; with cnt (not null) its new
// deposit key is counted there (see k_beam_push_keys).
template <typename R>
__global__ void __launch_bounds__(256) k_beam_push(Geo<R> g, BeamArgs<R> a, int64_t* __restrict__ cnt) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = p < a.n;
  int key = 0;
  if (act) {
    const BeamOld<R> b = beam_old<R>(a.x, a.y, a.xi, a.ux, a.uy, a.uz, a.w, p);
    const BeamNew<R> n = boris_state(g, a.fields, a.fpack, a.ring, a.qmh, a.dt, a.inv_dxi, a.xi_max, b, a.x, a.y,
                                     a.xi, a.ux, a.uy, a.uz, a.w, p);
    key = beam_key(g, n.x, n.y, n.xi, n.lost ? R(0) : b.w, a.inv_dxi);
  }
  if (cnt) (void)wave_run_add(cnt, key, act);
}

// The same push for the particles whose deposit keys lie in [k0, k1):
// perm[off[k0] .. off[k1]) (the permutation and chunk offsets of the beam
// deposit, so a slab range of keys is the particles of those slabs at the
// step's start); grid-stride, as the count is only known on the device.
// With cnt (not null) every pushed particle's new deposit key is counted
// there (cnt[key] += 1), so that the next deposit needs no pass of its own
// to count them.
template <typename R>
__global__ void __launch_bounds__(256) k_beam_push_keys(Geo<R> g, BeamArgs<R> a, const int* __restrict__ perm,
                                                        const int64_t* __restrict__ off, int64_t k0, int64_t k1,
                                                        int64_t* __restrict__ cnt) {
  const int64_t q1 = off[k1];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // block-uniform trip count: every lane reaches the wavefront's key count
  for (int64_t base = off[k0] + (int64_t)blockIdx.x * blockDim.x; base < q1; base += stride) {
    const int64_t q = base + threadIdx.x;
    const bool act = q < q1;
    int key = 0;
    if (act) {
      const int64_t p = (int64_t)perm[q];
      const BeamOld<R> b = beam_old<R>(a.x, a.y, a.xi, a.ux, a.uy, a.uz, a.w, p);
      const BeamNew<R> n = boris_state(g, a.fields, a.fpack, a.ring, a.qmh, a.dt, a.inv_dxi, a.xi_max, b, a.x,
                                       a.y, a.xi, a.ux, a.uy, a.uz, a.w, p);
      key = beam_key(g, n.x, n.y, n.xi, n.lost ? R(0) : b.w, a.inv_dxi);
    }
    if (cnt) (void)wave_run_add(cnt, key, act);
  }
}

// ---------------------------------------------------------------------------
// Beam steps in flight.  Lane k of a pipelined group sweeps beam step n0 + k
// QSA_PIPE_LAG slices behind lane k - 1.  Beam particles only drift to larger
// xi (1 - v_z > 0), so once lane k has finished slice jp + 3 it can push the
// particles of beam slab jp (the particles the group's opening sort put in
// cell rows (jp, *)) with its own fields and deposit them, now at step
// n0 + k + 1, as the sources of lane k + 1, which reaches those slices
// QSA_PIPE_LAG ticks later.
//
// Per tick and lane the slab's particles are counting-sorted by their new
// cell row, without global atomics: block l of the push takes the particles
// stored under cell row (jp, l), ranks them per new row in LDS and writes
// its row of the count matrix hist[l][L]; one block per lane scans the
// matrix (start of new row L, and of source row l's share in it); the place
// pass writes every particle's index to its slot of perm; block L of the
// deposit then reads exactly the particles now in cell row (jp, L) into an
// LDS tile of node slices (jp, jp+1) x node rows (L, L+1), stored to a
// two-slab ring; node slice s of the next lane's sources is reduced from the
// ring once slab s is in.  A particle that left slice cell jp (rare: the
// drift in xi is slow) deposits with atomics straight from the push.
//
// The schedule holds while every particle of slab jp sits in
// [jp - QSA_DRIFT_BACK, jp + QSA_PUSH_LAG) cells when pushed; a violation
// sets ERR_DRIFT and the host repeats the group from a copy of the beam.
// ---------------------------------------------------------------------------
template <typename R>
struct PipeBeam {
  Geo<R> g;
  int lag;                  // this lane's slice lag
  int ns;
  R* x[4];
  R* y[4];
  double* xi[4];
  R* ux[4];
  R* uy[4];
  R* uz[4];
  R* w[4];
  const int64_t* rowoff[4]; // slab partition [nxi*ny + 2]; rowoff[nxi*ny + 1] = particle count
  int* tag[4];              // new row and rank of a pushed particle (-1: none)
  int* perm[4];             // the slab's particles by new row
  R qmh[4];                 // (Z/M) dt/2
  R zq[4];                  // Z/(dx dy dxi)
  R dt;
  double inv_dxi;
  double xi_max;
  const R* fields;          // this lane's fields (the push)
  const R* fpack;           // this lane's packed ring of them (or null)
  int* hist;                // [4 species][ny source rows][ny new rows]: counts, then slots
  int* base;                // [4 species][ny + 1]: particles of each new row in the slab
  R* ring_next;             // next lane's slab ring [2][ny][2][2][4][nx]
  R* src_next;              // next lane's sources [4][nxi][ny][nx]
  int* err;
};

// Atomic deposit of one particle into dense sources [4][nxi][ny][nx].
template <typename R>
__device__ __forceinline__ void dense_add(const Geo<R>& g, R* __restrict__ src, int jc, int i, int l, R fz, R fy,
                                          R fx, const R (&v)[4]) {
  const int64_t plane = (int64_t)g.nxi * g.nperp;
  const int i1 = (i + 1 == g.nx) ? 0 : i + 1;
  const R wz[2] = {R(1) - fz, fz}, wy[2] = {R(1) - fy, fy}, wx[2] = {R(1) - fx, fx};
#pragma unroll
  for (int dj = 0; dj < 2; ++dj) {
    const int jj = jc + dj;
    if (jj < 0 || jj >= g.nxi) continue;
#pragma unroll
    for (int dl = 0; dl < 2; ++dl) {
      const int ll = (l + dl == g.ny) ? 0 : l + dl;
      const R wc = wz[dj] * wy[dl];
      R* base = src + (int64_t)jj * g.nperp + (int64_t)ll * g.nx;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        atomic_add(base + c * plane + i, v[c] * wc * wx[0]);
        atomic_add(base + c * plane + i1, v[c] * wc * wx[1]);
      }
    }
  }
}

// Rank of each active lane among the lanes of its wavefront and of earlier
// calls with the same class c (LDS counters cnt[c]): one LDS atomic per class
// present in the wavefront.  All 64 lanes must call it together.
__device__ __forceinline__ int wave_class_rank(int* cnt, int c, bool act) {
  const int lane = threadIdx.x & 63;
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  unsigned long long rem = __ballot(act);
  int rank = 0;
  while (rem) {
    const int leader = __ffsll((long long)rem) - 1;
    const int cl = __shfl(c, leader);
    const bool mine = act && c == cl;
    const unsigned long long m = __ballot(mine);
    int base = 0;
    if (lane == leader) base = atomicAdd(cnt + cl, __popcll(m));
    base = __shfl(base, leader);
    if (mine) rank = base + __popcll(m & below);
    rem &= ~m;
  }
  return rank;
}

template <typename R>
__device__ __forceinline__ BeamOld<R> pipe_old(const PipeBeam<R>& B, int s, int64_t p) {
  return beam_old<R>(B.x[s], B.y[s], B.xi[s], B.ux[s], B.uy[s], B.uz[s], B.w[s], p);
}

// Push particle p of species s from its loaded state b; with feeds, also
// its new cell row (-1: none, or deposited here).  Returns whether the
// schedule is broken.
template <typename R>
__device__ __forceinline__ bool pipe_push_one(const PipeBeam<R>& B, int s, int64_t p, const BeamOld<R>& b, int jp,
                                              bool slab, bool feeds, int& row) {
  const Geo<R>& g = B.g;
  bool bad = false;
  row = -1;
  const double gz = b.xi * B.inv_dxi;
  if (slab) {
    // fields are final up to node slice jp + QSA_PUSH_LAG; a deposit must
    // reach the next lane before it first reads node slice jp - QSA_DRIFT_BACK
    if (gz > -1.0 && gz < (double)g.nxi && gz >= (double)(jp + QSA_PUSH_LAG)) bad = true;
    if (feeds && b.w != R(0) && gz < (double)(jp - QSA_DRIFT_BACK)) bad = true;
  }
  const R w0 = b.w;
  const BeamNew<R> n = boris_state(g, B.fields, B.fpack, QSA_PACK_RING, B.qmh[s], B.dt, B.inv_dxi, B.xi_max, b,
                                   B.x[s], B.y[s],
                                   B.xi[s], B.ux[s], B.uy[s], B.uz[s], B.w[s], p);
  if (!feeds) return bad;
  const R w = n.lost ? R(0) : w0;
  const double gn = n.xi * B.inv_dxi;
  const bool deposits = w != R(0) && gn > -1.0 && gn < (double)g.nxi;
  if (!slab) return bad || deposits;   // not deposited for the next lane: must carry nothing
  if (deposits) {
    // its cell from the new state in registers; the sources only for a
    // particle that left slab jp (deposited here, with atomics)
    const int jc = (int)floor(gn);
    int i, l;
    R fx, fy;
    cell2(g, n.x, n.y, i, l, fx, fy);
    if (jc == jp) {
      row = l;
    } else {
      const R qw = B.zq[s] * w;
      const R v[4] = {qw * ((R(1) + n.up2) / (n.gam * (n.gam + n.uz))), qw * n.ux / n.gam, qw * n.uy / n.gam,
                      qw * n.uz / n.gam};
      dense_add(g, B.src_next, jc, i, l, (R)(gn - floor(gn)), fy, fx, v);
    }
  }
  return bad;
}

template <typename R>
__global__ void __launch_bounds__(256) k_pipe_push(const PipeBeam<R>* __restrict__ tab, int tick, int nlanes) {
  // blocks in launch order (all XCDs on the rows of one lane at a time)
  const int lane = blockIdx.z, l = blockIdx.x;
  const PipeBeam<R>& B = tab[lane];
  const Geo<R>& g = B.g;
  const int jp = tick - B.lag - QSA_PUSH_LAG;
  if (jp < 0 || jp > g.nxi - 2 || l >= g.ny) return;
  const bool feeds = lane + 1 < nlanes;
  const int64_t row = (int64_t)jp * g.ny + l;
  __shared__ int cnt[512];
  bool bad = false;
  for (int s = 0; s < B.ns; ++s) {
    for (int i = threadIdx.x; i < g.ny; i += blockDim.x) cnt[i] = 0;
    __syncthreads();
    const int64_t p0 = B.rowoff[s][row], p1 = B.rowoff[s][row + 1];
    // each thread loads its next particle before pushing the current one
    BeamOld<R> cur{}, nxt{};
    if (p0 + threadIdx.x < p1) cur = pipe_old(B, s, p0 + threadIdx.x);
    for (int64_t b0 = p0; b0 < p1; b0 += blockDim.x) {
      const int64_t p = b0 + threadIdx.x;
      const bool act = p < p1;
      if (p + blockDim.x < p1) nxt = pipe_old(B, s, p + blockDim.x);
      int L = -1;
      if (act) bad |= pipe_push_one(B, s, p, cur, jp, true, feeds, L);
      cur = nxt;
      if (!feeds) continue;
      const int r = wave_class_rank(cnt, L, act && L >= 0);
      if (act) B.tag[s][p] = (L >= 0) ? ((r << 9) | L) : -1;
    }
    if (feeds) {
      __syncthreads();
      int* h = B.hist + ((int64_t)s * g.ny + l) * g.ny;
      for (int i = threadIdx.x; i < g.ny; i += blockDim.x) h[i] = cnt[i];
    }
    if (jp == g.nxi - 2) {
      // the last pushable slab also takes slab nxi - 1 and the out-of-grid tail
      const int64_t nrows = (int64_t)g.nxi * g.ny;
      const int64_t t1 = B.rowoff[s][nrows + 1];
      for (int64_t p = B.rowoff[s][(int64_t)(jp + 1) * g.ny] + (int64_t)l * blockDim.x + threadIdx.x; p < t1;
           p += (int64_t)g.ny * blockDim.x) {
        int L;
        bad |= pipe_push_one(B, s, p, pipe_old(B, s, p), jp, false, feeds, L);
      }
    }
    __syncthreads();
  }
  if (bad) atomicOr(B.err, ERR_DRIFT);
}

// Exclusive prefix sums of n <= 2 blockDim.x values val(i), i < n, into
// out[0..n] in LDS (out[n] = their total); ws: LDS scratch of blockDim.x/64
// ints.  Every thread of the block calls this; it ends with a barrier.
template <typename F>
__device__ __forceinline__ void block_exclusive_scan(F val, int n, int* out, int* ws) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int a = (2 * t < n) ? val(2 * t) : 0;
  const int b = (2 * t + 1 < n) ? val(2 * t + 1) : 0;
  const int s = a + b;
  int inc = s;
  for (int o = 1; o < 64; o <<= 1) {
    const int u = __shfl_up(inc, o);
    if (lane >= o) inc += u;
  }
  if (lane == 63) ws[w] = inc;
  __syncthreads();
  int wb = 0;
  for (int k = 0; k < w; ++k) wb += ws[k];
  const int ex = wb + inc - s;
  if (2 * t < n) out[2 * t] = ex;
  if (2 * t + 1 < n) out[2 * t + 1] = ex + a;
  if (t == (int)blockDim.x - 1) out[n] = wb + inc;
  __syncthreads();
}

// Block L of a lane: the column of new row L in hist (its particles from
// each source row l) becomes its exclusive prefix over l, i.e. the first
// slot of source row l's particles within new row L; base[L] <- the row's
// count (k_pipe_place and k_pipe_deposit form the row starts from these).
template <typename R>
__global__ void __launch_bounds__(256) k_pipe_scan(const PipeBeam<R>* __restrict__ tab, int tick, int nlanes) {
  const int lane = blockIdx.z, L = blockIdx.x;
  if (lane + 1 >= nlanes) return;
  const PipeBeam<R>& B = tab[lane];
  const Geo<R>& g = B.g;
  const int jp = tick - B.lag - QSA_PUSH_LAG;
  if (jp < 0 || jp > g.nxi - 2 || L >= g.ny) return;
  __shared__ int col[513];
  __shared__ int ws[16];
  for (int s = 0; s < B.ns; ++s) {
    int* h = B.hist + (int64_t)s * g.ny * g.ny;
    block_exclusive_scan([&](int l) { return h[(int64_t)l * g.ny + L]; }, g.ny, col, ws);
    for (int l = threadIdx.x; l < g.ny; l += blockDim.x) h[(int64_t)l * g.ny + L] = col[l];
    if (threadIdx.x == 0) B.base[s * (g.ny + 1) + L] = col[g.ny];
    __syncthreads();
  }
}

// Block l writes the index of every particle stored under cell row (jp, l)
// to its slot in the slab's permutation by new row.
template <typename R>
__global__ void __launch_bounds__(256) k_pipe_place(const PipeBeam<R>* __restrict__ tab, int tick, int nlanes) {
  const int lane = blockIdx.z, l = blockIdx.x;
  if (lane + 1 >= nlanes) return;
  const PipeBeam<R>& B = tab[lane];
  const Geo<R>& g = B.g;
  const int jp = tick - B.lag - QSA_PUSH_LAG;
  if (jp < 0 || jp > g.nxi - 2 || l >= g.ny) return;
  const int64_t row = (int64_t)jp * g.ny + l;
  __shared__ int base[513];
  __shared__ int ws[16];
  for (int s = 0; s < B.ns; ++s) {
    const int64_t s0 = B.rowoff[s][(int64_t)jp * g.ny];
    const int* h = B.hist + ((int64_t)s * g.ny + l) * g.ny;
    const int* cnt = B.base + s * (g.ny + 1);
    block_exclusive_scan([&](int L) { return cnt[L]; }, g.ny, base, ws);
    const int64_t p1 = B.rowoff[s][row + 1];
    for (int64_t p = B.rowoff[s][row] + threadIdx.x; p < p1; p += blockDim.x) {
      const int t = B.tag[s][p];
      if (t < 0) continue;
      const int L = t & 511;
      B.perm[s][s0 + base[L] + h[L] + (t >> 9)] = (int)p;
    }
    __syncthreads();
  }
}

// Block L deposits the particles now in cell row (jp, L).
template <typename R>
__global__ void __launch_bounds__(BeamRowBlock<R>::THREADS) k_pipe_deposit(const PipeBeam<R>* __restrict__ tab,
                                                                             int tick, int nlanes) {
  int lane, L;
  lane_block(lane, L);
  if (lane + 1 >= nlanes) return;   // the last lane feeds no one
  const PipeBeam<R>& B = tab[lane];
  const Geo<R>& g = B.g;
  const int jp = tick - B.lag - QSA_PUSH_LAG;
  if (jp < 0 || jp > g.nxi - 2 || L >= g.ny) return;
  // LDS: the tile, the row starts (ny + 1), scan scratch (16)
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* tile = reinterpret_cast<double*>(smem_raw);   // float64 for either precision
  const int tn = 2 * 2 * 4 * g.nx;
  int* base = reinterpret_cast<int*>(tile + tn);
  int* ws = base + g.ny + 1;
  for (int i = threadIdx.x; i < tn; i += blockDim.x) tile[i] = 0.0;
  __syncthreads();
  for (int s = 0; s < B.ns; ++s) {
    const int* cnt = B.base + s * (g.ny + 1);
    block_exclusive_scan([&](int l) { return cnt[l]; }, g.ny, base, ws);
    const int64_t s0 = B.rowoff[s][(int64_t)jp * g.ny];
    const int64_t q0 = s0 + base[L], q1 = s0 + base[L + 1];
    __syncthreads();
    deposit_pairs<R>(tile, g.nx, q1 - q0, [&](int64_t k, int& t0, int& i, R& fz, R& fy, R& fx, R (&v)[4]) {
      const int p = B.perm[s][q0 + k];
      int jc, lc;
      beam_sources_of(g, B.x[s][p], B.y[s][p], B.xi[s][p], B.ux[s][p], B.uy[s][p], B.uz[s][p],
                      B.zq[s] * B.w[s][p], B.inv_dxi, jc, i, lc, fz, fy, fx, v);
      t0 = jc - jp;
    });
  }
  __syncthreads();
  R* out = B.ring_next + ((int64_t)(jp & 1) * g.ny + L) * tn;
  for (int i = threadIdx.x; i < tn; i += blockDim.x) out[i] = (R)tile[i];
}

// Node slice s of the next lane gets corner dj of slabs s - dj and corner k
// of cell rows L - k; slab nxi - 1 deposits nothing.
template <typename R>
__device__ __forceinline__ void pipe_reduce_slice(const PipeBeam<R>& B, int s, int o) {
  const Geo<R>& g = B.g;
  const int L = o / g.nx, i = o - L * g.nx;
  const int64_t plane = (int64_t)g.nxi * g.nperp;
  const int tn = 2 * 2 * 4 * g.nx;
  R acc[4] = {0, 0, 0, 0};
#pragma unroll
  for (int dj = 0; dj < 2; ++dj) {
    const int sj = s - dj;
    if (sj < 0 || sj > g.nxi - 2) continue;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      int ll = L - k;
      ll = (g.ny == 1) ? 0 : ((ll < 0) ? ll + g.ny : ll);
      const R* r = B.ring_next + ((int64_t)(sj & 1) * g.ny + ll) * tn + ((dj * 2 + k) * 4) * g.nx + i;
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] += r[c * g.nx];
    }
  }
  R* dst = B.src_next + (int64_t)s * g.nperp + o;
#pragma unroll
  for (int c = 0; c < 4; ++c) dst[c * plane] += acc[c];
}

template <typename R>
__global__ void __launch_bounds__(256) k_pipe_reduce(const PipeBeam<R>* __restrict__ tab, int tick, int nlanes) {
  if ((int)blockIdx.z + 1 >= nlanes) return;
  const PipeBeam<R>& B = tab[blockIdx.z];
  const Geo<R>& g = B.g;
  const int jp = tick - B.lag - QSA_PUSH_LAG;
  if (jp < 0 || jp > g.nxi - 2) return;
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= g.nperp) return;
  pipe_reduce_slice(B, jp, o);
  if (jp == g.nxi - 2) pipe_reduce_slice(B, jp + 1, o);   // the last node slice has no slab of its own
}

}  // namespace qsa
