// Reverse-mode derivative (adjoint) of the QSA step, for gradients of the
// transverse magnetic energy of a sweep with respect to the beam's weights.
//
// The adjoint differentiates the discrete scheme itself: every deposit,
// gather, spectral solve, predictor-corrector iteration, plasma push, k = 0
// leapfrog and beam Boris push of the forward path (see qsa_kernels.h for
// the scheme), in reverse order.  Its forward passes run the same scheme
// with kernels of their own (one thread per particle, deposits accumulated
// per block in an LDS tile, batched full complex transforms) that keep the
// plasma particles in a fixed order, so that particle identities carry
// across slices; they store what the reverse pass needs:
//   * per beam step: the beam state and the 7 stored field planes;
//   * per sweep: the plasma state and J_perp of the previous slice every
//     QSA_ADJ_CKPT slices (checkpoints);
//   * per checkpoint segment, recomputed in the reverse pass: the plasma
//     state at every slice, its predictor states and the B_perp iterates.
// Conventions of the transposes used here:
//   * gather g = sum_n F_n W_n  <->  deposit of g_bar W_n into F_bar;
//     d g / d x = sum_n F_n dW_n/dx (W piecewise linear);
//   * a real spectral operator with multiplier M(k) (Hermitian) has the
//     transpose with multiplier conj(M(k)); a k = 0 value set from a scalar
//     has the transpose "sum of the adjoint over all nodes";
//   * index floors and the lost-particle flag are piecewise constant.
#pragma once

#include "qsa_kernels.h"

namespace qsa {

#define QSA_ADJ_CKPT 16   // default plasma checkpoint stride in slices (qsa_params.ckpt_every = 0)

// ---------------------------------------------------------------------------
// Grid helpers: linear combinations, per-launch side jobs, scalar jobs.
// ---------------------------------------------------------------------------
// out[k] = (out[k] when add) + c0 + spc * (*sp) + sum_t c_t in_t[k]
template <typename R>
struct Lin {
  R* out;
  int add;
  int nt;
  double c0;
  const double* sp;   // optional device scalar
  double spc;
  const R* in[3];
  double c[3];
};

template <typename R>
__device__ __forceinline__ void lin_range(const Lin<R>& a, int64_t i0, int64_t n, int64_t step) {
  const double base = a.c0 + (a.sp ? a.spc * *a.sp : 0.0);
  for (int64_t i = i0; i < n; i += step) {
    double s = (a.add ? (double)a.out[i] : 0.0) + base;
    for (int t = 0; t < a.nt; ++t) s += a.c[t] * (double)a.in[t][i];
    a.out[i] = (R)s;
  }
}

template <typename R>
__global__ void __launch_bounds__(256) k_lin(Lin<R> a, int64_t n) {
  lin_range(a, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, n, (int64_t)gridDim.x * blockDim.x);
}

// Scalar jobs (the first wavefront of a launch), for the transverse-mean
// leapfrog; part[0..npart) are per-block partial sums written by an earlier
// launch, added by the wavefront:
//  SJ_ODE_FWD:  slice slot a = [e, p, s, ez0] (e = <E_z>_{j-1/2}, p = psi0_j,
//               s = sum J_z = *c + sum part): e' = e - h s/N,
//               ez0 = (e + e')/2, and the next slot b = [e', p + h e'];
//               v0 = h, v1 = N
//  SJ_ODE_ADJ:  a = [e_bar', p_bar'] of slice j + 1 (p_bar' still without
//               the sum part of its psi adjoint), b = slot of slice j,
//               c = sum of the E_z adjoint over the slice (ez0_bar):
//               b = [e_bar, p_bar (before its own psi-mean part), uniform
//               J_z adjoint per node]
enum { SJ_NONE = 0, SJ_ODE_FWD, SJ_ODE_ADJ };
struct ScalarJob {
  int kind;
  int npart;
  double* a;
  double* b;
  const double* c;
  const double* part;
  double v0, v1;
};

// every lane of wavefront 0 of block 0 calls this
__device__ __forceinline__ void run_scalar(const ScalarJob& j) {
  const int lane = threadIdx.x & 63;
  double ps = 0.0;
  for (int i = lane; i < j.npart; i += 64) ps += j.part[i];
  for (int off = 32; off >= 1; off >>= 1) ps += __shfl_xor(ps, off);
  if (lane != 0) return;
  switch (j.kind) {
    case SJ_ODE_FWD: {
      const double e = j.a[0], p = j.a[1], s = *j.c + ps;
      const double en = e - j.v0 * s / j.v1;
      j.a[2] = s;
      j.a[3] = 0.5 * (e + en);
      j.b[0] = en;
      j.b[1] = p + j.v0 * en;
      break;
    }
    case SJ_ODE_ADJ: {
      const double ez = *j.c;
      const double pb = j.a[1] + ps;
      const double en = j.a[0] + 0.5 * ez + j.v0 * pb;
      j.b[0] = en + 0.5 * ez;
      j.b[1] = pb;
      j.b[2] = -j.v0 * en / j.v1;
      break;
    }
    default: break;
  }
}

// Work a launch does besides its own: up to SIDE_LIN grid combinations of
// len nodes and two scalar jobs, none of which may touch what the launch's
// main work reads or writes (they run concurrently with it).
constexpr int SIDE_LIN = 6;
template <typename R>
struct Side {
  int nl, ns;
  int64_t len;
  Lin<R> op[SIDE_LIN];
  ScalarJob sj[2];
};

template <typename R>
__device__ __forceinline__ void run_side(const Side<R>& s) {
  const int64_t tid = ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nth = (int64_t)gridDim.x * gridDim.y * blockDim.x;
  if (tid < 64)
    for (int q = 0; q < s.ns; ++q) run_scalar(s.sj[q]);
  for (int q = 0; q < s.nl; ++q) lin_range(s.op[q], tid, s.len, nth);
}

// out[j] = sum over the nodes of slice j of src ([nz][nperp]); one block per slice
template <typename R>
__global__ void __launch_bounds__(256) k_slice_sums(const R* __restrict__ src, int nperp, double* __restrict__ out) {
  __shared__ double red[4];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < nperp; i += blockDim.x) s += (double)src[(int64_t)j * nperp + i];
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
    out[j] = t;
  }
}

// dst += c * sum(src^2) (the energy).
template <typename R>
__global__ void __launch_bounds__(256) k_sumsq(const R* __restrict__ src, int64_t n, double c,
                                               double* __restrict__ dst) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double v = (double)src[i];
    s += v * v;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(dst, c * red[0]);
}

// ---------------------------------------------------------------------------
// Batched spectral operators on real [ny][nx] fields:
//   r_o = Re IFFT( sum_t c_t M_t(k) FFT(in_{i_t}) ),  k = 0 optionally set,
// with each input a combination of up to three grids and each result r_o
// written to up to three destinations (dst = dst (when added) + c r_o).
// Three launches: forward row transforms (the half spectrum kx <= nx/2 is
// kept, the inputs being real), column transforms with the multipliers (one
// wavefront per input and per output transform, concurrently), inverse row
// transforms (the other half by Hermitian symmetry).
// ---------------------------------------------------------------------------
enum {
  SK_ONE = 0,     // 1
  SK_INVK2,       // 1/|k|^2, 0 at k = 0
  SK_IKX,         // i kdx
  SK_IKY,         // i kdy
  SK_IKX_K2,      // i kdx/|k|^2
  SK_IKY_K2,      // i kdy/|k|^2
  SK_DEN,         // 1/(-|k|^2 - kappa^2)
  SK_IKX_DEN,     // i kdx/(-|k|^2 - kappa^2)
  SK_IKY_DEN      // i kdy/(-|k|^2 - kappa^2)
};
constexpr int SPEC_IN = 5, SPEC_OUT = 5, SPEC_TERMS = 4, SPEC_COMB = 3;

template <typename R>
struct SpecOp {
  int ni, no;
  int nin[SPEC_IN];
  const R* in[SPEC_IN][SPEC_COMB];
  double inc[SPEC_IN][SPEC_COMB];
  int nd[SPEC_OUT];
  R* dst[SPEC_OUT][SPEC_COMB];
  double dc[SPEC_OUT][SPEC_COMB];
  int dadd[SPEC_OUT][SPEC_COMB];
  int nterm[SPEC_OUT];
  int kind[SPEC_OUT][SPEC_TERMS];
  int src[SPEC_OUT][SPEC_TERMS];
  double coef[SPEC_OUT][SPEC_TERMS];
  const double* mean[SPEC_OUT];     // k = 0 value (the result's mean), or null
  double* insum;                    // [ny] per-row sums of input 0, or null
  int conj;                         // 1: the transpose (conjugate multipliers)
  const double* ktab;               // multiplier tables (k_spec_table)
  C2<R>* work;                      // [max(ni, no)][ny][nx] complex scratch
};

// Wavenumber and derivative multiplier of FFT index m on an axis of n cells
// of size d: m_s in [-n/2, n/2), derivative 0 on the Nyquist index.
__device__ __forceinline__ void axis_k(int m, int n, double L, double& k, double& kd) {
  const int ms = (m < (n + 1) / 2) ? m : m - n;
  k = 2.0 * 3.141592653589793238 * ms / L;
  kd = (n > 1 && (n & 1) == 0 && m == n / 2) ? 0.0 : k;
}

// Multiplier tables of the half spectrum, [kx <= nx/2][ky][4] =
// (1/|k|^2 (0 at k = 0), 1/(-|k|^2 - kappa^2), kdx, kdy); one block per kx.
template <typename R>
__global__ void __launch_bounds__(256) k_spec_table(Geo<R> g, double kappa2, double* __restrict__ tab) {
  const int kx = blockIdx.x;
  double kxv, kdx;
  axis_k(kx, g.nx, (double)g.nx * (double)g.dx, kxv, kdx);
  for (int ky = threadIdx.x; ky < g.ny; ky += blockDim.x) {
    double kyv, kdy;
    axis_k(ky, g.ny, (double)g.ny * (double)g.dy, kyv, kdy);
    const double k2 = kxv * kxv + kyv * kyv;
    double* t = tab + ((int64_t)kx * g.ny + ky) * 4;
    t[0] = (k2 == 0.0) ? 0.0 : 1.0 / k2;
    t[1] = 1.0 / (-k2 - kappa2);
    t[2] = kdx;
    t[3] = kdy;
  }
}

__device__ __forceinline__ void spec_mult(int kind, double c, const double (&t)[4], bool conj, double& re,
                                          double& im) {
  const double ik2 = t[0], den = t[1], kdx = t[2], kdy = t[3];
  re = 0.0;
  im = 0.0;
  switch (kind) {
    case SK_ONE: re = c; break;
    case SK_INVK2: re = c * ik2; break;
    case SK_IKX: im = c * kdx; break;
    case SK_IKY: im = c * kdy; break;
    case SK_IKX_K2: im = c * kdx * ik2; break;
    case SK_IKY_K2: im = c * kdy * ik2; break;
    case SK_DEN: re = c * den; break;
    case SK_IKX_DEN: im = c * kdx * den; break;
    case SK_IKY_DEN: im = c * kdy * den; break;
    default: break;
  }
  if (conj) im = -im;
}

// one block (one wavefront) per (row, input)
template <typename R>
__global__ void __launch_bounds__(64) k_spec_rows_fwd(Geo<R> g, SpecOp<R> op, const C2<R>* __restrict__ twx,
                                                      Side<R> side) {
  run_side(side);
  const int l = blockIdx.x, f = blockIdx.y;
  if (l >= g.ny || f >= op.ni) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C2<R>* tw = reinterpret_cast<C2<R>*>(smem_raw);
  C2<R>* A = tw + g.nx;
  C2<R>* B = A + fft_cap(g.nx);
  const int t = threadIdx.x, tpt = blockDim.x;
  double rs = 0.0;
  for (int i = t; i < g.nx; i += tpt) {
    tw[i] = twx[i];
    double v = 0.0;
    for (int q = 0; q < op.nin[f]; ++q) v += op.inc[f][q] * (double)op.in[f][q][(int64_t)l * g.nx + i];
    rs += v;
    A[i] = C2<R>{(R)v, R(0)};
  }
  if (op.insum && f == 0) {
    for (int off = 32; off >= 1; off >>= 1) rs += __shfl_xor(rs, off);
    if (t == 0) op.insum[l] = rs;
  }
  __syncthreads();
  const C2<R>* r = fft_lds<R, false>(A, B, g.nx, g.lgx, t, tpt, tw);
  C2<R>* w = op.work + (int64_t)f * g.nperp + (int64_t)l * g.nx;
  for (int i = t; i <= g.nx / 2; i += tpt) w[i] = r[i];
}

// one block per column kx <= nx/2, one wavefront per transform; LDS:
// twiddles, then two buffers of ny per wavefront
template <typename R>
__global__ void __launch_bounds__(64 * SPEC_IN) k_spec_cols(Geo<R> g, SpecOp<R> op, const C2<R>* __restrict__ twy,
                                                            Side<R> side) {
  run_side(side);
  const int kx = blockIdx.x;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C2<R>* tw = reinterpret_cast<C2<R>*>(smem_raw);
  const int w = threadIdx.x >> 6, t = threadIdx.x & 63;
  const int cs = fft_cap(g.ny);
  C2<R>* A = tw + g.ny + (int64_t)(2 * w) * cs;
  C2<R>* B = A + cs;
  for (int i = threadIdx.x; i < g.ny; i += blockDim.x) tw[i] = twy[i];
  for (int i = t; i < g.ny; i += 64)
    A[i] = (w < op.ni) ? op.work[(int64_t)w * g.nperp + (int64_t)i * g.nx + kx] : C2<R>{R(0), R(0)};
  __syncthreads();
  // forward column transforms: every wavefront's result sits in the same
  // buffer of its pair (same pass count)
  const C2<R>* r = fft_lds<R, false>(A, B, g.ny, g.lgy, t, 64, tw);
  const bool inA = (r == A);
  auto res = [&](int f) -> const C2<R>* { return tw + g.ny + (int64_t)(2 * f + (inA ? 0 : 1)) * cs; };
  C2<R>* S = inA ? B : A;   // free buffer of this wavefront
  const double N = (double)g.nperp;
  if (w < op.no) {
    for (int ky = t; ky < g.ny; ky += 64) {
      const double* tp = op.ktab + ((int64_t)kx * g.ny + ky) * 4;
      const double tk[4] = {tp[0], tp[1], tp[2], tp[3]};
      double ar = 0.0, ai = 0.0;
      for (int q = 0; q < op.nterm[w]; ++q) {
        double mr, mi;
        spec_mult(op.kind[w][q], op.coef[w][q], tk, op.conj != 0, mr, mi);
        const C2<R> v = res(op.src[w][q])[ky];
        ar += mr * (double)v.x - mi * (double)v.y;
        ai += mr * (double)v.y + mi * (double)v.x;
      }
      if (kx == 0 && ky == 0 && op.mean[w]) {
        ar = *op.mean[w] * N;
        ai = 0.0;
      }
      S[ky] = C2<R>{(R)ar, (R)ai};
    }
  }
  __syncthreads();
  C2<R>* other = const_cast<C2<R>*>(res(w));
  const C2<R>* q = fft_lds<R, true>(S, other, g.ny, g.lgy, t, 64, tw);
  if (w < op.no)
    for (int i = t; i < g.ny; i += 64) op.work[(int64_t)w * g.nperp + (int64_t)i * g.nx + kx] = q[i];
}

// one block (one wavefront) per (row, output)
template <typename R>
__global__ void __launch_bounds__(64) k_spec_rows_inv(Geo<R> g, SpecOp<R> op, const C2<R>* __restrict__ twx,
                                                      Side<R> side) {
  run_side(side);
  const int l = blockIdx.x, o = blockIdx.y;
  if (l >= g.ny || o >= op.no) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C2<R>* tw = reinterpret_cast<C2<R>*>(smem_raw);
  C2<R>* A = tw + g.nx;
  C2<R>* B = A + fft_cap(g.nx);
  const int t = threadIdx.x, tpt = blockDim.x;
  const C2<R>* w = op.work + (int64_t)o * g.nperp + (int64_t)l * g.nx;
  const int h = g.nx / 2;
  for (int i = t; i < g.nx; i += tpt) {
    tw[i] = twx[i];
    if (i <= h) {
      A[i] = w[i];
    } else {
      const C2<R> v = w[g.nx - i];
      A[i] = C2<R>{v.x, -v.y};
    }
  }
  __syncthreads();
  const C2<R>* r = fft_lds<R, true>(A, B, g.nx, g.lgx, t, tpt, tw);
  const double s = 1.0 / (double)g.nperp;
  for (int d = 0; d < op.nd[o]; ++d) {
    R* out = op.dst[o][d] + (int64_t)l * g.nx;
    const double c = op.dc[o][d] * s;
    if (op.dadd[o][d])
      for (int i = t; i < g.nx; i += tpt) out[i] = (R)((double)out[i] + c * (double)r[i].x);
    else
      for (int i = t; i < g.nx; i += tpt) out[i] = (R)(c * (double)r[i].x);
  }
}

// ---------------------------------------------------------------------------
// Plasma: gathers with their transverse gradients, forward right-hand side
// and its transpose.
// ---------------------------------------------------------------------------
template <typename R>
struct Cic {
  int n00, n10, n01, n11;
  int i0, l0;          // lower cell
  double fx, fy;
};

template <typename R>
__device__ __forceinline__ Cic<R> cic(const Geo<R>& g, R x, R y) {
  Cic<R> c;
  int i0, l0;
  R fx, fy;
  cell2(g, x, y, i0, l0, fx, fy);
  const int i1 = (i0 + 1 == g.nx) ? 0 : i0 + 1;
  const int l1 = (l0 + 1 == g.ny) ? 0 : l0 + 1;
  c.n00 = l0 * g.nx + i0;
  c.n10 = l0 * g.nx + i1;
  c.n01 = l1 * g.nx + i0;
  c.n11 = l1 * g.nx + i1;
  c.i0 = i0;
  c.l0 = l0;
  c.fx = (double)fx;
  c.fy = (double)fy;
  return c;
}

// value, d/dx, d/dy of the linear interpolant of F
template <typename R>
__device__ __forceinline__ void cic_val(const Geo<R>& g, const R* __restrict__ F, const Cic<R>& c, double& v,
                                        double& dx, double& dy) {
  const double f00 = F[c.n00], f10 = F[c.n10], f01 = F[c.n01], f11 = F[c.n11];
  v = f00 * (1 - c.fx) * (1 - c.fy) + f10 * c.fx * (1 - c.fy) + f01 * (1 - c.fx) * c.fy + f11 * c.fx * c.fy;
  dx = ((f10 - f00) * (1 - c.fy) + (f11 - f01) * c.fy) / (double)g.dx;
  dy = ((f01 - f00) * (1 - c.fx) + (f11 - f10) * c.fx) / (double)g.dy;
}

template <typename R>
__device__ __forceinline__ void cic_add(R* __restrict__ F, const Cic<R>& c, double q) {
  if (q == 0.0) return;
  atomic_add(F + c.n00, (R)(q * (1 - c.fx) * (1 - c.fy)));
  atomic_add(F + c.n10, (R)(q * c.fx * (1 - c.fy)));
  atomic_add(F + c.n01, (R)(q * (1 - c.fx) * c.fy));
  atomic_add(F + c.n11, (R)(q * c.fx * c.fy));
}

// ---------------------------------------------------------------------------
// Block-local scatter accumulation.  Tile kernels number their particle
// chunks with xcd_block, so that neighbouring chunks (which flush to shared
// nodes) run on one XCD.  The particles of a block (consecutive
// in memory, hence close in space while the order of loading by cell holds)
// reduce the bounding box of the cells they scatter at.  When the box's
// nodes fit the LDS tile, the linear-shape weights accumulate there with LDS
// atomics and the block then adds every touched node to the grid with one
// global atomic per channel; otherwise each particle adds its nodes to the
// grid directly.  Same-address atomics of neighbouring particles, which
// serialize at the L2, are thereby merged.  Every thread of the block calls
// box_reduce, tile_zero and tile_flush (they hold barriers).  NZ = 1 for
// transverse grids [ny][nx] (cell slice 0), 2 for [nxi][ny][nx] grids.
// ---------------------------------------------------------------------------
struct BoxAcc {
  int lo[3], hi[3];    // cell (j, l, i) range of one thread
};
__device__ __forceinline__ void box_init(BoxAcc& b) {
  for (int d = 0; d < 3; ++d) {
    b.lo[d] = INT_MAX;
    b.hi[d] = INT_MIN;
  }
}
__device__ __forceinline__ void box_add(BoxAcc& b, int j, int l, int i) {
  b.lo[0] = min(b.lo[0], j);
  b.lo[1] = min(b.lo[1], l);
  b.lo[2] = min(b.lo[2], i);
  b.hi[0] = max(b.hi[0], j);
  b.hi[1] = max(b.hi[1], l);
  b.hi[2] = max(b.hi[2], i);
}

struct TileBox {
  int j0, l0, i0;      // lowest node
  int nl, ni, nodes;   // node extents (nodes = 0 unless fits)
  bool fits;
};

// red: LDS scratch of 6 ints per wavefront of the block
template <int NZ>
__device__ __forceinline__ TileBox box_reduce(BoxAcc b, int* red, int cap) {
  for (int off = 32; off >= 1; off >>= 1)
    for (int d = 0; d < 3; ++d) {
      b.lo[d] = min(b.lo[d], __shfl_xor(b.lo[d], off));
      b.hi[d] = max(b.hi[d], __shfl_xor(b.hi[d], off));
    }
  const int wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int d = 0; d < 3; ++d) {
      red[wave * 6 + d] = b.lo[d];
      red[wave * 6 + 3 + d] = b.hi[d];
    }
  __syncthreads();
  BoxAcc t;
  box_init(t);
  for (int w = 0; w < nw; ++w)
    for (int d = 0; d < 3; ++d) {
      t.lo[d] = min(t.lo[d], red[w * 6 + d]);
      t.hi[d] = max(t.hi[d], red[w * 6 + 3 + d]);
    }
  TileBox x;
  const bool any = t.hi[2] >= t.lo[2];
  x.j0 = t.lo[0];
  x.l0 = t.lo[1];
  x.i0 = t.lo[2];
  const long long nj = any ? (long long)t.hi[0] - t.lo[0] + NZ : 0;
  x.nl = any ? t.hi[1] - t.lo[1] + 2 : 0;
  x.ni = any ? t.hi[2] - t.lo[2] + 2 : 0;
  const long long nodes = nj * x.nl * x.ni;
  x.fits = any && nodes <= cap;
  x.nodes = x.fits ? (int)nodes : 0;
  return x;
}

template <typename T>
__device__ __forceinline__ void tile_zero(T* tile, const TileBox& b, int nch) {
  for (int t = threadIdx.x; t < nch * b.nodes; t += blockDim.x) tile[t] = T(0);
  __syncthreads();
}

// Lane-group merge.  Particles that share a cell sit on neighbouring lanes
// (4 plasma particles per cell in loading order, 8 beam particles per cell
// after sorting).  When an aligned group of G lanes (G = 4 or 8) scatters
// at one cell, the group sums its node weights with DPP lane moves and only
// its first lane adds them to the tile: a quarter (an eighth) of the LDS
// atomics, and none from several lanes to one address.  Every lane of the
// wavefront calls merge_of and the tile adds (converged code); a lane with
// nothing to add passes act = false, and its group adds lane by lane.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp_r(float v) {
  return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_r(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_i<CTRL>((int)(b & 0xffffffffll));
  const int hi = dpp_i<CTRL>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
constexpr int DPP_XOR1 = 0xB1;          // quad_perm [1, 0, 3, 2]
constexpr int DPP_XOR2 = 0x4E;          // quad_perm [2, 3, 0, 1]
constexpr int DPP_HALF_MIRROR = 0x141;  // lane i <-> 7 - i within 8 lanes

template <int G>
__device__ __forceinline__ void group_minmax(int& mn, int& mx) {
  mn = min(mn, dpp_i<DPP_XOR1>(mn));
  mx = max(mx, dpp_i<DPP_XOR1>(mx));
  mn = min(mn, dpp_i<DPP_XOR2>(mn));
  mx = max(mx, dpp_i<DPP_XOR2>(mx));
  if (G == 8) {
    mn = min(mn, dpp_i<DPP_HALF_MIRROR>(mn));
    mx = max(mx, dpp_i<DPP_HALF_MIRROR>(mx));
  }
}
template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
  v += dpp_r<DPP_XOR1>(v);
  v += dpp_r<DPP_XOR2>(v);
  if (G == 8) v += dpp_r<DPP_HALF_MIRROR>(v);
  return v;
}

struct Merge {
  bool uni;    // the lane's group shares one cell
  bool lead;   // first lane of its group
  bool act;    // the lane adds something at this position
};

// keys: the cell (two non-negative parts) when act
template <int G>
__device__ __forceinline__ Merge merge_of(bool act, int key0, int key1 = 0) {
  const int lane = threadIdx.x & 63;
  int a0 = act ? key0 : -1 - lane, b0 = a0;
  int a1 = act ? key1 : 0, b1 = a1;
  group_minmax<G>(a0, b0);
  group_minmax<G>(a1, b1);
  Merge m;
  m.uni = (a0 == b0) && (a1 == b1);
  m.lead = (lane & (G - 1)) == 0;
  m.act = act;
  return m;
}

template <int G, typename R>
__device__ __forceinline__ Merge merge_at(bool act, const Cic<R>& c, int nx) {
  return merge_of<G>(act, c.l0 * nx + c.i0);
}

// q times the linear shape at c into channel ch (transverse grid glob when
// the box did not fit)
template <int G, typename R, typename T>
__device__ __forceinline__ void tile_add(T* tile, const TileBox& b, int ch, const Cic<R>& c, double q, R* glob,
                                         const Merge& m) {
  if (!b.fits) {   // uniform over the block
    if (m.act && q != 0.0) cic_add(glob, c, q);
    return;
  }
  T w[4] = {T(0), T(0), T(0), T(0)};
  if (m.act) {
    w[0] = (T)(q * (1 - c.fx) * (1 - c.fy));
    w[1] = (T)(q * c.fx * (1 - c.fy));
    w[2] = (T)(q * (1 - c.fx) * c.fy);
    w[3] = (T)(q * c.fx * c.fy);
  }
  if (m.uni) {
#pragma unroll
    for (int n = 0; n < 4; ++n) w[n] = group_sum<G>(w[n]);
    if (!m.lead) return;
  } else if (!m.act || q == 0.0) {
    return;
  }
  T* t = tile + ch * b.nodes + (c.l0 - b.l0) * b.ni + (c.i0 - b.i0);
  atomicAdd(t, w[0]);
  atomicAdd(t + 1, w[1]);
  atomicAdd(t + b.ni, w[2]);
  atomicAdd(t + b.ni + 1, w[3]);
}

// the touched tile nodes into the grids dst[ch] ([nz][ny][nx], nz = 1 for
// a transverse grid); node slices outside [0, nz) are dropped
template <typename R, int NCH, typename T>
__device__ __forceinline__ void tile_flush(const Geo<R>& g, const T* tile, const TileBox& b, R* const* dst, int nz) {
  __syncthreads();
  const int nli = b.nl * b.ni;
  for (int t = threadIdx.x; t < b.nodes; t += blockDim.x) {
    const int jj = t / nli, r = t - jj * nli;
    const int ll = r / b.ni, ii = r - ll * b.ni;
    const int j = b.j0 + jj;
    if (j < 0 || j >= nz) continue;
    int l = b.l0 + ll;
    l -= (l >= g.ny) ? g.ny : 0;
    int i = b.i0 + ii;
    i -= (i >= g.nx) ? g.nx : 0;
    const int64_t off = (int64_t)j * g.nperp + (int64_t)l * g.nx + i;
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
      const T v = tile[ch * b.nodes + t];
      if (v != T(0)) atomic_add(dst[ch] + off, (R)v);
    }
  }
}

// The six fields a plasma particle sees, F = (psi, dxpsi, dypsi, Bx, By, Bz),
// at slice j (Fa) and the extrapolation (3 Fa - Fm1)/2 (when half is set).
template <typename R>
struct Six {
  const R* a[6];
  const R* m1[6];
};

template <typename R>
__device__ __forceinline__ void six_val(const Geo<R>& g, const Six<R>& F, bool half, const Cic<R>& c,
                                        double (&v)[6], double (&vx)[6], double (&vy)[6]) {
  for (int m = 0; m < 6; ++m) {
    double a, ax, ay;
    cic_val(g, F.a[m], c, a, ax, ay);
    if (half) {
      double b, bx, by;
      cic_val(g, F.m1[m], c, b, bx, by);
      a = 0.5 * (3.0 * a - b);
      ax = 0.5 * (3.0 * ax - bx);
      ay = 0.5 * (3.0 * ay - by);
    }
    v[m] = a;
    vx[m] = ax;
    vy[m] = ay;
  }
}

// Grid adjoints of the six fields: at slice j (a) and j - 1 (m1, the
// extrapolation (3 Fa - Fm1)/2 reads it).
template <typename R>
struct SixBar {
  R* a[6];
  R* m1[6];
};

// d(x, y, ux, uy)/dxi from the gathered six fields
__device__ __forceinline__ void rhs_val(const double (&v)[6], double ux, double uy, double (&f)[4]) {
  const double G = 1.0 + v[0];
  const double gam = (1.0 + ux * ux + uy * uy + G * G) / (2.0 * G);
  f[0] = ux / G;
  f[1] = uy / G;
  f[2] = gam * v[1] / G - v[4] - uy * v[5] / G;
  f[3] = gam * v[2] / G + v[3] + ux * v[5] / G;
}

// Transpose of rhs_val at (v, ux, uy): from f_bar, the adjoints of the six
// gathered values and of ux, uy.
__device__ __forceinline__ void rhs_adj(const double (&v)[6], double ux, double uy, const double (&fb)[4],
                                        double (&gb)[6], double& uxb, double& uyb) {
  const double G = 1.0 + v[0];
  const double u2 = ux * ux + uy * uy;
  const double gam = (1.0 + u2 + G * G) / (2.0 * G);
  const double A = gam / G;
  const double A_ux = ux / (G * G), A_uy = uy / (G * G);
  const double gam_G = 0.5 - (1.0 + u2) / (2.0 * G * G);
  const double A_G = gam_G / G - gam / (G * G);
  const double dxp = v[1], dyp = v[2], bz = v[5];
  uxb = fb[0] / G + fb[2] * A_ux * dxp + fb[3] * (A_ux * dyp + bz / G);
  uyb = fb[1] / G + fb[2] * (A_uy * dxp - bz / G) + fb[3] * A_uy * dyp;
  const double Gb = -fb[0] * ux / (G * G) - fb[1] * uy / (G * G) + fb[2] * (A_G * dxp + uy * bz / (G * G)) +
                    fb[3] * (A_G * dyp - ux * bz / (G * G));
  gb[0] = Gb;
  gb[1] = fb[2] * A;
  gb[2] = fb[3] * A;
  gb[3] = fb[3];
  gb[4] = -fb[2];
  gb[5] = -fb[2] * uy / G + fb[3] * ux / G;
}

// One RK2 (midpoint) step in double: Y' = Y + h f(Y + h/2 f(Y; Fj); Fh).
template <typename R>
__device__ __forceinline__ void rk2_val(const Geo<R>& g, const Six<R>& F, double h, const double (&Y)[4],
                                        double (&Ys)[4], double (&Yn)[4]) {
  double v[6], vx[6], vy[6], f[4];
  six_val(g, F, false, cic(g, (R)Y[0], (R)Y[1]), v, vx, vy);
  rhs_val(v, Y[2], Y[3], f);
  for (int c = 0; c < 4; ++c) Ys[c] = Y[c] + 0.5 * h * f[c];
  six_val(g, F, true, cic(g, (R)Ys[0], (R)Ys[1]), v, vx, vy);
  rhs_val(v, Ys[2], Ys[3], f);
  for (int c = 0; c < 4; ++c) Yn[c] = Y[c] + h * f[c];
}

// Transpose of rk2_val: Yb (adjoint of Y') adds to the adjoint of Y; the
// adjoints of the six values gathered at stage 1 (at Y, fields of slice j)
// and stage 2 (at Ys, extrapolated fields) with their stencils go to o.
template <typename R>
struct Rk2Bar {
  Cic<R> c0, c1;
  double g0[6], g1[6];
};

template <typename R>
__device__ __forceinline__ void rk2_adj(const Geo<R>& g, const Six<R>& F, double h, const double (&Y)[4],
                                        const double (&Ynb)[4], double (&Yb)[4], Rk2Bar<R>& o) {
  double v[6], vx[6], vy[6], f[4], Ys[4];
  o.c0 = cic(g, (R)Y[0], (R)Y[1]);
  six_val(g, F, false, o.c0, v, vx, vy);
  rhs_val(v, Y[2], Y[3], f);
  for (int c = 0; c < 4; ++c) Ys[c] = Y[c] + 0.5 * h * f[c];
  // stage 2 at Ys with Fh
  double v2[6], vx2[6], vy2[6];
  o.c1 = cic(g, (R)Ys[0], (R)Ys[1]);
  six_val(g, F, true, o.c1, v2, vx2, vy2);
  double fb[4], uxb, uyb;
  for (int c = 0; c < 4; ++c) {
    Yb[c] += Ynb[c];
    fb[c] = h * Ynb[c];
  }
  rhs_adj(v2, Ys[2], Ys[3], fb, o.g1, uxb, uyb);
  double Ysb[4] = {0, 0, uxb, uyb};
  for (int m = 0; m < 6; ++m) {
    Ysb[0] += o.g1[m] * vx2[m];
    Ysb[1] += o.g1[m] * vy2[m];
  }
  // stage 1 at Y with Fj
  for (int c = 0; c < 4; ++c) {
    Yb[c] += Ysb[c];
    fb[c] = 0.5 * h * Ysb[c];
  }
  rhs_adj(v, Y[2], Y[3], fb, o.g0, uxb, uyb);
  Yb[2] += uxb;
  Yb[3] += uyb;
  for (int m = 0; m < 6; ++m) {
    Yb[0] += o.g0[m] * vx[m];
    Yb[1] += o.g0[m] * vy[m];
  }
}

// channels 0..5: fields of slice j (stage 1, and 3/2 of stage 2); 6..11:
// fields of slice j - 1 (-1/2 of stage 2)
template <typename R>
__device__ __forceinline__ void rk2_bar_add(double* tile, const TileBox& b, const Rk2Bar<R>& o, const SixBar<R>& Fb,
                                            const Merge& m0, const Merge& m1) {
  for (int m = 0; m < 6; ++m) {
    tile_add<4>(tile, b, m, o.c0, o.g0[m], Fb.a[m], m0);
    tile_add<4>(tile, b, m, o.c1, 1.5 * o.g1[m], Fb.a[m], m1);
    tile_add<4>(tile, b, 6 + m, o.c1, -0.5 * o.g1[m], Fb.m1[m], m1);
  }
}

template <typename R>
struct AdjPlasma {
  Geo<R> g;
  int np;
  double nw;           // -w/(dx dy): rho - J_z of one plasma particle per unit area
  double h;
  const R* Y[4];       // state at slice j
  R* Yn[4];            // forward: state out; reverse: adjoint out
  const R* Yt[4];      // predictor state (stored)
  const R* Ynb[4];     // adjoint of the state after the push
  Six<R> F;            // fields of the push
  SixBar<R> Fb;        // their adjoints
  const R* psi;        // psi (J stage) or the extrapolated psi (predictor)
  R* psib;             // its adjoint
  R* Jx;               // deposits (forward) / their adjoints (reverse)
  R* Jy;
  R* Jz;
  double jscale;       // reverse: scale of the current adjoints (1/(2h) for D)
  const R* Sb;         // reverse: adjoint of S
  double* qzsum;       // forward J stage: per-block sums of the J_z deposits
  const double* jzs;   // reverse J stage: uniform part of the J_z adjoint
  int tile_bytes;      // dynamic LDS of the launch (scatter tile)
  int* err;
};

// LDS of a tile kernel (dynamic, tile_bytes of the launch): 512 bytes of
// scratch (box reduction: 6 ints per wavefront from byte 0; per-wavefront
// doubles from byte 384), then NCH channels of CAP_ nodes of type T.  The
// plasma transposes accumulate in float64 for either precision (LDS float32
// atomic adds are slower per instruction on this part); the beam kernels'
// 3D tiles measured faster in the working precision.
#define ADJ_TILE(NCH, BYTES, T)                                           \
  constexpr int NCH_ = (NCH);                                             \
  using T_ = T;                                                           \
  extern __shared__ __align__(16) unsigned char smem_raw[];               \
  int* red = reinterpret_cast<int*>(smem_raw);                            \
  T_* tile = reinterpret_cast<T_*>(smem_raw + 512);                       \
  const int CAP_ = ((int)(BYTES) - 512) / (NCH_ * (int)sizeof(T_));       \
  BoxAcc bx;                                                              \
  box_init(bx)

// S += -w W/(dx dy)
template <typename R>
__global__ void __launch_bounds__(256) k_af_dep_s(AdjPlasma<R> a, R* __restrict__ S, Side<R> side) {
  run_side(side);
  ADJ_TILE(1, a.tile_bytes, double);
  const int p = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const bool live = p < a.np;
  Cic<R> c{};
  if (live) {
    c = cic(a.g, a.Y[0][p], a.Y[1][p]);
    box_add(bx, 0, c.l0, c.i0);
  }
  const TileBox b = box_reduce<1>(bx, red, CAP_);
  tile_zero(tile, b, NCH_);
  const Merge m = merge_at<4>(live, c, a.g.nx);
  tile_add<4>(tile, b, 0, c, a.nw, S, m);
  R* const dst[1] = {S};
  tile_flush<R, 1>(a.g, tile, b, dst, 1);
}

// J stage: G = 1 + psi(Y); J += -w u/G W/(dx dy)
template <typename R>
__global__ void __launch_bounds__(256) k_af_dep_j(AdjPlasma<R> a, Side<R> side) {
  run_side(side);
  ADJ_TILE(3, a.tile_bytes, double);
  double* wsum = reinterpret_cast<double*>(smem_raw + 384);   // per-wavefront J_z sums
  const int p = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const bool live = p < a.np;
  Cic<R> c{};
  double q[3] = {0, 0, 0};
  if (live) {
    c = cic(a.g, a.Y[0][p], a.Y[1][p]);
    box_add(bx, 0, c.l0, c.i0);
    double ps, px, py;
    cic_val(a.g, a.psi, c, ps, px, py);
    const double G = 1.0 + ps;
    if (!(G > QSA_GMIN)) atomicOr(a.err, ERR_BREAKDOWN);
    const double ux = a.Y[2][p], uy = a.Y[3][p];
    const double gam = (1.0 + ux * ux + uy * uy + G * G) / (2.0 * G);
    q[0] = a.nw * ux / G;
    q[1] = a.nw * uy / G;
    q[2] = a.nw * (gam - G) / G;
  }
  {
    double qz = q[2];
    for (int off = 32; off >= 1; off >>= 1) qz += __shfl_xor(qz, off);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = qz;
  }
  const TileBox b = box_reduce<1>(bx, red, CAP_);   // its barrier publishes wsum
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += wsum[w];
    a.qzsum[blockIdx.x] = t;
  }
  tile_zero(tile, b, NCH_);
  R* const dst[3] = {a.Jx, a.Jy, a.Jz};
  const Merge m = merge_at<4>(live, c, a.g.nx);
  for (int k = 0; k < 3; ++k) tile_add<4>(tile, b, k, c, q[k], dst[k], m);
  tile_flush<R, 3>(a.g, tile, b, dst, 1);
}

// Predictor: Yt = RK2(Y; F); Jt_perp += -w ut/Gt with Gt = 1 + psit(Yt)
template <typename R>
__global__ void __launch_bounds__(256) k_af_pred(AdjPlasma<R> a, Side<R> side) {
  run_side(side);
  ADJ_TILE(2, a.tile_bytes, double);
  const int p = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const bool live = p < a.np;
  Cic<R> c{};
  double q[2] = {0, 0};
  if (live) {
    const double Y[4] = {a.Y[0][p], a.Y[1][p], a.Y[2][p], a.Y[3][p]};
    double Ys[4], Yt[4];
    rk2_val(a.g, a.F, a.h, Y, Ys, Yt);
    c = cic(a.g, (R)Yt[0], (R)Yt[1]);
    box_add(bx, 0, c.l0, c.i0);
    double ps, px, py;
    cic_val(a.g, a.psi, c, ps, px, py);
    const double G = 1.0 + ps;
    if (!(G > QSA_GMIN)) atomicOr(a.err, ERR_BREAKDOWN);
    q[0] = a.nw * Yt[2] / G;
    q[1] = a.nw * Yt[3] / G;
  }
  const TileBox b = box_reduce<1>(bx, red, CAP_);
  tile_zero(tile, b, NCH_);
  R* const dst[2] = {a.Jx, a.Jy};
  const Merge m = merge_at<4>(live, c, a.g.nx);
  for (int k = 0; k < 2; ++k) tile_add<4>(tile, b, k, c, q[k], dst[k], m);
  tile_flush<R, 2>(a.g, tile, b, dst, 1);
}

// Final advance: Yn = wrap(RK2(Y; F))
template <typename R>
__global__ void __launch_bounds__(256) k_af_final(AdjPlasma<R> a, Side<R> side) {
  run_side(side);
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.np) return;
  const double Y[4] = {a.Y[0][p], a.Y[1][p], a.Y[2][p], a.Y[3][p]};
  double Ys[4], Yn[4];
  rk2_val(a.g, a.F, a.h, Y, Ys, Yn);
  a.Yn[0][p] = wrap_pos((R)Yn[0], a.g.lx, a.g.inv_lx);
  a.Yn[1][p] = wrap_pos((R)Yn[1], a.g.ly, a.g.inv_ly);
  a.Yn[2][p] = (R)Yn[2];
  a.Yn[3][p] = (R)Yn[3];
}

template <typename R>
__device__ __forceinline__ void six_bar_dst(const SixBar<R>& Fb, R** dst) {
  for (int m = 0; m < 6; ++m) {
    dst[m] = Fb.a[m];
    dst[6 + m] = Fb.m1[m];
  }
}

// Reverse of the final advance: Yn (adjoint of Y) = RK2^T(Ynb); fields.
template <typename R>
__global__ void __launch_bounds__(256) k_ar_final(AdjPlasma<R> a, Side<R> side) {
  run_side(side);
  ADJ_TILE(12, a.tile_bytes, double);
  const int p = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const bool live = p < a.np;
  Rk2Bar<R> o{};
  if (live) {
    const double Y[4] = {a.Y[0][p], a.Y[1][p], a.Y[2][p], a.Y[3][p]};
    const double Ynb[4] = {a.Ynb[0][p], a.Ynb[1][p], a.Ynb[2][p], a.Ynb[3][p]};
    double Yb[4] = {0, 0, 0, 0};
    rk2_adj(a.g, a.F, a.h, Y, Ynb, Yb, o);
    for (int c = 0; c < 4; ++c) a.Yn[c][p] = (R)Yb[c];
    box_add(bx, 0, o.c0.l0, o.c0.i0);
    box_add(bx, 0, o.c1.l0, o.c1.i0);
  }
  const TileBox b = box_reduce<1>(bx, red, CAP_);
  tile_zero(tile, b, NCH_);
  rk2_bar_add(tile, b, o, a.Fb, merge_at<4>(live, o.c0, a.g.nx), merge_at<4>(live, o.c1, a.g.nx));
  R* dst[12];
  six_bar_dst(a.Fb, dst);
  tile_flush<R, 12>(a.g, tile, b, dst, 1);
}

// Reverse of predictor iteration: the adjoint of Jt_perp (jscale * (Jx, Jy))
// -> adjoint of Yt and of psit -> RK2^T into the adjoint of Y (added).
template <typename R>
__global__ void __launch_bounds__(256) k_ar_pred(AdjPlasma<R> a, Side<R> side) {
  run_side(side);
  ADJ_TILE(13, a.tile_bytes, double);
  const int p = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const bool live = p < a.np;
  const Geo<R>& g = a.g;
  Rk2Bar<R> o{};
  Cic<R> c{};
  double Gb = 0.0;
  if (live) {
    const double Yt[4] = {a.Yt[0][p], a.Yt[1][p], a.Yt[2][p], a.Yt[3][p]};
    c = cic(g, (R)Yt[0], (R)Yt[1]);
    double ps, psx, psy;
    cic_val(g, a.psi, c, ps, psx, psy);
    const double G = 1.0 + ps;
    double jx, jxx, jxy, jy, jyx, jyy;
    cic_val(g, a.Jx, c, jx, jxx, jxy);
    cic_val(g, a.Jy, c, jy, jyx, jyy);
    // nw (hence q) already holds the 1/(dx dy) of the deposit
    const double s = a.jscale;
    const double qx = a.nw * Yt[2] / G, qy = a.nw * Yt[3] / G;
    // q_bar (deposit transpose) and position terms of the deposit
    const double qxb = s * jx, qyb = s * jy;
    double Ytb[4];
    Ytb[0] = s * (qx * jxx + qy * jyx);
    Ytb[1] = s * (qx * jxy + qy * jyy);
    Ytb[2] = qxb * a.nw / G;
    Ytb[3] = qyb * a.nw / G;
    Gb = -(qxb * qx + qyb * qy) / G;
    Ytb[0] += Gb * psx;
    Ytb[1] += Gb * psy;
    const double Y[4] = {a.Y[0][p], a.Y[1][p], a.Y[2][p], a.Y[3][p]};
    double Yb[4] = {a.Yn[0][p], a.Yn[1][p], a.Yn[2][p], a.Yn[3][p]};
    rk2_adj(g, a.F, a.h, Y, Ytb, Yb, o);
    for (int k = 0; k < 4; ++k) a.Yn[k][p] = (R)Yb[k];
    box_add(bx, 0, c.l0, c.i0);
    box_add(bx, 0, o.c0.l0, o.c0.i0);
    box_add(bx, 0, o.c1.l0, o.c1.i0);
  }
  const TileBox b = box_reduce<1>(bx, red, CAP_);
  tile_zero(tile, b, NCH_);
  rk2_bar_add(tile, b, o, a.Fb, merge_at<4>(live, o.c0, g.nx), merge_at<4>(live, o.c1, g.nx));
  tile_add<4>(tile, b, 12, c, Gb, a.psib, merge_at<4>(live, c, g.nx));
  R* dst[13];
  six_bar_dst(a.Fb, dst);
  dst[12] = a.psib;
  tile_flush<R, 13>(g, tile, b, dst, 1);
}

// Reverse of the J stage (deposits of -w u/G with G = 1 + psi(Y); when Jx is
// set) or of the rho - J_z deposit of -w (adjoint Sb; when Sb is set): adds
// to the adjoint of Y and, for the J stage, of psi.  The two run as separate
// launches: the adjoint of S needs the psi adjoint the J stage completes.
template <typename R>
__global__ void __launch_bounds__(256) k_ar_jstage(AdjPlasma<R> a, Side<R> side) {
  run_side(side);
  ADJ_TILE(1, a.tile_bytes, double);
  const int p = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const bool live = p < a.np;
  const Geo<R>& g = a.g;
  Cic<R> c{};
  double Gb = 0.0;
  if (live) {
    c = cic(g, a.Y[0][p], a.Y[1][p]);
    double xb = 0.0, yb = 0.0, uxb = 0.0, uyb = 0.0;   // nw holds the 1/(dx dy) of the deposits
    if (a.Jx) {
      const double ux = a.Y[2][p], uy = a.Y[3][p];
      double ps, psx, psy;
      cic_val(g, a.psi, c, ps, psx, psy);
      const double G = 1.0 + ps;
      const double u2 = ux * ux + uy * uy;
      double jx, jxx, jxy, jy, jyx, jyy, jz, jzx, jzy;
      cic_val(g, a.Jx, c, jx, jxx, jxy);
      cic_val(g, a.Jy, c, jy, jyx, jyy);
      cic_val(g, a.Jz, c, jz, jzx, jzy);
      const double qx = a.nw * ux / G, qy = a.nw * uy / G;
      const double qz = a.nw * ((1.0 + u2 + G * G) / (2.0 * G * G) - 1.0);
      const double qxb = jx, qyb = jy, qzb = jz + (a.jzs ? *a.jzs : 0.0);
      xb = qx * jxx + qy * jyx + qz * jzx;
      yb = qx * jxy + qy * jyy + qz * jzy;
      uxb = a.nw * (qxb / G + qzb * ux / (G * G));
      uyb = a.nw * (qyb / G + qzb * uy / (G * G));
      Gb = a.nw * (-qxb * ux / (G * G) - qyb * uy / (G * G) - qzb * (1.0 + u2) / (G * G * G));
      xb += Gb * psx;
      yb += Gb * psy;
      box_add(bx, 0, c.l0, c.i0);
    }
    if (a.Sb) {
      double sv, sx, sy;
      cic_val(g, a.Sb, c, sv, sx, sy);
      xb += a.nw * sx;
      yb += a.nw * sy;
    }
    a.Yn[0][p] = (R)((double)a.Yn[0][p] + xb);
    a.Yn[1][p] = (R)((double)a.Yn[1][p] + yb);
    a.Yn[2][p] = (R)((double)a.Yn[2][p] + uxb);
    a.Yn[3][p] = (R)((double)a.Yn[3][p] + uyb);
  }
  if (!a.Jx) return;   // uniform over the launch
  const TileBox b = box_reduce<1>(bx, red, CAP_);
  tile_zero(tile, b, NCH_);
  tile_add<4>(tile, b, 0, c, Gb, a.psib, merge_at<4>(live, c, g.nx));
  R* const dst[1] = {a.psib};
  tile_flush<R, 1>(g, tile, b, dst, 1);
}

// Recompute of a checkpoint segment: each thread takes its plasma particle
// from the checkpointed state through slices j0 .. j0 + len - 1 with the
// taped fields and B_perp iterates (the predictor states need no deposit),
// storing the state at every slice and the K predictor states.
template <typename R>
struct AdjSeg {
  Geo<R> g;
  int np, K, j0, len;
  double h;
  const R* Y0[4];       // checkpoint (state at j0)
  R* segY;              // [len][4][np]
  R* segYt;             // [len][K][4][np]
  const R* fields;      // [N_STORED][nxi][ny][nx] of the sweep
  const R* biter;       // [K][2][nxi][ny][nx]
  const R* zero;
};

template <typename R>
__global__ void __launch_bounds__(256) k_af_segment(AdjSeg<R> a) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.np) return;
  const int64_t nperp = a.g.nperp, plane = (int64_t)a.g.nxi * nperp, np = a.np;
  double Y[4] = {a.Y0[0][p], a.Y0[1][p], a.Y0[2][p], a.Y0[3][p]};
  const int fm[6] = {F_PSI, F_DXPSI, F_DYPSI, F_BX, F_BY, F_BZ};
  for (int i = 0; i < a.len; ++i) {
    const int j = a.j0 + i;
    for (int c = 0; c < 4; ++c) a.segY[((int64_t)i * 4 + c) * np + p] = (R)Y[c];
    Six<R> F;
    for (int m = 0; m < 6; ++m) {
      F.a[m] = a.fields + fm[m] * plane + (int64_t)j * nperp;
      F.m1[m] = (j >= 1) ? F.a[m] - nperp : a.zero;
    }
    double Ys[4], Yn[4];
    for (int k = 0; k < a.K; ++k) {
      F.a[3] = a.biter + ((int64_t)k * 2 + 0) * plane + (int64_t)j * nperp;
      F.a[4] = a.biter + ((int64_t)k * 2 + 1) * plane + (int64_t)j * nperp;
      rk2_val(a.g, F, a.h, Y, Ys, Yn);
      for (int c = 0; c < 4; ++c) a.segYt[(((int64_t)i * a.K + k) * 4 + c) * np + p] = (R)Yn[c];
    }
    F.a[3] = a.fields + F_BX * plane + (int64_t)j * nperp;
    F.a[4] = a.fields + F_BY * plane + (int64_t)j * nperp;
    rk2_val(a.g, F, a.h, Y, Ys, Yn);
    Y[0] = wrap_pos((R)Yn[0], a.g.lx, a.g.inv_lx);
    Y[1] = wrap_pos((R)Yn[1], a.g.ly, a.g.inv_ly);
    Y[2] = (R)Yn[2];
    Y[3] = (R)Yn[3];
  }
}

// ---------------------------------------------------------------------------
// Beam: 3D linear shape with its gradient, sources and their transpose, the
// Boris push and its transpose.
// ---------------------------------------------------------------------------
template <typename R>
struct Cic3 {
  Cic<R> c;
  int j0;        // lower slice (may be -1 or nxi - 1)
  double fz;
  bool in;       // any node inside
};

template <typename R>
__device__ __forceinline__ Cic3<R> cic3(const Geo<R>& g, R x, R y, double xi, double inv_dxi) {
  Cic3<R> c;
  const double gz = xi * inv_dxi;
  c.in = gz > -1.0 && gz < (double)g.nxi;
  const double f0 = floor(gz);
  c.j0 = c.in ? (int)f0 : 0;
  c.fz = c.in ? gz - f0 : 0.0;
  c.c = cic(g, x, y);
  return c;
}

// value and gradient of the 3D interpolant of a [nxi][ny][nx] field
template <typename R>
__device__ __forceinline__ void cic3_val(const Geo<R>& g, const R* __restrict__ F, const Cic3<R>& c,
                                         double& v, double& vx, double& vy, double& vz) {
  v = vx = vy = vz = 0.0;
  if (!c.in) return;
  double a[2] = {0, 0}, ax[2] = {0, 0}, ay[2] = {0, 0};
  for (int d = 0; d < 2; ++d) {
    const int jj = c.j0 + d;
    if (jj < 0 || jj >= g.nxi) continue;
    cic_val(g, F + (int64_t)jj * g.nperp, c.c, a[d], ax[d], ay[d]);
  }
  v = (1.0 - c.fz) * a[0] + c.fz * a[1];
  vx = (1.0 - c.fz) * ax[0] + c.fz * ax[1];
  vy = (1.0 - c.fz) * ay[0] + c.fz * ay[1];
  vz = (a[1] - a[0]) / (double)g.dxi;
}

template <typename R>
__device__ __forceinline__ void cic3_add(const Geo<R>& g, R* __restrict__ F, const Cic3<R>& c, double q) {
  if (!c.in || q == 0.0) return;
  for (int d = 0; d < 2; ++d) {
    const int jj = c.j0 + d;
    if (jj < 0 || jj >= g.nxi) continue;
    cic_add(F + (int64_t)jj * g.nperp, c.c, q * (d ? c.fz : 1.0 - c.fz));
  }
}

// q times the 3D linear shape at c into channel ch of a tile over node
// slices (grid glob [nxi][ny][nx] when the box did not fit); m from
// merge_at3 (lanes whose particle has no node in the grid pass act = false)
template <int G, typename R>
__device__ __forceinline__ Merge merge_at3(bool act, const Cic3<R>& c, int nx) {
  return merge_of<G>(act && c.in, c.c.l0 * nx + c.c.i0, c.j0 + 1);
}

template <int G, typename R, typename T>
__device__ __forceinline__ void tile_add3(const Geo<R>& g, T* tile, const TileBox& b, int ch, const Cic3<R>& c,
                                          double q, R* glob, const Merge& m) {
  if (!b.fits) {   // uniform over the block
    if (m.act && q != 0.0) cic3_add(g, glob, c, q);
    return;
  }
  T w[2][4];
  for (int d = 0; d < 2; ++d) {
    const double qd = m.act ? q * (d ? c.fz : 1.0 - c.fz) : 0.0;
    w[d][0] = (T)(qd * (1 - c.c.fx) * (1 - c.c.fy));
    w[d][1] = (T)(qd * c.c.fx * (1 - c.c.fy));
    w[d][2] = (T)(qd * (1 - c.c.fx) * c.c.fy);
    w[d][3] = (T)(qd * c.c.fx * c.c.fy);
  }
  if (m.uni) {
#pragma unroll
    for (int d = 0; d < 2; ++d)
#pragma unroll
      for (int n = 0; n < 4; ++n) w[d][n] = group_sum<G>(w[d][n]);
    if (!m.lead) return;
  } else if (!m.act || q == 0.0) {
    return;
  }
  for (int d = 0; d < 2; ++d) {
    T* t = tile + ch * b.nodes + ((c.j0 + d - b.j0) * b.nl + (c.c.l0 - b.l0)) * b.ni + (c.c.i0 - b.i0);
    atomicAdd(t, w[d][0]);
    atomicAdd(t + 1, w[d][1]);
    atomicAdd(t + b.ni, w[d][2]);
    atomicAdd(t + b.ni + 1, w[d][3]);
  }
}

template <typename R>
struct AdjBeam {
  Geo<R> g;
  int64_t n;
  double zdv;          // Z/(dx dy dxi)
  double qh;           // (Z/M) dt/2
  double dt;
  double inv_dxi;
  double xi_max;
  const R* x;          // state at step n (tape)
  const R* y;
  const double* xi;
  const R* ux;
  const R* uy;
  const R* uz;
  const R* w;
  R* xo;               // forward: state at step n + 1
  R* yo;
  double* xio;
  R* uxo;
  R* uyo;
  R* uzo;
  R* wo;
  R* src;              // forward: sources [4][nxi][ny][nx]
  const R* srcb;       // reverse: their adjoint
  const R* fields;     // [7][nxi][ny][nx] of the step's sweep
  R* fieldsb;          // their adjoint
  R* b[7];             // adjoint of x, y, xi, ux, uy, uz, w (in place: step n+1 -> step n)
  int tile_bytes;      // dynamic LDS of the launch (scatter tile)
};

// 1 - v_z, v_x, v_y, v_z per unit charge and their u-derivatives
__device__ __forceinline__ void beam_v(double ux, double uy, double uz, double (&v)[4], double (&dv)[4][3]) {
  const double up2 = ux * ux + uy * uy;
  const double g2 = 1.0 + up2 + uz * uz;
  const double gam = sqrt(g2);
  const double P = 1.0 + up2, Q = gam * (gam + uz);
  v[0] = P / Q;
  v[1] = ux / gam;
  v[2] = uy / gam;
  v[3] = uz / gam;
  const double u[3] = {ux, uy, uz};
  const double g3 = gam * g2;
  for (int a = 0; a < 3; ++a) {
    const double dgam = u[a] / gam;
    const double dQ = (2.0 * gam + uz) * dgam + (a == 2 ? gam : 0.0);
    const double dP = (a < 2) ? 2.0 * u[a] : 0.0;
    dv[0][a] = (dP * Q - P * dQ) / (Q * Q);
    for (int b = 0; b < 3; ++b) dv[1 + b][a] = ((a == b) ? 1.0 / gam : 0.0) - u[b] * u[a] / g3;
  }
}

template <typename R>
__global__ void __launch_bounds__(256) k_ab_sources(AdjBeam<R> a) {
  ADJ_TILE(4, a.tile_bytes, R);
  const int64_t p = (int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const bool live = p < a.n && a.w[p] != R(0);
  Cic3<R> c{};
  double q[4] = {0, 0, 0, 0};
  if (live) {
    c = cic3(a.g, a.x[p], a.y[p], a.xi[p], a.inv_dxi);
    double v[4], dv[4][3];
    beam_v(a.ux[p], a.uy[p], a.uz[p], v, dv);
    const double qw = a.zdv * (double)a.w[p];
    for (int k = 0; k < 4; ++k) q[k] = qw * v[k];
    if (c.in) box_add(bx, c.j0, c.c.l0, c.c.i0);
  }
  const TileBox b = box_reduce<2>(bx, red, CAP_);
  tile_zero(tile, b, NCH_);
  const int64_t plane = (int64_t)a.g.nxi * a.g.nperp;
  R* const dst[4] = {a.src, a.src + plane, a.src + 2 * plane, a.src + 3 * plane};
  const Merge m = merge_at3<8>(live, c, a.g.nx);
  for (int k = 0; k < 4; ++k) tile_add3<8>(a.g, tile, b, k, c, q[k], dst[k], m);
  tile_flush<R, 4>(a.g, tile, b, dst, a.g.nxi);
}

// Transpose of the sources: adds to the adjoints of position, momentum and
// weight of step n.
template <typename R>
__global__ void __launch_bounds__(256) k_ab_sources_adj(AdjBeam<R> a) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.n || a.w[p] == R(0)) return;
  const Cic3<R> c = cic3(a.g, a.x[p], a.y[p], a.xi[p], a.inv_dxi);
  double v[4], dv[4][3];
  beam_v(a.ux[p], a.uy[p], a.uz[p], v, dv);
  const double q = a.zdv * (double)a.w[p];
  const int64_t plane = (int64_t)a.g.nxi * a.g.nperp;
  double gb[4], pos[3] = {0, 0, 0}, ub[3] = {0, 0, 0}, wb = 0.0;
  for (int k = 0; k < 4; ++k) {
    double s, sx, sy, sz;
    cic3_val(a.g, a.srcb + k * plane, c, s, sx, sy, sz);
    gb[k] = s;
    pos[0] += q * v[k] * sx;
    pos[1] += q * v[k] * sy;
    pos[2] += q * v[k] * sz;
    wb += a.zdv * v[k] * s;
    for (int d = 0; d < 3; ++d) ub[d] += q * s * dv[k][d];
  }
  a.b[0][p] = (R)((double)a.b[0][p] + pos[0]);
  a.b[1][p] = (R)((double)a.b[1][p] + pos[1]);
  a.b[2][p] = (R)((double)a.b[2][p] + pos[2]);
  a.b[3][p] = (R)((double)a.b[3][p] + ub[0]);
  a.b[4][p] = (R)((double)a.b[4][p] + ub[1]);
  a.b[5][p] = (R)((double)a.b[5][p] + ub[2]);
  a.b[6][p] = (R)((double)a.b[6][p] + wb);
}

__device__ __forceinline__ void cross3(const double (&a)[3], const double (&b)[3], double (&c)[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// The six beam-push fields (d_x psi, d_y psi, E_z, B_x, B_y, B_z) at the
// particle, with gradients.
template <typename R>
__device__ __forceinline__ void boris_fields(const AdjBeam<R>& a, const Cic3<R>& c, double (&f)[6],
                                             double (&fg)[6][3]) {
  const int slot[6] = {F_DXPSI, F_DYPSI, F_EZ, F_BX, F_BY, F_BZ};
  const int64_t plane = (int64_t)a.g.nxi * a.g.nperp;
  for (int m = 0; m < 6; ++m) cic3_val(a.g, a.fields + slot[m] * plane, c, f[m], fg[m][0], fg[m][1], fg[m][2]);
}

template <typename R>
__global__ void __launch_bounds__(256) k_ab_push(AdjBeam<R> a) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.n) return;
  const Cic3<R> c = cic3(a.g, a.x[p], a.y[p], a.xi[p], a.inv_dxi);
  double f[6], fg[6][3];
  boris_fields(a, c, f, fg);
  const double E[3] = {-f[0] + f[4], -f[1] - f[3], f[2]};
  const double B[3] = {f[3], f[4], f[5]};
  double um[3] = {a.ux[p] + a.qh * E[0], a.uy[p] + a.qh * E[1], a.uz[p] + a.qh * E[2]};
  const double gm = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
  const double t[3] = {a.qh * B[0] / gm, a.qh * B[1] / gm, a.qh * B[2] / gm};
  const double s = 2.0 / (1.0 + t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
  const double sv[3] = {s * t[0], s * t[1], s * t[2]};
  double cx[3], up[3], uq[3];
  cross3(um, t, cx);
  for (int d = 0; d < 3; ++d) up[d] = um[d] + cx[d];
  cross3(up, sv, cx);
  for (int d = 0; d < 3; ++d) uq[d] = um[d] + cx[d];
  const double un[3] = {uq[0] + a.qh * E[0], uq[1] + a.qh * E[1], uq[2] + a.qh * E[2]};
  const double up2 = un[0] * un[0] + un[1] * un[1];
  const double gam = sqrt(1.0 + up2 + un[2] * un[2]);
  a.xo[p] = wrap_pos((R)(a.x[p] + a.dt * un[0] / gam), a.g.lx, a.g.inv_lx);
  a.yo[p] = wrap_pos((R)(a.y[p] + a.dt * un[1] / gam), a.g.ly, a.g.inv_ly);
  const double xin = a.xi[p] + a.dt * (1.0 + up2) / (gam * (gam + un[2]));
  a.xio[p] = xin;
  a.uxo[p] = (R)un[0];
  a.uyo[p] = (R)un[1];
  a.uzo[p] = (R)un[2];
  a.wo[p] = (xin >= a.xi_max) ? R(0) : a.w[p];
}

// Transpose of the push: b (adjoints at step n + 1) -> adjoints at step n
// (in place), field adjoints deposited.
template <typename R>
__device__ __forceinline__ void push_adj_one(const AdjBeam<R>& a, int64_t p, const Cic3<R>& c, double (&gb)[6]);

template <typename R>
__global__ void __launch_bounds__(256) k_ab_push_adj(AdjBeam<R> a) {
  ADJ_TILE(6, a.tile_bytes, R);
  const int64_t p = (int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const bool live = p < a.n;
  Cic3<R> c{};
  double gb[6] = {0, 0, 0, 0, 0, 0};
  if (live) {
    c = cic3(a.g, a.x[p], a.y[p], a.xi[p], a.inv_dxi);
    push_adj_one(a, p, c, gb);
    if (c.in) box_add(bx, c.j0, c.c.l0, c.c.i0);
  }
  const TileBox b = box_reduce<2>(bx, red, CAP_);
  tile_zero(tile, b, NCH_);
  const int slot[6] = {F_DXPSI, F_DYPSI, F_EZ, F_BX, F_BY, F_BZ};
  const int64_t plane = (int64_t)a.g.nxi * a.g.nperp;
  R* dst[6];
  for (int m = 0; m < 6; ++m) dst[m] = a.fieldsb + slot[m] * plane;
  const Merge mg = merge_at3<8>(live, c, a.g.nx);
  for (int m = 0; m < 6; ++m) tile_add3<8>(a.g, tile, b, m, c, gb[m], dst[m], mg);
  tile_flush<R, 6>(a.g, tile, b, dst, a.g.nxi);
}

// One particle of the push transpose: its adjoints at step n + 1 -> step n
// (in place); gb: the adjoints of the six gathered field values.
template <typename R>
__device__ __forceinline__ void push_adj_one(const AdjBeam<R>& a, int64_t p, const Cic3<R>& c, double (&gb)[6]) {
  double f[6], fg[6][3];
  boris_fields(a, c, f, fg);
  const double qh = a.qh, dt = a.dt;
  const double E[3] = {-f[0] + f[4], -f[1] - f[3], f[2]};
  const double B[3] = {f[3], f[4], f[5]};
  double um[3] = {a.ux[p] + qh * E[0], a.uy[p] + qh * E[1], a.uz[p] + qh * E[2]};
  const double gm = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
  const double t[3] = {qh * B[0] / gm, qh * B[1] / gm, qh * B[2] / gm};
  const double tt = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
  const double s = 2.0 / (1.0 + tt);
  const double sv[3] = {s * t[0], s * t[1], s * t[2]};
  double cx[3], up[3], uq[3];
  cross3(um, t, cx);
  for (int d = 0; d < 3; ++d) up[d] = um[d] + cx[d];
  cross3(up, sv, cx);
  for (int d = 0; d < 3; ++d) uq[d] = um[d] + cx[d];
  const double un[3] = {uq[0] + qh * E[0], uq[1] + qh * E[1], uq[2] + qh * E[2]};
  const double up2 = un[0] * un[0] + un[1] * un[1];
  const double g2 = 1.0 + up2 + un[2] * un[2];
  const double gam = sqrt(g2);
  const double xin = a.xi[p] + dt * (1.0 + up2) / (gam * (gam + un[2]));
  // adjoints at step n + 1
  const double xb = a.b[0][p], yb = a.b[1][p], xib = a.b[2][p];
  double unb[3] = {a.b[3][p], a.b[4][p], a.b[5][p]};
  const double wb = (xin >= a.xi_max) ? 0.0 : (double)a.b[6][p];
  // x' = x + dt un_x/gam, y' likewise, xi' = xi + dt P/Q
  const double g3 = gam * g2;
  for (int d = 0; d < 3; ++d) {
    unb[d] += xb * dt * (((d == 0) ? 1.0 / gam : 0.0) - un[0] * un[d] / g3);
    unb[d] += yb * dt * (((d == 1) ? 1.0 / gam : 0.0) - un[1] * un[d] / g3);
  }
  {
    const double P = 1.0 + up2, Q = gam * (gam + un[2]);
    for (int d = 0; d < 3; ++d) {
      const double dgam = un[d] / gam;
      const double dQ = (2.0 * gam + un[2]) * dgam + (d == 2 ? gam : 0.0);
      const double dP = (d < 2) ? 2.0 * un[d] : 0.0;
      unb[d] += xib * dt * (dP * Q - P * dQ) / (Q * Q);
    }
  }
  // un = uq + qh E
  double Eb[3] = {qh * unb[0], qh * unb[1], qh * unb[2]};
  double uqb[3] = {unb[0], unb[1], unb[2]};
  // uq = um + up x sv
  double umb[3] = {uqb[0], uqb[1], uqb[2]};
  double upb[3], svb[3];
  cross3(sv, uqb, upb);     // up_bar += sv x uq_bar
  cross3(uqb, up, svb);     // sv_bar += uq_bar x up
  // sv = s t, s = 2/(1 + |t|^2)
  const double svt = svb[0] * t[0] + svb[1] * t[1] + svb[2] * t[2];
  double tb[3];
  for (int d = 0; d < 3; ++d) tb[d] = s * svb[d] - s * s * svt * t[d];
  // up = um + um x t
  for (int d = 0; d < 3; ++d) umb[d] += upb[d];
  double tmp[3];
  cross3(t, upb, tmp);      // um_bar += t x up_bar
  for (int d = 0; d < 3; ++d) umb[d] += tmp[d];
  cross3(upb, um, tmp);     // t_bar += up_bar x um
  for (int d = 0; d < 3; ++d) tb[d] += tmp[d];
  // t = qh B/gm
  double Bb[3];
  double gmb = 0.0;
  for (int d = 0; d < 3; ++d) {
    Bb[d] = qh * tb[d] / gm;
    gmb -= tb[d] * t[d] / gm;
  }
  // gm = sqrt(1 + |um|^2)
  for (int d = 0; d < 3; ++d) umb[d] += gmb * um[d] / gm;
  // um = u + qh E
  for (int d = 0; d < 3; ++d) Eb[d] += qh * umb[d];
  // field values: (dxpsi, dypsi, Ez, Bx, By, Bz)
  gb[0] = -Eb[0];
  gb[1] = -Eb[1];
  gb[2] = Eb[2];
  gb[3] = -Eb[1] + Bb[0];
  gb[4] = Eb[0] + Bb[1];
  gb[5] = Bb[2];
  double pos[3] = {xb, yb, xib};
  for (int m = 0; m < 6; ++m)
    for (int d = 0; d < 3; ++d) pos[d] += gb[m] * fg[m][d];
  a.b[0][p] = (R)pos[0];
  a.b[1][p] = (R)pos[1];
  a.b[2][p] = (R)pos[2];
  a.b[3][p] = (R)umb[0];
  a.b[4][p] = (R)umb[1];
  a.b[5][p] = (R)umb[2];
  a.b[6][p] = (R)wb;
}

// bins in the library's particle order: out[p] = bin_at_load[id[p]]
__global__ void __launch_bounds__(256) k_gather_bins(const int* __restrict__ bin_at_load,
                                                     const int64_t* __restrict__ id, int* __restrict__ out,
                                                     int64_t n) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) out[p] = bin_at_load[id[p]];
}

// weights scaled by their bin amplitude
template <typename R>
__global__ void __launch_bounds__(256) k_ab_scale_w(const R* __restrict__ w0, const int* __restrict__ bin,
                                                    const double* __restrict__ amp, int nb, R* __restrict__ w,
                                                    int64_t n) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int b = bin[p];
  w[p] = (b >= 0 && b < nb) ? (R)((double)w0[p] * amp[b]) : w0[p];
}

// gradient per bin: sum_p w_bar_p w0_p (LDS per-bin sums, one atomic per
// bin per block)
template <typename R>
__global__ void __launch_bounds__(256) k_ab_bin_grad(const R* __restrict__ wb, const R* __restrict__ w0,
                                                     const int* __restrict__ bin, int nb, double* __restrict__ grad,
                                                     int64_t n) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* acc = reinterpret_cast<double*>(smem_raw);
  for (int i = threadIdx.x; i < nb; i += blockDim.x) acc[i] = 0.0;
  __syncthreads();
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    const int b = bin[p];
    if (b >= 0 && b < nb) atomicAdd(acc + b, (double)wb[p] * (double)w0[p]);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nb; i += blockDim.x)
    if (acc[i] != 0.0) atomicAdd(grad + i, acc[i]);
}

}  // namespace qsa
