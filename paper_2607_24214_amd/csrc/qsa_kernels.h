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
enum { ERR_BREAKDOWN = 1 };

#define QSA_GMIN 1.0e-3

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

// ------------------------------------------------------------ row transforms
template <typename R>
struct RowR2CArgs {
  R* dep[4];          // deposit grid [nperp]: read, then cleared for the next deposit
  const R* add[4];    // grid added on load (beam source slice) or null
  R addc[4];          // constant added on load (ion background)
  C2<R>* out[4];      // half spectra [ny][nxh]
};

// Real rows -> half spectra along x.  Rows 2p and 2p+1 are packed as the
// real and imaginary parts of one complex transform and separated after it.
template <typename R>
__global__ void __launch_bounds__(256) k_row_r2c(Geo<R> g, RowR2CArgs<R> a,
                                                 const C2<R>* __restrict__ twx, int ppw) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C2<R>* sm = reinterpret_cast<C2<R>*>(smem_raw);
  const int f = blockIdx.y;
  const int tpt = g.nx >> 2;
  const int slot = threadIdx.x / tpt, t = threadIdx.x - slot * tpt;
  const int npairs = (g.ny + 1) >> 1;
  const int pair = blockIdx.x * ppw + slot;
  const bool v0 = pair < npairs;
  const int r0 = 2 * pair, r1 = 2 * pair + 1;
  const bool v1 = v0 && r1 < g.ny;
  C2<R>* A = sm + (size_t)slot * 2 * g.nx;
  C2<R>* B = A + g.nx;
  R* dep = a.dep[f];
  const R* add = a.add[f];
  const R c = a.addc[f];
  for (int i = t; i < g.nx; i += tpt) {
    R va = 0, vb = 0;
    if (v0) {
      const int o = r0 * g.nx + i;
      va = c;
      if (dep) {
        va += dep[o];
        dep[o] = 0;
      }
      if (add) va += add[o];
    }
    if (v1) {
      const int o = r1 * g.nx + i;
      vb = c;
      if (dep) {
        vb += dep[o];
        dep[o] = 0;
      }
      if (add) vb += add[o];
    }
    A[i] = C2<R>{va, vb};
  }
  __syncthreads();
  C2<R>* res = fft_lds<R, false>(A, B, g.nx, g.lgx, t, tpt, twx);
  if (v0) {
    C2<R>* out = a.out[f];
    for (int k = t; k < g.nxh; k += tpt) {
      const C2<R> z = res[k];
      const C2<R> zc = cconj(res[(g.nx - k) & (g.nx - 1)]);
      const C2<R> s = cadd(z, zc), d = csub(z, zc);
      out[r0 * g.nxh + k] = C2<R>{R(0.5) * s.x, R(0.5) * s.y};
      if (v1) out[r1 * g.nxh + k] = C2<R>{R(0.5) * d.y, R(-0.5) * d.x};
    }
  }
}

template <typename R>
struct RowC2RArgs {
  const C2<R>* in[4];  // half spectra [ny][nxh]
  R* out[4];           // real grids [nperp]
};

// Half spectra -> real rows (unnormalized inverse; the 1/(nx ny) factor is
// applied in the column pass).  Two rows are packed as A + iB.
template <typename R>
__global__ void __launch_bounds__(256) k_row_c2r(Geo<R> g, RowC2RArgs<R> a,
                                                 const C2<R>* __restrict__ twx, int ppw) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C2<R>* sm = reinterpret_cast<C2<R>*>(smem_raw);
  const int f = blockIdx.y;
  const int tpt = g.nx >> 2;
  const int slot = threadIdx.x / tpt, t = threadIdx.x - slot * tpt;
  const int npairs = (g.ny + 1) >> 1;
  const int pair = blockIdx.x * ppw + slot;
  const bool v0 = pair < npairs;
  const int r0 = 2 * pair, r1 = 2 * pair + 1;
  const bool v1 = v0 && r1 < g.ny;
  C2<R>* A = sm + (size_t)slot * 2 * g.nx;
  C2<R>* B = A + g.nx;
  const C2<R>* in = a.in[f];
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
  C2<R>* res = fft_lds<R, true>(A, B, g.nx, g.lgx, t, tpt, twx);
  if (v0) {
    R* out = a.out[f];
    for (int i = t; i < g.nx; i += tpt) {
      const C2<R> z = res[i];
      out[r0 * g.nx + i] = z.x;
      if (v1) out[r1 * g.nx + i] = z.y;
    }
  }
}

// ---------------------------------------------------------- column transforms
template <typename R>
struct ColArgs {
  const C2<R>* in[3];     // half spectra [ny][nxh] after the row pass
  C2<R>* out[4];          // outputs, y-inverse-transformed, for k_row_c2r
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

// Threads per column transform for ny rows (loops cover the rest).
__host__ __device__ __forceinline__ int col_tpt(int ny) {
  const int t = ny >> 2;
  return t < 1 ? 1 : (t > 64 ? 64 : t);
}

// Forward transform along y of each input column, the spectral solve of the
// mode, inverse transform along y of each output.  Each column is worked by
// G groups of tpt threads, one group per field transform, so the transforms
// of one column run side by side; cpw columns per block.
template <typename R, int MODE>
__global__ void __launch_bounds__(256) k_col(Geo<R> g, ColArgs<R> a,
                                             const C2<R>* __restrict__ twy, int cpw) {
  using S = ColShape<MODE>;
  constexpr int G = S::G;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C2<R>* sm = reinterpret_cast<C2<R>*>(smem_raw);
  const int ny = g.ny;
  const int tpt = col_tpt(ny);
  const int per_col = G * tpt;
  const int c = threadIdx.x / per_col;
  const int r = threadIdx.x - c * per_col;
  const int grp = r / tpt, t = r - grp * tpt;
  const int kx = blockIdx.x * cpw + c;
  const bool valid = kx < g.nxh;
  C2<R>* D = sm + (size_t)c * 2 * G * ny;   // G data columns
  C2<R>* Sx = D + G * ny;                   // G scratch columns
  C2<R>* mine = D + grp * ny;
  for (int y = t; y < ny; y += tpt)
    mine[y] = (valid && grp < S::NIN) ? a.in[grp][y * g.nxh + kx] : C2<R>{0, 0};
  __syncthreads();
  fft_lds_inplace<R, false>(mine, Sx + grp * ny, ny, g.lgy, t, tpt, twy);

  for (int y = r; y < ny; y += per_col) {
    C2<R> o[S::NOUT];
#pragma unroll
    for (int q = 0; q < S::NOUT; ++q) o[q] = C2<R>{0, 0};
    if (valid) {
      const int e = y * g.nxh + kx;
      const R kdx = a.kdx[kx], kdy = a.kdy[y];
      const R ksq = a.kx2[kx] + a.ky2[y];
      const bool k0 = (kx == 0 && y == 0);
      const R iks = k0 ? R(0) : R(1) / ksq;
      if (MODE == COL_PSI) {
        // -lap psi = rho - J_z; the k = 0 value is the transverse-mean wake
        C2<R> ph = cscale(D[y], iks);
        if (k0) ph = C2<R>{(R)a.ode[1] * a.n_perp, R(0)};
        o[0] = cscale(ph, a.inv_n);
        o[1] = cscale(cmul_ik(ph, kdx), a.inv_n);
        o[2] = cscale(cmul_ik(ph, kdy), a.inv_n);
      } else if (MODE == COL_J) {
        const C2<R> jx = D[y], jy = D[ny + y], jzv = D[2 * ny + y];
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
        const C2<R> dx = cscale(csub(D[y], a.jr_r[0][e]), i2h);
        const C2<R> dy = cscale(csub(D[ny + y], a.jr_r[1][e]), i2h);
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
    for (int q = 0; q < S::NOUT; ++q) D[q * ny + y] = o[q];
  }
  __syncthreads();
  fft_lds_inplace<R, true>(mine, Sx + grp * ny, ny, g.lgy, t, tpt, twy);
  if (valid && grp < S::NOUT)
    for (int y = t; y < ny; y += tpt) a.out[grp][y * g.nxh + kx] = mine[y];
}

// ---------------------------------------------------------- plasma particles
template <typename R>
struct PlasmaArgs {
  R* x;
  R* y;
  R* ux;
  R* uy;
  int np;
  R q;                // -w/(dx dy): rho - J_z per particle per unit area
  R* dep0;
  R* dep1;
  R* dep2;
  const R* F0[6];     // psi, d_x psi, d_y psi, B_x, B_y, B_z at slice j
  const R* F1[6];     // the same at j-1 (all null when j = 0)
  const R* psi_m2;    // psi at j-2 (null when j < 2)
  int* err;
  R h;
};

// Particle p of block b: the blocks of one XCD take consecutive chunks.
__device__ __forceinline__ int plasma_index() {
  return xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
}

template <typename R>
__global__ void __launch_bounds__(256) k_dep_S(Geo<R> g, PlasmaArgs<R> a) {
  __shared__ R tile[TileCap<R, 1>::NODES];
  __shared__ int bb[4];
  const int p = plasma_index();
  const bool live = p < a.np;
  int i0 = 0, l0 = 0;
  R fx = 0, fy = 0;
  if (live) cell2(g, a.x[p], a.y[p], i0, l0, fx, fy);
  const R v[1] = {a.q};
  R* const dst[1] = {a.dep0};
  block_deposit<R, 1>(g, live, i0, l0, fx, fy, v, dst, tile, bb);
}

template <typename R>
__global__ void __launch_bounds__(256) k_dep_J(Geo<R> g, PlasmaArgs<R> a) {
  __shared__ R tile[3 * TileCap<R, 3>::NODES];
  __shared__ int bb[4];
  const int p = plasma_index();
  const bool live = p < a.np;
  int i0 = 0, l0 = 0;
  R fx = 0, fy = 0;
  R v[3] = {0, 0, 0};
  if (live) {
    const R ux = a.ux[p], uy = a.uy[p];
    cell2(g, a.x[p], a.y[p], i0, l0, fx, fy);
    const Stencil<R> s = stencil2(g, a.x[p], a.y[p]);
    const R G = R(1) + gather(a.F0[0], s);
    if (!(G > R(QSA_GMIN))) atomicOr(a.err, ERR_BREAKDOWN);
    const R gam = (R(1) + ux * ux + uy * uy + G * G) / (R(2) * G);
    const R uz = gam - G;
    const R qg = a.q / G;
    v[0] = qg * ux;
    v[1] = qg * uy;
    v[2] = qg * uz;
  }
  R* const dst[3] = {a.dep0, a.dep1, a.dep2};
  block_deposit<R, 3>(g, live, i0, l0, fx, fy, v, dst, tile, bb);
}

// d/dxi of (x, y, u_x, u_y) from the six gathered fields
template <typename R>
__device__ __forceinline__ void plasma_rhs(const R f[6], R ux, R uy, R d[4], int* err) {
  const R G = R(1) + f[0];
  if (!(G > R(QSA_GMIN))) atomicOr(err, ERR_BREAKDOWN);
  const R iG = R(1) / G;
  const R gam = (R(1) + ux * ux + uy * uy + G * G) * R(0.5) * iG;
  d[0] = ux * iG;
  d[1] = uy * iG;
  d[2] = gam * f[1] * iG - f[4] - uy * f[5] * iG;
  d[3] = gam * f[2] * iG + f[3] + ux * f[5] * iG;
}

// RK2 (midpoint) push from slice j with F^j and F^{j+1/2} = (3F^j - F^{j-1})/2.
template <typename R>
__device__ __forceinline__ void rk2_push(const Geo<R>& g, const PlasmaArgs<R>& a, R x, R y, R ux,
                                         R uy, R& xn, R& yn, R& uxn, R& uyn) {
  const R hh = a.h;
  R f[6], d1[4], d2[4];
  {
    const Stencil<R> s = stencil2(g, x, y);
#pragma unroll
    for (int q = 0; q < 6; ++q) f[q] = gather(a.F0[q], s);
    plasma_rhs(f, ux, uy, d1, a.err);
  }
  const R xs = x + R(0.5) * hh * d1[0];
  const R ys = y + R(0.5) * hh * d1[1];
  const R uxs = ux + R(0.5) * hh * d1[2];
  const R uys = uy + R(0.5) * hh * d1[3];
  {
    const Stencil<R> s = stencil2(g, xs, ys);
    if (a.F1[0]) {
#pragma unroll
      for (int q = 0; q < 6; ++q) f[q] = R(0.5) * (R(3) * gather(a.F0[q], s) - gather(a.F1[q], s));
    } else {
#pragma unroll
      for (int q = 0; q < 6; ++q) f[q] = R(0.5) * (R(3) * gather(a.F0[q], s));
    }
    plasma_rhs(f, uxs, uys, d2, a.err);
  }
  xn = x + hh * d2[0];
  yn = y + hh * d2[1];
  uxn = ux + hh * d2[2];
  uyn = uy + hh * d2[3];
}

// Predictor: push a copy of Y^j to j+1 and deposit the predicted J_perp at
// j+1 with 1 + psi~ from psi~^{j+1} = 3 psi^j - 3 psi^{j-1} + psi^{j-2}.
template <typename R>
__global__ void __launch_bounds__(256) k_push_pred(Geo<R> g, PlasmaArgs<R> a) {
  __shared__ R tile[2 * TileCap<R, 2>::NODES];
  __shared__ int bb[4];
  const int p = plasma_index();
  const bool live = p < a.np;
  int i0 = 0, l0 = 0;
  R fx = 0, fy = 0;
  R v[2] = {0, 0};
  if (live) {
    R xn, yn, uxn, uyn;
    rk2_push(g, a, a.x[p], a.y[p], a.ux[p], a.uy[p], xn, yn, uxn, uyn);
    cell2(g, xn, yn, i0, l0, fx, fy);
    const Stencil<R> s = stencil2(g, xn, yn);
    R pt = R(3) * gather(a.F0[0], s);
    if (a.F1[0]) pt -= R(3) * gather(a.F1[0], s);
    if (a.psi_m2) pt += gather(a.psi_m2, s);
    const R G = R(1) + pt;
    if (!(G > R(QSA_GMIN))) atomicOr(a.err, ERR_BREAKDOWN);
    const R qg = a.q / G;
    v[0] = qg * uxn;
    v[1] = qg * uyn;
  }
  R* const dst[2] = {a.dep0, a.dep1};
  block_deposit<R, 2>(g, live, i0, l0, fx, fy, v, dst, tile, bb);
}

// Final advance: Y^{j+1} with the converged fields, positions wrapped.
template <typename R>
__global__ void __launch_bounds__(256) k_push_final(Geo<R> g, PlasmaArgs<R> a) {
  const int p = plasma_index();
  if (p >= a.np) return;
  R xn, yn, uxn, uyn;
  rk2_push(g, a, a.x[p], a.y[p], a.ux[p], a.uy[p], xn, yn, uxn, uyn);
  a.x[p] = wrap_pos(xn, g.lx, g.inv_lx);
  a.y[p] = wrap_pos(yn, g.ly, g.inv_ly);
  a.ux[p] = uxn;
  a.uy[p] = uyn;
}

// Counting sort of the plasma by cell (keeps the particles of a block close
// together, which is what makes the tiled deposits pay).
template <typename R>
__global__ void __launch_bounds__(256) k_sort_count(Geo<R> g, const R* __restrict__ x,
                                                    const R* __restrict__ y, int np,
                                                    int* __restrict__ cell_of, int* __restrict__ count) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  int i0, l0;
  R fx, fy;
  cell2(g, x[p], y[p], i0, l0, fx, fy);
  const int c = l0 * g.nx + i0;
  cell_of[p] = c;
  atomicAdd(&count[c], 1);
}

// Exclusive scan of v[0, n) in blocks of 1024: offsets within the block in
// place, block totals in bsum[block].
__global__ void __launch_bounds__(256) k_scan_local(int* __restrict__ v, int n, int* __restrict__ bsum) {
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
__global__ void __launch_bounds__(256) k_scan_blocks(int* __restrict__ bsum, int nb) {
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
__global__ void __launch_bounds__(256) k_sort_scatter(int np, const int* __restrict__ cell_of,
                                                      int* __restrict__ cursor, const int* __restrict__ bsum,
                                                      const R* __restrict__ x,
                                                      const R* __restrict__ y, const R* __restrict__ ux,
                                                      const R* __restrict__ uy, R* __restrict__ x2,
                                                      R* __restrict__ y2, R* __restrict__ ux2,
                                                      R* __restrict__ uy2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const int c = cell_of[p];
  const int d = atomicAdd(&cursor[c], 1) + bsum[c >> 10];
  x2[d] = x[p];
  y2[d] = y[p];
  ux2[d] = ux[p];
  uy2[d] = uy[p];
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
  R* src;             // [4][nxi][nperp]: rho - J_z, J_x, J_y, J_z
  const R* fields;    // [7][nxi][nperp]
  R zq;               // Z/(dx dy dxi)
  R qmh;              // (Z/M) dt/2
  R dt;
  double inv_dxi;
  double xi_max;      // (nxi - 1) dxi: particles at or beyond it leave the box
};

// 3D linear-shape deposit of the beam sources, staged through an LDS tile
// over the bounding box of the block's cells (same scheme as block_deposit,
// in (xi, y, x)); each thread brings BEAM_PPT particles.
#define BEAM_PPT 2
template <typename R>
__global__ void __launch_bounds__(256) k_beam_deposit(Geo<R> g, BeamArgs<R> a) {
  constexpr int CAP = TileCap<R, 4>::NODES;
  __shared__ R tile[4 * CAP];
  __shared__ int bb[6];
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)xcd_block(blockIdx.x, gridDim.x) * (256 * BEAM_PPT);
  bool live[BEAM_PPT];
  int j0[BEAM_PPT], l0[BEAM_PPT], i0[BEAM_PPT];
  R fz[BEAM_PPT], fx[BEAM_PPT], fy[BEAM_PPT], v[BEAM_PPT][4];
  if (tid == 0) {
    bb[0] = bb[1] = bb[2] = 0x7fffffff;
    bb[3] = bb[4] = bb[5] = -0x7fffffff;
  }
  for (int t = tid; t < 4 * CAP; t += 256) tile[t] = R(0);
#pragma unroll
  for (int k = 0; k < BEAM_PPT; ++k) {
    const int64_t p = base + k * 256 + tid;
    live[k] = false;
    j0[k] = l0[k] = i0[k] = 0;
    fz[k] = fx[k] = fy[k] = R(0);
    v[k][0] = v[k][1] = v[k][2] = v[k][3] = R(0);
    if (p < a.n) {
      const R w = a.w[p];
      const double gz = a.xi[p] * a.inv_dxi;
      if (w != R(0) && gz > -1.0 && gz < (double)g.nxi) {
        live[k] = true;
        const double fz0 = floor(gz);
        j0[k] = (int)fz0;
        fz[k] = (R)(gz - fz0);
        cell2(g, a.x[p], a.y[p], i0[k], l0[k], fx[k], fy[k]);
        const R ux = a.ux[p], uy = a.uy[p], uz = a.uz[p];
        const R up2 = ux * ux + uy * uy;
        const R gam = sqrt(R(1) + up2 + uz * uz);
        const R q = a.zq * w;
        v[k][0] = q * ((R(1) + up2) / (gam * (gam + uz)));   // 1 - v_z without cancellation
        v[k][1] = q * ux / gam;
        v[k][2] = q * uy / gam;
        v[k][3] = q * uz / gam;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < BEAM_PPT; ++k)
    if (live[k]) {
      atomicMin(&bb[0], j0[k]);
      atomicMin(&bb[1], l0[k]);
      atomicMin(&bb[2], i0[k]);
      atomicMax(&bb[3], j0[k]);
      atomicMax(&bb[4], l0[k]);
      atomicMax(&bb[5], i0[k]);
    }
  __syncthreads();
  const bool any = bb[3] >= bb[0];
  const int jmin = bb[0], lmin = bb[1], imin = bb[2];
  const int nj = any ? bb[3] - jmin + 2 : 0;
  const int nl = any ? bb[4] - lmin + 2 : 0;
  const int ni = any ? bb[5] - imin + 2 : 0;
  const bool fits = any && (int64_t)nj * nl * ni <= CAP;
  const int64_t plane = (int64_t)g.nxi * g.nperp;
#pragma unroll
  for (int k = 0; k < BEAM_PPT; ++k) {
    if (!live[k]) continue;
    const R wx[2] = {R(1) - fx[k], fx[k]};
    const R wy[2] = {R(1) - fy[k], fy[k]};
    const R wz[2] = {R(1) - fz[k], fz[k]};
#pragma unroll
    for (int dj = 0; dj < 2; ++dj)
#pragma unroll
      for (int dl = 0; dl < 2; ++dl)
#pragma unroll
        for (int di = 0; di < 2; ++di) {
          const R wt = wz[dj] * wy[dl] * wx[di];
          if (fits) {
            const int t = ((j0[k] + dj - jmin) * nl + (l0[k] + dl - lmin)) * ni + (i0[k] + di - imin);
#pragma unroll
            for (int c = 0; c < 4; ++c) atomicAdd(&tile[c * CAP + t], v[k][c] * wt);
          } else {
            const int jj = j0[k] + dj;
            if (jj < 0 || jj >= g.nxi) continue;
            int ll = l0[k] + dl;
            ll -= (ll >= g.ny) ? g.ny : 0;
            int ii = i0[k] + di;
            ii -= (ii >= g.nx) ? g.nx : 0;
            const int64_t node = (int64_t)jj * g.nperp + ll * g.nx + ii;
#pragma unroll
            for (int c = 0; c < 4; ++c) atomic_add(a.src + c * plane + node, v[k][c] * wt);
          }
        }
  }
  __syncthreads();
  if (fits) {
    const int nplane = nl * ni;
    for (int t = tid; t < nj * nplane; t += 256) {
      const int tj = t / nplane;
      const int r = t - tj * nplane;
      const int tl = r / ni, ti = r - tl * ni;
      const int jg = jmin + tj;
      if (jg < 0 || jg >= g.nxi) continue;
      int lg = lmin + tl;
      lg -= (lg >= g.ny) ? g.ny : 0;
      int ig = imin + ti;
      ig -= (ig >= g.nx) ? g.nx : 0;
      const int64_t node = (int64_t)jg * g.nperp + lg * g.nx + ig;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const R val = tile[c * CAP + t];
        if (val != R(0)) atomic_add(a.src + c * plane + node, val);
      }
    }
  }
}

// Boris push of the beam by dt in the stored fields, E = (-d_x psi + B_y,
// -d_y psi - B_x, E_z), B = (B_x, B_y, B_z), 3D linear shape, zero outside.
template <typename R>
__global__ void __launch_bounds__(256) k_beam_push(Geo<R> g, BeamArgs<R> a) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.n) return;
  const R x = a.x[p], y = a.y[p];
  const double xi = a.xi[p];
  R ux = a.ux[p], uy = a.uy[p], uz = a.uz[p];
  R fd[6] = {0, 0, 0, 0, 0, 0};   // d_x psi, d_y psi, E_z, B_x, B_y, B_z
  const double gz = xi * a.inv_dxi;
  if (gz > -1.0 && gz < (double)g.nxi) {
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
#pragma unroll
      for (int q = 0; q < 6; ++q)
        fd[q] += wz * gather(a.fields + slot[q] * plane + (int64_t)jj * g.nperp, s);
    }
  }
  const R ex = -fd[0] + fd[4];
  const R ey = -fd[1] - fd[3];
  const R ez = fd[2];
  const R bx = fd[3], by = fd[4], bz = fd[5];
  const R qh = a.qmh;
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
  a.x[p] = wrap_pos(x + a.dt * ux / gam, g.lx, g.inv_lx);
  a.y[p] = wrap_pos(y + a.dt * uy / gam, g.ly, g.inv_ly);
  const double xin = xi + (double)(a.dt * (R(1) + up2) / (gam * (gam + uz)));
  a.xi[p] = xin;
  a.ux[p] = ux;
  a.uy[p] = uy;
  a.uz[p] = uz;
  if (xin >= a.xi_max) a.w[p] = R(0);
}

}  // namespace qsa
