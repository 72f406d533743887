// Conducting-wall (Dirichlet) transverse solves by sine transforms: the
// sine-transform counterpart of the periodic Fourier solves of the field
// equations (the pseudo-potential's Poisson equation, Eq. (2) in its linear
// form, and the Helmholtz-shifted B_perp iteration), for boxes whose walls at
// x = 0, L_x and y = 0, L_y hold the potential at zero.
//
// On nx x ny interior nodes (x_i = i dx, i = 1..nx, L_x = (nx+1) dx; the same
// in y) the solution of (-lap_perp + kappa^2) u = f is expanded in the wall
// modes sin(m pi x/L_x) sin(n pi y/L_y), m <= nx, n <= ny, in which the
// operator is diagonal with eigenvalue (m pi/L_x)^2 + (n pi/L_y)^2 + kappa^2.
// The transform to those modes is the DST-I
//   S[m] = sum_{i=1..N} f[i] sin(pi i m/(N+1)),
// its own inverse up to the factor 2/(N+1).  A DST-I of length N is taken
// from one complex FFT of length M = 2(N+1) (a power of two): the odd
// extension a = (0, f_1..f_N, 0, -f_N..-f_1) has the transform A_m = -2i S_m,
// and two rows a, b packed as a + ib give Z_m = 2 S^b_m - 2i S^a_m, so
// S^a_m = -Im Z_m/2 and S^b_m = Re Z_m/2 from one transform.  The FFT is the
// LDS Stockham engine of the periodic solves (qsa_device.h).
//
// 2D: row pass (DST along x, in place), column pass (DST along y, divide by
// the eigenvalue, DST back along y, times 2/(ny+1)), row pass (DST back
// along x, times 2/(nx+1)).  Slab (ny = 1): one row pass that transforms,
// divides and transforms back.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "qsa_device.h"

namespace qsa {

// Twiddles exp(-2 pi i k/M), k < M, into LDS (no context: made per block).
template <typename R>
__device__ __forceinline__ void dst_twiddles(C2<R>* tw, int M) {
  for (int k = threadIdx.x; k < M; k += blockDim.x) {
    double s, c;
    sincospi(2.0 * (double)k / (double)M, &s, &c);
    tw[k] = C2<R>{(R)c, (R)(-s)};
  }
}

// Odd extension of two real sequences (a, b) of length N = M/2 - 1 as a + ib
// at position j of the length-M transform input: get(k) returns (a_k, b_k)
// for k = 1..N.
template <typename R, typename Get>
__device__ __forceinline__ C2<R> odd_pair(int j, int M, Get get) {
  const int N1 = M >> 1;   // N + 1
  if (j == 0 || j == N1) return C2<R>{R(0), R(0)};
  if (j < N1) return get(j);
  const C2<R> v = get(M - j);
  return C2<R>{-v.x, -v.y};
}

// Threads per transform of length M and transforms per 256-thread block.
__host__ __device__ __forceinline__ int dst_tpt(int M) { return M >= 4 ? M >> 2 : 1; }

// LDS bytes of a 256-thread block of transforms of length M: twiddles and
// two FFT buffers per transform.
template <typename R>
__host__ __device__ __forceinline__ size_t dst_lds(int M) {
  const int per = 256 / dst_tpt(M);
  return ((size_t)M + 2 * (size_t)per * fft_cap(M)) * sizeof(C2<R>);
}

// Rows of length nx (nrows of them, row-major, consecutive rows paired):
// out = scale * DST-I(in) along x; with `solve` (slab) the row's modes are
// divided by (m pi/L_x)^2 + kappa2 and transformed back before the scale.
// in and out may be the same array (each row is read before it is written,
// by the same block).
template <typename R>
__global__ void __launch_bounds__(256) k_dst_rows(int64_t nrows, int nx, int lg, const R* in, R* out,
                                                  double scale, int solve, double inv_lx, double kappa2) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C2<R>* tw = reinterpret_cast<C2<R>*>(smem_raw);
  const int M = 1 << lg;
  const int tpt = dst_tpt(M);
  const int per = blockDim.x / tpt;
  const int slot = threadIdx.x / tpt, t = threadIdx.x - slot * tpt;
  const int64_t pair = (int64_t)blockIdx.x * per + slot;
  const int64_t r0 = 2 * pair, r1 = 2 * pair + 1;
  const bool v0 = r0 < nrows, v1 = r1 < nrows;
  C2<R>* A = tw + M + (size_t)slot * 2 * fft_cap(M);
  C2<R>* B = A + fft_cap(M);
  dst_twiddles(tw, M);
  const R* a_in = in + r0 * nx;
  const R* b_in = in + r1 * nx;
  for (int j = t; j < M; j += tpt)
    A[j] = odd_pair<R>(j, M, [&](int k) {
      return C2<R>{v0 ? a_in[k - 1] : R(0), v1 ? b_in[k - 1] : R(0)};
    });
  __syncthreads();
  C2<R>* res = fft_lds<R, false>(A, B, M, lg, t, tpt, tw);
  if (solve) {
    // the modes S_m = (-Im Z_m/2, Re Z_m/2) over the eigenvalue, odd-extended
    // into the free buffer, and the second transform
    C2<R>* o = (res == A) ? B : A;
    for (int j = t; j < M; j += tpt)
      o[j] = odd_pair<R>(j, M, [&](int m) {
        const double km = 3.14159265358979323846 * (double)m * inv_lx;
        const double d = 1.0 / (km * km + kappa2);
        const C2<R> z = res[m];
        return C2<R>{(R)(-0.5 * (double)z.y * d), (R)(0.5 * (double)z.x * d)};
      });
    __syncthreads();
    C2<R>* other = (o == A) ? B : A;
    res = fft_lds<R, false>(o, other, M, lg, t, tpt, tw);
  }
  R* a_out = out + r0 * nx;
  R* b_out = out + r1 * nx;
  for (int m = 1 + t; m <= nx; m += tpt) {
    const C2<R> z = res[m];
    if (v0) a_out[m - 1] = (R)(-0.5 * scale * (double)z.y);
    if (v1) b_out[m - 1] = (R)(0.5 * scale * (double)z.x);
  }
}

// Columns of n_grid grids [ny][nx] (in place), two adjacent columns per
// transform: the y-DST, the division by the eigenvalue of the mode pair
// (m, n) (m = column + 1: the row pass has already taken x to modes), the
// y-DST back, times scale_y = 2/(ny+1).
template <typename R>
__global__ void __launch_bounds__(256) k_dst_cols(int n_grid, int nx, int ny, int lg, R* u, double inv_lx,
                                                  double inv_ly, double kappa2, double scale_y) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C2<R>* tw = reinterpret_cast<C2<R>*>(smem_raw);
  const int M = 1 << lg;
  const int tpt = dst_tpt(M);
  const int per = blockDim.x / tpt;
  const int slot = threadIdx.x / tpt, t = threadIdx.x - slot * tpt;
  const int cpairs = (nx + 1) >> 1;
  const int64_t q = (int64_t)blockIdx.x * per + slot;   // (grid, column pair)
  const bool live = q < (int64_t)n_grid * cpairs;
  const int64_t gi = live ? q / cpairs : 0;
  const int c0 = live ? 2 * (int)(q - gi * cpairs) : 0, c1 = c0 + 1;
  const bool v1 = live && c1 < nx;
  R* base = u + gi * (int64_t)ny * nx;
  C2<R>* A = tw + M + (size_t)slot * 2 * fft_cap(M);
  C2<R>* B = A + fft_cap(M);
  dst_twiddles(tw, M);
  for (int j = t; j < M; j += tpt)
    A[j] = odd_pair<R>(j, M, [&](int k) {
      const R* row = base + (int64_t)(k - 1) * nx;
      return C2<R>{live ? row[c0] : R(0), v1 ? row[c1] : R(0)};
    });
  __syncthreads();
  C2<R>* res = fft_lds<R, false>(A, B, M, lg, t, tpt, tw);
  C2<R>* o = (res == A) ? B : A;
  const double ka = 3.14159265358979323846 * (double)(c0 + 1) * inv_lx;
  const double kb = 3.14159265358979323846 * (double)(c1 + 1) * inv_lx;
  for (int j = t; j < M; j += tpt)
    o[j] = odd_pair<R>(j, M, [&](int n) {
      const double kn = 3.14159265358979323846 * (double)n * inv_ly;
      const C2<R> z = res[n];
      return C2<R>{(R)(-0.5 * (double)z.y / (ka * ka + kn * kn + kappa2)),
                   (R)(0.5 * (double)z.x / (kb * kb + kn * kn + kappa2))};
    });
  __syncthreads();
  C2<R>* other = (o == A) ? B : A;
  res = fft_lds<R, false>(o, other, M, lg, t, tpt, tw);
  for (int n = 1 + t; n <= ny; n += tpt) {
    const C2<R> z = res[n];
    R* row = base + (int64_t)(n - 1) * nx;
    if (live) row[c0] = (R)(-0.5 * scale_y * (double)z.y);
    if (v1) row[c1] = (R)(0.5 * scale_y * (double)z.x);
  }
}

}  // namespace qsa
