// Batched solver of the paper's single-mode linear model, Eq. (5):
//   [(d_xi^2 + 1) d_tau^2 - Gamma^2] dPsi = 0,
// written as the pair n = (d_xi^2 + 1) dPsi and the causal inverse
//   dPsi(xi) = int_0^xi sin(xi - xi') n(xi') dxi'
// (nothing ahead of the beam front), with d_tau^2 n = Gamma^2 dPsi advanced
// by classical RK4 in tau from n(xi, 0) = n0, d_tau n(xi, 0) = 0.  The xi
// integral is the trapezoid rule on the uniform grid xi_j = j dxi (end
// weight 1/2 at xi = 0; the integrand vanishes at xi' = xi).
//
// The quadrature sum_j c_j sin(xi_i - xi_j) n_j, c_0 = 1/2, is evaluated
// exactly as sin(xi_i) C_i - cos(xi_i) S_i with the prefix sums
// C_i = sum_{j<=i} c_j cos(xi_j) n_j and S_i = sum_{j<=i} c_j sin(xi_j) n_j:
// two block-wide scans per RK stage instead of a triangular matrix product.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qsa {

#define QSA_LIN_THREADS 1024
#define QSA_LIN_SEG 4          // xi points per thread: nxi <= 4096
#define QSA_LIN_MAX_OUT 256    // output times per call

struct LinOut {
  int64_t steps[QSA_LIN_MAX_OUT];   // cumulative RK4 steps at each output time
  int n;
};

// Exclusive block-wide prefix sums of (a, b) over the threads in order;
// ws: LDS scratch of 2 x 16 doubles.  Every thread calls it.
__device__ __forceinline__ void lin_block_scan(double& a, double& b, double* ws) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  double ia = a, ib = b;
  for (int o = 1; o < 64; o <<= 1) {
    const double ua = __shfl_up(ia, o), ub = __shfl_up(ib, o);
    if (lane >= o) {
      ia += ua;
      ib += ub;
    }
  }
  if (lane == 63) {
    ws[w] = ia;
    ws[16 + w] = ib;
  }
  __syncthreads();
  double oa = 0.0, ob = 0.0;
  for (int k = 0; k < w; ++k) {
    oa += ws[k];
    ob += ws[16 + k];
  }
  a = oa + ia - a;
  b = ob + ib - b;
  __syncthreads();
}

// q[k] = dxi sum_{j<=i} c_j sin(xi_i - xi_j) n_j at this thread's points
// i = t SEG + k (i < nxi), for values n at those points.
__device__ __forceinline__ void lin_volterra(const double (&n)[QSA_LIN_SEG], const double (&cs)[QSA_LIN_SEG],
                                             const double (&sn)[QSA_LIN_SEG], const double (&cw)[QSA_LIN_SEG],
                                             double dxi, double* ws, double (&q)[QSA_LIN_SEG]) {
  double ta = 0.0, tb = 0.0;
#pragma unroll
  for (int k = 0; k < QSA_LIN_SEG; ++k) {
    ta += cw[k] * cs[k] * n[k];
    tb += cw[k] * sn[k] * n[k];
  }
  double a = ta, b = tb;
  lin_block_scan(a, b, ws);
#pragma unroll
  for (int k = 0; k < QSA_LIN_SEG; ++k) {
    a += cw[k] * cs[k] * n[k];
    b += cw[k] * sn[k] * n[k];
    q[k] = dxi * (sn[k] * a - cs[k] * b);
  }
}

// One block per instance b: Gamma_b (per_point = 0) or the longitudinal
// profile Gamma_b(xi_i) = gamma[b][i] (per_point = 1), seed n0[b][nxi];
// outputs n_out[b][m][nxi] and psi_out[b][m][nxi] after out.steps[m] RK4
// steps.
__global__ void __launch_bounds__(QSA_LIN_THREADS) k_linear_model(int nxi, double dxi, double dtau,
                                                                  const double* __restrict__ gamma, int per_point,
                                                                  const double* __restrict__ n0, LinOut out,
                                                                  double* __restrict__ n_out,
                                                                  double* __restrict__ psi_out) {
  __shared__ double ws[32];
  const int b = blockIdx.x, t = threadIdx.x;
  double cs[QSA_LIN_SEG], sn[QSA_LIN_SEG], cw[QSA_LIN_SEG], n[QSA_LIN_SEG], v[QSA_LIN_SEG], g2[QSA_LIN_SEG];
#pragma unroll
  for (int k = 0; k < QSA_LIN_SEG; ++k) {
    const int i = t * QSA_LIN_SEG + k;
    const bool in = i < nxi;
    const double xi = (double)i * dxi;
    cs[k] = cos(xi);
    sn[k] = sin(xi);
    cw[k] = in ? (i == 0 ? 0.5 : 1.0) : 0.0;   // points past the grid carry nothing
    n[k] = in ? n0[(int64_t)b * nxi + i] : 0.0;
    v[k] = 0.0;
    const double gk = per_point ? (in ? gamma[(int64_t)b * nxi + i] : 0.0) : gamma[b];
    g2[k] = gk * gk;
  }
  auto emit = [&](int m) {
    double q[QSA_LIN_SEG];
    lin_volterra(n, cs, sn, cw, dxi, ws, q);
#pragma unroll
    for (int k = 0; k < QSA_LIN_SEG; ++k) {
      const int i = t * QSA_LIN_SEG + k;
      if (i < nxi) {
        const int64_t o = ((int64_t)b * out.n + m) * nxi + i;
        n_out[o] = n[k];
        psi_out[o] = q[k];
      }
    }
  };
  int64_t step = 0;
  for (int m = 0; m < out.n; ++m) {
    for (; step < out.steps[m]; ++step) {
      double an[QSA_LIN_SEG], av[QSA_LIN_SEG], sn_[QSA_LIN_SEG], q[QSA_LIN_SEG];
      // stage 1
      lin_volterra(n, cs, sn, cw, dxi, ws, q);
#pragma unroll
      for (int k = 0; k < QSA_LIN_SEG; ++k) {
        an[k] = v[k];
        av[k] = g2[k] * q[k];
        sn_[k] = n[k] + 0.5 * dtau * v[k];
      }
      double vs[QSA_LIN_SEG];
#pragma unroll
      for (int k = 0; k < QSA_LIN_SEG; ++k) vs[k] = v[k] + 0.5 * dtau * (g2[k] * q[k]);
      // stage 2
      lin_volterra(sn_, cs, sn, cw, dxi, ws, q);
      double k2n[QSA_LIN_SEG], k2v[QSA_LIN_SEG];
#pragma unroll
      for (int k = 0; k < QSA_LIN_SEG; ++k) {
        k2n[k] = vs[k];
        k2v[k] = g2[k] * q[k];
        an[k] += 2.0 * k2n[k];
        av[k] += 2.0 * k2v[k];
        sn_[k] = n[k] + 0.5 * dtau * k2n[k];
        vs[k] = v[k] + 0.5 * dtau * k2v[k];
      }
      // stage 3
      lin_volterra(sn_, cs, sn, cw, dxi, ws, q);
#pragma unroll
      for (int k = 0; k < QSA_LIN_SEG; ++k) {
        const double k3n = vs[k], k3v = g2[k] * q[k];
        an[k] += 2.0 * k3n;
        av[k] += 2.0 * k3v;
        sn_[k] = n[k] + dtau * k3n;
        vs[k] = v[k] + dtau * k3v;
      }
      // stage 4
      lin_volterra(sn_, cs, sn, cw, dxi, ws, q);
#pragma unroll
      for (int k = 0; k < QSA_LIN_SEG; ++k) {
        an[k] += vs[k];
        av[k] += g2[k] * q[k];
        n[k] += dtau / 6.0 * an[k];
        v[k] += dtau / 6.0 * av[k];
      }
    }
    emit(m);
  }
}

}  // namespace qsa
