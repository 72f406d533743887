// Device-side building blocks of the QSA slice sweep for gfx950 (wave64):
// complex arithmetic, in-LDS Stockham FFT passes, the linear (cloud-in-cell)
// particle shape on the periodic transverse grid, and atomics.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qsa {

template <typename R>
struct C2 {
  R x, y;
};

template <typename R>
__device__ __forceinline__ C2<R> cadd(C2<R> a, C2<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ C2<R> csub(C2<R> a, C2<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ C2<R> cmul(C2<R> a, C2<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R>
__device__ __forceinline__ C2<R> cconj(C2<R> a) { return {a.x, -a.y}; }
template <typename R>
__device__ __forceinline__ C2<R> cscale(C2<R> a, R s) { return {a.x * s, a.y * s}; }
// multiply by i*k (k real)
template <typename R>
__device__ __forceinline__ C2<R> cmul_ik(C2<R> a, R k) { return {-a.y * k, a.x * k}; }

// Grid geometry passed by value to every kernel.
template <typename R>
struct Geo {
  int nx, ny, nxi, nxh, nperp;  // nxh = nx/2 + 1 (half spectrum along x)
  int lgx, lgy;                 // log2 nx, log2 ny
  R dx, dy, dxi;
  R inv_dx, inv_dy;
  R lx, ly, inv_lx, inv_ly;
  // the same in float64, for the plasma positions (float64 in either
  // precision: a float32 position in a box of a few c/omega_p resolves only
  // about 1e-6, coarser than a slice's displacement allows)
  double inv_dxd, inv_dyd, lxd, lyd, inv_lxd, inv_lyd;
  R b0z;                        // uniform external B_z (guide field), 0 if none
};

// Wrap an integer cell index into [0, n) for n a power of two (the library
// accepts no other grid sizes): the two's-complement mask is the periodic
// wrap for negative indices too, and any input (also from a non-finite
// coordinate) lands inside the grid, so no access can leave the array.  (An
// integer remainder by a runtime n costs a long division sequence, several
// of them per particle.)
__device__ __forceinline__ int wrap_index(int v, int n) { return v & (n - 1); }

// Four nodes and weights of the linear shape at (x, y).
template <typename R>
struct Stencil {
  int n00, n10, n01, n11;
  R w00, w10, w01, w11;
};

// (x, y) of type P: the working precision R (beam particles) or float64
// (plasma particles); the cell offsets are taken in P, the weights in R.
template <typename R, typename P>
__device__ __forceinline__ Stencil<R> stencil2(const Geo<R>& g, P x, P y) {
  P gx = x * (P)g.inv_dxd;
  P gy = y * (P)g.inv_dyd;
  P fx0 = floor(gx);
  P fy0 = floor(gy);
  R fx = (R)(gx - fx0);
  R fy = (R)(gy - fy0);
  // coordinates are bounded (a few box lengths at most) for finite input;
  // the clamp keeps the float->int conversion defined for any input
  P cx = fmin(fmax(fx0, P(-1.0e9)), P(1.0e9));
  P cy = fmin(fmax(fy0, P(-1.0e9)), P(1.0e9));
  int i0 = wrap_index((int)cx, g.nx);
  int l0 = wrap_index((int)cy, g.ny);
  int i1 = (i0 + 1 == g.nx) ? 0 : i0 + 1;
  int l1 = (l0 + 1 == g.ny) ? 0 : l0 + 1;
  Stencil<R> s;
  s.n00 = l0 * g.nx + i0;
  s.n10 = l0 * g.nx + i1;
  s.n01 = l1 * g.nx + i0;
  s.n11 = l1 * g.nx + i1;
  R ax = R(1) - fx, ay = R(1) - fy;
  s.w00 = ax * ay;
  s.w10 = fx * ay;
  s.w01 = ax * fy;
  s.w11 = fx * fy;
  return s;
}

// Cell (i0, l0), wrapped into the grid, and the fractional offsets of (x, y).
template <typename R, typename P>
__device__ __forceinline__ void cell2(const Geo<R>& g, P x, P y, int& i0, int& l0, R& fx, R& fy) {
  P gx = x * (P)g.inv_dxd;
  P gy = y * (P)g.inv_dyd;
  P fx0 = floor(gx);
  P fy0 = floor(gy);
  fx = (R)(gx - fx0);
  fy = (R)(gy - fy0);
  P cx = fmin(fmax(fx0, P(-1.0e9)), P(1.0e9));
  P cy = fmin(fmax(fy0, P(-1.0e9)), P(1.0e9));
  i0 = wrap_index((int)cx, g.nx);
  l0 = wrap_index((int)cy, g.ny);
}

// Logical block index for a launch of nb blocks, so that the blocks one XCD
// runs (hardware dispatch is round-robin over the 8 XCDs) are consecutive:
// neighbouring particle chunks then share that XCD's L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int per = nb >> 3, rem = nb & 7;
  const int x = b & 7, k = b >> 3;
  return x * per + (x < rem ? x : rem) + k;
}

template <typename R>
__device__ __forceinline__ R gather(const R* __restrict__ f, const Stencil<R>& s) {
  return f[s.n00] * s.w00 + f[s.n10] * s.w10 + f[s.n01] * s.w01 + f[s.n11] * s.w11;
}

__device__ __forceinline__ void atomic_add(double* p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add(float* p, float v) { unsafeAtomicAdd(p, v); }

template <typename R>
__device__ __forceinline__ void scatter(R* __restrict__ f, const Stencil<R>& s, R q) {
  atomic_add(f + s.n00, q * s.w00);
  atomic_add(f + s.n10, q * s.w10);
  atomic_add(f + s.n01, q * s.w01);
  atomic_add(f + s.n11, q * s.w11);
}

// ---------------------------------------------------------------------------
// Block-level deposit through an LDS tile.  Each thread brings at most one
// particle (live) with cell (i0, l0), offsets (fx, fy) and NC values.  The
// block reduces the bounding box of its cells; when the box (plus the +1
// nodes) fits the tile, the particles accumulate there with LDS atomics and
// the block then adds the non-zero tile nodes to the grids with one global
// atomic each.  Otherwise every particle adds its four nodes to the grids
// directly.  Every thread of the block must call this (it has barriers).
// ---------------------------------------------------------------------------
template <typename R, int NC>
struct TileCap {
  static constexpr int BYTES = 32768;
  static constexpr int NODES = BYTES / (NC * (int)sizeof(R));
};

template <typename R, int NC>
__device__ __forceinline__ void block_deposit(const Geo<R>& g, bool live, int i0, int l0, R fx, R fy,
                                              const R (&v)[NC], R* const (&dst)[NC], R* tile,
                                              int* bb) {
  constexpr int CAP = TileCap<R, NC>::NODES;
  const int tid = threadIdx.x, nt = blockDim.x;
  if (tid == 0) {
    bb[0] = 0x7fffffff;
    bb[1] = 0x7fffffff;
    bb[2] = -1;
    bb[3] = -1;
  }
  for (int t = tid; t < NC * CAP; t += nt) tile[t] = R(0);
  __syncthreads();
  if (live) {
    atomicMin(&bb[0], l0);
    atomicMin(&bb[1], i0);
    atomicMax(&bb[2], l0);
    atomicMax(&bb[3], i0);
  }
  __syncthreads();
  const int lmin = bb[0], imin = bb[1];
  const bool any = bb[2] >= 0;
  const int nl = any ? bb[2] - lmin + 2 : 0;
  const int ni = any ? bb[3] - imin + 2 : 0;
  const bool fits = any && nl * ni <= CAP;
  if (live) {
    const R ax = R(1) - fx, ay = R(1) - fy;
    const R w[4] = {ax * ay, fx * ay, ax * fy, fx * fy};
    if (fits) {
      const int t00 = (l0 - lmin) * ni + (i0 - imin);
      const int off[4] = {t00, t00 + 1, t00 + ni, t00 + ni + 1};
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int q = 0; q < 4; ++q) atomicAdd(&tile[c * CAP + off[q]], v[c] * w[q]);
    } else {
      const int i1 = (i0 + 1 == g.nx) ? 0 : i0 + 1;
      const int l1 = (l0 + 1 == g.ny) ? 0 : l0 + 1;
      const int nodes[4] = {l0 * g.nx + i0, l0 * g.nx + i1, l1 * g.nx + i0, l1 * g.nx + i1};
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int q = 0; q < 4; ++q) atomic_add(dst[c] + nodes[q], v[c] * w[q]);
    }
  }
  __syncthreads();
  if (fits) {
    for (int t = tid; t < nl * ni; t += nt) {
      const int ll = t / ni, ii = t - ll * ni;
      int lg = lmin + ll;
      lg -= (lg >= g.ny) ? g.ny : 0;
      int ig = imin + ii;
      ig -= (ig >= g.nx) ? g.nx : 0;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const R val = tile[c * CAP + t];
        if (val != R(0)) atomic_add(dst[c] + lg * g.nx + ig, val);
      }
    }
  }
}

// Periodic wrap into [0, L); a value that rounds to L maps to 0.
template <typename R>
__device__ __forceinline__ R wrap_pos(R x, R L, R invL) {
  R r = x - L * floor(x * invL);
  return (r >= L) ? R(0) : r;
}

// ---------------------------------------------------------------------------
// Stockham autosort FFT in LDS.  A transform of length n (power of two) is
// worked by tpt threads (thread t in [0, tpt)); passes are radix 8 with one
// final radix-4 or radix-2 pass when log2 n is not a multiple of 3.  tw[m] = exp(-2 pi i m/n); INV uses
// the conjugate twiddles and is unnormalized.  Every pass ends with a
// workgroup barrier, so all threads of the workgroup must call with the same
// n (threads without a transform still take part).
//
// The input and the result are in natural order; the passes in between
// write a padded layout, one spare entry after every 8.  An early pass
// stores its 8 outputs at a stride of 8 (ns = 1) or in runs of 8 that are
// 64 entries apart (ns = 8): unpadded, a wavefront's stores then fall in a
// quarter of the LDS banks (16-way conflicts for 8-byte entries, 32-way for
// 16-byte ones); with a spare entry per 8 they spread over all banks.
// ---------------------------------------------------------------------------

// Number of passes fft_lds takes for log2 n = lg (its result sits in the
// input buffer when this is even).
__host__ __device__ __forceinline__ int fft_passes(int lg) { return lg / 3 + (lg % 3 != 0); }

// Entries an FFT work buffer of length n must hold (both of the two
// buffers a transform alternates between).
__host__ __device__ __forceinline__ int fft_cap(int n) { return n + (n >> 3); }

// Position of entry i in the padded (P) or natural layout.
template <bool P>
__device__ __forceinline__ int fpad(int i) { return P ? i + (i >> 3) : i; }

template <typename R, bool INV, bool PI>
__device__ __forceinline__ void fft_pass4(const C2<R>* in, C2<R>* out, int n, int ns, int t,
                                          int tpt, const C2<R>* __restrict__ tw) {
  const int q = n >> 2;
  const int stride = n / (4 * ns);
  for (int jj = t; jj < q; jj += tpt) {
    const int k = jj & (ns - 1);
    C2<R> a0 = in[fpad<PI>(jj)], a1 = in[fpad<PI>(jj + q)], a2 = in[fpad<PI>(jj + 2 * q)],
          a3 = in[fpad<PI>(jj + 3 * q)];
    if (ns > 1) {
      C2<R> w1 = tw[k * stride], w2 = tw[2 * k * stride], w3 = tw[3 * k * stride];
      if (INV) {
        w1 = cconj(w1);
        w2 = cconj(w2);
        w3 = cconj(w3);
      }
      a1 = cmul(a1, w1);
      a2 = cmul(a2, w2);
      a3 = cmul(a3, w3);
    }
    C2<R> t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), d = csub(a1, a3);
    // t3 = -i d (forward) or +i d (inverse)
    C2<R> t3 = INV ? C2<R>{-d.y, d.x} : C2<R>{d.y, -d.x};
    const int o = 4 * (jj - k) + k;
    out[o] = cadd(t0, t2);
    out[o + ns] = cadd(t1, t3);
    out[o + 2 * ns] = csub(t0, t2);
    out[o + 3 * ns] = csub(t1, t3);
  }
}

template <typename R, bool INV, bool PI>
__device__ __forceinline__ void fft_pass2(const C2<R>* in, C2<R>* out, int n, int ns, int t,
                                          int tpt, const C2<R>* __restrict__ tw) {
  const int h = n >> 1;
  const int stride = n / (2 * ns);
  for (int jj = t; jj < h; jj += tpt) {
    const int k = jj & (ns - 1);
    C2<R> a = in[fpad<PI>(jj)], b = in[fpad<PI>(jj + h)];
    if (ns > 1) {
      C2<R> w = tw[k * stride];
      if (INV) w = cconj(w);
      b = cmul(b, w);
    }
    const int o = 2 * (jj - k) + k;
    out[o] = cadd(a, b);
    out[o + ns] = csub(a, b);
  }
}

// Multiply by the 8th roots of unity W^q, W = exp(-+ 2 pi i/8) (INV: +).
template <typename R, bool INV>
__device__ __forceinline__ C2<R> mul_w8(C2<R> o, int q) {
  const R c = R(0.70710678118654752440084436210484903928);
  switch (q) {
    case 1: return INV ? C2<R>{c * (o.x - o.y), c * (o.x + o.y)} : C2<R>{c * (o.x + o.y), c * (o.y - o.x)};
    case 2: return INV ? C2<R>{-o.y, o.x} : C2<R>{o.y, -o.x};
    case 3: return INV ? C2<R>{-c * (o.x + o.y), c * (o.x - o.y)} : C2<R>{c * (o.y - o.x), -c * (o.x + o.y)};
    default: return o;
  }
}

// In-register 4-point DFT of (x0, x1, x2, x3) (unnormalized; INV: +i).
template <typename R, bool INV>
__device__ __forceinline__ void dft4(C2<R>& x0, C2<R>& x1, C2<R>& x2, C2<R>& x3) {
  const C2<R> t0 = cadd(x0, x2), t1 = csub(x0, x2), t2 = cadd(x1, x3), d = csub(x1, x3);
  const C2<R> t3 = INV ? C2<R>{-d.y, d.x} : C2<R>{d.y, -d.x};
  x0 = cadd(t0, t2);
  x1 = cadd(t1, t3);
  x2 = csub(t0, t2);
  x3 = csub(t1, t3);
}

// In-register 8-point DFT: the 4-point DFTs of the even and odd samples,
// combined with the twiddles W^q.
template <typename R, bool INV>
__device__ __forceinline__ void dft8(C2<R> (&a)[8]) {
  C2<R> e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
  C2<R> o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
  dft4<R, INV>(e0, e1, e2, e3);
  dft4<R, INV>(o0, o1, o2, o3);
  const C2<R> e[4] = {e0, e1, e2, e3};
  const C2<R> o[4] = {o0, mul_w8<R, INV>(o1, 1), mul_w8<R, INV>(o2, 2), mul_w8<R, INV>(o3, 3)};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    a[q] = cadd(e[q], o[q]);
    a[q + 4] = csub(e[q], o[q]);
  }
}

// Radix-8 Stockham pass: n/8 butterflies, thread t of tpt takes butterflies
// t, t + tpt, ...; ns = the product of the earlier passes' radices.  PI, PO:
// the input, output is in the padded layout.
template <typename R, bool INV, bool PI, bool PO>
__device__ __forceinline__ void fft_pass8(const C2<R>* in, C2<R>* out, int n, int ns, int t, int tpt,
                                          const C2<R>* __restrict__ tw) {
  const int q = n >> 3;
  const int stride = n / (8 * ns);
  for (int jj = t; jj < q; jj += tpt) {
    const int k = jj & (ns - 1);
    C2<R> a[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) a[m] = in[fpad<PI>(jj + m * q)];
    if (ns > 1) {
#pragma unroll
      for (int m = 1; m < 8; ++m) {
        C2<R> w = tw[m * k * stride];
        if (INV) w = cconj(w);
        a[m] = cmul(a[m], w);
      }
    }
    dft8<R, INV>(a);
    const int o = 8 * (jj - k) + k;
#pragma unroll
    for (int m = 0; m < 8; ++m) out[fpad<PO>(o + m * ns)] = a[m];
  }
}

// Returns the buffer (a or b) that holds the result, in natural order; each
// of a and b holds fft_cap(n) entries.  Radix-8 passes while
// at least three factors of two remain, then one radix-4 or radix-2 pass.
template <typename R, bool INV>
__device__ __forceinline__ C2<R>* fft_lds(C2<R>* a, C2<R>* b, int n, int lg, int t, int tpt,
                                          const C2<R>* __restrict__ tw) {
  const int np = fft_passes(lg);
  int ns = 1;
  int s = lg;
  int p = 0;
  while (s >= 3) {
    const bool pi = p > 0, po = p + 1 < np;
    if (pi && po)
      fft_pass8<R, INV, true, true>(a, b, n, ns, t, tpt, tw);
    else if (pi)
      fft_pass8<R, INV, true, false>(a, b, n, ns, t, tpt, tw);
    else if (po)
      fft_pass8<R, INV, false, true>(a, b, n, ns, t, tpt, tw);
    else
      fft_pass8<R, INV, false, false>(a, b, n, ns, t, tpt, tw);
    ++p;
    __syncthreads();
    C2<R>* tmp = a;
    a = b;
    b = tmp;
    ns <<= 3;
    s -= 3;
  }
  if (s == 2) {
    if (p > 0)
      fft_pass4<R, INV, true>(a, b, n, ns, t, tpt, tw);
    else
      fft_pass4<R, INV, false>(a, b, n, ns, t, tpt, tw);
    __syncthreads();
    C2<R>* tmp = a;
    a = b;
    b = tmp;
  } else if (s == 1) {
    if (p > 0)
      fft_pass2<R, INV, true>(a, b, n, ns, t, tpt, tw);
    else
      fft_pass2<R, INV, false>(a, b, n, ns, t, tpt, tw);
    __syncthreads();
    C2<R>* tmp = a;
    a = b;
    b = tmp;
  }
  return a;
}

// Threads per row transform of length n (two real rows packed as one
// complex row): n/4, so that the loads of the rows' inputs (a sum of partial
// rows and sources per value) have threads enough to be in flight together;
// the radix-8 passes use half of them.
__host__ __device__ __forceinline__ int row_tpt(int n) { return n >= 4 ? n >> 2 : 1; }

}  // namespace qsa
