// Host driver of the adjoint (qsa_adjoint_sweep); included by qsa.hip after
// the context and the forward engine are defined.
//
// Order of work for n beam steps:
//   forward  t = 0..n:  sources of beam(t); sweep(t), taping its fields and
//                       B_perp iterates, with plasma checkpoints every
//                       QSA_ADJ_CKPT slices; beam(t+1) = push (t < n);
//   loss              = 1/2 sum (B_x^2 + B_y^2) dV of sweep(n);
//   reverse  t = n..0:  sweep(t)^T, segment by segment (recompute the
//                       segment's plasma states from its checkpoint with one
//                       launch, then its slices in reverse); sources^T into
//                       the beam adjoint; push^T of step t - 1 into the beam
//                       adjoint and the field adjoint of sweep(t - 1);
//   gradient          = per bin, sum of (weight adjoint x loaded weight).
// A slice takes 9 + 4 n_corr launches forward and as many in reverse: grid
// initialisations, copies and the transverse-mean leapfrog are side jobs of
// launches that do not touch their data, input combinations and extra
// destinations fold into the spectral operators, the J_perp history and the
// field adjoints live in place (ping-pong by slice parity).

namespace {

template <typename R>
struct Adj {
  qsa_ctx* c;
  const qsa_params& p;
  const AdjLayout& A;
  Geo<R> g;
  int K;
  int64_t nperp, plane, np;
  double h;
  Side<R> none;
  bool overflow = false;
  int tile_small = 40960;    // LDS of a scatter tile (few channels)
  int tile_big = 40960;      // of the plasma transposes (12-13 channels), raised in run()

  Adj(qsa_ctx* ctx, const AdjLayout& lay) : c(ctx), p(ctx->p), A(lay) {
    g = Engine<R>::geo(p);
    K = std::max(p.n_corr, 0);
    nperp = g.nperp;
    plane = (int64_t)p.nxi * nperp;
    np = p.n_plasma;
    h = p.dxi;
    std::memset(&none, 0, sizeof(none));
  }

  hipStream_t st() const { return c->stream; }
  int thr_n = 0;   // slices enqueued, for the enqueue throttle
  qsa_status throttle() { return Engine<R>::throttle(c, st(), thr_n++); }
  R* grid(int k) const { return c->at<R>(A.grids) + (int64_t)k * nperp; }
  double* sc() const { return c->at<double>(A.sc); }
  double* scf(int par) const { return sc() + 8 * par; }        // forward leapfrog slot of a slice parity
  double* scr(int par) const { return sc() + 16 + 8 * par; }   // reverse
  double* jzsum() const { return c->at<double>(A.sums); }      // per slice: sum of the beam's J_z
  double* ezsum() const { return c->at<double>(A.sums) + p.nxi; }   // per slice: sum of the E_z adjoint
  double* jzpart() const { return c->at<double>(A.part); }              // per plasma block: sum of J_z deposits
  double* psipart() const { return c->at<double>(A.part) + blocks(np); }   // per row: sum of the psi adjoint
  R* fields(int t) const { return c->at<R>(A.fields) + (int64_t)t * N_STORED * plane; }
  R* field(int t, int f, int j) const { return fields(t) + (int64_t)f * plane + (int64_t)j * nperp; }
  R* fbar(int f, int j) const { return c->at<R>(A.fb) + (int64_t)f * plane + (int64_t)j * nperp; }
  R* src(int k, int j) const { return c->at<R>(A.src) + (int64_t)k * plane + (int64_t)j * nperp; }
  R* srcb(int k, int j) const { return c->at<R>(A.srcb) + (int64_t)k * plane + (int64_t)j * nperp; }
  R* biter_base(int t) const { return c->at<R>(A.biter) + (int64_t)t * std::max(K, 1) * 2 * plane; }
  // B_perp iterate k of slice j (k = K: the slice's field)
  R* bk(int t, int k, int comp, int j) const {
    if (k == K) return field(t, comp ? F_BY : F_BX, j);
    return biter_base(t) + ((int64_t)k * 2 + comp) * plane + (int64_t)j * nperp;
  }
  R* bstate(int t, int s, int k) const {
    const size_t cap = (size_t)p.beam_capacity[s];
    const size_t rs = sizeof(R);
    return reinterpret_cast<R*>(c->ws + A.beam[s] + (size_t)t * A.state[s] + (size_t)k * align_up(cap * rs));
  }
  double* bxi(int t, int s) const {
    const size_t cap = (size_t)p.beam_capacity[s];
    return reinterpret_cast<double*>(c->ws + A.beam[s] + (size_t)t * A.state[s] + 6 * align_up(cap * sizeof(R)));
  }
  R* yarr(size_t base, int i, int comp) const {   // [i][4][np]
    return c->at<R>(base) + ((int64_t)i * 4 + comp) * np;
  }
  R* ck(int t, int cidx, int comp) const {
    return reinterpret_cast<R*>(c->ws + A.ck + ((size_t)t * A.nseg + cidx) * A.ck_bytes) + (int64_t)comp * np;
  }

  static int blocks(int64_t n) { return (int)std::max<int64_t>(1, (n + 255) / 256); }

  // ---- builders ----------------------------------------------------------
  struct SideB {
    Side<R> s;
    Adj* owner;
    explicit SideB(Adj* o) : owner(o) {
      std::memset(&s, 0, sizeof(s));
      s.len = o->nperp;
    }
    SideB& lin(R* out, int add, std::initializer_list<std::pair<const R*, double>> terms,
               const double* sp = nullptr, double spc = 0.0) {
      if (s.nl >= SIDE_LIN || terms.size() > 3) {
        owner->overflow = true;
        return *this;
      }
      Lin<R>& a = s.op[s.nl++];
      a.out = out;
      a.add = add;
      a.nt = 0;
      a.c0 = 0.0;
      a.sp = sp;
      a.spc = spc;
      for (const auto& t : terms) {
        a.in[a.nt] = t.first;
        a.c[a.nt] = t.second;
        ++a.nt;
      }
      return *this;
    }
    SideB& scalar(int kind, double* x, double* y, const double* z, const double* part, int npart, double v0,
                  double v1) {
      if (s.ns >= 2) {
        owner->overflow = true;
        return *this;
      }
      ScalarJob& j = s.sj[s.ns++];
      j.kind = kind;
      j.a = x;
      j.b = y;
      j.c = z;
      j.part = part;
      j.npart = npart;
      j.v0 = v0;
      j.v1 = v1;
      return *this;
    }
  };

  struct SpecB {
    SpecOp<R> op;
    Adj* owner;
    SpecB(Adj* o, int conj) : owner(o) {
      std::memset(&op, 0, sizeof(op));
      op.conj = conj;
    }
    int input(std::initializer_list<std::pair<const R*, double>> terms) {
      if (op.ni >= SPEC_IN || terms.size() > (size_t)SPEC_COMB) {
        owner->overflow = true;
        return 0;
      }
      const int f = op.ni++;
      for (const auto& t : terms) {
        const int q = op.nin[f]++;
        op.in[f][q] = t.first;
        op.inc[f][q] = t.second;
      }
      return f;
    }
    int output() {
      if (op.no >= SPEC_OUT) {
        owner->overflow = true;
        return 0;
      }
      return op.no++;
    }
    void term(int o, int kind, int f, double coef) {
      if (op.nterm[o] >= SPEC_TERMS) {
        owner->overflow = true;
        return;
      }
      const int q = op.nterm[o]++;
      op.kind[o][q] = kind;
      op.src[o][q] = f;
      op.coef[o][q] = coef;
    }
    void dest(int o, R* d, double coef, int add) {
      if (op.nd[o] >= SPEC_COMB) {
        owner->overflow = true;
        return;
      }
      const int q = op.nd[o]++;
      op.dst[o][q] = d;
      op.dc[o][q] = coef;
      op.dadd[o][q] = add;
    }
  };

  qsa_status spec(SpecB& b, const Side<R>& s_rows, const Side<R>& s_cols, const Side<R>& s_inv) {
    if (overflow) return fail(c, QSA_E_INVALID, "adjoint: operator description overflow");
    SpecOp<R>& op = b.op;
    op.ktab = c->at<double>(A.ktab);
    op.work = c->at<C2<R>>(A.work);
    const int W = std::max(op.ni, op.no);
    const size_t rows_lds = ((size_t)g.nx + 2 * (size_t)fft_cap(g.nx)) * sizeof(C2<R>);
    const size_t cols_lds = ((size_t)g.ny + 2 * (size_t)W * fft_cap(g.ny)) * sizeof(C2<R>);
    hipLaunchKernelGGL(k_spec_rows_fwd<R>, dim3(g.ny, op.ni), dim3(64), rows_lds, st(), g, op,
                       (const C2<R>*)c->at<C2<R>>(c->L.twx), s_rows);
    hipLaunchKernelGGL(k_spec_cols<R>, dim3(g.nx / 2 + 1), dim3(64 * W), cols_lds, st(), g, op,
                       (const C2<R>*)c->at<C2<R>>(c->L.twy), s_cols);
    hipLaunchKernelGGL(k_spec_rows_inv<R>, dim3(g.ny, op.no), dim3(64), rows_lds, st(), g, op,
                       (const C2<R>*)c->at<C2<R>>(c->L.twx), s_inv);
    HIP_OK(hipGetLastError());
    return QSA_OK;
  }

  qsa_status lin(R* out, int add, std::initializer_list<std::pair<const R*, double>> terms, int64_t n) {
    SideB b(this);
    b.lin(out, add, terms);
    if (overflow) return fail(c, QSA_E_INVALID, "adjoint: operator description overflow");
    hipLaunchKernelGGL(k_lin<R>, dim3((unsigned)std::min<int64_t>(4096, blocks(n))), dim3(256), 0, st(),
                       b.s.op[0], n);
    HIP_OK(hipGetLastError());
    return QSA_OK;
  }

  // lds: the launch's dynamic LDS (a.tile_bytes for the scatter kernels)
  template <typename Kern>
  qsa_status plasma(Kern kern, const AdjPlasma<R>& a, const Side<R>& s, int lds) {
    if (overflow) return fail(c, QSA_E_INVALID, "adjoint: operator description overflow");
    hipLaunchKernelGGL(kern, dim3(blocks(np)), dim3(256), (size_t)lds, st(), a, s);
    HIP_OK(hipGetLastError());
    return QSA_OK;
  }

  AdjPlasma<R> plasma_args() const {
    AdjPlasma<R> a;
    std::memset(&a, 0, sizeof(a));
    a.g = g;
    a.np = (int)np;
    a.nw = -p.plasma_w / (p.dx * p.dy);
    a.h = h;
    a.tile_bytes = tile_small;
    a.err = c->at<int>(c->L.err);
    return a;
  }

  // the fields a plasma particle sees at slice j: psi, dxpsi, dypsi, B_z from
  // the tape, B_perp given; F^{j-1} from the tape (zeros before slice 0)
  void six(int t, int j, const R* bx, const R* by, Six<R>& F) const {
    const int fm[6] = {F_PSI, F_DXPSI, F_DYPSI, F_BX, F_BY, F_BZ};
    for (int m = 0; m < 6; ++m) {
      F.a[m] = field(t, fm[m], j);
      F.m1[m] = (j >= 1) ? field(t, fm[m], j - 1) : grid(AG_ZERO);
    }
    F.a[3] = bx;
    F.a[4] = by;
  }

  // ---- forward slice -------------------------------------------------------
  // Yin -> Yout at slice j of sweep t.  On entry AG_S holds the beam's
  // rho - J_z of slice j.
  qsa_status fwd_slice(int t, int j, R* const* Yin, R* const* Yout) {
    qsa_status st0;
    const int par = j & 1;
    const R* zero = grid(AG_ZERO);
    R* J[3] = {grid(AG_JF0 + 3 * par), grid(AG_JF0 + 3 * par + 1), grid(AG_JF0 + 3 * par + 2)};
    const R* jm1x = (j >= 1) ? grid(AG_JF0 + 3 * (1 - par)) : zero;
    const R* jm1y = (j >= 1) ? grid(AG_JF0 + 3 * (1 - par) + 1) : zero;
    double* si = scf(par);
    double* so = scf(1 - par);
    const bool last = j + 1 >= p.nxi;
    AdjPlasma<R> a = plasma_args();
    for (int k = 0; k < 4; ++k) a.Y[k] = Yin[k];
    // psi stage
    {
      SideB sd(this);
      sd.lin(J[0], 0, {{src(1, j), 1.0}}).lin(J[1], 0, {{src(2, j), 1.0}}).lin(J[2], 0, {{src(3, j), 1.0}});
      if (overflow) return fail(c, QSA_E_INVALID, "adjoint: operator description overflow");
      hipLaunchKernelGGL(k_af_dep_s<R>, dim3(blocks(np)), dim3(256), (size_t)a.tile_bytes, st(), a, grid(AG_S),
                         sd.s);
    }
    {
      SpecB b(this, 0);
      const int f = b.input({{grid(AG_S), 1.0}});
      const int o0 = b.output(), o1 = b.output(), o2 = b.output();
      b.term(o0, SK_INVK2, f, 1.0);
      b.term(o1, SK_IKX_K2, f, 1.0);
      b.term(o2, SK_IKY_K2, f, 1.0);
      b.dest(o0, field(t, F_PSI, j), 1.0, 0);
      b.dest(o1, field(t, F_DXPSI, j), 1.0, 0);
      b.dest(o2, field(t, F_DYPSI, j), 1.0, 0);
      b.op.mean[o0] = si + 1;
      // B_0 = 2 B^{j-1} - B^{j-2}
      const R* bm1x = (j >= 1) ? field(t, F_BX, j - 1) : zero;
      const R* bm1y = (j >= 1) ? field(t, F_BY, j - 1) : zero;
      const R* bm2x = (j >= 2) ? field(t, F_BX, j - 2) : zero;
      const R* bm2y = (j >= 2) ? field(t, F_BY, j - 2) : zero;
      SideB sr(this);
      sr.lin(bk(t, 0, 0, j), 0, {{bm1x, 2.0}, {bm2x, -1.0}}).lin(bk(t, 0, 1, j), 0, {{bm1y, 2.0}, {bm2y, -1.0}});
      if ((st0 = spec(b, sr.s, none, none)) != QSA_OK) return st0;
    }
    // J stage
    {
      a.psi = field(t, F_PSI, j);
      a.Jx = J[0];
      a.Jy = J[1];
      a.Jz = J[2];
      a.qzsum = jzpart();
      SideB sd(this);
      if (K > 0) {
        const R* pm1 = (j >= 1) ? field(t, F_PSI, j - 1) : zero;
        const R* pm2 = (j >= 2) ? field(t, F_PSI, j - 2) : zero;
        sd.lin(grid(AG_PSIT), 0, {{field(t, F_PSI, j), 3.0}, {pm1, -3.0}, {pm2, 1.0}});
        sd.lin(grid(AG_JT), 0, {{last ? zero : src(1, j + 1), 1.0}});
        sd.lin(grid(AG_JT + 1), 0, {{last ? zero : src(2, j + 1), 1.0}});
      }
      if ((st0 = plasma(k_af_dep_j<R>, a, sd.s, a.tile_bytes)) != QSA_OK) return st0;
      a.qzsum = nullptr;
    }
    {
      SpecB b(this, 0);
      const int fx = b.input({{J[0], 1.0}}), fy = b.input({{J[1], 1.0}});
      const int o0 = b.output(), o1 = b.output();
      b.term(o0, SK_IKY_K2, fx, -1.0);
      b.term(o0, SK_IKX_K2, fy, 1.0);
      b.term(o1, SK_IKX_K2, fx, -1.0);
      b.term(o1, SK_IKY_K2, fy, -1.0);
      b.dest(o0, field(t, F_BZ, j), 1.0, 0);
      b.dest(o1, field(t, F_EZ, j), 1.0, 0);
      b.op.mean[o1] = si + 3;
      SideB sr(this);
      sr.scalar(SJ_ODE_FWD, si, so, jzsum() + j, jzpart(), blocks(np), h, (double)nperp);
      if ((st0 = spec(b, sr.s, none, none)) != QSA_OK) return st0;
    }
    // B_perp predictor-corrector
    const double i2h = 1.0 / (2.0 * h);
    for (int k = 0; k < K; ++k) {
      AdjPlasma<R> b = a;
      six(t, j, bk(t, k, 0, j), bk(t, k, 1, j), b.F);
      b.psi = grid(AG_PSIT);
      b.Jx = grid(AG_JT);
      b.Jy = grid(AG_JT + 1);
      b.Jz = nullptr;
      if ((st0 = plasma(k_af_pred<R>, b, none, b.tile_bytes)) != QSA_OK) return st0;
      SpecB s(this, 0);
      const int fz = s.input({{J[2], 1.0}});
      const int fx = s.input({{grid(AG_JT), i2h}, {jm1x, -i2h}});
      const int fy = s.input({{grid(AG_JT + 1), i2h}, {jm1y, -i2h}});
      const int bx = s.input({{bk(t, k, 0, j), 1.0}});
      const int by = s.input({{bk(t, k, 1, j), 1.0}});
      const int o0 = s.output(), o1 = s.output();
      s.term(o0, SK_IKY_DEN, fz, -1.0);
      s.term(o0, SK_DEN, fy, -1.0);
      s.term(o0, SK_DEN, bx, -p.kappa2);
      s.term(o1, SK_IKX_DEN, fz, 1.0);
      s.term(o1, SK_DEN, fx, 1.0);
      s.term(o1, SK_DEN, by, -p.kappa2);
      s.dest(o0, bk(t, k + 1, 0, j), 1.0, 0);
      s.dest(o1, bk(t, k + 1, 1, j), 1.0, 0);
      SideB sc2(this);
      if (k + 1 < K) {
        sc2.lin(grid(AG_JT), 0, {{last ? zero : src(1, j + 1), 1.0}});
        sc2.lin(grid(AG_JT + 1), 0, {{last ? zero : src(2, j + 1), 1.0}});
      }
      if ((st0 = spec(s, none, sc2.s, none)) != QSA_OK) return st0;
    }
    // final advance; the next slice's rho - J_z source
    {
      AdjPlasma<R> b = a;
      six(t, j, field(t, F_BX, j), field(t, F_BY, j), b.F);
      for (int k = 0; k < 4; ++k) b.Yn[k] = Yout[k];
      SideB sd(this);
      if (!last) sd.lin(grid(AG_S), 0, {{src(0, j + 1), 1.0}});
      if ((st0 = plasma(k_af_final<R>, b, sd.s, 0)) != QSA_OK) return st0;
    }
    return QSA_OK;
  }

  qsa_status fwd_sweep(int t) {
    qsa_status st0;
    R* Ya[4];
    R* Yb2[4];
    for (int k = 0; k < 4; ++k) {
      Ya[k] = yarr(A.Y[0], 0, k);
      Yb2[k] = yarr(A.Y[1], 0, k);
      if (k >= 2 || sizeof(R) == 8) {
        HIP_OK(hipMemcpyAsync(Ya[k], c->ws + c->L.tmpl[k], np * sizeof(R), hipMemcpyDeviceToDevice, st()));
      } else {
        // the template keeps positions in float64
        hipLaunchKernelGGL(k_from_f64<R>, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st(),
                           (const double*)(c->ws + c->L.tmpl[k]), Ya[k], (int64_t)np);
      }
    }
    hipLaunchKernelGGL(k_fill<double>, dim3(1), dim3(64), 0, st(), sc(), (int64_t)16, 0.0);
    if ((st0 = lin(grid(AG_S), 0, {{src(0, 0), 1.0}}, nperp)) != QSA_OK) return st0;
    for (int j = 0; j < p.nxi; ++j) {
      if ((st0 = throttle()) != QSA_OK) return st0;
      if (j % A.ck_len == 0)
        for (int k = 0; k < 4; ++k)
          HIP_OK(hipMemcpyAsync(ck(t, j / A.ck_len, k), Ya[k], np * sizeof(R), hipMemcpyDeviceToDevice, st()));
      if ((st0 = fwd_slice(t, j, Ya, Yb2)) != QSA_OK) return st0;
      for (int k = 0; k < 4; ++k) std::swap(Ya[k], Yb2[k]);
    }
    return QSA_OK;
  }

  // ---- reverse of one slice ------------------------------------------------
  // segment slot i holds the plasma state at slice j; yin: adjoint of
  // Y^{j+1}; yout: adjoint of Y^j (written).
  qsa_status rev_slice(int t, int j, int i, R* const* yin, R* const* yout) {
    qsa_status st0;
    const int par = j & 1;
    double* ai = scr(1 - par);   // slice j + 1's results
    double* ao = scr(par);
    const int fm[6] = {F_PSI, F_DXPSI, F_DYPSI, F_BX, F_BY, F_BZ};
    auto m1 = [&](int f) { return (j >= 1) ? fbar(f, j - 1) : grid(AG_SINK + f); };
    auto m2 = [&](int f) { return (j >= 2) ? fbar(f, j - 2) : grid(AG_SINK + f); };
    R* JB[2] = {grid(AA_JB0 + 2 * par), grid(AA_JB0 + 2 * par + 1)};
    R* JBm1[2] = {(j >= 1) ? grid(AA_JB0 + 2 * (1 - par)) : grid(AG_SINK),
                  (j >= 1) ? grid(AA_JB0 + 2 * (1 - par) + 1) : grid(AG_SINK + 1)};
    const double i2h = 1.0 / (2.0 * h);
    AdjPlasma<R> a = plasma_args();
    for (int k = 0; k < 4; ++k) a.Y[k] = yarr(A.segY, i, k);
    SixBar<R> fbs;
    for (int m = 0; m < 6; ++m) {
      fbs.a[m] = fbar(fm[m], j);
      fbs.m1[m] = m1(fm[m]);
    }
    // final advance
    {
      AdjPlasma<R> b = a;
      six(t, j, field(t, F_BX, j), field(t, F_BY, j), b.F);
      b.Fb = fbs;
      for (int k = 0; k < 4; ++k) {
        b.Ynb[k] = yin[k];
        b.Yn[k] = yout[k];
      }
      SideB sd(this);
      sd.lin(grid(AA_JZ), 0, {});
      if (K > 0) {
        const R* pm1 = (j >= 1) ? field(t, F_PSI, j - 1) : grid(AG_ZERO);
        const R* pm2 = (j >= 2) ? field(t, F_PSI, j - 2) : grid(AG_ZERO);
        sd.lin(grid(AA_PSIT), 0, {});
        sd.lin(grid(AG_PSIT), 0, {{field(t, F_PSI, j), 3.0}, {pm1, -3.0}, {pm2, 1.0}});
      }
      if (j >= 1) sd.lin(JBm1[0], 0, {}).lin(JBm1[1], 0, {});
      sd.scalar(SJ_ODE_ADJ, ai, ao, ezsum() + j, psipart(), (j + 1 < p.nxi) ? (int)g.ny : 0, h, (double)nperp);
      b.tile_bytes = tile_big;
      if ((st0 = plasma(k_ar_final<R>, b, sd.s, b.tile_bytes)) != QSA_OK) return st0;
    }
    // predictor-corrector, iterations in reverse
    R* bcur[2] = {fbar(F_BX, j), fbar(F_BY, j)};
    int pi = 0;
    for (int k = K - 1; k >= 0; --k) {
      R* bnew[2] = {grid(AA_BP0 + 2 * pi), grid(AA_BP0 + 2 * pi + 1)};
      pi ^= 1;
      SpecB s(this, 1);
      const int f0 = s.input({{bcur[0], 1.0}}), f1 = s.input({{bcur[1], 1.0}});
      const int oz = s.output(), ox = s.output(), oy = s.output(), obx = s.output(), oby = s.output();
      s.term(oz, SK_IKY_DEN, f0, -1.0);
      s.term(oz, SK_IKX_DEN, f1, 1.0);
      s.dest(oz, grid(AA_JZ), 1.0, 1);
      s.term(ox, SK_DEN, f1, 1.0);
      s.dest(ox, grid(AA_DB), 1.0, 0);
      s.dest(ox, JBm1[0], -i2h, 1);
      s.term(oy, SK_DEN, f0, -1.0);
      s.dest(oy, grid(AA_DB + 1), 1.0, 0);
      s.dest(oy, JBm1[1], -i2h, 1);
      if (j + 1 < p.nxi) {
        s.dest(ox, srcb(1, j + 1), i2h, 1);
        s.dest(oy, srcb(2, j + 1), i2h, 1);
      }
      s.term(obx, SK_DEN, f0, -p.kappa2);
      s.dest(obx, bnew[0], 1.0, 0);
      s.term(oby, SK_DEN, f1, -p.kappa2);
      s.dest(oby, bnew[1], 1.0, 0);
      if ((st0 = spec(s, none, none, none)) != QSA_OK) return st0;
      AdjPlasma<R> b = a;
      six(t, j, bk(t, k, 0, j), bk(t, k, 1, j), b.F);
      b.Fb = fbs;
      b.Fb.a[3] = bnew[0];
      b.Fb.a[4] = bnew[1];
      for (int q = 0; q < 4; ++q) {
        b.Yt[q] = c->at<R>(A.segYt) + (((int64_t)i * K + k) * 4 + q) * np;
        b.Yn[q] = yout[q];
      }
      b.psi = grid(AG_PSIT);
      b.psib = grid(AA_PSIT);
      b.Jx = grid(AA_DB);
      b.Jy = grid(AA_DB + 1);
      b.jscale = i2h;
      b.tile_bytes = tile_big;
      if ((st0 = plasma(k_ar_pred<R>, b, none, b.tile_bytes)) != QSA_OK) return st0;
      bcur[0] = bnew[0];
      bcur[1] = bnew[1];
    }
    // (B_z, E_z) from J_perp; with it, B_0 = 2 B^{j-1} - B^{j-2} and the
    // psi extrapolation 3 psi^j - 3 psi^{j-1} + psi^{j-2} to the history
    {
      SpecB s(this, 1);
      const int f0 = s.input({{fbar(F_BZ, j), 1.0}}), f1 = s.input({{fbar(F_EZ, j), 1.0}});
      const int ox = s.output(), oy = s.output();
      s.term(ox, SK_IKY_K2, f0, -1.0);
      s.term(ox, SK_IKX_K2, f1, -1.0);
      s.dest(ox, JB[0], 1.0, 1);
      s.term(oy, SK_IKX_K2, f0, 1.0);
      s.term(oy, SK_IKY_K2, f1, -1.0);
      s.dest(oy, JB[1], 1.0, 1);
      SideB sr(this), scl(this);
      sr.lin(m1(F_BX), 1, {{bcur[0], 2.0}}).lin(m1(F_BY), 1, {{bcur[1], 2.0}});
      sr.lin(m2(F_BX), 1, {{bcur[0], -1.0}}).lin(m2(F_BY), 1, {{bcur[1], -1.0}});
      if (K > 0) {
        scl.lin(fbar(F_PSI, j), 1, {{grid(AA_PSIT), 3.0}});
        scl.lin(m1(F_PSI), 1, {{grid(AA_PSIT), -3.0}});
        scl.lin(m2(F_PSI), 1, {{grid(AA_PSIT), 1.0}});
      }
      if ((st0 = spec(s, sr.s, scl.s, none)) != QSA_OK) return st0;
    }
    // J stage (the uniform J_z adjoint of the leapfrog is ao[2]); the beam's
    // J sources of this slice take the current adjoints
    {
      AdjPlasma<R> b = a;
      b.psi = field(t, F_PSI, j);
      b.psib = fbar(F_PSI, j);
      b.Jx = JB[0];
      b.Jy = JB[1];
      b.Jz = grid(AA_JZ);
      b.jzs = ao + 2;
      for (int q = 0; q < 4; ++q) b.Yn[q] = yout[q];
      SideB sd(this);
      sd.lin(srcb(1, j), 1, {{JB[0], 1.0}}).lin(srcb(2, j), 1, {{JB[1], 1.0}});
      sd.lin(srcb(3, j), 1, {{grid(AA_JZ), 1.0}}, ao + 2, 1.0);
      if ((st0 = plasma(k_ar_jstage<R>, b, sd.s, b.tile_bytes)) != QSA_OK) return st0;
    }
    // psi stage: adjoint of S (and of the beam's rho - J_z), of psi0
    {
      SpecB s(this, 1);
      const int f0 = s.input({{fbar(F_PSI, j), 1.0}});
      const int f1 = s.input({{fbar(F_DXPSI, j), 1.0}});
      const int f2 = s.input({{fbar(F_DYPSI, j), 1.0}});
      const int o = s.output();
      s.term(o, SK_INVK2, f0, 1.0);
      s.term(o, SK_IKX_K2, f1, 1.0);
      s.term(o, SK_IKY_K2, f2, 1.0);
      s.dest(o, grid(AA_S), 1.0, 0);
      s.dest(o, srcb(0, j), 1.0, 1);
      s.op.insum = psipart();
      if ((st0 = spec(s, none, none, none)) != QSA_OK) return st0;
    }
    {
      AdjPlasma<R> b = a;
      b.Sb = grid(AA_S);
      for (int q = 0; q < 4; ++q) b.Yn[q] = yout[q];
      if ((st0 = plasma(k_ar_jstage<R>, b, none, b.tile_bytes)) != QSA_OK) return st0;
    }
    return QSA_OK;
  }

  // reverse of sweep t: fbar (field adjoint) -> srcb (source adjoint)
  qsa_status rev_sweep(int t) {
    qsa_status st0;
    if ((st0 = lin(c->at<R>(A.srcb), 0, {}, 4 * plane)) != QSA_OK) return st0;
    for (int k = 0; k < 4; ++k)
      if ((st0 = lin(grid(AA_JB0 + k), 0, {}, nperp)) != QSA_OK) return st0;
    hipLaunchKernelGGL(k_fill<double>, dim3(1), dim3(64), 0, st(), sc() + 16, (int64_t)16, 0.0);
    hipLaunchKernelGGL(k_slice_sums<R>, dim3(p.nxi), dim3(256), 0, st(), (const R*)fbar(F_EZ, 0), (int)nperp,
                       ezsum());
    R* yb[2][4];
    for (int i = 0; i < 2; ++i)
      for (int k = 0; k < 4; ++k) yb[i][k] = yarr(A.Yb[i], 0, k);
    for (int k = 0; k < 4; ++k)
      if ((st0 = lin(yb[0][k], 0, {}, np)) != QSA_OK) return st0;
    int cur = 0;
    for (int cidx = A.nseg - 1; cidx >= 0; --cidx) {
      const int j0 = cidx * A.ck_len, j1 = std::min(p.nxi, j0 + A.ck_len);
      AdjSeg<R> sg;
      std::memset(&sg, 0, sizeof(sg));
      sg.g = g;
      sg.np = (int)np;
      sg.K = K;
      sg.j0 = j0;
      sg.len = j1 - j0;
      sg.h = h;
      for (int k = 0; k < 4; ++k) sg.Y0[k] = ck(t, cidx, k);
      sg.segY = c->at<R>(A.segY);
      sg.segYt = c->at<R>(A.segYt);
      sg.fields = fields(t);
      sg.biter = biter_base(t);
      sg.zero = grid(AG_ZERO);
      hipLaunchKernelGGL(k_af_segment<R>, dim3(blocks(np)), dim3(256), 0, st(), sg);
      HIP_OK(hipGetLastError());
      for (int j = j1 - 1; j >= j0; --j) {
        if ((st0 = throttle()) != QSA_OK) return st0;
        if ((st0 = rev_slice(t, j, j - j0, yb[cur], yb[1 - cur])) != QSA_OK) return st0;
        cur = 1 - cur;
      }
    }
    return QSA_OK;
  }

  // ---- beam ------------------------------------------------------------------
  AdjBeam<R> beam_args(int t, int s) {
    AdjBeam<R> b;
    std::memset(&b, 0, sizeof(b));
    b.g = g;
    b.n = c->beam_n[s];
    b.zdv = p.species[s].Z / (p.dx * p.dy * p.dxi);
    b.qh = (double)p.species[s].Z / p.species[s].M * 0.5 * p.dt;
    b.dt = p.dt;
    b.inv_dxi = 1.0 / p.dxi;
    b.xi_max = (double)(p.nxi - 1) * p.dxi;
    b.x = bstate(t, s, 0);
    b.y = bstate(t, s, 1);
    b.ux = bstate(t, s, 2);
    b.uy = bstate(t, s, 3);
    b.uz = bstate(t, s, 4);
    b.w = bstate(t, s, 5);
    b.xi = bxi(t, s);
    if (t < A.steps) {
      b.xo = bstate(t + 1, s, 0);
      b.yo = bstate(t + 1, s, 1);
      b.uxo = bstate(t + 1, s, 2);
      b.uyo = bstate(t + 1, s, 3);
      b.uzo = bstate(t + 1, s, 4);
      b.wo = bstate(t + 1, s, 5);
      b.xio = bxi(t + 1, s);
    }
    b.src = c->at<R>(A.src);
    b.srcb = c->at<R>(A.srcb);
    b.fields = fields(t);
    b.fieldsb = c->at<R>(A.fb);
    for (int k = 0; k < 7; ++k) b.b[k] = c->at<R>(A.bb[s][k]);
    b.tile_bytes = tile_small;
    return b;
  }

  // beam sources of step t and the per-slice sums of their J_z
  qsa_status sources(int t) {
    qsa_status st0 = lin(c->at<R>(A.src), 0, {}, 4 * plane);
    if (st0 != QSA_OK) return st0;
    for (int s = 0; s < p.n_species; ++s) {
      if (c->beam_n[s] == 0) continue;
      hipLaunchKernelGGL(k_ab_sources<R>, dim3(blocks(c->beam_n[s])), dim3(256), (size_t)tile_small, st(),
                         beam_args(t, s));
    }
    hipLaunchKernelGGL(k_slice_sums<R>, dim3(p.nxi), dim3(256), 0, st(), (const R*)src(3, 0), (int)nperp, jzsum());
    HIP_OK(hipGetLastError());
    return QSA_OK;
  }

  qsa_status run(int nsteps, int nb, double* loss, double* grad) {
    qsa_status st0;
    {
      // column transforms: twiddles and two FFT buffers per wavefront
      const size_t cols_lds = ((size_t)g.ny + 2 * (size_t)SPEC_IN * fft_cap(g.ny)) * sizeof(C2<R>);
      if (cols_lds > 65536)
        HIP_OK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_spec_cols<R>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)cols_lds));
      // the plasma transposes scatter 12-13 channels: one block per CU
      // holds the launch anyway (256 particles per block), so their tile
      // takes most of the CU's LDS
      int dev = 0, optin = 0;
      HIP_OK(hipGetDevice(&dev));
      if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess) optin = 0;
      tile_big = std::max(tile_small, std::min(133120, optin));
      if (tile_big > 65536) {
        HIP_OK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_ar_final<R>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, tile_big));
        HIP_OK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_ar_pred<R>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, tile_big));
      }
    }
    if ((st0 = lin(grid(AG_ZERO), 0, {}, nperp)) != QSA_OK) return st0;
    hipLaunchKernelGGL(k_spec_table<R>, dim3(g.nx / 2 + 1), dim3(256), 0, st(), g, p.kappa2, c->at<double>(A.ktab));
    // step 0: the current beam with scaled weights
    for (int s = 0; s < p.n_species; ++s) {
      const int64_t n = c->beam_n[s];
      if (n == 0) continue;
      for (int k = 0; k < 5; ++k)
        HIP_OK(hipMemcpyAsync(bstate(0, s, k), c->ws + c->L.beam[s][k], n * sizeof(R), hipMemcpyDeviceToDevice,
                              st()));
      HIP_OK(hipMemcpyAsync(bxi(0, s), c->ws + c->L.beam[s][6], n * 8, hipMemcpyDeviceToDevice, st()));
      HIP_OK(hipMemcpyAsync(c->ws + A.w0[s], c->ws + c->L.beam[s][5], n * sizeof(R), hipMemcpyDeviceToDevice,
                            st()));
      hipLaunchKernelGGL(k_ab_scale_w<R>, dim3(blocks(n)), dim3(256), 0, st(), (const R*)c->at<R>(A.w0[s]),
                         (const int*)c->at<int>(A.bin[s]), (const double*)c->at<double>(A.amps), nb,
                         bstate(0, s, 5), n);
    }
    // forward
    for (int t = 0; t <= nsteps; ++t) {
      if ((st0 = sources(t)) != QSA_OK) return st0;
      if ((st0 = fwd_sweep(t)) != QSA_OK) return st0;
      if (t < nsteps)
        for (int s = 0; s < p.n_species; ++s) {
          if (c->beam_n[s] == 0) continue;
          hipLaunchKernelGGL(k_ab_push<R>, dim3(blocks(c->beam_n[s])), dim3(256), 0, st(), beam_args(t, s));
        }
      HIP_OK(hipGetLastError());
    }
    // loss and its field adjoint
    const double dV = p.dx * p.dy * p.dxi;
    double* L = sc() + 48;
    hipLaunchKernelGGL(k_fill<double>, dim3(1), dim3(64), 0, st(), L, (int64_t)1, 0.0);
    hipLaunchKernelGGL(k_sumsq<R>, dim3(256), dim3(256), 0, st(), (const R*)field(nsteps, F_BX, 0), plane, 0.5 * dV,
                       L);
    hipLaunchKernelGGL(k_sumsq<R>, dim3(256), dim3(256), 0, st(), (const R*)field(nsteps, F_BY, 0), plane, 0.5 * dV,
                       L);
    if ((st0 = lin(c->at<R>(A.fb), 0, {}, N_STORED * plane)) != QSA_OK) return st0;
    if ((st0 = lin(fbar(F_BX, 0), 0, {{field(nsteps, F_BX, 0), dV}}, plane)) != QSA_OK) return st0;
    if ((st0 = lin(fbar(F_BY, 0), 0, {{field(nsteps, F_BY, 0), dV}}, plane)) != QSA_OK) return st0;
    for (int s = 0; s < p.n_species; ++s)
      for (int k = 0; k < 7; ++k)
        if (c->beam_n[s] > 0 && (st0 = lin(c->at<R>(A.bb[s][k]), 0, {}, c->beam_n[s])) != QSA_OK) return st0;
    // reverse
    for (int t = nsteps; t >= 0; --t) {
      if ((st0 = rev_sweep(t)) != QSA_OK) return st0;
      for (int s = 0; s < p.n_species; ++s) {
        if (c->beam_n[s] == 0) continue;
        hipLaunchKernelGGL(k_ab_sources_adj<R>, dim3(blocks(c->beam_n[s])), dim3(256), 0, st(), beam_args(t, s));
      }
      if (t > 0) {
        if ((st0 = lin(c->at<R>(A.fb), 0, {}, N_STORED * plane)) != QSA_OK) return st0;
        for (int s = 0; s < p.n_species; ++s) {
          if (c->beam_n[s] == 0) continue;
          hipLaunchKernelGGL(k_ab_push_adj<R>, dim3(blocks(c->beam_n[s])), dim3(256), (size_t)tile_small, st(),
                             beam_args(t - 1, s));
        }
      }
      HIP_OK(hipGetLastError());
    }
    // gradient per bin
    double* gr = c->at<double>(A.grad);
    hipLaunchKernelGGL(k_fill<double>, dim3(16), dim3(256), 0, st(), gr, (int64_t)nb, 0.0);
    for (int s = 0; s < p.n_species; ++s) {
      const int64_t n = c->beam_n[s];
      if (n == 0) continue;
      hipLaunchKernelGGL(k_ab_bin_grad<R>, dim3((unsigned)std::min<int64_t>(1024, blocks(n))), dim3(256),
                         (size_t)nb * sizeof(double), st(), (const R*)c->at<R>(A.bb[s][6]),
                         (const R*)c->at<R>(A.w0[s]), (const int*)c->at<int>(A.bin[s]), nb, gr, n);
    }
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(loss, L, sizeof(double), hipMemcpyDeviceToHost, st()));
    HIP_OK(hipMemcpyAsync(grad, gr, nb * sizeof(double), hipMemcpyDeviceToHost, st()));
    HIP_OK(hipStreamSynchronize(st()));
    return QSA_OK;
  }
};

}  // namespace
