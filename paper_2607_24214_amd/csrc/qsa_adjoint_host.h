// Host driver of the adjoint (qsa_adjoint_sweep); included by qsa.hip after
// the context and the forward engine are defined.
//
// Order of work for n beam steps:
//   forward  t = 0..n:  sources of beam(t); sweep(t) with plasma checkpoints
//                       every QSA_ADJ_CKPT slices; beam(t+1) = push (t < n);
//   loss              = 1/2 sum (B_x^2 + B_y^2) dV of sweep(n);
//   reverse  t = n..0:  sources of beam(t) again (the recomputation needs
//                       them); sweep(t)^T, segment by segment (recompute the
//                       segment from its checkpoint, then its slices in
//                       reverse); sources^T into the beam adjoint; push^T of
//                       step t - 1 into the beam adjoint and the field
//                       adjoint of sweep(t - 1);
//   gradient          = per bin, sum of (weight adjoint x loaded weight).

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

  Adj(qsa_ctx* ctx, const AdjLayout& lay) : c(ctx), p(ctx->p), A(lay) {
    g = Engine<R>::geo(p);
    K = std::max(p.n_corr, 0);
    nperp = g.nperp;
    plane = (int64_t)p.nxi * nperp;
    np = p.n_plasma;
    h = p.dxi;
  }

  hipStream_t st() const { return c->stream; }
  R* grid(int k) const { return c->at<R>(A.grids) + (int64_t)k * nperp; }
  double* sc() const { return c->at<double>(A.sc); }
  R* fields(int t) const { return c->at<R>(A.fields) + (int64_t)t * N_STORED * plane; }
  R* field(int t, int f, int j) const { return fields(t) + (int64_t)f * plane + (int64_t)j * nperp; }
  R* fbar(int f, int j) const { return c->at<R>(A.fb) + (int64_t)f * plane + (int64_t)j * nperp; }
  R* src(int k, int j) const { return c->at<R>(A.src) + (int64_t)k * plane + (int64_t)j * nperp; }
  R* srcb(int k, int j) const { return c->at<R>(A.srcb) + (int64_t)k * plane + (int64_t)j * nperp; }
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
  R* segYt(int i, int k, int comp) const { return c->at<R>(A.segYt) + (((int64_t)i * K + k) * 4 + comp) * np; }
  R* segB(int i, int k, int comp) const { return c->at<R>(A.segB) + (((int64_t)i * K + k) * 2 + comp) * nperp; }
  char* ck(int t, int cidx) const { return c->ws + A.ck + ((size_t)t * A.nseg + cidx) * A.ck_bytes; }

  static int blocks(int64_t n) { return (int)std::max<int64_t>(1, (n + 255) / 256); }

  qsa_status lin(R* out, int add, double c0, std::initializer_list<std::pair<const R*, double>> terms,
                 int64_t n = -1) {
    Lin<R> a;
    std::memset(&a, 0, sizeof(a));
    a.out = out;
    a.add = add;
    a.c0 = c0;
    for (const auto& t : terms) {
      a.in[a.nt] = t.first;
      a.c[a.nt] = t.second;
      ++a.nt;
    }
    if (n < 0) n = nperp;
    hipLaunchKernelGGL(k_lin<R>, dim3(blocks(n)), dim3(256), 0, st(), a, n);
    HIP_OK(hipGetLastError());
    return QSA_OK;
  }

  qsa_status spec(SpecOp<R>& op) {
    op.kappa2 = p.kappa2;
    op.work = c->at<C2<R>>(A.work);
    const size_t rows_lds = 3 * (size_t)g.nx * sizeof(C2<R>);
    const size_t cols_lds = ((size_t)g.ny * (3 + op.ni)) * sizeof(C2<R>);
    hipLaunchKernelGGL(k_spec_rows_fwd<R>, dim3(g.ny, op.ni), dim3(64), rows_lds, st(), g, op,
                       (const C2<R>*)c->at<C2<R>>(c->L.twx));
    hipLaunchKernelGGL(k_spec_cols<R>, dim3(g.nx), dim3(64), cols_lds, st(), g, op,
                       (const C2<R>*)c->at<C2<R>>(c->L.twy));
    hipLaunchKernelGGL(k_spec_rows_inv<R>, dim3(g.ny, op.no), dim3(64), rows_lds, st(), g, op,
                       (const C2<R>*)c->at<C2<R>>(c->L.twx));
    HIP_OK(hipGetLastError());
    return QSA_OK;
  }

  static SpecOp<R> op0() {
    SpecOp<R> op;
    std::memset(&op, 0, sizeof(op));
    return op;
  }
  static void term(SpecOp<R>& op, int o, int kind, int in, double coef) {
    const int q = op.nterm[o]++;
    op.kind[o][q] = kind;
    op.src[o][q] = in;
    op.coef[o][q] = coef;
  }

  AdjPlasma<R> plasma_args() const {
    AdjPlasma<R> a;
    std::memset(&a, 0, sizeof(a));
    a.g = g;
    a.np = (int)np;
    a.nw = -p.plasma_w / (p.dx * p.dy);
    a.h = h;
    a.err = c->at<int>(c->L.err);
    return a;
  }

  // the fields a plasma particle sees at slice j: psi, dxpsi, dypsi from the
  // tape, B_perp given, B_z from the tape; F^{j-1} from the tape (zero ahead)
  void six(int t, int j, const R* bx, const R* by, Six<R>& F) const {
    F.a[0] = field(t, F_PSI, j);
    F.a[1] = field(t, F_DXPSI, j);
    F.a[2] = field(t, F_DYPSI, j);
    F.a[3] = bx;
    F.a[4] = by;
    F.a[5] = field(t, F_BZ, j);
    const int fm[6] = {F_PSI, F_DXPSI, F_DYPSI, F_BX, F_BY, F_BZ};
    for (int m = 0; m < 6; ++m) F.m1[m] = (j >= 1) ? field(t, fm[m], j - 1) : grid(AG_ZERO);
  }

  // ---- forward slice -------------------------------------------------------
  // Yin -> Yout at slice j of sweep t; with seg >= 0 the predictor states and
  // B_perp iterates go to segment slot seg.
  qsa_status fwd_slice(int t, int j, R* const* Yin, R* const* Yout, int seg) {
    qsa_status st0;
    const R* zero = grid(AG_ZERO);
    AdjPlasma<R> a = plasma_args();
    for (int k = 0; k < 4; ++k) a.Y[k] = Yin[k];
    // psi stage
    if ((st0 = lin(grid(AG_S), 0, 1.0, {{src(0, j), 1.0}})) != QSA_OK) return st0;
    hipLaunchKernelGGL(k_af_dep_s<R>, dim3(blocks(np)), dim3(256), 0, st(), a, grid(AG_S));
    {
      SpecOp<R> op = op0();
      op.ni = 1;
      op.no = 3;
      op.in[0] = grid(AG_S);
      op.out[0] = field(t, F_PSI, j);
      op.out[1] = field(t, F_DXPSI, j);
      op.out[2] = field(t, F_DYPSI, j);
      term(op, 0, SK_INVK2, 0, 1.0);
      term(op, 1, SK_IKX_K2, 0, 1.0);
      term(op, 2, SK_IKY_K2, 0, 1.0);
      op.mean[0] = sc() + 1;
      if ((st0 = spec(op)) != QSA_OK) return st0;
    }
    // J stage
    if ((st0 = lin(grid(AG_JX), 0, 0.0, {{src(1, j), 1.0}})) != QSA_OK) return st0;
    if ((st0 = lin(grid(AG_JY), 0, 0.0, {{src(2, j), 1.0}})) != QSA_OK) return st0;
    if ((st0 = lin(grid(AG_JZ), 0, 0.0, {{src(3, j), 1.0}})) != QSA_OK) return st0;
    a.psi = field(t, F_PSI, j);
    a.Jx = grid(AG_JX);
    a.Jy = grid(AG_JY);
    a.Jz = grid(AG_JZ);
    hipLaunchKernelGGL(k_af_dep_j<R>, dim3(blocks(np)), dim3(256), 0, st(), a);
    hipLaunchKernelGGL(k_fill<double>, dim3(1), dim3(64), 0, st(), sc() + 2, (int64_t)1, 0.0);
    hipLaunchKernelGGL(k_sum<R>, dim3(64), dim3(256), 0, st(), (const R*)grid(AG_JZ), nperp, 1.0, sc() + 2);
    hipLaunchKernelGGL(k_ode_fwd, dim3(1), dim3(64), 0, st(), sc(), h, (double)nperp);
    {
      SpecOp<R> op = op0();
      op.ni = 2;
      op.no = 2;
      op.in[0] = grid(AG_JX);
      op.in[1] = grid(AG_JY);
      op.out[0] = field(t, F_BZ, j);
      op.out[1] = field(t, F_EZ, j);
      term(op, 0, SK_IKY_K2, 0, -1.0);
      term(op, 0, SK_IKX_K2, 1, 1.0);
      term(op, 1, SK_IKX_K2, 0, -1.0);
      term(op, 1, SK_IKY_K2, 1, -1.0);
      op.mean[1] = sc() + 3;
      if ((st0 = spec(op)) != QSA_OK) return st0;
    }
    // B_perp predictor-corrector
    const R* bm1x = (j >= 1) ? field(t, F_BX, j - 1) : zero;
    const R* bm1y = (j >= 1) ? field(t, F_BY, j - 1) : zero;
    const R* bm2x = (j >= 2) ? field(t, F_BX, j - 2) : zero;
    const R* bm2y = (j >= 2) ? field(t, F_BY, j - 2) : zero;
    const R* pm1 = (j >= 1) ? field(t, F_PSI, j - 1) : zero;
    const R* pm2 = (j >= 2) ? field(t, F_PSI, j - 2) : zero;
    auto bk = [&](int k, int comp) -> R* {
      if (k == K) return field(t, comp ? F_BY : F_BX, j);
      if (seg >= 0) return segB(seg, k, comp);
      return grid((k & 1) ? (comp ? AG_BBY : AG_BBX) : (comp ? AG_BAY : AG_BAX));
    };
    if ((st0 = lin(bk(0, 0), 0, 0.0, {{bm1x, 2.0}, {bm2x, -1.0}})) != QSA_OK) return st0;
    if ((st0 = lin(bk(0, 1), 0, 0.0, {{bm1y, 2.0}, {bm2y, -1.0}})) != QSA_OK) return st0;
    if ((st0 = lin(grid(AG_PSIT), 0, 0.0, {{field(t, F_PSI, j), 3.0}, {pm1, -3.0}, {pm2, 1.0}})) != QSA_OK)
      return st0;
    for (int k = 0; k < K; ++k) {
      const bool last = j + 1 >= p.nxi;
      if ((st0 = lin(grid(AG_JTX), 0, 0.0, {{last ? zero : src(1, j + 1), 1.0}})) != QSA_OK) return st0;
      if ((st0 = lin(grid(AG_JTY), 0, 0.0, {{last ? zero : src(2, j + 1), 1.0}})) != QSA_OK) return st0;
      AdjPlasma<R> b = a;
      six(t, j, bk(k, 0), bk(k, 1), b.F);
      b.psi = grid(AG_PSIT);
      b.Jx = grid(AG_JTX);
      b.Jy = grid(AG_JTY);
      R* yt[4];
      for (int q = 0; q < 4; ++q) yt[q] = (seg >= 0) ? segYt(seg, k, q) : yarr(A.ytmp, 0, q);
      hipLaunchKernelGGL(k_af_pred<R>, dim3(blocks(np)), dim3(256), 0, st(), b, yt[0], yt[1], yt[2], yt[3]);
      const double i2h = 1.0 / (2.0 * h);
      if ((st0 = lin(grid(AG_DX), 0, 0.0, {{grid(AG_JTX), i2h}, {grid(AG_JM1X), -i2h}})) != QSA_OK) return st0;
      if ((st0 = lin(grid(AG_DY), 0, 0.0, {{grid(AG_JTY), i2h}, {grid(AG_JM1Y), -i2h}})) != QSA_OK) return st0;
      SpecOp<R> op = op0();
      op.ni = 5;
      op.no = 2;
      op.in[0] = grid(AG_JZ);
      op.in[1] = grid(AG_DX);
      op.in[2] = grid(AG_DY);
      op.in[3] = bk(k, 0);
      op.in[4] = bk(k, 1);
      op.out[0] = bk(k + 1, 0);
      op.out[1] = bk(k + 1, 1);
      term(op, 0, SK_IKY_DEN, 0, -1.0);
      term(op, 0, SK_DEN, 2, -1.0);
      term(op, 0, SK_DEN, 3, -p.kappa2);
      term(op, 1, SK_IKX_DEN, 0, 1.0);
      term(op, 1, SK_DEN, 1, 1.0);
      term(op, 1, SK_DEN, 4, -p.kappa2);
      if ((st0 = spec(op)) != QSA_OK) return st0;
    }
    // final advance
    {
      AdjPlasma<R> b = a;
      six(t, j, field(t, F_BX, j), field(t, F_BY, j), b.F);
      for (int k = 0; k < 4; ++k) b.Yn[k] = Yout[k];
      hipLaunchKernelGGL(k_af_final<R>, dim3(blocks(np)), dim3(256), 0, st(), b);
    }
    // history for the next slice: J_perp, <E_z> at j + 1/2, psi0 at j + 1
    if ((st0 = lin(grid(AG_JM1X), 0, 0.0, {{grid(AG_JX), 1.0}})) != QSA_OK) return st0;
    if ((st0 = lin(grid(AG_JM1Y), 0, 0.0, {{grid(AG_JY), 1.0}})) != QSA_OK) return st0;
    HIP_OK(hipMemcpyAsync(sc() + 0, sc() + 4, 2 * sizeof(double), hipMemcpyDeviceToDevice, st()));
    HIP_OK(hipGetLastError());
    return QSA_OK;
  }

  // checkpoint of slice j of sweep t: the plasma state, J_perp of j - 1,
  // <E_z> at j - 1/2 and psi0 at j
  qsa_status save_ck(int t, int cidx, R* const* Y) {
    char* base = ck(t, cidx);
    const size_t rs = sizeof(R);
    for (int k = 0; k < 4; ++k)
      HIP_OK(hipMemcpyAsync(base + k * np * rs, Y[k], np * rs, hipMemcpyDeviceToDevice, st()));
    char* jb = base + align_up(4 * np * rs);
    HIP_OK(hipMemcpyAsync(jb, grid(AG_JM1X), nperp * rs, hipMemcpyDeviceToDevice, st()));
    HIP_OK(hipMemcpyAsync(jb + nperp * rs, grid(AG_JM1Y), nperp * rs, hipMemcpyDeviceToDevice, st()));
    char* sb = jb + align_up(2 * nperp * rs);
    HIP_OK(hipMemcpyAsync(sb, sc(), 2 * sizeof(double), hipMemcpyDeviceToDevice, st()));
    return QSA_OK;
  }
  qsa_status load_ck(int t, int cidx, R* const* Y) {
    char* base = ck(t, cidx);
    const size_t rs = sizeof(R);
    for (int k = 0; k < 4; ++k)
      HIP_OK(hipMemcpyAsync(Y[k], base + k * np * rs, np * rs, hipMemcpyDeviceToDevice, st()));
    char* jb = base + align_up(4 * np * rs);
    HIP_OK(hipMemcpyAsync(grid(AG_JM1X), jb, nperp * rs, hipMemcpyDeviceToDevice, st()));
    HIP_OK(hipMemcpyAsync(grid(AG_JM1Y), jb + nperp * rs, nperp * rs, hipMemcpyDeviceToDevice, st()));
    char* sb = jb + align_up(2 * nperp * rs);
    HIP_OK(hipMemcpyAsync(sc(), sb, 2 * sizeof(double), hipMemcpyDeviceToDevice, st()));
    return QSA_OK;
  }

  qsa_status fwd_sweep(int t) {
    qsa_status st0;
    R* Ya[4];
    R* Yb2[4];
    for (int k = 0; k < 4; ++k) {
      Ya[k] = yarr(A.Y[0], 0, k);
      Yb2[k] = yarr(A.Y[1], 0, k);
      HIP_OK(hipMemcpyAsync(Ya[k], c->ws + c->L.tmpl[k], np * sizeof(R), hipMemcpyDeviceToDevice, st()));
    }
    if ((st0 = lin(grid(AG_ZERO), 0, 0.0, {})) != QSA_OK) return st0;
    if ((st0 = lin(grid(AG_JM1X), 0, 0.0, {})) != QSA_OK) return st0;
    if ((st0 = lin(grid(AG_JM1Y), 0, 0.0, {})) != QSA_OK) return st0;
    hipLaunchKernelGGL(k_fill<double>, dim3(1), dim3(64), 0, st(), sc(), (int64_t)16, 0.0);
    for (int j = 0; j < p.nxi; ++j) {
      if (j % A.ck_len == 0 && (st0 = save_ck(t, j / A.ck_len, Ya)) != QSA_OK) return st0;
      if ((st0 = fwd_slice(t, j, Ya, Yb2, -1)) != QSA_OK) return st0;
      for (int k = 0; k < 4; ++k) std::swap(Ya[k], Yb2[k]);
    }
    return QSA_OK;
  }

  // ---- reverse of one slice ------------------------------------------------
  // yin: adjoint of Y^{j+1}; yout: adjoint of Y^j (written); hout: history
  // adjoint from slice j + 1; hin: to slice j - 1 (written).
  qsa_status rev_slice(int t, int j, int seg, R* const* Y, R* const* yin, R* const* yout, int hout, int hin) {
    qsa_status st0;
    const R* zero = grid(AG_ZERO);
    double* ad = sc() + 16;
    auto H = [&](int set, int k) { return grid(set + k); };
    // adjoints of this slice's fields and history
    if ((st0 = lin(grid(AA_PSI), 0, 0.0, {{fbar(F_PSI, j), 1.0}, {H(hout, AH_FM1 + 0), 1.0}})) != QSA_OK) return st0;
    if ((st0 = lin(grid(AA_DXPSI), 0, 0.0, {{fbar(F_DXPSI, j), 1.0}, {H(hout, AH_FM1 + 1), 1.0}})) != QSA_OK)
      return st0;
    if ((st0 = lin(grid(AA_DYPSI), 0, 0.0, {{fbar(F_DYPSI, j), 1.0}, {H(hout, AH_FM1 + 2), 1.0}})) != QSA_OK)
      return st0;
    if ((st0 = lin(grid(AA_BKX), 0, 0.0, {{fbar(F_BX, j), 1.0}, {H(hout, AH_FM1 + 3), 1.0}})) != QSA_OK) return st0;
    if ((st0 = lin(grid(AA_BKY), 0, 0.0, {{fbar(F_BY, j), 1.0}, {H(hout, AH_FM1 + 4), 1.0}})) != QSA_OK) return st0;
    if ((st0 = lin(grid(AA_BZ), 0, 0.0, {{fbar(F_BZ, j), 1.0}, {H(hout, AH_FM1 + 5), 1.0}})) != QSA_OK) return st0;
    if ((st0 = lin(grid(AA_JX), 0, 0.0, {{H(hout, AH_JM1 + 0), 1.0}})) != QSA_OK) return st0;
    if ((st0 = lin(grid(AA_JY), 0, 0.0, {{H(hout, AH_JM1 + 1), 1.0}})) != QSA_OK) return st0;
    if ((st0 = lin(grid(AA_JZ), 0, 0.0, {})) != QSA_OK) return st0;
    if ((st0 = lin(grid(AA_PSIT), 0, 0.0, {})) != QSA_OK) return st0;
    for (int k = 0; k < 11; ++k) {
      const R* from = nullptr;
      if (k == AH_FM1 + 0) from = H(hout, AH_PSIM2);
      if (k == AH_FM1 + 3) from = H(hout, AH_BM2 + 0);
      if (k == AH_FM1 + 4) from = H(hout, AH_BM2 + 1);
      if (from) {
        if ((st0 = lin(H(hin, k), 0, 0.0, {{from, 1.0}})) != QSA_OK) return st0;
      } else if ((st0 = lin(H(hin, k), 0, 0.0, {})) != QSA_OK) {
        return st0;
      }
    }
    // <E_z> k = 0 value's adjoint
    hipLaunchKernelGGL(k_fill<double>, dim3(1), dim3(64), 0, st(), ad + 2, (int64_t)1, 0.0);
    hipLaunchKernelGGL(k_sum<R>, dim3(64), dim3(256), 0, st(), (const R*)fbar(F_EZ, j), nperp, 1.0, ad + 2);
    AdjPlasma<R> a = plasma_args();
    for (int k = 0; k < 4; ++k) a.Y[k] = Y[k];
    SixBar<R> fb;
    fb.a[0] = grid(AA_PSI);
    fb.a[1] = grid(AA_DXPSI);
    fb.a[2] = grid(AA_DYPSI);
    fb.a[5] = grid(AA_BZ);
    for (int m = 0; m < 6; ++m) fb.m1[m] = H(hin, AH_FM1 + m);
    // final advance
    {
      AdjPlasma<R> b = a;
      six(t, j, field(t, F_BX, j), field(t, F_BY, j), b.F);
      b.Fb = fb;
      b.Fb.a[3] = grid(AA_BKX);
      b.Fb.a[4] = grid(AA_BKY);
      for (int k = 0; k < 4; ++k) {
        b.Ynb[k] = yin[k];
        b.Yn[k] = yout[k];
      }
      hipLaunchKernelGGL(k_ar_final<R>, dim3(blocks(np)), dim3(256), 0, st(), b);
    }
    // predictor-corrector, iterations in reverse
    if (K > 0) {
      const R* pm1 = (j >= 1) ? field(t, F_PSI, j - 1) : zero;
      const R* pm2 = (j >= 2) ? field(t, F_PSI, j - 2) : zero;
      if ((st0 = lin(grid(AG_PSIT), 0, 0.0, {{field(t, F_PSI, j), 3.0}, {pm1, -3.0}, {pm2, 1.0}})) != QSA_OK)
        return st0;
    }
    int bcur = AA_BKX, bnew = AA_BNX;
    for (int k = K - 1; k >= 0; --k) {
      SpecOp<R> op = op0();
      op.conj = 1;
      op.ni = 2;
      op.no = 5;
      op.in[0] = grid(bcur);
      op.in[1] = grid(bcur + 1);
      op.out[0] = grid(AA_JZ);
      op.add[0] = 1;
      term(op, 0, SK_IKY_DEN, 0, -1.0);
      term(op, 0, SK_IKX_DEN, 1, 1.0);
      op.out[1] = grid(AA_DBX);
      term(op, 1, SK_DEN, 1, 1.0);
      op.out[2] = grid(AA_DBY);
      term(op, 2, SK_DEN, 0, -1.0);
      op.out[3] = grid(bnew);
      term(op, 3, SK_DEN, 0, -p.kappa2);
      op.out[4] = grid(bnew + 1);
      term(op, 4, SK_DEN, 1, -p.kappa2);
      if ((st0 = spec(op)) != QSA_OK) return st0;
      const double i2h = 1.0 / (2.0 * h);
      if ((st0 = lin(H(hin, AH_JM1 + 0), 1, 0.0, {{grid(AA_DBX), -i2h}})) != QSA_OK) return st0;
      if ((st0 = lin(H(hin, AH_JM1 + 1), 1, 0.0, {{grid(AA_DBY), -i2h}})) != QSA_OK) return st0;
      if (j + 1 < p.nxi) {
        if ((st0 = lin(srcb(1, j + 1), 1, 0.0, {{grid(AA_DBX), i2h}})) != QSA_OK) return st0;
        if ((st0 = lin(srcb(2, j + 1), 1, 0.0, {{grid(AA_DBY), i2h}})) != QSA_OK) return st0;
      }
      AdjPlasma<R> b = a;
      six(t, j, segB(seg, k, 0), segB(seg, k, 1), b.F);
      b.Fb = fb;
      b.Fb.a[3] = grid(bnew);
      b.Fb.a[4] = grid(bnew + 1);
      for (int q = 0; q < 4; ++q) {
        b.Yt[q] = segYt(seg, k, q);
        b.Yn[q] = yout[q];
      }
      b.psi = grid(AG_PSIT);
      b.psib = grid(AA_PSIT);
      b.Jx = grid(AA_DBX);
      b.Jy = grid(AA_DBY);
      b.jscale = i2h;
      hipLaunchKernelGGL(k_ar_pred<R>, dim3(blocks(np)), dim3(256), 0, st(), b);
      std::swap(bcur, bnew);
    }
    // B_0 = 2 B^{j-1} - B^{j-2}
    if ((st0 = lin(H(hin, AH_FM1 + 3), 1, 0.0, {{grid(bcur), 2.0}})) != QSA_OK) return st0;
    if ((st0 = lin(H(hin, AH_FM1 + 4), 1, 0.0, {{grid(bcur + 1), 2.0}})) != QSA_OK) return st0;
    if ((st0 = lin(H(hin, AH_BM2 + 0), 1, 0.0, {{grid(bcur), -1.0}})) != QSA_OK) return st0;
    if ((st0 = lin(H(hin, AH_BM2 + 1), 1, 0.0, {{grid(bcur + 1), -1.0}})) != QSA_OK) return st0;
    // psi extrapolated to j + 1
    if ((st0 = lin(grid(AA_PSI), 1, 0.0, {{grid(AA_PSIT), 3.0}})) != QSA_OK) return st0;
    if ((st0 = lin(H(hin, AH_FM1 + 0), 1, 0.0, {{grid(AA_PSIT), -3.0}})) != QSA_OK) return st0;
    if ((st0 = lin(H(hin, AH_PSIM2), 1, 0.0, {{grid(AA_PSIT), 1.0}})) != QSA_OK) return st0;
    // (B_z, E_z) from J_perp
    {
      SpecOp<R> op = op0();
      op.conj = 1;
      op.ni = 2;
      op.no = 2;
      op.in[0] = grid(AA_BZ);
      op.in[1] = fbar(F_EZ, j);
      op.out[0] = grid(AA_JX);
      op.add[0] = 1;
      term(op, 0, SK_IKY_K2, 0, -1.0);
      term(op, 0, SK_IKX_K2, 1, -1.0);
      op.out[1] = grid(AA_JY);
      op.add[1] = 1;
      term(op, 1, SK_IKX_K2, 0, 1.0);
      term(op, 1, SK_IKY_K2, 1, -1.0);
      if ((st0 = spec(op)) != QSA_OK) return st0;
    }
    // transverse-mean leapfrog
    hipLaunchKernelGGL(k_ode_adj, dim3(1), dim3(64), 0, st(), ad, h, (double)nperp);
    hipLaunchKernelGGL(k_add_scalar<R>, dim3(blocks(nperp)), dim3(256), 0, st(), grid(AA_JZ), nperp,
                       (const double*)(ad + 5), 1.0);
    // beam J sources of this slice
    if ((st0 = lin(srcb(1, j), 1, 0.0, {{grid(AA_JX), 1.0}})) != QSA_OK) return st0;
    if ((st0 = lin(srcb(2, j), 1, 0.0, {{grid(AA_JY), 1.0}})) != QSA_OK) return st0;
    if ((st0 = lin(srcb(3, j), 1, 0.0, {{grid(AA_JZ), 1.0}})) != QSA_OK) return st0;
    // J stage
    {
      AdjPlasma<R> b = a;
      b.psi = field(t, F_PSI, j);
      b.psib = grid(AA_PSI);
      b.Jx = grid(AA_JX);
      b.Jy = grid(AA_JY);
      b.Jz = grid(AA_JZ);
      for (int q = 0; q < 4; ++q) b.Yn[q] = yout[q];
      hipLaunchKernelGGL(k_ar_jstage<R>, dim3(blocks(np)), dim3(256), 0, st(), b);
    }
    // psi stage: adjoint of S, and of psi0 (the k = 0 value of psi)
    hipLaunchKernelGGL(k_sum<R>, dim3(64), dim3(256), 0, st(), (const R*)grid(AA_PSI), nperp, 1.0, ad + 4);
    {
      SpecOp<R> op = op0();
      op.conj = 1;
      op.ni = 3;
      op.no = 1;
      op.in[0] = grid(AA_PSI);
      op.in[1] = grid(AA_DXPSI);
      op.in[2] = grid(AA_DYPSI);
      op.out[0] = grid(AA_S);
      term(op, 0, SK_INVK2, 0, 1.0);
      term(op, 0, SK_IKX_K2, 1, 1.0);
      term(op, 0, SK_IKY_K2, 2, 1.0);
      if ((st0 = spec(op)) != QSA_OK) return st0;
    }
    if ((st0 = lin(srcb(0, j), 1, 0.0, {{grid(AA_S), 1.0}})) != QSA_OK) return st0;
    {
      AdjPlasma<R> b = a;
      b.Sb = grid(AA_S);
      for (int q = 0; q < 4; ++q) b.Yn[q] = yout[q];
      hipLaunchKernelGGL(k_ar_jstage<R>, dim3(blocks(np)), dim3(256), 0, st(), b);
    }
    // scalars for slice j - 1
    HIP_OK(hipMemcpyAsync(ad + 0, ad + 3, 2 * sizeof(double), hipMemcpyDeviceToDevice, st()));
    HIP_OK(hipGetLastError());
    return QSA_OK;
  }

  // reverse of sweep t: fbar (field adjoint) -> srcb (source adjoint)
  qsa_status rev_sweep(int t) {
    qsa_status st0;
    double* ad = sc() + 16;
    if ((st0 = lin(c->at<R>(A.srcb), 0, 0.0, {}, 4 * plane)) != QSA_OK) return st0;
    if ((st0 = lin(grid(AG_ZERO), 0, 0.0, {})) != QSA_OK) return st0;
    for (int k = 0; k < 11; ++k)
      if ((st0 = lin(grid(AH0 + k), 0, 0.0, {})) != QSA_OK) return st0;
    hipLaunchKernelGGL(k_fill<double>, dim3(1), dim3(64), 0, st(), ad, (int64_t)16, 0.0);
    R* yb[2][4];
    for (int i = 0; i < 2; ++i)
      for (int k = 0; k < 4; ++k) yb[i][k] = yarr(A.Yb[i], 0, k);
    for (int k = 0; k < 4; ++k)
      if ((st0 = lin(yb[0][k], 0, 0.0, {}, np)) != QSA_OK) return st0;
    int cur = 0, hset = AH0;
    for (int cidx = A.nseg - 1; cidx >= 0; --cidx) {
      const int j0 = cidx * A.ck_len, j1 = std::min(p.nxi, j0 + A.ck_len);
      // recompute the segment from its checkpoint
      R* y0[4];
      for (int k = 0; k < 4; ++k) y0[k] = yarr(A.segY, 0, k);
      if ((st0 = load_ck(t, cidx, y0)) != QSA_OK) return st0;
      for (int i = 0; i < j1 - j0; ++i) {
        R* yi[4];
        R* yo[4];
        for (int k = 0; k < 4; ++k) {
          yi[k] = yarr(A.segY, i, k);
          yo[k] = (i + 1 < j1 - j0) ? yarr(A.segY, i + 1, k) : yarr(A.ytmp, 0, k);
        }
        if ((st0 = fwd_slice(t, j0 + i, yi, yo, i)) != QSA_OK) return st0;
      }
      for (int j = j1 - 1; j >= j0; --j) {
        R* yj[4];
        for (int k = 0; k < 4; ++k) yj[k] = yarr(A.segY, j - j0, k);
        const int other = (hset == AH0) ? AH1 : AH0;
        if ((st0 = rev_slice(t, j, j - j0, yj, yb[cur], yb[1 - cur], hset, other)) != QSA_OK) return st0;
        cur = 1 - cur;
        hset = other;
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
    return b;
  }

  qsa_status sources(int t) {
    qsa_status st0 = lin(c->at<R>(A.src), 0, 0.0, {}, 4 * plane);
    if (st0 != QSA_OK) return st0;
    for (int s = 0; s < p.n_species; ++s) {
      if (c->beam_n[s] == 0) continue;
      hipLaunchKernelGGL(k_ab_sources<R>, dim3(blocks(c->beam_n[s])), dim3(256), 0, st(), beam_args(t, s));
    }
    HIP_OK(hipGetLastError());
    return QSA_OK;
  }

  qsa_status run(int nsteps, int nb, double* loss, double* grad) {
    qsa_status st0;
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
    if ((st0 = lin(c->at<R>(A.fb), 0, 0.0, {}, N_STORED * plane)) != QSA_OK) return st0;
    if ((st0 = lin(fbar(F_BX, 0), 0, 0.0, {{field(nsteps, F_BX, 0), dV}}, plane)) != QSA_OK) return st0;
    if ((st0 = lin(fbar(F_BY, 0), 0, 0.0, {{field(nsteps, F_BY, 0), dV}}, plane)) != QSA_OK) return st0;
    for (int s = 0; s < p.n_species; ++s)
      for (int k = 0; k < 7; ++k)
        if (c->beam_n[s] > 0 && (st0 = lin(c->at<R>(A.bb[s][k]), 0, 0.0, {}, c->beam_n[s])) != QSA_OK) return st0;
    // reverse
    for (int t = nsteps; t >= 0; --t) {
      if ((st0 = sources(t)) != QSA_OK) return st0;
      if ((st0 = rev_sweep(t)) != QSA_OK) return st0;
      for (int s = 0; s < p.n_species; ++s) {
        if (c->beam_n[s] == 0) continue;
        hipLaunchKernelGGL(k_ab_sources_adj<R>, dim3(blocks(c->beam_n[s])), dim3(256), 0, st(), beam_args(t, s));
      }
      if (t > 0) {
        if ((st0 = lin(c->at<R>(A.fb), 0, 0.0, {}, N_STORED * plane)) != QSA_OK) return st0;
        for (int s = 0; s < p.n_species; ++s) {
          if (c->beam_n[s] == 0) continue;
          hipLaunchKernelGGL(k_ab_push_adj<R>, dim3(blocks(c->beam_n[s])), dim3(256), 0, st(),
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
