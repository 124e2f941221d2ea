// Mixed-precision solve of y = b + K y (Sec. II.B.4, eq. m_pvg): FP64 iterative refinement around
// a mixed-precision GMRES, shared by faddeev_solve (all energies of a call) and the continuous
// batch (faddeev_batch_*, one refinement cycle per step).
//
//   outer (FP64): r = b - (I - K) y with FP64 blocks and G1 and the FP32-stored P0 accumulated in
//                 FP64 (r = b at y = 0);
//   inner:        m Arnoldi steps on (I - K~) started from r / |r|, K~ = P0(FP32) (v O^T)(BF16,
//                 MFMA) G1(FP32) O(BF16, MFMA); FP32 basis vectors kept unnormalised with FP64
//                 scale factors, classical Gram-Schmidt with FP64 sums (one pass: the outer
//                 refinement absorbs the inner loss of orthogonality); the small least-squares
//                 problem per column on the host in FP64; y += V z;
//   stop:         U = e0^T O y in FP64 after every correction; with D_k the relative change of U
//                 and rho = D_k / D_{k-1} the observed contraction, the error estimate is
//                 D_k rho / (1 - rho); a column stops when it is <= tol.
// A Neumann series in low precision would amplify every term's rounding by the growth of the
// divergent series, which is why the inner solver is orthogonalised.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>

#include "wpcd_objects.h"

using namespace wpcd;

static uint16_t host_bf16(double d) {
  float f = (float)d;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

wp_status wpcd::ensure_mixed(wp_lattice* L, hipStream_t s) {
  if (wp_status st = upload_waves(L)) return st;
  const int M = L->M;
  if (!L->d_Ob.p) {
    // bf16 copies of O and v O^T (hi) and of their rounding remainders (lo), padded to Mp
    const int Mp = (M + 15) / 16 * 16;
    const size_t MM = (size_t)Mp * Mp;
    const size_t n = MM * L->waves.size();
    std::vector<uint16_t> Oh(n, 0), Ol(n, 0), Wh(n, 0), Wl(n, 0);
    auto split = [](double d, uint16_t& hi, uint16_t& lo) {
      hi = host_bf16(d);
      uint32_t u = (uint32_t)hi << 16;
      float f;
      std::memcpy(&f, &u, 4);
      lo = host_bf16((double)((float)d - f));
    };
    for (size_t w = 0; w < L->waves.size(); ++w)
      for (int r = 0; r < M; ++r)
        for (int c = 0; c < M; ++c) {
          const size_t k = w * MM + (size_t)r * Mp + c;
          split(L->waves[w].O[(size_t)r * M + c], Oh[k], Ol[k]);
          split(L->waves[w].W[(size_t)r * M + c], Wh[k], Wl[k]);
        }
    if (!L->d_Ob.make(&L->al, n) || !L->d_Wb.make(&L->al, n) || !L->d_Ob_lo.make(&L->al, n) ||
        !L->d_Wb_lo.make(&L->al, n))
      return fail(WP_ENOMEM, "device allocation (bf16 blocks)");
    HIPCHECK(hipMemcpy(L->d_Ob.p, Oh.data(), n * 2, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(L->d_Wb.p, Wh.data(), n * 2, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(L->d_Ob_lo.p, Ol.data(), n * 2, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(L->d_Wb_lo.p, Wl.data(), n * 2, hipMemcpyHostToDevice));
    L->Mp = Mp;
  }
  if (!L->d_val32.p) {
    const int64_t n = L->blocks * L->vpb;
    if (!L->d_val32.make(&L->al, std::max<int64_t>(n, 1))) return fail(WP_ENOMEM, "device allocation (FP32 P0)");
    if (n > 0) HIPCHECK(launch_cvt_scalar(n, L->d_val64.p, L->d_val32.p, s));
  }
  return WP_OK;
}

// Least squares min || beta e1 - H z || for an (m+1) x m upper Hessenberg H (column-major by j:
// H[j*(m+1) + i]) by Givens rotations; returns z (m entries).
static std::vector<cplx> hessenberg_ls(std::vector<cplx> H, int m, double beta) {
  const int ld = m + 1;
  std::vector<cplx> g(m + 1, cplx(0, 0));
  g[0] = beta;
  for (int j = 0; j < m; ++j) {
    cplx a = H[j * ld + j], bb = H[j * ld + j + 1];
    double r = std::sqrt(std::norm(a) + std::norm(bb));
    if (r == 0.0) continue;
    cplx c = a / r, sn = bb / r;   // rotation [conj(c) conj(s); -s c]
    for (int k = j; k < m; ++k) {
      cplx x = H[k * ld + j], y = H[k * ld + j + 1];
      H[k * ld + j] = std::conj(c) * x + std::conj(sn) * y;
      H[k * ld + j + 1] = -sn * x + c * y;
    }
    cplx x = g[j], y = g[j + 1];
    g[j] = std::conj(c) * x + std::conj(sn) * y;
    g[j + 1] = -sn * x + c * y;
  }
  std::vector<cplx> z(m, cplx(0, 0));
  for (int j = m - 1; j >= 0; --j) {
    cplx v = g[j];
    for (int k = j + 1; k < m; ++k) v -= H[k * ld + j] * z[k];
    z[j] = std::abs(H[j * ld + j]) > 0.0 ? v / H[j * ld + j] : cplx(0, 0);
  }
  return z;
}

size_t wpcd::mixed_bytes_per_column(const wp_lattice* L, int m) {
  const size_t D = (size_t)L->M * L->N * L->nch;
  // FP64: G1, b, y, r, Ky, s; FP32: G1, basis (m + 1), t, Kv
  return D * (6 * sizeof(double2) + (m + 4) * sizeof(float2)) + (size_t)(m + 1) * (m + 2) * 24;
}

wp_status wpcd::MixedWork::make(wp_lattice* Lp, int B_, int m_, bool split_) {
  L = Lp;
  B = B_;
  m = m_;
  split = split_;
  nfin = (int)L->opens.size();
  R = (int64_t)L->M * L->N;
  D = R * L->nch;
  DB = D * B;
  fused = B >= 16 && L->nch <= 4;
  // grow-only, so that a work object kept by the lattice is reused by later calls
  DevAlloc* al = &L->al;
  if (!grow(dG64, al, DB) || !grow(db, al, DB) || !grow(dy, al, DB) || !grow(dr, al, DB) || !grow(dKy, al, DB) ||
      !grow(ds64, al, DB) || !grow(dcap, al, (size_t)B * nfin) || !grow(dcoef, al, (size_t)(m + 1) * B) ||
      !grow(H, al, (size_t)m * (m + 1) * B) || !grow(part, al, (size_t)kNblk * ARN_NV * B) || !grow(nrm, al, B) ||
      !grow(dG32, al, DB) || !grow(V, al, (size_t)(m + 1) * DB) || !grow(t32, al, DB) ||
      (!fused && !grow(kv32, al, DB)) || !grow(scl, al, (size_t)(m + 1) * B) || !grow(dj0, al, B) ||
      !grow(dfin, al, nfin))
    return fail(WP_ENOMEM, "device allocation (mixed solve)");
  hc.resize((size_t)B * nfin);
  hH.resize((size_t)m * (m + 1) * B);
  hn.resize(B);
  hsc.resize((size_t)(m + 1) * B);
  coef.resize((size_t)(m + 1) * B);
  return WP_OK;
}

// One refinement cycle on every column: FP64 residual (skipped when all y = 0), m Arnoldi steps,
// the least-squares corrections of the columns with active[c] (zero for the others), y += V z and
// the captured U of every column (hc, [c][final]).
wp_status wpcd::mixed_cycle(MixedWork& w, hipStream_t s, bool y_is_zero, const std::vector<char>& active) {
  wp_lattice* L = w.L;
  const int M = L->M, N = L->N, nch = L->nch, B = w.B, m = w.m, nfin = w.nfin;
  const int64_t D = w.D, DB = w.DB, R = w.R;
  // the Arnoldi sweep: residual (b itself on the first cycle), its norm and scaling, m Arnoldi
  // steps; replayed from a graph when the call asks for one
  auto record_sweep = [&](hipStream_t st) -> hipError_t {
    hipError_t e = hipSuccess;
    if (y_is_zero) {
      e = hipMemcpyAsync(w.dr.p, w.db.p, DB * sizeof(double2), hipMemcpyDeviceToDevice, st);
      if (e != hipSuccess) return e;
    } else {
      RotArgs ro{M, N, nch, B, L->d_O.p, L->d_wave.p, w.dG64.p, nullptr, w.dj0.p, w.dfin.p, nfin, 0};
      ro.tile = w.step_tile;
      {
        ProfScope ps("step64", st);
        e = launch_step64(ro, L->d_W.p, w.dy.p, w.ds64.p, st);
      }
      if (e != hipSuccess) return e;
      {
        ProfScope ps("spmv_f32v_f64x", st);
        e = launch_spmv_f32v_f64x(R, nch, B, L->d_rowptr.p, L->d_col.p, L->d_val32.p, w.ds64.p, w.dKy.p, st, 0, -1,
                                  spmv_order(L), pk_view(L, w.spmm_cols));
      }
      if (e != hipSuccess) return e;
      {
        ProfScope ps("residual", st);
        e = launch_residual(DB, w.db.p, w.dy.p, w.dKy.p, w.dr.p, st);
      }
      if (e != hipSuccess) return e;
    }
    if ((e = launch_norm2_f64(D, B, w.dr.p, w.part.p, kNblk, w.nrm.p, st)) != hipSuccess) return e;
    if ((e = launch_scale_d2f(D, B, w.nrm.p, w.dr.p, w.V.p, w.scl.p, st)) != hipSuccess) return e;
    ArnoldiArgs aa{R,         nch,     B,      m,    0,          L->d_rowptr.p, L->d_col.p, L->d_val32.p,
                   spmv_order(L), w.V.p, DB,    w.scl.p, w.H.p, w.part.p, kNblk, pk_view(L, w.spmm_cols)};
    RotArgsMixed rm{M,          N, nch, B, L->d_Ob.p, w.split ? L->d_Ob_lo.p : nullptr, L->d_Wb.p,
                    w.split ? L->d_Wb_lo.p : nullptr, L->Mp, L->d_wave.p, w.dG32.p, nullptr};
    for (int j = 0; j < m; ++j) {
      aa.j = j;
      rm.yscale = w.scl.p + (size_t)j * B;
      {
        ProfScope ps("step_bf16", st);
        e = launch_step_bf16(rm, w.V.p + (size_t)j * DB, w.t32.p, st);
      }
      if (e != hipSuccess) return e;
      if ((e = launch_arnoldi_product(aa, w.t32.p, w.kv32.p, st)) != hipSuccess) return e;   // profiled inside
      {
        ProfScope ps("arnoldi_orth", st);
        e = launch_arnoldi_orth(aa, st);
      }
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  if (w.graph && !profiling_enabled()) {
    const std::vector<int64_t> key{
        y_is_zero,          M, N, nch, B, m, w.split, w.step_tile, w.spmm_cols, (int64_t)w.dr.p, (int64_t)w.db.p,
        (int64_t)w.dy.p,    (int64_t)w.ds64.p, (int64_t)w.dKy.p, (int64_t)w.dG64.p, (int64_t)w.dG32.p,
        (int64_t)w.dj0.p,   (int64_t)w.dfin.p, (int64_t)w.part.p, (int64_t)w.nrm.p, (int64_t)w.V.p,
        (int64_t)w.scl.p,   (int64_t)w.H.p, (int64_t)w.t32.p, (int64_t)w.kv32.p, (int64_t)L->d_O.p,
        (int64_t)L->d_W.p,  (int64_t)L->d_wave.p, (int64_t)L->d_Ob.p, (int64_t)L->d_Ob_lo.p, (int64_t)L->d_Wb.p,
        (int64_t)L->d_Wb_lo.p, (int64_t)L->d_rowptr.p, (int64_t)L->d_col.p, (int64_t)L->d_val32.p,
        (int64_t)spmv_order(L), (int64_t)L->d_pkt.p, (int64_t)L->d_pkpos.p};
    HIPCHECK(graph_run(L, w.sweep_graph[y_is_zero ? 0 : 1], key, s, record_sweep));
  } else {
    HIPCHECK(record_sweep(s));
  }
  HIPCHECK(hipMemcpyAsync(w.hn.data(), w.nrm.p, B * sizeof(double2), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipMemcpyAsync(w.hH.data(), w.H.p, w.hH.size() * sizeof(double2), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipMemcpyAsync(w.hsc.data(), w.scl.p, w.hsc.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  std::fill(w.coef.begin(), w.coef.end(), make_double2(0.0, 0.0));
  std::vector<cplx> Hc((size_t)m * (m + 1));
  for (int c = 0; c < B; ++c) {
    if (!active[c]) continue;
    for (int j = 0; j < m; ++j)
      for (int i = 0; i <= m; ++i) {
        const double2 v = w.hH[((size_t)j * (m + 1) + i) * B + c];
        Hc[(size_t)j * (m + 1) + i] = cplx(v.x, v.y);
      }
    const double beta = std::sqrt(std::max(w.hn[c].x, 0.0));
    std::vector<cplx> z = hessenberg_ls(Hc, m, beta);
    for (int i = 0; i < m; ++i) {
      const cplx v = z[i] * w.hsc[(size_t)i * B + c];   // V_i = scl_i Vt_i
      w.coef[(size_t)i * B + c] = make_double2(v.real(), v.imag());
    }
  }
  HIPCHECK(hipMemcpyAsync(w.dcoef.p, w.coef.data(), w.coef.size() * sizeof(double2), hipMemcpyHostToDevice, s));
  WP_LAUNCH("lincomb", s, launch_lincomb(D, B, m, w.V.p, DB, w.dcoef.p, w.dy.p, s));
  WP_LAUNCH("capture", s,
            launch_capture64(M, nch, B, nfin, L->d_O.p, L->d_wave.p, w.dj0.p, w.dfin.p, w.dy.p, w.dcap.p, s));
  HIPCHECK(hipMemcpyAsync(w.hc.data(), w.dcap.p, w.hc.size() * sizeof(double2), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  return WP_OK;
}

// Error estimate of one column after a correction (see the stop rule above); true when done.
bool wpcd::MixedCol::update(const double2* u_new, int nfin, double tol) {
  double change = 0.0, mag = 0.0;
  if (U.size() != (size_t)nfin) U.assign(nfin, cplx(0, 0));
  for (int f = 0; f < nfin; ++f) {
    const cplx u(u_new[f].x, u_new[f].y);
    change = std::max(change, std::abs(u - U[f]));
    mag = std::max(mag, std::abs(u));
    U[f] = u;
  }
  const double d = change / std::max(mag, 1e-300);
  double est = 1.0;
  if (dprev >= 0.0) {
    const double rho = dprev > 0.0 ? d / dprev : 0.0;
    est = rho < 1.0 ? d * std::min(rho / (1.0 - rho), 1e6) : d * 1e6;
    if (d == 0.0) est = 0.0;
  }
  err = std::min(est, 1.0);
  dprev = d;
  return err <= tol;
}

// Breakup cells of three-body energy E: (g, k, j) for every channel g, continuum pseudostate k of
// its pair wave and q bin j whose energy range h2m [p_a^2, p_b^2] + (3/4) h2m [q_a^2, q_b^2] holds
// E strictly inside (the cells where Im G1 != 0).
std::vector<int> wpcd::shell_cells(const wp_lattice* L, double E) {
  std::vector<int> out;
  const double h = L->h2m, b3 = 0.75 * L->h2m;
  for (int g = 0; g < L->nch; ++g) {
    const PairWave& w = L->waves[L->wave_of[g]];
    for (int k = w.nb; k < L->M; ++k) {
      const double pa = w.bins[k - w.nb], pb = w.bins[k - w.nb + 1];
      for (int j = 0; j < L->N; ++j) {
        const double lo = h * pa * pa + b3 * L->qe[j] * L->qe[j];
        const double hi = h * pb * pb + b3 * L->qe[j + 1] * L->qe[j + 1];
        if (lo < E && E < hi) out.insert(out.end(), {g, k, j});
      }
    }
  }
  return out;
}

wp_status wpcd::solve_mixed(wp_lattice* L, const std::vector<double>& Elab, const wp_solve_opts& o, hipStream_t s,
                            wp_solution* sol) {
  const int M = L->M, N = L->N, nch = L->nch;
  const int nfin = (int)L->opens.size();
  const int nE = (int)Elab.size();
  const int B = nE * nfin;
  std::vector<int> j0(B), g0(B);
  std::vector<double> Etot(nE);
  sol->res.resize(nE);
  for (int e = 0; e < nE; ++e) {
    EnergyResult& r = sol->res[e];
    if (!kinematics(L, Elab[e], r)) return fail(WP_EINVAL, "on-shell momentum outside the q lattice");
    Etot[e] = r.E;
    for (int b = 0; b < nfin; ++b) {
      j0[e * nfin + b] = r.j0;
      g0[e * nfin + b] = L->opens[b];
    }
  }
  if (wp_status st = ensure_mixed(L, s)) return st;
  if (wp_status so = ensure_order(L, s)) return so;
  const int m = std::max(2, std::min(ARN_NV, o.refine_every > 0 ? o.refine_every : 8));
  const int max_outer = std::max(2, std::min(100, o.max_iter / (m + 1)));
  // the lattice's work object when no other call holds it, else one of this call's own
  std::unique_lock<std::mutex> ws_lock(L->ws_mu, std::try_to_lock);
  MixedWork own;
  if (ws_lock.owns_lock() && !L->mws) L->mws = std::make_shared<MixedWork>();
  MixedWork& w = ws_lock.owns_lock() ? *L->mws : own;
  StreamDrain drain{s};   // idle stream before the work object is released or handed on
  if (wp_status st = w.make(L, B, m, o.mode == WP_SOLVE_MIXED_SPLIT)) return st;
  w.step_tile = o.step_tile;
  w.spmm_cols = o.spmm_cols;
  w.graph = o.graph == 1;
  DBuf<int>& dg0 = w.dg0;
  DBuf<double>& dE = w.dE;
  DBuf<int64_t>& g1w = w.g1w;
  if (!grow(dg0, &L->al, B) || !grow(dE, &L->al, nE) || !g1_work(L, nE, g1w))
    return fail(WP_ENOMEM, "device allocation (mixed solve)");
  const int64_t DB = w.DB, R = w.R;
  HIPCHECK(hipMemcpyAsync(dE.p, Etot.data(), nE * 8, hipMemcpyHostToDevice, s));
  HIPCHECK(hipMemcpyAsync(w.dj0.p, j0.data(), B * sizeof(int), hipMemcpyHostToDevice, s));
  HIPCHECK(hipMemcpyAsync(dg0.p, g0.data(), B * sizeof(int), hipMemcpyHostToDevice, s));
  HIPCHECK(hipMemcpyAsync(w.dfin.p, L->opens.data(), nfin * sizeof(int), hipMemcpyHostToDevice, s));
  WP_LAUNCH("g1", s, launch_g1(g1_args(L, dE.p, nE, nfin, 0, B, w.dG64.p, g1w.p), s));
  HIPCHECK(launch_cvt_d2f(DB, w.dG64.p, w.dG32.p, s));
  HIPCHECK(launch_init_rhs64(M, N, nch, B, L->d_W.p, L->d_wave.p, w.dj0.p, dg0.p, w.ds64.p, s));
  WP_LAUNCH("spmv_f32v_f64x", s,
            launch_spmv_f32v_f64x(R, nch, B, L->d_rowptr.p, L->d_col.p, L->d_val32.p, w.ds64.p, w.db.p, s, 0, -1,
                                  spmv_order(L), pk_view(L, w.spmm_cols)));
  HIPCHECK(launch_fill0(w.dy.p, DB, s));
  std::vector<MixedCol> col(B);
  std::vector<char> active(B, 1);
  for (int outer = 0; outer < max_outer; ++outer) {
    if (wp_status st = mixed_cycle(w, s, outer == 0, active)) return st;
    bool all = true;
    for (int c = 0; c < B; ++c) {
      if (!active[c]) continue;
      col[c].iters += m + (outer > 0 ? 1 : 0);
      if (col[c].update(&w.hc[(size_t)c * nfin], nfin, std::max(o.tol, 1e-15))) active[c] = 0;
      all &= !active[c];
    }
    if (all) break;
  }
  if (o.breakup == 1) {
    // breakup: (O y) on every energy-shell cell of every column
    std::vector<int4> cells;
    std::vector<int> first(B + 1, 0);
    for (int e = 0; e < nE; ++e) {
      sol->res[e].bu_cells = shell_cells(L, Etot[e]);
      const std::vector<int>& sc = sol->res[e].bu_cells;
      for (int b = 0; b < nfin; ++b) {
        const int c = e * nfin + b;
        first[c] = (int)cells.size();
        for (size_t t = 0; t + 2 < sc.size(); t += 3) cells.push_back(make_int4(c, sc[t], sc[t + 1], sc[t + 2]));
      }
    }
    first[B] = (int)cells.size();
    if (!cells.empty()) {
      DBuf<int4> dcells;
      DBuf<double2> dout;
      if (!dcells.make(&L->al, cells.size()) || !dout.make(&L->al, cells.size()))
        return fail(WP_ENOMEM, "device allocation (breakup cells)");
      std::vector<double2> h(cells.size());
      HIPCHECK(hipMemcpyAsync(dcells.p, cells.data(), cells.size() * sizeof(int4), hipMemcpyHostToDevice, s));
      WP_LAUNCH("breakup", s, launch_project_cells(M, nch, B, L->d_O.p, L->d_wave.p, dcells.p, (int)cells.size(),
                                                  w.dy.p, dout.p, s));
      HIPCHECK(hipMemcpyAsync(h.data(), dout.p, h.size() * sizeof(double2), hipMemcpyDeviceToHost, s));
      HIPCHECK(hipStreamSynchronize(s));
      for (int e = 0; e < nE; ++e) {
        sol->res[e].bu.assign(nfin, {});
        for (int b = 0; b < nfin; ++b) {
          const int c = e * nfin + b;
          auto& v = sol->res[e].bu[b];
          for (int t = first[c]; t < first[c + 1]; ++t) v.emplace_back(h[t].x, h[t].y);
        }
      }
    }
  }
  bool allok = true;
  for (int e = 0; e < nE; ++e) {
    EnergyResult& r = sol->res[e];
    for (int b = 0; b < nfin; ++b) {
      const MixedCol& c = col[e * nfin + b];
      for (int f = 0; f < nfin; ++f) r.U[f * nfin + b] = c.U.empty() ? cplx(0, 0) : c.U[f];
      r.err[b] = c.err;
      r.iters[b] = c.iters;
      r.ok &= c.err <= o.accept;
    }
    allok &= r.ok;
  }
  return allok ? WP_OK : fail(WP_ENOCONV, "mixed refinement did not reach the accepted accuracy for some energy");
}
