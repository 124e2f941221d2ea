// Continuous batching of faddeev solves against one resident P0 (serving).
//
// A batch owns max_slots energy slots; slot s uses the columns s*n_open .. s*n_open + n_open - 1
// of the solve vectors (one column per open initial channel). Admission computes the slot's G1
// on the device (FP64) straight into the slot's columns and builds the slot's right-hand side
// b = P0 (v O^T) e0 with column-range kernels, so live slots are not disturbed.
//   FP64 batches: a step advances every column by `terms` Neumann terms with the same launches as
//     faddeev_solve; finished or free slots get G1 = 0, which keeps their vectors at zero.
//   Mixed batches: a step is one refinement cycle (FP64 residual, refine_every Arnoldi steps in
//     mixed precision, correction, captured U) over every column; a new slot starts from y = 0,
//     so its first residual is b exactly, and finished slots take no correction.
// The kernels are column-wise with a fixed reduction order, so a slot's FP64 numbers do not
// depend on which other slots are live; in a mixed batch the block-level partial sums of the
// Gram-Schmidt products are also per column, so the same holds there.
#include <algorithm>
#include <memory>

#include "wpcd_objects.h"

struct wp_batch {
  wp_lattice* L = nullptr;
  wp_solve_opts o{};
  bool mixed = false;
  int slots = 0, nfin = 0, B = 0, max_terms = 0, m = 0;
  int64_t D = 0;
  // FP64 path
  DBuf<double2> dG, dy, ds, dacap;
  DBuf<int> dj0, dfin;
  // mixed path
  MixedWork mw;
  // both
  DBuf<int> dg0;
  DBuf<double> dE;    // three-body energy of each slot
  DBuf<int64_t> g1w;  // G1 work list for one energy
  std::vector<int> j0, g0;
  struct Slot {
    bool live = false, done = false, fresh = true;
    EnergyResult r;
    std::vector<ColState> cs;
    std::vector<MixedCol> mc;
  };
  std::vector<Slot> s;
  std::vector<double2> hcap;
  // pinned staging of each slot's energy and on-shell bins (written only when the slot is
  // admitted again, by which time its previous copy has run)
  double* hE = nullptr;
  int* hj0 = nullptr;
  size_t per_slot = 0;
  ~wp_batch() {
    if (hE) (void)hipHostFree(hE);
    if (hj0) (void)hipHostFree(hj0);
  }
};

// Device bytes one slot of a batch takes (its columns of every solve vector).
static size_t slot_bytes(const wp_lattice* L, const wp_solve_opts& o, int m, int max_terms) {
  const int nfin = (int)L->opens.size();
  const int64_t D = (int64_t)L->M * L->N * L->nch;
  return o.mode != WP_SOLVE_FP64 ? (size_t)nfin * mixed_bytes_per_column(L, m)
                                 : (size_t)nfin * (3 * D * sizeof(double2) + max_terms * nfin * sizeof(double2));
}

extern "C" wp_status faddeev_batch_slot_bytes(const wp_lattice* L, const wp_solve_opts* o, size_t* bytes) {
  if (!L || !o || !bytes) return fail(WP_EINVAL, "NULL argument");
  const int m = std::max(2, std::min(ARN_NV, o->refine_every > 0 ? o->refine_every : 8));
  *bytes = slot_bytes(L, *o, m, 64);
  return WP_OK;
}

extern "C" wp_status faddeev_batch_create(wp_lattice* L, int max_slots, size_t hbm_budget, const wp_solve_opts* o,
                                          wp_batch** out) {
  if (!L || !o || !out || max_slots < 1) return fail(WP_EINVAL, "faddeev_batch_create: bad argument");
  *out = nullptr;
  if (!L->pseudo || !L->have_P) return fail(WP_ENOTREADY, "lattice needs pseudostates and P0");
  if (o->mode != WP_SOLVE_FP64 && o->mode != WP_SOLVE_MIXED && o->mode != WP_SOLVE_MIXED_SPLIT)
    return fail(WP_EINVAL, "unknown solve mode");
  if (!L->d_val64.p) return fail(WP_ENOTREADY, "batch needs P0 built with WP_P_FP64");
  if (o->tol <= 0 || o->accept <= 0 || o->max_iter < 4) return fail(WP_EINVAL, "bad solve options");
  if (wp_status st = upload_waves(L)) return st;
  if (wp_status st = ensure_order(L, nullptr)) return st;
  HIPCHECK(hipStreamSynchronize(nullptr));   // the order is ready before any step, on any stream
  std::unique_ptr<wp_batch> b(new wp_batch());
  b->L = L;
  b->o = *o;
  b->mixed = o->mode != WP_SOLVE_FP64;
  b->nfin = (int)L->opens.size();
  b->D = (int64_t)L->M * L->N * L->nch;
  b->max_terms = 64;
  b->m = std::max(2, std::min(ARN_NV, o->refine_every > 0 ? o->refine_every : 8));
  const size_t per_slot = slot_bytes(L, *o, b->m, b->max_terms);
  b->per_slot = per_slot;
  int cap = (int)std::min<size_t>((size_t)max_slots, hbm_budget / std::max<size_t>(per_slot, 1));
  if (cap < 1) return fail(WP_EBUDGET, "hbm_budget smaller than one slot");
  b->slots = cap;
  b->B = cap * b->nfin;
  const int B = b->B;
  DevAlloc* al = &L->al;
  if (!b->dg0.make(al, B) || !b->dE.make(al, cap) || !g1_work(L, cap, b->g1w))
    return fail(WP_ENOMEM, "device allocation (batch)");
  HIPCHECK(hipHostMalloc((void**)&b->hE, cap * sizeof(double), hipHostMallocDefault));
  HIPCHECK(hipHostMalloc((void**)&b->hj0, B * sizeof(int), hipHostMallocDefault));
  b->j0.assign(B, 0);
  b->g0.assign(B, 0);
  for (int c = 0; c < B; ++c) b->g0[c] = L->opens[c % b->nfin];
  HIPCHECK(hipMemcpy(b->dg0.p, b->g0.data(), B * sizeof(int), hipMemcpyHostToDevice));
  if (b->mixed) {
    if (wp_status st = ensure_mixed(L, nullptr)) return st;
    if (wp_status st = b->mw.make(L, B, b->m, o->mode == WP_SOLVE_MIXED_SPLIT)) return st;
    b->mw.step_tile = o->step_tile;
    b->mw.spmm_cols = o->spmm_cols;
    b->mw.graph = false;   // the batch's active columns change between cycles
    MixedWork& w = b->mw;
    for (auto* p : {&w.dG64, &w.db, &w.dy}) HIPCHECK(hipMemset(p->p, 0, w.DB * sizeof(double2)));
    HIPCHECK(hipMemset(w.dG32.p, 0, w.DB * sizeof(float2)));
    HIPCHECK(hipMemcpy(w.dj0.p, b->j0.data(), B * sizeof(int), hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(w.dfin.p, L->opens.data(), b->nfin * sizeof(int), hipMemcpyHostToDevice));
  } else {
    if (!b->dG.make(al, b->D * B) || !b->dy.make(al, b->D * B) ||
        !b->ds.make(al, b->D * B) || !b->dacap.make(al, (size_t)b->max_terms * B * b->nfin) || !b->dj0.make(al, B) ||
        !b->dfin.make(al, b->nfin))
      return fail(WP_ENOMEM, "device allocation (batch)");
    for (auto* p : {&b->dG, &b->dy, &b->ds}) HIPCHECK(launch_fill0(p->p, b->D * B, nullptr));
    HIPCHECK(hipMemcpy(b->dj0.p, b->j0.data(), B * sizeof(int), hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(b->dfin.p, L->opens.data(), b->nfin * sizeof(int), hipMemcpyHostToDevice));
    b->hcap.resize((size_t)b->max_terms * B * b->nfin);
  }
  HIPCHECK(hipDeviceSynchronize());
  b->s.resize(cap);
  *out = b.release();
  return WP_OK;
}

extern "C" wp_status faddeev_batch_live(const wp_batch* b, int* n) {
  if (!b || !n) return fail(WP_EINVAL, "NULL argument");
  int c = 0;
  for (auto& s : b->s) c += s.live;
  *n = c;
  return WP_OK;
}

// Admits E_lab[0 .. n) in order into the first run of adjacent free slots (as many as it
// holds), with one G1 launch and one right-hand-side product for all of them, on stream st.
static wp_status admit_run(wp_batch* b, int n, const double* E_lab, hipStream_t st, int* slots, int* n_admitted) {
  *n_admitted = 0;
  int sl0 = -1;
  for (int k = 0; k < b->slots; ++k)
    if (!b->s[k].live) {
      sl0 = k;
      break;
    }
  if (sl0 < 0 || n < 1) return WP_OK;
  int k = 0;
  while (k < n && sl0 + k < b->slots && !b->s[sl0 + k].live) ++k;
  wp_lattice* L = b->L;
  // kinematics first: a bad energy admits nothing
  std::vector<EnergyResult> rs(k);
  for (int e = 0; e < k; ++e)
    if (!kinematics(L, E_lab[e], rs[e])) return fail(WP_EINVAL, "on-shell momentum outside the q lattice");
  const int nf = b->nfin, c0 = sl0 * nf, c1 = (sl0 + k) * nf, B = b->B;
  const int64_t R = (int64_t)L->M * L->N;
  for (int e = 0; e < k; ++e) {
    auto& S = b->s[sl0 + e];
    S = wp_batch::Slot();
    S.r = rs[e];
    b->hE[sl0 + e] = S.r.E;
    for (int f = 0; f < nf; ++f) b->j0[c0 + e * nf + f] = b->hj0[c0 + e * nf + f] = S.r.j0;
  }
  HIPCHECK(hipMemcpyAsync(b->dE.p + sl0, b->hE + sl0, k * sizeof(double), hipMemcpyHostToDevice, st));
  if (b->mixed) {
    MixedWork& w = b->mw;
    WP_LAUNCH("g1", st, launch_g1(g1_args(L, b->dE.p + sl0, k, nf, c0, B, w.dG64.p, b->g1w.p), st));
    HIPCHECK(launch_cvt_d2f_cols(b->D, B, c0, c1, w.dG64.p, w.dG32.p, st));
    HIPCHECK(hipMemcpyAsync(w.dj0.p + c0, b->hj0 + c0, (c1 - c0) * sizeof(int), hipMemcpyHostToDevice, st));
    HIPCHECK(launch_init_rhs64(L->M, L->N, L->nch, B, L->d_W.p, L->d_wave.p, w.dj0.p, b->dg0.p, w.ds64.p, st, c0, c1));
    WP_LAUNCH("spmv_f32v_f64x", st,
              launch_spmv_f32v_f64x(R, L->nch, B, L->d_rowptr.p, L->d_col.p, L->d_val32.p, w.ds64.p, w.db.p, st, c0,
                                    c1, spmv_order(L), pk_view(L, b->o.spmm_cols)));
    HIPCHECK(launch_fill0_cols(w.dy.p, b->D, B, c0, c1, st));
    for (int e = 0; e < k; ++e) b->s[sl0 + e].mc.assign(nf, MixedCol());
  } else {
    WP_LAUNCH("g1", st, launch_g1(g1_args(L, b->dE.p + sl0, k, nf, c0, B, b->dG.p, b->g1w.p), st));
    HIPCHECK(hipMemcpyAsync(b->dj0.p + c0, b->hj0 + c0, (c1 - c0) * sizeof(int), hipMemcpyHostToDevice, st));
    HIPCHECK(launch_init_rhs64(L->M, L->N, L->nch, B, L->d_W.p, L->d_wave.p, b->dj0.p, b->dg0.p, b->ds.p, st, c0, c1));
    WP_LAUNCH("spmv64", st,
              launch_spmv_f64(R, L->nch, B, L->d_rowptr.p, L->d_col.p, L->d_val64.p, b->ds.p, b->dy.p, st, c0, c1,
                              spmv_order(L), pk_view(L, b->o.spmm_cols)));
    for (int e = 0; e < k; ++e) {
      auto& S = b->s[sl0 + e];
      S.cs.resize(nf);
      for (auto& c : S.cs) {
        c.w.resize(nf);
        c.S.assign(nf, cplx(0, 0));
      }
    }
  }
  for (int e = 0; e < k; ++e) {
    b->s[sl0 + e].live = true;
    slots[e] = sl0 + e;
  }
  *n_admitted = k;
  return WP_OK;
}

extern "C" wp_status faddeev_batch_admit_many(wp_batch* b, int n, const double* E_lab, void* stream, int* slots,
                                              int* n_admitted) {
  if (!b || !E_lab || !slots || !n_admitted || n < 0) return fail(WP_EINVAL, "NULL argument");
  *n_admitted = 0;
  for (int e = 0; e < n; ++e)
    if (!(E_lab[e] > 0)) return fail(WP_EINVAL, "E_lab must be positive");
  hipStream_t st = (hipStream_t)stream;
  int done = 0;
  while (done < n) {   // one run of adjacent free slots per pass
    int got = 0;
    if (wp_status s = admit_run(b, n - done, E_lab + done, st, slots + done, &got)) return s;
    if (got == 0) break;
    done += got;
  }
  *n_admitted = done;
  return WP_OK;
}

extern "C" wp_status faddeev_batch_admit(wp_batch* b, double E_lab, int* slot) {
  if (!b || !slot) return fail(WP_EINVAL, "NULL argument");
  if (!(E_lab > 0)) return fail(WP_EINVAL, "E_lab must be positive");
  int got = 0;
  if (wp_status s = admit_run(b, 1, &E_lab, nullptr, slot, &got)) return s;
  if (got == 0) return fail(WP_EBUDGET, "no free slot within the batch's device-memory budget");
  HIPCHECK(hipStreamSynchronize(nullptr));
  return WP_OK;
}

static void finish_slot(wp_batch* b, wp_batch::Slot& S) {
  const int nf = b->nfin;
  S.done = true;
  for (int f0 = 0; f0 < nf; ++f0) {
    if (b->mixed) {
      const MixedCol& c = S.mc[f0];
      for (int f = 0; f < nf; ++f) S.r.U[f * nf + f0] = c.U.empty() ? cplx(0, 0) : c.U[f];
      S.r.err[f0] = c.err;
      S.r.iters[f0] = c.iters;
      S.r.ok &= c.err <= b->o.accept;
    } else {
      ColState& cs = S.cs[f0];
      const std::vector<cplx>& est = cs.best.empty() ? cs.last : cs.best;
      for (int f = 0; f < nf; ++f) S.r.U[f * nf + f0] = est[f];
      S.r.err[f0] = cs.err;
      S.r.iters[f0] = cs.n;
      S.r.series[f0] = std::move(cs.terms);
      S.r.ok &= cs.ok;
    }
  }
}

static wp_status step_mixed(wp_batch* b, hipStream_t st, int* n_done, int* done_slots) {
  const int nf = b->nfin, B = b->B, m = b->m;
  const double tol = std::max(b->o.tol, 1e-15);
  std::vector<char> active(B, 0);
  bool y_zero = true;
  for (int sl = 0; sl < b->slots; ++sl) {
    const auto& S = b->s[sl];
    if (!S.live || S.done) continue;
    for (int f = 0; f < nf; ++f) active[sl * nf + f] = S.mc[f].err > tol ? 1 : 0;
    y_zero &= S.fresh;
  }
  if (wp_status s = mixed_cycle(b->mw, st, y_zero, active)) return s;
  for (int sl = 0; sl < b->slots; ++sl) {
    auto& S = b->s[sl];
    if (!S.live || S.done) continue;
    bool all = true;
    for (int f0 = 0; f0 < nf; ++f0) {
      MixedCol& c = S.mc[f0];
      const int col = sl * nf + f0;
      if (active[col]) {
        c.iters += m + (y_zero ? 0 : 1);
        c.update(&b->mw.hc[(size_t)col * nf], nf, tol);
      }
      all &= c.err <= tol || c.iters >= b->o.max_iter;
    }
    S.fresh = false;
    if (all) {
      finish_slot(b, S);
      if (done_slots) done_slots[*n_done] = sl;
      ++*n_done;
    }
  }
  return WP_OK;
}

extern "C" wp_status faddeev_batch_step(wp_batch* b, void* stream, int terms, int* n_done, int* done_slots) {
  if (!b || !n_done) return fail(WP_EINVAL, "NULL argument");
  if (terms < 1 || terms > b->max_terms) return fail(WP_EINVAL, "terms must be in [1, 64]");
  hipStream_t st = (hipStream_t)stream;
  wp_lattice* L = b->L;
  const int M = L->M, N = L->N, nch = L->nch, B = b->B, nf = b->nfin;
  *n_done = 0;
  bool any = false;
  for (auto& s : b->s) any |= (s.live && !s.done);
  if (!any) return WP_OK;
  if (b->mixed) return step_mixed(b, st, n_done, done_slots);
  for (int t = 0; t < terms; ++t) {
    RotArgs ro{M, N, nch, B, L->d_O.p, L->d_wave.p, b->dG.p, b->dacap.p, b->dj0.p, b->dfin.p, nf, (int64_t)t * B * nf};
    ro.tile = b->o.step_tile;
    WP_LAUNCH("step64", st, launch_step64(ro, L->d_W.p, b->dy.p, b->ds.p, st));
    WP_LAUNCH("spmv64", st, launch_spmv_f64((int64_t)M * N, nch, B, L->d_rowptr.p, L->d_col.p, L->d_val64.p, b->ds.p,
                                            b->dy.p, st, 0, -1, spmv_order(L), pk_view(L, b->o.spmm_cols)));
  }
  HIPCHECK(hipMemcpyAsync(b->hcap.data(), b->dacap.p, (size_t)terms * B * nf * sizeof(double2), hipMemcpyDeviceToHost,
                          st));
  HIPCHECK(hipStreamSynchronize(st));
  for (int sl = 0; sl < b->slots; ++sl) {
    auto& S = b->s[sl];
    if (!S.live || S.done) continue;
    bool all = true;
    for (int f0 = 0; f0 < nf; ++f0) {
      ColState& cs = S.cs[f0];
      const int c = sl * nf + f0;
      for (int t = 0; t < terms && !cs.done; ++t) {
        if (cs.n >= b->o.max_iter) {
          cs.done = true;
          cs.ok = cs.best_r <= b->o.accept;
          cs.err = cs.best_r;
          break;
        }
        std::vector<cplx> a(nf);
        for (int f = 0; f < nf; ++f) {
          double2 v = b->hcap[((size_t)t * B + c) * nf + f];
          a[f] = cplx(v.x, v.y);
        }
        column_push(cs, a.data(), nf, b->o.tol, b->o.accept);
      }
      all &= cs.done;
    }
    if (all) {
      finish_slot(b, S);
      // finished: G1 = 0 on the slot's columns keeps its vectors at zero until it is reused
      HIPCHECK(launch_fill0_cols(b->dG.p, b->D, b->B, sl * nf, sl * nf + nf, st));
      if (done_slots) done_slots[*n_done] = sl;
      ++*n_done;
    }
  }
  HIPCHECK(hipStreamSynchronize(st));
  return WP_OK;
}

extern "C" wp_status faddeev_batch_take(wp_batch* b, int slot, wp_solution** out) {
  if (!b || !out || slot < 0 || slot >= b->slots) return fail(WP_EINVAL, "bad argument");
  *out = nullptr;
  auto& S = b->s[slot];
  if (!S.live || !S.done) return fail(WP_ENOTREADY, "slot has no finished result");
  std::unique_ptr<wp_solution> sol(new wp_solution());
  sol->h2m = b->L->h2m;
  sol->res.push_back(S.r);
  const bool ok = S.r.ok;
  S = wp_batch::Slot();
  *out = sol.release();
  return ok ? WP_OK : fail(WP_ENOCONV, "slot's solve was not accepted (result still returned)");
}

extern "C" void faddeev_batch_free(wp_batch* b) { delete b; }
