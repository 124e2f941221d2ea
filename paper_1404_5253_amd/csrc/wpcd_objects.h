// Handle objects of libwpcd shared by the C-ABI translation units (capi.cpp, batch.cpp).
#pragma once

#include <cmath>
#include <memory>
#include <mutex>
#include <string>

#include "wpcd_internal.h"

namespace wpcd {
struct MixedWork;

// A HIP graph captured once and replayed while its key (every pointer, size and choice the
// captured launches depend on) is unchanged.
struct GraphCache {
  std::vector<int64_t> key;
  hipGraphExec_t exec = nullptr;
  GraphCache() = default;
  GraphCache(const GraphCache&) = delete;
  GraphCache& operator=(const GraphCache&) = delete;
  ~GraphCache() { reset(); }
  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    exec = nullptr;
    key.clear();
  }
};
}
using namespace wpcd;

#define HIPCHECK(expr)                                                                                     \
  do {                                                                                                     \
    hipError_t e_ = (expr);                                                                                \
    if (e_ != hipSuccess) return wpcd::fail(WP_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct PairWave {
  int l, s;
  std::vector<double> eps, O, v, W;  // O rows = eigenvectors; W = v O^T
  int nb = 0;
  std::vector<double> bins;          // continuum pseudostate momentum bins
};

struct wp_lattice {
  DevAlloc al;
  int M = 0, N = 0, nch = 0, two_J = 1, n_x = 8, n_phi = 8;
  double h2m = 41.471;
  int weights = WP_WEIGHTS_UNIT;
  std::vector<double> pe, qe;
  std::vector<Chan> ch;
  std::vector<MomKey> keys;
  std::vector<double> C;          // [nch][nch][nmom]
  int nz_pairs = 0;
  // pseudostates
  bool pseudo = false;
  std::vector<PairWave> waves;
  std::vector<int> wave_of;
  std::vector<int> opens;
  double eps0 = 0.0, strength = 0.0;
  // device tables
  DBuf<double> d_pe, d_qe, d_gx, d_gwx, d_gp, d_gwp, d_C, d_O, d_W;
  DBuf<int> d_keys, d_wave;
  // G1 tables: continuum bins per wave, bound states, quadrature rules
  DBuf<double> d_bins, d_epsb, d_ts_u, d_ts_v, d_ts_w, d_gl_x, d_gl_w;
  DBuf<int> d_nb;
  int nts = 0, ngl = 0;
  // mixed precision: bf16 copies of O and v O^T (padded to Mp), FP32 P0 values
  int Mp = 0;
  DBuf<uint16_t> d_Ob, d_Wb, d_Ob_lo, d_Wb_lo;
  // P0
  bool have_P = false;
  int prec = WP_P_FP64;
  int64_t blocks = 0;
  DBuf<int64_t> d_rowptr;
  DBuf<int32_t> d_col;
  DBuf<int32_t> d_order;   // block rows by decreasing length: SpMV work order
  bool order_ok = false;   // d_order holds the order of the resident P0 (or it is enqueued)
  hipEvent_t order_ev = nullptr;   // recorded after the order kernel
  std::mutex order_mu;
  DBuf<char> scratch_sel, scratch_cand;   // P0 build scratch kept between builds (grow-only)
  // Solve workspaces reused across calls (grow-only) by the call that holds ws_mu; a call that
  // finds it held (another thread on this lattice) allocates its own.
  std::mutex ws_mu;
  struct Solve64WS {
    DBuf<double2> dG, dy, ds, dacap;
    DBuf<int> dj0, dg0, dfin;
    DBuf<double> dE;
    DBuf<int64_t> g1w;
    wpcd::GraphCache chunk_graph[2];   // one full chunk of terms per capture slot
  } ws64;
  hipStream_t cap_stream = nullptr;   // graph capture (default priority, non-blocking)
  std::mutex cap_mu;
  std::shared_ptr<wpcd::MixedWork> mws;
  int64_t cand_cap = 0;                   // candidate blocks scratch_cand holds
  int64_t* h_tot = nullptr;               // pinned: the two totals of the last build
  hipEvent_t build_ev[2] = {nullptr, nullptr};   // start and end of a build (device time)
  // pinned host staging of the captured series terms (FP64 solve), reused across calls
  std::mutex pin_mu;
  double2* pin = nullptr;
  size_t pin_cap = 0;
  ~wp_lattice() {
    if (pin) (void)hipHostFree(pin);
    if (h_tot) (void)hipHostFree(h_tot);
    if (order_ev) (void)hipEventDestroy(order_ev);
    for (hipEvent_t e : build_ev)
      if (e) (void)hipEventDestroy(e);
    ws64.chunk_graph[0].reset();
    ws64.chunk_graph[1].reset();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
  }
  DBuf<double> d_val64;
  DBuf<float> d_val32;
  wp_perm_stats stats{};
  // packed block storage for many channels (nch > 4): vpb values per stored block; per packed
  // value its candidate-block entry (row-major g * nch + g') and its block position (u * nch + r)
  PackDesc pk;
  int vpb = 0;
  std::vector<int> pk_src, pk_pos;
  DBuf<int> d_pkt, d_pkpos, d_pksrc;
  // fused many-moment build (FusedArgs): factor-table extents, per moment its table offsets, per
  // stored value its nonzero coefficients; fz_ok when the shape fits the fused kernel
  FusedArgs fz{};
  bool fz_ok = false;
  DBuf<int> d_fkey, d_fcptr, d_fcm;
  DBuf<double> d_fcv;
};
inline PackView pk_view(const wp_lattice* L, int spmm_cols = 0) {
  return PackView{L->pk.npk, L->d_pkt.p, L->d_pkpos.p, spmm_cols > 0 ? spmm_cols : 16};
}

struct EnergyResult {
  double E_lab, E, q0, dq0;
  double afac;   // A = afac U: 2 / (3 h2m q0 dq_j0) (unit weights) or 1 / B_j0 (energy weights)
  int j0;
  int n_open;
  std::vector<cplx> U;      // [final][initial]
  std::vector<double> err;  // per initial column
  std::vector<int> iters;
  // FP64 path: the on-shell series terms a_n read for each initial column b, series[b][n * n_open + f]
  std::vector<std::vector<cplx>> series;
  // breakup (mixed modes, on request): the energy-shell cells (g, k, j) and, per initial
  // column, the transition element of each cell
  std::vector<int> bu_cells;
  std::vector<std::vector<cplx>> bu;
  bool ok = true;
};

struct wp_solution {
  double h2m;
  std::vector<EnergyResult> res;
};


namespace wpcd {

#define WP_LAUNCH(name, stream, expr)        \
  do {                                       \
    wpcd::ProfScope ps_(name, stream);       \
    HIPCHECK(expr);                          \
  } while (0)

wp_status fail(wp_status st, const std::string& msg);
wp_status upload_waves(wp_lattice* L);
wp_status ensure_mixed(wp_lattice* L, hipStream_t s);   // bf16 blocks + FP32 copy of P0
wp_status ensure_order(wp_lattice* L, hipStream_t s);   // SpMV row order of the resident P0 (on s)
// Row order the SpMV kernels take: longest rows first for many channels (the LDS-staged kernels),
// lattice order for few (rows of one q bin share their columns; measured faster at 1 to 64 columns).
inline const int32_t* spmv_order(const wp_lattice* L) { return L->nch > 4 ? L->d_order.p : nullptr; }

// ------------------------------------------------------------------ mixed path (mixed.cpp)
constexpr int kNblk = 1024;   // workgroups of the column reductions (4 per CU)
// device and host work space of the mixed refinement for B columns
struct MixedWork {
  wp_lattice* L = nullptr;
  int B = 0, m = 0, nfin = 0;
  int64_t R = 0, D = 0, DB = 0;
  bool fused = false, split = false;
  DBuf<double2> dG64, db, dy, dr, dKy, ds64, dcap, dcoef, H, part, nrm;
  DBuf<float2> dG32, V, t32, kv32;
  DBuf<double> scl;
  DBuf<int> dj0, dfin, dg0;
  DBuf<double> dE;        // energies, G1 work list: used by solve_mixed only
  DBuf<int64_t> g1w;
  std::vector<double2> hc, hH, hn, coef;
  std::vector<double> hsc;
  // launch choices of the current call (wp_solve_opts) and the graphs of the Arnoldi sweep
  // (index: the first cycle, whose residual is b, or a later one)
  int step_tile = 0, spmm_cols = 0;
  bool graph = false;
  GraphCache sweep_graph[2];
  wp_status make(wp_lattice* L, int B, int m, bool split);
};
// Enqueues record(stream) on s as a HIP graph: captured on the lattice's capture stream when the
// cache is empty or its key differs, then launched on s. record must only enqueue work (no host
// synchronisation) and return hipSuccess.
template <typename F>
hipError_t graph_run(wp_lattice* L, GraphCache& g, const std::vector<int64_t>& key, hipStream_t s, F record);
bool profiling_enabled();
// per-column state of the refinement's stop rule
struct MixedCol {
  std::vector<cplx> U;
  double dprev = -1.0, err = 1.0;
  int iters = 0;
  bool update(const double2* u_new, int nfin, double tol);
};
size_t mixed_bytes_per_column(const wp_lattice* L, int m);
wp_status mixed_cycle(MixedWork& w, hipStream_t s, bool y_is_zero, const std::vector<char>& active);
wp_status solve_mixed(wp_lattice* L, const std::vector<double>& Elab, const wp_solve_opts& o, hipStream_t s,
                      wp_solution* sol);
std::vector<int> shell_cells(const wp_lattice* L, double E);   // breakup cells (g, k, j) at energy E
// Device work list of the G1 kernels for nE energies (element list plus counter in slot 0).
bool g1_work(wp_lattice* L, int nE, DBuf<int64_t>& w);
// G1 arguments for energies dE[nE] written to columns col0 + e*nrep + f of G (B columns); work: the
// work list (counter in slot 0, then g1_work_elems entries)
G1Args g1_args(const wp_lattice* L, const double* dE, int nE, int nrep, int col0, int B, double2* G,
               int64_t* work);

// Kinematics of one energy: E, q0, on-shell bin j0 ((q_{j-1}, q_j] convention), its width.
inline bool kinematics(const wp_lattice* L, double E_lab, EnergyResult& r) {
  r.E_lab = E_lab;
  r.E = L->eps0 + 2.0 * E_lab / 3.0;
  r.q0 = std::sqrt(4.0 * (2.0 * E_lab / 3.0) / (3.0 * L->h2m));
  int jj = -1;
  for (int j = 0; j < L->N; ++j)
    if (L->qe[j] < r.q0 && r.q0 <= L->qe[j + 1]) jj = j;
  if (jj < 0) return false;
  r.j0 = jj;
  r.dq0 = L->qe[jj + 1] - L->qe[jj];
  r.afac = L->weights == WP_WEIGHTS_ENERGY
               ? 1.0 / (0.75 * L->h2m * (L->qe[jj + 1] * L->qe[jj + 1] - L->qe[jj] * L->qe[jj]))
               : 2.0 / (3.0 * L->h2m * r.q0) / r.dq0;
  r.n_open = (int)L->opens.size();
  r.U.assign(r.n_open * r.n_open, cplx(0, 0));
  r.err.assign(r.n_open, 0.0);
  r.iters.assign(r.n_open, 0);
  r.series.assign(r.n_open, std::vector<cplx>());
  r.ok = true;
  return true;
}

// Pade (Wynn epsilon) state of one column (energy x initial channel) over its final channels,
// with the stop rule: two successive relative changes <= tol, or a rounding plateau (no new
// minimum of the change for PLATEAU terms, or partial sums above 1e250) accepted when the
// smallest change <= accept.
struct ColState {
  std::vector<Wynn> w;      // per final
  std::vector<cplx> S, last, best;
  double best_r = INFINITY;
  double r_last = INFINITY;   // relative change at the newest term
  int best_n = 0, streak = 0, n = 0, plateau = 24;
  bool done = false, ok = false;
  double err = 0.0;
  std::vector<cplx> terms;    // every term pushed, [n][final]
};
constexpr int PLATEAU = 24;

// One term of the on-shell series of every final for a column; returns true when finished.
inline bool column_push(ColState& cs, const cplx* a, int nfin, double tol, double accept) {
  std::vector<cplx> est(nfin);
  double Smax = 0.0;
  cs.terms.insert(cs.terms.end(), a, a + nfin);
  for (int f = 0; f < nfin; ++f) {
    cs.S[f] += a[f];
    est[f] = cs.w[f].push(cs.S[f]);
    Smax = std::max(Smax, std::abs(cs.S[f]));
  }
  if (cs.n > 0) {
    double r = 0.0;
    for (int f = 0; f < nfin; ++f) r = std::max(r, std::abs(est[f] - cs.last[f]) / std::max(std::abs(est[f]), 1e-300));
    cs.r_last = r;
    if (r < cs.best_r) {
      cs.best_r = r;
      cs.best = est;
      cs.best_n = cs.n;
    }
    cs.streak = (r <= tol) ? cs.streak + 1 : 0;
    if (cs.streak >= 2) {
      cs.best = est;
      cs.err = r;
      cs.done = cs.ok = true;
    } else if (cs.n - cs.best_n >= cs.plateau || Smax > 1e250) {
      cs.done = true;
      cs.ok = cs.best_r <= accept;
      cs.err = cs.best_r;
    }
  }
  cs.last = est;
  cs.n++;
  return cs.done;
}


template <typename F>
hipError_t graph_run(wp_lattice* L, GraphCache& g, const std::vector<int64_t>& key, hipStream_t s, F record) {
  if (!g.exec || g.key != key) {
    g.reset();
    std::lock_guard<std::mutex> lk(L->cap_mu);   // one capture at a time on the lattice's stream
    if (!L->cap_stream) {
      const hipError_t e = hipStreamCreateWithFlags(&L->cap_stream, hipStreamNonBlocking);
      if (e != hipSuccess) return e;
    }
    hipError_t e = hipStreamBeginCapture(L->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    const hipError_t er = record(L->cap_stream);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(L->cap_stream, &graph);
    if (er != hipSuccess || e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return er != hipSuccess ? er : e;
    }
    e = hipGraphInstantiateWithFlags(&g.exec, graph, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      g.exec = nullptr;
      return e;
    }
    g.key = key;
  }
  return hipGraphLaunch(g.exec, s);
}

}  // namespace wpcd
