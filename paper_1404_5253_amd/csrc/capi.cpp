// C ABI of libwpcd (include/wpcd.h): handles, call order, device memory and the host side of
// the hot path (P0 build orchestration and the iteration / Pade loop).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <stdexcept>
#include <thread>
#include <tuple>

#include "wpcd_objects.h"

using namespace wpcd;

static thread_local std::string g_err;

wp_status wpcd::fail(wp_status st, const std::string& msg) {
  g_err = msg;
  return st;
}


extern "C" const char* wp_last_error(void) { return g_err.c_str(); }

// ------------------------------------------------------------------ launch profiling

namespace {
struct ProfRec {
  const char* name;
  hipEvent_t a, b;
};
struct Profiler {
  std::mutex mu;
  bool on = false;
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<std::string, std::pair<int64_t, double>>> agg;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};
Profiler& prof() {
  static Profiler p;
  return p;
}
}  // namespace

wpcd::ProfScope::ProfScope(const char* n, hipStream_t s) : name(n), st(s) {
  Profiler& p = prof();
  if (!p.on) return;
  std::lock_guard<std::mutex> g(p.mu);
  a = p.get();
  if (a) (void)hipEventRecord(a, st);
}

wpcd::ProfScope::~ProfScope() {
  if (!a) return;
  Profiler& p = prof();
  std::lock_guard<std::mutex> g(p.mu);
  hipEvent_t b = p.get();
  if (!b) return;
  (void)hipEventRecord(b, st);
  p.recs.push_back({name, a, b});
}

bool wpcd::profiling_enabled() { return prof().on; }

extern "C" wp_status wp_profile_enable(int on) {
  prof().on = on != 0;
  return WP_OK;
}

extern "C" wp_status wp_profile_reset(void) {
  Profiler& p = prof();
  std::lock_guard<std::mutex> g(p.mu);
  for (auto& r : p.recs) {
    p.pool.push_back(r.a);
    p.pool.push_back(r.b);
  }
  p.recs.clear();
  p.agg.clear();
  return WP_OK;
}

extern "C" wp_status wp_profile_read(int i, int* n, char* name, int64_t* launches, double* total_ms) {
  Profiler& p = prof();
  std::lock_guard<std::mutex> g(p.mu);
  if (!p.recs.empty()) {
    std::map<std::string, std::pair<int64_t, double>> m;
    for (auto& r : p.recs) {
      HIPCHECK(hipEventSynchronize(r.b));
      float ms = 0.f;
      HIPCHECK(hipEventElapsedTime(&ms, r.a, r.b));
      auto& e = m[r.name];
      e.first += 1;
      e.second += ms;
      p.pool.push_back(r.a);
      p.pool.push_back(r.b);
    }
    p.recs.clear();
    for (auto& kv : p.agg) {
      auto& e = m[kv.first];
      e.first += kv.second.first;
      e.second += kv.second.second;
    }
    p.agg.assign(m.begin(), m.end());
  }
  if (n) *n = (int)p.agg.size();
  if (i < 0) return WP_OK;
  if (i >= (int)p.agg.size()) return fail(WP_EINVAL, "profile index out of range");
  if (name) {
    std::strncpy(name, p.agg[i].first.c_str(), 63);
    name[63] = 0;
  }
  if (launches) *launches = p.agg[i].second.first;
  if (total_ms) *total_ms = p.agg[i].second.second;
  return WP_OK;
}

void* DevAlloc::alloc(size_t bytes) {
  if (bytes == 0) bytes = 1;
  if (custom) return a.alloc(bytes, a.ctx);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  return p;
}
void DevAlloc::release(void* p) {
  if (!p) return;
  if (custom)
    a.release(p, a.ctx);
  else
    (void)hipFree(p);
}

// ------------------------------------------------------------------ lattice

extern "C" wp_status wp_lattice_build(const wp_lattice_desc* d, const wp_allocator* alloc, wp_lattice** out) {
  if (!d || !out) return fail(WP_EINVAL, "wp_lattice_build: NULL argument");
  *out = nullptr;
  if (d->M < 2 || d->M > 1024 || d->N < 2 || d->N > 1024) return fail(WP_EINVAL, "M, N must be in [2, 1024]");
  if (d->two_T != 1) return fail(WP_EINVAL, "only T = 1/2 (two_T = 1) is supported");
  // the per-box quadrature kernels hold up to 256 nodes per cell pair
  if (d->n_x < 1 || d->n_x > 64 || d->n_phi < 1 || d->n_phi > 64 || d->n_x * d->n_phi > 256)
    return fail(WP_EINVAL, "n_x, n_phi must be in [1, 64] with n_x * n_phi <= 256");
  if (d->hbar2_over_m <= 0) return fail(WP_EINVAL, "hbar2_over_m must be positive");
  if (d->two_J < 1 || d->two_J % 2 == 0) return fail(WP_EINVAL, "two_J must be odd and positive");
  std::unique_ptr<wp_lattice> L(new (std::nothrow) wp_lattice());
  if (!L) return fail(WP_ENOMEM, "host allocation");
  if (alloc) {
    if (!alloc->alloc || !alloc->release) return fail(WP_EINVAL, "allocator needs alloc and release");
    L->al.a = *alloc;
    L->al.custom = true;
  }
  L->M = d->M;
  L->N = d->N;
  L->two_J = d->two_J;
  L->n_x = d->n_x;
  L->n_phi = d->n_phi;
  L->h2m = d->hbar2_over_m;
  if (d->grid_kind == 0) {
    if (d->alpha <= 0 || d->p_max <= 0 || d->q_max <= 0) return fail(WP_EINVAL, "alpha, p_max, q_max must be > 0");
    L->pe = tangent_edges(d->M, d->alpha, d->p_max);
    L->qe = tangent_edges(d->N, d->alpha, d->q_max);
  } else if (d->grid_kind == 1) {
    if (!d->p_edges || !d->q_edges) return fail(WP_EINVAL, "explicit grid needs p_edges and q_edges");
    L->pe.assign(d->p_edges, d->p_edges + d->M + 1);
    L->qe.assign(d->q_edges, d->q_edges + d->N + 1);
    for (auto* e : {&L->pe, &L->qe}) {
      if ((*e)[0] != 0.0) return fail(WP_EINVAL, "edges must start at 0");
      for (size_t i = 1; i < e->size(); ++i)
        if (!((*e)[i] > (*e)[i - 1])) return fail(WP_EINVAL, "edges must be strictly increasing");
    }
  } else {
    return fail(WP_EINVAL, "grid_kind must be 0 or 1");
  }
  L->ch = enumerate_channels(d->two_J, d->parity >= 0 ? 1 : -1, d->j_max, d->swave_only != 0);
  L->nch = (int)L->ch.size();
  if (L->nch < 1 || L->nch > 32) return fail(WP_EINVAL, "channel count must be in [1, 32]");
  // coefficient table C[g][g'][m] over distinct moments (k, a, b, l, l'), exponents a = l1 + l1'
  // (powers of q) and b = l2 + l2' (powers of q')
  std::map<std::tuple<int, int, int, int, int>, int> kidx;
  std::vector<std::tuple<int, int, int, double>> ent;
  for (int a = 0; a < L->nch; ++a)
    for (int b = 0; b < L->nch; ++b)
      for (const GTerm& t : g_table(L->ch[a], L->ch[b], d->two_J)) {
        auto key = std::make_tuple(t.k, t.l1 + t.l1p, (L->ch[a].l - t.l1) + (L->ch[b].l - t.l1p), L->ch[a].l, L->ch[b].l);
        auto it = kidx.find(key);
        int m;
        if (it == kidx.end()) {
          m = (int)L->keys.size();
          kidx[key] = m;
          L->keys.push_back({std::get<0>(key), std::get<1>(key), std::get<2>(key), std::get<3>(key), std::get<4>(key)});
        } else {
          m = it->second;
        }
        ent.emplace_back(a, b, m, t.g);
      }
  int nm = std::max<int>(1, (int)L->keys.size());
  if (L->keys.empty()) L->keys.push_back({0, 0, 0, 0, 0});
  L->C.assign((size_t)L->nch * L->nch * nm, 0.0);
  for (auto& e : ent) L->C[((size_t)std::get<0>(e) * L->nch + std::get<1>(e)) * nm + std::get<2>(e)] += std::get<3>(e);
  std::vector<char> nzp((size_t)L->nch * L->nch, 0);
  for (int p = 0; p < L->nch * L->nch; ++p) {
    bool nz = false;
    for (int m = 0; m < nm; ++m) nz |= L->C[(size_t)p * nm + m] != 0.0;
    nzp[p] = nz;
    L->nz_pairs += nz;
  }
  // many channels: blocks stored packed (the channel pairs without a coefficient are left out)
  L->vpb = L->nch * L->nch;
  if (L->nch > 4) {
    L->pk = make_pack(L->nch, nzp);
    const int nc = L->nch;
    for (int u = 0; u < nc; ++u)
      for (int r = L->pk.lo[u]; r < L->pk.hi[u]; ++r) {
        L->pk_src.push_back(L->pk.perm[r] * nc + L->pk.perm[u]);
        L->pk_pos.push_back(u * nc + r);
      }
    L->vpb = L->pk.npk;
  }
  *out = L.release();
  return WP_OK;
}

extern "C" wp_status wp_lattice_channels(const wp_lattice* L, int* n_ch, int* table) {
  if (!L || !n_ch) return fail(WP_EINVAL, "NULL argument");
  *n_ch = L->nch;
  if (table)
    for (int a = 0; a < L->nch; ++a) {
      const Chan& c = L->ch[a];
      int* r = table + 6 * a;
      r[0] = c.l; r[1] = c.s; r[2] = c.j; r[3] = c.lam; r[4] = c.two_I; r[5] = c.t;
    }
  return WP_OK;
}

extern "C" wp_status wp_lattice_info(const wp_lattice* L, int* n_moments, int* n_stored) {
  if (!L) return fail(WP_EINVAL, "NULL lattice");
  if (n_moments) *n_moments = (int)L->keys.size();
  if (n_stored) *n_stored = L->vpb;
  return WP_OK;
}

extern "C" wp_status wp_lattice_edges(const wp_lattice* L, double* p, double* q) {
  if (!L) return fail(WP_EINVAL, "NULL lattice");
  if (p) std::copy(L->pe.begin(), L->pe.end(), p);
  if (q) std::copy(L->qe.begin(), L->qe.end(), q);
  return WP_OK;
}

extern "C" wp_status wp_lattice_weights(wp_lattice* L, int kind) {
  if (!L) return fail(WP_EINVAL, "NULL lattice");
  if (kind != WP_WEIGHTS_UNIT && kind != WP_WEIGHTS_ENERGY) return fail(WP_EINVAL, "unknown weight kind");
  if (L->pseudo || L->have_P)
    return fail(WP_EINVAL, "wp_lattice_weights: set the weights before twobody_pseudostates and perm_matrix_build");
  L->weights = kind;
  return WP_OK;
}

extern "C" void wp_lattice_free(wp_lattice* L) { delete L; }

// ------------------------------------------------------------------ pseudostates

static double ground_energy(const std::vector<double>& h0, const std::vector<double>& v, int M) {
  std::vector<double> A(v);
  for (int i = 0; i < M; ++i) A[(size_t)i * M + i] += h0[i];
  std::vector<double> d;
  sym_eigen(M, A, d, nullptr);
  return d[0];
}

// Unit-strength Yukawa matrices in the WP basis depend only on the p edges, l, mu and the weights,
// not on the three-body block: lattices of several J^pi on one grid share them. A process-wide
// cache (keyed by the exact edge values; emptied when it would exceed 256 MB of matrices) saves
// recomputing them per lattice.
static std::vector<double> yukawa_cached(const std::vector<double>& pe, int l, double mu, bool ew) {
  struct Key {
    std::vector<double> pe;
    int l;
    double mu;
    bool ew;
    bool operator<(const Key& o) const {
      if (l != o.l) return l < o.l;
      if (mu != o.mu) return mu < o.mu;
      if (ew != o.ew) return ew < o.ew;
      return pe < o.pe;
    }
  };
  static std::mutex mu_cache;
  static std::map<Key, std::vector<double>> cache;
  static size_t cached_bytes = 0;
  constexpr size_t kMaxBytes = (size_t)256 << 20;
  Key k{pe, l, mu, ew};
  {
    std::lock_guard<std::mutex> lk(mu_cache);
    auto it = cache.find(k);
    if (it != cache.end()) return it->second;
  }
  std::vector<double> v = ew ? yukawa_wp_energy(pe, l, mu) : yukawa_wp(pe, l, mu);
  const size_t bytes = v.size() * sizeof(double);
  if (bytes > kMaxBytes) return v;
  std::lock_guard<std::mutex> lk(mu_cache);
  if (cached_bytes + bytes > kMaxBytes) {
    cache.clear();
    cached_bytes = 0;
  }
  if (cache.emplace(std::move(k), v).second) cached_bytes += bytes;
  return v;
}

static std::vector<double> wave_potential(const wp_lattice* L, const wp_potential_desc* p, int l, int s, double strength) {
  const int M = L->M;
  std::vector<double> v((size_t)M * M, 0.0);
  const bool ew = L->weights == WP_WEIGHTS_ENERGY;
  if (p->kind == 0) {
    if (l == 0 && s == 1) {
      auto G = ew ? yamaguchi_form_energy(L->pe, p->beta) : yamaguchi_form(L->pe, p->beta);
      for (int i = 0; i < M; ++i)
        for (int k = 0; k < M; ++k) v[(size_t)i * M + k] = -strength * G[i] * G[k];
    }
    return v;
  }
  auto YR = yukawa_cached(L->pe, l, p->mu_R, ew);
  auto YA = yukawa_cached(L->pe, l, p->mu_A, ew);
  double VA = s == 1 ? strength : p->singlet_ratio * strength;
  for (size_t e = 0; e < v.size(); ++e) v[e] = p->V_R * YR[e] - VA * YA[e];
  return v;
}

// root of f on [a, b] (f(a) f(b) < 0) by bisection safeguarded secant (Illinois variant)
template <class F>
static double find_root(F f, double a, double b, double tol) {
  double fa = f(a), fb = f(b);
  if (fa * fb > 0) throw std::runtime_error("strength tuning: target not bracketed");
  int side = 0;
  for (int it = 0; it < 200; ++it) {
    double c = (a * fb - b * fa) / (fb - fa);
    if (!(c > std::min(a, b) && c < std::max(a, b))) c = 0.5 * (a + b);
    double fc = f(c);
    if (fc == 0.0 || std::fabs(b - a) < tol * std::fabs(c)) return c;
    if (fc * fb > 0) {
      b = c;
      fb = fc;
      if (side == -1) fa *= 0.5;
      side = -1;
    } else {
      a = c;
      fa = fc;
      if (side == +1) fb *= 0.5;
      side = +1;
    }
  }
  return 0.5 * (a + b);
}

extern "C" wp_status twobody_pseudostates(wp_lattice* L, const wp_potential_desc* p, double* eps0, double* strength) {
  if (!L || !p) return fail(WP_EINVAL, "NULL argument");
  if (p->kind != 0 && p->kind != 1) return fail(WP_EINVAL, "potential kind must be 0 (Yamaguchi) or 1 (MT)");
  try {
    const int M = L->M;
    const bool ew = L->weights == WP_WEIGHTS_ENERGY;
    auto h0 = ew ? h0_diagonal_energy(L->pe, L->h2m) : h0_diagonal(L->pe, L->h2m);
    double str = p->kind == 0 ? p->lambda : p->V_A;
    if (p->tune) {
      if (p->target_BE <= 0) return fail(WP_EINVAL, "target_BE must be positive");
      if (p->kind == 0) {
        auto G = ew ? yamaguchi_form_energy(L->pe, p->beta) : yamaguchi_form(L->pe, p->beta);
        auto f = [&](double lam) {
          std::vector<double> v((size_t)M * M);
          for (int i = 0; i < M; ++i)
            for (int k = 0; k < M; ++k) v[(size_t)i * M + k] = -lam * G[i] * G[k];
          return ground_energy(h0, v, M) + p->target_BE;
        };
        str = find_root(f, 1.0, 2000.0, 1e-15);
      } else {
        auto YR = yukawa_cached(L->pe, 0, p->mu_R, ew);
        auto YA = yukawa_cached(L->pe, 0, p->mu_A, ew);
        auto f = [&](double VA) {
          std::vector<double> v(YR.size());
          for (size_t e = 0; e < v.size(); ++e) v[e] = p->V_R * YR[e] - VA * YA[e];
          return ground_energy(h0, v, M) + p->target_BE;
        };
        str = find_root(f, 10.0, 5000.0, 1e-15);
      }
    }
    L->waves.clear();
    L->wave_of.assign(L->nch, -1);
    int nbound = 0;
    for (int a = 0; a < L->nch; ++a) {
      int w = -1;
      for (size_t k = 0; k < L->waves.size(); ++k)
        if (L->waves[k].l == L->ch[a].l && L->waves[k].s == L->ch[a].s) w = (int)k;
      if (w < 0) {
        PairWave pw;
        pw.l = L->ch[a].l;
        pw.s = L->ch[a].s;
        pw.v = wave_potential(L, p, pw.l, pw.s, str);
        std::vector<double> A(pw.v);
        for (int i = 0; i < M; ++i) A[(size_t)i * M + i] += h0[i];
        sym_eigen(M, A, pw.eps, &pw.O);
        // sign convention of each pseudostate: its component of largest magnitude is positive
        // (projections onto single pseudostates, the breakup elements, depend on it)
        for (int k = 0; k < M; ++k) {
          double* row = pw.O.data() + (size_t)k * M;
          int im = 0;
          for (int i = 1; i < M; ++i)
            if (std::fabs(row[i]) > std::fabs(row[im])) im = i;
          if (row[im] < 0.0)
            for (int i = 0; i < M; ++i) row[i] = -row[i];
        }
        pw.nb = 0;
        while (pw.nb < M && pw.eps[pw.nb] < 0.0) ++pw.nb;
        nbound += pw.nb;
        // continuum bins: 0, midpoints of neighbouring p*_k, mirrored last edge (unit weights);
        // the same in energy, as momenta sqrt(e / h2m) (energy weights)
        int K = M - pw.nb;
        pw.bins.assign(K + 1, 0.0);
        if (ew) {
          std::vector<double> eb(K + 1, 0.0);
          for (int k = 1; k < K; ++k) eb[k] = 0.5 * (pw.eps[pw.nb + k - 1] + pw.eps[pw.nb + k]);
          eb[K] = 2.0 * pw.eps[pw.nb + K - 1] - eb[K - 1];
          for (int k = 0; k <= K; ++k) pw.bins[k] = std::sqrt(eb[k] / L->h2m);
        } else {
          std::vector<double> ps(K);
          for (int k = 0; k < K; ++k) ps[k] = std::sqrt(pw.eps[pw.nb + k] / L->h2m);
          for (int k = 1; k < K; ++k) pw.bins[k] = 0.5 * (ps[k - 1] + ps[k]);
          pw.bins[K] = 2.0 * ps[K - 1] - pw.bins[K - 1];
        }
        // W = v O^T
        pw.W.assign((size_t)M * M, 0.0);
        for (int i = 0; i < M; ++i)
          for (int k = 0; k < M; ++k) {
            double s = 0.0;
            for (int q = 0; q < M; ++q) s += pw.v[(size_t)i * M + q] * pw.O[(size_t)k * M + q];
            pw.W[(size_t)i * M + k] = s;
          }
        L->waves.push_back(std::move(pw));
        w = (int)L->waves.size() - 1;
      }
      L->wave_of[a] = w;
    }
    int deut = -1;
    for (size_t k = 0; k < L->waves.size(); ++k)
      if (L->waves[k].l == 0 && L->waves[k].s == 1) deut = (int)k;
    if (deut < 0 || L->waves[deut].nb != 1 || nbound != 1)
      return fail(WP_EINVAL, "expected exactly one two-body bound state, in 3S1");
    L->eps0 = L->waves[deut].eps[0];
    L->strength = str;
    L->opens.clear();
    for (int a = 0; a < L->nch; ++a)
      if (L->ch[a].l == 0 && L->ch[a].s == 1 && L->ch[a].j == 1) L->opens.push_back(a);
    if (L->opens.empty() || L->opens.size() > 4) return fail(WP_EINVAL, "1..4 open deuteron channels required");
    L->d_O.reset();
    L->d_W.reset();
    L->d_wave.reset();
    L->pseudo = true;
    if (eps0) *eps0 = L->eps0;
    if (strength) *strength = str;
  } catch (const std::exception& e) {
    return fail(WP_EINTERNAL, std::string("twobody_pseudostates: ") + e.what());
  }
  return WP_OK;
}

static wp_status upload_tables(wp_lattice* L);

// device copies of O and W of every pair wave and the channel -> wave map (first GPU use)
wp_status wpcd::upload_waves(wp_lattice* L) {
  if (L->d_O.p) return WP_OK;
  const size_t MM = (size_t)L->M * L->M;
  std::vector<double> O(MM * L->waves.size()), W(MM * L->waves.size());
  for (size_t k = 0; k < L->waves.size(); ++k) {
    std::copy(L->waves[k].O.begin(), L->waves[k].O.end(), O.begin() + k * MM);
    std::copy(L->waves[k].W.begin(), L->waves[k].W.end(), W.begin() + k * MM);
  }
  if (!L->d_O.make(&L->al, O.size()) || !L->d_W.make(&L->al, W.size()) || !L->d_wave.make(&L->al, L->nch))
    return fail(WP_ENOMEM, "device allocation (pseudostates)");
  HIPCHECK(hipMemcpy(L->d_O.p, O.data(), O.size() * 8, hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(L->d_W.p, W.data(), W.size() * 8, hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(L->d_wave.p, L->wave_of.data(), L->nch * sizeof(int), hipMemcpyHostToDevice));
  // G1 tables
  const int nw = (int)L->waves.size(), M = L->M;
  std::vector<double> bins((size_t)nw * (M + 1), 0.0), epsb(nw, 0.0);
  std::vector<int> nb(nw);
  for (int w = 0; w < nw; ++w) {
    std::copy(L->waves[w].bins.begin(), L->waves[w].bins.end(), bins.begin() + (size_t)w * (M + 1));
    nb[w] = L->waves[w].nb;
    epsb[w] = L->waves[w].nb ? L->waves[w].eps[0] : 0.0;
  }
  // tanh-sinh rule on [-1, 1]: t = k h, x = tanh(pi/2 sinh t), with the node position kept as a
  // fraction of the interval measured from the nearer end
  const double hts = 1.0 / 12.0;   // t in [-3.33, 3.33]: end weights below 1e-18
  const int K = 40;
  std::vector<double> tu, tv, tw;
  for (int k = -K; k <= K; ++k) {
    double t = k * hts, sarg = 0.5 * M_PI * std::sinh(t);
    tu.push_back(1.0 / (1.0 + std::exp(-2.0 * sarg)));
    tv.push_back(1.0 / (1.0 + std::exp(2.0 * sarg)));
    double ch = std::cosh(sarg);
    tw.push_back(hts * 0.5 * M_PI * std::cosh(t) / (ch * ch));
  }
  std::vector<double> glx(36), glw(36);   // 20-point rule, then the 16-point rule
  gauss_legendre(20, glx.data(), glw.data());
  gauss_legendre(16, glx.data() + 20, glw.data() + 20);
  L->nts = (int)tu.size();
  L->ngl = 20;
  if (!L->d_bins.make(&L->al, bins.size()) || !L->d_epsb.make(&L->al, nw) || !L->d_nb.make(&L->al, nw) ||
      !L->d_ts_u.make(&L->al, tu.size()) || !L->d_ts_v.make(&L->al, tv.size()) || !L->d_ts_w.make(&L->al, tw.size()) ||
      !L->d_gl_x.make(&L->al, 36) || !L->d_gl_w.make(&L->al, 36))
    return fail(WP_ENOMEM, "device allocation (G1 tables)");
  HIPCHECK(hipMemcpy(L->d_bins.p, bins.data(), bins.size() * 8, hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(L->d_epsb.p, epsb.data(), nw * 8, hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(L->d_nb.p, nb.data(), nw * sizeof(int), hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(L->d_ts_u.p, tu.data(), tu.size() * 8, hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(L->d_ts_v.p, tv.data(), tv.size() * 8, hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(L->d_ts_w.p, tw.data(), tw.size() * 8, hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(L->d_gl_x.p, glx.data(), 36 * 8, hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(L->d_gl_w.p, glw.data(), 36 * 8, hipMemcpyHostToDevice));
  return WP_OK;
}

bool wpcd::g1_work(wp_lattice* L, int nE, DBuf<int64_t>& w) {
  return grow(w, &L->al, (size_t)g1_work_elems((int)L->waves.size(), L->M, L->N, nE) + 1);
}

G1Args wpcd::g1_args(const wp_lattice* L, const double* dE, int nE, int nrep, int col0, int B, double2* G,
                     int64_t* work) {
  G1Args g{};
  g.M = L->M;
  g.N = L->N;
  g.nch = L->nch;
  g.B = B;
  g.nwave = (int)L->waves.size();
  g.nE = nE;
  g.nrep = nrep;
  g.col0 = col0;
  g.qe = L->d_qe.p;
  g.bins = L->d_bins.p;
  g.nb = L->d_nb.p;
  g.eps_b = L->d_epsb.p;
  g.wave = L->d_wave.p;
  g.E = dE;
  g.ts_u = L->d_ts_u.p;
  g.ts_v = L->d_ts_v.p;
  g.ts_w = L->d_ts_w.p;
  g.nts = L->nts;
  g.gl_x = L->d_gl_x.p;
  g.gl_w = L->d_gl_w.p;
  g.ngl = L->ngl;
  g.gl16_x = L->d_gl_x.p + 20;
  g.gl16_w = L->d_gl_w.p + 20;
  g.h2m = L->h2m;
  g.G = G;
  g.wl_n = reinterpret_cast<int*>(work);
  g.wl = work ? work + 1 : nullptr;
  g.ew = L->weights == WP_WEIGHTS_ENERGY ? 1 : 0;
  return g;
}

extern "C" wp_status wp_lattice_pseudostates(const wp_lattice* L, int channel, int* n_bound, double* eps, double* O,
                                             double* bins) {
  if (!L) return fail(WP_EINVAL, "NULL lattice");
  if (!L->pseudo) return fail(WP_ENOTREADY, "twobody_pseudostates has not run");
  if (channel < 0 || channel >= L->nch) return fail(WP_EINVAL, "channel out of range");
  const PairWave& w = L->waves[L->wave_of[channel]];
  if (n_bound) *n_bound = w.nb;
  if (eps) std::copy(w.eps.begin(), w.eps.end(), eps);
  if (O) std::copy(w.O.begin(), w.O.end(), O);
  if (bins) std::copy(w.bins.begin(), w.bins.end(), bins);
  return WP_OK;
}


extern "C" wp_status wp_lattice_resolvent(const wp_lattice* Lc, double E_lab, int channel, double* G) {
  wp_lattice* L = const_cast<wp_lattice*>(Lc);
  if (!L || !G) return fail(WP_EINVAL, "NULL argument");
  if (!L->pseudo) return fail(WP_ENOTREADY, "twobody_pseudostates has not run");
  if (channel < 0 || channel >= L->nch) return fail(WP_EINVAL, "channel out of range");
  if (!(E_lab > 0)) return fail(WP_EINVAL, "E_lab must be positive");
  if (wp_status st = upload_tables(L)) return st;
  if (wp_status st = upload_waves(L)) return st;
  const int64_t rows = (int64_t)L->M * L->N * L->nch;
  DBuf<double2> dG;
  DBuf<double> dE;
  DBuf<int64_t> g1w;
  if (!dG.make(&L->al, rows) || !dE.make(&L->al, 1) || !g1_work(L, 1, g1w))
    return fail(WP_ENOMEM, "device allocation (resolvent)");
  const double E = L->eps0 + 2.0 * E_lab / 3.0;
  HIPCHECK(hipMemcpy(dE.p, &E, 8, hipMemcpyHostToDevice));
  WP_LAUNCH("g1", nullptr, launch_g1(g1_args(L, dE.p, 1, 1, 0, 1, dG.p, g1w.p), nullptr));
  std::vector<double2> h(rows);
  HIPCHECK(hipMemcpy(h.data(), dG.p, rows * sizeof(double2), hipMemcpyDeviceToHost));
  for (int k = 0; k < L->M; ++k)
    for (int j = 0; j < L->N; ++j) {
      double2 v = h[((size_t)j * L->M + k) * L->nch + channel];
      G[2 * ((size_t)k * L->N + j)] = v.x;
      G[2 * ((size_t)k * L->N + j) + 1] = v.y;
    }
  return WP_OK;
}

// ------------------------------------------------------------------ P0 build

static wp_status upload_tables(wp_lattice* L) {
  if (L->d_pe.p) return WP_OK;
  std::vector<double> gx(L->n_x), gwx(L->n_x), gp(L->n_phi), gwp(L->n_phi);
  gauss_legendre(L->n_x, gx.data(), gwx.data());
  gauss_legendre(L->n_phi, gp.data(), gwp.data());
  std::vector<int> keys;
  for (auto& k : L->keys) keys.insert(keys.end(), {k.k, k.a, k.b, k.l, k.lp});
  if (!L->d_pe.make(&L->al, L->pe.size()) || !L->d_qe.make(&L->al, L->qe.size()) ||
      !L->d_gx.make(&L->al, L->n_x) || !L->d_gwx.make(&L->al, L->n_x) || !L->d_gp.make(&L->al, L->n_phi) ||
      !L->d_gwp.make(&L->al, L->n_phi) || !L->d_C.make(&L->al, L->C.size()) || !L->d_keys.make(&L->al, keys.size()))
    return fail(WP_ENOMEM, "device allocation (lattice tables)");
  HIPCHECK(hipMemcpy(L->d_pe.p, L->pe.data(), L->pe.size() * 8, hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(L->d_qe.p, L->qe.data(), L->qe.size() * 8, hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(L->d_gx.p, gx.data(), gx.size() * 8, hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(L->d_gwx.p, gwx.data(), gwx.size() * 8, hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(L->d_gp.p, gp.data(), gp.size() * 8, hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(L->d_gwp.p, gwp.data(), gwp.size() * 8, hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(L->d_C.p, L->C.data(), L->C.size() * 8, hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(L->d_keys.p, keys.data(), keys.size() * sizeof(int), hipMemcpyHostToDevice));
  if (L->nch > 4) {
    const int nc = L->nch;
    std::vector<int> pkt(4 * nc);
    for (int u = 0; u < nc; ++u) {
      pkt[u] = L->pk.perm[u];
      pkt[nc + u] = L->pk.lo[u];
      pkt[2 * nc + u] = L->pk.hi[u];
      pkt[3 * nc + u] = L->pk.off[u];
    }
    if (!L->d_pkt.make(&L->al, pkt.size()) || !L->d_pkpos.make(&L->al, L->pk_pos.size()) ||
        !L->d_pksrc.make(&L->al, L->pk_src.size()))
      return fail(WP_ENOMEM, "device allocation (packing tables)");
    HIPCHECK(hipMemcpy(L->d_pkt.p, pkt.data(), pkt.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(L->d_pkpos.p, L->pk_pos.data(), L->pk_pos.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(L->d_pksrc.p, L->pk_src.data(), L->pk_src.size() * sizeof(int), hipMemcpyHostToDevice));
  }
  // fused build tables (more than 8 moments)
  const int nm = (int)L->keys.size(), nc = L->nch;
  bool has_k0 = false;
  FusedArgs& fz = L->fz;
  fz.KM = fz.EA = fz.EB = fz.LL = fz.LP = 1;
  for (auto& k : L->keys) {
    has_k0 = has_k0 || k.k == 0;
    fz.KM = std::max(fz.KM, k.k + 1);
    fz.EA = std::max(fz.EA, k.a + 1);
    fz.EB = std::max(fz.EB, k.b + 1);
    fz.LL = std::max(fz.LL, k.l + 1);
    fz.LP = std::max(fz.LP, k.lp + 1);
  }
  fz.vpb = L->vpb;
  fz.ncoef = 0;
  for (int t = 0; t < L->vpb; ++t) {
    const int gg = nc > 4 ? L->pk_src[t] : (t % nc) * nc + t / nc;
    for (int m = 0; m < nm; ++m) fz.ncoef += L->C[(size_t)gg * nm + m] != 0.0;
  }
  fz.ncoef = std::max(fz.ncoef, 1);
  PBuildArgs shape{L->M, L->N, nc, nm, L->n_x, L->n_phi};
  // the stored set of the fused build equals that of the two-pass build when some moment has k = 0
  L->fz_ok = nm > 8 && has_k0 && fused_build_fits(shape, fz);
  if (L->fz_ok) {
    std::vector<int> fkey, cptr{0}, cm;
    std::vector<double> cv;
    for (auto& k : L->keys) fkey.insert(fkey.end(), {k.k, k.a * fz.EB + k.b, k.l * fz.LP + k.lp});
    for (int t = 0; t < L->vpb; ++t) {
      // canonical pair (g, g') of stored value t: packed (pk_src), or full column-major (t = g' nc + g)
      const int gg = nc > 4 ? L->pk_src[t] : (t % nc) * nc + t / nc;
      for (int m = 0; m < nm; ++m) {
        const double c = L->C[(size_t)gg * nm + m];
        if (c != 0.0) {
          cm.push_back(m);
          cv.push_back(c);
        }
      }
      cptr.push_back((int)cm.size());
    }
    if (cm.empty()) {   // all coefficients zero: keep the arrays non-empty
      cm.push_back(0);
      cv.push_back(0.0);
    }
    if ((int)cm.size() != fz.ncoef) return fail(WP_EINVAL, "fused build tables: coefficient count mismatch");
    if (!L->d_fkey.make(&L->al, fkey.size()) || !L->d_fcptr.make(&L->al, cptr.size()) ||
        !L->d_fcm.make(&L->al, cm.size()) || !L->d_fcv.make(&L->al, cv.size()))
      return fail(WP_ENOMEM, "device allocation (fused build tables)");
    HIPCHECK(hipMemcpy(L->d_fkey.p, fkey.data(), fkey.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(L->d_fcptr.p, cptr.data(), cptr.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(L->d_fcm.p, cm.data(), cm.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(L->d_fcv.p, cv.data(), cv.size() * sizeof(double), hipMemcpyHostToDevice));
    fz.fkey = L->d_fkey.p;
    fz.cptr = L->d_fcptr.p;
    fz.cm = L->d_fcm.p;
    fz.cv = L->d_fcv.p;
  }
  return WP_OK;
}

// Sub-allocations of one device buffer (256-byte aligned); with base = nullptr it only sizes.
struct Carve {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t n) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += n * sizeof(T);
    return p;
  }
};

extern "C" wp_status perm_matrix_build(wp_lattice* L, int precision, void* stream, wp_perm_stats* stats) {
  if (!L) return fail(WP_EINVAL, "NULL lattice");
  if (precision != WP_P_FP64 && precision != WP_P_FP32) return fail(WP_EINVAL, "precision must be FP64 or FP32");
  hipStream_t s = (hipStream_t)stream;
  wp_status st = upload_tables(L);
  if (st) return st;
  const int M = L->M, N = L->N, nch = L->nch, nc2 = nch * nch;
  const int64_t R = (int64_t)M * N;
  PBuildArgs a{M, N, nch, (int)L->keys.size(), L->n_x, L->n_phi, L->d_pe.p, L->d_qe.p, L->d_gx.p,
               L->d_gwx.p, L->d_gp.p, L->d_gwp.p, L->d_keys.p, L->d_C.p,
               L->weights == WP_WEIGHTS_ENERGY ? 1 : 0};
  // Scratch is carved from two grow-only buffers of the lattice (the selection arrays, sized by
  // the lattice, and the candidate arrays, sized by the candidate count), so that a rebuild
  // allocates nothing; a buffer above kKeepScratch is released when the build ends.
  // A rebuild whose candidate scratch and resident P0 arrays already exist runs every stage with
  // their capacities as bounds and reads the two totals (candidates, kept blocks) once at the end;
  // a first build, or one that outgrew those capacities, sizes each stage from the previous
  // stage's total instead (two host round trips).
  const size_t kKeepScratch = (size_t)512 << 20;
  const size_t nbox = (size_t)N * N * M;
  // node tables of every q-box in HBM, shared by selection and quadrature, when the moment count
  // allows it (weights padded to AS entries per node)
  const int nn = L->n_x * L->n_phi, nmom = (int)L->keys.size();
  const bool use_tab = nmom <= 4 && nn <= 128 && 9 * M + 1 <= 8192;
  const int AS = ((nmom <= 1 ? 1 : nmom <= 2 ? 2 : 4) + 2) & ~1;
  double *geo = nullptr, *aux = nullptr, *fgeo = nullptr;
  const bool fused = L->keys.size() > 8 && L->fz_ok;
  int *cnt, *lo, *segoff;
  int64_t *rowcnt, *rowptr_c, *tmp;
  auto sel_layout = [&](char* base) {
    Carve c{base};
    if (use_tab) {
      geo = c.take<double>((size_t)N * N * nn * 4);
      aux = c.take<double>((size_t)N * N * nn * AS);
    }
    if (fused) fgeo = c.take<double>((size_t)N * N * fused_geo_doubles(a));
    cnt = c.take<int>(nbox);
    lo = c.take<int>(nbox);
    segoff = c.take<int>(nbox);
    rowcnt = c.take<int64_t>(R);
    rowptr_c = c.take<int64_t>(R + 1);
    tmp = c.take<int64_t>(scan_tmp_size(R));
    return c.off;
  };
  const size_t sel_bytes = sel_layout(nullptr);
  if (L->scratch_sel.n < sel_bytes) {
    L->scratch_sel.reset();
    if (!L->scratch_sel.make(&L->al, sel_bytes)) return fail(WP_ENOMEM, "device allocation (selection)");
  }
  sel_layout(L->scratch_sel.p);
  if (L->d_rowptr.n < (size_t)(R + 1)) {
    L->d_rowptr.reset();
    if (!L->d_rowptr.make(&L->al, R + 1)) return fail(WP_ENOMEM, "device allocation (row pointer)");
  }
  if (!L->h_tot) HIPCHECK(hipHostMalloc((void**)&L->h_tot, 2 * sizeof(int64_t)));
  // the other precision's copy, derived from the previous P0, is dropped
  if (precision == WP_P_FP64) L->d_val32.reset();
  else L->d_val64.reset();
  const bool general = L->keys.size() > 8;
  const int nm = (int)L->keys.size();
  int32_t* col_c = nullptr;
  double *val_c = nullptr, *mom = nullptr, *nrm = nullptr, *Ct = nullptr;
  uint8_t* flag = nullptr;
  int64_t* dest = nullptr;
  auto cand_layout = [&](char* base, size_t nc) {
    Carve c{base};
    flag = c.take<uint8_t>(nc);
    if (fused) {   // per candidate: kept flag and final block index
      dest = c.take<int64_t>(nc);
      return c.off;
    }
    col_c = c.take<int32_t>(nc);
    val_c = c.take<double>(nc * nc2);
    mom = general ? c.take<double>(nc * nm) : nullptr;
    nrm = general ? c.take<double>(nc) : nullptr;
    Ct = general ? c.take<double>((size_t)nm * nc2) : nullptr;
    return c.off;
  };
  auto blk_cap = [&]() -> int64_t {
    const size_t nv = precision == WP_P_FP64 ? L->d_val64.n : L->d_val32.n;
    return (int64_t)std::min(L->d_col.n, nv / (size_t)L->vpb);
  };
  double* val64 = nullptr;
  float* val32 = nullptr;
  for (hipEvent_t& e : L->build_ev)
    if (!e) HIPCHECK(hipEventCreate(&e));
  hipEvent_t e0 = L->build_ev[0], e1 = L->build_ev[1];
  HIPCHECK(hipEventRecord(e0, s));
  if (use_tab) {
    WP_LAUNCH("node_table", s, launch_node_table(a, geo, aux, AS, s));
    WP_LAUNCH("select", s, launch_select_tab(a, geo, aux, AS, cnt, lo, s));
  } else {
    WP_LAUNCH("select", s, launch_select(a, cnt, lo, s));
  }
  auto pbuild = [&]() -> hipError_t {
    return use_tab ? launch_pbuild_tab(a, geo, aux, AS, cnt, lo, segoff, rowptr_c, col_c, val_c, flag, L->cand_cap, s)
                   : launch_pbuild(a, cnt, lo, segoff, rowptr_c, col_c, val_c, flag, L->cand_cap, s);
  };
  // fused build: kept flags, then the final row pointer from them
  auto fused_flags = [&]() -> wp_status {
    WP_LAUNCH("pflag", s, launch_pflag(a, cnt, lo, segoff, rowptr_c, flag, L->cand_cap, fgeo, s));
    WP_LAUNCH("rowcount", s, launch_rowcount(R, rowptr_c, flag, rowcnt, L->cand_cap, s));
    WP_LAUNCH("scan", s, launch_scan(rowcnt, L->d_rowptr.p, R, tmp, s));
    return WP_OK;
  };
  // fused build: final block index per candidate, then the values of every kept block
  auto fused_values = [&](int64_t cap_b) -> wp_status {
    WP_LAUNCH("cand_dest", s, launch_cand_dest(R, rowptr_c, flag, L->d_rowptr.p, dest, L->cand_cap, s));
    WP_LAUNCH("pbuild_fused", s, launch_pbuild_fused(a, L->fz, cnt, lo, segoff, rowptr_c, fgeo, dest, L->cand_cap,
                                                     L->d_col.p, val64, val32, cap_b, s));
    return WP_OK;
  };
  WP_LAUNCH("rowseg", s, launch_rowseg(M, N, cnt, segoff, rowcnt, s));
  WP_LAUNCH("scan", s, launch_scan(rowcnt, rowptr_c, R, tmp, s));
  int64_t ncand = -1, nblk = -1;
  bool done = false;
  const int64_t bcap0 = blk_cap();
  if ((!general || fused) && L->cand_cap > 0 && bcap0 > 0) {
    cand_layout(L->scratch_cand.p, (size_t)L->cand_cap);
    val64 = precision == WP_P_FP64 ? L->d_val64.p : nullptr;
    val32 = precision == WP_P_FP64 ? nullptr : L->d_val32.p;
    if (fused) {
      if (wp_status st = fused_flags()) return st;
      if (wp_status st = fused_values(bcap0)) return st;
    } else {
      WP_LAUNCH("pbuild", s, pbuild());
      WP_LAUNCH("rowcount", s, launch_rowcount(R, rowptr_c, flag, rowcnt, L->cand_cap, s));
      WP_LAUNCH("scan", s, launch_scan(rowcnt, L->d_rowptr.p, R, tmp, s));
      WP_LAUNCH("compact", s, launch_compact(R, nch, rowptr_c, col_c, val_c, flag, L->d_rowptr.p, L->d_col.p, val64,
                                             val32, L->cand_cap, bcap0, L->d_pksrc.p, L->vpb, s));
    }
    WP_LAUNCH("totals", s, launch_totals(rowptr_c + R, L->d_rowptr.p + R, L->h_tot, s));
    HIPCHECK(hipEventRecord(e1, s));
    HIPCHECK(hipEventSynchronize(e1));
    ncand = L->h_tot[0];
    nblk = L->h_tot[1];
    done = ncand <= L->cand_cap && nblk <= bcap0;
  }
  if (!done) {
    if (ncand < 0) {
      HIPCHECK(hipMemcpyAsync(L->h_tot, rowptr_c + R, sizeof(int64_t), hipMemcpyDeviceToHost, s));
      HIPCHECK(hipStreamSynchronize(s));
      ncand = L->h_tot[0];
    }
    const size_t nc = (size_t)std::max<int64_t>(ncand, 1);
    if ((size_t)L->cand_cap < nc) {
      L->scratch_cand.reset();
      L->cand_cap = 0;
      if (!L->scratch_cand.make(&L->al, cand_layout(nullptr, nc))) return fail(WP_ENOMEM, "device allocation (candidates)");
      L->cand_cap = (int64_t)nc;
    }
    cand_layout(L->scratch_cand.p, (size_t)L->cand_cap);
    if (ncand > 0 && fused) {
      if (wp_status st = fused_flags()) return st;
    } else if (ncand > 0 && general) {
      // transposed coefficient table [nmom][nch*nch] for the combine contraction
      std::vector<double> ct((size_t)nm * nc2);
      for (int gg = 0; gg < nc2; ++gg)
        for (int m = 0; m < nm; ++m) ct[(size_t)m * nc2 + gg] = L->C[(size_t)gg * nm + m];
      HIPCHECK(hipMemcpyAsync(Ct, ct.data(), ct.size() * 8, hipMemcpyHostToDevice, s));
      // profiled inside, per kernel (pbuild_mom, combine)
      HIPCHECK(launch_pbuild_general(a, Ct, cnt, lo, segoff, rowptr_c, ncand, col_c, mom, nrm, val_c, flag, s));
    } else if (ncand > 0) {
      WP_LAUNCH("pbuild", s, pbuild());
    }
    if (!(ncand > 0 && fused)) {
      if (ncand > 0) {
        WP_LAUNCH("rowcount", s, launch_rowcount(R, rowptr_c, flag, rowcnt, L->cand_cap, s));
      } else {
        HIPCHECK(hipMemsetAsync(rowcnt, 0, R * sizeof(int64_t), s));
      }
      WP_LAUNCH("scan", s, launch_scan(rowcnt, L->d_rowptr.p, R, tmp, s));
    }
    HIPCHECK(hipMemcpyAsync(L->h_tot + 1, L->d_rowptr.p + R, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    nblk = L->h_tot[1];
    // the resident P0 arrays are reused by a rebuild that fits them (grow-only)
    const size_t nb1 = (size_t)std::max<int64_t>(nblk, 1);
    if (L->d_col.n < nb1) {
      L->d_col.reset();
      if (!L->d_col.make(&L->al, nb1)) return fail(WP_ENOMEM, "device allocation (P0 columns)");
    }
    if (precision == WP_P_FP64) {
      if (L->d_val64.n < nb1 * L->vpb) {
        L->d_val64.reset();
        if (!L->d_val64.make(&L->al, nb1 * L->vpb)) return fail(WP_ENOMEM, "device allocation (P0)");
      }
    } else {
      if (L->d_val32.n < nb1 * L->vpb) {
        L->d_val32.reset();
        if (!L->d_val32.make(&L->al, nb1 * L->vpb)) return fail(WP_ENOMEM, "device allocation (P0)");
      }
    }
    val64 = precision == WP_P_FP64 ? L->d_val64.p : nullptr;
    val32 = precision == WP_P_FP64 ? nullptr : L->d_val32.p;
    if (ncand > 0 && fused) {
      if (wp_status st = fused_values(blk_cap())) return st;
    } else if (ncand > 0) {
      WP_LAUNCH("compact", s, launch_compact(R, nch, rowptr_c, col_c, val_c, flag, L->d_rowptr.p, L->d_col.p,
                                             val64, val32, L->cand_cap, blk_cap(), L->d_pksrc.p, L->vpb, s));
    }
    HIPCHECK(hipEventRecord(e1, s));
    HIPCHECK(hipEventSynchronize(e1));
  }
  float ms = 0.f;
  HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
  if (L->scratch_sel.n > kKeepScratch) L->scratch_sel.reset();
  if (L->scratch_cand.n > kKeepScratch) {
    L->scratch_cand.reset();
    L->cand_cap = 0;
  }
  L->order_ok = false;   // the SpMV row order is derived from this P0 at its first use
  L->blocks = nblk;
  L->prec = precision;
  L->have_P = true;
  L->stats.blocks = nblk;
  L->stats.nnz = nblk * L->nz_pairs;
  L->stats.candidates = ncand;
  L->stats.bytes = (R + 1) * 8 + nblk * 4 + nblk * (int64_t)L->vpb * (precision == WP_P_FP64 ? 8 : 4);
  L->stats.device_ms = ms;
  if (stats) *stats = L->stats;
  return WP_OK;
}

extern "C" wp_status perm_matrix_export(const wp_lattice* L, int64_t* rowptr, int32_t* col, double* val) {
  if (!L) return fail(WP_EINVAL, "NULL lattice");
  if (!L->have_P) return fail(WP_ENOTREADY, "perm_matrix_build has not run");
  const int64_t R = (int64_t)L->M * L->N;
  const int nc2 = L->nch * L->nch;
  if (rowptr) HIPCHECK(hipMemcpy(rowptr, L->d_rowptr.p, (R + 1) * 8, hipMemcpyDeviceToHost));
  if (col) HIPCHECK(hipMemcpy(col, L->d_col.p, L->blocks * 4, hipMemcpyDeviceToHost));
  if (val) {
    // device blocks are column-major (few channels) or packed (many channels); the export is
    // row-major: val[(blk * nch + g) * nch + g']
    const int vpb = L->vpb;
    std::vector<double> d(L->blocks * vpb);
    if (L->prec == WP_P_FP64) {
      HIPCHECK(hipMemcpy(d.data(), L->d_val64.p, d.size() * 8, hipMemcpyDeviceToHost));
    } else {
      std::vector<float> f(d.size());
      HIPCHECK(hipMemcpy(f.data(), L->d_val32.p, f.size() * 4, hipMemcpyDeviceToHost));
      for (size_t e = 0; e < f.size(); ++e) d[e] = f[e];
    }
    const int nch = L->nch;
    if (nch > 4) {
      std::fill(val, val + L->blocks * nc2, 0.0);
      for (int64_t b = 0; b < L->blocks; ++b)
        for (int t = 0; t < vpb; ++t) val[b * nc2 + L->pk_src[t]] = d[b * vpb + t];
    } else {
      for (int64_t b = 0; b < L->blocks; ++b)
        for (int g = 0; g < nch; ++g)
          for (int gp = 0; gp < nch; ++gp) val[b * nc2 + g * nch + gp] = d[b * nc2 + gp * nch + g];
    }
  }
  return WP_OK;
}

// ------------------------------------------------------------------ solve (FP64 path)

// SpMV work order of the resident P0 (made once per build, at the first solve): block rows by
// decreasing length, ties by index, so that the longest rows start first and do not trail at the
// end of a launch (rows hold 0 to ~10x the median number of blocks); the measured alternative,
// lattice order in one contiguous chunk per XCD, was slower.
// Computed on the device on stream s after each build; a call on another stream waits for it.
wp_status wpcd::ensure_order(wp_lattice* L, hipStream_t s) {
  if (!L->have_P || L->nch <= 4) return WP_OK;   // lattice order (spmv_order)
  std::lock_guard<std::mutex> lk(L->order_mu);
  if (!L->order_ev) HIPCHECK(hipEventCreateWithFlags(&L->order_ev, hipEventDisableTiming));
  if (L->order_ok) {
    HIPCHECK(hipStreamWaitEvent(s, L->order_ev, 0));
    return WP_OK;
  }
  const int64_t R = (int64_t)L->M * L->N;
  if (!grow(L->d_order, &L->al, (size_t)R)) return fail(WP_ENOMEM, "device allocation (row order)");
  WP_LAUNCH("row_order", s, launch_row_order(R, L->d_rowptr.p, L->d_order.p, s));
  HIPCHECK(hipEventRecord(L->order_ev, s));
  L->order_ok = true;
  return WP_OK;
}

static wp_status solve_fp64(wp_lattice* L, const std::vector<double>& Elab, const wp_solve_opts& o, hipStream_t s,
                            wp_solution* sol) {
  const int M = L->M, N = L->N, nch = L->nch;
  const int nfin = (int)L->opens.size();
  const int nE = (int)Elab.size();
  const int B = nE * nfin;  // columns: (energy, initial channel)
  const int64_t D = (int64_t)M * N * nch;
  const int64_t R = (int64_t)M * N;
  // per-energy kinematics; G1 is computed on the device
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
  const int max_iter = std::max(4, std::min(1000, o.max_iter));
  const int chunk = 8;
  if (wp_status us = upload_waves(L)) return us;
  if (wp_status so = ensure_order(L, s)) return so;
  const int32_t* order = spmv_order(L);
  // the lattice's workspace when no other call holds it, else one of this call's own
  std::unique_lock<std::mutex> ws_lock(L->ws_mu, std::try_to_lock);
  wp_lattice::Solve64WS own_ws;
  wp_lattice::Solve64WS& ws = ws_lock.owns_lock() ? L->ws64 : own_ws;
  StreamDrain drain{s};   // idle stream before the workspace is released or handed on
  DBuf<double2>&dG = ws.dG, &dy = ws.dy, &ds = ws.ds, &dacap = ws.dacap;
  DBuf<int>&dj0 = ws.dj0, &dg0 = ws.dg0, &dfin = ws.dfin;
  DBuf<double>& dE = ws.dE;
  DBuf<int64_t>& g1w = ws.g1w;
  DevAlloc* al = &L->al;
  if (!g1_work(L, nE, g1w)) return fail(WP_ENOMEM, "device allocation (G1 work list)");
  if (!grow(dG, al, D * B) || !grow(dy, al, D * B) || !grow(ds, al, D * B) ||
      !grow(dacap, al, (size_t)2 * chunk * B * nfin) || !grow(dj0, al, B) || !grow(dg0, al, B) ||
      !grow(dfin, al, nfin) || !grow(dE, al, nE))
    return fail(WP_ENOMEM, "device allocation (solve vectors)");
  HIPCHECK(hipMemcpyAsync(dE.p, Etot.data(), nE * sizeof(double), hipMemcpyHostToDevice, s));
  WP_LAUNCH("g1", s, launch_g1(g1_args(L, dE.p, nE, nfin, 0, B, dG.p, g1w.p), s));
  HIPCHECK(hipMemcpyAsync(dj0.p, j0.data(), B * sizeof(int), hipMemcpyHostToDevice, s));
  HIPCHECK(hipMemcpyAsync(dg0.p, g0.data(), B * sizeof(int), hipMemcpyHostToDevice, s));
  HIPCHECK(hipMemcpyAsync(dfin.p, L->opens.data(), nfin * sizeof(int), hipMemcpyHostToDevice, s));
  const double* val = L->d_val64.p;
  if (!val) return fail(WP_ENOTREADY, "FP64 solve needs P0 built with WP_P_FP64");
  HIPCHECK(launch_init_rhs64(M, N, nch, B, L->d_W.p, L->d_wave.p, dj0.p, dg0.p, ds.p, s));
  HIPCHECK(launch_spmv_f64(R, nch, B, L->d_rowptr.p, L->d_col.p, val, ds.p, dy.p, s, 0, -1, order, pk_view(L, o.spmm_cols)));
  std::vector<ColState> cs(B);
  for (auto& c : cs) {
    c.w.resize(nfin);
    c.S.assign(nfin, cplx(0, 0));
  }
  // Chunks of `chunk` iterations; the captured terms of a chunk go to pinned host memory. For
  // small batches (iterations of a few microseconds) chunk k + 1 is enqueued before chunk k is
  // read, so the device does not wait for the Pade check, at the price of at most one chunk
  // past convergence; large batches read each chunk before the next is enqueued.
  const size_t per_chunk = (size_t)chunk * B * nfin;
  const bool overlap = D * B <= ((int64_t)1 << 20);
  std::unique_lock<std::mutex> pin_lock(L->pin_mu, std::try_to_lock);
  double2* own = nullptr;
  double2* pin = nullptr;
  if (pin_lock.owns_lock()) {
    if (L->pin_cap < 2 * per_chunk) {
      if (L->pin) (void)hipHostFree(L->pin);
      L->pin = nullptr;
      L->pin_cap = 0;
      HIPCHECK(hipHostMalloc((void**)&L->pin, 2 * per_chunk * sizeof(double2), hipHostMallocDefault));
      L->pin_cap = 2 * per_chunk;
    }
    pin = L->pin;
  } else {   // another call on this lattice holds the shared buffer
    HIPCHECK(hipHostMalloc((void**)&own, 2 * per_chunk * sizeof(double2), hipHostMallocDefault));
    pin = own;
  }
  struct PinGuard {   // the stream drains before the staging buffer is released (also on errors)
    double2* own;
    hipStream_t s;
    ~PinGuard() {
      (void)hipStreamSynchronize(s);
      if (own) (void)hipHostFree(own);
    }
  } pin_guard{own, s};
  hipEvent_t ev[2];
  HIPCHECK(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
  HIPCHECK(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() {
      (void)hipEventDestroy(e[0]);
      (void)hipEventDestroy(e[1]);
    }
  } ev_guard{ev};
  int launched = 0;   // iterations enqueued
  int T_of[2] = {0, 0};
  // Terms still needed by the slowest unfinished column after the chunks read so far, predicted
  // from the geometric rate of its relative change over the last chunk (-1: unknown). With
  // overlap, the chunk enqueued while chunk k is read gets only that many terms beyond chunk k
  // (at least 2), so that little work runs past convergence. Only the schedule depends on it:
  // the terms are read in order and the stop rule ends every column at the same term.
  int need = -1;
  std::vector<double> r_prev(B, INFINITY);
  auto next_size = [&](int in_flight) {
    if (need < 0) return chunk;
    return std::max(2, std::min(chunk, need - in_flight + 1));
  };
  // T terms into capture slot `slot` (rows slot * chunk + t of dacap), then their copy to the
  // slot's pinned staging
  auto record_chunk = [&](hipStream_t st, int slot, int T) -> hipError_t {
    for (int t = 0; t < T; ++t) {
      RotArgs ro{M, N, nch, B, L->d_O.p, L->d_wave.p, dG.p, dacap.p, dj0.p, dfin.p, nfin,
                 (int64_t)(slot * chunk + t) * B * nfin};
      ro.tile = o.step_tile;
      hipError_t e;
      {
        ProfScope ps("step64", st);
        e = launch_step64(ro, L->d_W.p, dy.p, ds.p, st);
      }
      if (e != hipSuccess) return e;
      {
        ProfScope ps("spmv64", st);
        e = launch_spmv_f64(R, nch, B, L->d_rowptr.p, L->d_col.p, val, ds.p, dy.p, st, 0, -1, order,
                            pk_view(L, o.spmm_cols));
      }
      if (e != hipSuccess) return e;
    }
    return hipMemcpyAsync(pin + slot * per_chunk, dacap.p + (size_t)slot * per_chunk,
                          (size_t)T * B * nfin * sizeof(double2), hipMemcpyDeviceToHost, st);
  };
  // full chunks replayed from a graph (o.graph), kept by the work space between calls
  const bool use_graph = o.graph == 1 && !profiling_enabled();
  auto enqueue = [&](int slot, int want) -> wp_status {
    const int T = std::min(want, max_iter - launched);
    if (use_graph && T == chunk) {
      const std::vector<int64_t> key{slot, M, N, nch, B, nfin, chunk, o.step_tile, o.spmm_cols,
                                     (int64_t)dG.p, (int64_t)dy.p, (int64_t)ds.p, (int64_t)dacap.p, (int64_t)dj0.p,
                                     (int64_t)dfin.p, (int64_t)pin, (int64_t)L->d_O.p, (int64_t)L->d_W.p,
                                     (int64_t)L->d_wave.p, (int64_t)L->d_rowptr.p, (int64_t)L->d_col.p,
                                     (int64_t)val, (int64_t)order, (int64_t)L->d_pkt.p, (int64_t)L->d_pkpos.p};
      HIPCHECK(graph_run(L, ws.chunk_graph[slot], key, s, [&](hipStream_t st) { return record_chunk(st, slot, T); }));
    } else {
      HIPCHECK(record_chunk(s, slot, T));
    }
    HIPCHECK(hipEventRecord(ev[slot], s));
    T_of[slot] = T;
    launched += T;
    return WP_OK;
  };
  int pending = -1;   // slot of a chunk enqueued and not yet read
  if (overlap) {
    if (wp_status st0 = enqueue(0, chunk)) return st0;
    pending = 0;
  }
  for (int k = 0;; ++k) {
    int cur;
    if (overlap) {
      cur = pending;
      pending = -1;
      if (launched < max_iter) {
        // runs while chunk `cur` is read
        if (wp_status st1 = enqueue(cur ^ 1, next_size(T_of[cur]))) return st1;
        pending = cur ^ 1;
      }
    } else {
      if (launched >= max_iter) break;
      cur = k & 1;
      if (wp_status st1 = enqueue(cur, chunk)) return st1;
    }
    HIPCHECK(hipEventSynchronize(ev[cur]));
    const double2* hcap = pin + cur * per_chunk;
    bool all_done = true;
    for (int c = 0; c < B; ++c) {
      for (int t = 0; t < T_of[cur] && !cs[c].done; ++t) {
        std::vector<cplx> a(nfin);
        for (int f = 0; f < nfin; ++f) {
          double2 v = hcap[((size_t)t * B + c) * nfin + f];
          a[f] = cplx(v.x, v.y);
        }
        column_push(cs[c], a.data(), nfin, o.tol, o.accept);
      }
      all_done &= cs[c].done;
    }
    need = 0;
    for (int c = 0; c < B && need >= 0; ++c) {
      const ColState& q = cs[c];
      if (q.done) continue;
      const double r = q.r_last, r0 = r_prev[c];
      if (r <= o.tol) {
        need = std::max(need, 1);
      } else if (r > 0 && r < r0 && std::isfinite(r0)) {
        const double rate = std::pow(r / r0, 1.0 / std::max(1, T_of[cur]));   // per term, < 1
        need = std::max(need, (int)std::ceil(std::log(o.tol / r) / std::log(rate)) + 1);
      } else {
        need = -1;   // not (yet) contracting: no prediction
      }
    }
    for (int c = 0; c < B; ++c) r_prev[c] = cs[c].r_last;
    if (all_done || (overlap && pending < 0)) break;
  }
  HIPCHECK(hipStreamSynchronize(s));
  bool allok = true;
  for (int e = 0; e < nE; ++e) {
    EnergyResult& r = sol->res[e];
    for (int b = 0; b < nfin; ++b) {
      ColState& c = cs[e * nfin + b];
      if (!c.done) {
        c.ok = c.best_r <= o.accept;
        c.err = c.best_r;
      }
      const std::vector<cplx>& est = c.best.empty() ? c.last : c.best;
      for (int f = 0; f < nfin; ++f) r.U[f * nfin + b] = est[f];
      r.err[b] = c.err;
      r.iters[b] = c.n;
      r.series[b] = std::move(c.terms);
      r.ok &= c.ok;
    }
    allok &= r.ok;
  }
  return allok ? WP_OK : fail(WP_ENOCONV, "Pade summation did not reach the accepted accuracy for some energy");
}


extern "C" wp_status faddeev_solve(wp_lattice* L, int n_E, const double* E_lab, const wp_solve_opts* opts, void* stream,
                                   wp_solution** out) {
  if (!L || !E_lab || !opts || !out || n_E < 1) return fail(WP_EINVAL, "faddeev_solve: bad argument");
  *out = nullptr;
  if (!L->pseudo) return fail(WP_ENOTREADY, "twobody_pseudostates has not run");
  if (!L->have_P) return fail(WP_ENOTREADY, "perm_matrix_build has not run");
  if (opts->tol <= 0 || opts->accept <= 0 || opts->max_iter < 4) return fail(WP_EINVAL, "bad solve options");
  for (int e = 0; e < n_E; ++e)
    if (!(E_lab[e] > 0)) return fail(WP_EINVAL, "E_lab must be positive");
  std::unique_ptr<wp_solution> sol(new wp_solution());
  sol->h2m = L->h2m;
  std::vector<double> E(E_lab, E_lab + n_E);
  wp_status st;
  try {
    if (opts->mode == WP_SOLVE_FP64)
      st = solve_fp64(L, E, *opts, (hipStream_t)stream, sol.get());
    else if (opts->mode == WP_SOLVE_MIXED || opts->mode == WP_SOLVE_MIXED_SPLIT)
      st = solve_mixed(L, E, *opts, (hipStream_t)stream, sol.get());
    else
      return fail(WP_EINVAL, "unknown solve mode");
  } catch (const std::exception& e) {
    return fail(WP_EINTERNAL, std::string("faddeev_solve: ") + e.what());
  }
  if (st == WP_OK || st == WP_ENOCONV) *out = sol.release();
  return st;
}

extern "C" wp_status amplitude(const wp_solution* sol, int e_idx, int* n_open, double* A, double* S, double* delta,
                               double* eta, double* err, int* n_iter) {
  if (!sol || !n_open) return fail(WP_EINVAL, "NULL argument");
  if (e_idx < 0 || e_idx >= (int)sol->res.size()) return fail(WP_EINVAL, "energy index out of range");
  const EnergyResult& r = sol->res[e_idx];
  const int n = r.n_open;
  *n_open = n;
  if (!A && !S && !delta && !eta && !err && !n_iter) return WP_OK;
  // A = (2 / (3 h2m q0)) U / dq_j0 (unit weights) or U / B_j0 (energy weights),  S = 1 - 2 pi i A
  const double fac = r.afac;
  std::vector<cplx> Am(n * n), Sm(n * n);
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      Am[a * n + b] = fac * r.U[a * n + b];
      Sm[a * n + b] = (a == b ? 1.0 : 0.0) - cplx(0.0, 2.0 * M_PI) * Am[a * n + b];
    }
  for (int e = 0; e < n * n; ++e) {
    if (A) { A[2 * e] = Am[e].real(); A[2 * e + 1] = Am[e].imag(); }
    if (S) { S[2 * e] = Sm[e].real(); S[2 * e + 1] = Sm[e].imag(); }
  }
  for (int a = 0; a < n; ++a) {
    if (delta) delta[a] = 0.5 * std::arg(Sm[a * n + a]) * 180.0 / M_PI;
    if (eta) eta[a] = std::abs(Sm[a * n + a]);
    if (err) err[a] = r.err[a];
    if (n_iter) n_iter[a] = r.iters[a];
  }
  return WP_OK;
}

extern "C" wp_status faddeev_series(const wp_solution* sol, int e_idx, int initial, int* n_terms, double* a) {
  if (!sol || !n_terms) return fail(WP_EINVAL, "NULL argument");
  if (e_idx < 0 || e_idx >= (int)sol->res.size()) return fail(WP_EINVAL, "energy index out of range");
  const EnergyResult& r = sol->res[e_idx];
  if (initial < 0 || initial >= r.n_open) return fail(WP_EINVAL, "initial channel out of range");
  static const std::vector<cplx> none;
  const std::vector<cplx>& t = r.series.size() > (size_t)initial ? r.series[initial] : none;
  const int n = r.n_open > 0 ? (int)(t.size() / r.n_open) : 0;
  if (a) {
    if (*n_terms < n) return fail(WP_EINVAL, "faddeev_series: output holds fewer terms than the series");
    for (size_t k = 0; k < t.size(); ++k) {
      a[2 * k] = t[k].real();
      a[2 * k + 1] = t[k].imag();
    }
  }
  *n_terms = n;
  return WP_OK;
}

extern "C" wp_status faddeev_breakup(const wp_solution* sol, int e_idx, int initial, int* n_cells, int* cells,
                                     double* U) {
  if (!sol || !n_cells) return fail(WP_EINVAL, "NULL argument");
  if (e_idx < 0 || e_idx >= (int)sol->res.size()) return fail(WP_EINVAL, "energy index out of range");
  const EnergyResult& r = sol->res[e_idx];
  if (initial < 0 || initial >= r.n_open) return fail(WP_EINVAL, "initial channel out of range");
  const int n = (int)(r.bu_cells.size() / 3);
  if (cells) std::copy(r.bu_cells.begin(), r.bu_cells.end(), cells);
  if (U && n > 0) {
    const std::vector<cplx>& v = r.bu[initial];
    for (int t = 0; t < n; ++t) {
      U[2 * t] = v[t].real();
      U[2 * t + 1] = v[t].imag();
    }
  }
  *n_cells = n;
  return WP_OK;
}

extern "C" void wp_solution_free(wp_solution* s) { delete s; }
