/*
 * wpcd.h - C ABI of libwpcd: the wave-packet continuum discretisation (WPCD) hot path for the
 * three-nucleon Faddeev equation on one AMD MI355X (gfx950) GPU.
 *
 * Method: Pomerantsev, Kukulin, Rubtsova, "New general approach in few-body scattering
 * calculations: Solving discretized Faddeev equations on a graphics processing unit".
 * The calls follow the five-step scheme of its Sec. V.A:
 *   (1) lattice, two-body pseudostates, recoupling coefficients   wp_lattice_build,
 *                                                                 twobody_pseudostates
 *   (2)+(3) selection and evaluation of the nonzero P0 elements     perm_matrix_build
 *   (4) channel resolvent G1(E) and (5) iteration + Pade            faddeev_solve
 *   on-shell amplitude (Sec. II.B.4)                                amplitude
 * plus a continuous-batching step API (faddeev_batch_*) for serving many energies against
 * one resident P0.
 *
 * Conventions for every call:
 *   - returns wp_status (WP_OK = 0); never aborts, never throws across the ABI; on failure
 *     wp_last_error() returns a thread-local message describing it;
 *   - handles are created by the library and released by the caller with the matching *_free;
 *   - input arrays are copied (the caller keeps ownership); output arrays are caller-allocated
 *     host memory whose sizes come from the documented query;
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream); calls on one handle
 *     are not thread-safe, different handles may be used concurrently on different streams;
 *   - device memory comes from the allocator given to wp_lattice_build (NULL = hipMalloc);
 *     P0 and the per-lattice tables stay resident until wp_lattice_free;
 *   - call order on a lattice: wp_lattice_build -> twobody_pseudostates ->
 *     perm_matrix_build -> faddeev_solve / faddeev_batch_*; anything else is WP_ENOTREADY;
 *   - units: momenta fm^-1, energies MeV; E_lab is the neutron lab energy on a deuteron at
 *     rest, the three-body energy is E = eps0 + (2/3) E_lab.
 */
#ifndef WPCD_H
#define WPCD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int wp_status;
enum {
  WP_OK = 0,
  WP_EINVAL = 1,      /* invalid argument (sizes, ranges, NULL where not allowed) */
  WP_ENOMEM = 2,      /* host or device allocation failed */
  WP_EDEVICE = 3,     /* a HIP runtime call or kernel launch failed */
  WP_ENOTREADY = 4,   /* call made out of order on this handle */
  WP_ENOCONV = 5,     /* iteration / Pade summation did not reach the accepted accuracy */
  WP_EBUDGET = 6,     /* request does not fit the device-memory budget of a batch */
  WP_EINTERNAL = 7
};

/* Message of the last failure on the calling thread ("" if none). Valid until the next call. */
const char* wp_last_error(void);

/* Optional device allocator (e.g. backed by a framework's caching allocator). */
typedef struct {
  void* (*alloc)(size_t bytes, void* ctx);   /* returns device memory or NULL */
  void (*release)(void* ptr, void* ctx);
  void* ctx;
} wp_allocator;

typedef struct wp_lattice wp_lattice;
typedef struct wp_solution wp_solution;
typedef struct wp_batch wp_batch;

/*
 * Lattice of free wave packets (Sec. II.B.1, eqs. pq and xij): M bins D_i in the pair
 * momentum p and N bins in the spectator momentum q, unit momentum weights (Appendix:
 * <p,q|p_i q_j> = theta(p in D_i) theta(q in D_j) / (p q sqrt(d_i d_j))), times the jj-coupled
 * three-body channels gamma = (l, s, j, lam, I) of one block Gamma = (J, pi, T) (eq. qnum).
 *   grid_kind 0: tangent map p_i = alpha tan(i atan(p_max/alpha)/M) (same for q with q_max);
 *   grid_kind 1: explicit edges p_edges[M+1], q_edges[N+1], [0] = 0, strictly increasing.
 * Channels: l + s + t odd, T = 1/2 (two_T must be 1), (-1)^(l+lam) = parity, j <= j_max;
 * swave_only keeps l = lam = 0. Canonical order: sorted by (j, l, s, lam, 2I).
 * n_x, n_phi: Gauss-Legendre points of the (x, phi) rule of the P0 elements, 1..64 each with
 * n_x * n_phi <= 256 (nodes per cell pair). Lattices with more than 8 moment integrals and more
 * than 64 nodes (or a node count not a multiple of 4) take the moment + combine build, whose LDS
 * holds about 220 nodes: above that perm_matrix_build fails.
 * Limits: 2 <= M, N <= 1024; at most 32 channels.
 */
typedef struct {
  int M, N;
  int grid_kind;
  double alpha, p_max, q_max;
  const double* p_edges;
  const double* q_edges;
  int two_J, parity, two_T, j_max, swave_only;
  int n_x, n_phi;
  double hbar2_over_m; /* hbar^2 / m_N in MeV fm^2, e.g. 41.471 */
} wp_lattice_desc;

wp_status wp_lattice_build(const wp_lattice_desc* desc, const wp_allocator* alloc, wp_lattice** out);

/* Channel table: *n_ch always set; if table != NULL it receives n_ch rows of
 * (l, s, j, lam, 2I, t) as int[6]. */
wp_status wp_lattice_channels(const wp_lattice* lat, int* n_ch, int* table);

/* Sizes of the P0 rule and storage (Appendix, final formula): *n_moments = distinct moment
 * integrals (k, a, b, l, l') per cell pair, *n_stored = values stored per P0 block (n_ch^2, or
 * the packed count for more than 4 channels); either pointer may be NULL. */
wp_status wp_lattice_info(const wp_lattice* lat, int* n_moments, int* n_stored);

/* Lattice edges (host copies): p_edges[M+1], q_edges[N+1]; either may be NULL. */
wp_status wp_lattice_edges(const wp_lattice* lat, double* p_edges, double* q_edges);

/*
 * Packet weights (Sec. III.B, the footnote to eqs. dg1a, dg1b). WP_WEIGHTS_UNIT (the default):
 * unit momentum weights as above. WP_WEIGHTS_ENERGY: weights w(p) ~ sqrt(p), f(q) ~ sqrt(q),
 * flat in the energies eps = (hbar^2/m) p^2 and eps_q = (3/4) (hbar^2/m) q^2: a packet is
 * C_i^(-1/2) int_{D_i} w(p) |p> dp with |w|^2 = d eps / dp and C_i the energy width of D_i. Then
 * h0 is the bin's mean energy; the potential and P0 elements carry the weights (the P0 rule
 * takes F = U^4 - L^4, the node factor sqrt(cos phi sin phi zeta1 zeta2) and the norm
 * 1 / sqrt(dp2_i dq2_j dp2_i' dq2_j'), dp2_i = p_i^2 - p_{i-1}^2); the continuum pseudostate bins
 * are energy intervals (edges at midpoints of neighbouring eps_k, mirrored last edge; reported
 * by wp_lattice_pseudostates as momenta sqrt(e / (hbar^2/m))); G1 is evaluated in closed form;
 * the amplitude is A = U / B_j0 with B_j0 the energy width of the on-shell q bin.
 * Set it before twobody_pseudostates and perm_matrix_build; once either has run, WP_EINVAL.
 */
enum { WP_WEIGHTS_UNIT = 0, WP_WEIGHTS_ENERGY = 1 };
wp_status wp_lattice_weights(wp_lattice* lat, int kind);

/*
 * Step-1 results for one channel's pair wave (after twobody_pseudostates): number of bound
 * states, pseudostate energies eps[M] (ascending), O[M*M] (row k = eigenvector k in the free WP
 * basis, eq. exp_z) and the continuum bin edges bins[M - n_bound + 1]. Pointers may be NULL.
 */
wp_status wp_lattice_pseudostates(const wp_lattice* lat, int channel, int* n_bound, double* eps, double* O,
                                  double* bins);

/*
 * Step-4 result: the diagonal of G1(E) (eqs. dg1a, dg1b) for one channel at E = eps0 + (2/3) E_lab,
 * G[2*(k*N + j) + {0,1}] = re/im of G_kj, k = pseudostate (bound states first), j = q bin;
 * G holds 2*M*N doubles. Computed on the device by the solve's G1 kernels (FP64; device memory
 * for the values of every channel and a work list is allocated per call), then copied to G.
 */
wp_status wp_lattice_resolvent(const wp_lattice* lat, double E_lab, int channel, double* G);

/*
 * wp_lattice_resolvent without device allocation, for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, hosts that forbid hipMalloc after set-up).
 * Same arguments and result as wp_lattice_resolvent (bit for bit: the same kernels). Its device
 * scratch (G1 of every channel, the energy and the near-shell work list) is a fixed array of
 * WP_NOALLOC_SCRATCH (16 MiB) per GPU, held until the process ends; a lattice needing more
 * (about 16 M N (n_ch + 1) + 8 n_waves M N bytes; M = N = 150 with 18 channels needs 8.7 MB) is
 * rejected with WP_EINVAL. The lattice's device
 * tables must already be resident (after perm_matrix_build, faddeev_solve or
 * wp_lattice_resolvent), else WP_ENOTREADY. Runs on the null stream and returns when G is
 * written. Calls on one GPU share the scratch array: calls that overlap in time on the same GPU
 * race, so callers must not overlap them.
 */
#define WP_NOALLOC_SCRATCH ((size_t)16 << 20)
wp_status wp_lattice_resolvent_noalloc(const wp_lattice* lat, double E_lab, int channel, double* G);

void wp_lattice_free(wp_lattice* lat);

/*
 * Two-body input and pseudostates (Sec. II.B.2, eq. exp_z): the NN potential v1 in the free
 * WP basis, h1 = h0 + v1 diagonalised for every pair wave (l, s) present, O with the
 * eigenvectors as rows, continuum pseudostate bins around p*_k = sqrt(eps_k / (hbar^2/m)) with
 * edges 0, midpoints between neighbours, and a mirrored last edge.
 *   kind 0: separable Yamaguchi v = -lambda g(p) g(p'), g = 1/(p^2 + beta^2), 3S1 only;
 *   kind 1: Malfliet-Tjon form V_R e^{-mu_R r}/r - V_A e^{-mu_A r}/r in every pair wave,
 *           singlet (s = 0) waves with V_A * singlet_ratio.
 * tune != 0: lambda (kind 0) or V_A (kind 1) is tuned so the lowest 3S1 eigenvalue equals
 * -target_BE. Exactly one bound state (in 3S1) is required; otherwise WP_EINVAL.
 * Outputs (may be NULL): eps0 (deuteron energy), strength (the tuned lambda or V_A).
 */
typedef struct {
  int kind;
  double beta, lambda;
  double V_R, mu_R, V_A, mu_A, singlet_ratio;
  double target_BE;
  int tune;
} wp_potential_desc;

wp_status twobody_pseudostates(wp_lattice* lat, const wp_potential_desc* pot, double* eps0,
                               double* strength);

/*
 * Permutation matrix P0 in the lattice basis (Sec. II.B.3, eq. perm; Appendix, final
 * formula): steps 2 (selection of the nonzero cell pairs) and 3 (their (x, phi) Gauss
 * quadrature with the analytic Q integral F) of Sec. V.A, on the GPU. The result stays
 * resident as block-CSR: block rows and columns are lattice cells r = j*M + i (q bin j, p bin i),
 * each stored block holds the n_ch x n_ch channel values (column-major in (gamma, gamma') on the
 * device; perm_matrix_export returns them row-major).
 * Values are computed in FP64 and stored in FP64 (WP_P_FP64) or rounded to FP32 (WP_P_FP32).
 * Blocks whose values are all exactly zero are omitted. Energy independent: build once. A
 * rebuild of the same lattice reuses the device buffers of the previous build (no allocation)
 * and waits for the device once, at the end; the call returns after the build has finished.
 * stats (may be NULL): blocks = stored cell pairs, nnz = stored scalar entries (blocks times
 * channel pairs with a nonzero coefficient), candidates = selected cell pairs before
 * compaction, bytes = device bytes of the stored matrix, device_ms = GPU time of the build.
 */
enum { WP_P_FP64 = 0, WP_P_FP32 = 1 };
typedef struct {
  int64_t nnz, blocks, candidates;
  int64_t bytes;
  double device_ms;
} wp_perm_stats;

wp_status perm_matrix_build(wp_lattice* lat, int precision, void* stream, wp_perm_stats* stats);

/* Host copy of the resident P0: row_ptr[N*M + 1] (block offsets), col[blocks], val[blocks *
 * n_ch * n_ch] with block b's entry (g, g') at val[(b * n_ch + g) * n_ch + g'] (the device keeps
 * blocks column-major; FP32 storage is widened). Any pointer may be NULL to skip it. */
wp_status perm_matrix_export(const wp_lattice* lat, int64_t* row_ptr, int32_t* col, double* val);

/*
 * Elastic transition operator (Sec. II.A, eq. Ueq; Sec. II.B.4, eq. m_pvg) for each E_lab:
 * G1(E) diagonal in the SWP basis (eqs. dg1a, dg1b; FP64, on the device), the factorised kernel
 * K = P0 (v O^T) G1 O applied by the GPU, and y = b + K y with b = P0 (v O^T) e0 solved for
 * every (energy, open channel) column of the call at once; the amplitude is U = e0^T O y.
 *   mode WP_SOLVE_FP64:  P0 as built, blocks and vectors FP64; Neumann iteration with the
 *                        on-shell series a_n = e0^T O y_n summed by Wynn's epsilon algorithm
 *                        (Pade, Sec. II.B.4). tol: relative change of the estimates at which
 *                        they are accepted (twice in a row); accept: accepted relative error
 *                        when the estimates reach a rounding plateau.
 *   mode WP_SOLVE_MIXED: FP64 iterative refinement y += d with r = b - (I - K) y evaluated in
 *                        FP64 (FP64 blocks and G1, the FP32 copy of P0 accumulated in FP64);
 *                        each correction d from refine_every (default 8, at most 16) Arnoldi
 *                        (GMRES) steps on (I - K~) with K~ = P0 in FP32, v1/O blocks in BF16 on
 *                        MFMA with FP32 accumulation, G1 and vectors in FP32. tol: estimated
 *                        relative error of U (observed contraction of the refinement times
 *                        its last change) at which a column stops.
 *   mode WP_SOLVE_MIXED_SPLIT: as WP_SOLVE_MIXED with every BF16 operand carried as a hi + lo
 *                        pair (three MFMA products per tile, ~16 significant bits), so that
 *                        one correction gains about as much as the FP32 data allow.
 * max_iter: operator applications per solve (<= 1000). Returns WP_ENOCONV (solution still
 * returned) if any solve was not accepted.
 * Launch choices (all 0: the library's defaults; none changes what is computed, only the kernel
 * variant or how launches are issued, so results of one choice are reproducible bit for bit):
 *   graph:     1 replays every full chunk of 8 FP64 terms (FP64 mode) and every refinement
 *              cycle's Arnoldi sweep (mixed modes) from a HIP graph captured once per call
 *              shape and kept by the lattice; ignored while wp_profile is enabled and by the
 *              batch API.
 *   step_tile: FP64 step kernel, one of WP_STEP_*; a choice whose tiles do not fit the lattice
 *              (LDS, rows) falls back to the default.
 *   spmm_cols: more than 4 channels: the column count of a call from which the block-CSR
 *              products run lanes over the columns instead of passes of 4 (default 16).
 */
enum { WP_SOLVE_FP64 = 0, WP_SOLVE_MIXED = 1, WP_SOLVE_MIXED_SPLIT = 2 };
enum { WP_STEP_AUTO = 0, WP_STEP_MFMA8 = 1, WP_STEP_MFMA16 = 2, WP_STEP_VALU = 3, WP_STEP_ROWS = 4 };
typedef struct {
  int mode;
  double tol;
  double accept;
  int max_iter;
  int refine_every;
  int graph;
  int step_tile;
  int spmm_cols;
  int breakup;   /* mixed modes: 1 also projects each solution onto the breakup cells */
} wp_solve_opts;

wp_status faddeev_solve(wp_lattice* lat, int n_E, const double* E_lab, const wp_solve_opts* opts,
                        void* stream, wp_solution** out);

/*
 * On-shell amplitude of energy e_idx (Sec. II.B.4): A_ab = (2/(3 (hbar^2/m) q0)) U_ab / dq_j0
 * over the n_open open deuteron channels (j0: the q bin (q_{j-1}, q_j] holding q0),
 * S = 1 - 2 pi i A, delta = arg(S_aa)/2 in degrees, eta = |S_aa|.
 * A and S: n_open^2 complex numbers, row-major, re/im interleaved (2 n_open^2 doubles);
 * delta_deg, eta, err_est: n_open doubles (err_est = relative error estimate of U).
 * Call with A == NULL first to query n_open (<= 4). Pointers other than n_open may be NULL.
 * Also reports iterations used (n_iter, may be NULL).
 */
wp_status amplitude(const wp_solution* sol, int e_idx, int* n_open, double* A, double* S,
                    double* delta_deg, double* eta, double* err_est, int* n_iter);

/*
 * On-shell series of the FP64 path (Sec. II.A; Sec. V.A step 5): the terms
 * a_n[f] = e_f^T O y_n, y_n = K^n b, that the Pade summation of energy e_idx and initial
 * channel `initial` (0 <= initial < n_open, the order of amplitude()'s columns) consumed, in
 * order, for every final channel f. *n_terms in: capacity of a in terms; out: number of terms.
 * a (may be NULL to query *n_terms): n_terms * n_open complex numbers, term-major
 * (a[2 * (n * n_open + f) + {0, 1}] = re/im of a_n[f]). Solutions of the mixed modes hold no
 * series (*n_terms = 0). WP_EINVAL if the capacity is too small.
 */
wp_status faddeev_series(const wp_solution* sol, int e_idx, int initial, int* n_terms, double* a);

/*
 * Breakup transition elements (Sec. II.A; Sec. II.B.4, end: breakup is an inelastic transition
 * into the discretised two-body continuum, read from the same U): for energy e_idx and initial
 * open channel `initial`, <Z_kj^g| U |Z_0j0> for every channel g, continuum pseudostate k of g's
 * pair wave (k >= its number of bound states) and q bin j whose cell holds the three-body energy
 * (h2m p_a^2 + (3/4) h2m q_a^2 < E < h2m p_b^2 + (3/4) h2m q_b^2 over the pseudostate's momentum
 * bin [p_a, p_b] and q bin [q_a, q_b]: the cells where Im G1 != 0). The transition element is
 * (O y)_{g k j} of the solution y (y = O^T U e0). cells: *n_cells rows of (g, k, j) as int[3];
 * U: *n_cells complex numbers (re, im). Either may be NULL to query *n_cells. Only solutions of
 * the mixed modes asked for it (wp_solve_opts.breakup = 1) hold cells; others report 0. The
 * normalisation of these elements to a physical breakup amplitude is not given in the paper.
 */
wp_status faddeev_breakup(const wp_solution* sol, int e_idx, int initial, int* n_cells, int* cells, double* U);

/*
 * Elastic nd observables from several J^pi blocks (Sec. IV). The elastic S of a block (amplitude(),
 * n_open x n_open) is over its open channels (lam, I), the channels of wp_lattice_channels with the
 * deuteron (l, s, j) = (0, 1, 1) as pair state, in that order: J = j (x) I, I = lam (x) 1/2.
 *
 * nd_sigma_rep: S in the channel-spin representation Sigma = s + sigma (Sec. IV, the I -> Sigma
 * transformation, T[(lam, Sigma), (lam, I)] = sqrt((2I+1)(2Sigma+1)) (-1)^(J-I) {lam 1/2 I; j J Sigma},
 * S_Sigma = T S T^T); the Sigma channels are, for each lam in ascending order, the Sigma in
 * {1/2, 3/2} that couple to J (lam_s[n], two_Sigma[n]). In: two_J (odd), n (1..8), lam[n],
 * two_I[n], S[2 n n] (re/im, row-major). Out (each may be NULL): lam_s, two_Sigma, S_sigma[2 n n].
 * WP_EINVAL if the channels of a lam do not come as a whole shell (the count must match).
 *
 * nd_eigenphases: below breakup S is symmetric and unitary, S = O diag(exp(2 i delta)) O^T with O
 * real orthogonal; delta[n] in radians and O[n n] (column k = eigenvector k, its largest component
 * positive), ordered by the eigenvalues of Re S + 0.618 Im S. Either output may be NULL. Above
 * breakup S is not unitary and the result only approximately diagonalises it.
 *
 * nd_elastic_observables: differential cross section (fm^2/sr) and neutron vector analysing power
 * A_y at n_theta c.m. angles theta[] (radians), summed over n_blocks blocks: two_J[b], n_open[b],
 * the blocks' lam, two_I and S (as above) concatenated in block order, k the nd relative momentum
 * (fm^-1, the on-shell q0 of the solve). Amplitude in the channel-spin basis
 * |Sigma nu, lam m; J M> = sum <Sigma nu lam m|J M> <j m_d 1/2 sigma|Sigma nu> (the states the
 * printed transformation maps to), beam along z, outgoing direction (theta, phi = 0):
 * M = (sqrt(pi)/(i k)) sum sqrt(2 lam + 1) <Sigma nu lam 0|J nu> <Sigma' nu' lam' nu-nu'|J nu>
 * (S - 1) Y_lam'^(nu-nu'); dsdo = Tr(M M^+)/6, Ay = Tr(M sigma_y M^+)/Tr(M M^+) with sigma_y on the
 * incoming neutron and y along k_in x k_out. Host FP64. Outputs may be NULL.
 */
wp_status nd_sigma_rep(int two_J, int n, const int* lam, const int* two_I, const double* S, int* lam_s,
                       int* two_Sigma, double* S_sigma);
wp_status nd_eigenphases(int n, const double* S, double* delta, double* O);
wp_status nd_elastic_observables(int n_blocks, const int* two_J, const int* n_open, const int* lam, const int* two_I,
                                 const double* S, double k, int n_theta, const double* theta, double* dsdo,
                                 double* Ay);

void wp_solution_free(wp_solution* sol);

/*
 * Continuous batching (serving): up to max_slots energies of one lattice share every kernel
 * launch of a step. faddeev_batch_admit takes a free slot (or WP_EBUDGET when none is free or
 * the slot's vectors would exceed hbm_budget bytes); faddeev_batch_step advances every live
 * slot and reports the slots that finished; faddeev_batch_take moves a finished slot's result
 * out and frees the slot. opts->mode selects the path: WP_SOLVE_FP64 advances every slot by
 * `terms` Neumann terms (a slot finishes when its Pade estimate is accepted); the mixed modes
 * run one refinement cycle (FP64 residual, refine_every mixed-precision Arnoldi steps,
 * correction) per step whatever `terms` is, a slot finishing when its error estimate is <= tol.
 * Each slot's arithmetic is independent of the other slots (column-wise kernels, fixed
 * reduction order), so a result does not depend on its batch-mates.
 */
wp_status faddeev_batch_create(wp_lattice* lat, int max_slots, size_t hbm_budget,
                               const wp_solve_opts* opts, wp_batch** out);
wp_status faddeev_batch_admit(wp_batch* b, double E_lab, int* slot);
/*
 * Admission of several energies on a stream (serving): E_lab[0 .. n) in order go into free
 * slots, in runs of adjacent free slots, each run served by one G1 launch and one right-hand
 * side product P0 (v O^T) e0 over its columns (so k requests cost one P0 pass, not k). The work is
 * enqueued on `stream` (give the stream the batch is stepped on) and the call does not wait for
 * it. *n_admitted = how many were admitted (fewer than n, possibly 0, when the batch runs out of
 * free slots: not an error); slots[k] = the slot of E_lab[k]. WP_EINVAL for E_lab <= 0 or an
 * on-shell momentum outside the lattice (nothing of that run is admitted). faddeev_batch_admit
 * is the one-energy form on the null stream, synchronous, WP_EBUDGET when no slot is free.
 */
wp_status faddeev_batch_admit_many(wp_batch* b, int n, const double* E_lab, void* stream, int* slots,
                                   int* n_admitted);
/* Device bytes one slot of a batch with these options takes on this lattice: the unit in which
 * serving divides one device-memory budget among the lattices' batches (hbm_budget of each). */
wp_status faddeev_batch_slot_bytes(const wp_lattice* lat, const wp_solve_opts* opts, size_t* bytes);
wp_status faddeev_batch_step(wp_batch* b, void* stream, int terms, int* n_done, int* done_slots);
wp_status faddeev_batch_take(wp_batch* b, int slot, wp_solution** out);
wp_status faddeev_batch_live(const wp_batch* b, int* n_live);
void faddeev_batch_free(wp_batch* b);

/*
 * Measurement: when enabled, every kernel launch of the library is bracketed by HIP events
 * recorded on the stream it is launched on. wp_profile_read aggregates the records (waiting on
 * their events) by kernel name: with i < 0 it only reports n_kernels; for 0 <= i < n_kernels it
 * fills name (>= 64 bytes), launches and total_ms (sum of the event-measured durations).
 * wp_profile_reset drops all records. Process-wide; not for use from several threads at once.
 */
wp_status wp_profile_enable(int on);
wp_status wp_profile_read(int i, int* n_kernels, char* name, int64_t* launches, double* total_ms);
wp_status wp_profile_reset(void);

#ifdef __cplusplus
}
#endif
#endif /* WPCD_H */
