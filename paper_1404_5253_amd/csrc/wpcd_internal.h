// Internal declarations shared by the host numerics (host_math.cpp), the C ABI (capi.cpp) and
// the gfx950 kernels (kernels.hip). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/wpcd.h"

namespace wpcd {
// Launch profiling (wp_profile_*): records a pair of events around the launches of its scope on
// their stream when profiling is enabled (defined in capi.cpp).
struct ProfScope {
  const char* name;
  hipStream_t st;
  hipEvent_t a = nullptr;
  ProfScope(const char* n, hipStream_t s);
  ~ProfScope();
};
}  // namespace wpcd

namespace wpcd {

using cplx = std::complex<double>;

// ------------------------------------------------------------------ host numerics
// Gauss-Legendre nodes/weights on [-1, 1] (Newton iteration on P_n).
void gauss_legendre(int n, double* x, double* w);

std::vector<double> tangent_edges(int n, double alpha, double pmax);
std::vector<double> h0_diagonal(const std::vector<double>& edges, double h2m);

// NN potential in the free WP basis (M x M, row-major).
std::vector<double> yamaguchi_form(const std::vector<double>& edges, double beta);
std::vector<double> yukawa_wp(const std::vector<double>& edges, int l, double mu);
// energy-weight packets (weight sqrt(2 h2m p), norm h2m (p_i^2 - p_{i-1}^2))
std::vector<double> h0_diagonal_energy(const std::vector<double>& edges, double h2m);
std::vector<double> yamaguchi_form_energy(const std::vector<double>& edges, double beta);
std::vector<double> yukawa_wp_energy(const std::vector<double>& edges, int l, double mu);

// Wigner 6j symbol {a b c; d e f} with doubled arguments (Racah formula).
double sixj2(int a, int b, int c, int d, int e, int f);

// Symmetric eigenproblem: Householder tridiagonalisation + implicit QL.
// a (n x n row-major, destroyed) -> eigenvalues ascending in d, eigenvectors as ROWS of z.
void sym_eigen(int n, std::vector<double>& a, std::vector<double>& d, std::vector<double>* z);

// Recoupling
struct Chan { int l, s, j, lam, two_I, t; };
std::vector<Chan> enumerate_channels(int two_J, int parity, int j_max, bool swave_only);
struct MomKey { int k, a, b, l, lp; };
// g table of eq. gal for a channel pair: list of (l1, l1p, k, value)
struct GTerm { int l1, l1p, k; double g; };
std::vector<GTerm> g_table(const Chan& c, const Chan& cp, int two_J);

// Packed storage of the channel blocks of P0 for many channels. The channel pairs whose
// recoupling coefficients all vanish (eq. gal) are zero in every block, so a block stores only
// the others: channels are taken in a permuted order (position r -> canonical channel perm[r])
// chosen so that the stored rows of each block column u form one interval [lo[u], hi[u]) (even
// ends when nc is even, for two-row loads), stored at off[u] within the block's npk values.
constexpr int PK_MAX = 32;
struct PackDesc {
  int nc = 0, npk = 0;
  int perm[PK_MAX], lo[PK_MAX], hi[PK_MAX], off[PK_MAX];
};
// nz[g * nc + gp]: the pair (g, g') has a nonzero coefficient. Returns the packing with the
// fewest stored values among the orders of the groups of channels with equal rows (exhaustive up
// to 8 groups, else the canonical order of groups).
PackDesc make_pack(int nc, const std::vector<char>& nz);

// Wynn epsilon accumulator with the stop rule of faddeev_solve.
struct Wynn {
  std::vector<cplx> diag;
  cplx push(cplx S);
};

// ------------------------------------------------------------------ device helpers
struct DevAlloc {
  wp_allocator a{};
  bool custom = false;
  void* alloc(size_t bytes);
  void release(void* p);
};

template <class T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  DevAlloc* al = nullptr;
  void reset() {
    if (p && al) al->release(p);
    p = nullptr;
    n = 0;
  }
  bool make(DevAlloc* a, size_t count) {
    reset();
    al = a;
    n = count;
    if (count == 0) return true;
    p = static_cast<T*>(a->alloc(count * sizeof(T)));
    return p != nullptr;
  }
  ~DBuf() { reset(); }
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
};

// Grow-only: keeps b when it holds at least n elements, else reallocates it for n.
template <class T>
inline bool grow(DBuf<T>& b, DevAlloc* al, size_t n) {
  return (b.p && b.n >= n) || b.make(al, n);
}

// Waits for the stream when the scope ends, so that memory its work used may be released or
// handed to another call.
struct StreamDrain {
  hipStream_t s;
  ~StreamDrain() { (void)hipStreamSynchronize(s); }
};

// ------------------------------------------------------------------ kernel launchers
// (defined in kernels.hip; every launcher checks its shapes and returns hipError_t)
struct PBuildArgs {
  int M, N, nch, nmom, n_x, n_phi;
  const double* pe;    // device [M+1]
  const double* qe;    // device [N+1]
  const double* gx;    // device Gauss nodes x [n_x]
  const double* gwx;   // weights [n_x]
  const double* gp;    // Gauss nodes phi [n_phi]
  const double* gwp;   // weights [n_phi]
  const int* keys;     // device [nmom][5]
  const double* C;     // device [nch][nch][nmom]
  int ew = 0;          // energy-weight packets: F = U^4 - L^4, node factor sqrt(c s zeta1 zeta2),
                       // widths p_i^2 - p_{i-1}^2 in the norm (unit weights otherwise)
};

// Selection (step 2): per q-box and p-row the hull [lo, lo + cnt) of possibly nonzero p' bins.
hipError_t launch_select(const PBuildArgs& a, int* cnt, int* lo, hipStream_t s);
// Per lattice row, offsets of each box segment and the row total.
hipError_t launch_rowseg(int M, int N, const int* cnt, int* segoff, int64_t* rowcnt, hipStream_t s);
// Exclusive scan of n int64 values, each below 2^31, into out[n+1] (tmp: scan_tmp_size(n) int64).
size_t scan_tmp_size(int64_t n);
hipError_t launch_scan(const int64_t* in, int64_t* out, int64_t n, int64_t* tmp, hipStream_t s);
// Quadrature (step 3) into the candidate block-CSR (values in FP64, per-block nonzero flag).
// Node tables of all q-boxes: geo[box][nd] = (r1, r2, Q1, Q2), aux[box][nd] = (z1, w_0 .. w_{nmom-1},
// zeros up to AS entries); selection and quadrature reading them.
hipError_t launch_node_table(const PBuildArgs& a, double* geo, double* aux, int AS, hipStream_t s);
hipError_t launch_select_tab(const PBuildArgs& a, const double* geo, const double* aux, int AS, int* cnt, int* lo,
                             hipStream_t s);
hipError_t launch_pbuild_tab(const PBuildArgs& a, const double* geo, const double* aux, int AS, const int* cnt,
                             const int* lo, const int* segoff, const int64_t* rowptr_c, int32_t* col_c,
                             double* val_c, uint8_t* flag, int64_t cap, hipStream_t s);
// Candidate blocks at or past cap are not written (the caller checks the total and builds again).
hipError_t launch_pbuild(const PBuildArgs& a, const int* cnt, const int* lo, const int* segoff,
                         const int64_t* rowptr_c, int32_t* col_c, double* val_c, uint8_t* flag,
                         int64_t cap, hipStream_t s);
// Many moments: moments of every candidate pair, then values = norm * (moments x C^T).
// Ct is [nmom][nch*nch]; mom [ncand][nmom] and norm [ncand] are scratch.
hipError_t launch_pbuild_general(const PBuildArgs& a, const double* Ct, const int* cnt, const int* lo, const int* segoff,
                                 const int64_t* rowptr_c, int64_t ncand, int32_t* col_c, double* mom, double* norm,
                                 double* val_c, uint8_t* flag, hipStream_t s);
// Fused many-moment quadrature. The stored set is decided first from the node geometry alone
// (launch_pflag: a candidate is kept when F > 0 at one of its nodes), the final block-CSR offsets
// follow from it (rowcount, scan, launch_cand_dest: the final block index of every kept
// candidate, -1 otherwise), and launch_pbuild_fused then computes each kept block once, per
// q-box: the moment integrals on FP64 MFMA tiles (F of 16 candidates x 4 nodes times the moment
// weights of 4 nodes x 16 moments), contracted with the nonzero recoupling coefficients of every
// stored value, written to col / val of the final arrays.
struct FusedArgs {
  int KM, EA, EB, LL, LP;   // factor tables: P_k (k < KM), cos^(a+1) sin^(b+1) (a < EA, b < EB),
                            // zeta1^-(l'+1) zeta2^-(l+1) (l < LL, l' < LP)
  const int* fkey;          // [nmom][3]: k, a * EB + b, l * LP + l' of every moment
  const int* cptr;          // [vpb + 1]: coefficients of stored value t at [cptr[t], cptr[t + 1])
  const int* cm;            // moment index of each coefficient, ascending within a value
  const double* cv;         // the coefficient C[g][g'][m]
  int ncoef;                // entries of cm / cv
  int vpb;                  // stored values per block
};
// Shape limits of the fused kernel (nodes a multiple of 4 up to 64, up to 256 moments, LDS).
bool fused_build_fits(const PBuildArgs& a, const FusedArgs& f);
// geo [N N][fused_geo_doubles(a)]: node geometry of every box with candidates, for the fused kernel.
hipError_t launch_pflag(const PBuildArgs& a, const int* cnt, const int* lo, const int* segoff,
                        const int64_t* rowptr_c, uint8_t* flag, int64_t cap, double* geo, hipStream_t s);
inline int fused_geo_doubles(const PBuildArgs& a) { return 4 * a.n_x * a.n_phi + 5 * a.n_phi; }
hipError_t launch_cand_dest(int64_t rows, const int64_t* rowptr_c, const uint8_t* flag, const int64_t* rowptr,
                            int64_t* dest, int64_t cap_c, hipStream_t s);
hipError_t launch_pbuild_fused(const PBuildArgs& a, const FusedArgs& f, const int* cnt, const int* lo,
                               const int* segoff, const int64_t* rowptr_c, const double* geo, const int64_t* dest,
                               int64_t cap_c, int32_t* col, double* val64, float* val32, int64_t cap_b,
                               hipStream_t s);
hipError_t launch_rowcount(int64_t rows, const int64_t* rowptr_c, const uint8_t* flag, int64_t* rowcnt,
                           int64_t cap, hipStream_t s);
// Reads candidates below cap_c, writes kept blocks below cap_b.
// Many channels (nch > 4): the kept blocks are written packed, value t of a block taken from the
// candidate block's row-major entry pk_src[t] (vpb values per block); few channels: full
// column-major blocks (vpb = nch^2, pk_src unused).
hipError_t launch_compact(int64_t rows, int nch, const int64_t* rowptr_c, const int32_t* col_c,
                          const double* val_c, const uint8_t* flag, const int64_t* rowptr,
                          int32_t* col, double* val64, float* val32, int64_t cap_c, int64_t cap_b,
                          const int* pk_src, int vpb, hipStream_t s);
// SpMV work order of R block rows: by decreasing length (ties in any order).
hipError_t launch_row_order(int64_t R, const int64_t* rowptr, int32_t* order, hipStream_t s);
// host[0] = *a, host[1] = *b, with host in pinned host memory.
hipError_t launch_totals(const int64_t* a, const int64_t* b, int64_t* host, hipStream_t s);

// Solve kernels. Vector layout: x[((j*M + i)*nch + g)*B + c] complex (double2 / float2).
struct RotArgs {
  int M, N, nch, B;
  const double* A;       // [nwave][M][M] row-major
  const int* wave;       // [nch] pair wave of each channel
  const double2* G;      // scaling [j][k][g][c] or nullptr
  double2* acap;         // captured e^T O y entries or nullptr
  const int* j0;         // [B] on-shell bin per column
  const int* finals;     // [nfin] channels captured
  int nfin;
  int64_t acap_off;      // offset (in double2) of this term's capture row: acap[acap_off + c*nfin + f]
  int tile = 0;          // WP_STEP_* choice of kernel (0: by shape)
};
// fused s = W (G1 * (O y)) with capture; r.A = O, W = v O^T (same wave layout), r.G required
hipError_t launch_step64(const RotArgs& r, const double* W, const double2* y, double2* s_out, hipStream_t s);
// s0 = (v O^T) e0 on the columns [cb0, cb1): the deuteron column W[:, 0] of channel g0[c] at q bin j0[c]
hipError_t launch_init_rhs64(int M, int N, int nch, int B, const double* W, const int* wave,
                             const int* j0, const int* g0, double2* s0, hipStream_t st, int cb0 = 0,
                             int cb1 = -1);
hipError_t launch_fill0(double2* p, int64_t n, hipStream_t st);
// Device view of the packed block storage (many channels, PackDesc): npk values per block;
// pkt[4 nc] = perm, lo, hi, off; pos[npk] = position (u nc + r) of each packed value in the full
// column-major block of positions.
struct PackView {
  int npk = 0;
  const int* pkt = nullptr;
  const int* pos = nullptr;
  int spmm_min = 16;   // column count from which lanes run over the columns
};
// Block-CSR products for any storage/vector precision: lanes over columns when all B >= 16
// columns are requested, else lanes over blocks with a wave reduction. Few channels (<= 4): full
// column-major blocks; many channels: the packed blocks described by pk.
// order: the block rows in the sequence the wavefronts take them (longest first), or nullptr
hipError_t launch_spmv_f64(int64_t rows, int nch, int B, const int64_t* rowptr, const int32_t* col, const double* val,
                           const double2* x, double2* y, hipStream_t s, int cb0, int cb1, const int32_t* order,
                           const PackView& pk);
hipError_t launch_spmv_f32(int64_t rows, int nch, int B, const int64_t* rowptr, const int32_t* col, const float* val,
                           const float2* x, float2* y, hipStream_t s, int cb0, int cb1, const int32_t* order,
                           const PackView& pk);
hipError_t launch_spmv_f32v_f64x(int64_t rows, int nch, int B, const int64_t* rowptr, const int32_t* col,
                                 const float* val, const double2* x, double2* y, hipStream_t s, int cb0, int cb1,
                                 const int32_t* order, const PackView& pk);
// zero the columns [cb0, cb1) of a rows x B array
hipError_t launch_fill0_cols(double2* p, int64_t rows, int B, int cb0, int cb1, hipStream_t st);

// Channel resolvent G1 on the device (FP64). One lane per (wave, k, j, energy) element, one
// wavefront for the elements near the energy shell (work list wl / wl_n, g1_work_elems entries);
// the value is written to every channel of that pair wave and to the nrep columns of the energy:
// G[((j*M + k)*nch + g)*B + col0 + e*nrep + f].
struct G1Args {
  int M, N, nch, B, nwave, nE, nrep, col0;
  const double* qe;     // [N+1]
  const double* bins;   // [nwave][M+1] continuum bin edges (first M - nb + 1 used)
  const int* nb;        // [nwave] bound states (0 or 1)
  const double* eps_b;  // [nwave] bound-state energy
  const int* wave;      // [nch]
  const double* E;      // [nE] three-body energies
  const double* ts_u;   // tanh-sinh node fractions from the left end
  const double* ts_v;   //   ... and from the right end
  const double* ts_w;   //   weights on [-1, 1]
  int nts;
  const double* gl_x;   // Gauss-Legendre nodes / weights on [-1, 1]
  const double* gl_w;
  int ngl;
  const double* gl16_x; // 16-point Gauss-Legendre rule of the lane path
  const double* gl16_w;
  double h2m;
  double2* G;
  int64_t* wl;          // work list (g1_work_elems entries) and its counter
  int* wl_n;
  int ew = 0;           // energy-weight packets: closed forms, one lane per element (no work list)
};
int64_t g1_work_elems(int nwave, int M, int N, int nE);
hipError_t launch_g1(const G1Args& g, hipStream_t s);

// Mixed precision (FP32 P0, BF16 blocks on MFMA with FP32 accumulation, FP32 vectors)
struct RotArgsMixed {
  int M, N, nch, B;
  const uint16_t* A;      // O in bf16: [nwave][Mp][Mp] row-major, zero padded
  const uint16_t* A_lo;   // bf16(O - A) for the split representation, or nullptr
  const uint16_t* W;      // v O^T in bf16, same layout
  const uint16_t* W_lo;   // bf16(v O^T - W) or nullptr
  int Mp;                 // M rounded up to a multiple of 16
  const int* wave;
  const float2* G;        // G1 in FP32 [j][k][g][c]
  const double* yscale;   // per-column factor applied to y on load (nullptr: 1)
};
// s = W (G1 * (O y)) on MFMA (split representation when A_lo / W_lo are given)
hipError_t launch_step_bf16(const RotArgsMixed& r, const float2* y, float2* s_out, hipStream_t s);
hipError_t launch_cvt_d2f(int64_t n, const double2* in, float2* out, hipStream_t s);
hipError_t launch_cvt_d2f_cols(int64_t rows, int B, int c0, int c1, const double2* in, float2* out, hipStream_t s);
hipError_t launch_cvt_scalar(int64_t n, const double* in, float* out, hipStream_t s);
hipError_t launch_residual(int64_t n, const double2* b, const double2* y, const double2* Ky, double2* r,
                           hipStream_t s);
hipError_t launch_lincomb(int64_t rows, int B, int nv, const float2* vecs, int64_t vstride, const double2* coef,
                          double2* out, hipStream_t s);
// Arnoldi on B independent columns of [rows][B] FP32 vectors (rows = cells * nch). The basis is
// kept unnormalised: V_i = scl[i][c] * Vt_i (slots vstride apart); H column j holds h_i = <V_i, w>
// (rows 0..j) and the subdiagonal |w| (row j + 1); FP64 sums throughout.
#define ARN_NV 16   // Arnoldi steps per cycle at most
struct ArnoldiArgs {
  int64_t cells;
  int nch, B, m, j;
  const int64_t* rowptr;
  const int32_t* col;
  const float* val;     // FP32 P0 blocks
  const int32_t* order; // row sequence (longest first) or nullptr
  float2* V;            // basis slots [m + 1][rows][B]
  int64_t vstride;
  double* scl;          // [m + 1][B]
  double2* H;           // [m][m + 1][B]
  double2* part;        // [nblk][ARN_NV][B] partial sums
  int nblk;
  PackView pk;          // packed blocks (many channels)
};
// w = V_j - P0 t into slot j + 1 and H column j (rows 0..j); kv_scratch ([rows][B]) is used when
// the fused kernel does not apply (B < 16 or nch > 4)
hipError_t launch_arnoldi_product(const ArnoldiArgs& a, const float2* t, float2* kv_scratch, hipStream_t s);
// w -= sum_i h_i V_i, then H[j + 1][j] = |w| and scl[j + 1] = 1 / |w|
hipError_t launch_arnoldi_orth(const ArnoldiArgs& a, hipStream_t s);
int arn_blocks(int64_t rows, int B, int nblk);
// U[c][f] = e0^T O y at (g = finals[f], j = j0[c], k = 0), FP64
hipError_t launch_capture64(int M, int nch, int B, int nfin, const double* O, const int* wave, const int* j0,
                            const int* finals, const double2* y, double2* out, hipStream_t s);
// out[t] = (O y) of cell t = (column c, channel g, pseudostate k, q bin j), n cells
hipError_t launch_project_cells(int M, int nch, int B, const double* O, const int* wave, const int4* cells, int n,
                                const double2* y, double2* out, hipStream_t s);
hipError_t launch_norm2_f64(int64_t rows, int B, const double2* x, double2* part, int nblk, double2* out, hipStream_t s);
// out = x / |x| per column (FP64 in, FP32 out); scl0[c] = 1 when given
hipError_t launch_scale_d2f(int64_t rows, int B, const double2* nrm2, const double2* x, float2* out, double* scl0,
                            hipStream_t s);

}  // namespace wpcd
