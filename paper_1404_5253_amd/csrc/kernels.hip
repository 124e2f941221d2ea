// gfx950 kernels of the WPCD hot path.
//
// P0 build (steps 2 and 3 of the paper's Sec. V.A; Appendix, final formula):
//   k_node_table  the (x, phi) quadrature nodes of every q-box (j, j') and their moment weights,
//              once per build, into HBM for the two kernels below.
//   k_select_tab / k_select  per q-box, lanes over p rows i: the p' range with F > 0 at any node
//              is bracketed by the extreme node bounds and located by binary search: one hull
//              [lo, lo + cnt) per (box, i) (k_select builds its node table itself).
//   k_rowseg   per lattice row (j, i): offsets of the box segments and the row total.
//   k_scan_*   exclusive scans (row offsets of the candidate and of the final block-CSR).
//   k_pbuild_tab / k_pbuild  one wavefront per q-box, one candidate cell pair per lane, F and
//              the moments accumulated in registers, channel values sum_m C[g][g'][m] mom_m
//              written straight into the candidate block-CSR.
//   k_rowcount / k_compact  ballot + popcount compaction of the nonzero blocks into the
//              final block-CSR (deterministic, no atomics on the output path).
//   k_row_order  SpMV work order of the final block rows (longest first).
// Solve (step 5):
//   k_g1       G1(E) (eqs. dg1a, dg1b) in FP64, straight into the iteration layout.
//   k_step64 / k_step64m / k_step64r  per channel and column tile: t = O y, capture of
//              e0^T O y, t *= G1, s = (v O^T) t in FP64, on the VALU or on FP64 MFMA tiles (the
//              mixed-precision BF16 MFMA version is in kernels_mixed.hip).
//   k_spmm / k_spmv / k_spmv_gen  block-CSR P0 times complex vectors (lanes over energies,
//              over blocks, or over channel rows for large blocks).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "wpcd_internal.h"

namespace wpcd {

#define WARP 64

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WARP);
  return v;
}
__device__ __forceinline__ int wave_min(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, WARP));
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, WARP));
  return v;
}

// Row-per-wavefront launches: wavefront w takes row order[w] (the rows longest first), or row w
// without an order; -1 past the end.
__device__ __forceinline__ int64_t spmv_row(int64_t rows, const int32_t* __restrict__ order) {
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= rows) return -1;
  return order ? order[w] : w;
}

struct Node {
  double r1, r2, z1, Q1, Q2, w, x, c, s;
};

// Quadrature nodes of q-box (j, jp): x_a on [-1, 1], phi_b on [phi1, phi2] with
// phi1 = atan(q'_{j'-1}/q_j), phi2 = atan(q'_{j'}/q_{j-1}); zeta1, zeta2 and the Q range of the box.
// What depends on phi alone (cos, sin, the Q range) is tabulated once per phi node by
// box_phi_table, and box_node_at completes node nd = a * n_phi + b from that table; the values are
// the same, operation by operation, as evaluating every node from scratch.
#define PHI_STRIDE 5   // c, s, Q1, Q2, phi-weight factor per phi node
static_assert(PHI_STRIDE == 5, "fused_geo_doubles assumes 5 doubles per phi node");
// phi node ib of the box into tab[ib * PHI_STRIDE ...] (q edges qe, Gauss nodes gp on [-1, 1])
__device__ void box_phi_row_p(const double* qe, const double* gp, int j, int jp, int ib, double* tab) {
  const double qa = qe[j], qb = qe[j + 1], qpa = qe[jp], qpb = qe[jp + 1];
  const double phi1 = atan2(qpa, qb), phi2 = atan2(qpb, qa);
  const double hphi = 0.5 * (phi2 - phi1);
  const double phi = 0.5 * (phi1 + phi2) + hphi * gp[ib];
  double c, sn;
  sincos(phi, &sn, &c);
  double* t = tab + ib * PHI_STRIDE;
  t[0] = c;
  t[1] = sn;
  t[2] = fmax(qa / c, qpa / sn);
  t[3] = fmin(qb / c, qpb / sn);
  t[4] = hphi;
}
__device__ __forceinline__ void box_phi_row(const PBuildArgs& a, int j, int jp, int ib, double* tab) {
  box_phi_row_p(a.qe, a.gp, j, jp, ib, tab);
}
// node nd = ia * n_phi + ib from the phi table (x rule gx, gwx; phi weights gwp)
__device__ Node box_node_at_p(const double* gx, const double* gwx, const double* gwp, int n_phi, const double* tab,
                              int nd, bool ew = false) {
  Node n;
  const int ia = nd / n_phi, ib = nd - ia * n_phi;
  const double* t = tab + ib * PHI_STRIDE;
  n.c = t[0];
  n.s = t[1];
  n.Q1 = t[2];
  n.Q2 = t[3];
  n.w = gwx[ia] * t[4] * gwp[ib];
  n.x = gx[ia];
  const double cs = n.c * n.s;
  n.z1 = sqrt(n.c * n.c + 0.25 * n.s * n.s + n.x * cs);
  const double z2 = sqrt(0.25 * n.c * n.c + n.s * n.s + n.x * cs);
  n.r1 = 1.0 / n.z1;
  n.r2 = 1.0 / z2;
  if (ew) n.w *= sqrt(cs * n.z1 * z2);   // energy weights: Q^2 sqrt(c s zeta1 zeta2) per node
  return n;
}
__device__ __forceinline__ Node box_node_at(const PBuildArgs& a, const double* tab, int nd) {
  return box_node_at_p(a.gx, a.gwx, a.gwp, a.n_phi, tab, nd, a.ew != 0);
}
// F of one node and cell pair for U > L: (U^2 - L^2) / 2 (unit weights) or U^4 - L^4 (energy)
__device__ __forceinline__ double f_of(double U, double L, bool ew) {
  return ew ? (U - L) * (U + L) * fma(U, U, L * L) : 0.5 * (U - L) * (U + L);
}
// a bin's width in the norm of a P0 element: p_i - p_{i-1}, or p_i^2 - p_{i-1}^2 (energy weights)
__device__ __forceinline__ double bin_w(double lo, double hi, bool ew) {
  return ew ? (hi - lo) * (hi + lo) : hi - lo;
}
// the phi table of box (j, jp) in LDS, filled by the first n_phi threads of the workgroup
__device__ __forceinline__ void fill_phi_table(const PBuildArgs& a, int j, int jp, double* tab) {
  for (int ib = threadIdx.x; ib < a.n_phi; ib += blockDim.x) box_phi_row(a, j, jp, ib, tab);
}

// ------------------------------------------------------------------ step 2: selection

__global__ void __launch_bounds__(128) k_select(PBuildArgs a, int* __restrict__ cnt, int* __restrict__ lo_out) {
  // One workgroup per q-box (j, j'); lanes over p rows i. For row i and node n, F > 0 needs
  // A_n < B_n with A_n = max(Q1_n, p_{i-1}/zeta2_n), B_n = min(Q2_n, p_i/zeta2_n) and p' in
  // (A_n zeta1_n, B_n zeta1_n). The union over nodes is covered by the p' bins meeting
  // (min_n A_n zeta1_n, max_n B_n zeta1_n), found by two binary searches, widened by one bin.
  extern __shared__ double sh[];
  const int M = a.M;
  const int nn = a.n_x * a.n_phi;
  double* spe = sh;              // M + 1
  double* s_r2 = spe + M + 1;    // nn
  double* s_z1 = s_r2 + nn;
  double* s_Q1 = s_z1 + nn;
  double* s_Q2 = s_Q1 + nn;
  double* s_phi = s_Q2 + nn;     // n_phi * PHI_STRIDE
  const int box = blockIdx.x;
  const int j = box / a.N, jp = box - j * a.N;
  const int t = threadIdx.x;
  for (int i = t; i <= M; i += blockDim.x) spe[i] = a.pe[i];
  fill_phi_table(a, j, jp, s_phi);
  __syncthreads();
  for (int nd = t; nd < nn; nd += blockDim.x) {
    Node n = box_node_at(a, s_phi, nd);
    s_r2[nd] = n.r2;
    s_z1[nd] = n.z1;
    s_Q1[nd] = n.Q1;
    s_Q2[nd] = n.Q2;
  }
  __syncthreads();
  for (int i = t; i < M; i += blockDim.x) {
    const double pa = spe[i], pb = spe[i + 1];
    double xlo = INFINITY, xhi = -INFINITY;
    for (int nd = 0; nd < nn; ++nd) {
      const double r2 = s_r2[nd];
      const double A = fmax(s_Q1[nd], pa * r2);
      const double B = fmin(s_Q2[nd], pb * r2);
      if (A < B) {
        xlo = fmin(xlo, A * s_z1[nd]);
        xhi = fmax(xhi, B * s_z1[nd]);
      }
    }
    int c = 0, l2 = 0;
    if (xlo < xhi) {
      // lo: first bin i' with p'_{i'} (upper edge spe[i'+1]) > xlo
      int lo = 0, hi = M;   // search smallest e in [1, M] with spe[e] > xlo
      while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (spe[mid] > xlo) hi = mid;
        else lo = mid + 1;
      }
      int blo = max(lo - 1, 0);
      // hi: last bin i' with lower edge spe[i'] < xhi
      lo = 0;
      hi = M;
      while (lo < hi) {  // smallest e in [0, M] with spe[e] >= xhi
        int mid = (lo + hi) >> 1;
        if (spe[mid] >= xhi) hi = mid;
        else lo = mid + 1;
      }
      int bhi = min(lo - 1, M - 1);
      if (bhi >= blo) {
        l2 = max(0, blo - 1);
        int h2 = min(M - 1, bhi + 1);
        c = h2 - l2 + 1;
      }
    }
    cnt[(size_t)box * M + i] = c;
    lo_out[(size_t)box * M + i] = l2;
  }
}

// ------------------------------------------------------------------ node tables in HBM
__device__ double moment_weight(const Node& n, const int* key);

// The quadrature nodes of every q-box, computed once per build for both the selection and the
// quadrature: geo[box][nd] = (r1, r2, Q1, Q2) and aux[box][nd] = (z1, halved moment weights
// w_0 / 2 .. w_{nmom-1} / 2, zeros up to AS entries; halving is exact, and the quadrature takes the
// 1/2 of F from the weight). A workgroup takes BB consecutive boxes: first the phi rows of all of
// them (threads over (box, phi node), so that the arc tangents and sines fill the lanes), then
// their nodes (threads over (box, node), consecutive threads writing consecutive nodes).
#define BPW 4
__global__ void __launch_bounds__(256) k_node_table(PBuildArgs a, double* __restrict__ geo, double* __restrict__ aux,
                                                    int AS, int BB) {
  extern __shared__ double sh[];   // [BB][n_phi][PHI_STRIDE]
  const int nn = a.n_x * a.n_phi;
  const int nbox = a.N * a.N;
  const int box0 = blockIdx.x * BB;
  const int nb = min(BB, nbox - box0);
  for (int e = threadIdx.x; e < nb * a.n_phi; e += 256) {
    const int b = e / a.n_phi, ib = e - b * a.n_phi;
    const int box = box0 + b, j = box / a.N, jp = box - j * a.N;
    box_phi_row(a, j, jp, ib, sh + (size_t)b * a.n_phi * PHI_STRIDE);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nb * nn; e += 256) {
    const int b = e / nn, nd = e - b * nn;
    const Node n = box_node_at(a, sh + (size_t)b * a.n_phi * PHI_STRIDE, nd);
    const size_t k = (size_t)(box0 + b) * nn + nd;
    double* g = geo + k * 4;
    g[0] = n.r1;
    g[1] = n.r2;
    g[2] = n.Q1;
    g[3] = n.Q2;
    double* x = aux + k * AS;
    x[0] = n.z1;
    const double half = a.ew ? 1.0 : 0.5;   // energy weights: no 1/2 in F
    for (int m = 0; m < AS - 1; ++m) x[1 + m] = m < a.nmom ? half * moment_weight(n, a.keys + 5 * m) : 0.0;
  }
}

hipError_t launch_node_table(const PBuildArgs& a, double* geo, double* aux, int AS, hipStream_t s) {
  const int nn = a.n_x * a.n_phi;
  if (nn < 1 || nn > 256 || a.n_phi > 256 || AS < 1 + a.nmom) return hipErrorInvalidValue;
  const int nbox = a.N * a.N;
  const size_t row = (size_t)a.n_phi * PHI_STRIDE * sizeof(double);
  const int BB = (int)std::max<size_t>(1, std::min<size_t>(32, (32 * 1024) / row));
  hipLaunchKernelGGL(k_node_table, dim3((nbox + BB - 1) / BB), dim3(256), BB * row, s, a, geo, aux, AS, BB);
  return hipGetLastError();
}

// Selection from the node tables, with the arithmetic of k_select: one wavefront per q-box, BPW
// boxes per workgroup (the p edges shared in LDS). Rows are first restricted exactly: node n can
// be active in row i only if p_{i-1} r2 < Q2 and p_i r2 > Q1 (A >= p_{i-1} r2, B <= p_i r2), and
// with a positive factor r2 the rounded products are nondecreasing in i, so these rows form an
// interval [i0(n), i1(n)) found by binary search with the same products; rows outside the hull of
// the union have no active node and get an empty p' range. Inside it, lane l holds the nodes
// nd = (l mod 8) + 8u in registers and takes the rows (l / 8) + 8k; the bounds of a row are reduced
// over the eight lanes that share it (min and max are exact, so the hull is the same as node by
// node in one lane), then the binary searches run with lanes over rows.
template <int NPL>
__global__ void __launch_bounds__(64 * BPW) k_select_tab(PBuildArgs a, const double* __restrict__ geo,
                                                         const double* __restrict__ aux, int AS,
                                                         int* __restrict__ cnt, int* __restrict__ lo_out) {
  extern __shared__ double sh[];
  const int M = a.M;
  const int nn = a.n_x * a.n_phi;
  const int wv = threadIdx.x >> 6, t = threadIdx.x & 63;
  const int box = blockIdx.x * BPW + wv;
  const bool live = box < a.N * a.N;
  double* spe = sh;                                 // M + 1, shared
  double* s_xlo = spe + M + 1 + wv * 2 * M;         // M per wavefront
  double* s_xhi = s_xlo + M;                        // M per wavefront
  const double* G = geo + (size_t)(live ? box : 0) * nn * 4;
  const double* X = aux + (size_t)(live ? box : 0) * nn * AS;
  for (int i = threadIdx.x; i <= M; i += 64 * BPW) spe[i] = a.pe[i];
  __syncthreads();
  // hull [ilo, ihi) of the rows where any node can be active
  int ilo = M, ihi = 0;
  for (int nd = t; nd < nn; nd += 64) {
    const double r2n = G[nd * 4 + 1], Q1n = G[nd * 4 + 2], Q2n = G[nd * 4 + 3];
    if (!(Q1n < Q2n)) continue;
    int lo = 0, hi = M;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (spe[mid] * r2n >= Q2n) hi = mid;
      else lo = mid + 1;
    }
    const int i1 = lo;
    lo = 0;
    hi = M;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (spe[mid + 1] * r2n > Q1n) hi = mid;
      else lo = mid + 1;
    }
    const int i0 = lo;
    if (i0 < i1) {
      ilo = min(ilo, i0);
      ihi = max(ihi, i1);
    }
  }
  ilo = wave_min(ilo);
  ihi = wave_max(ihi);
  for (int i = t; i < M; i += 64)
    if (i < ilo || i >= ihi) {
      s_xlo[i] = INFINITY;
      s_xhi[i] = -INFINITY;
    }
  const int ng = t & 7, rg = t >> 3;
  double r2[NPL], z1[NPL], Q1[NPL], Q2[NPL];
#pragma unroll
  for (int u = 0; u < NPL; ++u) {
    const int nd = ng + 8 * u;
    const bool ok = nd < nn;
    const int ndc = ok ? nd : 0;
    r2[u] = ok ? G[ndc * 4 + 1] : 0.0;
    z1[u] = ok ? X[(size_t)ndc * AS] : 0.0;
    Q1[u] = ok ? G[ndc * 4 + 2] : 1.0;   // padding nodes: A >= 1 > 0 >= B, never active
    Q2[u] = ok ? G[ndc * 4 + 3] : 0.0;
  }
  for (int i0 = ilo; i0 < ihi; i0 += 8) {
    const int i = i0 + rg;
    const int ic = i < M ? i : M - 1;
    const double pa = spe[ic], pb = spe[ic + 1];
    double xlo = INFINITY, xhi = -INFINITY;
#pragma unroll
    for (int u = 0; u < NPL; ++u) {
      const double A = fmax(Q1[u], pa * r2[u]);
      const double B = fmin(Q2[u], pb * r2[u]);
      if (A < B) {
        xlo = fmin(xlo, A * z1[u]);
        xhi = fmax(xhi, B * z1[u]);
      }
    }
#pragma unroll
    for (int o = 1; o < 8; o <<= 1) {
      xlo = fmin(xlo, __shfl_xor(xlo, o, WARP));
      xhi = fmax(xhi, __shfl_xor(xhi, o, WARP));
    }
    if (ng == 0 && i < ihi) {
      s_xlo[i] = xlo;
      s_xhi[i] = xhi;
    }
  }
  __syncthreads();
  if (!live) return;
  for (int i = t; i < M; i += 64) {
    const double xlo = s_xlo[i], xhi = s_xhi[i];
    int c = 0, l2 = 0;
    if (xlo < xhi) {
      int lo = 0, hi = M;   // smallest e in [1, M] with spe[e] > xlo
      while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (spe[mid] > xlo) hi = mid;
        else lo = mid + 1;
      }
      int blo = max(lo - 1, 0);
      lo = 0;
      hi = M;
      while (lo < hi) {  // smallest e in [0, M] with spe[e] >= xhi
        int mid = (lo + hi) >> 1;
        if (spe[mid] >= xhi) hi = mid;
        else lo = mid + 1;
      }
      int bhi = min(lo - 1, M - 1);
      if (bhi >= blo) {
        l2 = max(0, blo - 1);
        int h2 = min(M - 1, bhi + 1);
        c = h2 - l2 + 1;
      }
    }
    cnt[(size_t)box * M + i] = c;
    lo_out[(size_t)box * M + i] = l2;
  }
}

hipError_t launch_select_tab(const PBuildArgs& a, const double* geo, const double* aux, int AS, int* cnt, int* lo,
                             hipStream_t s) {
  const int nn = a.n_x * a.n_phi;
  if (nn < 1 || nn > 128 || a.M < 1 || a.M > 1024 || a.N < 1 || a.N > 1024) return hipErrorInvalidValue;
  const size_t sh = (size_t)(a.M + 1 + BPW * 2 * a.M) * sizeof(double);
  if (sh > 64 * 1024) return hipErrorInvalidValue;
  const int npl = (nn + 7) / 8;
  const dim3 g((a.N * a.N + BPW - 1) / BPW), b(64 * BPW);
  if (npl <= 4) hipLaunchKernelGGL(k_select_tab<4>, g, b, sh, s, a, geo, aux, AS, cnt, lo);
  else if (npl <= 8) hipLaunchKernelGGL(k_select_tab<8>, g, b, sh, s, a, geo, aux, AS, cnt, lo);
  else hipLaunchKernelGGL(k_select_tab<16>, g, b, sh, s, a, geo, aux, AS, cnt, lo);
  return hipGetLastError();
}

hipError_t launch_select(const PBuildArgs& a, int* cnt, int* lo, hipStream_t s) {
  int nn = a.n_x * a.n_phi;
  if (nn < 1 || nn > 256 || a.M < 1 || a.M > 1024 || a.N < 1 || a.N > 1024) return hipErrorInvalidValue;
  size_t shmem = (a.M + 1) * sizeof(double) + (4 * nn + PHI_STRIDE * a.n_phi) * sizeof(double);
  hipLaunchKernelGGL(k_select, dim3(a.N * a.N), dim3(64), shmem, s, a, cnt, lo);
  return hipGetLastError();
}

// ------------------------------------------------------------------ row segments

// Four threads per row r = j*M + i: thread h sums the candidate counts of the boxes jp in its
// quarter, the four sums are scanned by shuffles, then each thread writes its boxes' offsets.
__global__ void k_rowseg(int M, int N, const int* __restrict__ cnt, int* __restrict__ segoff,
                         int64_t* __restrict__ rowcnt) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r = t >> 2;
  const int h = (int)(t & 3);
  const bool live = r < (int64_t)M * N;
  const int j = live ? (int)(r / M) : 0, i = live ? (int)(r - (int64_t)j * M) : 0;
  const int q = (N + 3) / 4, jp0 = min(N, h * q), jp1 = min(N, jp0 + q);
  int64_t part = 0;
  if (live) {
#pragma unroll 8
    for (int jp = jp0; jp < jp1; ++jp) part += cnt[((size_t)j * N + jp) * M + i];
  }
  // exclusive prefix over the four quarters of the row (lanes 4k .. 4k+3 of the wavefront)
  const int lane = threadIdx.x & 63, base = lane & ~3;
  int64_t before = 0, total = 0;
  for (int k = 0; k < 4; ++k) {
    const int64_t v = __shfl(part, base + k, WARP);
    if (k < h) before += v;
    total += v;
  }
  if (!live) return;
  int64_t run = before;
#pragma unroll 8
  for (int jp = jp0; jp < jp1; ++jp) {
    const size_t idx = ((size_t)j * N + jp) * M + i;
    segoff[idx] = (int)run;
    run += cnt[idx];
  }
  if (h == 0) rowcnt[r] = total;
}

hipError_t launch_rowseg(int M, int N, const int* cnt, int* segoff, int64_t* rowcnt, hipStream_t s) {
  const int64_t T = (int64_t)M * N * 4;   // four threads per row
  hipLaunchKernelGGL(k_rowseg, dim3((unsigned)((T + 255) / 256)), dim3(256), 0, s, M, N, cnt, segoff, rowcnt);
  return hipGetLastError();
}

// ------------------------------------------------------------------ exclusive scan (int64)

#define SCAN_T 256
#define SCAN_E 4
#define SCAN_CHUNK (SCAN_T * SCAN_E)

__device__ int64_t block_exclusive(int64_t v, int64_t* sbuf, int64_t* total) {
  // block-wide exclusive scan of one value per thread (SCAN_T threads)
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  int64_t x = v;
  for (int o = 1; o < 64; o <<= 1) {
    int64_t y = __shfl_up(x, o, WARP);
    if (lane >= o) x += y;
  }
  if (lane == 63) sbuf[wv] = x;
  __syncthreads();
  if (t == 0) {
    int64_t run = 0;
    for (int w = 0; w < SCAN_T / 64; ++w) {
      int64_t tmp = sbuf[w];
      sbuf[w] = run;
      run += tmp;
    }
    sbuf[SCAN_T / 64] = run;
  }
  __syncthreads();
  int64_t res = x - v + sbuf[wv];
  *total = sbuf[SCAN_T / 64];
  __syncthreads();
  return res;
}

__global__ void __launch_bounds__(SCAN_T) k_scan_local(const int64_t* __restrict__ in, int64_t* __restrict__ out,
                                                       int64_t n, int64_t* __restrict__ bsum) {
  __shared__ int64_t sbuf[SCAN_T / 64 + 1];
  int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + threadIdx.x * SCAN_E;
  int64_t v[SCAN_E];
  int64_t loc = 0;
  for (int e = 0; e < SCAN_E; ++e) {
    v[e] = (base + e < n) ? in[base + e] : 0;
    loc += v[e];
  }
  int64_t tot;
  int64_t off = block_exclusive(loc, sbuf, &tot);
  for (int e = 0; e < SCAN_E; ++e) {
    if (base + e < n) out[base + e] = off;
    off += v[e];
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(SCAN_T) k_scan_sums(int64_t* __restrict__ bsum, int nb, int64_t* __restrict__ total_out) {
  __shared__ int64_t sbuf[SCAN_T / 64 + 1];
  int64_t carry = 0;
  for (int base = 0; base < nb; base += SCAN_T) {
    int idx = base + threadIdx.x;
    int64_t v = idx < nb ? bsum[idx] : 0;
    int64_t tot;
    int64_t off = block_exclusive(v, sbuf, &tot);
    if (idx < nb) bsum[idx] = off + carry;
    carry += tot;
  }
  if (threadIdx.x == 0) *total_out = carry;
}

__global__ void k_scan_add(int64_t* __restrict__ out, int64_t n, const int64_t* __restrict__ bsum) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += bsum[i / SCAN_CHUNK];
}

size_t scan_tmp_size(int64_t n) { return (size_t)((n + SCAN_CHUNK - 1) / SCAN_CHUNK + 1); }

// Up to SCAN1_MAX entries: one workgroup of 1024 threads, thread t holding its run of at most 16
// consecutive entries in registers (all loads issued at once); the run totals are scanned across
// the workgroup and each thread writes its run's offsets (one launch instead of three).
#define SCAN1_T 1024
#define SCAN1_MAX (SCAN1_T * 16)
__global__ void __launch_bounds__(SCAN1_T) k_scan_single(const int64_t* __restrict__ in, int64_t* __restrict__ out,
                                                        int64_t n) {
  __shared__ int64_t wsum[SCAN1_T / 64];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int nn = (int)n;
  const int per = (nn + SCAN1_T - 1) / SCAN1_T;
  const int b0 = t * per;
  int64_t v[16];
  int64_t loc = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    v[k] = (k < per && b0 + k < nn) ? in[b0 + k] : 0;
    loc += v[k];
  }
  int64_t x = loc;   // inclusive scan over the wavefront
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = __shfl_up(x, o, WARP);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wv] = x;
  __syncthreads();
  int64_t before = 0, total = 0;
  for (int w = 0; w < SCAN1_T / 64; ++w) {
    const int64_t ws = wsum[w];
    if (w < wv) before += ws;
    total += ws;
  }
  int64_t run = before + x - loc;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    if (k < per && b0 + k < nn) out[b0 + k] = run;
    run += v[k];
  }
  if (t == 0) out[n] = total;
}

// the two totals of a build (candidates, kept blocks), stored straight into pinned host memory
__global__ void k_totals(const int64_t* __restrict__ a, const int64_t* __restrict__ b, int64_t* __restrict__ host) {
  if (threadIdx.x == 0) {
    host[0] = *a;
    host[1] = *b;
  }
}

hipError_t launch_totals(const int64_t* a, const int64_t* b, int64_t* host, hipStream_t s) {
  hipLaunchKernelGGL(k_totals, dim3(1), dim3(64), 0, s, a, b, host);
  return hipGetLastError();
}

// SpMV work order: the block rows by decreasing length (counting sort over 256 length buckets,
// rows of 255 blocks or more sharing the first), in one workgroup. Rows of one bucket land in
// arbitrary order; every row's product is computed on its own, so the order changes no result.
__global__ void __launch_bounds__(1024) k_row_order(int64_t R, const int64_t* __restrict__ rowptr,
                                                    int32_t* __restrict__ order) {
  __shared__ int hist[256];
  const int t = threadIdx.x;
  if (t < 256) hist[t] = 0;
  __syncthreads();
  for (int64_t r = t; r < R; r += 1024) {
    const int64_t len = rowptr[r + 1] - rowptr[r];
    atomicAdd(&hist[255 - (int)min(len, (int64_t)255)], 1);
  }
  __syncthreads();
  if (t < 64) {   // exclusive scan of the 256 bucket counts, four per lane
    int v[4], loc = 0;
    for (int k = 0; k < 4; ++k) {
      v[k] = hist[4 * t + k];
      loc += v[k];
    }
    int x = loc;
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o, WARP);
      if (t >= o) x += y;
    }
    int run = x - loc;
    for (int k = 0; k < 4; ++k) {
      hist[4 * t + k] = run;
      run += v[k];
    }
  }
  __syncthreads();
  for (int64_t r = t; r < R; r += 1024) {
    const int64_t len = rowptr[r + 1] - rowptr[r];
    const int pos = atomicAdd(&hist[255 - (int)min(len, (int64_t)255)], 1);
    order[pos] = (int32_t)r;
  }
}

hipError_t launch_row_order(int64_t R, const int64_t* rowptr, int32_t* order, hipStream_t s) {
  if (R < 1 || R > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_row_order, dim3(1), dim3(1024), 0, s, R, rowptr, order);
  return hipGetLastError();
}

hipError_t launch_scan(const int64_t* in, int64_t* out, int64_t n, int64_t* tmp, hipStream_t s) {
  if (n <= 0) return hipErrorInvalidValue;
  if (n <= SCAN1_MAX) {
    hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(SCAN1_T), 0, s, in, out, n);
    return hipGetLastError();
  }
  int nb = (int)((n + SCAN_CHUNK - 1) / SCAN_CHUNK);
  hipLaunchKernelGGL(k_scan_local, dim3(nb), dim3(SCAN_T), 0, s, in, out, n, tmp);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SCAN_T), 0, s, tmp, nb, out + n);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, n, tmp);
  return hipGetLastError();
}

// ------------------------------------------------------------------ step 3: quadrature

#define PB_MAXNODES 256
#define PB_MAXMOM 8

// Moment weight of key (k, a, b, l, l') at a node: w P_k(x) c^(a+1) s^(b+1) / (z1^(l'+1) z2^(l+1)).
__device__ double moment_weight(const Node& n, const int* key) {
  int k = key[0], ea = key[1], eb = key[2], l = key[3], lp = key[4];
  double p0 = 1.0, p1 = n.x, pk = (k == 0) ? 1.0 : n.x;
  for (int m = 2; m <= k; ++m) {
    double p2 = ((2.0 * m - 1.0) * n.x * p1 - (m - 1.0) * p0) / m;
    p0 = p1;
    p1 = p2;
    pk = p2;
  }
  double v = n.w * pk;
  for (int e = 0; e <= ea; ++e) v *= n.c;
  for (int e = 0; e <= eb; ++e) v *= n.s;
  for (int e = 0; e <= lp; ++e) v *= n.r1;
  for (int e = 0; e <= l; ++e) v *= n.r2;
  return v;
}

template <int NMOM>
__global__ void __launch_bounds__(64) k_pbuild(PBuildArgs a, const int* __restrict__ cnt, const int* __restrict__ lo,
                                               const int* __restrict__ segoff, const int64_t* __restrict__ rowptr_c,
                                               int32_t* __restrict__ col_c, double* __restrict__ val_c,
                                               uint8_t* __restrict__ flag, int64_t cap) {
  extern __shared__ double sh[];
  const int M = a.M, N = a.N;
  const int nn = a.n_x * a.n_phi;
  const int box = blockIdx.x;
  const int j = box / N, jp = box - j * N;
  const int t = threadIdx.x;
  // LDS: r1, r2, Q1, Q2 [nn], weights [NMOM][nn], phi table [n_phi][PHI_STRIDE], pe [M+1],
  // pref [M+1] (int), lo [M] (int)
  double* s_r1 = sh;
  double* s_r2 = s_r1 + nn;
  double* s_Q1 = s_r2 + nn;
  double* s_Q2 = s_Q1 + nn;
  double* s_w = s_Q2 + nn;
  double* s_phi = s_w + NMOM * nn;
  double* s_pe = s_phi + PHI_STRIDE * a.n_phi;
  int* s_pref = reinterpret_cast<int*>(s_pe + M + 1);
  int* s_lo = s_pref + M + 1;

  // exclusive prefix of the candidate counts over p rows i (wave scan in chunks of 64)
  int run = 0;
  for (int base = 0; base < M; base += 64) {
    int i = base + t;
    int c = (i < M) ? cnt[(size_t)box * M + i] : 0;
    int x = c;
    for (int o = 1; o < 64; o <<= 1) {
      int y = __shfl_up(x, o, WARP);
      if (t >= o) x += y;
    }
    if (i < M) {
      s_pref[i] = run + x - c;
      s_lo[i] = lo[(size_t)box * M + i];
    }
    run += __shfl(x, 63, WARP);
  }
  const int total = run;
  if (total == 0) return;
  if (t == 0) s_pref[M] = total;
  for (int i = t; i <= M; i += 64) s_pe[i] = a.pe[i];
  fill_phi_table(a, j, jp, s_phi);
  __syncthreads();
  for (int nd = t; nd < nn; nd += 64) {
    Node n = box_node_at(a, s_phi, nd);
    s_r1[nd] = n.r1;
    s_r2[nd] = n.r2;
    s_Q1[nd] = n.Q1;
    s_Q2[nd] = n.Q2;
    for (int m = 0; m < a.nmom; ++m) s_w[m * nn + nd] = moment_weight(n, a.keys + 5 * m);
  }
  __syncthreads();

  const double dq = bin_w(a.qe[j], a.qe[j + 1], a.ew), dqp = bin_w(a.qe[jp], a.qe[jp + 1], a.ew);
  const int nc = a.nch, nc2 = nc * nc;
  for (int e = t; e < total; e += 64) {
    // row i: last i with pref[i] <= e
    int lo_i = 0, hi_i = M - 1;
    while (lo_i < hi_i) {
      int mid = (lo_i + hi_i + 1) >> 1;
      if (s_pref[mid] <= e) lo_i = mid;
      else hi_i = mid - 1;
    }
    const int i = lo_i;
    const int ip = s_lo[i] + (e - s_pref[i]);
    const double pa = s_pe[i], pb = s_pe[i + 1], ppa = s_pe[ip], ppb = s_pe[ip + 1];
    double mom[NMOM];
#pragma unroll
    for (int m = 0; m < NMOM; ++m) mom[m] = 0.0;
    for (int nd = 0; nd < nn; ++nd) {
      const double r1 = s_r1[nd], r2 = s_r2[nd];
      const double U = fmin(s_Q2[nd], fmin(ppb * r1, pb * r2));
      const double L = fmax(s_Q1[nd], fmax(ppa * r1, pa * r2));
      const double F = (U > L) ? f_of(U, L, a.ew != 0) : 0.0;
#pragma unroll
      for (int m = 0; m < NMOM; ++m)
        if (m < a.nmom) mom[m] = fma(s_w[m * nn + nd], F, mom[m]);
    }
    const double norm = 1.0 / sqrt(bin_w(pa, pb, a.ew) * dq * bin_w(ppa, ppb, a.ew) * dqp);
    const int64_t blk = rowptr_c[(size_t)j * M + i] + segoff[(size_t)box * M + i] + (ip - s_lo[i]);
    if (blk >= cap) continue;   // the candidate arrays are too small: the caller sees the total and builds again
    col_c[blk] = jp * M + ip;
    bool nz = false;
    for (int gg = 0; gg < nc2; ++gg) {
      double v = 0.0;
#pragma unroll
      for (int m = 0; m < NMOM; ++m)
        if (m < a.nmom) v = fma(a.C[(size_t)gg * a.nmom + m], mom[m], v);
      v *= norm;
      val_c[blk * nc2 + gg] = v;
      nz |= (v != 0.0);
    }
    flag[blk] = nz ? 1 : 0;
  }
}

// Quadrature from the node tables: one wavefront per q-box, one candidate per lane, the box's
// node table staged in LDS and read by broadcast. Moment weights past nmom are zero in the table.
// Per node, w F = (w / 2) (U - L) (U + L) for U > L, else 0, is taken as
// fma(w / 2, max(U - L, 0) (U + L), mom): U + L > 0, and scaling by 1/2 commutes with rounding,
// so this is the same number as fma(w, F, mom) with one compare and two selects fewer.
// One wavefront per box, BPW boxes per workgroup (coefficients and p edges shared in LDS).
template <int NMOM, bool EW>
__global__ void __launch_bounds__(64 * BPW) k_pbuild_tab(PBuildArgs a, const double* __restrict__ geo,
                                                         const double* __restrict__ aux, int AS,
                                                         const int* __restrict__ cnt, const int* __restrict__ lo,
                                                         const int* __restrict__ segoff,
                                                         const int64_t* __restrict__ rowptr_c,
                                                         int32_t* __restrict__ col_c, double* __restrict__ val_c,
                                                         uint8_t* __restrict__ flag, int64_t cap) {
  extern __shared__ double sh[];
  const int M = a.M, N = a.N;
  const int nn = a.n_x * a.n_phi;
  const int wv = threadIdx.x >> 6, t = threadIdx.x & 63;
  const int box = blockIdx.x * BPW + wv;
  const bool live = box < N * N;
  const int j = live ? box / N : 0, jp = live ? box - j * N : 0;
  const int nc = a.nch, nc2 = nc * nc;
  // LDS: C [nc2][nmom] and pe [M+1] shared; per wavefront the node table [nn][4 + AS], base [M]
  // (int64), pref [M+1], lo [M] (int)
  double* s_C = sh;
  double* s_pe = s_C + nc2 * a.nmom;
  const int RS = 4 + AS;
  const size_t per_wave = (size_t)nn * RS * sizeof(double) + (size_t)M * sizeof(int64_t) + (2 * M + 1) * sizeof(int);
  char* wbase = reinterpret_cast<char*>(s_pe + M + 1) + wv * ((per_wave + 7) & ~(size_t)7);
  double* s_nd = reinterpret_cast<double*>(wbase);
  int64_t* s_base = reinterpret_cast<int64_t*>(s_nd + (size_t)nn * RS);
  int* s_pref = reinterpret_cast<int*>(s_base + M);
  int* s_lo = s_pref + M + 1;
  // per row: the candidate count, the first candidate column, and the output position of the
  // row's first candidate (all loaded at once from in-range addresses; box 0 stands in for a box
  // past the end, whose counts are taken as zero)
  const size_t bx = live ? (size_t)box : 0;
  int run = 0;
  for (int base = 0; base < M; base += 64) {
    const int i = base + t;
    const int ic = i < M ? i : M - 1;
    const int c_ld = cnt[bx * M + ic];
    const int lo_ld = lo[bx * M + ic];
    const int64_t rp = rowptr_c[(size_t)j * M + ic];
    const int sg = segoff[bx * M + ic];
    const int c = (live && i < M) ? c_ld : 0;
    int x = c;
    for (int o = 1; o < 64; o <<= 1) {
      int y = __shfl_up(x, o, WARP);
      if (t >= o) x += y;
    }
    if (i < M) {
      const int pref = run + x - c;
      s_pref[i] = pref;
      s_lo[i] = live ? lo_ld : 0;
      // candidate e of row i goes to block base[i] + e of the candidate block-CSR
      s_base[i] = c ? rp + sg - pref : 0;
    }
    run += __shfl(x, 63, WARP);
  }
  const int total = run;   // 0 for a box past the end
  if (t == 0) s_pref[M] = total;
  for (int i = threadIdx.x; i <= M; i += 64 * BPW) s_pe[i] = a.pe[i];
  for (int e = threadIdx.x; e < nc2 * a.nmom; e += 64 * BPW) s_C[e] = a.C[e];
  if (total > 0) {   // this box's node table, row nd = (r1, r2, Q1, Q2, z1, w ...)
    const double* Gg = geo + (size_t)box * nn * 4;
    const double* Xg = aux + (size_t)box * nn * AS;
    for (int e = t; e < nn * 4; e += 64) s_nd[(e >> 2) * RS + (e & 3)] = Gg[e];
    for (int e = t; e < nn * AS; e += 64) s_nd[(e / AS) * RS + 4 + e % AS] = Xg[e];
  }
  __syncthreads();
  if (total == 0) return;
  const double dq = bin_w(a.qe[j], a.qe[j + 1], a.ew), dqp = bin_w(a.qe[jp], a.qe[jp + 1], a.ew);
  for (int e0 = 0; e0 < total; e0 += 64) {
    const int e = min(e0 + t, total - 1);
    int lo_i = 0, hi_i = M - 1;   // row: last i with pref[i] <= e
    while (lo_i < hi_i) {
      int mid = (lo_i + hi_i + 1) >> 1;
      if (s_pref[mid] <= e) lo_i = mid;
      else hi_i = mid - 1;
    }
    const int i = lo_i;
    const int ip = s_lo[i] + (e - s_pref[i]);
    const double pa = s_pe[i], pb = s_pe[i + 1], ppa = s_pe[ip], ppb = s_pe[ip + 1];
    double mom[NMOM];
#pragma unroll
    for (int m = 0; m < NMOM; ++m) mom[m] = 0.0;
#pragma unroll 4
    for (int nd = 0; nd < nn; ++nd) {
      const double* q = s_nd + nd * RS;   // the same address in every lane: LDS broadcast
      const double r1 = q[0], r2 = q[1], Q1 = q[2], Q2 = q[3];
      const double U = fmin(Q2, fmin(ppb * r1, pb * r2));
      const double L = fmax(Q1, fmax(ppa * r1, pa * r2));
      double F2 = fmax(U - L, 0.0) * (U + L);   // 2 F (unit weights), with the unhalved weight:
      if (EW) F2 *= fma(U, U, L * L);           // U^4 - L^4 (energy weights)
#pragma unroll
      for (int m = 0; m < NMOM; ++m) mom[m] = fma(q[5 + m], F2, mom[m]);
    }
    const int64_t blk = s_base[i] + e;
    // past the end, or the candidate arrays are too small (the caller sees the total and builds again)
    if (e0 + t >= total || blk >= cap) continue;
    const double norm = 1.0 / sqrt(bin_w(pa, pb, EW) * dq * bin_w(ppa, ppb, EW) * dqp);
    bool nz = false;
    for (int gg = 0; gg < nc2; ++gg) {
      double v = 0.0;
#pragma unroll
      for (int m = 0; m < NMOM; ++m)
        if (m < a.nmom) v = fma(s_C[gg * a.nmom + m], mom[m], v);
      v *= norm;
      val_c[blk * nc2 + gg] = v;
      nz |= (v != 0.0);
    }
    col_c[blk] = jp * M + ip;
    flag[blk] = nz ? 1 : 0;
  }
}

hipError_t launch_pbuild_tab(const PBuildArgs& a, const double* geo, const double* aux, int AS, const int* cnt,
                             const int* lo, const int* segoff, const int64_t* rowptr_c, int32_t* col_c,
                             double* val_c, uint8_t* flag, int64_t cap, hipStream_t s) {
  if (a.nmom < 1 || a.nmom > 4 || AS < 1 + a.nmom || a.nch < 1) return hipErrorInvalidValue;
  const int nn = a.n_x * a.n_phi;
  const size_t per_wave = ((size_t)nn * (4 + AS) * sizeof(double) + (size_t)a.M * sizeof(int64_t) +
                           (2 * a.M + 1) * sizeof(int) + 7) & ~(size_t)7;
  const size_t sh = (size_t)(a.nch * a.nch * a.nmom + a.M + 1) * sizeof(double) + BPW * per_wave;
  if (sh > 64 * 1024) return hipErrorInvalidValue;
  dim3 g((a.N * a.N + BPW - 1) / BPW), b(64 * BPW);
#define WP_TAB(NM, EW) \
  hipLaunchKernelGGL((k_pbuild_tab<NM, EW>), g, b, sh, s, a, geo, aux, AS, cnt, lo, segoff, rowptr_c, col_c, val_c, \
                     flag, cap)
  const bool ew = a.ew != 0;
  if (a.nmom <= 1) {
    if (ew) WP_TAB(1, true); else WP_TAB(1, false);
  } else if (a.nmom <= 2) {
    if (ew) WP_TAB(2, true); else WP_TAB(2, false);
  } else {
    if (ew) WP_TAB(4, true); else WP_TAB(4, false);
  }
#undef WP_TAB
  return hipGetLastError();
}

hipError_t launch_pbuild(const PBuildArgs& a, const int* cnt, const int* lo, const int* segoff,
                         const int64_t* rowptr_c, int32_t* col_c, double* val_c, uint8_t* flag, int64_t cap,
                         hipStream_t s) {
  int nn = a.n_x * a.n_phi;
  if (nn < 1 || nn > PB_MAXNODES || a.nmom < 1 || a.nmom > PB_MAXMOM || a.nch < 1) return hipErrorInvalidValue;
  size_t shmem = (size_t)nn * (4 + (a.nmom <= 1 ? 1 : (a.nmom <= 2 ? 2 : (a.nmom <= 4 ? 4 : 8)))) * sizeof(double) +
                 (size_t)PHI_STRIDE * a.n_phi * sizeof(double) + (a.M + 1) * sizeof(double) +
                 (2 * a.M + 1) * sizeof(int);
  dim3 g(a.N * a.N), b(64);
  if (a.nmom <= 1)
    hipLaunchKernelGGL(k_pbuild<1>, g, b, shmem, s, a, cnt, lo, segoff, rowptr_c, col_c, val_c, flag, cap);
  else if (a.nmom <= 2)
    hipLaunchKernelGGL(k_pbuild<2>, g, b, shmem, s, a, cnt, lo, segoff, rowptr_c, col_c, val_c, flag, cap);
  else if (a.nmom <= 4)
    hipLaunchKernelGGL(k_pbuild<4>, g, b, shmem, s, a, cnt, lo, segoff, rowptr_c, col_c, val_c, flag, cap);
  else
    hipLaunchKernelGGL(k_pbuild<8>, g, b, shmem, s, a, cnt, lo, segoff, rowptr_c, col_c, val_c, flag, cap);
  return hipGetLastError();
}

// ------------------------------------------------------------------ compaction

__global__ void __launch_bounds__(256) k_rowcount(int64_t rows, const int64_t* __restrict__ rowptr_c,
                                                  const uint8_t* __restrict__ flag, int64_t* __restrict__ rowcnt,
                                                  int64_t cap) {
  int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  int lane = threadIdx.x & 63;
  if (row >= rows) return;
  // candidates at or past cap were not written (too small arrays; the caller builds again)
  int64_t b0 = min(rowptr_c[row], cap), b1 = min(rowptr_c[row + 1], cap);
  int64_t c = 0;
  for (int64_t e = b0 + lane; e < b1; e += 64) c += flag[e];
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, WARP);
  if (lane == 0) rowcnt[row] = c;
}

hipError_t launch_rowcount(int64_t rows, const int64_t* rowptr_c, const uint8_t* flag, int64_t* rowcnt, int64_t cap,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_rowcount, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, s, rows, rowptr_c, flag, rowcnt, cap);
  return hipGetLastError();
}

// The final blocks are stored column-major: P[g][g'] of block d at val[d * nc2 + g' * nch + g], so
// that lanes over the output channel g read contiguous memory for every g'.
__global__ void __launch_bounds__(256) k_compact(int64_t rows, int nch, const int64_t* __restrict__ rowptr_c,
                                                 const int32_t* __restrict__ col_c, const double* __restrict__ val_c,
                                                 const uint8_t* __restrict__ flag, const int64_t* __restrict__ rowptr,
                                                 int32_t* __restrict__ col, double* __restrict__ val64,
                                                 float* __restrict__ val32, int64_t cap_c, int64_t cap_b,
                                                 const int* __restrict__ pk_src, int vpb) {
  int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  int lane = threadIdx.x & 63;
  if (row >= rows) return;
  const int nc2 = nch * nch;
  // reads stay below cap_c (candidate arrays) and writes below cap_b (P0 arrays); a build that
  // outgrew either is run again by the caller
  int64_t b0 = min(rowptr_c[row], cap_c), b1 = min(rowptr_c[row + 1], cap_c);
  int64_t out = rowptr[row];
  for (int64_t base = b0; base < b1; base += 64) {
    int64_t e = base + lane;
    const bool kept = (e < b1) && flag[e];
    unsigned long long mask = __ballot(kept);
    int before = __popcll(mask & ((1ull << lane) - 1ull));
    const bool f = kept && out + before < cap_b;
    if (f) col[out + before] = col_c[e];
    if (nc2 <= 16) {   // a lane copies its own block
      if (f) {
        const int64_t d = out + before;
        for (int g = 0; g < nch; ++g)
          for (int gp = 0; gp < nch; ++gp) {
            const double v = val_c[e * nc2 + g * nch + gp];
            if (val64) val64[d * nc2 + gp * nch + g] = v;
            if (val32) val32[d * nc2 + gp * nch + g] = (float)v;
          }
      }
    } else {           // the wave copies each kept block, lanes over its packed values
      unsigned long long m = mask;
      int k = 0;
      while (m) {
        const int src = __ffsll((long long)m) - 1;
        m &= m - 1ull;
        const int64_t es = base + src, d = out + k;
        ++k;
        if (d >= cap_b) break;
        for (int t = lane; t < vpb; t += 64) {
          const double v = val_c[es * nc2 + pk_src[t]];
          if (val64) val64[d * vpb + t] = v;
          if (val32) val32[d * vpb + t] = (float)v;
        }
      }
    }
    out += __popcll(mask);
  }
}

hipError_t launch_compact(int64_t rows, int nch, const int64_t* rowptr_c, const int32_t* col_c, const double* val_c,
                          const uint8_t* flag, const int64_t* rowptr, int32_t* col, double* val64, float* val32,
                          int64_t cap_c, int64_t cap_b, const int* pk_src, int vpb, hipStream_t s) {
  if (nch > 4 && (!pk_src || vpb < 1 || vpb > nch * nch)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_compact, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, s, rows, nch, rowptr_c, col_c, val_c,
                     flag, rowptr, col, val64, val32, cap_c, cap_b, pk_src, vpb);
  return hipGetLastError();
}

// ------------------------------------------------------------------ solve: right-hand side

__global__ void k_fill0(double2* __restrict__ p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = make_double2(0.0, 0.0);
}

__global__ void k_set_rhs(int M, int nch, int B, int cb0, const double* __restrict__ W, const int* __restrict__ wave,
                          const int* __restrict__ j0, const int* __restrict__ g0, double2* __restrict__ s0) {
  int c = cb0 + blockIdx.x;
  int g = g0[c];
  const double* Wg = W + (size_t)wave[g] * M * M;
  for (int i = threadIdx.x; i < M; i += blockDim.x)
    s0[(((size_t)j0[c] * M + i) * nch + g) * B + c] = make_double2(Wg[(size_t)i * M + 0], 0.0);
}

__global__ void k_fill0_cols(double2* __restrict__ p, int64_t rows, int B, int cb0, int cb1) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int w = cb1 - cb0;
  if (i >= rows * w) return;
  int64_t r = i / w;
  int c = cb0 + (int)(i - r * w);
  p[r * B + c] = make_double2(0.0, 0.0);
}

hipError_t launch_init_rhs64(int M, int N, int nch, int B, const double* W, const int* wave, const int* j0,
                             const int* g0, double2* s0, hipStream_t st, int cb0, int cb1) {
  if (cb1 < 0) cb1 = B;
  if (cb0 < 0 || cb1 > B || cb0 >= cb1) return hipErrorInvalidValue;
  int64_t rows = (int64_t)M * N * nch;
  int64_t n = rows * (cb1 - cb0);
  hipLaunchKernelGGL(k_fill0_cols, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, s0, rows, B, cb0, cb1);
  hipLaunchKernelGGL(k_set_rhs, dim3(cb1 - cb0), dim3(128), 0, st, M, nch, B, cb0, W, wave, j0, g0, s0);
  return hipGetLastError();
}

hipError_t launch_fill0_cols(double2* p, int64_t rows, int B, int cb0, int cb1, hipStream_t st) {
  if (cb0 < 0 || cb1 > B || cb0 >= cb1) return hipErrorInvalidValue;
  int64_t n = rows * (cb1 - cb0);
  hipLaunchKernelGGL(k_fill0_cols, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, rows, B, cb0, cb1);
  return hipGetLastError();
}

hipError_t launch_fill0(double2* p, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_fill0, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

}  // namespace wpcd

namespace wpcd {

// ------------------------------------------------------------------ step 4: channel resolvent G1

// 1 - r(t)^2 on one edge of the box in the polar variables p = P r cos t, q = Q r sin t:
//   p edge (value v): r = v / (P cos t),  q edge: r = v / (Q sin t).
// ts is the angle at which the energy shell r = 1 meets the edge (acos(v/P) or asin(v/Q); < 0 when
// it does not). Near ts the difference is formed from the node's offset to the segment end it was
// placed from (t - ts = (base - ts) + off, exact when base is ts itself), using
// cos^2 t - cos^2 ts = -sin(t - ts) sin(t + ts) and sin^2 t - sin^2 ts = sin(t - ts) sin(t + ts),
// so that the logarithm keeps full relative accuracy next to its singular point.
__device__ __forceinline__ double g1_omr2(bool pedge, double v, double PQ, double ts, double t, double base,
                                          double off, double st, double ct) {
  if (ts < 0.0) {
    const double r = v / (PQ * (pedge ? ct : st));
    return 1.0 - r * r;
  }
  const double d = (base - ts) + off;
  const double num = sin(d) * sin(t + ts);
  return pedge ? -num / (ct * ct) : num / (st * st);
}

// Continuum element (1/(dp dq)) int int dp dq / (E + i0 - h p^2 - b3 q^2) (eq. dg1b, unit weights),
// evaluated by one wavefront: lanes share the quadrature nodes, a shuffle reduction sums them.
// E < 0: p integral in closed form (arctangent), then q = kappa sinh u with kappa^2 = -E/b3, which
// turns dq / sqrt(b3 q^2 - E) into du / sqrt(b3) and leaves a smooth integrand also when E is
// just below the breakup threshold (the branch points q = +-i kappa then nearly touch q = 0);
// two 20-point Gauss panels in u.
// E > 0: p = P r cos t, q = Q r sin t (P = sqrt(E/h), Q = sqrt(E/b3)) gives
//   Re = (1/sqrt(h b3)) int dt [-1/2 ln|1 - r^2|]_{r_lo(t)}^{r_hi(t)},
// split at the box corners and where the energy shell r = 1 crosses a box edge (log
// singularities), each piece by tanh-sinh; Im = -(pi / (2 sqrt(h b3))) x (angle of the shell
// inside the box).
__device__ double2 g1_continuum_wave(const G1Args& g, int lane, double pa, double pb, double qa, double qb, double E) {
  const double h = g.h2m, b3 = 0.75 * g.h2m;
  double re = 0.0, im = 0.0;
  if (E <= 0.0) {
    const double sh = sqrt(h), sb = sqrt(b3);
    const double kap = sqrt(-E / b3), sE = sqrt(-E);
    // E = 0 exactly (the breakup threshold): plain q, dq / (sb q)
    const double ua = E < 0.0 ? asinh(qa / kap) : qa, ub = E < 0.0 ? asinh(qb / kap) : qb;
    const double mid = 0.5 * (ua + ub);
    double part = 0.0;
    for (int idx = lane; idx < 2 * g.ngl; idx += 64) {
      const int panel = idx / g.ngl, n = idx - panel * g.ngl;
      const double a = panel ? mid : ua, b = panel ? ub : mid;
      const double u = 0.5 * (a + b) + 0.5 * (b - a) * g.gl_x[n];
      // k = sqrt(b3 q^2 - E) at q = kappa sinh u, and dq / k = du / sb
      const double k = E < 0.0 ? sE * cosh(u) : sb * u;
      const double jac = E < 0.0 ? 1.0 / sb : 1.0 / k;
      part += 0.5 * (b - a) * g.gl_w[n] * (-atan2(sh * (pb - pa) * k, k * k + h * pa * pb) / sh) * jac;
    }
    re = wave_sum(part);
  } else {
    const double P = sqrt(E / h), Q = sqrt(E / b3);
    const double t0 = atan2(qa / Q, pb / P), t1 = atan2(qb / Q, pa / P);
    // shell crossings of the four edges (-1: none)
    const double tpa = pa / P < 1.0 ? acos(pa / P) : -1.0, tpb = pb / P < 1.0 ? acos(pb / P) : -1.0;
    const double tqa = qa / Q < 1.0 ? asin(qa / Q) : -1.0, tqb = qb / Q < 1.0 ? asin(qb / Q) : -1.0;
    double pts[8];
    int np = 0;
    pts[np++] = t0;
    pts[np++] = t1;
    const double cand[6] = {atan2(qa / Q, pa / P), atan2(qb / Q, pb / P), tpa, tpb, tqa, tqb};
    for (int c = 0; c < 6; ++c)
      if (cand[c] > t0 && cand[c] < t1) pts[np++] = cand[c];
    for (int x = 1; x < np; ++x)  // insertion sort (np <= 8)
      for (int y = x; y > 0 && pts[y - 1] > pts[y]; --y) {
        double tmp = pts[y];
        pts[y] = pts[y - 1];
        pts[y - 1] = tmp;
      }
    double part = 0.0;
    const int total = (np - 1) * g.nts;
    for (int idx = lane; idx < total; idx += 64) {
      const int sgi = idx / g.nts, n = idx - sgi * g.nts;
      const double a = pts[sgi], b = pts[sgi + 1];
      if (!(b > a)) continue;
      const double u = g.ts_u[n];
      // node placed from the nearer end: t = base + off
      const double base = (u <= 0.5) ? a : b;
      const double off = (u <= 0.5) ? (b - a) * u : -(b - a) * g.ts_v[n];
      const double t = base + off;
      double st, ct;
      sincos(t, &st, &ct);
      // r_lo = max(pa / (P cos t), qa / (Q sin t)), r_hi = min(pb / (P cos t), qb / (Q sin t)),
      // remembering which edge gives each
      double rlo = 0.0;
      int elo = -1;   // 0: p edge pa, 1: q edge qa
      if (pa > 0.0) {
        rlo = pa / (P * ct);
        elo = 0;
      }
      if (qa > 0.0 && qa / (Q * st) > rlo) {
        rlo = qa / (Q * st);
        elo = 1;
      }
      const double rp = pb / (P * ct), rq = qb / (Q * st);
      const bool hp = rp <= rq;
      const double rhi = hp ? rp : rq;
      if (rhi > rlo) {
        const double xh = hp ? g1_omr2(true, pb, P, tpb, t, base, off, st, ct)
                             : g1_omr2(false, qb, Q, tqb, t, base, off, st, ct);
        double f = -0.5 * log(fabs(xh));
        if (elo >= 0) {
          const double xl = elo == 0 ? g1_omr2(true, pa, P, tpa, t, base, off, st, ct)
                                     : g1_omr2(false, qa, Q, tqa, t, base, off, st, ct);
          f += 0.5 * log(fabs(xl));
        }
        if (isfinite(f)) part += 0.5 * (b - a) * g.ts_w[n] * f;   // a node on the shell carries no weight
      }
    }
    re = wave_sum(part) / sqrt(h * b3);
    const double lo_p = acos(fmin(1.0, pb / P)), hi_p = acos(fmin(1.0, pa / P));
    const double lo_q = asin(fmin(1.0, qa / Q)), hi_q = asin(fmin(1.0, qb / Q));
    im = -M_PI / (2.0 * sqrt(h * b3)) * fmax(0.0, fmin(hi_p, hi_q) - fmax(lo_p, lo_q));
  }
  const double d = (pb - pa) * (qb - qa);
  return make_double2(re / d, im / d);
}

// Bound-continuum element (eq. dg1a): (1/dq) int dq / (E + i0 - eps0 - b3 q^2), E - eps0 = b3 q0^2.
__device__ double2 g1_bound_dev(double qa, double qb, double E, double eps0, double h2m) {
  const double b3 = 0.75 * h2m;
  const double q0 = sqrt((E - eps0) / b3);
  const double re = (log(fabs((q0 + qb) / (q0 - qb))) - log(fabs((q0 + qa) / (q0 - qa)))) / (2.0 * b3 * q0);
  const double im = (q0 > qa && q0 <= qb) ? -M_PI / (2.0 * b3 * q0) : 0.0;
  return make_double2(re / (qb - qa), im / (qb - qa));
}

// Element index el = ((w * M + k) * N + j) * nE + e: consecutive lanes take consecutive energies
// of one (w, k, j), so the stores of a wavefront are contiguous in the column index.
struct G1Elem {
  int e, w, k, j;
};
__device__ __forceinline__ G1Elem g1_decode(const G1Args& g, int64_t el) {
  G1Elem d;
  d.e = (int)(el % g.nE);
  int64_t r = el / g.nE;
  d.j = (int)(r % g.N);
  r /= g.N;
  d.k = (int)(r % g.M);
  d.w = (int)(r / g.M);
  return d;
}

__device__ __forceinline__ void g1_store(const G1Args& g, const G1Elem& d, double2 v, int lane0, int stride) {
  const int nout = g.nch * g.nrep;
  for (int o = lane0; o < nout; o += stride) {
    const int ch = o / g.nrep, f = o - ch * g.nrep;
    if (g.wave[ch] != d.w) continue;
    const size_t row = ((size_t)d.j * g.M + d.k) * g.nch + ch;
    g.G[row * g.B + g.col0 + (size_t)d.e * g.nrep + f] = v;
  }
}

// p integral of eq. dg1b in closed form for fixed q, kappa^2 = E - b3 q^2:
//   int_{pa}^{pb} dp / (kappa^2 - h p^2)
//   = atanh(sqrt(h) kappa dp / (kappa^2 - h pa pb)) / (sqrt(h) kappa)      kappa^2 > 0,
//   = -atan2(sqrt(h) dp k, k^2 + h pa pb) / (sqrt(h) k),  k^2 = -kappa^2    kappa^2 < 0,
// valid when kappa^2 is not in [h pa^2, h pb^2] (the pole is outside the p bin).
__device__ __forceinline__ double g1_pint(double k2, double pa, double pb, double sh) {
  const double dp = pb - pa, pp = sh * sh * pa * pb;
  if (k2 > 0.0) {
    const double c = sqrt(k2);
    return atanh(sh * c * dp / (k2 - pp)) / (sh * c);
  }
  if (k2 < 0.0) {
    const double k = sqrt(-k2);
    return -atan2(sh * dp * k, -k2 + pp) / (sh * k);
  }
  return -dp / pp;
}

// Lane rule for a continuum element whose box the energy shell does not cross. After the
// closed-form p integral the q integrand is analytic except on the set where kappa^2 reaches
// [h pa^2, h pb^2]; with q_s its point nearest to the q bin, the 16-point Gauss-Legendre rule is
// exact to rounding when the Bernstein ellipse parameter rho(q_s) of the bin is at least 3
// (error ~ rho^-32). Returns false (element left to the wavefront rule) otherwise.
// Four lanes per element (sub = 0 .. 3, aligned groups of four): each sums the Gauss nodes
// n = sub, sub + 4, ..., and the four partial sums are added by shuffles; the test before the sum
// depends on the element only, so the four lanes of a group always take the same branch.
__device__ bool g1_continuum_lane(const G1Args& g, int sub, double pa, double pb, double qa, double qb, double E,
                                  double2* out) {
  const double h = g.h2m, b3 = 0.75 * g.h2m;
  const double L2 = (E - h * pb * pb) / b3, U2 = (E - h * pa * pa) / b3;   // singular set in q^2
  double xr, xi;                                                           // q_s mapped to [-1, 1]
  const double mid = 0.5 * (qa + qb), half = 0.5 * (qb - qa);
  if (U2 <= 0.0) {
    xr = -mid / half;
    xi = sqrt(-U2) / half;
  } else if (sqrt(U2) < qa) {
    xr = (sqrt(U2) - mid) / half;
    xi = 0.0;
  } else if (L2 > 0.0 && sqrt(L2) > qb) {
    xr = (sqrt(L2) - mid) / half;
    xi = 0.0;
  } else {
    return false;
  }
  // rho = |x + sqrt(x^2 - 1)| on the branch with modulus > 1
  const double ar = xr * xr - xi * xi - 1.0, ai = 2.0 * xr * xi;
  const double mod = sqrt(sqrt(ar * ar + ai * ai));
  const double ang = 0.5 * atan2(ai, ar);
  const double sr = mod * cos(ang), si = mod * sin(ang);
  const double r1 = hypot(xr + sr, xi + si), r2 = hypot(xr - sr, xi - si);
  if (fmax(r1, r2) < 3.0) return false;
  const double sh = sqrt(h);
  double acc = 0.0;
#pragma unroll
  for (int n = sub; n < 16; n += 4) {
    const double q = mid + half * g.gl16_x[n];
    acc += g.gl16_w[n] * g1_pint(E - b3 * q * q, pa, pb, sh);
  }
  acc += __shfl_xor(acc, 1, WARP);
  acc += __shfl_xor(acc, 2, WARP);
  const double d = (pb - pa) * (qb - qa);
  *out = make_double2(acc * half / d, 0.0);   // no shell point inside: real
  return true;
}

// One lane per element: bound-continuum elements and the continuum elements the lane rule
// accepts are written; the others are appended to a work list for k_g1_wave.
__global__ void __launch_bounds__(256) k_g1_lane(G1Args g) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t el = tid >> 2;   // four lanes per element
  const int sub = (int)(tid & 3);
  const int lane = threadIdx.x & 63;
  const int64_t n = (int64_t)g.nwave * g.M * g.N * g.nE;
  bool defer = false;
  if (el < n) {
    const G1Elem d = g1_decode(g, el);
    const double E = g.E[d.e];
    const int nb = g.nb[d.w];
    double2 v;
    bool ok = true;
    if (d.k < nb) {
      v = g1_bound_dev(g.qe[d.j], g.qe[d.j + 1], E, g.eps_b[d.w], g.h2m);
    } else {
      const double* bins = g.bins + (size_t)d.w * (g.M + 1);
      ok = g1_continuum_lane(g, sub, bins[d.k - nb], bins[d.k - nb + 1], g.qe[d.j], g.qe[d.j + 1], E, &v);
    }
    if (ok && sub == 0) g1_store(g, d, v, 0, 1);
    defer = !ok && sub == 0;
  }
  const unsigned long long mask = __ballot(defer);
  if (mask) {
    const int leader = __ffsll((long long)mask) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(g.wl_n, __popcll(mask));
    base = __shfl(base, leader, WARP);
    if (defer) g.wl[base + __popcll(mask & ((1ull << lane) - 1ull))] = el;
  }
}

// One wavefront per deferred element (the boxes the energy shell crosses or passes close to).
__global__ void __launch_bounds__(256) k_g1_wave(G1Args g) {
  const int lane = threadIdx.x & 63;
  const int cnt = *g.wl_n;
  for (int64_t idx = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); idx < cnt; idx += (int64_t)gridDim.x * 4) {
    const G1Elem d = g1_decode(g, g.wl[idx]);
    const double* bins = g.bins + (size_t)d.w * (g.M + 1);
    const int nb = g.nb[d.w];
    const double2 v = g1_continuum_wave(g, lane, bins[d.k - nb], bins[d.k - nb + 1], g.qe[d.j], g.qe[d.j + 1],
                                        g.E[d.e]);
    g1_store(g, d, v, lane, 64);
  }
}

// Energy-weight packets (Sec. III.B, footnote to eqs. dg1a, dg1b): with |w|^2 dp = d eps and
// |f|^2 dq = d eps_q both elements are integrals over energy intervals, x = h p^2 over the
// pseudostate bin (width C), y = b3 q^2 over the q bin (width B).
// Bound-continuum: (1/B) int dy / (E + i0 - eps_n - y) = (1/B) [ln(z1) - ln(z2)],
// z_b = E - eps_n - y_b; Im = -pi / B where z1 > 0 >= z2 (the on-shell bin).
__device__ double2 g1_bound_energy(double qa, double qb, double E, double eps0, double h2m) {
  const double b3 = 0.75 * h2m;
  const double B = b3 * (qb - qa) * (qb + qa);
  const double z1 = (E - eps0) - b3 * qa * qa, z2 = z1 - B;
  const bool on = z1 > 0.0 && z2 <= 0.0;
  const double re = on ? log(z1 / -z2) : log1p(B / z2);   // ln|z1 / z2| = ln|1 + B / z2|
  return make_double2(re / B, on ? -M_PI / B : 0.0);
}
// Continuum: (1/(C B)) int int dx dy / (E + i0 - x - y). The x + y cross-sections of the box have
// the trapezoidal length l(s) (rising over min(C, B), flat, falling), so the element is the mean of
// 1 / (E + i0 - s) under the density l(s) / (C B) of s = X + Y, X, Y uniform on the two bins.
// Im = -pi l(E) / (C B). Re: away from the box (|E - s_c| > 2 (C + B), s_c its centre) the
// expansion 1/(d - u) = sum_n u^n / d^(n+1) over the even central moments mu_n of X + Y
// converges by a factor below 1/16 per term; nearer, the closed form, the sum of +-z ln|z| over
// the corners z = E - x_a - y_b, taken as psi_s(z_s) - psi_s(z_s - l) with s = min(C, B), l the other
// width, z_s the corner z11 - s and psi_s(u) = (u + s) ln|u + s| - u ln|u| = s ln|u + s| +
// u ln|1 + s/u| (log1p where u and u + s have one sign): the difference over the small width is
// formed without cancellation, and the one over the large width cancels at most a few digits.
__device__ __forceinline__ double g1_psi(double u, double s) {
  const double v = u + s;
  if (u == 0.0) return s * log(s);
  if (v == 0.0) return s * log(s);
  if ((u > 0.0) == (v > 0.0)) return s * log(fabs(v)) + u * log1p(s / u);
  return v * log(fabs(v)) - u * log(fabs(u));
}
__device__ double2 g1_continuum_energy(double pa, double pb, double qa, double qb, double E, double h2m) {
  const double h = h2m, b3 = 0.75 * h2m;
  const double x1 = h * pa * pa, y1 = b3 * qa * qa;
  const double C = h * (pb - pa) * (pb + pa), B = b3 * (qb - qa) * (qb + qa);
  const double s0 = x1 + y1;
  const double ell = fmax(0.0, fmin(fmin(E - s0, s0 + C + B - E), fmin(C, B)));
  const double im = -M_PI * ell / (C * B);
  const double d = E - (s0 + 0.5 * (C + B));
  double re;
  if (fabs(d) > 2.0 * (C + B)) {
    // mu_n = 2 (P^(n+2) - Q^(n+2)) / ((n + 1)(n + 2) C B), P = (C + B)/2, Q = (C - B)/2 (n even), so
    // re = (2 d / (C B)) sum_{n even} D_(n+2) / ((n + 1)(n + 2)) with D_m = p^m - q^m, p = P/d,
    // q = Q/d, from D_1 = B/d, D_2 = B C / d^2 and D_(m+2) = (p + q) D_(m+1) - p q D_m (the
    // differences are never formed from the powers themselves)
    const double sc = C / d, tb = B / d;
    const double pq = 0.25 * (sc - tb) * (sc + tb);
    double dm = tb, dm1 = tb * sc;
    double t[16];
#pragma unroll
    for (int h2 = 0; h2 < 16; ++h2) {   // n = 2 h2
      t[h2] = dm1 * (1.0 / ((2.0 * h2 + 1.0) * (2.0 * h2 + 2.0)));   // a constant once unrolled
      const double d3 = fma(sc, dm1, -pq * dm);
      const double d4 = fma(sc, d3, -pq * dm1);
      dm = d3;
      dm1 = d4;
    }
    double sum = 0.0;
#pragma unroll
    for (int h2 = 15; h2 >= 0; --h2) sum += t[h2];   // smallest terms first
    re = 2.0 * d / (C * B) * sum;
  } else {
    const double sw = fmin(C, B), lw = fmax(C, B);
    const double zs = (E - x1 - y1) - sw;
    re = (g1_psi(zs, sw) - g1_psi(zs - lw, sw)) / (C * B);
  }
  return make_double2(re, im);
}

// Energy-weight packets: one thread per output G[row * B + col0 + c], row = (j M + k) nch + ch,
// c = e nrep + f, consecutive threads writing consecutive addresses; the closed forms are cheap
// enough to evaluate again for every channel of a pair wave and every column of an energy.
__global__ void __launch_bounds__(256) k_g1_energy(G1Args g) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int W = g.nE * g.nrep;
  const int64_t n = (int64_t)g.M * g.N * g.nch * W;
  if (t >= n) return;
  const int64_t row = t / W;
  const int c = (int)(t - row * W);
  const int ch = (int)(row % g.nch);
  const int64_t jk = row / g.nch;
  const int k = (int)(jk % g.M), j = (int)(jk / g.M);
  const int w = g.wave[ch];
  const double E = g.E[c / g.nrep];
  const int nb = g.nb[w];
  double2 v;
  if (k < nb) {
    v = g1_bound_energy(g.qe[j], g.qe[j + 1], E, g.eps_b[w], g.h2m);
  } else {
    const double* bins = g.bins + (size_t)w * (g.M + 1);
    v = g1_continuum_energy(bins[k - nb], bins[k - nb + 1], g.qe[j], g.qe[j + 1], E, g.h2m);
  }
  g.G[row * g.B + g.col0 + c] = v;
}

__global__ void k_zero_i32(int* p) {
  if (threadIdx.x == 0) p[0] = 0;
}

int64_t g1_work_elems(int nwave, int M, int N, int nE) { return (int64_t)nwave * M * N * nE; }

hipError_t launch_g1(const G1Args& g, hipStream_t s) {
  if (g.M < 1 || g.N < 1 || g.nE < 1 || g.nwave < 1 || g.nrep < 1 || !g.wl || !g.wl_n) return hipErrorInvalidValue;
  if (g.col0 < 0 || g.col0 + (int64_t)g.nE * g.nrep > g.B) return hipErrorInvalidValue;
  const int64_t n = g1_work_elems(g.nwave, g.M, g.N, g.nE);
  if (g.ew) {
    const int64_t nout = (int64_t)g.M * g.N * g.nch * g.nE * g.nrep;
    hipLaunchKernelGGL(k_g1_energy, dim3((unsigned)((nout + 255) / 256)), dim3(256), 0, s, g);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, g.wl_n);
  hipLaunchKernelGGL(k_g1_lane, dim3((unsigned)((4 * n + 255) / 256)), dim3(256), 0, s, g);
  const int64_t wblocks = std::min<int64_t>(2048, std::max<int64_t>(1, (n + 3) / 4));
  hipLaunchKernelGGL(k_g1_wave, dim3((unsigned)wblocks), dim3(256), 0, s, g);
  return hipGetLastError();
}

}  // namespace wpcd

namespace wpcd {

// ------------------------------------------------------------------ solve: fused block step (FP64)
// For one channel g (pair wave w) and TC columns (j, c): y tile [M][TC] in LDS,
// t = O_w y (capture e0^T O y at k = 0, j = j0[c]), t *= G1, s = (v O^T)_w t, written out.
// Each column's sums run over i (then k) in a fixed order, independent of the tiling.
template <int TC>
__global__ void __launch_bounds__(256) k_step64(RotArgs r, const double* __restrict__ Wm,
                                                const double2* __restrict__ y, double2* __restrict__ s_out) {
  extern __shared__ double2 shc[];
  const int M = r.M, B = r.B, nch = r.nch;
  const int ncol = r.N * B;
  const int g = blockIdx.y;
  const size_t woff = (size_t)r.wave[g] * M * M;
  const double* O = r.A + woff;
  const double* W = Wm + woff;
  const int col0 = blockIdx.x * TC;
  double2* Xs = shc;            // [M][TC]
  double2* Ts = shc + M * TC;   // [M][TC]
  const int tid = threadIdx.x;
  const bool cfast = B >= TC;
  for (int e = tid; e < M * TC; e += 256) {
    int i, cc;
    if (cfast) {
      i = e / TC;
      cc = e - i * TC;
    } else {
      cc = e / M;
      i = e - cc * M;
    }
    const int col = col0 + cc;
    double2 v = make_double2(0.0, 0.0);
    if (col < ncol) {
      const int jj = col / B, cb = col - jj * B;
      v = y[(((size_t)jj * M + i) * nch + g) * B + cb];
    }
    Xs[i * TC + cc] = v;
  }
  __syncthreads();
  const int cc = tid % TC, rg = tid / TC, nrg = 256 / TC;
  const int col = col0 + cc;
  const bool live = col < ncol;
  const int jj = live ? col / B : 0, cb = live ? col - jj * B : 0;
  for (int k = rg; k < M; k += nrg) {
    // four partial sums over i = 0, 1, 2, 3 (mod 4), added in a fixed order: four loads of O in
    // flight per thread instead of one dependent chain
    double ar[4] = {0.0, 0.0, 0.0, 0.0}, ai[4] = {0.0, 0.0, 0.0, 0.0};
    const double* Ok = O + (size_t)k * M;
    int i = 0;
    for (; i + 4 <= M; i += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double a = Ok[i + u];
        const double2 x = Xs[(i + u) * TC + cc];
        ar[u] = fma(a, x.x, ar[u]);
        ai[u] = fma(a, x.y, ai[u]);
      }
    }
    for (int u = 0; i < M; ++i, ++u) {
      const double a = Ok[i];
      const double2 x = Xs[i * TC + cc];
      ar[u] = fma(a, x.x, ar[u]);
      ai[u] = fma(a, x.y, ai[u]);
    }
    double2 v = make_double2((ar[0] + ar[1]) + (ar[2] + ar[3]), (ai[0] + ai[1]) + (ai[2] + ai[3]));
    const double vr = v.x, vi = v.y;
    if (live) {
      if (r.acap && k == 0 && jj == r.j0[cb]) {
        for (int f = 0; f < r.nfin; ++f)
          if (r.finals[f] == g) r.acap[r.acap_off + (int64_t)cb * r.nfin + f] = v;
      }
      const double2 gv = r.G[(((size_t)jj * M + k) * nch + g) * B + cb];
      v = make_double2(vr * gv.x - vi * gv.y, vr * gv.y + vi * gv.x);
    }
    Ts[k * TC + cc] = v;
  }
  __syncthreads();
  for (int i = rg; i < M; i += nrg) {
    double sr[4] = {0.0, 0.0, 0.0, 0.0}, si[4] = {0.0, 0.0, 0.0, 0.0};
    const double* Wi = W + (size_t)i * M;
    int k = 0;
    for (; k + 4 <= M; k += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double a = Wi[k + u];
        const double2 t = Ts[(k + u) * TC + cc];
        sr[u] = fma(a, t.x, sr[u]);
        si[u] = fma(a, t.y, si[u]);
      }
    }
    for (int u = 0; k < M; ++k, ++u) {
      const double a = Wi[k];
      const double2 t = Ts[k * TC + cc];
      sr[u] = fma(a, t.x, sr[u]);
      si[u] = fma(a, t.y, si[u]);
    }
    if (live)
      s_out[(((size_t)jj * M + i) * nch + g) * B + cb] =
          make_double2((sr[0] + sr[1]) + (sr[2] + sr[3]), (si[0] + si[1]) + (si[2] + si[3]));
  }
}

// FP64 MFMA version (v_mfma_f64_16x16x4f64) for one channel g and 8*CT complex columns
// (16*CT real columns, re/im adjacent): Y and T tiles [Mp][16 CT + 1] in LDS (padded rows),
// O and v O^T read as the A operand. Operand layout of the 16x16x4 FP64 instruction: lane l holds
// A[l%16][l/16] and B[l/16][l%16]; the result D[l/16 + 4v][l%16], v = 0..3.
typedef double d4v __attribute__((ext_vector_type(4)));
template <int CT>
__global__ void __launch_bounds__(256) k_step64m(RotArgs r, const double* __restrict__ Wm,
                                                 const double2* __restrict__ y, double2* __restrict__ s_out, int Mp) {
  extern __shared__ double shd[];
  constexpr int RC = 16 * CT, CC = 8 * CT, RCP = RC + 1;
  const int M = r.M, B = r.B, nch = r.nch;
  const int ncol = r.N * B;
  // XCD-aware order (workgroups go round robin to the 8 XCDs by linear id): each XCD takes a
  // contiguous range of (channel, column tile) pairs, so it reads the O and vO^T tables of a few
  // channels, which stay in its L2; the map is a bijection over the grid
  const int ntx = gridDim.x, T = ntx * gridDim.y;
  const int lin = blockIdx.x + ntx * blockIdx.y;
  const int xcd = lin & 7, per = T >> 3, extra = T & 7;
  const int idx = xcd * per + min(xcd, extra) + (lin >> 3);
  const int g = idx / ntx, tile = idx - g * ntx;
  const size_t woff = (size_t)r.wave[g] * M * M;
  const double* O = r.A + woff;
  const double* W = Wm + woff;
  const int col0 = tile * CC;
  double* YT = shd;              // [Mp][RCP]
  double* TT = shd + Mp * RCP;   // [Mp][RCP]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int e = tid; e < CC * Mp; e += 256) {
    int i, cc;
    if (B >= CC) {   // consecutive threads -> consecutive energies
      i = e / CC;
      cc = e - i * CC;
    } else {
      cc = e / Mp;
      i = e - cc * Mp;
    }
    const int col = col0 + cc;
    double2 v = make_double2(0.0, 0.0);
    if (i < M && col < ncol) {
      const int jj = col / B, cb = col - jj * B;
      v = y[(((size_t)jj * M + i) * nch + g) * B + cb];
    }
    YT[i * RCP + 2 * cc] = v.x;
    YT[i * RCP + 2 * cc + 1] = v.y;
  }
  __syncthreads();
  const int r16 = lane & 15, q4 = lane >> 4, part = r16 & 1;
  const int nt = Mp / 16;
  // each wavefront takes two row tiles at a time: 2 x CT independent accumulator chains
  for (int kp = wv; 2 * kp < nt; kp += 4) {
    d4v acc2[2][CT];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) acc2[h][ct] = d4v{0.0, 0.0, 0.0, 0.0};
    const int krow0 = 2 * kp * 16 + r16, krow1 = krow0 + 16;
    const double* Ok0 = O + (size_t)min(krow0, M - 1) * M;
    const double* Ok1 = O + (size_t)min(krow1, M - 1) * M;
#pragma unroll 4
    for (int i0 = 0; i0 < Mp; i0 += 4) {
      const int ic = i0 + q4;
      const double a0 = (krow0 < M && ic < M) ? Ok0[ic] : 0.0;
      const double a1 = (krow1 < M && ic < M) ? Ok1[ic] : 0.0;
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const double b = YT[ic * RCP + ct * 16 + r16];
        acc2[0][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b, acc2[0][ct], 0, 0, 0);
        acc2[1][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b, acc2[1][ct], 0, 0, 0);
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
    const int kt = 2 * kp + h;
    if (kt >= nt) break;
    d4v* acc = acc2[h];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int cc = ct * 8 + (r16 >> 1);
      const int col = col0 + cc;
      const bool live = col < ncol;
      const int jj = live ? col / B : 0, cb = live ? col - jj * B : 0;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = kt * 16 + q4 + 4 * v;
        const double val = acc[ct][v];
        const double other = __shfl_xor(val, 1, WARP);
        const double re = part ? other : val, im = part ? val : other;
        double out = 0.0;
        if (live && k < M) {
          if (r.acap && k == 0 && part == 0 && jj == r.j0[cb]) {
            for (int f = 0; f < r.nfin; ++f)
              if (r.finals[f] == g) r.acap[r.acap_off + (int64_t)cb * r.nfin + f] = make_double2(re, im);
          }
          const double2 gv = r.G[(((size_t)jj * M + k) * nch + g) * B + cb];
          out = part ? (re * gv.y + im * gv.x) : (re * gv.x - im * gv.y);
        }
        TT[k * RCP + ct * 16 + r16] = out;
      }
    }
    }
  }
  __syncthreads();
  double* so = reinterpret_cast<double*>(s_out);
  for (int ip = wv; 2 * ip < nt; ip += 4) {
    d4v acc2[2][CT];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) acc2[h][ct] = d4v{0.0, 0.0, 0.0, 0.0};
    const int irow0 = 2 * ip * 16 + r16, irow1 = irow0 + 16;
    const double* Wi0 = W + (size_t)min(irow0, M - 1) * M;
    const double* Wi1 = W + (size_t)min(irow1, M - 1) * M;
#pragma unroll 4
    for (int k0 = 0; k0 < Mp; k0 += 4) {
      const int kc = k0 + q4;
      const double a0 = (irow0 < M && kc < M) ? Wi0[kc] : 0.0;
      const double a1 = (irow1 < M && kc < M) ? Wi1[kc] : 0.0;
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const double b = TT[kc * RCP + ct * 16 + r16];
        acc2[0][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b, acc2[0][ct], 0, 0, 0);
        acc2[1][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b, acc2[1][ct], 0, 0, 0);
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
    const int it = 2 * ip + h;
    if (it >= nt) break;
    d4v* acc = acc2[h];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int cc = ct * 8 + (r16 >> 1);
      const int col = col0 + cc;
      if (col >= ncol) continue;
      const int jj = col / B, cb = col - jj * B;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = it * 16 + q4 + 4 * v;
        if (i < M) so[2 * ((((size_t)jj * M + i) * nch + g) * B + cb) + part] = acc[ct][v];
      }
    }
    }
  }
}

// Small grids (one energy): one workgroup per 8 complex columns with one wavefront per 16-row
// output tile, so that all row tiles run at once. Each lane first loads its whole A-operand
// fragment (row kt*16 + l%16 of O, then of v O^T, every fourth column from l/16) into registers,
// so a product is one chain of Mp/4 MFMAs with no memory waits inside.
#define STEP64R_MAXK 32   // Mp / 4 for Mp <= 128: at most 8 wavefronts, so 256 VGPRs per lane
// NK = Mp / 4 is a template argument so that the fragment loads and the MFMA chains are straight-line
// code. Out-of-range fragment entries are loaded from a clamped address and kept: they meet only the
// zero rows (i, k >= M) of the LDS tiles or produce output rows that are never stored, and every
// entry of O and v O^T is finite, so they add exact zeros. Masking them instead would make the
// compiler wrap each load in a branch that waits for it.
template <int NK>
__global__ void __launch_bounds__(512) k_step64r(RotArgs r, const double* __restrict__ Wm,
                                                 const double2* __restrict__ y, double2* __restrict__ s_out) {
  extern __shared__ double shd[];
  constexpr int RCP = 17;   // 16 real columns + pad
  constexpr int Mp = 4 * NK;
  const int M = r.M, B = r.B, nch = r.nch;
  const int ncol = r.N * B;
  const int g = blockIdx.y;
  const size_t woff = (size_t)r.wave[g] * M * M;
  const double* O = r.A + woff;
  const double* W = Wm + woff;
  const int col0 = blockIdx.x * 8;
  double* YT = shd;              // [Mp][RCP]
  double* TT = shd + Mp * RCP;   // [Mp][RCP]
  const int tid = threadIdx.x, lane = tid & 63, kt = tid >> 6;
  const int r16 = lane & 15, q4 = lane >> 4, part = r16 & 1;
  const int row = kt * 16 + r16;
  const int rowc = row < M ? row : M - 1;
  // every global load of the kernel is issued here, so that their latencies overlap:
  // the A fragments of O and of v O^T for this wavefront's row tile,
  double af[NK], bf[NK];
  {
    const double* Ok = O + (size_t)rowc * M;
    const double* Wi = W + (size_t)rowc * M;
#pragma unroll
    for (int st = 0; st < NK; ++st) {
      const int ic = 4 * st + q4;
      af[st] = Ok[ic < M ? ic : M - 1];
      bf[st] = Wi[ic < M ? ic : M - 1];
    }
  }
  // the two entries of the y tile that this thread stages (blockDim = 4 Mp, tile = 8 Mp entries),
  double2 yv[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int e = tid + h * 4 * Mp;
    const int cc = e / Mp, i = e - cc * Mp;
    const int col = col0 + cc;
    yv[h] = make_double2(0.0, 0.0);
    if (i < M && col < ncol) {
      const int jj = col / B, cb = col - jj * B;
      yv[h] = y[(((size_t)jj * M + i) * nch + g) * B + cb];
    }
  }
  // and the G1 values of the four output rows this lane owns in the first product
  const int cc_out = r16 >> 1;
  const int col_out = col0 + cc_out;
  const bool live = col_out < ncol;
  const int jj_out = live ? col_out / B : 0, cb_out = live ? col_out - jj_out * B : 0;
  double2 gv[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int k = kt * 16 + q4 + 4 * v;
    gv[v] = r.G[(((size_t)jj_out * M + (k < M ? k : M - 1)) * nch + g) * B + cb_out];
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int e = tid + h * 4 * Mp;
    const int cc = e / Mp, i = e - cc * Mp;
    YT[i * RCP + 2 * cc] = yv[h].x;
    YT[i * RCP + 2 * cc + 1] = yv[h].y;
  }
  __syncthreads();
  d4v acc = d4v{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int st = 0; st < NK; ++st)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(af[st], YT[(4 * st + q4) * RCP + r16], acc, 0, 0, 0);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int k = kt * 16 + q4 + 4 * v;
    const double val = acc[v];
    const double other = __shfl_xor(val, 1, WARP);
    const double re = part ? other : val, im = part ? val : other;
    double out = 0.0;
    if (live && k < M) {
      if (r.acap && k == 0 && part == 0 && jj_out == r.j0[cb_out]) {
        for (int f = 0; f < r.nfin; ++f)
          if (r.finals[f] == g) r.acap[r.acap_off + (int64_t)cb_out * r.nfin + f] = make_double2(re, im);
      }
      out = part ? (re * gv[v].y + im * gv[v].x) : (re * gv[v].x - im * gv[v].y);
    }
    TT[k * RCP + r16] = out;
  }
  __syncthreads();
  acc = d4v{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int st = 0; st < NK; ++st)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[st], TT[(4 * st + q4) * RCP + r16], acc, 0, 0, 0);
  if (live) {
    double* so = reinterpret_cast<double*>(s_out);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = kt * 16 + q4 + 4 * v;
      if (i < M) so[2 * ((((size_t)jj_out * M + i) * nch + g) * B + cb_out) + part] = acc[v];
    }
  }
}

static size_t step64m_lds(int Mp, int ct) { return (size_t)2 * Mp * (16 * ct + 1) * sizeof(double); }

hipError_t launch_step64(const RotArgs& r, const double* W, const double2* y, double2* s_out, hipStream_t s) {
  if (r.M < 1 || r.N < 1 || r.B < 1 || r.nch < 1 || !r.G) return hipErrorInvalidValue;
  const int ncol = r.N * r.B;
  {
    // FP64 MFMA tiles: 16 complex columns per workgroup when the two tiles fit 64 KB of LDS and
    // that still gives every CU a workgroup, else 8
    const int Mp = (r.M + 15) / 16 * 16;
    const size_t lim = 64 * 1024;
    int ct = (step64m_lds(Mp, 2) <= lim && (int64_t)((ncol + 15) / 16) * r.nch >= 256) ? 2 : 1;
    // an explicit choice (WP_STEP_*) that fits the lattice replaces the choice by grid size
    const bool rows_fit = Mp / 4 <= STEP64R_MAXK && step64m_lds(Mp, 1) <= lim;
    bool use_rows = (int64_t)((ncol + 7) / 8) * r.nch < 256 && rows_fit && step64m_lds(Mp, ct) <= lim;
    bool use_m = !use_rows && step64m_lds(Mp, ct) <= lim && (int64_t)((ncol + 7) / 8) * r.nch >= 256;
    if (r.tile == WP_STEP_ROWS && rows_fit) {
      use_rows = true;
      use_m = false;
    } else if ((r.tile == WP_STEP_MFMA8 || r.tile == WP_STEP_MFMA16) &&
               step64m_lds(Mp, r.tile == WP_STEP_MFMA16 ? 2 : 1) <= lim) {
      use_rows = false;
      use_m = true;
      ct = r.tile == WP_STEP_MFMA16 ? 2 : 1;
    } else if (r.tile == WP_STEP_VALU && (size_t)2 * r.M * 2 * sizeof(double2) <= lim) {
      use_rows = use_m = false;
    }
    // a small grid (one energy on few channels) takes k_step64r, whose wavefronts run the row
    // tiles of a column tile in parallel instead of one MFMA chain per tile
    if (use_rows) {
      // small grid: all row tiles of a column tile at once, A fragments preloaded
      dim3 grid((ncol + 7) / 8, r.nch), block(64 * (Mp / 16));
      const size_t sh = step64m_lds(Mp, 1);
      switch (Mp / 16) {
        case 1: hipLaunchKernelGGL(k_step64r<4>, grid, block, sh, s, r, W, y, s_out); break;
        case 2: hipLaunchKernelGGL(k_step64r<8>, grid, block, sh, s, r, W, y, s_out); break;
        case 3: hipLaunchKernelGGL(k_step64r<12>, grid, block, sh, s, r, W, y, s_out); break;
        case 4: hipLaunchKernelGGL(k_step64r<16>, grid, block, sh, s, r, W, y, s_out); break;
        case 5: hipLaunchKernelGGL(k_step64r<20>, grid, block, sh, s, r, W, y, s_out); break;
        case 6: hipLaunchKernelGGL(k_step64r<24>, grid, block, sh, s, r, W, y, s_out); break;
        case 7: hipLaunchKernelGGL(k_step64r<28>, grid, block, sh, s, r, W, y, s_out); break;
        default: hipLaunchKernelGGL(k_step64r<32>, grid, block, sh, s, r, W, y, s_out); break;
      }
      return hipGetLastError();
    }
    if (use_m) {
      dim3 grid((ncol + 8 * ct - 1) / (8 * ct), r.nch);
      if (ct == 2) hipLaunchKernelGGL(k_step64m<2>, grid, dim3(256), step64m_lds(Mp, 2), s, r, W, y, s_out, Mp);
      else hipLaunchKernelGGL(k_step64m<1>, grid, dim3(256), step64m_lds(Mp, 1), s, r, W, y, s_out, Mp);
      return hipGetLastError();
    }
  }
  // large M: the VALU version
  // widest column tile that fits 64 KB of LDS and still gives every CU a workgroup (the threads of a
  // wavefront then share fewer rows of O, so its loads hit fewer cache lines)
  int tc = 16;
  while (tc > 2 && ((size_t)2 * r.M * tc * sizeof(double2) > 64 * 1024 || (int64_t)(ncol / tc) * r.nch < 256)) tc >>= 1;
  // (the large-M branch is also the one an explicit WP_STEP_VALU takes)
  const size_t shmem = (size_t)2 * r.M * tc * sizeof(double2);
  if (shmem > 64 * 1024) return hipErrorInvalidValue;
  dim3 grid((ncol + tc - 1) / tc, r.nch);
  switch (tc) {
    case 16: hipLaunchKernelGGL(k_step64<16>, grid, dim3(256), shmem, s, r, W, y, s_out); break;
    case 8: hipLaunchKernelGGL(k_step64<8>, grid, dim3(256), shmem, s, r, W, y, s_out); break;
    case 4: hipLaunchKernelGGL(k_step64<4>, grid, dim3(256), shmem, s, r, W, y, s_out); break;
    default: hipLaunchKernelGGL(k_step64<2>, grid, dim3(256), shmem, s, r, W, y, s_out); break;
  }
  return hipGetLastError();
}

}  // namespace wpcd

namespace wpcd {

// ------------------------------------------------------------------ block-CSR products, any precision
// VT: stored P0 value type (double / float); XT: vector element (double2 / float2); AT: accumulator.

template <typename XT> struct Acc;
template <> struct Acc<double2> { using T = double; };
template <> struct Acc<float2> { using T = float; };

__device__ __forceinline__ float wave_sum(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WARP);
  return v;
}

template <typename XT, typename AT>
__device__ __forceinline__ XT make_x(AT re, AT im) {
  XT v;
  v.x = re;
  v.y = im;
  return v;
}

// Lanes over the columns (energies): block values and column index are wave-uniform, the
// vector gathers are contiguous over c. For B >= 16.
template <typename VT, typename XT, typename AT, int NC>
__global__ void __launch_bounds__(256) k_spmm(int64_t rows, int B, int cb0, int cb1, const int64_t* __restrict__ rowptr,
                                              const int32_t* __restrict__ col, const VT* __restrict__ val,
                                              const XT* __restrict__ x, XT* __restrict__ y, const int32_t* __restrict__ order) {
  const int64_t row = spmv_row(rows, order);
  const int c = cb0 + blockIdx.y * 64 + (threadIdx.x & 63);
  if (row < 0 || c >= cb1) return;
  const int64_t b0 = rowptr[row], b1 = rowptr[row + 1];
  AT ar[NC], ai[NC];
#pragma unroll
  for (int g = 0; g < NC; ++g) ar[g] = ai[g] = AT(0);
  int64_t e = b0;
  for (; e + 4 <= b1; e += 4) {   // four blocks' gathers in flight; sums in block order
    int cc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) cc[u] = col[e + u];
    XT xv[4][NC];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int gp = 0; gp < NC; ++gp) xv[u][gp] = x[((size_t)cc[u] * NC + gp) * B + c];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const VT* v = val + (e + u) * NC * NC;
#pragma unroll
      for (int gp = 0; gp < NC; ++gp)
#pragma unroll
        for (int g = 0; g < NC; ++g) {
          const AT a = (AT)v[gp * NC + g];
          ar[g] = fma(a, (AT)xv[u][gp].x, ar[g]);
          ai[g] = fma(a, (AT)xv[u][gp].y, ai[g]);
        }
    }
  }
  for (; e < b1; ++e) {
    const int cc = col[e];
    const VT* v = val + e * NC * NC;
#pragma unroll
    for (int gp = 0; gp < NC; ++gp) {
      const XT xv = x[((size_t)cc * NC + gp) * B + c];
#pragma unroll
      for (int g = 0; g < NC; ++g) {
        const AT a = (AT)v[gp * NC + g];
        ar[g] = fma(a, (AT)xv.x, ar[g]);
        ai[g] = fma(a, (AT)xv.y, ai[g]);
      }
    }
  }
#pragma unroll
  for (int g = 0; g < NC; ++g) y[((size_t)row * NC + g) * B + c] = make_x<XT, AT>(ar[g], ai[g]);
}

// LPR lanes per row (half a wavefront as launched, 256 / LPR rows per workgroup), reduction
// within those lanes; for few columns. Rows have ~25 blocks at
// M = N = 100, so a few lanes per row keep the lanes busy with fewer wavefronts.
template <typename VT, typename XT, typename AT, int NC, int LPR>
__global__ void __launch_bounds__(256) k_spmv(int64_t rows, int B, int cb0, int cb1, const int64_t* __restrict__ rowptr,
                                              const int32_t* __restrict__ col, const VT* __restrict__ val,
                                              const XT* __restrict__ x, XT* __restrict__ y, const int32_t* __restrict__ order) {
  const int64_t w = (int64_t)blockIdx.x * (256 / LPR) + threadIdx.x / LPR;
  const int hl = threadIdx.x & (LPR - 1);
  const bool live = w < rows;
  const int64_t row = live ? (order ? order[w] : w) : 0;
  const int64_t b0 = live ? rowptr[row] : 0, b1 = live ? rowptr[row + 1] : 0;
  for (int c = cb0; c < cb1; ++c) {
    AT ar[NC], ai[NC];
#pragma unroll
    for (int g = 0; g < NC; ++g) ar[g] = ai[g] = AT(0);
    for (int64_t e = b0 + hl; e < b1; e += LPR) {
      const int cc = col[e];
      const VT* v = val + e * NC * NC;
#pragma unroll
      for (int gp = 0; gp < NC; ++gp) {
        const XT xv = x[((size_t)cc * NC + gp) * B + c];
#pragma unroll
        for (int g = 0; g < NC; ++g) {
          const AT a = (AT)v[gp * NC + g];
          ar[g] = fma(a, (AT)xv.x, ar[g]);
          ai[g] = fma(a, (AT)xv.y, ai[g]);
        }
      }
    }
#pragma unroll
    for (int g = 0; g < NC; ++g) {
      AT sr = ar[g], si = ai[g];
#pragma unroll
      for (int o = LPR / 2; o > 0; o >>= 1) {   // within the LPR lanes of the row
        sr += __shfl_xor(sr, o, WARP);
        si += __shfl_xor(si, o, WARP);
      }
      if (live && hl == g) y[((size_t)row * NC + g) * B + c] = make_x<XT, AT>(sr, si);
    }
  }
}

static int64_t spmv_blocks(int64_t rows, const int32_t*) { return (rows + 3) / 4; }

template <typename VT, typename XT, typename AT, int NC>
static void spmv_dispatch(int64_t rows, int B, int cb0, int cb1, const int64_t* rowptr, const int32_t* col,
                          const VT* val, const XT* x, XT* y, hipStream_t s, const int32_t* order) {
  // the choice depends on B only, so every launch on a given batch width sums in one order
  if (B >= 16) {
    dim3 grid((unsigned)spmv_blocks(rows, order), (cb1 - cb0 + 63) / 64);
    hipLaunchKernelGGL((k_spmm<VT, XT, AT, NC>), grid, dim3(256), 0, s, rows, B, cb0, cb1, rowptr, col, val, x, y, order);
  } else {
    // 32 lanes per row (16 measured slower at M = N = 100)
    hipLaunchKernelGGL((k_spmv<VT, XT, AT, NC, 32>), dim3((unsigned)((rows + 7) / 8)), dim3(256), 0, s, rows, B, cb0,
                       cb1, rowptr, col, val, x, y, order);
  }
}

template <typename VT, typename XT, typename AT>
hipError_t launch_spmv_gen(int64_t rows, int nch, int B, const int64_t* rowptr, const int32_t* col, const VT* val,
                           const XT* x, XT* y, hipStream_t s, int cb0, int cb1, const int32_t* order,
                           const PackView& pk);

template <typename VT, typename XT, typename AT>
static hipError_t spmv_any(int64_t rows, int nch, int B, const int64_t* rowptr, const int32_t* col, const VT* val,
                           const XT* x, XT* y, hipStream_t s, int cb0, int cb1, const int32_t* order,
                           const PackView& pk) {
  if (cb1 < 0) cb1 = B;
  if (cb0 < 0 || cb1 > B || cb0 >= cb1 || rows < 1) return hipErrorInvalidValue;
  if (nch > 4) return launch_spmv_gen<VT, XT, AT>(rows, nch, B, rowptr, col, val, x, y, s, cb0, cb1, order, pk);
  switch (nch) {
    case 1: spmv_dispatch<VT, XT, AT, 1>(rows, B, cb0, cb1, rowptr, col, val, x, y, s, order); break;
    case 2: spmv_dispatch<VT, XT, AT, 2>(rows, B, cb0, cb1, rowptr, col, val, x, y, s, order); break;
    case 3: spmv_dispatch<VT, XT, AT, 3>(rows, B, cb0, cb1, rowptr, col, val, x, y, s, order); break;
    case 4: spmv_dispatch<VT, XT, AT, 4>(rows, B, cb0, cb1, rowptr, col, val, x, y, s, order); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_spmv_f64(int64_t rows, int nch, int B, const int64_t* rowptr, const int32_t* col, const double* val,
                           const double2* x, double2* y, hipStream_t s, int cb0, int cb1, const int32_t* order,
                           const PackView& pk) {
  return spmv_any<double, double2, double>(rows, nch, B, rowptr, col, val, x, y, s, cb0, cb1, order, pk);
}
hipError_t launch_spmv_f32(int64_t rows, int nch, int B, const int64_t* rowptr, const int32_t* col, const float* val,
                           const float2* x, float2* y, hipStream_t s, int cb0, int cb1, const int32_t* order,
                           const PackView& pk) {
  return spmv_any<float, float2, float>(rows, nch, B, rowptr, col, val, x, y, s, cb0, cb1, order, pk);
}
hipError_t launch_spmv_f32v_f64x(int64_t rows, int nch, int B, const int64_t* rowptr, const int32_t* col,
                                 const float* val, const double2* x, double2* y, hipStream_t s, int cb0, int cb1,
                                 const int32_t* order, const PackView& pk) {
  return spmv_any<float, double2, double>(rows, nch, B, rowptr, col, val, x, y, s, cb0, cb1, order, pk);
}

}  // namespace wpcd

namespace wpcd {

// ------------------------------------------------------------------ step 3 for many channels
// With many channel pairs the P0 value of a cell pair is sum_m C[g][g'][m] I_m over the distinct
// moments I_m = int dx dphi F w_m (Appendix, final formula, one term per (k, l1, l1')). The
// moments of every candidate pair are computed first (node weights in LDS in chunks of MCH,
// F recomputed per chunk), then combined with C in a second, dense contraction.
#define MCH 32

__global__ void __launch_bounds__(256) k_pbuild_mom(PBuildArgs a, const int* __restrict__ cnt, const int* __restrict__ lo,
                                                    const int* __restrict__ segoff, const int64_t* __restrict__ rowptr_c,
                                                    int32_t* __restrict__ col_c, double* __restrict__ mom,
                                                    double* __restrict__ norm) {
  extern __shared__ double sh[];
  const int M = a.M, N = a.N;
  const int nn = a.n_x * a.n_phi;
  const int box = blockIdx.x;
  const int j = box / N, jp = box - j * N;
  const int t = threadIdx.x;
  double* s_r1 = sh;
  double* s_r2 = s_r1 + nn;
  double* s_Q1 = s_r2 + nn;
  double* s_Q2 = s_Q1 + nn;
  double* s_w = s_Q2 + nn;            // [MCH][nn]
  double* s_phi = s_w + MCH * nn;     // [n_phi][PHI_STRIDE]
  double* s_pe = s_phi + PHI_STRIDE * a.n_phi;   // M + 1
  int* s_pref = reinterpret_cast<int*>(s_pe + M + 1);
  int* s_lo = s_pref + M + 1;
  __shared__ int s_total;
  if (t == 0) {
    int run = 0;
    for (int i = 0; i < M; ++i) {
      s_pref[i] = run;
      s_lo[i] = lo[(size_t)box * M + i];
      run += cnt[(size_t)box * M + i];
    }
    s_pref[M] = run;
    s_total = run;
  }
  __syncthreads();
  const int total = s_total;
  if (total == 0) return;
  for (int i = t; i <= M; i += blockDim.x) s_pe[i] = a.pe[i];
  fill_phi_table(a, j, jp, s_phi);
  __syncthreads();
  for (int nd = t; nd < nn; nd += blockDim.x) {
    Node n = box_node_at(a, s_phi, nd);
    s_r1[nd] = n.r1;
    s_r2[nd] = n.r2;
    s_Q1[nd] = n.Q1;
    s_Q2[nd] = n.Q2;
  }
  __syncthreads();
  const double dq = bin_w(a.qe[j], a.qe[j + 1], a.ew), dqp = bin_w(a.qe[jp], a.qe[jp + 1], a.ew);
  for (int m0 = 0; m0 < a.nmom; m0 += MCH) {
    const int mc = min(MCH, a.nmom - m0);
    __syncthreads();
    for (int e = t; e < mc * nn; e += blockDim.x) {
      const int m = e / nn, nd = e - m * nn;
      Node n = box_node_at(a, s_phi, nd);
      s_w[m * nn + nd] = moment_weight(n, a.keys + 5 * (m0 + m));
    }
    __syncthreads();
    for (int e = t; e < total; e += blockDim.x) {
      int lo_i = 0, hi_i = M - 1;
      while (lo_i < hi_i) {
        int mid = (lo_i + hi_i + 1) >> 1;
        if (s_pref[mid] <= e) lo_i = mid;
        else hi_i = mid - 1;
      }
      const int i = lo_i;
      const int ip = s_lo[i] + (e - s_pref[i]);
      const double pa = s_pe[i], pb = s_pe[i + 1], ppa = s_pe[ip], ppb = s_pe[ip + 1];
      double acc[MCH];
#pragma unroll
      for (int m = 0; m < MCH; ++m) acc[m] = 0.0;
      for (int nd = 0; nd < nn; ++nd) {
        const double r1 = s_r1[nd], r2 = s_r2[nd];
        const double U = fmin(s_Q2[nd], fmin(ppb * r1, pb * r2));
        const double L = fmax(s_Q1[nd], fmax(ppa * r1, pa * r2));
        const double F = (U > L) ? f_of(U, L, a.ew != 0) : 0.0;
        if (F != 0.0) {
#pragma unroll
          for (int m = 0; m < MCH; ++m) acc[m] = fma(s_w[m * nn + nd], F, acc[m]);
        }
      }
      const int64_t blk = rowptr_c[(size_t)j * M + i] + segoff[(size_t)box * M + i] + (ip - s_lo[i]);
      for (int m = 0; m < mc; ++m) mom[blk * a.nmom + m0 + m] = acc[m];
      if (m0 == 0) {
        col_c[blk] = jp * M + ip;
        norm[blk] = 1.0 / sqrt(bin_w(pa, pb, a.ew) * dq * bin_w(ppa, ppb, a.ew) * dqp);
      }
    }
  }
}

// val[blk][gg] = norm[blk] * sum_m Ct[m][gg] mom[blk][m]; NBT candidate blocks per workgroup
// with their moments in LDS, threads over the channel pairs gg.
#define NBT 16
__global__ void __launch_bounds__(256) k_combine(int64_t nblk, int nmom, int nc2, const double* __restrict__ Ct,
                                                 const double* __restrict__ mom, const double* __restrict__ norm,
                                                 double* __restrict__ val, uint8_t* __restrict__ flag) {
  extern __shared__ double smom[];   // [NBT][nmom]
  __shared__ int snz[NBT];
  const int64_t b0 = (int64_t)blockIdx.x * NBT;
  const int nb = (int)min((int64_t)NBT, nblk - b0);
  for (int e = threadIdx.x; e < NBT * nmom; e += blockDim.x) {
    const int b = e / nmom, m = e - b * nmom;
    smom[e] = (b < nb) ? mom[(b0 + b) * nmom + m] : 0.0;
  }
  if (threadIdx.x < NBT) snz[threadIdx.x] = 0;
  __syncthreads();
  for (int gg = threadIdx.x; gg < nc2; gg += blockDim.x) {
    double acc[NBT];
#pragma unroll
    for (int b = 0; b < NBT; ++b) acc[b] = 0.0;
    for (int m = 0; m < nmom; ++m) {
      const double c = Ct[(size_t)m * nc2 + gg];
      if (c == 0.0) continue;
#pragma unroll
      for (int b = 0; b < NBT; ++b) acc[b] = fma(c, smom[b * nmom + m], acc[b]);
    }
    for (int b = 0; b < nb; ++b) {
      const double v = acc[b] * norm[b0 + b];
      val[(b0 + b) * nc2 + gg] = v;
      if (v != 0.0) snz[b] = 1;   // benign race: every writer stores 1
    }
  }
  __syncthreads();
  if (threadIdx.x < nb) flag[b0 + threadIdx.x] = (uint8_t)snz[threadIdx.x];
}

hipError_t launch_pbuild_general(const PBuildArgs& a, const double* Ct, const int* cnt, const int* lo, const int* segoff,
                                 const int64_t* rowptr_c, int64_t ncand, int32_t* col_c, double* mom, double* norm,
                                 double* val_c, uint8_t* flag, hipStream_t s) {
  const int nn = a.n_x * a.n_phi;
  if (nn < 1 || nn > PB_MAXNODES || a.nmom < 1 || a.nch < 1) return hipErrorInvalidValue;
  const size_t sh1 = (size_t)nn * (4 + MCH) * sizeof(double) + (size_t)PHI_STRIDE * a.n_phi * sizeof(double) +
                     (a.M + 1) * sizeof(double) + (2 * a.M + 1) * sizeof(int);
  if (sh1 > 64 * 1024) return hipErrorInvalidValue;
  const size_t sh2 = (size_t)NBT * a.nmom * sizeof(double);
  if (sh2 > 64 * 1024) return hipErrorInvalidValue;
  {
    ProfScope ps("pbuild_mom", s);
    hipLaunchKernelGGL(k_pbuild_mom, dim3(a.N * a.N), dim3(256), sh1, s, a, cnt, lo, segoff, rowptr_c, col_c, mom, norm);
  }
  {
    ProfScope ps("combine", s);
    hipLaunchKernelGGL(k_combine, dim3((unsigned)((ncand + NBT - 1) / NBT)), dim3(256), sh2, s, ncand, a.nmom,
                       a.nch * a.nch, Ct, mom, norm, val_c, flag);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ step 3 fused (many moments)
// The stored set is decided from the geometry alone: a candidate pair is kept when F > 0 at one of
// its nodes. With a moment of k = 0 among the keys (its weight is positive at every node) that is
// exactly the rule "some moment integral is nonzero" of the two-pass build above.

// Row prefix of q-box `box` (all threads of the workgroup): s_pref[i] = candidates of the rows
// before i (s_pref[M] = the box total, returned), s_lo[i] = first p' of row i, s_cb[i] = candidate
// index of (row i, p' = s_lo[i]). s_w holds one int per wavefront.
__device__ int box_rows(const PBuildArgs& a, int box, const int* __restrict__ cnt, const int* __restrict__ lo,
                        const int* __restrict__ segoff, const int64_t* __restrict__ rowptr_c, int* s_pref,
                        int* s_lo, int64_t* s_cb, int* s_w) {
  const int M = a.M, j = box / a.N;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, nw = blockDim.x >> 6;
  int carry = 0;
  for (int base = 0; base < M; base += blockDim.x) {
    const int i = base + t;
    int c = 0;
    if (i < M) {
      c = cnt[(size_t)box * M + i];
      s_lo[i] = lo[(size_t)box * M + i];
      s_cb[i] = rowptr_c[(size_t)j * M + i] + segoff[(size_t)box * M + i];
    }
    int v = c;
    for (int o = 1; o < 64; o <<= 1) {
      const int u = __shfl_up(v, o, WARP);
      if (lane >= o) v += u;
    }
    if (lane == 63) s_w[wv] = v;
    __syncthreads();
    int off = carry, tot = 0;
    for (int w = 0; w < nw; ++w) {
      if (w < wv) off += s_w[w];
      tot += s_w[w];
    }
    if (i < M) s_pref[i] = off + v - c;
    carry += tot;
    __syncthreads();
  }
  if (t == 0) s_pref[M] = carry;
  __syncthreads();
  return carry;
}
// the row i of the box's candidate e: the last row with s_pref[i] <= e (a row with candidates)
__device__ __forceinline__ int cand_row(const int* s_pref, int M, int e) {
  int lo_i = 0, hi_i = M - 1;
  while (lo_i < hi_i) {
    const int mid = (lo_i + hi_i + 1) >> 1;
    if (s_pref[mid] <= e) lo_i = mid;
    else hi_i = mid - 1;
  }
  return lo_i;
}

// Also stores the box's node geometry for k_pbuild_fused: geo[box][4 nn + PHI_STRIDE n_phi] =
// r1, r2, Q1, Q2 of every node, then the phi table (boxes without candidates are not written).
__global__ void __launch_bounds__(256) k_pflag(PBuildArgs a, const int* __restrict__ cnt, const int* __restrict__ lo,
                                               const int* __restrict__ segoff, const int64_t* __restrict__ rowptr_c,
                                               uint8_t* __restrict__ flag, int64_t cap, double* __restrict__ geo) {
  extern __shared__ double sh[];
  const int M = a.M, nn = a.n_x * a.n_phi;
  const int box = blockIdx.x, j = box / a.N, jp = box - j * a.N;
  double* s_r1 = sh;
  double* s_r2 = s_r1 + nn;
  double* s_Q1 = s_r2 + nn;
  double* s_Q2 = s_Q1 + nn;
  double* s_phi = s_Q2 + nn;
  int64_t* s_cb = reinterpret_cast<int64_t*>(s_phi + PHI_STRIDE * a.n_phi);
  int* s_pref = reinterpret_cast<int*>(s_cb + M);
  int* s_lo = s_pref + M + 1;
  __shared__ int s_w[4];
  const int total = box_rows(a, box, cnt, lo, segoff, rowptr_c, s_pref, s_lo, s_cb, s_w);
  if (total == 0) return;
  fill_phi_table(a, j, jp, s_phi);
  __syncthreads();
  for (int nd = threadIdx.x; nd < nn; nd += blockDim.x) {
    const Node n = box_node_at(a, s_phi, nd);
    s_r1[nd] = n.r1;
    s_r2[nd] = n.r2;
    s_Q1[nd] = n.Q1;
    s_Q2[nd] = n.Q2;
  }
  __syncthreads();
  const int GS = 4 * nn + PHI_STRIDE * a.n_phi;   // s_r1 .. s_phi are contiguous
  for (int x = threadIdx.x; x < GS; x += blockDim.x) geo[(size_t)box * GS + x] = sh[x];
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    const int i = cand_row(s_pref, M, e);
    const int off = e - s_pref[i];
    const int64_t cand = s_cb[i] + off;
    if (cand >= cap) continue;
    const int ip = s_lo[i] + off;
    const double pa = a.pe[i], pb = a.pe[i + 1], ppa = a.pe[ip], ppb = a.pe[ip + 1];
    bool f = false;
    for (int nd = 0; nd < nn && !f; ++nd) {
      const double r1 = s_r1[nd], r2 = s_r2[nd];
      const double U = fmin(s_Q2[nd], fmin(ppb * r1, pb * r2));
      const double L = fmax(s_Q1[nd], fmax(ppa * r1, pa * r2));
      f = U > L;
    }
    flag[cand] = f ? 1 : 0;
  }
}

// dest[e] = final block index of candidate e (rows of the final block-CSR at rowptr), -1 if dropped
__global__ void __launch_bounds__(256) k_cand_dest(int64_t rows, const int64_t* __restrict__ rowptr_c,
                                                   const uint8_t* __restrict__ flag, const int64_t* __restrict__ rowptr,
                                                   int64_t* __restrict__ dest, int64_t cap_c) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= rows) return;
  const int64_t b0 = min(rowptr_c[row], cap_c), b1 = min(rowptr_c[row + 1], cap_c);
  int64_t out = rowptr[row];
  for (int64_t base = b0; base < b1; base += 64) {
    const int64_t e = base + lane;
    const bool kept = e < b1 && flag[e];
    const unsigned long long mask = __ballot(kept);
    const int before = __popcll(mask & ((1ull << lane) - 1ull));
    if (e < b1) dest[e] = kept ? out + before : -1;
    out += __popcll(mask);
  }
}

__device__ __forceinline__ double legendre_p(int k, double x) {
  double p0 = 1.0, p1 = x, pk = (k == 0) ? 1.0 : x;
  for (int m = 2; m <= k; ++m) {
    const double p2 = ((2.0 * m - 1.0) * x * p1 - (m - 1.0) * p0) / m;
    p0 = p1;
    p1 = p2;
    pk = p2;
  }
  return pk;
}

// One workgroup (4 wavefronts) per q-box. The moment weight of node nd and moment m is the product
// of three small per-box tables, w_x P_k(x) * w_phi c^(a+1) s^(b+1) * zeta1^-(l'+1) zeta2^-(l+1); a
// wavefront keeps the weights of its moment tiles (tiles wv, wv + 4, ...) for all nodes in
// registers, as the B operand of v_mfma_f64_16x16x4f64. The kept candidates of the box are taken
// 16 at a time: their F at every node into LDS (the A operand), the 16 x (16 NTW per wavefront)
// moment integrals into LDS, then threads over (stored value t, 4 candidates) contract them with
// t's nonzero coefficients and write norm * sum to the final arrays (consecutive threads,
// consecutive values of a block). With CL the coefficient lists are staged in LDS once per box.
// LDS: the weight tables and the F / moment tiles share one region (the tables are dead once the
// weights are in registers).
#define FZ_KS 16    // node steps of 4: up to 64 nodes
#define FZ_LCH 256  // candidates listed per pass
#define FZ_MT 18    // LDS row of one moment: 16 candidates + 2 (16-byte aligned, spreads the banks)
struct alignas(16) FusedCoef {
  double cv;
  int m, pad;
};
// LDS layout of k_pbuild_fused (byte offsets). Per workgroup: p and q edges, the Gauss rules, the
// w_x P_k(x) table and (cl) the coefficient lists; per box: the phi and node tables, then one
// region used first for the weight tables (cos/sin powers, 1/zeta powers, node offsets) and then
// for the candidate tiles (F [16][FST], moments [ntl 16][FZ_MT]), the candidate list and the row
// prefix.
struct FusedLds {
  int nn, ntl, FST, EAB, LLP;
  unsigned o_pe, o_qe, o_g, o_PW, o_nof, o_ce, o_cp, o_geo, o_uni, o_mom, o_nrm, o_ld, o_cb, o_pref, o_lo, o_li, o_lip;
  int GS;   // node geometry doubles per box (as k_pflag stores them)
  unsigned total;
};
struct LdsCursor {   // LDS offsets are 32-bit
  unsigned o = 0;
  __host__ __device__ unsigned take(unsigned bytes, unsigned al) {
    o = (o + al - 1) / al * al;
    const unsigned r = o;
    o += bytes;
    return r;
  }
};
__host__ __device__ inline FusedLds fused_layout(const PBuildArgs& a, const FusedArgs& f, bool cl) {
  FusedLds L;
  L.nn = a.n_x * a.n_phi;
  L.ntl = (a.nmom + 15) >> 4;
  L.FST = 4 * FZ_KS + 1;
  L.EAB = f.EA * f.EB;
  L.LLP = f.LL * f.LP;
  LdsCursor c;
  L.o_pe = c.take((unsigned)(a.M + 1) * 8, 16);
  L.o_qe = c.take((unsigned)(a.N + 1) * 8, 8);
  L.o_g = c.take((unsigned)(2 * a.n_x + 2 * a.n_phi) * 8, 8);
  L.o_PW = c.take((unsigned)a.n_x * f.KM * 8, 8);
  L.o_nof = c.take((unsigned)L.nn * 8, 8);
  L.GS = 4 * L.nn + PHI_STRIDE * a.n_phi;
  L.o_ce = cl ? c.take((unsigned)f.ncoef * sizeof(FusedCoef), 16) : 0;
  L.o_cp = cl ? c.take((unsigned)f.vpb * 8, 8) : 0;
  L.o_geo = c.take((unsigned)L.GS * 8, 8);
  const unsigned setup = (unsigned)(a.n_phi * L.EAB + L.nn * L.LLP) * 8;
  const unsigned tiles = (unsigned)(16 * L.FST + L.ntl * 16 * FZ_MT) * 8;
  L.o_uni = c.take(setup > tiles ? setup : tiles, 16);
  L.o_mom = L.o_uni + (unsigned)(16 * L.FST) * 8;
  L.o_nrm = c.take(FZ_LCH * 8, 8);
  L.o_ld = c.take(FZ_LCH * 4, 16);
  L.o_cb = c.take((unsigned)a.M * 8, 8);
  L.o_pref = c.take((unsigned)(a.M + 1) * 4, 4);
  L.o_lo = c.take((unsigned)a.M * 4, 4);
  L.o_li = c.take(FZ_LCH * 4, 4);
  L.o_lip = c.take(FZ_LCH * 4, 4);
  L.total = c.o;
  return L;
}

// Persistent: workgroup b takes the q-boxes b, b + gridDim.x, ... (4 wavefronts each). The moment
// weight of node nd and moment m is the product of three tables, w_x P_k(x) (per workgroup) times
// w_phi c^(a+1) s^(b+1) times zeta1^-(l'+1) zeta2^-(l+1) (per box); a wavefront keeps the weights
// of its moment tiles (tiles wv, wv + 4, ...) for all nodes in registers, as the B operand of
// v_mfma_f64_16x16x4f64. The kept candidates of the box are taken 16 at a time: their F at every
// node into LDS (the A operand), the 16 x 16 NTW moment integrals of each wavefront into LDS
// (moment-major), then threads over (stored value t, 4 candidates) contract them with t's nonzero
// coefficients and write norm * sum to the final arrays (consecutive threads, consecutive values of
// a block). The row data of the next box are loaded while the current box is computed.
template <int NTW, bool CL, typename OT>
__global__ void __launch_bounds__(256, 2) k_pbuild_fused(PBuildArgs a, FusedArgs f, const int* __restrict__ cnt,
                                                      const int* __restrict__ lo, const int* __restrict__ segoff,
                                                      const int64_t* __restrict__ rowptr_c,
                                                      const double* __restrict__ geo,
                                                      const int64_t* __restrict__ dest, int64_t cap_c,
                                                      int32_t* __restrict__ col, OT* __restrict__ out, int64_t cap_b) {
  extern __shared__ __align__(16) unsigned char shb[];
  const FusedLds G = fused_layout(a, f, CL);
  const int GS = G.GS;
  const int M = a.M, N = a.N, nn = G.nn, nmom = a.nmom, ntl = G.ntl, FST = G.FST, EAB = G.EAB, LLP = G.LLP;
  const int n_x = a.n_x, n_phi = a.n_phi, vpb = f.vpb;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, r16 = lane & 15, q4 = lane >> 4;
  double* s_pe = reinterpret_cast<double*>(shb + G.o_pe);
  double* s_qe = reinterpret_cast<double*>(shb + G.o_qe);
  double* s_gx = reinterpret_cast<double*>(shb + G.o_g);
  double* s_gwx = s_gx + n_x;
  double* s_gp = s_gwx + n_x;
  double* s_gwp = s_gp + n_phi;
  double* s_PW = reinterpret_cast<double*>(shb + G.o_PW);          // [n_x][KM]
  FusedCoef* s_ce = reinterpret_cast<FusedCoef*>(shb + G.o_ce);    // [ncoef]  (CL)
  int2* s_cp = reinterpret_cast<int2*>(shb + G.o_cp);              // [vpb]    (CL)
  int2* s_nof = reinterpret_cast<int2*>(shb + G.o_nof);            // [nn] table offsets of a node
  double* s_r1 = reinterpret_cast<double*>(shb + G.o_geo);         // node geometry of the box, as
  double* s_r2 = s_r1 + nn;                                         // k_pflag stored it
  double* s_Q1 = s_r2 + nn;
  double* s_Q2 = s_Q1 + nn;
  double* s_phi = s_Q2 + nn;                                        // [n_phi][PHI_STRIDE]
  double* s_CS = reinterpret_cast<double*>(shb + G.o_uni);         // [n_phi][EA EB]  (set-up)
  double* s_RR = s_CS + n_phi * EAB;                                // [nn][LL LP]     (set-up)
  double* s_F = reinterpret_cast<double*>(shb + G.o_uni);          // [16][FST]       (tiles)
  double* s_mom = reinterpret_cast<double*>(shb + G.o_mom);        // [ntl 16][FZ_MT] (tiles)
  double* s_nrm = reinterpret_cast<double*>(shb + G.o_nrm);
  int* s_ld = reinterpret_cast<int*>(shb + G.o_ld);   // final block index (< cap_b < 2^31)
  int64_t* s_cb = reinterpret_cast<int64_t*>(shb + G.o_cb);
  int* s_pref = reinterpret_cast<int*>(shb + G.o_pref);
  int* s_lo = reinterpret_cast<int*>(shb + G.o_lo);
  int* s_li = reinterpret_cast<int*>(shb + G.o_li);
  int* s_lip = reinterpret_cast<int*>(shb + G.o_lip);
  __shared__ int s_w[4];
  // box-independent tables, once per workgroup
  for (int x = tid; x <= M; x += 256) s_pe[x] = a.pe[x];
  for (int x = tid; x <= N; x += 256) s_qe[x] = a.qe[x];
  for (int x = tid; x < n_x; x += 256) {
    s_gx[x] = a.gx[x];
    s_gwx[x] = a.gwx[x];
  }
  for (int x = tid; x < n_phi; x += 256) {
    s_gp[x] = a.gp[x];
    s_gwp[x] = a.gwp[x];
  }
  for (int x = tid; x < n_x * f.KM; x += 256) {
    const int ia = x / f.KM, k = x - ia * f.KM;
    s_PW[x] = a.gwx[ia] * legendre_p(k, a.gx[ia]);
  }
  if (CL) {
    for (int x = tid; x < f.ncoef; x += 256) {
      FusedCoef e;
      e.cv = f.cv[x];
      e.m = f.cm[x];
      e.pad = 0;
      s_ce[x] = e;
    }
    for (int x = tid; x < vpb; x += 256) s_cp[x] = make_int2(f.cptr[x], f.cptr[x + 1]);
  }
  for (int nd = tid; nd < nn; nd += 256) {
    const int ia = nd / n_phi, ib = nd - ia * n_phi;
    s_nof[nd] = make_int2(ia * f.KM, ib * EAB);
  }
  // moment keys of the wavefront's tiles
  int fk[NTW], fe[NTW], fl[NTW];
  bool fok[NTW];
#pragma unroll
  for (int nt = 0; nt < NTW; ++nt) {
    const int m = (wv + 4 * nt) * 16 + r16;
    fok[nt] = m < nmom;
    fk[nt] = fok[nt] ? f.fkey[3 * m] : 0;
    fe[nt] = fok[nt] ? f.fkey[3 * m + 1] : 0;
    fl[nt] = fok[nt] ? f.fkey[3 * m + 2] : 0;
  }
  const int nbox = N * N;
  // row data (thread = row; M <= 256) and node geometry (GS <= 3 * 256) of the first box
  int rc = 0, rl = 0;
  int64_t rb = 0;
  double rg[3] = {0.0, 0.0, 0.0};
  int box = blockIdx.x;
  if (box < nbox && tid < M) {
    rc = cnt[(size_t)box * M + tid];
    rl = lo[(size_t)box * M + tid];
    rb = rowptr_c[(size_t)(box / N) * M + tid] + segoff[(size_t)box * M + tid];
  }
  if (box < nbox) {
#pragma unroll
    for (int k = 0; k < 3; ++k)
      if (tid + 256 * k < GS) rg[k] = geo[(size_t)box * GS + tid + 256 * k];
  }
  __syncthreads();
  for (; box < nbox; box += gridDim.x) {
    const int j = box / N, jp = box - j * N;
    // row prefix of this box from the registers
    if (tid < M) {
      s_lo[tid] = rl;
      s_cb[tid] = rb;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k)
      if (tid + 256 * k < GS) s_r1[tid + 256 * k] = rg[k];
    int v = rc;
    for (int o = 1; o < 64; o <<= 1) {
      const int u = __shfl_up(v, o, WARP);
      if (lane >= o) v += u;
    }
    if (lane == 63) s_w[wv] = v;
    __syncthreads();
    int off = 0, total = 0;
    for (int w = 0; w < 4; ++w) {
      if (w < wv) off += s_w[w];
      total += s_w[w];
    }
    if (tid < M) s_pref[tid] = off + v - rc;
    if (tid == 0) s_pref[M] = total;
    // the next box's row data and node geometry, in flight while this box is computed
    {
      const int nb = box + gridDim.x;
      rc = 0;
      rl = 0;
      rb = 0;
      if (nb < nbox && tid < M) {
        rc = cnt[(size_t)nb * M + tid];
        rl = lo[(size_t)nb * M + tid];
        rb = rowptr_c[(size_t)(nb / N) * M + tid] + segoff[(size_t)nb * M + tid];
      }
      if (nb < nbox) {
#pragma unroll
        for (int k = 0; k < 3; ++k)
          if (tid + 256 * k < GS) rg[k] = geo[(size_t)nb * GS + tid + 256 * k];
      }
    }
    if (total == 0) {   // uniform; the next box writes LDS only after a barrier
      __syncthreads();
      continue;
    }
    // 1/zeta powers of every (node, l, l') over all threads (energy weights: times the node
    // factor sqrt(c s zeta1 zeta2))
    for (int y = tid; y < nn * LLP; y += 256) {
      const int nd = y / LLP, x = y - nd * LLP, l = x / f.LP, lp = x - l * f.LP;
      const double r1 = s_r1[nd], r2 = s_r2[nd];
      double w = 1.0;
      if (a.ew) {
        const double* t = s_phi + (nd % n_phi) * PHI_STRIDE;
        w = sqrt(t[0] * t[1] / (r1 * r2));
      }
      for (int e = 0; e <= lp; ++e) w *= r1;
      for (int e = 0; e <= l; ++e) w *= r2;
      s_RR[y] = w;
    }
    for (int x = tid; x < n_phi * EAB; x += 256) {
      const int ib = x / EAB, r = x - ib * EAB, ea = r / f.EB, eb = r - ea * f.EB;
      const double* t = s_phi + ib * PHI_STRIDE;
      double w = t[4] * s_gwp[ib];
      for (int e = 0; e <= ea; ++e) w *= t[0];
      for (int e = 0; e <= eb; ++e) w *= t[1];
      s_CS[x] = w;
    }
    __syncthreads();
    // B operands: wr[ks][nt] = weight of node 4 ks + q4, moment (wv + 4 nt) 16 + r16
    double wr[FZ_KS][NTW];
#pragma unroll
    for (int ks = 0; ks < FZ_KS; ++ks) {   // branch-free: reads in range, padding selected to zero
      const int nd = 4 * ks + q4;
      const bool nok = nd < nn;
      const int ndc = nok ? nd : 0;
      const int2 no = s_nof[ndc];
      const double* rr = s_RR + ndc * LLP;
#pragma unroll
      for (int nt = 0; nt < NTW; ++nt) {
        const double w = s_PW[no.x + fk[nt]] * s_CS[no.y + fe[nt]] * rr[fl[nt]];
        wr[ks][nt] = (nok && fok[nt]) ? w : 0.0;
      }
      __builtin_amdgcn_sched_barrier(0);   // bounds the table reads in flight (registers)
    }
    __syncthreads();   // the weight tables are overwritten by the candidate tiles below
    const double dq = bin_w(s_qe[j], s_qe[j + 1], a.ew), dqp = bin_w(s_qe[jp], s_qe[jp + 1], a.ew);
    for (int c0 = 0; c0 < total; c0 += FZ_LCH) {
      // the kept candidates among [c0, c0 + FZ_LCH), in candidate order
      const int e = c0 + tid;
      bool kept = false;
      int i = 0, ip = 0;
      int64_t d = -1;
      if (tid < FZ_LCH && e < total) {
        i = cand_row(s_pref, M, e);
        const int o = e - s_pref[i];
        const int64_t cand = s_cb[i] + o;
        ip = s_lo[i] + o;
        if (cand < cap_c) {
          d = dest[cand];
          kept = d >= 0 && d < cap_b;
        }
      }
      const unsigned long long mask = __ballot(kept);
      if (lane == 0) s_w[wv] = __popcll(mask);
      __syncthreads();
      int pos = __popcll(mask & ((1ull << lane) - 1ull)), nf = 0;
      for (int w = 0; w < 4; ++w) {
        if (w < wv) pos += s_w[w];
        nf += s_w[w];
      }
      if (kept) {
        s_li[pos] = i;
        s_lip[pos] = ip;
        s_ld[pos] = (int)d;
        s_nrm[pos] = 1.0 / sqrt(bin_w(s_pe[i], s_pe[i + 1], a.ew) * dq * bin_w(s_pe[ip], s_pe[ip + 1], a.ew) * dqp);
        col[d] = jp * M + ip;
      }
      __syncthreads();
      for (int r0 = 0; r0 < nf; r0 += 16) {
        const int nr = min(16, nf - r0);
        {  // F of candidate row tid / 16 at nodes tid % 16 + 16 k; nodes past nn stay zero
          const int r = tid >> 4;
          double pa = 0.0, pb = 0.0, ppa = 0.0, ppb = 0.0;
          if (r < nr) {
            const int ii = s_li[r0 + r], iip = s_lip[r0 + r];
            pa = s_pe[ii];
            pb = s_pe[ii + 1];
            ppa = s_pe[iip];
            ppb = s_pe[iip + 1];
          }
          for (int nd = tid & 15; nd < 4 * FZ_KS; nd += 16) {
            double F = 0.0;
            if (r < nr && nd < nn) {
              const double r1 = s_r1[nd], r2 = s_r2[nd];
              const double U = fmin(s_Q2[nd], fmin(ppb * r1, pb * r2));
              const double L = fmax(s_Q1[nd], fmax(ppa * r1, pa * r2));
              F = (U > L) ? f_of(U, L, a.ew != 0) : 0.0;
            }
            s_F[r * FST + nd] = F;
          }
        }
        __syncthreads();
        // branch-free: every node step and every tile of the wavefront (a tile past the last
        // moment has zero weights), so that the accumulators stay in place between instructions
        d4v acc[NTW];
#pragma unroll
        for (int nt = 0; nt < NTW; ++nt) acc[nt] = d4v{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < FZ_KS; ++ks) {
          const double av = s_F[r16 * FST + 4 * ks + q4];
#pragma unroll
          for (int nt = 0; nt < NTW; ++nt)
            acc[nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, wr[ks][nt], acc[nt], 0, 0, 0);
        }
        // moments times the block norm (rows past nr: F = 0, any norm)
        double nrm4[4];
#pragma unroll
        for (int v4 = 0; v4 < 4; ++v4) nrm4[v4] = s_nrm[r0 + q4 + 4 * v4];
#pragma unroll
        for (int nt = 0; nt < NTW; ++nt) {
          const int tg = wv + 4 * nt;
          if (tg < ntl) {
#pragma unroll
            for (int v4 = 0; v4 < 4; ++v4) s_mom[(tg * 16 + r16) * FZ_MT + q4 + 4 * v4] = acc[nt][v4] * nrm4[v4];
          }
        }
        __syncthreads();
        // items (t, rq) = t * nq + rq over (stored value t, 8 candidates rq): the lanes of one value
        // are adjacent, so they read its coefficients once (broadcast) and its moments as one
        // contiguous 128-byte row segment, and a wavefront walks 32 coefficient lists
        const int nq = (nr + 7) >> 3;
        const int nitems = nq * vpb;
        for (int item = tid; item < nitems; item += 256) {
          const int t = nq == 2 ? item >> 1 : item;
          const int rq = item - t * nq;
          const int2 ce = CL ? s_cp[t] : make_int2(f.cptr[t], f.cptr[t + 1]);
          const double* mb = s_mom + 8 * rq;
          double sacc[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) sacc[u] = 0.0;
          for (int c = ce.x; c < ce.y; ++c) {
            double cv;
            int m;
            if (CL) {
              const FusedCoef ec = s_ce[c];
              cv = ec.cv;
              m = ec.m;
            } else {
              cv = f.cv[c];
              m = f.cm[c];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const double2 x = *reinterpret_cast<const double2*>(mb + m * FZ_MT + 2 * u);
              sacc[2 * u] = fma(cv, x.x, sacc[2 * u]);
              sacc[2 * u + 1] = fma(cv, x.y, sacc[2 * u + 1]);
            }
          }
          const int r = 8 * rq;
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (r + u < nr) out[(int64_t)s_ld[r0 + r + u] * vpb + t] = (OT)sacc[u];
        }
        __syncthreads();
      }
    }
  }
}

static size_t pflag_lds(const PBuildArgs& a) {
  const int nn = a.n_x * a.n_phi;
  return ((size_t)4 * nn + PHI_STRIDE * a.n_phi) * 8 + (size_t)a.M * 8 + (2 * (size_t)a.M + 1) * 4;
}

bool fused_build_fits(const PBuildArgs& a, const FusedArgs& f) {
  const int nn = a.n_x * a.n_phi;
  if (nn < 4 || nn > 4 * FZ_KS || nn % 4 != 0 || a.M < 1 || a.M > 256 || 4 * nn + PHI_STRIDE * a.n_phi > 768)
    return false;
  if (a.nmom < 1 || a.nmom > 256 || f.vpb < 1 || f.ncoef < 1) return false;
  if (f.KM < 1 || f.EA < 1 || f.EB < 1 || f.LL < 1 || f.LP < 1) return false;
  return fused_layout(a, f, false).total <= 64 * 1024 && pflag_lds(a) <= 64 * 1024;
}

hipError_t launch_pflag(const PBuildArgs& a, const int* cnt, const int* lo, const int* segoff, const int64_t* rowptr_c,
                        uint8_t* flag, int64_t cap, double* geo, hipStream_t s) {
  const size_t sh = pflag_lds(a);
  if (sh > 64 * 1024 || !geo) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pflag, dim3(a.N * a.N), dim3(64), sh, s, a, cnt, lo, segoff, rowptr_c, flag, cap, geo);
  return hipGetLastError();
}

hipError_t launch_cand_dest(int64_t rows, const int64_t* rowptr_c, const uint8_t* flag, const int64_t* rowptr,
                            int64_t* dest, int64_t cap_c, hipStream_t s) {
  hipLaunchKernelGGL(k_cand_dest, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, s, rows, rowptr_c, flag, rowptr,
                     dest, cap_c);
  return hipGetLastError();
}

template <int NTW, bool CL, typename OT>
static hipError_t launch_fused_k(const PBuildArgs& a, const FusedArgs& f, const int* cnt, const int* lo,
                                 const int* segoff, const int64_t* rowptr_c, const double* geo, const int64_t* dest,
                                 int64_t cap_c, int32_t* col, OT* out, int64_t cap_b, size_t sh, hipStream_t s) {
  auto kern = k_pbuild_fused<NTW, CL, OT>;
  if (sh > 64 * 1024 &&
      hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh) !=
          hipSuccess)
    return hipErrorInvalidValue;
  // persistent: as many workgroups as fit on the device at once, at most one per box
  int dev = 0, ncu = 0, occ = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void*>(kern), 256, sh) != hipSuccess)
    return hipErrorInvalidValue;
  const int nbox = a.N * a.N;
  const int grid = std::max(1, std::min(nbox, std::max(1, occ) * ncu));
  hipLaunchKernelGGL(kern, dim3(grid), dim3(256), sh, s, a, f, cnt, lo, segoff, rowptr_c, geo, dest, cap_c, col, out,
                     cap_b);
  return hipGetLastError();
}

template <bool CL, typename OT>
static hipError_t launch_fused_t(const PBuildArgs& a, const FusedArgs& f, const int* cnt, const int* lo,
                                 const int* segoff, const int64_t* rowptr_c, const double* geo, const int64_t* dest,
                                 int64_t cap_c, int32_t* col, OT* out, int64_t cap_b, hipStream_t s) {
  const int ntw = ((a.nmom + 15) / 16 + 3) / 4;
  const size_t sh = fused_layout(a, f, CL).total;
  switch (ntw) {
    case 1: return launch_fused_k<1, CL>(a, f, cnt, lo, segoff, rowptr_c, geo, dest, cap_c, col, out, cap_b, sh, s);
    case 2: return launch_fused_k<2, CL>(a, f, cnt, lo, segoff, rowptr_c, geo, dest, cap_c, col, out, cap_b, sh, s);
    case 3: return launch_fused_k<3, CL>(a, f, cnt, lo, segoff, rowptr_c, geo, dest, cap_c, col, out, cap_b, sh, s);
    case 4: return launch_fused_k<4, CL>(a, f, cnt, lo, segoff, rowptr_c, geo, dest, cap_c, col, out, cap_b, sh, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename OT>
static hipError_t launch_fused_o(const PBuildArgs& a, const FusedArgs& f, const int* cnt, const int* lo,
                                 const int* segoff, const int64_t* rowptr_c, const double* geo, const int64_t* dest,
                                 int64_t cap_c, int32_t* col, OT* out, int64_t cap_b, hipStream_t s) {
  // the coefficient lists go to LDS when the device gives a workgroup enough of it
  int dev = 0, maxsh = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&maxsh, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return hipErrorInvalidValue;
  const bool cl = fused_layout(a, f, true).total <= (size_t)maxsh;
  return cl ? launch_fused_t<true>(a, f, cnt, lo, segoff, rowptr_c, geo, dest, cap_c, col, out, cap_b, s)
            : launch_fused_t<false>(a, f, cnt, lo, segoff, rowptr_c, geo, dest, cap_c, col, out, cap_b, s);
}

hipError_t launch_pbuild_fused(const PBuildArgs& a, const FusedArgs& f, const int* cnt, const int* lo,
                               const int* segoff, const int64_t* rowptr_c, const double* geo, const int64_t* dest,
                               int64_t cap_c, int32_t* col, double* val64, float* val32, int64_t cap_b,
                               hipStream_t s) {
  if (!fused_build_fits(a, f) || (!val64 == !val32) || !geo || cap_b > 0x7fffffff)
    return hipErrorInvalidValue;
  return val64 ? launch_fused_o(a, f, cnt, lo, segoff, rowptr_c, geo, dest, cap_c, col, val64, cap_b, s)
               : launch_fused_o(a, f, cnt, lo, segoff, rowptr_c, geo, dest, cap_c, col, val32, cap_b, s);
}

// ------------------------------------------------------------------ block-CSR product, many channels
// P0 blocks of many channels are stored packed (PackDesc): pkt[0, NC) = perm (position ->
// canonical channel), pkt[NC, 2NC) = lo, pkt[2NC, 3NC) = hi, pkt[3NC, 4NC) = off of each block
// column u (position), npk values per block. x and y keep the canonical channel order.

template <typename VT, int RPL> struct VecR;
template <> struct VecR<double, 1> { using T = double; };
template <> struct VecR<float, 1> { using T = float; };
template <> struct VecR<double, 2> { using T = double2; };
template <> struct VecR<float, 2> { using T = float2; };
template <typename T> __device__ __forceinline__ T vzero();
template <> __device__ __forceinline__ double vzero<double>() { return 0.0; }
template <> __device__ __forceinline__ float vzero<float>() { return 0.f; }
template <> __device__ __forceinline__ double2 vzero<double2>() { return make_double2(0.0, 0.0); }
template <> __device__ __forceinline__ float2 vzero<float2>() { return make_float2(0.f, 0.f); }
template <typename T> __device__ __forceinline__ T xzero();
template <> __device__ __forceinline__ double2 xzero<double2>() { return make_double2(0.0, 0.0); }
template <> __device__ __forceinline__ float2 xzero<float2>() { return make_float2(0.f, 0.f); }
template <typename T> __device__ __forceinline__ T szero() { return xzero<T>(); }
template <> __device__ __forceinline__ float4 szero<float4>() { return make_float4(0.f, 0.f, 0.f, 0.f); }
template <typename VR> __device__ __forceinline__ float vget(const VR& v, int k);
__device__ __forceinline__ double vget(const double2& v, int k) { return k ? v.y : v.x; }
__device__ __forceinline__ float vget(const float2& v, int k) { return k ? v.y : v.x; }
__device__ __forceinline__ double vget(const double& v, int) { return v; }
__device__ __forceinline__ float vget(const float& v, int) { return v; }

// Few columns (B < 16): one wavefront per block row (rows in the order given, longest first).
// Lanes over (slot s, h): a slot takes one block of the pass (SL blocks per pass), lane h of the
// slot owns the RPL channel rows RPL h .. RPL h + RPL - 1 (positions) and reads, for every block
// column u whose stored interval holds them, RPL consecutive values. The x entries of the pass's
// blocks (SL x NC x CT) are staged in the wavefront's LDS and read back by broadcast; the x loads
// of the next pass are issued into registers before the current pass computes, and the column
// indices one pass further ahead. The values of a pass are loaded UN block columns at a time (all
// of them before the staging when UN = NC). The slots of a row are summed by shuffles in a fixed
// order.
template <int NC, int CT, int UN, bool P2, typename VT, typename XT, typename AT>
__global__ void __launch_bounds__(256) k_spmv_pk(int64_t rows, int B, int cb0, int cb1,
                                                 const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                                                 const VT* __restrict__ val, int npk, const int* __restrict__ pkt,
                                                 const XT* __restrict__ x, XT* __restrict__ y,
                                                 const int32_t* __restrict__ order) {
  constexpr int RPL = (NC % 2 == 0) ? 2 : 1;
  // staging unit: one complex entry, or (P2) two adjacent columns as one 16-byte entry
  using ST = typename std::conditional<P2, float4, XT>::type;
  constexpr int SPC = P2 ? CT / 2 : CT;   // staging units per (slot, column u)
  constexpr int NH = NC / RPL, SL = 64 / NH, PER = NC * SPC, NST = (SL * PER + 63) / 64;
  static_assert(NC % UN == 0, "UN must divide NC");
  static_assert(!P2 || (CT % 2 == 0 && sizeof(XT) == 8), "pairs of complex FP32 columns only");
  using VR = typename VecR<VT, RPL>::T;
  __shared__ ST xs_all[4][SL * PER];
  const int64_t row = spmv_row(rows, order);
  const int lane = threadIdx.x & 63;
  ST* xs = xs_all[threadIdx.x >> 6];
  if (row < 0) return;
  const int s = lane / NH, h = lane - s * NH;
  const bool act = s < SL;
  const int64_t b0 = rowptr[row], b1 = rowptr[row + 1];
  const VR* vr = reinterpret_cast<const VR*>(val);
  const ST* xst = reinterpret_cast<const ST*>(x);
  const int npr = npk / RPL;   // VR entries per block
  const int bst = P2 ? B / 2 : B;   // staging units per (cell, channel)
  // block columns holding this lane's rows (bit u); column u's values start at (off_u - lo_u) / RPL + h
  unsigned inmask = 0;
#pragma unroll
  for (int u = 0; u < NC; ++u)
    if (RPL * h >= pkt[NC + u] && RPL * h < pkt[2 * NC + u]) inmask |= 1u << u;
  for (int c0 = cb0; c0 < cb1; c0 += CT) {
    // staging entry t = k 64 + lane -> (slot, column position u, unit q): its offset within the cell
    int xo[NST];
#pragma unroll
    for (int k = 0; k < NST; ++k) {
      const int t = k * 64 + lane;
      const int sl = t / PER, off = t - sl * PER, u = off / SPC, q = off - u * SPC;
      xo[k] = t < SL * PER ? pkt[u] * bst + (P2 ? (c0 / 2 + q) : min(c0 + q, cb1 - 1)) : 0;
    }
    AT ar[RPL][CT], ai[RPL][CT];
#pragma unroll
    for (int k = 0; k < RPL; ++k)
#pragma unroll
      for (int q = 0; q < CT; ++q) ar[k][q] = ai[k][q] = AT(0);
    ST xreg[NST];
    auto load_x = [&](int64_t cb, int colv) {
      const int nsl = (int)min((int64_t)SL, b1 - cb);
#pragma unroll
      for (int k = 0; k < NST; ++k) {
        const int t = k * 64 + lane, sl = t / PER;
        const int c2 = __shfl(colv, min(sl, SL - 1), WARP);
        // slots past the row end get zeros: their lanes multiply them by zero values
        xreg[k] = (t < SL * PER && sl < nsl) ? xst[(size_t)c2 * NC * bst + xo[k]] : szero<ST>();
      }
    };
    // x of the next pass ahead in registers for complex FP32 vectors; complex FP64 vectors are
    // staged within the pass (register budget)
    constexpr bool XA = sizeof(XT) == 8;
    int colreg = (lane < SL && b0 + lane < b1) ? col[b0 + lane] : 0;
    if (XA && b0 < b1) load_x(b0, colreg);
    int colnext = (lane < SL && b0 + SL + lane < b1) ? col[b0 + SL + lane] : 0;
    for (int64_t cb = b0; cb < b1; cb += SL) {
      if (!XA) load_x(cb, colreg);
#pragma unroll
      for (int k = 0; k < NST; ++k) {
        const int t = k * 64 + lane;
        if (t < SL * PER) xs[t] = xreg[k];
      }
      const int64_t e = cb + s;
      const bool ok = act && e < b1;
      const VR* v = vr + (ok ? e : 0) * npr + h;
      auto ld = [&](int u) -> VR {
        return (ok && ((inmask >> u) & 1u)) ? v[(pkt[3 * NC + u] - pkt[NC + u]) / RPL] : vzero<VR>();
      };
      VR a[UN];
      if (UN == NC) {
#pragma unroll
        for (int u = 0; u < UN; ++u) a[u] = ld(u);
      }
      const int64_t nb = cb + SL;
      if (XA) {
        if (nb < b1) load_x(nb, colnext);
        colnext = (lane < SL && nb + SL + lane < b1) ? col[nb + SL + lane] : 0;
      } else {
        colreg = colnext;
        colnext = (lane < SL && nb + SL + lane < b1) ? col[nb + SL + lane] : 0;
      }
      __builtin_amdgcn_wave_barrier();
      const ST* xr = xs + s * PER;
      // column groups of UN (a rolled loop when UN < NC keeps the register count down)
#pragma nounroll
      for (int u0 = 0; u0 < NC; u0 += UN) {
        if (UN < NC) {
#pragma unroll
          for (int w = 0; w < UN; ++w) a[w] = ld(u0 + w);
        }
#pragma unroll
        for (int w = 0; w < UN; ++w) {
          XT xv[CT];
          if constexpr (P2) {
#pragma unroll
            for (int qq = 0; qq < CT / 2; ++qq) {
              const float4 p = xr[(u0 + w) * SPC + qq];
              xv[2 * qq].x = p.x;
              xv[2 * qq].y = p.y;
              xv[2 * qq + 1].x = p.z;
              xv[2 * qq + 1].y = p.w;
            }
          } else {
#pragma unroll
            for (int q = 0; q < CT; ++q) xv[q] = xr[(u0 + w) * SPC + q];
          }
#pragma unroll
          for (int q = 0; q < CT; ++q) {
#pragma unroll
            for (int k = 0; k < RPL; ++k) {
              ar[k][q] = fma((AT)vget(a[w], k), (AT)xv[q].x, ar[k][q]);
              ai[k][q] = fma((AT)vget(a[w], k), (AT)xv[q].y, ai[k][q]);
            }
          }
        }
      }
      __builtin_amdgcn_wave_barrier();
    }
    // sum over the slots: lane (0, h) collects (s, h), s = 1 .. SL - 1, in order
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
      const int g = pkt[RPL * h + k];   // canonical channel of the lane's row k
#pragma unroll
      for (int q = 0; q < CT; ++q) {
        AT sr = ar[k][q], si = ai[k][q];
        for (int t = 1; t < SL; ++t) {
          const AT r2 = __shfl(ar[k][q], min(lane + t * NH, 63), WARP);
          const AT i2 = __shfl(ai[k][q], min(lane + t * NH, 63), WARP);
          if (s == 0) {
            sr += r2;
            si += i2;
          }
        }
        if (s == 0 && c0 + q < cb1) {
          XT out;
          out.x = sr;
          out.y = si;
          y[((size_t)row * NC + g) * B + c0 + q] = out;
        }
      }
    }
  }
}

// Many columns (B >= 16): lanes over columns, up to NCMAX channel accumulators per lane. The
// wavefront stages each block's packed values into a full NC x NC block (positions, column-major)
// in its own LDS slice, whose never-stored entries are zeroed once, and reads them back by
// broadcast, two rows per read.
#define NCMAX 24
template <typename VT, typename XT, typename AT>
__global__ void __launch_bounds__(256) k_spmm_pk(int64_t rows, int NC, int B, int cb0, int cb1,
                                                 const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                                                 const VT* __restrict__ val, int npk, const int* __restrict__ pkt,
                                                 const int* __restrict__ pk_pos, const XT* __restrict__ x,
                                                 XT* __restrict__ y, const int32_t* __restrict__ order) {
  __shared__ VT vs_all[4][NCMAX * NCMAX + 2];
  VT* vs = vs_all[threadIdx.x >> 6];
  const int64_t row = spmv_row(rows, order);
  const int lane = threadIdx.x & 63;
  const int c = cb0 + blockIdx.y * 64 + lane;
  if (row < 0) return;
  const bool live = c < cb1;
  const int cl = live ? c : cb1 - 1;
  const int64_t b0 = rowptr[row], b1 = rowptr[row + 1];
  const int nc2 = NC * NC;
  for (int t = lane; t < nc2 + 2; t += 64) vs[t] = VT(0);
  AT ar[NCMAX], ai[NCMAX];
#pragma unroll
  for (int g = 0; g < NCMAX; ++g) ar[g] = ai[g] = AT(0);
  for (int64_t e = b0; e < b1; ++e) {
    const int cc = col[e];
    const VT* v = val + e * npk;
    __builtin_amdgcn_wave_barrier();
    for (int t = lane; t < npk; t += 64) vs[pk_pos[t]] = v[t];
    __builtin_amdgcn_wave_barrier();
    for (int gp0 = 0; gp0 < NC; gp0 += 6) {   // six x loads in flight, then their products
      XT xg[6];
#pragma unroll
      for (int u = 0; u < 6; ++u)
        if (gp0 + u < NC) xg[u] = x[((size_t)cc * NC + pkt[gp0 + u]) * B + cl];
#pragma unroll
      for (int u = 0; u < 6; ++u) {
        if (gp0 + u >= NC) break;
        const XT xv = xg[u];
        const VT* vg = vs + (gp0 + u) * NC;   // column u of the block: rows r = 0 .. NC - 1
#pragma unroll
        for (int g = 0; g < NCMAX; g += 2) {
          if (g < NC) {
            const AT a0 = (AT)vg[g], a1 = (g + 1 < NC) ? (AT)vg[g + 1] : AT(0);
            ar[g] = fma(a0, (AT)xv.x, ar[g]);
            ai[g] = fma(a0, (AT)xv.y, ai[g]);
            if (g + 1 < NCMAX) {
              ar[g + 1] = fma(a1, (AT)xv.x, ar[g + 1]);
              ai[g + 1] = fma(a1, (AT)xv.y, ai[g + 1]);
            }
          }
        }
      }
    }
  }
  if (!live) return;
#pragma unroll
  for (int g = 0; g < NCMAX; ++g) {
    if (g < NC) {
      XT out;
      out.x = ar[g];
      out.y = ai[g];
      y[((size_t)row * NC + pkt[g]) * B + c] = out;
    }
  }
}

// values loaded UN block columns at a time: all NC ahead for FP32 values and vectors, else the
// largest of 6, 5, 4, 3, 2, 1 that divides NC (register budget of FP64 data)
template <int NC, typename VT, typename XT>
constexpr int spmv_pk_un() {
  if (sizeof(VT) == 4 && sizeof(XT) == 8) return NC;
  return NC % 6 == 0 ? 6 : NC % 5 == 0 ? 5 : NC % 4 == 0 ? 4 : NC % 3 == 0 ? 3 : NC % 2 == 0 ? 2 : 1;
}

template <int NC, int CT, bool P2, typename VT, typename XT, typename AT>
static void launch_spmv_pk_ct(const dim3& grid, int64_t rows, int B, int cb0, int cb1, const int64_t* rowptr,
                              const int32_t* col, const VT* val, int npk, const int* pkt, const XT* x, XT* y,
                              hipStream_t s, const int32_t* order) {
  hipLaunchKernelGGL((k_spmv_pk<NC, CT, spmv_pk_un<NC, VT, XT>(), P2, VT, XT, AT>), grid, dim3(256), 0, s, rows, B, cb0,
                     cb1, rowptr, col, val, npk, pkt, x, y, order);
}

template <int NC, typename VT, typename XT, typename AT>
static void launch_spmv_pk_nc(const dim3& grid, int64_t rows, int B, int cb0, int cb1, const int64_t* rowptr,
                              const int32_t* col, const VT* val, int npk, const int* pkt, const XT* x, XT* y,
                              hipStream_t s, const int32_t* order) {
  const int ncols = cb1 - cb0;
  // pairs of complex FP32 columns as 16-byte loads when every chunk of 4 is whole and aligned
  const bool p2 = sizeof(XT) == 8 && B % 2 == 0 && cb0 % 2 == 0 && ncols % 4 == 0;
  if constexpr (NC > NCMAX) {   // more than NCMAX channels: four columns per pass only
    launch_spmv_pk_ct<NC, 4, false, VT, XT, AT>(grid, rows, B, cb0, cb1, rowptr, col, val, npk, pkt, x, y, s, order);
  } else {
    if (ncols >= 4 && p2 && sizeof(XT) == 8)
      launch_spmv_pk_ct<NC, 4, sizeof(XT) == 8, VT, XT, AT>(grid, rows, B, cb0, cb1, rowptr, col, val, npk, pkt, x, y,
                                                             s, order);
    else if (ncols >= 4)
      launch_spmv_pk_ct<NC, 4, false, VT, XT, AT>(grid, rows, B, cb0, cb1, rowptr, col, val, npk, pkt, x, y, s, order);
    else if (ncols >= 2)
      launch_spmv_pk_ct<NC, 2, false, VT, XT, AT>(grid, rows, B, cb0, cb1, rowptr, col, val, npk, pkt, x, y, s, order);
    else
      launch_spmv_pk_ct<NC, 1, false, VT, XT, AT>(grid, rows, B, cb0, cb1, rowptr, col, val, npk, pkt, x, y, s, order);
  }
}

template <typename VT, typename XT, typename AT>
hipError_t launch_spmv_gen(int64_t rows, int nch, int B, const int64_t* rowptr, const int32_t* col, const VT* val,
                           const XT* x, XT* y, hipStream_t s, int cb0, int cb1, const int32_t* order,
                           const PackView& pk) {
  if (cb1 < 0) cb1 = B;
  if (cb0 < 0 || cb1 > B || cb0 >= cb1 || rows < 1 || nch < 5 || nch > PK_MAX || !pk.pkt || !pk.pos ||
      pk.npk < 1 || pk.npk > nch * nch)
    return hipErrorInvalidValue;
  // the choice depends on B and nch only, so every launch on a given batch width sums in one order
  const dim3 grid((unsigned)spmv_blocks(rows, order));
  if (B >= pk.spmm_min && nch <= NCMAX) {   // wide calls: lanes over the columns
    dim3 g2 = grid;
    g2.y = (cb1 - cb0 + 63) / 64;
    hipLaunchKernelGGL((k_spmm_pk<VT, XT, AT>), g2, dim3(256), 0, s, rows, nch, B, cb0, cb1, rowptr, col, val, pk.npk,
                       pk.pkt, pk.pos, x, y, order);
    return hipGetLastError();
  }
  switch (nch) {
#define WP_PK_CASE(n) \
  case n: launch_spmv_pk_nc<n, VT, XT, AT>(grid, rows, B, cb0, cb1, rowptr, col, val, pk.npk, pk.pkt, x, y, s, order); break;
    WP_PK_CASE(5) WP_PK_CASE(6) WP_PK_CASE(7) WP_PK_CASE(8) WP_PK_CASE(9) WP_PK_CASE(10) WP_PK_CASE(11)
    WP_PK_CASE(12) WP_PK_CASE(13) WP_PK_CASE(14) WP_PK_CASE(15) WP_PK_CASE(16) WP_PK_CASE(17) WP_PK_CASE(18)
    WP_PK_CASE(19) WP_PK_CASE(20) WP_PK_CASE(21) WP_PK_CASE(22) WP_PK_CASE(23) WP_PK_CASE(24)
    WP_PK_CASE(25) WP_PK_CASE(26) WP_PK_CASE(27) WP_PK_CASE(28) WP_PK_CASE(29) WP_PK_CASE(30) WP_PK_CASE(31)
    WP_PK_CASE(32)
#undef WP_PK_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template hipError_t launch_spmv_gen<double, double2, double>(int64_t, int, int, const int64_t*, const int32_t*,
                                                             const double*, const double2*, double2*, hipStream_t, int, int,
                                                             const int32_t*, const PackView&);
template hipError_t launch_spmv_gen<float, float2, float>(int64_t, int, int, const int64_t*, const int32_t*,
                                                          const float*, const float2*, float2*, hipStream_t, int, int,
                                                          const int32_t*, const PackView&);
template hipError_t launch_spmv_gen<float, double2, double>(int64_t, int, int, const int64_t*, const int32_t*,
                                                            const float*, const double2*, double2*, hipStream_t, int, int,
                                                            const int32_t*, const PackView&);

}  // namespace wpcd
