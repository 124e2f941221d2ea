// Mixed-precision kernels of the iteration (FP32 vectors, BF16 blocks on MFMA with FP32
// accumulation) and the FP64 helpers of the residual refinement.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "wpcd_internal.h"

namespace wpcd {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  // round to nearest even
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// One channel g (pair wave w) and 8*CT complex columns (16*CT real columns: re/im of each):
//   t = O y on MFMA 16x16x16 bf16, t *= G1 (FP32), s = (v O^T) t on MFMA, s written in FP32.
// SPLIT = false: y, t, O and v O^T rounded to bf16 once (one product per tile);
// SPLIT = true: every operand x is carried as hi + lo with hi = bf16(x), lo = bf16(x - hi), and
//   a tile product is A_hi B_hi + A_hi B_lo + A_lo B_hi (16 significant bits per operand).
// Accumulation is FP32 throughout.
// MFMA 16x16x16 bf16 operands: lane l holds A[l%16][4(l/16)+0..3], B[4(l/16)+0..3][l%16];
// the result D[4(l/16)+r][l%16], r = 0..3.
template <bool SPLIT, int CT>
__global__ void __launch_bounds__(256) k_step_bf16(RotArgsMixed r, const float2* __restrict__ y,
                                                   float2* __restrict__ s_out) {
  extern __shared__ uint16_t shb[];
  constexpr int NP = SPLIT ? 2 : 1;
  constexpr int RC = 16 * CT;     // real columns per block
  constexpr int CC = 8 * CT;      // complex columns per block
  const int M = r.M, Mp = r.Mp, B = r.B, nch = r.nch;
  const int ncol = r.N * B;
  // Workgroups are dispatched round robin to the 8 XCDs by linear id. Each XCD is given a
  // contiguous range of (channel, column tile) pairs instead, so that it reads the O and vO^T
  // tables of two or three channels (which then stay in its L2) rather than those of every
  // channel; the map is a bijection over the grid.
  const int ntx = gridDim.x, T = ntx * gridDim.y;
  const int lin = blockIdx.x + ntx * blockIdx.y;
  const int xcd = lin & 7, per = T >> 3, extra = T & 7;
  const int idx = xcd * per + min(xcd, extra) + (lin >> 3);
  const int g = idx / ntx, tile = idx - g * ntx;
  const size_t woff = (size_t)r.wave[g] * Mp * Mp;
  const uint16_t* Oh = r.A + woff;
  const uint16_t* Ol = SPLIT ? r.A_lo + woff : nullptr;
  const uint16_t* Wh = r.W + woff;
  const uint16_t* Wl = SPLIT ? r.W_lo + woff : nullptr;
  const int col0 = tile * CC;
  uint16_t* YT = shb;                      // [NP][RC][Mp], real column rc = 2 cc + part
  uint16_t* TT = shb + NP * RC * Mp;       // [NP][RC][Mp]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int e = tid; e < CC * Mp; e += 256) {
    int cc, i;
    if (B >= CC) {  // consecutive threads -> consecutive energies c
      i = e / CC;
      cc = e - i * CC;
    } else {        // consecutive threads -> consecutive p bins i
      cc = e / Mp;
      i = e - cc * Mp;
    }
    const int col = col0 + cc;
    float2 v = make_float2(0.f, 0.f);
    if (i < M && col < ncol) {
      const int jj = col / B, cb = col - jj * B;
      v = y[(((size_t)jj * M + i) * nch + g) * B + cb];
      if (r.yscale) {
        const float sc = (float)r.yscale[cb];
        v.x *= sc;
        v.y *= sc;
      }
    }
    const uint16_t hx = f2bf(v.x), hy = f2bf(v.y);
    YT[(2 * cc) * Mp + i] = hx;
    YT[(2 * cc + 1) * Mp + i] = hy;
    if (SPLIT) {
      YT[RC * Mp + (2 * cc) * Mp + i] = f2bf(v.x - bf2f(hx));
      YT[RC * Mp + (2 * cc + 1) * Mp + i] = f2bf(v.y - bf2f(hy));
    }
  }
  __syncthreads();
  const int rc = lane & 15, quad = lane >> 4;
  const int part = rc & 1;
  const int nt = Mp / 16;
  for (int kt = wv; kt < nt; kt += 4) {
    f32x4 acc[CT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[ct] = f32x4{0.f, 0.f, 0.f, 0.f};
    // the A operand of the next tile is read while the current one is multiplied (the index is
    // clamped at the last tile, so every read stays in the table)
    const size_t arow = (size_t)(kt * 16 + rc) * Mp + 4 * quad;
    bf16x4 ah_n = *reinterpret_cast<const bf16x4*>(Oh + arow), al_n;
    if (SPLIT) al_n = *reinterpret_cast<const bf16x4*>(Ol + arow);
    for (int it = 0; it < nt; ++it) {
      const bf16x4 ah = ah_n;
      bf16x4 al;
      if (SPLIT) al = al_n;
      const size_t an = arow + (size_t)min(it + 1, nt - 1) * 16;
      ah_n = *reinterpret_cast<const bf16x4*>(Oh + an);
      if (SPLIT) al_n = *reinterpret_cast<const bf16x4*>(Ol + an);
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const int bo = (ct * 16 + rc) * Mp + it * 16 + 4 * quad;
        const bf16x4 bh = *reinterpret_cast<const bf16x4*>(YT + bo);
        acc[ct] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc[ct], 0, 0, 0);
        if (SPLIT) {
          const bf16x4 bl = *reinterpret_cast<const bf16x4*>(YT + RC * Mp + bo);
          acc[ct] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc[ct], 0, 0, 0);
          acc[ct] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc[ct], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int cc = ct * 8 + (rc >> 1);
      const int col = col0 + cc;
      const bool live = col < ncol;
      const int jj = live ? col / B : 0, cb = live ? col - jj * B : 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = kt * 16 + 4 * quad + q;
        const float val = acc[ct][q];
        const float other = __shfl_xor(val, 1, 64);
        const float re = part ? other : val, im = part ? val : other;
        float out = 0.f;
        if (live && k < M) {
          const float2 gv = r.G[(((size_t)jj * M + k) * nch + g) * B + cb];
          out = part ? (re * gv.y + im * gv.x) : (re * gv.x - im * gv.y);
        }
        const uint16_t ho = f2bf(out);
        TT[(ct * 16 + rc) * Mp + k] = ho;
        if (SPLIT) TT[RC * Mp + (ct * 16 + rc) * Mp + k] = f2bf(out - bf2f(ho));
      }
    }
  }
  __syncthreads();
  float* so = reinterpret_cast<float*>(s_out);
  for (int itl = wv; itl < nt; itl += 4) {
    f32x4 acc[CT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[ct] = f32x4{0.f, 0.f, 0.f, 0.f};
    const size_t wrow = (size_t)(itl * 16 + rc) * Mp + 4 * quad;
    bf16x4 ah_n = *reinterpret_cast<const bf16x4*>(Wh + wrow), al_n;
    if (SPLIT) al_n = *reinterpret_cast<const bf16x4*>(Wl + wrow);
    for (int kt = 0; kt < nt; ++kt) {
      const bf16x4 ah = ah_n;
      bf16x4 al;
      if (SPLIT) al = al_n;
      const size_t an = wrow + (size_t)min(kt + 1, nt - 1) * 16;
      ah_n = *reinterpret_cast<const bf16x4*>(Wh + an);
      if (SPLIT) al_n = *reinterpret_cast<const bf16x4*>(Wl + an);
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const int bo = (ct * 16 + rc) * Mp + kt * 16 + 4 * quad;
        const bf16x4 bh = *reinterpret_cast<const bf16x4*>(TT + bo);
        acc[ct] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc[ct], 0, 0, 0);
        if (SPLIT) {
          const bf16x4 bl = *reinterpret_cast<const bf16x4*>(TT + RC * Mp + bo);
          acc[ct] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc[ct], 0, 0, 0);
          acc[ct] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc[ct], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int cc = ct * 8 + (rc >> 1);
      const int col = col0 + cc;
      if (col < ncol) {
        const int jj = col / B, cb = col - jj * B;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = itl * 16 + 4 * quad + q;
          if (i < M) so[2 * ((((size_t)jj * M + i) * nch + g) * B + cb) + part] = acc[ct][q];
        }
      }
    }
  }
}

size_t step_bf16_lds(int Mp, bool split, int ct) { return (size_t)2 * (split ? 2 : 1) * 16 * ct * Mp * sizeof(uint16_t); }

hipError_t launch_step_bf16(const RotArgsMixed& r, const float2* y, float2* s_out, hipStream_t s) {
  if (r.M < 1 || r.Mp < r.M || r.Mp % 16 || r.N < 1 || r.B < 1 || r.nch < 1 || !r.G || !r.A || !r.W)
    return hipErrorInvalidValue;
  const bool split = r.A_lo != nullptr;
  if (split && !r.W_lo) return hipErrorInvalidValue;
  const size_t lim = 64 * 1024;
  const int ct = step_bf16_lds(r.Mp, split, 2) <= lim ? 2 : 1;
  const size_t shmem = step_bf16_lds(r.Mp, split, ct);
  if (shmem > lim) return hipErrorInvalidValue;
  dim3 grid((r.N * r.B + 8 * ct - 1) / (8 * ct), r.nch);
  if (split) {
    if (ct == 2) hipLaunchKernelGGL((k_step_bf16<true, 2>), grid, dim3(256), shmem, s, r, y, s_out);
    else hipLaunchKernelGGL((k_step_bf16<true, 1>), grid, dim3(256), shmem, s, r, y, s_out);
  } else {
    if (ct == 2) hipLaunchKernelGGL((k_step_bf16<false, 2>), grid, dim3(256), shmem, s, r, y, s_out);
    else hipLaunchKernelGGL((k_step_bf16<false, 1>), grid, dim3(256), shmem, s, r, y, s_out);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ refinement helpers (FP64)

__global__ void k_cvt_d2f(int64_t n, const double2* __restrict__ in, float2* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = make_float2((float)in[i].x, (float)in[i].y);
}

__global__ void k_cvt_scalar(int64_t n, const double* __restrict__ in, float* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
}

hipError_t launch_cvt_scalar(int64_t n, const double* in, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_cvt_scalar, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, in, out);
  return hipGetLastError();
}

// the columns [c0, c1) of a [rows][B] array
__global__ void k_cvt_d2f_cols(int64_t rows, int B, int c0, int c1, const double2* __restrict__ in,
                               float2* __restrict__ out) {
  const int w = c1 - c0;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows * w) return;
  const int64_t d = t / w;
  const size_t i = (size_t)d * B + c0 + (int)(t - d * w);
  out[i] = make_float2((float)in[i].x, (float)in[i].y);
}

hipError_t launch_cvt_d2f_cols(int64_t rows, int B, int c0, int c1, const double2* in, float2* out, hipStream_t s) {
  if (c0 < 0 || c1 > B || c0 >= c1) return hipErrorInvalidValue;
  const int64_t n = rows * (c1 - c0);
  hipLaunchKernelGGL(k_cvt_d2f_cols, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, rows, B, c0, c1, in, out);
  return hipGetLastError();
}

hipError_t launch_cvt_d2f(int64_t n, const double2* in, float2* out, hipStream_t s) {
  hipLaunchKernelGGL(k_cvt_d2f, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, in, out);
  return hipGetLastError();
}

// r = b - y + Ky
__global__ void k_residual(int64_t n, const double2* __restrict__ b, const double2* __restrict__ y,
                           const double2* __restrict__ Ky, double2* __restrict__ r) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) r[i] = make_double2(b[i].x - y[i].x + Ky[i].x, b[i].y - y[i].y + Ky[i].y);
}

hipError_t launch_residual(int64_t n, const double2* b, const double2* y, const double2* Ky, double2* r, hipStream_t s) {
  hipLaunchKernelGGL(k_residual, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, b, y, Ky, r);
  return hipGetLastError();
}

// out[d][c] += sum_m coef[m][c] * vecs[m][d][c] (complex coefficients, FP64 accumulation)
__global__ void k_lincomb(int64_t rows, int B, int nv, const float2* __restrict__ vecs, int64_t vstride,
                          const double2* __restrict__ coef, double2* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * B) return;
  const int c = (int)(i % B);
  double sr = 0.0, si = 0.0;
  for (int m = 0; m < nv; ++m) {
    const double2 w = coef[(size_t)m * B + c];
    if (w.x == 0.0 && w.y == 0.0) continue;
    const float2 v = vecs[(size_t)m * vstride + i];
    sr += w.x * v.x - w.y * v.y;
    si += w.x * v.y + w.y * v.x;
  }
  out[i] = make_double2(out[i].x + sr, out[i].y + si);
}

hipError_t launch_lincomb(int64_t rows, int B, int nv, const float2* vecs, int64_t vstride, const double2* coef,
                          double2* out, hipStream_t s) {
  if (vstride < rows * B) return hipErrorInvalidValue;
  const int64_t n = rows * B;
  hipLaunchKernelGGL(k_lincomb, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, rows, B, nv, vecs, vstride, coef,
                     out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ Arnoldi (per column c)
// Vectors are [rows][B] float2 (rows = D lattice entries, row d = cell * nch + g); a basis is
// kept unnormalised, V_i = scl[i][c] * Vt_i, with the basis slots vstride apart. Every kernel
// below has lanes over 64 columns (blockIdx.y picks the column block) and waves striding over
// rows; FP64 partial sums per block are reduced in LDS and written to part[blk][i][c], which a
// wavefront-per-output pass sums in a fixed order (results do not depend on scheduling).

// Lane layout of the column kernels: with Bp = min(64, B rounded up to a power of two), lane l
// takes column blockIdx.y * 64 + l % Bp and row offset l / Bp, so a wavefront covers 64 / Bp rows
// per pass and no lane idles for small B.
struct ArnLanes {
  int Bp, R, cw, rsub, c;
  bool live;
};
__device__ __forceinline__ ArnLanes arn_lanes(int B) {
  ArnLanes a;
  const int lane = threadIdx.x & 63;
  const int bb = B - (int)blockIdx.y * 64;
  a.Bp = 64;
  if (bb < 64) {
    a.Bp = 1;
    while (a.Bp < bb) a.Bp <<= 1;
  }
  a.R = 64 / a.Bp;
  a.cw = lane % a.Bp;
  a.rsub = lane / a.Bp;
  a.c = (int)blockIdx.y * 64 + a.cw;
  a.live = a.c < B;
  return a;
}

// Sums the per-lane partials (hr, hi)[0 .. nv) of equal column over the lanes and waves of the
// block (fixed order: wave, then row offset) into part[blk][i][c].
template <int NV>
__device__ __forceinline__ void arn_block_reduce(const double (&hr)[NV], const double (&hi)[NV], int nv,
                                                 const ArnLanes& ln, int B, double2* __restrict__ part) {
  __shared__ double2 red[4][4][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  static_assert(NV % 4 == 0, "partials are reduced four at a time");
#pragma unroll
  for (int i0 = 0; i0 < NV; i0 += 4) {
    if (i0 < nv) {   // uniform over the block
#pragma unroll
      for (int q = 0; q < 4; ++q) red[wv][q][lane] = make_double2(hr[i0 + q], hi[i0 + q]);
      __syncthreads();
      const int q = wv, i = i0 + wv, l = lane;
      const int c = (int)blockIdx.y * 64 + l;
      if (l < ln.Bp && i < nv && c < B) {
        double2 t = make_double2(0.0, 0.0);
        for (int w4 = 0; w4 < 4; ++w4)
          for (int r = 0; r < ln.R; ++r) {
            t.x += red[w4][q][r * ln.Bp + l].x;
            t.y += red[w4][q][r * ln.Bp + l].y;
          }
        part[((size_t)blockIdx.x * nv + i) * B + c] = t;
      }
      __syncthreads();
    }
  }
}

template <int NV>
__device__ __forceinline__ void arn_dot_row(const float2* __restrict__ V, int64_t vstride, int nv, size_t idx,
                                            float wr, float wi, double (&hr)[NV], double (&hi)[NV]) {
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    if (q < nv) {
      const float2 v = V[(size_t)q * vstride + idx];
      hr[q] += (double)v.x * wr + (double)v.y * wi;
      hi[q] += (double)v.x * wi - (double)v.y * wr;
    }
  }
}

// Fused Arnoldi product for B >= 16, nch <= 4: w = V_j - P0 t (block-CSR, lanes over columns,
// the nonzero blocks of a row taken four at a time so their gathers overlap), w stored in basis
// slot j + 1, and the partial sums of conj(Vt_i) w for i <= j.
template <int NC>
__global__ void __launch_bounds__(256) k_spmm_arn(int64_t cells, int B, const int64_t* __restrict__ rowptr,
                                                  const int32_t* __restrict__ col, const float* __restrict__ val,
                                                  const int32_t* __restrict__ order,
                                                  const float2* __restrict__ t, float2* __restrict__ V,
                                                  int64_t vstride, int j, const double* __restrict__ scl,
                                                  double2* __restrict__ part) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  ArnLanes ln;
  ln.Bp = 64;
  ln.R = 1;
  ln.cw = lane;
  ln.rsub = 0;
  ln.c = blockIdx.y * 64 + lane;
  ln.live = ln.c < B;
  const int c = ln.c;
  const bool live = ln.live;
  const int cl = live ? c : B - 1;
  const float2* Vj = V + (size_t)j * vstride;
  float2* Wo = V + (size_t)(j + 1) * vstride;
  const float sj = (float)scl[(size_t)j * B + cl];
  const int nv = j + 1;
  double hr[ARN_NV], hi[ARN_NV];
#pragma unroll
  for (int q = 0; q < ARN_NV; ++q) hr[q] = hi[q] = 0.0;
  for (int64_t rw = (int64_t)blockIdx.x * 4 + wv; rw < cells; rw += (int64_t)gridDim.x * 4) {
    const int64_t row = order ? order[rw] : rw;
    float ar[NC], ai[NC];
#pragma unroll
    for (int g = 0; g < NC; ++g) ar[g] = ai[g] = 0.f;
    const int64_t b0 = rowptr[row], b1 = rowptr[row + 1];
    int64_t e = b0;
    for (; e + 8 <= b1; e += 8) {   // eight blocks' gathers in flight; sums in block order
      int cc[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) cc[u] = col[e + u];
      float2 xv[8][NC];
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int gp = 0; gp < NC; ++gp) xv[u][gp] = t[((size_t)cc[u] * NC + gp) * B + cl];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const float* v = val + (e + u) * NC * NC;
#pragma unroll
        for (int gp = 0; gp < NC; ++gp)
#pragma unroll
          for (int g = 0; g < NC; ++g) {
            const float a = v[gp * NC + g];
            ar[g] = fmaf(a, xv[u][gp].x, ar[g]);
            ai[g] = fmaf(a, xv[u][gp].y, ai[g]);
          }
      }
    }
    for (; e < b1; ++e) {
      const int cc = col[e];
      const float* v = val + e * NC * NC;
#pragma unroll
      for (int gp = 0; gp < NC; ++gp) {
        const float2 xv = t[((size_t)cc * NC + gp) * B + cl];
#pragma unroll
        for (int g = 0; g < NC; ++g) {
          const float a = v[gp * NC + g];
          ar[g] = fmaf(a, xv.x, ar[g]);
          ai[g] = fmaf(a, xv.y, ai[g]);
        }
      }
    }
#pragma unroll
    for (int g = 0; g < NC; ++g) {
      const size_t idx = ((size_t)row * NC + g) * B + cl;
      const float2 v = Vj[idx];
      const float wr = sj * v.x - ar[g], wi = sj * v.y - ai[g];
      if (live) Wo[idx] = make_float2(wr, wi);
      arn_dot_row(V, vstride, nv, idx, wr, wi, hr, hi);
    }
  }
  arn_block_reduce(hr, hi, nv, ln, B, part);
}

// Unfused variant (any B, any nch): w = V_j - kv with kv = P0 t from the general SpMM.
// NV: basis slots held per lane (8 when the cycle has at most 8 Arnoldi steps, else ARN_NV): fewer
// registers, more waves in flight for these bandwidth-bound passes.
template <int NV>
__global__ void __launch_bounds__(256) k_sub_dots(int64_t rows, int B, const float2* __restrict__ kv,
                                                  float2* __restrict__ V, int64_t vstride, int j,
                                                  const double* __restrict__ scl, double2* __restrict__ part) {
  const int wv = threadIdx.x >> 6;
  const ArnLanes ln = arn_lanes(B);
  const int cl = ln.live ? ln.c : B - 1;
  const float2* Vj = V + (size_t)j * vstride;
  float2* Wo = V + (size_t)(j + 1) * vstride;
  const float sj = (float)scl[(size_t)j * B + cl];
  const int nv = j + 1;
  double hr[NV], hi[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) hr[q] = hi[q] = 0.0;
  const int64_t step = (int64_t)gridDim.x * 4 * ln.R;
  // two rows per pass, all their reads issued before the store (the output slot shares the basis
  // buffer, so the reads of a later row could not move above it); the sums take the rows in the
  // same order as one row per pass
  for (int64_t d = ((int64_t)blockIdx.x * 4 + wv) * ln.R + ln.rsub; d < rows; d += 2 * step) {
    const bool two = d + step < rows;
    const size_t i1 = (size_t)d * B + cl, i2 = (size_t)(two ? d + step : d) * B + cl;
    const float2 v1 = Vj[i1], k1 = kv[i1], v2 = Vj[i2], k2 = kv[i2];
    float2 b1[NV], b2[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q)
      if (q < nv) {
        b1[q] = V[(size_t)q * vstride + i1];
        b2[q] = V[(size_t)q * vstride + i2];
      }
    const float w1r = sj * v1.x - k1.x, w1i = sj * v1.y - k1.y;
    const float w2r = sj * v2.x - k2.x, w2i = sj * v2.y - k2.y;
    if (ln.live) {
      Wo[i1] = make_float2(w1r, w1i);
      if (two) Wo[i2] = make_float2(w2r, w2i);
#pragma unroll
      for (int q = 0; q < NV; ++q)
        if (q < nv) {
          hr[q] += (double)b1[q].x * w1r + (double)b1[q].y * w1i;
          hi[q] += (double)b1[q].x * w1i - (double)b1[q].y * w1r;
        }
      if (two) {
#pragma unroll
        for (int q = 0; q < NV; ++q)
          if (q < nv) {
            hr[q] += (double)b2[q].x * w2r + (double)b2[q].y * w2i;
            hi[q] += (double)b2[q].x * w2i - (double)b2[q].y * w2r;
          }
      }
    }
  }
  arn_block_reduce(hr, hi, nv, ln, B, part);
}

// w -= sum_{i <= j} h_i V_i (FP64 arithmetic, FP32 storage) in basis slot j + 1, with the partial
// sums of |w|^2 of the stored values.
template <int NV>
__global__ void __launch_bounds__(256) k_orth_norm(int64_t rows, int B, float2* __restrict__ V, int64_t vstride, int j,
                                                   const double2* __restrict__ h, const double* __restrict__ scl,
                                                   double2* __restrict__ part) {
  const int wv = threadIdx.x >> 6;
  const ArnLanes ln = arn_lanes(B);
  const int cl = ln.live ? ln.c : B - 1;
  const int nv = j + 1;
  double cr[NV], ci[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    cr[q] = ci[q] = 0.0;
    if (q < nv) {
      const double sc = scl[(size_t)q * B + cl];
      cr[q] = h[(size_t)q * B + cl].x * sc;
      ci[q] = h[(size_t)q * B + cl].y * sc;
    }
  }
  float2* Wo = V + (size_t)(j + 1) * vstride;
  double acc[4], dummy[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = dummy[q] = 0.0;
  const int64_t step = (int64_t)gridDim.x * 4 * ln.R;
  // two rows per pass, their reads before the stores, sums in row order (as in k_sub_dots)
  for (int64_t d = ((int64_t)blockIdx.x * 4 + wv) * ln.R + ln.rsub; d < rows; d += 2 * step) {
    if (!ln.live) continue;
    const bool two = d + step < rows;
    const size_t i1 = (size_t)d * B + cl, i2 = (size_t)(two ? d + step : d) * B + cl;
    const float2 w1 = Wo[i1], w2 = Wo[i2];
    float2 b1[NV], b2[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q)
      if (q < nv) {
        b1[q] = V[(size_t)q * vstride + i1];
        b2[q] = V[(size_t)q * vstride + i2];
      }
    double x1r = w1.x, x1i = w1.y, x2r = w2.x, x2i = w2.y;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      if (q < nv) {
        x1r -= cr[q] * b1[q].x - ci[q] * b1[q].y;
        x1i -= cr[q] * b1[q].y + ci[q] * b1[q].x;
        x2r -= cr[q] * b2[q].x - ci[q] * b2[q].y;
        x2i -= cr[q] * b2[q].y + ci[q] * b2[q].x;
      }
    }
    const float2 o1 = make_float2((float)x1r, (float)x1i), o2 = make_float2((float)x2r, (float)x2i);
    Wo[i1] = o1;
    acc[0] += (double)o1.x * o1.x + (double)o1.y * o1.y;
    if (two) {
      Wo[i2] = o2;
      acc[0] += (double)o2.x * o2.x + (double)o2.y * o2.y;
    }
  }
  arn_block_reduce(acc, dummy, 1, ln, B, part);
}

__device__ __forceinline__ double wsum64(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// One wavefront per output (i, c), lanes over the blocks in a fixed order.
// mode 0: out[i][c] = scl[i][c] * sum_blk part[blk][i][c]       (Hessenberg column, i < nv)
// mode 1: n = sqrt(sum_blk part[blk][0][c].x); out[0][c] = n;    (subdiagonal entry)
//         scl_next[c] = 1 / n (0 for a zero vector)
__global__ void __launch_bounds__(256) k_arn_finish(int nblk, int B, int nv, const double2* __restrict__ part,
                                                    const double* __restrict__ scl, double2* __restrict__ out,
                                                    double* __restrict__ scl_next, int mode) {
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (t >= nv * B) return;
  const int i = t / B, c = t - i * B;
  double sr = 0.0, si = 0.0;
  for (int b = lane; b < nblk; b += 64) {
    const double2 v = part[((size_t)b * nv + i) * B + c];
    sr += v.x;
    si += v.y;
  }
  sr = wsum64(sr);
  si = wsum64(si);
  if (lane == 0) {
    if (mode == 0) {
      const double sc = scl ? scl[(size_t)i * B + c] : 1.0;
      out[t] = make_double2(sr * sc, si * sc);
    } else {
      const double n = sqrt(fmax(sr, 0.0));
      out[c] = make_double2(n, 0.0);
      scl_next[c] = n > 1e-300 ? 1.0 / n : 0.0;
    }
  }
}

static dim3 arn_grid(int64_t rows, int B, int nblk) {
  const int64_t need = (rows + 3) / 4;
  return dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(nblk, need)), (unsigned)((B + 63) / 64));
}

int arn_blocks(int64_t rows, int B, int nblk) { return (int)arn_grid(rows, B, nblk).x; }

template <int NC>
static void spmm_arn_launch(dim3 grid, hipStream_t s, int64_t cells, int B, const int64_t* rowptr, const int32_t* col,
                            const float* val, const int32_t* order, const float2* t, float2* V, int64_t vstride, int j,
                            const double* scl, double2* part) {
  hipLaunchKernelGGL(k_spmm_arn<NC>, grid, dim3(256), 0, s, cells, B, rowptr, col, val, order, t, V, vstride, j, scl,
                     part);
}

hipError_t launch_arnoldi_product(const ArnoldiArgs& a, const float2* t, float2* kv_scratch, hipStream_t s) {
  if (a.j < 0 || a.j + 1 >= ARN_NV + 1 || a.j >= a.m || a.B < 1 || a.nch < 1 || a.vstride < a.cells * a.nch * a.B)
    return hipErrorInvalidValue;
  const int64_t rows = a.cells * a.nch;
  if (a.B >= 16 && a.nch <= 4) {
    ProfScope ps("spmm_arnoldi", s);
    const dim3 grid = arn_grid(a.cells, a.B, a.nblk);
    switch (a.nch) {
      case 1: spmm_arn_launch<1>(grid, s, a.cells, a.B, a.rowptr, a.col, a.val, a.order, t, a.V, a.vstride, a.j, a.scl, a.part); break;
      case 2: spmm_arn_launch<2>(grid, s, a.cells, a.B, a.rowptr, a.col, a.val, a.order, t, a.V, a.vstride, a.j, a.scl, a.part); break;
      case 3: spmm_arn_launch<3>(grid, s, a.cells, a.B, a.rowptr, a.col, a.val, a.order, t, a.V, a.vstride, a.j, a.scl, a.part); break;
      default: spmm_arn_launch<4>(grid, s, a.cells, a.B, a.rowptr, a.col, a.val, a.order, t, a.V, a.vstride, a.j, a.scl, a.part); break;
    }
    const int nb = (int)grid.x;
    hipLaunchKernelGGL(k_arn_finish, dim3(((a.j + 1) * a.B + 3) / 4), dim3(256), 0, s, nb, a.B, a.j + 1, a.part, a.scl,
                       a.H + (size_t)a.j * (a.m + 1) * a.B, nullptr, 0);
  } else {
    if (!kv_scratch) return hipErrorInvalidValue;
    {
      ProfScope ps("spmv_f32", s);
      hipError_t e = launch_spmv_f32(a.cells, a.nch, a.B, a.rowptr, a.col, a.val, t, kv_scratch, s, 0, -1, a.order, a.pk);
      if (e != hipSuccess) return e;
    }
    ProfScope ps("arnoldi_dots", s);
    const dim3 grid = arn_grid(rows, a.B, a.nblk);
    if (a.m <= 8)
      hipLaunchKernelGGL(k_sub_dots<8>, grid, dim3(256), 0, s, rows, a.B, kv_scratch, a.V, a.vstride, a.j, a.scl, a.part);
    else
      hipLaunchKernelGGL(k_sub_dots<ARN_NV>, grid, dim3(256), 0, s, rows, a.B, kv_scratch, a.V, a.vstride, a.j, a.scl,
                         a.part);
    hipLaunchKernelGGL(k_arn_finish, dim3(((a.j + 1) * a.B + 3) / 4), dim3(256), 0, s, (int)grid.x, a.B, a.j + 1,
                       a.part, a.scl, a.H + (size_t)a.j * (a.m + 1) * a.B, nullptr, 0);
  }
  return hipGetLastError();
}

hipError_t launch_arnoldi_orth(const ArnoldiArgs& a, hipStream_t s) {
  if (a.j < 0 || a.j + 1 > ARN_NV || a.j + 1 > a.m) return hipErrorInvalidValue;
  const int64_t rows = a.cells * a.nch;
  const dim3 grid = arn_grid(rows, a.B, a.nblk);
  const double2* hcol = a.H + (size_t)a.j * (a.m + 1) * a.B;
  if (a.m <= 8)
    hipLaunchKernelGGL(k_orth_norm<8>, grid, dim3(256), 0, s, rows, a.B, a.V, a.vstride, a.j, hcol, a.scl, a.part);
  else
    hipLaunchKernelGGL(k_orth_norm<ARN_NV>, grid, dim3(256), 0, s, rows, a.B, a.V, a.vstride, a.j, hcol, a.scl, a.part);
  hipLaunchKernelGGL(k_arn_finish, dim3((a.B + 3) / 4), dim3(256), 0, s, (int)grid.x, a.B, 1, a.part, a.scl,
                     a.H + ((size_t)a.j * (a.m + 1) + a.j + 1) * a.B, a.scl + (size_t)(a.j + 1) * a.B, 1);
  return hipGetLastError();
}

// U[c][f] = e0^T O y at (g = finals[f], j = j0[c], k = 0): one wavefront per (c, f), lanes over i.
__global__ void __launch_bounds__(256) k_capture64(int M, int nch, int B, int nfin, const double* __restrict__ O,
                                                   const int* __restrict__ wave, const int* __restrict__ j0,
                                                   const int* __restrict__ finals, const double2* __restrict__ y,
                                                   double2* __restrict__ out) {
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (t >= B * nfin) return;
  const int c = t / nfin, f = t - c * nfin;
  const int g = finals[f];
  const double* o = O + (size_t)wave[g] * M * M;   // row k = 0
  double sr = 0.0, si = 0.0;
  for (int i = lane; i < M; i += 64) {
    const double2 v = y[(((size_t)j0[c] * M + i) * nch + g) * B + c];
    sr += o[i] * v.x;
    si += o[i] * v.y;
  }
  sr = wsum64(sr);
  si = wsum64(si);
  if (lane == 0) out[t] = make_double2(sr, si);
}

// Breakup projections (one wavefront per cell): out[t] = sum_i O[wave(g)][k][i] y[((j M + i) nch + g) B + c]
// for cell t = (c, g, k, j), the pair pseudostate k of channel g at spectator bin j.
__global__ void __launch_bounds__(256) k_project_cells(int M, int nch, int B, const double* __restrict__ O,
                                                       const int* __restrict__ wave, const int4* __restrict__ cells,
                                                       int n, const double2* __restrict__ y,
                                                       double2* __restrict__ out) {
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (t >= n) return;
  const int4 cl = cells[t];
  const int c = cl.x, g = cl.y, k = cl.z, j = cl.w;
  const double* o = O + ((size_t)wave[g] * M + k) * M;
  double sr = 0.0, si = 0.0;
  for (int i = lane; i < M; i += 64) {
    const double2 v = y[(((size_t)j * M + i) * nch + g) * B + c];
    sr += o[i] * v.x;
    si += o[i] * v.y;
  }
  sr = wsum64(sr);
  si = wsum64(si);
  if (lane == 0) out[t] = make_double2(sr, si);
}

hipError_t launch_project_cells(int M, int nch, int B, const double* O, const int* wave, const int4* cells, int n,
                                const double2* y, double2* out, hipStream_t s) {
  if (M < 1 || B < 1 || n < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_project_cells, dim3((n + 3) / 4), dim3(256), 0, s, M, nch, B, O, wave, cells, n, y, out);
  return hipGetLastError();
}

hipError_t launch_capture64(int M, int nch, int B, int nfin, const double* O, const int* wave, const int* j0,
                            const int* finals, const double2* y, double2* out, hipStream_t s) {
  if (M < 1 || B < 1 || nfin < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_capture64, dim3((B * nfin + 3) / 4), dim3(256), 0, s, M, nch, B, nfin, O, wave, j0, finals, y,
                     out);
  return hipGetLastError();
}

// FP64 residual -> squared norms per column (FP64)
__global__ void __launch_bounds__(256) k_norm2_f64(int64_t rows, int B, const double2* __restrict__ x,
                                                   double2* __restrict__ part) {
  const int wv = threadIdx.x >> 6;
  const ArnLanes ln = arn_lanes(B);
  double acc[4], dummy[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = dummy[q] = 0.0;
  const int64_t step = (int64_t)gridDim.x * 4 * ln.R;
  if (ln.live)
    for (int64_t d = ((int64_t)blockIdx.x * 4 + wv) * ln.R + ln.rsub; d < rows; d += step) {
      const double2 v = x[(size_t)d * B + ln.c];
      acc[0] += v.x * v.x + v.y * v.y;
    }
  arn_block_reduce(acc, dummy, 1, ln, B, part);
}

hipError_t launch_norm2_f64(int64_t rows, int B, const double2* x, double2* part, int nblk, double2* out, hipStream_t s) {
  const dim3 grid = arn_grid(rows, B, nblk);
  hipLaunchKernelGGL(k_norm2_f64, grid, dim3(256), 0, s, rows, B, x, part);
  hipLaunchKernelGGL(k_arn_finish, dim3((B + 3) / 4), dim3(256), 0, s, (int)grid.x, B, 1, part, nullptr, out, nullptr, 0);
  return hipGetLastError();
}

// out[d][c] = x[d][c] / sqrt(nrm2[c]) with x in FP64, out in FP32
__global__ void k_scale_d2f(int64_t n, int B, const double2* __restrict__ nrm2, const double2* __restrict__ x,
                            float2* __restrict__ out, double* __restrict__ scl0) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int c = (int)(t % B);
  if (scl0 && t < B) scl0[t] = 1.0;
  const double nr = sqrt(fmax(nrm2[c].x, 0.0));
  const double inv = nr > 1e-300 ? 1.0 / nr : 0.0;
  out[t] = make_float2((float)(x[t].x * inv), (float)(x[t].y * inv));
}

hipError_t launch_scale_d2f(int64_t rows, int B, const double2* nrm2, const double2* x, float2* out, double* scl0,
                            hipStream_t s) {
  const int64_t n = rows * B;
  hipLaunchKernelGGL(k_scale_d2f, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, B, nrm2, x, out, scl0);
  return hipGetLastError();
}

}  // namespace wpcd
