// Mixed-precision kernels of the iteration (FP32 vectors, BF16 blocks on MFMA with FP32
// accumulation) and the FP64 helpers of the residual refinement.
#include <hip/hip_runtime.h>

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

// One channel g (pair wave w) and 8 complex columns (16 real columns: re/im of each):
//   t = O y on MFMA 16x16x16 bf16 (y rounded to bf16), capture e0^T O y (FP32), t *= G1 (FP32),
//   s = (v O^T) t on MFMA (t rounded to bf16), s written in FP32.
// MFMA 16x16x16 bf16 operands: lane l holds A[l%16][4(l/16)+0..3], B[4(l/16)+0..3][l%16];
// the result D[4(l/16)+r][l%16], r = 0..3.
__global__ void __launch_bounds__(256) k_step_bf16(RotArgsMixed r, const uint16_t* __restrict__ Wb,
                                                   const float2* __restrict__ y, float2* __restrict__ s_out) {
  extern __shared__ uint16_t shb[];
  const int M = r.M, Mp = r.Mp, B = r.B, nch = r.nch;
  const int ncol = r.N * B;
  const int g = blockIdx.y;
  const size_t woff = (size_t)r.wave[g] * Mp * Mp;
  const uint16_t* O = r.A + woff;
  const uint16_t* W = Wb + woff;
  const int col0 = blockIdx.x * 8;
  uint16_t* YT = shb;             // [16][Mp], real column rc = 2 cc + part
  uint16_t* TT = shb + 16 * Mp;   // [16][Mp]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int e = tid; e < 8 * Mp; e += 256) {
    int cc, i;
    if (B >= 8) {   // consecutive threads -> consecutive energies c
      i = e >> 3;
      cc = e & 7;
    } else {        // consecutive threads -> consecutive p bins i
      cc = e / Mp;
      i = e - cc * Mp;
    }
    const int col = col0 + cc;
    float2 v = make_float2(0.f, 0.f);
    if (i < M && col < ncol) {
      const int jj = col / B, cb = col - jj * B;
      v = y[(((size_t)jj * M + i) * nch + g) * B + cb];
    }
    YT[(2 * cc) * Mp + i] = f2bf(v.x);
    YT[(2 * cc + 1) * Mp + i] = f2bf(v.y);
  }
  __syncthreads();
  const int rc = lane & 15, quad = lane >> 4;
  const int cc = rc >> 1, part = rc & 1;
  const int col = col0 + cc;
  const bool live = col < ncol;
  const int jj = live ? col / B : 0, cb = live ? col - jj * B : 0;
  const int nt = Mp / 16;
  for (int kt = wv; kt < nt; kt += 4) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int it = 0; it < nt; ++it) {
      const bf16x4 a = *reinterpret_cast<const bf16x4*>(O + (size_t)(kt * 16 + rc) * Mp + it * 16 + 4 * quad);
      const bf16x4 b = *reinterpret_cast<const bf16x4*>(YT + rc * Mp + it * 16 + 4 * quad);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = kt * 16 + 4 * quad + q;
      const float val = acc[q];
      const float other = __shfl_xor(val, 1, 64);
      const float re = part ? other : val, im = part ? val : other;
      float out = 0.f;
      if (live && k < M) {
        if (r.acap && k == 0 && part == 0 && jj == r.j0[cb]) {
          for (int f = 0; f < r.nfin; ++f)
            if (r.finals[f] == g) r.acap[r.acap_off + (int64_t)cb * r.nfin + f] = make_float2(re, im);
        }
        const float2 gv = r.G[(((size_t)jj * M + k) * nch + g) * B + cb];
        out = part ? (re * gv.y + im * gv.x) : (re * gv.x - im * gv.y);
      }
      TT[rc * Mp + k] = f2bf(out);
    }
  }
  __syncthreads();
  for (int itl = wv; itl < nt; itl += 4) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int kt = 0; kt < nt; ++kt) {
      const bf16x4 a = *reinterpret_cast<const bf16x4*>(W + (size_t)(itl * 16 + rc) * Mp + kt * 16 + 4 * quad);
      const bf16x4 b = *reinterpret_cast<const bf16x4*>(TT + rc * Mp + kt * 16 + 4 * quad);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
    if (live) {
      float* so = reinterpret_cast<float*>(s_out);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = itl * 16 + 4 * quad + q;
        if (i < M) so[2 * ((((size_t)jj * M + i) * nch + g) * B + cb) + part] = acc[q];
      }
    }
  }
}

hipError_t launch_step_bf16(const RotArgsMixed& r, const uint16_t* W, const float2* y, float2* s_out, hipStream_t s) {
  if (r.M < 1 || r.Mp < r.M || r.Mp % 16 || r.N < 1 || r.B < 1 || r.nch < 1 || !r.G) return hipErrorInvalidValue;
  const size_t shmem = (size_t)2 * 16 * r.Mp * sizeof(uint16_t);
  if (shmem > 64 * 1024) return hipErrorInvalidValue;
  dim3 grid((r.N * r.B + 7) / 8, r.nch);
  hipLaunchKernelGGL(k_step_bf16, grid, dim3(256), shmem, s, r, W, y, s_out);
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

// ------------------------------------------------------------------ Arnoldi helpers (per column c)
// Vectors are [rows][B] float2 (rows = D lattice entries); a basis is nv such vectors, vstride apart.

#define MD_MAXV 48

// part[blk][i][c] = sum over this block's rows of conj(V_i[d][c]) x[d][c], FP64 accumulation.
// Lanes over columns c, waves over rows; x[d][c] is loaded once per chunk of up to 8 basis
// vectors whose partial sums stay in registers; one LDS reduction over the waves per chunk.
__global__ void __launch_bounds__(256) k_mdot(int64_t rows, int B, int nv, const float2* __restrict__ V, int64_t vstride,
                                              const float2* __restrict__ x, int64_t rows_per_blk,
                                              double2* __restrict__ part) {
  __shared__ double2 red[4][8][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
  const int64_t r1 = min(rows, r0 + rows_per_blk);
  for (int cb = 0; cb < B; cb += 64) {
    const int c = cb + lane;
    for (int i0 = 0; i0 < nv; i0 += 8) {
      const int ni = min(8, nv - i0);
      double sr[8], si[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) sr[q] = si[q] = 0.0;
      if (c < B) {
        for (int64_t d = r0 + wv; d < r1; d += 4) {
          const float2 w = x[d * B + c];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            if (q < ni) {
              const float2 v = V[(size_t)(i0 + q) * vstride + d * B + c];
              sr[q] += (double)v.x * w.x + (double)v.y * w.y;
              si[q] += (double)v.x * w.y - (double)v.y * w.x;
            }
          }
        }
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) red[wv][q][lane] = make_double2(sr[q], si[q]);
      __syncthreads();
      // 8 x 64 results per chunk: thread t reduces entry (q = t / 64 ... ) over the 4 waves
      for (int e = threadIdx.x; e < 8 * 64; e += 256) {
        const int q = e >> 6, l = e & 63;
        const int cc = cb + l;
        if (q < ni && cc < B) {
          double2 t = red[0][q][l];
          for (int w4 = 1; w4 < 4; ++w4) {
            t.x += red[w4][q][l].x;
            t.y += red[w4][q][l].y;
          }
          part[((size_t)blockIdx.x * nv + i0 + q) * B + cc] = t;
        }
      }
      __syncthreads();
    }
  }
}

// out[i][c] (+)= sum_blk part[blk][i][c]: one wavefront per output, lanes over the blocks in a
// fixed order, then a shuffle reduction (the result does not depend on scheduling).
__device__ __forceinline__ double wsum64(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ void __launch_bounds__(256) k_mdot_finish(int nblk, int B, int nv, const double2* __restrict__ part,
                                                     double2* __restrict__ out, int accumulate) {
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
    if (accumulate) {
      out[t].x += sr;
      out[t].y += si;
    } else {
      out[t] = make_double2(sr, si);
    }
  }
}

hipError_t launch_mdot(int64_t rows, int B, int nv, const float2* V, int64_t vstride, const float2* x, double2* part,
                       int nblk, double2* out, int accumulate, hipStream_t s) {
  if (nv < 1 || nv > MD_MAXV || B < 1 || nblk < 1) return hipErrorInvalidValue;
  const int64_t rpb = (rows + nblk - 1) / nblk;
  hipLaunchKernelGGL(k_mdot, dim3(nblk), dim3(256), 0, s, rows, B, nv, V, vstride, x, rpb, part);
  hipLaunchKernelGGL(k_mdot_finish, dim3((nv * B + 3) / 4), dim3(256), 0, s, nblk, B, nv, part, out, accumulate);
  return hipGetLastError();
}

// x[d][c] -= sum_i h[i][c] V_i[d][c]   (FP64 arithmetic, FP32 storage)
__global__ void k_orth_update(int64_t n, int B, int nv, const float2* __restrict__ V, int64_t vstride,
                              const double2* __restrict__ h, float2* __restrict__ x) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int c = (int)(t % B);
  double xr = x[t].x, xi = x[t].y;
  for (int i = 0; i < nv; ++i) {
    const double2 hc = h[(size_t)i * B + c];
    const float2 v = V[(size_t)i * vstride + t];
    xr -= hc.x * v.x - hc.y * v.y;
    xi -= hc.x * v.y + hc.y * v.x;
  }
  x[t] = make_float2((float)xr, (float)xi);
}

hipError_t launch_orth_update(int64_t rows, int B, int nv, const float2* V, int64_t vstride, const double2* h, float2* x,
                              hipStream_t s) {
  const int64_t n = rows * B;
  hipLaunchKernelGGL(k_orth_update, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, B, nv, V, vstride, h, x);
  return hipGetLastError();
}

// out[d][c] = x[d][c] / sqrt(nrm[c]) (nrm = squared norm from k_mdot, real part); zero if tiny.
// Also stores the norm into hsub[c] (the subdiagonal entry of the Hessenberg matrix).
__global__ void k_normalize(int64_t n, int B, const double2* __restrict__ nrm2, const float2* __restrict__ x,
                            float2* __restrict__ out, double2* __restrict__ hsub) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int c = (int)(t % B);
  const double nr = sqrt(fmax(nrm2[c].x, 0.0));
  const double inv = nr > 1e-300 ? 1.0 / nr : 0.0;
  out[t] = make_float2((float)(x[t].x * inv), (float)(x[t].y * inv));
  if (t < B) hsub[t] = make_double2(sqrt(fmax(nrm2[t].x, 0.0)), 0.0);
}

hipError_t launch_normalize(int64_t rows, int B, const double2* nrm2, const float2* x, float2* out, double2* hsub,
                            hipStream_t s) {
  const int64_t n = rows * B;
  hipLaunchKernelGGL(k_normalize, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, B, nrm2, x, out, hsub);
  return hipGetLastError();
}

// w = v - kv (FP32): applies (I - K) given K v
__global__ void k_sub_f32(int64_t n, const float2* __restrict__ v, const float2* __restrict__ kv, float2* __restrict__ w) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) w[t] = make_float2(v[t].x - kv[t].x, v[t].y - kv[t].y);
}

hipError_t launch_sub_f32(int64_t n, const float2* v, const float2* kv, float2* w, hipStream_t s) {
  hipLaunchKernelGGL(k_sub_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, v, kv, w);
  return hipGetLastError();
}

// FP64 residual -> squared norms per column (FP64)
__global__ void __launch_bounds__(256) k_norm2_f64(int64_t rows, int B, const double2* __restrict__ x, int64_t rows_per_blk,
                                                   double2* __restrict__ part) {
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
  const int64_t r1 = min(rows, r0 + rows_per_blk);
  for (int cb = 0; cb < B; cb += 64) {
    const int c = cb + lane;
    double s2 = 0.0;
    if (c < B)
      for (int64_t d = r0 + wv; d < r1; d += 4) {
        const double2 v = x[d * B + c];
        s2 += v.x * v.x + v.y * v.y;
      }
    red[wv][lane] = s2;
    __syncthreads();
    if (wv == 0 && c < B) part[(size_t)blockIdx.x * B + c] = make_double2(red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane], 0.0);
    __syncthreads();
  }
}

hipError_t launch_norm2_f64(int64_t rows, int B, const double2* x, double2* part, int nblk, double2* out, hipStream_t s) {
  const int64_t rpb = (rows + nblk - 1) / nblk;
  hipLaunchKernelGGL(k_norm2_f64, dim3(nblk), dim3(256), 0, s, rows, B, x, rpb, part);
  hipLaunchKernelGGL(k_mdot_finish, dim3((B + 3) / 4), dim3(256), 0, s, nblk, B, 1, part, out, 0);
  return hipGetLastError();
}

// out[d][c] = x[d][c] / sqrt(nrm2[c]) with x in FP64, out in FP32
__global__ void k_scale_d2f(int64_t n, int B, const double2* __restrict__ nrm2, const double2* __restrict__ x,
                            float2* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int c = (int)(t % B);
  const double nr = sqrt(fmax(nrm2[c].x, 0.0));
  const double inv = nr > 1e-300 ? 1.0 / nr : 0.0;
  out[t] = make_float2((float)(x[t].x * inv), (float)(x[t].y * inv));
}

hipError_t launch_scale_d2f(int64_t rows, int B, const double2* nrm2, const double2* x, float2* out, hipStream_t s) {
  const int64_t n = rows * B;
  hipLaunchKernelGGL(k_scale_d2f, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, B, nrm2, x, out);
  return hipGetLastError();
}

}  // namespace wpcd
