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

}  // namespace wpcd
