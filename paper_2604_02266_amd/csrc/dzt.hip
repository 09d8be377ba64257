// Discrete Zak transform of received time-domain frames (Sec. III-A, Eq. zak) and its
// inverse (Eq. iZak), computed as the batched complex GEMM of Sec. IV-A (Eq. zak_gemm) on
// the matrix cores of gfx950.
//
// For a frame of M delay x N Doppler bins, the time-domain samples y[i M + k] (slot i,
// delay k) form an N x M matrix In[i][k] in memory order, and the DD frame in vector order
// q = l M + k is the N x M matrix Out[l][k] = sum_i F[l][i] In[i][k] with the unitary kernel
// F[l][i] = e^{-j 2 pi l i / N} / sqrt(N) (Eq. zak as written; the printed kernel matrix of
// Eq. zak_exp differs from it by the factor sqrt(N) (-1)^l, and the transform is kept
// unitary so that DD noise equals time-domain noise).  The inverse takes conj(F)^T, i.e.
// the same product with the opposite twiddle sign.  This is a dense contraction, so it
// runs on MFMA: FP32 inputs (v_mfma_f32_16x16x4_f32), complex products as four real
// products, FP32 accumulation.
//
// One wave computes a 16 x 64 block of Out (four 16 x 16 tiles side by side in k): per step
// of 4 slots i, the A operand F[l][i] comes from a twiddle table in LDS (index l i mod N,
// exact), the B operand In[i][k] straight from memory (one complex per lane per tile), and
// 16 MFMAs (4 tiles x 4 real products) accumulate.  A workgroup is 4 waves covering 16 x 256
// of one frame.  Rows l >= N and columns k >= M are computed on zero-padded operands and not
// stored; slots i >= N contribute zero.
#include <hip/hip_runtime.h>

#include <math.h>

#include "otfs_internal.h"

namespace otfs {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kDztThreads = 256;                 // 4 waves
constexpr int kDztRows = 16;                     // l per workgroup
constexpr int kDztCols = 256;                    // k per workgroup (64 per wave)

__global__ __launch_bounds__(kDztThreads) void k_dzt(int M, int N, int nframes, float sign,
                                                     const float2* __restrict__ in,
                                                     float2* __restrict__ out) {
  extern __shared__ float2 tw[];                 // tw[m] = e^{sign j 2 pi m / N} / sqrt(N)
  const int nlb = (N + kDztRows - 1) / kDztRows;
  const int nkb = (M + kDztCols - 1) / kDztCols;
  const int64_t b = blockIdx.x;
  const int f = (int)(b / ((int64_t)nlb * nkb));
  const int rem = (int)(b - (int64_t)f * nlb * nkb);
  const int l0 = (rem / nkb) * kDztRows;
  const int kb0 = (rem % nkb) * kDztCols;
  if (f >= nframes) return;
  const double scale = 1.0 / sqrt((double)N);
  for (int m = threadIdx.x; m < N; m += kDztThreads) {
    double s, c;
    sincospi(2.0 * (double)m / (double)N, &s, &c);
    tw[m] = make_float2((float)(c * scale), (float)(sign * s * scale));
  }
  __syncthreads();
  const int64_t E = (int64_t)M * N;
  const float2* src = in + (int64_t)f * E;
  float2* dst = out + (int64_t)f * E;
  const int lane = (int)threadIdx.x & 63;
  const int wave = (int)threadIdx.x >> 6;
  const int k0 = kb0 + wave * 64;                // this wave's 64 columns
  const int am = lane & 15, ak = lane >> 4;      // A[m][kk], B[kk][n]: lane = m + 16 kk
  const int la = l0 + am;                        // row of this lane's A element
  f32x4 re[4], im[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    re[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    im[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  // twiddle index (la * i) mod N for i = i0 + ak, advanced by 4 la per step
  const int64_t lan = la < N ? la : 0;
  int64_t idx = (lan * ak) % N;
  const int64_t step = (4 * lan) % N;
  for (int i0 = 0; i0 < N; i0 += 4) {
    const int i = i0 + ak;
    float2 a = make_float2(0.f, 0.f);
    if (la < N && i < N) a = tw[idx];
    idx += step;
    if (idx >= N) idx -= N;
    float2 v[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int k = k0 + t * 16 + am;
      v[t] = (i < N && k < M) ? src[(int64_t)i * M + k] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      // (a.x + j a.y)(v.x + j v.y): re += a.x v.x - a.y v.y, im += a.x v.y + a.y v.x
      re[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, v[t].x, re[t], 0, 0, 0);
      re[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(-a.y, v[t].y, re[t], 0, 0, 0);
      im[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, v[t].y, im[t], 0, 0, 0);
      im[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, v[t].x, im[t], 0, 0, 0);
    }
  }
  // D[m][n]: lane holds rows 4 (lane / 16) + r, r = 0..3, column lane % 16
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int k = k0 + t * 16 + am;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int l = l0 + 4 * ak + r;
      if (l < N && k < M) dst[(int64_t)l * M + k] = make_float2(re[t][r], im[t][r]);
    }
  }
}

}  // namespace

hipError_t launch_dzt(int M, int N, int nframes, bool inverse, const float2* in, float2* out,
                      hipStream_t s) {
  if (nframes <= 0) return hipSuccess;
  const int64_t nb = (int64_t)((N + kDztRows - 1) / kDztRows) * ((M + kDztCols - 1) / kDztCols) *
                     nframes;
  if (nb > 0x7fffffff) return hipErrorInvalidValue;
  if (N > kDztMaxN) return hipErrorInvalidValue;
  const size_t lds = (size_t)N * sizeof(float2);
  hipLaunchKernelGGL(k_dzt, dim3((unsigned)nb), dim3(kDztThreads), lds, s, M, N, nframes,
                     inverse ? 1.f : -1.f, in, out);
  return hipGetLastError();
}

}  // namespace otfs
