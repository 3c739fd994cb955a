// Per-bin complex matrix-vector products of one BLTT operator for a few inputs (Alg. 2 step 3
// when the batch is too small to feed the matrix cores): the product streams the operator
// store once, so it is bound by HBM bandwidth.
//   yh[b][r][l] = sum_c K[r][l][c] x[b][l][c]      (slot 0: componentwise, the packed real bins)
// K is the store Fs[r][l][c] (complex64, c padded to an even ncp with zeros), x the transformed
// inputs [b][l][c] with the same padding.  One wavefront per (r, l), lanes over c two complex
// values at a time (16-byte loads), a butterfly sum across the wavefront at the end.  When the
// inputs of one slot fit in 64 KB of LDS, a workgroup keeps them there and streams the rows of
// that slot; otherwise the inputs are read through L2.
#include <algorithm>

#include "s2w_internal.h"

namespace s2w {

typedef float gv_f4 __attribute__((ext_vector_type(4)));

// re + i im += k (x) x over two complex values; slot 0 multiplies componentwise
__device__ __forceinline__ void gv_mac(const float4& k, const float4& x, bool dc, float& re, float& im) {
  if (dc) {
    re += k.x * x.x + k.z * x.z;
    im += k.y * x.y + k.w * x.w;
  } else {
    re += k.x * x.x - k.y * x.y + k.z * x.z - k.w * x.w;
    im += k.x * x.y + k.y * x.x + k.z * x.w + k.w * x.z;
  }
}

// butterfly sum over the wavefront, lane 0 writes yh[b][r][l]
template <int NB>
__device__ __forceinline__ void gv_store(float (&re)[NB], float (&im)[NB], int lane, int B, float2* yh, int nrow,
                                         int r, int M, int l) {
#pragma unroll
  for (int b = 0; b < NB; ++b) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
      re[b] += __shfl_xor(re[b], m, 64);
      im[b] += __shfl_xor(im[b], m, 64);
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int b = 0; b < NB; ++b)
      if (b < B) yh[((int64_t)b * nrow + r) * M + l] = make_float2(re[b], im[b]);
  }
}

// One wavefront per (r, l) (tasks in store order), the inputs read through L2.
template <int NB>
__global__ __launch_bounds__(256) void k_bltt_gemv(const float4* __restrict__ K, const float4* __restrict__ X,
                                                   float2* __restrict__ yh, int nrow, int M, int nc4, int B) {
  const int lane = threadIdx.x & 63;
  const int64_t tasks = (int64_t)nrow * M;
  const int64_t nwave = (int64_t)gridDim.x * 4;
  for (int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); t < tasks; t += nwave) {
    const int r = (int)(t / M), l = (int)(t - (int64_t)r * M);
    const bool dc = (l == 0);
    const float4* a = K + t * nc4;
    float re[NB], im[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) re[b] = im[b] = 0.f;
#pragma unroll 4
    for (int i = lane; i < nc4; i += 64) {
      const gv_f4 kv = __builtin_nontemporal_load(reinterpret_cast<const gv_f4*>(a + i));  // streamed once
      const float4 k = make_float4(kv.x, kv.y, kv.z, kv.w);
#pragma unroll
      for (int b = 0; b < NB; ++b)
        if (b < B) gv_mac(k, X[((int64_t)b * M + l) * nc4 + i], dc, re[b], im[b]);
    }
    gv_store<NB>(re, im, lane, B, yh, nrow, r, M, l);
  }
}

// Workgroup per (slot l, range of rows): the inputs of slot l sit in LDS, and each wavefront
// streams whole store rows (r, l) of its range, one at a time.
template <int NB>
__global__ __launch_bounds__(256) void k_bltt_gemv_lds(const float4* __restrict__ K, const float4* __restrict__ X,
                                                       float2* __restrict__ yh, int nrow, int M, int nc4, int B,
                                                       int nsplit) {
  extern __shared__ float4 xs[];  // [b][i], b < B, i < nc4
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l = blockIdx.x % M, split = blockIdx.x / M;
  const bool dc = (l == 0);
  for (int j = threadIdx.x; j < B * nc4; j += 256) {
    const int b = j / nc4, i = j - b * nc4;
    xs[j] = X[((int64_t)b * M + l) * nc4 + i];
  }
  __syncthreads();
  const int r0 = (int)((int64_t)nrow * split / nsplit), r1 = (int)((int64_t)nrow * (split + 1) / nsplit);
  for (int r = r0 + wave; r < r1; r += 4) {
    const float4* a = K + ((int64_t)r * M + l) * nc4;
    float re[NB], im[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) re[b] = im[b] = 0.f;
#pragma unroll 4
    for (int i = lane; i < nc4; i += 64) {
      const gv_f4 kv = __builtin_nontemporal_load(reinterpret_cast<const gv_f4*>(a + i));  // streamed once
      const float4 k = make_float4(kv.x, kv.y, kv.z, kv.w);
#pragma unroll
      for (int b = 0; b < NB; ++b)
        if (b < B) gv_mac(k, xs[b * nc4 + i], dc, re[b], im[b]);
    }
    gv_store<NB>(re, im, lane, B, yh, nrow, r, M, l);
  }
}

// As k_bltt_gemv_lds for rows of at most 512 float4 (ncol <= 1024): the row's loads
// (8 x 64 x 16 bytes) are issued together, and the next row's go out before the current row is
// reduced, so that a wavefront always has a row in flight.
template <int NB>
__global__ __launch_bounds__(256) void k_bltt_gemv_row(const float4* __restrict__ K, const float4* __restrict__ X,
                                                       float2* __restrict__ yh, int nrow, int M, int nc4, int B,
                                                       int nsplit) {
  constexpr int NI = 8;           // float4 per lane and row: nc4 <= 512
  extern __shared__ float4 xs[];  // [b][i], b < B, i < nc4
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l = blockIdx.x % M, split = blockIdx.x / M;
  const bool dc = (l == 0);
  for (int j = threadIdx.x; j < B * nc4; j += 256) {
    const int b = j / nc4, i = j - b * nc4;
    xs[j] = X[((int64_t)b * M + l) * nc4 + i];
  }
  __syncthreads();
  const int r0 = (int)((int64_t)nrow * split / nsplit), r1 = (int)((int64_t)nrow * (split + 1) / nsplit);
  auto load_row = [&](int r, float4 (&kv)[NI]) {
    const float4* a = K + ((int64_t)r * M + l) * nc4;
#pragma unroll
    for (int t = 0; t < NI; ++t) {
      const int i = lane + 64 * t;
      if (i < nc4) {
        const gv_f4 v = __builtin_nontemporal_load(reinterpret_cast<const gv_f4*>(a + i));  // streamed once
        kv[t] = make_float4(v.x, v.y, v.z, v.w);
      } else {
        kv[t] = make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
  };
  float4 cur[NI], nxt[NI];
  int r = r0 + wave;
  if (r < r1) load_row(r, cur);
  for (; r < r1; r += 4) {
    if (r + 4 < r1) load_row(r + 4, nxt);
    float re[NB], im[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) re[b] = im[b] = 0.f;
#pragma unroll
    for (int t = 0; t < NI; ++t) {
      const int i = lane + 64 * t;
      if (i < nc4) {
#pragma unroll
        for (int b = 0; b < NB; ++b)
          if (b < B) gv_mac(cur[t], xs[b * nc4 + i], dc, re[b], im[b]);
      }
    }
    gv_store<NB>(re, im, lane, B, yh, nrow, r, M, l);
#pragma unroll
    for (int t = 0; t < NI; ++t) cur[t] = nxt[t];
  }
}

hipError_t launch_bltt_gemv(const float2* K, const float2* X, float2* yh, int nrow, int M, int ncp, int B, int ncu,
                            hipStream_t st) {
  if (B < 1 || B > 4 || (ncp & 1) || nrow < 1 || M < 1) return hipErrorInvalidValue;
  const int nc4 = ncp / 2;
  const float4* k4 = reinterpret_cast<const float4*>(K);
  const float4* x4 = reinterpret_cast<const float4*>(X);
  const size_t lds = (size_t)B * nc4 * sizeof(float4);
  if (lds <= 64 * 1024) {
    // inputs of a slot in LDS; enough row ranges per slot for about 16 workgroups per CU
    const int nsplit = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)ncu * 16 / M, (nrow + 3) / 4));
    const dim3 grid((unsigned)((int64_t)M * nsplit));
#define S2W_GV2(K_, NB_) hipLaunchKernelGGL((K_<NB_>), grid, dim3(256), lds, st, k4, x4, yh, nrow, M, nc4, B, nsplit)
    if (nc4 <= 512) {  // rows of at most 8 float4 per lane: whole rows in flight
      if (B == 1) S2W_GV2(k_bltt_gemv_row, 1); else if (B == 2) S2W_GV2(k_bltt_gemv_row, 2); else S2W_GV2(k_bltt_gemv_row, 4);
    } else {
      if (B == 1) S2W_GV2(k_bltt_gemv_lds, 1); else if (B == 2) S2W_GV2(k_bltt_gemv_lds, 2); else S2W_GV2(k_bltt_gemv_lds, 4);
    }
#undef S2W_GV2
    return hipGetLastError();
  }
  const int64_t tasks = (int64_t)nrow * M;
  const int64_t blocks = std::min<int64_t>((tasks + 3) / 4, (int64_t)ncu * 16);
  const dim3 grid((unsigned)blocks);
  if (B == 1)
    hipLaunchKernelGGL((k_bltt_gemv<1>), grid, dim3(256), 0, st, k4, x4, yh, nrow, M, nc4, B);
  else if (B == 2)
    hipLaunchKernelGGL((k_bltt_gemv<2>), grid, dim3(256), 0, st, k4, x4, yh, nrow, M, nc4, B);
  else
    hipLaunchKernelGGL((k_bltt_gemv<4>), grid, dim3(256), 0, st, k4, x4, yh, nrow, M, nc4, B);
  return hipGetLastError();
}

}  // namespace s2w
