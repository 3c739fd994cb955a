// Device-side building blocks shared by the transform and contraction kernels:
// complex arithmetic, the twiddle table, a workgroup-wide Stockham FFT in LDS,
// the packed real-FFT pre/post steps and the mid-chain round trip.
//
// Spectra of real length-L series are stored packed: slot 0 holds
// (Re X_0, Re X_{L/2}) -- both bins are real -- and slot k (1 <= k < L/2)
// holds X_k.  Forward transforms are unnormalised; inverse transforms carry
// the 1/L factor (folded into one multiply with the other scale factors).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace s2w {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int TWN = 1024;  // largest transform length L supported
// c_tw[k] = exp(-2 pi i k / TWN), k < TWN/2; rounded from double precision on the host.
extern __constant__ float2 c_tw[TWN / 2];

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// exp(-2 pi i k / L) for 0 <= k < L/2, L a power of two <= TWN
__device__ __forceinline__ float2 twiddle(int k, int L) { return c_tw[k * (TWN / L)]; }

// Complex FFT of R rows of length M (power of two, 2 <= M <= TWN/2) held row-major in LDS
// buffer `a`; `b` is scratch of the same size.  dir < 0: exp(-2 pi i nk/M) (forward);
// dir > 0: exp(+2 pi i nk/M) (inverse, unnormalised).  Stockham autosort, radix 2.
// Every thread of the block must call it; returns the buffer holding the result,
// after a barrier.
__device__ __forceinline__ float2* lds_cfft(float2* a, float2* b, int R, int M, int logM, int dir) {
  const int half = M >> 1;
  const int total = R * half;
  for (int st = 0; st < logM; ++st) {
    const int s = 1 << st;
    const int l = half >> st;
    for (int i = threadIdx.x; i < total; i += blockDim.x) {
      const int r = i >> (logM - 1);
      const int bi = i & (half - 1);
      const int p = bi >> st;
      const int q = bi & (s - 1);
      const float2* ar = a + r * M;
      const float2 x0 = ar[q + s * p];
      const float2 x1 = ar[q + s * (p + l)];
      float2 w = twiddle(p * s, M);
      if (dir > 0) w.y = -w.y;
      float2* br = b + r * M;
      br[q + 2 * s * p] = cadd(x0, x1);
      br[q + 2 * s * p + s] = cmul(csub(x0, x1), w);
    }
    __syncthreads();
    float2* t = a;
    a = b;
    b = t;
  }
  return a;
}

// Pre-step of the inverse real FFT: packed spectrum X (M slots, real length L = 2M)
// -> Z with z = IFFT_M(Z) giving L*x[2n] + i L*x[2n+1].
__device__ __forceinline__ float2 irfft_pre(const float2* X, int k, int M) {
  if (k == 0) {
    const float2 x0 = X[0];
    return make_float2(x0.x + x0.y, x0.x - x0.y);
  }
  const float2 xk = X[k];
  const float2 xc = cconj(X[M - k]);
  const float2 e = cadd(xk, xc);
  const float2 o = cmul(csub(xk, xc), cconj(twiddle(k, 2 * M)));
  return make_float2(e.x - o.y, e.y + o.x);  // e + i o
}

// Post-step of the forward real FFT: Z = FFT_M(x[2n] + i x[2n+1]) -> packed slot k.
__device__ __forceinline__ float2 rfft_post(const float2* Z, int k, int M) {
  if (k == 0) {
    const float2 z0 = Z[0];
    return make_float2(z0.x + z0.y, z0.x - z0.y);
  }
  const float2 zk = Z[k];
  const float2 zc = cconj(Z[M - k]);
  const float2 e = cscale(cadd(zk, zc), 0.5f);
  const float2 d = csub(zk, zc);
  const float2 o = make_float2(0.5f * d.y, -0.5f * d.x);  // d / (2i)
  return cadd(e, cmul(twiddle(k, 2 * M), o));
}

// Real time sample m (0 <= m < L) from the inverse-FFT output z (pairs).
__device__ __forceinline__ float zsample(const float2* z, int m) {
  const float2 p = z[m >> 1];
  return (m & 1) ? p.y : p.x;
}

// Difference modes of the mid-chain round trip.
enum MidMode { MID_NONE = 0, MID_BACKWARD = 1, MID_BACKWARD_T = 2 };

// Mid-chain round trip for R rows (Alg. 2 steps 4-5 of the first product, D_t, and
// steps 1-2 of the second): packed spectra `U` [R][M] (LDS) -> inverse real FFT ->
// keep samples n < nt -> temporal difference -> zero-pad -> forward real FFT ->
// packed spectra written to `V` [R][M] (LDS, may alias U).  `scale` multiplies the
// time series (it carries 1/L of the inverse transform and 1/dt of D_t).
// bufA and bufB are [R][M] scratch.  All threads of the block call it.
__device__ __forceinline__ void lds_midchain(const float2* U, float2* V, float2* bufA, float2* bufB, int R, int M,
                                             int logM, int nt, int mode, float scale) {
  const int n = R * M;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int r = i >> logM, k = i & (M - 1);
    bufA[i] = irfft_pre(U + r * M, k, M);
  }
  __syncthreads();
  float2* z = lds_cfft(bufA, bufB, R, M, logM, +1);
  float2* zz = (z == bufA) ? bufB : bufA;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int r = i >> logM, p = i & (M - 1);
    const float2* zr = z + r * M;
    float v[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int m = 2 * p + c;
      float val = 0.f;
      if (m < nt) {
        const float xm = zsample(zr, m);
        if (mode == MID_BACKWARD) {
          val = xm - (m > 0 ? zsample(zr, m - 1) : 0.f);
        } else if (mode == MID_BACKWARD_T) {
          val = xm - (m + 1 < nt ? zsample(zr, m + 1) : 0.f);
        } else {
          val = xm;
        }
      }
      v[c] = val * scale;
    }
    zz[i] = make_float2(v[0], v[1]);
  }
  __syncthreads();
  float2* Z = lds_cfft(zz, z, R, M, logM, -1);
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int r = i >> logM, k = i & (M - 1);
    V[i] = rfft_post(Z + r * M, k, M);
  }
  __syncthreads();
}

// Sum over the lanes of groups of `width` consecutive lanes (width a power of two <= 64).
__device__ __forceinline__ float group_sum(float v, int width) {
  for (int m = width >> 1; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

}  // namespace s2w
