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

#include "s2w_internal.h"

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

// exp(-2 pi i k / L) for 0 <= k < L/2, L a power of two <= TWN (from the constant table)
__device__ __forceinline__ float2 twiddle(int k, int L) { return c_tw[k * (TWN / L)]; }

// Per-workgroup twiddle tables in LDS for transforms of M complex points (real length L = 2M):
//   tw.c[k] = exp(-2 pi i k / M), k < M    (complex FFT, full circle)
//   tw.r[k] = exp(-2 pi i k / L), k < M    (real-FFT pre/post step)
struct Twiddles {
  float2* c;
  float2* r;
};

// Fill the tables (2*M float2 of LDS at `buf`); all threads call it; ends with a barrier.
__device__ __forceinline__ Twiddles lds_twiddles(float2* buf, int M) {
  Twiddles t{buf, buf + M};
  const int half = M >> 1;
  for (int k = threadIdx.x; k < M; k += blockDim.x) {
    float2 w = c_tw[(k < half ? k : k - half) * (TWN / M)];
    if (k >= half) w = make_float2(-w.x, -w.y);  // exp(-2 pi i (k - M/2)/M) * exp(-pi i)
    t.c[k] = w;
    t.r[k] = c_tw[k * (TWN / (2 * M))];
  }
  __syncthreads();
  return t;
}

__device__ __forceinline__ float2 cmul_dir(float2 a, float2 w, int dir) {
  // a * w (dir < 0) or a * conj(w) (dir > 0)
  return dir < 0 ? cmul(a, w) : cmul(a, cconj(w));
}

// Complex FFT of R rows of length M (power of two, 2 <= M <= TWN/2) held row-major in LDS
// buffer `a`; `b` is scratch of the same size.  dir < 0: exp(-2 pi i nk/M) (forward);
// dir > 0: exp(+2 pi i nk/M) (inverse, unnormalised).  Stockham autosort: radix-4 stages,
// then one radix-2 stage when log2(M) is odd.  Every thread of the block must call it;
// returns the buffer holding the result, after a barrier.
__device__ __forceinline__ float2* lds_cfft(float2* a, float2* b, int R, int M, int logM, int dir, const float2* tw) {
  int s = 1, lgs = 0;
  while (s * 4 <= M) {
    const int l = M / (4 * s);
    const int quarter = M >> 2;
    const int total = R * quarter;
    for (int i = threadIdx.x; i < total; i += blockDim.x) {
      const int r = i >> (logM - 2);
      const int bi = i & (quarter - 1);
      const int p = bi >> lgs, q = bi & (s - 1);
      const float2* ar = a + r * M + q + s * p;
      const float2 x0 = ar[0], x1 = ar[s * l], x2 = ar[2 * s * l], x3 = ar[3 * s * l];
      const float2 a0 = cadd(x0, x2), a1 = csub(x0, x2), a2 = cadd(x1, x3);
      const float2 d = csub(x1, x3);
      // (x1 - x3) * exp(dir * i pi / 2): forward multiplies by -i, inverse by +i
      const float2 a3 = dir < 0 ? make_float2(d.y, -d.x) : make_float2(-d.y, d.x);
      const int e = p * s;
      float2* br = b + r * M + q + s * 4 * p;
      br[0] = cadd(a0, a2);
      br[s] = cmul_dir(cadd(a1, a3), tw[e], dir);
      br[2 * s] = cmul_dir(csub(a0, a2), tw[2 * e], dir);
      br[3 * s] = cmul_dir(csub(a1, a3), tw[3 * e], dir);
    }
    __syncthreads();
    float2* t = a;
    a = b;
    b = t;
    s <<= 2;
    lgs += 2;
  }
  if (s < M) {
    const int half = M >> 1;
    const int total = R * half;
    for (int i = threadIdx.x; i < total; i += blockDim.x) {
      const int r = i >> (logM - 1);
      const int bi = i & (half - 1);
      const int p = bi >> lgs, q = bi & (s - 1);
      const float2* ar = a + r * M;
      const float2 x0 = ar[q + s * p];
      const float2 x1 = ar[q + s * (p + 1)];
      float2* br = b + r * M;
      br[q + 2 * s * p] = cadd(x0, x1);
      br[q + 2 * s * p + s] = cmul_dir(csub(x0, x1), tw[p * s], dir);
    }
    __syncthreads();
    float2* t = a;
    a = b;
    b = t;
  }
  return a;
}

// Pre-step of the inverse real FFT: packed spectrum X (M slots, real length L = 2M)
// -> Z with z = IFFT_M(Z) giving L*x[2n] + i L*x[2n+1].  tr = Twiddles::r.
// w: the twiddle tr[k] (unused for k = 0)
__device__ __forceinline__ float2 irfft_pre_w(const float2* X, int k, int M, float2 w) {
  if (k == 0) {
    const float2 x0 = X[0];
    return make_float2(x0.x + x0.y, x0.x - x0.y);
  }
  const float2 xk = X[k];
  const float2 xc = cconj(X[M - k]);
  const float2 e = cadd(xk, xc);
  const float2 o = cmul(csub(xk, xc), cconj(w));
  return make_float2(e.x - o.y, e.y + o.x);  // e + i o
}
__device__ __forceinline__ float2 irfft_pre(const float2* X, int k, int M, const float2* tr) {
  if (k == 0) return irfft_pre_w(X, 0, M, make_float2(1.f, 0.f));
  return irfft_pre_w(X, k, M, tr[k]);
}

// Post-step of the forward real FFT: Z = FFT_M(x[2n] + i x[2n+1]) -> packed slot k.
__device__ __forceinline__ float2 rfft_post_w(const float2* Z, int k, int M, float2 w) {
  if (k == 0) {
    const float2 z0 = Z[0];
    return make_float2(z0.x + z0.y, z0.x - z0.y);
  }
  const float2 zk = Z[k];
  const float2 zc = cconj(Z[M - k]);
  const float2 e = cscale(cadd(zk, zc), 0.5f);
  const float2 d = csub(zk, zc);
  const float2 o = make_float2(0.5f * d.y, -0.5f * d.x);  // d / (2i)
  return cadd(e, cmul(w, o));
}
__device__ __forceinline__ float2 rfft_post(const float2* Z, int k, int M, const float2* tr) {
  if (k == 0) return rfft_post_w(Z, 0, M, make_float2(1.f, 0.f));
  return rfft_post_w(Z, k, M, tr[k]);
}

// Real time sample m (0 <= m < L) from the inverse-FFT output z (pairs).
__device__ __forceinline__ float zsample(const float2* z, int m) {
  const float2 p = z[m >> 1];
  return (m & 1) ? p.y : p.x;
}

// Difference modes of the mid-chain round trip.
enum MidMode { MID_NONE = 0, MID_BACKWARD = 1, MID_BACKWARD_T = 2 };

// Output column of time step n, or -1 when n is not selected.
__device__ __forceinline__ int disp_col(const DispOut& d, int n) {
  if (d.all) return n;
  const int w = n >> 5;
  int col = 0;
  uint32_t word = 0;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    if (i < w) col += __popc(d.bits[i]);
    if (i == w) word = d.bits[i];
  }
  const uint32_t bit = 1u << (n & 31);
  return (word & bit) ? col + __popc(word & (bit - 1u)) : -1;
}

// Output column of every step n < nt into an LDS table (-1: not selected); all threads of the
// workgroup call it before the first capture, and a barrier follows before the table is read.
__device__ __forceinline__ void disp_fill_cols(const DispOut& d, int nt, short* tab) {
  for (int n = threadIdx.x; n < nt; n += blockDim.x) tab[n] = (short)disp_col(d, n);
}

// Where the transform rows of one tile or unit go: row r at base + r * row_stride, r < rows.
struct DispRows {
  float* base;
  int64_t row_stride;
  int rows;
  float scale;
};

// Capture sample n of transform row r (unnormalised value lval) through the column table.
__device__ __forceinline__ void disp_put(const DispRows* d, const short* tab, int r, int n, float lval) {
  if (d && r < d->rows) {
    const int c = tab[n];
    if (c >= 0) d->base[(int64_t)r * d->row_stride + c] = lval * d->scale;
  }
}

// Mid-chain round trip for R rows (Alg. 2 steps 4-5 of the first product, D_t, and
// steps 1-2 of the second): packed spectra in `X` [R][M] (LDS) -> inverse real FFT ->
// keep samples n < nt -> temporal difference -> zero-pad -> forward real FFT -> packed
// spectra.  `scale` multiplies the time series (it carries 1/L of the inverse transform
// and 1/dt of D_t).  `Y` is [R][M] LDS scratch.  Returns the buffer (X or Y) holding the
// result.  All threads of the block call it; it ends after a barrier.
__device__ __forceinline__ float2* lds_midchain2(float2* X, float2* Y, int R, int M, int logM, int nt, int mode,
                                                 float scale, const Twiddles& tw, const DispRows* disp = nullptr,
                                                 const short* dtab = nullptr) {
  const int n = R * M;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int r = i >> logM, k = i & (M - 1);
    Y[i] = irfft_pre(X + r * M, k, M, tw.r);
  }
  __syncthreads();
  float2* z = lds_cfft(Y, X, R, M, logM, +1, tw.c);
  float2* zz = (z == Y) ? X : Y;
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
        disp_put(disp, dtab, r, m, xm);
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
  float2* Z = lds_cfft(zz, z, R, M, logM, -1, tw.c);
  float2* V = (Z == X) ? Y : X;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int r = i >> logM, k = i & (M - 1);
    V[i] = rfft_post(Z + r * M, k, M, tw.r);
  }
  __syncthreads();
  return V;
}

// Three-buffer form: result written to V (may alias U); bufA, bufB scratch.
__device__ __forceinline__ void lds_midchain(const float2* U, float2* V, float2* bufA, float2* bufB, int R, int M,
                                             int logM, int nt, int mode, float scale, const Twiddles& tw) {
  const int n = R * M;
  for (int i = threadIdx.x; i < n; i += blockDim.x) bufA[i] = U[i];
  __syncthreads();
  float2* res = lds_midchain2(bufA, bufB, R, M, logM, nt, mode, scale, tw);
  for (int i = threadIdx.x; i < n; i += blockDim.x) V[i] = res[i];
  __syncthreads();
}


// ---------------------------------------------------------------------------------------------
// 256-point transforms in registers (the paper's L = 512: 256 packed slots), four-step form
// 256 = 16 x 16: index n = 16 n1 + n2, k = k1 + 16 k2,
//   X[k1 + 16 k2] = sum_{n2} W16^{n2 k2} W256^{n2 k1} sum_{n1} x[16 n1 + n2] W16^{n1 k1}.
// A thread owns one n2 (pass A) or one k1 (pass B) and holds 16 values.

// exp(-2 pi i m / 16), m < 16
__device__ __forceinline__ float2 w16(int m) {
  constexpr float C[16] = {1.0f,                  0.92387953251128674f,  0.70710678118654752f,  0.38268343236508977f,
                           0.0f,                 -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
                           -1.0f,                -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f,
                           0.0f,                  0.38268343236508977f,  0.70710678118654752f,  0.92387953251128674f};
  return make_float2(C[m & 15], -C[(m + 12) & 15]);  // (cos, -sin)
}

// in-register radix-4 DFT of (x0, x1, x2, x3); DIR < 0 forward, DIR > 0 inverse
template <int DIR>
__device__ __forceinline__ void dft4(float2& x0, float2& x1, float2& x2, float2& x3) {
  const float2 a0 = cadd(x0, x2), a1 = csub(x0, x2), a2 = cadd(x1, x3);
  const float2 d = csub(x1, x3);
  const float2 a3 = DIR < 0 ? make_float2(d.y, -d.x) : make_float2(-d.y, d.x);
  x0 = cadd(a0, a2);
  x1 = cadd(a1, a3);
  x2 = csub(a0, a2);
  x3 = csub(a1, a3);
}

// in-register 16-point DFT, natural order in and out (v[k] = sum_n v[n] W16^{DIR nk})
template <int DIR>
__device__ __forceinline__ void dft16(float2 (&v)[16]) {
  // n = 4 m1 + m2: DFT over m1 for each m2
#pragma unroll
  for (int m2 = 0; m2 < 4; ++m2) dft4<DIR>(v[m2], v[4 + m2], v[8 + m2], v[12 + m2]);
  // now v[4 k1 + m2] holds stage-1 output (k1, m2); twiddle W16^{m2 k1}
#pragma unroll
  for (int k1 = 1; k1 < 4; ++k1)
#pragma unroll
    for (int m2 = 1; m2 < 4; ++m2) {
      float2 w = w16(m2 * k1);
      if (DIR > 0) w.y = -w.y;
      v[4 * k1 + m2] = cmul(v[4 * k1 + m2], w);
    }
  // DFT over m2 for each k1: output index k1 + 4 k2
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) dft4<DIR>(v[4 * k1 + 0], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
  // v[4 k1 + k2] holds X[k1 + 4 k2]: transpose the 4 x 4 index to natural order
  float2 t[16];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) t[k1 + 4 * k2] = v[4 * k1 + k2];
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = t[i];
}

// Pass A of a 256-point transform for column n2 = c: v[n1] = x[16 n1 + c] in, out
// v[k1] = W256^{DIR c k1} * sum_{n1} x[16 n1 + c] W16^{DIR n1 k1}.
// The twiddles W256^{-c k1}, k1 = 1..15, are the thread's own (twA, in registers).
template <int DIR>
__device__ __forceinline__ void fft256_passA(float2 (&v)[16], const float2 (&twA)[15]) {
  dft16<DIR>(v);
#pragma unroll
  for (int k1 = 1; k1 < 16; ++k1) {
    float2 w = twA[k1 - 1];
    if (DIR > 0) w.y = -w.y;
    v[k1] = cmul(v[k1], w);
  }
}

// Pass-A twiddles of column c: twc[c * k1] for k1 = 1..15 (forward sign).
__device__ __forceinline__ void passA_twiddles(const float2* twc, int c, float2 (&twA)[15]) {
#pragma unroll
  for (int k1 = 1; k1 < 16; ++k1) twA[k1 - 1] = twc[c * k1];
}

// Real-transform twiddles of column c: twr[c + 16 j], j = 0..15.
__device__ __forceinline__ void real_twiddles(const float2* twr, int c, float2 (&twR)[16]) {
#pragma unroll
  for (int j = 0; j < 16; ++j) twR[j] = twr[c + 16 * j];
}

// Mid-chain round trip for R rows with M = 256, 16 threads per row (twA: passA_twiddles of
// column tid % 16): thread tid handles row
// r = tid / 16 and column c = tid % 16.  X (row stride ldx >= 256) holds the packed input
// spectra and is overwritten; T (LDS, at least R*16*17 values) receives the packed output
// spectra with row stride ldt (256 <= ldt <= 272).
// Same arithmetic as lds_midchain2 (inverse real FFT, truncate to nt, D_t, zero-pad, forward
// real FFT), with the complex transforms done as two 16-point passes in registers.  MODE is the
// MidMode, fixed at compile time so that the time step has no branches.  M = 256 means
// nt <= 256, so the packed series z[n] = x[2n] + i x[2n+1] is kept only for n < 128: the inverse
// transform's pass B writes only those outputs, and the forward transform's pass A takes zeros
// for n >= 128 (products with them are not formed).
template <int MODE>
__device__ __forceinline__ void mid256(float2* X, float2* T, int R, int nt, float scale, const Twiddles& tw,
                                       const float2 (&twA)[15], const float2 (&twR)[16], int ldx = 256,
                                       int ldt = 256, const DispRows* disp = nullptr, const short* dtab = nullptr) {
  constexpr int M = 256;
  const int tid = threadIdx.x;
  const int r = tid >> 4, c = tid & 15;
  const bool act = r < R;
  float2* Xr = X + r * ldx;
  float2* Tr = T + r * (16 * 17);
  float2 v[16];
  // inverse real FFT: pre-step fused into pass A (element 16 n1 + c)
  if (act) {
#pragma unroll
    for (int n1 = 0; n1 < 16; ++n1) v[n1] = irfft_pre_w(Xr, 16 * n1 + c, M, twR[n1]);
    fft256_passA<+1>(v, twA);
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) Tr[k1 * 17 + c] = v[k1];
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int n2 = 0; n2 < 16; ++n2) v[n2] = Tr[c * 17 + n2];
    dft16<+1>(v);
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2) Xr[c + 16 * k2] = v[k2];  // z[n] = L (x[2n] + i x[2n+1]), n < 128
  }
  __syncthreads();
  // time step (truncate, D_t, scale) fused into pass A of the forward FFT
  if (act) {
#pragma unroll
    for (int n1 = 0; n1 < 16; ++n1) {
      if (n1 >= 8) {  // n >= 128: samples 2n >= 256 >= nt are truncated
        v[n1] = make_float2(0.f, 0.f);
        continue;
      }
      const int n = 16 * n1 + c;
      const float2 z = Xr[n];
      const int m0 = 2 * n, m1 = m0 + 1;
      if (m0 < nt) disp_put(disp, dtab, r, m0, z.x);
      if (m1 < nt) disp_put(disp, dtab, r, m1, z.y);
      float a = 0.f, b = 0.f;
      // neighbours are read unconditionally (clamped index) and selected, so no lane branches
      if constexpr (MODE == MID_BACKWARD) {
        const float2 zp = Xr[n > 0 ? n - 1 : 0];
        const float xm1 = n > 0 ? zp.y : 0.f;
        a = m0 < nt ? z.x - xm1 : 0.f;
        b = m1 < nt ? z.y - z.x : 0.f;
      } else if constexpr (MODE == MID_BACKWARD_T) {
        const float2 zn = Xr[n + 1 < M ? n + 1 : M - 1];
        const float xp2 = (n + 1 < M && m1 + 1 < nt) ? zn.x : 0.f;
        a = m0 < nt ? z.x - (m1 < nt ? z.y : 0.f) : 0.f;
        b = m1 < nt ? z.y - xp2 : 0.f;
      } else {
        a = m0 < nt ? z.x : 0.f;
        b = m1 < nt ? z.y : 0.f;
      }
      v[n1] = make_float2(a * scale, b * scale);
    }
    fft256_passA<-1>(v, twA);
  }
  __syncthreads();  // all reads of X done before pass B below overwrites it
  if (act) {
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) Tr[k1 * 17 + c] = v[k1];
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int n2 = 0; n2 < 16; ++n2) v[n2] = Tr[c * 17 + n2];
    dft16<-1>(v);
#pragma unroll
    for (int k2 = 0; k2 < 16; ++k2) Xr[c + 16 * k2] = v[k2];
  }
  __syncthreads();
  // post-step of the forward real FFT, written row-major to T
  if (act) {
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int k = c + 16 * j;
      T[r * ldt + k] = rfft_post_w(Xr, k, M, twR[j]);
    }
  }
  __syncthreads();
}

// Sum over the lanes of groups of `width` consecutive lanes (width a power of two <= 64).
__device__ __forceinline__ float group_sum(float v, int width) {
  for (int m = width >> 1; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

}  // namespace s2w
