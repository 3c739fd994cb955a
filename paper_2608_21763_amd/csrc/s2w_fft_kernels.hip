// Transform kernels and the single-rupture contraction kernels.
//
// Stores (see s2w_api.cpp for sizes):
//   Gh[g][j][l]  elastic spectra, complex64, j padded to nsp (zero rows), l < M = L/2 packed slots
//   Fh[g][o][l]  acoustic-gravity spectra, complex64, o padded to nop (zero rows)
// Both are the temporal FFTs of the zero-padded response blocks (Alg. 2; Sec. II-C:
// computed once at setup and resident between calls).  Grid row g is contiguous, so a
// chunk of rows is one contiguous range, and each (g, column) spectrum is one contiguous
// run of M complex values.
#include <math.h>

#include <algorithm>

#include "s2w_device.h"
#include "s2w_internal.h"

namespace s2w {

__constant__ float2 c_tw[TWN / 2];

hipError_t upload_twiddles(int device) {
  (void)device;
  static float2 h[TWN / 2];
  for (int k = 0; k < TWN / 2; ++k) {
    const double a = -2.0 * M_PI * (double)k / (double)TWN;
    h[k] = make_float2((float)cos(a), (float)sin(a));
  }
  return hipMemcpyToSymbol(HIP_SYMBOL(c_tw), h, sizeof(h), 0, hipMemcpyHostToDevice);
}

static inline int rows_per_block(int M) { return M >= 4096 ? 1 : 4096 / M; }

// ---------------------------------------------------------------------------------------------
// Real rows -> packed spectra (zero-padded forward real FFT of length L = 2M, Alg. 2 steps 1-2).
__global__ __launch_bounds__(256) void k_rfft_rows(const float* __restrict__ in, int64_t nrows, int ninner,
                                                   int ninner_pad, float2* __restrict__ out, int64_t out_outer,
                                                   int64_t out_inner, int64_t out_slot, int nt, int M, int logM,
                                                   int R, float scale) {
  extern __shared__ float2 smem[];
  float2* A = smem;
  float2* Bf = smem + R * M;
  const Twiddles tw = lds_twiddles(smem + 2 * R * M, M);
  const int64_t row0 = (int64_t)blockIdx.x * R;
  for (int i = threadIdx.x; i < R * M; i += blockDim.x) {
    const int r = i >> logM, p = i & (M - 1);
    const int64_t row = row0 + r;
    float2 v = make_float2(0.f, 0.f);
    if (row < nrows) {
      const int64_t o = row / ninner_pad;
      const int inn = (int)(row - o * ninner_pad);
      if (inn < ninner) {
        const float* x = in + (o * ninner + inn) * (int64_t)nt;
        const int m0 = 2 * p, m1 = 2 * p + 1;
        v.x = m0 < nt ? x[m0] * scale : 0.f;
        v.y = m1 < nt ? x[m1] * scale : 0.f;
      }
    }
    A[i] = v;
  }
  __syncthreads();
  float2* Z = lds_cfft(A, Bf, R, M, logM, -1, tw.c);
  for (int i = threadIdx.x; i < R * M; i += blockDim.x) {
    const int r = i % R, k = i / R;
    const int64_t row = row0 + r;
    if (row < nrows) {
      const int64_t o = row / ninner_pad;
      const int inn = (int)(row - o * ninner_pad);
      out[o * out_outer + inn * out_inner + k * out_slot] = rfft_post(Z + r * M, k, M, tw.r);
    }
  }
}

hipError_t launch_rfft_rows(const float* in, int64_t nouter, int ninner, int ninner_pad, float2* out,
                            int64_t out_outer, int64_t out_inner, int64_t out_slot, const Geometry& g, float scale,
                            hipStream_t st) {
  const int R = rows_per_block(g.M);
  const int64_t nrows = nouter * ninner_pad;
  if (nrows == 0) return hipSuccess;
  const int64_t nblk = (nrows + R - 1) / R;
  hipLaunchKernelGGL(k_rfft_rows, dim3((unsigned)nblk), dim3(256), (2 * R + 2) * g.M * sizeof(float2), st, in, nrows,
                     ninner, ninner_pad, out, out_outer, out_inner, out_slot, g.nt, g.M, g.logM, R, scale);
  return hipGetLastError();
}

// Packed spectra -> real rows (inverse real FFT, Alg. 2 steps 4-5: keep n < nt).
__global__ __launch_bounds__(256) void k_irfft_rows(const float2* __restrict__ in, int64_t nrows, int64_t in_row,
                                                    int64_t in_slot, float* __restrict__ out, int64_t out_row,
                                                    int nt, int M, int logM, int R, float scale) {
  extern __shared__ float2 smem[];
  float2* X = smem;
  float2* A = smem + R * M;
  float2* Bf = smem + 2 * R * M;
  const Twiddles tw = lds_twiddles(smem + 3 * R * M, M);
  const int64_t row0 = (int64_t)blockIdx.x * R;
  for (int i = threadIdx.x; i < R * M; i += blockDim.x) {
    const int r = i % R, k = i / R;
    const int64_t row = row0 + r;
    X[r * M + k] = row < nrows ? in[row * in_row + k * in_slot] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < R * M; i += blockDim.x) {
    const int r = i >> logM, k = i & (M - 1);
    A[i] = irfft_pre(X + r * M, k, M, tw.r);
  }
  __syncthreads();
  float2* z = lds_cfft(A, Bf, R, M, logM, +1, tw.c);
  for (int i = threadIdx.x; i < R * nt; i += blockDim.x) {
    const int r = i / nt, m = i - r * nt;
    const int64_t row = row0 + r;
    if (row < nrows) out[row * out_row + m] = zsample(z + r * M, m) * scale;
  }
}

hipError_t launch_irfft_rows(const float2* in, int64_t nrows, int64_t in_row, int64_t in_slot, float* out,
                             int64_t out_row, const Geometry& g, float scale, hipStream_t st) {
  if (nrows == 0) return hipSuccess;
  const int R = rows_per_block(g.M);
  const int64_t nblk = (nrows + R - 1) / R;
  hipLaunchKernelGGL(k_irfft_rows, dim3((unsigned)nblk), dim3(256), (3 * R + 2) * g.M * sizeof(float2), st, in, nrows,
                     in_row, in_slot, out, out_row, g.nt, g.M, g.logM, R, scale);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Contractions over the stored column index c (subfault j or observer o).
//
// Layout of a store X[g][c][l]: for each grid row g and column c the M packed slots are
// contiguous, so a thread that owns the slot pair (2p, 2p+1) reads one float4 per (g, c)
// and a wavefront reads whole 1 KB runs.  Threads: NP = M/2 slot pairs x CG = 256/NP
// column groups; group cg handles columns c = cg, cg + CG, ...  No lane reductions are
// needed; the CG group partial sums meet once per tile in LDS.
//
// Complex product of a stored value x with a coefficient pair y, per slot:
//   plain:  x * y              conj:  conj(x) * y
// written as  out.re += x.re*c1 + x.im*c2,  out.im += x.re*c3 + x.im*c4
// so that the packed real slot 0 (two real bins) multiplies componentwise:
//   (c1, c2, c3, c4) = (y.re, 0, 0, y.im).
struct Coef {
  float c1, c2, c3, c4;
};

__device__ __forceinline__ Coef make_coef(float2 y, bool dc, bool conj) {
  Coef k;
  k.c1 = y.x;
  k.c2 = dc ? 0.f : (conj ? y.y : -y.y);
  k.c3 = dc ? 0.f : y.y;
  k.c4 = dc ? y.y : (conj ? -y.x : y.x);
  return k;
}

__device__ __forceinline__ void cmac2(v4f& acc, const v4f x, const Coef& a, const Coef& b) {
  acc.x += x.x * a.c1 + x.y * a.c2;
  acc.y += x.x * a.c3 + x.y * a.c4;
  acc.z += x.z * b.c1 + x.w * b.c2;
  acc.w += x.z * b.c3 + x.w * b.c4;
}

// D[t][l] = sum_c op(X[g0+t][c][l]) * Y[c][l] for t < T (rows t >= tr give zero), all slots.
// `red` is LDS scratch of 256*T float4.  All threads call it; ends after a barrier.
template <int T, bool CONJ>
__device__ __forceinline__ void contract_cols(const v4f* __restrict__ X, const v4f* __restrict__ Y, int g0, int tr,
                                              int nc, int ncp, int M, float2* D, v4f* red) {
  const int NP = M >> 1;
  const int CG = 256 / NP;
  const int tid = threadIdx.x;
  const int p = tid % NP, cg = tid / NP;
  const bool dc = (p == 0);
  v4f acc[T];
#pragma unroll
  for (int t = 0; t < T; ++t) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
  const int64_t row_stride = (int64_t)ncp * NP;  // float4 per grid row
  // Row offsets of the tile; rows past the tile end repeat its last row so that every
  // load is unconditional (their sums land in D rows >= tr, which callers ignore).
  int64_t roff[T];
#pragma unroll
  for (int t = 0; t < T; ++t) roff[t] = (int64_t)(g0 + min(t, tr - 1)) * row_stride + p;
  // Two columns per step (c and c + CG) so that 2T + 2 independent loads are in flight; a
  // second column past the end reloads column nc - 1 with a zero coefficient.
  for (int c = cg; c < nc; c += 2 * CG) {
    const int c2 = c + CG;
    const bool has2 = c2 < nc;
    const int c2c = has2 ? c2 : nc - 1;
    const v4f ya = Y[(int64_t)c * NP + p];
    v4f yb = Y[(int64_t)c2c * NP + p];
    v4f xa[T], xb[T];
#pragma unroll
    for (int t = 0; t < T; ++t) xa[t] = __builtin_nontemporal_load(X + (int64_t)c * NP + roff[t]);
#pragma unroll
    for (int t = 0; t < T; ++t) xb[t] = __builtin_nontemporal_load(X + (int64_t)c2c * NP + roff[t]);
    if (!has2) yb = v4f{0.f, 0.f, 0.f, 0.f};
    const Coef ka = make_coef(make_float2(ya.x, ya.y), dc, CONJ);
    const Coef kb = make_coef(make_float2(ya.z, ya.w), false, CONJ);
    const Coef kc = make_coef(make_float2(yb.x, yb.y), dc, CONJ);
    const Coef kd = make_coef(make_float2(yb.z, yb.w), false, CONJ);
#pragma unroll
    for (int t = 0; t < T; ++t) {
      cmac2(acc[t], xa[t], ka, kb);
      cmac2(acc[t], xb[t], kc, kd);
    }
  }
#pragma unroll
  for (int t = 0; t < T; ++t) red[(cg * T + t) * NP + p] = acc[t];
  __syncthreads();
  for (int i = tid; i < T * NP; i += 256) {
    const int t = i / NP, pp = i - t * NP;
    v4f s = v4f{0.f, 0.f, 0.f, 0.f};
    for (int k = 0; k < CG; ++k) s += red[(k * T + t) * NP + pp];
    D[t * M + 2 * pp] = make_float2(s.x, s.y);
    D[t * M + 2 * pp + 1] = make_float2(s.z, s.w);
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------------------------
// Single-rupture fused forward.  Persistent: workgroup w owns grid rows
// [ngrid*w/nwg, ngrid*(w+1)/nwg) and walks them in tiles of T rows:
//   1. U[t][l] = sum_j Gh[g][j][l] Sh[j][l]                  (eq. 1 per bin, Alg. 2 step 3)
//   2. U -> V in LDS: inverse FFT, truncate, D_t, zero-pad, FFT   (Alg. 1 line 3; Alg. 2 steps 4-5, 1-2)
//   3. acc[o][l] += sum_t Fh[g][o][l] V[t][l]                (eq. 2 per bin, accumulated over rows)
// The seafloor field never leaves the workgroup.  The accumulator (observers o = og + OG*i
// for the thread's slot pair) is written once, as this workgroup's partial spectrum
// part[w][o][l] (o < nop).
template <int T, int OPT, bool DISP>
__global__ __launch_bounds__(256, 1) void k_fused_forward(const v4f* __restrict__ Gh, const v4f* __restrict__ Fh,
                                                          const v4f* __restrict__ Sh, v4f* __restrict__ part,
                                                          int ngrid, int nsub, int nsp, int nobs, int nop, int M,
                                                          int logM, int nt, int mode, float mscale, DispOut disp) {
  extern __shared__ float2 smem[];
  float2* U = smem;
  float2* BA = U + T * M;
  v4f* red = reinterpret_cast<v4f*>(BA + T * M);
  const Twiddles tw = lds_twiddles(reinterpret_cast<float2*>(red + 256 * T), M);
  const int tid = threadIdx.x;
  const int NP = M >> 1, OG = 256 / NP;
  float* const disp_m = disp.base;
  __shared__ short dtab[DISP ? 512 : 1];
  if (DISP) {
    disp_fill_cols(disp, nt, dtab);
    __syncthreads();
  }
  const int p = tid % NP, og = tid / NP;
  const bool dc = (p == 0);
  const int wg = blockIdx.x, nwg = gridDim.x;
  const int r0 = (int)((int64_t)ngrid * wg / nwg), r1 = (int)((int64_t)ngrid * (wg + 1) / nwg);
  v4f acc[OPT];
#pragma unroll
  for (int k = 0; k < OPT; ++k) acc[k] = v4f{0.f, 0.f, 0.f, 0.f};
  const int64_t frow = (int64_t)nop * NP;  // float4 per grid row of Fh
  for (int g0 = r0; g0 < r1; g0 += T) {
    const int tr = min(T, r1 - g0);
    contract_cols<T, false>(Gh, Sh, g0, tr, nsub, nsp, M, U, red);
    const DispRows dr{disp_m + (int64_t)g0 * disp.row_stride, disp.row_stride, tr, disp.scale};
    const float2* Vt = lds_midchain2(U, BA, T, M, logM, nt, mode, mscale, tw, DISP ? &dr : nullptr, dtab);
    const v4f* fb = Fh + (int64_t)g0 * frow + p;
    for (int t = 0; t < tr; ++t) {
      const float2 va = Vt[t * M + 2 * p], vb = Vt[t * M + 2 * p + 1];
      const Coef ka = make_coef(va, dc, false), kb = make_coef(vb, false, false);
      const v4f* ft = fb + t * frow;
      // observer rows past the store repeat its last (zero-padding or valid) row; their
      // accumulators are never written out
      v4f f[OPT];
#pragma unroll
      for (int k = 0; k < OPT; ++k) f[k] = __builtin_nontemporal_load(ft + (int64_t)min(og + OG * k, nop - 1) * NP);
#pragma unroll
      for (int k = 0; k < OPT; ++k) cmac2(acc[k], f[k], ka, kb);
    }
    __syncthreads();
  }
  v4f* pw = part + (int64_t)wg * nop * NP + p;
#pragma unroll
  for (int k = 0; k < OPT; ++k) {
    const int o = og + OG * k;
    if (o < nop) pw[(int64_t)o * NP] = acc[k];
  }
}

static inline int next_pow2(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

static inline size_t tile_lds(int T, int M) {
  return 2 * (size_t)T * M * sizeof(float2) + 256 * (size_t)T * 16 + 2 * (size_t)M * sizeof(float2);
}

int fused_forward_opt(const Geometry& g) {
  const int OG = 256 / (g.M / 2);
  return (g.nobs + OG - 1) / OG;
}

template <int T, int OPT>
static hipError_t fused_fwd_t(const float2* Gh, const float2* Fh, const float2* Sh, float2* part, int nwg,
                              const Geometry& g, hipStream_t st, const DispOut& disp) {
  const int mode = g.diff ? MID_BACKWARD : MID_NONE;
  const float mscale = (float)(1.0 / ((double)g.L * (g.diff ? (double)g.dt : 1.0)));
  if (disp.base)
    hipLaunchKernelGGL((k_fused_forward<T, OPT, true>), dim3(nwg), dim3(256), tile_lds(T, g.M), st, (const v4f*)Gh,
                       (const v4f*)Fh, (const v4f*)Sh, (v4f*)part, g.ngrid, g.nsub, g.nsp, g.nobs, g.nop, g.M, g.logM,
                       g.nt, mode, mscale, disp);
  else
    hipLaunchKernelGGL((k_fused_forward<T, OPT, false>), dim3(nwg), dim3(256), tile_lds(T, g.M), st, (const v4f*)Gh,
                       (const v4f*)Fh, (const v4f*)Sh, (v4f*)part, g.ngrid, g.nsub, g.nsp, g.nobs, g.nop, g.M, g.logM,
                       g.nt, mode, mscale, disp);
  return hipGetLastError();
}

template <int T>
static hipError_t fused_fwd_rows(const float2* Gh, const float2* Fh, const float2* Sh, float2* part, int nwg,
                                 const Geometry& g, hipStream_t st, const DispOut& disp) {
  const int need = fused_forward_opt(g);
  if (need <= 4) return fused_fwd_t<T, 4>(Gh, Fh, Sh, part, nwg, g, st, disp);
  if (need <= 8) return fused_fwd_t<T, 8>(Gh, Fh, Sh, part, nwg, g, st, disp);
  if (need <= 16) return fused_fwd_t<T, 16>(Gh, Fh, Sh, part, nwg, g, st, disp);
  if (need <= 32) return fused_fwd_t<T, 32>(Gh, Fh, Sh, part, nwg, g, st, disp);
  return hipErrorInvalidValue;
}

hipError_t launch_fused_forward(const float2* Gh, const float2* Fh, const float2* Sh, float2* part, int nwg,
                                int tile_rows, const Geometry& g, hipStream_t st, const DispOut& disp) {
  if (tile_rows == 4) return fused_fwd_rows<4>(Gh, Fh, Sh, part, nwg, g, st, disp);
  return fused_fwd_rows<8>(Gh, Fh, Sh, part, nwg, g, st, disp);
}

// ---------------------------------------------------------------------------------------------
// Fixed-order sum of partial spectra: out[i] = sum_p part[p][i] for i < items (float4 units).
// QP threads share an item: thread q sums parts p = q, q + QP, ... (eight loads in flight),
// then the QP partial sums are added in the fixed order q = 0..QP-1.  Deterministic.
constexpr int QP = 8;
__global__ __launch_bounds__(256) void k_sum_parts(const v4f* __restrict__ part, int nparts, int64_t items,
                                                   v4f* __restrict__ out) {
  __shared__ v4f sh[256];
  const int q = threadIdx.x % QP;
  const int64_t it = (int64_t)blockIdx.x * (256 / QP) + threadIdx.x / QP;
  v4f s = v4f{0.f, 0.f, 0.f, 0.f};
  if (it < items) {
    int p = q;
    for (; p + 7 * QP < nparts; p += 8 * QP) {
      v4f a[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] = part[(int64_t)(p + u * QP) * items + it];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += a[u];
    }
    for (; p < nparts; p += QP) s += part[(int64_t)p * items + it];
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  if (q == 0 && it < items) {
    v4f t = sh[threadIdx.x];
#pragma unroll
    for (int k = 1; k < QP; ++k) t += sh[threadIdx.x + k];
    out[it] = t;
  }
}

hipError_t launch_sum_parts(const float2* part, int nparts, int64_t items_c, float2* out, hipStream_t st) {
  const int64_t items = items_c / 2;
  const int64_t per_blk = 256 / QP;
  const int64_t nblk = (items + per_blk - 1) / per_blk;
  hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)nblk), dim3(256), 0, st, (const v4f*)part, nparts, items,
                     (v4f*)out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Per-row stage with a mid-chain round trip, output Out[g][l]:
//   forward (CONJ = false):  Out = mid(sum_j Gh[g][j][l] Sh[j][l]),            D_t
//   adjoint (CONJ = true):   Out = mid(sum_o conj(Fh[g][o][l]) Rh[o][l]),      D_t transposed
// Used by the single-rupture adjoint and by the unfused forward.
template <int T, bool CONJ, bool DISP = false>
__global__ __launch_bounds__(256) void k_rows_mid(const v4f* __restrict__ X, const v4f* __restrict__ Y,
                                                  float2* __restrict__ Out, int ngrid, int nc, int ncp, int M,
                                                  int logM, int nt, int mode, float mscale, DispOut disp) {
  extern __shared__ float2 smem[];
  float2* U = smem;
  float2* BA = U + T * M;
  v4f* red = reinterpret_cast<v4f*>(BA + T * M);
  const Twiddles tw = lds_twiddles(reinterpret_cast<float2*>(red + 256 * T), M);
  const int wg = blockIdx.x, nwg = gridDim.x;
  const int r0 = (int)((int64_t)ngrid * wg / nwg), r1 = (int)((int64_t)ngrid * (wg + 1) / nwg);
  float* const disp_m = disp.base;
  __shared__ short dtab[DISP ? 512 : 1];
  if (DISP) {
    disp_fill_cols(disp, nt, dtab);
    __syncthreads();
  }
  for (int g0 = r0; g0 < r1; g0 += T) {
    const int tr = min(T, r1 - g0);
    contract_cols<T, CONJ>(X, Y, g0, tr, nc, ncp, M, U, red);
    const DispRows dr{disp_m + (int64_t)g0 * disp.row_stride, disp.row_stride, tr, disp.scale};
    const float2* Vt = lds_midchain2(U, BA, T, M, logM, nt, mode, mscale, tw, DISP ? &dr : nullptr, dtab);
    for (int i = threadIdx.x; i < tr * M; i += blockDim.x) Out[(int64_t)g0 * M + i] = Vt[i];
    __syncthreads();
  }
}

hipError_t launch_adjoint_rows(const float2* Fh, const float2* Rh, float2* Wp, int nwg, int tile_rows,
                               const Geometry& g, hipStream_t st) {
  const int mode = g.diff ? MID_BACKWARD_T : MID_NONE;
  const float mscale = (float)(1.0 / ((double)g.L * (g.diff ? (double)g.dt : 1.0)));
  if (tile_rows == 4)
    hipLaunchKernelGGL((k_rows_mid<4, true>), dim3(nwg), dim3(256), tile_lds(4, g.M), st, (const v4f*)Fh,
                       (const v4f*)Rh, Wp, g.ngrid, g.nobs, g.nop, g.M, g.logM, g.nt, mode, mscale, DispOut{});
  else
    hipLaunchKernelGGL((k_rows_mid<8, true>), dim3(nwg), dim3(256), tile_lds(8, g.M), st, (const v4f*)Fh,
                       (const v4f*)Rh, Wp, g.ngrid, g.nobs, g.nop, g.M, g.logM, g.nt, mode, mscale, DispOut{});
  return hipGetLastError();
}

hipError_t launch_forward_rows(const float2* Gh, const float2* Sh, float2* Vh, int nwg, const Geometry& g,
                               hipStream_t st, const DispOut& disp) {
  const int mode = g.diff ? MID_BACKWARD : MID_NONE;
  const float mscale = (float)(1.0 / ((double)g.L * (g.diff ? (double)g.dt : 1.0)));
  if (disp.base)
    hipLaunchKernelGGL((k_rows_mid<8, false, true>), dim3(nwg), dim3(256), tile_lds(8, g.M), st, (const v4f*)Gh,
                       (const v4f*)Sh, Vh, g.ngrid, g.nsub, g.nsp, g.M, g.logM, g.nt, mode, mscale, disp);
  else
    hipLaunchKernelGGL((k_rows_mid<8, false, false>), dim3(nwg), dim3(256), tile_lds(8, g.M), st, (const v4f*)Gh,
                       (const v4f*)Sh, Vh, g.ngrid, g.nsub, g.nsp, g.M, g.logM, g.nt, mode, mscale, disp);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Contraction over grid rows, per bin, split over row ranges:
//   CONJ = true:  part[split][c][l] = sum_{g in split} conj(X[g][c][l]) W[g][l]
//                 (single-rupture adjoint, transpose of eq. 1; c = subfault)
//   CONJ = false: part[split][c][l] = sum_{g in split} X[g][c][l] W[g][l]
//                 (unfused forward, eq. 2 per bin; c = observer)
// Workgroup (column block of CB columns, split).  Thread (cs, p): slot pair p, columns
// c0 + cs + CS*i.  W[g] for the thread's slot pair is reused across its columns.
template <int CPT, bool CONJ>
__global__ __launch_bounds__(256) void k_rows_contract(const v4f* __restrict__ X, const float2* __restrict__ W,
                                                       v4f* __restrict__ part, int ngrid, int nc, int ncp, int M) {
  const int NP = M >> 1, CS = 256 / NP;
  const int tid = threadIdx.x;
  const int p = tid % NP, cs = tid / NP;
  const bool dc = (p == 0);
  const int CB = CS * CPT;
  const int c0 = blockIdx.x * CB;
  const int split = blockIdx.y, splits = gridDim.y;
  const int r0 = (int)((int64_t)ngrid * split / splits), r1 = (int)((int64_t)ngrid * (split + 1) / splits);
  v4f acc[CPT];
#pragma unroll
  for (int i = 0; i < CPT; ++i) acc[i] = v4f{0.f, 0.f, 0.f, 0.f};
  const int64_t row_stride = (int64_t)ncp * NP;
  for (int g = r0; g < r1; ++g) {
    const float2 wa = W[(int64_t)g * M + 2 * p], wb = W[(int64_t)g * M + 2 * p + 1];
    const Coef ka = make_coef(wa, dc, CONJ), kb = make_coef(wb, false, CONJ);
    const v4f* xg = X + (int64_t)g * row_stride + p;
    v4f x[CPT];
#pragma unroll
    for (int i = 0; i < CPT; ++i) x[i] = __builtin_nontemporal_load(xg + (int64_t)min(c0 + cs + CS * i, ncp - 1) * NP);
#pragma unroll
    for (int i = 0; i < CPT; ++i) cmac2(acc[i], x[i], ka, kb);
  }
  v4f* pw = part + (int64_t)split * ncp * NP + p;
#pragma unroll
  for (int i = 0; i < CPT; ++i) {
    const int c = c0 + cs + CS * i;
    if (c < ncp) pw[(int64_t)c * NP] = acc[i];  // padding columns hold zero spectra
  }
}

template <bool CONJ>
static hipError_t rows_contract_t(const float2* X, const float2* W, float2* part, int cols_per_thread, int splits,
                                  int nc, int ncp, const Geometry& g, hipStream_t st) {
  const int CS = 256 / (g.M / 2);
  const int CPT = cols_per_thread >= 16 ? 16 : 8;
  const int CB = CS * CPT;
  dim3 grid((ncp + CB - 1) / CB, splits);
  if (CPT == 16)
    hipLaunchKernelGGL((k_rows_contract<16, CONJ>), grid, dim3(256), 0, st, (const v4f*)X, W, (v4f*)part, g.ngrid, nc,
                       ncp, g.M);
  else
    hipLaunchKernelGGL((k_rows_contract<8, CONJ>), grid, dim3(256), 0, st, (const v4f*)X, W, (v4f*)part, g.ngrid, nc,
                       ncp, g.M);
  return hipGetLastError();
}

hipError_t launch_adjoint_elastic(const float2* Gh, const float2* Wp, float2* part, int cols_per_thread, int splits,
                                  const Geometry& g, hipStream_t st) {
  return rows_contract_t<true>(Gh, Wp, part, cols_per_thread, splits, g.nsub, g.nsp, g, st);
}

hipError_t launch_rows_acoustic(const float2* Fh, const float2* Vh, float2* part, int cols_per_thread, int splits,
                                const Geometry& g, hipStream_t st) {
  return rows_contract_t<false>(Fh, Vh, part, cols_per_thread, splits, g.nobs, g.nop, g, st);
}

// ---------------------------------------------------------------------------------------------
// Batched mid-chain round trip on U[g][l][b] (complex, b < bp): for grid row g and ruptures
// b0 .. b0+R-1, gather all M slots, run inverse FFT -> truncate -> D_t -> zero-pad -> FFT in
// LDS (Alg. 1 line 3; Alg. 2 steps 4-5 and 1-2), multiply by the acoustic store's scale
// sF[g][l] and write the result back in place: as complex64 (PACK = 0), or as bfloat16
// high/low terms of the real and imaginary parts packed in two 32-bit words (PACK = 1), the
// acoustic GEMM's operand format.
typedef float s2w_f2v_t __attribute__((ext_vector_type(2)));
typedef __bf16 s2w_b2v_t __attribute__((ext_vector_type(2)));

// (a, b) rounded to nearest even bfloat16 in one word, a in the low half (hardware conversion)
__device__ __forceinline__ uint32_t bf16x2_rne(float a, float b) {
  const s2w_f2v_t v = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, s2w_b2v_t));
}

template <int PACK>
__device__ __forceinline__ void store_v(float2* dst, float2 v, float f) {
  v.x *= f;
  v.y *= f;
  if (PACK) {
    const uint32_t h = bf16x2_rne(v.x, v.y);
    const uint32_t lo = bf16x2_rne(v.x - __uint_as_float(h << 16), v.y - __uint_as_float(h & 0xffff0000u));
    *reinterpret_cast<uint2*>(dst) = make_uint2(h, lo);
  } else {
    *dst = v;
  }
}

// General M: rows staged through a padded transposition buffer, generic LDS transforms.
template <int R, int PACK, bool DISP>
__global__ __launch_bounds__(256) void k_mid_batch(float2* __restrict__ U, const float* __restrict__ sF, int ngrid,
                                                   int B, int bp, int M, int logM, int nt, int mode, float mscale,
                                                   DispOut disp) {
  extern __shared__ float2 smem[];
  // two buffers of M*(R+1) values: each serves as the row-major FFT buffer [R][M] and, while
  // free, as the padded transposition buffer [M][R+1] (conflict-free in both directions)
  const int BUF = M * (R + 1);
  float2* X = smem;
  float2* Y = X + BUF;
  const Twiddles tw = lds_twiddles(Y + BUF, M);
  const int nbb = (B + R - 1) / R;
  const int64_t units = (int64_t)ngrid * nbb;
  __shared__ short dtab[DISP ? 512 : 1];
  if (DISP) {
    disp_fill_cols(disp, nt, dtab);
    __syncthreads();
  }
  for (int64_t u = blockIdx.x; u < units; u += gridDim.x) {
    const int g = (int)(u / nbb);
    const int b0 = (int)(u % nbb) * R;
    const float2* src = U + (int64_t)g * M * bp + b0;
    for (int i = threadIdx.x; i < R * M; i += blockDim.x) {
      const int l = i / R, r = i % R;
      Y[l * (R + 1) + r] = b0 + r < B ? src[(int64_t)l * bp + r] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < R * M; i += blockDim.x) {
      const int r = i >> logM, l = i & (M - 1);
      X[i] = Y[l * (R + 1) + r];
    }
    __syncthreads();
    const DispRows dr{disp.base + (int64_t)g * disp.grid_stride + (int64_t)b0 * disp.row_stride, disp.row_stride,
                      B - b0, disp.scale};
    const float2* V = lds_midchain2(X, Y, R, M, logM, nt, mode, mscale, tw, DISP ? &dr : nullptr, dtab);
    float2* Tp = (V == X) ? Y : X;
    for (int i = threadIdx.x; i < R * M; i += blockDim.x) {
      const int r = i >> logM, l = i & (M - 1);
      Tp[l * (R + 1) + r] = V[i];
    }
    __syncthreads();
    float2* dst = U + (int64_t)g * M * bp + b0;
    for (int i = threadIdx.x; i < R * M; i += blockDim.x) {
      const int l = i / R, r = i % R;
      if (b0 + r < B) store_v<PACK>(dst + (int64_t)l * bp + r, Tp[l * (R + 1) + r], sF ? sF[(int64_t)g * M + l] : 1.f);
    }
    __syncthreads();
  }
}

// M = 256: 16 ruptures of one grid row per unit, the next unit's rows prefetched into
// registers while the current one is transformed; rows kept with a padded stride (257) so
// that the strided LDS writes and reads of the gather and scatter are conflict-free.
// With cmax, the grid is a multiple of the rupture blocks per row (nbb), so a workgroup always
// works on the same block of ruptures; it keeps the largest |Re|, |Im| of every (slot, rupture)
// it writes and leaves them in cmax[blockIdx / nbb][l][b] (b < bp; zero for b >= B).
template <int PACK, int R, bool DISP, int MODE>
__global__ __launch_bounds__(16 * R) void k_mid_batch256(float2* __restrict__ U, const float* __restrict__ sF,
                                                         int ngrid, int B, int bp, int nt, float mscale,
                                                         float* __restrict__ cmax, DispOut disp) {
  constexpr int M = 256, LD = 257;
  __shared__ float2 X[R * LD];
  __shared__ float2 T[R * 16 * 17];
  __shared__ float2 twb[2 * M];
  __shared__ short dtab[DISP ? 512 : 1];
  if (DISP) disp_fill_cols(disp, nt, dtab);  // the barrier in lds_twiddles orders it
  const Twiddles tw = lds_twiddles(twb, M);
  const int tid = threadIdx.x;
  const int r = tid % R, lq = tid / R;  // gather/scatter: rupture r, slots lq + 16 k
  float2 twA[15], twR[16];
  passA_twiddles(tw.c, tid & 15, twA);
  real_twiddles(tw.r, tid & 15, twR);
  const int nbb = (B + R - 1) / R;
  const int units = ngrid * nbb;  // the launcher checks that this fits an int
  float2 pre[16];
  float fs[16];
  float cmx[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) cmx[k] = 0.f;
  // loads are unconditional (ruptures past B read rupture B - 1 and are zeroed), so that the
  // gather has no lane branches
  auto fetch = [&](int u) {
    const int g = u / nbb;
    const int b = (u % nbb) * R + r;
    const float2* src = U + (int64_t)g * M * bp + (b < B ? b : B - 1);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int l = lq + 16 * k;
      const float2 v = src[(int64_t)l * bp];
      pre[k] = b < B ? v : make_float2(0.f, 0.f);
      fs[k] = sF ? sF[(int64_t)g * M + l] : 1.f;
    }
  };
  int u = blockIdx.x;
  if (u < units) fetch(u);
  for (; u < units; u += gridDim.x) {
    const int g = u / nbb;
    const int b = (u % nbb) * R + r;
#pragma unroll
    for (int k = 0; k < 16; ++k) X[r * LD + lq + 16 * k] = pre[k];
    float f[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) f[k] = fs[k];
    __syncthreads();
    if (u + (int)gridDim.x < units) fetch(u + gridDim.x);
    const int b0 = (u % nbb) * R;
    const DispRows dr{disp.base + (int64_t)g * disp.grid_stride + (int64_t)b0 * disp.row_stride, disp.row_stride,
                      B - b0, disp.scale};
    mid256<MODE>(X, T, R, nt, mscale, tw, twA, twR, LD, LD, DISP ? &dr : nullptr, dtab);
    float2* dst = U + (int64_t)g * M * bp + b;
    if (b < B) {
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int l = lq + 16 * k;
        const float2 v = T[r * LD + l];
        store_v<PACK>(dst + (int64_t)l * bp, v, f[k]);
        if (cmax) cmx[k] = fmaxf(cmx[k], fmaxf(fabsf(v.x * f[k]), fabsf(v.y * f[k])));
      }
    }
    __syncthreads();
  }
  if (cmax) {
    const int b = (int)(blockIdx.x % nbb) * R + r;
    if (b < bp) {
      float* o = cmax + (int64_t)(blockIdx.x / nbb) * M * bp + b;
#pragma unroll
      for (int k = 0; k < 16; ++k) o[(int64_t)(lq + 16 * k) * bp] = b < B ? cmx[k] : 0.f;
    }
  }
}

// Zero-padded forward real FFT of a batch of time rows into packed spectra ordered for the
// batched products, for M = 256 (Alg. 2 steps 1-2): in[b][j][n] (b < B, j < nrows, n < nt) ->
// out[l][j][b] at l * out_slot + j * bp + b; rows nrows <= j < nrows_pad are written as zeros,
// ruptures b >= B are not written.  A unit is one row index j and 16 ruptures: each time row is
// read as 128-byte runs, transformed by the two 16-point passes of the mid-chain in registers
// (nt <= 256, so the packed series z[n] = x[2n] + i x[2n+1] is zero for n >= 128), and the
// spectra go out through LDS as 128-byte runs of 16 ruptures per slot.  Persistent grid.
__global__ __launch_bounds__(256) void k_rfft_batch256(const float* __restrict__ in, int nrows, int nrows_pad, int B,
                                                       int bp, float2* __restrict__ out, int64_t out_slot, int nt,
                                                       float scale) {
  constexpr int M = 256, R = 16, LD = 257;
  __shared__ float2 X[R * LD];
  __shared__ float2 T[R * 16 * 17];
  __shared__ float2 twb[2 * M];
  const Twiddles tw = lds_twiddles(twb, M);
  const int tid = threadIdx.x;
  const int fr = tid >> 4, c = tid & 15;  // transform: row (rupture) fr, column c
  const int r = tid % R, lq = tid / R;    // scatter: rupture r, slots lq + 16 k
  float2 twA[15], twR[16];
  passA_twiddles(tw.c, c, twA);
  real_twiddles(tw.r, c, twR);
  const int nbb = (B + R - 1) / R;
  const int units = nrows_pad * nbb;
  for (int u = blockIdx.x; u < units; u += gridDim.x) {
    const int j = u / nbb, b0 = (u % nbb) * R;
    float2 v[16];
    {
      const int b = b0 + fr;
      const bool live = b < B && j < nrows;
      const float* x = in + ((int64_t)(live ? b : 0) * nrows + (live ? j : 0)) * nt;
#pragma unroll
      for (int n1 = 0; n1 < 16; ++n1) {
        if (n1 >= 8) {  // n >= 128: samples 2n >= 256 >= nt
          v[n1] = make_float2(0.f, 0.f);
          continue;
        }
        const int m0 = 2 * (c + 16 * n1);
        float2 xv = make_float2(0.f, 0.f);
        if (!(nt & 1)) {  // even rows: the pair is one aligned 8-byte load
          if (live && m0 < nt) xv = *reinterpret_cast<const float2*>(x + m0);
        } else {
          xv.x = (live && m0 < nt) ? x[m0] : 0.f;
          xv.y = (live && m0 + 1 < nt) ? x[m0 + 1] : 0.f;
        }
        v[n1] = make_float2(xv.x * scale, xv.y * scale);
      }
    }
    float2* Xr = X + fr * LD;
    float2* Tr = T + fr * (16 * 17);
    fft256_passA<-1>(v, twA);
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) Tr[k1 * 17 + c] = v[k1];
    __syncthreads();
#pragma unroll
    for (int n2 = 0; n2 < 16; ++n2) v[n2] = Tr[c * 17 + n2];
    dft16<-1>(v);
#pragma unroll
    for (int k2 = 0; k2 < 16; ++k2) Xr[c + 16 * k2] = v[k2];
    __syncthreads();
    // post-step of the real transform, row-major into T (T is read again only after the barrier)
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {
      const int k = c + 16 * jj;
      T[fr * LD + k] = rfft_post_w(Xr, k, M, twR[jj]);
    }
    __syncthreads();
    if (b0 + r < B) {
      float2* dst = out + (int64_t)j * bp + b0 + r;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int l = lq + 16 * k;
        dst[(int64_t)l * out_slot] = T[r * LD + l];
      }
    }
    __syncthreads();  // X and T are refilled by the next unit
  }
}

hipError_t launch_rfft_batch256(const float* in, int B, int nrows, int nrows_pad, float2* out, int bp, int64_t out_slot,
                                int nt, float scale, hipStream_t st) {
  if (B == 0 || nrows_pad == 0) return hipSuccess;
  if (B < 0 || nrows < 0 || nrows_pad < nrows || bp < B || nt < 1 || nt > 256) return hipErrorInvalidValue;
  const int64_t units = (int64_t)nrows_pad * ((B + 15) / 16);
  if (units > 0x7fffffff) return hipErrorInvalidValue;
  const int64_t nblk = std::min<int64_t>(units, 256 * 8);
  hipLaunchKernelGGL(k_rfft_batch256, dim3((unsigned)nblk), dim3(256), 0, st, in, nrows, nrows_pad, B, bp, out,
                     out_slot, nt, scale);
  return hipGetLastError();
}

// Sum of the split partials of a batched product and the inverse real FFT of the result, for
// M = 256: part[s][l][o][2 bp] (complex per rupture, s < splits) -> out[b][o][n], n < nt.
// A unit is one output row o and 16 ruptures; the partials are read as 128-byte runs (16
// ruptures of one slot), summed in split order, scaled by tau_down[l][b] when given, and
// transposed through LDS; the inverse transform (Alg. 2 steps 4-5) is the two 16-point passes of
// the mid-chain, and each row's samples go out as 128-byte runs.  The launcher checks the
// sizes; the grid is persistent.
__global__ __launch_bounds__(256) void k_sum_irfft256(const float2* __restrict__ part, int splits, int noq, int nrows,
                                                      int B, int bp, const float* __restrict__ tau_down,
                                                      float* __restrict__ out, int nt, float scale) {
  constexpr int M = 256, R = 16, LD = 257;
  __shared__ float2 X[R * LD];
  __shared__ float2 T[R * 16 * 17];
  __shared__ float2 twb[2 * M];
  const Twiddles tw = lds_twiddles(twb, M);
  const int tid = threadIdx.x;
  const int r = tid % R, lq = tid / R;  // gather: rupture r of the unit, slots lq + 16 k
  const int fr = tid >> 4, c = tid & 15;  // transform: row fr, column c
  float2 twA[15], twR[16];
  passA_twiddles(tw.c, c, twA);
  real_twiddles(tw.r, c, twR);
  const int nbb = (B + R - 1) / R;
  const int units = nrows * nbb;
  const int64_t s_stride = (int64_t)M * noq * bp;  // complex values per split
  for (int u = blockIdx.x; u < units; u += gridDim.x) {
    const int o = u / nbb, b0 = (u % nbb) * R;
    {
      const int b = b0 + r;
      const int bc = b < B ? b : B - 1;  // loads unconditional, ruptures past B zeroed
      const float2* src = part + (int64_t)o * bp + bc;
#pragma unroll 4
      for (int k = 0; k < 16; ++k) {
        const int l = lq + 16 * k;
        const float2* p = src + (int64_t)l * noq * bp;
        float re = 0.f, im = 0.f;
        for (int s = 0; s < splits; ++s) {
          const float2 v = p[s * s_stride];
          re += v.x;
          im += v.y;
        }
        const float td = tau_down ? tau_down[(int64_t)l * bp + bc] : 1.f;
        X[r * LD + l] = b < B ? make_float2(re * td, im * td) : make_float2(0.f, 0.f);
      }
    }
    __syncthreads();
    float2 v[16];
    const float2* Xr = X + fr * LD;
    float2* Tr = T + fr * (16 * 17);
#pragma unroll
    for (int n1 = 0; n1 < 16; ++n1) v[n1] = irfft_pre_w(Xr, 16 * n1 + c, M, twR[n1]);
    fft256_passA<+1>(v, twA);
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) Tr[k1 * 17 + c] = v[k1];
    __syncthreads();
#pragma unroll
    for (int n2 = 0; n2 < 16; ++n2) v[n2] = Tr[c * 17 + n2];
    dft16<+1>(v);
    // v[k2] = L (x[2n] + i x[2n+1]) for n = c + 16 k2; nt <= 256 needs n < 128
    const int b = b0 + fr;
    if (b < B) {
      float* dst = out + ((int64_t)b * nrows + o) * nt;
#pragma unroll
      for (int k2 = 0; k2 < 8; ++k2) {
        const int m0 = 2 * (c + 16 * k2);
        if (m0 + 1 < nt && !(nt & 1)) {
          *reinterpret_cast<float2*>(dst + m0) = make_float2(v[k2].x * scale, v[k2].y * scale);
        } else {
          if (m0 < nt) dst[m0] = v[k2].x * scale;
          if (m0 + 1 < nt) dst[m0 + 1] = v[k2].y * scale;
        }
      }
    }
    __syncthreads();  // X and T are refilled by the next unit
  }
}

hipError_t launch_sum_irfft256(const float* part, int splits, int noq, int nrows, int B, int bp,
                               const float* tau_down, float* out, int nt, float scale, hipStream_t st) {
  if (B == 0 || nrows == 0) return hipSuccess;
  if (B < 0 || nrows < 0 || splits < 1 || noq < nrows || bp < B || nt < 1 || nt > 256) return hipErrorInvalidValue;
  const int64_t units = (int64_t)nrows * ((B + 15) / 16);
  if (units > 0x7fffffff) return hipErrorInvalidValue;
  const int64_t nblk = std::min<int64_t>(units, 256 * 8);
  hipLaunchKernelGGL(k_sum_irfft256, dim3((unsigned)nblk), dim3(256), 0, st, (const float2*)part, splits, noq, nrows,
                     B, bp, tau_down, out, nt, scale);
  return hipGetLastError();
}

hipError_t launch_mid_batch(float2* U, const float* sF, int B, int bp, bool adjoint, bool pack_bf16,
                            const Geometry& g, hipStream_t st, int rupts, float* cmax, int64_t cmax_floats,
                            int* cmax_groups, const DispOut* disp) {
  if (cmax_groups) *cmax_groups = 0;
  const DispOut dd = disp ? *disp : DispOut{};
  constexpr int R = 16;
  const int mode = g.diff ? (adjoint ? MID_BACKWARD_T : MID_BACKWARD) : MID_NONE;
  const float mscale = (float)(1.0 / ((double)g.L * (g.diff ? (double)g.dt : 1.0)));
  const int64_t units = (int64_t)g.ngrid * ((B + R - 1) / R);
  const int64_t nblk = std::min<int64_t>(units, 256 * 8);
  if (g.M == 256) {
    // units of 16 or 32 ruptures of one grid row (32: 256-byte runs per slot, one 512-thread
    // workgroup per CU)
    const int ru = rupts == 32 ? 32 : 16;
    const int nbb = (B + ru - 1) / ru;
    const int64_t units256 = (int64_t)g.ngrid * nbb;
    int64_t nb256 = std::min<int64_t>(units256, 256 * 8);
    if (cmax) {
      // whole groups of nbb workgroups, as many groups as the partial maxima fit
      const int64_t gmax = cmax_floats / ((int64_t)g.M * bp);
      int64_t groups = std::min<int64_t>(std::max<int64_t>(1, nb256 / nbb), gmax);
      if (groups < 1) return hipErrorInvalidValue;
      nb256 = groups * nbb;
      if (cmax_groups) *cmax_groups = (int)groups;
    }
    if (B < 1 || g.nt > 256 || units256 > 0x7fffffff) return hipErrorInvalidValue;  // M = 256 implies nt <= 256
#define S2W_MID256K(P_, R_, D_, M_)                                                                              \
  hipLaunchKernelGGL((k_mid_batch256<P_, R_, D_, M_>), dim3((unsigned)nb256), dim3(16 * R_), 0, st, U, sF, g.ngrid, B, \
                     bp, g.nt, mscale, cmax, dd)
    // forward: packed or plain output, with or without displacement capture; adjoint: plain
#define S2W_MID256(P_, R_)                                                                                       \
  do {                                                                                                            \
    if (adjoint) {                                                                                                \
      if (mode == MID_BACKWARD_T) S2W_MID256K(0, R_, false, MID_BACKWARD_T);                                      \
      else S2W_MID256K(0, R_, false, MID_NONE);                                                                   \
    } else if (mode == MID_BACKWARD) {                                                                            \
      if (dd.base) S2W_MID256K(P_, R_, true, MID_BACKWARD); else S2W_MID256K(P_, R_, false, MID_BACKWARD);        \
    } else {                                                                                                      \
      if (dd.base) S2W_MID256K(P_, R_, true, MID_NONE); else S2W_MID256K(P_, R_, false, MID_NONE);                \
    }                                                                                                             \
  } while (0)
    if (adjoint && (pack_bf16 || dd.base)) return hipErrorInvalidValue;
    if (ru == 32) {
      if (pack_bf16) S2W_MID256(1, 32); else S2W_MID256(0, 32);
    } else {
      if (pack_bf16) S2W_MID256(1, 16); else S2W_MID256(0, 16);
    }
#undef S2W_MID256
#undef S2W_MID256K
    return hipGetLastError();
  }
  const size_t lds = (2 * (size_t)g.M * (R + 1) + 2 * (size_t)g.M) * sizeof(float2);
#define S2W_MIDG(P_, D_)                                                                                        \
  hipLaunchKernelGGL((k_mid_batch<R, P_, D_>), dim3((unsigned)nblk), dim3(256), lds, st, U, sF, g.ngrid, B, bp, g.M, \
                     g.logM, g.nt, mode, mscale, dd)
  if (pack_bf16) {
    if (dd.base) S2W_MIDG(1, true); else S2W_MIDG(1, false);
  } else {
    if (dd.base) S2W_MIDG(0, true); else S2W_MIDG(0, false);
  }
#undef S2W_MIDG
  return hipGetLastError();
}

}  // namespace s2w
