// Transform kernels and the single-rupture contraction kernels.
//
// Stores (see s2w_api.cpp for sizes):
//   Gh[g][l][j]  elastic spectra, complex64, j padded to nsp (zeros), l < M = L/2 packed slots
//   Fh[g][l][o]  acoustic-gravity spectra, complex64, o padded to nop (zeros)
// Both are the temporal FFTs of the zero-padded response blocks (Alg. 2; Sec. II-C:
// computed once at setup and resident between calls).  Grid row g is contiguous, so a
// chunk of rows is one contiguous range, and for a fixed (g, l) the contraction index
// (j or o) is contiguous.
#include <math.h>

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
  float2* Z = lds_cfft(A, Bf, R, M, logM, -1);
  for (int i = threadIdx.x; i < R * M; i += blockDim.x) {
    const int r = i % R, k = i / R;
    const int64_t row = row0 + r;
    if (row < nrows) {
      const int64_t o = row / ninner_pad;
      const int inn = (int)(row - o * ninner_pad);
      out[o * out_outer + inn * out_inner + k * out_slot] = rfft_post(Z + r * M, k, M);
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
  hipLaunchKernelGGL(k_rfft_rows, dim3((unsigned)nblk), dim3(256), 2 * R * g.M * sizeof(float2), st, in, nrows,
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
  const int64_t row0 = (int64_t)blockIdx.x * R;
  for (int i = threadIdx.x; i < R * M; i += blockDim.x) {
    const int r = i % R, k = i / R;
    const int64_t row = row0 + r;
    X[r * M + k] = row < nrows ? in[row * in_row + k * in_slot] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < R * M; i += blockDim.x) {
    const int r = i >> logM, k = i & (M - 1);
    A[i] = irfft_pre(X + r * M, k, M);
  }
  __syncthreads();
  float2* z = lds_cfft(A, Bf, R, M, logM, +1);
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
  hipLaunchKernelGGL(k_irfft_rows, dim3((unsigned)nblk), dim3(256), 3 * R * g.M * sizeof(float2), st, in, nrows,
                     in_row, in_slot, out, out_row, g.nt, g.M, g.logM, R, scale);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Wave reductions.

// V values per lane (V a power of two <= 64), summed over the 64 lanes.  Halving
// butterfly: after it, lane l holds the full sum of value index (l >> (6 - log2 V)) & (V-1).
template <int V>
__device__ __forceinline__ float wave_reduce_many(float (&a)[V], int lane) {
  int m = 32;
#pragma unroll
  for (int h = V / 2; h >= 1; h >>= 1) {
    const bool up = (lane & m) != 0;
#pragma unroll
    for (int i = 0; i < h; ++i) {
      const float send = up ? a[i] : a[i + h];
      const float keep = up ? a[i + h] : a[i];
      a[i] = keep + __shfl_xor(send, m, 64);
    }
    m >>= 1;
  }
  for (; m >= 1; m >>= 1) a[0] += __shfl_xor(a[0], m, 64);
  return a[0];
}

template <int V>
struct Log2 {
  static constexpr int value = 1 + Log2<V / 2>::value;
};
template <>
struct Log2<1> {
  static constexpr int value = 0;
};

// Reduce the per-lane partial dot products a[2T] (T complex values) of the slot
// owned by this lane group and write them to D[t][l] (LDS, complex).
template <int T>
__device__ __forceinline__ void group_reduce_store(float (&a)[2 * T], int lane, int lps, int sl, int l, bool lok,
                                                   float2* D, int M) {
  if (lps == 64) {
    const float v = wave_reduce_many<2 * T>(a, lane);
    constexpr int sh = 6 - Log2<2 * T>::value;
    if ((lane & ((1 << sh) - 1)) == 0 && lok) {
      const int idx = (lane >> sh) & (2 * T - 1);
      reinterpret_cast<float*>(D)[((idx >> 1) * M + l) * 2 + (idx & 1)] = v;
    }
  } else {
#pragma unroll
    for (int v = 0; v < 2 * T; ++v) a[v] = group_sum(a[v], lps);
    if (sl == 0 && lok) {
#pragma unroll
      for (int t = 0; t < T; ++t) D[t * M + l] = make_float2(a[2 * t], a[2 * t + 1]);
    }
  }
}

// Contract T grid rows of a store X[g][l][c] (c the contraction index, nc4 float4 per
// (g, l)) with a per-slot vector Y[l][c] for every slot l < M, writing D[t][l] (LDS).
//   CONJ = false:  D = sum_c X * Y          (elastic step of the forward map, eq. 1)
//   CONJ = true:   D = sum_c conj(X) * Y    (acoustic step of the adjoint, eq. 2 transposed)
// Slot 0 holds two real bins and multiplies componentwise.
// Lane layout: groups of `lps` lanes share one slot; each lane covers c = sl + lps*i.
template <int T, int IMAX, bool CONJ>
__device__ __forceinline__ void contract_rows(const v4f* __restrict__ X, const v4f* __restrict__ Y, int g0, int tr,
                                              int M, int nc4, int lps, float2* D) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const int spw = 64 / lps;
  const int sub = lane / lps, sl = lane - sub * lps;
  for (int lb = wave * spw; lb < M; lb += nwaves * spw) {
    const int l = lb + sub;
    const bool lok = l < M;
    v4f yv[IMAX];
#pragma unroll
    for (int i = 0; i < IMAX; ++i) {
      const int c = sl + lps * i;
      yv[i] = (lok && c < nc4) ? Y[(int64_t)l * nc4 + c] : v4f{0.f, 0.f, 0.f, 0.f};
    }
    float a[2 * T];
#pragma unroll
    for (int v = 0; v < 2 * T; ++v) a[v] = 0.f;
    if (l == 0) {
#pragma unroll
      for (int t = 0; t < T; ++t) {
        if (t < tr) {
          const v4f* xr = X + ((int64_t)(g0 + t) * M) * nc4;
#pragma unroll
          for (int i = 0; i < IMAX; ++i) {
            const int c = sl + lps * i;
            if (c < nc4) {
              const v4f x = __builtin_nontemporal_load(xr + c);
              const v4f y = yv[i];
              a[2 * t] += x.x * y.x + x.z * y.z;
              a[2 * t + 1] += x.y * y.y + x.w * y.w;
            }
          }
        }
      }
    } else {
#pragma unroll
      for (int t = 0; t < T; ++t) {
        if (t < tr) {
          const v4f* xr = X + ((int64_t)(g0 + t) * M + l) * nc4;
#pragma unroll
          for (int i = 0; i < IMAX; ++i) {
            const int c = sl + lps * i;
            if (lok && c < nc4) {
              const v4f x = __builtin_nontemporal_load(xr + c);
              const v4f y = yv[i];
              if (CONJ) {
                a[2 * t] += x.x * y.x + x.y * y.y + x.z * y.z + x.w * y.w;
                a[2 * t + 1] += x.x * y.y - x.y * y.x + x.z * y.w - x.w * y.z;
              } else {
                a[2 * t] += x.x * y.x - x.y * y.y + x.z * y.z - x.w * y.w;
                a[2 * t + 1] += x.x * y.y + x.y * y.x + x.z * y.w + x.w * y.z;
              }
            }
          }
        }
      }
    }
    group_reduce_store<T>(a, lane, lps, sl, l, lok, D, M);
  }
}

// ---------------------------------------------------------------------------------------------
// Single-rupture fused forward.  Persistent: workgroup w owns grid rows
// [ngrid*w/nwg, ngrid*(w+1)/nwg) and walks them in tiles of T rows:
//   1. U[t][l] = sum_j Gh[g][l][j] Sh[l][j]                  (eq. 1 per bin, Alg. 2 step 3)
//   2. U -> V in LDS: inverse FFT, truncate, D_t, zero-pad, FFT   (Alg. 1 line 3; Alg. 2 steps 4-5, 1-2)
//   3. acc[l][o] += sum_t Fh[g][l][o] V[t][l]                (eq. 2 per bin, accumulated over rows)
// The seafloor field never leaves the workgroup.  The accumulator is written once,
// as this workgroup's partial observation spectrum.
template <int T, int IMAX, int OPT>
__global__ __launch_bounds__(256, 1) void k_fused_forward(const v4f* __restrict__ Gh, const v4f* __restrict__ Fh,
                                                          const v4f* __restrict__ Sh, v4f* __restrict__ part,
                                                          int ngrid, int M, int logM, int nsp4, int nop4, int lps,
                                                          int nt, int mode, float mscale) {
  extern __shared__ float2 smem[];
  float2* U = smem;
  float2* BA = U + T * M;
  float2* BB = BA + T * M;
  const int tid = threadIdx.x;
  const int wg = blockIdx.x, nwg = gridDim.x;
  const int r0 = (int)((int64_t)ngrid * wg / nwg), r1 = (int)((int64_t)ngrid * (wg + 1) / nwg);
  const int nitems = M * nop4;
  v4f acc[OPT];
  int lk[OPT];
#pragma unroll
  for (int k = 0; k < OPT; ++k) {
    acc[k] = v4f{0.f, 0.f, 0.f, 0.f};
    lk[k] = (k * (int)blockDim.x + tid) / nop4;
  }
  for (int g0 = r0; g0 < r1; g0 += T) {
    const int tr = min(T, r1 - g0);
    contract_rows<T, IMAX, false>(Gh, Sh, g0, tr, M, nsp4, lps, U);
    __syncthreads();
    lds_midchain(U, U, BA, BB, T, M, logM, nt, mode, mscale);
    for (int t = 0; t < tr; ++t) {
      const v4f* fr = Fh + (int64_t)(g0 + t) * M * nop4;
#pragma unroll
      for (int k = 0; k < OPT; ++k) {
        const int it = k * (int)blockDim.x + tid;
        if (it < nitems) {
          const int l = lk[k];
          const float2 v = U[t * M + l];
          const bool dc = (l == 0);
          const float c1 = v.x, c2 = dc ? 0.f : -v.y, c3 = dc ? 0.f : v.y, c4 = dc ? v.y : v.x;
          const v4f f = __builtin_nontemporal_load(fr + it);
          acc[k].x += f.x * c1 + f.y * c2;
          acc[k].y += f.x * c3 + f.y * c4;
          acc[k].z += f.z * c1 + f.w * c2;
          acc[k].w += f.z * c3 + f.w * c4;
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < OPT; ++k) {
    const int it = k * (int)blockDim.x + tid;
    if (it < nitems) part[(int64_t)wg * nitems + it] = acc[k];
  }
}

template <int T, int IMAX, int OPT>
static hipError_t fused_fwd_t(const float2* Gh, const float2* Fh, const float2* Sh, float2* part, int nwg,
                              const Geometry& g, int lps, hipStream_t st) {
  const int mode = g.diff ? MID_BACKWARD : MID_NONE;
  const float mscale = (float)(1.0 / ((double)g.L * (g.diff ? (double)g.dt : 1.0)));
  const size_t lds = 3 * (size_t)T * g.M * sizeof(float2);
  hipLaunchKernelGGL((k_fused_forward<T, IMAX, OPT>), dim3(nwg), dim3(256), lds, st, (const v4f*)Gh, (const v4f*)Fh,
                     (const v4f*)Sh, (v4f*)part, g.ngrid, g.M, g.logM, g.nsp4, g.nop4, lps, g.nt, mode, mscale);
  return hipGetLastError();
}

static inline int next_pow2(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

template <int T, int IMAX>
static hipError_t fused_fwd_opt(const float2* Gh, const float2* Fh, const float2* Sh, float2* part, int nwg,
                                const Geometry& g, int lps, hipStream_t st) {
  const int need = (g.M * g.nop4 + 255) / 256;
  if (need <= 4) return fused_fwd_t<T, IMAX, 4>(Gh, Fh, Sh, part, nwg, g, lps, st);
  if (need <= 8) return fused_fwd_t<T, IMAX, 8>(Gh, Fh, Sh, part, nwg, g, lps, st);
  if (need <= 16) return fused_fwd_t<T, IMAX, 16>(Gh, Fh, Sh, part, nwg, g, lps, st);
  if (need <= 32) return fused_fwd_t<T, IMAX, 32>(Gh, Fh, Sh, part, nwg, g, lps, st);
  return hipErrorInvalidValue;
}

template <int T>
static hipError_t fused_fwd_imax(const float2* Gh, const float2* Fh, const float2* Sh, float2* part, int nwg,
                                 const Geometry& g, hipStream_t st) {
  const int lps = g.nsp4 >= 64 ? 64 : next_pow2(g.nsp4);
  const int imax = (g.nsp4 + lps - 1) / lps;
  if (imax <= 1) return fused_fwd_opt<T, 1>(Gh, Fh, Sh, part, nwg, g, lps, st);
  if (imax <= 2) return fused_fwd_opt<T, 2>(Gh, Fh, Sh, part, nwg, g, lps, st);
  if (imax <= 4) return fused_fwd_opt<T, 4>(Gh, Fh, Sh, part, nwg, g, lps, st);
  if (imax <= 8) return fused_fwd_opt<T, 8>(Gh, Fh, Sh, part, nwg, g, lps, st);
  return hipErrorInvalidValue;
}

hipError_t launch_fused_forward(const float2* Gh, const float2* Fh, const float2* Sh, float2* part, int nwg,
                                int tile_rows, const Geometry& g, hipStream_t st) {
  if (tile_rows == 4) return fused_fwd_imax<4>(Gh, Fh, Sh, part, nwg, g, st);
  return fused_fwd_imax<8>(Gh, Fh, Sh, part, nwg, g, st);
}

// ---------------------------------------------------------------------------------------------
// Fixed-order sum of per-workgroup partial spectra.  part[p][l][c] (float4 = two complex
// columns), items = M * ncols4 per part -> out[col][l] (complex, row stride M) for col < nvalid.
__global__ __launch_bounds__(256) void k_reduce_partials(const v4f* __restrict__ part, int nparts, int64_t items,
                                                         int M, int ncols4, int nvalid, float2* __restrict__ out) {
  const int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (it >= items) return;
  v4f s = v4f{0.f, 0.f, 0.f, 0.f};
  for (int p = 0; p < nparts; ++p) s += part[(int64_t)p * items + it];
  const int l = (int)(it / ncols4);
  const int c0 = 2 * (int)(it - (int64_t)l * ncols4);
  if (c0 < nvalid) out[(int64_t)c0 * M + l] = make_float2(s.x, s.y);
  if (c0 + 1 < nvalid) out[(int64_t)(c0 + 1) * M + l] = make_float2(s.z, s.w);
}

hipError_t launch_reduce_partials(const float2* part, int nparts, int64_t items, int M, int ncols, int nvalid,
                                  float2* out, hipStream_t st) {
  (void)ncols;
  const int ncols4 = (int)(items / M);
  const int64_t nblk = (items + 255) / 256;
  hipLaunchKernelGGL(k_reduce_partials, dim3((unsigned)nblk), dim3(256), 0, st, (const v4f*)part, nparts, items, M,
                     ncols4, nvalid, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Single-rupture adjoint, stage 1.  Per grid row g:
//   W[l]  = sum_o conj(Fh[g][l][o]) Rh[l][o]        (transpose of eq. 2, per bin)
//   W'    = rfft(pad(D_t^T trunc(irfft(W))))         (transposed mid-chain)
// written to Wp[g][l].
template <int T, int IMAX>
__global__ __launch_bounds__(256) void k_adjoint_rows(const v4f* __restrict__ Fh, const v4f* __restrict__ Rh,
                                                      float2* __restrict__ Wp, int ngrid, int M, int logM, int nop4,
                                                      int lps, int nt, int mode, float mscale) {
  extern __shared__ float2 smem[];
  float2* U = smem;
  float2* BA = U + T * M;
  float2* BB = BA + T * M;
  const int wg = blockIdx.x, nwg = gridDim.x;
  const int r0 = (int)((int64_t)ngrid * wg / nwg), r1 = (int)((int64_t)ngrid * (wg + 1) / nwg);
  for (int g0 = r0; g0 < r1; g0 += T) {
    const int tr = min(T, r1 - g0);
    contract_rows<T, IMAX, true>(Fh, Rh, g0, tr, M, nop4, lps, U);
    __syncthreads();
    lds_midchain(U, U, BA, BB, T, M, logM, nt, mode, mscale);
    for (int i = threadIdx.x; i < tr * M; i += blockDim.x) Wp[(int64_t)g0 * M + i] = U[i];
    __syncthreads();
  }
}

template <int T>
static hipError_t adjoint_rows_t(const float2* Fh, const float2* Rh, float2* Wp, int nwg, const Geometry& g,
                                 hipStream_t st) {
  const int lps = g.nop4 >= 64 ? 64 : next_pow2(g.nop4);
  const int imax = (g.nop4 + lps - 1) / lps;
  const int mode = g.diff ? MID_BACKWARD_T : MID_NONE;
  const float mscale = (float)(1.0 / ((double)g.L * (g.diff ? (double)g.dt : 1.0)));
  const size_t lds = 3 * (size_t)T * g.M * sizeof(float2);
#define S2W_ADJ_ROWS(IM)                                                                                        \
  hipLaunchKernelGGL((k_adjoint_rows<T, IM>), dim3(nwg), dim3(256), lds, st, (const v4f*)Fh, (const v4f*)Rh, Wp, \
                     g.ngrid, g.M, g.logM, g.nop4, lps, g.nt, mode, mscale)
  if (imax <= 1) S2W_ADJ_ROWS(1);
  else if (imax <= 2) S2W_ADJ_ROWS(2);
  else return hipErrorInvalidValue;
#undef S2W_ADJ_ROWS
  return hipGetLastError();
}

hipError_t launch_adjoint_rows(const float2* Fh, const float2* Rh, float2* Wp, int nwg, int tile_rows,
                               const Geometry& g, hipStream_t st) {
  if (tile_rows == 4) return adjoint_rows_t<4>(Fh, Rh, Wp, nwg, g, st);
  return adjoint_rows_t<8>(Fh, Rh, Wp, nwg, g, st);
}

// Contraction over grid rows, per bin, split over row ranges:
//   CONJ = true:  part[split][l][j] = sum_{g in split} conj(X[g][l][j]) W[g][l]
//                 (single-rupture adjoint, transpose of eq. 1)
//   CONJ = false: part[split][l][o] = sum_{g in split} X[g][l][o] W[g][l]
//                 (unfused forward, eq. 2 per bin)
// Workgroup (slot block, split); each thread owns float4 columns c = tid + 256 i.
template <int LT, int JMAX, bool CONJ>
__global__ __launch_bounds__(256) void k_rows_contract(const v4f* __restrict__ Gh, const float2* __restrict__ Wp,
                                                       v4f* __restrict__ part, int ngrid, int M, int nsp4) {
  const int l0 = blockIdx.x * LT;
  const int split = blockIdx.y, splits = gridDim.y;
  const int r0 = (int)((int64_t)ngrid * split / splits), r1 = (int)((int64_t)ngrid * (split + 1) / splits);
  const int tid = threadIdx.x;
  v4f acc[LT][JMAX];
#pragma unroll
  for (int a = 0; a < LT; ++a)
#pragma unroll
    for (int i = 0; i < JMAX; ++i) acc[a][i] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int g = r0; g < r1; ++g) {
    const v4f* gr = Gh + ((int64_t)g * M + l0) * nsp4;
    const float2* wr = Wp + (int64_t)g * M + l0;
#pragma unroll
    for (int a = 0; a < LT; ++a) {
      const float2 w = wr[a];
      const bool dc = (l0 + a) == 0;
      // conj(x) * w (or x * w) for complex slots; componentwise for the packed real slot
      const float c1 = w.x;
      const float c2 = dc ? 0.f : (CONJ ? w.y : -w.y);
      const float c3 = dc ? 0.f : w.y;
      const float c4 = dc ? w.y : (CONJ ? -w.x : w.x);
#pragma unroll
      for (int i = 0; i < JMAX; ++i) {
        const int c = tid + 256 * i;
        if (c < nsp4) {
          const v4f x = __builtin_nontemporal_load(gr + (int64_t)a * nsp4 + c);
          acc[a][i].x += x.x * c1 + x.y * c2;
          acc[a][i].y += x.x * c3 + x.y * c4;
          acc[a][i].z += x.z * c1 + x.w * c2;
          acc[a][i].w += x.z * c3 + x.w * c4;
        }
      }
    }
  }
#pragma unroll
  for (int a = 0; a < LT; ++a)
#pragma unroll
    for (int i = 0; i < JMAX; ++i) {
      const int c = tid + 256 * i;
      if (c < nsp4) part[((int64_t)split * M + l0 + a) * nsp4 + c] = acc[a][i];
    }
}

template <bool CONJ>
static hipError_t rows_contract_t(const float2* X, const float2* W, float2* part, int slots_per_wg, int splits,
                                  int nc4, const Geometry& g, hipStream_t st) {
  const int jmax = (nc4 + 255) / 256;
  const int LT = slots_per_wg == 4 ? 4 : 8;
  dim3 grid(g.M / LT, splits);
#define S2W_ROWS_C(L_, J_)                                                                                   \
  hipLaunchKernelGGL((k_rows_contract<L_, J_, CONJ>), grid, dim3(256), 0, st, (const v4f*)X, W, (v4f*)part, \
                     g.ngrid, g.M, nc4)
  if (LT == 4) {
    if (jmax <= 1) S2W_ROWS_C(4, 1);
    else if (jmax <= 2) S2W_ROWS_C(4, 2);
    else return hipErrorInvalidValue;
  } else {
    if (jmax <= 1) S2W_ROWS_C(8, 1);
    else if (jmax <= 2) S2W_ROWS_C(8, 2);
    else return hipErrorInvalidValue;
  }
#undef S2W_ROWS_C
  return hipGetLastError();
}

hipError_t launch_adjoint_elastic(const float2* Gh, const float2* Wp, float2* part, int slots_per_wg, int splits,
                                  const Geometry& g, hipStream_t st) {
  return rows_contract_t<true>(Gh, Wp, part, slots_per_wg, splits, g.nsp4, g, st);
}

hipError_t launch_rows_acoustic(const float2* Fh, const float2* Vh, float2* part, int slots_per_wg, int splits,
                                const Geometry& g, hipStream_t st) {
  return rows_contract_t<false>(Fh, Vh, part, slots_per_wg, splits, g.nop4, g, st);
}

// Unfused forward, stage 1: per grid row, the elastic contraction and the mid-chain
// round trip, written to Vh[g][l] (used when the fused kernel's accumulator does not fit).
template <int T, int IMAX>
__global__ __launch_bounds__(256) void k_forward_rows(const v4f* __restrict__ Gh, const v4f* __restrict__ Sh,
                                                      float2* __restrict__ Vh, int ngrid, int M, int logM, int nsp4,
                                                      int lps, int nt, int mode, float mscale) {
  extern __shared__ float2 smem[];
  float2* U = smem;
  float2* BA = U + T * M;
  float2* BB = BA + T * M;
  const int wg = blockIdx.x, nwg = gridDim.x;
  const int r0 = (int)((int64_t)ngrid * wg / nwg), r1 = (int)((int64_t)ngrid * (wg + 1) / nwg);
  for (int g0 = r0; g0 < r1; g0 += T) {
    const int tr = min(T, r1 - g0);
    contract_rows<T, IMAX, false>(Gh, Sh, g0, tr, M, nsp4, lps, U);
    __syncthreads();
    lds_midchain(U, U, BA, BB, T, M, logM, nt, mode, mscale);
    for (int i = threadIdx.x; i < tr * M; i += blockDim.x) Vh[(int64_t)g0 * M + i] = U[i];
    __syncthreads();
  }
}

hipError_t launch_forward_rows(const float2* Gh, const float2* Sh, float2* Vh, int nwg, const Geometry& g,
                               hipStream_t st) {
  constexpr int T = 8;
  const int lps = g.nsp4 >= 64 ? 64 : next_pow2(g.nsp4);
  const int imax = (g.nsp4 + lps - 1) / lps;
  const int mode = g.diff ? MID_BACKWARD : MID_NONE;
  const float mscale = (float)(1.0 / ((double)g.L * (g.diff ? (double)g.dt : 1.0)));
  const size_t lds = 3 * (size_t)T * g.M * sizeof(float2);
#define S2W_FWD_ROWS(IM)                                                                                          \
  hipLaunchKernelGGL((k_forward_rows<T, IM>), dim3(nwg), dim3(256), lds, st, (const v4f*)Gh, (const v4f*)Sh, Vh, \
                     g.ngrid, g.M, g.logM, g.nsp4, lps, g.nt, mode, mscale)
  if (imax <= 1) S2W_FWD_ROWS(1);
  else if (imax <= 2) S2W_FWD_ROWS(2);
  else if (imax <= 4) S2W_FWD_ROWS(4);
  else if (imax <= 8) S2W_FWD_ROWS(8);
  else return hipErrorInvalidValue;
#undef S2W_FWD_ROWS
  return hipGetLastError();
}

}  // namespace s2w
