// Direct time-domain evaluation of the map, no FFT: each block lower-triangular Toeplitz
// product is computed from its defining sum in the channel form of eq. (4),
//
//   out[r][n] = sum_c sum_{k=0}^{n} A(c, r, k) x_c[n - k],   n < Nt,
//
// on the float32 matrix cores.  This is the paper's direct reference evaluation (Sec. II-C2)
// of eq. (1) (rows r = grid points, channels c = subfaults, A = the elastic blocks), of eq. (2)
// (rows = observers, channels = grid points, A = the acoustic blocks), and, with the time axis
// reversed, of their transposes (the correlations of the adjoint).
//
// As a matrix product, for one channel c the operator row A(c, r, .) (Nt lags) multiplies the
// Toeplitz matrix T_c[k][n] = x_c[n - k] (zero for k > n).  With the time axis cut into blocks
// of 16, the block (kb, nb) of T_c is zero for kb > nb and depends only on d = nb - kb, so one
// channel is a sum over the 136 block pairs kb <= nb (Nt = 256) of 16 x 16 x 16 products: the
// upper triangle of T is never multiplied, except inside the diagonal blocks.
//
// MFMA v_mfma_f32_16x16x4_f32 fragments, lane l = 16 kq + li of 64:
//   A (16 x 4): row li, K entry kq;  B (4 x 16): column li, K entry kq;
//   D (16 x 16): column li, rows 4 kq .. 4 kq + 3.
// K order inside a block of 16 lags: in step q (0..3) lane group kq carries lag 16 kb + 4 kq + q,
// so a lane reads its four operator values of a block as one float4 and the matching Toeplitz
// entries x[16 d + li - 4 kq - q] from the channel's LDS copy.  Blocks are taken in pairs
// (2m, 2m + 1), one 128-byte line of the operator row per lane row, in the order
// 0, P-1, 1, P-2, ... so that the long early pairs and the short late ones alternate and every
// pair's operator loads are in flight during the previous pair's products.
#include "s2w_device.h"
#include "s2w_internal.h"

namespace s2w {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kDirectXs = 16 + 512;  // LDS floats per staged channel: 16 zeros, then x[0 .. ntp)

struct DirectArgs {
  const float* A;   // A(c, r, k) at A + c*a_c + r*a_r + k (k < ntp; zeros at k >= nt)
  int64_t a_c, a_r;
  int R;            // rows written (loads clamp below it)
  int nchan;
  const float* X;   // x_c[p] at X + c*x_c + (rev ? nt - 1 - p : p), p < nt
  int64_t x_c;
  int rev;
  float* out;       // out + split*o_s + r*o_r + n, n < nt
  int64_t o_s, o_r;
  int nt, ntp;      // ntp: nt rounded up to 16
  int nrt;          // row tiles (64 * RW rows each)
  int splits;       // channel splits, one partial output each
  int nranges;      // ranges of 16 output blocks (Nt > 256 needs two)
};

// Workgroup: four waves, wave w owns rows r0 + 16 RW w .. + 16 RW - 1 of the tile; all waves
// share the staged channel.  Grid: row tile x channel split x output range.
template <int RW>
__global__ __launch_bounds__(256, 2) void k_direct(const DirectArgs p) {
  __shared__ float xs[2][kDirectXs];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, kq = lane >> 4;
  int q = blockIdx.x;
  const int range = q % p.nranges;
  q /= p.nranges;
  const int split = q % p.splits;
  const int rt = q / p.splits;
  const int c0 = (int)((int64_t)p.nchan * split / p.splits);
  const int c1 = (int)((int64_t)p.nchan * (split + 1) / p.splits);
  const int nbt = p.ntp >> 4;                 // blocks of 16 output steps
  const int nb0 = 16 * range, nb1 = min(nb0 + 16, nbt);
  const int npairs = (nb1 + 1) >> 1;          // lag-block pairs touching the range
  const int r0 = rt * 64 * RW + wave * 16 * RW;

  // this lane's operator rows (clamped: rows past R are loaded but never written)
  const float* arow[RW];
#pragma unroll
  for (int rb = 0; rb < RW; ++rb) arow[rb] = p.A + (int64_t)min(r0 + 16 * rb + li, p.R - 1) * p.a_r + 4 * kq;

  f32x4 acc[RW][16];
#pragma unroll
  for (int rb = 0; rb < RW; ++rb)
#pragma unroll
    for (int j = 0; j < 16; ++j) acc[rb][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int i = tid; i < 16; i += 256) {
    xs[0][i] = 0.f;
    xs[1][i] = 0.f;
  }
  // staged channel values: thread t holds x[t] and x[t + 256]
  auto load_x = [&](int c, float (&v)[2]) {
    const float* xc = p.X + (int64_t)c * p.x_c;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int t = tid + 256 * h;
      v[h] = t < p.nt ? xc[p.rev ? p.nt - 1 - t : t] : 0.f;
    }
  };
  auto store_x = [&](int buf, const float (&v)[2]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int t = tid + 256 * h;
      if (t < p.ntp) xs[buf][16 + t] = v[h];
    }
  };
  // pair order: 0, P-1, 1, P-2, ...
  auto pair_of = [&](int i) { return (i & 1) ? npairs - 1 - (i >> 1) : (i >> 1); };
  auto load_a = [&](int c, int m, float4 (&a)[2][RW]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int kb = 2 * m + h;
#pragma unroll
      for (int rb = 0; rb < RW; ++rb)
        a[h][rb] = kb < nbt ? *reinterpret_cast<const float4*>(arow[rb] + (int64_t)c * p.a_c + 16 * kb)
                            : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  auto products = [&](const float* xb, int m, const float4 (&a)[2][RW]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int kb = 2 * m + h;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int nb = nb0 + j;
        if (nb >= kb && nb < nb1) {
          const float* t = xb + 16 + 16 * (nb - kb) + li - 4 * kq;
          const float b0 = t[0], b1 = t[-1], b2 = t[-2], b3 = t[-3];
#pragma unroll
          for (int rb = 0; rb < RW; ++rb) {
            acc[rb][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[h][rb].x, b0, acc[rb][j], 0, 0, 0);
            acc[rb][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[h][rb].y, b1, acc[rb][j], 0, 0, 0);
            acc[rb][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[h][rb].z, b2, acc[rb][j], 0, 0, 0);
            acc[rb][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[h][rb].w, b3, acc[rb][j], 0, 0, 0);
          }
        }
      }
    }
  };

  if (c0 < c1) {
    float xv[2];
    load_x(c0, xv);
    store_x(0, xv);
    float4 a0[2][RW], a1[2][RW];
    load_a(c0, pair_of(0), a0);
    __syncthreads();
    for (int c = c0; c < c1; ++c) {
      const int buf = (c - c0) & 1;
      const bool more = c + 1 < c1;
      if (more) load_x(c + 1, xv);
      const float* xb = xs[buf];
      // pairs two at a time, each pair's loads issued before the previous pair's products; the
      // last load of a channel fetches the first pair of the next one
      for (int i = 0; i < npairs; i += 2) {
        const bool second = i + 1 < npairs;
        if (second) load_a(c, pair_of(i + 1), a1);
        else if (more) load_a(c + 1, pair_of(0), a1);
        products(xb, pair_of(i), a0);
        if (second) {
          if (i + 2 < npairs) load_a(c, pair_of(i + 2), a0);
          else if (more) load_a(c + 1, pair_of(0), a0);
          products(xb, pair_of(i + 1), a1);
        } else {
          // odd pair count: the next channel's first pair sits in a1
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int rb = 0; rb < RW; ++rb) a0[h][rb] = a1[h][rb];
        }
      }
      if (more) store_x(buf ^ 1, xv);
      __syncthreads();
    }
  }
  float* ow = p.out + (int64_t)split * p.o_s;
#pragma unroll
  for (int rb = 0; rb < RW; ++rb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = r0 + 16 * rb + 4 * kq + v;
      if (r >= p.R) continue;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int n = 16 * (nb0 + j) + li;
        if (nb0 + j < nb1 && n < p.nt) ow[(int64_t)r * p.o_r + n] = acc[rb][j][v];
      }
    }
}

int direct_rows_per_tile(int rw) { return 64 * rw; }

hipError_t launch_direct(int rw, const float* A, int64_t a_c, int64_t a_r, int R, int nchan, const float* X,
                         int64_t x_c, bool rev, float* out, int64_t o_s, int64_t o_r, int nt, int splits,
                         hipStream_t st) {
  if ((rw != 1 && rw != 2) || nt < 1 || nt > 512 || R < 1 || nchan < 1 || splits < 1 || splits > nchan ||
      (a_c & 3) || (a_r & 3) || ((uintptr_t)A & 15))
    return hipErrorInvalidValue;
  DirectArgs a;
  a.A = A;
  a.a_c = a_c;
  a.a_r = a_r;
  a.R = R;
  a.nchan = nchan;
  a.X = X;
  a.x_c = x_c;
  a.rev = rev ? 1 : 0;
  a.out = out;
  a.o_s = o_s;
  a.o_r = o_r;
  a.nt = nt;
  a.ntp = (nt + 15) / 16 * 16;
  a.nrt = (R + 64 * rw - 1) / (64 * rw);
  a.splits = splits;
  a.nranges = (a.ntp / 16 + 15) / 16;
  const int64_t blocks = (int64_t)a.nrt * splits * a.nranges;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  if (rw == 1)
    hipLaunchKernelGGL((k_direct<1>), dim3((unsigned)blocks), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((k_direct<2>), dim3((unsigned)blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

// Fixed-order sum over partials with an optional backward difference and time reversal:
//   S(r, p)  = sum_{q < parts} part[q*p_s + r*p_r + (rev ? nt - 1 - p : p)]
//   out[r*o_r + p] = diff ? (S(r, p) - S(r, p - 1)) * scale : S(r, p) * scale,  S(r, -1) = 0.
// Between the two products it forms D_t of the seafloor field (forward) or, on the time-reversed
// correlation, D_t^T (the adjoint); at the end it sums the output partials.  In the forward map
// S is the seafloor displacement m of eq. (1), which `disp` may capture at selected steps.
__global__ __launch_bounds__(256) void k_direct_reduce(const float* __restrict__ part, int parts, int64_t p_s,
                                                       int64_t p_r, int R, int nt, int rev, int diff, float scale,
                                                       float* __restrict__ out, int64_t o_r, DispOut disp) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (int64_t)R * nt) return;
  const int r = (int)(i / nt), n = (int)(i % nt);
  const float* pr = part + (int64_t)r * p_r;
  const int t = rev ? nt - 1 - n : n;
  float s = 0.f;
  for (int q = 0; q < parts; ++q) s += pr[(int64_t)q * p_s + t];
  if (disp.base && r < disp.rows) {
    const int c = disp_col(disp, n);
    if (c >= 0) disp.base[(int64_t)r * disp.row_stride + c] = s * disp.scale;
  }
  if (diff && n > 0) {
    const int t1 = rev ? nt - n : n - 1;
    float s1 = 0.f;
    for (int q = 0; q < parts; ++q) s1 += pr[(int64_t)q * p_s + t1];
    s -= s1;
  }
  out[(int64_t)r * o_r + n] = s * scale;
}

hipError_t launch_direct_reduce(const float* part, int parts, int64_t p_s, int64_t p_r, int R, int nt, bool rev,
                                bool diff, float scale, float* out, int64_t o_r, hipStream_t st,
                                const DispOut* disp) {
  if (parts < 1 || R < 1 || nt < 1) return hipErrorInvalidValue;
  const int64_t items = (int64_t)R * nt;
  hipLaunchKernelGGL(k_direct_reduce, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, st, part, parts, p_s, p_r,
                     R, nt, rev ? 1 : 0, diff ? 1 : 0, scale, out, o_r, disp ? *disp : DispOut{});
  return hipGetLastError();
}

// Time-domain store rows: out[s][k] = in[s][k] for k < nt, 0 for nt <= k < ntp (series s < n).
__global__ __launch_bounds__(256) void k_pad_series(const float* __restrict__ in, int64_t n, int nt, int ntp,
                                                    float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n * ntp) return;
  const int64_t s = i / ntp;
  const int k = (int)(i % ntp);
  out[i] = k < nt ? in[s * nt + k] : 0.f;
}

hipError_t launch_pad_series(const float* in, int64_t n, int nt, int ntp, float* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t items = n * ntp;
  hipLaunchKernelGGL(k_pad_series, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, st, in, n, nt, ntp, out);
  return hipGetLastError();
}

}  // namespace s2w
