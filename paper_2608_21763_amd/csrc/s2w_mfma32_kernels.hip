// Batched float32 path on the matrix cores: per-slot complex GEMMs on v_mfma_f32_16x16x4_f32.
//
// Float32 stores of the batched layout (complex64):
//   Gs[g][l][j]  elastic spectra, j padded to nsk (a multiple of 8, zeros)
//   Fs[l][o][g]  acoustic spectra, o padded to nok (a multiple of 16, zeros), g padded to ngk
//                (a multiple of 8, zeros)
//
// One kernel serves the four per-slot products of the forward map and its adjoint
// (eq. 1 and eq. 2 per bin, Alg. 2 step 3, and their conjugate transposes):
//   out(row, b) = sum_k op(A(row, k)) X(k, b),    op = identity or complex conjugate,
// for every packed slot l.  A(row, k) is read either k-contiguous (Gs as [g][j], Fs as [o][g])
// or row-contiguous (the conjugate transposes: Fs^H as [g][o], Gs^H as [j][g]); X(k, b) is
// rupture-contiguous.
//
// Complex arithmetic on real matrix cores: the operator value a = ar + i ai contributes the two
// real K entries (ar, ai) of its row; each activation value x gives two output columns,
//   real column:       (xr, -xi)   [conjugated operator: (xr,  xi)]
//   imaginary column:  (xi,  xr)   [conjugated operator: (xi, -xr)]
// and the packed real slot 0 (bins 0 and L/2) uses (xr, 0) and (0, xi).
//
// MFMA v_mfma_f32_16x16x4_f32 fragments, lane l of 64:
//   A (16 x 4): row l%16, K entry l/16;  B (4 x 16): column l%16, K entry l/16;
//   D (16 x 16): column l%16, rows 4*(l/16) .. +3.
// K order: a chunk of 8 complex k (16 real entries) is four MFMA steps e = 0..3; in step e the
// lane group kq = l/16 carries complex k = 2*kq + e/2, real or imaginary part e%2.  A lane thus
// reads its operator values for a whole chunk as one float4 (complex k = 2kq, 2kq+1).
#include "s2w_internal.h"

namespace s2w {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// 16-byte unit c (0..3) of tile row r: XOR swizzle so that the 16 rows read together by a
// quarter wave spread over distinct bank groups.
__device__ __forceinline__ int swz32(int r, int c) { return r * 4 + (c ^ ((r >> 1) & 3)); }

template <bool CONJ>
__device__ __forceinline__ void embed32(float2 x, int ci, bool dc, float& v0, float& v1) {
  if (dc) {
    v0 = ci ? 0.f : x.x;
    v1 = ci ? x.y : 0.f;
  } else if (!CONJ) {
    v0 = ci ? x.y : x.x;
    v1 = ci ? x.x : -x.y;
  } else {
    v0 = ci ? x.y : x.x;
    v1 = ci ? -x.x : x.y;
  }
}

struct CGemmArgs {
  const float2* A;
  int64_t a_row, a_k, a_slot;  // complex strides of A(row, k) within slot l (one of a_row, a_k is 1)
  int nrows;                   // rows written
  int rows_alloc;              // rows readable (row loads clamp below it)
  int kvalid;                  // k < kvalid are real; later k read as zero
  int nchunks;                 // chunks of 8 complex k over the whole K range
  const float2* X;
  int64_t x_k, x_slot;         // complex strides of X(k, b); b contiguous
  int xk_alloc;                // k rows of X that exist (loads clamp below it)
  int bp;                      // rupture stride padding (even)
  float* out;
  int64_t o_row, o_slot, o_split;  // float strides; column n = 2*b + (0 re | 1 im)
  int ncols;                   // columns written (2*B)
  int M, nrt, nct, splits;
};

// Copies of chunk c of a float32 product into one LDS stage (see k_cgemm32d).
template <int NRT>
__device__ __forceinline__ int c32d_xsw(int kk) {
  return NRT >= 32 ? ((kk >> 1) & 3) * 4 : 0;
}

// XOR of the row-pair units of operator k row kk (row-contiguous operators, RT >= 64)
__device__ __forceinline__ int c32d_asw(int kk) { return ((kk >> 1) & 3) * 8; }

// Operator copy q of a wave: k-contiguous operators take asrc[q] + 8 c (asrc already holds the
// row and 16-byte unit of the lane); row-contiguous ones take k row 8 c + akk[q] (clamped below
// kvalid: k rows past it need not exist and their products are zeroed through the activation)
// at the row pair held in asrc[q].
template <int NRT, int A_PER_W, int X_PER_W, int X_LANES, bool RCONT>
__device__ __forceinline__ void c32d_issue(const float2* const (&asrc)[A_PER_W], const int (&akk)[A_PER_W],
                                           const float2* Xl, const CGemmArgs& p, int b0, int c, float4* a_dst,
                                           float4* x_dst, int wave, int lane) {
#pragma unroll
  for (int qq = 0; qq < A_PER_W; ++qq) {
    const float2* src = RCONT ? asrc[qq] + (int64_t)min(8 * c + akk[qq], p.kvalid - 1) * p.a_k : asrc[qq] + 8 * c;
    __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)(a_dst + 256 * qq), 16, 0, 0);
  }
  // all 64 lanes copy (no branch: a divergent copy makes the compiler drain every copy in
  // flight at the loop head); lane j >= X_LANES writes the unit that belongs at its position,
  // the same bytes as the wave that owns it, or past the block into padding
#pragma unroll
  for (int t = 0; t < X_PER_W; ++t) {
    const int u = min((wave * X_PER_W + t) * X_LANES + lane, 4 * NRT - 1);
    const int kk = u / (NRT / 2), pq = (u % (NRT / 2)) ^ c32d_xsw<NRT>(kk);
    const int k = min(8 * c + kk, p.xk_alloc - 1);
    const int b = min(b0 + 2 * pq, p.bp - 2);
    float4* dst = x_dst + (wave * X_PER_W + t) * X_LANES;
    __builtin_amdgcn_global_load_lds(Xl + (int64_t)k * p.x_k + b, (__attribute__((address_space(3))) void*)dst, 16, 0,
                                     0);
  }
}

// Workgroup = 4 waves in a WR x WC grid; wave tile MF x NF fragments of 16 x 16.  Tile: RT =
// WR*MF*16 rows x NRT = WC*NF*8 ruptures; K in chunks of 8 complex values.  Blocks are decoded
// so that all tiles of slot l run on XCD l mod 8 (workgroups are dealt to the eight XCDs
// round-robin), keeping a slot's activation panel in one L2.
// The tiles are copied straight from global memory into LDS (global_load_lds_dwordx4, no
// register staging) in NS stages: register-staged copies cap a streaming kernel near half the
// HBM bandwidth.  Each wave copies RT/64 operator blocks of 1 KB and a quarter of the
// activation block (the 8 k x NRT ruptures of a chunk, NRT float2 per k row, NRT/16 KB) per
// chunk.  A k-contiguous operator block is 16 rows x 64 bytes, the lanes assigned so that the
// linear LDS placement is the swz32 layout; a row-contiguous operator is held k-major (RT
// complex per k row, row pairs XOR-swizzled by c32d_asw) and its fragment is read as two 8-byte
// halves.  Entries k >= kvalid are zeroed in the activation, in registers (operator values
// there are finite: rows past kvalid are clamped to existing ones).
template <int MF, int NF, int WR, int WC, int NS, bool RCONT, bool CONJ>
__global__ __launch_bounds__(256, 2) void k_cgemm32d(const CGemmArgs p) {
  static_assert(WR * WC == 4, "four waves");
  constexpr int RT = WR * MF * 16;
  constexpr int NRT = WC * NF * 8;
  constexpr int A_BLK = RT / 16;                        // 1 KB operator blocks per chunk
  constexpr int A_PER_W = A_BLK / 4;
  constexpr int X_U4 = 4 * NRT;                         // activation 16-byte units per chunk
  constexpr int X_PER_W = X_U4 / 4 > 64 ? X_U4 / 256 : 1;  // activation copies per wave and chunk
  constexpr int X_LANES = X_U4 / 4 > 64 ? 64 : X_U4 / 4;   // active lanes of an activation copy
  constexpr int PER_W = A_PER_W + X_PER_W;
  constexpr int STAGE = A_BLK * 64 + X_U4 + 64 - X_LANES;  // float4 per stage, with copy padding
  constexpr int PENDING = (NS - 2) * PER_W;
  static_assert(A_BLK % 4 == 0 && X_U4 % 4 == 0, "every wave issues the same copies");
  static_assert(NS >= 2 && NS <= 4 && PENDING < 16, "stages and wait counts");
  __shared__ float4 st0[STAGE];
  __shared__ float4 st1[STAGE];
  __shared__ float4 st2[NS > 2 ? STAGE : 1];
  __shared__ float4 st3[NS > 3 ? STAGE : 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave / WC, wc = wave % WC;
  const int ci = lane & 1, kq = lane >> 4;
  const int x = blockIdx.x & 7, q = blockIdx.x >> 3;
  const int per_slot = p.nrt * p.nct * p.splits;
  const int l = x + 8 * (q / per_slot);
  int rem = q % per_slot;
  const int split = rem % p.splits;
  rem /= p.splits;
  const int ct = rem % p.nct, rt = rem / p.nct;
  const bool dc = (l == 0);
  const int c0 = (int)((int64_t)p.nchunks * split / p.splits);
  const int c1 = (int)((int64_t)p.nchunks * (split + 1) / p.splits);
  const int row0 = rt * RT, b0 = ct * NRT;
  const float2* Al = p.A + (int64_t)l * p.a_slot;
  const float2* Xl = p.X + (int64_t)l * p.x_slot;
  // operator copy q of this wave fills 1 KB block wave + 4 q of the stage.  k-contiguous: 16 rows,
  // lane -> row lane / 4 and the 16-byte unit cc whose linear LDS slot is swz32(row, cc).
  // Row-contiguous: unit u = 64 (wave + 4 q) + lane is slot s = u % (RT / 2) of k row
  // kk = u / (RT / 2) and holds row pair s ^ c32d_asw(kk).
  const float2* asrc[A_PER_W];
  int akk[A_PER_W];
#pragma unroll
  for (int qq = 0; qq < A_PER_W; ++qq) {
    if (!RCONT) {
      const int r = 16 * (wave + 4 * qq) + (lane >> 2);
      const int cc = (lane & 3) ^ ((r >> 1) & 3);
      asrc[qq] = Al + (int64_t)min(row0 + r, p.rows_alloc - 1) * p.a_row + 2 * cc;
      akk[qq] = 0;
    } else {
      const int u = 64 * (wave + 4 * qq) + lane;
      akk[qq] = u / (RT / 2);
      const int rp = (u % (RT / 2)) ^ c32d_asw(akk[qq]);
      asrc[qq] = Al + min(row0 + 2 * rp, p.rows_alloc - 2);
    }
  }
  // activation copy: unit u = (wave * X_PER_W + t) * X_LANES + lane is slot s = u % (NRT / 2) of k
  // row kk = u / (NRT / 2) and holds rupture pair s ^ c32d_xsw(kk): the XOR spreads the four k
  // rows read together by a wave over distinct LDS banks.  Past the range, a copy of the last
  // chunk is issued (never read), so that every step has the same number of copies in flight.
  auto issue = [&](int c, float4* stage) {
    c32d_issue<NRT, A_PER_W, X_PER_W, X_LANES, RCONT>(asrc, akk, Xl, p, b0, min(c, c1 - 1), stage + wave * 64,
                                                       stage + A_BLK * 64, wave, lane);
  };

  f32x4 acc[MF][NF];
#pragma unroll
  for (int a = 0; a < MF; ++a)
#pragma unroll
    for (int f = 0; f < NF; ++f) acc[a][f] = f32x4{0.f, 0.f, 0.f, 0.f};

  auto compute = [&](int c, const float4* cur) {
    const float2* lx = reinterpret_cast<const float2*>(cur + A_BLK * 64);
    float4 av[MF];
#pragma unroll
    for (int a = 0; a < MF; ++a) {
      const int row = wr * MF * 16 + 16 * a + (lane & 15);
      if (!RCONT) {
        av[a] = cur[swz32(row, kq)];
      } else {
        // complex (k, row) at k * RT + 2 ((row / 2) ^ c32d_asw(k)) + row % 2; k = 2 kq, 2 kq + 1
        const float2* la = reinterpret_cast<const float2*>(cur);
        const int ra = 2 * ((row >> 1) ^ c32d_asw(2 * kq)) + (row & 1);  // same XOR for both k rows
        const float2 a0 = la[(2 * kq) * RT + ra], a1 = la[(2 * kq + 1) * RT + ra];
        av[a] = make_float4(a0.x, a0.y, a1.x, a1.y);
      }
    }
    // K entries of this lane: complex k = 8 c + 2 kq (+1); activation rows past kvalid are zero
    const bool k0ok = 8 * c + 2 * kq < p.kvalid, k1ok = 8 * c + 2 * kq + 1 < p.kvalid;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const int rl = wc * NF * 8 + f * 8 + ((lane & 15) >> 1);
      const int xs = 2 * ((rl >> 1) ^ c32d_xsw<NRT>(2 * kq)) + (rl & 1);  // same XOR for rows 2 kq, 2 kq + 1
      float2 x0 = lx[(2 * kq) * NRT + xs];
      float2 x1 = lx[(2 * kq + 1) * NRT + xs];
      if (!k0ok) x0 = make_float2(0.f, 0.f);
      if (!k1ok) x1 = make_float2(0.f, 0.f);
      float bv[4];
      embed32<CONJ>(x0, ci, dc, bv[0], bv[1]);
      embed32<CONJ>(x1, ci, dc, bv[2], bv[3]);
#pragma unroll
      for (int a = 0; a < MF; ++a) {
        acc[a][f] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a].x, bv[0], acc[a][f], 0, 0, 0);
        acc[a][f] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a].y, bv[1], acc[a][f], 0, 0, 0);
        acc[a][f] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a].z, bv[2], acc[a][f], 0, 0, 0);
        acc[a][f] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a].w, bv[3], acc[a][f], 0, 0, 0);
      }
    }
  };
  // chunk c is read from stage (c - c0) % NS, which is then refilled with chunk c + NS - 1
  // after the next barrier; every chunk issues its copies so that the count in flight is the
  // same on every path (the wait counts below rely on it)
  if (c0 < c1) {
    issue(c0, st0);
    if (NS > 2) issue(c0 + 1, st1);
    if (NS > 3) issue(c0 + 2, st2);
#define S2W_C32D_STEP(K, CUR, NEXT)                                     \
  do {                                                                  \
    __builtin_amdgcn_s_waitcnt(0x0F70 | PENDING);                       \
    asm volatile("" ::: "memory");                                      \
    __builtin_amdgcn_s_barrier();                                       \
    asm volatile("" ::: "memory");                                      \
    issue((K) + NS - 1, NEXT);                                          \
    if ((K) < c1) compute((K), CUR);                                    \
  } while (0)
    for (int k0 = c0; k0 < c1; k0 += NS) {
      if (NS == 2) {
        S2W_C32D_STEP(k0, st0, st1);
        S2W_C32D_STEP(k0 + 1, st1, st0);
      } else if (NS == 3) {
        S2W_C32D_STEP(k0, st0, st2);
        S2W_C32D_STEP(k0 + 1, st1, st0);
        S2W_C32D_STEP(k0 + 2, st2, st1);
      } else {
        S2W_C32D_STEP(k0, st0, st3);
        S2W_C32D_STEP(k0 + 1, st1, st0);
        S2W_C32D_STEP(k0 + 2, st2, st1);
        S2W_C32D_STEP(k0 + 3, st3, st2);
      }
    }
#undef S2W_C32D_STEP
  }
  // no copy into LDS may still be in flight when the workgroup ends
  __builtin_amdgcn_s_waitcnt(0);
  float* ow = p.out + (int64_t)split * p.o_split + (int64_t)l * p.o_slot;
#pragma unroll
  for (int a = 0; a < MF; ++a)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = row0 + wr * MF * 16 + 16 * a + 4 * kq + r;
      if (row >= p.nrows) continue;
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const int n = 2 * b0 + wc * NF * 16 + 16 * f + (lane & 15);
        if (n < p.ncols) ow[(int64_t)row * p.o_row + n] = acc[a][f][r];
      }
    }
}

// Tile shapes (rows x ruptures): 0: 64 x 128, 1: 128 x 32, 2: 256 x 8, 3: 64 x 64.
int cgemm32_rows(int cfg) { return cfg == 0 ? 64 : cfg == 1 ? 128 : cfg == 2 ? 256 : 64; }
int cgemm32_ruptures(int cfg) { return cfg == 0 ? 128 : cfg == 1 ? 32 : cfg == 2 ? 8 : 64; }

template <bool RCONT, bool CONJ>
static void cgemm32d_dispatch(int cfg, dim3 grid, hipStream_t st, const CGemmArgs& a) {
  switch (cfg) {
    case 0: hipLaunchKernelGGL((k_cgemm32d<2, 8, 2, 2, 3, RCONT, CONJ>), grid, dim3(256), 0, st, a); break;
    case 1: hipLaunchKernelGGL((k_cgemm32d<4, 2, 2, 2, 3, RCONT, CONJ>), grid, dim3(256), 0, st, a); break;
    case 2: hipLaunchKernelGGL((k_cgemm32d<4, 1, 4, 1, 4, RCONT, CONJ>), grid, dim3(256), 0, st, a); break;
    default: hipLaunchKernelGGL((k_cgemm32d<2, 4, 2, 2, 3, RCONT, CONJ>), grid, dim3(256), 0, st, a); break;
  }
}

hipError_t launch_cgemm32(int cfg, bool rcont, bool conj, const float2* A, int64_t a_row, int64_t a_k,
                          int64_t a_slot, int nrows, int rows_alloc, int kvalid, int kpad, const float2* X,
                          int64_t x_k, int64_t x_slot, int xk_alloc, int B, int bp, float* out, int64_t o_row,
                          int64_t o_slot, int64_t o_split, int M, int splits, hipStream_t st) {
  if (cfg < 0 || cfg > 3 || (M & 7) || (bp & 1) || bp < 2 || kpad % 8 || splits < 1) return hipErrorInvalidValue;
  if (rcont && (rows_alloc < 2 || (rows_alloc & 1))) return hipErrorInvalidValue;
  CGemmArgs a;
  a.A = A;
  a.a_row = a_row;
  a.a_k = a_k;
  a.a_slot = a_slot;
  a.nrows = nrows;
  a.rows_alloc = rows_alloc;
  a.kvalid = kvalid;
  a.nchunks = kpad / 8;
  a.X = X;
  a.x_k = x_k;
  a.x_slot = x_slot;
  a.xk_alloc = xk_alloc;
  a.bp = bp;
  a.out = out;
  a.o_row = o_row;
  a.o_slot = o_slot;
  a.o_split = o_split;
  a.ncols = 2 * B;
  a.M = M;
  a.nrt = (nrows + cgemm32_rows(cfg) - 1) / cgemm32_rows(cfg);
  a.nct = (B + cgemm32_ruptures(cfg) - 1) / cgemm32_ruptures(cfg);
  a.splits = splits;
  const int64_t blocks = (int64_t)M * a.nrt * a.nct * splits;
  if (blocks <= 0 || blocks > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 grid((unsigned)blocks);
  if (!rcont && !conj) cgemm32d_dispatch<false, false>(cfg, grid, st, a);
  else if (!rcont && conj) cgemm32d_dispatch<false, true>(cfg, grid, st, a);
  else if (rcont && !conj) cgemm32d_dispatch<true, false>(cfg, grid, st, a);
  else cgemm32d_dispatch<true, true>(cfg, grid, st, a);
  return hipGetLastError();
}

}  // namespace s2w
