// Batched path on the matrix cores: per-bin complex GEMMs with half-precision operators.
//
// Half-precision stores (HT = 1: bfloat16, HT = 2: float16), one 32-bit word per complex
// value (low half = real part, high half = imaginary part):
//   Gq            elastic spectra G[g][l][j], j padded to nsq (a multiple of 16, zeros), stored
//                 row-block-major: Gq[l][g/16][j/16][g%16][j%16], so that the 16 x 16 block of
//                 one K step of 16 grid rows is 1 KB of contiguous memory (grid rows padded to
//                 a multiple of 16)
//   Fq[l][o][g]   acoustic spectra, o padded to noq (multiple of 16), g padded to ngq (multiple of 16)
//   sG[g][l], sF[g][l]  float32 power-of-two scales: true value = scale * stored value
//
// A complex product sum_k A_k B_k is carried on real matrix cores by embedding each complex
// operand value a = ar + i ai as the two K entries (ar, ai) and each complex activation value
// b = br + i bi as the 2x2 block [[br, bi], [-bi, br]] (rows: K entries ar, ai; columns: real
// and imaginary output).  Slot 0 packs the two real bins (0 and L/2) and uses
// [[b0, 0], [0, bN]] instead.  Activations are split into a high and a low half-precision
// term (H = 2) so that their rounding stays below the operator's; products accumulate in
// float32.
//
// MFMA v_mfma_f32_16x16x32 (bf16/f16) fragments, lane l of 64:
//   A (16 x 32): row l%16, K entries 8*(l/16) .. +7      (16 bytes, 4 complex operand values)
//   B (32 x 16): column l%16, K entries 8*(l/16) .. +7
//   D (16 x 16): column l%16, rows 4*(l/16) .. +3        (4 floats)
#include <algorithm>

#include "s2w_half.h"
#include "s2w_internal.h"

namespace s2w {

// ---------------------------------------------------------------------------------------------
// Setup: quantize rows of float32 spectra.  staging[r][l][c] (complex, c < ncp stored, c < nc
// valid) -> out + (row0 + r)*sg + l*sl + c*sc (32-bit words), scale[(row0 + r)*M + l].
// One block per (r, l): the scale is a power of two mapping the row's largest |re|, |im| into
// [2^14, 2^15).
template <int HT>
__global__ __launch_bounds__(256) void k_quant_rows(const float2* __restrict__ staging, int M, int nc, int ncp,
                                                    uint32_t* __restrict__ out, int64_t row0, int64_t sg, int64_t sl,
                                                    int64_t sc, float* __restrict__ scale, int ng16) {
  __shared__ float red[256];
  const int r = blockIdx.x / M, l = blockIdx.x % M;
  const float2* row = staging + ((int64_t)r * M + l) * ncp;
  float mx = 0.f;
  for (int c = threadIdx.x; c < nc; c += 256) {
    const float2 v = row[c];
    mx = fmaxf(mx, fmaxf(fabsf(v.x), fabsf(v.y)));
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  float up, down;
  pow2_scale(red[0], up, down);
  const int64_t g = row0 + r;
  if (threadIdx.x == 0) scale[g * M + l] = down;
  if (ng16 > 0) {
    // row-block-major store: word (((l * ng16 + g / 16) * (ncp / 16) + c / 16) * 16 + g % 16) * 16 + c % 16
    uint32_t* o = out + (((int64_t)l * ng16 + (g >> 4)) * (ncp >> 4) * 16 + (g & 15)) * 16;
    for (int c = threadIdx.x; c < ncp; c += 256) {
      const float2 v = c < nc ? row[c] : make_float2(0.f, 0.f);
      o[(int64_t)(c >> 4) * 256 + (c & 15)] = pack_half2<HT>(v.x * up, v.y * up);
    }
    return;
  }
  uint32_t* o = out + g * sg + (int64_t)l * sl;
  for (int c = threadIdx.x; c < ncp; c += 256) {
    const float2 v = c < nc ? row[c] : make_float2(0.f, 0.f);
    o[(int64_t)c * sc] = to_half_bits<HT>(v.x * up) | (to_half_bits<HT>(v.y * up) << 16);
  }
}

hipError_t launch_quant_rows(int ht, const float2* staging, int64_t nrows, int M, int nc, int ncp, uint32_t* out,
                             int64_t row0, int64_t sg, int64_t sl, int64_t sc, float* scale, int ng16, hipStream_t st) {
  if (nrows == 0) return hipSuccess;
  if (ng16 > 0 && (ncp % 16)) return hipErrorInvalidValue;
  dim3 grid((unsigned)(nrows * M));
  if (ht == 1)
    hipLaunchKernelGGL(k_quant_rows<1>, grid, dim3(256), 0, st, staging, M, nc, ncp, out, row0, sg, sl, sc, scale,
                       ng16);
  else
    hipLaunchKernelGGL(k_quant_rows<2>, grid, dim3(256), 0, st, staging, M, nc, ncp, out, row0, sg, sl, sc, scale,
                       ng16);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Activation scales: sig[l][b] = power of two mapping max_j |S[l][j][b]| (re, im) into
// [2^14, 2^15) (the inverse is applied to the GEMM result).  S is [l][nsq][bp] complex.
// Workgroup of 16 columns (l, b..b+15) x 16 row groups: thread (jg, c) takes rows j = jg, jg +
// 16, ... of column c (consecutive threads read consecutive columns), then the 16 partial maxima
// of a column are combined in LDS.  Columns b >= B get unit scales.
__global__ __launch_bounds__(256) void k_act_scale(const float2* __restrict__ S, int M, int nsub, int nsq, int B,
                                                   int bp, float* __restrict__ sig_up, float* __restrict__ sig_down) {
  __shared__ float part[16][17];
  const int c = threadIdx.x & 15, jg = threadIdx.x >> 4;
  const int64_t col = (int64_t)blockIdx.x * 16 + c;  // l * bp + b
  const bool inb = col < (int64_t)M * bp;
  const int l = inb ? (int)(col / bp) : 0, b = inb ? (int)(col - (int64_t)l * bp) : 0;
  float mx = 0.f;
  if (inb && b < B)
    for (int j = jg; j < nsub; j += 16) {
      const float2 v = S[((int64_t)l * nsq + j) * bp + b];
      mx = fmaxf(mx, fmaxf(fabsf(v.x), fabsf(v.y)));
    }
  part[jg][c] = mx;
  __syncthreads();
  if (jg == 0 && inb) {
#pragma unroll
    for (int k = 1; k < 16; ++k) mx = fmaxf(mx, part[k][c]);
    float up, down;
    pow2_scale(mx, up, down);
    sig_up[col] = up;
    sig_down[col] = down;
  }
}

// B operand of the elastic GEMM in fragment order: Bop[l][ks][cb][h][lane] (16 bytes each).
// Column n = 16*cb + lane%16 is output (rupture n/2, real part if n even, imaginary if odd);
// K entry k = 8*(lane/16) + e covers subfault j = 16*ks + k/2, component k&1.
template <int HT, int H>
__global__ __launch_bounds__(256) void k_prep_act(const float2* __restrict__ S, const float* __restrict__ sig_up,
                                                  int M, int nsub, int nsq, int B, int bp, int nks, int ncb,
                                                  uint4* __restrict__ Bop) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t total = (int64_t)M * nks * ncb * 64;
  if (i >= total) return;
  const int lane = (int)(i & 63);
  int64_t q = i >> 6;
  const int cb = (int)(q % ncb);
  q /= ncb;
  const int ks = (int)(q % nks);
  const int l = (int)(q / nks);
  const int n = 16 * cb + (lane & 15);
  const int b = n >> 1, c = n & 1;
  const bool dc = (l == 0);
  uint32_t hi[4], lo[4];
#pragma unroll
  for (int e2 = 0; e2 < 4; ++e2) {
    const int j = 16 * ks + 4 * (lane >> 4) + e2;
    float2 s = make_float2(0.f, 0.f);
    if (b < B && j < nsub) {
      s = S[((int64_t)l * nsq + j) * bp + b];
      const float u = sig_up[(int64_t)l * bp + b];
      s.x *= u;
      s.y *= u;
    }
    // K entries (re component a = 0, im component a = 1) for this output column
    float v0, v1;
    if (dc) {
      v0 = c == 0 ? s.x : 0.f;
      v1 = c == 0 ? 0.f : s.y;
    } else {
      v0 = c == 0 ? s.x : s.y;
      v1 = c == 0 ? -s.y : s.x;
    }
    const uint32_t h0 = to_half_bits<HT>(v0), h1 = to_half_bits<HT>(v1);
    hi[e2] = h0 | (h1 << 16);
    if (H == 2) {
      const uint32_t l0 = to_half_bits<HT>(v0 - from_half_bits<HT>(h0));
      const uint32_t l1 = to_half_bits<HT>(v1 - from_half_bits<HT>(h1));
      lo[e2] = l0 | (l1 << 16);
    }
  }
  uint4* dst = Bop + (((int64_t)l * nks + ks) * ncb + cb) * H * 64 + lane;
  dst[0] = make_uint4(hi[0], hi[1], hi[2], hi[3]);
  if (H == 2) dst[64] = make_uint4(lo[0], lo[1], lo[2], lo[3]);
}

// Unit scales: bfloat16 activations keep float32's exponent range, so they are split without
// a range scale (scaling by a power of two would change no rounding).
__global__ __launch_bounds__(256) void k_unit_scale(int64_t n, float* __restrict__ sig_up, float* __restrict__ sig_down) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) {
    sig_up[i] = 1.f;
    sig_down[i] = 1.f;
  }
}

hipError_t launch_prep_act(int ht, int hterms, const float2* S, float* sig_up, float* sig_down, int M, int nsub,
                           int nsq, int B, int bp, int nks, int ncb, uint4* Bop, hipStream_t st) {
  const int64_t ns = (int64_t)M * bp;
  if (ht == 1)
    hipLaunchKernelGGL(k_unit_scale, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, st, ns, sig_up, sig_down);
  else
    hipLaunchKernelGGL(k_act_scale, dim3((unsigned)((ns + 15) / 16)), dim3(256), 0, st, S, M, nsub, nsq, B, bp,
                       sig_up, sig_down);
  const int64_t total = (int64_t)M * nks * ncb * 64;
  dim3 grid((unsigned)((total + 255) / 256));
#define S2W_PREP(HT_, H_) \
  hipLaunchKernelGGL((k_prep_act<HT_, H_>), grid, dim3(256), 0, st, S, sig_up, M, nsub, nsq, B, bp, nks, ncb, Bop)
  if (ht == 1 && hterms == 2) S2W_PREP(1, 2);
  else if (ht == 2 && hterms == 1) S2W_PREP(2, 1);
  else return hipErrorInvalidValue;
#undef S2W_PREP
  return hipGetLastError();
}

// Real-column activation fragments: Bre[l][ks][rcb][h][lane] (16 bytes each) hold only the
// real-part output column of rupture 16*rcb + lane%16 (K entries (Re s, -Im s) of subfaults
// 16*ks + 4*(lane/16) .. +3; slot 0: (Re s, Im s)).  The imaginary-part column (Im s, Re s)
// (slot 0: (0, Im s)) is formed from it in registers, so the store and its copies are half the
// size of Bop.  The words equal those of k_prep_act for the same columns.
template <int HT, int H>
__global__ __launch_bounds__(256) void k_prep_act_re(const float2* __restrict__ S, const float* __restrict__ sig_up,
                                                     int M, int nsub, int nsq, int B, int bp, int nks, int nrcb,
                                                     uint4* __restrict__ Bre) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t total = (int64_t)M * nks * nrcb * 64;
  if (i >= total) return;
  const int lane = (int)(i & 63);
  int64_t q = i >> 6;
  const int rcb = (int)(q % nrcb);
  q /= nrcb;
  const int ks = (int)(q % nks);
  const int l = (int)(q / nks);
  const int b = 16 * rcb + (lane & 15);
  const bool dc = (l == 0);
  uint32_t hi[4], lo[4];
#pragma unroll
  for (int e2 = 0; e2 < 4; ++e2) {
    const int j = 16 * ks + 4 * (lane >> 4) + e2;
    float2 s = make_float2(0.f, 0.f);
    if (b < B && j < nsub) {
      s = S[((int64_t)l * nsq + j) * bp + b];
      const float u = sig_up[(int64_t)l * bp + b];
      s.x *= u;
      s.y *= u;
    }
    const float v0 = s.x, v1 = dc ? s.y : -s.y;
    const uint32_t h0 = to_half_bits<HT>(v0), h1 = to_half_bits<HT>(v1);
    hi[e2] = h0 | (h1 << 16);
    if (H == 2) {
      const uint32_t l0 = to_half_bits<HT>(v0 - from_half_bits<HT>(h0));
      const uint32_t l1 = to_half_bits<HT>(v1 - from_half_bits<HT>(h1));
      lo[e2] = l0 | (l1 << 16);
    }
  }
  uint4* dst = Bre + (((int64_t)l * nks + ks) * nrcb + rcb) * H * 64 + lane;
  dst[0] = make_uint4(hi[0], hi[1], hi[2], hi[3]);
  if (H == 2) dst[64] = make_uint4(lo[0], lo[1], lo[2], lo[3]);
}

hipError_t launch_prep_act_re(int ht, int hterms, const float2* S, float* sig_up, float* sig_down, int M, int nsub,
                              int nsq, int B, int bp, int nks, int nrcb, uint4* Bre, hipStream_t st) {
  const int64_t ns = (int64_t)M * bp;
  if (ht == 1)
    hipLaunchKernelGGL(k_unit_scale, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, st, ns, sig_up, sig_down);
  else
    hipLaunchKernelGGL(k_act_scale, dim3((unsigned)((ns + 15) / 16)), dim3(256), 0, st, S, M, nsub, nsq, B, bp,
                       sig_up, sig_down);
  const int64_t total = (int64_t)M * nks * nrcb * 64;
  dim3 grid((unsigned)((total + 255) / 256));
#define S2W_PREPR(HT_, H_) \
  hipLaunchKernelGGL((k_prep_act_re<HT_, H_>), grid, dim3(256), 0, st, S, sig_up, M, nsub, nsq, B, bp, nks, nrcb, Bre)
  if (ht == 1 && hterms == 2) S2W_PREPR(1, 2);
  else if (ht == 2 && hterms == 1) S2W_PREPR(2, 1);
  else return hipErrorInvalidValue;
#undef S2W_PREPR
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Elastic GEMM per bin (eq. 1, Alg. 2 step 3, batched):
//   U[g][l][b] = sG[g][l] * sig_down[l][b] * sum_j Gq[g][l][j] (x) Sq[l][j][b]
// Persistent and XCD-aware: workgroup w runs on XCD w % 8 (round-robin dispatch) and takes the
// tiles of bins l = w % 8 (mod 8), so the 32 workgroups of an XCD share one bin's activation
// in that XCD's L2.  Tile: MG = MW*WR grid rows x NG = NW*WC output columns; wave (wr, wc)
// owns MW x NW.
template <int HT, int H, int MW, int NW, int WR, int WC>
__global__ __launch_bounds__(64 * WR * WC, 1) void k_gemm_g(const uint4* __restrict__ Gq, const float* __restrict__ sG,
                                                            const uint4* __restrict__ Bop,
                                                            const float* __restrict__ sig_down, float* __restrict__ U,
                                                            int ngrid, int M, int nks, int ncb, int B, int bp, int nrb,
                                                            int nct) {
  constexpr int MF = MW / 16, NF = NW / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave / WC, wc = wave % WC;
  const int nwg = gridDim.x, w = blockIdx.x;
  const int nx = 8 < M ? 8 : M;  // bins are dealt to XCDs round-robin
  const int x = w % nx, wi = w / nx, nwx = (nwg - x + nx - 1) / nx;
  const int slots_x = (M - x + nx - 1) / nx;
  const int64_t per_slot = (int64_t)nrb * nct;
  const int64_t items = (int64_t)slots_x * per_slot;
  const int ng16 = (ngrid + 15) >> 4;
  for (int64_t it = wi; it < items; it += nwx) {
    const int l = x + nx * (int)(it / per_slot);
    const int64_t rem = it % per_slot;
    const int rb = (int)(rem / nct), ct = (int)(rem % nct);
    const int g0 = rb * MW * WR + wr * MW;
    const int cb0 = ct * NF * WC + wc * NF;
    f32x4 acc[MF][NF];
#pragma unroll
    for (int a = 0; a < MF; ++a)
#pragma unroll
      for (int b = 0; b < NF; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    const uint4* arow[MF];
#pragma unroll
    for (int a = 0; a < MF; ++a) {
      const int g = min(g0 + 16 * a + (lane & 15), ngrid - 1);
      arow[a] = gq_row(Gq, g, l, ng16, nks) + (lane >> 4);
    }
    const uint4* bb = Bop + (int64_t)l * nks * ncb * H * 64 + lane;
    const bool colok = cb0 < ncb;
#pragma unroll 2
    for (int ks = 0; ks < nks; ++ks) {
      uint4 av[MF], bv[NF][H];
#pragma unroll
      for (int a = 0; a < MF; ++a) av[a] = op_word<HT>(ntload(arow[a] + kGqStepU4 * ks));
#pragma unroll
      for (int b = 0; b < NF; ++b)
#pragma unroll
        for (int h = 0; h < H; ++h) {
          const int cb = min(cb0 + b, ncb - 1);
          bv[b][h] = bb[(((int64_t)ks * ncb + cb) * H + h) * 64];
        }
#pragma unroll
      for (int a = 0; a < MF; ++a)
#pragma unroll
        for (int b = 0; b < NF; ++b)
#pragma unroll
          for (int h = 0; h < H; ++h) acc[a][b] = mfma16<kActT<HT>>(av[a], bv[b][h], acc[a][b]);
    }
    if (!colok) continue;
#pragma unroll
    for (int a = 0; a < MF; ++a)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int g = g0 + 16 * a + 4 * (lane >> 4) + r;
        if (g >= ngrid) continue;
        const float sg = sG[(int64_t)g * M + l];
#pragma unroll
        for (int b = 0; b < NF; ++b) {
          const int n = 16 * (cb0 + b) + (lane & 15);
          const int rup = n >> 1;
          if (cb0 + b < ncb && rup < B)
            U[(((int64_t)g * M + l) * bp + rup) * 2 + (n & 1)] =
                acc[a][b][r] * sg * sig_down[(int64_t)l * bp + rup];
        }
      }
  }
}

// LDS slot of 16-byte chunk c (0..3) of operator-tile row r: the chunk index is XORed with
// bits 1-2 of the row so that the eight rows read together by a quarter wave fall into
// eight distinct 16-byte bank groups.
__device__ __forceinline__ int swz(int r, int c) { return r * 4 + (c ^ ((r >> 1) & 3)); }

// Elastic GEMM fed by direct global-to-LDS copies (global_load_lds_dwordx4): the same tile
// and wave arrangement as the register-staged tiles, but the operator and activation tiles of a K step
// travel from global memory to LDS without passing through registers, so NS stages can be in
// flight at once (NS - 1 K steps ahead of the matrix cores).  A copy instruction moves 1 KB
// per wave, lane p landing at byte 16*p of the wave's LDS target; for the operator tile the
// lanes are assigned so that this linear placement is the chunk-swizzled layout the fragment
// reads expect, and the activation blocks are already stored in fragment order.
// Copies of K step ks (clamped to the last step: copies past the end land in a stage that is
// never read) into `stage`; every wave issues PER_W of them.
template <int PER_W, int NWAVE>
__device__ __forceinline__ void g4_issue(const uint4* const* src, const int64_t* sstep, int ks, int nks, uint4* stage,
                                         int wave) {
  const int kc = min(ks, nks - 1);
#pragma unroll
  for (int q = 0; q < PER_W; ++q)
    __builtin_amdgcn_global_load_lds(src[q] + (int64_t)kc * sstep[q],
                                     (__attribute__((address_space(3))) void*)(stage + (wave + NWAVE * q) * 64), 16, 0,
                                     0);
}

// Wait for this wave's copies of the current step (at most the NS - 2 later steps' copies stay
// in flight), then a workgroup barrier without a memory fence; the empty asm statements keep
// the compiler from moving LDS accesses across it.
template <int PENDING>
__device__ __forceinline__ void g4_sync() {
  __builtin_amdgcn_s_waitcnt(0x0F70 | PENDING);
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

template <int HT, int H, int MF, int NF, int MW, int A_BLK, int WC>
__device__ __forceinline__ void g4_compute(const uint4* cur, f32x4 (&acc)[MF][NF], int wr, int wc, int lane) {
  const uint4* lb = cur + A_BLK * 64;
  if constexpr (HT == 3 && H == 1) {
    // converted bfloat16 words: fragment a + 1 is converted (12 vector ALU instructions) under
    // the NF products of fragment a, instead of all conversions ahead of all products; each
    // output still takes its products in the same order
    uint4 raw[MF], bv[NF];
#pragma unroll
    for (int a = 0; a < MF; ++a) raw[a] = cur[swz(wr * MW + 16 * a + (lane & 15), lane >> 4)];
#pragma unroll
    for (int b = 0; b < NF; ++b) bv[b] = lb[(wc * NF + b) * 64 + lane];
    uint4 av = op_word<3>(raw[0]);
    __builtin_amdgcn_sched_group_barrier(0x002, 12, 0);
#pragma unroll
    for (int a = 0; a < MF; ++a) {
      const uint4 nxt = op_word<3>(raw[a + 1 < MF ? a + 1 : a]);
#pragma unroll
      for (int b = 0; b < NF; ++b) acc[a][b] = mfma16<2>(av, bv[b], acc[a][b]);
      av = nxt;
#pragma unroll
      for (int b = 0; b < NF; ++b) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        if (a + 1 < MF) __builtin_amdgcn_sched_group_barrier(0x002, 12 / NF, 0);
      }
    }
    return;
  }
  uint4 av[MF];
#pragma unroll
  for (int a = 0; a < MF; ++a) av[a] = op_word<HT>(cur[swz(wr * MW + 16 * a + (lane & 15), lane >> 4)]);
#pragma unroll
  for (int b = 0; b < NF; ++b)
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const uint4 bv = lb[((wc * NF + b) * H + h) * 64 + lane];
#pragma unroll
      for (int a = 0; a < MF; ++a) acc[a][b] = mfma16<kActT<HT>>(av[a], bv, acc[a][b]);
    }
  (void)WC;
}

// Products of one K step from real-column fragments (layout of k_prep_act_re): for rupture
// block q of this wave, the stored fragment gives the real-part columns and, with its halves
// swapped and the new low half negated (slot 0: masked), the imaginary-part columns; tiles
// 2q and 2q + 1 of acc take them.  Every tile accumulates its terms in the same order as
// g4_compute does for the same output columns.
__device__ __forceinline__ uint32_t im_word(uint32_t w, bool dc) {
  return dc ? (w & 0xffff0000u) : (((w >> 16) | (w << 16)) ^ 0x8000u);
}

template <int HT, int H, int MF, int NF, int MW, int A_BLK, int WC>
__device__ __forceinline__ void g4_compute_re(const uint4* cur, f32x4 (&acc)[MF][NF], int wr, int wc, int lane,
                                              bool dc) {
  const uint4* lb = cur + A_BLK * 64;
  if constexpr (HT == 3 && H == 1) {
    // converted bfloat16 words, as in g4_compute: the real- and imaginary-column fragments
    // first, then fragment a + 1 converted under the products of fragment a
    uint4 raw[MF], re[NF / 2], im[NF / 2];
#pragma unroll
    for (int a = 0; a < MF; ++a) raw[a] = cur[swz(wr * MW + 16 * a + (lane & 15), lane >> 4)];
#pragma unroll
    for (int q = 0; q < NF / 2; ++q) {
      const uint4 w = lb[(wc * (NF / 2) + q) * 64 + lane];
      re[q] = dc ? make_uint4(w.x & 0xffffu, w.y & 0xffffu, w.z & 0xffffu, w.w & 0xffffu) : w;
      im[q] = make_uint4(im_word(w.x, dc), im_word(w.y, dc), im_word(w.z, dc), im_word(w.w, dc));
    }
    uint4 av = op_word<3>(raw[0]);
    __builtin_amdgcn_sched_group_barrier(0x002, 12 + 20 * (NF / 2), 0);
#pragma unroll
    for (int a = 0; a < MF; ++a) {
      const uint4 nxt = op_word<3>(raw[a + 1 < MF ? a + 1 : a]);
#pragma unroll
      for (int q = 0; q < NF / 2; ++q) {
        acc[a][2 * q] = mfma16<2>(av, re[q], acc[a][2 * q]);
        acc[a][2 * q + 1] = mfma16<2>(av, im[q], acc[a][2 * q + 1]);
      }
      av = nxt;
#pragma unroll
      for (int b = 0; b < NF; ++b) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        if (a + 1 < MF) __builtin_amdgcn_sched_group_barrier(0x002, 12 / NF, 0);
      }
    }
    return;
  }
  uint4 av[MF];
#pragma unroll
  for (int a = 0; a < MF; ++a) av[a] = op_word<HT>(cur[swz(wr * MW + 16 * a + (lane & 15), lane >> 4)]);
#pragma unroll
  for (int q = 0; q < NF / 2; ++q)
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const uint4 w = lb[((wc * (NF / 2) + q) * H + h) * 64 + lane];
      const uint4 re = dc ? make_uint4(w.x & 0xffffu, w.y & 0xffffu, w.z & 0xffffu, w.w & 0xffffu) : w;
      const uint4 im = make_uint4(im_word(w.x, dc), im_word(w.y, dc), im_word(w.z, dc), im_word(w.w, dc));
#pragma unroll
      for (int a = 0; a < MF; ++a) acc[a][2 * q] = mfma16<kActT<HT>>(av[a], re, acc[a][2 * q]);
#pragma unroll
      for (int a = 0; a < MF; ++a) acc[a][2 * q + 1] = mfma16<kActT<HT>>(av[a], im, acc[a][2 * q + 1]);
    }
  (void)WC;
}

// RE: the activation store is the real-column layout of k_prep_act_re (ncb then counts its
// 16-rupture blocks) and the imaginary-part columns are formed in registers.
template <int HT, int H, int MW, int NW, int NS, int WR, int WC, int MINB = 1, bool RE = false>
__global__ __launch_bounds__(64 * WR * WC, MINB) void k_gemm_g4(const uint4* __restrict__ Gq, const float* __restrict__ sG,
                                                    const uint4* __restrict__ Bop, const float* __restrict__ sig_down,
                                                    float* __restrict__ U, int ngrid, int M, int nks, int ncb, int B,
                                                    int bp, int nrb, int nct) {
  constexpr int MF = MW / 16, NF = NW / 16;
  constexpr int NWAVE = WR * WC;
  constexpr int RT = WR * MW;                // rows per tile
  constexpr int CBT = WC * NF;               // column blocks per tile
  constexpr int A_BLK = RT / 16;             // 1 KB copy blocks of the operator tile per K step
  constexpr int B_BLK = (RE ? CBT / 2 : CBT) * H;  // 1 KB copy blocks of the activation tile per K step
  static_assert(!RE || (NF % 2 == 0), "real-column fragments cover whole 16-rupture blocks");
  constexpr int NBLK = A_BLK + B_BLK;
  constexpr int PER_W = NBLK / NWAVE;        // copy instructions per wave per K step
  constexpr int STAGE = NBLK * 64;           // uint4 per stage
  constexpr int PENDING = (NS - 2) * PER_W;  // copies of later steps allowed in flight
  static_assert(NBLK % NWAVE == 0, "every wave issues the same number of copies per K step");
  static_assert(NS >= 2 && NS <= 4 && PENDING < 16, "stages and wait counts");
  // one LDS object per stage, so that the compiler can tell the stages apart when it orders
  // the fragment reads after the copies
  __shared__ uint4 st0[STAGE];
  __shared__ uint4 st1[STAGE];
  __shared__ uint4 st2[NS > 2 ? STAGE : 1];
  __shared__ uint4 st3[NS > 3 ? STAGE : 1];
  __shared__ float sg_s[RT];  // row scales of the tile for the epilogue
  static_assert(RT <= 64 * NWAVE, "one thread per tile row loads its scale");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave / WC, wc = wave % WC;
  const int nwg = gridDim.x, w = blockIdx.x;
  const int nx = 8 < M ? 8 : M;
  const int x = w % nx, wi = w / nx, nwx = (nwg - x + nx - 1) / nx;
  const int slots_x = (M - x + nx - 1) / nx;
  const int64_t per_slot = (int64_t)nrb * nct;
  const int64_t items = (int64_t)slots_x * per_slot;
  const int ng16 = (ngrid + 15) >> 4;
  // operator lanes: block row rr = lane/4, chunk c such that the linear LDS slot is swz(rr, c)
  const int a_rr = lane >> 2, a_c = (lane & 3) ^ ((a_rr >> 1) & 3);
  // start skew: every workgroup runs the same sequence of equal tiles, so without it all of them
  // reach their epilogue (the U stores of a tile) at the same moment; sixteen start offsets of
  // about 4 us spread those store bursts over the read stream of the other workgroups (0.3-0.4 ms
  // less per call at B = 256, tile 24, same box alternating).  Workgroups 2m and 2m + 1 of an
  // XCD, which take the two column tiles of the same operator rows, keep one offset, so that the
  // second still finds those rows in L2.  At most about 50 us.
  for (int i = 0; i < ((wi >> 1) & 15); ++i) __builtin_amdgcn_s_sleep(127);
  for (int64_t it = wi; it < items; it += nwx) {
    const int l = x + nx * (int)(it / per_slot);
    const int64_t rem = it % per_slot;
    const int rb = (int)(rem / nct), ct = (int)(rem % nct);
    const int g0 = rb * RT;
    const int cbt0 = ct * CBT;
    // per copy slot of this wave: global source at K step 0 and its stride per K step
    const uint4* src[PER_W];
    int64_t sstep[PER_W];
#pragma unroll
    for (int q = 0; q < PER_W; ++q) {
      const int blk = wave + NWAVE * q;
      if (blk < A_BLK) {
        const int g = min(g0 + 16 * blk + a_rr, ngrid - 1);
        src[q] = gq_row(Gq, g, l, ng16, nks) + a_c;
        sstep[q] = kGqStepU4;
      } else {
        const int j = blk - A_BLK;
        const int cb = min((RE ? cbt0 / 2 : cbt0) + j / H, ncb - 1), h = j % H;
        src[q] = Bop + (((int64_t)l * nks * ncb + cb) * H + h) * 64 + lane;
        sstep[q] = (int64_t)ncb * H * 64;
      }
    }
    f32x4 acc[MF][NF];
#pragma unroll
    for (int a = 0; a < MF; ++a)
#pragma unroll
      for (int b = 0; b < NF; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    // every copy of the previous item has landed and every wave is past its reads
    g4_sync<0>();
    g4_issue<PER_W, NWAVE>(src, sstep, 0, nks, st0, wave);
    if (NS > 2) g4_issue<PER_W, NWAVE>(src, sstep, 1, nks, st1, wave);
    if (NS > 3) g4_issue<PER_W, NWAVE>(src, sstep, 2, nks, st2, wave);
    // the tile's row scales, loaded under the K loop and passed through LDS to the epilogue
    const float sgv = tid < RT ? sG[(int64_t)min(g0 + tid, ngrid - 1) * M + l] : 0.f;
    // step ks reads stage ks % NS and refills stage (ks - 1) % NS with step ks + NS - 1; every
    // step issues its copies so that the count in flight is the same on every path
#define S2W_G4_STEP(K, CUR, NEXT)                                      \
  do {                                                                  \
    g4_sync<PENDING>();                                                 \
    g4_issue<PER_W, NWAVE>(src, sstep, (K) + NS - 1, nks, NEXT, wave);  \
    if ((K) < nks) {                                                  \
      if (RE) g4_compute_re<HT, H, MF, NF, MW, A_BLK, WC>(CUR, acc, wr, wc, lane, l == 0); \
      else g4_compute<HT, H, MF, NF, MW, A_BLK, WC>(CUR, acc, wr, wc, lane); \
    }                                                                   \
  } while (0)
    for (int k0 = 0; k0 < nks; k0 += NS) {
      if (NS == 2) {
        S2W_G4_STEP(k0, st0, st1);
        S2W_G4_STEP(k0 + 1, st1, st0);
      } else if (NS == 3) {
        S2W_G4_STEP(k0, st0, st2);
        S2W_G4_STEP(k0 + 1, st1, st0);
        S2W_G4_STEP(k0 + 2, st2, st1);
      } else {
        S2W_G4_STEP(k0, st0, st3);
        S2W_G4_STEP(k0 + 1, st1, st0);
        S2W_G4_STEP(k0 + 2, st2, st1);
        S2W_G4_STEP(k0 + 3, st3, st2);
      }
    }
#undef S2W_G4_STEP
    // epilogue: U[g][l][rup][c] = acc * sG[g][l] * sig_down[l][rup].  Column scales, validity
    // and offsets are per lane and column block, so each row takes one address computation and
    // its stores use constant offsets from it; with RE the real and imaginary part of a rupture
    // sit in one lane and go out as one 8-byte store.
    float sdn[NF];
    bool cok[NF];
    // first output float of this lane's column block 0, relative to the row's start
    const int rup0 = RE ? 16 * (cbt0 / 2 + wc * (NF / 2)) + (lane & 15) : (16 * (cbt0 + wc * NF) + (lane & 15)) >> 1;
    const int c0 = RE ? 0 : (lane & 1);
#pragma unroll
    for (int b = 0; b < NF; ++b) {
      const int blk = RE ? cbt0 / 2 + wc * (NF / 2) + (b >> 1) : cbt0 + wc * NF + b;
      const int rup = RE ? rup0 + 16 * (b >> 1) : rup0 + 8 * b;
      cok[b] = blk < ncb && rup < B;
      sdn[b] = cok[b] ? sig_down[(int64_t)l * bp + rup] : 0.f;
    }
    float* colp = U + ((int64_t)l * bp + rup0) * 2 + c0;
    const int64_t row_stride = (int64_t)M * bp * 2;
    // every wave read sg_s of the previous tile before the barrier at this tile's start
    if (tid < RT) sg_s[tid] = sgv;
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): the scale is in LDS
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
#pragma unroll
    for (int a = 0; a < MF; ++a)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gt = wr * MW + 16 * a + 4 * (lane >> 4) + r;  // row within the tile
        const int g = g0 + gt;
        if (g >= ngrid) continue;
        const float sg = sg_s[gt];
        float* p = colp + (int64_t)g * row_stride;
#pragma unroll
        for (int b = 0; b < NF; ++b) {
          if (RE) {
            if ((b & 1) == 0 && cok[b])
              *reinterpret_cast<float2*>(p + 32 * (b >> 1)) =
                  make_float2(acc[a][b][r] * sg * sdn[b], acc[a][b + 1][r] * sg * sdn[b]);
          } else {
            if (cok[b]) p[16 * b] = acc[a][b][r] * sg * sdn[b];
          }
        }
      }
  }
  // no copy into LDS may still be in flight when the workgroup ends
  __builtin_amdgcn_s_waitcnt(0);
}

template <int HT, int H>
static hipError_t gemm_g_h(int cfg, const uint4* Gq, const float* sG, const uint4* Bop, const float* sig_down,
                           float* U, int nwg, int ngrid, int M, int nks, int ncb, int B, int bp, hipStream_t st) {
  switch (cfg) {
    case 0: {
      // narrow batches: register tile of 64 rows x 16 columns per wave, four waves down
      const int nrb = (ngrid + 255) / 256;
      const int nct = ncb;
      hipLaunchKernelGGL((k_gemm_g<HT, H, 64, 16, 4, 1>), dim3(nwg), dim3(256), 0, st, Gq, sG, Bop, sig_down, U, ngrid, M,
                         nks, ncb, B, bp, nrb, nct);
      break;
    }
    case 17:
    case 18: {
      // 256 x 256 tiles on real-column activation fragments (k_prep_act_re): 17 with four
      // stages of 32 KB, 18 with three
      const int nrcb = (B + 15) / 16;
      const int nrb = (ngrid + 255) / 256;
      const int nct = (nrcb + 7) / 8;
      if (cfg == 17)
        hipLaunchKernelGGL((k_gemm_g4<HT, H, 128, 64, 4, 2, 4, 1, true>), dim3(nwg), dim3(512), 0, st, Gq, sG, Bop,
                           sig_down, U, ngrid, M, nks, nrcb, B, bp, nrb, nct);
      else
        hipLaunchKernelGGL((k_gemm_g4<HT, H, 128, 64, 3, 2, 4, 1, true>), dim3(nwg), dim3(512), 0, st, Gq, sG, Bop,
                           sig_down, U, ngrid, M, nks, nrcb, B, bp, nrb, nct);
      break;
    }
    case 24: {
      // 256 x 256 tiles with wave tiles of 64 rows x 128 columns (waves 4 x 2): half the
      // operator fragments per wave of tile 10, so half the conversions of bfloat16 words
      const int nrb = (ngrid + 255) / 256;
      const int nct = (ncb + 15) / 16;
      hipLaunchKernelGGL((k_gemm_g4<HT, H, 64, 128, 3, 4, 2>), dim3(nwg), dim3(512), 0, st, Gq, sG, Bop, sig_down, U,
                         ngrid, M, nks, ncb, B, bp, nrb, nct);
      break;
    }
    case 10:
    case 12: {
      // direct-to-LDS copies, eight waves: 10 = 256 x 256 (three stages), 12 = 256 x 128 (four stages)
      const int NW = cfg == 12 ? 32 : 64;
      const int nrb = (ngrid + 255) / 256;
      const int nct = (ncb + 4 * (NW / 16) - 1) / (4 * (NW / 16));
      if (cfg == 10)
        hipLaunchKernelGGL((k_gemm_g4<HT, H, 128, 64, 3, 2, 4>), dim3(nwg), dim3(512), 0, st, Gq, sG, Bop, sig_down,
                           U, ngrid, M, nks, ncb, B, bp, nrb, nct);
      else
        hipLaunchKernelGGL((k_gemm_g4<HT, H, 128, 32, 4, 2, 4>), dim3(nwg), dim3(512), 0, st, Gq, sG, Bop, sig_down,
                           U, ngrid, M, nks, ncb, B, bp, nrb, nct);
      break;
    }
    case 16: {
      // direct-to-LDS copies, four waves of 128 x 64, two stages, two workgroups per compute unit
      const int nrb = (ngrid + 255) / 256;
      const int nct = (ncb + 7) / 8;
      hipLaunchKernelGGL((k_gemm_g4<HT, H, 128, 64, 2, 2, 2, 2>), dim3(2 * nwg), dim3(256), 0, st, Gq, sG, Bop,
                         sig_down, U, ngrid, M, nks, ncb, B, bp, nrb, nct);
      break;
    }
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_gemm_g(int ht, int hterms, int cfg, const uint4* Gq, const float* sG, const uint4* Bop,
                         const float* sig_down, float* U, int nwg, int ngrid, int M, int nks, int ncb, int B, int bp,
                         hipStream_t st) {
  // operand pairs of the plans: bf16 words with two bf16 activation terms, f16 words with one
  // f16 term, bf16 words converted to f16 with one f16 term
  if (ht == 1 && hterms == 2) return gemm_g_h<1, 2>(cfg, Gq, sG, Bop, sig_down, U, nwg, ngrid, M, nks, ncb, B, bp, st);
  if (ht == 2 && hterms == 1) return gemm_g_h<2, 1>(cfg, Gq, sG, Bop, sig_down, U, nwg, ngrid, M, nks, ncb, B, bp, st);
  if (ht == 3 && hterms == 1) return gemm_g_h<3, 1>(cfg, Gq, sG, Bop, sig_down, U, nwg, ngrid, M, nks, ncb, B, bp, st);
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------------------------
// Fragment word of the 2x2 embedding for output column parity c (0 real, 1 imaginary) from a
// packed (re | im << 16) word; dc selects the packed real slot.
__device__ __forceinline__ uint32_t embed_word(uint32_t w, int c, bool dc) {
  if (dc) return c == 0 ? (w & 0xffffu) : (w & 0xffff0000u);
  return c == 0 ? (w ^ 0x80000000u) : ((w >> 16) | (w << 16));
}

// Acoustic GEMM, LDS-staged, for the packed bfloat16 activation: workgroup (l, split, column
// tile) of four waves; per K step (16 grid rows) the operator tile (noq observers x 64 bytes,
// chunk-swizzled) and the activation tile (16 rows x NR ruptures x 8 bytes, rows padded by 64
// bytes) are double-buffered in LDS, the next step's tiles loaded while the matrix cores
// consume the current ones.
template <int MF, int NF>
__global__ __launch_bounds__(256, 2) void k_gemm_f2(const uint4* __restrict__ Fq, const uint2* __restrict__ V,
                                                    float* __restrict__ part, int ngrid, int ngq, int M, int noq,
                                                    int B, int bp) {
  constexpr int NR = 4 * NF * 8;            // ruptures per tile
  constexpr int LDB = NR + 8;               // padded LDS row (uint2)
  constexpr int A_U4 = MF * 16 * 4;         // operator tile uint4
  constexpr int B_U4 = 16 * NR / 2;         // activation tile uint4
  constexpr int T_U4 = A_U4 + B_U4;
  constexpr int PER_T = (T_U4 + 255) / 256;
  constexpr int LDS_A = A_U4, LDS_B = 16 * LDB / 2;
  __shared__ uint4 lds[2][LDS_A + LDS_B];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c = lane & 1;
  const int l = blockIdx.x;
  const bool dc = (l == 0);
  const int split = blockIdx.y, splits = gridDim.y;
  const int b0 = blockIdx.z * NR;
  const int nks = ngq / 16;
  const int kst0 = (int)((int64_t)nks * split / splits), kst1 = (int)((int64_t)nks * (split + 1) / splits);
  const int64_t frow = (int64_t)ngq / 4;  // uint4 per (l, o) row of Fq
  const uint4* src[PER_T];
  int64_t sstep[PER_T];
  bool valid[PER_T];
  int dst[PER_T];
#pragma unroll
  for (int k = 0; k < PER_T; ++k) {
    const int i = tid + 256 * k;
    valid[k] = i < T_U4;
    if (i < A_U4) {
      const int r = i >> 2, cc = i & 3;
      src[k] = Fq + ((int64_t)l * noq + r) * frow + 4 * kst0 + cc;
      sstep[k] = 4;
      dst[k] = swz(r, cc);
    } else {
      const int j = min(i - A_U4, B_U4 - 1);
      const int gl = j / (NR / 2), q = j % (NR / 2);
      const int bb = min(b0 + 2 * q, bp - 2);
      // rows past the grid read the last row; their operator entries are zero padding
      const int g = min(16 * kst0 + gl, ngrid - 1);
      src[k] = reinterpret_cast<const uint4*>(V + ((int64_t)g * M + l) * bp + bb);
      sstep[k] = 16 * (int64_t)M * bp / 2;
      dst[k] = LDS_A + (gl * LDB) / 2 + q;
      if (16 * kst0 + gl >= ngrid) sstep[k] = 0;
    }
  }
  f32x4 acc[MF][NF];
#pragma unroll
  for (int a = 0; a < MF; ++a)
#pragma unroll
    for (int b = 0; b < NF; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  if (kst0 < kst1) {
    uint4 stage[PER_T];
#pragma unroll
    for (int k = 0; k < PER_T; ++k)
      if (valid[k]) stage[k] = ntload(src[k]);
#pragma unroll
    for (int k = 0; k < PER_T; ++k)
      if (valid[k]) lds[0][dst[k]] = stage[k];
    __syncthreads();
    for (int ks = kst0; ks < kst1; ++ks) {
      const int cur = (ks - kst0) & 1;
      const bool more = ks + 1 < kst1;
      if (more) {
#pragma unroll
        for (int k = 0; k < PER_T; ++k) {
          if (!valid[k]) continue;
          // activation rows stop advancing past the last grid row (sstep is then zero, or the
          // row is clamped below)
          const uint4* pk = src[k] + (int64_t)(ks + 1 - kst0) * sstep[k];
          if (k * 256 + tid >= A_U4) {
            const int j = min(k * 256 + tid - A_U4, B_U4 - 1);
            const int gl = j / (NR / 2);
            if (16 * (ks + 1) + gl >= ngrid) {
              const int q = j % (NR / 2);
              const int bb = min(b0 + 2 * q, bp - 2);
              pk = reinterpret_cast<const uint4*>(V + ((int64_t)(ngrid - 1) * M + l) * bp + bb);
            }
          }
          stage[k] = ntload(pk);
        }
      }
      const uint4* la = &lds[cur][0];
      const uint2* lb = reinterpret_cast<const uint2*>(&lds[cur][LDS_A]);
      uint4 av[MF];
#pragma unroll
      for (int a = 0; a < MF; ++a) av[a] = la[swz(16 * a + (lane & 15), lane >> 4)];
#pragma unroll
      for (int b = 0; b < NF; ++b) {
        const int rl = wave * (NF * 8) + b * 8 + ((lane & 15) >> 1);
        uint32_t hw[4], lw[4];
#pragma unroll
        for (int e2 = 0; e2 < 4; ++e2) {
          const uint2 wv = lb[(4 * (lane >> 4) + e2) * LDB + rl];
          hw[e2] = embed_word(wv.x, c, dc);
          lw[e2] = embed_word(wv.y, c, dc);
        }
        const uint4 bh = make_uint4(hw[0], hw[1], hw[2], hw[3]);
        const uint4 bl = make_uint4(lw[0], lw[1], lw[2], lw[3]);
#pragma unroll
        for (int a = 0; a < MF; ++a) {
          acc[a][b] = mfma16<1>(av[a], bh, acc[a][b]);
          acc[a][b] = mfma16<1>(av[a], bl, acc[a][b]);
        }
      }
      if (more) {
#pragma unroll
        for (int k = 0; k < PER_T; ++k)
          if (valid[k]) lds[cur ^ 1][dst[k]] = stage[k];
      }
      __syncthreads();
    }
  }
  // part[split][l][o][n], n = 2*rupture + re/im
  float* pw = part + ((int64_t)split * M + l) * noq * (2 * bp);
#pragma unroll
  for (int a = 0; a < MF; ++a)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int o = 16 * a + 4 * (lane >> 4) + r;
#pragma unroll
      for (int b = 0; b < NF; ++b) {
        const int rup = b0 + wave * (NF * 8) + b * 8 + ((lane & 15) >> 1);
        if (rup < bp) pw[(int64_t)o * (2 * bp) + 2 * rup + c] = acc[a][b][r];
      }
    }
}

hipError_t launch_gemm_f2(const uint4* Fq, const uint2* V, float* part, int ngrid, int ngq, int M, int noq, int B,
                          int bp, int splits, hipStream_t st) {
  const int mf = noq / 16;
  const int nf = B > 64 ? 8 : 2;
  const int nr = 4 * nf * 8;
  dim3 grid(M, splits, (B + nr - 1) / nr);
#define S2W_F2(MF_, NF_) \
  hipLaunchKernelGGL((k_gemm_f2<MF_, NF_>), grid, dim3(256), 0, st, Fq, V, part, ngrid, ngq, M, noq, B, bp)
  if (nf == 8) {
    if (mf == 1) S2W_F2(1, 8); else if (mf == 2) S2W_F2(2, 8); else if (mf == 4) S2W_F2(4, 8);
    else return hipErrorInvalidValue;
  } else {
    if (mf == 1) S2W_F2(1, 2); else if (mf == 2) S2W_F2(2, 2); else if (mf == 4) S2W_F2(4, 2);
    else if (mf == 8) S2W_F2(8, 2);
    else return hipErrorInvalidValue;
  }
#undef S2W_F2
  return hipGetLastError();
}

hipError_t launch_act_scale(const float2* S, int M, int nk, int nkp, int B, int bp, float* sig_up, float* sig_down,
                            hipStream_t st) {
  const int64_t ns = (int64_t)M * bp;
  hipLaunchKernelGGL(k_act_scale, dim3((unsigned)((ns + 15) / 16)), dim3(256), 0, st, S, M, nk, nkp, B, bp, sig_up,
                     sig_down);
  return hipGetLastError();
}

// Column scales of the acoustic GEMM's activation (float16 operands only): for each (l, b),
// a power of two mapping max_g |V[g][l][b]| (re, im) into [2^14, 2^15).  First pass: partial
// maxima part[s][l][b] over grid-row ranges s (many workgroups, four loads in flight per
// thread); second pass: the maximum over the ranges and the scale.
__global__ __launch_bounds__(256) void k_col_max(const float2* __restrict__ V, int ngrid, int M, int B, int bp,
                                                 int splits, float* __restrict__ part) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int s = blockIdx.y;
  if (i >= (int64_t)M * bp) return;
  const int l = (int)(i / bp), b = (int)(i - (int64_t)l * bp);
  const int g0 = (int)((int64_t)ngrid * s / splits), g1 = (int)((int64_t)ngrid * (s + 1) / splits);
  float m0 = 0.f, m1 = 0.f, m2 = 0.f, m3 = 0.f;
  if (b < B) {
    const float2* v = V + (int64_t)l * bp + b;
    const int64_t gs = (int64_t)M * bp;
    int g = g0;
    for (; g + 4 <= g1; g += 4) {
      const float2 x0 = v[(int64_t)g * gs], x1 = v[(int64_t)(g + 1) * gs];
      const float2 x2 = v[(int64_t)(g + 2) * gs], x3 = v[(int64_t)(g + 3) * gs];
      m0 = fmaxf(m0, fmaxf(fabsf(x0.x), fabsf(x0.y)));
      m1 = fmaxf(m1, fmaxf(fabsf(x1.x), fabsf(x1.y)));
      m2 = fmaxf(m2, fmaxf(fabsf(x2.x), fabsf(x2.y)));
      m3 = fmaxf(m3, fmaxf(fabsf(x3.x), fabsf(x3.y)));
    }
    for (; g < g1; ++g) {
      const float2 x = v[(int64_t)g * gs];
      m0 = fmaxf(m0, fmaxf(fabsf(x.x), fabsf(x.y)));
    }
  }
  part[(int64_t)s * M * bp + i] = fmaxf(fmaxf(m0, m1), fmaxf(m2, m3));
}

__global__ __launch_bounds__(256) void k_col_scale_final(const float* __restrict__ part, int splits, int64_t n,
                                                         int B, int bp, float* __restrict__ tau_up,
                                                         float* __restrict__ tau_down) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  float mx = 0.f;
  if ((int)(i % bp) < B)
    for (int s = 0; s < splits; ++s) mx = fmaxf(mx, part[(int64_t)s * n + i]);
  float up, down;
  pow2_scale(mx, up, down);
  tau_up[i] = up;
  tau_down[i] = down;
}

hipError_t launch_col_scale(const float2* V, int ngrid, int M, int B, int bp, float* tau_up, float* tau_down,
                            float* part, int64_t part_floats, hipStream_t st) {
  const int64_t n = (int64_t)M * bp;
  const int64_t nblk = (n + 255) / 256;
  int splits = (int)std::max<int64_t>(1, std::min<int64_t>(64, 8192 / std::max<int64_t>(1, nblk)));
  splits = std::min(splits, std::max(1, ngrid));
  while (splits > 1 && (int64_t)splits * n > part_floats) --splits;
  if ((int64_t)splits * n > part_floats) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_col_max, dim3((unsigned)nblk, (unsigned)splits), dim3(256), 0, st, V, ngrid, M, B, bp, splits,
                     part);
  hipLaunchKernelGGL(k_col_scale_final, dim3((unsigned)nblk), dim3(256), 0, st, part, splits, n, B, bp, tau_up,
                     tau_down);
  return hipGetLastError();
}

hipError_t launch_col_scale_final(const float* part, int splits, int M, int B, int bp, float* tau_up, float* tau_down,
                                  hipStream_t st) {
  const int64_t n = (int64_t)M * bp;
  hipLaunchKernelGGL(k_col_scale_final, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, part, splits, n, B, bp,
                     tau_up, tau_down);
  return hipGetLastError();
}

// Zero 32-bit words: out[i * stride + k] for i < n, k < width.
__global__ __launch_bounds__(256) void k_zero_strided(uint32_t* __restrict__ out, int64_t n, int64_t stride, int width) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n * width) return;
  const int64_t r = i / width;
  out[r * stride + (i - r * width)] = 0u;
}

hipError_t launch_zero_strided(uint32_t* out, int64_t n, int64_t stride, int width, hipStream_t st) {
  const int64_t tot = n * width;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_strided, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, out, n, stride, width);
  return hipGetLastError();
}

// Sum the acoustic partials over splits, undo the activation scale, and lay the result out
// as rows yh[b][o][l] (complex) for the inverse transform.
__global__ __launch_bounds__(256) void k_sum_f(const float* __restrict__ part, int splits, int M, int noq, int nobs,
                                               int B, int bp, const float* __restrict__ tau_down, float2* __restrict__ yh) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;  // over (l, o, b)
  const int64_t total = (int64_t)M * nobs * B;
  if (i >= total) return;
  const int b = (int)(i % B);
  const int64_t q = i / B;
  const int o = (int)(q % nobs), l = (int)(q / nobs);
  float re = 0.f, im = 0.f;
  for (int s = 0; s < splits; ++s) {
    const float* p = part + (((int64_t)s * M + l) * noq + o) * (2 * bp) + 2 * b;
    re += p[0];
    im += p[1];
  }
  const float td = tau_down ? tau_down[(int64_t)l * bp + b] : 1.f;
  yh[((int64_t)b * nobs + o) * M + l] = make_float2(re * td, im * td);
}

hipError_t launch_sum_f(const float* part, int splits, int M, int noq, int nobs, int B, int bp, const float* tau_down,
                        float2* yh, hipStream_t st) {
  const int64_t total = (int64_t)M * nobs * B;
  hipLaunchKernelGGL(k_sum_f, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, part, splits, M, noq, nobs, B,
                     bp, tau_down, yh);
  return hipGetLastError();
}

}  // namespace s2w
