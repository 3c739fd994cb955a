// Adjoint of the batched half-precision path on the matrix cores: conjugate-transposed per-bin
// complex GEMMs over half-precision operator stores (the layouts and the complex embedding of
// the forward kernels, with conjugation folded into the operator's imaginary sign).
#include <algorithm>

#include "s2w_half.h"
#include "s2w_half_re.h"
#include "s2w_internal.h"

namespace s2w {

// ---------------------------------------------------------------------------------------------
// Conjugate-transposed half-precision GEMM per slot (the adjoint's per-bin products):
//   out(row, b) = rowscale(row, l) * down(l, b) * sum_k conj(A(k, row)) * up(l, b) * X(k, b)
// A is a half-precision store read transposed: A(k, row) at Aq + l*a_slot + (k/16)*a_k16 +
// (k%16)*a_k + (row/16)*a_r16 + row%16 (32-bit words re | im << 16; rows contiguous within
// blocks of 16); rows < rows_alloc are readable, k < kvalid are real.
// X is a complex64 activation X(k, b) at X + l*x_slot + k*x_k + b, split into H half terms in
// registers after the optional power-of-two scale up(l, b).  The operator tile of a K step (16
// k x RT rows) is staged through LDS (double-buffered) and read back as fragments of four
// consecutive k; conjugation flips the sign of the imaginary halves, except in the packed real
// slot 0 where the products are componentwise.  K may be split over workgroups (one partial
// per split, out + split*o_split).
struct TArgs {
  const uint32_t* Aq;
  int64_t a_slot, a_k16, a_k, a_r16;
  int nrows, rows_alloc, kvalid, nks;  // nks: K steps of 16 over the padded K range
  const float2* X;
  int64_t x_slot, x_k;
  int xk_alloc;
  const float* up;                     // [l][bp] or null
  const float* down;                   // [l][bp] or null
  const float* rowscale;               // rowscale[row * rs_row + l * rs_l] or null
  int64_t rs_row, rs_l;
  float* out;
  int64_t o_split, o_slot, o_row;      // float strides; column n = 2*b + (0 re, 1 im)
  int B, bp, nrt, nct, splits;
};

// word offset of A(k, row) within a slot (row a multiple of 4: four rows are contiguous)
__device__ __forceinline__ int64_t a_off(const TArgs& p, int k, int row) {
  return (int64_t)(k >> 4) * p.a_k16 + (int64_t)(k & 15) * p.a_k + (int64_t)(row >> 4) * p.a_r16 + (row & 15);
}

// Eight waves per workgroup, a 256-row x 32*NF-column tile (waves 4 x 2, each 64 rows x 16*NF
// columns).  Per K step of 16 both operands pass through LDS, double
// buffered with one barrier per step: the operator tile as [k][row] words, the activation
// converted once per workgroup into MFMA B fragments (H terms) by threads that each own four
// consecutive k of one rupture.  The next step's global loads are issued before the current
// step's matrix products.
template <int NF>
struct T2Geo {
  static constexpr int RT = 256, LDA = RT + 4, RB = 16 * NF;  // rows, LDS row words, ruptures per tile
  static constexpr int NCB = 2 * NF;                           // 16-column blocks per tile
};

// RE = true keeps only the real-column fragments in LDS (one granule per rupture and four k):
// off the DC bin the stored word is (x, -y) and the imaginary column (y, x) is that word with its
// halves swapped and the new low half negated; on the DC bin the stored word is (x, y) and the two
// columns are its halves masked.  Both columns are then the same bits as the RE = false layout
// converts, so the products and their accumulation order are unchanged, while the activation
// copies, LDS writes and LDS fragment reads halve.
template <int HT, int H, int NF, bool RE>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(NF <= 4 ? 4 : 2))) void k_gemm_t2(const TArgs p) {
  using Gm = T2Geo<NF>;
  constexpr int RT = Gm::RT, LDA = Gm::LDA, RB = Gm::RB, NCB = Gm::NCB;
  constexpr int MF = 4;
  constexpr int NBS = RE ? NCB / 2 : NCB;  // fragment blocks held in LDS per step
  __shared__ uint32_t la_s[2][16 * LDA];
  __shared__ uint4 lb_s[2][NBS * H * 64];
  __shared__ float rs_s[RT];  // row scales of the tile for the epilogue
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int x = blockIdx.x & 7, q = blockIdx.x >> 3;
  const int per_slot = p.nrt * p.nct * p.splits;
  const int l = x + 8 * (q / per_slot);
  int rem = q % per_slot;
  const int split = rem % p.splits;
  rem /= p.splits;
  const int ct = rem % p.nct, rt = rem / p.nct;
  const bool dc = (l == 0);
  const uint32_t cmask = dc ? 0u : 0x80000000u;
  const int ks0 = (int)((int64_t)p.nks * split / p.splits), ks1 = (int)((int64_t)p.nks * (split + 1) / p.splits);
  const int row0 = rt * RT;
  if (tid < RT)
    rs_s[tid] = p.rowscale ? p.rowscale[(int64_t)min(row0 + tid, p.nrows - 1) * p.rs_row + (int64_t)l * p.rs_l] : 1.f;
  __syncthreads();
  const uint32_t* Al = p.Aq + (int64_t)l * p.a_slot;
  const float2* Xl = p.X + (int64_t)l * p.x_slot;
  // activation ownership: granule slot s = tid + 512 * rep -> column block s / 64, lane s % 64
  constexpr int XSLOTS = NBS * 64, XREP = (XSLOTS + 511) / 512;
  int bx[XREP], xkg[XREP];
  float upx[XREP];
#pragma unroll
  for (int rp = 0; rp < XREP; ++rp) {
    const int s = min(tid + 512 * rp, XSLOTS - 1);
    const int L = s & 63;
    xkg[rp] = L >> 4;
    bx[rp] = RE ? min(ct * RB + 16 * (s >> 6) + (L & 15), p.bp - 1)
                : min(ct * RB + 8 * (s >> 6) + ((L & 15) >> 1), p.bp - 1);
    upx[rp] = p.up ? p.up[(int64_t)l * p.bp + bx[rp]] : 1.f;
  }
  f32x4 acc[MF][NF];
#pragma unroll
  for (int a = 0; a < MF; ++a)
#pragma unroll
    for (int f = 0; f < NF; ++f) acc[a][f] = f32x4{0.f, 0.f, 0.f, 0.f};
  uint4 ast[2];
  float2 xv[XREP][4];
  auto fetch = [&](int ks) {
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const int i = tid + 512 * it;  // 16 k x 64 row groups
      const int kk = i >> 6, rg = i & 63;
      const int k = 16 * ks + kk;
      const int row = min(row0 + 4 * rg, p.rows_alloc - 4);
      uint4 v = *reinterpret_cast<const uint4*>(Al + a_off(p, min(k, p.kvalid - 1), row));
      ast[it] = k < p.kvalid ? v : make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
    for (int rp = 0; rp < XREP; ++rp)
      if (XSLOTS % 512 == 0 || tid + 512 * rp < XSLOTS)  // whole waves without a granule skip the loads
#pragma unroll
      for (int e2 = 0; e2 < 4; ++e2) {
        const int k = 16 * ks + 4 * xkg[rp] + e2;
        const float2 v = Xl[(int64_t)min(k, p.xk_alloc - 1) * p.x_k + bx[rp]];
        xv[rp][e2] = k < p.kvalid ? v : make_float2(0.f, 0.f);
      }
  };
  auto stage = [&](int buf) {
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const int i = tid + 512 * it;
      const int kk = i >> 6, rg = i & 63;
      *reinterpret_cast<uint4*>(&la_s[buf][kk * LDA + 4 * rg]) = op_word<HT>(ast[it]);
    }
#pragma unroll
    for (int rp = 0; rp < XREP; ++rp) {
      const int s = tid + 512 * rp;
      if (s < XSLOTS) {
        uint4* dst = &lb_s[buf][(s >> 6) * H * 64 + (s & 63)];
        if (RE) t2_convert_re<kActT<HT>, H>(xv[rp], upx[rp], dc, dst);
        else t2_convert<kActT<HT>, H>(xv[rp], upx[rp], dc, s & 1, dst);
      }
    }
  };
  // RE: masks that take the real and imaginary column out of a stored word
  const uint32_t mre = dc ? 0x0000ffffu : 0xffffffffu;
  if (ks0 < ks1) {
    fetch(ks0);
    stage(0);
    __syncthreads();
    for (int ks = ks0; ks < ks1; ++ks) {
      const int cur = (ks - ks0) & 1;
      const bool more = ks + 1 < ks1;
      if (more) fetch(ks + 1);
      uint4 av[MF];
#pragma unroll
      for (int a = 0; a < MF; ++a) {
        const int r = 16 * (MF * wr + a) + (lane & 15);
        const uint32_t* la = &la_s[cur][(4 * (lane >> 4)) * LDA + r];
        av[a] = make_uint4(la[0] ^ cmask, la[LDA] ^ cmask, la[2 * LDA] ^ cmask, la[3 * LDA] ^ cmask);
      }
      if (RE) {
#pragma unroll
        for (int fr = 0; fr < NF / 2; ++fr) {
          const int cb = (NF / 2) * wc + fr;
#pragma unroll
          for (int t = 0; t < H; ++t) {
            const uint4 w = lb_s[cur][cb * H * 64 + 64 * t + lane];
            const uint4 br = make_uint4(w.x & mre, w.y & mre, w.z & mre, w.w & mre);
            const uint4 bi = make_uint4(t2_im_word(w.x, dc), t2_im_word(w.y, dc), t2_im_word(w.z, dc),
                                        t2_im_word(w.w, dc));
#pragma unroll
            for (int a = 0; a < MF; ++a) acc[a][2 * fr] = mfma16<kActT<HT>>(av[a], br, acc[a][2 * fr]);
#pragma unroll
            for (int a = 0; a < MF; ++a) acc[a][2 * fr + 1] = mfma16<kActT<HT>>(av[a], bi, acc[a][2 * fr + 1]);
          }
        }
      } else {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
          const int cb = NF * wc + f;
          const uint4 bh = lb_s[cur][cb * H * 64 + lane];
#pragma unroll
          for (int a = 0; a < MF; ++a) acc[a][f] = mfma16<kActT<HT>>(av[a], bh, acc[a][f]);
          if (H == 2) {
            const uint4 bo = lb_s[cur][cb * H * 64 + 64 + lane];
#pragma unroll
            for (int a = 0; a < MF; ++a) acc[a][f] = mfma16<kActT<HT>>(av[a], bo, acc[a][f]);
          }
        }
      }
      if (more) stage(cur ^ 1);
      __syncthreads();
    }
  }
  float* ow = p.out + (int64_t)split * p.o_split + (int64_t)l * p.o_slot;
  // per column block of this lane: rupture, validity and down scale, hoisted out of the rows;
  // each row takes one address computation and its stores use constant offsets
  constexpr int NC = RE ? NF / 2 : NF;
  const int b0 = RE ? ct * RB + 16 * ((NF / 2) * wc) + (lane & 15) : (2 * ct * RB + 16 * NF * wc + (lane & 15)) >> 1;
  float dn[NC];
  bool ok[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int b = RE ? b0 + 16 * c : b0 + 8 * c;
    ok[c] = b < p.B;
    dn[c] = (ok[c] && p.down) ? p.down[(int64_t)l * p.bp + b] : 1.f;
  }
  float* colp = ow + 2 * b0 + (RE ? 0 : (lane & 1));
#pragma unroll
  for (int a = 0; a < MF; ++a)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int rt_row = 16 * (MF * wr + a) + 4 * (lane >> 4) + r;  // row within the tile
      const int row = row0 + rt_row;
      if (row < p.nrows) {
        const float rs = rs_s[rt_row];
        float* pr = colp + (int64_t)row * p.o_row;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          if (!ok[c]) continue;
          if (RE)
            *reinterpret_cast<float2*>(pr + 32 * c) =
                make_float2(acc[a][2 * c][r] * rs * dn[c], acc[a][2 * c + 1][r] * rs * dn[c]);
          else
            pr[16 * c] = acc[a][c][r] * rs * dn[c];
        }
      }
    }
}

// shapes 2, 3: eight waves, 256 rows x 64 or 128 columns, both operands staged in LDS;
// shapes 5, 6, 7: the same with 64, 128 or 256 columns on real-column activation fragments
hipError_t launch_gemm_t(int ht, int hterms, int shape, const uint32_t* Aq, int64_t a_slot, int64_t a_k16, int64_t a_k,
                         int64_t a_r16, int nrows,
                         int rows_alloc, int kvalid, int kpad, const float2* X, int64_t x_slot, int64_t x_k,
                         int xk_alloc, const float* up, const float* down, const float* rowscale, int64_t rs_row,
                         int64_t rs_l, float* out, int64_t o_split, int64_t o_slot, int64_t o_row, int B, int bp,
                         int M, int splits, hipStream_t st) {
  if ((M & 7) || kpad % 16 || kpad < kvalid || kvalid < 1 || rows_alloc % 4 || rows_alloc < nrows || nrows < 1 ||
      splits < 1 || xk_alloc < kvalid || B < 1 || B > bp || !(shape == 2 || shape == 3 || (shape >= 5 && shape <= 7)) ||
      (o_row & 1) || (o_slot & 1) || (o_split & 1))
    return hipErrorInvalidValue;
  const int rt = 256;
  const int sh = shape >= 5 ? shape - 3 : shape;  // shapes 5, 6, 7: shapes 2, 3, 4 on real-column fragments
  const int ctc = sh == 2 ? 64 : sh == 3 ? 128 : 256;
  TArgs a;
  a.Aq = Aq;
  a.a_slot = a_slot;
  a.a_k16 = a_k16;
  a.a_k = a_k;
  a.a_r16 = a_r16;
  a.nrows = nrows;
  a.rows_alloc = rows_alloc;
  a.kvalid = kvalid;
  a.nks = kpad / 16;
  a.X = X;
  a.x_slot = x_slot;
  a.x_k = x_k;
  a.xk_alloc = xk_alloc;
  a.up = up;
  a.down = down;
  a.rowscale = rowscale;
  a.rs_row = rs_row;
  a.rs_l = rs_l;
  a.out = out;
  a.o_split = o_split;
  a.o_slot = o_slot;
  a.o_row = o_row;
  a.B = B;
  a.bp = bp;
  a.nrt = (nrows + rt - 1) / rt;
  a.nct = (2 * B + ctc - 1) / ctc;
  a.splits = std::min(splits, a.nks);
  const int64_t blocks = (int64_t)M * a.nrt * a.nct * a.splits;
  if (blocks <= 0 || blocks > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 grid((unsigned)blocks);
#define S2W_GT2(HT_, H_, NF_, RE_) hipLaunchKernelGGL((k_gemm_t2<HT_, H_, NF_, RE_>), grid, dim3(512), 0, st, a)
#define S2W_GT2_NF(HT_, H_) \
  do {                                                                        \
    if (shape == 2) S2W_GT2(HT_, H_, 2, false);                               \
    else if (shape == 3) S2W_GT2(HT_, H_, 4, false);                          \
    else if (shape == 5) S2W_GT2(HT_, H_, 2, true);                           \
    else if (shape == 6) S2W_GT2(HT_, H_, 4, true);                           \
    else S2W_GT2(HT_, H_, 8, true);                                           \
  } while (0)
  // operand pairs of the plans (as in the forward kernels)
  if (ht == 1 && hterms == 2) S2W_GT2_NF(1, 2);
  else if (ht == 2 && hterms == 1) S2W_GT2_NF(2, 1);
  else if (ht == 3 && hterms == 1) S2W_GT2_NF(3, 1);
  else return hipErrorInvalidValue;
#undef S2W_GT2
#undef S2W_GT2_NF
  return hipGetLastError();
}

}  // namespace s2w
