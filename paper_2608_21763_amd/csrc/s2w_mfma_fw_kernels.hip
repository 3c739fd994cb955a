// Acoustic per-bin GEMM of the batched half-precision path with eight waves across the output
// columns (eq. 2 per bin, Alg. 2 step 3 of the second product):
//   part[split][l][o][n] = sum_{g in split} Fq[l][o][g] (x) up(l, b) V[g][l][b]
// The acoustic store Fq[l][o][g] (32-bit words re | im << 16) gives MFMA A fragments of four
// consecutive grid rows directly; the operator tile of a K step (16 grid rows x 64 observers)
// is loaded once per workgroup into LDS in fragment order, and the complex64 activation V is
// converted once per workgroup into B fragments (H half terms, after the optional
// power-of-two column scale up), both double-buffered with one barrier per step.  A
// workgroup covers 64 observers x 128*NF output columns (64*NF ruptures) of one slot and one
// range of grid rows; the fixed-order sum over ranges follows.
#include <algorithm>

#include "s2w_half.h"
#include "s2w_half_re.h"
#include "s2w_internal.h"

namespace s2w {

struct FWArgs {
  const uint32_t* Fq;
  const float2* V;
  const float* up;  // [l][bp] or null
  float* part;
  int ngrid, ngq, noq, nobs, M, B, bp, nks, nrt, nct, splits;
};

// RE = true (NF even) keeps only the real-column fragments in LDS, one block of 16 ruptures
// per pair of output column blocks, and forms the imaginary columns in registers (same bits,
// same products in the same order).
template <int HT, int H, int NF, bool RE>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(RE ? 4 : 1))) void k_gemm_fw(const FWArgs p) {
  static_assert(!RE || NF % 2 == 0, "real-column fragments pair the column blocks of a wave");
  constexpr int MF = 4, RT = 64, NCB = 8 * NF, RB = 64 * NF;
  constexpr int NBS = RE ? NCB / 2 : NCB;  // fragment blocks held in LDS per step
  constexpr int XSLOTS = NBS * 64, XREP = (XSLOTS + 511) / 512;
  __shared__ uint4 la_s[2][MF * 64];
  __shared__ uint4 lb_s[2][NBS * H * 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int x = blockIdx.x & 7, q = blockIdx.x >> 3;
  const int per_slot = p.nrt * p.nct * p.splits;
  const int l = x + 8 * (q / per_slot);
  int rem = q % per_slot;
  const int split = rem % p.splits;
  rem /= p.splits;
  const int ct = rem % p.nct, rt = rem / p.nct;
  const bool dc = (l == 0);
  const int ks0 = (int)((int64_t)p.nks * split / p.splits), ks1 = (int)((int64_t)p.nks * (split + 1) / p.splits);
  const int row0 = rt * RT;
  // operator ownership (threads < 256): fragment a = tid / 64, lane L = tid % 64 -> observer
  // row0 + 16 a + L % 16, grid rows 4 (L / 16) .. +3 of the step
  const bool aown = tid < MF * 64;
  const int ao = min(row0 + 16 * (tid >> 6) + (tid & 15), p.noq - 1);
  const uint32_t* Arow = p.Fq + ((int64_t)l * p.noq + ao) * p.ngq + 4 * ((tid & 63) >> 4);
  // activation ownership: granule slot s = tid + 512 * rep -> column block s / 64, lane s % 64
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
  const float2* Vl = p.V + (int64_t)l * p.bp;
  const int64_t vstep = (int64_t)p.M * p.bp;
  f32x4 acc[MF][NF];
#pragma unroll
  for (int a = 0; a < MF; ++a)
#pragma unroll
    for (int f = 0; f < NF; ++f) acc[a][f] = f32x4{0.f, 0.f, 0.f, 0.f};
  uint4 ast;
  float2 xv[XREP][4];
  auto fetch = [&](int ks) {
    if (aown) ast = *reinterpret_cast<const uint4*>(Arow + 16 * ks);
#pragma unroll
    for (int rp = 0; rp < XREP; ++rp)
      if (XSLOTS % 512 == 0 || tid + 512 * rp < XSLOTS)  // whole waves without a granule skip the loads
#pragma unroll
      for (int e2 = 0; e2 < 4; ++e2) {
        const int g = 16 * ks + 4 * xkg[rp] + e2;
        const float2 v = Vl[(int64_t)min(g, p.ngrid - 1) * vstep + bx[rp]];
        xv[rp][e2] = g < p.ngrid ? v : make_float2(0.f, 0.f);
      }
  };
  auto stage = [&](int buf) {
    if (aown) la_s[buf][tid] = op_word<HT>(ast);
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
  const uint32_t mre = dc ? 0x0000ffffu : 0xffffffffu;  // RE: real column of a stored word
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
      for (int a = 0; a < MF; ++a) av[a] = la_s[cur][a * 64 + lane];
      if (RE) {
#pragma unroll
        for (int fr = 0; fr < NF / 2; ++fr) {
          const int cb = (NF / 2) * wave + fr;
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
          const int cb = NF * wave + f;
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
  float* ow = p.part + (((int64_t)split * p.M + l) * p.noq) * (2 * (int64_t)p.bp);
#pragma unroll
  for (int a = 0; a < MF; ++a)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int o = row0 + 16 * a + 4 * (lane >> 4) + r;
      if (o < p.nobs) {
        if (RE) {
#pragma unroll
          for (int fr = 0; fr < NF / 2; ++fr) {
            const int b = ct * RB + 16 * ((NF / 2) * wave + fr) + (lane & 15);
            if (b < p.B)
              *reinterpret_cast<float2*>(&ow[(int64_t)o * (2 * p.bp) + 2 * b]) =
                  make_float2(acc[a][2 * fr][r], acc[a][2 * fr + 1][r]);
          }
        } else {
#pragma unroll
          for (int f = 0; f < NF; ++f) {
            const int n = 2 * ct * RB + 16 * (NF * wave + f) + (lane & 15);
            if ((n >> 1) < p.B) ow[(int64_t)o * (2 * p.bp) + n] = acc[a][f][r];
          }
        }
      }
    }
}

int gemm_fw_nf(int hterms, int B, bool re) {
  if (B <= 64) return 1;
  if (B <= 128 || (hterms == 2 && !re)) return 2;
  return 4;
}

hipError_t launch_gemm_fw(int ht, int hterms, const uint32_t* Fq, const float2* V, const float* up, float* part,
                          int ngrid, int ngq, int M, int noq, int nobs, int B, int bp, int splits, bool re,
                          hipStream_t st) {
  const int nf = gemm_fw_nf(hterms, B, re);
  re = re && nf >= 2;  // one column block per wave has no pair to share fragments
  if ((M & 7) || ngq % 16 || ngq < ngrid || noq % 16 || nobs > noq || B < 1 || B > bp || splits < 1)
    return hipErrorInvalidValue;
  FWArgs a;
  a.Fq = Fq;
  a.V = V;
  a.up = up;
  a.part = part;
  a.ngrid = ngrid;
  a.ngq = ngq;
  a.noq = noq;
  a.nobs = nobs;
  a.M = M;
  a.B = B;
  a.bp = bp;
  a.nks = ngq / 16;
  a.nrt = (nobs + 63) / 64;
  a.nct = (B + 64 * nf - 1) / (64 * nf);
  a.splits = std::min(splits, a.nks);
  const int64_t blocks = (int64_t)M * a.nrt * a.nct * a.splits;
  if (blocks <= 0 || blocks > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 grid((unsigned)blocks);
#define S2W_FW1(HT_, H_, NF_, RE_) hipLaunchKernelGGL((k_gemm_fw<HT_, H_, NF_, RE_>), grid, dim3(512), 0, st, a)
#define S2W_FW(HT_, H_, NF_)             \
  do {                                   \
    if (NF_ > 1 && re)                   \
      S2W_FW1(HT_, H_, NF_, (NF_ > 1)); \
    else                                 \
      S2W_FW1(HT_, H_, NF_, false);      \
  } while (0)
  // operand pairs of the plans: bf16 words with two bf16 activation terms, f16 words with one
  // f16 term, bf16 words converted to f16 with one f16 term
  if (ht == 1 && hterms == 2) {
    if (nf == 1) S2W_FW(1, 2, 1); else if (nf == 2) S2W_FW(1, 2, 2); else S2W_FW1(1, 2, 4, true);
  } else if (ht == 2 && hterms == 1) {
    if (nf == 1) S2W_FW(2, 1, 1); else if (nf == 2) S2W_FW(2, 1, 2); else S2W_FW(2, 1, 4);
  } else if (ht == 3 && hterms == 1) {
    if (nf == 1) S2W_FW(3, 1, 1); else if (nf == 2) S2W_FW(3, 1, 2); else S2W_FW(3, 1, 4);
  } else {
    return hipErrorInvalidValue;
  }
#undef S2W_FW
#undef S2W_FW1
  return hipGetLastError();
}

}  // namespace s2w
