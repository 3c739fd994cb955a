// Internal declarations shared by the host side of the library and the kernel
// translation units.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace s2w {

// Geometry of a plan, derived from the public descriptor.
struct Geometry {
  int nsub, ngrid, nobs, nt;
  int L, M, logM;      // transform length, packed slots (L/2), log2(M)
  int nsp;             // nsub padded to a multiple of 2 (complex values per (row, slot) of the elastic store)
  int nop;             // nobs padded to a multiple of 2
  int nsp4, nop4;      // float4 (two complex) per (row, slot) row of the stores
  int diff;
  float dt;
};

// Optional capture of the seafloor displacement m (eq. 1: the first product's inverse
// transform, truncated to n < nt, before D_t) at selected time steps, written where the
// mid-chain forms it.  Sample n of transform row r goes to
//   base[r * row_stride + column(n)]   (rows r < rows only),
// column(n) = n when every step is selected, else the rank of n among the selected steps
// (bit n of `bits`).  `scale` turns the unnormalised inverse transform into m (1/L).
// Kernels whose transform rows are ruptures of one grid row also take the grid-row stride
// `grid_stride` and offset `base` themselves.
struct DispOut {
  float* base;          // nullptr: nothing captured
  int64_t row_stride;
  int64_t grid_stride;
  int rows;
  int all;
  float scale;
  uint32_t bits[16];    // steps 0 .. 511
};

// Twiddle table upload (once per device).
hipError_t upload_twiddles(int device);

// s[rows][nt] real rows (row = outer * ninner + inner, rows with inner >= ninner
// are zero) -> packed spectra at out + outer*out_outer + inner*out_inner + slot*out_slot.
hipError_t launch_rfft_rows(const float* in, int64_t nouter, int ninner, int ninner_pad, float2* out,
                            int64_t out_outer, int64_t out_inner, int64_t out_slot, const Geometry& g, float scale,
                            hipStream_t st);
// Forward real FFT of time rows in[b][j][n] into out[l][j][b] (l * out_slot + j * bp + b), M = 256 only.
hipError_t launch_rfft_batch256(const float* in, int B, int nrows, int nrows_pad, float2* out, int bp, int64_t out_slot,
                                int nt, float scale, hipStream_t st);

// packed spectra rows (in + row*in_row + slot*in_slot) -> real rows out[row][n], n < nt, times scale
hipError_t launch_irfft_rows(const float2* in, int64_t nrows, int64_t in_row, int64_t in_slot, float* out,
                             int64_t out_row, const Geometry& g, float scale, hipStream_t st);

// Single-rupture fused forward: every workgroup contracts its grid rows against the
// source spectrum, runs the mid-chain round trip in LDS and accumulates its partial
// observation spectra; part receives [nwg][nop][M] complex.
hipError_t launch_fused_forward(const float2* Gh, const float2* Fh, const float2* Sh, float2* part, int nwg,
                                int tile_rows, const Geometry& g, hipStream_t st, const DispOut& disp);

// Fixed-order sum of partial spectra: out[i] = sum_p part[p][i], i < items_c (complex values).
hipError_t launch_sum_parts(const float2* part, int nparts, int64_t items_c, float2* out, hipStream_t st);

// Observers per thread the fused forward needs (it supports up to 32).
int fused_forward_opt(const Geometry& g);

// Single-rupture adjoint, stage 1: per grid row, conj-transposed acoustic contraction,
// mid-chain round trip with the transposed difference; Wp[g][slot] (complex).
hipError_t launch_adjoint_rows(const float2* Fh, const float2* Rh, float2* Wp, int nwg, int tile_rows,
                               const Geometry& g, hipStream_t st);

// Single-rupture adjoint, stage 2: part[split][j][slot] = sum over the split's grid rows of
// conj(Gh[g][j][slot]) * Wp[g][slot].
hipError_t launch_adjoint_elastic(const float2* Gh, const float2* Wp, float2* part, int cols_per_thread, int splits,
                                  const Geometry& g, hipStream_t st);

// Unfused forward: stage 1 writes the per-row mid-chain output Vh[g][l]; stage 2
// contracts it with the acoustic store per bin, split over grid rows.
hipError_t launch_forward_rows(const float2* Gh, const float2* Sh, float2* Vh, int nwg, const Geometry& g,
                               hipStream_t st, const DispOut& disp);
hipError_t launch_rows_acoustic(const float2* Fh, const float2* Vh, float2* part, int cols_per_thread, int splits,
                                const Geometry& g, hipStream_t st);

// ---- batched path (matrix cores, half-precision stores); ht: 1 = bf16, 2 = f16 ----
// ng16 > 0 selects the row-block-major layout of the elastic store (ng16 = blocks of 16 grid
// rows; sg, sl, sc unused): word (((l*ng16 + g/16)*(ncp/16) + c/16)*16 + g%16)*16 + c%16.
hipError_t launch_quant_rows(int ht, const float2* staging, int64_t nrows, int M, int nc, int ncp, uint32_t* out,
                             int64_t row0, int64_t sg, int64_t sl, int64_t sc, float* scale, int ng16, hipStream_t st);
hipError_t launch_prep_act(int ht, int hterms, const float2* S, float* sig_up, float* sig_down, int M, int nsub,
                           int nsq, int B, int bp, int nks, int ncb, uint4* Bop, hipStream_t st);
// Real-column activation fragments for the elastic GEMM tiles 17 and 18: Bre[l][ks][rcb][h][lane]
// with rcb < (B + 15) / 16 blocks of 16 ruptures (half the size of Bop).
hipError_t launch_prep_act_re(int ht, int hterms, const float2* S, float* sig_up, float* sig_down, int M, int nsub,
                              int nsq, int B, int bp, int nks, int nrcb, uint4* Bre, hipStream_t st);
hipError_t launch_gemm_g(int ht, int hterms, int cfg, const uint4* Gq, const float* sG, const uint4* Bop,
                         const float* sig_down, float* U, int nwg, int ngrid, int M, int nks, int ncb, int B, int bp,
                         hipStream_t st);
// LDS-staged acoustic GEMM (packed bfloat16 activation): supported observer paddings and the
// number of rupture tiles it launches for a batch of B.
inline bool gemm_f2_supported(int noq, int B) {
  const int mf = noq / 16;
  return mf == 1 || mf == 2 || mf == 4 || (B <= 64 && mf == 8);
}
inline int gemm_f2_col_tiles(int B) {
  const int nr = B > 64 ? 256 : 64;
  return (B + nr - 1) / nr;
}
// Acoustic GEMM with eight waves across the output columns, both operands staged in LDS:
// part[split][l][o][n] (o < nobs, n < 2B) from complex64 V[g][l][b] (scaled by up[l][b] when
// given, converted to hterms half terms).  Splits: grid-row ranges (clamped to the K steps).
int gemm_fw_nf(int hterms, int B, bool re);
inline int gemm_fw_col_tiles(int hterms, int B, bool re) {
  return (B + 64 * gemm_fw_nf(hterms, B, re) - 1) / (64 * gemm_fw_nf(hterms, B, re));
}
hipError_t launch_gemm_fw(int ht, int hterms, const uint32_t* Fq, const float2* V, const float* up, float* part,
                          int ngrid, int ngq, int M, int noq, int nobs, int B, int bp, int splits, bool re, hipStream_t st);
// Few-input per-bin products of one BLTT operator (B <= 4), HBM-bound: yh[b][r][l] from the
// store K[r][l][c] and inputs X[b][l][c] (c padded to an even ncp with zeros).
hipError_t launch_bltt_gemv(const float2* K, const float2* X, float2* yh, int nrow, int M, int ncp, int B, int ncu,
                            hipStream_t st);
hipError_t launch_gemm_f2(const uint4* Fq, const uint2* V, float* part, int ngrid, int ngq, int M, int noq, int B,
                          int bp, int splits, hipStream_t st);
// rupts: ruptures per unit of the M = 256 kernel (16 or 32; other values mean 16).  With cmax
// (M = 256 only) the kernel also leaves per-(slot, rupture) maxima of |Re|, |Im| of what it
// writes in cmax[group][l][b] (at most cmax_floats floats) and sets *cmax_groups to the group
// count; elsewhere *cmax_groups is 0 and no maxima are produced.
hipError_t launch_mid_batch(float2* U, const float* sF, int B, int bp, bool adjoint, bool pack_bf16,
                            const Geometry& g, hipStream_t st, int rupts = 16, float* cmax = nullptr,
                            int64_t cmax_floats = 0, int* cmax_groups = nullptr, const DispOut* disp = nullptr);
// Power-of-two column scales from partial maxima part[s][l][b], s < splits (columns b >= B get 1).
hipError_t launch_col_scale_final(const float* part, int splits, int M, int B, int bp, float* tau_up, float* tau_down,
                                  hipStream_t st);
hipError_t launch_col_scale(const float2* V, int ngrid, int M, int B, int bp, float* tau_up, float* tau_down,
                            float* part, int64_t part_floats, hipStream_t st);
hipError_t launch_sum_f(const float* part, int splits, int M, int noq, int nobs, int B, int bp, const float* tau_down,
                        float2* yh, hipStream_t st);
// Sum of split partials part[s][l][o][2 bp] and inverse real FFT into out[b][o][n] (M = 256 only).
hipError_t launch_sum_irfft256(const float* part, int splits, int noq, int nrows, int B, int bp,
                               const float* tau_down, float* out, int nt, float scale, hipStream_t st);
hipError_t launch_zero_strided(uint32_t* out, int64_t n, int64_t stride, int width, hipStream_t st);
hipError_t launch_act_scale(const float2* S, int M, int nk, int nkp, int B, int bp, float* sig_up, float* sig_down,
                            hipStream_t st);
// Conjugate-transposed half-precision GEMM per slot (adjoint products); see the kernel.
// shape 0: tall operator (many rows, short K); shape 1: few rows, long K.
hipError_t launch_gemm_t(int ht, int hterms, int shape, const uint32_t* Aq, int64_t a_slot, int64_t a_k16, int64_t a_k,
                         int64_t a_r16, int nrows,
                         int rows_alloc, int kvalid, int kpad, const float2* X, int64_t x_slot, int64_t x_k,
                         int xk_alloc, const float* up, const float* down, const float* rowscale, int64_t rs_row,
                         int64_t rs_l, float* out, int64_t o_split, int64_t o_slot, int64_t o_row, int B, int bp,
                         int M, int splits, hipStream_t st);

// ---- batched path (matrix cores, float32 stores) ----
// Per-slot complex GEMM out(row, b) = sum_k op(A(row, k)) X(k, b) for every slot l < M:
//   A(row, k) at A + l*a_slot + row*a_row + k*a_k (complex; rcont: a_row == 1, else a_k == 1),
//   rows < rows_alloc readable, k < kvalid nonzero, K padded to kpad (multiple of 8);
//   X(k, b) at X + l*x_slot + k*x_k + b, rows k < xk_alloc readable;
//   out float index split*o_split + l*o_slot + row*o_row + (2*b + re/im), rows < nrows, b < B;
//   K split over `splits` ranges (one partial per split).
int cgemm32_rows(int cfg);
int cgemm32_ruptures(int cfg);
hipError_t launch_cgemm32(int cfg, bool rcont, bool conj, const float2* A, int64_t a_row, int64_t a_k,
                          int64_t a_slot, int nrows, int rows_alloc, int kvalid, int kpad, const float2* X,
                          int64_t x_k, int64_t x_slot, int xk_alloc, int B, int bp, float* out, int64_t o_row,
                          int64_t o_slot, int64_t o_split, int M, int splits, hipStream_t st);

// ---- direct time-domain path (float32 matrix cores, no FFT) ----
// out[split][r][n] = sum over the split's channels c of sum_{k<=n} A(c, r, k) x_c[n - k], n < nt,
// A(c, r, k) at A + c*a_c + r*a_r + k (16-byte aligned rows, zeros at k >= nt up to nt rounded to
// 16), x_c[p] at X + c*x_c + (rev ? nt - 1 - p : p); rw = 1 or 2 row blocks of 16 per wave.
int direct_rows_per_tile(int rw);
hipError_t launch_direct(int rw, const float* A, int64_t a_c, int64_t a_r, int R, int nchan, const float* X,
                         int64_t x_c, bool rev, float* out, int64_t o_s, int64_t o_r, int nt, int splits,
                         hipStream_t st);
// out[r*o_r + n] = scale * (S(r, n) - diff * S(r, n-1)), S(r, n) = sum_q part[q*p_s + r*p_r + (rev ? nt-1-n : n)]
hipError_t launch_direct_reduce(const float* part, int parts, int64_t p_s, int64_t p_r, int R, int nt, bool rev,
                                bool diff, float scale, float* out, int64_t o_r, hipStream_t st,
                                const DispOut* disp = nullptr);
// out[s][k] = in[s][k] (k < nt), 0 (nt <= k < ntp), for n series
hipError_t launch_pad_series(const float* in, int64_t n, int nt, int ntp, float* out, hipStream_t st);

}  // namespace s2w
