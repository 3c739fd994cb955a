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

// Twiddle table upload (once per device).
hipError_t upload_twiddles(int device);

// s[rows][nt] real rows (row = outer * ninner + inner, rows with inner >= ninner
// are zero) -> packed spectra at out + outer*out_outer + inner*out_inner + slot*out_slot.
hipError_t launch_rfft_rows(const float* in, int64_t nouter, int ninner, int ninner_pad, float2* out,
                            int64_t out_outer, int64_t out_inner, int64_t out_slot, const Geometry& g, float scale,
                            hipStream_t st);

// packed spectra rows (in + row*in_row + slot*in_slot) -> real rows out[row][n], n < nt, times scale
hipError_t launch_irfft_rows(const float2* in, int64_t nrows, int64_t in_row, int64_t in_slot, float* out,
                             int64_t out_row, const Geometry& g, float scale, hipStream_t st);

// Single-rupture fused forward: every workgroup contracts its grid rows against the
// source spectrum, runs the mid-chain round trip in LDS and accumulates its partial
// observation spectra; part receives [nwg][M][nop] complex.
hipError_t launch_fused_forward(const float2* Gh, const float2* Fh, const float2* Sh, float2* part, int nwg,
                                int tile_rows, const Geometry& g, hipStream_t st);

// Sum the partials over workgroups in a fixed order: out[o][slot] (complex, row stride M).
hipError_t launch_reduce_partials(const float2* part, int nparts, int64_t items, int M, int nop, int nvalid_cols,
                                  float2* out, hipStream_t st);

// Single-rupture adjoint, stage 1: per grid row, conj-transposed acoustic contraction,
// mid-chain round trip with the transposed difference; Wp[g][slot] (complex).
hipError_t launch_adjoint_rows(const float2* Fh, const float2* Rh, float2* Wp, int nwg, int tile_rows,
                               const Geometry& g, hipStream_t st);

// Single-rupture adjoint, stage 2: part[split][slot][j] = sum over the split's grid rows of
// conj(Gh[g][slot][j]) * Wp[g][slot].
hipError_t launch_adjoint_elastic(const float2* Gh, const float2* Wp, float2* part, int slots_per_wg, int splits,
                                  const Geometry& g, hipStream_t st);

// Unfused forward: stage 1 writes the per-row mid-chain output Vh[g][l]; stage 2
// contracts it with the acoustic store per bin, split over grid rows.
hipError_t launch_forward_rows(const float2* Gh, const float2* Sh, float2* Vh, int nwg, const Geometry& g,
                               hipStream_t st);
hipError_t launch_rows_acoustic(const float2* Fh, const float2* Vh, float2* part, int slots_per_wg, int splits,
                                const Geometry& g, hipStream_t st);

// Largest F-stage item count per thread the fused kernel supports (items = M * nop/2).
constexpr int FUSED_MAX_ITEMS = 32 * 256;

}  // namespace s2w
