// Real-column activation fragments for the half-precision GEMMs whose activations are
// converted in the workgroup (the transposed products and the eight-wave acoustic product).
// A complex activation x + iy enters the real 2x2 embedding of a complex product as two
// columns: the real-part column (x, -y) and the imaginary-part column (y, x), each a 32-bit
// word of two half values; on the DC bin (two real spectra packed in one slot) the columns are
// (x, 0) and (0, y).  Only the real-part words are converted and kept; the imaginary-part ones
// follow in registers with the same bits the full conversion gives.
#pragma once

#include "s2w_half.h"

namespace s2w {

// Real-column granule for the RE layout: lane L = 16*kg + c16 of block rb holds the four
// k = 4*kg + e of rupture 16*rb + c16 as words (x, -y), or (x, y) on the DC bin.
template <int HT, int H>
__device__ __forceinline__ void t2_convert_re(const float2* v, float up, bool dc, uint4* dst) {
  uint32_t hi[4], lo[4];
#pragma unroll
  for (int e2 = 0; e2 < 4; ++e2) {
    const float c0 = v[e2].x * up, y = v[e2].y * up;
    const float c1 = dc ? y : -y;
    hi[e2] = pack_half2<HT>(c0, c1);
    if (H == 2)
      lo[e2] = pack_half2<HT>(c0 - from_half_bits<HT>(hi[e2] & 0xffffu), c1 - from_half_bits<HT>(hi[e2] >> 16));
  }
  dst[0] = make_uint4(hi[0], hi[1], hi[2], hi[3]);
  if (H == 2) dst[64] = make_uint4(lo[0], lo[1], lo[2], lo[3]);
}

// Imaginary-column word from a stored real-column word: (x, -y) -> (y, x) off the DC bin
// (rounding to half is sign-symmetric, so this is the word (y, x) converts to), (x, y) -> (0, y)
// on it.
__device__ __forceinline__ uint32_t t2_im_word(uint32_t w, bool dc) {
  return dc ? (w & 0xffff0000u) : (((w >> 16) | (w << 16)) ^ 0x8000u);
}

}  // namespace s2w
