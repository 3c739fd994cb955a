// Half-precision helpers shared by the matrix-core kernels: operand types, rounding to
// bfloat16 / float16 (nearest even), the 16x16x32 MFMA, and power-of-two row scales.
//
// MFMA v_mfma_f32_16x16x32 (bf16/f16) fragments, lane l of 64:
//   A (16 x 32): row l%16, K entries 8*(l/16) .. +7      (16 bytes, 4 complex operand values)
//   B (32 x 16): column l%16, K entries 8*(l/16) .. +7
//   D (16 x 16): column l%16, rows 4*(l/16) .. +3        (4 floats)
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace s2w {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// streaming 16-byte load that bypasses cache retention
__device__ __forceinline__ uint4 ntload(const uint4* p) {
  const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
  return make_uint4(v.x, v.y, v.z, v.w);
}

// float -> half bits, round to nearest even
template <int HT>
__device__ __forceinline__ uint32_t to_half_bits(float v);
template <>
__device__ __forceinline__ uint32_t to_half_bits<1>(float v) {
  // round to nearest even (the hardware conversion)
  const __bf16 h = (__bf16)v;
  return (uint32_t)__builtin_bit_cast(uint16_t, h);
}
template <>
__device__ __forceinline__ uint32_t to_half_bits<2>(float v) {
  _Float16 h = (_Float16)v;
  return (uint32_t)__builtin_bit_cast(uint16_t, h);
}
typedef float s2w_f2v __attribute__((ext_vector_type(2)));
typedef __bf16 s2w_b2v __attribute__((ext_vector_type(2)));
typedef _Float16 s2w_h2v __attribute__((ext_vector_type(2)));

// Two values rounded to nearest even into one word: a in the low half, b in the high half.
template <int HT>
__device__ __forceinline__ uint32_t pack_half2(float a, float b) {
  const s2w_f2v v = {a, b};
  if constexpr (HT == 1)
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, s2w_b2v));
  else
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, s2w_h2v));
}

template <int HT>
__device__ __forceinline__ float from_half_bits(uint32_t b);
template <>
__device__ __forceinline__ float from_half_bits<1>(uint32_t b) {
  return __uint_as_float(b << 16);
}
template <>
__device__ __forceinline__ float from_half_bits<2>(uint32_t b) {
  return (float)__builtin_bit_cast(_Float16, (uint16_t)b);
}

template <int HT>
__device__ __forceinline__ f32x4 mfma16(uint4 a, uint4 b, f32x4 c) {
  if constexpr (HT == 1)
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0,
                                                  0, 0);
}

// Product types.  HT names the operator words and the products: 1 bfloat16 words, bfloat16
// products; 2 float16 words and products; 3 bfloat16 words converted to float16 in registers
// (op_word), float16 products.  kActT<HT> is the type of the activation terms and of the
// matrix-core instruction.
template <int HT>
constexpr int kActT = HT == 3 ? 2 : HT;

// bfloat16 pair -> float16 pair, low half first.  The stores' power-of-two row scales put every
// row maximum in [2^14, 2^15], inside float16's range; bfloat16's 8 significant bits fit
// float16's grid down to 2^-17 (normals from 2^-14, subnormal steps of 2^-24), so every word
// within 2^31 of its row maximum converts exactly, and smaller ones (below 2^-17) are cut
// toward zero by at most 2^-24 absolute.
__device__ __forceinline__ uint32_t bf16x2_to_f16x2(uint32_t w) {
  const float lo = __uint_as_float(w << 16), hi = __uint_as_float(w & 0xffff0000u);
  return __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(lo, hi));
}

// Operator fragment (8 half words) in the instruction's type.
template <int HT>
__device__ __forceinline__ uint4 op_word(uint4 a) {
  if constexpr (HT == 3)
    return make_uint4(bf16x2_to_f16x2(a.x), bf16x2_to_f16x2(a.y), bf16x2_to_f16x2(a.z), bf16x2_to_f16x2(a.w));
  else
    return a;
}

// power-of-two scale that maps a row maximum mx into [2^14, 2^15); returns the multiplier
// applied before rounding (`up`) and its inverse (`down`)
__device__ __forceinline__ void pow2_scale(float mx, float& up, float& down) {
  if (!(mx > 0.f) || !isfinite(mx)) {
    up = 1.f;
    down = 1.f;
    return;
  }
  int ex;
  frexpf(mx, &ex);  // mx = f * 2^ex, f in [0.5, 1)
  // rows whose largest entry is below 2^-111 keep the multiplier finite (<= 2^126); their
  // scaled values then sit below 2^15 without filling the range, which is harmless
  ex = ex < -111 ? -111 : ex;
  up = ldexpf(1.f, 15 - ex);
  down = ldexpf(1.f, ex - 15);
}

// One B-fragment granule per thread and term: lane L = 16*kg + c16 of column block cb holds the
// four k = 4*kg + e of column n = 16*cb + c16 (rupture n/2; real part if n even, else imaginary).
template <int HT, int H>
__device__ __forceinline__ void t2_convert(const float2* v, float up, bool dc, int cim, uint4* dst) {
  uint32_t hi[4], lo[4];
#pragma unroll
  for (int e2 = 0; e2 < 4; ++e2) {
    const float x = v[e2].x * up, y = v[e2].y * up;
    // column re: (x, -y) (DC: (x, 0)); column im: (y, x) (DC: (0, y))
    const float c0 = cim ? (dc ? 0.f : y) : x;
    const float c1 = cim ? (dc ? y : x) : (dc ? 0.f : -y);
    hi[e2] = pack_half2<HT>(c0, c1);
    if (H == 2)
      lo[e2] = pack_half2<HT>(c0 - from_half_bits<HT>(hi[e2] & 0xffffu), c1 - from_half_bits<HT>(hi[e2] >> 16));
  }
  dst[0] = make_uint4(hi[0], hi[1], hi[2], hi[3]);
  if (H == 2) dst[64] = make_uint4(lo[0], lo[1], lo[2], lo[3]);
}

// Row-block-major elastic store Gq[l][g/16][ks][g%16][16 words]: chunk 0 of grid row g (bin l)
// at K step 0, as uint4; K step ks of the same row is ks * kGqStepU4 further on.
constexpr int kGqStepU4 = 64;
__device__ __forceinline__ const uint4* gq_row(const uint4* Gq, int g, int l, int ng16, int nks) {
  return Gq + (((int64_t)l * ng16 + (g >> 4)) * nks * 16 + (g & 15)) * 4;
}

}  // namespace s2w
