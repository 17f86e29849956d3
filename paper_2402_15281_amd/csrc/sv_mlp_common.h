// Device building blocks shared by the BF16 network kernels (inference and training).
//
// MFMA used: v_mfma_f32_32x32x16_bf16.  Operand layouts (lane l of a wave):
//   A (32 x 16): A[l % 32][8 (l / 32) + e], e = 0..7
//   B (16 x 32): B[8 (l / 32) + e][l % 32]
//   C (32 x 32): acc[4 j + i] = C[8 j + 4 (l / 32) + i][l % 32]
// Layers are computed transposed: C[f][r] = sum_k W[f][k] H[r][k], so A is a weight
// tile (packed in this order ahead of time) and B is read from the activation tile
// H[r][k] in LDS (8 consecutive k of one row per lane).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sv {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kTileRows = 64;   // rows (queries / samples) per workgroup
constexpr int kLdsPad = 8;      // BF16 elements of padding per LDS row

// Softplus for values that are rounded to BF16 afterwards:
// max(z, 0) + ln2 * log2(1 + 2^(-|z| log2 e)) with the hardware exp2/log2.
__device__ __forceinline__ float softplus_fast(float z) {
  const float e = __builtin_amdgcn_exp2f(-fabsf(z) * 1.44269504088896341f);
  return fmaf(0.693147180559945309f, __builtin_amdgcn_logf(1.0f + e), fmaxf(z, 0.f));
}

// Derivative of softplus from its output a = softplus(z): sigmoid(z) = 1 - exp(-a).
__device__ __forceinline__ float softplus_grad_from_out(float a) {
  return 1.0f - __builtin_amdgcn_exp2f(-a * 1.44269504088896341f);
}

// One layer's MFMA loop for one wave: output features [64 wid, 64 wid + 64) of the
// 64 tile rows, i.e. 2 feature blocks (fb) x 2 row blocks (rb) of 32 x 32.
// Wp: packed weights of this layer; Hin: LDS tile [64][W + pad].
template <int W>
__device__ __forceinline__ void layer_mfma(const __bf16* __restrict__ Wp, const __bf16* Hin, int wid, int lane,
                                           f32x16& acc00, f32x16& acc01, f32x16& acc10, f32x16& acc11) {
  constexpr int KS = W / 16;
  constexpr int LD = W + kLdsPad;
  const int half = lane >> 5, col = lane & 31;
  const bf16x8* A0 = reinterpret_cast<const bf16x8*>(Wp) + ((size_t)(2 * wid) * KS) * 64 + lane;
  const bf16x8* A1 = A0 + (size_t)KS * 64;
  const __bf16* B0 = Hin + col * LD + 8 * half;
  const __bf16* B1 = B0 + 32 * LD;
  acc00 = f32x16{};
  acc01 = f32x16{};
  acc10 = f32x16{};
  acc11 = f32x16{};
  bf16x8 a0 = A0[0], a1 = A1[0];
#pragma unroll 2
  for (int ks = 0; ks < KS; ++ks) {
    const bf16x8 b0 = *reinterpret_cast<const bf16x8*>(B0 + ks * 16);
    const bf16x8 b1 = *reinterpret_cast<const bf16x8*>(B1 + ks * 16);
    const int kn = ks + 1 < KS ? ks + 1 : ks;
    const bf16x8 na0 = A0[(size_t)kn * 64], na1 = A1[(size_t)kn * 64];
    acc00 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc00, 0, 0, 0);
    acc01 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b1, acc01, 0, 0, 0);
    acc10 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b0, acc10, 0, 0, 0);
    acc11 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, acc11, 0, 0, 0);
    a0 = na0;
    a1 = na1;
  }
}

// Packing of a W x W weight matrix M (row-major, FP32) into MFMA A-operand order:
// element (fb, ks, lane, e) = M[fb*32 + lane%32][ks*16 + 8*(lane/32) + e], or of
// M's transpose when `transpose` is set.  o indexes the packed array of one layer.
__device__ __forceinline__ void packed_coords(int64_t o, int W, bool transpose, int* row, int* colk) {
  const int e = (int)(o & 7);
  const int ln = (int)((o >> 3) & 63);
  const int64_t blk = o >> 9;
  const int ks = (int)(blk % (W / 16));
  const int fb = (int)(blk / (W / 16));
  const int r = fb * 32 + (ln & 31);
  const int k = ks * 16 + 8 * (ln >> 5) + e;
  *row = transpose ? k : r;
  *colk = transpose ? r : k;
}

}  // namespace sv
