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

// max(z, 0) of an MFMA result as med3(z, 0, FLT_MAX), one instruction: fmaxf compiles to
// a NaN-quieting max(z, z) first, since the compiler cannot tell that MFMA results are
// already quiet.  The same value for every finite z (+inf gives FLT_MAX).
__device__ __forceinline__ float relu_acc(float z) { return __builtin_amdgcn_fmed3f(z, 0.f, 3.402823466e38f); }

// Softplus for values that are rounded to BF16 afterwards:
// max(z, 0) + ln2 * log2(1 + 2^(-|z| log2 e)) with the hardware exp2/log2.
__device__ __forceinline__ float softplus_fast(float z) {
  const float e = __builtin_amdgcn_exp2f(-fabsf(z) * 1.44269504088896341f);
  return fmaf(0.693147180559945309f, __builtin_amdgcn_logf(1.0f + e), relu_acc(z));
}

// Derivative of softplus from its output a = softplus(z): sigmoid(z) = 1 - exp(-a).
__device__ __forceinline__ float softplus_grad_from_out(float a) {
  return 1.0f - __builtin_amdgcn_exp2f(-a * 1.44269504088896341f);
}

// Weight tiles are read with buffer loads: the wave's slice of packed weights is one
// buffer resource (a wave-uniform base and byte range in scalar registers), the lane's
// 16-byte part of a tile is a 32-bit vector offset, and the tile index goes into the
// scalar offset.  Unlike 64-bit per-lane pointers this needs no vector address
// arithmetic in the MFMA loop, and a read past the range returns zeros instead of
// touching other memory.  0x00020000 is the resource's format word for the gfx9 family.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t weight_rsrc(const __bf16* slice, int tiles) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)slice, (short)0, tiles * 1024, 0x00020000);
}
__device__ __forceinline__ bf16x8 load_tile(__amdgpu_buffer_rsrc_t rs, int lane_off, int tile) {
  return __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(rs, lane_off, tile * 1024, 0));
}

// One layer's MFMA loop for a wave owning FB feature blocks (32 FB features from feature
// 32 FB wf) of RB row blocks (32 RB rows from row 32 RB wr): FB x RB MFMA tiles,
// acc[fb][rb].  Each weight tile is used RB times and each activation tile FB times
// per load, so weight traffic per MFMA is 1/RB KB and LDS traffic 1/FB KB.
// Ring depth D for the weight tiles.
// K: inputs (columns of the layer's weights and of the activation tile), LD: the tile's
// row stride in elements.  kPrio raises the wave's issue priority for the loop, so that
// on a SIMD shared with a wave in its epilogue the MFMAs go first and the epilogue's
// VALU work fills the cycles between them.
template <int K, int LD, int FB, int RB, int D, bool kPrio = false>
__device__ __forceinline__ void layer_mfma_k(const __bf16* __restrict__ Wp, const __bf16* Hin, int wf, int wr,
                                             int lane, const float* __restrict__ bias, f32x16 (&acc)[FB][RB]) {
  constexpr int KS = K / 16;
  static_assert(KS % D == 0, "k-steps must fill the load ring");
  const int half = lane >> 5, col = lane & 31;
  const int wf_u = __builtin_amdgcn_readfirstlane(wf);
  const __amdgpu_buffer_rsrc_t rs = weight_rsrc(Wp + (size_t)(FB * wf_u) * KS * 512, FB * KS);
  const int lo = lane * 16;
  const __bf16* B = Hin + (32 * RB * wr + col) * LD + 8 * half;
#pragma unroll
  for (int fb = 0; fb < FB; ++fb) {
    acc[fb][0] = f32x16{};
    if (bias) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float4 c = *reinterpret_cast<const float4*>(bias + 32 * (FB * wf + fb) + 8 * j + 4 * half);
        acc[fb][0][4 * j + 0] = c.x;
        acc[fb][0][4 * j + 1] = c.y;
        acc[fb][0][4 * j + 2] = c.z;
        acc[fb][0][4 * j + 3] = c.w;
      }
    }
#pragma unroll
    for (int rb = 1; rb < RB; ++rb) acc[fb][rb] = acc[fb][0];
  }
  bf16x8 a[D][FB];
#pragma unroll
  for (int s = 0; s < D; ++s)
#pragma unroll
    for (int fb = 0; fb < FB; ++fb) a[s][fb] = load_tile(rs, lo, fb * KS + s);
  bf16x8 b[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) b[rb] = *reinterpret_cast<const bf16x8*>(B + 32 * rb * LD);
  if constexpr (kPrio) __builtin_amdgcn_s_setprio(1);
  for (int ks = 0; ks < KS; ks += D) {
#pragma unroll
    for (int s = 0; s < D; ++s) {
      const int kc = ks + s;
      bf16x8 nb[RB];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        nb[rb] = b[rb];
        if (kc + 1 < KS) nb[rb] = *reinterpret_cast<const bf16x8*>(B + 32 * rb * LD + (kc + 1) * 16);
      }
      // the next k-step's LDS reads go out before this step's MFMAs, whose in-order
      // issue then covers their latency
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int fb = 0; fb < FB; ++fb)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
          acc[fb][rb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[s][fb], b[rb], acc[fb][rb], 0, 0, 0);
      if (ks + D < KS) {
#pragma unroll
        for (int fb = 0; fb < FB; ++fb) a[s][fb] = load_tile(rs, lo, fb * KS + kc + D);
      }
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) b[rb] = nb[rb];
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  if constexpr (kPrio) __builtin_amdgcn_s_setprio(0);
}

// A square layer (W inputs) over a tile [rows][W + kLdsPad].
template <int W, int FB, int RB, int D, bool kPrio = false>
__device__ __forceinline__ void layer_mfma_fb(const __bf16* __restrict__ Wp, const __bf16* Hin, int wf, int wr,
                                              int lane, const float* __restrict__ bias, f32x16 (&acc)[FB][RB]) {
  layer_mfma_k<W, W + kLdsPad, FB, RB, D, kPrio>(Wp, Hin, wf, wr, lane, bias, acc);
}

// Parameter offsets of the residual network's block b (0-based) in the flat vector:
// Wh [W][W], Wx [W][in_dim], c, gamma, beta, mu, var [W] each; the output layer follows
// the last block, at res_block_base(W, in_dim, n_blocks).
__host__ __device__ inline size_t res_block_stride(int W, int in_dim) {
  return (size_t)W * W + (size_t)W * in_dim + 5 * (size_t)W;
}
__host__ __device__ inline size_t res_block_base(int W, int in_dim, int b) {
  return (size_t)W * in_dim + W + (size_t)b * res_block_stride(W, in_dim);
}

// Packing of a W x W weight matrix M (row-major, FP32) into MFMA A-operand order:
// element (fb, ks, lane, e) = M[fb*32 + lane%32][ks*16 + 8*(lane/32) + e], or of
// M's transpose when `transpose` is set.  o indexes the packed array of one layer.
// K: the columns of M (W for a square layer).
__device__ __forceinline__ void packed_coords(int64_t o, int K, bool transpose, int* row, int* colk) {
  const int e = (int)(o & 7);
  const int ln = (int)((o >> 3) & 63);
  const int64_t blk = o >> 9;
  const int ks = (int)(blk % (K / 16));
  const int fb = (int)(blk / (K / 16));
  const int r = fb * 32 + (ln & 31);
  const int k = ks * 16 + 8 * (ln >> 5) + e;
  *row = transpose ? k : r;
  *colk = transpose ? r : k;
}

}  // namespace sv
