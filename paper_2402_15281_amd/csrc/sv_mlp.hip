// Swept-volume network f_theta(x, q0, q1) -> delta_hat (paper Sec. IV-A, Fig. 1).
//
// Two architectures (the parameter layouts are given with sv_mlp):
//   - a plain softplus MLP: h_0 = [x; q0; q1], h_l = softplus(W_l h_{l-1} + b_l) for
//     l = 1..L, delta_hat = w_out . h_L + b_out;
//   - the paper's residual network: an initial linear layer, L blocks of linear (over
//     the block input with the network input concatenated), ReLU, BatchNorm and a skip
//     connection, and the output layer.
//
// Kernels:
//   k_mlp_f32      FP32 throughout (VALU, activations in LDS); the precise path.
//   k_pack_bf16    FP32 hidden-layer weights -> BF16 (round to nearest even), laid out in
//                  the A-operand order of v_mfma_f32_32x32x16_bf16.
//   k_mlp_bf16     fused BF16 path: layer 0 in FP32 (split into a per-motion part and a
//                  per-point part), hidden layers as BF16 MFMA with FP32 accumulation,
//                  softplus in FP32, output layer in FP32.  Optionally writes every
//                  prediction and/or appends the points with delta_hat < tau to a
//                  per-motion list (screening).
//   k_res_bf16, k_res_f32, k_pack_res, k_fold_bn: the same for the residual network.
#include <math.h>

#include "sv_geom_common.h"
#include "sv_internal.h"
#include "sv_mlp_common.h"

namespace sv {
namespace {

// Accurate softplus for the FP32 path: max(z, 0) + log1p(exp(-|z|)).
__device__ __forceinline__ float softplus_precise(float z) { return fmaxf(z, 0.f) + log1pf(expf(-fabsf(z))); }

// ----------------------------------------------------------------- FP32
// Block: 256 threads, R rows (queries) of one motion.  LDS holds the current layer's
// activations [R][W].  Thread t computes output features t, t + 256, ... for all rows.
constexpr int kF32Rows = 16;
constexpr int kF32MaxChunks = 4;   // W <= 1024

// Inputs: every (motion, point) pair of (mo, c), or with `rows` the c.n rows
// rows[i][0:in_dim] (one motion slot, m = 0).
__global__ __launch_bounds__(256) void k_mlp_f32(MlpArgs net, MotionArgs mo, CloudArgs c, int tiles,
                                                 const float* __restrict__ rows, int64_t row_stride,
                                                 float* __restrict__ out) {
  extern __shared__ float hs[];    // [kF32Rows][W]
  const int W = net.width, in_dim = net.in_dim, dof = net.dof;
  const int m = blockIdx.x / tiles;
  const int tile = blockIdx.x - m * tiles;
  const int r0 = tile * kF32Rows;
  const int tid = threadIdx.x;
  __shared__ float h0[kF32Rows][3 + 2 * SV_MAX_DOF];
  for (int e = tid; e < kF32Rows * in_dim; e += 256) {
    const int r = e / in_dim, j = e - r * in_dim;
    const int i = min(r0 + r, c.n - 1);
    float v;
    if (rows) v = rows[(size_t)i * row_stride + j];
    else if (j < 3) v = (j == 0 ? c.x : (j == 1 ? c.y : c.z))[i];
    else if (j < 3 + dof) v = mo.q0[(size_t)m * dof + (j - 3)];
    else v = mo.q1[(size_t)m * dof + (j - 3 - dof)];
    h0[r][j] = v;
  }
  __syncthreads();
  const float* p = net.params;
  // layer 0: [in_dim] -> [W]
  {
    const float* W0 = p;
    const float* b0 = p + (size_t)W * in_dim;
    for (int cch = 0; cch < kF32MaxChunks; ++cch) {
      const int f = tid + 256 * cch;
      if (f >= W) break;
      for (int r = 0; r < kF32Rows; ++r) {
        float z = b0[f];
        for (int j = 0; j < in_dim; ++j) z = fmaf(W0[(size_t)f * in_dim + j], h0[r][j], z);
        hs[r * W + f] = softplus_precise(z);
      }
    }
    p += (size_t)W * in_dim + W;
  }
  __syncthreads();
  for (int l = 1; l < net.n_hidden; ++l) {
    const float* Wl = p;
    const float* bl = p + (size_t)W * W;
    float acc[kF32MaxChunks][kF32Rows];
#pragma unroll
    for (int cch = 0; cch < kF32MaxChunks; ++cch)
#pragma unroll
      for (int r = 0; r < kF32Rows; ++r) acc[cch][r] = 0.f;
#pragma unroll
    for (int cch = 0; cch < kF32MaxChunks; ++cch) {
      const int f = tid + 256 * cch;
      if (f < W) {
        const float* wrow = Wl + (size_t)f * W;
        for (int k = 0; k < W; k += 4) {
          const float4 w4 = *reinterpret_cast<const float4*>(wrow + k);
#pragma unroll
          for (int r = 0; r < kF32Rows; ++r) {
            const float4 h4 = *reinterpret_cast<const float4*>(hs + r * W + k);
            acc[cch][r] = fmaf(w4.x, h4.x, fmaf(w4.y, h4.y, fmaf(w4.z, h4.z, fmaf(w4.w, h4.w, acc[cch][r]))));
          }
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int cch = 0; cch < kF32MaxChunks; ++cch) {
      const int f = tid + 256 * cch;
      if (f < W)
#pragma unroll
        for (int r = 0; r < kF32Rows; ++r) hs[r * W + f] = softplus_precise(acc[cch][r] + bl[f]);
    }
    __syncthreads();
    p += (size_t)W * W + W;
  }
  // output layer: one wave per row group, fixed-order reduction
  const int lane = tid & 63, wid = tid >> 6;
  for (int r = wid; r < kF32Rows; r += 4) {
    float s = 0.f;
    for (int f = lane; f < W; f += 64) s = fmaf(p[f], hs[r * W + f], s);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    const int i = r0 + r;
    if (lane == 0 && i < c.n) out[(size_t)m * c.n + i] = s + p[W];
  }
}

// ----------------------------------------------------------------- BF16
// Packed hidden-layer weights: for layer l (1..L-1), feature block fb (32 rows of W_l),
// k-step ks (16 inputs): 64 lanes x 8 BF16 = the A operand of one MFMA, where lane ln
// holds W_l[fb*32 + ln%32][ks*16 + 8*(ln/32) + e], e = 0..7.
// With `transpose`, W_l^T is packed instead (the operand of the backward pass).
__global__ void k_pack_bf16(MlpArgs net, __bf16* __restrict__ packed, __bf16* __restrict__ packedT) {
  // One lane part (8 BF16 values, 16 bytes) of each operand per thread: for row r and
  // inputs k .. k + 7 of that part, W_l[r][k .. k + 7] (two 16-byte loads) goes to
  // `packed` and W_l[k .. k + 7][r] (W_l^T's part at the same position) to `packedT`,
  // each when its pointer is set.  W is a power of two (128 .. 1024), so the position
  // splits by shifts.
  const int W = net.width;
  const int lw = 31 - __builtin_clz(W);
  const int64_t per_layer = (int64_t)1 << (2 * lw - 3);      // parts per layer
  const int64_t total = per_layer * (net.n_hidden - 1);
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < total; c += (int64_t)gridDim.x * blockDim.x) {
    const int l = (int)(c >> (2 * lw - 3));                  // 0-based hidden-layer index (layer l+2 of 1..L)
    const int64_t cl = c & (per_layer - 1);
    const int ln = (int)(cl & 63);
    const int64_t blk = cl >> 6;
    const int ks = (int)(blk & ((W >> 4) - 1)), fb = (int)(blk >> (lw - 4));
    const int r = fb * 32 + (ln & 31), k = ks * 16 + 8 * (ln >> 5);
    const float* Wl = net.params + (size_t)W * net.in_dim + W + (size_t)l * ((size_t)W * W + W);
    if (packed) {
      const float4 u = *reinterpret_cast<const float4*>(Wl + (size_t)r * W + k);
      const float4 v = *reinterpret_cast<const float4*>(Wl + (size_t)r * W + k + 4);
      const bf16x8 o = {(__bf16)u.x, (__bf16)u.y, (__bf16)u.z, (__bf16)u.w,
                        (__bf16)v.x, (__bf16)v.y, (__bf16)v.z, (__bf16)v.w};
      *reinterpret_cast<bf16x8*>(packed + 8 * c) = o;
    }
    if (packedT) {
      bf16x8 t;
#pragma unroll
      for (int e = 0; e < 8; ++e) t[e] = (__bf16)Wl[(size_t)(k + e) * W + r];
      *reinterpret_cast<bf16x8*>(packedT + 8 * c) = t;
    }
  }
}

// Block: W / (32 FB) waves, each owning FB feature blocks (32 FB output features) of
// all R = 32 RB rows (queries) of one motion, i.e. FB x RB MFMA tiles of 32 x 32.
// LDS holds one activation tile [R][K + 8] BF16 (the pad spreads rows over the LDS
// banks), updated in place: every wave reads the whole tile in a layer's MFMA loop,
// a barrier, then every wave writes its outputs, a barrier.
// The weight tiles stream from L2 through the vector L1, whose data path bounds the
// MFMA loop (RB rows per weight tile set that traffic: 1/RB KB per MFMA).  FB = 4,
// RB = 2 keeps the block at 64 rows and about 70 KB of LDS up to W = 512, so two blocks
// share a CU and one block's epilogue overlaps the other's MFMA loop; FB = 2, RB = 4
// halves the weight traffic but needs twice the LDS (one block per CU) and measures
// slower.  W = 1024 (8 waves, about 140 KB of LDS) runs one block per CU.
constexpr int kPad = kLdsPad;
constexpr int kRing = 2;               // weight-load ring depth (k-steps)
constexpr int kFB = 4;                 // feature blocks per wave
constexpr int kRB = 8 / kFB;           // row blocks per wave (FB x RB = 8 tiles, 128 accumulators)
constexpr int kBRows = 32 * kRB;       // rows per block
constexpr int kMaxIn = 3 + 2 * SV_MAX_DOF;

template <int W>
constexpr int mlp_threads() { return 64 * (W / (32 * kFB)); }
// Blocks per CU the LDS tile allows (the launch bound, so that the register budget
// matches the occupancy).
template <int W>
constexpr int mlp_blocks_per_cu() { return W <= 512 ? 2 : 1; }

// Output modes (one kernel instance each, so profiles tell the launches apart):
//   kScreen: every (motion, point) pair of (mo, c); indices of the points with
//            prediction < tau appended to lists[m][*], counts[m] advanced;
//   kDense:  every pair; prediction written to out[m][point];
//   kRows:   the c.n rows rows[i][0:in_dim] (one motion slot, m = 0; layer 0 then runs
//            unsplit per row); prediction written to out[i];
//   kMin:    every pair; the per-motion minimum over the cloud is folded into counts[m]
//            read as an order-preserving unsigned key of the float (NaN predictions are
//            skipped).
constexpr int kScreen = 0, kDense = 1, kRows = 2, kMin = 3;

// Input j of tile row r: kRows mode from h0s, else [x; q0; q1] of point xyz[r], motion m.
template <int kMode>
__device__ __forceinline__ float tile_input(const MlpArgs& net, const MotionArgs& mo, int m, const float4* xyz,
                                            const float (*h0s)[kMaxIn], int r, int j) {
  if constexpr (kMode == kRows) {
    return h0s[r][j];
  } else {
    const int dof = net.dof;
    if (j < 3) return j == 0 ? xyz[r].x : (j == 1 ? xyz[r].y : xyz[r].z);
    if (j < 3 + dof) return mo.q0[(size_t)m * dof + (j - 3)];
    return mo.q1[(size_t)m * dof + (j - 3 - dof)];
  }
}

// Layer 0 of the tile's R rows, z = W0 x_in + b0 in FP32, then softplus (kSoftplus) or
// none, rounded to BF16 into H (row stride LD).  Thread t owns the adjacent features
// 2p, 2p + 1 (p = t mod W/2) of the rows of its row group and writes them as one 32-bit
// LDS store per row.  Outside kRows mode the per-motion part of z is hoisted:
// z[f] = W0[f][0:3] . x + u[f], u[f] = W0[f][3:] . [q0; q1] + b0[f].
// Fills xyz (kRows: h0s) first; ends with a barrier.
template <int W, int NT, int R, int LD, int kMode, bool kSoftplus>
__device__ void tile_layer0(const MlpArgs& net, const MotionArgs& mo, const CloudArgs& c, const float* rows,
                            int64_t row_stride, int m, int r0, __bf16* H, float4* xyz, float (*h0s)[kMaxIn]) {
  constexpr int P = W / 2;      // feature pairs
  constexpr int RG = NT / P;    // row groups (rows R / RG each)
  static_assert(NT % P == 0 || P % NT == 0, "layer-0 mapping");
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  const int tid = threadIdx.x;
  const int dof = net.dof, in_dim = net.in_dim;
  const int pr = tid % P, rg = tid / P;
  const int ra = rg * (R / (RG > 0 ? RG : 1)), rz = ra + R / (RG > 0 ? RG : 1);
  auto act = [](float z) { return kSoftplus ? softplus_fast(z) : z; };
  if constexpr (kMode == kRows) {
    for (int e = tid; e < R * in_dim; e += NT) {
      const int r = e / in_dim, j = e - r * in_dim;
      h0s[r][j] = rows[(size_t)min(r0 + r, c.n - 1) * row_stride + j];
    }
    __syncthreads();
    float w[2][kMaxIn], b0[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int f = 2 * pr + h;
#pragma unroll
      for (int j = 0; j < kMaxIn; ++j) {
        w[h][j] = 0.f;
        if (j < in_dim) w[h][j] = net.params[(size_t)f * in_dim + j];
      }
      b0[h] = net.params[(size_t)W * in_dim + f];
    }
    for (int r = ra; r < rz; ++r) {
      float z0 = b0[0], z1 = b0[1];
#pragma unroll
      for (int j = 0; j < kMaxIn; ++j)
        if (j < in_dim) {
          z0 = fmaf(w[0][j], h0s[r][j], z0);
          z1 = fmaf(w[1][j], h0s[r][j], z1);
        }
      const bf16x2 v = {(__bf16)act(z0), (__bf16)act(z1)};
      *reinterpret_cast<bf16x2*>(H + r * LD + 2 * pr) = v;
    }
  } else {
    if (tid < R) {
      const int i = min(r0 + tid, c.n - 1);
      xyz[tid] = make_float4(c.x[i], c.y[i], c.z[i], 0.f);
    }
    __syncthreads();
    float u[2], wx[2], wy[2], wz[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int f = 2 * pr + h;
      const float* w0 = net.params + (size_t)f * in_dim;
      float uu = net.params[(size_t)W * in_dim + f];
      for (int j = 0; j < dof; ++j) {
        uu = fmaf(w0[3 + j], mo.q0[(size_t)m * dof + j], uu);
        uu = fmaf(w0[3 + dof + j], mo.q1[(size_t)m * dof + j], uu);
      }
      u[h] = uu;
      wx[h] = w0[0];
      wy[h] = w0[1];
      wz[h] = w0[2];
    }
#pragma unroll 4
    for (int r = ra; r < rz; ++r) {
      const float4 p = xyz[r];
      const float z0 = fmaf(wx[0], p.x, fmaf(wy[0], p.y, fmaf(wz[0], p.z, u[0])));
      const float z1 = fmaf(wx[1], p.x, fmaf(wy[1], p.y, fmaf(wz[1], p.z, u[1])));
      const bf16x2 v = {(__bf16)act(z0), (__bf16)act(z1)};
      *reinterpret_cast<bf16x2*>(H + r * LD + 2 * pr) = v;
    }
  }
  __syncthreads();
}

// The output stage of a tile: part[w][r] holds wave w's partial sums of the output
// layer for row r; prediction y = b_out + sum_w part[w][r], then the mode's output.
// Starts with a barrier.
template <int NW, int R, int kMode>
__device__ void tile_emit(float (*part)[R], float b_out, int r0, int m, const CloudArgs& c, float* __restrict__ out,
                          float tau, int* __restrict__ lists, int* __restrict__ counts) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  __syncthreads();
  if (wid < R / 64) {
    const int r = 64 * wid + lane;
    float y = b_out;
#pragma unroll
    for (int w = 0; w < NW; ++w) y += part[w][r];
    const int i = r0 + r;
    const bool valid = i < c.n;
    if constexpr (kMode == kDense || kMode == kRows) {
      if (valid) out[(size_t)m * c.n + i] = y;
    } else if constexpr (kMode == kMin) {
      float v = valid ? y : INFINITY;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v = fminf(v, __shfl_xor(v, off, 64));
      if (lane == 0 && v < INFINITY) atomicMin(reinterpret_cast<unsigned*>(counts) + m, ord_f32(v));
    } else {
      const bool hit = valid && y < tau;
      const unsigned long long mask = __ballot(hit);
      const int n_hit = __popcll(mask);
      int base = 0;
      if (lane == 0 && n_hit) base = atomicAdd(counts + m, n_hit);
      base = __shfl(base, 0, 64);
      const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0));
      if (hit) lists[(size_t)m * c.n + base + rank] = i;
    }
  }
}

// Lanes col and col + 32 hold disjoint features of the same rows: their sums of the
// output layer, per row block, into part[wid][row].
template <int R>
__device__ __forceinline__ void tile_partials(const float (&p)[kRB], float (*part)[R], int wid, int lane) {
  const int half = lane >> 5, col = lane & 31;
#pragma unroll
  for (int rb = 0; rb < kRB; ++rb) {
    const float q = p[rb] + __shfl_xor(p[rb], 32, 64);
    if (half == 0) part[wid][32 * rb + col] = q;
  }
}

template <int W, int kMode>
__global__ __launch_bounds__(mlp_threads<W>(), mlp_blocks_per_cu<W>()) void k_mlp_bf16(MlpArgs net, MotionArgs mo, CloudArgs c, int tiles,
                                                               const float* __restrict__ rows, int64_t row_stride,
                                                               const __bf16* __restrict__ packed,
                                                               float* __restrict__ out, float tau,
                                                               int* __restrict__ lists, int* __restrict__ counts) {
  constexpr int NT = mlp_threads<W>();   // threads
  constexpr int NW = NT / 64;            // waves
  constexpr int R = kBRows;              // rows
  constexpr int LD = W + kPad;           // LDS row stride (elements)
  extern __shared__ __align__(16) unsigned char smem[];
  __bf16* H = reinterpret_cast<__bf16*>(smem);
  __shared__ float part[NW][R];
  __shared__ float4 xyz[R];
  __shared__ float h0s[R][kMaxIn];

  const int m = blockIdx.x / tiles;
  const int tile = blockIdx.x - m * tiles;
  const int r0 = tile * R;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int in_dim = net.in_dim;
  tile_layer0<W, NT, R, LD, kMode, true>(net, mo, c, rows, row_stride, m, r0, H, xyz, h0s);

  const float* bias_base = net.params + (size_t)W * in_dim + W;   // start of layer 2
  const float* wout = bias_base + (size_t)(net.n_hidden - 1) * ((size_t)W * W + W);
  const int half = lane >> 5, col = lane & 31;
  float p[kRB];   // output-layer partial sums for rows 32 rb + col
#pragma unroll
  for (int rb = 0; rb < kRB; ++rb) p[rb] = 0.f;
  for (int l = 1; l < net.n_hidden; ++l) {
    const __bf16* Wp = packed + (size_t)(l - 1) * W * W;
    const float* bl = bias_base + (size_t)(l - 1) * ((size_t)W * W + W) + (size_t)W * W;
    f32x16 acc[kFB][kRB];
    layer_mfma_fb<W, kFB, kRB, kRing, true>(Wp, H, wid, 0, lane, bl, acc);
    const bool last = l + 1 == net.n_hidden;
    if (!last) __syncthreads();   // every wave has read the tile
    // Epilogue: acc[fb][rb][4j+i] is feature 32 (FB wid + fb) + 8j + 4 half + i of row
    // 32 rb + col (the bias is already in the accumulators).
#pragma unroll
    for (int fb = 0; fb < kFB; ++fb) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int f = 32 * (kFB * wid + fb) + 8 * j + 4 * half;
        float4 wo = make_float4(0.f, 0.f, 0.f, 0.f);
        if (last) wo = *reinterpret_cast<const float4*>(wout + f);
#pragma unroll
        for (int rb = 0; rb < kRB; ++rb) {
          const float s0 = softplus_fast(acc[fb][rb][4 * j + 0]), s1 = softplus_fast(acc[fb][rb][4 * j + 1]);
          const float s2 = softplus_fast(acc[fb][rb][4 * j + 2]), s3 = softplus_fast(acc[fb][rb][4 * j + 3]);
          if (last) {
            p[rb] = fmaf(wo.x, s0, fmaf(wo.y, s1, fmaf(wo.z, s2, fmaf(wo.w, s3, p[rb]))));
          } else {
            bf16x4 v = {(__bf16)s0, (__bf16)s1, (__bf16)s2, (__bf16)s3};
            *reinterpret_cast<bf16x4*>(H + (32 * rb + col) * LD + f) = v;
          }
        }
      }
    }
    if (!last) __syncthreads();   // the new tile is complete
  }
  if (net.n_hidden == 1) {
    // no hidden MFMA layer: output layer straight from layer 0 (FP32 accumulate of BF16 h1)
    for (int r = wid; r < R; r += NW) {
      float s = 0.f;
      for (int f = lane; f < W; f += 64) s = fmaf(wout[f], (float)H[r * LD + f], s);
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
      if (lane == 0) part[0][r] = s;
    }
    __syncthreads();
    for (int w = 1; w < NW; ++w)
      for (int r = tid; r < R; r += NT) part[w][r] = 0.f;
  } else {
    tile_partials<R>(p, part, wid, lane);
  }
  tile_emit<NW, R, kMode>(part, wout[W], r0, m, c, out, tau, lists, counts);
}

// ----------------------------------------------------------------- BF16 residual
// The paper's network (Sec. IV-A, Fig. 1) on the same tiles.  The tile has K = W +
// kResXCols columns: the block input h (BF16) and the network input x_in, each value as
// a BF16 high part and the BF16 rounding of the remainder (columns W + j and W +
// in_dim + j), zeros after.  Each block's linear layer over [h; x_in] is then one MFMA
// loop over K inputs, with packed weights [Wh | Wx | Wx | 0] and the bias c in the
// accumulators; its epilogue applies ReLU, the folded BatchNorm (scale, shift per
// feature, from k_fold_bn) and the skip connection, h += scale relu(z) + shift, in FP32
// on the BF16 block input, and stores the result in BF16 in place.  The last block's
// FP32 result feeds the output layer.


template <int W, int kMode>
__global__ __launch_bounds__(mlp_threads<W>(), mlp_blocks_per_cu<W>()) void k_res_bf16(MlpArgs net, MotionArgs mo, CloudArgs c, int tiles,
                                                               const float* __restrict__ rows, int64_t row_stride,
                                                               const __bf16* __restrict__ packed,
                                                               float* __restrict__ out, float tau,
                                                               int* __restrict__ lists, int* __restrict__ counts) {
  constexpr int NT = mlp_threads<W>();
  constexpr int NW = NT / 64;
  constexpr int R = kBRows;
  constexpr int K = W + kResXCols;
  constexpr int LD = K + kPad;
  extern __shared__ __align__(16) unsigned char smem[];
  __bf16* H = reinterpret_cast<__bf16*>(smem);
  __shared__ float part[NW][R];
  __shared__ float4 xyz[R];
  __shared__ float h0s[R][kMaxIn];

  const int m = blockIdx.x / tiles;
  const int tile = blockIdx.x - m * tiles;
  const int r0 = tile * R;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int in_dim = net.in_dim, nb = net.n_hidden;
  tile_layer0<W, NT, R, LD, kMode, false>(net, mo, c, rows, row_stride, m, r0, H, xyz, h0s);
  // the network input as BF16 high and low parts (xyz / h0s are complete: the layer-0
  // helper ends with a barrier)
  for (int e = tid; e < R * kResXCols; e += NT) {
    const int r = e / kResXCols, j = e - r * kResXCols;
    __bf16 v = (__bf16)0.f;
    if (j < 2 * in_dim) {
      const float x = tile_input<kMode>(net, mo, m, xyz, h0s, r, j < in_dim ? j : j - in_dim);
      const __bf16 hi = (__bf16)x;
      v = j < in_dim ? hi : (__bf16)(x - (float)hi);
    }
    H[r * LD + W + j] = v;
  }
  __syncthreads();

  const float2* bn = reinterpret_cast<const float2*>(packed + (size_t)nb * W * K);   // [nb][W] (scale, shift)
  const float* wout = net.params + res_block_base(W, in_dim, nb);
  const int half = lane >> 5, col = lane & 31;
  float p[kRB];
#pragma unroll
  for (int rb = 0; rb < kRB; ++rb) p[rb] = 0.f;
  for (int b = 0; b < nb; ++b) {
    const __bf16* Wp = packed + (size_t)b * W * K;
    const float* cb = net.params + res_block_base(W, in_dim, b) + (size_t)W * W + (size_t)W * in_dim;
    f32x16 acc[kFB][kRB];
    layer_mfma_k<K, LD, kFB, kRB, kRing>(Wp, H, wid, 0, lane, cb, acc);
    const bool last = b + 1 == nb;
    if (!last) __syncthreads();   // every wave has read the tile
#pragma unroll
    for (int fb = 0; fb < kFB; ++fb) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int f = 32 * (kFB * wid + fb) + 8 * j + 4 * half;
        const float4 bn01 = *reinterpret_cast<const float4*>(bn + (size_t)b * W + f);
        const float4 bn23 = *reinterpret_cast<const float4*>(bn + (size_t)b * W + f + 2);
        float4 wo = make_float4(0.f, 0.f, 0.f, 0.f);
        if (last) wo = *reinterpret_cast<const float4*>(wout + f);
#pragma unroll
        for (int rb = 0; rb < kRB; ++rb) {
          __bf16* hp = H + (32 * rb + col) * LD + f;
          const bf16x4 h = *reinterpret_cast<const bf16x4*>(hp);
          const float y0 = fmaf(bn01.x, relu_acc(acc[fb][rb][4 * j + 0]), bn01.y) + (float)h[0];
          const float y1 = fmaf(bn01.z, relu_acc(acc[fb][rb][4 * j + 1]), bn01.w) + (float)h[1];
          const float y2 = fmaf(bn23.x, relu_acc(acc[fb][rb][4 * j + 2]), bn23.y) + (float)h[2];
          const float y3 = fmaf(bn23.z, relu_acc(acc[fb][rb][4 * j + 3]), bn23.w) + (float)h[3];
          if (last) {
            p[rb] = fmaf(wo.x, y0, fmaf(wo.y, y1, fmaf(wo.z, y2, fmaf(wo.w, y3, p[rb]))));
          } else {
            const bf16x4 v = {(__bf16)y0, (__bf16)y1, (__bf16)y2, (__bf16)y3};
            *reinterpret_cast<bf16x4*>(hp) = v;
          }
        }
      }
    }
    if (!last) __syncthreads();   // the new tile is complete
  }
  tile_partials<R>(p, part, wid, lane);
  tile_emit<NW, R, kMode>(part, wout[W], r0, m, c, out, tau, lists, counts);
}

// Packed block weights of the residual network: block b is a W x K matrix [Wh | Wx |
// Wx | 0] in A-operand order (packed_coords with K columns).
__global__ void k_pack_res(MlpArgs net, __bf16* __restrict__ packed) {
  const int W = net.width, in_dim = net.in_dim, K = W + kResXCols;
  const int64_t per_block = (int64_t)W * K;
  const int64_t total = per_block * net.n_hidden;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(g / per_block);
    int f, k;
    packed_coords(g - (int64_t)b * per_block, K, false, &f, &k);
    const float* base = net.params + res_block_base(W, in_dim, b);
    float v = 0.f;
    if (k < W) v = base[(size_t)f * W + k];
    else if (k < W + 2 * in_dim) v = base[(size_t)W * W + (size_t)f * in_dim + ((k - W) % in_dim)];
    packed[g] = (__bf16)v;
  }
}

// Inference BatchNorm of block b, feature f, as scale and shift:
// scale = gamma / sqrt(var + eps), shift = beta - scale mu.
__global__ void k_fold_bn(MlpArgs net, float2* __restrict__ bn) {
  const int W = net.width, in_dim = net.in_dim;
  const int64_t total = (int64_t)net.n_hidden * W;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(g / W), f = (int)(g - (int64_t)b * W);
    const float* q = net.params + res_block_base(W, in_dim, b) + (size_t)W * W + (size_t)W * in_dim + W;
    const float gamma = q[f], beta = q[W + f], mu = q[2 * W + f], var = q[3 * W + f];
    const float scale = gamma / sqrtf(var + net.bn_eps);
    bn[g] = make_float2(scale, beta - scale * mu);
  }
}

// ----------------------------------------------------------------- FP32 residual
// The precise path of the residual network: block of 256 threads, kF32Rows rows;
// hs [R][W] holds the block input, x0 [R][in_dim] the network input.  Thread t
// computes features t, t + 256, ... of all rows.
__global__ __launch_bounds__(256) void k_res_f32(MlpArgs net, MotionArgs mo, CloudArgs c, int tiles,
                                                 const float* __restrict__ rows, int64_t row_stride,
                                                 float* __restrict__ out) {
  extern __shared__ float hs[];    // [kF32Rows][W]
  const int W = net.width, in_dim = net.in_dim, dof = net.dof;
  const int m = blockIdx.x / tiles;
  const int tile = blockIdx.x - m * tiles;
  const int r0 = tile * kF32Rows;
  const int tid = threadIdx.x;
  __shared__ float x0[kF32Rows][kMaxIn];
  for (int e = tid; e < kF32Rows * in_dim; e += 256) {
    const int r = e / in_dim, j = e - r * in_dim;
    const int i = min(r0 + r, c.n - 1);
    float v;
    if (rows) v = rows[(size_t)i * row_stride + j];
    else if (j < 3) v = (j == 0 ? c.x : (j == 1 ? c.y : c.z))[i];
    else if (j < 3 + dof) v = mo.q0[(size_t)m * dof + (j - 3)];
    else v = mo.q1[(size_t)m * dof + (j - 3 - dof)];
    x0[r][j] = v;
  }
  __syncthreads();
  const float* p = net.params;
  for (int cch = 0; cch < kF32MaxChunks; ++cch) {   // h_0 = W_0 x_in + b_0
    const int f = tid + 256 * cch;
    if (f >= W) break;
    for (int r = 0; r < kF32Rows; ++r) {
      float z = p[(size_t)W * in_dim + f];
      for (int j = 0; j < in_dim; ++j) z = fmaf(p[(size_t)f * in_dim + j], x0[r][j], z);
      hs[r * W + f] = z;
    }
  }
  __syncthreads();
  for (int b = 0; b < net.n_hidden; ++b) {
    const float* Wh = p + res_block_base(W, in_dim, b);
    const float* Wx = Wh + (size_t)W * W;
    const float* cb = Wx + (size_t)W * in_dim;
    const float* q = cb + W;   // gamma, beta, mu, var
    float acc[kF32MaxChunks][kF32Rows];
#pragma unroll
    for (int cch = 0; cch < kF32MaxChunks; ++cch) {
      const int f = tid + 256 * cch;
#pragma unroll
      for (int r = 0; r < kF32Rows; ++r) acc[cch][r] = 0.f;
      if (f < W) {
        const float* wrow = Wh + (size_t)f * W;
        for (int k = 0; k < W; k += 4) {
          const float4 w4 = *reinterpret_cast<const float4*>(wrow + k);
#pragma unroll
          for (int r = 0; r < kF32Rows; ++r) {
            const float4 h4 = *reinterpret_cast<const float4*>(hs + r * W + k);
            acc[cch][r] = fmaf(w4.x, h4.x, fmaf(w4.y, h4.y, fmaf(w4.z, h4.z, fmaf(w4.w, h4.w, acc[cch][r]))));
          }
        }
#pragma unroll
        for (int r = 0; r < kF32Rows; ++r) {
          float z = acc[cch][r] + cb[f];
          for (int j = 0; j < in_dim; ++j) z = fmaf(Wx[(size_t)f * in_dim + j], x0[r][j], z);
          acc[cch][r] = z;
        }
      }
    }
    __syncthreads();   // every thread has read the block input
#pragma unroll
    for (int cch = 0; cch < kF32MaxChunks; ++cch) {
      const int f = tid + 256 * cch;
      if (f < W) {
        const float scale = q[f] / sqrtf(q[3 * W + f] + net.bn_eps);
        const float shift = q[W + f] - scale * q[2 * W + f];
#pragma unroll
        for (int r = 0; r < kF32Rows; ++r) hs[r * W + f] += fmaf(scale, fmaxf(acc[cch][r], 0.f), shift);
      }
    }
    __syncthreads();
  }
  const float* wout = p + res_block_base(W, in_dim, net.n_hidden);
  const int lane = tid & 63, wid = tid >> 6;
  for (int r = wid; r < kF32Rows; r += 4) {
    float s = 0.f;
    for (int f = lane; f < W; f += 64) s = fmaf(wout[f], hs[r * W + f], s);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    const int i = r0 + r;
    if (lane == 0 && i < c.n) out[(size_t)m * c.n + i] = s + wout[W];
  }
}

inline unsigned grid_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

// One launch of the BF16 kernel (k_mlp_bf16 or, for a residual network, k_res_bf16).
template <int W, int kMode>
hipError_t launch_bf16_mode(const MlpArgs& net, const MotionArgs& mo, const CloudArgs& c, const float* rows,
                            int64_t row_stride, const __bf16* packed, float* out, float tau, int* lists, int* counts,
                            hipStream_t st) {
  const int tiles = (c.n + kBRows - 1) / kBRows;
  const int64_t blocks = (kMode == kRows ? 1 : mo.n) * tiles;
  if (blocks == 0) return hipSuccess;
  const bool res = net.kind == SV_NET_RESIDUAL;
  const size_t lds = (size_t)kBRows * ((res ? W + kResXCols : W) + kPad) * sizeof(__bf16);
  auto kern = res ? &k_res_bf16<W, kMode> : &k_mlp_bf16<W, kMode>;
  static bool attr_set[2] = {false, false};
  if (!attr_set[res]) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    attr_set[res] = true;
  }
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(mlp_threads<W>()), lds, st, net, mo, c, tiles, rows,
                     row_stride, packed, out, tau, lists, counts);
  return hipGetLastError();
}

template <int W>
hipError_t launch_bf16_t(const MlpArgs& net, const MotionArgs& mo, const CloudArgs& c, const float* rows,
                         int64_t row_stride, const __bf16* packed, float* out, float tau, int* lists, int* counts,
                         hipStream_t st) {
  if (rows) return launch_bf16_mode<W, kRows>(net, mo, c, rows, row_stride, packed, out, tau, lists, counts, st);
  if (lists) return launch_bf16_mode<W, kScreen>(net, mo, c, rows, row_stride, packed, out, tau, lists, counts, st);
  return launch_bf16_mode<W, kDense>(net, mo, c, rows, row_stride, packed, out, tau, lists, counts, st);
}

hipError_t launch_f32(const MlpArgs& net, const MotionArgs& mo, const CloudArgs& c, const float* rows,
                      int64_t row_stride, float* out, hipStream_t st) {
  const int tiles = (c.n + kF32Rows - 1) / kF32Rows;
  const int64_t blocks = (rows ? 1 : mo.n) * tiles;
  if (blocks == 0) return hipSuccess;
  const size_t lds = (size_t)kF32Rows * net.width * sizeof(float);
  const bool res = net.kind == SV_NET_RESIDUAL;
  auto kern = res ? &k_res_f32 : &k_mlp_f32;
  static bool attr_set[2] = {false, false};
  if (!attr_set[res]) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                       65536);
    if (e != hipSuccess) return e;
    attr_set[res] = true;
  }
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(256), lds, st, net, mo, c, tiles, rows, row_stride, out);
  return hipGetLastError();
}

}  // namespace

bool mlp_bf16_supported(int width) { return width == 128 || width == 256 || width == 512 || width == 1024; }

size_t mlp_packed_elems(const MlpArgs& net) {
  const size_t W = (size_t)net.width;
  if (net.kind == SV_NET_RESIDUAL)   // block weights, then (scale, shift) per block and feature: 4 BF16 slots
    return (size_t)net.n_hidden * W * (W + kResXCols) + (size_t)net.n_hidden * W * 4;
  return W * W * (net.n_hidden - 1);
}

hipError_t launch_mlp_f32(const MlpArgs& net, const MotionArgs& mo, const CloudArgs& c, float* out, hipStream_t st) {
  return launch_f32(net, mo, c, nullptr, 0, out, st);
}

hipError_t launch_mlp_rows(const MlpArgs& net, int bf16, const __bf16* packed, const float* rows, int64_t row_stride,
                           int64_t n, float* out, hipStream_t st) {
  const MotionArgs none{SV_LINEAR, 1, 1, nullptr, nullptr, nullptr};
  const CloudArgs c{(int)n, nullptr, nullptr, nullptr};
  if (!bf16) return launch_f32(net, none, c, rows, row_stride, out, st);
  switch (net.width) {
    case 128: return launch_bf16_t<128>(net, none, c, rows, row_stride, packed, out, 0.f, nullptr, nullptr, st);
    case 256: return launch_bf16_t<256>(net, none, c, rows, row_stride, packed, out, 0.f, nullptr, nullptr, st);
    case 512: return launch_bf16_t<512>(net, none, c, rows, row_stride, packed, out, 0.f, nullptr, nullptr, st);
    case 1024: return launch_bf16_t<1024>(net, none, c, rows, row_stride, packed, out, 0.f, nullptr, nullptr, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pack_bf16(const MlpArgs& net, int transpose, __bf16* packed, hipStream_t st) {
  if (net.kind == SV_NET_RESIDUAL) {
    if (transpose) return hipErrorInvalidValue;   // the transposed pack serves training only
    const int64_t wt = (int64_t)net.n_hidden * net.width * (net.width + kResXCols);
    hipLaunchKernelGGL(k_pack_res, dim3((unsigned)std::min<int64_t>(grid_for(wt, 256), 4096)), dim3(256), 0, st, net,
                       packed);
    const int64_t nbn = (int64_t)net.n_hidden * net.width;
    hipLaunchKernelGGL(k_fold_bn, dim3((unsigned)std::min<int64_t>(grid_for(nbn, 256), 1024)), dim3(256), 0, st, net,
                       reinterpret_cast<float2*>(packed + wt));
    return hipGetLastError();
  }
  const int64_t total = (int64_t)mlp_packed_elems(net);
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pack_bf16, dim3((unsigned)std::min<int64_t>(grid_for(total / 8, 256), 4096)), dim3(256), 0, st,
                     net, transpose ? nullptr : packed, transpose ? packed : nullptr);
  return hipGetLastError();
}

hipError_t launch_pack_bf16_both(const MlpArgs& net, __bf16* packed, __bf16* packedT, hipStream_t st) {
  if (net.kind == SV_NET_RESIDUAL) return hipErrorInvalidValue;
  const int64_t total = (int64_t)mlp_packed_elems(net);
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pack_bf16, dim3((unsigned)std::min<int64_t>(grid_for(total / 8, 256), 4096)), dim3(256), 0, st,
                     net, packed, packedT);
  return hipGetLastError();
}

hipError_t launch_mlp_min(const MlpArgs& net, const MotionArgs& mo, const CloudArgs& c, const __bf16* packed,
                          unsigned* min_keys, hipStream_t st) {
  int* k = reinterpret_cast<int*>(min_keys);
  switch (net.width) {
    case 128: return launch_bf16_mode<128, kMin>(net, mo, c, nullptr, 0, packed, nullptr, 0.f, nullptr, k, st);
    case 256: return launch_bf16_mode<256, kMin>(net, mo, c, nullptr, 0, packed, nullptr, 0.f, nullptr, k, st);
    case 512: return launch_bf16_mode<512, kMin>(net, mo, c, nullptr, 0, packed, nullptr, 0.f, nullptr, k, st);
    case 1024: return launch_bf16_mode<1024, kMin>(net, mo, c, nullptr, 0, packed, nullptr, 0.f, nullptr, k, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_mlp_bf16(const MlpArgs& net, const MotionArgs& mo, const CloudArgs& c, const __bf16* packed,
                           float* out, float tau, int* lists, int* counts, hipStream_t st) {
  switch (net.width) {
    case 128: return launch_bf16_t<128>(net, mo, c, nullptr, 0, packed, out, tau, lists, counts, st);
    case 256: return launch_bf16_t<256>(net, mo, c, nullptr, 0, packed, out, tau, lists, counts, st);
    case 512: return launch_bf16_t<512>(net, mo, c, nullptr, 0, packed, out, tau, lists, counts, st);
    case 1024: return launch_bf16_t<1024>(net, mo, c, nullptr, 0, packed, out, tau, lists, counts, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sv
