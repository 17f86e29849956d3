// Training step of the swept-volume network on samples (x, q0, q1, delta) produced by
// the exact check (paper Sec. IV-C: training tuples; Sec. V: Adam with PyTorch's
// default constants).  Loss: mean over the batch of |y - clamp(delta)|, clamp to
// [-sigma, sigma] on the targets only, or mean |clamp(y) - clamp(delta)| (clamp_pred;
// DeepSDF's form: no gradient where |y| >= sigma).  BF16 hidden layers on
// MFMA with FP32 accumulation, FP32 first and output layers, FP32 master weights,
// FP32 Adam state.
//
// Workspace layouts (Bp = batch rounded up to 256 rows; rows >= batch carry zero
// gradient):
//   aT[l][b/64][f][b%64]   BF16 activation of hidden layer l+1 (64-row tiles,
//                          feature-major within a tile; tix())
//   dzT[l][b/64][f][b%64]  BF16 gradient w.r.t. the pre-activation of hidden layer l+1
//   h0T[j][b]     FP32 network input, feature-major
//   y[b], dy[b]   FP32 prediction and d loss / d y
// Kernels, in launch order:
//   k_pack_bf16       W_l and W_l^T in MFMA operand order, one launch (sv_mlp.hip)
//   k_train_fwd       per 64-row tile: all layers, activations to aT, y, dy and the
//                     tile's sum of the loss terms (the inference kernel's tile shape,
//                     one in-place LDS tile, two blocks per CU)
//   k_train_loss_sum  the loss (fixed-order sum of the tiles' sums)
//   k_train_bwd       per 64-row tile: dz of every layer via W_l^T MFMA, to dzT
//   k_grad_w          dW_l = dz_l^T a_{l-1} for l >= 2 (MFMA, split over the batch; both
//                     operands staged in LDS)
//   k_grad_reduce     fixed-order sum of the splits
//   k_grad_out        w_out and b_out gradients (blocks stream runs of tiles) + fixed-order
//                     sum of the blocks' partials
//   k_grad_w1         dW_1 = dz_1^T h0 and db_1 on MFMA (the FP32 input as BF16 high and
//                     low parts, a column of ones for the bias; split over the batch) +
//                     fixed-order sum (db_l for l >= 2 is summed by k_grad_w from its
//                     staged dz rows)
//   k_adam            Adam update of the FP32 masters
#include <math.h>

#include "sv_internal.h"
#include "sv_mlp_common.h"

namespace sv {
namespace {

constexpr int kRows = kTileRows;
constexpr int kSplitW = 9;        // batch splits of the dW GEMM (8 x 512: 7 layers x 9 x 4 tiles = 252 blocks, one round on 256 CUs)
constexpr int kGwXcd = 1;         // 1: the tiles of one (layer, split) on one XCD

struct TrainArgs {
  MlpArgs net;
  const float* samples;   // [n][in_dim + 1]
  const int* idx;         // [B]
  int B, Bp;
  __bf16* aT;             // [L][Bp / 64][W][64]
  __bf16* dzT;            // [L][Bp / 64][W][64]
  float* h0T;             // [in_dim][Bp]
  float* y;               // [Bp]
  float* dy;              // [Bp]
  const __bf16* packed;   // forward operands, layers 2..L
  const __bf16* packedT;  // backward operands, layers 2..L
  float* grad;            // [n_params]
  int clamp_pred;         // 1: the loss clamps the prediction as well as the target
  float sigma;            // the loss clamp
  float* loss_part;       // [Bp / 64] the forward's per-tile sums of the loss terms
};

// Parameter offsets of the flat vector (see sv_mlp in sv.h), 1-based layer l.
__host__ __device__ inline size_t off_w(const MlpArgs& n, int l) {
  const size_t W = n.width;
  return l == 1 ? 0 : W * n.in_dim + W + (size_t)(l - 2) * (W * W + W);
}
__host__ __device__ inline size_t off_b(const MlpArgs& n, int l) {
  const size_t W = n.width;
  return off_w(n, l) + (l == 1 ? W * n.in_dim : W * W);
}
__host__ __device__ inline size_t off_out(const MlpArgs& n) {
  const size_t W = n.width;
  return W * n.in_dim + W + (size_t)(n.n_hidden - 1) * (W * W + W);
}

// Forward and backward tiles: 64 rows (samples) per block; each wave owns kTFB feature
// blocks (32 kTFB output features) of both row blocks, the inference kernel's shape.
// One activation tile [64][W + pad] in LDS, updated in place, so two blocks share a CU.
constexpr int kTFB = 4, kTRB = 2;
template <int W>
constexpr int train_threads() { return 64 * (W / (32 * kTFB)); }

// Layout of each layer's block of aT and dzT (W x Bp BF16 values): tiles of 64 batch
// rows, each holding its W features' 64 values in a row, so that one tile's layer is
// 64 KB of consecutive memory (at W = 512) and a feature's values of one tile are one
// 128-byte line.  Element (feature f, batch row b) of a block:
__host__ __device__ inline size_t tix(int W, int f, int b) { return ((size_t)(b >> 6) * W + f) * 64 + (b & 63); }

// The activation and dz streams (hundreds of MB per step, each byte read once by the
// next kernel) are written and read with the non-temporal cache policy, so that they do
// not push the packed weights (3.7 MB, read by every tile) out of L2: 1.14 -> 1.07 ms per
// training step (8 x 512, batch 65,536).
//
// Copy the LDS tile H[64][LD] (features 0..W-1) to the layer block outT (features f, rows r0 .. r0 + 63) in blocks
// of 8 rows x 8 features: a lane reads its block with eight 16-byte LDS reads (rows),
// transposes it in registers and writes eight 16-byte stores (features).  In a wave the
// lane's feature group runs fastest (conflict-free LDS reads: the 8 groups of a phase
// cover all banks) and its row group slowest (the 8 row groups of a feature write one
// 128-byte line).
template <int W, int NT, int LD = W + kLdsPad>
__device__ __forceinline__ void store_tile_T(const __bf16* H, __bf16* outT, int r0) {
  static_assert(kRows == 64, "8 row groups of 8");
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int rg = lane >> 3;   // rows 8 rg .. 8 rg + 7
#pragma unroll 1
  for (int fb = w; fb < W / 64; fb += NW) {
    const int fg = 8 * fb + (lane & 7);   // features 8 fg .. 8 fg + 7
    bf16x8 in[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) in[r] = *reinterpret_cast<const bf16x8*>(H + (8 * rg + r) * LD + 8 * fg);
#pragma unroll
    for (int f = 0; f < 8; ++f) {
      bf16x8 o;
#pragma unroll
      for (int r = 0; r < 8; ++r) o[r] = in[r][f];
      __builtin_nontemporal_store(o, reinterpret_cast<bf16x8*>(outT + tix(W, 8 * fg + f, r0 + 8 * rg)));
    }
  }
}

// The inverse: features f, rows r0 .. r0 + 63 of the layer block inT into the LDS tile H[64][LD],
// with the same 8 x 8 blocks and lane order.
template <int W, int NT, int LD = W + kLdsPad>
__device__ __forceinline__ void load_tile_T(const __bf16* inT, __bf16* H, int r0) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int rg = lane >> 3;
#pragma unroll 1
  for (int fb = w; fb < W / 64; fb += NW) {
    const int fg = 8 * fb + (lane & 7);
    bf16x8 in[8];
#pragma unroll
    for (int f = 0; f < 8; ++f) in[f] = *reinterpret_cast<const bf16x8*>(inT + tix(W, 8 * fg + f, r0 + 8 * rg));
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      bf16x8 o;
#pragma unroll
      for (int f = 0; f < 8; ++f) o[f] = in[f][r];
      *reinterpret_cast<bf16x8*>(H + (8 * rg + r) * LD + 8 * fg) = o;
    }
  }
}

// load_tile_T in two halves: the global loads into registers (issued before the
// layer's MFMA loop, so that they are in flight during it), then the transposed LDS
// writes.
template <int W, int NT>
__device__ __forceinline__ void fetch_tile_T(const __bf16* inT, int r0, bf16x8 (&in)[W / 64 / (NT / 64)][8]) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int rg = lane >> 3;
#pragma unroll
  for (int q = 0; q < W / 64 / NW; ++q) {
    const int fg = 8 * (w + q * NW) + (lane & 7);
#pragma unroll
    for (int f = 0; f < 8; ++f) in[q][f] = __builtin_nontemporal_load(reinterpret_cast<const bf16x8*>(inT + tix(W, 8 * fg + f, r0 + 8 * rg)));
  }
}
template <int W, int NT, int LD = W + kLdsPad>
__device__ __forceinline__ void put_tile_T(const bf16x8 (&in)[W / 64 / (NT / 64)][8], __bf16* H) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int rg = lane >> 3;
#pragma unroll
  for (int q = 0; q < W / 64 / NW; ++q) {
    const int fg = 8 * (w + q * NW) + (lane & 7);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      bf16x8 o;
#pragma unroll
      for (int f = 0; f < 8; ++f) o[f] = in[q][f][r];
      *reinterpret_cast<bf16x8*>(H + (8 * rg + r) * LD + 8 * fg) = o;
    }
  }
}

template <int W>
__global__ __launch_bounds__(train_threads<W>(), 2) void k_train_fwd(TrainArgs a) {
  constexpr int NT = train_threads<W>(), NW = NT / 64;
  constexpr int LD = W + kLdsPad;
  constexpr int kMaxIn = 3 + 2 * SV_MAX_DOF;
  constexpr int kInPad = (kMaxIn + 3) / 4 * 4;   // input row padded with zeros to whole float4s
  constexpr int FPT = W / NT;                     // first-layer features per thread
  static_assert(FPT * NT == W, "whole features per thread");
  extern __shared__ __align__(16) unsigned char smem[];
  __bf16* H = reinterpret_cast<__bf16*>(smem);
  __shared__ __align__(16) float h0s[kRows][kInPad];
  __shared__ float part[NW][kRows];
  const MlpArgs& n = a.net;
  const int in_dim = n.in_dim, L = n.n_hidden;
  const int r0 = blockIdx.x * kRows;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int half = lane >> 5, col = lane & 31;
  for (int e = tid; e < kRows * kInPad; e += NT) {
    const int r = e / kInPad, j = e - r * kInPad;
    float v = 0.f;
    if (j < in_dim) {
      const int b = min(r0 + r, a.B - 1);
      v = a.samples[(size_t)a.idx[b] * (in_dim + 1) + j];
    }
    h0s[r][j] = v;
  }
  __syncthreads();
  // the inputs feature-major for the dW_1 kernel: consecutive threads on consecutive rows
  for (int e = tid; e < kRows * in_dim; e += NT) {
    const int j = e / kRows, r = e - j * kRows;
    a.h0T[(size_t)j * a.Bp + r0 + r] = h0s[r][j];
  }
  // Layer 1 in FP32, FPT features per thread.  Inputs and weights past in_dim are zero,
  // so the fixed-length chain adds exact zeros after the in_dim real terms.
  float w[FPT][kInPad], b1[FPT];
#pragma unroll
  for (int q = 0; q < FPT; ++q) {
    const int f = tid + q * NT;
    const float* w1 = n.params + (size_t)f * in_dim;
    b1[q] = n.params[off_b(n, 1) + f];
#pragma unroll
    for (int j = 0; j < kInPad; ++j) w[q][j] = j < in_dim ? w1[j] : 0.f;
  }
#pragma unroll 2
  for (int r = 0; r < kRows; ++r) {
    float h[kInPad];
#pragma unroll
    for (int j = 0; j < kInPad; j += 4) {
      const float4 v = *reinterpret_cast<const float4*>(&h0s[r][j]);
      h[j] = v.x; h[j + 1] = v.y; h[j + 2] = v.z; h[j + 3] = v.w;
    }
#pragma unroll
    for (int q = 0; q < FPT; ++q) {
      float z = b1[q];
#pragma unroll
      for (int j = 0; j < kInPad; ++j) z = fmaf(w[q][j], h[j], z);
      H[r * LD + tid + q * NT] = (__bf16)softplus_fast(z);
    }
  }
  __syncthreads();
  store_tile_T<W, NT>(H, a.aT, r0);
  float p[kTRB] = {0.f, 0.f};
  const float* wout = n.params + off_out(n);
  for (int l = 2; l <= L; ++l) {
    f32x16 acc[kTFB][kTRB];
    layer_mfma_fb<W, kTFB, kTRB, 2, true>(a.packed + (size_t)(l - 2) * W * W, H, wid, 0, lane, n.params + off_b(n, l),
                                    acc);
    const bool last = l == L;
    __syncthreads();   // every wave has read the tile (and copied it out)
#pragma unroll
    for (int fb = 0; fb < kTFB; ++fb)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int f = 32 * (kTFB * wid + fb) + 8 * j + 4 * half;
        float4 wo = make_float4(0.f, 0.f, 0.f, 0.f);
        if (last) wo = *reinterpret_cast<const float4*>(wout + f);
#pragma unroll
        for (int rb = 0; rb < kTRB; ++rb) {
          const float s0 = softplus_fast(acc[fb][rb][4 * j + 0]), s1 = softplus_fast(acc[fb][rb][4 * j + 1]);
          const float s2 = softplus_fast(acc[fb][rb][4 * j + 2]), s3 = softplus_fast(acc[fb][rb][4 * j + 3]);
          if (last) p[rb] = fmaf(wo.x, s0, fmaf(wo.y, s1, fmaf(wo.z, s2, fmaf(wo.w, s3, p[rb]))));
          const bf16x4 v = {(__bf16)s0, (__bf16)s1, (__bf16)s2, (__bf16)s3};
          *reinterpret_cast<bf16x4*>(H + (32 * rb + col) * LD + f) = v;
        }
      }
    __syncthreads();   // the new tile is complete
    store_tile_T<W, NT>(H, a.aT + (size_t)(l - 1) * W * a.Bp, r0);
  }
  if (L == 1) {
    for (int r = wid; r < kRows; r += NW) {
      float s = 0.f;
      for (int f = lane; f < W; f += 64) s = fmaf(wout[f], (float)H[r * LD + f], s);
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
      if (lane == 0) part[0][r] = s;
    }
    for (int w = 1; w < NW; ++w)
      if (tid < kRows) part[w][tid] = 0.f;
  } else {
#pragma unroll
    for (int rb = 0; rb < kTRB; ++rb) {
      const float q = p[rb] + __shfl_xor(p[rb], 32, 64);
      if (half == 0) part[wid][32 * rb + col] = q;
    }
  }
  __syncthreads();
  if (tid < kRows) {   // wave 0: row r0 + lane
    float yv = wout[W];
#pragma unroll
    for (int w = 0; w < NW; ++w) yv += part[w][tid];
    const int b = r0 + tid;
    a.y[b] = yv;
    // the loss term and dy of the row; rows past the batch carry neither
    float s = 0.f, g = 0.f;
    if (b < a.B) {
      const float sg = a.sigma;
      const float d = a.samples[(size_t)a.idx[b] * (in_dim + 1) + in_dim];
      const bool live = !a.clamp_pred || fabsf(yv) < sg;   // d clamp(y) / dy
      const float yc = a.clamp_pred ? fminf(fmaxf(yv, -sg), sg) : yv;
      const float r = yc - fminf(fmaxf(d, -sg), sg);
      s = fabsf(r);
      g = live ? (r > 0.f ? 1.f : (r < 0.f ? -1.f : 0.f)) / (float)a.B : 0.f;
    }
    a.dy[b] = g;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);   // fixed order
    if (tid == 0) a.loss_part[blockIdx.x] = s;
  }
}

// The loss: the sum of the forward's per-tile sums in a fixed order, / B.
__global__ __launch_bounds__(1024) void k_train_loss_sum(TrainArgs a, const float* __restrict__ part, int n,
                                                         float* __restrict__ loss_out) {
  __shared__ float red[1024];
  float s = 0.f;
  for (int i = threadIdx.x; i < n; i += 1024) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss_out) *loss_out = red[0] / (float)a.B;
}

template <int W>
__global__ __launch_bounds__(train_threads<W>(), 2) void k_train_bwd(TrainArgs a) {
  constexpr int NT = train_threads<W>();
  constexpr int LD = W + kLdsPad;
  extern __shared__ __align__(16) unsigned char smem[];
  __bf16* H = reinterpret_cast<__bf16*>(smem);
  const MlpArgs& n = a.net;
  const int L = n.n_hidden;
  const int r0 = blockIdx.x * kRows;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int half = lane >> 5, col = lane & 31;
  {   // dz_L = dy * w_out * sigma(z_L), in the 8 x 8 blocks of fetch_tile_T (16-byte loads
      // and stores of feature rows, transposed writes into the LDS tile)
    constexpr int NQ = W / 64 / (NT / 64);
    const int rg = lane >> 3;
    bf16x8 av[NQ][8];
    fetch_tile_T<W, NT>(a.aT + (size_t)(L - 1) * W * a.Bp, r0, av);
    const float4 d0 = *reinterpret_cast<const float4*>(a.dy + r0 + 8 * rg);
    const float4 d1 = *reinterpret_cast<const float4*>(a.dy + r0 + 8 * rg + 4);
    const float dyv[8] = {d0.x, d0.y, d0.z, d0.w, d1.x, d1.y, d1.z, d1.w};
    __bf16* dzL = a.dzT + (size_t)(L - 1) * W * a.Bp;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int fg = 8 * (wid + q * (NT / 64)) + (lane & 7);
#pragma unroll
      for (int f = 0; f < 8; ++f) {
        const float wo = n.params[off_out(n) + 8 * fg + f];
        bf16x8 out;
#pragma unroll
        for (int e = 0; e < 8; ++e) out[e] = (__bf16)(dyv[e] * wo * softplus_grad_from_out((float)av[q][f][e]));
        av[q][f] = out;
        __builtin_nontemporal_store(out, reinterpret_cast<bf16x8*>(dzL + tix(W, 8 * fg + f, r0 + 8 * rg)));
      }
    }
    put_tile_T<W, NT>(av, H);
  }
  __syncthreads();
  for (int l = L; l >= 2; --l) {
    // dh_{l-1}[r][k] = sum_f dz_l[r][f] W_l[f][k]: A operand = W_l^T packed
    bf16x8 pre[W / 64 / (NT / 64)][8];   // the activations of layer l - 1, in flight during the MFMAs
    fetch_tile_T<W, NT>(a.aT + (size_t)(l - 2) * W * a.Bp, r0, pre);
    f32x16 acc[kTFB][kTRB];
    layer_mfma_fb<W, kTFB, kTRB, 2, true>(a.packedT + (size_t)(l - 2) * W * W, H, wid, 0, lane, nullptr, acc);
    __syncthreads();   // every wave has read the tile (and copied it out)
    put_tile_T<W, NT>(pre, H);   // into the free tile, then dz_{l-1} over them in place
    __syncthreads();
#pragma unroll
    for (int fb = 0; fb < kTFB; ++fb)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = 32 * (kTFB * wid + fb) + 8 * j + 4 * half;
#pragma unroll
        for (int rb = 0; rb < kTRB; ++rb) {
          bf16x4* hp = reinterpret_cast<bf16x4*>(H + (32 * rb + col) * LD + k);
          const bf16x4 ap = *hp;
          bf16x4 v;
#pragma unroll
          for (int i = 0; i < 4; ++i) v[i] = (__bf16)(acc[fb][rb][4 * j + i] * softplus_grad_from_out((float)ap[i]));
          *hp = v;
        }
      }
    __syncthreads();   // the new tile is complete
    store_tile_T<W, NT>(H, a.dzT + (size_t)(l - 2) * W * a.Bp, r0);
  }
}

// Partial dW_l[f][k] = sum over one batch split of dz_l[f][b] a_{l-1}[k][b], l >= 2.
// Both operands are batch-contiguous rows ([feature][batch]), so a block (a TF x TK tile
// of dW_l) stages chunks of kGwChunk batch rows of its TF dz rows and TK activation
// rows in LDS and its 4 waves read the MFMA fragments from there: wave (wf, wk) owns
// rows (TF / 2) wf .. and columns (TK / 2) wk .. as (TF / 64) x (TK / 64) tiles of
// 32 x 32.  At W >= 256 the block tile is 256 x 256 (256 accumulator registers per
// lane, one wave per SIMD, one block per CU).  The kernel is bound by the bytes in
// flight per CU: the chunks are moved by direct-to-LDS loads (global_load_lds_dwordx4,
// no registers), kGwStages LDS buffers deep, so that kGwStages - 1 chunks are in flight
// while the MFMAs run on one.  A chunk row is 64 contiguous bytes (4 segments of 16);
// the DMA writes each wave's 64 segments to 1 KB of consecutive LDS, so the swizzle
// that keeps the fragment reads free of bank conflicts is applied on the global side:
// LDS slot s' of row r holds segment s' ^ ((r >> 1) & 3).  The waits are explicit vmcnt
// counts with raw barriers (a __syncthreads would wait for every load in flight); each
// buffer is its own LDS variable and the loop is unrolled over them, so that the
// compiler can tell the buffers apart (it still adds a full wait before one of the four
// buffers' reads).
constexpr int kGwChunk = 32;                   // batch rows per LDS stage (two MFMA k-steps)
constexpr int kGwStages = 4;                   // LDS buffers
constexpr int kGwStageElems = 512 * kGwChunk;  // (TF + TK) rows at most
__shared__ __align__(16) __bf16 gw_buf0[kGwStageElems];
__shared__ __align__(16) __bf16 gw_buf1[kGwStageElems];
__shared__ __align__(16) __bf16 gw_buf2[kGwStageElems];
__shared__ __align__(16) __bf16 gw_buf3[kGwStageElems];
template <int B>
__device__ __forceinline__ __bf16* gw_buf() {
  return B == 0 ? gw_buf0 : B == 1 ? gw_buf1 : B == 2 ? gw_buf2 : gw_buf3;
}
__device__ __forceinline__ int gw_slot(int r, int seg) { return seg ^ ((r >> 1) & 3); }

template <int W>
constexpr int gw_tk() { return W >= 256 ? 256 : W; }   // output columns per block
template <int W>
constexpr int gw_tf() { return W >= 256 ? 256 : W; }   // output rows per block

// Block -> (column tile tk, row tile tf, split s, layer l).  The tiles of one (layer,
// split) read the same dz and activation rows; the 4 (at W = 512) are given block
// indices 8 apart, which the dispatcher deals to the same XCD, so that the rows one
// tile fetches are found in that XCD's L2 by the others.  Blocks past the last whole
// group of 8 (layer, split) pairs keep the plain order.
template <int W>
__device__ __forceinline__ void gw_coords(int b, int nblocks, int* tk, int* tf, int* s, int* l) {
  constexpr int NT = (W / gw_tk<W>()) * (W / gw_tf<W>());   // tiles per (layer, split)
  int g, t;
  if (kGwXcd && NT > 1 && b < nblocks / (8 * NT) * (8 * NT)) {
    const int sg = b / (8 * NT), r = b - sg * 8 * NT;
    g = sg * 8 + (r & 7);
    t = r >> 3;
  } else {
    g = b / NT;
    t = b - g * NT;
  }
  *tk = t % (W / gw_tk<W>());
  *tf = t / (W / gw_tk<W>());
  *s = g % kSplitW;
  *l = g / kSplitW + 2;
}

// vmcnt(n) for the waits of k_grad_w (n loads of this wave still in flight).
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

template <int W>
struct GwCtx {
  static constexpr int TF = gw_tf<W>(), TK = gw_tk<W>();
  static constexpr int NQ = (TF + TK) * (kGwChunk / 8) / 256;   // 16-byte loads per thread and chunk
  const __bf16* dz;
  const __bf16* ap;
  int f0, k0, b_begin, nch, tid, wid, lane;
  int off[NQ];   // element offset of this thread's q-th segment from its chunk's start
};

// The direct-to-LDS loads of chunk c (batch rows b_begin + kGwChunk c ..) into buffer B.
template <int W, int B>
__device__ __forceinline__ void gw_issue(const GwCtx<W>& x, int c) {
  using C = GwCtx<W>;
  const int b = x.b_begin + kGwChunk * c;          // a multiple of 32: the chunk lies in one 64-row tile
  const size_t base = (size_t)(b >> 6) * W * 64 + (b & 63);
#pragma unroll
  for (int q = 0; q < C::NQ; ++q) {
    // rows 64 q + tid / 4: the first TF are dz rows (q < NQ / 2 when TF == TK)
    const __bf16* src = (64 * q < C::TF ? x.dz : x.ap) + base + x.off[q];
    __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)(gw_buf<B>() + (256 * q + 64 * x.wid) * 8),
                                     16, 0, 0);
  }
}

// Step c on buffer B: wait for chunk c, refill the buffer freed by step c - 1 with chunk
// c + kGwStages - 1, add the bias sums and run the MFMAs of the chunk.
template <int W, int B>
__device__ __forceinline__ void gw_step(const GwCtx<W>& x, int c, bool bias, float& dbs,
                                       f32x16 (&acc)[gw_tf<W>() / 64][gw_tk<W>() / 64]) {
  using C = GwCtx<W>;
  constexpr int TF = C::TF, TK = C::TK, NQ = C::NQ, FBW = TF / 64, RB = TK / 64;
  // chunks issued after c that may still be in flight: min(nch - 1 - c, kGwStages - 2)
  const int later = min(x.nch - 1 - c, kGwStages - 2);
  if (later >= 2) wait_vm<2 * NQ>();
  else if (later == 1) wait_vm<NQ>();
  else wait_vm<0>();
  __builtin_amdgcn_s_barrier();                    // chunk c has landed for every wave; c - 1 is consumed
  if (c + kGwStages - 1 < x.nch) gw_issue<W, (B + kGwStages - 1) % kGwStages>(x, c + kGwStages - 1);
  const __bf16* S = gw_buf<B>();
  const int half = x.lane >> 5, col = x.lane & 31, wf = x.wid & 1, wk = x.wid >> 1;
  if (bias) {   // db_l[f] = sum_b dz_l[f][b]: 256 / TF threads per row
    constexpr int TPR = 256 / TF, SPT = 4 / TPR;   // segments per thread
    const int r = x.tid / TPR;
#pragma unroll
    for (int u = 0; u < SPT; ++u) {
      const bf16x8 v = *reinterpret_cast<const bf16x8*>(S + r * kGwChunk + 8 * gw_slot(r, SPT * (x.tid % TPR) + u));
#pragma unroll
      for (int e = 0; e < 8; ++e) dbs += (float)v[e];
    }
  }
#pragma unroll
  for (int ks = 0; ks < kGwChunk / 16; ++ks) {
    bf16x8 xa[FBW], yb[RB];
#pragma unroll
    for (int fb = 0; fb < FBW; ++fb) {
      const int r = (TF / 2) * wf + 32 * fb + col;
      xa[fb] = *reinterpret_cast<const bf16x8*>(S + r * kGwChunk + 8 * gw_slot(r, 2 * ks + half));
    }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const int r = TF + (TK / 2) * wk + 32 * rb + col;
      yb[rb] = *reinterpret_cast<const bf16x8*>(S + r * kGwChunk + 8 * gw_slot(r, 2 * ks + half));
    }
#pragma unroll
    for (int fb = 0; fb < FBW; ++fb)
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
        acc[fb][rb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa[fb], yb[rb], acc[fb][rb], 0, 0, 0);
  }
}

template <int W>
__global__ __launch_bounds__(256) void k_grad_w(TrainArgs a, float* __restrict__ part) {
  constexpr int TF = gw_tf<W>(), TK = gw_tk<W>();
  constexpr int FBW = TF / 64;                       // row (feature) blocks per wave
  constexpr int RB = TK / 64;                        // column blocks per wave
  static_assert((TF + TK) * kGwChunk <= kGwStageElems && kGwStages == 4, "stage buffers");
  int tk, tf, s, l;
  gw_coords<W>(blockIdx.x, gridDim.x, &tk, &tf, &s, &l);
  GwCtx<W> x;
  x.tid = threadIdx.x;
  x.lane = x.tid & 63;
  x.wid = x.tid >> 6;
  x.f0 = tf * TF;
  x.k0 = tk * TK;
  const int tiles = a.Bp / 64;                      // splits: whole 64-row tiles, as even as they come
  x.b_begin = (int)((int64_t)s * tiles / kSplitW) * 64;
  x.nch = ((int)((int64_t)(s + 1) * tiles / kSplitW) * 64 - x.b_begin) / kGwChunk;
  x.dz = a.dzT + (size_t)(l - 1) * W * a.Bp;        // layer blocks
  x.ap = a.aT + (size_t)(l - 2) * W * a.Bp;
  static_assert(TF % 64 == 0, "a load pass holds rows of one operand");
#pragma unroll
  for (int q = 0; q < GwCtx<W>::NQ; ++q) {           // thread's row r and segment of load q: tix(W, f, 8 seg) in a chunk
    const int id = 256 * q + x.tid, r = id >> 2, seg = gw_slot(r, id & 3);
    x.off[q] = (r < TF ? x.f0 + r : x.k0 + r - TF) * 64 + 8 * seg;
  }
  const int half = x.lane >> 5, col = x.lane & 31, wf = x.wid & 1, wk = x.wid >> 1;
  f32x16 acc[FBW][RB];
#pragma unroll
  for (int fb = 0; fb < FBW; ++fb)
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) acc[fb][rb] = f32x16{};
  float dbs = 0.f;   // this thread's share of its dz row's sum (the bias gradient, tk == 0)
  const bool bias = tk == 0;
  if (x.nch > 0) gw_issue<W, 0>(x, 0);
  if (x.nch > 1) gw_issue<W, 1>(x, 1);
  if (x.nch > 2) gw_issue<W, 2>(x, 2);
  for (int c = 0; c < x.nch; c += kGwStages) {
    gw_step<W, 0>(x, c, bias, dbs, acc);
    if (c + 1 < x.nch) gw_step<W, 1>(x, c + 1, bias, dbs, acc);
    if (c + 2 < x.nch) gw_step<W, 2>(x, c + 2, bias, dbs, acc);
    if (c + 3 < x.nch) gw_step<W, 3>(x, c + 3, bias, dbs, acc);
  }
  float* P = part + ((size_t)(l - 2) * kSplitW + s) * W * W;
#pragma unroll
  for (int fb = 0; fb < FBW; ++fb)
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          P[(size_t)(x.f0 + (TF / 2) * wf + 32 * fb + 8 * j + 4 * half + i) * W + x.k0 + (TK / 2) * wk + 32 * rb + col] =
              acc[fb][rb][4 * j + i];
  if (bias) {   // bias partials after the weight partials: [L - 1][kSplitW][W]
    constexpr int TPR = 256 / TF;
    const float d = TPR == 2 ? dbs + __shfl_xor(dbs, 1, 64) : dbs;
    if (x.tid % TPR == 0)
      part[(size_t)(a.net.n_hidden - 1) * kSplitW * W * W + ((size_t)(l - 2) * kSplitW + s) * W + x.f0 + x.tid / TPR] = d;
  }
}

// Fixed-order sums over the splits: dW_l, then db_l (layers 2..L).
__global__ void k_grad_reduce(TrainArgs a, const float* __restrict__ part) {
  const int W = a.net.width;
  const int64_t per = (int64_t)W * W;
  const int64_t total = per * (a.net.n_hidden - 1);
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total + (int64_t)W * (a.net.n_hidden - 1);
       g += (int64_t)gridDim.x * blockDim.x) {
    float s = 0.f;
    if (g < total) {
      const int l = (int)(g / per) + 2;
      const int64_t o = g - (int64_t)(l - 2) * per;
      for (int sp = 0; sp < kSplitW; ++sp) s += part[((size_t)(l - 2) * kSplitW + sp) * per + o];
      a.grad[off_w(a.net, l) + o] = s;
    } else {
      const int64_t h = g - total;
      const int l = (int)(h / W) + 2, f = (int)(h - (int64_t)(l - 2) * W);
      const float* pb = part + total * kSplitW + (size_t)(l - 2) * kSplitW * W;
      for (int sp = 0; sp < kSplitW; ++sp) s += pb[(size_t)sp * W + f];
      a.grad[off_b(a.net, l) + f] = s;
    }
  }
}

// Output-layer gradients: w_out[f] = sum_b dy[b] a_L[f][b] and b_out = sum_b dy[b].  A
// block streams a contiguous run of 64-row tiles of the last hidden layer's block (each
// tile's layer is W x 64 consecutive BF16 values): wave w takes features w W/4 .. and
// every load of a wave reads 1 KB of consecutive memory, 8 features x 64 rows, so lane l
// always meets feature 8 q + l/8 of its quarter and rows 8 (l % 8) .. + 7 of the tile.
// Per-lane sums run over the block's tiles; lanes of one feature are then combined and
// the block writes its partial row [W + 1]; k_sum_splits adds the blocks' rows in a
// fixed order.
constexpr int kOutBlocks = 256;    // blocks (at most) of k_grad_out
__host__ __device__ inline int out_blocks(int Bp) { return Bp / 64 < kOutBlocks ? Bp / 64 : kOutBlocks; }

template <int W>
__global__ __launch_bounds__(256) void k_grad_out(TrainArgs a, float* __restrict__ part) {
  constexpr int Q = W / 32;                            // loads per wave and tile
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int tiles = a.Bp / 64, nb = out_blocks(a.Bp);
  const int t_begin = (int)((int64_t)blockIdx.x * tiles / nb), t_end = (int)((int64_t)(blockIdx.x + 1) * tiles / nb);
  const int fw = wid * (W / 4);
  const __bf16* v = a.aT + (size_t)(a.net.n_hidden - 1) * W * a.Bp;   // the last hidden layer's block
  float acc[Q], sdy = 0.f;
#pragma unroll
  for (int q = 0; q < Q; ++q) acc[q] = 0.f;
  for (int t = t_begin; t < t_end; ++t) {
    const __bf16* base = v + ((size_t)t * W + fw) * 64 + 8 * lane;
    bf16x8 x[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) x[q] = *reinterpret_cast<const bf16x8*>(base + 512 * q);
    const float4 d0 = *reinterpret_cast<const float4*>(a.dy + (size_t)t * 64 + 8 * (lane & 7));
    const float4 d1 = *reinterpret_cast<const float4*>(a.dy + (size_t)t * 64 + 8 * (lane & 7) + 4);
    const float d[8] = {d0.x, d0.y, d0.z, d0.w, d1.x, d1.y, d1.z, d1.w};
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int e = 0; e < 8; ++e) acc[q] = fmaf((float)x[q][e], d[e], acc[q]);
    if (wid == 0 && lane < 8) sdy += ((d[0] + d[1]) + (d[2] + d[3])) + ((d[4] + d[5]) + (d[6] + d[7]));
  }
  float* P = part + (size_t)blockIdx.x * (W + 1);
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    float u = acc[q];
    u += __shfl_xor(u, 1, 64);
    u += __shfl_xor(u, 2, 64);
    u += __shfl_xor(u, 4, 64);
    if ((lane & 7) == 0) P[fw + 8 * q + (lane >> 3)] = u;
  }
  if (wid == 0) {
    sdy += __shfl_xor(sdy, 1, 64);
    sdy += __shfl_xor(sdy, 2, 64);
    sdy += __shfl_xor(sdy, 4, 64);
    if (lane == 0) P[W] = sdy;
  }
}

// sum over r < R of part[r n + o], in a fixed order, valid in wave 0: a block of 16
// waves takes 64 consecutive outputs (o = block * 64 + lane); wave w sums rows w R/16 ..
// in order, 8 loads in flight, and the 16 wave sums are added in order.  Many short sums
// in parallel instead of one long chain per output (the splits of the gradient kernels
// are up to 256 rows).  ws: [16][64] floats of LDS; one barrier.
__device__ __forceinline__ float split_sum_64(const float* __restrict__ part, int R, int n, int o,
                                              float (*ws)[64]) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int r0 = (int)((int64_t)wid * R / 16), r1 = (int)((int64_t)(wid + 1) * R / 16);
  float acc = 0.f;
  if (o < n) {
    int r = r0;
    for (; r + 8 <= r1; r += 8) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = part[(size_t)(r + u) * n + o];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += v[u];
    }
    for (; r < r1; ++r) acc += part[(size_t)r * n + o];
  }
  ws[wid][lane] = acc;
  __syncthreads();
  float t = 0.f;
  if (wid == 0) {
#pragma unroll
    for (int w = 0; w < 16; ++w) t += ws[w][lane];
  }
  return t;
}

// out[o] = sum over r < R of part[r n + o] (split_sum_64).
__global__ __launch_bounds__(1024) void k_sum_splits(const float* __restrict__ part, int R, int n,
                                                     float* __restrict__ out) {
  __shared__ float ws[16][64];
  const int o = blockIdx.x * 64 + (threadIdx.x & 63);
  const float t = split_sum_64(part, R, n, o, ws);
  if (threadIdx.x < 64 && o < n) out[o] = t;
}

hipError_t launch_sum_splits(const float* part, int R, int n, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)((n + 63) / 64)), dim3(1024), 0, st, part, R, n, out);
  return hipGetLastError();
}

// dW_1[f][j] = sum_b dz_1[f][b] h0[j][b] and db_1[f] = sum_b dz_1[f][b] on MFMA.  The FP32
// input is split into a BF16 high part and the BF16 rounding of the remainder (about 16
// significant bits together), so that two MFMAs per 16 batch rows, with dz_1 as the A
// operand, give C_hi[f][j] over the high parts, whose column in_dim is a column of ones
// (the bias), and C_lo[f][j] over the low parts; dW_1 = C_hi + C_lo.  A block takes one
// batch split and 4 waves of 64 features each (two feature blocks of 32); the B
// fragments of the split are built once per block in LDS, in chunks of kW1Chunk k-steps
// of 16 rows.  The splits' partial rows [W][in_dim] then [W] go to part, summed in a
// fixed order by k_sum_splits.
constexpr int kW1MaxSplits = 128;
constexpr int kW1Chunk = 16;      // k-steps per LDS chunk (256 rows)
constexpr int kW1Unroll = 8;      // k-steps whose dz loads are in flight together
__host__ __device__ inline int w1_splits(int Bp) { return Bp / 16 < kW1MaxSplits ? Bp / 16 : kW1MaxSplits; }

__global__ __launch_bounds__(256) void k_grad_w1(TrainArgs a, float* __restrict__ part) {
  __shared__ __align__(16) bf16x8 Bf[kW1Chunk][2][64];   // [k-step][high, low][lane]
  const int W = a.net.width, in_dim = a.net.in_dim;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int half = lane >> 5, col = lane & 31;
  const int S = w1_splits(a.Bp), nks = a.Bp / 16, s = blockIdx.y;
  // blockIdx.z: the dz slot (the residual network's W_0 and its blocks' Wx_b, c_b, one
  // launch; a single slot for the softplus network), each with its own partials
  const __bf16* dz = a.dzT + (size_t)blockIdx.z * W * a.Bp;
  part += (size_t)blockIdx.z * S * W * (in_dim + 1);
  const int ks_begin = (int)((int64_t)s * nks / S), ks_end = (int)((int64_t)(s + 1) * nks / S);
  const int f0 = (blockIdx.x * 4 + wid) * 64;
  const bool active = f0 < W;                      // wave-uniform; every wave takes the barriers
  f32x16 hi[2] = {f32x16{}, f32x16{}}, lo[2] = {f32x16{}, f32x16{}};
  for (int c0 = ks_begin; c0 < ks_end; c0 += kW1Chunk) {
    const int nc = min(kW1Chunk, ks_end - c0);
    __syncthreads();                               // the last chunk's fragments are consumed
    for (int it = tid; it < nc * 64; it += 256) {  // fragment (k-step, lane l): column l % 32, rows 8 (l / 32) ..
      const int k = it >> 6, l = it & 63, j = l & 31;
      const int b = (c0 + k) * 16 + 8 * (l >> 5);
      bf16x8 h = {}, r = {};
      if (j < in_dim) {
        const float4 u0 = *reinterpret_cast<const float4*>(a.h0T + (size_t)j * a.Bp + b);
        const float4 u1 = *reinterpret_cast<const float4*>(a.h0T + (size_t)j * a.Bp + b + 4);
        const float x[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          h[e] = (__bf16)x[e];
          r[e] = (__bf16)(x[e] - (float)h[e]);
        }
      } else if (j == in_dim) {
#pragma unroll
        for (int e = 0; e < 8; ++e) h[e] = (__bf16)1.0f;
      }
      Bf[k][0][l] = h;
      Bf[k][1][l] = r;
    }
    __syncthreads();
    if (active) {
      for (int k0 = 0; k0 < nc; k0 += kW1Unroll) {
        bf16x8 x[kW1Unroll][2];
#pragma unroll
        for (int u = 0; u < kW1Unroll; ++u)
#pragma unroll
          for (int fb = 0; fb < 2; ++fb)
            if (k0 + u < nc)
              x[u][fb] = *reinterpret_cast<const bf16x8*>(dz + tix(W, f0 + 32 * fb + col, (c0 + k0 + u) * 16 + 8 * half));
#pragma unroll
        for (int u = 0; u < kW1Unroll; ++u) {
          if (k0 + u >= nc) break;
          const bf16x8 bh = Bf[k0 + u][0][lane], bl = Bf[k0 + u][1][lane];
#pragma unroll
          for (int fb = 0; fb < 2; ++fb) {
            hi[fb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x[u][fb], bh, hi[fb], 0, 0, 0);
            lo[fb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x[u][fb], bl, lo[fb], 0, 0, 0);
          }
        }
      }
    }
  }
  if (!active) return;
  // C[f][j]: acc[4 jj + i] is feature 32 fb + 8 jj + 4 half + i, column col
  float* ps = part + (size_t)s * W * (in_dim + 1);   // this split: dW_1 [W][in_dim], then db_1 [W]
#pragma unroll
  for (int fb = 0; fb < 2; ++fb)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int f = f0 + 32 * fb + 8 * (e >> 2) + 4 * half + (e & 3);
      if (col < in_dim) ps[(size_t)f * in_dim + col] = hi[fb][e] + lo[fb][e];
      else if (col == in_dim) ps[(size_t)W * in_dim + f] = hi[fb][e];
    }
}

// Adam, PyTorch's form: p -= (lr / (1 - b1^t)) * m / (sqrt(v) / sqrt(1 - b2^t) + eps).
__global__ void k_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, int64_t n, float lr, float b1, float b2, float eps,
                       float step_size, float inv_sqrt_bc2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = fmaf(b1, m[i], (1.f - b1) * gi);
    const float vi = fmaf(b2, v[i], (1.f - b2) * gi * gi);
    m[i] = mi;
    v[i] = vi;
    p[i] -= step_size * mi / (sqrtf(vi) * inv_sqrt_bc2 + eps);
  }
  (void)lr;
}

template <int W>
hipError_t set_lds_attr(const void* fn, bool* done) {
  if (*done) return hipSuccess;
  const int lds = kRows * (W + kLdsPad) * (int)sizeof(__bf16);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e == hipSuccess) *done = true;
  return e;
}

template <int W>
hipError_t launch_train_t(TrainArgs a, float* part_w, float* part_w1, float sigma, float* loss_out, hipStream_t st) {
  const size_t lds = (size_t)kRows * (W + kLdsPad) * sizeof(__bf16);
  const unsigned tiles = (unsigned)(a.Bp / kRows);
  hipError_t e;
  static bool fwd_attr = false, bwd_attr = false;
  if ((e = set_lds_attr<W>(reinterpret_cast<const void*>(&k_train_fwd<W>), &fwd_attr)) != hipSuccess) return e;
  if ((e = set_lds_attr<W>(reinterpret_cast<const void*>(&k_train_bwd<W>), &bwd_attr)) != hipSuccess) return e;
  // the forward writes dy and the per-tile loss sums; those borrow part_w1, which
  // k_grad_w1 fills only later in the step
  a.sigma = sigma;
  a.loss_part = part_w1;
  hipLaunchKernelGGL((k_train_fwd<W>), dim3(tiles), dim3(train_threads<W>()), lds, st, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_train_loss_sum, dim3(1), dim3(1024), 0, st, a, part_w1, a.Bp / 64, loss_out);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL((k_train_bwd<W>), dim3(tiles), dim3(train_threads<W>()), lds, st, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int L = a.net.n_hidden;
  if (L >= 2) {
    const unsigned blocks = (unsigned)((W / gw_tf<W>()) * (W / gw_tk<W>()) * kSplitW * (L - 1));
    hipLaunchKernelGGL((k_grad_w<W>), dim3(blocks), dim3(256), 0, st, a, part_w);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_grad_reduce, dim3(2048), dim3(256), 0, st, a, part_w);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // the output-layer partials, then the dW_1 splits, use part_w1 in turn
  hipLaunchKernelGGL((k_grad_out<W>), dim3((unsigned)out_blocks(a.Bp)), dim3(256), 0, st, a, part_w1);
  if ((e = launch_sum_splits(part_w1, out_blocks(a.Bp), W + 1, a.grad + off_out(a.net), st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_grad_w1, dim3((unsigned)((W + 255) / 256), (unsigned)w1_splits(a.Bp)), dim3(256), 0, st, a,
                     part_w1);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // dW_1 and db_1 are contiguous at the start of the flat vector
  return launch_sum_splits(part_w1, w1_splits(a.Bp), W * (a.net.in_dim + 1), a.grad, st);
}

// ----------------------------------------------------------------- residual network
// Training of the paper's network (Sec. IV-A, Fig. 1) with its BatchNorm layers in the
// training form PyTorch uses (Sec. V): each block normalises relu(z_b) with the mean and
// (biased) variance of the batch, and its running statistics then move towards them
// with momentum kBnMomentum, the variance taking the unbiased batch variance.  Every
// batch statistic is a reduction over all rows, so a block is one launch over the row
// tiles (linear layer, ReLU, per-tile sums) followed by a reduction launch:
//   k_rt_fwd(b)    h_{b-1} (h_0 = W_0 x + b_0; else the previous block's BatchNorm and
//                  skip, h_{b-1} = h_{b-2} + gamma (a_{b-1} - mu) inv + beta), z_b over
//                  [h_{b-1}; x_hi; x_lo] on MFMA (the inference kernel's packing),
//                  a_b = relu(z_b) in BF16, per-tile sums of a_b and a_b^2;
//   k_rt_stats     batch mean, inverse standard deviation and variance per feature
//                  (tiles combined in FP64, fixed order);
//   k_rt_out       h_L in FP32, the prediction, the loss, dy, per-tile sums for the
//                  output layer's gradient and for the last block's BatchNorm backward;
//   backward, b = L..1: k_rt_bstats (per-tile sums of g = dL/dh_b and g n_b, b < L),
//                  k_rt_stats (their batch sums: the BatchNorm gradients), k_rt_bwd
//                  (dz_b = gamma inv (g - mean g - n mean(g n)) [a_b > 0], then
//                  g_{b-1} = g + dz_b Wh_b on MFMA, in place);
//   weight gradients: k_grad_w over (dz_b, h_{b-1}) for Wh_b, k_grad_w1 over (dz slot,
//                  x) for Wx_b and c_b (contiguous in the flat vector) and for W_0 and
//                  b_0; running statistics (k_rt_running); Adam.
// Stored per step (Bp rows, tiled like aT): h_0..h_{L-1} and a_1..a_L in BF16, dz slots
// 0..L in BF16 (slot 0: g_0 = dL/dh_0, rounded to BF16 for the W_0 and b_0 sums), g in
// FP32.  Rows >= B carry no statistic and no gradient.
constexpr float kBnMomentum = 0.1f;   // PyTorch's default

struct ResTrainArgs {
  MlpArgs net;            // SV_NET_RESIDUAL, n_hidden = L blocks
  const float* samples;   // [n][in_dim + 1]
  const int* idx;         // [B]
  int B, Bp;
  float* xT;              // [in_dim][Bp] network input
  __bf16* hT;             // [L] slabs of W x Bp (tix layout): h_0 .. h_{L-1}
  __bf16* aT;             // [L] slabs: a_1 .. a_L
  __bf16* dzT;            // [L + 1] slabs: g_0, dz_1 .. dz_L
  float* g;               // one FP32 slab: dL/dh_b
  float* part;            // [Bp / 64][2][W] per-tile sums
  float* stats;           // [L][3][W]: batch mean, 1 / sqrt(var + eps), var (biased)
  float* bsum;            // [2][W]: sum g, sum g n of the current backward block
  float* y;               // [Bp]
  float* dy;              // [Bp]
  float* pout;            // [Bp / 64][W + 2]: output-layer and loss partials
  const __bf16* packed;   // [L][W][W + kResXCols] forward operands (k_pack_res order)
  const __bf16* packedT;  // [L][W][W] Wh_b^T in A-operand order
  float* grad;            // [n_params]
  float sigma;            // loss clamp
};

__device__ __forceinline__ const float* rt_block(const ResTrainArgs& a, int b) {   // block b, 1-based
  return a.net.params + res_block_base(a.net.width, a.net.in_dim, b - 1);
}

template <int W>
__global__ __launch_bounds__(train_threads<W>(), 2) void k_rt_fwd(ResTrainArgs a, int b) {
  constexpr int NT = train_threads<W>(), NW = NT / 64;
  constexpr int K = W + kResXCols, LD = K + kLdsPad;
  constexpr int kMaxIn = 3 + 2 * SV_MAX_DOF;
  constexpr int kInPad = (kMaxIn + 3) / 4 * 4;
  extern __shared__ __align__(16) unsigned char smem[];
  __bf16* H = reinterpret_cast<__bf16*>(smem);
  __shared__ __align__(16) float xs[kRows][kInPad];
  const MlpArgs& n = a.net;
  const int in_dim = n.in_dim;
  const int tile = blockIdx.x, r0 = tile * kRows;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int half = lane >> 5, col = lane & 31;
  const size_t slab = (size_t)W * a.Bp;
  for (int e = tid; e < kRows * kInPad; e += NT) {
    const int r = e / kInPad, j = e - r * kInPad;
    float v = 0.f;
    if (j < in_dim) v = a.samples[(size_t)a.idx[min(r0 + r, a.B - 1)] * (in_dim + 1) + j];
    xs[r][j] = v;
  }
  __syncthreads();
  if (b == 1)   // the input feature-major for the input-column gradients: consecutive threads on consecutive rows
    for (int e = tid; e < kRows * in_dim; e += NT) {
      const int j = e / kRows, r = e - j * kRows;
      a.xT[(size_t)j * a.Bp + r0 + r] = xs[r][j];
    }
  // the network input as BF16 high and low parts, columns W .. W + 2 in_dim - 1
  for (int e = tid; e < kRows * kResXCols; e += NT) {
    const int r = e / kResXCols, j = e - r * kResXCols;
    __bf16 v = (__bf16)0.f;
    if (j < 2 * in_dim) {
      const float x = xs[r][j < in_dim ? j : j - in_dim];
      const __bf16 hi = (__bf16)x;
      v = j < in_dim ? hi : (__bf16)(x - (float)hi);
    }
    H[r * LD + W + j] = v;
  }
  if (b == 1) {   // h_0 = W_0 x + b_0 in FP32 (inputs past in_dim are zero), rounded to BF16
    for (int f = tid; f < W; f += NT) {
      float w[kInPad];
#pragma unroll
      for (int j = 0; j < kInPad; ++j) w[j] = j < in_dim ? n.params[(size_t)f * in_dim + j] : 0.f;
      const float b0 = n.params[(size_t)W * in_dim + f];
      for (int r = 0; r < kRows; ++r) {
        float z = b0;
#pragma unroll
        for (int j = 0; j < kInPad; ++j) z = fmaf(w[j], xs[r][j], z);
        H[r * LD + f] = (__bf16)z;
      }
    }
    __syncthreads();
    store_tile_T<W, NT, LD>(H, a.hT, r0);
  } else {        // h_{b-1} = h_{b-2} + gamma (a_{b-1} - mu) inv + beta, rounded to BF16
    // In 8 x 8 blocks (rows 8 rg.., features 8 fg..; the lane order of fetch_tile_T):
    // h_{b-2} and a_{b-1} come in with 16-byte loads, h_{b-1} goes out feature-major with
    // 16-byte stores and into the LDS tile by the transposed writes.
    constexpr int NQ = W / 64 / NW;
    const float* q = rt_block(a, b - 1) + (size_t)W * W + (size_t)W * in_dim + W;   // gamma, beta
    const float* st = a.stats + (size_t)(b - 2) * 3 * W;
    bf16x8 hv[NQ][8], av[NQ][8];
    fetch_tile_T<W, NT>(a.hT + (size_t)(b - 2) * slab, r0, hv);
    fetch_tile_T<W, NT>(a.aT + (size_t)(b - 2) * slab, r0, av);
    const int rg = lane >> 3;
    __bf16* hout = a.hT + (size_t)(b - 1) * slab;
#pragma unroll
    for (int qq = 0; qq < NQ; ++qq) {
      const int fg = 8 * (wid + qq * NW) + (lane & 7);
#pragma unroll
      for (int f = 0; f < 8; ++f) {
        const int ff = 8 * fg + f;
        const float gi = q[ff] * st[W + ff], mu = st[ff], be = q[W + ff];
        bf16x8 o;
#pragma unroll
        for (int e = 0; e < 8; ++e) o[e] = (__bf16)((float)hv[qq][f][e] + fmaf(gi, (float)av[qq][f][e] - mu, be));
        hv[qq][f] = o;
        __builtin_nontemporal_store(o, reinterpret_cast<bf16x8*>(hout + tix(W, ff, r0 + 8 * rg)));
      }
    }
    put_tile_T<W, NT, LD>(hv, H);
    __syncthreads();
  }
  f32x16 acc[kTFB][kTRB];
  layer_mfma_k<K, LD, kTFB, kTRB, 2>(a.packed + (size_t)(b - 1) * W * K, H, wid, 0, lane,
                                     rt_block(a, b) + (size_t)W * W + (size_t)W * in_dim, acc);
  __syncthreads();   // every wave has read the tile
#pragma unroll
  for (int fb = 0; fb < kTFB; ++fb)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int f = 32 * (kTFB * wid + fb) + 8 * j + 4 * half;
#pragma unroll
      for (int rb = 0; rb < kTRB; ++rb) {
        const bf16x4 v = {(__bf16)relu_acc(acc[fb][rb][4 * j + 0]), (__bf16)relu_acc(acc[fb][rb][4 * j + 1]),
                          (__bf16)relu_acc(acc[fb][rb][4 * j + 2]), (__bf16)relu_acc(acc[fb][rb][4 * j + 3])};
        *reinterpret_cast<bf16x4*>(H + (32 * rb + col) * LD + f) = v;
      }
    }
  __syncthreads();
  store_tile_T<W, NT, LD>(H, a.aT + (size_t)(b - 1) * slab, r0);
  const int nv = min(kRows, a.B - r0);   // valid rows of the tile
  for (int f = tid; f < W; f += NT) {
    float s = 0.f, s2 = 0.f;
    for (int r = 0; r < nv; ++r) {
      const float v = (float)H[r * LD + f];
      s += v;
      s2 = fmaf(v, v, s2);
    }
    a.part[((size_t)tile * 2) * W + f] = s;
    a.part[((size_t)tile * 2 + 1) * W + f] = s2;
  }
}

// Batch sums per feature from the per-tile sums in a.part: 64 features per block, 16
// thread groups over consecutive runs of tiles, combined in FP64 in a fixed order.
// mode 0 (forward, block b): stats[b] = (mean, 1 / sqrt(var + eps), var) of a_b.
// mode 1 (backward, block b): bsum = (sum g, sum g n); the gradients of beta_b and gamma_b.
constexpr int kStatGroups = 16;
__global__ __launch_bounds__(64 * kStatGroups) void k_rt_stats(ResTrainArgs a, int b, int mode) {
  __shared__ double red[2][kStatGroups][64];
  const int W = a.net.width, tiles = a.Bp / kRows;
  const int fl = threadIdx.x & 63, tg = threadIdx.x >> 6;
  const int f = blockIdx.x * 64 + fl;
  const int t0 = (int)((int64_t)tg * tiles / kStatGroups), t1 = (int)((int64_t)(tg + 1) * tiles / kStatGroups);
  double s0 = 0.0, s1 = 0.0;
  if (f < W) {
    // tiles in order; eight tiles' loads in flight before their adds
    int t = t0;
    for (; t + 8 <= t1; t += 8) {
      float v0[8], v1[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        v0[u] = a.part[((size_t)(t + u) * 2) * W + f];
        v1[u] = a.part[((size_t)(t + u) * 2 + 1) * W + f];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        s0 += v0[u];
        s1 += v1[u];
      }
    }
    for (; t < t1; ++t) {
      s0 += a.part[((size_t)t * 2) * W + f];
      s1 += a.part[((size_t)t * 2 + 1) * W + f];
    }
  }
  red[0][tg][fl] = s0;
  red[1][tg][fl] = s1;
  __syncthreads();
  if (tg != 0 || f >= W) return;
  double S0 = 0.0, S1 = 0.0;
#pragma unroll
  for (int q = 0; q < kStatGroups; ++q) {
    S0 += red[0][q][fl];
    S1 += red[1][q][fl];
  }
  if (mode == 0) {
    const double mu = S0 / a.B, v = fmax(S1 / a.B - mu * mu, 0.0);
    float* st = a.stats + (size_t)(b - 1) * 3 * W;
    st[f] = (float)mu;
    st[W + f] = (float)(1.0 / sqrt(v + (double)a.net.bn_eps));
    st[2 * W + f] = (float)v;
  } else {
    a.bsum[f] = (float)S0;
    a.bsum[W + f] = (float)S1;
    const size_t gb = res_block_base(W, a.net.in_dim, b - 1) + (size_t)W * W + (size_t)W * a.net.in_dim;
    a.grad[gb + W + f] = (float)S1;       // gamma
    a.grad[gb + 2 * W + f] = (float)S0;   // beta
  }
}

// h_L = h_{L-1} + gamma_L (a_L - mu) inv + beta_L in FP32, the prediction, the loss
// terms and dy of the tile's rows, then per feature: the tile's sums of dy h_L (the
// w_out gradient; h_L formed again from the same operands, which is cheaper than an FP32
// tile in LDS that would hold the kernel to one block per CU) and, for the last block's
// BatchNorm backward with g = dy w_out, of g and g n_L.
template <int W>
__global__ __launch_bounds__(256) void k_rt_out(ResTrainArgs a) {
  __shared__ float ys[4][kRows];
  __shared__ float dys[kRows], ls[kRows];
  const MlpArgs& n = a.net;
  const int L = n.n_hidden, in_dim = n.in_dim;
  const int tile = blockIdx.x, r0 = tile * kRows;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const size_t slab = (size_t)W * a.Bp;
  const float* q = rt_block(a, L) + (size_t)W * W + (size_t)W * in_dim + W;   // gamma, beta
  const float* st = a.stats + (size_t)(L - 1) * 3 * W;
  const float* wout = rt_block(a, L + 1);
  const __bf16* hp = a.hT + (size_t)(L - 1) * slab;
  const __bf16* ap = a.aT + (size_t)(L - 1) * slab;
  // Prediction partials: wave w sums wout[f] h_L[r][f] over f = w, w + 4, ... in order
  // for row r = lane.  h_L is formed in chunks of 64 features: 16-byte loads of h_{L-1}
  // and a_L (8 rows of one feature), FP32 results into hs[row][feature] (row stride 65:
  // conflict-free), then each wave reads its features of the chunk.
  __shared__ float hs[kRows][65];
  float yp = 0.f;
  for (int c0 = 0; c0 < W; c0 += 64) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int sgi = tid + 256 * u, fc = sgi >> 3, rg = sgi & 7, f = c0 + fc;
      const size_t o = tix(W, f, r0 + 8 * rg);
      const bf16x8 hv = *reinterpret_cast<const bf16x8*>(hp + o), av = *reinterpret_cast<const bf16x8*>(ap + o);
#pragma unroll
      for (int e = 0; e < 8; ++e) hs[8 * rg + e][fc] = (float)hv[e] + fmaf(q[f] * st[W + f], (float)av[e] - st[f], q[W + f]);
    }
    __syncthreads();
#pragma unroll
    for (int fc = wid; fc < 64; fc += 4) yp = fmaf(wout[c0 + fc], hs[lane][fc], yp);
    __syncthreads();
  }
  ys[wid][lane] = yp;
  __syncthreads();
  if (tid < kRows) {
    const int r = r0 + tid;
    const float yv = wout[W] + ((ys[0][tid] + ys[1][tid]) + (ys[2][tid] + ys[3][tid]));
    const bool valid = r < a.B;
    const float d = valid ? a.samples[(size_t)a.idx[r] * (in_dim + 1) + in_dim] : 0.f;
    const float res = yv - fminf(fmaxf(d, -a.sigma), a.sigma);
    const float dyv = valid ? (res > 0.f ? 1.f : (res < 0.f ? -1.f : 0.f)) / (float)a.B : 0.f;
    a.y[r] = yv;
    a.dy[r] = dyv;
    dys[tid] = dyv;
    ls[tid] = valid ? fabsf(res) : 0.f;
  }
  __syncthreads();
  float* po = a.pout + (size_t)tile * (W + 2);
  float sdy = 0.f;
  for (int r = 0; r < kRows; ++r) sdy += dys[r];
  // Per feature, in row order: sum dy h_L and sum dy n_L.  The same chunks of 64 features
  // as above (coalesced loads; h_L and n_L into LDS), then wave 0's lane f sums feature
  // c0 + f.
  __shared__ float ns[kRows][65];
  for (int c0 = 0; c0 < W; c0 += 64) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int sgi = tid + 256 * u, fc = sgi >> 3, rg = sgi & 7, f = c0 + fc;
      const size_t o = tix(W, f, r0 + 8 * rg);
      const bf16x8 hv = *reinterpret_cast<const bf16x8*>(hp + o), av = *reinterpret_cast<const bf16x8*>(ap + o);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        hs[8 * rg + e][fc] = (float)hv[e] + fmaf(q[f] * st[W + f], (float)av[e] - st[f], q[W + f]);
        ns[8 * rg + e][fc] = ((float)av[e] - st[f]) * st[W + f];
      }
    }
    __syncthreads();
    if (wid == 0) {
      const int f = c0 + lane;
      float sh = 0.f, sn = 0.f;
      for (int r = 0; r < kRows; ++r) {
        sh = fmaf(dys[r], hs[r][lane], sh);
        sn = fmaf(dys[r], ns[r][lane], sn);
      }
      po[f] = sh;
      a.part[((size_t)tile * 2) * W + f] = wout[f] * sdy;
      a.part[((size_t)tile * 2 + 1) * W + f] = wout[f] * sn;
    }
    __syncthreads();
  }
  if (tid == 0) {
    float sl = 0.f;
    for (int r = 0; r < kRows; ++r) sl += ls[r];
    po[W] = sdy;
    po[W + 1] = sl;
  }
}

// The output layer's gradient and the loss from the per-tile partials [tiles][W + 2], in
// a fixed order (split_sum_64: 16 waves over runs of tiles per 64 outputs).
__global__ __launch_bounds__(1024) void k_rt_out_reduce(ResTrainArgs a, float* __restrict__ loss_out) {
  __shared__ float ws[16][64];
  const int W = a.net.width, tiles = a.Bp / kRows;
  const int o = blockIdx.x * 64 + (threadIdx.x & 63);
  const float s = split_sum_64(a.pout, tiles, W + 2, o, ws);
  if (threadIdx.x < 64 && o < W + 2) {
    if (o <= W) a.grad[res_block_base(W, a.net.in_dim, a.net.n_hidden) + o] = s;
    else if (loss_out) *loss_out = s / (float)a.B;
  }
}

// Per-tile sums of g = dL/dh_b and g n_b (b < L), each feature's 64 rows summed in row
// order by one lane.  A wave stages 32 features at a time in LDS (the tile's g and a_b
// of 32 consecutive features are 8 KB and 4 KB of consecutive memory: 16-byte loads,
// consecutive lanes on consecutive pieces), so that the loads are coalesced; lane f then
// reads its feature's rows from LDS (row stride 65: conflict-free).
template <int W>
__global__ __launch_bounds__(256) void k_rt_bstats(ResTrainArgs a, int b) {
  constexpr int kF = 32;   // features per wave and pass
  __shared__ float gs[4][kF][kRows + 1], as[4][kF][kRows + 1];
  const int tile = blockIdx.x, r0 = tile * kRows;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const float* st = a.stats + (size_t)(b - 1) * 3 * W;
  const __bf16* ap = a.aT + (size_t)(b - 1) * W * a.Bp;
  float (*G)[kRows + 1] = gs[wid];
  float (*A)[kRows + 1] = as[wid];
  for (int f0 = kF * wid; f0 < W; f0 += 4 * kF) {
    const float4* g4 = reinterpret_cast<const float4*>(a.g + tix(W, f0, r0));   // kF x 64 floats
    const bf16x8* a8 = reinterpret_cast<const bf16x8*>(ap + tix(W, f0, r0));    // kF x 64 BF16
    float4 gq[kF * kRows / 4 / 64];
    bf16x8 aq[kF * kRows / 8 / 64];
#pragma unroll
    for (int u = 0; u < kF * kRows / 4 / 64; ++u) gq[u] = g4[lane + 64 * u];
#pragma unroll
    for (int u = 0; u < kF * kRows / 8 / 64; ++u) aq[u] = a8[lane + 64 * u];
#pragma unroll
    for (int u = 0; u < kF * kRows / 4 / 64; ++u) {
      const int q = lane + 64 * u, f = q >> 4, r = 4 * (q & 15);
      G[f][r] = gq[u].x; G[f][r + 1] = gq[u].y; G[f][r + 2] = gq[u].z; G[f][r + 3] = gq[u].w;
    }
#pragma unroll
    for (int u = 0; u < kF * kRows / 8 / 64; ++u) {
      const int q = lane + 64 * u, f = q >> 3, r = 8 * (q & 7);
#pragma unroll
      for (int e = 0; e < 8; ++e) A[f][r + e] = (float)aq[u][e];
    }
    __builtin_amdgcn_wave_barrier();   // the wave's LDS writes come before its reads
    if (lane < kF) {
      const int f = f0 + lane;
      const float mu = st[f], iv = st[W + f];
      float s = 0.f, sn = 0.f;
      for (int r = 0; r < kRows; ++r) {
        const float gv = G[lane][r];
        s += gv;
        sn = fmaf(gv, (A[lane][r] - mu) * iv, sn);
      }
      a.part[((size_t)tile * 2) * W + f] = s;
      a.part[((size_t)tile * 2 + 1) * W + f] = sn;
    }
    __builtin_amdgcn_wave_barrier();   // reads done before the next pass overwrites
  }
}

// Block b's backward over one tile: dz_b from g (b = L: dy w_out) and the batch sums,
// in BF16 to dz slot b and the LDS tile; then g <- g + dz_b Wh_b (MFMA with Wh_b^T), in
// place, or for b = 1 the result g_0 in BF16 to dz slot 0.
template <int W>
__global__ __launch_bounds__(train_threads<W>(), 2) void k_rt_bwd(ResTrainArgs a, int b) {
  constexpr int NT = train_threads<W>(), NW = NT / 64;
  constexpr int LD = W + kLdsPad;
  extern __shared__ __align__(16) unsigned char smem[];
  __bf16* H = reinterpret_cast<__bf16*>(smem);
  const MlpArgs& n = a.net;
  const int L = n.n_hidden, in_dim = n.in_dim;
  const int tile = blockIdx.x, r0 = tile * kRows;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int half = lane >> 5, col = lane & 31;
  const size_t slab = (size_t)W * a.Bp;
  const float* gamma = rt_block(a, b) + (size_t)W * W + (size_t)W * in_dim + W;
  const float* st = a.stats + (size_t)(b - 1) * 3 * W;
  const float* wout = rt_block(a, L + 1);
  const __bf16* ap = a.aT + (size_t)(b - 1) * slab;
  __bf16* dzs = a.dzT + (size_t)b * slab;
  const float invB = 1.f / (float)a.B;
  // dz_b in 8 x 8 blocks (rows 8 rg.., features 8 fg..; the lane order of fetch_tile_T):
  // a_b, g (FP32) and dz_b move as 16-byte pieces of feature rows, dz_b goes into the
  // LDS tile by transposed writes.
  constexpr int NQ = W / 64 / NW;
  const int rg = lane >> 3;
  float dyv[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) dyv[e] = 0.f;
  if (b == L) {
    const float4 d0 = *reinterpret_cast<const float4*>(a.dy + r0 + 8 * rg);
    const float4 d1 = *reinterpret_cast<const float4*>(a.dy + r0 + 8 * rg + 4);
    dyv[0] = d0.x; dyv[1] = d0.y; dyv[2] = d0.z; dyv[3] = d0.w;
    dyv[4] = d1.x; dyv[5] = d1.y; dyv[6] = d1.z; dyv[7] = d1.w;
  }
#pragma unroll
  for (int qq = 0; qq < NQ; ++qq) {
    const int fg = 8 * (wid + qq * NW) + (lane & 7);
    bf16x8 av[8], dz16[8];
#pragma unroll
    for (int f = 0; f < 8; ++f) av[f] = *reinterpret_cast<const bf16x8*>(ap + tix(W, 8 * fg + f, r0 + 8 * rg));
#pragma unroll
    for (int f = 0; f < 8; ++f) {
      const int ff = 8 * fg + f;
      const size_t o = tix(W, ff, r0 + 8 * rg);
      float gl[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      if (b < L) {
        const float4 g0 = *reinterpret_cast<const float4*>(a.g + o);
        const float4 g1 = *reinterpret_cast<const float4*>(a.g + o + 4);
        gl[0] = g0.x; gl[1] = g0.y; gl[2] = g0.z; gl[3] = g0.w;
        gl[4] = g1.x; gl[5] = g1.y; gl[6] = g1.z; gl[7] = g1.w;
      }
      const float gm = gamma[ff], iv = st[W + ff], mu = st[ff], s0 = a.bsum[ff], s1 = a.bsum[W + ff], wo = wout[ff];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const bool valid = r0 + 8 * rg + e < a.B;
        const float gv = b == L ? dyv[e] * wo : gl[e];
        const float avf = (float)av[f][e];
        const float nn = (avf - mu) * iv;
        const float dz = (valid && avf > 0.f) ? gm * iv * (gv - s0 * invB - nn * (s1 * invB)) : 0.f;
        dz16[f][e] = (__bf16)dz;
      }
      *reinterpret_cast<bf16x8*>(dzs + o) = dz16[f];
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      bf16x8 t;
#pragma unroll
      for (int f = 0; f < 8; ++f) t[f] = dz16[f][r];
      *reinterpret_cast<bf16x8*>(H + (8 * rg + r) * LD + 8 * fg) = t;
    }
  }
  __syncthreads();
  f32x16 acc[kTFB][kTRB];
  layer_mfma_fb<W, kTFB, kTRB, 2>(a.packedT + (size_t)(b - 1) * W * W, H, wid, 0, lane, nullptr, acc);
  // g <- g + dz_b Wh_b in two halves of 32 rows through the LDS tile, which is free after
  // the loop: the accumulators go in row-major FP32 ([32][W + 4], 16-byte writes), then
  // a thread updates 8 consecutive rows of one feature with 16-byte accesses of g
  // (instead of one 4-byte access per accumulator).
  constexpr int TS = W + 4;
  static_assert(32 * TS * sizeof(float) <= kRows * LD * sizeof(__bf16), "half a tile in FP32 fits the LDS tile");
  float* T = reinterpret_cast<float*>(smem);
#pragma unroll
  for (int rb = 0; rb < kTRB; ++rb) {
    __syncthreads();   // the tile (rb = 0) or the previous half (rb = 1) has been read
#pragma unroll
    for (int fb = 0; fb < kTFB; ++fb)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = 32 * (kTFB * wid + fb) + 8 * j + 4 * half;
        *reinterpret_cast<float4*>(T + col * TS + k) =
            make_float4(acc[fb][rb][4 * j], acc[fb][rb][4 * j + 1], acc[fb][rb][4 * j + 2], acc[fb][rb][4 * j + 3]);
      }
    __syncthreads();
    for (int task = tid; task < 4 * W; task += NT) {   // (feature k, rows 32 rb + 8 rr ..)
      const int k = task >> 2, rr = task & 3;
      const int rl = 32 * rb + 8 * rr;
      const size_t o = tix(W, k, r0 + rl);
      float gv[8];
      if (b == L) {
#pragma unroll
        for (int e = 0; e < 8; ++e) gv[e] = a.dy[r0 + rl + e] * wout[k];
      } else {
        const float4 g0 = *reinterpret_cast<const float4*>(a.g + o);
        const float4 g1 = *reinterpret_cast<const float4*>(a.g + o + 4);
        gv[0] = g0.x; gv[1] = g0.y; gv[2] = g0.z; gv[3] = g0.w;
        gv[4] = g1.x; gv[5] = g1.y; gv[6] = g1.z; gv[7] = g1.w;
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) gv[e] = gv[e] + T[(8 * rr + e) * TS + k];
      if (b > 1) {
        *reinterpret_cast<float4*>(a.g + o) = make_float4(gv[0], gv[1], gv[2], gv[3]);
        *reinterpret_cast<float4*>(a.g + o + 4) = make_float4(gv[4], gv[5], gv[6], gv[7]);
      } else {
        bf16x8 d;
#pragma unroll
        for (int e = 0; e < 8; ++e) d[e] = (__bf16)gv[e];
        *reinterpret_cast<bf16x8*>(a.dzT + o) = d;
      }
    }
  }
}

// The sums of the dW_1 splits of every dz slot (k_grad_w1 with one slot per blockIdx.z):
// slot 0 into W_0 and b_0, slot b into block b's Wx_b and c_b (split_sum_64).
__global__ __launch_bounds__(1024) void k_rt_sum_w1(ResTrainArgs a, const float* __restrict__ part, int R) {
  __shared__ float ws[16][64];
  const int W = a.net.width, in_dim = a.net.in_dim, nw1 = W * (in_dim + 1), s = blockIdx.y;
  const int o = blockIdx.x * 64 + (threadIdx.x & 63);
  const float t = split_sum_64(part + (size_t)s * R * nw1, R, nw1, o, ws);
  float* out = a.grad + (s == 0 ? 0 : res_block_base(W, in_dim, s - 1) + (size_t)W * W);
  if (threadIdx.x < 64 && o < nw1) out[o] = t;
}

// Wh_b^T of every block in MFMA A-operand order (packed_coords, transposed).
__global__ void k_pack_resT(MlpArgs net, __bf16* __restrict__ packedT) {
  const int W = net.width;
  const int64_t per = (int64_t)W * W, total = per * net.n_hidden;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(g / per);
    int row, colk;
    packed_coords(g - (int64_t)b * per, W, true, &row, &colk);
    packedT[g] = (__bf16)net.params[res_block_base(W, net.in_dim, b) + (size_t)row * W + colk];
  }
}

// Fixed-order sums of the dW splits of k_grad_w (blocks 1..L as its layers 2..L+1): Wh_b.
// (Its bias sums are not used here: c_b comes with Wx_b from k_grad_w1.)
__global__ void k_rt_grad_reduce(ResTrainArgs a, const float* __restrict__ part) {
  const int W = a.net.width, in_dim = a.net.in_dim, L = a.net.n_hidden;
  const int64_t per = (int64_t)W * W, total = per * L;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(g / per);
    const int64_t o = g - b * per;
    float s = 0.f;
    for (int sp = 0; sp < kSplitW; ++sp) s += part[((size_t)b * kSplitW + sp) * per + o];
    a.grad[res_block_base(W, in_dim, b) + o] = s;
  }
}

// Running statistics of every block: mu <- (1 - m) mu + m mean, var <- (1 - m) var +
// m var_B B / (B - 1) (B > 1; the variance is left as it is for a single row).
__global__ void k_rt_running(ResTrainArgs a, float* __restrict__ params) {
  const int W = a.net.width, L = a.net.n_hidden;
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < W * L; g += gridDim.x * blockDim.x) {
    const int b = g / W, f = g - b * W;
    const float* st = a.stats + (size_t)b * 3 * W;
    float* q = params + res_block_base(W, a.net.in_dim, b) + (size_t)W * W + (size_t)W * a.net.in_dim + 3 * W;
    q[f] = (1.f - kBnMomentum) * q[f] + kBnMomentum * st[f];
    if (a.B > 1)
      q[W + f] = (1.f - kBnMomentum) * q[W + f] + kBnMomentum * (float)((double)st[2 * W + f] * a.B / (a.B - 1));
  }
}

__global__ void k_fill_f32(float* __restrict__ p, int64_t n, float v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

template <int W>
hipError_t launch_train_res_t(ResTrainArgs a, float* part_w, float* part_w1, float* loss_out, hipStream_t st) {
  const MlpArgs& n = a.net;
  const int L = n.n_hidden;
  const unsigned tiles = (unsigned)(a.Bp / kRows);
  const size_t lds_f = (size_t)kRows * (W + kResXCols + kLdsPad) * sizeof(__bf16);
  const size_t lds_b = (size_t)kRows * (W + kLdsPad) * sizeof(__bf16);
  static bool attr = false;
  hipError_t e;
  if (!attr) {
    if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_rt_fwd<W>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_f)) != hipSuccess ||
        (e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_rt_bwd<W>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_b)) != hipSuccess)
      return e;
    attr = true;
  }
  const int64_t np = (int64_t)res_block_base(W, n.in_dim, L) + W + 1;
  hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)std::min<int64_t>((np + 255) / 256, 4096)), dim3(256), 0, st, a.grad,
                     np, 0.f);
  const unsigned sgrid = (unsigned)((W + 63) / 64);
  for (int b = 1; b <= L; ++b) {
    hipLaunchKernelGGL((k_rt_fwd<W>), dim3(tiles), dim3(train_threads<W>()), lds_f, st, a, b);
    hipLaunchKernelGGL(k_rt_stats, dim3(sgrid), dim3(64 * kStatGroups), 0, st, a, b, 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_rt_out<W>), dim3(tiles), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_rt_out_reduce, dim3((W + 2 + 63) / 64), dim3(1024), 0, st, a, loss_out);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  for (int b = L; b >= 1; --b) {
    if (b < L) hipLaunchKernelGGL((k_rt_bstats<W>), dim3(tiles), dim3(256), 0, st, a, b);
    hipLaunchKernelGGL(k_rt_stats, dim3(sgrid), dim3(64 * kStatGroups), 0, st, a, b, 1);
    hipLaunchKernelGGL((k_rt_bwd<W>), dim3(tiles), dim3(train_threads<W>()), lds_b, st, a, b);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // Wh_b and c_b: k_grad_w over (dz slot b, h slot b - 1) as its layers 2..L+1
  TrainArgs t{};
  t.net = n;
  t.net.n_hidden = L + 1;
  t.B = a.B;
  t.Bp = a.Bp;
  t.dzT = a.dzT;
  t.aT = a.hT;
  t.grad = a.grad;
  const unsigned gw_blocks = (unsigned)((W / gw_tf<W>()) * (W / gw_tk<W>()) * kSplitW * L);
  hipLaunchKernelGGL((k_grad_w<W>), dim3(gw_blocks), dim3(256), 0, st, t, part_w);
  hipLaunchKernelGGL(k_rt_grad_reduce, dim3(2048), dim3(256), 0, st, a, part_w);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // W_0 and b_0 (dz slot 0 = g_0), Wx_b and c_b (slot b) against the FP32 input: all
  // L + 1 slots in one launch, then their fixed-order sums in one launch
  {
    TrainArgs u = t;
    u.dzT = a.dzT;
    u.h0T = a.xT;
    hipLaunchKernelGGL(k_grad_w1, dim3((unsigned)((W + 255) / 256), (unsigned)w1_splits(a.Bp), (unsigned)(L + 1)),
                       dim3(256), 0, st, u, part_w1);
    const int nw1 = W * (n.in_dim + 1);
    hipLaunchKernelGGL(k_rt_sum_w1, dim3((unsigned)((nw1 + 63) / 64), (unsigned)(L + 1)), dim3(1024), 0, st, a,
                       part_w1, w1_splits(a.Bp));
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipGetLastError();
}

}  // namespace

int64_t train_rows_padded(int64_t B) { return (B + 255) / 256 * 256; }

size_t train_part_w_elems(const MlpArgs& n) {   // dW_l splits, then db_l splits
  return n.n_hidden >= 2 ? (size_t)kSplitW * (n.n_hidden - 1) * n.width * (n.width + 1) : 0;
}
size_t train_part_w1_elems(const MlpArgs& n, int64_t Bp) {
  // the dW_1 splits; the loss partials (Bp / 64 floats) and the output-layer partials
  // borrow the same space first
  return std::max({(size_t)w1_splits((int)Bp) * n.width * (n.in_dim + 1), (size_t)(Bp / 64),
                   (size_t)out_blocks((int)Bp) * (n.width + 1)});
}

hipError_t launch_train_step(const MlpArgs& net, const float* samples, const int* idx, int B, int Bp, __bf16* aT,
                             __bf16* dzT, float* h0T, float* y, float* dy, const __bf16* packed,
                             const __bf16* packedT, float* grad, float* part_w, float* part_w1, float sigma,
                             int clamp_pred, float* loss_out, hipStream_t st) {
  TrainArgs a{net, samples, idx, B, Bp, aT, dzT, h0T, y, dy, packed, packedT, grad, clamp_pred};
  switch (net.width) {
    case 128: return launch_train_t<128>(a, part_w, part_w1, sigma, loss_out, st);
    case 256: return launch_train_t<256>(a, part_w, part_w1, sigma, loss_out, st);
    case 512: return launch_train_t<512>(a, part_w, part_w1, sigma, loss_out, st);
    default: return hipErrorInvalidValue;
  }
}

size_t train_res_part_w_elems(const MlpArgs& n) { return (size_t)kSplitW * n.n_hidden * n.width * (n.width + 1); }
size_t train_res_part_w1_elems(const MlpArgs& n, int64_t Bp) {   // one region per dz slot
  return (size_t)w1_splits((int)Bp) * n.width * (n.in_dim + 1) * (n.n_hidden + 1);
}

hipError_t launch_train_step_res(const MlpArgs& net, const float* samples, const int* idx, int B, int Bp,
                                 const ResTrainWs& w, float sigma, float* grad, float* loss_out, hipStream_t st) {
  const int W = net.width;
  hipError_t e = launch_pack_bf16(net, 0, w.packed, st);
  if (e != hipSuccess) return e;
  const int64_t nT = (int64_t)net.n_hidden * W * W;
  hipLaunchKernelGGL(k_pack_resT, dim3((unsigned)std::min<int64_t>((nT + 255) / 256, 4096)), dim3(256), 0, st, net,
                     w.packedT);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  ResTrainArgs a{net,    samples, idx,    B,      Bp,     w.xT, w.hT,     w.aT,      w.dzT, w.g,
                 w.part, w.stats, w.bsum, w.y,    w.dy,   w.pout, w.packed, w.packedT, grad,  sigma};
  switch (W) {
    case 128: return launch_train_res_t<128>(a, w.part_w, w.part_w1, loss_out, st);
    case 256: return launch_train_res_t<256>(a, w.part_w, w.part_w1, loss_out, st);
    case 512: return launch_train_res_t<512>(a, w.part_w, w.part_w1, loss_out, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_bn_running(const MlpArgs& net, const ResTrainWs& w, int B, float* params, hipStream_t st) {
  ResTrainArgs a{};
  a.net = net;
  a.B = B;
  a.stats = w.stats;
  hipLaunchKernelGGL(k_rt_running, dim3((unsigned)((net.width * net.n_hidden + 255) / 256)), dim3(256), 0, st, a,
                     params);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, float* m, float* v, const float* g, int64_t n, float lr, float b1, float b2,
                       float eps, int64_t step, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const double bc1 = 1.0 - pow((double)b1, (double)step);
  const double bc2 = 1.0 - pow((double)b2, (double)step);
  const float step_size = (float)(lr / bc1);
  const float inv_sqrt_bc2 = (float)(1.0 / sqrt(bc2));
  hipLaunchKernelGGL(k_adam, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)), dim3(256), 0, st, p, m, v, g,
                     n, lr, b1, b2, eps, step_size, inv_sqrt_bc2);
  return hipGetLastError();
}

}  // namespace sv
