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
//   k_pack_bf16 (x2)  W_l and W_l^T in MFMA operand order (sv_mlp.hip)
//   k_train_fwd       per 64-row tile: all layers, activations to aT, y (the inference
//                     kernel's tile shape, one in-place LDS tile, two blocks per CU)
//   k_train_loss      dy and per-block loss partials; k_train_loss_sum: the loss
//                     (fixed-order reductions)
//   k_train_bwd       per 64-row tile: dz of every layer via W_l^T MFMA, to dzT
//   k_grad_w          dW_l = dz_l^T a_{l-1} for l >= 2 (MFMA, split over the batch; both
//                     operands staged in LDS)
//   k_grad_reduce     fixed-order sum of the splits
//   k_grad_rows       w_out and b_out gradients (one block per output)
//   k_grad_w1         dW_1 = dz_1^T h0 and db_1 in FP32 (lanes along the batch, split over
//                     the batch) + fixed-order sum (db_l for l >= 2 is summed by k_grad_w
//                     from its staged dz rows)
//   k_adam            Adam update of the FP32 masters
#include <math.h>

#include "sv_internal.h"
#include "sv_mlp_common.h"

namespace sv {
namespace {

constexpr int kRows = kTileRows;
constexpr int kSplitW = 16;       // batch splits of the dW GEMM

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
      *reinterpret_cast<bf16x8*>(outT + tix(W, 8 * fg + f, r0 + 8 * rg)) = o;
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
      a.h0T[(size_t)j * a.Bp + r0 + r] = v;
    }
    h0s[r][j] = v;
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
  __syncthreads();
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
    layer_mfma_fb<W, kTFB, kTRB, 2>(a.packed + (size_t)(l - 2) * W * W, H, wid, 0, lane, n.params + off_b(n, l),
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
  if (tid < kRows) {
    float yv = wout[W];
#pragma unroll
    for (int w = 0; w < NW; ++w) yv += part[w][tid];
    a.y[r0 + tid] = yv;
  }
}

// dy of 256 rows per block and the block's sum of the clamped L1 terms (fixed-order tree)
// into part[block]; k_train_loss_sum adds the partials in a fixed order.
__global__ __launch_bounds__(256) void k_train_loss(TrainArgs a, float sigma, float* __restrict__ part) {
  __shared__ float red[256];
  const int in_dim = a.net.in_dim;
  const int b = blockIdx.x * 256 + threadIdx.x;   // < Bp
  float s = 0.f, g = 0.f;
  if (b < a.B) {
    const float yv = a.y[b];
    const float d = a.samples[(size_t)a.idx[b] * (in_dim + 1) + in_dim];
    const bool live = !a.clamp_pred || fabsf(yv) < sigma;   // d clamp(y) / dy
    const float yc = a.clamp_pred ? fminf(fmaxf(yv, -sigma), sigma) : yv;
    const float r = yc - fminf(fmaxf(d, -sigma), sigma);
    s = fabsf(r);
    g = live ? (r > 0.f ? 1.f : (r < 0.f ? -1.f : 0.f)) / (float)a.B : 0.f;
  }
  a.dy[b] = g;
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// The mean clamped-L1 loss from the n block partials, in a fixed order (one block).
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
  for (int f = tid; f < W; f += NT) {   // dz_L = dy * w_out * sigma(z_L)
    const float wo = n.params[off_out(n) + f];
    const __bf16* aL = a.aT + (size_t)(L - 1) * W * a.Bp + tix(W, f, r0);
    __bf16* dzL = a.dzT + (size_t)(L - 1) * W * a.Bp + tix(W, f, r0);
#pragma unroll
    for (int c = 0; c < kRows / 8; ++c) {
      const bf16x8 av = *reinterpret_cast<const bf16x8*>(aL + 8 * c);
      bf16x8 out;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int r = 8 * c + e;
        const float g = a.dy[r0 + r] * wo * softplus_grad_from_out((float)av[e]);
        out[e] = (__bf16)g;
        H[r * LD + f] = out[e];
      }
      *reinterpret_cast<bf16x8*>(dzL + 8 * c) = out;
    }
  }
  __syncthreads();
  for (int l = L; l >= 2; --l) {
    // dh_{l-1}[r][k] = sum_f dz_l[r][f] W_l[f][k]: A operand = W_l^T packed
    f32x16 acc[kTFB][kTRB];
    layer_mfma_fb<W, kTFB, kTRB, 2>(a.packedT + (size_t)(l - 2) * W * W, H, wid, 0, lane, nullptr, acc);
    __syncthreads();   // every wave has read the tile (and copied it out)
    // the activations of layer l - 1 into the free tile, then dz_{l-1} over them in place:
    // each lane reads and writes the same (row, 4 features) pieces
    load_tile_T<W, NT>(a.aT + (size_t)(l - 2) * W * a.Bp, H, r0);
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
// Both operands are batch-contiguous rows ([feature][batch]); a lane's MFMA fragment is
// 16 bytes of one row, so reading fragments straight from memory touches a cache line
// per lane and re-fetches each line once per k-step.  Instead a block stages chunks of
// kGwChunk batch rows of its TF dz rows and TK a rows in LDS with coalesced 16-byte
// loads (a row's chunk is one 128-byte line), prefetching the next chunk into registers
// during the MFMAs, and its 4 waves read fragments from LDS: wave (wf, wk) owns rows
// (TF / 2) wf .. and columns (TK / 2) wk .. as (TF / 64) x (TK / 64) MFMA tiles of
// 32 x 32.  At W >= 256 the block tile is 256 x 256 (each dz and activation row read by
// two blocks; 256 accumulator registers per lane, one wave per SIMD): 1.71 ms per
// training step, against 1.81 for 128 x 256 tiles in 128-row chunks and 2.22 for
// 128 x 256 in 64-row chunks with two blocks per CU.
constexpr int kGwChunk = 64;                   // batch rows per LDS stage
constexpr int kGwLd = kGwChunk + kLdsPad;      // LDS row stride (elements)

template <int W>
constexpr int gw_tk() { return W >= 256 ? 256 : W; }   // output columns per block
template <int W>
constexpr int gw_tf() { return W >= 256 ? 256 : W; }   // output rows per block

template <int W>
__global__ __launch_bounds__(256) void k_grad_w(TrainArgs a, float* __restrict__ part) {
  constexpr int TF = gw_tf<W>(), TK = gw_tk<W>();
  constexpr int FBW = TF / 64;                       // row (feature) blocks per wave
  constexpr int RB = TK / 64;                        // column blocks per wave
  constexpr int SEG = kGwChunk / 8;                  // 16-byte segments per row and chunk
  __shared__ __align__(16) __bf16 As[TF * kGwLd];
  __shared__ __align__(16) __bf16 Bs[TK * kGwLd];
  int g = blockIdx.x;
  const int tk = g % (W / TK); g /= (W / TK);
  const int tf = g % (W / TF); g /= (W / TF);
  const int s = g % kSplitW; g /= kSplitW;
  const int l = g + 2;                              // layer 2..L
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int half = lane >> 5, col = lane & 31;
  const int wf = wid & 1, wk = wid >> 1;
  const int f0 = tf * TF, k0 = tk * TK;
  const int per = a.Bp / kSplitW;                   // multiple of 16 (Bp is a multiple of 256)
  const int b_begin = s * per, b_end = b_begin + per;
  const __bf16* dz = a.dzT + (size_t)(l - 1) * W * a.Bp;   // layer blocks
  const __bf16* ap = a.aT + (size_t)(l - 2) * W * a.Bp;
  f32x16 acc[FBW][RB];
#pragma unroll
  for (int fb = 0; fb < FBW; ++fb)
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) acc[fb][rb] = f32x16{};
  float dbs = 0.f;   // this thread's half-row sum of dz for the bias gradient (tk == 0)
  // thread tid moves segments tid + 256 q, q < NQ, of each chunk: row r, columns c8..
  constexpr int NQ = (TF + TK) * SEG / 256;
  static_assert((TF + TK) * SEG % 256 == 0, "whole passes");
  bf16x8 stage[NQ];
  auto fetch = [&](int b, int kc) {                  // the chunk at b into registers
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int id = tid + 256 * q, r = id / SEG, c8 = 8 * (id - r * SEG);
      const __bf16* src = r < TF ? dz + tix(W, f0 + r, b + c8) : ap + tix(W, k0 + r - TF, b + c8);
      if (c8 < kc) stage[q] = *reinterpret_cast<const bf16x8*>(src);
    }
  };
  fetch(b_begin, min(kGwChunk, b_end - b_begin));
  for (int b = b_begin; b < b_end; b += kGwChunk) {
    const int kc = min(kGwChunk, b_end - b);        // multiple of 16
    __syncthreads();                                // every wave is done with the last stage
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int id = tid + 256 * q, r = id / SEG, c8 = 8 * (id - r * SEG);
      __bf16* dst = r < TF ? As + r * kGwLd : Bs + (r - TF) * kGwLd;
      if (c8 < kc) *reinterpret_cast<bf16x8*>(dst + c8) = stage[q];
    }
    __syncthreads();
    if (b + kGwChunk < b_end) fetch(b + kGwChunk, min(kGwChunk, b_end - b - kGwChunk));   // in flight during the MFMAs
    if (tk == 0) {   // the bias gradient db_l[f] = sum_b dz_l[f][b]: 256 / TF threads per row
      constexpr int TPR = 256 / TF, CPT = kGwChunk / TPR;
      const __bf16* row = As + (tid / TPR) * kGwLd + CPT * (tid % TPR);
      const int n = min(CPT, kc - CPT * (tid % TPR));
      for (int c = 0; c < n; ++c) dbs += (float)row[c];
    }
    for (int ks = 0; ks < kc / 16; ++ks) {
      bf16x8 x[FBW], y[RB];
#pragma unroll
      for (int fb = 0; fb < FBW; ++fb)
        x[fb] = *reinterpret_cast<const bf16x8*>(As + ((TF / 2) * wf + 32 * fb + col) * kGwLd + 16 * ks + 8 * half);
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
        y[rb] = *reinterpret_cast<const bf16x8*>(Bs + ((TK / 2) * wk + 32 * rb + col) * kGwLd + 16 * ks + 8 * half);
#pragma unroll
      for (int fb = 0; fb < FBW; ++fb)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
          acc[fb][rb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x[fb], y[rb], acc[fb][rb], 0, 0, 0);
    }
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
          P[(size_t)(f0 + (TF / 2) * wf + 32 * fb + 8 * j + 4 * half + i) * W + k0 + (TK / 2) * wk + 32 * rb + col] =
              acc[fb][rb][4 * j + i];
  if (tk == 0) {   // bias partials after the weight partials: [L - 1][kSplitW][W]
    constexpr int TPR = 256 / TF;
    const float d = TPR == 2 ? dbs + __shfl_xor(dbs, 1, 64) : dbs;
    if (tid % TPR == 0)
      part[(size_t)(a.net.n_hidden - 1) * kSplitW * W * W + ((size_t)(l - 2) * kSplitW + s) * W + f0 + tid / TPR] = d;
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

// One block of 256 threads per output: rows 0 .. W-1 are the w_out gradient
// (sum_b dy[b] a_L[f][b]), row W is b_out's (sum_b dy[b]).  Each thread sums a strided
// share of the batch with four loads in flight, then the block combines the shares in
// a fixed order.  (Every hidden layer's bias gradient comes with its weights: db_1 from
// k_grad_w1, db_l, l >= 2, from k_grad_w.)
__global__ __launch_bounds__(256) void k_grad_rows(TrainArgs a) {
  __shared__ float red[4];
  const MlpArgs& n = a.net;
  const int W = n.width, L = n.n_hidden;
  const int row = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  float s = 0.f;
  if (row < W) {
    const __bf16* v = a.aT + (size_t)(L - 1) * W * a.Bp;   // the last hidden layer's block
    float u[4] = {0.f, 0.f, 0.f, 0.f};
    for (int b0 = 8 * tid; b0 < a.Bp; b0 += 4 * 2048) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int b = b0 + q * 2048;
        if (b < a.Bp) {
          const bf16x8 x = *reinterpret_cast<const bf16x8*>(v + tix(W, row, b));
#pragma unroll
          for (int e = 0; e < 8; ++e) u[q] = fmaf((float)x[e], a.dy[b + e], u[q]);
        }
      }
    }
    s = (u[0] + u[1]) + (u[2] + u[3]);
  } else {
    for (int b = tid; b < a.Bp; b += 256) s += a.dy[b];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) red[wid] = s;
  __syncthreads();
  if (tid == 0) a.grad[off_out(n) + row] = (red[0] + red[1]) + (red[2] + red[3]);
}

// dW_1[f][j] = sum_b dz_1[f][b] h0[j][b] and db_1[f] = sum_b dz_1[f][b] in FP32, over one
// batch split per block.  A wave takes kW1F features; its lanes run along the batch (8
// consecutive rows each, so one load reads a 1 KB stretch of a dz row and of an input
// row), and every lane keeps kW1F x (in_dim + 1) partial sums, combined across the wave
// at the end in a fixed order.
constexpr int kW1F = 4;            // features per wave
constexpr int kW1Split = 16;       // batch splits

__global__ __launch_bounds__(256) void k_grad_w1(TrainArgs a, float* __restrict__ part) {
  constexpr int kMaxIn = 3 + 2 * SV_MAX_DOF;
  const int W = a.net.width, in_dim = a.net.in_dim;
  const int lane = threadIdx.x & 63;
  const int fw = (blockIdx.x * 4 + (threadIdx.x >> 6)) * kW1F;   // first feature of the wave
  const int s = blockIdx.y;
  if (fw >= W) return;                                             // wave-uniform
  const int per = a.Bp / kW1Split;                                 // multiple of 16
  const int b_begin = s * per, b_end = b_begin + per;
  float acc[kW1F][kMaxIn], accb[kW1F];
#pragma unroll
  for (int q = 0; q < kW1F; ++q) {
    accb[q] = 0.f;
#pragma unroll
    for (int jj = 0; jj < kMaxIn; ++jj) acc[q][jj] = 0.f;
  }
  for (int b = b_begin + 8 * lane; b < b_end; b += 512) {
    float g[kW1F][8];
#pragma unroll
    for (int q = 0; q < kW1F; ++q) {
      const bf16x8 x = *reinterpret_cast<const bf16x8*>(a.dzT + tix(W, fw + q, b));
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        g[q][e] = (float)x[e];
        accb[q] += g[q][e];
      }
    }
#pragma unroll
    for (int jj = 0; jj < kMaxIn; ++jj) {
      if (jj >= in_dim) continue;
      const float4 u = *reinterpret_cast<const float4*>(a.h0T + (size_t)jj * a.Bp + b);
      const float4 v = *reinterpret_cast<const float4*>(a.h0T + (size_t)jj * a.Bp + b + 4);
      const float h[8] = {u.x, u.y, u.z, u.w, v.x, v.y, v.z, v.w};
#pragma unroll
      for (int q = 0; q < kW1F; ++q)
#pragma unroll
        for (int e = 0; e < 8; ++e) acc[q][jj] = fmaf(g[q][e], h[e], acc[q][jj]);
    }
  }
  float* ps = part + (size_t)s * W * (in_dim + 1);   // this split: dW_1 [W][in_dim], then db_1 [W]
#pragma unroll
  for (int q = 0; q < kW1F; ++q) {
#pragma unroll
    for (int jj = 0; jj < kMaxIn; ++jj) {
      if (jj >= in_dim) continue;
      float v = acc[q][jj];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      if (lane == 0) ps[(size_t)(fw + q) * in_dim + jj] = v;
    }
    float v = accb[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) ps[(size_t)W * in_dim + fw + q] = v;
  }
}

// dW_1 and db_1 (contiguous in the flat vector) from the splits, in a fixed order.
__global__ void k_grad_w1_reduce(TrainArgs a, const float* __restrict__ part, int chunks) {
  const int n = a.net.width * (a.net.in_dim + 1);
  for (int o = blockIdx.x * blockDim.x + threadIdx.x; o < n; o += gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int c = 0; c < chunks; ++c) s += part[(size_t)c * n + o];
    a.grad[o] = s;
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
  hipLaunchKernelGGL((k_train_fwd<W>), dim3(tiles), dim3(train_threads<W>()), lds, st, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // the loss partials borrow part_w1, which k_grad_w1 fills only later in the step
  hipLaunchKernelGGL(k_train_loss, dim3((unsigned)(a.Bp / 256)), dim3(256), 0, st, a, sigma, part_w1);
  hipLaunchKernelGGL(k_train_loss_sum, dim3(1), dim3(1024), 0, st, a, part_w1, a.Bp / 256, loss_out);
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
  hipLaunchKernelGGL(k_grad_rows, dim3((unsigned)(W + 1)), dim3(256), 0, st, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_grad_w1, dim3((unsigned)((W / kW1F + 3) / 4), kW1Split), dim3(256), 0, st, a, part_w1);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_grad_w1_reduce, dim3(64), dim3(256), 0, st, a, part_w1, kW1Split);
  return hipGetLastError();
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
    if (j < in_dim) {
      v = a.samples[(size_t)a.idx[min(r0 + r, a.B - 1)] * (in_dim + 1) + j];
      if (b == 1) a.xT[(size_t)j * a.Bp + r0 + r] = v;
    }
    xs[r][j] = v;
  }
  __syncthreads();
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
    load_tile_T<W, NT, LD>(a.hT + (size_t)(b - 2) * slab, H, r0);
    __syncthreads();
    const float* q = rt_block(a, b - 1) + (size_t)W * W + (size_t)W * in_dim + W;   // gamma, beta
    const float* st = a.stats + (size_t)(b - 2) * 3 * W;
    const __bf16* ap = a.aT + (size_t)(b - 2) * slab;
    for (int f = wid; f < W; f += NW) {   // lane = row: one 128-byte line of a per feature
      const float av = (float)ap[tix(W, f, r0 + lane)];
      __bf16* hp = H + lane * LD + f;
      *hp = (__bf16)((float)*hp + fmaf(q[f] * st[W + f], av - st[f], q[W + f]));
    }
    __syncthreads();
    store_tile_T<W, NT, LD>(H, a.hT + (size_t)(b - 1) * slab, r0);
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
        const bf16x4 v = {(__bf16)fmaxf(acc[fb][rb][4 * j + 0], 0.f), (__bf16)fmaxf(acc[fb][rb][4 * j + 1], 0.f),
                          (__bf16)fmaxf(acc[fb][rb][4 * j + 2], 0.f), (__bf16)fmaxf(acc[fb][rb][4 * j + 3], 0.f)};
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

// Batch sums per feature from the per-tile sums in a.part: 64 features per block, four
// thread groups over the tiles, combined in FP64 in a fixed order.
// mode 0 (forward, block b): stats[b] = (mean, 1 / sqrt(var + eps), var) of a_b.
// mode 1 (backward, block b): bsum = (sum g, sum g n); the gradients of beta_b and gamma_b.
__global__ __launch_bounds__(256) void k_rt_stats(ResTrainArgs a, int b, int mode) {
  __shared__ double red[2][4][64];
  const int W = a.net.width, tiles = a.Bp / kRows;
  const int fl = threadIdx.x & 63, tg = threadIdx.x >> 6;
  const int f = blockIdx.x * 64 + fl;
  double s0 = 0.0, s1 = 0.0;
  if (f < W)
    for (int t = tg; t < tiles; t += 4) {
      s0 += a.part[((size_t)t * 2) * W + f];
      s1 += a.part[((size_t)t * 2 + 1) * W + f];
    }
  red[0][tg][fl] = s0;
  red[1][tg][fl] = s1;
  __syncthreads();
  if (tg != 0 || f >= W) return;
  const double S0 = (red[0][0][fl] + red[0][1][fl]) + (red[0][2][fl] + red[0][3][fl]);
  const double S1 = (red[1][0][fl] + red[1][1][fl]) + (red[1][2][fl] + red[1][3][fl]);
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

// h_L = h_{L-1} + gamma_L (a_L - mu) inv + beta_L in FP32 (kept in LDS), the prediction,
// the loss terms and dy of the tile's rows, then per feature: the tile's sums of dy h_L
// (the w_out gradient) and, for the last block's BatchNorm backward with g = dy w_out,
// of g and g n_L.
template <int W>
__global__ __launch_bounds__(256) void k_rt_out(ResTrainArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  float (*hs)[W + 1] = reinterpret_cast<float (*)[W + 1]>(smem);
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
  float yp = 0.f;
  for (int f = wid; f < W; f += 4) {   // lane = row
    const size_t o = tix(W, f, r0 + lane);
    const float h = (float)hp[o] + fmaf(q[f] * st[W + f], (float)ap[o] - st[f], q[W + f]);
    hs[lane][f] = h;
    yp = fmaf(wout[f], h, yp);
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
  for (int f = tid; f < W; f += 256) {
    float sh = 0.f, sn = 0.f;
    const bf16x8* arow = reinterpret_cast<const bf16x8*>(ap + tix(W, f, r0));
    for (int c = 0; c < kRows / 8; ++c) {
      const bf16x8 av = arow[c];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int r = 8 * c + e;
        sh = fmaf(dys[r], hs[r][f], sh);
        sn = fmaf(dys[r], ((float)av[e] - st[f]) * st[W + f], sn);
      }
    }
    po[f] = sh;
    a.part[((size_t)tile * 2) * W + f] = wout[f] * sdy;
    a.part[((size_t)tile * 2 + 1) * W + f] = wout[f] * sn;
  }
  if (tid == 0) {
    float sl = 0.f;
    for (int r = 0; r < kRows; ++r) sl += ls[r];
    po[W] = sdy;
    po[W + 1] = sl;
  }
}

// The output layer's gradient and the loss from the per-tile partials, in a fixed order.
__global__ void k_rt_out_reduce(ResTrainArgs a, float* __restrict__ loss_out) {
  const int W = a.net.width, tiles = a.Bp / kRows;
  float* gout = a.grad + res_block_base(W, a.net.in_dim, a.net.n_hidden);
  for (int o = blockIdx.x * blockDim.x + threadIdx.x; o < W + 2; o += gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int t = 0; t < tiles; ++t) s += a.pout[(size_t)t * (W + 2) + o];
    if (o <= W) gout[o] = s;
    else if (loss_out) *loss_out = s / (float)a.B;
  }
}

// Per-tile sums of g = dL/dh_b and g n_b (b < L): one thread per feature, 64 rows each.
template <int W>
__global__ __launch_bounds__(256) void k_rt_bstats(ResTrainArgs a, int b) {
  const int tile = blockIdx.x, r0 = tile * kRows;
  const float* st = a.stats + (size_t)(b - 1) * 3 * W;
  const __bf16* ap = a.aT + (size_t)(b - 1) * W * a.Bp;
  for (int f = threadIdx.x; f < W; f += 256) {
    const float4* grow = reinterpret_cast<const float4*>(a.g + tix(W, f, r0));
    const bf16x8* arow = reinterpret_cast<const bf16x8*>(ap + tix(W, f, r0));
    float s = 0.f, sn = 0.f;
    for (int c = 0; c < kRows / 8; ++c) {
      const float4 g0 = grow[2 * c], g1 = grow[2 * c + 1];
      const float gv[8] = {g0.x, g0.y, g0.z, g0.w, g1.x, g1.y, g1.z, g1.w};
      const bf16x8 av = arow[c];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        s += gv[e];
        sn = fmaf(gv[e], ((float)av[e] - st[f]) * st[W + f], sn);
      }
    }
    a.part[((size_t)tile * 2) * W + f] = s;
    a.part[((size_t)tile * 2 + 1) * W + f] = sn;
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
  const bool valid = r0 + lane < a.B;
  const float dyr = b == L ? a.dy[r0 + lane] : 0.f;
  for (int f = wid; f < W; f += NW) {   // lane = row
    const size_t o = tix(W, f, r0 + lane);
    const float gv = b == L ? dyr * wout[f] : a.g[o];
    const float av = (float)ap[o];
    const float nn = (av - st[f]) * st[W + f];
    const float dz = (valid && av > 0.f)
                         ? gamma[f] * st[W + f] * (gv - a.bsum[f] * invB - nn * (a.bsum[W + f] * invB))
                         : 0.f;
    const __bf16 d16 = (__bf16)dz;
    H[lane * LD + f] = d16;
    dzs[o] = d16;
  }
  __syncthreads();
  f32x16 acc[kTFB][kTRB];
  layer_mfma_fb<W, kTFB, kTRB, 2>(a.packedT + (size_t)(b - 1) * W * W, H, wid, 0, lane, nullptr, acc);
#pragma unroll
  for (int fb = 0; fb < kTFB; ++fb)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k = 32 * (kTFB * wid + fb) + 8 * j + 4 * half + i;
#pragma unroll
        for (int rb = 0; rb < kTRB; ++rb) {
          const int r = 32 * rb + col;
          const size_t o = tix(W, k, r0 + r);
          const float gb = b == L ? a.dy[r0 + r] * wout[k] : a.g[o];
          const float gn = gb + acc[fb][rb][4 * j + i];
          if (b > 1) a.g[o] = gn;
          else a.dzT[o] = (__bf16)gn;
        }
      }
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
  const size_t lds_o = (size_t)kRows * (W + 1) * sizeof(float);
  static bool attr = false;
  hipError_t e;
  if (!attr) {
    if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_rt_fwd<W>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_f)) != hipSuccess ||
        (e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_rt_bwd<W>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_b)) != hipSuccess ||
        (e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_rt_out<W>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_o)) != hipSuccess)
      return e;
    attr = true;
  }
  const int64_t np = (int64_t)res_block_base(W, n.in_dim, L) + W + 1;
  hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)std::min<int64_t>((np + 255) / 256, 4096)), dim3(256), 0, st, a.grad,
                     np, 0.f);
  const unsigned sgrid = (unsigned)((W + 63) / 64);
  for (int b = 1; b <= L; ++b) {
    hipLaunchKernelGGL((k_rt_fwd<W>), dim3(tiles), dim3(train_threads<W>()), lds_f, st, a, b);
    hipLaunchKernelGGL(k_rt_stats, dim3(sgrid), dim3(256), 0, st, a, b, 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_rt_out<W>), dim3(tiles), dim3(256), lds_o, st, a);
  hipLaunchKernelGGL(k_rt_out_reduce, dim3((W + 2 + 255) / 256), dim3(256), 0, st, a, loss_out);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  for (int b = L; b >= 1; --b) {
    if (b < L) hipLaunchKernelGGL((k_rt_bstats<W>), dim3(tiles), dim3(256), 0, st, a, b);
    hipLaunchKernelGGL(k_rt_stats, dim3(sgrid), dim3(256), 0, st, a, b, 1);
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
  // W_0 and b_0 (dz slot 0 = g_0), Wx_b and c_b (slot b) against the FP32 input
  for (int s = 0; s <= L; ++s) {
    TrainArgs u = t;
    u.dzT = a.dzT + (size_t)s * W * a.Bp;
    u.h0T = a.xT;
    u.grad = a.grad + (s == 0 ? 0 : res_block_base(W, n.in_dim, s - 1) + (size_t)W * W);
    hipLaunchKernelGGL(k_grad_w1, dim3((unsigned)((W / kW1F + 3) / 4), kW1Split), dim3(256), 0, st, u, part_w1);
    hipLaunchKernelGGL(k_grad_w1_reduce, dim3(64), dim3(256), 0, st, u, part_w1, kW1Split);
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
  // the dW_1 splits; the loss partials (Bp / 256 floats) borrow the same space first
  return std::max<size_t>((size_t)kW1Split * n.width * (n.in_dim + 1), (size_t)(Bp / 256));
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
size_t train_res_part_w1_elems(const MlpArgs& n) { return (size_t)kW1Split * n.width * (n.in_dim + 1); }

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
