// Swept-volume network f_theta(x, q0, q1) -> delta_hat (paper Sec. IV-A, Fig. 1).
//
// The network is a plain softplus MLP: h_0 = [x; q0; q1], h_l = softplus(W_l h_{l-1}
// + b_l) for l = 1..L, delta_hat = w_out . h_L + b_out.  Parameters arrive as one flat
// FP32 vector, per layer W (row-major [out][in]) then b.
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
#include <math.h>

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
__global__ void k_pack_bf16(MlpArgs net, int transpose, __bf16* __restrict__ packed) {
  const int W = net.width;
  const int64_t per_layer = (int64_t)W * W;
  const int64_t total = per_layer * (net.n_hidden - 1);
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
    const int l = (int)(g / per_layer);               // 0-based hidden-layer index (layer l+2 of 1..L)
    int row, colk;
    packed_coords(g - (int64_t)l * per_layer, W, transpose != 0, &row, &colk);
    const float* Wl = net.params + (size_t)W * net.in_dim + W + (size_t)l * (per_layer + W);
    packed[g] = (__bf16)Wl[(size_t)row * W + colk];
  }
}

// Block: W/64 waves x 64 threads, R = 64 rows (queries) of one motion.  LDS holds two
// activation buffers [64][W + 8] BF16 (the pad spreads rows over the LDS banks).
// Wave w owns output features [64w, 64w + 64) = 2 feature blocks x 2 row blocks of
// 32x32 MFMA tiles.
constexpr int kBRows = kTileRows;
constexpr int kPad = kLdsPad;

// Inputs: every (motion, point) pair of (mo, c), or with `rows` the c.n rows
// rows[i][0:in_dim] (one motion slot, m = 0; layer 0 then runs unsplit per row).
template <int W>
__global__ __launch_bounds__(W) void k_mlp_bf16(MlpArgs net, MotionArgs mo, CloudArgs c, int tiles,
                                                const float* __restrict__ rows, int64_t row_stride,
                                                const __bf16* __restrict__ packed, float* __restrict__ out,
                                                float tau, int* __restrict__ lists, int* __restrict__ counts) {
  constexpr int NW = W / 64;          // waves
  constexpr int LD = W + kPad;        // LDS row stride (elements)
  constexpr int kMaxIn = 3 + 2 * SV_MAX_DOF;
  extern __shared__ __align__(16) unsigned char smem[];
  __bf16* H0 = reinterpret_cast<__bf16*>(smem);
  __bf16* H1 = H0 + kBRows * LD;
  __shared__ float part[NW][kBRows];
  __shared__ float xyz[3][kBRows];
  __shared__ float h0s[kBRows][kMaxIn];

  const int m = blockIdx.x / tiles;
  const int tile = blockIdx.x - m * tiles;
  const int r0 = tile * kBRows;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int dof = net.dof;
  if (rows) {
    // Layer 0 per row in FP32: z[f] = W0[f] . h0 + b0[f]; thread f.
    for (int e = tid; e < kBRows * net.in_dim; e += W) {
      const int r = e / net.in_dim, j = e - r * net.in_dim;
      h0s[r][j] = rows[(size_t)min(r0 + r, c.n - 1) * row_stride + j];
    }
    const int f = tid;
    float w[kMaxIn];
#pragma unroll
    for (int j = 0; j < kMaxIn; ++j) {
      w[j] = 0.f;
      if (j < net.in_dim) w[j] = net.params[(size_t)f * net.in_dim + j];
    }
    const float b0 = net.params[(size_t)W * net.in_dim + f];
    __syncthreads();
    for (int r = 0; r < kBRows; ++r) {
      float z = b0;
#pragma unroll
      for (int j = 0; j < kMaxIn; ++j)
        if (j < net.in_dim) z = fmaf(w[j], h0s[r][j], z);
      H0[r * LD + f] = (__bf16)softplus_fast(z);
    }
  } else if (tid < kBRows) {
    const int i = min(r0 + tid, c.n - 1);
    xyz[0][tid] = c.x[i];
    xyz[1][tid] = c.y[i];
    xyz[2][tid] = c.z[i];
  }
  // Layer 0 in FP32: z[f] = W0[f][0:3] . x + (W0[f][3:] . [q0; q1] + b0[f]); thread f.
  if (!rows) {
    const int f = tid;
    const float* w0 = net.params + (size_t)f * net.in_dim;
    float u = net.params[(size_t)W * net.in_dim + f];
    for (int j = 0; j < dof; ++j) {
      u = fmaf(w0[3 + j], mo.q0[(size_t)m * dof + j], u);
      u = fmaf(w0[3 + dof + j], mo.q1[(size_t)m * dof + j], u);
    }
    const float wx = w0[0], wy = w0[1], wz = w0[2];
    __syncthreads();
#pragma unroll 4
    for (int r = 0; r < kBRows; ++r) {
      const float z = fmaf(wx, xyz[0][r], fmaf(wy, xyz[1][r], fmaf(wz, xyz[2][r], u)));
      H0[r * LD + f] = (__bf16)softplus_fast(z);
    }
  }
  __syncthreads();

  const float* bias_base = net.params + (size_t)W * net.in_dim + W;   // start of layer 1
  const int half = lane >> 5, col = lane & 31;
  __bf16* Hin = H0;
  __bf16* Hout = H1;
  float p0 = 0.f, p1 = 0.f;   // output-layer partial sums for rows col and 32 + col
  for (int l = 1; l < net.n_hidden; ++l) {
    const __bf16* Wp = packed + (size_t)(l - 1) * W * W;
    const float* bl = bias_base + (size_t)(l - 1) * ((size_t)W * W + W) + (size_t)W * W;
    f32x16 acc00, acc01, acc10, acc11;
    layer_mfma<W>(Wp, Hin, wid, lane, acc00, acc01, acc10, acc11);
    // Epilogue.  acc index 4j+i of tile (fb, rb) is feature 64 wid + 32 fb + 8j + 4 half + i
    // of row 32 rb + col.
    const bool last = l + 1 == net.n_hidden;
    const float* wout = bias_base + (size_t)(net.n_hidden - 1) * ((size_t)W * W + W);
#pragma unroll
    for (int fb = 0; fb < 2; ++fb) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int f = 64 * wid + 32 * fb + 8 * j + 4 * half;
        const float4 bb = *reinterpret_cast<const float4*>(bl + f);
        const f32x16& t0 = fb == 0 ? acc00 : acc10;
        const f32x16& t1 = fb == 0 ? acc01 : acc11;
        const float s00 = softplus_fast(t0[4 * j + 0] + bb.x), s01 = softplus_fast(t0[4 * j + 1] + bb.y);
        const float s02 = softplus_fast(t0[4 * j + 2] + bb.z), s03 = softplus_fast(t0[4 * j + 3] + bb.w);
        const float s10 = softplus_fast(t1[4 * j + 0] + bb.x), s11 = softplus_fast(t1[4 * j + 1] + bb.y);
        const float s12 = softplus_fast(t1[4 * j + 2] + bb.z), s13 = softplus_fast(t1[4 * j + 3] + bb.w);
        if (last) {
          const float4 wo = *reinterpret_cast<const float4*>(wout + f);
          p0 = fmaf(wo.x, s00, fmaf(wo.y, s01, fmaf(wo.z, s02, fmaf(wo.w, s03, p0))));
          p1 = fmaf(wo.x, s10, fmaf(wo.y, s11, fmaf(wo.z, s12, fmaf(wo.w, s13, p1))));
        } else {
          bf16x4 v0 = {(__bf16)s00, (__bf16)s01, (__bf16)s02, (__bf16)s03};
          bf16x4 v1 = {(__bf16)s10, (__bf16)s11, (__bf16)s12, (__bf16)s13};
          *reinterpret_cast<bf16x4*>(Hout + col * LD + f) = v0;
          *reinterpret_cast<bf16x4*>(Hout + (32 + col) * LD + f) = v1;
        }
      }
    }
    __syncthreads();
    __bf16* t = Hin;
    Hin = Hout;
    Hout = t;
  }
  if (net.n_hidden == 1) {
    // no hidden MFMA layer: output layer straight from layer 0 (FP32 accumulate of BF16 h1)
    const float* wout = bias_base;
    for (int r = wid; r < kBRows; r += NW) {
      float s = 0.f;
      for (int f = lane; f < W; f += 64) s = fmaf(wout[f], (float)Hin[r * LD + f], s);
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
      if (lane == 0) part[0][r] = s;
    }
    __syncthreads();
    for (int w = 1; w < NW; ++w)
      if (tid < kBRows) part[w][tid] = 0.f;
  } else {
    // lanes col and col + 32 hold disjoint features of the same rows
    p0 += __shfl_xor(p0, 32, 64);
    p1 += __shfl_xor(p1, 32, 64);
    if (half == 0) {
      part[wid][col] = p0;
      part[wid][32 + col] = p1;
    }
  }
  __syncthreads();
  if (wid == 0) {
    const float* wout = bias_base + (size_t)(net.n_hidden - 1) * ((size_t)W * W + W);
    float y = wout[W];
#pragma unroll
    for (int w = 0; w < NW; ++w) y += part[w][lane];
    const int i = r0 + lane;
    const bool valid = i < c.n;
    if (out && valid) out[(size_t)m * c.n + i] = y;
    if (lists) {
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

inline unsigned grid_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

template <int W>
hipError_t launch_bf16_t(const MlpArgs& net, const MotionArgs& mo, const CloudArgs& c, const float* rows,
                         int64_t row_stride, const __bf16* packed, float* out, float tau, int* lists, int* counts,
                         hipStream_t st) {
  const int tiles = (c.n + kBRows - 1) / kBRows;
  const int64_t blocks = (rows ? 1 : mo.n) * tiles;
  if (blocks == 0) return hipSuccess;
  const size_t lds = 2 * (size_t)kBRows * (W + kPad) * sizeof(__bf16);
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mlp_bf16<W>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((k_mlp_bf16<W>), dim3((unsigned)blocks), dim3(W), lds, st, net, mo, c, tiles, rows, row_stride,
                     packed, out, tau, lists, counts);
  return hipGetLastError();
}

hipError_t launch_f32(const MlpArgs& net, const MotionArgs& mo, const CloudArgs& c, const float* rows,
                      int64_t row_stride, float* out, hipStream_t st) {
  const int tiles = (c.n + kF32Rows - 1) / kF32Rows;
  const int64_t blocks = (rows ? 1 : mo.n) * tiles;
  if (blocks == 0) return hipSuccess;
  const size_t lds = (size_t)kF32Rows * net.width * sizeof(float);
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mlp_f32),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(k_mlp_f32, dim3((unsigned)blocks), dim3(256), lds, st, net, mo, c, tiles, rows, row_stride, out);
  return hipGetLastError();
}

}  // namespace

bool mlp_bf16_supported(int width) { return width == 128 || width == 256 || width == 512; }

size_t mlp_packed_elems(const MlpArgs& net) { return (size_t)net.width * net.width * (net.n_hidden - 1); }

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
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pack_bf16(const MlpArgs& net, int transpose, __bf16* packed, hipStream_t st) {
  const int64_t total = (int64_t)mlp_packed_elems(net);
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pack_bf16, dim3((unsigned)std::min<int64_t>(grid_for(total, 256), 4096)), dim3(256), 0, st, net,
                     transpose, packed);
  return hipGetLastError();
}

hipError_t launch_mlp_bf16(const MlpArgs& net, const MotionArgs& mo, const CloudArgs& c, const __bf16* packed,
                           float* out, float tau, int* lists, int* counts, hipStream_t st) {
  switch (net.width) {
    case 128: return launch_bf16_t<128>(net, mo, c, nullptr, 0, packed, out, tau, lists, counts, st);
    case 256: return launch_bf16_t<256>(net, mo, c, nullptr, 0, packed, out, tau, lists, counts, st);
    case 512: return launch_bf16_t<512>(net, mo, c, nullptr, 0, packed, out, tau, lists, counts, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sv
