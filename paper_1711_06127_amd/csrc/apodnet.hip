// Learned adaptive apodization: a four-layer 1D convolutional network (32 channels, kernel 5)
// that maps the delayed channel samples of a pixel to one weight per element, trained to
// reproduce minimum-variance weights.  Training and inference run on the matrix cores:
// every convolution is an implicit GEMM on v_mfma_f32_32x32x16_bf16 (bf16 operands, binary32
// accumulation), for the forward pass, the data gradient (the same convolution with the
// kernel flipped and transposed) and the weight gradient (a GEMM whose reduction runs over
// pixels and positions).  Adam keeps binary32 master weights.
//
// Layout conventions (M = elements per pixel, a multiple of 32):
//   activations / gradients  bf16 [pixel][M][C]   (C = 32, or 1 for the network's input/output)
//   weights                  float W[co][ci][5], biases b[co]; flattened parameter vector
//                            W1 b1 W2 b2 W3 b3 W4 b4 (10657 values)
//   packed MFMA weights      bf16 [k-step][lane][8]: the B operand of each k-step of a layer
//
// MFMA 32x32x16 operand layout (per lane l of the wave):
//   A[i][k], i = l % 32, k = 8 (l / 32) + 0..7        (8 bf16 per lane)
//   B[k][j], j = l % 32, k = 8 (l / 32) + 0..7
//   D[i][j], j = l % 32, i = 8 (r / 4) + 4 (l / 32) + r % 4, r = 0..15  (16 floats per lane)
#include <type_traits>

#include "common.h"

namespace usbf {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kNC = 32;   // channels
constexpr int kKS = 5;    // kernel size
constexpr int kNetThreads = 256;

// parameter offsets in the flattened vector
constexpr int kW1 = 0, kB1 = 160, kW2 = 192, kB2 = 5312, kW3 = 5344, kB3 = 10464, kW4 = 10496, kB4 = 10656;
constexpr int kNParams = 10657;

// packed weights (bf16): forward L1 (1 step), L2, L3 (10 steps), L4 (10 steps);
// data-gradient L4' (1 step), L3', L2' (10 steps)
constexpr int kStepElems = 64 * 8;
constexpr int kPkF1 = 0, kPkF2 = kPkF1 + 1 * kStepElems, kPkF3 = kPkF2 + 10 * kStepElems,
              kPkF4 = kPkF3 + 10 * kStepElems, kPkD4 = kPkF4 + 10 * kStepElems, kPkD3 = kPkD4 + 1 * kStepElems,
              kPkD2 = kPkD3 + 10 * kStepElems, kPkEnd = kPkD2 + 10 * kStepElems;

// network state in one caller-owned device buffer
struct NetState {
  float* params;  // [kNParams] binary32 master weights
  float* m;       // Adam first moments
  float* v;       // Adam second moments
  int* step;      // Adam step count
  __bf16* packed; // [kPkEnd]
};

constexpr size_t align256(size_t b) { return (b + 255) & ~size_t(255); }
constexpr size_t kStateBytes = 3 * align256(kNParams * sizeof(float)) + 256 + align256(kPkEnd * sizeof(__bf16));

__host__ __device__ inline NetState carve_state(void* base) {
  char* p = static_cast<char*>(base);
  NetState s;
  s.params = reinterpret_cast<float*>(p);
  s.m = reinterpret_cast<float*>(p + align256(kNParams * sizeof(float)));
  s.v = reinterpret_cast<float*>(p + 2 * align256(kNParams * sizeof(float)));
  s.step = reinterpret_cast<int*>(p + 3 * align256(kNParams * sizeof(float)));
  s.packed = reinterpret_cast<__bf16*>(p + 3 * align256(kNParams * sizeof(float)) + 256);
  return s;
}

__device__ inline float bf(__bf16 v) { return float(v); }

// ---------------------------------------------------------------- weight packing

// B operand of k-step s of a convolution with CI input channels and kernel Wf(co, ci, t):
// B[k][j] = Wf(co = j, ci, t) with kappa = 16 s + k = t * CI + ci (CI = 32), kappa = t (CI = 1);
// zero where kappa >= 5 CI or co >= CO.
template <typename WF>
__device__ inline __bf16 packed_value(WF wf, int CI, int CO, int s, int lane, int e) {
  const int j = lane % 32, k = 8 * (lane / 32) + e;
  const int kappa = 16 * s + k;
  if (j >= CO || kappa >= kKS * CI) return __bf16(0.0f);
  const int t = kappa / CI, ci = kappa % CI;
  return __bf16(wf(j, ci, t));
}

__global__ void pack_kernel(NetState st) {
  const float* p = st.params;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < kPkEnd; idx += gridDim.x * blockDim.x) {
    int base, steps, CI, CO, layer;
    bool flip;
    if (idx < kPkF2) { base = kPkF1; CI = 1; CO = 32; layer = 1; flip = false; }
    else if (idx < kPkF3) { base = kPkF2; CI = 32; CO = 32; layer = 2; flip = false; }
    else if (idx < kPkF4) { base = kPkF3; CI = 32; CO = 32; layer = 3; flip = false; }
    else if (idx < kPkD4) { base = kPkF4; CI = 32; CO = 1; layer = 4; flip = false; }
    else if (idx < kPkD3) { base = kPkD4; CI = 1; CO = 32; layer = 4; flip = true; }
    else if (idx < kPkD2) { base = kPkD3; CI = 32; CO = 32; layer = 3; flip = true; }
    else { base = kPkD2; CI = 32; CO = 32; layer = 2; flip = true; }
    (void)steps;
    const int rel = idx - base;
    const int s = rel / kStepElems, lane = (rel % kStepElems) / 8, e = rel % 8;
    if (base == kPkF4) {
      // forward output layer as a product over channels only: A[t][ci] = W4[0][ci][t] (two
      // k-steps of 16 channels; rows t >= 5 and the remaining steps are zero)
      const int t = lane % 32, ci = 16 * s + 8 * (lane / 32) + e;
      st.packed[idx] = __bf16((s < 2 && t < kKS) ? p[kW4 + ci * kKS + t] : 0.0f);
      continue;
    }
    const int off = layer == 1 ? kW1 : layer == 2 ? kW2 : layer == 3 ? kW3 : kW4;
    const int lci = (layer == 1) ? 1 : 32;  // the layer's own input channels
    // forward: W[co][ci][t]; data gradient: W'[ci'][co'][t'] = W[co'][ci'][4 - t'] with the
    // roles of input and output channels exchanged
    auto wf = [&](int co, int ci, int t) -> float {
      if (!flip) return p[off + (co * lci + ci) * kKS + t];
      return p[off + (ci * lci + co) * kKS + (kKS - 1 - t)];
    };
    st.packed[idx] = packed_value(wf, CI, CO, s, lane, e);
  }
}

// ---------------------------------------------------------------- convolution on MFMA

enum Epilogue { kRelu = 0, kLinear = 1, kMasked = 2 };

// out[p][m][co] = epi( sum_{t, ci} in[p][m + t - 2][ci] W(co, ci, t) ), CI, CO in {1, 32}.
//   kRelu:   bf16(relu(acc + b[co]))            (hidden layers)
//   kLinear: float(acc + b[0]) into outf[p][m]  (CO = 1: the network output)
//   kMasked: bf16(acc * (mask[p][m][co] > 0))   (data gradient through the ReLU of the layer below)
// One workgroup stages one pixel's input rows (with two zero rows at each end) in LDS; each
// wave computes 32-position tiles.
template <int CI, int CO, int EPI>
__global__ __launch_bounds__(kNetThreads) void conv_kernel(const __bf16* __restrict__ in, int n_pix, int M,
                                                           const __bf16* __restrict__ packed,
                                                           const float* __restrict__ bias,
                                                           const __bf16* __restrict__ mask,
                                                           __bf16* __restrict__ outb, float* __restrict__ outf) {
  constexpr int STEPS = CI == 1 ? 1 : (kKS * CI) / 16;
  constexpr int ROW = CI == 1 ? 1 : CI;  // bf16 per LDS row
  extern __shared__ __align__(16) __bf16 rows[];  // [(M + 4) * ROW] (+8 slack for CI = 1)
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  bf16x8 bw[STEPS];
#pragma unroll
  for (int s = 0; s < STEPS; ++s) bw[s] = *reinterpret_cast<const bf16x8*>(packed + (s * 64 + lane) * 8);
  const int j = lane % 32, hi = lane / 32;
  const float bj = (EPI != kMasked && j < CO) ? bias[j] : 0.0f;
  const int n_mt = M / 32;
  for (int p = blockIdx.x; p < n_pix; p += gridDim.x) {
    __syncthreads();
    const __bf16* ip = in + size_t(p) * M * ROW;
    const int total = (M + 4) * ROW + (CI == 1 ? 8 : 0);
    for (int idx = threadIdx.x; idx < total; idx += kNetThreads) {
      const int r = idx / ROW - 2;
      rows[idx] = (r >= 0 && r < M) ? ip[r * ROW + idx % ROW] : __bf16(0.0f);
    }
    __syncthreads();
    for (int mt = wave; mt < n_mt; mt += kNetThreads / 64) {
      f32x16 acc = {};
      const int i = lane % 32;
#pragma unroll
      for (int s = 0; s < STEPS; ++s) {
        bf16x8 a;
        if constexpr (CI == 1) {
          // A[i][k] = in[32 mt + i + k - 2] for k < 5, else 0
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const int k = 8 * hi + e;
            a[e] = (k < kKS) ? rows[32 * mt + i + k] : __bf16(0.0f);
          }
        } else {
          // kappa = 16 s + k: tap t = s / 2, channels (s % 2) * 16 + 8 hi .. +8
          const int t = s / 2, ci0 = (s % 2) * 16 + 8 * hi;
          a = *reinterpret_cast<const bf16x8*>(rows + (32 * mt + i + t) * ROW + ci0);
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bw[s], acc, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = 32 * mt + 8 * (r / 4) + 4 * hi + (r % 4);
        if (j >= CO) continue;
        const size_t o = (size_t(p) * M + m) * CO + j;
        if constexpr (EPI == kRelu) {
          outb[o] = __bf16(fmaxf(acc[r] + bj, 0.0f));
        } else if constexpr (EPI == kLinear) {
          outf[size_t(p) * M + m] = acc[r] + bj;
        } else {
          outb[o] = __bf16(bf(mask[o]) > 0.0f ? acc[r] : 0.0f);
        }
      }
    }
  }
}

// ---------------------------------------------------------------- fused forward

// The whole forward pass of one pixel in one workgroup of four waves, activations kept in LDS:
// normalise into a0, then the four convolutions; wave v computes the 32-position tiles
// v, v + 4, ... of every layer.  Each product is issued transposed, D[co][position] =
// W[co][kappa] act[kappa][position] (the packed weights serve as the A operand: the MFMA lane
// layouts of A and B coincide), so that every lane ends with four runs of four consecutive
// channels of one position, stored with 8-byte LDS writes.  The one-channel output layer is
// computed as Z[t][position] = sum_ci W4[ci][t] a3[position][ci] (two k-steps instead of ten)
// and w[m] = b4 + sum_t Z[t][m + t - 2] on the vector ALUs.  The packed weights stay in
// registers for the workgroup's lifetime, and the next pixel's samples are prefetched into
// registers.  With SAVE the layer inputs a0..a3 are also written to global memory for the
// backward pass; with y the weighted sum y = sum_m w[m] x[m] (the delay-and-sum fallback where
// a weight is not finite) is formed in the same pass.
// LDS: a0 [M + 16] bf16 (position m at index m + 2, zeros around); two buffers of M + 4 rows
// of kRowStride bf16 (position m at row m + 2; rows 0, 1, M + 2, M + 3 stay zero; 32 channels
// and 8 bf16 of padding, so that the 16-byte operand reads of consecutive positions spread
// over the banks); the output layer's Z [5][M + 4] float in the second buffer; biases.
constexpr int kFwdThreads = 256;
constexpr int kRowStride = kNC + 8;

__host__ __device__ constexpr size_t fused_buf_elems(int M) { return size_t(M + 4) * kRowStride; }
__host__ __device__ constexpr size_t fused_lds_bytes(int M) {
  return (size_t(M + 16) + 2 * fused_buf_elems(M)) * sizeof(__bf16) + 3 * kNC * sizeof(float);
}

typedef float f32x2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
typedef short i16x2v __attribute__((ext_vector_type(2)));
// ReLU of two values rounded to bf16 (round to nearest even), packed: one packed conversion and
// one packed integer max -- a bf16 with the sign bit set is a negative int16, so max(., 0)
// zeroes it.  Rounding preserves sign and order, so this equals rounding the ReLU.
__device__ inline uint32_t relu_bf16x2(float lo, float hi) {
  const bf16x2v v = __builtin_convertvector((f32x2v){lo, hi}, bf16x2v);
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(i16x2v, v), (i16x2v){0, 0}));
}

template <bool SAVE>
__global__ __launch_bounds__(kFwdThreads) __attribute__((amdgpu_waves_per_eu(3))) void fused_forward_kernel(
    const float* __restrict__ x, int n_pix, int M, const __bf16* __restrict__ packed,
    const float* __restrict__ params, float* __restrict__ w, const float* __restrict__ fallback,
    float* __restrict__ y, __bf16* __restrict__ a0g, __bf16* __restrict__ a1g, __bf16* __restrict__ a2g,
    __bf16* __restrict__ a3g) {
  extern __shared__ __align__(16) __bf16 lds[];
  __bf16* a0 = lds;
  __bf16* bufA = lds + (M + 16);
  __bf16* bufB = bufA + fused_buf_elems(M);
  float* zt = reinterpret_cast<float*>(bufB + 2 * kRowStride);              // [5][M + 4], bufB past its zero rows
  float* bias = reinterpret_cast<float*>(bufB + fused_buf_elems(M));        // [3][32]
  const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
  const int j = lane % 32, hi = lane / 32;
  const int n_mt = M / 32;

  const bf16x8 w1 = *reinterpret_cast<const bf16x8*>(packed + kPkF1 + lane * 8);
  bf16x8 w2[10], w3[10], w4[2];
#pragma unroll
  for (int s = 0; s < 10; ++s) {
    w2[s] = *reinterpret_cast<const bf16x8*>(packed + kPkF2 + (s * 64 + lane) * 8);
    w3[s] = *reinterpret_cast<const bf16x8*>(packed + kPkF3 + (s * 64 + lane) * 8);
  }
#pragma unroll
  for (int s = 0; s < 2; ++s) w4[s] = *reinterpret_cast<const bf16x8*>(packed + kPkF4 + (s * 64 + lane) * 8);
  const float b4 = params[kB4];
  if (tid < 3 * kNC) bias[tid] = params[(tid < kNC ? kB1 : tid < 2 * kNC ? kB2 - kNC : kB3 - 2 * kNC) + tid];
  // zero margins (never written afterwards)
  if (tid < 16) a0[tid < 2 ? tid : M + tid] = __bf16(0.0f);  // 0, 1, M + 2 .. M + 15
  for (int k = tid; k < 4 * kRowStride; k += kFwdThreads) {
    const int row = k / kRowStride < 2 ? k / kRowStride : M + k / kRowStride;  // rows 0, 1, M + 2, M + 3
    bufA[row * kRowStride + k % kRowStride] = __bf16(0.0f);
    bufB[row * kRowStride + k % kRowStride] = __bf16(0.0f);
  }

  // accumulator initialised with the biases of the 16 channels this lane's rows hold
  auto bias_init = [&](int layer) {
    f32x16 acc;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 b = *reinterpret_cast<const float4*>(bias + layer * kNC + 8 * q + 4 * hi);
      acc[4 * q + 0] = b.x;
      acc[4 * q + 1] = b.y;
      acc[4 * q + 2] = b.z;
      acc[4 * q + 3] = b.w;
    }
    return acc;
  };
  // ReLU, bf16 and the stores of a tile's D[co][position] into dst.  Lane (j, hi) holds
  // channels 8q + 4 hi .. + 3 of position j for q = 0..3; one exchange with lane j + 32
  // (v_permlane32_swap: the upper half-wave of the first operand trades places with the lower
  // half-wave of the second) leaves lane hi = 0 with channels 0..15 and lane hi = 1 with
  // 16..31, written as two 16-byte stores -- 8-byte stores of consecutive rows kRowStride apart
  // would meet every bank group twice in a pass (16-byte stores of 8 lanes do not).
  auto store_relu = [&](const f32x16& acc, int mt, __bf16* dst) {
    uint32_t v[4][2];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      v[q][0] = relu_bf16x2(acc[4 * q + 0], acc[4 * q + 1]);
      v[q][1] = relu_bf16x2(acc[4 * q + 2], acc[4 * q + 3]);
    }
    uint4 o[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const auto s0 = __builtin_amdgcn_permlane32_swap(v[h][0], v[h + 2][0], false, false);
      const auto s1 = __builtin_amdgcn_permlane32_swap(v[h][1], v[h + 2][1], false, false);
      o[h] = make_uint4(s0[0], s1[0], s0[1], s1[1]);
    }
    __bf16* row = dst + (32 * mt + j + 2) * kRowStride + 16 * hi;
    *reinterpret_cast<uint4*>(row) = o[0];
    *reinterpret_cast<uint4*>(row + 8) = o[1];
  };
  // 32 x 32 channel layer from src into dst
  auto layer32 = [&](const __bf16* src, const bf16x8* wk, int layer, __bf16* dst) {
    for (int mt = wave; mt < n_mt; mt += kFwdThreads / 64) {
      f32x16 acc = bias_init(layer);
#pragma unroll
      for (int s = 0; s < 10; ++s) {
        const int t = s / 2, ci0 = (s % 2) * 16 + 8 * hi;
        const bf16x8 b = *reinterpret_cast<const bf16x8*>(src + (32 * mt + j + t) * kRowStride + ci0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wk[s], b, acc, 0, 0, 0);
      }
      store_relu(acc, mt, dst);
    }
  };
  // copy the M rows of a 32-channel LDS buffer to global [M][32] with 16-byte stores
  auto save32 = [&](const __bf16* buf, __bf16* g) {
    for (int k = tid; k < M * 4; k += kFwdThreads)
      reinterpret_cast<uint4*>(g)[k] = *reinterpret_cast<const uint4*>(buf + (k / 4 + 2) * kRowStride + 8 * (k % 4));
  };

  // the pixel's samples, prefetched one pixel ahead: lane holds positions lane + 64 k (every
  // wave the whole pixel, so that each forms the sum of squares itself without a cross-wave step)
  float xr[4];
  auto load_x = [&](int pp) {
    const float* xp = x + size_t(pp) * M;
#pragma unroll
    for (int k = 0; k < 4; ++k) xr[k] = (lane + 64 * k < M) ? xp[lane + 64 * k] : 0.0f;
  };
  if (int(blockIdx.x) < n_pix) load_x(blockIdx.x);
  for (int p = blockIdx.x; p < n_pix; p += gridDim.x) {
    __syncthreads();  // the previous pixel is done with a0 and the buffers
    float ss = 0.0f, xm = 0.0f, xc[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      ss = __builtin_fmaf(xr[k], xr[k], ss);
      xm = (k == wave) ? xr[k] : xm;  // position tid = lane + 64 wave
      if constexpr (!SAVE) xc[k] = xr[k];  // kept past the prefetch of the next pixel (for y)
    }
    for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
    const float inv = 1.0f / sqrtf(ss / float(M) + 1e-12f);
    if (p + int(gridDim.x) < n_pix) load_x(p + gridDim.x);
    if (tid < M) {
      const __bf16 v = __bf16(xm * inv);
      a0[tid + 2] = v;
      if constexpr (SAVE) a0g[size_t(p) * M + tid] = v;
    }
    __syncthreads();
    // layer 1 (one input channel): B[k][position] = a0[position + k - 2] for k < 5.  Every lane
    // loads the eight samples a0[p .. p + 7], p = position + 8 hi (two bytes apart, so from
    // five aligned words with funnel shifts): the packed weights are zero for k >= 5, and the
    // samples there are finite, so they add nothing.
    for (int mt = wave; mt < n_mt; mt += kFwdThreads / 64) {
      const int p = 32 * mt + j + 8 * hi;
      const uint32_t* m = reinterpret_cast<const uint32_t*>(a0) + (p >> 1);
      const uint32_t sh = (p & 1) * 16;
      uint32_t d[5];
#pragma unroll
      for (int k = 0; k < 5; ++k) d[k] = m[k];
      uint4 bw;
      bw.x = __builtin_amdgcn_alignbit(d[1], d[0], sh);
      bw.y = __builtin_amdgcn_alignbit(d[2], d[1], sh);
      bw.z = __builtin_amdgcn_alignbit(d[3], d[2], sh);
      bw.w = __builtin_amdgcn_alignbit(d[4], d[3], sh);
      const bf16x8 b = __builtin_bit_cast(bf16x8, bw);
      const f32x16 acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w1, b, bias_init(0), 0, 0, 0);
      store_relu(acc, mt, bufA);
    }
    __syncthreads();
    if constexpr (SAVE) save32(bufA, a1g + size_t(p) * M * kNC);
    layer32(bufA, w2, 1, bufB);
    __syncthreads();
    if constexpr (SAVE) save32(bufB, a2g + size_t(p) * M * kNC);
    layer32(bufB, w3, 2, bufA);
    __syncthreads();
    if constexpr (SAVE) save32(bufA, a3g + size_t(p) * M * kNC);
    // output layer: Z[t][position] for t < 5 (rows t of D; lane hi = 0 holds t = 0..3, hi = 1 t = 4)
    for (int mt = wave; mt < n_mt; mt += kFwdThreads / 64) {
      f32x16 acc = {};
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const bf16x8 b = *reinterpret_cast<const bf16x8*>(bufA + (32 * mt + j + 2) * kRowStride + 16 * s + 8 * hi);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w4[s], b, acc, 0, 0, 0);
      }
      // Z[t][position] at zt[t][position + 2]: consecutive lanes write consecutive words
      float* zc = zt + 32 * mt + j + 2;
      if (hi == 0) {
#pragma unroll
        for (int t = 0; t < 4; ++t) zc[t * (M + 4)] = acc[t];
      } else {
        zc[4 * (M + 4)] = acc[0];
      }
    }
    // the two words before and after each row are zero (layer 2 used this memory)
    if (tid < 4 * kKS) zt[(tid / 4) * (M + 4) + ((tid & 3) < 2 ? (tid & 3) : M + (tid & 3))] = 0.0f;
    __syncthreads();
    float wm = 0.0f;
    if (tid < M) {
      // w[m] = b4 + sum_t Z[t][m + t - 2] (positions outside the pixel contribute 0)
      float s = 0.0f;
#pragma unroll
      for (int t = 0; t < kKS; ++t) s += zt[t * (M + 4) + tid + t];
      wm = s + b4;
      if (w) w[size_t(p) * M + tid] = wm;
    }
    if (!SAVE && y && wave == kFwdThreads / 64 - 1) {
      // the last wave (which holds no position for M <= 192) forms y = sum_m w[m] x[m] alone:
      // it has every sample of the pixel and re-forms the weights from Z exactly as above
      float acc = 0.0f;
      int bad = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int m = lane + 64 * k;
        if (m < M) {
          float s = 0.0f;
#pragma unroll
          for (int t = 0; t < kKS; ++t) s += zt[t * (M + 4) + m + t];
          const float wk = s + b4;
          acc = __builtin_fmaf(wk, xc[k], acc);
          bad |= !(fabsf(wk) < INFINITY);
        }
      }
      for (int off = 32; off > 0; off >>= 1) {
        acc += __shfl_xor(acc, off, 64);
        bad |= __shfl_xor(bad, off, 64);
      }
      if (lane == 0) y[p] = (bad && fallback) ? fallback[p] : acc;
    }
  }
}

// ---------------------------------------------------------------- loss and its gradient

// g4[p][m] = bf16(2 M (w - t) / P); per-block partial sums of (M w - M t)^2
__global__ void loss_kernel(const float* __restrict__ w, const float* __restrict__ target, int n_pix, int M,
                            __bf16* __restrict__ g4, float* __restrict__ loss_part) {
  __shared__ float red[kNetThreads / 64];
  const int64_t n = int64_t(n_pix) * M;
  const float scale = 2.0f * float(M) / float(n_pix);
  float ss = 0.0f;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    const float d = w[i] - target[i];
    g4[i] = __bf16(scale * d);
    const float e = float(M) * d;
    ss = __builtin_fmaf(e, e, ss);
  }
  for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = ss;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.0f;
    for (int k = 0; k < kNetThreads / 64; ++k) t += red[k];
    loss_part[blockIdx.x] = t;
  }
}

// ---------------------------------------------------------------- weight gradient on MFMA

// Partial sums over this workgroup's pixels of
//   dW[co][ci][t] = sum_{p, m} g[p][m][co] a[p][m + t - 2][ci],   db[co] = sum_{p, m} g[p][m][co]
// as D[co][kappa] = sum_m A[co][m] B[m][kappa] with A = g^T and B the shifted activations.
// Both are staged transposed in LDS ([channel][position], positions padded by 2 zeros at the
// front and 6 at the back so every 16-byte read is aligned); the 4 waves split the position
// k-steps of a pixel and their partial products are summed at the end.
// part[block][co * (5 CI) + kappa] and part[block][CO * 5 CI + co] (bias).
template <int CI, int CO>
__global__ __launch_bounds__(kNetThreads) void wgrad_kernel(const __bf16* __restrict__ g, const __bf16* __restrict__ a,
                                                            int n_pix, int M, float* __restrict__ part) {
  constexpr int NT = CI == 1 ? 1 : kKS;  // N-tiles of 32 columns of kappa
  constexpr int NK = kKS * CI;           // kappa columns used
  extern __shared__ __align__(16) __bf16 lds[];
  const int RS = M + 8;                  // padded row length
  __bf16* gT = lds;                      // [32][RS]
  __bf16* aT = lds + 32 * RS;            // [32][RS]
  float* red = reinterpret_cast<float*>(aT + 32 * RS);  // [32][NK + 1]
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int i = lane % 32, hi = lane / 32;
  f32x16 acc[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) acc[nt] = f32x16{};
  float dbias = 0.0f;
  const int ksteps = M / 16;
  for (int p = blockIdx.x; p < n_pix; p += gridDim.x) {
    __syncthreads();
    // transpose-stage g (CO channels; rows >= CO are zero) and a (CI channels)
    for (int idx = threadIdx.x; idx < 32 * RS; idx += kNetThreads) {
      const int c = idx / RS, q = idx % RS;
      const int m = q - 2;
      const bool in_m = m >= 0 && m < M;
      gT[idx] = (c < CO && q < M) ? g[(size_t(p) * M + q) * CO + c] : __bf16(0.0f);
      aT[idx] = (c < CI && in_m) ? a[(size_t(p) * M + m) * CI + c] : __bf16(0.0f);
    }
    __syncthreads();
    for (int s = wave; s < ksteps; s += kNetThreads / 64) {
      const int m0 = 16 * s + 8 * hi;
      const bf16x8 av = *reinterpret_cast<const bf16x8*>(gT + i * RS + m0);
      if (i < CO) {
#pragma unroll
        for (int e = 0; e < 8; ++e) dbias += bf(av[e]);
      }
      // positions m0 .. m0+7 shifted by t - 2 live at aT[.][m0 + t .. m0 + t + 7]
      const int col = CI == 1 ? 0 : i;  // channel of this lane's B column (CI = 32)
      const bf16x8 c0 = *reinterpret_cast<const bf16x8*>(aT + col * RS + m0);
      const bf16x8 c1 = *reinterpret_cast<const bf16x8*>(aT + col * RS + m0 + 8);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        bf16x8 b;
        if constexpr (CI == 1) {
          // column j = tap t (t < 5): B[m][t] = a0[m + t - 2]
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const int sh = e + i;  // element index into c0|c1
            const __bf16 v = sh < 8 ? c0[sh < 8 ? sh : 0] : c1[sh >= 8 && sh < 16 ? sh - 8 : 0];
            b[e] = (i < kKS) ? v : __bf16(0.0f);
          }
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e) b[e] = (e + nt < 8) ? c0[(e + nt) & 7] : c1[(e + nt - 8) & 7];
        }
        acc[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, b, acc[nt], 0, 0, 0);
      }
    }
  }
  // sum the four waves' partial products and bias sums
  __syncthreads();
  for (int w = 0; w < kNetThreads / 64; ++w) {
    if (wave == w) {
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int co = 8 * (r / 4) + 4 * hi + (r % 4);
          const int kappa = 32 * nt + i;
          if (co < CO && kappa < NK) {
            float& dst = red[co * (NK + 1) + kappa];
            dst = (w == 0 ? 0.0f : dst) + acc[nt][r];
          }
        }
      float db = dbias + __shfl_xor(dbias, 32, 64);
      if (hi == 0 && i < CO) {
        float& dst = red[i * (NK + 1) + NK];
        dst = (w == 0 ? 0.0f : dst) + db;
      }
    }
    __syncthreads();
  }
  float* out = part + size_t(blockIdx.x) * (CO * NK + CO);
  for (int idx = threadIdx.x; idx < CO * NK; idx += kNetThreads) out[idx] = red[(idx / NK) * (NK + 1) + idx % NK];
  for (int c = threadIdx.x; c < CO; c += kNetThreads) out[CO * NK + c] = red[c * (NK + 1) + NK];
}

// sum the per-block partials (fixed order) into the flattened gradient
__global__ void reduce_grad_kernel(const float* __restrict__ part, int n_blocks, int CO, int NK, int w_off, int b_off,
                                   float* __restrict__ grad) {
  const int n = CO * NK + CO;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += gridDim.x * blockDim.x) {
    float s = 0.0f;
    for (int b = 0; b < n_blocks; ++b) s += part[size_t(b) * n + idx];
    if (idx < CO * NK) {
      // kappa = t * CI + ci  ->  W[co][ci][t]
      const int co = idx / NK, kappa = idx % NK;
      const int CI = NK / kKS;
      const int t = kappa / CI, ci = kappa % CI;
      grad[w_off + (co * CI + ci) * kKS + t] = s;
    } else {
      grad[b_off + (idx - CO * NK)] = s;
    }
  }
}

__global__ void sum_kernel(const float* __restrict__ part, int n, float scale, float* __restrict__ out) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    float s = 0.0f;
    for (int i = 0; i < n; ++i) s += part[i];
    *out = s * scale;
  }
}

// ---------------------------------------------------------------- Adam

__global__ void adam_kernel(NetState st, const float* __restrict__ grad, float lr, float beta1, float beta2, float eps) {
  const int t = *st.step + 1;
  const float c1 = 1.0f - powf(beta1, float(t)), c2 = 1.0f - powf(beta2, float(t));
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kNParams; i += gridDim.x * blockDim.x) {
    const float g = grad[i];
    const float m = beta1 * st.m[i] + (1.0f - beta1) * g;
    const float v = beta2 * st.v[i] + (1.0f - beta2) * g * g;
    st.m[i] = m;
    st.v[i] = v;
    st.params[i] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
  }
}

__global__ void step_kernel(NetState st) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *st.step += 1;
}

// ---------------------------------------------------------------- weighted sum with DAS fallback

// y[p] = sum_e w[p][e] x[p][e]; a pixel with any non-finite weight takes fallback[p]
__global__ void weighted_kernel(const float* __restrict__ x, const float* __restrict__ w,
                                const float* __restrict__ fallback, int n_pix, int M, float* __restrict__ y) {
  const int lane = threadIdx.x % 64;
  const int p = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  if (p >= n_pix) return;
  float s = 0.0f;
  int bad = 0;
  for (int m = lane; m < M; m += 64) {
    const float wm = w[size_t(p) * M + m];
    bad |= !(fabsf(wm) < INFINITY);
    s = __builtin_fmaf(wm, x[size_t(p) * M + m], s);
  }
  for (int off = 32; off > 0; off >>= 1) {
    s += __shfl_xor(s, off, 64);
    bad |= __shfl_xor(bad, off, 64);
  }
  if (lane == 0) y[p] = (bad && fallback) ? fallback[p] : s;
}

// ---------------------------------------------------------------- host side

struct NetWs {
  __bf16 *a0, *a1, *a2, *a3, *g4, *g3, *g2, *g1;
  float *w, *part, *grad, *loss_part;
};

constexpr int kConvBlocks = 2048;
constexpr int kWgradBlocks = 512;
constexpr int kLossBlocks = 256;

size_t net_ws_bytes(int64_t n_pix, int64_t M, bool train) {
  const size_t act1 = align256(size_t(n_pix) * M * sizeof(__bf16));
  const size_t act32 = align256(size_t(n_pix) * M * kNC * sizeof(__bf16));
  const size_t wout = align256(size_t(n_pix) * M * sizeof(float));
  if (!train) return 0;  // the fused forward pass needs no workspace
  size_t b = act1 + 3 * act32 + wout;
  if (train)
    b += act1 + 3 * act32 + align256(size_t(kWgradBlocks) * (kNC * kKS * kNC + kNC) * sizeof(float)) +
         align256(kNParams * sizeof(float)) + align256(kLossBlocks * sizeof(float));
  return b;
}

static NetWs carve_ws(void* base, int64_t n_pix, int64_t M, bool train) {
  char* p = static_cast<char*>(base);
  const size_t act1 = align256(size_t(n_pix) * M * sizeof(__bf16));
  const size_t act32 = align256(size_t(n_pix) * M * kNC * sizeof(__bf16));
  NetWs w{};
  w.a0 = reinterpret_cast<__bf16*>(p); p += act1;
  w.a1 = reinterpret_cast<__bf16*>(p); p += act32;
  w.a2 = reinterpret_cast<__bf16*>(p); p += act32;
  w.a3 = reinterpret_cast<__bf16*>(p); p += act32;
  w.w = reinterpret_cast<float*>(p); p += align256(size_t(n_pix) * M * sizeof(float));
  if (train) {
    w.g4 = reinterpret_cast<__bf16*>(p); p += act1;
    w.g3 = reinterpret_cast<__bf16*>(p); p += act32;
    w.g2 = reinterpret_cast<__bf16*>(p); p += act32;
    w.g1 = reinterpret_cast<__bf16*>(p); p += act32;
    w.part = reinterpret_cast<float*>(p); p += align256(size_t(kWgradBlocks) * (kNC * kKS * kNC + kNC) * sizeof(float));
    w.grad = reinterpret_cast<float*>(p); p += align256(kNParams * sizeof(float));
    w.loss_part = reinterpret_cast<float*>(p);
  }
  return w;
}

template <int CI, int CO, int EPI>
static void launch_conv(const __bf16* in, int n_pix, int M, const __bf16* packed, const float* bias,
                        const __bf16* mask, __bf16* outb, float* outf, hipStream_t s) {
  const int blocks = std::min(n_pix, kConvBlocks);
  const size_t lds = (size_t(M + 4) * (CI == 1 ? 1 : CI) + 8) * sizeof(__bf16);
  hipLaunchKernelGGL((conv_kernel<CI, CO, EPI>), dim3(blocks), dim3(kNetThreads), lds, s, in, n_pix, M, packed, bias,
                     mask, outb, outf);
}

template <int CI, int CO>
static void launch_wgrad(const __bf16* g, const __bf16* a, int n_pix, int M, float* part, float* grad, int w_off,
                         int b_off, hipStream_t s) {
  constexpr int NK = kKS * CI;
  const int blocks = std::min(n_pix, kWgradBlocks);
  const size_t lds = size_t(2 * 32 * (M + 8)) * sizeof(__bf16) + size_t(32) * (NK + 1) * sizeof(float);
  hipLaunchKernelGGL((wgrad_kernel<CI, CO>), dim3(blocks), dim3(kNetThreads), lds, s, g, a, n_pix, M, part);
  hipLaunchKernelGGL(reduce_grad_kernel, dim3(8), dim3(256), 0, s, part, blocks, CO, NK, w_off, b_off, grad);
}

// a resident grid: as many workgroups as the compute units hold at once (the pixel loop is
// grid-strided, so a second round of workgroups would only start when the first has finished
// all its pixels)
template <bool SAVE>
static int fused_grid(int n_pix, size_t lds) {
  int dev = 0, n_cu = 256, per_cu = 0;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fused_forward_kernel<SAVE>, kFwdThreads, lds) !=
          hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  return std::max(1, std::min(n_pix, per_cu * n_cu));
}

// forward pass; with `save` the layer inputs go to the workspace for the backward pass; without,
// y (if given) receives the weighted sum as well (w may then be null)
static void net_forward(const NetState& st, const float* x, int n_pix, int M, const NetWs& w, bool save,
                        hipStream_t s, const float* fallback = nullptr, float* y = nullptr) {
  const size_t lds = fused_lds_bytes(M);
  if (save)
    hipLaunchKernelGGL(fused_forward_kernel<true>, dim3(fused_grid<true>(n_pix, lds)), dim3(kFwdThreads), lds, s, x, n_pix, M,
                       st.packed, st.params, w.w, fallback, y, w.a0, w.a1, w.a2, w.a3);
  else
    hipLaunchKernelGGL(fused_forward_kernel<false>, dim3(fused_grid<false>(n_pix, lds)), dim3(kFwdThreads), lds, s, x, n_pix, M,
                       st.packed, st.params, w.w, fallback, y, nullptr, nullptr, nullptr, nullptr);
}

static int check_net_args(int n_pix, int M) {
  USBF_REQUIRE(n_pix >= 1, USBF_EINVAL, "n_pix must be >= 1");
  USBF_REQUIRE(M >= 32 && M <= 256 && M % 32 == 0, USBF_EUNSUPPORTED, "n_el %d: must be a multiple of 32 in 32..256",
               M);
  return USBF_OK;
}

}  // namespace usbf

using namespace usbf;

extern "C" size_t usbf_apodnet_state_bytes(void) { return kStateBytes; }

extern "C" int32_t usbf_apodnet_num_params(void) { return kNParams; }

extern "C" int usbf_apodnet_init(void* state, const float* params, hipStream_t stream) {
  USBF_REQUIRE(state && params, USBF_EINVAL, "null state or params");
  NetState st = carve_state(state);
  if (hipMemcpyAsync(st.params, params, kNParams * sizeof(float), hipMemcpyDeviceToDevice, stream) != hipSuccess)
    return fail(USBF_EDEVICE, "copy of the initial parameters failed");
  if (hipMemsetAsync(st.m, 0, 2 * align256(kNParams * sizeof(float)) + 256, stream) != hipSuccess)
    return fail(USBF_EDEVICE, "clearing the optimiser state failed");
  hipLaunchKernelGGL(pack_kernel, dim3(64), dim3(256), 0, stream, st);
  return check_launch("pack_kernel");
}

extern "C" int usbf_apodnet_forward(const void* state, const float* x, int32_t n_pix, int32_t n_el, float* w,
                                    void* ws, size_t ws_bytes, hipStream_t stream) {
  USBF_REQUIRE(state && x && w, USBF_EINVAL, "null state, x or w");
  int st_ = check_net_args(n_pix, n_el);
  if (st_) return st_;
  (void)ws;  // the fused forward pass keeps its activations in LDS
  (void)ws_bytes;
  const NetState st = carve_state(const_cast<void*>(state));
  NetWs wsp{};
  wsp.w = w;  // the last layer writes the caller's buffer
  net_forward(st, x, n_pix, n_el, wsp, false, stream);
  return check_launch("apodnet forward");
}

extern "C" int usbf_apodnet_apply(const void* state, const float* x, int32_t n_pix, int32_t n_el,
                                  const float* y_fallback, float* w, float* y, hipStream_t stream) {
  USBF_REQUIRE(state && x && y, USBF_EINVAL, "null state, x or y");
  int st_ = check_net_args(n_pix, n_el);
  if (st_) return st_;
  const NetState st = carve_state(const_cast<void*>(state));
  NetWs wsp{};
  wsp.w = w;  // optional copy of the weights
  net_forward(st, x, n_pix, n_el, wsp, false, stream, y_fallback, y);
  return check_launch("apodnet apply");
}

extern "C" int usbf_apodnet_train_step(void* state, const float* x, const float* w_target, int32_t n_pix, int32_t n_el,
                                       float lr, float* loss, void* ws, size_t ws_bytes, hipStream_t stream) {
  USBF_REQUIRE(state && x && w_target, USBF_EINVAL, "null state, x or target");
  int st_ = check_net_args(n_pix, n_el);
  if (st_) return st_;
  USBF_REQUIRE(lr > 0.0f && lr < 1.0f, USBF_EINVAL, "learning rate must be in (0, 1)");
  const size_t need = net_ws_bytes(n_pix, n_el, true);
  USBF_REQUIRE(ws && ws_bytes >= need, USBF_EWORKSPACE, "apodnet training needs %zu workspace bytes", need);
  const NetState st = carve_state(state);
  NetWs w = carve_ws(ws, n_pix, n_el, true);
  const int M = n_el;
  net_forward(st, x, n_pix, M, w, true, stream);
  const int lb = std::min(kLossBlocks, (n_pix * M + 255) / 256);
  hipLaunchKernelGGL(loss_kernel, dim3(lb), dim3(kNetThreads), 0, stream, w.w, w_target, n_pix, M, w.g4, w.loss_part);
  if (loss)
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(64), 0, stream, w.loss_part, lb, 1.0f / (float(n_pix) * M), loss);
  // layer 4: weight gradient, then the data gradient into layer 3's outputs
  launch_wgrad<32, 1>(w.g4, w.a3, n_pix, M, w.part, w.grad, kW4, kB4, stream);
  launch_conv<1, 32, kMasked>(w.g4, n_pix, M, st.packed + kPkD4, nullptr, w.a3, w.g3, nullptr, stream);
  launch_wgrad<32, 32>(w.g3, w.a2, n_pix, M, w.part, w.grad, kW3, kB3, stream);
  launch_conv<32, 32, kMasked>(w.g3, n_pix, M, st.packed + kPkD3, nullptr, w.a2, w.g2, nullptr, stream);
  launch_wgrad<32, 32>(w.g2, w.a1, n_pix, M, w.part, w.grad, kW2, kB2, stream);
  launch_conv<32, 32, kMasked>(w.g2, n_pix, M, st.packed + kPkD2, nullptr, w.a1, w.g1, nullptr, stream);
  launch_wgrad<1, 32>(w.g1, w.a0, n_pix, M, w.part, w.grad, kW1, kB1, stream);
  hipLaunchKernelGGL(adam_kernel, dim3(42), dim3(256), 0, stream, st, w.grad, lr, 0.9f, 0.999f, 1e-8f);
  hipLaunchKernelGGL(step_kernel, dim3(1), dim3(64), 0, stream, st);
  hipLaunchKernelGGL(pack_kernel, dim3(64), dim3(256), 0, stream, st);
  return check_launch("apodnet train step");
}

extern "C" int usbf_apodnet_gradients(const void* state, const float* x, const float* w_target, int32_t n_pix,
                                      int32_t n_el, float* grad, void* ws, size_t ws_bytes, hipStream_t stream) {
  // the train step without the update: gradients of the loss for the current parameters
  USBF_REQUIRE(state && x && w_target && grad, USBF_EINVAL, "null argument");
  int st_ = check_net_args(n_pix, n_el);
  if (st_) return st_;
  const size_t need = net_ws_bytes(n_pix, n_el, true);
  USBF_REQUIRE(ws && ws_bytes >= need, USBF_EWORKSPACE, "apodnet gradients need %zu workspace bytes", need);
  const NetState st = carve_state(const_cast<void*>(state));
  NetWs w = carve_ws(ws, n_pix, n_el, true);
  const int M = n_el;
  net_forward(st, x, n_pix, M, w, true, stream);
  const int lb = std::min(kLossBlocks, (n_pix * M + 255) / 256);
  hipLaunchKernelGGL(loss_kernel, dim3(lb), dim3(kNetThreads), 0, stream, w.w, w_target, n_pix, M, w.g4, w.loss_part);
  launch_wgrad<32, 1>(w.g4, w.a3, n_pix, M, w.part, grad, kW4, kB4, stream);
  launch_conv<1, 32, kMasked>(w.g4, n_pix, M, st.packed + kPkD4, nullptr, w.a3, w.g3, nullptr, stream);
  launch_wgrad<32, 32>(w.g3, w.a2, n_pix, M, w.part, grad, kW3, kB3, stream);
  launch_conv<32, 32, kMasked>(w.g3, n_pix, M, st.packed + kPkD3, nullptr, w.a2, w.g2, nullptr, stream);
  launch_wgrad<32, 32>(w.g2, w.a1, n_pix, M, w.part, grad, kW2, kB2, stream);
  launch_conv<32, 32, kMasked>(w.g2, n_pix, M, st.packed + kPkD2, nullptr, w.a1, w.g1, nullptr, stream);
  launch_wgrad<1, 32>(w.g1, w.a0, n_pix, M, w.part, grad, kW1, kB1, stream);
  return check_launch("apodnet gradients");
}

extern "C" int usbf_beamform_weighted(const float* x, const float* w, const float* y_fallback, int32_t n_pix,
                                      int32_t n_el, float* y, hipStream_t stream) {
  USBF_REQUIRE(x && w && y, USBF_EINVAL, "null x, w or y");
  USBF_REQUIRE(n_pix >= 1 && n_el >= 1, USBF_EINVAL, "empty input");
  hipLaunchKernelGGL(weighted_kernel, dim3((n_pix + 3) / 4), dim3(256), 0, stream, x, w, y_fallback, n_pix, n_el, y);
  return check_launch("weighted_kernel");
}
