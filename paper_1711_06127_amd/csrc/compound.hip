// Coherent compounding of beamformed lines over transmits (plane-wave imaging: every line is
// beamformed once per steered plane wave, and the results are averaged before detection), and
// its general form, a weighted combination of beams per output line (overlapping multi-line
// layouts, where a line between two transmits is interpolated from both transmits' beams).
#include "common.h"

namespace usbf {

// out[f][i] = (1 / n_groups) sum_g in[f][g][i], summed in group order
__global__ __launch_bounds__(256) void compound_kernel(const float* __restrict__ in, int n_groups, int64_t group_len,
                                                      float* __restrict__ out) {
  const float inv = 1.0f / float(n_groups);
  const float* src = in + int64_t(blockIdx.y) * n_groups * group_len;
  float* dst = out + int64_t(blockIdx.y) * group_len;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < group_len;
       i += int64_t(gridDim.x) * blockDim.x) {
    float s = 0.0f;
    for (int g = 0; g < n_groups; ++g) s += src[g * group_len + i];
    dst[i] = s * inv;
  }
}

// out[f][o][i] = sum_k w[o][k] in[f][src[o][k]][i] over the k whose source is a line of the
// input, summed in k order.  Grid: (depth blocks, output lines, frames).
__global__ __launch_bounds__(256) void combine_kernel(const float* __restrict__ in, int n_in, int64_t len,
                                                     const int32_t* __restrict__ src, const float* __restrict__ w,
                                                     int K, float* __restrict__ out) {
  const int o = blockIdx.y;
  const float* fin = in + int64_t(blockIdx.z) * n_in * len;
  float* dst = out + (int64_t(blockIdx.z) * gridDim.y + o) * len;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < len; i += int64_t(gridDim.x) * blockDim.x) {
    float s = 0.0f;
    for (int k = 0; k < K; ++k) {
      const int sl = src[o * K + k];
      if (sl >= 0 && sl < n_in) s = __builtin_fmaf(w[o * K + k], fin[int64_t(sl) * len + i], s);
    }
    dst[i] = s;
  }
}

}  // namespace usbf

using namespace usbf;

extern "C" int usbf_compound(const float* in, int32_t n_frames, int32_t n_groups, int64_t group_len, float* out,
                             hipStream_t stream) {
  USBF_REQUIRE(in && out, USBF_EINVAL, "null in or out");
  USBF_REQUIRE(n_frames >= 1 && n_frames <= 65535 && n_groups >= 1 && group_len >= 1, USBF_EINVAL, "empty input");
  const int64_t total = int64_t(n_frames) * n_groups * group_len;
  const int64_t out_len = int64_t(n_frames) * group_len;
  USBF_REQUIRE(out + out_len <= in || out >= in + total, USBF_EINVAL, "out overlaps the input");
  const int64_t blocks = std::min<int64_t>((group_len + 255) / 256, 4096);
  hipLaunchKernelGGL(compound_kernel, dim3(unsigned(blocks), unsigned(n_frames)), dim3(256), 0, stream, in, n_groups,
                     group_len, out);
  return check_launch("compound_kernel");
}

extern "C" int usbf_combine_lines(const float* in, int32_t n_frames, int32_t n_in, int64_t len, const int32_t* src,
                                  const float* w, int32_t k, int32_t n_out, float* out, hipStream_t stream) {
  USBF_REQUIRE(in && out && src && w, USBF_EINVAL, "null in, out, src or w");
  USBF_REQUIRE(n_frames >= 1 && n_frames <= 65535, USBF_EINVAL, "n_frames %d outside 1..65535", n_frames);
  USBF_REQUIRE(n_in >= 1 && len >= 1, USBF_EINVAL, "empty input");
  USBF_REQUIRE(n_out >= 1 && n_out <= 65535, USBF_EINVAL, "n_out %d outside 1..65535", n_out);
  USBF_REQUIRE(k >= 1 && k <= 64, USBF_EUNSUPPORTED, "k %d outside 1..64", k);
  const int64_t total = int64_t(n_frames) * n_in * len;
  const int64_t out_len = int64_t(n_frames) * n_out * len;
  USBF_REQUIRE(out + out_len <= in || out >= in + total, USBF_EINVAL, "out overlaps the input");
  const int64_t blocks = std::min<int64_t>((len + 255) / 256, 1024);
  hipLaunchKernelGGL(combine_kernel, dim3(unsigned(blocks), unsigned(n_out), unsigned(n_frames)), dim3(256), 0, stream,
                     in, n_in, len, src, w, int(k), out);
  return check_launch("combine_kernel");
}
