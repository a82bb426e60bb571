// Coherent compounding of beamformed lines over transmits (plane-wave imaging: every line is
// beamformed once per steered plane wave, and the results are averaged before detection).
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
