// Receive beamforming by delay and sum (Sec. 1 pipeline list, "receive beamforming";
// Sec. 2 method list items 1-2) and the exported delay-index map.
//
// Work decomposition: one workgroup per (line, run of 256 depth samples); one lane per
// output sample.  The per-(line, element) receive constants are staged once in LDS; every
// lane evaluates the binary32 delay rule of its (pixel, element) pairs once and reuses the
// tap for a block of FB frames, so the delay arithmetic is amortised over the batch while
// each int16 channel sample is fetched once per frame.
#include "common.h"
#include "tof.h"

namespace usbf {

constexpr int kDasThreads = 256;

template <int FB>
__global__ __launch_bounds__(kDasThreads) void das_gather_kernel(const int16_t* __restrict__ rf, int n_frames,
                                                                 DasArgs a, float* __restrict__ out) {
  extern __shared__ float4 s_el[];  // (A, B, dx, dy) per element for this workgroup's line
  const int l = blockIdx.y;
  const int j = blockIdx.x * kDasThreads + threadIdx.x;
  LineGeom L;
  line_geom(a, l, L);
  for (int e = threadIdx.x; e < a.n_el; e += kDasThreads) {
    ElemGeom E = elem_geom(a, L, e);
    s_el[e] = make_float4(E.A, E.B, E.dx, E.dy);
  }
  __syncthreads();
  if (j >= a.n_depth) return;

  const size_t line_stride = size_t(a.n_depth);
  const size_t frame_out = size_t(a.n_lines) * line_stride;
  float* o = out + size_t(l) * line_stride + j;
  if (L.tx < 0) {
    for (int f = 0; f < n_frames; ++f) o[f * frame_out] = 0.0f;
    return;
  }
  const int32_t b = a.depth_start + a.depth_step * j;
  const float r = (float)b * a.h;
  const float r2 = r + r;
  const float rr = r * r;
  const float dtx = small_tx_delay(L, r);
  const float inv_w = r > 0.0f ? a.f_number / r : 0.0f;
  const int S = a.n_samples;
  const size_t frame_stride = size_t(a.n_tx) * a.n_el * S;
  const int16_t* trace0 = rf + size_t(L.tx) * a.n_el * S;

  for (int f0 = 0; f0 < n_frames; f0 += FB) {
    float acc[FB];
#pragma unroll
    for (int f = 0; f < FB; ++f) acc[f] = 0.0f;
    float den = 0.0f;
    const int nf = min(FB, n_frames - f0);
    const int16_t* tr = trace0 + size_t(f0) * frame_stride;
    for (int e = 0; e < a.n_el; ++e) {
      const float4 c = s_el[e];
      ElemGeom E{c.x, c.y, c.z, c.w};
      if (!in_aperture(a, E, r)) continue;
      const float w = apod_weight(a.window, a.array_dims, E.dx, E.dy, inv_w);
      den += w;
      const float drx = small_rx_delay(E.A, E.B, r, r2, rr);
      const Tap t = delay_tap(a, b, dtx, drx);
      if (t.i0 < 0 || t.i0 > S - 2) continue;
      const float w1 = w * t.phi;
      const float w0 = w - w1;
      const int16_t* p = tr + size_t(e) * S + t.i0;
#pragma unroll
      for (int f = 0; f < FB; ++f) {
        if (f < nf) {
          const int16_t* q = p + f * frame_stride;
          acc[f] = __builtin_fmaf(w0, (float)q[0], __builtin_fmaf(w1, (float)q[1], acc[f]));
        }
      }
    }
    const float inv = den > 0.0f ? 1.0f / den : 0.0f;
#pragma unroll
    for (int f = 0; f < FB; ++f)
      if (f < nf) o[size_t(f0 + f) * frame_out] = acc[f] * inv;
  }
}

__global__ void delay_index_kernel(DasArgs a, int32_t* __restrict__ i0, uint8_t* __restrict__ flags,
                                   float* __restrict__ phi) {
  const int64_t n = int64_t(a.n_lines) * a.n_depth * a.n_el;
  for (int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; idx < n;
       idx += int64_t(gridDim.x) * blockDim.x) {
    const int e = int(idx % a.n_el);
    const int64_t p = idx / a.n_el;
    const int j = int(p % a.n_depth);
    const int l = int(p / a.n_depth);
    LineGeom L;
    line_geom(a, l, L);
    const int32_t b = a.depth_start + a.depth_step * j;
    const float r = (float)b * a.h;
    const float r2 = r + r;
    const float rr = r * r;
    const float dtx = small_tx_delay(L, r);
    ElemGeom E = elem_geom(a, L, e);
    const float drx = small_rx_delay(E.A, E.B, r, r2, rr);
    const Tap t = delay_tap(a, b, dtx, drx);
    const bool act = in_aperture(a, E, r);
    const bool val = t.i0 >= 0 && t.i0 <= a.n_samples - 2;
    i0[idx] = t.i0;
    flags[idx] = uint8_t((act ? 1 : 0) | (val ? 2 : 0));
    if (phi) phi[idx] = t.phi;
  }
}

template <int FB>
static void launch_das(const int16_t* rf, int n_frames, const DasArgs& a, float* out, hipStream_t s) {
  dim3 grid((a.n_depth + kDasThreads - 1) / kDasThreads, a.n_lines);
  size_t lds = size_t(a.n_el) * sizeof(float4);
  hipLaunchKernelGGL(das_gather_kernel<FB>, grid, dim3(kDasThreads), lds, s, rf, n_frames, a, out);
}

int beamform_enqueue(const int16_t* rf, int32_t n_frames, const DasArgs& a, float* out, hipStream_t s) {
  if (n_frames >= 32)
    launch_das<32>(rf, n_frames, a, out, s);
  else if (n_frames >= 16)
    launch_das<16>(rf, n_frames, a, out, s);
  else if (n_frames >= 8)
    launch_das<8>(rf, n_frames, a, out, s);
  else if (n_frames >= 4)
    launch_das<4>(rf, n_frames, a, out, s);
  else if (n_frames >= 2)
    launch_das<2>(rf, n_frames, a, out, s);
  else
    launch_das<1>(rf, n_frames, a, out, s);
  return check_launch("das_gather_kernel");
}

}  // namespace usbf

using namespace usbf;

extern "C" int usbf_beamform(const int16_t* rf, int32_t n_frames, const usbf_geometry* geom, const usbf_rx* rx,
                             float* out, hipStream_t stream) {
  DasArgs a;
  int st = make_das_args(geom, rx, &a);
  if (st) return st;
  USBF_REQUIRE(rf && out, USBF_EINVAL, "null rf or out");
  USBF_REQUIRE(n_frames >= 1 && n_frames <= USBF_MAX_FRAMES, USBF_EINVAL, "n_frames %d out of range", n_frames);
  return beamform_enqueue(rf, n_frames, a, out, stream);
}

extern "C" int usbf_delay_index_map(const usbf_geometry* geom, const usbf_rx* rx, int32_t* i0, uint8_t* flags,
                                    float* phi, hipStream_t stream) {
  DasArgs a;
  int st = make_das_args(geom, rx, &a);
  if (st) return st;
  USBF_REQUIRE(i0 && flags, USBF_EINVAL, "null i0 or flags");
  const int64_t n = int64_t(a.n_lines) * a.n_depth * a.n_el;
  USBF_REQUIRE(n < (int64_t(1) << 31), USBF_EUNSUPPORTED, "index map larger than 2^31 entries");
  int blocks = int(std::min<int64_t>((n + 255) / 256, 65536));
  hipLaunchKernelGGL(delay_index_kernel, dim3(blocks), dim3(256), 0, stream, a, i0, flags, phi);
  return check_launch("delay_index_kernel");
}
