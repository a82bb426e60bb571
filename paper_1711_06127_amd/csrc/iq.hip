// Envelope by IQ demodulation with frequency compounding (Sec. 2 method list item 3: the
// paper's own envelope node).  Mixing band k down to baseband and low-passing with the
// prototype h is, up to a phase factor of unit magnitude, the complex band-pass
//   z_k[n] = sum_m g_k[m] y[n + c - m],   g_k[m] = h[m] exp(2 pi i f_k (m - c) / fs),
// so env[n] = (2 / K) sum_k |z_k[n]|.  h is the Hamming-windowed sinc with cutoff
// bandwidth / 2 and unit gain at DC, c = (L - 1) / 2, zeros outside the row.
//
// One workgroup per row at a time (grid-stride over rows): the taps are built once per
// workgroup in LDS, the row is staged in LDS with c zeros on either side, and every lane
// computes R consecutive outputs.  h is even, so g_k[c - d] = conj(g_k[c + d]) and
//   z_k[n] = h[c] y[n] + sum_{d=1..c} ( Re g_k[c+d] (y[n-d] + y[n+d]) + i Im g_k[c+d] (y[n-d] - y[n+d]) ),
// whose sum and difference are shared by all K bands; two register windows slide outwards
// from the output, one LDS read each per tap pair.  Bound by the arithmetic, K (L + 1) + L - 1
// operations per output sample.
#include "common.h"

namespace usbf {

constexpr int kIqThreads = 256;
constexpr int kIqOut = 8;           // outputs per lane and pass
constexpr int kIqMaxBands = 4;
constexpr int kIqMaxTaps = 127;
constexpr int kIqMaxLength = 8192;

struct IqArgs {
  int n, L, c, K;
  float fs, bw;
  float f[kIqMaxBands];
};

template <int K>
__global__ __launch_bounds__(kIqThreads) void envelope_iq_kernel(const float* __restrict__ in, int64_t n_rows, IqArgs a,
                                                                 float* __restrict__ env, float* __restrict__ row_max) {
  extern __shared__ __align__(16) float sm[];
  float* gre = sm;                        // [K][c + 1]: Re g_k[c + d]
  float* gim = gre + K * kIqMaxTaps;      // [K][c + 1]: Im g_k[c + d]
  float* row = gim + K * kIqMaxTaps;      // [n + 2c + kIqOut]
  __shared__ float red[kIqThreads / 64];
  const int tid = threadIdx.x;
  const int L = a.L, c = a.c, n = a.n;

  // ---- taps: prototype, its DC gain, then the K modulated copies for d = 0 .. c
  const float fc2 = a.bw / a.fs;  // 2 * cutoff in cycles per sample
  float hm = 0.0f;
  if (tid < L) {
    const int d = tid <= c ? c - tid : tid - c;  // the window is even: use |m - c|
    const float x = float(d);
    const float s = (d == 0) ? fc2 : sinpif(fc2 * x) / (3.14159265358979323846f * x);
    const float w = 0.54f + 0.46f * cospif(x / float(c));  // 0.54 - 0.46 cos(2 pi m / (L - 1))
    hm = s * w;
  }
  float sum = hm;
  for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
  if ((tid & 63) == 0) red[tid >> 6] = sum;
  __syncthreads();
  const float dc = red[0] + red[1];  // L <= 127 < 128: the first two waves hold every tap
  if (tid >= c && tid < L) {
    const int d = tid - c;
    const float h = hm / dc;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      float sn, cs;
      sincospif(2.0f * a.f[k] * float(d) / a.fs, &sn, &cs);
      gre[k * kIqMaxTaps + d] = h * cs;
      gim[k * kIqMaxTaps + d] = h * sn;
    }
  }
  const int padded = n + 2 * c + kIqOut;
  for (int64_t r = blockIdx.x; r < n_rows; r += gridDim.x) {
    __syncthreads();  // taps ready; the previous row is done with `row` and `red`
    const float* y = in + r * n;
    for (int i = tid; i < padded; i += kIqThreads) row[i] = (i >= c && i < c + n) ? y[i - c] : 0.0f;
    __syncthreads();
    float mx = 0.0f;
    for (int n0 = tid * kIqOut; n0 < n; n0 += kIqThreads * kIqOut) {
      // y[t] sits at row[t + c]; output n0 + i needs y[n0 + i - d] and y[n0 + i + d]
      float re[K][kIqOut], im[K][kIqOut];
      float vl[kIqOut], vr[kIqOut];
#pragma unroll
      for (int i = 0; i < kIqOut; ++i) vl[i] = vr[i] = row[n0 + c + i];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const float g0 = gre[k * kIqMaxTaps];
#pragma unroll
        for (int i = 0; i < kIqOut; ++i) {
          re[k][i] = g0 * vl[i];
          im[k][i] = 0.0f;
        }
      }
      for (int d = 1; d <= c; ++d) {
        // slide: vl[i] = y[n0 + i - d] (leftwards), vr[i] = y[n0 + i + d] (rightwards)
#pragma unroll
        for (int i = kIqOut - 1; i > 0; --i) vl[i] = vl[i - 1];
        vl[0] = row[n0 + c - d];  // index >= n0 >= 0
#pragma unroll
        for (int i = 0; i < kIqOut - 1; ++i) vr[i] = vr[i + 1];
        vr[kIqOut - 1] = row[n0 + c + kIqOut - 1 + d];  // index < n + 2c + kIqOut
        float sp[kIqOut], sm_[kIqOut];
#pragma unroll
        for (int i = 0; i < kIqOut; ++i) {
          sp[i] = vl[i] + vr[i];
          sm_[i] = vl[i] - vr[i];
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const float gr = gre[k * kIqMaxTaps + d], gi = gim[k * kIqMaxTaps + d];
#pragma unroll
          for (int i = 0; i < kIqOut; ++i) {
            re[k][i] = __builtin_fmaf(gr, sp[i], re[k][i]);
            im[k][i] = __builtin_fmaf(gi, sm_[i], im[k][i]);
          }
        }
      }
      float* e = env + r * n;
#pragma unroll
      for (int i = 0; i < kIqOut; ++i) {
        float s = 0.0f;
#pragma unroll
        // hardware square root (within 1 ulp): the band magnitudes are values, compared to 1e-4
        for (int k = 0; k < K; ++k) s += __builtin_amdgcn_sqrtf(__builtin_fmaf(re[k][i], re[k][i], im[k][i] * im[k][i]));
        const float val = s * (2.0f / float(K));
        if (n0 + i < n) {
          e[n0 + i] = val;
          mx = fmaxf(mx, val);
        }
      }
    }
    if (row_max) {
      for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
      if ((tid & 63) == 0) red[tid >> 6] = mx;
      __syncthreads();
      if (tid == 0) row_max[r] = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    }
  }
}

}  // namespace usbf

using namespace usbf;

extern "C" int usbf_envelope_iq(const float* in, int64_t n_rows, int32_t n, float fs, const float* freqs,
                                int32_t n_bands, float bandwidth, int32_t n_taps, float* env, float* row_max,
                                hipStream_t stream) {
  USBF_REQUIRE(in && env && freqs, USBF_EINVAL, "null in, env or freqs");
  USBF_REQUIRE(in != env, USBF_EINVAL, "the IQ envelope cannot run in place");
  USBF_REQUIRE(n_rows >= 1, USBF_EINVAL, "n_rows must be >= 1");
  USBF_REQUIRE(n >= 8 && n <= kIqMaxLength, USBF_EUNSUPPORTED, "row length %d outside 8..%d", n, kIqMaxLength);
  USBF_REQUIRE(finite_pos(fs), USBF_EINVAL, "fs must be finite and > 0");
  USBF_REQUIRE(n_bands >= 1 && n_bands <= kIqMaxBands, USBF_EUNSUPPORTED, "n_bands %d outside 1..%d", n_bands,
               kIqMaxBands);
  USBF_REQUIRE(n_taps >= 3 && n_taps <= kIqMaxTaps && n_taps % 2 == 1, USBF_EUNSUPPORTED,
               "n_taps %d: must be odd in 3..%d", n_taps, kIqMaxTaps);
  USBF_REQUIRE(finite_pos(bandwidth) && bandwidth <= fs, USBF_EINVAL, "bandwidth must be in (0, fs]");
  IqArgs a{};
  a.n = n;
  a.L = n_taps;
  a.c = (n_taps - 1) / 2;
  a.K = n_bands;
  a.fs = fs;
  a.bw = bandwidth;
  for (int k = 0; k < n_bands; ++k) {
    USBF_REQUIRE(freqs[k] > 0.0f && freqs[k] < 0.5f * fs, USBF_EINVAL, "band %d: frequency outside (0, fs/2)", k);
    a.f[k] = freqs[k];
  }
  int dev = 0, n_cu = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  const size_t lds = (size_t(2) * kIqMaxBands * kIqMaxTaps + n + 2 * a.c + kIqOut) * sizeof(float);
  const int per_cu = std::max(1, std::min(8, int(163840 / (lds + 64))));
  const unsigned blocks = unsigned(std::min<int64_t>(n_rows, int64_t(n_cu) * per_cu));
  switch (n_bands) {
    case 1: hipLaunchKernelGGL(envelope_iq_kernel<1>, dim3(blocks), dim3(kIqThreads), lds, stream, in, n_rows, a, env, row_max); break;
    case 2: hipLaunchKernelGGL(envelope_iq_kernel<2>, dim3(blocks), dim3(kIqThreads), lds, stream, in, n_rows, a, env, row_max); break;
    case 3: hipLaunchKernelGGL(envelope_iq_kernel<3>, dim3(blocks), dim3(kIqThreads), lds, stream, in, n_rows, a, env, row_max); break;
    default: hipLaunchKernelGGL(envelope_iq_kernel<4>, dim3(blocks), dim3(kIqThreads), lds, stream, in, n_rows, a, env, row_max); break;
  }
  return check_launch("envelope_iq_kernel");
}
