// Delayed channel samples (delay-gather) and minimum-variance (Capon) apodization weights.
//
// Delay-gather: for each listed pixel, every element's channel sample interpolated at the
// two-way travel time of the binary32 delay rule (the beamformer's taps, without weights or
// summation); 0 outside the record.
//
// Minimum variance: spatially smoothed covariance of the delayed samples over subapertures of
// L elements (binary32, from lag sums updated along the aperture), diagonal loading
// eps = loading * trace / L, then the Cholesky factorisation and the two triangular solves of
// (R + eps I) v = 1 in binary64 -- the only binary64 arithmetic in the library -- and
// w = v / 1^T v expanded onto the full aperture.  Thirty-two lanes own one pixel: lane i holds
// row i of the matrix during the factorisation.
#include "common.h"
#include "tof.h"

namespace usbf {

constexpr int kGatherPix = 64;     // pixels per workgroup
constexpr int kGatherChunk = 128;  // elements per LDS transpose chunk

// Output row q = p * n_avg + t holds listed pixel p's samples at depth j_p + t - n_avg / 2,
// clamped to the line (n_avg = 1: the pixel itself).
__global__ __launch_bounds__(256) void gather_kernel(const int16_t* __restrict__ rf, int n_frames, DasArgs a,
                                                     const int32_t* __restrict__ pix, int n_pix, int n_avg,
                                                     float* __restrict__ x) {
  __shared__ float tile[kGatherPix][kGatherChunk + 1];
  const int pl = threadIdx.x % kGatherPix;
  const int eg = threadIdx.x / kGatherPix;  // 4 element lanes per pixel
  const int64_t n_rows = int64_t(n_pix) * n_avg;
  const int64_t q = int64_t(blockIdx.x) * kGatherPix + pl;
  int f = 0, l = 0, j = 0;
  bool ok = q < n_rows;
  if (ok) {
    const int64_t p = q / n_avg;
    const int t = int(q - p * n_avg);
    f = pix[3 * p];
    l = pix[3 * p + 1];
    j = pix[3 * p + 2];
    ok = f >= 0 && f < n_frames && l >= 0 && l < a.n_lines && j >= 0 && j < a.n_depth;
    j = min(max(j + t - n_avg / 2, 0), a.n_depth - 1);
  }
  LineGeom L;
  line_geom(a, ok ? l : 0, L);
  ok = ok && L.tx >= 0;
  const int32_t b = a.depth_start + a.depth_step * j;
  const float r = (float)b * a.h;
  const float r2 = r + r, rr = r * r;
  const float dtx = small_tx_delay(L, r);
  const int S = a.n_samples;
  const int16_t* tr = rf + ((size_t(ok ? f : 0) * a.n_tx + (ok ? L.tx : 0)) * a.n_el) * S;
  for (int c0 = 0; c0 < a.n_el; c0 += kGatherChunk) {
    const int nc = min(kGatherChunk, a.n_el - c0);
    for (int k = eg; k < nc; k += 4) {
      const int e = c0 + k;
      float v = 0.0f;
      if (ok) {
        const ElemGeom E = elem_geom(a, L, e);
        const Tap t = fast_tap(a, b, dtx, E.A, E.B, r, r2, rr);
        if (t.i0 >= 0 && t.i0 <= S - 2) {
          const int16_t* q = tr + size_t(e) * S + t.i0;
          const float s0 = float(q[0]), s1 = float(q[1]);
          v = __builtin_fmaf(t.phi, s1 - s0, s0);
        }
      }
      tile[pl][k] = v;
    }
    __syncthreads();
    // coalesced write-out: consecutive lanes write consecutive elements of one pixel row
    for (int idx = threadIdx.x; idx < kGatherPix * nc; idx += 256) {
      const int pp = idx / nc, k = idx - pp * nc;
      const int64_t qg = int64_t(blockIdx.x) * kGatherPix + pp;
      if (qg < n_rows) x[size_t(qg) * a.n_el + c0 + k] = tile[pp][k];
    }
    __syncthreads();
  }
}

constexpr int kMvL = 32;            // subaperture length handled by the kernel
constexpr int kMvMaxEl = 256;       // elements per pixel the kernel supports
constexpr int kMvPixPerBlock = 2;   // one wave: two pixels of 32 lanes

struct MvLds {
  float x[kMvMaxEl];
  float R[kMvL][kMvL + 1];
  double Lm[kMvL][kMvL + 1];
  double pre[kMvMaxEl + 1];
};

__device__ inline double shfl32(double v, int src) {
  // broadcast within the lane's 32-lane half of the wave
  return __shfl(v, src, 32);
}

// x: [n_pix][T][M]; the covariance averages the T rows (neighbouring depths), the weights
// apply to row T / 2 (the pixel's own samples).  AVG = false: T = 1, plain spatial smoothing
// (the same arithmetic without the row loop).
template <bool AVG>
__global__ __launch_bounds__(64) void mv_kernel(const float* __restrict__ xin, int n_pix, int T, int M, float loading,
                                                float* __restrict__ w_full, float* __restrict__ y) {
  __shared__ MvLds lds[kMvPixPerBlock];
  const int half = threadIdx.x / kMvL;
  const int i = threadIdx.x % kMvL;  // lane within the pixel's group: row i / lag i
  const int p = blockIdx.x * kMvPixPerBlock + half;
  const bool ok = p < n_pix;
  MvLds& s = lds[half];
  const int K = M - kMvL + 1;
  const float* xp = xin + size_t(ok ? p : 0) * T * M;

  // spatially smoothed covariance of each row: lane d sweeps the d-th diagonal,
  // S_d(a) = sum_{k=a}^{a+K-1} x[k] x[k+d], summed over the rows into R[a][a+d] = R[a+d][a],
  // then divided by T K
  if constexpr (!AVG) {
    for (int e = i; e < M; e += kMvL) s.x[e] = ok ? xp[e] : 0.0f;
    __syncthreads();
    const int d = i;
    float S = 0.0f;
    for (int k = 0; k < K; ++k) S = __builtin_fmaf(s.x[k], s.x[k + d], S);
    const float invK = 1.0f / float(K);
    for (int a0 = 0; a0 + d < kMvL; ++a0) {
      const float v = S * invK;
      s.R[a0][a0 + d] = v;
      s.R[a0 + d][a0] = v;
      if (a0 + d + 1 < kMvL)
        S = __builtin_fmaf(s.x[a0 + K], s.x[a0 + K + d], __builtin_fmaf(-s.x[a0], s.x[a0 + d], S));
    }
  } else {
    for (int a0 = 0; a0 + i < kMvL; ++a0) s.R[a0][a0 + i] = 0.0f;
    for (int t = 0; t < T; ++t) {
      __syncthreads();  // the previous row's sweep is done with s.x
      for (int e = i; e < M; e += kMvL) s.x[e] = ok ? xp[size_t(t) * M + e] : 0.0f;
      __syncthreads();
      const int d = i;
      float S = 0.0f;
      for (int k = 0; k < K; ++k) S = __builtin_fmaf(s.x[k], s.x[k + d], S);
      for (int a0 = 0; a0 + d < kMvL; ++a0) {
        s.R[a0][a0 + d] += S;
        if (a0 + d + 1 < kMvL)
          S = __builtin_fmaf(s.x[a0 + K], s.x[a0 + K + d], __builtin_fmaf(-s.x[a0], s.x[a0 + d], S));
      }
    }
    {
      const float inv = 1.0f / (float(K) * float(T));
      for (int a0 = 0; a0 + i < kMvL; ++a0) {
        const float v = s.R[a0][a0 + i] * inv;
        s.R[a0][a0 + i] = v;
        s.R[a0 + i][a0] = v;
      }
    }
    // the pixel's own samples for the output
    if (T > 1) {
      __syncthreads();
      for (int e = i; e < M; e += kMvL) s.x[e] = ok ? xp[size_t(T / 2) * M + e] : 0.0f;
    }
  }
  __syncthreads();

  // row i of A = R + eps I in binary64
  double arow[kMvL];
#pragma unroll
  for (int j = 0; j < kMvL; ++j) arow[j] = double(s.R[i][j]);
  double tr = double(s.R[i][i]);
#pragma unroll
  for (int off = 16; off > 0; off >>= 1) tr += __shfl_xor(tr, off, 32);
  // all-zero data (trace 0): eps = 1 makes A = I and the weights uniform
  const double eps = tr > 0.0 ? double(loading) * tr / double(kMvL) : 1.0;
#pragma unroll
  for (int j = 0; j < kMvL; ++j) arow[j] += (j == i) ? eps : 0.0;

  // Cholesky, right-looking: after step k, arow[k] holds L[i][k]
#pragma unroll
  for (int k = 0; k < kMvL; ++k) {
    const double piv = shfl32(arow[k], k);
    const double dk = sqrt(piv);
    const double lik = (i == k) ? dk : arow[k] / dk;
    arow[k] = lik;
#pragma unroll
    for (int jj = k + 1; jj < kMvL; ++jj) {
      const double ljk = shfl32(lik, jj);
      arow[jj] = fma(-lik, ljk, arow[jj]);
    }
  }
#pragma unroll
  for (int j = 0; j < kMvL; ++j) s.Lm[i][j] = (j <= i) ? arow[j] : 0.0;
  __syncthreads();

  // L z = 1 (forward), then L^T v = z (backward); lane i owns z_i, v_i
  double z = 0.0, acc = 0.0;
  for (int k = 0; k < kMvL; ++k) {
    double zk = 0.0;
    if (i == k) zk = (1.0 - acc) / s.Lm[k][k];
    zk = shfl32(zk, k);
    if (i == k) z = zk;
    if (i > k) acc = fma(s.Lm[i][k], zk, acc);
  }
  double v = 0.0;
  acc = 0.0;
  for (int k = kMvL - 1; k >= 0; --k) {
    double vk = 0.0;
    if (i == k) vk = (z - acc) / s.Lm[k][k];
    vk = shfl32(vk, k);
    if (i == k) v = vk;
    if (i < k) acc = fma(s.Lm[k][i], vk, acc);
  }
  double sum = v;
#pragma unroll
  for (int off = 16; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 32);
  const double w = v / sum;

  // full-aperture weights: w_full[e] = (1/K) sum_{i = max(0, e-K+1)}^{min(L-1, e)} w[i]
  s.pre[i + 1] = w;  // prefix sums of w (serial over 32 values in one lane)
  __syncthreads();
  if (i == 0) {
    s.pre[0] = 0.0;
    for (int k = 1; k <= kMvL; ++k) s.pre[k] += s.pre[k - 1];
  }
  __syncthreads();
  double ysum = 0.0;
  for (int e = i; e < M; e += kMvL) {
    const int hi = min(kMvL - 1, e), lo = max(0, e - K + 1);
    const double wf = (s.pre[hi + 1] - s.pre[lo]) / double(K);
    if (ok && w_full) w_full[size_t(p) * M + e] = float(wf);
    ysum = fma(wf, double(s.x[e]), ysum);
  }
#pragma unroll
  for (int off = 16; off > 0; off >>= 1) ysum += __shfl_xor(ysum, off, 32);
  if (ok && y && i == 0) y[p] = float(ysum);
}

}  // namespace usbf

using namespace usbf;

static int gather_launch(const int16_t* rf, int32_t n_frames, const usbf_geometry* geom, const usbf_rx* rx,
                         const int32_t* pix, int32_t n_pix, int32_t n_avg, float* x, hipStream_t stream) {
  DasArgs a;
  int st = make_das_args(geom, rx, &a);
  if (st) return st;
  USBF_REQUIRE(rf && pix && x, USBF_EINVAL, "null rf, pix or x");
  USBF_REQUIRE(n_frames >= 1 && n_pix >= 1, USBF_EINVAL, "n_frames and n_pix must be >= 1");
  USBF_REQUIRE(n_avg >= 1 && n_avg <= 255 && n_avg % 2 == 1, USBF_EINVAL, "n_avg %d: must be odd in 1..255", n_avg);
  const int64_t blocks = (int64_t(n_pix) * n_avg + kGatherPix - 1) / kGatherPix;
  USBF_REQUIRE(blocks <= 0x7fffffff, USBF_EUNSUPPORTED, "too many gathered rows");
  hipLaunchKernelGGL(gather_kernel, dim3(unsigned(blocks)), dim3(256), 0, stream, rf, n_frames, a, pix, n_pix,
                     int(n_avg), x);
  return check_launch("gather_kernel");
}

extern "C" int usbf_delay_gather(const int16_t* rf, int32_t n_frames, const usbf_geometry* geom, const usbf_rx* rx,
                                 const int32_t* pix, int32_t n_pix, float* x, hipStream_t stream) {
  return gather_launch(rf, n_frames, geom, rx, pix, n_pix, 1, x, stream);
}

extern "C" int usbf_delay_gather_depths(const int16_t* rf, int32_t n_frames, const usbf_geometry* geom,
                                        const usbf_rx* rx, const int32_t* pix, int32_t n_pix, int32_t n_avg, float* x,
                                        hipStream_t stream) {
  return gather_launch(rf, n_frames, geom, rx, pix, n_pix, n_avg, x, stream);
}

static int mv_launch(const float* x, int32_t n_pix, int32_t n_avg, int32_t n_el, int32_t subap, float loading,
                     float* w_full, float* y, hipStream_t stream) {
  USBF_REQUIRE(x && (w_full || y), USBF_EINVAL, "null x, or neither w_full nor y requested");
  USBF_REQUIRE(n_pix >= 1, USBF_EINVAL, "n_pix must be >= 1");
  USBF_REQUIRE(n_avg >= 1 && n_avg <= 255 && n_avg % 2 == 1, USBF_EINVAL, "n_avg %d: must be odd in 1..255", n_avg);
  USBF_REQUIRE(subap == kMvL, USBF_EUNSUPPORTED, "subaperture %d: only %d is implemented", subap, kMvL);
  USBF_REQUIRE(n_el >= subap && n_el <= kMvMaxEl, USBF_EUNSUPPORTED, "n_el %d outside %d..%d", n_el, subap,
               kMvMaxEl);
  USBF_REQUIRE(loading > 0.0f && loading < 1e30f, USBF_EINVAL, "loading must be finite and > 0");
  const int blocks = (n_pix + kMvPixPerBlock - 1) / kMvPixPerBlock;
  if (n_avg == 1)
    hipLaunchKernelGGL(mv_kernel<false>, dim3(blocks), dim3(64), 0, stream, x, n_pix, 1, n_el, loading, w_full, y);
  else
    hipLaunchKernelGGL(mv_kernel<true>, dim3(blocks), dim3(64), 0, stream, x, n_pix, int(n_avg), n_el, loading, w_full,
                       y);
  return check_launch("mv_kernel");
}

extern "C" int usbf_mv_weights(const float* x, int32_t n_pix, int32_t n_el, int32_t subap, float loading,
                               float* w_full, float* y, hipStream_t stream) {
  return mv_launch(x, n_pix, 1, n_el, subap, loading, w_full, y, stream);
}

extern "C" int usbf_mv_weights_averaged(const float* x, int32_t n_pix, int32_t n_avg, int32_t n_el, int32_t subap,
                                        float loading, float* w_full, float* y, hipStream_t stream) {
  return mv_launch(x, n_pix, n_avg, n_el, subap, loading, w_full, y, stream);
}
