// Delayed channel samples (delay-gather) and minimum-variance (Capon) apodization weights.
//
// Delay-gather: for each listed pixel, every element's channel sample interpolated at the
// two-way travel time of the binary32 delay rule (the beamformer's taps, without weights or
// summation); 0 outside the record.  The same taps serve real (int16) channel data and its
// analytic signal (complex binary32).
//
// Minimum variance: spatially smoothed covariance of the delayed samples over subapertures of
// L = 32 elements (binary32, from lag sums slid along the aperture), diagonal loading
// eps = loading * trace / L, then the Cholesky factorisation and the two triangular solves of
// (R + eps I) v = 1 in binary64 -- the only binary64 arithmetic in the library -- and the
// normalisation w = v / 1^T v; the expansion of w onto the full aperture and the weighted
// sum are binary32.  The real estimator works on delayed RF, the complex one on the delayed
// analytic signal with the Hermitian covariance (R = (1/K) sum_l z_l z_l^H, A = C C^H).
//
// Layout: 32 lanes own one pixel (two pixels per wave, one wave per workgroup).  Lane d
// builds the d-th diagonal of the covariance; lane i then holds row i of the loaded matrix in
// registers during the right-looking factorisation, which broadcasts each new column through
// a 32-entry LDS buffer (one write per lane, broadcast reads); the factor is also written to
// LDS, packed row by row, for the back substitution, which needs it transposed.  LDS per
// pixel: the packed triangle (528 entries of binary64, aliasing the binary32 covariance) plus
// the samples, about 4.7 KB for 128 real elements.
#include <algorithm>
#include <type_traits>

#include "common.h"
#include "tof.h"

namespace usbf {

// ------------------------------------------------------------------ delay-gather

struct cf32 {
  float x, y;
};

constexpr int kGatherPix = 64;  // pixels per workgroup

// one delayed sample: int16 channel data (real) or its analytic signal (complex binary32)
__device__ inline float lerp_tap(const int16_t* q, float phi) {
  const float s0 = float(q[0]), s1 = float(q[1]);
  return __builtin_fmaf(phi, s1 - s0, s0);
}
__device__ inline cf32 lerp_tap(const cf32* q, float phi) {
  const cf32 a = q[0], b = q[1];
  return {__builtin_fmaf(phi, b.x - a.x, a.x), __builtin_fmaf(phi, b.y - a.y, a.y)};
}
template <typename T>
__device__ inline T zero_of();
template <>
__device__ inline float zero_of<float>() { return 0.0f; }
template <>
__device__ inline cf32 zero_of<cf32>() { return {0.0f, 0.0f}; }

// Output row q = p * n_avg + t holds listed pixel p's samples at depth j_p + t - n_avg / 2,
// clamped to the line (n_avg = 1: the pixel itself).  Src: int16_t (out float) or cf32
// (out cf32).  Rows are transposed through LDS in chunks of CHUNK elements so that the
// [pixel][element] output is written coalesced.
template <typename Src, typename Out, int CHUNK>
__global__ __launch_bounds__(256) void gather_kernel(const Src* __restrict__ rf, int n_frames, DasArgs a,
                                                     const int32_t* __restrict__ pix, int n_pix, int n_avg,
                                                     Out* __restrict__ x) {
  __shared__ Out tile[kGatherPix][CHUNK + 1];
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
  const Src* tr = rf + ((size_t(ok ? f : 0) * a.n_tx + (ok ? L.tx : 0)) * a.n_el) * S;
  for (int c0 = 0; c0 < a.n_el; c0 += CHUNK) {
    const int nc = min(CHUNK, a.n_el - c0);
    for (int k = eg; k < nc; k += 4) {
      const int e = c0 + k;
      Out v = zero_of<Out>();
      if (ok) {
        const ElemGeom E = elem_geom(a, L, e);
        const Tap t = fast_tap(a, b, dtx, E.A, E.B, r, r2, rr);
        if (t.i0 >= 0 && t.i0 <= S - 2) v = lerp_tap(tr + size_t(e) * S + t.i0, t.phi);
      }
      tile[pl][k] = v;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < kGatherPix * nc; idx += 256) {
      const int pp = idx / nc, k = idx - pp * nc;
      const int64_t qg = int64_t(blockIdx.x) * kGatherPix + pp;
      if (qg < n_rows) x[size_t(qg) * a.n_el + c0 + k] = tile[pp][k];
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ minimum variance

constexpr int kMvL = 32;         // subaperture length handled by the kernel
constexpr int kMvMaxEl = 256;    // elements per pixel the kernel supports
constexpr int kMvTri = kMvL * (kMvL + 1) / 2;  // entries of a packed triangle

struct cf64 {
  double x, y;
};

// Arithmetic of the two fields: binary32 samples (float / cf32) and binary64 factorisation
// (double / cf64).  conj() of a real number is the number.
__device__ inline float conj_(float a) { return a; }
__device__ inline cf32 conj_(cf32 a) { return {a.x, -a.y}; }
__device__ inline double conj_(double a) { return a; }
__device__ inline cf64 conj_(cf64 a) { return {a.x, -a.y}; }
__device__ inline float re_(float a) { return a; }
__device__ inline float re_(cf32 a) { return a.x; }
__device__ inline double re_(double a) { return a; }
__device__ inline double re_(cf64 a) { return a.x; }
__device__ inline float add_(float a, float b) { return a + b; }
__device__ inline cf32 add_(cf32 a, cf32 b) { return {a.x + b.x, a.y + b.y}; }
__device__ inline double add_(double a, double b) { return a + b; }
__device__ inline cf64 add_(cf64 a, cf64 b) { return {a.x + b.x, a.y + b.y}; }
__device__ inline float sub_(float a, float b) { return a - b; }
__device__ inline cf32 sub_(cf32 a, cf32 b) { return {a.x - b.x, a.y - b.y}; }
__device__ inline double sub_(double a, double b) { return a - b; }
__device__ inline cf64 sub_(cf64 a, cf64 b) { return {a.x - b.x, a.y - b.y}; }
__device__ inline float neg_(float a) { return -a; }
__device__ inline cf32 neg_(cf32 a) { return {-a.x, -a.y}; }
__device__ inline double neg_(double a) { return -a; }
__device__ inline cf64 neg_(cf64 a) { return {-a.x, -a.y}; }
__device__ inline float scale_(float a, float s) { return a * s; }
__device__ inline cf32 scale_(cf32 a, float s) { return {a.x * s, a.y * s}; }
__device__ inline double scale_(double a, double s) { return a * s; }
__device__ inline cf64 scale_(cf64 a, double s) { return {a.x * s, a.y * s}; }
// acc + a * conj(b)
__device__ inline float fma_conj(float a, float b, float acc) { return __builtin_fmaf(a, b, acc); }
__device__ inline cf32 fma_conj(cf32 a, cf32 b, cf32 acc) {
  return {__builtin_fmaf(a.x, b.x, __builtin_fmaf(a.y, b.y, acc.x)),
          __builtin_fmaf(a.y, b.x, __builtin_fmaf(-a.x, b.y, acc.y))};
}
__device__ inline double fma_conj(double a, double b, double acc) { return fma(a, b, acc); }
__device__ inline cf64 fma_conj(cf64 a, cf64 b, cf64 acc) {
  return {fma(a.x, b.x, fma(a.y, b.y, acc.x)), fma(a.y, b.x, fma(-a.x, b.y, acc.y))};
}
// acc + a * b
__device__ inline double fma_(double a, double b, double acc) { return fma(a, b, acc); }
__device__ inline cf64 fma_(cf64 a, cf64 b, cf64 acc) {
  return {fma(a.x, b.x, fma(-a.y, b.y, acc.x)), fma(a.x, b.y, fma(a.y, b.x, acc.y))};
}
__device__ inline double widen(float a) { return double(a); }
__device__ inline cf64 widen(cf32 a) { return {double(a.x), double(a.y)}; }
__device__ inline float narrow(double a) { return float(a); }
__device__ inline cf32 narrow(cf64 a) { return {float(a.x), float(a.y)}; }
// a / b
__device__ inline double div_(double a, double b) { return a / b; }
__device__ inline cf64 div_(cf64 a, cf64 b) {
  const double d = fma(b.x, b.x, b.y * b.y);
  return {fma(a.x, b.x, a.y * b.y) / d, fma(a.y, b.x, -a.x * b.y) / d};
}
// 1 / sqrt(a) for a > 0: the hardware estimate refined by two Newton steps,
// r <- r (3/2 - (a/2) r^2), each of which doubles the number of correct bits
__device__ inline double rsqrt_nr(double a) {
  double r = __builtin_amdgcn_rsq(a);
  const double h = 0.5 * a;
  r = r * fma(-h * r, r, 1.5);
  r = r * fma(-h * r, r, 1.5);
  return r;
}
// 32-lane shuffles (within the lane's half of the wave)
__device__ inline float shfl32(float v, int src) { return __shfl(v, src, 32); }
__device__ inline cf32 shfl32(cf32 v, int src) { return {__shfl(v.x, src, 32), __shfl(v.y, src, 32)}; }
__device__ inline double shfl32(double v, int src) { return __shfl(v, src, 32); }
__device__ inline cf64 shfl32(cf64 v, int src) { return {__shfl(v.x, src, 32), __shfl(v.y, src, 32)}; }
__device__ inline float shfl_up32(float v, int d) { return __shfl_up(v, d, 32); }
__device__ inline cf32 shfl_up32(cf32 v, int d) { return {__shfl_up(v.x, d, 32), __shfl_up(v.y, d, 32)}; }
template <typename T>
__device__ inline T sum32(T v) {
#pragma unroll
  for (int off = 16; off > 0; off >>= 1) {
    if constexpr (std::is_arithmetic<T>::value) {
      v = v + __shfl_xor(v, off, 32);
    } else {
      v.x = v.x + __shfl_xor(v.x, off, 32);
      v.y = v.y + __shfl_xor(v.y, off, 32);
    }
  }
  return v;
}

// offset of diagonal d in the packed upper triangle (diagonal d holds R[a][a + d], a < L - d)
__device__ __host__ constexpr int diag_off(int d) { return d * kMvL - d * (d - 1) / 2; }
// offset of row i in the packed lower triangle of the factor (row i holds C[i][0 .. i])
__device__ __host__ constexpr int row_off(int i) { return i * (i + 1) / 2; }

// LDS bytes one pixel uses: the packed triangle (binary64 factor, aliasing the binary32
// covariance) and the samples (aliased later by the column buffer and the prefix sums)
template <bool CPLX>
__host__ __device__ constexpr size_t mv_tri_bytes() {
  return (size_t(kMvTri) * (CPLX ? sizeof(cf64) : sizeof(double)) + 15) & ~size_t(15);
}
template <bool CPLX>
__host__ size_t mv_pixel_lds(int M) {
  using F = typename std::conditional<CPLX, cf32, float>::type;
  using D = typename std::conditional<CPLX, cf64, double>::type;
  const size_t tail = std::max({size_t(M) * sizeof(F), size_t(kMvL) * sizeof(D), size_t(kMvL + 1) * sizeof(F)});
  return mv_tri_bytes<CPLX>() + ((tail + 15) & ~size_t(15));
}

// x: [n_pix][T][M] (F = float, or cf32 for the analytic signal); the covariance averages the
// T rows (neighbouring depths), the weights apply to row T / 2 (the pixel's own samples).
// AVG = false: T = 1, plain spatial smoothing.  The weighted sum is y = w_full^H x.
template <bool CPLX, bool AVG>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(CPLX ? 2 : 4))) void mv_kernel(const void* __restrict__ xin_, int n_pix, int T, int M, float loading,
                                                void* __restrict__ w_full_, void* __restrict__ y_, size_t pix_lds) {
  using F = typename std::conditional<CPLX, cf32, float>::type;
  using D = typename std::conditional<CPLX, cf64, double>::type;
  const F* xin = static_cast<const F*>(xin_);
  F* w_full = static_cast<F*>(w_full_);
  F* y = static_cast<F*>(y_);
  extern __shared__ __align__(16) unsigned char mv_lds[];
  const int half = threadIdx.x / kMvL;
  const int i = threadIdx.x % kMvL;  // lane within the pixel's group: row i / diagonal i
  const int p = blockIdx.x * 2 + half;
  const bool ok = p < n_pix;
  unsigned char* base = mv_lds + half * pix_lds;
  F* Rp = reinterpret_cast<F*>(base);                   // packed covariance, diagonal-major
  D* Lp = reinterpret_cast<D*>(base);                   // packed factor, row-major (after Rp is read)
  F* xs = reinterpret_cast<F*>(base + mv_tri_bytes<CPLX>());  // samples of one row
  D* col = reinterpret_cast<D*>(base + mv_tri_bytes<CPLX>()); // one column of the factor
  F* pre = reinterpret_cast<F*>(base + mv_tri_bytes<CPLX>()); // prefix sums of w
  const int K = M - kMvL + 1;
  const F* xp = xin + size_t(ok ? p : 0) * T * M;

  // smoothed covariance: lane d sweeps the d-th diagonal,
  // S_d(a) = sum_{k=a}^{a+K-1} x[k] conj(x[k+d]) = K R[a][a+d], summed over the T rows
  const int d = i;
  F* Rd = Rp + diag_off(d);
  for (int t = 0; t < T; ++t) {
    if (t > 0) __syncthreads();  // the previous row's sweep is done with xs
    for (int e = i; e < M; e += kMvL) xs[e] = ok ? xp[size_t(t) * M + e] : zero_of<F>();
    __syncthreads();
    F S = zero_of<F>();
    for (int k = 0; k < K; ++k) S = fma_conj(xs[k], xs[k + d], S);
    const float invK = 1.0f / float(K);
    for (int a0 = 0; a0 + d < kMvL; ++a0) {
      if constexpr (AVG)
        Rd[a0] = (t == 0) ? S : add_(Rd[a0], S);
      else
        Rd[a0] = scale_(S, invK);
      if (a0 + d + 1 < kMvL)
        S = fma_conj(xs[a0 + K], xs[a0 + K + d], fma_conj(neg_(xs[a0]), xs[a0 + d], S));
    }
  }
  if constexpr (AVG) {
    const float inv = 1.0f / (float(K) * float(T));
    for (int a0 = 0; a0 + d < kMvL; ++a0) Rd[a0] = scale_(Rd[a0], inv);
  }
  __syncthreads();

  // row i of A = R + eps I in binary64 (R[i][j] = conj(R[j][i]) below the diagonal)
  D arow[kMvL];
#pragma unroll
  for (int j = 0; j < kMvL; ++j)
    arow[j] = widen(j >= i ? Rp[diag_off(j - i) + i] : conj_(Rp[diag_off(i - j) + j]));
  double dii = 0.0;
#pragma unroll
  for (int j = 0; j < kMvL; ++j) dii = (j == i) ? re_(arow[j]) : dii;
  const double tr = sum32(dii);
  // all-zero data (trace 0): eps = 1 makes A = I and the weights uniform
  const double eps = tr > 0.0 ? double(loading) * tr / double(kMvL) : 1.0;
#pragma unroll
  for (int j = 0; j < kMvL; ++j) {
    if (j == i) {
      if constexpr (CPLX)
        arow[j].x += eps;
      else
        arow[j] += eps;
    }
  }
  __syncthreads();  // every lane has read its row: the factor may overwrite the covariance

  // Cholesky A = C C^H, right-looking: at step k lane i (i >= k) finds C[i][k], publishes
  // it in `col` and in the packed factor, and updates its row's trailing entries.  Lanes
  // above the pivot row contribute nothing (their entries right of the diagonal are unused).
  double rdi = 0.0;  // 1 / C[i][i]
#pragma unroll
  for (int k = 0; k < kMvL; ++k) {
    const double piv = shfl32(re_(arow[k]), k);
    const double rdk = rsqrt_nr(piv);  // 1 / sqrt(pivot)
    const double dk = piv * rdk;
    D lik = scale_(arow[k], rdk);
    if (i == k) {
      if constexpr (CPLX) lik = cf64{dk, 0.0}; else lik = dk;
      rdi = rdk;
    }
    if (i < k) lik = widen(zero_of<F>());
    arow[k] = lik;
    col[i] = lik;
    if (i >= k) Lp[row_off(i) + k] = lik;
    __syncthreads();
#pragma unroll
    for (int jj = k + 1; jj < kMvL; ++jj) arow[jj] = fma_conj(neg_(lik), col[jj], arow[jj]);
    __syncthreads();  // `col` is rewritten by the next step
  }

  // C u = 1 (forward; lane i owns u_i and its row of C), then C^H v = u (backward; the
  // entries conj(C[k][i]) come from the packed factor)
  D acc = widen(zero_of<F>());
  D u = acc;
#pragma unroll
  for (int k = 0; k < kMvL; ++k) {
    D one;
    if constexpr (CPLX) one = cf64{1.0, 0.0}; else one = 1.0;
    D uk = scale_(sub_(one, acc), rdi);
    uk = shfl32(uk, k);
    if (i == k) u = uk;
    if (i > k) acc = fma_(arow[k], uk, acc);
  }
  D v = widen(zero_of<F>());
  acc = v;
#pragma unroll
  for (int k = kMvL - 1; k >= 0; --k) {
    D vk = scale_(sub_(u, acc), rdi);
    vk = shfl32(vk, k);
    if (i == k) v = vk;
    if (i < k) acc = fma_(conj_(Lp[row_off(k) + i]), vk, acc);
  }
  // w = v / 1^T v (so that 1^T w = 1), then binary32
  const D vsum = sum32(v);
  const F w = narrow(div_(v, vsum));

  // full-aperture weights: w_full[e] = (1/K) sum_{i = max(0, e-K+1)}^{min(L-1, e)} w[i], from
  // the inclusive prefix sums of w (pre[0] = 0)
  F sc = w;
#pragma unroll
  for (int off = 1; off < kMvL; off <<= 1) {
    const F o = shfl_up32(sc, off);
    if (i >= off) sc = add_(sc, o);
  }
  __syncthreads();  // the last reads of `col` are done: `pre` aliases it
  pre[i + 1] = sc;
  if (i == 0) pre[0] = zero_of<F>();
  __syncthreads();
  const float invK = 1.0f / float(K);
  const F* xw = xp + size_t(AVG ? T / 2 : 0) * M;  // the pixel's own samples
  F ys = zero_of<F>();
  for (int e = i; e < M; e += kMvL) {
    const int hi = min(kMvL - 1, e), lo = max(0, e - K + 1);
    const F wf = scale_(sub_(pre[hi + 1], pre[lo]), invK);
    if (ok && w_full) w_full[size_t(p) * M + e] = wf;
    ys = fma_conj(ok ? xw[e] : zero_of<F>(), wf, ys);  // conj(wf) x
  }
  ys = sum32(ys);
  if (ok && y && i == 0) y[p] = ys;
}

}  // namespace usbf

using namespace usbf;

template <typename Src, typename Out, int CHUNK>
static int gather_launch(const Src* rf, int32_t n_frames, const usbf_geometry* geom, const usbf_rx* rx,
                         const int32_t* pix, int32_t n_pix, int32_t n_avg, Out* x, hipStream_t stream) {
  DasArgs a;
  int st = make_das_args(geom, rx, &a);
  if (st) return st;
  USBF_REQUIRE(rf && pix && x, USBF_EINVAL, "null channel data, pix or x");
  USBF_REQUIRE(n_frames >= 1 && n_pix >= 1, USBF_EINVAL, "n_frames and n_pix must be >= 1");
  USBF_REQUIRE(n_avg >= 1 && n_avg <= 255 && n_avg % 2 == 1, USBF_EINVAL, "n_avg %d: must be odd in 1..255", n_avg);
  const int64_t blocks = (int64_t(n_pix) * n_avg + kGatherPix - 1) / kGatherPix;
  USBF_REQUIRE(blocks <= 0x7fffffff, USBF_EUNSUPPORTED, "too many gathered rows");
  hipLaunchKernelGGL((gather_kernel<Src, Out, CHUNK>), dim3(unsigned(blocks)), dim3(256), 0, stream, rf, n_frames, a,
                     pix, n_pix, int(n_avg), x);
  return check_launch("gather_kernel");
}

extern "C" int usbf_delay_gather(const int16_t* rf, int32_t n_frames, const usbf_geometry* geom, const usbf_rx* rx,
                                 const int32_t* pix, int32_t n_pix, float* x, hipStream_t stream) {
  return gather_launch<int16_t, float, 128>(rf, n_frames, geom, rx, pix, n_pix, 1, x, stream);
}

extern "C" int usbf_delay_gather_depths(const int16_t* rf, int32_t n_frames, const usbf_geometry* geom,
                                        const usbf_rx* rx, const int32_t* pix, int32_t n_pix, int32_t n_avg, float* x,
                                        hipStream_t stream) {
  return gather_launch<int16_t, float, 128>(rf, n_frames, geom, rx, pix, n_pix, n_avg, x, stream);
}

extern "C" int usbf_delay_gather_complex(const float* za, int32_t n_frames, const usbf_geometry* geom,
                                         const usbf_rx* rx, const int32_t* pix, int32_t n_pix, float* z,
                                         hipStream_t stream) {
  return gather_launch<cf32, cf32, 64>(reinterpret_cast<const cf32*>(za), n_frames, geom, rx, pix, n_pix, 1,
                                       reinterpret_cast<cf32*>(z), stream);
}

template <bool CPLX>
static int mv_launch(const float* x, int32_t n_pix, int32_t n_avg, int32_t n_el, int32_t subap, float loading,
                     float* w_full, float* y, hipStream_t stream) {
  USBF_REQUIRE(x && (w_full || y), USBF_EINVAL, "null x, or neither w_full nor y requested");
  USBF_REQUIRE(n_pix >= 1, USBF_EINVAL, "n_pix must be >= 1");
  USBF_REQUIRE(n_avg >= 1 && n_avg <= 255 && n_avg % 2 == 1, USBF_EINVAL, "n_avg %d: must be odd in 1..255", n_avg);
  USBF_REQUIRE(subap == kMvL, USBF_EUNSUPPORTED, "subaperture %d: only %d is implemented", subap, kMvL);
  USBF_REQUIRE(n_el >= subap && n_el <= kMvMaxEl, USBF_EUNSUPPORTED, "n_el %d outside %d..%d", n_el, subap,
               kMvMaxEl);
  USBF_REQUIRE(loading > 0.0f && loading < 1e30f, USBF_EINVAL, "loading must be finite and > 0");
  const int blocks = (n_pix + 1) / 2;
  const size_t pix_lds = mv_pixel_lds<CPLX>(n_el);
  const size_t lds = 2 * pix_lds;
  if (n_avg == 1) {
    hipLaunchKernelGGL((mv_kernel<CPLX, false>), dim3(blocks), dim3(64), lds, stream, x, n_pix, 1, n_el, loading,
                       w_full, y, pix_lds);
  } else {
    hipLaunchKernelGGL((mv_kernel<CPLX, true>), dim3(blocks), dim3(64), lds, stream, x, n_pix, int(n_avg), n_el,
                       loading, w_full, y, pix_lds);
  }
  return check_launch("mv_kernel");
}

extern "C" int usbf_mv_weights(const float* x, int32_t n_pix, int32_t n_el, int32_t subap, float loading,
                               float* w_full, float* y, hipStream_t stream) {
  return mv_launch<false>(x, n_pix, 1, n_el, subap, loading, w_full, y, stream);
}

extern "C" int usbf_mv_weights_averaged(const float* x, int32_t n_pix, int32_t n_avg, int32_t n_el, int32_t subap,
                                        float loading, float* w_full, float* y, hipStream_t stream) {
  return mv_launch<false>(x, n_pix, n_avg, n_el, subap, loading, w_full, y, stream);
}

extern "C" int usbf_mv_weights_complex(const float* z, int32_t n_pix, int32_t n_el, int32_t subap, float loading,
                                       float* w_full, float* y, hipStream_t stream) {
  return mv_launch<true>(z, n_pix, 1, n_el, subap, loading, w_full, y, stream);
}
