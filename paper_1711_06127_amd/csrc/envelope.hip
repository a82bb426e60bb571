// Envelope detection (Sec. 1 pipeline list; Hilbert-transform envelope of the PSF study,
// Sec. 3.2): env = |IDFT(H . DFT(y))| per row, H keeping DC (and Nyquist), doubling the
// positive and removing the negative frequencies.
//
// One workgroup owns a row at a time (grid-stride over rows so the twiddle table is built
// once per workgroup) and runs a mixed-radix self-sorting Stockham FFT in LDS: radix 8, 4, 2,
// 3, 5 butterflies, and the plain DFT for prime factors 7 ... 31.
// The inverse transform is done as a forward transform of the conjugate: the magnitude of
// conj(FFT(conj(X))) / n needs no final conjugation.
#include "common.h"

namespace usbf {

constexpr int kEnvThreads = 256;
constexpr int kMaxStages = 16;
// three n-point complex buffers (two ping-pong, one twiddle table) must fit the 64 KiB LDS
// a workgroup gets without opting in to more
constexpr int kMaxEnvelopeLength = 2048;

struct FftPlan {
  int n;
  int n_stages;
  int radix[kMaxStages];
};

struct alignas(8) c32 {
  float x, y;
};

// LDS arrays are padded by one element per 16 so that the strided accesses of the early
// stages (and of the twiddle table) spread over the banks
__host__ __device__ constexpr int pad(int i) { return i + (i >> 4); }
__host__ __device__ constexpr int padded_len(int n) { return pad(n) + 1; }

// Power-of-two transforms permute LDS indices instead of padding them: bits 0-3 of an index are
// XORed with bits 3-6 and bits 5-8.  Bit 3 changes only by bits 6 and 8, so the map is a
// bijection on every aligned block of 16 elements.  On gfx950 8-byte LDS reads are served 32
// lanes at a time from 64 banks of 4 bytes and 8-byte writes 16 lanes at a time from 32 banks;
// with this map every stage's reads, writes and twiddle reads take the minimum number of
// passes (one element of padding per 16 leaves them 2-way).
__host__ __device__ constexpr int swz(int i) { return i ^ (((i >> 3) ^ (i >> 5)) & 15); }
__host__ __device__ constexpr int swz_len(int n) { return (n + 15) & ~15; }

__device__ inline c32 cadd(c32 a, c32 b) { return {a.x + b.x, a.y + b.y}; }
__device__ inline c32 csub(c32 a, c32 b) { return {a.x - b.x, a.y - b.y}; }
__device__ inline c32 cmul(c32 a, c32 b) {
  return {__builtin_fmaf(a.x, b.x, -a.y * b.y), __builtin_fmaf(a.x, b.y, a.y * b.x)};
}
__device__ inline c32 cscale(c32 a, float s) { return {a.x * s, a.y * s}; }
__device__ inline c32 mul_mi(c32 a) { return {a.y, -a.x}; }  // -i * a
// |a|: the hardware square root (within 1 ulp) -- magnitudes are values, compared to 1e-4 of a
// row's maximum, and the correctly rounded sequence costs some twenty instructions more
__device__ inline float cabs(float x, float y) { return __builtin_amdgcn_sqrtf(__builtin_fmaf(x, x, y * y)); }

// In-register forward DFTs of size 2, 3, 4, 5 (kernel e^{-2 pi i m q / R}).
__device__ inline void dft2(c32* v) {
  c32 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}
__device__ inline void dft4(c32* v) {
  c32 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
  c32 t2 = cadd(v[1], v[3]), t3 = mul_mi(csub(v[1], v[3]));
  v[0] = cadd(t0, t2);
  v[2] = csub(t0, t2);
  v[1] = cadd(t1, t3);
  v[3] = csub(t1, t3);
}
// size 8: two size-4 transforms of the even and odd inputs, combined with e^{-2 pi i k / 8}
__device__ inline void dft8(c32* v) {
  const float h = 0.70710678118654752440f;  // sqrt(1/2)
  c32 a[4] = {v[0], v[2], v[4], v[6]}, b[4] = {v[1], v[3], v[5], v[7]};
  dft4(a);
  dft4(b);
  const c32 t1 = {h * (b[1].x + b[1].y), h * (b[1].y - b[1].x)};    // b1 e^{-i pi/4}
  const c32 t2 = mul_mi(b[2]);                                       // b2 e^{-i pi/2}
  const c32 t3 = {h * (b[3].y - b[3].x), -h * (b[3].x + b[3].y)};   // b3 e^{-3 i pi/4}
  v[0] = cadd(a[0], b[0]);
  v[4] = csub(a[0], b[0]);
  v[1] = cadd(a[1], t1);
  v[5] = csub(a[1], t1);
  v[2] = cadd(a[2], t2);
  v[6] = csub(a[2], t2);
  v[3] = cadd(a[3], t3);
  v[7] = csub(a[3], t3);
}

__device__ inline void dft3(c32* v) {
  const float h = 0.86602540378443864676f;  // sqrt(3)/2
  c32 s = cadd(v[1], v[2]);
  c32 d = csub(v[1], v[2]);
  c32 m = {v[0].x - 0.5f * s.x, v[0].y - 0.5f * s.y};
  c32 jd = mul_mi(cscale(d, h));
  v[0] = cadd(v[0], s);
  v[1] = cadd(m, jd);
  v[2] = csub(m, jd);
}
__device__ inline void dft5(c32* v) {
  const float c1 = 0.30901699437494742410f, c2 = -0.80901699437494742410f;
  const float s1 = 0.95105651629515357212f, s2 = 0.58778525229247312917f;
  c32 a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
  c32 a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
  c32 x0 = v[0];
  c32 p1 = {x0.x + c1 * a1.x + c2 * a2.x, x0.y + c1 * a1.y + c2 * a2.y};
  c32 p2 = {x0.x + c2 * a1.x + c1 * a2.x, x0.y + c2 * a1.y + c1 * a2.y};
  c32 q1 = mul_mi({s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y});
  c32 q2 = mul_mi({s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y});
  v[0] = {x0.x + a1.x + a2.x, x0.y + a1.y + a2.y};
  v[1] = cadd(p1, q1);
  v[4] = csub(p1, q1);
  v[2] = cadd(p2, q2);
  v[3] = csub(p2, q2);
}

// Forward DFT of prime size R by its definition, y_k = sum_m v_m e^{-2 pi i m k / R}, each
// output written straight to its destination; the roots come from the n-point table
// (tw[q * n / R] = e^{-2 pi i q / R}).
template <int R>
__device__ inline void dft_prime_store(const c32* v, const c32* __restrict__ tw, int tw_r, c32* __restrict__ dst,
                                       int o, int stride) {
  for (int k = 0; k < R; ++k) {
    c32 acc = v[0];
#pragma unroll
    for (int m = 1; m < R; ++m) acc = cadd(acc, cmul(v[m], tw[pad(((m * k) % R) * tw_r)]));
    dst[pad(o + k * stride)] = acc;
  }
}

template <int R>
__device__ inline void stage(const c32* __restrict__ a, c32* __restrict__ b, const c32* __restrict__ tw, int n, int ns) {
  const int m = n / R;
  const int tw_step = n / (ns * R);
  for (int j = threadIdx.x; j < m; j += kEnvThreads) {
    c32 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = a[pad(j + r * m)];
    const int k = j % ns;
#pragma unroll
    for (int r = 1; r < R; ++r) v[r] = cmul(v[r], tw[pad(r * k * tw_step)]);
    if constexpr (R == 2) dft2(v);
    if constexpr (R == 3) dft3(v);
    if constexpr (R == 4) dft4(v);
    const int o = (j / ns) * ns * R + k;
    if constexpr (R == 8) {
      dft8(v);
#pragma unroll
      for (int r = 0; r < R; ++r) b[pad(o + r * ns)] = v[r];
    } else if constexpr (R > 5) {
      dft_prime_store<R>(v, tw, m, b, o, ns);
    } else {
      if constexpr (R == 5) dft5(v);
#pragma unroll
      for (int r = 0; r < R; ++r) b[pad(o + r * ns)] = v[r];
    }
  }
}

// Power-of-two lengths: the same Stockham stages with every size, stride and twiddle step a
// compile-time constant (radix 8 stages, then one radix 4 or 2 stage), so the index
// arithmetic reduces to shifts and masks and the first stage skips its unit twiddles.
template <int N, int R, int NS>
__device__ inline void stage_c(const c32* __restrict__ a, c32* __restrict__ b, const c32* __restrict__ tw) {
  constexpr int M = N / R, TWS = N / (NS * R);
  for (int j = threadIdx.x; j < M; j += kEnvThreads) {
    c32 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = a[pad(j + r * M)];
    const int k = j % NS;
    if constexpr (NS > 1) {
      // twiddles W^(r k TWS) as powers of W^(k TWS): one table read per butterfly
      const c32 w1 = tw[pad(k * TWS)];
      c32 w = w1;
      v[1] = cmul(v[1], w);
#pragma unroll
      for (int r = 2; r < R; ++r) {
        w = cmul(w, w1);
        v[r] = cmul(v[r], w);
      }
    }
    if constexpr (R == 2) dft2(v);
    if constexpr (R == 4) dft4(v);
    if constexpr (R == 8) dft8(v);
    const int o = (j / NS) * NS * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) b[pad(o + r * NS)] = v[r];
  }
}

template <int N, int NS>
__device__ inline int fft_pow2_from(c32* a, c32* b, const c32* tw, int cur) {
  if constexpr (NS >= N) {
    return cur;
  } else {
    constexpr int left = N / NS;
    constexpr int R = left >= 8 ? 8 : left;  // radix 8 while it divides, then 4 or 2
    stage_c<N, R, NS>(a, b, tw);
    __syncthreads();
    return fft_pow2_from<N, NS * R>(b, a, tw, cur ^ 1);
  }
}

// ---- power-of-two rows with fused ends: the first stage takes its inputs from registers
// (the prefetched row), the last stage of the forward transform writes the analytic-signal
// spectrum (weights and conjugation applied), and the last stage of the inverse writes the
// magnitudes straight to global memory -- three LDS round trips and barriers fewer per row.
template <int N, int NS>
__host__ __device__ constexpr int radix_at() {
  return (N / NS) >= 8 ? 8 : N / NS;
}

// One Stockham stage with a custom source (element j + r M of the input) and destination.
template <int N, int NS, typename Load, typename Store>
__device__ inline void stage_ls(const c32* __restrict__ tw, Load load, Store store) {
  constexpr int R = radix_at<N, NS>();
  constexpr int M = N / R, TWS = N / (NS * R);
  for (int j = threadIdx.x; j < M; j += kEnvThreads) {
    c32 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = load(j, r, M);
    const int k = j % NS;
    if constexpr (NS > 1) {
      // twiddles W^(r k TWS) as powers of W^(k TWS): one table read per butterfly
      const c32 w1 = tw[swz(k * TWS)];
      c32 w = w1;
      v[1] = cmul(v[1], w);
#pragma unroll
      for (int r = 2; r < R; ++r) {
        w = cmul(w, w1);
        v[r] = cmul(v[r], w);
      }
    }
    if constexpr (R == 2) dft2(v);
    if constexpr (R == 4) dft4(v);
    if constexpr (R == 8) dft8(v);
    const int o = (j / NS) * NS * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) store(o + r * NS, v[r]);
  }
}

// Stages NS .. N of a transform whose input is in LDS buffer a; every stage but the last
// writes the other buffer, the last hands its outputs to fin(k, value).
template <int N, int NS, typename Fin>
__device__ inline void stages_from(c32* a, c32* b, const c32* tw, Fin fin) {
  constexpr int R = radix_at<N, NS>();
  auto from_a = [&](int j, int r, int M) { return a[swz(j + r * M)]; };
  if constexpr (NS * R == N) {
    stage_ls<N, NS>(tw, from_a, fin);
  } else {
    stage_ls<N, NS>(tw, from_a, [&](int i, c32 v) { b[swz(i)] = v; });
    __syncthreads();
    stages_from<N, NS * R>(b, a, tw, fin);
  }
}

// the buffer the last stage of a transform starting (at stage NS) in buffer 0 reads
template <int N, int NS>
__host__ __device__ constexpr int last_src(int cur) {
  return (NS * radix_at<N, NS>() == N) ? cur : last_src<N, NS * radix_at<N, NS>()>(cur ^ 1);
}

// Largest twiddle index the power-of-two transform reads, (NS - 1) * N / (NS * R) over its
// stages, plus one: the table holds W^0 .. W^(that - 1) only.
template <int N, int NS = 1>
__host__ __device__ constexpr int pow2_twiddles() {
  if constexpr (NS >= N) {
    return 1;
  } else {
    constexpr int R = radix_at<N, NS>();
    constexpr int here = (NS - 1) * (N / (NS * R)) + 1;
    constexpr int rest = pow2_twiddles<N, NS * R>();
    return here > rest ? here : rest;
  }
}
template <int N>
__host__ __device__ constexpr size_t pow2_lds_bytes() {
  return (size_t(2) * swz_len(N) + swz_len(pow2_twiddles<N>())) * sizeof(c32);
}

// in == env is allowed (the pipeline detects in place): every row is read whole before any
// of it is written, and the prefetched next row is another row, so neither pointer is
// declared restrict.
template <int N>
__global__ __launch_bounds__(kEnvThreads) void envelope_pow2_kernel(const float* in, int64_t n_rows, float* env,
                                                                    float* __restrict__ row_max) {
  static_assert(N >= 64 && (N & (N - 1)) == 0 && N <= kMaxEnvelopeLength, "power-of-two length");
  extern __shared__ c32 lds[];
  constexpr int np = swz_len(N);
  constexpr int M1 = N / 8;  // butterflies of the first (radix 8) stage
  c32* buf0 = lds;
  c32* buf1 = lds + np;
  c32* tw = lds + 2 * np;
  const int tid = threadIdx.x;
  for (int k = tid; k < pow2_twiddles<N>(); k += kEnvThreads) {
    float s, c;
    sincospif(2.0f * float(k) / float(N), &s, &c);
    tw[swz(k)] = {c, -s};
  }
  __shared__ float red[kEnvThreads / 64];
  // prefetched row, laid out as the first stage reads it: lane j holds x[j + r N/8]
  float pre[8];
  auto load_row = [&](int64_t row) {
    const float* x = in + row * N;
    if (tid < M1) {
#pragma unroll
      for (int r = 0; r < 8; ++r) pre[r] = x[tid + r * M1];
    }
  };
  if (int64_t(blockIdx.x) < n_rows) load_row(blockIdx.x);
  __syncthreads();  // twiddles
  for (int64_t row = blockIdx.x; row < n_rows; row += gridDim.x) {
    // forward transform: first stage from registers into buf0
    stage_ls<N, 1>(tw, [&](int, int r, int) { return c32{pre[r], 0.0f}; }, [&](int i, c32 v) { buf0[swz(i)] = v; });
    if (row + gridDim.x < n_rows) load_row(row + gridDim.x);
    __syncthreads();
    // remaining stages; the last writes H X, conjugated (inverse by forward transform), into
    // the buffer it does not read
    constexpr int src1 = last_src<N, 8>(0);
    c32* spec = src1 == 0 ? buf1 : buf0;
    // (the bins above N/2 are zero: neither written nor read)
    stages_from<N, 8>(buf0, buf1, tw, [&](int k, c32 v) {
      const float hk = (k == 0 || k == N / 2) ? 1.0f : 2.0f;
      if (k <= N / 2) spec[swz(k)] = c32{v.x * hk, -v.y * hk};
    });
    __syncthreads();
    c32* other = spec == buf0 ? buf1 : buf0;
    // inverse, first (radix 8) stage: input j + r N/8 is bin N/2 + j for r = 4 (nonzero only for
    // j = 0) and above N/2 for r > 4
    stage_ls<N, 1>(tw,
                   [&](int j, int r, int M) {
                     if (r > 4) return c32{0.0f, 0.0f};
                     if (r == 4) return j == 0 ? spec[swz(N / 2)] : c32{0.0f, 0.0f};
                     return spec[swz(j + r * M)];
                   },
                   [&](int i, c32 v) { other[swz(i)] = v; });
    __syncthreads();
    float mx = 0.0f;
    float* e = env + row * N;
    stages_from<N, 8>(other, spec, tw, [&](int k, c32 v) {
      const float m = cabs(v.x, v.y) * (1.0f / float(N));
      e[k] = m;
      mx = fmaxf(mx, m);
    });
    if (row_max) {
      for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
      if ((tid & 63) == 0) red[tid >> 6] = mx;
    }
    __syncthreads();
    if (row_max && tid == 0) {
      float m = red[0];
      for (int w = 1; w < kEnvThreads / 64; ++w) m = fmaxf(m, red[w]);
      row_max[row] = m;
    }
  }
}

// Forward FFT of buf[0] (result in buf[0] or buf[1]); returns the buffer holding the result.
// PRIMES: the plan may hold radices 7 ... 31 (kept out of the common kernel: their register
// footprint would cut its occupancy).
template <bool PRIMES>
__device__ inline int fft_lds(c32* buf0, c32* buf1, const c32* tw, const FftPlan& P) {
  c32* a = buf0;
  c32* b = buf1;
  int ns = 1;
  int cur = 0;
  for (int s = 0; s < P.n_stages; ++s) {
    const int R = P.radix[s];
    switch (R) {
      case 8: stage<8>(a, b, tw, P.n, ns); break;
      case 4: stage<4>(a, b, tw, P.n, ns); break;
      case 2: stage<2>(a, b, tw, P.n, ns); break;
      case 3: stage<3>(a, b, tw, P.n, ns); break;
      case 5: stage<5>(a, b, tw, P.n, ns); break;
      default:
        if constexpr (PRIMES) {
          switch (R) {
            case 7: stage<7>(a, b, tw, P.n, ns); break;
            case 11: stage<11>(a, b, tw, P.n, ns); break;
            case 13: stage<13>(a, b, tw, P.n, ns); break;
            case 17: stage<17>(a, b, tw, P.n, ns); break;
            case 19: stage<19>(a, b, tw, P.n, ns); break;
            case 23: stage<23>(a, b, tw, P.n, ns); break;
            case 29: stage<29>(a, b, tw, P.n, ns); break;
            default: stage<31>(a, b, tw, P.n, ns); break;
          }
        }
        break;
    }
    __syncthreads();
    c32* t = a;
    a = b;
    b = t;
    cur ^= 1;
    ns *= R;
  }
  return cur;
}

// N > 0: power-of-two length N with the compile-time transform; N = 0: any supported length
// with the plan's mixed-radix transform (PRIMES: radices above 8 present)
template <int N, bool PRIMES>
__global__ __launch_bounds__(kEnvThreads) void envelope_kernel(const float* in, int64_t n_rows, FftPlan P,
                                                               float* env, float* __restrict__ row_max) {
  extern __shared__ c32 lds[];
  const int n = P.n;
  const int np = padded_len(n);
  c32* buf[2] = {lds, lds + np};
  c32* tw = lds + 2 * np;
  for (int k = threadIdx.x; k < n; k += kEnvThreads) {
    float s, c;
    sincospif(2.0f * float(k) / float(n), &s, &c);
    tw[pad(k)] = {c, -s};
  }
  const int half = n / 2;
  const bool even = (n % 2) == 0;
  const float inv_n = 1.0f / float(n);
  __shared__ float red[kEnvThreads / 64];
  // rows are taken grid-stride; the next row is loaded into registers while this one is
  // transformed, so its memory latency hides behind the FFTs
  constexpr int kPer = kMaxEnvelopeLength / kEnvThreads;
  float pre[kPer];
  auto load_row = [&](int64_t row) {
    const float* x = in + row * n;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int k = threadIdx.x + i * kEnvThreads;
      pre[i] = (k < n) ? x[k] : 0.0f;
    }
  };
  if (int64_t(blockIdx.x) < n_rows) load_row(blockIdx.x);
  for (int64_t row = blockIdx.x; row < n_rows; row += gridDim.x) {
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int k = threadIdx.x + i * kEnvThreads;
      if (k < n) buf[0][pad(k)] = {pre[i], 0.0f};
    }
    if (row + gridDim.x < n_rows) load_row(row + gridDim.x);
    __syncthreads();
    int cur;
    if constexpr (N > 0)
      cur = fft_pow2_from<N, 1>(buf[0], buf[1], tw, 0);
    else
      cur = fft_lds<PRIMES>(buf[0], buf[1], tw, P);
    // analytic-signal weights, then conjugate for the inverse-by-forward transform
    c32* X = buf[cur];
    for (int k = threadIdx.x; k < n; k += kEnvThreads) {
      float hk;
      if (k == 0 || (even && k == half))
        hk = 1.0f;
      else if (k < (n + 1) / 2)
        hk = 2.0f;
      else
        hk = 0.0f;
      c32 v = X[pad(k)];
      X[pad(k)] = {v.x * hk, -v.y * hk};
    }
    __syncthreads();
    int cur2;
    if constexpr (N > 0)
      cur2 = fft_pow2_from<N, 1>(X, buf[cur ^ 1], tw, 0);
    else
      cur2 = fft_lds<PRIMES>(X, buf[cur ^ 1], tw, P);
    c32* Y = (cur2 == 0) ? X : buf[cur ^ 1];
    float mx = 0.0f;
    float* e = env + row * n;
    for (int k = threadIdx.x; k < n; k += kEnvThreads) {
      c32 v = Y[pad(k)];
      float m = cabs(v.x, v.y) * inv_n;
      e[k] = m;
      mx = fmaxf(mx, m);
    }
    if (row_max) {
      for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
      if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    }
    __syncthreads();
    if (row_max && threadIdx.x == 0) {
      float m = red[0];
      for (int w = 1; w < kEnvThreads / 64; ++w) m = fmaxf(m, red[w]);
      row_max[row] = m;
    }
  }
}

// Analytic signal of int16 channel traces (the input of the complex minimum-variance
// estimator): z = IDFT(H . DFT(x)) per row, written as (re, im) pairs.  The same transform
// and weights as the envelope, with the final conjugation of the inverse-by-forward
// transform applied instead of the magnitude.  Rows of up to kMaxAnalyticLength samples:
// three n-point complex buffers in up to 104 KB of LDS.
constexpr int kMaxAnalyticLength = 4096;

template <bool PRIMES>
__global__ __launch_bounds__(kEnvThreads) void analytic_kernel(const int16_t* __restrict__ in, int64_t n_rows,
                                                               FftPlan P, c32* __restrict__ out) {
  extern __shared__ c32 lds[];
  const int n = P.n;
  const int np = padded_len(n);
  c32* buf[2] = {lds, lds + np};
  c32* tw = lds + 2 * np;
  for (int k = threadIdx.x; k < n; k += kEnvThreads) {
    float s, c;
    sincospif(2.0f * float(k) / float(n), &s, &c);
    tw[pad(k)] = {c, -s};
  }
  const int half = n / 2;
  const bool even = (n % 2) == 0;
  const float inv_n = 1.0f / float(n);
  for (int64_t row = blockIdx.x; row < n_rows; row += gridDim.x) {
    const int16_t* x = in + row * n;
    for (int k = threadIdx.x; k < n; k += kEnvThreads) buf[0][pad(k)] = {float(x[k]), 0.0f};
    __syncthreads();
    const int cur = fft_lds<PRIMES>(buf[0], buf[1], tw, P);
    c32* X = buf[cur];
    for (int k = threadIdx.x; k < n; k += kEnvThreads) {
      const float hk = (k == 0 || (even && k == half)) ? 1.0f : (k < (n + 1) / 2 ? 2.0f : 0.0f);
      const c32 v = X[pad(k)];
      X[pad(k)] = {v.x * hk, -v.y * hk};
    }
    __syncthreads();
    const int cur2 = fft_lds<PRIMES>(X, buf[cur ^ 1], tw, P);
    const c32* Y = (cur2 == 0) ? X : buf[cur ^ 1];
    c32* z = out + row * n;
    for (int k = threadIdx.x; k < n; k += kEnvThreads) {
      const c32 v = Y[pad(k)];
      z[k] = {v.x * inv_n, -v.y * inv_n};
    }
    __syncthreads();  // the next row overwrites the buffers
  }
}

int make_fft_plan(int n, FftPlan* P) {
  P->n = n;
  P->n_stages = 0;
  int m = n;
  const int order[13] = {8, 4, 2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31};
  for (int R : order) {
    while (m % R == 0) {
      if (P->n_stages >= kMaxStages) return USBF_EUNSUPPORTED;
      P->radix[P->n_stages++] = R;
      m /= R;
    }
  }
  return m == 1 ? USBF_OK : USBF_EUNSUPPORTED;
}

bool envelope_length_ok(int n) {
  FftPlan P;
  return n >= 8 && n <= kMaxEnvelopeLength && make_fft_plan(n, &P) == USBF_OK;
}

int envelope_enqueue(const float* in, int64_t n_rows, int n, float* env, float* row_max, hipStream_t s) {
  FftPlan P;
  USBF_REQUIRE(make_fft_plan(n, &P) == USBF_OK, USBF_EUNSUPPORTED, "envelope length %d has a prime factor above 31", n);
  // a resident grid (the twiddle table is built once per workgroup): 160 KB of LDS per CU
  // holds 160 KB / (24 n) workgroups
  int dev = 0, n_cu = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  size_t lds = size_t(3) * padded_len(n) * sizeof(c32);
  if (n == 2048) lds = pow2_lds_bytes<2048>();
  if (n == 1024) lds = pow2_lds_bytes<1024>();
  if (n == 512) lds = pow2_lds_bytes<512>();
  if (n == 256) lds = pow2_lds_bytes<256>();
  const int per_cu = std::max(1, std::min(8, int(163840 / (lds + 64))));
  const int64_t blocks = std::min<int64_t>(n_rows, int64_t(n_cu) * per_cu);
  bool primes = false;
  for (int k = 0; k < P.n_stages; ++k) primes = primes || (P.radix[k] > 5 && P.radix[k] != 8);
  const dim3 grid = dim3(static_cast<unsigned>(blocks)), block = dim3(kEnvThreads);
  switch (n) {
    case 2048: hipLaunchKernelGGL((envelope_pow2_kernel<2048>), grid, block, lds, s, in, n_rows, env, row_max); break;
    case 1024: hipLaunchKernelGGL((envelope_pow2_kernel<1024>), grid, block, lds, s, in, n_rows, env, row_max); break;
    case 512: hipLaunchKernelGGL((envelope_pow2_kernel<512>), grid, block, lds, s, in, n_rows, env, row_max); break;
    case 256: hipLaunchKernelGGL((envelope_pow2_kernel<256>), grid, block, lds, s, in, n_rows, env, row_max); break;
    default:
      if (primes)
        hipLaunchKernelGGL((envelope_kernel<0, true>), grid, block, lds, s, in, n_rows, P, env, row_max);
      else
        hipLaunchKernelGGL((envelope_kernel<0, false>), grid, block, lds, s, in, n_rows, P, env, row_max);
  }
  return check_launch("envelope_kernel");
}

}  // namespace usbf

extern "C" int usbf_analytic_channels(const int16_t* rf, int64_t n_rows, int32_t n, float* za, hipStream_t stream) {
  using namespace usbf;
  USBF_REQUIRE(rf && za, USBF_EINVAL, "null rf or za");
  USBF_REQUIRE((reinterpret_cast<uintptr_t>(za) & 7) == 0, USBF_EINVAL, "za must be 8-byte aligned");
  USBF_REQUIRE(n_rows >= 1, USBF_EINVAL, "n_rows must be >= 1");
  USBF_REQUIRE(n >= 8 && n <= kMaxAnalyticLength, USBF_EUNSUPPORTED, "trace length %d outside 8..%d", n,
               kMaxAnalyticLength);
  FftPlan P;
  USBF_REQUIRE(make_fft_plan(n, &P) == USBF_OK, USBF_EUNSUPPORTED, "trace length %d has a prime factor above 31", n);
  bool primes = false;
  for (int k = 0; k < P.n_stages; ++k) primes = primes || (P.radix[k] > 5 && P.radix[k] != 8);
  const size_t lds = size_t(3) * padded_len(n) * sizeof(c32);
  const void* fn = primes ? reinterpret_cast<const void*>(&analytic_kernel<true>)
                          : reinterpret_cast<const void*>(&analytic_kernel<false>);
  if (lds > 65536) {
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    USBF_REQUIRE(e == hipSuccess, USBF_EDEVICE, "hipFuncSetAttribute: %s", hipGetErrorString(e));
  }
  int dev = 0, n_cu = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  const int per_cu = std::max(1, std::min(8, int(163840 / (lds + 64))));
  const int64_t blocks = std::min<int64_t>(n_rows, int64_t(n_cu) * per_cu);
  c32* out = reinterpret_cast<c32*>(za);
  if (primes)
    hipLaunchKernelGGL((analytic_kernel<true>), dim3(unsigned(blocks)), dim3(kEnvThreads), lds, stream, rf, n_rows, P,
                       out);
  else
    hipLaunchKernelGGL((analytic_kernel<false>), dim3(unsigned(blocks)), dim3(kEnvThreads), lds, stream, rf, n_rows,
                       P, out);
  return check_launch("analytic_kernel");
}

extern "C" int usbf_envelope(const float* in, int64_t n_rows, int32_t n, float* env, float* row_max,
                             hipStream_t stream) {
  USBF_REQUIRE(in && env, USBF_EINVAL, "null in or env");
  USBF_REQUIRE(n_rows >= 1, USBF_EINVAL, "n_rows must be >= 1");
  USBF_REQUIRE(n >= 8 && n <= usbf::kMaxEnvelopeLength, USBF_EUNSUPPORTED, "envelope length %d outside 8..%d", n,
               usbf::kMaxEnvelopeLength);
  return usbf::envelope_enqueue(in, n_rows, n, env, row_max, stream);
}
