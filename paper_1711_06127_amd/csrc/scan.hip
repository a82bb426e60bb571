// Log compression (Sec. 1 pipeline list; Sec. 2 method list item 4) and scan conversion
// (Sec. 1 pipeline list, last step; Sec. 2 method list item 5), plus the fused
// log-then-scan kernel used by the whole-pipeline call.
#include "common.h"

namespace usbf {

constexpr int kScanThreads = 256;

struct ScanArgs {
  int kind, nx, ny, nz;
  float x0, hx, y0, hy, z0, hz;
  const float* line_u;
  const float* line_v;
  int n_u, n_v;
  float r0, dr;
  int n_depth;
  float fill;
  int64_t grid;      // pixels per frame
  int64_t frame_in;  // line samples per frame
};

int make_scan_args(const usbf_scan* s, ScanArgs* a) {
  USBF_REQUIRE(s, USBF_EINVAL, "null scan");
  USBF_REQUIRE(s->kind >= 0 && s->kind <= 2, USBF_EINVAL, "scan kind must be 0, 1 or 2");
  USBF_REQUIRE(s->line_u && (s->kind != 1 || s->line_v), USBF_EINVAL, "null line table");
  USBF_REQUIRE(s->nx >= 1 && s->nz >= 1 && (s->kind != 1 || s->ny >= 1), USBF_EINVAL, "empty grid");
  USBF_REQUIRE(s->n_u >= 2 && (s->kind != 1 || s->n_v >= 2) && s->n_depth >= 2, USBF_ESHAPE,
               "scan conversion needs >= 2 lines per axis and >= 2 depth samples");
  USBF_REQUIRE(finite_pos(s->dr), USBF_EINVAL, "dr must be finite and > 0");
  a->kind = s->kind;
  a->nx = s->nx;
  a->ny = s->kind == 1 ? s->ny : 1;
  a->nz = s->nz;
  a->x0 = s->x0;
  a->hx = s->hx;
  a->y0 = s->y0;
  a->hy = s->hy;
  a->z0 = s->z0;
  a->hz = s->hz;
  a->line_u = s->line_u;
  a->line_v = s->line_v;
  a->n_u = s->n_u;
  a->n_v = s->kind == 1 ? s->n_v : 1;
  a->r0 = s->r0;
  a->dr = s->dr;
  a->n_depth = s->n_depth;
  a->fill = s->fill;
  a->grid = int64_t(a->nx) * a->ny * a->nz;
  a->frame_in = int64_t(a->n_u) * a->n_v * a->n_depth;
  USBF_REQUIRE(a->grid < (int64_t(1) << 31) && a->frame_in < (int64_t(1) << 31), USBF_EUNSUPPORTED,
               "grid or line data larger than 2^31");
  return USBF_OK;
}

int validate_scan(const usbf_scan* s) {
  ScanArgs a;
  return make_scan_args(s, &a);
}

#pragma clang fp contract(off)

// Largest i in [0, n-2] with t[i] <= u (t strictly increasing, t[0] <= u assumed).
__device__ inline int last_le(const float* t, int n, float u) {
  int lo = 0, hi = n - 1;  // invariant: t[lo] <= u, answer < hi or u >= t[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (t[mid] <= u)
      lo = mid;
    else
      hi = mid;
  }
  return lo > n - 2 ? n - 2 : lo;
}

struct Cell {
  int base;   // (line index of the lower corner) * n_depth + jd, -1 outside
  int n_u;    // line stride between the two u corners is 1, between v corners n_u
  float fu, fv, fd;
};

// Binary32 cell-index rule (usbf_scan_index_map) and interpolation fractions for pixel p.
__device__ inline Cell scan_cell(const ScanArgs& a, int64_t p) {
  const int i = int(p % a.nx);
  const int64_t q = p / a.nx;
  const int jy = int(q % a.ny);
  const int k = int(q / a.ny);
  const float x = a.x0 + float(i) * a.hx;
  const float y = a.y0 + float(jy) * a.hy;
  const float z = a.z0 + float(k) * a.hz;
  Cell c;
  c.base = -1;
  c.n_u = a.n_u;
  c.fu = c.fv = c.fd = 0.0f;
  float u, v = 0.0f, range;
  if (a.kind == 0) {
    u = x;
    range = z;
  } else {
    if (!(z > 0.0f)) return c;
    u = x / z;
    if (a.kind == 1) {
      v = y / z;
      float s = x * x + y * y;
      range = sqrtf(s + z * z);
    } else {
      range = sqrtf(x * x + z * z);
    }
  }
  const float qd = (range - a.r0) / a.dr;
  const float* U = a.line_u;
  if (!(u >= U[0] && u <= U[a.n_u - 1])) return c;
  if (!(qd >= 0.0f && qd <= float(a.n_depth - 1))) return c;
  int iv = 0;
  if (a.kind == 1) {
    const float* V = a.line_v;
    if (!(v >= V[0] && v <= V[a.n_v - 1])) return c;
    iv = last_le(V, a.n_v, v);
    c.fv = (v - V[iv]) / (V[iv + 1] - V[iv]);
  }
  const int iu = last_le(U, a.n_u, u);
  int jd = int(floorf(qd));
  jd = jd > a.n_depth - 2 ? a.n_depth - 2 : jd;
  c.fu = (u - U[iu]) / (U[iu + 1] - U[iu]);
  c.fd = qd - float(jd);
  c.base = (iv * a.n_u + iu) * a.n_depth + jd;
  return c;
}

#pragma clang fp contract(on)

struct LogMap {
  float scale;    // 20 log10(2) / dyn_range  (per log2 unit)
  float offset;   // 1 - scale * log2(ref)
  bool zero;      // ref not positive: everything maps to 0
};

__device__ inline LogMap log_map(float dyn_range_db, float ref) {
  LogMap m;
  m.zero = !(ref > 0.0f);
  m.scale = (20.0f * 0.30102999566398119521f) / dyn_range_db;
  m.offset = 1.0f - m.scale * (m.zero ? 0.0f : __log2f(ref));
  return m;
}

__device__ inline float log_apply(const LogMap& m, float env) {
  if (m.zero || !(env > 0.0f)) return 0.0f;
  float b = __builtin_fmaf(m.scale, __log2f(env), m.offset);
  return fminf(fmaxf(b, 0.0f), 1.0f);
}

__device__ inline float cell_value(const float* __restrict__ L, const Cell& c, int n_depth, int kind) {
  const float* p = L + c.base;
  float a0 = p[0], a1 = p[1], b0 = p[n_depth], b1 = p[n_depth + 1];
  float lo = __builtin_fmaf(c.fu, __builtin_fmaf(c.fd, b1 - b0, b0) - __builtin_fmaf(c.fd, a1 - a0, a0),
                            __builtin_fmaf(c.fd, a1 - a0, a0));
  if (kind != 1) return lo;
  const float* q = p + int64_t(c.n_u) * n_depth;
  float c0 = q[0], c1 = q[1], d0 = q[n_depth], d1 = q[n_depth + 1];
  float cd0 = __builtin_fmaf(c.fd, c1 - c0, c0);
  float hi = __builtin_fmaf(c.fu, __builtin_fmaf(c.fd, d1 - d0, d0) - cd0, cd0);
  return __builtin_fmaf(c.fv, hi - lo, lo);
}

template <bool LOG>
__device__ inline float cell_value_log(const float* __restrict__ L, const Cell& c, int n_depth, int kind,
                                       const LogMap& m) {
  if constexpr (!LOG) {
    return cell_value(L, c, n_depth, kind);
  } else {
    const float* p = L + c.base;
    float a0 = log_apply(m, p[0]), a1 = log_apply(m, p[1]);
    float b0 = log_apply(m, p[n_depth]), b1 = log_apply(m, p[n_depth + 1]);
    float ad = __builtin_fmaf(c.fd, a1 - a0, a0);
    float lo = __builtin_fmaf(c.fu, __builtin_fmaf(c.fd, b1 - b0, b0) - ad, ad);
    if (kind != 1) return lo;
    const float* q = p + int64_t(c.n_u) * n_depth;
    float c0 = log_apply(m, q[0]), c1 = log_apply(m, q[1]);
    float d0 = log_apply(m, q[n_depth]), d1 = log_apply(m, q[n_depth + 1]);
    float cd0 = __builtin_fmaf(c.fd, c1 - c0, c0);
    float hi = __builtin_fmaf(c.fu, __builtin_fmaf(c.fd, d1 - d0, d0) - cd0, cd0);
    return __builtin_fmaf(c.fv, hi - lo, lo);
  }
}

// One lane per output pixel; the cell is computed once and applied to every frame.  Frames go
// in groups of kScanFrames whose corner reads are all issued before any is used (the reads
// are gathers from L2; one frame at a time would leave the lane waiting on each in turn).
// A workgroup covers a 16 x 16 block of pixels (x by rows, a row being one (y, z) of the
// grid), each wave an 8 x 8 quarter of it: neighbouring output rows read neighbouring depths
// of the same lines, so a wave's corner reads fall on a few line segments instead of one
// line per lane, as a row-major wave would have them.
constexpr int kScanFrames = 4;
constexpr int kScanTile = 16;

__device__ inline int64_t scan_pixel(const ScanArgs& a, bool& ok) {
  const int64_t rows = a.grid / a.nx;
  const int64_t tiles_x = (a.nx + kScanTile - 1) / kScanTile;
  const int64_t b = blockIdx.x;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t x = (b % tiles_x) * kScanTile + (w & 1) * 8 + (l & 7);
  const int64_t r = (b / tiles_x) * kScanTile + (w >> 1) * 8 + (l >> 3);
  ok = x < a.nx && r < rows;
  return r * a.nx + x;
}

__host__ inline int64_t scan_blocks(const ScanArgs& a) {
  const int64_t rows = a.grid / a.nx;
  return ((a.nx + kScanTile - 1) / kScanTile) * ((rows + kScanTile - 1) / kScanTile);
}

template <bool LOG>
__global__ __launch_bounds__(kScanThreads) void scan_kernel(const float* __restrict__ in, int n_frames, ScanArgs a,
                                                            const float* __restrict__ frame_ref, float dyn_range_db,
                                                            float* __restrict__ out) {
  bool ok;
  const int64_t p = scan_pixel(a, ok);
  if (!ok) return;
  const Cell c = scan_cell(a, p);
  if (c.base < 0) {
    for (int f = 0; f < n_frames; ++f) out[int64_t(f) * a.grid + p] = a.fill;
    return;
  }
  auto frame_value = [&](int f) {
    LogMap m{};
    if constexpr (LOG) m = log_map(dyn_range_db, frame_ref[f]);
    return cell_value_log<LOG>(in + int64_t(f) * a.frame_in, c, a.n_depth, a.kind, m);
  };
  int f = 0;
  for (; f + kScanFrames <= n_frames; f += kScanFrames) {
    float v[kScanFrames];
#pragma unroll
    for (int u = 0; u < kScanFrames; ++u) v[u] = frame_value(f + u);
#pragma unroll
    for (int u = 0; u < kScanFrames; ++u) out[int64_t(f + u) * a.grid + p] = v[u];
  }
  for (; f < n_frames; ++f) out[int64_t(f) * a.grid + p] = frame_value(f);
}

__global__ void scan_index_kernel(ScanArgs a, int32_t* __restrict__ base) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= a.grid) return;
  base[p] = scan_cell(a, p).base;
}

// ---------------------------------------------------------------- reductions and log map

__global__ void fill_kernel(float* p, int64_t n, float v) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Max of each frame; env >= 0 so the binary32 ordering equals the unsigned-integer ordering
// of the bit patterns and an integer atomic max is exact and order independent.
__global__ void frame_max_kernel(const float* __restrict__ x, int64_t frame_len, int chunks,
                                 unsigned int* __restrict__ fmax) {
  const int f = blockIdx.y;
  const int64_t per = (frame_len + chunks - 1) / chunks;
  const int64_t lo = per * blockIdx.x, hi = min(frame_len, lo + per);
  const float* p = x + int64_t(f) * frame_len;
  float m = 0.0f;
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) m = fmaxf(m, p[i]);
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0 && m > 0.0f) atomicMax(fmax + f, __float_as_uint(m));
}

__global__ void log_kernel(const float* env, int64_t frame_len, const float* __restrict__ frame_ref, float ref,
                           float dyn_range_db, float* out) {
  const int f = blockIdx.y;
  const LogMap m = log_map(dyn_range_db, frame_ref ? frame_ref[f] : ref);
  const float* e = env + int64_t(f) * frame_len;
  float* o = out + int64_t(f) * frame_len;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < frame_len; i += int64_t(gridDim.x) * blockDim.x)
    o[i] = log_apply(m, e[i]);
}

// Max of each frame by one workgroup per frame, written directly (frames of up to 4096 values,
// e.g. the row maxima of a frame): no zero fill and no atomics.
__global__ __launch_bounds__(256) void frame_max_direct_kernel(const float* __restrict__ x, int64_t frame_len,
                                                               float* __restrict__ fmax) {
  __shared__ float red[4];
  const float* p = x + int64_t(blockIdx.x) * frame_len;
  float m = 0.0f;
  for (int64_t i = threadIdx.x; i < frame_len; i += blockDim.x) m = fmaxf(m, p[i]);
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) fmax[blockIdx.x] = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

int frame_max_enqueue(const float* x, int n_frames, int64_t frame_len, float* ws, hipStream_t s) {
  if (frame_len <= 4096) {
    hipLaunchKernelGGL(frame_max_direct_kernel, dim3(n_frames), dim3(256), 0, s, x, frame_len, ws);
    return check_launch("frame_max_direct_kernel");
  }
  hipLaunchKernelGGL(fill_kernel, dim3((n_frames + 255) / 256), dim3(256), 0, s, ws, int64_t(n_frames), 0.0f);
  int chunks = int(std::min<int64_t>((frame_len + 4095) / 4096, 256));
  hipLaunchKernelGGL(frame_max_kernel, dim3(chunks, n_frames), dim3(256), 0, s, x, frame_len, chunks,
                     reinterpret_cast<unsigned int*>(ws));
  return check_launch("frame_max_kernel");
}

int scan_enqueue(const float* in, int n_frames, const ScanArgs& a, const float* frame_ref, float dr_db, bool log,
                 float* out, hipStream_t s) {
  static_assert(kScanThreads == kScanTile * kScanTile, "one lane per pixel of a tile");
  const int64_t blocks = scan_blocks(a);
  if (blocks > 0x7fffffff) return fail(USBF_EUNSUPPORTED, "scan grid too large");
  const dim3 grid(static_cast<unsigned>(blocks));
  if (log)
    hipLaunchKernelGGL(scan_kernel<true>, grid, dim3(kScanThreads), 0, s, in, n_frames, a, frame_ref, dr_db, out);
  else
    hipLaunchKernelGGL(scan_kernel<false>, grid, dim3(kScanThreads), 0, s, in, n_frames, a, frame_ref, dr_db, out);
  return check_launch("scan_kernel");
}

}  // namespace usbf

using namespace usbf;

extern "C" int usbf_log_compress(const float* env, int32_t n_frames, int64_t frame_len, float dyn_range_db, float ref,
                                 float* out, void* ws, size_t ws_bytes, hipStream_t stream) {
  USBF_REQUIRE(env && out, USBF_EINVAL, "null env or out");
  USBF_REQUIRE(n_frames >= 1 && n_frames <= USBF_MAX_FRAMES && frame_len >= 1, USBF_EINVAL, "empty input");
  USBF_REQUIRE(finite_pos(dyn_range_db), USBF_EINVAL, "dyn_range_db must be finite and > 0");
  USBF_REQUIRE(ref == ref, USBF_EINVAL, "ref is NaN");
  const float* fref = nullptr;
  if (!(ref > 0.0f)) {
    size_t need = usbf_workspace_bytes(USBF_OP_LOG_COMPRESS, n_frames, 0, 0);
    USBF_REQUIRE(ws && ws_bytes >= need, USBF_EWORKSPACE, "log compression needs %zu workspace bytes", need);
    int st = frame_max_enqueue(env, n_frames, frame_len, static_cast<float*>(ws), stream);
    if (st) return st;
    fref = static_cast<const float*>(ws);
  }
  const int64_t blocks = std::min<int64_t>((frame_len + 255) / 256, 4096);
  hipLaunchKernelGGL(log_kernel, dim3(unsigned(blocks), n_frames), dim3(256), 0, stream, env, frame_len, fref, ref,
                     dyn_range_db, out);
  return check_launch("log_kernel");
}

extern "C" int usbf_scan_convert(const float* in, int32_t n_frames, const usbf_scan* scan, float* out,
                                 hipStream_t stream) {
  ScanArgs a;
  int st = make_scan_args(scan, &a);
  if (st) return st;
  USBF_REQUIRE(in && out, USBF_EINVAL, "null in or out");
  USBF_REQUIRE(n_frames >= 1 && n_frames <= USBF_MAX_FRAMES, USBF_EINVAL, "n_frames out of range");
  return scan_enqueue(in, n_frames, a, nullptr, 1.0f, false, out, stream);
}

// Reference of each frame for the fused log/scan path: given, or the max of the row maxima,
// or the max of the data.
static int frame_reference(const float* env, const float* row_max, int n_frames, int64_t frame_len,
                           int64_t rows_per_frame, float* ws, hipStream_t s) {
  if (row_max) return frame_max_enqueue(row_max, n_frames, rows_per_frame, ws, s);
  return frame_max_enqueue(env, n_frames, frame_len, ws, s);
}

extern "C" int usbf_log_scan_convert(const float* env, const float* row_max, int32_t n_frames, const usbf_scan* scan,
                                     float dyn_range_db, float ref, float* out, void* ws, size_t ws_bytes,
                                     hipStream_t stream) {
  ScanArgs a;
  int st = make_scan_args(scan, &a);
  if (st) return st;
  USBF_REQUIRE(env && out, USBF_EINVAL, "null env or out");
  USBF_REQUIRE(n_frames >= 1 && n_frames <= USBF_MAX_FRAMES, USBF_EINVAL, "n_frames out of range");
  USBF_REQUIRE(finite_pos(dyn_range_db), USBF_EINVAL, "dyn_range_db must be finite and > 0");
  USBF_REQUIRE(ref == ref, USBF_EINVAL, "ref is NaN");
  size_t need = usbf_workspace_bytes(USBF_OP_LOG_SCAN, n_frames, 0, 0);
  USBF_REQUIRE(ws && ws_bytes >= need, USBF_EWORKSPACE, "log/scan conversion needs %zu workspace bytes", need);
  float* fref = static_cast<float*>(ws);
  if (ref > 0.0f) {
    hipLaunchKernelGGL(fill_kernel, dim3((n_frames + 255) / 256), dim3(256), 0, stream, fref, int64_t(n_frames), ref);
  } else {
    st = frame_reference(env, row_max, n_frames, a.frame_in, int64_t(a.n_u) * a.n_v, fref, stream);
    if (st) return st;
  }
  return scan_enqueue(env, n_frames, a, fref, dyn_range_db, true, out, stream);
}

extern "C" int usbf_scan_index_map(const usbf_scan* scan, int32_t* base, hipStream_t stream) {
  ScanArgs a;
  int st = make_scan_args(scan, &a);
  if (st) return st;
  USBF_REQUIRE(base, USBF_EINVAL, "null base");
  hipLaunchKernelGGL(scan_index_kernel, dim3(unsigned((a.grid + 255) / 256)), dim3(256), 0, stream, a, base);
  return check_launch("scan_index_kernel");
}
