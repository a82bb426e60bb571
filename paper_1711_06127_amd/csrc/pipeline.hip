// The whole receive pipeline in one call, in the paper's stage order (Sec. 1 pipeline list):
// delay-and-sum beamforming -> envelope detection -> log compression -> scan conversion.
// Log compression is applied to the four (eight) corner samples inside the scan converter,
// which gives exactly the result of compressing every line sample first.
#include <mutex>

#include "common.h"

namespace usbf {
int beamform_enqueue(const int16_t* rf, int32_t n_frames, const DasArgs& a, float* out, hipStream_t s);
int envelope_enqueue(const float* in, int64_t n_rows, int n, float* env, float* row_max, hipStream_t s);
int frame_max_enqueue(const float* x, int n_frames, int64_t frame_len, float* ws, hipStream_t s);
int validate_scan(const usbf_scan* s);

namespace {

// Validates a B-mode request; on success `a` holds the beamformer's arguments and `need` the
// workspace bytes (beamformed lines, per-row maxima, per-frame maxima).
int bmode_validate(const int16_t* rf, int32_t n_frames, const usbf_geometry* geom, const usbf_rx* rx,
                   const usbf_scan* scan, float dyn_range_db, const float* image, DasArgs* a, size_t* need) {
  int st = make_das_args(geom, rx, a);
  if (st) return st;
  USBF_REQUIRE(rf && image && scan, USBF_EINVAL, "null rf, image or scan");
  USBF_REQUIRE(n_frames >= 1 && n_frames <= USBF_MAX_FRAMES, USBF_EINVAL, "n_frames out of range");
  USBF_REQUIRE(finite_pos(dyn_range_db), USBF_EINVAL, "dyn_range_db must be finite and > 0");
  USBF_REQUIRE(scan->n_depth == rx->n_depth, USBF_ESHAPE, "scan n_depth %d != rx n_depth %d", scan->n_depth,
               rx->n_depth);
  const int64_t scan_lines = int64_t(scan->n_u) * (scan->kind == 1 ? scan->n_v : 1);
  USBF_REQUIRE(scan_lines == geom->n_lines, USBF_ESHAPE, "scan covers %lld lines, geometry has %d",
               (long long)scan_lines, geom->n_lines);
  USBF_REQUIRE(envelope_length_ok(a->n_depth), USBF_EUNSUPPORTED,
               "n_depth %d: not in 8..2048 or a prime factor above 31", a->n_depth);
  st = validate_scan(scan);
  if (st) return st;
  *need = usbf_workspace_bytes(USBF_OP_BMODE, n_frames, a->n_lines, a->n_depth);
  return USBF_OK;
}

// Enqueues the three stages on a validated request; `ws` holds at least the workspace bytes.
int bmode_enqueue(const int16_t* rf, int32_t n_frames, const DasArgs& a, const usbf_scan* scan, float dyn_range_db,
                  float* image, char* ws, hipStream_t stream) {
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  const int64_t rows = int64_t(n_frames) * a.n_lines;
  float* lines = reinterpret_cast<float*>(ws);
  float* row_max = reinterpret_cast<float*>(ws + al(size_t(rows) * a.n_depth * sizeof(float)));
  float* frame_ws = reinterpret_cast<float*>(reinterpret_cast<char*>(row_max) + al(size_t(rows) * sizeof(float)));
  int st = beamform_enqueue(rf, n_frames, a, lines, stream);
  if (st) return st;
  st = envelope_enqueue(lines, rows, a.n_depth, lines, row_max, stream);
  if (st) return st;
  return usbf_log_scan_convert(lines, row_max, n_frames, scan, dyn_range_db, 0.0f, image, frame_ws,
                               al(size_t(n_frames) * sizeof(float)), stream);
}

// Library-owned workspace of usbf_bmode_noalloc: one copy per GPU, held until the process
// ends.  In host code `scratch` names a host-side stand-in, not device memory; its device
// address is looked up per device and kept in g_scratch.
__device__ __align__(256) char scratch[USBF_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of the current device's copy of `scratch` (looked up once per device).
int scratch_for_current_device(char** out) {
  int dev = -1;
  USBF_REQUIRE(hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < kMaxDevices, USBF_EDEVICE,
               "no current HIP device (or device index %d beyond %d)", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    USBF_REQUIRE(e == hipSuccess && p, USBF_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                 hipGetErrorString(e));
    g_scratch[dev] = p;
  }
  *out = static_cast<char*>(g_scratch[dev]);
  return USBF_OK;
}

}  // namespace
}  // namespace usbf

extern "C" int usbf_bmode(const int16_t* rf, int32_t n_frames, const usbf_geometry* geom, const usbf_rx* rx,
                          const usbf_scan* scan, float dyn_range_db, float* image, void* ws, size_t ws_bytes,
                          hipStream_t stream) {
  using namespace usbf;
  DasArgs a;
  size_t need = 0;
  int st = bmode_validate(rf, n_frames, geom, rx, scan, dyn_range_db, image, &a, &need);
  if (st) return st;
  USBF_REQUIRE(ws && ws_bytes >= need, USBF_EWORKSPACE, "bmode needs %zu workspace bytes", need);
  return bmode_enqueue(rf, n_frames, a, scan, dyn_range_db, image, static_cast<char*>(ws), stream);
}

extern "C" int usbf_bmode_noalloc(const int16_t* rf, int32_t n_frames, const usbf_geometry* geom, const usbf_rx* rx,
                                  const usbf_scan* scan, float dyn_range_db, float* image, hipStream_t stream) {
  using namespace usbf;
  DasArgs a;
  size_t need = 0;
  int st = bmode_validate(rf, n_frames, geom, rx, scan, dyn_range_db, image, &a, &need);
  if (st) return st;
  USBF_REQUIRE(need <= size_t(USBF_NOALLOC_SCRATCH_BYTES), USBF_EUNSUPPORTED,
               "bmode needs %zu workspace bytes, the library's scratch holds %zu", need,
               size_t(USBF_NOALLOC_SCRATCH_BYTES));
  char* ws = nullptr;
  st = scratch_for_current_device(&ws);
  if (st) return st;
  return bmode_enqueue(rf, n_frames, a, scan, dyn_range_db, image, ws, stream);
}
