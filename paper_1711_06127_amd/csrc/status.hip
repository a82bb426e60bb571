// Status codes, per-thread error detail, argument packing and workspace sizes.
#include <cstdarg>
#include <cstring>

#include "common.h"

namespace usbf {

static thread_local char g_detail[512] = "";

int fail(int status, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_detail, sizeof(g_detail), fmt, ap);
  va_end(ap);
  return status;
}

int check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(USBF_EDEVICE, "%s: %s", what, hipGetErrorString(e));
  return USBF_OK;
}

int make_das_args(const usbf_geometry* g, const usbf_rx* rx, DasArgs* a) {
  USBF_REQUIRE(g && rx && a, USBF_EINVAL, "null geometry or receive parameters");
  USBF_REQUIRE(g->el_pos && g->tx_origin && g->tx_dir && g->tx_focus && g->line_origin && g->line_dir &&
                   g->line_tx,
               USBF_EINVAL, "null geometry array");
  USBF_REQUIRE(g->n_el >= 1 && g->n_tx >= 1 && g->n_lines >= 1, USBF_ESHAPE,
               "n_el, n_tx, n_lines must be >= 1 (got %d, %d, %d)", g->n_el, g->n_tx, g->n_lines);
  USBF_REQUIRE(g->n_el <= USBF_MAX_ELEMENTS, USBF_EUNSUPPORTED, "n_el %d > %d", g->n_el, USBF_MAX_ELEMENTS);
  USBF_REQUIRE(g->n_lines <= 65535, USBF_EUNSUPPORTED, "n_lines %d > 65535", g->n_lines);
  USBF_REQUIRE(g->array_dims == 1 || g->array_dims == 2, USBF_EINVAL, "array_dims must be 1 or 2");
  USBF_REQUIRE(finite_pos(rx->c) && finite_pos(rx->fs), USBF_EINVAL, "c and fs must be finite and > 0");
  USBF_REQUIRE(rx->t0 == rx->t0 && rx->t0 > -1.0f && rx->t0 < 1.0f, USBF_EINVAL, "t0 out of range");
  USBF_REQUIRE(finite_pos(rx->f_number), USBF_EINVAL, "f_number must be finite and > 0");
  USBF_REQUIRE(rx->window == USBF_WINDOW_RECT || rx->window == USBF_WINDOW_HANN, USBF_EINVAL, "unknown window");
  USBF_REQUIRE(rx->n_samples >= 2, USBF_EINVAL, "n_samples must be >= 2");
  USBF_REQUIRE(rx->depth_start >= 0 && rx->depth_step >= 1 && rx->n_depth >= 1, USBF_EINVAL,
               "depth grid needs depth_start >= 0, depth_step >= 1, n_depth >= 1");
  USBF_REQUIRE((int64_t)rx->depth_start + (int64_t)rx->depth_step * (rx->n_depth - 1) < (1LL << 24),
               USBF_EUNSUPPORTED, "deepest sample index must stay below 2^24");
  a->el_pos = g->el_pos;
  a->tx_origin = g->tx_origin;
  a->tx_dir = g->tx_dir;
  a->tx_focus = g->tx_focus;
  a->line_origin = g->line_origin;
  a->line_dir = g->line_dir;
  a->line_tx = g->line_tx;
  a->n_el = g->n_el;
  a->n_tx = g->n_tx;
  a->n_lines = g->n_lines;
  a->array_dims = g->array_dims;
  USBF_REQUIRE(g->lines_per_tx >= 0, USBF_EINVAL, "lines_per_tx must be >= 0");
  a->lines_per_tx = g->lines_per_tx;
  a->n_samples = rx->n_samples;
  a->depth_start = rx->depth_start;
  a->depth_step = rx->depth_step;
  a->n_depth = rx->n_depth;
  // binary32 constants of the delay rule, one IEEE operation each
  volatile float c = rx->c, fs = rx->fs, t0 = rx->t0, fn = rx->f_number;
  float two_fs = fs + fs;
  a->h = c / two_fs;
  a->K = fs / c;
  a->T0 = fs * t0;
  a->F2 = fn + fn;
  a->f_number = fn;
  a->window = rx->window;
  a->n_sets = 1;
  for (int k = 0; k < kMaxSets; ++k) {
    a->set_F2[k] = a->F2;
    a->set_fn[k] = fn;
    a->set_window[k] = rx->window;
  }
  a->set_stride = 0;
  return USBF_OK;
}

}  // namespace usbf

extern "C" {

const char* usbf_status_string(int s) {
  switch (s) {
    case USBF_OK: return "ok";
    case USBF_EINVAL: return "invalid argument";
    case USBF_ESHAPE: return "inconsistent sizes";
    case USBF_EUNSUPPORTED: return "unsupported";
    case USBF_EWORKSPACE: return "workspace too small";
    case USBF_EDEVICE: return "device error";
    default: return "unknown status";
  }
}

const char* usbf_last_error_detail(void) { return usbf::g_detail; }

const char* usbf_version(void) { return "usbf 0.1 gfx950"; }

size_t usbf_workspace_bytes(int32_t op, int64_t n_frames, int64_t n_lines, int64_t n_depth) {
  if (n_frames < 0 || n_lines < 0 || n_depth < 0) return 0;
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  switch (op) {
    case USBF_OP_LOG_COMPRESS:
    case USBF_OP_LOG_SCAN:
      return al(size_t(n_frames) * sizeof(float));
    case USBF_OP_BMODE:
      // beamformed/envelope lines, per-row maxima, per-frame maxima
      return al(size_t(n_frames) * n_lines * n_depth * sizeof(float)) + al(size_t(n_frames) * n_lines * sizeof(float)) +
             al(size_t(n_frames) * sizeof(float));
    case USBF_OP_APODNET:
      return usbf::net_ws_bytes(n_frames, n_lines, false);
    case USBF_OP_APODNET_TRAIN:
      return usbf::net_ws_bytes(n_frames, n_lines, true);
    default:
      return 0;
  }
}

}  // extern "C"
