// Internal helpers shared by the library's translation units: status handling,
// argument checks and launch utilities.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/usbf.h"

namespace usbf {

// Records why the calling thread's last call failed; returns `status`.
int fail(int status, const char* fmt, ...);
// Checks the last launch on this thread; USBF_EDEVICE with the HIP message on error.
int check_launch(const char* what);

#define USBF_REQUIRE(cond, status, ...)       \
  do {                                        \
    if (!(cond)) return ::usbf::fail((status), __VA_ARGS__); \
  } while (0)

inline bool finite_pos(float v) { return v > 0.0f && v < 3.0e38f; }

// Number of workgroups dispatched round-robin over the MI355X's accelerator dies (XCDs).
constexpr int kNumXcd = 8;

// Remaps a linear workgroup id so that consecutive logical tiles run on the same XCD
// (each XCD has its own L2): hardware dispatches id i to XCD i % 8.
__device__ inline uint32_t xcd_swizzle(uint32_t bid, uint32_t nblocks) {
  uint32_t per = nblocks / kNumXcd;
  uint32_t rem = nblocks % kNumXcd;
  uint32_t xcd = bid % kNumXcd;
  uint32_t idx = bid / kNumXcd;
  // XCDs [0, rem) own per+1 logical tiles, the rest own per
  uint32_t start = xcd * per + (xcd < rem ? xcd : rem);
  return start + idx;
}

// Geometry in kernel-argument form (device pointers, sizes) plus the binary32 constants of
// the delay rule, computed once on the host with the same IEEE operations the rule names.
constexpr int kMaxSets = 4;

struct DasArgs {
  const float* el_pos;
  const float* tx_origin;
  const float* tx_dir;
  const float* tx_focus;
  const float* line_origin;
  const float* line_dir;
  const int32_t* line_tx;
  int32_t n_el, n_tx, n_lines, array_dims, lines_per_tx;
  int32_t n_samples, depth_start, depth_step, n_depth;
  float h, K, T0, F2, f_number;
  int32_t window;
  // apodization parameter sets beamformed together from one staging of the channel data: tile
  // slot s / (G / n_sets) uses set s; set 0 is (f_number, window) above.  Output of set s
  // starts set_stride floats after that of set 0.
  int32_t n_sets;
  float set_F2[kMaxSets], set_fn[kMaxSets];
  int32_t set_window[kMaxSets];
  int64_t set_stride;
};

int make_das_args(const usbf_geometry* g, const usbf_rx* rx, DasArgs* a);

// envelope lengths the FFT supports: 8 <= n <= 2048, every prime factor <= 31
bool envelope_length_ok(int n);

// workspace of the learned-apodization network for n_pix pixels of M elements
size_t net_ws_bytes(int64_t n_pix, int64_t M, bool train);

}  // namespace usbf
