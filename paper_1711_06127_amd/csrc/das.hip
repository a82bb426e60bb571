// Receive beamforming by delay and sum: tile dispatch, the persistent batched kernel and the
// exported delay-index map.  The tile itself is in das_tile.h.
#include "das_tile.h"

namespace usbf {

// Persistent delay-and-sum over a table of items of different sizes (one frame each): every
// workgroup takes work units -- one tile of one item -- from a device counter until the counter
// passes the total, so the grid drains once every unit has been taken.  Units are numbered
// item by item, items ordered as the host chose (most expensive first).
template <bool VEC>
__global__ __launch_bounds__(kDasThreads) void das_persistent_kernel(const BatchItemDev* __restrict__ items,
                                                                     int n_items, int total_units,
                                                                     int* __restrict__ counter) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ int s_unit;
  for (;;) {
    __syncthreads();  // the previous tile is done with LDS and s_unit
    if (threadIdx.x == 0) s_unit = atomicAdd(counter, 1);
    __syncthreads();
    const int u = s_unit;
    if (u >= total_units) break;
    int lo = 0, hi = n_items - 1;  // last item whose first unit is <= u
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (items[mid].unit_begin <= u) lo = mid; else hi = mid - 1;
    }
    const BatchItemDev& it = items[lo];
    const int local = u - it.unit_begin;
    const int group = local / it.ta.n_dtiles, dt = local % it.ta.n_dtiles;
    if (it.G == 4)
      das_tile<VEC, 4, 1, 1>(it.rf, 0, 1, it.a, it.ta, it.out, lds_raw, group, dt);
    else
      das_tile<VEC, 1, 1, 1>(it.rf, 0, 1, it.a, it.ta, it.out, lds_raw, group, dt);
  }
}

__global__ void reset_counter_kernel(int* counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
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
    // the index through the beamformer's own path (fast evaluation with exact fallback),
    // the fraction from the rule itself
    const Tap t = fast_tap(a, b, dtx, E.A, E.B, r, r2, rr);
    const bool act = in_aperture(a, E, r);
    const bool val = t.i0 >= 0 && t.i0 <= a.n_samples - 2;
    i0[idx] = t.i0;
    flags[idx] = uint8_t((act ? 1 : 0) | (val ? 2 : 0));
    if (phi) phi[idx] = delay_tap(a, b, dtx, small_rx_delay(E.A, E.B, r, r2, rr)).phi;
  }
}

template <int G>
static TileArgs single_frame_tiles(const DasArgs& a) {
  using SH = Shape<G, 1>;
  TileArgs ta;
  ta.span = (a.depth_step * SH::TD + kWindowMargin + 3) & ~3;
  ta.ec = std::min(SH::EC, SH::BUFV / ta.span);
  if (ta.ec < 1) {
    ta.ec = 1;
    ta.span = SH::BUFV & ~3;
  }
  ta.pshift = (a.depth_step % 2 == 0) ? 1 : 0;
  ta.n_dtiles = (a.n_depth + SH::TD - 1) / SH::TD;
  return ta;
}

int batch_item_setup(const DasArgs& a, int G, int chunk_div, BatchItemDev* it) {
  USBF_REQUIRE(G == 1 || G == 4, USBF_EUNSUPPORTED, "batched tiles group 1 or 4 lines");
  USBF_REQUIRE(chunk_div >= 1, USBF_EINVAL, "chunk_div must be >= 1");
  it->a = a;
  it->G = G;
  it->ta = G == 4 ? single_frame_tiles<4>(a) : single_frame_tiles<1>(a);
  it->ta.ec = std::max(1, it->ta.ec / chunk_div);
  const int64_t units = int64_t((a.n_lines + G - 1) / G) * it->ta.n_dtiles;
  USBF_REQUIRE(units < (int64_t(1) << 30), USBF_EUNSUPPORTED, "too many tiles");
  it->n_units = int(units);
  return USBF_OK;
}

size_t persistent_lds_bytes(int max_n_el_g1, int max_n_el_g4) {
  size_t b = 0;
  if (max_n_el_g1 > 0) b = std::max(b, tile_lds_bytes<1, 1>(max_n_el_g1));
  if (max_n_el_g4 > 0) b = std::max(b, tile_lds_bytes<4, 1>(max_n_el_g4));
  return b;
}

int launch_persistent(const BatchItemDev* d_items, int n_items, int total_units, int* counter, bool vec, int grid,
                      size_t lds, hipStream_t s) {
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, s, counter);
  if (lds > 65536 && allow_lds(vec ? (const void*)das_persistent_kernel<true> : (const void*)das_persistent_kernel<false>,
                               lds))
    return USBF_EDEVICE;
  if (vec)
    hipLaunchKernelGGL(das_persistent_kernel<true>, dim3(grid), dim3(kDasThreads), lds, s, d_items, n_items,
                       total_units, counter);
  else
    hipLaunchKernelGGL(das_persistent_kernel<false>, dim3(grid), dim3(kDasThreads), lds, s, d_items, n_items,
                       total_units, counter);
  return check_launch("das_persistent_kernel");
}

// Lines per tile: the lines of a transmit come in runs of lines_per_tx (a hint; any mapping is
// beamformed correctly), so tiles of 8, 4 or 2 lines share their staged channel data.  With
// several apodization sets every line takes one slot per set: a tile holds G / n_sets lines
// (G <= 8 slots), and all sets of those lines are summed from the same staged windows.
int beamform_enqueue(const int16_t* rf, int32_t n_frames, const DasArgs& a, float* out, hipStream_t s) {
  const int lpt = a.lines_per_tx;
  int gl = lpt == 8 ? 8 : (lpt >= 4 && lpt % 4 == 0) ? 4 : (lpt >= 2 && lpt % 2 == 0) ? 2 : 1;
  while (gl > 1 && gl * a.n_sets > 8) gl >>= 1;
  if (a.n_sets > 1) {
    switch (gl * a.n_sets) {
      case 8: return launch_das_g<8, true>(rf, n_frames, a, out, s);
      case 4: return launch_das_g<4, true>(rf, n_frames, a, out, s);
      default: return launch_das_g<2, true>(rf, n_frames, a, out, s);
    }
  }
  switch (gl) {
    case 8: return launch_das_g<8, false>(rf, n_frames, a, out, s);
    case 4: return launch_das_g<4, false>(rf, n_frames, a, out, s);
    case 2: return launch_das_g<2, false>(rf, n_frames, a, out, s);
    default: return launch_das_g<1, false>(rf, n_frames, a, out, s);
  }
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

extern "C" int usbf_beamform_sets(const int16_t* rf, int32_t n_frames, const usbf_geometry* geom, const usbf_rx* rx,
                                  int32_t n_sets, const float* f_numbers, const int32_t* windows, float* out,
                                  hipStream_t stream) {
  DasArgs a;
  int st = make_das_args(geom, rx, &a);
  if (st) return st;
  USBF_REQUIRE(rf && out && f_numbers && windows, USBF_EINVAL, "null rf, out, f_numbers or windows");
  USBF_REQUIRE(n_frames >= 1 && n_frames <= USBF_MAX_FRAMES, USBF_EINVAL, "n_frames %d out of range", n_frames);
  USBF_REQUIRE(n_sets == 1 || n_sets == 2 || n_sets == 4, USBF_EUNSUPPORTED, "n_sets must be 1, 2 or 4 (got %d)",
               n_sets);
  for (int k = 0; k < n_sets; ++k) {
    USBF_REQUIRE(finite_pos(f_numbers[k]), USBF_EINVAL, "set %d: f_number must be finite and > 0", k);
    USBF_REQUIRE(windows[k] == USBF_WINDOW_RECT || windows[k] == USBF_WINDOW_HANN, USBF_EINVAL,
                 "set %d: unknown window", k);
    volatile float fn = f_numbers[k];
    a.set_F2[k] = fn + fn;  // the same binary32 operation as for a single set
    a.set_fn[k] = fn;
    a.set_window[k] = windows[k];
  }
  a.n_sets = n_sets;
  a.set_stride = int64_t(n_frames) * a.n_lines * a.n_depth;
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
