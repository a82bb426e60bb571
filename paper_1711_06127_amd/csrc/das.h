// Delay-and-sum tiling shared by the per-call kernels and the persistent batched kernel.
#pragma once

#include "common.h"

namespace usbf {

struct TileArgs {
  int span;      // staged samples per element (multiple of 4)
  int ec;        // elements per chunk
  int n_dtiles;  // depth tiles per line
  int pshift;    // 1: windows split into even and odd samples (even depth_step), else 0
};

// One item of a persistent batch: a single frame (or volume) with its own geometry.
struct BatchItemDev {
  const int16_t* rf;  // [n_tx][n_el][n_samples]
  float* out;         // [n_lines][n_depth]
  DasArgs a;
  TileArgs ta;
  int G;              // lines per tile: 4 (lines grouped by transmit) or 1
  int unit_begin;     // first work unit of the item
  int n_units;        // (lines / G) * depth tiles
};

// Fills the tiling of an item for tiles of G lines (G = 1 or 4), one frame per block, with
// the tile's largest element chunk divided by chunk_div.
int batch_item_setup(const DasArgs& a, int G, int chunk_div, BatchItemDev* it);
// LDS bytes the persistent kernel needs for 1-line tiles of up to max_n_el_g1 elements and
// 4-line tiles of up to max_n_el_g4 elements (0: no such tiles).
size_t persistent_lds_bytes(int max_n_el_g1, int max_n_el_g4);
int launch_persistent(const BatchItemDev* d_items, int n_items, int total_units, int* counter, bool vec, int grid,
                      size_t lds, hipStream_t s);

}  // namespace usbf
