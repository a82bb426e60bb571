// Receive beamforming by delay and sum (Sec. 1 pipeline list, "receive beamforming";
// Sec. 2 method list items 1-2): the tile shared by the per-call kernels and the persistent
// batched kernel, and the per-call launchers.
//
// Work decomposition.  A workgroup of 256 lanes owns a tile of G consecutive scanlines that
// share one transmit (multi-line acquisition) times 256/G consecutive depth samples, one lane
// per output sample, for a block of FB frames.  Elements are processed in chunks of up to 8:
//   1. every lane evaluates the binary32 delay rule for its pixel and the chunk's elements
//      once and keeps (LDS offset, (1-phi) w, phi w) in registers -- the delay arithmetic is
//      thus shared by all FB frames;
//   2. for each stage of FS frames the workgroup copies, with wide coalesced loads, the part
//      of each element's int16 trace that the tile can touch (its window, known from the
//      delays at the tile's first and last depth because the delay grows with depth) into
//      LDS as binary32, frames innermost;
//   3. every lane reads the two neighbouring samples of all FS frames with two 16-byte LDS
//      reads and accumulates with two FMAs per frame.
// A (pixel, element) pair whose samples fall outside the staged window (only for unusual
// geometry) reads global memory directly, so the result never depends on the tiling.
#pragma once

#include <climits>
#include <type_traits>

#include "common.h"
#include "das.h"
#include "tof.h"

namespace usbf {

constexpr int kDasThreads = 256;
// Tile tunables (compile-time; the defaults are the fastest measured on gfx950): the bytes of
// one staging buffer (two per workgroup) for multi-line tiles, single-line multi-frame tiles
// and single-frame tiles, and the most elements per chunk.
#ifndef USBF_DAS_BUF_MULTI
#define USBF_DAS_BUF_MULTI 16384
#endif
#ifndef USBF_DAS_BUF_SINGLE
#define USBF_DAS_BUF_SINGLE 78336
#endif
#ifndef USBF_DAS_BUF_FRAME
#define USBF_DAS_BUF_FRAME 5448
#endif
#ifndef USBF_DAS_MAX_CHUNK
#define USBF_DAS_MAX_CHUNK 12
#endif
constexpr int kMaxChunk = USBF_DAS_MAX_CHUNK;
#ifndef USBF_DAS_WINDOW_MARGIN
#define USBF_DAS_WINDOW_MARGIN 32
#endif
constexpr int kWindowMargin = USBF_DAS_WINDOW_MARGIN;  // samples beyond 2 * depths per line in a window
constexpr int kMaxTileLds = 160 * 1024;  // LDS a workgroup may use on gfx950

__host__ __device__ constexpr int buffer_bytes(int G, int FS) {
  return G > 1 ? USBF_DAS_BUF_MULTI : (FS > 1 ? USBF_DAS_BUF_SINGLE : USBF_DAS_BUF_FRAME);
}
__host__ __device__ constexpr int max_chunk(int FS) { return FS > 1 ? kMaxChunk : (kMaxChunk < 8 ? kMaxChunk : 8); }

template <int FS>
struct FVec;
template <>
struct FVec<1> {
  using T = float;
  __device__ static float get(const T& v, int) { return v; }
  __device__ static void set(T& v, int, float x) { v = x; }
};
template <>
struct FVec<2> {
  using T = float2;
  __device__ static float get(const T& v, int f) { return f == 0 ? v.x : v.y; }
  __device__ static void set(T& v, int f, float x) { (f == 0 ? v.x : v.y) = x; }
};
template <>
struct FVec<4> {
  using T = float4;
  __device__ static float get(const T& v, int f) { return f == 0 ? v.x : f == 1 ? v.y : f == 2 ? v.z : v.w; }
  __device__ static void set(T& v, int f, float x) { (f == 0 ? v.x : f == 1 ? v.y : f == 2 ? v.z : v.w) = x; }
};

// Element type of a staged window: single-frame windows keep the int16 samples as they are
// (the sum converts its two taps), multi-frame windows hold binary32 vectors of FS frames.
template <int FS>
struct WinT {
  using T = typename FVec<FS>::T;
};
template <>
struct WinT<1> {
  using T = int16_t;
};

// Compile-time shape of a tile: G lines x TD depths; a window of SPAN samples per element for
// depth_step <= 2; EC elements per chunk so that one staging buffer fits buffer_bytes(G, FS); IPT
// staging items (4 samples x FS frames) per lane.
template <int G, int FS>
struct Shape {
  static constexpr int TD = kDasThreads / G;
  static constexpr int SPAN = 2 * TD + kWindowMargin;
  static constexpr int EC0 = buffer_bytes(G, FS) / (SPAN * int(sizeof(typename WinT<FS>::T)));
  static constexpr int EC = EC0 < max_chunk(FS) ? (EC0 < 1 ? 1 : EC0) : max_chunk(FS);
  static constexpr int BUFV = EC * SPAN;  // staging buffer length in window elements
  // buffer pitch: each buffer ends in two zero vectors (four zero samples for int16 windows,
  // which keeps the second buffer 8-byte aligned)
  static constexpr int BSTRIDE = BUFV + (FS == 1 ? 4 : 2);
  static constexpr int IPT = (EC * (SPAN / 4) + kDasThreads - 1) / kDasThreads;
};

// Tiles of one line (3D volumes, single-line frames): everything about an element except the
// depth is the same for all lanes.  For each chunk the workgroup tabulates those constants once
// per element, next to the chunk's staging buffer, and the lanes read them with two broadcast
// LDS reads per element instead of re-deriving them per pixel.  (The code handles any tile
// whose waves each cover one line, G <= 4; for the multi-line multi-frame tiles, whose taps
// serve up to 32 frames, the extra registers of the table path cost more than it saves.)
template <int G, int FS, bool SETS = false>
__host__ __device__ constexpr bool line_per_wave() {
  return G == 1 && !SETS;
}
// The one-line single-frame tile (3D volumes; many elements, little reuse) keeps no
// per-element geometry tables in LDS: the lanes that tabulate a chunk load the positions from
// the geometry arrays a chunk ahead.
template <int G, int FS>
__host__ __device__ constexpr bool geo_from_global() {
  return G == 1 && FS == 1;
}

struct alignas(16) ChunkTap {
  float A, B;  // receive constants of the line (ElemGeom)
  float dx;    // lateral x offset (Hann factor)
  float dy;    // lateral y offset
  float thr;   // F2 times the lateral offset the aperture tests: inside iff thr <= r
  int base;    // taps i0 in [lo, lo + n) are summed from the staged window (n = 0 when nothing
  int lo;      // is staged); base is the byte offset of tap lo in the buffer for int16 windows
  int n;       // (FS = 1), the window's first sample for FS > 1
};

// after a chunk's table: its elements' lateral y offsets if there are at most two of them
struct alignas(16) ChunkHdr {
  float dyA, dyB;
  int two;  // every element's y offset is dyA or dyB
  int one;  // every element's y offset is dyA
};
static_assert(sizeof(ChunkHdr) <= sizeof(ChunkTap), "the header takes one table entry");

// LDS of one workgroup: two staging buffers, the per-(line, element) receive constants of the
// G lines, their LineGeom, and per element the tap window [lo, hi] and flags.
// A staged window holds the samples of one element for FS frames; with pshift = 1 (and FS > 1:
// single-frame windows are read 4 bytes per lane, where the split does not pay) it is split
// into even and odd samples, sample i at index (i & 1) * span/2 + half_slot(i / 2): lanes on
// consecutive depths read taps depth_step = 2 samples apart, so their reads are consecutive in
// LDS.  half_slot swaps the two vectors of every other pair of quads (index m ^ bit 3 of m):
// a staging item writes indices 2q and 2q + 1 of each half for its quad q, and on gfx950
// 16-byte LDS writes are served 8 lanes at a time from 32 banks, so without the swap the 8
// lanes of a pass would write 4 distinct bank groups twice; reads are unaffected.
template <int G, int FS>
struct TileLds {
  typename WinT<FS>::T* win;  // [2][BSTRIDE]: window data, then all-zero vectors
  ChunkTap* ctab;             // [2][G][EC + 1], line_per_wave tiles only: element constants of each
                              // buffer's chunk for each line, then the line's header (ChunkHdr)
  float2* geo;                // [G][n_el]: (A, B) of the receive path
  float2* exy;                // [n_el]: element x, y (lateral offsets are taken from the lines)
  LineGeom* lines;            // [G]
  int4* wnd;                  // [n_el]: (lo | flags, hi, flo, fn); lo a multiple of 4, flags bit 0
                              // needed, bit 1 staged; hi the last sample to stage (INT_MIN when
                              // none is); taps i0 in [flo, flo + fn) are summed from the staged
                              // window (inside the record, the window and its span)
  int* flg;                   // [(n_el + 3) / 4]: the flags, a byte per element, while they are
                              // built; then a byte per chunk: some element of it is needed
};

// two staging buffers, each followed by two all-zero frame vectors (kept zero for the whole
// kernel): taps that contribute nothing read them, at the same offset in either buffer, so the
// accumulation needs neither a branch nor a per-buffer select (and an unsplit window's two
// neighbouring samples are always read from consecutive vectors)
template <int G, int FS>
__host__ __device__ constexpr size_t window_bytes() {
  return 2 * size_t(Shape<G, FS>::BSTRIDE) * sizeof(typename WinT<FS>::T);
}

template <int G, int FS, bool SETS>
__host__ __device__ constexpr size_t ctab_bytes() {
  return line_per_wave<G, FS, SETS>() ? 2 * size_t(G) * (Shape<G, FS>::EC + 1) * sizeof(ChunkTap) : 0;
}

// per-(line, element) receive constants and element positions (geo_from_global tiles derive
// them from the geometry arrays when they tabulate a chunk instead)
template <int G, int FS>
__host__ __device__ constexpr size_t geo_entries(int n_el) {
  return geo_from_global<G, FS>() ? 0 : size_t(G + 1) * n_el;
}

template <int G, int FS, bool SETS = false>
__host__ __device__ inline size_t tile_lds_bytes(int n_el) {
  return window_bytes<G, FS>() + ctab_bytes<G, FS, SETS>() + geo_entries<G, FS>(n_el) * sizeof(float2) +
         G * sizeof(LineGeom) + size_t(n_el) * sizeof(int4) + size_t((n_el + 3) / 4) * sizeof(int);
}

template <int G, int FS, bool SETS = false>
__device__ inline TileLds<G, FS> carve(unsigned char* base, int n_el) {
  static_assert(window_bytes<G, FS>() % 16 == 0, "the tap table after the buffers needs 16-byte alignment");
  TileLds<G, FS> t;
  t.win = reinterpret_cast<typename WinT<FS>::T*>(base);
  t.ctab = reinterpret_cast<ChunkTap*>(base + window_bytes<G, FS>());
  t.geo = reinterpret_cast<float2*>(base + window_bytes<G, FS>() + ctab_bytes<G, FS, SETS>());
  t.exy = t.geo + size_t(G) * n_el;  // (neither table exists when geo_from_global)
  t.lines = reinterpret_cast<LineGeom*>(t.geo + geo_entries<G, FS>(n_el));
  t.wnd = reinterpret_cast<int4*>(t.lines + G);
  t.flg = reinterpret_cast<int*>(t.wnd + n_el);
  return t;
}

__device__ inline int32_t rule_tap(const DasArgs& a, const LineGeom& L, const float2& E, int j) {
  const int32_t b = a.depth_start + a.depth_step * j;
  const float r = (float)b * a.h;
  return fast_tap(a, b, small_tx_delay(L, r), E.x, E.y, r, r + r, r * r).i0;
}

// apodization set s of a tile slot (selects: an indexed read of the kernel-argument arrays would
// go through scratch memory)
__device__ inline void set_params(const DasArgs& a, int s, LineGeom& L) {
  L.F2 = s == 0 ? a.set_F2[0] : s == 1 ? a.set_F2[1] : s == 2 ? a.set_F2[2] : a.set_F2[3];
  L.fn = s == 0 ? a.set_fn[0] : s == 1 ? a.set_fn[1] : s == 2 ? a.set_fn[2] : a.set_fn[3];
  L.window = s == 0 ? a.set_window[0] : s == 1 ? a.set_window[1] : s == 2 ? a.set_window[2] : a.set_window[3];
}

// index within one half of a split window (see TileLds)
__host__ __device__ constexpr int half_slot(int m) { return m ^ ((m >> 3) & 1); }

__device__ inline float lo16(uint32_t d) { return float(int16_t(d & 0xffffu)); }
__device__ inline float hi16(uint32_t d) { return float(int16_t(d >> 16)); }

// One staging item: four consecutive samples of one element's window.  `voff` is the byte
// offset of the first sample within the transmit's block of a frame (clamped into the
// record); `dst` the window-relative LDS index of the first sample, bit 30 set when a split
// window swaps the quad's vectors (half_slot); dst < 0: nothing to stage.
// Window samples outside the record are staged as whatever the clamped load returns: a tap is
// summed from the window only when both of its samples lie inside the record, so they are
// never read.

template <int IPT>
struct Items {
  uint32_t voff[IPT];
  int dst[IPT];
};

// The lane's staging items of a chunk: item threadIdx.x + it * kDasThreads is quad q of the
// chunk's element k; the decomposition depends only on the lane and the window length, so it
// is computed once per tile.
template <int IPT>
struct ItemSlots {
  int k[IPT];      // element of the chunk
  int q4[IPT];     // first sample of the quad within the window
  int kS[IPT];     // k * n_samples: the element's record relative to the chunk's first
  int dst[IPT];    // window-relative LDS index of the quad's first sample (bit 30: vectors swapped)
};

template <int IPT, int FS>
__device__ inline ItemSlots<IPT> item_slots(const TileArgs& ta, int S) {
  ItemSlots<IPT> s;
  const int quads = ta.span >> 2;
#pragma unroll
  for (int it = 0; it < IPT; ++it) {
    const int item = threadIdx.x + it * kDasThreads;
    const int k = item / quads, q = item - k * quads;
    s.k[it] = k;
    s.q4[it] = 4 * q;
    s.kS[it] = k * S;
    // split windows: bit 30 says the quad's two vectors per half are swapped (half_slot)
    s.dst[it] = (FS > 1 && ta.pshift) ? (k * ta.span + 2 * q) | (((q >> 2) & 1) << 30) : k * ta.span + 4 * q;
  }
  return s;
}

template <bool VEC, int G, int FS, int IPT>
__device__ inline Items<IPT> chunk_items(const TileLds<G, FS>& t, const TileArgs& ta, const DasArgs& a,
                                         const ItemSlots<IPT>& sl, int c) {
  Items<IPT> d;
  const int e0 = c * ta.ec;
  const int ec = min(ta.ec, a.n_el - e0);
  const int S = a.n_samples;
  const int e0S = e0 * S;
#pragma unroll
  for (int it = 0; it < IPT; ++it) {
    const int k = sl.k[it];
    const bool ok = (c >= 0) & (k < ec);
    // the window's start and its last needed sample (INT_MIN when nothing is staged)
    const int2 wd = *reinterpret_cast<const int2*>(&t.wnd[ok ? e0 + k : 0]);
    const int i = (wd.x & ~3) + sl.q4[it];
    const bool take = ok & (i <= wd.y);
    // A quad with no sample inside the record loads the record's first samples instead:
    // windows reach past either end of the record for deep pixels at the edge of the aperture.
    // Window starts are multiples of 4, so a quad that starts before the record lies wholly
    // before it; a quad that reaches past the end starts inside it (i < S), and its samples
    // beyond the end are clamped in issue_stage (VEC: S % 4 == 0, the quad is wholly inside).
    // Every load therefore stays inside element e's record.
    const int ic = uint32_t(i) < uint32_t(S) ? i : 0;
    d.voff[it] = take ? uint32_t(e0S + sl.kS[it] + ic) * uint32_t(sizeof(int16_t)) : 0u;
    d.dst[it] = take ? sl.dst[it] : -1;
  }
  return d;
}

template <bool VEC, int FS, int IPT>
struct Prefetch {
  uint2 d[IPT][FS];
};

// Buffer resource over `base` (gfx9 raw buffer, no range clamping: every offset used is
// inside the channel data -- chunk_items clamps each staging item into its element's record).
__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, int(0xffffffffu), 0x00020000);
}

// Global loads of one staging step: frames fr .. fr+FS-1 of the transmit block `rsrc` starts
// at, `fbytes` bytes apart.  Each load is a buffer load with the lane's offset in a VGPR and
// the frame's offset in an SGPR, so addressing costs no vector instructions.
template <bool VEC, int FS, int IPT>
__device__ inline void issue_stage(Prefetch<VEC, FS, IPT>& pf, const Items<IPT>& it_, __amdgpu_buffer_rsrc_t rsrc,
                                   uint32_t fr_off, uint32_t fbytes, int S) {
#pragma unroll
  for (int it = 0; it < IPT; ++it) {
#pragma unroll
    for (int f = 0; f < FS; ++f) {
      const uint32_t so = fr_off + uint32_t(f) * fbytes;
      if constexpr (VEC) {
        pf.d[it][f] = __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(rsrc, it_.voff[it], so, 0));
      } else {
        // samples one by one, each clamped into the record
        const int i = int((it_.voff[it] / sizeof(int16_t)) % uint32_t(S));
        uint32_t h[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const uint32_t o = it_.voff[it] + uint32_t((i + s < S) ? s : 0) * 2u;
          h[s] = __builtin_amdgcn_raw_buffer_load_b16(rsrc, o, so, 0);
        }
        pf.d[it][f] = make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
      }
    }
  }
}

template <bool VEC, int G, int FS, int IPT>
__device__ inline void store_stage(const Prefetch<VEC, FS, IPT>& pf, const Items<IPT>& it_,
                                   typename WinT<FS>::T* win, int span, int pshift) {
  using V = typename FVec<FS>::T;
  const int half = span >> 1;
#pragma unroll
  for (int it = 0; it < IPT; ++it) {
    const int dst = it_.dst[it];
    if (dst < 0) continue;
    if constexpr (FS == 1) {
      // int16 window: the four samples as loaded
      *reinterpret_cast<uint2*>(win + dst) = pf.d[it][0];
    } else {
      V x[4];
#pragma unroll
      for (int f = 0; f < FS; ++f) {
        const uint32_t dx = pf.d[it][f].x, dy = pf.d[it][f].y;
        FVec<FS>::set(x[0], f, lo16(dx));
        FVec<FS>::set(x[1], f, hi16(dx));
        FVec<FS>::set(x[2], f, lo16(dy));
        FVec<FS>::set(x[3], f, hi16(dy));
      }
      V* w = win + (dst & 0x3fffffff);
      if (pshift) {
        // samples 4q and 4q + 2 go to half indices 2q and 2q + 1, swapped when bit 2 of q is
        // set (half_slot)
        const int f = dst >> 30;
        w[f] = x[0];
        w[1 - f] = x[2];
        w[half + f] = x[1];
        w[half + 1 - f] = x[3];
      } else {
        w[0] = x[0];
        w[1] = x[1];
        w[2] = x[2];
        w[3] = x[3];
      }
    }
  }
}

// f(integral_constant<int, 0>) ... f(integral_constant<int, N - 1>)
template <int N, int I = 0, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<N, I + 1>(f);
  }
}

// Delay-and-sum of one tile -- lines [group G, group G + G) x depths [dt TD, dt TD + TD) --
// for frames [frame0, frame0 + n_blocks * FB) of the batch.  Every lane of the workgroup
// calls it with the same tile.  SETS: the G slots hold G / n_sets lines x n_sets apodization
// sets, each slot with its own f-number and window (per-lane values); otherwise all slots
// take the call's single set from the kernel arguments (wave-uniform scalars).
template <bool VEC, int G, int FB, int FS, bool SETS = false>
__device__ __forceinline__ void das_tile(const int16_t* __restrict__ rf, int frame0, int n_blocks, const DasArgs& a,
                                         const TileArgs& ta, float* __restrict__ out, unsigned char* lds_raw,
                                         int group, int dt) {
  using V = typename FVec<FS>::T;
  using W = typename WinT<FS>::T;
  using SH = Shape<G, FS>;
  constexpr int TD = SH::TD;
  constexpr int NS = FB / FS;
  constexpr int IPT = SH::IPT;
  const TileLds<G, FS> t = carve<G, FS, SETS>(lds_raw, a.n_el);

  const int tid = threadIdx.x;
  // slot g of the tile: line l0 + g % gl with apodization set g / gl (gl = G with one set)
  const int g = tid / TD;
  const int gl = SETS ? G / a.n_sets : G;
  const int l0 = group * gl;
  const int l = SETS ? l0 + g % gl : l0 + g;
  const int set = SETS ? g / gl : 0;
  const int j = dt * TD + tid % TD;
  const int j_first = dt * TD;
  const int j_last = min(a.n_depth, j_first + TD) - 1;
  const bool line_ok = l < a.n_lines;
  const bool pix_ok = line_ok && j < a.n_depth;
  const int S = a.n_samples;
  const int t0 = a.line_tx[l0];
  const int t_grp = (t0 >= 0 && t0 < a.n_tx) ? t0 : -1;

  // ---- prologue: line constants, per-(line, element) receive constants, tap windows
  constexpr int ZERO = SH::BUFV;  // index of a buffer's zero vector
  if (tid < G) {
    line_geom(a, min(l0 + tid % gl, a.n_lines - 1), t.lines[tid]);
    if (SETS) set_params(a, tid / gl, t.lines[tid]);
  }
  if (tid == 0) {
    using W = typename WinT<FS>::T;
    W z;
    if constexpr (FS == 1) {
      z = 0;
    } else {
#pragma unroll
      for (int f = 0; f < FS; ++f) FVec<FS>::set(z, f, 0.0f);
    }
    for (int b = 0; b < 2; ++b)
      for (int k = ZERO; k < SH::BSTRIDE; ++k) t.win[b * SH::BSTRIDE + k] = z;
  }
  for (int e = tid; e < a.n_el; e += kDasThreads) {
    t.wnd[e] = make_int4(INT_MAX, INT_MIN, 0, 0);
    if constexpr (!geo_from_global<G, FS>()) t.exy[e] = make_float2(a.el_pos[3 * e], a.el_pos[3 * e + 1]);
  }
  for (int e = tid; e < (a.n_el + 3) / 4; e += kDasThreads) t.flg[e] = 0;
  __syncthreads();
  {
    const float r_last = (float)(a.depth_start + a.depth_step * j_last) * a.h;
    for (int idx = tid; idx < a.n_el * G; idx += kDasThreads) {
      const int gg = idx / a.n_el, e = idx - gg * a.n_el;
      const LineGeom& Lg = t.lines[gg];
      const ElemGeom E = elem_geom(a, Lg, e);
      const float2 E2 = make_float2(E.A, E.B);
      if constexpr (!geo_from_global<G, FS>()) t.geo[gg * a.n_el + e] = E2;
      if (l0 + gg % gl >= a.n_lines || Lg.tx < 0) continue;
      if (!in_aperture(SETS ? Lg.F2 : a.F2, a.array_dims, E, r_last)) continue;
      const int shift = 8 * (e & 3);
      if (Lg.tx != t_grp) {
        atomicOr(&t.flg[e >> 2], 1 << shift);
        continue;
      }
      atomicMin(&t.wnd[e].x, rule_tap(a, Lg, E2, j_first));
      atomicMax(&t.wnd[e].y, rule_tap(a, Lg, E2, j_last) + 1);
      atomicOr(&t.flg[e >> 2], 3 << shift);
    }
  }
  __syncthreads();
  // window start aligned down to 4 samples, flags folded into its two low bits; the taps summed
  // from the window: inside the record (both samples), at or after its start, with the next
  // sample staged and inside the buffer's span
  for (int e = tid; e < a.n_el; e += kDasThreads) {
    const int f = (t.flg[e >> 2] >> (8 * (e & 3))) & 3;
    const int hi = t.wnd[e].y;
    int lo4 = 0, flo = 0, fn = 0;
    if (f & 2) {
      const int lo = t.wnd[e].x;
      lo4 = lo >= 0 ? (lo & ~3) : -((-lo + 3) & ~3);
      if (hi - lo4 + 1 > ta.span) {  // wider than the buffer: keep the deep end
        lo4 = hi + 1 - ta.span;
        lo4 = lo4 >= 0 ? ((lo4 + 3) & ~3) : -((-lo4) & ~3);
      }
      flo = max(lo4, 0);
      const int fhi = min(min(hi - 1, lo4 + ta.span - 2), S - 2);
      fn = fhi >= flo ? fhi - flo + 1 : 0;
    }
    t.wnd[e] = make_int4(lo4 | f, (f & 2) ? hi : INT_MIN, flo, fn);
  }
  __syncthreads();
  // a byte per chunk, in the flags' space: does any of its elements need beamforming
  const int n_chunks = (a.n_el + ta.ec - 1) / ta.ec;
  uint8_t* const cneed = reinterpret_cast<uint8_t*>(t.flg);
  for (int c = tid; c < n_chunks; c += kDasThreads) {
    int any = 0;
    for (int k = 0; k < ta.ec && c * ta.ec + k < a.n_el; ++k) any |= t.wnd[c * ta.ec + k].x & 3;
    cneed[c] = any != 0;
  }
  __syncthreads();

  // ---- this lane's pixel
  const LineGeom& L = t.lines[g];
  const bool on_grp = line_ok && L.tx >= 0 && L.tx == t_grp;
  const bool lane_ok = pix_ok && L.tx >= 0;
  const int32_t b = a.depth_start + a.depth_step * j;
  const float r = (float)b * a.h;
  const float r2 = r + r;
  const float rr = r * r;
  const float dtx = small_tx_delay(L, r);
  // apodization of this lane's slot
  const float ap_F2 = SETS ? L.F2 : a.F2;
  const int ap_window = SETS ? L.window : a.window;
  const float inv_w = r > 0.0f ? (SETS ? L.fn : a.f_number) / r : 0.0f;
  const size_t tx_block = size_t(a.n_el) * S;              // samples per transmit
  const size_t frame_stride = size_t(a.n_tx) * tx_block;   // samples per frame
  const int16_t* grp_block = rf + size_t(t_grp < 0 ? 0 : t_grp) * tx_block;
  const int16_t* own_block = rf + size_t(L.tx < 0 ? 0 : L.tx) * tx_block;
  const float2* geo = t.geo + g * a.n_el;
  const int half = ta.span >> 1;

  auto next_chunk = [&](int c) {
    for (++c; c < n_chunks; ++c)
      if (cneed[c]) return c;
    return n_chunks;
  };
  const uint32_t fbytes = uint32_t(std::min<uint64_t>(frame_stride * sizeof(int16_t), 0xffffffffull));

  // Channel-data steps -- one FS-frame stage of one chunk -- run in order q = 0, 1, ...  Step q
  // is summed from LDS buffer q & 1 while the loads of step q + 2 are in flight into register
  // set q & 1 (which step q's data left at the end of step q - 1); at the end of step q the
  // data of step q + 1 (register set (q + 1) & 1) is converted into LDS buffer (q + 1) & 1.
  // Two steps of loads are thus in flight behind every sum.  With an even number of stages
  // per chunk the parities follow the stage index; with one stage per chunk they follow the
  // chunk ordinal, and the chunk loop is unrolled by two so that they stay compile-time.
  static_assert(NS == 1 || NS % 2 == 0, "stages per chunk must be 1 or even");
  Prefetch<VEC, FS, IPT> pf[2];
  const bool stage_any = t_grp >= 0;
  const ItemSlots<IPT> slots = item_slots<IPT, FS>(ta, S);

  // the last y offset whose Hann factor was computed, and that factor (separable windows)
  float hy_dy = __builtin_nanf(""), hy = 0.0f;
  struct Taps {
    int off0[SH::EC], off1[SH::EC];
    float w0[SH::EC], w1[SH::EC];
    float scale;  // line_per_wave tiles: a factor common to the chunk's weights
    uint32_t slow;
  };
  // taps of this lane's pixel for chunk c, shared by every frame; a tap that contributes
  // nothing, or whose samples are not staged, reads the zero vector
  constexpr bool UNI = line_per_wave<G, FS, SETS>();
  constexpr bool GEO_G = geo_from_global<G, FS>();
  constexpr int EC1 = SH::EC + 1;  // table entries per (buffer, line): the chunk's, then a header
  // line_per_wave tiles: tabulate the constants of chunk c's elements for every line of the tile
  // into table buffer tb, and in each line's header the chunk's lateral y offsets when there are
  // at most two of them (a chunk of a matrix array spans at most two rows).  Lanes
  // 0 .. G EC - 1 (all in the first wave) take one (line, element) each; the expressions are
  // those of the general path below, so the decisions are the same.  With GEO_G the positions
  // come from `ep`, loaded a chunk earlier (load_ep), otherwise from the LDS tables.
  auto load_ep = [&](int c) {
    float3 ep = make_float3(0.0f, 0.0f, 0.0f);
    const int e = c * ta.ec + tid;
    if (tid < SH::EC && c >= 0 && c < n_chunks && tid < ta.ec && e < a.n_el)
      ep = make_float3(a.el_pos[3 * e], a.el_pos[3 * e + 1], a.el_pos[3 * e + 2]);
    return ep;
  };
  auto fill_ctab = [&](int c, int tb, float3 ep) {
    if (tid >= G * SH::EC) return;
    const int gg = tid / SH::EC, k = tid - gg * SH::EC, e = c * ta.ec + k;
    const LineGeom& Lg = t.lines[gg];
    const bool valid = c >= 0 && c < n_chunks;
    const bool here = valid && k < ta.ec && e < a.n_el;
    const bool on_g = l0 + gg < a.n_lines && Lg.tx >= 0 && Lg.tx == t_grp;
    ChunkTap x;
    x.A = x.B = x.dx = x.dy = 0.0f;
    x.thr = __builtin_inff();  // never inside the aperture
    x.lo = 0;
    x.n = 0;
    x.base = 0;
    if (here) {
      ElemGeom E;
      if constexpr (GEO_G) {
        E = elem_geom(ep.x, ep.y, ep.z, Lg);
      } else {
        const float2 E2 = t.geo[gg * a.n_el + e];
        const float2 xy = t.exy[e];
        E = ElemGeom{E2.x, E2.y, xy.x - Lg.olx, xy.y - Lg.oly};
      }
      x.A = E.A;
      x.B = E.B;
      x.dx = E.dx;
      x.dy = E.dy;
      x.thr = a.F2 * (a.array_dims == 2 ? fmaxf(fabsf(E.dx), fabsf(E.dy)) : fabsf(E.dx));
      // taps read from the window: inside the record, inside the staged samples [ws, hi] and
      // with both neighbours inside the buffer's span
      const int4 wd = t.wnd[e];
      const int ws = wd.x & ~3;
      if (on_g) {
        x.lo = wd.z;
        x.n = wd.w;
        x.base = FS == 1 ? (k * ta.span + wd.z - ws) * int(sizeof(W)) : ws;
      }
    }
    ChunkTap* ct = t.ctab + (tb * G + gg) * EC1;
    ct[k] = x;
    // the line's header, from the y offsets of its lanes (its first lane holds an element
    // whenever the chunk is valid)
    const int first = gg * SH::EC;
    const uint64_t mine = ((uint64_t(1) << SH::EC) - 1) << first;
    const float dyA = __shfl(x.dy, first);
    const uint64_t other = __builtin_amdgcn_ballot_w64(here && x.dy != dyA) & mine;
    float dyB = dyA;
    int two = 1;
    if (other != 0) {
      dyB = __shfl(x.dy, int(__builtin_ctzll(other)));
      two = (__builtin_amdgcn_ballot_w64(here && x.dy != dyA && x.dy != dyB) & mine) == 0;
    }
    if (k == 0) {
      ChunkHdr h;
      h.dyA = dyA;
      h.dyB = dyB;
      h.two = two;
      h.one = other == 0;
      *reinterpret_cast<ChunkHdr*>(ct + SH::EC) = h;
    }
  };
  // taps of a line_per_wave tile from the table of the wave's line.  MODE (chosen per chunk,
  // wave-uniform): 0 rect window, 1 Hann over x, 2 separable Hann whose chunk spans at most two
  // y offsets (the y factors computed once per chunk), 3 separable Hann in general (the y factor
  // kept while the offset repeats), 4 separable Hann whose chunk lies on one y offset (its y
  // factor is the chunk's common factor T.scale, applied to the chunk's sums and to its share
  // of the weight total instead of to every weight).  An element is evaluated by the whole
  // wave as soon as one lane has it inside its aperture (masking the others off would save no
  // issue cycles); the lanes outside take weight zero.  Single-frame tiles keep the weight and
  // the fraction of each tap (the sum interpolates, then weights); multi-frame tiles keep the
  // two tap weights.  T.slow is set in the lanes that have some tap inside the record but
  // outside the staged window (slow_taps_uni finds which).
  const uint64_t lane_mask = __builtin_amdgcn_ballot_w64(lane_ok);
  auto uni_taps = [&](auto mode_, const ChunkTap* ct, float& den) {
    constexpr int MODE = decltype(mode_)::value;
    Taps T;
    bool slow = false;
    const ChunkHdr hd = *reinterpret_cast<const ChunkHdr*>(ct + SH::EC);
    float hyA = 1.0f, hyB = 1.0f;
    if constexpr (MODE == 2) {
      hyA = hann(hd.dyA, inv_w);
      hyB = hann(hd.dyB, inv_w);
    }
    if constexpr (MODE == 4) {
      // consecutive chunks mostly lie on the same row: keep its factor
      if (__any(hd.dyA != hy_dy)) {
        hy = hann(hd.dyA, inv_w);
        hy_dy = hd.dyA;
      }
    }
    T.scale = MODE == 4 ? hy : 1.0f;
    float pden = 0.0f;  // the chunk's weights, before T.scale
#pragma unroll
    for (int k = 0; k < SH::EC; ++k) {
      // (the zero taps are set where the element is skipped: set ahead, they would cost two
      // moves per element)
      if (k >= ta.ec) {
        T.off0[k] = T.off1[k] = ZERO * int(sizeof(W));
        T.w0[k] = T.w1[k] = 0.0f;
        continue;
      }
      // the entry in two 16-byte reads (taken apart, its fields would be read one by one
      // inside branches)
      const float4 xg = *reinterpret_cast<const float4*>(ct + k);
      const int4 xw = *reinterpret_cast<const int4*>(reinterpret_cast<const char*>(ct + k) + 16);
      ChunkTap x;
      x.A = xg.x;
      x.B = xg.y;
      x.dx = xg.z;
      x.dy = xg.w;
      x.thr = __int_as_float(xw.x);
      x.base = xw.y;
      x.lo = xw.z;
      x.n = xw.w;
      const float dy = x.dy;
      const bool inside = (x.thr <= r) & lane_ok;
      if ((__builtin_amdgcn_ballot_w64(x.thr <= r) & lane_mask) != 0) {
        float w = 1.0f;
        if constexpr (MODE >= 1) w = hann(x.dx, inv_w);
        if constexpr (MODE == 2) w *= dy == hd.dyA ? hyA : hyB;
        if constexpr (MODE == 3) {
          if (__any(dy != hy_dy)) {
            hy = hann(dy, inv_w);
            hy_dy = dy;
          }
          w *= hy;
        }
        w = inside ? w : 0.0f;
        pden += w;
        const Tap tp = fast_tap(a, b, dtx, x.A, x.B, r, r2, rr);
        if constexpr (FS == 1) {
          T.w0[k] = w;
          T.w1[k] = tp.phi;
        } else {
          const float wp = w * tp.phi;
          T.w1[k] = wp;
          T.w0[k] = w - wp;
        }
        // a tap not summed from the window reads the zero vector (its weights need no masking)
        const uint32_t d = uint32_t(tp.i0) - uint32_t(x.lo);
        const bool fast = d < uint32_t(x.n);
        if constexpr (FS == 1) {
          T.off0[k] = fast ? x.base + int(d) * int(sizeof(W)) : ZERO * int(sizeof(W));
        } else {
          const int rel = tp.i0 - x.base, wbase = k * ta.span;
          const int p0 = ta.pshift ? ((rel & 1) * half + half_slot(rel >> 1)) : rel;
          const int p1 = ta.pshift ? (((rel + 1) & 1) * half + half_slot((rel + 1) >> 1)) : rel + 1;
          T.off0[k] = (fast ? wbase + p0 : ZERO) * int(sizeof(W));
          T.off1[k] = (fast ? wbase + p1 : ZERO) * int(sizeof(W));
        }
        slow |= inside & !fast & (uint32_t(tp.i0) <= uint32_t(S - 2));
      } else {
        T.off0[k] = T.off1[k] = ZERO * int(sizeof(W));
        T.w0[k] = T.w1[k] = 0.0f;
      }
      // one element at a time: hoisting the table reads of later elements would hold them all
      // in registers at once
      if constexpr (FS > 1) __builtin_amdgcn_sched_barrier(0);
    }
    T.slow = slow ? 1u : 0u;
    den = __builtin_fmaf(T.scale, pden, den);
    return T;
  };
  auto make_taps = [&](int c, float& den, int P) {
    if constexpr (UNI) {
      const ChunkTap* ct = t.ctab + (P * G + g) * EC1;
      if (ap_window == USBF_WINDOW_RECT) return uni_taps(std::integral_constant<int, 0>{}, ct, den);
      if (a.array_dims != 2) return uni_taps(std::integral_constant<int, 1>{}, ct, den);
      const ChunkHdr* hd = reinterpret_cast<const ChunkHdr*>(ct + SH::EC);
      if (hd->one) return uni_taps(std::integral_constant<int, 4>{}, ct, den);
      if (hd->two) return uni_taps(std::integral_constant<int, 2>{}, ct, den);
      return uni_taps(std::integral_constant<int, 3>{}, ct, den);
    } else {
      // window and array kind as compile-time cases where they are the same for the whole
      // launch (case 0: read per slot at run time, for apodization sets)
      auto gen_taps = [&](auto mode_) {
        constexpr int MODE = decltype(mode_)::value;  // 1, 2: Hann; 3, 4: rect; 2, 4: matrix arrays
        const bool hann_w = MODE == 0 ? ap_window != USBF_WINDOW_RECT : MODE <= 2;
        const int dims = MODE == 0 ? a.array_dims : (MODE == 2 || MODE == 4) ? 2 : 1;
        Taps T;
        T.slow = 0u;
        T.scale = 1.0f;
        // the chunk is the same for every lane: make that visible, so element data comes
        // through scalar loads
        const int e0 = __builtin_amdgcn_readfirstlane(c * ta.ec);
#pragma unroll
        for (int k = 0; k < SH::EC; ++k) {
          T.off0[k] = T.off1[k] = ZERO * int(sizeof(W));
          T.w0[k] = T.w1[k] = 0.0f;
          if (k >= ta.ec) continue;
          const int e = min(e0 + k, a.n_el - 1);
          const float2 E2 = geo[e];
          const float2 xy = t.exy[e];
          const ElemGeom E{E2.x, E2.y, xy.x - L.olx, dims == 2 ? xy.y - L.oly : 0.0f};
          const int4 wd = t.wnd[e];
          // lanes outside the aperture keep the zero weights; the block is skipped when the
          // whole wave is outside
          if ((e0 + k < a.n_el) & lane_ok & in_aperture(ap_F2, dims, E, r)) {
            float w = 1.0f;
            if (hann_w) {
              if (dims == 2) {
                // separable window: the y factor is kept while consecutive elements share their
                // row (a wave-uniform branch: skipped unless some lane meets a new row)
                if (__any(E.dy != hy_dy)) {
                  hy = hann(E.dy, inv_w);
                  hy_dy = E.dy;
                }
                w = hann(E.dx, inv_w) * hy;
              } else {
                w = hann(E.dx, inv_w);
              }
            }
            den += w;
            const Tap tp = fast_tap(a, b, dtx, E.A, E.B, r, r2, rr);
            // a tap not summed from the window reads the zero vector (its weights need no
            // masking)
            const float wp = w * tp.phi;
            T.w1[k] = wp;
            T.w0[k] = w - wp;
            const bool fast = on_grp & (uint32_t(tp.i0) - uint32_t(wd.z) < uint32_t(wd.w));
            const int rel = tp.i0 - (wd.x & ~3);
            const int wbase = k * ta.span;
            const bool split = FS > 1 && ta.pshift;
            const int p0 = split ? ((rel & 1) * half + half_slot(rel >> 1)) : rel;
            const int p1 = split ? (((rel + 1) & 1) * half + half_slot((rel + 1) >> 1)) : rel + 1;
            // byte offsets within a buffer
            T.off0[k] = (fast ? wbase + p0 : ZERO) * int(sizeof(W));
            T.off1[k] = (fast ? wbase + p1 : ZERO) * int(sizeof(W));
            T.slow |= (!fast & (uint32_t(tp.i0) <= uint32_t(S - 2))) ? (1u << k) : 0u;
          }
        }
        return T;
      };
      if constexpr (SETS) {
        return gen_taps(std::integral_constant<int, 0>{});
      } else {
        const bool d2 = a.array_dims == 2;
        if (a.window != USBF_WINDOW_RECT)
          return d2 ? gen_taps(std::integral_constant<int, 2>{}) : gen_taps(std::integral_constant<int, 1>{});
        return d2 ? gen_taps(std::integral_constant<int, 4>{}) : gen_taps(std::integral_constant<int, 3>{});
      }
    }
  };
  // Taps inside the record but outside the staged window (unusual geometry only) read global
  // memory.  line_per_wave tiles: the lanes with T.slow set re-derive their taps of the chunk
  // from its table (the same operations, so the same index) and read those that are neither
  // staged nor outside the record.
  auto slow_taps_uni = [&](const Taps& T, const ChunkTap* ct, int c, int fb, float* acc) {
    const int e0 = c * ta.ec;
    for (int k = 0; k < ta.ec; ++k) {
      const ChunkTap& x = ct[k];
      if (!((x.thr <= r) & lane_ok)) continue;
      const Tap tp = fast_tap(a, b, dtx, x.A, x.B, r, r2, rr);
      if ((uint32_t(tp.i0) - uint32_t(x.lo) < uint32_t(x.n)) | (uint32_t(tp.i0) > uint32_t(S - 2))) continue;
      float sw0 = 0.0f, sw1 = 0.0f;
#pragma unroll
      for (int kk = 0; kk < SH::EC; ++kk)
        if (kk == k) {
          sw0 = T.w0[kk];
          sw1 = T.w1[kk];
        }
      if constexpr (FS == 1) {  // weight and fraction
        const float wp = sw0 * sw1;
        sw1 = wp;
        sw0 = sw0 - wp;
      }
      sw0 *= T.scale;
      sw1 *= T.scale;
      const int16_t* p = own_block + size_t(e0 + k) * S + tp.i0;
#pragma unroll
      for (int f = 0; f < FB; ++f) {
        const int16_t* q = p + size_t(fb + f) * frame_stride;
        acc[f] = __builtin_fmaf(sw0, float(q[0]), __builtin_fmaf(sw1, float(q[1]), acc[f]));
      }
    }
  };
  // Other tiles: bit k of T.slow marks this lane's tap of the chunk's element k.
  auto slow_taps = [&](const Taps& T, int c, int fb, float* acc) {
    const int e0 = c * ta.ec;
    for (int k = 0; k < ta.ec; ++k) {
      if (!(T.slow & (1u << k))) continue;
      float2 E2;
      if constexpr (GEO_G) {
        const ElemGeom E = elem_geom(a, L, e0 + k);
        E2 = make_float2(E.A, E.B);
      } else {
        E2 = geo[e0 + k];
      }
      const Tap tp = fast_tap(a, b, dtx, E2.x, E2.y, r, r2, rr);
      const int16_t* p = own_block + size_t(e0 + k) * S + tp.i0;
      float sw0 = 0.0f, sw1 = 0.0f;
#pragma unroll
      for (int kk = 0; kk < SH::EC; ++kk)
        if (kk == k) {
          sw0 = T.w0[kk];
          sw1 = T.w1[kk];
        }
#pragma unroll
      for (int f = 0; f < FB; ++f) {
        const int16_t* q = p + size_t(fb + f) * frame_stride;
        acc[f] = __builtin_fmaf(sw0, float(q[0]), __builtin_fmaf(sw1, float(q[1]), acc[f]));
      }
    }
  };

  for (int blk = 0; blk < n_blocks; ++blk) {
    const int fb = frame0 + blk * FB;
    const __amdgpu_buffer_rsrc_t rsrc = make_rsrc(grp_block + size_t(fb) * frame_stride);
    float acc[FB];
#pragma unroll
    for (int f = 0; f < FB; ++f) acc[f] = 0.0f;
    float den = 0.0f;
    int c = next_chunk(-1);
    Items<IPT> items = chunk_items<VEC, G, FS, IPT>(t, ta, a, slots, c < n_chunks && stage_any ? c : -1);
    // sum one stage (frames s FS .. s FS + FS - 1 of the block) from LDS buffer `buf`
    auto sum_stage = [&](const Taps& T, int buf, auto s_) {
      constexpr int s = decltype(s_)::value;
      const char* w = reinterpret_cast<const char*>(t.win + buf * SH::BSTRIDE);
      if constexpr (UNI) {
        // the chunk summed on its own, then added times T.scale
        float part[FS];
#pragma unroll
        for (int f = 0; f < FS; ++f) part[f] = 0.0f;
#pragma unroll
        for (int k = 0; k < SH::EC; ++k) {
          if constexpr (FS == 1) {  // weight and fraction: interpolate, then weight
            const int16_t* p = reinterpret_cast<const int16_t*>(w + T.off0[k]);
            const float x0 = float(p[0]), x1 = float(p[1]);
            part[0] = __builtin_fmaf(T.w0[k], __builtin_fmaf(T.w1[k], x1 - x0, x0), part[0]);
          } else {
            const V x0 = *reinterpret_cast<const V*>(w + T.off0[k]);
            const V x1 = *reinterpret_cast<const V*>(w + T.off1[k]);
#pragma unroll
            for (int f = 0; f < FS; ++f)
              part[f] = __builtin_fmaf(T.w0[k], FVec<FS>::get(x0, f),
                                       __builtin_fmaf(T.w1[k], FVec<FS>::get(x1, f), part[f]));
          }
        }
#pragma unroll
        for (int f = 0; f < FS; ++f) acc[s * FS + f] = __builtin_fmaf(T.scale, part[f], acc[s * FS + f]);
      } else {
#pragma unroll
        for (int k = 0; k < SH::EC; ++k) {
          // the zero vector sits after both buffers: index relative to this buffer
          if constexpr (FS == 1) {
            const int16_t* p = reinterpret_cast<const int16_t*>(w + T.off0[k]);
            acc[s] = __builtin_fmaf(T.w0[k], float(p[0]), __builtin_fmaf(T.w1[k], float(p[1]), acc[s]));
          } else {
            const V x0 = *reinterpret_cast<const V*>(w + T.off0[k]);
            const V x1 = *reinterpret_cast<const V*>(w + T.off1[k]);
#pragma unroll
            for (int f = 0; f < FS; ++f)
              acc[s * FS + f] = __builtin_fmaf(T.w0[k], FVec<FS>::get(x0, f),
                                               __builtin_fmaf(T.w1[k], FVec<FS>::get(x1, f), acc[s * FS + f]));
          }
        }
      }
      // pin this stage's sums here: otherwise the accumulation may be sunk below later stages,
      // keeping every stage's LDS reads alive at once
#pragma unroll
      for (int f = 0; f < FS; ++f) asm volatile("" : "+v"(acc[s * FS + f]));
    };

    if constexpr (NS == 1) {
      int cn = c < n_chunks ? next_chunk(c) : n_chunks;
      Items<IPT> items_n = chunk_items<VEC, G, FS, IPT>(t, ta, a, slots, cn < n_chunks && stage_any ? cn : -1);
      issue_stage<VEC, FS, IPT>(pf[0], items, rsrc, 0u, fbytes, S);
      store_stage<VEC, G, FS, IPT>(pf[0], items, t.win, ta.span, ta.pshift);
      issue_stage<VEC, FS, IPT>(pf[1], items_n, rsrc, 0u, fbytes, S);
      float3 ep_next = make_float3(0.0f, 0.0f, 0.0f);  // positions for the next table (GEO_G)
      if constexpr (UNI) {
        fill_ctab(c, 0, GEO_G ? load_ep(c) : ep_next);
        if constexpr (GEO_G) ep_next = load_ep(cn);
      }
      __syncthreads();
      // chunk c sits in LDS buffer P, chunk cn is in flight into register set P ^ 1
      auto body = [&](auto P_) {
        constexpr int P = decltype(P_)::value;
        const int cnn = cn < n_chunks ? next_chunk(cn) : n_chunks;
        const Items<IPT> items_nn =
            chunk_items<VEC, G, FS, IPT>(t, ta, a, slots, cnn < n_chunks && stage_any ? cnn : -1);
        if (cnn < n_chunks && stage_any) issue_stage<VEC, FS, IPT>(pf[P], items_nn, rsrc, 0u, fbytes, S);
        const Taps T = make_taps(c, den, P);
        // keep the scheduler from interleaving the tap set-up with the sums (it would hoist
        // LDS reads across it and run out of registers)
        __builtin_amdgcn_sched_barrier(0);
        sum_stage(T, P, std::integral_constant<int, 0>{});
        __builtin_amdgcn_sched_barrier(0);
        if (cn < n_chunks && stage_any)
          store_stage<VEC, G, FS, IPT>(pf[P ^ 1], items_n, t.win + (P ^ 1) * SH::BSTRIDE, ta.span, ta.pshift);
        if constexpr (UNI) {
          fill_ctab(cn, P ^ 1, ep_next);
          if constexpr (GEO_G) ep_next = load_ep(cnn);  // consumed at the end of the next step
        }
        __syncthreads();
        if constexpr (UNI) {
          if (T.slow) slow_taps_uni(T, t.ctab + (P * G + g) * EC1, c, fb, acc);
        } else {
          if (T.slow) slow_taps(T, c, fb, acc);
        }
        c = cn;
        cn = cnn;
        items_n = items_nn;
      };
      while (c < n_chunks) {
        body(std::integral_constant<int, 0>{});
        if (c >= n_chunks) break;
        body(std::integral_constant<int, 1>{});
      }
    } else {
      issue_stage<VEC, FS, IPT>(pf[0], items, rsrc, 0u, fbytes, S);
      store_stage<VEC, G, FS, IPT>(pf[0], items, t.win, ta.span, ta.pshift);
      issue_stage<VEC, FS, IPT>(pf[1], items, rsrc, uint32_t(FS) * fbytes, fbytes, S);
      int tb = 0;  // table buffer of chunk c (line_per_wave tiles)
      if constexpr (UNI) fill_ctab(c, 0, make_float3(0.0f, 0.0f, 0.0f));
      __syncthreads();
      while (c < n_chunks) {
        const int cn = next_chunk(c);
        const Items<IPT> next_items =
            chunk_items<VEC, G, FS, IPT>(t, ta, a, slots, cn < n_chunks && stage_any ? cn : -1);
        const Taps T = make_taps(c, den, tb);
        __builtin_amdgcn_sched_barrier(0);
        auto step = [&](auto s_) {
          constexpr int s = decltype(s_)::value;
          constexpr bool wrap = s + 2 >= NS;  // step q + 2 is in the next chunk
          constexpr bool last = s + 1 == NS;  // step q + 1 is in the next chunk
          const bool has_ahead = wrap ? (cn < n_chunks && stage_any) : stage_any;
          if (has_ahead)
            issue_stage<VEC, FS, IPT>(pf[s & 1], wrap ? next_items : items, rsrc,
                                      uint32_t(((s + 2) % NS) * FS) * fbytes, fbytes, S);
          sum_stage(T, s & 1, s_);
          __builtin_amdgcn_sched_barrier(0);
          const bool has_next = last ? (cn < n_chunks && stage_any) : stage_any;
          if (has_next)
            store_stage<VEC, G, FS, IPT>(pf[(s + 1) & 1], last ? next_items : items,
                                         t.win + ((s + 1) & 1) * SH::BSTRIDE, ta.span, ta.pshift);
          // the next chunk's table, into the buffer this chunk's taps did not read (in the last
          // stage, where they are no longer live)
          if constexpr (UNI && last) fill_ctab(cn, tb ^ 1, make_float3(0.0f, 0.0f, 0.0f));
          __syncthreads();
        };
        static_for<NS>(step);
        tb ^= 1;
        if constexpr (UNI) {
          if (T.slow) slow_taps_uni(T, t.ctab + ((tb ^ 1) * G + g) * EC1, c, fb, acc);
        } else {
          if (T.slow) slow_taps(T, c, fb, acc);
        }
        items = next_items;
        c = cn;
      }
    }
    if (pix_ok) {
      const float inv = den > 0.0f ? 1.0f / den : 0.0f;
      float* o = out + size_t(set) * size_t(a.set_stride) + size_t(l) * a.n_depth + j;
      const size_t frame_out = size_t(a.n_lines) * a.n_depth;
#pragma unroll
      for (int f = 0; f < FB; ++f) o[size_t(fb + f) * frame_out] = acc[f] * inv;
    }
    __syncthreads();
  }
}

// One workgroup per tile.  Workgroup ids are remapped so that the depth tiles of a line group
// run one after another on the same XCD (they share the edges of their channel-data windows in
// L2), and the line groups are dealt to the XCDs round-robin (workgroup id i runs on XCD i % 8):
// the aperture of lines near the ends of the array is cut by the array's edge, so contiguous
// blocks of groups would leave the XCDs holding the edges idle at the end while the others
// still work on the centre.
#ifndef USBF_DAS_ONE_LINE_WAVES
#define USBF_DAS_ONE_LINE_WAVES 1
#endif
// waves per SIMD the register allocation must leave room for (1: no constraint)
template <int G, int FS, bool SETS>
constexpr int das_min_waves() {
  return (line_per_wave<G, FS, SETS>() && geo_from_global<G, FS>()) ? USBF_DAS_ONE_LINE_WAVES : 1;
}

template <bool VEC, int G, int FB, int FS, bool SETS>
__global__ __launch_bounds__(kDasThreads) __attribute__((amdgpu_waves_per_eu(das_min_waves<G, FS, SETS>())))
void das_tile_kernel(const int16_t* __restrict__ rf, int frame0,
                                                               int n_blocks, DasArgs a, TileArgs ta,
                                                               float* __restrict__ out) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const uint32_t n_groups = gridDim.x / uint32_t(ta.n_dtiles);
  int group, dt;
  if (n_groups % kNumXcd == 0) {
    const uint32_t xcd = blockIdx.x % kNumXcd, idx = blockIdx.x / kNumXcd;
    int k = int(idx / uint32_t(ta.n_dtiles));  // the XCD's k-th line group
    if constexpr (G > 1) {
      // multi-line tiles: an XCD takes its groups from the centre of the array outwards
      // (M/2, M/2 - 1, M/2 + 1, ...; a permutation of 0 .. M - 1 for every M), the groups with
      // the widest apertures first
      const int M = int(n_groups / kNumXcd), off = (k + 1) >> 1;
      const int kc = (k & 1) ? (M >> 1) - off : (M >> 1) + off;
      if (kc >= 0 && kc < M) k = kc;
    }
    group = k * kNumXcd + int(xcd);
    dt = int(idx % uint32_t(ta.n_dtiles));
  } else {
    const uint32_t bid = xcd_swizzle(blockIdx.x, gridDim.x);
    group = int(bid / ta.n_dtiles);
    dt = int(bid % ta.n_dtiles);
  }
  // multi-line tiles take a line group's depth tiles deepest first: the deep tiles have the
  // widest apertures and the most work, so the last workgroups to start are the light shallow
  // ones and the launch's tail is shorter (with the centre-out group order above, 4 % on the
  // 32-frame batch; one-line tiles, whose apertures cover most of the array at all but the
  // first depths, gain nothing)
  if constexpr (G > 1) dt = ta.n_dtiles - 1 - dt;
  das_tile<VEC, G, FB, FS, SETS>(rf, frame0, n_blocks, a, ta, out, lds_raw, group, dt);
}

// dynamic LDS above 64 KB has to be allowed per kernel
inline int allow_lds(const void* kernel, size_t lds) {
  const hipError_t e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  if (e != hipSuccess) return fail(USBF_EDEVICE, "cannot allow %zu bytes of LDS: %s", lds, hipGetErrorString(e));
  return USBF_OK;
}

template <int G, int FB, int FS, bool SETS>
int launch_das(const int16_t* rf, int frame0, int n_blocks, const DasArgs& a, float* out, hipStream_t s) {
  using SH = Shape<G, FS>;
  TileArgs ta;
  ta.span = (a.depth_step * SH::TD + kWindowMargin + 3) & ~3;
  ta.ec = std::min(SH::EC, SH::BUFV / ta.span);
  if (ta.ec < 1) {  // very large depth_step: one element per chunk, windows capped
    ta.ec = 1;
    ta.span = SH::BUFV & ~3;
  }
  ta.pshift = (a.depth_step % 2 == 0) ? 1 : 0;
  ta.n_dtiles = (a.n_depth + SH::TD - 1) / SH::TD;
  const int gl = SETS ? G / a.n_sets : G;  // lines per tile
  const int64_t blocks = int64_t((a.n_lines + gl - 1) / gl) * ta.n_dtiles;
  if (blocks > 0x7fffffff) return fail(USBF_EUNSUPPORTED, "too many tiles");
  const size_t lds = tile_lds_bytes<G, FS, SETS>(a.n_el);
  if (lds > size_t(kMaxTileLds))
    return fail(USBF_EUNSUPPORTED, "%d elements need %zu bytes of LDS per tile", a.n_el, lds);
  const bool vec = (a.n_samples % 4) == 0 && (reinterpret_cast<uintptr_t>(rf) & 7) == 0;
  if (vec) {
    if (lds > 65536 && allow_lds((const void*)das_tile_kernel<true, G, FB, FS, SETS>, lds)) return USBF_EDEVICE;
    hipLaunchKernelGGL((das_tile_kernel<true, G, FB, FS, SETS>), dim3(unsigned(blocks)), dim3(kDasThreads), lds, s, rf,
                       frame0, n_blocks, a, ta, out);
  } else {
    if (lds > 65536 && allow_lds((const void*)das_tile_kernel<false, G, FB, FS, SETS>, lds)) return USBF_EDEVICE;
    hipLaunchKernelGGL((das_tile_kernel<false, G, FB, FS, SETS>), dim3(unsigned(blocks)), dim3(kDasThreads), lds, s, rf,
                       frame0, n_blocks, a, ta, out);
  }
  return check_launch("das_tile_kernel");
}

// Frames are processed in blocks of FB sharing one evaluation of the delays; the batch is
// split into launches of whole blocks, largest first (e.g. 37 = 32 + 4 + 1).
template <int G, bool SETS>
int launch_das_g(const int16_t* rf, int n_frames, const DasArgs& a, float* out, hipStream_t s) {
  int f0 = 0, st = USBF_OK;
  const uint64_t frame_bytes = uint64_t(a.n_tx) * a.n_el * a.n_samples * sizeof(int16_t);
  auto run = [&](int FB, auto fn) {
    // frame offsets inside a block are 32-bit buffer offsets
    if (uint64_t(FB - 1) * frame_bytes > 0xffffffffull) return;
    const int nb = (n_frames - f0) / FB;
    if (nb > 0 && st == USBF_OK) {
      st = fn(f0, nb);
      f0 += nb * FB;
    }
  };
  run(32, [&](int f, int nb) { return launch_das<G, 32, 4, SETS>(rf, f, nb, a, out, s); });
  run(16, [&](int f, int nb) { return launch_das<G, 16, 4, SETS>(rf, f, nb, a, out, s); });
  run(8, [&](int f, int nb) { return launch_das<G, 8, 4, SETS>(rf, f, nb, a, out, s); });
  run(4, [&](int f, int nb) { return launch_das<G, 4, 4, SETS>(rf, f, nb, a, out, s); });
  run(2, [&](int f, int nb) { return launch_das<G, 2, 2, SETS>(rf, f, nb, a, out, s); });
  run(1, [&](int f, int nb) { return launch_das<G, 1, 1, SETS>(rf, f, nb, a, out, s); });
  return st;
}

// instantiated once each, in das_g<G>.hip
extern template int launch_das_g<1, false>(const int16_t*, int, const DasArgs&, float*, hipStream_t);
extern template int launch_das_g<2, false>(const int16_t*, int, const DasArgs&, float*, hipStream_t);
extern template int launch_das_g<4, false>(const int16_t*, int, const DasArgs&, float*, hipStream_t);
extern template int launch_das_g<8, false>(const int16_t*, int, const DasArgs&, float*, hipStream_t);
extern template int launch_das_g<2, true>(const int16_t*, int, const DasArgs&, float*, hipStream_t);
extern template int launch_das_g<4, true>(const int16_t*, int, const DasArgs&, float*, hipStream_t);
extern template int launch_das_g<8, true>(const int16_t*, int, const DasArgs&, float*, hipStream_t);

}  // namespace usbf
