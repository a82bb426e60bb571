// Device side of the binary32 delay rule (see usbf_delay_index_map in usbf.h).
//
// Two-way travel time of a focused transmit and the receive path, for pixel p at depth r on
// line l and element e:  tau = fs (T_tx(p) + |e - p| / c) - fs t0.  The large exact part
// 2 r fs / c = b (an integer) is kept out of floating point; what remains is
//   (fs / c) (dtx + drx) - fs t0
// with dtx = c T_tx - r and drx = |e - p| - r, both written without cancellation.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.h"

namespace usbf {

#pragma clang fp contract(off)

struct LineGeom {
  float olx, oly, olz;     // line origin
  float ulx, uly, ulz;     // unit line direction
  float g, k;              // (o_l - o_t).u_t ; u_l.u_t - 1
  float Ux, Uy, Uz;        // (o_l - o_t) - g u_t
  float Vx, Vy, Vz;        // u_l - (u_l.u_t) u_t
  float F;                 // focal range of the line's transmit
  int same;                // line and transmit share origin and direction bit for bit
  int tx;                  // transmit index, -1 if out of range
  float F2, fn;            // apodization: 2 f_number (aperture test) and f_number
  int window;
};

__device__ inline float dot3(float ax, float ay, float az, float bx, float by, float bz) {
  float s = ax * bx;
  s = s + ay * by;
  s = s + az * bz;
  return s;
}

__device__ inline void unit3(float x, float y, float z, float& ux, float& uy, float& uz) {
  float n = sqrtf(dot3(x, y, z, x, y, z));
  ux = x / n;
  uy = y / n;
  uz = z / n;
}

__device__ inline void line_geom(const DasArgs& a, int l, LineGeom& L) {
  int t = a.line_tx[l];
  L.tx = (t >= 0 && t < a.n_tx) ? t : -1;
  if (L.tx < 0) t = 0;
  const float* ol = a.line_origin + 3 * l;
  const float* dl = a.line_dir + 3 * l;
  const float* ot = a.tx_origin + 3 * t;
  const float* dt = a.tx_dir + 3 * t;
  float olx = ol[0], oly = ol[1], olz = ol[2];
  float dlx = dl[0], dly = dl[1], dlz = dl[2];
  float otx = ot[0], oty = ot[1], otz = ot[2];
  float dtx = dt[0], dty = dt[1], dtz = dt[2];
  L.olx = olx;
  L.oly = oly;
  L.olz = olz;
  unit3(dlx, dly, dlz, L.ulx, L.uly, L.ulz);
  float utx, uty, utz;
  unit3(dtx, dty, dtz, utx, uty, utz);
  L.same = (__float_as_uint(olx) == __float_as_uint(otx)) && (__float_as_uint(oly) == __float_as_uint(oty)) &&
           (__float_as_uint(olz) == __float_as_uint(otz)) && (__float_as_uint(dlx) == __float_as_uint(dtx)) &&
           (__float_as_uint(dly) == __float_as_uint(dty)) && (__float_as_uint(dlz) == __float_as_uint(dtz));
  float Dx = olx - otx, Dy = oly - oty, Dz = olz - otz;
  L.g = dot3(Dx, Dy, Dz, utx, uty, utz);
  float cl = dot3(L.ulx, L.uly, L.ulz, utx, uty, utz);
  L.k = cl - 1.0f;
  L.Ux = Dx - L.g * utx;
  L.Uy = Dy - L.g * uty;
  L.Uz = Dz - L.g * utz;
  L.Vx = L.ulx - cl * utx;
  L.Vy = L.uly - cl * uty;
  L.Vz = L.ulz - cl * utz;
  L.F = a.tx_focus[t];
  L.F2 = a.F2;
  L.fn = a.f_number;
  L.window = a.window;
}

// c T_tx - r for depth r on the line.
__device__ inline float small_tx_delay(const LineGeom& L, float r) {
  float amr, l2;
  if (L.same) {
    amr = 0.0f;
    l2 = 0.0f;
  } else {
    amr = L.g + r * L.k;
    float w0 = L.Ux + r * L.Vx;
    float w1 = L.Uy + r * L.Vy;
    float w2 = L.Uz + r * L.Vz;
    l2 = w0 * w0;
    l2 = l2 + w1 * w1;
    l2 = l2 + w2 * w2;
  }
  if (isinf(L.F)) return amr;  // plane wave (infinite focus): the projection part alone
  float m = amr + (r - L.F);
  float den = sqrtf(m * m + l2) + fabsf(m);
  if (den > 0.0f) return amr + (m >= 0.0f ? l2 : -l2) / den;
  return amr;
}

// Per (line, element) constants of the receive path.
struct ElemGeom {
  float A;      // |e - o_l|^2
  float B;      // (e - o_l) . u_l
  float dx, dy; // lateral offsets from the line origin
};

__device__ inline ElemGeom elem_geom(float ex, float ey, float ez, const LineGeom& L) {
  float x = ex - L.olx, y = ey - L.oly, z = ez - L.olz;
  ElemGeom E;
  E.A = dot3(x, y, z, x, y, z);
  E.B = dot3(x, y, z, L.ulx, L.uly, L.ulz);
  E.dx = x;
  E.dy = y;
  return E;
}

__device__ inline ElemGeom elem_geom(const DasArgs& a, const LineGeom& L, int e) {
  const float* ep = a.el_pos + 3 * e;
  return elem_geom(ep[0], ep[1], ep[2], L);
}

// |e - p| - r for depth r; r2 = r + r and rr = r * r precomputed per pixel.
__device__ inline float small_rx_delay(float A, float B, float r, float r2, float rr) {
  float q = A - r2 * B;
  float X = q + rr;
  X = (X > 0.0f) ? X : 0.0f;
  float s = sqrtf(X) + r;
  return (s > 0.0f) ? q / s : 0.0f;
}

struct Tap {
  int32_t i0;
  float phi;
};

__device__ inline Tap delay_tap(const DasArgs& a, int32_t b, float dtx, float drx) {
  float d = a.K * (dtx + drx) - a.T0;
  float fl = floorf(d);
  Tap t;
  t.phi = d - fl;
  t.i0 = b + (int32_t)fl;
  return t;
}

// The same tap, computed with the hardware square root and reciprocal (each within 1 ulp)
// instead of the correctly rounded ones, and with the constant part of the delay folded into
// one fused multiply-add: d = fma(K, drx, K dtx - T0).  q and X are formed exactly as the rule
// forms them, so their rounding is common to both; X is not clamped at zero (a negative X, from
// rounding where the element is at the pixel, gives a NaN, and a NaN takes the rule below).
// With u = 2^-24 and first-order terms:
//   |drx_fast - drx_rule| <= 9 u |drx|   (3u for the rule's sqrt/add/divide, 6u for the fast
//                                         sqrt/add/reciprocal/multiply)
//   rule, after drx       <= u (2 K |D| + |d|)          (D = dtx + drx, d = K D - T0)
//   fast, after drx       <= u (2 K |dtx| + |T0| + |d|)
// so |d_fast - d_rule| <= u (K (13 |drx| + 6 |dtx|) + 3 |T0|).  Twice that is the guard band:
// outside it floor(d_fast) = floor(d_rule) and the fast value is kept (the fraction then
// differs from the rule's by less than the band); inside it -- or where the fast value is not
// finite (X < 0, or r = 0 and the element on the line's origin) -- the rule itself is
// evaluated.  The integer index is therefore always the rule's.
__device__ inline Tap fast_tap(const DasArgs& a, int32_t b, float dtx, float A, float B, float r, float r2,
                               float rr) {
  const float q = A - r2 * B;
  const float X = q + rr;
  const float s = __builtin_amdgcn_sqrtf(X) + r;
  const float drx = q * __builtin_amdgcn_rcpf(s);
  const float c = a.K * dtx - a.T0;  // per pixel (hoisted out of element loops)
  const float d = __builtin_fmaf(a.K, drx, c);
  constexpr float u = 5.9604645e-08f;  // 2^-24
  const float base = u * (12.0f * fabsf(a.K * dtx) + 6.0f * fabsf(a.T0)) + 1e-30f;  // per pixel
  const float eps = __builtin_fmaf(26.0f * u * a.K, fabsf(drx), base);
  const float fl = floorf(d);
  const float fr = d - fl;
  Tap t;
  if (fr > eps && fr < 1.0f - eps) {
    t.phi = fr;
    t.i0 = b + (int32_t)fl;
    return t;
  }
  return delay_tap(a, b, dtx, small_rx_delay(A, B, r, r2, rr));
}

// F2 |dx| <= r (and F2 |dy| <= r): one product of the larger offset, which rounds to the larger
// of the two products (rounding is monotonic), so the decision is the rule's.
__device__ inline bool in_aperture(float F2, int array_dims, const ElemGeom& E, float r) {
  const float m = array_dims == 2 ? fmaxf(fabsf(E.dx), fabsf(E.dy)) : fabsf(E.dx);
  return F2 * m <= r;
}

__device__ inline bool in_aperture(const DasArgs& a, const ElemGeom& E, float r) {
  return in_aperture(a.F2, a.array_dims, E, r);
}

#pragma clang fp contract(on)

// Hann factor 1/2 + 1/2 cos(2 pi u) of an offset d at inv_w = f_number / r; the hardware
// cosine takes its argument in revolutions.
__device__ inline float hann(float d, float inv_w) { return 0.5f + 0.5f * __builtin_amdgcn_cosf(d * inv_w); }

// Apodization weight (a value, not part of the index rule).  inv_w = f_number / r.
__device__ inline float apod_weight(int window, int dims, float dx, float dy, float inv_w) {
  if (window == USBF_WINDOW_RECT) return 1.0f;
  float w = hann(dx, inv_w);
  if (dims == 2) w *= hann(dy, inv_w);
  return w;
}

}  // namespace usbf
