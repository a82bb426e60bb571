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

__device__ inline ElemGeom elem_geom(const DasArgs& a, const LineGeom& L, int e) {
  const float* ep = a.el_pos + 3 * e;
  float x = ep[0] - L.olx, y = ep[1] - L.oly, z = ep[2] - L.olz;
  ElemGeom E;
  E.A = dot3(x, y, z, x, y, z);
  E.B = dot3(x, y, z, L.ulx, L.uly, L.ulz);
  E.dx = x;
  E.dy = y;
  return E;
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
// instead of the correctly rounded ones.  Let u = 2^-24.  The fast receive delay differs from
// the rule's by at most 9u relative (3u for the rule's sqrt/add/divide, 6u for the fast
// sqrt/add/reciprocal/multiply), and the three further roundings of dtx + drx, K (.) and
// - T0 add at most 2u of each intermediate, so
//   |dt_fast - dt_rule| <= u (10 K|drx| + 4 K|dtx + drx| + 2 |dt|)     (first order).
// Twice that bound is used as a guard band: outside it floor(dt_fast) = floor(dt_rule) and the
// fast value is kept (phi then differs from the rule's by less than the band); inside it the
// rule itself is evaluated.  The integer index is therefore always the rule's.
__device__ inline Tap fast_tap(const DasArgs& a, int32_t b, float dtx, float A, float B, float r, float r2,
                               float rr) {
  const float q = A - r2 * B;
  float X = q + rr;
  X = (X > 0.0f) ? X : 0.0f;
  const float s = __builtin_amdgcn_sqrtf(X) + r;
  const float drx = (s > 0.0f) ? q * __builtin_amdgcn_rcpf(s) : 0.0f;
  const float D = dtx + drx;
  const float KD = a.K * D;
  const float d = KD - a.T0;
  const float fl = floorf(d);
  const float fr = d - fl;
  const float eps = 1.1920929e-07f * (20.0f * fabsf(a.K * drx) + 8.0f * fabsf(KD) + 4.0f * fabsf(d)) + 1e-30f;
  Tap t;
  if (fr > eps && fr < 1.0f - eps) {
    t.phi = fr;
    t.i0 = b + (int32_t)fl;
    return t;
  }
  return delay_tap(a, b, dtx, small_rx_delay(A, B, r, r2, rr));
}

__device__ inline bool in_aperture(float F2, int array_dims, const ElemGeom& E, float r) {
  bool act = F2 * fabsf(E.dx) <= r;
  if (array_dims == 2) act = act && (F2 * fabsf(E.dy) <= r);
  return act;
}

__device__ inline bool in_aperture(const DasArgs& a, const ElemGeom& E, float r) {
  return in_aperture(a.F2, a.array_dims, E, r);
}

#pragma clang fp contract(on)

// Apodization weight (a value, not part of the index rule).  inv_w = f_number / r.
__device__ inline float apod_weight(int window, int dims, float dx, float dy, float inv_w) {
  if (window == USBF_WINDOW_RECT) return 1.0f;
  // Hann: 1/2 + 1/2 cos(2 pi u); the hardware cosine takes its argument in revolutions.
  float w = 0.5f + 0.5f * __builtin_amdgcn_cosf(dx * inv_w);
  if (dims == 2) w *= 0.5f + 0.5f * __builtin_amdgcn_cosf(dy * inv_w);
  return w;
}

}  // namespace usbf
