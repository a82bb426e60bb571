/*
 * CPU oracle for receive delay-and-sum beamforming -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg load this
 * library.  It shares no source with the GPU library.
 *
 * What it computes (the paper's receive-beamforming step, Sec. 1 pipeline list and
 * Sec. 2 method list item 2, "delay and sum" after Shattuck 1984): for every output
 * sample p on a scanline and every receive element e, the channel signal of the
 * transmit that insonified the line is read at the two-way travel time
 *     tau = fs * (T_tx(p) + |e - p| / c) - fs * t0        [in samples]
 * (linear interpolation between samples), weighted by a receive apodization that
 * grows with depth (aperture width depth / F#, Hann or rectangular), summed over
 * elements and normalised by the sum of weights.  T_tx is the time a focused
 * transmit wave needs to reach p, modelled as a wave converging on (and diverging
 * from) a virtual source at the focus; an infinite focus is a plane wave, whose
 * wavefront passes the transmit origin at t = 0 (c T_tx = (p - o_t).u_t; plane-wave
 * imaging is among the protocols the paper intends to add, Sec. 2).  Everything here is
 * float64 except the
 * integer decisions (sample index, aperture membership, record bounds), which are
 * taken by tof32() below in binary32 exactly as the GPU library takes them.
 *
 * Binary32 delay rule (tof32): each operation one IEEE binary32 op, round to nearest
 * even, sqrt and division correctly rounded, no fused multiply-add, sums left to
 * right.  The expression is the same travel time rearranged so that the large
 * part (2 r fs / c = j0 + m j, an exact integer) never enters floating point:
 *   r      = (float)(j0 + m j) * h,  h = c / (fs + fs)
 *   d_rx   = q / (sqrt(max(q + r r, 0)) + r),  q = |e-o|^2 - (r+r) ((e-o).u_l)   (0 if denominator 0)
 *   d_tx   = (a - r) + s l2 / (|p - f| + |a - F|)                                (0 if denominator 0)
 *   dt     = (fs/c) (d_tx + d_rx) - fs t0;   i0 = j0 + m j + floor(dt),  phi = dt - floor(dt)
 * with a - r = g + r (u_l.u_t - 1) and l2 = |U + r V|^2 per line constants, both set
 * to 0 when the line and its transmit share origin and direction bit for bit.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#pragma STDC FP_CONTRACT OFF

typedef struct {
  int32_t n_el;
  const float* el_pos;       /* [n_el][3] */
  int32_t n_tx;
  const float* tx_origin;    /* [n_tx][3] */
  const float* tx_dir;       /* [n_tx][3] */
  const float* tx_focus;     /* [n_tx]    */
  int32_t n_lines;
  const float* line_origin;  /* [n_lines][3] */
  const float* line_dir;     /* [n_lines][3] */
  const int32_t* line_tx;    /* [n_lines] */
  int32_t array_dims;        /* 1 linear, 2 matrix */
  float c, fs, t0;
  int32_t n_samples, depth_start, depth_step, n_depth;
  float f_number;
  int32_t window;            /* 0 rect, 1 Hann */
} og_t;

/* ------------------------------------------------------------------ binary32 rule */

typedef struct {
  float ul[3], ut[3];
  float g, k;        /* g = (o_l - o_t).u_t ; k = u_l.u_t - 1 */
  float U[3], V[3];  /* U = (o_l - o_t) - g u_t ; V = u_l - (u_l.u_t) u_t */
  int same;
  float F;
} line32_t;

static float dot3f(const float* a, const float* b) {
  float s = a[0] * b[0];
  s = s + a[1] * b[1];
  s = s + a[2] * b[2];
  return s;
}

static void unit3f(const float* d, float* u) {
  float n = sqrtf(dot3f(d, d));
  u[0] = d[0] / n;
  u[1] = d[1] / n;
  u[2] = d[2] / n;
}

static void line32_setup(const og_t* G, int l, line32_t* L) {
  int t = G->line_tx[l];
  const float* ol = G->line_origin + 3 * l;
  const float* dl = G->line_dir + 3 * l;
  const float* ot = G->tx_origin + 3 * t;
  const float* dt = G->tx_dir + 3 * t;
  unit3f(dl, L->ul);
  unit3f(dt, L->ut);
  L->same = (memcmp(ol, ot, 12) == 0) && (memcmp(dl, dt, 12) == 0);
  float dO[3] = {ol[0] - ot[0], ol[1] - ot[1], ol[2] - ot[2]};
  L->g = dot3f(dO, L->ut);
  float cl = dot3f(L->ul, L->ut);
  L->k = cl - 1.0f;
  for (int i = 0; i < 3; ++i) {
    L->U[i] = dO[i] - L->g * L->ut[i];
    L->V[i] = L->ul[i] - cl * L->ut[i];
  }
  L->F = G->tx_focus[t];
}

/* transmit part of the small delay, for depth r on the line */
static float dtx32(const line32_t* L, float r) {
  float amr, l2;
  if (L->same) {
    amr = 0.0f;
    l2 = 0.0f;
  } else {
    amr = L->g + r * L->k;
    float w0 = L->U[0] + r * L->V[0];
    float w1 = L->U[1] + r * L->V[1];
    float w2 = L->U[2] + r * L->V[2];
    l2 = w0 * w0;
    l2 = l2 + w1 * w1;
    l2 = l2 + w2 * w2;
  }
  if (isinf(L->F)) return amr; /* plane wave: c T_tx - r is the projection part alone */
  float amF = amr + (r - L->F);
  float pf = sqrtf(amF * amF + l2);
  float den = pf + fabsf(amF);
  if (den > 0.0f) {
    float corr = (amF >= 0.0f ? l2 : -l2) / den;
    return amr + corr;
  }
  return amr;
}

typedef struct {
  int32_t i0;
  float phi;
  int active, valid;
} tof32_t;

static void tof32(const og_t* G, int l, const line32_t* L, int j, int e, tof32_t* out) {
  const float h = G->c / (G->fs + G->fs);
  const float K = G->fs / G->c;
  const float T0 = G->fs * G->t0;
  const float F2 = G->f_number + G->f_number;
  int32_t b = G->depth_start + G->depth_step * j;
  float r = (float)b * h;
  const float* ep = G->el_pos + 3 * e;
  const float* ol = G->line_origin + 3 * l;
  float ex[3] = {ep[0] - ol[0], ep[1] - ol[1], ep[2] - ol[2]};
  float A = dot3f(ex, ex);
  float B = dot3f(ex, L->ul);
  float q = A - (r + r) * B;
  float X = q + r * r;
  if (!(X > 0.0f)) X = 0.0f;
  float s = sqrtf(X) + r;
  float drx = (s > 0.0f) ? q / s : 0.0f;
  float d = K * (dtx32(L, r) + drx) - T0;
  float fl = floorf(d);
  out->phi = d - fl;
  out->i0 = b + (int32_t)fl;
  int act = (F2 * fabsf(ex[0]) <= r);
  if (G->array_dims == 2) act = act && (F2 * fabsf(ex[1]) <= r);
  out->active = act;
  out->valid = (out->i0 >= 0) && (out->i0 <= G->n_samples - 2);
}

/* Index map for a list of (line, depth) pixels x all elements.
 * pix: [n_pix][2] (line, j) or NULL for every pixel in line-major order.
 * i0 [n_pix][n_el] int32, phi [n_pix][n_el] float (nullable), flags [n_pix][n_el]:
 * bit0 active, bit1 valid. */
void oracle_tof32(const og_t* G, int64_t n_pix, const int32_t* pix, int32_t* i0, float* phi,
                  uint8_t* flags) {
  #pragma omp parallel for schedule(dynamic, 64)
  for (int64_t p = 0; p < n_pix; ++p) {
    int l = pix ? pix[2 * p] : (int)(p / G->n_depth);
    int j = pix ? pix[2 * p + 1] : (int)(p % G->n_depth);
    line32_t L;
    line32_setup(G, l, &L);
    for (int e = 0; e < G->n_el; ++e) {
      tof32_t t;
      tof32(G, l, &L, j, e, &t);
      int64_t o = p * G->n_el + e;
      i0[o] = t.i0;
      if (phi) phi[o] = t.phi;
      flags[o] = (uint8_t)(t.active | (t.valid << 1));
    }
  }
}

/* ------------------------------------------------------------------ float64 geometry */

typedef struct {
  double o[3], u[3];       /* line origin, unit direction */
  double ot[3], ut[3], F;  /* transmit origin, unit direction, focal range */
  double f[3];             /* virtual source (focus) */
} line64_t;

static void unit3d(const float* d, double* u) {
  double x = d[0], y = d[1], z = d[2];
  double n = sqrt(x * x + y * y + z * z);
  u[0] = x / n;
  u[1] = y / n;
  u[2] = z / n;
}

static void line64_setup(const og_t* G, int l, line64_t* L) {
  int t = G->line_tx[l];
  for (int i = 0; i < 3; ++i) {
    L->o[i] = G->line_origin[3 * l + i];
    L->ot[i] = G->tx_origin[3 * t + i];
  }
  unit3d(G->line_dir + 3 * l, L->u);
  unit3d(G->tx_dir + 3 * t, L->ut);
  L->F = G->tx_focus[t];
  for (int i = 0; i < 3; ++i) L->f[i] = isinf(L->F) ? 0.0 : L->ot[i] + L->F * L->ut[i];
}

static double dist3(const double* a, const double* b) {
  double x = a[0] - b[0], y = a[1] - b[1], z = a[2] - b[2];
  return sqrt(x * x + y * y + z * z);
}

/* depth of output sample j (float64) */
static double depth64(const og_t* G, int j) {
  return (double)(G->depth_start + G->depth_step * j) * ((double)G->c / (2.0 * (double)G->fs));
}

/* pixel position and transmit travel distance c*T_tx */
static void pixel64(const line64_t* L, double r, double* p, double* ctx) {
  for (int i = 0; i < 3; ++i) p[i] = L->o[i] + r * L->u[i];
  double a = (p[0] - L->ot[0]) * L->ut[0] + (p[1] - L->ot[1]) * L->ut[1] + (p[2] - L->ot[2]) * L->ut[2];
  if (isinf(L->F)) { /* plane wave: the wavefront passes the transmit origin at t = 0 */
    *ctx = a;
    return;
  }
  double pf = dist3(p, L->f);
  *ctx = (a >= L->F) ? L->F + pf : L->F - pf;
}

/* two-way delay in samples, float64 */
static double tau64(const og_t* G, const double* p, double ctx, int e) {
  double ep[3] = {G->el_pos[3 * e], G->el_pos[3 * e + 1], G->el_pos[3 * e + 2]};
  double drx = dist3(ep, p);
  return (double)G->fs * (ctx + drx) / (double)G->c - (double)G->fs * (double)G->t0;
}

/* Float64 delays tau for (line, j) pixels x elements (for checking the binary32 rule). */
void oracle_tau64(const og_t* G, int64_t n_pix, const int32_t* pix, double* tau) {
  #pragma omp parallel for schedule(dynamic, 64)
  for (int64_t q = 0; q < n_pix; ++q) {
    int l = pix ? pix[2 * q] : (int)(q / G->n_depth);
    int j = pix ? pix[2 * q + 1] : (int)(q % G->n_depth);
    line64_t L;
    line64_setup(G, l, &L);
    double p[3], ctx;
    pixel64(&L, depth64(G, j), p, &ctx);
    for (int e = 0; e < G->n_el; ++e) tau[q * G->n_el + e] = tau64(G, p, ctx, e);
  }
}

static double window64(int window, double u) {
  if (window == 1) return 0.5 + 0.5 * cos(2.0 * M_PI * u);
  return 1.0;
}

/* receive apodization weight of element e for pixel depth r on line l (float64) */
static double apod64(const og_t* G, int l, int e, double r) {
  double dx = (double)G->el_pos[3 * e] - (double)G->line_origin[3 * l];
  double dy = (double)G->el_pos[3 * e + 1] - (double)G->line_origin[3 * l + 1];
  if (r <= 0.0) return 1.0;  /* only elements at zero offset are active at r = 0 */
  double F = G->f_number;
  double w = window64(G->window, dx * F / r);
  if (G->array_dims == 2) w *= window64(G->window, dy * F / r);
  return w;
}

/* linear interpolation of one channel at tau (float64), tau clamped into [0, S-1] */
static double sample64(const int16_t* trace, int S, double tau) {
  if (tau < 0.0) tau = 0.0;
  if (tau > (double)(S - 1)) tau = (double)(S - 1);
  double fl = floor(tau);
  int i = (int)fl;
  double ph = tau - fl;
  if (i >= S - 1) return (double)trace[S - 1];
  return (1.0 - ph) * (double)trace[i] + ph * (double)trace[i + 1];
}

/* DAS for a list of pixels.
 * rf: [n_frames][n_tx][n_el][S]; pix: [n_pix][3] (frame, line, j), or NULL for every pixel
 * of every frame in (frame, line, j) order; out[n_pix] float64. */
void oracle_das(const og_t* G, const int16_t* rf, int32_t n_frames, int64_t n_pix,
                const int32_t* pix, double* out) {
  const int64_t S = G->n_samples;
  #pragma omp parallel for schedule(dynamic, 16)
  for (int64_t q = 0; q < n_pix; ++q) {
    int f, l, j;
    if (pix) {
      f = pix[3 * q];
      l = pix[3 * q + 1];
      j = pix[3 * q + 2];
    } else {
      int64_t per = (int64_t)G->n_lines * G->n_depth;
      f = (int)(q / per);
      l = (int)((q % per) / G->n_depth);
      j = (int)(q % G->n_depth);
    }
    int t = G->line_tx[l];
    if (t < 0 || t >= G->n_tx) { /* a line without a transmit is a line of zeros */
      out[q] = 0.0;
      continue;
    }
    line32_t L32;
    line32_setup(G, l, &L32);
    line64_t L;
    line64_setup(G, l, &L);
    double r = depth64(G, j);
    double p[3], ctx;
    pixel64(&L, r, p, &ctx);
    const int16_t* base = rf + (((int64_t)f * G->n_tx + t) * G->n_el) * S;
    double num = 0.0, den = 0.0;
    for (int e = 0; e < G->n_el; ++e) {
      tof32_t d;
      tof32(G, l, &L32, j, e, &d);
      if (!d.active) continue;
      double w = apod64(G, l, e, r);
      den += w;
      if (!d.valid) continue;
      num += w * sample64(base + (int64_t)e * S, (int)S, tau64(G, p, ctx, e));
    }
    out[q] = den > 0.0 ? num / den : 0.0;
  }
}

/* Delayed channel samples without summation: x[q][e] for every element (no aperture
 * limit); samples outside the record are 0.  pix as in oracle_das. */
void oracle_delay_gather(const og_t* G, const int16_t* rf, int64_t n_pix, const int32_t* pix,
                         double* x) {
  const int64_t S = G->n_samples;
  #pragma omp parallel for schedule(dynamic, 16)
  for (int64_t q = 0; q < n_pix; ++q) {
    int f = pix[3 * q], l = pix[3 * q + 1], j = pix[3 * q + 2];
    int t = G->line_tx[l];
    if (t < 0 || t >= G->n_tx) {
      for (int e = 0; e < G->n_el; ++e) x[q * G->n_el + e] = 0.0;
      continue;
    }
    line32_t L32;
    line32_setup(G, l, &L32);
    line64_t L;
    line64_setup(G, l, &L);
    double p[3], ctx;
    pixel64(&L, depth64(G, j), p, &ctx);
    const int16_t* base = rf + (((int64_t)f * G->n_tx + t) * G->n_el) * S;
    for (int e = 0; e < G->n_el; ++e) {
      tof32_t d;
      tof32(G, l, &L32, j, e, &d);
      x[q * G->n_el + e] = d.valid ? sample64(base + (int64_t)e * S, (int)S, tau64(G, p, ctx, e)) : 0.0;
    }
  }
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  extern int omp_get_max_threads(void);
  return omp_get_max_threads();
#else
  return 1;
#endif
}
