/*
 * usbf -- ultrasound receive pipeline on AMD Instinct MI355X (gfx950).
 *
 * The receive chain of a software-defined ultrasound system (Goebl, Navab, Hennersperger,
 * "SUPRA: open source software defined ultrasound processing for real-time applications",
 * arXiv:1711.06127): receive beamforming by delay and sum, envelope detection, log
 * compression and scan conversion (Sec. 1 pipeline list; Sec. 2 method list items 1-5),
 * for 2D linear and 3D matrix probes.
 *
 * Conventions for every entry point below
 *  - Array arguments are DEVICE pointers, owned by the caller, contiguous, row-major, and
 *    must stay valid until the work enqueued on `stream` has finished.  Struct arguments
 *    are HOST pointers read during the call only.  Nothing is retained after a call returns.
 *  - Every call is asynchronous on `stream` (a HIP stream, 0 = the null stream) and never
 *    synchronises the host.  Device faults surface at the caller's next synchronisation.
 *  - Arguments are validated before anything is enqueued; on any error nothing is enqueued
 *    and the outputs are untouched.  Return values: USBF_OK or a negative USBF_E* code;
 *    usbf_status_string() gives the text, usbf_last_error_detail() the reason of the
 *    calling thread's last failure.
 *  - Stateless calls are reentrant: two beamformers with different parameters may read the
 *    same channel data concurrently (the paper runs two differently parametrised
 *    beamformers on one input, Sec. 2).
 *  - Lengths in metres, times in seconds, all floating-point parameters binary32.
 */
#ifndef USBF_H
#define USBF_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define USBF_OK            0
#define USBF_EINVAL       -1  /* null pointer or a parameter outside its valid range      */
#define USBF_ESHAPE       -2  /* sizes inconsistent with each other                        */
#define USBF_EUNSUPPORTED -3  /* valid request beyond what the kernels implement           */
#define USBF_EWORKSPACE   -4  /* workspace missing or smaller than usbf_workspace_bytes()  */
#define USBF_EDEVICE      -5  /* HIP launch or runtime error                               */

#define USBF_WINDOW_RECT 0
#define USBF_WINDOW_HANN 1

#define USBF_MAX_ELEMENTS 1024
#define USBF_MAX_FRAMES   65535

/*
 * Probe, transmit and scanline geometry (device arrays).
 *   el_pos      [n_el][3]    element centres; the array lies in the plane z = 0.
 *   tx_origin   [n_tx][3]    transmit beam origin;  tx_dir [n_tx][3] its direction (any
 *                            length > 0, normalised inside);  tx_focus [n_tx] signed focal
 *                            range F along tx_dir.  The wave is modelled as converging on,
 *                            then diverging from, a virtual source at tx_origin + F u, reached
 *                            at t = F / c: F > 0 is a focused transmit; F < 0 a diverging wave
 *                            from a source |F| behind the array; +infinity a plane wave, whose
 *                            wavefront passes tx_origin at t = 0 (transmit time
 *                            (p - tx_origin).u / c; plane-wave imaging, Sec. 2).  F = 0 is a
 *                            spherical wave from tx_origin itself; NaN is not meaningful
 *                            (not checked: the array is in device memory).
 *   line_origin [n_lines][3] scanline origin; line_dir [n_lines][3] its direction;
 *   line_tx     [n_lines]    transmit whose echoes form the line (multi-line acquisition
 *                            when several lines share one transmit, Sec. 2 method list item 1).
 *   array_dims  1: linear array, receive aperture limited along x only;
 *               2: matrix array, separable aperture along x and y.
 *   lines_per_tx  work-grouping hint, no effect on results: G > 1 announces that each run of
 *               G consecutive lines starting at a multiple of G shares one transmit, so the
 *               channel data of that transmit is staged once for the lines of a tile (tiles of
 *               8 lines for G = 8, of 4 for other multiples of 4, of 2 for other even G; 0 or
 *               1: no grouping).  A wrong hint only costs speed.
 * The receive aperture is centred on the line origin.
 */
typedef struct usbf_geometry {
  int32_t n_el;
  const float* el_pos;
  int32_t n_tx;
  const float* tx_origin;
  const float* tx_dir;
  const float* tx_focus;
  int32_t n_lines;
  const float* line_origin;
  const float* line_dir;
  const int32_t* line_tx;
  int32_t array_dims;
  int32_t lines_per_tx;
} usbf_geometry;

/*
 * Receive parameters.
 *   c speed of sound (> 0), fs sampling rate (> 0), t0 time of sample 0 relative to the
 *   transmit's virtual-source arrival reference.
 *   n_samples S >= 2 samples per channel.
 *   Output sample j of every line lies at depth r_j = (depth_start + depth_step * j) * c / (2 fs),
 *   j = 0 .. n_depth-1 (depth_start >= 0, depth_step >= 1, n_depth >= 1).
 *   f_number > 0: at depth r the aperture is r / f_number wide; window USBF_WINDOW_*.
 */
typedef struct usbf_rx {
  float c, fs, t0;
  int32_t n_samples;
  int32_t depth_start, depth_step, n_depth;
  float f_number;
  int32_t window;
} usbf_rx;

/*
 * Scan-conversion grid (Sec. 1 pipeline list, last step; Sec. 2 method list item 5).
 *   kind 0: 2D, parallel vertical lines at x = line_u[k]; pixel (i, k) at
 *           (x0 + i*hx, z0 + k*hz), line depth = z.
 *   kind 1: 3D, steered lines with tangents (line_u[iu], line_v[iv]) of the angles in x and
 *           y; line index = iv * n_u + iu; voxel (i, j, k) at (x0 + i hx, y0 + j hy, z0 + k hz)
 *           maps to u = x/z, v = y/z, range sqrt((x x + y y) + z z).
 *   kind 2: 2D sector, lines with tangents line_u from a common apex at the origin;
 *           u = x/z, range sqrt(x x + z z).
 *   line_u[n_u], line_v[n_v]: device arrays, strictly increasing.  Line samples are at range
 *   r0 + n*dr, n = 0 .. n_depth-1.  Pixels outside the lines' hull get `fill`.
 *   Output layout [nz][nx] (2D) or [nz][ny][nx] (3D).
 */
typedef struct usbf_scan {
  int32_t kind;
  int32_t nx, ny, nz;
  float x0, hx, y0, hy, z0, hz;
  const float* line_u;
  const float* line_v;
  int32_t n_u, n_v;
  float r0, dr;
  int32_t n_depth;
  float fill;
} usbf_scan;

/* ---------------------------------------------------------------- the pipeline stages */

/*
 * Receive beamforming by delay and sum (Sec. 1 pipeline list, "receive beamforming";
 * Sec. 2 method list items 1-2): for every frame f, line l and depth sample j,
 *   out[f][l][j] = sum_e w_e s_e / sum_e w_e  over the elements e inside the aperture,
 * where s_e is channel e of transmit line_tx[l] in frame f, linearly interpolated at the
 * two-way travel time tau = fs (T_tx + |e - p| / c) - fs t0 (0 outside samples 0..S-1;
 * such elements still count in the denominator), w_e the window over the aperture
 * (Hann: 1/2 + 1/2 cos(2 pi u), u = offset / aperture width), and out = 0 where no element
 * is inside the aperture.  The integer sample index floor(tau) and the aperture and
 * record-bound decisions follow the binary32 delay rule documented with
 * usbf_delay_index_map(); the sum accumulates in binary32.
 *   rf   int16 [n_frames][n_tx][n_el][n_samples]
 *   out  float [n_frames][n_lines][n_depth]
 * 1 <= n_frames <= USBF_MAX_FRAMES, 1 <= n_el <= USBF_MAX_ELEMENTS.
 * A line_tx entry outside [0, n_tx) yields a line of zeros.
 */
int usbf_beamform(const int16_t* rf, int32_t n_frames, const usbf_geometry* geom,
                  const usbf_rx* rx, float* out, hipStream_t stream);

/*
 * Several differently parameterised delay-and-sum beamformers over the same channel data in
 * one pass (Sec. 2: two differently parametrised beamforming runs on the same input): set k
 * has its own f-number f_numbers[k] and window windows[k] (USBF_WINDOW_*), everything else
 * (geometry, depth grid, c, fs, t0) is shared.  Set k's result equals usbf_beamform() with
 * rx->f_number = f_numbers[k] and rx->window = windows[k] (the same binary32 rule and the
 * same summation order); the channel data is staged once for all sets, so the pass costs
 * far less than n_sets separate calls.  rx->f_number and rx->window must still be valid
 * and are otherwise unused.
 *   rf         int16 [n_frames][n_tx][n_el][n_samples] (device)
 *   f_numbers  float [n_sets], windows int32 [n_sets] (host; read during the call)
 *   out        float [n_sets][n_frames][n_lines][n_depth] (device)
 * n_sets = 1, 2 or 4; other limits as usbf_beamform().
 */
int usbf_beamform_sets(const int16_t* rf, int32_t n_frames, const usbf_geometry* geom,
                       const usbf_rx* rx, int32_t n_sets, const float* f_numbers,
                       const int32_t* windows, float* out, hipStream_t stream);

/*
 * Envelope detection (Sec. 1 pipeline list, "envelope detection"; the Hilbert-transform
 * envelope of the PSF study, Sec. 3.2): for each of n_rows rows of length n,
 *   env = | IDFT( H . DFT(in) ) |,  H[0] = 1, H[k] = 2 for 0 < k < n/2, H[n/2] = 1 (n even),
 *   H[k] = 0 otherwise (circular, no padding).
 *   in, env  float [n_rows][n]  (in == env allowed: in place)
 *   row_max  float [n_rows] maximum of each env row, or NULL.
 * 8 <= n <= 2048 and every prime factor of n at most 31 (e.g. 1000, 1024, 1408, 1664, 950).
 */
int usbf_envelope(const float* in, int64_t n_rows, int32_t n, float* env, float* row_max,
                  hipStream_t stream);

/*
 * Envelope by IQ demodulation with frequency compounding (Sec. 2 method list item 3, the
 * paper's own envelope node): each row is mixed down to baseband for every band k, low-passed
 * and its magnitude taken; the bands are averaged:
 *   env[n] = (2 / K) sum_k | sum_m g_k[m] in[n + c - m] |,  g_k[m] = h[m] exp(2 pi i f_k (m - c) / fs)
 * (mixing and low-passing, up to a unit-magnitude phase), with h the Hamming-windowed sinc of
 * n_taps = 2c + 1 taps, cutoff bandwidth / 2, unit gain at DC; samples outside the row are 0.
 * A tone of amplitude A at a band's centre has envelope A.
 *   in, env   float [n_rows][n] device (in != env), 8 <= n <= 8192
 *   freqs     host float [n_bands], 0 < f_k < fs / 2;  1 <= n_bands <= 4
 *   n_taps    odd, 3..127;  0 < bandwidth <= fs
 *   row_max   float [n_rows] maximum of each env row, or NULL.
 */
int usbf_envelope_iq(const float* in, int64_t n_rows, int32_t n, float fs, const float* freqs, int32_t n_bands,
                     float bandwidth, int32_t n_taps, float* env, float* row_max, hipStream_t stream);

/*
 * Coherent compounding (plane-wave imaging, Sec. 2: every line is beamformed once per steered
 * plane wave and the results are averaged before detection):
 *   out[f][i] = (1 / n_groups) sum_g in[f][g][i],  summed in group order.
 *   in   float [n_frames][n_groups][group_len] device;  out float [n_frames][group_len] device,
 *        not overlapping in.  1 <= n_frames <= 65535.
 */
int usbf_compound(const float* in, int32_t n_frames, int32_t n_groups, int64_t group_len, float* out,
                  hipStream_t stream);

/*
 * Weighted combination of beamformed lines (overlapping multi-line layouts: a line between
 * two transmits is interpolated from both transmits' beams of it; Sec. 3.3, Table 1: 255 lines from 128
 * transmits).  For every frame f, output line o and sample i:
 *   out[f][o][i] = sum_k w[o][k] * in[f][src[o][k]][i]
 * over the k = 0 .. k-1 whose source src[o][k] lies in [0, n_in) (others, e.g. -1, add
 * nothing), accumulated in binary32 in k order.
 *   in   float [n_frames][n_in][len]  (device);  out float [n_frames][n_out][len] (device),
 *        not overlapping in
 *   src  int32 [n_out][k], w float [n_out][k] (device)
 * 1 <= n_frames, n_out <= 65535; 1 <= k <= 64.
 */
int usbf_combine_lines(const float* in, int32_t n_frames, int32_t n_in, int64_t len,
                       const int32_t* src, const float* w, int32_t k, int32_t n_out,
                       float* out, hipStream_t stream);

/*
 * Log compression to a display range (Sec. 1 pipeline list; Sec. 2 method list item 4):
 *   out = clamp(1 + (20 / dyn_range_db) log10(env / ref), 0, 1),  out = 0 where env <= 0,
 * with ref the given reference, or when ref <= 0 the maximum of each frame.
 *   env, out float [n_frames][frame_len] (in place allowed).
 *   ws: device workspace of at least usbf_workspace_bytes(USBF_OP_LOG_COMPRESS, n_frames, 0, 0)
 *   bytes when ref <= 0 (may be NULL otherwise).
 */
int usbf_log_compress(const float* env, int32_t n_frames, int64_t frame_len, float dyn_range_db,
                      float ref, float* out, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * Scan conversion of line data onto a Cartesian grid (Sec. 1 pipeline list, last step;
 * Sec. 2 method list item 5): bilinear (kind 0, 2) or trilinear (kind 1) interpolation in
 * (line coordinate, range).  The integer cell indices follow the binary32 rule documented
 * with usbf_scan_index_map().
 *   in  float [n_frames][n_lines][scan->n_depth], n_lines = n_u (2D) or n_u * n_v (3D)
 *   out float [n_frames][grid]
 */
int usbf_scan_convert(const float* in, int32_t n_frames, const usbf_scan* scan, float* out,
                      hipStream_t stream);

/*
 * Log compression fused into scan conversion: out = scan_convert(log_compress(env)) with the
 * same results as the two calls in sequence (the paper's order: envelope, log compression,
 * scan conversion).  ref <= 0 uses each frame's maximum; if row_max (the envelope's
 * per-row maxima, [n_frames][n_lines]) is given it supplies that maximum, otherwise it is
 * computed.  ws as for usbf_log_compress.
 */
int usbf_log_scan_convert(const float* env, const float* row_max, int32_t n_frames,
                          const usbf_scan* scan, float dyn_range_db, float ref, float* out,
                          void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * The whole receive pipeline, channel data to display image: beamform -> envelope ->
 * log compression (frame maximum reference) -> scan conversion.
 *   rf     int16 [n_frames][n_tx][n_el][n_samples]
 *   image  float [n_frames][grid]
 *   ws     at least usbf_workspace_bytes(USBF_OP_BMODE, n_frames, n_lines, n_depth) bytes.
 * scan->n_depth must equal rx->n_depth and the scan's line count must equal n_lines.
 */
int usbf_bmode(const int16_t* rf, int32_t n_frames, const usbf_geometry* geom, const usbf_rx* rx,
               const usbf_scan* scan, float dyn_range_db, float* image, void* ws, size_t ws_bytes,
               hipStream_t stream);

/*
 * usbf_bmode without a workspace argument, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same stages and results as usbf_bmode, with the workspace taken from a buffer the library
 * holds on each GPU it runs on (USBF_NOALLOC_SCRATCH_BYTES, allocated with the library's code
 * object and kept until the process ends).  The call itself allocates nothing.
 *   Requests whose usbf_workspace_bytes(USBF_OP_BMODE, n_frames, n_lines, n_depth) exceeds
 *   USBF_NOALLOC_SCRATCH_BYTES fail with USBF_EUNSUPPORTED before anything is enqueued (e.g. up
 *   to 15 frames of 256 lines x 2048 depths, or 8 volumes of 1024 lines x 1000 depths).
 *   Every call on one GPU shares that GPU's buffer: calls that overlap in time on one GPU
 *   (several streams or host threads) race and must be serialised by the caller.
 * Other arguments, limits and status codes as usbf_bmode().
 */
#define USBF_NOALLOC_SCRATCH_BYTES (32u << 20)
int usbf_bmode_noalloc(const int16_t* rf, int32_t n_frames, const usbf_geometry* geom, const usbf_rx* rx,
                       const usbf_scan* scan, float dyn_range_db, float* image, hipStream_t stream);

/* ---------------------------------------------------------------- adaptive apodization */

/*
 * Delayed channel samples (the beamformer's taps without weights or summation): for each
 * listed pixel, every element's channel sample linearly interpolated at the two-way travel
 * time of the binary32 delay rule (usbf_delay_index_map), 0 outside the record.  Input to the
 * minimum-variance weights and the learned apodization below; an extension beyond the
 * paper's delay-and-sum (Sec. 2 method list item 2).
 *   rf   int16 [n_frames][n_tx][n_el][n_samples]
 *   pix  int32 [n_pix][3] (frame, line, depth index); entries out of range give a row of zeros
 *   x    float [n_pix][n_el]
 */
int usbf_delay_gather(const int16_t* rf, int32_t n_frames, const usbf_geometry* geom, const usbf_rx* rx,
                      const int32_t* pix, int32_t n_pix, float* x, hipStream_t stream);

/*
 * Minimum-variance (Capon) apodization per pixel, spatially smoothed over subapertures of
 * `subap` elements with diagonal loading (Synnevaag, Austeng and Holm 2007):
 *   R = (1/K) sum_l x_l x_l^T, x_l = x[l .. l+subap-1], K = n_el - subap + 1  (binary32)
 *   (R + loading * trace(R)/subap * I) v = 1 by Cholesky factorisation     (binary64)
 *   w = v / 1^T v;  w_full[e] = (1/K) sum_{l: 0 <= e-l < subap} w[e-l];  y = w_full^T x
 *   (a pixel whose samples are all zero gets loading 1 in place of loading * trace / subap,
 *   i.e. uniform weights)
 *   x      float [n_pix][n_el];  w_full float [n_pix][n_el] or NULL;  y float [n_pix] or NULL.
 * subap must be 32 and subap <= n_el <= 256.
 */
int usbf_mv_weights(const float* x, int32_t n_pix, int32_t n_el, int32_t subap, float loading,
                    float* w_full, float* y, hipStream_t stream);

/*
 * Delayed channel samples at neighbouring depths, the input of temporally averaged minimum
 * variance (usbf_mv_weights_averaged): for each listed pixel (frame f, line l, depth j) the
 * samples of usbf_delay_gather at the n_avg depths j - n_avg/2 .. j + n_avg/2 of line l,
 * each clamped to 0 .. n_depth - 1 (at the ends of a line the edge depth repeats).
 *   pix  int32 [n_pix][3], as usbf_delay_gather (a listed pixel out of range gives n_avg rows
 *        of zeros);  n_avg odd, 1..255
 *   x    float [n_pix][n_avg][n_el]: row t of pixel p is depth j + t - n_avg/2 (clamped)
 * n_avg = 1 is usbf_delay_gather.  Same status codes as usbf_delay_gather, plus USBF_EINVAL
 * for an even or out-of-range n_avg.
 */
int usbf_delay_gather_depths(const int16_t* rf, int32_t n_frames, const usbf_geometry* geom, const usbf_rx* rx,
                             const int32_t* pix, int32_t n_pix, int32_t n_avg, float* x, hipStream_t stream);

/*
 * Minimum variance with temporal averaging (the same estimator, not in the paper): the
 * covariance also averages over n_avg neighbouring depth samples of the pixel's line,
 *   R = (1/(n_avg K)) sum_t sum_l x_{t,l} x_{t,l}^T   (binary32, rows in order t = 0 ..),
 * and the weights apply to the middle row, y = w_full^T x_{n_avg/2}.  Loading, solve and
 * expansion as usbf_mv_weights(), which is the case n_avg = 1 (bit for bit).
 *   x  float [n_pix][n_avg][n_el]: for each pixel the delayed samples at n_avg consecutive
 *      depths, as usbf_delay_gather_depths() writes them (clamped at the ends of a line);
 *   n_avg odd, 1..255; other arguments as usbf_mv_weights().
 */
int usbf_mv_weights_averaged(const float* x, int32_t n_pix, int32_t n_avg, int32_t n_el, int32_t subap,
                             float loading, float* w_full, float* y, hipStream_t stream);

/*
 * Analytic signal of channel traces, the input of the complex (analytic-signal) minimum-
 * variance estimator below (not in the paper; the usual form of that estimator): for each of
 * n_rows int16 traces of length n,
 *   za = IDFT( H . DFT(rf) ),  H as in usbf_envelope (circular over the trace, no padding),
 * written as binary32 (re, im) pairs.
 *   rf  int16 [n_rows][n] (e.g. [n_frames][n_tx][n_el][n_samples] with n_rows = n_frames n_tx n_el)
 *   za  float [n_rows][n][2], 8-byte aligned (USBF_EINVAL otherwise)
 * 8 <= n <= 4096 and every prime factor of n at most 31.
 */
int usbf_analytic_channels(const int16_t* rf, int64_t n_rows, int32_t n, float* za, hipStream_t stream);

/*
 * Delayed complex samples: usbf_delay_gather applied to analytic channel data, the same
 * taps (binary32 delay rule; linear interpolation of the real and imaginary parts at the same
 * fraction; 0 outside the record, for out-of-range pixels and for lines without a transmit).
 *   za  float [n_frames][n_tx][n_el][n_samples][2] (usbf_analytic_channels output)
 *   pix int32 [n_pix][3] (frame, line, depth index)
 *   z   float [n_pix][n_el][2]
 */
int usbf_delay_gather_complex(const float* za, int32_t n_frames, const usbf_geometry* geom, const usbf_rx* rx,
                              const int32_t* pix, int32_t n_pix, float* z, hipStream_t stream);

/*
 * Minimum variance on the delayed analytic signal (the complex form of usbf_mv_weights, not
 * in the paper): the Hermitian spatially smoothed covariance
 *   R = (1/K) sum_l z_l z_l^H,  z_l = z[l .. l+subap-1], K = n_el - subap + 1       (binary32)
 *   (R + loading * trace(R)/subap * I) v = 1 by the complex Cholesky factorisation R = C C^H
 *                                                                                    (binary64)
 *   w = v / 1^T v;  w_full[e] = (1/K) sum_{l: 0 <= e-l < subap} w[e-l];  y = w_full^H z
 * (all-zero pixels: uniform weights, as usbf_mv_weights).  |y| is the pixel's envelope.  For
 * real z the results are those of usbf_mv_weights (imaginary parts 0).
 *   z      float [n_pix][n_el][2];  w_full float [n_pix][n_el][2] or NULL;  y float [n_pix][2] or NULL.
 * subap must be 32 and subap <= n_el <= 256.
 */
int usbf_mv_weights_complex(const float* z, int32_t n_pix, int32_t n_el, int32_t subap, float loading,
                            float* w_full, float* y, hipStream_t stream);

/*
 * Learned apodization: a 1D convolutional network -- four layers, 32 channels, kernel 5,
 * ReLU between layers, "same" zero padding -- maps the delayed samples x of a pixel
 * (normalised by their RMS) to one weight per element; trained to reproduce minimum-variance
 * weights (loss = mean over pixels and elements of (n_el w - n_el w_target)^2, Adam with
 * beta 0.9 / 0.999, eps 1e-8).  All products run on the matrix cores with bfloat16 operands
 * (layer inputs, weights and back-propagated gradients rounded to nearest even) and binary32
 * accumulation; the master weights are binary32.
 *   state   caller-owned device buffer of usbf_apodnet_state_bytes(): parameters, Adam moments,
 *           step count and the weights packed for the matrix cores.
 *   params  float [10657] = W1[32][1][5] b1[32] W2[32][32][5] b2[32] W3[32][32][5] b3[32]
 *           W4[1][32][5] b4[1] (device), copied in by usbf_apodnet_init (moments reset).
 *   x, w, w_target  float [n_pix][n_el], n_el a multiple of 32 in 32..256 (LDS-resident rows).
 *   ws      workspace of usbf_workspace_bytes(USBF_OP_APODNET_TRAIN, n_pix, n_el, 0) bytes for
 *           the train step and the gradients; the forward pass keeps its activations in LDS and
 *           needs none (usbf_workspace_bytes(USBF_OP_APODNET, ...) = 0, ws may be NULL).
 *   loss    device float receiving the step's loss (before the update), or NULL.
 * usbf_apodnet_gradients returns the loss gradient [10657] without updating anything.
 */
size_t usbf_apodnet_state_bytes(void);
int32_t usbf_apodnet_num_params(void);
int usbf_apodnet_init(void* state, const float* params, hipStream_t stream);
int usbf_apodnet_forward(const void* state, const float* x, int32_t n_pix, int32_t n_el, float* w, void* ws,
                         size_t ws_bytes, hipStream_t stream);
int usbf_apodnet_train_step(void* state, const float* x, const float* w_target, int32_t n_pix, int32_t n_el,
                            float lr, float* loss, void* ws, size_t ws_bytes, hipStream_t stream);
int usbf_apodnet_gradients(const void* state, const float* x, const float* w_target, int32_t n_pix, int32_t n_el,
                           float* grad, void* ws, size_t ws_bytes, hipStream_t stream);
/*
 * Learned apodization applied in one pass: the network's weights for each pixel and the
 * weighted sum y[p] = sum_e w[p][e] x[p][e] (usbf_beamform_weighted, with y_fallback[p] where a
 * weight is not finite), without writing the weights unless w is given.
 *   x float [n_pix][n_el]; y_fallback float [n_pix] or NULL; w float [n_pix][n_el] or NULL;
 *   y float [n_pix].  No workspace.
 */
int usbf_apodnet_apply(const void* state, const float* x, int32_t n_pix, int32_t n_el, const float* y_fallback,
                       float* w, float* y, hipStream_t stream);

/*
 * Adaptively weighted sum: y[p] = sum_e w[p][e] x[p][e]; a pixel whose weights are not all
 * finite takes y_fallback[p] (the delay-and-sum value), if given.
 */
int usbf_beamform_weighted(const float* x, const float* w, const float* y_fallback, int32_t n_pix, int32_t n_el,
                           float* y, hipStream_t stream);

/* ---------------------------------------------------------------- batched, persistent */

/*
 * A batch of frames and volumes of different sizes, taken through the whole pipeline
 * (delay and sum -> envelope -> log compression -> scan conversion) by one persistent
 * delay-and-sum launch followed by the per-item epilogues, captured once in a HIP graph and
 * replayed by usbf_batch_run.  For streams of acquisitions whose geometry repeats (the
 * paper runs every acquisition through the same node graph, Sec. 2).
 *   rf       int16 [n_tx][n_el][n_samples], one frame or volume
 *   lines    float [n_lines][n_depth], receives the beamformed lines, then their envelope
 *   row_max  float [n_lines]
 *   image    float [grid] B-mode, reference = the item's maximum, dyn_range_db below it -> 0
 * All buffers are caller-owned device memory that must stay valid while the plan exists;
 * their contents (rf) may change between runs.  n_samples must be a multiple of 4 for every
 * item or for none; n_depth must satisfy usbf_envelope's length rule.
 */
typedef struct usbf_batch_item {
  const int16_t* rf;
  usbf_geometry geom;
  usbf_rx rx;
  usbf_scan scan;
  float dyn_range_db;
  float* lines;
  float* row_max;
  float* image;
} usbf_batch_item;

typedef struct usbf_batch_plan usbf_batch_plan;

/*
 * Launch shape of a plan (what usbf_autotune searches):
 *   groups_per_cu    workgroups per compute unit of the persistent launch, 1..8
 *   cost_order       1: work units of the most expensive items (most elements) first
 *   multi_line_tile  lines per tile for items with >= 4 lines per transmit: 4 (the lines of a
 *                    transmit share their staged channel data) or 1
 *   chunk_div        elements per chunk = the tile's largest chunk / chunk_div, 1..8
 */
typedef struct usbf_batch_shape {
  int32_t groups_per_cu;
  int32_t cost_order;
  int32_t multi_line_tile;
  int32_t chunk_div;
} usbf_batch_shape;

/*
 * Validates the items, uploads their descriptors, orders the work units (most expensive
 * items first), and captures the graph on `stream`.  tune_cache: path of a JSON file written
 * by usbf_autotune (NULL or missing entry: default launch shape).  The plan owns a few KB of
 * device memory and a graph; it is not thread-safe.
 */
int usbf_batch_plan_create(const usbf_batch_item* items, int32_t n_items, const char* tune_cache,
                           usbf_batch_plan** plan, hipStream_t stream);
/* The same with an explicit launch shape (EINVAL for a shape outside the ranges above). */
int usbf_batch_plan_create_shaped(const usbf_batch_item* items, int32_t n_items, const usbf_batch_shape* shape,
                                  usbf_batch_plan** plan, hipStream_t stream);
int usbf_batch_run(usbf_batch_plan* plan, hipStream_t stream);
int usbf_batch_plan_destroy(usbf_batch_plan* plan);
/* Launch shape of the plan. */
int usbf_batch_plan_shape(const usbf_batch_plan* plan, usbf_batch_shape* shape);

/*
 * Times the batch with every candidate launch shape (workgroups per compute unit 1..4 x
 * multi-line tile 4 or 1 x chunk divisor 1 or 2, cost order) by graph replays and records the
 * fastest in the JSON file `tune_cache`, keyed by the device architecture and a signature of
 * the item sizes.  Synchronises `stream`.
 */
int usbf_autotune(const usbf_batch_item* items, int32_t n_items, const char* tune_cache, hipStream_t stream);

#define USBF_OP_LOG_COMPRESS 1
#define USBF_OP_LOG_SCAN     2
#define USBF_OP_BMODE        3
#define USBF_OP_MV           4
#define USBF_OP_APODNET      5
#define USBF_OP_APODNET_TRAIN 6

/* Workspace bytes needed by operation `op` for the given sizes (0 if none). */
size_t usbf_workspace_bytes(int32_t op, int64_t n_frames, int64_t n_lines, int64_t n_depth);

/* ---------------------------------------------------------------- index maps (exported for tests) */

/*
 * The binary32 delay rule used by every beamforming kernel, evaluated for all
 * (line, depth, element): each operation one IEEE binary32 op rounded to nearest, sqrt and
 * division correctly rounded, no fused multiply-add, sums left to right.
 *   per line:  u_l = d_l / sqrt(d_l.d_l), u_t likewise;  D = o_l - o_t;  g = D.u_t;
 *              cl = u_l.u_t;  k = cl - 1;  U = D - g u_t;  V = u_l - cl u_t;
 *              same = (o_l, d_l) equal bit for bit to (o_t, d_t)
 *   constants: h = c / (fs + fs),  K = fs / c,  T0 = fs t0,  F2 = f_number + f_number
 *   per pixel: b = depth_start + depth_step j (integer);  r = (float)b * h
 *              a = same ? 0 : g + r k;   L2 = same ? 0 : |U + r V|^2
 *              m = a + (r - F);  den = sqrt(m m + L2) + |m|
 *              dtx = den > 0 ? a + (m >= 0 ? L2 : -L2) / den : a
 *   per element: x = e - o_l;  A = x.x;  B = x.u_l;  q = A - (r + r) B
 *              X = q + r r (0 if not > 0);  s = sqrt(X) + r;  drx = s > 0 ? q / s : 0
 *              dt = K (dtx + drx) - T0;  i0 = b + floor(dt);  phi = dt - floor(dt)
 *              active: F2 |x.x| <= r  (and F2 |x.y| <= r for matrix arrays)
 *              valid:  0 <= i0 <= S - 2
 * This is the exact travel time rearranged so that the large, exact part 2 r fs / c = b
 * never enters floating point.
 *   i0    int32 [n_lines][n_depth][n_el];  flags uint8 same shape, bit0 active, bit1 valid;
 *   phi   float same shape, or NULL.
 */
int usbf_delay_index_map(const usbf_geometry* geom, const usbf_rx* rx, int32_t* i0, uint8_t* flags,
                         float* phi, hipStream_t stream);

/*
 * The binary32 cell-index rule of the scan converter, per output pixel:
 *   x = x0 + (float)i * hx  (likewise y, z; separate multiply and add);
 *   kind 0: u = x, range = z;  kind 2: u = x / z, range = sqrt(x x + z z);
 *   kind 1: u = x / z, v = y / z, range = sqrt((x x + y y) + z z);  (kinds 1, 2 need z > 0)
 *   q = (range - r0) / dr;  iu = largest index with line_u[iu] <= u, capped at n_u - 2
 *   (iv likewise);  jd = floor(q) capped at n_depth - 2;
 *   inside iff line_u[0] <= u <= line_u[n_u-1] (likewise v) and 0 <= q <= n_depth - 1.
 *   base int32 [grid]: (line index of the lower corner) * n_depth + jd, or -1 outside.
 */
int usbf_scan_index_map(const usbf_scan* scan, int32_t* base, hipStream_t stream);

/* ---------------------------------------------------------------- status */
const char* usbf_status_string(int status);
const char* usbf_last_error_detail(void);
const char* usbf_version(void);

#ifdef __cplusplus
}
#endif
#endif /* USBF_H */
