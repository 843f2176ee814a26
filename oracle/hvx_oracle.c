/*
 * CPU reference for OpenVX-style point and local operators.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark load this file's library.  The GPU library
 * neither includes, links nor calls anything from here, and nothing here is
 * taken from the GPU library.
 *
 * Every function below is the plain definition of one graph node, applied to
 * a whole image that is stored densely (row pitch = width * element size).
 * Each node applies its own border mode to its own inputs: this is the
 * node-by-node execution model of an OpenVX graph (Section 3.1): every
 * intermediate image exists in full before its consumers run.
 *
 * Point operators compute an output pixel from the input pixels at the same
 * position; local operators compute it from a window of input pixels around
 * that position (Section 4, Table 2).  The paper defers each function's
 * arithmetic to the OpenVX specification; the reading taken for each one is
 * stated at the function.
 *
 * Floating-point nodes (the corner response) run in double precision.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#define ORC_BORDER_UNDEFINED 0
#define ORC_BORDER_CONSTANT 1
#define ORC_BORDER_REPLICATE 2
#define ORC_BORDER_MIRROR 3
#define ORC_BORDER_REPEAT 4

/* ---- border fetch (one per input element type) ------------------------- */
/* REPLICATE: nearest in-image pixel.  CONSTANT: the constant outside.
 * MIRROR: the image reflected about its first and last pixel (reflect-101:
 * ... c b | a b c ... x y | x w ...), repeated as often as needed; a single
 * row or column repeats its pixel.
 * REPEAT: the image tiled periodically in both directions, so position x
 * reads pixel x mod n (the non-negative remainder).
 * UNDEFINED: the result there is unspecified; the replicated value is used so
 * that the computation is defined, and callers exclude those pixels. */

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

static int mirror_index(int x, int n) {
  if (n == 1) return 0;
  while (x < 0 || x >= n) {
    if (x < 0) x = -x;
    if (x >= n) x = 2 * (n - 1) - x;
  }
  return x;
}

static int repeat_index(int x, int n) {
  int r = x % n;
  return r < 0 ? r + n : r;
}

/* The in-image position read for (x, y) outside the image under MIRROR,
 * REPEAT, REPLICATE or UNDEFINED. */
static void outside_pos(int border, int w, int h, int* x, int* y) {
  if (border == ORC_BORDER_MIRROR) {
    *x = mirror_index(*x, w);
    *y = mirror_index(*y, h);
  } else if (border == ORC_BORDER_REPEAT) {
    *x = repeat_index(*x, w);
    *y = repeat_index(*y, h);
  }
  *x = clampi(*x, 0, w - 1);
  *y = clampi(*y, 0, h - 1);
}

static int64_t fetch_u8(const uint8_t* img, int w, int h, int x, int y, int border, int64_t c) {
  if (x < 0 || y < 0 || x >= w || y >= h) {
    if (border == ORC_BORDER_CONSTANT) return c;
    outside_pos(border, w, h, &x, &y);
  }
  return img[(size_t)y * w + x];
}

static int64_t fetch_s16(const int16_t* img, int w, int h, int x, int y, int border, int64_t c) {
  if (x < 0 || y < 0 || x >= w || y >= h) {
    if (border == ORC_BORDER_CONSTANT) return c;
    outside_pos(border, w, h, &x, &y);
  }
  return img[(size_t)y * w + x];
}

static double fetch_f64(const double* img, int w, int h, int x, int y, int border, double c) {
  if (x < 0 || y < 0 || x >= w || y >= h) {
    if (border == ORC_BORDER_CONSTANT) return c;
    outside_pos(border, w, h, &x, &y);
  }
  return img[(size_t)y * w + x];
}

/* ---- point operators ---------------------------------------------------- */

/* Channel extract, luma of UYVY 4:2:2 (bytes U Y0 V Y1 per pixel pair):
 * Y(x, y) is byte 2x+1 of row y.  The input row holds 2*w bytes. */
void orc_channel_extract_y(const uint8_t* uyvy, uint8_t* out, int w, int h) {
  for (int y = 0; y < h; ++y)
    for (int x = 0; x < w; ++x) out[(size_t)y * w + x] = uyvy[(size_t)y * 2 * w + 2 * x + 1];
}

/* Floor of the square root of s, exact: a start from the double square root,
 * then corrected until q*q <= s < (q+1)*(q+1). */
static uint64_t isqrt_exact(uint64_t s) {
  uint64_t q = (uint64_t)sqrt((double)s);
  while (q * q > s) --q;
  while ((q + 1) * (q + 1) <= s) ++q;
  return q;
}

/* Magnitude of a gradient pair: sqrt(gx^2 + gy^2) rounded to nearest.  For an
 * integer s, sqrt(s) is never exactly halfway between two integers, so the
 * rounding is q + 1 exactly when s - q^2 > q (q = floor(sqrt(s))).  The
 * result saturates to the S16 maximum. */
void orc_magnitude(const int16_t* gx, const int16_t* gy, int16_t* out, int w, int h) {
  size_t n = (size_t)w * h;
  for (size_t i = 0; i < n; ++i) {
    int64_t a = gx[i], b = gy[i];
    uint64_t s = (uint64_t)(a * a + b * b);
    uint64_t q = isqrt_exact(s);
    uint64_t m = q + ((s - q * q) > q ? 1 : 0);
    out[i] = (int16_t)(m > 32767 ? 32767 : m);
  }
}

/* Phase (orientation) of a gradient pair, quantised to 256 levels per turn:
 * theta = atan2(gy, gx) taken in [0, 2*pi), then round(theta * 256 / (2*pi))
 * modulo 256.  atan2(0, 0) = 0. */
void orc_phase(const int16_t* gx, const int16_t* gy, uint8_t* out, int w, int h) {
  const double two_pi = 6.283185307179586476925286766559;
  size_t n = (size_t)w * h;
  for (size_t i = 0; i < n; ++i) {
    double t = atan2((double)gy[i], (double)gx[i]);
    if (t < 0) t += two_pi;
    long q = (long)floor(t * 256.0 / two_pi + 0.5);
    out[i] = (uint8_t)(q & 255);
  }
}

/* Binary threshold: true_v where in > thresh (strict), false_v elsewhere.
 * kind 0: U8 input, 1: S16 input, 2: double input. */
void orc_threshold(const void* in, int kind, double thresh, int true_v, int false_v, uint8_t* out, int w,
                   int h) {
  size_t n = (size_t)w * h;
  for (size_t i = 0; i < n; ++i) {
    double v;
    if (kind == 0)
      v = ((const uint8_t*)in)[i];
    else if (kind == 1)
      v = ((const int16_t*)in)[i];
    else
      v = ((const double*)in)[i];
    out[i] = (uint8_t)(v > thresh ? true_v : false_v);
  }
}

/* Add with an overflow policy: sum = a + b in wide integers, then either
 * saturated to the output range (policy 0) or wrapped to the output width
 * (policy 1).  kind_a/kind_b/kind_out: 0 = U8, 1 = S16. */
void orc_add(const void* a, int kind_a, const void* b, int kind_b, void* out, int kind_out, int policy, int w,
             int h) {
  size_t n = (size_t)w * h;
  for (size_t i = 0; i < n; ++i) {
    int64_t va = kind_a == 0 ? ((const uint8_t*)a)[i] : ((const int16_t*)a)[i];
    int64_t vb = kind_b == 0 ? ((const uint8_t*)b)[i] : ((const int16_t*)b)[i];
    int64_t s = va + vb;
    if (kind_out == 0) {
      if (policy == 0) s = s < 0 ? 0 : (s > 255 ? 255 : s);
      ((uint8_t*)out)[i] = (uint8_t)(s & 255);
    } else {
      if (policy == 0) {
        s = s < -32768 ? -32768 : (s > 32767 ? 32767 : s);
      } else {
        s &= 0xFFFF;
        if (s >= 32768) s -= 65536;
      }
      ((int16_t*)out)[i] = (int16_t)s;
    }
  }
}

/* Product of two S16 images as a real number (the corner graph's gx*gx,
 * gy*gy and gx*gy planes).  Exact in double. */
void orc_multiply_f64(const int16_t* a, const int16_t* b, double* out, int w, int h) {
  size_t n = (size_t)w * h;
  for (size_t i = 0; i < n; ++i) out[i] = (double)a[i] * (double)b[i];
}

/* Corner response of the structure-tensor sums: R = det - k * trace^2 with
 * det = Sxx*Syy - Sxy^2 and trace = Sxx + Syy. */
void orc_harris_response(const double* sxx, const double* syy, const double* sxy, double k, double* out, int w,
                         int h) {
  size_t n = (size_t)w * h;
  for (size_t i = 0; i < n; ++i) {
    double det = sxx[i] * syy[i] - sxy[i] * sxy[i];
    double tr = sxx[i] + syy[i];
    out[i] = det - k * tr * tr;
  }
}

/* ---- local operators ---------------------------------------------------- */

/* Separable binomial smoothing of a U8 image with weights w (length n, odd),
 * sum over the full n x n window of w[i]*w[j]*in, then an arithmetic right
 * shift by `shift` (floor division by the weight total). */
static void binomial_u8(const uint8_t* in, uint8_t* out, int w, int h, int border, int c, const int* wt, int n,
                        int shift) {
  int r = n / 2;
  for (int y = 0; y < h; ++y)
    for (int x = 0; x < w; ++x) {
      int64_t s = 0;
      for (int j = -r; j <= r; ++j)
        for (int i = -r; i <= r; ++i) s += (int64_t)wt[i + r] * wt[j + r] * fetch_u8(in, w, h, x + i, y + j, border, c);
      out[(size_t)y * w + x] = (uint8_t)(s >> shift);
    }
}

/* Gaussian 3x3: weights (1 2 1) x (1 2 1), total 16, floor. */
void orc_gaussian3x3(const uint8_t* in, uint8_t* out, int w, int h, int border, int c) {
  static const int wt[3] = {1, 2, 1};
  binomial_u8(in, out, w, h, border, c, wt, 3, 4);
}

/* Gaussian 5x5: weights (1 4 6 4 1) x (1 4 6 4 1), total 256, floor. */
void orc_gaussian5x5(const uint8_t* in, uint8_t* out, int w, int h, int border, int c) {
  static const int wt[5] = {1, 4, 6, 4, 1};
  binomial_u8(in, out, w, h, border, c, wt, 5, 8);
}

/* Box 3x3: sum of the 9 window pixels divided by 9, floor. */
void orc_box3x3(const uint8_t* in, uint8_t* out, int w, int h, int border, int c) {
  for (int y = 0; y < h; ++y)
    for (int x = 0; x < w; ++x) {
      int64_t s = 0;
      for (int j = -1; j <= 1; ++j)
        for (int i = -1; i <= 1; ++i) s += fetch_u8(in, w, h, x + i, y + j, border, c);
      out[(size_t)y * w + x] = (uint8_t)(s / 9);
    }
}

/* Dilate 3x3 / Erode 3x3 (Table 2, local operators with a MAX / MIN
 * reduction): the largest / smallest of the 9 window pixels. */
void orc_dilate3x3(const uint8_t* in, uint8_t* out, int w, int h, int border, int c) {
  for (int y = 0; y < h; ++y)
    for (int x = 0; x < w; ++x) {
      int64_t m = 0;
      for (int j = -1; j <= 1; ++j)
        for (int i = -1; i <= 1; ++i) {
          int64_t v = fetch_u8(in, w, h, x + i, y + j, border, c);
          if (v > m) m = v;
        }
      out[(size_t)y * w + x] = (uint8_t)m;
    }
}

void orc_erode3x3(const uint8_t* in, uint8_t* out, int w, int h, int border, int c) {
  for (int y = 0; y < h; ++y)
    for (int x = 0; x < w; ++x) {
      int64_t m = 255;
      for (int j = -1; j <= 1; ++j)
        for (int i = -1; i <= 1; ++i) {
          int64_t v = fetch_u8(in, w, h, x + i, y + j, border, c);
          if (v < m) m = v;
        }
      out[(size_t)y * w + x] = (uint8_t)m;
    }
}

/* Median 3x3 (Table 2, local operator with a MEDIAN reduction): the 9
 * window pixels sorted ascending (insertion sort), the fifth one. */
void orc_median3x3(const uint8_t* in, uint8_t* out, int w, int h, int border, int c) {
  for (int y = 0; y < h; ++y)
    for (int x = 0; x < w; ++x) {
      int64_t v[9];
      int n = 0;
      for (int j = -1; j <= 1; ++j)
        for (int i = -1; i <= 1; ++i) {
          int64_t t = fetch_u8(in, w, h, x + i, y + j, border, c);
          int k = n++;
          while (k > 0 && v[k - 1] > t) {
            v[k] = v[k - 1];
            --k;
          }
          v[k] = t;
        }
      out[(size_t)y * w + x] = (uint8_t)v[4];
    }
}

/* NonLinearFilter (Table 2, local operator): over the window pixels where
 * the cols x rows mask (row-major, centred) is nonzero, the median, the
 * minimum or the maximum (func 0, 1, 2).  The median of n values is the one
 * at index n / 2 of the ascending order (the upper one when n is even). */
void orc_nonlinear(const uint8_t* in, const uint8_t* mask, int cols, int rows, int func, uint8_t* out, int w, int h,
                   int border, int c) {
  const int rx = cols / 2, ry = rows / 2;
  for (int y = 0; y < h; ++y)
    for (int x = 0; x < w; ++x) {
      int64_t v[81];
      int n = 0;
      for (int j = -ry; j <= ry; ++j)
        for (int i = -rx; i <= rx; ++i) {
          if (!mask[(j + ry) * cols + (i + rx)]) continue;
          int64_t t = fetch_u8(in, w, h, x + i, y + j, border, c);
          int k = n++;
          while (k > 0 && v[k - 1] > t) {
            v[k] = v[k - 1];
            --k;
          }
          v[k] = t;
        }
      int64_t r = func == 1 ? v[0] : (func == 2 ? v[n - 1] : v[n / 2]);
      out[(size_t)y * w + x] = (uint8_t)r;
    }
}

/* NonMaxSuppression (Table 2, local operator) over a win x win window of a
 * U8 (s16 == 0) or S16 image: the pixel is kept where every window pixel
 * before it in raster order is smaller and every one after it is not larger,
 * otherwise it becomes the format's minimum (0, -32768).  Of a plateau of
 * equal maxima the first pixel in raster order is kept. */
void orc_nonmax(const void* in, void* out, int s16, int win, int w, int h, int border, int c) {
  const int r = win / 2;
  for (int y = 0; y < h; ++y)
    for (int x = 0; x < w; ++x) {
      int64_t p = s16 ? fetch_s16((const int16_t*)in, w, h, x, y, border, c)
                      : fetch_u8((const uint8_t*)in, w, h, x, y, border, c);
      int keep = 1;
      for (int j = -r; j <= r; ++j)
        for (int i = -r; i <= r; ++i) {
          if (i == 0 && j == 0) continue;
          int64_t q = s16 ? fetch_s16((const int16_t*)in, w, h, x + i, y + j, border, c)
                          : fetch_u8((const uint8_t*)in, w, h, x + i, y + j, border, c);
          int before = j < 0 || (j == 0 && i < 0);
          if (before ? q >= p : q > p) keep = 0;
        }
      if (s16) ((int16_t*)out)[(size_t)y * w + x] = (int16_t)(keep ? p : -32768);
      else ((uint8_t*)out)[(size_t)y * w + x] = (uint8_t)(keep ? p : 0);
    }
}

/* Sobel 3x3 gradients of a U8 image.  x grows to the right, y downwards.
 * gx = (right column - left column) weighted (1 2 1) along y;
 * gy = (bottom row - top row) weighted (1 2 1) along x.
 * Either output may be NULL. */
void orc_sobel3x3(const uint8_t* in, int16_t* gx, int16_t* gy, int w, int h, int border, int c) {
  static const int kx[3][3] = {{-1, 0, 1}, {-2, 0, 2}, {-1, 0, 1}};
  static const int ky[3][3] = {{-1, -2, -1}, {0, 0, 0}, {1, 2, 1}};
  for (int y = 0; y < h; ++y)
    for (int x = 0; x < w; ++x) {
      int64_t sx = 0, sy = 0;
      for (int j = -1; j <= 1; ++j)
        for (int i = -1; i <= 1; ++i) {
          int64_t v = fetch_u8(in, w, h, x + i, y + j, border, c);
          sx += kx[j + 1][i + 1] * v;
          sy += ky[j + 1][i + 1] * v;
        }
      if (gx) gx[(size_t)y * w + x] = (int16_t)sx;
      if (gy) gy[(size_t)y * w + x] = (int16_t)sy;
    }
}

/* Convolution of a U8 image with an integer mask of cols x rows (both odd),
 * coefficients row-major, centre at (cols/2, rows/2):
 *   S(x, y) = sum_{i,j} m(i, j) * in(x - i, y - j)
 * (a true convolution: the mask is applied rotated by 180 degrees), then
 * S / scale truncated toward zero and saturated to the output type
 * (out_kind 0 = U8, 1 = S16). */
void orc_convolve(const uint8_t* in, const int16_t* coeffs, int cols, int rows, int scale, void* out, int out_kind,
                  int w, int h, int border, int c) {
  int rx = cols / 2, ry = rows / 2;
  for (int y = 0; y < h; ++y)
    for (int x = 0; x < w; ++x) {
      int64_t s = 0;
      for (int j = -ry; j <= ry; ++j)
        for (int i = -rx; i <= rx; ++i)
          s += (int64_t)coeffs[(j + ry) * cols + (i + rx)] * fetch_u8(in, w, h, x - i, y - j, border, c);
      int64_t q = s / scale; /* C division truncates toward zero */
      if (out_kind == 0) {
        q = q < 0 ? 0 : (q > 255 ? 255 : q);
        ((uint8_t*)out)[(size_t)y * w + x] = (uint8_t)q;
      } else {
        q = q < -32768 ? -32768 : (q > 32767 ? 32767 : q);
        ((int16_t*)out)[(size_t)y * w + x] = (int16_t)q;
      }
    }
}

/* Unnormalised 5x5 box sum of a real-valued image (the corner graph's
 * structure-tensor window). */
void orc_box5x5_f64(const double* in, double* out, int w, int h, int border, double c) {
  for (int y = 0; y < h; ++y)
    for (int x = 0; x < w; ++x) {
      double s = 0.0;
      for (int j = -2; j <= 2; ++j)
        for (int i = -2; i <= 2; ++i) s += fetch_f64(in, w, h, x + i, y + j, border, c);
      out[(size_t)y * w + x] = s;
    }
}

/* S16 input variant of the border fetch, exported for completeness of the
 * reference (used by tests that run local operators on S16 data). */
int64_t orc_fetch_s16(const int16_t* img, int w, int h, int x, int y, int border, int64_t c) {
  return fetch_s16(img, w, h, x, y, border, c);
}
