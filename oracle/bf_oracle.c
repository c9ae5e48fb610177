/*
 * FP64 reference bilateral filters -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg use
 * this file.  It shares no code with the GPU library: it evaluates the two
 * filters of the paper straight from their definitions, one output pixel at a
 * time, in double precision, with no blocking, separability or reordering.
 *
 *   oracle_direct   -- eq. (1): the bilateral filter with the true range
 *                      kernel phi (Gaussian eq. (3), exponential, or a table
 *                      of phi on the integers 0..T).
 *   oracle_fourier  -- eq. (9): the same sum with phi replaced by the cosine
 *                      series of eq. (6), phi_K(t) = d_0 + sum_k d_k cos(k w t),
 *                      w = pi / T.  For integer differences |t| <= T the
 *                      series is tabulated once; otherwise it is summed.
 *
 * Conventions (readings of points the paper leaves open):
 *   - spatial kernel: Gaussian eq. (2) exp(-(x^2+y^2)/(2 sigma_s^2)) or a box
 *     (w = 1) on the window [-W, W]^2, scaled to unit sum (the scale cancels
 *     in eq. (1); unit sum is the assumption behind eq. (12));
 *   - borders: half-sample symmetric extension, index -1 -> 0, -2 -> 1,
 *     n -> n-1, n+1 -> n-2; requires W < min(H, width);
 *   - the image f is read with a row pitch (elements).
 */
#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { SPATIAL_GAUSSIAN = 0, SPATIAL_BOX = 1 };
enum { RANGE_GAUSSIAN = 0, RANGE_EXPONENTIAL = 1, RANGE_TABLE = 2 };

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Sets the number of threads later calls use (n >= 1); returns the previous
   number.  Only the timing of the CPU baseline changes it. */
int oracle_set_threads(int n) {
  const int prev = oracle_num_threads();
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#endif
  return prev;
}

/* half-sample symmetric reflection of an index into [0, n) (one fold) */
static long reflect(long i, long n) {
  if (i < 0) return -i - 1;
  if (i >= n) return 2 * n - i - 1;
  return i;
}

/* 1-D spatial profile on [-W, W]; the 2-D weight is w1[x] * w1[y] / s^2 */
static double* spatial_profile(int kind, double sigma_s, int W, double* sum_out) {
  double* w1 = (double*)malloc(sizeof(double) * (size_t)(2 * W + 1));
  double s = 0.0;
  for (int x = -W; x <= W; ++x) {
    double v = (kind == SPATIAL_BOX) ? 1.0 : exp(-(double)x * (double)x / (2.0 * sigma_s * sigma_s));
    w1[x + W] = v;
    s += v;
  }
  *sum_out = s;
  return w1;
}

/* centre weight w(0) of the unit-sum 2-D spatial kernel */
double oracle_center_weight(int kind, double sigma_s, int W) {
  double s;
  double* w1 = spatial_profile(kind, sigma_s, W, &s);
  double c = w1[W] * w1[W] / (s * s);
  free(w1);
  return c;
}

/* the true range kernel phi(t) */
static double range_phi(int kind, double sigma_r, const double* table, int T, double t) {
  double a = fabs(t);
  if (kind == RANGE_GAUSSIAN) return exp(-t * t / (2.0 * sigma_r * sigma_r));
  if (kind == RANGE_EXPONENTIAL) return exp(-a / sigma_r);
  /* table: phi sampled on the integers 0..T (symmetric kernel) */
  long r = (long)floor(a + 0.5);
  if (r > T) r = T;
  return table[r];
}

/* the shiftable cosine series phi_K(t), eq. (6) */
static double phi_series(const double* d, int K, int T, double t) {
  const double w = M_PI / (double)T;
  double s = d[0];
  for (int k = 1; k <= K; ++k) s += d[k] * cos((double)k * w * t);
  return s;
}

/*
 * Shared routine: evaluates eq. (1) or eq. (9) at the requested pixels.
 * mode 0: true kernel phi; mode 1: cosine series phi_K.
 * pix (length npix) lists linear output indices r * width + c; NULL means
 * every pixel in row-major order (npix is then ignored).
 * out[n], and optionally P[n], Q[n] (numerator / denominator of the ratio).
 */
static int run_filter(int mode, const float* f, long H, long Wd, long pitch,
                      int spatial_kind, double sigma_s, int W,
                      int range_kind, double sigma_r, const double* table,
                      const double* d, int K, int T,
                      const long* pix, long npix, double* out, double* P, double* Q) {
  if (!f || !out || H <= 0 || Wd <= 0 || pitch < Wd || W < 0 || W >= H || W >= Wd) return -1;
  if (mode == 1 && (!d || K < 0 || T < 1)) return -1;
  if (mode == 0 && range_kind == RANGE_TABLE && (!table || T < 1)) return -1;
  if (spatial_kind == SPATIAL_GAUSSIAN && !(sigma_s > 0.0)) return -1;
  double s;
  double* w1 = spatial_profile(spatial_kind, sigma_s, W, &s);
  const double norm = 1.0 / (s * s);
  /* phi_K on the integers -T..T, used whenever the difference is such an integer */
  double* tab = NULL;
  if (mode == 1) {
    tab = (double*)malloc(sizeof(double) * (size_t)(2 * T + 1));
    for (int t = -T; t <= T; ++t) tab[t + T] = phi_series(d, K, T, (double)t);
  }
  const long n_out = pix ? npix : H * Wd;
#pragma omp parallel for schedule(dynamic, 64)
  for (long n = 0; n < n_out; ++n) {
    const long lin = pix ? pix[n] : n;
    const long r = lin / Wd, c = lin % Wd;
    const double fi = (double)f[r * pitch + c];
    double num = 0.0, den = 0.0;
    for (int jy = -W; jy <= W; ++jy) {
      const long rr = reflect(r - jy, H);
      for (int jx = -W; jx <= W; ++jx) {
        const long cc = reflect(c - jx, Wd);
        const double fj = (double)f[rr * pitch + cc];
        const double t = fj - fi;
        double ph;
        if (mode == 0) {
          ph = range_phi(range_kind, sigma_r, table, T, t);
        } else {
          const double tr = floor(t + 0.5);
          if (tr == t && fabs(t) <= (double)T) ph = tab[(long)t + T];
          else ph = phi_series(d, K, T, t);
        }
        const double wgt = w1[jy + W] * w1[jx + W] * norm * ph;
        num += wgt * fj;
        den += wgt;
      }
    }
    out[n] = num / den;
    if (P) P[n] = num;
    if (Q) Q[n] = den;
  }
  free(w1);
  free(tab);
  return 0;
}

int oracle_direct(const float* f, long H, long Wd, long pitch,
                  int spatial_kind, double sigma_s, int W,
                  int range_kind, double sigma_r, const double* table, int T,
                  const long* pix, long npix, double* out, double* P, double* Q) {
  return run_filter(0, f, H, Wd, pitch, spatial_kind, sigma_s, W, range_kind, sigma_r, table,
                    NULL, 0, T, pix, npix, out, P, Q);
}

int oracle_fourier(const float* f, long H, long Wd, long pitch,
                   int spatial_kind, double sigma_s, int W,
                   const double* d, int K, int T,
                   const long* pix, long npix, double* out, double* P, double* Q) {
  return run_filter(1, f, H, Wd, pitch, spatial_kind, sigma_s, W, RANGE_GAUSSIAN, 1.0, NULL,
                    d, K, T, pix, npix, out, P, Q);
}
