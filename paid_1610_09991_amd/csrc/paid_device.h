// paid_device.h -- data layout and device helpers shared by the libpaid
// kernels (gfx950).  Library-internal: not part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace paid {

// ---------------------------------------------------------------------------
// Rule pair (Sec. 3): N = 4 intervals per axis for Q_N, 2N = 8 for Q_2N.
// A parent's four children share 17 coordinates per axis (9 + 9 - 1).
constexpr int kNF = 9;    // fine-rule nodes per axis of one rectangle
constexpr int kNCo = 5;   // coarse-rule nodes per axis
constexpr int kNX = 17;   // distinct coordinates per axis over 4 children
constexpr int kMaxL = 2;  // box basis order: up to 5 harmonics per axis
constexpr int kMaxNB = 2 * kMaxL + 1;
constexpr int kMaxMB = kMaxNB * kMaxNB;       // 25 box functions
constexpr int kMaxMU = kMaxMB * (kMaxMB + 1) / 2;

// ---------------------------------------------------------------------------
// Frequency-sum tables.  For one parameter row the scalar integrand depends
// on the energies only through the odd function
//   S(x) = T sum_{n in Z} hdot(w_n) / (i w_n - x),   hdot = d/dOmega theta^2
// (theta^2 itself for the non-differentiated bubble), because partial
// fractions give K_ph(a,b) = S[a,b] = (S(a)-S(b))/(a-b) and
// K_pp(a,b) = -S[a,-b].  S is analytic except at x = +-i w_n, so on each
// interval of x >= 0 it is a short Taylor series.  Intervals are uniform in
// s = asinh(x / (pi T)): the half-width of each is one tenth of the distance
// from its centre to the nearest singularity, which makes degree 15 exact to
// rounding and lets a divided difference of two close energies be formed on
// one polynomial without cancellation.
constexpr int kTabDeg = 15;
constexpr int kTabStride = 20;                 // c, 1/h, h, pad, coef[16]
constexpr double kTabDs = 0.2;                 // interval width in s
constexpr double kTabS1 = 0.09983407889920758; // asinh(0.1): central half-width
constexpr int kTabPts = 32;                    // Cauchy points per interval
constexpr double kTabRho = 2.0;                // Cauchy radius in half-widths
constexpr int kTabKTail = 24;                  // tail expansion terms
constexpr double kDdSwitch2 = 0.0025;          // (0.05)^2: close-pair switch

struct Entry {        // one parameter row
  double t, tp, mu, T, Om;
  double emax;        // bound of |eps| over the zone
  double w, inv_w;    // pi T and its inverse
  int J;              // number of intervals
  int nmats;          // Matsubara head terms used to build the table
  int kind;           // PAID_BUBBLE_DOT / PAID_BUBBLE / ...
  int tab_off;        // offset of this row's table (in doubles)
};

struct Ctr {          // one container (parameter row, transfer momentum, channel)
  int entry, ch;      // ch: 0 = pp, 1 = ph
  double cLx, sLx, cLy, sLy;  // cos/sin of l/2 per axis
};

// ---------------------------------------------------------------------------
// Region codes: depth in bits 56..63, ix in 28..55, iy in 0..27.
__host__ __device__ inline uint64_t make_code(int d, uint64_t ix, uint64_t iy) {
  return ((uint64_t)d << 56) | (ix << 28) | iy;
}
__host__ __device__ inline int code_depth(uint64_t c) { return (int)(c >> 56); }
__host__ __device__ inline uint64_t code_ix(uint64_t c) { return (c >> 28) & 0xFFFFFFFull; }
__host__ __device__ inline uint64_t code_iy(uint64_t c) { return c & 0xFFFFFFFull; }

// ---------------------------------------------------------------------------
// Frequency-sum table evaluation.
__device__ inline int tab_index(const Entry &e, double ax) {
  float v = (float)(ax * e.inv_w);
  float s = __logf(v + __fsqrt_rn(fmaf(v, v, 1.0f)));
  int j = (s < (float)kTabS1) ? 0 : 1 + (int)((s - (float)kTabS1) * (float)(1.0 / kTabDs));
  return j < e.J - 1 ? j : e.J - 1;
}

__device__ inline double tab_poly(const double *cf, double t) {
  double r = cf[kTabDeg];
#pragma unroll
  for (int k = kTabDeg - 1; k >= 0; --k) r = fma(r, t, cf[k]);
  return r;
}

// S(x) for any real x (odd function)
__device__ inline double S_eval(const Entry &e, const double *tab, double x) {
  double ax = fabs(x);
  int j = tab_index(e, ax);
  const double *row = tab + j * kTabStride;
  if (j == 0) return tab_poly(row + 4, x * row[1]);  // central interval, centred at 0
  double v = tab_poly(row + 4, (ax - row[0]) * row[1]);
  return x < 0.0 ? -v : v;
}

// divided difference S[x, y]
__device__ inline double S_dd(const Entry &e, const double *tab, double x, double y) {
  double d = x - y, m = 0.5 * (x + y);
  if (d * d >= kDdSwitch2 * (m * m + e.w * e.w)) return (S_eval(e, tab, x) - S_eval(e, tab, y)) / d;
  int j = tab_index(e, fabs(m));
  const double *row = tab + j * kTabStride;
  double tx, ty;
  if (j == 0) {
    tx = x * row[1];
    ty = y * row[1];
  } else {
    if (m < 0.0) { x = -x; y = -y; }  // S[x,y] = S[-x,-y] for odd S
    tx = (x - row[0]) * row[1];
    ty = (y - row[0]) * row[1];
  }
  // Horner at tx carries the quotient coefficients; Horner of those at ty is
  // the divided difference of the polynomial (no subtraction of values).
  const double *cf = row + 4;
  double q = cf[kTabDeg], r = 0.0;
#pragma unroll
  for (int k = kTabDeg - 1; k >= 0; --k) {
    r = fma(r, ty, q);
    q = fma(q, tx, cf[k]);
  }
  return r * row[1];
}

// kernel K_j(a, b): ph = S[a,b], pp = -S[a,-b].  Branch-free in the data:
// both the two-value and the one-polynomial forms run in the same loop, so
// lanes of a wavefront never diverge on the node's energies.
__device__ inline double K_eval(const Entry &e, const double *tab, int ch, double a, double b) {
  const double x = a, y = ch ? b : -b;
  const double d = x - y, m = 0.5 * (x + y);
  const bool close = d * d < kDdSwitch2 * (m * m + e.w * e.w);
  const double *rx, *ry;
  double tx, ty, sx = 1.0, sy = 1.0;
  if (close) {
    int j = tab_index(e, fabs(m));
    rx = ry = tab + j * kTabStride;
    double xx = x, yy = y;
    if (j != 0 && m < 0.0) { xx = -x; yy = -y; }  // S[x,y] = S[-x,-y]
    tx = (xx - rx[0]) * rx[1];
    ty = (yy - rx[0]) * rx[1];
  } else {
    int jx = tab_index(e, fabs(x)), jy = tab_index(e, fabs(y));
    rx = tab + jx * kTabStride;
    ry = tab + jy * kTabStride;
    tx = jx == 0 ? x * rx[1] : (fabs(x) - rx[0]) * rx[1];
    ty = jy == 0 ? y * ry[1] : (fabs(y) - ry[0]) * ry[1];
    if (jx != 0 && x < 0.0) sx = -1.0;
    if (jy != 0 && y < 0.0) sy = -1.0;
  }
  // q: Horner at tx on rx; py: Horner at ty on ry; r: Horner at ty of the
  // quotient coefficients of q, i.e. the divided difference on one polynomial
  const double *cx = rx + 4, *cy = ry + 4;
  double q = cx[kTabDeg], py = cy[kTabDeg], r = 0.0;
#pragma unroll 4
  for (int k = kTabDeg - 1; k >= 0; --k) {
    r = fma(r, ty, q);
    q = fma(q, tx, cx[k]);
    py = fma(py, ty, cy[k]);
  }
  double s = close ? r * rx[1] : (sx * q - sy * py) / d;
  return ch ? s : -s;
}

}  // namespace paid
