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
// K_pp(a,b) = -S[a,-b].  S is analytic except at x = +-i w_n, so on short
// intervals of x >= 0 it is a short Taylor series.  In units of w = pi T
// (the distance of the nearest singularity from the real axis) the
// intervals are: P + 1 central ones centred at 0, 1/P, ..., 1 with
// half-width 1/(2P), then P per octave, [2^e (1 + m/P), 2^e (1 + (m+1)/P)),
// m = 0..P-1, so the index follows from the exponent and top log2(P)
// mantissa bits of |x|/w.  Every half-width is at most 1/(2P) of the
// distance from its centre to the nearest singularity; with P = 8, degree 13
// is exact to rounding on the interval (and accurate out to 1.5 half-widths,
// where the divided difference of two close energies is formed on the
// polynomial of one of them).
// Row layout: -c/h, 1/h, coef[deg + 1] of P(t) = S(c + h t), padded to an odd
// number of doubles.  c/h is an integer (2j in the centre, 2P + 1 + 2m in an
// octave), so t = x/h - c/h is one fused multiply-add.  An odd stride in
// doubles spreads the rows that the lanes of a wave read at one coefficient
// over the LDS banks (with P = 8, 18 and 20 doubles are slower than 17, 16
// much slower).
constexpr int kTabDeg = 13;
constexpr int kTabLogOct = 3;                  // log2 of the intervals per octave
constexpr int kTabPerOct = 1 << kTabLogOct;    // intervals per octave above |x| = w
constexpr int kTabCentral = kTabPerOct + 1;    // central intervals
constexpr int kTabStride = (kTabDeg + 3) | 1;  // -c/h, 1/h, coef[deg + 1], odd
constexpr int kTabCoef = 2;                    // offset of the coefficients in a row
constexpr int kTabPts = 32;                    // Cauchy points per interval
constexpr double kTabRho = 2.0;                // Cauchy radius in half-widths
constexpr int kTabKTail = 24;                  // tail expansion terms
constexpr double kDdSwitch2 = 0.0004;          // (0.02)^2: close-pair switch

// interval j in units of w: centre c and half-width h (j >= 0)
__host__ __device__ inline void tab_interval(int j, double w, double &c, double &h) {
  constexpr double inv_p = 1.0 / kTabPerOct;
  if (j < kTabCentral) {
    c = w * (inv_p * j);
    h = w * (0.5 * inv_p);
  } else {
    const int k = j - kTabCentral, e = k / kTabPerOct, m = k - e * kTabPerOct;
    const double s = ldexp(w, e);
    c = s * (1.0 + inv_p * (m + 0.5));
    h = s * (0.5 * inv_p);
  }
}

// rows needed to cover |x| <= top
__host__ __device__ inline int tab_rows(double top, double w) {
  if (top < w) return kTabCentral;
  int E = 0;
  (void)frexp(top / w, &E);  // top/w in [2^(E-1), 2^E)
  return kTabCentral + kTabPerOct * E;
}

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
// interval of |x| (no transcendental: exponent and top mantissa bits of
// v = |x|/w).  Central intervals: jc = round(P v), at most P; octave
// intervals from the high word of v, whose bits above the top log2(P)
// mantissa bits are (exponent << log2(P) | m).  For v < 1 the octave index
// is at most jc and for v >= 1 at least P + 1 > jc, so the larger of the
// two is the interval: no compare or select.
__device__ inline int tab_index(const Entry &e, double ax) {
  const double v = fabs(ax) * e.inv_w;  // a negative zero is the interval of 0
  const int jc = min((int)fma(v, (double)kTabPerOct, 0.5), kTabPerOct);
  const unsigned hi = (unsigned)(__double_as_longlong(v) >> 32);
  const int jo = kTabCentral - 1023 * kTabPerOct + (int)(hi >> (20 - kTabLogOct));
  const int j = max(jc, jo);
  return j < e.J - 1 ? j : e.J - 1;
}

// FP32 copy of a per-pair error estimate (the stored E and the running sums
// built from it): rounded to nearest, except that a positive estimate below
// the smallest normal float is kept as that float, an upper bound, instead of
// flushing towards zero and passing a tolerance it does not meet.
__device__ inline float err_f32(double e) {
  const float f = (float)e;
  return (e > 0.0 && f < 1.17549435e-38f) ? 1.17549435e-38f : f;
}

// n / d for a normal, non-zero d: the hardware reciprocal estimate refined by
// two Newton-Raphson steps, then one residual correction of the quotient
// (Markstein's scheme); no scaling for extreme exponents, which the far
// pairs (|d| >= 0.02 w) never reach.
__device__ inline double div_nr(double n, double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(fma(-d, r, 1.0), r, r);
  r = fma(fma(-d, r, 1.0), r, r);
  const double q = n * r;
  return fma(fma(-d, q, n), r, q);
}

// kernel K_j(a, b): ph = S[a,b], pp = -S[a,-b], with x = a and y = b (ph) or
// -b (pp).  S is odd and S[x,y] = S[-x,-y], so both are flipped to x >= 0.
// Far pairs take two values, S[x,y] = (P_jx(tx) - sign(y) P_jy(ty))/(x - y);
// close pairs (|x - y| < 0.02 sqrt(x^2 + w^2)) take the divided difference on
// the polynomial of x's interval: Horner at tx carries the quotient
// coefficients, Horner of those at ty is the divided difference (no
// subtraction of values; there |ty| <= 1.5, a tenth of the radius of
// convergence in units of the half-width).  Both forms are written as one
// loop with the second row and argument chosen per lane (the compiler moves
// the chain that a lane's form does not use into a branch).  The sign
// flips are XORs of sign bits: x = |a|, y = +-b with the signs of a and of
// the channel (pp: -b), and the result's sign by the channel.
__device__ inline double K_eval(const Entry &e, const double *tab, int ch, double a, double b) {
  constexpr unsigned long long kSign = 0x8000000000000000ull;
  const unsigned long long sc = ch ? 0ull : kSign;
  const double x = fabs(a);
  const double y = __longlong_as_double(__double_as_longlong(b) ^ (__double_as_longlong(a) & kSign) ^ sc);
  const double d = x - y;
  const bool close = d * d < kDdSwitch2 * (x * x + e.w * e.w);
  const double ay = fabs(y);
  // row offsets by 24-bit multiplies (full rate; the 32-bit one is not)
  const double *rx = tab + __umul24(tab_index(e, x), kTabStride);
  const double *ry = close ? rx : tab + __umul24(tab_index(e, ay), kTabStride);
  const double tx = fma(x, rx[1], rx[0]);
  const double ty = fma(close ? y : ay, ry[1], ry[0]);
  const double *cx = rx + kTabCoef, *cy = ry + kTabCoef;
  double q = cx[kTabDeg], py = cy[kTabDeg], r = 0.0;
#pragma unroll
  for (int k = kTabDeg - 1; k >= 0; --k) {
    r = fma(r, ty, q);
    q = fma(q, tx, cx[k]);
    py = fma(py, ty, cy[k]);
  }
  const double sy = __longlong_as_double(__double_as_longlong(py) ^ (__double_as_longlong(y) & kSign));
  const double s = close ? r * rx[1] : div_nr(q - sy, d);
  return __longlong_as_double(__double_as_longlong(s) ^ sc);
}

}  // namespace paid
