// tables.hip -- per-parameter-row tables of the frequency-summed propagator
// product (Sec. 2: the frequency integral done in closed form per scale).
//
// For every parameter row the odd function
//   S(z) = T sum_{n in Z} W(w_n) / (i w_n - z) = -2 z T sum_{n >= 0} W(w_n) / (w_n^2 + z^2)
// with W = d/dOmega theta^2 = -4 Omega w^4/(w^2+Omega^2)^3 (or theta^2 for the
// non-differentiated bubble) is sampled on circles in the complex plane and
// turned into Taylor coefficients on real intervals (Cauchy's formula with a
// trapezoid rule in the angle, exponentially accurate).  The Matsubara sum
// is done directly for the first `nmats` frequencies; the rest is expanded
// in v = 1/w^2 (w_N^2 exceeds |z|^2 and Omega^2 sixteenfold, so the expansion
// converges geometrically) and summed with
//   sum_{n >= N} w_n^{-2k} = (2 pi T)^{-2k} zeta(2k, N + 1/2)  (Hurwitz zeta).
#include <math.h>

#include "launch.h"

namespace paid {

namespace {

constexpr double kPi = 3.14159265358979323846;

// Hurwitz zeta sum_{j >= 0} (q + j)^-s by Euler-Maclaurin after shifting q.
__device__ double hurwitz_zeta(double s, double q) {
  const double B2[10] = {1.0 / 6,   -1.0 / 30,        1.0 / 42,     -1.0 / 30,      5.0 / 66,
                         -691.0 / 2730, 7.0 / 6, -3617.0 / 510, 43867.0 / 798, -174611.0 / 330};
  int J = (int)ceil(s + 25.0 - q);
  if (J < 0) J = 0;
  double head = 0.0;
  for (int j = J - 1; j >= 0; --j) head += pow(q + j, -s);
  double a = q + J, as = pow(a, -s);
  double tail = a * as / (s - 1.0) + 0.5 * as;
  double term = s * as / a;  // s a^{-s-1}
  double fac = 2.0;          // (2i)!
  for (int i = 1; i <= 10; ++i) {
    tail += B2[i - 1] / fac * term;
    term *= (s + 2 * i - 1) * (s + 2 * i) / (a * a);
    fac *= (2.0 * i + 1) * (2.0 * i + 2);
  }
  return head + tail;
}

__global__ void k_zeta(const Entry *entries, int n, double *zeta) {
  int e = blockIdx.x, k = threadIdx.x;
  if (e >= n || k > kTabKTail) return;
  const Entry E = entries[e];
  double z = 0.0;
  if (k >= 1) z = pow(2.0 * kPi * E.T, -2.0 * k) * hurwitz_zeta(2.0 * k, E.nmats + 0.5);
  zeta[e * (kTabKTail + 1) + k] = z;
}


// S(z) at one complex point
__device__ double2 S_complex(const Entry &E, const double *zeta, double zr, double zi) {
  const double T = E.T, Om = E.Om, O2 = Om * Om;
  const double z2r = zr * zr - zi * zi, z2i = 2.0 * zr * zi;  // z^2
  double sr = 0.0, si = 0.0;
  for (int n = E.nmats - 1; n >= 0; --n) {  // small terms first
    double w = (2.0 * n + 1.0) * kPi * T, u = w * w, d = u + O2;
    double W = (E.kind == 0) ? -4.0 * Om * u * u / (d * d * d) : u * u / (d * d);
    double dr = u + z2r, di = z2i, inv = W / (dr * dr + di * di);
    sr += dr * inv;
    si -= di * inv;
  }
  // tail: series in v = 1/w^2 of W(w)/(w^2+z^2)
  double cr[kTabKTail + 1], ci[kTabKTail + 1];
  for (int k = 0; k <= kTabKTail; ++k) cr[k] = ci[k] = 0.0;
  int nom;
  if (E.kind == 0) { cr[2] = -4.0 * Om; nom = 3; }   // -4 Omega v^2 (1+O2 v)^-3 (1+z^2 v)^-1
  else { cr[1] = 1.0; nom = 2; }                      // v (1+O2 v)^-2 (1+z^2 v)^-1
  for (int k = 1; k <= kTabKTail; ++k) {              // divide by (1 + z^2 v)
    double pr = cr[k - 1], pi_ = ci[k - 1];
    cr[k] -= z2r * pr - z2i * pi_;
    ci[k] -= z2r * pi_ + z2i * pr;
  }
  for (int r = 0; r < nom; ++r)                       // divide by (1 + Omega^2 v)
    for (int k = 1; k <= kTabKTail; ++k) {
      cr[k] -= O2 * cr[k - 1];
      ci[k] -= O2 * ci[k - 1];
    }
  for (int k = kTabKTail; k >= 1; --k) {
    sr += cr[k] * zeta[k];
    si += ci[k] * zeta[k];
  }
  // S = -2 z T (sum)
  double f = -2.0 * T;
  return make_double2(f * (zr * sr - zi * si), f * (zr * si + zi * sr));
}

__global__ void k_tab_points(TabArgs a) {
  long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long per = (long)a.max_J * kTabPts;
  int e = (int)(gid / per);
  if (e >= a.n_entries) return;
  int j = (int)((gid % per) / kTabPts), p = (int)(gid % kTabPts);
  const Entry E = a.entries[e];
  if (j >= E.J || E.kind > 1) return;
  double c, h;
  tab_interval(j, E.w, c, h);
  double th = 2.0 * kPi * p / kTabPts, sn, cs;
  sincos(th, &sn, &cs);
  double zr = c + kTabRho * h * cs, zi = kTabRho * h * sn;
  a.svals[((long)e * a.max_J + j) * kTabPts + p] =
      S_complex(E, a.zeta + (long)e * (kTabKTail + 1), zr, zi);
}

__global__ void k_tab_coef(TabArgs a) {
  long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long per = (long)a.max_J * (kTabDeg + 1);
  int e = (int)(gid / per);
  if (e >= a.n_entries) return;
  int j = (int)((gid % per) / (kTabDeg + 1)), k = (int)(gid % (kTabDeg + 1));
  const Entry E = a.entries[e];
  if (j >= E.J) return;
  double *row = a.tab + E.tab_off + (long)j * kTabStride;
  double c, h;
  tab_interval(j, E.w, c, h);
  if (k == 0) {
    // -c/h, exact: 2j for a central interval, 2P + 1 + 2m for interval m of an octave
    row[0] = -(double)(j < kTabCentral ? 2 * j
                                       : 2 * kTabPerOct + 1 + 2 * ((j - kTabCentral) % kTabPerOct));
    row[1] = 1.0 / h;
  }
  double coef = 0.0;
  if (E.kind <= 1 && !(j == 0 && (k & 1) == 0)) {  // S is odd: even terms vanish at 0
    const double2 *sv = a.svals + ((long)e * a.max_J + j) * kTabPts;
    double s = 0.0;
    for (int p = 0; p < kTabPts; ++p) {
      double sn, cs;
      sincos(2.0 * kPi * (double)((k * p) % kTabPts) / kTabPts, &sn, &cs);
      s += sv[p].x * cs + sv[p].y * sn;  // Re(S e^{-i k th})
    }
    coef = s / kTabPts / pow(kTabRho, (double)k);
  }
  row[kTabCoef + k] = coef;
}

}  // namespace

hipError_t launch_tables(const TabArgs &a, hipStream_t s) {
  if (a.n_entries == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zeta, dim3(a.n_entries), dim3(64), 0, s, a.entries, a.n_entries, a.zeta);
  long n1 = (long)a.n_entries * a.max_J * kTabPts;
  hipLaunchKernelGGL(k_tab_points, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, s, a);
  long n2 = (long)a.n_entries * a.max_J * (kTabDeg + 1);
  hipLaunchKernelGGL(k_tab_coef, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

// container constants: parameter row, channel, cos/sin of l/2 per axis
namespace {
__global__ void k_container_setup(Ctr *ctr, int n_ctr, const double *q, int n_q, int n_ch,
                                  int ch_first) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_ctr) return;
  int ich = c % n_ch, iq = (c / n_ch) % n_q, ip = c / (n_ch * n_q);
  Ctr r;
  r.entry = ip;
  r.ch = (n_ch == 2) ? ich : ch_first;
  sincos(0.5 * q[2 * iq], &r.sLx, &r.cLx);
  sincos(0.5 * q[2 * iq + 1], &r.sLy, &r.cLy);
  ctr[c] = r;
}
}  // namespace

hipError_t launch_container_setup(Ctr *ctr, int n_ctr, const double *q, int n_q, int n_ch,
                                  int ch_first, hipStream_t s) {
  if (n_ctr == 0) return hipSuccess;
  hipLaunchKernelGGL(k_container_setup, dim3((n_ctr + 255) / 256), dim3(256), 0, s, ctr, n_ctr, q,
                     n_q, n_ch, ch_first);
  return hipGetLastError();
}

}  // namespace paid
