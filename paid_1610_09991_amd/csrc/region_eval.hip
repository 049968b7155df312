// region_eval.hip -- the hot kernel: evaluation of rectangles with the nested
// Clenshaw-Curtis pair (Sec. 3) for all form-factor pairs at once.
//
// One wavefront owns one work item: a parent rectangle and its four children
// (Alg. 2: split into 4, evaluate Q_N and Q_2N on each).  The children share
// 17 x 17 node coordinates, so the integrand g is evaluated 289 times instead
// of 324.  Per child the projection onto the box basis U[node][m] is the
// weighted Gram contraction
//     Q_2N = U^T diag(w_2N g) U,    Q_N = U^T diag(w_N g) U,   E = Q_2N - Q_N,
// and err of a child is sum_pq |E_pq| (the paper's error summed over pairs).
// Two ways to form it:
//   - separable (default): U[node][(a,b)] = u_a(x) u_b(y) and the weights are
//     tensor products, so the sum runs first over y for every x and every
//     product u_b u_d, then over x for every product u_a u_c; for 9 form
//     factors this is ~4.4k FMAs per parent instead of a 16x16x84 tile pair;
//   - dense Gram on the FP64 matrix cores (16x16x4 tiles; a 9-function basis
//     fills one tile, 25 functions 2x2 tiles of which the lower-left one is
//     skipped by symmetry).
// The frequency-sum table of the parameter row is staged in LDS once per
// workgroup and shared by its waves.
#include <math.h>

#include "launch.h"

namespace paid {

__constant__ RuleConst c_rule;

hipError_t set_rule_constants(const RuleConst &rc) {
  return hipMemcpyToSymbol(HIP_SYMBOL(c_rule), &rc, sizeof(RuleConst));
}

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 6.28318530717958647692;
constexpr double kSqrt2 = 1.41421356237309504880;

typedef double d4 __attribute__((ext_vector_type(4)));

template <int L>
struct Dims {
  static constexpr int NB = 2 * L + 1;          // harmonics per axis
  static constexpr int MB = NB * NB;            // box functions
  static constexpr int NP = NB * (NB + 1) / 2;  // products u_a u_c, a <= c
  static constexpr int MU = MB * (MB + 1) / 2;  // pairs of box functions
  // the four children's x-sums fit in the storage of the integrand values
  static constexpr bool XALL = 4 * 2 * NP * NP <= kNX * kNX;
};

// per-wave scratch in LDS.  Buffers of different phases share storage: the
// integrand g is dead once the y-sums are formed (separable path), the
// per-axis cosines once g is, and the separable path never uses the box
// harmonics of the dense Gram.
template <int L>
struct WaveLds {
  static constexpr int NB = Dims<L>::NB, MB = Dims<L>::MB, NP = Dims<L>::NP, MU = Dims<L>::MU;
  double pp[2][kNX][NP];           // products u_a u_c of the box harmonics per axis
  union {
    double g[kNX * kNX];           // integrand at the shared nodes
    struct {
      double g2[NP * NP], g1[NP * NP];  // x-sums of one child (separable path)
    };
    struct {  // x-sums of all four children (where XALL)
      double g2b[Dims<L>::XALL ? 4 : 1][NP * NP], g1b[Dims<L>::XALL ? 4 : 1][NP * NP];
    };
  };
  union {
    struct {
      double cp[2][kNX], cm[2][kNX];    // cos(l/2 + p), cos(l/2 - p) per axis
      double pos[2][kNX];               // coordinates
    };
    double h1[2][kNCo * 2 - 1][NP];     // y-sums with the coarse weights (even x)
  };
  union {
    double h2[2][kNX][NP];         // y-sums with the fine weights, per child row
    double u[2][kNX][NB];          // box harmonics per axis (dense Gram)
  };
  double cq[MU], ce[MU];           // one child's Q_2N and E over form-factor pairs
  // general form-factor sets only (dropped from the allocation otherwise)
  double tq[MB * MB], ts[MB * MB], tr[MB * MB];
};

template <int L>
constexpr size_t wave_lds_doubles(bool identity) {
  return (sizeof(WaveLds<L>) - (identity ? 3 * sizeof(double) * Dims<L>::MB * Dims<L>::MB : 0)) /
         sizeof(double);
}

// wave-local synchronisation for LDS traffic between lanes of one wave
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline int lane_id() { return threadIdx.x & 63; }

__device__ inline int pair_index(int p, int q, int M) { return p * M - p * (p - 1) / 2 + (q - p); }

template <int NB>
__device__ inline int prod_index(int a, int c) {  // (a, c) -> index of u_a u_c
  if (a > c) { int t = a; a = c; c = t; }
  return a * NB - a * (a - 1) / 2 + (c - a);
}

// parity of box function m = a NB + b under p -> -p: 1 if it has one sine
// factor (u_{2k} = sqrt2 sin kx is odd, 1 and the cosines are even)
template <int NB>
__device__ inline int box_odd(int m) {
  const int a = m / NB, b = m - a * NB;
  return ((a > 0 && !(a & 1)) ? 1 : 0) ^ ((b > 0 && !(b & 1)) ? 1 : 0);
}

// weight of a box pair in the half-zone mode: 0 for odd joint parity (the
// full-zone integral vanishes), else 2 (the two halves are equal)
template <int NB>
__device__ inline double half_zone_factor(int m, int n) {
  return (box_odd<NB>(m) ^ box_odd<NB>(n)) ? 0.0 : 2.0;
}

// sin and cos of |x| <= pi (+ rounding): reduction by pi/2 in two parts
// (Cody-Waite; q*pi/2 is exact for |q| <= 2) to |r| <= pi/4, then the Taylor
// series of sin and cos to degree 17/18 (truncation below 1e-19 there).
__device__ inline void sincos_zone(double x, double *s, double *c) {
  const double pio2_hi = 1.5707963267948966, pio2_lo = 6.123233995736766e-17;
  const double q = rint(x * 0.63661977236758134);
  const double r = (x - q * pio2_hi) - q * pio2_lo, r2 = r * r;
  double ps = 1.0 / 355687428096000.0;  // 1/17!
  ps = fma(ps, r2, -1.0 / 1307674368000.0);
  ps = fma(ps, r2, 1.0 / 6227020800.0);
  ps = fma(ps, r2, -1.0 / 39916800.0);
  ps = fma(ps, r2, 1.0 / 362880.0);
  ps = fma(ps, r2, -1.0 / 5040.0);
  ps = fma(ps, r2, 1.0 / 120.0);
  ps = fma(ps, r2, -1.0 / 6.0);
  const double sr = fma(ps * r2, r, r);
  double pc = 1.0 / 6402373705728000.0;  // 1/18!
  pc = fma(pc, r2, -1.0 / 20922789888000.0);
  pc = fma(pc, r2, 1.0 / 87178291200.0);
  pc = fma(pc, r2, -1.0 / 479001600.0);
  pc = fma(pc, r2, 1.0 / 3628800.0);
  pc = fma(pc, r2, -1.0 / 40320.0);
  pc = fma(pc, r2, 1.0 / 720.0);
  pc = fma(pc, r2, -1.0 / 24.0);
  pc = fma(pc, r2, 0.5);
  const double cr = fma(-pc, r2, 1.0);
  const int k = ((int)q) & 3;
  *s = (k == 0) ? sr : (k == 1) ? cr : (k == 2) ? -sr : -cr;
  *c = (k == 0) ? cr : (k == 1) ? -sr : (k == 2) ? -cr : sr;
}

// Coordinates of one axis: nco = 17 (four children of a rectangle of width
// wdt starting at x0) or 9 (a single rectangle).
__device__ inline double axis_coord(int j, int nco, double x0, double wdt) {
  if (nco == kNF) return x0 + 0.5 * wdt + 0.5 * wdt * c_rule.xi[j];
  if (j <= 8) return x0 + 0.25 * wdt + 0.25 * wdt * c_rule.xi[j];
  return x0 + 0.75 * wdt + 0.25 * wdt * c_rule.xi[j - 8];
}

// Per-axis data and the integrand on the nco x nco node grid.  `tab` is the
// parameter row's frequency-sum table (LDS or global memory).
template <int L>
__device__ void fill_nodes(WaveLds<L> &S, const Problem &P, const Ctr &C, const Entry &E,
                           const double *tab, int nco, double x0, double y0, double wdt) {
  constexpr int NB = Dims<L>::NB;
  const int lane = lane_id();
  if (lane < 2 * nco) {
    int ax = lane >= nco, j = lane - ax * nco;
    double p = axis_coord(j, nco, ax ? y0 : x0, wdt);
    double sp, cpp;
    sincos_zone(p, &sp, &cpp);
    double cL = ax ? C.cLy : C.cLx, sL = ax ? C.sLy : C.sLx;
    S.pos[ax][j] = p;
    S.cp[ax][j] = cL * cpp - sL * sp;  // cos(l/2 + p)
    S.cm[ax][j] = cL * cpp + sL * sp;  // cos(l/2 - p)
    double u[NB];
    u[0] = 1.0;
    if (L >= 1) {
      u[1] = kSqrt2 * cpp;
      u[2] = kSqrt2 * sp;
    }
    if (L >= 2) {
      u[3] = kSqrt2 * (cpp - sp) * (cpp + sp);
      u[4] = kSqrt2 * 2.0 * sp * cpp;
    }
#pragma unroll
    for (int a = 0; a < NB; ++a) {
      S.u[ax][j][a] = u[a];
#pragma unroll
      for (int c = a; c < NB; ++c) S.pp[ax][j][prod_index<NB>(a, c)] = u[a] * u[c];
    }
  }
  wave_sync();
  const int nn = nco * nco;
#pragma unroll 1
  for (int v = lane; v < nn; v += 64) {
    int ix = v / nco, iy = v - ix * nco;
    double g;
    if (P.kind <= 1) {
      double px = S.cp[0][ix], py = S.cp[1][iy], mx = S.cm[0][ix], my = S.cm[1][iy];
      double a = -2.0 * E.t * (px + py) - 4.0 * E.tp * px * py - E.mu;
      double b = -2.0 * E.t * (mx + my) - 4.0 * E.tp * mx * my - E.mu;
      g = K_eval(E, tab, C.ch, a, b);
    } else if (P.kind == 2) {
      g = 1.0;
    } else {
      double dx = S.pos[0][ix] - P.gauss_x, dy = S.pos[1][iy] - P.gauss_y;
      g = exp(-(dx * dx + dy * dy) / (2.0 * P.gauss_s * P.gauss_s));
    }
    S.g[v] = g;
  }
  wave_sync();
}

// ------------------------------------------------------------- separable
// Stage 1: for every x of the grid and each child row cy, the y-sums
//   h2[cy][x][k] = sum_b w2_b g(x, y_b) P_k(y_b),  h1 likewise with w1 on even b.
template <int L>
__device__ void sep_stage1(WaveLds<L> &S, int nco, int nrow) {
  constexpr int NP = Dims<L>::NP;
  const int lane = lane_id();
  for (int idx = lane; idx < nrow * nco * NP; idx += 64) {
    int cy = idx / (nco * NP), rem = idx - cy * nco * NP, x = rem / NP, k = rem - x * NP;
    const double *gr = &S.g[x * nco + 8 * cy];
    double s2 = 0.0, s1 = 0.0;
#pragma unroll
    for (int b = 0; b < kNF; ++b) {
      double v = gr[b] * S.pp[1][8 * cy + b][k];
      s2 = fma(c_rule.w2[b], v, s2);
      if (!(b & 1)) s1 = fma(c_rule.w1[b >> 1], v, s1);
    }
    S.h2[cy][x][k] = s2;
    if (!(x & 1)) S.h1[cy][x >> 1][k] = s1;
  }
  wave_sync();
}

// Stage 2 for child (cx, cy), then the form-factor pairs (identity basis) or
// the full box Gram (general sets) scaled by the area factor fa.
// the four children's x-sums in one pass over the lanes (where they fit:
// 144 tasks in 3 passes instead of 36 in each of 4)
template <int L>
constexpr bool kXsumsAll = Dims<L>::XALL;

template <int L>
__device__ void sep_xsums_all(WaveLds<L> &S) {
  constexpr int NP = Dims<L>::NP;
  const int lane = lane_id();
  for (int idx = lane; idx < 4 * NP * NP; idx += 64) {
    const int ch = idx / (NP * NP), r = idx - ch * (NP * NP), cx = ch & 1, cy = ch >> 1;
    const int j = r / NP, k = r - j * NP;
    double s2 = 0.0, s1 = 0.0;
#pragma unroll
    for (int a = 0; a < kNF; ++a) {
      int x = 8 * cx + a;
      double pj = S.pp[0][x][j];
      s2 = fma(c_rule.w2[a] * pj, S.h2[cy][x][k], s2);
      if (!(a & 1)) s1 = fma(c_rule.w1[a >> 1] * pj, S.h1[cy][x >> 1][k], s1);
    }
    S.g2b[ch][r] = s2;
    S.g1b[ch][r] = s1;
  }
  wave_sync();
}

template <int L>
__device__ void sep_stage2(WaveLds<L> &S, const Problem &P, const int *pidmap, const int *podd,
                           int cx, int cy, double fa, bool xsums_done) {
  constexpr int NB = Dims<L>::NB, NP = Dims<L>::NP, MB = Dims<L>::MB, MU = Dims<L>::MU;
  const int lane = lane_id();
  const double *G2 = S.g2, *G1 = S.g1;
  bool done = false;
  if constexpr (kXsumsAll<L>) {
    if (xsums_done) {
      G2 = S.g2b[2 * cy + cx];
      G1 = S.g1b[2 * cy + cx];
      done = true;
    }
  }
  if (!done) {
    for (int idx = lane; idx < NP * NP; idx += 64) {
      int j = idx / NP, k = idx - j * NP;
      double s2 = 0.0, s1 = 0.0;
#pragma unroll
      for (int a = 0; a < kNF; ++a) {
        int x = 8 * cx + a;
        double pj = S.pp[0][x][j];
        s2 = fma(c_rule.w2[a] * pj, S.h2[cy][x][k], s2);
        if (!(a & 1)) s1 = fma(c_rule.w1[a >> 1] * pj, S.h1[cy][x >> 1][k], s1);
      }
      S.g2[idx] = s2;
      S.g1[idx] = s1;
    }
    wave_sync();
  }
  if (P.ff_identity) {
    for (int pid = lane; pid < MU; pid += 64) {
      int jk = pidmap[pid];
      double q2 = G2[jk], f = fa;
      if (P.sym) f = podd[pid] ? 0.0 : 2.0 * fa;
      S.cq[pid] = f * q2;
      S.ce[pid] = f * (q2 - G1[jk]);
    }
  } else {
    for (int idx = lane; idx < MB * MB; idx += 64) {
      int m = idx / MB, n = idx - m * MB;
      int jk = prod_index<NB>(m / NB, n / NB) * NP + prod_index<NB>(m % NB, n % NB);
      double q2 = G2[jk], f = fa;
      if (P.sym) f = half_zone_factor<NB>(m, n) * fa;
      S.tq[idx] = f * q2;
      S.ts[idx] = f * (q2 - G1[jk]);
    }
  }
  wave_sync();
}

// ------------------------------------------------------------- dense MFMA
// Weighted Gram of one rectangle on the matrix cores.  Its 9 x 9 nodes are
// rows offx.. and columns offy.. of the nco x nco grid.  A row of A is a box
// function times w g (fine weights for Q_2N, w_2N - w_N for E, which keeps the
// error estimate free of a rounding floor in reduced precision), B is the box
// function; results are scaled by fa and widened to FP64.

// one product term of the Gram at a node: values for this lane's A and B
struct GramVals {
  double aq0, ae0, b0, aq1, ae1, b1;
};

template <int L>
__device__ inline GramVals gram_node_vals(const WaveLds<L> &S, int nu, int nco, int offx, int offy,
                                         bool v0, bool v1, int a0, int b0, int a1, int b1) {
  GramVals r = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (nu < kNF * kNF) {
    int a = nu / kNF, b = nu - a * kNF;
    int gx = offx + a, gy = offy + b;
    double g = S.g[gx * nco + gy];
    double w2 = c_rule.w2[a] * c_rule.w2[b];
    double wn = ((a | b) & 1) ? 0.0 : c_rule.w1[a >> 1] * c_rule.w1[b >> 1];
    double gq = g * w2, ge = g * (w2 - wn);
    if (v0) {
      r.b0 = S.u[0][gx][a0] * S.u[1][gy][b0];
      r.aq0 = r.b0 * gq;
      r.ae0 = r.b0 * ge;
    }
    if (v1) {
      r.b1 = S.u[0][gx][a1] * S.u[1][gy][b1];
      r.aq1 = r.b1 * gq;
      r.ae1 = r.b1 * ge;
    }
  }
  return r;
}

// store the accumulated tiles: element (i, j) of tile t
template <int L>
__device__ inline void gram_put(WaveLds<L> &S, const Problem &P, int i, int j, double q, double e) {
  constexpr int MB = Dims<L>::MB;
  if (i < MB && j < MB && i <= j) {
    if (P.sym) {
      const double f = half_zone_factor<Dims<L>::NB>(i, j);
      q *= f;
      e *= f;
    }
    if (P.ff_identity) {
      int pid = pair_index(i, j, MB);
      S.cq[pid] = q;
      S.ce[pid] = e;
    } else {
      S.tq[i * MB + j] = q;
      S.tq[j * MB + i] = q;
      S.ts[i * MB + j] = e;
      S.ts[j * MB + i] = e;
    }
  }
}

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

// three-term bf16 split x = hi + mid + lo (8 significant bits each)
__device__ inline void split3(double x, __bf16 &hi, __bf16 &mid, __bf16 &lo) {
  float f = (float)x;
  hi = (__bf16)f;
  float r1 = f - (float)hi;
  mid = (__bf16)r1;
  lo = (__bf16)(r1 - (float)mid);
}

template <int L, int PREC>
__device__ void gram_mfma(WaveLds<L> &S, const Problem &P, int nco, int offx, int offy, double fa) {
  constexpr int NB = Dims<L>::NB, MB = Dims<L>::MB, NT = MB > 16 ? 2 : 1;
  constexpr int NACC = NT * (NT + 1) / 2;
  const int lane = lane_id(), m = lane & 15, kk = lane >> 4;
  const bool v0 = m < MB, v1 = (NT == 2) && (m + 16 < MB);
  const int a0 = v0 ? m / NB : 0, b0 = v0 ? m % NB : 0;
  const int a1 = v1 ? (m + 16) / NB : 0, b1 = v1 ? (m + 16) % NB : 0;
  if (PREC == PAID_FP64) {
    d4 aq[NACC], ae[NACC];
#pragma unroll
    for (int t = 0; t < NACC; ++t) {
      aq[t] = d4{0.0, 0.0, 0.0, 0.0};
      ae[t] = d4{0.0, 0.0, 0.0, 0.0};
    }
#pragma unroll 3
    for (int kb = 0; kb < 21; ++kb) {
      GramVals v = gram_node_vals<L>(S, 4 * kb + kk, nco, offx, offy, v0, v1, a0, b0, a1, b1);
      aq[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(v.aq0, v.b0, aq[0], 0, 0, 0);
      ae[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(v.ae0, v.b0, ae[0], 0, 0, 0);
      if (NT == 2) {
        aq[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(v.aq0, v.b1, aq[1], 0, 0, 0);
        ae[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(v.ae0, v.b1, ae[1], 0, 0, 0);
        aq[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(v.aq1, v.b1, aq[2], 0, 0, 0);
        ae[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(v.ae1, v.b1, ae[2], 0, 0, 0);
      }
    }
    // f64 16x16x4 result: row = 4 r + lane >> 4, col = lane & 15
#pragma unroll
    for (int t = 0; t < NACC; ++t) {
      int tr = (NT == 2 && t == 2) ? 1 : 0, tc = (NT == 2 && t >= 1) ? 1 : 0;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        gram_put<L>(S, P, 16 * tr + 4 * r + kk, 16 * tc + m, fa * aq[t][r], fa * ae[t][r]);
    }
  } else if (PREC == PAID_FP32) {
    f4v aq[NACC], ae[NACC];
#pragma unroll
    for (int t = 0; t < NACC; ++t) {
      aq[t] = f4v{0.f, 0.f, 0.f, 0.f};
      ae[t] = f4v{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll 3
    for (int kb = 0; kb < 21; ++kb) {
      GramVals v = gram_node_vals<L>(S, 4 * kb + kk, nco, offx, offy, v0, v1, a0, b0, a1, b1);
      aq[0] = __builtin_amdgcn_mfma_f32_16x16x4f32((float)v.aq0, (float)v.b0, aq[0], 0, 0, 0);
      ae[0] = __builtin_amdgcn_mfma_f32_16x16x4f32((float)v.ae0, (float)v.b0, ae[0], 0, 0, 0);
      if (NT == 2) {
        aq[1] = __builtin_amdgcn_mfma_f32_16x16x4f32((float)v.aq0, (float)v.b1, aq[1], 0, 0, 0);
        ae[1] = __builtin_amdgcn_mfma_f32_16x16x4f32((float)v.ae0, (float)v.b1, ae[1], 0, 0, 0);
        aq[2] = __builtin_amdgcn_mfma_f32_16x16x4f32((float)v.aq1, (float)v.b1, aq[2], 0, 0, 0);
        ae[2] = __builtin_amdgcn_mfma_f32_16x16x4f32((float)v.ae1, (float)v.b1, ae[2], 0, 0, 0);
      }
    }
    // f32 16x16x4 result: row = 4 (lane >> 4) + r, col = lane & 15
#pragma unroll
    for (int t = 0; t < NACC; ++t) {
      int tr = (NT == 2 && t == 2) ? 1 : 0, tc = (NT == 2 && t >= 1) ? 1 : 0;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        gram_put<L>(S, P, 16 * tr + 4 * kk + r, 16 * tc + m, fa * (double)aq[t][r],
                    fa * (double)ae[t][r]);
    }
  } else {  // three-term bf16 split, 16x16x32 tiles, FP32 accumulation
    f4v aq[NACC], ae[NACC];
#pragma unroll
    for (int t = 0; t < NACC; ++t) {
      aq[t] = f4v{0.f, 0.f, 0.f, 0.f};
      ae[t] = f4v{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll 1
    for (int kb = 0; kb < 3; ++kb) {
      // this lane: row/col m, nodes 32 kb + 8 kk + e, e = 0..7
      bf8v q0[3], e0[3], c0[3], q1[3], e1[3], c1[3];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        GramVals v = gram_node_vals<L>(S, 32 * kb + 8 * kk + e, nco, offx, offy, v0, v1, a0, b0,
                                       a1, b1);
        __bf16 h, md, lo;
        split3(v.aq0, h, md, lo); q0[0][e] = h; q0[1][e] = md; q0[2][e] = lo;
        split3(v.ae0, h, md, lo); e0[0][e] = h; e0[1][e] = md; e0[2][e] = lo;
        split3(v.b0, h, md, lo); c0[0][e] = h; c0[1][e] = md; c0[2][e] = lo;
        if (NT == 2) {
          split3(v.aq1, h, md, lo); q1[0][e] = h; q1[1][e] = md; q1[2][e] = lo;
          split3(v.ae1, h, md, lo); e1[0][e] = h; e1[1][e] = md; e1[2][e] = lo;
          split3(v.b1, h, md, lo); c1[0][e] = h; c1[1][e] = md; c1[2][e] = lo;
        }
      }
      // A B ~ hi hi + hi mid + mid hi + hi lo + lo hi + mid mid (terms >= 2^-16)
      const int ia[6] = {0, 0, 1, 0, 2, 1}, ib[6] = {0, 1, 0, 2, 0, 1};
#pragma unroll
      for (int t6 = 0; t6 < 6; ++t6) {
        const int x = ia[t6], y = ib[t6];
        aq[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(q0[x], c0[y], aq[0], 0, 0, 0);
        ae[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(e0[x], c0[y], ae[0], 0, 0, 0);
        if (NT == 2) {
          aq[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(q0[x], c1[y], aq[1], 0, 0, 0);
          ae[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(e0[x], c1[y], ae[1], 0, 0, 0);
          aq[2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(q1[x], c1[y], aq[2], 0, 0, 0);
          ae[2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(e1[x], c1[y], ae[2], 0, 0, 0);
        }
      }
    }
    // bf16 16x16x32 result: row = 4 (lane >> 4) + r, col = lane & 15
#pragma unroll
    for (int t = 0; t < NACC; ++t) {
      int tr = (NT == 2 && t == 2) ? 1 : 0, tc = (NT == 2 && t >= 1) ? 1 : 0;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        gram_put<L>(S, P, 16 * tr + 4 * kk + r, 16 * tc + m, fa * (double)aq[t][r],
                    fa * (double)ae[t][r]);
    }
  }
  wave_sync();
}

// General form-factor sets: Q_ff = C Q_box C^T for both Q and E.
template <int L>
__device__ void transform_ff(WaveLds<L> &S, const Problem &P) {
  constexpr int MB = Dims<L>::MB;
  const int lane = lane_id(), M = P.M;
  double *R = S.tr;
  for (int which = 0; which < 2; ++which) {
    const double *G = which ? S.ts : S.tq;
    for (int idx = lane; idx < MB * M; idx += 64) {  // R[a][q] = sum_b G[a][b] C[q][b]
      int a = idx / M, q = idx - a * M;
      double s = 0.0;
      for (int b = 0; b < MB; ++b) s = fma(G[a * MB + b], P.ffc[q * MB + b], s);
      R[idx] = s;
    }
    wave_sync();
    double *dst = which ? S.ce : S.cq;
    for (int pid = lane; pid < P.MU; pid += 64) {
      int p = 0, k = pid;
      while (k >= M - p) { k -= M - p; ++p; }
      int q = p + k;
      double s = 0.0;
      for (int a = 0; a < MB; ++a) s = fma(P.ffc[p * MB + a], R[a * M + q], s);
      dst[pid] = s;
    }
    wave_sync();
  }
}

// a double moved between lanes by a DPP pattern (both halves; VALU, no LDS)
// v from another lane of the same row (CTRL: a quad permutation or a row
// mirror, which every lane reads within its row, so no lane keeps an old
// value and none need be set up)
template <int CTRL>
__device__ inline double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ inline double lane_value(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// sum over the 64 lanes in a fixed order, the same in every lane: within
// each row of 16 lanes by DPP exchanges (partners lane ^ 1, lane ^ 2, then
// the mirror images within 8 and within 16 lanes; a + b = b + a exactly, so
// partners agree), then the four row sums as (r0 + r1) + (r2 + r3)
__device__ inline double wave_sum(double v) {
  v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x141>(v);  // row_half_mirror
  v += dpp_move<0x140>(v);  // row_mirror
  return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

// Store one evaluated rectangle (S.cq, S.ce) into pool slot `ri` of slot s,
// return its key.
template <int L>
__device__ double store_region(WaveLds<L> &S, const Problem &P, int s, long ri, uint64_t code) {
  const int lane = lane_id();
  const long base = slot_base(P, s) + ri;
  double part = 0.0;
  for (int pid = lane; pid < P.MU; pid += 64) {
    double q = S.cq[pid], e = fabs(S.ce[pid]);
    P.Q[base * P.MU + pid] = q;
    if (P.E) P.E[base * P.MU + pid] = err_f32(e);
    part += (P.err_mode != 0) ? e * (double)P.itau[(long)s * P.MU + pid] : e;
  }
  double key = wave_sum(part);
  if (lane == 0) {
    P.key[base] = key;
    P.code[base] = code;
  }
  return key;
}

// One rectangle of the grid (child (cx, cy) of the 17-grid, or the 9-grid
// root with cx = cy = 0): fills S.cq / S.ce.
// GRAM: 0..2 = dense Gram on the matrix cores in FP64 / FP32 / bf16x3,
// 3 = separable FP64
constexpr int kSep = 3;

template <int L, int GRAM>
__device__ void eval_rect(WaveLds<L> &S, const Problem &P, const int *pidmap, const int *podd,
                          int nco, int cx, int cy, double fa, bool xsums_done = false) {
  if (GRAM == kSep) {
    sep_stage2<L>(S, P, pidmap, podd, cx, cy, fa, xsums_done);
  } else {
    gram_mfma<L, GRAM>(S, P, nco, 8 * cx, 8 * cy, fa);
  }
  if (!P.ff_identity) transform_ff<L>(S, P);
}

// pair index -> index into the x-sum matrix of the separable form
// and whether the pair has odd joint parity (half-zone mode)
template <int L>
__device__ void build_pidmap(int *map, int *odd, int tid, int nthr) {
  constexpr int NB = Dims<L>::NB, MB = Dims<L>::MB, NP = Dims<L>::NP, MU = Dims<L>::MU;
  for (int pid = tid; pid < MU; pid += nthr) {
    int m = 0, k = pid;
    while (k >= MB - m) { k -= MB - m; ++m; }
    int n = m + k;
    map[pid] = prod_index<NB>(m / NB, n / NB) * NP + prod_index<NB>(m % NB, n % NB);
    odd[pid] = box_odd<NB>(m) ^ box_odd<NB>(n);
  }
}

// ---------------------------------------------------------------- root
// A region that the seed tree splits is stored as a placeholder: zero value,
// error and key.  It is split in a later round of the seed phase before any
// termination test runs, so the running sums never miss it.
template <int L>
__device__ void store_zero(const Problem &P, int s, long ri, uint64_t code) {
  const int lane = lane_id();
  const long base = slot_base(P, s) + ri;
  for (int pid = lane; pid < P.MU; pid += 64) {
    P.Q[base * P.MU + pid] = 0.0;
    if (P.E) P.E[base * P.MU + pid] = 0.0f;
  }
  if (lane == 0) {
    P.key[base] = 0.0;
    P.code[base] = code;
  }
}

// Seed admission (one wave): pyramid of predicted leaf counts in the
// container's frame, n = max(0, 2^y - 1) per cell and 2 x 2 sums upwards,
// and the depth bound D, lowered from seed_dmax until the seed tree has at
// most seed_limit leaves.  Returns D.
__device__ int seed_admit(const Problem &P, int s, int c, double *spyr) {
  const int t = threadIdx.x;
  const float *y = P.seed_y + (long)c * (kSeedG * kSeedG);
  const int fold = P.seed_fold[c];
  for (int cell = t; cell < kSeedG * kSeedG; cell += 64) {
    double n = exp2((double)y[seed_model_cell(fold, cell & 15, cell >> 4)]) - 1.0;
    spyr[pyr_off(4) + cell] = n > 0.0 ? n : 0.0;
  }
  __syncthreads();
  for (int d = 3; d >= 0; --d) {
    const int w = 1 << d, o = pyr_off(d), o1 = pyr_off(d + 1);
    for (int k = t; k < w * w; k += 64) {
      int i = k % w, j = k / w;
      const double *ch = spyr + o1;
      const int w1 = 2 * w;
      spyr[o + k] = ((ch[(2 * j) * w1 + 2 * i] + ch[(2 * j) * w1 + 2 * i + 1]) +
                     ch[(2 * j + 1) * w1 + 2 * i]) + ch[(2 * j + 1) * w1 + 2 * i + 1];
    }
    __syncthreads();
  }
  double *py = P.pyr + (long)s * kPyr;
  for (int k = t; k < kPyr; k += 64) py[k] = spyr[k];
  const double th = P.seed_thresh;
  int D = P.seed_dmax;
  for (; D > 0; --D) {
    long long leaves = 0;
    for (int k = t; k < kPyr; k += 64) {
      int d = 0;
      while (k >= pyr_off(d + 1)) ++d;
      if (d > D) continue;
      const int w = 1 << d, i = (k - pyr_off(d)) % w, j = (k - pyr_off(d)) / w;
      bool exists = true;
      for (int a = 0; a < d; ++a) {
        int sh = d - a;
        double ca = spyr[pyr_off(a) + ((j >> sh) << a) + (i >> sh)];
        exists = exists && (a < D) && (ca >= th);
      }
      if (!exists) continue;
      const double cn = spyr[k];
      if (d < 4) {
        if (!(d < D && cn >= th)) leaves += 1;
      } else {  // uniform subtree below a cell: levels split while the share >= th
        int lev = 0;
        double v = cn;
        while (4 + lev < D && v >= th) {
          ++lev;
          v *= 0.25;
        }
        leaves += 1LL << (2 * lev);
      }
    }
    for (int off = 32; off >= 1; off >>= 1) leaves += __shfl_xor(leaves, off, 64);
    if (leaves <= P.seed_limit) break;
  }
  return D;
}

template <int L, int GRAM>
__global__ void __launch_bounds__(64) k_root(Problem P) {
  extern __shared__ double lds_raw[];
  __shared__ int pidmap[Dims<L>::MU], podd[Dims<L>::MU];
  __shared__ double spyr[kPyr];
  WaveLds<L> &S = *reinterpret_cast<WaveLds<L> *>(lds_raw);
  const int s = blockIdx.x;
  if (s >= P.W || P.state[s] != SLOT_NEW) return;
  build_pidmap<L>(pidmap, podd, threadIdx.x, 64);
  const int c = P.cid[s];
  // key weights: the pair weights in the weighted mode, else one (the
  // per-integral mode refreshes them with 1/tau every round)
  for (int pid = threadIdx.x; pid < P.MU; pid += 64) {
    float w = 1.0f;
    if (P.err_mode == 2) {
      const int M = P.M;
      int p = 0, k = pid;
      while (k >= M - p) { k -= M - p; ++p; }
      const int q = p + k;
      const double *W = P.pair_w + (long)c * M * M;
      w = (float)((p == q) ? W[p * M + p] : W[p * M + q] + W[q * M + p]);
    }
    P.itau[(long)s * P.MU + pid] = w;
  }
  __syncthreads();
  int D = 0;
  bool placeholder = false;
  if (P.seed_y) {
    D = seed_admit(P, s, c, spyr);
    placeholder = D > 0 && spyr[0] >= P.seed_thresh;
  }
  double key = 0.0;
  const int nroot = P.sym ? 2 : 1;  // leaves the container starts from
  if (placeholder) {
    store_zero<L>(P, s, 0, make_code(0, 0, 0));
    for (int pid = threadIdx.x; pid < P.MU; pid += 64) {
      P.val[(long)s * P.MU + pid] = 0.0;
      if (P.errp) P.errp[(long)s * P.MU + pid] = 0.0;
    }
  } else {
    const Ctr C = P.ctr[c];
    const Entry E = P.entries[C.entry];
    const double *tab = P.tab + E.tab_off;
    // the zone, or in the half-zone mode its two quadrants with p_y >= 0
    const double wr = P.sym ? kPi : kTwoPi;
    for (int h = 0; h < nroot; ++h) {
      fill_nodes<L>(S, P, C, E, tab, kNF, -kPi + h * wr, P.sym ? 0.0 : -kPi, wr);
      if (GRAM == kSep) sep_stage1<L>(S, kNF, 1);
      eval_rect<L, GRAM>(S, P, pidmap, podd, kNF, 0, 0, (0.5 * wr) * (0.5 * wr) / (4.0 * kPi * kPi));
      key += store_region<L>(S, P, s, h, P.sym ? make_code(1, h, 1) : make_code(0, 0, 0));
      for (int pid = threadIdx.x; pid < P.MU; pid += 64) {
        const long o = (long)s * P.MU + pid;
        const double e = (double)err_f32(fabs(S.ce[pid]));
        P.val[o] = h ? P.val[o] + S.cq[pid] : S.cq[pid];
        if (P.errp) P.errp[o] = h ? P.errp[o] + e : e;
      }
      wave_sync();
    }
  }
  if (threadIdx.x == 0) {
    P.err[s] = key;
    P.nleaf[s] = placeholder ? 1 : nroot;
    P.st_rounds[s] = 0;
    P.st_splits[s] = 0;
    P.st_evals[s] = placeholder ? 0 : nroot * kNF * kNF;
    P.st_depth[s] = nroot - 1;
    if (P.born)
      for (int h = 0; h < nroot; ++h) P.born[slot_base(P, s) + h] = h;
    P.flags[s] = P.seed_y ? kFlagSeed : 0;
    if (P.seed_y) P.seed_d[s] = D;
    P.state[s] = SLOT_ACTIVE;
  }
}

// ---------------------------------------------------------------- children
// slot of a work item: woff is an exclusive prefix over slots
__device__ inline int item_slot(const Problem &P, int w) {
  int lo = 0, hi = P.W;  // woff[lo] <= w < woff[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (P.woff[mid] <= w) lo = mid; else hi = mid;
  }
  return lo;
}

// Work item r of slot s: split the selected leaf into its four children.
// tab: the table of the slot's parameter row (LDS or global memory).
template <int L, int GRAM>
__device__ void do_item(WaveLds<L> &S, const Problem &P, const int *pidmap, const int *podd, int s, int r,
                        const double *tab) {
  const Ctr C = P.ctr[P.cid[s]];
  const Entry E = P.entries[C.entry];
  // the pool and the deltas hold P.MU form-factor pairs (<= the box pairs)
  constexpr int KMAX = (Dims<L>::MU + 63) / 64;
  const int MU = P.MU;
  const int lane = lane_id();
  const long leaf = P.sel[(long)s * P.bmax + r];
  const long nold = P.nleaf[s];
  const long pbase = slot_base(P, s) + leaf;
  const uint64_t pc = P.code[pbase];
  const double pkey = P.key[pbase];
  // delta of the container sums: minus the parent, plus its children
  double dv[KMAX], dp[KMAX];
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    int pid = lane + 64 * k;
    dv[k] = (pid < MU) ? -P.Q[pbase * MU + pid] : 0.0;
    dp[k] = (pid < MU && P.E) ? -(double)P.E[pbase * MU + pid] : 0.0;
  }
  const int d = code_depth(pc);
  const uint64_t ix = code_ix(pc), iy = code_iy(pc);
  // children that the seed tree splits again become placeholders (uniform
  // in the wave); a parent with four of them needs no integrand values
  int skip = 0;
  if (P.seed_y && (P.flags[s] & kFlagSeed)) {
    for (int ch = 0; ch < 4; ++ch)
      if (seed_split(P, s, make_code(d + 1, 2 * ix + (ch & 1), 2 * iy + (ch >> 1)))) skip |= 1 << ch;
  }
  const double wdt = kTwoPi * ldexp(1.0, -d);
  const double x0 = -kPi + (double)ix * wdt, y0 = -kPi + (double)iy * wdt;
  if (skip != 15) {
    fill_nodes<L>(S, P, C, E, tab, kNX, x0, y0, wdt);
    if (GRAM == kSep) sep_stage1<L>(S, kNX, 2);
    if constexpr (GRAM == kSep && kXsumsAll<L>) sep_xsums_all<L>(S);
  }
  const double fa = (0.25 * wdt) * (0.25 * wdt) / (4.0 * kPi * kPi);
  double dkey = -pkey;
#pragma unroll 1
  for (int ch = 0; ch < 4; ++ch) {
    int cx = ch & 1, cy = ch >> 1;
    long ri = (ch == 0) ? leaf : nold + 3L * r + (ch - 1);
    const uint64_t cc = make_code(d + 1, 2 * ix + cx, 2 * iy + cy);
    if (P.born && lane == 0)  // the split is the container's st_splits-th (one per round)
      P.born[slot_base(P, s) + ri] = (unsigned int)(1 + 4 * P.st_splits[s] + ch);
    if ((skip >> ch) & 1) {
      store_zero<L>(P, s, ri, cc);
      wave_sync();
      continue;
    }
    if constexpr (GRAM == kSep && kXsumsAll<L>) {
      if (P.ff_identity) {
        // box-basis pairs straight from the x-sums into the child's record
        // and the parent's delta, without staging them in LDS
        const double *G2 = S.g2b[ch], *G1 = S.g1b[ch];
        const long base = slot_base(P, s) + ri;
        double part = 0.0;
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
          const int pid = lane + 64 * k;
          if (pid < MU) {
            const int jk = pidmap[pid];
            double f = fa;
            if (P.sym) f = podd[pid] ? 0.0 : 2.0 * fa;
            const double q2 = G2[jk], q = f * q2, e = fabs(f * (q2 - G1[jk]));
            P.Q[base * MU + pid] = q;
            if (P.E) P.E[base * MU + pid] = err_f32(e);
            part += (P.err_mode != 0) ? e * (double)P.itau[(long)s * MU + pid] : e;
            dv[k] += q;
            dp[k] += (double)err_f32(e);
          }
        }
        const double key = wave_sum(part);
        if (lane == 0) {
          P.key[base] = key;
          P.code[base] = cc;
        }
        dkey += key;
        wave_sync();
        continue;
      }
    }
    eval_rect<L, GRAM>(S, P, pidmap, podd, kNX, cx, cy, fa, true);
    dkey += store_region<L>(S, P, s, ri, cc);
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      int pid = lane + 64 * k;
      if (pid < MU) {
        dv[k] += S.cq[pid];
        // the same float-rounded value that is stored and later subtracted,
        // so the running per-pair error sums carry no rounding residue
        dp[k] += (double)err_f32(fabs(S.ce[pid]));
      }
    }
    wave_sync();
  }
  const long it = (long)s * P.bmax + r;
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    int pid = lane + 64 * k;
    if (pid < MU) {
      P.dv[it * MU + pid] = dv[k];
      if (P.dep) P.dep[it * MU + pid] = dp[k];
    }
  }
  if (lane == 0) {
    P.de[it] = dkey;
    if (P.ifill) P.ifill[it] = skip != 15;
    if (d + 1 > P.st_depth[s]) atomicMax(&P.st_depth[s], d + 1);
  }
}

// parameter row of slot s
__device__ inline int slot_entry(const Problem &P, int s) { return P.ctr[P.cid[s]].entry; }

// The problem description of a kernel whose only argument is a Problem, read
// through a pointer into the kernel-argument segment that the compiler cannot
// follow across loop iterations: its fields are then loaded (scalar loads
// from the constant cache) where an item uses them, instead of being held in
// scalar registers across the whole item loop, which overflowed them into
// vector-register lanes.
__device__ inline const Problem &kernarg_problem(const Problem &P) {
#ifdef __HIP_DEVICE_COMPILE__
  typedef const __attribute__((address_space(4))) Problem CP;
  CP *pk = (CP *)__builtin_amdgcn_kernarg_segment_ptr();
  asm volatile("" : "+s"(pk));
  return *(const Problem *)pk;
#else
  return P;
#endif
}

// Work items [i0, i1) of this workgroup.  Guided partition: workgroup b
// starts at item total (1 - k^b) with k = 1 - 1/S, S the workgroups resident
// at once, so the ranges shrink geometrically and the workgroups dispatched
// last (the tail of the launch) are short; k is lowered where the grid would
// otherwise leave its last workgroup more than four items.
__device__ inline void item_range(const Problem &P, int &i0, int &i1) {
  const int total = P.counters[2];
  if (P.eval_slots > 0) {
    const double keep = fmin(1.0 - 1.0 / (double)P.eval_slots,
                             exp(log(4.0 / fmax((double)total, 4.0)) / (double)gridDim.x));
    auto start = [&](int b) -> int {
      return b >= (int)gridDim.x ? total : (int)((double)total * (1.0 - pow(keep, (double)b)));
    };
    i0 = start(blockIdx.x);
    i1 = min(start(blockIdx.x + 1), total);
  } else {
    const int per = (total + gridDim.x - 1) / gridDim.x;
    i0 = blockIdx.x * per;
    i1 = min(i0 + per, total);
  }
}

// Each workgroup takes a contiguous range of work items; its waves take every
// nw-th item of it, so at any time they work on neighbouring parents, mostly
// of one container and parameter row.  The range is cut into segments of
// consecutive slots of one parameter row (usually a single one); at the
// start of a segment the workgroup stages that row's table in LDS (two
// barriers), and inside a segment there is no workgroup barrier: each wave
// runs through its items on its own.  The slot of an item is found by a
// search only when the wave's items leave the current slot's range.
template <int L, int GRAM>
__global__ void __launch_bounds__(256) k_children(Problem P) {
  extern __shared__ double lds_raw[];
  __shared__ int pidmap[Dims<L>::MU], podd[Dims<L>::MU];
  double *tabl = lds_raw;
  // the wave index is uniform in a wave: keep it (and all per-item
  // bookkeeping derived from it) in scalar registers
  const int nw = blockDim.x >> 6, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  WaveLds<L> &S = *reinterpret_cast<WaveLds<L> *>(lds_raw + (size_t)P.tab_rows * kTabStride +
                                                  (size_t)wv * P.lds_wave_doubles);
  int i0, i1;
  item_range(P, i0, i1);
  if (i0 >= i1) return;  // uniform in the workgroup
  build_pidmap<L>(pidmap, podd, threadIdx.x, blockDim.x);
  int s = item_slot(P, i0), lo = P.woff[s], hi = P.woff[s + 1];  // current slot, its items
  int w = i0 + wv, seg = i0, loaded = -1;
#pragma unroll 1
  while (seg < i1) {
    // segment [seg, seg_hi): slots from s on while they hold items of row e
    // (slots without items are passed over)
    const int e = slot_entry(P, s);
    int t = s + 1;
    while (t < P.W && P.woff[t] < i1 && (P.woff[t + 1] == P.woff[t] || slot_entry(P, t) == e)) ++t;
    const int seg_hi = (t < P.W && P.woff[t] < i1) ? P.woff[t] : i1;
    if (e != loaded) {
      __syncthreads();  // every wave is done with the previous table
      const Entry E0 = P.entries[e];
      const double *src = P.tab + E0.tab_off;
      for (int i = threadIdx.x; i < E0.J * kTabStride; i += blockDim.x) tabl[i] = src[i];
      __syncthreads();
      loaded = e;
    }
#pragma unroll 1
    for (; w < seg_hi; w += nw) {
      if (w >= hi) {  // find the slot holding item w (woff is non-decreasing)
        int a = s + 1, b = P.W;  // woff[a] <= w < woff[b]
        while (b - a > 1) {
          const int mid = (a + b) >> 1;
          if (P.woff[mid] <= w) a = mid; else b = mid;
        }
        s = a;
        lo = P.woff[s];
        hi = P.woff[s + 1];
      }
      do_item<L, GRAM>(S, kernarg_problem(P), pidmap, podd, s, w - lo, tabl);
    }
    // the next segment starts at slot t (its first item is seg_hi)
    seg = seg_hi;
    if (seg < i1) {
      s = t;
      lo = P.woff[s];
      hi = P.woff[s + 1];
    }
  }
}

// ---------------------------------------------------------------- two lanes per child
// Region evaluation for the 9-function box basis (L = 1) with the separable
// FP64 projection, arranged so that every sum stays in registers: a wave
// holds 8 work items (parents); lane 8 it + 2 ch + h evaluates child ch of
// item it together with its partner lane (h = 0, 1).  The products of two
// box harmonics u_a u_c (u_0 = 1, u_1 = sqrt2 cos, u_2 = sqrt2 sin) lie in
// the span of five functions phi = {1, sqrt2 cos, sqrt2 sin, cos 2x,
// sin 2x} (2 cos^2 = 1 + cos 2x, 2 cos sin = sin 2x, 2 sin^2 = 1 - cos 2x),
// so every pair of box functions of a rectangle is a signed sum of the 25
// integrals I_jk = int g phi_j(x) phi_k(y).  Lane h = 0 accumulates I for
// the fine rule (Q_2N); lane h = 1 accumulates the same sums with the weight
// difference of the two rules (E = Q_2N - Q_N, the error estimate), so the
// key of the child (sum over pairs of |E|) needs no lanes but its own.
// The two lanes of a child share its 81 nodes column by column: lane 0
// takes columns 0-3 and rows 0-4 of column 4, lane 1 columns 8-5 and rows
// 5-8 of column 4; after each column the partners swap their y-sums so
// that each adds both columns to its x-sums.  Nodes on the edges shared by
// neighbouring children are evaluated once per child (324 evaluations for
// the 289 distinct nodes of a parent).
namespace lpc {

constexpr int kItems = 8;              // work items per wave
constexpr int kYRow = 6;               // doubles per node row: C, D, phi_1..phi_4
// the 9 node rows of one child row, padded to an odd number of doubles so
// that the blocks the lanes of a wave read at one time fall on distinct banks
constexpr int kYBlock = kNF * kYRow + 1;
constexpr int kYDoubles = kItems * 2 * kYBlock;  // per-wave LDS: rows of both child rows
constexpr int kPairs = 45;             // pairs of the 9 box functions
// per-wave LDS: the node rows while the sums run, then (in the same space)
// per item the parent's Q, E and key weights for the records
__host__ __device__ constexpr int wave_doubles(bool with_e, bool with_w) {
  const int par = kItems * kPairs * (1 + (with_e ? 1 : 0) + (with_w ? 1 : 0));
  return par > kYDoubles ? par : kYDoubles;
}

// phi index and sign of the terms of the product u_a u_c (a <= c)
struct Terms {
  int n, j0, s0, j1, s1;
};
__host__ __device__ constexpr Terms prod_terms(int a, int c) {
  return (a == 0 && c == 0) ? Terms{1, 0, 1, 0, 0}
       : (a == 0 && c == 1) ? Terms{1, 1, 1, 0, 0}
       : (a == 0 && c == 2) ? Terms{1, 2, 1, 0, 0}
       : (a == 1 && c == 1) ? Terms{2, 0, 1, 3, 1}
       : (a == 1 && c == 2) ? Terms{1, 4, 1, 0, 0}
                            : Terms{2, 0, 1, 3, -1};  // (2, 2)
}

// the 45 box pairs (m, n), m <= n, m = 3 a + b: x terms of u_am u_an
// (phi index j0, optional j1 with sign) and y terms of u_bm u_bn; -1 = none
struct PairTab {
  signed char t[45][6];  // jx0, jx1, sx1, ky0, ky1, sy1
};
__host__ __device__ constexpr PairTab make_pair_tab() {
  PairTab T{};
  int p = 0;
  for (int m = 0; m < 9; ++m)
    for (int n = m; n < 9; ++n) {
      const int am = m / 3, bm = m % 3, an = n / 3, bn = n % 3;
      const Terms tx = prod_terms(am < an ? am : an, am < an ? an : am);
      const Terms ty = prod_terms(bm < bn ? bm : bn, bm < bn ? bn : bm);
      T.t[p][0] = (signed char)tx.j0;
      T.t[p][1] = (signed char)(tx.n == 2 ? tx.j1 : -1);
      T.t[p][2] = (signed char)tx.s1;
      T.t[p][3] = (signed char)ty.j0;
      T.t[p][4] = (signed char)(ty.n == 2 ? ty.j1 : -1);
      T.t[p][5] = (signed char)ty.s1;
      ++p;
    }
  return T;
}

// sum of v over the four children of the item, the same in all lanes of the
// item with the same h: ((c0 + c1) + (c2 + c3)) with a + b = b + a exactly
__device__ inline double child_sum(double v) {
  v += dpp_move<0x4E>(v);                 // quad_perm [2,3,0,1]: child ch ^ 1, same h
  const double o = dpp_move<0x141>(dpp_move<0xB1>(v));  // lane ^ 1, then 7 - lane: other quad, same h
  return v + o;
}

__device__ inline double swap_h(double v) { return dpp_move<0xB1>(v); }  // partner lane (h ^ 1)

}  // namespace lpc

// Sine and cosine of one coordinate, out of line: the constants of the
// series then live only while it runs instead of occupying registers across
// the caller's loops.
__device__ __noinline__ double2 sincos_out_of_line(double x) {
  double sn, cs;
  sincos_zone(x, &sn, &cs);
  return make_double2(sn, cs);
}

// Slot, item and parent of lane group `it` of a wave whose first item is g0
// in slot s0 (items g0 + it >= gend repeat the last item and store nothing).
struct LpcItem {
  int s, r;
  long leaf, pbase;
  uint64_t pc;
};
__device__ inline LpcItem lpc_item(const Problem &P, int w, int s0) {
  LpcItem q;
  int s = s0;
  while (P.woff[s + 1] <= w) ++s;
  q.s = s;
  q.r = w - P.woff[s];
  q.leaf = P.sel[(long)s * P.bmax + q.r];
  q.pbase = slot_base(P, s) + q.leaf;
  q.pc = P.code[q.pbase];
  return q;
}

// a value that is the same in every lane, held in scalar registers
__device__ inline double wave_uniform(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)b);
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// One group of up to 8 work items of one parameter row (row entry erow,
// table tab in LDS, the wave's LDS at Yw), first item g0 in slot s0; items
// g0 + it >= gend are inactive (their lanes repeat the last item and store
// nothing).  BUB: the bubble integrands (kinds 0 and 1); otherwise the unit
// integrand.  WE: per-pair errors are stored (FP32 records and deltas);
// otherwise the children's errors only form their keys.  WW: the keys weigh
// the pairs (per-integral and weighted modes); otherwise they are plain sums.
template <bool BUB, bool WE, bool WW>
__device__ void lpc_group(const Problem &P, int erow, const double *tab, double *Yw, int g0,
                          int gend, int s0) {
  using namespace lpc;
  // the parameter row's constants in scalar registers (read for each group
  // rather than held in vector registers across the kernel's loops)
  const Entry &Erow = P.entries[erow];
  Entry E;
  E.t = wave_uniform(Erow.t);
  E.tp = wave_uniform(Erow.tp);
  E.mu = wave_uniform(Erow.mu);
  E.w = wave_uniform(Erow.w);
  E.inv_w = wave_uniform(Erow.inv_w);
  E.J = __builtin_amdgcn_readfirstlane(Erow.J);
  // the lane's place, formed anew for every group rather than held in
  // registers across the kernel's loops
  int lane = lane_id();
  asm volatile("" : "+v"(lane));
  const int it = lane >> 3, ch = (lane >> 1) & 3, h = lane & 1;
  const int cx = ch & 1, cy = ch >> 1;
  const int w = min(g0 + it, gend - 1);
  const int MU = P.MU;

  // ---- the items: placeholders, node rows
  int d, chl;
  double cxm = 0.0, sxm = 0.0, cLx, sLx;
  unsigned long long pm;
  bool wave_skip;
  {
    const LpcItem q = lpc_item(P, w, s0);
    const Ctr C = P.ctr[P.cid[q.s]];
    chl = C.ch;
    cLx = C.cLx;
    sLx = C.sLx;
    d = code_depth(q.pc);
    const uint64_t ix = code_ix(q.pc), iy = code_iy(q.pc);
    const uint64_t ccode = make_code(d + 1, 2 * ix + cx, 2 * iy + cy);
    // seed phase: children the seed tree splits again are placeholders
    const bool valid = g0 + it < gend;
    const bool phc = P.seed_y && (P.flags[q.s] & kFlagSeed) && seed_split(P, q.s, ccode);
    pm = __ballot(phc && valid);
    wave_skip = pm == __ballot(valid);  // every child of the group is one
    // trigonometric values of the nodes by angle addition: node a of a child
    // lies at offset delta_a (a table per depth) from the child's centre,
    // whose sine and cosine each lane pair forms once (lane 0 for x, lane 1
    // for y)
    if (!wave_skip) {
      const double wdt = kTwoPi * ldexp(1.0, -d);
      const double xm = -kPi + (double)ix * wdt + (0.25 + 0.5 * cx) * wdt;
      const double ym = -kPi + (double)iy * wdt + (0.25 + 0.5 * cy) * wdt;
      const double2 sc = sincos_out_of_line(h ? ym : xm);
      const double c1 = sc.y, s1 = sc.x;
      const double c2 = lpc::swap_h(c1), s2 = lpc::swap_h(s1);
      cxm = h ? c2 : c1;
      sxm = h ? s2 : s1;
      // rows of both child rows of every item: cos(l_y/2 + y), cos(l_y/2 - y), phi_1..4(y)
#pragma unroll 1
      for (int t0 = 0; t0 < kItems * 2 * kNF; t0 += 64) {
        // every lane takes part in the exchanges; lanes past the last row idle after them
        const int t = t0 + lane, ti = min(t / (2 * kNF), kItems - 1);
        const int rem = t - ti * (2 * kNF), tcy = min(rem / kNF, 1), b = rem - tcy * kNF;
        const int src = 8 * ti + 4 * tcy + 1;  // lane 1 of child (0, tcy) of item ti
        const double cm = __shfl(c1, src, 64), sm = __shfl(s1, src, 64);
        const double cL = __shfl(C.cLy, src, 64), sL = __shfl(C.sLy, src, 64);
        const int td = __shfl(d, 8 * ti, 64);
        if (t >= kItems * 2 * kNF) continue;
        const int bb = b < 5 ? b : 8 - b;
        const double cd = c_rule.cdel[td][bb];
        const double sd = b < 5 ? c_rule.sdel[td][bb] : -c_rule.sdel[td][bb];
        const double cyv = cm * cd - sm * sd, sy = sm * cd + cm * sd;
        double *row = Yw + (ti * 2 + tcy) * kYBlock + b * kYRow;
        row[0] = cL * cyv - sL * sy;  // cos(l_y/2 + y)
        row[1] = cL * cyv + sL * sy;  // cos(l_y/2 - y)
        row[2] = kSqrt2 * cyv;
        row[3] = kSqrt2 * sy;
        row[4] = (cyv - sy) * (cyv + sy);
        row[5] = 2.0 * sy * cyv;
      }
    }
  }
  wave_sync();

  // ---- the integrand and the sums
  const double *Yc = Yw + (it * 2 + cy) * kYBlock;
  const double mt2 = -2.0 * E.t, mtp4 = -4.0 * E.tp;
  double I[5][5];
#pragma unroll
  for (int j = 0; j < 5; ++j)
#pragma unroll
    for (int k = 0; k < 5; ++k) I[j][k] = 0.0;

  // cos and sin of column a of this lane's child
  auto column_trig = [&](int a, double &cxv, double &sx) {
    const int aa = a < 5 ? a : 8 - a;
    const double cd = c_rule.cdel[d][aa], sd = a < 5 ? c_rule.sdel[d][aa] : -c_rule.sdel[d][aa];
    cxv = cxm * cd - sxm * sd;
    sx = sxm * cd + cxm * sd;
  };
  // the integrand along rows [b0, b1) of column a: y-sums with the fine (H2)
  // and the coarse (H1) weights
  auto column = [&](int a, int b0, int b1, double (&H2)[5], double (&H1)[5]) {
    double cxv, sx;
    column_trig(a, cxv, sx);
    const double Cx = cLx * cxv - sLx * sx, Dx = cLx * cxv + sLx * sx;
    // the energies along the column are affine in the row's cosine:
    // -2t (Cx + py) - 4t' Cx py - mu = (-2t Cx - mu) + py (-2t - 4t' Cx)
    const double Aa = fma(mt2, Cx, -E.mu), Ba = fma(mtp4, Cx, mt2);
    const double Ab = fma(mt2, Dx, -E.mu), Bb = fma(mtp4, Dx, mt2);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      H2[k] = 0.0;
      H1[k] = 0.0;
    }
#pragma unroll 1
    for (int b = b0; b < b1; ++b) {
      const double *row = Yc + b * kYRow;
      double g = 1.0;  // PAID_UNIT
      if constexpr (BUB) g = K_eval(E, tab, chl, fma(row[0], Ba, Aa), fma(row[1], Bb, Ab));
      const double g2 = c_rule.w2[b] * g, g1 = ((b & 1) ? 0.0 : c_rule.w1[b >> 1]) * g;
      H2[0] += g2;
      H1[0] += g1;
#pragma unroll
      for (int k = 1; k < 5; ++k) {
        H2[k] = fma(g2, row[1 + k], H2[k]);
        H1[k] = fma(g1, row[1 + k], H1[k]);
      }
    }
  };
  // phi_j at column a
  auto column_basis = [&](int a, double (&px)[5]) {
    double cxv, sx;
    column_trig(a, cxv, sx);
    px[0] = 1.0;
    px[1] = kSqrt2 * cxv;
    px[2] = kSqrt2 * sx;
    px[3] = (cxv - sx) * (cxv + sx);
    px[4] = 2.0 * sx * cxv;
  };
  // x-sums of one column from its y-sum vector dk: lane 0 adds the fine
  // rule's sums (wf H2), lane 1 fine minus coarse (wf H2 - wc H1)
  auto xsum = [&](const double (&dk)[5], const double (&px)[5]) {
#pragma unroll
    for (int k = 0; k < 5; ++k) I[0][k] += dk[k];
#pragma unroll
    for (int j = 1; j < 5; ++j)
#pragma unroll
      for (int k = 0; k < 5; ++k) I[j][k] = fma(px[j], dk[k], I[j][k]);
  };
  // one step: this lane's column a and the partner's; each lane forms the
  // y-sum vector the partner needs from its own column and swaps it
  auto step = [&](int a, int b0, int b1, double wf, double wc, bool split) {
    double H2[5], H1[5];
    column(a, b0, b1, H2, H1);
    if (split) {  // both lanes hold part of the same column: add the parts
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        H2[k] += lpc::swap_h(H2[k]);
        H1[k] += lpc::swap_h(H1[k]);
      }
    }
    const double wown = h ? wc : 0.0, wsend = h ? 0.0 : wc;
    double dk[5], sk[5], px[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      dk[k] = fma(wf, H2[k], -wown * H1[k]);
      sk[k] = fma(wf, H2[k], -wsend * H1[k]);
    }
    column_basis(a, px);
    xsum(dk, px);
    if (!split) {
#pragma unroll
      for (int k = 0; k < 5; ++k) sk[k] = lpc::swap_h(sk[k]);
#pragma unroll
      for (int j = 1; j < 5; ++j) px[j] = lpc::swap_h(px[j]);
      xsum(sk, px);
    }
  };

  if (!wave_skip) {
    // columns s (lane 0) and 8 - s (lane 1), s = 0..3: the CC weights are
    // symmetric, so both columns of a step carry the same weights
#pragma unroll 1
    for (int st = 0; st < 4; ++st)
      step(h ? 8 - st : st, 0, kNF, c_rule.w2[st], (st & 1) ? 0.0 : c_rule.w1[st >> 1], false);
    // column 4: rows 0-4 on lane 0, rows 5-8 on lane 1
    step(4, h ? 5 : 0, h ? kNF : 5, c_rule.w2[4], c_rule.w1[2], true);
  }
  // the item's bookkeeping is read again below rather than held in
  // registers across the loops above
  asm volatile("" ::: "memory");

  // ---- records: lane 0 writes the child's Q_2N, lane 1 its |E| and key;
  // the lanes of child 0 write the item's deltas (children minus parent, the
  // parent's values from LDS), summed over the four children
  const LpcItem q = lpc_item(P, w, s0);
  // the parents' values (their records are overwritten by child 0 below):
  // Q, and E and the key weights where the mode uses them, in the LDS that
  // held the node rows
  double *PQ = Yw, *PE = PQ + kItems * lpc::kPairs;
  double *PW = PE + (P.E ? kItems * lpc::kPairs : 0);
  for (int k = lane & 7; k < MU; k += 8) {
    PQ[it * lpc::kPairs + k] = P.Q[q.pbase * MU + k];
    if (P.E) PE[it * lpc::kPairs + k] = (double)P.E[q.pbase * MU + k];
    if (P.err_mode != 0) PW[it * lpc::kPairs + k] = (double)P.itau[(long)q.s * MU + k];
  }
  wave_sync();
  const bool valid = g0 + it < gend;
  const int dd = code_depth(q.pc);
  const uint64_t ix = code_ix(q.pc), iy = code_iy(q.pc);
  const uint64_t ccode = make_code(dd + 1, 2 * ix + cx, 2 * iy + cy);
  const bool phc = (pm >> lane) & 1ull;
  const bool item_skip = ((pm >> (8 * it)) & 0xFFull) == 0xFFull;
  const double pkey = P.key[q.pbase];
  const double wdt = kTwoPi * ldexp(1.0, -dd);
  const double fa = (0.25 * wdt) * (0.25 * wdt) / (4.0 * kPi * kPi);
  const double fx = phc ? 0.0 : fa;  // placeholders store zeros
  const long ri = (ch == 0) ? q.leaf : (long)P.nleaf[q.s] + 3L * q.r + (ch - 1);
  const long base = slot_base(P, q.s) + ri;
  const long itm = (long)q.s * P.bmax + q.r;
  const bool head = valid && ch == 0;
  const double *par = (h ? PE : PQ) + it * lpc::kPairs;
  [[maybe_unused]] const double *wgt = P.err_mode != 0 ? PW + it * lpc::kPairs : nullptr;
  double *dst = h ? P.dep : P.dv;
  double key = 0.0;
  constexpr lpc::PairTab PT = lpc::make_pair_tab();
#pragma unroll
  for (int p = 0; p < lpc::kPairs; ++p) {
    const signed char *tp = PT.t[p];
    double v = I[tp[0]][tp[3]];
    if (tp[4] >= 0) v = tp[5] > 0 ? v + I[tp[0]][tp[4]] : v - I[tp[0]][tp[4]];
    if (tp[1] >= 0) {
      double u = I[tp[1]][tp[3]];
      if (tp[4] >= 0) u = tp[5] > 0 ? u + I[tp[1]][tp[4]] : u - I[tp[1]][tp[4]];
      v = tp[2] > 0 ? v + u : v - u;
    }
    const double x = fx * v;  // lane 0: Q_2N of the pair, lane 1: E
    const double e = fabs(x);
    if constexpr (WW)
      key += wgt ? e * wgt[p] : e;  // (the test keeps the weights' loads where they are used)
    else
      key += e;
    // lane 1's term of the children's sum: the same float-rounded error
    // that is stored and later subtracted (without stored errors lane 1's
    // sum is not used)
    double term = x;
    if constexpr (WE) {
      const float ef = err_f32(e);
      if (h == 1 && valid) P.E[base * MU + p] = ef;
      if (h) term = (double)ef;
    }
    if (h == 0 && valid) P.Q[base * MU + p] = x;
    const double sum = lpc::child_sum(term);
    if (head && dst) dst[itm * MU + p] = sum - par[p];
  }
  // child keys (lane 1) and the item's key delta
  const double kk = lpc::child_sum(h ? key : 0.0);
  if (valid) {
    if (h == 1) P.key[base] = key;
    else P.code[base] = ccode;
    if (P.born && h == 0) P.born[base] = (unsigned int)(1 + 4 * P.st_splits[q.s] + ch);
  }
  if (head && h == 1) P.de[itm] = kk - pkey;
  if (head && h == 0) {
    if (P.ifill) P.ifill[itm] = !item_skip;
    if (dd + 1 > P.st_depth[q.s]) atomicMax(&P.st_depth[q.s], dd + 1);
  }
}

// The same work partition and table staging as k_children; inside a segment
// (items of one parameter row) wave wv takes the groups of 8 items that
// start at seg + 8 (wv + nw k).
template <bool BUB, bool WE, bool WW>
__global__ void __launch_bounds__(512) k_children_lpc(Problem P) {
  extern __shared__ double lds_raw[];
  double *tabl = lds_raw;
  const int nw = blockDim.x >> 6, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  double *Yw = lds_raw + (size_t)P.tab_rows * kTabStride + (size_t)wv * P.lds_wave_doubles;
  int i0, i1;
  item_range(P, i0, i1);
  if (i0 >= i1) return;  // uniform in the workgroup
  int s = item_slot(P, i0), hi = P.woff[s + 1];
  int seg = i0, loaded = -1;
#pragma unroll 1
  while (seg < i1) {
    const int e = __builtin_amdgcn_readfirstlane(slot_entry(P, s));
    int t = s + 1;
    while (t < P.W && P.woff[t] < i1 && (P.woff[t + 1] == P.woff[t] || slot_entry(P, t) == e)) ++t;
    const int seg_hi = (t < P.W && P.woff[t] < i1) ? P.woff[t] : i1;
    if (e != loaded) {
      __syncthreads();  // every wave is done with the previous table
      const Entry E0 = P.entries[e];
      const double *src = P.tab + E0.tab_off;
      for (int i = threadIdx.x; i < E0.J * kTabStride; i += blockDim.x) tabl[i] = src[i];
      __syncthreads();
      loaded = e;
    }
#pragma unroll 1
    for (int g = seg + lpc::kItems * wv; g < seg_hi; g += lpc::kItems * nw) {
      if (g >= hi) {  // slot holding item g (woff is non-decreasing)
        int a = s + 1, b = P.W;  // woff[a] <= g < woff[b]
        while (b - a > 1) {
          const int mid = (a + b) >> 1;
          if (P.woff[mid] <= g) a = mid; else b = mid;
        }
        s = a;
        hi = P.woff[s + 1];
      }
      lpc_group<BUB, WE, WW>(kernarg_problem(P), e, tabl, Yw, g, seg_hi, s);
    }
    seg = seg_hi;
    if (seg < i1) {
      s = t;
      hi = P.woff[s + 1];
    }
  }
}

// ---------------------------------------------------------------- diagnostics
__global__ void k_kernel_eval(const Entry *e, const double *tab, int ch, const double *a,
                              const double *b, int n, double *out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Entry E = *e;
  out[i] = K_eval(E, tab + E.tab_off, ch, a[i], b[i]);
}

template <int L, int GRAM>
hipError_t launch_root_t(const Problem &p, hipStream_t s) {
  size_t sh = sizeof(double) * wave_lds_doubles<L>(p.ff_identity);
  hipLaunchKernelGGL((k_root<L, GRAM>), dim3(p.W), dim3(64), sh, s, p);
  return hipGetLastError();
}

// Dynamic LDS of the evaluation kernel: the largest table plus one WaveLds
// per wave, as many waves (up to 4) as fit in 64 KiB, or one wave in the
// device's limit when the table is larger.  Returns 0 if not even that fits.
template <int L>
size_t eval_lds_t(const Problem &p, int *waves_out, int *wave_doubles_out) {
  const size_t wave_b = sizeof(double) * wave_lds_doubles<L>(p.ff_identity);
  // fixed: the kernel's static LDS (two int tables over the form-factor pairs)
  const size_t tab_b = sizeof(double) * (size_t)p.tab_rows * kTabStride, fixed = 4096;
  size_t budget = 65536;
  if (tab_b + wave_b + fixed > budget) budget = p.lds_limit > 0 ? (size_t)p.lds_limit : 65536;
  if (tab_b + wave_b + fixed > budget) return 0;
  int waves = (int)((budget - fixed - tab_b) / wave_b);
  waves = waves > 4 ? 4 : waves;
  if (waves_out) *waves_out = waves;
  if (wave_doubles_out) *wave_doubles_out = (int)(wave_b / sizeof(double));
  return tab_b + (size_t)waves * wave_b;
}

template <int L, int GRAM>
int eval_occupancy_t(Problem p) {
  int waves = 0, wd = 0;
  const size_t sh = eval_lds_t<L>(p, &waves, &wd);
  if (sh == 0) return 1;
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void *>(&k_children<L, GRAM>),
                                                   64 * waves, sh) != hipSuccess || n < 1)
    n = 1;
  return n;
}

template <int L, int GRAM>
hipError_t launch_eval_t(Problem p, int grid, hipStream_t s) {
  int waves = 0, wd = 0;
  const size_t sh = eval_lds_t<L>(p, &waves, &wd);
  if (sh == 0) return hipErrorInvalidValue;
  p.lds_wave_doubles = wd;
  hipLaunchKernelGGL((k_children<L, GRAM>), dim3(grid), dim3(64 * waves), sh, s, p);
  return hipGetLastError();
}

// per-wave LDS of the two-lanes-per-child kernel (doubles)
int lpc_wave_doubles(const Problem &p) {
  return lpc::wave_doubles(p.E != nullptr, p.err_mode != 0);
}

// Dynamic LDS of the two-lanes-per-child kernel: the table and each wave's
// node rows and parent values.  The table is staged once per workgroup, so
// the number of waves per workgroup (4, 6 or 8; fewer only if nothing else
// fits the device's per-workgroup limit) is the one that keeps the most
// waves resident per CU, by the runtime's occupancy calculator; the choice
// is remembered per table and wave size.
// the two-lanes-per-child kernel for the problem's integrand
const void *lpc_kernel(const Problem &p) {
  static const void *const k[8] = {
      reinterpret_cast<const void *>(&k_children_lpc<false, false, false>),
      reinterpret_cast<const void *>(&k_children_lpc<false, false, true>),
      reinterpret_cast<const void *>(&k_children_lpc<false, true, false>),
      reinterpret_cast<const void *>(&k_children_lpc<false, true, true>),
      reinterpret_cast<const void *>(&k_children_lpc<true, false, false>),
      reinterpret_cast<const void *>(&k_children_lpc<true, false, true>),
      reinterpret_cast<const void *>(&k_children_lpc<true, true, false>),
      reinterpret_cast<const void *>(&k_children_lpc<true, true, true>)};
  return k[(p.kind <= 1 ? 4 : 0) + (p.E ? 2 : 0) + (p.err_mode != 0 ? 1 : 0)];
}

size_t lpc_lds(const Problem &p, int *waves_out) {
  const size_t wave_b = sizeof(double) * lpc_wave_doubles(p);
  const size_t tab_b = sizeof(double) * (size_t)p.tab_rows * kTabStride;
  const size_t limit = p.lds_limit > 0 ? (size_t)p.lds_limit : 65536;
  thread_local size_t memo_tab = 0, memo_wave = 0, memo_limit = 0;
  thread_local int memo_waves = 0;
  thread_local const void *memo_kern = nullptr;
  if (memo_waves == 0 || memo_tab != tab_b || memo_wave != wave_b || memo_limit != limit ||
      memo_kern != lpc_kernel(p)) {
    int best = 0, best_w = 0;
    for (int w : {4, 6, 8, 2, 1}) {
      const size_t sh = tab_b + (size_t)w * wave_b;
      if (sh > limit || (best > 0 && w < 4)) continue;
      int n = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, lpc_kernel(p), 64 * w, sh) != hipSuccess)
        n = 0;
      if (n < 1) n = (w < 4 && best == 0) ? 1 : 0;  // a last resort still runs
      if (n * w > best) {
        best = n * w;
        best_w = w;
      }
    }
    if (best_w == 0) return 0;
    memo_tab = tab_b;
    memo_kern = lpc_kernel(p);
    memo_wave = wave_b;
    memo_limit = limit;
    memo_waves = best_w;
  }
  if (waves_out) *waves_out = memo_waves;
  return tab_b + (size_t)memo_waves * wave_b;
}

}  // namespace

namespace {
// projection/precision mode of a problem: separable FP64, or the dense Gram
// in the requested precision
int gram_mode(const Problem &p) { return p.gram == PAID_GRAM_SEPARABLE ? kSep : p.precision; }

// the two-lanes-per-child kernel serves the 9-function box basis itself with
// the separable FP64 projection over the full zone (bubble and unit integrands)
bool use_lpc(const Problem &p) {
  return p.eval_layout == 0 && p.L == 1 && p.ff_identity && !p.sym && gram_mode(p) == kSep &&
         p.kind != PAID_GAUSS;
}

template <int L>
hipError_t launch_root_l(const Problem &p, hipStream_t s) {
  switch (gram_mode(p)) {
    case kSep: return launch_root_t<L, kSep>(p, s);
    case PAID_FP32: return launch_root_t<L, PAID_FP32>(p, s);
    case PAID_BF16X3: return launch_root_t<L, PAID_BF16X3>(p, s);
    default: return launch_root_t<L, PAID_FP64>(p, s);
  }
}

template <int L>
int eval_occupancy_l(const Problem &p) {
  switch (gram_mode(p)) {
    case kSep: return eval_occupancy_t<L, kSep>(p);
    case PAID_FP32: return eval_occupancy_t<L, PAID_FP32>(p);
    case PAID_BF16X3: return eval_occupancy_t<L, PAID_BF16X3>(p);
    default: return eval_occupancy_t<L, PAID_FP64>(p);
  }
}

template <int L>
hipError_t launch_eval_l(const Problem &p, int grid, hipStream_t s) {
  switch (gram_mode(p)) {
    case kSep: return launch_eval_t<L, kSep>(p, grid, s);
    case PAID_FP32: return launch_eval_t<L, PAID_FP32>(p, grid, s);
    case PAID_BF16X3: return launch_eval_t<L, PAID_BF16X3>(p, grid, s);
    default: return launch_eval_t<L, PAID_FP64>(p, grid, s);
  }
}
}  // namespace

hipError_t launch_root(const Problem &p, hipStream_t s) {
  switch (p.L) {
    case 0: return launch_root_l<0>(p, s);
    case 1: return launch_root_l<1>(p, s);
    default: return launch_root_l<2>(p, s);
  }
}

size_t eval_lds_bytes(const Problem &p) {
  if (use_lpc(p)) return lpc_lds(p, nullptr);
  switch (p.L) {
    case 0: return eval_lds_t<0>(p, nullptr, nullptr);
    case 1: return eval_lds_t<1>(p, nullptr, nullptr);
    default: return eval_lds_t<2>(p, nullptr, nullptr);
  }
}

int eval_occupancy(const Problem &p) {
  if (use_lpc(p)) {
    int waves = 0, n = 0;
    const size_t sh = lpc_lds(p, &waves);
    if (sh == 0) return 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, lpc_kernel(p), 64 * waves, sh) != hipSuccess || n < 1)
      n = 1;
    return n;
  }
  switch (p.L) {
    case 0: return eval_occupancy_l<0>(p);
    case 1: return eval_occupancy_l<1>(p);
    default: return eval_occupancy_l<2>(p);
  }
}

hipError_t launch_eval(const Problem &p, int grid, hipStream_t s) {
  if (use_lpc(p)) {
    int waves = 0;
    const size_t sh = lpc_lds(p, &waves);
    if (sh == 0) return hipErrorInvalidValue;
    Problem q = p;
    q.lds_wave_doubles = lpc_wave_doubles(p);
    void *args[] = {&q};
    const hipError_t e = hipLaunchKernel(lpc_kernel(p), dim3(grid), dim3(64 * waves), args, sh, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
  }
  switch (p.L) {
    case 0: return launch_eval_l<0>(p, grid, s);
    case 1: return launch_eval_l<1>(p, grid, s);
    default: return launch_eval_l<2>(p, grid, s);
  }
}

hipError_t launch_kernel_eval(const Entry *e, const double *tab, int ch, const double *a,
                              const double *b, int n, double *out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_kernel_eval, dim3((n + 255) / 256), dim3(256), 0, s, e, tab, ch, a, b, n,
                     out);
  return hipGetLastError();
}

}  // namespace paid
