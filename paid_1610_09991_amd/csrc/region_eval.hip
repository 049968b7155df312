// region_eval.hip -- the hot kernel: evaluation of rectangles with the nested
// Clenshaw-Curtis pair (Sec. 3) for all form-factor pairs at once.
//
// One wavefront owns one work item: a parent rectangle and its four children
// (Alg. 2: split into 4, evaluate Q_N and Q_2N on each).  The children share
// 17 x 17 node coordinates, so the integrand g is evaluated 289 times instead
// of 324.  Per child the projection onto the form factors is the weighted
// Gram contraction
//     Q_2N = U^T diag(w_2N g) U,   E = U^T diag((w_2N - w_N) g) U = Q_2N - Q_N,
// with U[node][m] the box basis at the 81 nodes, on the FP64 matrix cores
// (16x16x4 tiles; a 9-function basis fills one tile, 25 functions 2x2 tiles of
// which the lower-left one is skipped by symmetry).  err of a child is
// sum_pq |E_pq| (the paper's global error summed over pairs).
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

// per-wave scratch in LDS
struct WaveLds {
  double g[kNX * kNX];             // integrand at the shared nodes
  double cp[2][kNX], cm[2][kNX];   // cos(l/2 + p), cos(l/2 - p) per axis
  double u[2][kNX][kMaxNB];        // box harmonics per axis
  double pos[2][kNX];              // coordinates
  double cq[kMaxMU], ce[kMaxMU];   // one child's Q_2N and E over form-factor pairs
  double tq[kMaxMB * kMaxMB];      // box Gram of Q_2N (general form-factor sets only)
  double ts[kMaxMB * kMaxMB];      // box Gram of E
  double tr[kMaxMB * kMaxMB];      // half-transformed Gram
};

__device__ inline void wave_sync() { __syncthreads(); }  // one wave per workgroup

__device__ inline int pair_index(int p, int q, int M) { return p * M - p * (p - 1) / 2 + (q - p); }

// Coordinates of one axis: nco = 17 (four children of a rectangle of width
// wdt starting at x0) or 9 (a single rectangle).
__device__ inline double axis_coord(int j, int nco, double x0, double wdt) {
  if (nco == kNF) return x0 + 0.5 * wdt + 0.5 * wdt * c_rule.xi[j];
  if (j <= 8) return x0 + 0.25 * wdt + 0.25 * wdt * c_rule.xi[j];
  return x0 + 0.75 * wdt + 0.25 * wdt * c_rule.xi[j - 8];
}

// Fill per-axis data and the integrand on the nco x nco node grid.
__device__ void fill_nodes(WaveLds &S, const Problem &P, const Ctr &C, const Entry &E,
                           const double *tab, int nco, double x0, double y0, double wdt) {
  const int lane = threadIdx.x;
  if (lane < 2 * nco) {
    int ax = lane >= nco, j = lane - ax * nco;
    double p = axis_coord(j, nco, ax ? y0 : x0, wdt);
    double sp, cpp;
    sincos(p, &sp, &cpp);
    double cL = ax ? C.cLy : C.cLx, sL = ax ? C.sLy : C.sLx;
    S.pos[ax][j] = p;
    S.cp[ax][j] = cL * cpp - sL * sp;  // cos(l/2 + p)
    S.cm[ax][j] = cL * cpp + sL * sp;  // cos(l/2 - p)
    S.u[ax][j][0] = 1.0;
    if (P.L >= 1) {
      S.u[ax][j][1] = kSqrt2 * cpp;
      S.u[ax][j][2] = kSqrt2 * sp;
    }
    if (P.L >= 2) {
      S.u[ax][j][3] = kSqrt2 * (cpp - sp) * (cpp + sp);
      S.u[ax][j][4] = kSqrt2 * 2.0 * sp * cpp;
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

// Weighted Gram of one rectangle on the FP64 matrix cores.  Its 9 x 9 nodes
// are rows offx.. and columns offy.. of the nco x nco grid.  Results go to
// S.cq / S.ce (identity form factors) or S.tq / S.ts (box Gram, general).
template <int NT>
__device__ void gram_fp64(WaveLds &S, const Problem &P, int nco, int offx, int offy, double fa) {
  const int lane = threadIdx.x, m = lane & 15, kk = lane >> 4;
  const int MB = P.MB, nb = P.nb;
  const bool v0 = m < MB, v1 = (NT == 2) && (m + 16 < MB);
  const int a0 = v0 ? m / nb : 0, b0 = v0 ? m - (m / nb) * nb : 0;
  const int a1 = v1 ? (m + 16) / nb : 0, b1 = v1 ? (m + 16) - ((m + 16) / nb) * nb : 0;
  constexpr int NACC = NT * (NT + 1) / 2;
  d4 aq[NACC], ae[NACC];
#pragma unroll
  for (int t = 0; t < NACC; ++t) {
    aq[t] = d4{0.0, 0.0, 0.0, 0.0};
    ae[t] = d4{0.0, 0.0, 0.0, 0.0};
  }
#pragma unroll 3
  for (int kb = 0; kb < 21; ++kb) {
    int nu = 4 * kb + kk;
    double u0 = 0.0, u1 = 0.0, gq = 0.0, ge = 0.0;
    if (nu < kNF * kNF) {
      int a = nu / kNF, b = nu - a * kNF;
      int gx = offx + a, gy = offy + b;
      double g = S.g[gx * nco + gy];
      double w2 = c_rule.w2[a] * c_rule.w2[b];
      double wn = ((a | b) & 1) ? 0.0 : c_rule.w1[a >> 1] * c_rule.w1[b >> 1];
      gq = g * w2;
      ge = g * (w2 - wn);
      if (v0) u0 = S.u[0][gx][a0] * S.u[1][gy][b0];
      if (v1) u1 = S.u[0][gx][a1] * S.u[1][gy][b1];
    }
    aq[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(u0 * gq, u0, aq[0], 0, 0, 0);
    ae[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(u0 * ge, u0, ae[0], 0, 0, 0);
    if (NT == 2) {
      aq[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(u0 * gq, u1, aq[1], 0, 0, 0);
      ae[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(u0 * ge, u1, ae[1], 0, 0, 0);
      aq[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(u1 * gq, u1, aq[2], 0, 0, 0);
      ae[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(u1 * ge, u1, ae[2], 0, 0, 0);
    }
  }
  // result lane layout of the f64 16x16x4 tile: row = 4 r + lane >> 4, col = lane & 15
#pragma unroll
  for (int t = 0; t < NACC; ++t) {
    int tr = (NT == 2 && t == 2) ? 1 : 0, tc = (NT == 2 && t >= 1) ? 1 : 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int i = 16 * tr + 4 * r + kk, j = 16 * tc + m;
      if (i < MB && j < MB && i <= j) {
        double q = fa * aq[t][r], e = fa * ae[t][r];
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
  }
  wave_sync();
}

// General form-factor sets: Q_ff = C Q_box C^T for both Q and E.
__device__ void transform_ff(WaveLds &S, const Problem &P) {
  const int lane = threadIdx.x, MB = P.MB, M = P.M;
  double *R = S.tr;
  for (int which = 0; which < 2; ++which) {
    const double *G = which ? S.ts : S.tq;
    // R[a][q] = sum_b G[a][b] C[q][b]
    for (int idx = lane; idx < MB * M; idx += 64) {
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

__device__ inline double wave_sum(double v) {
  // fixed butterfly order: deterministic
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Store one evaluated rectangle (S.cq, S.ce) into pool slot `ri` of slot s,
// return its key.
__device__ double store_region(WaveLds &S, const Problem &P, int s, long ri, uint64_t code) {
  const int lane = threadIdx.x;
  const long base = (long)s * P.cap + ri;
  double part = 0.0;
  for (int pid = lane; pid < P.MU; pid += 64) {
    double q = S.cq[pid], e = fabs(S.ce[pid]);
    P.Q[base * P.MU + pid] = q;
    if (P.E) P.E[base * P.MU + pid] = (float)e;
    part += (P.err_mode == 1) ? e * (double)P.itau[(long)s * P.MU + pid] : e;
  }
  double key = wave_sum(part);
  if (lane == 0) {
    P.key[base] = key;
    P.code[base] = code;
  }
  return key;
}

template <int NT>
__device__ void eval_rect(WaveLds &S, const Problem &P, int nco, int offx, int offy, double fa) {
  gram_fp64<NT>(S, P, nco, offx, offy, fa);
  if (!P.ff_identity) transform_ff(S, P);
}

// ---------------------------------------------------------------- root
template <int NT>
__global__ void __launch_bounds__(64) k_root(Problem P) {
  extern __shared__ double lds_raw[];
  WaveLds &S = *reinterpret_cast<WaveLds *>(lds_raw);
  const int s = blockIdx.x;
  if (s >= P.W || P.state[s] != SLOT_NEW) return;
  const int c = P.cid[s];
  const Ctr C = P.ctr[c];
  const Entry E = P.entries[C.entry];
  const double *tab = P.tab + E.tab_off;
  // key weights for the per-integral mode start at one
  for (int pid = threadIdx.x; pid < P.MU; pid += 64) P.itau[(long)s * P.MU + pid] = 1.0f;
  wave_sync();
  fill_nodes(S, P, C, E, tab, kNF, -kPi, -kPi, kTwoPi);
  eval_rect<NT>(S, P, kNF, 0, 0, kPi * kPi / (4.0 * kPi * kPi));
  double key = store_region(S, P, s, 0, make_code(0, 0, 0));
  for (int pid = threadIdx.x; pid < P.MU; pid += 64) {
    P.val[(long)s * P.MU + pid] = S.cq[pid];
    if (P.errp) P.errp[(long)s * P.MU + pid] = (double)(float)fabs(S.ce[pid]);
  }
  if (threadIdx.x == 0) {
    P.err[s] = key;
    P.nleaf[s] = 1;
    P.st_rounds[s] = 0;
    P.st_splits[s] = 0;
    P.st_depth[s] = 0;
    P.flags[s] = 0;
    P.state[s] = SLOT_ACTIVE;
  }
}

// ---------------------------------------------------------------- children
template <int NT>
__global__ void __launch_bounds__(64) k_children(Problem P) {
  extern __shared__ double lds_raw[];
  WaveLds &S = *reinterpret_cast<WaveLds *>(lds_raw);
  const int lane = threadIdx.x;
  const int total = P.counters[2];
#pragma unroll 1
  for (int w = blockIdx.x; w < total; w += gridDim.x) {
    // slot of this work item: woff is an exclusive prefix over slots
    int lo = 0, hi = P.W;  // woff[lo] <= w < woff[hi]
    while (hi - lo > 1) {
      int mid = (lo + hi) >> 1;
      if (P.woff[mid] <= w) lo = mid; else hi = mid;
    }
    const int s = lo, r = w - P.woff[s];
    const long leaf = P.sel[(long)s * P.bmax + r];
    const long nold = P.nleaf[s];
    const long pbase = (long)s * P.cap + leaf;
    const uint64_t pc = P.code[pbase];
    const double pkey = P.key[pbase];
    const Ctr C = P.ctr[P.cid[s]];
    const Entry E = P.entries[C.entry];
    const double *tab = P.tab + E.tab_off;
    // delta of the container sums: minus the parent, plus its children
    constexpr int KMAX = NT == 1 ? (136 + 63) / 64 : (kMaxMU + 63) / 64;
    double dv[KMAX], dp[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      int pid = lane + 64 * k;
      dv[k] = (pid < P.MU) ? -P.Q[pbase * P.MU + pid] : 0.0;
      dp[k] = (pid < P.MU && P.E) ? -(double)P.E[pbase * P.MU + pid] : 0.0;
    }
    const int d = code_depth(pc);
    const uint64_t ix = code_ix(pc), iy = code_iy(pc);
    const double wdt = kTwoPi * ldexp(1.0, -d);
    const double x0 = -kPi + (double)ix * wdt, y0 = -kPi + (double)iy * wdt;
    fill_nodes(S, P, C, E, tab, kNX, x0, y0, wdt);
    const double fa = (0.25 * wdt) * (0.25 * wdt) / (4.0 * kPi * kPi);
    double dkey = -pkey;
#pragma unroll 1
    for (int ch = 0; ch < 4; ++ch) {
      int cx = ch & 1, cy = ch >> 1;
      eval_rect<NT>(S, P, kNX, 8 * cx, 8 * cy, fa);
      long ri = (ch == 0) ? leaf : nold + 3L * r + (ch - 1);
      dkey += store_region(S, P, s, ri, make_code(d + 1, 2 * ix + cx, 2 * iy + cy));
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        int pid = lane + 64 * k;
        if (pid < P.MU) {
          dv[k] += S.cq[pid];
          // the same float-rounded value that is stored and later subtracted,
          // so the running per-pair error sums carry no rounding residue
          dp[k] += (double)(float)fabs(S.ce[pid]);
        }
      }
      wave_sync();
    }
    const long it = (long)s * P.bmax + r;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      int pid = lane + 64 * k;
      if (pid < P.MU) {
        P.dv[it * P.MU + pid] = dv[k];
        if (P.dep) P.dep[it * P.MU + pid] = dp[k];
      }
    }
    if (lane == 0) {
      P.de[it] = dkey;
      if (d + 1 > P.st_depth[s]) atomicMax(&P.st_depth[s], d + 1);
    }
  }
}

size_t lds_bytes(const Problem &P) {
  // the general-form-factor scratch sits at the end and is dropped otherwise
  size_t full = sizeof(WaveLds);
  return P.ff_identity ? full - 3 * sizeof(double) * kMaxMB * kMaxMB : full;
}

// ---------------------------------------------------------------- diagnostics
__global__ void k_kernel_eval(const Entry *e, const double *tab, int ch, const double *a,
                              const double *b, int n, double *out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Entry E = *e;
  out[i] = K_eval(E, tab + E.tab_off, ch, a[i], b[i]);
}

}  // namespace

hipError_t launch_root(const Problem &p, hipStream_t s) {
  size_t sh = lds_bytes(p);
  if (p.MB > 16)
    hipLaunchKernelGGL(k_root<2>, dim3(p.W), dim3(64), sh, s, p);
  else
    hipLaunchKernelGGL(k_root<1>, dim3(p.W), dim3(64), sh, s, p);
  return hipGetLastError();
}

hipError_t launch_eval(const Problem &p, int grid, hipStream_t s) {
  size_t sh = lds_bytes(p);
  if (p.MB > 16)
    hipLaunchKernelGGL(k_children<2>, dim3(grid), dim3(64), sh, s, p);
  else
    hipLaunchKernelGGL(k_children<1>, dim3(grid), dim3(64), sh, s, p);
  return hipGetLastError();
}

hipError_t launch_kernel_eval(const Entry *e, const double *tab, int ch, const double *a,
                              const double *b, int n, double *out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_kernel_eval, dim3((n + 255) / 256), dim3(256), 0, s, e, tab, ch, a, b, n,
                     out);
  return hipGetLastError();
}

}  // namespace paid
