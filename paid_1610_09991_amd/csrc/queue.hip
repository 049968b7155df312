// queue.hip -- the task container of Alg. 2 on the device: admission of
// containers into resident slots, worst-error-first bulk extraction, the
// flattened work list, the error/value updates and the final sums.
//
// Paper correspondence (Sec. 4): the heap keyed on the error becomes, per
// container, a histogram of the leaf keys (4 bins per octave) from which the
// largest keys are taken in order; Listing 2's MaxTask extraction becomes a
// per-round count that is at least `bmin`, covers every leaf whose key alone
// exceeds the tolerance (those must be split before the container can
// converge), and covers the error deficit ERR - eps; Listing 4's update
// (ERR -= parent, += children) is a fixed-order FP64 sum of per-parent
// deltas; the termination test of Listing 5 is re-checked on sums recomputed
// from the leaves before it is accepted.
#include <math.h>

#include "launch.h"

namespace paid {

namespace {

constexpr int kBins = 512;
constexpr int kSelThreads = 512;
// region codes hold ix and iy in 28 bits each: a rectangle of depth 28 (side
// 2 pi / 2^28) is the smallest one a code can hold and is never split
constexpr int kMaxDepth = 28;

// Block reductions over the pairwise tree that halves the block at every
// level (t with t + o, o = blockDim/2, ..., 1), evaluated in that order: the
// levels o >= 64 pair whole waves, so the first wave forms them per lane from
// one LDS write of the block, and the levels o < 64 are a butterfly of lane
// exchanges within it (lane t < o pairs with t + o, as in the tree).  Three
// barriers instead of one per level; the result is bit-identical to the tree
// for a fixed block size (a power of two, 64..1024).  sh holds blockDim + 1
// doubles (the last one broadcasts the result).
template <class Op>
__device__ inline double block_tree(double v, double *sh, Op op) {
  const int t = threadIdx.x, lane = t & 63, nw = blockDim.x >> 6;
  sh[t] = v;
  __syncthreads();
  if (t < 64) {
    double x[16];
#pragma unroll
    for (int w = 0; w < 16; ++w) x[w] = w < nw ? sh[w * 64 + lane] : 0.0;
#pragma unroll
    for (int h = 8; h >= 1; h >>= 1)
      if (h < nw)
#pragma unroll
        for (int w = 0; w < h; ++w) x[w] = op(x[w], x[w + h]);
    double r = x[0];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const double y = __shfl_xor(r, o, 64);
      r = lane < o ? op(r, y) : op(y, r);
    }
    if (t == 0) sh[blockDim.x] = r;
  }
  __syncthreads();
  const double r = sh[blockDim.x];
  __syncthreads();
  return r;
}

__device__ inline double block_sum(double v, double *sh) {
  return block_tree(v, sh, [](double a, double b) { return a + b; });
}

__device__ inline double block_max(double v, double *sh) {
  return block_tree(v, sh, [](double a, double b) { return fmax(a, b); });
}

// exclusive block prefix of an int flag/count; returns the block total
__device__ inline int block_scan(int v, int *sh, int &excl) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, nw = blockDim.x >> 6;
  int x = v;
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[wv] = x;
  __syncthreads();
  int before = 0, tot = 0;
  for (int w = 0; w < nw; ++w) {
    if (w < wv) before += sh[w];
    tot += sh[w];
  }
  excl = before + x - v;
  __syncthreads();
  return tot;
}

// Column sums of a row-major block A[rows][ncol] (float or double), in a
// fixed order: with ncol <= blockDim, thread t owns column t % ncol and the
// rows congruent to t / ncol modulo R = blockDim / ncol, reads are coalesced
// and four independent accumulators keep loads in flight; the R partials of
// a column are then added in order.  Wider blocks go column by column.
template <class T>
__device__ void column_sums(const T *A, long rows, int ncol, double *out, double *shd) {
  const int t = threadIdx.x, nt = blockDim.x;
  if (ncol <= nt) {
    const int R = nt / ncol, span = R * ncol;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    if (t < span) {
      const long N = rows * ncol;
      long e = t;
      for (; e + 3 * (long)span < N; e += 4 * (long)span) {
        a0 += (double)A[e];
        a1 += (double)A[e + span];
        a2 += (double)A[e + 2 * (long)span];
        a3 += (double)A[e + 3 * (long)span];
      }
      for (; e < N; e += span) a0 += (double)A[e];
    }
    shd[t] = (a0 + a1) + (a2 + a3);
    __syncthreads();
    if (t < ncol) {
      double s = 0.0;
      for (int r = 0; r < R; ++r) s += shd[r * ncol + t];
      out[t] = s;
    }
    __syncthreads();
  } else {
    for (int c = t; c < ncol; c += nt) {
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      long i = 0;
      for (; i + 3 < rows; i += 4) {
        a0 += (double)A[i * ncol + c];
        a1 += (double)A[(i + 1) * ncol + c];
        a2 += (double)A[(i + 2) * ncol + c];
        a3 += (double)A[(i + 3) * ncol + c];
      }
      for (; i < rows; ++i) a0 += (double)A[i * ncol + c];
      out[c] = (a0 + a1) + (a2 + a3);
    }
    __syncthreads();
  }
}

// Sum of the leaf keys of a slot (fixed order); with per-pair errors stored,
// also their column sums.  The values themselves are the running FP64 sums
// of Q over the leaves (updated at every split).
__device__ double resum_errors(const Problem &P, int s, double *shd) {
  const int t = threadIdx.x;
  const long n = P.nleaf[s], base = slot_base(P, s);
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  long i = t;
  const long st = blockDim.x;
  for (; i + 3 * st < n; i += 4 * st) {
    a0 += P.key[base + i];
    a1 += P.key[base + i + st];
    a2 += P.key[base + i + 2 * st];
    a3 += P.key[base + i + 3 * st];
  }
  for (; i < n; i += st) a0 += P.key[base + i];
  double k = block_sum((a0 + a1) + (a2 + a3), shd);
  if (t == 0) P.err[s] = k;
  if (P.E) column_sums(P.E + base * P.MU, n, P.MU, P.errp + (long)s * P.MU, shd);
  __syncthreads();
  return k;
}

// Relative margin below which the running error sums pass the termination
// test without being recomputed from the leaves.  The running sums drift
// from the leaf sums only by rounding: each round adds a fixed-order sum of
// the split items' deltas, each bounded by the largest running sum S, so
// the drift is at most about 2^-52 S per split and per round, 2e-10 S over a
// million splits; with S up to ~1e6 times the tolerance at rtol 1e-6 a
// margin of 1e-3 leaves a factor of five over that.
constexpr double kResumMargin = 1e-3;

// tolerance: 0 if the termination test fails, 1 if it passes but within
// the margin (the error sums must be recomputed from the leaves before it is
// accepted), 2 if it passes by more than the margin.  In the per-integral
// mode also refreshes the key weights 1/tau used for new children.
__device__ int tolerance_test(const Problem &P, int s, double *shd, double &eps, double &deficit) {
  const int t = threadIdx.x;
  double a = 0.0, mx = 0.0;
  for (int pid = t; pid < P.MU; pid += blockDim.x) {
    double v = fabs(P.val[(long)s * P.MU + pid]);
    a += v;
    mx = fmax(mx, v);
  }
  double l1 = block_sum(a, shd), vmax = block_max(mx, shd);
  if (P.err_mode == 0 || P.err_mode == 2) {
    if (P.err_mode == 0) {
      eps = fmax(P.atol, P.rtol * l1);
    } else {  // weighted sums (the keys carry the same weights)
      double aw = 0.0;
      for (int pid = t; pid < P.MU; pid += blockDim.x)
        aw += (double)P.itau[(long)s * P.MU + pid] * fabs(P.val[(long)s * P.MU + pid]);
      eps = fmax(P.atol, P.rtol * block_sum(aw, shd));
    }
    const double E = P.err[s];
    deficit = E - eps;
    return E <= eps * (1.0 - kResumMargin) ? 2 : (E <= eps ? 1 : 0);
  }
  // per integral: every pair within its own tolerance; deficit in tau units
  double ex = 0.0;
  int bad = 0, near = 0;
  for (int pid = t; pid < P.MU; pid += blockDim.x) {
    double v = fabs(P.val[(long)s * P.MU + pid]);
    double tau = fmax(P.atol, P.rtol * fmax(v, P.nu * vmax));
    double e = P.errp[(long)s * P.MU + pid];
    if (!(e <= tau)) {  // a NaN error fails the test
      bad = 1;
      ex += (e - tau) / tau;
    } else if (e > tau * (1.0 - kResumMargin)) {
      near = 1;
    }
    // FP32 weight, held at the largest float where tau is below FP32's range
    P.itau[(long)s * P.MU + pid] = (float)(tau > 0.0 ? fmin(1.0 / tau, 3.4028234663852886e38) : 0.0);
  }
  double excess = block_sum(ex, shd);
  double nbad = block_sum((double)bad, shd);
  double nnear = block_sum((double)near, shd);
  eps = 0.0;
  deficit = excess;
  return nbad != 0.0 ? 0 : (nnear != 0.0 ? 1 : 2);
}

__device__ inline int key_bin(double k, int emax_bits) {
  if (!(k > 0.0)) return kBins - 1;
  int b = emax_bits - (int)(__double_as_longlong(k) >> 50);
  return b < 0 ? 0 : (b > kBins - 1 ? kBins - 1 : b);
}

__global__ void __launch_bounds__(kSelThreads) k_select(Problem P) {
  __shared__ double shd[2 * kSelThreads];
  __shared__ int shi[kSelThreads];
  __shared__ unsigned int hcnt[kBins];
  __shared__ unsigned long long hsum[kBins];
  __shared__ int s_bfull, s_bpart, s_part, s_k;
  const int s = blockIdx.x, t = threadIdx.x;
  if (s >= P.W) return;
  if (P.state[s] != SLOT_ACTIVE) {
    if (t == 0) P.selcnt[s] = 0;
    return;
  }
  if (P.flags[s] & kFlagSeed) {
    // seed phase: the leaves the seed tree splits, in index order; no
    // termination test while placeholders may exist.  The seed tree has at
    // most cap/4 leaves, so the capacity is never reached here.
    const long n = P.nleaf[s], base = slot_base(P, s);
    long kl = (slot_cap(P, s) - n) / 3;
    if (kl > P.bmax) kl = P.bmax;
    if (kl > n) kl = n;
    const int kmax = (int)kl;
    int *sel = P.sel + (long)s * P.bmax;
    int out = 0;
    for (long b0 = 0; b0 < n && out < kmax; b0 += blockDim.x) {
      long i = b0 + t;
      int flag = (i < n) && seed_split(P, s, P.code[base + i]), ex;
      int tot = block_scan(flag, shi, ex);
      if (flag && out + ex < kmax) sel[out + ex] = (int)i;
      out += tot;
    }
    if (out > 0) {
      if (t == 0) P.selcnt[s] = out < kmax ? out : kmax;
      return;
    }
    __syncthreads();
    if (t == 0) P.flags[s] &= ~kFlagSeed;
    __syncthreads();
  }
  double eps, deficit;
  int conv = tolerance_test(P, s, shd, eps, deficit);
  if (conv == 1) {  // within the drift margin: accept only on sums recomputed from the leaves
    resum_errors(P, s, shd);
    conv = tolerance_test(P, s, shd, eps, deficit) != 0;
  }
  if (conv) {
    if (t == 0) {
      P.selcnt[s] = 0;
      P.flags[s] |= 1;
      P.state[s] = SLOT_DONE;
    }
    return;
  }
  const long n = P.nleaf[s], base = slot_base(P, s), cap = slot_cap(P, s);
  // in a small slot the container moves to a large one rather than split
  // fewer leaves than it would there
  const bool movable = P.Wb > 0 && s >= P.Wb;
  if (n + 3 > cap) {
    if (t == 0) {
      P.selcnt[s] = 0;
      if (movable) {
        P.state[s] = SLOT_MOVE;
      } else {
        P.flags[s] |= 2;
        P.state[s] = SLOT_DONE;
      }
    }
    return;
  }
  if (P.born) {
    // one leaf per round: the largest key, ties by creation order (the
    // serial algorithm's heap order)
    double bk = -1.0;
    unsigned int bb = 0xFFFFFFFFu;
    long bi = 0;
    for (long i = t; i < n; i += blockDim.x) {
      const double k = P.key[base + i];
      const unsigned int b = P.born[base + i];
      if (k > bk || (k == bk && b < bb)) {
        bk = k;
        bb = b;
        bi = i;
      }
    }
    for (int o = 32; o >= 1; o >>= 1) {  // within the wave
      const double k2 = __shfl_xor(bk, o, 64);
      const unsigned int b2 = __shfl_xor(bb, o, 64);
      const long i2 = __shfl_xor(bi, o, 64);
      if (k2 > bk || (k2 == bk && b2 < bb)) {
        bk = k2;
        bb = b2;
        bi = i2;
      }
    }
    if ((t & 63) == 0) {
      shd[t >> 6] = bk;
      shi[t >> 6] = (int)bb;
      shi[kSelThreads / 64 + (t >> 6)] = (int)bi;
    }
    __syncthreads();
    if (t == 0) {
      for (int w2 = 1; w2 < (int)(blockDim.x >> 6); ++w2) {
        const double k2 = shd[w2];
        const unsigned int b2 = (unsigned int)shi[w2];
        if (k2 > bk || (k2 == bk && b2 < bb)) {
          bk = k2;
          bb = b2;
          bi = shi[kSelThreads / 64 + w2];
        }
      }
      const int deep = code_depth(P.code[base + bi]) >= kMaxDepth;
      P.sel[(long)s * P.bmax] = (int)bi;
      P.selcnt[s] = deep ? 0 : 1;
      if (deep) {
        P.flags[s] |= 2;
        P.state[s] = SLOT_DONE;
      }
    }
    return;
  }
  long kmaxl = ((movable ? P.capb : cap) - n) / 3;
  if (kmaxl > P.bmax) kmaxl = P.bmax;
  if (kmaxl > n) kmaxl = n;
  const int kmax = (int)kmaxl;
  // pass 1: largest key (four loads in flight per thread)
  const long st = blockDim.x;
  double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0;
  {
    long i = t;
    for (; i + 3 * st < n; i += 4 * st) {
      m0 = fmax(m0, P.key[base + i]);
      m1 = fmax(m1, P.key[base + i + st]);
      m2 = fmax(m2, P.key[base + i + 2 * st]);
      m3 = fmax(m3, P.key[base + i + 3 * st]);
    }
    for (; i < n; i += st) m0 = fmax(m0, P.key[base + i]);
  }
  const double maxkey = block_max(fmax(fmax(m0, m1), fmax(m2, m3)), shd);
  // keys are binned and summed as k 2^-ke with ke = ilogb(maxkey): the same
  // bins as k itself wherever both are normal, and bins a quarter octave wide
  // also for keys in the subnormal range (whose raw exponent bits are zero)
  const bool kfin = maxkey > 0.0 && isfinite(maxkey);
  const int ke = kfin ? ilogb(maxkey) : 0;
  const int eb = (int)(__double_as_longlong(maxkey > 0.0 ? ldexp(maxkey, -ke) : 1.0) >> 50);
  // pass 2: histogram of counts and fixed-point sums (exact, order-free)
  for (int b = t; b < kBins; b += blockDim.x) {
    hcnt[b] = 0u;
    hsum[b] = 0ull;
  }
  __syncthreads();
  // fixed-point value of a key k: (k 2^-ke) * scale with scale =
  // 2^(62 - ceil(log2 n)) / (maxkey 2^-ke), i.e. k 2^(62 - ceil(log2 n)) / maxkey
  // with the power of two applied apart, so that the scale stays finite for a
  // subnormal maxkey. n keys of at most maxkey sum to at most 2^62, so no
  // bin, prefix or deficit overflows 64 bits.
  const int lgn = n > 1 ? 64 - __clzll((unsigned long long)(n - 1)) : 0;
  const double scale = kfin ? ldexp(1.0, 62 - lgn) / ldexp(maxkey, -ke) : 0.0;
  {
    long i = t;
    for (; i + 3 * st < n; i += 4 * st) {
      double k[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) k[j] = ldexp(P.key[base + i + j * st], -ke);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int b = key_bin(k[j], eb);
        atomicAdd(&hcnt[b], 1u);
        atomicAdd(&hsum[b], (unsigned long long)(k[j] * scale));
      }
    }
    for (; i < n; i += st) {
      const double k = ldexp(P.key[base + i], -ke);
      const int b = key_bin(k, eb);
      atomicAdd(&hcnt[b], 1u);
      atomicAdd(&hsum[b], (unsigned long long)(k * scale));
    }
  }
  __syncthreads();
  if (t < 64) {  // one wave scans the bins: 8 per lane
    const int lane = t;
    unsigned int c8 = 0;
    unsigned long long s8 = 0;
    for (int j = 0; j < 8; ++j) {
      c8 += hcnt[lane * 8 + j];
      s8 += hsum[lane * 8 + j];
    }
    unsigned int cinc = c8;
    unsigned long long sinc = s8;
    for (int o = 1; o < 64; o <<= 1) {
      unsigned int yc = __shfl_up(cinc, o, 64);
      unsigned long long ys = __shfl_up(sinc, o, 64);
      if (lane >= o) {
        cinc += yc;
        sinc += ys;
      }
    }
    unsigned int cex = cinc - c8;
    unsigned long long sex = sinc - s8;
    double dd = ldexp(deficit, -ke) * scale;
    unsigned long long dfix = dd >= 4.0e18 ? 4000000000000000000ull : (unsigned long long)(dd > 0 ? dd : 0.0);
    int beps = (P.err_mode != 1) ? key_bin(ldexp(eps, -ke), eb) : 0;
    if (P.err_mode != 1 && eps >= maxkey) beps = -1;  // no single leaf exceeds eps
    // first bin b (in this lane's 8) meeting all conditions
    int found = kBins, fcnt = 0;
    unsigned int cc = cex;
    unsigned long long ss = sex;
    for (int j = 0; j < 8; ++j) {
      int b = lane * 8 + j;
      cc += hcnt[b];
      ss += hsum[b];
      if (found == kBins && ss >= dfix && b >= beps && (int)cc >= P.bmin) {
        found = b;
        fcnt = (int)cc;
      }
    }
    // smallest lane with a hit
    int best = found;
    for (int o = 32; o >= 1; o >>= 1) best = min(best, __shfl_xor(best, o, 64));
    int bcnt = (found == best) ? fcnt : 0;
    for (int o = 32; o >= 1; o >>= 1) bcnt = max(bcnt, __shfl_xor(bcnt, o, 64));
    if (best == kBins) { best = kBins - 1; bcnt = (int)n; }
    int k = bcnt < kmax ? bcnt : kmax;
    // whole bins up to bfull, then `part` leaves of bin bfull+1 in index order
    int bfull = best, part = 0;
    if (bcnt > kmax) {
      // largest b with cumulative count <= kmax
      int lastb = -1;
      unsigned int c2 = cex;
      for (int j = 0; j < 8; ++j) {
        int b = lane * 8 + j;
        c2 += hcnt[b];
        if ((int)c2 <= kmax) lastb = b;
      }
      for (int o = 32; o >= 1; o >>= 1) lastb = max(lastb, __shfl_xor(lastb, o, 64));
      bfull = lastb;
      int cnt_full = 0;
      // cumulative count through bfull
      unsigned int c3 = cex;
      int mine = -1;
      for (int j = 0; j < 8; ++j) {
        int b = lane * 8 + j;
        c3 += hcnt[b];
        if (b == bfull) mine = (int)c3;
      }
      for (int o = 32; o >= 1; o >>= 1) mine = max(mine, __shfl_xor(mine, o, 64));
      cnt_full = bfull >= 0 ? mine : 0;
      part = kmax - cnt_full;
    }
    if (lane == 0) {
      s_bfull = bfull;
      s_bpart = bfull + 1;
      s_part = part;
      s_k = k;
    }
  }
  __syncthreads();
  if (movable && n + 3L * s_k > cap) {  // the round would overflow the small slot
    if (t == 0) {
      P.selcnt[s] = 0;
      P.state[s] = SLOT_MOVE;
    }
    return;
  }
  const int bfull = s_bfull, bpart = s_bpart, part = s_part;
  // pass 3: order-preserving compaction, four consecutive leaves per thread
  // and chunk.  One scan of both counts (16 bits each): the leaves of bin
  // bpart are taken in index order while room is left, so the place of a
  // taken leaf follows from the full-bin leaves and the bpart leaves before it
  int out = 0, seenpart = 0;
  int *sel = P.sel + (long)s * P.bmax;
  for (long b0 = 0; b0 < n; b0 += 4 * st) {
    const long i0 = b0 + 4 * t;
    int isp[4], full[4], np = 0, nf = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int bin = (i0 + j < n) ? key_bin(ldexp(P.key[base + i0 + j], -ke), eb) : kBins;
      isp[j] = (bin == bpart && i0 + j < n) ? 1 : 0;
      full[j] = (bin <= bfull && i0 + j < n) ? 1 : 0;
      np += isp[j];
      nf += full[j];
    }
    int ex;
    const int tot = block_scan(np | (nf << 16), shi, ex);
    const int totp = tot & 0xFFFF;
    const int room = part - seenpart > 0 ? part - seenpart : 0;
    int rp = ex & 0xFFFF, rf = ex >> 16;  // bpart and full-bin leaves before this one
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int pos = out + rf + (rp < room ? rp : room);
      if ((full[j] || (isp[j] && rp < room)) && pos < s_k) sel[pos] = (int)(i0 + j);
      rp += isp[j];
      rf += full[j];
    }
    out += (tot >> 16) + (totp < room ? totp : room);
    seenpart += totp;
    if (out >= s_k) break;
  }
  // a selected leaf at the deepest level a code can hold cannot be split:
  // the container stops with the budget flag, as on an exhausted pool
  const int ksel = out < s_k ? out : s_k;
  __syncthreads();  // sel is complete
  int deep = 0;
  for (int j = t; j < ksel; j += blockDim.x)
    deep |= code_depth(P.code[base + sel[j]]) >= kMaxDepth ? 1 : 0;
  deep = __syncthreads_or(deep);
  if (t == 0) {
    if (deep) {
      P.selcnt[s] = 0;
      P.flags[s] |= 2;
      P.state[s] = SLOT_DONE;
    } else {
      P.selcnt[s] = ksel;
    }
  }
}

__global__ void k_worklist(Problem P) {
  __shared__ int shi[1024];
  const int t = threadIdx.x;
  int carry = 0;
  for (int b0 = 0; b0 < P.W; b0 += blockDim.x) {
    int s = b0 + t, v = (s < P.W) ? P.selcnt[s] : 0, ex;
    int tot = block_scan(v, shi, ex);
    if (s < P.W) P.woff[s] = carry + ex;
    carry += tot;
  }
  if (t == 0) {
    P.woff[P.W] = carry;
    P.counters[2] = carry;
  }
}

// Container admission: empty slots take the next containers of the queue in
// slot order.
__global__ void k_admit(Problem P) {
  __shared__ int shi[1024];
  __shared__ int s_head;
  const int t = threadIdx.x;
  if (t == 0) s_head = *P.qhead;
  __syncthreads();
  if (s_head >= P.n_ctr) return;
  int head = s_head;
  for (int b0 = 0; b0 < P.W; b0 += blockDim.x) {
    // new containers start in small slots (all slots when there is one kind)
    int s = b0 + t, e = (s < P.W && s >= P.Wb && P.state[s] == SLOT_EMPTY) ? 1 : 0, ex;
    int tot = block_scan(e, shi, ex);
    if (e && head + ex < P.n_ctr) {
      const int k = head + ex;
      P.cid[s] = P.row_perm ? P.row_perm[k / P.per_row] * P.per_row + k % P.per_row : k;
      P.state[s] = SLOT_NEW;
    }
    head += tot;
  }
  if (t == 0) *P.qhead = head < P.n_ctr ? head : P.n_ctr;
}

// The per-parent deltas of a round, summed per container in a fixed order:
// a container's k work items are split into up to kUpdChunks chunks of at
// least kUpdMinRows consecutive items, each summed by its own workgroup
// (k_update_part), and the chunk sums are added in chunk order (k_update).
// With one chunk (k <= kUpdMinRows) the sums are those of one workgroup over
// all the items.
constexpr int kUpdChunks = 8, kUpdMinRows = 512;

__device__ inline int upd_chunks(int k) {
  const int c = (k + kUpdMinRows - 1) / kUpdMinRows;
  return c < kUpdChunks ? c : kUpdChunks;
}

// one chunk's sums: [MU] values, [MU] per-pair errors, key delta, filled items
__global__ void __launch_bounds__(kSelThreads) k_update_part(Problem P) {
  __shared__ double shd[2 * kSelThreads];
  const int s = blockIdx.x, c = blockIdx.y, t = threadIdx.x;
  if (s >= P.W) return;
  const int k = P.selcnt[s], nch = upd_chunks(k);
  if (c >= nch) return;
  const int per = (k + nch - 1) / nch, r0 = c * per, r1 = r0 + per < k ? r0 + per : k;
  const long it0 = (long)s * P.bmax + r0;
  const long MU = P.MU;
  double *part = P.upart + ((long)s * kUpdChunks + c) * (2 * MU + 2);
  column_sums(P.dv + it0 * MU, r1 - r0, P.MU, part, shd);
  if (P.dep) column_sums(P.dep + it0 * MU, r1 - r0, P.MU, part + MU, shd);
  double de = 0.0, nf = 0.0;
  for (int r = t; r < r1 - r0; r += blockDim.x) {
    de += P.de[it0 + r];
    nf += (double)P.ifill[it0 + r];
  }
  const double d = block_sum(de, shd);
  const double fills = block_sum(nf, shd);
  if (t == 0) {
    part[2 * MU] = d;
    part[2 * MU + 1] = fills;
  }
}

__global__ void __launch_bounds__(kSelThreads) k_update(Problem P) {
  const int s = blockIdx.x, t = threadIdx.x;
  if (s >= P.W) return;
  const int k = P.selcnt[s];
  if (k == 0) return;
  const int nch = upd_chunks(k);
  const long MU = P.MU;
  const double *part = P.upart + (long)s * kUpdChunks * (2 * MU + 2);
  for (long pid = t; pid < MU; pid += blockDim.x) {
    double v = part[pid];
    for (int c = 1; c < nch; ++c) v += part[c * (2 * MU + 2) + pid];
    P.val[(long)s * MU + pid] += v;
    if (P.dep) {  // per-pair error sums are kept where the deltas carry them
      double e = part[MU + pid];
      for (int c = 1; c < nch; ++c) e += part[c * (2 * MU + 2) + MU + pid];
      P.errp[(long)s * MU + pid] += e;
    }
  }
  if (t == 0) {
    double d = part[2 * MU], fills = part[2 * MU + 1];
    for (int c = 1; c < nch; ++c) {
      d += part[c * (2 * MU + 2) + 2 * MU];
      fills += part[c * (2 * MU + 2) + 2 * MU + 1];
    }
    P.err[s] += d;
    P.st_evals[s] += (long)fills * (kNX * kNX);
    P.nleaf[s] += 3 * k;
    P.st_rounds[s] += 1;
    P.st_splits[s] += k;
  }
}

// Labels of a finished tree: per cell of the 16 x 16 grid, log2(1 + n) with
// n the number of leaves in the cell (a leaf larger than a cell counts with
// the share of its area inside), written at the model cell of the container.
// All shares are powers of 1/4, so the LDS sums are exact in any order.
__device__ void tree_labels(const Problem &P, int s, long c, double *cnt) {
  const int t = threadIdx.x;
  for (int k = t; k < kSeedG * kSeedG; k += blockDim.x) cnt[k] = 0.0;
  __syncthreads();
  const long n = P.nleaf[s], base = slot_base(P, s);
  for (long i = t; i < n; i += blockDim.x) {
    const uint64_t code = P.code[base + i];
    const int d = code_depth(code), ix = (int)code_ix(code), iy = (int)code_iy(code);
    if (d >= 4) {
      atomicAdd(&cnt[((iy >> (d - 4)) << 4) + (ix >> (d - 4))], 1.0);
    } else {
      const int span = 1 << (4 - d);
      const double f = ldexp(1.0, -2 * (4 - d));
      for (int b = 0; b < span; ++b)
        for (int a = 0; a < span; ++a) atomicAdd(&cnt[((iy * span + b) << 4) + ix * span + a], f);
    }
  }
  __syncthreads();
  const int fold = P.seed_fold[c];
  for (int k = t; k < kSeedG * kSeedG; k += blockDim.x)
    P.labels[c * (kSeedG * kSeedG) + seed_model_cell(fold, k & 15, k >> 4)] = (float)log2(1.0 + cnt[k]);
}

__global__ void __launch_bounds__(kSelThreads) k_finalize(Problem P) {
  __shared__ double shd[2 * kSelThreads];
  const int s = blockIdx.x, t = threadIdx.x;
  if (s >= P.W || P.state[s] != SLOT_DONE) return;
  if (P.flags[s] & 2) resum_errors(P, s, shd);  // budget exit: error sums from the leaves
  const long c = P.cid[s];
  if (P.labels) tree_labels(P, s, c, shd);
  if (P.leaf_codes) {  // the leaves in pool order (codes and Q_2N), -1 past the last
    const long n = P.nleaf[s], base = slot_base(P, s);
    for (long i = t; i < P.leaf_cap; i += blockDim.x) {
      int *cd = P.leaf_codes + (c * P.leaf_cap + i) * 3;
      if (i < n) {
        const uint64_t code = P.code[base + i];
        cd[0] = code_depth(code);
        cd[1] = (int)code_ix(code);
        cd[2] = (int)code_iy(code);
        for (int k = 0; k < P.MU; ++k)
          P.leaf_q[(c * P.leaf_cap + i) * P.MU + k] = P.Q[(base + i) * P.MU + k];
      } else {
        cd[0] = cd[1] = cd[2] = -1;
      }
    }
  }
  const int M = P.M;
  for (int pid = t; pid < P.MU; pid += blockDim.x) {
    int p = 0, k = pid;
    while (k >= M - p) { k -= M - p; ++p; }
    int q = p + k;
    double v = P.val[(long)s * P.MU + pid];
    P.out[c * M * M + p * M + q] = v;
    P.out[c * M * M + q * M + p] = v;
    if (P.err_out) {
      double e = P.errp[(long)s * P.MU + pid];
      P.err_out[c * M * M + p * M + q] = e;
      P.err_out[c * M * M + q * M + p] = e;
    }
  }
  __syncthreads();
  if (t == 0) {
    atomicAdd(&P.counters[0], 1);
    if (P.flags[s] & 2) atomicAdd(&P.counters[1], 1);
    atomicAdd((unsigned long long *)&P.gstats[0], (unsigned long long)P.st_rounds[s]);
    atomicAdd((unsigned long long *)&P.gstats[1], (unsigned long long)P.st_splits[s]);
    atomicAdd((unsigned long long *)&P.gstats[2], (unsigned long long)P.nleaf[s]);
    atomicMax((unsigned long long *)&P.gstats[3], (unsigned long long)P.st_depth[s]);
    atomicAdd((unsigned long long *)&P.gstats[4], (unsigned long long)P.st_evals[s]);
    P.state[s] = SLOT_EMPTY;
  }
}

}  // namespace

// Moves from small to large slots, matched in slot order: the k-th waiting
// small slot takes the k-th free large slot (promo[b]: the small slot moving
// into large slot b this round, -1 if none).  One workgroup.
__global__ void k_move_match(Problem P) {
  __shared__ int shi[1024];
  const int t = threadIdx.x;
  int nw = 0;  // waiting small slots, in slot order, into moveq
  for (int b0 = P.Wb; b0 < P.W; b0 += blockDim.x) {
    const int s = b0 + t, e = (s < P.W && P.state[s] == SLOT_MOVE) ? 1 : 0;
    int ex;
    const int tot = block_scan(e, shi, ex);
    if (e) P.moveq[nw + ex] = s;
    nw += tot;
  }
  __syncthreads();  // moveq complete
  int nf = 0;  // free large slots so far
  for (int b0 = 0; b0 < P.Wb; b0 += blockDim.x) {
    const int b = b0 + t, e = (b < P.Wb && P.state[b] == SLOT_EMPTY) ? 1 : 0;
    int ex;
    const int tot = block_scan(e, shi, ex);
    if (b < P.Wb) P.promo[b] = (e && nf + ex < nw) ? P.moveq[nf + ex] : -1;
    nf += tot;
  }
}

// the leaves of each moving container, copied to its large slot (grid: large
// slots x chunks of the leaf range)
__global__ void k_move_copy(Problem P) {
  const int b = blockIdx.x, src = P.promo[b];
  if (src < 0) return;
  const long n = P.nleaf[src], per = (n + gridDim.y - 1) / gridDim.y;
  const long i0 = (long)blockIdx.y * per, i1 = i0 + per < n ? i0 + per : n;
  if (i0 >= i1) return;
  const long sb = slot_base(P, src), db = slot_base(P, b);
  for (long i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    P.code[db + i] = P.code[sb + i];
    P.key[db + i] = P.key[sb + i];
    if (P.born) P.born[db + i] = P.born[sb + i];
  }
  const long MU = P.MU;
  for (long e = i0 * MU + threadIdx.x; e < i1 * MU; e += blockDim.x) {
    P.Q[db * MU + e] = P.Q[sb * MU + e];
    if (P.E) P.E[db * MU + e] = P.E[sb * MU + e];
  }
}

// the moving containers' sums and bookkeeping; the large slot becomes active
// and the small one free for the next admission (grid: large slots)
__global__ void k_move_finish(Problem P) {
  const int b = blockIdx.x, src = P.promo[b], t = threadIdx.x;
  if (src < 0) return;
  const long MU = P.MU;
  for (long pid = t; pid < MU; pid += blockDim.x) {
    P.val[(long)b * MU + pid] = P.val[(long)src * MU + pid];
    P.itau[(long)b * MU + pid] = P.itau[(long)src * MU + pid];
    if (P.errp) P.errp[(long)b * MU + pid] = P.errp[(long)src * MU + pid];
  }
  if (P.pyr)
    for (int k = t; k < kPyr; k += blockDim.x) P.pyr[(long)b * kPyr + k] = P.pyr[(long)src * kPyr + k];
  if (t == 0) {
    P.cid[b] = P.cid[src];
    P.nleaf[b] = P.nleaf[src];
    P.flags[b] = P.flags[src];
    P.st_depth[b] = P.st_depth[src];
    P.st_rounds[b] = P.st_rounds[src];
    P.st_splits[b] = P.st_splits[src];
    P.st_evals[b] = P.st_evals[src];
    P.err[b] = P.err[src];
    if (P.seed_d) P.seed_d[b] = P.seed_d[src];
    P.selcnt[b] = 0;
    P.selcnt[src] = 0;
    P.state[b] = SLOT_ACTIVE;
    P.state[src] = SLOT_EMPTY;
  }
}

constexpr int kMoveChunks = 64;  // workgroups per moving container in k_move_copy

hipError_t launch_move(const Problem &p, hipStream_t s) {
  if (p.Wb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_move_match, dim3(1), dim3(1024), 0, s, p);
  hipLaunchKernelGGL(k_move_copy, dim3(p.Wb, kMoveChunks), dim3(256), 0, s, p);
  hipLaunchKernelGGL(k_move_finish, dim3(p.Wb), dim3(64), 0, s, p);
  return hipGetLastError();
}

// Predicted leaves of parameter row r: the sum over its containers (a
// contiguous block of per_row) and the 256 model cells of max(0, 2^y - 1).
__global__ void __launch_bounds__(kSelThreads) k_seed_rowsize(const float *y, int per_row, double *out) {
  __shared__ double shd[2 * kSelThreads];
  const long n = (long)per_row * kMlpOut, base = (long)blockIdx.x * n;
  double a = 0.0;
  for (long i = threadIdx.x; i < n; i += blockDim.x) {
    const double v = exp2((double)y[base + i]) - 1.0;
    a += v > 0.0 ? v : 0.0;
  }
  const double tot = block_sum(a, shd);
  if (threadIdx.x == 0) out[blockIdx.x] = tot;
}

hipError_t launch_seed_rowsize(const float *y, int n_rows, int per_row, double *out, hipStream_t s) {
  if (n_rows == 0) return hipSuccess;
  hipLaunchKernelGGL(k_seed_rowsize, dim3(n_rows), dim3(kSelThreads), 0, s, y, per_row, out);
  return hipGetLastError();
}

hipError_t launch_admit(const Problem &p, hipStream_t s) {
  hipLaunchKernelGGL(k_admit, dim3(1), dim3(1024), 0, s, p);
  return hipGetLastError();
}
hipError_t launch_select(const Problem &p, hipStream_t s) {
  hipLaunchKernelGGL(k_select, dim3(p.W), dim3(kSelThreads), 0, s, p);
  return hipGetLastError();
}
hipError_t launch_worklist(const Problem &p, hipStream_t s) {
  hipLaunchKernelGGL(k_worklist, dim3(1), dim3(1024), 0, s, p);
  return hipGetLastError();
}
hipError_t launch_update(const Problem &p, hipStream_t s) {
  hipLaunchKernelGGL(k_update_part, dim3(p.W, kUpdChunks), dim3(kSelThreads), 0, s, p);
  hipLaunchKernelGGL(k_update, dim3(p.W), dim3(64), 0, s, p);
  return hipGetLastError();
}

size_t update_scratch_doubles(int W, int MU) { return (size_t)W * kUpdChunks * (2 * (size_t)MU + 2); }
hipError_t launch_finalize(const Problem &p, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(p.W), dim3(kSelThreads), 0, s, p);
  return hipGetLastError();
}

}  // namespace paid
