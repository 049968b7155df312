/*
 * paid_oracle.c -- plain FP64 CPU oracle (test infrastructure only; see
 * paid_oracle.h).  Serial per problem, no blocking or fusion: each function
 * is the definition it cites, written out.
 *
 * Readings of the paper that this file commits to:
 *  - finite temperature: the frequency integral of Eqs. chi_pp / chi_ph is a
 *    Matsubara sum T sum_n over w_n = (2n+1) pi T, which becomes the
 *    continuous integral as T -> 0;
 *  - measure d^2p/(2pi)^2 over the zone [-pi,pi)^2 (so the integral of 1 is 1);
 *  - the "dot" is d/dOmega of the whole product of the two regulated
 *    propagators, i.e. of theta(w)^2 (Sec. 2);
 *  - the rule order N counts intervals per axis: the coarse 2-D rule has
 *    (N+1)^2 nodes and they are a subset of the (2N+1)^2 nodes of the fine
 *    rule (Sec. 3, n2 = 2 n1 with node reuse);
 *  - a region is split once in each dimension at its midpoints, children in
 *    the order (x-lo,y-lo), (x-hi,y-lo), (x-lo,y-hi), (x-hi,y-hi) (Alg. 2);
 *  - ties of the priority key are broken by creation order.
 */
#include "paid_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define PO_PI 3.14159265358979323846264338327950288
#define PO_KTAIL 24     /* terms of the large-frequency expansion of the tail */

/* ------------------------------------------------------------------------ */
/* Clenshaw-Curtis rule (Sec. 3; the weights are the classical closed form
 * w_k = c_k/n [1 - sum_{j=1}^{n/2} b_j cos(2 j k pi/n)/(4j^2-1)],
 * c_0 = c_n = 1, c_k = 2 otherwise, b_{n/2} = 1, b_j = 2 otherwise).        */
int po_cc_rule(int n, double *x, double *w) {
  if (n < 1) return -1;
  for (int k = 0; k <= n; ++k) {
    /* cos(k pi / n), written as a sine so that the middle node is exactly 0,
       the rule is exactly antisymmetric, and the n-rule nodes are bitwise
       equal to the even nodes of the 2n-rule. */
    x[k] = sin(PO_PI * (double)(n - 2 * k) / (2.0 * n));
    double th = k * PO_PI / n, s = 0.0;
    for (int j = 1; 2 * j <= n; ++j) {
      double b = (2 * j == n) ? 1.0 : 2.0;
      s += b * cos(2.0 * j * th) / (4.0 * j * j - 1.0);
    }
    double c = (k == 0 || k == n) ? 1.0 : 2.0;
    w[k] = c / n * (1.0 - s);
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Hurwitz zeta by Euler-Maclaurin summation after shifting q upwards.       */
double po_hurwitz_zeta(double s, double q) {
  static const double B2[12] = {1.0 / 6,         -1.0 / 30,          1.0 / 42,
                                -1.0 / 30,       5.0 / 66,           -691.0 / 2730,
                                7.0 / 6,         -3617.0 / 510,      43867.0 / 798,
                                -174611.0 / 330, 854513.0 / 138,     -236364091.0 / 2730};
  double need = fmax(24.0, s + 20.0);
  int J = (q < need) ? (int)ceil(need - q) : 0;
  double sum = 0.0;
  for (int j = J - 1; j >= 0; --j) sum += pow(q + j, -s); /* small terms first */
  double Q = q + J, Qs = pow(Q, -s);
  double tail = Q * Qs / (s - 1.0) + 0.5 * Qs;
  double fact = 1.0, rising = s, Qp = Qs / Q;
  for (int i = 1; i <= 12; ++i) {
    fact *= (2.0 * i - 1.0) * (2.0 * i);
    tail += B2[i - 1] / fact * rising * Qp;
    rising *= (s + 2.0 * i - 1.0) * (s + 2.0 * i);
    Qp /= Q * Q;
  }
  return sum + tail;
}

/* ------------------------------------------------------------------------ */
/* Dispersion of the t-t' square lattice (Sec. 2).                          */
double po_dispersion(double t, double tp, double mu, double kx, double ky) {
  double cx = cos(kx), cy = cos(ky);
  return -2.0 * t * (cx + cy) - 4.0 * tp * cx * cy - mu;
}

double po_fermi(double e, double T) {
  if (e > 0) {
    double x = exp(-e / T);
    return x / (1.0 + x);
  }
  return 1.0 / (1.0 + exp(e / T));
}

/* ------------------------------------------------------------------------ */
/* Frequency sums.
 *
 * With u = w^2, the regulated product at Matsubara frequency w_n is, after
 * pairing w_n with -w_n (the imaginary parts cancel),
 *   ph:  G(w,a) G(w,b)   -> (a b - u) / ((u + a^2)(u + b^2))
 *   pp:  G(w,a) G(-w,b)  -> (u + a b) / ((u + a^2)(u + b^2))
 * times theta(w)^2 = u^2/(u+Omega^2)^2 (kind BUBBLE) or its Omega-derivative
 * d/dOmega theta^2 = -4 Omega u^2/(u+Omega^2)^3 (kind BUBBLE_DOT), and
 *   K = 2 T sum_{n >= 0} (...).
 * The first N terms are summed directly; the rest is expanded in v = 1/u
 * (convergent because u_N exceeds Omega^2, a^2, b^2 by a factor >= 16) and
 * summed with sum_{n>=N} u_n^-k = (2 pi T)^-2k zeta(2k, N + 1/2).            */
typedef struct {
  int kind, N;
  double T, Omega;
  double *u, *W;                 /* u_n and the regulator factor at u_n */
  double Z[PO_KTAIL + 1];        /* sum_{n>=N} u_n^-k */
} po_msum;

static double po_regulator(int kind, double u, double Om) {
  double d = u + Om * Om;
  if (kind == PO_BUBBLE_DOT) return -4.0 * Om * u * u / (d * d * d);
  return u * u / (d * d);
}

static int po_msum_init(po_msum *m, int kind, double Omega, double T, double emax) {
  double big = fmax(fmax(fabs(Omega), emax), PO_PI * T);
  /* w_N = (2N+1) pi T >= 4 big */
  int N = (int)ceil((4.0 * big / (PO_PI * T) - 1.0) / 2.0);
  if (N < 8) N = 8;
  m->kind = kind;
  m->N = N;
  m->T = T;
  m->Omega = Omega;
  m->u = (double *)malloc(sizeof(double) * N);
  m->W = (double *)malloc(sizeof(double) * N);
  if (!m->u || !m->W) return -1;
  for (int n = 0; n < N; ++n) {
    double w = (2.0 * n + 1.0) * PO_PI * T;
    m->u[n] = w * w;
    m->W[n] = po_regulator(kind, m->u[n], Omega);
  }
  double s2 = 2.0 * PO_PI * T;
  m->Z[0] = 0.0;
  for (int k = 1; k <= PO_KTAIL; ++k)
    m->Z[k] = pow(s2, -2.0 * k) * po_hurwitz_zeta(2.0 * k, N + 0.5);
  return 0;
}

static void po_msum_free(po_msum *m) {
  free(m->u);
  free(m->W);
  m->u = m->W = NULL;
}

/* multiply the power series c (in v) by 1/(1 + alpha v) in place */
static void po_series_div1(double *c, int K, double alpha) {
  for (int k = 1; k <= K; ++k) c[k] -= alpha * c[k - 1];
}

static double po_msum_eval(const po_msum *m, int channel, double a, double b) {
  const double a2 = a * a, b2 = b * b, ab = a * b;
  const double sg = (channel == PO_PH) ? -1.0 : 1.0; /* P(u) = ab + sg*u */
  double head = 0.0;
  for (int n = 0; n < m->N; ++n) {
    double u = m->u[n];
    head += m->W[n] * (ab + sg * u) / ((u + a2) * (u + b2));
  }
  /* tail: P(u)/((u+a^2)(u+b^2)) = v (sg + ab v) / ((1+a^2 v)(1+b^2 v)) */
  double c[PO_KTAIL + 1];
  memset(c, 0, sizeof c);
  c[1] = sg;
  c[2] = ab;
  po_series_div1(c, PO_KTAIL, a2);
  po_series_div1(c, PO_KTAIL, b2);
  const double O2 = m->Omega * m->Omega;
  if (m->kind == PO_BUBBLE_DOT) {
    /* -4 Omega v (1 + Omega^2 v)^-3 */
    for (int r = 0; r < 3; ++r) po_series_div1(c, PO_KTAIL, O2);
    for (int k = PO_KTAIL; k >= 1; --k) c[k] = -4.0 * m->Omega * c[k - 1];
    c[0] = 0.0;
  } else {
    /* (1 + Omega^2 v)^-2 */
    for (int r = 0; r < 2; ++r) po_series_div1(c, PO_KTAIL, O2);
  }
  double tail = 0.0;
  for (int k = PO_KTAIL; k >= 1; --k) tail += c[k] * m->Z[k];
  return 2.0 * m->T * (head + tail);
}

double po_kernel(int kind, int channel, double a, double b, double Omega, double T) {
  if (kind == PO_UNIT) return 1.0;
  if (!(T > 0) || (kind != PO_BUBBLE_DOT && kind != PO_BUBBLE)) return NAN;
  po_msum m;
  if (po_msum_init(&m, kind, Omega, T, fmax(fabs(a), fabs(b))) != 0) return NAN;
  double r = po_msum_eval(&m, channel, a, b);
  po_msum_free(&m);
  return r;
}

/* ------------------------------------------------------------------------ */
/* Box basis u_0 = 1, u_{2k-1} = sqrt2 cos(k x), u_{2k} = sqrt2 sin(k x),
 * k = 1..L; a form factor is f(p) = sum_{alpha,beta} C[alpha(2L+1)+beta]
 * u_alpha(p_x) u_beta(p_y) (orthonormal lattice harmonics, Sec. 2).         */
void po_box_basis(int L, double x, double *u) {
  u[0] = 1.0;
  for (int k = 1; k <= L; ++k) {
    u[2 * k - 1] = sqrt(2.0) * cos(k * x);
    u[2 * k] = sqrt(2.0) * sin(k * x);
  }
}

static void po_form_factors(const po_problem *pr, double px, double py, double *f) {
  int nb = 2 * pr->ff_L + 1;
  double ux[64], uy[64];
  po_box_basis(pr->ff_L, px, ux);
  po_box_basis(pr->ff_L, py, uy);
  for (int m = 0; m < pr->n_ff; ++m) {
    const double *C = pr->ff + (long)m * nb * nb;
    double s = 0.0;
    for (int al = 0; al < nb; ++al)
      for (int be = 0; be < nb; ++be) s += C[al * nb + be] * ux[al] * uy[be];
    f[m] = s;
  }
}

static double po_emax(const po_problem *pr) {
  return 4.0 * fabs(pr->t) + 4.0 * fabs(pr->tp) + fabs(pr->mu);
}

/* g(p): a = eps(l/2 + p), b = eps(l/2 - p) for both channels (eps is even) */
static double po_integrand_m(const po_problem *pr, const po_msum *m, double px, double py) {
  switch (pr->kind) {
    case PO_UNIT:
      return 1.0;
    case PO_GAUSS: {
      double dx = px - pr->gx, dy = py - pr->gy;
      return exp(-(dx * dx + dy * dy) / (2.0 * pr->gsigma * pr->gsigma));
    }
    default: {
      double a = po_dispersion(pr->t, pr->tp, pr->mu, 0.5 * pr->lx + px, 0.5 * pr->ly + py);
      double b = po_dispersion(pr->t, pr->tp, pr->mu, 0.5 * pr->lx - px, 0.5 * pr->ly - py);
      return po_msum_eval(m, pr->channel, a, b);
    }
  }
}

static int po_problem_msum(const po_problem *pr, po_msum *m) {
  memset(m, 0, sizeof *m);
  if (pr->kind != PO_BUBBLE_DOT && pr->kind != PO_BUBBLE) return 0;
  return po_msum_init(m, pr->kind, pr->Omega, pr->T, po_emax(pr));
}

double po_integrand(const po_problem *pr, double px, double py) {
  po_msum m;
  if (po_problem_msum(pr, &m) != 0) return NAN;
  double g = po_integrand_m(pr, &m, px, py);
  po_msum_free(&m);
  return g;
}

/* ------------------------------------------------------------------------ */
/* One rectangle, tensor-product CC pair (Sec. 3).                           */
typedef struct {
  const po_problem *pr;
  po_msum ms;
  int N, M, MU;
  double x1[65], w1[65];   /* N-rule  */
  double x2[129], w2[129]; /* 2N-rule */
  double *f;               /* scratch [M] */
  long kernel_evals;
} po_ctx;

static int po_ctx_init(po_ctx *c, const po_problem *pr, int N) {
  memset(c, 0, sizeof *c);
  if (N < 1 || N > 64 || pr->n_ff < 1 || pr->ff_L < 0 || pr->ff_L > 31) return -1;
  if ((pr->kind == PO_BUBBLE_DOT || pr->kind == PO_BUBBLE) && !(pr->T > 0)) return -1;
  c->pr = pr;
  c->N = N;
  c->M = pr->n_ff;
  c->MU = c->M * (c->M + 1) / 2;
  po_cc_rule(N, c->x1, c->w1);
  po_cc_rule(2 * N, c->x2, c->w2);
  c->f = (double *)malloc(sizeof(double) * c->M);
  if (!c->f) return -1;
  return po_problem_msum(pr, &c->ms);
}

static void po_ctx_free(po_ctx *c) {
  free(c->f);
  po_msum_free(&c->ms);
}

/* all pairs (pair < 0) or one pair index; qn/q2n hold MU (or 1) values */
static void po_rect(po_ctx *c, double x0, double x1, double y0, double y1, int pair,
                    double *qn, double *q2n) {
  const int N = c->N, M = c->M, n2 = 2 * N + 1;
  const int np = (pair < 0) ? c->MU : 1;
  int pp = 0, pq = 0;
  if (pair >= 0) { /* decode the upper-triangle index */
    int k = pair;
    while (k >= M - pp) { k -= M - pp; ++pp; }
    pq = pp + k;
  }
  for (int k = 0; k < np; ++k) qn[k] = q2n[k] = 0.0;
  const double cx = 0.5 * (x0 + x1), hx = 0.5 * (x1 - x0);
  const double cy = 0.5 * (y0 + y1), hy = 0.5 * (y1 - y0);
  for (int i = 0; i < n2; ++i) {
    double px = cx + hx * c->x2[i];
    for (int j = 0; j < n2; ++j) {
      double py = cy + hy * c->x2[j];
      double g = po_integrand_m(c->pr, &c->ms, px, py);
      c->kernel_evals++;
      po_form_factors(c->pr, px, py, c->f);
      double W2 = hx * hy * c->w2[i] * c->w2[j] * g;
      int coarse = (i % 2 == 0) && (j % 2 == 0);
      double WN = coarse ? hx * hy * c->w1[i / 2] * c->w1[j / 2] * g : 0.0;
      if (pair >= 0) {
        double ff = c->f[pp] * c->f[pq];
        q2n[0] += W2 * ff;
        qn[0] += WN * ff;
      } else {
        int idx = 0;
        for (int p = 0; p < M; ++p)
          for (int q = p; q < M; ++q, ++idx) {
            double ff = c->f[p] * c->f[q];
            q2n[idx] += W2 * ff;
            qn[idx] += WN * ff;
          }
      }
    }
  }
  const double norm = 1.0 / (4.0 * PO_PI * PO_PI);
  for (int k = 0; k < np; ++k) {
    qn[k] *= norm;
    q2n[k] *= norm;
  }
}

int po_region_eval(const po_problem *pr, int N, double x0, double x1, double y0, double y1,
                   double *qn, double *q2n) {
  po_ctx c;
  if (po_ctx_init(&c, pr, N) != 0) {
    po_ctx_free(&c);
    return -1;
  }
  po_rect(&c, x0, x1, y0, y1, -1, qn, q2n);
  po_ctx_free(&c);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Task container: a binary max-heap on the error key (Sec. 4, Listing 1),   */
/* ties broken by creation order.                                            */
typedef struct {
  double key;
  long id; /* creation index == index into the task store */
} po_hent;

typedef struct {
  po_hent *a;
  long n, cap;
} po_heap;

static int po_hless(const po_hent *x, const po_hent *y) { /* x below y? */
  if (x->key != y->key) return x->key < y->key;
  return x->id > y->id;
}

static int po_heap_push(po_heap *h, double key, long id) {
  if (h->n == h->cap) {
    long nc = h->cap ? 2 * h->cap : 1024;
    po_hent *na = (po_hent *)realloc(h->a, sizeof(po_hent) * nc);
    if (!na) return -1;
    h->a = na;
    h->cap = nc;
  }
  long i = h->n++;
  h->a[i].key = key;
  h->a[i].id = id;
  while (i > 0) {
    long p = (i - 1) / 2;
    if (!po_hless(&h->a[p], &h->a[i])) break;
    po_hent t = h->a[p];
    h->a[p] = h->a[i];
    h->a[i] = t;
    i = p;
  }
  return 0;
}

static po_hent po_heap_pop(po_heap *h) {
  po_hent top = h->a[0];
  h->a[0] = h->a[--h->n];
  long i = 0;
  for (;;) {
    long l = 2 * i + 1, r = l + 1, m = i;
    if (l < h->n && po_hless(&h->a[m], &h->a[l])) m = l;
    if (r < h->n && po_hless(&h->a[m], &h->a[r])) m = r;
    if (m == i) break;
    po_hent t = h->a[m];
    h->a[m] = h->a[i];
    h->a[i] = t;
    i = m;
  }
  return top;
}

/* task store: geometry, pair, Q_2N and err per pair (np values each) */
typedef struct {
  long n, cap;
  int np;
  double *geo; /* x0,x1,y0,y1 */
  int *depth, *pair;
  double *q2n, *err;
  char *leaf;
} po_store;

static int po_store_grow(po_store *s, long need) {
  if (need <= s->cap) return 0;
  long nc = s->cap ? s->cap : 1024;
  while (nc < need) nc *= 2;
  double *g = (double *)realloc(s->geo, sizeof(double) * 4 * nc);
  if (!g) return -1;
  s->geo = g;
  int *d = (int *)realloc(s->depth, sizeof(int) * nc);
  if (!d) return -1;
  s->depth = d;
  int *p = (int *)realloc(s->pair, sizeof(int) * nc);
  if (!p) return -1;
  s->pair = p;
  double *q = (double *)realloc(s->q2n, sizeof(double) * s->np * nc);
  if (!q) return -1;
  s->q2n = q;
  double *e = (double *)realloc(s->err, sizeof(double) * s->np * nc);
  if (!e) return -1;
  s->err = e;
  char *l = (char *)realloc(s->leaf, nc);
  if (!l) return -1;
  s->leaf = l;
  s->cap = nc;
  return 0;
}

static void po_store_free(po_store *s) {
  free(s->geo);
  free(s->depth);
  free(s->pair);
  free(s->q2n);
  free(s->err);
  free(s->leaf);
}

/* tolerance per pair from the current values (Sec. 3 global criterion read
 * as relative to the values; the per-integral variant floors small entries
 * at nu times the largest one). */
static void po_tolerances(const po_options *o, int MU, const double *val, const double *w,
                          double *tau, double *eps_global) {
  double vmax = 0.0, l1 = 0.0;
  for (int k = 0; k < MU; ++k) {
    vmax = fmax(vmax, fabs(val[k]));
    l1 += (o->err_mode == PO_ERR_WEIGHTED ? w[k] : 1.0) * fabs(val[k]);
  }
  for (int k = 0; k < MU; ++k)
    tau[k] = fmax(o->atol, o->rtol * fmax(fabs(val[k]), o->nu * vmax));
  *eps_global = fmax(o->atol, o->rtol * l1);
}

/* Global criterion (Sec. 3): sum over pairs of the error against eps; with
 * pair weights (Eq. P_globerr: the error of the contracted matrix is
 * bounded by the couplings times the pair errors) the sum is weighted. */
static int po_converged(const po_options *o, int MU, const double *ERR, const double *w,
                        const double *tau, double eps_global) {
  if (o->err_mode == PO_ERR_GLOBAL || o->err_mode == PO_ERR_WEIGHTED) {
    double s = 0.0;
    for (int k = 0; k < MU; ++k) s += (o->err_mode == PO_ERR_WEIGHTED ? w[k] : 1.0) * ERR[k];
    return s <= eps_global;
  }
  for (int k = 0; k < MU; ++k)
    if (ERR[k] > tau[k]) return 0;
  return 1;
}

static void po_split_geo(const double *g, int a, double *c) {
  double xm = 0.5 * (g[0] + g[1]), ym = 0.5 * (g[2] + g[3]);
  c[0] = (a & 1) ? xm : g[0];
  c[1] = (a & 1) ? g[1] : xm;
  c[2] = (a & 2) ? ym : g[2];
  c[3] = (a & 2) ? g[3] : ym;
}

/* recompute per-pair value and ERR from the current leaves (guards against
 * drift of the incrementally updated sums before accepting convergence) */
static void po_resum(const po_store *s, int mode, int MU, double *val, double *ERR) {
  for (int k = 0; k < MU; ++k) val[k] = ERR[k] = 0.0;
  for (long i = 0; i < s->n; ++i) {
    if (!s->leaf[i]) continue;
    if (mode == PO_MODE_B) {
      for (int k = 0; k < MU; ++k) {
        val[k] += s->q2n[i * MU + k];
        ERR[k] += s->err[i * MU + k];
      }
    } else {
      val[s->pair[i]] += s->q2n[i];
      ERR[s->pair[i]] += s->err[i];
    }
  }
}

static double po_key(const po_options *o, int np, int pair, const double *err,
                     const double *inv_tau) {
  double k = 0.0;
  for (int j = 0; j < np; ++j) {
    int pj = (pair < 0) ? j : pair;
    k += (o->err_mode == PO_ERR_GLOBAL) ? err[j] : err[j] * inv_tau[pj];  /* 1/tau or w */
  }
  return k;
}

/* leaves of the final tree (mode B): rectangles and Q_2N per pair, in
   creation order, at most cap of them; *n receives the leaf count */
typedef struct {
  double *rects, *q2n;
  long cap, *n;
} po_leaf_out;

static int po_integrate_impl(const po_problem *pr, const po_options *o, double *value,
                             double *errout, po_stats *st, double *labels,
                             const po_leaf_out *lo);

int po_integrate(const po_problem *pr, const po_options *o, double *value, double *errout,
                 po_stats *st) {
  return po_integrate_impl(pr, o, value, errout, st, NULL, NULL);
}

int po_integrate_labels(const po_problem *pr, const po_options *o, double *value, double *err,
                        po_stats *st, double labels[256]) {
  if (!labels || !o || o->mode != PO_MODE_B) return -2;
  return po_integrate_impl(pr, o, value, err, st, labels, NULL);
}

int po_integrate_leaves(const po_problem *pr, const po_options *o, double *value, double *err,
                        po_stats *st, double *rects, double *q2n, long cap, long *n_leaves) {
  if (!o || o->mode != PO_MODE_B || !n_leaves || cap < 0) return -2;
  po_leaf_out lo = {rects, q2n, cap, n_leaves};
  return po_integrate_impl(pr, o, value, err, st, NULL, &lo);
}

static int po_integrate_impl(const po_problem *pr, const po_options *o, double *value,
                             double *errout, po_stats *st, double *labels,
                             const po_leaf_out *lo) {
  if (!pr || !o || !value || o->batch < 1 || !(o->rtol >= 0) || !(o->atol >= 0) ||
      (o->rtol <= 0 && o->atol <= 0) || o->max_regions < 1)
    return -2;
  po_ctx c;
  if (po_ctx_init(&c, pr, o->N) != 0) {
    po_ctx_free(&c);
    return -2;
  }
  const int M = c.M, MU = c.MU, modeB = (o->mode == PO_MODE_B);
  po_store s;
  memset(&s, 0, sizeof s);
  s.np = modeB ? MU : 1;
  po_heap h = {0, 0, 0};
  double *val = (double *)calloc(MU, sizeof(double));
  double *ERR = (double *)calloc(MU, sizeof(double));
  double *tau = (double *)calloc(MU, sizeof(double));
  double *itau = (double *)calloc(MU, sizeof(double));
  double *pw = (double *)calloc(MU, sizeof(double)); /* pair weights (weighted mode) */
  double *qn = (double *)calloc(MU, sizeof(double));
  long *pick = (long *)calloc(o->batch, sizeof(long));
  po_stats S;
  memset(&S, 0, sizeof S);
  int rc = -3;
  if (!val || !ERR || !tau || !itau || !pw || !qn || !pick) goto done;
  if (o->err_mode == PO_ERR_WEIGHTED) {
    if (!pr->pair_w) goto done;
    int k = 0;
    for (int p = 0; p < M; ++p)
      for (int q = p; q < M; ++q, ++k)
        pw[k] = (p == q) ? pr->pair_w[p * M + p] : pr->pair_w[p * M + q] + pr->pair_w[q * M + p];
  }

  /* Listing 1: root task(s) on the whole zone */
  {
    const double root[4] = {-PO_PI, PO_PI, -PO_PI, PO_PI};
    int nroot = modeB ? 1 : MU;
    if (po_store_grow(&s, nroot) != 0) goto done;
    for (int r = 0; r < nroot; ++r) {
      long id = s.n++;
      memcpy(&s.geo[4 * id], root, sizeof root);
      s.depth[id] = 0;
      s.pair[id] = modeB ? -1 : r;
      s.leaf[id] = 1;
      po_rect(&c, root[0], root[1], root[2], root[3], s.pair[id], qn, &s.q2n[id * s.np]);
      for (int k = 0; k < s.np; ++k) s.err[id * s.np + k] = fabs(qn[k] - s.q2n[id * s.np + k]);
    }
    po_resum(&s, o->mode, MU, val, ERR);
    double eg;
    po_tolerances(o, MU, val, pw, tau, &eg);
    for (int k = 0; k < MU; ++k) itau[k] = (o->err_mode == PO_ERR_WEIGHTED) ? pw[k] : 1.0 / tau[k];
    for (long id = 0; id < s.n; ++id)
      if (po_heap_push(&h, po_key(o, s.np, s.pair[id], &s.err[id * s.np], itau), id) != 0)
        goto done;
  }

  for (;;) {
    /* termination test (master thread in Listing 5), with an exact re-sum
       from the leaves before it is accepted */
    double eg;
    po_tolerances(o, MU, val, pw, tau, &eg);
    if (po_converged(o, MU, ERR, pw, tau, eg)) {
      po_resum(&s, o->mode, MU, val, ERR);
      po_tolerances(o, MU, val, pw, tau, &eg);
      if (po_converged(o, MU, ERR, pw, tau, eg)) {
        S.converged = 1;
        break;
      }
    }
    if (h.n == 0) break;
    long leaves = h.n;
    if (leaves + 3 > o->max_regions) break;
    if (o->err_mode == PO_ERR_PER_INTEGRAL)
      for (int k = 0; k < MU; ++k) itau[k] = 1.0 / tau[k];
    /* Listing 2: extract up to MaxTask tasks of largest error */
    int nb = 0;
    while (nb < o->batch && h.n > 0 && leaves + 3 * (nb + 1) <= o->max_regions)
      pick[nb++] = po_heap_pop(&h).id;
    if (po_store_grow(&s, s.n + 4L * nb) != 0) goto done;
    /* Listing 3: divide into 4 and evaluate; Listing 4: update and insert */
    for (int b = 0; b < nb; ++b) {
      long pid = pick[b];
      s.leaf[pid] = 0;
      for (int a = 0; a < 4; ++a) {
        long id = s.n++;
        po_split_geo(&s.geo[4 * pid], a, &s.geo[4 * id]);
        s.depth[id] = s.depth[pid] + 1;
        s.pair[id] = s.pair[pid];
        s.leaf[id] = 1;
        double *g = &s.geo[4 * id];
        po_rect(&c, g[0], g[1], g[2], g[3], s.pair[id], qn, &s.q2n[id * s.np]);
        for (int k = 0; k < s.np; ++k) s.err[id * s.np + k] = fabs(qn[k] - s.q2n[id * s.np + k]);
        if (s.depth[id] > S.max_depth) S.max_depth = s.depth[id];
      }
      for (int a = 0; a < 4; ++a) {
        long id = s.n - 4 + a;
        if (po_heap_push(&h, po_key(o, s.np, s.pair[id], &s.err[id * s.np], itau), id) != 0)
          goto done;
      }
      /* ERR -= parent, += children; value likewise */
      for (int k = 0; k < s.np; ++k) {
        int pk = modeB ? k : s.pair[pid];
        double dv = -s.q2n[pid * s.np + k], de = -s.err[pid * s.np + k];
        for (int a = 0; a < 4; ++a) {
          long id = s.n - 4 + a;
          dv += s.q2n[id * s.np + k];
          de += s.err[id * s.np + k];
        }
        val[pk] += dv;
        ERR[pk] += de;
      }
      S.splits++;
    }
    S.rounds++;
  }
  po_resum(&s, o->mode, MU, val, ERR);
  {
    int idx = 0;
    for (int p = 0; p < M; ++p)
      for (int q = p; q < M; ++q, ++idx) {
        value[p * M + q] = value[q * M + p] = val[idx];
        if (errout) errout[p * M + q] = errout[q * M + p] = ERR[idx];
      }
  }
  S.regions = h.n;
  S.kernel_evals = c.kernel_evals;
  if (labels) {
    long nl = 0;
    double *rl = (double *)malloc(sizeof(double) * 4 * (s.n > 0 ? s.n : 1));
    if (!rl) goto done;
    for (long i = 0; i < s.n; ++i)
      if (s.leaf[i]) memcpy(&rl[4 * nl++], &s.geo[4 * i], 4 * sizeof(double));
    po_tree_labels(rl, nl, labels);
    free(rl);
  }
  if (lo) {
    long nl = 0;
    for (long i = 0; i < s.n; ++i) {
      if (!s.leaf[i]) continue;
      if (nl < lo->cap) {
        if (lo->rects) memcpy(&lo->rects[4 * nl], &s.geo[4 * i], 4 * sizeof(double));
        if (lo->q2n) memcpy(&lo->q2n[nl * MU], &s.q2n[i * MU], MU * sizeof(double));
      }
      ++nl;
    }
    *lo->n = nl;
  }
  rc = S.converged ? 0 : 1;
done:
  if (st) *st = S;
  free(val);
  free(ERR);
  free(tau);
  free(itau);
  free(pw);
  free(qn);
  free(pick);
  free(h.a);
  po_store_free(&s);
  po_ctx_free(&c);
  return rc;
}

int po_integrate_batch(const po_problem *prs, int n, const po_options *o, double *values,
                       double *errs, po_stats *sts, int nthreads) {
  if (n < 0) return -2;
  int bad = 0, notconv = 0;
  if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) reduction(+ : bad, notconv)
  for (int i = 0; i < n; ++i) {
    long MM = (long)prs[i].n_ff * prs[i].n_ff;
    int r = po_integrate(&prs[i], o, values + (long)i * MM, errs ? errs + (long)i * MM : NULL,
                         sts ? &sts[i] : NULL);
    if (r < 0) bad++;
    if (r == 1) notconv++;
  }
  return bad ? -2 : notconv;
}

/* ------------------------------------------------------------------------ */
/* Brute force: periodic trapezoid rule on an L x L grid.                    */
int po_brute(const po_problem *pr, int L, double *value) {
  if (L < 1 || pr->n_ff < 1) return -2;
  po_msum m;
  if (po_problem_msum(pr, &m) != 0) return -3;
  const int M = pr->n_ff;
  double *f = (double *)malloc(sizeof(double) * M);
  double *acc = (double *)calloc((size_t)M * M, sizeof(double));
  if (!f || !acc) {
    free(f);
    free(acc);
    po_msum_free(&m);
    return -3;
  }
  const double h = 2.0 * PO_PI / L;
  for (int i = 0; i < L; ++i) {
    double px = -PO_PI + (i + 0.5) * h;
    for (int j = 0; j < L; ++j) {
      double py = -PO_PI + (j + 0.5) * h;
      double g = po_integrand_m(pr, &m, px, py);
      po_form_factors(pr, px, py, f);
      for (int p = 0; p < M; ++p)
        for (int q = p; q < M; ++q) acc[p * M + q] += g * f[p] * f[q];
    }
  }
  for (int p = 0; p < M; ++p)
    for (int q = p; q < M; ++q) value[p * M + q] = value[q * M + p] = acc[p * M + q] / ((double)L * L);
  free(f);
  free(acc);
  po_msum_free(&m);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Subdivision-density model: plain FP64 multilayer perceptron.              */
static const int po_dims[5] = {PO_MLP_IN, PO_MLP_HID, PO_MLP_HID, PO_MLP_HID, PO_MLP_OUT};

long po_mlp_nparams(void) {
  long n = 0;
  for (int l = 0; l < 4; ++l) n += (long)po_dims[l + 1] * po_dims[l] + po_dims[l + 1];
  return n;
}

static double po_gelu(double z) { return 0.5 * z * (1.0 + erf(z / sqrt(2.0))); }
static double po_gelu_d(double z) {
  return 0.5 * (1.0 + erf(z / sqrt(2.0))) + z * exp(-0.5 * z * z) / sqrt(2.0 * PO_PI);
}

/* pre-activations z[l] and activations a[l] of one sample, l = 0..4 (a[0] = x) */
static void po_mlp_sample(const double *w, const double *x, double a[5][PO_MLP_OUT],
                          double z[5][PO_MLP_OUT]) {
  for (int i = 0; i < PO_MLP_IN; ++i) a[0][i] = x[i];
  const double *p = w;
  for (int l = 0; l < 4; ++l) {
    int ni = po_dims[l], no = po_dims[l + 1];
    const double *W = p, *b = p + (long)no * ni;
    for (int o = 0; o < no; ++o) {
      double s = b[o];
      for (int i = 0; i < ni; ++i) s += W[(long)o * ni + i] * a[l][i];
      z[l + 1][o] = s;
      a[l + 1][o] = (l < 3) ? po_gelu(s) : s;
    }
    p += (long)no * ni + no;
  }
}

void po_mlp_forward(const double *w, const double *x, int n, double *yhat) {
  double a[5][PO_MLP_OUT], z[5][PO_MLP_OUT];
  for (int s = 0; s < n; ++s) {
    po_mlp_sample(w, x + (long)s * PO_MLP_IN, a, z);
    for (int o = 0; o < PO_MLP_OUT; ++o) yhat[(long)s * PO_MLP_OUT + o] = a[4][o];
  }
}

double po_mlp_loss_grad(const double *w, const double *x, const double *y, int n, double *grad) {
  long np = po_mlp_nparams();
  for (long k = 0; k < np; ++k) grad[k] = 0.0;
  long off[4];
  off[0] = 0;
  for (int l = 1; l < 4; ++l) off[l] = off[l - 1] + (long)po_dims[l] * po_dims[l - 1] + po_dims[l];
  double loss = 0.0, a[5][PO_MLP_OUT], z[5][PO_MLP_OUT], d[PO_MLP_OUT], dn[PO_MLP_OUT];
  const double scale = 1.0 / ((double)n * PO_MLP_OUT);
  for (int s = 0; s < n; ++s) {
    po_mlp_sample(w, x + (long)s * PO_MLP_IN, a, z);
    for (int o = 0; o < PO_MLP_OUT; ++o) {
      double r = a[4][o] - y[(long)s * PO_MLP_OUT + o];
      loss += r * r;
      d[o] = 2.0 * r * scale;  /* dL/dz of the linear output layer */
    }
    for (int l = 3; l >= 0; --l) {  /* layer l maps a[l] -> z[l+1] */
      int ni = po_dims[l], no = po_dims[l + 1];
      const double *W = w + off[l];
      double *gW = grad + off[l], *gb = grad + off[l] + (long)no * ni;
      for (int o = 0; o < no; ++o) {
        gb[o] += d[o];
        for (int i = 0; i < ni; ++i) gW[(long)o * ni + i] += d[o] * a[l][i];
      }
      if (l > 0) {
        for (int i = 0; i < ni; ++i) {
          double s2 = 0.0;
          for (int o = 0; o < no; ++o) s2 += W[(long)o * ni + i] * d[o];
          dn[i] = s2 * po_gelu_d(z[l][i]);
        }
        for (int i = 0; i < ni; ++i) d[i] = dn[i];
      }
    }
  }
  return loss * scale;
}

void po_mlp_adam(double *w, const double *g, double *m, double *v, long np, int t, double lr) {
  const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
  const double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
  for (long k = 0; k < np; ++k) {
    m[k] = b1 * m[k] + (1.0 - b1) * g[k];
    v[k] = b2 * v[k] + (1.0 - b2) * g[k] * g[k];
    w[k] -= lr * (m[k] / c1) / (sqrt(v[k] / c2) + eps);
  }
}

/* ------------------------------------------------------------------------ */
/* Seeding: features, labels, seed tree.                                     */
void po_seed_features(double t, double tp, double mu, double T, double Omega, double lx,
                      double ly, int channel, double x[7], int cellmap[256]) {
  /* reduce l to [-pi, pi)^2; an odd number of 2 pi shifts moves p by pi */
  double nx = floor((lx + PO_PI) / (2.0 * PO_PI)), ny = floor((ly + PO_PI) / (2.0 * PO_PI));
  double rx = lx - 2.0 * PO_PI * nx, ry = ly - 2.0 * PO_PI * ny;
  int hx = ((long)nx) & 1, hy = ((long)ny) & 1;
  /* D4 element taking (rx, ry) to the wedge: mirrors first, then the swap */
  int mx = rx < 0.0, my = ry < 0.0;
  double ax = fabs(rx), ay = fabs(ry);
  int sw = ay > ax;
  x[0] = (sw ? ay : ax) / PO_PI;
  x[1] = (sw ? ax : ay) / PO_PI;
  x[2] = mu / t;
  x[3] = log10(T / t);
  x[4] = tp / t;
  x[5] = log10(Omega / t);
  x[6] = (channel == PO_PH) ? 1.0 : -1.0;
  /* cell map by geometry: the centre of container cell c, moved the same way */
  const double w = 2.0 * PO_PI / PO_SEED_G;
  for (int j = 0; j < PO_SEED_G; ++j)
    for (int i = 0; i < PO_SEED_G; ++i) {
      double px = -PO_PI + (i + 0.5) * w, py = -PO_PI + (j + 0.5) * w;
      if (hx) px += PO_PI;
      if (hy) py += PO_PI;
      if (px >= PO_PI) px -= 2.0 * PO_PI;
      if (py >= PO_PI) py -= 2.0 * PO_PI;
      if (mx) px = -px;
      if (my) py = -py;
      if (sw) {
        double tt = px;
        px = py;
        py = tt;
      }
      int ci = (int)floor((px + PO_PI) / w), cj = (int)floor((py + PO_PI) / w);
      cellmap[j * PO_SEED_G + i] = cj * PO_SEED_G + ci;
    }
}

/* area of [a0,a1) x [b0,b1) inside cell (i, j), as a fraction of the cell */
static double po_cell_overlap(const double *r, int i, int j) {
  const double w = 2.0 * PO_PI / PO_SEED_G;
  double cx0 = -PO_PI + i * w, cy0 = -PO_PI + j * w;
  double ox = fmin(r[1], cx0 + w) - fmax(r[0], cx0);
  double oy = fmin(r[3], cy0 + w) - fmax(r[2], cy0);
  if (ox <= 0.0 || oy <= 0.0) return 0.0;
  /* quadtree rectangles cover dyadic fractions of a cell (multiples of
     4^-20 down to depth 24): snap away the rounding of the coordinates */
  return nearbyint((ox / w) * (oy / w) * 1099511627776.0) / 1099511627776.0;
}

void po_tree_labels(const double *rects, long n, double y[256]) {
  double cnt[256];
  for (int c = 0; c < 256; ++c) cnt[c] = 0.0;
  const double cell_area = (2.0 * PO_PI / PO_SEED_G) * (2.0 * PO_PI / PO_SEED_G);
  for (long k = 0; k < n; ++k) {
    const double *r = &rects[4 * k];
    double area = (r[1] - r[0]) * (r[3] - r[2]);
    for (int j = 0; j < PO_SEED_G; ++j)
      for (int i = 0; i < PO_SEED_G; ++i) {
        double f = po_cell_overlap(r, i, j);
        if (f > 0.0) cnt[j * PO_SEED_G + i] += f * cell_area / area;
      }
  }
  for (int c = 0; c < 256; ++c) y[c] = log2(1.0 + cnt[c]);
}

static double po_node_count(const double count[256], const double *r) {
  double s = 0.0;
  for (int j = 0; j < PO_SEED_G; ++j)
    for (int i = 0; i < PO_SEED_G; ++i) {
      double f = po_cell_overlap(r, i, j);
      if (f > 0.0) s += f * count[j * PO_SEED_G + i];
    }
  return s;
}

/* leaves under node r at depth d; appends them to rects while room is left */
static long po_seed_rec(const double count[256], const double *r, int d, int D, double thresh,
                        double *rects, long *nw, long limit) {
  if (d < D && po_node_count(count, r) >= thresh) {
    long n = 0;
    for (int a = 0; a < 4; ++a) {
      double cr[4];
      po_split_geo(r, a, cr);
      n += po_seed_rec(count, cr, d + 1, D, thresh, rects, nw, limit);
    }
    return n;
  }
  if (rects && *nw < limit) memcpy(&rects[4 * (*nw)], r, 4 * sizeof(double));
  ++*nw;
  return 1;
}

long po_seed_tree(const double count[256], int dmax, double thresh, long limit, double *rects,
                  int *dmax_used) {
  const double root[4] = {-PO_PI, PO_PI, -PO_PI, PO_PI};
  for (int D = dmax; D >= 0; --D) {
    long nw = 0;
    long n = po_seed_rec(count, root, 0, D, thresh, NULL, &nw, 0);
    if (n <= limit || D == 0) {
      if (rects) {
        nw = 0;
        po_seed_rec(count, root, 0, D, thresh, rects, &nw, limit);
      }
      if (dmax_used) *dmax_used = D;
      return n;
    }
  }
  return -1;
}
