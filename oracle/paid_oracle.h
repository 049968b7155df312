/*
 * paid_oracle.h -- plain FP64 CPU oracle for the adaptive Brillouin-zone
 * quadrature of the scale-derivative bubbles (Lichtenstein, Sanchez de la
 * Pena, Di Napoli et al., "Parallel adaptive integration in high-performance
 * functional Renormalization Group computations", arXiv:1610.09991).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against a slow, obviously correct implementation.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.
 * It shares no code, header or table with the GPU library.
 *
 * Everything here is double precision, serial per problem, and follows the
 * paper's definitions directly:
 *   - dispersion eps(k) of the t-t' square lattice           (Sec. 2)
 *   - regulated propagator G = theta/(i k0 - eps),
 *     theta(k0) = k0^2/(k0^2+Omega^2)                        (Sec. 2)
 *   - bubbles chi^pp, chi^ph with the frequency sum done as a Matsubara sum
 *     at temperature T; the "dot" is d/dOmega of the whole regulated product
 *                                                            (Eqs. chi_pp, chi_ph)
 *   - nested Clenshaw-Curtis pair Q_N / Q_2N, err = |Q_N - Q_2N| (Sec. 3)
 *   - adaptive subdivision with a global error criterion     (Alg. 1, Alg. 2)
 *     and MaxTask bulk extraction                             (Sec. 4, Listings 1-5)
 */
#ifndef PAID_ORACLE_H
#define PAID_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* integrand kinds */
enum { PO_BUBBLE_DOT = 0, /* d/dOmega of the regulated bubble (the flow integrand) */
       PO_BUBBLE = 1,     /* regulated bubble itself (theta^2 G G), for derivative checks */
       PO_UNIT = 2,       /* g = 1: integral of f_m f_n, orthonormality check */
       PO_GAUSS = 3 };    /* g = exp(-|p-p0|^2/(2 sigma^2)), closed-form check */
/* channels */
enum { PO_PP = 0, PO_PH = 1 };
/* task granularity of Alg. 2 */
enum { PO_MODE_A = 0,  /* one task = (region, form-factor pair), paper-literal */
       PO_MODE_B = 1 };/* one task = region, all pairs refined together (shared tree) */
/* termination */
enum { PO_ERR_GLOBAL = 0, PO_ERR_PER_INTEGRAL = 1,
       PO_ERR_WEIGHTED = 2 };  /* global criterion with pair weights (Eq. P_globerr) */

typedef struct {
  int kind, channel;
  double t, tp, mu, T, Omega;   /* dispersion and scale */
  double lx, ly;                /* transfer momentum l */
  int ff_L;                     /* box basis order: (2L+1)^2 basis functions */
  int n_ff;                     /* number of form factors M */
  const double *ff;             /* [n_ff][(2L+1)^2] coefficients over the box basis */
  double gx, gy, gsigma;        /* PO_GAUSS centre and width */
  const double *pair_w;         /* PO_ERR_WEIGHTED: [n_ff][n_ff] weights of the full
                                   matrix entries; the stored pair p < q carries
                                   w_pq + w_qp, the pair p = p carries w_pp */
} po_problem;

typedef struct {
  int N;            /* coarse rule: N intervals per axis; fine rule 2N */
  int mode;         /* PO_MODE_A / PO_MODE_B */
  int err_mode;     /* PO_ERR_GLOBAL / PO_ERR_PER_INTEGRAL */
  int batch;        /* MaxTask: tasks extracted per round, >= 1 */
  double rtol, atol, nu;
  long max_regions; /* budget of leaf tasks per problem */
} po_options;

typedef struct {
  long regions;      /* leaf tasks at exit */
  long splits;       /* tasks subdivided */
  long kernel_evals; /* evaluations of the scalar integrand g */
  long rounds;       /* extraction rounds */
  int converged;     /* 1 if the termination test passed */
  int max_depth;
} po_stats;

/* Clenshaw-Curtis rule on [-1,1] with n intervals: nodes cos(k pi/n), k=0..n. */
int po_cc_rule(int n, double *nodes, double *weights);
/* Hurwitz zeta sum_{j>=0} (q+j)^-s for s > 1, q > 0. */
double po_hurwitz_zeta(double s, double q);
/* t-t' dispersion. */
double po_dispersion(double t, double tp, double mu, double kx, double ky);
/* frequency-summed kernel g = K(a,b) for the given kind/channel. */
double po_kernel(int kind, int channel, double a, double b, double Omega, double T);
/* Fermi function, for checks */
double po_fermi(double e, double T);
/* box basis values u_0..u_{2L} at x */
void po_box_basis(int L, double x, double *u);
/* scalar integrand g(p) of a problem */
double po_integrand(const po_problem *pr, double px, double py);
/* Q_N and Q_2N over one rectangle for all unique pairs (p<=q, row-major
   upper triangle), measure d^2p/(2pi)^2. */
int po_region_eval(const po_problem *pr, int N, double x0, double x1, double y0,
                   double y1, double *qn, double *q2n);
/* Adaptive integration of one problem. value/err: [n_ff][n_ff], both halves.
   Returns 0 on convergence, 1 if max_regions was hit, <0 on bad input. */
int po_integrate(const po_problem *pr, const po_options *opt, double *value,
                 double *err, po_stats *st);
/* po_integrate in mode B that also returns the leaves of the final tree in
   creation order: rects [cap][4] = (x0, x1, y0, y1) and q2n [cap][n_ff (n_ff+1)/2]
   (either may be NULL), the first cap of them; *n_leaves = their number. */
int po_integrate_leaves(const po_problem *pr, const po_options *opt, double *value,
                        double *err, po_stats *st, double *rects, double *q2n, long cap,
                        long *n_leaves);
/* Many problems, OpenMP over problems when nthreads > 1. Returns the number
   of problems that did not converge, or <0 on bad input. */
int po_integrate_batch(const po_problem *prs, int n, const po_options *opt,
                       double *values, double *errs, po_stats *sts, int nthreads);
/* Periodic trapezoid on an L x L grid (brute force). value: [n_ff][n_ff] */
int po_brute(const po_problem *pr, int L, double *value);

/* ------------------------------------------------------------------------
 * Subdivision-density model (the learned seeding of the initial partition):
 * a multilayer perceptron 7 -> 128 -> 128 -> 128 -> 256 with GELU(z) =
 * z Phi(z) on the hidden layers and a linear output layer.  Parameters are
 * one array: W1[128][7], b1[128], W2[128][128], b2[128], W3[128][128], b3[128],
 * W4[256][128], b4[256] (row-major, out x in).  Loss: mean over samples and
 * outputs of (yhat - y)^2.  FP64, plain loops. */
#define PO_MLP_IN 7
#define PO_MLP_HID 128
#define PO_MLP_OUT 256
long po_mlp_nparams(void);
/* yhat [n][256] */
void po_mlp_forward(const double *w, const double *x, int n, double *yhat);
/* loss and its gradient (same layout as w) */
double po_mlp_loss_grad(const double *w, const double *x, const double *y, int n, double *grad);
/* one Adam step (beta1 0.9, beta2 0.999, eps 1e-8); m, v: moments, t: step >= 1 */
void po_mlp_adam(double *w, const double *g, double *m, double *v, long np, int t, double lr);

/* ------------------------------------------------------------------------
 * Seeding the initial partition from a predicted subdivision density.
 * The density lives on a 16 x 16 grid of cells over [-pi,pi)^2; cell (i, j)
 * covers x in [-pi + i pi/8, -pi + (i+1) pi/8) and likewise y, stored at
 * index 16 j + i.  Labels of a tree: y_c = log2(1 + n_c), n_c = the number
 * of leaves in cell c, a leaf larger than a cell counting with the fraction
 * of its area inside the cell.
 *
 * Model frame: the integrand at transfer momentum l equals the integrand at
 * l - 2 pi e_x shifted by pi e_x in p (both energies are periodic), and the
 * lattice is symmetric under the point group D4; so the model sees l
 * reduced to [-pi,pi)^2 and then to the wedge 0 <= l_y <= l_x, and the cell
 * map takes each cell of the container to the matching model cell.
 * Features: l_x/pi, l_y/pi (reduced), mu/t, log10(T/t), t'/t, log10(Omega/t),
 * channel (-1 pp, +1 ph). */
#define PO_SEED_G 16
void po_seed_features(double t, double tp, double mu, double T, double Omega, double lx,
                      double ly, int channel, double x[7], int cellmap[256]);
/* labels of n leaf rectangles [n][4] = (x0, x1, y0, y1) */
void po_tree_labels(const double *rects, long n, double y[256]);
/* po_integrate, also returning the labels of the final tree (mode B only) */
int po_integrate_labels(const po_problem *pr, const po_options *opt, double *value,
                        double *err, po_stats *st, double labels[256]);
/* Seed tree from per-cell predicted leaf counts (container frame): a node is
 * split while its predicted count (the area-weighted sum over the cells it
 * overlaps) is >= thresh and its depth is < D.  D starts at dmax and is
 * lowered until the tree has at most `limit` leaves.  Writes the leaves to
 * rects [n][4] when non-NULL (capacity `limit`), *dmax_used = D; returns the
 * leaf count. */
long po_seed_tree(const double count[256], int dmax, double thresh, long limit, double *rects,
                  int *dmax_used);

#ifdef __cplusplus
}
#endif
#endif
