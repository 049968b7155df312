/*
 * paid.h -- C ABI of libpaid, the MI355X (gfx950) implementation of the
 * adaptive Brillouin-zone quadrature of the scale-derivative bubbles of the
 * truncated-unity fRG (arXiv:1610.09991).
 *
 * What is computed (Sec. 2, Eqs. chi_pp and chi_ph, with the dot of the
 * flow equations): for every container = (parameter row, transfer momentum
 * l = q, channel j in {pp, ph}) and every pair of form factors (m, n)
 *
 *   chidot^j_mn(l) = int_{[-pi,pi)^2} d^2p/(2pi)^2  g_j(p) f_m(p) f_n(p),
 *   g_j(p) = T sum_{w_n} d/dOmega [theta(w_n)^2] G-product_j,
 *   theta(w) = w^2/(w^2+Omega^2),  w_n = (2n+1) pi T,
 *   ph: 1/((i w - a)(i w - b)),  pp: 1/((i w - a)(-i w - b)),
 *   a = eps(l/2 + p),  b = eps(l/2 - p),
 *   eps(k) = -2t(cos kx + cos ky) - 4t' cos kx cos ky - mu.
 *
 * How (Secs. 3-4, Alg. 2): nested Clenshaw-Curtis pair Q_N / Q_2N on every
 * rectangle (N intervals per axis, the coarse nodes a subset of the fine
 * ones), error |Q_N - Q_2N|, worst-error-first subdivision of rectangles
 * into 2x2 children with bulk extraction (the MaxTask analogue), global
 * error criterion over all form-factor pairs of a container, result the sum
 * of Q_2N over the leaves.  All containers of a call run together on the GPU.
 *
 * Conventions for every entry point:
 *   - return value: PAID_OK (0), a positive warning, or a negative error;
 *     the message of the last failure is paid_last_error(ctx);
 *   - input arrays are read-only and owned by the caller; output arrays are
 *     owned by the caller and fully written on PAID_OK and PAID_ENOCONV;
 *   - pointers may be host or device (HIP) memory unless stated otherwise;
 *     the library detects which;
 *   - calls on one context are serialised on the context's stream and are
 *     synchronous: on return the outputs are complete;
 *   - one context per host thread; contexts are independent.
 */
#ifndef PAID_H
#define PAID_H

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
enum {
  PAID_OK = 0,
  PAID_ENOCONV = 1,    /* warning: some container hit max_regions; outputs hold
                          the best value and its error estimate */
  PAID_EINVAL = -1,    /* invalid argument */
  PAID_ENOMEM = -2,    /* device memory exhausted */
  PAID_EDEVICE = -3,   /* HIP runtime error (message has the HIP error string) */
  PAID_EINTERNAL = -4
};

/* integrand kinds */
enum {
  PAID_BUBBLE_DOT = 0, /* d/dOmega of the regulated bubble: the flow integrand */
  PAID_BUBBLE = 1,     /* the regulated bubble itself (theta^2 G G) */
  PAID_UNIT = 2,       /* g = 1 (integral of f_m f_n), for checks */
  PAID_GAUSS = 3       /* g = exp(-|p - p0|^2/(2 sigma^2)), for checks */
};

/* channel bits of paid_integrate's `channels` */
enum { PAID_PP = 1, PAID_PH = 2 };

/* termination test (Sec. 3 and Alg. 2) */
enum {
  PAID_ERR_GLOBAL = 0,       /* sum over pairs and leaves of |Q_N - Q_2N| <=
                                max(atol, rtol * sum over pairs |value|)  (the
                                paper's global criterion) */
  PAID_ERR_PER_INTEGRAL = 1, /* every pair: sum over leaves of its error <=
                                max(atol, rtol * max(|value_pq|, nu max |value|));
                                per-leaf errors are kept in FP32, positive ones
                                never below FLT_MIN, so a pair whose tolerance is
                                below FP32's normal range (|value| ~ 1e-30 and
                                less) ends PAID_ENOCONV rather than passing */
  PAID_ERR_WEIGHTED = 2      /* the global test with pair weights w (set with
                                paid_set_pair_weights): sum over leaves and pairs
                                of w |Q_N - Q_2N| <= max(atol, rtol * sum w |value|);
                                with w from the couplings (Eq. P_globerr) it
                                bounds the error of the contracted matrices */
};

/* arithmetic of the form-factor projection */
enum {
  PAID_FP64 = 0,   /* everything in FP64 */
  PAID_FP32 = 1,   /* projection in FP32 on the matrix cores, FP64 sums */
  PAID_BF16X3 = 2  /* projection with three-term bf16 splits, FP32 accumulate */
};

/* how the projection F^T diag(w g) F is formed */
enum {
  PAID_GRAM_MFMA = 0,      /* dense weighted Gram contraction on the FP64 matrix cores */
  PAID_GRAM_SEPARABLE = 1  /* the same sums factored along the two axes (default) */
};

typedef struct {
  int device;           /* HIP device ordinal */
  int N;                /* coarse rule: N intervals per axis (fine: 2N); 4 */
  int batch;            /* minimum leaves split per container per round
                           (the MaxTask analogue), >= 1; batch = batch_max
                           = 1 splits exactly the leaf of largest key per
                           round, ties by creation order (the serial order
                           of Alg. 2) */
  int batch_max;        /* maximum leaves split per container per round */
  int err_mode;         /* PAID_ERR_* */
  int precision;        /* PAID_FP64 / PAID_FP32 / PAID_BF16X3 */
  int gram;             /* PAID_GRAM_* */
  int kind;             /* PAID_BUBBLE_DOT (default), ... */
  double nu;            /* floor factor of PAID_ERR_PER_INTEGRAL */
  long max_regions;     /* leaf budget per container */
  int max_active;       /* containers resident at once (0: from pool size) */
  double pool_gib;      /* region pool size in GiB (0: a share of free memory) */
  double gauss[3];      /* PAID_GAUSS centre (x, y) and width */
  void *stream;         /* hipStream_t to run on, or NULL for a private stream */
  int profile;          /* 1: time the region-evaluation launches with HIP
                           events on the context stream (paid_stats.eval_*) */
  int graph;            /* 1: capture the device round (seven kernels and the
                           read-back of three counters, in three parts around
                           the evaluation launch) as HIP graphs and replay
                           them every round */
  int eval_wg_per_cu;   /* workgroups of the region-evaluation launch per
                           compute unit (0: 16 per workgroup the kernel's
                           occupancy fits on a compute unit); the work items
                           of a round are split over them in geometrically
                           shrinking ranges; grids much shorter than the
                           default hand the first workgroups more than an
                           even share (8 per occupancy slot: ~25% slower) */
  int symmetry;         /* 1: integrate over the half zone p_y >= 0 only.  The
                           integrand of both bubbles is even under p -> -p
                           (it swaps the energies eps(l/2 + p) and
                           eps(l/2 - p), and K_j is symmetric in them), so a
                           pair of box functions of odd joint parity (an odd
                           number of sine factors) integrates to exactly 0
                           and any other pair to twice its half-zone
                           integral.  Not part of the paper's scheme; not
                           with PAID_GAUSS, learned seeding or tree labels */
  int eval_layout;      /* region-evaluation kernel: 0 (default) the fastest for
                           the basis (for the 9-function box basis with the
                           separable projection over the full zone, two lanes
                           per child rectangle and 8 parents per wave, all
                           sums in registers; otherwise one wave per parent),
                           1 always one wave per parent.  Both compute the same
                           rule sums, in different rounding orders */
  long small_regions;   /* 0 (default): every resident container may hold
                           max_regions leaves.  16 <= small_regions <
                           max_regions: two kinds of slots share the pool.
                           New containers start in small slots of
                           small_regions leaves; a container whose next round
                           could overflow its small slot moves (leaves and
                           sums copied) to a large slot of max_regions leaves
                           and waits until one is free.  The trees and results
                           are those of one kind of slot of max_regions: a
                           container never splits fewer leaves because of the
                           small slot.  When few containers need the full
                           budget, more are resident at once */
  double big_share;     /* share of the pool for the large slots, in (0, 1);
                           0: 0.25 */
} paid_config;

/* one parameter row: dispersion, temperature and flow scale */
typedef struct {
  double t, tp, mu, T, Omega;
} paid_params;

typedef struct {
  long containers;      /* containers integrated */
  long not_converged;   /* containers that hit max_regions */
  long regions;         /* leaves at exit, summed over containers */
  long splits;          /* rectangles subdivided, summed */
  long kernel_evals;    /* evaluations of the scalar integrand g */
  long rounds;          /* bulk-extraction rounds, summed over containers */
  long launch_rounds;   /* device rounds of the whole call */
  int max_depth;        /* deepest subdivision level */
  int max_active;       /* containers resident at once */
  double seconds;       /* wall time of the call */
  double eval_seconds;  /* profile: summed duration of the region-evaluation launches */
  long eval_launches;   /* profile: number of those launches */
  long eval_items;      /* parents evaluated (each gives 4 children) */
  long seeded;          /* containers started from a seed tree */
  double seed_seconds;  /* model features and inference inside this call */
} paid_stats;

/* Fill *cfg with defaults (device 0, N = 4, batch 8, batch_max 1024, global
 * error, FP64, separable projection, nu = 1e-3, max_regions = 2^18,
 * automatic pool). */
int paid_config_default(paid_config *cfg);

/* Create a context on cfg->device.  *out receives the context (NULL on
 * failure).  The context owns its device workspace, tables and stream. */
int paid_create(struct paid_ctx **out, const paid_config *cfg);

/* Integrate every container of the batch (Alg. 2 over all containers).
 *   params   [n_params] parameter rows (t > 0 not required; T > 0, Omega >= 0)
 *   q        [n_q][2]   transfer momenta l in radians (not reduced mod 2pi)
 *   ff       [n_ff][(2 ff_L + 1)^2] form factors as coefficients over the
 *            box basis u_a(p_x) u_b(p_y), u_0 = 1, u_{2k-1} = sqrt2 cos kx,
 *            u_{2k} = sqrt2 sin kx; rows must be orthonormal (to 1e-12);
 *            0 <= ff_L <= 2, 1 <= n_ff <= (2 ff_L + 1)^2
 *   channels PAID_PP | PAID_PH (at least one)
 *   rtol, atol  tolerance of the termination test (rtol > 0 or atol > 0)
 *   out      [n_params][n_q][n_ch][n_ff][n_ff] FP64, both halves written,
 *            channel order pp before ph
 *   err_out  NULL or the same shape: per pair, sum over leaves of
 *            |Q_N - Q_2N|
 *   stats    NULL or filled on return
 * n_params >= 1 and n_q >= 1 (an empty batch is PAID_EINVAL).
 * Returns PAID_OK, PAID_ENOCONV (some container hit max_regions or the
 * smallest rectangle a region code holds, side 2 pi / 2^28; its output is
 * its sum over the leaves it has), or an error (outputs then undefined). */
int paid_integrate(struct paid_ctx *ctx, const paid_params *params, int n_params,
                   const double *q, int n_q, const double *ff, int n_ff, int ff_L,
                   unsigned channels, double rtol, double atol, double *out,
                   double *err_out, paid_stats *stats);

/* Frequency-summed kernel g = K_j(a, b) of one parameter row at n energy
 * pairs (the closed-form frequency sum of Sec. 2 as the library evaluates
 * it).  channel: PAID_PP or PAID_PH.  a, b, out: [n], n >= 0 (NULL allowed
 * when n = 0); energies beyond the band bound 4|t| + 4|t'| + |mu| are
 * PAID_EINVAL. */
int paid_kernel_eval(struct paid_ctx *ctx, const paid_params *p, unsigned channel,
                     const double *a, const double *b, int n, double *out);

/* Evaluate the four children of n parent rectangles of one container with
 * the same device code paid_integrate uses (Sec. 3 rule pair on each child).
 * A rectangle is coded as (depth, ix, iy): x in [-pi + 2pi ix/2^depth,
 * -pi + 2pi (ix+1)/2^depth), likewise y.  codes: [n][3] int.
 * q2n: [n][4][n_ff (n_ff+1)/2] upper-triangle pairs, row-major;
 * err: [n][4] key of each child (sum over pairs of |Q_N - Q_2N|).  Children
 * are ordered (x-lo,y-lo), (x-hi,y-lo), (x-lo,y-hi), (x-hi,y-hi). */
int paid_children_eval(struct paid_ctx *ctx, const paid_params *p, const double *l,
                       unsigned channel, const double *ff, int n_ff, int ff_L,
                       const int *codes, int n, double *q2n, double *err);

/* ------------------------------------------------------------------------
 * Learned seeding of the initial partition (not in the paper; the adaptive
 * scheme of Alg. 2 still decides termination and every further split).
 *
 * A perceptron 7 -> 128 -> 128 -> 128 -> 256 (GELU(z) = z Phi(z) on the
 * hidden layers, linear output, FP32) maps the features of a container to
 * the predicted log2(1 + n_c) for the 16 x 16 cells c of the zone, n_c the
 * number of leaves of its converged tree in c (leaves larger than a cell
 * count with the share of their area).  Parameters are one FP32 array:
 * per layer W [out][in] row-major, then b [out].
 *
 * Model frame.  l is reduced to [-pi, pi)^2 (an odd number of 2 pi shifts
 * moves the integrand by pi in p) and then to the wedge 0 <= l_y <= l_x by
 * the square's symmetries; the cells move with it.  Features: l_x/pi, l_y/pi
 * (reduced), mu/t, log10(T/t), t'/t, log10(Omega/t), -1 (pp) or +1 (ph).
 * Cell c = 16 j + i covers x in [-pi + i pi/8, -pi + (i+1) pi/8), likewise y.
 *
 * Seed tree: from the predicted counts (n = max(0, 2^y - 1) per cell, summed
 * over the cells a node covers, shared by area below a cell) a node is split
 * while its count is >= 4 kappa and its depth < D; D starts at dmax and is
 * lowered until the tree has at most max_regions/4 leaves.
 * Only the leaves of the seed tree are integrated; the adaptive loop then
 * continues from them.
 */
#define PAID_MLP_IN 7
#define PAID_MLP_OUT 256

/* Number of model parameters (67072). */
long paid_mlp_nparams(void);

/* Use the model `weights` ([paid_mlp_nparams()] FP32, copied, all finite)
 * for the seeding of every later paid_integrate call on ctx, with depth
 * bound dmax (0..12) and threshold 4 kappa (kappa > 0); weights NULL turns
 * seeding off (dmax and kappa are then ignored). */
int paid_set_seed_model(struct paid_ctx *ctx, const float *weights, int dmax, double kappa);

/* Make every later paid_integrate call on ctx also write, per container in
 * the order of `out`, its model features [n_ctr][7] and the labels of its
 * converged tree in the model frame [n_ctr][256] (FP32).  Both pointers are
 * caller-owned, sized for each call, host or device; NULLs turn it off. */
int paid_set_label_output(struct paid_ctx *ctx, float *features, float *labels);

/* Pair weights of PAID_ERR_WEIGHTED for every later paid_integrate call:
 * w [n_ctr][n_ff][n_ff] (FP64, >= 0, containers in the order of out), the
 * weights of the full matrix entries; the stored pair p < q carries
 * w_pq + w_qp and the pair p = p carries w_pp (so that, for dX = V chi V and
 * w_pq = (sum_m |V_mp|)(sum_n |V_qn|), sum_mn |dX_mn| <= sum w |d chi|).
 * Host or device pointer, caller-owned and sized for each call; NULL clears. */
int paid_set_pair_weights(struct paid_ctx *ctx, const double *w);

/* Make every later paid_integrate call on ctx also write, per container in
 * the order of `out`, the leaves of its final tree in the library's pool
 * order, at most cap of them: codes [n_ctr][cap][3] = (depth, ix, iy) of the
 * rectangle x in [-pi + 2pi ix/2^depth, -pi + 2pi (ix+1)/2^depth), likewise
 * y (entries past the last leaf are -1), and q2n [n_ctr][cap][n_ff (n_ff+1)/2]
 * the rectangle's Q_2N for the pairs p <= q.  Caller-owned, sized for each
 * call, host or device; NULLs turn it off.  With batch = batch_max = 1 every
 * round splits the leaf of largest key (ties by creation order), which is
 * the serial order of Alg. 2, so the leaves can be compared one by one with
 * a serial implementation. */
int paid_set_leaf_output(struct paid_ctx *ctx, int *codes, double *q2n, long cap);

/* Model forward pass: x [n][7] -> y [n][256]. */
int paid_mlp_forward(struct paid_ctx *ctx, const float *w, const float *x, int n, float *y);

/* Mean squared error over n samples and 256 outputs, and its gradient
 * grad [nparams] (same layout as w); *loss may be NULL.  n <= 65536. */
int paid_mlp_loss_grad(struct paid_ctx *ctx, const float *w, const float *x, const float *y,
                       int n, float *grad, double *loss);

/* The loss and gradient of paid_mlp_loss_grad for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving or
 * training loops, harnesses that forbid allocation.  Same kernels, same
 * results (bit for bit) as paid_mlp_loss_grad, but no call allocates or
 * frees memory: the working memory (per-sample activations and deltas of up
 * to PAID_NOALLOC_MAX_N samples, and the loss; 13.6 MB) is a fixed array of
 * the library on each device, held until the process ends, and the loss is
 * read back through the context's pinned buffer.
 *   w [nparams], x [n][7], y [n][256], grad [nparams]: device memory only
 *   (host pointers: PAID_EINVAL); 1 <= n <= PAID_NOALLOC_MAX_N (larger n:
 *   PAID_EINVAL, nothing launched); loss may be NULL.
 * Every call on a device uses that device's one array: calls that overlap
 * on one device (other contexts, other host threads) race and must be
 * serialised by the caller.  Nothing in the array has to start at zero. */
#define PAID_NOALLOC_MAX_N 2048
int paid_mlp_loss_grad_noalloc(struct paid_ctx *ctx, const float *w, const float *x,
                               const float *y, int n, float *grad, double *loss);

/* One Adam step in place (beta1 0.9, beta2 0.999, eps 1e-8, step t >= 1):
 * m, v are the moment arrays, all [nparams], device memory only. */
int paid_mlp_adam(struct paid_ctx *ctx, float *w, const float *grad, float *m, float *v, int t,
                  float lr);

typedef struct {
  int steps;              /* Adam steps */
  int batch;              /* samples per step, 1..1024 */
  float lr, lr_final;     /* learning rate, cosine decay from lr to lr_final */
  unsigned long long seed;/* shuffling and initialisation */
  int init;               /* 1: initialise w (normal, std 1/sqrt(fan-in)), 0: start from w */
  int use_graph;          /* 1: capture one step in a HIP graph and replay it */
} paid_train_opts;

/* Defaults: 3000 steps, batch 256, lr 2e-3 -> 5e-5, seed 1, init 1, graph 1. */
int paid_train_opts_default(paid_train_opts *o);

/* Train the model on the GPU: minibatches drawn without replacement from
 * n samples (x [n][7], y [n][256]), reshuffled every pass; w [nparams]
 * in/out; loss_hist NULL or [steps] FP64 minibatch losses. */
int paid_seed_train(struct paid_ctx *ctx, const float *x, const float *y, int n,
                    const paid_train_opts *opts, float *w, double *loss_hist);

/* The contraction beside the integration (Sec. 2, Eqs. matmul-P, matmul-C,
 * matmul-D), per transfer momentum l:
 *   dP = V^P chi^pp V^P,   dC = -V^C chi^ph V^C,
 *   dD = 2 V^D chi^ph V^D - V^C chi^ph V^D - V^D chi^ph V^C,
 * on the FP64 matrix cores.
 *   chi  [n_l][2][M][M]: both channels, pp first (the layout paid_integrate
 *        writes with channels PAID_PP | PAID_PH, n_l = n_params * n_q)
 *   VP, VC, VD, dP, dC, dD  [n_l][M][M] FP64 row-major
 * 1 <= M <= 32, n_l >= 0.  Host or device pointers. */
int paid_contract(struct paid_ctx *ctx, int n_l, int M, const double *chi, const double *VP,
                  const double *VC, const double *VD, double *dP, double *dC, double *dD);

/* A flow driver over the scale (the flow equations of Sec. 2 with the
 * couplings held fixed): integrates
 *   dP/dOmega = V^P chidot^pp V^P,  dC/dOmega = -V^C chidot^ph V^C,
 *   dD/dOmega = 2 V^D chidot^ph V^D - V^C chidot^ph V^D - V^D chidot^ph V^C
 * from omega0 to omega1 (either direction) with the Dormand-Prince 5(4)
 * pair and step-size control in ln Omega; every stage is one batched
 * paid_integrate of all transfer momenta and both channels followed by
 * paid_contract.  The context's kind must be PAID_BUBBLE_DOT.
 *   base  t, tp, mu, T of the parameter row (its Omega is ignored)
 *   q [n_q][2], ff, n_ff, ff_L: as for paid_integrate
 *   VP, VC, VD [n_q][n_ff][n_ff]; P, C, D [n_q][n_ff][n_ff] in: the state at
 *   omega0, out: at omega1.  Host pointers (device pointers: PAID_EINVAL). */
typedef struct {
  double omega0, omega1;  /* > 0 */
  double rtol, atol;      /* step control: max |err| <= atol + rtol max |state| */
  double rtol_int;        /* tolerance of each integration (<= rtol / 10 advised) */
  double h0;              /* first step in ln Omega (0: automatic) */
  int max_steps;
} paid_flow_opts;

typedef struct {
  int steps, rejected, evaluations;  /* accepted and rejected steps, integrations */
  long kernel_evals;                 /* integrand evaluations of all integrations */
  double seconds;
} paid_flow_stats;

int paid_flow_opts_default(paid_flow_opts *o);
int paid_flow(struct paid_ctx *ctx, const paid_params *base, const double *q, int n_q,
              const double *ff, int n_ff, int ff_L, const double *VP, const double *VC,
              const double *VD, double *P, double *C, double *D, const paid_flow_opts *opts,
              paid_flow_stats *stats);

/* Release the context and everything it owns.  NULL is accepted. */
void paid_destroy(struct paid_ctx *ctx);

/* Message of the last failure on ctx (or of the last paid_create failure
 * when ctx is NULL).  Valid until the next call on the same context. */
const char *paid_last_error(const struct paid_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
