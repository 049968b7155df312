// launch.h -- host-side launch interface between the C ABI (api.hip) and the
// kernel translation units.  Library-internal.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "paid.h"
#include "paid_device.h"

namespace paid {

// rule constants, filled once per device (ascending node order on [-1,1])
constexpr int kDelDepths = 29;  // parent depths 0..28
struct RuleConst {
  double xi[kNF];   // fine nodes
  double w2[kNF];   // fine weights
  double w1[kNCo];  // coarse weights (at fine nodes 0,2,4,6,8)
  // cos and sin of the offsets of a child's nodes from its centre,
  // delta_a = (pi 2^-(d+1)) xi_a for parent depth d and a = 0..4 (the nodes
  // a = 5..8 have the opposite offsets)
  double cdel[kDelDepths][5], sdel[kDelDepths][5];
};

// ------------------------------------------------------------------ tables
struct TabArgs {
  Entry *entries;    // [n_entries], J/tab_off/nmats/emax filled by the host
  int n_entries;
  int max_J;
  double *tab;       // table buffer
  double *zeta;      // [n_entries][kTabKTail+1] scratch
  double2 *svals;    // [n_entries][max_J][kTabPts] scratch
};
hipError_t launch_tables(const TabArgs &a, hipStream_t s);

// ------------------------------------------------------------------ setup
hipError_t launch_container_setup(Ctr *ctr, int n_ctr, const double *q, int n_q, int n_ch,
                                  int ch_first, hipStream_t s);

// ------------------------------------------------------------------ pool and queue
// SLOT_MOVE: a container in a small slot waiting for a large one
enum SlotState { SLOT_EMPTY = 0, SLOT_NEW = 1, SLOT_ACTIVE = 2, SLOT_DONE = 3, SLOT_MOVE = 4 };

struct Problem {      // everything the round kernels need, passed by value
  // static description
  const Entry *entries;
  const double *tab;
  const Ctr *ctr;
  int n_ctr;
  int kind;
  int err_mode;
  int precision;
  int gram;
  double gauss_x, gauss_y, gauss_s;
  double rtol, atol, nu;
  // form factors
  int L, nb, MB, M, MU;       // box order, harmonics per axis, box size, n_ff, pairs
  int ff_identity;            // 1: form factors are the box basis itself
  const double *ffc;          // [M][MB]
  // pool
  int W;                      // slots
  long cap;                   // regions per slot (per small slot when Wb > 0)
  int Wb;                     // large slots 0..Wb-1 of capb regions each (0: one kind)
  long capb;                  // regions per large slot
  int *promo;                 // [Wb] small slot moving into each large slot this round, -1: none
  int *moveq;                 // [W] scratch: the waiting small slots in slot order
  int bmin, bmax;
  int lds_wave_doubles;       // per-wave LDS of the evaluation kernel (set at launch)
  int tab_rows;               // rows of the largest frequency-sum table (the LDS table)
  int lds_limit;              // bytes of LDS a workgroup may use on the device
  int eval_slots;             // evaluation workgroups resident at once (0: even partition)
  int sym;                    // 1: half zone p_y >= 0 with the parity factors of the pairs
  int eval_layout;            // 0: the fastest evaluation kernel for the basis, 1: one wave per parent
  uint64_t *code;             // [regions], slot s from slot_base(s)
  double *key;                // [regions]
  double *Q;                  // [regions*MU]
  float *E;                   // [regions*MU] or NULL
  // slot state
  int *cid, *state, *nleaf, *selcnt, *sel, *woff;  // sel: [W*bmax], woff: [W+1]
  int *flags;                 // [W]: bit0 = converged, bit1 = budget hit
  double *val;                // [W*MU]
  double *err;                // [W]   (sum of keys)
  double *errp;               // [W*MU] per pair (when E != NULL)
  float *itau;                // [W*MU] key weights (per-integral mode)
  double *dv;                 // [W*bmax*MU]
  double *de;                 // [W*bmax]
  double *dep;                // [W*bmax*MU] (when E != NULL)
  double *upart;              // [W][chunks][2*MU + 2] chunk sums of the deltas
  long *st_rounds, *st_splits;  // [W]
  int *st_depth;              // [W]
  // queue and global counters
  int *qhead;                 // next container to admit
  int *counters;              // [0] done, [1] not converged, [2] total work items
  long long *gstats;          // [0] rounds [1] splits [2] leaves [3] max depth
  // outputs (device)
  double *out, *err_out;      // [n_ctr][M][M]
  // learned seeding (seed_y == NULL: every container starts from the root)
  const float *seed_y;        // [n_ctr][256] predicted log2(1 + leaves) per model cell
  const int *seed_fold;       // [n_ctr] container -> model frame (bits: hx hy mx my swap)
  double *pyr;                // [W][kPyr] predicted leaf counts, levels 0..4
  int *seed_d;                // [W] depth bound of the seed tree
  int seed_dmax;
  double seed_thresh;         // split while the predicted count >= this
  long seed_limit;            // most leaves a seed tree may have
  // admission order (NULL: container index order): queue position k takes
  // container row_perm[k / per_row] * per_row + k % per_row
  const int *row_perm;        // [n_params] parameter rows, largest predicted trees first
  int per_row;                // containers per parameter row (q points x channels)
  long *st_evals;             // [W] integrand evaluations
  int *ifill;                 // [W*bmax] 1 if the work item evaluated its node grid
  // tree labels of finished containers (model frame), NULL = off
  float *labels;              // [n_ctr][256]
  // pair weights of the weighted global test (err_mode 2)
  const double *pair_w;       // [n_ctr][M][M] full-matrix weights
  // one leaf per round (batch = batch_max = 1): creation index of every leaf,
  // the exact worst leaf is selected, ties by creation order; NULL otherwise
  unsigned int *born;         // [regions]
  // leaves of finished containers, NULL = off
  int *leaf_codes;            // [n_ctr][leaf_cap][3] (depth, ix, iy), -1 past the last leaf
  double *leaf_q;             // [n_ctr][leaf_cap][MU]
  long leaf_cap;
};

// first region and capacity of slot s (the large slots come first)
__host__ __device__ inline long slot_base(const Problem &P, int s) {
  return s < P.Wb ? (long)s * P.capb : (long)P.Wb * P.capb + (long)(s - P.Wb) * P.cap;
}
__host__ __device__ inline long slot_cap(const Problem &P, int s) { return s < P.Wb ? P.capb : P.cap; }

constexpr int kSeedG = 16;                    // cells per axis of the density grid
constexpr int kPyr = 1 + 4 + 16 + 64 + 256;   // pyramid levels 0..4
constexpr int kFlagSeed = 4;                  // slot flag: seed phase

// model cell read by container cell (i, j) (x index i, y index j)
__host__ __device__ inline int seed_model_cell(int fold, int i, int j) {
  if (fold & 1) i = (i + kSeedG / 2) & (kSeedG - 1);
  if (fold & 2) j = (j + kSeedG / 2) & (kSeedG - 1);
  if (fold & 4) i = kSeedG - 1 - i;
  if (fold & 8) j = kSeedG - 1 - j;
  if (fold & 16) {
    int t = i;
    i = j;
    j = t;
  }
  return j * kSeedG + i;
}

// level offset of depth d in the pyramid
__host__ __device__ inline int pyr_off(int d) { return ((1 << (2 * d)) - 1) / 3; }

// predicted leaf count of the quadtree node `code` of slot s
__device__ inline double seed_count(const Problem &P, int s, uint64_t code) {
  const int d = code_depth(code);
  const double *py = P.pyr + (long)s * kPyr;
  const int ix = (int)code_ix(code), iy = (int)code_iy(code);
  if (d <= 4) return py[pyr_off(d) + (iy << d) + ix];
  const int sh = d - 4;
  return ldexp(py[pyr_off(4) + ((iy >> sh) << 4) + (ix >> sh)], -2 * sh);
}

// does the seed tree split this node?  (only while the slot is seeding)
__device__ inline bool seed_split(const Problem &P, int s, uint64_t code) {
  return (P.flags[s] & kFlagSeed) && code_depth(code) < P.seed_d[s] &&
         seed_count(P, s, code) >= P.seed_thresh;
}

hipError_t launch_admit(const Problem &p, hipStream_t s);
// doubles of the chunk sums of the per-parent deltas (Problem::upart)
size_t update_scratch_doubles(int W, int MU);
// moves of waiting containers from small to large slots (p.Wb > 0)
hipError_t launch_move(const Problem &p, hipStream_t s);
// predicted leaves of every parameter row (sum over its containers and cells
// of max(0, 2^y - 1)), in a fixed summation order
hipError_t launch_seed_rowsize(const float *y, int n_rows, int per_row, double *out, hipStream_t s);
hipError_t launch_root(const Problem &p, hipStream_t s);
hipError_t launch_select(const Problem &p, hipStream_t s);
hipError_t launch_worklist(const Problem &p, hipStream_t s);
// dynamic LDS bytes of the evaluation kernel for p (0: the table does not fit)
size_t eval_lds_bytes(const Problem &p);
// evaluation workgroups that fit on one compute unit at once for p
int eval_occupancy(const Problem &p);
hipError_t launch_eval(const Problem &p, int grid, hipStream_t s);
hipError_t launch_update(const Problem &p, hipStream_t s);
hipError_t launch_finalize(const Problem &p, hipStream_t s);

// diagnostics
hipError_t launch_kernel_eval(const Entry *e, const double *tab, int ch, const double *a,
                              const double *b, int n, double *out, hipStream_t s);

hipError_t set_rule_constants(const RuleConst &rc);

// ------------------------------------------------------------------ density model
constexpr int kMlpIn = 7, kMlpHid = 128, kMlpOut = 256;
struct MlpLayout {
  int ni[4], no[4];
  long w[4], b[4];   // offsets of W_l [out][in] and b_l [out]
  long total;
};
struct MlpAct {        // per-sample buffers: Z pre-activations, A activations, D deltas
  float *Z[4];         // Z[0..2] [n][128] (Z[3] unused)
  float *A[3];         // [n][128]
  float *D[3];         // [n][128]
};
MlpLayout mlp_layout();
hipError_t launch_seed_features(const Entry *entries, const double *q, int n_ctr, int n_q, int n_ch,
                                int ch_first, float *X, int *fold, hipStream_t s);
hipError_t mlp_forward(const float *w, const float *x, int n, MlpAct &a, float *y, hipStream_t s);
hipError_t mlp_backward(const float *w, const float *x, int n, MlpAct &a, float *dY, float *grad,
                        hipStream_t s);
hipError_t mlp_mse(const float *yhat, const float *y, long ne, float *dY, double *loss,
                   const int *step, hipStream_t s);
hipError_t mlp_adam(float *w, const float *g, float *m, float *v, long np, int t, const int *tdev,
                    float lr0, float lr1, int steps, hipStream_t s);
hipError_t mlp_gather(const float *X, const float *Y, const int *idx, const int *step, int bs,
                      float *Xb, float *Yb, hipStream_t s);
hipError_t mlp_count(int *c, hipStream_t s);

// fixed working memory of paid_mlp_loss_grad_noalloc: per-sample buffers of
// at most kNoAllocMaxN samples (9 x 128 + 2 x 256 floats each) and the loss
// (two floats' room for one double, 256-byte aligned after the buffers)
constexpr int kNoAllocMaxN = PAID_NOALLOC_MAX_N;
constexpr long kNoAllocActFloats = (long)kNoAllocMaxN * (9 * kMlpHid + 2 * kMlpOut);
constexpr long kNoAllocFloats = kNoAllocActFloats + 64;
// device address of this device's copy of the array (call with the device current)
hipError_t noalloc_scratch_address(float **ptr);

// ------------------------------------------------------------------ contraction
hipError_t launch_contract(int n_l, int M, const double *chi, const double *VP, const double *VC,
                           const double *VD, double *dP, double *dC, double *dD, hipStream_t s);

}  // namespace paid
