// launch.h -- host-side launch interface between the C ABI (api.hip) and the
// kernel translation units.  Library-internal.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "paid.h"
#include "paid_device.h"

namespace paid {

// rule constants, filled once per device (ascending node order on [-1,1])
struct RuleConst {
  double xi[kNF];   // fine nodes
  double w2[kNF];   // fine weights
  double w1[kNCo];  // coarse weights (at fine nodes 0,2,4,6,8)
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
enum SlotState { SLOT_EMPTY = 0, SLOT_NEW = 1, SLOT_ACTIVE = 2, SLOT_DONE = 3 };

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
  long cap;                   // regions per slot
  int bmin, bmax;
  int lds_wave_doubles;       // per-wave LDS of the evaluation kernel (set at launch)
  uint64_t *code;             // [W*cap]
  double *key;                // [W*cap]
  double *Q;                  // [W*cap*MU]
  float *E;                   // [W*cap*MU] or NULL
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
  long *st_rounds, *st_splits;  // [W]
  int *st_depth;              // [W]
  // queue and global counters
  int *qhead;                 // next container to admit
  int *counters;              // [0] done, [1] not converged, [2] total work items
  long long *gstats;          // [0] rounds [1] splits [2] leaves [3] max depth
  // outputs (device)
  double *out, *err_out;      // [n_ctr][M][M]
};

hipError_t launch_admit(const Problem &p, hipStream_t s);
hipError_t launch_root(const Problem &p, hipStream_t s);
hipError_t launch_select(const Problem &p, hipStream_t s);
hipError_t launch_worklist(const Problem &p, hipStream_t s);
hipError_t launch_eval(const Problem &p, int grid, hipStream_t s);
hipError_t launch_update(const Problem &p, hipStream_t s);
hipError_t launch_finalize(const Problem &p, hipStream_t s);

// diagnostics
hipError_t launch_kernel_eval(const Entry *e, const double *tab, int ch, const double *a,
                              const double *b, int n, double *out, hipStream_t s);

hipError_t set_rule_constants(const RuleConst &rc);

}  // namespace paid
