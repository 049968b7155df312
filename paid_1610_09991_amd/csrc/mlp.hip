// mlp.hip -- the subdivision-density model of the learned seeding: model
// features of each container, and the FP32 kernels of a 7 -> 128 -> 128 ->
// 128 -> 256 perceptron (GELU on the hidden layers): forward, backward, mean
// squared error, Adam.  Training and inference share the same kernels.
//
// The model predicts, per cell of a 16 x 16 grid over the zone, log2(1 + n)
// with n the number of leaves the converged adaptive tree has in that cell.
// It works in a reduced frame: the integrand at transfer momentum l equals
// the integrand at l - 2 pi e_x moved by pi e_x in p (both energies are
// 2 pi periodic), and the dispersion is invariant under the square's point
// group, so l is reduced to [-pi, pi)^2 and then to the wedge
// 0 <= l_y <= l_x, and each container cell is read from the matching model
// cell.  None of this is in the paper; the adaptive loop of Alg. 2 still
// decides every split that the seed does not and the termination.
#include <math.h>

#include "launch.h"

namespace paid {

namespace {

constexpr int kBM = 64, kBN = 64, kBK = 16;

__device__ inline float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_d(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
         z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// Tiled FP32 product C[m][n] = sum_k A(m,k) B(k,n), A(m,k) = A[m*sam + k*sak],
// B(k,n) = B[k*sbk + n*sbn]; each of 256 threads owns a 4 x 4 block of a
// 64 x 64 tile, k runs in chunks of 16 staged through LDS and in a fixed
// order, so results do not depend on the launch.
// Epilogues: kFwd: z = C + bias[n] -> Z (if non-null), Y = act ? gelu(z) : z
//            kBwdData: Y = C * gelu'(Zp[m][n])
//            kPlain: Y = C
enum { kFwd = 0, kBwdData = 1, kPlain = 2 };

template <int EPI>
__global__ void __launch_bounds__(256)
    k_gemm(int Mr, int Nc, int K, const float *__restrict__ A, long sam, long sak,
           const float *__restrict__ B, long sbk, long sbn, const float *__restrict__ bias,
           const float *__restrict__ Zp, float *__restrict__ Z, float *__restrict__ Y, int act) {
  __shared__ float As[kBK][kBM + 4];
  __shared__ float Bs[kBK][kBN + 4];
  const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
  const int m0 = blockIdx.x * kBM, n0 = blockIdx.y * kBN;
  float acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0f;
  for (int k0 = 0; k0 < K; k0 += kBK) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int e = t + 256 * r;
      // A tile: 64 rows x 16 k; B tile: 16 k x 64 cols
      int am = e / kBK, ak = e % kBK;
      int gm = m0 + am, gk = k0 + ak;
      As[ak][am] = (gm < Mr && gk < K) ? A[(long)gm * sam + (long)gk * sak] : 0.0f;
      int bk = e / kBN, bn = e % kBN;
      int gk2 = k0 + bk, gn = n0 + bn;
      Bs[bk][bn] = (gk2 < K && gn < Nc) ? B[(long)gk2 * sbk + (long)gn * sbn] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kBK; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    int gm = m0 + ty * 4 + i;
    if (gm >= Mr) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int gn = n0 + tx * 4 + j;
      if (gn >= Nc) continue;
      long o = (long)gm * Nc + gn;
      float v = acc[i][j];
      if (EPI == kFwd) {
        v += bias[gn];
        if (Z) Z[o] = v;
        Y[o] = act ? gelu(v) : v;
      } else if (EPI == kBwdData) {
        Y[o] = v * gelu_d(Zp[o]);
      } else {
        Y[o] = v;
      }
    }
  }
}

template <int EPI>
void gemm(hipStream_t s, int Mr, int Nc, int K, const float *A, long sam, long sak, const float *B,
          long sbk, long sbn, const float *bias, const float *Zp, float *Z, float *Y, int act) {
  dim3 grid((Mr + kBM - 1) / kBM, (Nc + kBN - 1) / kBN);
  hipLaunchKernelGGL((k_gemm<EPI>), grid, dim3(256), 0, s, Mr, Nc, K, A, sam, sak, B, sbk, sbn,
                     bias, Zp, Z, Y, act);
}

// gb[o] = sum_n dZ[n][o], rows in order
__global__ void k_bias_grad(const float *dZ, int n, int no, float *gb) {
  int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= no) return;
  float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
  int r = 0;
  for (; r + 3 < n; r += 4) {
    a0 += dZ[(long)r * no + o];
    a1 += dZ[(long)(r + 1) * no + o];
    a2 += dZ[(long)(r + 2) * no + o];
    a3 += dZ[(long)(r + 3) * no + o];
  }
  for (; r < n; ++r) a0 += dZ[(long)r * no + o];
  gb[o] = (a0 + a1) + (a2 + a3);
}

// dZ = 2 (yhat - y) / (n * 256); loss = mean of squares (FP64, one block,
// fixed order), written to loss[*step] when a history is kept
__global__ void __launch_bounds__(1024) k_mse(const float *yhat, const float *y, long ne,
                                              float *dZ, double *loss, const int *step) {
  __shared__ double sh[1024];
  const int t = threadIdx.x;
  const float sc = (float)(2.0 / (double)ne);
  double a = 0.0;
  for (long e = t; e < ne; e += 1024) {
    float r = yhat[e] - y[e];
    dZ[e] = sc * r;
    a += (double)r * (double)r;
  }
  sh[t] = a;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (t < o) sh[t] += sh[t + o];
    __syncthreads();
  }
  if (t == 0 && loss) loss[step ? *step : 0] = sh[0] / (double)ne;
}

// Adam (beta1 0.9, beta2 0.999, eps 1e-8) with cosine decay of the rate from
// lr0 to lr1 over `steps`; the step t (from 1) is *tdev + 1 when tdev is set
__global__ void k_adam(float *w, const float *g, float *m, float *v, long np, int t_host,
                       const int *tdev, float lr0, float lr1, int steps) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const int t = tdev ? *tdev + 1 : t_host;
  double lr = lr0;
  if (steps > 0) lr = lr1 + 0.5 * (lr0 - lr1) * (1.0 + cos(3.14159265358979323846 * (double)(t - 1) / steps));
  const float c1 = (float)(1.0 - pow(0.9, (double)t)), c2 = (float)(1.0 - pow(0.999, (double)t));
  float gi = g[i];
  float mi = 0.9f * m[i] + 0.1f * gi;
  float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= (float)lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

__global__ void k_gather(const float *X, const float *Y, const int *idx, const int *step, int bs,
                         float *Xb, float *Yb) {
  const int r = blockIdx.x, t = threadIdx.x;
  const long src = idx[(long)(*step) * bs + r];
  if (t < kMlpIn) Xb[(long)r * kMlpIn + t] = X[src * kMlpIn + t];
  Yb[(long)r * kMlpOut + t] = Y[src * kMlpOut + t];
}

__global__ void k_count(int *c) {
  if (threadIdx.x == 0) *c += 1;
}

// features and fold of every container (same container order as the setup)
__global__ void k_seed_features(const Entry *entries, const double *q, int n_ctr, int n_q, int n_ch,
                                int ch_first, float *X, int *fold) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_ctr) return;
  int ich = c % n_ch, iq = (c / n_ch) % n_q, ip = c / (n_ch * n_q);
  const Entry e = entries[ip];
  const int ch = (n_ch == 2) ? ich : ch_first;
  const double pi = 3.14159265358979323846;
  double lx = q[2 * iq], ly = q[2 * iq + 1];
  double nx = floor((lx + pi) / (2.0 * pi)), ny = floor((ly + pi) / (2.0 * pi));
  double rx = lx - 2.0 * pi * nx, ry = ly - 2.0 * pi * ny;
  int hx = ((long long)nx) & 1, hy = ((long long)ny) & 1;
  int mx = rx < 0.0, my = ry < 0.0;
  double ax = fabs(rx), ay = fabs(ry);
  int sw = ay > ax;
  float *x = X + (long)c * kMlpIn;
  x[0] = (float)((sw ? ay : ax) / pi);
  x[1] = (float)((sw ? ax : ay) / pi);
  x[2] = (float)(e.mu / e.t);
  x[3] = (float)log10(e.T / e.t);
  x[4] = (float)(e.tp / e.t);
  x[5] = (float)log10(e.Om / e.t);
  x[6] = ch == 1 ? 1.0f : -1.0f;
  fold[c] = hx | (hy << 1) | (mx << 2) | (my << 3) | (sw << 4);
}

}  // namespace

// ------------------------------------------------------------------ host side
hipError_t launch_seed_features(const Entry *entries, const double *q, int n_ctr, int n_q, int n_ch,
                                int ch_first, float *X, int *fold, hipStream_t s) {
  if (n_ctr == 0) return hipSuccess;
  hipLaunchKernelGGL(k_seed_features, dim3((n_ctr + 255) / 256), dim3(256), 0, s, entries, q, n_ctr,
                     n_q, n_ch, ch_first, X, fold);
  return hipGetLastError();
}

// Parameter layout: per layer l, W_l [out][in] row-major, then b_l [out].
MlpLayout mlp_layout() {
  MlpLayout L;
  const int dims[5] = {kMlpIn, kMlpHid, kMlpHid, kMlpHid, kMlpOut};
  long off = 0;
  for (int l = 0; l < 4; ++l) {
    L.ni[l] = dims[l];
    L.no[l] = dims[l + 1];
    L.w[l] = off;
    off += (long)dims[l + 1] * dims[l];
    L.b[l] = off;
    off += dims[l + 1];
  }
  L.total = off;
  return L;
}

hipError_t mlp_forward(const float *w, const float *x, int n, MlpAct &a, float *y, hipStream_t s) {
  const MlpLayout L = mlp_layout();
  const float *in = x;
  for (int l = 0; l < 4; ++l) {
    const int ni = L.ni[l], no = L.no[l];
    float *Z = a.Z[l], *Y = (l == 3) ? y : a.A[l];
    gemm<kFwd>(s, n, no, ni, in, ni, 1, w + L.w[l], 1, ni, w + L.b[l], nullptr, Z, Y, l < 3);
    in = Y;
  }
  return hipGetLastError();
}

hipError_t mlp_backward(const float *w, const float *x, int n, MlpAct &a, float *dY, float *grad,
                        hipStream_t s) {
  const MlpLayout L = mlp_layout();
  // dY holds dLoss/dz of the output layer; walk the layers down
  float *d = dY;
  for (int l = 3; l >= 0; --l) {
    const int ni = L.ni[l], no = L.no[l];
    const float *Ain = (l == 0) ? x : a.A[l - 1];
    // gW[o][i] = sum_r d[r][o] Ain[r][i]
    gemm<kPlain>(s, no, ni, n, d, 1, no, Ain, ni, 1, nullptr, nullptr, nullptr, grad + L.w[l], 0);
    hipLaunchKernelGGL(k_bias_grad, dim3((no + 255) / 256), dim3(256), 0, s, d, n, no,
                       grad + L.b[l]);
    if (l > 0) {
      // d_prev[r][i] = (sum_o d[r][o] W[o][i]) * gelu'(Z_{l-1}[r][i])
      float *dn = a.D[l - 1];
      gemm<kBwdData>(s, n, ni, no, d, no, 1, w + L.w[l], ni, 1, nullptr, a.Z[l - 1], nullptr, dn, 0);
      d = dn;
    }
  }
  return hipGetLastError();
}

hipError_t mlp_mse(const float *yhat, const float *y, long ne, float *dY, double *loss,
                   const int *step, hipStream_t s) {
  hipLaunchKernelGGL(k_mse, dim3(1), dim3(1024), 0, s, yhat, y, ne, dY, loss, step);
  return hipGetLastError();
}

hipError_t mlp_adam(float *w, const float *g, float *m, float *v, long np, int t, const int *tdev,
                    float lr0, float lr1, int steps, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, w, g, m, v, np, t,
                     tdev, lr0, lr1, steps);
  return hipGetLastError();
}

hipError_t mlp_gather(const float *X, const float *Y, const int *idx, const int *step, int bs,
                      float *Xb, float *Yb, hipStream_t s) {
  hipLaunchKernelGGL(k_gather, dim3(bs), dim3(kMlpOut), 0, s, X, Y, idx, step, bs, Xb, Yb);
  return hipGetLastError();
}

hipError_t mlp_count(int *c, hipStream_t s) {
  hipLaunchKernelGGL(k_count, dim3(1), dim3(64), 0, s, c);
  return hipGetLastError();
}

// ------------------------------------------------------------------ fixed working memory
// Working memory of the loss-and-gradient entry point that allocates
// nothing: the per-sample buffers of kNoAllocMaxN samples (pre-activations,
// activations, deltas, outputs, output deltas) and the FP64 loss.  Every
// element a call reads is written earlier in the same call, so nothing has
// to start at zero.  Each device holds its own copy of the array at its own
// address; host code must use that address (from hipGetSymbolAddress), never
// the array's name, which on the host is only a stand-in.
static __device__ __align__(256) float scratch[kNoAllocFloats];

hipError_t noalloc_scratch_address(float **ptr) {
  void *p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  *ptr = static_cast<float *>(p);
  return hipSuccess;
}

}  // namespace paid
