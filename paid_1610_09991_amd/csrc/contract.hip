// contract.hip -- the contraction beside the integration (Sec. 2, Eqs.
// matmul-P, matmul-C, matmul-D): per transfer momentum l, with the bubbles
// chi^pp(l), chi^ph(l) of the adaptive integration and the couplings
// V^P(l), V^C(l), V^D(l) (M x M over form factors),
//   dP = V^P chi^pp V^P,
//   dC = - V^C chi^ph V^C,
//   dD = 2 V^D chi^ph V^D - V^C chi^ph V^D - V^D chi^ph V^C.
// One wave per l.  Matrices are staged in LDS zero-padded to 32 x 32 and
// multiplied on the FP64 matrix cores (16 x 16 x 4 tiles); dD is formed as
// (2 V^D - V^C) (chi^ph V^D) - V^D (chi^ph V^C), reusing chi^ph V^C from dC.
#include "launch.h"

namespace paid {

namespace {

constexpr int kCM = 32;                 // padded order
constexpr int kCLd = kCM + 1;           // leading dimension in LDS (bank spread)
constexpr int kCMat = kCM * kCLd;       // doubles per staged matrix
constexpr int kCBufs = 6;               // staged matrices per wave

typedef double c4 __attribute__((ext_vector_type(4)));

__device__ inline void cwave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// X (LDS, padded) <- src [M][M] (global), zero outside M x M
__device__ inline void stage(double *X, const double *src, int M) {
  const int lane = threadIdx.x & 63;
  for (int e = lane; e < kCM * kCM; e += 64) {
    const int i = e / kCM, j = e % kCM;
    X[i * kCLd + j] = (i < M && j < M) ? src[i * M + j] : 0.0;
  }
}

// C = alpha A B + beta C on padded 32 x 32 LDS matrices; tiles beyond the
// order M (nt = 1 or 2 tiles per side) are skipped.
__device__ void mm(const double *A, const double *B, double *C, int nt, double alpha, double beta) {
  const int lane = threadIdx.x & 63, m = lane & 15, kk = lane >> 4;
  c4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = c4{0.0, 0.0, 0.0, 0.0};
  const int nk = 4 * nt;  // k-steps of 4 over 16 nt
  for (int kb = 0; kb < nk; ++kb) {
    const int k = 4 * kb + kk;
#pragma unroll
    for (int tr = 0; tr < 2; ++tr) {
      if (tr >= nt) continue;
      const double a = A[(16 * tr + m) * kCLd + k];
#pragma unroll
      for (int tc = 0; tc < 2; ++tc) {
        if (tc >= nt) continue;
        const double b = B[k * kCLd + 16 * tc + m];
        acc[2 * tr + tc] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[2 * tr + tc], 0, 0, 0);
      }
    }
  }
  cwave_sync();
  // f64 16x16x4 result: row = 4 r + lane >> 4, col = lane & 15
#pragma unroll
  for (int tr = 0; tr < 2; ++tr)
#pragma unroll
    for (int tc = 0; tc < 2; ++tc) {
      if (tr >= nt || tc >= nt) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double *c = &C[(16 * tr + 4 * r + kk) * kCLd + 16 * tc + m];
        *c = alpha * acc[2 * tr + tc][r] + (beta != 0.0 ? beta * *c : 0.0);
      }
    }
  cwave_sync();
}

__device__ inline void unstage(double *dst, const double *X, int M) {
  const int lane = threadIdx.x & 63;
  for (int e = lane; e < M * M; e += 64) dst[e] = X[(e / M) * kCLd + e % M];
}

__global__ void __launch_bounds__(256) k_contract(int n_l, int M, const double *chi,
                                                 const double *VP, const double *VC,
                                                 const double *VD, double *dP, double *dC,
                                                 double *dD) {
  extern __shared__ double craw[];
  const int wv = threadIdx.x >> 6;
  const long l = (long)blockIdx.x * (blockDim.x >> 6) + wv;
  if (l >= n_l) return;  // whole waves only: nothing below synchronises the workgroup
  double *X = craw + (size_t)wv * kCBufs * kCMat;
  double *Vp = X, *Ch = X + kCMat, *Vc = X + 2 * kCMat, *T1 = X + 3 * kCMat,
         *T2 = X + 4 * kCMat, *T3 = X + 5 * kCMat;
  const int nt = M > 16 ? 2 : 1;
  const long mm2 = (long)M * M;
  const double *cpp = chi + (2 * l) * mm2, *cph = chi + (2 * l + 1) * mm2;
  // dP = V^P (chi^pp V^P)
  stage(Vp, VP + l * mm2, M);
  stage(Ch, cpp, M);
  cwave_sync();
  mm(Ch, Vp, T1, nt, 1.0, 0.0);
  mm(Vp, T1, T3, nt, 1.0, 0.0);
  unstage(dP + l * mm2, T3, M);
  // dC = -V^C (chi^ph V^C); keep T2 = chi^ph V^C
  stage(Vc, VC + l * mm2, M);
  stage(Ch, cph, M);
  cwave_sync();
  mm(Ch, Vc, T2, nt, 1.0, 0.0);
  mm(Vc, T2, T3, nt, -1.0, 0.0);
  unstage(dC + l * mm2, T3, M);
  // dD = (2 V^D - V^C) (chi^ph V^D) - V^D (chi^ph V^C)
  stage(Vp, VD + l * mm2, M);  // Vp now holds V^D
  cwave_sync();
  mm(Ch, Vp, T1, nt, 1.0, 0.0);  // T1 = chi^ph V^D
  {
    const int lane = threadIdx.x & 63;
    for (int e = lane; e < kCM * kCM; e += 64) {
      const int i = e / kCM, j = e % kCM;
      Vc[i * kCLd + j] = 2.0 * Vp[i * kCLd + j] - Vc[i * kCLd + j];
    }
  }
  cwave_sync();
  mm(Vc, T1, T3, nt, 1.0, 0.0);
  mm(Vp, T2, T3, nt, -1.0, 1.0);
  unstage(dD + l * mm2, T3, M);
}

}  // namespace

hipError_t launch_contract(int n_l, int M, const double *chi, const double *VP, const double *VC,
                           const double *VD, double *dP, double *dC, double *dD, hipStream_t s) {
  if (n_l <= 0) return hipSuccess;
  const int waves = 1;  // 6 staged matrices = 50.7 KB of LDS per workgroup
  const size_t sh = sizeof(double) * (size_t)waves * kCBufs * kCMat;
  hipLaunchKernelGGL(k_contract, dim3((n_l + waves - 1) / waves), dim3(64 * waves), sh, s, n_l, M,
                     chi, VP, VC, VD, dP, dC, dD);
  return hipGetLastError();
}

}  // namespace paid
