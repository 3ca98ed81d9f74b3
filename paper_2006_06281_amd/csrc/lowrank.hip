// CPD-L: the original M-step (eq. 21) with Phi replaced by its rank-K
// approximation Phi~ = U L U^T (eq. 19), the fourth method of the paper's
// runtime comparison (Section IV-B).  The paper prints no update for it; the
// matrix inversion lemma gives one with a K x K system per iteration.  With
// w_m = P1_m / (lambda sigma^2) (the diagonal of A^-1, A = lambda sigma^2
// d(P1)^-1) and t = w o (d(P1)^-1 PY - X) = w o (Yt - X):
//   S = L^-1 + U^T d(w) U,   S z = U^T t,
//   W = t - w o (U z),       Xt_new = X + Phi~ W = X + U z.
// Eigenpairs with lam <= 0 carry no part of Phi~ and are dropped (their row
// and column of S become the identity, their q entry 0).
//
// FP64 throughout (U64): S's diagonal spans 1/lam_1 .. 1/lam_K.
//   k_lr_prep    t (M x 4) and Uw = d(w) U (M x K)
//   gram         S = U^T Uw (eigen-prep's fixed-order Gram kernels)
//   k_lr_qpart   q partials over row chunks: U^T t
//   k_lr_system  S += L^-1, q = sum of partials, dropped pairs
//   Cholesky     the blocked factorisation and solves of the original method
//   k_lr_apply   Xt_new = X + U z, W = t - w o U z (16 lanes per row)
#include "common.hpp"
#include "kernels.hpp"
#include "lowrank.hpp"
#include "eig.hpp"
#include "orig.hpp"

namespace fcpd {

namespace {
constexpr int kQRows = 1024;  // rows per q partial
size_t al(size_t b) { return (b + 255) & ~(size_t)255; }
}  // namespace

LowRankLayout lowrank_layout(int M, int K, size_t start) {
  LowRankLayout L;
  size_t off = start;
  auto take = [&](size_t b) {
    const size_t o = off;
    off += al(b);
    return o;
  };
  const int nblk = (K + kCholBlock - 1) / kCholBlock;
  L.t = take((size_t)M * 4 * sizeof(double));
  L.Uw = take((size_t)M * K * sizeof(double));
  L.S = take((size_t)K * K * sizeof(double));
  L.gpart = take(gram_partial_doubles(M, K) * sizeof(double));
  L.Linv = take((size_t)nblk * kCholBlock * kCholBlock * sizeof(double));
  L.pan = take((size_t)K * kCholPanel * sizeof(double));
  L.q = take((size_t)K * 4 * sizeof(double));
  L.qchunks = (M + kQRows - 1) / kQRows;
  L.qpart = take((size_t)L.qchunks * K * 4 * sizeof(double));
  L.end = off;
  return L;
}

template <typename T>
__global__ __launch_bounds__(256) void k_lr_prep(const P4<T>* __restrict__ X,
                                                 const P4<T>* __restrict__ Yt,
                                                 const T* __restrict__ P1,
                                                 const double* __restrict__ U64, int M, int K,
                                                 double lmbda, DevScalars* __restrict__ sc,
                                                 int gate, double* __restrict__ t,
                                                 double* __restrict__ Uw) {
  if (gate && sc->done) return;
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i == 0) sc->chol_fail = 0;  // this iteration's factorisation starts clean
  if (i >= (size_t)M * K) return;
  const int m = (int)(i / K), k = (int)(i % K);
  const double w = fmax((double)P1[m], 1e-20) / (lmbda * sc->sigma2);
  Uw[i] = w * U64[i];
  if (k == 0) {
    const P4<T> y = Yt[m], x = X[m];
    double* tm = t + (size_t)m * 4;
    tm[0] = w * ((double)y.x - (double)x.x);
    tm[1] = w * ((double)y.y - (double)x.y);
    tm[2] = w * ((double)y.z - (double)x.z);
    tm[3] = 0.0;
  }
}

// qpart[chunk][k][d] = sum over the chunk's rows of U[m][k] t[m][d]
__global__ __launch_bounds__(256) void k_lr_qpart(const double* __restrict__ U64,
                                                  const double* __restrict__ t, int M, int K,
                                                  const DevScalars* __restrict__ sc, int gate,
                                                  double* __restrict__ qpart) {
  if (gate && sc->done) return;
  const int c = blockIdx.x;
  const int m0 = c * kQRows, m1 = min(M, m0 + kQRows);
  for (int k = threadIdx.x; k < K; k += 256) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int m = m0; m < m1; ++m) {
      const double u = U64[(size_t)m * K + k];
      const double* tm = t + (size_t)m * 4;
      a0 = fma(u, tm[0], a0);
      a1 = fma(u, tm[1], a1);
      a2 = fma(u, tm[2], a2);
    }
    double* o = qpart + ((size_t)c * K + k) * 4;
    o[0] = a0;
    o[1] = a1;
    o[2] = a2;
    o[3] = 0.0;
  }
}

// S += L^-1 on kept pairs, identity rows/columns for dropped ones; q = sum
// of the partials (0 for dropped pairs).  One thread per k; the dropped
// pairs' off-diagonal entries are cleared by the threads of their row.
__global__ __launch_bounds__(256) void k_lr_system(double* __restrict__ S,
                                                   const double* __restrict__ lam, int K,
                                                   const double* __restrict__ qpart, int chunks,
                                                   const DevScalars* __restrict__ sc, int gate,
                                                   double* __restrict__ q) {
  if (gate && sc->done) return;
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= K) return;
  const bool keep = lam[k] > 0.0;
  double* Sk = S + (size_t)k * K;
  if (keep) {
    Sk[k] += 1.0 / lam[k];
  } else {
    for (int j = 0; j < K; ++j) Sk[j] = 0.0;
    Sk[k] = 1.0;
  }
  for (int j = 0; j < K; ++j)  // column k of a dropped pair j is cleared by row j's thread
    if (!(lam[j] > 0.0) && j != k) Sk[j] = 0.0;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  if (keep)
    for (int c = 0; c < chunks; ++c) {
      const double* o = qpart + ((size_t)c * K + k) * 4;
      a0 += o[0];
      a1 += o[1];
      a2 += o[2];
    }
  double* qk = q + (size_t)k * 4;
  qk[0] = a0;
  qk[1] = a1;
  qk[2] = a2;
  qk[3] = 0.0;
}

// Xt_new = X + U z, W = t - w o U z; 16 lanes per row (z, K x 4 doubles,
// is read through the cache: every row reads all of it).
template <typename T>
__global__ __launch_bounds__(256) void k_lr_apply(const P4<T>* __restrict__ X,
                                                  const T* __restrict__ P1,
                                                  const double* __restrict__ U64,
                                                  const double* __restrict__ t,
                                                  const double* __restrict__ sz, int M, int K,
                                                  double lmbda, DevScalars* __restrict__ sc,
                                                  int gate, P4<T>* __restrict__ Xnew,
                                                  P4<T>* __restrict__ W) {
  if (gate && sc->done) return;
  if (sc->chol_fail) {  // S was not positive definite: report, keep the last iterate
    if (blockIdx.x == 0 && threadIdx.x == 0) sc->nonfinite = 2;
    return;
  }
  const int l16 = threadIdx.x & 15;
  const int m = blockIdx.x * 16 + (threadIdx.x >> 4);
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  if (m < M) {
    const double* u = U64 + (size_t)m * K;
    for (int k = l16; k < K; k += 16) {
      const double v = u[k];
      s0 = fma(v, sz[4 * k], s0);
      s1 = fma(v, sz[4 * k + 1], s1);
      s2 = fma(v, sz[4 * k + 2], s2);
    }
  }
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) {
    s0 += __shfl_xor(s0, o, 16);
    s1 += __shfl_xor(s1, o, 16);
    s2 += __shfl_xor(s2, o, 16);
  }
  if (m < M && l16 == 0) {
    const double w = fmax((double)P1[m], 1e-20) / (lmbda * sc->sigma2);
    const P4<T> x = X[m];
    const double* tm = t + (size_t)m * 4;
    Xnew[m] = P4<T>{(T)((double)x.x + s0), (T)((double)x.y + s1), (T)((double)x.z + s2), (T)0};
    W[m] = P4<T>{(T)(tm[0] - w * s0), (T)(tm[1] - w * s1), (T)(tm[2] - w * s2), (T)0};
  }
}

template <typename T> void lowrank_mstep_launch(const LowRankArgs<T>& a, hipStream_t st) {
  const LowRankLayout& L = *a.L;
  auto at = [&](size_t off) { return reinterpret_cast<double*>(a.ws + off); };
  double *t = at(L.t), *Uw = at(L.Uw), *S = at(L.S), *q = at(L.q), *qpart = at(L.qpart);
  const int g = a.gate;
  const int* done = g ? &a.sc->done : nullptr;
  const size_t MK = (size_t)a.M * a.K;
  hipLaunchKernelGGL(k_lr_prep<T>, dim3((unsigned)((MK + 255) / 256)), dim3(256), 0, st, a.X,
                     a.Yt, a.P1, a.U64, a.M, a.K, a.lmbda, a.sc, g, t, Uw);
  gram_sym_launch(a.U64, Uw, a.M, a.K, S, at(L.gpart), st);
  hipLaunchKernelGGL(k_lr_qpart, dim3(L.qchunks), dim3(256), 0, st, a.U64, t, a.M, a.K, a.sc, g,
                     qpart);
  hipLaunchKernelGGL(k_lr_system, dim3((a.K + 255) / 256), dim3(256), 0, st, S, a.lam, a.K, qpart,
                     L.qchunks, a.sc, g, q);
  chol_blocked_launch(S, a.K, a.K, at(L.Linv), at(L.pan), &a.sc->chol_fail, done, st);
  chol_solve_launch(S, a.K, a.K, at(L.Linv), q, &a.sc->chol_fail, done, st);
  hipLaunchKernelGGL(k_lr_apply<T>, dim3((a.M + 15) / 16), dim3(256), 0, st, a.X, a.P1, a.U64, t,
                     q, a.M, a.K, a.lmbda, a.sc, g, a.Xnew, a.W);
}

template void lowrank_mstep_launch<float>(const LowRankArgs<float>&, hipStream_t);
template void lowrank_mstep_launch<double>(const LowRankArgs<double>&, hipStream_t);

}  // namespace fcpd
