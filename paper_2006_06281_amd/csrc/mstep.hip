// Fast CPD M-step (Section III, eq. 17 and its top-K form eq. 20), the
// sigma^2 update (eq. 18 with the row-normalised posterior) and the small
// set-up kernels.
//
// With U (M x K) and Lam precomputed, one M-step is
//   T   = U^T (Yt - X)                         K x D, reduction over M
//   g_k = 1 / (max(lam_k, 0) + lambda sigma^2),  h_k = max(lam_k, 0) g_k
//   W   = U (g o T),   Xt_new = X + U (h o T)  ( = X + Phi W for exact U)
// Both products stream U once; at D = 3 they run at ~2 flop/byte, so they are
// bandwidth kernels: U is read with full-row coalesced loads and the K x D
// factors are tiny.
#include "common.hpp"
#include "kernels.hpp"

namespace fcpd {

// ---------------------------------------------------------------- T = U^T R
// Block (row chunk, k-group of 256*KT): thread t accumulates
// sum_m U[m][k] R_m for k = k0 + t + 256 j, j < KT; R_m = Yt_m - X_m is uniform
// across the block (scalar loads).  U rows are read with coalesced loads.
template <typename T, int KT>
__device__ __forceinline__ void tpart_body(const P4<T>* __restrict__ X,
                                               const P4<T>* __restrict__ Yt,
                                               const T* __restrict__ U, int M, int K, int rows,
                                               const DevScalars* __restrict__ sc,
                                               T* __restrict__ tpart, int gate, int bx_, int by_, int gx_) {
  if (gate && sc->done) return;
  const int k0 = by_ * 256 * KT + threadIdx.x;
  const int m0 = bx_ * rows;
  const int m1 = min(M, m0 + rows);
  T ax[KT], ay[KT], az[KT];
#pragma unroll
  for (int j = 0; j < KT; ++j) ax[j] = ay[j] = az[j] = (T)0;
#pragma unroll 4
  for (int m = m0; m < m1; ++m) {
    const P4<T> y = Yt[m], x = X[m];
    const T rx = y.x - x.x, ry = y.y - x.y, rz = y.z - x.z;
    const T* u = U + (size_t)m * K;
#pragma unroll
    for (int j = 0; j < KT; ++j) {
      const int k = k0 + 256 * j;
      const T uk = k < K ? u[k] : (T)0;
      ax[j] = fma(uk, rx, ax[j]);
      ay[j] = fma(uk, ry, ay[j]);
      az[j] = fma(uk, rz, az[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < KT; ++j) {
    const int k = k0 + 256 * j;
    if (k < K) {
      T* o = tpart + ((size_t)bx_ * K + k) * 4;
      o[0] = ax[j];
      o[1] = ay[j];
      o[2] = az[j];
      o[3] = (T)0;
    }
  }
}

template <typename T, int KT>
__global__ __launch_bounds__(256) void k_tpart(const P4<T>* __restrict__ X,
                                               const P4<T>* __restrict__ Yt,
                                               const T* __restrict__ U, int M, int K, int rows,
                                               const DevScalars* __restrict__ sc,
                                               T* __restrict__ tpart, int gate) {
  tpart_body<T, KT>(X, Yt, U, M, K, rows, sc, tpart, gate, blockIdx.x, blockIdx.y, gridDim.x);
}

// One wave per eigenpair k: T_k = sum over row chunks (fixed order: lane
// strides, then a fixed butterfly), GT_k = g_k T_k, HT_k = h_k T_k with
// g_k = 1/(max(lam_k, 0) + lambda sigma^2) and h_k = max(lam_k, 0) g_k.
template <typename T>
__device__ __forceinline__ void tmerge_body(const T* __restrict__ tpart, int chunks,
                                               const double* __restrict__ lam, int K,
                                               double lmbda, const DevScalars* __restrict__ sc,
                                               P4<T>* __restrict__ GT, P4<T>* __restrict__ HT,
                                               int gate, int bx_, int by_, int gx_) {
  if (gate && sc->done) return;
  const int k = bx_;
  const int lane = threadIdx.x;
  T tx = 0, ty = 0, tz = 0;
  for (int c = lane; c < chunks; c += 64) {
    const T* p = tpart + ((size_t)c * K + k) * 4;
    tx += p[0];
    ty += p[1];
    tz += p[2];
  }
  tx = wave_sum(tx);
  ty = wave_sum(ty);
  tz = wave_sum(tz);
  if (lane == 0) {
    const double lp = fmax(lam[k], 0.0);
    const double g = 1.0 / (lp + lmbda * sc->sigma2);
    const double h = lp * g;
    GT[k] = P4<T>{(T)(g * tx), (T)(g * ty), (T)(g * tz), (T)0};
    HT[k] = P4<T>{(T)(h * tx), (T)(h * ty), (T)(h * tz), (T)0};
  }
}

template <typename T>
__global__ __launch_bounds__(64) void k_tmerge(const T* __restrict__ tpart, int chunks,
                                               const double* __restrict__ lam, int K,
                                               double lmbda, const DevScalars* __restrict__ sc,
                                               P4<T>* __restrict__ GT, P4<T>* __restrict__ HT,
                                               int gate) {
  tmerge_body<T>(tpart, chunks, lam, K, lmbda, sc, GT, HT, gate, blockIdx.x, blockIdx.y, gridDim.x);
}

// Xnew_m = X_m + U_m . HT, W_m = U_m . GT.  Sixteen lanes per row (four rows
// per wave), 64 rows per block; GT and HT staged in LDS when they fit.
template <typename T, bool LDS>
__device__ __forceinline__ void apply_body(const P4<T>* __restrict__ X,
                                               const T* __restrict__ U,
                                               const P4<T>* __restrict__ GTg,
                                               const P4<T>* __restrict__ HTg, int M, int K,
                                               const DevScalars* __restrict__ sc,
                                               P4<T>* __restrict__ Xnew, P4<T>* __restrict__ W,
                                               int gate, int bx_, int by_, int gx_) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (gate && sc->done) return;
  const P4<T>* GT = GTg;
  const P4<T>* HT = HTg;
  if (LDS) {
    P4<T>* sG = reinterpret_cast<P4<T>*>(smem);
    P4<T>* sH = sG + K;
    for (int k = threadIdx.x; k < K; k += 256) {
      sG[k] = GTg[k];
      sH[k] = HTg[k];
    }
    __syncthreads();
    GT = sG;
    HT = sH;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int sub = lane >> 4, l16 = lane & 15;
  for (int it = 0; it < 4; ++it) {
    const int m = bx_ * 64 + wave * 16 + it * 4 + sub;
    T hx = 0, hy = 0, hz = 0, gx = 0, gy = 0, gz = 0;
    if (m < M) {
      const T* u = U + (size_t)m * K;
      for (int k = l16; k < K; k += 16) {
        const T uk = u[k];
        const P4<T> h = HT[k], g = GT[k];
        hx = fma(uk, h.x, hx);
        hy = fma(uk, h.y, hy);
        hz = fma(uk, h.z, hz);
        gx = fma(uk, g.x, gx);
        gy = fma(uk, g.y, gy);
        gz = fma(uk, g.z, gz);
      }
    }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) {
      hx += __shfl_xor(hx, o, 16);
      hy += __shfl_xor(hy, o, 16);
      hz += __shfl_xor(hz, o, 16);
      gx += __shfl_xor(gx, o, 16);
      gy += __shfl_xor(gy, o, 16);
      gz += __shfl_xor(gz, o, 16);
    }
    if (l16 == 0 && m < M) {
      const P4<T> x = X[m];
      Xnew[m] = P4<T>{x.x + hx, x.y + hy, x.z + hz, (T)0};
      W[m] = P4<T>{gx, gy, gz, (T)0};
    }
  }
}

template <typename T, bool LDS>
__global__ __launch_bounds__(256) void k_apply(const P4<T>* __restrict__ X,
                                               const T* __restrict__ U,
                                               const P4<T>* __restrict__ GTg,
                                               const P4<T>* __restrict__ HTg, int M, int K,
                                               const DevScalars* __restrict__ sc,
                                               P4<T>* __restrict__ Xnew, P4<T>* __restrict__ W,
                                               int gate) {
  apply_body<T, LDS>(X, U, GTg, HTg, M, K, sc, Xnew, W, gate, blockIdx.x, blockIdx.y, gridDim.x);
}

// The same two products with 16-byte loads of U, for FP32 with K a multiple
// of 4 (rows of U then start 16-byte aligned) and K <= 1024.
//
// T: the block's threads split into RP = 256 / (K/4) row lanes of K/4
// threads; thread (r, q) accumulates k = 4q..4q+3 over rows m = m0 + r,
// m0 + r + RP, ...; the row lanes are summed in LDS in a fixed order.
__device__ __forceinline__ void tpart4_body(const P4<float>* __restrict__ X,
                                                const P4<float>* __restrict__ Yt,
                                                const float* __restrict__ U, int M, int K,
                                                int rows, const DevScalars* __restrict__ sc,
                                                float* __restrict__ tpart, int gate, int bx_) {
  __shared__ float red[256 * 12];
  if (gate && sc->done) return;
  const int KQ = K >> 2, RP = 256 / KQ;
  const int r = threadIdx.x / KQ, q = threadIdx.x - r * KQ;
  const float4* U4 = reinterpret_cast<const float4*>(U);
  float a[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) a[i] = 0.f;
  const int m0 = bx_ * rows, m1 = min(M, m0 + rows);
  if (r < RP) {
#pragma unroll 4
    for (int m = m0 + r; m < m1; m += RP) {
      const P4<float> y = Yt[m], x = X[m];
      const float rx = y.x - x.x, ry = y.y - x.y, rz = y.z - x.z;
      const float4 u = U4[(size_t)m * KQ + q];
      const float uk[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        a[3 * j + 0] = fmaf(uk[j], rx, a[3 * j + 0]);
        a[3 * j + 1] = fmaf(uk[j], ry, a[3 * j + 1]);
        a[3 * j + 2] = fmaf(uk[j], rz, a[3 * j + 2]);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 12; ++i) red[threadIdx.x * 12 + i] = a[i];
  __syncthreads();
  if (threadIdx.x < KQ) {
#pragma unroll
    for (int i = 0; i < 12; ++i) {
      float t = 0.f;
      for (int rr = 0; rr < RP; ++rr) t += red[(rr * KQ + q) * 12 + i];
      a[i] = t;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float* o = tpart + ((size_t)bx_ * K + 4 * q + j) * 4;
      *reinterpret_cast<float4*>(o) = make_float4(a[3 * j], a[3 * j + 1], a[3 * j + 2], 0.f);
    }
  }
}

__global__ __launch_bounds__(256) void k_tpart4(const P4<float>* __restrict__ X,
                                                const P4<float>* __restrict__ Yt,
                                                const float* __restrict__ U, int M, int K,
                                                int rows, const DevScalars* __restrict__ sc,
                                                float* __restrict__ tpart, int gate) {
  tpart4_body(X, Yt, U, M, K, rows, sc, tpart, gate, blockIdx.x);
}

// Xnew_m = X_m + U_m . HT, W_m = U_m . GT: sixteen lanes per row, four rows
// per wave in flight together, 64 rows per block.  GT and HT sit in LDS as
// six float arrays, so the four factors of a lane's float4 of U are 16-byte
// reads that fall on distinct banks across the sixteen lanes.
__device__ __forceinline__ void apply4_body(const P4<float>* __restrict__ X,
                                                const float* __restrict__ U,
                                                const P4<float>* __restrict__ GTg,
                                                const P4<float>* __restrict__ HTg, int M, int K,
                                                const DevScalars* __restrict__ sc,
                                                P4<float>* __restrict__ Xnew,
                                                P4<float>* __restrict__ W, int gate,
                                                P4<float>* __restrict__ Xt,
                                                const P4<float>* __restrict__ Yt,
                                                const float* __restrict__ tbar,
                                                double* __restrict__ sigpart, int bx_) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double sh[16];
  if (gate && sc->done) return;
  float* f = reinterpret_cast<float*>(smem);  // gx gy gz hx hy hz, K each
  for (int k = threadIdx.x; k < K; k += 256) {
    const P4<float> g = GTg[k], h = HTg[k];
    f[k] = g.x;
    f[K + k] = g.y;
    f[2 * K + k] = g.z;
    f[3 * K + k] = h.x;
    f[4 * K + k] = h.y;
    f[5 * K + k] = h.z;
  }
  __syncthreads();
  const float4* F4 = reinterpret_cast<const float4*>(f);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int sub = lane >> 4, l16 = lane & 15;
  const int KQ = K >> 2;
  const float4* U4 = reinterpret_cast<const float4*>(U);
  float acc[4][6];
#pragma unroll
  for (int it = 0; it < 4; ++it) {
    const int m = bx_ * 64 + wave * 16 + it * 4 + sub;
#pragma unroll
    for (int c = 0; c < 6; ++c) acc[it][c] = 0.f;
    if (m < M) {
      const float4* u = U4 + (size_t)m * KQ;
      for (int qq = l16; qq < KQ; qq += 16) {
        const float4 v = u[qq];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          const float4 w = F4[c * KQ + qq];
          acc[it][c] = fmaf(v.x, w.x, fmaf(v.y, w.y, fmaf(v.z, w.z, fmaf(v.w, w.w, acc[it][c]))));
        }
      }
    }
  }
  const bool retire = sigpart && !sc->nonfinite;  // a failed M-step keeps the iterate
  double v = 0.0;
#pragma unroll
  for (int it = 0; it < 4; ++it) {
#pragma unroll
    for (int c = 0; c < 6; ++c)
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) acc[it][c] += __shfl_xor(acc[it][c], o, 16);
    const int m = bx_ * 64 + wave * 16 + it * 4 + sub;
    if (l16 == 0 && m < M) {
      const P4<float> x = X[m];
      const P4<float> a{x.x + acc[it][3], x.y + acc[it][4], x.z + acc[it][5], 0.f};
      Xnew[m] = a;
      W[m] = P4<float>{acc[it][0], acc[it][1], acc[it][2], 0.f};
      if (sigpart) {  // the row's sigma^2 term (sig_part_body) and the retirement
        const P4<float> b = Xt[m], y = Yt[m];
        const double bx = b.x, by = b.y, bz = b.z;
        const double ex = bx - a.x, ey = by - a.y, ez = bz - a.z;
        const double cross = ((double)y.x - bx) * ex + ((double)y.y - by) * ey +
                             ((double)y.z - bz) * ez;
        v += (double)tbar[m] + 2.0 * cross + ex * ex + ey * ey + ez * ez;
        if (retire) Xt[m] = a;
      }
    }
  }
  if (sigpart) {
    const double s1 = block_sum_d(v, sh);
    if (threadIdx.x == 0) {
      sigpart[2 * bx_] = s1;
      sigpart[2 * bx_ + 1] = 0.0;
    }
  }
}

__global__ __launch_bounds__(256) void k_apply4(const P4<float>* __restrict__ X,
                                                const float* __restrict__ U,
                                                const P4<float>* __restrict__ GTg,
                                                const P4<float>* __restrict__ HTg, int M, int K,
                                                const DevScalars* __restrict__ sc,
                                                P4<float>* __restrict__ Xnew,
                                                P4<float>* __restrict__ W, int gate,
                                                P4<float>* __restrict__ Xt,
                                                const P4<float>* __restrict__ Yt,
                                                const float* __restrict__ tbar,
                                                double* __restrict__ sigpart) {
  apply4_body(X, U, GTg, HTg, M, K, sc, Xnew, W, gate, Xt, Yt, tbar, sigpart, blockIdx.x);
}

// T_k over the row chunks with 16-byte loads: one block of 256 threads per
// k (lane-strided chunk sums, then waves, in a fixed order), then GT_k, HT_k
// as in tmerge_body.
__global__ __launch_bounds__(256) void k_tmerge4(const float* __restrict__ tpart, int chunks,
                                                 const double* __restrict__ lam, int K,
                                                 double lmbda, const DevScalars* __restrict__ sc,
                                                 P4<float>* __restrict__ GT,
                                                 P4<float>* __restrict__ HT, int gate) {
  __shared__ float sh[4][3];
  if (gate && sc->done) return;
  const int k = blockIdx.x, lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  float tx = 0.f, ty = 0.f, tz = 0.f;
  for (int c = threadIdx.x; c < chunks; c += 256) {
    const float4 v = *reinterpret_cast<const float4*>(tpart + ((size_t)c * K + k) * 4);
    tx += v.x;
    ty += v.y;
    tz += v.z;
  }
  tx = wave_sum(tx);
  ty = wave_sum(ty);
  tz = wave_sum(tz);
  if (lane == 0) {
    sh[wid][0] = tx;
    sh[wid][1] = ty;
    sh[wid][2] = tz;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    tx = (sh[0][0] + sh[1][0]) + (sh[2][0] + sh[3][0]);
    ty = (sh[0][1] + sh[1][1]) + (sh[2][1] + sh[3][1]);
    tz = (sh[0][2] + sh[1][2]) + (sh[2][2] + sh[3][2]);
    const double lp = fmax(lam[k], 0.0);
    const double g = 1.0 / (lp + lmbda * sc->sigma2);
    const double h = lp * g;
    GT[k] = P4<float>{(float)(g * tx), (float)(g * ty), (float)(g * tz), 0.f};
    HT[k] = P4<float>{(float)(h * tx), (float)(h * ty), (float)(h * tz), 0.f};
  }
}

// rows per partial of T = U^T R: 128 (391 blocks at 50k) measured 3.4 us
// faster per M-step than 64 (fewer partials for the merge) and 1 us faster
// than 256 (too few blocks to keep every CU streaming U)
constexpr int kTRows = 128;
constexpr size_t kApplyLdsBytes = 65536;

template <typename T> int fast_mstep_chunks(int M, int* rows_per_chunk) {
  *rows_per_chunk = kTRows;
  return (M + kTRows - 1) / kTRows;
}

template <typename T> bool fast_mstep_vec4(int K) {
  return sizeof(T) == 4 && K % 4 == 0 && K <= 1024;
}

template <typename T> int fast_mstep_launch(const FastMArgs<T>& a, hipStream_t st) {
  if (fast_mstep_vec4<T>(a.K)) {
    const float* U = reinterpret_cast<const float*>(a.U);
    const P4<float>* X = reinterpret_cast<const P4<float>*>(a.X);
    hipLaunchKernelGGL(k_tpart4, dim3(a.chunks), dim3(256), 0, st, X,
                       reinterpret_cast<const P4<float>*>(a.Yt), U, a.M, a.K, a.rows_per_chunk,
                       a.sc, reinterpret_cast<float*>(a.tpart), a.gate);
    hipLaunchKernelGGL(k_tmerge4, dim3(a.K), dim3(256), 0, st,
                       reinterpret_cast<const float*>(a.tpart), a.chunks, a.lam, a.K, a.lmbda, a.sc,
                       reinterpret_cast<P4<float>*>(a.GT), reinterpret_cast<P4<float>*>(a.HT),
                       a.gate);
    hipLaunchKernelGGL(k_apply4, dim3((a.M + 63) / 64), dim3(256), 6 * a.K * sizeof(float), st,
                       X, U, reinterpret_cast<const P4<float>*>(a.GT),
                       reinterpret_cast<const P4<float>*>(a.HT), a.M, a.K, a.sc,
                       reinterpret_cast<P4<float>*>(a.Xnew), reinterpret_cast<P4<float>*>(a.W),
                       a.gate, reinterpret_cast<P4<float>*>(a.Xt),
                       reinterpret_cast<const P4<float>*>(a.Yt),
                       reinterpret_cast<const float*>(a.tbar), a.sigpart);
    return a.sigpart ? (a.M + 63) / 64 : 0;
  }
  const int kt = a.K <= 256 ? 1 : (a.K <= 512 ? 2 : 4);
  dim3 g1(a.chunks, (a.K + 256 * kt - 1) / (256 * kt));
  if (kt == 1)
    hipLaunchKernelGGL((k_tpart<T, 1>), g1, dim3(256), 0, st, a.X, a.Yt, a.U, a.M, a.K, a.rows_per_chunk, a.sc, a.tpart, a.gate);
  else if (kt == 2)
    hipLaunchKernelGGL((k_tpart<T, 2>), g1, dim3(256), 0, st, a.X, a.Yt, a.U, a.M, a.K, a.rows_per_chunk, a.sc, a.tpart, a.gate);
  else
    hipLaunchKernelGGL((k_tpart<T, 4>), g1, dim3(256), 0, st, a.X, a.Yt, a.U, a.M, a.K, a.rows_per_chunk, a.sc, a.tpart, a.gate);
  hipLaunchKernelGGL(k_tmerge<T>, dim3(a.K), dim3(64), 0, st, a.tpart, a.chunks, a.lam, a.K,
                     a.lmbda, a.sc, a.GT, a.HT, a.gate);
  const dim3 g3((a.M + 63) / 64);
  if (2 * (size_t)a.K * sizeof(P4<T>) <= kApplyLdsBytes)
    hipLaunchKernelGGL((k_apply<T, true>), g3, dim3(256), 2 * a.K * sizeof(P4<T>), st, a.X, a.U,
                       a.GT, a.HT, a.M, a.K, a.sc, a.Xnew, a.W, a.gate);
  else
    hipLaunchKernelGGL((k_apply<T, false>), g3, dim3(256), 0, st, a.X, a.U, a.GT, a.HT, a.M,
                       a.K, a.sc, a.Xnew, a.W, a.gate);
  return 0;
}

// ------------------------------------------------------------------ sigma^2
// Per row, with b = xt_old, a = xt_new and sum_n p'_mn = 1:
//   sum_n p'_mn |y_n - a|^2 = tbar_m + 2 (yt_m - b).(b - a) + |b - a|^2
// (no cancellation of large terms, unlike the trace form of eq. 18).  For the
// original method the row carries its weight P1_m and sigma^2 divides by
// N_P = sum_m P1_m instead of M.  The kernel also retires the old iterate.
template <typename T>
__device__ __forceinline__ void sig_part_body(P4<T>* __restrict__ Xt,
                                                  const P4<T>* __restrict__ Xnew,
                                                  const P4<T>* __restrict__ Yt,
                                                  const T* __restrict__ tbar,
                                                  const T* __restrict__ P1, int M,
                                                  const DevScalars* __restrict__ sc,
                                                  double* __restrict__ part, int gate, int bx_, int by_, int gx_) {
  __shared__ double sh[16];
  if (gate && sc->done) return;
  if (sc->nonfinite) return;  // a failed M-step leaves the iterate as it was
  const int m = bx_ * blockDim.x + threadIdx.x;
  double v = 0.0, wsum = 0.0;
  if (m < M) {
    const P4<T> b = Xt[m], a = Xnew[m], y = Yt[m];
    const double bx = b.x, by = b.y, bz = b.z;
    const double ex = bx - a.x, ey = by - a.y, ez = bz - a.z;
    const double cross = ((double)y.x - bx) * ex + ((double)y.y - by) * ey + ((double)y.z - bz) * ez;
    v = (double)tbar[m] + 2.0 * cross + ex * ex + ey * ey + ez * ez;
    if (P1) {
      wsum = (double)P1[m];
      v *= wsum;
    }
    Xt[m] = a;
  }
  const double s1 = block_sum_d(v, sh);
  const double s2 = block_sum_d(wsum, sh);
  if (threadIdx.x == 0) {
    part[2 * bx_] = s1;
    part[2 * bx_ + 1] = s2;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_sig_part(P4<T>* __restrict__ Xt,
                                                  const P4<T>* __restrict__ Xnew,
                                                  const P4<T>* __restrict__ Yt,
                                                  const T* __restrict__ tbar,
                                                  const T* __restrict__ P1, int M,
                                                  const DevScalars* __restrict__ sc,
                                                  double* __restrict__ part, int gate) {
  sig_part_body<T>(Xt, Xnew, Yt, tbar, P1, M, sc, part, gate, blockIdx.x, blockIdx.y, gridDim.x);
}

template <typename T>
__device__ __forceinline__ void sig_final_body(const double* __restrict__ part, int blocks,
                                                   const double* __restrict__ llpart,
                                                   int llblocks, int M, int N, int D, double w,
                                                   int weighted, DevScalars* sc, int gate, int bx_, int by_, int gx_) {
  __shared__ double sh[16];
  if (gate && sc->done) return;
  double a = 0.0, b = 0.0, c = 0.0;
  for (int i = threadIdx.x; i < blocks; i += blockDim.x) {
    a += part[2 * i];
    b += part[2 * i + 1];
  }
  for (int i = threadIdx.x; i < llblocks; i += blockDim.x) c += llpart[i];
  a = block_sum_d(a, sh);
  b = block_sum_d(b, sh);
  c = block_sum_d(c, sh);
  if (threadIdx.x == 0) {
    if (sc->nonfinite) {
      sc->iter += 1;
      sc->done = 1;
      return;
    }
    const double s2old = sc->sigma2;
    const double denom = weighted ? (double)D * b : (double)D * (double)M;
    double s2 = a / denom;
    const bool finite = isfinite(s2);
    if (finite) s2 = fmax(s2, sc->sigma2_floor);
    const double ds = fabs(s2 - s2old);
    // eq. 3: sum_n ln[w/N + (1-w)/M (2 pi s2)^(-D/2) sum_m exp(.)]
    //      = sum_n ln d_n + N (ln((1-w)/M) - D/2 ln(2 pi s2))
    sc->loglik = c + (double)N * (log1p(-w) - log((double)M) -
                                  0.5 * D * log(2.0 * 3.14159265358979323846 * s2old));
    sc->iter += 1;
    if (!finite) {
      sc->nonfinite = 1;
      sc->done = 1;
      return;
    }
    sc->sigma2 = s2;
    sc->dsigma2 = ds;
    sc->converged = ds < sc->tol;
    if (sc->converged || sc->iter >= sc->max_iter) sc->done = 1;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_sig_final(const double* __restrict__ part, int blocks,
                                                   const double* __restrict__ llpart,
                                                   int llblocks, int M, int N, int D, double w,
                                                   int weighted, DevScalars* sc, int gate) {
  sig_final_body<T>(part, blocks, llpart, llblocks, M, N, D, w, weighted, sc, gate, blockIdx.x, blockIdx.y, gridDim.x);
}

template <typename T> int sigma2_blocks(int M) { return (M + 255) / 256; }

template <typename T> void sigma2_launch(const Sigma2Args<T>& a, hipStream_t st) {
  if (!a.fused)
    hipLaunchKernelGGL(k_sig_part<T>, dim3(a.blocks), dim3(256), 0, st, a.Xt, a.Xnew, a.Yt,
                       a.tbar, a.P1, a.M, a.sc, a.part, a.gate);
  hipLaunchKernelGGL(k_sig_final<T>, dim3(1), dim3(256), 0, st, a.part, a.blocks, a.llpart,
                     a.llblocks, a.M, a.N, a.D, a.w, a.P1 != nullptr ? 1 : 0, a.sc, a.gate);
}

// -------------------------------------------------------------------- init
template <typename T>
__global__ __launch_bounds__(256) void k_pack(const T* __restrict__ src, P4<T>* __restrict__ dst,
                                              P4<T>* __restrict__ dst2, int M, int D,
                                              const int* __restrict__ perm,
                                              const double* __restrict__ origin) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  const T* s = src + (size_t)(perm ? perm[i] : i) * D;
  P4<T> p{s[0], D > 1 ? s[1] : (T)0, D > 2 ? s[2] : (T)0, (T)0};
  if (origin) {  // into the iteration's frame (shift in double)
    p.x = (T)((double)p.x - origin[0]);
    if (D > 1) p.y = (T)((double)p.y - origin[1]);
    if (D > 2) p.z = (T)((double)p.z - origin[2]);
  }
  dst[i] = p;
  if (dst2) dst2[i] = p;
}

template <typename T>
__global__ __launch_bounds__(256) void k_unpack(const P4<T>* __restrict__ src, T* __restrict__ dst,
                                                int M, int D, const int* __restrict__ perm,
                                                const double* __restrict__ origin) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  const P4<T> p = src[i];
  T* d = dst + (size_t)(perm ? perm[i] : i) * D;
  if (origin) {  // back to the caller's frame (shift in double)
    d[0] = (T)((double)p.x + origin[0]);
    if (D > 1) d[1] = (T)((double)p.y + origin[1]);
    if (D > 2) d[2] = (T)((double)p.z + origin[2]);
    return;
  }
  d[0] = p.x;
  if (D > 1) d[1] = p.y;
  if (D > 2) d[2] = p.z;
}

// Partial sums of (u, |u|^2) over both sets with u = p - X[0] (shift keeps
// the double sums well scaled): part[blk * 8 + ...].
template <typename T>
__global__ __launch_bounds__(256) void k_s2init_part(const P4<T>* __restrict__ X,
                                                     const P4<T>* __restrict__ Y, int M, int N,
                                                     double* __restrict__ part) {
  __shared__ double sh[16];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const P4<T> o = X[0];
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (i < M + N) {
    const P4<T> p = i < M ? X[i] : Y[i - M];
    const double ux = (double)p.x - o.x, uy = (double)p.y - o.y, uz = (double)p.z - o.z;
    const int b = i < M ? 0 : 4;
    v[b] = ux;
    v[b + 1] = uy;
    v[b + 2] = uz;
    v[b + 3] = ux * ux + uy * uy + uz * uz;
  }
  for (int j = 0; j < 8; ++j) {
    const double s = block_sum_d(v[j], sh);
    if (threadIdx.x == 0) part[blockIdx.x * 8 + j] = s;
  }
}

// sigma^2_0 = sum_mn |y_n - x_m|^2 / (D M N)
//          = (N sum|u|^2 + M sum|v|^2 - 2 (sum u).(sum v)) / (D M N)
// The floor below which sigma^2 is not lowered is 1e-10 times the run's
// starting sigma^2, and at least floor_rel D times the closed-form value of
// the data at init (floor_rel > 0 for the BF16X mode, whose exponent error
// grows as 1 / sigma^2).
//   mode kS2Init   init: sigma^2 = given (> 0) or the closed form at X; it is
//                  also kept as sigma2_start, the start of a run from X
//   mode kS2Warm   a run from a warm start Xt = X + Phi W0: sigma^2 = the
//                  closed form at Xt (sigma2_start is left alone)
//   mode kS2Start  a run from the start state: sigma^2 = sigma2_start
//   mode kS2Given  a run with a caller-given start: sigma^2 = given (> 0)
__global__ __launch_bounds__(256) void k_s2init_final(const double* __restrict__ part, int blocks,
                                                      int M, int N, int D, double given,
                                                      double tol, int max_iter, int mode,
                                                      DevScalars* sc, double floor_rel) {
  __shared__ double sh[16];
  double v[8];
  for (int j = 0; j < 8; ++j) {
    double a = 0.0;
    for (int i = threadIdx.x; i < blocks; i += blockDim.x) a += part[i * 8 + j];
    v[j] = block_sum_d(a, sh);
  }
  if (threadIdx.x == 0) {
    const double cross = v[0] * v[4] + v[1] * v[5] + v[2] * v[6];
    const double s2closed = ((double)N * v[3] + (double)M * v[7] - 2.0 * cross) / ((double)D * M * N);
    double s2;
    if (mode == kS2Init) {
      s2 = given > 0.0 ? given : s2closed;
      sc->sigma2_start = s2;
      sc->floor_data = floor_rel * D * s2closed;
      sc->loglik = 0.0;
      sc->tol = tol;
      sc->iter = 0;
      sc->max_iter = max_iter;
      sc->diam2 = 0.0;  // set by the spatial ordering when the handle sorts
      sc->origin[0] = sc->origin[1] = sc->origin[2] = 0.0;
    } else {
      s2 = mode == kS2Warm ? s2closed : (mode == kS2Given ? given : sc->sigma2_start);
    }
    sc->sigma2 = s2;
    sc->sigma2_floor = fmax(1e-10 * s2, sc->floor_data);
    sc->dsigma2 = 0.0;
    sc->done = 0;
    sc->converged = 0;
    sc->nonfinite = 0;
    sc->chol_fail = 0;
  }
}

int init_blocks(int M, int N) { return (M + N + 255) / 256; }

template <typename T>
void init_launch(const T* Xin, const T* Yin, P4<T>* X, P4<T>* Xt, P4<T>* Y, int M, int N, int D,
                 double sigma2_init, double tol, int max_iter, DevScalars* sc, double* part,
                 hipStream_t st, double floor_rel) {
  hipLaunchKernelGGL(k_pack<T>, dim3((M + 255) / 256), dim3(256), 0, st, Xin, X, Xt, M, D,
                     (const int*)nullptr, (const double*)nullptr);
  hipLaunchKernelGGL(k_pack<T>, dim3((N + 255) / 256), dim3(256), 0, st, Yin, Y, (P4<T>*)nullptr,
                     N, D, (const int*)nullptr, (const double*)nullptr);
  const int blocks = init_blocks(M, N);
  hipLaunchKernelGGL(k_s2init_part<T>, dim3(blocks), dim3(256), 0, st, Xt, Y, M, N, part);
  hipLaunchKernelGGL(k_s2init_final, dim3(1), dim3(256), 0, st, part, blocks, M, N, D,
                     sigma2_init, tol, max_iter, kS2Init, sc, floor_rel);
}

template <typename T>
void reset_sigma2_launch(const P4<T>* Xt, const P4<T>* Y, int M, int N, int D, DevScalars* sc,
                         double* part, hipStream_t st, int mode, double given) {
  const int blocks = mode == kS2Warm ? init_blocks(M, N) : 0;
  if (blocks > 0)
    hipLaunchKernelGGL(k_s2init_part<T>, dim3(blocks), dim3(256), 0, st, Xt, Y, M, N, part);
  hipLaunchKernelGGL(k_s2init_final, dim3(1), dim3(256), 0, st, part, blocks, M, N, D, given, 0.0,
                     0, mode, sc, 0.0);
}

template <typename T>
void unpack_launch(const P4<T>* src, T* dst, int M, int D, hipStream_t st, const int* perm,
                   const double* origin) {
  hipLaunchKernelGGL(k_unpack<T>, dim3((M + 255) / 256), dim3(256), 0, st, src, dst, M, D, perm,
                     origin);
}
template <typename T>
void pack_launch(const T* src, P4<T>* dst, int M, int D, hipStream_t st, const int* perm,
                 const double* origin) {
  hipLaunchKernelGGL(k_pack<T>, dim3((M + 255) / 256), dim3(256), 0, st, src, dst,
                     (P4<T>*)nullptr, M, D, perm, origin);
}

// --------------------------------------------------------- Xt = X + Phi W
// One wave per row m; Phi_mj = exp(-|x_m - x_j|^2 / (2 beta^2)) is formed on
// the fly (eq. 11).  Sums in double.
template <typename T>
__global__ __launch_bounds__(256) void k_phi_apply(const P4<T>* __restrict__ X,
                                                   const T* __restrict__ W, P4<T>* __restrict__ Xt,
                                                   int M, int D, double beta) {
  const int lane = threadIdx.x & 63;
  const int m = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (m >= M) return;
  const double inv = 1.0 / (2.0 * beta * beta);
  const P4<T> a = X[m];
  double sx = 0, sy = 0, sz = 0;
  for (int j = lane; j < M; j += 64) {
    const P4<T> b = X[j];
    const double dx = (double)a.x - b.x, dy = (double)a.y - b.y, dz = (double)a.z - b.z;
    const double p = exp(-(dx * dx + dy * dy + dz * dz) * inv);
    const T* wj = W + (size_t)j * D;
    sx += p * (double)wj[0];
    if (D > 1) sy += p * (double)wj[1];
    if (D > 2) sz += p * (double)wj[2];
  }
  sx = wave_sum(sx);
  sy = wave_sum(sy);
  sz = wave_sum(sz);
  if (lane == 0) Xt[m] = P4<T>{(T)(a.x + sx), (T)(a.y + sy), (T)(a.z + sz), (T)0};
}

template <typename T>
void phi_apply_launch(const P4<T>* X, const T* Wrm, P4<T>* Xt, int M, int D, double beta,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_phi_apply<T>, dim3((M + 3) / 4), dim3(256), 0, st, X, Wrm, Xt, M, D, beta);
}

// ---------------------------------------------------------- eig import
template <typename T>
__global__ __launch_bounds__(256) void k_import_eig(const double* __restrict__ Uin,
                                                    const double* __restrict__ lamin,
                                                    T* __restrict__ U, double* __restrict__ lam,
                                                    double* __restrict__ U64, int M, int K,
                                                    const int* __restrict__ perm) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t n = (size_t)M * K;
  if (i < n) {
    const size_t r = i / K, k = i % K;
    const double v = Uin[(perm ? (size_t)perm[r] : r) * K + k];
    U[i] = (T)v;
    if (U64) U64[i] = v;
  }
  if (i < (size_t)K) lam[i] = lamin[i];
}

template <typename T>
void import_eig_launch(const double* Uin, const double* lamin, T* U, double* lam, double* U64,
                       int M, int K, hipStream_t st, const int* perm) {
  const size_t n = (size_t)M * K;
  const size_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_import_eig<T>, dim3((unsigned)blocks), dim3(256), 0, st, Uin, lamin, U,
                     lam, U64, M, K, perm);
}

// ------------------------------------------------------------ batched
template <int KT>
__global__ __launch_bounds__(256) void kb_tpart(const InstDesc* __restrict__ d,
                                                const int4* __restrict__ items) {
  const int4 it = items[blockIdx.x];
  const InstDesc& D = d[it.x];
  tpart_body<float, KT>(D.X, D.Yt, D.U, D.M, D.K, D.mrows, D.sc, D.tpart, 1, it.y, it.z, 0);
}
__global__ __launch_bounds__(64) void kb_tmerge(const InstDesc* __restrict__ d,
                                                const int4* __restrict__ items) {
  const int4 it = items[blockIdx.x];
  const InstDesc& D = d[it.x];
  tmerge_body<float>(D.tpart, D.mchunks, D.lam, D.K, D.lmbda, D.sc, D.GT, D.HT, 1, it.y, 0, 0);
}
template <bool LDS>
__global__ __launch_bounds__(256) void kb_apply(const InstDesc* __restrict__ d,
                                                const int4* __restrict__ items) {
  const int4 it = items[blockIdx.x];
  const InstDesc& D = d[it.x];
  apply_body<float, LDS>(D.X, D.U, D.GT, D.HT, D.M, D.K, D.sc, D.Xnew, D.W, 1, it.y, 0, 0);
}
// Instances whose U rows allow 16-byte loads (fast_mstep_vec4) run the
// single-handle bodies; their apply also writes the sigma^2 partials and
// retires the iterate, so they have no kb_sigpart items.
__global__ __launch_bounds__(256) void kb_tpart4(const InstDesc* __restrict__ d,
                                                 const int4* __restrict__ items) {
  const int4 it = items[blockIdx.x];
  const InstDesc& D = d[it.x];
  tpart4_body(D.X, D.Yt, D.U, D.M, D.K, D.mrows, D.sc, D.tpart, 1, it.y);
}
__global__ __launch_bounds__(256) void kb_apply4(const InstDesc* __restrict__ d,
                                                 const int4* __restrict__ items) {
  const int4 it = items[blockIdx.x];
  const InstDesc& D = d[it.x];
  apply4_body(D.X, D.U, D.GT, D.HT, D.M, D.K, D.sc, D.Xnew, D.W, 1, D.Xt, D.Yt, D.tbar,
              D.sigpart, it.y);
}
__global__ __launch_bounds__(256) void kb_sigpart(const InstDesc* __restrict__ d,
                                                  const int4* __restrict__ items) {
  const int4 it = items[blockIdx.x];
  const InstDesc& D = d[it.x];
  sig_part_body<float>(D.Xt, D.Xnew, D.Yt, D.tbar, (const float*)nullptr, D.M, D.sc, D.sigpart, 1,
                       it.y, 0, 0);
}
__global__ __launch_bounds__(256) void kb_sigfinal(const InstDesc* __restrict__ d,
                                                   const int4* __restrict__ items) {
  const int4 it = items[blockIdx.x];
  const InstDesc& D = d[it.x];
  sig_final_body<float>(D.sigpart, D.sigblocks, D.llpart, D.llblocks, D.M, D.N, 3, D.w, 0, D.sc,
                        1, 0, 0, 0);
}
__global__ __launch_bounds__(256) void kb_count_done(const InstDesc* __restrict__ d, int B,
                                                     int* __restrict__ out) {
  __shared__ double sh[16];
  double c = 0.0;
  for (int i = threadIdx.x; i < B; i += 256) c += d[i].sc->done ? 1.0 : 0.0;
  c = block_sum_d(c, sh);
  if (threadIdx.x == 0) out[0] = (int)c;
}

void batch_mstep_sigma_launch(const InstDesc* d, const BatchItems& it, hipStream_t st) {
  if (it.n_tpart > 0) {
    if (it.kt == 1)
      hipLaunchKernelGGL(kb_tpart<1>, dim3(it.n_tpart), dim3(256), 0, st, d, it.tpart);
    else if (it.kt == 2)
      hipLaunchKernelGGL(kb_tpart<2>, dim3(it.n_tpart), dim3(256), 0, st, d, it.tpart);
    else
      hipLaunchKernelGGL(kb_tpart<4>, dim3(it.n_tpart), dim3(256), 0, st, d, it.tpart);
  }
  if (it.n_tpart4 > 0)
    hipLaunchKernelGGL(kb_tpart4, dim3(it.n_tpart4), dim3(256), 0, st, d, it.tpart4);
  hipLaunchKernelGGL(kb_tmerge, dim3(it.n_tmerge), dim3(64), 0, st, d, it.tmerge);
  if (it.n_apply > 0) {
    const size_t lds = 2 * (size_t)it.maxK * sizeof(P4<float>);
    if (lds <= kApplyLdsBytes)
      hipLaunchKernelGGL(kb_apply<true>, dim3(it.n_apply), dim3(256), lds, st, d, it.apply);
    else
      hipLaunchKernelGGL(kb_apply<false>, dim3(it.n_apply), dim3(256), 0, st, d, it.apply);
  }
  if (it.n_apply4 > 0)
    hipLaunchKernelGGL(kb_apply4, dim3(it.n_apply4), dim3(256), 6 * (size_t)it.maxK4 * sizeof(float),
                       st, d, it.apply4);
  if (it.n_sigpart > 0)
    hipLaunchKernelGGL(kb_sigpart, dim3(it.n_sigpart), dim3(256), 0, st, d, it.sigpart);
  hipLaunchKernelGGL(kb_sigfinal, dim3(it.n_inst), dim3(256), 0, st, d, it.inst);
  hipLaunchKernelGGL(kb_count_done, dim3(1), dim3(256), 0, st, d, it.n_inst, it.done_count);
}

void batch_iteration_launch(const InstDesc* d, const BatchItems& it, hipStream_t st) {
  batch_estep_launch(d, it, st);
  batch_mstep_sigma_launch(d, it, st);
}

#define FCPD_INST(T)                                                                          \
  template int fast_mstep_launch<T>(const FastMArgs<T>&, hipStream_t);                       \
  template int fast_mstep_chunks<T>(int, int*);                                              \
  template bool fast_mstep_vec4<T>(int);                                                     \
  template void sigma2_launch<T>(const Sigma2Args<T>&, hipStream_t);                         \
  template int sigma2_blocks<T>(int);                                                        \
  template void init_launch<T>(const T*, const T*, P4<T>*, P4<T>*, P4<T>*, int, int, int,     \
                               double, double, int, DevScalars*, double*, hipStream_t,       \
                               double);                                                       \
  template void reset_sigma2_launch<T>(const P4<T>*, const P4<T>*, int, int, int, DevScalars*, \
                                       double*, hipStream_t, int, double);                            \
  template void unpack_launch<T>(const P4<T>*, T*, int, int, hipStream_t, const int*,       \
                                 const double*);                                              \
  template void pack_launch<T>(const T*, P4<T>*, int, int, hipStream_t, const int*,        \
                               const double*);                                                \
  template void phi_apply_launch<T>(const P4<T>*, const T*, P4<T>*, int, int, double,         \
                                    hipStream_t);                                             \
  template void import_eig_launch<T>(const double*, const double*, T*, double*, double*, int,  \
                                     int, hipStream_t, const int*);
FCPD_INST(float)
FCPD_INST(double)

}  // namespace fcpd
