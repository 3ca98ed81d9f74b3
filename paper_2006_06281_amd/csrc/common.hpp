// Shared device-side types and helpers of libfastcpd (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fcpd {

constexpr int kWave = 64;

// A point padded to four lanes: (x, y, z, extra).  The fourth slot carries a
// per-point scalar where a kernel needs one next to the coordinates.
template <typename T> struct alignas(4 * sizeof(T)) P4 { T x, y, z, w; };

// Device-resident scalars of one registration.  Everything that changes
// from iteration to iteration lives here so that a step never needs the host.
struct DevScalars {
  double sigma2;        // current sigma^2
  double sigma2_start;  // sigma^2 after init: the start of a run from Xt = X
  double sigma2_floor;  // lower clamp of the current run
  double dsigma2;       // |sigma^2 change| of the last step
  double loglik;        // eq. 3 at the last E-step
  double tol;
  int32_t iter;         // completed iterations
  int32_t max_iter;
  int32_t done;         // converged or capped: later steps are no-ops
  int32_t converged;
  int32_t nonfinite;    // 1: sigma^2 became NaN/Inf, 2: Cholesky breakdown
  int32_t chol_fail;    // the original method's factorisation broke down
  double diam2;         // squared diagonal of the joint bounding box of X and Y
                        // at init (gates far-tile culling; 0 = never)
  double origin[3];     // the iteration's frame is the caller's minus origin
                        // (centre of the scene's bounding box; 0 unless sorted)
  double floor_data;    // the part of the floor set by the data's scale at init
                        // (BF16X; 0 otherwise): floor = max(1e-10 s2_run, this)
};

__device__ __forceinline__ float fexp2(float v) { return __builtin_amdgcn_exp2f(v); }
__device__ __forceinline__ double fexp2(double v) { return exp2(v); }
__device__ __forceinline__ float flog2(float v) { return __builtin_amdgcn_logf(v); }
__device__ __forceinline__ double flog2(double v) { return log2(v); }

// log2(e)
constexpr double kLog2e = 1.4426950408889634074;
constexpr double kLn2 = 0.69314718055994530942;

// Fixed reference (log2 units) that every pass-A exponent is measured from:
// max(log2 c, -100).  With the outlier sink c > 0 this keeps each term
// <= 2^100 and drops only terms below 2^-126 of d_n.
constexpr double kRefFloor = -100.0;

// log2 of eq. 4's outlier constant c = (2 pi s2)^(D/2) w/(1-w) M/N;
// -inf when w == 0.
__device__ __forceinline__ double log2_c(double s2, int D, double w, int M, int N) {
  if (w <= 0.0) return -__builtin_inf();
  return 0.5 * D * log2(2.0 * 3.14159265358979323846 * s2) + log2(w) - log2(1.0 - w)
         + log2((double)M) - log2((double)N);
}

// kappa = log2(e) / (2 sigma^2): a squared distance times kappa is the
// exponent of eq. 4's Gaussian in base 2.
__device__ __forceinline__ double kappa_of(double s2) { return kLog2e / (2.0 * s2); }

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  return v;
}

// Block-wide sum of a double (blockDim.x a multiple of 64, <= 1024).
__device__ __forceinline__ double block_sum_d(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  const int nw = blockDim.x >> 6;
  double r = 0.0;
  if (wid == 0) {
    r = lane < nw ? sh[lane] : 0.0;
    r = wave_sum(r);
  }
  __syncthreads();
  return r;  // valid in thread 0
}

}  // namespace fcpd
