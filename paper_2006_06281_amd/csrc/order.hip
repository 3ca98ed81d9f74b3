// Spatial ordering of the point sets.  The E-step's far-tile culling skips
// tiles of consecutive points (64 in FP32 / FP64, 16 in BF16X) whose
// exponentials all underflow; that only pays when the
// points of a tile are close together, so at init the model and scene points
// are sorted along a Hilbert curve over their joint bounding box (unlike a
// Morton curve it has no long jumps between consecutive cells, so a run of
// 64 points does not straddle two distant clusters: on a 50k surface the
// culled E-step keeps 11% of the 64 x 64 tile pairs instead of 14%).
// The registration result does not depend on the order (every sum of the
// method is over all points); the permutations are kept so that every
// per-point array crossing the C ABI is in the caller's order.
//
// Sort: 30-bit Hilbert index (10 bits per axis of the common cube; Skilling's
// transpose algorithm, "Programming the Hilbert curve", AIP Conf. Proc. 707,
// 2004) in the high word, the original index in the low word, so keys are
// distinct and the order is deterministic; bitonic sorting network over the
// next power of two (padding keys are all ones).
#include "common.hpp"
#include "kernels.hpp"

namespace fcpd {

namespace {
constexpr int kBBoxBlocks = 256;
typedef unsigned long long u64;

__device__ __forceinline__ uint32_t spread10(uint32_t v) {
  // bits b9..b0 -> positions 27, 24, ..., 0
  v &= 0x3FFu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}
}  // namespace

int order_bbox_doubles(int) { return 6 * kBBoxBlocks + 6; }

template <typename T>
__global__ __launch_bounds__(256) void k_bbox_part(const P4<T>* __restrict__ X, int M,
                                                   const P4<T>* __restrict__ Y, int N,
                                                   double* __restrict__ part) {
  __shared__ double sh[6][256];
  const int tid = threadIdx.x;
  const double inf = __builtin_inf();
  double v[6] = {inf, inf, inf, -inf, -inf, -inf};
  for (int i = blockIdx.x * 256 + tid; i < M + N; i += gridDim.x * 256) {
    const P4<T> p = i < M ? X[i] : Y[i - M];
    const double c[3] = {(double)p.x, (double)p.y, (double)p.z};
    for (int d = 0; d < 3; ++d) {
      v[d] = fmin(v[d], c[d]);
      v[3 + d] = fmax(v[3 + d], c[d]);
    }
  }
  for (int d = 0; d < 6; ++d) sh[d][tid] = v[d];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o)
      for (int d = 0; d < 6; ++d)
        sh[d][tid] = d < 3 ? fmin(sh[d][tid], sh[d][tid + o]) : fmax(sh[d][tid], sh[d][tid + o]);
    __syncthreads();
  }
  if (tid < 6) part[blockIdx.x * 6 + tid] = sh[tid][0];
}

__global__ __launch_bounds__(64) void k_bbox_final(double* __restrict__ part, int blocks,
                                                   DevScalars* __restrict__ sc, int what) {
  __shared__ double r6[6];
  const int d = threadIdx.x;
  if (d < 6) {
    double r = part[d];
    for (int b = 1; b < blocks; ++b)
      r = d < 3 ? fmin(r, part[b * 6 + d]) : fmax(r, part[b * 6 + d]);
    part[blocks * 6 + d] = r;
    r6[d] = r;
  }
  __syncthreads();
  if (d == 0) {
    if (what == 0) {  // the frame: centre of this box
      for (int k = 0; k < 3; ++k) sc->origin[k] = 0.5 * (r6[k] + r6[3 + k]);
    } else {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += (r6[3 + k] - r6[k]) * (r6[3 + k] - r6[k]);
      sc->diam2 = s;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_shift(P4<T>* __restrict__ P, int n,
                                               const DevScalars* __restrict__ sc) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  P4<T> p = P[i];
  p.x = (T)((double)p.x - sc->origin[0]);
  p.y = (T)((double)p.y - sc->origin[1]);
  p.z = (T)((double)p.z - sc->origin[2]);
  P[i] = p;
}

// Hilbert index of a cell of the 1024^3 grid: the coordinates are turned
// into the curve's transposed form (undo the excess work of the inverse
// walk, then Gray-code) and their bits interleaved, x most significant.
__device__ __forceinline__ uint32_t hilbert3_10(uint32_t x, uint32_t y, uint32_t z) {
  uint32_t X[3] = {x, y, z};
  constexpr uint32_t top = 1u << 9;
  for (uint32_t Q = top; Q > 1; Q >>= 1) {
    const uint32_t P = Q - 1;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      if (X[i] & Q) {
        X[0] ^= P;  // invert the low bits of the first axis
      } else {      // exchange the low bits of the first axis and axis i
        const uint32_t t = (X[0] ^ X[i]) & P;
        X[0] ^= t;
        X[i] ^= t;
      }
    }
  }
  X[1] ^= X[0];
  X[2] ^= X[1];
  uint32_t t = 0;
  for (uint32_t Q = top; Q > 1; Q >>= 1)
    if (X[2] & Q) t ^= Q - 1;
  X[0] ^= t;
  X[1] ^= t;
  X[2] ^= t;
  return (spread10(X[0]) << 2) | (spread10(X[1]) << 1) | spread10(X[2]);
}

template <typename T>
__global__ __launch_bounds__(256) void k_curve_key(const P4<T>* __restrict__ P, int n, int n2,
                                                const double* __restrict__ box,
                                                u64* __restrict__ keys) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n2) return;
  if (i >= n) {
    keys[i] = ~0ull;
    return;
  }
  const double ext = fmax(fmax(box[3] - box[0], box[4] - box[1]), fmax(box[5] - box[2], 1e-300));
  const double s = 1024.0 / ext;
  const P4<T> p = P[i];
  auto q = [&](double c, double lo) {
    const double t = (c - lo) * s;
    return (uint32_t)(t < 0.0 ? 0.0 : (t > 1023.0 ? 1023.0 : t));
  };
  const uint32_t code = hilbert3_10(q((double)p.x, box[0]), q((double)p.y, box[1]),
                                    q((double)p.z, box[2]));
  keys[i] = ((u64)code << 32) | (u64)(uint32_t)i;
}

__global__ __launch_bounds__(256) void k_bitonic(u64* __restrict__ a, int j, int k, int n2) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n2) return;
  const int l = i ^ j;
  if (l <= i) return;
  const u64 x = a[i], y = a[l];
  const bool up = (i & k) == 0;
  if ((x > y) == up) {
    a[i] = y;
    a[l] = x;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_perm_gather(const u64* __restrict__ keys, int n,
                                                     int* __restrict__ perm,
                                                     int* __restrict__ inv,
                                                     const P4<T>* __restrict__ src,
                                                     P4<T>* __restrict__ dst) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int idx = (int)(uint32_t)(keys[i] & 0xFFFFFFFFull);
  perm[i] = idx;
  if (inv) inv[idx] = i;
  dst[i] = src[idx];
}

template <typename T>
void spatial_order_launch(P4<T>* X, int M, P4<T>* Y, int N, int* permX, int* permY, int* invY,
                          u64* keys, double* bbox, P4<T>* tmp, P4<T>* Xraw, DevScalars* sc,
                          hipStream_t st) {
  // the origin of the iteration's frame: centre of the scene's bounding box;
  // then the joint box for the curve's grid
  hipLaunchKernelGGL(k_bbox_part<T>, dim3(kBBoxBlocks), dim3(256), 0, st, Y, N, Y, 0, bbox);
  hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(64), 0, st, bbox, kBBoxBlocks, sc, 0);
  hipLaunchKernelGGL(k_bbox_part<T>, dim3(kBBoxBlocks), dim3(256), 0, st, X, M, Y, N, bbox);
  hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(64), 0, st, bbox, kBBoxBlocks, sc, 1);
  const double* box = bbox + 6 * kBBoxBlocks;
  auto one = [&](P4<T>* P, int n, int* perm, int* inv) {
    int n2 = 1;
    while (n2 < n) n2 <<= 1;
    const unsigned g = (unsigned)((n2 + 255) / 256);
    hipLaunchKernelGGL(k_curve_key<T>, dim3(g), dim3(256), 0, st, P, n, n2, box, keys);
    for (int k = 2; k <= n2; k <<= 1)
      for (int j = k >> 1; j > 0; j >>= 1)
        hipLaunchKernelGGL(k_bitonic, dim3(g), dim3(256), 0, st, keys, j, k, n2);
    hipLaunchKernelGGL(k_perm_gather<T>, dim3((n + 255) / 256), dim3(256), 0, st, keys, n, perm,
                       inv, P, tmp);
    (void)hipMemcpyAsync(P, tmp, sizeof(P4<T>) * (size_t)n, hipMemcpyDeviceToDevice, st);
  };
  one(X, M, permX, nullptr);
  one(Y, N, permY, invY);
  // the caller's frame is kept for the Gram matrix; the iteration runs in
  // the centred frame (unused coordinates are 0 and stay 0)
  (void)hipMemcpyAsync(Xraw, X, sizeof(P4<T>) * (size_t)M, hipMemcpyDeviceToDevice, st);
  hipLaunchKernelGGL(k_shift<T>, dim3((M + 255) / 256), dim3(256), 0, st, X, M, sc);
  hipLaunchKernelGGL(k_shift<T>, dim3((N + 255) / 256), dim3(256), 0, st, Y, N, sc);
}

template <typename T>
__global__ __launch_bounds__(256) void k_gather_rows(const T* __restrict__ src, T* __restrict__ dst,
                                                     const int* __restrict__ perm, int rows,
                                                     int cols) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (size_t)rows * cols) return;
  const size_t r = i / cols, c = i % cols;
  dst[i] = src[(size_t)perm[r] * cols + c];
}

template <typename T>
__global__ __launch_bounds__(256) void k_scatter_rows(const T* __restrict__ src,
                                                      T* __restrict__ dst,
                                                      const int* __restrict__ perm, int rows,
                                                      int cols) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (size_t)rows * cols) return;
  const size_t r = i / cols, c = i % cols;
  dst[(size_t)perm[r] * cols + c] = src[i];
}

template <typename T>
void gather_rows_launch(const T* src, T* dst, const int* perm, int rows, int cols,
                        hipStream_t st) {
  const size_t n = (size_t)rows * cols;
  hipLaunchKernelGGL(k_gather_rows<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src,
                     dst, perm, rows, cols);
}

template <typename T>
void scatter_rows_launch(const T* src, T* dst, const int* perm, int rows, int cols,
                         hipStream_t st) {
  const size_t n = (size_t)rows * cols;
  hipLaunchKernelGGL(k_scatter_rows<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src,
                     dst, perm, rows, cols);
}

template void spatial_order_launch<float>(P4<float>*, int, P4<float>*, int, int*, int*, int*,
                                          u64*, double*, P4<float>*, P4<float>*, DevScalars*,
                                          hipStream_t);
template void spatial_order_launch<double>(P4<double>*, int, P4<double>*, int, int*, int*, int*,
                                           u64*, double*, P4<double>*, P4<double>*, DevScalars*,
                                           hipStream_t);
template void gather_rows_launch<float>(const float*, float*, const int*, int, int, hipStream_t);
template void gather_rows_launch<double>(const double*, double*, const int*, int, int,
                                         hipStream_t);
template void scatter_rows_launch<float>(const float*, float*, const int*, int, int, hipStream_t);
template void scatter_rows_launch<double>(const double*, double*, const int*, int, int,
                                          hipStream_t);

}  // namespace fcpd
