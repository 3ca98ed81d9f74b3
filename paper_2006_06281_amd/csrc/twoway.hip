// Two-way registration for one-sided occlusion (Section IV-A): after the
// scene has been registered onto the model, one-to-one correspondences are
// taken as mutual nearest neighbours, and the model's transformation is
// solved from them alone (eq. 21 with P1 the matched indicator; the solve
// itself is the CPD-L K x K system in lowrank.hip).
//   k_nearest    for every point of A, the index of its nearest point of B
//                (squared distance in the working precision; lowest index on
//                ties); one thread per A point, B streamed as wave-uniform
//                scalar loads
//   k_match_out  mutual check and the caller's row order
//   k_match_in   P1 (indicator) and Yt (matched scene point) in the
//                library's order from the caller's match list
#include "common.hpp"
#include "kernels.hpp"

namespace fcpd {

template <typename T>
__global__ __launch_bounds__(256) void k_nearest(const P4<T>* __restrict__ A, int na,
                                                 const P4<T>* __restrict__ B, int nb,
                                                 int* __restrict__ idx) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const P4<T> a = i < na ? A[i] : P4<T>{(T)0, (T)0, (T)0, (T)0};
  T best = (T)__builtin_inf();
  int bi = 0;
  for (int j = 0; j < nb; ++j) {
    const P4<T> b = B[j];
    const T dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
    const T d2 = dx * dx + dy * dy + dz * dz;
    if (d2 < best) {
      best = d2;
      bi = j;
    }
  }
  if (i < na) idx[i] = bi;
}

// match_out[permY[n]] = permX[nnYX[n]] when (not mutual_only or
// nnXY[nnYX[n]] == n), else -1.  perm NULL: identity.
__global__ __launch_bounds__(256) void k_match_out(const int* __restrict__ nnYX,
                                                   const int* __restrict__ nnXY, int N,
                                                   int mutual_only, const int* __restrict__ permX,
                                                   const int* __restrict__ permY,
                                                   int32_t* __restrict__ out) {
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (n >= N) return;
  const int m = nnYX[n];
  const bool keep = !mutual_only || nnXY[m] == n;
  out[permY ? permY[n] : n] = keep ? (permX ? permX[m] : m) : -1;
}

// From the caller's match list (model row -> scene row or -1): internal
// P1 in {0, 1} and Yt = the matched scene point (the model point itself when
// unmatched, so its residual is 0).  invY maps caller scene rows to internal
// rows (NULL: identity).  Out-of-range entries count as unmatched.
template <typename T>
__global__ __launch_bounds__(256) void k_match_in(const int32_t* __restrict__ match, int M, int N,
                                                  const int* __restrict__ permX,
                                                  const int* __restrict__ invY,
                                                  const P4<T>* __restrict__ X,
                                                  const P4<T>* __restrict__ Y,
                                                  T* __restrict__ P1, P4<T>* __restrict__ Yt) {
  const int m = blockIdx.x * 256 + threadIdx.x;
  if (m >= M) return;
  const int s = match[permX ? permX[m] : m];
  if (s >= 0 && s < N) {
    P1[m] = (T)1;
    Yt[m] = Y[invY ? invY[s] : s];
  } else {
    P1[m] = (T)0;
    Yt[m] = X[m];
  }
}

template <typename T>
void matches_launch(const P4<T>* Xt, int M, const P4<T>* Y, int N, int mutual_only,
                    const int* permX, const int* permY, int* nnXY, int* nnYX, int32_t* out,
                    hipStream_t st) {
  hipLaunchKernelGGL(k_nearest<T>, dim3((N + 255) / 256), dim3(256), 0, st, Y, N, Xt, M, nnYX);
  if (mutual_only)
    hipLaunchKernelGGL(k_nearest<T>, dim3((M + 255) / 256), dim3(256), 0, st, Xt, M, Y, N, nnXY);
  hipLaunchKernelGGL(k_match_out, dim3((N + 255) / 256), dim3(256), 0, st, nnYX, nnXY, N,
                     mutual_only, permX, permY, out);
}

template <typename T>
void match_in_launch(const int32_t* match, int M, int N, const int* permX, const int* invY,
                     const P4<T>* X, const P4<T>* Y, T* P1, P4<T>* Yt, hipStream_t st) {
  hipLaunchKernelGGL(k_match_in<T>, dim3((M + 255) / 256), dim3(256), 0, st, match, M, N, permX,
                     invY, X, Y, P1, Yt);
}

template void matches_launch<float>(const P4<float>*, int, const P4<float>*, int, int, const int*,
                                    const int*, int*, int*, int32_t*, hipStream_t);
template void matches_launch<double>(const P4<double>*, int, const P4<double>*, int, int,
                                     const int*, const int*, int*, int*, int32_t*, hipStream_t);
template void match_in_launch<float>(const int32_t*, int, int, const int*, const int*,
                                     const P4<float>*, const P4<float>*, float*, P4<float>*,
                                     hipStream_t);
template void match_in_launch<double>(const int32_t*, int, int, const int*, const int*,
                                      const P4<double>*, const P4<double>*, double*, P4<double>*,
                                      hipStream_t);

}  // namespace fcpd
