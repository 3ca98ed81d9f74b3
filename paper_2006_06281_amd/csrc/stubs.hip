// Temporary: entry points of modes still being written.
#include "eig.hpp"
#include "kernels.hpp"
#include "orig.hpp"

namespace fcpd {
int eig_topk_max_cols() { return 1024; }
int eig_full_capacity(int M) { return M < 1024 ? M : 1024; }
EigLayout eig_layout(int, int, int, int, size_t start) { EigLayout L; L.end = start; return L; }
int eig_prepare_run(const EigRun&, int*, std::string* msg) { *msg = "not implemented"; return 3; }
template <typename T>
__global__ void k_conv(const double* a, T* b, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (T)a[i];
}
template <typename T> void convert_u_launch(const double* U64, T* U, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_conv<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, U64, U, n);
}
template void convert_u_launch<float>(const double*, float*, size_t, hipStream_t);
template void convert_u_launch<double>(const double*, double*, size_t, hipStream_t);
OrigLayout orig_layout(int, int, size_t start) { OrigLayout L; L.end = start; return L; }
template <typename T> void orig_mstep_launch(const OrigArgs<T>&, hipStream_t) {}
template <typename T> void orig_prepare(const P4<T>*, int, double, char*, const OrigLayout&, hipStream_t) {}
template void orig_mstep_launch<float>(const OrigArgs<float>&, hipStream_t);
template void orig_mstep_launch<double>(const OrigArgs<double>&, hipStream_t);
template void orig_prepare<float>(const P4<float>*, int, double, char*, const OrigLayout&, hipStream_t);
template void orig_prepare<double>(const P4<double>*, int, double, char*, const OrigLayout&, hipStream_t);
void estep_bf16x_launch(const EStepArgs<float>& a, hipStream_t st) { estep_launch<float>(a, st); }
}  // namespace fcpd
