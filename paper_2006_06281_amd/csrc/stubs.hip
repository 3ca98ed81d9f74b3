// Temporary: entry points of modes still being written.
#include "kernels.hpp"
#include "orig.hpp"

namespace fcpd {
OrigLayout orig_layout(int, int, size_t start) { OrigLayout L; L.end = start; return L; }
template <typename T> void orig_mstep_launch(const OrigArgs<T>&, hipStream_t) {}
template <typename T> void orig_prepare(const P4<T>*, int, double, char*, const OrigLayout&, hipStream_t) {}
template void orig_mstep_launch<float>(const OrigArgs<float>&, hipStream_t);
template void orig_mstep_launch<double>(const OrigArgs<double>&, hipStream_t);
template void orig_prepare<float>(const P4<float>*, int, double, char*, const OrigLayout&, hipStream_t);
template void orig_prepare<double>(const P4<double>*, int, double, char*, const OrigLayout&, hipStream_t);
void estep_bf16x_launch(const EStepArgs<float>& a, hipStream_t st) { estep_launch<float>(a, st); }
}  // namespace fcpd
