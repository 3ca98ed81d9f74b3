// Entry points of modes still being written.
#include "kernels.hpp"

namespace fcpd {
void estep_bf16x_launch(const EStepArgs<float>& a, hipStream_t st) { estep_launch<float>(a, st); }
}  // namespace fcpd
