// Learned warm-start network: interfaces (see net.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace fcpd {

constexpr int H = 256;

// Offsets (in floats) of every parameter inside the flat fp32 master array.
struct NetOffsets {
  size_t W1, b1, W2, b2, W3, b3, W4, b4, Wa, Wb, Wc, bh, Wo, bo, count;
};
NetOffsets net_offsets();

// Storage precision of the network's activations and weight copies.
constexpr int kNetBf16 = 0, kNetFp32 = 1;

// Byte offsets inside the network workspace for (batch, M, N, precision).
struct NetWs {
  size_t aX[4], aY[4], z, dA, dB, gX, gY, iX, iY, u, du, dgX, dgY, W0, R, dW0, lossp, loss,
      part, red, wbf, end;
};
NetWs net_ws_layout(int batch, int M, int N, int precision);

void net_init_launch(float* params, uint64_t seed, float out_scale, hipStream_t st);
void net_synth_launch(float* X, float* Y, float* V, float* Wscratch, int batch, int M, int shape,
                      double beta, double coef, double jitter, double outlier_frac,
                      uint64_t seed0, hipStream_t st);
void net_forward_launch(const float* params, const float* X, const float* Y, int batch, int M,
                        int N, float* W0, char* ws, const NetWs& L, int precision,
                        hipStream_t st);
void net_loss_grad_launch(const float* params, const float* X, const float* Y, const float* V,
                          int batch, int M, int N, double beta, float* grad, double* loss_dev,
                          char* ws, const NetWs& L, int precision, hipStream_t st);
void net_adam_launch(float* params, float* m, float* v, const float* grad, int step, float lr,
                     hipStream_t st);

}  // namespace fcpd
