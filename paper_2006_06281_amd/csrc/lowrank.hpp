// CPD-L M-step (eq. 21 with the rank-K Gram of eq. 19): interfaces.
#pragma once
#include <stddef.h>

#include "common.hpp"

namespace fcpd {

struct LowRankLayout {
  size_t end = 0;
  size_t t = 0, Uw = 0, S = 0, gpart = 0, Linv = 0, pan = 0, q = 0, qpart = 0;
  int qchunks = 1;
};
LowRankLayout lowrank_layout(int M, int K, size_t start);

template <typename T> struct LowRankArgs {
  const P4<T>* X;
  const P4<T>* Yt;      // d(P1)^-1 P Y
  const T* P1;
  const double* U64;    // M x K eigenvectors (FP64)
  const double* lam;    // K eigenvalues
  int M, K;
  double lmbda;
  DevScalars* sc;
  int gate;
  char* ws;
  const LowRankLayout* L;
  P4<T>* Xnew;
  P4<T>* W;
};
template <typename T> void lowrank_mstep_launch(const LowRankArgs<T>& a, hipStream_t st);

}  // namespace fcpd
