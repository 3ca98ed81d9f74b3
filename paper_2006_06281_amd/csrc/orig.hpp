// Original CPD M-step (eq. 21), the comparator of Fast CPD: interfaces.
#pragma once
#include <stddef.h>

#include "common.hpp"

namespace fcpd {

struct OrigLayout {
  size_t end = 0;
  size_t phi = 0, A = 0, rhs = 0, info = 0, misc = 0;
  int M = 0, elem = 0, nb = 0;
};
OrigLayout orig_layout(int M, int elem_bytes, size_t start);

template <typename T> struct OrigArgs {
  const P4<T>* X;
  const P4<T>* Yt;
  const T* P1;
  int M, D;
  double lmbda;
  DevScalars* sc;
  int gate;
  char* ws;
  const OrigLayout* L;
  P4<T>* Xnew;
  P4<T>* W;
};
template <typename T> void orig_mstep_launch(const OrigArgs<T>& a, hipStream_t st);
template <typename T>
void orig_prepare(const P4<T>* X, int M, double beta, char* ws, const OrigLayout& L,
                  hipStream_t st);

}  // namespace fcpd
