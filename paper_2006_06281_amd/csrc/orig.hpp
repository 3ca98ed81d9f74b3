// Original CPD M-step (eq. 21), the comparator of Fast CPD: interfaces.
#pragma once
#include <stddef.h>

#include "common.hpp"

namespace fcpd {

constexpr int kCholBlock = 128;
constexpr int kCholPanel = 2 * kCholBlock;  // panel width of the two-level blocking

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
// Blocked right-looking Cholesky (panels of kCholPanel columns, each factored
// as blocks of kCholBlock) of the lower triangle of the n x n FP64 matrix A
// (row stride lda), in place.  Linv receives the inverses of the diagonal
// blocks (ceil(n / NB) blocks of NB x NB, row-major, lower), P is panel
// scratch of n x kCholPanel doubles.  A pivot
// that is not positive sets *chol_fail and the remaining launches return at
// once; with done != NULL nothing runs while *done is set.
void chol_blocked_launch(double* A, int lda, int n, double* Linv, double* P, int* chol_fail,
                         const int* done, hipStream_t st);
// Solves L L^T x = b in place with the factor and block inverses left by
// chol_blocked_launch; b holds n rows of 4 doubles (columns 0..2 used).
void chol_solve_launch(const double* A, int lda, int n, const double* Linv, double* b,
                       const int* chol_fail, const int* done, hipStream_t st);
template <typename T> void orig_mstep_launch(const OrigArgs<T>& a, hipStream_t st);
template <typename T>
void orig_prepare(const P4<T>* X, int M, double beta, char* ws, const OrigLayout& L,
                  hipStream_t st);

}  // namespace fcpd
