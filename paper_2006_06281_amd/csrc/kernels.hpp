// Launcher interfaces between the C ABI runtime (api.cpp) and the kernels.
#pragma once
#include "common.hpp"

namespace fcpd {

template <typename T> struct EStepArgs {
  const P4<T>* Xt;   // current transformed model (M)
  const P4<T>* Y;    // scene (N)
  P4<T>* xs;         // prescaled model scratch (M)
  P4<T>* ys;         // prescaled scene + L_n scratch (N)
  int M, N, D;
  double w;
  DevScalars* sc;
  int gate;          // 1: skip when sc->done
  int splitsA, chunkA, splitsB, chunkB;
  T* partA;          // splitsA * N
  T* partB;          // splitsB * 5 * M
  int* badcols;      // N
  int* badrows;      // M
  double* llpart;    // ceil(N / 256)
  T* logd_out;       // nullable (N)
  P4<T>* Yt;         // out (M)
  T* P1;             // out (M)
  T* tbar;           // out (M)
  hipEvent_t* ev;    // nullable: 5 events recorded between the stages
  __bf16* featX;     // BF16X: model feature vectors (32 bf16 per point, padded)
  __bf16* featY;     // BF16X: scene feature vectors
};

template <typename T> void estep_launch(const EStepArgs<T>& a, hipStream_t st);
// pieces shared with the BF16X E-step
template <typename T> void prescale_launch(const EStepArgs<T>& a, hipStream_t st);
template <typename T> void colmerge_fix_launch(const EStepArgs<T>& a, hipStream_t st);
template <typename T> void rowmerge_fix_launch(const EStepArgs<T>& a, hipStream_t st, int relative);
void bfx_splits(int M, int N, int* splitsA, int* chunkA, int* splitsB, int* chunkB);
inline int pad256(int n) { return (n + 255) & ~255; }
template <typename T>
void estep_splits(int M, int N, int* splitsA, int* chunkA, int* splitsB, int* chunkB);

template <typename T> struct FastMArgs {
  const P4<T>* X;    // original model (M)
  const P4<T>* Yt;   // E-step target (M)
  const T* U;        // M x K row-major
  const double* lam; // K
  int M, K, D;
  double lmbda;
  DevScalars* sc;
  int gate;
  int rows_per_chunk, chunks;
  T* tpart;          // chunks * K * 4
  P4<T>* GT;         // K: g_k T_k
  P4<T>* HT;         // K: h_k T_k
  P4<T>* Xnew;       // out (M)
  P4<T>* W;          // out (M)
};
template <typename T> void fast_mstep_launch(const FastMArgs<T>& a, hipStream_t st);
template <typename T> int fast_mstep_chunks(int M, int* rows_per_chunk);

template <typename T> struct Sigma2Args {
  P4<T>* Xt;          // old iterate; overwritten with Xnew
  const P4<T>* Xnew;
  const P4<T>* Yt;
  const T* tbar;
  const T* P1;        // weights for the original method (nullable for Fast)
  int M, N, D;
  double w;
  DevScalars* sc;
  int gate;
  double* part;       // 2 * blocks
  int blocks;
  const double* llpart;
  int llblocks;
};
template <typename T> void sigma2_launch(const Sigma2Args<T>& a, hipStream_t st);
template <typename T> int sigma2_blocks(int M);

// init: pack row-major X (M x D) and Y (N x D) into P4 arrays, sigma^2_0.
template <typename T>
void init_launch(const T* Xin, const T* Yin, P4<T>* X, P4<T>* Xt, P4<T>* Y, int M, int N, int D,
                 double sigma2_init, double tol, int max_iter, DevScalars* sc, double* part,
                 hipStream_t st);
int init_blocks(int M, int N);
template <typename T>
void reset_sigma2_launch(const P4<T>* Xt, const P4<T>* Y, int M, int N, int D, DevScalars* sc,
                         double* part, hipStream_t st);

// pack / unpack between row-major M x D arrays and P4 arrays
template <typename T> void unpack_launch(const P4<T>* src, T* dst, int M, int D, hipStream_t st);
template <typename T> void pack_launch(const T* src, P4<T>* dst, int M, int D, hipStream_t st);

// Xt = X + Phi(X, beta) W (Phi formed on the fly), W row-major M x D
template <typename T>
void phi_apply_launch(const P4<T>* X, const T* Wrm, P4<T>* Xt, int M, int D, double beta,
                      hipStream_t st);

// eigen-prep helpers
template <typename T>
void import_eig_launch(const double* Uin, const double* lamin, T* U, double* lam, double* U64,
                       int M, int K, hipStream_t st);

}  // namespace fcpd

namespace fcpd {
// E-step with squared distances from bf16 matrix-core products.
void estep_bf16x_launch(const EStepArgs<float>& a, hipStream_t st);
}  // namespace fcpd

namespace fcpd {
// ------------------------------------------------------------------ batched
// One registration of a batch, as the batched kernels see it (FP32, D = 3).
struct InstDesc {
  const P4<float>* X;
  P4<float>* Xt;
  P4<float>* Xnew;
  const P4<float>* Y;
  P4<float>* W;
  P4<float>* xs;
  P4<float>* ys;
  P4<float>* Yt;
  float* P1;
  float* tbar;
  float* partA;
  float* partB;
  int* badcols;
  int* badrows;
  double* llpart;
  double* sigpart;
  const float* U;
  const double* lam;
  float* tpart;
  P4<float>* GT;
  P4<float>* HT;
  DevScalars* sc;
  int M, N, K;
  int splitsA, chunkA, splitsB, chunkB;
  int mchunks, mrows, sigblocks, llblocks;
  double w, lmbda;
};

// Work items: (instance, block index x, block index y, unused), one per
// workgroup of the corresponding stage.
struct BatchItems {
  const int4 *prescale, *colsum, *colmerge, *fix, *rowsum, *rowmerge, *tpart, *tmerge, *apply,
      *sigpart, *inst;
  int n_prescale, n_colsum, n_colmerge, n_fix, n_rowsum, n_rowmerge, n_tpart, n_tmerge, n_apply,
      n_sigpart, n_inst;
  int kt;             // eigenpairs per thread in k_tpart (from the largest K)
  int maxK;
  int* done_count;    // device counter of finished instances
};
void batch_iteration_launch(const InstDesc* d, const BatchItems& it, hipStream_t st);
void batch_estep_launch(const InstDesc* d, const BatchItems& it, hipStream_t st);
void batch_mstep_sigma_launch(const InstDesc* d, const BatchItems& it, hipStream_t st);
}  // namespace fcpd
