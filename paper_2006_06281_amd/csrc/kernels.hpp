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
  double* llpart;    // ceil(N / 256)
  T* logd_out;       // nullable (N)
  P4<T>* Yt;         // out (M)
  T* P1;             // out (M)
  T* tbar;           // out (M)
  hipEvent_t* ev;    // nullable: 5 events recorded between the stages
  __bf16* featX;     // BF16X: model feature vectors (32 bf16 per point, padded)
  __bf16* featY;     // BF16X: scene feature vectors
  __bf16* featY_L;   // BF16X: featY, refreshed with L_n by the column merge (else NULL)
  __bf16* featV;     // BF16X: scene sum operands of pass B (32 bf16 per point, padded)
  // Far-tile culling (nullable: no culling).  Per tile of 2^box_shift
  // prescaled points (64 in the FP32 / FP64 passes, 16 in BF16X), box[2t] =
  // lower corner, box[2t + 1] = upper corner; boxY[2t].w receives min L_n
  // over the tile after pass A.
  P4<T>* boxX;       // ceil(M / 2^box_shift) tiles
  P4<T>* boxY;       // ceil(N / 2^box_shift) tiles
  int box_shift = 6;
};

// A tile pair whose smallest possible base-2 exponent reaches this value
// contributes exactly zero: 2^-160 (float) and 2^-1100 (double) are below
// half the smallest subnormal, so every exp2 of the tile rounds to +0 and
// skipping the tile leaves every sum bit-identical.
template <typename T> struct CullLimit;
template <> struct CullLimit<float> { static constexpr float value = 160.0f; };
template <> struct CullLimit<double> { static constexpr double value = 1100.0; };

// Lower bound of |u - v|^2 over u in box a, v in box b (corners lo, hi; hi.w
// holds the largest squared norm of the tile's points).  2^-12 of the larger
// squared norm is subtracted: it covers the rounding of the squared distances
// the kernels compute (direct differences, or the split-bf16 dot products of
// the matrix-core path).
template <typename T>
__device__ __forceinline__ T box_gap2(const P4<T>& alo, const P4<T>& ahi, const P4<T>& blo,
                                      const P4<T>& bhi) {
  const T gx = fmax(fmax(alo.x - bhi.x, blo.x - ahi.x), (T)0);
  const T gy = fmax(fmax(alo.y - bhi.y, blo.y - ahi.y), (T)0);
  const T gz = fmax(fmax(alo.z - bhi.z, blo.z - ahi.z), (T)0);
  return gx * gx + gy * gy + gz * gz - (T)0x1p-12 * fmax(ahi.w, bhi.w);
}

// Whether tile checks can pay at this sigma^2: only when pairs half the
// problem's diameter apart already underflow.  Skipping the checks is always
// exact (every tile is evaluated), so this is a cost heuristic only.
__device__ __forceinline__ bool cull_worthwhile(const DevScalars* sc, double ref, double limit) {
  return 0.25 * sc->diam2 * kappa_of(sc->sigma2) + ref >= limit;
}
template <typename T> void estep_launch(const EStepArgs<T>& a, hipStream_t st);
// pieces shared with the BF16X E-step
template <typename T> void colmerge_fix_launch(const EStepArgs<T>& a, hipStream_t st);
template <typename T> void rowmerge_fix_launch(const EStepArgs<T>& a, hipStream_t st, int relative);
// BF16X split plan; capB: resident pass-B blocks on the device (0: unknown).
void bfx_splits(int M, int N, int capB, int* splitsA, int* chunkA, int* splitsB, int* chunkB);
int bfx_splitsB_max(int M, int N);  // the most pass-B splits any capB can give
int bfx_resident_blocksB();         // on the current device; 0 if it cannot say
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
  // Optional (sigpart non-null): where the vectorised apply kernel runs
  // (FP32, K % 4 == 0, K <= 1024) it also writes the per-block partials of
  // the sigma^2 update and retires the iterate into Xt (the sig_part work);
  // fast_mstep_launch then returns the number of partials, else 0.
  P4<T>* Xt = nullptr;
  const T* tbar = nullptr;
  double* sigpart = nullptr;  // 2 per block of 64 rows
};
template <typename T> int fast_mstep_launch(const FastMArgs<T>& a, hipStream_t st);
template <typename T> int fast_mstep_chunks(int M, int* rows_per_chunk);
// FP32 with K % 4 == 0 and K <= 1024: the M-step takes 16-byte loads of U
template <typename T> bool fast_mstep_vec4(int K);

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
  int fused = 0;      // 1: the M-step wrote the partials and retired the iterate
};
template <typename T> void sigma2_launch(const Sigma2Args<T>& a, hipStream_t st);
template <typename T> int sigma2_blocks(int M);

// init: pack row-major X (M x D) and Y (N x D) into P4 arrays, sigma^2_0.
template <typename T>
void init_launch(const T* Xin, const T* Yin, P4<T>* X, P4<T>* Xt, P4<T>* Y, int M, int N, int D,
                 double sigma2_init, double tol, int max_iter, DevScalars* sc, double* part,
                 hipStream_t st, double floor_rel = 0.0);
int init_blocks(int M, int N);
// Start of a new run: kS2Warm sets sigma^2 to the closed form at Xt (a warm
// start Xt = X + Phi W0), kS2Start back to the value set at init, kS2Given to
// `given`; all keep the data's part of the floor (kS2Init is cpd_init's own
// mode).
enum { kS2Init = 0, kS2Warm = 1, kS2Start = 2, kS2Given = 3 };
template <typename T>
void reset_sigma2_launch(const P4<T>* Xt, const P4<T>* Y, int M, int N, int D, DevScalars* sc,
                         double* part, hipStream_t st, int mode, double given = -1.0);
// sigma^2 floor of the BF16X mode, relative to D times the data's closed-form
// sigma^2_0: keeps its worst-case exponent error (2^-21 3 kappa R^2 base-2
// units, R the extent of the points) to tens of units, far from where an
// exponential overflows, while sitting below the sigma^2 that noisy data
// converge to (1e-5 was measured to bind on a noisy 50k sphere and cut its
// iterations short).
constexpr double kBfxSigma2FloorRel = 1e-7;

// pack / unpack between row-major M x D arrays and P4 arrays; with perm
// (internal row i <-> caller row perm[i]) pack gathers and unpack scatters;
// with origin (device, 3 doubles) pack subtracts and unpack adds it.
template <typename T>
void unpack_launch(const P4<T>* src, T* dst, int M, int D, hipStream_t st,
                   const int* perm = nullptr, const double* origin = nullptr);
template <typename T>
void pack_launch(const T* src, P4<T>* dst, int M, int D, hipStream_t st,
                 const int* perm = nullptr, const double* origin = nullptr);

// Xt = X + Phi(X, beta) W (Phi formed on the fly), W row-major M x D
template <typename T>
void phi_apply_launch(const P4<T>* X, const T* Wrm, P4<T>* Xt, int M, int D, double beta,
                      hipStream_t st);

// eigen-prep helpers
template <typename T>
void import_eig_launch(const double* Uin, const double* lamin, T* U, double* lam, double* U64,
                       int M, int K, hipStream_t st, const int* perm = nullptr);

// ---------------------------------------------------------- spatial order
// Sorts the model and scene points (P4, in place) along a Hilbert curve over
// their joint bounding box, so runs of consecutive points (the culling
// tiles) are spatially compact.  permX[i] / permY[i] = the caller's row of
// internal row i.  Scratch: keys (next power of two >= max(M, N) uint64),
// bbox (order_bbox_doubles(M + N) doubles), tmp (max(M, N) P4).  invY is
// the inverse of permY (internal row of a caller's scene row).  Xraw
// receives the sorted model points in the caller's frame; then both sets
// are moved (in double) into the iteration's frame, centred on the scene's
// bounding box: sc->origin.  sc->diam2 = squared diagonal of the joint box.
int order_bbox_doubles(int n);
template <typename T>
void spatial_order_launch(P4<T>* X, int M, P4<T>* Y, int N, int* permX, int* permY,
                          int* invY, unsigned long long* keys, double* bbox, P4<T>* tmp,
                          P4<T>* Xraw, DevScalars* sc, hipStream_t st);
// ------------------------------------------------------- two-way matching
// out (N, caller order): for every scene point its nearest transformed model
// point (caller's row), -1 when mutual_only and the pair is not mutual.
template <typename T>
void matches_launch(const P4<T>* Xt, int M, const P4<T>* Y, int N, int mutual_only,
                    const int* permX, const int* permY, int* nnXY, int* nnYX, int32_t* out,
                    hipStream_t st);
// P1 (indicator) and Yt (matched scene point) from a caller-order match list.
template <typename T>
void match_in_launch(const int32_t* match, int M, int N, const int* permX, const int* invY,
                     const P4<T>* X, const P4<T>* Y, T* P1, P4<T>* Yt, hipStream_t st);

// dst[i, :] = src[perm[i], :] (gather rows) and dst[perm[i], :] = src[i, :]
// (scatter rows), row-major with `cols` columns.
template <typename T>
void gather_rows_launch(const T* src, T* dst, const int* perm, int rows, int cols,
                        hipStream_t st);
template <typename T>
void scatter_rows_launch(const T* src, T* dst, const int* perm, int rows, int cols,
                         hipStream_t st);

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
  double* llpart;
  double* sigpart;
  const float* U;
  const double* lam;
  float* tpart;
  P4<float>* GT;
  P4<float>* HT;
  P4<float>* boxX;  // 64-point tile boxes of the prescaled points (NULL: no culling)
  P4<float>* boxY;
  DevScalars* sc;
  int M, N, K;
  int splitsA, chunkA, splitsB, chunkB;
  int mchunks, mrows, sigblocks, llblocks;
  double w, lmbda;
};

// Work items: (instance, block index x, block index y, unused), one per
// workgroup of the corresponding stage.
struct BatchItems {
  const int4 *prescale, *colsum, *colmerge, *rowsum, *rowmerge, *tpart, *tpart4, *tmerge, *apply,
      *apply4, *sigpart, *inst;
  int n_prescale, n_colsum, n_colmerge, n_rowsum, n_rowmerge, n_tpart, n_tpart4, n_tmerge,
      n_apply, n_apply4, n_sigpart, n_inst;
  int nb;             // points per thread in the E-step passes (tiles of 256 nb)
  int kt;             // eigenpairs per thread in kb_tpart (from the largest K it serves)
  int maxK;           // largest K among instances on the generic M-step kernels
  int maxK4;          // largest K among instances on the 16-byte-load kernels
  int* done_count;    // device counter of finished instances
};
void batch_iteration_launch(const InstDesc* d, const BatchItems& it, hipStream_t st);
void batch_estep_launch(const InstDesc* d, const BatchItems& it, hipStream_t st);
void batch_mstep_sigma_launch(const InstDesc* d, const BatchItems& it, hipStream_t st);
}  // namespace fcpd
