// Original CPD M-step (eq. 21), the comparator the paper measures Fast CPD
// against: every iteration solves the M x M SPD system
//   (Phi + lambda sigma^2 d(P1)^-1) W = d(P1)^-1 P Y - X = Yt - X
// and sets Xt = X + Phi W.  Phi (eq. 11) is built once at prepare and kept in
// HBM; the system matrix A is refreshed from it each iteration (lower
// triangle only) and factorised in place by a blocked right-looking Cholesky.
//
// The factorisation runs in FP64 in every precision mode: A's condition
// number reaches lam_1(Phi) max(P1) / (lambda sigma^2) ~ 1e8 near convergence,
// beyond FP32's 1/eps, where an FP32 Cholesky breaks down (and iterative
// refinement from an FP32 factor diverges).
//
// Two-level blocking: panels of NP = 256 columns, each factored as two
// blocks of NB = 128.  Per block k of a panel:
//   diag   factor the NB x NB diagonal block in LDS, keep L_kk^-1
//   panel  P[:, k] = A[below, k] L_kk^-T     (FP64, into the panel buffer)
//   store  P[:, k] back into A
//   inner  after the first block: A[below, second block] -= P1 P1^T (the
//          panel's own second block columns, FP64 matrix cores)
// then one trailing update with the whole 256-wide panel,
//   syrk   A[below panel, below panel] -= P P^T, lower tiles only,
// which re-reads and rewrites the trailing triangle once per 256 columns
// instead of once per 128.  The two triangular solves reuse the saved
// L_kk^-1 blocks.
#include <algorithm>

#include "common.hpp"
#include "orig.hpp"

namespace fcpd {

namespace {
constexpr int NB = kCholBlock;
size_t al(size_t b) { return (b + 255) & ~(size_t)255; }
}  // namespace

OrigLayout orig_layout(int M, int elem_bytes, size_t start) {
  OrigLayout L;
  L.M = M;
  L.elem = elem_bytes;
  L.nb = NB;
  const int nblk = (M + NB - 1) / NB;
  size_t off = start;
  auto take = [&](size_t b) {
    const size_t o = off;
    off += al(b);
    return o;
  };
  L.phi = take((size_t)M * M * sizeof(double));
  L.A = take((size_t)M * M * sizeof(double));
  L.rhs = take((size_t)M * 4 * sizeof(double) * 2);     // rhs (z) and w
  L.misc = take((size_t)M * kCholPanel * sizeof(double));  // panel P
  L.info = take((size_t)nblk * NB * NB * sizeof(double) + 256);  // L_kk^-1 blocks
  L.end = off;
  return L;
}

// ------------------------------------------------------------------ build
template <typename PT>
__global__ __launch_bounds__(256) void k_phi_build(const P4<PT>* __restrict__ X, int M,
                                                   double inv2b2, double* __restrict__ Phi) {
  const int i = blockIdx.x;
  const P4<PT> a = X[i];
  for (int j = threadIdx.x; j < M; j += blockDim.x) {
    const P4<PT> b = X[j];
    const double dx = (double)a.x - b.x, dy = (double)a.y - b.y, dz = (double)a.z - b.z;
    Phi[(size_t)i * M + j] = exp(-(dx * dx + dy * dy + dz * dz) * inv2b2);
  }
}

// A = lower(Phi) + lambda sigma^2 d(1/max(P1, floor)); rhs = Yt - X (FP64).
template <typename T>
__global__ __launch_bounds__(256) void k_build_system(const double* __restrict__ Phi,
                                                      double* __restrict__ A,
                                                      const T* __restrict__ P1,
                                                      const P4<T>* __restrict__ Yt,
                                                      const P4<T>* __restrict__ X,
                                                      double* __restrict__ rhs, int M,
                                                      double lmbda, DevScalars* sc, int gate) {
  if (gate && sc->done) return;
  const int i = blockIdx.x;
  const double* src = Phi + (size_t)i * M;
  double* dst = A + (size_t)i * M;
  for (int j = threadIdx.x; j < i; j += blockDim.x) dst[j] = src[j];
  if (threadIdx.x == 0) {
    const double p1 = fmax((double)P1[i], 1e-20);
    dst[i] = src[i] + lmbda * sc->sigma2 / p1;
    const P4<T> y = Yt[i], x = X[i];
    double* r = rhs + (size_t)i * 4;
    r[0] = (double)y.x - (double)x.x;
    r[1] = (double)y.y - (double)x.y;
    r[2] = (double)y.z - (double)x.z;
    r[3] = 0.0;
    if (i == 0) sc->chol_fail = 0;
  }
}

// ------------------------------------------------------------- diagonal
// Cholesky of the nb x nb diagonal block at (k0, k0), in LDS; writes L_kk back
// (lower; the strict upper part is left as is) and Linv = L_kk^-1 (lower,
// nb x nb, row-major with stride NB).  Breakdown sets *chol_fail.  The
// inverse is built in the tile's free upper triangle (Linv[r][c] at s[c][r]),
// one row per step, all columns of the row in parallel.
__global__ __launch_bounds__(1024) void k_potrf_diag(double* __restrict__ A, int lda, int k0,
                                                     int nb, double* __restrict__ Linv,
                                                     int* chol_fail, const int* done) {
  __shared__ double s[NB][NB + 1];
  __shared__ int fail;
  if (done && *done) return;
  if (*chol_fail) return;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int tx = tid & 31, ty = tid >> 5;  // 32 x 32 thread grid for updates
  for (int e = tid; e < nb * nb; e += nt) {
    const int r = e / nb, c = e % nb;
    s[r][c] = c <= r ? A[(size_t)(k0 + r) * lda + k0 + c] : 0.0;
  }
  if (tid == 0) fail = 0;
  __syncthreads();
  // one barrier per column: step j updates the trailing triangle with the
  // unscaled column j (s[r][c] -= s[r][j] s[c][j] / d_j) and scales column
  // j - 1, which no thread reads any more
  double dprev = 1.0;
  for (int j = 0; j < nb; ++j) {
    const double d = s[j][j];  // every thread reads the same pivot
    if (!(d > 0.0) || !isfinite(d)) {
      if (tid == 0) fail = 1;
      break;
    }
    const double inv = 1.0 / d;
    for (int r = j + 1 + ty; r < nb; r += 32) {
      const double lr = s[r][j] * inv;
      for (int c = j + 1 + tx; c <= r; c += 32) s[r][c] -= lr * s[c][j];
    }
    if (j > 0) {
      const double piv = sqrt(dprev);
      for (int r = j - 1 + tid; r < nb; r += nt) s[r][j - 1] = r == j - 1 ? piv : s[r][j - 1] / piv;
    }
    dprev = d;
    __syncthreads();
  }
  __syncthreads();
  if (fail) {
    if (tid == 0) *chol_fail = 1;
    return;
  }
  {
    const double piv = sqrt(dprev);
    for (int r = nb - 1 + tid; r < nb; r += nt) s[r][nb - 1] = piv;
  }
  __syncthreads();
  for (int e = tid; e < nb * nb; e += nt) {
    const int r = e / nb, c = e % nb;
    if (c <= r) A[(size_t)(k0 + r) * lda + k0 + c] = s[r][c];
  }
  // X = L^-1 row by row: X[r][c] = -(sum_{c<=k<r} L[r][k] X[k][c]) / L[r][r]
  // for c < r, all columns at once, eight threads per column splitting the
  // sum (X[k][c] for k > c lives at s[c][k]; X[c][c] = 1 / L[c][c]).  A
  // column's eight threads sit in one wave and read only L (fixed now) and
  // their own column's earlier X, and a wave's LDS accesses complete in
  // program order, so the rows need no workgroup barrier between them.
  {
    const int c = tid >> 3, g = tid & 7;
    for (int r = 1; r < nb; ++r) {
      double v = 0.0;
      if (c < r) {
        if (g == 0) v = s[r][c] / s[c][c];
        for (int k = c + 1 + g; k < r; k += 8) v = fma(s[r][k], s[c][k], v);
      }
      v += __shfl_xor(v, 1, 8);
      v += __shfl_xor(v, 2, 8);
      v += __shfl_xor(v, 4, 8);
      if (c < r && g == 0) s[c][r] = -v / s[r][r];
      __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
  }
  for (int e = tid; e < NB * NB; e += nt) {
    const int r = e / NB, c = e % NB;
    double v = 0.0;
    if (r < nb && c < nb) v = r == c ? 1.0 / s[r][r] : (r > c ? s[c][r] : 0.0);
    Linv[e] = v;
  }
}

// P[r][c] = sum_t A[k0+nb+r][k0+t] Linv[c][t]  (P = A_panel L_kk^-T), 64 rows
// per block, all nb columns; L_kk^-T staged in LDS, the panel rows read
// through the cache (four threads share a row).
__global__ __launch_bounds__(256) void k_panel(const double* __restrict__ A, int lda, int k0,
                                               int nb, int rows, const double* __restrict__ Linv,
                                               double* __restrict__ P, int ldp,
                                               const int* chol_fail, const int* done) {
  __shared__ double sL[NB][NB + 1];  // sL[t][c] = Linv[c][t]
  if (done && *done) return;
  if (*chol_fail) return;
  const int tid = threadIdx.x;
  for (int e = tid; e < NB * NB; e += 256) {
    const int c = e / NB, t = e % NB;
    sL[t][c] = (c < nb && t < nb) ? Linv[(size_t)c * NB + t] : 0.0;
  }
  __syncthreads();
  // thread: row r = tid / 4 (64 rows), columns c = (tid % 4) + 4 j
  const int r = tid >> 2, cg = tid & 3;
  const int gr = blockIdx.x * 64 + r;
  if (gr >= rows) return;
  const double* arow = A + (size_t)(k0 + nb + gr) * lda + k0;
  double acc[NB / 4];
#pragma unroll
  for (int j = 0; j < NB / 4; ++j) acc[j] = 0.0;
  for (int t = 0; t < nb; ++t) {
    const double a = arow[t];
#pragma unroll
    for (int j = 0; j < NB / 4; ++j) acc[j] = fma(a, sL[t][cg + 4 * j], acc[j]);
  }
#pragma unroll
  for (int j = 0; j < NB / 4; ++j) {
    const int c = cg + 4 * j;
    if (c < nb) P[(size_t)gr * ldp + c] = acc[j];
  }
}

// Update A[k1+i][k1+j] -= sum_t P[i][t] P[j][t], t < nb, for i >= j, on the
// FP64 matrix cores (P row i at P + i ldp).  Tiles of 128 x 128; in the
// triangle mode (cols = 0) the grid walks the tiles on or below the diagonal
// of the R x R trailing matrix, in the column mode (cols > 0) the tiles of
// the first `cols` columns of its R rows (one column tile).  Four waves of
// 64 x 64 (4 x 4 v_mfma_f64_16x16x4f64 accumulators each); the panel rows
// are staged in LDS 16 k at a time, double-buffered, the next stage's loads
// in flight during the current stage's products.  MFMA operands: A lane l =
// row l%16, k l/16; B lane l = column l%16, k l/16; D lane l, register r =
// row 4r + l/16, column l%16.
constexpr int ST = 128, SK = 16;
typedef double dbl4_t __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256, 2) void k_syrk(double* __restrict__ A, int lda, int k1, int R,
                                                 int cols, const double* __restrict__ P, int ldp,
                                                 int nb, const int* chol_fail, const int* done) {
  __shared__ double sa[2][SK][ST + 2];
  __shared__ double sb[2][SK][ST + 2];
  if (done && *done) return;
  if (*chol_fail) return;
  int bi, bj;
  if (cols > 0) {
    bi = blockIdx.x;
    bj = 0;
  } else {  // decode the lower-triangular tile index
    const int t = blockIdx.x;
    bi = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((bi + 1) * (bi + 2) / 2 <= t) ++bi;
    while (bi * (bi + 1) / 2 > t) --bi;
    bj = t - bi * (bi + 1) / 2;
  }
  const int ncol = cols > 0 ? cols : R;
  const int i0 = bi * ST, j0 = bj * ST;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;
  dbl4_t acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = dbl4_t{0.0, 0.0, 0.0, 0.0};
  // 128 rows x 16 k of each operand per stage: 2048 values, 8 per thread
  double va[8], vb[8];
  auto gload = [&](int kk) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = tid + 256 * q;
      const int r = e >> 4, k = e & 15;
      const int gk = kk + k;
      const int ri = i0 + r, rj = j0 + r;
      va[q] = (ri < R && gk < nb) ? P[(size_t)ri * ldp + gk] : 0.0;
      vb[q] = (rj < ncol && gk < nb) ? P[(size_t)rj * ldp + gk] : 0.0;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = tid + 256 * q;
      sa[buf][e & 15][e >> 4] = va[q];
      sb[buf][e & 15][e >> 4] = vb[q];
    }
  };
  gload(0);
  sstore(0);
  __syncthreads();
  int buf = 0;
  for (int kk = 0; kk < nb; kk += SK) {
    const bool more = kk + SK < nb;
    if (more) gload(kk + SK);
#pragma unroll
    for (int ks = 0; ks < SK / 4; ++ks) {
      const int k = 4 * ks + lk;
      double x[4], y[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        x[q] = sa[buf][k][wr + 16 * q + li];
        y[q] = sb[buf][k][wc + 16 * q + li];
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[a], y[b], acc[a][b], 0, 0, 0);
    }
    if (more) sstore(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + wr + 16 * a + 4 * r + lk;
      if (i >= R) continue;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int j = j0 + wc + 16 * b + li;
        if (j <= i && j < ncol) A[(size_t)(k1 + i) * lda + k1 + j] -= acc[a][b][r];
      }
    }
}

__global__ __launch_bounds__(256) void k_store_panel(double* __restrict__ A, int lda, int k0,
                                                     int nb, int rows,
                                                     const double* __restrict__ P, int ldp,
                                                     const int* chol_fail, const int* done) {
  if (done && *done) return;
  if (*chol_fail) return;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)rows * nb) return;
  const int r = (int)(e / nb), c = (int)(e % nb);
  A[(size_t)(k0 + nb + r) * lda + k0 + c] = P[(size_t)r * ldp + c];
}

// ------------------------------------------------------- triangular solves
// rhs rows are 4 doubles (x, y, z, 0).  Forward: z_k = Linv_k b_k, then
// b_i -= L[i, k-block] z_k for the rows below.
__global__ __launch_bounds__(256) void k_fwd_diag(double* __restrict__ b, int k0, int nb,
                                                  const double* __restrict__ Linv,
                                                  const int* chol_fail, const int* done) {
  __shared__ double sb[NB][4];
  if (done && *done) return;
  if (*chol_fail) return;
  const int tid = threadIdx.x;
  for (int e = tid; e < nb * 4; e += 256) sb[e / 4][e % 4] = b[(size_t)(k0 + e / 4) * 4 + e % 4];
  __syncthreads();
  for (int e = tid; e < nb * 3; e += 256) {
    const int r = e / 3, d = e % 3;
    double v = 0.0;
    for (int t = 0; t <= r; ++t) v = fma(Linv[(size_t)r * NB + t], sb[t][d], v);
    b[(size_t)(k0 + r) * 4 + d] = v;
  }
}

__global__ __launch_bounds__(256) void k_fwd_update(double* __restrict__ b,
                                                    const double* __restrict__ A, int lda, int k0,
                                                    int nb, int M, const int* chol_fail,
                                                    const int* done) {
  __shared__ double sz[NB][4];
  if (done && *done) return;
  if (*chol_fail) return;
  const int tid = threadIdx.x;
  for (int e = tid; e < nb * 4; e += 256) sz[e / 4][e % 4] = b[(size_t)(k0 + e / 4) * 4 + e % 4];
  __syncthreads();
  // 16 lanes per row
  const int lane16 = tid & 15;
  const int row = k0 + nb + blockIdx.x * 16 + (tid >> 4);
  double s0 = 0, s1 = 0, s2 = 0;
  if (row < M) {
    const double* a = A + (size_t)row * lda + k0;
    for (int t = lane16; t < nb; t += 16) {
      const double l = a[t];
      s0 = fma(l, sz[t][0], s0);
      s1 = fma(l, sz[t][1], s1);
      s2 = fma(l, sz[t][2], s2);
    }
  }
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) {
    s0 += __shfl_xor(s0, o, 16);
    s1 += __shfl_xor(s1, o, 16);
    s2 += __shfl_xor(s2, o, 16);
  }
  if (row < M && lane16 == 0) {
    double* r = b + (size_t)row * 4;
    r[0] -= s0;
    r[1] -= s1;
    r[2] -= s2;
  }
}

// Backward: w_k = Linv_k^T z_k, then z_i -= sum_t L[k0+t][i] w_k[t] for i < k0.
__global__ __launch_bounds__(256) void k_bwd_diag(double* __restrict__ z, int k0, int nb,
                                                  const double* __restrict__ Linv,
                                                  const int* chol_fail, const int* done) {
  __shared__ double sz[NB][4];
  if (done && *done) return;
  if (*chol_fail) return;
  const int tid = threadIdx.x;
  for (int e = tid; e < nb * 4; e += 256) sz[e / 4][e % 4] = z[(size_t)(k0 + e / 4) * 4 + e % 4];
  __syncthreads();
  for (int e = tid; e < nb * 3; e += 256) {
    const int r = e / 3, d = e % 3;
    double v = 0.0;
    for (int t = r; t < nb; ++t) v = fma(Linv[(size_t)t * NB + r], sz[t][d], v);
    z[(size_t)(k0 + r) * 4 + d] = v;
  }
}

__global__ __launch_bounds__(256) void k_bwd_update(double* __restrict__ z,
                                                    const double* __restrict__ A, int lda, int k0,
                                                    int nb, const int* chol_fail,
                                                    const int* done) {
  __shared__ double sw[NB][4];
  if (done && *done) return;
  if (*chol_fail) return;
  const int tid = threadIdx.x;
  for (int e = tid; e < nb * 4; e += 256) sw[e / 4][e % 4] = z[(size_t)(k0 + e / 4) * 4 + e % 4];
  __syncthreads();
  const int i = blockIdx.x * 256 + tid;
  if (i >= k0) return;
  double s0 = 0, s1 = 0, s2 = 0;
  for (int t = 0; t < nb; ++t) {
    const double l = A[(size_t)(k0 + t) * lda + i];
    s0 = fma(l, sw[t][0], s0);
    s1 = fma(l, sw[t][1], s1);
    s2 = fma(l, sw[t][2], s2);
  }
  double* r = z + (size_t)i * 4;
  r[0] -= s0;
  r[1] -= s1;
  r[2] -= s2;
}

// Xnew = X + Phi W, W = the solved rhs; a breakdown flags non-finite.
template <typename T>
__global__ __launch_bounds__(256) void k_phi_apply_stored(const double* __restrict__ Phi,
                                                          const double* __restrict__ w,
                                                          const P4<T>* __restrict__ X, int M,
                                                          P4<T>* __restrict__ Xnew,
                                                          P4<T>* __restrict__ W,
                                                          DevScalars* sc, int gate) {
  if (gate && sc->done) return;
  const int lane = threadIdx.x & 63;
  const int m = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (m >= M) return;
  if (sc->chol_fail) {
    if (m == 0 && lane == 0) sc->nonfinite = 2;
    return;
  }
  const double* phi = Phi + (size_t)m * M;
  double s0 = 0, s1 = 0, s2 = 0;
  for (int j = lane; j < M; j += 64) {
    const double p = phi[j];
    const double* wj = w + (size_t)j * 4;
    s0 = fma(p, wj[0], s0);
    s1 = fma(p, wj[1], s1);
    s2 = fma(p, wj[2], s2);
  }
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  if (lane == 0) {
    const P4<T> x = X[m];
    Xnew[m] = P4<T>{(T)((double)x.x + s0), (T)((double)x.y + s1), (T)((double)x.z + s2), (T)0};
    const double* wm = w + (size_t)m * 4;
    W[m] = P4<T>{(T)wm[0], (T)wm[1], (T)wm[2], (T)0};
  }
}

// ------------------------------------------------------------- launchers
template <typename T>
void orig_prepare(const P4<T>* X, int M, double beta, char* ws, const OrigLayout& L,
                  hipStream_t st) {
  hipLaunchKernelGGL(k_phi_build<T>, dim3(M), dim3(256), 0, st, X, M, 1.0 / (2.0 * beta * beta),
                     reinterpret_cast<double*>(ws + L.phi));
}

void chol_blocked_launch(double* A, int lda, int n, double* Linv, double* P, int* chol_fail,
                         const int* done, hipStream_t st) {
  constexpr int NP = kCholPanel;
  for (int K0 = 0; K0 < n; K0 += NP) {
    const int w = std::min(NP, n - K0);
    // P row r holds row K0 + NB + r of the factor's panel columns
    for (int k0 = K0; k0 < K0 + w; k0 += NB) {
      const int kb = k0 / NB;
      const int nb = std::min(NB, K0 + w - k0);
      double* Li = Linv + (size_t)kb * NB * NB;
      hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(1024), 0, st, A, lda, k0, nb, Li, chol_fail,
                         done);
      const int R = n - k0 - nb;
      if (R <= 0) break;
      double* Pk = P + (size_t)(k0 - K0) * NP + (k0 - K0);  // rows from k0 + nb, columns k0 - K0
      hipLaunchKernelGGL(k_panel, dim3((R + 63) / 64), dim3(256), 0, st, A, lda, k0, nb, R, Li,
                         Pk, NP, chol_fail, done);
      const size_t cnt = (size_t)R * nb;
      hipLaunchKernelGGL(k_store_panel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, A,
                         lda, k0, nb, R, Pk, NP, chol_fail, done);
      const int rest = K0 + w - (k0 + nb);  // columns of this panel still to factor
      if (rest > 0)
        hipLaunchKernelGGL(k_syrk, dim3((R + ST - 1) / ST), dim3(256), 0, st, A, lda, k0 + nb, R,
                           rest, Pk, NP, nb, chol_fail, done);
    }
    const int R2 = n - K0 - w;
    if (R2 <= 0) continue;
    const int T_ = (R2 + ST - 1) / ST;
    const double* Pt = P + (size_t)(w - NB) * NP;  // rows from K0 + w
    hipLaunchKernelGGL(k_syrk, dim3(T_ * (T_ + 1) / 2), dim3(256), 0, st, A, lda, K0 + w, R2, 0,
                       Pt, NP, w, chol_fail, done);
  }
}

void chol_solve_launch(const double* A, int lda, int n, const double* Linv, double* b,
                       const int* chol_fail, const int* done, hipStream_t st) {
  const int nblk = (n + NB - 1) / NB;
  for (int kb = 0; kb < nblk; ++kb) {
    const int k0 = kb * NB;
    const int nb = std::min(NB, n - k0);
    const double* Li = Linv + (size_t)kb * NB * NB;
    hipLaunchKernelGGL(k_fwd_diag, dim3(1), dim3(256), 0, st, b, k0, nb, Li, chol_fail, done);
    const int R = n - k0 - nb;
    if (R > 0)
      hipLaunchKernelGGL(k_fwd_update, dim3((R + 15) / 16), dim3(256), 0, st, b, A, lda, k0, nb, n,
                         chol_fail, done);
  }
  for (int kb = nblk - 1; kb >= 0; --kb) {
    const int k0 = kb * NB;
    const int nb = std::min(NB, n - k0);
    const double* Li = Linv + (size_t)kb * NB * NB;
    hipLaunchKernelGGL(k_bwd_diag, dim3(1), dim3(256), 0, st, b, k0, nb, Li, chol_fail, done);
    if (k0 > 0)
      hipLaunchKernelGGL(k_bwd_update, dim3((k0 + 255) / 256), dim3(256), 0, st, b, A, lda, k0, nb,
                         chol_fail, done);
  }
}

template <typename T> void orig_mstep_launch(const OrigArgs<T>& a, hipStream_t st) {
  const OrigLayout& L = *a.L;
  const int M = a.M;
  double* Phi = reinterpret_cast<double*>(a.ws + L.phi);
  double* A = reinterpret_cast<double*>(a.ws + L.A);
  double* b = reinterpret_cast<double*>(a.ws + L.rhs);
  double* P = reinterpret_cast<double*>(a.ws + L.misc);
  double* Linv = reinterpret_cast<double*>(a.ws + L.info);
  const int g = a.gate;
  hipLaunchKernelGGL(k_build_system<T>, dim3(M), dim3(256), 0, st, Phi, A, a.P1, a.Yt, a.X, b, M,
                     a.lmbda, a.sc, g);
  const int* done = g ? &a.sc->done : nullptr;
  chol_blocked_launch(A, M, M, Linv, P, &a.sc->chol_fail, done, st);
  chol_solve_launch(A, M, M, Linv, b, &a.sc->chol_fail, done, st);
  hipLaunchKernelGGL(k_phi_apply_stored<T>, dim3((M + 3) / 4), dim3(256), 0, st, Phi, b, a.X, M,
                     a.Xnew, a.W, a.sc, g);
}

template void orig_mstep_launch<float>(const OrigArgs<float>&, hipStream_t);
template void orig_mstep_launch<double>(const OrigArgs<double>&, hipStream_t);
template void orig_prepare<float>(const P4<float>*, int, double, char*, const OrigLayout&,
                                  hipStream_t);
template void orig_prepare<double>(const P4<double>*, int, double, char*, const OrigLayout&,
                                   hipStream_t);

}  // namespace fcpd
