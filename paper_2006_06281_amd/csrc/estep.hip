// E-step of (Fast) CPD on gfx950: the posterior of eq. 4 with the outlier
// term, and the row normalisation of eq. 5, reduced to the per-row and
// per-column quantities the M-step and the sigma^2 update need.  The M x N
// posterior is never stored.
//
// Exponents are kept in base 2 on prescaled coordinates: with
// kappa = log2(e)/(2 sigma^2) and x^ = sqrt(kappa) x, eq. 4's Gaussian is
// 2^(-|y^_n - x^_m|^2), so each pair costs three differences, three
// multiply-adds and one v_exp_f32.
//
// Pass A (columns): L_n = log2 d_n, d_n = sum_m 2^(-|y^_n - x^_m|^2) + c,
//   measured from a fixed reference ref = max(log2 c, -100).  The outlier
//   sink makes the fixed reference exact: every term is <= 2^(-ref) and a
//   term that underflows is < 2^-126 * c <= 2^-126 * d_n.  Columns whose sum
//   still falls below 2^-60 of the reference (only possible with w = 0 or an
//   extreme c) are recomputed exactly, with their own maximum, by their
//   wave inside the column merge.
// Pass B (rows): p_mn = 2^(-|y^_n - x^_m|^2 - L_n) <= 1; per row m it sums
//   r_m = sum_n p_mn (P1, eq. 21), sum_n p_mn (y^_n - x^_m) (gives P'Y of
//   eq. 5 relative to the point itself) and sum_n p_mn |y^_n - x^_m|^2.
//   Rows whose r_m underflows (a model point far from every scene point) are
//   recomputed exactly inside the row merge, shifted by the row's own
//   maximum -- the constrained posterior p'_mn = p_mn / r_m is then still
//   defined.
//
// Both passes split the long reduction axis over blockIdx.y so a launch has
// thousands of workgroups; partial sums go to a [split][...] buffer and are
// merged in a fixed order (deterministic, no float atomics).
#include "bf16x_feat.hpp"
#include "common.hpp"
#include "kernels.hpp"

namespace fcpd {

// ---------------------------------------------------------------- prescale
template <typename T>
__device__ __forceinline__ P4<T> prescale_point(const P4<T>& p, T s) {
  return P4<T>{p.x * s, p.y * s, p.z * s, (T)0};
}

template <typename T>
__device__ __forceinline__ void prescale_body(const P4<T>* __restrict__ Xt,
                                                  const P4<T>* __restrict__ Y,
                                                  P4<T>* __restrict__ xs,
                                                  P4<T>* __restrict__ ys, int M, int N,
                                                  DevScalars* sc, int gate, int bx_, int by_, int gx_) {
  if (gate && sc->done) return;
  const T s = (T)sqrt(kappa_of(sc->sigma2));
  const int i = bx_ * blockDim.x + threadIdx.x;
  if (i < M) {
    xs[i] = prescale_point<T>(Xt[i], s);
  } else if (i < M + N) {
    ys[i - M] = prescale_point<T>(Y[i - M], s);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_prescale(const P4<T>* __restrict__ Xt,
                                                  const P4<T>* __restrict__ Y,
                                                  P4<T>* __restrict__ xs,
                                                  P4<T>* __restrict__ ys, int M, int N,
                                                  DevScalars* sc, int gate) {
  prescale_body<T>(Xt, Y, xs, ys, M, N, sc, gate, blockIdx.x, blockIdx.y, gridDim.x);
}

template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, kWave));
  return v;
}

// Prescale plus the bounding box of every 64-point tile of the prescaled
// model and scene.  Threads [0, M64) cover the model (M64 = M rounded up to
// 64), the rest the scene, so every wave sits inside one tile.
template <typename T>
__device__ __forceinline__ void prescale_box_body(const P4<T>* __restrict__ Xt,
                                                  const P4<T>* __restrict__ Y,
                                                  P4<T>* __restrict__ xs,
                                                  P4<T>* __restrict__ ys, int M, int N,
                                                  DevScalars* sc, int gate,
                                                  P4<T>* __restrict__ boxX,
                                                  P4<T>* __restrict__ boxY, int bx_) {
  if (gate && sc->done) return;
  const T s = (T)sqrt(kappa_of(sc->sigma2));
  const int i = bx_ * blockDim.x + threadIdx.x;
  const int M64 = (M + 63) & ~63;
  const bool isX = i < M64;
  const int k = isX ? i : i - M64;
  const bool valid = k < (isX ? M : N);
  const T inf = (T)__builtin_inf();
  T lx = inf, ly = inf, lz = inf, hx = -inf, hy = -inf, hz = -inf, n2 = 0;
  if (valid) {
    const P4<T> q = prescale_point<T>(isX ? Xt[k] : Y[k], s);
    if (isX)
      xs[k] = q;
    else
      ys[k] = q;
    lx = hx = q.x;
    ly = hy = q.y;
    lz = hz = q.z;
    n2 = q.x * q.x + q.y * q.y + q.z * q.z;
  }
  lx = wave_min(lx);
  ly = wave_min(ly);
  lz = wave_min(lz);
  hx = wave_max(hx);
  hy = wave_max(hy);
  hz = wave_max(hz);
  n2 = wave_max(n2);
  if ((threadIdx.x & 63) == 0 && valid) {
    P4<T>* box = isX ? boxX : boxY;
    const int t = k >> 6;
    box[2 * t] = P4<T>{lx, ly, lz, (T)0};
    box[2 * t + 1] = P4<T>{hx, hy, hz, n2};
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_prescale_box(const P4<T>* __restrict__ Xt,
                                                      const P4<T>* __restrict__ Y,
                                                      P4<T>* __restrict__ xs,
                                                      P4<T>* __restrict__ ys, int M, int N,
                                                      DevScalars* sc, int gate,
                                                      P4<T>* __restrict__ boxX,
                                                      P4<T>* __restrict__ boxY) {
  prescale_box_body<T>(Xt, Y, xs, ys, M, N, sc, gate, boxX, boxY, blockIdx.x);
}

// ------------------------------------------------------------------ pass A
template <typename T, int D>
__device__ __forceinline__ T sq3(const P4<T>& a, T bx, T by, T bz, T init) {
  T dx = a.x - bx;
  T q = fma(dx, dx, init);
  if (D > 1) {
    T dy = a.y - by;
    q = fma(dy, dy, q);
  }
  if (D > 2) {
    T dz = a.z - bz;
    q = fma(dz, dz, q);
  }
  return q;
}

// part[split * N + n] = sum over this split's model points (every S-th
// 64-point tile from tile `split`) of 2^(-(|y^_n - x^_m|^2 + ref)).  A wave
// owns 64 NB consecutive scene points (lane + 64 j); with boxes it skips
// every model tile whose smallest exponent against the wave's tiles reaches
// CullLimit (all its terms are +0).
template <typename T, int D, int NB>
__device__ __forceinline__ void colsum_body(const P4<T>* __restrict__ xs,
                                                const P4<T>* __restrict__ ys, int M, int N,
                                                int S, const DevScalars* __restrict__ sc,
                                                double w, T* __restrict__ part,
                                                const P4<T>* __restrict__ boxX,
                                                const P4<T>* __restrict__ boxY, int gate,
                                                int bx_, int by_, int gx_) {
  if (gate && sc->done) return;
  const double l2c = log2_c(sc->sigma2, D, w, M, N);
  const T ref = (T)fmax(l2c, kRefFloor);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw0 = bx_ * (256 * NB) + wave * (64 * NB);
  if (nw0 >= N) return;  // padding only: nothing of it is stored
  const int tiles = (M + 63) >> 6;
  T yx[NB], yy[NB], yz[NB], s[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int n = nw0 + 64 * j + lane;
    P4<T> p = n < N ? ys[n] : P4<T>{(T)0, (T)0, (T)0, (T)0};
    yx[j] = p.x;
    yy[j] = p.y;
    yz[j] = p.z;
    s[j] = (T)0;
  }
  const bool cull = boxX != nullptr && nw0 < N &&
                    cull_worthwhile(sc, (double)ref, (double)CullLimit<T>::value);
  P4<T> blo{}, bhi{};
  if (cull) {
    const int t0 = nw0 >> 6, t1 = min((N + 63) >> 6, t0 + NB);
    blo = boxY[2 * t0];
    bhi = boxY[2 * t0 + 1];
    for (int t = t0 + 1; t < t1; ++t) {
      const P4<T> lo = boxY[2 * t], hi = boxY[2 * t + 1];
      blo = P4<T>{fmin(blo.x, lo.x), fmin(blo.y, lo.y), fmin(blo.z, lo.z), (T)0};
      bhi = P4<T>{fmax(bhi.x, hi.x), fmax(bhi.y, hi.y), fmax(bhi.z, hi.z), fmax(bhi.w, hi.w)};
    }
  }
  const T lim = CullLimit<T>::value - ref;
  // in groups of 64 tiles: one lane tests one tile's box, a ballot gives the
  // tiles to evaluate
  for (int i0 = 0; by_ + S * i0 < tiles; i0 += 64) {
    const int t0 = by_ + S * i0;
    const int ntiles = min(64, (tiles - t0 + S - 1) / S);
    uint64_t keep = ntiles == 64 ? ~0ull : ((1ull << ntiles) - 1);
    if (cull) {
      bool kp = false;
      if (lane < ntiles) {
        const int t = t0 + S * lane;
        kp = box_gap2(boxX[2 * t], boxX[2 * t + 1], blo, bhi) < lim;
      }
      keep = __ballot(kp);
    }
    while (keep) {
      const int mt = 64 * (t0 + S * __builtin_ctzll(keep));
      keep &= keep - 1;
      const int me = min(M, mt + 64);
      int m = mt;
      for (; m + 4 <= me; m += 4) {
        P4<T> a0 = xs[m], a1 = xs[m + 1], a2 = xs[m + 2], a3 = xs[m + 3];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          T e0 = fexp2(-sq3<T, D>(a0, yx[j], yy[j], yz[j], ref));
          T e1 = fexp2(-sq3<T, D>(a1, yx[j], yy[j], yz[j], ref));
          T e2 = fexp2(-sq3<T, D>(a2, yx[j], yy[j], yz[j], ref));
          T e3 = fexp2(-sq3<T, D>(a3, yx[j], yy[j], yz[j], ref));
          s[j] += (e0 + e1) + (e2 + e3);
        }
      }
      for (; m < me; ++m) {
        P4<T> a0 = xs[m];
#pragma unroll
        for (int j = 0; j < NB; ++j) s[j] += fexp2(-sq3<T, D>(a0, yx[j], yy[j], yz[j], ref));
      }
    }
  }
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int n = nw0 + 64 * j + lane;
    if (n < N) part[(size_t)by_ * N + n] = s[j];
  }
}

template <typename T, int D, int NB>
__global__ __launch_bounds__(256) void k_colsum(const P4<T>* __restrict__ xs,
                                                const P4<T>* __restrict__ ys, int M, int N,
                                                const DevScalars* __restrict__ sc,
                                                double w, T* __restrict__ part,
                                                const P4<T>* __restrict__ boxX,
                                                const P4<T>* __restrict__ boxY, int gate) {
  colsum_body<T, D, NB>(xs, ys, M, N, gridDim.y, sc, w, part, boxX, boxY, gate, blockIdx.x,
                        blockIdx.y, gridDim.x);
}

// Exact L_n of one scene point y by the whole wave: two sweeps over all
// model points, the first for the column maximum, the second for the
// shifted sum.  Every lane returns the same value.
template <typename T, int D>
__device__ double exact_col_L(const P4<T>* __restrict__ xs, const P4<T> y, int M, double l2c) {
  const int lane = threadIdx.x & 63;
  double mx = l2c;
  for (int m = lane; m < M; m += 64) mx = fmax(mx, -(double)sq3<T, D>(xs[m], y.x, y.y, y.z, (T)0));
  mx = wave_max(mx);
  double s = 0.0;
  for (int m = lane; m < M; m += 64) s += exp2(-(double)sq3<T, D>(xs[m], y.x, y.y, y.z, (T)0) - mx);
  s = wave_sum(s) + exp2(l2c - mx);
  return mx + log2(s);
}

template <typename T>
__device__ double exact_col_L(const P4<T>* __restrict__ xs, const P4<T> y, int M, double l2c,
                              int D) {
  switch (D) {
    case 1: return exact_col_L<T, 1>(xs, y, M, l2c);
    case 2: return exact_col_L<T, 2>(xs, y, M, l2c);
    default: return exact_col_L<T, 3>(xs, y, M, l2c);
  }
}

// L_n = ref + log2(sum_splits part + 2^(log2 c - ref)) into ys[n].w, and a
// per-block partial of sum_n ln d_n.  A column whose sum falls below 2^-60
// of the reference takes the exact path: its wave computes it here, all
// lanes together, one such column after another (rare: w = 0 or an
// extreme c; it costs nothing when no column needs it).
template <typename T>
__device__ __forceinline__ void colmerge_body(const T* __restrict__ part, int splits,
                                                  P4<T>* __restrict__ ys, T* __restrict__ logd_out,
                                                  int M, int N, int D, DevScalars* sc, double w,
                                                  double* __restrict__ llpart,
                                                  P4<T>* __restrict__ boxY, int box_shift,
                                                  __bf16* __restrict__ featL,
                                                  const P4<T>* __restrict__ xs, int gate,
                                                  int bx_, int by_, int gx_) {
  __shared__ double sh[16];
  if (gate && sc->done) return;
  const double l2c = log2_c(sc->sigma2, D, w, M, N);
  const double refd = fmax(l2c, kRefFloor);
  const T ref = (T)refd;
  const int n = bx_ * blockDim.x + threadIdx.x;
  double ln_d = 0.0;
  T lmin = (T)__builtin_inf();
  T L = (T)0;
  bool bad = false;
  if (n < N) {
    T s = (T)0;
    // unrolled so that several splits' loads are in flight (the sum keeps
    // its order)
#pragma unroll 8
    for (int k = 0; k < splits; ++k) s += part[(size_t)k * N + n];
    s += (T)exp2(l2c - refd);  // the outlier sink c, relative to ref (0 if w = 0)
    L = ref + flog2(s);
    bad = !(s >= (T)0x1p-60) || !isfinite(L);
  }
  {
    const int lane = threadIdx.x & 63;
    for (uint64_t bm = __ballot(bad); bm; bm &= bm - 1) {
      const int j = __builtin_ctzll(bm);
      const double Lx = exact_col_L<T>(xs, ys[n - lane + j], M, l2c, D);
      if (lane == j) L = (T)Lx;
    }
  }
  if (n < N) {
    ys[n].w = L;
    if (logd_out) logd_out[n] = (T)((double)L * kLn2);
    if constexpr (sizeof(T) == 4) {  // BF16X: the scene features of pass B
      if (featL) {
        const P4<T> y = ys[n];
        scene_feat(P4<float>{y.x, y.y, y.z, L}, true, L, featL + (size_t)n * 32);
      }
    }
    ln_d = (double)L * kLn2;
    lmin = isfinite(L) ? L : -(T)__builtin_inf();
  }
  if (boxY) {  // min over the 2^box_shift columns of the tile (4 or 6)
    for (int o = 1 << (box_shift - 1); o > 0; o >>= 1) lmin = fmin(lmin, __shfl_xor(lmin, o, kWave));
    if ((threadIdx.x & ((1 << box_shift) - 1)) == 0 && n < N) boxY[2 * (n >> box_shift)].w = lmin;
  }
  const double b = block_sum_d(ln_d, sh);
  if (threadIdx.x == 0) llpart[bx_] = b;
}

template <typename T>
__global__ __launch_bounds__(256) void k_colmerge(const T* __restrict__ part, int splits,
                                                  P4<T>* __restrict__ ys, T* __restrict__ logd_out,
                                                  int M, int N, int D, DevScalars* sc, double w,
                                                  double* __restrict__ llpart,
                                                  P4<T>* __restrict__ boxY, int box_shift,
                                                  __bf16* __restrict__ featL,
                                                  const P4<T>* __restrict__ xs, int gate) {
  colmerge_body<T>(part, splits, ys, logd_out, M, N, D, sc, w, llpart, boxY, box_shift, featL, xs,
                   gate, blockIdx.x, blockIdx.y, gridDim.x);
}

// ------------------------------------------------------------------ pass B
// part layout: [split][5][M]: r, sum p dx, sum p dy, sum p dz, sum p d2
// (prescaled differences y^_n - x^_m).  A wave owns 64 NB consecutive model
// points (lane + 64 j); with boxes it skips every 64-point scene tile whose
// smallest exponent |y^ - x^|^2 + min L_n against the wave's tiles reaches
// CullLimit (all its terms are +0).
template <typename T, int D, int NB>
__device__ __forceinline__ void rowsum_body(const P4<T>* __restrict__ xs,
                                                const P4<T>* __restrict__ ys, int M, int N,
                                                int S, const DevScalars* __restrict__ sc,
                                                T* __restrict__ part,
                                                const P4<T>* __restrict__ boxX,
                                                const P4<T>* __restrict__ boxY, int gate,
                                                int bx_, int by_, int gx_) {
  if (gate && sc->done) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int mw0 = bx_ * (256 * NB) + wave * (64 * NB);
  if (mw0 >= M) return;  // padding only: nothing of it is stored
  const int tiles = (N + 63) >> 6;
  T ax[NB], ay[NB], az[NB], r[NB], px[NB], py[NB], pz[NB], t[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int m = mw0 + 64 * j + lane;
    P4<T> p = m < M ? xs[m] : P4<T>{(T)0, (T)0, (T)0, (T)0};
    ax[j] = p.x;
    ay[j] = p.y;
    az[j] = p.z;
    r[j] = px[j] = py[j] = pz[j] = t[j] = (T)0;
  }
  // (the gate takes L_n ~ 0: it only decides whether checking can pay)
  const bool cull = boxX != nullptr && mw0 < M &&
                    cull_worthwhile(sc, 0.0, (double)CullLimit<T>::value);
  P4<T> alo{}, ahi{};
  if (cull) {
    const int t0 = mw0 >> 6, t1 = min((M + 63) >> 6, t0 + NB);
    alo = boxX[2 * t0];
    ahi = boxX[2 * t0 + 1];
    for (int k = t0 + 1; k < t1; ++k) {
      const P4<T> lo = boxX[2 * k], hi = boxX[2 * k + 1];
      alo = P4<T>{fmin(alo.x, lo.x), fmin(alo.y, lo.y), fmin(alo.z, lo.z), (T)0};
      ahi = P4<T>{fmax(ahi.x, hi.x), fmax(ahi.y, hi.y), fmax(ahi.z, hi.z), fmax(ahi.w, hi.w)};
    }
  }
  // in groups of 64 tiles: one lane tests one tile's box, a ballot gives the
  // tiles to evaluate
  for (int i0 = 0; by_ + S * i0 < tiles; i0 += 64) {
    const int t0 = by_ + S * i0;
    const int ntiles = min(64, (tiles - t0 + S - 1) / S);
    uint64_t keep = ntiles == 64 ? ~0ull : ((1ull << ntiles) - 1);
    if (cull) {
      bool kp = false;
      if (lane < ntiles) {
        const int k = t0 + S * lane;
        const P4<T> lo = boxY[2 * k];  // lo.w = min L_n of the tile
        kp = box_gap2(alo, ahi, lo, boxY[2 * k + 1]) + lo.w < CullLimit<T>::value;
      }
      keep = __ballot(kp);
    }
    while (keep) {
      const int nt = 64 * (t0 + S * __builtin_ctzll(keep));
      keep &= keep - 1;
      const int nE = min(N, nt + 64);
      for (int n = nt; n < nE; ++n) {
        const P4<T> y = ys[n];  // (x^, y^, z^, L_n)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          const T dx = y.x - ax[j];
          T d2 = dx * dx;
          T dy = (T)0, dz = (T)0;
          if (D > 1) {
            dy = y.y - ay[j];
            d2 = fma(dy, dy, d2);
          }
          if (D > 2) {
            dz = y.z - az[j];
            d2 = fma(dz, dz, d2);
          }
          const T e = fexp2(-(d2 + y.w));
          r[j] += e;
          px[j] = fma(e, dx, px[j]);
          if (D > 1) py[j] = fma(e, dy, py[j]);
          if (D > 2) pz[j] = fma(e, dz, pz[j]);
          t[j] = fma(e, d2, t[j]);
        }
      }
    }
  }
  T* base = part + (size_t)by_ * 5 * M;
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int m = mw0 + 64 * j + lane;
    if (m < M) {
      base[m] = r[j];
      base[(size_t)M + m] = px[j];
      base[(size_t)2 * M + m] = py[j];
      base[(size_t)3 * M + m] = pz[j];
      base[(size_t)4 * M + m] = t[j];
    }
  }
}

template <typename T, int D, int NB>
__global__ __launch_bounds__(256) void k_rowsum(const P4<T>* __restrict__ xs,
                                                const P4<T>* __restrict__ ys, int M, int N,
                                                const DevScalars* __restrict__ sc,
                                                T* __restrict__ part,
                                                const P4<T>* __restrict__ boxX,
                                                const P4<T>* __restrict__ boxY, int gate) {
  rowsum_body<T, D, NB>(xs, ys, M, N, gridDim.y, sc, part, boxX, boxY, gate, blockIdx.x,
                        blockIdx.y, gridDim.x);
}

// Exact pass B of one model row m by the whole wave: shift by the row
// maximum of -(|y^_n - x^_m|^2 + L_n), then the sums r, p (y^ - x^), p d2.
// Every lane returns the same values; P1_m = r 2^mx.
template <typename T, int D>
__device__ void exact_row(const P4<T>* __restrict__ xs, const P4<T>* __restrict__ ys, int m,
                          int N, double& r, double& px, double& py, double& pz, double& t,
                          double& mx) {
  const int lane = threadIdx.x & 63;
  const P4<T> a = xs[m];
  mx = -__builtin_inf();
  for (int n = lane; n < N; n += 64) {
    const P4<T> y = ys[n];
    mx = fmax(mx, -((double)sq3<T, D>(a, y.x, y.y, y.z, (T)0) + (double)y.w));
  }
  mx = wave_max(mx);
  r = px = py = pz = t = 0.0;
  for (int n = lane; n < N; n += 64) {
    const P4<T> y = ys[n];
    const double dx = (double)y.x - a.x;
    const double dy = D > 1 ? (double)y.y - a.y : 0.0;
    const double dz = D > 2 ? (double)y.z - a.z : 0.0;
    const double d2 = dx * dx + dy * dy + dz * dz;
    const double e = exp2(-(d2 + (double)y.w) - mx);
    r += e;
    px += e * dx;
    py += e * dy;
    pz += e * dz;
    t += e * d2;
  }
  r = wave_sum(r);
  px = wave_sum(px);
  py = wave_sum(py);
  pz = wave_sum(pz);
  t = wave_sum(t);
}

// Row m's outputs from the exact (shifted, well-scaled) sums: P1 keeps its
// true (tiny or zero) value, Yt and tbar come from the shifted sums.
template <typename T>
__device__ __forceinline__ void store_exact_row(const P4<T>* __restrict__ Xt,
                                                P4<T>* __restrict__ Yt, T* __restrict__ P1,
                                                T* __restrict__ tbar, int m, double kap,
                                                double r, double px, double py, double pz,
                                                double t, double mx) {
  const double isk = 1.0 / sqrt(kap);
  const P4<T> x = Xt[m];
  Yt[m] = P4<T>{(T)(x.x + px / r * isk), (T)(x.y + py / r * isk), (T)(x.z + pz / r * isk), (T)0};
  P1[m] = (T)(r * exp2(mx));
  tbar[m] = (T)(t / r / kap);
}

// Row merge: P1_m = r_m, Yt_m = xt_m + (sum p (y - xt)) / r_m, tbar_m.
// relative = 1: the sums hold p (y^ - x^) (direct-difference pass B);
// relative = 0: they hold p y^ (absolute, the matrix-core pass B).
// A row whose r_m underflows takes the exact path: its wave computes it
// here, one such row after another.
template <typename T>
__device__ __forceinline__ void rowmerge_body(const T* __restrict__ part, int splits,
                                                  const P4<T>* __restrict__ Xt,
                                                  P4<T>* __restrict__ Yt, T* __restrict__ P1,
                                                  T* __restrict__ tbar, int M, DevScalars* sc,
                                                  int relative, const P4<T>* __restrict__ xs,
                                                  const P4<T>* __restrict__ ys, int N, int D,
                                                  int gate, int bx_, int by_, int gx_) {
  if (gate && sc->done) return;
  const int m = bx_ * blockDim.x + threadIdx.x;
  const double kap = kappa_of(sc->sigma2);
  T r = 0, px = 0, py = 0, pz = 0, t = 0;
  if (m < M) {
#pragma unroll 4
    for (int k = 0; k < splits; ++k) {
      const T* b = part + (size_t)k * 5 * M;
      r += b[m];
      px += b[(size_t)M + m];
      py += b[(size_t)2 * M + m];
      pz += b[(size_t)3 * M + m];
      t += b[(size_t)4 * M + m];
    }
  }
  const bool tiny = m < M && !(r >= (T)(sizeof(T) == 4 ? 0x1p-60 : 0x1p-900));
  {
    const int lane = threadIdx.x & 63;
    for (uint64_t bm = __ballot(tiny); bm; bm &= bm - 1) {
      const int j = __builtin_ctzll(bm);
      const int mj = m - lane + j;
      double er, ex, ey, ez, et, mx;
      switch (D) {
        case 1: exact_row<T, 1>(xs, ys, mj, N, er, ex, ey, ez, et, mx); break;
        case 2: exact_row<T, 2>(xs, ys, mj, N, er, ex, ey, ez, et, mx); break;
        default: exact_row<T, 3>(xs, ys, mj, N, er, ex, ey, ez, et, mx); break;
      }
      if (lane == j) store_exact_row<T>(Xt, Yt, P1, tbar, mj, kap, er, ex, ey, ez, et, mx);
    }
    if (tiny || m >= M) return;
  }
  const T inv = (T)1 / r;
  const T isk = (T)(1.0 / sqrt(kap));
  P4<T> x = Xt[m];
  if (!relative) x = P4<T>{(T)0, (T)0, (T)0, (T)0};
  Yt[m] = P4<T>{x.x + px * inv * isk, x.y + py * inv * isk, x.z + pz * inv * isk, (T)0};
  P1[m] = r;
  tbar[m] = t * inv * (T)(1.0 / kap);
}

template <typename T>
__global__ __launch_bounds__(256) void k_rowmerge(const T* __restrict__ part, int splits,
                                                  const P4<T>* __restrict__ Xt,
                                                  P4<T>* __restrict__ Yt, T* __restrict__ P1,
                                                  T* __restrict__ tbar, int M, DevScalars* sc,
                                                  int relative, const P4<T>* __restrict__ xs,
                                                  const P4<T>* __restrict__ ys, int N, int D,
                                                  int gate) {
  rowmerge_body<T>(part, splits, Xt, Yt, P1, tbar, M, sc, relative, xs, ys, N, D, gate, blockIdx.x,
                   blockIdx.y, gridDim.x);
}

// ------------------------------------------------------------- launchers
template <typename T> void prescale_launch(const EStepArgs<T>& a, hipStream_t st) {
  if (a.boxX) {
    const int nthr = ((a.M + 63) & ~63) + a.N;
    hipLaunchKernelGGL(k_prescale_box<T>, dim3((nthr + 255) / 256), dim3(256), 0, st, a.Xt, a.Y,
                       a.xs, a.ys, a.M, a.N, a.sc, a.gate, a.boxX, a.boxY);
    return;
  }
  const int nthr = a.M + a.N;
  hipLaunchKernelGGL(k_prescale<T>, dim3((nthr + 255) / 256), dim3(256), 0, st, a.Xt, a.Y, a.xs,
                     a.ys, a.M, a.N, a.sc, a.gate);
}

template <typename T> void colmerge_fix_launch(const EStepArgs<T>& a, hipStream_t st) {
  const int gate = a.gate;
  // the exact path for underflowed columns runs inside the merge
  hipLaunchKernelGGL(k_colmerge<T>, dim3((a.N + 255) / 256), dim3(256), 0, st, a.partA, a.splitsA,
                     a.ys, a.logd_out, a.M, a.N, a.D, a.sc, a.w, a.llpart, a.boxY, a.box_shift,
                     a.featY_L, (const P4<T>*)a.xs, gate);
}

template <typename T>
void rowmerge_fix_launch(const EStepArgs<T>& a, hipStream_t st, int relative) {
  const int gate = a.gate;
  // the exact path for underflowed rows runs inside the merge
  hipLaunchKernelGGL(k_rowmerge<T>, dim3((a.M + 255) / 256), dim3(256), 0, st, a.partB, a.splitsB,
                     a.Xt, a.Yt, a.P1, a.tbar, a.M, a.sc, relative, (const P4<T>*)a.xs,
                     (const P4<T>*)a.ys, a.N, a.D, gate);
}

template <typename T>
void estep_launch(const EStepArgs<T>& a, hipStream_t st) {
  constexpr int NB = sizeof(T) == 4 ? 4 : 2;
  const int gate = a.gate;
  prescale_launch<T>(a, st);
  if (a.ev) (void)hipEventRecord(a.ev[0], st);
  {
    const int tiles = (a.N + 256 * NB - 1) / (256 * NB);
    dim3 grid(tiles, a.splitsA);
    switch (a.D) {
      case 1: hipLaunchKernelGGL((k_colsum<T, 1, NB>), grid, dim3(256), 0, st, a.xs, a.ys, a.M, a.N, a.sc, a.w, a.partA, a.boxX, a.boxY, gate); break;
      case 2: hipLaunchKernelGGL((k_colsum<T, 2, NB>), grid, dim3(256), 0, st, a.xs, a.ys, a.M, a.N, a.sc, a.w, a.partA, a.boxX, a.boxY, gate); break;
      default: hipLaunchKernelGGL((k_colsum<T, 3, NB>), grid, dim3(256), 0, st, a.xs, a.ys, a.M, a.N, a.sc, a.w, a.partA, a.boxX, a.boxY, gate); break;
    }
  }
  if (a.ev) (void)hipEventRecord(a.ev[1], st);
  colmerge_fix_launch<T>(a, st);
  if (a.ev) (void)hipEventRecord(a.ev[2], st);
  {
    const int tiles = (a.M + 256 * NB - 1) / (256 * NB);
    dim3 grid(tiles, a.splitsB);
    switch (a.D) {
      case 1: hipLaunchKernelGGL((k_rowsum<T, 1, NB>), grid, dim3(256), 0, st, a.xs, a.ys, a.M, a.N, a.sc, a.partB, a.boxX, a.boxY, gate); break;
      case 2: hipLaunchKernelGGL((k_rowsum<T, 2, NB>), grid, dim3(256), 0, st, a.xs, a.ys, a.M, a.N, a.sc, a.partB, a.boxX, a.boxY, gate); break;
      default: hipLaunchKernelGGL((k_rowsum<T, 3, NB>), grid, dim3(256), 0, st, a.xs, a.ys, a.M, a.N, a.sc, a.partB, a.boxX, a.boxY, gate); break;
    }
  }
  if (a.ev) (void)hipEventRecord(a.ev[3], st);
  rowmerge_fix_launch<T>(a, st, 1);
  if (a.ev) (void)hipEventRecord(a.ev[4], st);
}

template <typename T>
void estep_splits(int M, int N, int* splitsA, int* chunkA, int* splitsB, int* chunkB) {
  constexpr int NB = sizeof(T) == 4 ? 4 : 2;
  const int target = 4096;
  auto plan = [&](int cols, int len, int* splits, int* chunk) {
    const int tiles = (cols + 256 * NB - 1) / (256 * NB);
    int s = (target + tiles - 1) / tiles;
    const int smax = (len + 63) / 64;  // at least 64 reduction steps per split
    s = s < 1 ? 1 : (s > smax ? smax : s);
    int c = (len + s - 1) / s;
    c = (c + 63) & ~63;  // whole 64-point tiles per split (a split takes every S-th tile)
    *chunk = c;
    *splits = (len + c - 1) / c;
  };
  plan(N, M, splitsA, chunkA);
  plan(M, N, splitsB, chunkB);
}

// ------------------------------------------------------------ batched
// The same bodies driven by a work list over every instance of a batch.
__global__ __launch_bounds__(256) void kb_prescale(const InstDesc* __restrict__ d,
                                                   const int4* __restrict__ items) {
  const int4 it = items[blockIdx.x];
  const InstDesc& D = d[it.x];
  if (D.boxX)
    prescale_box_body<float>(D.Xt, D.Y, D.xs, D.ys, D.M, D.N, D.sc, 1, D.boxX, D.boxY, it.y);
  else
    prescale_body<float>(D.Xt, D.Y, D.xs, D.ys, D.M, D.N, D.sc, 1, it.y, 0, 0);
}
// NB scene (model) points per thread: tiles of 256 NB points per block.
template <int NB>
__global__ __launch_bounds__(256) void kb_colsum(const InstDesc* __restrict__ d,
                                                 const int4* __restrict__ items) {
  const int4 it = items[blockIdx.x];
  const InstDesc& D = d[it.x];
  colsum_body<float, 3, NB>(D.xs, D.ys, D.M, D.N, D.splitsA, D.sc, D.w, D.partA, D.boxX, D.boxY,
                           1, it.y, it.z, 0);
}
__global__ __launch_bounds__(256) void kb_colmerge(const InstDesc* __restrict__ d,
                                                   const int4* __restrict__ items) {
  const int4 it = items[blockIdx.x];
  const InstDesc& D = d[it.x];
  colmerge_body<float>(D.partA, D.splitsA, D.ys, (float*)nullptr, D.M, D.N, 3, D.sc, D.w,
                       D.llpart, D.boxY, 6, (__bf16*)nullptr, D.xs, 1, it.y, 0, 0);
}
template <int NB>
__global__ __launch_bounds__(256) void kb_rowsum(const InstDesc* __restrict__ d,
                                                 const int4* __restrict__ items) {
  const int4 it = items[blockIdx.x];
  const InstDesc& D = d[it.x];
  rowsum_body<float, 3, NB>(D.xs, D.ys, D.M, D.N, D.splitsB, D.sc, D.partB, D.boxX, D.boxY, 1,
                           it.y, it.z, 0);
}
__global__ __launch_bounds__(256) void kb_rowmerge(const InstDesc* __restrict__ d,
                                                   const int4* __restrict__ items) {
  const int4 it = items[blockIdx.x];
  const InstDesc& D = d[it.x];
  rowmerge_body<float>(D.partB, D.splitsB, D.Xt, D.Yt, D.P1, D.tbar, D.M, D.sc, 1, D.xs, D.ys,
                       D.N, 3, 1, it.y, 0, 0);
}
void batch_estep_launch(const InstDesc* d, const BatchItems& it, hipStream_t st) {
  hipLaunchKernelGGL(kb_prescale, dim3(it.n_prescale), dim3(256), 0, st, d, it.prescale);
  if (it.nb == 2)
    hipLaunchKernelGGL(kb_colsum<2>, dim3(it.n_colsum), dim3(256), 0, st, d, it.colsum);
  else
    hipLaunchKernelGGL(kb_colsum<4>, dim3(it.n_colsum), dim3(256), 0, st, d, it.colsum);
  hipLaunchKernelGGL(kb_colmerge, dim3(it.n_colmerge), dim3(256), 0, st, d, it.colmerge);
  if (it.nb == 2)
    hipLaunchKernelGGL(kb_rowsum<2>, dim3(it.n_rowsum), dim3(256), 0, st, d, it.rowsum);
  else
    hipLaunchKernelGGL(kb_rowsum<4>, dim3(it.n_rowsum), dim3(256), 0, st, d, it.rowsum);
  hipLaunchKernelGGL(kb_rowmerge, dim3(it.n_rowmerge), dim3(256), 0, st, d, it.rowmerge);
}

template void estep_launch<float>(const EStepArgs<float>&, hipStream_t);
template void estep_launch<double>(const EStepArgs<double>&, hipStream_t);
template void colmerge_fix_launch<float>(const EStepArgs<float>&, hipStream_t);
template void rowmerge_fix_launch<float>(const EStepArgs<float>&, hipStream_t, int);
template void estep_splits<float>(int, int, int*, int*, int*, int*);
template void estep_splits<double>(int, int, int*, int*, int*, int*);

}  // namespace fcpd
