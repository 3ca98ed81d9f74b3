// BF16X precision mode of the E-step: the squared distances of eq. 4 come
// from the matrix cores (bf16 operands, fp32 accumulation), the exponentials
// and sums stay in fp32 on the VALU.
//
// |u - v|^2 = |u|^2 + |v|^2 - 2 u.v is one dot product of two 32-slot feature
// vectors per point.  Each fp32 coordinate is split into three bf16 pieces
// u = u1 + u2 + u3 (u1 = bf16(u), u2 = bf16(u - u1), u3 = bf16(u - u1 - u2),
// 24 significant bits in total), and the cross term keeps the six products
// u1v1, u1v2, u2v1, u1v3, u2v2, u3v1, dropping terms below 2^-24 relative
// (the split-precision scheme of Henry, Tang & Heinecke, "Leveraging the
// bfloat16 artificial intelligence datatype for higher-precision
// computations", ARITH 2019).  Norms (and the per-column offset: the pass-A
// reference, or L_n = log2 d_n in pass B) enter as three bf16 pieces times 1.
//   model   F(u) = [u1 u1 u2 u1 u2 u3]xyz, |u|^2 (3 pieces), 1 1 1, 0...
//   scene   G(v) = -2[v1 v2 v1 v3 v2 v1]xyz, 1 1 1, |v|^2 + extra (3 pieces), 0...
// so F(u).G(v) = |u - v|^2 + extra in prescaled units (base-2 exponent).
// The remaining error is the fp32 accumulation of terms of size ~kappa |x|^2,
// about 2^-23 * 3 kappa max|x|^2 in the exponent.
//
// v_mfma_f32_16x16x32_bf16 layout (checked on the device): A lane l holds
// row l%16, k = 8(l/16)..+7; B lane l holds column l%16, the same k slice;
// D lane l holds rows 4(l/16)..+3 of column l%16.  A feature vector is 64
// bytes, so a lane's operand is the 16-byte slice (l/16) of point l%16.
//
// Pass A: a wave keeps four 16-column scene tiles (B operands) in registers
// and streams 16-point model tiles (A); per pair: one v_exp_f32 and one add.
// Pass B: a wave keeps four 16-point model tiles (B) and streams scene tiles
// (A, extra = L_n); per pair: exp, and the sums of p, p*v, p*|u - v|^2 as a
// second matrix product with p as its A operand.
// Padded points carry a 3e30 offset so their exponentials are exactly 0.
#include "bf16x_feat.hpp"
#include "common.hpp"
#include "kernels.hpp"

namespace fcpd {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// The iteration's first kernel in this mode: prescale (xs, ys), the boxes of
// 16-point tiles when culling is on, the model features,
// the scene features with the pass-A reference and pass B's sum operands.
// Threads [0, M64) cover the model rows (M64 = M rounded up to 64), the next
// Npad the scene rows (so every 16-lane group sits inside one tile), the last
// 4 Npad the sum operands (64 lanes per 16-point scene tile).
__global__ __launch_bounds__(256) void k_bfx_prescale(const P4<float>* __restrict__ Xt,
                                                      const P4<float>* __restrict__ Y,
                                                      P4<float>* __restrict__ xs,
                                                      P4<float>* __restrict__ ys, int M, int N,
                                                      int Mpad, int Npad, DevScalars* sc,
                                                      int gate, P4<float>* __restrict__ boxX,
                                                      P4<float>* __restrict__ boxY,
                                                      __bf16* __restrict__ F,
                                                      __bf16* __restrict__ G,
                                                      __bf16* __restrict__ V, double w, int D) {
  if (gate && sc->done) return;
  const float s = (float)sqrt(kappa_of(sc->sigma2));
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int M64 = (M + 63) & ~63;
  if (i >= M64 + Npad) {
    const int j = i - (M64 + Npad);
    if (j < 4 * Npad) sum_operand(Y, N, s, j >> 6, j & 63, V);
    return;
  }
  const bool isX = i < M64;
  const int k = isX ? i : i - M64;
  const bool valid = k < (isX ? M : N);
  P4<float> q{0.f, 0.f, 0.f, 0.f};
  if (valid) {
    const P4<float> p = isX ? Xt[k] : Y[k];
    q = P4<float>{p.x * s, p.y * s, p.z * s, 0.f};
    if (isX)
      xs[k] = q;
    else
      ys[k] = q;
  }
  if (isX && k < Mpad) model_feat(q, valid, F + (size_t)k * 32);
  if (!isX && k < Npad) {
    const float ref = (float)fmax(log2_c(sc->sigma2, D, w, M, N), kRefFloor);
    scene_feat(q, valid, ref, G + (size_t)k * 32);
  }
  if (boxX) {  // boxes of 16-point tiles
    const float inf = __builtin_inff();
    float lx = inf, ly = inf, lz = inf, hx = -inf, hy = -inf, hz = -inf, n2 = 0.f;
    if (valid) {
      lx = hx = q.x;
      ly = hy = q.y;
      lz = hz = q.z;
      n2 = q.x * q.x + q.y * q.y + q.z * q.z;
    }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) {
      lx = fminf(lx, __shfl_xor(lx, o, 64));
      ly = fminf(ly, __shfl_xor(ly, o, 64));
      lz = fminf(lz, __shfl_xor(lz, o, 64));
      hx = fmaxf(hx, __shfl_xor(hx, o, 64));
      hy = fmaxf(hy, __shfl_xor(hy, o, 64));
      hz = fmaxf(hz, __shfl_xor(hz, o, 64));
      n2 = fmaxf(n2, __shfl_xor(n2, o, 64));
    }
    if ((threadIdx.x & 15) == 0 && valid) {
      P4<float>* box = isX ? boxX : boxY;
      const int t = k >> 4;
      box[2 * t] = P4<float>{lx, ly, lz, 0.f};
      box[2 * t + 1] = P4<float>{hx, hy, hz, n2};
    }
  }
}

__device__ __forceinline__ bf16x8 load_op(const __bf16* __restrict__ feat, int point, int lane) {
  return *reinterpret_cast<const bf16x8*>(feat + (size_t)point * 32 + 8 * (lane >> 4));
}

// A compile-time flag passed to a generic lambda: the culled and the plain
// tile loops are compiled separately, so the plain one keeps its straight-line
// schedule.
template <bool B>
struct Flag {
  static constexpr bool value = B;
};

// Boxes of a wave's four 16-point tiles (first tile t0, `valid` of them);
// the missing ones are empty (every gap to them is infinite).
__device__ __forceinline__ void wave_boxes(const P4<float>* __restrict__ box, int t0, int valid,
                                           P4<float> lo[4], P4<float> hi[4]) {
  const float inf = __builtin_inff();
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (j < valid) {
      lo[j] = box[2 * (t0 + j)];
      hi[j] = box[2 * (t0 + j) + 1];
    } else {
      lo[j] = P4<float>{inf, inf, inf, 0.f};
      hi[j] = P4<float>{-inf, -inf, -inf, 0.f};
    }
  }
}

// Pass A partials: part[split][n] = sum over the split's model points (with
// culling every S-th 16-point tile, else a contiguous range) of
// 2^-(|u - v|^2 + ref).  Block: 4 waves x 64 scene points.  With boxes a
// wave skips every 16-point model tile whose smallest exponent against its
// 64 scene points reaches CullLimit (all its terms are +0).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_bfx_colsum(const __bf16* __restrict__ F,
                                                    const __bf16* __restrict__ G, int Mpad, int N,
                                                    const DevScalars* __restrict__ sc,
                                                    float* __restrict__ part,
                                                    const P4<float>* __restrict__ boxX,
                                                    const P4<float>* __restrict__ boxY, double w,
                                                    int M, int gate) {
  if (gate && sc->done) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n0 = blockIdx.x * 256 + wave * 64;  // this wave's 64 scene columns
  if (n0 >= N) return;  // padding only: nothing of it is stored
  // the per-column offset the scene features carry (see k_bfx_prescale)
  const float ref = (float)fmax(log2_c(sc->sigma2, 3, w, M, N), kRefFloor);
  bf16x8 b[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) b[s] = load_op(G, n0 + 16 * s + (lane & 15), lane);
  // with culling, this split's model tiles are every S-th 16-row tile from
  // tile blockIdx.y (S = gridDim.y splits): the tiles near any scene column,
  // consecutive in the spatial order, then spread evenly over the splits
  const int S = gridDim.y, tiles = Mpad >> 4;
  const int aoff = (lane & 15) * 32 + 8 * (lane >> 4);  // this lane's A operand slice
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  // the split layout follows the sigma^2 gate alone, so a handle without
  // boxes adds the same terms in the same order (culling stays bit-exact)
  const bool spread = cull_worthwhile(sc, (double)ref, (double)CullLimit<float>::value);
  const bool cull = boxX != nullptr && spread;
  const float lim = CullLimit<float>::value - ref;
  // in groups of 64 tiles: one lane tests one tile's box, a ballot gives the
  // tiles to evaluate
  // (while culling cannot pay every tile is evaluated and consecutive tiles
  // per split read better, so the split then takes a contiguous range)
  const int per = (tiles + S - 1) / S;
  const int tb = spread ? (int)blockIdx.y : (int)blockIdx.y * per, ts = spread ? S : 1;
  const int tn = spread ? (tiles - (int)blockIdx.y + S - 1) / S : min(per, tiles - tb);
  auto tiles_loop = [&](auto masked) {
    constexpr bool MASK = decltype(masked)::value;
    for (int i0 = 0; i0 < tn; i0 += 64) {
      const int t0 = tb + ts * i0;
      const int ntiles = min(64, tn - i0);
      uint64_t keep = ntiles == 64 ? ~0ull : ((1ull << ntiles) - 1);
      int cols = 15;  // per tile (lane): the column tiles it is evaluated against
      if (MASK) {
        // the wave's four 16-column tiles (reloaded per group, not held in
        // registers): a model tile is evaluated against each of them only
        // where it can contribute
        P4<float> blo[4], bhi[4];
        wave_boxes(boxY, n0 >> 4, min(4, (N - n0 + 15) >> 4), blo, bhi);
        cols = 0;
        if (lane < ntiles) {
          const int t = t0 + ts * lane;
          const P4<float> lo = boxX[2 * t], hi = boxX[2 * t + 1];
#pragma unroll
          for (int j = 0; j < 4; ++j) cols |= (box_gap2(lo, hi, blo[j], bhi[j]) < lim) << j;
        }
        keep = __ballot(cols != 0);
      }
      // kept tiles two at a time: the second tile's operand is requested
      // before the first is evaluated (tiles still added in order)
      auto eval = [&](int k, const bf16x8& a) {
        const int cm = MASK ? __builtin_amdgcn_readfirstlane(__shfl(cols, k, 64)) : 15;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          if (MASK && !(cm & (1 << s))) continue;  // all its terms are +0
          const f32x4 d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[s], zero, 0, 0, 0);
          acc[s] += (fexp2(-d[0]) + fexp2(-d[1])) + (fexp2(-d[2]) + fexp2(-d[3]));
        }
      };
      while (keep) {
        const int k0 = __builtin_ctzll(keep);
        keep &= keep - 1;
        // uniform tile bases, per-lane offsets
        const bf16x8 a0 = *reinterpret_cast<const bf16x8*>(F + (size_t)(16 * (t0 + ts * k0)) * 32 + aoff);
        if (keep) {
          const int k1 = __builtin_ctzll(keep);
          keep &= keep - 1;
          const bf16x8 a1 =
              *reinterpret_cast<const bf16x8*>(F + (size_t)(16 * (t0 + ts * k1)) * 32 + aoff);
          eval(k0, a0);
          eval(k1, a1);
        } else {
          eval(k0, a0);
        }
      }
    }
  };
  if (cull)
    tiles_loop(Flag<true>{});
  else
    tiles_loop(Flag<false>{});
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    acc[s] += __shfl_xor(acc[s], 16, 64);
    acc[s] += __shfl_xor(acc[s], 32, 64);
  }
  if (lane < 16) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int n = n0 + 16 * s + lane;
      if (n < N) part[(size_t)blockIdx.y * N + n] = acc[s];
    }
  }
}

// Pass B partials: part[split][5][M] = sum over the split's scene points
// (with culling every S-th 16-point tile, else a contiguous range) of p, p*v
// (prescaled, absolute), p*|u - v|^2 with p = 2^-(|u - v|^2 + L_n).
//
// The sums run on the matrix cores as a product P V: the distance product
// leaves lane l with p for model point l % 16 and scene points 4 (l / 16)
// .. + 3, which is the row and k slice of the A operand of a second
// 16x16x32 product once each p is split into a high and a low bf16 part
// (p - hi is exact in fp32; together they keep 16 significant bits, so each
// term carries a relative error below 2^-17).  The B operand holds, per
// scene point, 1, the three bf16 pieces of each coordinate and of |v|^2
// (`sum_operand`), so the accumulator's columns are sum p, sum p v and
// sum p |v|^2, each to 24 bits.  The epilogue forms
// sum p |u - v|^2 = sum p |v|^2 - 2 u . sum p v + |u|^2 sum p per model
// point, in FP64.  Per pair the vector ALU spends one exponential, one
// two-value conversion per pair of values (high parts), one dot2 per value
// (the low part, p - hi) and one conversion per pair of values (low parts).
__global__ __launch_bounds__(256) void k_bfx_rowsum(const __bf16* __restrict__ F,
                                                    const __bf16* __restrict__ G,
                                                    const __bf16* __restrict__ V,
                                                    const P4<float>* __restrict__ xs, int M,
                                                    int Npad, const DevScalars* __restrict__ sc,
                                                    float* __restrict__ part,
                                                    const P4<float>* __restrict__ boxX,
                                                    const P4<float>* __restrict__ boxY, int gate) {
  if (gate && sc->done) return;
  __shared__ float red[4][64 * 17];  // per wave: 64 model points x 16 columns (+1 pad)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m0 = blockIdx.x * 256 + wave * 64;  // this wave's 64 model columns
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  f32x4 acc[4] = {zero, zero, zero, zero};
  if (m0 < M) {  // (a wave of padding only skips to the block's barrier)
    bf16x8 b[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) b[s] = load_op(F, m0 + 16 * s + (lane & 15), lane);
    // with culling, this split's scene tiles are every S-th 16-row tile from
    // tile blockIdx.y (S = gridDim.y splits): the tiles near any model point,
    // consecutive in the spatial order, then spread evenly over the splits
    const int S = gridDim.y, tiles = Npad >> 4;
    const int aoff = (lane & 15) * 32 + 8 * (lane >> 4);  // this lane's A operand slice
    // p - hi(p) for the first / second value of a bf16 pair, as a dot2 with
    // the pair (-1, 0) or (0, -1).  Both are kept in registers: as an inline
    // constant the compiler encodes (-1, 0) as the operand -1.0, which the
    // hardware does not read as the bf16 pair
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    uint32_t nlo = 0x0000bf80u, nhi = 0xbf800000u;
    asm volatile("" : "+v"(nlo), "+v"(nhi));
    const bf16x2 neg_lo = __builtin_bit_cast(bf16x2, nlo), neg_hi = __builtin_bit_cast(bf16x2, nhi);
    // with boxes: skip 16-point scene tiles whose smallest exponent
    // |u - v|^2 + min L_n against this wave's model points reaches CullLimit
    // (the split layout follows the sigma^2 gate alone: see pass A)
    const bool spread = cull_worthwhile(sc, 0.0, (double)CullLimit<float>::value);
    const bool cull = boxX != nullptr && spread;
    // in groups of 64 tiles: one lane tests one tile's box, a ballot gives the
    // tiles to evaluate
    // (while culling cannot pay every tile is evaluated and consecutive tiles
    // per split read better, so the split then takes a contiguous range)
    const int per = (tiles + S - 1) / S;
    const int tb = spread ? (int)blockIdx.y : (int)blockIdx.y * per, ts = spread ? S : 1;
    const int tn = spread ? (tiles - (int)blockIdx.y + S - 1) / S : min(per, tiles - tb);
    auto tiles_loop = [&](auto masked) {
      constexpr bool MASK = decltype(masked)::value;
      for (int i0 = 0; i0 < tn; i0 += 64) {
        const int t0 = tb + ts * i0;
        const int ntiles = min(64, tn - i0);
        uint64_t keep = ntiles == 64 ? ~0ull : ((1ull << ntiles) - 1);
        int rows = 15;  // per tile (lane): the model row tiles it is evaluated against
        if (MASK) {
          // the wave's four 16-row model tiles (reloaded per group): a scene
          // tile is evaluated against each of them only where it can contribute
          P4<float> alo[4], ahi[4];
          wave_boxes(boxX, m0 >> 4, min(4, (M - m0 + 15) >> 4), alo, ahi);
          rows = 0;
          if (lane < ntiles) {
            const int k = t0 + ts * lane;
            const P4<float> lo = boxY[2 * k], hi = boxY[2 * k + 1];  // lo.w = min L_n
#pragma unroll
            for (int j = 0; j < 4; ++j)
              rows |= (box_gap2(alo[j], ahi[j], lo, hi) + lo.w < CullLimit<float>::value) << j;
          }
          keep = __ballot(rows != 0);
        }
        while (keep) {
          const int i = __builtin_ctzll(keep);
          keep &= keep - 1;
          const int nt = 16 * (t0 + ts * i);
          const int rm = MASK ? __builtin_amdgcn_readfirstlane(__shfl(rows, i, 64)) : 15;
          // the tile's bases are uniform, so only the lane offsets are per lane
          const bf16x8 a = *reinterpret_cast<const bf16x8*>(G + (size_t)nt * 32 + aoff);
          const bf16x8 v = *reinterpret_cast<const bf16x8*>(V + (size_t)nt * 32 + 8 * lane);
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            if (MASK && !(rm & (1 << s))) continue;  // all its terms are +0
            const f32x4 d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[s], zero, 0, 0, 0);
            const float p0 = fexp2(-d[0]), p1 = fexp2(-d[1]), p2 = fexp2(-d[2]), p3 = fexp2(-d[3]);
            const bf16x2 h01 = {(__bf16)p0, (__bf16)p1}, h23 = {(__bf16)p2, (__bf16)p3};
            const float l0 = __builtin_amdgcn_fdot2_f32_bf16(h01, neg_lo, p0, false);
            const float l1 = __builtin_amdgcn_fdot2_f32_bf16(h01, neg_hi, p1, false);
            const float l2 = __builtin_amdgcn_fdot2_f32_bf16(h23, neg_lo, p2, false);
            const float l3 = __builtin_amdgcn_fdot2_f32_bf16(h23, neg_hi, p3, false);
            const bf16x8 pa = {h01[0], h01[1], h23[0], h23[1],
                               (__bf16)l0, (__bf16)l1, (__bf16)l2, (__bf16)l3};
            acc[s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pa, v, acc[s], 0, 0, 0);
          }
        }
      }
    };
    if (cull)
      tiles_loop(Flag<true>{});
    else
      tiles_loop(Flag<false>{});
  }
  // accumulator lane l: column l % 16 of model points 16 s + 4 (l / 16) .. + 3
  float* r = red[wave];
  {
    const int f = lane & 15, g = lane >> 4;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int q = 0; q < 4; ++q) r[(16 * s + 4 * g + q) * 17 + f] = acc[s][q];
  }
  __syncthreads();
  const int m = m0 + lane;
  if (m < M) {
    const float* c = r + lane * 17;
    const double s0 = c[0];
    const double sx = ((double)c[3] + c[2]) + c[1];
    const double sy = ((double)c[6] + c[5]) + c[4];
    const double sz = ((double)c[9] + c[8]) + c[7];
    const double s2 = ((double)c[12] + c[11]) + c[10];
    const P4<float> u = xs[m];
    const double ux = u.x, uy = u.y, uz = u.z;
    const double t = s2 - 2.0 * (ux * sx + uy * sy + uz * sz) + (ux * ux + uy * uy + uz * uz) * s0;
    float* base = part + (size_t)blockIdx.y * 5 * M;
    base[m] = (float)s0;
    base[(size_t)M + m] = (float)sx;
    base[(size_t)2 * M + m] = (float)sy;
    base[(size_t)3 * M + m] = (float)sz;
    base[(size_t)4 * M + m] = (float)fmax(t, 0.0);  // a sum of non-negative terms
  }
}

namespace {
constexpr int kBfxTarget = 4096;  // blocks per pass before any device fitting

// Split count s for `len` reduction points over `cols` output points, and
// its chunk; the plain plan, or (q > 0) the layout for q splits.
int bfx_plan(int cols, int len, int q, int* chunk) {
  const int lenp = (len + 15) & ~15;
  const int tiles = (cols + 255) / 256;
  int s = q > 0 ? q : (kBfxTarget + tiles - 1) / tiles;
  const int smax = (lenp + 127) / 128;  // at least 128 reduction steps per split
  s = s < 1 ? 1 : (s > smax ? smax : s);
  int c = (lenp + s - 1) / s;
  c = (c + 63) & ~63;
  *chunk = c;
  return (lenp + c - 1) / c;
}
}  // namespace

// capB > 0: resident k_bfx_rowsum blocks on the device.  Pass B's split
// count is then raised (by at most half) until the launch is just under a
// whole number of rounds of resident blocks, so the last round is not a thin
// tail that leaves most SIMDs short of the waves that hide the latency (pass
// B runs few waves per SIMD, its register budget; pass A is left as
// planned).  Every choice fits the buffer bfx_splitsB_max sizes.
void bfx_splits(int M, int N, int capB, int* splitsA, int* chunkA, int* splitsB, int* chunkB) {
  *splitsA = bfx_plan(N, M, 0, chunkA);
  int c = 0;
  const int s0 = bfx_plan(M, N, 0, &c);
  *splitsB = s0;
  *chunkB = c;
  if (capB <= 0) return;
  const int tiles = (M + 255) / 256;
  for (int q = s0; q <= s0 + s0 / 2; ++q) {
    int cq = 0;
    const int Sq = bfx_plan(M, N, q, &cq);
    const double r = (double)tiles * Sq / capB;
    if (std::ceil(r) - r < 0.1) {
      *splitsB = Sq;
      *chunkB = cq;
      return;
    }
  }
}

int bfx_splitsB_max(int M, int N) {
  int c = 0, best = 0;
  const int s0 = bfx_plan(M, N, 0, &c);
  for (int q = s0; q <= s0 + s0 / 2; ++q) best = std::max(best, bfx_plan(M, N, q, &c));
  return best;
}

int bfx_resident_blocksB() {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_bfx_rowsum, 256, 0) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return cus * per;
}

void estep_bf16x_launch(const EStepArgs<float>& a, hipStream_t st) {
  const int Mpad = (a.M + 15) & ~15, Npad = (a.N + 15) & ~15;
  const int gate = a.gate;
  const int nthr = ((a.M + 63) & ~63) + 5 * Npad;
  hipLaunchKernelGGL(k_bfx_prescale, dim3((nthr + 255) / 256), dim3(256), 0, st, a.Xt, a.Y, a.xs,
                     a.ys, a.M, a.N, Mpad, Npad, a.sc, gate, a.boxX, a.boxY, a.featX, a.featY,
                     a.featV, a.w, a.D);
  if (a.ev) (void)hipEventRecord(a.ev[0], st);
  hipLaunchKernelGGL(k_bfx_colsum, dim3((a.N + 255) / 256, a.splitsA), dim3(256), 0, st, a.featX,
                     a.featY, Mpad, a.N, a.sc, a.partA, a.boxX, a.boxY, a.w, a.M, gate);
  if (a.ev) (void)hipEventRecord(a.ev[1], st);
  colmerge_fix_launch<float>(a, st);  // also refreshes the scene features with L_n
  if (a.ev) (void)hipEventRecord(a.ev[2], st);
  hipLaunchKernelGGL(k_bfx_rowsum, dim3((a.M + 255) / 256, a.splitsB), dim3(256), 0, st, a.featX,
                     a.featY, a.featV, a.xs, a.M, Npad, a.sc, a.partB, a.boxX, a.boxY, gate);
  if (a.ev) (void)hipEventRecord(a.ev[3], st);
  rowmerge_fix_launch<float>(a, st, /*relative=*/0);
  if (a.ev) (void)hipEventRecord(a.ev[4], st);
}

}  // namespace fcpd
