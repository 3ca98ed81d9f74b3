// Feature vectors of the BF16X E-step (split-bf16 squared distances on the
// matrix cores; the layout is described in bf16x.hip).  Shared by the BF16X
// kernels and by the column merge, which refreshes a scene point's features
// once its L_n is known.
#pragma once
#include "common.hpp"

namespace fcpd {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr float kPadOffset = 3.0e30f;

__device__ __forceinline__ void split3(float u, __bf16& a, __bf16& b, __bf16& c) {
  a = (__bf16)u;
  const float r1 = u - (float)a;
  b = (__bf16)r1;
  const float r2 = r1 - (float)b;
  c = (__bf16)r2;
}

// Feature vector of one prescaled model point (valid = false: a padding row,
// whose norm slot carries kPadOffset).
__device__ __forceinline__ void model_feat(const P4<float>& p, bool valid,
                                           __bf16* __restrict__ dst) {
  __bf16 f[32];
  for (int k = 0; k < 32; ++k) f[k] = (__bf16)0.0f;
  if (valid) {
    const float c[3] = {p.x, p.y, p.z};
    for (int d = 0; d < 3; ++d) {
      __bf16 a, b, e;
      split3(c[d], a, b, e);
      f[6 * d + 0] = a;
      f[6 * d + 1] = a;
      f[6 * d + 2] = b;
      f[6 * d + 3] = a;
      f[6 * d + 4] = b;
      f[6 * d + 5] = e;
    }
    const float n = p.x * p.x + p.y * p.y + p.z * p.z;
    split3(n, f[18], f[19], f[20]);
  } else {
    f[18] = (__bf16)kPadOffset;
  }
  f[21] = f[22] = f[23] = (__bf16)1.0f;
  bf16x8* out = reinterpret_cast<bf16x8*>(dst);
  for (int q = 0; q < 4; ++q) {
    bf16x8 v;
    for (int t = 0; t < 8; ++t) v[t] = f[8 * q + t];
    out[q] = v;
  }
}

// Feature vector of one prescaled scene point with its offset `extra`.
__device__ __forceinline__ void scene_feat(const P4<float>& p, bool valid, float extra,
                                           __bf16* __restrict__ dst) {
  __bf16 g[32];
  for (int k = 0; k < 32; ++k) g[k] = (__bf16)0.0f;
  g[18] = g[19] = g[20] = (__bf16)1.0f;
  if (valid) {
    const float c[3] = {p.x, p.y, p.z};
    for (int d = 0; d < 3; ++d) {
      __bf16 a, b, e;
      split3(c[d], a, b, e);
      const __bf16 a2 = (__bf16)(-2.0f * (float)a), b2 = (__bf16)(-2.0f * (float)b),
                   e2 = (__bf16)(-2.0f * (float)e);
      g[6 * d + 0] = a2;
      g[6 * d + 1] = b2;
      g[6 * d + 2] = a2;
      g[6 * d + 3] = e2;
      g[6 * d + 4] = b2;
      g[6 * d + 5] = a2;
    }
    const float m = p.x * p.x + p.y * p.y + p.z * p.z + extra;
    split3(m, g[21], g[22], g[23]);
  } else {
    g[21] = (__bf16)kPadOffset;
  }
  bf16x8* out = reinterpret_cast<bf16x8*>(dst);
  for (int q = 0; q < 4; ++q) {
    bf16x8 v;
    for (int t = 0; t < 8; ++t) v[t] = g[8 * q + t];
    out[q] = v;
  }
}

// Pass B's sum operands: for the 16-point scene tile `tile`, the 16 bytes that
// lane `lane` of a wave feeds as the B operand of the product P V, where the
// lane's column f = lane % 16 and its k slice covers the tile's points
// 4 (lane / 16) .. + 3, each twice (the P operand holds their high and low
// bf16 parts).  Columns: 1; the three bf16 pieces of each prescaled
// coordinate (1-9); the three pieces of |y|^2 (10-12); zero (13-15).  Points
// past N (padding) have every column 0.
__device__ __forceinline__ void sum_operand(const P4<float>* __restrict__ Y, int N, float s,
                                            int tile, int lane, __bf16* __restrict__ dst) {
  const int f = lane & 15, n0 = 16 * tile + 4 * (lane >> 4);
  bf16x8 v;
  for (int q = 0; q < 4; ++q) {
    const int n = n0 + q;
    __bf16 o = (__bf16)0.0f;
    if (n < N && f < 13) {
      if (f == 0) {
        o = (__bf16)1.0f;
      } else {
        const P4<float> p = Y[n];
        const float x = p.x * s, y = p.y * s, z = p.z * s;  // as the prescaled scene
        const int c = (f - 1) / 3;
        const float u = c == 0 ? x : c == 1 ? y : c == 2 ? z : x * x + y * y + z * z;
        __bf16 a, b, e;
        split3(u, a, b, e);
        const int piece = (f - 1) % 3;
        o = piece == 0 ? a : piece == 1 ? b : e;
      }
    }
    v[q] = o;
    v[q + 4] = o;
  }
  *reinterpret_cast<bf16x8*>(dst + ((size_t)tile * 64 + lane) * 8) = v;
}

}  // namespace fcpd
