// Device helpers shared by the DVNR kernels: counter-based random numbers,
// grid positions, corner indices and trilinear weights.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dvnr_internal.h"

namespace dvnrk {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies with Weyl-sequence key bumps between rounds.
// ---------------------------------------------------------------------------
struct U4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
  }
  return c;
}

constexpr uint32_t kCoordTag = 0x44564E52u;  // 'DVNR': fourth counter word of coordinate draws
constexpr uint32_t kInitTag = 0x494E4954u;   // 'INIT': parameter initialization draws
constexpr uint32_t kBoundTag = 0x44564E42u;  // 'DVNB': fourth counter word of boundary-sample draws

// uniform in [0,1): top 24 bits scaled by 2^-24 (exact in float32)
__device__ __forceinline__ float u24(uint32_t u) { return (float)(u >> 8) * 5.9604644775390625e-8f; }

// Training coordinate of sample i of a block at one step.  Samples below
// n_uni are uniform in [0,1)^3 (Philox words 0..2 of counter (i, step, block,
// 'DVNR')).  The others are boundary-centered (Sec. III-C, Eq. (2)), read as
// an equal mixture over the six cube faces: counter (i, step, block, 'DVNB');
// face = floor(6 u3 / 2^32) picks axis face/2 and side face%2, the distance
// to the face is the half-normal quantile sigma sqrt(2) erfinv(v) of
// v = u24(u2) (clipped to 1), and the two tangential coordinates, in
// increasing axis order, are u24(u0) and u24(u1).
__device__ __forceinline__ void train_coord(uint32_t i, uint32_t step, uint32_t block, int n_uni,
                                            float sigma_sqrt2, uint64_t seed, float& x, float& y, float& z) {
  const bool bnd = (int)i >= n_uni;
  const U4 u = philox4x32_10(U4{i, step, block, bnd ? kBoundTag : kCoordTag}, (uint32_t)seed, (uint32_t)(seed >> 32));
  if (!bnd) {
    x = u24(u.x);
    y = u24(u.y);
    z = u24(u.z);
    return;
  }
  const uint32_t face = __umulhi(u.w, 6u);
  const uint32_t axis = face >> 1;
  const float d = fminf(sigma_sqrt2 * erfinvf(u24(u.z)), 1.0f);
  const float nc = (face & 1u) ? 1.0f - d : d;
  const float t0 = u24(u.x), t1 = u24(u.y);
  x = axis == 0 ? nc : t0;
  y = axis == 1 ? nc : (axis == 0 ? t0 : t1);
  z = axis == 2 ? nc : t1;
}

// ---------------------------------------------------------------------------
// Adam factors of update t (t = 1, 2, ...; Sec. III-F): the bias corrections
// 1/(1 - b1^t) and 1/(1 - b2^t), with 1 - b^t = -expm1(t ln b), and the
// learning rate lr0 2^(((t - start) / interval) log2(base)) once t > start
// (interval <= 0: constant).  ln b and log2(base) come from the host, so the
// factors are evaluated in the parameters' own precision (float for the fp32
// and mixed paths).  t, t - start and the interval are clamped to 2^30.
// ---------------------------------------------------------------------------
template <typename P>
__device__ __forceinline__ void adam_factors(int64_t t, P lr0, P ln_b1, P ln_b2, P log2_decay, int64_t start,
                                             int64_t interval, P& bc1, P& bc2, P& lr) {
  constexpr int64_t kCap = (int64_t)1 << 30;
  const P tp = (P)(int32_t)(t < kCap ? t : kCap);
  lr = lr0;
  if constexpr (sizeof(P) == 4) {
    bc1 = 1.0f / -expm1f(tp * ln_b1);
    bc2 = 1.0f / -expm1f(tp * ln_b2);
  } else {
    bc1 = 1.0 / -expm1(tp * ln_b1);
    bc2 = 1.0 / -expm1(tp * ln_b2);
  }
  if (interval > 0 && t > start) {
    const int64_t dt = t - start;
    const P e = (P)(int32_t)(dt < kCap ? dt : kCap) / (P)(int32_t)(interval < kCap ? interval : kCap) * log2_decay;
    if constexpr (sizeof(P) == 4)
      lr = lr0 * exp2f(e);
    else
      lr = lr0 * exp2(e);
  }
}

// ---------------------------------------------------------------------------
// Round-to-nearest fp32 operations that the compiler may not contract into an
// FMA with a neighbouring operation (each result is rounded on its own).
// ---------------------------------------------------------------------------
__device__ __forceinline__ float fmul_nc(float a, float b) {
#pragma clang fp contract(off)
  return a * b;
}
__device__ __forceinline__ float fadd_nc(float a, float b) {
#pragma clang fp contract(off)
  return a + b;
}
__device__ __forceinline__ float fsub_nc(float a, float b) {
#pragma clang fp contract(off)
  return a - b;
}

// fp16 bits (round to nearest even) of the fp32 value x itself.  The empty asm
// keeps the compiler from fusing the conversion into the FMA that produced x:
// the fused form (v_fma_mix) rounds the unrounded result straight to fp16,
// which differs from rounding the stored fp32 value where that value is a
// tie between two fp16 neighbours.
__device__ __forceinline__ uint32_t half_bits_of(float x) {
  asm volatile("" : "+v"(x));
  const __half h = __float2half_rn(x);
  return (uint32_t)(*reinterpret_cast<const uint16_t*>(&h));
}

// ---------------------------------------------------------------------------
// Grid position on a level of R vertices per axis.  x is clamped to [0,1];
// p = x*(R-1) is a single round-to-nearest float multiply (never contracted
// into an FMA), i0 = min(floor(p), R-2), t = p - i0 (exact).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void grid_pos(float x, float scale, int R, int& i0, float& t) {
  x = fminf(fmaxf(x, 0.0f), 1.0f);
  const float p = fmul_nc(x, scale);
  int i = (int)floorf(p);
  i = min(i, R - 2);
  i0 = i;
  t = fsub_nc(p, (float)i);
}

// Spatial hash of the multiresolution hash encoding: XOR of coordinate
// times prime (1, 2654435761, 805459861) modulo 2^32, masked to the table.
// A dense level has R^3 <= T <= 2^24 entries, so its index is formed with
// 24-bit products (full-rate instructions; a 32-bit multiply is quarter rate).
__device__ __forceinline__ uint32_t corner_index(int dense, int R, uint32_t mask, uint32_t vx, uint32_t vy,
                                                 uint32_t vz) {
  if (dense) return vx + __umul24((uint32_t)R, vy + __umul24((uint32_t)R, vz));
  return (vx ^ (vy * 2654435761u) ^ (vz * 805459861u)) & mask;
}

// The 8 corner indices and weights of one sample on one level (corner c =
// cx + 2cy + 4cz).
struct Corners {
  uint32_t idx[8];
  float w[8];
};

__device__ __forceinline__ void level_corners(const LevelDesc& ld, int l, float x, float y, float z, Corners& c) {
  int ix, iy, iz;
  float tx, ty, tz;
  const int R = ld.R[l];
  const float sc = ld.scale[l];
  grid_pos(x, sc, R, ix, tx);
  grid_pos(y, sc, R, iy, ty);
  grid_pos(z, sc, R, iz, tz);
  const int dense = ld.dense[l];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const uint32_t cx = k & 1, cy = (k >> 1) & 1, cz = (k >> 2) & 1;
    c.idx[k] = corner_index(dense, R, ld.T_mask, ix + cx, iy + cy, iz + cz);
    c.w[k] = (cx ? tx : 1.0f - tx) * (cy ? ty : 1.0f - ty) * (cz ? tz : 1.0f - tz);
  }
}

// Spatial bins of the ordered sampler: B bins per axis of the unit cube.
__device__ __forceinline__ int bin_1d(float x, int B) { return min((int)(x * (float)B), B - 1); }

__device__ __forceinline__ int bin_of(float x, float y, float z, int B) {
  return bin_1d(x, B) + B * (bin_1d(y, B) + B * bin_1d(z, B));
}

// Smallest and largest float32 x in [0, 1] that bin_1d puts in bin k (bin_1d
// is monotone in x; k / B rounded is within an ulp of the boundary).
__device__ __forceinline__ void bin_x_range(int k, int B, float& lo, float& hi) {
  lo = (float)k / (float)B;
  for (int it = 0; it < 4 && lo > 0.0f && bin_1d(nextafterf(lo, -1.0f), B) >= k; ++it) lo = nextafterf(lo, -1.0f);
  for (int it = 0; it < 4 && bin_1d(lo, B) < k; ++it) lo = nextafterf(lo, 2.0f);
  hi = 1.0f;
  if (k < B - 1) {
    hi = (float)(k + 1) / (float)B;
    for (int it = 0; it < 4 && bin_1d(hi, B) > k; ++it) hi = nextafterf(hi, -1.0f);
    for (int it = 0; it < 4 && hi < 1.0f && bin_1d(nextafterf(hi, 2.0f), B) <= k; ++it) hi = nextafterf(hi, 2.0f);
  }
}

// Wave-level helpers
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ uint32_t xcc_id() {
  // hardware register XCC_ID, bits [3:0]: the accelerator complex die this wave runs on
  return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 0xf;
}

// Map a linear workgroup id of a level-major launch to (tile, level).  With
// xcd_map and at least 8 levels, the workgroups dispatched to XCD x
// (round-robin dispatch puts workgroup w on XCD w % 8) work on levels l with
// l % 8 == x: each XCD's L2 holds only its own levels' tables, and every XCD
// pairs coarse (cheap) with fine (expensive) levels, which balances the XCDs.
// With fewer levels, each XCD serves one level.
// Any mapping is correct; this one only improves locality and balance.
// Returns false for idle workgroups.  Levels of the launch are [l0, l0 + L).
__host__ __device__ __forceinline__ bool level_major_item(int wg, int l0, int L, int n_tiles, int xcd_map, int& tile,
                                                 int& level) {
  if (L <= 0) return false;
  if (xcd_map && L >= 8) {
    const int lp = (L + 7) / 8;
    const int x = wg & 7, r = wg >> 3;
    const int slot = r % lp;
    tile = r / lp;
    level = x + 8 * slot;
    const bool ok = level < L && tile < n_tiles;
    level += l0;
    return ok;
  }
  if (xcd_map) {
    // fewer levels than XCDs: XCD x serves level x % L alone, sharing its tiles
    // with the other XCDs of that level (rank x / L of nx)
    const int x = wg & 7, r = wg >> 3;
    const int lvl = x % L;
    const int nx = (8 - lvl + L - 1) / L;
    tile = r * nx + x / L;
    level = l0 + lvl;
    return tile < n_tiles;
  }
  // plain: consecutive workgroups take the levels of one tile, rotated by the
  // tile index so that no XCD (workgroup w % 8) is left with a single level
  // when L is a multiple of 8
  tile = wg / L;
  level = l0 + (wg % L + tile) % L;
  return tile < n_tiles;
}

__host__ __device__ inline int level_major_grid(int L, int n_tiles, int xcd_map) {
  if (L <= 0 || n_tiles <= 0) return 0;
  if (xcd_map && L >= 8) return 8 * ((L + 7) / 8) * n_tiles;
  if (xcd_map) {
    const int nx_min = 8 / L;  // XCDs of the least-served level
    return 8 * ((n_tiles + nx_min - 1) / nx_min);
  }
  return L * n_tiles;
}

}  // namespace dvnrk
