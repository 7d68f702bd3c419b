// Destination-partitioned encoding backward (gfx950) for levels with large
// tables.
//
// On a fine level nearly every (sample, corner) contribution of a step lands
// on its own table entry, spread over the whole table by the spatial hash, so
// neither a bin's LDS box nor wave aggregation merges them: one global atomic
// per contribution is paid at the L2 atomic units' request rate.  Here the
// contributions are instead routed to their destination.  The table of such a
// level is cut into slices of up to kPartSliceMax fp32 accumulators (LDS):
//   pass 1 (k_part_bucket), one workgroup per (tile of samples, level): the 8
//     corner entries and contributions w * dL/dy of each sample become
//     records, counting-sorted by slice in LDS; one global atomic per
//     (workgroup, nonempty slice) reserves room in that slice's bucket, and
//     each slice's run of records is written contiguously;
//   pass 2 (k_part_accum), one workgroup per (block, level, slice): sums its
//     bucket's records into LDS and adds the slice to the gradient table in
//     coalesced rows, so every entry of the slice is written once per step.
// The LDS sums are 64-bit fixed point: LDS float atomics run at a small
// fraction of the rate of integer ones on this chip.  Pass 1 records the
// largest |contribution| of each tile; a bucket of n records whose block's
// largest contribution is M is summed in units of 2^-K with n M 2^K <= 2^62,
// so no sum can overflow, each contribution is rounded by at most 2^-(K+1)
// <= n M 2^-63 (far below fp32 rounding of the sums), and the sums do not
// depend on record order.
// Appends to one bucket are spread over up to kPartSub sub-buckets (by tile),
// so that the atomics reserving room in a bucket do not queue on one address.
// A sub-bucket that fills up (possible only for very uneven slice loads)
// sends its excess records to the gradient table as direct float atomics.
#include "dvnr_device.h"

namespace dvnrk {

#ifndef DVNR_PART_ACCUM_THREADS
#define DVNR_PART_ACCUM_THREADS 1024
#endif
constexpr int kPartAccumThreads = DVNR_PART_ACCUM_THREADS;  // threads of a slice-pass workgroup

// Word 3 of a raw buffer resource on gfx9-family chips (32-bit data format,
// no swizzle, stride 0): accesses are range-checked against the byte count
// of word 2.
constexpr int kBufferDword3 = 0x00020000;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// Exclusive prefix sum over the 256 lanes of a workgroup; `total` receives the sum.
__device__ __forceinline__ int wg_exclusive_scan(int v, int* wsum, int& total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  int pre = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int s = wsum[i];
    pre += i < w ? s : 0;
    tot += s;
  }
  total = tot;
  return pre + x - v;
}

// Records.  Generic F: 1 + F words, (slice << 16 | entry within the slice)
// then the F fp32 contributions.  F == 2: one 64-bit word — entry within the
// slice (bits 0..12), exponent e + 127 of the larger |contribution| (bits
// 13..20; 0 for a zero record), and the two contributions as 21-bit two's-
// complement mantissas m_i (bits 21..41, 42..62), contribution i = m_i 2^(e-20)
// with |m_i| < 2^20: each contribution keeps 2^-20 of the pair's larger
// magnitude (the slice is implied by the bucket).
template <int F> struct PartRec {
  static constexpr int RW = F == 2 ? 2 : 1 + F;  // 32-bit words per record
};

__device__ __forceinline__ uint64_t pack_rec2(uint32_t ent, float c0, float c1) {
  const float a = fmaxf(fabsf(c0), fabsf(c1));
  int e = 0;
  (void)frexpf(a, &e);  // a < 2^e
  if (!(a > 0.0f) || e < -126) return (uint64_t)ent;
  const float sc = ldexpf(1.0f, 20 - e);
  const int m0 = max(-(1 << 20) + 1, min((1 << 20) - 1, (int)rintf(c0 * sc)));
  const int m1 = max(-(1 << 20) + 1, min((1 << 20) - 1, (int)rintf(c1 * sc)));
  return (uint64_t)ent | ((uint64_t)(e + 127) << 13) | ((uint64_t)((uint32_t)m0 & 0x1FFFFFu) << 21) |
         ((uint64_t)((uint32_t)m1 & 0x1FFFFFu) << 42);
}

// Fields of a packed record: exponent field (0: zero record) and the two mantissas.
__device__ __forceinline__ void unpack_rec2(uint64_t r, int& ex, int& m0, int& m1) {
  ex = (int)((r >> 13) & 0xFFu);
  m0 = ((int)((uint32_t)(r >> 21) << 11)) >> 11;  // sign-extend 21 bits
  m1 = ((int)((uint32_t)(r >> 42) << 11)) >> 11;
}

// m 2^s as a 64-bit integer, rounding to nearest when s < 0.
__device__ __forceinline__ long long shift_fixed(int m, int s) {
  if (s >= 0) return (long long)m << min(s, 42);  // |m 2^s| <= M 2^K <= 2^62 keeps s <= 42
  if (s < -40) return 0;
  return ((long long)m + (1ll << (-s - 1))) >> (-s);
}

template <int F>
__global__ __launch_bounds__(256) void k_part_bucket(LevelDesc ld, PartDesc pd, const BlockMeta* __restrict__ meta,
                                                     const Tile* __restrict__ tiles, int n_tiles,
                                                     const BlockPlan* __restrict__ plan,
                                                     const PartBlock* __restrict__ pb,
                                                     const float* __restrict__ coords,
                                                     const float* __restrict__ dfeat, int64_t ls,
                                                     int32_t* __restrict__ cursor, uint32_t* __restrict__ recs,
                                                     float* __restrict__ tmax, uint8_t* __restrict__ ovf,
                                                     float* __restrict__ grad) {
  constexpr int RW = PartRec<F>::RW;
  constexpr bool PACK = F == 2;
  __shared__ __align__(16) uint32_t stage[8 * kTile * RW];  // records in slice order
  __shared__ uint8_t stq[PACK ? 8 * kTile : 1];  // slice of each packed record
  __shared__ int hist[kPartMaxSlices], lbase[kPartMaxSlices], gbase[kPartMaxSlices], wsum[4];
  __shared__ float wmax[4];
  const int tid = threadIdx.x;
  int tile, l;
  if (!level_major_item(blockIdx.x, pd.l0, pd.nl, n_tiles, 0, tile, l)) return;
  const Tile t = tiles[tile];
  const int b = t.block;
  const int sh = pd.sh[l];
  const int sub = tile % pd.nsub;
  const uint32_t smask = (1u << sh) - 1u;
  hist[tid] = 0;
  __syncthreads();
  const bool valid = tid < t.count;
  uint32_t e[8];
  float w[8], d[F];
  int rk[8];
  float m = 0.0f;  // largest |w * dL/dy| of the lane
  if (valid) {
    const int64_t gi = plan[b].sample_off + t.start + tid;
    const int R = ld.R[l];
    const float sc = ld.scale[l];
    int ix, iy, iz;
    float tx, ty, tz;
    grid_pos(coords[3 * gi + 0], sc, R, ix, tx);
    grid_pos(coords[3 * gi + 1], sc, R, iy, ty);
    grid_pos(coords[3 * gi + 2], sc, R, iz, tz);
    float dm = 0.0f;
#pragma unroll
    for (int f = 0; f < F; ++f) {
      d[f] = dfeat[(int64_t)l * ls + gi * F + f];
      dm = fmaxf(dm, fabsf(d[f]));
    }
    const int dense = ld.dense[l];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint32_t cx = k & 1, cy = (k >> 1) & 1, cz = k >> 2;
      e[k] = corner_index(dense, R, ld.T_mask, ix + cx, iy + cy, iz + cz);
      w[k] = (cx ? tx : 1.0f - tx) * (cy ? ty : 1.0f - ty) * (cz ? tz : 1.0f - tz);
      m = fmaxf(m, w[k] * dm);  // bounds |w * d[f]| for every f (rounding is monotone)
      rk[k] = atomicAdd(&hist[e[k] >> sh], 1);
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  if ((tid & 63) == 0) wmax[tid >> 6] = m;
  __syncthreads();
  if (tid == 0)
    tmax[(int64_t)(l - pd.l0) * n_tiles + tile] = fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]));
  // slice runs in LDS, and room for them in the slices' sub-buckets
  const int c = hist[tid];
  int total;
  lbase[tid] = wg_exclusive_scan(c, wsum, total);
  if (c > 0)
    gbase[tid] = atomicAdd(&cursor[((int64_t)b * pd.nq + pd.qbase[l] + tid) * kPartSub + sub], c);
  __syncthreads();
  if (valid) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint32_t q = e[k] >> sh;
      const int i = lbase[q] + rk[k];
      if constexpr (PACK) {
        reinterpret_cast<uint64_t*>(stage)[i] = pack_rec2(e[k] & smask, w[k] * d[0], w[k] * d[1]);
        stq[i] = (uint8_t)q;
      } else {
        stage[i * RW] = (q << 16) | (e[k] & smask);
#pragma unroll
        for (int f = 0; f < F; ++f) stage[i * RW + 1 + f] = __float_as_uint(w[k] * d[f]);
      }
    }
  }
  __syncthreads();
  const int64_t off = pb[b].off[l];
  const int cap = pb[b].cap[l];
  for (int i = tid; i < total; i += 256) {
    const uint32_t w0 = stage[i * RW];
    const int q = PACK ? (int)stq[i] : (int)(w0 >> 16);
    const int j = gbase[q] + i - lbase[q];
    const int64_t rec = off + ((int64_t)q * pd.nsub + sub) * cap + j;
    if (j < cap) {
      if constexpr (PACK) {
        reinterpret_cast<uint64_t*>(recs)[rec] = reinterpret_cast<const uint64_t*>(stage)[i];
      } else {
#pragma unroll
        for (int k = 0; k < RW; ++k) recs[rec * RW + k] = stage[i * RW + k];
      }
    } else {
      ovf[(int64_t)b * pd.nq + pd.qbase[l] + q] = 1;
      float* g = grad + meta[b].param_off + ((int64_t)ld.off[l] + ((int64_t)q << sh) + (w0 & smask)) * F;
      if constexpr (PACK) {
        int ex, m0, m1;
        unpack_rec2(reinterpret_cast<const uint64_t*>(stage)[i], ex, m0, m1);
        if (ex) {
          unsafeAtomicAdd(&g[0], ldexpf((float)m0, ex - 147));
          unsafeAtomicAdd(&g[1], ldexpf((float)m1, ex - 147));
        }
      } else {
#pragma unroll
        for (int f = 0; f < F; ++f) unsafeAtomicAdd(&g[f], __uint_as_float(stage[i * RW + 1 + f]));
      }
    }
  }
}

// 1024 threads with at most 64 VGPRs: two workgroups of an 8192-accumulator
// slice (64 KB of LDS each) share a CU with 32 waves, enough loads in flight
// to stream the Adam operands (512 threads at 98 VGPRs: 16 waves, the pass
// 15 % slower on the 64-block workload).  Waves per SIMD to plan registers
// for: two workgroups where the LDS allows two, one otherwise (and for F = 8,
// whose records would not fit 64 registers without spilling).
constexpr int part_accum_waves(int F, int SF, int NT) {
  // workgroups per CU: the LDS (160 KB) holds 160 KB / (8 SF), the CU 32 waves
  const int by_lds = kLdsBytes / (8 * SF), by_waves = 2048 / NT;
  const int wgs = F > 4 ? 1 : (by_lds < by_waves ? by_lds : by_waves);
  return (wgs < 1 ? 1 : wgs) * NT / 256;
}

template <int F, int SF, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(part_accum_waves(F, SF, NT)))) void k_part_accum(LevelDesc ld, PartDesc pd, const BlockMeta* __restrict__ meta,
                                                    int n_tiles, const BlockPlan* __restrict__ plan,
                                                    const PartBlock* __restrict__ pb, int32_t* __restrict__ cursor,
                                                    const uint32_t* __restrict__ recs,
                                                    const float* __restrict__ tmax, float* __restrict__ grad,
                                                    PartAdam adam, int do_adam, uint8_t* __restrict__ ovf) {
  constexpr int RW = PartRec<F>::RW;
  constexpr bool PACK = F == 2;
  constexpr int U = NT >= 1024 ? 4 : 8;  // records per lane and batch (two batches in flight)
  __shared__ unsigned long long acc[SF];
  __shared__ int sstart[kPartSub + 1];
  __shared__ float wmax[NT / 64];
  const int tid = threadIdx.x;
  const int b = blockIdx.x / pd.nq, q = blockIdx.x % pd.nq;
  if (plan[b].n == 0) return;  // no sample, no record: the bucket's cursors are still zero
  int l = pd.l0;
  while (l + 1 < pd.l0 + pd.nl && q >= pd.qbase[l + 1]) ++l;
  const int s = q - pd.qbase[l];
  const int sh = pd.sh[l];
  const uint32_t smask = (1u << sh) - 1u;
  const int cap = pb[b].cap[l];
  // sub-bucket record counts (cursors cleared for the next step's pass 1)
  if (tid < kPartSub) {
    int cnt = 0;
    if (tid < pd.nsub) {
      int32_t* cur = cursor + ((int64_t)b * pd.nq + q) * kPartSub + tid;
      cnt = min(*cur, cap);
      *cur = 0;
    }
    sstart[tid + 1] = cnt;
  }
  // largest contribution over the block's tiles on this level
  {
    const float* tm = tmax + (int64_t)(l - pd.l0) * n_tiles + pb[b].tile0;
    float m = 0.0f;
    for (int i = tid; i < pb[b].ntiles; i += NT) m = fmaxf(m, tm[i]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if ((tid & 63) == 0) wmax[tid >> 6] = m;
  }
  for (int i = tid; i < (F << sh); i += NT) acc[i] = 0ull;
  __syncthreads();
  if (tid == 0) {
    sstart[0] = 0;
    for (int g = 0; g < kPartSub; ++g) sstart[g + 1] += sstart[g];
  }
  __syncthreads();
  const int n = sstart[kPartSub];
  float M = 0.0f;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) M = fmaxf(M, wmax[i]);
  // fixed-point unit 2^-K: n M 2^K <= 2^62 with n M < 2^E
  int E = 0;
  (void)frexpf((float)n * M, &E);
  const int K = max(-120, min(120, 62 - E));
  const float scale = ldexpf(1.0f, K);
  const int kshift = K - 147;  // packed record: contribution i in units 2^-K is m_i 2^(ex - 147 + K)
  const uint32_t* r = recs + (pb[b].off[l] + (int64_t)s * pd.nsub * cap) * RW;
  // a batch of U records per lane from j0 on: unconditional loads (lanes past
  // the end re-read the last record and skip it when summing), so that all of
  // them are in flight together; record j of the bucket is record
  // j - sstart[g] of sub-bucket g
  auto load_batch = [&](int j0, uint32_t(&v)[U][RW]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = max(0, min(j0 + u * NT + tid, n - 1));
      int g = 0;
#pragma unroll
      for (int k = 1; k < kPartSub; ++k) g += j >= sstart[k] ? 1 : 0;
      const uint32_t* rr = r + ((int64_t)g * cap + (j - sstart[g])) * RW;
      // records are read once: non-temporal loads keep them from displacing
      // the volume and table lines the next kernels read from the caches
      if constexpr (PACK) {
        const uint64_t t64 = __builtin_nontemporal_load(reinterpret_cast<const uint64_t*>(rr));
        v[u][0] = (uint32_t)t64;
        v[u][1] = (uint32_t)(t64 >> 32);
      } else {
#pragma unroll
        for (int k = 0; k < RW; ++k) v[u][k] = __builtin_nontemporal_load(rr + k);
      }
    }
  };
  // the slice's elements and its Adam operands (loaded after the record sums:
  // issuing the first batch before them measured slower)
  const int64_t e0 = (int64_t)s << sh;
  const int nf = (int)min((int64_t)1 << sh, (int64_t)pd.E[l] - e0) * F;
  const int64_t el0 = meta[b].param_off + ((int64_t)ld.off[l] + e0) * F;  // first element of the slice
  constexpr int VW = F % 2 == 0 ? 2 : 1;  // elements per access (the slice starts at an even element)
  constexpr int PT = SF / NT / VW, KB = PT < 4 ? PT : 4;
  typedef float fv __attribute__((ext_vector_type(VW)));
  const int nv = nf / VW;  // accesses covering the slice (nf is a multiple of F)
  auto ldv = [&](const float* base, uint32_t a) {
    fv x;
    __builtin_memcpy(&x, base + a * VW, sizeof(fv));
    return x;
  };
  // The Adam operands are accessed through buffer resources that span the
  // slice's body exactly: the hardware range check turns loads past its end
  // into zeros and drops stores there, so the accesses need neither clamping
  // nor branches, and all of them share one 32-bit offset register.  With
  // even F the body is read and written in 16-byte accesses from the first
  // 16-byte aligned element; an F = 2 slice can start 8 bytes past such an
  // element, and then its first and last entry (the head and the tail pair)
  // are updated apart by one lane each.
  constexpr int AW = F % 2 == 0 ? 4 : 1;                    // elements per Adam access
  constexpr int APT = SF / NT / AW, AKB = APT < 4 ? APT : 4;  // body accesses per lane, per batch
  static_assert(APT >= 1 && APT * NT * AW == SF, "a slice's body is APT accesses per lane");
  typedef float av __attribute__((ext_vector_type(AW)));
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  const int head = (AW == 4 && (el0 & 3)) ? 2 : 0;  // el0 is even for even F
  const int nb = (nf - head) / AW;                  // body accesses
  const int tail = nf - head - nb * AW;             // 0, or 2 (F = 2)
  const int64_t eb = el0 + head;                    // first body element
  const uint32_t bbytes = (uint32_t)nb * AW * 4;
  auto rsrc = [&](const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kBufferDword3);
  };
  auto bld = [&](__amdgpu_buffer_rsrc_t r, uint32_t a) -> av {
    if constexpr (AW == 4) {
      const u32x4 x = __builtin_amdgcn_raw_buffer_load_b128(r, a * 16u, 0, 0);
      return av{__uint_as_float(x[0]), __uint_as_float(x[1]), __uint_as_float(x[2]), __uint_as_float(x[3])};
    } else {
      return av(__uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, a * 4u, 0, 0)));
    }
  };
  auto bst = [&](__amdgpu_buffer_rsrc_t r, uint32_t a, av x) {
    if constexpr (AW == 4)
      __builtin_amdgcn_raw_buffer_store_b128(
          u32x4{__float_as_uint(x[0]), __float_as_uint(x[1]), __float_as_uint(x[2]), __float_as_uint(x[3])}, r,
          a * 16u, 0, 0);
    else
      __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x[0]), r, a * 4u, 0, 0);
  };
  av th[AKB], mm[AKB], vv[AKB];  // Adam operands of the batch in flight
  auto load_adam = [&](int k0) {
    const auto rp = rsrc(adam.params + eb, bbytes), rm = rsrc(adam.m + eb, bbytes), rv = rsrc(adam.v + eb, bbytes);
#pragma unroll
    for (int k = 0; k < AKB; ++k) {
      const uint32_t a = (uint32_t)(tid + NT * (k0 + k));
      th[k] = bld(rp, a);
      mm[k] = bld(rm, a);
      vv[k] = bld(rv, a);
    }
  };
  uint32_t vn[U][RW];
  if (n > 0) load_batch(0, vn);
  // while the first batch is in flight: this bucket's overflow flag and the
  // Adam factors of this update (published by the barrier after the sums)
  __shared__ int has_ovf;
  __shared__ float hbc[3];
  if (tid == 0) {
    uint8_t* fl = ovf + (int64_t)b * pd.nq + q;
    has_ovf = *fl;
    *fl = 0;
    if (do_adam) {
      // this update's index t = step + 1 (the slot reduction advances the counter later)
      adam_factors<float>(adam.ctr->step + 1, adam.lr0, adam.ln_b1, adam.ln_b2, adam.log2_decay, adam.decay_start,
                          adam.decay_interval, hbc[0], hbc[1], hbc[2]);
    }
  }
  // software pipeline: the next batch's loads are issued before this batch's
  // LDS sums
  for (int j0 = 0; j0 < n; j0 += NT * U) {
    uint32_t v[U][RW];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < RW; ++k) v[u][k] = vn[u][k];
    if (j0 + NT * U < n) load_batch(j0 + NT * U, vn);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (j0 + u * NT + tid < n) {
        const uint32_t ent = v[u][0] & smask;
        if constexpr (PACK) {
          const uint64_t r64 = (uint64_t)v[u][0] | ((uint64_t)v[u][1] << 32);
          int ex, m0, m1;
          unpack_rec2(r64, ex, m0, m1);
          if (ex) {
            atomicAdd(&acc[ent * 2], (unsigned long long)shift_fixed(m0, ex + kshift));
            atomicAdd(&acc[ent * 2 + 1], (unsigned long long)shift_fixed(m1, ex + kshift));
          }
        } else {
#pragma unroll
          for (int f = 0; f < F; ++f)
            atomicAdd(&acc[ent * F + f], (unsigned long long)__float2ll_rn(__uint_as_float(v[u][1 + f]) * scale));
        }
      }
    }
  }
  __syncthreads();
  // fixed-point sums back to float: a correctly rounded int64 -> float
  // conversion and an exact scaling by 2^-K
  float* g = grad + el0;
  // overflow records of this bucket went to the gradient by atomics
  if (!do_adam) {
    // read-add-write of the slice's nonzero sums, KB accesses per lane at a time
    for (int k0 = 0; k0 < PT; k0 += KB) {
      fv gv[KB];
#pragma unroll
      for (int k = 0; k < KB; ++k) gv[k] = ldv(g, min(tid + NT * (k0 + k), nv - 1));
#pragma unroll
      for (int k = 0; k < KB; ++k) {
        const int a = tid + NT * (k0 + k);
        if (a < nv) {
#pragma unroll
          for (int c = 0; c < VW; ++c) {
            const long long s64 = (long long)acc[a * VW + c];
            if (s64 != 0) g[a * VW + c] = gv[k][c] + ldexpf((float)s64, -K);
          }
        }
      }
    }
    return;
  }
  // The Adam update of the slice in batches of KB accesses per lane; the next
  // batch's operands are loaded before this batch is updated.  No store is
  // conditional (a branch around the stores made the compiler wait for the
  // next batch's loads before each update).  OVF: the bucket overflowed and
  // its excess records went to the gradient by atomics; W16: the 16-bit
  // working copy is written too.
  load_adam(0);
  const float bc2 = hbc[1], lrbc1 = hbc[2] * hbc[0];
  // Adam of one element from its fixed-point sum, its gradient-table value g0
  // (nonzero only after an overflow) and its operands
  auto adam1 = [&](int e, float g0, float th0, float m0, float v0) -> float3 {
    const float gg = g0 + ldexpf((float)(long long)acc[e], -K) + adam.wd * th0;
    const float m1 = adam.b1 * m0 + adam.omb1 * gg;
    const float v1 = adam.b2 * v0 + adam.omb2 * gg * gg;
    // hardware square root and reciprocal (about 1 ulp each): the step
    // lr m_hat / (sqrt(v_hat) + eps) is within a few float roundings
    const float t1 = th0 - lrbc1 * m1 * __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(v1 * bc2) + adam.eps);
    return make_float3(t1, m1, v1);
  };
  auto half_bits = [](float x) -> uint32_t { return half_bits_of(x); };
  auto update = [&](auto ovf_tag, auto w16_tag) {
    constexpr bool OVF = decltype(ovf_tag)::value, W16 = decltype(w16_tag)::value;
    const auto rp = rsrc(adam.params + eb, bbytes), rm = rsrc(adam.m + eb, bbytes), rv = rsrc(adam.v + eb, bbytes);
    const auto rg = rsrc(g + head, bbytes), rw = rsrc(adam.work16 + eb, bbytes / 2);
    for (int k0 = 0; k0 < APT; k0 += AKB) {
      av gv[AKB];
#pragma unroll
      for (int k = 0; k < AKB; ++k) {
        if constexpr (OVF)
          gv[k] = bld(rg, (uint32_t)(tid + NT * (k0 + k)));
        else
          gv[k] = av(0.0f);
      }
      av th0[AKB], mm0[AKB], vv0[AKB];
#pragma unroll
      for (int k = 0; k < AKB; ++k) {
        th0[k] = th[k];
        mm0[k] = mm[k];
        vv0[k] = vv[k];
      }
      if (k0 + AKB < APT) load_adam(k0 + AKB);
#pragma unroll
      for (int k = 0; k < AKB; ++k) {
        const uint32_t a = (uint32_t)(tid + NT * (k0 + k));
        // lanes past the body's end compute on zero operands (their stores are
        // dropped) and read the accumulators at an index clamped into the slice
        const int e0a = head + (int)min(a, (uint32_t)max(nb - 1, 0)) * AW;
        av t1, m1, v1;
#pragma unroll
        for (int c = 0; c < AW; ++c) {
          const float3 r = adam1(e0a + c, gv[k][c], th0[k][c], mm0[k][c], vv0[k][c]);
          t1[c] = r.x;
          m1[c] = r.y;
          v1[c] = r.z;
        }
        bst(rp, a, t1);
        bst(rm, a, m1);
        bst(rv, a, v1);
        if constexpr (W16) {
          if constexpr (AW == 4)
            __builtin_amdgcn_raw_buffer_store_b64(
                u32x2{half_bits(t1[0]) | half_bits(t1[1]) << 16, half_bits(t1[2]) | half_bits(t1[3]) << 16}, rw,
                a * 8u, 0, 0);
          else
            __builtin_amdgcn_raw_buffer_store_b16((unsigned short)half_bits(t1[0]), rw, a * 2u, 0, 0);
        }
        if constexpr (OVF) bst(rg, a, av(0.0f));
      }
    }
    // the head pair of an F = 2 slice that starts 8 bytes past a 16-byte
    // boundary (lane 0) and the tail pair of one whose body leaves two
    // elements (lane 1), in 8-byte accesses
    if (AW == 4 && tid < 2) {
      const int e = tid == 0 ? 0 : nf - 2;
      if (tid == 0 ? head != 0 : tail != 0) {
        float2 tp, mp, vp, gp = make_float2(0.0f, 0.0f);
        __builtin_memcpy(&tp, adam.params + el0 + e, 8);
        __builtin_memcpy(&mp, adam.m + el0 + e, 8);
        __builtin_memcpy(&vp, adam.v + el0 + e, 8);
        if constexpr (OVF) __builtin_memcpy(&gp, g + e, 8);
        const float3 r0 = adam1(e, gp.x, tp.x, mp.x, vp.x), r1 = adam1(e + 1, gp.y, tp.y, mp.y, vp.y);
        const float2 t1 = make_float2(r0.x, r1.x), m1 = make_float2(r0.y, r1.y), v1 = make_float2(r0.z, r1.z);
        __builtin_memcpy(adam.params + el0 + e, &t1, 8);
        __builtin_memcpy(adam.m + el0 + e, &m1, 8);
        __builtin_memcpy(adam.v + el0 + e, &v1, 8);
        if constexpr (W16) {
          const uint32_t hh = half_bits(t1.x) | half_bits(t1.y) << 16;
          __builtin_memcpy(adam.work16 + el0 + e, &hh, 4);
        }
        if constexpr (OVF) {
          const float2 z = make_float2(0.0f, 0.0f);
          __builtin_memcpy(g + e, &z, 8);
        }
      }
    }
  };
  if (has_ovf) {
    if (adam.work16)
      update(std::true_type{}, std::true_type{});
    else
      update(std::true_type{}, std::false_type{});
  } else {
    if (adam.work16)
      update(std::false_type{}, std::true_type{});
    else
      update(std::false_type{}, std::false_type{});
  }
}

hipError_t launch_part_bucket(const LevelDesc& ld, const PartDesc& pd, const BlockMeta* meta, const Tile* tiles,
                              int n_tiles, const BlockPlan* plan, const PartBlock* pb, const float* coords,
                              const float* dfeat, int64_t ls, int32_t* cursor, uint32_t* recs, float* tmax,
                              uint8_t* ovf, float* grad, hipStream_t s) {
  if (pd.nl <= 0 || n_tiles <= 0) return hipSuccess;
  const int64_t grid = (int64_t)n_tiles * pd.nl;
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  // bucket ids fit the LDS histogram and the record's upper 16 bits
  if (pd.nsub < 1 || pd.nsub > kPartSub) return hipErrorInvalidValue;
  for (int l = pd.l0; l < pd.l0 + pd.nl; ++l)
    if (pd.ns[l] > kPartMaxSlices || pd.sh[l] > 16 || ((int64_t)pd.ns[l] << pd.sh[l]) < pd.E[l])
      return hipErrorInvalidValue;
  switch (ld.F) {
#define DVNR_PART_B(FF)                                                                                          \
  case FF:                                                                                                       \
    hipLaunchKernelGGL(k_part_bucket<FF>, dim3((unsigned)grid), dim3(256), 0, s, ld, pd, meta, tiles, n_tiles,   \
                       plan, pb, coords, dfeat, ls, cursor, recs, tmax, ovf, grad);                                         \
    break;
    DVNR_PART_B(1)
    DVNR_PART_B(2)
    DVNR_PART_B(4)
    DVNR_PART_B(8)
#undef DVNR_PART_B
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_part_accum(const LevelDesc& ld, const PartDesc& pd, const BlockMeta* meta, int n_blocks,
                             int n_tiles, const BlockPlan* plan, const PartBlock* pb, int32_t* cursor,
                             const uint32_t* recs, const float* tmax, float* grad, const PartAdam* adam,
                             uint8_t* ovf, hipStream_t s) {
  const PartAdam ad = adam ? *adam : PartAdam{};
  const int do_adam = adam ? 1 : 0;
  if (pd.nl <= 0 || n_blocks <= 0 || pd.nq <= 0) return hipSuccess;
  const int64_t grid = (int64_t)n_blocks * pd.nq;
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  // every level's slice (2^sh entries x F) fits the launch's accumulators
  if (pd.nsub < 1 || pd.nsub > kPartSub) return hipErrorInvalidValue;
  for (int l = pd.l0; l < pd.l0 + pd.nl; ++l)
    if (((int64_t)ld.F << pd.sh[l]) > pd.slice_floats || pd.ns[l] > kPartMaxSlices) return hipErrorInvalidValue;
#define DVNR_PART_A(FF, SS)                                                                                      \
  hipLaunchKernelGGL((k_part_accum<FF, SS, kPartAccumThreads>), dim3((unsigned)grid), dim3(kPartAccumThreads), 0, s, \
                     ld, pd, meta, n_tiles, plan, pb, cursor, recs, tmax, grad, ad, do_adam, ovf)
#define DVNR_PART_SF(FF)                                                                                         \
  case FF:                                                                                                       \
    if (pd.slice_floats == 4096) DVNR_PART_A(FF, 4096);                                                          \
    else if (pd.slice_floats == 8192) DVNR_PART_A(FF, 8192);                                                     \
    else if (pd.slice_floats == 16384) DVNR_PART_A(FF, 16384);                                                   \
    else return hipErrorInvalidValue;                                                                            \
    break;
  switch (ld.F) {
    DVNR_PART_SF(1)
    DVNR_PART_SF(2)
    DVNR_PART_SF(4)
    DVNR_PART_SF(8)
    default: return hipErrorInvalidValue;
  }
#undef DVNR_PART_SF
#undef DVNR_PART_A
  return hipGetLastError();
}

}  // namespace dvnrk
