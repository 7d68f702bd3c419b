// Spatially ordered sampling and bin-privatized encoding backward (gfx950).
//
// The training samples of a step are an unordered set: drawing them with
// Philox and then storing them grouped by spatial bin (a B x B x B partition
// of the block's unit cube) leaves every per-sample quantity and every sum
// unchanged up to floating-point summation order.  Grouping lets one
// workgroup own all samples of one bin, so the gradient of a coarse level's
// vertices around that bin can be accumulated in LDS and written back with
// one atomic per touched table entry, laid out so that consecutive lanes hit
// consecutive entries (dense levels) or entries within the same aligned group
// (hashed levels: the x prime is 1, so a row of consecutive x vertices maps
// into few aligned 64-byte segments).
//
// Counting sort in three kernels, no global atomics:
//   k_sort_count : per group of samples, histogram of bins -> counts[group][bin]
//   k_sort_scan  : per block, exclusive prefix over groups per bin (in place)
//                  and over bins -> bin_start[block][bin]
//   k_sort_place : recompute each sample, place it at
//                  bin_start + prefix + rank-within-group, fetch its target.
#include "dvnr_device.h"

namespace dvnrk {

__device__ __forceinline__ int bin_of(float x, float y, float z, int B) {
  const int bx = min((int)(x * (float)B), B - 1);
  const int by = min((int)(y * (float)B), B - 1);
  const int bz = min((int)(z * (float)B), B - 1);
  return bx + B * (by + B * bz);
}

__device__ __forceinline__ void draw_coords(const Tile& gr, int i_in_block, uint32_t step, uint64_t seed, float& x,
                                            float& y, float& z) {
  const U4 u = philox4x32_10(U4{(uint32_t)i_in_block, step, (uint32_t)gr.block, kCoordTag}, (uint32_t)seed,
                             (uint32_t)(seed >> 32));
  x = u24(u.x);
  y = u24(u.y);
  z = u24(u.z);
}

// groups: Tile entries with count <= kSortGroup samples of one block.
__global__ __launch_bounds__(256) void k_sort_count(const Tile* __restrict__ groups, int B, uint64_t seed,
                                                    const Counters* __restrict__ ctr, uint32_t* __restrict__ counts) {
  __shared__ uint32_t hist[kMaxBins];
  const int nbins = B * B * B;
  for (int i = threadIdx.x; i < nbins; i += blockDim.x) hist[i] = 0u;
  __syncthreads();
  const Tile gr = groups[blockIdx.x];
  const uint32_t step = (uint32_t)ctr->step;
  for (int j = threadIdx.x; j < gr.count; j += blockDim.x) {
    float x, y, z;
    draw_coords(gr, gr.start + j, step, seed, x, y, z);
    atomicAdd(&hist[bin_of(x, y, z, B)], 1u);
  }
  __syncthreads();
  uint32_t* out = counts + (int64_t)blockIdx.x * nbins;
  for (int i = threadIdx.x; i < nbins; i += blockDim.x) out[i] = hist[i];
}

// One workgroup per block; thread k owns bin k (nbins <= blockDim).  Groups of
// block b are [g0, g1).
__global__ __launch_bounds__(512) void k_sort_scan(const int32_t* __restrict__ group_range, int B,
                                                   uint32_t* __restrict__ counts, int32_t* __restrict__ bin_start) {
  __shared__ uint32_t tot[kMaxBins];
  const int b = blockIdx.x;
  const int nbins = B * B * B;
  const int g0 = group_range[2 * b], g1 = group_range[2 * b + 1];
  const int k = threadIdx.x;
  uint32_t run = 0;
  if (k < nbins) {
    // exclusive prefix over the block's groups, loads batched 8 at a time
    int g = g0;
    for (; g + 8 <= g1; g += 8) {
      uint32_t c[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) c[u] = counts[(int64_t)(g + u) * nbins + k];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        counts[(int64_t)(g + u) * nbins + k] = run;
        run += c[u];
      }
    }
    for (; g < g1; ++g) {
      const uint32_t c = counts[(int64_t)g * nbins + k];
      counts[(int64_t)g * nbins + k] = run;
      run += c;
    }
  }
  tot[k] = k < nbins ? run : 0u;
  __syncthreads();
  // exclusive scan of bin totals (Hillis-Steele on 512 entries)
  for (int o = 1; o < (int)blockDim.x; o <<= 1) {
    const uint32_t v = (k >= o) ? tot[k - o] : 0u;
    __syncthreads();
    tot[k] += v;
    __syncthreads();
  }
  if (k < nbins) bin_start[b * (kMaxBins + 1) + k] = (int32_t)(tot[k] - run);
  if (k == nbins - 1) bin_start[b * (kMaxBins + 1) + nbins] = (int32_t)tot[k];
}

__device__ __forceinline__ void cell_pos_s(float x, int n, int g, int N, int& i0, float& t) {
  const float p = x * (float)n - 0.5f + (float)g;
  int i = (int)floorf(p);
  i = max(0, min(i, N - 2));
  i0 = i;
  t = fminf(fmaxf(p - (float)i, 0.0f), 1.0f);
}

__global__ __launch_bounds__(256) void k_sort_place(const Tile* __restrict__ groups, int B, uint64_t seed,
                                                    const Counters* __restrict__ ctr,
                                                    const uint32_t* __restrict__ prefix,
                                                    const int32_t* __restrict__ bin_start,
                                                    const BlockMeta* __restrict__ meta,
                                                    const BlockRange* __restrict__ range,
                                                    const BlockPlan* __restrict__ plan, float* __restrict__ coords,
                                                    float* __restrict__ target) {
  __shared__ uint32_t cursor[kMaxBins];
  const int nbins = B * B * B;
  const Tile gr = groups[blockIdx.x];
  const uint32_t* pre = prefix + (int64_t)blockIdx.x * nbins;
  const int32_t* bs = bin_start + gr.block * (kMaxBins + 1);
  for (int i = threadIdx.x; i < nbins; i += blockDim.x) cursor[i] = pre[i] + (uint32_t)bs[i];
  __syncthreads();
  const uint32_t step = (uint32_t)ctr->step;
  const BlockMeta bm = meta[gr.block];
  const BlockRange br = range[gr.block];
  const int64_t base = plan[gr.block].sample_off;
  const int g = bm.ghost;
  const int NX = bm.dims[0] + 2 * g, NY = bm.dims[1] + 2 * g, NZ = bm.dims[2] + 2 * g;
  for (int j = threadIdx.x; j < gr.count; j += blockDim.x) {
    float x, y, z;
    draw_coords(gr, gr.start + j, step, seed, x, y, z);
    const uint32_t dst = atomicAdd(&cursor[bin_of(x, y, z, B)], 1u);
    const int64_t gi = base + dst;
    coords[3 * gi + 0] = x;
    coords[3 * gi + 1] = y;
    coords[3 * gi + 2] = z;
    int ix, iy, iz;
    float tx, ty, tz;
    cell_pos_s(x, bm.dims[0], g, NX, ix, tx);
    cell_pos_s(y, bm.dims[1], g, NY, iy, ty);
    cell_pos_s(z, bm.dims[2], g, NZ, iz, tz);
    const float* v = bm.vol + ((int64_t)iz * NY + iy) * NX + ix;
    const int64_t sy = NX, sz = (int64_t)NX * NY;
    const float c00 = v[0] + tx * (v[1] - v[0]);
    const float c10 = v[sy] + tx * (v[sy + 1] - v[sy]);
    const float c01 = v[sz] + tx * (v[sz + 1] - v[sz]);
    const float c11 = v[sz + sy] + tx * (v[sz + sy + 1] - v[sz + sy]);
    const float c0 = c00 + ty * (c10 - c00);
    const float c1 = c01 + ty * (c11 - c01);
    target[gi] = (c0 + tz * (c1 - c0) - br.vmin) * br.inv_range;
  }
}

hipError_t launch_sorted_sample(const Tile* groups, int n_groups, const int32_t* group_range, int n_blocks, int B,
                                uint64_t seed, const Counters* ctr, uint32_t* counts, int32_t* bin_start,
                                const BlockMeta* meta, const BlockRange* range, const BlockPlan* plan, float* coords,
                                float* target, hipStream_t s) {
  if (n_groups <= 0) return hipSuccess;
  if (B < 1 || B * B * B > kMaxBins) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sort_count, dim3(n_groups), dim3(256), 0, s, groups, B, seed, ctr, counts);
  hipLaunchKernelGGL(k_sort_scan, dim3(n_blocks), dim3(kMaxBins), 0, s, group_range, B, counts, bin_start);
  hipLaunchKernelGGL(k_sort_place, dim3(n_groups), dim3(256), 0, s, groups, B, seed, ctr, counts, bin_start, meta,
                     range, plan, coords, target);
  return hipGetLastError();
}

// ===========================================================================
// Bin-privatized encoding backward for levels [l0, l1).  One workgroup per
// (block, bin, level).  The vertex box touched by the bin's samples is found
// by a min/max reduction over their cell origins; when its F floats per
// vertex fit the LDS budget, the workgroup accumulates there and flushes one
// atomic per touched (vertex, feature); otherwise it falls back to grouped
// direct atomics.
// ===========================================================================
constexpr int kPrivFloats = 16384;  // 64 KiB of fp32 accumulators

template <int F>
__global__ __launch_bounds__(256) void k_scatter_priv(LevelDesc ld, int l0, int nlev, int B,
                                                      const BlockMeta* __restrict__ meta,
                                                      const BlockPlan* __restrict__ plan,
                                                      const int32_t* __restrict__ bin_start,
                                                      const float* __restrict__ coords,
                                                      const float* __restrict__ dfeat, int64_t ls,
                                                      float* __restrict__ grad) {
  __shared__ float acc[kPrivFloats];
  __shared__ int box[6];
  const int nbins = B * B * B;
  const int wg = blockIdx.x;
  const int l = l0 + wg % nlev;
  const int bin = (wg / nlev) % nbins;
  const int b = wg / (nlev * nbins);
  const int32_t* bs = bin_start + b * (kMaxBins + 1);
  const int s0 = bs[bin], s1 = bs[bin + 1];
  if (s0 >= s1) return;
  const int64_t base = plan[b].sample_off;
  const int R = ld.R[l];
  const float sc = ld.scale[l];
  const int dense = ld.dense[l];
  float* g = grad + meta[b].param_off + (int64_t)ld.off[l] * F;
  // ---- vertex box of the bin's samples
  int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-1, -1, -1};
  for (int j = s0 + (int)threadIdx.x; j < s1; j += blockDim.x) {
    const int64_t gi = base + j;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      int i0;
      float t;
      grid_pos(coords[3 * gi + a], sc, R, i0, t);
      lo[a] = min(lo[a], i0);
      hi[a] = max(hi[a], i0);
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      lo[a] = min(lo[a], __shfl_xor(lo[a], o, 64));
      hi[a] = max(hi[a], __shfl_xor(hi[a], o, 64));
    }
  }
  if (threadIdx.x == 0)
    for (int a = 0; a < 3; ++a) {
      box[a] = 1 << 30;
      box[3 + a] = -1;
    }
  __syncthreads();
  if ((threadIdx.x & 63) == 0)
    for (int a = 0; a < 3; ++a) {
      atomicMin(&box[a], lo[a]);
      atomicMax(&box[3 + a], hi[a]);
    }
  __syncthreads();
  const int bx0 = box[0], by0 = box[1], bz0 = box[2];
  const int dx = box[3] - bx0 + 2, dy = box[4] - by0 + 2, dz = box[5] - bz0 + 2;  // vertices per axis
  const int64_t nv = (int64_t)dx * dy * dz;
  if (nv * F <= kPrivFloats) {
    for (int i = threadIdx.x; i < nv * F; i += blockDim.x) acc[i] = 0.0f;
    __syncthreads();
    for (int j = s0 + (int)threadIdx.x; j < s1; j += blockDim.x) {
      const int64_t gi = base + j;
      int ix, iy, iz;
      float tx, ty, tz;
      grid_pos(coords[3 * gi + 0], sc, R, ix, tx);
      grid_pos(coords[3 * gi + 1], sc, R, iy, ty);
      grid_pos(coords[3 * gi + 2], sc, R, iz, tz);
      float d[F];
#pragma unroll
      for (int f = 0; f < F; ++f) d[f] = dfeat[(int64_t)l * ls + gi * F + f];
      const int lx = ix - bx0, ly = iy - by0, lz = iz - bz0;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int cx = k & 1, cy = (k >> 1) & 1, cz = (k >> 2) & 1;
        const float w = (cx ? tx : 1.0f - tx) * (cy ? ty : 1.0f - ty) * (cz ? tz : 1.0f - tz);
        const int v = (lx + cx) + dx * ((ly + cy) + dy * (lz + cz));
#pragma unroll
        for (int f = 0; f < F; ++f) atomicAdd(&acc[v * F + f], w * d[f]);
      }
    }
    __syncthreads();
    // flush: element e = v * F + f, x fastest, so consecutive lanes hit consecutive entries
    for (int e = threadIdx.x; e < nv * F; e += blockDim.x) {
      const float val = acc[e];
      if (val == 0.0f) continue;
      const int v = e / F, f = e % F;
      const int vx = bx0 + v % dx, vy = by0 + (v / dx) % dy, vz = bz0 + v / (dx * dy);
      const uint32_t ent = corner_index(dense, R, ld.T_mask, (uint32_t)vx, (uint32_t)vy, (uint32_t)vz);
      unsafeAtomicAdd(&g[(int64_t)ent * F + f], val);
    }
  } else {
    // box too large for LDS: grouped direct atomics (2F lanes per x-neighbour pair)
    constexpr int G = 2 * F;
    const int q = threadIdx.x % G;
    const int cx = q / F, f = q % F;
    const int items = (s1 - s0) * 4;
    for (int it = threadIdx.x / G; it < items; it += blockDim.x / G) {
      const int64_t gi = base + s0 + (it >> 2);
      const int yz = it & 3;
      int ix, iy, iz;
      float tx, ty, tz;
      grid_pos(coords[3 * gi + 0], sc, R, ix, tx);
      grid_pos(coords[3 * gi + 1], sc, R, iy, ty);
      grid_pos(coords[3 * gi + 2], sc, R, iz, tz);
      const uint32_t cy = yz & 1, cz = yz >> 1;
      const uint32_t e = corner_index(dense, R, ld.T_mask, ix + cx, iy + cy, iz + cz);
      const float w = (cx ? tx : 1.0f - tx) * (cy ? ty : 1.0f - ty) * (cz ? tz : 1.0f - tz);
      unsafeAtomicAdd(&g[(int64_t)e * F + f], w * dfeat[(int64_t)l * ls + gi * F + f]);
    }
  }
}

hipError_t launch_scatter_priv(const LevelDesc& ld, int l0, int l1, int B, int n_blocks, const BlockMeta* meta,
                               const BlockPlan* plan, const int32_t* bin_start, const float* coords,
                               const float* dfeat, int64_t ls, float* grad, hipStream_t s) {
  const int nlev = l1 - l0;
  if (nlev <= 0) return hipSuccess;
  const int grid = n_blocks * B * B * B * nlev;
  switch (ld.F) {
    case 1: hipLaunchKernelGGL(k_scatter_priv<1>, dim3(grid), dim3(256), 0, s, ld, l0, nlev, B, meta, plan, bin_start, coords, dfeat, ls, grad); break;
    case 2: hipLaunchKernelGGL(k_scatter_priv<2>, dim3(grid), dim3(256), 0, s, ld, l0, nlev, B, meta, plan, bin_start, coords, dfeat, ls, grad); break;
    case 4: hipLaunchKernelGGL(k_scatter_priv<4>, dim3(grid), dim3(256), 0, s, ld, l0, nlev, B, meta, plan, bin_start, coords, dfeat, ls, grad); break;
    case 8: hipLaunchKernelGGL(k_scatter_priv<8>, dim3(grid), dim3(256), 0, s, ld, l0, nlev, B, meta, plan, bin_start, coords, dfeat, ls, grad); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace dvnrk
