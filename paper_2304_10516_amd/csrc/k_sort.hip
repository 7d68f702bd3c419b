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

// Exclusive prefix over the groups of each block, per bin, in place, and the
// per-bin totals.  Workgroup (block b, chunk of 64 bins), 1024 threads: lane
// k of the chunk's 64 bins, row r of 16 that owns a contiguous run of the
// block's groups [g0, g1).  Pass 1 sums each row's run, the 16 row sums are
// prefixed in LDS, pass 2 writes the running prefix.
__global__ __launch_bounds__(1024) void k_sort_scan(const int32_t* __restrict__ group_range, int B,
                                                    uint32_t* __restrict__ counts, uint32_t* __restrict__ totals) {
  __shared__ uint32_t part[16][64];
  const int b = blockIdx.x;
  const int nbins = B * B * B;
  const int k = blockIdx.y * 64 + threadIdx.x % 64;
  const int r = threadIdx.x / 64;
  const int g0 = group_range[2 * b], g1 = group_range[2 * b + 1];
  const int per = (g1 - g0 + 15) / 16;
  const int ra = g0 + r * per, rb = min(g1, ra + per);
  uint32_t sum = 0;
  if (k < nbins)
    for (int g = ra; g < rb; ++g) sum += counts[(int64_t)g * nbins + k];
  part[r][threadIdx.x % 64] = sum;
  __syncthreads();
  uint32_t base = 0;
  for (int q = 0; q < r; ++q) base += part[q][threadIdx.x % 64];
  if (k < nbins) {
    for (int g = ra; g < rb; ++g) {
      const uint32_t c = counts[(int64_t)g * nbins + k];
      counts[(int64_t)g * nbins + k] = base;
      base += c;
    }
    if (r == 15) totals[b * kMaxBins + k] = base;  // the last row ends with the bin total
  }
}

__device__ __forceinline__ void cell_pos_s(float x, int n, int g, int N, int& i0, float& t) {
  const float p = x * (float)n - 0.5f + (float)g;
  int i = (int)floorf(p);
  i = max(0, min(i, N - 2));
  i0 = i;
  t = fminf(fmaxf(p - (float)i, 0.0f), 1.0f);
}

// Bin starts are the exclusive scan of the block's bin totals; every
// workgroup computes them in LDS, the block's first group also stores them
// (bin_start[b][0..nbins], last = sample count) for the privatized scatter.
__global__ __launch_bounds__(256) void k_sort_place(const Tile* __restrict__ groups, const int32_t* __restrict__ grange,
                                                    int B, uint64_t seed, const Counters* __restrict__ ctr,
                                                    const uint32_t* __restrict__ prefix,
                                                    const uint32_t* __restrict__ totals,
                                                    int32_t* __restrict__ bin_start,
                                                    const BlockMeta* __restrict__ meta,
                                                    const BlockRange* __restrict__ range,
                                                    const BlockPlan* __restrict__ plan, float* __restrict__ coords,
                                                    float* __restrict__ target) {
  __shared__ uint32_t cursor[kMaxBins];
  __shared__ uint32_t scan[kMaxBins];
  const int nbins = B * B * B;
  const Tile gr = groups[blockIdx.x];
  const uint32_t* pre = prefix + (int64_t)blockIdx.x * nbins;
  const uint32_t* tot = totals + gr.block * kMaxBins;
  // exclusive scan of the bin totals: each thread owns 2 consecutive bins
  const int t = threadIdx.x;
  const uint32_t a0 = 2 * t < nbins ? tot[2 * t] : 0u, a1 = 2 * t + 1 < nbins ? tot[2 * t + 1] : 0u;
  scan[t] = a0 + a1;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    const uint32_t v = t >= o ? scan[t - o] : 0u;
    __syncthreads();
    scan[t] += v;
    __syncthreads();
  }
  const uint32_t ex = scan[t] - a0 - a1;  // start of bin 2t
  const bool first = grange[2 * gr.block] == (int)blockIdx.x;
  int32_t* bs = bin_start + gr.block * (kMaxBins + 1);
  if (2 * t < nbins) {
    cursor[2 * t] = ex + pre[2 * t];
    if (first) bs[2 * t] = (int32_t)ex;
  }
  if (2 * t + 1 < nbins) {
    cursor[2 * t + 1] = ex + a0 + pre[2 * t + 1];
    if (first) bs[2 * t + 1] = (int32_t)(ex + a0);
  }
  if (first && t == 255) bs[nbins] = (int32_t)scan[255];
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
                                uint64_t seed, const Counters* ctr, uint32_t* counts, uint32_t* totals,
                                int32_t* bin_start, const BlockMeta* meta, const BlockRange* range,
                                const BlockPlan* plan, float* coords, float* target, hipStream_t s) {
  if (n_groups <= 0) return hipSuccess;
  if (B < 1 || B * B * B > kMaxBins) return hipErrorInvalidValue;
  const int nbins = B * B * B;
  hipLaunchKernelGGL(k_sort_count, dim3(n_groups), dim3(256), 0, s, groups, B, seed, ctr, counts);
  hipLaunchKernelGGL(k_sort_scan, dim3(n_blocks, (nbins + 63) / 64), dim3(1024), 0, s, group_range, B, counts,
                     totals);
  hipLaunchKernelGGL(k_sort_place, dim3(n_groups), dim3(256), 0, s, groups, group_range, B, seed, ctr, counts,
                     totals, bin_start, meta, range, plan, coords, target);
  return hipGetLastError();
}

// ===========================================================================
// Bin-privatized encoding backward for levels [l0, l1).  One workgroup per
// (block, bin, level), in gather form:
//   1. the cell box touched by the bin's samples (min/max of cell origins);
//   2. a counting sort of the samples by cell inside the box (one integer LDS
//      atomic per sample) that stores each sample's fractions t and dL/dy in
//      cell order;
//   3. one lane per (box vertex, feature) sums w_c * dy over the samples of
//      the up to 8 cells that have the vertex as a corner (no float atomics),
//      and adds the sum to the table gradient with one global atomic; lanes
//      walk vertices x fastest, so an atomic instruction covers contiguous
//      entries (dense) or a few aligned segments (hashed, x prime 1).
// A bin whose cell box exceeds the LDS budget falls back to grouped direct
// atomics.  Samples beyond kPrivRecs per bin are processed in chunks.
// ===========================================================================
constexpr int kPrivCells = 8192;  // cells of the box (int counters / starts)
constexpr int kPrivRecs = 1024;   // samples per chunk held in LDS

template <int F>
__global__ __launch_bounds__(256) void k_scatter_priv(LevelDesc ld, int l0, int nlev, int B,
                                                      const BlockMeta* __restrict__ meta,
                                                      const BlockPlan* __restrict__ plan,
                                                      const int32_t* __restrict__ bin_start,
                                                      const float* __restrict__ coords,
                                                      const float* __restrict__ dfeat, int64_t ls,
                                                      float* __restrict__ grad) {
  __shared__ int cstart[kPrivCells + 1];
  __shared__ float4 rt[kPrivRecs];       // tx, ty, tz of each placed sample
  __shared__ float rd[kPrivRecs * F];    // dL/dy of each placed sample
  __shared__ int part[256];
  __shared__ int box[6];
  constexpr int PER = kPrivRecs / 256;   // samples per thread in a chunk
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
  const int tid = threadIdx.x;
  // ---- 1. cell box of the bin's samples
  int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-1, -1, -1};
  for (int j = s0 + tid; j < s1; j += 256) {
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
  if (tid == 0)
    for (int a = 0; a < 3; ++a) {
      box[a] = 1 << 30;
      box[3 + a] = -1;
    }
  __syncthreads();
  if ((tid & 63) == 0)
    for (int a = 0; a < 3; ++a) {
      atomicMin(&box[a], lo[a]);
      atomicMax(&box[3 + a], hi[a]);
    }
  __syncthreads();
  const int bx0 = box[0], by0 = box[1], bz0 = box[2];
  const int cx_n = box[3] - bx0 + 1, cy_n = box[4] - by0 + 1, cz_n = box[5] - bz0 + 1;  // cells per axis
  const int64_t C = (int64_t)cx_n * cy_n * cz_n;
  if (C > kPrivCells) {
    // box too large for LDS: grouped direct atomics (2F lanes per x-neighbour pair)
    constexpr int G = 2 * F;
    const int q = tid % G;
    const int cx = q / F, f = q % F;
    const int items = (s1 - s0) * 4;
    for (int it = tid / G; it < items; it += 256 / G) {
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
    return;
  }
  const int vx_n = cx_n + 1, vy_n = cy_n + 1, vz_n = cz_n + 1;  // vertices per axis
  const int NV = vx_n * vy_n * vz_n;
  for (int c0 = s0; c0 < s1; c0 += kPrivRecs) {
    const int cn = min(kPrivRecs, s1 - c0);
    for (int i = tid; i <= C; i += 256) cstart[i] = 0;
    __syncthreads();
    // ---- 2a. cell of each sample and its rank within the cell
    int mcell[PER], mrank[PER];
    float mt[PER][3], md[PER][F];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int j = tid + 256 * u;
      mcell[u] = -1;
      if (j < cn) {
        const int64_t gi = base + c0 + j;
        int i0[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) grid_pos(coords[3 * gi + a], sc, R, i0[a], mt[u][a]);
#pragma unroll
        for (int f = 0; f < F; ++f) md[u][f] = dfeat[(int64_t)l * ls + gi * F + f];
        mcell[u] = (i0[0] - bx0) + cx_n * ((i0[1] - by0) + cy_n * (i0[2] - bz0));
        mrank[u] = atomicAdd(&cstart[mcell[u]], 1);
      }
    }
    __syncthreads();
    // ---- 2b. exclusive scan of the C cell counts (contiguous chunk per thread)
    {
      const int chunk = (int)((C + 255) / 256);
      const int a0 = tid * chunk, a1 = min((int)C, a0 + chunk);
      int run = 0;
      for (int i = a0; i < a1; ++i) run += cstart[i];
      part[tid] = run;
      __syncthreads();
      for (int o = 1; o < 256; o <<= 1) {
        const int v = tid >= o ? part[tid - o] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
      }
      int acc = part[tid] - run;
      for (int i = a0; i < a1; ++i) {
        const int c = cstart[i];
        cstart[i] = acc;
        acc += c;
      }
      if (tid == 255) cstart[C] = part[255];
      __syncthreads();
    }
    // ---- 2c. place the samples in cell order
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      if (mcell[u] >= 0) {
        const int p = cstart[mcell[u]] + mrank[u];
        rt[p] = make_float4(mt[u][0], mt[u][1], mt[u][2], 0.0f);
#pragma unroll
        for (int f = 0; f < F; ++f) rd[p * F + f] = md[u][f];
      }
    }
    __syncthreads();
    // ---- 3. gather per (vertex, feature), x fastest, and one atomic per touched entry
    for (int e = tid; e < NV * F; e += 256) {
      const int v = e / F, f = e % F;
      const int lx = v % vx_n, ly = (v / vx_n) % vy_n, lz = v / (vx_n * vy_n);
      float acc = 0.0f;
      bool touched = false;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int ccx = k & 1, ccy = (k >> 1) & 1, ccz = (k >> 2) & 1;  // corner of the cell
        const int x = lx - ccx, y = ly - ccy, z = lz - ccz;                 // the cell
        if (x < 0 || y < 0 || z < 0 || x >= cx_n || y >= cy_n || z >= cz_n) continue;
        const int cell = x + cx_n * (y + cy_n * z);
        const int p0 = cstart[cell], p1 = cstart[cell + 1];
        for (int p = p0; p < p1; ++p) {
          const float4 t = rt[p];
          const float w = (ccx ? t.x : 1.0f - t.x) * (ccy ? t.y : 1.0f - t.y) * (ccz ? t.z : 1.0f - t.z);
          acc += w * rd[p * F + f];
          touched = true;
        }
      }
      if (touched) {
        const uint32_t ent = corner_index(dense, R, ld.T_mask, (uint32_t)(bx0 + lx), (uint32_t)(by0 + ly),
                                          (uint32_t)(bz0 + lz));
        unsafeAtomicAdd(&g[(int64_t)ent * F + f], acc);
      }
    }
    __syncthreads();
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
