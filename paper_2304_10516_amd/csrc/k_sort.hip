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


// groups: Tile entries with count <= kSortGroup samples of one block; one
// workgroup of kSortGroup threads per group (one sample per thread).
__global__ __launch_bounds__(kSortGroup) void k_sort_count(const Tile* __restrict__ groups, int B, uint64_t seed,
                                                    SampleDist dist, const BlockPlan* __restrict__ plan,
                                                    const Counters* __restrict__ ctr, uint32_t step_off,
                                                    uint32_t* __restrict__ counts) {
  __shared__ uint32_t hist[kMaxBins];
  const int nbins = B * B * B;
  for (int i = threadIdx.x; i < nbins; i += blockDim.x) hist[i] = 0u;
  __syncthreads();
  const Tile gr = groups[blockIdx.x];
  const uint32_t step = (uint32_t)ctr->step + step_off;
  const int n_uni = plan[gr.block].n_uni;
  for (int j = threadIdx.x; j < gr.count; j += blockDim.x) {
    float x, y, z;
    train_coord((uint32_t)(gr.start + j), step, (uint32_t)gr.block, n_uni, dist.sigma_sqrt2, seed, x, y, z);
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
  // a row of up to PR groups keeps its counts in registers, loaded together
  // (clamped indices, masked values) instead of one dependent load at a time
  constexpr int PR = 16;
  const bool regs = per <= PR && g1 > g0;  // uniform over the workgroup
  uint32_t cv[PR];
  uint32_t sum = 0;
  if (regs) {
    const int kk = min(k, nbins - 1);
#pragma unroll
    for (int i = 0; i < PR; ++i) {
      const int gg = min(ra + i, g1 - 1);
      const uint32_t v = counts[(int64_t)gg * nbins + kk];
      cv[i] = (k < nbins && ra + i < rb) ? v : 0u;
      sum += cv[i];
    }
  } else if (k < nbins) {
    for (int g = ra; g < rb; ++g) sum += counts[(int64_t)g * nbins + k];
  }
  part[r][threadIdx.x % 64] = sum;
  __syncthreads();
  uint32_t base = 0;
  for (int q = 0; q < r; ++q) base += part[q][threadIdx.x % 64];
  if (k < nbins) {
    if (regs) {
#pragma unroll
      for (int i = 0; i < PR; ++i)
        if (ra + i < rb) {
          counts[(int64_t)(ra + i) * nbins + k] = base;
          base += cv[i];
        }
    } else {
      for (int g = ra; g < rb; ++g) {
        const uint32_t c = counts[(int64_t)g * nbins + k];
        counts[(int64_t)g * nbins + k] = base;
        base += c;
      }
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
__global__ __launch_bounds__(kSortGroup) void k_sort_place(const Tile* __restrict__ groups, const int32_t* __restrict__ grange,
                                                    int B, uint64_t seed, SampleDist dist,
                                                    const Counters* __restrict__ ctr, uint32_t step_off,
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
  // exclusive scan of the bin totals: threads 0..255 own 2 consecutive bins each
  const int t = threadIdx.x;
  const bool scanner = t < 256;
  uint32_t a0 = 0u, a1 = 0u;
  if (scanner) {
    a0 = 2 * t < nbins ? tot[2 * t] : 0u;
    a1 = 2 * t + 1 < nbins ? tot[2 * t + 1] : 0u;
    scan[t] = a0 + a1;
  }
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    const uint32_t v = scanner && t >= o ? scan[t - o] : 0u;
    __syncthreads();
    if (scanner) scan[t] += v;
    __syncthreads();
  }
  const bool first = grange[2 * gr.block] == (int)blockIdx.x;
  int32_t* bs = bin_start + gr.block * (kMaxBins + 1);
  if (scanner) {
    const uint32_t ex = scan[t] - a0 - a1;  // start of bin 2t
    if (2 * t < nbins) {
      cursor[2 * t] = ex + pre[2 * t];
      if (first) bs[2 * t] = (int32_t)ex;
    }
    if (2 * t + 1 < nbins) {
      cursor[2 * t + 1] = ex + a0 + pre[2 * t + 1];
      if (first) bs[2 * t + 1] = (int32_t)(ex + a0);
    }
    if (first && t == 255) bs[nbins] = (int32_t)scan[255];
  }
  __syncthreads();
  const uint32_t step = (uint32_t)ctr->step + step_off;
  const BlockMeta bm = meta[gr.block];
  const BlockRange br = range[gr.block];
  const int64_t base = plan[gr.block].sample_off;
  const int n_uni = plan[gr.block].n_uni;
  const int g = bm.ghost;
  const int NX = bm.dims[0] + 2 * g, NY = bm.dims[1] + 2 * g, NZ = bm.dims[2] + 2 * g;
  // the volume is global memory: the address-space cast lets the compiler use
  // global (not flat) loads, which do not wait on the LDS counter
  typedef const __attribute__((address_space(1))) float gfloat;
  for (int j = threadIdx.x; j < gr.count; j += blockDim.x) {
    float x, y, z;
    train_coord((uint32_t)(gr.start + j), step, (uint32_t)gr.block, n_uni, dist.sigma_sqrt2, seed, x, y, z);
    // voxel loads first, so that they are in flight during the LDS atomic below
    int ix, iy, iz;
    float tx, ty, tz;
    cell_pos_s(x, bm.dims[0], g, NX, ix, tx);
    cell_pos_s(y, bm.dims[1], g, NY, iy, ty);
    cell_pos_s(z, bm.dims[2], g, NZ, iz, tz);
    gfloat* v = (gfloat*)(bm.vol + ((int64_t)iz * NY + iy) * NX + ix);
    const int64_t sy = NX, sz = (int64_t)NX * NY;
    const float v000 = v[0], v100 = v[1], v010 = v[sy], v110 = v[sy + 1];
    const float v001 = v[sz], v101 = v[sz + 1], v011 = v[sz + sy], v111 = v[sz + sy + 1];
    const uint32_t dst = atomicAdd(&cursor[bin_of(x, y, z, B)], 1u);
    const int64_t gi = base + dst;
    coords[3 * gi + 0] = x;
    coords[3 * gi + 1] = y;
    coords[3 * gi + 2] = z;
    const float c00 = v000 + tx * (v100 - v000);
    const float c10 = v010 + tx * (v110 - v010);
    const float c01 = v001 + tx * (v101 - v001);
    const float c11 = v011 + tx * (v111 - v011);
    const float c0 = c00 + ty * (c10 - c00);
    const float c1 = c01 + ty * (c11 - c01);
    target[gi] = (c0 + tz * (c1 - c0) - br.vmin) * br.inv_range;
  }
}

hipError_t launch_sorted_sample(const Tile* groups, int n_groups, const int32_t* group_range, int n_blocks, int B,
                                uint64_t seed, SampleDist dist, const Counters* ctr, uint32_t step_off,
                                uint32_t* counts, uint32_t* totals,
                                int32_t* bin_start, const BlockMeta* meta, const BlockRange* range,
                                const BlockPlan* plan, float* coords, float* target, hipStream_t s) {
  if (n_groups <= 0) return hipSuccess;
  if (B < 1 || B * B * B > kMaxBins) return hipErrorInvalidValue;
  const int nbins = B * B * B;
  hipLaunchKernelGGL(k_sort_count, dim3(n_groups), dim3(kSortGroup), 0, s, groups, B, seed, dist, plan, ctr, step_off,
                     counts);
  hipLaunchKernelGGL(k_sort_scan, dim3(n_blocks, (nbins + 63) / 64), dim3(1024), 0, s, group_range, B, counts,
                     totals);
  hipLaunchKernelGGL(k_sort_place, dim3(n_groups), dim3(kSortGroup), 0, s, groups, group_range, B, seed, dist, ctr,
                     step_off, counts,
                     totals, bin_start, meta, range, plan, coords, target);
  return hipGetLastError();
}

// ===========================================================================
// Bin-privatized encoding backward for levels [l0, l1).  One workgroup per
// (block, bin, level):
//   1. the cell box touched by the bin's samples (min/max of cell origins);
//   2. a counting sort of the samples by cell inside the box (one integer LDS
//      atomic per sample) that stores each sample's fractions t and dL/dy in
//      cell order (chunks of RECS samples);
//   3. cell pass: the lanes of a cell (1, 2, 4 or 8, more when the box has few
//      cells) sum w_c * dy over the cell's samples for its 8 corners and F
//      features in registers, combine their sums with shuffles, and the cell's
//      first lane adds them to an LDS accumulator of the box vertices (8 F LDS
//      atomics per occupied cell instead of per sample);
//   4. vertex pass: one global atomic per nonzero (box vertex, feature) sum;
//      lanes walk vertices x fastest, so an atomic instruction covers
//      contiguous entries (dense levels) or a few aligned segments (hashed
//      levels, whose x prime is 1).
// A bin whose box exceeds the LDS budget falls back to grouped direct atomics.
// ===========================================================================
// LDS budget classes: CELLS box cells, VFLOATS box vertices x F accumulators,
// RECS samples per chunk.  CELLS == 0 is the direct class (no LDS: levels
// whose boxes never fit take the direct path at full occupancy).
template <int F, int CELLS, int VFLOATS, int RECS>
__global__ __launch_bounds__(256) void k_scatter_priv(LevelDesc ld, int l0, int nlev, int B, int n_blocks,
                                                      const BlockMeta* __restrict__ meta,
                                                      const BlockPlan* __restrict__ plan,
                                                      const int32_t* __restrict__ bin_start,
                                                      const float* __restrict__ coords,
                                                      const float* __restrict__ dfeat, int64_t ls,
                                                      float* __restrict__ grad, int xcd_map) {
  constexpr int kPrivRecs = RECS > 0 ? RECS : 256;
  __shared__ int cstart[CELLS + 1];
  __shared__ float vacc[VFLOATS > 0 ? VFLOATS : 1];
  __shared__ float4 rt[RECS > 0 ? RECS : 1];            // tx, ty, tz of each placed sample
  __shared__ float rd[RECS > 0 ? RECS * F : 1];         // dL/dy of each placed sample
  __shared__ int part[CELLS > 0 ? 256 : 1];
  constexpr int PER = kPrivRecs / 256;   // samples per thread in a chunk
  const int nbins = B * B * B;
  int unit, l;  // unit = block * nbins + bin
  if (!level_major_item(blockIdx.x, l0, nlev, n_blocks * nbins, xcd_map, unit, l)) return;
  const int bin = unit % nbins;
  const int b = unit / nbins;
  if (plan[b].n == 0) return;  // no sample this step: its bin starts were not rewritten
  const int32_t* bs = bin_start + b * (kMaxBins + 1);
  const int s0 = bs[bin], s1 = bs[bin + 1];
  if (s0 >= s1) return;
  const int64_t base = plan[b].sample_off;
  const int R = ld.R[l];
  const float sc = ld.scale[l];
  const int dense = ld.dense[l];
  float* g = grad + meta[b].param_off + (int64_t)ld.off[l] * F;
  const int tid = threadIdx.x;
  // ---- 1. cell box of the bin: cell origins of its extreme coordinates (grid_pos
  // and bin_1d are both monotone in x, so every sample of the bin lies inside)
  int bo[3], bn[3];
  {
    const int bc[3] = {bin % B, (bin / B) % B, bin / (B * B)};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      float xl, xh, t;
      bin_x_range(bc[a], B, xl, xh);
      int il, ih;
      grid_pos(xl, sc, R, il, t);
      grid_pos(xh, sc, R, ih, t);
      bo[a] = il;
      bn[a] = ih - il + 1;
    }
  }
  const int bx0 = bo[0], by0 = bo[1], bz0 = bo[2];
  const int cx_n = bn[0], cy_n = bn[1], cz_n = bn[2];  // cells per axis
  const int vx_n = cx_n + 1, vy_n = cy_n + 1, vz_n = cz_n + 1;                           // vertices per axis
  const int64_t C = (int64_t)cx_n * cy_n * cz_n;
  const int64_t NV = (int64_t)vx_n * vy_n * vz_n;
  if (CELLS == 0 || C > CELLS || NV * F > VFLOATS) {
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
  const int nc = (int)C, nvf = (int)NV * F;
  for (int i = tid; i < nvf; i += 256) vacc[i] = 0.0f;
  // lanes per cell in the cell pass: the largest power of two <= min(8, 256 / nc),
  // so that a cell's lanes are aligned neighbours within one wave
  const int sub = nc > 128 ? 1 : (nc > 64 ? 2 : (nc > 32 ? 4 : 8));
  for (int c0 = s0; c0 < s1; c0 += kPrivRecs) {
    const int cn = min(kPrivRecs, s1 - c0);
    for (int i = tid; i <= nc; i += 256) cstart[i] = 0;
    __syncthreads();
    // ---- 2a. cell of each sample and its rank within the cell.  All of the
    // lane's coordinates and dL/dy are loaded first (indices clamped into the
    // chunk), so that the loads are in flight together
    int mcell[PER], mrank[PER];
    float mt[PER][3], md[PER][F], mx[PER][3];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int64_t gi = base + c0 + min(tid + 256 * u, cn - 1);
#pragma unroll
      for (int a = 0; a < 3; ++a) mx[u][a] = coords[3 * gi + a];
#pragma unroll
      for (int f = 0; f < F; ++f) md[u][f] = dfeat[(int64_t)l * ls + gi * F + f];
    }
    // cells of every sample (unconditionally, so that no load is sunk into
    // a branch and waited for there), then the ranks
    int mi[PER][3];
#pragma unroll
    for (int u = 0; u < PER; ++u)
#pragma unroll
      for (int a = 0; a < 3; ++a) grid_pos(mx[u][a], sc, R, mi[u][a], mt[u][a]);
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int j = tid + 256 * u;
      mcell[u] = -1;
      if (j < cn) {
        const int* i0 = mi[u];
        const int lx = i0[0] - bx0, ly = i0[1] - by0, lz = i0[2] - bz0;
        if ((unsigned)lx < (unsigned)cx_n && (unsigned)ly < (unsigned)cy_n && (unsigned)lz < (unsigned)cz_n) {
          mcell[u] = lx + cx_n * (ly + cy_n * lz);
          mrank[u] = atomicAdd(&cstart[mcell[u]], 1);
        } else {
          // outside the bin's box (not expected; kept for safety): direct atomics
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const int kx = k & 1, ky = (k >> 1) & 1, kz = k >> 2;
            const uint32_t e = corner_index(dense, R, ld.T_mask, i0[0] + kx, i0[1] + ky, i0[2] + kz);
            const float w = (kx ? mt[u][0] : 1.0f - mt[u][0]) * (ky ? mt[u][1] : 1.0f - mt[u][1]) *
                            (kz ? mt[u][2] : 1.0f - mt[u][2]);
#pragma unroll
            for (int f = 0; f < F; ++f) unsafeAtomicAdd(&g[(int64_t)e * F + f], w * md[u][f]);
          }
        }
      }
    }
    __syncthreads();
    // ---- 2b. exclusive scan of the cell counts (contiguous chunk per thread)
    {
      const int chunk = (nc + 255) / 256;
      const int a0 = tid * chunk, a1 = min(nc, a0 + chunk);
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
      if (tid == 255) cstart[nc] = part[255];
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
    // ---- 3. cell pass: corner sums in registers, one LDS atomic per (corner, feature)
    for (int q0 = 0; q0 < nc * sub; q0 += 256) {  // uniform trip count: the whole wave shuffles
      const int q = q0 + tid;
      const bool live = q < nc * sub;
      const int c = live ? q / sub : 0, s = q & (sub - 1);
      int p = 0, p1 = 0;
      if (live) {
        p1 = cstart[c + 1];
        p = cstart[c] + s;
      }
      float acc[8][F];
#pragma unroll
      for (int k = 0; k < 8; ++k)
#pragma unroll
        for (int f = 0; f < F; ++f) acc[k][f] = 0.0f;
      for (; p < p1; p += sub) {
        const float4 t = rt[p];
        float d[F];
#pragma unroll
        for (int f = 0; f < F; ++f) d[f] = rd[p * F + f];
        const float wx[2] = {1.0f - t.x, t.x}, wy[2] = {1.0f - t.y, t.y}, wz[2] = {1.0f - t.z, t.z};
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const float w = wx[k & 1] * wy[(k >> 1) & 1] * wz[k >> 2];
#pragma unroll
          for (int f = 0; f < F; ++f) acc[k][f] += w * d[f];
        }
      }
      // the cell's sub lanes combine their partial sums; its first lane adds them
      for (int o = 1; o < sub; o <<= 1)
#pragma unroll
        for (int k = 0; k < 8; ++k)
#pragma unroll
          for (int f = 0; f < F; ++f) acc[k][f] += __shfl_xor(acc[k][f], o, 64);
      if (!live || s != 0 || cstart[c] == p1) continue;
      const int lx = c % cx_n, ly = (c / cx_n) % cy_n, lz = c / (cx_n * cy_n);
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int v = (lx + (k & 1)) + vx_n * ((ly + ((k >> 1) & 1)) + vy_n * (lz + (k >> 2)));
#pragma unroll
        for (int f = 0; f < F; ++f) atomicAdd(&vacc[v * F + f], acc[k][f]);
      }
    }
    __syncthreads();
  }
  // ---- 4. vertex pass, x fastest: one global atomic per nonzero sum
  for (int e = tid; e < nvf; e += 256) {
    const float acc = vacc[e];
    if (acc == 0.0f) continue;
    const int v = e / F, f = e - v * F;
    const int lx = v % vx_n, ly = (v / vx_n) % vy_n, lz = v / (vx_n * vy_n);
    const uint32_t ent = corner_index(dense, R, ld.T_mask, (uint32_t)(bx0 + lx), (uint32_t)(by0 + ly),
                                      (uint32_t)(bz0 + lz));
    unsafeAtomicAdd(&g[(int64_t)ent * F + f], acc);
  }
}

hipError_t launch_scatter_priv(const LevelDesc& ld, int l0, int l1, int B, int n_blocks, const BlockMeta* meta,
                               const BlockPlan* plan, const int32_t* bin_start, const float* coords,
                               const float* dfeat, int64_t ls, float* grad, int xcd_map, int size_class,
                               hipStream_t s) {
  const int nlev = l1 - l0;
  if (nlev <= 0) return hipSuccess;
  const int grid = level_major_grid(nlev, n_blocks * B * B * B, xcd_map);
  if (grid <= 0) return hipSuccess;
#define DVNR_PRIV_LAUNCH(FF, CC, VV, RR)                                                                         \
  hipLaunchKernelGGL((k_scatter_priv<FF, CC, VV, RR>), dim3(grid), dim3(256), 0, s, ld, l0, nlev, B, n_blocks, meta, \
                     plan, bin_start, coords, dfeat, ls, grad, xcd_map)
#define DVNR_PRIV_CLASSES(FF)                                                                                 \
  if (size_class == 0) DVNR_PRIV_LAUNCH(FF, 0, 0, 0);                                                         \
  else if (size_class == 1) DVNR_PRIV_LAUNCH(FF, kPrivCellsSmall, kPrivVertFloatsSmall, 512);                 \
  else DVNR_PRIV_LAUNCH(FF, kPrivCells, kPrivVertFloats, 1024);
  switch (ld.F) {
    case 1: DVNR_PRIV_CLASSES(1) break;
    case 2: DVNR_PRIV_CLASSES(2) break;
    case 4: DVNR_PRIV_CLASSES(4) break;
    case 8: DVNR_PRIV_CLASSES(8) break;
    default: return hipErrorInvalidValue;
  }
#undef DVNR_PRIV_CLASSES
#undef DVNR_PRIV_LAUNCH
  return hipGetLastError();
}

}  // namespace dvnrk
