// Sampler, hash-grid encoding forward, encoding backward (scatter-add), Adam,
// slot reduction and small utility kernels of the DVNR hot path (gfx950).
#include "dvnr_device.h"

namespace dvnrk {

// ===========================================================================
// Element conversion helpers
// ===========================================================================
template <typename T> __device__ __forceinline__ float to_f(T v) { return (float)v; }
template <> __device__ __forceinline__ float to_f<__half>(__half v) { return __half2float(v); }
template <typename T> __device__ __forceinline__ double to_d(T v) { return (double)v; }
template <> __device__ __forceinline__ double to_d<__half>(__half v) { return (double)__half2float(v); }

template <typename T> __device__ __forceinline__ T from_f(float v) { return (T)v; }
template <> __device__ __forceinline__ __bf16 from_f<__bf16>(float v) { return (__bf16)v; }

// Sample addressing shared by the level-major kernels: either a tile table
// (training: tiles of one block each) or a direct range [0, n_direct) of one
// block's samples (autograd building blocks).
struct SampleRef {
  int64_t gi;       // sample index in the coordinate / feature buffers
  int block;        // block id (0 in direct mode)
  bool valid;
};

__device__ __forceinline__ SampleRef sample_ref(const Tile* tiles, const BlockPlan* plan, int tile, int64_t n_direct,
                                                int direct_block, int j) {
  SampleRef r;
  if (tiles) {
    const Tile tl = tiles[tile];
    r.block = tl.block;
    r.valid = j < tl.count;
    r.gi = plan[tl.block].sample_off + tl.start + j;
  } else {
    r.block = direct_block;
    r.gi = (int64_t)tile * kTile + j;
    r.valid = r.gi < n_direct;
  }
  return r;
}

// ===========================================================================
// Sampler: uniform coordinates (Philox4x32-10, counter (i, step, block, tag),
// key = seed) and trilinear ground truth in cell-centered convention:
// stored-index position p = x*n - 1/2 + g, i0 = clamp(floor p, 0, N-2),
// t = clamp(p - i0, 0, 1); target = (v - vmin) / (vmax - vmin).
// ===========================================================================
__device__ __forceinline__ void cell_pos(float x, int n, int g, int N, int& i0, float& t) {
  const float p = x * (float)n - 0.5f + (float)g;
  int i = (int)floorf(p);
  i = max(0, min(i, N - 2));
  i0 = i;
  t = fminf(fmaxf(p - (float)i, 0.0f), 1.0f);
}

__global__ __launch_bounds__(256) void k_sample(const BlockMeta* __restrict__ meta,
                                                const BlockRange* __restrict__ range,
                                                const BlockPlan* __restrict__ plan, const Tile* __restrict__ tiles,
                                                int64_t n_direct, int direct_block, int gen, uint64_t seed,
                                                SampleDist dist, const Counters* __restrict__ ctr,
                                                int64_t step_override,
                                                float* __restrict__ coords, float* __restrict__ target) {
  Tile tl;
  int64_t gi;
  const int j = threadIdx.x;
  if (tiles) {
    tl = tiles[blockIdx.x];
    if (j >= tl.count) return;
    gi = plan[tl.block].sample_off + tl.start + j;
  } else {
    tl.block = direct_block;
    tl.start = blockIdx.x * kTile;
    gi = tl.start + j;
    if (gi >= n_direct) return;
  }
  const int b = tl.block;
  float x, y, z;
  if (gen) {
    const uint32_t step = (uint32_t)(step_override >= 0 ? step_override : ctr->step);
    const int n_uni = tiles ? plan[b].n_uni : dist.direct_n_uni;
    train_coord((uint32_t)(tl.start + j), step, (uint32_t)b, n_uni, dist.sigma_sqrt2, seed, x, y, z);
    coords[3 * gi + 0] = x;
    coords[3 * gi + 1] = y;
    coords[3 * gi + 2] = z;
  } else {
    x = coords[3 * gi + 0];
    y = coords[3 * gi + 1];
    z = coords[3 * gi + 2];
  }
  const BlockMeta bm = meta[b];
  const int g = bm.ghost;
  const int NX = bm.dims[0] + 2 * g, NY = bm.dims[1] + 2 * g, NZ = bm.dims[2] + 2 * g;
  int ix, iy, iz;
  float tx, ty, tz;
  cell_pos(x, bm.dims[0], g, NX, ix, tx);
  cell_pos(y, bm.dims[1], g, NY, iy, ty);
  cell_pos(z, bm.dims[2], g, NZ, iz, tz);
  const float* v = bm.vol + ((int64_t)iz * NY + iy) * NX + ix;
  const int64_t sy = NX, sz = (int64_t)NX * NY;
  const float c00 = v[0] + tx * (v[1] - v[0]);
  const float c10 = v[sy] + tx * (v[sy + 1] - v[sy]);
  const float c01 = v[sz] + tx * (v[sz + 1] - v[sz]);
  const float c11 = v[sz + sy] + tx * (v[sz + sy + 1] - v[sz + sy]);
  const float c0 = c00 + ty * (c10 - c00);
  const float c1 = c01 + ty * (c11 - c01);
  const float val = c0 + tz * (c1 - c0);
  const BlockRange br = range[b];
  target[gi] = (val - br.vmin) * br.inv_range;
}

hipError_t launch_sample(const BlockMeta* meta, const BlockRange* range, const BlockPlan* plan, const Tile* tiles,
                         int n_tiles, int direct_block, int gen, uint64_t seed, SampleDist dist, const Counters* ctr,
                         int64_t step_override, float* coords, float* target, hipStream_t s) {
  int64_t n_direct = 0;
  int nt = n_tiles;
  if (!tiles) {
    n_direct = n_tiles;
    nt = (int)((n_direct + kTile - 1) / kTile);
  }
  if (nt <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sample, dim3(nt), dim3(kTile), 0, s, meta, range, plan, tiles, n_direct, direct_block, gen,
                     seed, dist, ctr, step_override, coords, target);
  return hipGetLastError();
}

// ===========================================================================
// Encoding forward: two lanes per (sample, level); level-major workgroups of
// one tile (kTile samples) and one level.
// y[l*F + f] = sum_c w_c * table[(off_l + idx_c) * F + f]
// Lane cx of a sample's pair gathers the four corners with that x offset, so
// that one load instruction reads both x-neighbours of a (cy, cz) pair from
// adjacent lanes: adjacent entries on dense levels, and on hashed levels
// entries that differ in their low index bits only (the x prime is 1), which
// mostly share a cache line and are served by one request.  Each lane sums its
// four corners in the order (cy, cz) = (0,0), (1,0), (0,1), (1,1); the pair's
// sums are added (cx = 0 first).
// ===========================================================================
// With LPW = 2 (a launch of more than 8 levels on the XCD-aware mapping) a
// workgroup takes both levels that its XCD serves, x and x + 8, for SPT
// consecutive tiles: each sample's coordinates are read once and a lane has
// 4 LPW SPT gathers in flight.  When level x + 8 is not in the launch the
// lane repeats level x's loads and skips the second write; a sample past its
// tile's end interpolates the cube's center and writes nothing.
#ifndef DVNR_ENCODE_LEVELS_PER_WG
#define DVNR_ENCODE_LEVELS_PER_WG 2
#endif
constexpr int kEncodeLevelsPerWg = DVNR_ENCODE_LEVELS_PER_WG;  // 1 or 2
#ifndef DVNR_ENCODE_TILES_PER_WG
#define DVNR_ENCODE_TILES_PER_WG 2
#endif
constexpr int kEncodeTilesPerWg = DVNR_ENCODE_TILES_PER_WG;  // tiles per workgroup with two levels (1 or 2)

template <typename TT, typename WT, typename OT, int F, int LPW, int SPT>
__global__ __launch_bounds__(2 * kTile) void k_encode(LevelDesc ld, const BlockMeta* __restrict__ meta,
                                                      const Tile* __restrict__ tiles, int n_tiles, int64_t n_direct,
                                                      int direct_block, const BlockPlan* __restrict__ plan,
                                                      const float* __restrict__ coords, const TT* __restrict__ table,
                                                      OT* __restrict__ out, int64_t ss, int64_t ls, int xcd_map,
                                                      int l0, int nl) {
  static_assert(LPW == 2 || SPT == 1, "several tiles per workgroup only with two levels");
  int tile0, lv[LPW];
  bool second = false;
  if constexpr (LPW == 1) {
    if (!level_major_item(blockIdx.x, l0, nl, n_tiles, xcd_map, tile0, lv[0])) return;
  } else {
    const int x = blockIdx.x & 7;
    tile0 = (blockIdx.x >> 3) * SPT;
    if (tile0 >= n_tiles || x >= nl) return;
    second = x + 8 < nl;
    lv[0] = l0 + x;
    lv[1] = second ? l0 + x + 8 : l0 + x;
  }
  const uint32_t cx = threadIdx.x & 1;
  // both lanes of a pair share the samples, so they leave together
  SampleRef r[SPT];
  bool any = false;
#pragma unroll
  for (int t = 0; t < SPT; ++t) {
    if (tile0 + t < n_tiles) {
      r[t] = sample_ref(tiles, plan, tile0 + t, n_direct, direct_block, threadIdx.x >> 1);
    } else {
      r[t] = r[0];
      r[t].valid = false;
    }
    any |= r[t].valid;
  }
  if (!any) return;
  WT wx[SPT][LPW], wy[SPT][LPW][2], wz[SPT][LPW][2];
  TT v[SPT][LPW][4][F];
  // every sample's coordinates before any gather (a load issued after the
  // gathers would make the wait for it wait for them too)
  float px[SPT], py[SPT], pz[SPT];
#pragma unroll
  for (int t = 0; t < SPT; ++t) {
    const int64_t gi = r[t].valid ? r[t].gi : r[0].gi;
    px[t] = coords[3 * gi + 0];
    py[t] = coords[3 * gi + 1];
    pz[t] = coords[3 * gi + 2];
  }
#pragma unroll
  for (int t = 0; t < SPT; ++t) {
    const float x = r[t].valid ? px[t] : 0.5f, y = r[t].valid ? py[t] : 0.5f, z = r[t].valid ? pz[t] : 0.5f;
    const TT* tab0 = table + (meta ? meta[r[t].block].param_off : 0);
#pragma unroll
    for (int j = 0; j < LPW; ++j) {  // loads first, all in flight together
      const int l = lv[j];
      int ix, iy, iz;
      float tx, ty, tz;
      const int R = ld.R[l];
      grid_pos(x, ld.scale[l], R, ix, tx);
      grid_pos(y, ld.scale[l], R, iy, ty);
      grid_pos(z, ld.scale[l], R, iz, tz);
      const TT* tab = tab0 + (int64_t)ld.off[l] * F;
      const int dense = ld.dense[l];
      wx[t][j] = cx ? (WT)tx : (WT)1 - (WT)tx;
      wy[t][j][0] = (WT)1 - (WT)ty;
      wy[t][j][1] = (WT)ty;
      wz[t][j][0] = (WT)1 - (WT)tz;
      wz[t][j][1] = (WT)tz;
      // the four indices first, branch-free (both forms, then a select), so
      // that the four loads issue back to back from one basic block
      uint32_t e[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t cy = k & 1, cz = k >> 1;
        const uint32_t gx = ix + cx, gy = iy + cy, gz = iz + cz;
        const uint32_t ed = gx + __umul24((uint32_t)R, gy + __umul24((uint32_t)R, gz));
        const uint32_t eh = (gx ^ (gy * 2654435761u) ^ (gz * 805459861u)) & ld.T_mask;
        e[k] = dense ? ed : eh;
      }
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int f = 0; f < F; ++f) v[t][j][k][f] = tab[(int64_t)e[k] * F + f];
    }
  }
#pragma unroll
  for (int t = 0; t < SPT; ++t)
#pragma unroll
    for (int j = 0; j < LPW; ++j) {
      WT acc[F];
#pragma unroll
      for (int f = 0; f < F; ++f) acc[f] = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const WT w = wx[t][j] * wy[t][j][k & 1] * wz[t][j][k >> 1];
#pragma unroll
        for (int f = 0; f < F; ++f) {
          if constexpr (sizeof(WT) == 8)
            acc[f] += w * to_d(v[t][j][k][f]);
          else
            acc[f] += w * to_f(v[t][j][k][f]);
        }
      }
#pragma unroll
      for (int f = 0; f < F; ++f) {
        const WT o = __shfl_xor(acc[f], 1, 64);
        acc[f] = cx ? o + acc[f] : acc[f] + o;  // (cx = 0 sum) + (cx = 1 sum) on both lanes
      }
      if (cx == 0 && r[t].valid && (j == 0 || second)) {
        OT* o = out + r[t].gi * ss + (int64_t)lv[j] * ls;
#pragma unroll
        for (int f = 0; f < F; ++f) o[f] = (OT)acc[f];
      }
    }
}

template <typename TT, typename WT, typename OT>
static hipError_t enc_dispatch(const LevelDesc& ld, const BlockMeta* meta, const Tile* tiles, int n_tiles,
                               int64_t n_direct, int direct_block, const BlockPlan* plan, const float* coords, const void* table,
                               void* out, int64_t ss, int64_t ls, int xcd_map, int l0, int nl, hipStream_t s) {
  // two levels per workgroup where the XCD-aware mapping gives an XCD two
  // levels (9 to 16 levels in the launch)
  const bool two = kEncodeLevelsPerWg == 2 && xcd_map && nl > 8 && nl <= 16;
  constexpr int SPT = kEncodeTilesPerWg;
  const int64_t grid =
      two ? 8 * (((int64_t)n_tiles + SPT - 1) / SPT) : (int64_t)level_major_grid(nl, n_tiles, xcd_map);
  if (grid <= 0) return hipSuccess;
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  const TT* t = (const TT*)table;
  OT* o = (OT*)out;
#define DVNR_ENC_LAUNCH(FF, LL, SS)                                                                          \
  hipLaunchKernelGGL((k_encode<TT, WT, OT, FF, LL, SS>), dim3((unsigned)grid), dim3(2 * kTile), 0, s, ld, meta, \
                     tiles, n_tiles, n_direct, direct_block, plan, coords, t, o, ss, ls, xcd_map, l0, nl)
#define DVNR_ENC_CASE(FF)          \
  case FF:                         \
    if (two)                       \
      DVNR_ENC_LAUNCH(FF, 2, SPT); \
    else                           \
      DVNR_ENC_LAUNCH(FF, 1, 1);   \
    break;
  switch (ld.F) {
    DVNR_ENC_CASE(1)
    DVNR_ENC_CASE(2)
    DVNR_ENC_CASE(4)
    DVNR_ENC_CASE(8)
    default: return hipErrorInvalidValue;
  }
#undef DVNR_ENC_CASE
#undef DVNR_ENC_LAUNCH
  return hipGetLastError();
}

// out_kind: 0 = float, 1 = bf16, 2 = double.  Direct mode when tiles == nullptr
// (then n_tiles is the sample count).
hipError_t launch_encode(Prec tp, int out_kind, const LevelDesc& ld, const BlockMeta* meta, const Tile* tiles,
                         int n_tiles, int direct_block, const BlockPlan* plan, const float* coords, const void* table,
                         void* out, int64_t ss, int64_t ls, int xcd_map, hipStream_t s, int l0, int l1) {
  if (l1 < 0) l1 = ld.L;
  const int nl = l1 - l0;
  if (nl <= 0) return hipSuccess;
  int64_t n_direct = 0;
  int nt = n_tiles;
  if (!tiles) {
    n_direct = n_tiles;
    nt = (int)((n_direct + kTile - 1) / kTile);
  }
  if (tp == Prec::F64) return enc_dispatch<double, double, double>(ld, meta, tiles, nt, n_direct, direct_block, plan, coords, table, out, ss, ls, xcd_map, l0, nl, s);
  if (tp == Prec::MIXED) {
    if (out_kind == 1) return enc_dispatch<__half, float, __bf16>(ld, meta, tiles, nt, n_direct, direct_block, plan, coords, table, out, ss, ls, xcd_map, l0, nl, s);
    return enc_dispatch<__half, float, float>(ld, meta, tiles, nt, n_direct, direct_block, plan, coords, table, out, ss, ls, xcd_map, l0, nl, s);
  }
  return enc_dispatch<float, float, float>(ld, meta, tiles, nt, n_direct, direct_block, plan, coords, table, out, ss, ls, xcd_map, l0, nl, s);
}

// ===========================================================================
// Encoding backward: grad[(off_l + idx_c) * F + f] += w_c * dy[l*F + f].
//
// Plain variant: one thread per (sample, level) issues its 8*F atomics.
// Grouped variant: 2F consecutive lanes own the two x-neighbour corners
// (cx = 0, 1) of one (sample, level, cy, cz) and all F features, so one
// atomic instruction covers 16 contiguous bytes per lane group (F = 2):
// dense levels place the pair side by side, and the hash (x prime 1) keeps
// it within one aligned 64-byte segment in most cases.  The atomic unit
// serves one 64-byte segment per request, so this cuts requests ~4x.
// ===========================================================================
template <typename GT, typename DT, int F, bool GROUPED>
__global__ __launch_bounds__(256) void k_scatter(LevelDesc ld, const BlockMeta* __restrict__ meta,
                                                 const Tile* __restrict__ tiles, int n_tiles, int64_t n_direct,
                                                 int direct_block, const BlockPlan* __restrict__ plan,
                                                 const float* __restrict__ coords, const DT* __restrict__ dfeat,
                                                 int64_t ss, int64_t ls, GT* __restrict__ grad, int xcd_map,
                                                 int l0, int nl, int strided) {
  int tile, l;
  if (!level_major_item(blockIdx.x, l0, nl, n_tiles, xcd_map, tile, l)) return;
  const int R = ld.R[l];
  const float sc = ld.scale[l];
  const int dense = ld.dense[l];
  if constexpr (!GROUPED) {
    const SampleRef r = sample_ref(tiles, plan, tile, n_direct, direct_block, threadIdx.x);
    if (!r.valid) return;
    const float x = coords[3 * r.gi + 0], y = coords[3 * r.gi + 1], z = coords[3 * r.gi + 2];
    int ix, iy, iz;
    float tx, ty, tz;
    grid_pos(x, sc, R, ix, tx);
    grid_pos(y, sc, R, iy, ty);
    grid_pos(z, sc, R, iz, tz);
    using WT = typename std::conditional<sizeof(GT) == 8, double, float>::type;
    const WT wx[2] = {(WT)1 - (WT)tx, (WT)tx};
    const WT wy[2] = {(WT)1 - (WT)ty, (WT)ty};
    const WT wz[2] = {(WT)1 - (WT)tz, (WT)tz};
    const DT* d = dfeat + r.gi * ss + (int64_t)l * ls;
    WT dv[F];
#pragma unroll
    for (int f = 0; f < F; ++f) dv[f] = (WT)d[f];
    GT* g = grad + (meta ? meta[r.block].param_off : 0) + (int64_t)ld.off[l] * F;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint32_t cx = k & 1, cy = (k >> 1) & 1, cz = (k >> 2) & 1;
      const uint32_t e = corner_index(dense, R, ld.T_mask, ix + cx, iy + cy, iz + cz);
      const WT w = wx[cx] * wy[cy] * wz[cz];
#pragma unroll
      for (int f = 0; f < F; ++f) unsafeAtomicAdd(&g[(int64_t)e * F + f], (GT)(w * dv[f]));
    }
  } else {
    constexpr int G = 2 * F;               // lanes per (sample, cy, cz) item
    const int q = threadIdx.x % G;         // lane within the group
    const int cx = q / F, f = q % F;
    int count;
    int64_t base;
    int block;
    // strided: tile t' of a block with n samples takes samples j * ceil(n/256) + t', so
    // that the lanes of an instruction do not come from one spatial bin of an ordered
    // sample buffer (neighbouring samples would hit the same entries and serialize)
    int64_t stride = 0, first = 0, n_valid = 0;
    if (tiles) {
      const Tile tl = tiles[tile];
      block = tl.block;
      if (strided) {
        n_valid = plan[tl.block].n;
        stride = (n_valid + kTile - 1) / kTile;
        first = tl.start / kTile;
        base = plan[tl.block].sample_off;
        count = kTile;
      } else {
        count = tl.count;
        base = plan[tl.block].sample_off + tl.start;
      }
    } else {
      base = (int64_t)tile * kTile;
      count = (int)min((int64_t)kTile, n_direct - base);
      block = direct_block;
    }
    GT* g = grad + (meta ? meta[block].param_off : 0) + (int64_t)ld.off[l] * F;
    const int items = count * 4;
    for (int it = threadIdx.x / G; it < items; it += kTile / G) {
      const int j = it >> 2, yz = it & 3;
      int64_t si = j;
      if (stride) {
        si = (int64_t)j * stride + first;
        if (si >= n_valid) continue;
      }
      const int64_t gi = base + si;
      const float x = coords[3 * gi + 0], y = coords[3 * gi + 1], z = coords[3 * gi + 2];
      int ix, iy, iz;
      float tx, ty, tz;
      grid_pos(x, sc, R, ix, tx);
      grid_pos(y, sc, R, iy, ty);
      grid_pos(z, sc, R, iz, tz);
      const uint32_t cy = yz & 1, cz = yz >> 1;
      const uint32_t e = corner_index(dense, R, ld.T_mask, ix + cx, iy + cy, iz + cz);
      const float w = (cx ? tx : 1.0f - tx) * (cy ? ty : 1.0f - ty) * (cz ? tz : 1.0f - tz);
      const float dv = (float)dfeat[gi * ss + (int64_t)l * ls + f];
      unsafeAtomicAdd(&g[(int64_t)e * F + f], (GT)(w * dv));
    }
  }
}

template <typename GT, typename DT, bool GROUPED>
static hipError_t scat_dispatch(const LevelDesc& ld, int l0, int nl, const BlockMeta* meta, const Tile* tiles, int nt,
                                int64_t n_direct, int direct_block, const BlockPlan* plan, const float* coords,
                                const void* dfeat, int64_t ss, int64_t ls, void* grad, int xcd_map, int strided,
                                hipStream_t s) {
  const int grid = level_major_grid(nl, nt, xcd_map);
  if (grid <= 0 || nl <= 0) return hipSuccess;
  const DT* d = (const DT*)dfeat;
  GT* g = (GT*)grad;
  switch (ld.F) {
    case 1: hipLaunchKernelGGL((k_scatter<GT, DT, 1, GROUPED>), dim3(grid), dim3(kTile), 0, s, ld, meta, tiles, nt, n_direct, direct_block, plan, coords, d, ss, ls, g, xcd_map, l0, nl, strided); break;
    case 2: hipLaunchKernelGGL((k_scatter<GT, DT, 2, GROUPED>), dim3(grid), dim3(kTile), 0, s, ld, meta, tiles, nt, n_direct, direct_block, plan, coords, d, ss, ls, g, xcd_map, l0, nl, strided); break;
    case 4: hipLaunchKernelGGL((k_scatter<GT, DT, 4, GROUPED>), dim3(grid), dim3(kTile), 0, s, ld, meta, tiles, nt, n_direct, direct_block, plan, coords, d, ss, ls, g, xcd_map, l0, nl, strided); break;
    case 8: hipLaunchKernelGGL((k_scatter<GT, DT, 8, GROUPED>), dim3(grid), dim3(kTile), 0, s, ld, meta, tiles, nt, n_direct, direct_block, plan, coords, d, ss, ls, g, xcd_map, l0, nl, strided); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_scatter(Prec gp, const LevelDesc& ld, int l0, int l1, const BlockMeta* meta, const Tile* tiles,
                          int n_tiles, int direct_block, const BlockPlan* plan, const float* coords, const void* dfeat,
                          int64_t ss, int64_t ls, void* grad, int grouped, int xcd_map, int strided, hipStream_t s) {
  int64_t n_direct = 0;
  int nt = n_tiles;
  if (!tiles) {
    n_direct = n_tiles;
    nt = (int)((n_direct + kTile - 1) / kTile);
    strided = 0;
  }
  const int nl = l1 - l0;
  if (gp == Prec::F64)
    return scat_dispatch<double, double, false>(ld, l0, nl, meta, tiles, nt, n_direct, direct_block, plan, coords, dfeat, ss, ls, grad, xcd_map, 0, s);
  if (grouped)
    return scat_dispatch<float, float, true>(ld, l0, nl, meta, tiles, nt, n_direct, direct_block, plan, coords, dfeat, ss, ls, grad, xcd_map, strided, s);
  return scat_dispatch<float, float, false>(ld, l0, nl, meta, tiles, nt, n_direct, direct_block, plan, coords, dfeat, ss, ls, grad, xcd_map, 0, s);
}

// ===========================================================================
// Slot reduction: per block, sum the dW / loss partials written by the
// workgroups that processed the block's tiles.  Slots of block b are
// [slot_ranges[2b], slot_ranges[2b+1]).  Writes the MLP gradient (overwrite)
// and the block's mean loss into the loss ring.  A workgroup covers 32
// consecutive elements; its 8 rows of 32 lanes split the slot range
// (coalesced 128-byte rows, eight slots in flight per lane), then reduce
// through LDS in a fixed order.
// ===========================================================================
template <typename GT>
__global__ __launch_bounds__(256) void k_reduce_slots(const float* __restrict__ slots, int64_t slot_stride,
                                                      const int32_t* __restrict__ ranges, int64_t n_mlp,
                                                      int64_t mlp_rel_off, int64_t block_stride,
                                                      GT* __restrict__ grad, float* __restrict__ loss_ring,
                                                      Counters* __restrict__ ctr, int n_blocks, int bump) {
  __shared__ float part[8][33];
  const int b = blockIdx.y;
  const int c = threadIdx.x % 32, r = threadIdx.x / 32;
  const int64_t e = (int64_t)blockIdx.x * 32 + c;
  const int s0 = ranges[2 * b], s1 = ranges[2 * b + 1];
  // a row walks slots s0 + r, s0 + r + 8, ...: eight independent partial sums
  // keep eight loads in flight per lane (the summation order stays fixed)
  float a8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (e <= n_mlp) {
    int sl = s0 + r;
    for (; sl + 56 < s1; sl += 64) {
      float v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) v[k] = slots[(int64_t)(sl + 8 * k) * slot_stride + e];
#pragma unroll
      for (int k = 0; k < 8; ++k) a8[k] += v[k];
    }
#pragma unroll
    for (int k = 0; k < 7; ++k)
      if (sl + 8 * k < s1) a8[k] += slots[(int64_t)(sl + 8 * k) * slot_stride + e];
  }
  float acc = 0.0f;
#pragma unroll
  for (int k = 0; k < 8; ++k) acc += a8[k];
  part[r][c] = acc;
  __syncthreads();
  if (r != 0 || e > n_mlp) return;
  float sum = 0.0f;
#pragma unroll
  for (int k = 0; k < 8; ++k) sum += part[k][c];
  if (e < n_mlp) {
    grad[(int64_t)b * block_stride + mlp_rel_off + e] = (GT)sum;
  } else {
    // one lane per block reads the step counter; the last of them to finish
    // advances it (all reads precede every arrival on the done counter)
    const int64_t step = ctr->step;
    loss_ring[(step % kLossRing) * n_blocks + b] = sum;
    if (!isfinite(sum)) ctr->nonfinite = 1;
    if (bump) {
      __threadfence();
      if (atomicAdd(&ctr->done, 1) == n_blocks - 1) {
        ctr->done = 0;
        ctr->step = step + 1;
      }
    }
  }
}

hipError_t launch_reduce_slots(const float* slots, int64_t slot_stride, const int32_t* slot_ranges, int n_blocks,
                               int64_t n_mlp, int64_t mlp_rel_off, int64_t block_stride, Prec gp, void* grad,
                               float* loss_ring, Counters* ctr, int bump, hipStream_t s) {
  dim3 grid((unsigned)((n_mlp + 1 + 31) / 32), (unsigned)n_blocks);
  if (gp == Prec::F64)
    hipLaunchKernelGGL(k_reduce_slots<double>, grid, dim3(256), 0, s, slots, slot_stride, slot_ranges, n_mlp,
                       mlp_rel_off, block_stride, (double*)grad, loss_ring, ctr, n_blocks, bump);
  else
    hipLaunchKernelGGL(k_reduce_slots<float>, grid, dim3(256), 0, s, slots, slot_stride, slot_ranges, n_mlp,
                       mlp_rel_off, block_stride, (float*)grad, loss_ring, ctr, n_blocks, bump);
  return hipGetLastError();
}

// ===========================================================================
// Adam with L2 weight decay (every parameter, every step):
//   g += wd*theta; m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
//   theta -= lr_t * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps); g = 0,
// lr_t = lr * base^(max(0, t - start) / interval) (exponential decay; interval
// 0: constant).
// Mixed precision also refreshes the 16-bit working copy (fp16 tables, bf16
// weights, round to nearest even).  4 elements per thread (block_stride is
// a multiple of 64, so a group of 4 never straddles two blocks).
// ===========================================================================
template <typename P>
__global__ __launch_bounds__(256) void k_adam(P* __restrict__ params, P* __restrict__ grad, P* __restrict__ mom,
                                              P* __restrict__ vel, uint16_t* __restrict__ work16,
                                              int64_t block_stride, int64_t n_table, int64_t n_used,
                                              const BlockPlan* __restrict__ plan, const Counters* __restrict__ ctr,
                                              P lr0, P b1, P b2, P omb1, P omb2, P eps, P wd, P ln_b1,
                                              P ln_b2, P log2_decay, int64_t decay_start,
                                              int64_t decay_interval, int64_t skip0, int64_t skip1) {
  // grid (element groups of the block, blocks): no division per element, one
  // uniform skip for a block that drew no sample this step
  const int b = blockIdx.y;
  if (plan && plan[b].n == 0) return;
  __shared__ P bc[3];
  if (threadIdx.x == 0) {
    // this update's index t (1, 2, ...): the slot reduction advanced the counter
    adam_factors<P>(ctr->step, lr0, ln_b1, ln_b2, log2_decay, decay_start, decay_interval, bc[0], bc[1], bc[2]);
  }
  __syncthreads();
  const P bc1 = bc[0], bc2 = bc[1], lr = bc[2];
  // with a skipped range, the first pre = ceil(skip0 / 1024) workgroup columns
  // cover [0, 1024 pre) and the others [max(1024 pre, skip1 rounded down to
  // 1024), n_used): every element outside the range exactly once
  int64_t gx = blockIdx.x, base = 0;
  if (skip1 > skip0) {
    const int64_t pre = (skip0 + 1023) / 1024;
    if (gx >= pre) {
      base = max(pre * 1024, skip1 / 1024 * 1024);
      gx -= pre;
    }
  }
  const int64_t j0 = base + 4 * (gx * blockDim.x + threadIdx.x);
  if (j0 >= n_used) return;
  if (j0 >= skip0 && j0 + 4 <= skip1) return;  // updated by the slice pass
  const int64_t i0 = (int64_t)b * block_stride + j0;
  P th[4], g[4], m[4], v[4];
  if constexpr (sizeof(P) == 4) {
    // each stream is touched once per step: non-temporal 16-byte accesses
    // (except the gradient store below)
    typedef float f4 __attribute__((ext_vector_type(4)));
    const f4 a = __builtin_nontemporal_load(reinterpret_cast<const f4*>(params + i0));
    const f4 bg = __builtin_nontemporal_load(reinterpret_cast<const f4*>(grad + i0));
    const f4 bm = __builtin_nontemporal_load(reinterpret_cast<const f4*>(mom + i0));
    const f4 bv = __builtin_nontemporal_load(reinterpret_cast<const f4*>(vel + i0));
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      th[k] = a[k];
      g[k] = bg[k];
      m[k] = bm[k];
      v[k] = bv[k];
    }
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      th[k] = params[i0 + k];
      g[k] = grad[i0 + k];
      m[k] = mom[i0 + k];
      v[k] = vel[i0 + k];
    }
  }
  bool keep[4];  // elements of a group straddling the skipped range keep their values
#pragma unroll
  for (int k = 0; k < 4; ++k) keep[k] = j0 + k >= skip0 && j0 + k < skip1;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (j0 + k >= n_used) {
      g[k] = 0;
      continue;
    }
    if (keep[k]) continue;
    const P gg = g[k] + wd * th[k];
    m[k] = b1 * m[k] + omb1 * gg;
    v[k] = b2 * v[k] + omb2 * gg * gg;
    if constexpr (sizeof(P) == 4)  // hardware square root and reciprocal (about 1 ulp each)
      th[k] = th[k] - lr * bc1 * m[k] * __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(v[k] * bc2) + eps);
    else
      th[k] = th[k] - lr * (m[k] * bc1) / (sqrt(v[k] * bc2) + eps);
    g[k] = 0;
  }
  if constexpr (sizeof(P) == 4) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    __builtin_nontemporal_store(f4{th[0], th[1], th[2], th[3]}, reinterpret_cast<f4*>(params + i0));
    // the zeroed gradient stays cached: the next step's scatter atomics land on it
    *reinterpret_cast<f4*>(grad + i0) = f4{g[0], g[1], g[2], g[3]};
    __builtin_nontemporal_store(f4{m[0], m[1], m[2], m[3]}, reinterpret_cast<f4*>(mom + i0));
    __builtin_nontemporal_store(f4{v[0], v[1], v[2], v[3]}, reinterpret_cast<f4*>(vel + i0));
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      params[i0 + k] = th[k];
      grad[i0 + k] = g[k];
      mom[i0 + k] = m[k];
      vel[i0 + k] = v[k];
    }
  }
  if (work16) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (keep[k]) continue;
      const float f = (float)th[k];
      uint16_t bits;
      if (j0 + k < n_table) {
        const __half h = __float2half_rn(f);
        bits = *reinterpret_cast<const uint16_t*>(&h);
      } else {
        const __bf16 h = (__bf16)f;
        bits = *reinterpret_cast<const uint16_t*>(&h);
      }
      work16[i0 + k] = bits;
    }
  }
}

hipError_t launch_adam(Prec p, void* params, void* grad, void* m, void* v, uint16_t* work16, int n_blocks,
                       int64_t block_stride, int64_t n_table_params, int64_t n_used, const BlockPlan* plan,
                       const Counters* ctr, double lr, double b1, double b2, double eps, double wd,
                       double decay_base, int64_t decay_start, int64_t decay_interval, hipStream_t s,
                       int64_t skip0, int64_t skip1) {
  if (n_blocks <= 0 || n_used <= 0) return hipSuccess;
  if (n_blocks > 65535) return hipErrorInvalidValue;
  int64_t gx = (n_used + 1023) / 1024;
  if (skip1 > skip0) {
    const int64_t pre = (skip0 + 1023) / 1024, base = std::max(pre * 1024, skip1 / 1024 * 1024);
    gx = pre + std::max<int64_t>(0, (n_used - base + 1023) / 1024);
  }
  const dim3 grid((unsigned)gx, (unsigned)n_blocks);
  // once on the host: 1 - b (rounded once, not formed from the rounded b: with
  // b2 = 0.999, 1 - (float)b2 is 1.3e-5 away from 1 - b2), the logarithms of
  // the decay rates and of the learning-rate decay base
  const double omb1 = 1.0 - b1, omb2 = 1.0 - b2;
  const double ln_b1 = std::log(b1), ln_b2 = std::log(b2);
  const double log2_decay = decay_interval > 0 ? std::log2(decay_base) : 0.0;
  if (p == Prec::F64)
    hipLaunchKernelGGL(k_adam<double>, grid, dim3(256), 0, s, (double*)params, (double*)grad, (double*)m, (double*)v,
                       nullptr, block_stride, n_table_params, n_used, plan, ctr, lr, b1, b2, omb1, omb2, eps, wd,
                       ln_b1, ln_b2, log2_decay, decay_start, decay_interval, skip0, skip1);
  else
    hipLaunchKernelGGL(k_adam<float>, grid, dim3(256), 0, s, (float*)params, (float*)grad, (float*)m, (float*)v,
                       work16, block_stride, n_table_params, n_used, plan, ctr, (float)lr, (float)b1, (float)b2,
                       (float)omb1, (float)omb2, (float)eps, (float)wd, (float)ln_b1, (float)ln_b2,
                       (float)log2_decay, decay_start, decay_interval, skip0, skip1);
  return hipGetLastError();
}

// ===========================================================================
// Utilities
// ===========================================================================
__device__ __forceinline__ uint32_t order_key(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float key_float(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

__global__ void k_minmax_init(Counters* ctr, int n_blocks) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < n_blocks) {
    ctr->minmax[2 * b] = 0xffffffffu;
    ctr->minmax[2 * b + 1] = 0u;
  }
}

__global__ __launch_bounds__(256) void k_minmax(const BlockMeta* __restrict__ meta, Counters* __restrict__ ctr,
                                                const int64_t* __restrict__ nvox) {
  const int b = blockIdx.y;
  const float* v = meta[b].vol;
  const int64_t n = nvox[b];
  uint32_t lo = 0xffffffffu, hi = 0u;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t k = order_key(v[i]);
    lo = min(lo, k);
    hi = max(hi, k);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo = min(lo, (uint32_t)__shfl_xor((int)lo, o, 64));
    hi = max(hi, (uint32_t)__shfl_xor((int)hi, o, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMin(&ctr->minmax[2 * b], lo);
    atomicMax(&ctr->minmax[2 * b + 1], hi);
  }
}

__global__ void k_minmax_final(const Counters* ctr, BlockRange* range, int n_blocks) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_blocks) return;
  const float lo = key_float(ctr->minmax[2 * b]), hi = key_float(ctr->minmax[2 * b + 1]);
  BlockRange r;
  r.vmin = lo;
  r.vmax = hi;
  r.range = hi > lo ? hi - lo : 1.0f;
  r.inv_range = hi > lo ? 1.0f / (hi - lo) : 1.0f;
  range[b] = r;
}

hipError_t launch_minmax(const BlockMeta* meta, BlockRange* range, Counters* ctr, int n_blocks,
                         const int64_t* dev_voxels, hipStream_t s) {
  hipLaunchKernelGGL(k_minmax_init, dim3((n_blocks + 255) / 256), dim3(256), 0, s, ctr, n_blocks);
  hipLaunchKernelGGL(k_minmax, dim3(64, n_blocks), dim3(256), 0, s, meta, ctr, dev_voxels);
  hipLaunchKernelGGL(k_minmax_final, dim3((n_blocks + 255) / 256), dim3(256), 0, s, ctr, range, n_blocks);
  return hipGetLastError();
}

// Tables U(-1e-4, 1e-4), weight matrices Glorot-uniform U(-a, a) with
// a = sqrt(6 / (fan_in + fan_out)); Philox4x32-10 counter (j, block, 'INIT', 0).
template <typename P>
__global__ __launch_bounds__(256) void k_init(P* __restrict__ params, int64_t n_total, int64_t block_stride,
                                              int64_t n_table, MlpDesc md, uint64_t seed) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = i / block_stride, j = i % block_stride;
    float a = 0.0f;
    if (j < n_table) {
      a = 1e-4f;
    } else if (j < n_table + md.n_mlp) {
      const int64_t k = j - n_table;
      const int nl = md.n_hidden + 1;
      for (int q = 0; q < nl; ++q) {
        if (k >= md.off[q] && k < md.off[q + 1]) {
          const int fan_in = (q == 0) ? md.in_dim : md.width;
          const int fan_out = (q == nl - 1) ? 1 : md.width;
          a = sqrtf(6.0f / (float)(fan_in + fan_out));
        }
      }
    }
    const U4 u = philox4x32_10(U4{(uint32_t)j, (uint32_t)b, kInitTag, 0u}, (uint32_t)seed, (uint32_t)(seed >> 32));
    params[i] = (P)((2.0f * u24(u.x) - 1.0f) * a);
  }
}

hipError_t launch_init_params(Prec p, void* params, int n_blocks, int64_t block_stride, int64_t n_table_params,
                              const MlpDesc& md, uint64_t seed, hipStream_t s) {
  const int64_t n = (int64_t)n_blocks * block_stride;
  const int grid = (int)std::min<int64_t>((n + 255) / 256, 8192);
  if (p == Prec::F64)
    hipLaunchKernelGGL(k_init<double>, dim3(grid), dim3(256), 0, s, (double*)params, n, block_stride,
                       n_table_params, md, seed);
  else
    hipLaunchKernelGGL(k_init<float>, dim3(grid), dim3(256), 0, s, (float*)params, n, block_stride,
                       n_table_params, md, seed);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_refresh16(const float* __restrict__ params, uint16_t* __restrict__ w16,
                                                   int64_t n_total, int64_t block_stride, int64_t n_table) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = i % block_stride;
    const float f = params[i];
    uint16_t bits;
    if (j < n_table) {
      const __half h = __float2half_rn(f);
      bits = *reinterpret_cast<const uint16_t*>(&h);
    } else {
      const __bf16 h = (__bf16)f;
      bits = *reinterpret_cast<const uint16_t*>(&h);
    }
    w16[i] = bits;
  }
}

hipError_t launch_refresh16(void* params, uint16_t* work16, int n_blocks, int64_t block_stride,
                            int64_t n_table_params, int64_t n_mlp, hipStream_t s) {
  (void)n_mlp;
  const int64_t n = (int64_t)n_blocks * block_stride;
  const int grid = (int)std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_refresh16, dim3(grid), dim3(256), 0, s, (const float*)params, work16, n, block_stride,
                     n_table_params);
  return hipGetLastError();
}

// Zero fill with a kernel (graph-safe, unlike a memset node).
__global__ __launch_bounds__(256) void k_zero(uint32_t* __restrict__ p, int64_t n_words) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_words; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

hipError_t launch_zero(void* p, int64_t bytes, hipStream_t s) {
  const int64_t n = bytes / 4;
  if (n <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_zero, dim3(grid), dim3(256), 0, s, (uint32_t*)p, n);
  return hipGetLastError();
}

__global__ void k_bump_step(Counters* __restrict__ ctr) {
  if (threadIdx.x == 0) ctr->step += 1;
}

hipError_t launch_bump_step(Counters* ctr, hipStream_t s) {
  hipLaunchKernelGGL(k_bump_step, dim3(1), dim3(64), 0, s, ctr);
  return hipGetLastError();
}

// Voxel-center coordinates x = (i + 1/2) / n of owned voxels [first, first + n) of a block.
__global__ __launch_bounds__(256) void k_voxel_coords(const BlockMeta* __restrict__ meta, int block, int64_t first,
                                                      int64_t n, float* __restrict__ coords) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const BlockMeta bm = meta[block];
  const int64_t v = first + i;
  const int64_t nx = bm.dims[0], ny = bm.dims[1];
  const int64_t ix = v % nx, iy = (v / nx) % ny, iz = v / (nx * ny);
  coords[3 * i + 0] = __fdiv_rn((float)ix + 0.5f, (float)bm.dims[0]);
  coords[3 * i + 1] = __fdiv_rn((float)iy + 0.5f, (float)bm.dims[1]);
  coords[3 * i + 2] = __fdiv_rn((float)iz + 0.5f, (float)bm.dims[2]);
}

hipError_t launch_voxel_coords(const BlockMeta* meta, int block, int64_t first, int64_t n, float* coords,
                               hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_voxel_coords, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, meta, block, first, n,
                     coords);
  return hipGetLastError();
}

// Sum of squared differences (fp64) between a decoded block [nz][ny][nx] and
// its owned stored voxels.
__global__ __launch_bounds__(256) void k_mse(const BlockMeta* __restrict__ meta, int block,
                                             const float* __restrict__ dec, double* __restrict__ acc) {
  const BlockMeta bm = meta[block];
  const int64_t nx = bm.dims[0], ny = bm.dims[1], nz = bm.dims[2];
  const int g = bm.ghost;
  const int64_t NX = nx + 2 * g, NY = ny + 2 * g;
  const int64_t n = nx * ny * nz;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ix = i % nx, iy = (i / nx) % ny, iz = i / (nx * ny);
    const double d = (double)dec[i] - (double)bm.vol[((iz + g) * NY + (iy + g)) * NX + (ix + g)];
    s += d * d;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) unsafeAtomicAdd(acc, red[0] + red[1] + red[2] + red[3]);
}

hipError_t launch_mse(const BlockMeta* meta, int block, const float* decoded, double* acc, hipStream_t s) {
  hipLaunchKernelGGL(k_mse, dim3(1024), dim3(256), 0, s, meta, block, decoded, acc);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_debug_indices(LevelDesc ld, int l, int64_t n,
                                                       const float* __restrict__ coords, uint32_t* __restrict__ idx,
                                                       float* __restrict__ w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  Corners c;
  level_corners(ld, l, coords[3 * i], coords[3 * i + 1], coords[3 * i + 2], c);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    idx[8 * i + k] = c.idx[k];
    w[8 * i + k] = c.w[k];
  }
}

hipError_t launch_debug_indices(const LevelDesc& ld, int level, int64_t n, const float* coords, uint32_t* idx,
                                float* w, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_debug_indices, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ld, level, n, coords,
                     idx, w);
  return hipGetLastError();
}

}  // namespace dvnrk
