// Encoding forward over spatially ordered samples with LDS-staged vertex
// boxes (gfx950).
#include "dvnr_device.h"

namespace dvnrk {

// ===========================================================================
// Encoding forward over ordered samples, one workgroup per (block, bin,
// level).  The bin's cell box follows from the bin bounds as in the backward;
// its (cells + 1)^3 vertices are loaded into LDS row by row (x fastest: a row
// is contiguous in a dense table and falls into a few aligned groups of a
// hashed one, whose x prime is 1), then every sample of the bin interpolates
// its 8 corners from LDS.  The arithmetic is that of k_encode (same weights,
// same order), so both give identical features.  Bins whose box exceeds the
// LDS budget, and samples outside the box (not expected), gather directly.
// ===========================================================================
template <typename T> __device__ __forceinline__ float enc_val(T v) { return (float)v; }
template <> __device__ __forceinline__ float enc_val<__half>(__half v) { return __half2float(v); }

template <typename TT, typename OT, int F>
__global__ __launch_bounds__(256) void k_encode_binned(LevelDesc ld, int l0, int nlev, int B, int n_blocks,
                                                       const BlockMeta* __restrict__ meta,
                                                       const BlockPlan* __restrict__ plan,
                                                       const int32_t* __restrict__ bin_start,
                                                       const float* __restrict__ coords,
                                                       const TT* __restrict__ table, OT* __restrict__ out,
                                                       int64_t ss, int64_t ls) {
  constexpr int BOXV = kEncBoxBytes / (F * (int)sizeof(TT));  // vertices held in LDS
  constexpr int VB = F * (int)sizeof(TT);                       // bytes of one vertex
  __shared__ __align__(16) TT box[BOXV * F];
  const int nbins = B * B * B;
  int unit, l;
  if (!level_major_item(blockIdx.x, l0, nlev, n_blocks * nbins, 0, unit, l)) return;
  const int bin = unit % nbins;
  const int b = unit / nbins;
  if (plan[b].n == 0) return;
  const int32_t* bs = bin_start + b * (kMaxBins + 1);
  const int s0 = bs[bin], s1 = bs[bin + 1];
  if (s0 >= s1) return;
  const int64_t base = plan[b].sample_off;
  const int R = ld.R[l];
  const float sc = ld.scale[l];
  const int dense = ld.dense[l];
  const TT* tab = table + meta[b].param_off + (int64_t)ld.off[l] * F;
  const int tid = threadIdx.x;
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
      bn[a] = ih - il + 1;  // cells per axis
    }
  }
  const int vx = bn[0] + 1, vy = bn[1] + 1, vz = bn[2] + 1;
  const int64_t NV = (int64_t)vx * vy * vz;
  const bool staged = NV <= BOXV;  // uniform over the workgroup
  if (staged) {
    for (int v = tid; v < (int)NV; v += 256) {
      const int lx = v % vx, ly = (v / vx) % vy, lz = v / (vx * vy);
      const uint32_t e = corner_index(dense, R, ld.T_mask, (uint32_t)(bo[0] + lx), (uint32_t)(bo[1] + ly),
                                      (uint32_t)(bo[2] + lz));
      if constexpr (VB == 4) {
        reinterpret_cast<uint32_t*>(box)[v] = reinterpret_cast<const uint32_t*>(tab)[e];
      } else if constexpr (VB == 8) {
        reinterpret_cast<uint2*>(box)[v] = reinterpret_cast<const uint2*>(tab)[e];
      } else {
#pragma unroll
        for (int f = 0; f < F; ++f) box[v * F + f] = tab[(int64_t)e * F + f];
      }
    }
  }
  __syncthreads();
  for (int j = s0 + tid; j < s1; j += 256) {
    const int64_t gi = base + j;
    const float x = coords[3 * gi + 0], y = coords[3 * gi + 1], z = coords[3 * gi + 2];
    int ix, iy, iz;
    float tx, ty, tz;
    grid_pos(x, sc, R, ix, tx);
    grid_pos(y, sc, R, iy, ty);
    grid_pos(z, sc, R, iz, tz);
    const int lx = ix - bo[0], ly = iy - bo[1], lz = iz - bo[2];
    const bool in_box = staged && (unsigned)lx < (unsigned)bn[0] && (unsigned)ly < (unsigned)bn[1] &&
                        (unsigned)lz < (unsigned)bn[2];
    // the tile encoding's order: per x offset cx, the four (cy, cz) corners in
    // order (0,0), (1,0), (0,1), (1,1); then (cx = 0 sum) + (cx = 1 sum)
    float acc[2][F];
#pragma unroll
    for (int f = 0; f < F; ++f) acc[0][f] = acc[1][f] = 0.0f;
    const float wx[2] = {1.0f - tx, tx};
    const float wy[2] = {1.0f - ty, ty};
    const float wz[2] = {1.0f - tz, tz};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint32_t cx = k & 1, cy = (k >> 1) & 1, cz = (k >> 2) & 1;
      const float w = wx[cx] * wy[cy] * wz[cz];
      if (in_box) {
        const TT* p = box + (int64_t)((lx + cx) + vx * ((ly + cy) + vy * (lz + cz))) * F;
#pragma unroll
        for (int f = 0; f < F; ++f) acc[cx][f] += w * enc_val(p[f]);
      } else {
        const uint32_t e = corner_index(dense, R, ld.T_mask, ix + cx, iy + cy, iz + cz);
        const TT* p = tab + (int64_t)e * F;
#pragma unroll
        for (int f = 0; f < F; ++f) acc[cx][f] += w * enc_val(p[f]);
      }
    }
    OT* o = out + gi * ss + (int64_t)l * ls;
#pragma unroll
    for (int f = 0; f < F; ++f) o[f] = (OT)(acc[0][f] + acc[1][f]);
  }
}

template <typename TT, typename OT>
static hipError_t enc_binned_dispatch(const LevelDesc& ld, int l0, int nlev, int B, int n_blocks, const BlockMeta* meta,
                                      const BlockPlan* plan, const int32_t* bin_start, const float* coords,
                                      const void* table, void* out, int64_t ss, int64_t ls, hipStream_t s) {
  const int grid = level_major_grid(nlev, n_blocks * B * B * B, 0);
  if (grid <= 0) return hipSuccess;
  const TT* t = (const TT*)table;
  OT* o = (OT*)out;
  switch (ld.F) {
    case 1: hipLaunchKernelGGL((k_encode_binned<TT, OT, 1>), dim3(grid), dim3(256), 0, s, ld, l0, nlev, B, n_blocks, meta, plan, bin_start, coords, t, o, ss, ls); break;
    case 2: hipLaunchKernelGGL((k_encode_binned<TT, OT, 2>), dim3(grid), dim3(256), 0, s, ld, l0, nlev, B, n_blocks, meta, plan, bin_start, coords, t, o, ss, ls); break;
    case 4: hipLaunchKernelGGL((k_encode_binned<TT, OT, 4>), dim3(grid), dim3(256), 0, s, ld, l0, nlev, B, n_blocks, meta, plan, bin_start, coords, t, o, ss, ls); break;
    case 8: hipLaunchKernelGGL((k_encode_binned<TT, OT, 8>), dim3(grid), dim3(256), 0, s, ld, l0, nlev, B, n_blocks, meta, plan, bin_start, coords, t, o, ss, ls); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_encode_binned(Prec tp, int out_kind, const LevelDesc& ld, int l0, int l1, int B, int n_blocks,
                                const BlockMeta* meta, const BlockPlan* plan, const int32_t* bin_start,
                                const float* coords, const void* table, void* out, int64_t ss, int64_t ls,
                                hipStream_t s) {
  const int nlev = l1 - l0;
  if (nlev <= 0) return hipSuccess;
  if (tp == Prec::MIXED && out_kind == 1)
    return enc_binned_dispatch<__half, __bf16>(ld, l0, nlev, B, n_blocks, meta, plan, bin_start, coords, table, out, ss,
                                               ls, s);
  if (tp == Prec::MIXED)
    return enc_binned_dispatch<__half, float>(ld, l0, nlev, B, n_blocks, meta, plan, bin_start, coords, table, out, ss,
                                              ls, s);
  if (tp == Prec::F32)
    return enc_binned_dispatch<float, float>(ld, l0, nlev, B, n_blocks, meta, plan, bin_start, coords, table, out, ss,
                                             ls, s);
  return hipErrorInvalidValue;
}

}  // namespace dvnrk
