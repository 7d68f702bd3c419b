// Fused decode of a block to its owned voxel grid (gfx950): voxel-center
// coordinates, hash-grid encoding and the MLP forward in one kernel.
//
// A workgroup decodes a brick of 16 x 4 x 4 voxels.  For each level the brick
// touches a small box of grid vertices (its cell origins are monotonic in the
// voxel index), so the workgroup first loads that box once into LDS
// (cooperatively: consecutive lanes load consecutive x vertices, contiguous
// for dense levels, within few aligned segments for hashed levels with the x
// prime 1), then every voxel interpolates its 8 corners from LDS.  This
// replaces ~128 scattered global gathers per voxel by ~10 global loads per
// voxel plus LDS reads.  Boxes that do not fit (a level much finer than the
// voxel grid) fall back to direct gathers.  The features (bf16 or fp32) stay
// in LDS and feed the MFMA MLP forward, whose weight operands a small kernel
// arranges once per block in operand order (staged element by element from
// the weights by every brick, they took most of the decode's time); with bf16
// each lane loads its operands straight into registers.  LDS is kept small
// (the box in the table's own fp16 elements, no operand copy in LDS) for five
// workgroups per CU.  At that occupancy the kernel issues VALU instructions
// on nearly every cycle, so the per-level work is kept lean: the box bounds
// of all levels are computed once per brick, box vertices are split into
// (x, y, z) with float reciprocals instead of integer division, and each lane
// fills two box vertices per pass with both loads in flight.
#include "dvnr_device.h"

namespace dvnrk {

typedef __bf16 bf16x8d __attribute__((ext_vector_type(8)));
typedef float f32x4d __attribute__((ext_vector_type(4)));

constexpr int kBX = 16, kBY = 4, kBZ = 4;  // brick of 256 voxels
constexpr int kBoxElems = 4096;           // LDS box capacity (table elements: entries x F)

template <typename TT> __device__ __forceinline__ float tload(const TT* p) { return (float)*p; }
template <> __device__ __forceinline__ float tload<__half>(const __half* p) { return __half2float(*p); }

// MFMA forward of 16 voxels per group; features [256][32] in LDS (element FE).
template <bool BF16, int W, int NH>
struct DecMlp {
  static constexpr int MT = W / 16;
  static constexpr int KN = BF16 ? 32 : 4;
  static constexpr int VPL = BF16 ? 8 : 1;
  static constexpr int KS_IN = 32 / KN;
  static constexpr int KS_H = (W + KN - 1) / KN;
  static constexpr int N_A0 = MT * KS_IN;
  static constexpr int N_AH = (NH - 1) * MT * KS_H;
  static constexpr int N_SLOTS = N_A0 + N_AH;
  static __host__ __device__ constexpr int src_m(int s, int j) { return BF16 ? 2 * s + j / 4 : s / 4; }
  static __host__ __device__ constexpr int src_i(int s, int j) { return BF16 ? j % 4 : s % 4; }
};

// Forward operand e of the A side (slot e / 64, lane e % 64) from the block's
// weights ws (W_1 .. W_out, row-major), in the MFMA operand order the
// forward below consumes.
template <bool BF16, int W, int NH, typename WT>
__device__ __forceinline__ typename std::conditional<BF16, bf16x8d, float>::type dec_operand(const WT* __restrict__ ws,
                                                                                         const MlpDesc& md, int e) {
  using S = DecMlp<BF16, W, NH>;
  using op_t = typename std::conditional<BF16, bf16x8d, float>::type;
  const int slot = e / 64, lane = e % 64;
  const int row = lane % 16, g = lane / 16;
  const int in_dim = md.in_dim;
  op_t v;
  for (int j = 0; j < S::VPL; ++j) {
    float x = 0.0f;
    if (slot < S::N_A0) {
      const int m = slot / S::KS_IN, s = slot % S::KS_IN;
      const int f = 8 * g + s * S::VPL + j;
      if (f < in_dim) x = (float)ws[md.off[0] + (16 * m + row) * in_dim + f];
    } else {
      const int r = slot - S::N_A0;
      const int k = 1 + r / (S::MT * S::KS_H), m = (r / S::KS_H) % S::MT, s = r % S::KS_H;
      const int n = 4 * g + S::src_i(s, j) + 16 * S::src_m(s, j);
      if (S::src_m(s, j) < S::MT) x = (float)ws[md.off[k] + (16 * m + row) * W + n];
    }
    if constexpr (BF16) v[j] = (__bf16)x; else v = x;
  }
  return v;
}

// The block's forward operands in operand order (N_SLOTS * 64 entries), then
// the output layer's W floats: written once per decode, copied by every brick
// with 16-byte loads.
template <bool BF16, int W, int NH, typename WT>
__global__ __launch_bounds__(256) void k_dec_operands(MlpDesc md, const BlockMeta* __restrict__ meta, int block,
                                                      const WT* __restrict__ wsrc_all, int64_t n_table_params,
                                                      void* __restrict__ dst) {
  using S = DecMlp<BF16, W, NH>;
  using op_t = typename std::conditional<BF16, bf16x8d, float>::type;
  const WT* ws = wsrc_all + meta[block].param_off + n_table_params;
  op_t* A = reinterpret_cast<op_t*>(dst);
  float* wout = reinterpret_cast<float*>(A + S::N_SLOTS * 64);
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e < S::N_SLOTS * 64) A[e] = dec_operand<BF16, W, NH, WT>(ws, md, e);
  if (e < W) wout[e] = (float)ws[md.off[NH] + e];
}

template <bool BF16, int W, int NH, typename TT, typename WT, int F>
__global__ __launch_bounds__(256) void k_decode_fused(LevelDesc ld, MlpDesc md, const BlockMeta* __restrict__ meta,
                                                      const BlockRange* __restrict__ range, int block,
                                                      const TT* __restrict__ table_all,
                                                      const void* __restrict__ opnd, float* __restrict__ out) {
  using S = DecMlp<BF16, W, NH>;
  using op_t = typename std::conditional<BF16, bf16x8d, float>::type;
  using fe_t = typename std::conditional<BF16, __bf16, float>::type;
  constexpr int FROW = 32 + (BF16 ? 8 : 4);  // padded feature row (elements)
  // bf16: each lane keeps its forward operands in registers (loaded from the
  // arranged copy); fp32 (many more operands): staged in LDS
  constexpr bool AREG = BF16;
  __shared__ __align__(16) op_t A[AREG ? 1 : S::N_SLOTS * 64];
  __shared__ float wout[64];
  // the box in the table's own element type (fp16 halves the LDS of a box)
  __shared__ __align__(16) TT boxv[kBoxElems + 8];  // + one spare vertex slot (F <= 8)
  __shared__ __align__(16) fe_t feat[256 * FROW];
  __shared__ int lbox[kMaxLevels][6];  // per level: box origin (3), dx, dy, vertex count
  __shared__ float lrcp[kMaxLevels][2];  // 1 / dx, 1 / dy

  const BlockMeta bm = meta[block];
  const int nx = bm.dims[0], ny = bm.dims[1], nz = bm.dims[2];
  const int bxn = (nx + kBX - 1) / kBX, byn = (ny + kBY - 1) / kBY;
  // Workgroup w runs on XCD w % 8 (round-robin dispatch): each XCD takes a
  // contiguous range of bricks, so that the boxes neighbouring bricks share
  // stay in that XCD's L2 (L2 misses per decode of a 256^3 grid: 5.2 M ->
  // 1.9 M).  Any mapping is correct; this one only improves locality.
  const int nbk = bxn * byn * ((nz + kBZ - 1) / kBZ);
  const int per = (nbk + 7) / 8;
  const int brick = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (brick >= nbk) return;  // the whole workgroup leaves before any barrier
  const int x0 = (brick % bxn) * kBX, y0 = ((brick / bxn) % byn) * kBY, z0 = (brick / (bxn * byn)) * kBZ;
  const int tid = threadIdx.x;
  const int vx = x0 + tid % kBX, vy = y0 + (tid / kBX) % kBY, vz = z0 + tid / (kBX * kBY);
  const bool valid = vx < nx && vy < ny && vz < nz;
  // brick extent (clamped to the grid) for the box bounds
  const int x1 = min(x0 + kBX, nx) - 1, y1 = min(y0 + kBY, ny) - 1, z1 = min(z0 + kBZ, nz) - 1;
  auto center = [](int i, int n) { return __fdiv_rn((float)i + 0.5f, (float)n); };
  const float px = center(min(vx, nx - 1), nx), py = center(min(vy, ny - 1), ny), pz = center(min(vz, nz - 1), nz);
  const float ax0 = center(x0, nx), ax1 = center(x1, nx);
  const float ay0 = center(y0, ny), ay1 = center(y1, ny);
  const float az0 = center(z0, nz), az1 = center(z1, nz);

  // ---- forward operands of this block, arranged by k_dec_operands
  {
    const op_t* src = reinterpret_cast<const op_t*>(opnd);
    if constexpr (!AREG)
      for (int e = tid; e < S::N_SLOTS * 64; e += 256) A[e] = src[e];
    const float* wo = reinterpret_cast<const float*>(src + S::N_SLOTS * 64);
    for (int e = tid; e < W; e += 256) wout[e] = wo[e];
  }

  // ---- the brick's vertex box on every level, computed once: lane l of the
  // first wave takes level l (the bounds are the same for every voxel)
  if (tid < ld.L) {
    const int R = ld.R[tid];
    const float sc = ld.scale[tid];
    int lo[3], hi[3];
    float tt;
    grid_pos(ax0, sc, R, lo[0], tt);
    grid_pos(ax1, sc, R, hi[0], tt);
    grid_pos(ay0, sc, R, lo[1], tt);
    grid_pos(ay1, sc, R, hi[1], tt);
    grid_pos(az0, sc, R, lo[2], tt);
    grid_pos(az1, sc, R, hi[2], tt);
    const int dx = hi[0] - lo[0] + 2, dy = hi[1] - lo[1] + 2, dz = hi[2] - lo[2] + 2;
    lbox[tid][0] = lo[0];
    lbox[tid][1] = lo[1];
    lbox[tid][2] = lo[2];
    lbox[tid][3] = dx;
    lbox[tid][4] = dy;
    lbox[tid][5] = dx * dy * dz;
    lrcp[tid][0] = 1.0f / (float)dx;
    lrcp[tid][1] = 1.0f / (float)dy;
  }
  __syncthreads();

  // ---- encoding, level by level through the LDS box
  const TT* tab0 = table_all + bm.param_off;
  for (int l = 0; l < ld.L; ++l) {
    const int R = ld.R[l];
    const float sc = ld.scale[l];
    const int dense = ld.dense[l];
    const TT* tab = tab0 + (int64_t)ld.off[l] * F;
    const int lo0 = lbox[l][0], lo1 = lbox[l][1], lo2 = lbox[l][2];
    const int dx = lbox[l][3], dy = lbox[l][4], nv = lbox[l][5];
    int ix, iy, iz;
    float tx, ty, tz;
    grid_pos(px, sc, R, ix, tx);
    grid_pos(py, sc, R, iy, ty);
    grid_pos(pz, sc, R, iz, tz);
    float acc[F];
#pragma unroll
    for (int f = 0; f < F; ++f) acc[f] = 0.0f;
    if (nv * F <= kBoxElems) {
      const float rdx = lrcp[l][0], rdy = lrcp[l][1];
      // box vertex v -> table entry.  v = lx + dx (ly + dy lz) is split with
      // float reciprocals: for v < 2^22, (v + 1/2) / dx is at least 1/(2 dx)
      // away from an integer and the two roundings move it by less, so the
      // truncation is exactly floor(v / dx) (likewise for dy).
      auto entry = [&](int v) -> uint32_t {
        const int q = (int)(((float)v + 0.5f) * rdx);
        const int lx = v - q * dx;
        const int lz = (int)(((float)q + 0.5f) * rdy);
        const int ly = q - lz * dy;
        const uint32_t gx = (uint32_t)(lo0 + lx), gy = (uint32_t)(lo1 + ly), gz = (uint32_t)(lo2 + lz);
        // dense levels have R^3 <= T <= 2^24 entries: 24-bit products suffice
        if (dense) return gx + __umul24((uint32_t)R, gy + __umul24((uint32_t)R, gz));
        return (gx ^ (gy * 2654435761u) ^ (gz * 805459861u)) & ld.T_mask;
      };
      __syncthreads();  // previous level done with the box
      // two vertices per lane and pass, both loads in flight together: the
      // second index is clamped into the box and, past its end, stored to a
      // spare slot behind the box (never read), so nothing is conditional
      for (int v0 = tid; v0 < nv; v0 += 512) {
        const int v1 = v0 + 256;
        const uint32_t e0 = entry(v0), e1 = entry(min(v1, nv - 1));
        const int s1 = v1 < nv ? v1 : kBoxElems / F;
        if constexpr (sizeof(TT) * F % 4 == 0) {
          // an entry's F elements as 4-byte words (tables start 4-byte aligned)
          constexpr int NW = sizeof(TT) * F / 4;
          const uint32_t* tw = reinterpret_cast<const uint32_t*>(tab);
          uint32_t* bw = reinterpret_cast<uint32_t*>(boxv);
          uint32_t r0[NW], r1[NW];
#pragma unroll
          for (int w = 0; w < NW; ++w) {
            r0[w] = tw[(int64_t)e0 * NW + w];
            r1[w] = tw[(int64_t)e1 * NW + w];
          }
#pragma unroll
          for (int w = 0; w < NW; ++w) {
            bw[v0 * NW + w] = r0[w];
            bw[s1 * NW + w] = r1[w];
          }
        } else {
          TT r0[F], r1[F];
#pragma unroll
          for (int f = 0; f < F; ++f) {
            r0[f] = tab[(int64_t)e0 * F + f];
            r1[f] = tab[(int64_t)e1 * F + f];
          }
#pragma unroll
          for (int f = 0; f < F; ++f) {
            boxv[v0 * F + f] = r0[f];
            boxv[s1 * F + f] = r1[f];
          }
        }
      }
      __syncthreads();
      const int dxy = dx * dy;
      const int base = (ix - lo0) + __mul24(dx, (iy - lo1) + __mul24(dy, iz - lo2));
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int cx = k & 1, cy = (k >> 1) & 1, cz = (k >> 2) & 1;
        const float w = (cx ? tx : 1.0f - tx) * (cy ? ty : 1.0f - ty) * (cz ? tz : 1.0f - tz);
        const int v = base + cx + (cy ? dx : 0) + (cz ? dxy : 0);
#pragma unroll
        for (int f = 0; f < F; ++f) acc[f] += w * tload(&boxv[v * F + f]);
      }
    } else {
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const uint32_t cx = k & 1, cy = (k >> 1) & 1, cz = (k >> 2) & 1;
        const float w = (cx ? tx : 1.0f - tx) * (cy ? ty : 1.0f - ty) * (cz ? tz : 1.0f - tz);
        const uint32_t e = corner_index(dense, R, ld.T_mask, ix + cx, iy + cy, iz + cz);
#pragma unroll
        for (int f = 0; f < F; ++f) acc[f] += w * tload(tab + (int64_t)e * F + f);
      }
    }
#pragma unroll
    for (int f = 0; f < F; ++f) feat[tid * FROW + l * F + f] = (fe_t)acc[f];
  }
  for (int f = ld.L * F; f < 32; ++f) feat[tid * FROW + f] = (fe_t)0.0f;
  __syncthreads();

  // ---- MLP forward, 16 voxels per group, 4 groups per wave
  const int wave = tid / 64, lane = tid % 64;
  const int g = lane / 16, c = lane % 16;
  const BlockRange br = range[block];
  op_t areg[AREG ? S::N_SLOTS : 1];
  if constexpr (AREG) {
    const op_t* src = reinterpret_cast<const op_t*>(opnd);
#pragma unroll
    for (int e = 0; e < S::N_SLOTS; ++e) areg[e] = src[e * 64 + lane];
  }
  auto opA = [&](int e) -> op_t {
    if constexpr (AREG)
      return areg[e];
    else
      return A[e * 64 + lane];
  };
  for (int q = 0; q < 4; ++q) {
    const int vi = wave * 64 + q * 16 + c;  // voxel of the brick
    op_t xb[S::KS_IN];
#pragma unroll
    for (int s = 0; s < S::KS_IN; ++s) {
      if constexpr (BF16)
        xb[s] = *reinterpret_cast<const op_t*>(&feat[vi * FROW + 8 * g]);
      else
        xb[s] = feat[vi * FROW + 8 * g + s];
    }
    f32x4d h[S::MT];
#pragma unroll
    for (int m = 0; m < S::MT; ++m) {
      f32x4d acc = {0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < S::KS_IN; ++s) {
        if constexpr (BF16)
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(opA(m * S::KS_IN + s), xb[s], acc, 0, 0, 0);
        else
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(opA(m * S::KS_IN + s), xb[s], acc, 0, 0, 0);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) h[m][i] = fmaxf(acc[i], 0.0f);
    }
#pragma unroll
    for (int k = 1; k < NH; ++k) {
      op_t hb[S::KS_H];
#pragma unroll
      for (int s = 0; s < S::KS_H; ++s)
#pragma unroll
        for (int j = 0; j < S::VPL; ++j) {
          const int m = S::src_m(s, j), i = S::src_i(s, j);
          const float v = m < S::MT ? h[m][i] : 0.0f;
          if constexpr (BF16) hb[s][j] = (__bf16)v; else hb[s] = v;
        }
      f32x4d hn[S::MT];
#pragma unroll
      for (int m = 0; m < S::MT; ++m) {
        f32x4d acc = {0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < S::KS_H; ++s) {
          const op_t a = opA(S::N_A0 + ((k - 1) * S::MT + m) * S::KS_H + s);
          if constexpr (BF16)
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, hb[s], acc, 0, 0, 0);
          else
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, hb[s], acc, 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) hn[m][i] = fmaxf(acc[i], 0.0f);
      }
#pragma unroll
      for (int m = 0; m < S::MT; ++m) h[m] = hn[m];
    }
    float op = 0.0f;
#pragma unroll
    for (int m = 0; m < S::MT; ++m)
#pragma unroll
      for (int i = 0; i < 4; ++i) op += wout[16 * m + 4 * g + i] * h[m][i];
    op += __shfl_xor(op, 16, 64);
    op += __shfl_xor(op, 32, 64);
    const int ox = x0 + vi % kBX, oy = y0 + (vi / kBX) % kBY, oz = z0 + vi / (kBX * kBY);
    if (g == 0 && ox < nx && oy < ny && oz < nz)
      out[((int64_t)oz * ny + oy) * nx + ox] = op * br.range + br.vmin;
  }
  (void)valid;
}

template <bool BF16, int W, int NH, typename TT, typename WT>
static hipError_t run_decode(const LevelDesc& ld, const MlpDesc& md, const BlockMeta* meta, const BlockRange* range,
                             int block, const int32_t* dims, const void* table, const void* wsrc, int64_t n_table,
                             void* opnd, float* out, hipStream_t s) {
  using S = DecMlp<BF16, W, NH>;
  const int64_t bricks = (int64_t)((dims[0] + kBX - 1) / kBX) * ((dims[1] + kBY - 1) / kBY) *
                         ((dims[2] + kBZ - 1) / kBZ);
  if (bricks <= 0) return hipSuccess;
  if (bricks > 0x7fffffff - 7) return hipErrorInvalidValue;
  const int64_t grid = 8 * ((bricks + 7) / 8);  // whole rounds of the 8 XCDs
  static_assert(S::N_SLOTS * 64 * (BF16 ? 16 : 4) + 4 * W <= kDecOperandBytes, "operand buffer too small");
  hipLaunchKernelGGL((k_dec_operands<BF16, W, NH, WT>), dim3((S::N_SLOTS * 64 + 255) / 256), dim3(256), 0, s, md,
                     meta, block, (const WT*)wsrc, n_table, opnd);
  switch (ld.F) {
    case 1: hipLaunchKernelGGL((k_decode_fused<BF16, W, NH, TT, WT, 1>), dim3((unsigned)grid), dim3(256), 0, s, ld, md, meta, range, block, (const TT*)table, opnd, out); break;
    case 2: hipLaunchKernelGGL((k_decode_fused<BF16, W, NH, TT, WT, 2>), dim3((unsigned)grid), dim3(256), 0, s, ld, md, meta, range, block, (const TT*)table, opnd, out); break;
    case 4: hipLaunchKernelGGL((k_decode_fused<BF16, W, NH, TT, WT, 4>), dim3((unsigned)grid), dim3(256), 0, s, ld, md, meta, range, block, (const TT*)table, opnd, out); break;
    case 8: hipLaunchKernelGGL((k_decode_fused<BF16, W, NH, TT, WT, 8>), dim3((unsigned)grid), dim3(256), 0, s, ld, md, meta, range, block, (const TT*)table, opnd, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_decode_fused(Prec p, const LevelDesc& ld, const MlpDesc& md, const BlockMeta* meta,
                               const BlockRange* range, int block, const int32_t* dims, const void* table,
                               const void* wsrc, int64_t n_table_params, void* opnd, float* out, hipStream_t s) {
#define X(WW, NN)                                                                                                \
  if (md.width == WW && md.n_hidden == NN) {                                                                     \
    if (p == Prec::MIXED)                                                                                        \
      return run_decode<true, WW, NN, __half, __bf16>(ld, md, meta, range, block, dims, table, wsrc,             \
                                                      n_table_params, opnd, out, s);                              \
    return run_decode<false, WW, NN, float, float>(ld, md, meta, range, block, dims, table, wsrc, n_table_params, \
                                                   opnd, out, s);                                                 \
  }
  X(16, 1) X(16, 2) X(16, 3) X(32, 1) X(32, 2) X(32, 3) X(64, 1) X(64, 2) X(64, 3)
#undef X
  return hipErrorInvalidValue;
}

}  // namespace dvnrk
