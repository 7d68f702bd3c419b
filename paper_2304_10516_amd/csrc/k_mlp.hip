// Fused MLP forward + loss (L2, or the L1 of the boundary loss) + backward of
// the DVNR network on MFMA (gfx950),
// and the simple thread-per-sample MLP used by the autograd building blocks.
//
// Network (paper Sec. III): bias-free, ReLU after every hidden layer, linear
// scalar output.  Matrices W_0 [W][in] (in = L*F <= 32, zero padded to 32),
// W_1..W_{NH-1} [W][W], w_out [W].
//
// MFMA layout (16x16xK, one wave): lane l = 16 g + c holds, for output tile
// m, the accumulator rows 4g + i (i = 0..3) of column c.  Samples are the
// columns (16 per group) and neurons the rows, so a layer's output D already
// sits in the lanes of the sample it belongs to.  The next layer's B operand
// wants, in lane (g, c), K entries of sample c; since the order of a
// contraction's K index is free, we relabel K so that lane group g supplies
// exactly the neurons it already holds, and apply the same relabelling to the
// columns of the weight operand A.  Activations therefore never leave
// registers between layers.  The weight-gradient contraction runs over
// samples (K = samples), which needs the transposed layout: per-wave LDS
// staging of dZ and layer inputs as [neuron][sample].
#include "dvnr_device.h"

namespace dvnrk {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct TrBF16 {
  typedef bf16x8 op_t;
  typedef __bf16 st_t;   // LDS staging element and feature element
  static constexpr int VPL = 8;
  static constexpr int KN = 32;
  __device__ static __forceinline__ f32x4 mma(op_t a, op_t b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ void put(op_t& v, int j, float x) { v[j] = (__bf16)x; }
  __device__ static __forceinline__ float get(const op_t& v, int j) { return (float)v[j]; }
  // 8 consecutive staged elements (16-byte aligned)
  __device__ static __forceinline__ op_t ld(const st_t* p) { return *reinterpret_cast<const op_t*>(p); }
  __host__ __device__ static constexpr int src_m(int s, int j) { return 2 * s + j / 4; }
  __host__ __device__ static constexpr int src_i(int s, int j) { return j % 4; }
};

struct TrF32 {
  typedef float op_t;
  typedef float st_t;
  static constexpr int VPL = 1;
  static constexpr int KN = 4;
  __device__ static __forceinline__ f32x4 mma(op_t a, op_t b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ void put(op_t& v, int, float x) { v = x; }
  __device__ static __forceinline__ float get(const op_t& v, int) { return v; }
  __device__ static __forceinline__ op_t ld(const st_t* p) { return *p; }
  __host__ __device__ static constexpr int src_m(int s, int) { return s / 4; }
  __host__ __device__ static constexpr int src_i(int s, int) { return s % 4; }
};

template <class TR, int W, int NH>
struct MlpShape {
  static constexpr int MT = W / 16;                        // 16-row tiles of a hidden layer
  static constexpr int KS_IN = 32 / TR::KN;                // K steps of the input layer (in padded to 32)
  static constexpr int KS_H = (W + TR::KN - 1) / TR::KN;   // K steps over a hidden layer
  static constexpr int DWS = TR::KN > 16 ? TR::KN : 16;    // samples per weight-gradient pass
  static constexpr int GP = DWS / 16;                      // 16-sample groups per pass
  static constexpr int KS_DW = DWS / TR::KN;               // K steps of one weight-gradient pass
  // A-operand slots (64 lanes each): forward W_0, forward hidden, transposed hidden, transposed W_0
  static constexpr int N_A0 = MT * KS_IN;
  static constexpr int N_AH = (NH - 1) * MT * KS_H;
  static constexpr int N_A0T = 2 * KS_H;
  static constexpr int N_SLOTS = N_A0 + 2 * N_AH + N_A0T;
  // staging: per layer k, dZ_k [W] rows and input_k rows (32 for k = 0, W otherwise)
  static constexpr int RS = DWS + 16 / (int)sizeof(typename TR::st_t);  // padded row stride (elements, 16B multiple)
  static constexpr int ROWS = NH * W + 32 + (NH - 1) * W;
  static constexpr int STAGE_ELEMS = ROWS * RS;
};

// Neuron that K step s, slot j of lane group g refers to (hidden layers).
template <class TR>
__host__ __device__ constexpr int kneuron(int s, int g, int j) {
  return 4 * g + TR::src_i(s, j) + 16 * TR::src_m(s, j);
}

template <class TR, int MT, int KS>
__device__ __forceinline__ void pack_b(const f32x4 (&h)[MT], typename TR::op_t (&b)[KS]) {
#pragma unroll
  for (int s = 0; s < KS; ++s)
#pragma unroll
    for (int j = 0; j < TR::VPL; ++j) {
      const int m = TR::src_m(s, j), i = TR::src_i(s, j);
      TR::put(b[s], j, m < MT ? h[m][i] : 0.0f);
    }
}

// Load a block's weights into the LDS A-operand slots.
template <class TR, int W, int NH, typename WSRC>
__device__ void load_weights(const WSRC* __restrict__ wsrc, const MlpDesc& md, typename TR::op_t* __restrict__ A,
                             float* __restrict__ wout) {
  using S = MlpShape<TR, W, NH>;
  const int in_dim = md.in_dim;
  for (int e = threadIdx.x; e < S::N_SLOTS * 64; e += blockDim.x) {
    const int slot = e / 64, lane = e % 64;
    const int row = lane % 16, g = lane / 16;
    typename TR::op_t v;
    for (int j = 0; j < TR::VPL; ++j) {
      float x = 0.0f;
      if (slot < S::N_A0) {
        const int m = slot / S::KS_IN, s = slot % S::KS_IN;
        const int f = 8 * g + s * TR::VPL + j;
        if (f < in_dim) x = (float)wsrc[md.off[0] + (16 * m + row) * in_dim + f];
      } else if (slot < S::N_A0 + S::N_AH) {
        const int r = slot - S::N_A0;
        const int k = 1 + r / (S::MT * S::KS_H), m = (r / S::KS_H) % S::MT, s = r % S::KS_H;
        const int n = kneuron<TR>(s, g, j);
        if (TR::src_m(s, j) < S::MT) x = (float)wsrc[md.off[k] + (16 * m + row) * W + n];
      } else if (slot < S::N_A0 + 2 * S::N_AH) {
        const int r = slot - S::N_A0 - S::N_AH;
        const int k = 1 + r / (S::MT * S::KS_H), m = (r / S::KS_H) % S::MT, s = r % S::KS_H;
        const int n = kneuron<TR>(s, g, j);
        if (TR::src_m(s, j) < S::MT) x = (float)wsrc[md.off[k] + n * W + 16 * m + row];
      } else {
        const int r = slot - S::N_A0 - 2 * S::N_AH;
        const int m = r / S::KS_H, s = r % S::KS_H;
        const int n = kneuron<TR>(s, g, j);
        const int f = 16 * m + row;
        if (TR::src_m(s, j) < S::MT && f < in_dim) x = (float)wsrc[md.off[0] + n * in_dim + f];
      }
      TR::put(v, j, x);
    }
    A[e] = v;
  }
  for (int e = threadIdx.x; e < W; e += blockDim.x) wout[e] = (float)wsrc[md.off[NH] + e];
}

template <typename T> __device__ __forceinline__ float ldf(const T* p) { return (float)*p; }


// ---------------------------------------------------------------------------
// Training kernel.  Persistent: workgroup w processes tiles
// [w*n_tiles/G, (w+1)*n_tiles/G) with NW waves (4 or 8), each taking
// kTile/NW samples of a tile.  Per pass every wave stages DWS samples; after a
// barrier the NW waves split the weight-gradient output tiles and contract
// each over all NW*DWS staged samples.  With 8 waves the workgroup fills two
// waves per SIMD, whose latencies overlap, and the staging rows lose their
// padding so that it fits the LDS beside the weight operands.  At every block change the
// workgroup writes its partial dW and loss of the finished block into slot
// (w + block) and loads the new block's weights.
// ---------------------------------------------------------------------------
// MINW: waves per SIMD the 4-wave kernel's register allocation must allow
// (2 trades spills for latency hiding; option mlp_waves).  The 8-wave kernel
// runs two waves per SIMD by its workgroup size.
template <class TR, int W, int NH, typename FT, typename WSRC, int MINW, int NW>
__global__ __launch_bounds__(64 * NW, MINW) void k_mlp_train(MlpDesc md, int F, const BlockMeta* __restrict__ meta,
                                                   const BlockPlan* __restrict__ plan,
                                                   const Tile* __restrict__ tiles, int n_tiles,
                                                   const FT* __restrict__ feat, const float* __restrict__ target,
                                                   const WSRC* __restrict__ wsrc_all, float* __restrict__ dfeat,
                                                   int64_t plane, float* __restrict__ slots, int64_t slot_stride,
                                                   int64_t n_table_params, int l1) {
  using S = MlpShape<TR, W, NH>;
  using op_t = typename TR::op_t;
  using st_t = typename TR::st_t;
  constexpr int T_ALL = 2 * S::MT + (NH - 1) * S::MT * S::MT;  // 16x16 output tiles of all dW
  constexpr int U = (T_ALL + NW - 1) / NW;                      // tiles per wave
  static_assert(NW == 4 || NW == 8, "4 or 8 waves per workgroup");
  constexpr int RS = NW == 4 ? S::RS : S::DWS;  // staging row stride (elements)
  constexpr int STAGE = S::ROWS * RS;           // staging elements of one wave
  extern __shared__ __align__(16) unsigned char smem[];
  op_t* A = reinterpret_cast<op_t*>(smem);
  float* wout = reinterpret_cast<float*>(smem + sizeof(op_t) * S::N_SLOTS * 64);
  float* red = wout + 64;  // NW waves x (64 + 1) floats: output-layer gradient and loss
  st_t* stage_all = reinterpret_cast<st_t*>(smem + sizeof(op_t) * S::N_SLOTS * 64 + sizeof(float) * (64 + NW * 65 + 4));

  const int G = gridDim.x, w = blockIdx.x;
  const int t0 = (int)(((int64_t)w * n_tiles) / G), t1 = (int)(((int64_t)(w + 1) * n_tiles) / G);
  if (t0 >= t1) return;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int g = lane / 16, c = lane % 16;
  // staging rows of one wave: SZ[k] at k*W rows; SI[0] (32 rows) at NH*W; SI[k>=1] at NH*W + 32 + (k-1)*W
  auto SZ = [&](int ws, int k) { return stage_all + ws * STAGE + (k * W) * RS; };
  auto SI = [&](int ws, int k) {
    return stage_all + ws * STAGE + (k == 0 ? NH * W : NH * W + 32 + (k - 1) * W) * RS;
  };

  f32x4 dwt[U];
  float dwo[S::MT][4];
  float loss_acc = 0.0f;
  auto reset = [&]() {
#pragma unroll
    for (int u = 0; u < U; ++u) dwt[u] = f32x4{0, 0, 0, 0};
#pragma unroll
    for (int m = 0; m < S::MT; ++m)
#pragma unroll
      for (int i = 0; i < 4; ++i) dwo[m][i] = 0.0f;
    loss_acc = 0.0f;
  };
  // decode tile id -> (layer k, row tile m, column tile n)
  auto tile_kmn = [&](int t, int& k, int& m, int& n) {
    if (t < 2 * S::MT) {
      k = 0;
      m = t / 2;
      n = t % 2;
    } else {
      const int r = t - 2 * S::MT;
      k = 1 + r / (S::MT * S::MT);
      m = (r / S::MT) % S::MT;
      n = r % S::MT;
    }
  };
  auto flush = [&](int b) {
    float* out = slots + (int64_t)(w + b) * slot_stride;
    const int in_dim = md.in_dim;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = wave + NW * u;
      if (t < T_ALL) {
        int k, m, n;
        tile_kmn(t, k, m, n);
        const int in_k = k == 0 ? in_dim : W;
        const int col = 16 * n + c;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int r = 16 * m + 4 * g + i;
          if (col < in_k) out[md.off[k] + r * in_k + col] = dwt[u][i];
        }
      }
    }
    // output layer gradient and loss: reduce over the 16 sample lanes, then over waves
#pragma unroll
    for (int m = 0; m < S::MT; ++m)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float v = dwo[m][i];
        v += __shfl_xor(v, 1, 64);
        v += __shfl_xor(v, 2, 64);
        v += __shfl_xor(v, 4, 64);
        v += __shfl_xor(v, 8, 64);
        if (c == 0) red[wave * 65 + 16 * m + 4 * g + i] = v;
      }
    const float ls = wave_sum(loss_acc);
    if (lane == 0) red[wave * 65 + 64] = ls;
    __syncthreads();
    if (threadIdx.x < W) {
      const int e = threadIdx.x;
      float v = 0.0f;
#pragma unroll
      for (int ws = 0; ws < NW; ++ws) v += red[65 * ws + e];
      out[md.off[NH] + e] = v;
    }
    if (threadIdx.x == 0) {
      float v = 0.0f;
#pragma unroll
      for (int ws = 0; ws < NW; ++ws) v += red[65 * ws + 64];
      out[md.n_mlp] = v;
    }
    __syncthreads();
  };

  int cur_block = -1;
  reset();
  // element offsets (without the sample term gi * F) of the features this lane
  // reads (8 g + i) and of the feature gradients it writes (16 mm + 4 g + i);
  // -1 past the input width.  The launcher keeps L * plane * F below 2^31.
  int fo[8], dxo[2][4];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int f = 8 * g + i;
    fo[i] = f < md.in_dim ? (f / F) * (int)plane * F + f % F : -1;
  }
#pragma unroll
  for (int mm = 0; mm < 2; ++mm)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int f = 16 * mm + 4 * g + i;
      dxo[mm][i] = f < md.in_dim ? (f / F) * (int)plane * F + f % F : -1;
    }
  for (int t = t0; t < t1; ++t) {
    const Tile tl = tiles[t];
    if (tl.block != cur_block) {
      if (cur_block >= 0) {
        flush(cur_block);
        reset();
      }
      __syncthreads();  // every wave is done reading the previous weights
      cur_block = tl.block;
      const WSRC* ws = wsrc_all + meta[cur_block].param_off + n_table_params;
      load_weights<TR, W, NH>(ws, md, A, wout);
      __syncthreads();
    }
    const int64_t base = plan[tl.block].sample_off + tl.start;
    const float inv_n = plan[tl.block].inv_n;
    st_t* mySZ[NH];
    st_t* mySI[NH];
#pragma unroll
    for (int k = 0; k < NH; ++k) {
      mySZ[k] = SZ(wave, k);
      mySI[k] = SI(wave, k);
    }
    // this wave's kTile/NW samples of the tile: groups of 16, passes of DWS
    // samples; the features and target of group k+1 are loaded while group k
    // computes
    constexpr int SW = kTile / NW, NG = SW / 16;
    static_assert(NG % S::GP == 0, "a wave's groups fill whole passes");
    // raw features and target of a group, prefetched one group ahead (at the
    // last group the first one is reloaded, unused); loads are unconditional (element 0
    // stands in for a missing sample or feature) and values are converted and
    // masked only where they are used, so that no wait follows the loads
    FT xr[8];
    float yr;
    auto load_group = [&](int k, FT (&x)[8], float& y) {
      const int sl = wave * SW + k * 16 + c;
      const bool ok = sl < tl.count;
      const int gF = ok ? (int)(base + sl) * F : 0;
#pragma unroll
      for (int i = 0; i < 8; ++i) x[i] = feat[fo[i] >= 0 ? fo[i] + gF : 0];
      y = target[ok ? base + sl : 0];
    };
    load_group(0, xr, yr);
#pragma unroll 1
    for (int kg = 0; kg < NG; ++kg) {
      const int q = kg % S::GP;
      FT xn[8];
      float yn;
      load_group(kg + 1 < NG ? kg + 1 : 0, xn, yn);
      {
        const int sl = wave * SW + kg * 16 + c;  // sample within the tile
        const bool valid = sl < tl.count;
        const int64_t gi = base + sl;
        const int scol = q * 16 + c;              // staging column
        // ---- input features (B operand of layer 0) and their staging
        op_t xb[S::KS_IN];
#pragma unroll
        for (int s = 0; s < S::KS_IN; ++s)
#pragma unroll
          for (int j = 0; j < TR::VPL; ++j) {
            const int f = 8 * g + s * TR::VPL + j;
            const float x = (valid && fo[s * TR::VPL + j] >= 0) ? (float)xr[s * TR::VPL + j] : 0.0f;
            TR::put(xb[s], j, x);
            mySI[0][f * RS + scol] = (st_t)x;
          }
        // ---- forward
        f32x4 h[NH][S::MT];
#pragma unroll
        for (int m = 0; m < S::MT; ++m) {
          f32x4 acc = {0, 0, 0, 0};
#pragma unroll
          for (int s = 0; s < S::KS_IN; ++s) acc = TR::mma(A[(m * S::KS_IN + s) * 64 + lane], xb[s], acc);
#pragma unroll
          for (int i = 0; i < 4; ++i) h[0][m][i] = fmaxf(acc[i], 0.0f);
        }
#pragma unroll
        for (int k = 1; k < NH; ++k) {
          op_t hb[S::KS_H];
          pack_b<TR, S::MT, S::KS_H>(h[k - 1], hb);
#pragma unroll
          for (int m = 0; m < S::MT; ++m) {
            f32x4 acc = {0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < S::KS_H; ++s)
              acc = TR::mma(A[(S::N_A0 + ((k - 1) * S::MT + m) * S::KS_H + s) * 64 + lane], hb[s], acc);
#pragma unroll
            for (int i = 0; i < 4; ++i) h[k][m][i] = fmaxf(acc[i], 0.0f);
          }
        }
        float op = 0.0f;
#pragma unroll
        for (int m = 0; m < S::MT; ++m)
#pragma unroll
          for (int i = 0; i < 4; ++i) op += wout[16 * m + 4 * g + i] * h[NH - 1][m][i];
        op += __shfl_xor(op, 16, 64);
        op += __shfl_xor(op, 32, 64);
        // ---- loss: L2, dL/do = 2 (o - y) / n_b; L1, dL/do = sign(o - y) / n_b
        const float y = valid ? yr : 0.0f;
        const float r = op - y;
        const float sg = r > 0.0f ? inv_n : (r < 0.0f ? -inv_n : 0.0f);
        const float dO = valid ? (l1 ? sg : 2.0f * r * inv_n) : 0.0f;
        if (valid && g == 0) loss_acc += l1 ? fabsf(r) * inv_n : r * r * inv_n;
        // ---- backward through the output layer
        f32x4 dz[S::MT];
#pragma unroll
        for (int m = 0; m < S::MT; ++m)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const float hv = h[NH - 1][m][i];
            dwo[m][i] += dO * hv;
            dz[m][i] = hv > 0.0f ? wout[16 * m + 4 * g + i] * dO : 0.0f;
          }
        // ---- hidden layers: stage dZ_k and the layer input, then dZ_{k-1} = mask * W_k^T dZ_k
#pragma unroll
        for (int k = NH - 1; k >= 0; --k) {
#pragma unroll
          for (int m = 0; m < S::MT; ++m)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int n = 16 * m + 4 * g + i;
              mySZ[k][n * RS + scol] = (st_t)dz[m][i];
              if (k >= 1) mySI[k][n * RS + scol] = (st_t)h[k - 1][m][i];
            }
          if (k >= 1) {
            op_t db[S::KS_H];
            pack_b<TR, S::MT, S::KS_H>(dz, db);
            f32x4 nz[S::MT];
#pragma unroll
            for (int m = 0; m < S::MT; ++m) {
              f32x4 acc = {0, 0, 0, 0};
#pragma unroll
              for (int s = 0; s < S::KS_H; ++s)
                acc = TR::mma(A[(S::N_A0 + S::N_AH + ((k - 1) * S::MT + m) * S::KS_H + s) * 64 + lane], db[s], acc);
#pragma unroll
              for (int i = 0; i < 4; ++i) nz[m][i] = h[k - 1][m][i] > 0.0f ? acc[i] : 0.0f;
            }
#pragma unroll
            for (int m = 0; m < S::MT; ++m) dz[m] = nz[m];
          }
        }
        // ---- dX = W_0^T dZ_0 (features 16 m' + 4 g + i), level-major f32
        {
          op_t db[S::KS_H];
          pack_b<TR, S::MT, S::KS_H>(dz, db);
#pragma unroll
          for (int mm = 0; mm < 2; ++mm) {
            f32x4 acc = {0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < S::KS_H; ++s)
              acc = TR::mma(A[(S::N_A0 + 2 * S::N_AH + mm * S::KS_H + s) * 64 + lane], db[s], acc);
            if (valid) {
#pragma unroll
              for (int i = 0; i < 4; ++i)
                if (dxo[mm][i] >= 0) dfeat[dxo[mm][i] + (int)gi * F] = acc[i];
            }
          }
        }
      }  // group kg
#pragma unroll
      for (int i = 0; i < 8; ++i) xr[i] = xn[i];
      yr = yn;
      if (q != S::GP - 1) continue;
      __syncthreads();  // all waves' staging of this pass is complete
      // ---- weight gradients: this wave's output tiles over all NW waves' staged samples
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int t = wave + NW * u;
        if (t < T_ALL) {
          int k, m, n;
          tile_kmn(t, k, m, n);
#pragma unroll 1
          for (int ws = 0; ws < NW; ++ws) {
            const st_t* za = SZ(ws, k) + (16 * m + c) * RS + g * TR::VPL;
            const st_t* ib = SI(ws, k) + (16 * n + c) * RS + g * TR::VPL;
#pragma unroll
            for (int ks = 0; ks < S::KS_DW; ++ks)
              dwt[u] = TR::mma(TR::ld(za + ks * TR::KN), TR::ld(ib + ks * TR::KN), dwt[u]);
          }
        }
      }
      __syncthreads();  // staging may be overwritten by the next pass
    }  // groups
  }
  flush(cur_block);
}

// ---------------------------------------------------------------------------
// Inference kernel: forward only, output de-normalized with the block range.
// Direct tiles (tiles == nullptr): samples [0, n) of block `block0`.
// ---------------------------------------------------------------------------
template <class TR, int W, int NH, typename FT, typename WSRC>
__global__ __launch_bounds__(256) void k_mlp_infer(MlpDesc md, int F, const BlockMeta* __restrict__ meta,
                                                   const BlockRange* __restrict__ range,
                                                   const BlockPlan* __restrict__ plan,
                                                   const Tile* __restrict__ tiles, int n_tiles, int direct_block,
                                                   const FT* __restrict__ feat, const WSRC* __restrict__ wsrc_all,
                                                   int64_t plane, float* __restrict__ out, int64_t n_table_params) {
  using S = MlpShape<TR, W, NH>;
  using op_t = typename TR::op_t;
  extern __shared__ __align__(16) unsigned char smem[];
  op_t* A = reinterpret_cast<op_t*>(smem);
  float* wout = reinterpret_cast<float*>(smem + sizeof(op_t) * S::N_SLOTS * 64);
  Tile tl;
  int64_t base;
  if (tiles) {
    tl = tiles[blockIdx.x];
    base = plan[tl.block].sample_off + tl.start;
  } else {  // direct: samples [0, n_tiles) of block direct_block
    tl.block = direct_block;
    base = (int64_t)blockIdx.x * kTile;
    tl.count = (int)min((int64_t)kTile, (int64_t)n_tiles - base);
  }
  const WSRC* ws = wsrc_all + meta[tl.block].param_off + n_table_params;
  load_weights<TR, W, NH>(ws, md, A, wout);
  __syncthreads();
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int g = lane / 16, c = lane % 16;
  const BlockRange br = range[tl.block];
  int fo[S::KS_IN * TR::VPL];  // element offsets of this lane's features (-1 past the input width)
#pragma unroll
  for (int s = 0; s < S::KS_IN; ++s)
#pragma unroll
    for (int j = 0; j < TR::VPL; ++j) {
      const int f = 8 * g + s * TR::VPL + j;
      fo[s * TR::VPL + j] = f < md.in_dim ? (f / F) * (int)plane * F + f % F : -1;
    }
  for (int q = 0; q < 4; ++q) {
    const int sl = wave * 64 + q * 16 + c;
    const bool valid = sl < tl.count;
    const int64_t gi = base + sl;
    op_t xb[S::KS_IN];
#pragma unroll
    for (int s = 0; s < S::KS_IN; ++s)
#pragma unroll
      for (int j = 0; j < TR::VPL; ++j) {
        const int o = fo[s * TR::VPL + j];
        const float v = (float)feat[(valid && o >= 0) ? o + (int)gi * F : 0];  // unconditional load
        TR::put(xb[s], j, (valid && o >= 0) ? v : 0.0f);
      }
    f32x4 h[S::MT];
#pragma unroll
    for (int m = 0; m < S::MT; ++m) {
      f32x4 acc = {0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < S::KS_IN; ++s) acc = TR::mma(A[(m * S::KS_IN + s) * 64 + lane], xb[s], acc);
#pragma unroll
      for (int i = 0; i < 4; ++i) h[m][i] = fmaxf(acc[i], 0.0f);
    }
#pragma unroll
    for (int k = 1; k < NH; ++k) {
      op_t hb[S::KS_H];
      pack_b<TR, S::MT, S::KS_H>(h, hb);
      f32x4 hn[S::MT];
#pragma unroll
      for (int m = 0; m < S::MT; ++m) {
        f32x4 acc = {0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < S::KS_H; ++s)
          acc = TR::mma(A[(S::N_A0 + ((k - 1) * S::MT + m) * S::KS_H + s) * 64 + lane], hb[s], acc);
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
    if (valid && g == 0) out[gi] = op * br.range + br.vmin;
  }
}

template <class TR, int W, int NH, int NW>
static size_t train_smem() {
  using S = MlpShape<TR, W, NH>;
  return sizeof(typename TR::op_t) * S::N_SLOTS * 64 + sizeof(float) * (64 + NW * 65 + 4) +
         sizeof(typename TR::st_t) * S::ROWS * (NW == 4 ? S::RS : S::DWS) * NW;
}
template <class TR, int W, int NH>
static size_t infer_smem() {
  using S = MlpShape<TR, W, NH>;
  return sizeof(typename TR::op_t) * S::N_SLOTS * 64 + sizeof(float) * 64;
}

template <class TR, int W, int NH, typename FT, typename WSRC, int MINW = 1, int NW = 4>
static hipError_t run_train(const MlpDesc& md, int F, const BlockMeta* meta, const BlockPlan* plan, const Tile* tiles,
                            int n_tiles, const void* feat, const float* target, const void* wsrc, float* dfeat,
                            int64_t plane, float* slots, int64_t slot_stride, int grid, int64_t n_table, int l1,
                            hipStream_t s) {
  const size_t sm = train_smem<TR, W, NH, NW>();
  auto kern = k_mlp_train<TR, W, NH, FT, WSRC, MINW, NW>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * NW), sm, s, md, F, meta, plan, tiles, n_tiles, (const FT*)feat,
                     target, (const WSRC*)wsrc, dfeat, plane, slots, slot_stride, n_table, l1);
  return hipGetLastError();
}

template <class TR, int W, int NH, typename FT, typename WSRC>
static hipError_t run_infer(const MlpDesc& md, int F, const BlockMeta* meta, const BlockRange* range,
                            const BlockPlan* plan, const Tile* tiles, int n_tiles, int direct_block, const void* feat,
                            const void* wsrc, int64_t plane, float* out, int64_t n_table, hipStream_t s) {
  const size_t sm = infer_smem<TR, W, NH>();
  auto kern = k_mlp_infer<TR, W, NH, FT, WSRC>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
  if (e != hipSuccess) return e;
  const int grid = tiles ? n_tiles : (n_tiles + kTile - 1) / kTile;
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(256), sm, s, md, F, meta, range, plan, tiles, n_tiles, direct_block,
                     (const FT*)feat, (const WSRC*)wsrc, plane, out, n_table);
  return hipGetLastError();
}

#define DVNR_MLP_SHAPES(X) \
  X(16, 1) X(16, 2) X(16, 3) X(32, 1) X(32, 2) X(32, 3) X(64, 1) X(64, 2) X(64, 3)

hipError_t launch_mlp_train(Prec p, const MlpDesc& md, const LevelDesc& ld, const BlockMeta* meta,
                            const BlockPlan* plan, const Tile* tiles, int n_tiles, const void* feat,
                            const float* target, const void* weights_src, float* dfeat, int64_t plane,
                            float* slots, int64_t slot_stride, int grid, int loss_l1, int min_waves, int wg_waves,
                            hipStream_t s) {
  // weights_src points at the MLP weights of block 0 (element n_table_params);
  // the kernel adds each block's parameter offset.  Feature offsets are 32-bit.
  if ((int64_t)md.in_dim * plane >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
#define X(WW, NN)                                                                                                   \
  if (md.width == WW && md.n_hidden == NN) {                                                                        \
    if (p == Prec::MIXED && wg_waves == 8 && train_smem<TrBF16, WW, NN, 8>() <= (size_t)kLdsBytes)                  \
      return run_train<TrBF16, WW, NN, __bf16, __bf16, 1, 8>(md, ld.F, meta, plan, tiles, n_tiles, feat, target,    \
                                                              weights_src, dfeat, plane, slots, slot_stride, grid,  \
                                                              (int64_t)0, loss_l1, s);                              \
    if (p == Prec::MIXED && min_waves >= 2)                                                                         \
      return run_train<TrBF16, WW, NN, __bf16, __bf16, 2>(md, ld.F, meta, plan, tiles, n_tiles, feat, target,       \
                                                           weights_src, dfeat, plane, slots, slot_stride, grid,     \
                                                           (int64_t)0, loss_l1, s);                                 \
    if (p == Prec::MIXED)                                                                                           \
      return run_train<TrBF16, WW, NN, __bf16, __bf16>(md, ld.F, meta, plan, tiles, n_tiles, feat, target,          \
                                                        weights_src, dfeat, plane, slots, slot_stride, grid,        \
                                                        (int64_t)0, loss_l1, s);                                           \
    return run_train<TrF32, WW, NN, float, float>(md, ld.F, meta, plan, tiles, n_tiles, feat, target, weights_src, \
                                                   dfeat, plane, slots, slot_stride, grid, (int64_t)0, loss_l1, s); \
  }
  DVNR_MLP_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_mlp_infer(Prec p, const MlpDesc& md, const LevelDesc& ld, const BlockMeta* meta,
                            const BlockRange* range, const BlockPlan* plan, const Tile* tiles, int n_tiles,
                            int direct_block, const void* feat, const void* weights_src, int64_t plane, float* out,
                            hipStream_t s) {
  if ((int64_t)md.in_dim * plane >= ((int64_t)1 << 31)) return hipErrorInvalidValue;  // 32-bit feature offsets
#define X(WW, NN)                                                                                                 \
  if (md.width == WW && md.n_hidden == NN) {                                                                      \
    if (p == Prec::MIXED)                                                                                         \
      return run_infer<TrBF16, WW, NN, __bf16, __bf16>(md, ld.F, meta, range, plan, tiles, n_tiles, direct_block, \
                                                        feat, weights_src, plane, out, (int64_t)0, s);            \
    return run_infer<TrF32, WW, NN, float, float>(md, ld.F, meta, range, plan, tiles, n_tiles, direct_block, feat, \
                                                   weights_src, plane, out, (int64_t)0, s);                       \
  }
  DVNR_MLP_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Simple thread-per-sample MLP (autograd building blocks, any precision).
// feats [n][in], weights [n_mlp] (block layout), out [n].
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(128) void k_mlp_simple_fwd(MlpDesc md, int64_t n, const T* __restrict__ x,
                                                        const T* __restrict__ w, T* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T a[64], b[64];
  const int in = md.in_dim, W = md.width;
  for (int k = 0; k < in; ++k) a[k] = x[i * in + k];
  int cur = in;
  for (int layer = 0; layer < md.n_hidden; ++layer) {
    const T* M = w + md.off[layer];
    for (int r = 0; r < W; ++r) {
      T s = 0;
      for (int k = 0; k < cur; ++k) s += M[r * cur + k] * a[k];
      b[r] = s > T(0) ? s : T(0);
    }
    for (int r = 0; r < W; ++r) a[r] = b[r];
    cur = W;
  }
  T s = 0;
  for (int k = 0; k < W; ++k) s += w[md.off[md.n_hidden] + k] * a[k];
  out[i] = s;
}

template <typename T>
__global__ __launch_bounds__(64) void k_mlp_simple_bwd(MlpDesc md, int64_t n, const T* __restrict__ x,
                                                       const T* __restrict__ w, const T* __restrict__ dout,
                                                       T* __restrict__ dx, T* __restrict__ dw) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int in = md.in_dim, W = md.width, NH = md.n_hidden;
  T act[5][64];  // act[0] = input, act[k] = output of hidden layer k
  for (int k = 0; k < in; ++k) act[0][k] = x[i * in + k];
  for (int layer = 0; layer < NH; ++layer) {
    const int cur = layer == 0 ? in : W;
    const T* M = w + md.off[layer];
    for (int r = 0; r < W; ++r) {
      T s = 0;
      for (int k = 0; k < cur; ++k) s += M[r * cur + k] * act[layer][k];
      act[layer + 1][r] = s > T(0) ? s : T(0);
    }
  }
  const T d = dout[i];
  T g[64], gn[64];
  const T* wo = w + md.off[NH];
  for (int r = 0; r < W; ++r) {
    unsafeAtomicAdd(&dw[md.off[NH] + r], d * act[NH][r]);
    g[r] = act[NH][r] > T(0) ? wo[r] * d : T(0);
  }
  for (int layer = NH - 1; layer >= 0; --layer) {
    const int cur = layer == 0 ? in : W;
    const T* M = w + md.off[layer];
    for (int r = 0; r < W; ++r)
      for (int k = 0; k < cur; ++k) unsafeAtomicAdd(&dw[md.off[layer] + r * cur + k], g[r] * act[layer][k]);
    for (int k = 0; k < cur; ++k) {
      T s = 0;
      for (int r = 0; r < W; ++r) s += M[r * cur + k] * g[r];
      gn[k] = (layer == 0 || act[layer][k] > T(0)) ? s : T(0);
    }
    for (int k = 0; k < cur; ++k) g[k] = gn[k];
  }
  for (int k = 0; k < in; ++k) dx[i * in + k] = g[k];
}

hipError_t launch_mlp_simple_fwd(Prec p, const MlpDesc& md, int64_t n, const void* feats, const void* w, void* out,
                                 hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned grid = (unsigned)((n + 127) / 128);
  if (p == Prec::F64)
    hipLaunchKernelGGL(k_mlp_simple_fwd<double>, dim3(grid), dim3(128), 0, s, md, n, (const double*)feats,
                       (const double*)w, (double*)out);
  else
    hipLaunchKernelGGL(k_mlp_simple_fwd<float>, dim3(grid), dim3(128), 0, s, md, n, (const float*)feats,
                       (const float*)w, (float*)out);
  return hipGetLastError();
}

hipError_t launch_mlp_simple_bwd(Prec p, const MlpDesc& md, int64_t n, const void* feats, const void* w,
                                 const void* dout, void* dfeats, void* dw, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned grid = (unsigned)((n + 63) / 64);
  if (p == Prec::F64)
    hipLaunchKernelGGL(k_mlp_simple_bwd<double>, dim3(grid), dim3(64), 0, s, md, n, (const double*)feats,
                       (const double*)w, (const double*)dout, (double*)dfeats, (double*)dw);
  else
    hipLaunchKernelGGL(k_mlp_simple_bwd<float>, dim3(grid), dim3(64), 0, s, md, n, (const float*)feats,
                       (const float*)w, (const float*)dout, (float*)dfeats, (float*)dw);
  return hipGetLastError();
}

}  // namespace dvnrk
