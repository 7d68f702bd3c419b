// Internal structures and launcher declarations of the DVNR HIP library.
// Shared between the host-side C ABI (dvnr_host.hip) and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dvnrk {

constexpr int kMaxLevels = 16;
constexpr int kTile = 256;        // samples per tile (work item of the training kernels)
constexpr int kLdsBytes = 163840;  // LDS of one compute unit (the most one workgroup can take)
constexpr int kMlpGrid = 256;     // workgroups of the persistent MLP kernel (one per CU)
constexpr int kLossRing = 1024;   // steps of per-block loss history kept on the device
constexpr int kMaxBins = 512;     // spatial bins per block (B^3, B <= 8) of the ordered sampler
constexpr int kBinSamples = 192;  // fewest samples per bin the automatic bin count keeps
constexpr int kSortGroup = 1024;  // samples per counting-sort group
constexpr int kPrivCells = 4096;  // cells of a bin's box in the privatized backward (LDS counters)
constexpr int kPrivVertFloats = 8192;  // box vertices x features accumulated in LDS
constexpr int kPrivCellsSmall = 512;   // the small LDS class (coarse levels, higher occupancy)
constexpr int kPrivVertFloatsSmall = 2048;

// Level table, passed by value to kernels.
struct LevelDesc {
  int32_t L, F, log2T, in_dim;
  uint32_t T_mask;
  int32_t R[kMaxLevels];
  int32_t dense[kMaxLevels];
  int32_t off[kMaxLevels];     // entry offset of the level inside a block's table
  float scale[kMaxLevels];     // (float)(R - 1)
};

struct MlpDesc {
  int32_t n_hidden, width, in_dim;
  int32_t n_mlp;               // weights per block
  int32_t off[6];              // element offset of W_1 .. W_out relative to the block's MLP start
};

// Static per-block description (device array).
struct BlockMeta {
  const float* vol;            // stored voxels (nz+2g)(ny+2g)(nx+2g), x fastest
  int32_t dims[3];
  int32_t ghost;
  int64_t param_off;           // element offset of the block in the parameter index space
};

struct BlockRange {
  float vmin, vmax;            // value range over stored voxels
  float inv_range, range;      // 1/(vmax-vmin) and vmax-vmin (1 and 1 for a constant block)
};

// Per-call sample plan (device array): samples of block b occupy
// [sample_off, sample_off + n) in the per-step sample buffers.
struct BlockPlan {
  int64_t sample_off;
  int32_t n;
  float inv_n;                 // 1/n (0 when n == 0)
  int32_t n_uni;               // samples [0, n_uni) uniform, [n_uni, n) boundary-centered
  int32_t pad;
};

// Sampling distribution of a step (boundary loss of Sec. III-C, Eq. (2)).
struct SampleDist {
  float sigma_sqrt2;           // sigma * sqrt(2): half-normal quantile scale of boundary samples
  int32_t direct_n_uni;        // n_uni of the block of a direct-mode draw
};

struct Tile {
  int32_t block;
  int32_t start;               // first sample index within the block
  int32_t count;               // samples in this tile (<= kTile)
  int32_t slot_first;          // unused by kernels; kept for alignment
};

struct Counters {
  int64_t step;                // optimizer steps taken (Adam t = step after the update)
  int32_t nonfinite;           // set when a non-finite loss was reduced
  int32_t done;                // blocks whose loss the slot reduction has written this step (reset to 0)
  uint32_t minmax[2 * 1024];   // scratch for order-preserving float min/max keys (up to 1024 blocks per pass)
};

// Element types of the training buffers
enum class Prec { F32 = 0, MIXED = 1, F64 = 2 };

// ----------------------------------------------------------------------------
// Launchers (defined in the kernel files).  All enqueue on `s`.
// ----------------------------------------------------------------------------
hipError_t launch_minmax(const BlockMeta* meta, BlockRange* range, Counters* ctr, int n_blocks,
                         const int64_t* dev_voxels, hipStream_t s);
hipError_t launch_init_params(Prec p, void* params, int n_blocks, int64_t block_stride, int64_t n_table_params,
                              const MlpDesc& md, uint64_t seed, hipStream_t s);
hipError_t launch_refresh16(void* params, uint16_t* work16, int n_blocks, int64_t block_stride,
                            int64_t n_table_params, int64_t n_mlp, hipStream_t s);
hipError_t launch_zero(void* p, int64_t bytes, hipStream_t s);
// ctr->step += 1 (one thread): the index of an optimizer update taken outside a training step.
hipError_t launch_bump_step(Counters* ctr, hipStream_t s);

// Sampler: coordinates (generated when gen != 0, else read from `coords`)
// and normalized trilinear targets.
// Direct mode when tiles == nullptr: n_tiles is then the sample count of block
// direct_block, written to coords/target [0, n).
hipError_t launch_sample(const BlockMeta* meta, const BlockRange* range, const BlockPlan* plan, const Tile* tiles,
                         int n_tiles, int direct_block, int gen, uint64_t seed, SampleDist dist, const Counters* ctr,
                         int64_t step_override, float* coords, float* target, hipStream_t s);

// Encoding forward.  Output element (sample i, level l, feature f) goes to
// out[i*ss + l*ls + f].  Tables: `table` points at element 0 of the parameter
// index space (block offsets added inside) or, when meta == nullptr, directly
// at one block's table.
hipError_t launch_encode(Prec tp, int out_kind, const LevelDesc& ld, const BlockMeta* meta, const Tile* tiles,
                         int n_tiles, int direct_block, const BlockPlan* plan, const float* coords, const void* table,
                         void* out, int64_t ss, int64_t ls, int xcd_map, hipStream_t s, int l0 = 0, int l1 = -1);
// Encoding forward of levels [l0, l1) over ordered samples (needs the ordered
// sampler): one workgroup per (block, bin, level) stages the bin's vertex box
// in LDS with coalesced rows and interpolates every sample of the bin from
// it; a bin whose box exceeds the LDS budget gathers directly.
hipError_t launch_encode_binned(Prec tp, int out_kind, const LevelDesc& ld, int l0, int l1, int B, int n_blocks,
                                const BlockMeta* meta, const BlockPlan* plan, const int32_t* bin_start,
                                const float* coords, const void* table, void* out, int64_t ss, int64_t ls,
                                hipStream_t s);
// Vertices of the LDS box budget of the binned encoding per table element size (bytes of F features).
constexpr int kEncBoxBytes = 16384;

// Encoding backward (scatter-add into gradient tables) of levels [l0, l1).
hipError_t launch_scatter(Prec gp, const LevelDesc& ld, int l0, int l1, const BlockMeta* meta, const Tile* tiles,
                          int n_tiles, int direct_block, const BlockPlan* plan, const float* coords, const void* dfeat,
                          int64_t ss, int64_t ls, void* grad, int grouped, int xcd_map, int strided, hipStream_t s);

// Destination-partitioned encoding backward of the levels [l0, l0 + nl): the
// gradient table of such a level is cut into slices of 2^sh[l] entries (at
// most kPartSliceMax fp32 accumulators); slice s of level l of a block owns
// bucket q = qbase[l] + s of that block (nq buckets per block).
constexpr int kPartSliceMax = 16384;  // accumulators of one slice (64 KB of LDS)
constexpr int kPartMaxSlices = 256;   // slices of one level
constexpr int kPartMinEntries = 1 << 12;      // smallest table that may be partitioned ("scatter_part")
constexpr int kPartAutoMinEntries = 1 << 15;  // smallest table the automatic choice partitions
constexpr int kPartSub = 16;          // sub-buckets per bucket (tile t appends to sub-bucket t % kPartSub)
constexpr int kPartSliceRecords = 16384;  // records per slice the slice sizes aim at
struct PartDesc {
  int32_t l0, nl;
  int32_t nq;                    // buckets per block
  int32_t slice_floats;          // accumulators per slice (2^sh[l] * F)
  int32_t nsub;                  // sub-buckets per bucket in use (1 .. kPartSub)
  int32_t sh[kMaxLevels];        // log2 of entries per slice
  int32_t ns[kMaxLevels];        // slices of level l (ceil(entries / 2^sh), <= kPartMaxSlices)
  int32_t qbase[kMaxLevels];     // first bucket of level l
  int32_t E[kMaxLevels];         // entries of level l
};
// Per-block bucket layout: sub-bucket g of bucket (level l, slice s) starts at
// record off[l] + (s * nsub + g) * cap[l] of the record buffer and holds at
// most cap[l] records; its cursor is cursor[(b * nq + q) * kPartSub + g].  The
// block's tiles are [tile0, tile0 + ntiles).
struct PartBlock {
  int64_t off[kMaxLevels];
  int32_t cap[kMaxLevels];
  int32_t tile0, ntiles;
};
// Pass 1 over the tiles: every (sample, corner) contribution of the levels is
// appended, as one record of 1 + F words (slice << 16 | entry within the
// slice, then F floats), to its slice's bucket (sub-bucket tile % nsub);
// a full sub-bucket's overflow is added to `grad` directly; tmax[(l - l0) *
// n_tiles + tile] receives the tile's largest |contribution|.  Pass 2: one
// workgroup per (block, level, slice) sums its bucket in LDS (64-bit fixed
// point scaled by the block's largest contribution), adds the slice into
// `grad` and clears the bucket's cursors (cursors start at zero and are left
// at zero).
// ovf[b * nq + q] is set to 1 when a record of bucket q of block b took the
// overflow atomics (the slice pass then also reads the gradient, and clears
// the flag).
hipError_t launch_part_bucket(const LevelDesc& ld, const PartDesc& pd, const BlockMeta* meta, const Tile* tiles,
                              int n_tiles, const BlockPlan* plan, const PartBlock* pb, const float* coords,
                              const float* dfeat, int64_t ls, int32_t* cursor, uint32_t* recs, float* tmax,
                              uint8_t* ovf, float* grad, hipStream_t s);
// Adam applied by the slice pass to its slice (fp32 parameters, fp16 working
// copy of the table when work16 != nullptr); the step counter is read before
// the slot reduction advances it, so the update's index is ctr->step + 1.
struct PartAdam {
  float* params;
  float* m;
  float* v;
  uint16_t* work16;
  const Counters* ctr;
  float lr0, b1, b2, eps, wd;
  float omb1, omb2;        // 1 - b1, 1 - b2, evaluated on the host and rounded once
  float ln_b1, ln_b2;      // log(b1), log(b2), evaluated on the host
  float log2_decay;        // log2 of the learning-rate decay base
  int64_t decay_start, decay_interval;
};
// adam == nullptr: the slice pass adds its sums into `grad`; otherwise it
// updates the slice's parameters and leaves their gradient at zero.
hipError_t launch_part_accum(const LevelDesc& ld, const PartDesc& pd, const BlockMeta* meta, int n_blocks,
                             int n_tiles, const BlockPlan* plan, const PartBlock* pb, int32_t* cursor,
                             const uint32_t* recs, const float* tmax, float* grad, const PartAdam* adam,
                             uint8_t* ovf, hipStream_t s);

// Spatially ordered sampler: Philox draws of every group (<= kSortGroup
// samples of one block) stored grouped by B^3 spatial bins; bin_start
// [n_blocks][kMaxBins + 1] receives each bin's first sample (within the block).
// The draws are those of step ctr->step + step_off.
hipError_t launch_sorted_sample(const Tile* groups, int n_groups, const int32_t* group_range, int n_blocks, int B,
                                uint64_t seed, SampleDist dist, const Counters* ctr, uint32_t step_off,
                                uint32_t* counts, uint32_t* totals,
                                int32_t* bin_start, const BlockMeta* meta, const BlockRange* range,
                                const BlockPlan* plan, float* coords, float* target, hipStream_t s);
// Bin-privatized encoding backward of levels [l0, l1) (needs the ordered
// sampler); size_class 0: direct atomics only, 1: small LDS boxes, 2: large.
hipError_t launch_scatter_priv(const LevelDesc& ld, int l0, int l1, int B, int n_blocks, const BlockMeta* meta,
                               const BlockPlan* plan, const int32_t* bin_start, const float* coords,
                               const float* dfeat, int64_t ls, float* grad, int xcd_map, int size_class,
                               hipStream_t s);

// MLP training pass (forward, L2 loss, backward) on MFMA; writes dfeat
// (level-major f32) and per-wave dW/loss partials into slots.  min_waves:
// waves per SIMD the 4-wave kernel's registers allow (1 or 2); wg_waves: 8
// runs the mixed-precision kernel with 8 waves per workgroup where its LDS
// fits, else 4.
hipError_t launch_mlp_train(Prec p, const MlpDesc& md, const LevelDesc& ld, const BlockMeta* meta,
                            const BlockPlan* plan, const Tile* tiles, int n_tiles, const void* feat,
                            const float* target, const void* weights_src, float* dfeat, int64_t plane,
                            float* slots, int64_t slot_stride, int grid, int loss_l1, int min_waves, int wg_waves,
                            hipStream_t s);
// MLP inference: out[i] = INR output de-normalized with the block range.
hipError_t launch_mlp_infer(Prec p, const MlpDesc& md, const LevelDesc& ld, const BlockMeta* meta,
                            const BlockRange* range, const BlockPlan* plan, const Tile* tiles, int n_tiles,
                            int direct_block, const void* feat, const void* weights_src, int64_t plane, float* out,
                            hipStream_t s);

// Sum slots into gradients and per-block losses; with bump, the last block to
// finish advances the step counter.
hipError_t launch_reduce_slots(const float* slots, int64_t slot_stride, const int32_t* slot_ranges, int n_blocks,
                               int64_t n_mlp, int64_t mlp_rel_off, int64_t block_stride, Prec gp, void* grad,
                               float* loss_ring, Counters* ctr, int bump, hipStream_t s);

// skip0 <= skip1: block-relative elements [skip0, skip1) are left alone (the
// slice pass updated them).
// Adam reads this update's index t from ctr->step (advanced before it runs).
hipError_t launch_adam(Prec p, void* params, void* grad, void* m, void* v, uint16_t* work16, int n_blocks,
                       int64_t block_stride, int64_t n_table_params, int64_t n_used, const BlockPlan* plan,
                       const Counters* ctr, double lr, double b1, double b2, double eps, double wd,
                       double decay_base, int64_t decay_start, int64_t decay_interval, hipStream_t s,
                       int64_t skip0 = 0, int64_t skip1 = 0);

// Reference-style building blocks (thread per sample) for the autograd pieces.
hipError_t launch_mlp_simple_fwd(Prec p, const MlpDesc& md, int64_t n, const void* feats, const void* w,
                                 void* out, hipStream_t s);
hipError_t launch_mlp_simple_bwd(Prec p, const MlpDesc& md, int64_t n, const void* feats, const void* w,
                                 const void* dout, void* dfeats, void* dw, hipStream_t s);

// Fused decode of one block (voxel centers, encoding through LDS-staged vertex
// boxes, MLP forward); table / wsrc point at element 0 of the parameter index
// space (fp16 / bf16 working copy for mixed precision, fp32 masters otherwise).
hipError_t launch_decode_fused(Prec p, const LevelDesc& ld, const MlpDesc& md, const BlockMeta* meta,
                               const BlockRange* range, int block, const int32_t* dims, const void* table,
                               const void* wsrc, int64_t n_table_params, void* opnd, float* out, hipStream_t s);
// Device scratch of the fused decode: the block's MLP operands in operand order.
constexpr int kDecOperandBytes = 1 << 16;

// Direct volume rendering by sample streaming (one block's unit cube).
struct RayCamera {
  float eye[3], center[3], up[3];
  float tan_h;                 // tan(vertical field of view / 2)
};
hipError_t launch_ray_init(const RayCamera& cam, int width, int height, float* dirs, float* t01, float* rgba,
                           int32_t* active, int32_t* counter, hipStream_t s);
hipError_t launch_ray_gen(const RayCamera& cam, const int32_t* active, int n_rays, int k_base, int S, float dt,
                          const float* dirs, const float* t01, float* coords, hipStream_t s);
hipError_t launch_ray_shade(const int32_t* active, int n_rays, int k_base, int S, float dt, float opacity_exp,
                            float alpha_stop, const float* t01, const float* values, const float* tf, int n_tf,
                            float tf_lo, float tf_inv_range, float* rgba, int32_t* next, int32_t* next_count,
                            hipStream_t s);

hipError_t launch_voxel_coords(const BlockMeta* meta, int block, int64_t first, int64_t n, float* coords,
                               hipStream_t s);
hipError_t launch_mse(const BlockMeta* meta, int block, const float* decoded, double* acc, hipStream_t s);
hipError_t launch_debug_indices(const LevelDesc& ld, int level, int64_t n, const float* coords, uint32_t* idx,
                                float* w, hipStream_t s);

}  // namespace dvnrk
