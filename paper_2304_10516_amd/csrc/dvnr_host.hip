// Host side of the DVNR C ABI (include/dvnr.h): configuration checks, storage
// layout, workspace carving, per-step sample plans, the training step
// sequence and its hipGraph capture.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dvnr.h"
#include "dvnr_internal.h"

using namespace dvnrk;

namespace {

thread_local std::string g_err;

dvnr_status fail(dvnr_status code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(expr)                                                                             \
  do {                                                                                           \
    hipError_t e_ = (expr);                                                                      \
    if (e_ != hipSuccess) return fail(DVNR_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

}  // namespace

struct dvnr {
  dvnr_encoding enc{};
  dvnr_mlp mlp{};
  dvnr_optim opt{};
  Prec prec = Prec::F32;
  int nb = 0;
  std::vector<dvnr_block> blocks;
  int64_t max_batch = 0;
  uint64_t seed = 0;

  LevelDesc ld{};
  MlpDesc md{};
  int64_t n_entries = 0, n_table = 0, n_mlp = 0, stride = 0, n_params = 0;

  // workspace layout (byte offsets)
  int64_t o_meta = 0, o_range = 0, o_plan = 0, o_ctr = 0, o_vox = 0, o_tiles = 0, o_ranges = 0, o_coords = 0,
          o_target = 0, o_feat = 0, o_dfeat = 0, o_out = 0, o_slots = 0, o_ring = 0, o_mse = 0, ws_bytes = 0;
  int64_t o_decop = 0;  // fused decode: the block's MLP operands in operand order
  // second set of a step's samples (coordinates, targets, bin starts): the
  // sampler of step i + 1 fills one set while step i trains on the other
  int64_t o_coords2 = 0, o_target2 = 0, o_binstart2 = 0;
  int64_t max_tiles = 0, slot_stride = 0, n_slots = 0, feat_elem = 0;

  dvnr_buffers buf{};
  std::vector<const float*> vols;
  bool bound = false, prepared = false;

  // current training plan
  int64_t plan_total = -1;
  int n_tiles = 0, mlp_grid = 0;
  std::vector<BlockPlan> hplan;
  std::vector<Tile> htiles;
  std::vector<int32_t> hranges;

  int64_t host_step = 0;  // mirror of the device step counter
  int scatter_grouped = 0;
  int scatter_strided = 1;  // direct scatter over ordered samples: spread a tile over the block's bins
  int use_graph = 1;
  int xcd_map = 1;
  int mlp_cap = kMlpGrid;  // workgroups of the persistent MLP kernel (autotuned)
  int mlp_waves = 1;       // waves per SIMD the mixed-precision MLP kernel is compiled for (1 or 2)
  int mlp_wg_waves = 8;    // waves per workgroup of the mixed-precision MLP kernel (4 or 8)
  int decode_fused = 1;    // decode with the fused brick kernel (else encode + MLP over chunks)
  int apply_update = 1;
  // sliding-window model cache: capacity snapshots of the inference parameters
  // and block ranges in a caller buffer, oldest first from cache_head
  char* cache_buf = nullptr;
  int cache_cap = 0, cache_head = 0, cache_count = 0;
  std::vector<int64_t> cache_keys;
  // loss (Sec. III-C, Eq. (3)): 0 L2, 1 L1; fraction and spread of boundary-centered samples
  int loss_l1 = 0;
  double bnd_frac = 0.0, bnd_sigma = 0.005;
  SampleDist dist() const { return SampleDist{(float)(bnd_sigma * 1.4142135623730951), 0}; }
  // spatially ordered sampling and bin-privatized scatter of the coarse levels
  int spatial_sort = 0;
  int priv_levels = -1;  // -1: chosen per plan
  int sort_bins = 0;     // bins per axis of ordered sampling (0: at least kBinSamples samples per bin)
  int sort_B = 0, priv_L = 0, n_groups = 0;
  int priv_small = 0, priv_direct = 0;  // LDS classes: small [0, priv_small), large up to priv_direct, then direct
  int priv_classes = -1;  // launch the privatized levels by LDS class (0: one launch; -1: one block, partitioned)
  int encode_binned = 0;                // ordered samples: LDS-staged encoding of the levels whose box fits
  int enc_binned = 0;                   // levels [0, enc_binned) of the current plan
  std::vector<Tile> hgroups;
  std::vector<int32_t> hgrange;
  int64_t o_groups = 0, o_grange = 0, o_counts = 0, o_binstart = 0, o_totals = 0, max_groups = 0;
  // per-phase event timing (eager steps only): ring of kProfRing steps x 7 events
  static constexpr int kProfRing = 128;
  int profile = 0;
  std::vector<hipEvent_t> prof_ev;
  int64_t prof_recorded = 0, prof_accumulated = 0;
  // sample, encode, mlp, scatter (privatized), scatter (direct), partition pass 1, pass 2, reduce, adam
  static constexpr int kPhases = DVNR_N_PHASES;
  double prof_ms[kPhases] = {};
  hipGraphExec_t graph = nullptr;
  hipStream_t graph_stream = nullptr;
  int64_t graph_total = -1;

  unsigned char* ws() const { return (unsigned char*)buf.workspace; }
  BlockMeta* d_meta() const { return (BlockMeta*)(ws() + o_meta); }
  BlockRange* d_range() const { return (BlockRange*)(ws() + o_range); }
  BlockPlan* d_plan() const { return (BlockPlan*)(ws() + o_plan); }
  Counters* d_ctr() const { return (Counters*)(ws() + o_ctr); }
  int64_t* d_vox() const { return (int64_t*)(ws() + o_vox); }
  Tile* d_tiles() const { return (Tile*)(ws() + o_tiles); }
  int32_t* d_ranges() const { return (int32_t*)(ws() + o_ranges); }
  float* d_coords() const { return (float*)(ws() + o_coords); }
  float* d_coords(int set) const { return (float*)(ws() + (set ? o_coords2 : o_coords)); }
  float* d_target(int set) const { return (float*)(ws() + (set ? o_target2 : o_target)); }
  int32_t* d_binstart(int set) const { return (int32_t*)(ws() + (set ? o_binstart2 : o_binstart)); }
  float* d_target() const { return (float*)(ws() + o_target); }
  void* d_feat() const { return (void*)(ws() + o_feat); }
  float* d_dfeat() const { return (float*)(ws() + o_dfeat); }
  float* d_out() const { return (float*)(ws() + o_out); }
  float* d_slots() const { return (float*)(ws() + o_slots); }
  float* d_ring() const { return (float*)(ws() + o_ring); }
  double* d_mse() const { return (double*)(ws() + o_mse); }
  Tile* d_groups() const { return (Tile*)(ws() + o_groups); }
  int32_t* d_grange() const { return (int32_t*)(ws() + o_grange); }
  uint32_t* d_counts() const { return (uint32_t*)(ws() + o_counts); }
  int32_t* d_binstart() const { return (int32_t*)(ws() + o_binstart); }
  uint32_t* d_totals() const { return (uint32_t*)(ws() + o_totals); }
  size_t pelem() const { return prec == Prec::F64 ? 8 : 4; }
  size_t ielem() const { return prec == Prec::MIXED ? 2 : pelem(); }  // inference copy element

  // second stream (default priority): the direct-class levels of the
  // privatized backward run on it concurrently with the LDS-class levels,
  // forked and joined with events inside the step (also under graph capture)
  int scatter_concurrent = 0;
  int part_concurrent = 1;  // option: partitioned passes on the second stream, concurrent with the privatized levels
  int encode_concurrent = 1;  // option: binned encoding on the second stream, concurrent with the tile encoding
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_fork2 = nullptr, ev_join2 = nullptr, ev_fork3 = nullptr,
             ev_join3 = nullptr;
  // sampler look-ahead (option "sample_ahead", graph replays with ordered
  // sampling): a third stream draws step i + 1's samples while step i trains
  int sample_ahead = 2;
  hipStream_t ahead = nullptr;
  hipEvent_t ev_fork4 = nullptr, ev_join4 = nullptr;
  hipGraphExec_t graph_ahead[2] = {nullptr, nullptr};  // the step on sample set p, drawing into 1 - p
  // destination-partitioned backward of the fine levels [part_l0, L): bucket
  // layout, cursors and records in one library-owned allocation (grown on demand)
  int scatter_part = -1;  // option: first partitioned level (-1: chosen per plan; >= L: none)
  int part_cap = 0;       // option: bucket capacity override in records (0: automatic)
  int part_slice_floats = 8192;  // option: fp32 accumulators per slice
  int part_min = 0;       // first level that may be partitioned (workspace sized for [part_min, L))
  int part_l0 = 0;
  PartDesc pdesc{};
  int64_t o_pblk = 0, o_pcur = 0, o_precs = 0, o_ptmax = 0, o_povf = 0;
  uint8_t* d_povf() const { return (uint8_t*)(ws() + o_povf); }  // [nb][nq] overflow flags
  int part_adam = 1;  // option: the slice pass applies Adam to the partitioned levels
  PartBlock* d_pblk() const { return (PartBlock*)(ws() + o_pblk); }
  float* d_ptmax() const { return (float*)(ws() + o_ptmax); }  // [levels][tiles] largest contribution
  int32_t* d_pcur() const { return (int32_t*)(ws() + o_pcur); }
  uint32_t* d_precs() const { return (uint32_t*)(ws() + o_precs); }
  ~dvnr() {
    if (graph) (void)hipGraphExecDestroy(graph);
    for (hipGraphExec_t g : graph_ahead)
      if (g) (void)hipGraphExecDestroy(g);
    for (hipEvent_t e : prof_ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : {ev_fork, ev_join, ev_fork2, ev_join2, ev_fork3, ev_join3, ev_fork4, ev_join4})
      if (e) (void)hipEventDestroy(e);
    if (side) (void)hipStreamDestroy(side);
    if (ahead) (void)hipStreamDestroy(ahead);
  }
};

// Drop the captured step graphs (their kernels' arguments no longer hold).
static void drop_graphs(dvnr_t* h) {
  if (h->graph) (void)hipGraphExecDestroy(h->graph);
  h->graph = nullptr;
  for (hipGraphExec_t& g : h->graph_ahead) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
}

static int64_t owned_voxels(const dvnr_block& b) { return (int64_t)b.dims[0] * b.dims[1] * b.dims[2]; }
static int64_t stored_voxels(const dvnr_block& b) {
  return (int64_t)(b.dims[0] + 2 * b.ghost) * (b.dims[1] + 2 * b.ghost) * (b.dims[2] + 2 * b.ghost);
}

// Per-level vertex resolutions R_l = floor(R_0 * b^l + 1e-6) (see dvnr.h).
static bool build_levels(const dvnr_encoding& e, LevelDesc& ld, int64_t& n_entries, std::string& err) {
  const int L = e.n_levels;
  double b;
  if (e.per_level_scale > 0) {
    b = e.per_level_scale;
  } else if (L == 1) {
    b = 1.0;
  } else {
    if (e.finest_resolution < e.base_resolution) {
      err = "finest_resolution must be >= base_resolution";
      return false;
    }
    b = std::exp(std::log((double)e.finest_resolution / (double)e.base_resolution) / (double)(L - 1));
  }
  const int64_t T = (int64_t)1 << e.log2_table_size;
  ld.L = L;
  ld.F = e.n_features;
  ld.log2T = e.log2_table_size;
  ld.in_dim = L * e.n_features;
  ld.T_mask = (uint32_t)(T - 1);
  int64_t off = 0;
  for (int l = 0; l < kMaxLevels; ++l) {
    ld.R[l] = 2;
    ld.dense[l] = 1;
    ld.off[l] = 0;
    ld.scale[l] = 1.0f;
  }
  for (int l = 0; l < L; ++l) {
    const int64_t R = (int64_t)std::floor((double)e.base_resolution * std::pow(b, (double)l) + 1e-6);
    if (R < 2 || R > (1 << 20)) {
      err = "level resolution out of range [2, 2^20]";
      return false;
    }
    const bool dense = R * R * R <= T;
    const int64_t E = dense ? R * R * R : T;
    ld.R[l] = (int32_t)R;
    ld.dense[l] = dense ? 1 : 0;
    ld.off[l] = (int32_t)off;
    ld.scale[l] = (float)(R - 1);
    off += E;
  }
  n_entries = off;
  if (off * e.n_features >= ((int64_t)1 << 31)) {
    err = "table too large";
    return false;
  }
  return true;
}

// Table entries of level l.
static int64_t level_entries(const dvnr_t* h, int l) {
  const int64_t R = h->ld.R[l];
  return h->ld.dense[l] ? R * R * R : ((int64_t)1 << h->enc.log2_table_size);
}

// Sub-bucket capacity: 1.25x the mean load of a block's (slice, sub-bucket)
// plus 8 records.  Sub-buckets per bucket: about one per 512 records of the
// lightest bucket, a power of two in [1, kPartSub]; then a level's ns * nsub
// <= max(ns, 8 n / 512) for every block, so its records are at most
// 10 n + 9 (kPartMaxSlices + n / 64) per block (the workspace bound).
static int64_t part_bucket_cap(int64_t n, int ns, int nsub) {
  return n > 0 ? (10 * n + (int64_t)ns * nsub - 1) / ((int64_t)ns * nsub) + 8 : 0;
}
static int64_t part_level_records(int64_t max_batch, int n_blocks) {
  return 10 * max_batch + 9 * (max_batch / 64 + 1) + (int64_t)9 * kPartMaxSlices * n_blocks;
}

extern "C" {

const char* dvnr_last_error(void) { return g_err.c_str(); }

dvnr_status dvnr_create(const dvnr_encoding* enc, const dvnr_mlp* mlp, const dvnr_optim* opt,
                        dvnr_precision precision, int32_t n_blocks, const dvnr_block* blocks, int64_t max_batch,
                        uint64_t seed, dvnr_t** out) {
  try {
    if (!enc || !mlp || !opt || !blocks || !out) return fail(DVNR_E_INVALID, "null argument");
    *out = nullptr;
    const dvnr_encoding& e = *enc;
    if (e.n_levels < 1 || e.n_levels > kMaxLevels) return fail(DVNR_E_INVALID, "n_levels must be in [1, 16]");
    if (!(e.n_features == 1 || e.n_features == 2 || e.n_features == 4 || e.n_features == 8))
      return fail(DVNR_E_INVALID, "n_features must be 1, 2, 4 or 8");
    if (e.n_levels * e.n_features > 32) return fail(DVNR_E_INVALID, "n_levels * n_features must be <= 32");
    if (e.log2_table_size < 4 || e.log2_table_size > 24) return fail(DVNR_E_INVALID, "log2_table_size must be in [4, 24]");
    if (e.base_resolution < 2) return fail(DVNR_E_INVALID, "base_resolution must be >= 2");
    if (!(mlp->width == 16 || mlp->width == 32 || mlp->width == 64))
      return fail(DVNR_E_INVALID, "width must be 16, 32 or 64");
    if (mlp->n_hidden_layers < 1 || mlp->n_hidden_layers > 3)
      return fail(DVNR_E_INVALID, "n_hidden_layers must be in [1, 3]");
    if (mlp->out_dim != 1) return fail(DVNR_E_UNSUPPORTED, "out_dim must be 1");
    if (precision < DVNR_FP32 || precision > DVNR_FP64) return fail(DVNR_E_INVALID, "bad precision");
    if (n_blocks < 1 || n_blocks > 1024) return fail(DVNR_E_INVALID, "n_blocks must be in [1, 1024]");
    if (max_batch < 256 || max_batch > ((int64_t)1 << 28)) return fail(DVNR_E_INVALID, "max_batch must be in [256, 2^28]");
    if (!(opt->lr > 0) || !(opt->beta1 >= 0 && opt->beta1 < 1) || !(opt->beta2 >= 0 && opt->beta2 < 1) ||
        !(opt->eps > 0) || !(opt->weight_decay >= 0) ||
        (opt->lr_decay_interval > 0 && !(opt->lr_decay_base > 0 && opt->lr_decay_base <= 1)) ||
        opt->lr_decay_start < 0)
      return fail(DVNR_E_INVALID, "bad optimizer settings");
    for (int b = 0; b < n_blocks; ++b) {
      const dvnr_block& bl = blocks[b];
      if (bl.dims[0] < 1 || bl.dims[1] < 1 || bl.dims[2] < 1 || bl.ghost < 0 || bl.ghost > 8)
        return fail(DVNR_E_INVALID, "block dims must be >= 1 and ghost in [0, 8]");
      if (bl.dims[0] + 2 * bl.ghost < 2 || bl.dims[1] + 2 * bl.ghost < 2 || bl.dims[2] + 2 * bl.ghost < 2)
        return fail(DVNR_E_INVALID, "each stored block axis needs >= 2 voxels");
      if (stored_voxels(bl) >= ((int64_t)1 << 31)) return fail(DVNR_E_INVALID, "block too large");
    }
    dvnr* h = new dvnr();
    h->enc = e;
    h->mlp = *mlp;
    h->opt = *opt;
    h->prec = (Prec)precision;
    h->nb = n_blocks;
    h->blocks.assign(blocks, blocks + n_blocks);
    h->max_batch = max_batch;
    h->seed = seed;
    std::string err;
    if (!build_levels(e, h->ld, h->n_entries, err)) {
      delete h;
      return fail(DVNR_E_INVALID, err);
    }
    h->n_table = h->n_entries * e.n_features;
    MlpDesc& md = h->md;
    md.n_hidden = mlp->n_hidden_layers;
    md.width = mlp->width;
    md.in_dim = e.n_levels * e.n_features;
    int64_t pos = 0;
    for (int k = 0; k <= md.n_hidden; ++k) {
      md.off[k] = (int32_t)pos;
      const int fan_in = k == 0 ? md.in_dim : md.width;
      const int fan_out = k == md.n_hidden ? 1 : md.width;
      pos += (int64_t)fan_in * fan_out;
    }
    for (int k = md.n_hidden + 1; k < 6; ++k) md.off[k] = (int32_t)pos;
    md.n_mlp = (int32_t)pos;
    h->n_mlp = pos;
    h->stride = align_up(h->n_table + h->n_mlp, 64);
    h->n_params = h->stride * n_blocks;
    h->scatter_grouped = (h->prec == Prec::MIXED) ? 1 : 0;

    // workspace carving
    const int64_t A = 256;
    int64_t o = 0;
    auto take = [&](int64_t bytes) {
      const int64_t at = o;
      o = align_up(o + std::max<int64_t>(bytes, 1), A);
      return at;
    };
    h->max_tiles = max_batch / kTile + n_blocks + 1;
    h->slot_stride = align_up(h->n_mlp + 1, 64);
    h->n_slots = (int64_t)(2 * kMlpGrid + n_blocks);  // slot w + b for w < MLP workgroups (<= 2 kMlpGrid)
    h->feat_elem = h->prec == Prec::MIXED ? 2 : (h->prec == Prec::F64 ? 8 : 4);
    const int64_t in_dim = md.in_dim;
    h->o_meta = take(sizeof(BlockMeta) * n_blocks);
    h->o_range = take(sizeof(BlockRange) * n_blocks);
    h->o_plan = take(sizeof(BlockPlan) * n_blocks);
    h->o_ctr = take(sizeof(Counters));
    h->o_vox = take(sizeof(int64_t) * n_blocks);
    h->o_tiles = take(sizeof(Tile) * h->max_tiles);
    h->o_ranges = take(sizeof(int32_t) * 2 * n_blocks);
    h->o_coords = take(sizeof(float) * 3 * max_batch);
    h->o_target = take(sizeof(float) * max_batch);
    h->o_coords2 = take(sizeof(float) * 3 * max_batch);
    h->o_target2 = take(sizeof(float) * max_batch);
    h->o_feat = take(h->feat_elem * in_dim * max_batch);
    h->o_dfeat = take((h->prec == Prec::F64 ? 8 : 4) * in_dim * max_batch);
    h->o_out = take(sizeof(float) * max_batch);
    h->o_slots = take(sizeof(float) * h->n_slots * h->slot_stride);
    h->o_ring = take(sizeof(float) * kLossRing * n_blocks);
    h->o_mse = take(sizeof(double) * 8);
    h->o_decop = take(kDecOperandBytes);
    h->max_groups = max_batch / kSortGroup + n_blocks + 1;
    h->o_groups = take(sizeof(Tile) * h->max_groups);
    h->o_grange = take(sizeof(int32_t) * 2 * n_blocks);
    h->o_counts = take(sizeof(uint32_t) * kMaxBins * h->max_groups);
    h->o_binstart = take(sizeof(int32_t) * (kMaxBins + 1) * n_blocks);
    h->o_binstart2 = take(sizeof(int32_t) * (kMaxBins + 1) * n_blocks);
    h->o_totals = take(sizeof(uint32_t) * kMaxBins * n_blocks);
    // destination-partitioned backward: the suffix of levels whose tables have
    // at least kPartMinEntries entries and fit kPartMaxSlices of the largest slices
    {
      int pm = e.n_levels;
      while (pm > 0) {
        const int64_t E = level_entries(h, pm - 1);
        if (E < kPartMinEntries || E > (int64_t)kPartMaxSlices * (kPartSliceMax / e.n_features)) break;
        --pm;
      }
      h->part_min = pm;
      h->part_l0 = e.n_levels;
      const int64_t nl = e.n_levels - pm;
      h->o_pblk = take(sizeof(PartBlock) * n_blocks);
      h->o_ptmax = take(sizeof(float) * nl * h->max_tiles);
      h->o_povf = take(sizeof(uint8_t) * kPartMaxSlices * nl * n_blocks);
      h->o_pcur = take(sizeof(int32_t) * kPartSub * kPartMaxSlices * nl * n_blocks);
      h->o_precs = take(sizeof(uint32_t) * (1 + e.n_features) * nl * part_level_records(max_batch, n_blocks));
    }
    h->spatial_sort = (h->prec == Prec::MIXED) ? 1 : 0;
    h->ws_bytes = o;
    *out = h;
    return DVNR_OK;
  } catch (const std::exception& ex) {
    return fail(DVNR_E_INVALID, ex.what());
  } catch (...) {
    return fail(DVNR_E_INVALID, "unknown error");
  }
}

void dvnr_destroy(dvnr_t* h) {
  try {
    delete h;
  } catch (...) {
  }
}

dvnr_status dvnr_get_sizes(const dvnr_t* h, dvnr_sizes* out) {
  if (!h || !out) return fail(DVNR_E_INVALID, "null argument");
  out->n_levels = h->enc.n_levels;
  out->n_entries = h->n_entries;
  out->n_table_params = h->n_table;
  out->n_mlp_params = h->n_mlp;
  out->block_stride = h->stride;
  out->n_params = h->n_params;
  out->param_bytes = h->n_params * (int64_t)h->pelem();
  out->work16_bytes = h->prec == Prec::MIXED ? h->n_params * 2 : 0;
  out->workspace_bytes = h->ws_bytes;
  return DVNR_OK;
}

dvnr_status dvnr_level_info(const dvnr_t* h, int32_t* R, int32_t* dense, int64_t* off, int64_t* E) {
  if (!h) return fail(DVNR_E_INVALID, "null handle");
  const int64_t T = (int64_t)1 << h->enc.log2_table_size;
  for (int l = 0; l < h->enc.n_levels; ++l) {
    if (R) R[l] = h->ld.R[l];
    if (dense) dense[l] = h->ld.dense[l];
    if (off) off[l] = h->ld.off[l];
    if (E) E[l] = h->ld.dense[l] ? (int64_t)h->ld.R[l] * h->ld.R[l] * h->ld.R[l] : T;
  }
  return DVNR_OK;
}

dvnr_status dvnr_bind(dvnr_t* h, const dvnr_buffers* b) {
  try {
    if (!h || !b) return fail(DVNR_E_INVALID, "null argument");
    if (!b->params || !b->grads || !b->adam_m || !b->adam_v || !b->workspace || !b->volumes)
      return fail(DVNR_E_INVALID, "missing buffer");
    if (h->prec == Prec::MIXED && !b->work16) return fail(DVNR_E_INVALID, "mixed precision needs work16");
    const void* ptrs[] = {b->params, b->grads, b->adam_m, b->adam_v, b->workspace, b->work16};
    for (const void* p : ptrs)
      if (p && ((uintptr_t)p % 256)) return fail(DVNR_E_INVALID, "device buffers must be 256-byte aligned");
    for (int i = 0; i < h->nb; ++i)
      if (!b->volumes[i]) return fail(DVNR_E_INVALID, "missing block volume");
    h->buf = *b;
    h->vols.assign(b->volumes, b->volumes + h->nb);
    h->buf.volumes = h->vols.data();
    std::vector<BlockMeta> meta(h->nb);
    std::vector<int64_t> vox(h->nb);
    for (int i = 0; i < h->nb; ++i) {
      meta[i].vol = h->vols[i];
      for (int a = 0; a < 3; ++a) meta[i].dims[a] = h->blocks[i].dims[a];
      meta[i].ghost = h->blocks[i].ghost;
      meta[i].param_off = (int64_t)i * h->stride;
      vox[i] = stored_voxels(h->blocks[i]);
    }
    HIPCHK(hipMemcpy(h->d_meta(), meta.data(), sizeof(BlockMeta) * h->nb, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(h->d_vox(), vox.data(), sizeof(int64_t) * h->nb, hipMemcpyHostToDevice));
    HIPCHK(hipMemset(h->d_ctr(), 0, sizeof(Counters)));
    HIPCHK(hipMemset(h->d_slots(), 0, sizeof(float) * h->n_slots * h->slot_stride));
    HIPCHK(hipMemset(h->d_ring(), 0, sizeof(float) * kLossRing * h->nb));
    h->host_step = 0;
    h->plan_total = -1;
    drop_graphs(h);
    h->bound = true;
    h->prepared = false;
    return DVNR_OK;
  } catch (...) {
    return fail(DVNR_E_INVALID, "bind failed");
  }
}

dvnr_status dvnr_prepare(dvnr_t* h, void* stream) {
  if (!h) return fail(DVNR_E_INVALID, "null handle");
  if (!h->bound) return fail(DVNR_E_STATE, "dvnr_prepare before dvnr_bind");
  HIPCHK(launch_minmax(h->d_meta(), h->d_range(), h->d_ctr(), h->nb, h->d_vox(), (hipStream_t)stream));
  h->prepared = true;
  return DVNR_OK;
}

dvnr_status dvnr_get_ranges(dvnr_t* h, float* vmin, float* vmax, void* stream) {
  if (!h) return fail(DVNR_E_INVALID, "null handle");
  if (!h->prepared) return fail(DVNR_E_STATE, "call dvnr_prepare first");
  std::vector<BlockRange> r(h->nb);
  HIPCHK(hipMemcpyAsync(r.data(), h->d_range(), sizeof(BlockRange) * h->nb, hipMemcpyDeviceToHost, (hipStream_t)stream));
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  for (int i = 0; i < h->nb; ++i) {
    if (vmin) vmin[i] = r[i].vmin;
    if (vmax) vmax[i] = r[i].vmax;
  }
  return DVNR_OK;
}

static dvnr_status clear_optimizer(dvnr_t* h, hipStream_t s) {
  const int64_t bytes = h->n_params * (int64_t)h->pelem();
  HIPCHK(launch_zero(h->buf.adam_m, bytes, s));
  HIPCHK(launch_zero(h->buf.adam_v, bytes, s));
  HIPCHK(launch_zero(h->buf.grads, bytes, s));
  HIPCHK(launch_zero(h->d_ctr(), 16, s));  // step counter and non-finite flag
  h->host_step = 0;
  return DVNR_OK;
}

dvnr_status dvnr_init_params(dvnr_t* h, uint64_t seed, void* stream) {
  if (!h) return fail(DVNR_E_INVALID, "null handle");
  if (!h->bound) return fail(DVNR_E_STATE, "dvnr_init_params before dvnr_bind");
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(launch_init_params(h->prec, h->buf.params, h->nb, h->stride, h->n_table, h->md, seed, s));
  if (h->prec == Prec::MIXED)
    HIPCHK(launch_refresh16(h->buf.params, (uint16_t*)h->buf.work16, h->nb, h->stride, h->n_table, h->n_mlp, s));
  return clear_optimizer(h, s);
}

dvnr_status dvnr_params_updated(dvnr_t* h, void* stream) {
  if (!h) return fail(DVNR_E_INVALID, "null handle");
  if (!h->bound) return fail(DVNR_E_STATE, "dvnr_params_updated before dvnr_bind");
  hipStream_t s = (hipStream_t)stream;
  if (h->prec == Prec::MIXED)
    HIPCHK(launch_refresh16(h->buf.params, (uint16_t*)h->buf.work16, h->nb, h->stride, h->n_table, h->n_mlp, s));
  HIPCHK(launch_zero(h->buf.grads, h->n_params * (int64_t)h->pelem(), s));
  return DVNR_OK;
}

dvnr_status dvnr_reset_optimizer(dvnr_t* h, void* stream) {
  if (!h) return fail(DVNR_E_INVALID, "null handle");
  if (!h->bound) return fail(DVNR_E_STATE, "dvnr_reset_optimizer before dvnr_bind");
  return clear_optimizer(h, (hipStream_t)stream);
}

// Largest-remainder apportionment of `total` samples in units of 256 by owned voxel count.
static std::vector<int64_t> apportion(const dvnr_t* h, int64_t total) {
  std::vector<int64_t> n(h->nb, 0);
  if (h->nb == 1) {
    n[0] = total;
    return n;
  }
  const int64_t units = total / kTile;
  double sum = 0;
  for (const auto& b : h->blocks) sum += (double)owned_voxels(b);
  std::vector<double> frac(h->nb);
  int64_t used = 0;
  for (int b = 0; b < h->nb; ++b) {
    const double q = (double)units * (double)owned_voxels(h->blocks[b]) / sum;
    n[b] = (int64_t)std::floor(q);
    frac[b] = q - (double)n[b];
    used += n[b];
  }
  std::vector<int> order(h->nb);
  for (int b = 0; b < h->nb; ++b) order[b] = b;
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return frac[a] > frac[c]; });
  for (int64_t k = 0; k < units - used; ++k) n[order[k]] += 1;
  for (auto& v : n) v *= kTile;
  return n;
}

// Build and upload a training plan for the given per-block sample counts.
// Boundary samples among n: boundary_frac * n rounded half up.
static int64_t boundary_count(int64_t n, double frac) { return (int64_t)std::floor(frac * (double)n + 0.5); }

// Levels of the destination-partitioned backward and their bucket layout.
// Auto choice (mixed precision): the longest suffix of the levels with at
// least kPartAutoMinEntries entries and, unless the slice pass applies Adam
// itself, whose tables receive at least one contribution per entry per step
// on average over the sampled blocks (with Adam fused, every entry is
// updated anyway and the slice pass does it in 26 instead of 34 bytes, so
// sparse levels qualify too: 512 blocks of 128^3 with 2^21 samples, 29.4 ->
// 18.2 ms per step).  The
// workspace holds buckets from part_min (tables of at least kPartMinEntries
// entries), so "scatter_part" may ask for coarser levels too.  Only levels with at most
// kPartMaxSlices slices qualify.
static dvnr_status plan_partition(dvnr_t* h, const std::vector<int64_t>& n, hipStream_t s) {
  const int L = h->enc.n_levels, F = h->enc.n_features;
  const int sf = h->part_slice_floats;
  int sh = 0;
  while (((int64_t)2 << sh) * F <= sf) ++sh;
  const int64_t S = (int64_t)1 << sh;
  int64_t sum = 0, act = 0;
  for (auto v : n)
    if (v > 0) sum += v, ++act;
  const double avg = act ? (double)sum / (double)act : 0.0;
  int lf = L;
  if (h->scatter_part >= 0) {
    lf = std::min(h->scatter_part, L);
  } else if (h->prec == Prec::MIXED) {
    const bool fused_adam = h->part_adam != 0;
    while (lf > h->part_min && level_entries(h, lf - 1) >= kPartAutoMinEntries &&
           (fused_adam || 8.0 * avg >= (double)level_entries(h, lf - 1)))
      --lf;
  }
  lf = std::max(lf, h->part_min);
  for (int l = lf; l < L; ++l)
    if (level_entries(h, l) > kPartMaxSlices * S) lf = l + 1;
  if (act == 0) lf = L;
  h->part_l0 = lf;
  PartDesc& pd = h->pdesc;
  pd = PartDesc{};
  pd.l0 = lf;
  pd.nl = L - lf;
  pd.slice_floats = sf;
  int nq = 0;
  // slice size per level: at most the "part_slice" accumulators, halved while
  // a slice's bucket still averages kPartSliceRecords records (the dense
  // levels' small tables get many contributions per entry) and the level
  // keeps at most kPartMaxSlices slices
  for (int l = lf; l < L; ++l) {
    const int64_t E = level_entries(h, l);
    int shl = sh;
    while (shl > 0) {
      const int64_t half = (int64_t)1 << (shl - 1);
      if (8.0 * avg * (double)half / (double)E < (double)kPartSliceRecords || (E + half - 1) / half > kPartMaxSlices)
        break;
      --shl;
    }
    pd.E[l] = (int32_t)E;
    pd.sh[l] = shl;
    pd.ns[l] = (int32_t)((E + ((int64_t)1 << shl) - 1) >> shl);
    pd.qbase[l] = nq;
    nq += pd.ns[l];
  }
  pd.nq = nq;
  if (lf >= L) return DVNR_OK;
  {
    int64_t n_min = INT64_MAX;
    int ns_max = 1;
    for (auto v : n)
      if (v > 0) n_min = std::min(n_min, v);
    for (int l = lf; l < L; ++l) ns_max = std::max(ns_max, (int)pd.ns[l]);
    int g = 1;
    while (2 * g <= kPartSub && 8 * n_min >= (int64_t)2 * g * 512 * ns_max) g *= 2;
    pd.nsub = g;
  }
  std::vector<PartBlock> pbv(h->nb, PartBlock{});
  int64_t rec = 0;
  for (int b = 0; b < h->nb; ++b) {
    for (int l = lf; l < L; ++l) {
      int64_t cap = part_bucket_cap(n[b], pd.ns[l], pd.nsub);
      if (h->part_cap > 0) cap = std::min<int64_t>(cap, h->part_cap);
      pbv[b].off[l] = rec;
      pbv[b].cap[l] = (int32_t)cap;
      rec += cap * pd.ns[l] * pd.nsub;
    }
  }
  for (int t = h->n_tiles - 1; t >= 0; --t) pbv[h->htiles[t].block].tile0 = t;
  for (int t = 0; t < h->n_tiles; ++t) pbv[h->htiles[t].block].ntiles += 1;
  if (rec > (int64_t)(L - h->part_min) * part_level_records(h->max_batch, h->nb) ||
      (int64_t)nq * h->nb > (int64_t)(L - h->part_min) * kPartMaxSlices * h->nb || h->n_tiles > h->max_tiles)
    return fail(DVNR_E_INVALID, "partitioned backward exceeds its workspace");
  HIPCHK(hipMemcpyAsync(h->d_pblk(), pbv.data(), sizeof(PartBlock) * h->nb, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemsetAsync(h->d_pcur(), 0, sizeof(int32_t) * kPartSub * h->nb * nq, s));
  HIPCHK(hipMemsetAsync(h->d_povf(), 0, sizeof(uint8_t) * h->nb * nq, s));
  return DVNR_OK;
}

static dvnr_status set_plan(dvnr_t* h, const std::vector<int64_t>& n, hipStream_t s) {
  int64_t total = 0;
  for (auto v : n) total += v;
  if (total > h->max_batch) return fail(DVNR_E_INVALID, "samples per step exceed max_batch");
  h->hplan.assign(h->nb, BlockPlan{});
  h->htiles.clear();
  int64_t off = 0;
  std::vector<int> first_tile(h->nb, -1), last_tile(h->nb, -1);
  for (int b = 0; b < h->nb; ++b) {
    h->hplan[b].sample_off = off;
    h->hplan[b].n = (int32_t)n[b];
    h->hplan[b].inv_n = n[b] > 0 ? (float)(1.0 / (double)n[b]) : 0.0f;
    h->hplan[b].n_uni = (int32_t)(n[b] - boundary_count(n[b], h->bnd_frac));
    h->hplan[b].pad = 0;
    for (int64_t st = 0; st < n[b]; st += kTile) {
      if (first_tile[b] < 0) first_tile[b] = (int)h->htiles.size();
      last_tile[b] = (int)h->htiles.size();
      h->htiles.push_back(Tile{b, (int32_t)st, (int32_t)std::min<int64_t>(kTile, n[b] - st), 0});
    }
    off += n[b];
  }
  h->n_tiles = (int)h->htiles.size();
  if (h->n_tiles > h->max_tiles) return fail(DVNR_E_INVALID, "too many tiles");
  h->mlp_grid = std::max(1, std::min(h->mlp_cap, h->n_tiles));
  const int G = h->mlp_grid, T = h->n_tiles;
  auto wg_of_tile = [&](int t) {
    // the workgroup w with floor(w*T/G) <= t < floor((w+1)*T/G)
    int w = (int)(((int64_t)t * G) / std::max(T, 1));
    while (w > 0 && ((int64_t)w * T) / G > t) --w;
    while (w + 1 < G && ((int64_t)(w + 1) * T) / G <= t) ++w;
    return w;
  };
  // the MLP kernel's workgroup w writes block b's partials into slot w + b
  h->hranges.assign(2 * h->nb, 0);
  for (int b = 0; b < h->nb; ++b) {
    if (first_tile[b] < 0) continue;
    const int w0 = wg_of_tile(first_tile[b]), w1 = wg_of_tile(last_tile[b]);
    h->hranges[2 * b] = w0 + b;
    h->hranges[2 * b + 1] = w1 + b + 1;
  }
  // ordered sampling: counting-sort groups, bins per axis and privatized levels
  h->hgroups.clear();
  h->hgrange.assign(2 * h->nb, 0);
  int64_t min_n = INT64_MAX;
  for (int b = 0; b < h->nb; ++b) {
    h->hgrange[2 * b] = (int32_t)h->hgroups.size();
    for (int64_t st = 0; st < n[b]; st += kSortGroup)
      h->hgroups.push_back(Tile{b, (int32_t)st, (int32_t)std::min<int64_t>(kSortGroup, n[b] - st), 0});
    h->hgrange[2 * b + 1] = (int32_t)h->hgroups.size();
    if (n[b] > 0) min_n = std::min(min_n, n[b]);
  }
  h->n_groups = (int)h->hgroups.size();
  if (h->n_groups > h->max_groups) return fail(DVNR_E_INVALID, "too many sort groups");
  // at least kBinSamples samples per bin in the block with the fewest
  int B = 1;
  while (B < 8 && (int64_t)(B + 1) * (B + 1) * (B + 1) * kBinSamples <= min_n) ++B;
  if (h->sort_bins > 0) B = h->sort_bins;
  h->sort_B = B;
  // Ordered sampling privatizes every level by default: a (bin, level)
  // workgroup accumulates in LDS when the bin's cell box fits, and otherwise
  // issues grouped direct atomics over its bin's samples, which keeps each
  // XCD on its own levels' tables (a separate direct launch over the fine
  // levels would spread them over every XCD).
  const int pl = h->enc.n_levels;
  // LDS class of each level from a bound on its bin box: ceil((R - 1) / B) + 2
  // cells per axis (the analytic box spans at most ceil((R - 1) / B) + 1)
  // binned encoding: leading levels whose bin box ((ceil((R-1)/B) + 2)^3
  // vertices at most) fits the LDS budget and holds at most half as many
  // vertices as the bin's samples would gather directly (8 per sample)
  {
    const int64_t vbytes = (int64_t)h->enc.n_features * (h->prec == Prec::MIXED ? 2 : 4);
    const int64_t boxv = kEncBoxBytes / vbytes;
    const int64_t per_bin = min_n / ((int64_t)B * B * B);
    int le = 0;
    while (le < h->enc.n_levels) {
      const int64_t side = (h->ld.R[le] - 1 + B - 1) / B + 2;
      if (side * side * side > boxv || side * side * side > 4 * per_bin) break;
      ++le;
    }
    h->enc_binned = le;
  }
  // levels are ordered by resolution: the small class is a prefix, direct a suffix
  {
    int a = 0;
    while (a < h->enc.n_levels) {
      const int64_t side = (h->ld.R[a] - 1 + B - 1) / B + 2, F = h->enc.n_features;
      if (side * side * side > kPrivCellsSmall || (side + 1) * (side + 1) * (side + 1) * F > kPrivVertFloatsSmall)
        break;
      ++a;
    }
    h->priv_small = a;
    int c = a;
    while (c < h->enc.n_levels) {
      const int64_t side = (h->ld.R[c] - 1 + B - 1) / B + 2, F = h->enc.n_features;
      if (side * side * side > kPrivCells || (side + 1) * (side + 1) * (side + 1) * F > kPrivVertFloats) break;
      ++c;
    }
    h->priv_direct = c;
  }
  h->priv_L = h->priv_levels >= 0 ? std::min(h->priv_levels, h->enc.n_levels) : pl;
  {
    dvnr_status st = plan_partition(h, n, s);
    if (st) return st;
  }
  HIPCHK(hipMemcpyAsync(h->d_plan(), h->hplan.data(), sizeof(BlockPlan) * h->nb, hipMemcpyHostToDevice, s));
  if (h->n_tiles)
    HIPCHK(hipMemcpyAsync(h->d_tiles(), h->htiles.data(), sizeof(Tile) * h->n_tiles, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(h->d_ranges(), h->hranges.data(), sizeof(int32_t) * 2 * h->nb, hipMemcpyHostToDevice, s));
  if (h->n_groups)
    HIPCHK(hipMemcpyAsync(h->d_groups(), h->hgroups.data(), sizeof(Tile) * h->n_groups, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(h->d_grange(), h->hgrange.data(), sizeof(int32_t) * 2 * h->nb, hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  drop_graphs(h);
  return DVNR_OK;
}

// Fold the event times of recorded step `k` (ring slot k % kProfRing) into the sums.
static dvnr_status prof_accumulate_one(dvnr_t* h, int64_t k) {
  constexpr int NE = dvnr::kPhases + 1;
  hipEvent_t* ev = &h->prof_ev[(size_t)(k % dvnr::kProfRing) * NE];
  HIPCHK(hipEventSynchronize(ev[dvnr::kPhases]));
  for (int p = 0; p < dvnr::kPhases; ++p) {
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, ev[p], ev[p + 1]));
    h->prof_ms[p] += ms;
  }
  return DVNR_OK;
}

// Event marking the boundary before phase p of the step being recorded (p = kPhases: end).
static dvnr_status prof_mark(dvnr_t* h, int p, hipStream_t s) {
  constexpr int NE = dvnr::kPhases + 1;
  if (!h->profile) return DVNR_OK;
  if (p == 0) {
    if (h->prof_ev.empty()) {
      h->prof_ev.resize((size_t)dvnr::kProfRing * NE);
      for (auto& e : h->prof_ev) HIPCHK(hipEventCreate(&e));
    }
    if (h->prof_recorded - h->prof_accumulated >= dvnr::kProfRing) {
      dvnr_status st = prof_accumulate_one(h, h->prof_accumulated);
      if (st) return st;
      h->prof_accumulated += 1;
    }
  }
  HIPCHK(hipEventRecord(h->prof_ev[(size_t)(h->prof_recorded % dvnr::kProfRing) * NE + p], s));
  if (p == dvnr::kPhases) h->prof_recorded += 1;
  return DVNR_OK;
}

#define PROF(p)                          \
  do {                                   \
    dvnr_status st_ = prof_mark(h, p, s); \
    if (st_) return st_;                 \
  } while (0)

// The second stream (default priority) and its fork/join events, created on first use.
static hipError_t ensure_side(dvnr_t* h) {
  if (h->side) return hipSuccess;
  hipError_t e = hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking);
  for (hipEvent_t* ev : {&h->ev_fork, &h->ev_join, &h->ev_fork2, &h->ev_join2, &h->ev_fork3, &h->ev_join3})
    if (e == hipSuccess) e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
  return e;
}

// One training step on the current plan (coordinates generated when gen != 0).
// Ordered sampler of the step `step_off` steps after the device counter's,
// into sample set `set`.
static dvnr_status enqueue_sorted_sample(dvnr_t* h, int set, uint32_t step_off, hipStream_t s) {
  HIPCHK(launch_sorted_sample(h->d_groups(), h->n_groups, h->d_grange(), h->nb, h->sort_B, h->seed, h->dist(),
                              h->d_ctr(), step_off, h->d_counts(), h->d_totals(), h->d_binstart(set), h->d_meta(),
                              h->d_range(), h->d_plan(), h->d_coords(set), h->d_target(set), s));
  return DVNR_OK;
}

// One training step on the current plan.  gen != 0: the step's samples are
// generated (Philox draws at the device step counter), else the coordinates
// are given in sample set 0.  set: the sample set the step trains on.
// ahead (ordered sampling only): this step's samples are already in `set`,
// and a third stream draws the next step's into 1 - set while this step
// trains (joined before the slot reduction advances the counter).
static dvnr_status enqueue_step(dvnr_t* h, int gen, hipStream_t s, int set = 0, bool ahead = false) {
  const bool mixed = h->prec == Prec::MIXED;
  const int64_t F = h->enc.n_features;
  const bool sorted = gen && h->spatial_sort && h->n_groups > 0;
  if (ahead && !sorted) return fail(DVNR_E_STATE, "sampler look-ahead needs ordered sampling");
  PROF(0);
  // the next step's sampler on the third stream, forked at the point of this
  // step that option sample_ahead names (1: its start, 2: after the encoding,
  // 3: after the MLP)
  auto fork_ahead = [&](int at) -> dvnr_status {
    if (!ahead || h->sample_ahead != at) return DVNR_OK;
    if (!h->ahead) {
      HIPCHK(hipStreamCreateWithFlags(&h->ahead, hipStreamNonBlocking));
      HIPCHK(hipEventCreateWithFlags(&h->ev_fork4, hipEventDisableTiming));
      HIPCHK(hipEventCreateWithFlags(&h->ev_join4, hipEventDisableTiming));
    }
    HIPCHK(hipEventRecord(h->ev_fork4, s));
    HIPCHK(hipStreamWaitEvent(h->ahead, h->ev_fork4, 0));
    dvnr_status st = enqueue_sorted_sample(h, 1 - set, 1, h->ahead);
    if (st) return st;
    HIPCHK(hipEventRecord(h->ev_join4, h->ahead));
    return DVNR_OK;
  };
  if (ahead) {
    dvnr_status st = fork_ahead(1);
    if (st) return st;
  } else if (sorted) {
    dvnr_status st = enqueue_sorted_sample(h, set, 0, s);
    if (st) return st;
  } else {
    HIPCHK(launch_sample(h->d_meta(), h->d_range(), h->d_plan(), h->d_tiles(), h->n_tiles, 0, gen, h->seed,
                         h->dist(), h->d_ctr(), -1, h->d_coords(set), h->d_target(set), s));
  }
  PROF(1);
  const void* table = mixed ? h->buf.work16 : h->buf.params;
  // ordered samples: levels [0, enc_binned) interpolate from LDS-staged bin boxes
  const int le = sorted && h->encode_binned ? h->enc_binned : 0;
  // encode_concurrent: the binned (LDS-bound) levels on the second stream while
  // the tile encoding gathers the others
  const bool econc = h->encode_concurrent && le > 0 && le < h->enc.n_levels;
  if (econc) {
    HIPCHK(ensure_side(h));
    HIPCHK(hipEventRecord(h->ev_fork3, s));
    HIPCHK(hipStreamWaitEvent(h->side, h->ev_fork3, 0));
  }
  if (le > 0)
    HIPCHK(launch_encode_binned(h->prec, mixed ? 1 : 0, h->ld, 0, le, h->sort_B, h->nb, h->d_meta(), h->d_plan(),
                                h->d_binstart(set), h->d_coords(set), table, h->d_feat(), F, h->max_batch * F,
                                econc ? h->side : s));
  if (econc) HIPCHK(hipEventRecord(h->ev_join3, h->side));
  HIPCHK(launch_encode(h->prec, mixed ? 1 : 0, h->ld, h->d_meta(), h->d_tiles(), h->n_tiles, 0, h->d_plan(),
                       h->d_coords(set), table, h->d_feat(), F, h->max_batch * F, h->xcd_map, s, le,
                       h->enc.n_levels));
  if (econc) HIPCHK(hipStreamWaitEvent(s, h->ev_join3, 0));
  PROF(2);
  {
    dvnr_status st = fork_ahead(2);
    if (st) return st;
  }
  const void* wsrc = mixed ? (const void*)((const uint16_t*)h->buf.work16 + h->n_table)
                           : (const void*)((const float*)h->buf.params + h->n_table);
  HIPCHK(launch_mlp_train(h->prec, h->md, h->ld, h->d_meta(), h->d_plan(), h->d_tiles(), h->n_tiles, h->d_feat(),
                          h->d_target(set), wsrc, h->d_dfeat(), h->max_batch, h->d_slots(), h->slot_stride, h->mlp_grid,
                          h->loss_l1, h->mlp_waves, h->mlp_wg_waves, s));
  {
    dvnr_status st = fork_ahead(3);
    if (st) return st;
  }
  PROF(3);
  const int lf = h->part_l0;  // levels [lf, L): destination-partitioned
  const int lp = std::min(sorted ? h->priv_L : 0, lf);
  // part_concurrent: the partitioned passes (HBM streams) run on the second
  // stream while the privatized levels (LDS and latency bound) run on `s`
  const bool pconc = h->part_concurrent && lf < h->enc.n_levels && lp > 0;
  // part_adam: the slice pass applies Adam to the partitioned levels itself
  // (their gradient never goes through memory); it reads the step counter
  // before the slot reduction advances it
  const bool padam = h->part_adam && h->apply_update && lf < h->enc.n_levels;
  PartAdam pa{};
  if (padam) {
    pa.params = (float*)h->buf.params;
    pa.m = (float*)h->buf.adam_m;
    pa.v = (float*)h->buf.adam_v;
    pa.work16 = mixed ? (uint16_t*)h->buf.work16 : nullptr;
    pa.ctr = h->d_ctr();
    pa.lr0 = (float)h->opt.lr;
    pa.b1 = (float)h->opt.beta1;
    pa.b2 = (float)h->opt.beta2;
    pa.eps = (float)h->opt.eps;
    pa.wd = (float)h->opt.weight_decay;
    pa.omb1 = (float)(1.0 - h->opt.beta1);
    pa.omb2 = (float)(1.0 - h->opt.beta2);
    pa.ln_b1 = (float)std::log(h->opt.beta1);
    pa.ln_b2 = (float)std::log(h->opt.beta2);
    pa.log2_decay = h->opt.lr_decay_interval > 0 ? (float)std::log2(h->opt.lr_decay_base) : 0.0f;
    pa.decay_start = h->opt.lr_decay_start;
    pa.decay_interval = h->opt.lr_decay_interval > 0 ? h->opt.lr_decay_interval : 0;
  }
  auto part_bucket = [&](hipStream_t st) {
    return launch_part_bucket(h->ld, h->pdesc, h->d_meta(), h->d_tiles(), h->n_tiles, h->d_plan(), h->d_pblk(),
                              h->d_coords(set), h->d_dfeat(), h->max_batch * F, h->d_pcur(), h->d_precs(),
                              h->d_ptmax(), h->d_povf(), (float*)h->buf.grads, st);
  };
  auto part_accum = [&](hipStream_t st) {
    return launch_part_accum(h->ld, h->pdesc, h->d_meta(), h->nb, h->n_tiles, h->d_plan(), h->d_pblk(),
                             h->d_pcur(), h->d_precs(), h->d_ptmax(), (float*)h->buf.grads, padam ? &pa : nullptr,
                             h->d_povf(), st);
  };
  if (pconc) {
    HIPCHK(ensure_side(h));
    HIPCHK(hipEventRecord(h->ev_fork2, s));
    HIPCHK(hipStreamWaitEvent(h->side, h->ev_fork2, 0));
    HIPCHK(part_bucket(h->side));
    HIPCHK(part_accum(h->side));
    HIPCHK(hipEventRecord(h->ev_join2, h->side));
  }
  // privatized levels [0, lp) in up to three launches by LDS class: small boxes
  // (coarse levels, high occupancy), large boxes, and levels whose boxes never
  // fit (direct atomics over each bin's samples, no LDS).  Plain workgroup
  // mapping: each launch spreads its levels over every XCD (balance measured
  // to matter more than per-XCD table locality here).
  {
    // priv_classes 0: one launch (large class) for all privatized levels, so that
    // the LDS-bound coarse and the atomic-bound fine levels overlap on the chip;
    // -1 (default): by class when the partitioned backward has taken the fine
    // levels of a single block (only coarse ones are left, and the small-box
    // class runs at higher occupancy beside the partitioned passes; with many
    // blocks one launch measured faster); scatter_concurrent: the direct-class
    // levels on the second stream instead
    const bool conc = h->scatter_concurrent != 0;
    const bool classes = h->priv_classes > 0 || (h->priv_classes < 0 && lf < h->enc.n_levels && h->nb == 1);
    const int a = classes ? std::min(h->priv_small, lp) : 0;
    const int c = classes || conc ? std::min(std::max(h->priv_direct, a), lp) : lp;
    if (conc && c < lp) {
      HIPCHK(ensure_side(h));
      HIPCHK(hipEventRecord(h->ev_fork, s));
      HIPCHK(hipStreamWaitEvent(h->side, h->ev_fork, 0));
      HIPCHK(launch_scatter_priv(h->ld, c, lp, h->sort_B, h->nb, h->d_meta(), h->d_plan(), h->d_binstart(set),
                                 h->d_coords(set), h->d_dfeat(), h->max_batch * F, (float*)h->buf.grads, 0, 0,
                                 h->side));
      HIPCHK(hipEventRecord(h->ev_join, h->side));
    }
    const int cls[3][3] = {{0, a, 1}, {a, c, 2}, {c, conc ? c : lp, 0}};
    for (const auto& r : cls)
      if (r[1] > r[0])
        HIPCHK(launch_scatter_priv(h->ld, r[0], r[1], h->sort_B, h->nb, h->d_meta(), h->d_plan(), h->d_binstart(set),
                                   h->d_coords(set), h->d_dfeat(), h->max_batch * F, (float*)h->buf.grads, 0, r[2],
                                   s));
    if (conc && c < lp) HIPCHK(hipStreamWaitEvent(s, h->ev_join, 0));
  }
  PROF(4);
  HIPCHK(launch_scatter(Prec::F32, h->ld, lp, lf, h->d_meta(), h->d_tiles(), h->n_tiles, 0, h->d_plan(),
                        h->d_coords(set), h->d_dfeat(), F, h->max_batch * F, h->buf.grads, h->scatter_grouped,
                        h->xcd_map, sorted ? h->scatter_strided : 0, s));
  PROF(5);
  if (lf < h->enc.n_levels && !pconc) HIPCHK(part_bucket(s));
  PROF(6);
  if (lf < h->enc.n_levels && !pconc) HIPCHK(part_accum(s));
  PROF(7);
  // the weight-gradient reduction needs only the MLP's slots and writes the
  // weights' gradient: with the concurrent passes it runs before the join,
  // unless the slice pass still has to read the step counter it advances
  if (pconc && padam) HIPCHK(hipStreamWaitEvent(s, h->ev_join2, 0));
  if (ahead) HIPCHK(hipStreamWaitEvent(s, h->ev_join4, 0));  // it read the counter before the advance
  HIPCHK(launch_reduce_slots(h->d_slots(), h->slot_stride, h->d_ranges(), h->nb, h->n_mlp, h->n_table, h->stride,
                             Prec::F32, h->buf.grads, h->d_ring(), h->d_ctr(), 1, s));
  if (pconc && !padam) HIPCHK(hipStreamWaitEvent(s, h->ev_join2, 0));
  PROF(8);
  if (!h->apply_update) {
    PROF(9);
    return DVNR_OK;
  }
  // Adam over the parameters the slice pass did not update: the partitioned
  // levels' tables are the block-relative elements [off_lf F, n_table)
  const int64_t skip0 = padam ? (int64_t)h->ld.off[lf] * F : 0, skip1 = padam ? h->n_table : 0;
  HIPCHK(launch_adam(h->prec, h->buf.params, h->buf.grads, h->buf.adam_m, h->buf.adam_v,
                     mixed ? (uint16_t*)h->buf.work16 : nullptr, h->nb, h->stride, h->n_table, h->n_table + h->n_mlp,
                     h->d_plan(), h->d_ctr(), h->opt.lr, h->opt.beta1, h->opt.beta2, h->opt.eps,
                     h->opt.weight_decay, h->opt.lr_decay_interval > 0 ? h->opt.lr_decay_base : 1.0,
                     h->opt.lr_decay_start, h->opt.lr_decay_interval > 0 ? h->opt.lr_decay_interval : 0, s, skip0,
                     skip1));
  PROF(9);
  return DVNR_OK;
}

// Copy ring rows of steps [s0, s0 + n) into out [n][nb].
static dvnr_status copy_losses(dvnr_t* h, int64_t s0, int64_t n, float* out, hipStream_t s) {
  int64_t done = 0;
  while (done < n) {
    const int64_t row = (s0 + done) % kLossRing;
    const int64_t cnt = std::min(n - done, (int64_t)kLossRing - row);
    HIPCHK(hipMemcpyAsync(out + done * h->nb, h->d_ring() + row * h->nb, sizeof(float) * cnt * h->nb,
                          hipMemcpyDeviceToDevice, s));
    done += cnt;
  }
  return DVNR_OK;
}

// Host copy of the losses of steps [s0, s0 + n) (n <= kLossRing): out[k][b].  Synchronizes s.
static dvnr_status copy_losses_host(dvnr_t* h, int64_t s0, int64_t n, float* out, hipStream_t s) {
  int64_t done = 0;
  while (done < n) {
    const int64_t row = (s0 + done) % kLossRing;
    const int64_t cnt = std::min(n - done, (int64_t)kLossRing - row);
    HIPCHK(hipMemcpyAsync(out + done * h->nb, h->d_ring() + row * h->nb, sizeof(float) * cnt * h->nb,
                          hipMemcpyDeviceToHost, s));
    done += cnt;
  }
  HIPCHK(hipStreamSynchronize(s));
  return DVNR_OK;
}

static dvnr_status train_ready(dvnr_t* h) {
  if (!h) return fail(DVNR_E_INVALID, "null handle");
  if (!h->bound) return fail(DVNR_E_STATE, "train before dvnr_bind");
  if (!h->prepared) return fail(DVNR_E_STATE, "train before dvnr_prepare");
  if (h->prec == Prec::F64) return fail(DVNR_E_UNSUPPORTED, "fp64 handles provide the autograd building blocks only");
  return DVNR_OK;
}

// n_steps generated-sample steps with the current plan: replays of one
// captured step (hipGraph, keyed by stream and `plan_key`) on a non-default
// stream, else eager launches.  Losses of the steps go to loss_out (device
// float [n_steps][n_blocks]) when given.
// Capture one step as a graph (kernel arguments are fixed at capture).
static dvnr_status capture_step(dvnr_t* h, hipStream_t s, int set, bool ahead, hipGraphExec_t* out) {
  hipGraph_t g;
  HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  dvnr_status st = enqueue_step(h, 1, s, set, ahead);
  hipError_t ce = hipStreamEndCapture(s, &g);
  if (st) return st;
  if (ce != hipSuccess) return fail(DVNR_E_HIP, std::string("graph capture: ") + hipGetErrorString(ce));
  ce = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ce != hipSuccess) return fail(DVNR_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(ce));
  return DVNR_OK;
}

static dvnr_status run_steps(dvnr_t* h, int64_t n_steps, int64_t plan_key, float* loss_out, hipStream_t s) {
  dvnr_status st = DVNR_OK;
  const int64_t s0 = h->host_step;
  int64_t done = 0;
  const bool graph_ok = h->use_graph && !h->profile && s != nullptr;
  // sampler look-ahead: the first step's samples are drawn here into set 0;
  // every replayed step trains on set p and draws the next step's into 1 - p
  // (the last step's draw is not used).  No drawn samples outlive the call,
  // so changes of the volumes or ranges between calls are always seen.
  const bool ahead = graph_ok && h->sample_ahead && h->spatial_sort && h->n_groups > 0 && n_steps > 0;
  if (ahead) {
    if (!h->graph_ahead[0] || h->graph_stream != s || h->graph_total != plan_key) {
      drop_graphs(h);
      for (int p = 0; p < 2; ++p) {
        st = capture_step(h, s, p, true, &h->graph_ahead[p]);
        if (st) return st;
      }
      h->graph_stream = s;
      h->graph_total = plan_key;
    }
    st = enqueue_sorted_sample(h, 0, 0, s);
    if (st) return st;
  }
  int set = 0;
  while (done < n_steps) {
    const int64_t chunk = std::min<int64_t>(n_steps - done, kLossRing);
    if (ahead) {
      for (int64_t k = 0; k < chunk; ++k, set ^= 1) HIPCHK(hipGraphLaunch(h->graph_ahead[set], s));
    } else if (graph_ok && (!h->graph || h->graph_stream != s || h->graph_total != plan_key)) {
      drop_graphs(h);
      st = capture_step(h, s, 0, false, &h->graph);
      if (st) return st;
      h->graph_stream = s;
      h->graph_total = plan_key;
    }
    for (int64_t k = 0; k < chunk && !ahead; ++k) {
      if (graph_ok) {
        HIPCHK(hipGraphLaunch(h->graph, s));
      } else {
        st = enqueue_step(h, 1, s);
        if (st) return st;
      }
    }
    h->host_step += chunk;
    if (loss_out) {
      st = copy_losses(h, s0 + done, chunk, loss_out + done * h->nb, s);
      if (st) return st;
    }
    done += chunk;
  }
  return DVNR_OK;
}

dvnr_status dvnr_train_steps(dvnr_t* h, int32_t n_steps, int64_t samples_per_step, float* loss_out, void* stream) {
  try {
    dvnr_status st = train_ready(h);
    if (st) return st;
    if (n_steps < 0) return fail(DVNR_E_INVALID, "n_steps < 0");
    if (samples_per_step < 1 || samples_per_step > h->max_batch)
      return fail(DVNR_E_INVALID, "samples_per_step must be in [1, max_batch]");
    if (h->nb > 1 && samples_per_step % kTile)
      return fail(DVNR_E_INVALID, "with several blocks samples_per_step must be a multiple of 256");
    hipStream_t s = (hipStream_t)stream;
    if (h->plan_total != samples_per_step) {
      st = set_plan(h, apportion(h, samples_per_step), s);
      if (st) return st;
      h->plan_total = samples_per_step;
    }
    return run_steps(h, n_steps, samples_per_step, loss_out, s);
  } catch (...) {
    return fail(DVNR_E_INVALID, "train failed");
  }
}

dvnr_status dvnr_train_until(dvnr_t* h, const dvnr_stop_policy* pol, int64_t samples_per_step, int64_t* steps_out,
                             double* avg_loss_out, void* stream) {
  try {
    dvnr_status st = train_ready(h);
    if (st) return st;
    if (!pol || !steps_out) return fail(DVNR_E_INVALID, "null argument");
    if (pol->min_steps < 0 || pol->epochs < 0 || pol->window < 1 || pol->window > kLossRing ||
        pol->check_every < 1 || !(pol->loss_threshold == pol->loss_threshold))
      return fail(DVNR_E_INVALID, "bad stop policy");
    if (samples_per_step < 1 || samples_per_step > h->max_batch)
      return fail(DVNR_E_INVALID, "samples_per_step must be in [1, max_batch]");
    if (h->nb > 1 && samples_per_step % kTile)
      return fail(DVNR_E_INVALID, "with several blocks samples_per_step must be a multiple of 256");
    hipStream_t s = (hipStream_t)stream;
    const std::vector<int64_t> n = apportion(h, samples_per_step);
    // per-block step budget N_max = max(N_min, ceil(N_vox / n_b) * N_epoch)
    std::vector<int64_t> n_max(h->nb, 0);
    std::vector<char> active(h->nb, 0);
    for (int b = 0; b < h->nb; ++b) {
      steps_out[b] = 0;
      if (avg_loss_out) avg_loss_out[b] = std::nan("");
      if (n[b] <= 0) continue;
      const int64_t nv = (int64_t)h->blocks[b].dims[0] * h->blocks[b].dims[1] * h->blocks[b].dims[2];
      n_max[b] = std::max<int64_t>(pol->min_steps, (nv + n[b] - 1) / n[b] * pol->epochs);
      active[b] = n_max[b] > 0;
    }
    const bool use_loss = pol->loss_threshold > 0.0;
    std::vector<float> ring;
    int64_t done = 0;
    bool replan = true;
    for (;;) {
      int64_t next_end = INT64_MAX;
      for (int b = 0; b < h->nb; ++b)
        if (active[b]) next_end = std::min(next_end, n_max[b]);
      if (next_end == INT64_MAX) break;
      if (replan) {
        // stopped blocks draw no samples (their updates are skipped); the others keep their n_b
        std::vector<int64_t> nm(h->nb);
        for (int b = 0; b < h->nb; ++b) nm[b] = active[b] ? n[b] : 0;
        st = set_plan(h, nm, s);
        if (st) return st;
        h->plan_total = -1;  // the next dvnr_train_steps rebuilds its plan
        replan = false;
      }
      const int64_t next_check = use_loss ? (done / pol->check_every + 1) * pol->check_every : INT64_MAX;
      const int64_t chunk = std::min(next_end, next_check) - done;
      st = run_steps(h, chunk, -2, nullptr, s);
      if (st) return st;
      done += chunk;
      for (int b = 0; b < h->nb; ++b)
        if (active[b] && done >= n_max[b]) {
          active[b] = 0;
          steps_out[b] = done;
          replan = true;
        }
      if (use_loss && done % pol->check_every == 0 && done >= pol->window) {
        // moving average of the last `window` losses of every block (device ring of kLossRing steps)
        ring.assign((size_t)pol->window * h->nb, 0.0f);
        st = copy_losses_host(h, h->host_step - pol->window, pol->window, ring.data(), s);
        if (st) return st;
        for (int b = 0; b < h->nb; ++b) {
          if (!active[b] && steps_out[b] != done) continue;
          double acc = 0.0;
          for (int k = 0; k < pol->window; ++k) acc += (double)ring[(size_t)k * h->nb + b];
          const double ma = acc / pol->window;
          if (avg_loss_out) avg_loss_out[b] = ma;
          if (active[b] && ma < pol->loss_threshold) {
            active[b] = 0;
            steps_out[b] = done;
            replan = true;
          }
        }
      }
    }
    HIPCHK(hipStreamSynchronize(s));
    return DVNR_OK;
  } catch (...) {
    return fail(DVNR_E_INVALID, "train failed");
  }
}

dvnr_status dvnr_train_step_coords(dvnr_t* h, const float* coords, const int64_t* n_per_block, float* loss_out,
                                   void* stream) {
  try {
    dvnr_status st = train_ready(h);
    if (st) return st;
    if (!coords || !n_per_block) return fail(DVNR_E_INVALID, "null argument");
    hipStream_t s = (hipStream_t)stream;
    std::vector<int64_t> n(n_per_block, n_per_block + h->nb);
    int64_t total = 0;
    for (auto v : n) {
      if (v < 0) return fail(DVNR_E_INVALID, "negative sample count");
      total += v;
    }
    if (total < 1 || total > h->max_batch) return fail(DVNR_E_INVALID, "total samples must be in [1, max_batch]");
    st = set_plan(h, n, s);
    if (st) return st;
    h->plan_total = -1;  // the next dvnr_train_steps rebuilds its plan
    HIPCHK(hipMemcpyAsync(h->d_coords(), coords, sizeof(float) * 3 * total, hipMemcpyDeviceToDevice, s));
    st = enqueue_step(h, 0, s);
    if (st) return st;
    const int64_t s0 = h->host_step;
    h->host_step += 1;
    if (loss_out) return copy_losses(h, s0, 1, loss_out, s);
    return DVNR_OK;
  } catch (...) {
    return fail(DVNR_E_INVALID, "train failed");
  }
}

dvnr_status dvnr_draw_training_samples(dvnr_t* h, int32_t block, int64_t step, int64_t n, float* coords,
                                       float* target, void* stream) {
  if (!h) return fail(DVNR_E_INVALID, "null handle");
  if (!h->prepared) return fail(DVNR_E_STATE, "call dvnr_prepare first");
  if (block < 0 || block >= h->nb) return fail(DVNR_E_INVALID, "bad block");
  if (n < 0 || n >= ((int64_t)1 << 31) || step < 0 || !coords || !target) return fail(DVNR_E_INVALID, "bad arguments");
  if (n == 0) return DVNR_OK;
  SampleDist d = h->dist();
  d.direct_n_uni = (int32_t)(n - boundary_count(n, h->bnd_frac));
  HIPCHK(launch_sample(h->d_meta(), h->d_range(), nullptr, nullptr, (int)n, block, 1, h->seed, d, h->d_ctr(), step,
                       coords, target, (hipStream_t)stream));
  return DVNR_OK;
}

// INR output at `n` coordinates of block b (chunks of max_batch), de-normalized.
static constexpr int64_t align256(int64_t v) { return (v + 255) / 256 * 256; }

// Parameters a query reads: the inference copy of every block (the fp16 / bf16
// working copy for mixed precision, fp32 masters otherwise) and the block
// value ranges; the live model or a cached snapshot.
struct ModelSrc {
  const void* params;
  const BlockRange* range;
};

static ModelSrc live_src(const dvnr_t* h) {
  return ModelSrc{h->prec == Prec::MIXED ? (const void*)h->buf.work16 : (const void*)h->buf.params, h->d_range()};
}

static dvnr_status infer_coords(dvnr_t* h, int b, int64_t n, const float* coords, float* out, hipStream_t s,
                                const ModelSrc& src) {
  const bool mixed = h->prec == Prec::MIXED;
  const int64_t F = h->enc.n_features;
  const void* table = src.params;
  const void* wsrc = mixed ? (const void*)((const uint16_t*)src.params + h->n_table)
                           : (const void*)((const float*)src.params + h->n_table);
  for (int64_t c0 = 0; c0 < n; c0 += h->max_batch) {
    const int64_t cn = std::min(h->max_batch, n - c0);
    HIPCHK(launch_encode(h->prec, mixed ? 1 : 0, h->ld, h->d_meta(), nullptr, (int)cn, b, nullptr, coords + 3 * c0,
                         table, h->d_feat(), F, h->max_batch * F, h->xcd_map, s));
    HIPCHK(launch_mlp_infer(h->prec, h->md, h->ld, h->d_meta(), src.range, nullptr, nullptr, (int)cn, b,
                            h->d_feat(), wsrc, h->max_batch, out + c0, s));
  }
  return DVNR_OK;
}

static dvnr_status access_ready(dvnr_t* h, int32_t block) {
  if (!h) return fail(DVNR_E_INVALID, "null handle");
  if (!h->prepared) return fail(DVNR_E_STATE, "call dvnr_prepare first");
  if (h->prec == Prec::F64) return fail(DVNR_E_UNSUPPORTED, "fp64 handles provide the autograd building blocks only");
  if (block < 0 || block >= h->nb) return fail(DVNR_E_INVALID, "bad block");
  return DVNR_OK;
}

dvnr_status dvnr_sample(dvnr_t* h, int32_t block, int64_t n, const float* coords, float* out, void* stream) {
  dvnr_status st = access_ready(h, block);
  if (st) return st;
  if (n < 0 || (n > 0 && (!coords || !out))) return fail(DVNR_E_INVALID, "bad arguments");
  return infer_coords(h, block, n, coords, out, (hipStream_t)stream, live_src(h));
}

static dvnr_status decode_impl(dvnr_t* h, int32_t block, float* out, hipStream_t s, const ModelSrc& src) {
  const int b0 = block < 0 ? 0 : block, b1 = block < 0 ? h->nb : block + 1;
  int64_t out_off = 0;
  dvnr_status st = DVNR_OK;
  for (int b = b0; b < b1; ++b) {
    const int64_t nvox = owned_voxels(h->blocks[b]);
    if (h->decode_fused) {
      HIPCHK(launch_decode_fused(h->prec, h->ld, h->md, h->d_meta(), src.range, b, h->blocks[b].dims, src.params,
                                 src.params, h->n_table, h->ws() + h->o_decop, out + out_off, s));
      out_off += nvox;
      continue;
    }
    for (int64_t c0 = 0; c0 < nvox; c0 += h->max_batch) {
      const int64_t cn = std::min(h->max_batch, nvox - c0);
      HIPCHK(launch_voxel_coords(h->d_meta(), b, c0, cn, h->d_coords(), s));
      st = infer_coords(h, b, cn, h->d_coords(), out + out_off + c0, s, src);
      if (st) return st;
    }
    out_off += nvox;
  }
  return DVNR_OK;
}

dvnr_status dvnr_decode(dvnr_t* h, int32_t block, float* out, void* stream) {
  if (!out) return fail(DVNR_E_INVALID, "null output");
  dvnr_status st = access_ready(h, block < 0 ? 0 : block);
  if (st) return st;
  if (block >= h->nb) return fail(DVNR_E_INVALID, "bad block");
  return decode_impl(h, block, out, (hipStream_t)stream, live_src(h));
}

// ---------------------------------------------------------------------------
// Direct volume rendering (sample streaming)
// ---------------------------------------------------------------------------
static constexpr int64_t render_ws_bytes(int64_t n) {
  // directions [n][3], (t0, t1) [n][2], two active-ray lists [n], two counters
  return align256(12 * n) + align256(8 * n) + 2 * align256(4 * n) + 256;
}

dvnr_status dvnr_render_workspace_bytes(const dvnr_t* h, int32_t width, int32_t height, int64_t* bytes) {
  if (!h || !bytes) return fail(DVNR_E_INVALID, "null argument");
  if (width < 1 || height < 1 || (int64_t)width * height > (1 << 28)) return fail(DVNR_E_INVALID, "bad image size");
  *bytes = render_ws_bytes((int64_t)width * height);
  return DVNR_OK;
}

// Argument checks shared by both render entry points (the workspace aside).
static dvnr_status render_args(dvnr_t* h, int32_t block, const dvnr_camera* cam, const dvnr_render_params* rp,
                               const float* tf, float* image) {
  dvnr_status st = access_ready(h, block);
  if (st) return st;
  if (!cam || !rp || !tf || !image) return fail(DVNR_E_INVALID, "null argument");
  if (cam->width < 1 || cam->height < 1 || (int64_t)cam->width * cam->height > (1 << 28))
    return fail(DVNR_E_INVALID, "bad image size");
  if (!(cam->fovy_deg > 0.0f && cam->fovy_deg < 180.0f)) return fail(DVNR_E_INVALID, "fovy must be in (0, 180)");
  if (!(rp->step > 0.0f) || !(rp->ref_step > 0.0f) || rp->n_tf < 2 || !(rp->tf_hi > rp->tf_lo) ||
      !(rp->alpha_stop > 0.0f && rp->alpha_stop <= 1.0f) || rp->samples_per_round < 1 ||
      rp->samples_per_round > h->max_batch)
    return fail(DVNR_E_INVALID, "bad render parameters");
  return DVNR_OK;
}

// The renderer proper on a checked argument set; `workspace` holds
// render_ws_bytes(width * height) bytes, 256-byte aligned.
static dvnr_status render_impl(dvnr_t* h, int32_t block, const dvnr_camera* cam, const dvnr_render_params* rp,
                               const float* tf, void* workspace, float* image, int64_t* samples_out, void* stream) {
  try {
    dvnr_status st = DVNR_OK;
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = (int64_t)cam->width * cam->height;
    char* ws = (char*)workspace;
    float* dirs = (float*)ws;
    float* t01 = (float*)(ws + align256(12 * n));
    int32_t* list[2] = {(int32_t*)(ws + align256(12 * n) + align256(8 * n)),
                        (int32_t*)(ws + align256(12 * n) + align256(8 * n) + align256(4 * n))};
    int32_t* counters = (int32_t*)(ws + align256(12 * n) + align256(8 * n) + 2 * align256(4 * n));
    RayCamera rc;
    for (int a = 0; a < 3; ++a) {
      rc.eye[a] = cam->eye[a];
      rc.center[a] = cam->center[a];
      rc.up[a] = cam->up[a];
    }
    rc.tan_h = (float)std::tan((double)cam->fovy_deg * 3.14159265358979323846 / 360.0);
    const int S = rp->samples_per_round;
    const float opacity_exp = (float)((double)rp->step / (double)rp->ref_step);
    const float tf_inv = (float)(1.0 / ((double)rp->tf_hi - (double)rp->tf_lo));
    const ModelSrc src = live_src(h);
    HIPCHK(launch_zero(counters, 2 * sizeof(int32_t), s));
    HIPCHK(launch_ray_init(rc, cam->width, cam->height, dirs, t01, image, list[0], counters, s));
    int32_t n_active = 0;
    HIPCHK(hipMemcpyAsync(&n_active, counters, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const int chunk = std::max<int64_t>(1, h->max_batch / S);
    int cur = 0;
    int64_t generated = 0;
    for (int k_base = 0; n_active > 0; k_base += S) {
      HIPCHK(launch_zero(counters + 1, sizeof(int32_t), s));
      generated += (int64_t)n_active * S;
      for (int c0 = 0; c0 < n_active; c0 += chunk) {
        const int cn = std::min(chunk, n_active - c0);
        HIPCHK(launch_ray_gen(rc, list[cur] + c0, cn, k_base, S, rp->step, dirs, t01, h->d_coords(), s));
        st = infer_coords(h, block, (int64_t)cn * S, h->d_coords(), h->d_target(), s, src);
        if (st) return st;
        HIPCHK(launch_ray_shade(list[cur] + c0, cn, k_base, S, rp->step, opacity_exp, rp->alpha_stop, t01,
                                h->d_target(), tf, rp->n_tf, rp->tf_lo, tf_inv, image, list[1 - cur], counters + 1,
                                s));
      }
      HIPCHK(hipMemcpyAsync(&n_active, counters + 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      cur = 1 - cur;
    }
    if (samples_out) *samples_out = generated;
    return DVNR_OK;
  } catch (...) {
    return fail(DVNR_E_INVALID, "render failed");
  }
}

dvnr_status dvnr_render(dvnr_t* h, int32_t block, const dvnr_camera* cam, const dvnr_render_params* rp,
                        const float* tf, void* workspace, float* image, int64_t* samples_out, void* stream) {
  dvnr_status st = render_args(h, block, cam, rp, tf, image);
  if (st) return st;
  if (!workspace) return fail(DVNR_E_INVALID, "null workspace");
  if (((uintptr_t)workspace) % 256) return fail(DVNR_E_INVALID, "workspace must be 256-byte aligned");
  return render_impl(h, block, cam, rp, tf, workspace, image, samples_out, stream);
}

// ---------------------------------------------------------------------------
// Rendering without a caller workspace: the ray state lives in one static
// device array per GPU.  Host code never passes `scratch` itself to a kernel
// (on the host its name is only a stand-in for the symbol): its device address
// is looked up once per device and used instead.
// ---------------------------------------------------------------------------
static constexpr int64_t kRenderStaticBytes = render_ws_bytes(DVNR_RENDER_STATIC_MAX_RAYS);  // 28 MiB + 256 B
static __device__ __align__(256) char scratch[kRenderStaticBytes];

static std::mutex g_scratch_mu;
static std::vector<void*> g_scratch_ptr;  // per device ordinal; nullptr until looked up

// Device address of this GPU's `scratch` (the current device's copy).
static dvnr_status static_scratch(void** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p || ((uintptr_t)p) % 256) return fail(DVNR_E_HIP, "static render scratch has no aligned device address");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return DVNR_OK;
}

dvnr_status dvnr_render_static(dvnr_t* h, int32_t block, const dvnr_camera* cam, const dvnr_render_params* rp,
                               const float* tf, float* image, int64_t* samples_out, void* stream) {
  dvnr_status st = render_args(h, block, cam, rp, tf, image);
  if (st) return st;
  if ((int64_t)cam->width * cam->height > DVNR_RENDER_STATIC_MAX_RAYS)
    return fail(DVNR_E_INVALID, "dvnr_render_static: image larger than DVNR_RENDER_STATIC_MAX_RAYS pixels");
  void* ws = nullptr;
  st = static_scratch(&ws);
  if (st) return st;
  return render_impl(h, block, cam, rp, tf, ws, image, samples_out, stream);
}

// ---------------------------------------------------------------------------
// Sliding-window model cache
// ---------------------------------------------------------------------------
static int64_t snap_param_bytes(const dvnr_t* h) { return align256((int64_t)h->nb * h->stride * h->ielem()); }

static int64_t snap_bytes(const dvnr_t* h) {
  return snap_param_bytes(h) + align256((int64_t)sizeof(BlockRange) * h->nb);
}

dvnr_status dvnr_cache_snapshot_bytes(const dvnr_t* h, int64_t* bytes) {
  if (!h || !bytes) return fail(DVNR_E_INVALID, "null argument");
  if (h->prec == Prec::F64) return fail(DVNR_E_UNSUPPORTED, "fp64 handles have no model cache");
  *bytes = snap_bytes(h);
  return DVNR_OK;
}

dvnr_status dvnr_cache_bind(dvnr_t* h, int32_t capacity, void* buffer) {
  if (!h) return fail(DVNR_E_INVALID, "null handle");
  if (h->prec == Prec::F64) return fail(DVNR_E_UNSUPPORTED, "fp64 handles have no model cache");
  if (capacity < 0 || (capacity > 0 && !buffer)) return fail(DVNR_E_INVALID, "bad cache buffer");
  if (((uintptr_t)buffer) % 256) return fail(DVNR_E_INVALID, "cache buffer must be 256-byte aligned");
  h->cache_buf = (char*)buffer;
  h->cache_cap = capacity;
  h->cache_head = 0;
  h->cache_count = 0;
  h->cache_keys.assign(capacity, 0);
  return DVNR_OK;
}

static int cache_slot_of(const dvnr_t* h, int64_t key) {
  for (int k = 0; k < h->cache_count; ++k) {
    const int slot = (h->cache_head + k) % h->cache_cap;
    if (h->cache_keys[slot] == key) return slot;
  }
  return -1;
}

static ModelSrc cache_src(const dvnr_t* h, int slot) {
  const char* base = h->cache_buf + (int64_t)slot * snap_bytes(h);
  return ModelSrc{base, (const BlockRange*)(base + snap_param_bytes(h))};
}

dvnr_status dvnr_cache_push(dvnr_t* h, int64_t key, void* stream) {
  if (!h) return fail(DVNR_E_INVALID, "null handle");
  if (!h->prepared) return fail(DVNR_E_STATE, "call dvnr_prepare first");
  if (h->cache_cap < 1) return fail(DVNR_E_STATE, "no cache bound");
  if (cache_slot_of(h, key) >= 0) return fail(DVNR_E_INVALID, "key already cached");
  hipStream_t s = (hipStream_t)stream;
  int slot;
  if (h->cache_count < h->cache_cap) {
    slot = (h->cache_head + h->cache_count) % h->cache_cap;
    ++h->cache_count;
  } else {  // full: the oldest snapshot makes room
    slot = h->cache_head;
    h->cache_head = (h->cache_head + 1) % h->cache_cap;
  }
  h->cache_keys[slot] = key;
  const ModelSrc live = live_src(h);
  char* dst = h->cache_buf + (int64_t)slot * snap_bytes(h);
  HIPCHK(hipMemcpyAsync(dst, live.params, (size_t)((int64_t)h->nb * h->stride * h->ielem()), hipMemcpyDeviceToDevice,
                        s));
  HIPCHK(hipMemcpyAsync(dst + snap_param_bytes(h), live.range, sizeof(BlockRange) * h->nb, hipMemcpyDeviceToDevice,
                        s));
  return DVNR_OK;
}

dvnr_status dvnr_cache_keys(const dvnr_t* h, int64_t* keys, int32_t* count) {
  if (!h || !count) return fail(DVNR_E_INVALID, "null argument");
  *count = h->cache_count;
  if (keys)
    for (int k = 0; k < h->cache_count; ++k) keys[k] = h->cache_keys[(h->cache_head + k) % h->cache_cap];
  return DVNR_OK;
}

dvnr_status dvnr_cache_decode(dvnr_t* h, int64_t key, int32_t block, float* out, void* stream) {
  if (!out) return fail(DVNR_E_INVALID, "null output");
  dvnr_status st = access_ready(h, block < 0 ? 0 : block);
  if (st) return st;
  if (block >= h->nb) return fail(DVNR_E_INVALID, "bad block");
  const int slot = h->cache_cap > 0 ? cache_slot_of(h, key) : -1;
  if (slot < 0) return fail(DVNR_E_INVALID, "key not cached");
  return decode_impl(h, block, out, (hipStream_t)stream, cache_src(h, slot));
}

dvnr_status dvnr_cache_sample(dvnr_t* h, int64_t key, int32_t block, int64_t n, const float* coords, float* out,
                              void* stream) {
  dvnr_status st = access_ready(h, block);
  if (st) return st;
  if (n < 0 || (n > 0 && (!coords || !out))) return fail(DVNR_E_INVALID, "bad arguments");
  const int slot = h->cache_cap > 0 ? cache_slot_of(h, key) : -1;
  if (slot < 0) return fail(DVNR_E_INVALID, "key not cached");
  return infer_coords(h, block, n, coords, out, (hipStream_t)stream, cache_src(h, slot));
}

dvnr_status dvnr_mse_fp64(dvnr_t* h, int32_t block, const float* decoded, double* sse, int64_t* count,
                          void* stream) {
  if (!h) return fail(DVNR_E_INVALID, "null handle");
  if (!h->bound) return fail(DVNR_E_STATE, "dvnr_mse_fp64 before dvnr_bind");
  if (block < 0 || block >= h->nb || !decoded || !sse) return fail(DVNR_E_INVALID, "bad arguments");
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(launch_zero(h->d_mse(), sizeof(double), s));
  HIPCHK(launch_mse(h->d_meta(), block, decoded, h->d_mse(), s));
  double v = 0;
  HIPCHK(hipMemcpyAsync(&v, h->d_mse(), sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  *sse = v;
  if (count) *count = owned_voxels(h->blocks[block]);
  return DVNR_OK;
}

// Autograd building blocks: `block` selects the block whose bound buffers a
// NULL table / weights / gradient pointer stands for.
static dvnr_status building_block_ready(dvnr_t* h, int32_t block, bool needs_bound) {
  if (!h) return fail(DVNR_E_INVALID, "null handle");
  if (block < 0 || block >= h->nb) return fail(DVNR_E_INVALID, "bad block");
  if (needs_bound && !h->bound) return fail(DVNR_E_STATE, "a NULL parameter pointer needs dvnr_bind");
  return DVNR_OK;
}

static char* block_elem(const dvnr_t* h, void* base, int32_t block, int64_t rel) {
  return (char*)base + (size_t)(((int64_t)block * h->stride + rel) * (int64_t)h->pelem());
}

dvnr_status dvnr_encode_forward(dvnr_t* h, int32_t block, int64_t n, const float* coords, const void* table,
                                void* feats, void* stream) {
  dvnr_status st = building_block_ready(h, block, !table);
  if (st) return st;
  if (n < 0 || n >= ((int64_t)1 << 31) || (n > 0 && (!coords || !feats))) return fail(DVNR_E_INVALID, "bad arguments");
  if (!table) table = block_elem(h, h->buf.params, block, 0);
  const int64_t LF = h->md.in_dim;
  const Prec tp = h->prec == Prec::F64 ? Prec::F64 : Prec::F32;
  HIPCHK(launch_encode(tp, tp == Prec::F64 ? 2 : 0, h->ld, nullptr, nullptr, (int)n, 0, nullptr, coords, table, feats,
                       LF, h->enc.n_features, 0, (hipStream_t)stream));
  return DVNR_OK;
}

dvnr_status dvnr_encode_backward(dvnr_t* h, int32_t block, int64_t n, const float* coords, const void* dfeats,
                                 void* dtable, void* stream) {
  dvnr_status st = building_block_ready(h, block, !dtable);
  if (st) return st;
  if (n < 0 || n >= ((int64_t)1 << 31) || (n > 0 && (!coords || !dfeats))) return fail(DVNR_E_INVALID, "bad arguments");
  if (!dtable) dtable = block_elem(h, h->buf.grads, block, 0);
  const int64_t LF = h->md.in_dim;
  const Prec gp = h->prec == Prec::F64 ? Prec::F64 : Prec::F32;
  HIPCHK(launch_scatter(gp, h->ld, 0, h->enc.n_levels, nullptr, nullptr, (int)n, 0, nullptr, coords, dfeats, LF,
                        h->enc.n_features, dtable,
                        0, 0, 0, (hipStream_t)stream));
  return DVNR_OK;
}

dvnr_status dvnr_mlp_forward(dvnr_t* h, int32_t block, int64_t n, const void* feats, const void* weights, void* out,
                             void* stream) {
  dvnr_status st = building_block_ready(h, block, !weights);
  if (st) return st;
  if (n < 0 || (n > 0 && (!feats || !out))) return fail(DVNR_E_INVALID, "bad arguments");
  if (!weights) weights = block_elem(h, h->buf.params, block, h->n_table);
  const Prec p = h->prec == Prec::F64 ? Prec::F64 : Prec::F32;
  HIPCHK(launch_mlp_simple_fwd(p, h->md, n, feats, weights, out, (hipStream_t)stream));
  return DVNR_OK;
}

dvnr_status dvnr_mlp_backward(dvnr_t* h, int32_t block, int64_t n, const void* feats, const void* weights,
                              const void* dout, void* dfeats, void* dweights, void* stream) {
  dvnr_status st = building_block_ready(h, block, !weights || !dweights);
  if (st) return st;
  if (n < 0 || (n > 0 && (!feats || !dout || !dfeats))) return fail(DVNR_E_INVALID, "bad arguments");
  if (!weights) weights = block_elem(h, h->buf.params, block, h->n_table);
  if (!dweights) dweights = block_elem(h, h->buf.grads, block, h->n_table);
  const Prec p = h->prec == Prec::F64 ? Prec::F64 : Prec::F32;
  HIPCHK(launch_mlp_simple_bwd(p, h->md, n, feats, weights, dout, dfeats, dweights, (hipStream_t)stream));
  return DVNR_OK;
}

dvnr_status dvnr_adam_step(dvnr_t* h, void* stream) {
  if (!h) return fail(DVNR_E_INVALID, "null handle");
  if (!h->bound) return fail(DVNR_E_STATE, "dvnr_adam_step before dvnr_bind");
  hipStream_t s = (hipStream_t)stream;
  // this update's index t = step + 1, then every parameter of every block
  HIPCHK(launch_bump_step(h->d_ctr(), s));
  HIPCHK(launch_adam(h->prec, h->buf.params, h->buf.grads, h->buf.adam_m, h->buf.adam_v,
                     h->prec == Prec::MIXED ? (uint16_t*)h->buf.work16 : nullptr, h->nb, h->stride, h->n_table,
                     h->n_table + h->n_mlp, nullptr, h->d_ctr(), h->opt.lr, h->opt.beta1, h->opt.beta2, h->opt.eps,
                     h->opt.weight_decay, h->opt.lr_decay_interval > 0 ? h->opt.lr_decay_base : 1.0,
                     h->opt.lr_decay_start, h->opt.lr_decay_interval > 0 ? h->opt.lr_decay_interval : 0, s));
  h->host_step += 1;
  return DVNR_OK;
}

dvnr_status dvnr_debug_indices(dvnr_t* h, int32_t level, int64_t n, const float* coords, uint32_t* idx, float* w,
                               void* stream) {
  if (!h) return fail(DVNR_E_INVALID, "null handle");
  if (level < 0 || level >= h->enc.n_levels) return fail(DVNR_E_INVALID, "bad level");
  if (n < 0 || (n > 0 && (!coords || !idx || !w))) return fail(DVNR_E_INVALID, "bad arguments");
  HIPCHK(launch_debug_indices(h->ld, level, n, coords, idx, w, (hipStream_t)stream));
  return DVNR_OK;
}

dvnr_status dvnr_sync(dvnr_t* h, void* stream) {
  if (!h) return fail(DVNR_E_INVALID, "null handle");
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipGetLastError());
  if (h->bound) {
    int32_t flag = 0;
    HIPCHK(hipMemcpy(&flag, (char*)h->d_ctr() + offsetof(Counters, nonfinite), sizeof(int32_t), hipMemcpyDeviceToHost));
    if (flag) {
      HIPCHK(hipMemset((char*)h->d_ctr() + offsetof(Counters, nonfinite), 0, sizeof(int32_t)));
      return fail(DVNR_E_NONFINITE, "non-finite training loss");
    }
  }
  return DVNR_OK;
}

dvnr_status dvnr_autotune(dvnr_t* h, int64_t samples_per_step, int32_t n_trial_steps, double* best_ms,
                          void* stream) {
  try {
    dvnr_status st = train_ready(h);
    if (st) return st;
    if (samples_per_step < 1 || samples_per_step > h->max_batch)
      return fail(DVNR_E_INVALID, "samples_per_step must be in [1, max_batch]");
    if (h->nb > 1 && samples_per_step % kTile)
      return fail(DVNR_E_INVALID, "with several blocks samples_per_step must be a multiple of 256");
    if (n_trial_steps < 1 || n_trial_steps > 1000) return fail(DVNR_E_INVALID, "n_trial_steps must be in [1, 1000]");
    hipStream_t s = (hipStream_t)stream;
    const int save_update = h->apply_update, save_profile = h->profile;
    const int64_t saved_step = h->host_step;
    const std::vector<int64_t> n = apportion(h, samples_per_step);
    // the automatic privatized-level count of this plan
    h->priv_levels = -1;
    h->spatial_sort = 1;
    st = set_plan(h, n, s);
    if (st) return st;
    const int auto_pl = h->priv_L, L = h->enc.n_levels;
    struct Cand {
      int sort, priv, cap;
    };
    std::vector<Cand> cands = {{0, 0, kMlpGrid},
                               {1, auto_pl, kMlpGrid},
                               {1, std::max(0, L - 3), kMlpGrid},
                               {1, std::max(0, L - 5), kMlpGrid},
                               {1, auto_pl, kMlpGrid / 2},
                               {1, auto_pl, 2 * kMlpGrid}};
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    h->apply_update = 0;
    h->profile = 0;
    double best = 1e300;
    Cand pick = cands[1];
    for (const Cand& c : cands) {
      h->spatial_sort = c.sort;
      h->priv_levels = c.priv;
      h->mlp_cap = c.cap;
      st = set_plan(h, n, s);
      if (st) break;
      for (int k = 0; k < 2 && !st; ++k) st = enqueue_step(h, 1, s);
      if (st) break;
      HIPCHK(hipEventRecord(e0, s));
      for (int k = 0; k < n_trial_steps && !st; ++k) st = enqueue_step(h, 1, s);
      if (st) break;
      HIPCHK(hipEventRecord(e1, s));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0.0f;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      const double per = (double)ms / n_trial_steps;
      if (per < best) {
        best = per;
        pick = c;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    h->apply_update = save_update;
    h->profile = save_profile;
    if (st) return st;
    // restore the step counter and clear the trial gradients
    int64_t* dstep = (int64_t*)((char*)h->d_ctr() + offsetof(Counters, step));
    HIPCHK(hipMemcpyAsync(dstep, &saved_step, sizeof(int64_t), hipMemcpyHostToDevice, s));
    HIPCHK(launch_zero(h->buf.grads, h->n_params * (int64_t)h->pelem(), s));
    HIPCHK(hipStreamSynchronize(s));
    h->host_step = saved_step;
    h->spatial_sort = pick.sort;
    h->priv_levels = pick.priv;
    h->mlp_cap = pick.cap;
    st = set_plan(h, n, s);
    if (st) return st;
    h->plan_total = samples_per_step;
    if (best_ms) *best_ms = best;
    return DVNR_OK;
  } catch (...) {
    return fail(DVNR_E_INVALID, "autotune failed");
  }
}

dvnr_status dvnr_plan_info(const dvnr_t* h, int32_t* bins_per_axis, int32_t* priv_levels) {
  if (!h) return fail(DVNR_E_INVALID, "null handle");
  const bool on = h->spatial_sort && h->n_groups > 0;
  if (bins_per_axis) *bins_per_axis = on ? h->sort_B : 0;
  if (priv_levels) *priv_levels = on ? std::min(h->priv_L, h->part_l0) : 0;
  return DVNR_OK;
}

dvnr_status dvnr_plan_partition(const dvnr_t* h, int32_t* first_level) {
  if (!h || !first_level) return fail(DVNR_E_INVALID, "null argument");
  *first_level = h->part_l0;
  return DVNR_OK;
}

dvnr_status dvnr_phase_times(dvnr_t* h, double* ms, int64_t* n_steps) {
  if (!h || !ms) return fail(DVNR_E_INVALID, "null argument");
  while (h->prof_accumulated < h->prof_recorded) {
    dvnr_status st = prof_accumulate_one(h, h->prof_accumulated);
    if (st) return st;
    h->prof_accumulated += 1;
  }
  for (int p = 0; p < dvnr::kPhases; ++p) {
    ms[p] = h->prof_ms[p];
    h->prof_ms[p] = 0.0;
  }
  if (n_steps) *n_steps = h->prof_recorded;
  h->prof_recorded = h->prof_accumulated = 0;
  return DVNR_OK;
}

dvnr_status dvnr_set_option(dvnr_t* h, const char* name, int64_t value) {
  if (!h || !name) return fail(DVNR_E_INVALID, "null argument");
  const std::string n(name);
  if (n == "scatter_grouped") {
    h->scatter_grouped = value ? 1 : 0;
  } else if (n == "use_graph") {
    h->use_graph = value ? 1 : 0;
  } else if (n == "mlp_waves") {
    h->mlp_waves = value >= 2 ? 2 : 1;
  } else if (n == "mlp_wg_waves") {
    if (value != 4 && value != 8) return fail(DVNR_E_INVALID, "mlp_wg_waves: 4 or 8");
    h->mlp_wg_waves = (int)value;
  } else if (n == "mlp_grid") {
    h->mlp_cap = (int)std::max<int64_t>(1, std::min<int64_t>(value, 2 * kMlpGrid));
    h->plan_total = -1;
  } else if (n == "scatter_part") {
    h->scatter_part = (int)std::max<int64_t>(-1, std::min<int64_t>(value, kMaxLevels));
    h->plan_total = -1;  // the partitioned levels and buckets live in the plan
  } else if (n == "part_slice") {
    if (value != 4096 && value != 8192 && value != 16384) return fail(DVNR_E_INVALID, "part_slice: 4096, 8192 or 16384");
    h->part_slice_floats = (int)value;
    h->plan_total = -1;
  } else if (n == "part_capacity") {
    h->part_cap = (int)std::max<int64_t>(0, std::min<int64_t>(value, 1 << 30));
    h->plan_total = -1;
  } else if (n == "part_adam") {
    h->part_adam = value ? 1 : 0;
    h->plan_total = -1;  // the automatic partition depends on it
  } else if (n == "encode_concurrent") {
    h->encode_concurrent = value ? 1 : 0;
  } else if (n == "part_concurrent") {
    h->part_concurrent = value ? 1 : 0;
  } else if (n == "scatter_concurrent") {
    h->scatter_concurrent = value ? 1 : 0;
  } else if (n == "encode_binned") {
    h->encode_binned = value ? 1 : 0;
  } else if (n == "priv_classes") {
    h->priv_classes = value < 0 ? -1 : (value ? 1 : 0);
  } else if (n == "scatter_strided") {
    h->scatter_strided = value ? 1 : 0;
  } else if (n == "xcd_map") {
    h->xcd_map = value ? 1 : 0;
  } else if (n == "apply_update") {
    h->apply_update = value ? 1 : 0;
  } else if (n == "decode_fused") {
    h->decode_fused = value ? 1 : 0;
  } else if (n == "spatial_sort") {
    h->spatial_sort = value ? 1 : 0;
  } else if (n == "sample_ahead") {
    if (value < 0 || value > 3) return fail(DVNR_E_INVALID, "sample_ahead: 0 (off), 1, 2 or 3");
    h->sample_ahead = (int)value;
  } else if (n == "sort_bins") {
    if (value < 0 || value > 8) return fail(DVNR_E_INVALID, "sort_bins: 0 (automatic) or 1..8");
    h->sort_bins = (int)value;
    h->plan_total = -1;
  } else if (n == "priv_levels") {
    h->priv_levels = (int)std::max<int64_t>(-1, std::min<int64_t>(value, kMaxLevels));
    h->plan_total = -1;  // recompute the plan's privatized level count
  } else if (n == "profile_phases") {
    h->profile = value ? 1 : 0;
  } else {
    return fail(DVNR_E_INVALID, "unknown option " + n);
  }
  drop_graphs(h);
  return DVNR_OK;
}

dvnr_status dvnr_set_loss(dvnr_t* h, int32_t loss, double boundary_frac, double sigma) {
  if (!h) return fail(DVNR_E_INVALID, "null handle");
  if (loss != DVNR_LOSS_L2 && loss != DVNR_LOSS_L1) return fail(DVNR_E_INVALID, "unknown loss");
  if (!(boundary_frac >= 0.0 && boundary_frac <= 1.0)) return fail(DVNR_E_INVALID, "boundary_frac must be in [0, 1]");
  if (!(sigma > 0.0 && sigma <= 1.0)) return fail(DVNR_E_INVALID, "sigma must be in (0, 1]");
  h->loss_l1 = loss == DVNR_LOSS_L1 ? 1 : 0;
  h->bnd_frac = boundary_frac;
  h->bnd_sigma = sigma;
  h->plan_total = -1;  // per-block boundary counts live in the plan
  drop_graphs(h);
  return DVNR_OK;
}

}  // extern "C"
