/*
 * dvnr.h -- C ABI of the MI355X (gfx950) DVNR hot path.
 *
 * DVNR (distributed volumetric neural representation) trains one implicit
 * neural representation (INR) per box-shaped volume partition ("block"),
 * independently of every other block (paper Sec. III-A, model parallelism).
 * Each INR maps a block-normalized position x in [0,1]^3 to a normalized
 * value (Eq. (1)); it is a multiresolution hash-grid encoding followed by a
 * small bias-free ReLU MLP (Sec. III).  Training draws random coordinates
 * (uniform, optionally mixed with boundary-centered half-normal samples,
 * Sec. III-C, Eq. (2)), fetches trilinearly interpolated ground truth from the block's
 * voxels, and takes Adam steps on an L2 or L1 loss (Sec. III-B, III-C Eq. (3),
 * III-F).  Trained
 * models are queried at arbitrary coordinates or decoded back to the voxel
 * grid (Sec. III, on-demand inference and decoding).
 *
 * Conventions
 *  - Every pointer argument documented as "device" is a device address
 *    (allocated by the caller, e.g. with torch); "host" pointers are ordinary
 *    host memory.  The library allocates no device memory of its own: the
 *    caller sizes the buffers with dvnr_get_sizes() and hands them over with
 *    dvnr_bind().  Device buffers must be 256-byte aligned.  The one device
 *    array the library holds is the static scratch of dvnr_render_static.
 *  - Every entry point that launches work takes a hipStream_t (passed as
 *    void*; NULL = the default stream) and only enqueues; no entry point
 *    synchronizes except dvnr_sync() and dvnr_mse_fp64() (which returns a host
 *    value).
 *  - Status codes: DVNR_OK (0) on success.  Argument errors are reported
 *    synchronously and leave the handle unchanged; the message is available
 *    from dvnr_last_error() (thread-local, valid until the next call on the
 *    same thread).  No C++ exception crosses this boundary.
 *  - A handle is not thread-safe; calls on one handle must be serialized.
 *
 * Parameter layout (one block; blocks are concatenated at a stride of
 * `block_stride` elements, so block b starts at element b*block_stride):
 *    level tables  [sum_l E_l][F]      (feature-minor; level l starts at entry
 *                                       off_l, E_l = R_l^3 if R_l^3 <= T else T)
 *    W_1           [width][L*F]        (row-major, out x in)
 *    W_2..W_K      [width][width]
 *    W_out         [out_dim][width]
 * The same element index space is used by the master parameters, gradients,
 * Adam moments and (mixed precision) the 16-bit working copy.
 */
#ifndef DVNR_H
#define DVNR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dvnr_status;
enum {
  DVNR_OK = 0,
  DVNR_E_INVALID = 1,      /* bad argument or configuration */
  DVNR_E_UNSUPPORTED = 2,  /* valid but not compiled / not implemented for this shape */
  DVNR_E_HIP = 3,          /* a HIP runtime call failed */
  DVNR_E_STATE = 4,        /* call made in the wrong order (e.g. before dvnr_bind) */
  DVNR_E_NONFINITE = 5     /* a non-finite training loss was observed */
};

typedef struct dvnr dvnr_t; /* opaque handle */

/* Multiresolution grid (Sec. III, encoding of the cited instant neural
 * graphics primitives).  R_l = floor(base_resolution * b^l + 1e-6) vertices
 * per axis, b = per_level_scale if > 0, else
 * (finest_resolution / base_resolution)^(1/(n_levels-1)).  A level with
 * R_l^3 <= 2^log2_table_size is stored densely, otherwise hashed. */
typedef struct dvnr_encoding {
  int32_t n_levels;          /* L, 1..16 */
  int32_t n_features;        /* F, 1, 2, 4 or 8; L*F <= 32 */
  int32_t log2_table_size;   /* log2 T, 4..24 */
  int32_t base_resolution;   /* R_0 >= 2 */
  double per_level_scale;    /* b, or 0 to derive it from finest_resolution */
  int32_t finest_resolution; /* used when per_level_scale == 0 */
} dvnr_encoding;

/* Bias-free MLP with ReLU after every hidden layer, linear output (Sec. III). */
typedef struct dvnr_mlp {
  int32_t n_hidden_layers; /* 1..4 */
  int32_t width;           /* 16, 32 or 64 */
  int32_t out_dim;         /* must be 1 (scalar fields) */
} dvnr_mlp;

/* Adam with L2 weight decay added to the gradient and an optional exponential
 * learning-rate decay (Sec. III-F): update t (t = 1, 2, ... since the last
 * optimizer reset) uses lr * lr_decay_base^(max(0, t - lr_decay_start) /
 * lr_decay_interval); lr_decay_interval <= 0 keeps lr constant (the default
 * when the fields are zero). */
typedef struct dvnr_optim {
  double lr, beta1, beta2, eps, weight_decay;
  double lr_decay_base;       /* (0, 1] when lr_decay_interval > 0 */
  int64_t lr_decay_start;     /* >= 0 */
  int64_t lr_decay_interval;  /* <= 0: no decay */
} dvnr_optim;

typedef enum dvnr_precision {
  DVNR_FP32 = 0,       /* plain: fp32 tables and MLP, one thread per sample, plain atomics */
  DVNR_MIXED_BF16 = 1, /* fp16 tables + bf16 MFMA MLP (fp32 accumulation), fp32 masters */
  DVNR_FP64 = 2        /* fp64 everywhere; building blocks for gradient checking */
} dvnr_precision;

/* One block: owned voxels per axis (x, y, z) and the width of the halo of
 * ghost voxels stored around them (Sec. III-C). */
typedef struct dvnr_block {
  int32_t dims[3];
  int32_t ghost;
} dvnr_block;

typedef struct dvnr_sizes {
  int64_t n_levels;
  int64_t n_entries;        /* table entries per block */
  int64_t n_table_params;   /* n_entries * F */
  int64_t n_mlp_params;
  int64_t block_stride;     /* elements between consecutive blocks (>= table + mlp, multiple of 64) */
  int64_t n_params;         /* n_blocks * block_stride */
  int64_t param_bytes;      /* bytes of one parameter-sized buffer: 4 (fp32) or 8 (fp64) per element */
  int64_t work16_bytes;     /* mixed precision 16-bit working copy (0 otherwise) */
  int64_t workspace_bytes;  /* scratch for up to max_batch samples per step */
} dvnr_sizes;

typedef struct dvnr_buffers {
  void* params;             /* device, master parameters (fp32; fp64 for DVNR_FP64) */
  void* grads;              /* device, same type and size */
  void* adam_m;             /* device, same type and size */
  void* adam_v;             /* device, same type and size */
  void* work16;             /* device, mixed only: fp16 table / bf16 MLP copies, 2 B per element */
  void* workspace;          /* device, workspace_bytes */
  const float* const* volumes; /* host array of n_blocks device pointers: each block's voxels,
                                  float32 [nz+2g][ny+2g][nx+2g] (x fastest), read-only, zero-copy */
} dvnr_buffers;

/* Create a handle for n_blocks INRs sharing one configuration: one model per
 * box-shaped partition, each trained only on its own partition's voxels and
 * its ghost layer (Sec. III-A model parallelism; the INR of Eq. (1) is the
 * encoding + MLP above).  blocks: host array of n_blocks geometries.
 * max_batch: the largest total number of training samples per step (all
 * blocks together) and the largest chunk used by decode/sample.
 * seed: key of the Philox sample draws.  *out receives the handle (owned by
 * the caller, released with dvnr_destroy).  Returns DVNR_E_INVALID for
 * out-of-range settings.  Allocates host memory only. */
dvnr_status dvnr_create(const dvnr_encoding* enc, const dvnr_mlp* mlp, const dvnr_optim* opt,
                        dvnr_precision precision, int32_t n_blocks, const dvnr_block* blocks,
                        int64_t max_batch, uint64_t seed, dvnr_t** out);
void dvnr_destroy(dvnr_t* h);
const char* dvnr_last_error(void);

dvnr_status dvnr_get_sizes(const dvnr_t* h, dvnr_sizes* out);
/* Host copy of the level table: R[l], dense[l] (0/1), entry offset off[l], entries E[l].
 * Each array has n_levels elements; any pointer may be NULL. */
dvnr_status dvnr_level_info(const dvnr_t* h, int32_t* R, int32_t* dense, int64_t* off, int64_t* E);

/* Bind caller-owned buffers (see dvnr_buffers).  Rebinding is allowed. */
dvnr_status dvnr_bind(dvnr_t* h, const dvnr_buffers* b);

/* Per-block value range over every stored voxel, ghosts included (Sec. III-A
 * output normalization).  Must run once after dvnr_bind and before training,
 * sampling or decoding; enqueued on `stream`. */
dvnr_status dvnr_prepare(dvnr_t* h, void* stream);
/* Host copy of the per-block ranges computed by dvnr_prepare (synchronizes the stream). */
dvnr_status dvnr_get_ranges(dvnr_t* h, float* vmin, float* vmax, void* stream);

/* Initialize masters (the paper does not state an initialization; this is the
 * reading of the cited hash encoding's: tables U(-1e-4, 1e-4), weights
 * Glorot-uniform), drawn with Philox4x32-10 from `seed`; clears gradients and
 * the optimizer state (Sec. III-F Adam).  Needs dvnr_bind; DVNR_E_STATE
 * before it. */
dvnr_status dvnr_init_params(dvnr_t* h, uint64_t seed, void* stream);
/* After the caller overwrote the master parameters: refresh the 16-bit copy
 * (mixed precision; no-op otherwise) and clear gradients. */
dvnr_status dvnr_params_updated(dvnr_t* h, void* stream);
/* Warm start (Sec. III-E weight caching): keep the parameters, zero the Adam
 * moments and the step counter. */
dvnr_status dvnr_reset_optimizer(dvnr_t* h, void* stream);

/* n_steps optimizer steps (Sec. III-B: per iteration, stochastic uniform
 * samples, trilinear ground truth, one optimization step; Sec. III-F Adam).
 * Each step draws samples_per_step coordinates
 * split over blocks in proportion to owned voxel counts (largest remainder
 * in units of 256).  Of a block's n samples, the first n - nb are uniform,
 * Philox4x32-10 counter (sample, step, block, 'DVNR') and key (seed lo,
 * seed hi); the last nb = floor(boundary_frac * n + 1/2) are boundary-centered
 * (dvnr_set_loss; nb = 0 by default).  Then forward, the loss (mean per block;
 * L2 by default), backward and Adam; a block that draws no sample in a step
 * is left unchanged by that step.  loss_out: device float
 * [n_steps][n_blocks] or NULL.  samples_per_step <= max_batch. */
dvnr_status dvnr_train_steps(dvnr_t* h, int32_t n_steps, int64_t samples_per_step, float* loss_out,
                             void* stream);
/* Training length (Sec. III-B).  Block b trains at most
 *   N_max(b) = max(min_steps, ceil(N_vox(b) / n_b) * epochs)
 * steps (N_vox = owned voxels, n_b = its samples per step), and stops earlier
 * when loss_threshold > 0 and, at a multiple of check_every steps with at
 * least `window` steps done, the plain mean of its last `window` losses is
 * below loss_threshold (min_steps bounds only N_max). */
typedef struct dvnr_stop_policy {
  int64_t min_steps;      /* N_train^min, >= 0 */
  int64_t epochs;         /* N_epoch, >= 0 */
  double loss_threshold;  /* <= 0 disables the loss criterion */
  int32_t window;         /* 1 .. 1024 */
  int32_t check_every;    /* >= 1 */
} dvnr_stop_policy;

/* Train every block under `policy` with samples_per_step split as in
 * dvnr_train_steps; blocks stop independently: a stopped block draws no
 * samples and its parameters and Adam state stay unchanged while the others
 * continue (the step counter is shared).  steps_out: host int64[n_blocks],
 * steps each block trained; avg_loss_out: host double[n_blocks] or NULL, the
 * moving average at the block's last check (NaN if none).  Synchronizes
 * `stream`; the moving average is read back from the device every
 * check_every steps. */
dvnr_status dvnr_train_until(dvnr_t* h, const dvnr_stop_policy* policy, int64_t samples_per_step,
                             int64_t* steps_out, double* avg_loss_out, void* stream);

/* One optimizer step on caller-given coordinates: coords device float
 * [sum_b n_b][3] grouped by block, n_per_block host int64[n_blocks].
 * loss_out: device float [n_blocks] or NULL. */
dvnr_status dvnr_train_step_coords(dvnr_t* h, const float* coords, const int64_t* n_per_block,
                                   float* loss_out, void* stream);

/* Training samples of one block at step `step` as dvnr_train_steps draws
 * them: coords device float [n][3], target device float [n] (normalized). */
dvnr_status dvnr_draw_training_samples(dvnr_t* h, int32_t block, int64_t step, int64_t n, float* coords,
                                       float* target, void* stream);

/* On-demand inference (Sec. III and Sec. IV-A: the model is queried at any
 * coordinate): out[i] = INR_b(coords[i]) de-normalized with the block range
 * (Sec. III-A output normalization).  coords device float [n][3] in the
 * block's [0,1]^3 (clamped), out device float [n]; chunks of max_batch. */
dvnr_status dvnr_sample(dvnr_t* h, int32_t block, int64_t n, const float* coords, float* out, void* stream);
/* Decode back to the grid (Sec. III and Sec. IV-A): block b's owned voxels at
 * voxel centers (i+1/2)/n, out device float [nz][ny][nx] (x fastest),
 * de-normalized with the block range; block -1 decodes every block, one
 * after the other, into consecutive grids. */
dvnr_status dvnr_decode(dvnr_t* h, int32_t block, float* out, void* stream);
/* Direct volume rendering of one block's INR (Sec. IV, sample streaming).
 * Rays of a pinhole camera, in the block's unit-cube coordinates, march front
 * to back with step `step`: sample k of a ray sits at t_k = t0 + (k + 1/2) step
 * from the eye, for every t_k before the ray leaves the cube ([t0, t1] is the
 * ray's intersection with the cube, t0 >= 0).  A sample's de-normalized INR
 * value v maps through the piecewise-linear transfer function tf (device float
 * [n_tf][4] RGBA at n_tf equally spaced values over [tf_lo, tf_hi], v
 * clamped); its opacity a, given for the length ref_step, becomes
 * alpha = 1 - (1 - a)^(step / ref_step); then C += (1 - A) alpha rgb and
 * A += (1 - A) alpha.  A ray stops after the sample that brings A to
 * alpha_stop or above (1 disables early termination).
 * Rays advance samples_per_round samples per round: coordinate generation,
 * INR inference over the batch, shading (chunks of max_batch samples).
 * Camera: pixel (i, j), row 0 at the top, looks along
 * normalize(f + px r + py u) with f = normalize(center - eye),
 * r = normalize(f x up), u = r x f, px = (2 (i + 1/2) / width - 1) tan(fovy/2)
 * width / height, py = (1 - 2 (j + 1/2) / height) tan(fovy/2), all in float32
 * round-to-nearest in that order (the sample count of a ray is decided by
 * them).  image: device float [height][width][4], premultiplied (C, A).
 * workspace: device, 256-byte aligned, dvnr_render_workspace_bytes bytes.
 * samples_out (host, may be NULL): samples generated and inferred, the
 * rounds' active rays times samples_per_round.  Synchronizes `stream`. */
typedef struct dvnr_camera {
  float eye[3], center[3], up[3];
  float fovy_deg;        /* (0, 180) */
  int32_t width, height; /* width * height <= 2^28 */
} dvnr_camera;

typedef struct dvnr_render_params {
  float step;             /* > 0, unit-cube units */
  float ref_step;         /* > 0, length the transfer-function opacity refers to */
  float alpha_stop;       /* (0, 1] */
  float tf_lo, tf_hi;     /* tf_hi > tf_lo */
  int32_t n_tf;           /* >= 2 */
  int32_t samples_per_round; /* 1 .. max_batch */
} dvnr_render_params;

dvnr_status dvnr_render_workspace_bytes(const dvnr_t* h, int32_t width, int32_t height, int64_t* bytes);
dvnr_status dvnr_render(dvnr_t* h, int32_t block, const dvnr_camera* cam, const dvnr_render_params* params,
                        const float* tf, void* workspace, float* image, int64_t* samples_out, void* stream);

/* dvnr_render for callers that cannot allocate device memory (code under
 * stream or graph capture, serving loops, harnesses that forbid hipMalloc):
 * the same renderer and the same image, but the per-ray state (the
 * `workspace` of dvnr_render) lives in one static device array of the library,
 * one copy per GPU, sized for at most DVNR_RENDER_STATIC_MAX_RAYS pixels
 * (width * height; 28 MiB of device memory per GPU the library runs on, held
 * until the process ends).  Larger images: DVNR_E_INVALID, nothing enqueued.
 * Calls no allocator.  The first call on a device looks up that device's copy
 * (the current device) and may return DVNR_E_HIP if that fails.  Every call on
 * one GPU, from any handle or thread, shares that GPU's array and the array
 * keeps the last call's contents; calls that overlap on one GPU (different
 * streams or threads) race and must be serialized by the caller.  The
 * handle's own bound workspace carries the sample batches, as in
 * dvnr_render.  Synchronizes `stream`. */
#define DVNR_RENDER_STATIC_MAX_RAYS (1 << 20)
dvnr_status dvnr_render_static(dvnr_t* h, int32_t block, const dvnr_camera* cam, const dvnr_render_params* params,
                               const float* tf, float* image, int64_t* samples_out, void* stream);

/* Sliding-window model cache (Sec. III-E weight caching; Sec. IV temporal
 * caching): snapshots of the trained models of past timesteps, kept on the
 * device so that any cached timestep can be decoded or sampled on demand.
 * A snapshot holds the inference parameters of every block (fp16 tables and
 * bf16 weights for mixed precision, fp32 otherwise) and the blocks' value
 * ranges at push time; decoding it runs the same kernels as dvnr_decode.
 *
 * dvnr_cache_snapshot_bytes : bytes of one snapshot (*bytes).
 * dvnr_cache_bind           : caller-owned device buffer of capacity snapshots
 *                             (256-byte aligned, capacity * snapshot bytes);
 *                             clears the cache.  capacity 0 unbinds.
 * dvnr_cache_push           : snapshot the current model under `key` (e.g. the
 *                             timestep), stream-ordered after earlier work;
 *                             when full, the oldest snapshot is dropped.
 *                             DVNR_E_INVALID if `key` is already cached.
 * dvnr_cache_keys           : cached keys, oldest first (host int64[capacity],
 *                             may be NULL), and their count.
 * dvnr_cache_decode / _sample : as dvnr_decode / dvnr_sample on the snapshot
 *                             of `key`; DVNR_E_INVALID if it is not cached.
 * Block geometry is the handle's; the volumes need not be bound any more. */
dvnr_status dvnr_cache_snapshot_bytes(const dvnr_t* h, int64_t* bytes);
dvnr_status dvnr_cache_bind(dvnr_t* h, int32_t capacity, void* buffer);
dvnr_status dvnr_cache_push(dvnr_t* h, int64_t key, void* stream);
dvnr_status dvnr_cache_keys(const dvnr_t* h, int64_t* keys, int32_t* count);
dvnr_status dvnr_cache_decode(dvnr_t* h, int64_t key, int32_t block, float* out, void* stream);
dvnr_status dvnr_cache_sample(dvnr_t* h, int64_t key, int32_t block, int64_t n, const float* coords, float* out,
                              void* stream);

/* Reconstruction error for the PSNR (Sec. V-B: PSNR from the mean squared
 * error over all partitions, data normalized to [0,1]): sum of squared
 * differences, accumulated in fp64 (the only fp64 arithmetic of the fp32 and
 * mixed paths), between a decoded block (device float [nz][ny][nx]) and the
 * block's owned stored voxels: host *sse, *count (owned voxels).  Summing
 * sse and count over blocks gives the voxel-weighted global MSE.
 * Synchronizes `stream`. */
dvnr_status dvnr_mse_fp64(dvnr_t* h, int32_t block, const float* decoded, double* sse, int64_t* count,
                          void* stream);

/* Autograd building blocks of block `block` (the two halves of Eq. (1)'s
 * model, Sec. III: the multiresolution hash encoding and the ReLU MLP, with
 * their hand-written backward).  Element type is double for a DVNR_FP64
 * handle, float otherwise.  All pointers are device pointers.
 *  encode_forward : coords float [n][3] -> feats [n][L*F] (sample-major) from
 *                   the level tables `table` [n_table_params]
 *  encode_backward: dtable [n_table_params] += d(feats)/d(table)^T dfeats
 *  mlp_forward    : feats [n][L*F] -> out [n] (normalized INR output) with
 *                   `weights` [n_mlp_params] (W_1 .. W_out, row-major)
 *  mlp_backward   : given dout [n]: dfeats [n][L*F] (overwritten), dweights
 *                   [n_mlp_params] (accumulated); recomputes the forward.
 * A NULL table / weights stands for block `block`'s bound master parameters,
 * a NULL dtable / dweights for its bound gradient (so that dvnr_adam_step can
 * apply them); NULL needs dvnr_bind (DVNR_E_STATE otherwise).  DVNR_E_INVALID
 * for block outside [0, n_blocks) or n outside [0, 2^31). */
dvnr_status dvnr_encode_forward(dvnr_t* h, int32_t block, int64_t n, const float* coords, const void* table,
                                void* feats, void* stream);
dvnr_status dvnr_encode_backward(dvnr_t* h, int32_t block, int64_t n, const float* coords, const void* dfeats,
                                 void* dtable, void* stream);
dvnr_status dvnr_mlp_forward(dvnr_t* h, int32_t block, int64_t n, const void* feats, const void* weights, void* out,
                             void* stream);
dvnr_status dvnr_mlp_backward(dvnr_t* h, int32_t block, int64_t n, const void* feats, const void* weights,
                              const void* dout, void* dfeats, void* dweights, void* stream);
/* One Adam update (Sec. III-F: beta1 0.9, beta2 0.999, eps 1e-8, L2 weight
 * decay added to the gradient, exponential learning-rate decay as in
 * dvnr_optim) of every parameter of every block from the bound gradient
 * buffer, e.g. filled by the building blocks above: advances the shared step
 * counter t, refreshes the 16-bit working copy (mixed precision) and leaves
 * the gradient at zero.  Arithmetic in the handle's precision.  Needs
 * dvnr_bind (DVNR_E_STATE otherwise); only enqueues on `stream`. */
dvnr_status dvnr_adam_step(dvnr_t* h, void* stream);

/* Parity/debug: corner entry indices (within level `level`) and trilinear
 * weights of n coordinates: idx device uint32 [n][8], w device float [n][8]. */
dvnr_status dvnr_debug_indices(dvnr_t* h, int32_t level, int64_t n, const float* coords, uint32_t* idx, float* w,
                               void* stream);

/* Per-phase device time in milliseconds, summed over the training steps run
 * with the "profile_phases" option since the previous call (those steps run
 * eagerly, with HIP events on the training stream between the phases):
 * ms[0] sampler, [1] encoding forward, [2] MLP forward/loss/backward,
 * [3] encoding backward of the bin-privatized levels, [4] encoding backward
 * by direct atomics, [5] and [6] the two passes of the destination-partitioned
 * encoding backward (bucketing, slice sums), [7] weight-gradient reduction,
 * [8] Adam; `ms` holds DVNR_N_PHASES doubles.  *n_steps (may be NULL)
 * receives the number of steps covered.  Waits for those steps to finish;
 * resets the sums. */
#define DVNR_N_PHASES 9
dvnr_status dvnr_phase_times(dvnr_t* h, double* ms, int64_t* n_steps);

/* Autotuner: time the candidate step configurations (unordered or spatially
 * ordered sampling, the number of bin-privatized coarse levels, the number of
 * workgroups of the persistent MLP kernel) on n_trial_steps gradient-only
 * steps of samples_per_step samples each, and keep the fastest for later
 * dvnr_train_steps calls with that sample count.  Parameters and optimizer
 * state are unchanged: trial steps apply no update, their gradients are
 * cleared and the step counter is restored.  Synchronizes `stream`.
 * *best_ms (may be NULL) receives the chosen configuration's time per step
 * without the Adam update. */
dvnr_status dvnr_autotune(dvnr_t* h, int64_t samples_per_step, int32_t n_trial_steps, double* best_ms,
                          void* stream);

/* Layout of the current training plan (the last samples_per_step given to
 * dvnr_train_steps): spatial bins per axis of the ordered sampler and the
 * number of coarse levels whose encoding backward is bin-privatized (levels
 * [0, *priv_levels)); 0 when ordered sampling is off.  Any pointer may be NULL. */
dvnr_status dvnr_plan_info(const dvnr_t* h, int32_t* bins_per_axis, int32_t* priv_levels);

/* First level of the current training plan whose encoding backward is
 * destination-partitioned (levels [*first_level, n_levels)); n_levels when
 * none is.  See the "scatter_part" option. */
dvnr_status dvnr_plan_partition(const dvnr_t* h, int32_t* first_level);

/* Wait for `stream`; reports HIP errors and a non-finite loss seen since the
 * last dvnr_sync (DVNR_E_NONFINITE). */
dvnr_status dvnr_sync(dvnr_t* h, void* stream);

/* Loss and sampling distribution of training (Sec. III-C, Eqs. (2)-(3)).
 *  loss          : DVNR_LOSS_L2 (mean squared error, the default) or
 *                  DVNR_LOSS_L1 (mean absolute error, dL/do = sign(o - y)/n
 *                  with sign(0) = 0).
 *  boundary_frac : lambda in [0, 1], the share of each block's samples drawn
 *                  near the block faces (0 by default; the paper uses 0.15
 *                  with the L1 loss).  The total per step is unchanged.
 *  sigma         : spread in (0, 1] of the boundary samples (paper: 0.005).
 *                  A boundary sample, Philox counter (sample, step, block,
 *                  'DVNB'), output words u0..u3: face = floor(6 u3 / 2^32)
 *                  (axis face/2, low side if face is even); distance to the
 *                  face sigma sqrt(2) erfinv((u2 >> 8) 2^-24) (a half-normal
 *                  quantile), clipped to 1; the two other coordinates, in
 *                  increasing axis order, (u0 >> 8) 2^-24 and (u1 >> 8) 2^-24.
 * Takes effect at the next training call.  DVNR_E_INVALID for values out of
 * range. */
#define DVNR_LOSS_L2 0
#define DVNR_LOSS_L1 1
dvnr_status dvnr_set_loss(dvnr_t* h, int32_t loss, double boundary_frac, double sigma);

/* Options (runtime switches):
 *  "scatter_grouped" 0/1 : grouped-lane scatter (default 1 for mixed, 0 for fp32)
 *  "use_graph"       0/1 : capture one step in a hipGraph and replay it on a
 *                          non-default stream (default 1)
 *  "xcd_map"         0/1 : XCD-aware level-to-workgroup mapping (default 1)
 *  "apply_update"    0/1 : run the Adam update after the backward (default 1).
 *                          With 0 a step leaves this step's gradient in `grads`
 *                          (parity checks of the backward).
 *  "profile_phases"  0/1 : record HIP events between the phases of every
 *                          training step (steps then run without a graph);
 *                          read with dvnr_phase_times().
 *  "spatial_sort"    0/1 : store each step's samples grouped by spatial bin
 *                          (default 1 for mixed, 0 for fp32); enables the
 *                          bin-privatized backward of the coarse levels
 *  "priv_levels"     n   : privatize levels [0, n) (-1: chosen per plan)
 *  "sample_ahead"  0..3 : with ordered sampling and graph replays, draw step
 *                          i + 1's samples on a third stream while step i
 *                          trains (two sample sets), forked at the start of
 *                          step i (1), after its encoding (2, the default)
 *                          or after its MLP (3); 0: off.  The first step of
 *                          each training call draws its own.
 *  "sort_bins"       n   : spatial bins per axis of ordered sampling, 1..8
 *                          (0, the default: the most that keep at least 192
 *                          samples per bin in the block with the fewest)
 *  "scatter_concurrent" 0/1 : run the privatized levels whose bin boxes never
 *                          fit LDS (direct atomics) on a second stream,
 *                          concurrently with the others (default 0)
 *  "encode_binned"   0/1 : with ordered sampling, interpolate the coarse levels
 *                          (bin box within 16 KB and at most half the bin's
 *                          direct gathers) from LDS-staged boxes (default 0:
 *                          the tile encoding, two levels per workgroup, is
 *                          faster on every level)
 *  "priv_classes"  -1/0/1 : launch the privatized levels in three LDS-size
 *                          classes (small boxes, large boxes, direct) instead
 *                          of one launch (-1, the default: by class when the
 *                          destination-partitioned backward takes the fine
 *                          levels of a single block, one launch otherwise)
 *  "scatter_strided" 0/1 : direct backward over ordered samples takes each
 *                          tile's samples strided across the block (default 1)
 *  "decode_fused"    0/1 : decode with the fused brick kernel (default 1)
 *  "mlp_waves"       1/2 : register budget of the 4-wave mixed-precision MLP
 *                          training kernel, in waves per SIMD (default 1)
 *  "mlp_wg_waves"    4/8 : waves per workgroup of the mixed-precision MLP
 *                          training kernel (8: two waves per SIMD, used where
 *                          its LDS fits, else 4; default 8)
 *  "mlp_grid"        n   : workgroups of the persistent MLP training kernel
 *                          (1 .. 512, default 256; also set by dvnr_autotune)
 *  "scatter_part"    n   : destination-partitioned encoding backward of the
 *                          levels [n, n_levels) (-1, the default: for mixed
 *                          precision, the longest suffix of levels with at
 *                          least 2^15 entries that, unless "part_adam" is
 *                          off, get at least one contribution per table
 *                          entry per step; none for fp32; >= n_levels:
 *                          none).  Each step sorts the levels'
 *                          (sample, corner) contributions into per-slice
 *                          buckets (slices of "part_slice" / F entries) and sums
 *                          each bucket in LDS, instead of one global atomic per
 *                          contribution.  Levels with more than 256 slices stay
 *                          on the atomic paths, and so do levels with fewer
 *                          than 2^12 entries (the workspace holds buckets
 *                          for the others: about 40 (1 + F) bytes per
 *                          sample of max_batch and level).
 *  "part_slice"      n   : fp32 accumulators per slice: 4096, 8192 (default)
 *                          or 16384
 *  "encode_concurrent" 0/1 : run the binned encoding of the coarse levels on
 *                          a second stream concurrently with the tile encoding
 *                          of the others (default 1)
 *  "part_concurrent" 0/1 : run the two partitioned passes on a second stream
 *                          (default priority), forked and joined with events
 *                          inside the step, concurrently with the bin-privatized
 *                          levels (default 1)
 *  "part_capacity"   n   : cap every bucket at n records (0, the default: 1.25x
 *                          the mean load plus 32); records beyond a bucket's
 *                          capacity are added by direct atomics (tests)
 * Returns DVNR_E_INVALID for an unknown name. */
dvnr_status dvnr_set_option(dvnr_t* h, const char* name, int64_t value);

#ifdef __cplusplus
}
#endif
#endif /* DVNR_H */
