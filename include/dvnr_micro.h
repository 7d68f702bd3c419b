/*
 * dvnr_micro.h -- measurement kernels of libdvnr.so (not part of the method).
 *
 * The training step's phases are bound by different memory-system rates:
 * Adam and the record passes stream through HBM, the encoding gathers 4-byte
 * table entries at random, the encoding backward adds fp32 values at random
 * (hardware float atomics), and the MLP runs on the matrix cores.  The vendor
 * peaks (8 TB/s HBM, 2.5 PFLOP/s dense bf16) bound only the first and the
 * last; these kernels measure what the chip attains for each pattern, at a
 * given footprint, so that a phase's fraction can be stated against the rate
 * its own access pattern allows.  bench.py times them with events on the
 * stream it passes.
 *
 * All pointers are device pointers (caller-allocated); every call only
 * enqueues on `stream` (NULL = default stream).  Return value: 0 on success,
 * 1 for an invalid argument (nothing enqueued), 3 if the launch failed.
 */
#ifndef DVNR_MICRO_H
#define DVNR_MICRO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* dst[0 .. bytes) = src[0 .. bytes): 16-byte loads and stores, grid-stride;
 * nontemporal != 0 uses non-temporal loads and stores (as the Adam kernels
 * do).  bytes a positive multiple of 16, both pointers 16-byte aligned;
 * the ranges must not overlap.  Moves 2 * bytes through HBM. */
int32_t dvnr_micro_copy(const void* src, void* dst, int64_t bytes, int32_t nontemporal, void* stream);

/* n_threads * per_thread random 4-byte loads from table [n_entries]
 * (n_entries a power of two <= 2^32): lookup k of thread i reads
 * table[fmix32((i * per_thread + k) ^ seed) & (n_entries - 1)] (MurmurHash3's
 * finalizer), eight loads in flight per thread; out [n_threads] receives each
 * thread's sum.  n_threads a positive multiple of 256, per_thread a positive
 * multiple of 8. */
int32_t dvnr_micro_gather(const uint32_t* table, int64_t n_entries, int64_t n_threads, int32_t per_thread,
                          uint32_t seed, uint32_t* out, void* stream);

/* n_threads * per_thread fp32 atomic adds of 1.0 (no return value) into
 * table [n_entries] (a power of two <= 2^32): `group` consecutive lanes
 * (a power of two <= 64 and <= n_entries) add to `group` consecutive elements
 * at a random group-aligned position, as a grouped-lane scatter does;
 * group = 1 is a fully scattered add.  n_threads a positive multiple of 256. */
int32_t dvnr_micro_atomic(float* table, int64_t n_entries, int64_t n_threads, int32_t per_thread, int32_t group,
                          uint32_t seed, void* stream);

/* Dense bf16 matrix-core rate: n_workgroups workgroups of 256 threads (4
 * waves), each wave issuing iters x 8 back-to-back 16x16x32 bf16 MFMAs with
 * fp32 accumulation (8 independent accumulators), 16384 flop each; out
 * [n_workgroups * 256] receives per-lane sums. */
int32_t dvnr_micro_mfma_bf16(int64_t n_workgroups, int32_t iters, float* out, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* DVNR_MICRO_H */
