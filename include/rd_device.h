/*
 * rd_device.h -- recording a HIP kernel's events on the device, straight into a trace that
 * rd_trace_upload(events_on_device = 1) binds: the paper's instrumentation layer (Section 5, the
 * NVBit tool that logs every memory and synchronisation event of a kernel) without its host channel.
 *
 * The kernel under test calls these functions around its own operations.  Each call appends one
 * record per calling lane: the lanes of a wavefront that call together take one ticket range with a
 * single atomic add and write their records contiguously (coalesced 16-byte stores), so the buffer
 * order is a global order of the calls that respects every lane's program order.  Records follow
 * include/rd.h: tid = block * threads_per_block + thread (blocks and threads flattened x-major),
 * the grid of the trace is (total blocks, threads per block).
 *
 * Where a call goes relative to the operation it records, so that the trace order is one the
 * execution allows (the ordering the checker's release -> acquire edges need):
 *   - writes, atomics that publish (a flag store, a lock release) and barriers: record first, then
 *     perform (rd_syncthreads records and then synchronises);
 *   - reads, atomics that observe (a flag load, a successful lock acquire): perform first, then
 *     record;
 *   - fences: record in program order between the accesses they separate (a fence orders nothing by
 *     itself; an atomic right after a fence is a release, right before one an acquire).
 * The buffer holds `capacity` records; calls past it count but write nothing (rd_dev_log::count
 * then exceeds capacity and the trace is incomplete: the caller checks it).  Warp barriers are not
 * recorded: a wavefront of gfx950 has 64 lanes and the record format's lane masks hold 32.
 *
 * Header-only device code; include it in the HIP source of the kernel under test.
 */
#ifndef RD_DEVICE_H
#define RD_DEVICE_H

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rd.h"

typedef struct {
    rd_event *ev;                /* device buffer of `capacity` records */
    unsigned long long *count;   /* device counter, zero before the kernel */
    unsigned long long capacity;
    const void *gbase;           /* global words are numbered from here: (p - gbase) / 4, which must
                                    stay below 2^32 (keep the recorded data within 16 GiB of it) */
} rd_dev_log;

/* The calling thread's trace id: its block (flattened) times threads per block plus its thread. */
__device__ inline uint32_t rd_dev_tid() {
    const uint32_t blk = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    const uint32_t thr = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    return blk * (blockDim.x * blockDim.y * blockDim.z) + thr;
}

/* One record per calling lane (kind, scope and space as in include/rd.h; `site` goes to aux). */
__device__ inline void rd_dev_record(rd_dev_log L, uint32_t kind, uint32_t scope, uint32_t space, uint32_t addr,
                                     uint32_t site) {
    const uint64_t active = __ballot(1);
    const uint32_t lane = __lane_id();
    const uint32_t leader = (uint32_t)__builtin_ctzll(active);
    const uint32_t rank = (uint32_t)__popcll(active & ((1ull << lane) - 1ull));
    unsigned long long base = 0;
    if (lane == leader) base = atomicAdd(L.count, (unsigned long long)__popcll(active));
    base = __shfl(base, (int)leader, 64);
    const unsigned long long slot = base + rank;
    if (slot < L.capacity) {
        rd_event e;
        e.addr = addr;
        e.tid = rd_dev_tid();
        e.meta = (kind & 15u) | ((scope & 3u) << 4) | ((space & 1u) << 6);
        e.aux = site;
        L.ev[slot] = e;
    }
}

/* Word index of a global address (4-byte words from L.gbase) and of a shared-memory address (its
 * word offset in the block's LDS: shared words are numbered per block). */
__device__ inline uint32_t rd_dev_gword(rd_dev_log L, const void *p) {
    return (uint32_t)(((uintptr_t)p - (uintptr_t)L.gbase) >> 2);
}
__device__ inline uint32_t rd_dev_sword(const void *p) {
    return (uint32_t)(((uintptr_t)p & 0xffffffffu) >> 2);
}

__device__ inline void rd_dev_read(rd_dev_log L, const void *p, uint32_t site) {
    rd_dev_record(L, RD_READ, RD_BLOCK, RD_GLOBAL, rd_dev_gword(L, p), site);
}
__device__ inline void rd_dev_write(rd_dev_log L, const void *p, uint32_t site) {
    rd_dev_record(L, RD_WRITE, RD_BLOCK, RD_GLOBAL, rd_dev_gword(L, p), site);
}
__device__ inline void rd_dev_read_shared(rd_dev_log L, const void *p, uint32_t site) {
    rd_dev_record(L, RD_READ, RD_BLOCK, RD_SHARED, rd_dev_sword(p), site);
}
__device__ inline void rd_dev_write_shared(rd_dev_log L, const void *p, uint32_t site) {
    rd_dev_record(L, RD_WRITE, RD_BLOCK, RD_SHARED, rd_dev_sword(p), site);
}
__device__ inline void rd_dev_atomic(rd_dev_log L, const void *p, uint32_t scope, uint32_t site) {
    rd_dev_record(L, RD_ATOMIC, scope, RD_GLOBAL, rd_dev_gword(L, p), site);
}
__device__ inline void rd_dev_fence(rd_dev_log L, uint32_t scope) { rd_dev_record(L, RD_FENCE, scope, RD_GLOBAL, 0, 0); }
__device__ inline void rd_dev_acquire(rd_dev_log L, const void *lock, uint32_t scope, uint32_t site) {
    rd_dev_record(L, RD_ACQ, scope, RD_GLOBAL, rd_dev_gword(L, lock), site);
}
__device__ inline void rd_dev_release(rd_dev_log L, const void *lock, uint32_t scope, uint32_t site) {
    rd_dev_record(L, RD_REL, scope, RD_GLOBAL, rd_dev_gword(L, lock), site);
}

/* A block barrier recorded by every thread that reaches it, then the barrier itself. */
__device__ inline void rd_syncthreads(rd_dev_log L) {
    rd_dev_record(L, RD_BAR, RD_BLOCK, RD_GLOBAL, 0, 0);
    __syncthreads();
}

#endif /* RD_DEVICE_H */
