// rd_demo.hip -- example kernels recorded with include/rd_device.h: what a user of the device-side
// producer writes around a kernel's own operations.  Built as librd_demo.so (not part of librd.so);
// the tests and the bench run them and check the traces they produce.
//
// Every global word the kernels touch lies in one caller buffer `mem` (the trace numbers global
// words from its start), laid out as: [0, n) input items, [n, n + B) published block values,
// [n + B, n + 2B) flags, then the accumulator and the lock word.  Waits on other blocks spin at most
// DEMO_SPIN times and then give up (the kernel sets mem's error word and returns), so every wave
// ends whatever the scheduler does.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rd_device.h"

namespace {

constexpr int DEMO_SPIN = 1 << 22;

struct DemoMem {
    int *in, *pub, *flag, *acc, *lock, *err;
};

__device__ inline DemoMem demo_mem(int *mem, int n, int nb) {
    DemoMem m;
    m.in = mem;
    m.pub = mem + n;
    m.flag = mem + n + nb;
    m.acc = mem + n + 2 * nb;
    m.lock = m.acc + 1;
    m.err = m.acc + 2;
    return m;
}

// Block sums in LDS by a tree of barriers, then thread 0 of every block adds its block's sum to one
// global accumulator inside a device-scoped critical section (a spin lock on `lock`).
//   plant & 1: the accumulator is updated without the lock (blocks race on it);
//   plant & 2: each thread also reads its right neighbour's LDS slot before the first barrier
//              (a race inside every block).
__global__ void k_demo_reduce(int *mem, int n, int plant, rd_dev_log L) {
    extern __shared__ int sh[];
    const int t = threadIdx.x, nt = blockDim.x, g = blockIdx.x * nt + t;
    const DemoMem m = demo_mem(mem, n, gridDim.x);
    const int v = m.in[g];
    rd_dev_read(L, &m.in[g], 1);
    rd_dev_write_shared(L, &sh[t], 2);
    sh[t] = v;
    if (plant & 2) {
        const int r = (t + 1) % nt;
        (void)*(volatile int *)&sh[r];
        rd_dev_read_shared(L, &sh[r], 3);
    }
    rd_syncthreads(L);
    for (int s = nt / 2; s > 0; s >>= 1) {
        if (t < s) {
            const int a = sh[t];
            rd_dev_read_shared(L, &sh[t], 4);
            const int b = sh[t + s];
            rd_dev_read_shared(L, &sh[t + s], 5);
            rd_dev_write_shared(L, &sh[t], 6);
            sh[t] = a + b;
        }
        rd_syncthreads(L);
    }
    if (t != 0) return;
    const int total = sh[0];
    rd_dev_read_shared(L, &sh[0], 7);
    const bool locked = !(plant & 1);
    if (locked) {
        int spin = 0;
        while (atomicCAS(m.lock, 0, 1) != 0) {
            if (++spin > DEMO_SPIN) {
                atomicOr(m.err, 1);
                return;
            }
        }
        __threadfence();
        rd_dev_acquire(L, m.lock, RD_DEVICE, 8);
    }
    const int a = *(volatile int *)m.acc;
    rd_dev_read(L, m.acc, 9);
    rd_dev_write(L, m.acc, 10);
    *(volatile int *)m.acc = a + total;
    if (locked) {
        rd_dev_release(L, m.lock, RD_DEVICE, 11);
        __threadfence();
        atomicExch(m.lock, 0);
    }
}

// A chain of publications: block b writes its value, then thread 0 fences and raises flag b (an
// atomic right after a fence: a release); block b + 1's thread 0 waits for flag b, then atomically
// reads it and fences (an atomic right before a fence: an acquire), a barrier hands that to the
// block, and its threads read block b's value.
//   plant & 1: block 0's release and block 1's acquire fence with block scope only (two blocks:
//              no edge, block 1 races with block 0's value);
//   plant & 2: block 1's threads read block 0's value before waiting.
__global__ void k_demo_chain(int *mem, int n, int plant, rd_dev_log L) {
    const int t = threadIdx.x, b = blockIdx.x;
    const DemoMem m = demo_mem(mem, n, gridDim.x);
    if (t == 0) {
        rd_dev_write(L, &m.pub[b], 20);
        *(volatile int *)&m.pub[b] = b + 1;
        const uint32_t scope = (b == 0 && (plant & 1)) ? RD_BLOCK : RD_DEVICE;
        rd_dev_fence(L, scope);
        __threadfence();
        rd_dev_atomic(L, &m.flag[b], RD_DEVICE, 21);
        __threadfence();
        atomicExch(&m.flag[b], 1);
    }
    if (b == 0) return;
    if (b == 1 && (plant & 2)) {
        (void)*(volatile int *)&m.pub[0];
        rd_dev_read(L, &m.pub[0], 22);
    }
    if (t == 0) {
        int spin = 0;
        while (atomicAdd(&m.flag[b - 1], 0) == 0) {
            if (++spin > DEMO_SPIN) {
                atomicOr(m.err, 2);
                break;
            }
        }
        __threadfence();
        rd_dev_atomic(L, &m.flag[b - 1], RD_DEVICE, 23);
        rd_dev_fence(L, (b == 1 && (plant & 1)) ? RD_BLOCK : RD_DEVICE);
    }
    rd_syncthreads(L);
    (void)*(volatile int *)&m.pub[b - 1];
    rd_dev_read(L, &m.pub[b - 1], 24);
}

}  // namespace

extern "C" {

// Words of `mem` the demos need for nb blocks of nt threads: n = nb * nt input items, nb published
// values, nb flags, the accumulator, the lock and an error word.
uint64_t rd_demo_mem_words(uint32_t nb, uint32_t nt) { return (uint64_t)nb * nt + 2ull * nb + 3; }

// Runs one demo (0: reduce, 1: chain) over nb blocks of nt threads (nt a power of two, <= 1024)
// on `stream`, recording into ev (capacity records) with the counter *count (device memory, both
// zeroed by the caller).  mem: rd_demo_mem_words() ints, the input items filled and the rest zero.
// Returns 0, or -1 for bad arguments.
int rd_demo_run(int demo, uint32_t nb, uint32_t nt, int plant, int *mem, rd_event *ev, uint64_t capacity,
                unsigned long long *count, hipStream_t stream) {
    if (!mem || !ev || !count || nb == 0 || nt == 0 || nt > 1024 || (nt & (nt - 1))) return -1;
    rd_dev_log L;
    L.ev = ev;
    L.count = count;
    L.capacity = capacity;
    L.gbase = mem;
    const int n = (int)(nb * nt);
    if (demo == 0) {
        hipLaunchKernelGGL(k_demo_reduce, dim3(nb), dim3(nt), nt * sizeof(int), stream, mem, n, plant, L);
    } else if (demo == 1) {
        hipLaunchKernelGGL(k_demo_chain, dim3(nb), dim3(nt), 0, stream, mem, n, plant, L);
    } else {
        return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // extern "C"
