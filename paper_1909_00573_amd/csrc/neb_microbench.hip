// Device-scope atomic throughput on gfx950: the ceiling that the octree's
// lock-free counting (Sec. 5.1, 5.2: compare-and-swap increments of leaf
// counters) is measured against.
//
// Every thread performs `ops` increments of words picked by a hash of
// (thread, k) among n_words words spaced `stride` words apart.  kind 0:
// atomicAdd with the returned value used; kind 1: a compare-and-swap loop
// (load, then CAS old -> old + 1 until it succeeds), the octree's counting
// primitive.  Each thread folds the returned values into one word so that
// no atomic is dead code.
#include <hip/hip_runtime.h>

#include "neb.h"

namespace {

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7FEB352Du;
    x ^= x >> 15;
    x *= 0x846CA68Bu;
    x ^= x >> 16;
    return x;
}

__global__ void __launch_bounds__(256) k_atomic_probe(int32_t* __restrict__ words, int32_t n_words, int32_t stride,
                                                      int32_t ops, int32_t kind, int32_t* __restrict__ sink) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    int32_t acc = 0;
    for (int k = 0; k < ops; ++k) {
        const uint32_t w = mix32(tid * 0x9E3779B9u + (uint32_t)k) % (uint32_t)n_words;
        int32_t* p = words + (size_t)w * (size_t)stride;
        if (kind == 0) {
            acc += atomicAdd(p, 1);
        } else {
            int32_t old = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            for (;;) {
                int32_t seen = atomicCAS(p, old, old + 1);
                if (seen == old) break;
                old = seen;
            }
            acc += old;
        }
    }
    sink[tid] = acc;
}

}  // namespace

extern "C" neb_status neb_atomic_probe(int32_t* words, int32_t n_words, int32_t stride, int32_t blocks, int32_t ops,
                                       int32_t kind, int32_t* sink, void* stream) {
    if (!words || !sink || n_words < 1 || stride < 1 || blocks < 1 || ops < 1 || (kind != 0 && kind != 1))
        return NEB_ERR_INVALID_ARG;
    if ((int64_t)n_words * stride > ((int64_t)1 << 31)) return NEB_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_atomic_probe, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, words, n_words,
                       stride, ops, kind, sink);
    return hipGetLastError() == hipSuccess ? NEB_OK : NEB_ERR_DEVICE;
}
