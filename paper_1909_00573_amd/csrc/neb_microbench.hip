// Measurement kernels.  Device-scope atomic throughput on gfx950: the
// ceiling that the octree's lock-free counting (Sec. 5.1, 5.2:
// compare-and-swap increments of leaf counters) is measured against; and
// random-access read throughput, the ceiling of the photon merges' lookups
// (Sec. 3.2: the view vertices within r of each photon hit).
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

// Random-access read throughput: every thread reads `ops` records of
// `width` 16-byte words (1 or 4: 16 or 64 bytes, a record aligned to its
// size) at indices picked by a hash of (thread, k) among the n_words words
// of buf, eight reads in flight per thread, and writes the sum of what it
// read to sink[thread].  This is the access pattern of the photon merges'
// cell lookups, candidate runs and merge records, over a buffer the size of
// their working set.
__global__ void __launch_bounds__(256) k_gather_probe(const float4* __restrict__ buf, int64_t n_words, int32_t width,
                                                      int32_t ops, float* __restrict__ sink) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t n_rec = (uint64_t)n_words / (uint64_t)width;
    float acc = 0.f;
    for (int k0 = 0; k0 < ops; k0 += 8) {
        float4 v[8][4];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t h = mix32(tid * 0x9E3779B9u + (uint32_t)(k0 + u) * 0x85EBCA6Bu);
            const uint64_t rec = ((uint64_t)h * n_rec) >> 32;
            const float4* p = buf + rec * (uint64_t)width;
#pragma unroll
            for (int w = 0; w < 4; ++w) v[u][w] = (w < width && k0 + u < ops) ? p[w] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int w = 0; w < 4; ++w) acc += v[u][w].x + v[u][w].y + v[u][w].z + v[u][w].w;
    }
    sink[tid] = acc;
}

}  // namespace

extern "C" neb_status neb_gather_probe(const float* buf, int64_t n_words, int32_t width, int32_t blocks, int32_t ops,
                                       float* sink, void* stream) {
    if (!buf || !sink || n_words < 4 || (width != 1 && width != 4) || blocks < 1 || ops < 1)
        return NEB_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_gather_probe, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                       (const float4*)buf, n_words, width, ops, sink);
    return hipGetLastError() == hipSuccess ? NEB_OK : NEB_ERR_DEVICE;
}

extern "C" neb_status neb_atomic_probe(int32_t* words, int32_t n_words, int32_t stride, int32_t blocks, int32_t ops,
                                       int32_t kind, int32_t* sink, void* stream) {
    if (!words || !sink || n_words < 1 || stride < 1 || blocks < 1 || ops < 1 || (kind != 0 && kind != 1))
        return NEB_ERR_INVALID_ARG;
    if ((int64_t)n_words * stride > ((int64_t)1 << 31)) return NEB_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_atomic_probe, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, words, n_words,
                       stride, ops, kind, sink);
    return hipGetLastError() == hipSuccess ? NEB_OK : NEB_ERR_DEVICE;
}
