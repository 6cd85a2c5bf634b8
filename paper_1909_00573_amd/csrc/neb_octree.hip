// Lock-free sparse density octree (Sec. 5 of the paper, class of Appendix B)
// on gfx950: device-scope atomics on an int32 node pool, compare-and-swap
// counting and splits allocated with one fetch-add.  No lane ever waits for
// another lane.
//
// Node word: >= 0 is a count (bit 30 marks a leaf whose split could not be
// allocated; it keeps counting), < 0 is minus the index of the first of 8
// consecutive children.
//
// Differences from the listing, and why:
//  - the listing lets a thread that finds a full leaf without a published
//    child pointer spin until the pointer appears.  On a 64-wide wavefront
//    the splitter may sit in the same wave as the spinner, and the
//    compiler places the split (which follows the loop-exiting CAS) after
//    the loop's reconvergence point: the wave deadlocks.  Here such a
//    deposit is deferred to a queue and retried by the next launch; the
//    kernel boundary guarantees the split has been published.  A deposit
//    is deferred at most once per level, so kOctMaxDepth + 1 retry rounds
//    bound the work;
//  - no increment is overwritten by the pointer store (deposits never
//    count past the threshold), so the ledger
//        S = sum(leaf counts) - 4 * sum(iteration of each allocated block)
//    equals the number of deposits exactly;
//  - the splitter writes the eight children's start count (the current
//    iteration, i.e. parent/4) before it publishes the pointer with release
//    ordering, instead of prefilling every unused node per iteration;
//  - node words are read with cacheable loads; a negative word never
//    changes again and every other decision is validated by the CAS;
//  - nodes at depth 20 never split (FP32 positions cannot resolve finer
//    cells).
#include "neb_device.h"

namespace neb {

// Every decision taken on a loaded node word is either safe when the word is
// stale (a negative word never changes again; a deferral is always allowed)
// or validated by the compare-and-swap, which is resolved at the device's
// coherence point and returns the current word.  Loads can therefore be
// cacheable: no acquire, no L2 invalidation per tree level.
__device__ __forceinline__ int32_t ld_node(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

enum { kInsRejected = 0, kInsCounted = 1, kInsDeferred = 2 };

// The split of a full leaf: allocate 8 children, start them at the current
// iteration (parent / 4), publish the pointer.  Called by exactly one lane,
// the one whose CAS brought the count to the threshold.
__device__ __forceinline__ void oct_split(int32_t* nodes, OctState* st, const OctParams& P, int32_t idx, int level) {
    int32_t child = atomicAdd(&st->alloc, 8);
    if (child >= P.capacity) {
        atomicExch(&st->alloc, P.capacity + 1);
        __hip_atomic_fetch_or(nodes + idx, kOctFailed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        atomicAdd(&st->overflow, 1);
        return;
    }
    // the wait retires the eight atomic writes (CDNA tracks them in vmcnt)
    // before the pointer is published, so a lane that follows the pointer
    // and CASes a child compares against the started count
#pragma unroll
    for (int c = 0; c < 8; ++c)
        __hip_atomic_exchange(nodes + child + c, P.iter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __hip_atomic_exchange(nodes + idx, -child, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    atomicAdd(&st->block_iter_sum, (unsigned long long)P.iter);
    atomicMax(&st->depth, level + 1);
}

// one deposit attempt; never waits for another lane
__device__ __forceinline__ int oct_insert(int32_t* nodes, OctState* st, const OctParams& P, f3 p) {
    float q[3];
    if (!oct_norm(P, p, q)) return kInsRejected;
    int32_t idx = 0;
    int level = 0;
    int32_t v = ld_node(nodes);
    for (int step = 0; step < 4096; ++step) {
        if (v < 0) {
            ++level;
            float sc = (float)(1 << level);
            int32_t c = (((int32_t)(q[0] * sc)) & 1) | ((((int32_t)(q[1] * sc)) & 1) << 1) |
                        ((((int32_t)(q[2] * sc)) & 1) << 2);
            idx = c - v;
            v = ld_node(nodes + idx);
            continue;
        }
        int32_t cnt = v & kOctCountMask;
        bool can_split = !(v & kOctFailed) && level < kOctMaxDepth;
        if (can_split && cnt >= P.split_count) return kInsDeferred;  // a split is being published
        int32_t expected = v;
        if (!__hip_atomic_compare_exchange_strong(nodes + idx, &expected, v + 1, __ATOMIC_RELAXED,
                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            v = expected;  // the current word: retry with it
            continue;
        }
        if (can_split && cnt + 1 == P.split_count) oct_split(nodes, st, P, idx, level);
        return kInsCounted;
    }
    return kInsDeferred;  // heavy contention: try again after the launch
}

// Wave-cooperative deposit of one point per lane.  Lanes that reach the
// same node word with the same observed value form a group; its first lane
// adds the group's size (capped at the split threshold) with one CAS, the
// lanes beyond the cap defer, and the lane whose addition reaches the
// threshold splits.  A burst of deposits into one cell (every deposit of
// the first iteration starts at the root) thus costs one atomic per wave
// instead of one per lane.  Must be called by all lanes of the wave.
__device__ __forceinline__ int oct_insert_wave(int32_t* nodes, OctState* st, const OctParams& P, bool has, f3 p) {
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
    float q[3] = {0.f, 0.f, 0.f};
    bool active = has && oct_norm(P, p, q);
    int result = (has && !active) ? kInsRejected : kInsDeferred;
    int32_t idx = 0;
    int level = 0;
    int32_t v = active ? ld_node(nodes) : 0;
    for (int step = 0; step < 4096; ++step) {
        if (!__any(active)) break;
        if (active && v < 0) {
            ++level;
            float sc = (float)(1 << level);
            int32_t c = (((int32_t)(q[0] * sc)) & 1) | ((((int32_t)(q[1] * sc)) & 1) << 1) |
                        ((((int32_t)(q[2] * sc)) & 1) << 2);
            idx = c - v;
            v = ld_node(nodes + idx);
        }
        bool want = active && v >= 0;
        unsigned long long pend = __ballot(want);
        while (pend) {
            int leader = __ffsll((long long)pend) - 1;
            int32_t lidx = __shfl(idx, leader, 64);
            int32_t lv = __shfl(v, leader, 64);
            int llevel = __shfl(level, leader, 64);
            bool in = want && idx == lidx && v == lv;
            unsigned long long gm = __ballot(in);
            int k = __popcll(gm);
            int32_t cnt = lv & kOctCountMask;
            bool can_split = !(lv & kOctFailed) && llevel < kOctMaxDepth;
            int m = can_split ? min(k, max(0, P.split_count - cnt)) : k;
            int ok = 0;
            int32_t cur = lv;
            if (lane == leader && m > 0) {
                int32_t e = lv;
                ok = __hip_atomic_compare_exchange_strong(nodes + lidx, &e, lv + m, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT);
                cur = e;
                if (ok && can_split && cnt + m == P.split_count) oct_split(nodes, st, P, lidx, llevel);
            }
            ok = __shfl(ok, leader, 64);
            cur = __shfl(cur, leader, 64);
            if (in) {
                if (m == 0) {  // full leaf, split in flight: retry after the launch
                    result = kInsDeferred;
                    active = false;
                } else if (ok) {
                    result = __popcll(gm & below) < m ? kInsCounted : kInsDeferred;
                    active = false;
                } else {
                    v = cur;  // the word changed: retry with its current value
                }
            }
            want = want && !in;
            pend &= ~gm;
        }
    }
    return result;
}

__device__ __forceinline__ void oct_account(OctState* st, int counted, int rejected) {
    // one atomic per wave for each tally (all lanes of the block reach this)
    unsigned long long c = (unsigned long long)counted;
    int r = rejected;
    for (int off = 32; off > 0; off >>= 1) {
        c += __shfl_xor(c, off, 64);
        r += __shfl_xor(r, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        if (c) atomicAdd(&st->deposits, c);
        if (r) atomicAdd(&st->rejected, r);
    }
}

// Deposit items [0, n) (round 0, items == nullptr) or the deferred items of
// the previous round.  Positions are float3 (stride 3) or float4 vertex
// records (stride 4).  Deferred items go to defer_out; the counter of the
// round after next is cleared here (three counters rotate).
__global__ void __launch_bounds__(256) k_oct_insert(int32_t* nodes, OctState* st, OctParams P,
                                                    const float* __restrict__ pos, int stride,
                                                    const int32_t* __restrict__ items, const int32_t* n_dev,
                                                    int32_t n_host, int32_t* __restrict__ defer_out,
                                                    int32_t* defer_count, int32_t* clear_count) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *clear_count = 0;
    int32_t n = n_dev ? min(*n_dev, n_host) : n_host;
    int counted = 0, rejected = 0;
    if (!P.stop_filling) {
        int64_t stride_all = (int64_t)gridDim.x * blockDim.x;
        int64_t nn = (n + stride_all - 1) / stride_all * stride_all;  // uniform trip count per wave
        for (int64_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nn; i += stride_all) {
            bool has = i < n;
            int32_t item = 0;
            f3 pt = mk3(0.f, 0.f, 0.f);
            if (has) {
                item = items ? items[i] : (int32_t)i;
                const float* pp = pos + (size_t)stride * item;
                pt = mk3(pp[0], pp[1], pp[2]);
            }
            int r = oct_insert_wave(nodes, st, P, has, pt);
            bool defer = has && r == kInsDeferred;
            counted += has && r == kInsCounted;
            rejected += has && r == kInsRejected;
            int slot = wave_reserve(defer_count, defer);
            if (defer) defer_out[slot] = item;
        }
    }
    oct_account(st, counted, rejected);
}

__global__ void k_oct_insert_single(int32_t* nodes, OctState* st, OctParams P, const float* __restrict__ pos,
                                    int stride, const int32_t* __restrict__ order, int32_t n) {
    if (threadIdx.x != 0 || blockIdx.x != 0 || P.stop_filling) return;
    unsigned long long counted = 0, lost = 0;
    int rejected = 0;
    for (int32_t i = 0; i < n; ++i) {
        int32_t item = order ? order[i] : i;
        if (item < 0) continue;
        const float* pp = pos + (size_t)stride * item;
        int r = oct_insert(nodes, st, P, mk3(pp[0], pp[1], pp[2]));
        counted += r == kInsCounted;
        rejected += r == kInsRejected;
        lost += r == kInsDeferred;  // impossible without concurrency
    }
    atomicAdd(&st->deposits, counted);
    atomicAdd(&st->rejected, rejected);
    atomicAdd(&st->lost, lost);
}

// deposits still deferred after the last round are reported as lost
__global__ void k_oct_report_lost(OctState* st, const int32_t* remaining) {
    if (*remaining) atomicAdd(&st->lost, (unsigned long long)*remaining);
}

__global__ void __launch_bounds__(256) k_oct_density_xyz(const int32_t* __restrict__ nodes, const OctState* st,
                                                         OctParams P, const float* __restrict__ pos,
                                                         const float* __restrict__ nrm, int32_t n, int robust,
                                                         float* __restrict__ out) {
    int depth = st->depth;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        f3 p = load3(pos + 3 * (size_t)i);
        f3 nn = normalize3(load3(nrm + 3 * (size_t)i));
        out[i] = robust ? oct_query_robust(nodes, P, depth, p, nn) : oct_query(nodes, P, depth, p, nn, false, nullptr);
    }
}

__global__ void k_oct_init(int32_t* nodes, OctState* st, int32_t capacity) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < capacity; i += gridDim.x * blockDim.x) nodes[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->alloc = 1;
        st->depth = 0;
        st->overflow = 0;
        st->rejected = 0;
        st->block_iter_sum = 0;
        st->deposits = 0;
        st->lost = 0;
    }
}

__global__ void k_oct_clear(int32_t* nodes, OctState* st, int32_t capacity) {
    int32_t n = min(st->alloc, capacity);
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int32_t v = nodes[i];
        if (v > 0) nodes[i] = 0;
    }
}

// after clear: the ledger restarts (runs as a separate launch so that the
// clear kernel can read alloc while this one resets the sums)
__global__ void k_oct_clear_ledger(OctState* st) {
    st->block_iter_sum = 0;
    st->deposits = 0;
}

__global__ void k_oct_clear_counter(int32_t* c) { *c = 0; }

static int grid_for(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    return (int)g;
}

void octree_params_init(OctParams& p, const float smin[3], const float smax[3], int32_t capacity) {
    float size[3];
    for (int i = 0; i < 3; ++i) {
        size[i] = (smax[i] - smin[i]) * 1.002f;
        p.size_inv[i] = 1.0f / size[i];
    }
    float sq = size[0] * size[0];
    sq = sq + size[1] * size[1];
    sq = sq + size[2] * size[2];
    p.scene_scale = sqrtf(sq);
    const float rel = 0.001f / 1.002f;
    for (int i = 0; i < 3; ++i) p.min_bound[i] = smin[i] - size[i] * rel;
    p.capacity = 1 + ((capacity + 7) & ~7);
    octree_params_set_iteration(p, 1);
}

void octree_params_set_iteration(OctParams& p, int32_t iter) {
    int32_t ic = iter < kOctFillIterations ? iter : kOctFillIterations;
    p.stop_filling = iter > kOctFillIterations;
    p.density_scale = 1.0f / (float)ic;
    p.split_count = kOctSplitFactor * ic;
    p.iter = iter;
}

hipError_t octree_init_nodes(Octree& o, hipStream_t s) {
    hipLaunchKernelGGL(k_oct_init, dim3(grid_for(o.prm.capacity, 256)), dim3(256), 0, s, o.nodes, o.state,
                       o.prm.capacity);
    return hipGetLastError();
}

static hipError_t insert_rounds(const Octree& o, const float* pos, int stride, const int32_t* n_dev, int32_t n_host,
                                hipStream_t s) {
    int32_t* cnt = o.defer_cnt;
    hipLaunchKernelGGL(k_oct_clear_counter, dim3(1), dim3(1), 0, s, cnt + 1);
    hipLaunchKernelGGL(k_oct_insert, dim3(grid_for(n_host, 256)), dim3(256), 0, s, o.nodes, o.state, o.prm, pos, stride,
                       (const int32_t*)nullptr, n_dev, n_host, o.defer[0], cnt + 1, cnt + 2);
    for (int r = 1; r <= kOctMaxDepth + 1; ++r) {
        hipLaunchKernelGGL(k_oct_insert, dim3(64), dim3(256), 0, s, o.nodes, o.state, o.prm, pos, stride,
                           (const int32_t*)o.defer[(r - 1) & 1], (const int32_t*)(cnt + (r % 3)), n_host,
                           o.defer[r & 1], cnt + ((r + 1) % 3), cnt + ((r + 2) % 3));
    }
    hipLaunchKernelGGL(k_oct_report_lost, dim3(1), dim3(1), 0, s, o.state,
                       (const int32_t*)(cnt + ((kOctMaxDepth + 2) % 3)));
    return hipGetLastError();
}

hipError_t octree_reserve(Octree& o, int64_t n) {
    if (n <= o.defer_cap) return hipSuccess;
    if (o.defer[0]) (void)hipFree(o.defer[0]);
    if (o.defer[1]) (void)hipFree(o.defer[1]);
    o.defer[0] = o.defer[1] = nullptr;
    o.defer_cap = 0;
    hipError_t e = hipMalloc(&o.defer[0], 4 * (size_t)n);
    if (e == hipSuccess) e = hipMalloc(&o.defer[1], 4 * (size_t)n);
    if (e == hipSuccess && !o.defer_cnt) e = hipMalloc(&o.defer_cnt, 4 * 3);
    if (e == hipSuccess) o.defer_cap = n;
    return e;
}

void octree_release(Octree& o) {
    if (o.defer[0]) (void)hipFree(o.defer[0]);
    if (o.defer[1]) (void)hipFree(o.defer[1]);
    if (o.defer_cnt) (void)hipFree(o.defer_cnt);
    if (o.nodes) (void)hipFree(o.nodes);
    if (o.state) (void)hipFree(o.state);
    o = Octree();
}

hipError_t octree_increment_xyz(Octree& o, const float* pos, int32_t n, int single, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (single) {
        hipLaunchKernelGGL(k_oct_insert_single, dim3(1), dim3(64), 0, s, o.nodes, o.state, o.prm, pos, 3,
                           (const int32_t*)nullptr, n);
        return hipGetLastError();
    }
    hipError_t e = octree_reserve(o, n);
    if (e != hipSuccess) return e;
    return insert_rounds(o, pos, 3, nullptr, n, s);
}

hipError_t octree_increment_vertices(const Octree& o, const float4* vpos, const int32_t* nvert, int32_t cap,
                                     hipStream_t s) {
    return insert_rounds(o, reinterpret_cast<const float*>(vpos), 4, nvert, cap, s);
}

hipError_t octree_increment_slots(const Octree& o, const float4* vpos, const int32_t* slots, int32_t n_slots,
                                  hipStream_t s) {
    hipLaunchKernelGGL(k_oct_insert_single, dim3(1), dim3(64), 0, s, o.nodes, o.state, o.prm,
                       reinterpret_cast<const float*>(vpos), 4, slots, n_slots);
    return hipGetLastError();
}

hipError_t octree_density_xyz(const Octree& o, const float* pos, const float* nrm, int32_t n, int robust, float* out,
                              hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_oct_density_xyz, dim3(grid_for(n, 256)), dim3(256), 0, s, o.nodes, o.state, o.prm, pos,
                       nrm, n, robust, out);
    return hipGetLastError();
}

hipError_t octree_clear(const Octree& o, hipStream_t s) {
    hipLaunchKernelGGL(k_oct_clear, dim3(grid_for(o.prm.capacity, 256)), dim3(256), 0, s, o.nodes, o.state,
                       o.prm.capacity);
    hipLaunchKernelGGL(k_oct_clear_ledger, dim3(1), dim3(1), 0, s, o.state);
    return hipGetLastError();
}

}  // namespace neb
