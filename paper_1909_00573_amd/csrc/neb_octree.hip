// Lock-free sparse density octree (Sec. 5 of the paper, class of Appendix B)
// on gfx950: device-scope atomics on an int32 node pool, compare-and-swap
// counting and splits allocated with one fetch-add.  No lane ever waits for
// another lane.  Several octrees (one per scene of a batch) can share one
// pool; each owns the words [root, end) and has its own OctState.
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
//    the loop's reconvergence point: the wave deadlocks.  Here the lanes of
//    a wave that reach the same node word add their count with one CAS
//    (capped at the split threshold), the lane whose addition fills the
//    leaf splits it on the spot, and the lanes beyond the cap follow the
//    pointer their own wave has just published; so a full leaf without a
//    pointer was always filled by another wave.  Such a deposit is deferred
//    to a queue retried by the next round, once that wave's split is
//    certainly published: rounds 1 .. kOctLaunchRounds - 1 are launches of
//    their own (the kernel boundary), later rounds run in one block,
//    separated by the block's barrier and an agent-scope acquire.  A deposit is deferred at
//    most once per level, so kOctMaxDepth + 1 retry rounds bound the work.
//    (Re-reading the word a bounded number of times instead was measured
//    slower: a wave keeps looping while any lane waits);
//  - no increment is overwritten by the pointer store (deposits never
//    count past the threshold), so the ledger
//        S = sum(leaf counts) - 4 * sum(iteration of each allocated block)
//    equals the number of deposits exactly;
//  - the splitter writes the eight children's start count (the current
//    iteration, i.e. parent/4) before it publishes the pointer, instead of
//    prefilling every unused node per iteration;
//  - node words are read with cacheable loads; a negative word never
//    changes again and every other decision is validated by the CAS;
//  - nodes at depth 20 never split (FP32 positions cannot resolve finer
//    cells).
#include <algorithm>

#include "neb_device.h"

namespace neb {

__device__ __forceinline__ int32_t ld_node(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

enum { kInsRejected = 0, kInsCounted = 1, kInsDeferred = 2 };

// deposit rounds run as launches of their own (measured: while a reset tree
// grows, rounds 1-3 still hold many deferred items; afterwards only round 1)
constexpr int kOctLaunchRounds = 4;

__device__ __forceinline__ int child_index(const float q[3], int level) {
    float sc = (float)(1 << level);
    return (((int32_t)(q[0] * sc)) & 1) | ((((int32_t)(q[1] * sc)) & 1) << 1) | ((((int32_t)(q[2] * sc)) & 1) << 2);
}

// what a lane's splits add to its octree's state; flushed once per wave
struct SplitTally {
    unsigned long long iter_sum = 0;  // iteration of each block it allocated
    int depth = 0;                    // deepest level it created
    int failed = 0;                   // splits refused by a full pool
};

// Children of a full leaf whose word holds `full`, in the block `child`
// (allocated by the caller; >= P.end means the pool is exhausted): start
// the eight children at the current iteration (parent / 4), then publish
// the pointer.  Returns the node word afterwards: the child pointer, or
// `full` marked as a failed split.
__device__ __forceinline__ int32_t oct_make_children(int32_t* nodes, const OctParams& P, const OctDyn& D,
                                                     int32_t idx, int level, int32_t full, int32_t child,
                                                     SplitTally& T) {
    if (child >= P.end) {
        __hip_atomic_fetch_or(nodes + idx, kOctFailed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        T.failed += 1;
        return full | kOctFailed;
    }
    // the wait retires the eight atomic writes (CDNA tracks them in vmcnt)
    // before the pointer is published, so a lane that follows the pointer
    // and CASes a child compares against the started count
#pragma unroll
    for (int c = 0; c < 8; ++c)
        __hip_atomic_exchange(nodes + child + c, D.iter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __hip_atomic_exchange(nodes + idx, -child, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    T.iter_sum += (unsigned long long)D.iter;
    T.depth = max(T.depth, level + 1);
    return -child;
}

// next free block of n blocks of 8 in an octree, or P.end if the pool is
// full (a full pool is seen with a plain read, without an atomic)
__device__ __forceinline__ int32_t oct_alloc(OctState* st, const OctParams& P, int n) {
    if (__hip_atomic_load(&st->alloc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= P.end) return P.end;
    return atomicAdd(&st->alloc, 8 * n);
}

__device__ __forceinline__ void flush_tally(OctState* st, const SplitTally& T) {
    if (T.iter_sum) atomicAdd(&st->block_iter_sum, T.iter_sum);
    if (T.depth) atomicMax(&st->depth, T.depth);
    if (T.failed) atomicAdd(&st->overflow, T.failed);
}

// one deposit by one thread alone (sequential insertion, the oracle's order)
__device__ __forceinline__ int oct_insert(int32_t* nodes, OctState* st, const OctParams& P, const OctDyn& D, f3 p) {
    float q[3];
    if (!oct_norm(P, p, q)) return kInsRejected;
    int32_t idx = P.root;
    int level = 0;
    int32_t v = ld_node(nodes + idx);
    for (int step = 0; step < 4096; ++step) {
        if (v < 0) {
            ++level;
            idx = child_index(q, level) - v;
            v = ld_node(nodes + idx);
            continue;
        }
        int32_t cnt = v & kOctCountMask;
        bool can_split = !(v & kOctFailed) && level < kOctMaxDepth;
        if (can_split && cnt >= D.split_count) return kInsDeferred;
        int32_t expected = v;
        if (!__hip_atomic_compare_exchange_strong(nodes + idx, &expected, v + 1, __ATOMIC_RELAXED,
                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            v = expected;
            continue;
        }
        if (can_split && cnt + 1 == D.split_count) {
            SplitTally T;
            oct_make_children(nodes, P, D, idx, level, v + 1, oct_alloc(st, P, 1), T);
            flush_tally(st, T);
        }
        return kInsCounted;
    }
    return kInsDeferred;
}

// Wave-cooperative deposit of one point per lane (lanes may belong to
// different octrees of the pool).  Each pass: lanes that reach the same
// node word with the same observed value form a group, and the group's
// first lane adds the group's size (capped at the split threshold) with one
// CAS; then every group whose addition filled its leaf splits, with one
// block allocation per octree for all of the wave's splits of the pass.
// The lanes beyond a cap follow the pointer their own wave has just
// published (nobody waits for anybody).  Lanes that find a leaf filled by
// another wave, whose split may still be in flight, defer to the next
// launch.  Must be called by all lanes of the wave.
__device__ __forceinline__ int oct_insert_wave(int32_t* nodes, OctState* st, const OctParams& P, const OctDyn& D,
                                               bool has, f3 p, SplitTally& tally) {
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
    const unsigned long long stkey = (unsigned long long)(uintptr_t)st;
    float q[3] = {0.f, 0.f, 0.f};
    bool active = has && oct_norm(P, p, q);
    int result = (has && !active) ? kInsRejected : kInsDeferred;
    int32_t idx = P.root;
    int level = 0;
    int32_t v = active ? ld_node(nodes + idx) : 0;
    for (int step = 0; step < 4096; ++step) {
        if (!__any(active)) break;
        if (active && v < 0) {
            ++level;
            idx = child_index(q, level) - v;
            v = ld_node(nodes + idx);
        }
        const bool grouped = active && v >= 0;
        bool want = grouped;
        unsigned long long pend = __ballot(want);
        // phase 1: the lanes at the same word form a group (its first lane
        // leads) and take m of its free counts; then every leader issues its
        // group's CAS at once, so the wave waits for one atomic round trip,
        // not one per group
        int my_leader = lane, my_rank = 0, my_m = 0;
        int lead_m = 0;  // this lane leads a group taking lead_m counts
        bool lead_split = false;
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
            int m = can_split ? min(k, max(0, D.split_count - cnt)) : k;
            if (in) {
                my_leader = leader;
                my_rank = __popcll(gm & below);
                my_m = m;
            }
            if (lane == leader) {
                lead_m = m;
                lead_split = can_split && cnt + m == D.split_count;
            }
            want = want && !in;
            pend &= ~gm;
        }
        int l_ok = 0, l_split = 0;
        int32_t l_cur = v, l_full = v;
        if (lead_m > 0) {  // a leader's own idx and v are its group's
            int32_t e = v;
            l_ok = __hip_atomic_compare_exchange_strong(nodes + idx, &e, v + lead_m, __ATOMIC_RELAXED,
                                                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            l_cur = e;
            l_full = v + lead_m;
            l_split = l_ok && lead_split;
        }
        // phase 2: the pass's splits, one allocation per octree
        int32_t l_after = l_full;
        unsigned long long spl = __ballot(l_split);
        while (spl) {
            int first = __ffsll((long long)spl) - 1;
            unsigned long long key = __shfl(stkey, first, 64);
            bool mine = l_split && stkey == key;
            unsigned long long sm = __ballot(mine);
            int32_t base = 0;
            if (lane == first) base = oct_alloc(st, P, __popcll(sm));
            base = __shfl(base, first, 64);
            if (mine) l_after = oct_make_children(nodes, P, D, idx, level, l_full, base + 8 * __popcll(sm & below), tally);
            spl &= ~sm;
        }
        // phase 3: every grouped lane learns its group's outcome
        int ok = __shfl(l_ok, my_leader, 64);
        int32_t cur = __shfl(l_cur, my_leader, 64);
        int32_t after = __shfl(l_after, my_leader, 64);
        if (grouped) {
            if (my_m == 0) {  // full leaf, split in flight: retry after the launch
                result = kInsDeferred;
                active = false;
            } else if (ok) {
                if (my_rank < my_m) {
                    result = kInsCounted;
                    active = false;
                } else {
                    v = after;  // this wave split the leaf: go on from its new word
                }
            } else {
                v = cur;  // the word changed: retry with its current value
            }
        }
    }
    return result;
}

// one atomic per wave and state for each tally; lanes of a wave may belong
// to different octree states
__device__ __forceinline__ void oct_account(OctState* states, int scene, int counted, int rejected,
                                            const SplitTally& T) {
    const int lane = threadIdx.x & 63;
    unsigned long long pend =
        __ballot(counted != 0 || rejected != 0 || T.iter_sum != 0 || T.depth != 0 || T.failed != 0);
    while (pend) {
        int leader = __ffsll((long long)pend) - 1;
        int ls = __shfl(scene, leader, 64);
        bool in = ((pend >> lane) & 1ull) && scene == ls;
        unsigned long long c = in ? (unsigned long long)counted : 0ull;
        int r = in ? rejected : 0;
        SplitTally S;
        if (in) S = T;
        for (int off = 32; off > 0; off >>= 1) {
            c += __shfl_xor(c, off, 64);
            r += __shfl_xor(r, off, 64);
            S.iter_sum += __shfl_xor(S.iter_sum, off, 64);
            S.failed += __shfl_xor(S.failed, off, 64);
            S.depth = max(S.depth, __shfl_xor(S.depth, off, 64));
        }
        if (lane == leader) {
            if (c) atomicAdd(&states[ls].deposits[blockIdx.x & (kDepositStripes - 1)].v, c);
            if (r) atomicAdd(&states[ls].rejected, r);
            flush_tally(states + ls, S);
        }
        pend &= ~__ballot(in);
    }
}

__device__ __forceinline__ int item_scene(const int32_t* scene_word, int stride, int shift, int32_t item) {
    return scene_word ? ((scene_word[(size_t)stride * item] >> shift) & 0xFF) : 0;
}

// One pass of deposits over n items, by threads t0, t0 + step, ...: items
// [0, n) (items == nullptr) or the listed ones.  Positions are float3
// (stride 3) or the xyz of float4 records (stride 4); the octree of an item
// is read from scene_word.  Deferred items go to defer_out.
__device__ __forceinline__ void oct_insert_pass(int32_t* nodes, OctState* states, const OctParams* prm,
                                                const OctDyn& D, const float* __restrict__ pos, int stride,
                                                const int32_t* __restrict__ scene_word, int shift,
                                                const int32_t* __restrict__ items, int32_t n, int64_t t0,
                                                int64_t step, int32_t* __restrict__ defer_out,
                                                int32_t* defer_count) {
    int64_t nn = (n + step - 1) / step * step;  // uniform trip count per wave
    for (int64_t i = t0; i < nn; i += step) {
        bool has = i < n;
        int32_t item = 0;
        f3 pt = mk3(0.f, 0.f, 0.f);
        int s = 0;
        if (has) {
            item = items ? items[i] : (int32_t)i;
            const float* pp = pos + (size_t)stride * item;
            pt = mk3(pp[0], pp[1], pp[2]);
            s = item_scene(scene_word, stride, shift, item);
        }
        const OctParams P = prm[s];
        SplitTally tally;
        int r = oct_insert_wave(nodes, states + s, P, D, has, pt, tally);
        bool defer = has && r == kInsDeferred;
        oct_account(states, s, has && r == kInsCounted, has && r == kInsRejected, tally);
        int slot = wave_reserve(defer_count, defer);
        if (defer) defer_out[slot] = item;
    }
}

// Round 0 (items == nullptr: items [0, n)) or one of the rounds 1 ..
// kOctLaunchRounds - 1 (the items deferred in the round before) of a
// deposit; the counter of the round after next is cleared here (three
// counters rotate).
__global__ void __launch_bounds__(256) k_oct_insert(int32_t* nodes, OctState* states, const OctParams* prm,
                                                    const OctDyn* dyn, const float* __restrict__ pos, int stride,
                                                    const int32_t* __restrict__ scene_word, int shift,
                                                    const int32_t* __restrict__ items, const int32_t* n_dev,
                                                    int32_t n_host, int32_t* __restrict__ defer_out,
                                                    int32_t* defer_count, int32_t* clear_count) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *clear_count = 0;
    const OctDyn D = *dyn;
    int32_t n = n_dev ? min(*n_dev, n_host) : n_host;
    if (D.stop_filling) return;
    oct_insert_pass(nodes, states, prm, D, pos, stride, scene_word, shift, items, n,
                    blockIdx.x * (int64_t)blockDim.x + threadIdx.x, (int64_t)gridDim.x * blockDim.x, defer_out,
                    defer_count);
}

// Rounds kOctLaunchRounds .. kOctMaxDepth + 1 in one block (after the
// launched rounds hardly any item is left, even while a reset tree grows):
// the block's barrier separates the rounds, and an agent-scope acquire
// after it makes the splits of the round before visible to this CU (what a
// new launch would do).  Round r reads list (r - 1) & 1 counted by
// cnt[r % 3] and appends to list r & 1 counted by cnt[(r + 1) % 3].  Items
// still deferred after the last round cannot occur (each round resolves at
// least one level) and would be reported as lost.
__global__ void __launch_bounds__(256) k_oct_insert_tail(int32_t* nodes, OctState* states, const OctParams* prm,
                                                         const OctDyn* dyn, const float* __restrict__ pos, int stride,
                                                         const int32_t* __restrict__ scene_word, int shift,
                                                         int32_t* defer0, int32_t* defer1, int32_t* cnt,
                                                         int32_t n_host) {
    __shared__ int32_t sn;
    const OctDyn D = *dyn;
    if (D.stop_filling) return;
    int r = kOctLaunchRounds;
    for (; r <= kOctMaxDepth + 1; ++r) {
        int32_t* in_cnt = cnt + (r % 3);
        int32_t* out_cnt = cnt + ((r + 1) % 3);
        if (threadIdx.x == 0) {
            sn = min(__hip_atomic_load(in_cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), n_host);
            __hip_atomic_store(out_cnt, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        const int32_t n = sn;
        if (n == 0) break;
        oct_insert_pass(nodes, states, prm, D, pos, stride, scene_word, shift, (r & 1) ? defer0 : defer1, n,
                        threadIdx.x, blockDim.x, (r & 1) ? defer1 : defer0, out_cnt);
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    if (r > kOctMaxDepth + 1 && threadIdx.x == 0) {
        int32_t rem = __hip_atomic_load(cnt + ((kOctMaxDepth + 2) % 3), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (rem) atomicAdd(&states->lost, (unsigned long long)rem);
    }
}

// sequential insertion by one thread; order == nullptr means 0..n-1, else
// the listed items (negative entries skipped)
__global__ void k_oct_insert_single(int32_t* nodes, OctState* states, const OctParams* prm, const OctDyn* dyn,
                                    const float* __restrict__ pos, int stride, const int32_t* __restrict__ scene_word,
                                    int shift, const int32_t* __restrict__ order, int32_t n) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const OctDyn D = *dyn;
    if (D.stop_filling) return;
    for (int32_t i = 0; i < n; ++i) {
        int32_t item = order ? order[i] : i;
        if (item < 0) continue;
        const float* pp = pos + (size_t)stride * item;
        int s = item_scene(scene_word, stride, shift, item);
        int r = oct_insert(nodes, states + s, prm[s], D, mk3(pp[0], pp[1], pp[2]));
        if (r == kInsCounted) states[s].deposits[0].v += 1;
        if (r == kInsRejected) states[s].rejected += 1;
        if (r == kInsDeferred) states[s].lost += 1;  // impossible without concurrency
    }
}

__global__ void __launch_bounds__(256) k_oct_density_xyz(const int32_t* __restrict__ nodes, const OctState* st,
                                                         OctParams P, const OctDyn* dyn, const float* __restrict__ pos,
                                                         const float* __restrict__ nrm, int32_t n, int robust,
                                                         float* __restrict__ out) {
    int depth = st->depth;
    float scale = dyn->density_scale;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        f3 p = load3(pos + 3 * (size_t)i);
        f3 nn = normalize3(load3(nrm + 3 * (size_t)i));
        out[i] = robust ? oct_query_robust(nodes, P, scale, depth, p, nn)
                        : oct_query(nodes, P, scale, depth, p, nn, false, nullptr);
    }
}

__global__ void k_oct_init(int32_t* nodes, OctState* st, OctDyn* dyn, int32_t root, int32_t capacity, OctDyn d0) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < capacity; i += gridDim.x * blockDim.x)
        nodes[root + i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->alloc = root + 1;
        st->depth = 0;
        st->overflow = 0;
        st->rejected = 0;
        st->block_iter_sum = 0;
        for (int k = 0; k < kDepositStripes; ++k) st->deposits[k].v = 0;
        st->lost = 0;
        if (dyn) *dyn = d0;
    }
}

__global__ void k_oct_clear(int32_t* nodes, OctState* st, int32_t root, int32_t end) {
    int32_t n = min(st->alloc, end);
    for (int32_t i = root + blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int32_t v = nodes[i];
        if (v > 0) nodes[i] = 0;
    }
}

// after clear: the ledger restarts (a separate launch so that the clear
// kernel can read alloc while this one resets the sums)
__global__ void k_oct_clear_ledger(OctState* st) {
    st->block_iter_sum = 0;
    for (int k = 0; k < kDepositStripes; ++k) st->deposits[k].v = 0;
}

__global__ void k_oct_clear_counter(int32_t* c) { *c = 0; }

__global__ void k_oct_set_dyn(OctDyn* dyn, OctDyn d) { *dyn = d; }

static int grid_for(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    return (int)g;
}

int32_t octree_capacity_rounded(int32_t capacity) { return 1 + ((capacity + 7) & ~7); }

void octree_params_init(OctParams& p, const float smin[3], const float smax[3], int32_t root, int32_t capacity) {
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
    p.root = root;
    p.end = root + octree_capacity_rounded(capacity);
}

void octree_dyn_for(OctDyn& d, int32_t iter) {
    int32_t ic = iter < kOctFillIterations ? iter : kOctFillIterations;
    d.iter = iter;
    d.stop_filling = iter > kOctFillIterations;
    d.density_scale = 1.0f / (float)ic;
    d.split_count = kOctSplitFactor * ic;
}

hipError_t octree_insert_rounds(int32_t* nodes, OctState* states, const OctParams* prm, const OctDyn* dyn,
                                const float* pos, int stride, const int32_t* scene_word, int shift,
                                const int32_t* n_dev, int32_t n_host, int32_t* const defer[2], int32_t* cnt,
                                hipStream_t s) {
    hipLaunchKernelGGL(k_oct_clear_counter, dim3(1), dim3(1), 0, s, cnt + 1);
    hipLaunchKernelGGL(k_oct_insert, dim3(grid_for(n_host, 256)), dim3(256), 0, s, nodes, states, prm, dyn, pos, stride,
                       scene_word, shift, (const int32_t*)nullptr, n_dev, n_host, defer[0], cnt + 1, cnt + 2);
    for (int r = 1; r < kOctLaunchRounds; ++r) {
        hipLaunchKernelGGL(k_oct_insert, dim3(std::min(grid_for(n_host, 256), 1024)), dim3(256), 0, s, nodes, states,
                           prm, dyn, pos, stride, scene_word, shift, (const int32_t*)defer[(r - 1) & 1],
                           (const int32_t*)(cnt + (r % 3)), n_host, defer[r & 1], cnt + ((r + 1) % 3),
                           cnt + ((r + 2) % 3));
    }
    hipLaunchKernelGGL(k_oct_insert_tail, dim3(1), dim3(256), 0, s, nodes, states, prm, dyn, pos, stride, scene_word,
                       shift, defer[0], defer[1], cnt, n_host);
    return hipGetLastError();
}

hipError_t octree_insert_single(int32_t* nodes, OctState* states, const OctParams* prm, const OctDyn* dyn,
                                const float* pos, int stride, const int32_t* scene_word, int shift,
                                const int32_t* order, int32_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_oct_insert_single, dim3(1), dim3(64), 0, s, nodes, states, prm, dyn, pos, stride, scene_word,
                       shift, order, n);
    return hipGetLastError();
}

hipError_t octree_init_range(int32_t* nodes, OctState* st, int32_t root, int32_t capacity, hipStream_t s) {
    OctDyn d0;
    octree_dyn_for(d0, 1);
    hipLaunchKernelGGL(k_oct_init, dim3(grid_for(capacity, 256)), dim3(256), 0, s, nodes, st, (OctDyn*)nullptr, root,
                       capacity, d0);
    return hipGetLastError();
}

hipError_t octree_set_dyn(OctDyn* dyn, const OctDyn& d, hipStream_t s) {
    hipLaunchKernelGGL(k_oct_set_dyn, dim3(1), dim3(1), 0, s, dyn, d);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// standalone octree: one octree, root 0, params copied to the device
// ---------------------------------------------------------------------------
hipError_t octree_reserve(Octree& o, int64_t n) {
    hipError_t e = hipSuccess;
    if (!o.defer_cnt) e = hipMalloc(&o.defer_cnt, 4 * 3);
    if (e != hipSuccess || n <= o.defer_cap) return e;
    if (o.defer[0]) (void)hipFree(o.defer[0]);
    if (o.defer[1]) (void)hipFree(o.defer[1]);
    o.defer[0] = o.defer[1] = nullptr;
    o.defer_cap = 0;
    e = hipMalloc(&o.defer[0], 4 * (size_t)n);
    if (e == hipSuccess) e = hipMalloc(&o.defer[1], 4 * (size_t)n);
    if (e == hipSuccess) o.defer_cap = n;
    return e;
}

void octree_release(Octree& o) {
    if (o.defer[0]) (void)hipFree(o.defer[0]);
    if (o.defer[1]) (void)hipFree(o.defer[1]);
    if (o.defer_cnt) (void)hipFree(o.defer_cnt);
    if (o.nodes) (void)hipFree(o.nodes);
    if (o.state) (void)hipFree(o.state);
    if (o.dyn) (void)hipFree(o.dyn);
    if (o.prm_dev) (void)hipFree(o.prm_dev);
    o = Octree();
}

hipError_t octree_reset(Octree& o, hipStream_t s) {
    OctDyn d0;
    octree_dyn_for(d0, 1);
    hipLaunchKernelGGL(k_oct_init, dim3(grid_for(o.capacity, 256)), dim3(256), 0, s, o.nodes, o.state, o.dyn, 0,
                       o.capacity, d0);
    return hipGetLastError();
}

hipError_t octree_increment_xyz(Octree& o, const float* pos, int32_t n, int single, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (single) return octree_insert_single(o.nodes, o.state, o.prm_dev, o.dyn, pos, 3, nullptr, 0, nullptr, n, s);
    hipError_t e = octree_reserve(o, n);
    if (e != hipSuccess) return e;
    return octree_insert_rounds(o.nodes, o.state, o.prm_dev, o.dyn, pos, 3, nullptr, 0, nullptr, n, o.defer,
                                o.defer_cnt, s);
}

hipError_t octree_density_raw(const int32_t* nodes, const OctState* st, const OctParams& P, const OctDyn* dyn,
                              const float* pos, const float* nrm, int32_t n, int robust, float* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_oct_density_xyz, dim3(grid_for(n, 256)), dim3(256), 0, s, nodes, st, P, dyn, pos, nrm, n,
                       robust, out);
    return hipGetLastError();
}

hipError_t octree_density_xyz(const Octree& o, const float* pos, const float* nrm, int32_t n, int robust, float* out,
                              hipStream_t s) {
    return octree_density_raw(o.nodes, o.state, o.prm, o.dyn, pos, nrm, n, robust, out, s);
}

hipError_t octree_clear(const Octree& o, hipStream_t s) {
    hipLaunchKernelGGL(k_oct_clear, dim3(grid_for(o.capacity, 256)), dim3(256), 0, s, o.nodes, o.state, o.prm.root,
                       o.prm.end);
    hipLaunchKernelGGL(k_oct_clear_ledger, dim3(1), dim3(1), 0, s, o.state);
    return hipGetLastError();
}

}  // namespace neb
