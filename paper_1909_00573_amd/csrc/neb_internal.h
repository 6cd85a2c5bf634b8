// Internal declarations shared by the HIP translation units of libneb.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "neb.h"

namespace neb {

constexpr int kOctMaxDepth = 20;           // nodes at this depth never split
constexpr int kOctFillIterations = 1000;   // counting stops afterwards
constexpr int kOctSplitFactor = 4;         // split threshold = 4 * iteration
constexpr int32_t kOctFailed = 0x40000000; // "split failed" mark on a full leaf
constexpr int32_t kOctCountMask = 0x3FFFFFFF;
constexpr int kMaxPathLen = 16;
constexpr int kBvhStackMax = 64;           // deepest LDS traversal stack (entries per lane)
constexpr int kTraceBlock = 64;            // threads per traversal block (one wave)

constexpr uint32_t kTagCamera = 1, kTagBsdf = 2, kTagNee = 3, kTagPhoton = 4, kTagMlp = 5, kTagProbe = 6,
                   kTagLight = 7;

// Static scalars of one octree (the members of the class of Appendix B that
// do not change with the iteration), passed by value.  Several octrees can
// share one node pool: each owns the words [root, end).
struct OctParams {
    float min_bound[3];
    float size_inv[3];
    float scene_scale;
    int32_t root;   // index of the root word in the pool
    int32_t end;    // root + capacity (capacity = 8n + 1)
};

// Iteration-dependent scalars (Appendix B set_iteration), device resident so
// that a captured graph of one iteration can be replayed for every iteration.
struct OctDyn {
    int32_t iter;
    int32_t split_count;
    float density_scale;
    int32_t stop_filling;
};

// device-resident octree state updated by atomics
// The allocation counter (hit by every split), the split tallies and the
// deposit tally (one atomic per wave of every insertion launch) sit in cache
// lines of their own; the deposit tally is striped over kDepositStripes
// lines (a block adds into stripe blockIdx.x mod kDepositStripes), its value
// is the sum of the stripes (oct_deposits).
constexpr int kDepositStripes = 16;
struct alignas(128) TallyLine {
    unsigned long long v;
};
struct OctState {
    alignas(128) int32_t alloc;
    alignas(128) int32_t depth;
    int32_t overflow;
    int32_t rejected;
    unsigned long long block_iter_sum;
    unsigned long long lost;
    TallyLine deposits[kDepositStripes];
};
__host__ __device__ inline unsigned long long oct_deposits(const OctState& st) {
    unsigned long long d = 0;
    for (int k = 0; k < kDepositStripes; ++k) d += st.deposits[k].v;
    return d;
}

// a standalone octree (the Appendix-B surface of the C ABI)
struct Octree {
    int32_t* nodes = nullptr;   // device, capacity words
    OctState* state = nullptr;  // device
    OctDyn* dyn = nullptr;      // device
    OctParams* prm_dev = nullptr;  // device copy of prm (the kernels take an array of them)
    OctParams prm{};
    int32_t capacity = 0;
    int32_t last_iter = 0;
    int32_t* defer[2] = {nullptr, nullptr};  // deferred deposits, ping-pong
    int32_t* defer_cnt = nullptr;            // three rotating counters
    int64_t defer_cap = 0;
};

struct CamParams {
    float eye[3], f[3], r[3], u[3];
    float tan_half, aspect;
    int32_t w, h;
};

// read-only geometry and light pools shared by every scene of a context
struct SceneView {
    const float4* bvh;         // 8 float4 per node (four child boxes, child links, leaf counts), all scenes
    const float4* tri;         // 3 float4 per triangle in leaf order; tri[0].w = global prim id bits
    const float4* prim_n;      // per prim: unit geometric normal, .w = global material id bits
    const int32_t* prim_light; // per prim: global light index or -1
    const neb_material* mats;
    const float4* lights;      // 5 float4 per light
    const float* light_cdf;    // per scene: inclusive cumulative selection probabilities
    const int32_t* light_guide; // per scene, same layout: where pick_light starts its search
};

// device counters of one context
// Work statistics, striped: a block adds into stripe blockIdx.x mod
// kStatStripes, so the end-of-kernel atomics of concurrent waves spread over
// separate cache lines instead of serialising on one; the host sums the
// stripes.
constexpr int kStatStripes = 16;
struct alignas(128) StatLine {
    unsigned long long paths, vertices, photons, photon_segments, merges, nee_visible, events;
    unsigned long long camera_rays, shadow_rays, photon_rays;
    unsigned long long photon_items, photon_continued, grid_cells, candidates;
    // traversal work (nodes fetched, triangles tested) by ray kind: camera,
    // photon and shadow rays (the ray_kind of k_extend)
    unsigned long long bvh_nodes[3], bvh_tris[3];
    unsigned long long light_photons;
};

// Photon queues (and their hit arrays) rotate over kPhotonBufs buffers, so
// that the closest hits and scatter of a bounce can run while the merges of
// the two bounces before it still read theirs.
constexpr int kPhotonBufs = 3;

// A closest-hit launch hands out its rays through kWorkParts counters, one
// cache line each (its blocks run on eight XCDs; one counter per XCD).
constexpr int kWorkParts = 8;
struct alignas(128) WorkLine {
    int32_t next;
};

// Device counters.  Every queue counter sits in a cache line of its own:
// atomics on one line are serialised by the cache, and counters that
// different kernels (or one kernel's reservations and its statistics) hit
// at the same time must not share one.
struct Counters {
    alignas(128) int32_t qcount[2];  // camera path queues
    alignas(128) int32_t pcount[kPhotonBufs];  // photon queues
    alignas(128) int32_t mcount[kPhotonBufs];  // their lengths for the merge launches (copied by the scatter)
    alignas(128) int32_t n_vertices[2];  // per parity of the iteration (two vertex stores)
    alignas(128) int32_t n_events[2];
    alignas(128) int32_t n_shadow;   // NEE shadow rays queued this iteration
    alignas(128) int32_t iter;       // current iteration (incremented at the start of each one)
    alignas(128) int32_t iter_cam;   // iteration of the camera pass in flight (it may run one ahead)
    alignas(128) int32_t lp_count;   // light photons emitted this iteration (the first entries of photon queue 0)
    WorkLine trace_next[kWorkParts]; // per part: rays a closest-hit launch handed out (reset by its last block)
    alignas(128) int32_t trace_done; // blocks of that launch that finished
    WorkLine cam_next[kWorkParts];   // the same for the camera pass's closest-hit launches, which may
    alignas(128) int32_t cam_done;   // run beside the photon bounces' ones
    StatLine st[kStatStripes];
};

// octree (neb_octree.hip)
void octree_params_init(OctParams& p, const float smin[3], const float smax[3], int32_t root, int32_t capacity);
void octree_dyn_for(OctDyn& d, int32_t iter);
int32_t octree_capacity_rounded(int32_t capacity);
hipError_t octree_reserve(Octree& o, int64_t n);
void octree_release(Octree& o);
hipError_t octree_reset(Octree& o, hipStream_t s);
hipError_t octree_increment_xyz(Octree& o, const float* pos, int32_t n, int single, hipStream_t s);
hipError_t octree_density_xyz(const Octree& o, const float* pos, const float* nrm, int32_t n, int robust, float* out,
                              hipStream_t s);
hipError_t octree_density_raw(const int32_t* nodes, const OctState* st, const OctParams& P, const OctDyn* dyn,
                              const float* pos, const float* nrm, int32_t n, int robust, float* out, hipStream_t s);
hipError_t octree_clear(const Octree& o, hipStream_t s);
// deposits of NEE vertices of many scenes: per-vertex scene from the record
hipError_t octree_insert_rounds(int32_t* nodes, OctState* states, const OctParams* prm, const OctDyn* dyn,
                                const float* pos, int stride, const int32_t* scene_of_item, int scene_shift,
                                const int32_t* n_dev, int32_t n_host, int32_t* const defer[2], int32_t* defer_cnt,
                                hipStream_t s);
hipError_t octree_insert_single(int32_t* nodes, OctState* states, const OctParams* prm, const OctDyn* dyn,
                                const float* pos, int stride, const int32_t* scene_of_item, int scene_shift,
                                const int32_t* order, int32_t n, hipStream_t s);
hipError_t octree_init_range(int32_t* nodes, OctState* st, int32_t root, int32_t capacity, hipStream_t s);
hipError_t octree_set_dyn(OctDyn* dyn, const OctDyn& d, hipStream_t s);

}  // namespace neb
