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
constexpr int kBvhStack = 48;              // LDS traversal stack entries per lane
constexpr int kTraceBlock = 64;            // threads per traversal block (one wave)
constexpr int kTraceBlocksPerCU = 13;      // resident traversal blocks per CU (LDS bound)

constexpr uint32_t kTagCamera = 1, kTagBsdf = 2, kTagNee = 3, kTagPhoton = 4;

// kernel-argument copy of the octree's scalars (Appendix B members)
struct OctParams {
    float min_bound[3];
    float size_inv[3];
    float scene_scale;
    float density_scale;
    int32_t capacity;
    int32_t split_count;
    int32_t stop_filling;
    int32_t iter;
};

// device-resident octree state updated by atomics
struct OctState {
    int32_t alloc;
    int32_t depth;
    int32_t overflow;
    int32_t rejected;
    unsigned long long block_iter_sum;
    unsigned long long deposits;
    unsigned long long lost;
};

struct Octree {
    int32_t* nodes = nullptr;   // device
    OctState* state = nullptr;  // device
    OctParams prm{};
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

// read-only scene view passed to kernels
struct SceneView {
    const float4* bvh;       // 4 float4 per node (two child boxes + child links)
    const float4* tri;       // 3 float4 per triangle in leaf order; tri[0].w = prim id bits
    const float4* prim_n;    // per prim: unit geometric normal, .w = material id bits
    const int32_t* prim_light; // per prim: light index or -1
    const neb_material* mats;
    const float4* lights;    // 5 float4 per light
    const float* light_cdf;  // inclusive cumulative selection probabilities
    int32_t n_lights;
    float eps;               // ray origin offset along the normal
};

// device counters of one context
struct Counters {
    int32_t qcount[2];       // camera path queues
    int32_t pcount[2];       // photon queues
    int32_t n_vertices;
    int32_t n_events;
    int32_t pad[2];
    unsigned long long paths, vertices, photons, photon_segments, merges, nee_visible, events;
    unsigned long long camera_rays, shadow_rays, photon_rays;
    unsigned long long photon_items, photon_continued, grid_cells, candidates;
    unsigned long long bvh_nodes, bvh_tris;   // traversal work of closest-hit and shadow rays
};

// octree kernels (neb_octree.hip)
hipError_t octree_init_nodes(Octree& o, hipStream_t s);
hipError_t octree_reserve(Octree& o, int64_t n);
void octree_release(Octree& o);
hipError_t octree_increment_xyz(Octree& o, const float* pos, int32_t n, int single, hipStream_t s);
hipError_t octree_increment_vertices(const Octree& o, const float4* vpos, const int32_t* nvert,
                                     int32_t cap, hipStream_t s);
hipError_t octree_increment_slots(const Octree& o, const float4* vpos, const int32_t* slots,
                                  int32_t n_slots, hipStream_t s);
hipError_t octree_density_xyz(const Octree& o, const float* pos, const float* nrm, int32_t n, int robust,
                              float* out, hipStream_t s);
hipError_t octree_clear(const Octree& o, hipStream_t s);
void octree_params_init(OctParams& p, const float smin[3], const float smax[3], int32_t capacity);
void octree_params_set_iteration(OctParams& p, int32_t iter);

}  // namespace neb
