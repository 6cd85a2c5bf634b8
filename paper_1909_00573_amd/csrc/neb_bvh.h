// Host BVH builder interface.
#pragma once
#include <stdint.h>

#include <vector>

namespace neb {

struct BvhHost {
    // 16 floats per node: child0 box (lo xyz, hi xyz), child1 box, then four
    // int32 (child0 link, child1 link, child0 leaf count, child1 leaf count);
    // a count > 0 marks a leaf whose link is the first triangle, count 0 an
    // inner node whose link is a node index, link -1 an empty child.
    std::vector<float> nodes;
    // 12 floats per triangle in leaf order: v0 (w = prim id bits), v1, v2
    std::vector<float> tris;
    int n_nodes = 0;
    int max_depth = 0;
};

bool build_bvh(const float* vertices, int32_t nv, const int32_t* tris, int32_t nt, BvhHost& out);

}  // namespace neb
