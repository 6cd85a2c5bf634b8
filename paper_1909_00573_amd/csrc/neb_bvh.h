// Host BVH builder interface.
#pragma once
#include <stdint.h>

#include <vector>

namespace neb {

struct BvhHost {
    // 32 floats per node (128 bytes), up to four children: lo x, lo y, lo z,
    // hi x, hi y, hi z of the four child boxes (four floats each, child c in
    // lane c), then four int32 links and four int32 leaf counts; a count > 0
    // marks a leaf whose link is its first triangle, count 0 an inner node
    // whose link is a node index, link -1 an empty slot.
    std::vector<float> nodes;
    // 12 floats per triangle in leaf order: v0 (w = prim id bits), v1, v2
    std::vector<float> tris;
    int n_nodes = 0;
    int stack_need = 0;  // traversal stack entries the deepest descent needs
};

bool build_bvh(const float* vertices, int32_t nv, const int32_t* tris, int32_t nt, BvhHost& out);

}  // namespace neb
