// Host BVH builder: binned SAH over triangle centroids (32 bins on each
// axis, the cheapest split of the three), collapsed into four-wide
// 128-byte nodes that hold the boxes of up to four children (one node
// fetch, one cache line, tests four boxes).  Subtrees deeper than kSahDepth
// switch to object-median splits so that the traversal stack stays short.
#include "neb_bvh.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace neb {

namespace {

struct Box {
    float lo[3] = {INFINITY, INFINITY, INFINITY};
    float hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    void grow(const float* p) {
        for (int i = 0; i < 3; ++i) {
            lo[i] = std::min(lo[i], p[i]);
            hi[i] = std::max(hi[i], p[i]);
        }
    }
    void grow(const Box& b) {
        for (int i = 0; i < 3; ++i) {
            lo[i] = std::min(lo[i], b.lo[i]);
            hi[i] = std::max(hi[i], b.hi[i]);
        }
    }
    float area() const {
        float d[3];
        for (int i = 0; i < 3; ++i) d[i] = std::max(0.0f, hi[i] - lo[i]);
        return 2.0f * (d[0] * d[1] + d[1] * d[2] + d[0] * d[2]);
    }
};

struct BuildNode {
    Box box;
    int child[2] = {-1, -1};  // internal: build-node indices
    int first = 0, count = 0; // leaf: range in the prim index array
};

constexpr int kBins = 32;
constexpr int kMaxLeaf = 4;
constexpr int kSahDepth = 20;

struct Builder {
    std::vector<Box> pbox;
    std::vector<float> cent;  // 3 per prim
    std::vector<int> idx;
    std::vector<BuildNode> nodes;

    int make_leaf(int first, int count, const Box& b) {
        BuildNode n;
        n.box = b;
        n.first = first;
        n.count = count;
        nodes.push_back(n);
        return (int)nodes.size() - 1;
    }

    // returns build-node index
    int build(int first, int count, int depth) {
        Box b, cb;
        for (int i = first; i < first + count; ++i) {
            b.grow(pbox[idx[i]]);
            cb.grow(&cent[3 * idx[i]]);
        }
        if (count <= 1) return make_leaf(first, count, b);
        int axis = 0;
        float ext[3];
        for (int i = 0; i < 3; ++i) ext[i] = cb.hi[i] - cb.lo[i];
        if (ext[1] > ext[axis]) axis = 1;
        if (ext[2] > ext[axis]) axis = 2;
        int mid = -1;
        if (ext[axis] <= 0.0f) {
            if (count <= kMaxLeaf) return make_leaf(first, count, b);
            mid = first + count / 2;  // identical centroids: split the list
        } else if (depth >= kSahDepth) {
            if (count <= kMaxLeaf) return make_leaf(first, count, b);
            mid = first + count / 2;
            std::nth_element(idx.begin() + first, idx.begin() + mid, idx.begin() + first + count,
                             [&](int a, int c) { return cent[3 * a + axis] < cent[3 * c + axis]; });
        } else {
            // binned SAH on each axis with extent; the cheapest split wins
            float best = INFINITY;
            int best_k = -1, best_axis = axis;
            for (int ax = 0; ax < 3; ++ax) {
                if (ext[ax] <= 0.0f) continue;
                Box bb[kBins];
                int bc[kBins] = {0};
                const float scale = kBins / ext[ax];
                for (int i = first; i < first + count; ++i) {
                    const int p = idx[i];
                    int k = std::min(kBins - 1, std::max(0, (int)((cent[3 * p + ax] - cb.lo[ax]) * scale)));
                    bc[k]++;
                    bb[k].grow(pbox[p]);
                }
                float right_area[kBins];
                int right_cnt[kBins];
                Box acc;
                int n = 0;
                for (int k = kBins - 1; k > 0; --k) {
                    acc.grow(bb[k]);
                    n += bc[k];
                    right_area[k] = acc.area();
                    right_cnt[k] = n;
                }
                Box lacc;
                int ln = 0;
                for (int k = 1; k < kBins; ++k) {
                    lacc.grow(bb[k - 1]);
                    ln += bc[k - 1];
                    if (ln == 0 || right_cnt[k] == 0) continue;
                    float c = lacc.area() * ln + right_area[k] * right_cnt[k];
                    if (c < best) {
                        best = c;
                        best_k = k;
                        best_axis = ax;
                    }
                }
            }
            const float scale = kBins / ext[best_axis];
            auto bin_of = [&](int p) {
                int k = (int)((cent[3 * p + best_axis] - cb.lo[best_axis]) * scale);
                return std::min(kBins - 1, std::max(0, k));
            };
            float leaf_cost = b.area() * count;
            float split_cost = b.area() * 0.5f + best;  // traversal ~ half a triangle test
            if (count <= kMaxLeaf && (best_k < 0 || split_cost >= leaf_cost)) return make_leaf(first, count, b);
            if (best_k < 0) {
                mid = first + count / 2;
                std::nth_element(idx.begin() + first, idx.begin() + mid, idx.begin() + first + count,
                                 [&](int a, int c) { return cent[3 * a + axis] < cent[3 * c + axis]; });
            } else {
                auto it = std::partition(idx.begin() + first, idx.begin() + first + count,
                                         [&](int p) { return bin_of(p) < best_k; });
                mid = (int)(it - idx.begin());
                if (mid == first || mid == first + count) mid = first + count / 2;
            }
        }
        int me = (int)nodes.size();
        nodes.emplace_back();
        nodes[me].box = b;
        int l = build(first, mid - first, depth + 1);
        int r = build(mid, first + count - mid, depth + 1);
        nodes[me].child[0] = l;
        nodes[me].child[1] = r;
        return me;
    }
};

void put_box(float* dst, const Box& b) {
    dst[0] = b.lo[0];
    dst[1] = b.lo[1];
    dst[2] = b.lo[2];
    dst[3] = b.hi[0];
    dst[4] = b.hi[1];
    dst[5] = b.hi[2];
}

}  // namespace

bool build_bvh(const float* vertices, int32_t nv, const int32_t* tris, int32_t nt, BvhHost& out) {
    (void)nv;
    Builder B;
    B.pbox.resize(nt);
    B.cent.resize(3 * (size_t)nt);
    B.idx.resize(nt);
    for (int32_t t = 0; t < nt; ++t) {
        for (int k = 0; k < 3; ++k) B.pbox[t].grow(vertices + 3 * (size_t)tris[3 * t + k]);
        for (int i = 0; i < 3; ++i) B.cent[3 * t + i] = 0.5f * (B.pbox[t].lo[i] + B.pbox[t].hi[i]);
        B.idx[t] = t;
    }
    B.nodes.reserve(2 * (size_t)nt);
    int root = B.build(0, nt, 0);

    // Collapse to four-wide nodes: a binary inner node gathers its children,
    // and while it holds fewer than four, the inner one with the largest
    // surface area is replaced by its two children.  One device node (one
    // 128-byte line) then tests up to four boxes, about halving the
    // dependent node fetches of a ray.  A leaf root gets a parent of its own.
    auto inner = [&](int n) { return B.nodes[n].child[0] >= 0; };
    auto collapse = [&](int n, int* ch) {
        int k = 2;
        ch[0] = B.nodes[n].child[0];
        ch[1] = B.nodes[n].child[1];
        while (k < 4) {
            int pick = -1;
            float best = -1.0f;
            for (int i = 0; i < k; ++i)
                if (inner(ch[i]) && B.nodes[ch[i]].box.area() > best) {
                    best = B.nodes[ch[i]].box.area();
                    pick = i;
                }
            if (pick < 0) break;
            const int p = ch[pick];
            ch[pick] = B.nodes[p].child[0];
            ch[k++] = B.nodes[p].child[1];
        }
        return k;
    };
    // device order: depth first, a node before its subtrees
    std::vector<int> order;
    std::vector<int> kids;  // four per wide node (-1: empty slot)
    std::vector<int> dev_of(B.nodes.size(), -1);
    if (inner(root)) {
        std::vector<int> stack{root};
        while (!stack.empty()) {
            const int n = stack.back();
            stack.pop_back();
            dev_of[n] = (int)order.size();
            order.push_back(n);
            int ch[4] = {-1, -1, -1, -1};
            collapse(n, ch);
            kids.insert(kids.end(), ch, ch + 4);
            for (int c = 3; c >= 0; --c)
                if (ch[c] >= 0 && inner(ch[c])) stack.push_back(ch[c]);
        }
    } else {
        order.push_back(-1);
        kids.insert(kids.end(), {root, -1, -1, -1});
    }
    const int n_dev = (int)order.size();
    // traversal stack entries a ray can need: a visit pushes all but the
    // nearest of the inner children it enters, so below a node the stack
    // grows by (inner children - 1) plus the most any inner child needs
    std::vector<int> need(n_dev, 0);
    for (int d = n_dev - 1; d >= 0; --d) {
        int ic = 0, sub = 0;
        for (int c = 0; c < 4; ++c) {
            const int ch = kids[4 * (size_t)d + c];
            if (ch >= 0 && inner(ch)) {
                ++ic;
                sub = std::max(sub, need[dev_of[ch]]);
            }
        }
        need[d] = std::max(0, ic - 1) + sub;
    }
    out.stack_need = need[0];

    out.nodes.assign(32 * (size_t)n_dev, 0.0f);
    out.tris.assign(12 * (size_t)nt, 0.0f);
    int tri_cursor = 0;
    auto emit_leaf = [&](int bn, int& first, int& count) {
        const BuildNode& L = B.nodes[bn];
        first = tri_cursor;
        count = L.count;
        for (int i = L.first; i < L.first + L.count; ++i) {
            int p = B.idx[i];
            float* dst = &out.tris[12 * (size_t)tri_cursor];
            for (int k = 0; k < 3; ++k) {
                const float* v = vertices + 3 * (size_t)tris[3 * p + k];
                dst[4 * k + 0] = v[0];
                dst[4 * k + 1] = v[1];
                dst[4 * k + 2] = v[2];
                dst[4 * k + 3] = 0.0f;
            }
            int32_t pid = p;
            std::memcpy(&dst[3], &pid, 4);
            ++tri_cursor;
        }
    };
    for (int d = 0; d < n_dev; ++d) {
        float* dst = &out.nodes[32 * (size_t)d];
        int32_t link[4] = {-1, -1, -1, -1}, cnt[4] = {0, 0, 0, 0};
        for (int c = 0; c < 4; ++c) {
            const int ch = kids[4 * (size_t)d + c];
            Box b;  // an empty slot (link -1) is never entered; its box is zero
            if (ch >= 0) {
                b = B.nodes[ch].box;
                if (inner(ch)) {
                    link[c] = dev_of[ch];
                } else {
                    emit_leaf(ch, link[c], cnt[c]);
                    if (cnt[c] == 0) link[c] = -1;
                }
            }
            for (int a = 0; a < 3; ++a) {
                dst[4 * a + c] = link[c] < 0 ? 0.0f : b.lo[a];
                dst[12 + 4 * a + c] = link[c] < 0 ? 0.0f : b.hi[a];
            }
        }
        std::memcpy(dst + 24, link, sizeof(link));
        std::memcpy(dst + 28, cnt, sizeof(cnt));
    }
    out.n_nodes = n_dev;
    return tri_cursor == nt;
}

}  // namespace neb
