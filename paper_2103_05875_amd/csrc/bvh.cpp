// Host BVH builder: triangles whose boxes are large against the scene's
// average are first split into several references with clipped boxes (early
// split clipping: a ground plane spanning the scene would otherwise put a
// scene-sized box under the root that every ray enters); then a binned
// surface-area heuristic over reference centroids builds a binary tree (a
// node whose remaining depth budget is tight switches to balanced median
// splits), collapsed into the 4-wide quantized nodes of the GPU traversal
// with a proved bound on its stack. A split triangle appears in several
// leaves; every copy carries the same id, so closest and any hit are
// unchanged.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace pv {
namespace {

struct Box {
    float lo[3], hi[3];
    void reset() {
        for (int k = 0; k < 3; ++k) {
            lo[k] = INFINITY;
            hi[k] = -INFINITY;
        }
    }
    void grow(const float *p) {
        for (int k = 0; k < 3; ++k) {
            lo[k] = std::min(lo[k], p[k]);
            hi[k] = std::max(hi[k], p[k]);
        }
    }
    void grow(const Box &b) {
        for (int k = 0; k < 3; ++k) {
            lo[k] = std::min(lo[k], b.lo[k]);
            hi[k] = std::max(hi[k], b.hi[k]);
        }
    }
    bool empty() const { return !(lo[0] <= hi[0]); }
    float half_area() const {
        if (empty()) return 0.f;
        float dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
        return dx * dy + dy * dz + dz * dx;
    }
};

struct Ref {
    Box box;
    float c[3];
    int tri;
};

// Box of the part of triangle t (9 floats) inside box clip: the triangle
// clipped against the six planes (Sutherland-Hodgman), then bounded.
Box clipped_box(const float *t, const Box &clip) {
    float poly[2][12][3];
    int n = 3, cur = 0;
    for (int v = 0; v < 3; ++v)
        for (int k = 0; k < 3; ++k) poly[0][v][k] = t[3 * v + k];
    for (int axis = 0; axis < 3 && n > 0; ++axis)
        for (int side = 0; side < 2 && n > 0; ++side) {
            const float bound = side ? clip.hi[axis] : clip.lo[axis];
            auto inside = [&](const float *p) { return side ? p[axis] <= bound : p[axis] >= bound; };
            int m = 0;
            for (int i = 0; i < n; ++i) {
                const float *a = poly[cur][i], *c = poly[cur][(i + 1) % n];
                const bool ia = inside(a), ic = inside(c);
                if (ia && m < 12) {
                    for (int k = 0; k < 3; ++k) poly[cur ^ 1][m][k] = a[k];
                    ++m;
                }
                if (ia != ic && m < 12) {
                    const float s = (bound - a[axis]) / (c[axis] - a[axis]);
                    for (int k = 0; k < 3; ++k) poly[cur ^ 1][m][k] = a[k] + s * (c[k] - a[k]);
                    poly[cur ^ 1][m][axis] = bound;
                    ++m;
                }
            }
            n = m;
            cur ^= 1;
        }
    Box out;
    out.reset();
    for (int i = 0; i < n; ++i) out.grow(poly[cur][i]);
    // clipping rounds: never let the box leave the triangle's own box
    Box own;
    own.reset();
    for (int v = 0; v < 3; ++v) own.grow(t + 3 * v);
    for (int k = 0; k < 3 && !out.empty(); ++k) {
        out.lo[k] = std::max(out.lo[k], own.lo[k]);
        out.hi[k] = std::min(out.hi[k], own.hi[k]);
    }
    return out;
}

// Splits the references whose box half-area exceeds 16 times the mean (and
// 1/4096 of the scene's) at the middle of their longest axis, clipping the
// triangle to each half, until every box is small enough or the references
// number 2n. Deterministic (first-in, first-out).
void split_large(const float *tri9, int n, const Box &scene, std::vector<Ref> &refs) {
    double mean = 0.0;
    for (const Ref &r : refs) mean += r.box.half_area();
    mean /= std::max(n, 1);
    const float limit = std::max((float)(16.0 * mean), scene.half_area() / 4096.f);
    const size_t budget = bvh_max_refs(n);
    std::vector<Ref> out, queue;
    out.reserve(budget);
    for (const Ref &r : refs) (r.box.half_area() > limit ? queue : out).push_back(r);
    for (size_t qi = 0; qi < queue.size(); ++qi) {
        const Ref r = queue[qi];
        const size_t pending = queue.size() - qi - 1;
        if (r.box.half_area() <= limit || out.size() + pending + 2 > budget) {
            out.push_back(r);
            continue;
        }
        int axis = 0;
        for (int k = 1; k < 3; ++k)
            if (r.box.hi[k] - r.box.lo[k] > r.box.hi[axis] - r.box.lo[axis]) axis = k;
        const float mid = 0.5f * (r.box.lo[axis] + r.box.hi[axis]);
        for (int half = 0; half < 2; ++half) {
            Box h = r.box;
            (half ? h.lo : h.hi)[axis] = mid;
            Ref c;
            c.tri = r.tri;
            c.box = clipped_box(tri9 + 9 * (size_t)r.tri, h);
            if (c.box.empty()) continue;
            for (int k = 0; k < 3; ++k) c.c[k] = 0.5f * (c.box.lo[k] + c.box.hi[k]);
            queue.push_back(c);
        }
    }
    refs.swap(out);
}

struct BNode {
    Box box;
    int left = -1, right = -1;
    int first = 0, count = 0;  // leaf range in refs
};

int levels_needed(int count) {
    int leaves = (count + kLeafMax - 1) / kLeafMax;
    int d = 0;
    while ((1 << d) < leaves) ++d;
    return d;
}

class Builder {
  public:
    Builder(std::vector<Ref> &refs, int max_depth = kMaxDepth) : refs_(refs), limit_(max_depth) {}

    int build(int first, int count, int depth) {
        int id = (int)nodes_.size();
        nodes_.emplace_back();
        Box box, cbox;
        box.reset();
        cbox.reset();
        for (int i = first; i < first + count; ++i) {
            box.grow(refs_[i].box);
            cbox.grow(refs_[i].c);
        }
        nodes_[id].box = box;
        max_depth_ = std::max(max_depth_, depth);
        if (count <= 1 || (count <= kLeafMax && prefer_leaf(first, count, box))) {
            make_leaf(id, first, count);
            return id;
        }
        int mid = -1;
        bool tight = depth + levels_needed(count) + 1 >= limit_;
        if (!tight) mid = sah_split(first, count, box, cbox);
        if (mid <= first || mid >= first + count) mid = median_split(first, count, cbox);
        int l = build(first, mid - first, depth + 1);
        int r = build(mid, first + count - mid, depth + 1);
        nodes_[id].left = l;
        nodes_[id].right = r;
        return id;
    }

    std::vector<BNode> nodes_;
    int max_depth_ = 0;

  private:
    void make_leaf(int id, int first, int count) {
        nodes_[id].first = first;
        nodes_[id].count = count;
    }

    bool prefer_leaf(int first, int count, const Box &box) {
        // leaf cost N against the best binned split; small leaves are kept
        // when splitting does not pay
        if (count <= 2) return true;
        Box cb;
        cb.reset();
        for (int i = first; i < first + count; ++i) cb.grow(refs_[i].c);
        float best;
        int axis, bin;
        if (!best_bin(first, count, box, cb, best, axis, bin)) return true;
        return (float)count <= best;
    }

    // 128 centroid bins per axis: against 16 bins, 10% fewer node visits
    // on the city's primary rays for under a second of build per 200k
    // triangles (static scenes are built once)
    static constexpr int kBins = 128;

    bool best_bin(int first, int count, const Box &box, const Box &cbox, float &best_cost, int &best_axis,
                  int &best_split) {
        best_cost = INFINITY;
        best_axis = -1;
        best_split = -1;
        float parent = box.half_area();
        if (parent <= 0.f) parent = 1.f;
        for (int a = 0; a < 3; ++a) {
            float ext = cbox.hi[a] - cbox.lo[a];
            if (!(ext > 0.f)) continue;
            Box bb[kBins];
            int bn[kBins] = {0};
            for (int b = 0; b < kBins; ++b) bb[b].reset();
            float scale = kBins / ext;
            for (int i = first; i < first + count; ++i) {
                int b = (int)((refs_[i].c[a] - cbox.lo[a]) * scale);
                b = std::min(std::max(b, 0), kBins - 1);
                bb[b].grow(refs_[i].box);
                bn[b]++;
            }
            float right_area[kBins];
            int right_n[kBins];
            Box acc;
            acc.reset();
            int n = 0;
            for (int b = kBins - 1; b > 0; --b) {
                acc.grow(bb[b]);
                n += bn[b];
                right_area[b] = acc.half_area();
                right_n[b] = n;
            }
            acc.reset();
            n = 0;
            for (int b = 0; b < kBins - 1; ++b) {
                acc.grow(bb[b]);
                n += bn[b];
                int nr = right_n[b + 1];
                if (n == 0 || nr == 0) continue;
                float cost = 1.0f + (acc.half_area() * n + right_area[b + 1] * nr) / parent;
                if (cost < best_cost) {
                    best_cost = cost;
                    best_axis = a;
                    best_split = b;
                }
            }
        }
        return best_axis >= 0;
    }

    int sah_split(int first, int count, const Box &box, const Box &cbox) {
        float cost;
        int axis, split;
        if (!best_bin(first, count, box, cbox, cost, axis, split)) return -1;
        float ext = cbox.hi[axis] - cbox.lo[axis];
        float scale = kBins / ext;
        auto it = std::partition(refs_.begin() + first, refs_.begin() + first + count, [&](const Ref &r) {
            int b = (int)((r.c[axis] - cbox.lo[axis]) * scale);
            b = std::min(std::max(b, 0), kBins - 1);
            return b <= split;
        });
        return (int)(it - refs_.begin());
    }

    int median_split(int first, int count, const Box &cbox) {
        int axis = 0;
        for (int a = 1; a < 3; ++a)
            if (cbox.hi[a] - cbox.lo[a] > cbox.hi[axis] - cbox.lo[axis]) axis = a;
        int mid = first + count / 2;
        std::nth_element(refs_.begin() + first, refs_.begin() + mid, refs_.begin() + first + count,
                         [&](const Ref &x, const Ref &y) {
                             if (x.c[axis] != y.c[axis]) return x.c[axis] < y.c[axis];
                             return x.tri < y.tri;
                         });
        return mid;
    }

    std::vector<Ref> &refs_;
    int limit_;
};

float bits_as_float(int v) {
    float f;
    std::memcpy(&f, &v, 4);
    return f;
}

}  // namespace

namespace {

struct Collapse {
    const std::vector<BNode> &bn;
    // tree of 4-wide nodes in creation order: children slots hold either a
    // leaf BNode (count > 0) or a 4-wide node id (count == 0)
    struct N4 {
        int nk = 0;
        int kid_bnode[4] = {-1, -1, -1, -1};
        int kid_n4[4] = {-1, -1, -1, -1};
    };
    std::vector<N4> tree;
    std::vector<GpuNode4> out;
    std::vector<int> leaf_order;  // output triangle slot -> builder reference index
    Collapse(const std::vector<BNode> &b) : bn(b) {}

    // children of a 4-wide node: expand the largest inner child until 4
    void gather(int id, std::vector<int> &kids) const {
        kids = {bn[id].left, bn[id].right};
        while (kids.size() < 4) {
            int best = -1;
            float area = -1.f;
            for (size_t i = 0; i < kids.size(); ++i)
                if (bn[kids[i]].count == 0 && bn[kids[i]].box.half_area() > area) {
                    area = bn[kids[i]].box.half_area();
                    best = (int)i;
                }
            if (best < 0) break;
            int k = kids[best];
            kids.erase(kids.begin() + best);
            kids.push_back(bn[k].left);
            kids.push_back(bn[k].right);
        }
    }

    // builds the subtree of BNode id; returns its N4 id, depth and the
    // worst-case number of stack entries its traversal can add
    int build(int id, int &depth, int &need) {
        std::vector<int> kids;
        if (bn[id].count > 0)
            kids = {id};  // single-leaf root
        else
            gather(id, kids);
        const int me = (int)tree.size();
        tree.emplace_back();
        int sub_depth = 0, sub_need = 0, inner = 0;
        for (size_t c = 0; c < kids.size(); ++c) {
            tree[me].kid_bnode[c] = kids[c];
            if (bn[kids[c]].count == 0) {
                int cd, cn;
                const int ci = build(kids[c], cd, cn);
                tree[me].kid_n4[c] = ci;
                sub_depth = std::max(sub_depth, cd);
                sub_need = std::max(sub_need, cn);
                ++inner;
            }
        }
        tree[me].nk = (int)kids.size();
        depth = sub_depth + 1;
        // descending into one inner child leaves at most the other inner
        // children of this node on the stack
        need = inner > 0 ? sub_need + (inner - 1) : 0;
        return me;
    }

    // nodes numbered breadth first, so the top levels are a prefix; the
    // triangles of a node's leaf children are stored back to back in slot
    // order, so one node's leaf triangles span at most 4 * kLeafMax slots
    void emit(int root) {
        std::vector<int> order, index(tree.size(), -1);
        order.push_back(root);
        for (size_t i = 0; i < order.size(); ++i)
            for (int c = 0; c < tree[order[i]].nk; ++c)
                if (tree[order[i]].kid_n4[c] >= 0) order.push_back(tree[order[i]].kid_n4[c]);
        for (size_t i = 0; i < order.size(); ++i) index[order[i]] = (int)i;
        out.resize(order.size());
        for (size_t i = 0; i < order.size(); ++i) {
            const N4 &t = tree[order[i]];
            int child[4] = {-1, -1, -1, -1}, count[4] = {0, 0, 0, 0}, offset[4] = {0, 0, 0, 0};
            int base = -1;
            Box box[4];
            for (int c = 0; c < t.nk; ++c) {
                const BNode &k = bn[t.kid_bnode[c]];
                box[c] = k.box;
                if (k.count > 0) {
                    child[c] = (int)leaf_order.size();
                    count[c] = k.count;
                    if (base < 0) base = child[c];
                    offset[c] = child[c] - base;
                    for (int r = k.first; r < k.first + k.count; ++r) leaf_order.push_back(r);
                } else {
                    child[c] = index[t.kid_n4[c]];
                }
            }
            quantize(out[i], (size_t)t.nk, box, child, count, offset, base);
        }
    }

    void quantize(GpuNode4 &g, size_t nk, const Box *box, const int *child, const int *count, const int *offset,
                  int base) const {
        float L[3], H[3];
        for (int a = 0; a < 3; ++a) {
            L[a] = INFINITY;
            H[a] = -INFINITY;
            for (size_t c = 0; c < nk; ++c) {
                L[a] = std::min(L[a], box[c].lo[a]);
                H[a] = std::max(H[a], box[c].hi[a]);
            }
        }
        int eb[3];
        double scale[3];
        for (int a = 0; a < 3; ++a) {
            const double ext = (double)H[a] - (double)L[a];
            int e = -126;
            while (std::ldexp(255.0, e) < ext) ++e;
            eb[a] = e + 127;
            scale[a] = std::ldexp(1.0, e);
        }
        uint8_t q[6][4];
        for (int c = 0; c < 4; ++c)
            for (int a = 0; a < 3; ++a) {
                if ((size_t)c < nk) {
                    double lo = std::floor(((double)box[c].lo[a] - L[a]) / scale[a]);
                    double hi = std::ceil(((double)box[c].hi[a] - L[a]) / scale[a]);
                    // outward: decoded lo <= box lo, decoded hi >= box hi
                    while (lo > 0 && L[a] + lo * scale[a] > box[c].lo[a]) lo -= 1;
                    while (hi < 255 && L[a] + hi * scale[a] < box[c].hi[a]) hi += 1;
                    q[2 * a][c] = (uint8_t)std::min(std::max(lo, 0.0), 255.0);
                    q[2 * a + 1][c] = (uint8_t)std::min(std::max(hi, 0.0), 255.0);
                } else {
                    q[2 * a][c] = 255;  // empty: lo above hi
                    q[2 * a + 1][c] = 0;
                }
            }
        auto pack = [](const uint8_t *v) {
            return (uint32_t)v[0] | ((uint32_t)v[1] << 8) | ((uint32_t)v[2] << 16) | ((uint32_t)v[3] << 24);
        };
        uint32_t fb[3];
        std::memcpy(fb, L, 12);
        g.w0 = make_uint4(fb[0], fb[1], fb[2], (uint32_t)eb[0] | ((uint32_t)eb[1] << 8) | ((uint32_t)eb[2] << 16));
        g.w1 = make_uint4(pack(q[0]), pack(q[1]), pack(q[2]), pack(q[3]));
        // leaf byte: triangle count (bits 0-2) and the leaf's first slot
        // relative to the node's first leaf slot (bits 3-6); 0 = inner / empty
        uint8_t cnt[4];
        for (int c = 0; c < 4; ++c) cnt[c] = (uint8_t)(count[c] | (count[c] > 0 ? offset[c] << 3 : 0));
        g.w2 = make_uint4(pack(q[4]), pack(q[5]), pack(cnt), (uint32_t)(base < 0 ? 0 : base));
        g.w3 = make_uint4((uint32_t)child[0], (uint32_t)child[1], (uint32_t)child[2], (uint32_t)child[3]);
    }
};

}  // namespace

bool build_bvh4(const float *tri9, int n, int id_base, HostBvh4 &out, std::string &err) {
    out.nodes.clear();
    out.tris.clear();
    out.depth = out.stack_need = 0;
    if (n <= 0) return true;
    for (int limit = kMaxDepth; limit >= 8; limit -= 2) {
        std::vector<Ref> refs(n);
        Box scene;
        scene.reset();
        for (int i = 0; i < n; ++i) {
            const float *t = tri9 + 9 * (size_t)i;
            for (int k = 0; k < 9; ++k)
                if (!std::isfinite(t[k])) {
                    err = "triangle " + std::to_string(i) + " has a non-finite coordinate";
                    return false;
                }
            refs[i].box.reset();
            for (int v = 0; v < 3; ++v) refs[i].box.grow(t + 3 * v);
            for (int k = 0; k < 3; ++k) refs[i].c[k] = (t[k] + t[3 + k] + t[6 + k]) / 3.0f;
            refs[i].tri = i;
            scene.grow(refs[i].box);
        }
        split_large(tri9, n, scene, refs);
        const int m = (int)refs.size();
        if (levels_needed(m) + 2 > limit) break;
        Builder b(refs, limit);
        b.build(0, m, 0);
        // conservative padding of every box (rounding of the slab test)
        float diag = 0.f;
        for (int k = 0; k < 3; ++k) diag += (scene.hi[k] - scene.lo[k]) * (scene.hi[k] - scene.lo[k]);
        diag = std::sqrt(diag);
        const float pad_abs = diag * 9.5367431640625e-7f;
        for (BNode &nd : b.nodes_)
            for (int k = 0; k < 3; ++k) {
                nd.box.lo[k] -= pad_abs + std::fabs(nd.box.lo[k]) * 2.384185791015625e-7f;
                nd.box.hi[k] += pad_abs + std::fabs(nd.box.hi[k]) * 2.384185791015625e-7f;
            }
        Collapse col(b.nodes_);
        int depth, need;
        const int root = col.build(0, depth, need);
        if (need > kStack4) continue;  // lower the binary depth limit and retry
        col.emit(root);
        out.nodes = std::move(col.out);
        out.depth = depth;
        out.stack_need = need;
        if ((int)col.leaf_order.size() != m) {
            err = "internal: leaf triangles do not cover the scene";
            return false;
        }
        out.tris.resize(m);
        for (int i = 0; i < m; ++i) {
            const int src = refs[col.leaf_order[i]].tri;
            const float *t = tri9 + 9 * (size_t)src;
            GpuTri g;
            g.v0 = make_float4(t[0], t[1], t[2], bits_as_float(id_base + src));
            g.v1 = make_float4(t[3], t[4], t[5], 0.f);
            g.v2 = make_float4(t[6], t[7], t[8], 0.f);
            out.tris[i] = g;
        }
        return true;
    }
    err = "cannot bound the traversal stack of this scene";
    return false;
}

}  // namespace pv
