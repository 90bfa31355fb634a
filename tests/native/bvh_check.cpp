// Host check of the BVH builder, built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_sanitizers_cpu.py: seeded scenes
// (random triangles of widely spread sizes, degenerate triangles, a ground
// plane under many boxes that the builder splits, duplicates, one triangle)
// are built, and every node is checked: child slots in range, inner children
// after their parent, leaf runs inside the triangle array and in child order,
// every input triangle referenced, the stack bound within the traversal's.
// Exit status 0 when every check passes.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "trace_layout.h"

namespace {

struct Rng {
    uint64_t s;
    explicit Rng(uint64_t seed) : s(seed * 0x9E3779B97F4A7C15ull + 1) {}
    double next() {
        s ^= s << 13;
        s ^= s >> 7;
        s ^= s << 17;
        return (double)(s >> 11) * (1.0 / 9007199254740992.0);
    }
};

int failures = 0;

void fail(const std::string &scene, const std::string &what) {
    std::fprintf(stderr, "%s: %s\n", scene.c_str(), what.c_str());
    ++failures;
}

void check(const std::string &name, const std::vector<float> &tri9) {
    const int n = (int)(tri9.size() / 9);
    pv::HostBvh4 b;
    std::string err;
    if (!pv::build_bvh4(tri9.data(), n, 0, b, err)) return fail(name, "build failed: " + err);
    if (n == 0) {
        if (!b.nodes.empty() || !b.tris.empty()) fail(name, "nodes for an empty scene");
        return;
    }
    if (b.nodes.empty()) return fail(name, "no nodes");
    if (b.stack_need > pv::kStack4) fail(name, "stack bound above the traversal's");
    if (b.tris.size() > pv::bvh_max_refs(n)) fail(name, "more triangle slots than the stated maximum");
    std::vector<int> seen(n, 0);
    for (const pv::GpuTri &t : b.tris) {
        int id;
        std::memcpy(&id, &t.v0.w, 4);
        if (id < 0 || id >= n) return fail(name, "triangle id out of range");
        seen[id] = 1;
    }
    for (int i = 0; i < n; ++i)
        if (!seen[i]) return fail(name, "triangle " + std::to_string(i) + " in no leaf");
    std::vector<int> reached(b.nodes.size(), 0);
    reached[0] = 1;
    for (size_t k = 0; k < b.nodes.size(); ++k) {
        const pv::GpuNode4 &g = b.nodes[k];
        if (!reached[k]) fail(name, "node " + std::to_string(k) + " unreachable");
        const uint32_t leaf = g.w2.z, base = g.w2.w;
        const uint32_t child[4] = {g.w3.x, g.w3.y, g.w3.z, g.w3.w};
        uint32_t next_off = 0;
        for (int c = 0; c < 4; ++c) {
            const uint32_t lb = (leaf >> (8 * c)) & 0xffu;
            const uint32_t count = lb & 7u, off = lb >> 3;
            const int32_t ch = (int32_t)child[c];
            if (count) {
                if (count > (uint32_t)pv::kLeafMax) fail(name, "leaf larger than the leaf maximum");
                if (off != next_off) fail(name, "leaf runs not consecutive in child order");
                next_off = off + count;
                if ((size_t)base + off + count > b.tris.size()) fail(name, "leaf run past the triangle array");
                if ((uint32_t)ch != base + off) fail(name, "leaf child is not its first triangle");
            } else if (ch >= 0) {
                if ((size_t)ch >= b.nodes.size()) {
                    fail(name, "inner child out of range");
                } else {
                    if ((size_t)ch <= k) fail(name, "inner child not after its parent");
                    reached[ch] = 1;
                }
            } else if (ch != -1) {
                fail(name, "empty slot not marked -1");
            }
        }
    }
}

void add_tri(std::vector<float> &v, const float *p) { v.insert(v.end(), p, p + 9); }

}  // namespace

int main() {
    check("empty", {});
    {
        std::vector<float> v;
        const float t[9] = {0, 0, 0, 1, 0, 0, 0, 1, 0};
        add_tri(v, t);
        check("one triangle", v);
    }
    for (int n : {2, 7, 100, 5000}) {
        Rng r(n);
        std::vector<float> v;
        for (int i = 0; i < n; ++i) {
            const double size = std::exp(std::log(1e-4) + r.next() * (std::log(50.0) - std::log(1e-4)));
            const double cx = 100 * r.next(), cy = 100 * r.next(), cz = 100 * r.next();
            float t[9];
            for (int k = 0; k < 9; ++k) t[k] = (float)((k % 3 == 0 ? cx : k % 3 == 1 ? cy : cz) + size * (r.next() - 0.5));
            add_tri(v, t);
        }
        check("random " + std::to_string(n), v);
    }
    {
        // degenerate: zero area (collinear), a point, the same triangle many times
        std::vector<float> v;
        const float line[9] = {0, 0, 0, 1, 1, 1, 2, 2, 2}, point[9] = {3, 3, 3, 3, 3, 3, 3, 3, 3};
        const float same[9] = {5, 0, 0, 6, 0, 0, 5, 1, 0};
        for (int i = 0; i < 40; ++i) add_tri(v, line);
        for (int i = 0; i < 40; ++i) add_tri(v, point);
        for (int i = 0; i < 200; ++i) add_tri(v, same);
        check("degenerate", v);
    }
    {
        // a ground plane of two triangles under 2,000 small boxes (12 triangles each)
        std::vector<float> v;
        const float g0[9] = {0, 0, 0, 64, 0, 0, 64, 0, 64}, g1[9] = {0, 0, 0, 64, 0, 64, 0, 0, 64};
        add_tri(v, g0);
        add_tri(v, g1);
        Rng r(7);
        for (int i = 0; i < 2000; ++i) {
            const float x = (float)(64 * r.next()), z = (float)(64 * r.next()), h = (float)(0.5 + 8 * r.next());
            const float a = 0.4f;
            const float c[8][3] = {{x, 0, z}, {x + a, 0, z}, {x + a, 0, z + a}, {x, 0, z + a},
                                   {x, h, z}, {x + a, h, z}, {x + a, h, z + a}, {x, h, z + a}};
            const int f[12][3] = {{0, 1, 2}, {0, 2, 3}, {4, 6, 5}, {4, 7, 6}, {0, 4, 5}, {0, 5, 1},
                                  {1, 5, 6}, {1, 6, 2}, {2, 6, 7}, {2, 7, 3}, {3, 7, 4}, {3, 4, 0}};
            for (auto &tri : f) {
                float t[9];
                for (int vtx = 0; vtx < 3; ++vtx)
                    for (int k = 0; k < 3; ++k) t[3 * vtx + k] = c[tri[vtx]][k];
                add_tri(v, t);
            }
        }
        check("ground and boxes", v);
    }
    {
        // a non-finite coordinate is refused
        std::vector<float> v = {0, 0, 0, 1, 0, 0, 0, NAN, 0};
        pv::HostBvh4 b;
        std::string err;
        if (pv::build_bvh4(v.data(), 1, 0, b, err) || err.empty()) fail("non-finite", "not refused");
    }
    if (failures) std::fprintf(stderr, "%d check(s) failed\n", failures);
    else std::printf("bvh builder: every check passed\n");
    return failures ? 1 : 0;
}
