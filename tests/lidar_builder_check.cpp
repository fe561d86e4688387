// Host check of the LiDAR hierarchy builder (no GPU use): for seeded primitive sets (uniform,
// clustered, on a line, all centres equal; 5 to 200k primitives) every primitive sits in
// exactly one leaf of at most kLeafSize, the depth-first layout holds (left child next, right
// child after the left subtree, skip = end of the subtree), every node box holds its
// primitives' boxes and centres, and the depth stays within the tracer's stack.
#include "../paper_2507_21981_amd/csrc/gsr_lidar.hip"

#include <cstdio>
#include <functional>
#include <random>

using namespace gsr;

static int fails = 0;
#define CHECK(c, ...)                     \
    do {                                  \
        if (!(c)) {                       \
            printf("FAIL: " __VA_ARGS__); \
            printf("\n");                 \
            if (++fails > 20) exit(1);    \
        }                                 \
    } while (0)

int main() {
    std::mt19937 g(11);
    for (int trial = 0; trial < 40; ++trial) {
        std::uniform_int_distribution<int> nd(5, trial < 10 ? 40 : (trial < 35 ? 5000 : 200000));
        const int m = nd(g);
        std::normal_distribution<float> N(0.f, 1.f);
        std::uniform_real_distribution<float> U(0.f, 1.f);
        std::vector<float> box, cen;
        for (int i = 0; i < m; ++i) {
            float c[3];
            for (int j = 0; j < 3; ++j) {
                if (trial % 5 == 0) c[j] = 0.25f;
                else if (trial % 5 == 1) c[j] = (i % 3 == 0) ? 10.f + 0.01f * N(g) : N(g);
                else if (trial % 5 == 2) c[j] = j == 0 ? U(g) * 100.f : 0.f;
                else c[j] = N(g);
            }
            for (int j = 0; j < 3; ++j) cen.push_back(c[j]);
            const float e = std::exp(-5.f + 4.f * U(g));
            for (int j = 0; j < 3; ++j) box.push_back(c[j] - e);
            for (int j = 0; j < 3; ++j) box.push_back(c[j] + e);
        }
        std::vector<uint64_t> keys(m);
        for (int p = 0; p < m; ++p) keys[p] = ((uint64_t)(g() & 0x3fffffffu) << 32) | (uint64_t)p;
        std::sort(keys.begin(), keys.end());
        Builder B;
        B.keys = &keys;
        B.box = &box;
        B.cen = &cen;
        B.prim_base = 0;
        B.make(0, m);
        CHECK(B.max_depth <= kLidarStack, "trial %d: depth %d", trial, B.max_depth);
        std::vector<int> seen(m, 0);
        const int nn = (int)B.skip.size();
        std::function<void(int)> walk = [&](int id) {
            CHECK(id >= 0 && id < nn, "node %d of %d", id, nn);
            if (B.leaf_count[id]) {
                CHECK(B.leaf_count[id] <= kLeafSize, "leaf of %d", B.leaf_count[id]);
                CHECK(B.skip[id] == id + 1, "leaf skip");
                for (int i = B.leaf_first[id]; i < B.leaf_first[id] + B.leaf_count[id]; ++i) {
                    CHECK(i >= 0 && i < m, "primitive slot %d", i);
                    const uint32_t p = (uint32_t)(keys[i] & 0xffffffffu);
                    CHECK(p < (uint32_t)m, "primitive %u", p);
                    ++seen[p];
                    for (int j = 0; j < 3; ++j) {
                        CHECK(B.nlo[3 * id + j] <= box[6 * p + j] && B.nhi[3 * id + j] >= box[6 * p + 3 + j], "box");
                        CHECK(B.clo[3 * id + j] <= cen[3 * p + j] && B.chi[3 * id + j] >= cen[3 * p + j], "centres");
                    }
                }
                return;
            }
            const int l = id + 1, r = B.right[id];
            CHECK(r > l && r < B.skip[id], "right child %d of node %d (skip %d)", r, id, B.skip[id]);
            CHECK(B.skip[l] == r, "left subtree ends at the right child");
            CHECK(B.skip[r] == B.skip[id], "right subtree ends with its parent's");
            for (int c : {l, r})
                for (int j = 0; j < 3; ++j) {
                    CHECK(B.nlo[3 * id + j] <= B.nlo[3 * c + j] && B.nhi[3 * id + j] >= B.nhi[3 * c + j], "child box");
                    CHECK(B.clo[3 * id + j] <= B.clo[3 * c + j] && B.chi[3 * id + j] >= B.chi[3 * c + j], "child centres");
                }
            walk(l);
            walk(r);
        };
        walk(0);
        CHECK(B.skip[0] == nn, "root skip");
        for (int p = 0; p < m; ++p) CHECK(seen[p] == 1, "trial %d: primitive %d in %d leaves", trial, p, seen[p]);
    }
    printf(fails ? "FAILED\n" : "ok\n");
    return fails != 0;
}
