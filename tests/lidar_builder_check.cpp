// Host check of the LiDAR hierarchy builder (no GPU use).
// Boxes: for seeded anisotropic, rotated Gaussians of opacity 1/255 .. 1, a Gaussian's box
// holds every point of its ellipsoid at the Mahalanobis radius sqrt(2 ln(255 o)) (where
// o exp(-D^2 / 2) falls to 1/255; points sampled on it through M = R diag(s)), and is no more
// than 1% wider than the ellipsoid's extreme points m +- k Sigma e_j / sqrt(Sigma_jj)
// (Sigma = M M^T) plus its stated widening.
// Trees: for seeded primitive sets (uniform, clustered, on a line, all centres equal; 5 to 200k
// primitives; and 120 centres at 2^i on a line, which the surface-area splits peel one at a
// time) every primitive sits in exactly one leaf of at most kLeafSize, the depth-first
// layout holds (left child next, right child after the left subtree, skip = end of the
// subtree), every node box holds its primitives' boxes and centres, the depth stays within
// the tracer's stack, and building the top subtrees on their own threads gives the same tree
// as one thread.
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

static void check_boxes() {
    std::mt19937 g(5);
    std::normal_distribution<double> N(0.0, 1.0);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    for (int it = 0; it < 2000; ++it) {
        double m[3], s[3], q[4];
        for (int j = 0; j < 3; ++j) m[j] = 10.0 * N(g);
        for (int j = 0; j < 3; ++j) s[j] = std::exp(-5.0 + 5.0 * U(g));
        double qn = 0.0;
        for (int j = 0; j < 4; ++j) {
            q[j] = N(g);
            qn += q[j] * q[j];
        }
        qn = std::sqrt(qn);
        const double w = q[0] / qn, x = q[1] / qn, y = q[2] / qn, z = q[3] / qn;
        const double R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                             2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                             2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
        const double o = it == 0 ? 1.0 / 255.0 * 1.0001 : (it == 1 ? 1.0 : 1.0 / 255.0 + (1.0 - 1.0 / 255.0) * U(g));
        float lo[3], hi[3];
        gaussian_box(m, s, R, o, lo, hi);
        const double k = std::sqrt(2.0 * std::log(255.0 * o));
        double M[9], S[9];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) M[a * 3 + b] = R[a * 3 + b] * s[b];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                S[a * 3 + b] = 0.0;
                for (int c = 0; c < 3; ++c) S[a * 3 + b] += M[a * 3 + c] * M[b * 3 + c];
            }
        // points of the ellipsoid: m + M (k u), |u| = 1
        for (int t = 0; t < 64; ++t) {
            double u[3], un = 0.0;
            for (int j = 0; j < 3; ++j) {
                u[j] = N(g);
                un += u[j] * u[j];
            }
            un = std::sqrt(un);
            for (int a = 0; a < 3; ++a) {
                double p = m[a];
                for (int c = 0; c < 3; ++c) p += M[a * 3 + c] * k * u[c] / un;
                CHECK((double)lo[a] <= p && p <= (double)hi[a], "box %d misses an ellipsoid point on axis %d", it, a);
            }
        }
        // the extreme points along each axis lie on the ellipsoid and bound the box's width
        for (int j = 0; j < 3; ++j) {
            const double ext = k * std::sqrt(S[j * 3 + j]);
            double pe[3], v[3];
            for (int a = 0; a < 3; ++a) pe[a] = k * S[a * 3 + j] / std::sqrt(S[j * 3 + j]);
            // Mahalanobis radius of pe: |diag(1/s) R^T pe|
            double r2 = 0.0;
            for (int c = 0; c < 3; ++c) {
                v[c] = 0.0;
                for (int a = 0; a < 3; ++a) v[c] += R[a * 3 + c] * pe[a];
                v[c] /= s[c];
                r2 += v[c] * v[c];
            }
            CHECK(std::fabs(std::sqrt(r2) - k) <= 1e-9 * (k + 1.0), "extreme point off the ellipsoid");
            CHECK(std::fabs(pe[j] - ext) <= 1e-9 * (ext + 1e-30), "extreme point extent");
            const double half = 0.5 * ((double)hi[j] - (double)lo[j]);
            const double allowed = 1.01 * std::sqrt(k * k + 0.01) / k * ext + 1e-5 * (std::fabs(m[j]) + 1.0) + 1e-6 * (std::fabs(m[j]) + 1.0);
            CHECK(half <= allowed, "box %d axis %d half-extent %g above %g", it, j, half, allowed);
        }
    }
}

int main() {
    check_boxes();
    std::mt19937 g(11);
    for (int trial = 0; trial < 41; ++trial) {
        std::uniform_int_distribution<int> nd(5, trial < 10 ? 40 : (trial < 35 ? 5000 : 200000));
        // the last trial: 120 centres at 2^i on a line, where every surface-area split peels off
        // one primitive, so only the depth rule keeps the tree within the stack
        const bool chain = trial == 40;
        const int m = chain ? 120 : nd(g);
        std::normal_distribution<float> N(0.f, 1.f);
        std::uniform_real_distribution<float> U(0.f, 1.f);
        std::vector<float> box, cen;
        for (int i = 0; i < m; ++i) {
            float c[3];
            for (int j = 0; j < 3; ++j) {
                if (chain) c[j] = j == 0 ? std::ldexp(1.0f, i) : 0.f;
                else if (trial % 5 == 0) c[j] = 0.25f;
                else if (trial % 5 == 1) c[j] = (i % 3 == 0) ? 10.f + 0.01f * N(g) : N(g);
                else if (trial % 5 == 2) c[j] = j == 0 ? U(g) * 100.f : 0.f;
                else c[j] = N(g);
            }
            for (int j = 0; j < 3; ++j) cen.push_back(c[j]);
            const float e = chain ? 1.0f : std::exp(-5.f + 4.f * U(g));
            for (int j = 0; j < 3; ++j) box.push_back(c[j] - e);
            for (int j = 0; j < 3; ++j) box.push_back(c[j] + e);
        }
        std::vector<uint64_t> keys(m);
        for (int p = 0; p < m; ++p) keys[p] = ((uint64_t)(g() & 0x3fffffffu) << 32) | (uint64_t)p;
        std::sort(keys.begin(), keys.end());
        std::vector<uint64_t> keys1 = keys;
        Builder B;
        B.keys = &keys;
        B.box = &box;
        B.cen = &cen;
        B.prim_base = 0;
        B.par_min = 64;  // threads for the top subtrees of every trial but the smallest
        B.make(0, m);
        // the same tree when every subtree is built on the calling thread
        Builder B1;
        B1.keys = &keys1;
        B1.box = &box;
        B1.cen = &cen;
        B1.prim_base = 0;
        B1.par_depth = 0;
        B1.make(0, m);
        CHECK(keys1 == keys && B1.skip == B.skip && B1.right == B.right && B1.leaf_first == B.leaf_first &&
                  B1.leaf_count == B.leaf_count && B1.nlo == B.nlo && B1.nhi == B.nhi && B1.clo == B.clo &&
                  B1.chi == B.chi && B1.max_depth == B.max_depth,
              "trial %d: the threaded build differs from the serial one", trial);
        CHECK(B.max_depth <= kLidarStack, "trial %d: depth %d", trial, B.max_depth);
        if (chain) printf("chain of %d: depth %d\n", m, B.max_depth);
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
