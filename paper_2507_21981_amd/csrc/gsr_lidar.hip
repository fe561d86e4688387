// LiDAR sensor by Gaussian ray tracing (paper Sec. III-C: LiDAR from a BVH-accelerated native
// Gaussian ray tracer, next to the splatted RGB and depth).
//
// Acceleration structure: one bounding-volume hierarchy per scene node, over the node-local
// bounding boxes of its Gaussians' ellipsoids at the Mahalanobis radius where alpha can still
// reach 1/255 (sqrt(2 ln(255 o)), 3.33 sigma at opacity 1).  Node-local, so the per-step rigid
// poses of object nodes never touch it: a ray is moved into each node's frame instead
// (two-level tracing).  Built once per composed topology on the host (binary splits by a
// binned surface-area heuristic over the centres, median splits below a fixed depth), stored
// depth-first (the left child follows its parent, the parent keeps the right child's index).
//
// Tracing (k_lidar, a wavefront per packet of up to 64 rays): repeated passes over the env's
// nodes, each collecting per lane in registers the K next hits in (t_c, id) order after the
// last one composited -- a hit being a Gaussian whose centre lies at t_c = (mu - o) . d inside
// (tmin, tmax) and whose peak response along the ray, alpha = min(0.99, o exp(-D^2 / 2)),
// reaches 1/255 -- then compositing them front to back with the camera's rules until the
// transmittance stop or the last hit.  The wavefront walks each hierarchy once for all its rays
// (a LiDAR's neighbouring beams cross mostly the same boxes); a subtree is skipped when no ray
// may enter it: the ray's line misses its box, every centre in it lies before the ray's last
// composited hit or outside (tmin, tmax), or, once K hits are held, beyond the K-th.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <system_error>
#include <thread>
#include <vector>

#include "gsr_internal.h"

namespace gsr {

constexpr int kLidarK = 16;      // hits per pass
constexpr int kLeafSize = 24;    // primitives per BVH leaf at most
constexpr int kLeafShift = 27;   // a node's reference: leaf count << kLeafShift | first primitive, or
                                 //   the right child's index (count 0)
static_assert(kLeafSize < (1 << (32 - kLeafShift)), "a leaf's count fits its field");
constexpr int kLidarStack = 48;  // traversal stack entries per ray (hierarchy depth at most)

struct LidarScene {
    float4* bnodes = nullptr;   // 4 per BVH node: (lo, skip), (hi, leaf: count << kLeafShift | first prim, or right
                                //   child), the box of the centres (clo, -), (chi, -)
    float4* prims = nullptr;    // 4 per primitive: (mu, opacity), (A row 0, A10), (A11, A12, A20, A21), (A22, id)
    int2* roots = nullptr;      // per scene node: (first BVH node, BVH node count)
    size_t n_bnodes = 0, n_prims = 0;
    int n_nodes = 0;
};

void lidar_free(LidarScene* L) {
    if (!L) return;
    if (L->bnodes) hipFree(L->bnodes);
    if (L->prims) hipFree(L->prims);
    if (L->roots) hipFree(L->roots);
    delete L;
}

namespace {

uint32_t spread10(uint32_t x) {
    x &= 0x3ffu;
    x = (x | (x << 16)) & 0x030000ffu;
    x = (x | (x << 8)) & 0x0300f00fu;
    x = (x | (x << 4)) & 0x030c30c3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

// Box of a Gaussian (centre m, scales s, rotation R row-major, opacity o >= 1/255) holding the
// ellipsoid inside which o exp(-D^2 / 2) reaches 1/255: Mahalanobis radius
// k = sqrt(2 ln(255 o)) (3.33 at o = 1), half extent k sqrt(Sigma_jj) with
// Sigma = R diag(s^2) R^T; k^2 is raised by 0.01 and the extent widened so that the FP32 alpha
// test and slab test stay conservative.
void gaussian_box(const double m[3], const double s[3], const double R[9], double o, float lo[3], float hi[3]) {
    const double kr = std::sqrt(2.0 * std::log(255.0 * o) + 0.01);
    for (int j = 0; j < 3; ++j) {
        double sjj = 0.0;
        for (int c = 0; c < 3; ++c) sjj += R[j * 3 + c] * R[j * 3 + c] * s[c] * s[c];
        const double e = kr * std::sqrt(sjj) * (1.0 + 1e-4) + 1e-5 * (std::fabs(m[j]) + 1.0);
        lo[j] = (float)(m[j] - e);
        hi[j] = (float)(m[j] + e);
    }
}

struct Builder {
    std::vector<uint64_t>* keys;        // (Morton code << 32 | index); ranges reordered by the splits
    const std::vector<float>* box;      // per primitive: lo[3], hi[3]
    const std::vector<float>* cen;      // per primitive: centre[3]
    std::vector<float> nlo, nhi, clo, chi;  // per node: box of the ellipsoids, box of the centres
    std::vector<int> skip, leaf_first, leaf_count, right;
    size_t prim_base = 0;
    int max_depth = 0;
    int par_depth = 3;         // the right subtrees of nodes up to this depth are built on
    size_t par_min = 65536;    // their own threads when they hold at least par_min primitives

    static constexpr int kBins = 128;

    uint32_t prim(size_t i) const { return (uint32_t)((*keys)[i] & 0xffffffffu); }
    static double area(const float* lo, const float* hi) {
        const double dx = (double)hi[0] - lo[0], dy = (double)hi[1] - lo[1], dz = (double)hi[2] - lo[2];
        return dx * dy + dy * dz + dz * dx;
    }

    // Where to split [lo, hi): binned surface-area heuristic over the centres along their
    // longest extent (cost = box area x primitives, summed over the two sides), or the median
    // along that extent when the bins cannot separate the range or when the depth left needs
    // halving: with lv the halvings that bring the range to kLeafSize, the heuristic is used
    // only while depth + lv <= kLidarStack - 2, so every node keeps depth + lv <= kLidarStack - 1
    // (a child of either split has no larger lv; a median child has one less) and leaves stay
    // within the tracer's stack.
    size_t split(size_t lo, size_t hi, int depth) {
        float cmin[3] = {INFINITY, INFINITY, INFINITY}, cmax[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (size_t i = lo; i < hi; ++i) {
            const float* c = &(*cen)[3 * prim(i)];
            for (int j = 0; j < 3; ++j) {
                cmin[j] = std::min(cmin[j], c[j]);
                cmax[j] = std::max(cmax[j], c[j]);
            }
        }
        int ax = 0;
        for (int j = 1; j < 3; ++j)
            if (cmax[j] - cmin[j] > cmax[ax] - cmin[ax]) ax = j;
        const double ext = (double)cmax[ax] - (double)cmin[ax];
        const size_t half = (lo + hi) / 2;
        auto median = [&]() {
            std::nth_element(keys->begin() + lo, keys->begin() + half, keys->begin() + hi,
                             [&](uint64_t a, uint64_t b) {
                                 return (*cen)[3 * (a & 0xffffffffu) + ax] < (*cen)[3 * (b & 0xffffffffu) + ax];
                             });
            return half;
        };
        int lv = 0;
        while (((size_t)kLeafSize << lv) < hi - lo) ++lv;
        if (!(ext > 0.0) || depth + lv > kLidarStack - 2) return median();
        auto bin = [&](uint32_t p) {
            const int b = (int)(((double)(*cen)[3 * p + ax] - (double)cmin[ax]) / ext * kBins);
            return std::min(kBins - 1, std::max(0, b));
        };
        size_t cnt[kBins] = {};
        float blo[kBins][3], bhi[kBins][3];
        for (int b = 0; b < kBins; ++b)
            for (int j = 0; j < 3; ++j) {
                blo[b][j] = INFINITY;
                bhi[b][j] = -INFINITY;
            }
        for (size_t i = lo; i < hi; ++i) {
            const uint32_t p = prim(i);
            const int b = bin(p);
            ++cnt[b];
            for (int j = 0; j < 3; ++j) {
                blo[b][j] = std::min(blo[b][j], (*box)[6 * p + j]);
                bhi[b][j] = std::max(bhi[b][j], (*box)[6 * p + 3 + j]);
            }
        }
        // areas and counts of the bins at and right of k
        double ra[kBins];
        size_t rn[kBins];
        float lo3[3] = {INFINITY, INFINITY, INFINITY}, hi3[3] = {-INFINITY, -INFINITY, -INFINITY};
        size_t n = 0;
        for (int b = kBins - 1; b >= 0; --b) {
            n += cnt[b];
            for (int j = 0; j < 3; ++j) {
                lo3[j] = std::min(lo3[j], blo[b][j]);
                hi3[j] = std::max(hi3[j], bhi[b][j]);
            }
            ra[b] = n ? area(lo3, hi3) : 0.0;
            rn[b] = n;
        }
        for (int j = 0; j < 3; ++j) {
            lo3[j] = INFINITY;
            hi3[j] = -INFINITY;
        }
        n = 0;
        int best = -1;
        double best_cost = INFINITY;
        for (int b = 1; b < kBins; ++b) {  // left = bins below b
            n += cnt[b - 1];
            for (int j = 0; j < 3; ++j) {
                lo3[j] = std::min(lo3[j], blo[b - 1][j]);
                hi3[j] = std::max(hi3[j], bhi[b - 1][j]);
            }
            if (n == 0 || rn[b] == 0) continue;
            const double c = area(lo3, hi3) * (double)n + ra[b] * (double)rn[b];
            if (c < best_cost) {
                best_cost = c;
                best = b;
            }
        }
        if (best < 0) return median();
        const auto it = std::partition(keys->begin() + lo, keys->begin() + hi,
                                       [&](uint64_t k) { return bin((uint32_t)(k & 0xffffffffu)) < best; });
        const size_t mid = (size_t)(it - keys->begin());
        return (mid > lo && mid < hi) ? mid : median();
    }

    int make(size_t lo, size_t hi, int depth = 1) {
        const int id = (int)skip.size();
        max_depth = std::max(max_depth, depth);
        skip.push_back(0);
        leaf_first.push_back(0);
        leaf_count.push_back(0);
        right.push_back(0);
        for (int j = 0; j < 3; ++j) {
            nlo.push_back(INFINITY);
            nhi.push_back(-INFINITY);
            clo.push_back(INFINITY);
            chi.push_back(-INFINITY);
        }
        if (hi - lo <= (size_t)kLeafSize) {
            leaf_first[id] = (int)(prim_base + lo);
            leaf_count[id] = (int)(hi - lo);
            for (size_t i = lo; i < hi; ++i) {
                const uint32_t p = prim(i);
                for (int j = 0; j < 3; ++j) {
                    nlo[3 * id + j] = std::min(nlo[3 * id + j], (*box)[6 * p + j]);
                    nhi[3 * id + j] = std::max(nhi[3 * id + j], (*box)[6 * p + 3 + j]);
                    clo[3 * id + j] = std::min(clo[3 * id + j], (*cen)[3 * p + j]);
                    chi[3 * id + j] = std::max(chi[3 * id + j], (*cen)[3 * p + j]);
                }
            }
        } else {
            const size_t mid = split(lo, hi, depth);
            int l = -1, r = -1;
            if (depth <= par_depth && hi - mid >= par_min) {
                // the two halves partition disjoint ranges of the keys; the right one is built
                // by its own builder and appended where the serial walk would place it
                Builder rb;
                rb.keys = keys;
                rb.box = box;
                rb.cen = cen;
                rb.prim_base = prim_base;
                rb.par_depth = par_depth;
                rb.par_min = par_min;
                try {
                    std::thread t([&rb, mid, hi, depth] { rb.make(mid, hi, depth + 1); });
                    l = make(lo, mid, depth + 1);
                    t.join();
                    r = append(rb);
                } catch (const std::system_error&) {
                    if (l < 0) l = make(lo, mid, depth + 1);  // no thread: the serial walk
                    r = make(mid, hi, depth + 1);
                }
            } else {
                l = make(lo, mid, depth + 1);
                r = make(mid, hi, depth + 1);
            }
            right[id] = r;
            for (int j = 0; j < 3; ++j) {
                nlo[3 * id + j] = std::min(nlo[3 * l + j], nlo[3 * r + j]);
                nhi[3 * id + j] = std::max(nhi[3 * l + j], nhi[3 * r + j]);
                clo[3 * id + j] = std::min(clo[3 * l + j], clo[3 * r + j]);
                chi[3 * id + j] = std::max(chi[3 * l + j], chi[3 * r + j]);
            }
        }
        skip[id] = (int)skip.size();
        return id;
    }

    // Appends the nodes of a subtree built by another builder (root at its index 0), shifting
    // its node references by the index its root lands at; returns that index.
    int append(const Builder& b) {
        const int off = (int)skip.size();
        for (size_t i = 0; i < b.skip.size(); ++i) {
            skip.push_back(b.skip[i] + off);
            leaf_first.push_back(b.leaf_first[i]);
            leaf_count.push_back(b.leaf_count[i]);
            right.push_back(b.leaf_count[i] ? b.right[i] : b.right[i] + off);
        }
        nlo.insert(nlo.end(), b.nlo.begin(), b.nlo.end());
        nhi.insert(nhi.end(), b.nhi.begin(), b.nhi.end());
        clo.insert(clo.end(), b.clo.begin(), b.clo.end());
        chi.insert(chi.end(), b.chi.begin(), b.chi.end());
        max_depth = std::max(max_depth, b.max_depth);
        return off;
    }
};

inline float as_float(int v) {
    float f;
    memcpy(&f, &v, 4);
    return f;
}

}  // namespace

// Build the hierarchies of every node (host arrays of the scene's nodes; the Gaussian data is
// read back from the device).  Returns 0 or a message.
std::string lidar_build(const std::vector<Node>& nodes, LidarScene** out) {
    *out = nullptr;
    std::vector<float4> all_nodes, all_prims;
    std::vector<int2> roots(nodes.size());
    for (size_t k = 0; k < nodes.size(); ++k) {
        const Node& nd = nodes[k];
        const size_t n = nd.n;
        std::vector<float> mu(3 * n), sc(3 * n), qt(4 * n), op(n);
        if (n) {
            if (hipMemcpy(mu.data(), nd.means, 12 * n, hipMemcpyDeviceToHost) != hipSuccess ||
                hipMemcpy(sc.data(), nd.scales, 12 * n, hipMemcpyDeviceToHost) != hipSuccess ||
                hipMemcpy(qt.data(), nd.quats, 16 * n, hipMemcpyDeviceToHost) != hipSuccess ||
                hipMemcpy(op.data(), nd.opac, 4 * n, hipMemcpyDeviceToHost) != hipSuccess)
                return "reading node parameters back failed";
        }
        // primitives that can be hit: finite, opacity >= 1/255, positive scales
        std::vector<uint32_t> idx;
        std::vector<float> box, cen;
        std::vector<float4> prim;
        double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (size_t i = 0; i < n; ++i) {
            const double m[3] = {mu[3 * i], mu[3 * i + 1], mu[3 * i + 2]};
            const double s[3] = {sc[3 * i], sc[3 * i + 1], sc[3 * i + 2]};
            double q[4] = {qt[4 * i], qt[4 * i + 1], qt[4 * i + 2], qt[4 * i + 3]};
            bool fin = std::isfinite(op[i]);
            for (int j = 0; j < 3; ++j) fin = fin && std::isfinite(m[j]) && std::isfinite(s[j]) && s[j] > 0.0;
            for (int j = 0; j < 4; ++j) fin = fin && std::isfinite(q[j]);
            const double qn = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
            if (!fin || !(qn > 0.0) || !(op[i] >= (float)(1.0 / 255.0))) continue;
            for (int j = 0; j < 4; ++j) q[j] /= qn;
            const double w = q[0], x = q[1], y = q[2], z = q[3];
            const double R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                                 2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                                 2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
            float lo[3], hi[3];
            gaussian_box(m, s, R, op[i], lo, hi);
            for (int j = 0; j < 3; ++j) {
                clo[j] = std::min(clo[j], m[j]);
                chi[j] = std::max(chi[j], m[j]);
            }
            for (int j = 0; j < 3; ++j) box.push_back(lo[j]);
            for (int j = 0; j < 3; ++j) box.push_back(hi[j]);
            for (int j = 0; j < 3; ++j) cen.push_back((float)m[j]);
            // A = S^-1 R^T: row c is column c of R divided by s_c
            float A[9];
            for (int c = 0; c < 3; ++c)
                for (int j = 0; j < 3; ++j) A[c * 3 + j] = (float)(R[j * 3 + c] / s[c]);
            const uint32_t gid = nd.gid_base + (uint32_t)i;
            prim.push_back(make_float4((float)m[0], (float)m[1], (float)m[2], op[i]));
            prim.push_back(make_float4(A[0], A[1], A[2], A[3]));
            prim.push_back(make_float4(A[4], A[5], A[6], A[7]));
            prim.push_back(make_float4(A[8], as_float((int)gid), 0.0f, 0.0f));
            idx.push_back((uint32_t)i);
        }
        const size_t m = idx.size();
        roots[k] = make_int2((int)(all_nodes.size() / 4), 0);
        if (m == 0) continue;
        std::vector<uint64_t> keys(m);
        for (size_t p = 0; p < m; ++p) {
            uint32_t code = 0;
            for (int j = 0; j < 3; ++j) {
                const double c = 0.5 * ((double)box[6 * p + j] + (double)box[6 * p + 3 + j]);
                const double ext = chi[j] - clo[j];
                const double u = ext > 0.0 ? (c - clo[j]) / ext : 0.0;
                const uint32_t qv = (uint32_t)std::min(1023.0, std::max(0.0, std::floor(u * 1024.0)));
                code |= spread10(qv) << j;
            }
            keys[p] = ((uint64_t)code << 32) | (uint64_t)p;
        }
        std::sort(keys.begin(), keys.end());
        Builder B;
        B.keys = &keys;
        B.box = &box;
        B.cen = &cen;
        B.prim_base = all_prims.size() / 4;
        B.make(0, m);
        if (B.max_depth > kLidarStack) return "a hierarchy deeper than the tracer's stack allows";
        const int node_base = (int)(all_nodes.size() / 4);
        const size_t nb = B.skip.size();
        for (size_t i = 0; i < nb; ++i) {
            // leaf: count << kLeafShift | first primitive; internal: the right child (the left is next)
            const int leaf = B.leaf_count[i]
                                 ? (int)(((uint32_t)B.leaf_count[i] << kLeafShift) | (uint32_t)B.leaf_first[i])
                                 : node_base + B.right[i];
            all_nodes.push_back(make_float4(B.nlo[3 * i], B.nlo[3 * i + 1], B.nlo[3 * i + 2], as_float(node_base + B.skip[i])));
            all_nodes.push_back(make_float4(B.nhi[3 * i], B.nhi[3 * i + 1], B.nhi[3 * i + 2], as_float(leaf)));
            all_nodes.push_back(make_float4(B.clo[3 * i], B.clo[3 * i + 1], B.clo[3 * i + 2], 0.0f));
            all_nodes.push_back(make_float4(B.chi[3 * i], B.chi[3 * i + 1], B.chi[3 * i + 2], 0.0f));
        }
        for (size_t p = 0; p < m; ++p) {
            const uint32_t src = (uint32_t)(keys[p] & 0xffffffffu);
            for (int j = 0; j < 4; ++j) all_prims.push_back(prim[4 * src + j]);
        }
        roots[k] = make_int2(node_base, (int)nb);
        if (all_prims.size() / 4 >= (1u << kLeafShift)) return "more than 2^27 primitives";
        if (all_nodes.size() / 4 >= (1u << kLeafShift)) return "more than 2^27 hierarchy nodes";
    }
    LidarScene* L = new LidarScene();
    L->n_bnodes = all_nodes.size() / 4;
    L->n_prims = all_prims.size() / 4;
    L->n_nodes = (int)nodes.size();
    if (hipMalloc(&L->bnodes, std::max<size_t>(all_nodes.size(), 1) * sizeof(float4)) != hipSuccess ||
        hipMalloc(&L->prims, std::max<size_t>(all_prims.size(), 1) * sizeof(float4)) != hipSuccess ||
        hipMalloc(&L->roots, std::max<size_t>(roots.size(), 1) * sizeof(int2)) != hipSuccess) {
        lidar_free(L);
        return "device allocation failed";
    }
    if ((!all_nodes.empty() &&
         hipMemcpy(L->bnodes, all_nodes.data(), all_nodes.size() * sizeof(float4), hipMemcpyHostToDevice) != hipSuccess) ||
        (!all_prims.empty() &&
         hipMemcpy(L->prims, all_prims.data(), all_prims.size() * sizeof(float4), hipMemcpyHostToDevice) != hipSuccess) ||
        hipMemcpy(L->roots, roots.data(), roots.size() * sizeof(int2), hipMemcpyHostToDevice) != hipSuccess) {
        lidar_free(L);
        return "upload failed";
    }
    *out = L;
    return std::string();
}

size_t lidar_bytes(const LidarScene* L) { return L ? (L->n_bnodes * 64 + L->n_prims * 64) : 0; }

// ------------------------------------------------------------------------------------------
// tracing
// ------------------------------------------------------------------------------------------
__device__ inline uint64_t hit_key(float t, uint32_t id) { return ((uint64_t)__float_as_uint(t) << 32) | id; }

// Where a ray may enter a box: the line meets it, some centre in it lies at a distance along
// the ray after the last composited hit and inside the window, and -- once K hits are held --
// before the K-th.  Returns the smallest centre distance over the box (the visiting order) or
// +inf when the box is skipped.
// Where a ray may enter a node: the line meets its box, some centre in it lies at a distance
// along the ray after the last composited hit and inside the window, and -- once K hits are
// held -- before the K-th.  The distances come from the box of the node's centres.  Returns the
// smallest centre distance over that box (the visiting order) or +inf when the node is skipped.
__device__ inline float lidar_enter(const float4* __restrict__ nd, float o0, float o1, float o2, float d0, float d1,
                                    float d2, float i0, float i1, float i2, float t_last, float tmin, float tmax,
                                    float t_kth) {
    const float4 a = nd[0], b = nd[1];
    const float ta0 = (a.x - o0) * i0, tb0 = (b.x - o0) * i0;
    const float ta1 = (a.y - o1) * i1, tb1 = (b.y - o1) * i1;
    const float ta2 = (a.z - o2) * i2, tb2 = (b.z - o2) * i2;
    const float tin = fmaxf(fmaxf(fminf(ta0, tb0), fminf(ta1, tb1)), fminf(ta2, tb2));
    const float tout = fminf(fminf(fmaxf(ta0, tb0), fmaxf(ta1, tb1)), fmaxf(ta2, tb2));
    if (!(tin <= tout + 1e-6f * (fabsf(tin) + fabsf(tout)))) return INFINITY;
    const float4 c = nd[2], e = nd[3];
    const float pa0 = d0 * (c.x - o0), pb0 = d0 * (e.x - o0);
    const float pa1 = d1 * (c.y - o1), pb1 = d1 * (e.y - o1);
    const float pa2 = d2 * (c.z - o2), pb2 = d2 * (e.z - o2);
    const float tl = fminf(pa0, pb0) + fminf(pa1, pb1) + fminf(pa2, pb2);
    const float th = fmaxf(pa0, pb0) + fmaxf(pa1, pb1) + fmaxf(pa2, pb2);
    // slack for the rounding of these sums (centres are exact FP32 values)
    const float slack = 1e-5f * (fabsf(tl) + fabsf(th)) + 1e-5f * (fabsf(o0) + fabsf(o1) + fabsf(o2)) + 1e-6f;
    const bool in = th + slack >= t_last && tl - slack <= tmax && th + slack >= tmin && tl - slack <= t_kth;
    return in ? tl : INFINITY;
}

// A ray moved into one node's frame.
struct LocalRay {
    float o0, o1, o2, d0, d1, d2, i0, i1, i2;
};

__device__ inline LocalRay local_ray(const gsr_ray& ray, const gsr_pose& P) {
    LocalRay l;
    const float ox = ray.origin[0] - P.t[0], oy = ray.origin[1] - P.t[1], oz = ray.origin[2] - P.t[2];
    l.o0 = fmaf(P.R[0], ox, fmaf(P.R[3], oy, P.R[6] * oz));
    l.o1 = fmaf(P.R[1], ox, fmaf(P.R[4], oy, P.R[7] * oz));
    l.o2 = fmaf(P.R[2], ox, fmaf(P.R[5], oy, P.R[8] * oz));
    l.d0 = fmaf(P.R[0], ray.dir[0], fmaf(P.R[3], ray.dir[1], P.R[6] * ray.dir[2]));
    l.d1 = fmaf(P.R[1], ray.dir[0], fmaf(P.R[4], ray.dir[1], P.R[7] * ray.dir[2]));
    l.d2 = fmaf(P.R[2], ray.dir[0], fmaf(P.R[5], ray.dir[1], P.R[8] * ray.dir[2]));
    l.i0 = 1.0f / (l.d0 != 0.0f ? l.d0 : 1e-30f);
    l.i1 = 1.0f / (l.d1 != 0.0f ? l.d1 : 1e-30f);
    l.i2 = 1.0f / (l.d2 != 0.0f ? l.d2 : 1e-30f);
    return l;
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// One wavefront traces up to 64 rays together (a packet: a LiDAR's neighbouring beams share
// most of the boxes they cross).  The walk over a hierarchy is the wavefront's: a node is
// visited when any of its rays may enter it, children nearer (by majority) first, one stack
// per wavefront in LDS, node loads the same for every lane.  Each ray keeps its own K next
// hits, last composited key and pruning bounds (alike on each of its 64 / rpw lanes, which
// test a leaf's primitives side by side); a ray that visits a node it would have skipped only
// tests primitives that cannot change its K nearest, so the result is the ray's alone.  Passes
// repeat until every ray has stopped or seen all its hits.  Held to three wavefronts per SIMD
// (168 VGPRs, a few bytes spilled): at two the tracer is slower.
__global__ __launch_bounds__(64, 3) void k_lidar(const float4* __restrict__ bnodes, const float4* __restrict__ prims,
                                              const int2* __restrict__ roots, const Env* __restrict__ envs,
                                              const gsr_pose* __restrict__ poses, int n_envs, int rays_per_env,
                                              const gsr_ray* __restrict__ rays, float* range_out, float* alpha_out,
                                              uint32_t* hits_out, int rpw) {
    __shared__ int s_stack[kLidarStack];
    const int lane = threadIdx.x;
    const long long n = (long long)n_envs * rays_per_env;
    // rays r0 .. r0 + nv - 1 (rpw rays per wavefront, a power of two): lane h rpw + i holds ray
    // r0 + i, so each ray has 64 / rpw lanes with the same state (the same walk, hits and
    // compositing) that share the tests of a leaf's primitives; lanes of rays past the end take
    // the first ray's values and stay done
    const long long r0 = (long long)blockIdx.x * rpw;
    const int nv = (int)(n - r0 < rpw ? n - r0 : rpw);
    const int lg = __builtin_ctz((unsigned)rpw);
    const int ri = lane & (rpw - 1), h = lane >> lg, lpr = 64 >> lg;
    const long long r = r0 + ri;
    const bool valid = ri < nv;
    const long long rr = valid ? r : r0;
    const int env = (int)(rr / rays_per_env);
    const gsr_ray ray = rays[rr];
    const float thr = (float)(1.0 / 255.0);
    float T = 1.0f, R = 0.0f;
    uint32_t nh = 0;
    const float tmin = fmaxf(ray.tmin, 0.0f), tmax = ray.tmax;  // keys order as their bits for t >= 0
    uint64_t last = hit_key(tmin, 0u);  // keys at or below it are done (tmin itself is excluded)
    bool done = !valid;
    // rays are env-major, so the wavefront's envs are a contiguous range
    const int e_lo = uniform(env), e_hi = __builtin_amdgcn_readlane(env, nv - 1);
    while (__any(!done)) {
        uint64_t key[kLidarK];
        float al[kLidarK];
#pragma unroll
        for (int j = 0; j < kLidarK; ++j) {
            key[j] = ~0ull;
            al[j] = 0.0f;
        }
        int found = 0;
        const float t_last = __uint_as_float((uint32_t)(last >> 32));
        auto kth = [&]() { return found == kLidarK ? __uint_as_float((uint32_t)(key[kLidarK - 1] >> 32)) : INFINITY; };
        for (int e = e_lo; e <= e_hi; ++e) {
            const bool part = !done && env == e;
            if (!__any(part)) continue;
            const Env ev = envs[e];
            for (int k = ev.node_begin; k < ev.node_end; ++k) {
                const int2 rt = roots[k];
                if (rt.y == 0) continue;
                const LocalRay l = local_ray(ray, poses[k]);
                auto enters = [&](int node) {
                    return part && lidar_enter(bnodes + 4 * node, l.o0, l.o1, l.o2, l.d0, l.d1, l.d2, l.i0, l.i1, l.i2,
                                               t_last, tmin, tmax, kth()) != INFINITY;
                };
                if (!__any(enters(rt.x))) continue;
                int cur = rt.x, sp = 0;
                while (true) {
                    const int info = uniform(__float_as_int(bnodes[4 * cur + 1].w));
                    bool pop = false;
                    if ((uint32_t)info >> kLeafShift) {
                        const int cnt = (int)((uint32_t)info >> kLeafShift), p0 = info & ((1 << kLeafShift) - 1);
                        // the leaf's primitives in batches of 64 / rpw: lane h of a ray tests
                        // primitive pb + h against the ray's hits as they stood at the batch's
                        // start, then every lane of the ray inserts the batch's hits in primitive
                        // order (each checked against the K-th key again), so the ray keeps the
                        // same K nearest hits as with one primitive at a time
                        for (int pb = 0; pb < cnt; pb += lpr) {
                            bool hit = false;
                            uint64_t hk = 0ull;
                            float ha = 0.0f;
                            if (part && pb + h < cnt) do {
                                const int p = p0 + pb + h;
                                const float4 m = prims[4 * p], A0 = prims[4 * p + 1], A1 = prims[4 * p + 2],
                                             A2 = prims[4 * p + 3];
                                const float q0 = m.x - l.o0, q1 = m.y - l.o1, q2 = m.z - l.o2;
                                const float tc = fmaf(q0, l.d0, fmaf(q1, l.d1, q2 * l.d2));
                                if (!(tc > tmin && tc < tmax)) break;
                                const uint32_t gid = (uint32_t)__float_as_int(A2.y);
                                const uint64_t kk = hit_key(tc, gid);
                                if (kk <= last || kk >= key[kLidarK - 1]) break;
                                // closest-approach offset and the Mahalanobis minimum along the ray
                                const float e0 = fmaf(tc, l.d0, -q0), e1 = fmaf(tc, l.d1, -q1),
                                            e2 = fmaf(tc, l.d2, -q2);
                                const float x0 = fmaf(A0.x, e0, fmaf(A0.y, e1, A0.z * e2));
                                const float x1 = fmaf(A0.w, e0, fmaf(A1.x, e1, A1.y * e2));
                                const float x2 = fmaf(A1.z, e0, fmaf(A1.w, e1, A2.x * e2));
                                const float y0 = fmaf(A0.x, l.d0, fmaf(A0.y, l.d1, A0.z * l.d2));
                                const float y1 = fmaf(A0.w, l.d0, fmaf(A1.x, l.d1, A1.y * l.d2));
                                const float y2 = fmaf(A1.z, l.d0, fmaf(A1.w, l.d1, A2.x * l.d2));
                                const float dd = fmaf(x0, x0, fmaf(x1, x1, x2 * x2));
                                const float xy = fmaf(x0, y0, fmaf(x1, y1, x2 * y2));
                                const float yy = fmaf(y0, y0, fmaf(y1, y1, y2 * y2));
                                const float D2 = fmaxf(dd - xy * (xy / yy), 0.0f);
                                // alpha = o exp(-D^2 / 2) = o 2^(-D^2 log2(e) / 2)
                                const float araw = m.w * __builtin_amdgcn_exp2f(-0.7213475204444817f * D2);
                                if (!(araw >= thr)) break;
                                hit = true;
                                hk = kk;
                                ha = fminf(0.99f, araw);
                            } while (false);
                            const int nb = cnt - pb < lpr ? cnt - pb : lpr;
                            for (int j = 0; j < nb; ++j) {
                                const int src = ri + (j << lg);  // the lane of this ray testing pb + j
                                const int hj = __shfl((int)hit, src, 64);
                                if (!__any(hj)) continue;
                                const uint32_t klo = __shfl((unsigned)(uint32_t)hk, src, 64);
                                const uint32_t khi = __shfl((unsigned)(uint32_t)(hk >> 32), src, 64);
                                const float aj = __shfl(ha, src, 64);
                                uint64_t ck = ((uint64_t)khi << 32) | klo;
                                if (!hj || ck >= key[kLidarK - 1]) continue;
                                // insert in key order (the last entry drops out)
                                float ca = aj;
#pragma unroll
                                for (int q = 0; q < kLidarK; ++q) {
                                    if (ck < key[q]) {
                                        const uint64_t tk = key[q];
                                        const float ta = al[q];
                                        key[q] = ck;
                                        al[q] = ca;
                                        ck = tk;
                                        ca = ta;
                                    }
                                }
                                found = found < kLidarK ? found + 1 : kLidarK;
                            }
                        }
                        pop = true;
                    } else {
                        // inner node: the children any ray may enter, nearer first by majority
                        const int cl = cur + 1, cr = info;
                        const float tk = kth();
                        float tL = INFINITY, tR = INFINITY;
                        if (part) {
                            tL = lidar_enter(bnodes + 4 * cl, l.o0, l.o1, l.o2, l.d0, l.d1, l.d2, l.i0, l.i1, l.i2,
                                             t_last, tmin, tmax, tk);
                            tR = lidar_enter(bnodes + 4 * cr, l.o0, l.o1, l.o2, l.d0, l.d1, l.d2, l.i0, l.i1, l.i2,
                                             t_last, tmin, tmax, tk);
                        }
                        const bool aL = __any(tL != INFINITY), aR = __any(tR != INFINITY);
                        if (aL && aR) {
                            const bool both = tL != INFINITY && tR != INFINITY;
                            const int left_first = __popcll(__ballot(both && tL <= tR)),
                                      right_first = __popcll(__ballot(both && tL > tR));
                            const bool lf = left_first >= right_first;
                            s_stack[sp++] = lf ? cr : cl;
                            cur = lf ? cl : cr;
                        } else if (aL || aR) {
                            cur = aL ? cl : cr;
                        } else {
                            pop = true;
                        }
                    }
                    if (pop) {
                        // the next stacked subtree some ray may still enter
                        bool got = false;
                        while (sp > 0) {
                            const int nd = uniform(s_stack[--sp]);
                            if (__any(enters(nd))) {
                                cur = nd;
                                got = true;
                                break;
                            }
                        }
                        if (!got) break;
                    }
                    cur = uniform(cur);
                }
            }
        }
        // composite this pass's hits front to back
        if (!done) {
#pragma unroll
            for (int j = 0; j < kLidarK; ++j) {
                if (j >= found || done) continue;
                const float a = al[j];
                const float Tn = T * (1.0f - a);
                if (Tn < 1e-4f) {
                    done = true;
                    continue;
                }
                R = fmaf(a * T, __uint_as_float((uint32_t)(key[j] >> 32)), R);
                T = Tn;
                ++nh;
            }
            if (found < kLidarK) done = true;
            last = key[kLidarK - 1];
        }
    }
    if (!valid) return;
    range_out[r] = R;
    alpha_out[r] = 1.0f - T;
    if (hits_out) hits_out[r] = nh;
}

// Rays per wavefront (a power of two, 2 to 64): about kLidarWaves wavefronts per frame.  A
// packet walks the union of its rays' paths and stays until its slowest ray is done, so small
// packets waste fewer visits and many short wavefronts balance the device (composed workload:
// 131k rays 32.7 ms at 64 per wavefront, 20.3 ms at 8; 32k rays 38.2 ms at 64, 14.8 ms at 2).
constexpr long long kLidarWaves = 16384;
static int lidar_rays_per_wave(long long n) {
    int rpw = 64;
    while (rpw > 2 && rpw * kLidarWaves > n) rpw >>= 1;
    return rpw;
}

hipError_t launch_lidar(const LidarScene* L, const Env* envs, const gsr_pose* poses, int n_envs, int rays_per_env,
                        const gsr_ray* rays, float* range, float* alpha, uint32_t* hits, hipStream_t s) {
    const long long n = (long long)n_envs * rays_per_env;
    if (n <= 0) return hipSuccess;
    const int rpw = lidar_rays_per_wave(n);
    hipLaunchKernelGGL(k_lidar, dim3((unsigned)((n + rpw - 1) / rpw)), dim3(64), 0, s, L->bnodes, L->prims, L->roots,
                       envs, poses, n_envs, rays_per_env, rays, range, alpha, hits, rpw);
    return hipGetLastError();
}

}  // namespace gsr
