// Mesh-to-Gaussian transfer (paper Sec. IV-B, "Mesh-Gaussian Transfer"): the step before
// scene composition for interactive nodes that come as textured meshes.  One Gaussian per
// facet: centre at the barycentre; the ellipsoid flattened to a planar primitive whose local
// frame is (unit edge a->b, n x t1, unit normal n); both tangent scales the mean distance from
// the barycentre to the vertices, the normal scale `flatten` times that; colour the mean vertex
// colour as the degree-0 SH coefficient, higher orders zero; degenerate facets (zero area)
// transparent with the identity rotation.  One thread per facet; the facet's three vertices
// (and colours) are gathered, so the kernel is bound by memory.
#include <algorithm>

#include "gsr_internal.h"

namespace gsr {

__device__ inline float3 f3(const float* p, int i) { return make_float3(p[3 * i + 0], p[3 * i + 1], p[3 * i + 2]); }
__device__ inline float3 sub3(float3 a, float3 b) { return make_float3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ inline float3 cross3(float3 a, float3 b) {
    return make_float3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ inline float norm3(float3 a) { return sqrtf(a.x * a.x + a.y * a.y + a.z * a.z); }

__global__ __launch_bounds__(256) void k_mesh_to_gs(long long n_faces, long long n_verts, const float* __restrict__ verts,
                                                    const float* __restrict__ colours, const int32_t* __restrict__ faces,
                                                    float flatten, float opacity, int K, gsr_gaussian_grads out,
                                                    uint32_t* bad) {
    for (long long f = (long long)blockIdx.x * blockDim.x + threadIdx.x; f < n_faces;
         f += (long long)gridDim.x * blockDim.x) {
        const int ia = faces[3 * f + 0], ib = faces[3 * f + 1], ic = faces[3 * f + 2];
        const bool in_range = ia >= 0 && ib >= 0 && ic >= 0 && ia < n_verts && ib < n_verts && ic < n_verts;
        float3 g = make_float3(0.f, 0.f, 0.f), col = make_float3(0.5f, 0.5f, 0.5f);
        float st = 0.f, qw = 1.f, qx = 0.f, qy = 0.f, qz = 0.f, op = 0.f;
        if (!in_range) {
            atomicAdd(bad, 1u);
        } else {
            const float3 a = f3(verts, ia), b = f3(verts, ib), c = f3(verts, ic);
            g = make_float3((a.x + b.x + c.x) / 3.0f, (a.y + b.y + c.y) / 3.0f, (a.z + b.z + c.z) / 3.0f);
            st = (norm3(sub3(a, g)) + norm3(sub3(b, g)) + norm3(sub3(c, g))) / 3.0f;
            const float3 e = sub3(b, a), cr = cross3(e, sub3(c, a));
            const float area2 = norm3(cr), el = norm3(e);
            if (colours) {
                const float3 ca = f3(colours, ia), cb = f3(colours, ib), cc = f3(colours, ic);
                col = make_float3((ca.x + cb.x + cc.x) / 3.0f, (ca.y + cb.y + cc.y) / 3.0f, (ca.z + cb.z + cc.z) / 3.0f);
            }
            if (area2 > 0.0f && el > 0.0f) {
                op = opacity;
                const float3 n = make_float3(cr.x / area2, cr.y / area2, cr.z / area2);
                const float3 t1 = make_float3(e.x / el, e.y / el, e.z / el);
                const float3 t2 = cross3(n, t1);
                // columns (t1, t2, n) -> unit quaternion by Shepperd's method: the largest of
                // 4w^2, 4x^2, 4y^2, 4z^2 is taken from the trace or a diagonal element, the
                // other components from the off-diagonal sums and differences
                const float R00 = t1.x, R01 = t2.x, R02 = n.x, R10 = t1.y, R11 = t2.y, R12 = n.y, R20 = t1.z,
                            R21 = t2.z, R22 = n.z;
                const float tr = R00 + R11 + R22;
                if (tr > 0.0f) {
                    const float s = 2.0f * sqrtf(tr + 1.0f);
                    qw = 0.25f * s; qx = (R21 - R12) / s; qy = (R02 - R20) / s; qz = (R10 - R01) / s;
                } else if (R00 > R11 && R00 > R22) {
                    const float s = 2.0f * sqrtf(1.0f + R00 - R11 - R22);
                    qw = (R21 - R12) / s; qx = 0.25f * s; qy = (R01 + R10) / s; qz = (R02 + R20) / s;
                } else if (R11 > R22) {
                    const float s = 2.0f * sqrtf(1.0f + R11 - R00 - R22);
                    qw = (R02 - R20) / s; qx = (R01 + R10) / s; qy = 0.25f * s; qz = (R12 + R21) / s;
                } else {
                    const float s = 2.0f * sqrtf(1.0f + R22 - R00 - R11);
                    qw = (R10 - R01) / s; qx = (R02 + R20) / s; qy = (R12 + R21) / s; qz = 0.25f * s;
                }
            }
        }
        if (out.means) {
            out.means[3 * f + 0] = g.x;
            out.means[3 * f + 1] = g.y;
            out.means[3 * f + 2] = g.z;
        }
        if (out.scales) {
            out.scales[3 * f + 0] = st;
            out.scales[3 * f + 1] = st;
            out.scales[3 * f + 2] = flatten * st;
        }
        if (out.quats) {
            out.quats[4 * f + 0] = qw;
            out.quats[4 * f + 1] = qx;
            out.quats[4 * f + 2] = qy;
            out.quats[4 * f + 3] = qz;
        }
        if (out.opacities) out.opacities[f] = op;
        if (out.sh) {
            // DC coefficient (colour - 1/2) / C0 with C0 = 1 / (2 sqrt(pi))
            const float ic0 = 3.5449077018110318f;  // 2 sqrt(pi)
            float* sh = out.sh + f * (3 * K);
            sh[0] = (col.x - 0.5f) * ic0;
            sh[1] = (col.y - 0.5f) * ic0;
            sh[2] = (col.z - 0.5f) * ic0;
            for (int k = 3; k < 3 * K; ++k) sh[k] = 0.0f;
        }
    }
}

hipError_t launch_mesh_to_gs(long long n_faces, long long n_verts, const float* verts, const float* colours,
                             const int32_t* faces, float flatten, float opacity, int K, const gsr_gaussian_grads& out,
                             uint32_t* bad, int num_cu, hipStream_t s) {
    if (n_faces <= 0) return hipSuccess;
    const long long want = (n_faces + 255) / 256, cap = (long long)num_cu * 16;
    hipLaunchKernelGGL(k_mesh_to_gs, dim3((unsigned)std::max(1ll, std::min(want, cap))), dim3(256), 0, s, n_faces,
                       n_verts, verts, colours, faces, flatten, opacity, K, out, bad);
    return hipGetLastError();
}

}  // namespace gsr
