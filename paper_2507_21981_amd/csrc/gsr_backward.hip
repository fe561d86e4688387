// Backward path: gradients of a loss on the RGB, depth and alpha frames with respect to the
// node-local Gaussian parameters (means, activated scales, unnormalised quaternions,
// activated opacities, SH coefficients).  Optimising Gaussians against depth and opacity
// terms (paper Sec. IV-B, mesh-to-Gaussian transfer) needs exactly these gradients.
//
//   k_zero            clear the per-(image, Gaussian) record gradients
//   k_composite_bwd   per tile, back to front from each pixel's last blended entry; the
//                     transmittance in front of an entry is recomputed as T / (1 - alpha)
//                     rather than stored; per-entry gradients are summed over a wavefront
//                     before one atomic add per record field
//   k_project_bwd     per Gaussian, all cameras of its env: chain from the record gradients
//                     (u, v, conic, opacity, colour, z) to the parameters, accumulated (+=)
//
// Compositing gradients for a blended entry i with transmittance T_i in front of it, weight
// w_i = alpha_i T_i, and behind-sums S^C_i = sum_{j>i} c_j w_j + T_final bg, S^D_i likewise
// with z and no background:
//   dL/dc_i = gC w_i,  dL/dz_i = gD w_i,
//   dL/dalpha_i = gC.(c_i T_i - S^C_i/(1 - alpha_i)) + gD (z_i T_i - S^D_i/(1 - alpha_i))
//                 + gA T_final/(1 - alpha_i),
// then through alpha = o G (no gradient where the 0.99 clamp is active) and
// G = exp(-1/2 (A dx^2 + C dy^2) - B dx dy) to o, (u, v) and the conic (A, B, C).
#include <algorithm>

#include "gsr_internal.h"

namespace gsr {

__global__ void k_zero(float4* p, size_t n4) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (size_t)gridDim.x * blockDim.x)
        p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// v + (v of another lane) by a DPP move: ctrl selects the source lane, row_mask the rows of
// 16 lanes that add (the others add zero)
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_add(float v) {
    const int m = __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, false);
    return v + __int_as_float(m);
}
// Sum over the wavefront, complete in lane 63, with data-parallel-primitive moves only (no
// LDS crossbar): quads (swap neighbours, then pairs), half rows (mirror), rows (mirror), then
// row 0 into row 1 and row 2 into row 3 (broadcast of lane 15), rows 0-1 into rows 2-3
// (broadcast of lane 31).
__device__ __forceinline__ float wave_sum63(float v) {
    v = dpp_add<0xB1, 0xF>(v);   // quad_perm [1, 0, 3, 2]
    v = dpp_add<0x4E, 0xF>(v);   // quad_perm [2, 3, 0, 1]
    v = dpp_add<0x141, 0xF>(v);  // row_half_mirror
    v = dpp_add<0x140, 0xF>(v);  // row_mirror
    v = dpp_add<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v = dpp_add<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}

// x + y across the two halves of the wavefront, x's sum in lanes 0-31 and y's in lanes 32-63
// (lane i < 32: x[i] + x[i + 32]; lane i >= 32: y[i - 32] + y[i]): one lane-half swap
__device__ __forceinline__ float half_pair(float x, float y) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_int(x), __float_as_int(y), false, false);
    return __int_as_float(r[0]) + __int_as_float(r[1]);
}
// for p, q each holding one field per half (from half_pair): rows 0 and 1 of the result hold
// p's and q's lower-half fields summed over rows 0+1, rows 2 and 3 their upper-half fields
// summed over rows 2+3: one row swap (odd rows of p with even rows of q)
__device__ __forceinline__ float row_pair(float p, float q) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_int(p), __float_as_int(q), false, false);
    return __int_as_float(r[0]) + __int_as_float(r[1]);
}
// the sum over each row of 16 lanes, in every lane of the row
__device__ __forceinline__ float row_sum16(float v) {
    v = dpp_add<0xB1, 0xF>(v);   // quad_perm [1, 0, 3, 2]
    v = dpp_add<0x4E, 0xF>(v);   // quad_perm [2, 3, 0, 1]
    v = dpp_add<0x141, 0xF>(v);  // row_half_mirror
    v = dpp_add<0x140, 0xF>(v);  // row_mirror
    return v;
}

// One wavefront per tile; each lane takes PPT = TW TH / 64 pixels of one column (pixel p of a
// lane sits 64 / TW rows below pixel p - 1).  The wavefront walks the tile's list back to front
// from the largest contributor count among its pixels, in batches of 64 entries staged in LDS;
// entries that cannot reach the batch's participating pixels (the forward's conservative
// rectangle test on their bounding box) are dropped from each batch first (they blended
// nothing there).  A lane sums its pixels' gradient contributions to an entry in registers,
// so each (tile, entry) costs one wavefront reduction and one atomic add per record field.
template <int TW, int TH>
__global__ __launch_bounds__(64) void k_composite_bwd(BwdArgs b) {
    constexpr int PPT = TW * TH / 64;
    constexpr int LR = 64 / TW;  // rows between a lane's pixels
    const FwdArgs& a = b.f;
    __shared__ float4 s0[64], s1[64], s2[64];
    __shared__ long long s_rec[64];
    __shared__ uint32_t s_e[64];
    __shared__ uint32_t s_tile;
    const int lane = threadIdx.x;
    // tiles longest list first (the forward's length classes, longest class first, the tiles
    // with at most one entry last), so the longest walks do not start at the end of the grid
    if (lane == 0) {
        uint32_t i = blockIdx.x;
        const int order[kNumClasses] = {kLenLong, 4, 3, 2, 1, 0, kLenNone};
        uint32_t tile = 0u;
        for (int k = 0; k < kNumClasses; ++k) {
            const uint32_t n = a.status->cls[order[k]];
            if (i < n) {
                tile = a.cls_list[(size_t)order[k] * a.tiles + i];
                break;
            }
            i -= n;
        }
        s_tile = tile;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const long long t = (long long)s_tile;
    const int image = (int)(t / a.tpi);
    const int lt = (int)(t - (long long)image * a.tpi);
    const int ty = lt / a.tiles_x, tx = lt - ty * a.tiles_x;
    const int px = tx * TW + lane % TW, py0 = ty * TH + lane / TW;
    const uint32_t start = a.starts[t];
    const int env = image / a.C, cam = image - env * a.C;
    const Env ev = a.envs[env];
    const long long rec_off = (long long)a.C * ev.gid_base + (long long)cam * ev.n - (long long)ev.gid_base;
    const gsr_camera& cm = a.cams[image];
    const float bgr = cm.bg[0], bgg = cm.bg[1], bgb = cm.bg[2];
    bool inside[PPT];
    uint32_t last[PPT];
    float Tf[PPT], gr[PPT], gg[PPT], gb[PPT], gD[PPT], gA[PPT], T[PPT], SCr[PPT], SCg[PPT], SCb[PPT], SD[PPT],
        fpy[PPT];
    uint32_t wmax = 0;
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int py = py0 + q * LR;
        inside[q] = px < a.width && py < a.height;
        fpy[q] = (float)py + 0.5f;
        last[q] = 0;
        Tf[q] = 1.0f;
        gr[q] = gg[q] = gb[q] = gD[q] = gA[q] = 0.0f;
        if (inside[q]) {
            const size_t p = ((size_t)image * a.height + py) * a.width + px;
            last[q] = a.n_contrib[p];
            Tf[q] = a.T_final[p];
            gr[q] = b.d_rgb[3 * p + 0];
            gg[q] = b.d_rgb[3 * p + 1];
            gb[q] = b.d_rgb[3 * p + 2];
            gD[q] = b.d_depth ? b.d_depth[p] : 0.0f;
            gA[q] = b.d_alpha ? b.d_alpha[p] : 0.0f;
        }
        T[q] = Tf[q];
        SCr[q] = Tf[q] * bgr;
        SCg[q] = Tf[q] * bgg;
        SCb[q] = Tf[q] * bgb;
        SD[q] = 0.0f;
        wmax = last[q] > wmax ? last[q] : wmax;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t o = __shfl_xor(wmax, off, 64);
        wmax = o > wmax ? o : wmax;
    }
    const float fpx = (float)px + 0.5f;
    const float thr = (float)(1.0 / 255.0);
    const float qcut = -7.994353436858858f - 1e-3f;  // log2(1/255) - 1e-3, as in the forward
    const float rx0 = (float)(tx * TW) + 0.5f, ry0 = (float)(ty * TH) + 0.5f;  // first pixel's centre
    for (uint32_t hi = wmax; hi > 0;) {
        const uint32_t lo = hi > 64u ? hi - 64u : 0u;
        // bounding box of the pixels that take part in this batch (those with a contributor
        // count above lo; lane l holds column l % TW and row l / TW + q LR): entries that
        // cannot reach it change no pixel and receive no gradient from this tile
        unsigned long long act = 0;
        int ar0 = TH, ar1 = -1;
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            const unsigned long long m = __ballot(inside[q] && last[q] > lo);
            if (m) {
                act |= m;
                ar0 = min(ar0, (int)__builtin_ctzll(m) / TW + q * LR);
                ar1 = max(ar1, (63 - (int)__builtin_clzll(m)) / TW + q * LR);
            }
        }
        if (!act) break;  // not reached: the pixel with count wmax takes part in every batch
#pragma unroll
        for (int sft = 32; sft >= TW; sft >>= 1) act |= act >> sft;
        act &= (TW == 32 ? 0xffffffffull : ((1ull << TW) - 1ull));
        const float bx0 = rx0 + (float)__builtin_ctzll(act), bx1 = rx0 + (float)(63 - (int)__builtin_clzll(act));
        const float by0 = ry0 + (float)ar0, by1 = ry0 + (float)ar1;
        // stage entries hi - 1, hi - 2, ... (descending) that can reach this tile's pixels
        const uint32_t e = hi - 1u - (uint32_t)lane;
        bool keep = false;
        Record R;
        long long rec = -1;
        if (lane < (int)(hi - lo)) {
            const uint32_t gid = (uint32_t)a.pairs[start + e];
            if (gid - ev.gid_base < ev.n) {
                rec = rec_off + gid;
                R = a.records[rec];
                keep = reaches_rect(R, bx0, bx1, by0, by1, qcut);
            }
        }
        const unsigned long long km = __ballot(keep);
        if (keep) {
            const int slot = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(km >> 32),
                                                            __builtin_amdgcn_mbcnt_lo((uint32_t)km, 0u));
            s0[slot] = R.r0;
            s1[slot] = R.r1;
            s2[slot] = R.r2;
            s_rec[slot] = rec;
            s_e[slot] = e;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int n = __popcll(km);
        for (int k = 0; k < n; ++k) {
            const uint32_t ek = s_e[k];
            const float4 r0 = s0[k];
            const float4 r1 = s1[k];
            const float4 r2 = s2[k];
            const float A2 = -0.7213475204444817f * r1.x, B2 = -1.4426950408889634f * r1.y,
                        C2 = -0.7213475204444817f * r1.z;
            const float dx = fpx - r0.x;
            const float Adx = A2 * dx, Bdx = B2 * dx;
            const float qx = fmaf(Adx, dx, r1.w);
            const float io = __builtin_amdgcn_rcpf(r0.z);  // 1 / opacity
            float g_u = 0.f, g_v = 0.f, g_A = 0.f, g_B = 0.f, g_C = 0.f, g_o = 0.f, g_r = 0.f, g_g = 0.f,
                  g_b = 0.f, g_z = 0.f;
            bool contrib = false;
#pragma unroll
            for (int q = 0; q < PPT; ++q) {
                if (!(inside[q] && ek < last[q])) continue;
                const float dy = fpy[q] - r0.y;
                // the forward's operations exactly, so the same entries are blended:
                // q = A' dx^2 + B' dx dy + C' dy^2 + log2 o, alpha = min(0.99, exp2(q))
                const float qq = fmaf(Bdx, dy, fmaf(C2 * dy, dy, qx));
                const float oG = __builtin_amdgcn_exp2f(qq);  // o G, alpha before the clamp
                const float al = fminf(0.99f, oG);
                if (!(al >= thr)) continue;
                contrib = true;
                const float om = 1.0f - al;
                // the transmittance in front, T / (1 - alpha); values only, no decision
                // depends on them, so the hardware reciprocal (about 1 ulp) is enough
                const float iom = __builtin_amdgcn_rcpf(om);
                const float Ti = T[q] * iom;
                const float w = al * Ti;
                g_r = fmaf(gr[q], w, g_r);
                g_g = fmaf(gg[q], w, g_g);
                g_b = fmaf(gb[q], w, g_b);
                g_z = fmaf(gD[q], w, g_z);
                float dLda = gr[q] * (r2.x * Ti - SCr[q] * iom) + gg[q] * (r2.y * Ti - SCg[q] * iom) +
                             gb[q] * (r2.z * Ti - SCb[q] * iom);
                dLda += gD[q] * (r0.w * Ti - SD[q] * iom);
                dLda += gA[q] * Tf[q] * iom;
                SCr[q] = fmaf(r2.x, w, SCr[q]);
                SCg[q] = fmaf(r2.y, w, SCg[q]);
                SCb[q] = fmaf(r2.z, w, SCb[q]);
                SD[q] = fmaf(r0.w, w, SD[q]);
                T[q] = Ti;
                if (oG < 0.99f) {
                    g_o = fmaf(dLda, oG * io, g_o);  // d alpha / d o = G
                    const float dp = dLda * oG;        // dL/dpower, power = -1/2 A dx^2 - B dx dy - 1/2 C dy^2
                    g_u = fmaf(dp, r1.x * dx + r1.y * dy, g_u);
                    g_v = fmaf(dp, r1.z * dy + r1.y * dx, g_v);
                    g_A = fmaf(-0.5f * dp, dx * dx, g_A);
                    g_B = fmaf(-dp, dx * dy, g_B);
                    g_C = fmaf(-0.5f * dp, dy * dy, g_C);
                }
            }
            // one atomic per field per tile and entry, after a transposing wavefront reduction:
            // lane-half swaps pair the ten fields into five registers (lanes 0-31 one field,
            // 32-63 another), row swaps pair those into two registers holding four fields (one
            // per row of 16 lanes) and one holding two, and row sums by DPP finish them, so the
            // ten totals sit in lanes 15, 31, 47, 63 of three registers
            if (__any(contrib)) {
                const float R0 = half_pair(g_u, g_v), R1 = half_pair(g_A, g_B), R2 = half_pair(g_C, g_o),
                            R3 = half_pair(g_r, g_g), R4 = half_pair(g_b, g_z);
                // rows of Z0: u, A, v, B; rows of Z1: C, r, o, g
                const float Z0 = row_sum16(row_pair(R0, R1)), Z1 = row_sum16(row_pair(R2, R3));
                const float Z2 = dpp_add<0x142, 0xA>(row_sum16(R4));  // rows 1 and 3: b and z
                if ((lane & 15) == 15) {
                    float* o = b.g2d + (size_t)s_rec[k] * 12;
                    const int row = lane >> 4, f = (row & 1) * 2 + (row >> 1);  // rows 0-3 -> 0, 2, 1, 3
                    atomicAdd(o + f, Z0);
                    atomicAdd(o + 4 + f, Z1);
                    if (row & 1) atomicAdd(o + 8 + (row >> 1), Z2);
                }
            }
        }
        // all lanes are done reading this batch before the next one overwrites it
        __builtin_amdgcn_wave_barrier();
        hi = lo;
    }
}

// d/d(x, y, z) of the SH basis polynomials (the forms used by the forward pass); the caller
// projects onto the sphere's tangent plane, which removes the radial part where the
// polynomial extensions of a basis function may differ.
template <int L>
__device__ inline void sh_basis_grad(float x, float y, float z, float* gx, float* gy, float* gz) {
    gx[0] = gy[0] = gz[0] = 0.f;
    if (L >= 1) {
        const float c1 = 0.48860251903533936f;
        gx[1] = 0.f; gy[1] = -c1; gz[1] = 0.f;
        gx[2] = 0.f; gy[2] = 0.f; gz[2] = c1;
        gx[3] = -c1; gy[3] = 0.f; gz[3] = 0.f;
    }
    if (L >= 2) {
        const float a = 1.0925484895706177f, b = 0.31539157032966614f, c = 0.5462742447853088f;
        gx[4] = a * y; gy[4] = a * x; gz[4] = 0.f;
        gx[5] = 0.f; gy[5] = -a * z; gz[5] = -a * y;
        gx[6] = -2.f * b * x; gy[6] = -2.f * b * y; gz[6] = 4.f * b * z;
        gx[7] = -a * z; gy[7] = 0.f; gz[7] = -a * x;
        gx[8] = 2.f * c * x; gy[8] = -2.f * c * y; gz[8] = 0.f;
        if (L >= 3) {
            const float d = 0.5900436043739319f, e = 2.890611410140991f, f = 0.4570457935333252f,
                        g = 0.37317633628845215f, h = 1.4453057050704956f;
            const float xx = x * x, yy = y * y, zz = z * z;
            gx[9] = -6.f * d * x * y; gy[9] = -3.f * d * (xx - yy); gz[9] = 0.f;
            gx[10] = e * y * z; gy[10] = e * x * z; gz[10] = e * x * y;
            gx[11] = 2.f * f * x * y; gy[11] = -f * (4.f * zz - xx - 3.f * yy); gz[11] = -8.f * f * y * z;
            gx[12] = -6.f * g * x * z; gy[12] = -6.f * g * y * z; gz[12] = g * (6.f * zz - 3.f * xx - 3.f * yy);
            gx[13] = -f * (4.f * zz - 3.f * xx - yy); gy[13] = 2.f * f * x * y; gz[13] = -8.f * f * x * z;
            gx[14] = 2.f * h * x * z; gy[14] = -2.f * h * y * z; gz[14] = h * (xx - yy);
            gx[15] = -3.f * d * (xx - yy); gy[15] = 6.f * d * x * y; gz[15] = 0.f;
        }
    }
}

template <int L>
__device__ inline void sh_basis_b(float x, float y, float z, float* Y) {
    Y[0] = 0.282094806432724f;
    if (L >= 1) {
        Y[1] = -0.48860251903533936f * y;
        Y[2] = 0.48860251903533936f * z;
        Y[3] = -0.48860251903533936f * x;
    }
    if (L >= 2) {
        const float xx = x * x, yy = y * y, zz = z * z;
        Y[4] = 1.0925484895706177f * (x * y);
        Y[5] = -1.0925484895706177f * (y * z);
        Y[6] = 0.31539157032966614f * (2.0f * zz - xx - yy);
        Y[7] = -1.0925484895706177f * (x * z);
        Y[8] = 0.5462742447853088f * (xx - yy);
        if (L >= 3) {
            Y[9] = -0.5900436043739319f * y * (3.0f * xx - yy);
            Y[10] = 2.890611410140991f * (x * y) * z;
            Y[11] = -0.4570457935333252f * y * (4.0f * zz - xx - yy);
            Y[12] = 0.37317633628845215f * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
            Y[13] = -0.4570457935333252f * x * (4.0f * zz - xx - yy);
            Y[14] = 1.4453057050704956f * z * (xx - yy);
            Y[15] = -0.5900436043739319f * x * (xx - 3.0f * yy);
        }
    }
}

// One Gaussian (lane i of block blk) of the backward projection.  pose[0..5] receives its share
// of the node-pose gradient in node-local terms: A = mu x g_p + sum_c (c_c x g_d,c) + vee(dRq Rq^T)
// and B = g_p + g_d, with g_p the mean's gradient through the projection, g_d,c that through
// camera c's view direction (centre c_c, node frame) and dRq that of the rotation R(q/|q|).
template <int L>
__device__ __forceinline__ void project_bwd_gaussian(const BwdArgs& b, const Block& blk, int i, float* pose) {
    const FwdArgs& a = b.f;
    constexpr int K = (L + 1) * (L + 1);
    const Node nd = a.nodes[blk.node];
    const Env ev = a.envs[blk.env];
    const gsr_gaussian_grads gd = b.grads_dev[blk.node];
    const int C = a.C;
    const uint32_t gid = blk.gid0 + i;
    const size_t li = gid - nd.gid_base;
    const size_t lg = gid - ev.gid_base;
    const float mu0 = nd.means[3 * li + 0], mu1 = nd.means[3 * li + 1], mu2 = nd.means[3 * li + 2];
    float dmu0 = 0.f, dmu1 = 0.f, dmu2 = 0.f, ds0 = 0.f, ds1 = 0.f, ds2 = 0.f, dop = 0.f;
    float dR[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) dR[k] = 0.f;
    float dsh[K * 3];
#pragma unroll
    for (int k = 0; k < K * 3; ++k) dsh[k] = 0.f;
    float gp0 = 0.f, gp1 = 0.f, gp2 = 0.f, cg0 = 0.f, cg1 = 0.f, cg2 = 0.f;  // pose terms
    bool any = false;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, qw = 0.f, qx = 0.f, qy = 0.f, qz = 0.f, rn = 0.f;
    float R00 = 0.f, R01 = 0.f, R02 = 0.f, R10 = 0.f, R11 = 0.f, R12 = 0.f, R20 = 0.f, R21 = 0.f, R22 = 0.f;
    for (int c = 0; c < C; ++c) {
        const size_t rec = (size_t)C * ev.gid_base + (size_t)c * ev.n + lg;
        const float4* g4 = reinterpret_cast<const float4*>(b.g2d + rec * 12);
        const float4 ga = g4[0], gb4 = g4[1], gc = g4[2];
        // ga = (du, dv, dA, dB), gb4 = (dC, do, dr, dg), gc = (db, dz, -, -)
        if (ga.x == 0.f && ga.y == 0.f && ga.z == 0.f && ga.w == 0.f && gb4.x == 0.f && gb4.y == 0.f &&
            gb4.z == 0.f && gb4.w == 0.f && gc.x == 0.f && gc.y == 0.f)
            continue;
        if (!any) {
            any = true;
            s0 = nd.scales[3 * li + 0]; s1 = nd.scales[3 * li + 1]; s2 = nd.scales[3 * li + 2];
            const float4 q = reinterpret_cast<const float4*>(nd.quats)[li];
            const float n2 = fmaf(q.x, q.x, fmaf(q.y, q.y, fmaf(q.z, q.z, q.w * q.w)));
            rn = 1.0f / sqrtf(n2);
            qw = q.x * rn; qx = q.y * rn; qy = q.z * rn; qz = q.w * rn;
            const float xx = qx * qx, yy = qy * qy, zz = qz * qz;
            const float xy = qx * qy, xzq = qx * qz, yzq = qy * qz;
            const float wx = qw * qx, wy = qw * qy, wz = qw * qz;
            R00 = fmaf(-2.0f, yy + zz, 1.0f); R01 = 2.0f * (xy - wz); R02 = 2.0f * (xzq + wy);
            R10 = 2.0f * (xy + wz); R11 = fmaf(-2.0f, xx + zz, 1.0f); R12 = 2.0f * (yzq - wx);
            R20 = 2.0f * (xzq - wy); R21 = 2.0f * (yzq + wx); R22 = fmaf(-2.0f, xx + yy, 1.0f);
        }
        const View& v = a.views[blk.node * C + c];
        // forward quantities, same operations as the projection
        const float p0 = fmaf(v.W[0], mu0, fmaf(v.W[1], mu1, fmaf(v.W[2], mu2, v.w[0])));
        const float p1 = fmaf(v.W[3], mu0, fmaf(v.W[4], mu1, fmaf(v.W[5], mu2, v.w[1])));
        const float z = fmaf(v.W[6], mu0, fmaf(v.W[7], mu1, fmaf(v.W[8], mu2, v.w[2])));
        const float iz = 1.0f / z;
        const float xz = p0 * iz, yz = p1 * iz;
        float G[9], M[9];
        const float Rm[9] = {R00, R01, R02, R10, R11, R12, R20, R21, R22};
        const float sv[3] = {s0, s1, s2};
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                G[r * 3 + cc] = fmaf(v.W[r * 3 + 0], Rm[0 * 3 + cc], fmaf(v.W[r * 3 + 1], Rm[1 * 3 + cc], v.W[r * 3 + 2] * Rm[2 * 3 + cc]));
                M[r * 3 + cc] = G[r * 3 + cc] * sv[cc];
            }
        const float S00 = fmaf(M[0], M[0], fmaf(M[1], M[1], M[2] * M[2]));
        const float S01 = fmaf(M[0], M[3], fmaf(M[1], M[4], M[2] * M[5]));
        const float S02 = fmaf(M[0], M[6], fmaf(M[1], M[7], M[2] * M[8]));
        const float S11 = fmaf(M[3], M[3], fmaf(M[4], M[4], M[5] * M[5]));
        const float S12 = fmaf(M[3], M[6], fmaf(M[4], M[7], M[5] * M[8]));
        const float S22 = fmaf(M[6], M[6], fmaf(M[7], M[7], M[8] * M[8]));
        const bool clx = xz < -v.limx || xz > v.limx, cly = yz < -v.limy || yz > v.limy;
        const float xc = fminf(fmaxf(xz, -v.limx), v.limx);
        const float yc = fminf(fmaxf(yz, -v.limy), v.limy);
        const float j00 = v.fx * iz, j11 = v.fy * iz;
        const float j02 = -(j00 * xc), j12 = -(j11 * yc);
        const float T00 = fmaf(j00, S00, j02 * S02), T01 = fmaf(j00, S01, j02 * S12), T02 = fmaf(j00, S02, j02 * S22);
        const float T10 = fmaf(j11, S01, j12 * S02), T11 = fmaf(j11, S11, j12 * S12), T12 = fmaf(j11, S12, j12 * S22);
        const float ca = fmaf(T00, j00, T02 * j02) + 0.3f;
        const float cb = fmaf(T01, j11, T02 * j12);
        const float cc2 = fmaf(T11, j11, T12 * j12) + 0.3f;
        const float idet = 1.0f / fmaf(ca, cc2, -(cb * cb));
        const float QA = cc2 * idet, QB = -cb * idet, QC = ca * idet;
        // conic -> Sigma2D: H = -Q Gm Q with Gm = [[dA, dB/2], [dB/2, dC]]
        const float dA = ga.z, dB = ga.w, dC = gb4.x;
        const float m00 = QA * dA + QB * 0.5f * dB, m01 = QA * 0.5f * dB + QB * dC;
        const float m10 = QB * dA + QC * 0.5f * dB, m11 = QB * 0.5f * dB + QC * dC;
        const float H00 = -(m00 * QA + m01 * QB), H01 = -(m00 * QB + m01 * QC), H11 = -(m10 * QB + m11 * QC);
        // Sigma2D = J Sigma J^T: dSigma = J^T H J, dJ = 2 H J Sigma
        const float dS00 = j00 * j00 * H00;
        const float dS01 = j00 * j11 * H01;
        const float dS02 = j00 * (H00 * j02 + H01 * j12);
        const float dS11 = j11 * j11 * H11;
        const float dS12 = j11 * (H01 * j02 + H11 * j12);
        const float dS22 = j02 * j02 * H00 + 2.f * j02 * j12 * H01 + j12 * j12 * H11;
        const float dJ00 = 2.f * (H00 * T00 + H01 * T10);
        const float dJ02 = 2.f * (H00 * T02 + H01 * T12);
        const float dJ11 = 2.f * (H01 * T01 + H11 * T11);
        const float dJ12 = 2.f * (H01 * T02 + H11 * T12);
        // camera-space mean
        const float du = ga.x, dv = ga.y, dz = gc.y;
        float dp0 = du * v.fx * iz;
        float dp1 = dv * v.fy * iz;
        float dp2 = -du * v.fx * xz * iz - dv * v.fy * yz * iz + dz;
        dp2 += -(dJ00 * v.fx + dJ11 * v.fy) * iz * iz;
        if (!clx) { dp0 += -dJ02 * v.fx * iz * iz; dp2 += 2.f * dJ02 * v.fx * xz * iz * iz; }
        else dp2 += dJ02 * v.fx * xc * iz * iz;
        if (!cly) { dp1 += -dJ12 * v.fy * iz * iz; dp2 += 2.f * dJ12 * v.fy * yz * iz * iz; }
        else dp2 += dJ12 * v.fy * yc * iz * iz;
        // p = W mu + w
        {
            const float m0 = v.W[0] * dp0 + v.W[3] * dp1 + v.W[6] * dp2;
            const float m1 = v.W[1] * dp0 + v.W[4] * dp1 + v.W[7] * dp2;
            const float m2 = v.W[2] * dp0 + v.W[5] * dp1 + v.W[8] * dp2;
            dmu0 += m0; dmu1 += m1; dmu2 += m2;
            gp0 += m0; gp1 += m1; gp2 += m2;
        }
        // Sigma = M M^T: dM = 2 dSigma M  (dSigma symmetric)
        const float dSm[9] = {dS00, dS01, dS02, dS01, dS11, dS12, dS02, dS12, dS22};
        float dG[9];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                const float dM = 2.f * (dSm[r * 3 + 0] * M[0 * 3 + cc] + dSm[r * 3 + 1] * M[1 * 3 + cc] + dSm[r * 3 + 2] * M[2 * 3 + cc]);
                if (cc == 0) ds0 += dM * G[r * 3 + cc];
                if (cc == 1) ds1 += dM * G[r * 3 + cc];
                if (cc == 2) ds2 += dM * G[r * 3 + cc];
                dG[r * 3 + cc] = dM * sv[cc];
            }
        // G = W R: dR += W^T dG
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc)
                dR[r * 3 + cc] += v.W[0 * 3 + r] * dG[0 * 3 + cc] + v.W[1 * 3 + r] * dG[1 * 3 + cc] + v.W[2 * 3 + r] * dG[2 * 3 + cc];
        // opacity
        dop += gb4.y;
        // colour: c = max(0, sum sh Y(d) + 0.5), d = mu - centre (node-local)
        const float ddx = mu0 - v.cl[0], ddy = mu1 - v.cl[1], ddz = mu2 - v.cl[2];
        const float len = sqrtf(ddx * ddx + ddy * ddy + ddz * ddz);
        const float il = 1.0f / len;
        const float x = ddx * il, y = ddy * il, zq = ddz * il;
        float Y[K], gx[K], gy[K], gz[K];
        sh_basis_b<L>(x, y, zq, Y);
        const float* shp = nd.sh + li * (K * 3);
        float pre[3] = {0.5f, 0.5f, 0.5f};
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) pre[ch] = fmaf(Y[k], shp[3 * k + ch], pre[ch]);
        const float gcol[3] = {pre[0] < 0.f ? 0.f : gb4.z, pre[1] < 0.f ? 0.f : gb4.w, pre[2] < 0.f ? 0.f : gc.x};
        if (gcol[0] != 0.f || gcol[1] != 0.f || gcol[2] != 0.f) {
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) dsh[3 * k + ch] = fmaf(gcol[ch], Y[k], dsh[3 * k + ch]);
            if (L > 0) {
                sh_basis_grad<L>(x, y, zq, gx, gy, gz);
                float ex = 0.f, ey = 0.f, ez = 0.f;
#pragma unroll
                for (int k = 1; k < K; ++k) {
                    const float wk = gcol[0] * shp[3 * k + 0] + gcol[1] * shp[3 * k + 1] + gcol[2] * shp[3 * k + 2];
                    ex = fmaf(wk, gx[k], ex);
                    ey = fmaf(wk, gy[k], ey);
                    ez = fmaf(wk, gz[k], ez);
                }
                const float dot = ex * x + ey * y + ez * zq;
                const float d0 = (ex - dot * x) * il, d1 = (ey - dot * y) * il, d2 = (ez - dot * zq) * il;
                dmu0 += d0;
                dmu1 += d1;
                dmu2 += d2;
                cg0 += v.cl[1] * d2 - v.cl[2] * d1;
                cg1 += v.cl[2] * d0 - v.cl[0] * d2;
                cg2 += v.cl[0] * d1 - v.cl[1] * d0;
            }
        }
    }
    if (!any) return;
    {
        // N = dRq Rq^T; its antisymmetric part is the rotation frame's share of the pose gradient
        const float Rm[9] = {R00, R01, R02, R10, R11, R12, R20, R21, R22};
        float N[9];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc)
                N[r * 3 + cc] = dR[r * 3 + 0] * Rm[cc * 3 + 0] + dR[r * 3 + 1] * Rm[cc * 3 + 1] + dR[r * 3 + 2] * Rm[cc * 3 + 2];
        pose[0] = mu1 * gp2 - mu2 * gp1 + cg0 + (N[7] - N[5]);
        pose[1] = mu2 * gp0 - mu0 * gp2 + cg1 + (N[2] - N[6]);
        pose[2] = mu0 * gp1 - mu1 * gp0 + cg2 + (N[3] - N[1]);
        pose[3] = dmu0;
        pose[4] = dmu1;
        pose[5] = dmu2;
    }
    // R(q_hat) -> q_hat (w, x, y, z), then through q_hat = q / |q|
    const float* Gq = dR;
    float dw = 2.f * (-qz * Gq[1] + qy * Gq[2] + qz * Gq[3] - qx * Gq[5] - qy * Gq[6] + qx * Gq[7]);
    float dx = 2.f * (qy * Gq[1] + qz * Gq[2] + qy * Gq[3] - 2.f * qx * Gq[4] - qw * Gq[5] + qz * Gq[6] + qw * Gq[7] - 2.f * qx * Gq[8]);
    float dy = 2.f * (-2.f * qy * Gq[0] + qx * Gq[1] + qw * Gq[2] + qx * Gq[3] + qz * Gq[5] - qw * Gq[6] + qz * Gq[7] - 2.f * qy * Gq[8]);
    float dzq = 2.f * (-2.f * qz * Gq[0] - qw * Gq[1] + qx * Gq[2] + qw * Gq[3] - 2.f * qz * Gq[4] + qy * Gq[5] + qx * Gq[6] + qy * Gq[7]);
    const float dd = dw * qw + dx * qx + dy * qy + dzq * qz;
    if (gd.means) {
        gd.means[3 * li + 0] += dmu0;
        gd.means[3 * li + 1] += dmu1;
        gd.means[3 * li + 2] += dmu2;
    }
    if (gd.scales) {
        gd.scales[3 * li + 0] += ds0;
        gd.scales[3 * li + 1] += ds1;
        gd.scales[3 * li + 2] += ds2;
    }
    if (gd.quats) {
        gd.quats[4 * li + 0] += (dw - qw * dd) * rn;
        gd.quats[4 * li + 1] += (dx - qx * dd) * rn;
        gd.quats[4 * li + 2] += (dy - qy * dd) * rn;
        gd.quats[4 * li + 3] += (dzq - qz * dd) * rn;
    }
    if (gd.opacities) gd.opacities[li] += dop;
    if (gd.sh) {
        float* o = gd.sh + li * (K * 3);
#pragma unroll
        for (int k = 0; k < K * 3; ++k) o[k] += dsh[k];
    }
}

template <int L>
__global__ __launch_bounds__(kBlock) void k_project_bwd(BwdArgs b) {
    const Block blk = b.f.blocks[blockIdx.x];
    float pose[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if ((int)threadIdx.x < (int)blk.count) project_bwd_gaussian<L>(b, blk, (int)threadIdx.x, pose);
    if (!b.d_poses) return;
    // the block's sums of the pose terms (one node per block), in a fixed order
    __shared__ float s_pose[kBlock / 64][6];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        const float t = wave_sum63(pose[j]);
        if (lane == 63) s_pose[w][j] = t;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        float t = 0.f;
#pragma unroll
        for (int q = 0; q < kBlock / 64; ++q) t += s_pose[q][threadIdx.x];
        b.pose_part[(size_t)blockIdx.x * 8 + threadIdx.x] = t;
    }
}

// Per node k with pose (R_k, t_k): sums A and B of its blocks, then
// omega = R_k A + t_k x (R_k B), rho = R_k B, added to d_poses[6 k ..] = (omega, rho): the
// derivative along the world-frame perturbation R' = exp([omega]x) R_k, t' = exp([omega]x) t_k + rho.
__global__ __launch_bounds__(256) void k_pose_grad(BwdArgs b) {
    const FwdArgs& a = b.f;
    const int k = blockIdx.x;
    const Node nd = a.nodes[k];
    const int nb = (int)((nd.n + kBlock - 1) / kBlock);
    float acc[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int q = threadIdx.x; q < nb; q += blockDim.x)
#pragma unroll
        for (int j = 0; j < 6; ++j) acc[j] += b.pose_part[(size_t)(nd.block_begin + q) * 8 + j];
    __shared__ float s_acc[4][6];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        const float t = wave_sum63(acc[j]);
        if (lane == 63) s_acc[w][j] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float A[3], B[3];
        for (int j = 0; j < 3; ++j) {
            A[j] = s_acc[0][j] + s_acc[1][j] + s_acc[2][j] + s_acc[3][j];
            B[j] = s_acc[0][3 + j] + s_acc[1][3 + j] + s_acc[2][3 + j] + s_acc[3][3 + j];
        }
        const gsr_pose P = a.poses[k];
        float RA[3], RB[3];
        for (int r = 0; r < 3; ++r) {
            RA[r] = P.R[r * 3 + 0] * A[0] + P.R[r * 3 + 1] * A[1] + P.R[r * 3 + 2] * A[2];
            RB[r] = P.R[r * 3 + 0] * B[0] + P.R[r * 3 + 1] * B[1] + P.R[r * 3 + 2] * B[2];
        }
        float* o = b.d_poses + 6 * (size_t)k;
        o[0] += RA[0] + (P.t[1] * RB[2] - P.t[2] * RB[1]);
        o[1] += RA[1] + (P.t[2] * RB[0] - P.t[0] * RB[2]);
        o[2] += RA[2] + (P.t[0] * RB[1] - P.t[1] * RB[0]);
        o[3] += RB[0];
        o[4] += RB[1];
        o[5] += RB[2];
    }
}

// Gradient descriptors of up to kDescPerLaunch nodes, passed by value (3.9 KB of kernel
// arguments), so that the host array may go away as soon as the call returns.
constexpr int kDescPerLaunch = 96;
struct DescBatch {
    gsr_gaussian_grads g[kDescPerLaunch];
    int first, count;
};

__global__ void k_set_grads(DescBatch d, gsr_gaussian_grads* out) {
    if ((int)threadIdx.x < d.count) out[d.first + threadIdx.x] = d.g[threadIdx.x];
}

hipError_t launch_set_grads(const gsr_gaussian_grads* host, int n, gsr_gaussian_grads* dev, hipStream_t s) {
    for (int first = 0; first < n; first += kDescPerLaunch) {
        DescBatch d;
        d.first = first;
        d.count = std::min(kDescPerLaunch, n - first);
        for (int i = 0; i < d.count; ++i) d.g[i] = host[first + i];
        hipLaunchKernelGGL(k_set_grads, dim3(1), dim3(kDescPerLaunch), 0, s, d, dev);
    }
    return hipGetLastError();
}

template <int TW, int TH>
static void launch_cbwd(const BwdArgs& b, hipStream_t s) {
    hipLaunchKernelGGL((k_composite_bwd<TW, TH>), dim3((unsigned)b.f.tiles), dim3(64), 0, s, b);
}

hipError_t launch_backward(const BwdArgs& b, size_t n_records, hipStream_t s) {
    const FwdArgs& a = b.f;
    const size_t n4 = n_records * 3;
    if (n4) hipLaunchKernelGGL(k_zero, dim3((unsigned)std::min<size_t>((n4 + 255) / 256, 65536)), dim3(256), 0, s,
                               reinterpret_cast<float4*>(b.g2d), n4);
    if (a.tw == 16 && a.th == 16) launch_cbwd<16, 16>(b, s);
    else if (a.tw == 16 && a.th == 8) launch_cbwd<16, 8>(b, s);
    else if (a.tw == 8 && a.th == 8) launch_cbwd<8, 8>(b, s);
    else launch_cbwd<32, 8>(b, s);
    if (a.n_blocks > 0) {
        switch (a.sh_degree) {
            case 0: hipLaunchKernelGGL(k_project_bwd<0>, dim3(a.n_blocks), dim3(kBlock), 0, s, b); break;
            case 1: hipLaunchKernelGGL(k_project_bwd<1>, dim3(a.n_blocks), dim3(kBlock), 0, s, b); break;
            case 2: hipLaunchKernelGGL(k_project_bwd<2>, dim3(a.n_blocks), dim3(kBlock), 0, s, b); break;
            default: hipLaunchKernelGGL(k_project_bwd<3>, dim3(a.n_blocks), dim3(kBlock), 0, s, b); break;
        }
        if (b.d_poses) hipLaunchKernelGGL(k_pose_grad, dim3(a.n_nodes), dim3(256), 0, s, b);
    }
    return hipGetLastError();
}

}  // namespace gsr
