// Forward path of the gfx950 Gaussian-splatting RGB-D renderer.
//
// Stages (all on one stream, no host synchronisation between them):
//   k_views        per (node, camera): camera<-node map composed in FP64, rounded once to FP32
//                  (scene composition: background plus rigidly posed nodes, paper Sec. III-B)
//   k_project      per Gaussian, all cameras of its env: EWA projection ("splatting"), tile
//                  rectangle and depth key (the FP32 key specification below), SH colour
//                  (paper Sec. III-A), projected record; per (super-block, camera) the list
//                  of visible Gaussians, appended in id order
//   k_seg, k_gather, k_radix_*   per image, its visible Gaussians ordered by depth bits, ties
//                  by id: the id-ordered lists gathered into the image's segment, then a
//                  stable LSD radix sort over the four bytes of the depth bits whose passes
//                  move (key, source position) and whose last pass gathers the ids and tile
//                  rectangles ("efficient sorting")
//   k_pair_*, k_chunk_starts   each image's depth-ordered Gaussians cut into chunks of about
//                  equal pair counts
//   k_tile_counts  per chunk: pairs per tile, from a difference grid in LDS
//   k_tile_seg, k_tile_ranges   a two-level scan over each image's chunks: each chunk's
//                  first slot in every tile bucket, the tiles' [start, end) ranges, tiles
//                  grouped by list length (persistent compositor's order)
//   k_emit         Gaussian ids written into their tiles' buckets in depth order, so every
//                  bucket is sorted by (depth bits, id) as it is written
//   k_composite    per tile, front-to-back alpha blending of colour and camera-space z
//                  (RGB and depth sensors, paper Sec. III-C), early exit when every pixel of a
//                  wavefront is saturated
//
// Compiled with -ffp-contract=off: every a*b+c below is two rounded operations unless an
// explicit fmaf() is written, and / and sqrtf are correctly rounded.  This makes the key
// specification in k_project reproducible bit for bit by any IEEE FP32 implementation of
// the same operation sequence.
#include <algorithm>

#include "gsr_internal.h"

namespace gsr {

// --------------------------------------------------------------------------------------------
// views
// --------------------------------------------------------------------------------------------
__global__ void k_views(FwdArgs a) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx == 0) {
        Status* st = a.status;
        st->flags = 0;
        st->nonfinite = 0;
        st->pairs = 0;
        st->max_tile = 0;
        for (int c = 0; c < 8; ++c) st->cls[c] = 0;
        for (int x = 0; x < 8; ++x) a.emit_next[x * kEmitQueueStride] = 0u;
        for (int q = 0; q < kParts; ++q) st->visible[q] = st->visible_any[q] = st->evals[q] = 0;
    }

    if (idx >= a.n_nodes * a.C) return;
    const int k = idx / a.C, c = idx % a.C;
    const Node nd = a.nodes[k];
    const gsr_camera cam = a.cams[nd.env * a.C + c];
    const gsr_pose P = a.poses[k];
    View v;
    double Wd[9], wd[3];
    // W = Rc Rk and w = Rc tk + tc, each sum left to right in FP64 (products of two FP32
    // values are exact in FP64), rounded once to FP32.
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) {
            double s = (double)cam.R[i * 3 + 0] * (double)P.R[0 * 3 + j];
            s = s + (double)cam.R[i * 3 + 1] * (double)P.R[1 * 3 + j];
            s = s + (double)cam.R[i * 3 + 2] * (double)P.R[2 * 3 + j];
            Wd[i * 3 + j] = s;
            v.W[i * 3 + j] = (float)s;
        }
        double s = (double)cam.R[i * 3 + 0] * (double)P.t[0];
        s = s + (double)cam.R[i * 3 + 1] * (double)P.t[1];
        s = s + (double)cam.R[i * 3 + 2] * (double)P.t[2];
        s = s + (double)cam.t[i];
        wd[i] = s;
        v.w[i] = (float)s;
    }
    // camera centre in node-local coordinates: -W^T w
    for (int j = 0; j < 3; ++j) v.cl[j] = (float)(-((Wd[0 * 3 + j] * wd[0] + Wd[1 * 3 + j] * wd[1]) + Wd[2 * 3 + j] * wd[2]));
    v.fx = cam.fx;
    v.fy = cam.fy;
    v.cx = cam.cx;
    v.cy = cam.cy;
    v.znear = cam.znear;
    v.limx = 1.3f * ((0.5f * (float)a.width) / cam.fx);
    v.limy = 1.3f * ((0.5f * (float)a.height) / cam.fy);
    v.pad[0] = v.pad[1] = 0.0f;
    a.views[idx] = v;
}

// --------------------------------------------------------------------------------------------
// SH colour: real spherical harmonics (Condon-Shortley phase, z polar axis, index l*l + m + l),
// colour = max(0, sum_k c_k Y_k(d) + 0.5), d the unit vector from the camera centre to the mean.
// Normalisation constants written from their closed forms.
// --------------------------------------------------------------------------------------------
template <int L>
__device__ inline void sh_basis(float x, float y, float z, float* Y) {
    Y[0] = 0.282094806432724f;                              // sqrt(1/(4pi))
    if (L >= 1) {
        Y[1] = -0.48860251903533936f * y;                   // sqrt(3/(4pi))
        Y[2] = 0.48860251903533936f * z;
        Y[3] = -0.48860251903533936f * x;
    }
    if (L >= 2) {
        const float xx = x * x, yy = y * y, zz = z * z;
        Y[4] = 1.0925484895706177f * (x * y);               // sqrt(15/(4pi))
        Y[5] = -1.0925484895706177f * (y * z);
        Y[6] = 0.31539157032966614f * (2.0f * zz - xx - yy); // sqrt(5/(16pi)) (3z^2 - 1)
        Y[7] = -1.0925484895706177f * (x * z);
        Y[8] = 0.5462742447853088f * (xx - yy);             // sqrt(15/(16pi))
        if (L >= 3) {
            Y[9] = -0.5900436043739319f * y * (3.0f * xx - yy);       // sqrt(35/(32pi))
            Y[10] = 2.890611410140991f * (x * y) * z;                 // sqrt(105/(4pi))
            Y[11] = -0.4570457935333252f * y * (4.0f * zz - xx - yy); // sqrt(21/(32pi)) (5z^2 - 1)
            Y[12] = 0.37317633628845215f * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);  // sqrt(7/(16pi))
            Y[13] = -0.4570457935333252f * x * (4.0f * zz - xx - yy);
            Y[14] = 1.4453057050704956f * z * (xx - yy);              // sqrt(105/(16pi))
            Y[15] = -0.5900436043739319f * x * (xx - 3.0f * yy);
        }
    }
}

// colour = max(0, sum_k c_k Y_k(d) + 1/2) for coefficients c[3 K] (k-major, rgb) and the
// direction d (not necessarily unit).  The normalisation uses the hardware reciprocal square
// root: the colour enters no key, only pixel values.
template <int L>
__device__ inline float3 sh_colour(const float* c, float dx, float dy, float dz) {
    constexpr int K = (L + 1) * (L + 1);
    const float inv = __builtin_amdgcn_rsqf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
    float Y[K];
    sh_basis<L>(dx * inv, dy * inv, dz * inv, Y);
    float r = 0.5f, g = 0.5f, b = 0.5f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        r = fmaf(Y[k], c[3 * k + 0], r);
        g = fmaf(Y[k], c[3 * k + 1], g);
        b = fmaf(Y[k], c[3 * k + 2], b);
    }
    return make_float3(fmaxf(r, 0.0f), fmaxf(g, 0.0f), fmaxf(b, 0.0f));
}

// one Gaussian's SH coefficients into registers (global loads; the compiler merges them)
template <int L>
__device__ inline void load_sh(const float* __restrict__ shp, float* c) {
    constexpr int K3 = 3 * (L + 1) * (L + 1);
    const auto* sh = global_ptr(shp);
#pragma unroll
    for (int i = 0; i < K3; ++i) c[i] = sh[i];
}

// --------------------------------------------------------------------------------------------
// projection with the FP32 key specification
//
// For a Gaussian with mean mu, scales s, quaternion q = (w, x, y, z), opacity o, seen through
// the view (W, w) of its node and camera:
//   cull (non-finite) unless every input and p is finite; cull unless o >= (float)(1/255)
//   p_r  = fmaf(W_r0, mu0, fmaf(W_r1, mu1, fmaf(W_r2, mu2, w_r)));  z = p_2; cull unless z > znear
//   iz = 1/z; xz = p0*iz; yz = p1*iz; u = fmaf(fx, xz, cx); v = fmaf(fy, yz, cy)
//   n2 = fmaf(q0,q0, fmaf(q1,q1, fmaf(q2,q2, q3*q3))); cull unless n2 > 0; rn = 1/sqrtf(n2)
//   unit quaternion, R(q) with the diagonal as fmaf(-2, yy + zz, 1) and off-diagonals 2*(xy - wz) ...
//   M_rc = fmaf(W_r0, R_0c, fmaf(W_r1, R_1c, W_r2*R_2c)) * s_c       (camera-frame axes, scaled)
//   Sigma_ab = fmaf(M_a0, M_b0, fmaf(M_a1, M_b1, M_a2*M_b2))
//   xc, yc = xz, yz clamped to +-lim (lim = 1.3 * ((0.5*width)/fx)); j00 = fx*iz, j11 = fy*iz,
//   j02 = -(j00*xc), j12 = -(j11*yc); T0k = fmaf(j00, S0k, j02*S2k); T1k = fmaf(j11, S1k, j12*S2k)
//   a = fmaf(T00, j00, T02*j02) + 0.3; b = fmaf(T01, j11, T02*j12); c = fmaf(T11, j11, T12*j12) + 0.3
//   det = fmaf(a, c, -(b*b)); cull unless det > 0
//   rx = fmaf(3.33, sqrtf(a), 1/64); ry = fmaf(3.33, sqrtf(c), 1/64)   (3.33 >= sqrt(2 ln 255))
//   tiles [floor((u-rx)/tw), floor((u+rx)/tw)] x [floor((v-ry)/th), floor((v+ry)/th)], each
//   bound clamped to [0, tiles] in float before conversion; cull if empty
//   depth key = the IEEE bit pattern of z
// The rectangle bounds the ellipse o * G >= 1/255 for any o <= 1, so tile lists hold every
// Gaussian that can reach a pixel of the tile.
// --------------------------------------------------------------------------------------------
// The read-only scene tables come in as separate restrict-qualified arguments: the compiler
// may then keep them in the scalar cache (s_load) instead of issuing vector loads, which would
// put a memory round trip in front of every chunk and every camera.
template <int L>
__global__ __launch_bounds__(kBlock) void k_project(FwdArgs a, const Super* __restrict__ supers,
                                                     const Env* __restrict__ envs, const Block* __restrict__ blocks,
                                                     const Node* __restrict__ nodes, const View* __restrict__ views) {
    // LDS: per (wavefront, camera) the running length of the camera's visible list (every
    // wavefront keeps its own copy of the same value), and the wavefronts' counts of the
    // current append (two sets, used alternately)
    extern __shared__ uint32_t s_run[];  // [kBlock / 64][C]
    __shared__ uint32_t s_wc[2][kBlock / 64];
    const Super sb = supers[blockIdx.x];
    const Env ev = envs[sb.env];
    const int C = a.C;
    const int i = threadIdx.x, lane = i & 63, wave = i >> 6;
    for (int k = i; k < (kBlock / 64) * C; k += kBlock) s_run[k] = 0u;
    __syncthreads();
    constexpr int K = (L + 1) * (L + 1);
    const float thr = (float)(1.0 / 255.0);
    const float itw = 1.0f / (float)a.tw, ith = 1.0f / (float)a.th;
    const unsigned long long below = (1ull << lane) - 1ull;
    int n_vis = 0, n_any = 0, nonfinite = 0, par = 0;
    // this thread's Gaussian of the next chunk, loaded one chunk ahead so that its latency
    // overlaps the current chunk's arithmetic
    float nm0 = 0.f, nm1 = 0.f, nm2 = 0.f, no = 0.f, ns0 = 0.f, ns1 = 0.f, ns2 = 0.f;
    float4 nq = make_float4(0.f, 0.f, 0.f, 0.f);
    auto fetch = [&](int ch) {
        const Block blk = blocks[ch];
        if (i < (int)blk.count) {
            const Node& nd = nodes[blk.node];
            const size_t li = blk.gid0 + (uint32_t)i - nd.gid_base;
            const auto* means = global_ptr(nd.means);
            const auto* scales = global_ptr(nd.scales);
            nm0 = means[3 * li + 0]; nm1 = means[3 * li + 1]; nm2 = means[3 * li + 2];
            no = global_ptr(nd.opac)[li];
            ns0 = scales[3 * li + 0]; ns1 = scales[3 * li + 1]; ns2 = scales[3 * li + 2];
            const auto* quats = global_ptr(nd.quats);
            nq = make_float4(quats[4 * li + 0], quats[4 * li + 1], quats[4 * li + 2], quats[4 * li + 3]);
        }
    };
    if (sb.chunk_begin < sb.chunk_end) fetch(sb.chunk_begin);
    for (int ch = sb.chunk_begin; ch < sb.chunk_end; ++ch) {
        const Block blk = blocks[ch];
        const float mu0 = nm0, mu1 = nm1, mu2 = nm2, o = no, s0 = ns0, s1 = ns1, s2 = ns2;
        const float q0 = nq.x, q1 = nq.y, q2 = nq.z, q3 = nq.w;
        if (ch + 1 < sb.chunk_end) fetch(ch + 1);
        // every thread stays in the loop: the appends below take block-wide barriers
        bool ok = i < (int)blk.count;
        const Node& nd = nodes[blk.node];
        const uint32_t gid = blk.gid0 + i;
        const size_t li = gid - nd.gid_base;
        const size_t lg = gid - ev.gid_base;
        if (ok && !(isfinite(mu0) && isfinite(mu1) && isfinite(mu2) && isfinite(o) && isfinite(s0) && isfinite(s1) &&
                    isfinite(s2) && isfinite(q0) && isfinite(q1) && isfinite(q2) && isfinite(q3))) {
            nonfinite += C;  // culled and counted once per camera
            ok = false;
        }
        if (!(o >= thr)) ok = false;
        // the rotation of the unit quaternion (camera independent)
        const float n2 = fmaf(q0, q0, fmaf(q1, q1, fmaf(q2, q2, q3 * q3)));
        float R00 = 0.f, R01 = 0.f, R02 = 0.f, R10 = 0.f, R11 = 0.f, R12 = 0.f, R20 = 0.f, R21 = 0.f, R22 = 0.f;
        if (ok && n2 > 0.0f) {
            const float rn = 1.0f / sqrtf(n2);
            const float qw = q0 * rn, qx = q1 * rn, qy = q2 * rn, qz = q3 * rn;
            const float xx = qx * qx, yy = qy * qy, zz = qz * qz;
            const float xy = qx * qy, xzq = qx * qz, yzq = qy * qz;
            const float wx = qw * qx, wy = qw * qy, wz = qw * qz;
            R00 = fmaf(-2.0f, yy + zz, 1.0f); R01 = 2.0f * (xy - wz); R02 = 2.0f * (xzq + wy);
            R10 = 2.0f * (xy + wz); R11 = fmaf(-2.0f, xx + zz, 1.0f); R12 = 2.0f * (yzq - wx);
            R20 = 2.0f * (xzq - wy); R21 = 2.0f * (yzq + wx); R22 = fmaf(-2.0f, xx + yy, 1.0f);
        }
        const float lo = __log2f(o);  // pixel values only
        float shc[3 * K];
        bool have_sh = false, vis_any = false;
        for (int c = 0; c < C; ++c) {
            bool vis = false;
            uint4 ent = make_uint4(0u, 0u, 0u, 0u);
            if (ok) do {
                const View& v = views[blk.node * C + c];
                const size_t rec = (size_t)C * ev.gid_base + (size_t)c * ev.n + lg;
                const float p0 = fmaf(v.W[0], mu0, fmaf(v.W[1], mu1, fmaf(v.W[2], mu2, v.w[0])));
                const float p1 = fmaf(v.W[3], mu0, fmaf(v.W[4], mu1, fmaf(v.W[5], mu2, v.w[1])));
                const float p2 = fmaf(v.W[6], mu0, fmaf(v.W[7], mu1, fmaf(v.W[8], mu2, v.w[2])));
                if (!(isfinite(p0) && isfinite(p1) && isfinite(p2))) { ++nonfinite; break; }
                const float z = p2;
                if (!(z > v.znear)) break;
                if (!(n2 > 0.0f)) break;
                const float iz = 1.0f / z;
                const float xz = p0 * iz, yz = p1 * iz;
                const float u = fmaf(v.fx, xz, v.cx), vv = fmaf(v.fy, yz, v.cy);
                float M[9];
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    M[r * 3 + 0] = fmaf(v.W[r * 3 + 0], R00, fmaf(v.W[r * 3 + 1], R10, v.W[r * 3 + 2] * R20)) * s0;
                    M[r * 3 + 1] = fmaf(v.W[r * 3 + 0], R01, fmaf(v.W[r * 3 + 1], R11, v.W[r * 3 + 2] * R21)) * s1;
                    M[r * 3 + 2] = fmaf(v.W[r * 3 + 0], R02, fmaf(v.W[r * 3 + 1], R12, v.W[r * 3 + 2] * R22)) * s2;
                }
                const float S00 = fmaf(M[0], M[0], fmaf(M[1], M[1], M[2] * M[2]));
                const float S01 = fmaf(M[0], M[3], fmaf(M[1], M[4], M[2] * M[5]));
                const float S02 = fmaf(M[0], M[6], fmaf(M[1], M[7], M[2] * M[8]));
                const float S11 = fmaf(M[3], M[3], fmaf(M[4], M[4], M[5] * M[5]));
                const float S12 = fmaf(M[3], M[6], fmaf(M[4], M[7], M[5] * M[8]));
                const float S22 = fmaf(M[6], M[6], fmaf(M[7], M[7], M[8] * M[8]));
                const float xc = fminf(fmaxf(xz, -v.limx), v.limx);
                const float yc = fminf(fmaxf(yz, -v.limy), v.limy);
                const float j00 = v.fx * iz, j11 = v.fy * iz;
                const float j02 = -(j00 * xc), j12 = -(j11 * yc);
                const float T00 = fmaf(j00, S00, j02 * S02);
                const float T01 = fmaf(j00, S01, j02 * S12);
                const float T02 = fmaf(j00, S02, j02 * S22);
                const float T11 = fmaf(j11, S11, j12 * S12);
                const float T12 = fmaf(j11, S12, j12 * S22);
                const float ca = fmaf(T00, j00, T02 * j02) + 0.3f;
                const float cb = fmaf(T01, j11, T02 * j12);
                const float cc = fmaf(T11, j11, T12 * j12) + 0.3f;
                const float det = fmaf(ca, cc, -(cb * cb));
                if (!(det > 0.0f)) break;
                const float rx = fmaf(3.33f, sqrtf(ca), 0.015625f);
                const float ry = fmaf(3.33f, sqrtf(cc), 0.015625f);
                const float tx0f = fminf(fmaxf(floorf((u - rx) * itw), 0.0f), (float)a.tiles_x);
                const float tx1f = fminf(fmaxf(floorf((u + rx) * itw) + 1.0f, 0.0f), (float)a.tiles_x);
                const float ty0f = fminf(fmaxf(floorf((vv - ry) * ith), 0.0f), (float)a.tiles_y);
                const float ty1f = fminf(fmaxf(floorf((vv + ry) * ith) + 1.0f, 0.0f), (float)a.tiles_y);
                const int tx0 = (int)tx0f, tx1 = (int)tx1f, ty0 = (int)ty0f, ty1 = (int)ty1f;
                if (tx0 >= tx1 || ty0 >= ty1) break;
                // visible: projected record (the conic and colour enter pixel values only, so
                // the hardware reciprocal suffices there)
                const float idet = __builtin_amdgcn_rcpf(det);
                if (!have_sh) {
                    load_sh<L>(nd.sh + li * (3 * K), shc);
                    have_sh = true;
                }
                const float3 col = sh_colour<L>(shc, mu0 - v.cl[0], mu1 - v.cl[1], mu2 - v.cl[2]);
                Record R;
                R.r0 = make_float4(u, vv, o, z);
                R.r1 = make_float4(cc * idet, -cb * idet, ca * idet, lo);
                R.r2 = make_float4(col.x, col.y, col.z, det);
                a.records[rec] = R;
                ent = make_uint4((uint32_t)tx0 | ((uint32_t)ty0 << 16), (uint32_t)tx1 | ((uint32_t)ty1 << 16),
                                 __float_as_uint(z), gid);
                vis = true;
            } while (false);
            // append to this super-block's list for camera c in id order: slot = list length
            // so far + visible threads before this one (wavefront ballots, block-wide prefix)
            const unsigned long long m = __ballot(vis);
            if (lane == 0) s_wc[par][wave] = (uint32_t)__popcll(m);
            __syncthreads();
            uint32_t before = s_run[wave * C + c], tot = 0u;
#pragma unroll
            for (int w = 0; w < kBlock / 64; ++w) {
                const uint32_t cw = s_wc[par][w];
                before += w < wave ? cw : 0u;
                tot += cw;
            }
            if (vis) {
                a.vis[((size_t)blockIdx.x * C + c) * a.sb_cap + before + (uint32_t)__popcll(m & below)] = ent;
                ++n_vis;
                vis_any = true;
            }
            // the wavefront's own copy; every lane has read it above
            if (lane == 0) s_run[wave * C + c] += tot;
            par ^= 1;
        }
        n_any += vis_any ? 1 : 0;
    }
    if (nonfinite) atomicAdd(&a.status->nonfinite, (uint32_t)nonfinite);
    for (int k = i; k < C; k += kBlock) a.sbvis[(size_t)blockIdx.x * C + k] = s_run[wave * C + k];  // own copy
    // block sums of visible records: one atomic per block into its counter slot
    unsigned long long nv = (unsigned long long)n_vis, na = (unsigned long long)n_any;
    for (int off = 32; off > 0; off >>= 1) {
        nv += __shfl_xor(nv, off, 64);
        na += __shfl_xor(na, off, 64);
    }
    __shared__ unsigned long long s_sum[2 * (kBlock / 64)];
    if (lane == 0) {
        s_sum[2 * wave] = nv;
        s_sum[2 * wave + 1] = na;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) {
            nv += s_sum[2 * w];
            na += s_sum[2 * w + 1];
        }
        if (nv) {
            atomicAdd(&a.status->visible[blockIdx.x % kParts], nv);
            atomicAdd(&a.status->visible_any[blockIdx.x % kParts], na);
        }
    }
}

// --------------------------------------------------------------------------------------------
// depth sort.  Image i keeps its visible (z bits, Gaussian id, tile rectangle) triples in a
// segment of the sort buffers: k_seg counts them (the lengths of the image's lists) and lays
// the segments out in image order, each starting at a multiple of kSortTile, so that every
// radix chunk (kSortTile positions) below the end lies inside one image's segment and holds at
// least one item.
// The (super-block, camera) lists, which hold an image's Gaussians in id order when taken in
// super-block order, are first copied into the segment in that order (k_gather).  The sort is
// then a stable LSD radix sort over the four bytes of the z bits (positive floats order as
// their bit patterns), so Gaussians of equal depth bits stay in id order: the result is the
// (z bits, id) order of the keys.  Each pass is a per-chunk
// digit histogram, a per-image scan of the histograms (chunks in order, digits in order) and
// a scatter that ranks each item among its chunk's items of the same digit, stages the chunk
// in LDS in digit order and writes every digit's run to consecutive slots.
// --------------------------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_seg(FwdArgs a) {
    // G threads per image (a power of two, at most one wavefront), each over a contiguous
    // range of the image's lists; 1024 / G images per pass
    int G = 64;
    while (G > 1 && G * a.images > 1024) G >>= 1;
    const int t = threadIdx.x, grp = t / G, r = t % G, lane = t & 63, wave = t >> 6;
    __shared__ uint32_t s_w[16];
    __shared__ uint32_t s_carry;
    if (t == 0) s_carry = 0u;
    __syncthreads();
    constexpr int B = 16;  // loads in flight
    for (int b0 = 0; b0 < a.images; b0 += 1024 / G) {
        const int img = b0 + grp;
        const bool valid = img < a.images;
        size_t l0 = 0;
        int k0 = 0, k1 = 0;
        if (valid) {
            const int e = img / a.C, c = img - e * a.C;
            const Env ev = a.envs[e];
            l0 = (size_t)ev.sb_begin * a.C + c;
            k0 = (int)((long long)ev.sb_count * r / G);
            k1 = (int)((long long)ev.sb_count * (r + 1) / G);
        }
        const uint32_t* p = a.sbvis + l0;
        uint32_t sum = 0u;
        for (int k = k0; k < k1; k += B) {
            uint32_t v[B];
#pragma unroll
            for (int q = 0; q < B; ++q) v[q] = k + q < k1 ? p[(size_t)(k + q) * a.C] : 0u;
#pragma unroll
            for (int q = 0; q < B; ++q) sum += v[q];
        }
        // the group's scan (the group lies inside one wavefront)
        uint32_t incl = sum;
        for (int off = 1; off < G; off <<= 1) {
            const uint32_t y = __shfl_up(incl, off, G);
            if (r >= off) incl += y;
        }
        const uint32_t n = __shfl(incl, G - 1, G);  // the image's visible Gaussians
        if (valid && r == 0) a.seg_n[img] = n;
        // segment starts: block scan of the rounded lengths (one per group)
        const uint32_t len = (valid && r == 0) ? (n + kSortTile - 1) / kSortTile * kSortTile : 0u;
        uint32_t bi = len;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(bi, off, 64);
            if (lane >= off) bi += y;
        }
        if (lane == 63) s_w[wave] = bi;
        __syncthreads();
        uint32_t before = s_carry;
        for (int w = 0; w < wave; ++w) before += s_w[w];
        const uint32_t seg0 = __shfl(before + bi - len, 0, G);  // from the group's first thread
        if (valid && r == 0) a.seg_start[img] = seg0;
        // each list's first position: the segment start plus the image's earlier lists
        uint32_t run = seg0 + incl - sum;
        for (int k = k0; k < k1; k += B) {
            uint32_t v[B];
#pragma unroll
            for (int q = 0; q < B; ++q) v[q] = k + q < k1 ? p[(size_t)(k + q) * a.C] : 0u;
#pragma unroll
            for (int q = 0; q < B; ++q) {
                if (k + q < k1) a.loff[l0 + (size_t)(k + q) * a.C] = run;
                run += v[q];
            }
        }
        __syncthreads();
        if (t == 1023) s_carry = before + bi;
        __syncthreads();
    }
    if (t == 0) a.seg_start[a.images] = s_carry;
}

// the (super-block, camera) lists copied into their image segments, in list order: the keys
// into key buffer 1 (the first pass's input), ids and rectangles into buffer 0, which the sort
// leaves in place (its last pass gathers them in sorted order into buffer 1)
__global__ __launch_bounds__(256) void k_gather(FwdArgs a) {
    uint32_t l0, l1, ls;
    xcd_items((uint32_t)(a.n_supers * a.C), l0, l1, ls);
    constexpr int U = 4;  // loads in flight per thread
    for (uint32_t l = l0; l < l1; l += ls) {
        const uint32_t n = a.sbvis[l], dst = a.loff[l];
        const uint4* lst = a.vis + (size_t)l * a.sb_cap;
        for (uint32_t k0 = threadIdx.x; k0 < n; k0 += 256 * U) {
            uint4 e[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t k = k0 + 256u * u;
                if (k < n) e[u] = lst[k];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t k = k0 + 256u * u;
                if (k < n) {
                    a.skey[1][dst + k] = e[u].z;
                    a.sgid[0][dst + k] = e[u].w;
                    a.srect[0][dst + k] = make_uint2(e[u].x, e[u].y);
                }
            }
        }
    }
}

// the image whose segment contains position pos (below the end): the last image whose segment
// starts at or before pos (empty images share their start with the next one)
__device__ inline int pos_image(const uint32_t* __restrict__ seg_start, int images, uint32_t pos) {
    int lo = 0, hi = images - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (seg_start[mid] <= pos) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// the lanes (among those with valid set) whose 8-bit digit equals this lane's
__device__ inline unsigned long long match_digit(uint32_t d, bool valid) {
    unsigned long long m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const unsigned long long bb = __ballot(bit);
        m &= bit ? bb : ~bb;
    }
    return m;
}

// Radix chunks: kSortTile positions of the sort buffers.  Pass p reads key and source buffer
// (p + 1) & 1 and writes buffer p & 1 (the gather fills key buffer 1; the first pass takes
// each item's position as its source); the last pass writes, instead, the ids and rectangles
// of the items' sources into buffer 1.
__device__ inline uint32_t radix_chunks(const FwdArgs& a) { return a.seg_start[a.images] / (uint32_t)kSortTile; }
// Items of radix chunk j; pos receives the chunk's first position.
__device__ inline uint32_t radix_chunk(const FwdArgs& a, uint32_t j, uint32_t& pos) {
    pos = j * (uint32_t)kSortTile;
    const int img = pos_image(a.seg_start, a.images, pos);
    const uint32_t end = a.seg_start[img] + a.seg_n[img];
    return end - pos < (uint32_t)kSortTile ? end - pos : (uint32_t)kSortTile;
}

__global__ __launch_bounds__(256) void k_radix_hist(FwdArgs a, int pass) {
    __shared__ uint32_t s_h[256];
    const int t = threadIdx.x, lane = t & 63;
    const int sh = 8 * pass;
    const uint32_t nch = radix_chunks(a);
    const uint32_t* kin = a.skey[(pass + 1) & 1];
    for (uint32_t j = blockIdx.x; j < nch; j += gridDim.x) {
        uint32_t pos;
        const uint32_t n = radix_chunk(a, j, pos);
        s_h[t] = 0u;
        __syncthreads();
        for (uint32_t k0 = 0; k0 < n; k0 += 256) {
            const uint32_t k = k0 + (uint32_t)t;
            const bool valid = k < n;
            const uint32_t d = valid ? (kin[pos + k] >> sh) & 255u : 0u;
            const unsigned long long m = match_digit(d, valid);
            // one LDS atomic per distinct digit of the wavefront (its highest lane)
            if (valid && (m >> lane) == 1ull) atomicAdd(&s_h[d], (uint32_t)__popcll(m));
        }
        __syncthreads();
        a.hist[(size_t)j * 256 + t] = s_h[t];
        __syncthreads();
    }
}

// One block per image: thread (g, d) takes digit d of the g-th quarter of the image's chunks.
// Each chunk's first slot per digit = segment start + items of smaller digits + items of this
// digit in earlier chunks.
__global__ __launch_bounds__(1024) void k_radix_scan(FwdArgs a) {
    __shared__ uint32_t s_tot[4][256];
    __shared__ uint32_t s_w[4];
    const int img = blockIdx.x, d = threadIdx.x & 255, g = threadIdx.x >> 8, lane = threadIdx.x & 63;
    const uint32_t base = a.seg_start[img];
    const int nch = (int)((a.seg_n[img] + kSortTile - 1) / kSortTile);
    const int per = (nch + 3) / 4;
    const int c0 = g * per, c1 = min(nch, c0 + per);
    uint32_t* h = a.hist + (size_t)(base / kSortTile) * 256 + d;
    constexpr int B = 16;  // loads in flight per thread
    uint32_t tot = 0u;
    for (int k0 = c0; k0 < c1; k0 += B) {
        uint32_t v[B];
#pragma unroll
        for (int k = 0; k < B; ++k) v[k] = k0 + k < c1 ? h[(size_t)(k0 + k) * 256] : 0u;
#pragma unroll
        for (int k = 0; k < B; ++k) tot += v[k];
    }
    s_tot[g][d] = tot;
    __syncthreads();
    uint32_t run = 0u;
    if (g == 0) {
        // digit totals, exclusive scan over digits (threads 0..255 = 4 wavefronts)
        const uint32_t dt = s_tot[0][d] + s_tot[1][d] + s_tot[2][d] + s_tot[3][d];
        uint32_t incl = dt;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(incl, off, 64);
            if (lane >= off) incl += y;
        }
        if (lane == 63) s_w[d >> 6] = incl;
        run = incl - dt;
    }
    __syncthreads();
    if (g == 0) {
        for (int w = 0; w < (d >> 6); ++w) run += s_w[w];
        // group starts within the digit
        uint32_t r = base + run;
        for (int q = 0; q < 4; ++q) {
            const uint32_t v = s_tot[q][d];
            s_tot[q][d] = r;
            r += v;
        }
    }
    __syncthreads();
    run = s_tot[g][d];
    for (int k0 = c0; k0 < c1; k0 += B) {
        uint32_t v[B];
#pragma unroll
        for (int k = 0; k < B; ++k) v[k] = k0 + k < c1 ? h[(size_t)(k0 + k) * 256] : 0u;
#pragma unroll
        for (int k = 0; k < B; ++k) {
            if (k0 + k < c1) h[(size_t)(k0 + k) * 256] = run;
            run += v[k];
        }
    }
}

// Wavefront w ranks chunk items [R 64 w, R 64 (w + 1)) in rounds of 64 consecutive items:
// rank = items of the same digit in earlier rounds (a per-wavefront LDS counter) + matching
// lanes below it.  Local position = items of smaller digits in the chunk + items of the same
// digit in earlier wavefronts + rank, so the chunk is staged in LDS in stable digit order, and
// local position p of digit d goes to slot p + (chunk slot of d - local start of d).  All of
// the chunk's loads are issued before the ranking.
__global__ __launch_bounds__(256) void k_radix_scatter(FwdArgs a, int pass) {
    constexpr int R = kSortTile / 256;  // rounds per wavefront
    __shared__ uint32_t s_wc[4][256];
    __shared__ uint32_t s_delta[256];
    __shared__ uint32_t s_w[4];
    __shared__ unsigned long long s_buf[kSortTile];
    __shared__ uint8_t s_dig[kSortTile];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int sh = 8 * pass;
    const int ib = (pass + 1) & 1, ob = pass & 1;
    const unsigned long long below = (1ull << lane) - 1ull;
    uint32_t j0, j1, js;
    xcd_items(radix_chunks(a), j0, j1, js);
    for (uint32_t j = j0; j < j1; j += js) {
        uint32_t pos;
        const uint32_t n = radix_chunk(a, j, pos);
        for (int k = lane; k < 256; k += 64) s_wc[wave][k] = 0u;  // read back by this wavefront only
        const uint32_t w0 = (uint32_t)(wave * 64 * R);
        // rounds of this wavefront that hold items (uniform across the wavefront)
        const int nr = n > w0 ? (int)min((n - w0 + 63u) / 64u, (uint32_t)R) : 0;
        const uint32_t* kin = a.skey[ib] + pos;
        uint32_t key[R], rk[R], src[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t k = w0 + (uint32_t)(r * 64 + lane);
            const bool in = r < nr && k < n;
            key[r] = in ? kin[k] : 0u;
            // the first pass reads the gathered order, so an item's source is its position
            src[r] = in ? (pass == 0 ? pos + k : a.ssrc[ib][pos + k]) : 0u;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (r >= nr) break;
            const uint32_t k = w0 + (uint32_t)(r * 64 + lane);
            const bool valid = k < n;
            const uint32_t d = (key[r] >> sh) & 255u;
            const unsigned long long m = match_digit(d, valid);
            const uint32_t before = valid ? s_wc[wave][d] : 0u;
            rk[r] = before + (uint32_t)__popcll(m & below);
            if (valid && (m >> lane) == 1ull) s_wc[wave][d] = before + (uint32_t)__popcll(m);
        }
        __syncthreads();
        {
            // thread t = digit t: local start (scan over digits), per-wavefront bases
            const uint32_t c0 = s_wc[0][t], c1 = s_wc[1][t], c2 = s_wc[2][t], c3 = s_wc[3][t];
            const uint32_t cnt = c0 + c1 + c2 + c3;
            uint32_t incl = cnt;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t y = __shfl_up(incl, off, 64);
                if (lane >= off) incl += y;
            }
            if (lane == 63) s_w[wave] = incl;
            __syncthreads();
            uint32_t ls = incl - cnt;
            for (int w = 0; w < wave; ++w) ls += s_w[w];
            s_wc[0][t] = ls;
            s_wc[1][t] = ls + c0;
            s_wc[2][t] = ls + c0 + c1;
            s_wc[3][t] = ls + c0 + c1 + c2;
            s_delta[t] = a.hist[(size_t)j * 256 + t] - ls;  // modulo 2^32
        }
        __syncthreads();
        // local positions replace the ranks; the chunk staged in LDS in digit order
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t k = w0 + (uint32_t)(r * 64 + lane);
            if (r < nr && k < n) {
                const uint32_t d = (key[r] >> sh) & 255u;
                rk[r] += s_wc[wave][d];
                s_buf[rk[r]] = ((unsigned long long)src[r] << 32) | (unsigned long long)key[r];
                s_dig[rk[r]] = (uint8_t)d;
            }
        }
        __syncthreads();
        // each digit's run to consecutive slots: keys and sources, or, in the last pass (whose
        // keys nothing reads), the items' ids and rectangles gathered from their sources (an
        // image's segment, a few hundred KB, stays in its XCD's L2)
        if (pass < 3) {
            for (uint32_t lp = t; lp < n; lp += 256) {
                const unsigned long long u = s_buf[lp];
                const uint32_t dst = lp + s_delta[s_dig[lp]];
                a.skey[ob][dst] = (uint32_t)u;
                a.ssrc[ob][dst] = (uint32_t)(u >> 32);
            }
        } else {
            for (uint32_t lp = t; lp < n; lp += 256) {
                const uint32_t sp = (uint32_t)(s_buf[lp] >> 32);
                const uint32_t dst = lp + s_delta[s_dig[lp]];
                a.sgid[1][dst] = a.sgid[0][sp];
                a.srect[1][dst] = a.srect[0][sp];
            }
        }
        __syncthreads();
    }
}

// --------------------------------------------------------------------------------------------
// emission chunks.  Each image's depth-ordered Gaussians are cut into chunks of about
// chunk_pairs pairs: with e_i the pairs of the image's Gaussians before Gaussian i, chunk q
// holds the Gaussians with floor(e_i / chunk_pairs) = q (empty when one Gaussian spans several
// multiples).  Per block of kPairBlock positions: its pairs (k_pair_blocks); per image: the
// blocks' prefix and the chunk count (k_pair_scan); per Gaussian: the chunks it starts
// (k_chunk_starts).
// --------------------------------------------------------------------------------------------
__device__ inline uint32_t rect_area(uint2 r) {
    return ((r.y & 0xffffu) - (r.x & 0xffffu)) * ((r.y >> 16) - (r.x >> 16));
}

// positions [pos, pos + n) of pair block b (n = 0 in the padding after an image's items)
__device__ inline uint32_t pair_block(const FwdArgs& a, uint32_t b, uint32_t& pos, int& img) {
    pos = b * (uint32_t)kPairBlock;
    img = pos_image(a.seg_start, a.images, pos);
    const uint32_t end = a.seg_start[img] + a.seg_n[img];
    return pos < end ? (end - pos < (uint32_t)kPairBlock ? end - pos : (uint32_t)kPairBlock) : 0u;
}

__global__ __launch_bounds__(256) void k_pair_blocks(FwdArgs a) {
    __shared__ uint32_t s_w[4];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const uint32_t nb = a.seg_start[a.images] / (uint32_t)kPairBlock;
    for (uint32_t b = blockIdx.x; b < nb; b += gridDim.x) {
        uint32_t pos;
        int img;
        const uint32_t n = pair_block(a, b, pos, img);
        uint32_t sum = 0u;
        for (uint32_t k = t; k < n; k += 256) sum += rect_area(a.srect[1][pos + k]);
        for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
        if (lane == 0) s_w[wave] = sum;
        __syncthreads();
        if (t == 0) a.blk_pairs[b] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
        __syncthreads();
    }
}

// One block: per image (one thread each) the exclusive prefix of its blocks' pairs and its
// chunk count; chunk, pair and segment bases by scans over images.  Total pairs and overflow
// into the status word; on overflow no image gets chunks (nothing is emitted; the host grows
// the capacity).
__global__ __launch_bounds__(1024) void k_pair_scan(FwdArgs a) {
    __shared__ uint32_t s_w[16], s_ws[16];
    __shared__ unsigned long long s_wp[16];
    __shared__ uint32_t s_carry, s_scarry;
    __shared__ unsigned long long s_pairs;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    if (t == 0) {
        s_carry = s_scarry = 0u;
        s_pairs = 0ull;
    }
    __syncthreads();
    const uint32_t PC = (uint32_t)a.chunk_pairs;
    for (int b0 = 0; b0 < a.images; b0 += 1024) {
        const int img = b0 + t;
        uint32_t nchk = 0u, run = 0u;
        if (img < a.images) {
            const uint32_t s = a.seg_start[img] / kPairBlock;
            const int nb = (int)((a.seg_n[img] + kPairBlock - 1) / kPairBlock);
            constexpr int B = 16;
            for (int k0 = 0; k0 < nb; k0 += B) {
                uint32_t v[B];
#pragma unroll
                for (int k = 0; k < B; ++k) v[k] = k0 + k < nb ? a.blk_pairs[s + k0 + k] : 0u;
#pragma unroll
                for (int k = 0; k < B; ++k) {
                    if (k0 + k < nb) a.blk_pairs[s + k0 + k] = run;
                    run += v[k];
                }
            }
            nchk = (run + PC - 1) / PC;
        }
        // chunk, pair and segment bases: exclusive scans over images
        const uint32_t nseg = (nchk + kSegChunks - 1) / kSegChunks;
        uint32_t incl = nchk, incls = nseg;
        unsigned long long inclp = run;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(incl, off, 64), ys = __shfl_up(incls, off, 64);
            const unsigned long long yp = __shfl_up(inclp, off, 64);
            if (lane >= off) {
                incl += y;
                incls += ys;
                inclp += yp;
            }
        }
        if (lane == 63) {
            s_w[wave] = incl;
            s_ws[wave] = incls;
            s_wp[wave] = inclp;
        }
        __syncthreads();
        uint32_t before = s_carry, befores = s_scarry;
        unsigned long long beforep = s_pairs;
        for (int w = 0; w < wave; ++w) {
            before += s_w[w];
            befores += s_ws[w];
            beforep += s_wp[w];
        }
        if (img < a.images) {
            a.chunk_base[img] = before + incl - nchk;
            a.seg_base[img] = befores + incls - nseg;
            a.pair_base[img] = (uint32_t)(beforep + inclp - run);  // < pair_cap unless overflowed
        }
        __syncthreads();
        if (t == 1023) {
            s_carry = before + incl;
            s_scarry = befores + incls;
            s_pairs = beforep + inclp;
        }
        __syncthreads();
    }
    // at most chunks / kSegChunks + images segments: within the workspace when the chunks are
    const bool over = s_pairs > (unsigned long long)a.pair_cap || s_carry > (uint32_t)a.chunk_cap;
    if (over)
        for (int i = t; i < a.images; i += 1024) a.chunk_base[i] = a.pair_base[i] = a.seg_base[i] = 0u;
    if (t == 0) {
        a.chunk_base[a.images] = over ? 0u : s_carry;
        a.seg_base[a.images] = over ? 0u : s_scarry;
        a.status->pairs = s_pairs;
        if (over) atomicOr(&a.status->flags, (uint32_t)GSR_STATUS_OVERFLOW);
    }
}

// Per pair block: each Gaussian's pair offset e within its image (block prefix + in-block
// scan); Gaussian i starts the chunks q with e_(i-1) < q chunk_pairs <= e_i (the image's first
// Gaussian starts chunk 0); chunks past the image's last Gaussian start at the image's end.
__global__ __launch_bounds__(256) void k_chunk_starts(FwdArgs a) {
    constexpr int E = kPairBlock / 256;  // Gaussians per thread (blocked)
    __shared__ uint32_t s_w[4];
    __shared__ uint32_t s_last[256];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const uint32_t PC = (uint32_t)a.chunk_pairs;
    const uint32_t nb = a.seg_start[a.images] / (uint32_t)kPairBlock;
    for (uint32_t b = blockIdx.x; b < nb; b += gridDim.x) {
        uint32_t pos;
        int img;
        const uint32_t n = pair_block(a, b, pos, img);
        const uint32_t cb = a.chunk_base[img], nci = a.chunk_base[img + 1] - cb;
        if (n == 0u || a.chunk_base[a.images] == 0u) continue;  // uniform
        uint32_t ar[E];
        uint32_t sum = 0u;
#pragma unroll
        for (int q = 0; q < E; ++q) {
            const uint32_t k = (uint32_t)t * E + q;
            ar[q] = k < n ? rect_area(a.srect[1][pos + k]) : 0u;
            sum += ar[q];
        }
        uint32_t incl = sum;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(incl, off, 64);
            if (lane >= off) incl += y;
        }
        if (lane == 63) s_w[wave] = incl;
        s_last[t] = ar[E - 1];
        __syncthreads();
        uint32_t e = a.blk_pairs[b] + incl - sum;
        for (int w = 0; w < wave; ++w) e += s_w[w];
        uint32_t prev = t > 0 ? s_last[t - 1] : 0u;  // pairs of the Gaussian before
        const uint32_t seg0 = a.seg_start[img], end = seg0 + a.seg_n[img];
        if (t == 0 && pos > seg0) prev = rect_area(a.srect[1][pos - 1]);
#pragma unroll
        for (int q = 0; q < E; ++q) {
            const uint32_t k = (uint32_t)t * E + q;
            if (k < n) {
                const uint32_t p = pos + k;
                const uint32_t qlo = p == seg0 ? 0u : (e - prev) / PC + 1u;
                const uint32_t qhi = e / PC;
                for (uint32_t c = qlo; c <= qhi && c < nci; ++c) {
                    a.cstart[cb + c] = p;
                    a.cimg[cb + c] = (uint32_t)img;
                }
                if (p + 1 == end)
                    for (uint32_t c = qhi + 1; c < nci; ++c) {
                        a.cstart[cb + c] = end;
                        a.cimg[cb + c] = (uint32_t)img;
                    }
            }
            prev = ar[q];
            e += ar[q];
        }
        __syncthreads();
    }
}

// Gaussians [s, e) of emission chunk q and its image
__device__ inline uint32_t emit_chunk(const FwdArgs& a, uint32_t q, uint32_t& s, int& img) {
    img = (int)a.cimg[q];
    s = a.cstart[q];
    const uint32_t e = q + 1 < a.chunk_base[img + 1] ? a.cstart[q + 1] : a.seg_start[img] + a.seg_n[img];
    return e - s;
}

constexpr int kCountThreads = 64;  // one wavefront per chunk: many chunks in flight per CU

// --------------------------------------------------------------------------------------------
// per emission chunk: pairs per tile of the image.  A rectangle adds +1/-1 at the four corners
// of a (tiles_y + 1) x (tiles_x + 1) difference grid in LDS; the 2D prefix gives the counts.
// --------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kCountThreads) void k_tile_counts(FwdArgs a) {
    extern __shared__ int s_grid[];
    const int gx = a.tiles_x + 1, gy = a.tiles_y + 1, gsz = gx * gy;
    const uint32_t nq = a.chunk_base[a.images];
    for (uint32_t q = blockIdx.x; q < nq; q += gridDim.x) {
        uint32_t s;
        int img;
        const uint32_t n = emit_chunk(a, q, s, img);
        for (int k = threadIdx.x; k < gsz; k += kCountThreads) s_grid[k] = 0;
        __syncthreads();
        const uint2* rects = a.srect[1] + s;
        for (uint32_t k = threadIdx.x; k < n; k += kCountThreads) {
            const uint2 r = rects[k];
            const uint32_t x0 = r.x & 0xffffu, y0 = r.x >> 16, x1 = r.y & 0xffffu, y1 = r.y >> 16;
            atomicAdd(&s_grid[y0 * gx + x0], 1);
            atomicAdd(&s_grid[y0 * gx + x1], -1);
            atomicAdd(&s_grid[y1 * gx + x0], -1);
            atomicAdd(&s_grid[y1 * gx + x1], 1);
        }
        __syncthreads();
        for (int r = threadIdx.x; r < gy; r += kCountThreads) {
            int* row = s_grid + r * gx;
            int acc = 0;
            for (int x = 0; x < gx; ++x) { acc += row[x]; row[x] = acc; }
        }
        __syncthreads();
        for (int col = threadIdx.x; col < gx; col += kCountThreads) {
            int acc = 0;
            for (int y = 0; y < gy; ++y) { acc += s_grid[y * gx + col]; s_grid[y * gx + col] = acc; }
        }
        __syncthreads();
        uint32_t* out = a.ecnt + (size_t)q * a.tpi;
        for (int j = threadIdx.x; j < a.tpi; j += kCountThreads) {
            const int ty = j / a.tiles_x, tx = j - ty * a.tiles_x;
            out[j] = (uint32_t)s_grid[ty * gx + tx];
        }
        __syncthreads();
    }
}

// --------------------------------------------------------------------------------------------
// tile ranges: a two-level scan, per tile, over its image's emission chunks in depth order.
// Segments of kSegChunks consecutive chunks of one image, all in parallel (k_tile_seg): each
// chunk's count is replaced by the tile's pairs of the earlier chunks of its segment, and the
// segment's count is kept.  Per image, one thread per tile (1024 at a time, k_tile_ranges):
// the tile's total over the image's segments; the totals, scanned over the image's tiles from
// the image's pair base, give the tiles' starts (the range table); each segment's count is
// replaced by its first slot in the tile's bucket.  A chunk's first slot in a bucket is its
// segment's slot plus its offset within the segment.  Tiles are also grouped by list length
// (at most 512, 1024, ..., 8192 pairs, longer, at most one pair): the persistent compositor
// takes them longest class first.
// --------------------------------------------------------------------------------------------
// the image holding global segment sg < seg_base[images] (the last image whose first segment
// is not after sg; images without segments share their successor's base)
__device__ inline int seg_image(const uint32_t* __restrict__ seg_base, int images, uint32_t sg) {
    int lo = 0, hi = images - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (seg_base[mid] <= sg) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

constexpr int kSegThreads = 256;

__global__ __launch_bounds__(kSegThreads) void k_tile_seg(FwdArgs a) {
    const uint32_t groups = (uint32_t)((a.tpi + kSegThreads - 1) / kSegThreads);
    const uint32_t items = a.seg_base[a.images] * groups;
    for (uint32_t w = blockIdx.x; w < items; w += gridDim.x) {
        const uint32_t sg = w / groups;
        const int t = (int)(w - sg * groups) * kSegThreads + (int)threadIdx.x;
        const int img = seg_image(a.seg_base, a.images, sg);
        const uint32_t q = a.chunk_base[img] + (sg - a.seg_base[img]) * (uint32_t)kSegChunks;
        const uint32_t left = a.chunk_base[img + 1] - q;
        const uint32_t m = left < (uint32_t)kSegChunks ? left : (uint32_t)kSegChunks;
        if (t < a.tpi) {
            uint32_t* p = a.ecnt + (size_t)q * a.tpi + t;
            uint32_t v[kSegChunks];
#pragma unroll
            for (int k = 0; k < kSegChunks; ++k) v[k] = (uint32_t)k < m ? p[(size_t)k * a.tpi] : 0u;
            uint32_t run = 0u;
#pragma unroll
            for (int k = 0; k < kSegChunks; ++k) {
                if ((uint32_t)k < m) p[(size_t)k * a.tpi] = run;
                run += v[k];
            }
            a.segoff[(size_t)sg * a.tpi + t] = run;
        }
    }
}

// append a wavefront's flagged lanes to a device list with one atomic; returns each flagged
// lane's slot
__device__ inline uint32_t wave_append(uint32_t* counter, bool pred) {
    const unsigned long long m = __ballot(pred);
    if (m == 0ull) return 0u;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((long long)m) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(counter, (uint32_t)__popcll(m));
    base = __shfl(base, leader, 64);
    return base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
}

__global__ __launch_bounds__(1024) void k_tile_ranges(FwdArgs a) {
    __shared__ uint32_t s_w[16];
    __shared__ uint32_t s_carry;
    const int img = blockIdx.x, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t s0 = a.seg_base[img];
    const int ns = (int)(a.seg_base[img + 1] - s0);
    if (threadIdx.x == 0) s_carry = a.pair_base[img];
    __syncthreads();
    constexpr int B = 16;  // loads in flight
    const size_t stride = (size_t)a.tpi;
    uint32_t mx = 0u;
    for (int t0 = 0; t0 < a.tpi; t0 += 1024) {
        const int t = t0 + (int)threadIdx.x;
        uint32_t* p = a.segoff + (size_t)s0 * a.tpi + t;
        uint32_t run = 0u;
        if (t < a.tpi)
            for (int k0 = 0; k0 < ns; k0 += B) {
                const int m = ns - k0 < B ? ns - k0 : B;
#pragma unroll
                for (int k = 0; k < B; ++k) run += k < m ? p[(size_t)(k0 + k) * stride] : 0u;
            }
        mx = run > mx ? run : mx;
        uint32_t incl = run;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(incl, off, 64);
            if (lane >= off) incl += y;
        }
        if (lane == 63) s_w[wave] = incl;
        __syncthreads();
        uint32_t st = s_carry;
        for (int w = 0; w < wave; ++w) st += s_w[w];
        st += incl - run;
        const long long gt = (long long)img * a.tpi + t;
        int cls = -1;
        if (t < a.tpi) {
            a.starts[gt] = st;
            uint32_t slot = st;
            for (int k0 = 0; k0 < ns; k0 += B) {
                const int m = ns - k0 < B ? ns - k0 : B;
                uint32_t v[B];
#pragma unroll
                for (int k = 0; k < B; ++k) v[k] = k < m ? p[(size_t)(k0 + k) * stride] : 0u;
#pragma unroll
                for (int k = 0; k < B; ++k) {
                    if (k < m) p[(size_t)(k0 + k) * stride] = slot;
                    slot += v[k];
                }
            }
            const uint32_t n = run;
            if ((unsigned long long)st + n > (unsigned long long)a.pair_cap || n <= 1) cls = kLenNone;
            else if (n <= 512) cls = 0;
            else if (n <= 1024) cls = 1;
            else if (n <= 2048) cls = 2;
            else if (n <= 4096) cls = 3;
            else if (n <= 8192) cls = 4;
            else cls = kLenLong;
        }
#pragma unroll
        for (int c = 0; c < kNumClasses; ++c) {
            const uint32_t pos = wave_append(&a.status->cls[c], cls == c);
            if (cls == c) a.cls_list[(size_t)c * a.tiles + pos] = (uint32_t)gt;
        }
        __syncthreads();
        if (threadIdx.x == 1023) s_carry = st + run;
        __syncthreads();
    }
    if (img == a.images - 1 && threadIdx.x == 0) a.starts[a.tiles] = s_carry;  // total pairs
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t o = __shfl_xor(mx, off, 64);
        mx = o > mx ? o : mx;
    }
    if (lane == 0 && mx) atomicMax(&a.status->max_tile, mx);
}

// --------------------------------------------------------------------------------------------
// pair emission.  One block per emission chunk walks the chunk's depth-ordered Gaussians in
// rounds of 64 and writes their ids into the tile buckets (one 4-byte id per (tile, Gaussian)
// pair), so each bucket receives its entries in (z bits, id) order: chunks in order (first
// slots from the tile offsets), rounds in order (a running slot per tile in LDS) and, within a
// round, by the Gaussian's rank in the round: the set bits below it in the tile's 64-bit round
// mask.
// A round's pairs are numbered by a prefix over the rectangle areas and split into equal runs
// of consecutive pairs, one per thread, walked twice: set the mask bits; write the pairs.
// Then each tile's slot advances by its count in the round and its mask is cleared (a third
// walk, at the tile's highest Gaussian of the round, or a pass over the tile table when the
// round has at least half as many pairs as the image has tiles).  Chunks hold about the same
// number of pairs, so the blocks' work is balanced even where the nearest (largest) splats of
// an image crowd into its first chunk.  The W wavefronts of a
// block share the chunk's tile table (12 bytes per tile), so large tile grids do not cap the
// wavefronts per CU, and split each round's pairs W ways.
// --------------------------------------------------------------------------------------------
template <int W>
__global__ __launch_bounds__(64 * W) void k_emit(FwdArgs a) {
    constexpr int NT = 64 * W;
    extern __shared__ unsigned long long s_mask[];  // [tpi] round masks, then [tpi] u32 slots
    __shared__ uint32_t s_off[65], s_x0[64], s_y0[64], s_w[64], s_id[64], s_q;
    const int tid = threadIdx.x, lane = tid & 63;
    uint32_t* s_slot = reinterpret_cast<uint32_t*>(s_mask + a.tpi);
    const unsigned long long cap = (unsigned long long)a.pair_cap;
    const int tx_n = a.tiles_x;
    for (int t = tid; t < a.tpi; t += NT) s_mask[t] = 0ull;  // masks are left clear by each round
    // the blocks of XCD x take the chunks of its eighth of the list in order from a counter, so
    // the chunks in flight on an XCD stay consecutive and the bucket lines they share are
    // completed in its L2 (block b runs on XCD b % 8; any placement is still correct)
    const uint32_t x = blockIdx.x & 7u, n_all = a.chunk_base[a.images];
    const uint32_t lo = (uint32_t)(((unsigned long long)n_all * x) >> 3);
    const uint32_t hi = (uint32_t)(((unsigned long long)n_all * (x + 1u)) >> 3);
    if (tid == 0) s_q = lo + atomicAdd(&a.emit_next[x * kEmitQueueStride], 1u);
    __syncthreads();
    for (uint32_t q = s_q; q < hi;) {
        __syncthreads();  // every thread has read s_q
        uint32_t pos;
        int img;
        const uint32_t n = emit_chunk(a, q, pos, img);
        if (n != 0u) {
            const uint32_t* so = a.ecnt + (size_t)q * a.tpi;
            const uint32_t* st =
                a.segoff + (size_t)(a.seg_base[img] + (q - a.chunk_base[img]) / (uint32_t)kSegChunks) * a.tpi;
            for (int t = tid; t < a.tpi; t += NT) s_slot[t] = st[t] + so[t];
            const uint32_t* gids = a.sgid[1] + pos;
            const uint2* rects = a.srect[1] + pos;
            // the next round's Gaussian, loaded one round ahead (by the first wavefront)
            uint2 nr = make_uint2(0u, 0u);
            uint32_t ni = 0u;
            if (tid < 64 && (uint32_t)lane < n) {
                nr = rects[lane];
                ni = gids[lane];
            }
            for (uint32_t r0 = 0; r0 < n; r0 += 64) {
                if (tid < 64) {
                    const uint32_t k = r0 + (uint32_t)lane;
                    uint32_t area = 0u;
                    if (k < n) {
                        const uint32_t x0 = nr.x & 0xffffu, y0 = nr.x >> 16, x1 = nr.y & 0xffffu, y1 = nr.y >> 16;
                        s_x0[lane] = x0;
                        s_y0[lane] = y0;
                        s_w[lane] = x1 - x0;
                        s_id[lane] = ni;
                        area = (x1 - x0) * (y1 - y0);
                    }
                    if (k + 64u < n) {
                        nr = rects[k + 64u];
                        ni = gids[k + 64u];
                    }
                    const uint32_t incl = wave_incl_scan(area);
                    s_off[lane + 1] = incl;
                    if (lane == 0) s_off[0] = 0u;
                }
                __syncthreads();
                const uint32_t total = s_off[64];
                const uint32_t per = (total + (uint32_t)NT - 1u) / (uint32_t)NT;
                const uint32_t k0 = (uint32_t)tid * per, k1 = k0 + per < total ? k0 + per : total;
                // where this lane's pairs start: the Gaussian of pair k0 (first o with
                // s_off[o + 1] > k0) and the tile of that pair
                int o0 = 0;
                uint32_t w0 = 1u, x00 = 0u, tx0 = 0u, ty0 = 0u, left0 = 0u;
                if (k0 < k1) {
                    int hi = 63;
                    while (o0 < hi) {
                        const int mid = (o0 + hi) >> 1;
                        if (s_off[mid + 1] > k0) hi = mid;
                        else o0 = mid + 1;
                    }
                    w0 = s_w[o0];
                    x00 = s_x0[o0];
                    const uint32_t j = k0 - s_off[o0];
                    const uint32_t jy = j / w0;
                    tx0 = x00 + (j - jy * w0);
                    ty0 = s_y0[o0] + jy;
                    left0 = s_off[o0 + 1] - k0;
                }
                // calls f(o, tile) for this lane's pairs [k0, k1), in order (every listed rectangle
                // is non-empty; k < total guarantees a next Gaussian with pairs)
                auto walk = [&](auto&& f) {
                    int o = o0;
                    uint32_t w = w0, x0 = x00, tx = tx0, ty = ty0, left = left0;
                    for (uint32_t kk = k0; kk < k1; ++kk) {
                        while (left == 0u) {
                            ++o;
                            w = s_w[o];
                            x0 = s_x0[o];
                            tx = x0;
                            ty = s_y0[o];
                            left = s_off[o + 1] - s_off[o];
                        }
                        f(o, ty * (uint32_t)tx_n + tx);
                        --left;
                        if (++tx == x0 + w) {
                            tx = x0;
                            ++ty;
                        }
                    }
                };
                walk([&](int o, uint32_t t) { atomicOr(&s_mask[t], 1ull << o); });
                __syncthreads();
                walk([&](int o, uint32_t t) {
                    const unsigned long long m = s_mask[t];
                    const uint32_t p = s_slot[t] + (uint32_t)__popcll(m & ((1ull << o) - 1ull));
                    if ((unsigned long long)p < cap) a.pairs[p] = s_id[o];
                });
                __syncthreads();
                // advance each touched tile's slot by its round count and clear its mask: over
                // the round's pairs (at the tile's highest Gaussian) when they are few, else over
                // the tile table (consecutive, conflict-free LDS accesses)
                if (2u * total < (uint32_t)a.tpi) {
                    walk([&](int o, uint32_t t) {
                        const unsigned long long m = s_mask[t];
                        if ((m >> o) == 1ull) {
                            s_slot[t] += (uint32_t)__popcll(m);
                            s_mask[t] = 0ull;
                        }
                    });
                } else {
                    for (int t = tid; t < a.tpi; t += NT) {
                        const unsigned long long m = s_mask[t];
                        if (m) {
                            s_slot[t] += (uint32_t)__popcll(m);
                            s_mask[t] = 0ull;
                        }
                    }
                }
                __syncthreads();
            }
        }
        // the next chunk, taken when this one is done (taking it ahead doubles the chunks in
        // flight and the open bucket lines)
        if (tid == 0) s_q = lo + atomicAdd(&a.emit_next[x * kEmitQueueStride], 1u);
        __syncthreads();
        q = s_q;
    }
}

// --------------------------------------------------------------------------------------------
// front-to-back compositing.  One tile per block (tiles taken longest list first, by the
// length classes of the tile ranges), one sub-tile per wavefront; each lane shades
// PPT pixels of one column, sharing the LDS reads and the dx terms.  List entries are staged
// in LDS per batch with the conic pre-scaled, so that for a pixel offset (dx, dy)
//   q = A' dx^2 + B' dx dy + C' dy^2 + log2(o),   A' = -1/2 log2(e) A, B' = -log2(e) B,
//   C' = -1/2 log2(e) C,   alpha = min(0.99, exp2(q)) = min(0.99, o G).
// The backward evaluates q with the same operations, so both passes take the same decisions.
// Per pixel: skip if alpha < 1/255; stop (without blending) if T (1 - alpha) < 1e-4; else
// C += alpha T c, D += alpha T z, T *= 1 - alpha.  rgb = C + T bg, depth = D, alpha = 1 - T.
// Each batch of the list is culled against the bounding box of the wavefront's live pixels
// (those not yet stopped) and compacted (in list order) before the pixel loop; the loop is
// predicated (after the cull nearly every entry reaches some live pixel, so a per-entry
// wavefront skip costs more than it saves) and the wavefront leaves the list as soon as none
// of its pixels is live.
// --------------------------------------------------------------------------------------------
// Sub-tile of one wavefront: SW x SH pixels, 64 lanes x PPT pixels per lane (pixel p of a
// lane sits 64 / SW rows below pixel p - 1).  8 x 8 squares when the tile allows.
template <int TW, int TH, int PPT>
struct SubTile {
    // the narrowest of 8, 16, 32 columns whose 64 PPT / width rows fit the tile's height
    static constexpr int SW = (TW >= 8 && TH % (8 * PPT) == 0) ? 8 : ((TW >= 16 && TH % (4 * PPT) == 0) ? 16 : 32);
    static constexpr int SH = 64 * PPT / SW;
    static constexpr int WAVES = (TW / SW) * (TH / SH);
    static constexpr int LROWS = 64 / SW;
    static_assert(TW % SW == 0 && TH % SH == 0, "sub-tile must tile the tile");
};

// One wavefront composites its sub-tile of tile t, walking the tile's whole list in batches of
// 64 entries staged in the wavefront's own LDS (wavefront-level synchronisation only, so each
// wavefront stops as soon as its own pixels are saturated).
template <int TW, int TH, int PPT, bool SAVE, bool COUNT>
__device__ __forceinline__ void composite_sub(const FwdArgs& a, const long long t, const int wave, const int lane,
                                              float4* s0, float4* s1, float4* s2, const uint32_t* __restrict__ starts,
                                              const Env* __restrict__ envs) {
    using ST = SubTile<TW, TH, PPT>;
    const int image = (int)(t / a.tpi);
    const int lt = (int)(t - (long long)image * a.tpi);
    const int ty = lt / a.tiles_x, tx = lt - ty * a.tiles_x;
    const int sx = wave % (TW / ST::SW), sy = wave / (TW / ST::SW);
    const int px = tx * TW + sx * ST::SW + lane % ST::SW;
    const int py0 = ty * TH + sy * ST::SH + lane / ST::SW;
    uint32_t start = starts[t], end = starts[t + 1];
    if ((unsigned long long)end > (unsigned long long)a.pair_cap) end = start;  // overflow
    const int env = image / a.C, cam = image - env * a.C;
    const Env ev = envs[env];
    const long long rec_off = (long long)a.C * ev.gid_base + (long long)cam * ev.n - (long long)ev.gid_base;
    const float fpx = (float)px + 0.5f;
    const float thr = (float)(1.0 / 255.0);
    // Per pixel: T > 0 is the transmittance while the pixel is live; at the stop T becomes
    // -T (the sign marks a stopped pixel and |T| keeps its final transmittance), so later
    // entries add nothing.  Pixels outside the image start stopped.
    float fpy[PPT], T[PPT], Cr[PPT], Cg[PPT], Cb[PPT], D[PPT];
    uint32_t last[PPT], evals[PPT];
    bool inside[PPT];
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const int py = py0 + p * ST::LROWS;
        inside[p] = px < a.width && py < a.height;
        fpy[p] = (float)py + 0.5f;
        T[p] = inside[p] ? 1.0f : -1.0f;
        Cr[p] = Cg[p] = Cb[p] = D[p] = 0.0f;
        last[p] = 0;
        evals[p] = 0;
    }
    // an entry with q below this at every pixel of the sub-tile cannot pass the 1/255 test
    // (exp2 is accurate to ~1e-7 relative, the margin is 1e-3 in the exponent)
    const float qcut = -7.994353436858858f - 1e-3f;  // log2(1/255) - 1e-3
    // centre of the sub-tile's first pixel
    const float rx0 = (float)(tx * TW + sx * ST::SW) + 0.5f;
    const float ry0 = (float)(ty * TH + sy * ST::SH) + 0.5f;
    // software pipeline over batches of 64 list entries: the ids of batch b + 2 and the
    // records of batch b + 1 are loaded while batch b is composited
    const uint32_t nid = ev.n;
    auto load_id = [&](uint32_t j) -> uint32_t {
        return j < end ? (uint32_t)a.pairs[j] - ev.gid_base : 0xffffffffu;  // local id, or none
    };
    auto load_rec = [&](uint32_t lid, Record& R) {
        if (lid < nid) R = a.records[rec_off + ev.gid_base + lid];
    };
    uint32_t lid_cur = load_id(start + lane), lid_next = load_id(start + 64u + lane);
    Record R_cur;
    load_rec(lid_cur, R_cur);
    for (uint32_t base = start; base < end; base += 64) {
        // bounding box of the wavefront's live pixels (lane l holds column l % SW and row
        // l / SW + p LROWS of the sub-tile): entries that cannot reach it blend nothing at any
        // live pixel and are not staged
        unsigned long long live = 0;
        int lr0 = ST::SH, lr1 = -1;
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            const unsigned long long m = __ballot(T[p] > 0.0f);
            if (m) {
                live |= m;
                lr0 = min(lr0, (int)__builtin_ctzll(m) / ST::SW + p * ST::LROWS);
                lr1 = max(lr1, (63 - (int)__builtin_clzll(m)) / ST::SW + p * ST::LROWS);
            }
        }
        if (!live) break;
#pragma unroll
        for (int sft = 32; sft >= ST::SW; sft >>= 1) live |= live >> sft;
        live &= (ST::SW == 32 ? 0xffffffffull : ((1ull << ST::SW) - 1ull));
        const float lx0 = rx0 + (float)__builtin_ctzll(live), lx1 = rx0 + (float)(63 - (int)__builtin_clzll(live));
        const float ly0 = ry0 + (float)lr0, ly1 = ry0 + (float)lr1;
        // stage the batch's entries that can reach this sub-tile, compacted in list order
        const uint32_t j = base + lane;
        const Record R = R_cur;
        const uint32_t lid = lid_cur;
        lid_cur = lid_next;
        load_rec(lid_cur, R_cur);
        lid_next = load_id(j + 128u);
        bool keep = false;
        if (j < end) {
            if (lid < nid) {
                keep = reaches_rect(R, lx0, lx1, ly0, ly1, qcut);
            } else {  // never produced by a consistent emission; blends nothing
                atomicOr(&a.status->flags, 2u);
            }
        }
        const unsigned long long km = __ballot(keep);
        if (keep) {
            const int slot = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(km >> 32),
                                                            __builtin_amdgcn_mbcnt_lo((uint32_t)km, 0u));
            s0[slot] = make_float4(R.r0.x, R.r0.y, -0.7213475204444817f * R.r1.x, -1.4426950408889634f * R.r1.y);
            s1[slot] = make_float4(-0.7213475204444817f * R.r1.z, R.r1.w, R.r0.w, R.r2.x);
            s2[slot] = make_float4(R.r2.y, R.r2.z, __uint_as_float(j - start + 1u), 0.0f);
        }
        const int n = __popcll(km);
        // pad the staged entries to a multiple of 4 with entries that blend nothing at any
        // pixel (log2 opacity -inf: q = -inf, alpha 0 < 1/255, colour and depth 0, index 0),
        // so the walk below needs no per-entry bound
        const int n4 = (n + 3) & ~3;
        if (lane >= n && lane < n4) {
            s0[lane] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            s1[lane] = make_float4(0.0f, -__builtin_inff(), 0.0f, 0.0f);
            s2[lane] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
        // the wavefront's LDS writes are visible to its own later reads
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int k0 = 0; k0 < n4; k0 += 4) {
            bool wl = false;
#pragma unroll
            for (int p = 0; p < PPT; ++p) wl |= T[p] > 0.0f;
            if (!__any(wl)) break;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = k0 + u;
                const float4 e0 = s0[k];
                const float4 e1 = s1[k];
                const float dx = fpx - e0.x;
                const float Adx = e0.z * dx, Bdx = e0.w * dx;
                const float qx = fmaf(Adx, dx, e1.y);
                float q[PPT];
#pragma unroll
                for (int p = 0; p < PPT; ++p) {
                    const float dy = fpy[p] - e0.y;
                    q[p] = fmaf(Bdx, dy, fmaf(e1.x * dy, dy, qx));
                    if (COUNT) evals[p] += (T[p] > 0.0f && k < n) ? 1u : 0u;
                }
                const float4 e2 = s2[k];
                const uint32_t idx1 = __float_as_uint(e2.z);
#pragma unroll
                for (int p = 0; p < PPT; ++p) {
                    const float al = fminf(0.99f, __builtin_amdgcn_exp2f(q[p]));
                    const float w = al >= thr ? al * T[p] : 0.0f;
                    const float Tn = T[p] - w;
                    const bool st = Tn < 1e-4f;  // also true for a stopped pixel (T < 0)
                    const float wb = st ? 0.0f : w;
                    Cr[p] = fmaf(wb, e1.w, Cr[p]);
                    Cg[p] = fmaf(wb, e2.x, Cg[p]);
                    Cb[p] = fmaf(wb, e2.y, Cb[p]);
                    D[p] = fmaf(wb, e1.z, D[p]);
                    T[p] = st ? -fabsf(T[p]) : Tn;
                    if (SAVE) last[p] = wb > 0.0f ? idx1 : last[p];
                }
            }
        }
        // all lanes are done reading this batch before the next one overwrites it
        __builtin_amdgcn_wave_barrier();
    }
    const gsr_camera& cm = a.cams[image];
    unsigned long long nev = 0;
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        nev += evals[p];
        if (!inside[p]) continue;
        const float Tf = fabsf(T[p]);
        const int py = py0 + p * ST::LROWS;
        const size_t q = ((size_t)image * a.height + py) * a.width + px;
        float r = fmaf(Tf, cm.bg[0], Cr[p]), g = fmaf(Tf, cm.bg[1], Cg[p]), b = fmaf(Tf, cm.bg[2], Cb[p]);
        if (a.aug) {
            const float3 o = augment_pixel(r, g, b, a.aug[image], a.overlay ? a.overlay + 3 * q : nullptr);
            r = o.x;
            g = o.y;
            b = o.z;
        }
        a.rgb[3 * q + 0] = r;
        a.rgb[3 * q + 1] = g;
        a.rgb[3 * q + 2] = b;
        a.depth[q] = D[p];
        if (a.alpha) a.alpha[q] = 1.0f - Tf;
        if (SAVE) {
            a.T_final[q] = Tf;
            a.n_contrib[q] = last[p];
        }
    }
    if (COUNT) {
        for (int off = 32; off > 0; off >>= 1) nev += __shfl_xor(nev, off, 64);
        if (lane == 0 && nev) atomicAdd(&a.status->evals[blockIdx.x % kParts], nev);
    }
}

template <int TW, int TH, int PPT, bool SAVE, bool COUNT>
__global__ __launch_bounds__((64 * SubTile<TW, TH, PPT>::WAVES)) void k_composite(FwdArgs a, const uint32_t* __restrict__ starts,
                                                                              const Env* __restrict__ envs,
                                                                              const Status* __restrict__ status,
                                                                              const uint32_t* __restrict__ cls_list) {
    constexpr int NW = SubTile<TW, TH, PPT>::WAVES;
    __shared__ float4 s0[NW][64], s1[NW][64];
    __shared__ float4 s2[NW][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // tiles longest list first (length classes 5, 4, ..., 0, then class 6), so the longest
    // lists do not start at the end of the grid
    uint32_t k = blockIdx.x;
    int cls = kLenLong;
    while (cls >= 0 && k >= status->cls[cls]) {
        k -= status->cls[cls];
        --cls;
    }
    if (cls < 0) cls = kLenNone;
    composite_sub<TW, TH, PPT, SAVE, COUNT>(a, (long long)cls_list[(size_t)cls * a.tiles + k], wave, lane, s0[wave],
                                            s1[wave], s2[wave], starts, envs);
}

// persistent grid: block b takes queue items b, b + G, b + 2G, ... of the longest-first queue
// (length classes from the longest lists down, then the lists of at most one entry).  A static
// interleave needs no shared counter: a single global atomic per tile would serialise the
// grid.  The wavefronts of a block work on the same tile independently.
template <int TW, int TH, int PPT, bool SAVE, bool COUNT>
__global__ __launch_bounds__((64 * SubTile<TW, TH, PPT>::WAVES)) void k_composite_persistent(
    FwdArgs a, const uint32_t* __restrict__ starts, const Env* __restrict__ envs, const Status* __restrict__ status,
    const uint32_t* __restrict__ cls_list) {
    constexpr int NW = SubTile<TW, TH, PPT>::WAVES;
    __shared__ float4 s0[NW][64], s1[NW][64];
    __shared__ float4 s2[NW][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const Status* st = status;
    uint32_t cnt[kNumClasses];
#pragma unroll
    for (int c = 0; c < kNumClasses; ++c) cnt[c] = st->cls[c];
    for (long long item = blockIdx.x; item < a.tiles; item += gridDim.x) {
        // queue order: longest class first (5, 4, ..., 0), then class 6
        uint32_t k = (uint32_t)item;
        int cls = kLenLong;
        while (cls >= 0 && k >= cnt[cls]) {
            k -= cnt[cls];
            --cls;
        }
        if (cls < 0) cls = kLenNone;
        composite_sub<TW, TH, PPT, SAVE, COUNT>(a, (long long)cls_list[(size_t)cls * a.tiles + k], wave, lane, s0[wave],
                                                s1[wave], s2[wave], starts, envs);
    }
}

// the (tile, depth bits) key of every slot, rebuilt from the slot's Gaussian id and the depth
// its camera record holds (the projection writes the same z to the record and to the key)
__global__ void k_copy_pairs(FwdArgs a, uint64_t* keys, uint32_t* vals, uint32_t* ranges) {
    const long long t = blockIdx.x;
    const int image = (int)(t / a.tpi);
    const int env = image / a.C, cam = image - env * a.C;
    const Env ev = a.envs[env];
    const long long rec_off = (long long)a.C * ev.gid_base + (long long)cam * ev.n - (long long)ev.gid_base;
    const uint32_t s = a.starts[t], e = a.starts[t + 1];
    if (threadIdx.x == 0) {
        ranges[2 * t] = s;
        ranges[2 * t + 1] = e;
    }
    for (uint32_t i = s + threadIdx.x; i < e; i += blockDim.x) {
        const uint32_t gid = a.pairs[i];
        const uint32_t zb = gid - ev.gid_base < ev.n ? __float_as_uint(a.records[rec_off + gid].r0.w) : 0xffffffffu;
        keys[i] = ((unsigned long long)t << 32) | zb;
        vals[i] = gid;
    }
}

// image-space domain randomisation of finished frames, one thread per pixel (grid-stride)
__global__ __launch_bounds__(256) void k_augment(size_t n_pix, size_t pix_per_image, const float* __restrict__ rgb,
                                                 const float* __restrict__ overlay,
                                                 const gsr_augment* __restrict__ params, float* out) {
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n_pix; q += (size_t)gridDim.x * blockDim.x) {
        const size_t image = q / pix_per_image;
        const float r = rgb[3 * q + 0], g = rgb[3 * q + 1], b = rgb[3 * q + 2];
        const float3 o = augment_pixel(r, g, b, params[image], overlay ? overlay + 3 * q : nullptr);
        out[3 * q + 0] = o.x;
        out[3 * q + 1] = o.y;
        out[3 * q + 2] = o.z;
    }
}

hipError_t launch_augment(int images, int width, int height, const float* rgb, const float* overlay,
                          const gsr_augment* params, float* out, int num_cu, hipStream_t s) {
    const size_t ppi = (size_t)width * height, n = ppi * (size_t)images;
    const size_t want = (n + 255) / 256, cap = (size_t)num_cu * 16;
    hipLaunchKernelGGL(k_augment, dim3((unsigned)std::max<size_t>(1, std::min(want, cap))), dim3(256), 0, s, n, ppi,
                       rgb, overlay, params, out);
    return hipGetLastError();
}

// --------------------------------------------------------------------------------------------
// launch sequence
// --------------------------------------------------------------------------------------------
template <int L>
static hipError_t launch_project(const FwdArgs& a, hipStream_t s) {
    const size_t lds = (size_t)(kBlock / 64) * a.C * sizeof(uint32_t);
    hipLaunchKernelGGL((k_project<L>), dim3(a.n_supers), dim3(kBlock), lds, s, a, a.supers, a.envs, a.blocks, a.nodes,
                       a.views);
    return hipGetLastError();
}

template <int TW, int TH, int PPT, bool SAVE, bool COUNT>
static void launch_composite_s(const FwdArgs& a, hipStream_t s) {
    constexpr int NT = 64 * SubTile<TW, TH, PPT>::WAVES;
    if (a.persistent) {
        // persistent_grid counts 256-thread blocks
        const long long want = (long long)a.persistent_grid * 256 / NT;
        const long long g = want < a.tiles ? want : a.tiles;
        hipLaunchKernelGGL((k_composite_persistent<TW, TH, PPT, SAVE, COUNT>), dim3((unsigned)(g > 0 ? g : 1)), dim3(NT),
                           0, s, a, a.starts, a.envs, a.status, a.cls_list);
    } else {
        hipLaunchKernelGGL((k_composite<TW, TH, PPT, SAVE, COUNT>), dim3((unsigned)a.tiles), dim3(NT), 0, s, a, a.starts,
                           a.envs, a.status, a.cls_list);
    }
}

template <int TW, int TH, int PPT>
static void launch_composite(const FwdArgs& a, hipStream_t s) {
    if (a.save) {
        if (a.count) launch_composite_s<TW, TH, PPT, true, true>(a, s);
        else launch_composite_s<TW, TH, PPT, true, false>(a, s);
    } else {
        if (a.count) launch_composite_s<TW, TH, PPT, false, true>(a, s);
        else launch_composite_s<TW, TH, PPT, false, false>(a, s);
    }
}

static size_t emit_lds(const FwdArgs& a) { return (size_t)a.tpi * (sizeof(unsigned long long) + sizeof(uint32_t)); }
// wavefronts per emission block: 4, or 16 once the image's tile table is large (large tile
// grids come with many tiles per Gaussian, so a round's pairs keep 1024 threads busy)
static int emit_waves(const FwdArgs& a) { return emit_lds(a) > kEmitLdsSmall ? 16 : 4; }
static const void* emit_kernel(const FwdArgs& a) {
    return emit_waves(a) == 16 ? (const void*)k_emit<16> : (const void*)k_emit<4>;
}
static size_t counts_lds(const FwdArgs& a) { return (size_t)(a.tiles_x + 1) * (a.tiles_y + 1) * sizeof(int); }

hipError_t forward_lds_limits(const FwdArgs& a) {
    // only grids beyond 48 KiB of dynamic LDS need the raised limit (it persists per kernel)
    constexpr size_t kDefault = 48 * 1024;
    hipError_t e = hipSuccess;
    if (emit_lds(a) > kDefault)
        e = hipFuncSetAttribute(emit_kernel(a), hipFuncAttributeMaxDynamicSharedMemorySize, (int)emit_lds(a));
    if (e == hipSuccess && counts_lds(a) > kDefault)
        e = hipFuncSetAttribute((const void*)k_tile_counts, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)counts_lds(a));
    return e;
}

hipError_t launch_forward(const FwdArgs& a, hipStream_t s) {
    auto mark = [&](int i) {
        if (a.stage_events) hipEventRecord(a.stage_events[i], s);
    };
    const int nv = a.n_nodes * a.C;
    mark(0);
    hipLaunchKernelGGL(k_views, dim3((nv + 63) / 64), dim3(64), 0, s, a);
    mark(1);
    if (a.n_supers > 0) {
        hipError_t e;
        switch (a.sh_degree) {
            case 0: e = launch_project<0>(a, s); break;
            case 1: e = launch_project<1>(a, s); break;
            case 2: e = launch_project<2>(a, s); break;
            default: e = launch_project<3>(a, s); break;
        }
        if (e != hipSuccess) return e;
    }
    mark(2);
    const int nl = a.n_supers * a.C;
    const unsigned ncu = (unsigned)(a.num_cu > 0 ? a.num_cu : 256);
    auto grid = [&](long long items, unsigned per_cu) {  // a multiple of 8 (one block per XCD at least)
        const long long g = std::min<long long>(items, (long long)ncu * per_cu);
        return dim3((unsigned)((std::max<long long>(g, 1) + 7) / 8 * 8));
    };
    hipLaunchKernelGGL(k_seg, dim3(1), dim3(1024), 0, s, a);
    if (nl > 0) hipLaunchKernelGGL(k_gather, grid(nl, 16), dim3(256), 0, s, a);
    mark(3);
    for (int pass = 0; pass < 4; ++pass) {
        hipLaunchKernelGGL(k_radix_hist, grid(a.sort_chunks, 8), dim3(256), 0, s, a, pass);
        hipLaunchKernelGGL(k_radix_scan, dim3(a.images), dim3(1024), 0, s, a);
        hipLaunchKernelGGL(k_radix_scatter, grid(a.sort_chunks, 6), dim3(256), 0, s, a, pass);
    }
    mark(4);
    const long long n_blocks = (long long)a.sort_chunks * (kSortTile / kPairBlock);
    hipLaunchKernelGGL(k_pair_blocks, grid(n_blocks, 8), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_pair_scan, dim3(1), dim3(1024), 0, s, a);
    hipLaunchKernelGGL(k_chunk_starts, grid(n_blocks, 8), dim3(256), 0, s, a);
    mark(5);
    hipLaunchKernelGGL(k_tile_counts, grid(a.chunk_cap, 32), dim3(kCountThreads), counts_lds(a), s, a);
    mark(6);
    const long long n_segs = (long long)a.chunk_cap / kSegChunks + a.images + 1;
    hipLaunchKernelGGL(k_tile_seg, grid(n_segs * ((a.tpi + kSegThreads - 1) / kSegThreads), 8), dim3(kSegThreads),
                       0, s, a);
    hipLaunchKernelGGL(k_tile_ranges, dim3(a.images), dim3(1024), 0, s, a);
    mark(7);
    if (emit_waves(a) == 16) hipLaunchKernelGGL(k_emit<16>, grid(a.chunk_cap, 2), dim3(1024), emit_lds(a), s, a);
    else hipLaunchKernelGGL(k_emit<4>, grid(a.chunk_cap, 8), dim3(256), emit_lds(a), s, a);
    mark(8);
    if (a.tw == 16 && a.th == 16) {
        if (a.ppt == 4) launch_composite<16, 16, 4>(a, s);
        else if (a.ppt == 2) launch_composite<16, 16, 2>(a, s);
        else launch_composite<16, 16, 1>(a, s);
    } else if (a.tw == 16 && a.th == 8) {
        if (a.ppt == 2) launch_composite<16, 8, 2>(a, s);
        else launch_composite<16, 8, 1>(a, s);
    } else if (a.tw == 8 && a.th == 8) {
        launch_composite<8, 8, 1>(a, s);
    } else {
        if (a.ppt == 4) launch_composite<32, 8, 4>(a, s);
        else if (a.ppt == 2) launch_composite<32, 8, 2>(a, s);
        else launch_composite<32, 8, 1>(a, s);
    }
    mark(9);
    return hipGetLastError();
}

hipError_t launch_copy_pairs(const FwdArgs& a, uint64_t* keys, uint32_t* values, uint32_t* ranges, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_pairs, dim3((unsigned)a.tiles), dim3(256), 0, s, a, keys, values, ranges);
    return hipGetLastError();
}

}  // namespace gsr
