// Forward path of the gfx950 Gaussian-splatting RGB-D renderer.
//
// Stages (all on one stream, no host synchronisation between them):
//   k_views        per (node, camera): camera<-node map composed in FP64, rounded once to FP32
//                  (scene composition: background plus rigidly posed nodes, paper Sec. III-B)
//   k_project      per Gaussian, all cameras of its env: EWA projection ("splatting"), tile
//                  rectangle and depth key (the FP32 key specification below), SH colour
//                  (paper Sec. III-A), projected record; per super-block (runs of an env's
//                  Gaussians) per-tile pair counts via a difference grid kept in LDS
//   k_tile_offsets per (image, tile): scan over the env's super-blocks of their pair counts
//   k_scan         exclusive scan of per-tile counts -> per-tile [start, end) ranges
//   k_emit         (depth bits, Gaussian id) pairs written into their tile's bucket; each
//                  super-block starts at its precomputed slot, so only LDS atomics are used
//   k_classify, k_sort_*   each tile's bucket sorted by (depth bits, id) in LDS; lists longer
//                  than one LDS load are chunk-sorted then merged ("efficient sorting")
//   k_composite    per tile, front-to-back alpha blending of colour and camera-space z
//                  (RGB and depth sensors, paper Sec. III-C), early exit when every pixel of a
//                  wavefront is saturated
//
// Compiled with -ffp-contract=off: every a*b+c below is two rounded operations unless an
// explicit fmaf() is written, and / and sqrtf are correctly rounded.  This makes the key
// specification in k_project reproducible bit for bit by any IEEE FP32 implementation of
// the same operation sequence.
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
        st->work_head = 0;
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

// one Gaussian's SH coefficients into registers (16-byte loads when the row allows)
template <int L>
__device__ inline void load_sh(const float* __restrict__ sh, float* c) {
    constexpr int K3 = 3 * (L + 1) * (L + 1);
    if constexpr (K3 % 4 == 0) {
        const float4* s4 = reinterpret_cast<const float4*>(sh);
#pragma unroll
        for (int i = 0; i < K3 / 4; ++i) {
            const float4 q = s4[i];
            c[4 * i + 0] = q.x; c[4 * i + 1] = q.y; c[4 * i + 2] = q.z; c[4 * i + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < K3; ++i) c[i] = sh[i];
    }
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
    // LDS: per camera, the count of this super-block's visible Gaussians, then a
    // (tiles_y + 1) x (tiles_x + 1) difference grid of pair counts: a rectangle adds +1/-1 at
    // its four corners; the 2D prefix gives pairs per tile
    extern __shared__ int s_lds[];
    const Super sb = supers[blockIdx.x];
    const Env ev = envs[sb.env];
    const int C = a.C;
    const int gx = a.tiles_x + 1, gy = a.tiles_y + 1, gsz = gx * gy;
    uint32_t* s_nvis = reinterpret_cast<uint32_t*>(s_lds);
    int* s_grid = s_lds + C;
    for (int i = threadIdx.x; i < C * gsz + C; i += kBlock) s_lds[i] = 0;
    __syncthreads();
    constexpr int K = (L + 1) * (L + 1);
    const int i = threadIdx.x;
    const float thr = (float)(1.0 / 255.0);
    const float itw = 1.0f / (float)a.tw, ith = 1.0f / (float)a.th;
    int n_vis = 0, n_any = 0, nonfinite = 0;
    // this thread's Gaussian of the next chunk, loaded one chunk ahead so that its latency
    // overlaps the current chunk's arithmetic
    float nm0 = 0.f, nm1 = 0.f, nm2 = 0.f, no = 0.f, ns0 = 0.f, ns1 = 0.f, ns2 = 0.f;
    float4 nq = make_float4(0.f, 0.f, 0.f, 0.f);
    auto fetch = [&](int ch) {
        const Block blk = blocks[ch];
        if (i < (int)blk.count) {
            const Node& nd = nodes[blk.node];
            const size_t li = blk.gid0 + (uint32_t)i - nd.gid_base;
            nm0 = nd.means[3 * li + 0]; nm1 = nd.means[3 * li + 1]; nm2 = nd.means[3 * li + 2];
            no = nd.opac[li];
            ns0 = nd.scales[3 * li + 0]; ns1 = nd.scales[3 * li + 1]; ns2 = nd.scales[3 * li + 2];
            nq = reinterpret_cast<const float4*>(nd.quats)[li];
        }
    };
    if (sb.chunk_begin < sb.chunk_end) fetch(sb.chunk_begin);
    for (int ch = sb.chunk_begin; ch < sb.chunk_end; ++ch) {
        const Block blk = blocks[ch];
        const float mu0 = nm0, mu1 = nm1, mu2 = nm2, o = no, s0 = ns0, s1 = ns1, s2 = ns2;
        const float q0 = nq.x, q1 = nq.y, q2 = nq.z, q3 = nq.w;
        if (ch + 1 < sb.chunk_end) fetch(ch + 1);
        if (i >= (int)blk.count) continue;
        const Node& nd = nodes[blk.node];
        const uint32_t gid = blk.gid0 + i;
        const size_t li = gid - nd.gid_base;
        const size_t lg = gid - ev.gid_base;
        if (!(isfinite(mu0) && isfinite(mu1) && isfinite(mu2) && isfinite(o) && isfinite(s0) && isfinite(s1) &&
              isfinite(s2) && isfinite(q0) && isfinite(q1) && isfinite(q2) && isfinite(q3))) {
            nonfinite += C;  // culled and counted once per camera
            continue;
        }
        if (!(o >= thr)) continue;
        // the rotation of the unit quaternion (camera independent)
        const float n2 = fmaf(q0, q0, fmaf(q1, q1, fmaf(q2, q2, q3 * q3)));
        float R00 = 0.f, R01 = 0.f, R02 = 0.f, R10 = 0.f, R11 = 0.f, R12 = 0.f, R20 = 0.f, R21 = 0.f, R22 = 0.f;
        if (n2 > 0.0f) {
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
            const View& v = views[blk.node * C + c];
            const size_t rec = (size_t)C * ev.gid_base + (size_t)c * ev.n + lg;
            const float p0 = fmaf(v.W[0], mu0, fmaf(v.W[1], mu1, fmaf(v.W[2], mu2, v.w[0])));
            const float p1 = fmaf(v.W[3], mu0, fmaf(v.W[4], mu1, fmaf(v.W[5], mu2, v.w[1])));
            const float p2 = fmaf(v.W[6], mu0, fmaf(v.W[7], mu1, fmaf(v.W[8], mu2, v.w[2])));
            if (!(isfinite(p0) && isfinite(p1) && isfinite(p2))) { ++nonfinite; continue; }
            const float z = p2;
            if (!(z > v.znear)) continue;
            if (!(n2 > 0.0f)) continue;
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
            if (!(det > 0.0f)) continue;
            const float rx = fmaf(3.33f, sqrtf(ca), 0.015625f);
            const float ry = fmaf(3.33f, sqrtf(cc), 0.015625f);
            const float tx0f = fminf(fmaxf(floorf((u - rx) * itw), 0.0f), (float)a.tiles_x);
            const float tx1f = fminf(fmaxf(floorf((u + rx) * itw) + 1.0f, 0.0f), (float)a.tiles_x);
            const float ty0f = fminf(fmaxf(floorf((vv - ry) * ith), 0.0f), (float)a.tiles_y);
            const float ty1f = fminf(fmaxf(floorf((vv + ry) * ith) + 1.0f, 0.0f), (float)a.tiles_y);
            const int tx0 = (int)tx0f, tx1 = (int)tx1f, ty0 = (int)ty0f, ty1 = (int)ty1f;
            if (tx0 >= tx1 || ty0 >= ty1) continue;
            // visible: projected record (the conic and colour enter pixel values only, so the
            // hardware reciprocal suffices there)
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
            // append to this super-block's visible list for camera c
            const uint32_t slot = atomicAdd(&s_nvis[c], 1u);
            a.vis[((size_t)blockIdx.x * C + c) * a.sb_cap + slot] =
                make_uint4((uint32_t)tx0 | ((uint32_t)ty0 << 16), (uint32_t)tx1 | ((uint32_t)ty1 << 16),
                           __float_as_uint(z), gid);
            // pair counts: +1/-1 corners of the rectangle in the image's difference grid
            int* h = s_grid + c * gsz;
            atomicAdd(h + ty0 * gx + tx0, 1);
            atomicAdd(h + ty0 * gx + tx1, -1);
            atomicAdd(h + ty1 * gx + tx0, -1);
            atomicAdd(h + ty1 * gx + tx1, 1);
            ++n_vis;
            vis_any = true;
        }
        n_any += vis_any ? 1 : 0;
    }
    if (nonfinite) atomicAdd(&a.status->nonfinite, (uint32_t)nonfinite);
    __syncthreads();
    // 2D prefix of every camera's grid: along x, then along y
    for (int r = threadIdx.x; r < C * gy; r += kBlock) {
        int* row = s_grid + (r / gy) * gsz + (r % gy) * gx;
        int acc = 0;
        for (int x = 0; x < gx; ++x) { acc += row[x]; row[x] = acc; }
    }
    __syncthreads();
    for (int col = threadIdx.x; col < C * gx; col += kBlock) {
        int* g = s_grid + (col / gx) * gsz + (col % gx);
        int acc = 0;
        for (int y = 0; y < gy; ++y) { acc += g[y * gx]; g[y * gx] = acc; }
    }
    __syncthreads();
    // this super-block's pairs per (camera, tile) and visible-list lengths, plain stores
    if (threadIdx.x < C) a.sbvis[(size_t)blockIdx.x * C + threadIdx.x] = s_nvis[threadIdx.x];
    uint32_t* out = a.sbcnt + (size_t)blockIdx.x * C * a.tpi;
    for (int j = threadIdx.x; j < C * a.tpi; j += kBlock) {
        const int c = j / a.tpi, t = j - c * a.tpi;
        const int ty = t / a.tiles_x, tx = t - ty * a.tiles_x;
        out[j] = (uint32_t)s_grid[c * gsz + ty * gx + tx];
    }
    // block sums of visible records: one atomic per block into its counter slot
    unsigned long long nv = (unsigned long long)n_vis, na = (unsigned long long)n_any;
    for (int off = 32; off > 0; off >>= 1) {
        nv += __shfl_xor(nv, off, 64);
        na += __shfl_xor(na, off, 64);
    }
    __shared__ unsigned long long s_sum[2 * (kBlock / 64)];
    if ((threadIdx.x & 63) == 0) {
        s_sum[2 * (threadIdx.x >> 6)] = nv;
        s_sum[2 * (threadIdx.x >> 6) + 1] = na;
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
// per (image, tile): exclusive scan over the env's super-blocks -> each super-block's first
// slot within the tile's bucket; the tile total -> pairs per tile
// --------------------------------------------------------------------------------------------
__global__ void k_tile_offsets(FwdArgs a) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.tiles) return;
    const int image = (int)(idx / a.tpi);
    const int t = (int)(idx - (long long)image * a.tpi);
    const int env = image / a.C, c = image - env * a.C;
    const Env ev = a.envs[env];
    // 16 super-blocks at a time: all loads issued before the first store, so they overlap
    constexpr int B = 16;
    const size_t stride = (size_t)a.C * a.tpi;
    uint32_t* p = a.sbcnt + ((size_t)ev.sb_begin * a.C + c) * a.tpi + t;
    uint32_t run = 0;
    for (int k0 = 0; k0 < ev.sb_count; k0 += B) {
        const int m = ev.sb_count - k0 < B ? ev.sb_count - k0 : B;
        uint32_t v[B];
#pragma unroll
        for (int k = 0; k < B; ++k) v[k] = k < m ? p[(size_t)(k0 + k) * stride] : 0u;
#pragma unroll
        for (int k = 0; k < B; ++k) {
            if (k < m) p[(size_t)(k0 + k) * stride] = run;
            run += v[k];
        }
    }
    a.counts[idx] = run;
}

// --------------------------------------------------------------------------------------------
// exclusive scan of per-tile counts (one block, coalesced 1024-tile chunks); total pairs and
// overflow into the status word
// --------------------------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_scan(FwdArgs a) {
    __shared__ unsigned long long s_wave[16];
    __shared__ unsigned long long s_carry;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    const long long T = a.tiles;
    uint32_t mx = 0;
    for (long long base = 0; base < T; base += 1024) {
        const long long i = base + threadIdx.x;
        const uint32_t v = i < T ? a.counts[i] : 0u;
        mx = v > mx ? v : mx;
        unsigned long long x = v;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const unsigned long long y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        if (lane == 63) s_wave[wave] = x;
        __syncthreads();
        unsigned long long before = s_carry;
        for (int w = 0; w < wave; ++w) before += s_wave[w];
        const unsigned long long excl = before + x - v;
        if (i < T) {
            const uint32_t st = excl > 0xffffffffull ? 0xffffffffu : (uint32_t)excl;
            a.starts[i] = st;
        }
        __syncthreads();
        if (threadIdx.x == 1023) s_carry = excl + v;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const unsigned long long total = s_carry;
        a.starts[T] = total > 0xffffffffull ? 0xffffffffu : (uint32_t)total;
        a.status->pairs = total;
        if (total > (unsigned long long)a.pair_cap) atomicOr(&a.status->flags, (uint32_t)GSR_STATUS_OVERFLOW);
    }
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t o = __shfl_xor(mx, off, 64);
        mx = o > mx ? o : mx;
    }
    if (lane == 0 && mx) atomicMax(&a.status->max_tile, mx);
}

// --------------------------------------------------------------------------------------------
// pair emission into tile buckets.  Each (super-block, camera) walks its compact list of
// visible Gaussians and knows, per tile, the first slot of its pairs (tile start + the offsets
// of the env's earlier super-blocks), so slots are taken with LDS atomics only.  Within a
// batch of 256 list entries, the (Gaussian, tile) pairs are numbered by a block-wide prefix
// over rectangle areas and split into equal runs of consecutive pairs, one per thread, so
// large rectangles are shared by all threads.
// Pair = (z bits << 32) | Gaussian id.
// --------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_emit(FwdArgs a, const Super* __restrict__ supers,
                                                  const uint32_t* __restrict__ sbvis) {
    extern __shared__ uint32_t s_slot[];
    __shared__ uint32_t s_off[kBlock + 1];
    __shared__ uint32_t s_x0[kBlock], s_y0[kBlock], s_w[kBlock], s_z[kBlock], s_id[kBlock];
    const Super sb = supers[blockIdx.x];
    const int c = blockIdx.y;
    const size_t image = (size_t)sb.env * a.C + c;
    const int tpi = a.tpi;
    const uint32_t* so = a.sbcnt + ((size_t)blockIdx.x * a.C + c) * tpi;
    for (int t = threadIdx.x; t < tpi; t += kBlock) s_slot[t] = a.starts[image * tpi + t] + so[t];
    const int i = threadIdx.x;
    const unsigned long long cap = (unsigned long long)a.pair_cap;
    const uint32_t nv = sbvis[(size_t)blockIdx.x * a.C + c];
    const uint4* lst = a.vis + ((size_t)blockIdx.x * a.C + c) * a.sb_cap;
    for (uint32_t b0 = 0; b0 < nv; b0 += kBlock) {
        uint32_t n_i = 0;
        if (b0 + i < nv) {
            const uint4 r = lst[b0 + i];
            const uint32_t x0 = r.x & 0xffffu, y0 = r.x >> 16, x1 = r.y & 0xffffu, y1 = r.y >> 16;
            n_i = (x1 - x0) * (y1 - y0);
            s_x0[i] = x0;
            s_y0[i] = y0;
            s_w[i] = x1 - x0;
            s_z[i] = r.z;
            s_id[i] = r.w;
        }
        // block-wide exclusive scan of n_i (Hillis-Steele in LDS)
        s_off[i + 1] = n_i;
        if (i == 0) s_off[0] = 0;
        __syncthreads();
        for (int off = 1; off < kBlock; off <<= 1) {
            const uint32_t v = (i + 1 > off) ? s_off[i + 1 - off] : 0u;
            __syncthreads();
            s_off[i + 1] += v;
            __syncthreads();
        }
        // thread i takes the consecutive pairs [k0, k1): one search for the owner of k0, then
        // a walk along the owners' rectangles (row-major tiles)
        const uint32_t total = s_off[kBlock];
        const uint32_t per = (total + kBlock - 1) / kBlock;
        const uint32_t k0 = (uint32_t)i * per, k1 = k0 + per < total ? k0 + per : total;
        if (k0 < k1) {
            int o = 0, hi = kBlock - 1;  // first owner with s_off[owner + 1] > k0
            while (o < hi) {
                const int mid = (o + hi) >> 1;
                if (s_off[mid + 1] > k0) hi = mid; else o = mid + 1;
            }
            uint32_t j = k0 - s_off[o];
            uint32_t w = s_w[o], x0 = s_x0[o];
            uint32_t tx = x0 + j % w, ty = s_y0[o] + j / w;
            uint32_t left = s_off[o + 1] - k0;  // pairs of owner o from k0 on
            unsigned long long val = ((unsigned long long)s_z[o] << 32) | (unsigned long long)s_id[o];
            for (uint32_t k = k0; k < k1; ++k) {
                while (left == 0) {  // next owner with pairs; k < total guarantees one exists
                    ++o;
                    w = s_w[o];
                    x0 = s_x0[o];
                    tx = x0;
                    ty = s_y0[o];
                    left = s_off[o + 1] - s_off[o];
                    val = ((unsigned long long)s_z[o] << 32) | (unsigned long long)s_id[o];
                }
                const uint32_t pos = atomicAdd(&s_slot[ty * a.tiles_x + tx], 1u);
                if ((unsigned long long)pos < cap) a.pairs[pos] = val;
                --left;
                if (++tx == x0 + w) {
                    tx = x0;
                    ++ty;
                }
            }
        }
        __syncthreads();
    }
}

// --------------------------------------------------------------------------------------------
// per-tile sort by (z bits, id): tiles are classed by list length (classes 0..4: at most
// 512, 1024, 2048, 4096, 8192 entries, sorted in LDS by one block; class 5: longer, sorted in
// chunks and merged; class 6: at most one entry or overflowed, not sorted); each class is sorted by a persistent
// grid pulling tiles from its list.  The lists also order the persistent compositor's queue,
// longest class first.
// --------------------------------------------------------------------------------------------
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

__global__ void k_classify(FwdArgs a) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int cls = -1;
    if (t < a.tiles) {
        const uint32_t s = a.starts[t], e = a.starts[t + 1];
        const uint32_t n = e - s;
        if ((unsigned long long)e > (unsigned long long)a.pair_cap || n <= 1) cls = kSortNone;
        else if (n <= 512) cls = 0;
        else if (n <= 1024) cls = 1;
        else if (n <= 2048) cls = 2;
        else if (n <= 4096) cls = 3;
        else if (n <= 8192) cls = 4;
        else cls = kSortBig;
    }
#pragma unroll
    for (int c = 0; c < kNumClasses; ++c) {
        const uint32_t pos = wave_append(&a.status->cls[c], cls == c);
        if (cls == c) a.cls_list[(size_t)c * a.tiles + pos] = (uint32_t)t;
    }
}


// Per-tile sort by (depth bits, Gaussian id) in LDS, for lists of at most NT * E entries.
// Each entry is packed into one 64-bit word X = (z bits - zmin) << ib | (id - idmin), whose
// order is the order of (z bits, id) and whose significant bits number TB = (bits of the
// depth range) + ib.  An LSD radix sort with 4-bit digits over the top 16 significant bits
// (12 for lists of at most 1024 entries; at most four passes) leaves the list in runs of equal
// top bits, in order; each entry then
// takes its place inside its run by counting the run's smaller words.  Runs are short for any
// spread of depths; if a run is longer than 64 entries, the tile is sorted again by LSD passes
// over all TB bits (so the result is exact for any input, and fast for the usual one).
// A pass: thread t owns entries [t E, t E + E) ("blocked") and ranks them among its own
// entries with 4-bit per-digit counters (one 64-bit word per 8 entries); the (digit, thread)
// counts are scanned in digit-major order across the block, and each entry is scattered to
// its digit's offset plus its rank, which keeps the pass stable.
// LDS layouts are padded so that the blocked accesses hit distinct banks: entry i lives at
// i + i / E, and count f of the digit-major table at f + 2 (f / 16) u16 slots.
template <int NT, int E>
__device__ __forceinline__ void sort_list(unsigned long long* p, const uint32_t n, unsigned long long* s_x, uint16_t* s_cnt,
                          uint32_t* s_w, uint32_t* s_long_p) {
    constexpr int CAP = NT * E;
    constexpr int NW = NT / 64;
    constexpr int NG = E / 8;
    constexpr int LE = E == 8 ? 3 : 4;
    static_assert((1 << LE) == E, "E must be 8 or 16");
    uint32_t& s_long = *s_long_p;
    if (n <= 1) return;  // nothing to order (uniform across the block); a chunk may hold one entry
    const auto P = [](uint32_t i) { return i + (i >> LE); };
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    // count (d, t) of the digit-major table lives at Q(d NT + t) = Q(t) + d DSTRIDE, with
    // Q(f) = f + 2 (f / 16) (NT is a multiple of 16)
    constexpr uint32_t DSTRIDE = NT + NT / 8;
    const uint32_t qt = (uint32_t)t + (((uint32_t)t >> 4) << 1);
    unsigned long long x[E];
    // one stable pass on the 4-bit digit at bit sh; x[] holds the thread's entries (blocked)
    // before and after, and s_x the whole list after
    // threads whose entries are all padding (t E >= n) only report their counts: padding words
    // are all-ones, so they always land in digit 15 behind every entry and are never stored
    const bool live = (uint32_t)t * E < n;
    auto pass = [&](int sh) {
        unsigned long long c[NG];
        uint32_t rk[E / 4];
#pragma unroll
        for (int g = 0; g < NG; ++g) c[g] = live ? 0ull : 8ull << 60;  // 8 entries in digit 15
#pragma unroll
        for (int k = 0; k < E / 4; ++k) rk[k] = 0u;
        if (live) {
#pragma unroll
            for (int r = 0; r < E; ++r) {
                const uint32_t s4 = ((uint32_t)(x[r] >> sh) & 15u) << 2;
                rk[r >> 2] |= ((uint32_t)(c[r >> 3] >> s4) & 15u) << ((r & 3) << 3);
                c[r >> 3] += 1ull << s4;
            }
        }
#pragma unroll
        for (int d = 0; d < 16; ++d) {
            uint32_t tot = 0;
#pragma unroll
            for (int g = 0; g < NG; ++g) tot += (uint32_t)(c[g] >> (4 * d)) & 15u;
            s_cnt[qt + d * DSTRIDE] = (uint16_t)tot;
        }
        __syncthreads();
        // exclusive scan in digit-major order: thread t takes counts 16 t .. 16 t + 15
        uint32_t tot = 0;
#pragma unroll
        for (int j = 0; j < 16; ++j) tot += s_cnt[18 * t + j];
        uint32_t incl = tot;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(incl, off, 64);
            if (lane >= off) incl += y;
        }
        if (lane == 63) s_w[wave] = incl;
        __syncthreads();
        uint32_t base = incl - tot;
#pragma unroll 1
        for (int i = 0; i < wave; ++i) base += s_w[i];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const uint32_t v = s_cnt[18 * t + j];
            s_cnt[18 * t + j] = (uint16_t)base;
            base += v;
        }
        __syncthreads();
        if (live) {
            // recompute the digits below instead of keeping E of them alive across the scan
#pragma unroll
            for (int r = 0; r < E; ++r) asm volatile("" : "+v"(x[r]));
#pragma unroll
            for (int r = 0; r < E; ++r) {
                const uint32_t s4 = ((uint32_t)(x[r] >> sh) & 15u) << 2;
                uint32_t rank = (rk[r >> 2] >> ((r & 3) << 3)) & 255u;
#pragma unroll
                for (int g = 0; g < (r >> 3); ++g) rank += (uint32_t)(c[g] >> s4) & 15u;
                const uint32_t dest = (uint32_t)s_cnt[qt + (s4 >> 2) * DSTRIDE] + rank;
                if (dest < n) s_x[P(dest)] = x[r];  // positions >= n hold padding only
                if ((r & 7) == 7) asm volatile("" ::: "memory");  // bounds the scheduling window (registers)
            }
        }
        __syncthreads();
        if (live) {
#pragma unroll
            for (int r = 0; r < E; ++r) x[r] = (uint32_t)(t * E + r) < n ? s_x[t * (E + 1) + r] : ~0ull;
        }
        __syncthreads();
    };
    // striped copy into LDS (entry t + k NT lives at P(t) + k (NT + NT / E))
#pragma unroll 1
    for (int k = 0; k < E; ++k) {
        const uint32_t i = (uint32_t)(t + k * NT);
        s_x[P((uint32_t)t) + (uint32_t)k * (NT + NT / E)] = i < n ? p[i] : ~0ull;
    }
    __syncthreads();
    // ranges of depth bits and ids
    uint32_t zmin = 0xffffffffu, zmax = 0u, imin = 0xffffffffu, imax = 0u;
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const unsigned long long u = s_x[t * (E + 1) + r];
        x[r] = u;
        if ((uint32_t)(t * E + r) < n) {
            const uint32_t z = (uint32_t)(u >> 32), id = (uint32_t)u;
            zmin = z < zmin ? z : zmin;
            zmax = z > zmax ? z : zmax;
            imin = id < imin ? id : imin;
            imax = id > imax ? id : imax;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t a1 = __shfl_xor(zmin, off, 64), a2 = __shfl_xor(zmax, off, 64);
        const uint32_t a3 = __shfl_xor(imin, off, 64), a4 = __shfl_xor(imax, off, 64);
        zmin = a1 < zmin ? a1 : zmin;
        zmax = a2 > zmax ? a2 : zmax;
        imin = a3 < imin ? a3 : imin;
        imax = a4 > imax ? a4 : imax;
    }
    if (lane == 0) {
        s_w[4 * wave + 0] = zmin;
        s_w[4 * wave + 1] = zmax;
        s_w[4 * wave + 2] = imin;
        s_w[4 * wave + 3] = imax;
    }
    if (t == 0) s_long = 0u;
    __syncthreads();
#pragma unroll 1
    for (int i = 0; i < NW; ++i) {
        zmin = s_w[4 * i + 0] < zmin ? s_w[4 * i + 0] : zmin;
        zmax = s_w[4 * i + 1] > zmax ? s_w[4 * i + 1] : zmax;
        imin = s_w[4 * i + 2] < imin ? s_w[4 * i + 2] : imin;
        imax = s_w[4 * i + 3] > imax ? s_w[4 * i + 3] : imax;
    }
    __syncthreads();  // s_w is reused by the passes
    const uint32_t zr = zmax - zmin, ir = imax - imin;
    const int zb = zr ? 32 - __clz((int)zr) : 0;
    const int ib = ir ? 32 - __clz((int)ir) : 0;
    const int TB = zb + ib;
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const uint32_t z = (uint32_t)(x[r] >> 32), id = (uint32_t)x[r];
        x[r] = (uint32_t)(t * E + r) < n ? ((unsigned long long)(z - zmin) << ib) | (unsigned long long)(id - imin)
                                          : ~0ull;
    }
    const int sh0 = TB > 16 ? TB - 16 : 0;
    for (int sh = sh0; sh < TB; sh += 4) pass(sh);
    // a run of more than 64 equal top words: sort by every bit instead
    bool lng = false;
#pragma unroll 1
    for (uint32_t i = t; i + 64 < n; i += NT) lng |= (s_x[P(i)] >> sh0) == (s_x[P(i + 64)] >> sh0);
    if (__any(lng) && lane == 0) s_long = 1u;
    __syncthreads();
    const bool full = s_long != 0u;
    if (full)
        for (int sh = 0; sh < TB; sh += 4) pass(sh);
    const int shr = full ? 0 : sh0;
#pragma unroll 1
    for (uint32_t i = t; i < n; i += NT) {
        const unsigned long long u = s_x[P(i)];
        const unsigned long long top = u >> shr;
        uint32_t pos = i;
        const bool prev = i > 0 && (s_x[P(i - 1)] >> shr) == top;
        const bool next = i + 1 < n && (s_x[P(i + 1)] >> shr) == top;
        if (prev || next) {  // inside a run: place by the number of smaller words
            uint32_t b = i, e = i + 1;
            while (b > 0 && (s_x[P(b - 1)] >> shr) == top) --b;
            while (e < n && (s_x[P(e)] >> shr) == top) ++e;
            uint32_t rank = 0;
            for (uint32_t j = b; j < e; ++j) rank += s_x[P(j)] < u ? 1u : 0u;
            pos = b + rank;
        }
        const uint32_t z = (uint32_t)(u >> ib) + zmin;
        const uint32_t id = (uint32_t)(u & ((1ull << ib) - 1ull)) + imin;
        p[pos] = ((unsigned long long)z << 32) | (unsigned long long)id;
    }
    __syncthreads();
}

// one block per tile of the class, lists of at most NT * E entries
template <int NT, int E>
__global__ __launch_bounds__(NT) void k_sort_radix(FwdArgs a, int cls, const Status* __restrict__ status,
                                                   const uint32_t* __restrict__ cls_list,
                                                   const uint32_t* __restrict__ starts) {
    __shared__ unsigned long long s_x[NT * E + NT];
    __shared__ uint16_t s_cnt[18 * NT];
    __shared__ uint32_t s_w[4 * (NT / 64)];
    __shared__ uint32_t s_long;
    const uint32_t count = status->cls[cls];
    for (uint32_t w = blockIdx.x; w < count; w += gridDim.x) {
        const uint32_t tile = cls_list[(size_t)cls * a.tiles + w];
        const uint32_t st = starts[tile], n = starts[tile + 1] - st;
        sort_list<NT, E>(a.pairs + st, n, s_x, s_cnt, s_w, &s_long);
    }
}

// Lists longer than one LDS sort (class kSortBig) are cut into chunks of CH entries.  Every
// (tile, chunk) is a work item of the grid, so long lists use many CUs at once:
//   k_sort_chunks   sorts each chunk in LDS (the same routine as the single-block classes);
//   k_merge_chunks  places each element of a chunk at its rank in the whole list: its index
//                   in its own chunk plus, for every other chunk of the tile (staged in LDS),
//                   the number of smaller keys there (keys are unique); writes pairs_alt;
//   k_copy_chunks   copies the merged lists back.
// The item count uses the longest list of the render (max_tile) as the chunk bound.
__device__ inline uint32_t big_chunks(const Status* __restrict__ status, uint32_t ch) {
    return (status->max_tile + ch - 1) / ch;
}

template <int NT, int E>
__global__ __launch_bounds__(NT) void k_sort_chunks(FwdArgs a, const Status* __restrict__ status,
                                                    const uint32_t* __restrict__ cls_list,
                                                    const uint32_t* __restrict__ starts) {
    constexpr uint32_t CH = NT * E;
    __shared__ unsigned long long s_x[NT * E + NT];
    __shared__ uint16_t s_cnt[18 * NT];
    __shared__ uint32_t s_w[4 * (NT / 64)];
    __shared__ uint32_t s_long;
    const uint32_t mc = big_chunks(status, CH);
    const uint32_t items = status->cls[kSortBig] * mc;
    for (uint32_t it = blockIdx.x; it < items; it += gridDim.x) {
        const uint32_t w = it / mc, c = it - w * mc;
        const uint32_t tile = cls_list[(size_t)kSortBig * a.tiles + w];
        const uint32_t st = starts[tile], n = starts[tile + 1] - st;
        if (c * CH >= n) continue;
        sort_list<NT, E>(a.pairs + st + c * CH, (n - c * CH < CH) ? n - c * CH : CH, s_x, s_cnt, s_w, &s_long);
    }
}

template <int NT, int E>
__global__ __launch_bounds__(NT) void k_merge_chunks(FwdArgs a, const Status* __restrict__ status,
                                                     const uint32_t* __restrict__ cls_list,
                                                     const uint32_t* __restrict__ starts) {
    constexpr uint32_t CH = NT * E;
    __shared__ unsigned long long s_o[CH];
    const uint32_t mc = big_chunks(status, CH);
    const uint32_t items = status->cls[kSortBig] * mc;
    for (uint32_t it = blockIdx.x; it < items; it += gridDim.x) {
        const uint32_t w = it / mc, c = it - w * mc;
        const uint32_t tile = cls_list[(size_t)kSortBig * a.tiles + w];
        const uint32_t st = starts[tile], n = starts[tile + 1] - st;
        if (c * CH >= n) continue;
        const uint32_t nc = (n + CH - 1) / CH;
        const uint32_t len = (n - c * CH < CH) ? n - c * CH : CH;
        const unsigned long long* src = a.pairs + st;
        unsigned long long x[E];
        uint32_t pos[E];
#pragma unroll
        for (int k = 0; k < E; ++k) {
            const uint32_t i = threadIdx.x + (uint32_t)k * NT;
            x[k] = i < len ? src[c * CH + i] : 0ull;
            pos[k] = i;  // rank within its own (sorted) chunk
        }
        for (uint32_t o = 0; o < nc; ++o) {
            if (o == c) continue;
            const uint32_t lo = (n - o * CH < CH) ? n - o * CH : CH;
            __syncthreads();
            for (uint32_t i = threadIdx.x; i < lo; i += NT) s_o[i] = src[o * CH + i];
            __syncthreads();
#pragma unroll
            for (int k = 0; k < E; ++k) {
                uint32_t l = 0, h = lo;  // keys of chunk o smaller than x[k]
                while (l < h) {
                    const uint32_t m = (l + h) >> 1;
                    if (s_o[m] < x[k]) l = m + 1; else h = m;
                }
                pos[k] += l;
            }
        }
#pragma unroll
        for (int k = 0; k < E; ++k) {
            const uint32_t i = threadIdx.x + (uint32_t)k * NT;
            if (i < len) a.pairs_alt[st + pos[k]] = x[k];
        }
        __syncthreads();
    }
}

template <int NT, int E>
__global__ __launch_bounds__(NT) void k_copy_chunks(FwdArgs a, const Status* __restrict__ status,
                                                    const uint32_t* __restrict__ cls_list,
                                                    const uint32_t* __restrict__ starts) {
    constexpr uint32_t CH = NT * E;
    const uint32_t mc = big_chunks(status, CH);
    const uint32_t items = status->cls[kSortBig] * mc;
    for (uint32_t it = blockIdx.x; it < items; it += gridDim.x) {
        const uint32_t w = it / mc, c = it - w * mc;
        const uint32_t tile = cls_list[(size_t)kSortBig * a.tiles + w];
        const uint32_t st = starts[tile], n = starts[tile + 1] - st;
        if (c * CH >= n) continue;
        const uint32_t len = (n - c * CH < CH) ? n - c * CH : CH;
        for (uint32_t i = threadIdx.x; i < len; i += NT) a.pairs[st + c * CH + i] = a.pairs_alt[st + c * CH + i];
    }
}

// --------------------------------------------------------------------------------------------
// front-to-back compositing.  One tile per block, one sub-tile per wavefront; each lane shades
// PPT pixels of one column, sharing the LDS reads and the dx terms.  List entries are staged
// in LDS per batch with the conic pre-scaled, so that for a pixel offset (dx, dy)
//   q = A' dx^2 + B' dx dy + C' dy^2 + log2(o),   A' = -1/2 log2(e) A, B' = -log2(e) B,
//   C' = -1/2 log2(e) C,   alpha = min(0.99, exp2(q)) = min(0.99, o G).
// Per pixel: skip if alpha < 1/255; stop (without blending) if T (1 - alpha) < 1e-4; else
// C += alpha T c, D += alpha T z, T *= 1 - alpha.  rgb = C + T bg, depth = D, alpha = 1 - T.
// Each batch of the list is culled against the wavefront's sub-tile and compacted (in list
// order) before the pixel loop; the loop is predicated (after the cull nearly every entry
// reaches some pixel of the sub-tile, so a per-entry wavefront skip costs more than it saves)
// and the wavefront leaves the list as soon as none of its pixels is live.
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
    // the wavefront's pixel-centre rectangle
    const float rx0 = (float)(tx * TW + sx * ST::SW) + 0.5f, rx1 = rx0 + (float)(ST::SW - 1);
    const float ry0 = (float)(ty * TH + sy * ST::SH) + 0.5f, ry1 = ry0 + (float)(ST::SH - 1);
    for (uint32_t base = start; base < end; base += 64) {
        bool any = false;
#pragma unroll
        for (int p = 0; p < PPT; ++p) any |= T[p] > 0.0f;
        if (!__any(any)) break;
        // stage the batch's entries that can reach this sub-tile, compacted in list order
        const uint32_t j = base + lane;
        Record R;
        bool keep = false;
        if (j < end) {
            const uint32_t gid = (uint32_t)a.pairs[j];
            if (gid - ev.gid_base < ev.n) {
                R = a.records[rec_off + gid];
                keep = reaches_rect(R, rx0, rx1, ry0, ry1, qcut);
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
        // the wavefront's LDS writes are visible to its own later reads
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int n = __popcll(km);
        for (int k = 0; k < n; ++k) {
            if ((k & 3) == 0) {
                bool wl = false;
#pragma unroll
                for (int p = 0; p < PPT; ++p) wl |= T[p] > 0.0f;
                if (!__any(wl)) break;
            }
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
                if (COUNT) evals[p] += T[p] > 0.0f ? 1u : 0u;
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
        a.rgb[3 * q + 0] = fmaf(Tf, cm.bg[0], Cr[p]);
        a.rgb[3 * q + 1] = fmaf(Tf, cm.bg[1], Cg[p]);
        a.rgb[3 * q + 2] = fmaf(Tf, cm.bg[2], Cb[p]);
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
                                                                              const Env* __restrict__ envs) {
    constexpr int NW = SubTile<TW, TH, PPT>::WAVES;
    __shared__ float4 s0[NW][64], s1[NW][64];
    __shared__ float4 s2[NW][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    composite_sub<TW, TH, PPT, SAVE, COUNT>(a, xcd_tile(blockIdx.x, a.tiles), wave, lane, s0[wave], s1[wave], s2[wave],
                                            starts, envs);
}

// persistent grid: block b takes queue items b, b + G, b + 2G, ... of the longest-first queue
// (sort classes from the longest lists down, then the lists of at most one entry).  A static
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
        int cls = kSortBig;
        while (cls >= 0 && k >= cnt[cls]) {
            k -= cnt[cls];
            --cls;
        }
        if (cls < 0) cls = kSortNone;
        composite_sub<TW, TH, PPT, SAVE, COUNT>(a, (long long)cls_list[(size_t)cls * a.tiles + k], wave, lane, s0[wave],
                                                s1[wave], s2[wave], starts, envs);
    }
}

__global__ void k_copy_pairs(FwdArgs a, uint64_t* keys, uint32_t* vals, uint32_t* ranges) {
    const long long t = blockIdx.x;
    const uint32_t s = a.starts[t], e = a.starts[t + 1];
    if (threadIdx.x == 0) {
        ranges[2 * t] = s;
        ranges[2 * t + 1] = e;
    }
    for (uint32_t i = s + threadIdx.x; i < e; i += blockDim.x) {
        const unsigned long long u = a.pairs[i];
        keys[i] = ((unsigned long long)t << 32) | (u >> 32);
        vals[i] = (uint32_t)u;
    }
}

// --------------------------------------------------------------------------------------------
// launch sequence
// --------------------------------------------------------------------------------------------
template <int L>
static hipError_t launch_project(const FwdArgs& a, hipStream_t s) {
    const int gsz = (a.tiles_x + 1) * (a.tiles_y + 1);
    const size_t lds = (size_t)a.C * (gsz + 1) * sizeof(int);
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
                           a.envs);
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

static int g_num_cu = 0;

hipError_t launch_forward(const FwdArgs& a, hipStream_t s) {
    if (g_num_cu == 0) {
        int dev = 0;
        hipGetDevice(&dev);
        hipDeviceGetAttribute(&g_num_cu, hipDeviceAttributeMultiprocessorCount, dev);
        if (g_num_cu <= 0) g_num_cu = 256;
    }
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
    hipLaunchKernelGGL(k_tile_offsets, dim3((unsigned)((a.tiles + 255) / 256)), dim3(256), 0, s, a);
    mark(3);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, a);
    mark(4);
    if (a.n_supers > 0)
        hipLaunchKernelGGL(k_emit, dim3(a.n_supers, a.C), dim3(kBlock), (size_t)a.tpi * sizeof(uint32_t), s, a,
                           a.supers, a.sbvis);
    mark(5);
    hipLaunchKernelGGL(k_classify, dim3((unsigned)((a.tiles + 255) / 256)), dim3(256), 0, s, a);
    mark(6);
    hipLaunchKernelGGL((k_sort_radix<64, 8>), dim3(g_num_cu * 32), dim3(64), 0, s, a, 0, a.status, a.cls_list, a.starts);
    hipLaunchKernelGGL((k_sort_radix<128, 8>), dim3(g_num_cu * 16), dim3(128), 0, s, a, 1, a.status, a.cls_list, a.starts);
    hipLaunchKernelGGL((k_sort_radix<256, 8>), dim3(g_num_cu * 8), dim3(256), 0, s, a, 2, a.status, a.cls_list, a.starts);
    mark(7);
    hipLaunchKernelGGL((k_sort_radix<512, 8>), dim3(g_num_cu * 4), dim3(512), 0, s, a, 3, a.status, a.cls_list, a.starts);
    hipLaunchKernelGGL((k_sort_radix<1024, 8>), dim3(g_num_cu * 2), dim3(1024), 0, s, a, 4, a.status, a.cls_list, a.starts);
    mark(8);
    hipLaunchKernelGGL((k_sort_chunks<1024, 8>), dim3(g_num_cu * 2), dim3(1024), 0, s, a, a.status, a.cls_list, a.starts);
    hipLaunchKernelGGL((k_merge_chunks<1024, 8>), dim3(g_num_cu * 2), dim3(1024), 0, s, a, a.status, a.cls_list, a.starts);
    hipLaunchKernelGGL((k_copy_chunks<1024, 8>), dim3(g_num_cu * 2), dim3(1024), 0, s, a, a.status, a.cls_list, a.starts);
    mark(9);
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
    mark(10);
    return hipGetLastError();
}

hipError_t launch_copy_pairs(const FwdArgs& a, uint64_t* keys, uint32_t* values, uint32_t* ranges, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_pairs, dim3((unsigned)a.tiles), dim3(256), 0, s, a, keys, values, ranges);
    return hipGetLastError();
}

}  // namespace gsr
