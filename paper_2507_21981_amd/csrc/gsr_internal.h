// Internal device-side tables and kernel launchers of the gfx950 renderer.
// Shared only between the library's own translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gsr.h"

namespace gsr {

constexpr int kBlock = 256;          // Gaussians per projection block (one chunk)
// Tile-length classes: classes 0 .. 4 hold tiles with at most 512, 1024, ..., 8192 pairs,
// class kLenLong longer lists, class kLenNone tiles with at most one pair (and overflowed
// tiles).  They order the persistent compositor's queue, longest lists first.
constexpr int kLenClasses = 5;
constexpr int kLenLong = 5;
constexpr int kLenNone = 6;
constexpr int kNumClasses = 7;
constexpr int kLdsHistLimit = 40000; // int counters of one image's tile difference grid in LDS
// Depth sort and emission: each image's visible Gaussians occupy a segment of the sort buffers
// made of radix chunks of kSortTile items; tile counts and emission work on chunks of the
// depth-ordered Gaussians holding about the same number of pairs.  An image has at most
// kMaxTilesPerImage tiles: the emission keeps 12 bytes per tile in LDS (160 KB per block on
// gfx950).
constexpr int kSortTile = 2048;
constexpr int kPairBlock = 1024;     // positions per block of the pair-prefix kernels
constexpr int kSegChunks = 16;       // emission chunks per segment of the tile-range scan
constexpr int kChunkPairsPerTile = 6; // emission chunk size: pairs per tile of the image
constexpr int kEmitQueueStride = 64;  // u32 between the per-XCD emission counters (own lines)
constexpr int kEmitLdsSmall = 8192;   // emission tile table (bytes) above which blocks have 16 wavefronts
constexpr int kMaxTilesPerImage = 13312;

// One (node, camera) view: the camera<-node map composed in FP64 and rounded
// once to FP32, the camera centre in node-local coordinates, intrinsics and
// the J-clamp limits.  96 bytes.
struct View {
    float W[9];
    float w[3];
    float cl[3];
    float fx, fy, cx, cy, znear, limx, limy;
    float pad[2];
};

struct Node {
    const float* means;
    const float* scales;
    const float* quats;
    const float* opac;
    const float* sh;
    uint32_t gid_base;  // scene-global id of the node's first Gaussian
    uint32_t n;
    int32_t env;
    int32_t block_begin;  // the node's first chunk in the block table (its chunks are contiguous)
};

struct Env {
    uint32_t gid_base;  // scene-global id of the env's first Gaussian
    uint32_t n;         // Gaussians in the env
    int32_t node_begin, node_end;
    int32_t sb_begin, sb_count;  // the env's super-blocks
};

// A chunk of at most kBlock consecutive Gaussians of one node.
struct Block {
    int32_t node;
    int32_t env;
    uint32_t gid0;
    uint32_t count;
};

// Consecutive chunks of one env processed by one projection / emission block, so that the
// block's per-tile pair counts cover many Gaussians.
struct Super {
    int32_t env;
    int32_t chunk_begin, chunk_end;
    int32_t pad;
};

constexpr int kMaxChunksPerSuper = 16;
static_assert(kSortTile % kPairBlock == 0, "pair-prefix blocks tile the radix chunks");

constexpr int kParts = 64;

struct Status {
    uint32_t flags;
    uint32_t nonfinite;
    unsigned long long pairs;
    uint32_t max_tile;
    uint32_t cls[8];      // tile counts per length class
    uint32_t pad[6];
    // counters summed on the host over kParts slots (block b adds into slot b % kParts): a
    // single address taking an atomic from every wavefront serialises the grid
    unsigned long long visible[kParts];      // visible (image, Gaussian) records
    unsigned long long visible_any[kParts];  // Gaussians visible in at least one camera
    unsigned long long evals[kParts];        // Gaussian-pixel evaluations of the compositor
};

constexpr int kStages = 9;  // views, project, gather, depth_sort, chunks, tile_counts, tile_ranges,
                            // emit, composite

// Projected record of one (image, Gaussian): r0 = (u, v, opacity, z),
// r1 = (A, B, C, log2 opacity) with (A, B, C) the conic (inverse dilated 2D covariance),
// r2 = (r, g, b, D) SH colour and D the determinant of the dilated 2D covariance (so that
// the covariance entries are recovered without cancellation: Sxx = C D, Syy = A D).  48 bytes.
struct Record {
    float4 r0, r1, r2;
};

// Whether a projected entry can pass the skip test q >= qcut at some pixel centre of the
// rectangle [x0, x1] x [y0, y1].  With m(d) = A dx^2 + 2 B dx dy + C dy^2 (the conic's form),
// q = log2(o) - m log2(e) / 2, so the test is m <= rho2 = 2 ln 2 (log2(o) - qcut).  The minimum
// of m over the rectangle is 0 when the mean lies inside; otherwise it lies on an edge that
// faces the mean, where m is minimised in closed form along the edge and clamped to it.  Each
// candidate is evaluated as a sum of two non-negative squares (completing the square, with
// the covariance entries C D and A D), which has no cancellation.  The slack covers the
// rounding of that evaluation and of the compositor's own FP32 evaluation of q, whose error
// grows with the magnitude of the form's terms over the rectangle (tmax); it is hundreds of
// times the error of the hardware reciprocal (about 1 ulp), which therefore stands in for the
// four divisions.  Entries that fail the test change no pixel, so dropping them leaves the
// result bit-identical.
__device__ inline bool reaches_rect(const Record& R, float x0, float x1, float y0, float y1, float qcut) {
    const float u = R.r0.x, v = R.r0.y, A = R.r1.x, B = R.r1.y, C = R.r1.z, lo = R.r1.w, D = R.r2.w;
    const float rho2 = 1.3862943611198906f * (lo - qcut);
    if (!(rho2 > 0.0f)) return false;
    const float gx = fmaxf(fmaxf(x0 - u, u - x1), 0.0f);
    const float gy = fmaxf(fmaxf(y0 - v, v - y1), 0.0f);
    if (gx == 0.0f && gy == 0.0f) return true;
    const float Dx = fmaxf(fabsf(x0 - u), fabsf(x1 - u)), Dy = fmaxf(fabsf(y0 - v), fabsf(y1 - v));
    const float tmax = A * Dx * Dx + 2.0f * fabsf(B) * Dx * Dy + C * Dy * Dy + fabsf(lo);
    const float slack = 4e-6f * tmax + 1e-4f * rho2 + 1e-3f;
    float mmin = INFINITY;
    if (gx > 0.0f) {  // the facing vertical edge
        const float dx = u < x0 ? x0 - u : x1 - u;
        const float bc = B * __builtin_amdgcn_rcpf(C);
        const float dy = fminf(fmaxf(-bc * dx, y0 - v), y1 - v);
        const float t = dy + bc * dx;
        mmin = C * t * t + dx * dx * __builtin_amdgcn_rcpf(C * D);
    }
    if (gy > 0.0f) {  // the facing horizontal edge
        const float dy = v < y0 ? y0 - v : y1 - v;
        const float ba = B * __builtin_amdgcn_rcpf(A);
        const float dx = fminf(fmaxf(-ba * dy, x0 - u), x1 - u);
        const float t = dx + ba * dy;
        mmin = fminf(mmin, A * t * t + dy * dy * __builtin_amdgcn_rcpf(A * D));
    }
    return mmin <= rho2 + slack;
}

// The scene's per-node arrays are reached through pointers stored in tables, which the
// compiler must treat as generic (flat) addresses.  Flat loads count on the same wait counter
// as scalar and LDS loads, so every wait for a table entry would also wait for the node data
// in flight; reading through a global address-space pointer keeps them apart.
template <class T>
__device__ inline const __attribute__((address_space(1))) T* global_ptr(const T* p) {
    return (const __attribute__((address_space(1))) T*)p;
}

// Workgroups are handed to the chip's 8 XCDs (each with its own L2) in turn, so block b runs
// on XCD b % 8.  Mapping block b to tile (b % 8) Q + b / 8 (Q = tiles / 8; the last tiles % 8
// blocks map to themselves) gives each XCD a contiguous run of tiles: neighbouring tiles, which
// gather the same Gaussians' records, then share an L2.
__device__ inline long long xcd_tile(long long b, long long tiles) {
    const long long q = tiles >> 3;
    return b < (q << 3) ? (b & 7) * q + (b >> 3) : b;
}

// v + (v of another lane) by a DPP move (ctrl selects the source lane; lanes whose source is
// outside their row, and rows outside row_mask, add zero)
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_add_u32(uint32_t v) {
    return v + (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xF, false);
}
// Inclusive prefix sum over the wavefront's 64 lanes with DPP moves only (no LDS crossbar):
// shifts by 1, 2, 4, 8 within rows of 16 lanes, then lane 15 of rows 0 and 2 into rows 1 and
// 3, then lane 31 into rows 2 and 3.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    v = dpp_add_u32<0x111, 0xF>(v);  // row_shr:1
    v = dpp_add_u32<0x112, 0xF>(v);  // row_shr:2
    v = dpp_add_u32<0x114, 0xF>(v);  // row_shr:4
    v = dpp_add_u32<0x118, 0xF>(v);  // row_shr:8
    v = dpp_add_u32<0x142, 0xA>(v);  // row_bcast:15
    v = dpp_add_u32<0x143, 0xC>(v);  // row_bcast:31
    return v;
}

// Grid-stride split for kernels whose neighbouring work items write the same cache lines:
// block b runs on XCD b % 8 and takes items of that XCD's contiguous eighth of [0, n), so the
// lines are assembled in one L2 instead of being written back in pieces from several.  The
// grid must be a multiple of 8.
__device__ inline void xcd_items(uint32_t n, uint32_t& first, uint32_t& last, uint32_t& step) {
    const uint32_t x = blockIdx.x & 7u;
    first = (uint32_t)(((unsigned long long)n * x) >> 3) + (blockIdx.x >> 3);
    last = (uint32_t)(((unsigned long long)n * (x + 1u)) >> 3);
    step = gridDim.x >> 3;
}

struct FwdArgs {
    // scene
    const Node* nodes;
    const Env* envs;
    const Block* blocks;
    int n_blocks;
    const Super* supers;
    int n_supers;
    int n_nodes;
    int sh_degree;
    const gsr_pose* poses;
    // cameras / images
    const gsr_camera* cams;
    int C;          // cameras per env
    int images;
    int width, height;
    int tw, th, tiles_x, tiles_y, tpi;  // tile shape, tiles per image
    long long tiles;                     // images * tpi
    // workspace
    View* views;
    Record* records;
    uint4* vis;          // per (super-block, camera): the visible Gaussians in id order,
                         //   {x0 | y0 << 16, x1 | y1 << 16, z bits, Gaussian id}
    uint32_t* sbvis;     // per (super-block, camera): length of that list
    uint32_t* loff;      // per (super-block, camera): the list's first position in the sort buffers
    int sb_cap;          // list capacity per (super-block, camera)
    // depth sort (two ping-pong buffers; the last pass leaves the result in buffer 1)
    uint32_t* skey[2];   // z bits (ping-pong between the passes)
    uint32_t* ssrc[2];   // the item's position in the gathered (id-ordered) segment (ping-pong)
    uint32_t* sgid[2];   // Gaussian id: [0] gathered, [1] sorted
    uint2* srect[2];     // tile rectangle {x0 | y0 << 16, x1 | y1 << 16}: [0] gathered, [1] sorted
    uint32_t* hist;      // per radix chunk (pass 0: per list): 256 digit counts, then first slots
    uint32_t* seg_n;     // per image: visible Gaussians (the length of its segment)
    uint32_t* seg_start; // per image + 1: first position of its segment (kSortTile multiples)
    int sort_chunks;     // radix chunks the sort buffers can hold
    uint32_t* blk_pairs; // per kPairBlock positions of the sorted buffer: pairs, then the
                         //   image's pairs before the block
    uint32_t* chunk_base;  // per image + 1: first emission chunk of the image
    uint32_t* pair_base; // per image: pairs of the earlier images (its first bucket slot)
    uint32_t* cstart;    // per emission chunk: first position of its Gaussians
    uint32_t* cimg;      // per emission chunk: its image
    int chunk_cap;       // emission chunks the workspace holds
    int chunk_pairs;     // pairs per emission chunk (a chunk starts at every multiple)
    uint32_t* ecnt;      // per (emission chunk, tile): pairs, then the chunk's pairs of the tile
                         //   before it within its segment (kSegChunks chunks of one image)
    uint32_t* emit_next; // per XCD (at a stride of kEmitQueueStride): emission chunks taken
    uint32_t* seg_base;  // per image + 1: first segment of the image
    uint32_t* segoff;    // per (segment, tile): pairs, then the segment's first slot in the
                         //   tile's bucket
    int num_cu;          // compute units (grid sizes of the grid-stride kernels)
    uint32_t* starts;    // per tile + 1
    uint32_t* cls_list;  // kNumClasses lists of `tiles` entries
    uint32_t* pairs;     // per tile bucket slot: the Gaussian id, buckets in depth order
    long long pair_cap;
    Status* status;
    // outputs
    float* rgb;
    float* depth;
    float* alpha;
    float* T_final;
    uint32_t* n_contrib;
    int persistent;
    int persistent_grid;
    const gsr_augment* aug;  // per image, applied to rgb in the compositor's epilogue, or null
    const float* overlay;    // overlay frames [images][H][W][3] for aug, or null
    int ppt;   // pixels per compositor thread (1 or 2; 8x8 tiles use 1)
    int save;  // write per-pixel T_final and contributor counts for the backward
    int count; // count Gaussian-pixel evaluations into the status word
    hipEvent_t* stage_events;  // kStages + 1 events recorded between stages, or null
};

// Image-space domain randomisation of one pixel (the colour as rendered, background
// included): clamp to [0, 1], blend with the overlay pixel ov (null: none), hexcone HSV with
// the hue shifted modulo one turn and saturation and value scaled and clamped, back to RGB,
// then each channel to the power gamma.  Pixel values only, so the hardware log2 / exp2
// (about 1 ulp) serve for the power.
__device__ inline float3 augment_pixel(float r, float g, float b, const gsr_augment& p, const float* ov) {
    r = fminf(fmaxf(r, 0.0f), 1.0f);
    g = fminf(fmaxf(g, 0.0f), 1.0f);
    b = fminf(fmaxf(b, 0.0f), 1.0f);
    if (ov) {
        const float l = p.overlay_weight, k = 1.0f - l;
        r = fmaf(l, fminf(fmaxf(ov[0], 0.0f), 1.0f), k * r);
        g = fmaf(l, fminf(fmaxf(ov[1], 0.0f), 1.0f), k * g);
        b = fmaf(l, fminf(fmaxf(ov[2], 0.0f), 1.0f), k * b);
    }
    const float v = fmaxf(r, fmaxf(g, b)), m = fminf(r, fminf(g, b)), c = v - m;
    const float s = v > 0.0f ? c / v : 0.0f;
    float h6 = 0.0f;  // hue in sixths of a turn
    if (c > 0.0f) {
        if (v == r) {
            h6 = (g - b) / c;
            if (h6 < 0.0f) h6 += 6.0f;
        } else if (v == g) {
            h6 = (b - r) / c + 2.0f;
        } else {
            h6 = (r - g) / c + 4.0f;
        }
    }
    float h = fmaf(h6, 1.0f / 6.0f, p.hue_shift);
    h -= floorf(h);
    const float s2 = fminf(fmaxf(s * p.saturation_scale, 0.0f), 1.0f);
    const float v2 = fminf(fmaxf(v * p.value_scale, 0.0f), 1.0f);
    float H = h * 6.0f;
    if (H >= 6.0f) H = 0.0f;
    const float c2 = v2 * s2;
    const float x2 = c2 * (1.0f - fabsf(H - 2.0f * floorf(0.5f * H) - 1.0f));
    const float m2 = v2 - c2;
    const int sector = (int)H;
    float r2, g2, b2;
    switch (sector) {
        case 0: r2 = c2; g2 = x2; b2 = 0.0f; break;
        case 1: r2 = x2; g2 = c2; b2 = 0.0f; break;
        case 2: r2 = 0.0f; g2 = c2; b2 = x2; break;
        case 3: r2 = 0.0f; g2 = x2; b2 = c2; break;
        case 4: r2 = x2; g2 = 0.0f; b2 = c2; break;
        default: r2 = c2; g2 = 0.0f; b2 = x2; break;
    }
    r2 += m2;
    g2 += m2;
    b2 += m2;
    const float gm = p.gamma;
    r2 = r2 > 0.0f ? __builtin_amdgcn_exp2f(gm * __builtin_amdgcn_logf(r2)) : 0.0f;
    g2 = g2 > 0.0f ? __builtin_amdgcn_exp2f(gm * __builtin_amdgcn_logf(g2)) : 0.0f;
    b2 = b2 > 0.0f ? __builtin_amdgcn_exp2f(gm * __builtin_amdgcn_logf(b2)) : 0.0f;
    return make_float3(r2, g2, b2);
}

struct BwdArgs {
    FwdArgs f;
    const float* d_rgb;
    const float* d_depth;
    const float* d_alpha;
    float* g2d;          // per (image, Gaussian) record gradients, 12 floats
    const gsr_gaussian_grads* grads_dev;  // per node, device copy
    float* pose_part;    // per projection block: 8 floats, its Gaussians' pose-gradient sums (A, B)
    float* d_poses;      // per node: 6 floats (omega, rho), accumulated; null = not requested
};

// forward stages
hipError_t launch_forward(const FwdArgs& a, hipStream_t s);
// raise the dynamic LDS limit of the kernels whose LDS grows with the tile grid (host side,
// before launches or graph capture)
hipError_t forward_lds_limits(const FwdArgs& a);
hipError_t launch_augment(int images, int width, int height, const float* rgb, const float* overlay,
                          const gsr_augment* params, float* out, int num_cu, hipStream_t s);
hipError_t launch_mesh_to_gs(long long n_faces, long long n_verts, const float* verts, const float* colours,
                             const int32_t* faces, float flatten, float opacity, int K, const gsr_gaussian_grads& out,
                             uint32_t* bad, int num_cu, hipStream_t s);
// LiDAR: per-node bounding-volume hierarchies of a scene and the ray tracer
struct LidarScene;
}  // namespace gsr
#include <string>
#include <vector>
namespace gsr {
std::string lidar_build(const std::vector<Node>& nodes, LidarScene** out);
void lidar_free(LidarScene* L);
size_t lidar_bytes(const LidarScene* L);
hipError_t launch_lidar(const LidarScene* L, const Env* envs, const gsr_pose* poses, int n_envs, int rays_per_env,
                        const gsr_ray* rays, float* range, float* alpha, uint32_t* hits, hipStream_t s);
hipError_t launch_copy_pairs(const FwdArgs& a, uint64_t* keys, uint32_t* values, uint32_t* ranges, hipStream_t s);
// backward stages
hipError_t launch_backward(const BwdArgs& a, size_t n_records, hipStream_t s);
// copy n host gradient descriptors to the device table through kernel arguments
hipError_t launch_set_grads(const gsr_gaussian_grads* host, int n, gsr_gaussian_grads* dev, hipStream_t s);

}  // namespace gsr
