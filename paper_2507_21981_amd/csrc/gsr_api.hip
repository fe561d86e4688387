// Host side of the renderer's C ABI: contexts, scene composition, workspace, status,
// hipGraph capture and the autotuner.  See include/gsr.h for the contract of each call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "gsr_internal.h"

using namespace gsr;

namespace {

std::string g_err = "no error";

template <typename T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    void release() {
        if (p) hipFree(p);
        p = nullptr;
        n = 0;
    }
};

struct GraphKey {
    const gsr_scene* scene;
    const void* cams;
    const void* rgb;
    const void* depth;
    const void* alpha;
    int C, W, H, tw, th, persistent, ppt;
    uint32_t flags;
    hipStream_t stream;
    long long pair_cap;
    const void* aug;
    const void* overlay;
    bool operator==(const GraphKey& o) const {
        return scene == o.scene && cams == o.cams && rgb == o.rgb && depth == o.depth && alpha == o.alpha &&
               aug == o.aug && overlay == o.overlay &&
               C == o.C && W == o.W && H == o.H && tw == o.tw && th == o.th && persistent == o.persistent &&
               ppt == o.ppt &&
               flags == o.flags && stream == o.stream && pair_cap == o.pair_cap;
    }
};

constexpr int kMaxGroups = 4;  // stream groups of a render (gsr_set_stream_groups)

}  // namespace

struct gsr_scene {
    gsr_context* ctx = nullptr;
    int n_envs = 0, n_nodes = 0, sh_degree = 0;
    long long total = 0;
    std::vector<int32_t> env_offsets;
    std::vector<Node> nodes_h;
    std::vector<Env> envs_h;
    std::vector<Block> blocks_h;
    std::vector<Super> supers_h;
    Node* nodes_d = nullptr;
    Env* envs_d = nullptr;
    Block* blocks_d = nullptr;
    Super* supers_d = nullptr;
    const gsr_pose* poses = nullptr;
    uint64_t version = 0;
    int sb_cap = kBlock;  // Gaussians per super-block at most
    LidarScene* lidar = nullptr;  // per-node hierarchies of the LiDAR tracer (gsr_lidar_build)
    uint64_t lidar_version = 0;   // scene version they were built for
    // grouped renders: one scene per group of environments [sub_env[g], sub_env[g + 1]),
    // composed on the owning context's sub-context g for scene version sub_version
    gsr_scene* sub[kMaxGroups] = {};
    int sub_groups = 0;
    int sub_env[kMaxGroups + 1] = {};
    uint64_t sub_version = 0;
};

struct gsr_context {
    int device = 0;
    int num_cu = 256;
    gsr_config cfg{};
    std::string err = "no error";
    Status* d_status = nullptr;
    Status* h_status = nullptr;  // pinned
    DevBuf<uint32_t> pairs;
    long long pair_cap = 0;
    DevBuf<Record> records;
    DevBuf<uint4> vis;
    DevBuf<uint32_t> sbvis, loff;
    DevBuf<uint32_t> skey0, skey1, ssrc0, ssrc1, sgid0, sgid1;
    DevBuf<uint2> srect0, srect1;
    DevBuf<uint32_t> hist, seg_n, seg_start, blk_pairs, chunk_base, pair_base, cstart, cimg, ecnt, seg_base, segoff, emit_next;
    DevBuf<uint32_t> starts, cls_list;
    DevBuf<View> views;
    DevBuf<float> T_final;
    DevBuf<uint32_t> n_contrib;
    DevBuf<float> g2d;
    DevBuf<gsr_gaussian_grads> grads_dev;
    DevBuf<float> pose_part;
    DevBuf<uint32_t> counter;  // one device counter for synchronous calls (mesh transfer)
    const gsr_augment* aug = nullptr;  // bound by gsr_set_augment for GSR_FLAG_AUGMENT renders
    const float* overlay = nullptr;
    uint64_t render_serial = 0;  // renders issued on this context
    uint64_t saved_id = 0;       // serial of the render whose state backward may use (0: none)
    // last forward, for backward / inspection
    bool have_last = false;
    bool saved = false;
    FwdArgs last{};
    const gsr_scene* last_scene = nullptr;
    uint64_t last_scene_version = 0;
    hipStream_t last_stream = nullptr;
    // graph cache
    bool graph_valid = false;
    GraphKey gkey{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    // autotune cache: (images, W, H, gaussians) -> (tw, th, persistent, ppt, stream groups)
    std::map<std::tuple<int, int, int, long long>, std::tuple<int, int, int, int, int>> tune;
    hipEvent_t stage_ev[kStages + 1] = {};
    bool timed = false;
    hipStream_t cap_stream = nullptr;  // private stream used only to capture graphs
    // stream groups: sub-contexts (own workspace), their streams, fork and join events
    gsr_context* sub[kMaxGroups] = {};
    hipStream_t gstream[kMaxGroups] = {};
    hipEvent_t fork_ev = nullptr;
    hipEvent_t join_ev[kMaxGroups] = {};
    int last_groups = 1;  // groups of the last render
    std::vector<gsr_scene*> scenes;  // live scenes composed on this context (detached on destroy)
};

static int fail(gsr_context* ctx, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    g_err = buf;
    return code;
}

#define HIPCHK(ctx, expr)                                                                     \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail((ctx), GSR_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

static void drop_graph(gsr_context* ctx);
static int scratch_setup(int device);

// Grow a workspace buffer.  A reallocation invalidates any captured graph (its kernel
// arguments hold the old pointers).
template <typename T>
static int ensure(gsr_context* ctx, DevBuf<T>& b, size_t n, bool zero = false) {
    if (b.n >= n && b.p) return GSR_OK;
    drop_graph(ctx);
    b.release();
    size_t want = std::max<size_t>(n, 1);
    if (hipMalloc(&b.p, want * sizeof(T)) != hipSuccess) {
        b.p = nullptr;
        (void)hipGetLastError();
        return fail(ctx, GSR_E_NOMEM, "device allocation of %zu bytes failed", want * sizeof(T));
    }
    b.n = want;
    if (zero && hipMemset(b.p, 0, want * sizeof(T)) != hipSuccess) return fail(ctx, GSR_E_HIP, "hipMemset failed");
    return GSR_OK;
}

static void drop_graph(gsr_context* ctx) {
    if (ctx->gexec) hipGraphExecDestroy(ctx->gexec);
    if (ctx->graph) hipGraphDestroy(ctx->graph);
    ctx->gexec = nullptr;
    ctx->graph = nullptr;
    ctx->graph_valid = false;
}

static bool tile_ok(int tw, int th) {
    return (tw == 16 && th == 16) || (tw == 16 && th == 8) || (tw == 8 && th == 8) || (tw == 32 && th == 8);
}

extern "C" {

int gsr_create(int device, const gsr_config* cfg, gsr_context** out) {
    if (!out) return fail(nullptr, GSR_E_INVALID, "gsr_create: out is NULL");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        return fail(nullptr, GSR_E_HIP, "gsr_create: no HIP device available (%s)", hipGetErrorString(e));
    }
    if (device < 0 || device >= n) return fail(nullptr, GSR_E_HIP, "gsr_create: device %d out of range (%d devices)", device, n);
    gsr_config c{};
    if (cfg) c = *cfg;
    if (c.tile_w == 0 && c.tile_h == 0) { c.tile_w = 16; c.tile_h = 16; }
    if (!tile_ok(c.tile_w, c.tile_h)) return fail(nullptr, GSR_E_UNSUPPORTED, "gsr_create: tile %dx%d not supported", c.tile_w, c.tile_h);
    if (c.pair_capacity <= 0) c.pair_capacity = 1ll << 22;
    if (hipSetDevice(device) != hipSuccess) return fail(nullptr, GSR_E_HIP, "gsr_create: hipSetDevice(%d) failed", device);
    gsr_context* ctx = new gsr_context();
    ctx->device = device;
    hipDeviceGetAttribute(&ctx->num_cu, hipDeviceAttributeMultiprocessorCount, device);
    if (c.persistent_grid <= 0) c.persistent_grid = 8 * std::max(ctx->num_cu, 1);
    if (c.pixels_per_thread == 0) c.pixels_per_thread = 2;
    if (c.stream_groups == 0) c.stream_groups = 1;
    if (c.stream_groups < 1 || c.stream_groups > kMaxGroups) {
        delete ctx;
        return fail(nullptr, GSR_E_UNSUPPORTED, "gsr_create: stream_groups must be 1..%d", kMaxGroups);
    }
    if (c.pixels_per_thread != 1 && c.pixels_per_thread != 2 && c.pixels_per_thread != 4) {
        delete ctx;
        return fail(nullptr, GSR_E_UNSUPPORTED, "gsr_create: pixels_per_thread must be 1, 2 or 4");
    }
    ctx->cfg = c;
    // the device address of the no-allocation backward's static scratch, once per device
    if (int rs = scratch_setup(device)) {
        delete ctx;
        return rs;
    }
    if (hipMalloc(&ctx->d_status, sizeof(Status)) != hipSuccess ||
        hipHostMalloc(&ctx->h_status, sizeof(Status)) != hipSuccess) {
        delete ctx;
        return fail(nullptr, GSR_E_NOMEM, "gsr_create: status allocation failed");
    }
    hipMemset(ctx->d_status, 0, sizeof(Status));
    memset(ctx->h_status, 0, sizeof(Status));
    *out = ctx;
    return GSR_OK;
}

void gsr_destroy(gsr_context* ctx) {
    if (!ctx) return;
    hipSetDevice(ctx->device);
    hipDeviceSynchronize();
    // scenes that outlive the context keep their tables until gsr_scene_destroy, which then
    // no longer touches the context (nor the sub-contexts, for their groups' scenes)
    for (gsr_scene* sc : ctx->scenes) sc->ctx = nullptr;
    ctx->scenes.clear();
    for (int g = 0; g < kMaxGroups; ++g) {
        if (ctx->sub[g]) gsr_destroy(ctx->sub[g]);
        if (ctx->gstream[g]) hipStreamDestroy(ctx->gstream[g]);
        if (ctx->join_ev[g]) hipEventDestroy(ctx->join_ev[g]);
    }
    if (ctx->fork_ev) hipEventDestroy(ctx->fork_ev);
    drop_graph(ctx);
    for (auto& e : ctx->stage_ev)
        if (e) hipEventDestroy(e);
    if (ctx->cap_stream) hipStreamDestroy(ctx->cap_stream);
    ctx->pairs.release(); ctx->records.release(); ctx->vis.release(); ctx->sbvis.release(); ctx->loff.release();
    ctx->skey0.release(); ctx->skey1.release(); ctx->sgid0.release(); ctx->sgid1.release();
    ctx->ssrc0.release(); ctx->ssrc1.release();
    ctx->srect0.release(); ctx->srect1.release(); ctx->hist.release(); ctx->seg_n.release(); ctx->ecnt.release();
    ctx->seg_start.release(); ctx->blk_pairs.release(); ctx->chunk_base.release(); ctx->cstart.release();
    ctx->cimg.release(); ctx->pair_base.release(); ctx->seg_base.release(); ctx->segoff.release();
    ctx->emit_next.release();
    ctx->starts.release();
    ctx->cls_list.release(); ctx->views.release(); ctx->T_final.release(); ctx->n_contrib.release();
    ctx->g2d.release(); ctx->grads_dev.release(); ctx->pose_part.release(); ctx->counter.release();
    if (ctx->d_status) hipFree(ctx->d_status);
    if (ctx->h_status) hipHostFree(ctx->h_status);
    delete ctx;
}

const char* gsr_last_error(const gsr_context* ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

int gsr_get_config(const gsr_context* ctx, gsr_config* out) {
    if (!ctx || !out) return fail(nullptr, GSR_E_INVALID, "gsr_get_config: NULL argument");
    *out = ctx->cfg;
    return GSR_OK;
}

int gsr_set_tile(gsr_context* ctx, int32_t tw, int32_t th) {
    if (!ctx) return fail(nullptr, GSR_E_INVALID, "gsr_set_tile: ctx is NULL");
    if (!tile_ok(tw, th)) return fail(ctx, GSR_E_UNSUPPORTED, "gsr_set_tile: tile %dx%d not supported", tw, th);
    if (tw != ctx->cfg.tile_w || th != ctx->cfg.tile_h) drop_graph(ctx);
    ctx->cfg.tile_w = tw;
    ctx->cfg.tile_h = th;
    return GSR_OK;
}

int gsr_set_pixels_per_thread(gsr_context* ctx, int32_t ppt) {
    if (!ctx) return fail(nullptr, GSR_E_INVALID, "gsr_set_pixels_per_thread: ctx is NULL");
    if (ppt != 1 && ppt != 2 && ppt != 4)
        return fail(ctx, GSR_E_UNSUPPORTED, "gsr_set_pixels_per_thread: %d not 1, 2 or 4", ppt);
    if (ppt != ctx->cfg.pixels_per_thread) drop_graph(ctx);
    ctx->cfg.pixels_per_thread = ppt;
    return GSR_OK;
}

int gsr_set_stream_groups(gsr_context* ctx, int32_t groups) {
    if (!ctx) return fail(nullptr, GSR_E_INVALID, "gsr_set_stream_groups: ctx is NULL");
    if (groups < 1 || groups > kMaxGroups)
        return fail(ctx, GSR_E_UNSUPPORTED, "gsr_set_stream_groups: %d outside 1..%d", groups, kMaxGroups);
    ctx->cfg.stream_groups = groups;
    return GSR_OK;
}

void gsr_scene_destroy(gsr_scene* sc) {
    if (!sc) return;
    for (auto& sub : sc->sub) {
        gsr_scene_destroy(sub);
        sub = nullptr;
    }
    if (sc->lidar) {
        hipDeviceSynchronize();
        lidar_free(sc->lidar);
    }
    if (sc->nodes_d) hipFree(sc->nodes_d);
    if (sc->envs_d) hipFree(sc->envs_d);
    if (sc->blocks_d) hipFree(sc->blocks_d);
    if (sc->supers_d) hipFree(sc->supers_d);
    if (gsr_context* ctx = sc->ctx) {  // null once its context was destroyed
        if (ctx->last_scene == sc) {
            ctx->have_last = ctx->saved = false;
            ctx->saved_id = 0;
            ctx->last_scene = nullptr;
        }
        if (ctx->graph_valid && ctx->gkey.scene == sc) drop_graph(ctx);
        ctx->scenes.erase(std::remove(ctx->scenes.begin(), ctx->scenes.end(), sc), ctx->scenes.end());
    }
    delete sc;
}

int64_t gsr_scene_gaussians(const gsr_scene* sc, int32_t env) {
    if (!sc) return -1;
    if (env < 0) return sc->total;
    if (env >= sc->n_envs) return -1;
    return sc->envs_h[env].n;
}

int gsr_compose_scene(gsr_context* ctx, int32_t n_envs, const int32_t* off, const gsr_gaussians* nodes,
                      int32_t n_nodes, const gsr_pose* poses, gsr_scene** inout) {
    if (!ctx) return fail(nullptr, GSR_E_INVALID, "gsr_compose_scene: ctx is NULL");
    if (!inout || !off || !nodes || !poses) return fail(ctx, GSR_E_INVALID, "gsr_compose_scene: NULL argument");
    if (n_envs < 1 || n_nodes < 1) return fail(ctx, GSR_E_INVALID, "gsr_compose_scene: n_envs and n_nodes must be >= 1");
    if (off[0] != 0 || off[n_envs] != n_nodes)
        return fail(ctx, GSR_E_INVALID, "gsr_compose_scene: env_node_offsets must run from 0 to n_nodes");
    for (int e = 0; e < n_envs; ++e)
        if (off[e + 1] <= off[e]) return fail(ctx, GSR_E_INVALID, "gsr_compose_scene: env %d has no node", e);
    const int deg = nodes[0].sh_degree;
    long long total = 0;
    for (int k = 0; k < n_nodes; ++k) {
        const gsr_gaussians& g = nodes[k];
        if (g.n < 0) return fail(ctx, GSR_E_INVALID, "gsr_compose_scene: node %d has n < 0", k);
        if (g.sh_degree < 0 || g.sh_degree > 3) return fail(ctx, GSR_E_INVALID, "gsr_compose_scene: node %d sh_degree %d outside 0..3", k, g.sh_degree);
        if (g.sh_degree != deg) return fail(ctx, GSR_E_INVALID, "gsr_compose_scene: nodes differ in sh_degree");
        if (g.n > 0 && (!g.means || !g.scales || !g.quats || !g.opacities || !g.sh))
            return fail(ctx, GSR_E_INVALID, "gsr_compose_scene: node %d has a NULL parameter pointer", k);
        if (g.n > 0 && ((uintptr_t)g.quats % 16 != 0 || (uintptr_t)g.sh % 16 != 0))
            return fail(ctx, GSR_E_INVALID, "gsr_compose_scene: node %d quats/sh not 16-byte aligned", k);
        total += g.n;
    }
    if (total > 0x7fffffffll) return fail(ctx, GSR_E_INVALID, "gsr_compose_scene: more than 2^31-1 Gaussians");
    gsr_scene* sc = *inout;
    bool same = sc && sc->ctx == ctx && sc->n_envs == n_envs && sc->n_nodes == n_nodes && sc->sh_degree == deg &&
                std::equal(off, off + n_envs + 1, sc->env_offsets.begin());
    if (same)
        for (int k = 0; k < n_nodes && same; ++k) same = (long long)sc->nodes_h[k].n == nodes[k].n;
    if (!same) {
        gsr_scene_destroy(sc);
        *inout = nullptr;
        sc = new gsr_scene();
        sc->ctx = ctx;
        ctx->scenes.push_back(sc);
    }
    hipSetDevice(ctx->device);
    sc->n_envs = n_envs;
    sc->n_nodes = n_nodes;
    sc->sh_degree = deg;
    sc->total = total;
    sc->env_offsets.assign(off, off + n_envs + 1);
    sc->poses = poses;
    sc->nodes_h.resize(n_nodes);
    sc->envs_h.resize(n_envs);
    sc->blocks_h.clear();
    uint32_t gid = 0;
    for (int e = 0; e < n_envs; ++e) {
        Env& ev = sc->envs_h[e];
        ev.gid_base = gid;
        ev.node_begin = off[e];
        ev.node_end = off[e + 1];
        for (int k = off[e]; k < off[e + 1]; ++k) {
            Node& nd = sc->nodes_h[k];
            nd.means = nodes[k].means; nd.scales = nodes[k].scales; nd.quats = nodes[k].quats;
            nd.opac = nodes[k].opacities; nd.sh = nodes[k].sh;
            nd.gid_base = gid;
            nd.n = (uint32_t)nodes[k].n;
            nd.env = e;
            nd.block_begin = (int32_t)sc->blocks_h.size();
            for (uint32_t s = 0; s < nd.n; s += kBlock)
                sc->blocks_h.push_back(Block{k, e, gid + s, std::min<uint32_t>(kBlock, nd.n - s)});
            gid += nd.n;
        }
        ev.n = gid - ev.gid_base;
    }
    // super-blocks: runs of an env's chunks, sized so the grid still has ~8 blocks per CU
    const long long nchunks = (long long)sc->blocks_h.size();
    const int cps = (int)std::max(1ll, std::min<long long>(kMaxChunksPerSuper, nchunks / (8ll * std::max(ctx->num_cu, 1))));
    sc->supers_h.clear();
    sc->sb_cap = cps * kBlock;
    {
        size_t ch = 0;
        for (int e = 0; e < n_envs; ++e) {
            Env& ev = sc->envs_h[e];
            ev.sb_begin = (int32_t)sc->supers_h.size();
            size_t end = ch;
            while (end < sc->blocks_h.size() && sc->blocks_h[end].env == e) ++end;
            for (size_t b = ch; b < end; b += cps)
                sc->supers_h.push_back(Super{e, (int32_t)b, (int32_t)std::min(end, b + cps), 0});
            if (end == ch) sc->supers_h.push_back(Super{e, (int32_t)ch, (int32_t)ch, 0});  // empty env
            ev.sb_count = (int32_t)sc->supers_h.size() - ev.sb_begin;
            ch = end;
        }
    }
    auto up = [&](auto*& dptr, const auto& vec) -> int {
        using T = typename std::remove_reference<decltype(vec)>::type::value_type;
        if (!same && dptr == nullptr) {
            if (hipMalloc(&dptr, std::max<size_t>(vec.size(), 1) * sizeof(T)) != hipSuccess) {
                dptr = nullptr;
                return fail(ctx, GSR_E_NOMEM, "gsr_compose_scene: table allocation failed");
            }
        }
        if (!vec.empty() && hipMemcpy(dptr, vec.data(), vec.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
            return fail(ctx, GSR_E_HIP, "gsr_compose_scene: table upload failed");
        return GSR_OK;
    };
    int r;
    if ((r = up(sc->nodes_d, sc->nodes_h)) != GSR_OK) { if (!same) gsr_scene_destroy(sc); return r; }
    if ((r = up(sc->envs_d, sc->envs_h)) != GSR_OK) { if (!same) gsr_scene_destroy(sc); return r; }
    if ((r = up(sc->blocks_d, sc->blocks_h)) != GSR_OK) { if (!same) gsr_scene_destroy(sc); return r; }
    if ((r = up(sc->supers_d, sc->supers_h)) != GSR_OK) { if (!same) gsr_scene_destroy(sc); return r; }
    sc->version++;
    if (ctx->graph_valid && ctx->gkey.scene == sc) drop_graph(ctx);
    *inout = sc;
    return GSR_OK;
}

}  // extern "C"

// Fill FwdArgs and make sure the workspace holds this render.
static int prepare(gsr_context* ctx, const gsr_scene* sc, int C, const gsr_camera* cams, int W, int H, float* rgb,
                   float* depth, float* alpha, int persistent, int save, FwdArgs& a) {
    const int tw = ctx->cfg.tile_w, th = ctx->cfg.tile_h;
    memset(&a, 0, sizeof a);
    a.nodes = sc->nodes_d;
    a.envs = sc->envs_d;
    a.blocks = sc->blocks_d;
    a.n_blocks = (int)sc->blocks_h.size();
    a.supers = sc->supers_d;
    a.n_supers = (int)sc->supers_h.size();
    a.n_nodes = sc->n_nodes;
    a.sh_degree = sc->sh_degree;
    a.poses = sc->poses;
    a.cams = cams;
    a.C = C;
    a.images = sc->n_envs * C;
    a.width = W;
    a.height = H;
    a.tw = tw;
    a.th = th;
    a.tiles_x = (W + tw - 1) / tw;
    a.tiles_y = (H + th - 1) / th;
    a.tpi = a.tiles_x * a.tiles_y;
    a.tiles = (long long)a.images * a.tpi;
    const long long gsz = (long long)(a.tiles_x + 1) * (a.tiles_y + 1);
    if (gsz > kLdsHistLimit || a.tpi > kMaxTilesPerImage)
        return fail(ctx, GSR_E_UNSUPPORTED, "%dx%d images with %dx%d tiles exceed %d tiles per image", W, H, tw, th,
                    kMaxTilesPerImage);
    if (a.tiles >= 0xffffffffll) return fail(ctx, GSR_E_UNSUPPORTED, "too many tiles");
    const size_t nrec = (size_t)C * (size_t)sc->total;
    const size_t npix = (size_t)a.images * W * H;
    // depth-sort buffers: each image's segment is rounded up to whole radix chunks
    const size_t sort_len = ((nrec + kSortTile - 1) / kSortTile + (size_t)a.images) * kSortTile;
    if (sort_len >= 0xffffffffull) return fail(ctx, GSR_E_UNSUPPORTED, "too many (image, Gaussian) records");
    a.sort_chunks = (int)(sort_len / kSortTile);
    const size_t n_lists = (size_t)a.n_supers * C;
    const size_t n_pblocks = sort_len / kPairBlock;
    int r;
    const int sb_cap = sc->sb_cap;
    if ((r = ensure(ctx, ctx->records, nrec)) || (r = ensure(ctx, ctx->vis, n_lists * sb_cap)) ||
        (r = ensure(ctx, ctx->sbvis, n_lists)) || (r = ensure(ctx, ctx->loff, n_lists)) || (r = ensure(ctx, ctx->skey0, sort_len)) ||
        (r = ensure(ctx, ctx->skey1, sort_len)) || (r = ensure(ctx, ctx->ssrc0, sort_len)) ||
        (r = ensure(ctx, ctx->ssrc1, sort_len)) || (r = ensure(ctx, ctx->sgid0, sort_len)) ||
        (r = ensure(ctx, ctx->sgid1, sort_len)) || (r = ensure(ctx, ctx->srect0, sort_len)) ||
        (r = ensure(ctx, ctx->srect1, sort_len)) ||
        (r = ensure(ctx, ctx->hist, (size_t)a.sort_chunks * 256)) ||
        (r = ensure(ctx, ctx->seg_n, a.images)) || (r = ensure(ctx, ctx->seg_start, a.images + 1)) ||
        (r = ensure(ctx, ctx->blk_pairs, n_pblocks)) || (r = ensure(ctx, ctx->chunk_base, a.images + 1)) || (r = ensure(ctx, ctx->pair_base, a.images)) ||
        (r = ensure(ctx, ctx->seg_base, a.images + 1)) || (r = ensure(ctx, ctx->emit_next, 8 * kEmitQueueStride)) ||
        (r = ensure(ctx, ctx->starts, a.tiles + 1)) ||
        (r = ensure(ctx, ctx->cls_list, (size_t)kNumClasses * a.tiles)) ||
        (r = ensure(ctx, ctx->views, (size_t)sc->n_nodes * C)) || (r = ensure(ctx, ctx->T_final, npix)) ||
        (r = ensure(ctx, ctx->n_contrib, npix)))
        return r;
    if (ctx->pair_cap < ctx->cfg.pair_capacity) ctx->pair_cap = ctx->cfg.pair_capacity;
    if (ctx->pair_cap >= 0xffffffffll) return fail(ctx, GSR_E_UNSUPPORTED, "pair capacity beyond 32-bit slots");
    // emission chunks of about chunk_pairs pairs (at most pairs / chunk_pairs + 1 per image).
    // Small chunks give the emission more wavefronts; each chunk adds a count and an offset per
    // tile of its image, so chunks hold at least kChunkPairsPerTile pairs per tile
    a.chunk_pairs = std::max(1024, kChunkPairsPerTile * a.tpi);
    a.chunk_cap = (int)(ctx->pair_cap / a.chunk_pairs + a.images + 1);
    if ((r = ensure(ctx, ctx->pairs, ctx->pair_cap)) || (r = ensure(ctx, ctx->cstart, (size_t)a.chunk_cap)) ||
        (r = ensure(ctx, ctx->cimg, (size_t)a.chunk_cap)) ||
        (r = ensure(ctx, ctx->ecnt, (size_t)a.chunk_cap * a.tpi)) ||
        (r = ensure(ctx, ctx->segoff, ((size_t)a.chunk_cap / kSegChunks + a.images + 1) * a.tpi)))
        return r;
    a.views = ctx->views.p;
    a.records = ctx->records.p;
    a.vis = ctx->vis.p;
    a.sbvis = ctx->sbvis.p;
    a.loff = ctx->loff.p;
    a.sb_cap = sb_cap;
    a.skey[0] = ctx->skey0.p;
    a.skey[1] = ctx->skey1.p;
    a.ssrc[0] = ctx->ssrc0.p;
    a.ssrc[1] = ctx->ssrc1.p;
    a.sgid[0] = ctx->sgid0.p;
    a.sgid[1] = ctx->sgid1.p;
    a.srect[0] = ctx->srect0.p;
    a.srect[1] = ctx->srect1.p;
    a.hist = ctx->hist.p;
    a.seg_n = ctx->seg_n.p;
    a.seg_start = ctx->seg_start.p;
    a.blk_pairs = ctx->blk_pairs.p;
    a.chunk_base = ctx->chunk_base.p;
    a.pair_base = ctx->pair_base.p;
    a.cstart = ctx->cstart.p;
    a.cimg = ctx->cimg.p;
    a.ecnt = ctx->ecnt.p;
    a.seg_base = ctx->seg_base.p;
    a.emit_next = ctx->emit_next.p;
    a.segoff = ctx->segoff.p;
    a.num_cu = ctx->num_cu;
    if (forward_lds_limits(a) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, GSR_E_UNSUPPORTED, "%d tiles per image exceed the device's LDS per block", a.tpi);
    }
    a.starts = ctx->starts.p;
    a.cls_list = ctx->cls_list.p;
    a.pairs = ctx->pairs.p;
    a.pair_cap = ctx->pair_cap;
    a.status = ctx->d_status;
    a.rgb = rgb;
    a.depth = depth;
    a.alpha = alpha;
    a.T_final = ctx->T_final.p;
    a.n_contrib = ctx->n_contrib.p;
    a.persistent = persistent;
    a.persistent_grid = ctx->cfg.persistent_grid;
    // at most one wavefront's worth of pixels per lane group: 8x8 tiles take 1, 16x8 up to 2
    a.ppt = std::min(ctx->cfg.pixels_per_thread, tw * th / 64);
    a.save = save;
    a.count = 0;
    return GSR_OK;
}

static int read_status(gsr_context* ctx, hipStream_t s) {
    HIPCHK(ctx, hipMemcpyAsync(ctx->h_status, ctx->d_status, sizeof(Status), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    return GSR_OK;
}

extern "C" {

// Stream groups: the configured count, at most one per environment; one for renders whose
// state or parameters belong to the context (saved for backward, timed, augmented).
static int render_groups(const gsr_context* ctx, const gsr_scene* sc, uint32_t flags) {
    if (ctx->cfg.stream_groups <= 1 || (flags & (GSR_FLAG_SAVE | GSR_FLAG_TIMING | GSR_FLAG_AUGMENT))) return 1;
    return std::min(ctx->cfg.stream_groups, sc->n_envs);
}

// G sub-contexts (the parent's tile shape and pixels per thread), their streams and the
// fork / join events.
static int ensure_groups(gsr_context* ctx, int G) {
    gsr_config c = ctx->cfg;
    c.stream_groups = 1;
    if (!ctx->fork_ev) HIPCHK(ctx, hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming));
    for (int g = 0; g < G; ++g) {
        if (!ctx->sub[g]) {
            const int r = gsr_create(ctx->device, &c, &ctx->sub[g]);
            if (r) return fail(ctx, r, "stream group %d: %s", g, gsr_last_error(nullptr));
        }
        gsr_context* sub = ctx->sub[g];
        int r = GSR_OK;
        if (sub->cfg.tile_w != c.tile_w || sub->cfg.tile_h != c.tile_h) r = gsr_set_tile(sub, c.tile_w, c.tile_h);
        if (!r && sub->cfg.pixels_per_thread != c.pixels_per_thread) r = gsr_set_pixels_per_thread(sub, c.pixels_per_thread);
        if (r) return fail(ctx, r, "stream group %d: %s", g, sub->err.c_str());
        if (!ctx->gstream[g]) HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->gstream[g], hipStreamNonBlocking));
        if (!ctx->join_ev[g]) HIPCHK(ctx, hipEventCreateWithFlags(&ctx->join_ev[g], hipEventDisableTiming));
    }
    return GSR_OK;
}

// The scene's G groups: contiguous environment ranges of about equal Gaussian counts (at
// least one environment each), group g composed on sub-context g over the same borrowed
// Gaussians and pose buffer.  Composed again after the scene is.
static int ensure_subscenes(gsr_context* ctx, gsr_scene* sc, int G) {
    if (sc->sub_groups == G && sc->sub_version == sc->version) return GSR_OK;
    const int E = sc->n_envs;
    std::vector<long long> cum(E + 1, 0);
    for (int e = 0; e < E; ++e) cum[e + 1] = cum[e] + (long long)sc->envs_h[e].n;
    int b[kMaxGroups + 1];
    b[0] = 0;
    b[G] = E;
    for (int g = 1; g < G; ++g) {
        const long long target = cum[E] * g / G;
        int e = (int)(std::lower_bound(cum.begin(), cum.end(), target) - cum.begin());
        b[g] = std::min(std::max(e, b[g - 1] + 1), E - (G - g));
    }
    for (int g = 0; g < G; ++g) {
        const int lo = b[g], hi = b[g + 1];
        const int k0 = sc->env_offsets[lo], k1 = sc->env_offsets[hi];
        std::vector<int32_t> off(hi - lo + 1);
        for (int i = 0; i <= hi - lo; ++i) off[i] = sc->env_offsets[lo + i] - k0;
        std::vector<gsr_gaussians> nd(k1 - k0);
        for (int k = k0; k < k1; ++k) {
            const Node& n = sc->nodes_h[k];
            gsr_gaussians& d = nd[k - k0];
            d.n = n.n;
            d.sh_degree = sc->sh_degree;
            d.reserved = 0;
            d.means = n.means;
            d.scales = n.scales;
            d.quats = n.quats;
            d.opacities = n.opac;
            d.sh = n.sh;
        }
        const int r = gsr_compose_scene(ctx->sub[g], hi - lo, off.data(), nd.data(), k1 - k0, sc->poses + k0, &sc->sub[g]);
        if (r) return fail(ctx, r, "stream group %d: %s", g, ctx->sub[g]->err.c_str());
        sc->sub_env[g] = lo;
    }
    sc->sub_env[G] = E;
    for (int g = G; g < kMaxGroups; ++g) {
        gsr_scene_destroy(sc->sub[g]);
        sc->sub[g] = nullptr;
    }
    sc->sub_groups = G;
    sc->sub_version = sc->version;
    return GSR_OK;
}

// A grouped render: each group's images rendered by its sub-context on its own stream, after
// the work already on `s` (fork event) and before later work on `s` (join events).
static int render_grouped(gsr_context* ctx, const gsr_scene* sc0, int G, int32_t C, const gsr_camera* cams, int32_t W,
                          int32_t H, float* rgb, float* depth, float* alpha, uint32_t flags, hipStream_t s) {
    gsr_scene* sc = const_cast<gsr_scene*>(sc0);  // the sub-scene cache only
    int r;
    if ((r = ensure_groups(ctx, G)) || (r = ensure_subscenes(ctx, sc, G))) return r;
    HIPCHK(ctx, hipEventRecord(ctx->fork_ev, s));
    const size_t img_px = (size_t)W * H;
    for (int g = 0; g < G; ++g) {
        const size_t img0 = (size_t)sc->sub_env[g] * C, px = img0 * img_px;
        HIPCHK(ctx, hipStreamWaitEvent(ctx->gstream[g], ctx->fork_ev, 0));
        r = gsr_render_rgbd(ctx->sub[g], sc->sub[g], C, cams + img0, W, H, rgb + 3 * px, depth + px,
                            alpha ? alpha + px : nullptr, flags, ctx->gstream[g]);
        if (r) return fail(ctx, r, "stream group %d: %s", g, ctx->sub[g]->err.c_str());
        HIPCHK(ctx, hipEventRecord(ctx->join_ev[g], ctx->gstream[g]));
        HIPCHK(ctx, hipStreamWaitEvent(s, ctx->join_ev[g], 0));
    }
    ctx->last_groups = G;
    ctx->last_stream = s;
    ctx->have_last = ctx->saved = ctx->timed = false;
    ctx->saved_id = 0;
    ctx->render_serial++;
    return GSR_OK;
}

int gsr_render_rgbd(gsr_context* ctx, const gsr_scene* sc, int32_t C, const gsr_camera* cams, int32_t W, int32_t H,
                    float* rgb, float* depth, float* alpha, uint32_t flags, void* stream) {
    if (!ctx) return fail(nullptr, GSR_E_INVALID, "gsr_render_rgbd: ctx is NULL");
    if (!sc || !cams || !rgb || !depth) return fail(ctx, GSR_E_INVALID, "gsr_render_rgbd: NULL scene, cams, rgb or depth");
    if (sc->ctx != ctx) return fail(ctx, GSR_E_INVALID, "gsr_render_rgbd: scene belongs to another context");
    if (C < 1) return fail(ctx, GSR_E_INVALID, "gsr_render_rgbd: cams_per_env must be >= 1");
    if (W < 1 || H < 1 || W > 8192 || H > 8192) return fail(ctx, GSR_E_INVALID, "gsr_render_rgbd: image size %dx%d outside 1..8192", W, H);
    hipStream_t s = (hipStream_t)stream;
    hipSetDevice(ctx->device);
    const int G = render_groups(ctx, sc, flags);
    if (G > 1) return render_grouped(ctx, sc, G, C, cams, W, H, rgb, depth, alpha, flags, s);
    ctx->last_groups = 1;
    const int persistent = (flags & GSR_FLAG_PERSISTENT) ? 1 : 0;
    const int save = (flags & GSR_FLAG_SAVE) ? 1 : 0;
    FwdArgs a;
    int r = prepare(ctx, sc, C, cams, W, H, rgb, depth, alpha, persistent, save, a);
    if (r) return r;
    const int count = (flags & GSR_FLAG_CHECK) ? 1 : 0;
    a.count = count;
    if (flags & GSR_FLAG_AUGMENT) {
        if (save) return fail(ctx, GSR_E_INVALID, "gsr_render_rgbd: GSR_FLAG_AUGMENT with GSR_FLAG_SAVE");
        if (!ctx->aug) return fail(ctx, GSR_E_INVALID, "gsr_render_rgbd: GSR_FLAG_AUGMENT without gsr_set_augment");
        a.aug = ctx->aug;
        a.overlay = ctx->overlay;
    }
    ctx->last_stream = s;
    if (flags & GSR_FLAG_GRAPH) {
        GraphKey k{sc, cams, rgb, depth, alpha, C, W, H, ctx->cfg.tile_w, ctx->cfg.tile_h, persistent, a.ppt,
                   flags, s, ctx->pair_cap, a.aug, a.overlay};
        if (!(ctx->graph_valid && ctx->gkey == k)) {
            drop_graph(ctx);
            // capture on a private stream (the caller's may be the legacy default stream,
            // which cannot be captured); capturing runs nothing, the replay goes on `s`
            if (!ctx->cap_stream) HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
            HIPCHK(ctx, hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
            hipError_t e = launch_forward(a, ctx->cap_stream);
            hipGraph_t g = nullptr;
            hipError_t e2 = hipStreamEndCapture(ctx->cap_stream, &g);
            if (e != hipSuccess || e2 != hipSuccess) {
                if (g) hipGraphDestroy(g);
                return fail(ctx, GSR_E_HIP, "graph capture failed: %s / %s", hipGetErrorString(e), hipGetErrorString(e2));
            }
            ctx->graph = g;
            HIPCHK(ctx, hipGraphInstantiate(&ctx->gexec, g, nullptr, nullptr, 0));
            ctx->gkey = k;
            ctx->graph_valid = true;
        }
        HIPCHK(ctx, hipGraphLaunch(ctx->gexec, s));
    } else {
        if (flags & GSR_FLAG_TIMING) {
            for (auto& e : ctx->stage_ev)
                if (!e) HIPCHK(ctx, hipEventCreate(&e));
            a.stage_events = ctx->stage_ev;
        }
        ctx->timed = (flags & GSR_FLAG_TIMING) != 0;
        for (int attempt = 0;; ++attempt) {
            HIPCHK(ctx, launch_forward(a, s));
            if (!(flags & GSR_FLAG_CHECK)) break;
            if ((r = read_status(ctx, s))) return r;
            if (!(ctx->h_status->flags & GSR_STATUS_OVERFLOW)) break;
            if (attempt >= 2)
                return fail(ctx, GSR_E_CAPACITY, "pair capacity %lld still short of %llu", ctx->pair_cap,
                            (unsigned long long)ctx->h_status->pairs);
            ctx->pair_cap = (long long)(ctx->h_status->pairs * 5 / 4) + 1024;
            drop_graph(ctx);
            if ((r = prepare(ctx, sc, C, cams, W, H, rgb, depth, alpha, persistent, save, a))) return r;
            a.count = count;
            if (flags & GSR_FLAG_AUGMENT) {
                a.aug = ctx->aug;
                a.overlay = ctx->overlay;
            }
            if (flags & GSR_FLAG_TIMING) a.stage_events = ctx->stage_ev;
        }
        a.stage_events = nullptr;
    }
    ctx->have_last = true;
    ctx->saved = (flags & GSR_FLAG_SAVE) != 0;
    ctx->saved_id = ctx->saved ? ctx->render_serial + 1 : 0;
    ctx->render_serial++;
    ctx->last = a;
    ctx->last_scene = sc;
    ctx->last_scene_version = sc->version;
    return GSR_OK;
}

int gsr_lidar_build(gsr_context* ctx, gsr_scene* sc) {
    if (!ctx) return fail(nullptr, GSR_E_INVALID, "gsr_lidar_build: ctx is NULL");
    if (!sc || sc->ctx != ctx) return fail(ctx, GSR_E_INVALID, "gsr_lidar_build: no scene of this context");
    hipSetDevice(ctx->device);
    HIPCHK(ctx, hipDeviceSynchronize());
    if (sc->lidar) lidar_free(sc->lidar);
    sc->lidar = nullptr;
    LidarScene* L = nullptr;
    const std::string err = lidar_build(sc->nodes_h, &L);
    if (!err.empty()) return fail(ctx, GSR_E_NOMEM, "gsr_lidar_build: %s", err.c_str());
    sc->lidar = L;
    sc->lidar_version = sc->version;
    return GSR_OK;
}

int gsr_render_lidar(gsr_context* ctx, const gsr_scene* sc, int32_t rays_per_env, const gsr_ray* rays, float* range,
                     float* alpha, uint32_t* hits, void* stream) {
    if (!ctx) return fail(nullptr, GSR_E_INVALID, "gsr_render_lidar: ctx is NULL");
    if (!sc || !rays || !range || !alpha) return fail(ctx, GSR_E_INVALID, "gsr_render_lidar: NULL argument");
    if (sc->ctx != ctx) return fail(ctx, GSR_E_INVALID, "gsr_render_lidar: scene belongs to another context");
    if (rays_per_env < 1) return fail(ctx, GSR_E_INVALID, "gsr_render_lidar: rays_per_env must be >= 1");
    if (!sc->lidar || sc->lidar_version != sc->version)
        return fail(ctx, GSR_E_STATE, "gsr_render_lidar: call gsr_lidar_build after composing the scene");
    hipSetDevice(ctx->device);
    HIPCHK(ctx, launch_lidar(sc->lidar, sc->envs_d, sc->poses, sc->n_envs, rays_per_env, rays, range, alpha, hits,
                             (hipStream_t)stream));
    return GSR_OK;
}

int gsr_augment_rgb(gsr_context* ctx, int32_t images, int32_t W, int32_t H, const float* rgb, const float* overlay,
                    const gsr_augment* params, float* out, void* stream) {
    if (!ctx) return fail(nullptr, GSR_E_INVALID, "gsr_augment_rgb: ctx is NULL");
    if (!rgb || !params || !out) return fail(ctx, GSR_E_INVALID, "gsr_augment_rgb: NULL rgb, params or out");
    if (images < 1 || W < 1 || H < 1 || W > 8192 || H > 8192)
        return fail(ctx, GSR_E_INVALID, "gsr_augment_rgb: %d images of %dx%d", images, W, H);
    hipSetDevice(ctx->device);
    HIPCHK(ctx, launch_augment(images, W, H, rgb, overlay, params, out, ctx->num_cu, (hipStream_t)stream));
    return GSR_OK;
}

int gsr_mesh_to_gaussians(gsr_context* ctx, int64_t n_vertices, const float* vertices, const float* vertex_colors,
                          int64_t n_faces, const int32_t* faces, float flatten, float opacity, int32_t sh_degree,
                          const gsr_gaussian_grads* out, void* stream) {
    if (!ctx) return fail(nullptr, GSR_E_INVALID, "gsr_mesh_to_gaussians: ctx is NULL");
    if (!out || n_vertices < 0 || n_faces < 0 || (n_faces > 0 && (!vertices || !faces)))
        return fail(ctx, GSR_E_INVALID, "gsr_mesh_to_gaussians: NULL arrays or negative sizes");
    if (sh_degree < 0 || sh_degree > 3) return fail(ctx, GSR_E_INVALID, "gsr_mesh_to_gaussians: sh_degree %d", sh_degree);
    if (!(flatten >= 0.0f) || !(opacity >= 0.0f && opacity <= 1.0f))
        return fail(ctx, GSR_E_INVALID, "gsr_mesh_to_gaussians: flatten %g or opacity %g out of range", flatten, opacity);
    if (n_faces > 0x7fffffffll || n_vertices > 0x7fffffffll)
        return fail(ctx, GSR_E_INVALID, "gsr_mesh_to_gaussians: more than 2^31 - 1 faces or vertices");
    hipSetDevice(ctx->device);
    hipStream_t s = (hipStream_t)stream;
    int r = ensure(ctx, ctx->counter, 1);
    if (r) return r;
    HIPCHK(ctx, hipMemsetAsync(ctx->counter.p, 0, sizeof(uint32_t), s));
    const int K = (sh_degree + 1) * (sh_degree + 1);
    HIPCHK(ctx, launch_mesh_to_gs(n_faces, n_vertices, vertices, vertex_colors, faces, flatten, opacity, K, *out,
                                  ctx->counter.p, ctx->num_cu, s));
    uint32_t bad = 0;
    HIPCHK(ctx, hipMemcpyAsync(&bad, ctx->counter.p, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    if (bad) return fail(ctx, GSR_E_INVALID, "gsr_mesh_to_gaussians: %u faces index outside 0..%lld (written transparent)",
                         bad, (long long)n_vertices - 1);
    return GSR_OK;
}

int gsr_set_augment(gsr_context* ctx, const gsr_augment* params, const float* overlay) {
    if (!ctx) return fail(nullptr, GSR_E_INVALID, "gsr_set_augment: ctx is NULL");
    if (!params) return fail(ctx, GSR_E_INVALID, "gsr_set_augment: params is NULL");
    ctx->aug = params;
    ctx->overlay = overlay;
    return GSR_OK;
}

int gsr_query_status(gsr_context* ctx, gsr_status_info* out) {
    if (!ctx || !out) return fail(ctx, GSR_E_INVALID, "gsr_query_status: NULL argument");
    hipSetDevice(ctx->device);
    if (ctx->last_groups > 1) {  // the groups' counters combined
        gsr_status_info sum{};
        for (int g = 0; g < ctx->last_groups; ++g) {
            gsr_status_info o{};
            const int r = gsr_query_status(ctx->sub[g], &o);
            if (r) return fail(ctx, r, "stream group %d: %s", g, ctx->sub[g]->err.c_str());
            sum.flags |= o.flags;
            sum.nonfinite += o.nonfinite;
            sum.pairs += o.pairs;
            sum.pair_capacity += o.pair_capacity;
            sum.max_tile_pairs = std::max(sum.max_tile_pairs, o.max_tile_pairs);
            sum.visible += o.visible;
            sum.visible_any += o.visible_any;
            sum.evals += o.evals;
        }
        *out = sum;
        return GSR_OK;
    }
    int r = read_status(ctx, ctx->last_stream);
    if (r) return r;
    const Status& st = *ctx->h_status;
    out->flags = st.flags;
    out->nonfinite = st.nonfinite;
    out->pairs = st.pairs;
    out->pair_capacity = (uint64_t)ctx->pair_cap;
    out->max_tile_pairs = st.max_tile;
    out->reserved = 0;
    out->visible = out->visible_any = out->evals = 0;
    for (int q = 0; q < kParts; ++q) {
        out->visible += st.visible[q];
        out->visible_any += st.visible_any[q];
        out->evals += st.evals[q];
    }
    return GSR_OK;
}

int gsr_stage_times(gsr_context* ctx, float* ms) {
    if (!ctx || !ms) return fail(ctx, GSR_E_INVALID, "gsr_stage_times: NULL argument");
    if (!ctx->timed || !ctx->stage_ev[0]) return fail(ctx, GSR_E_STATE, "gsr_stage_times: last render was not timed");
    hipSetDevice(ctx->device);
    HIPCHK(ctx, hipEventSynchronize(ctx->stage_ev[kStages]));
    for (int i = 0; i < kStages; ++i) HIPCHK(ctx, hipEventElapsedTime(&ms[i], ctx->stage_ev[i], ctx->stage_ev[i + 1]));
    return GSR_OK;
}

int gsr_copy_pairs(gsr_context* ctx, uint64_t* keys, uint32_t* values, uint32_t* ranges, int64_t capacity, int64_t* n_pairs) {
    if (!ctx || !keys || !values || !ranges || !n_pairs) return fail(ctx, GSR_E_INVALID, "gsr_copy_pairs: NULL argument");
    if (ctx->last_groups > 1) return fail(ctx, GSR_E_STATE, "gsr_copy_pairs: the last render was split into stream groups");
    if (!ctx->have_last) return fail(ctx, GSR_E_STATE, "gsr_copy_pairs: nothing rendered yet");
    hipSetDevice(ctx->device);
    int r = read_status(ctx, ctx->last_stream);
    if (r) return r;
    *n_pairs = (int64_t)ctx->h_status->pairs;
    if (ctx->h_status->flags & GSR_STATUS_OVERFLOW) return fail(ctx, GSR_E_CAPACITY, "gsr_copy_pairs: last render overflowed");
    if (capacity < *n_pairs) return fail(ctx, GSR_E_CAPACITY, "gsr_copy_pairs: capacity %lld < %lld pairs", (long long)capacity, (long long)*n_pairs);
    HIPCHK(ctx, launch_copy_pairs(ctx->last, keys, values, ranges, ctx->last_stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->last_stream));
    return GSR_OK;
}

int gsr_copy_pixel_state(gsr_context* ctx, float* T_final, uint32_t* n_contrib) {
    if (!ctx) return fail(nullptr, GSR_E_INVALID, "gsr_copy_pixel_state: ctx is NULL");
    if (ctx->last_groups > 1)
        return fail(ctx, GSR_E_STATE, "gsr_copy_pixel_state: the last render was split into stream groups");
    if (!ctx->have_last) return fail(ctx, GSR_E_STATE, "gsr_copy_pixel_state: nothing rendered yet");
    hipSetDevice(ctx->device);
    const size_t npix = (size_t)ctx->last.images * ctx->last.width * ctx->last.height;
    if (T_final) HIPCHK(ctx, hipMemcpyAsync(T_final, ctx->T_final.p, npix * sizeof(float), hipMemcpyDeviceToDevice, ctx->last_stream));
    if (n_contrib) HIPCHK(ctx, hipMemcpyAsync(n_contrib, ctx->n_contrib.p, npix * sizeof(uint32_t), hipMemcpyDeviceToDevice, ctx->last_stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->last_stream));
    return GSR_OK;
}

int gsr_saved_render(const gsr_context* ctx, uint64_t* render_id, int32_t* images, int32_t* width,
                     int32_t* height) {
    if (!ctx || !render_id) return fail(nullptr, GSR_E_INVALID, "gsr_saved_render: NULL argument");
    const bool ok = ctx->have_last && ctx->saved && ctx->saved_id != 0;
    *render_id = ok ? ctx->saved_id : 0;
    if (images) *images = ok ? ctx->last.images : 0;
    if (width) *width = ok ? ctx->last.width : 0;
    if (height) *height = ok ? ctx->last.height : 0;
    return GSR_OK;
}

}  // extern "C"

// Shared by both backward entry points: checks, then the launches with the given scratch.
static int backward_check(gsr_context* ctx, const gsr_scene* sc, uint64_t render_id, const float* d_rgb,
                          const gsr_gaussian_grads* grads, const char* who) {
    if (!ctx) return fail(nullptr, GSR_E_INVALID, "%s: ctx is NULL", who);
    if (!sc || !d_rgb || !grads) return fail(ctx, GSR_E_INVALID, "%s: NULL scene, d_rgb or grads", who);
    if (!ctx->have_last || !ctx->saved || ctx->last_scene != sc || ctx->last_scene_version != sc->version)
        return fail(ctx, GSR_E_STATE, "%s: no saved forward for this scene", who);
    if (render_id != ctx->saved_id)
        return fail(ctx, GSR_E_STATE, "%s: render %llu is not the saved one (%llu): a later render replaced its state",
                    who, (unsigned long long)render_id, (unsigned long long)ctx->saved_id);
    return GSR_OK;
}

static int backward_launch(gsr_context* ctx, const gsr_scene* sc, const float* d_rgb, const float* d_depth,
                           const float* d_alpha, const gsr_gaussian_grads* grads, float* d_poses, float* g2d,
                           gsr_gaussian_grads* grads_dev, float* pose_part, hipStream_t s) {
    BwdArgs b;
    memset(&b, 0, sizeof b);
    b.f = ctx->last;
    b.d_rgb = d_rgb;
    b.d_depth = d_depth;
    b.d_alpha = d_alpha;
    b.d_poses = d_poses;
    b.g2d = g2d;
    b.grads_dev = grads_dev;
    b.pose_part = pose_part;
    // the gradient descriptors travel as kernel arguments (no host staging, nothing to wait for)
    HIPCHK(ctx, launch_set_grads(grads, sc->n_nodes, grads_dev, s));
    HIPCHK(ctx, launch_backward(b, (size_t)b.f.C * (size_t)sc->total, s));
    ctx->last_stream = s;
    return GSR_OK;
}

// Scratch of gsr_render_backward_noalloc: per-record gradients, the device copy of the
// gradient descriptors and per-block pose sums, in this file-scope array.  Host code never
// uses the array's name as an address: gsr_create looks up its device address once per
// device (g_scratch_ptr) and only that pointer reaches kernels.
constexpr size_t kScratchBytes = 256ull << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
static void* g_scratch_ptr[kMaxDevices] = {};

static int scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return fail(nullptr, GSR_E_UNSUPPORTED, "device %d beyond %d", device, kMaxDevices);
    if (g_scratch_ptr[device]) return GSR_OK;
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return fail(nullptr, GSR_E_HIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", device, hipGetErrorString(e));
    }
    g_scratch_ptr[device] = p;
    return GSR_OK;
}

static size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

extern "C" {

int gsr_render_backward(gsr_context* ctx, const gsr_scene* sc, uint64_t render_id, const float* d_rgb,
                        const float* d_depth, const float* d_alpha, const gsr_gaussian_grads* grads, float* d_poses,
                        void* stream) {
    int r = backward_check(ctx, sc, render_id, d_rgb, grads, "gsr_render_backward");
    if (r) return r;
    hipSetDevice(ctx->device);
    const size_t nrec = (size_t)ctx->last.C * (size_t)sc->total;
    if ((r = ensure(ctx, ctx->g2d, nrec * 12)) || (r = ensure(ctx, ctx->grads_dev, (size_t)sc->n_nodes)) ||
        (r = ensure(ctx, ctx->pose_part, (size_t)std::max(ctx->last.n_blocks, 1) * 8)))
        return r;
    return backward_launch(ctx, sc, d_rgb, d_depth, d_alpha, grads, d_poses, ctx->g2d.p, ctx->grads_dev.p,
                           ctx->pose_part.p, (hipStream_t)stream);
}

int gsr_render_backward_noalloc(gsr_context* ctx, const gsr_scene* sc, uint64_t render_id, const float* d_rgb,
                                const float* d_depth, const float* d_alpha, const gsr_gaussian_grads* grads,
                                float* d_poses, void* stream) {
    int r = backward_check(ctx, sc, render_id, d_rgb, grads, "gsr_render_backward_noalloc");
    if (r) return r;
    if (ctx->device < 0 || ctx->device >= kMaxDevices || !g_scratch_ptr[ctx->device])
        return fail(ctx, GSR_E_STATE, "gsr_render_backward_noalloc: no scratch address for device %d", ctx->device);
    const size_t nrec = (size_t)ctx->last.C * (size_t)sc->total;
    const size_t b_desc = align256(sizeof(gsr_gaussian_grads) * (size_t)sc->n_nodes);
    const size_t b_pose = align256(sizeof(float) * 8 * (size_t)std::max(ctx->last.n_blocks, 1));
    const size_t b_g2d = sizeof(float) * 12 * nrec;
    if (b_desc + b_pose + b_g2d > kScratchBytes)
        return fail(ctx, GSR_E_CAPACITY,
                    "gsr_render_backward_noalloc: needs %zu bytes of scratch (%zu records, %d nodes), the static "
                    "scratch holds %zu",
                    b_desc + b_pose + b_g2d, nrec, sc->n_nodes, kScratchBytes);
    hipSetDevice(ctx->device);
    unsigned char* base = (unsigned char*)g_scratch_ptr[ctx->device];
    return backward_launch(ctx, sc, d_rgb, d_depth, d_alpha, grads, d_poses, (float*)(base + b_desc + b_pose),
                           (gsr_gaussian_grads*)base, (float*)(base + b_desc), (hipStream_t)stream);
}

int gsr_autotune(gsr_context* ctx, const gsr_scene* sc, int32_t C, const gsr_camera* cams, int32_t W, int32_t H,
                 float* rgb, float* depth, float* alpha, int32_t* tile_w, int32_t* tile_h, int32_t* persistent,
                 void* stream) {
    if (!ctx) return fail(nullptr, GSR_E_INVALID, "gsr_autotune: ctx is NULL");
    if (!sc || !cams || !rgb || !depth) return fail(ctx, GSR_E_INVALID, "gsr_autotune: NULL argument");
    hipSetDevice(ctx->device);
    auto key = std::make_tuple(sc->n_envs * C, (int)W, (int)H, sc->total);
    auto it = ctx->tune.find(key);
    if (it == ctx->tune.end()) {
        hipStream_t s = (hipStream_t)stream;
        const int shapes[4][2] = {{16, 16}, {16, 8}, {8, 8}, {32, 8}};
        float best = 1e30f;
        std::tuple<int, int, int, int, int> choice{16, 16, 0, 2, 1};
        ctx->cfg.stream_groups = 1;  // tile shapes are compared on one group
        hipEvent_t e0, e1;
        HIPCHK(ctx, hipEventCreate(&e0));
        HIPCHK(ctx, hipEventCreate(&e1));
        for (auto& sh : shapes) {
            for (int ppt = 1; ppt <= 4; ppt *= 2) {
                if (ppt > sh[0] * sh[1] / 64) continue;
                for (int pers = 0; pers < 2; ++pers) {
                    int r = gsr_set_tile(ctx, sh[0], sh[1]);
                    if (!r) r = gsr_set_pixels_per_thread(ctx, ppt);
                    if (r) return r;
                    const uint32_t fl = pers ? GSR_FLAG_PERSISTENT : 0u;
                    r = gsr_render_rgbd(ctx, sc, C, cams, W, H, rgb, depth, alpha, fl | GSR_FLAG_CHECK, stream);
                    if (r) return r;
                    float ms = 0.0f;
                    HIPCHK(ctx, hipEventRecord(e0, s));
                    for (int it2 = 0; it2 < 3; ++it2) {
                        r = gsr_render_rgbd(ctx, sc, C, cams, W, H, rgb, depth, alpha, fl, stream);
                        if (r) return r;
                    }
                    HIPCHK(ctx, hipEventRecord(e1, s));
                    HIPCHK(ctx, hipEventSynchronize(e1));
                    HIPCHK(ctx, hipEventElapsedTime(&ms, e0, e1));
                    // a later candidate must be 2% faster: timing noise does not flip near-ties
                    if (ms < 0.98f * best) {
                        best = ms;
                        choice = std::make_tuple(sh[0], sh[1], pers, ppt, 1);
                    }
                }
            }
        }
        // stream groups with the chosen shape (several environments only), timed as replays of
        // their graphs (one group included), since their gain is the overlap of whole renders
        if (sc->n_envs >= 2) {
            const uint32_t fl = std::get<2>(choice) ? GSR_FLAG_PERSISTENT : 0u;
            float best_g = 1e30f;
            for (int G = 1; G <= std::min(3, sc->n_envs); ++G) {
                int r = gsr_set_tile(ctx, std::get<0>(choice), std::get<1>(choice));
                if (!r) r = gsr_set_pixels_per_thread(ctx, std::get<3>(choice));
                if (!r) r = gsr_set_stream_groups(ctx, G);
                if (!r) r = gsr_render_rgbd(ctx, sc, C, cams, W, H, rgb, depth, alpha, fl | GSR_FLAG_CHECK, stream);
                if (!r) r = gsr_render_rgbd(ctx, sc, C, cams, W, H, rgb, depth, alpha, fl | GSR_FLAG_GRAPH, stream);
                if (r) return r;
                float ms = 0.0f;
                HIPCHK(ctx, hipEventRecord(e0, s));
                for (int it2 = 0; it2 < 5; ++it2) {
                    r = gsr_render_rgbd(ctx, sc, C, cams, W, H, rgb, depth, alpha, fl | GSR_FLAG_GRAPH, stream);
                    if (r) return r;
                }
                HIPCHK(ctx, hipEventRecord(e1, s));
                HIPCHK(ctx, hipEventSynchronize(e1));
                HIPCHK(ctx, hipEventElapsedTime(&ms, e0, e1));
                if (ms < 0.98f * best_g) {
                    best_g = ms;
                    std::get<4>(choice) = G;
                }
            }
        }
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        it = ctx->tune.emplace(key, choice).first;
    }
    int r = gsr_set_tile(ctx, std::get<0>(it->second), std::get<1>(it->second));
    if (!r) r = gsr_set_pixels_per_thread(ctx, std::get<3>(it->second));
    if (!r) r = gsr_set_stream_groups(ctx, std::get<4>(it->second));
    if (r) return r;
    if (tile_w) *tile_w = std::get<0>(it->second);
    if (tile_h) *tile_h = std::get<1>(it->second);
    if (persistent) *persistent = std::get<2>(it->second);
    return GSR_OK;
}

}  // extern "C"
