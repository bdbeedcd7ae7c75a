// Many volumes of uneven size and many views in one persistent launch.
//
// One workgroup of 1024 threads per compute unit pops tasks from a device
// queue (an atomic counter over a task table built on the host).  The table
// lists every task of every volume phase by phase:
//   HIST   histogram of a run of voxels of a volume (or of its top slices)
//   SEL1   per-chunk pass of the threshold selection      (after all HIST)
//   SEL2   per-chunk search                                (after all SEL1)
//   SEL3   finish: threshold, keep mask; clears the histograms for the next
//          launch and the occupancy for this one          (after all SEL2)
//   DOWN   fused threshold + level-1 tiles                 (after SEL3)
//   BRICK  level 1 to the brick layout + occupancy         (after all DOWN)
//   RENDER one ray tile of one view                        (after all BRICK)
// RENDER tiles are not run by the persistent kernel: its 128 KiB LDS union
// (sized by the histogram) and 128 registers leave four waves per SIMD,
// half of what the ray caster runs at.  A second kernel, launched behind it
// on the same stream (and captured into the same graph), renders every tile
// of every item in one-wave workgroups, 16 per tile, with the TF knots in
// 4 KiB of LDS; stream order makes every brick complete before it starts.
// A task waits (thread 0 spins with agent-scope acquire loads) until the
// counters of the phase it depends on reach their totals; a finished task
// bumps its phase counter with a release.  Tasks are claimed in table order
// and depend only on earlier tasks, so the lowest claimed unfinished task is
// always runnable: no deadlock, whatever the residency.  Spins are bounded;
// on a time-out the workgroup records an error flag and moves on, so every
// wave exits.  The last workgroup to finish resets the queue and counters, so
// the launch can be replayed (HIP graph) without host work.
#include <algorithm>
#include <cstring>
#include <vector>

#include "brick_dev.h"
#include "downsample_dev.h"
#include "hist_dev.h"
#include "raycast_dev.h"
#include "select_dev.h"

namespace {

constexpr int kT = 1024;
enum TaskType { T_HIST = 0, T_SEL1, T_SEL2, T_SEL3, T_DOWN, T_BRICK, T_RENDER };
enum Counter { C_HIST = 0, C_SEL1, C_SEL2, C_SEL3, C_DOWN, C_BRICK, C_COUNT };
constexpr uint64_t kSpinLimit = 1ull << 26;     // polls (with sleeps) before giving up

struct Task {
    int32_t type, item;
    int64_t a, b;            // meaning depends on the type
};

struct ItemDev {
    const uint16_t* vol;
    int nx, ny, nz, aligned;
    uint64_t* H;
    uint64_t* Ht;
    uint32_t* result;
    uint32_t* keep;
    int64_t top_voxels;
    uint16_t* level1;
    int lx, ly, lz;
    int down_tiles_x, down_tiles_y;
    uint16_t* bricked;
    uint8_t* occ;
    int64_t occ_bytes;
    int nbx, nby, nbz, nmx, nmy, nslab_x;
    float* frames;
    int n_views;
    int need[C_COUNT];       // tasks each phase must finish
    vr::rc::Scene S;
    vr::rc::Views V;
};

struct BatchDev {
    const ItemDev* items;
    const Task* tasks;
    int64_t n_tasks;
    uint32_t* counters;      // [n_items][C_COUNT]
    uint32_t* head;          // queue position
    uint32_t* finished;      // workgroups done
    uint32_t* status;        // non-zero after a spin time-out
    int64_t n_pre;           // tasks before the render phase (the workgroup queue)
    int64_t n_render_waves;  // render pieces: 16 waves per render tile (the render launch)
    unsigned long long* samples;   // [2] samples taken / evaluated (accumulated)
    const float4* tf;
    int n_items;
    int rule, rule_param, n_chunks;
    int wave_w, wave_h, waves_x;   // render tile: waves of wave_w x wave_h pixels, waves_x across
    int tiles_per_row;             // render tiles across an image
    int brick8;                    // level 1 in 8^3 bricks (else 4^3)
};

union BatchLds {
    uint32_t hist[vr::hg::kWords];
    vr::sel::SelLds sel;
    struct {
        uint32_t bits[VR_KEEP_WORDS];
        vr::ds::TileLds g[kT / vr::ds::kThreads];
        uint32_t first, bad;
    } down;
    vr::bk::SlabLds<uint16_t> brick[kT / vr::bk::kThreads];
};

__device__ inline void wait_ge(const BatchDev& B, const uint32_t* c, uint32_t need)
{
    if (threadIdx.x == 0) {
        uint64_t spins = 0;
        while (__hip_atomic_load(c, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < need) {
            __builtin_amdgcn_s_sleep(2);
            if (++spins > kSpinLimit) {
                __hip_atomic_fetch_or(B.status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
    }
    __syncthreads();
}

__device__ inline void signal(uint32_t* c)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        __hip_atomic_fetch_add(c, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__device__ inline void zero_u64(uint64_t* p, int n)
{
    for (int i = threadIdx.x; i < n; i += kT) p[i] = 0;
}

__device__ void run_task(const BatchDev& B, const Task& t, BatchLds& L)
{
    const ItemDev& it = B.items[t.item];
    uint32_t* cnt = B.counters + (int64_t)t.item * C_COUNT;
    const int tid = threadIdx.x;
    switch (t.type) {
    case T_HIST: {
        // a = first voxel, b = voxel count; item.top_voxels > 0 marks the top-slice run
        uint64_t* gh = t.b < 0 ? it.Ht : it.H;
        const int64_t n = t.b < 0 ? -t.b : t.b;
        vr::hg::zero_lds(L.hist);
        __syncthreads();
        vr::hg::count_range(L.hist, gh, it.vol + t.a, n, tid, kT);
        __syncthreads();
        vr::hg::flush_lds(L.hist, gh);
        signal(cnt + C_HIST);
        break;
    }
    case T_SEL1:
        wait_ge(B, cnt + C_HIST, it.need[C_HIST]);
        vr::sel::chunk_pass(L.sel, (int)t.a, it.H, B.rule, B.rule_param, it.keep);
        signal(cnt + C_SEL1);
        break;
    case T_SEL2:
        wait_ge(B, cnt + C_SEL1, it.need[C_SEL1]);
        vr::sel::chunk_search(L.sel, (int)t.a, it.H, B.rule, B.rule_param, B.n_chunks, it.keep);
        signal(cnt + C_SEL2);
        break;
    case T_SEL3:
        wait_ge(B, cnt + C_HIST, it.need[C_HIST]);
        wait_ge(B, cnt + C_SEL2, it.need[C_SEL2]);
        if (it.need[C_SEL2] == 0) wait_ge(B, cnt + C_SEL1, it.need[C_SEL1]);
        vr::sel::finish(L.sel, it.H, it.Ht, B.rule, B.rule_param, B.n_chunks, it.result, it.keep);
        __syncthreads();
        // the histograms start the next launch from zero; the occupancy this one
        zero_u64(it.H, VR_NBINS);
        zero_u64(it.Ht, VR_NBINS);
        for (int64_t i = tid; i < it.occ_bytes; i += kT) it.occ[i] = 0;
        signal(cnt + C_SEL3);
        break;
    case T_DOWN: {
        // tiles [a, b): four 256-thread groups, one tile each per round
        wait_ge(B, cnt + C_SEL3, 1);
        const uint32_t T = vr::ds::load_mask(it.keep, L.down.bits, L.down.first, L.down.bad);
        vr::ds::LevelOut lo{};
        lo.p[0] = it.level1;
        lo.nx[0] = it.lx;
        lo.ny[0] = it.ly;
        lo.nz[0] = it.lz;
        const int g = tid / vr::ds::kThreads, lt = tid % vr::ds::kThreads;
        const int groups = kT / vr::ds::kThreads;
        const int n_tiles = it.down_tiles_x * it.down_tiles_y * ((it.nz + vr::ds::TZ - 1) / vr::ds::TZ);
        for (int64_t base = t.a; base < t.b; base += groups) {
            const int tile = (int)(base + g);
            const bool active = tile < t.b && tile < n_tiles;
            if (T <= VR_NBINS)
                vr::ds::tile_body<true>(it.vol, it.nx, it.ny, it.nz, it.aligned, L.down.bits, T, 1, lo,
                                        it.down_tiles_x, it.down_tiles_y, active ? tile : 0, active, lt, L.down.g[g]);
            else
                vr::ds::tile_body<false>(it.vol, it.nx, it.ny, it.nz, it.aligned, L.down.bits, 0u, 1, lo,
                                         it.down_tiles_x, it.down_tiles_y, active ? tile : 0, active, lt, L.down.g[g]);
        }
        signal(cnt + C_DOWN);
        break;
    }
    case T_BRICK: {
        wait_ge(B, cnt + C_DOWN, it.need[C_DOWN]);
        if (B.brick8) {
            // 8-voxel row pieces [a, b), one per thread
            for (int64_t r = t.a + tid; r < t.b; r += kT)
                vr::bk::row8_body<uint16_t>(it.level1, it.lx, it.ly, it.lz, it.nbx, it.nby, it.bricked, it.occ,
                                            it.occ + (int64_t)it.nbx * it.nby * it.nbz, it.nmx, it.nmy, 0u, r);
            signal(cnt + C_BRICK);
            break;
        }
        // slabs [a, b): slab s = (bz * nby + by) * nslab_x + sx
        const int g = tid / vr::bk::kThreads, lt = tid % vr::bk::kThreads;
        const int groups = kT / vr::bk::kThreads;
        const int64_t n_slabs = (int64_t)it.nslab_x * it.nby * it.nbz;
        for (int64_t base = t.a; base < t.b; base += groups) {
            const int64_t s = base + g;
            const bool active = s < t.b && s < n_slabs;
            const int64_t ss = active ? s : 0;
            const int sx = (int)(ss % it.nslab_x);
            const int by = (int)((ss / it.nslab_x) % it.nby);
            const int bz = (int)(ss / ((int64_t)it.nslab_x * it.nby));
            vr::bk::slab_body<uint16_t>(it.level1, it.lx, it.ly, it.lz, it.nbx, it.nby, it.bricked, it.occ,
                                        it.occ + (int64_t)it.nbx * it.nby * it.nbz, it.nmx, it.nmy,
                                        0u, sx * 16, by, bz, active, lt, L.brick[g]);
        }
        signal(cnt + C_BRICK);
        break;
    }
    default:
        break;
    }
}

// The render launch: workgroup b (in XCD-aware order, so that an XCD renders
// consecutive pieces) is wave r % 16 of render tile r / 16 (the render tasks
// at the end of the table), the pieces of one tile being consecutive so that
// neighbouring waves render neighbouring pixels.
__global__ void __launch_bounds__(64) batch_render_kernel(const BatchDev B)
{
    __shared__ vr::rc::TfLds tf;
    vr::rc::stage_tf(tf, B.tf, (int)threadIdx.x, 64);
    __syncthreads();
    const uint32_t r = (uint32_t)vr::rc::xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const int lane = threadIdx.x & 63;
    const int tile_w = B.wave_w * B.waves_x, tile_h = B.wave_h * (16 / B.waves_x);
    const Task t = B.tasks[B.n_pre + r / 16];
    const int w = (int)(r % 16);
    const ItemDev& it = B.items[t.item];
    const vr::rc::Scene& S = it.S;
    const bool skip = vr::rc::can_skip(S, tf);
    const int tx = (int)(t.b % B.tiles_per_row), ty = (int)(t.b / B.tiles_per_row);
    const int i = tx * tile_w + (w % B.waves_x) * B.wave_w + lane % B.wave_w;
    const int j = ty * tile_h + (w / B.waves_x) * B.wave_h + lane / B.wave_w;
    uint32_t cr = 0, er = 0;
    if (i < S.W && j < S.H) {
        const float4 rgba =
            B.brick8 ? vr::rc::march<uint16_t, VR_LAYOUT_BRICK8, true, false, false>(
                           S, it.V.v[t.a], it.bricked, tf, skip, i, j, cr, er)
                     : vr::rc::march<uint16_t, VR_LAYOUT_BRICK4, true, false, false>(
                           S, it.V.v[t.a], it.bricked, tf, skip, i, j, cr, er);
        reinterpret_cast<float4*>(it.frames)[((int64_t)t.a * S.H + j) * S.W + i] = rgba;
    }
    if (B.samples) {
        unsigned long long c = cr, e = er;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            c += __shfl_xor(c, off);
            e += __shfl_xor(e, off);
        }
        if (lane == 0 && c) atomicAdd(B.samples, c);
        if (lane == 0 && e) atomicAdd(B.samples + 1, e);
    }
}

__global__ void __launch_bounds__(kT) batch_kernel(const BatchDev B)
{
    __shared__ BatchLds L;
    __shared__ int64_t s_task[2];
    if (threadIdx.x == 0)
        s_task[0] = __hip_atomic_fetch_add(B.head, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    for (;;) {
        const int64_t cur = s_task[0];
        if (cur >= B.n_pre) break;
        // claim the next task now, so its queue latency overlaps this one
        if (threadIdx.x == 0)
            s_task[1] = __hip_atomic_fetch_add(B.head, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const Task t = B.tasks[cur];
        run_task(B, t, L);
        __syncthreads();
        if (threadIdx.x == 0) s_task[0] = s_task[1];
        __syncthreads();
    }
    __syncthreads();
    // the last workgroup out resets the queues for the next launch
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t done = __hip_atomic_fetch_add(B.finished, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (done == gridDim.x - 1) {
            for (int64_t i = 0; i < (int64_t)B.n_items * C_COUNT; ++i) B.counters[i] = 0;
            *B.head = 0;
            __threadfence();
            __hip_atomic_store(B.finished, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Carves the workspace: a bump allocator over the caller's buffer.
struct Carver {
    char* base;
    size_t used, cap;
    void* take(size_t bytes)
    {
        used = align_up(used, 256);
        void* p = base ? base + used : nullptr;
        used += bytes;
        return p;
    }
};

}  // namespace

struct vr_batch_plan {
    BatchDev dev{};
    int grid = 0;
    std::vector<ItemDev> items;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int device = 0;
};

namespace {

int layout_plan(const vr_batch_item* items, int n_items, const vr_batch_config* cfg, Carver& C,
                vr_batch_plan* P, std::vector<Task>* tasks)
{
    VR_REQUIRE(items && cfg && n_items >= 1, VR_ERR_NULL, "vr_batch: NULL argument");
    VR_REQUIRE(cfg->rule == VR_RULE_VALLEY || cfg->rule == VR_RULE_OTSU || cfg->rule == VR_RULE_ITS ||
                   cfg->rule == VR_RULE_NONE, VR_ERR_RANGE, "vr_batch: rule %d", cfg->rule);
    VR_REQUIRE(cfg->rule != VR_RULE_VALLEY || (cfg->rule_param >= 1 && cfg->rule_param <= 1023),
               VR_ERR_RANGE, "vr_batch: smoothing radius %d", cfg->rule_param);
    VR_REQUIRE(cfg->rule == VR_RULE_VALLEY || cfg->rule == VR_RULE_NONE ||
                   (cfg->rule_param >= 0 && cfg->rule_param <= 12), VR_ERR_RANGE,
               "vr_batch: bin width shift %d", cfg->rule_param);
    const int ww = cfg->wave_w, wh = cfg->wave_h, wx = cfg->waves_x;
    VR_REQUIRE(ww >= 1 && wh >= 1 && ww * wh == 64 && wx >= 1 && 16 % wx == 0, VR_ERR_RANGE,
               "vr_batch: ray tile %d x %d pixels per wave, %d waves across", ww, wh, wx);
    VR_REQUIRE(cfg->top_slices >= 1, VR_ERR_RANGE, "vr_batch: top_slices %d", cfg->top_slices);
    VR_REQUIRE(cfg->hist_task_voxels >= 8192, VR_ERR_RANGE, "vr_batch: hist_task_voxels %lld",
               (long long)cfg->hist_task_voxels);
    VR_REQUIRE(cfg->down_tiles_per_task >= 1 && cfg->slabs_per_task >= 1 && cfg->render_tiles_per_task == 1,
               VR_ERR_RANGE, "vr_batch: task sizes");
    VR_REQUIRE(cfg->brick_edge == 0 || cfg->brick_edge == 4 || cfg->brick_edge == 8, VR_ERR_RANGE,
               "vr_batch: brick edge %d (4 or 8)", cfg->brick_edge);
    const bool b8 = cfg->brick_edge == 8;
    const int be = b8 ? 8 : 4;

    const int bins = cfg->rule == VR_RULE_VALLEY || cfg->rule == VR_RULE_NONE ? VR_NBINS : (VR_NBINS >> cfg->rule_param);
    const int n_chunks = (bins + kT - 1) / kT;
    const int tile_w = ww * wx, tile_h = wh * (16 / wx);
    const int tiles_per_row = (cfg->width + tile_w - 1) / tile_w;
    const int tiles_per_col = (cfg->height + tile_h - 1) / tile_h;

    P->items.assign(n_items, ItemDev{});
    std::vector<std::vector<Task>> phase(7);
    for (int v = 0; v < n_items; ++v) {
        const vr_batch_item& in = items[v];
        ItemDev& it = P->items[v];
        VR_REQUIRE(in.d_vol && in.d_frames && in.h_cams, VR_ERR_NULL, "vr_batch: item %d has a NULL pointer", v);
        VR_REQUIRE(in.nx >= 1 && in.ny >= 1 && in.nz >= 1 && in.nx < (1 << 20) && in.ny < (1 << 20) &&
                       in.nz < (1 << 20), VR_ERR_DIMS, "vr_batch: item %d dims", v);
        VR_REQUIRE(in.n_views >= 1 && in.n_views <= VR_MAX_VIEWS_PER_LAUNCH, VR_ERR_RANGE,
                   "vr_batch: item %d has %d views (1..%d)", v, in.n_views, VR_MAX_VIEWS_PER_LAUNCH);
        VR_REQUIRE(cfg->top_slices <= in.nz, VR_ERR_RANGE, "vr_batch: item %d has fewer slices than top_slices", v);
        it.vol = in.d_vol;
        it.nx = (int)in.nx;
        it.ny = (int)in.ny;
        it.nz = (int)in.nz;
        it.aligned = (in.nx % 8 == 0) && ((reinterpret_cast<uintptr_t>(in.d_vol) & 15u) == 0);
        it.H = static_cast<uint64_t*>(C.take(VR_NBINS * 8));
        it.Ht = static_cast<uint64_t*>(C.take(VR_NBINS * 8));
        it.result = static_cast<uint32_t*>(C.take(16));
        it.keep = static_cast<uint32_t*>(C.take(VR_KEEP_WORDS * 4));
        it.lx = (it.nx + 1) / 2;
        it.ly = (it.ny + 1) / 2;
        it.lz = (it.nz + 1) / 2;
        it.level1 = static_cast<uint16_t*>(C.take((size_t)it.lx * it.ly * it.lz * 2));
        it.down_tiles_x = (it.nx + vr::ds::TX - 1) / vr::ds::TX;
        it.down_tiles_y = (it.ny + vr::ds::TY - 1) / vr::ds::TY;
        it.nbx = (it.lx + be - 1) / be;
        it.nby = (it.ly + be - 1) / be;
        it.nbz = (it.lz + be - 1) / be;
        it.nmx = (it.nbx + 3) / 4;
        it.nmy = (it.nby + 3) / 4;
        const int nmz = (it.nbz + 3) / 4;
        it.nslab_x = (it.nbx + 15) / 16;
        const int64_t nbricks = (int64_t)it.nbx * it.nby * it.nbz;
        it.occ_bytes = nbricks + (int64_t)it.nmx * it.nmy * nmz;
        // the bricks and their apron (not cleared: the ray caster gives apron taps weight 0)
        it.bricked = static_cast<uint16_t*>(
            C.take((size_t)(nbricks + vr::bk::apron_bricks(it.nbx, it.nby)) * be * be * be * 2));
        it.occ = static_cast<uint8_t*>(C.take((size_t)it.occ_bytes));
        it.frames = in.d_frames;
        it.n_views = in.n_views;
        it.top_voxels = (int64_t)it.nx * it.ny * cfg->top_slices;

        // render scene of level 1 (bricked, with occupancy); spacing is the level's voxel
        vr_volume vol{};
        vol.data = it.bricked ? it.bricked : reinterpret_cast<const void*>(16);
        vol.dtype = VR_U16_NORM;
        vol.layout = b8 ? VR_LAYOUT_BRICK8 : VR_LAYOUT_BRICK4;
        vol.nx = it.lx;
        vol.ny = it.ly;
        vol.nz = it.lz;
        for (int a = 0; a < 3; ++a) vol.spacing[a] = in.spacing[a] > 0.0 ? in.spacing[a] : 1.0;
        vol.occupancy = it.occ;
        vr_render_opts o{};
        o.width = cfg->width;
        o.height = cfg->height;
        o.step = cfg->step;
        o.ert_eps = cfg->ert_eps;
        for (int c = 0; c < 4; ++c) o.bg[c] = cfg->bg[c];
        int rc = vr::rc::build_scene(&vol, reinterpret_cast<const float*>(16), in.h_cams, in.n_views, &o, it.S);
        if (rc) return rc;
        VR_REQUIRE(!vr::rc::needs_wide(it.S), VR_ERR_DIMS,
                   "vr_batch_plan_create: item %d has a level of more than 2^24 bricks", v);
        it.S.data = it.bricked;
        it.S.occ = it.occ;
        it.S.dist = nullptr;     // the batch keeps the marks and the group marks only
        it.S.view0 = 0;
        rc = vr::rc::build_views(in.h_cams, in.n_views, it.V);
        if (rc) return rc;

        // tasks
        const int64_t nvox = (int64_t)it.nx * it.ny * it.nz;
        const int64_t per = std::max<int64_t>(cfg->hist_task_voxels, 8192);
        int n_hist = 0;
        for (int64_t a = 0; a < nvox; a += per, ++n_hist)
            phase[T_HIST].push_back({T_HIST, v, a, std::min(per, nvox - a)});
        phase[T_HIST].push_back({T_HIST, v, 0, -it.top_voxels});
        it.need[C_HIST] = n_hist + 1;
        if (cfg->rule != VR_RULE_NONE) {
            for (int c = 0; c < n_chunks; ++c) phase[T_SEL1].push_back({T_SEL1, v, c, 0});
            it.need[C_SEL1] = n_chunks;
            if (cfg->rule != VR_RULE_ITS) {
                for (int c = 0; c < n_chunks; ++c) phase[T_SEL2].push_back({T_SEL2, v, c, 0});
                it.need[C_SEL2] = n_chunks;
            }
        }
        phase[T_SEL3].push_back({T_SEL3, v, 0, 0});
        it.need[C_SEL3] = 1;
        const int64_t n_tiles = (int64_t)it.down_tiles_x * it.down_tiles_y * ((it.nz + vr::ds::TZ - 1) / vr::ds::TZ);
        int n_down = 0;
        for (int64_t a = 0; a < n_tiles; a += cfg->down_tiles_per_task, ++n_down)
            phase[T_DOWN].push_back({T_DOWN, v, a, std::min<int64_t>(n_tiles, a + cfg->down_tiles_per_task)});
        it.need[C_DOWN] = n_down;
        // 4^3: slabs of 16 bricks along x; 8^3: 8-voxel row pieces, 256 per slab's worth
        const int64_t n_units = b8 ? (int64_t)it.nbx * (it.nby * 8) * (it.nbz * 8)
                                   : (int64_t)it.nslab_x * it.nby * it.nbz;
        const int64_t per_task = b8 ? (int64_t)cfg->slabs_per_task * 256 : (int64_t)cfg->slabs_per_task;
        int n_brick = 0;
        for (int64_t a = 0; a < n_units; a += per_task, ++n_brick)
            phase[T_BRICK].push_back({T_BRICK, v, a, std::min<int64_t>(n_units, a + per_task)});
        it.need[C_BRICK] = n_brick;
        for (int view = 0; view < in.n_views; ++view)
            for (int tt = 0; tt < tiles_per_row * tiles_per_col; ++tt)
                phase[T_RENDER].push_back({T_RENDER, v, view, tt});
    }
    // the SEL1 phase waits on nothing it cannot see: when the rule is NONE,
    // SEL3 depends on the histograms directly
    if (cfg->rule == VR_RULE_NONE)
        for (auto& it : P->items) it.need[C_SEL2] = 0, it.need[C_SEL1] = 0;
    for (auto& ph : phase) tasks->insert(tasks->end(), ph.begin(), ph.end());
    const int64_t n_render = (int64_t)phase[T_RENDER].size();
    VR_REQUIRE(16 * n_render < (int64_t(1) << 31), VR_ERR_DIMS, "vr_batch: too many render tiles");

    BatchDev& B = P->dev;
    B.n_tasks = (int64_t)tasks->size();
    B.n_pre = B.n_tasks - n_render;
    B.n_render_waves = 16 * n_render;
    B.n_items = n_items;
    B.rule = cfg->rule;
    B.rule_param = cfg->rule_param;
    B.n_chunks = n_chunks;
    B.wave_w = ww;
    B.wave_h = wh;
    B.waves_x = wx;
    B.tiles_per_row = tiles_per_row;
    B.brick8 = b8 ? 1 : 0;
    B.items = static_cast<const ItemDev*>(C.take(sizeof(ItemDev) * n_items));
    B.tasks = static_cast<const Task*>(C.take(sizeof(Task) * tasks->size()));
    B.counters = static_cast<uint32_t*>(C.take(sizeof(uint32_t) * (C_COUNT * n_items + 3)));
    B.head = B.counters ? B.counters + C_COUNT * n_items : nullptr;
    B.finished = B.head ? B.head + 1 : nullptr;
    B.status = B.head ? B.head + 2 : nullptr;
    B.samples = static_cast<unsigned long long*>(C.take(16));
    return VR_OK;
}

}  // namespace

extern "C" int vr_batch_workspace_size(const vr_batch_item* items, int n_items, const vr_batch_config* cfg,
                                       int64_t* bytes)
{
    vr::clear_error();
    VR_REQUIRE(bytes != nullptr, VR_ERR_NULL, "vr_batch_workspace_size: bytes is NULL");
    vr_batch_plan P;
    Carver C{nullptr, 0, 0};
    std::vector<Task> tasks;
    int rc = layout_plan(items, n_items, cfg, C, &P, &tasks);
    if (rc) return rc;
    *bytes = (int64_t)align_up(C.used, 256);
    return VR_OK;
}

extern "C" int vr_batch_plan_create(const vr_batch_item* items, int n_items, const vr_batch_config* cfg,
                                    const float* d_tf, void* d_workspace, int64_t workspace_bytes,
                                    vr_batch_plan** plan)
{
    vr::clear_error();
    VR_REQUIRE(plan && d_tf && d_workspace, VR_ERR_NULL, "vr_batch_plan_create: NULL argument");
    *plan = nullptr;
    auto* P = new vr_batch_plan();
    Carver C{static_cast<char*>(d_workspace), 0, (size_t)workspace_bytes};
    std::vector<Task> tasks;
    int rc = layout_plan(items, n_items, cfg, C, P, &tasks);
    if (rc == VR_OK && (int64_t)C.used > workspace_bytes)
        rc = vr::fail(VR_ERR_WORKSPACE, "vr_batch_plan_create: workspace of %lld bytes, %lld needed",
                      (long long)workspace_bytes, (long long)C.used);
    if (rc) {
        delete P;
        return rc;
    }
    P->dev.tf = reinterpret_cast<const float4*>(d_tf);
    hipError_t e = hipGetDevice(&P->device);
    // descriptors and tasks to the device; counters, histograms and flags start at zero
    if (e == hipSuccess)
        e = hipMemcpy(const_cast<ItemDev*>(P->dev.items), P->items.data(), sizeof(ItemDev) * n_items,
                             hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(const_cast<Task*>(P->dev.tasks), tasks.data(), sizeof(Task) * tasks.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(P->dev.counters, 0, sizeof(uint32_t) * (C_COUNT * n_items + 3));
    if (e == hipSuccess) e = hipMemset(P->dev.samples, 0, 16);
    for (int v = 0; e == hipSuccess && v < n_items; ++v) {
        e = hipMemset(P->items[v].H, 0, VR_NBINS * 8);
        if (e == hipSuccess) e = hipMemset(P->items[v].Ht, 0, VR_NBINS * 8);
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        delete P;
        return vr::fail(VR_ERR_HIP, "vr_batch_plan_create: %s", hipGetErrorString(e));
    }
    // every workgroup of the persistent grid is resident: one per compute unit
    P->grid = vr::num_cus();
    *plan = P;
    return VR_OK;
}

extern "C" int vr_batch_launch(vr_batch_plan* plan, void* stream)
{
    vr::clear_error();
    VR_REQUIRE(plan != nullptr, VR_ERR_NULL, "vr_batch_launch: plan is NULL");
    hipStream_t s = vr::as_stream(stream);
    if (plan->exec) {
        const hipError_t e = hipGraphLaunch(plan->exec, s);
        VR_REQUIRE(e == hipSuccess, VR_ERR_HIP, "vr_batch_launch: %s", hipGetErrorString(e));
        return VR_OK;
    }
    batch_kernel<<<plan->grid, kT, 0, s>>>(plan->dev);
    if (plan->dev.n_render_waves > 0)
        batch_render_kernel<<<(unsigned)plan->dev.n_render_waves, 64, 0, s>>>(plan->dev);
    return vr::check_launch("vr_batch_launch");
}

extern "C" int vr_batch_capture(vr_batch_plan* plan, void* stream)
{
    vr::clear_error();
    VR_REQUIRE(plan != nullptr, VR_ERR_NULL, "vr_batch_capture: plan is NULL");
    VR_REQUIRE(plan->exec == nullptr, VR_ERR_RANGE, "vr_batch_capture: already captured");
    hipStream_t s = vr::as_stream(stream);
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    VR_REQUIRE(e == hipSuccess, VR_ERR_HIP, "vr_batch_capture: begin: %s", hipGetErrorString(e));
    batch_kernel<<<plan->grid, kT, 0, s>>>(plan->dev);
    if (plan->dev.n_render_waves > 0)
        batch_render_kernel<<<(unsigned)plan->dev.n_render_waves, 64, 0, s>>>(plan->dev);
    hipError_t le = hipGetLastError();
    e = hipStreamEndCapture(s, &plan->graph);
    VR_REQUIRE(le == hipSuccess && e == hipSuccess, VR_ERR_HIP, "vr_batch_capture: %s",
               hipGetErrorString(le != hipSuccess ? le : e));
    e = hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0);
    VR_REQUIRE(e == hipSuccess, VR_ERR_HIP, "vr_batch_capture: instantiate: %s", hipGetErrorString(e));
    return VR_OK;
}

extern "C" int vr_batch_status(vr_batch_plan* plan, uint32_t* h_status, uint64_t* h_samples)
{
    vr::clear_error();
    VR_REQUIRE(plan && h_status, VR_ERR_NULL, "vr_batch_status: NULL argument");
    hipError_t e = hipMemcpy(h_status, plan->dev.status, 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess && h_samples) e = hipMemcpy(h_samples, plan->dev.samples, 16, hipMemcpyDeviceToHost);
    VR_REQUIRE(e == hipSuccess, VR_ERR_HIP, "vr_batch_status: %s", hipGetErrorString(e));
    return VR_OK;
}

extern "C" int vr_batch_item_outputs(const vr_batch_plan* plan, int item, uint16_t** d_level1,
                                     uint32_t** d_result, int64_t* n_tasks)
{
    vr::clear_error();
    VR_REQUIRE(plan != nullptr, VR_ERR_NULL, "vr_batch_item_outputs: plan is NULL");
    VR_REQUIRE(item >= 0 && item < (int)plan->items.size(), VR_ERR_RANGE, "vr_batch_item_outputs: item %d", item);
    if (d_level1) *d_level1 = plan->items[item].level1;
    if (d_result) *d_result = plan->items[item].result;
    if (n_tasks) *n_tasks = plan->dev.n_tasks;
    return VR_OK;
}

extern "C" int vr_batch_plan_destroy(vr_batch_plan* plan)
{
    vr::clear_error();
    if (plan == nullptr) return VR_OK;
    hipError_t e = hipSuccess;
    if (plan->exec) e = hipGraphExecDestroy(plan->exec);
    if (plan->graph) {
        const hipError_t g = hipGraphDestroy(plan->graph);
        if (e == hipSuccess) e = g;
    }
    delete plan;
    VR_REQUIRE(e == hipSuccess, VR_ERR_HIP, "vr_batch_plan_destroy: %s", hipGetErrorString(e));
    return VR_OK;
}
