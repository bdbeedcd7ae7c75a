// Container removal (Section III-B): the circle of the cylindrical sample
// container in the top slice by the Hough transform of Ioannou et al. (a 2D
// accumulation of centre votes along gradient lines, then a histogram of
// radii about the centre found), and the discard of every voxel outside it.
//
// Steps on the device, each its own launch, no host synchronisation:
//   1. the largest squared Sobel gradient of the slice's interior;
//   2. the edge list: pixels whose squared gradient is at least 2^-shift of
//      it, gathered per workgroup in LDS and appended with one atomic each;
//   3. votes: one thread per (edge, step) adds one vote to the cell of the
//      digital line from the edge against its gradient, for the steps whose
//      distance along the line lies in [r_min, r_max] (integer arithmetic);
//   4. the accumulator summed over (2w+1)^2 boxes (rows through LDS, then
//      column windows) and its first maximum in row-major order, as one
//      64-bit key (box sum above, complemented pixel index below) under
//      atomicMax;
//   5. the radius histogram of the edges whose gradient points away from the
//      centre, and its first maximum, written with the centre as the record
//      [found, cx, cy, r, R, centre votes, radius count, edges].
// Every decision is integer arithmetic, so the record is exact.
#include <algorithm>
#include <mutex>

#include "disc_dev.h"

namespace {

using namespace vr::disc;

constexpr int kT = 256;
constexpr int kMaxSide = 8192;             // pixels per slice side
constexpr int kMaxRadius = 4096;
constexpr int kIdxBits = 26;               // 8192^2 pixel indices
constexpr uint64_t kIdxMask = (uint64_t(1) << kIdxBits) - 1;
constexpr int kSeg = 16;                   // rows per column-window thread
constexpr int kRadBits = 13;               // radius field of the radius key

struct Ws {
    unsigned long long* scal;   // [0] largest m2, [1] centre key, [2] edge count
    uint32_t* rhist;            // r_max + 1 radius counts
    uint32_t* acc;              // ny * nx votes
    uint64_t* box;              // ny * nx row box sums
    int4* edges;                // (x, y, gx, gy) of the edge pixels
};

int64_t align256(int64_t b) { return (b + 255) & ~int64_t(255); }

// Carves the workspace (base may be NULL to size it); returns the bytes used.
int64_t carve(void* base, int64_t nx, int64_t ny, int r_max, Ws* w)
{
    int64_t off = 0;
    char* p = static_cast<char*>(base);
    auto take = [&](int64_t bytes) {
        char* q = p ? p + off : nullptr;
        off += align256(bytes);
        return q;
    };
    Ws ws;
    ws.scal = reinterpret_cast<unsigned long long*>(take(3 * 8));
    ws.rhist = reinterpret_cast<uint32_t*>(take(4 * (int64_t)(r_max + 1)));
    ws.acc = reinterpret_cast<uint32_t*>(take(4 * nx * ny));
    ws.box = reinterpret_cast<uint64_t*>(take(8 * nx * ny));
    ws.edges = reinterpret_cast<int4*>(take(16 * std::max<int64_t>(1, (nx - 2) * (ny - 2))));
    if (w) *w = ws;
    return off;
}

__device__ __forceinline__ unsigned long long wave_max(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long u = __shfl_xor(v, o);
        v = u > v ? u : v;
    }
    return v;
}

__global__ void __launch_bounds__(kT) clear_ws(Ws w, int64_t n, int nr)
{
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) w.acc[i] = 0u;
    if (blockIdx.x == 0) {
        for (int i = threadIdx.x; i < nr; i += kT) w.rhist[i] = 0u;
        if (threadIdx.x < 3) w.scal[threadIdx.x] = 0ull;
    }
}

// 3 x 3 Sobel gradient at interior pixel (x, y)
__device__ __forceinline__ void sobel(const uint16_t* __restrict__ s, int64_t nx, int64_t x, int64_t y, int& gx,
                                      int& gy)
{
    const uint16_t* r0 = s + (y - 1) * nx + x;
    const uint16_t* r1 = r0 + nx;
    const uint16_t* r2 = r1 + nx;
    const int a = r0[-1], b = r0[0], c = r0[1], d = r1[-1], f = r1[1], g = r2[-1], h = r2[0], i = r2[1];
    gx = (c + 2 * f + i) - (a + 2 * d + g);
    gy = (g + 2 * h + i) - (a + 2 * b + c);
}

// block-level maximum, one atomic per workgroup
__global__ void __launch_bounds__(kT) grad_max(const uint16_t* __restrict__ s, int64_t nx, int64_t ny, Ws w)
{
    __shared__ unsigned long long red[kT / 64];
    const uint32_t iw = (uint32_t)(nx - 2), n = iw * (uint32_t)(ny - 2);
    unsigned long long m = 0;
    for (uint32_t q = blockIdx.x * kT + threadIdx.x; q < n; q += gridDim.x * kT) {
        int gx, gy;
        sobel(s, nx, 1 + q % iw, 1 + q / iw, gx, gy);
        const unsigned long long m2 = (unsigned long long)((int64_t)gx * gx + (int64_t)gy * gy);
        m = m2 > m ? m2 : m;
    }
    m = wave_max(m);
    if (__lane_id() == 0) red[threadIdx.x / 64] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < kT / 64; ++i) m = red[i] > m ? red[i] : m;
        if (m) atomicMax(w.scal, m);
    }
}

constexpr int kEdgeBuf = 2048;             // edges a workgroup gathers before one global append

// Each workgroup walks a contiguous run of interior pixels, gathers its edges
// in LDS and appends them to the list with one global atomic per flush.
__global__ void __launch_bounds__(kT) edge_list(const uint16_t* __restrict__ s, int64_t nx, int64_t ny, int shift, Ws w)
{
    __shared__ int4 buf[kEdgeBuf];
    __shared__ uint32_t count;
    __shared__ unsigned long long base;
    const uint32_t iw = (uint32_t)(nx - 2), n = iw * (uint32_t)(ny - 2);
    const uint32_t per = (n + gridDim.x - 1) / gridDim.x;
    const uint32_t q0 = blockIdx.x * per, q1 = min(n, q0 + per);
    const unsigned long long G2 = w.scal[0];
    if (threadIdx.x == 0) count = 0;
    __syncthreads();
    auto flush = [&]() {
        if (threadIdx.x == 0) base = count ? atomicAdd(w.scal + 2, (unsigned long long)count) : 0ull;
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < count; i += kT) w.edges[base + i] = buf[i];
        __syncthreads();
        if (threadIdx.x == 0) count = 0;
        __syncthreads();
    };
    // the loop bound is uniform over the workgroup, so the barriers are reached by all
    for (uint32_t b = q0; b < q1; b += kT) {
        const uint32_t q = b + threadIdx.x;
        if (q < q1) {
            const uint32_t x = 1 + q % iw, y = 1 + q / iw;
            int gx, gy;
            sobel(s, nx, x, y, gx, gy);
            const unsigned long long m2 = (unsigned long long)((int64_t)gx * gx + (int64_t)gy * gy);
            if (m2 > 0 && (m2 << shift) >= G2) buf[atomicAdd(&count, 1u)] = make_int4((int)x, (int)y, gx, gy);
        }
        __syncthreads();
        if (count > kEdgeBuf - kT) flush();
    }
    flush();
}

__device__ __forceinline__ int64_t sgn(int v) { return (v > 0) - (v < 0); }

// one thread per (edge, step k0 + i); the distance of step k is k |g| / g_major
__global__ void __launch_bounds__(kT) vote(int64_t nx, int64_t ny, int r_min, int r_max, int k0, Ws w)
{
    const uint64_t E = w.scal[2];
    const uint64_t K = (uint64_t)(r_max - k0 + 1);
    const uint64_t total = E * K;
    const bool narrow = total < (uint64_t(1) << 32);       // 32-bit division suffices
    const int64_t lo2 = (int64_t)r_min * r_min, hi2 = (int64_t)r_max * r_max;
    for (uint64_t i = (uint64_t)blockIdx.x * kT + threadIdx.x; i < total; i += (uint64_t)gridDim.x * kT) {
        const uint64_t e = narrow ? (uint64_t)((uint32_t)i / (uint32_t)K) : i / K;
        const int64_t k = k0 + (int64_t)(i - e * K);
        const int4 p = w.edges[e];
        const int64_t ax = p.z < 0 ? -(int64_t)p.z : p.z, ay = p.w < 0 ? -(int64_t)p.w : p.w;
        const bool xmaj = ax >= ay;
        const int64_t gmaj = xmaj ? ax : ay, gmin = xmaj ? ay : ax;
        const int64_t d2 = k * k * (ax * ax + ay * ay), g2 = gmaj * gmaj;
        if (d2 < lo2 * g2 || d2 > hi2 * g2) continue;
        // below 2^32: 2 k gmin + gmaj <= 2 * 4096 * 262140 + 262140
        const int64_t j = (uint32_t)(2 * k * gmin + gmaj) / (uint32_t)(2 * gmaj);
        const int64_t cx = p.x - (xmaj ? k : j) * sgn(p.z);
        const int64_t cy = p.y - (xmaj ? j : k) * sgn(p.w);
        if (cx < 0 || cx >= nx || cy < 0 || cy >= ny) continue;
        atomicAdd(w.acc + cy * nx + cx, 1u);
    }
}

// row box sums: box[y][x] = sum of acc[y][x - wb .. x + wb]
__global__ void __launch_bounds__(kT) box_rows(int64_t nx, int64_t ny, int wb, Ws w)
{
    __shared__ uint32_t row[kMaxSide];
    for (int64_t y = blockIdx.x; y < ny; y += gridDim.x) {
        for (int64_t x = threadIdx.x; x < nx; x += kT) row[x] = w.acc[y * nx + x];
        __syncthreads();
        for (int64_t x = threadIdx.x; x < nx; x += kT) {
            const int64_t lo = x - wb < 0 ? 0 : x - wb, hi = x + wb > nx - 1 ? nx - 1 : x + wb;
            uint64_t s = 0;
            for (int64_t t = lo; t <= hi; ++t) s += row[t];
            w.box[y * nx + x] = s;
        }
        __syncthreads();
    }
}

// column windows of the row sums; the largest key (box sum, then the lowest
// pixel index) over the slice
__global__ void __launch_bounds__(kT) box_cols(int64_t nx, int64_t ny, int wb, Ws w)
{
    const int64_t nseg = (ny + kSeg - 1) / kSeg;
    unsigned long long best = 0;
    for (int64_t q = (int64_t)blockIdx.x * kT + threadIdx.x; q < nx * nseg; q += (int64_t)gridDim.x * kT) {
        const int64_t x = q % nx, y0 = (q / nx) * kSeg;
        const int64_t y1 = y0 + kSeg < ny ? y0 + kSeg : ny;
        uint64_t S = 0;
        const int64_t t0 = y0 - wb < 0 ? 0 : y0 - wb, t1 = y0 + wb > ny - 1 ? ny - 1 : y0 + wb;
        for (int64_t t = t0; t <= t1; ++t) S += w.box[t * nx + x];
        for (int64_t y = y0; y < y1; ++y) {
            if (y > y0) {
                if (y + wb < ny) S += w.box[(y + wb) * nx + x];
                if (y - wb - 1 >= 0) S -= w.box[(y - wb - 1) * nx + x];
            }
            const unsigned long long key = (S << kIdxBits) | (kIdxMask - (uint64_t)(y * nx + x));
            best = key > best ? key : best;
        }
    }
    best = wave_max(best);
    if (__lane_id() == 0 && best) atomicMax(w.scal + 1, best);
}

// round(sqrt(D)) with halves up (no ties occur for integer D)
__device__ __forceinline__ int64_t round_sqrt(int64_t D)
{
    int64_t d = (int64_t)floor(sqrt((double)D) + 0.5);
    while (d > 0 && (2 * d - 1) * (2 * d - 1) > 4 * D) --d;
    while ((2 * d + 1) * (2 * d + 1) <= 4 * D) ++d;
    return d;
}

// each workgroup counts its edges' radii in LDS, then adds its non-zero counts
__global__ void __launch_bounds__(kT) radius_hist(int64_t nx, int r_min, int r_max, Ws w)
{
    __shared__ uint32_t h[kMaxRadius + 1];
    const unsigned long long key = w.scal[1];
    if ((key >> kIdxBits) == 0) return;
    for (int r = threadIdx.x; r <= r_max; r += kT) h[r] = 0u;
    __syncthreads();
    const int64_t idx = (int64_t)(kIdxMask - (key & kIdxMask));
    const int64_t cx = idx % nx, cy = idx / nx;
    const uint64_t E = w.scal[2];
    for (uint64_t e = (uint64_t)blockIdx.x * kT + threadIdx.x; e < E; e += (uint64_t)gridDim.x * kT) {
        const int4 p = w.edges[e];
        const int64_t dx = p.x - cx, dy = p.y - cy;
        if ((int64_t)p.z * dx + (int64_t)p.w * dy <= 0) continue;
        const int64_t d = round_sqrt(dx * dx + dy * dy);
        if (d >= r_min && d <= r_max) atomicAdd(h + d, 1u);
    }
    __syncthreads();
    for (int r = r_min + threadIdx.x; r <= r_max; r += kT)
        if (h[r]) atomicAdd(w.rhist + r, h[r]);
}

__global__ void __launch_bounds__(kT) finish(int64_t nx, int r_min, int r_max, int margin, Ws w, int32_t* rec)
{
    __shared__ unsigned long long red[kT];
    unsigned long long best = 0;
    for (int r = r_min + threadIdx.x; r <= r_max; r += kT) {
        const unsigned long long c = w.rhist[r];
        const unsigned long long k = c ? (c << kRadBits) | (unsigned long long)((1 << kRadBits) - 1 - r) : 0ull;
        best = k > best ? k : best;
    }
    red[threadIdx.x] = best;
    __syncthreads();
    for (int o = kT / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o && red[threadIdx.x + o] > red[threadIdx.x]) red[threadIdx.x] = red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x >= 8) return;
    const unsigned long long key = w.scal[1];
    const uint64_t votes = key >> kIdxBits;
    const int64_t idx = (int64_t)(kIdxMask - (key & kIdxMask));
    const unsigned long long b = red[0];
    const int r = (1 << kRadBits) - 1 - (int)(b & ((1u << kRadBits) - 1));
    const bool found = votes > 0 && b != 0;
    int32_t v = 0;
    switch (threadIdx.x) {
    case kFound: v = found; break;
    case kCx: v = votes ? (int32_t)(idx % nx) : 0; break;
    case kCy: v = votes ? (int32_t)(idx / nx) : 0; break;
    case kR: v = found ? r : 0; break;
    case kKeepR: v = found ? (r > margin ? r - margin : 0) : 0; break;
    case kVotes: v = (int32_t)(votes > 0x7FFFFFFFull ? 0x7FFFFFFFull : votes); break;
    case kRadiusVotes: v = found ? (int32_t)(b >> kRadBits) : 0; break;
    default: v = (int32_t)w.scal[2]; break;
    }
    rec[threadIdx.x] = v;
}

// zero n voxels from p: lanes of one wave, 16-byte stores where aligned
__device__ __forceinline__ void zero_run(uint16_t* p, int64_t n, int lane)
{
    if (n <= 0) return;
    int64_t head = (int64_t)(((16u - (reinterpret_cast<uintptr_t>(p) & 15u)) & 15u) / 2u);
    if (head > n) head = n;
    if (lane < head) p[lane] = 0;
    const int64_t nb = (n - head) / 8;
    uint4* b = reinterpret_cast<uint4*>(p + head);
    for (int64_t i = lane; i < nb; i += 64) b[i] = make_uint4(0u, 0u, 0u, 0u);
    const int64_t t0 = head + nb * 8;
    if (lane < n - t0) p[t0 + lane] = 0;
}

// one wave per row: every voxel outside the row's kept run becomes 0
__global__ void __launch_bounds__(kT) remove_outside(uint16_t* __restrict__ vol, int64_t nx, int64_t ny, int64_t nz,
                                                     const int32_t* __restrict__ rec)
{
    const Disc d = load_disc(rec);
    if (!d.found) return;
    const int lane = (int)__lane_id();
    const int64_t wpb = kT / 64;
    const int64_t nw = (int64_t)gridDim.x * wpb;
    for (int64_t row = (int64_t)blockIdx.x * wpb + threadIdx.x / 64; row < ny * nz; row += nw) {
        int64_t x0, x1;
        row_span(d, row % ny, nx, x0, x1);
        uint16_t* p = vol + row * nx;
        if (x0 > x1) {
            zero_run(p, nx, lane);
        } else {
            zero_run(p, x0, lane);
            zero_run(p + x1 + 1, nx - 1 - x1, lane);
        }
    }
}

unsigned grid_for(int64_t items, int64_t cap)
{
    int64_t g = (items + kT - 1) / kT;
    if (g > cap) g = cap;
    return (unsigned)(g < 1 ? 1 : g);
}

int check_find(int64_t nx, int64_t ny, int r_min, int r_max, int shift, int margin)
{
    VR_REQUIRE(nx >= 3 && ny >= 3 && nx <= kMaxSide && ny <= kMaxSide, VR_ERR_DIMS,
               "vr_find_container: slice %lld x %lld outside [3, %d]^2", (long long)nx, (long long)ny, kMaxSide);
    VR_REQUIRE(r_min >= 1 && r_min <= r_max && r_max <= kMaxRadius, VR_ERR_RANGE,
               "vr_find_container: radii [%d, %d] outside 1 <= r_min <= r_max <= %d", r_min, r_max, kMaxRadius);
    VR_REQUIRE(shift >= 0 && shift <= 16, VR_ERR_RANGE, "vr_find_container: edge shift %d outside [0, 16]", shift);
    VR_REQUIRE(margin >= 0, VR_ERR_RANGE, "vr_find_container: margin %d < 0", margin);
    return VR_OK;
}

}  // namespace

extern "C" int vr_container_workspace_size(int64_t nx, int64_t ny, int r_max, int64_t* bytes)
{
    vr::clear_error();
    VR_REQUIRE(bytes != nullptr, VR_ERR_NULL, "vr_container_workspace_size: bytes is NULL");
    int rc = check_find(nx, ny, 1, r_max, 0, 0);
    if (rc) return rc;
    *bytes = carve(nullptr, nx, ny, r_max, nullptr);
    return VR_OK;
}

namespace {

// The steps of vr_find_container on a carved workspace w.
int find_on(const uint16_t* d_slice, int64_t nx, int64_t ny, int r_min, int r_max, int edge_shift, int margin,
            const Ws& w, int32_t* d_circle, hipStream_t s)
{
    int rc;
    const int64_t cap = (int64_t)vr::num_cus() * 8;
    const int64_t n = nx * ny, interior = (nx - 2) * (ny - 2);
    const int wb = std::max(1, r_max / 16);
    const int k0 = std::max(1, (r_min * 181) >> 8);     // below r_min / sqrt(2): no step reaches r_min

    // every counter and accumulator the later steps add to starts at zero here
    clear_ws<<<grid_for(n, cap), kT, 0, s>>>(w, n, r_max + 1);
    if ((rc = vr::check_launch("vr_find_container: clear"))) return rc;
    const int64_t cap2 = (int64_t)vr::num_cus() * 2;
    grad_max<<<grid_for(interior, cap2), kT, 0, s>>>(d_slice, nx, ny, w);
    if ((rc = vr::check_launch("vr_find_container: gradient"))) return rc;
    edge_list<<<grid_for(interior, cap2), kT, 0, s>>>(d_slice, nx, ny, edge_shift, w);
    if ((rc = vr::check_launch("vr_find_container: edges"))) return rc;
    vote<<<(unsigned)cap, kT, 0, s>>>(nx, ny, r_min, r_max, k0, w);
    if ((rc = vr::check_launch("vr_find_container: votes"))) return rc;
    box_rows<<<(unsigned)std::min<int64_t>(ny, cap), kT, 0, s>>>(nx, ny, wb, w);
    if ((rc = vr::check_launch("vr_find_container: row boxes"))) return rc;
    box_cols<<<grid_for(nx * ((ny + kSeg - 1) / kSeg), cap), kT, 0, s>>>(nx, ny, wb, w);
    if ((rc = vr::check_launch("vr_find_container: column boxes"))) return rc;
    // the edge count is known on the device only: enough workgroups for a slice
    // whose interior were all edges, capped at a few per compute unit
    radius_hist<<<grid_for(interior, (int64_t)vr::num_cus() * 2), kT, 0, s>>>(nx, r_min, r_max, w);
    if ((rc = vr::check_launch("vr_find_container: radii"))) return rc;
    finish<<<1, kT, 0, s>>>(nx, r_min, r_max, margin, w, d_circle);
    return vr::check_launch("vr_find_container: record");
}

// Workspace of vr_find_container_noalloc: a file-scope device array, one copy
// per GPU, held until the process ends.  Host code never passes its name to a
// kernel (on the host the name is a stand-in, not a device address): the
// device address comes from hipGetSymbolAddress, once per device.
constexpr int64_t kScratchBytes = VR_CONTAINER_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array (looked up on the
// first call on that device).
int scratch_ptr(void** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    VR_REQUIRE(e == hipSuccess, VR_ERR_HIP, "vr_find_container_noalloc: hipGetDevice: %s", hipGetErrorString(e));
    VR_REQUIRE(dev >= 0 && dev < kMaxDevices, VR_ERR_UNSUPPORTED,
               "vr_find_container_noalloc: device %d beyond the %d this build tracks", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        VR_REQUIRE(e == hipSuccess && p != nullptr, VR_ERR_HIP,
                   "vr_find_container_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return VR_OK;
}

}  // namespace

extern "C" int vr_find_container(const uint16_t* d_slice, int64_t nx, int64_t ny, int r_min, int r_max,
                                 int edge_shift, int margin, void* d_work, int64_t work_bytes,
                                 int32_t* d_circle, void* stream)
{
    vr::clear_error();
    VR_REQUIRE(d_slice && d_work && d_circle, VR_ERR_NULL, "vr_find_container: NULL pointer");
    int rc = check_find(nx, ny, r_min, r_max, edge_shift, margin);
    if (rc) return rc;
    const int64_t need = carve(nullptr, nx, ny, r_max, nullptr);
    VR_REQUIRE(work_bytes >= need, VR_ERR_WORKSPACE, "vr_find_container: workspace %lld bytes, %lld needed",
               (long long)work_bytes, (long long)need);
    VR_REQUIRE((reinterpret_cast<uintptr_t>(d_work) & 255u) == 0, VR_ERR_RANGE,
               "vr_find_container: workspace not 256-byte aligned");
    Ws w;
    carve(d_work, nx, ny, r_max, &w);
    return find_on(d_slice, nx, ny, r_min, r_max, edge_shift, margin, w, d_circle, vr::as_stream(stream));
}

extern "C" int vr_find_container_noalloc(const uint16_t* d_slice, int64_t nx, int64_t ny, int r_min, int r_max,
                                         int edge_shift, int margin, int32_t* d_circle, void* stream)
{
    vr::clear_error();
    VR_REQUIRE(d_slice && d_circle, VR_ERR_NULL, "vr_find_container_noalloc: NULL pointer");
    int rc = check_find(nx, ny, r_min, r_max, edge_shift, margin);
    if (rc) return rc;
    const int64_t need = carve(nullptr, nx, ny, r_max, nullptr);
    VR_REQUIRE(need <= kScratchBytes, VR_ERR_WORKSPACE,
               "vr_find_container_noalloc: a %lld x %lld slice needs %lld bytes of scratch, above the %lld "
               "this build holds",
               (long long)nx, (long long)ny, (long long)need, (long long)kScratchBytes);
    void* base = nullptr;
    if ((rc = scratch_ptr(&base))) return rc;
    Ws w;
    carve(base, nx, ny, r_max, &w);
    return find_on(d_slice, nx, ny, r_min, r_max, edge_shift, margin, w, d_circle, vr::as_stream(stream));
}

extern "C" int vr_remove_container(uint16_t* d_vol, int64_t nx, int64_t ny, int64_t nz, const int32_t* d_circle,
                                   void* stream)
{
    vr::clear_error();
    VR_REQUIRE(d_vol && d_circle, VR_ERR_NULL, "vr_remove_container: NULL pointer");
    VR_REQUIRE(nx >= 1 && ny >= 1 && nz >= 1, VR_ERR_DIMS, "vr_remove_container: dims %lld x %lld x %lld",
               (long long)nx, (long long)ny, (long long)nz);
    hipStream_t s = vr::as_stream(stream);
    const int64_t rows = ny * nz;
    const int64_t blocks = std::min<int64_t>((rows + kT / 64 - 1) / (kT / 64), (int64_t)vr::num_cus() * 16);
    remove_outside<<<(unsigned)std::max<int64_t>(1, blocks), kT, 0, s>>>(d_vol, nx, ny, nz, d_circle);
    return vr::check_launch("vr_remove_container");
}
