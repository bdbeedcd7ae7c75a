/*
 * vr.h — C ABI of the MI355X (gfx950) preview library.
 *
 * The library computes the data-parallel core of low-latency visual previews
 * of 16-bit micro-CT volumes (Tan Jerome et al., "Low-latency Visual Previews
 * of Large Synchrotron Micro-CT Datasets"): histogram filtering and
 * thresholding of the volume (Sections III-A and III-D), a multi-resolution
 * box-filtered pyramid (abstract; Section II, interactive preview) packed into
 * slicemap atlases (Section III), and emission-absorption ray casting of the
 * reduced volume into turntable frames (Section III-C, rotation about Z),
 * plus the adjoint of that ray caster.
 *
 * Conventions shared by every entry point
 *   - Return value: VR_OK (0) or a negative VR_ERR_* code.  Argument errors
 *     are detected before anything is enqueued; launch errors are read back
 *     with hipGetLastError.  vr_last_error() gives a message for the last
 *     failing call on the calling host thread.
 *   - Pointers prefixed d_ are device pointers (hipMalloc'd or equivalent),
 *     h_ are host pointers read only during the call.  The caller owns every
 *     buffer; the single-call entry points never allocate or free memory.
 *   - Every call is asynchronous on `stream` (a hipStream_t, NULL = the
 *     default stream) and never synchronises the host, so a sequence of calls
 *     can be captured into a HIP graph.  Output buffers are written entirely
 *     by the call (including zeroing of accumulated outputs) unless stated
 *     otherwise.
 *   - Volumes are C-contiguous [nz][ny][nx] with x fastest: slice z is the
 *     z-th reconstructed 2D slice of the stack (Section III).  Voxel (x, y, z)
 *     covers [x, x+1) x [y, y+1) x [z, z+1) times the spacing in world units.
 *   - Calls are reentrant; concurrent calls on different streams are safe as
 *     long as their output buffers do not overlap.
 */
#ifndef VR_H
#define VR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VR_NBINS 65536            /* 16-bit grey values */
#define VR_KEEP_WORDS 2048        /* keep mask: bin b -> bit (b % 32) of word b / 32 */
#define VR_MAX_LEVELS 8           /* pyramid levels produced by one call */
#define VR_MAX_VIEWS_PER_LAUNCH 48
#define VR_BRICK_DIST_CAP 8       /* cap of the brick distance grid, see vr_brick_volume */

enum {
    VR_OK = 0,
    VR_ERR_NULL = -1,          /* a required pointer is NULL */
    VR_ERR_DIMS = -2,          /* a size is < 1 or too large */
    VR_ERR_RANGE = -3,         /* a parameter is outside its documented range */
    VR_ERR_DTYPE = -4,         /* unsupported element type for this call */
    VR_ERR_HIP = -5,           /* the HIP runtime reported an error */
    VR_ERR_UNSUPPORTED = -6,   /* valid request this build does not implement */
    VR_ERR_WORKSPACE = -7      /* workspace too small */
};

/* threshold rules for vr_select_threshold */
enum {
    VR_RULE_VALLEY = 0,        /* first valley above the air peak (param = smoothing radius) */
    VR_RULE_OTSU = 1,          /* Algorithm 1 (param = log2 of the bin width, 0 or 8 typical) */
    VR_RULE_ITS = 2,           /* Algorithm 2 (param = log2 of the bin width) */
    VR_RULE_NONE = 3           /* T = 0: only the top-slice histogram filter applies */
};

/* volume element types */
enum { VR_U16_NORM = 0, VR_F32 = 1 };

/* volume layouts for rendering */
enum {
    VR_LAYOUT_LINEAR = 0,      /* [nz][ny][nx], x fastest */
    VR_LAYOUT_BRICK4 = 1,      /* 4x4x4 bricks, see vr_brick_volume */
    VR_LAYOUT_BRICK4_PAIRS = 2, /* 4x4x4 bricks of x-tap pairs, see vr_brick_volume */
    VR_LAYOUT_BRICK8 = 3,      /* 8x8x8 bricks, see vr_brick_volume */
    VR_LAYOUT_BRICK4_OVERLAP = 4 /* 4x4x4 bricks overlapping by one voxel in x, see vr_brick_volume */
};

/*
 * Histogram of grey values (Section III-D: the volume histogram, and the
 * histogram of the first three slices that holds the signature of air and
 * container).  d_hist[b] = number of voxels of value b among slices
 * z0 <= z < z0 + nz_range of the u16 volume d_vol [nz][ny][nx].
 *   d_hist: 65536 uint64 counters, overwritten.
 *   nz_range may be 0 (all counters become 0).
 * Errors: VR_ERR_NULL, VR_ERR_DIMS (a size < 1), VR_ERR_RANGE (z-range not
 * inside [0, nz)), VR_ERR_HIP.
 */
int vr_histogram(const uint16_t* d_vol, int64_t nx, int64_t ny, int64_t nz,
                 int64_t z0, int64_t nz_range, uint64_t* d_hist, void* stream);

/*
 * Threshold selection and keep mask, entirely on the device (no host sync).
 * Thresholding classifies each voxel as kept or removed by its grey value
 * (Section III-A); histogram filtering removes every grey value that occurs
 * in the top-slice histogram (Section III-D).  The keep mask is
 *   keep[b] = (b >= T) && (d_hist_top == NULL || d_hist_top[b] == 0).
 * T is chosen by `rule`:
 *   VR_RULE_VALLEY: S = d_hist box-smoothed with radius `param` (1..1023);
 *     p = first argmax of S; T = start of the plateau of the first bin above
 *     p where 2*S[b] <= S[p] and S[b+1] > S[b]; 65535 if none.
 *   VR_RULE_OTSU: Algorithm 1 on the histogram with bins of width 2^param
 *     (param 0..12), between-class variance evaluated in IEEE FP64 in the
 *     order w_a*w_b*(mu_a-mu_b)^2, classes [0,T) and [T,B-1], lowest T on
 *     ties; the result is scaled back to 16-bit grey values (T << param).
 *   VR_RULE_ITS: Algorithm 2 (isodata), T <- floor((mu_1+mu_2)/2) in FP64
 *     from the middle of the occupied range until T repeats, same bins.
 *   VR_RULE_NONE: T = 0.
 *   d_result: 4 uint32 written: [0] = T (16-bit grey value), [1] = the air
 *     peak p (valley) or the iteration count (ITS), [2] = b* (valley), [3] = 0.
 *   d_hist: 16-byte aligned (read in 16-byte pieces).
 *   d_keep_bits: 2048 uint32, overwritten (also used as scratch by the call).
 * Errors: VR_ERR_NULL, VR_ERR_RANGE (rule, param or alignment), VR_ERR_HIP.
 */
int vr_select_threshold(const uint64_t* d_hist, const uint64_t* d_hist_top, int rule, int param,
                        uint32_t* d_result, uint32_t* d_keep_bits, void* stream);

/*
 * Both histograms Section III-D needs, in one launch: d_hist over the whole
 * volume and d_hist_top over its first top_slices slices (1..nz); the same
 * counts as two vr_histogram calls.  Both outputs are overwritten.
 * Errors: VR_ERR_NULL, VR_ERR_DIMS, VR_ERR_RANGE, VR_ERR_HIP.
 */
int vr_histogram_with_top(const uint16_t* d_vol, int64_t nx, int64_t ny, int64_t nz,
                          int64_t top_slices, uint64_t* d_hist, uint64_t* d_hist_top, void* stream);

/*
 * Container removal (Section III-B).  The sample container is a cylinder
 * about the z axis; its circle is found in one slice (the top slice, slice 0
 * of the stack) with the Hough transform of Ioannou et al., and every voxel
 * outside it is discarded in every slice.  The circle record is 8 int32:
 *   [0] found (1/0), [1] cx, [2] cy (pixel of the centre), [3] r (detected
 *   radius of the wall's inner boundary), [4] R = max(r - margin, 0) (kept
 *   radius), [5] centre votes (box sum, saturated to 2^31 - 1), [6] count of
 *   the radius, [7] edge pixels.
 * The kept disc holds the pixels with (x - cx)^2 + (y - cy)^2 <= R^2; a record
 * with found = 0 keeps every pixel.
 */
#define VR_CIRCLE_INTS 8

/* Workspace bytes vr_find_container needs for an nx x ny slice and r_max.
 * Errors: VR_ERR_NULL, VR_ERR_DIMS, VR_ERR_RANGE (as vr_find_container). */
int vr_container_workspace_size(int64_t nx, int64_t ny, int r_max, int64_t* bytes);

/*
 * The container's circle in the u16 slice d_slice [ny][nx] (3..8192 pixels a
 * side), all on the device:
 *   edges: the integer 3 x 3 Sobel gradient g of the interior pixels; a pixel
 *     is an edge when |g|^2 > 0 and |g|^2 * 2^edge_shift >= the slice's
 *     largest |g|^2 (edge_shift 0..16, 4 typical);
 *   votes: each edge pixel votes once for every cell of the digital line from
 *     it against its gradient (one cell per step along the gradient's major
 *     axis, the minor offset rounded half up) whose distance from it along the
 *     line lies in [r_min, r_max] (1 <= r_min <= r_max <= 4096);
 *   centre: the first maximum, in row-major order, of the votes summed over
 *     (2w+1)^2 boxes, w = max(1, r_max / 16);
 *   radius: the first maximum (smallest radius) of round(|p - c|) over the
 *     edge pixels p whose gradient points away from the centre, in
 *     [r_min, r_max]; kept radius R = max(r - margin, 0), margin >= 0.
 * All decisions are integer arithmetic.
 *   d_work: >= vr_container_workspace_size bytes, 256-byte aligned, scratch.
 *   d_circle: VR_CIRCLE_INTS int32, overwritten.
 * Errors: VR_ERR_NULL, VR_ERR_DIMS, VR_ERR_RANGE (radii, shift, margin or
 * workspace alignment), VR_ERR_WORKSPACE, VR_ERR_HIP.
 */
int vr_find_container(const uint16_t* d_slice, int64_t nx, int64_t ny, int r_min, int r_max,
                      int edge_shift, int margin, void* d_work, int64_t work_bytes,
                      int32_t* d_circle, void* stream);

/*
 * vr_find_container for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops that forbid allocation): the same steps
 * and the same record, with the workspace taken from a fixed device array of
 * VR_CONTAINER_SCRATCH_BYTES that the library holds on each GPU it runs on
 * until the process ends, instead of a caller's buffer.  Nothing is allocated
 * or freed by the call.
 *   Size limit: the slice's vr_container_workspace_size must not exceed
 *     VR_CONTAINER_SCRATCH_BYTES (any slice of at most 1024 x 1024 pixels, for
 *     every r_max); larger requests return VR_ERR_WORKSPACE before anything is
 *     enqueued.
 *   The array belongs to the device current on the calling thread, and
 *   `stream` must belong to that device.  Every call on one GPU shares it:
 *   calls that overlap on one GPU (on different streams, or from several host
 *   threads) race and give undefined records; calls in one stream order are
 *   safe, since each starts by clearing what it accumulates.  The first call
 *   on a device looks the array's address up (hipGetSymbolAddress).
 * Errors: as vr_find_container (VR_ERR_WORKSPACE for the size limit), and
 * VR_ERR_UNSUPPORTED for a device index above 63.
 */
#define VR_CONTAINER_SCRATCH_BYTES (32ll << 20)
int vr_find_container_noalloc(const uint16_t* d_slice, int64_t nx, int64_t ny, int r_min, int r_max,
                              int edge_shift, int margin, int32_t* d_circle, void* stream);

/* Sets every voxel outside the kept disc of d_circle to 0, in every slice of
 * d_vol [nz][ny][nx], in place (nothing changes when the circle was not
 * found).  Errors: VR_ERR_NULL, VR_ERR_DIMS, VR_ERR_HIP. */
int vr_remove_container(uint16_t* d_vol, int64_t nx, int64_t ny, int64_t nz, const int32_t* d_circle,
                        void* stream);

/* vr_histogram_with_top restricted to the voxels inside the kept disc of
 * d_circle: voxels outside it take no part in either histogram.  d_hist_top
 * may be NULL (top_slices is then ignored).  Both outputs are overwritten.
 * Errors: VR_ERR_NULL, VR_ERR_DIMS, VR_ERR_RANGE, VR_ERR_HIP. */
int vr_histogram_in_disc(const uint16_t* d_vol, int64_t nx, int64_t ny, int64_t nz, int64_t top_slices,
                         const int32_t* d_circle, uint64_t* d_hist, uint64_t* d_hist_top, void* stream);

/* A slicemap atlas written as a side output of vr_threshold_downsample. */
typedef struct {
    int32_t level;             /* pyramid level (1..n_levels) packed into the atlas */
    int32_t tiles_x, tiles_y;  /* tile grid; tiles_x * tiles_y >= that level's nz */
    int32_t out_bits;          /* 16 or 8, as vr_pack_slicemap */
    void* data;                /* device pointer, [tiles_y*ny_k][tiles_x*nx_k] */
} vr_atlas_spec;

/*
 * Thresholding fused with the multi-resolution pyramid (abstract and
 * Section II: a coarse resolution is delivered before the full data).
 * f = keep[v] ? v : 0 per voxel (d_keep_bits NULL keeps every voxel); level
 * k = 1..n_levels has dims ceil(n / 2^k) per axis and
 *   L_k = (S_k + 2^(3k-1)) >> 3k,
 * S_k the exact integer sum of f over the 2^k cube at 2^k*(x, y, z), with
 * voxels past the volume's end counted as 0 (round-half-up mean over the
 * full cube, each level from its own exact sum).  One pass over the volume
 * writes levels 1..4; levels 5..n_levels are then summed, exactly, from the
 * level-4 sums by a second, small launch.
 *   h_levels: host array of n_levels device pointers, level k at
 *     h_levels[k-1], each [nz_k][ny_k][nx_k] u16, overwritten.
 *   n_levels: 1..VR_MAX_LEVELS.
 *   h_level_sums: NULL, or a host array of n_levels device pointers, each
 *     NULL or [nz_k][ny_k][nx_k] u64 receiving the exact S_k (overwritten;
 *     for verification).  With n_levels > 4, h_level_sums[3] is required:
 *     the levels past the fourth are formed from it.
 *   atlas: NULL, or a slicemap atlas of one of the levels to write in the
 *     same call (the layout and values of vr_pack_slicemap, overwritten).
 * Errors: VR_ERR_NULL (incl. a missing level-4 sums buffer when n_levels > 4),
 * VR_ERR_DIMS, VR_ERR_RANGE (n_levels, atlas), VR_ERR_HIP.
 */
int vr_threshold_downsample(const uint16_t* d_vol, int64_t nx, int64_t ny, int64_t nz,
                            const uint32_t* d_keep_bits, int n_levels,
                            uint16_t* const* h_levels, uint64_t* const* h_level_sums,
                            const vr_atlas_spec* atlas, void* stream);

/* vr_threshold_downsample with every voxel outside the kept disc of d_circle
 * (see vr_find_container) counted as removed, so the levels equal those of
 * the volume after vr_remove_container; d_vol is not modified.  Slices of at
 * most 8192 x 8192.  Errors: as vr_threshold_downsample, and VR_ERR_NULL for
 * d_circle. */
int vr_threshold_downsample_in_disc(const uint16_t* d_vol, int64_t nx, int64_t ny, int64_t nz,
                                    const uint32_t* d_keep_bits, const int32_t* d_circle, int n_levels,
                                    uint16_t* const* h_levels, uint64_t* const* h_level_sums,
                                    const vr_atlas_spec* atlas, void* stream);

/*
 * Hollow data preview (Section II: a preview that keeps the object's outer
 * geometry and drops its interior volume; the paper gives no algorithm).
 * A voxel of the [nz][ny][nx] u16 volume d_src is kept when it is non-zero
 * and some voxel within city-block distance `thickness` of it is zero or lies
 * outside the volume: the shell that `thickness` binary erosions of the
 * non-zero set with the 6-neighbourhood (zero border) take away.  Kept voxels
 * keep their value in d_dst; every other voxel of d_dst becomes 0.  Cavities
 * inside the object are background too, so their walls are kept.
 *   thickness: 1 .. VR_HOLLOW_MAX_THICKNESS voxels.
 *   d_dst: nx*ny*nz u16, overwritten; must not overlap d_src.
 *   d_kept: NULL or one u64, overwritten with the number of kept voxels.
 * Errors: VR_ERR_NULL, VR_ERR_DIMS, VR_ERR_RANGE (thickness, overlap),
 * VR_ERR_HIP.
 */
#define VR_HOLLOW_MAX_THICKNESS 8
int vr_hollow(const uint16_t* d_src, int64_t nx, int64_t ny, int64_t nz, int thickness, uint16_t* d_dst,
              uint64_t* d_kept, void* stream);

/*
 * Slicemap atlas of a volume level (Section III, slicemaps of the cited
 * prior work): a 2D image of tiles_y x tiles_x tiles of nx x ny pixels in
 * which atlas pixel (tx*nx + x, ty*ny + y) = L[z][y][x] with
 * z = ty*tiles_x + tx; tiles past the last slice are 0.
 *   d_atlas: [tiles_y*ny][tiles_x*nx] of u16 (out_bits 16) or u8 (out_bits 8,
 *     value min(255, (L + 128) >> 8)), overwritten.
 * Errors: VR_ERR_NULL, VR_ERR_DIMS, VR_ERR_RANGE (tiles_x*tiles_y < nz or
 * out_bits not 8/16), VR_ERR_HIP.
 */
int vr_pack_slicemap(const uint16_t* d_level, int64_t nx, int64_t ny, int64_t nz, int tiles_x,
                     int tiles_y, int out_bits, void* d_atlas, void* stream);

/*
 * Render layout (not in the paper; a memory layout for the ray caster): the
 * volume as 4 x 4 x 4-voxel bricks, brick (bx, by, bz) at element
 * ((bz*nby + by)*nbx + bx)*64 with nbx = ceil(nx / 4) (and so on), voxel (x, y, z) at
 * ((z&3)*16 + (y&3)*4 + (x&3)) inside it (voxels past the volume's end are 0),
 * then an apron of nbx*nby + nbx + 1 bricks of zeros: the ray caster reads the
 * far taps of cells on the volume's last voxel layer there (and in the padding
 * voxels) without a bounds check, with weight 0.
 * Optional occupancy: one byte per brick, non-zero iff a marking voxel (one
 * above mark_above: with mark_above 0, any non-zero voxel) is one of the 8
 * taps of a trilinear fetch whose base (floor, clamped) tap lies in that
 * brick, followed by one byte per 4 x 4 x 4 bricks (16^3 voxels,
 * [ceil(nbz/4)][ceil(nby/4)][ceil(nbx/4)]) that is non-zero iff any of its
 * bricks is, then one byte per brick (brick order) holding the Chebyshev
 * distance in bricks, max over axes of |b - b'|, to the nearest occupied
 * brick b', capped at VR_BRICK_DIST_CAP (0 for an occupied brick; the cap
 * where none is nearer), then one byte per brick of working storage.  The
 * ray caster passes over samples of unoccupied bricks when every transfer-
 * function entry such a sample can reach has zero extinction (and finite
 * colour): with mark_above 0 the sample has density 0 and reaches entry 0;
 * with mark_above V > 0 its eight taps are at most V, so its TF coordinate
 * s * 255 / 65535 stays below floor(V * 255 / 65535 * (1 + 2^-16)) + 1 and it
 * reaches the entries up to one past that (vr_volume.occupancy_above passes V
 * to the ray caster, which checks those entries on the device and otherwise
 * marches every sample).  Such samples change neither colour nor
 * transmittance, so the result is bit-identical.  A caller whose TF has zero
 * extinction up to entry z - 1 (z >= 2) may use V = 257 * (z - 1) - 1.  From an empty brick whose distance is r it leaves in one
 * step the cube of bricks within r - 1 of it, all of them empty.
 * Layout VR_LAYOUT_BRICK4_PAIRS orders elements the same way, but element
 * (x, y, z) holds two voxels, (x, y, z) then (min(x + 1, nx - 1), y, z)
 * (two u16 in one 32-bit word, low half first, or two f32): the two x taps
 * of a trilinear fetch come in one load, at twice the memory.
 * Layout VR_LAYOUT_BRICK8 is the same with 8 x 8 x 8-voxel bricks: brick
 * (bx, by, bz) at element ((bz*nby + by)*nbx + bx)*512 with nbx = ceil(nx / 8),
 * voxel (x, y, z) at ((z&7)*64 + (y&7)*8 + (x&7)) inside it, then the same
 * apron in these bricks; its occupancy is the same four grids over these
 * bricks (groups of 4 x 4 x 4 of them, 32^3 voxels), sized by
 * vr_brick_count_layout.
 * Layout VR_LAYOUT_BRICK4_OVERLAP (u16 only) stores 4 x 4 x 4-voxel bricks
 * that overlap by one voxel in x: brick (bx, by, bz) holds voxels
 * x = 3 bx .. 3 bx + 3 (0 past the volume's end), y = 4 by .. 4 by + 3 and
 * z = 4 bz .. 4 bz + 3, voxel (x, y, z) at ((z&3)*16 + (y&3)*4 + (x - 3 bx))
 * inside it, with nbx = (nx - 1) / 3 + 1, in the brick order and with the
 * apron of VR_LAYOUT_BRICK4.  A brick serves the trilinear cells whose base
 * tap has x in 3 bx .. 3 bx + 2 (and y, z in the brick), so both x taps of a
 * cell lie in one brick row and one 32-bit load brings them.  Its occupancy
 * is the four grids over these bricks.
 *   d_src: [nz][ny][nx] of u16 (dtype VR_U16_NORM) or f32 (VR_F32).
 *   layout: VR_LAYOUT_BRICK4, VR_LAYOUT_BRICK4_PAIRS, VR_LAYOUT_BRICK8 or
 *     VR_LAYOUT_BRICK4_OVERLAP (u16).
 *   d_bricked: the elements of vr_brick_count_layout (bricks and apron;
 *     for 4^3 bricks (n_bricks + nbx*nby + nbx + 1) * 64, x2 voxels for
 *     pairs), 16-byte aligned,
 *     overwritten.
 *   d_occupancy: NULL or the occupancy_bytes of vr_brick_count_layout,
 *     overwritten.
 *   mark_above: the marking level V, 0..65535 for u16; 0 for f32.
 * Errors: VR_ERR_NULL, VR_ERR_DTYPE, VR_ERR_DIMS, VR_ERR_RANGE (layout,
 * alignment, mark_above), VR_ERR_HIP.
 */
int vr_brick_volume(const void* d_src, int dtype, int layout, int64_t nx, int64_t ny, int64_t nz,
                    void* d_bricked, uint8_t* d_occupancy, int32_t mark_above, void* stream);

/*
 * Inverse of vr_brick_volume for VR_LAYOUT_BRICK4: writes the [nz][ny][nx]
 * volume whose brick layout is d_bricked (the padding voxels past the
 * volume's end are dropped).  Used to bring a density gradient that
 * vr_raycast_backward produced in the brick layout back to the grid's own
 * layout.
 *   d_bricked: vr_brick_count(...) * 64 elements of u16 (VR_U16_NORM) or f32.
 *   d_dst: nx * ny * nz elements of the same type, overwritten.
 * Errors: VR_ERR_NULL, VR_ERR_DTYPE, VR_ERR_DIMS, VR_ERR_HIP.
 */
int vr_unbrick_volume(const void* d_bricked, int dtype, int64_t nx, int64_t ny, int64_t nz, void* d_dst,
                      void* stream);

/* Number of 4x4x4 bricks of an nx x ny x nz volume and the size of its
 * occupancy (nullable; the grids vr_brick_volume describes: 3 bytes per brick
 * plus one per 4x4x4 bricks) in bytes (host only). */
int vr_brick_count(int64_t nx, int64_t ny, int64_t nz, int64_t* n_bricks, int64_t* occupancy_bytes);

/* vr_brick_count for any brick layout: bricks of the layout's edge (4 for
 * VR_LAYOUT_BRICK4 and VR_LAYOUT_BRICK4_PAIRS, 8 for VR_LAYOUT_BRICK8, 4
 * overlapping in x, (nx - 1) / 3 + 1 of them along x, for
 * VR_LAYOUT_BRICK4_OVERLAP),
 * elements of the bricked volume (nullable; (bricks + nbx*nby + nbx + 1) x
 * edge^3 with the apron, doubled for the pair layout), and the occupancy's
 * bytes (nullable).
 * Errors: VR_ERR_NULL, VR_ERR_DIMS, VR_ERR_RANGE (layout). */
int vr_brick_count_layout(int layout, int64_t nx, int64_t ny, int64_t nz, int64_t* n_bricks, int64_t* elements,
                          int64_t* occupancy_bytes);

/* A volume to render. dtype VR_U16_NORM (value / 65535) or VR_F32 (value). */
typedef struct {
    const void* data;          /* device pointer in `layout` */
    int32_t dtype;
    int32_t layout;            /* VR_LAYOUT_LINEAR or a brick layout (VR_LAYOUT_BRICK4_OVERLAP: u16 only) */
    int64_t nx, ny, nz;
    double spacing[3];         /* world units per voxel along x, y, z (> 0) */
    const uint8_t* occupancy;  /* NULL, or the brick occupancy (brick layouts only) */
    int32_t occupancy_above;   /* the mark_above the occupancy was built with (0: non-zero voxels) */
} vr_volume;

/* A pinhole (fov_y_deg > 0) or orthographic (fov_y_deg == 0) camera. */
typedef struct {
    double eye[3], target[3], up[3];
    double fov_y_deg;          /* vertical field of view, 0 < fov < 180, or 0 */
    double ortho_half_h;       /* half height of the orthographic view (> 0) */
} vr_camera;

typedef struct {
    int32_t width, height;     /* pixels, >= 1 */
    float step;                /* sample spacing along the ray, world units (> 0) */
    float ert_eps;             /* stop a ray once its transmittance < ert_eps; 0 = never */
    float bg[4];               /* background RGBA behind the volume */
    uint32_t* view_hist;       /* NULL, or [n_views][256] device counts, overwritten by
                                  vr_raycast with the grey-value histogram of each frame
                                  as vr_frame_entropy defines it (for vr_entropy_from_counts) */
    uint32_t flags;            /* 0, or VR_RENDER_STAGED (vr_raycast only) */
} vr_render_opts;

/* vr_render_opts.flags: march in depth windows whose voxels are staged in LDS
 * instead of reading the taps through the caches (u16 volumes in
 * VR_LAYOUT_BRICK4 with their occupancy, otherwise VR_ERR_UNSUPPORTED).  The
 * frames and counts are bit-identical; on the turntable benchmark it is the
 * slower of the two marches. */
#define VR_RENDER_STAGED 1u

/*
 * Emission-absorption ray casting (Section III-C renders the reduced data to
 * 2D images while rotating about Z).  For the pixel centre (i+1/2, j+1/2),
 * row 0 at the top, with f = normalise(target - eye), r = normalise(f x up),
 * u = r x f, ndc_x = (2(i+1/2)/W - 1) W/H, ndc_y = 1 - 2(j+1/2)/H:
 *   perspective: origin eye, direction normalise(f + tan(fov/2)(ndc_x r + ndc_y u));
 *   orthographic: origin eye + h (ndc_x r + ndc_y u), direction f.
 * The ray is clipped to the world box [0, n*spacing]^3: t0 = max(entry, 0)
 * and L = the distance from the entry point to the first face the ray leaves
 * through (t1 - t0, taken from coordinates inside the box);
 * n = max(1, ceil(L/step)) midpoint samples of length step, the last one
 * ending exactly at t0 + L (no longer than step).  Density = trilinear
 * interpolation of cell-centred voxels with taps clamped to the volume; the
 * transfer function d_tf (256 x (r, g, b, sigma) f32, sigma = extinction per
 * world unit) is interpolated linearly at x = 255 clamp(s, 0, 1).  Front to
 * back: alpha = 1 - exp(-sigma len), C += T alpha rgb, T *= exp(-sigma len);
 * output RGB = C + T bg_rgb, A = 1 - T (1 - bg_a).  Missing rays get bg.
 *   d_rgba: [n_views][height][width][4] f32, overwritten.
 *   d_samples: NULL or two uint64 counters the call adds to (the caller
 *     zeroes them): [0] the samples of the definition above taken before
 *     early termination, [1] the samples evaluated (those not passed over as
 *     empty, see occupancy below).
 *   h_cams: n_views cameras (any n_views >= 1; views are launched in groups
 *     of VR_MAX_VIEWS_PER_LAUNCH).
 * All arithmetic is FP32; per-ray results do not depend on the launch shape,
 * the layout or the occupancy (bit-identical).  With vol->occupancy set and
 * tf[0].sigma == 0, samples whose eight taps are all zero are passed over
 * without being evaluated (they are still counted in d_samples).
 * Errors: VR_ERR_NULL, VR_ERR_DIMS, VR_ERR_RANGE (step, fov, spacing),
 * VR_ERR_DTYPE, VR_ERR_HIP.
 */
int vr_raycast(const vr_volume* vol, const float* d_tf, const vr_camera* h_cams, int n_views,
               const vr_render_opts* opts, float* d_rgba, uint64_t* d_samples, void* stream);

/*
 * Best-view snapshot (Section III-C, Eq. 2).  For each of n_views RGBA frames
 * (f32 [n_views][height][width][4], background already composited, alpha
 * ignored) the 256-bin histogram of the pixels' grey values, each RGB channel
 * coded as q = floor(255 clamp(c, 0, 1) + 1/2) in FP32 (product, then sum)
 * and grey = (77 q_r + 150 q_g + 29 q_b + 128) >> 8; its Shannon entropy
 * H = -sum_i p_i log2 p_i over the non-empty bins (p_i = count_i / pixels,
 * FP64); and the first view of maximal entropy.
 *   d_hist: [n_views][256] uint32, overwritten (the counts).
 *   d_entropy: [n_views] double, overwritten (bits).
 *   d_best: one int32, overwritten (the view index).
 * Errors: VR_ERR_NULL, VR_ERR_DIMS (empty or more than 2^32 - 1 pixels per
 * frame, more than 65535 views), VR_ERR_HIP.
 */
int vr_frame_entropy(const float* d_rgba, int n_views, int width, int height, uint32_t* d_hist,
                     double* d_entropy, int32_t* d_best, void* stream);

/* The entropies and the best view of vr_frame_entropy from grey-value counts
 * already taken (vr_raycast with opts->view_hist set), pixels per frame.
 * Errors: VR_ERR_NULL, VR_ERR_DIMS, VR_ERR_HIP. */
int vr_entropy_from_counts(const uint32_t* d_hist, int n_views, int64_t pixels, double* d_entropy,
                           int32_t* d_best, void* stream);

/*
 * Adjoint of vr_raycast for an f32 density grid: given dLoss/dRGBA, adds
 * dLoss/dDensity to d_grad_density ([nz][ny][nx] f32) and dLoss/dTF to
 * d_grad_tf (256 x 4 f32).  Accumulates: the caller zeroes both first.  Each
 * ray is re-marched with the same samples and the same early-termination
 * decisions as the forward pass (nothing is stored per sample); d_rgba_fwd
 * must be the forward output of the same inputs.
 * Gradient of sample i (length len, transmittance T_i before it, colour
 * prefix P_i including it, output I):
 *   dI_rgb/drgb_i = T_i alpha_i,
 *   dI_rgb/dsigma_i = len (T_i e_i rgb_i - (I_rgb - P_i)),
 *   dI_a/dsigma_i = len (1 - I_a),
 * then through the transfer-function interpolation to the two knots, and
 * through the trilinear weights to the eight taps (f32 atomics; the
 * summation order is not deterministic).
 * The density must be VR_F32 in VR_LAYOUT_LINEAR or VR_LAYOUT_BRICK4
 * (VR_ERR_DTYPE, VR_ERR_UNSUPPORTED otherwise); d_grad_density has the
 * density's layout ([nz][ny][nx], or vr_brick_count(...) * 64 elements in
 * bricks, to be brought back with vr_unbrick_volume).  The brick layout is
 * the faster one: a cell's eight taps share one or two cache lines there, and
 * the gradient's atomics go out a cache line at a time.  vol->occupancy may be NULL, or the
 * occupancy grid that vr_brick_volume wrote for the same grid (marks of
 * non-zero voxels: occupancy_above is 0 for f32): then, when the
 * TF's first segment has zero extinction (tf[0].sigma = tf[1].sigma = 0,
 * finite colour), runs of samples whose base tap lies in an empty brick are
 * not marched.  Their colour, transmittance and density gradient are
 * unchanged, and the one gradient they carry, len * (grad . (T tf[0].rgb -
 * (I - P)) + grad_a (1 - I_a)) to tf[0].sigma, is added once per run (the same
 * value up to floating-point summation order).
 * Errors: as vr_raycast.
 */
int vr_raycast_backward(const vr_volume* vol, const float* d_tf, const vr_camera* h_cams,
                        int n_views, const vr_render_opts* opts, const float* d_rgba_fwd,
                        const float* d_grad_rgba, float* d_grad_density, float* d_grad_tf,
                        void* stream);

/*
 * Batched previews in one persistent launch (beyond the paper: many scans
 * processed together, as a preview service would).  For every item: both
 * histograms (vr_histogram_with_top), threshold selection, the fused level-1
 * pyramid step, the brick layout with occupancy of level 1, and n_views
 * frames ray cast from level 1 (vr_raycast semantics; the cameras are in the
 * level-1 volume's world frame, whose voxel size is `spacing`).  A launch is
 * a persistent kernel (one workgroup per compute unit) running a device task
 * queue with per-item dependency counters for the reduction and brick phases,
 * then, on the same stream, one kernel that renders every item's tiles in
 * one-wave workgroups; the launch can be captured into a HIP graph
 * (vr_batch_capture, both kernels in one graph) and replayed.  Results equal those of the
 * single-volume calls (bit-identical reduction, and bit-identical frames for
 * the same bricked level).
 *
 * The caller provides one workspace of vr_batch_workspace_size bytes holding
 * every intermediate (histograms, masks, levels, bricks, occupancy, task
 * table, counters); the plan keeps pointers into it.  The first call of the
 * plan's lifetime initialises it (synchronously); launches never allocate.
 * Items must not change between launches (their pointers are in the plan).
 */
typedef struct vr_batch_plan vr_batch_plan;

typedef struct {
    const uint16_t* d_vol;     /* [nz][ny][nx] u16 */
    int64_t nx, ny, nz;
    double spacing[3];         /* world units per level-1 voxel (> 0) */
    int32_t n_views;           /* 1..VR_MAX_VIEWS_PER_LAUNCH */
    const vr_camera* h_cams;   /* host, read during plan creation */
    float* d_frames;           /* [n_views][height][width][4] f32 */
} vr_batch_item;

typedef struct {
    int32_t width, height;     /* frame size of every view */
    float step, ert_eps;       /* as vr_render_opts */
    float bg[4];
    int32_t rule, rule_param;  /* as vr_select_threshold */
    int32_t top_slices;        /* slices of the top histogram (3 in the paper) */
    int32_t wave_w, wave_h;    /* ray tile of one wave, wave_w * wave_h == 64 */
    int32_t waves_x;           /* waves across a render task's tile (16 waves per task; divides 16) */
    int64_t hist_task_voxels;  /* voxels per histogram task (>= 8192) */
    int32_t down_tiles_per_task;   /* 64x16x16 tiles per pyramid task */
    int32_t slabs_per_task;    /* 16-brick slabs per brick task (8^3 bricks: 256 row pieces each) */
    int32_t render_tiles_per_task; /* must be 1 */
    int32_t brick_edge;        /* level-1 bricks of 4 (or 0) or 8 voxels a side */
} vr_batch_config;

int vr_batch_workspace_size(const vr_batch_item* items, int n_items, const vr_batch_config* cfg,
                            int64_t* bytes);
int vr_batch_plan_create(const vr_batch_item* items, int n_items, const vr_batch_config* cfg,
                         const float* d_tf, void* d_workspace, int64_t workspace_bytes,
                         vr_batch_plan** plan);
/* One launch on `stream`: the persistent kernel, then the render kernel (the
 * captured graph once vr_batch_capture ran). */
int vr_batch_launch(vr_batch_plan* plan, void* stream);
/* Capture the launch into a HIP graph; later vr_batch_launch calls replay it. */
int vr_batch_capture(vr_batch_plan* plan, void* stream);
/* Synchronous: status != 0 if a task timed out waiting; samples [taken, evaluated] so far. */
int vr_batch_status(vr_batch_plan* plan, uint32_t* h_status, uint64_t* h_samples);
/* Device pointers of an item's level 1 and selection result, and the task count. */
int vr_batch_item_outputs(const vr_batch_plan* plan, int item, uint16_t** d_level1,
                          uint32_t** d_result, int64_t* n_tasks);
int vr_batch_plan_destroy(vr_batch_plan* plan);

/* Message for the last non-zero return on this host thread ("" if none). */
const char* vr_last_error(void);

/* Library version string. */
const char* vr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* VR_H */
