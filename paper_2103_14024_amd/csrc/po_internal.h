// Internal declarations shared by the host API (po_api.cpp) and the HIP
// kernels (po_kernels.hip) of libplenoctree.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime_api.h>
#include <hip/hip_vector_types.h>
#include <stdint.h>

#include "plenoctree.h"

// Kernel-side view of a bound tree (plain data, passed by value).
struct KTree {
    // Child entries the walk reads: the caller's child array [n_top][8], or
    // the library's traversal index (po_tree_build_index): the nodes above
    // brick_level, renumbered, [n_top][8], then one brick of 8x8x8 cells per
    // internal node of level brick_level, [n_bricks][512].  An entry of a
    // level-brick_level cell >= n_top names brick (entry - n_top).  A brick
    // entry is ((leaf + 1) << 2) | (D - level) of the leaf holding the cell
    // (0 << 2 for empty space), indexed by the child slots of the three levels
    // below the brick's cube (slot1 << 6 | slot2 << 3 | slot3).
    const int32_t* child;
    const void* sigma;      // [n_leaves] float or half
    const void* sh;         // [n_leaves][stride] float or half
    union {                 // a tree has SG lobes or a codebook, never both
        const float* lobes;     // cb_entries == 0: nullptr (SH basis) or [K][4] spherical-Gaussian lobes
        const void* codebook;   // cb_entries > 0: [K][cb_entries][4] float16 colours; sh holds uint16 indices
    };
    int32_t n_top;          // nodes in `child` (all of the caller's nodes when brick_level == depth)
    int32_t n_leaves;
    int32_t stride;         // elements per SH record
    int16_t depth;          // D
    int16_t brick_level;    // M: cells below level M are resolved by bricks; M == D: no bricks
    uint32_t index_bytes;   // bytes readable through `child`
    int32_t cb_entries;     // codebook entries per basis function (0: no codebook)
    uint32_t sigma_bytes;   // n_leaves * element size (< 2^32)
    uint32_t sh_bytes;      // n_leaves * stride * element size (< 2^32 - 256)
    double lo[3];           // box minimum corner, world units
    double scale;           // grid units (finest cells) per world unit: 2^D / (2 half)
};

struct KOpts {
    float bg[3];
    float stop_T;
    int32_t max_steps;
    uint32_t flags;
    uint32_t sh_off;        // viewer: SH basis functions left out
    float clip[4];          // viewer: slicing half-space n.x + w >= 0 (all zero: none)
};

// True when a render needs the viewer kernels (aux outputs with depth, SH
// subsets or a slicing plane); the plain kernels serve every other call.
inline bool po_view_opts(const KOpts& k, const float* aux) {
    return aux != nullptr || k.sh_off != 0u || k.clip[0] != 0.0f || k.clip[1] != 0.0f || k.clip[2] != 0.0f ||
           k.clip[3] != 0.0f;
}

// Compiled variants of the forward render: plain with the SH basis, plain
// with spherical Gaussians, and the viewer kernel (either basis, chosen per
// tree at run time).  The plain kernels carry no code for the other basis.
// Codebook trees render with PO_FWD_CB and take no viewer options.
enum { PO_FWD_SH = 0, PO_FWD_SG = 1, PO_FWD_VIEW = 2, PO_FWD_CB = 3 };
inline int po_fwd_variant(const KOpts& k, const float* aux, const KTree& t) {
    if (t.cb_entries > 0) return PO_FWD_CB;
    return po_view_opts(k, aux) ? PO_FWD_VIEW : (t.lobes ? PO_FWD_SG : PO_FWD_SH);
}

struct KCam {
    float c2w[12];
    int32_t W, H;
    float fx, fy, cx, cy;
};

// One camera job of a batched launch.
struct KJob {
    KTree tr;
    KCam cam;
    KOpts op;
    float* rgb;
    float* aux;
    int32_t tile_begin;     // first 16x16 tile of the image rendered by this job
    int32_t block_begin;    // first workgroup (before the XCD swizzle) of this job: 4 per 16x16 tile
    int32_t tiles_x;        // ceil(W / 16)
    int32_t pad_;
};

// Work queues of the split camera render: rays whose walk outlasts
// split_steps cells are handed on as 1-16 chunks, and chunks that outlast
// chunk_cap cells hand their remainder on as 1-16 sub-chunks.  Each queue has
// kSplitRegions regions of region_slots slots (a multiple of 64), one counter
// each: kSplitRegionSlots for the queues the library allocates,
// kNoAllocRegionSlots for the fixed queue of the entry point that allocates
// nothing.  A walk whose region is full finishes in its own lane, so the size
// changes the speed, never the result.
#ifndef PO_SPLIT_REGION_SLOTS
#define PO_SPLIT_REGION_SLOTS 16384
#endif
constexpr int kSplitRegions = 64;
constexpr int kSplitRegionSlots = PO_SPLIT_REGION_SLOTS;
constexpr int kNoAllocRegionSlots = 8192;
constexpr int kSplitMaxChunks = 16;
#ifndef PO_SPLIT_STEPS
#define PO_SPLIT_STEPS 28
#endif
#ifndef PO_CHUNK_STEPS
#define PO_CHUNK_STEPS 24
#endif
#ifndef PO_SUB_STEPS
#define PO_SUB_STEPS 10
#endif
#ifndef PO_CHUNK_CAP
#define PO_CHUNK_CAP 24
#endif
// (0.3 against 0.2: 800x800 0.531 against 0.536 ms, 512x512 0.361 against
// 0.366 ms, 1920x1080 unchanged, 1280x720 0.841 against 0.834 ms)
#ifndef PO_SPLIT_UB_FRAC
#define PO_SPLIT_UB_FRAC 0.3f
#endif
// Cells the first walk of a split camera render takes before it hands a ray
// on, from the number of waves in the launch (four per 16x16 tile).  About
// kResidentWaves waves fit on the chip at once (256 CUs x 4 SIMDs x 4 waves
// at 128 VGPRs); a launch of several such rounds keeps the chip busy through
// its first walk, so its rays walk further before the hand-off and fewer of
// them wait in the chunk queues (depth-9 scene, float32 leaves: 800x800 0.588
// -> 0.551 ms, 1920x1080 1.78 -> 1.38 ms against a fixed 28 cells; the
// regions of a 1920x1080 frame no longer overflow; 18 cells per round with
// 10-cell sub-chunks instead of 16 with 12: 800x800 0.5365 against 0.5409 ms,
// 1920x1080 1.357 against 1.352 ms).  Ray-list passes keep PO_SPLIT_STEPS:
// their render and backward must cut the rays alike.
constexpr int64_t kResidentWaves = 4096;
inline int po_camera_split_steps(int64_t waves) {
    const int64_t s = 20 + 18 * waves / kResidentWaves;
    return (int)(s < PO_SPLIT_STEPS ? PO_SPLIT_STEPS : s > 192 ? 192 : s);
}
// piece sizes of ray-list passes (render and backward) of fewer than
// PO_RAYS_SMALL rays
#ifndef PO_RAYS_SMALL
#define PO_RAYS_SMALL (1 << 18)
#endif
#ifndef PO_RAYS_SPLIT_STEPS
#define PO_RAYS_SPLIT_STEPS 4
#endif
#ifndef PO_RAYS_CHUNK_STEPS
#define PO_RAYS_CHUNK_STEPS 6
#endif
#ifndef PO_RAYS_CHUNK_CAP
#define PO_RAYS_CHUNK_CAP 12
#endif
#ifndef PO_RAYS_UB_FRAC
#define PO_RAYS_UB_FRAC 0.2f
#endif
struct KSplit {
    int32_t* count;        // [kSplitRegions] chunk slots claimed (may exceed the region); count2 follows
    int32_t* count2;       // [kSplitRegions] sub-chunk slots claimed
    int4* info;            // [slots] {first chunk slot of the ray (-1: unused), chunk | count << 8, next chunk slot, 0}
    void* head;            // [slots] 32-byte ray states, at the first slot of each ray
    void* part;            // [slots] 32-byte chunk results
    int4* info2;           // [slots] the same for the sub-chunks of remainders
    void* head2;           // [slots] 32-byte remainders, at their first slot
    void* part2;           // [slots] 32-byte sub-chunk results
    int4* view_part;       // [slots] viewer variant: chunk samples, cells and cut flags
    int4* view_part2;      // [slots] the same for the sub-chunks
    int32_t region_slots;  // slots per region; slots = kSplitRegions * region_slots
    int32_t split_steps;   // cells walked before a ray is handed on
    int32_t chunk_steps;   // target cells per chunk
    int32_t sub_steps;     // target cells per sub-chunk
    int32_t chunk_cap;     // cells a chunk walks before its remainder is handed on
    float ub_frac;         // pieces cover at least this fraction of the finest-cell faces ahead
    const float* ray_o;    // ray-list renders: origins [n_rays][3] (camera renders: unused)
    const float* ray_d;    // ray-list renders: directions [n_rays][3]
    int64_t n_rays;
    int32_t* ray_slot;     // kept ray-list render: [n_rays] first chunk slot of each ray, -1 if not handed on
};
// Piece sizes of a split pass over a list of n rays.  The render and the
// backward of the same rays cut them alike: the transmittance in front of
// every piece is then the same float product in both, so the backward stops
// on the sample where the render that produced its colour stopped.
// (Training step, 65,536 random rays of the depth-8 tree, forward and
// backward over the same pieces: 0.558 ms with a 28-cell first walk and
// 8-cell pieces (cap 16), 0.460 ms with a 4-cell first walk and 6-cell
// pieces (cap 12).)
inline void po_rays_piece_sizes(int64_t n, KSplit* S) {
    if (n < PO_RAYS_SMALL) {
        S->split_steps = PO_RAYS_SPLIT_STEPS;
        S->chunk_steps = PO_RAYS_CHUNK_STEPS;
        S->sub_steps = PO_RAYS_CHUNK_STEPS;
        S->chunk_cap = PO_RAYS_CHUNK_CAP;
        S->ub_frac = PO_RAYS_UB_FRAC;
    }
}
// Device bytes of the queues with region_slots slots per region (counters,
// then info, head, part and viewer record of each queue).
constexpr size_t po_split_bytes(int region_slots) {
    return 512 + 2 * (size_t)kSplitRegions * (size_t)region_slots * (16 + 32 + 32 + 16);
}
// Points S at queues laid out in `base` (po_split_bytes(region_slots) bytes)
// and sets the default piece sizes.
void po_split_layout(void* base, int region_slots, KSplit* S);
// Bytes of the fixed queue of po_render_camera_noalloc (one copy per device,
// a static device array of the library: about 100 MB).
constexpr size_t kNoAllocBytes = po_split_bytes(kNoAllocRegionSlots);
// Images the fixed queue is sized for: larger ones are rejected.
constexpr int64_t kNoAllocMaxPixels = int64_t(1) << 22;
// Points S at the fixed queue of the current device (its device address is
// looked up once per device, under a lock); allocates nothing.
hipError_t po_noalloc_queue(KSplit* S);

struct po_tree {
    po_tree_desc desc;
    int64_t n_nodes, n_leaves;
    const int32_t* child;
    const void* sigma;
    const void* sh;
    int32_t K;              // coefficients per channel
    int32_t stride;         // elements per SH record
    int32_t vec_bytes;      // widest aligned load of a record: 16, 8 or 4
    bool codebook;          // records are codebook indices (float16 densities)
    void* d_index;          // traversal index owned by the handle (nullptr: none built)
    int index_device;       // device holding d_index
    int64_t n_bricks;
    KTree kt;
};

// Sets the thread's po_last_error message (cleared for PO_OK) and returns s.
po_status po_report(po_status s, const char* msg);

// Launchers (po_kernels.hip).  Arguments are validated by the caller.
hipError_t po_launch_rays(const po_tree* t, int64_t n, const float* o, const float* d,
                          const KOpts& op, float* rgb, float* aux, hipStream_t s);
hipError_t po_launch_backward(const po_tree* t, int64_t n, const float* o, const float* d,
                              const KOpts& op, const float* rgb_fwd, const float* grad_rgb,
                              float* grad_sigma, float* grad_sh, hipStream_t s);
// Renders camera jobs that all share dtype, K and vec_bytes (at most
// PO_BATCH_MAX_JOBS) and the same po_fwd_variant; n_blocks counts
// workgroups, four per 16x16 tile.
hipError_t po_launch_camera_jobs(const po_tree* first, int n_jobs, KJob* jobs, int n_blocks, int variant,
                                 hipStream_t s);
// One camera job as the split render (any forward variant): clears the queue
// counters and launches the four render kernels.
// The queue must not be in use by work on another stream.
hipError_t po_launch_camera_split(const po_tree* t, const KJob& job, int n_blocks, int variant, const KSplit& S,
                                  hipStream_t s);
// n rays (n < 2^31) as the split render (any forward variant; aux for the
// viewer variant); the queue must not be in use by work on another stream.
hipError_t po_launch_rays_split(const po_tree* t, int64_t n, const float* o, const float* d, const KOpts& op,
                                float* rgb, float* aux, const KSplit& S, hipStream_t s);
// Backward of n rays (n < 2^31, float32 tree) in pieces: the first walk,
// the forward of the pieces, their prefixes, then the backward of the pieces.
hipError_t po_launch_backward_split(const po_tree* t, int64_t n, const float* o, const float* d, const KOpts& op,
                                    const float* rgb_fwd, const float* grad, float* gsig, float* gsh,
                                    const KSplit& S, hipStream_t s);
// Backward of the n rays of a kept split render (po_launch_rays_split with
// S.ray_slot set, same rays, options and queue, nothing else on the queue in
// between): the first walk, the prefixes of the render's own pieces, then
// the backward of the pieces.  Consumes the kept pieces.
hipError_t po_launch_backward_kept(const po_tree* t, int64_t n, const float* o, const float* d, const KOpts& op,
                                   const float* rgb_fwd, const float* grad, float* gsig, float* gsh,
                                   const KSplit& S, hipStream_t s);
hipError_t po_launch_camera_rays(const KCam& cam, float* o, float* d, hipStream_t s);
// Visibility filter: mode 0 alpha, 1 contribution; weight[n_leaves] raised in place, alpha[H*W] or nullptr.
hipError_t po_launch_leaf_weights(const po_tree* t, const KCam& cam, const KOpts& op, int mode, float* weight,
                                  float* alpha, hipStream_t s);
// Traversal statistics: writes h_sums[4] = {rays, samples, cells,
// child-entry loads} of the one-pass walk of every pixel ray of *cam, or
// (cam NULL) of the n rays (o, d), waiting for the stream.  Calls must not
// overlap (one device buffer).
hipError_t po_traversal_stats_sync(const po_tree* t, const KCam* cam, int64_t n, const float* o, const float* d,
                                   const KOpts& op, unsigned long long* h_sums, hipStream_t s);
hipError_t po_launch_mse_grad(int64_t n, const float* rgb, const float* target, float scale, float* grad,
                              float* sq_sum, hipStream_t s);
hipError_t po_launch_sgd(int64_t n, float* param, float* grad, float lr, bool zero_grad, hipStream_t s);
hipError_t po_launch_gather_rays(int64_t n, const int64_t* idx, int64_t n_src, const float* o, const float* d,
                                 const float* t, float* bo, float* bd, float* bt, hipStream_t s);
hipError_t po_launch_draw_batch(int64_t n, uint64_t seed, uint64_t first, int64_t n_src, const float* o,
                               const float* d, const float* t, float* bo, float* bd, float* bt, float* sq_sum,
                               hipStream_t s);
hipError_t po_read_device_errors(unsigned long long* out);
// Kernel variant a tree renders with (dtype, K, record-load plan); jobs of one
// batched launch must share it.
int po_plan_id(const po_tree* t);
hipError_t po_reset_device_errors();
