// Internal declarations shared by the host API (po_api.cpp) and the HIP
// kernels (po_kernels.hip) of libplenoctree.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "plenoctree.h"

// Kernel-side view of a bound tree (plain data, passed by value).
struct KTree {
    const int32_t* child;   // [n_nodes][8]
    const void* sigma;      // [n_leaves] float or half
    const void* sh;         // [n_leaves][stride] float or half
    union {                 // a tree has SG lobes or a codebook, never both
        const float* lobes;     // cb_entries == 0: nullptr (SH basis) or [K][4] spherical-Gaussian lobes
        const void* codebook;   // cb_entries > 0: [K][cb_entries][4] float16 colours; sh holds uint16 indices
    };
    int32_t n_nodes;
    int32_t n_leaves;
    int32_t stride;         // elements per SH record
    int32_t depth;          // D
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
hipError_t po_launch_camera_rays(const KCam& cam, float* o, float* d, hipStream_t s);
// Visibility filter: mode 0 alpha, 1 contribution; weight[n_leaves] raised in place, alpha[H*W] or nullptr.
hipError_t po_launch_leaf_weights(const po_tree* t, const KCam& cam, const KOpts& op, int mode, float* weight,
                                  float* alpha, hipStream_t s);
hipError_t po_launch_mse_grad(int64_t n, const float* rgb, const float* target, float scale, float* grad,
                              float* sq_sum, hipStream_t s);
hipError_t po_launch_sgd(int64_t n, float* param, float* grad, float lr, bool zero_grad, hipStream_t s);
hipError_t po_read_device_errors(unsigned long long* out);
// Kernel variant a tree renders with (dtype, K, record-load plan); jobs of one
// batched launch must share it.
int po_plan_id(const po_tree* t);
hipError_t po_reset_device_errors();
