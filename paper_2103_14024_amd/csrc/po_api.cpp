// Host side of libplenoctree: the extern "C" entry points declared in
// include/plenoctree.h.  Validates every argument before any GPU work,
// builds octrees from leaf-cell lists (Sec. 4.2, "Filtering": surviving
// voxels become leaves, everything else is empty), checks child arrays, and
// forwards renders to the HIP launchers in po_kernels.hip.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "po_internal.h"

namespace {

thread_local std::string g_err;

po_status fail(po_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

po_status ok() {
    g_err.clear();
    return PO_OK;
}

po_status device_fail(hipError_t e, const char* what) {
    return fail(PO_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool finite(float v) { return std::isfinite(v); }

// Camera renders of at least kSplitMinPixels pixels and ray-list renders of
// at least kSplitMinRays rays use the split render.  Its five launches each
// end with their own longest walk, which outweighs the shorter critical path
// for small launches.
constexpr int64_t kSplitMinPixels = 1 << 16;
#ifndef PO_SPLIT_MIN_RAYS
#define PO_SPLIT_MIN_RAYS (1 << 16)
#endif
constexpr int64_t kSplitMinRays = PO_SPLIT_MIN_RAYS;
// Backward passes of at least this many rays run in pieces.
#ifndef PO_SPLIT_MIN_BACKWARD
#define PO_SPLIT_MIN_BACKWARD (1 << 16)
#endif
constexpr int64_t kSplitMinBackward = PO_SPLIT_MIN_BACKWARD;

// Work queues of the split camera render, one per (device, stream), made on
// first use and kept until the process ends.
std::mutex g_split_mu;
std::map<std::pair<int, void*>, void*> g_split;

// The last kept ray-list render on a queue (po_render_rays_keep): its pieces
// stay valid until the next split launch on that queue or the backward that
// consumes them.  Guarded by g_split_mu.
struct Kept {
    bool valid = false, split = false;
    const po_tree* t = nullptr;
    int64_t n = 0;
    const float* o = nullptr;
    const float* d = nullptr;
    const int32_t* slot = nullptr;
    po_render_opts opts;
};
std::map<std::pair<int, void*>, Kept> g_kept;

// The queue of (current device, stream), allocated on first use; every
// split launch takes it through here, which ends the validity of a kept
// render's pieces in it.
bool split_queue(void* stream, KSplit* S) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    void* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_split_mu);
        g_kept[{dev, stream}].valid = false;
        auto it = g_split.find({dev, stream});
        if (it != g_split.end()) {
            base = it->second;
        } else {
            if (hipMalloc(&base, po_split_bytes(kSplitRegionSlots)) != hipSuccess) {
                (void)hipGetLastError();
                return false;
            }
            g_split[{dev, stream}] = base;
        }
    }
    po_split_layout(base, kSplitRegionSlots, S);
    return true;
}

}  // namespace

po_status po_report(po_status s, const char* msg) { return s == PO_OK ? ok() : fail(s, "%s", msg); }

void po_split_layout(void* base, int region_slots, KSplit* S) {
    char* p = static_cast<char*>(base);
    const size_t n = (size_t)kSplitRegions * (size_t)region_slots;
    S->count = reinterpret_cast<int32_t*>(p);
    S->count2 = S->count + kSplitRegions;
    p += 512;
    S->info = reinterpret_cast<int4*>(p);
    S->head = p + n * 16;
    S->part = p + n * 48;
    S->view_part = reinterpret_cast<int4*>(p + n * 80);
    p += n * 96;
    S->info2 = reinterpret_cast<int4*>(p);
    S->head2 = p + n * 16;
    S->part2 = p + n * 48;
    S->view_part2 = reinterpret_cast<int4*>(p + n * 80);
    S->region_slots = region_slots;
    S->split_steps = PO_SPLIT_STEPS;
    S->chunk_steps = PO_CHUNK_STEPS;
    S->sub_steps = PO_SUB_STEPS;
    S->chunk_cap = PO_CHUNK_CAP;
    S->ub_frac = PO_SPLIT_UB_FRAC;
    S->ray_o = nullptr;
    S->ray_d = nullptr;
    S->n_rays = 0;
    S->ray_slot = nullptr;
}

namespace {

int elem_size(int32_t dtype) { return dtype == PO_F16 ? 2 : 4; }

// codebook: the records are K uint16 indices per leaf (stride in uint16, 0 =
// K rounded up to a multiple of 4) and the densities must be float16.
po_status check_desc(const po_tree_desc* d, bool codebook = false) {
    if (!d) return fail(PO_ERR_INVALID, "tree description is NULL");
    if (d->depth < 1 || d->depth > PO_MAX_DEPTH)
        return fail(PO_ERR_INVALID, "depth %d outside [1, %d]", d->depth, PO_MAX_DEPTH);
    if (d->sh_degree < 0 || d->sh_degree > PO_MAX_SH_DEGREE)
        return fail(PO_ERR_INVALID, "sh_degree %d outside [0, %d]", d->sh_degree, PO_MAX_SH_DEGREE);
    if (!(d->half_size > 0.0f) || !finite(d->half_size))
        return fail(PO_ERR_INVALID, "half_size must be finite and > 0");
    for (int k = 0; k < 3; ++k)
        if (!finite(d->center[k])) return fail(PO_ERR_INVALID, "center must be finite");
    if (d->dtype != PO_F32 && d->dtype != PO_F16) return fail(PO_ERR_INVALID, "unknown dtype %d", d->dtype);
    const int K = (d->sh_degree + 1) * (d->sh_degree + 1);
    if (codebook) {
        if (d->dtype != PO_F16) return fail(PO_ERR_INVALID, "codebook trees keep float16 densities (dtype PO_F16)");
        const int stride = d->sh_stride ? d->sh_stride : (K + 3) / 4 * 4;
        if (stride < K) return fail(PO_ERR_INVALID, "index stride %d < K = %d", stride, K);
        if (stride % 2) return fail(PO_ERR_INVALID, "index stride %d must be even (whole 4-byte words)", stride);
        return PO_OK;
    }
    const int stride = d->sh_stride ? d->sh_stride : 3 * K;
    if (stride < 3 * K) return fail(PO_ERR_INVALID, "sh_stride %d < 3*K = %d", stride, 3 * K);
    if ((stride * elem_size(d->dtype)) % 4 != 0)
        return fail(PO_ERR_INVALID, "sh_stride * element size (%d bytes) must be a multiple of 4",
                    stride * elem_size(d->dtype));
    return PO_OK;
}

po_status check_opts(const po_render_opts* o) {
    if (!o) return fail(PO_ERR_INVALID, "render options are NULL");
    for (int k = 0; k < 3; ++k)
        if (!finite(o->bg[k])) return fail(PO_ERR_INVALID, "background must be finite");
    if (!(o->stop_T >= 0.0f) || !finite(o->stop_T)) return fail(PO_ERR_INVALID, "stop_T must be finite and >= 0");
    if (o->max_steps < 0) return fail(PO_ERR_INVALID, "max_steps must be >= 0");
    if (o->flags & ~(PO_OUT_AUX | PO_ONE_PASS)) return fail(PO_ERR_INVALID, "unknown flags 0x%x", o->flags);
    for (int k = 0; k < 4; ++k)
        if (!finite(o->clip[k])) return fail(PO_ERR_INVALID, "slicing plane must be finite");
    return PO_OK;
}

KOpts kopts(const po_tree* t, const po_render_opts* o) {
    KOpts k;
    for (int i = 0; i < 3; ++i) k.bg[i] = o->bg[i];
    k.stop_T = o->stop_T;
    k.max_steps = o->max_steps ? o->max_steps : 3 * (1 << t->desc.depth) + 8;
    k.flags = o->flags;
    k.sh_off = o->sh_off;
    for (int i = 0; i < 4; ++i) k.clip[i] = o->clip[i];
    return k;
}

po_status check_camera(const po_camera* c) {
    if (!c) return fail(PO_ERR_INVALID, "camera is NULL");
    if (c->width < 1 || c->height < 1 || c->width > 16384 || c->height > 16384)
        return fail(PO_ERR_INVALID, "image size %dx%d outside [1, 16384]", c->width, c->height);
    if (!finite(c->fx) || !finite(c->fy) || c->fx == 0.0f || c->fy == 0.0f || !finite(c->cx) || !finite(c->cy))
        return fail(PO_ERR_INVALID, "camera intrinsics must be finite with fx, fy != 0");
    for (int i = 0; i < 12; ++i)
        if (!finite(c->c2w[i])) return fail(PO_ERR_INVALID, "camera pose must be finite");
    return PO_OK;
}

int32_t tiles_of(const po_camera* c) {
    return ((c->width + PO_TILE - 1) / PO_TILE) * ((c->height + PO_TILE - 1) / PO_TILE);
}

KCam kcam(const po_camera* c) {
    KCam k;
    std::memcpy(k.c2w, c->c2w, sizeof k.c2w);
    k.W = c->width;
    k.H = c->height;
    k.fx = c->fx;
    k.fy = c->fy;
    k.cx = c->cx;
    k.cy = c->cy;
    return k;
}

// Morton key of finest-level coordinates: bit b of x, y, z goes to bits
// 3b+2, 3b+1, 3b, so the low three bits of a level-L prefix are the child
// slot 4*xbit + 2*ybit + zbit.
uint64_t morton(uint64_t x, uint64_t y, uint64_t z, int D) {
    uint64_t k = 0;
    for (int b = 0; b < D; ++b)
        k |= (((x >> b) & 1ull) << (3 * b + 2)) | (((y >> b) & 1ull) << (3 * b + 1)) | (((z >> b) & 1ull) << (3 * b));
    return k;
}

}  // namespace

struct po_builder {
    po_tree_desc desc;
    int64_t n_cells = 0;
    std::vector<int64_t> order;          // cells sorted by Morton key of their corner
    std::vector<uint64_t> key;           // key of order[r]
    std::vector<int32_t> level;          // level of order[r]
    std::vector<std::vector<uint64_t>> prefixes;  // per level 0..D-1: sorted prefixes of internal nodes
    std::vector<int64_t> offset;         // first node id of each level
    int64_t n_nodes = 0;
};

extern "C" {

const char* po_status_str(po_status s) {
    switch (s) {
        case PO_OK: return "ok";
        case PO_ERR_INVALID: return "invalid argument";
        case PO_ERR_TREE: return "malformed tree";
        case PO_ERR_OOM: return "out of host memory";
        case PO_ERR_DEVICE: return "HIP device error";
        case PO_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char* po_last_error(void) { return g_err.c_str(); }

const char* po_version(void) { return "plenoctree-mi355x 0.1 gfx950"; }

po_status po_builder_create(const po_tree_desc* desc, int64_t n_cells, const int32_t* h_cells, po_builder** out) {
    if (po_status s = check_desc(desc)) return s;
    if (!out) return fail(PO_ERR_INVALID, "out is NULL");
    if (n_cells < 0 || n_cells >= (1ll << 31) - 1) return fail(PO_ERR_INVALID, "n_cells %lld out of range", (long long)n_cells);
    if (n_cells > 0 && !h_cells) return fail(PO_ERR_INVALID, "cells is NULL");
    const int D = desc->depth;
    po_builder* b = new (std::nothrow) po_builder();
    if (!b) return fail(PO_ERR_OOM, "builder allocation");
    try {
        b->desc = *desc;
        b->n_cells = n_cells;
        std::vector<uint64_t> keys((size_t)n_cells);
        for (int64_t q = 0; q < n_cells; ++q) {
            const int32_t lv = h_cells[4 * q], i = h_cells[4 * q + 1], j = h_cells[4 * q + 2], k = h_cells[4 * q + 3];
            if (lv < 1 || lv > D) {
                delete b;
                return fail(PO_ERR_TREE, "cell %lld: level %d outside [1, %d]", (long long)q, lv, D);
            }
            const int64_t n = 1ll << lv;
            if (i < 0 || j < 0 || k < 0 || i >= n || j >= n || k >= n) {
                delete b;
                return fail(PO_ERR_TREE, "cell %lld: coordinates (%d, %d, %d) outside level %d", (long long)q, i, j, k, lv);
            }
            const int s = D - lv;
            keys[q] = morton((uint64_t)i << s, (uint64_t)j << s, (uint64_t)k << s, D);
        }
        b->order.resize((size_t)n_cells);
        for (int64_t q = 0; q < n_cells; ++q) b->order[q] = q;
        std::sort(b->order.begin(), b->order.end(), [&](int64_t a, int64_t c) {
            if (keys[a] != keys[c]) return keys[a] < keys[c];
            return a < c;
        });
        b->key.resize((size_t)n_cells);
        b->level.resize((size_t)n_cells);
        for (int64_t r = 0; r < n_cells; ++r) {
            b->key[r] = keys[b->order[r]];
            b->level[r] = h_cells[4 * b->order[r]];
        }
        // A cell is the Morton interval [key, key + 8^(D - level)); cells overlap iff intervals do.
        for (int64_t r = 1; r < n_cells; ++r) {
            const uint64_t end_prev = b->key[r - 1] + (1ull << (3 * (D - b->level[r - 1])));
            if (b->key[r] < end_prev) {
                const long long a = (long long)b->order[r - 1], c = (long long)b->order[r];
                delete b;
                return fail(PO_ERR_TREE, "cells %lld and %lld overlap", a, c);
            }
        }
        b->prefixes.assign(D, {});
        b->prefixes[0].push_back(0);  // the root always exists
        for (int L = 1; L < D; ++L) {
            auto& P = b->prefixes[L];
            for (int64_t r = 0; r < n_cells; ++r) {
                if (b->level[r] <= L) continue;
                const uint64_t p = b->key[r] >> (3 * (D - L));
                if (P.empty() || P.back() != p) P.push_back(p);
            }
        }
        b->offset.assign(D, 0);
        int64_t total = 0;
        for (int L = 0; L < D; ++L) {
            b->offset[L] = total;
            total += (int64_t)b->prefixes[L].size();
        }
        if (total >= (1ll << 31) / 8) {
            delete b;
            return fail(PO_ERR_INVALID, "tree needs %lld nodes, too many for int32 child entries", (long long)total);
        }
        b->n_nodes = total;
    } catch (const std::bad_alloc&) {
        delete b;
        return fail(PO_ERR_OOM, "builder allocation");
    }
    *out = b;
    return ok();
}

po_status po_builder_sizes(const po_builder* b, int64_t* n_nodes, int64_t* n_leaves) {
    if (!b || !n_nodes || !n_leaves) return fail(PO_ERR_INVALID, "NULL argument");
    *n_nodes = b->n_nodes;
    *n_leaves = b->n_cells;
    return ok();
}

po_status po_builder_emit(const po_builder* b, int32_t* h_child, int64_t* h_leaf_perm) {
    if (!b || !h_child || (b->n_cells > 0 && !h_leaf_perm)) return fail(PO_ERR_INVALID, "NULL argument");
    const int D = b->desc.depth;
    std::memset(h_child, 0, sizeof(int32_t) * 8 * (size_t)b->n_nodes);
    auto node_id = [&](int L, uint64_t p) -> int64_t {
        const auto& P = b->prefixes[L];
        const auto it = std::lower_bound(P.begin(), P.end(), p);
        return b->offset[L] + (it - P.begin());
    };
    for (int L = 1; L < D; ++L) {
        const auto& P = b->prefixes[L];
        for (size_t q = 0; q < P.size(); ++q) {
            const int64_t parent = node_id(L - 1, P[q] >> 3);
            h_child[parent * 8 + (P[q] & 7)] = (int32_t)(b->offset[L] + (int64_t)q);
        }
    }
    for (int64_t r = 0; r < b->n_cells; ++r) {
        const int lv = b->level[r];
        const uint64_t p = b->key[r] >> (3 * (D - lv));
        const int64_t parent = node_id(lv - 1, p >> 3);
        h_child[parent * 8 + (p & 7)] = (int32_t)(-r - 1);
        h_leaf_perm[r] = b->order[r];
    }
    return ok();
}

po_status po_builder_destroy(po_builder* b) {
    delete b;
    return ok();
}

// po_tree_validate's checks; codebook: desc describes a codebook tree (its
// records are index records, whose stride rules differ)
static po_status validate_tree(const po_tree_desc* desc, int64_t n_nodes, const int32_t* h_child,
                               int64_t n_leaves, const void* h_sigma, bool codebook) {
    if (po_status s = check_desc(desc, codebook)) return s;
    if (n_nodes < 1 || n_nodes >= (1ll << 31) / 8) return fail(PO_ERR_INVALID, "n_nodes %lld out of range", (long long)n_nodes);
    if (n_leaves < 0 || n_leaves >= (1ll << 31) - 1) return fail(PO_ERR_INVALID, "n_leaves %lld out of range", (long long)n_leaves);
    if (!h_child) return fail(PO_ERR_INVALID, "child array is NULL");
    const int D = desc->depth;
    try {
        std::vector<int32_t> lvl((size_t)n_nodes, -1);
        std::vector<uint8_t> leaf_seen((size_t)n_leaves, 0);
        std::vector<int64_t> queue;
        queue.reserve((size_t)n_nodes);
        lvl[0] = 0;
        queue.push_back(0);
        for (size_t h = 0; h < queue.size(); ++h) {
            const int64_t v = queue[h];
            for (int c = 0; c < 8; ++c) {
                const int32_t e = h_child[v * 8 + c];
                if (e > 0) {
                    if (e >= n_nodes)
                        return fail(PO_ERR_TREE, "node %lld slot %d: child %d outside [1, %lld)", (long long)v, c, e, (long long)n_nodes);
                    if (lvl[e] >= 0)
                        return fail(PO_ERR_TREE, "node %d is referenced more than once (cycle or shared subtree)", e);
                    if (lvl[v] + 1 >= D)
                        return fail(PO_ERR_TREE, "node %d is an internal node at depth %d (max depth %d)", e, lvl[v] + 1, D);
                    lvl[e] = lvl[v] + 1;
                    queue.push_back(e);
                } else if (e < 0) {
                    const int64_t leaf = -(int64_t)e - 1;
                    if (leaf >= n_leaves)
                        return fail(PO_ERR_TREE, "node %lld slot %d: leaf %lld outside [0, %lld)", (long long)v, c, (long long)leaf, (long long)n_leaves);
                    if (leaf_seen[leaf]) return fail(PO_ERR_TREE, "leaf %lld is referenced more than once", (long long)leaf);
                    leaf_seen[leaf] = 1;
                }
            }
        }
        if ((int64_t)queue.size() != n_nodes)
            return fail(PO_ERR_TREE, "%lld of %lld nodes are unreachable from the root", (long long)(n_nodes - (int64_t)queue.size()), (long long)n_nodes);
    } catch (const std::bad_alloc&) {
        return fail(PO_ERR_OOM, "validator allocation");
    }
    if (h_sigma) {
        for (int64_t i = 0; i < n_leaves; ++i) {
            bool bad;
            if (desc->dtype == PO_F32) {
                bad = !std::isfinite(static_cast<const float*>(h_sigma)[i]);
            } else {
                const uint16_t h = static_cast<const uint16_t*>(h_sigma)[i];
                bad = ((h >> 10) & 0x1f) == 0x1f;
            }
            if (bad) return fail(PO_ERR_TREE, "leaf %lld has a non-finite density", (long long)i);
        }
    }
    return ok();
}

po_status po_tree_validate(const po_tree_desc* desc, int64_t n_nodes, const int32_t* h_child, int64_t n_leaves,
                           const void* h_sigma) {
    return validate_tree(desc, n_nodes, h_child, n_leaves, h_sigma, false);
}

po_status po_tree_leaf_cells(const po_tree_desc* desc, int64_t n_nodes, const int32_t* h_child, int64_t n_leaves,
                             int32_t* h_cells) {
    if (po_status s = po_tree_validate(desc, n_nodes, h_child, n_leaves, nullptr)) return s;
    if (!h_cells && n_leaves > 0) return fail(PO_ERR_INVALID, "cells array is NULL");
    for (int64_t i = 0; i < 4 * n_leaves; ++i) h_cells[i] = -1;
    try {
        // breadth-first from the root with each node's cell (level, i, j, k)
        struct Item {
            int32_t node, level, i, j, k;
        };
        std::vector<Item> queue;
        queue.reserve((size_t)n_nodes);
        queue.push_back({0, 0, 0, 0, 0});
        for (size_t h = 0; h < queue.size(); ++h) {
            const Item v = queue[h];
            for (int c = 0; c < 8; ++c) {
                const int32_t e = h_child[(int64_t)v.node * 8 + c];
                const Item ch = {e, v.level + 1, 2 * v.i + ((c >> 2) & 1), 2 * v.j + ((c >> 1) & 1), 2 * v.k + (c & 1)};
                if (e > 0) {
                    queue.push_back(ch);
                } else if (e < 0) {
                    int32_t* out = h_cells + 4 * (-(int64_t)e - 1);
                    out[0] = ch.level;
                    out[1] = ch.i;
                    out[2] = ch.j;
                    out[3] = ch.k;
                }
            }
        }
    } catch (const std::bad_alloc&) {
        return fail(PO_ERR_OOM, "leaf cell walk allocation");
    }
    return ok();
}

static po_status bind_impl(const po_tree_desc* desc, int64_t n_nodes, const int32_t* d_child, int64_t n_leaves,
                           const void* d_sigma, const void* d_sh, const float* d_lobes, const void* d_codebook,
                           int32_t cb_entries, po_tree** out) {
    const bool cb = d_codebook != nullptr;
    if (po_status s = check_desc(desc, cb)) return s;
    if (!out) return fail(PO_ERR_INVALID, "out is NULL");
    if (n_nodes < 1 || n_nodes >= (1ll << 31) / 8) return fail(PO_ERR_INVALID, "n_nodes %lld out of range", (long long)n_nodes);
    if (n_leaves < 0 || n_leaves >= (1ll << 31) - 1) return fail(PO_ERR_INVALID, "n_leaves %lld out of range", (long long)n_leaves);
    if (!d_child) return fail(PO_ERR_INVALID, "child array is NULL");
    if (n_leaves > 0 && (!d_sigma || !d_sh)) return fail(PO_ERR_INVALID, "leaf arrays are NULL");
    const int es = elem_size(desc->dtype);
    if (((uintptr_t)d_child) % 4 || ((uintptr_t)d_sigma) % es || ((uintptr_t)d_sh) % 4)
        return fail(PO_ERR_INVALID, "misaligned device array");
    {
        // the kernels address each array through a 32-bit buffer offset
        const int K = (desc->sh_degree + 1) * (desc->sh_degree + 1);
        const int64_t stride = desc->sh_stride ? desc->sh_stride : (cb ? (K + 3) / 4 * 4 : 3 * K);
        const uint64_t lim = (1ull << 32) - 256;
        if ((uint64_t)n_nodes * 32u >= lim || (uint64_t)n_leaves * es >= lim ||
            (uint64_t)n_leaves * (uint64_t)stride * es >= lim)
            return fail(PO_ERR_UNSUPPORTED, "a tree array exceeds 4 GiB");
    }
    if (cb && (cb_entries < 1 || cb_entries > 65536))
        return fail(PO_ERR_INVALID, "codebook size %d outside [1, 65536]", cb_entries);
    if (cb && ((uintptr_t)d_codebook) % 8) return fail(PO_ERR_INVALID, "codebook must be 8-byte aligned");
    po_tree* t = new (std::nothrow) po_tree();
    if (!t) return fail(PO_ERR_OOM, "tree handle allocation");
    t->desc = *desc;
    t->n_nodes = n_nodes;
    t->n_leaves = n_leaves;
    t->child = d_child;
    t->sigma = d_sigma;
    t->sh = d_sh;
    t->K = (desc->sh_degree + 1) * (desc->sh_degree + 1);
    t->codebook = cb;
    t->d_index = nullptr;
    t->index_device = -1;
    t->n_bricks = 0;
    t->stride = desc->sh_stride ? desc->sh_stride : (cb ? (t->K + 3) / 4 * 4 : 3 * t->K);
    const size_t rb = (size_t)t->stride * es;
    t->vec_bytes = 4;
    for (int v : {16, 8}) {
        if (((uintptr_t)d_sh) % v == 0 && rb % v == 0) {
            t->vec_bytes = v;
            break;
        }
    }
    KTree& k = t->kt;
    k.child = d_child;
    k.sigma = d_sigma;
    k.sh = d_sh;
    if (cb)
        k.codebook = d_codebook;
    else
        k.lobes = d_lobes;
    k.cb_entries = cb ? cb_entries : 0;
    k.n_top = (int32_t)n_nodes;
    k.brick_level = (int16_t)desc->depth;  // no bricks until po_tree_build_index
    k.index_bytes = (uint32_t)(n_nodes * 32);
    k.n_leaves = (int32_t)n_leaves;
    k.stride = t->stride;
    k.depth = (int16_t)desc->depth;
    k.sigma_bytes = (uint32_t)(n_leaves * es);
    k.sh_bytes = (uint32_t)(n_leaves * (int64_t)t->stride * es);
    for (int a = 0; a < 3; ++a) k.lo[a] = (double)desc->center[a] - (double)desc->half_size;
    k.scale = (double)(1 << desc->depth) / (2.0 * (double)desc->half_size);
    *out = t;
    return ok();
}

po_status po_tree_bind(const po_tree_desc* desc, int64_t n_nodes, const int32_t* d_child, int64_t n_leaves,
                       const void* d_sigma, const void* d_sh, po_tree** out) {
    return bind_impl(desc, n_nodes, d_child, n_leaves, d_sigma, d_sh, nullptr, nullptr, 0, out);
}

po_status po_tree_bind_codebook(const po_tree_desc* desc, int64_t n_nodes, const int32_t* d_child, int64_t n_leaves,
                                const void* d_sigma, const uint16_t* d_index, const void* d_codebook, int32_t M,
                                po_tree** out) {
    if (!d_codebook) return fail(PO_ERR_INVALID, "codebook is NULL");
    return bind_impl(desc, n_nodes, d_child, n_leaves, d_sigma, d_index, nullptr, d_codebook, M, out);
}

po_status po_tree_bind_sg(const po_tree_desc* desc, int64_t n_nodes, const int32_t* d_child, int64_t n_leaves,
                          const void* d_sigma, const void* d_sh, const float* d_lobes, po_tree** out) {
    if (!d_lobes) return fail(PO_ERR_INVALID, "lobe array is NULL");
    if (((uintptr_t)d_lobes) % 16) return fail(PO_ERR_INVALID, "lobe array must be 16-byte aligned");
    return bind_impl(desc, n_nodes, d_child, n_leaves, d_sigma, d_sh, d_lobes, nullptr, 0, out);
}

// Traversal index of a valid tree of depth D >= 4 (host copy h of its child
// array): the nodes above level M = D - 3 renumbered in breadth-first order,
// their entries of level-M internal nodes replaced by n_top + brick number,
// then one 512-entry brick per internal node of level M.
static po_status index_of(const po_tree_desc* desc, bool codebook, int64_t n, const int32_t* h, int64_t n_leaves,
                          std::vector<int32_t>& index, int64_t& n_top, int64_t& n_bricks) {
    if (po_status st = validate_tree(desc, n, h, n_leaves, nullptr, codebook)) return st;
    const int D = desc->depth;
    const int M = D - 3;
    if (n_leaves >= (1ll << 29) - 1)
        return fail(PO_ERR_UNSUPPORTED, "traversal index: %lld leaves exceed 2^29 - 2", (long long)n_leaves);
    try {
        // levels in breadth-first order from the root (the array is a valid tree)
        std::vector<int32_t> lvl((size_t)n, -1), id((size_t)n, -1);
        std::vector<int64_t> order;
        order.reserve((size_t)n);
        lvl[0] = 0;
        order.push_back(0);
        for (size_t q = 0; q < order.size(); ++q)
            for (int c = 0; c < 8; ++c) {
                const int32_t ch = h[(size_t)order[q] * 8 + c];
                if (ch > 0) {
                    lvl[ch] = lvl[order[q]] + 1;
                    order.push_back(ch);
                }
            }
        // nodes above level M keep their breadth-first order from 0; the
        // internal nodes of level M become bricks in the same order
        n_top = 0;
        n_bricks = 0;
        for (int64_t v : order) {
            if (lvl[v] < M)
                id[v] = (int32_t)n_top++;
            else if (lvl[v] == M)
                id[v] = (int32_t)n_bricks++;
        }
        const uint64_t words = (uint64_t)n_top * 8 + (uint64_t)n_bricks * 512;
        if (words * 4 >= (1ull << 32) - 256 || n_top + n_bricks >= (1ll << 31))
            return fail(PO_ERR_UNSUPPORTED, "traversal index of %llu bytes exceeds 4 GiB",
                        (unsigned long long)(words * 4));
        index.assign((size_t)words, 0);
        // a brick entry: (leaf + 1) << 2 | (D - level) of the leaf holding the cell
        auto enc = [](int32_t entry, int up) {
            return (int32_t)((uint32_t)(entry < 0 ? -entry : 0) << 2 | (uint32_t)up);
        };
        for (int64_t v : order) {
            if (lvl[v] < M) {
                int32_t* out = &index[(size_t)id[v] * 8];
                for (int c = 0; c < 8; ++c) {
                    const int32_t ch = h[(size_t)v * 8 + c];
                    out[c] = ch <= 0 ? ch : (lvl[ch] < M ? id[ch] : (int32_t)(n_top + id[ch]));
                }
            } else if (lvl[v] == M) {
                int32_t* B = &index[(size_t)n_top * 8 + (size_t)id[v] * 512];
                for (int s1 = 0; s1 < 8; ++s1) {
                    const int32_t e1 = h[(size_t)v * 8 + s1];
                    if (e1 <= 0) {
                        for (int q = 0; q < 64; ++q) B[s1 * 64 + q] = enc(e1, 2);
                        continue;
                    }
                    for (int s2 = 0; s2 < 8; ++s2) {
                        const int32_t e2 = h[(size_t)e1 * 8 + s2];
                        if (e2 <= 0) {
                            for (int q = 0; q < 8; ++q) B[s1 * 64 + s2 * 8 + q] = enc(e2, 1);
                            continue;
                        }
                        // children of a level D-1 node are leaves or empty (validated)
                        for (int s3 = 0; s3 < 8; ++s3) B[s1 * 64 + s2 * 8 + s3] = enc(h[(size_t)e2 * 8 + s3], 0);
                    }
                }
            }
        }
    } catch (const std::bad_alloc&) {
        return fail(PO_ERR_OOM, "traversal index: host allocation");
    }
    return ok();
}

po_status po_tree_index_host(const po_tree_desc* desc, int64_t n_nodes, const int32_t* h_child, int64_t n_leaves,
                             int64_t* n_top, int64_t* n_bricks, int32_t* h_index) {
    if (po_status s = check_desc(desc)) return s;
    if (!n_top || !n_bricks) return fail(PO_ERR_INVALID, "n_top or n_bricks is NULL");
    if (desc->depth < 4) return fail(PO_ERR_INVALID, "trees of depth %d < 4 have no traversal index", desc->depth);
    std::vector<int32_t> index;
    int64_t nt = 0, nb = 0;
    if (po_status s = index_of(desc, false, n_nodes, h_child, n_leaves, index, nt, nb)) return s;
    *n_top = nt;
    *n_bricks = nb;
    if (h_index) std::memcpy(h_index, index.data(), index.size() * sizeof(int32_t));
    return ok();
}

po_status po_tree_build_index(po_tree* t, void* stream) {
    if (!t) return fail(PO_ERR_INVALID, "tree is NULL");
    const int D = t->desc.depth;
    if (t->d_index || D < 4) return ok();  // built already, or too shallow for 8x8x8 bricks
    const int64_t n = t->n_nodes;
    hipStream_t s = (hipStream_t)stream;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return device_fail(e, "traversal index: current device");
    std::vector<int32_t> h, index;
    int64_t n_top = 0, n_bricks = 0;
    try {
        h.resize((size_t)n * 8);
    } catch (const std::bad_alloc&) {
        return fail(PO_ERR_OOM, "traversal index: host allocation");
    }
    e = hipMemcpyAsync(h.data(), t->child, (size_t)n * 32, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_fail(e, "traversal index: reading the child array");
    if (po_status st = index_of(&t->desc, t->codebook, n, h.data(), t->n_leaves, index, n_top, n_bricks)) return st;
    const size_t bytes = index.size() * sizeof(int32_t);
    void* d = nullptr;
    if ((e = hipMalloc(&d, bytes)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(PO_ERR_OOM, "traversal index: %zu bytes of device memory", bytes);
    }
    e = hipMemcpyAsync(d, index.data(), bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return device_fail(e, "traversal index: upload");
    }
    t->d_index = d;
    t->index_device = dev;
    t->n_bricks = n_bricks;
    t->kt.child = static_cast<const int32_t*>(d);
    t->kt.n_top = (int32_t)n_top;
    t->kt.brick_level = (int16_t)(D - 3);
    t->kt.index_bytes = (uint32_t)bytes;
    return ok();
}

po_status po_tree_destroy(po_tree* t) {
    if (t && t->d_index) {
        // the index may still be read by queued work: wait for its device
        int cur = 0;
        const bool have_cur = hipGetDevice(&cur) == hipSuccess;
        hipError_t e = hipSetDevice(t->index_device);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e == hipSuccess) e = hipFree(t->d_index);
        if (have_cur) (void)hipSetDevice(cur);
        delete t;
        if (e != hipSuccess) return device_fail(e, "freeing the traversal index");
        return ok();
    }
    delete t;
    return ok();
}

po_status po_render_rays(const po_tree* t, int64_t n, const float* d_origins, const float* d_dirs,
                         const po_render_opts* opts, float* d_rgb, float* d_aux, void* stream) {
    if (!t) return fail(PO_ERR_INVALID, "tree is NULL");
    if (po_status s = check_opts(opts)) return s;
    if (n < 0) return fail(PO_ERR_INVALID, "n = %lld < 0", (long long)n);
    if (n == 0) return ok();
    if (n > (1ll << 40)) return fail(PO_ERR_INVALID, "n = %lld too large", (long long)n);
    if (!d_origins || !d_dirs || !d_rgb) return fail(PO_ERR_INVALID, "ray or output array is NULL");
    if ((opts->flags & PO_OUT_AUX) && !d_aux) return fail(PO_ERR_INVALID, "PO_OUT_AUX set but aux is NULL");
    float* aux = (opts->flags & PO_OUT_AUX) ? d_aux : nullptr;
    if (t->codebook && po_view_opts(kopts(t, opts), aux))
        return fail(PO_ERR_UNSUPPORTED, "codebook trees render without aux outputs, sh_off or a slicing plane");
    const KOpts k = kopts(t, opts);
    const int variant = po_fwd_variant(k, aux, t->kt);
    KSplit S;
    hipError_t e;
    if (!(k.flags & PO_ONE_PASS) && n >= kSplitMinRays && n < (1ll << 31) && k.max_steps > PO_SPLIT_STEPS &&
        split_queue(stream, &S))
        e = po_launch_rays_split(t, n, d_origins, d_dirs, k, d_rgb, variant == PO_FWD_VIEW ? aux : nullptr, S,
                                 (hipStream_t)stream);
    else
        e = po_launch_rays(t, n, d_origins, d_dirs, k, d_rgb, aux, (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "render_rays launch");
    return ok();
}

// po_render_camera and po_render_camera_noalloc: the same render, with the
// per-stream queue (allocated on first use) or the fixed per-device one.
static po_status render_camera_impl(const po_tree* t, const po_camera* cam, const po_render_opts* opts,
                                    float* d_rgb, float* d_aux, void* stream, bool noalloc) {
    if (!t) return fail(PO_ERR_INVALID, "tree is NULL");
    if (po_status s = check_camera(cam)) return s;
    if (po_status s = check_opts(opts)) return s;
    if (noalloc && (int64_t)cam->width * cam->height > kNoAllocMaxPixels)
        return fail(PO_ERR_INVALID,
                    "po_render_camera_noalloc: %d x %d = %lld pixels exceeds the %lld its fixed queue is sized for; "
                    "use po_render_camera",
                    cam->width, cam->height, (long long)cam->width * cam->height, (long long)kNoAllocMaxPixels);
    if (!d_rgb) return fail(PO_ERR_INVALID, "output image is NULL");
    if ((opts->flags & PO_OUT_AUX) && !d_aux) return fail(PO_ERR_INVALID, "PO_OUT_AUX set but aux is NULL");
    KJob j;
    std::memset(&j, 0, sizeof j);
    j.tr = t->kt;
    j.cam = kcam(cam);
    j.op = kopts(t, opts);
    j.rgb = d_rgb;
    j.aux = (opts->flags & PO_OUT_AUX) ? d_aux : nullptr;
    if (t->codebook && po_view_opts(j.op, j.aux))
        return fail(PO_ERR_UNSUPPORTED, "codebook trees render without aux outputs, sh_off or a slicing plane");
    j.tile_begin = 0;
    j.block_begin = 0;
    j.tiles_x = (cam->width + PO_TILE - 1) / PO_TILE;
    const int variant = po_fwd_variant(j.op, j.aux, t->kt);
    KSplit S;
    hipError_t e;
    const bool split = !(j.op.flags & PO_ONE_PASS) && (int64_t)cam->width * cam->height >= kSplitMinPixels &&
                       j.op.max_steps > PO_SPLIT_STEPS;
    if (split && noalloc) {
        if ((e = po_noalloc_queue(&S)) != hipSuccess) return device_fail(e, "locating the fixed work queue");
        S.split_steps = po_camera_split_steps(4 * (int64_t)tiles_of(cam));
        e = po_launch_camera_split(t, j, 4 * tiles_of(cam), variant, S, (hipStream_t)stream);
    } else if (split && split_queue(stream, &S)) {
        S.split_steps = po_camera_split_steps(4 * (int64_t)tiles_of(cam));
        e = po_launch_camera_split(t, j, 4 * tiles_of(cam), variant, S, (hipStream_t)stream);
    } else {
        e = po_launch_camera_jobs(t, 1, &j, 4 * tiles_of(cam), variant, (hipStream_t)stream);
    }
    if (e != hipSuccess) return device_fail(e, "render_camera launch");
    return ok();
}

po_status po_render_camera(const po_tree* t, const po_camera* cam, const po_render_opts* opts, float* d_rgb,
                           float* d_aux, void* stream) {
    return render_camera_impl(t, cam, opts, d_rgb, d_aux, stream, false);
}

po_status po_render_camera_noalloc(const po_tree* t, const po_camera* cam, const po_render_opts* opts,
                                   float* d_rgb, float* d_aux, void* stream) {
    return render_camera_impl(t, cam, opts, d_rgb, d_aux, stream, true);
}

po_status po_render_rays_backward(const po_tree* t, int64_t n, const float* d_origins, const float* d_dirs,
                                  const po_render_opts* opts, const float* d_rgb_fwd, const float* d_grad_rgb,
                                  float* d_grad_sigma, float* d_grad_sh, void* stream) {
    if (!t) return fail(PO_ERR_INVALID, "tree is NULL");
    if (po_status s = check_opts(opts)) return s;
    if (t->desc.dtype != PO_F32) return fail(PO_ERR_UNSUPPORTED, "gradients need float32 leaves");
    if (po_view_opts(kopts(t, opts), nullptr))
        return fail(PO_ERR_UNSUPPORTED, "gradients of renders with sh_off or a slicing plane are not provided");
    if (n < 0) return fail(PO_ERR_INVALID, "n = %lld < 0", (long long)n);
    if (n == 0) return ok();
    if (n > (1ll << 40)) return fail(PO_ERR_INVALID, "n = %lld too large", (long long)n);
    if (!d_origins || !d_dirs || !d_rgb_fwd || !d_grad_rgb || !d_grad_sigma || !d_grad_sh)
        return fail(PO_ERR_INVALID, "NULL array");
    const KOpts k = kopts(t, opts);
    KSplit S;
    hipError_t e;
    if (!(k.flags & PO_ONE_PASS) && n >= kSplitMinBackward && n < (1ll << 31) && k.max_steps > PO_SPLIT_STEPS &&
        split_queue(stream, &S))
        e = po_launch_backward_split(t, n, d_origins, d_dirs, k, d_rgb_fwd, d_grad_rgb, d_grad_sigma, d_grad_sh, S,
                                     (hipStream_t)stream);
    else
        e = po_launch_backward(t, n, d_origins, d_dirs, k, d_rgb_fwd, d_grad_rgb, d_grad_sigma, d_grad_sh,
                               (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "backward launch");
    return ok();
}

po_status po_render_rays_keep(const po_tree* t, int64_t n, const float* d_origins, const float* d_dirs,
                              const po_render_opts* opts, float* d_rgb, int32_t* d_ray_slot, void* stream) {
    if (!t) return fail(PO_ERR_INVALID, "tree is NULL");
    if (po_status s = check_opts(opts)) return s;
    if (t->desc.dtype != PO_F32) return fail(PO_ERR_UNSUPPORTED, "a kept render is for gradients, which need float32 leaves");
    if (opts->flags & PO_OUT_AUX) return fail(PO_ERR_UNSUPPORTED, "a kept render writes no aux outputs");
    if (po_view_opts(kopts(t, opts), nullptr))
        return fail(PO_ERR_UNSUPPORTED, "gradients of renders with sh_off or a slicing plane are not provided");
    if (n < 0 || n > (1ll << 40)) return fail(PO_ERR_INVALID, "n = %lld out of range", (long long)n);
    if (n == 0) return ok();
    if (!d_origins || !d_dirs || !d_rgb || !d_ray_slot) return fail(PO_ERR_INVALID, "NULL array");
    int dev = 0;
    if (hipError_t e = hipGetDevice(&dev)) return device_fail(e, "hipGetDevice");
    const KOpts k = kopts(t, opts);
    KSplit S;
    bool split = !(k.flags & PO_ONE_PASS) && n >= kSplitMinRays && n < (1ll << 31) && k.max_steps > PO_SPLIT_STEPS &&
                 split_queue(stream, &S);
    hipError_t e;
    if (split) {
        S.ray_slot = d_ray_slot;
        e = po_launch_rays_split(t, n, d_origins, d_dirs, k, d_rgb, nullptr, S, (hipStream_t)stream);
    } else {
        e = po_launch_rays(t, n, d_origins, d_dirs, k, d_rgb, nullptr, (hipStream_t)stream);
    }
    if (e != hipSuccess) return device_fail(e, "render_rays_keep launch");
    std::lock_guard<std::mutex> lk(g_split_mu);
    Kept& kp = g_kept[{dev, stream}];
    kp.valid = true;
    kp.split = split;
    kp.t = t;
    kp.n = n;
    kp.o = d_origins;
    kp.d = d_dirs;
    kp.slot = d_ray_slot;
    kp.opts = *opts;
    return ok();
}

po_status po_render_rays_backward_kept(const po_tree* t, int64_t n, const float* d_origins, const float* d_dirs,
                                       const po_render_opts* opts, const float* d_rgb_fwd, const float* d_grad_rgb,
                                       float* d_grad_sigma, float* d_grad_sh, const int32_t* d_ray_slot,
                                       void* stream) {
    if (!t) return fail(PO_ERR_INVALID, "tree is NULL");
    if (po_status s = check_opts(opts)) return s;
    if (t->desc.dtype != PO_F32) return fail(PO_ERR_UNSUPPORTED, "gradients need float32 leaves");
    if (n < 0 || n > (1ll << 40)) return fail(PO_ERR_INVALID, "n = %lld out of range", (long long)n);
    if (n == 0) return ok();
    if (!d_origins || !d_dirs || !d_rgb_fwd || !d_grad_rgb || !d_grad_sigma || !d_grad_sh || !d_ray_slot)
        return fail(PO_ERR_INVALID, "NULL array");
    int dev = 0;
    if (hipError_t e = hipGetDevice(&dev)) return device_fail(e, "hipGetDevice");
    Kept kp;
    void* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_split_mu);
        auto it = g_kept.find({dev, stream});
        if (it == g_kept.end() || !it->second.valid || it->second.t != t || it->second.n != n ||
            it->second.o != d_origins || it->second.d != d_dirs || it->second.slot != d_ray_slot ||
            std::memcmp(&it->second.opts, opts, sizeof *opts) != 0)
            return fail(PO_ERR_INVALID,
                        "no kept render of these rays is pending on this stream: po_render_rays_keep must be the last "
                        "split work on the stream's queue, with the same tree, n, arrays, ray_slot and options");
        kp = it->second;
        it->second.valid = false;  // the prefix pass overwrites the pieces' results
        if (kp.split) {
            auto q = g_split.find({dev, stream});
            if (q == g_split.end()) return fail(PO_ERR_INVALID, "the kept render's queue was released");
            base = q->second;
        }
    }
    const KOpts k = kopts(t, opts);
    hipError_t e;
    if (kp.split) {
        KSplit S;
        po_split_layout(base, kSplitRegionSlots, &S);
        S.ray_slot = const_cast<int32_t*>(d_ray_slot);
        e = po_launch_backward_kept(t, n, d_origins, d_dirs, k, d_rgb_fwd, d_grad_rgb, d_grad_sigma, d_grad_sh, S,
                                    (hipStream_t)stream);
    } else {
        e = po_launch_backward(t, n, d_origins, d_dirs, k, d_rgb_fwd, d_grad_rgb, d_grad_sigma, d_grad_sh,
                               (hipStream_t)stream);
    }
    if (e != hipSuccess) return device_fail(e, "backward_kept launch");
    return ok();
}

po_status po_camera_rays(const po_camera* cam, float* d_origins, float* d_dirs, void* stream) {
    if (po_status s = check_camera(cam)) return s;
    if (!d_origins || !d_dirs) return fail(PO_ERR_INVALID, "NULL array");
    hipError_t e = po_launch_camera_rays(kcam(cam), d_origins, d_dirs, (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "camera_rays launch");
    return ok();
}

po_status po_mse_grad(int64_t n, const float* d_rgb, const float* d_target, float scale, float* d_grad_rgb,
                      float* d_sq_sum, void* stream) {
    if (n < 0 || n > (1ll << 40)) return fail(PO_ERR_INVALID, "n = %lld out of range", (long long)n);
    if (!finite(scale)) return fail(PO_ERR_INVALID, "scale must be finite");
    if (n == 0) return ok();
    if (!d_rgb || !d_target || !d_grad_rgb || !d_sq_sum) return fail(PO_ERR_INVALID, "NULL array");
    hipError_t e = po_launch_mse_grad(n, d_rgb, d_target, scale, d_grad_rgb, d_sq_sum, (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "mse_grad launch");
    return ok();
}

po_status po_sgd_step(int64_t n, float* d_param, float* d_grad, float lr, int32_t zero_grad, void* stream) {
    if (n < 0 || n > (1ll << 40)) return fail(PO_ERR_INVALID, "n = %lld out of range", (long long)n);
    if (!finite(lr)) return fail(PO_ERR_INVALID, "lr must be finite");
    if (n == 0) return ok();
    if (!d_param || !d_grad) return fail(PO_ERR_INVALID, "NULL array");
    hipError_t e = po_launch_sgd(n, d_param, d_grad, lr, zero_grad != 0, (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "sgd launch");
    return ok();
}

po_status po_gather_rays(int64_t n, const int64_t* d_idx, int64_t n_src, const float* d_o, const float* d_d,
                         const float* d_t, float* d_bo, float* d_bd, float* d_bt, void* stream) {
    if (n < 0 || n >= (1ll << 40)) return fail(PO_ERR_INVALID, "n = %lld out of range", (long long)n);
    if (n_src < 1 || n_src >= (1ll << 40)) return fail(PO_ERR_INVALID, "n_src = %lld out of range", (long long)n_src);
    if (n == 0) return ok();
    if (!d_idx || !d_o || !d_d || !d_t || !d_bo || !d_bd || !d_bt) return fail(PO_ERR_INVALID, "NULL array");
    hipError_t e = po_launch_gather_rays(n, d_idx, n_src, d_o, d_d, d_t, d_bo, d_bd, d_bt, (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "gather_rays launch");
    return ok();
}

po_status po_draw_batch(int64_t n, uint64_t seed, uint64_t first, int64_t n_src, const float* d_o, const float* d_d,
                        const float* d_t, float* d_bo, float* d_bd, float* d_bt, float* d_sq_sum, void* stream) {
    if (n < 0 || n >= (1ll << 31)) return fail(PO_ERR_INVALID, "n = %lld out of range", (long long)n);
    if (n_src < 1 || n_src >= (1ll << 40)) return fail(PO_ERR_INVALID, "n_src = %lld out of range", (long long)n_src);
    if (n == 0) return ok();
    if (!d_o || !d_d || !d_t || !d_bo || !d_bd || !d_bt) return fail(PO_ERR_INVALID, "NULL array");
    hipError_t e = po_launch_draw_batch(n, seed, first, n_src, d_o, d_d, d_t, d_bo, d_bd, d_bt, d_sq_sum,
                                        (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "draw_batch launch");
    return ok();
}

po_status po_camera_tiles(const po_camera* cam, int32_t* n_tiles) {
    if (po_status s = check_camera(cam)) return s;
    if (!n_tiles) return fail(PO_ERR_INVALID, "n_tiles is NULL");
    *n_tiles = tiles_of(cam);
    return ok();
}

po_status po_render_batch(int32_t n_jobs, const po_job* jobs, void* stream) {
    if (n_jobs < 0 || n_jobs > PO_BATCH_MAX_JOBS)
        return fail(PO_ERR_INVALID, "n_jobs %d outside [0, %d]", n_jobs, PO_BATCH_MAX_JOBS);
    if (n_jobs == 0) return ok();
    if (!jobs) return fail(PO_ERR_INVALID, "jobs is NULL");
    for (int i = 0; i < n_jobs; ++i) {
        const po_job& J = jobs[i];
        if (!J.tree) return fail(PO_ERR_INVALID, "job %d: tree is NULL", i);
        if (po_status s = check_camera(&J.cam)) return fail(s, "job %d: %s", i, g_err.c_str());
        if (po_status s = check_opts(&J.opts)) return fail(s, "job %d: %s", i, g_err.c_str());
        if (!J.d_rgb) return fail(PO_ERR_INVALID, "job %d: output image is NULL", i);
        if ((J.opts.flags & PO_OUT_AUX) && !J.d_aux) return fail(PO_ERR_INVALID, "job %d: PO_OUT_AUX set but aux is NULL", i);
        if (J.tree->codebook && po_view_opts(kopts(J.tree, &J.opts), (J.opts.flags & PO_OUT_AUX) ? J.d_aux : nullptr))
            return fail(PO_ERR_UNSUPPORTED, "job %d: codebook trees render without aux outputs, sh_off or a slicing plane", i);
        if (J.tile_begin < 0 || J.tile_end < J.tile_begin || J.tile_end > tiles_of(&J.cam))
            return fail(PO_ERR_INVALID, "job %d: tile range [%d, %d) outside [0, %d]", i, J.tile_begin, J.tile_end,
                        tiles_of(&J.cam));
    }
    // group jobs by kernel variant, one launch per group, in order of first appearance
    auto variant = [&](int q) {
        const po_job& J = jobs[q];
        const float* aux = (J.opts.flags & PO_OUT_AUX) ? J.d_aux : nullptr;
        return 4 * po_plan_id(J.tree) + po_fwd_variant(kopts(J.tree, &J.opts), aux, J.tree->kt);
    };
    bool done[PO_BATCH_MAX_JOBS] = {false};
    // jobs of at least kSplitMinPixels pixels (whole tiles) are rendered in
    // pieces, each on its own, as po_render_camera renders a large image
    for (int i = 0; i < n_jobs; ++i) {
        const po_job& J = jobs[i];
        const int nt = J.tile_end - J.tile_begin;
        const KOpts k = kopts(J.tree, &J.opts);
        KSplit S;
        if ((k.flags & PO_ONE_PASS) || (int64_t)nt * PO_TILE * PO_TILE < kSplitMinPixels ||
            k.max_steps <= PO_SPLIT_STEPS || !split_queue(stream, &S))
            continue;
        done[i] = true;
        KJob kj;
        std::memset(&kj, 0, sizeof kj);
        kj.tr = J.tree->kt;
        kj.cam = kcam(&J.cam);
        kj.op = k;
        kj.rgb = J.d_rgb;
        kj.aux = (J.opts.flags & PO_OUT_AUX) ? J.d_aux : nullptr;
        kj.tile_begin = J.tile_begin;
        kj.block_begin = 0;
        kj.tiles_x = (J.cam.width + PO_TILE - 1) / PO_TILE;
        S.split_steps = po_camera_split_steps(4 * (int64_t)nt);
        hipError_t e = po_launch_camera_split(J.tree, kj, 4 * nt, variant(i) % 4, S, (hipStream_t)stream);
        if (e != hipSuccess) return device_fail(e, "render_batch launch");
    }
    for (int i = 0; i < n_jobs; ++i) {
        if (done[i]) continue;
        const int plan = variant(i);
        KJob kj[PO_BATCH_MAX_JOBS];
        int nj = 0, blocks = 0;
        for (int q = i; q < n_jobs; ++q) {
            if (done[q] || variant(q) != plan) continue;
            done[q] = true;
            const po_job& J = jobs[q];
            const int nt = J.tile_end - J.tile_begin;
            if (nt == 0) continue;
            KJob& k = kj[nj++];
            std::memset(&k, 0, sizeof k);
            k.tr = J.tree->kt;
            k.cam = kcam(&J.cam);
            k.op = kopts(J.tree, &J.opts);
            k.rgb = J.d_rgb;
            k.aux = (J.opts.flags & PO_OUT_AUX) ? J.d_aux : nullptr;
            k.tile_begin = J.tile_begin;
            k.block_begin = blocks;
            k.tiles_x = (J.cam.width + PO_TILE - 1) / PO_TILE;
            blocks += 4 * nt;
        }
        if (nj == 0) continue;
        hipError_t e = po_launch_camera_jobs(jobs[i].tree, nj, kj, blocks, plan % 4, (hipStream_t)stream);
        if (e != hipSuccess) return device_fail(e, "render_batch launch");
    }
    return ok();
}

po_status po_leaf_weights(const po_tree* t, const po_camera* cam, const po_render_opts* opts, int32_t mode,
                          float* d_weight, float* d_alpha, void* stream) {
    if (!t) return fail(PO_ERR_INVALID, "tree is NULL");
    if (po_status s = check_camera(cam)) return s;
    if (po_status s = check_opts(opts)) return s;
    if (mode != PO_WEIGHT_ALPHA && mode != PO_WEIGHT_CONTRIB) return fail(PO_ERR_INVALID, "unknown weight mode %d", mode);
    if (opts->flags != 0) return fail(PO_ERR_INVALID, "filter renders take no output flags");
    const KOpts k = kopts(t, opts);
    if (po_view_opts(k, nullptr))
        return fail(PO_ERR_UNSUPPORTED, "filter renders take no sh_off or slicing plane");
    if (!d_weight && t->n_leaves > 0) return fail(PO_ERR_INVALID, "weight array is NULL");
    hipError_t e = po_launch_leaf_weights(t, kcam(cam), k, mode, d_weight, d_alpha, (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "leaf_weights launch");
    return ok();
}

namespace {
po_status traversal_stats(const po_tree* t, const po_camera* cam, int64_t n, const float* d_o, const float* d_d,
                          const po_render_opts* opts, int64_t* h_stats, void* stream) {
    if (!h_stats) return fail(PO_ERR_INVALID, "stats array is NULL");
    if (opts->flags != 0) return fail(PO_ERR_INVALID, "statistics take no output flags");
    const KOpts k = kopts(t, opts);
    if (po_view_opts(k, nullptr)) return fail(PO_ERR_UNSUPPORTED, "statistics take no sh_off or slicing plane");
    unsigned long long v[4] = {0, 0, 0, 0};
    hipError_t e = hipSuccess;
    if (cam || n > 0) {
        static std::mutex mu;
        std::lock_guard<std::mutex> lk(mu);
        KCam kc;
        if (cam) kc = kcam(cam);
        e = po_traversal_stats_sync(t, cam ? &kc : nullptr, n, d_o, d_d, k, v, (hipStream_t)stream);
    }
    if (e != hipSuccess) return device_fail(e, "traversal_stats");
    for (int i = 0; i < 4; ++i) h_stats[i] = (int64_t)v[i];
    return ok();
}
}  // namespace

po_status po_traversal_stats(const po_tree* t, const po_camera* cam, const po_render_opts* opts, int64_t* h_stats,
                             void* stream) {
    if (!t) return fail(PO_ERR_INVALID, "tree is NULL");
    if (po_status s = check_camera(cam)) return s;
    if (po_status s = check_opts(opts)) return s;
    return traversal_stats(t, cam, 0, nullptr, nullptr, opts, h_stats, stream);
}

po_status po_traversal_stats_rays(const po_tree* t, int64_t n, const float* d_origins, const float* d_dirs,
                                  const po_render_opts* opts, int64_t* h_stats, void* stream) {
    if (!t) return fail(PO_ERR_INVALID, "tree is NULL");
    if (po_status s = check_opts(opts)) return s;
    if (n < 0 || n >= (1ll << 37)) return fail(PO_ERR_INVALID, "n = %lld out of range", (long long)n);
    if (n > 0 && (!d_origins || !d_dirs)) return fail(PO_ERR_INVALID, "ray array is NULL");
    return traversal_stats(t, nullptr, n, d_origins, d_dirs, opts, h_stats, stream);
}

po_status po_reserve_queues(void* stream) {
    KSplit S;
    if (!split_queue(stream, &S))
        return fail(PO_ERR_DEVICE, "could not allocate the split-render work queue (%zu bytes)",
                    po_split_bytes(kSplitRegionSlots));
    return ok();
}

po_status po_release_queues(void) {
    std::lock_guard<std::mutex> lk(g_split_mu);
    if (g_split.empty()) return ok();
    hipError_t first = hipSuccess;
    int cur = 0;
    const bool have_cur = hipGetDevice(&cur) == hipSuccess;
    for (auto& kv : g_split) {
        hipError_t e = hipSetDevice(kv.first.first);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e == hipSuccess) e = hipFree(kv.second);
        if (e != hipSuccess && first == hipSuccess) first = e;
    }
    g_split.clear();
    g_kept.clear();
    if (have_cur) (void)hipSetDevice(cur);
    if (first != hipSuccess) return device_fail(first, "releasing the split-render queues");
    return ok();
}

po_status po_device_errors(int64_t* count) {
    if (!count) return fail(PO_ERR_INVALID, "count is NULL");
    unsigned long long v = 0;
    hipError_t e = po_read_device_errors(&v);
    if (e != hipSuccess) return device_fail(e, "reading the device error counter");
    *count = (int64_t)v;
    return ok();
}

po_status po_device_errors_reset(void) {
    hipError_t e = po_reset_device_errors();
    if (e != hipSuccess) return device_fail(e, "resetting the device error counter");
    return ok();
}

}  // extern "C"
