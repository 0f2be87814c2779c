// HIP kernels of libplenoctree for gfx950 (MI355X).
//
// One ray per lane.  A ray is cut into the exact segments between voxel
// boundaries of the sparse octree (Sec. 4.2, "Rendering"): the current
// position is kept as integer coordinates of a finest-level cell; each step
// descends from the root to the leaf containing it, computes the parameter at
// which the ray leaves that leaf's cube (the nearest exit plane), composites
// the segment if the leaf holds data, and moves the coordinates across the
// exit face.  Large empty cubes are therefore crossed in one step.  Each data
// segment is shaded with the sigmoid of the real-SH expansion in the ray
// direction (Sec. 4.1; SH of App. B.1) and composited front to back with
// alpha = 1 - exp(-sigma delta) (Sec. 3, eqn:quad); marching stops once the
// transmittance falls below the threshold (Sec. 4.2) and the background
// takes the remaining transmittance (App. B.3).
//
// The backward kernel replays the identical segment sequence and applies the
// analytic derivatives of App. B.3 with the prefix scheme of its Remark.
//
// Ray geometry (crossing parameters, positions) is evaluated in FP64, leaf
// values, SH and compositing in FP32.  The library is compiled with
// -ffp-contract=off: every fused multiply-add is written out, so the forward
// and backward kernels take bit-identical steps.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <type_traits>

#include "po_internal.h"

// The library is built from this file compiled once per part (PO_PART = 0 ..
// PO_PARTS - 1), in parallel: each part instantiates the kernels of some of
// the launchers below.  Device variables are per part, so each part keeps its
// own error counter and part 0 sums them.
#ifndef PO_PART
#error "compile with -DPO_PART=<n>, 0 <= n < PO_PARTS"
#endif
#define PO_PARTS 8

namespace {
// malformed child entries and step-cap hits met by this part's kernels
__device__ unsigned long long g_po_errors = 0;
#if PO_PART == 0
// sums of po_traversal_stats: rays, samples, cells, child-entry loads
__device__ unsigned long long g_po_stats[4];
// Work queue of po_render_camera_noalloc: a file-scope device array (one
// copy per GPU the library runs on, held until the process ends).  Host code
// never passes this name to a kernel: it is a host-side stand-in there, and
// po_noalloc_queue looks up each device's own address of the array.
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];
#endif

// One wave64 per workgroup: rays finish unevenly, and single-wave workgroups
// let the dispatcher refill a SIMD as soon as any wave retires, which
// shortens the tail of a launch.
constexpr int kBlock = 64;

// ---------------------------------------------------------------------------
// Real SH basis up to degree 4 at a unit direction (App. B.1), written as
// polynomials in x, y, z.  Index l*l + l + m.  Sign convention: P_l^m carries
// the Condon-Shortley phase, which cancels the (-1)^m of the real
// combination, so every coefficient below is positive.
// ---------------------------------------------------------------------------
template <int K>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float (&Y)[K]) {
    Y[0] = 0.28209479177387814f;  // 1/(2 sqrt(pi))
    if constexpr (K > 1) {
        Y[1] = 0.4886025119029199f * y;  // sqrt(3/(4 pi))
        Y[2] = 0.4886025119029199f * z;
        Y[3] = 0.4886025119029199f * x;
    }
    if constexpr (K > 4) {
        const float xx = x * x, yy = y * y, zz = z * z;
        Y[4] = 1.0925484305920792f * (x * y);              // sqrt(15/pi)/2
        Y[5] = 1.0925484305920792f * (y * z);
        Y[6] = 0.31539156525252005f * (3.0f * zz - 1.0f);  // sqrt(5/pi)/4
        Y[7] = 1.0925484305920792f * (x * z);
        Y[8] = 0.5462742152960396f * (xx - yy);            // sqrt(15/pi)/4
        if constexpr (K > 9) {
            Y[9] = 0.5900435899266435f * (y * (3.0f * xx - yy));   // sqrt(35/(2 pi))/4
            Y[10] = 2.890611442640554f * (x * y * z);              // sqrt(105/pi)/2
            Y[11] = 0.4570457994644658f * (y * (5.0f * zz - 1.0f)); // sqrt(21/(2 pi))/4
            Y[12] = 0.3731763325901154f * (z * (5.0f * zz - 3.0f)); // sqrt(7/pi)/4
            Y[13] = 0.4570457994644658f * (x * (5.0f * zz - 1.0f));
            Y[14] = 1.445305721320277f * (z * (xx - yy));           // sqrt(105/pi)/4
            Y[15] = 0.5900435899266435f * (x * (xx - 3.0f * yy));
            if constexpr (K > 16) {
                const float z7a = 7.0f * zz - 1.0f, z7b = 7.0f * zz - 3.0f;
                Y[16] = 2.5033429417967046f * (x * y * (xx - yy));          // 3 sqrt(35/pi)/4
                Y[17] = 1.7701307697799304f * (y * z * (3.0f * xx - yy));   // 3 sqrt(35/(2 pi))/4
                Y[18] = 0.9461746957575601f * (x * y * z7a);                // 3 sqrt(5/pi)/4
                Y[19] = 0.6690465435572892f * (y * z * z7b);                // 3 sqrt(5/(2 pi))/4
                Y[20] = 0.10578554691520431f * ((35.0f * zz - 30.0f) * zz + 3.0f);  // 3/(16 sqrt(pi))
                Y[21] = 0.6690465435572892f * (x * z * z7b);
                Y[22] = 0.47308734787878004f * ((xx - yy) * z7a);           // 3 sqrt(5/pi)/8
                Y[23] = 1.7701307697799304f * (x * z * (xx - 3.0f * yy));
                Y[24] = 0.6258357354491761f * (xx * (xx - 3.0f * yy) - yy * (3.0f * xx - yy));  // 3 sqrt(35/pi)/16
            }
        }
    }
}

// Spherical-Gaussian basis (App. B.1): G_j(d) = exp(lambda_j (d . p_j - 1))
// for the tree's K lobes (axis p_j, normalised here, and bandwidth lambda_j),
// in place of the SH of the same index.  The lobes are uniform across the
// wave and read once per ray.
template <int K>
__device__ __forceinline__ void sg_basis(const float* __restrict__ lobes, float x, float y, float z,
                                         float (&Y)[K]) {
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const float px = lobes[4 * j], py = lobes[4 * j + 1], pz = lobes[4 * j + 2], lam = lobes[4 * j + 3];
        const float c = (x * px + y * py + z * pz) * rsqrtf(px * px + py * py + pz * pz);
        Y[j] = __expf(lam * (c - 1.0f));
    }
}

// Colour basis of a tree at the unit direction (x, y, z).
template <int K>
__device__ __forceinline__ void colour_basis(const KTree& tr, float x, float y, float z, float (&Y)[K]) {
    if (tr.lobes)
        sg_basis<K>(tr.lobes, x, y, z, Y);
    else
        sh_basis<K>(x, y, z, Y);
}

// Buffer resource for raw (byte-addressed) loads from one array: loads at
// offsets outside [0, bytes) return 0 instead of faulting (gfx9 descriptor
// word 3 = 0x00020000: raw buffer, 32-bit data format).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

// ---------------------------------------------------------------------------
// Leaf record access.  T is float or __half; values are widened to float.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float load_sigma(const float* p, int i) { return p[i]; }
__device__ __forceinline__ float load_sigma(const __half* p, int i) { return __half2float(p[i]); }

// Number of 32-bit words holding NL elements of type T.
template <typename T, int NL>
struct Words {
    static constexpr int NB = NL * (int)sizeof(T);
    static constexpr int N = (NB + 3) / 4;
};

// Loads NL elements of one SH record at `base` as raw 32-bit words using
// VEC-byte loads (16, 8 or 4; `base` is VEC-aligned), then dword loads and,
// for an odd number of halves, one 2-byte load.  The host guarantees the NL
// elements lie inside the record (NL <= stride).  The loads are only issued
// here; the words are consumed later, so their latency can overlap other work.
template <typename T, int NL, int VEC>
__device__ __forceinline__ void load_words(const char* __restrict__ base, uint32_t (&w)[Words<T, NL>::N]) {
    constexpr int NB = Words<T, NL>::NB;
    constexpr int NV = NB / VEC;
    constexpr int DONE = NV * VEC / 4;
    constexpr int FULLW = NB / 4;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        if constexpr (VEC == 16) {
            const uint4 q = *reinterpret_cast<const uint4*>(base + 16 * v);
            w[4 * v + 0] = q.x;
            w[4 * v + 1] = q.y;
            w[4 * v + 2] = q.z;
            w[4 * v + 3] = q.w;
        } else if constexpr (VEC == 8) {
            const uint2 q = *reinterpret_cast<const uint2*>(base + 8 * v);
            w[2 * v + 0] = q.x;
            w[2 * v + 1] = q.y;
        } else {
            w[v] = *reinterpret_cast<const uint32_t*>(base + 4 * v);
        }
    }
#pragma unroll
    for (int i = DONE; i < FULLW; ++i) w[i] = *reinterpret_cast<const uint32_t*>(base + 4 * i);
    if constexpr (NB % 4 != 0) w[FULLW] = *reinterpret_cast<const uint16_t*>(base + 4 * FULLW);
}

// Same as load_words, through a raw buffer descriptor at byte offset `off`.
// An offset at or beyond the end of the buffer returns zeros and touches no
// memory, which lets lanes without a sample run the same straight-line code.
template <typename T, int NL, int VEC>
__device__ __forceinline__ void load_words_buf(__amdgpu_buffer_rsrc_t rs, uint32_t off,
                                               uint32_t (&w)[Words<T, NL>::N]) {
    constexpr int NB = Words<T, NL>::NB;
    constexpr int NV = NB / VEC;
    constexpr int DONE = NV * VEC / 4;
    constexpr int FULLW = NB / 4;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        if constexpr (VEC == 16) {
            const auto q = __builtin_amdgcn_raw_buffer_load_b128(rs, off + 16 * v, 0, 0);
            w[4 * v + 0] = q[0];
            w[4 * v + 1] = q[1];
            w[4 * v + 2] = q[2];
            w[4 * v + 3] = q[3];
        } else if constexpr (VEC == 8) {
            const auto q = __builtin_amdgcn_raw_buffer_load_b64(rs, off + 8 * v, 0, 0);
            w[2 * v + 0] = q[0];
            w[2 * v + 1] = q[1];
        } else {
            w[v] = __builtin_amdgcn_raw_buffer_load_b32(rs, off + 4 * v, 0, 0);
        }
    }
#pragma unroll
    for (int i = DONE; i < FULLW; ++i) w[i] = __builtin_amdgcn_raw_buffer_load_b32(rs, off + 4 * i, 0, 0);
    if constexpr (NB % 4 != 0) w[FULLW] = __builtin_amdgcn_raw_buffer_load_b16(rs, off + 4 * FULLW, 0, 0);
}

__device__ __forceinline__ float sigma_buf(__amdgpu_buffer_rsrc_t rs, uint32_t off, float*) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0));
}
__device__ __forceinline__ float sigma_buf(__amdgpu_buffer_rsrc_t rs, uint32_t off, __half*) {
    return __half2float(__ushort_as_half(__builtin_amdgcn_raw_buffer_load_b16(rs, off, 0, 0)));
}

// Element i of a record held as raw words, widened to float.
template <typename T, int NW>
__device__ __forceinline__ float word_elem(const uint32_t (&w)[NW], int i) {
    if constexpr (sizeof(T) == 4) {
        return __uint_as_float(w[i]);
    } else {
        const uint32_t h = (i & 1) ? (w[i >> 1] >> 16) : (w[i >> 1] & 0xffffu);
        return __half2float(__ushort_as_half((unsigned short)h));
    }
}

// Logistic sigmoid (Sec. 4.1) with the hardware reciprocal (1 ulp): the
// correctly rounded division costs ~10 instructions per colour channel.
__device__ __forceinline__ float sigmoid(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }

// ---------------------------------------------------------------------------
// Ray geometry in grid units: the box spans [0, 2^D]^3 and finest cells have
// unit edge.  The ray is og + s * dg with dg the caller's (unnormalised)
// direction scaled to grid units, so no rounding enters the direction; the
// origin transform, the plane-crossing parameters s and the positions are
// evaluated in FP64.  In FP32 the crossing parameter of a far plane carries
// an error of about 2^-24 of the distance travelled, which becomes an error of
// every segment length; with densities of several hundred per unit length
// that exceeds 1e-4 in colour.  Leaf values, SH and compositing stay FP32.
// A segment's length in world units is (s_exit - s_entry) * |d|.
// ---------------------------------------------------------------------------
struct Ray {
    double og[3];  // origin, grid units
    double dg[3];  // direction (caller's length), grid units per unit of s
    double inv[3]; // 1 / dg
    double len;    // |d| in world units
    float dn[3];   // unit direction, world (SH argument)
    int c[3];      // finest-level coordinates of the current cell
    double s;      // current parameter
    double s_end;  // end of the rendered part (slicing plane), else 1e300
    double s_exit; // end of the walk: min(s_end, box exit)
    bool more;     // split walks: the walk stopped at its step limit with cells left
};

// The walk covers the parameters s in [max(s_lo, 0), s_hi] inside the box.
__device__ __forceinline__ bool ray_setup(const KTree& tr, const double (&o)[3], const double (&d)[3], Ray& r,
                                          double s_lo = 0.0, double s_hi = 1e300) {
    const double len2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (!(len2 > 0.0) || !(len2 < 1e300)) return false;
    r.len = sqrt(len2);
    const double il = 1.0 / r.len;
#pragma unroll
    for (int k = 0; k < 3; ++k) r.dn[k] = (float)(d[k] * il);
    const double N = (double)(1 << tr.depth);
    double s0 = fmax(s_lo, 0.0), s1 = s_hi;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        r.og[k] = (o[k] - tr.lo[k]) * tr.scale;
        if (!(fabs(r.og[k]) < 1e300)) return false;
        // A ray lying in a grid plane (zero component) belongs to the cell
        // above it (half-open cells): a positive direction component of
        // 1e-300 grid units gives exactly that, with exit parameters of
        // ~1e300 that never win, and needs no special case in the walk.
        const double g = d[k] * tr.scale;
        r.dg[k] = (g == 0.0) ? 1e-300 : g;
        r.inv[k] = 1.0 / r.dg[k];
        const double ta = (0.0 - r.og[k]) * r.inv[k];
        const double tb = (N - r.og[k]) * r.inv[k];
        s0 = fmax(s0, fmin(ta, tb));
        s1 = fmin(s1, fmax(ta, tb));
    }
    if (!(s1 > s0)) return false;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double p = fma(s0, r.dg[k], r.og[k]);
        r.c[k] = (int)fmin(fmax(floor(p), 0.0), N - 1.0);
    }
    r.s = s0;
    r.s_end = s_hi;
    r.s_exit = s1;
    return true;
}

// Parameter range [s_lo, s_hi] of the ray o + s d inside the slicing
// half-space n.x + w >= 0 of the viewer (Sec. 5.5); a ray parallel to the
// plane and outside it gets an empty range.  An all-zero plane keeps the
// whole ray.
__device__ __forceinline__ void clip_range(const KOpts& op, const double (&o)[3], const double (&d)[3],
                                           double& s_lo, double& s_hi) {
    const double nx = op.clip[0], ny = op.clip[1], nz = op.clip[2], w = op.clip[3];
    const double p0 = nx * o[0] + ny * o[1] + nz * o[2] + w;
    const double pd = nx * d[0] + ny * d[1] + nz * d[2];
    const double t = -p0 / pd;  // crossing (unused when pd == 0)
    s_lo = pd > 0.0 ? t : (((pd == 0.0) & (p0 < 0.0)) ? 1e300 : 0.0);
    s_hi = pd < 0.0 ? t : 1e300;
}

// Child slot of cell c below a node of level L (bits D-1-L of the coordinates).
__device__ __forceinline__ uint32_t child_slot(const int (&c)[3], int D, int L) {
    const int sft = D - 1 - L;
    return (uint32_t)((((c[0] >> sft) & 1) << 2) | (((c[1] >> sft) & 1) << 1) | ((c[2] >> sft) & 1));
}

// Walks the segments of a ray.  Data leaves crossed over a positive length
// go through a two-stage sampler: smp.issue(leaf, delta, t) starts the loads
// of the leaf's density and SH record (leaf -1: a lane without a sample,
// which loads nothing; t is the segment's start distance from the origin),
// and smp.consume() shades and composites the sample one step later and
// returns true to stop the walk; smp.flush() then runs with every lane still
// walking.  A sampler with kClip set also ends the walk at r.s_end.  The samples, their order and the
// stop point are those of the plain front-to-back walk.  Returns the number
// of cells visited.
//
// Per step: finish the descent to the leaf holding cell c; compute the exit
// parameter and the next cell; prefetch the next cell's first child entry;
// composite the previous sample; start this cell's gather.  Loads complete in
// issue order, so the next descent waits only for its own entry and not for
// the gather, and compositing runs while that entry is in flight.
//
// stk is this lane's column of a [level][kBlock] node stack in LDS holding
// the node of every level on the path to c.  The next descent restarts from
// the deepest ancestor shared by the old and the new cell (the level of the
// highest differing coordinate bit) instead of the root, so a step costs one
// or two dependent loads instead of ~D.  The child array is read through a
// buffer descriptor: an entry beyond the array reads as 0 (empty), and an
// internal entry below depth D or past the node count is counted as
// malformed and taken as empty.
//
// SPLIT: reaching max_steps with cells left is not an error; the walk then
// leaves r.s and r.c at the start of the next cell and sets r.more (unless
// the last sample ended it by early stopping), so that it can be resumed or
// handed on.  A chunk sampler (kChunk) learns for every sample whether its
// cell ends inside the walked range (cpl_next) or is cut by r.s_end.
template <class S, class = void>
struct is_chunk : std::false_type {};
template <class S>
struct is_chunk<S, std::void_t<decltype(S::kChunk)>> : std::bool_constant<S::kChunk> {};
// A sampler with kCountLoads set counts the child entries the walk reads
// from memory (member `loads`); the out-of-range prefetch after the last
// step reads nothing and is not counted.
template <class S, class = void>
struct counts_loads : std::false_type {};
template <class S>
struct counts_loads<S, std::void_t<decltype(S::kCountLoads)>> : std::bool_constant<S::kCountLoads> {};

// Spreads the three low bits of b to bits 0, 3 and 6.
__device__ __forceinline__ uint32_t spread3(uint32_t b) { return (b | (b << 2) | (b << 4)) & 0x49u; }

// Index of a finest cell in its 8x8x8 brick: the child slots of the three
// levels below the brick's cube, slot1 << 6 | slot2 << 3 | slot3 (slot =
// 4 x + 2 y + z of that level's coordinate bits).
__device__ __forceinline__ uint32_t brick_cell(const int (&c)[3]) {
    return (spread3((uint32_t)c[0] & 7u) << 2) | (spread3((uint32_t)c[1] & 7u) << 1) | spread3((uint32_t)c[2] & 7u);
}

template <class Sampler, bool SPLIT = false>
__device__ __forceinline__ int march(const KTree& tr, Ray& r, int max_steps, int* __restrict__ stk,
                                     Sampler& smp) {
    const int D = tr.depth;
    const int M = tr.brick_level;
    const int N = 1 << D;
    const uint32_t idx_end = tr.index_bytes;
    const __amdgpu_buffer_rsrc_t child = raw_rsrc(tr.child, idx_end);
    const uint32_t brick0 = (uint32_t)tr.n_top * 32u;  // byte offset of brick 0
    int steps = 0;
    bool pending = false, bad = false, cap_end = false;
    // L: level of the node whose entry e is (e describes a level-(L+1) cell),
    // or, with inb set, e is the brick entry of the cell c
    int L = 0, node = 0;
    bool inb = false;
    uint32_t bofs = 0;  // byte offset of the brick holding c (valid while inb)
    stk[0] = 0;
    int e = __builtin_amdgcn_raw_buffer_load_b32(child, child_slot(r.c, D, 0) << 2, 0, 0);
    if constexpr (counts_loads<Sampler>::value) smp.loads += 1;
    // an empty gather, so that every path into the loop has the same loads in
    // flight behind the entry (the compiler then waits for the entry alone)
    smp.issue(-1, 0.0f, 0.0f);
    while (true) {
        // finish the descent to the leaf holding c: its number (-1: empty) and level
        int leaf, lvl;
        if (inb) {
            lvl = D - (e & 3);
            leaf = (int)((uint32_t)e >> 2) - 1;
        } else {
            ++L;  // e is the entry of the level-L cell holding c
            // further levels (each waits for its own load, and for any older one)
            while ((e > 0) & (e < tr.n_top) & (L < M)) {
                node = e;
                stk[L * kBlock] = node;
                e = __builtin_amdgcn_raw_buffer_load_b32(
                    child, ((uint32_t)node << 5) | (child_slot(r.c, D, L) << 2), 0, 0);
                if constexpr (counts_loads<Sampler>::value) smp.loads += 1;
                ++L;
            }
            if ((e > 0) & (L == M) & (M < D) & (e >= tr.n_top)) {
                // the level-M cube holding c is a brick: one load gives the leaf
                bofs = brick0 + (uint32_t)(e - tr.n_top) * 2048u;
                e = __builtin_amdgcn_raw_buffer_load_b32(child, bofs + (brick_cell(r.c) << 2), 0, 0);
                if constexpr (counts_loads<Sampler>::value) smp.loads += 1;
                inb = true;
                lvl = D - (e & 3);
                leaf = (int)((uint32_t)e >> 2) - 1;
            } else {
                // a leaf or empty cube of level L; any other positive entry
                // (past the nodes, or internal at the deepest level) is malformed
                const bool malformed = e > 0;
                bad |= malformed;
                leaf = malformed ? -1 : -1 - e;
                lvl = L;
            }
        }
        if (leaf >= tr.n_leaves) {
            bad = true;
            leaf = -1;
        }
        // exit parameter: the nearest far face (branch-free; pos = moving up the axis)
        const int csz = 1 << (D - lvl);
        int lo[3];
        bool pos[3];
        double sk[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            lo[k] = r.c[k] & ~(csz - 1);
            pos[k] = r.dg[k] > 0.0;
            sk[k] = ((double)(lo[k] + (pos[k] ? csz : 0)) - r.og[k]) * r.inv[k];
        }
        double se = fmax(fmin(fmin(sk[0], sk[1]), sk[2]), r.s);
        bool cpl = true;
        if constexpr (Sampler::kClip) {
            if constexpr (is_chunk<Sampler>::value) {
                // a piece's cell is cut when the next piece starts inside it;
                // that piece finds its first cell from the point at s_end as
                // ray_setup does, so the two agree on every cell (a cell
                // ending at s_end up to rounding is complete here exactly
                // when the next piece starts in a later cell)
                if (se > r.s_end) {
                    bool inside = true;
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        const double q = fmin(fmax(floor(fma(r.s_end, r.dg[k], r.og[k])), 0.0), (double)(N - 1));
                        inside &= (q >= (double)lo[k]) & (q < (double)(lo[k] + csz));
                    }
                    cpl = !inside;
                }
            } else {
                cpl = se <= r.s_end;
            }
            se = fmin(se, r.s_end);
        }
        const float delta = (float)((se - r.s) * r.len);
        const float t_in = (float)(r.s * r.len);
        ++steps;
        // next cell: axes whose face is reached step to the neighbouring cell;
        // the others take the finest cell of the exit point, kept inside the
        // current cube and never moving against the ray (truncation equals
        // floor here: the result is clamped to >= lo >= 0)
        bool out = false;
        int nc[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int stepped = pos[k] ? lo[k] + csz : lo[k] - 1;
            const int q = min(max((int)fma(se, r.dg[k], r.og[k]), lo[k]), lo[k] + csz - 1);
            const int kept = pos[k] ? max(q, r.c[k]) : min(q, r.c[k]);
            const bool cross = sk[k] <= se;
            nc[k] = cross ? stepped : kept;
            out |= cross & ((stepped < 0) | (stepped >= N));
        }
        if constexpr (Sampler::kClip) out |= se >= r.s_end;
        r.s = se;
        const bool capped = !out & (steps >= max_steps);
        if constexpr (!SPLIT) bad |= capped;
        const bool last = out | capped;
        // prefetch the next cell's entry.  The cells agree on the coordinate
        // bits above the highest differing one: inside the same brick the
        // brick entry is read directly, else the walk restarts below the
        // deepest common ancestor above the brick level (from the stack).
        // The load is issued on every path (out of range after the last
        // step) so the compiler can count the loads in flight exactly.
        uint32_t pf = idx_end;
        if (!last) {
            const int diff = (r.c[0] ^ nc[0]) | (r.c[1] ^ nc[1]) | (r.c[2] ^ nc[2]);
            const int la = D - 32 + __clz(diff);
            r.c[0] = nc[0];
            r.c[1] = nc[1];
            r.c[2] = nc[2];
            if (inb & (la >= M)) {
                pf = bofs + (brick_cell(r.c) << 2);
            } else {
                inb = false;
                L = la;
                node = stk[L * kBlock];
                pf = ((uint32_t)node << 5) | (child_slot(r.c, D, L) << 2);
            }
        }
        if constexpr (SPLIT) {
            if (capped) {
                r.c[0] = nc[0];
                r.c[1] = nc[1];
                r.c[2] = nc[2];
            }
        }
        e = __builtin_amdgcn_raw_buffer_load_b32(child, pf, 0, 0);
        if constexpr (counts_loads<Sampler>::value) smp.loads += last ? 0 : 1;
        // composite the previous sample (its loads precede the prefetch)
        bool stop = false;
        if (pending) {
            pending = false;
            stop = smp.consume();
        }
        smp.flush();
        // start this cell's gather; lanes without a sample load nothing.  The
        // walk ends only at the bottom of the body, so every path back to the
        // top has issued the same loads.
        const bool take = !stop & (leaf >= 0) & (delta > 0.0f);
        if constexpr (is_chunk<Sampler>::value) {
            smp.cpl_next = cpl;
            // a piece's first cell without a sample (the zero-length rest of
            // a cell the previous piece cut, or a start on a face) still
            // carries the stop test at its end
            if ((steps == 1) & !take & !stop) stop = smp.test_first(cpl);
        }
        smp.issue(take ? leaf : -1, delta, t_in);
        pending = take;
        if constexpr (SPLIT) cap_end = capped & !stop;
        if (last | stop) break;
    }
    bool end_stop = false;
    if (pending) end_stop = smp.consume();
    smp.flush();
    if constexpr (SPLIT) r.more = cap_end & !end_stop;
    // a lane that met a malformed entry or the step cap is counted once
    if (bad) atomicAdd(&g_po_errors, 1ull);
    return steps;
}

template <typename T, int K, int NW>
__device__ __forceinline__ float dot_channel(const uint32_t (&w)[NW], int base, const float (&Y)[K]) {
    float z = word_elem<T>(w, base) * Y[0];
#pragma unroll
    for (int k = 1; k < K; ++k) z = fmaf(word_elem<T>(w, base + k), Y[k], z);
    return z;
}

// Forward shading and compositing of the samples of one ray (Sec. 3
// eqn:quad, Sec. 4.1 colour, App. B.3 clamp of the raw density).  VIEW adds
// the viewer outputs of Sec. 5.5: the expected termination distance and the
// end of the walk at a slicing plane.
template <typename T, int K, int VEC, int NL, bool VIEW>
struct FwdSampler {
    static constexpr int NW = Words<T, NL>::N;
    static constexpr bool kClip = VIEW;
    // float16 records: the basis values live in LDS ([k][lane], written by
    // init_basis) instead of K registers, which takes the float16 chunk and
    // sub-chunk walks to 5 waves per SIMD (depth-9 800x800 frame 0.461 ->
    // 0.451 ms, 1920x1080 1.13 -> 1.06 ms)
    static constexpr bool kLdsY = std::is_same<T, __half>::value && !VIEW;
    __amdgpu_buffer_rsrc_t sig, shb;
    uint32_t sig_end, sh_end, rec_bytes;
    float stopT;
    float Y[kLdsY ? 1 : K];
    float* Yl;  // kLdsY: this lane's column of the LDS basis values
    float c0 = 0.0f, c1 = 0.0f, c2 = 0.0f, Tl = 1.0f;
    float dep = 0.0f;
    int ns = 0;
    // in flight
    float raw, delta, ta;
    uint32_t w[NW];

    // leaf < 0: no sample; the out-of-range offsets load zeros without memory traffic
    __device__ __forceinline__ void issue(int leaf, float d, float t_in) {
        raw = sigma_buf(sig, leaf < 0 ? sig_end : (uint32_t)leaf * (uint32_t)sizeof(T), (T*)nullptr);
        load_words_buf<T, NL, VEC>(shb, leaf < 0 ? sh_end : (uint32_t)leaf * rec_bytes, w);
        delta = d;
        if constexpr (VIEW) ta = t_in;
    }
    __device__ __forceinline__ void flush() {}
    __device__ __forceinline__ bool consume() {
        ++ns;
        const float s = fmaxf(raw, 0.0f);
        if (!(s > 0.0f)) return false;
        const float ex = __expf(-(s * delta));
        const float wgt = Tl * (1.0f - ex);
        if constexpr (kLdsY) {
            float Yv[K];
#pragma unroll
            for (int k = 0; k < K; ++k) Yv[k] = Yl[k * kBlock];
            c0 = fmaf(wgt, sigmoid(dot_channel<T, K>(w, 0, Yv)), c0);
            c1 = fmaf(wgt, sigmoid(dot_channel<T, K>(w, K, Yv)), c1);
            c2 = fmaf(wgt, sigmoid(dot_channel<T, K>(w, 2 * K, Yv)), c2);
        } else {
            c0 = fmaf(wgt, sigmoid(dot_channel<T, K>(w, 0, Y)), c0);
            c1 = fmaf(wgt, sigmoid(dot_channel<T, K>(w, K, Y)), c1);
            c2 = fmaf(wgt, sigmoid(dot_channel<T, K>(w, 2 * K, Y)), c2);
        }
        if constexpr (VIEW) {
            // integral of t sigma T(t) over the segment [ta, ta + delta]:
            // Tl (ta alpha + delta f), f = alpha / tau - e^-tau, from its
            // series below tau = 0.05 (alpha / tau cancels there)
            const float tau = s * delta;
            const float al = 1.0f - ex;
            const float f = tau < 0.05f
                                ? tau * (0.5f - tau * (1.0f / 3.0f - tau * (0.125f - tau * (1.0f / 30.0f - tau * (1.0f / 144.0f)))))
                                : al / tau - ex;
            dep = fmaf(Tl, fmaf(ta, al, delta * f), dep);
        }
        Tl = Tl * ex;
        return Tl < stopT;
    }
};

// The SH or SG basis at the ray direction (once per ray) for a plain
// forward sampler: into its registers, or for float16 records into this
// lane's column of an LDS array (one per kernel, K x kBlock floats).
template <typename T, int K, int V, class Smp>
__device__ __forceinline__ void init_basis(Smp& smp, const KTree& tr, const Ray& r) {
    if constexpr (Smp::kLdsY) {
        __shared__ float s_Y[K * kBlock];
        float Yt[K];
        if constexpr (V == PO_FWD_SG)
            sg_basis<K>(tr.lobes, r.dn[0], r.dn[1], r.dn[2], Yt);
        else
            sh_basis<K>(r.dn[0], r.dn[1], r.dn[2], Yt);
        smp.Yl = s_Y + threadIdx.x;
#pragma unroll
        for (int k = 0; k < K; ++k) smp.Yl[k * kBlock] = Yt[k];
    } else if constexpr (V == PO_FWD_SG) {
        sg_basis<K>(tr.lobes, r.dn[0], r.dn[1], r.dn[2], smp.Y);
    } else {
        sh_basis<K>(r.dn[0], r.dn[1], r.dn[2], smp.Y);
    }
}

// Codebook leaves (App. B.2): the record holds one 16-bit codebook position
// per basis function; consume() gathers the K float16 colours (8 bytes each,
// from the per-basis codebooks) and shades as an SH leaf.  The gathers are in
// flight together with the next cell's entry prefetch, which the walk waits
// for next anyway.
template <int K, int VEC, int NL>
struct CbSampler {
    static constexpr int NW = Words<__half, NL>::N;
    static constexpr bool kClip = false;
    __amdgpu_buffer_rsrc_t sig, shb, cb;
    uint32_t sig_end, sh_end, rec_bytes, cb_basis_bytes;
    float stopT;
    float Y[K];
    float c0 = 0.0f, c1 = 0.0f, c2 = 0.0f, Tl = 1.0f;
    float dep = 0.0f;
    int ns = 0;
    // in flight
    float raw, delta;
    uint32_t w[NW];

    __device__ __forceinline__ void issue(int leaf, float d, float) {
        raw = sigma_buf(sig, leaf < 0 ? sig_end : (uint32_t)leaf * 2u, (__half*)nullptr);
        load_words_buf<__half, NL, VEC>(shb, leaf < 0 ? sh_end : (uint32_t)leaf * rec_bytes, w);
        delta = d;
    }
    __device__ __forceinline__ void flush() {}
    __device__ __forceinline__ bool consume() {
        ++ns;
        const float s = fmaxf(raw, 0.0f);
        if (!(s > 0.0f)) return false;
        uint32_t e0[K], e1[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint32_t pos = (w[k >> 1] >> (16 * (k & 1))) & 0xffffu;
            const auto q = __builtin_amdgcn_raw_buffer_load_b64(cb, (uint32_t)k * cb_basis_bytes + pos * 8u, 0, 0);
            e0[k] = q[0];
            e1[k] = q[1];
        }
        float z0 = 0.0f, z1 = 0.0f, z2 = 0.0f;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            z0 = fmaf(__half2float(__ushort_as_half((unsigned short)(e0[k] & 0xffffu))), Y[k], z0);
            z1 = fmaf(__half2float(__ushort_as_half((unsigned short)(e0[k] >> 16))), Y[k], z1);
            z2 = fmaf(__half2float(__ushort_as_half((unsigned short)(e1[k] & 0xffffu))), Y[k], z2);
        }
        const float ex = __expf(-(s * delta));
        const float wgt = Tl * (1.0f - ex);
        c0 = fmaf(wgt, sigmoid(z0), c0);
        c1 = fmaf(wgt, sigmoid(z1), c1);
        c2 = fmaf(wgt, sigmoid(z2), c2);
        Tl = Tl * ex;
        return Tl < stopT;
    }
};

// One chunk [s_lo, s_hi] of a split ray.  The chunk composites from T = 1
// (or from a known transmittance when it is walked again); because
// compositing is associative, chunk results combine front to back with the
// over operator.  Early stopping is tested where the sequential walk tests it,
// at the end of a cell: a sample whose cell continues past s_hi (cut by the
// chunk boundary: the next chunk starts inside it) is composited without a
// test, and its remainder, the first cell of the next chunk, carries the
// test, also when it has zero length and takes no sample.  Tlast is T after the last
// tested sample (-1: none); the chunk stops itself once T < stopT there,
// since its walk cannot matter past that point for any transmittance in
// front of it.
template <class Base, bool COUNT = false>
struct ChunkOf : Base {
    static constexpr bool kClip = true;
    static constexpr bool kChunk = true;
    bool cpl_next = true, cpl = true;
    bool hit = false;       // stopped by stopT
    bool smp_cut = false;   // the last composited sample was cut by the walk's end
    int issued = 0;         // issue() calls: the walk's first is its placeholder gather
    int skip0 = 0;          // 1: the first cell had zero length (the walk began on its far face)
    float Tlast = -1.0f;

    __device__ __forceinline__ void issue(int leaf, float d, float t_in) {
        Base::issue(leaf, d, t_in);
        cpl = cpl_next;
        if constexpr (COUNT) {
            if (issued == 1) skip0 = d > 0.0f ? 0 : 1;
            ++issued;
        }
    }
    __device__ __forceinline__ bool consume() {
        const bool st = Base::consume();
        if constexpr (COUNT) smp_cut = !cpl;
        if (!cpl) return false;
        Tlast = this->Tl;
        hit |= st;
        return st;
    }
    // the stop test at the end of a first cell that took no sample (c: the
    // cell ends inside the piece)
    __device__ __forceinline__ bool test_first(bool c) {
        if (!c) return false;
        Tlast = this->Tl;
        const bool st = this->Tl < this->stopT;
        hit |= st;
        return st;
    }
};

// Samplers of the split render: the first walk's, and a piece's.
template <typename T, int K, int VEC, int NL, int V>
using FirstSampler = std::conditional_t<V == PO_FWD_CB, CbSampler<K, VEC, NL>,
                                        FwdSampler<T, K, VEC, NL, V == PO_FWD_VIEW>>;
template <typename T, int K, int VEC, int NL, int V>
using ChunkSampler = ChunkOf<FirstSampler<T, K, VEC, NL, V>, V == PO_FWD_VIEW>;

// Renders one ray: colour (background included), final T, samples, steps
// and, in the viewer variant, the expected termination distance, SH subsets
// and the slicing plane.  V is a PO_FWD_* variant.
template <typename T, int K, int VEC, int NL, int V>
__device__ __forceinline__ void render_one(const KTree& tr, const KOpts& op, const double (&o)[3],
                                           const double (&d)[3], int* __restrict__ stk, float (&C)[3], float& Tr,
                                           int& ns, int& steps, float& dep) {
    C[0] = C[1] = C[2] = 0.0f;
    Tr = 1.0f;
    ns = 0;
    steps = 0;
    dep = 0.0f;
    constexpr bool VIEW = V == PO_FWD_VIEW;
    Ray r;
    double s_lo = 0.0, s_hi = 1e300;
    if constexpr (VIEW) clip_range(op, o, d, s_lo, s_hi);
    if (ray_setup(tr, o, d, r, s_lo, s_hi)) {
        using Smp = std::conditional_t<V == PO_FWD_CB, CbSampler<K, VEC, NL>, FwdSampler<T, K, VEC, NL, VIEW>>;
        Smp smp;
        smp.sig = raw_rsrc(tr.sigma, tr.sigma_bytes);
        smp.shb = raw_rsrc(tr.sh, tr.sh_bytes);
        smp.sig_end = tr.sigma_bytes;
        smp.sh_end = tr.sh_bytes;
        smp.rec_bytes = (uint32_t)tr.stride * (uint32_t)sizeof(T);
        smp.stopT = op.stop_T;
        if constexpr (V == PO_FWD_CB) {
            smp.cb_basis_bytes = (uint32_t)tr.cb_entries * 8u;
            smp.cb = raw_rsrc(tr.codebook, (uint32_t)K * smp.cb_basis_bytes);
        }
        if constexpr (V == PO_FWD_SH || V == PO_FWD_SG)
            init_basis<T, K, V>(smp, tr, r);
        else if constexpr (V == PO_FWD_CB)
            sh_basis<K>(r.dn[0], r.dn[1], r.dn[2], smp.Y);
        else
            colour_basis<K>(tr, r.dn[0], r.dn[1], r.dn[2], smp.Y);
        if constexpr (VIEW) {
#pragma unroll
            for (int k = 0; k < K; ++k)
                if ((op.sh_off >> k) & 1u) smp.Y[k] = 0.0f;
        }
        steps = march(tr, r, op.max_steps, stk, smp);
        C[0] = smp.c0;
        C[1] = smp.c1;
        C[2] = smp.c2;
        Tr = smp.Tl;
        ns = smp.ns;
        dep = smp.dep;
    }
    C[0] = fmaf(Tr, op.bg[0], C[0]);
    C[1] = fmaf(Tr, op.bg[1], C[1]);
    C[2] = fmaf(Tr, op.bg[2], C[2]);
}

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs on
// XCD b % 8).  Remap so that each XCD receives one contiguous range of the
// logical workgroup order (neighbouring tiles share its L2).  The grid has
// 8 * ceil(n / 8) workgroups; returns -1 for the padding ones.
__device__ __forceinline__ int64_t xcd_swizzle(int64_t b, int64_t n_logical) {
    const int64_t per = (n_logical + 7) / 8;
    const int64_t l = (b % 8) * per + b / 8;
    return l < n_logical ? l : -1;
}

// Logical workgroup of hardware workgroup b when runs of `chunk` logical
// workgroups (a tile row) are dealt round-robin over the 8 XCDs: XCD x gets
// runs x, x + 8, ...  The grid has 8 * chunk * ceil(ceil(n_logical / chunk) / 8)
// workgroups (rows_grid); returns -1 for the padding ones.  Camera walks deal
// tile rows this way: every XCD then holds a share of the frame's longest
// walks, which crowd into the middle rows (one-pass depth-9 800x800 FP32
// frame: 0.706 against 0.854 ms with a contiguous band of rows per XCD).
__device__ __forceinline__ int64_t xcd_interleave(int64_t b, int64_t n_logical, int64_t chunk) {
    const int64_t x = b & 7, j = b >> 3;
    const int64_t l = ((j / chunk) * 8 + x) * chunk + (j % chunk);
    return l < n_logical ? l : -1;
}
template <typename T, int K, int VEC, int NL, int V>
__global__ __launch_bounds__(kBlock) void k_render_rays(KTree tr, int64_t n, int64_t n_blocks,
                                                        const float* __restrict__ o,
                                                        const float* __restrict__ d, KOpts op,
                                                        float* __restrict__ rgb, float* __restrict__ aux) {
    const int64_t blk = xcd_swizzle(blockIdx.x, n_blocks);
    if (blk < 0) return;
    const int64_t i = blk * kBlock + threadIdx.x;
    if (i >= n) return;
    const double ro[3] = {(double)o[3 * i], (double)o[3 * i + 1], (double)o[3 * i + 2]};
    const double rd[3] = {(double)d[3 * i], (double)d[3 * i + 1], (double)d[3 * i + 2]};
    float C[3], Tr, dep;
    int ns, steps;
    extern __shared__ int po_stack[];
    render_one<T, K, VEC, NL, V>(tr, op, ro, rd, po_stack + threadIdx.x, C, Tr, ns, steps, dep);
    rgb[3 * i + 0] = C[0];
    rgb[3 * i + 1] = C[1];
    rgb[3 * i + 2] = C[2];
    if constexpr (V == PO_FWD_VIEW) {
        if (aux) {
            aux[4 * i + 0] = Tr;
            aux[4 * i + 1] = (float)ns;
            aux[4 * i + 2] = (float)steps;
            aux[4 * i + 3] = dep;
        }
    }
}

// Pinhole ray through the centre of pixel (px, py), in FP64 like the rest of
// the ray geometry (direction not normalised).
__device__ __forceinline__ void pixel_ray(const KCam& cam, int px, int py, double (&ro)[3], double (&rd)[3]) {
    const double x = ((double)px + 0.5 - (double)cam.cx) / (double)cam.fx;
    const double y = -(((double)py + 0.5 - (double)cam.cy) / (double)cam.fy);
    const float* M = cam.c2w;
    rd[0] = (double)M[0] * x + (double)M[1] * y - (double)M[2];
    rd[1] = (double)M[4] * x + (double)M[5] * y - (double)M[6];
    rd[2] = (double)M[8] * x + (double)M[9] * y - (double)M[10];
    ro[0] = (double)M[3];
    ro[1] = (double)M[7];
    ro[2] = (double)M[11];
}

__global__ __launch_bounds__(256) void k_camera_rays(KCam cam, float* __restrict__ o, float* __restrict__ d) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= (int64_t)cam.W * cam.H) return;
    double ro[3], rd[3];
    pixel_ray(cam, (int)(p % cam.W), (int)(p / cam.W), ro, rd);
    const double il = 1.0 / sqrt(rd[0] * rd[0] + rd[1] * rd[1] + rd[2] * rd[2]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        o[3 * p + k] = (float)ro[k];
        d[3 * p + k] = (float)(rd[k] * il);
    }
}

template <int MAXJ>
struct KBatch {
    KJob job[MAXJ];
    int32_t n_jobs;
    int32_t n_blocks;
};
// passed by value as the kernel argument block, limited to 4 KiB
static_assert(sizeof(KBatch<PO_BATCH_MAX_JOBS>) <= 4096, "batched kernel arguments exceed 4 KiB");

// Camera jobs: a 16x16 tile is rendered by four single-wave workgroups, one
// per 8x8 quadrant; lane l takes the pixel (l & 7, l >> 3) of its quadrant.
template <typename T, int K, int VEC, int NL, int MAXJ, int V>
__global__ __launch_bounds__(kBlock) void k_render_camera(KBatch<MAXJ> B) {
    // one camera: tile rows dealt over the XCDs; batches: one contiguous range per XCD
    const int64_t b = MAXJ == 1 ? xcd_interleave(blockIdx.x, B.n_blocks, 4 * (int64_t)B.job[0].tiles_x)
                                : xcd_swizzle(blockIdx.x, B.n_blocks);
    if (b < 0) return;
    int j = 0;
    if constexpr (MAXJ > 1) {
        for (int q = 1; q < B.n_jobs; ++q)
            if (b >= B.job[q].block_begin) j = q;
    }
    const KJob& J = B.job[j];
    const int q = (int)(b - J.block_begin);
    const int tile = J.tile_begin + (q >> 2), quad = q & 3;
    const int tx = tile % J.tiles_x, ty = tile / J.tiles_x;
    const int lane = threadIdx.x;
    const int px = tx * 16 + (quad & 1) * 8 + (lane & 7);
    const int py = ty * 16 + (quad >> 1) * 8 + (lane >> 3);
    if (px >= J.cam.W || py >= J.cam.H) return;
    double ro[3], rd[3];
    pixel_ray(J.cam, px, py, ro, rd);
    float C[3], Tr, dep;
    int ns, steps;
    extern __shared__ int po_stack[];
    render_one<T, K, VEC, NL, V>(J.tr, J.op, ro, rd, po_stack + threadIdx.x, C, Tr, ns, steps, dep);
    const size_t p = (size_t)py * J.cam.W + px;
    J.rgb[3 * p + 0] = C[0];
    J.rgb[3 * p + 1] = C[1];
    J.rgb[3 * p + 2] = C[2];
    if constexpr (V == PO_FWD_VIEW) {
        if (J.aux) {
            J.aux[4 * p + 0] = Tr;
            J.aux[4 * p + 1] = (float)ns;
            J.aux[4 * p + 2] = (float)steps;
            J.aux[4 * p + 3] = dep;
        }
    }
}

// ---------------------------------------------------------------------------
// Split camera render.  The frame time of a one-pass render is set by its
// longest walks (a few hundred cells, against a median of a few), which run
// one cell at a time while most of the chip idles.  Compositing is
// associative (Sec. 3, eqn:quad: a range of segments acts on what lies behind
// it as (C, T) -> C_range + T_range C), so a long walk can be cut into
// pieces walked in parallel and joined front to back:
//   k_render_camera_split  walks every ray for at most split_steps cells;
//                          a ray with cells left is handed on: its state
//                          (s, T, C) and 1-16 chunks, equal parameter
//                          intervals of the rest of the ray;
//   k_render_chunks        walks one chunk per lane for at most chunk_cap
//                          cells; a chunk with cells left hands its
//                          remainder on as 1-16 sub-chunks (cells are
//                          bunched along a ray, so equal intervals are not
//                          equal work; the walked part of the chunk tells
//                          how dense the rest is);
//   k_render_subchunks     walks one sub-chunk per lane to its end;
//   k_render_join          combines each ray's pieces in order and writes
//                          the pixel.  Where early stopping ends the ray
//                          inside a piece (T below stop_T after a cell), the
//                          piece is walked again from its start with the
//                          known transmittance and stops where the one-pass
//                          walk stops.
// The result equals the one-pass render up to float rounding.  The queues
// are split into regions (one counter each) to spread the slot claims; a
// walk that finds its region full finishes in the lane that holds it.
// ---------------------------------------------------------------------------

// Queues are XCD-local: workgroup b runs on XCD b % 8 (the dispatcher deals
// workgroups round-robin over the XCDs), claims its pieces in one of that
// XCD's eight regions (8 x + (b / 8) mod 8), and the piece kernels take the
// slots of XCD x's regions with workgroups that run on XCD x (split_slot).
// A piece's head, its result and the join's reads of it then stay in the L2
// of the XCD that wrote them (each XCD has its own L2).  The first walk
// deals tile rows over the XCDs (xcd_interleave), so that every XCD gets a
// share of the frame's long walks and its regions fill evenly.  Depth-9
// 800x800 FP32: 0.586 against 0.631 ms with regions shared by all XCDs;
// with XCD-local regions but contiguous screen bands per XCD, 1.01 ms (the
// middle bands hold most long walks).
__device__ __forceinline__ int claim_region() { return (int)((blockIdx.x & 7) * 8 + ((blockIdx.x >> 3) & 7)); }
struct ContHead {
    double s;             // parameter where the first walk stopped (start of the next cell)
    float T, c0, c1, c2;  // transmittance and colour so far
    int32_t pix;          // pixel index py * W + px
    int32_t pad;
};
static_assert(sizeof(ContHead) == 32, "queue record layout");

struct SubHead {
    double lo, hi;        // remainder of a chunk: [lo, hi] (hi 1e300: to the box exit)
    int32_t pix;
    int32_t pad[3];
};
static_assert(sizeof(SubHead) == 32, "queue record layout");

// Result of a walked piece: colour and transmittance composited from T = 1,
// T after its last tested sample (-1: none), and for a chunk its remainder's
// sub-chunks (first slot, count; -1 none).
// dep: the viewer variant's depth integral of the piece (from T = 1); its
// samples and cells, and whether its last sample / cell was cut by the
// piece's end (the next piece counts that cell again), go to a side record
// {ns, steps, cut_smp, cut} that only the viewer variant touches.
struct PieceOut {
    float c0, c1, c2, T;
    float Tlast;
    int32_t sub, n_sub;
    float dep;
};
static_assert(sizeof(PieceOut) == 32, "queue record layout");

template <typename T, int K, int V, class Smp>
__device__ __forceinline__ void fwd_init(Smp& smp, const KTree& tr, const KOpts& op, const Ray& r) {
    smp.sig = raw_rsrc(tr.sigma, tr.sigma_bytes);
    smp.shb = raw_rsrc(tr.sh, tr.sh_bytes);
    smp.sig_end = tr.sigma_bytes;
    smp.sh_end = tr.sh_bytes;
    smp.rec_bytes = (uint32_t)tr.stride * (uint32_t)sizeof(T);
    smp.stopT = op.stop_T;
    if constexpr (V == PO_FWD_CB) {
        smp.cb_basis_bytes = (uint32_t)tr.cb_entries * 8u;
        smp.cb = raw_rsrc(tr.codebook, (uint32_t)K * smp.cb_basis_bytes);
    }
    if constexpr (V == PO_FWD_SH || V == PO_FWD_SG) {
        init_basis<T, K, V>(smp, tr, r);
    } else if constexpr (V == PO_FWD_VIEW) {
        colour_basis<K>(tr, r.dn[0], r.dn[1], r.dn[2], smp.Y);
#pragma unroll
        for (int k = 0; k < K; ++k)
            if ((op.sh_off >> k) & 1u) smp.Y[k] = 0.0f;
    } else {
        sh_basis<K>(r.dn[0], r.dn[1], r.dn[2], smp.Y);
    }
}


// Ray idx of a split render: pixel idx = py * W + px of the job's camera
// (SRC 0) or entry idx of the caller's ray arrays (SRC 1).
template <int SRC>
__device__ __forceinline__ void ray_of(const KJob& J, const KSplit& S, int idx, double (&ro)[3], double (&rd)[3]) {
    if constexpr (SRC == 0) {
        pixel_ray(J.cam, idx % J.cam.W, idx / J.cam.W, ro, rd);
    } else {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            ro[k] = (double)S.ray_o[3 * (size_t)idx + k];
            rd[k] = (double)S.ray_d[3 * (size_t)idx + k];
        }
    }
}

// End parameter of a split ray's walk: the slicing plane of the viewer
// variant, else 1e300 (the box exit).
template <int V, int SRC>
__device__ __forceinline__ double walk_end(const KJob& J, const KSplit& S, int idx) {
    if constexpr (V == PO_FWD_VIEW) {
        double ro[3], rd[3];
        ray_of<SRC>(J, S, idx, ro, rd);
        double lo, hi;
        clip_range(J.op, ro, rd, lo, hi);
        return hi;
    } else {
        return 1e300;
    }
}

// Piece k of n of the parameter range [a, hi] of ray idx: equal intervals of
// [a, min(hi, box exit)], the last one running to hi itself.  Sets up r for
// the walk of the piece; false when the piece is empty.
template <int SRC>
__device__ __forceinline__ bool piece_setup(const KJob& J, const KSplit& S, int idx, double a, double hi, int k,
                                            int n, Ray& r) {
    double ro[3], rd[3];
    ray_of<SRC>(J, S, idx, ro, rd);
    if (!ray_setup(J.tr, ro, rd, r, a, hi)) return false;
    const double len = r.s_exit - a;
    const double lo = k == 0 ? a : a + len * (double)k / (double)n;
    const double up = k + 1 < n ? a + len * (double)(k + 1) / (double)n : hi;
    return ray_setup(J.tr, ro, rd, r, lo, up);
}

// Bounds of piece k of n of [a, hi] (as piece_setup cuts it).
template <int SRC>
__device__ __forceinline__ void piece_bounds(const KJob& J, const KSplit& S, int idx, double a, double hi, int k,
                                             int n, double& lo, double& up) {
    double ro[3], rd[3];
    ray_of<SRC>(J, S, idx, ro, rd);
    Ray r;
    const double e = ray_setup(J.tr, ro, rd, r, a, hi) ? r.s_exit : a;
    lo = k == 0 ? a : a + (e - a) * (double)k / (double)n;
    up = k + 1 < n ? a + (e - a) * (double)(k + 1) / (double)n : hi;
}

// Pieces wanted for the rest [r.s, r.s_exit] of a walk that crossed `steps`
// cells since s_first: about chunk_steps cells each, from the cells per unit
// parameter so far, and at least ub_frac of the finest-cell faces ahead.
__device__ __forceinline__ int pieces_wanted(const Ray& r, double s_first, int steps, const KSplit& S,
                                             int target) {
    const double rest = r.s_exit - r.s;
    double est = (double)steps * rest / fmax(r.s - s_first, 1e-300);
    est = fmax(est, (double)S.ub_frac * rest * (fabs(r.dg[0]) + fabs(r.dg[1]) + fabs(r.dg[2])));
    return (int)fmin(fmax(ceil(est / (double)target), 1.0), (double)kSplitMaxChunks);
}

// Claims the wave's pieces in one atomic: sum(want) slots of a region, laid
// out level-major (piece 0 of every lane that wants pieces, in lane order,
// then piece 1, ...), so that a wave of consecutive slots walks neighbouring
// rays at similar depths.  Writes every claimed slot's info {first slot of
// its piece list, piece | count << 8, next slot or -1, 0} and returns this
// lane's first slot, or -1 (want == 0, or the region cannot hold the claim:
// its claimed slots are then marked unused).  Every lane of the wave must
// call it.
__device__ __forceinline__ int claim_pieces(int32_t* count, int4* __restrict__ info, int region, int want,
                                            int region_slots) {
    const int lane = (int)threadIdx.x;
    int tot = want;
#pragma unroll
    for (int o = kBlock / 2; o >= 1; o >>= 1) tot += __shfl_xor(tot, o);
    if (tot == 0) return -1;
    int base = 0;
    if (lane == 0) base = atomicAdd(count + region, tot);
    base = __shfl(base, 0);
    const int rbase = region * region_slots;
    if (base + tot > region_slots) {
        for (int i = base + lane; i < min(base + tot, region_slots); i += kBlock) info[rbase + i].x = -1;
        return -1;
    }
    const uint64_t below = (1ull << lane) - 1ull;
    uint64_t mk = __ballot(want > 0);
    int at = rbase + base, first = -1;
    for (int j = 0; j < kSplitMaxChunks && mk != 0ull; ++j) {
        const uint64_t mk1 = __ballot(want > j + 1);
        const int at1 = at + __popcll(mk);
        if (want > j) {
            const int slot = at + __popcll(mk & below);
            if (j == 0) first = slot;
            const int next = want > j + 1 ? at1 + __popcll(mk1 & below) : -1;
            info[slot] = make_int4(first, j | (want << 8), next, 0);
        }
        at = at1;
        mk = mk1;
    }
    return first;
}

// The first walk of a split render for ray idx (valid: idx names a ray):
// at most split_steps cells, then the ray is handed on or, if its region of
// the queue is full, walked to its end here.  Every lane of the wave must
// call it.
template <typename T, int K, int VEC, int NL, int V, int SRC>
__device__ __forceinline__ void first_walk(const KJob& J, const KSplit& S, int idx, bool valid) {
    const KTree& tr = J.tr;
    const KOpts& op = J.op;
    extern __shared__ int po_stack[];
    int* stk = po_stack + threadIdx.x;
    using Smp = FirstSampler<T, K, VEC, NL, V>;
    Smp smp;
    Ray r;
    int want = 0, steps = 0;
    if (valid) {
        double ro[3], rd[3];
        ray_of<SRC>(J, S, idx, ro, rd);
        double s_lo = 0.0, s_hi = 1e300;
        if constexpr (V == PO_FWD_VIEW) clip_range(op, ro, rd, s_lo, s_hi);
        if (ray_setup(tr, ro, rd, r, s_lo, s_hi)) {
            const double s_first = r.s;
            fwd_init<T, K, V>(smp, tr, op, r);
            steps = march<Smp, true>(tr, r, min(S.split_steps, op.max_steps), stk, smp);
            if (r.more) {
                if (steps >= op.max_steps)
                    atomicAdd(&g_po_errors, 1ull);  // the step cap proper
                else
                    want = pieces_wanted(r, s_first, steps, S, S.chunk_steps);
            }
        }
    }
    const int h = claim_pieces(S.count, S.info, claim_region(), want, S.region_slots);
    bool handed = false;
    if (want > 0) {
        if (h >= 0) {
            ContHead hd;
            hd.s = r.s;
            hd.T = smp.Tl;
            hd.c0 = smp.c0;
            hd.c1 = smp.c1;
            hd.c2 = smp.c2;
            hd.pix = idx;
            hd.pad = 0;
            reinterpret_cast<ContHead*>(S.head)[h] = hd;
            handed = true;
        } else {
            steps += march<Smp>(tr, r, op.max_steps - steps, stk, smp);  // region full: finish here
        }
    }
    const size_t p = (size_t)idx;
    if constexpr (SRC == 1) {
        // a kept render records which rays it handed on, for its backward
        if (valid && S.ray_slot) S.ray_slot[p] = handed ? h : -1;
    }
    if (valid && !handed) {
        J.rgb[3 * p + 0] = fmaf(smp.Tl, op.bg[0], smp.c0);
        J.rgb[3 * p + 1] = fmaf(smp.Tl, op.bg[1], smp.c1);
        J.rgb[3 * p + 2] = fmaf(smp.Tl, op.bg[2], smp.c2);
    }
    if constexpr (V == PO_FWD_VIEW) {
        // aux of a handed-on ray: the first walk's counts and depth, which
        // the join completes
        if (valid && J.aux) {
            J.aux[4 * p + 0] = smp.Tl;
            J.aux[4 * p + 1] = (float)smp.ns;
            J.aux[4 * p + 2] = (float)steps;
            J.aux[4 * p + 3] = smp.dep;
        }
    }
}

template <typename T, int K, int VEC, int NL, int V>
__global__ __launch_bounds__(kBlock) void k_render_camera_split(KBatch<1> B, KSplit S) {
    const int64_t b = xcd_interleave(blockIdx.x, B.n_blocks, 4 * B.job[0].tiles_x);
    if (b < 0) return;
    const KJob& J = B.job[0];
    const int q = (int)b;
    const int tile = J.tile_begin + (q >> 2), quad = q & 3;
    const int tx = tile % J.tiles_x, ty = tile / J.tiles_x;
    const int lane = threadIdx.x;
    const int px = tx * 16 + (quad & 1) * 8 + (lane & 7);
    const int py = ty * 16 + (quad >> 1) * 8 + (lane >> 3);
    const bool valid = (px < J.cam.W) & (py < J.cam.H);
    first_walk<T, K, VEC, NL, V, 0>(J, S, valid ? py * J.cam.W + px : 0, valid);
}

template <typename T, int K, int VEC, int NL, int V>
__global__ __launch_bounds__(kBlock) void k_render_rays_split(KBatch<1> B, KSplit S) {
    const int64_t b = xcd_swizzle(blockIdx.x, B.n_blocks);
    if (b < 0) return;
    const int64_t i = b * kBlock + threadIdx.x;
    const bool valid = i < S.n_rays;
    first_walk<T, K, VEC, NL, V, 1>(B.job[0], S, valid ? (int)i : 0, valid);
}

__global__ void k_zero_i32(int32_t* __restrict__ p, int n) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) p[i] = 0;
}

// Queue slot of this thread (workgroup blockIdx.x - first, first a multiple
// of 8), or -1 past the claimed slots.  Workgroup b serves the regions of
// its own XCD x = b % 8, and within them consecutive workgroups take
// consecutive 64-slot blocks of the claimed slots, region after region
// (faster than interleaving the regions: 735 against 1035 us per depth-9
// frame).  The grid covers the queue's capacity, which the claims fill only
// in part: with the blocks of each region counted from its claims, the
// workgroups past the claimed blocks of all eight regions are the last ones
// dispatched and find nothing, instead of each region's empty blocks
// standing in the dispatch order in front of the next region's work.
__device__ __forceinline__ int split_slot(const int32_t* count, int region_slots, int first = 0) {
    const int b = (int)blockIdx.x - first;
    const int x = b & 7;
    int t = b >> 3;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int n = min(count[8 * x + i], region_slots);
        const int nb = (n + kBlock - 1) / kBlock;
        if (t < nb) {
            const int local = t * kBlock + (int)threadIdx.x;
            return local < n ? (8 * x + i) * region_slots + local : -1;
        }
        t -= nb;
    }
    return -1;
}

// The plain (SH, SG) chunk and sub-chunk walks of records up to 192 bytes
// are held to 128 VGPRs (4 waves per SIMD; unconstrained the float32 K=16
// chunk kernel takes 131 and 3 waves): 0.639 against 0.671 ms per depth-9
// 800x800 frame; float16 SH records of K <= 16 with the basis values in
// LDS, to 96 VGPRs (5 waves; 20 bytes of scratch outside the loop).  Larger
// records and the viewer and codebook variants would spill (K=25 float32:
// 180 bytes of scratch, half the frame rate; float16 K=25 at 5 waves: 144),
// so they keep 4 waves or their natural count.
template <typename T, int K, int V>
constexpr int kPieceWaves = (V == PO_FWD_SH || V == PO_FWD_SG) && sizeof(T) * 3 * K <= 192
                                ? (sizeof(T) == 2 && V == PO_FWD_SH && K <= 16 ? 5 : 4)
                                : 1;

template <typename T, int K, int VEC, int NL, int V, int SRC>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kPieceWaves<T, K, V>, 8))) void k_render_chunks(
    KBatch<1> B, KSplit S) {
    const int q = split_slot(S.count, S.region_slots);
    const int4 in = q < 0 ? make_int4(-1, 0, -1, 0) : S.info[q];
    const int h = in.x;
    const KJob& J = B.job[0];
    using Smp = ChunkSampler<T, K, VEC, NL, V>;
    Smp smp;
    Ray r;
    int want = 0, steps = 0, pix = 0;
    extern __shared__ int po_stack[];
    int* stk = po_stack + threadIdx.x;
    if (h >= 0) {
        const int mj = in.y;
        const ContHead hd = reinterpret_cast<const ContHead*>(S.head)[h];
        pix = hd.pix;
        if (piece_setup<SRC>(J, S, pix, hd.s, walk_end<V, SRC>(J, S, pix), mj & 255, mj >> 8, r)) {
            const double s_first = r.s;
            fwd_init<T, K, V>(smp, J.tr, J.op, r);
            steps = march<Smp, true>(J.tr, r, min(S.chunk_cap, J.op.max_steps), stk, smp);
            if (r.more) {
                if (steps >= J.op.max_steps) {
                    atomicAdd(&g_po_errors, 1ull);
                } else {
                    want = pieces_wanted(r, s_first, steps, S, S.sub_steps);
#ifdef PO_MIN_SUB
                    if (want < PO_MIN_SUB) {
                        march<Smp>(J.tr, r, J.op.max_steps - steps, stk, smp);
                        want = 0;
                    }
#endif
                }
            }
        }
    }
    int sub = claim_pieces(S.count2, S.info2, claim_region(), want, S.region_slots);
    if (want > 0) {
        if (sub >= 0) {
            SubHead sh;
            sh.lo = r.s;
            sh.hi = r.s_end;
            sh.pix = pix;
            sh.pad[0] = sh.pad[1] = sh.pad[2] = 0;
            reinterpret_cast<SubHead*>(S.head2)[sub] = sh;
        } else {
            steps += march<Smp>(J.tr, r, J.op.max_steps - steps, stk, smp);  // region full: finish here
            want = 0;
        }
    }
    if (h >= 0) {
        PieceOut o;
        o.c0 = smp.c0;
        o.c1 = smp.c1;
        o.c2 = smp.c2;
        o.T = smp.Tl;
        o.Tlast = smp.Tlast;
        o.sub = sub;
        o.n_sub = want;
        o.dep = smp.dep;
        reinterpret_cast<PieceOut*>(S.part)[q] = o;
        if constexpr (V == PO_FWD_VIEW)
            S.view_part[q] = make_int4(smp.ns, steps - smp.skip0, smp.smp_cut ? 1 : 0,
                                       (want == 0 && !smp.cpl) ? 1 : 0);
    }
}

template <typename T, int K, int VEC, int NL, int V, int SRC>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kPieceWaves<T, K, V>, 8))) void k_render_subchunks(
    KBatch<1> B, KSplit S) {
    const int q = split_slot(S.count2, S.region_slots);
    if (q < 0) return;
    const int4 in = S.info2[q];
    const int h = in.x;
    if (h < 0) return;
    const int mj = in.y;
    const SubHead sh = reinterpret_cast<const SubHead*>(S.head2)[h];
    const KJob& J = B.job[0];
    using Smp = ChunkSampler<T, K, VEC, NL, V>;
    Smp smp;
    Ray r;
    int steps = 0;
    if (piece_setup<SRC>(J, S, sh.pix, sh.lo, sh.hi, mj & 255, mj >> 8, r)) {
        fwd_init<T, K, V>(smp, J.tr, J.op, r);
        extern __shared__ int po_stack[];
        steps = march(J.tr, r, J.op.max_steps, po_stack + threadIdx.x, smp);
    }
    PieceOut o;
    o.c0 = smp.c0;
    o.c1 = smp.c1;
    o.c2 = smp.c2;
    o.T = smp.Tl;
    o.Tlast = smp.Tlast;
    o.sub = -1;
    o.n_sub = 0;
    o.dep = smp.dep;
    reinterpret_cast<PieceOut*>(S.part2)[q] = o;
    if constexpr (V == PO_FWD_VIEW)
        S.view_part2[q] = make_int4(smp.ns, steps - smp.skip0, smp.smp_cut ? 1 : 0, smp.cpl ? 0 : 1);
}

// Running state of a join: transmittance and colour in front, and for the
// viewer variant the depth integral, sample and cell counts, and whether the
// last piece joined ended in a cut cell (counted again by the next piece).
struct JoinAcc {
    float Tp;
    float c[3];
    float dep;
    int ns, steps, cut_smp, cut;
};

// Front-to-back join of one piece with result o: piece k of n of [a, hi]; a
// chunk whose remainder was handed on (o.n_sub > 0) ends where its remainder
// begins.  Returns true when early stopping ends the ray in this piece.
template <typename T, int K, int VEC, int NL, int V, int SRC>
__device__ __forceinline__ bool join_piece(const KJob& J, const KSplit& S, int pix, double a, double hi, int k,
                                           int n, const PieceOut& o, const int4* vp, JoinAcc& A) {
    if (o.Tlast >= 0.0f && A.Tp * o.Tlast < J.op.stop_T) {
        // the walk stops inside this piece: walk it again from Tp
        double lo, up;
        piece_bounds<SRC>(J, S, pix, a, hi, k, n, lo, up);
        if (o.n_sub > 0) up = reinterpret_cast<const SubHead*>(S.head2)[o.sub].lo;
        using Smp = ChunkSampler<T, K, VEC, NL, V>;
        Smp smp;
        smp.Tl = A.Tp;
        Ray r;
        int steps = 0;
        if (piece_setup<SRC>(J, S, pix, lo, up, 0, 1, r)) {
            fwd_init<T, K, V>(smp, J.tr, J.op, r);
            extern __shared__ int po_stack[];
            steps = march(J.tr, r, J.op.max_steps, po_stack + threadIdx.x, smp);
        }
        A.c[0] += smp.c0;
        A.c[1] += smp.c1;
        A.c[2] += smp.c2;
        A.Tp = smp.Tl;
        if constexpr (V == PO_FWD_VIEW) {
            A.dep += smp.dep;
            A.cut_smp = smp.hit ? 0 : (smp.smp_cut ? 1 : 0);
            A.cut = (smp.hit || o.n_sub > 0 || smp.cpl) ? 0 : 1;
            A.ns += smp.ns - A.cut_smp;
            A.steps += steps - smp.skip0 - A.cut;
        }
        // (rounding can leave T just above stop_T; then the later pieces still count)
        return smp.hit;
    }
    A.c[0] = fmaf(A.Tp, o.c0, A.c[0]);
    A.c[1] = fmaf(A.Tp, o.c1, A.c[1]);
    A.c[2] = fmaf(A.Tp, o.c2, A.c[2]);
    if constexpr (V == PO_FWD_VIEW) {
        const int4 c = *vp;  // ns, steps, cut_smp, cut
        A.dep = fmaf(A.Tp, o.dep, A.dep);
        A.ns += c.x - c.z;
        A.steps += c.y - c.w;
        A.cut_smp = c.z;
        A.cut = c.w;
    }
    A.Tp = A.Tp * o.T;
    return false;
}

template <typename T, int K, int VEC, int NL, int V, int SRC>
__global__ __launch_bounds__(kBlock) void k_render_join(KBatch<1> B, KSplit S) {
    const int q = split_slot(S.count, S.region_slots);
    if (q < 0) return;
    const int4 in = S.info[q];
    if (in.x != q) return;  // not the first slot of a ray
    const int m = in.y >> 8;
    const ContHead hd = reinterpret_cast<const ContHead*>(S.head)[q];
    const KJob& J = B.job[0];
    PieceOut* part = reinterpret_cast<PieceOut*>(S.part);
    PieceOut* part2 = reinterpret_cast<PieceOut*>(S.part2);
    const SubHead* head2 = reinterpret_cast<const SubHead*>(S.head2);
    const size_t p = (size_t)hd.pix;
    // the join of a kept ray-list render also writes, over each piece's
    // result, the transmittance and colour prefix in front of it and whether
    // it lies before the early stop (Tlast 1) or not (-1): the prefixes its
    // backward differentiates from (what k_piece_prefix computes otherwise)
    bool keep = false;
    if constexpr (SRC == 1 && V != PO_FWD_VIEW) keep = S.ray_slot != nullptr;
    JoinAcc A;
    auto prefix = [&](PieceOut* rec, PieceOut o, bool past) {
        o.c0 = A.c[0];
        o.c1 = A.c[1];
        o.c2 = A.c[2];
        o.T = A.Tp;
        o.Tlast = past ? -1.0f : 1.0f;
        *rec = o;
    };
    A.Tp = hd.T;
    A.c[0] = hd.c0;
    A.c[1] = hd.c1;
    A.c[2] = hd.c2;
    A.dep = 0.0f;
    A.ns = A.steps = A.cut_smp = A.cut = 0;
    if constexpr (V == PO_FWD_VIEW) {
        if (J.aux) {
            A.ns = (int)J.aux[4 * p + 1];
            A.steps = (int)J.aux[4 * p + 2];
            A.dep = J.aux[4 * p + 3];
        }
    }
    const double end = walk_end<V, SRC>(J, S, hd.pix);
    bool done = false;
    int qj = q;
    for (int j = 0; j < m && (keep || !done); ++j) {
        const PieceOut o = part[qj];
        const int qo = qj;
        qj = S.info[qj].z;
        if (keep) prefix(part + qo, o, done);
        if (!done) done = join_piece<T, K, VEC, NL, V, SRC>(J, S, hd.pix, hd.s, end, j, m, o, S.view_part + qo, A);
        if (o.n_sub > 0 && (keep || !done)) {
            // the remainder's sub-chunks (bounds read only to walk one again)
            double slo = 0.0, shi = 0.0;
            int qk = o.sub;
            for (int k = 0; k < o.n_sub && (keep || !done); ++k) {
                const PieceOut o2 = part2[qk];
                const int qo2 = qk;
                qk = S.info2[qk].z;
                if (keep) prefix(part2 + qo2, o2, done);
                if (done) continue;
                if (o2.Tlast >= 0.0f && A.Tp * o2.Tlast < J.op.stop_T && shi == 0.0) {
                    const SubHead sh = head2[o.sub];
                    slo = sh.lo;
                    shi = sh.hi;
                }
                done = join_piece<T, K, VEC, NL, V, SRC>(J, S, hd.pix, slo, shi, k, o.n_sub, o2, S.view_part2 + qo2,
                                                         A);
            }
        }
    }
    J.rgb[3 * p + 0] = fmaf(A.Tp, J.op.bg[0], A.c[0]);
    J.rgb[3 * p + 1] = fmaf(A.Tp, J.op.bg[1], A.c[1]);
    J.rgb[3 * p + 2] = fmaf(A.Tp, J.op.bg[2], A.c[2]);
    if constexpr (V == PO_FWD_VIEW) {
        if (J.aux) {
            // the last piece's cut cell (at the slicing plane) has no next piece
            J.aux[4 * p + 0] = A.Tp;
            J.aux[4 * p + 1] = (float)(A.ns + A.cut_smp);
            J.aux[4 * p + 2] = (float)(A.steps + A.cut);
            J.aux[4 * p + 3] = A.dep;
        }
    }
}

// Gradient of one ray's samples (App. B.3): the forward colour C is the
// first pass; this second pass keeps the prefix P_i of w_k c_k, so that
// dC/dsigma_i = delta_i (c_i T_{i+1} - (C - P_i)) (zero where the raw density
// is <= 0) and dC/dk = w_i c_i (1 - c_i) Y, contracted with dL/dC and added
// to the leaf gradients with float atomics.  The density gradient is added
// by its own lane; the 3K coefficient gradients of the wave's samples are
// staged in LDS and added cooperatively (flush), so that one atomic
// instruction covers one or two records instead of 64 scattered ones.
template <int K, int VEC, int NL>
struct BwdSampler {
    static constexpr int NW = Words<float, NL>::N;
    static constexpr bool kClip = false;
    static constexpr int NE = 3 * K;
    static constexpr int SW = (NE + 3) / 4 * 4;  // LDS slot: one sample's products
    __amdgpu_buffer_rsrc_t sig, shb;
    uint32_t sig_end, sh_end, rec_bytes;
    int stride;
    float stopT;
    float Y[K];
    float g0, g1, g2, C0, C1, C2;
    float* gsig;
    float* gsh;
    float* sprod;
    int* sleaf;
    float Tl = 1.0f, P0 = 0.0f, P1 = 0.0f, P2 = 0.0f;
    bool has = false;
    float z0, z1, z2;
    // in flight
    int leaf;
    float raw, delta;
    uint32_t w[NW];

    __device__ __forceinline__ void issue(int l, float d, float) {
        leaf = l;
        raw = sigma_buf(sig, l < 0 ? sig_end : (uint32_t)l * 4u, (float*)nullptr);
        load_words_buf<float, NL, VEC>(shb, l < 0 ? sh_end : (uint32_t)l * rec_bytes, w);
        delta = d;
    }
    __device__ __forceinline__ bool consume() {
        const float s = fmaxf(raw, 0.0f);
        if (!(s > 0.0f)) return false;  // no density: zero weight, and dC/dsigma is masked
        const float ex = __expf(-(s * delta));
        const float wgt = Tl * (1.0f - ex);
        const float Tn = Tl * ex;
        const float c0 = sigmoid(dot_channel<float, K>(w, 0, Y));
        const float c1 = sigmoid(dot_channel<float, K>(w, K, Y));
        const float c2 = sigmoid(dot_channel<float, K>(w, 2 * K, Y));
        P0 = fmaf(wgt, c0, P0);
        P1 = fmaf(wgt, c1, P1);
        P2 = fmaf(wgt, c2, P2);
        float gs = g0 * (c0 * Tn - (C0 - P0));
        gs = fmaf(g1, c1 * Tn - (C1 - P1), gs);
        gs = fmaf(g2, c2 * Tn - (C2 - P2), gs);
        atomicAdd(gsig + leaf, gs * delta);
        z0 = g0 * wgt * c0 * (1.0f - c0);
        z1 = g1 * wgt * c1 * (1.0f - c1);
        z2 = g2 * wgt * c2 * (1.0f - c2);
        has = true;
        Tl = Tn;
        return Tl < stopT;
    }
    // Runs with every lane still walking: the lanes that composited a sample
    // write its 3K coefficient gradients to consecutive LDS slots, then all
    // active lanes add them to the leaves, consecutive lanes taking
    // consecutive coefficients of a record.
    __device__ __forceinline__ void flush() {
        const uint64_t m = __ballot(has);
        if (m == 0) return;
        if (has) {
            const int slot = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            float* dst = sprod + slot * SW;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                dst[k] = z0 * Y[k];
                dst[K + k] = z1 * Y[k];
                dst[2 * K + k] = z2 * Y[k];
            }
            sleaf[slot] = leaf;
            has = false;
        }
        __builtin_amdgcn_wave_barrier();
        const uint64_t act = __ballot(1);
        const int na = __popcll(act);
        const int r = __builtin_amdgcn_mbcnt_hi((uint32_t)(act >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)act, 0u));
        const int total = __popcll(m) * SW;
        for (int it = r; it < total; it += na) {
            const int j = it / SW, e = it - j * SW;
            if (e < NE) atomicAdd(gsh + (size_t)sleaf[j] * stride + e, sprod[it]);
        }
        __builtin_amdgcn_wave_barrier();
    }
};

// Backward kernel: replays the forward walk of each ray.
template <int K, int VEC, int NL>
__global__ __launch_bounds__(kBlock) void k_backward(KTree tr, int64_t n, int64_t n_blocks,
                                                     const float* __restrict__ o,
                                                     const float* __restrict__ d, KOpts op,
                                                     const float* __restrict__ rgb_fwd,
                                                     const float* __restrict__ grad,
                                                     float* __restrict__ gsig, float* __restrict__ gsh) {
    const int64_t blk = xcd_swizzle(blockIdx.x, n_blocks);
    if (blk < 0) return;
    const int64_t i = blk * kBlock + threadIdx.x;
    if (i >= n) return;
    const double ro[3] = {(double)o[3 * i], (double)o[3 * i + 1], (double)o[3 * i + 2]};
    const double rd[3] = {(double)d[3 * i], (double)d[3 * i + 1], (double)d[3 * i + 2]};
    Ray r;
    if (!ray_setup(tr, ro, rd, r)) return;
    BwdSampler<K, VEC, NL> smp;
    smp.g0 = grad[3 * i];
    smp.g1 = grad[3 * i + 1];
    smp.g2 = grad[3 * i + 2];
    if (smp.g0 == 0.0f && smp.g1 == 0.0f && smp.g2 == 0.0f) return;
    smp.C0 = rgb_fwd[3 * i];
    smp.C1 = rgb_fwd[3 * i + 1];
    smp.C2 = rgb_fwd[3 * i + 2];
    smp.sig = raw_rsrc(tr.sigma, tr.sigma_bytes);
    smp.shb = raw_rsrc(tr.sh, tr.sh_bytes);
    smp.sig_end = tr.sigma_bytes;
    smp.sh_end = tr.sh_bytes;
    smp.rec_bytes = (uint32_t)tr.stride * 4u;
    smp.stride = tr.stride;
    smp.stopT = op.stop_T;
    smp.gsig = gsig;
    smp.gsh = gsh;
    __shared__ float s_prod[kBlock * BwdSampler<K, VEC, NL>::SW];
    __shared__ int s_leaf[kBlock];
    smp.sprod = s_prod;
    smp.sleaf = s_leaf;
    colour_basis<K>(tr, r.dn[0], r.dn[1], r.dn[2], smp.Y);
    extern __shared__ int po_stack[];
    march(tr, r, op.max_steps, po_stack + threadIdx.x, smp);
}

// ---------------------------------------------------------------------------
// Split backward.  The gradient of a ray's pieces needs, at the start of each
// piece, the transmittance T and the colour prefix P = sum of w_k c_k of
// everything in front of it (App. B.3: dC/dsigma_i = delta_i (c_i T_{i+1} -
// (C - P_i)), dC/dk = w_i c_i (1 - c_i) Y).  A piece that cuts a cell is a
// segment of its own: the two parts' gradients add up to the whole cell's.
//   k_backward_split      the backward of the first split_steps cells of
//                         every ray, which then hands the rest on as chunks
//                         (head state: s, T, P);
//   k_render_chunks,
//   k_render_subchunks    the forward of the pieces (colour and transmittance
//                         from T = 1), as in the split render;
//   k_piece_prefix        per ray, front to back: T and P at the start of
//                         every piece and which pieces lie before the early
//                         stop (the piece holding it walked again, as in the
//                         join), written over the piece's forward result;
//   k_backward_pieces     the backward of every piece before the stop, from
//                         its T and P (chunks, then sub-chunks).
// ---------------------------------------------------------------------------
template <int K, class Smp>
__device__ __forceinline__ void bwd_init(Smp& smp, const KTree& tr, const KOpts& op, const Ray& r, size_t i,
                                         const float* __restrict__ rgb_fwd, const float* __restrict__ grad,
                                         float* gsig, float* gsh, float* sprod, int* sleaf) {
    smp.g0 = grad[3 * i];
    smp.g1 = grad[3 * i + 1];
    smp.g2 = grad[3 * i + 2];
    smp.C0 = rgb_fwd[3 * i];
    smp.C1 = rgb_fwd[3 * i + 1];
    smp.C2 = rgb_fwd[3 * i + 2];
    smp.sig = raw_rsrc(tr.sigma, tr.sigma_bytes);
    smp.shb = raw_rsrc(tr.sh, tr.sh_bytes);
    smp.sig_end = tr.sigma_bytes;
    smp.sh_end = tr.sh_bytes;
    smp.rec_bytes = (uint32_t)tr.stride * 4u;
    smp.stride = tr.stride;
    smp.stopT = op.stop_T;
    smp.gsig = gsig;
    smp.gsh = gsh;
    smp.sprod = sprod;
    smp.sleaf = sleaf;
    colour_basis<K>(tr, r.dn[0], r.dn[1], r.dn[2], smp.Y);
}

template <int K, int VEC, int NL>
__global__ __launch_bounds__(kBlock) void k_backward_split(KBatch<1> B, KSplit S, const float* __restrict__ rgb_fwd,
                                                           const float* __restrict__ grad, float* __restrict__ gsig,
                                                           float* __restrict__ gsh) {
    const int64_t b = xcd_swizzle(blockIdx.x, B.n_blocks);
    if (b < 0) return;
    const int64_t i = b * kBlock + threadIdx.x;
    const KJob& J = B.job[0];
    const KTree& tr = J.tr;
    using Smp = BwdSampler<K, VEC, NL>;
    Smp smp;
    __shared__ float s_prod[kBlock * Smp::SW];
    __shared__ int s_leaf[kBlock];
    extern __shared__ int po_stack[];
    int* stk = po_stack + threadIdx.x;
    Ray r;
    int want = 0, steps = 0;
    bool live = false;
    if (i < S.n_rays) {
        double ro[3], rd[3];
        ray_of<1>(J, S, (int)i, ro, rd);
        if (ray_setup(tr, ro, rd, r)) {
            bwd_init<K>(smp, tr, J.op, r, (size_t)i, rgb_fwd, grad, gsig, gsh, s_prod, s_leaf);
            live = !(smp.g0 == 0.0f && smp.g1 == 0.0f && smp.g2 == 0.0f);
        }
    }
    if (live) {
        const double s_first = r.s;
        steps = march<Smp, true>(tr, r, min(S.split_steps, J.op.max_steps), stk, smp);
        if (r.more) {
            if (steps >= J.op.max_steps)
                atomicAdd(&g_po_errors, 1ull);
            else
                want = pieces_wanted(r, s_first, steps, S, S.chunk_steps);
        }
    }
    const int h = claim_pieces(S.count, S.info, claim_region(), want, S.region_slots);
    if (want > 0) {
        if (h >= 0) {
            ContHead hd;
            hd.s = r.s;
            hd.T = smp.Tl;
            hd.c0 = smp.P0;
            hd.c1 = smp.P1;
            hd.c2 = smp.P2;
            hd.pix = (int)i;
            hd.pad = 0;
            reinterpret_cast<ContHead*>(S.head)[h] = hd;
        } else {
            march<Smp>(tr, r, J.op.max_steps - steps, stk, smp);  // region full: finish here
        }
    }
}

// The backward's first walk over the rays of a kept render
// (po_render_rays_keep): the render's pieces, their heads (s, T and the
// colour prefix P after its first walk) and ray_slot stay in the queue, so
// a ray the render handed on is differentiated over the same first
// split_steps cells and its pieces are not walked forward again; a ray it
// did not hand on (ended within the first walk, or its region was full) is
// differentiated to its end here.
template <int K, int VEC, int NL>
__global__ __launch_bounds__(kBlock) void k_backward_first_kept(KBatch<1> B, KSplit S,
                                                                const float* __restrict__ rgb_fwd,
                                                                const float* __restrict__ grad,
                                                                float* __restrict__ gsig, float* __restrict__ gsh) {
    const int64_t b = xcd_swizzle(blockIdx.x, B.n_blocks);
    if (b < 0) return;
    const int64_t i = b * kBlock + threadIdx.x;
    const KJob& J = B.job[0];
    const KTree& tr = J.tr;
    using Smp = BwdSampler<K, VEC, NL>;
    Smp smp;
    __shared__ float s_prod[kBlock * Smp::SW];
    __shared__ int s_leaf[kBlock];
    extern __shared__ int po_stack[];
    Ray r;
    bool live = false, handed = false;
    if (i < S.n_rays) {
        double ro[3], rd[3];
        ray_of<1>(J, S, (int)i, ro, rd);
        if (ray_setup(tr, ro, rd, r)) {
            bwd_init<K>(smp, tr, J.op, r, (size_t)i, rgb_fwd, grad, gsig, gsh, s_prod, s_leaf);
            live = !(smp.g0 == 0.0f && smp.g1 == 0.0f && smp.g2 == 0.0f);
            handed = S.ray_slot[i] >= 0;
        }
    }
    if (live) {
        const int cap = handed ? min(S.split_steps, J.op.max_steps) : J.op.max_steps;
        const int steps = march<Smp, true>(tr, r, cap, po_stack + threadIdx.x, smp);
        if (r.more & (steps >= J.op.max_steps)) atomicAdd(&g_po_errors, 1ull);  // the step cap proper
    }
}

// Prefix of one piece: its forward result o is replaced by (P, T) in front
// of it and whether it lies before the early stop (Tlast 1) or not (-1).
template <int K, int VEC, int NL, int V>
__device__ __forceinline__ void prefix_piece(const KJob& J, const KSplit& S, int pix, double a, double hi, int k,
                                             int n, PieceOut* rec, float& Tp, float (&P)[3], bool& done) {
    const PieceOut o = *rec;
    PieceOut w = o;
    w.c0 = P[0];
    w.c1 = P[1];
    w.c2 = P[2];
    w.T = Tp;
    w.Tlast = done ? -1.0f : 1.0f;
    *rec = w;
    if (!done) {
        JoinAcc A;
        A.Tp = Tp;
        A.c[0] = P[0];
        A.c[1] = P[1];
        A.c[2] = P[2];
        A.dep = 0.0f;
        A.ns = A.steps = A.cut_smp = A.cut = 0;
        done = join_piece<float, K, VEC, NL, V, 1>(J, S, pix, a, hi, k, n, o, nullptr, A);
        Tp = A.Tp;
        P[0] = A.c[0];
        P[1] = A.c[1];
        P[2] = A.c[2];
    }
}

template <int K, int VEC, int NL, int V>
__global__ __launch_bounds__(kBlock) void k_piece_prefix(KBatch<1> B, KSplit S) {
    const int q = split_slot(S.count, S.region_slots);
    if (q < 0) return;
    const int4 in = S.info[q];
    if (in.x != q) return;
    const int m = in.y >> 8;
    const ContHead hd = reinterpret_cast<const ContHead*>(S.head)[q];
    const KJob& J = B.job[0];
    PieceOut* part = reinterpret_cast<PieceOut*>(S.part);
    PieceOut* part2 = reinterpret_cast<PieceOut*>(S.part2);
    const SubHead* head2 = reinterpret_cast<const SubHead*>(S.head2);
    float Tp = hd.T;
    float P[3] = {hd.c0, hd.c1, hd.c2};
    bool done = false;
    int qj = q;
    for (int j = 0; j < m; ++j) {
        const int n_sub = part[qj].n_sub, sub = part[qj].sub;
        prefix_piece<K, VEC, NL, V>(J, S, hd.pix, hd.s, 1e300, j, m, part + qj, Tp, P, done);
        if (n_sub > 0) {
            const SubHead sh = head2[sub];
            int qk = sub;
            for (int k = 0; k < n_sub; ++k) {
                prefix_piece<K, VEC, NL, V>(J, S, hd.pix, sh.lo, sh.hi, k, n_sub, part2 + qk, Tp, P, done);
                qk = S.info2[qk].z;
            }
        }
        qj = S.info[qj].z;
    }
}

// The first kSplitRegions * region_slots / kBlock workgroups take the walked parts of the
// chunks, the others the sub-chunks: the two sets are independent once their
// prefixes are known, so one launch overlaps their tails.
template <int K, int VEC, int NL>
__global__ __launch_bounds__(kBlock) void k_backward_pieces(KBatch<1> B, KSplit S, const float* __restrict__ rgb_fwd,
                                                            const float* __restrict__ grad, float* __restrict__ gsig,
                                                            float* __restrict__ gsh) {
    const int half = kSplitRegions * (S.region_slots / kBlock);
    const bool sub = blockIdx.x >= (unsigned)half;
    const int q = split_slot(sub ? S.count2 : S.count, S.region_slots, sub ? half : 0);
    if (q < 0) return;
    const int4 in = (sub ? S.info2 : S.info)[q];
    if (in.x < 0) return;
    const PieceOut o = reinterpret_cast<const PieceOut*>(sub ? S.part2 : S.part)[q];
    if (o.Tlast < 0.0f) return;  // behind the early stop
    const KJob& J = B.job[0];
    const int k = in.y & 255, n = in.y >> 8;
    int idx;
    Ray r;
    bool ok;
    if (sub) {
        const SubHead sh = reinterpret_cast<const SubHead*>(S.head2)[in.x];
        idx = sh.pix;
        ok = piece_setup<1>(J, S, idx, sh.lo, sh.hi, k, n, r);
    } else {
        const ContHead hd = reinterpret_cast<const ContHead*>(S.head)[in.x];
        idx = hd.pix;
        double lo, up;
        piece_bounds<1>(J, S, idx, hd.s, 1e300, k, n, lo, up);
        if (o.n_sub > 0) up = reinterpret_cast<const SubHead*>(S.head2)[o.sub].lo;
        ok = piece_setup<1>(J, S, idx, lo, up, 0, 1, r);
    }
    if (!ok) return;
    using Smp = ChunkOf<BwdSampler<K, VEC, NL>>;
    Smp smp;
    __shared__ float s_prod[kBlock * BwdSampler<K, VEC, NL>::SW];
    __shared__ int s_leaf[kBlock];
    bwd_init<K>(smp, J.tr, J.op, r, (size_t)idx, rgb_fwd, grad, gsig, gsh, s_prod, s_leaf);
    if (smp.g0 == 0.0f && smp.g1 == 0.0f && smp.g2 == 0.0f) return;  // (a kept render's rays without gradient)
    smp.Tl = o.T;
    smp.P0 = o.c0;
    smp.P1 = o.c1;
    smp.P2 = o.c2;
    extern __shared__ int po_stack[];
    march(J.tr, r, J.op.max_steps, po_stack + threadIdx.x, smp);
}

// Visibility filter of the conversion (Sec. 4.2, "Filtering"): alpha
// renders of a camera that raise every leaf's weight to the largest weight
// of a segment in it, MODE 0 the segment's alpha 1 - exp(-sigma delta),
// MODE 1 its contribution T alpha.  Only the densities are gathered.  The
// weights are non-negative floats, whose bit patterns order like unsigned
// integers, so the maximum is an integer atomic.
template <typename T, int MODE>
struct WeightSampler {
    static constexpr bool kClip = false;
    __amdgpu_buffer_rsrc_t sig;
    uint32_t sig_end;
    float stopT;
    unsigned* wt;
    float Tl = 1.0f;
    // in flight
    int leaf;
    float raw, delta;

    __device__ __forceinline__ void issue(int l, float d, float) {
        leaf = l;
        raw = sigma_buf(sig, l < 0 ? sig_end : (uint32_t)l * (uint32_t)sizeof(T), (T*)nullptr);
        delta = d;
    }
    __device__ __forceinline__ void flush() {}
    __device__ __forceinline__ bool consume() {
        const float s = fmaxf(raw, 0.0f);
        if (!(s > 0.0f)) return false;
        const float ex = __expf(-(s * delta));
        const float al = 1.0f - ex;
        const float w = MODE ? Tl * al : al;
        if (w > 0.0f) atomicMax(wt + leaf, __float_as_uint(w));
        Tl = Tl * ex;
        return Tl < stopT;
    }
};

// One camera, 16x16 tiles of four 8x8 single-wave workgroups as in
// k_render_camera; alpha (or nullptr) receives 1 - T per pixel.
template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void k_leaf_weights(KTree tr, KCam cam, KOpts op, int n_blocks,
                                                         unsigned* __restrict__ wt, float* __restrict__ alpha) {
    const int tiles_x = (cam.W + 15) / 16;
    const int64_t b = xcd_interleave(blockIdx.x, n_blocks, 4 * (int64_t)tiles_x);
    if (b < 0) return;
    const int tile = (int)(b >> 2), quad = (int)(b & 3);
    const int lane = threadIdx.x;
    const int px = (tile % tiles_x) * 16 + (quad & 1) * 8 + (lane & 7);
    const int py = (tile / tiles_x) * 16 + (quad >> 1) * 8 + (lane >> 3);
    if (px >= cam.W || py >= cam.H) return;
    double ro[3], rd[3];
    pixel_ray(cam, px, py, ro, rd);
    float Tr = 1.0f;
    Ray r;
    if (ray_setup(tr, ro, rd, r)) {
        WeightSampler<T, MODE> smp;
        smp.sig = raw_rsrc(tr.sigma, tr.sigma_bytes);
        smp.sig_end = tr.sigma_bytes;
        smp.stopT = op.stop_T;
        smp.wt = wt;
        extern __shared__ int po_stack[];
        march(tr, r, op.max_steps, po_stack + threadIdx.x, smp);
        Tr = smp.Tl;
    }
    if (alpha) alpha[(size_t)py * cam.W + px] = 1.0f - Tr;
}

// Traversal statistics of a camera render: the plain walk with a sampler
// that gathers only the densities (the early stop depends on nothing else;
// its transmittance arithmetic is the render's, so it stops at the same
// sample) and counts, per ray, the data samples (segments of positive length
// in data leaves, as the aux output counts them), the cells visited and the
// child entries read from memory.  Sums over the image go to sums[4] =
// {rays, samples, cells, child-entry loads}, one atomic per wave and counter.
template <typename T>
struct StatSampler {
    static constexpr bool kClip = false;
    static constexpr bool kCountLoads = true;
    __amdgpu_buffer_rsrc_t sig;
    uint32_t sig_end;
    float stopT;
    float Tl = 1.0f;
    int ns = 0;
    int loads = 0;
    // in flight
    float raw, delta;

    __device__ __forceinline__ void issue(int l, float d, float) {
        raw = sigma_buf(sig, l < 0 ? sig_end : (uint32_t)l * (uint32_t)sizeof(T), (T*)nullptr);
        delta = d;
    }
    __device__ __forceinline__ void flush() {}
    __device__ __forceinline__ bool consume() {
        ++ns;
        const float s = fmaxf(raw, 0.0f);
        if (!(s > 0.0f)) return false;
        Tl = Tl * __expf(-(s * delta));
        return Tl < stopT;
    }
};

// SRC 0: the pixel rays of cam (16x16 tiles of four 8x8 waves); SRC 1: the
// n rays (o, d), 64 per wave.
template <typename T, int SRC>
__global__ __launch_bounds__(kBlock) void k_traversal_stats(KTree tr, KCam cam, const float* __restrict__ o,
                                                            const float* __restrict__ d, int64_t n, KOpts op,
                                                            int n_blocks, unsigned long long* __restrict__ sums) {
    const int64_t b = xcd_swizzle(blockIdx.x, n_blocks);
    if (b < 0) return;
    const int lane = threadIdx.x;
    bool valid;
    double ro[3], rd[3];
    if constexpr (SRC == 0) {
        const int tiles_x = (cam.W + 15) / 16;
        const int tile = (int)(b >> 2), quad = (int)(b & 3);
        const int px = (tile % tiles_x) * 16 + (quad & 1) * 8 + (lane & 7);
        const int py = (tile / tiles_x) * 16 + (quad >> 1) * 8 + (lane >> 3);
        valid = (px < cam.W) & (py < cam.H);
        if (valid) pixel_ray(cam, px, py, ro, rd);
    } else {
        const int64_t i = b * kBlock + lane;
        valid = i < n;
        if (valid) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                ro[k] = (double)o[3 * i + k];
                rd[k] = (double)d[3 * i + k];
            }
        }
    }
    unsigned long long v[4] = {valid ? 1ull : 0ull, 0ull, 0ull, 0ull};
    if (valid) {
        Ray r;
        if (ray_setup(tr, ro, rd, r)) {
            StatSampler<T> smp;
            smp.sig = raw_rsrc(tr.sigma, tr.sigma_bytes);
            smp.sig_end = tr.sigma_bytes;
            smp.stopT = op.stop_T;
            extern __shared__ int po_stack[];
            v[2] = (unsigned long long)march(tr, r, op.max_steps, po_stack + threadIdx.x, smp);
            v[1] = (unsigned long long)smp.ns;
            v[3] = (unsigned long long)smp.loads;
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        unsigned long long x = v[k];
        for (int o = kBlock / 2; o >= 1; o >>= 1) x += __shfl_xor(x, o);
        if (lane == 0 && x != 0ull) atomicAdd(sums + k, x);
    }
}

// Loss gradient of the NeRF loss (Sec. 3, eqn:nerfloss) for one batch: one
// thread per ray; squared errors are summed within the wave and added once
// per wave.
// Grid-stride over the rays; the squared errors are summed per workgroup
// (waves, then LDS) and added with one float atomic per workgroup: one
// atomic per wave on the single sum address serialised in L2 (15 us for
// 65536 rays).
__global__ __launch_bounds__(256) void k_mse_grad(int64_t n, const float* __restrict__ rgb,
                                                  const float* __restrict__ target, float scale,
                                                  float* __restrict__ grad, float* __restrict__ sq_sum) {
    float e2 = 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float e = rgb[3 * i + c] - target[3 * i + c];
            grad[3 * i + c] = scale * (2.0f * e);
            e2 = fmaf(e, e, e2);
        }
    }
    for (int off = 32; off > 0; off >>= 1) e2 += __shfl_xor(e2, off, 64);
    __shared__ float part[4];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = e2;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float t = (part[0] + part[1]) + (part[2] + part[3]);
        if (t != 0.0f) atomicAdd(sq_sum, t);
    }
}

// Batch rows of a training step: three rows of 3 floats per ray.
__global__ __launch_bounds__(256) void k_gather_rays(int64_t n, const int64_t* __restrict__ idx, int64_t n_src,
                                                     const float* __restrict__ o, const float* __restrict__ d,
                                                     const float* __restrict__ t, float* __restrict__ bo,
                                                     float* __restrict__ bd, float* __restrict__ bt) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int64_t j = idx[i];
    const bool ok = (j >= 0) & (j < n_src);
    if (!ok) atomicAdd(&g_po_errors, 1ull);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        bo[3 * i + c] = ok ? o[3 * j + c] : 0.0f;
        bd[3 * i + c] = ok ? d[3 * j + c] : 0.0f;
        bt[3 * i + c] = ok ? t[3 * j + c] : 0.0f;
    }
}

// A training batch drawn on the device: element `first + i` of the SplitMix64
// sequence of `seed` (Steele, Lea and Flood, "Fast splittable pseudorandom
// number generators", OOPSLA 2014: the state advances by the golden-ratio
// increment and each output is the state passed through the variant-13
// finaliser) picks row floor(z * n_src / 2^64), and the three rows are
// gathered.  Thread 0 also clears the loss accumulator of the batch.
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__global__ __launch_bounds__(256) void k_draw_batch(int64_t n, uint64_t seed, uint64_t first, int64_t n_src,
                                                    const float* __restrict__ o, const float* __restrict__ d,
                                                    const float* __restrict__ t, float* __restrict__ bo,
                                                    float* __restrict__ bd, float* __restrict__ bt,
                                                    float* __restrict__ sq_sum) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    if (i == 0 && sq_sum) sq_sum[0] = 0.0f;
    const int64_t j = (int64_t)__umul64hi(splitmix64(seed, first + (uint64_t)i), (uint64_t)n_src);
    for (int c = 0; c < 3; ++c) {
        bo[3 * i + c] = o[3 * j + c];
        bd[3 * i + c] = d[3 * j + c];
        bt[3 * i + c] = t[3 * j + c];
    }
}

// Plain SGD on the leaf values (Sec. 4.3): p -= lr g, optionally clearing g.
__global__ __launch_bounds__(256) void k_sgd(int64_t n, float* __restrict__ p, float* __restrict__ g, float lr,
                                             int zero_grad) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    p[i] = fmaf(-lr, gi, p[i]);
    if (zero_grad) g[i] = 0.0f;
}

inline int64_t grid_for(int64_t n_blocks) { return 8 * ((n_blocks + 7) / 8); }
// Grid of xcd_interleave over n_blocks logical workgroups in runs of chunk.
inline int64_t rows_grid(int64_t n_blocks, int64_t chunk) { return 8 * chunk * (((n_blocks + chunk - 1) / chunk + 7) / 8); }

// Dynamic LDS of the node stack: one int per lane and tree level.
inline size_t stack_bytes(int depth) { return sizeof(int) * kBlock * (size_t)depth; }

// Record-load plan: "fast" loads the padded record with the widest vectors,
// "generic" uses dword loads of exactly the record (rounded to whole dwords).
template <typename T, int K>
struct Plan {
    static constexpr int NE = 3 * K;
    static constexpr int FAST_VEC = (sizeof(T) == 4) ? 16 : ((NE * 2) % 16 == 0 ? 16 : 8);
    static constexpr int FAST_NL = ((NE * (int)sizeof(T) + FAST_VEC - 1) / FAST_VEC) * FAST_VEC / (int)sizeof(T);
    static constexpr int GEN_NL = (sizeof(T) == 2) ? ((NE + 1) / 2) * 2 : NE;
};

template <typename T, int K>
bool use_fast(const po_tree* t) {
    using P = Plan<T, K>;
    return t->vec_bytes >= P::FAST_VEC && t->stride >= P::FAST_NL &&
           ((size_t)t->stride * sizeof(T)) % P::FAST_VEC == 0;
}

// Load plan of codebook records: K 16-bit positions.
template <int K>
struct CbPlan {
    static constexpr int FAST_VEC = (2 * K) % 16 == 0 ? 16 : 8;
    static constexpr int FAST_NL = ((2 * K + FAST_VEC - 1) / FAST_VEC) * FAST_VEC / 2;
    static constexpr int GEN_NL = (K + 1) / 2 * 2;
};

template <int K>
bool use_fast_cb(const po_tree* t) {
    using P = CbPlan<K>;
    return t->vec_bytes >= P::FAST_VEC && t->stride >= P::FAST_NL && ((size_t)t->stride * 2) % P::FAST_VEC == 0;
}

template <typename T, int K>
hipError_t rays_t(const po_tree* t, int64_t n, const float* o, const float* d, const KOpts& op, float* rgb,
                  float* aux, hipStream_t s) {
    using P = Plan<T, K>;
    const int64_t nb = (n + kBlock - 1) / kBlock;
    dim3 grid((unsigned)grid_for(nb)), block(kBlock);
    const size_t lds = stack_bytes(t->kt.depth);
    const bool fast = use_fast<T, K>(t);
    const int v = po_fwd_variant(op, aux, t->kt);
    if (v != PO_FWD_VIEW) aux = nullptr;
    if constexpr (std::is_same_v<T, __half>) {
        if (v == PO_FWD_CB) {
            using Q = CbPlan<K>;
            if (use_fast_cb<K>(t))
                hipLaunchKernelGGL((k_render_rays<T, K, Q::FAST_VEC, Q::FAST_NL, PO_FWD_CB>), grid, block, lds, s,
                                   t->kt, n, nb, o, d, op, rgb, nullptr);
            else
                hipLaunchKernelGGL((k_render_rays<T, K, 4, Q::GEN_NL, PO_FWD_CB>), grid, block, lds, s, t->kt, n, nb,
                                   o, d, op, rgb, nullptr);
            return hipGetLastError();
        }
    }
#define PO_RAYS(V_)                                                                                              \
    do {                                                                                                        \
        if (fast)                                                                                               \
            hipLaunchKernelGGL((k_render_rays<T, K, P::FAST_VEC, P::FAST_NL, V_>), grid, block, lds, s, t->kt, n, \
                               nb, o, d, op, rgb, aux);                                                         \
        else                                                                                                    \
            hipLaunchKernelGGL((k_render_rays<T, K, 4, P::GEN_NL, V_>), grid, block, lds, s, t->kt, n, nb, o, d, \
                               op, rgb, aux);                                                                   \
    } while (0)
    if (v == PO_FWD_VIEW)
        PO_RAYS(PO_FWD_VIEW);
    else if (v == PO_FWD_SG)
        PO_RAYS(PO_FWD_SG);
    else
        PO_RAYS(PO_FWD_SH);
#undef PO_RAYS
    return hipGetLastError();
}

template <typename T, int K, int MAXJ>
hipError_t camera_t(const po_tree* t, int n_jobs, KJob* jobs, int n_blocks, int variant, hipStream_t s) {
    using P = Plan<T, K>;
    KBatch<MAXJ> B;
    for (int j = 0; j < n_jobs; ++j) B.job[j] = jobs[j];
    for (int j = n_jobs; j < MAXJ; ++j) B.job[j] = jobs[0];
    B.n_jobs = n_jobs;
    B.n_blocks = n_blocks;
    int depth = 1;
    for (int j = 0; j < n_jobs; ++j) depth = max(depth, jobs[j].tr.depth);
    dim3 grid((unsigned)(MAXJ == 1 ? rows_grid(n_blocks, 4 * (int64_t)jobs[0].tiles_x) : grid_for(n_blocks))),
        block(kBlock);
    const size_t lds = stack_bytes(depth);
    if constexpr (std::is_same_v<T, __half>) {
        if (variant == PO_FWD_CB) {
            using Q = CbPlan<K>;
            if (use_fast_cb<K>(t))
                hipLaunchKernelGGL((k_render_camera<T, K, Q::FAST_VEC, Q::FAST_NL, MAXJ, PO_FWD_CB>), grid, block, lds,
                                   s, B);
            else
                hipLaunchKernelGGL((k_render_camera<T, K, 4, Q::GEN_NL, MAXJ, PO_FWD_CB>), grid, block, lds, s, B);
            return hipGetLastError();
        }
    }
    const bool fast = use_fast<T, K>(t);
#define PO_CAM(V_)                                                                                               \
    do {                                                                                                        \
        if (fast)                                                                                               \
            hipLaunchKernelGGL((k_render_camera<T, K, P::FAST_VEC, P::FAST_NL, MAXJ, V_>), grid, block, lds, s, B); \
        else                                                                                                    \
            hipLaunchKernelGGL((k_render_camera<T, K, 4, P::GEN_NL, MAXJ, V_>), grid, block, lds, s, B);        \
    } while (0)
    if (variant == PO_FWD_VIEW)
        PO_CAM(PO_FWD_VIEW);
    else if (variant == PO_FWD_SG)
        PO_CAM(PO_FWD_SG);
    else
        PO_CAM(PO_FWD_SH);
#undef PO_CAM
    return hipGetLastError();
}

template <typename T, int K, int SRC>
hipError_t split_t(const po_tree* t, const KJob& job, int n_blocks, int variant, const KSplit& S, hipStream_t s) {
    using P = Plan<T, K>;
    KBatch<1> B;
    B.job[0] = job;
    B.n_jobs = 1;
    B.n_blocks = n_blocks;
    // counters cleared by a kernel rather than a memset node, so that the
    // launches can also be captured in a graph
    hipLaunchKernelGGL(k_zero_i32, dim3(2), dim3(kSplitRegions), 0, s, S.count, 2 * kSplitRegions);
    // camera: tile rows dealt over the XCDs (xcd_interleave)
    const int64_t g1n = SRC == 0 ? rows_grid(n_blocks, 4 * (int64_t)job.tiles_x) : grid_for(n_blocks);
    dim3 g1((unsigned)g1n), g2((unsigned)(kSplitRegions * (S.region_slots / kBlock))), blk(kBlock);
    const size_t lds = stack_bytes(job.tr.depth);
    const bool fast = use_fast<T, K>(t);
#define PO_SPLIT(VEC_, NL_, V_)                                                                        \
    do {                                                                                              \
        if constexpr (SRC == 0)                                                                       \
            hipLaunchKernelGGL((k_render_camera_split<T, K, VEC_, NL_, V_>), g1, blk, lds, s, B, S);  \
        else                                                                                          \
            hipLaunchKernelGGL((k_render_rays_split<T, K, VEC_, NL_, V_>), g1, blk, lds, s, B, S);    \
        hipLaunchKernelGGL((k_render_chunks<T, K, VEC_, NL_, V_, SRC>), g2, blk, lds, s, B, S);      \
        hipLaunchKernelGGL((k_render_subchunks<T, K, VEC_, NL_, V_, SRC>), g2, blk, lds, s, B, S);   \
        hipLaunchKernelGGL((k_render_join<T, K, VEC_, NL_, V_, SRC>), g2, blk, lds, s, B, S);        \
    } while (0)
    if constexpr (std::is_same_v<T, __half>) {
        if (variant == PO_FWD_CB) {
            using Q = CbPlan<K>;
            if (use_fast_cb<K>(t))
                PO_SPLIT(Q::FAST_VEC, Q::FAST_NL, PO_FWD_CB);
            else
                PO_SPLIT(4, Q::GEN_NL, PO_FWD_CB);
            return hipGetLastError();
        }
    }
    if (variant == PO_FWD_SG) {
        if (fast)
            PO_SPLIT(P::FAST_VEC, P::FAST_NL, PO_FWD_SG);
        else
            PO_SPLIT(4, P::GEN_NL, PO_FWD_SG);
    } else if (variant == PO_FWD_VIEW) {
        if (fast)
            PO_SPLIT(P::FAST_VEC, P::FAST_NL, PO_FWD_VIEW);
        else
            PO_SPLIT(4, P::GEN_NL, PO_FWD_VIEW);
    } else {
        if (fast)
            PO_SPLIT(P::FAST_VEC, P::FAST_NL, PO_FWD_SH);
        else
            PO_SPLIT(4, P::GEN_NL, PO_FWD_SH);
    }
#undef PO_SPLIT
    return hipGetLastError();
}

template <int K>
hipError_t backward_split_t(const po_tree* t, int64_t n, const float* o, const float* d, const KOpts& op,
                            const float* rgb_fwd, const float* grad, float* gsig, float* gsh, const KSplit& S0,
                            hipStream_t s) {
    using P = Plan<float, K>;
    KBatch<1> B;
    std::memset(&B, 0, sizeof B);
    B.job[0].tr = t->kt;
    B.job[0].op = op;
    B.n_jobs = 1;
    B.n_blocks = (int)((n + kBlock - 1) / kBlock);
    KSplit S = S0;
    S.ray_o = o;
    S.ray_d = d;
    S.n_rays = n;
    // the pieces of the render of the same rays (before the grids: they
    // cover the queue regions as this pass lays them out)
    po_rays_piece_sizes(n, &S);
    hipLaunchKernelGGL(k_zero_i32, dim3(2), dim3(kSplitRegions), 0, s, S.count, 2 * kSplitRegions);
    dim3 g1((unsigned)grid_for(B.n_blocks)), g2((unsigned)(kSplitRegions * (S.region_slots / kBlock))),
        g3(2u * g2.x), blk(kBlock);
    const size_t lds = stack_bytes(t->kt.depth);
    const bool sg = t->kt.lobes != nullptr;
#define PO_BSPLIT(VEC_, NL_)                                                                                    \
    do {                                                                                                       \
        hipLaunchKernelGGL((k_backward_split<K, VEC_, NL_>), g1, blk, lds, s, B, S, rgb_fwd, grad, gsig, gsh); \
        if (sg) {                                                                                              \
            hipLaunchKernelGGL((k_render_chunks<float, K, VEC_, NL_, PO_FWD_SG, 1>), g2, blk, lds, s, B, S);   \
            hipLaunchKernelGGL((k_render_subchunks<float, K, VEC_, NL_, PO_FWD_SG, 1>), g2, blk, lds, s, B, S); \
            hipLaunchKernelGGL((k_piece_prefix<K, VEC_, NL_, PO_FWD_SG>), g2, blk, lds, s, B, S);              \
        } else {                                                                                               \
            hipLaunchKernelGGL((k_render_chunks<float, K, VEC_, NL_, PO_FWD_SH, 1>), g2, blk, lds, s, B, S);   \
            hipLaunchKernelGGL((k_render_subchunks<float, K, VEC_, NL_, PO_FWD_SH, 1>), g2, blk, lds, s, B, S); \
            hipLaunchKernelGGL((k_piece_prefix<K, VEC_, NL_, PO_FWD_SH>), g2, blk, lds, s, B, S);              \
        }                                                                                                      \
        hipLaunchKernelGGL((k_backward_pieces<K, VEC_, NL_>), g3, blk, lds, s, B, S, rgb_fwd, grad, gsig, gsh);    \
    } while (0)
    if (use_fast<float, K>(t))
        PO_BSPLIT(P::FAST_VEC, P::FAST_NL);
    else
        PO_BSPLIT(4, P::GEN_NL);
#undef PO_BSPLIT
    return hipGetLastError();
}

// The backward of a kept render: its pieces are in the queue already, and
// its join wrote each piece's prefix over the piece's result, so neither
// the chunk and sub-chunk kernels nor k_piece_prefix run again, and the
// counters are not cleared.
template <int K>
hipError_t backward_kept_t(const po_tree* t, int64_t n, const float* o, const float* d, const KOpts& op,
                           const float* rgb_fwd, const float* grad, float* gsig, float* gsh, const KSplit& S0,
                           hipStream_t s) {
    using P = Plan<float, K>;
    KBatch<1> B;
    std::memset(&B, 0, sizeof B);
    B.job[0].tr = t->kt;
    B.job[0].op = op;
    B.n_jobs = 1;
    B.n_blocks = (int)((n + kBlock - 1) / kBlock);
    KSplit S = S0;
    S.ray_o = o;
    S.ray_d = d;
    S.n_rays = n;
    po_rays_piece_sizes(n, &S);
    dim3 g1((unsigned)grid_for(B.n_blocks)), g3(2u * (unsigned)(kSplitRegions * (S.region_slots / kBlock))),
        blk(kBlock);
    const size_t lds = stack_bytes(t->kt.depth);
#define PO_BKEPT(VEC_, NL_)                                                                                       \
    do {                                                                                                         \
        hipLaunchKernelGGL((k_backward_first_kept<K, VEC_, NL_>), g1, blk, lds, s, B, S, rgb_fwd, grad, gsig,    \
                           gsh);                                                                                 \
        hipLaunchKernelGGL((k_backward_pieces<K, VEC_, NL_>), g3, blk, lds, s, B, S, rgb_fwd, grad, gsig, gsh);  \
    } while (0)
    if (use_fast<float, K>(t))
        PO_BKEPT(P::FAST_VEC, P::FAST_NL);
    else
        PO_BKEPT(4, P::GEN_NL);
#undef PO_BKEPT
    return hipGetLastError();
}

template <int K>
hipError_t backward_t(const po_tree* t, int64_t n, const float* o, const float* d, const KOpts& op,
                      const float* rgb_fwd, const float* grad, float* gsig, float* gsh, hipStream_t s) {
    using P = Plan<float, K>;
    const int64_t nb = (n + kBlock - 1) / kBlock;
    dim3 grid((unsigned)grid_for(nb)), block(kBlock);
    if (use_fast<float, K>(t))
        hipLaunchKernelGGL((k_backward<K, P::FAST_VEC, P::FAST_NL>), grid, block, stack_bytes(t->kt.depth), s,
                           t->kt, n, nb, o, d, op, rgb_fwd, grad, gsig, gsh);
    else
        hipLaunchKernelGGL((k_backward<K, 4, P::GEN_NL>), grid, block, stack_bytes(t->kt.depth), s, t->kt, n, nb,
                           o, d, op, rgb_fwd, grad, gsig, gsh);
    return hipGetLastError();
}

}  // namespace

#define PO_DISPATCH_K(K_, EXPR)                      \
    switch (K_) {                                    \
        case 1: { constexpr int KK = 1; return EXPR; }   \
        case 4: { constexpr int KK = 4; return EXPR; }   \
        case 9: { constexpr int KK = 9; return EXPR; }   \
        case 16: { constexpr int KK = 16; return EXPR; } \
        case 25: { constexpr int KK = 25; return EXPR; } \
        default: return hipErrorInvalidValue;        \
    }

// Launchers of the parts, by leaf type (defined in the part named).
hipError_t po_camera_jobs_f32(const po_tree* first, int n_jobs, KJob* jobs, int n_blocks, int variant,
                              hipStream_t s);                                                   // part 1
hipError_t po_camera_jobs_f16(const po_tree* first, int n_jobs, KJob* jobs, int n_blocks, int variant,
                              hipStream_t s);                                                   // part 2
hipError_t po_camera_split_f32(const po_tree* t, const KJob& job, int n_blocks, int variant, const KSplit& S,
                               hipStream_t s);                                                  // part 3
hipError_t po_camera_split_f16(const po_tree* t, const KJob& job, int n_blocks, int variant, const KSplit& S,
                               hipStream_t s);                                                  // part 4
hipError_t po_rays_split_f32(const po_tree* t, const KJob& job, int n_blocks, int variant, const KSplit& S,
                             hipStream_t s);                                                    // part 5
hipError_t po_rays_split_f16(const po_tree* t, const KJob& job, int n_blocks, int variant, const KSplit& S,
                             hipStream_t s);                                                    // part 6
// Reads (and with reset, clears) part n's error counter; the device is synchronised by the caller.
#define PO_PART_ERRORS_DECL(n) hipError_t po_part_errors_##n(unsigned long long* out, bool reset);
PO_PART_ERRORS_DECL(0)
PO_PART_ERRORS_DECL(1)
PO_PART_ERRORS_DECL(2)
PO_PART_ERRORS_DECL(3)
PO_PART_ERRORS_DECL(4)
PO_PART_ERRORS_DECL(5)
PO_PART_ERRORS_DECL(6)
PO_PART_ERRORS_DECL(7)
#undef PO_PART_ERRORS_DECL

#define PO_PART_ERRORS_DEF(n)                                                                              \
    hipError_t po_part_errors_##n(unsigned long long* out, bool reset) {                                  \
        if (reset) {                                                                                       \
            const unsigned long long zero = 0ull;                                                          \
            return hipMemcpyToSymbol(HIP_SYMBOL(g_po_errors), &zero, sizeof(zero), 0, hipMemcpyHostToDevice); \
        }                                                                                                  \
        return hipMemcpyFromSymbol(out, HIP_SYMBOL(g_po_errors), sizeof(unsigned long long), 0,            \
                                   hipMemcpyDeviceToHost);                                                 \
    }

#if PO_PART == 1
PO_PART_ERRORS_DEF(1)
hipError_t po_camera_jobs_f32(const po_tree* first, int n_jobs, KJob* jobs, int n_blocks, int variant,
                              hipStream_t s) {
    if (n_jobs == 1) {
        PO_DISPATCH_K(first->K, (camera_t<float, KK, 1>(first, n_jobs, jobs, n_blocks, variant, s)));
    }
    PO_DISPATCH_K(first->K, (camera_t<float, KK, PO_BATCH_MAX_JOBS>(first, n_jobs, jobs, n_blocks, variant, s)));
}
#endif

#if PO_PART == 2
PO_PART_ERRORS_DEF(2)
hipError_t po_camera_jobs_f16(const po_tree* first, int n_jobs, KJob* jobs, int n_blocks, int variant,
                              hipStream_t s) {
    if (n_jobs == 1) {
        PO_DISPATCH_K(first->K, (camera_t<__half, KK, 1>(first, n_jobs, jobs, n_blocks, variant, s)));
    }
    PO_DISPATCH_K(first->K, (camera_t<__half, KK, PO_BATCH_MAX_JOBS>(first, n_jobs, jobs, n_blocks, variant, s)));
}
#endif

#if PO_PART == 3
PO_PART_ERRORS_DEF(3)
hipError_t po_camera_split_f32(const po_tree* t, const KJob& job, int n_blocks, int variant, const KSplit& S,
                               hipStream_t s) {
    PO_DISPATCH_K(t->K, (split_t<float, KK, 0>(t, job, n_blocks, variant, S, s)));
}
#endif

#if PO_PART == 4
PO_PART_ERRORS_DEF(4)
hipError_t po_camera_split_f16(const po_tree* t, const KJob& job, int n_blocks, int variant, const KSplit& S,
                               hipStream_t s) {
    PO_DISPATCH_K(t->K, (split_t<__half, KK, 0>(t, job, n_blocks, variant, S, s)));
}
#endif

#if PO_PART == 5
PO_PART_ERRORS_DEF(5)
hipError_t po_rays_split_f32(const po_tree* t, const KJob& job, int n_blocks, int variant, const KSplit& S,
                             hipStream_t s) {
    PO_DISPATCH_K(t->K, (split_t<float, KK, 1>(t, job, n_blocks, variant, S, s)));
}
#endif

#if PO_PART == 6
PO_PART_ERRORS_DEF(6)
hipError_t po_rays_split_f16(const po_tree* t, const KJob& job, int n_blocks, int variant, const KSplit& S,
                             hipStream_t s) {
    PO_DISPATCH_K(t->K, (split_t<__half, KK, 1>(t, job, n_blocks, variant, S, s)));
}
#endif

#if PO_PART == 7
PO_PART_ERRORS_DEF(7)
hipError_t po_launch_backward_split(const po_tree* t, int64_t n, const float* o, const float* d, const KOpts& op,
                                    const float* rgb_fwd, const float* grad, float* gsig, float* gsh,
                                    const KSplit& S, hipStream_t s) {
    PO_DISPATCH_K(t->K, (backward_split_t<KK>(t, n, o, d, op, rgb_fwd, grad, gsig, gsh, S, s)));
}

hipError_t po_launch_backward_kept(const po_tree* t, int64_t n, const float* o, const float* d, const KOpts& op,
                                   const float* rgb_fwd, const float* grad, float* gsig, float* gsh,
                                   const KSplit& S, hipStream_t s) {
    PO_DISPATCH_K(t->K, (backward_kept_t<KK>(t, n, o, d, op, rgb_fwd, grad, gsig, gsh, S, s)));
}
#endif

#if PO_PART == 0
PO_PART_ERRORS_DEF(0)
hipError_t po_launch_rays(const po_tree* t, int64_t n, const float* o, const float* d, const KOpts& op,
                          float* rgb, float* aux, hipStream_t s) {
    if (t->desc.dtype == PO_F32) {
        PO_DISPATCH_K(t->K, (rays_t<float, KK>(t, n, o, d, op, rgb, aux, s)));
    } else {
        PO_DISPATCH_K(t->K, (rays_t<__half, KK>(t, n, o, d, op, rgb, aux, s)));
    }
}

hipError_t po_launch_camera_jobs(const po_tree* first, int n_jobs, KJob* jobs, int n_blocks, int variant,
                                 hipStream_t s) {
    return first->desc.dtype == PO_F32 ? po_camera_jobs_f32(first, n_jobs, jobs, n_blocks, variant, s)
                                       : po_camera_jobs_f16(first, n_jobs, jobs, n_blocks, variant, s);
}

hipError_t po_launch_camera_split(const po_tree* t, const KJob& job, int n_blocks, int variant, const KSplit& S,
                                  hipStream_t s) {
    return t->desc.dtype == PO_F32 ? po_camera_split_f32(t, job, n_blocks, variant, S, s)
                                   : po_camera_split_f16(t, job, n_blocks, variant, S, s);
}

hipError_t po_launch_rays_split(const po_tree* t, int64_t n, const float* o, const float* d, const KOpts& op,
                                float* rgb, float* aux, const KSplit& S0, hipStream_t s) {
    KJob job;
    std::memset(&job, 0, sizeof job);
    job.tr = t->kt;
    job.op = op;
    job.rgb = rgb;
    job.aux = aux;
    KSplit S = S0;
    S.ray_o = o;
    S.ray_d = d;
    S.n_rays = n;
    // a batch of rays below a frame's size fills the chip less: a shorter
    // first walk and smaller pieces (65536 random rays of the depth-8
    // training tree: 203 us with 8-cell pieces, 325 us with the frame's 32,
    // 300 us in one pass)
    po_rays_piece_sizes(n, &S);
    const int n_blocks = (int)((n + kBlock - 1) / kBlock);
    const int variant = po_fwd_variant(op, aux, t->kt);
    return t->desc.dtype == PO_F32 ? po_rays_split_f32(t, job, n_blocks, variant, S, s)
                                   : po_rays_split_f16(t, job, n_blocks, variant, S, s);
}

hipError_t po_launch_backward(const po_tree* t, int64_t n, const float* o, const float* d, const KOpts& op,
                              const float* rgb_fwd, const float* grad, float* gsig, float* gsh, hipStream_t s) {
    PO_DISPATCH_K(t->K, (backward_t<KK>(t, n, o, d, op, rgb_fwd, grad, gsig, gsh, s)));
}

hipError_t po_launch_leaf_weights(const po_tree* t, const KCam& cam, const KOpts& op, int mode, float* weight,
                                  float* alpha, hipStream_t s) {
    const int n_blocks = 4 * ((cam.W + 15) / 16) * ((cam.H + 15) / 16);
    dim3 grid((unsigned)rows_grid(n_blocks, 4 * (int64_t)((cam.W + 15) / 16))), block(kBlock);
    const size_t lds = stack_bytes(t->kt.depth);
    unsigned* wt = reinterpret_cast<unsigned*>(weight);
    if (t->desc.dtype == PO_F32) {
        if (mode == 0)
            hipLaunchKernelGGL((k_leaf_weights<float, 0>), grid, block, lds, s, t->kt, cam, op, n_blocks, wt, alpha);
        else
            hipLaunchKernelGGL((k_leaf_weights<float, 1>), grid, block, lds, s, t->kt, cam, op, n_blocks, wt, alpha);
    } else {
        if (mode == 0)
            hipLaunchKernelGGL((k_leaf_weights<__half, 0>), grid, block, lds, s, t->kt, cam, op, n_blocks, wt, alpha);
        else
            hipLaunchKernelGGL((k_leaf_weights<__half, 1>), grid, block, lds, s, t->kt, cam, op, n_blocks, wt, alpha);
    }
    return hipGetLastError();
}

hipError_t po_traversal_stats_sync(const po_tree* t, const KCam* cam, int64_t n, const float* o, const float* d,
                                   const KOpts& op, unsigned long long* h_sums, hipStream_t s) {
    // the sums live in this part's g_po_stats; the caller serialises calls
    unsigned long long* d_sums = nullptr;
    hipError_t e = hipGetSymbolAddress((void**)&d_sums, HIP_SYMBOL(g_po_stats));
    if (e != hipSuccess) return e;
    if ((e = hipMemsetAsync(d_sums, 0, 4 * sizeof(unsigned long long), s)) != hipSuccess) return e;
    KCam c;
    std::memset(&c, 0, sizeof c);
    if (cam) c = *cam;
    const int n_blocks = cam ? 4 * ((c.W + 15) / 16) * ((c.H + 15) / 16) : (int)((n + kBlock - 1) / kBlock);
    dim3 grid((unsigned)grid_for(n_blocks)), block(kBlock);
    const size_t lds = stack_bytes(t->kt.depth);
    const bool f32 = t->desc.dtype == PO_F32;
    if (cam && f32)
        hipLaunchKernelGGL((k_traversal_stats<float, 0>), grid, block, lds, s, t->kt, c, o, d, n, op, n_blocks, d_sums);
    else if (cam)
        hipLaunchKernelGGL((k_traversal_stats<__half, 0>), grid, block, lds, s, t->kt, c, o, d, n, op, n_blocks, d_sums);
    else if (f32)
        hipLaunchKernelGGL((k_traversal_stats<float, 1>), grid, block, lds, s, t->kt, c, o, d, n, op, n_blocks, d_sums);
    else
        hipLaunchKernelGGL((k_traversal_stats<__half, 1>), grid, block, lds, s, t->kt, c, o, d, n, op, n_blocks, d_sums);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(h_sums, d_sums, 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s)) !=
        hipSuccess)
        return e;
    return hipStreamSynchronize(s);
}

hipError_t po_launch_camera_rays(const KCam& cam, float* o, float* d, hipStream_t s) {
    const int64_t n = (int64_t)cam.W * cam.H;
    hipLaunchKernelGGL(k_camera_rays, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, cam, o, d);
    return hipGetLastError();
}

hipError_t po_launch_mse_grad(int64_t n, const float* rgb, const float* target, float scale, float* grad,
                              float* sq_sum, hipStream_t s) {
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_mse_grad, dim3((unsigned)(blocks < 512 ? blocks : 512)), dim3(256), 0, s, n, rgb, target,
                       scale, grad, sq_sum);
    return hipGetLastError();
}

hipError_t po_launch_gather_rays(int64_t n, const int64_t* idx, int64_t n_src, const float* o, const float* d,
                                 const float* t, float* bo, float* bd, float* bt, hipStream_t s) {
    hipLaunchKernelGGL(k_gather_rays, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, idx, n_src, o, d, t,
                       bo, bd, bt);
    return hipGetLastError();
}

hipError_t po_launch_draw_batch(int64_t n, uint64_t seed, uint64_t first, int64_t n_src, const float* o,
                               const float* d, const float* t, float* bo, float* bd, float* bt, float* sq_sum,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_draw_batch, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, seed, first, n_src, o, d,
                       t, bo, bd, bt, sq_sum);
    return hipGetLastError();
}

hipError_t po_launch_sgd(int64_t n, float* param, float* grad, float lr, bool zero_grad, hipStream_t s) {
    hipLaunchKernelGGL(k_sgd, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, param, grad, lr,
                       zero_grad ? 1 : 0);
    return hipGetLastError();
}

hipError_t po_read_device_errors(unsigned long long* out) {
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return e;
    hipError_t (*const part[PO_PARTS])(unsigned long long*, bool) = {
        po_part_errors_0, po_part_errors_1, po_part_errors_2, po_part_errors_3,
        po_part_errors_4, po_part_errors_5, po_part_errors_6, po_part_errors_7};
    unsigned long long sum = 0;
    for (int i = 0; i < PO_PARTS; ++i) {
        unsigned long long v = 0;
        if ((e = part[i](&v, false)) != hipSuccess) return e;
        sum += v;
    }
    *out = sum;
    return hipSuccess;
}

hipError_t po_reset_device_errors() {
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return e;
    hipError_t (*const part[PO_PARTS])(unsigned long long*, bool) = {
        po_part_errors_0, po_part_errors_1, po_part_errors_2, po_part_errors_3,
        po_part_errors_4, po_part_errors_5, po_part_errors_6, po_part_errors_7};
    for (int i = 0; i < PO_PARTS; ++i)
        if ((e = part[i](nullptr, true)) != hipSuccess) return e;
    return hipSuccess;
}

namespace {
constexpr int kNoAllocDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kNoAllocDevices];  // device address of `scratch`, per device (nullptr: not looked up yet)
}  // namespace

hipError_t po_noalloc_queue(KSplit* S) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kNoAllocDevices) return hipErrorInvalidDevice;
    void* ptr = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_noalloc_mu);
        if (!g_noalloc_ptr[dev]) {
            // first call on this device, which is current: its copy of the array
            e = hipGetSymbolAddress(&g_noalloc_ptr[dev], HIP_SYMBOL(scratch));
            if (e != hipSuccess) {
                g_noalloc_ptr[dev] = nullptr;
                return e;
            }
        }
        ptr = g_noalloc_ptr[dev];
    }
    po_split_layout(ptr, kNoAllocRegionSlots, S);
    return hipSuccess;
}

int po_plan_id(const po_tree* t) {
    // record kind (float32, float16, codebook), K and the load plan
    const int kind = t->codebook ? 2 : (t->desc.dtype == PO_F32 ? 0 : 1);
    bool fast = false;
    switch (t->K) {
#define PO_PLAN_CASE(KK)                                                                                    \
    case KK:                                                                                                \
        fast = kind == 2 ? use_fast_cb<KK>(t) : (kind == 0 ? use_fast<float, KK>(t) : use_fast<__half, KK>(t)); \
        break;
        PO_PLAN_CASE(1)
        PO_PLAN_CASE(4)
        PO_PLAN_CASE(9)
        PO_PLAN_CASE(16)
        PO_PLAN_CASE(25)
#undef PO_PLAN_CASE
    }
    return (kind * 64 + t->K) * 2 + (fast ? 1 : 0);
}
#endif  // PO_PART == 0
