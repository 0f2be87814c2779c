// Codebook compression of leaf coefficients (App. B.2): for every basis
// function the RGB coefficient triples of all leaves are quantised by median
// cut into at most 2^16 colours, stored as float16, and every leaf keeps one
// 16-bit index per basis function.  Host only; one thread per basis function.
//
// The median cut is specified exactly so that its result is reproducible:
// start from one box holding every point; repeatedly split the box whose
// longest side is longest (ties: lowest box number) along that side (ties:
// lowest axis); the lower half is the floor(m/2) points first in the order
// (coordinate, point index) and keeps the box number, the upper half takes
// the next number; boxes of one point or zero extent are not split; stop at
// M boxes.  A box's colour is the mean of its points, summed in double
// precision in ascending point order and rounded to float16 (nearest, ties
// to even).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <exception>
#include <mutex>
#include <queue>
#include <thread>
#include <vector>

#include "po_internal.h"

namespace {

// IEEE binary16 bits of a double, round to nearest with ties to even,
// assembled from the double's own bit fields.
uint16_t half_from_double(double x) {
    uint64_t b;
    std::memcpy(&b, &x, sizeof b);
    const uint16_t sign = (uint16_t)((b >> 48) & 0x8000u);
    const int e = (int)((b >> 52) & 0x7ff);
    const uint64_t frac = b & ((1ull << 52) - 1);
    if (e == 0x7ff) return (uint16_t)(sign | (frac ? 0x7e00u : 0x7c00u));
    if (e == 0) return sign;  // below 2^-1022: rounds to zero
    const int E = e - 1023;
    if (E > 15) return (uint16_t)(sign | 0x7c00u);
    const uint64_t sig = frac | (1ull << 52);  // 53-bit significand
    // bits dropped: the half keeps 11 significant bits when normal (E >= -14),
    // fewer below, where its unit is 2^-24
    const int shift = E >= -14 ? 42 : 28 - E;
    if (shift > 63) return sign;
    uint64_t kept = sig >> shift;
    const uint64_t rem = sig & ((1ull << shift) - 1);
    const uint64_t halfway = 1ull << (shift - 1);
    if (rem > halfway || (rem == halfway && (kept & 1u))) kept += 1;
    if (E >= -14) {
        int hexp = E + 15;
        if (kept == 2048) {  // carried into the next binade
            kept = 1024;
            hexp += 1;
        }
        if (hexp >= 31) return (uint16_t)(sign | 0x7c00u);
        return (uint16_t)(sign | (uint16_t)(hexp << 10) | (uint16_t)(kept - 1024));
    }
    return (uint16_t)(sign | (uint16_t)kept);  // 1024 is the smallest normal
}

struct Box {
    int64_t begin, end;  // range of the permutation
    double extent;
    int axis;
};

// Median cut of the n points p[3i..3i+2] into at most M boxes.  Writes box
// numbers to idx[i * idx_stride] and colours to cb[4 * box + c] (float16
// bits, fourth entry 0).  Returns the number of boxes.
int64_t median_cut(const float* p, int64_t n, int32_t M, uint16_t* idx, int64_t idx_stride, uint16_t* cb) {
    std::memset(cb, 0, sizeof(uint16_t) * 4 * (size_t)M);
    if (n == 0) return 0;
    std::vector<int64_t> perm((size_t)n);
    for (int64_t i = 0; i < n; ++i) perm[(size_t)i] = i;
    std::vector<Box> boxes;
    boxes.reserve((size_t)M);
    auto measure = [&](Box& bx) {
        bx.extent = 0.0;
        bx.axis = 0;
        for (int ax = 0; ax < 3; ++ax) {
            double lo = p[3 * perm[(size_t)bx.begin] + ax], hi = lo;
            for (int64_t q = bx.begin + 1; q < bx.end; ++q) {
                const double v = p[3 * perm[(size_t)q] + ax];
                lo = std::min(lo, v);
                hi = std::max(hi, v);
            }
            if (hi - lo > bx.extent) {
                bx.extent = hi - lo;
                bx.axis = ax;
            }
        }
    };
    // splittable boxes, longest extent first, then lowest number
    auto later = [&](int64_t a, int64_t b) {
        const Box &A = boxes[(size_t)a], &B = boxes[(size_t)b];
        return A.extent < B.extent || (A.extent == B.extent && a > b);
    };
    std::priority_queue<int64_t, std::vector<int64_t>, decltype(later)> q(later);
    auto offer = [&](int64_t id) {
        const Box& bx = boxes[(size_t)id];
        if (bx.end - bx.begin >= 2 && bx.extent > 0.0) q.push(id);
    };
    boxes.push_back({0, n, 0.0, 0});
    measure(boxes[0]);
    offer(0);
    while ((int64_t)boxes.size() < M && !q.empty()) {
        const int64_t id = q.top();
        q.pop();
        Box lo = boxes[(size_t)id];
        const int ax = lo.axis;
        const int64_t mid = lo.begin + (lo.end - lo.begin) / 2;
        std::nth_element(perm.begin() + lo.begin, perm.begin() + mid, perm.begin() + lo.end,
                         [&](int64_t a, int64_t b) {
                             const float va = p[3 * a + ax], vb = p[3 * b + ax];
                             return va < vb || (va == vb && a < b);
                         });
        Box hi = {mid, lo.end, 0.0, 0};
        lo.end = mid;
        measure(lo);
        measure(hi);
        boxes[(size_t)id] = lo;
        boxes.push_back(hi);
        offer(id);
        offer((int64_t)boxes.size() - 1);
    }
    const int64_t nb = (int64_t)boxes.size();
    std::vector<int32_t> box_of((size_t)n);
    for (int64_t b = 0; b < nb; ++b)
        for (int64_t q2 = boxes[(size_t)b].begin; q2 < boxes[(size_t)b].end; ++q2)
            box_of[(size_t)perm[(size_t)q2]] = (int32_t)b;
    std::vector<double> sum((size_t)nb * 3, 0.0);
    std::vector<int64_t> cnt((size_t)nb, 0);
    for (int64_t i = 0; i < n; ++i) {
        const int32_t b = box_of[(size_t)i];
        for (int c = 0; c < 3; ++c) sum[(size_t)b * 3 + c] += (double)p[3 * i + c];
        cnt[(size_t)b] += 1;
        idx[i * idx_stride] = (uint16_t)b;
    }
    for (int64_t b = 0; b < nb; ++b)
        for (int c = 0; c < 3; ++c) cb[4 * b + c] = half_from_double(sum[(size_t)b * 3 + c] / (double)cnt[(size_t)b]);
    return nb;
}

}  // namespace

extern "C" po_status po_codebook_build(int64_t n_leaves, int32_t K, const float* h_coef, int64_t coef_stride,
                                       int32_t M, uint16_t* h_codebook, uint16_t* h_index, int64_t index_stride,
                                       int32_t* h_boxes) {
    if (n_leaves < 0 || n_leaves >= (1ll << 31)) return po_report(PO_ERR_INVALID, "n_leaves out of range");
    const int Kmax = (PO_MAX_SH_DEGREE + 1) * (PO_MAX_SH_DEGREE + 1);
    if (K < 1 || K > Kmax) return po_report(PO_ERR_INVALID, "K out of range");
    if (M < 1 || M > 65536) return po_report(PO_ERR_INVALID, "codebook size must be in [1, 65536]");
    if (coef_stride < 3 * (int64_t)K) return po_report(PO_ERR_INVALID, "coef_stride must be >= 3K");
    if (index_stride < K) return po_report(PO_ERR_INVALID, "index_stride must be >= K");
    if (!h_codebook || (n_leaves > 0 && (!h_coef || !h_index)))
        return po_report(PO_ERR_INVALID, "NULL array");
    for (int64_t i = 0; i < n_leaves * coef_stride; ++i) {
        const int64_t j = i % coef_stride;
        if (j < 3 * K && !std::isfinite(h_coef[i])) return po_report(PO_ERR_INVALID, "non-finite coefficient");
    }
    try {
        std::vector<std::thread> pool;
        std::vector<int64_t> nbox((size_t)K, 0);
        std::exception_ptr err = nullptr;
        std::mutex err_mu;
        const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        for (unsigned t = 0; t < std::min<unsigned>(hw, (unsigned)K); ++t) {
            pool.emplace_back([&, t] {
                try {
                    std::vector<float> pts((size_t)n_leaves * 3);
                    for (int k = (int)t; k < K; k += (int)hw) {
                        for (int64_t i = 0; i < n_leaves; ++i)
                            for (int c = 0; c < 3; ++c)
                                pts[(size_t)i * 3 + c] = h_coef[i * coef_stride + c * K + k];
                        nbox[(size_t)k] = median_cut(pts.data(), n_leaves, M, h_index + k, index_stride,
                                                     h_codebook + (size_t)k * M * 4);
                    }
                } catch (...) {
                    std::lock_guard<std::mutex> lk(err_mu);
                    err = std::current_exception();
                }
            });
        }
        for (auto& th : pool) th.join();
        if (err) std::rethrow_exception(err);
        for (int64_t i = 0; i < n_leaves; ++i)
            for (int64_t j = K; j < index_stride; ++j) h_index[i * index_stride + j] = 0;
        if (h_boxes)
            for (int k = 0; k < K; ++k) h_boxes[k] = (int32_t)nbox[(size_t)k];
    } catch (const std::bad_alloc&) {
        return po_report(PO_ERR_OOM, "codebook allocation");
    } catch (...) {
        return po_report(PO_ERR_INVALID, "codebook construction failed");
    }
    return po_report(PO_OK, "");
}
