// C ABI of libnufft_mi355x: plan lifetime, validation, binning, work-item
// construction and the stage sequences of the NUFFT pair
//   forward  y = V F S x        (paper Section 2.1, Eq. A = VFS)
//   adjoint  x = S^H F^H V^H y  (Section 2.1 "Adjoint PyNUFFT")
// with batch mode (Section 2.1) and coil maps (Section 2.2, multi-coil).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <vector>

#include "../../include/nufft_mi355x.h"
#include "nufft_internal.h"

using namespace nufft;

thread_local LaunchEvents *nufft::g_launch_events = nullptr;

namespace {

constexpr uint64_t kMagic = 0x4e55464654333535ull;  // "NUFFT355"
constexpr double kPi = 3.14159265358979323846;

thread_local std::string g_last_error;
std::mutex g_registry_mu;
std::set<const void *> g_registry;

int fail(int status, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return status;
}

int hip_fail(hipError_t e, const char *what) {
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return fail(NUFFT_ERR_OOM, "%s: %s", what, hipGetErrorString(e));
    return fail(NUFFT_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                          \
    do {                                             \
        hipError_t e_ = (expr);                      \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

template <class T>
hipError_t dmalloc(T **p, size_t count) {
    *p = nullptr;
    if (count == 0) return hipSuccess;
    return hipMalloc(reinterpret_cast<void **>(p), count * sizeof(T));
}

template <class T>
void dfree(T *&p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

template <class T>
hipError_t upload(T **p, const std::vector<T> &v) {
    hipError_t e = dmalloc(p, v.size());
    if (e != hipSuccess || v.empty()) return e;
    return hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
}

// Copy v into *p, reusing the buffer when it holds v (capacity *cap in
// elements, grown, never shrunk): re-binning a trajectory of the same size
// then allocates nothing.
template <class T>
hipError_t upload_into(T **p, size_t *cap, const std::vector<T> &v) {
    if (v.size() > *cap || !*p) {
        dfree(*p);
        *cap = 0;
        hipError_t e = dmalloc(p, std::max<size_t>(v.size(), 1));
        if (e != hipSuccess) return e;
        *cap = std::max<size_t>(v.size(), 1);
    }
    if (v.empty()) return hipSuccess;
    return hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
}

bool smooth235(int64_t k) {
    for (int p : {2, 3, 5})
        while (k % p == 0) k /= p;
    return k == 1;
}

}  // namespace

struct nufft_plan_s {
    uint64_t magic = kMagic;
    int device = 0;
    int d = 0;
    int64_t N[kMaxDim] = {1, 1, 1};
    int64_t K[kMaxDim] = {1, 1, 1};
    int J = 0;
    int64_t M = 0;
    AxisKernel ker[kMaxDim];
    RadixPlan rp[kMaxDim];
    int T[kMaxDim] = {1, 1, 1};
    int nt[kMaxDim] = {1, 1, 1};
    int R[kMaxDim] = {1, 1, 1};
    int tile_cells = 1;
    int64_t nbins = 1;
    int chunk = 2048;
    int fft_groups = 1024;
    int64_t img_elems = 1, grid_elems = 1, tmp_elems = 1;

    // device constants
    float *scale[kMaxDim] = {nullptr, nullptr, nullptr};
    float2 *tw[kMaxDim] = {nullptr, nullptr, nullptr};
    bool minmax = false;                                   // min-max interpolator
    float2 *phase[kMaxDim] = {nullptr, nullptr, nullptr};  // its grid phase e^{-i pi k / K}
    float *coef[kMaxDim] = {nullptr, nullptr, nullptr};
    int nq[kMaxDim] = {0, 0, 0};
    int nq_d[kMaxDim] = {0, 0, 0};
    float *dcoef[kMaxDim] = {nullptr, nullptr, nullptr};
    // trajectory and binning
    float *om = nullptr;
    float *om_sorted = nullptr;
    int *perm = nullptr;
    int *sub_start = nullptr;  // [nbins * 2^d + 1]
    GridItem *items = nullptr;
    int64_t n_items = 0;
    InterpItem *iitems = nullptr;  // nullptr: the gather reads the grid directly
    int64_t n_iitems = 0;
    bool staged_interp = true;
    int interp_merge = 1;  // tiles along the last axis one gather item may cover
    bool presort = false;      // gridding reads samples permuted into sorted order
    bool fuse_reduce = false;  // first inverse FFT pass sums the partial tiles
    bool grid_mfma = false;    // gridding on the matrix cores by row tiles
    bool grid_blk = false;     // 3D gridding on the matrix cores by 4 x 4 blocks
    int grid_waves = 4;        // its wavefronts per work item (1 or 4)
    int rec_stride = 0;        // its LDS floats per staged sample
    int seg_len = 16, segs = 1;
    int group_lanes = 64;
    int stage_floats = 0;
    HotTile *hot = nullptr;
    int2 *split_of_tile = nullptr;  // [nbins]: (first partial slot, chunks), chunks 0 if not split
    int2 *item_segs = nullptr;      // [n_items][kMaxNeighbors + 1]: (segment start, offset in the item's list)
    int64_t n_hot = 0;
    int64_t n_slots = 0;
    // capacities of the binning tables above (elements; grown, never shrunk)
    size_t cap_sub_start = 0, cap_items = 0, cap_iitems = 0, cap_hot = 0, cap_split = 0, cap_item_segs = 0;
    // binning scratch, sized at plan creation, so re-binning allocates nothing
    int *bkeys = nullptr, *bkeys_sorted = nullptr, *biota = nullptr, *bcounts = nullptr, *bflag = nullptr;
    void *sort_temp = nullptr;
    size_t sort_temp_bytes = 0;
    float *om_prev = nullptr;  // the trajectory in force while a new one is binned
    // per sorted sample its window (first taps and weights), made with the
    // binning when the plan asks for it (option weight_table), else nullptr
    bool use_wtab = false;
    float *wtab = nullptr;
    size_t cap_wtab = 0;  // floats
    // coils
    float2 *coils = nullptr;
    int C = 1;
    bool coil_mode = false;
    // workspace
    int cap_grids = 0;
    int64_t cap_slots = -1;
    float2 *grid = nullptr;
    float2 *tmp = nullptr;
    float2 *partials = nullptr;
    float2 *ysorted = nullptr;  // [cap_grids][M] samples in sorted order for the gridding
    hipStream_t last_stream = nullptr;
    // optional per-kernel event timing
    bool timing = false;
    struct TimingRec {
        int kernel;
        hipEvent_t start, stop;
    };
    std::vector<TimingRec> timing_recs;
    std::vector<hipEvent_t> event_pool;

    SampleGeom geom() const {
        SampleGeom g{};
        g.d = d;
        g.J = J;
        g.jp = coef_row_width(J);
        g.minmax = minmax ? 1 : 0;
        for (int a = 0; a < d; ++a) {
            g.K[a] = int(K[a]);
            g.C[a] = double(K[a]) / (2.0 * kPi);
            g.nq[a] = nq[a];
            g.nq_d[a] = nq_d[a];
            g.coef[a] = coef[a];
            g.dcoef[a] = dcoef[a];
        }
        g.wtab = use_wtab ? wtab : nullptr;
        g.wtab_stride = use_wtab ? table_stride(d, J) : 0;
        return g;
    }
};

namespace {

int check_plan(nufft_plan_t p) {
    if (!p) return fail(NUFFT_ERR_BAD_PLAN, "plan handle is NULL");
    std::lock_guard<std::mutex> lk(g_registry_mu);
    if (!g_registry.count(p)) return fail(NUFFT_ERR_BAD_PLAN, "plan handle is not a live plan");
    if (p->magic != kMagic) return fail(NUFFT_ERR_BAD_PLAN, "plan handle is corrupted");
    return NUFFT_OK;
}

enum KernelId {
    kFirstPass, kStridedFwd, kStridedInv, kLastPass, kInterp, kGrid, kReduce, kGrad, kPermute, kNumKernels
};
const char *const kKernelNames[kNumKernels] = {"k_first_pass", "k_strided_pass<fwd>", "k_strided_pass<inv>",
                                               "k_last_pass", "k_interp", "k_grid", "k_reduce_partials",
                                               "k_grad", "k_permute_samples"};

hipError_t take_event(nufft_plan_s *p, hipEvent_t *ev) {
    if (!p->event_pool.empty()) {
        *ev = p->event_pool.back();
        p->event_pool.pop_back();
        return hipSuccess;
    }
    return hipEventCreate(ev);
}

// Launch through `fn`; when the plan collects timings, its kernel launch
// stamps a pair of events at the kernel's start and end.
template <class F>
hipError_t timed(nufft_plan_s *p, int kernel, hipStream_t s, F fn) {
    if (!p->timing) return fn();
    hipEvent_t a, b;
    hipError_t e = take_event(p, &a);
    if (e != hipSuccess) return e;
    if ((e = take_event(p, &b)) != hipSuccess) return e;
    // the stage's kernel launch records a and b at its own start and end
    LaunchEvents ev{a, b, false};
    g_launch_events = &ev;
    e = fn();
    g_launch_events = nullptr;
    if (e != hipSuccess || !ev.used) {  // failed, or nothing to launch
        p->event_pool.push_back(a);
        p->event_pool.push_back(b);
        return e;
    }
    p->timing_recs.push_back({kernel, a, b});
    return hipSuccess;
}

void recycle_timing(nufft_plan_s *p) {
    for (auto &r : p->timing_recs) {
        p->event_pool.push_back(r.start);
        p->event_pool.push_back(r.stop);
    }
    p->timing_recs.clear();
}

void free_plan(nufft_plan_s *p) {
    recycle_timing(p);
    for (hipEvent_t e : p->event_pool) (void)hipEventDestroy(e);
    p->event_pool.clear();
    for (int a = 0; a < kMaxDim; ++a) {
        dfree(p->scale[a]);
        dfree(p->tw[a]);
        dfree(p->coef[a]);
        dfree(p->dcoef[a]);
        dfree(p->phase[a]);
    }
    dfree(p->bkeys);
    dfree(p->bkeys_sorted);
    dfree(p->biota);
    dfree(p->bcounts);
    dfree(p->bflag);
    if (p->sort_temp) (void)hipFree(p->sort_temp);
    p->sort_temp = nullptr;
    dfree(p->om_prev);
    dfree(p->wtab);
    dfree(p->om);
    dfree(p->om_sorted);
    dfree(p->perm);
    dfree(p->sub_start);
    dfree(p->items);
    dfree(p->iitems);
    dfree(p->hot);
    dfree(p->split_of_tile);
    dfree(p->item_segs);
    dfree(p->coils);
    dfree(p->grid);
    dfree(p->tmp);
    dfree(p->partials);
    dfree(p->ysorted);
}

// Tile edge on one axis: the largest divisor of K that is <= target, raised
// to the smallest divisor >= need = J - 1 when it would be smaller, so a
// window of J taps reaches at most two tiles per axis.
int choose_tile(int64_t K, int target, int need) {
    int best = 1;
    for (int64_t t = 1; t <= K && t <= target; ++t)
        if (K % t == 0) best = int(t);
    if (best < need) {
        for (int64_t t = need; t <= K; ++t)
            if (K % t == 0) return int(t);
        return int(K);
    }
    return best;
}

int bits_for(int64_t n) {
    int b = 1;
    while ((int64_t(1) << b) < n) ++b;
    return b;
}

// Bin the trajectory om (device, caller order) into the plan: sorted copy,
// permutation, sub-bin offsets, gather and gridding work items.  Synchronous.
int bin_points(nufft_plan_s *p, const float *om_dev, hipStream_t s) {
    const int64_t M = p->M;
    const int d = p->d;
    const int64_t nkeys = p->nbins << d;
    if (M > 0) HIP_TRY(hipMemcpyAsync(p->om, om_dev, size_t(M) * d * sizeof(float), hipMemcpyDeviceToDevice, s),
                       "copy trajectory");
    int *keys = p->bkeys, *keys_sorted = p->bkeys_sorted, *iota = p->biota, *counts = p->bcounts, *flag = p->bflag;
    std::vector<int> hcounts(size_t(nkeys), 0);
    int hflag = 0;
    hipError_t e = hipSuccess;
    do {
        if ((e = hipMemsetAsync(counts, 0, size_t(nkeys) * sizeof(int), s)) != hipSuccess) break;
        if ((e = hipMemsetAsync(flag, 0, sizeof(int), s)) != hipSuccess) break;
        BinArgs ba{};
        ba.om = p->om;
        ba.M = M;
        ba.d = d;
        ba.J = p->J;
        for (int a = 0; a < d; ++a) {
            ba.K[a] = int(p->K[a]);
            ba.C[a] = double(p->K[a]) / (2.0 * kPi);
            ba.T[a] = p->T[a];
            ba.nt[a] = p->nt[a];
        }
        ba.keys = keys;
        ba.counts = counts;
        ba.flag = flag;
        if ((e = launch_bin_keys(ba, s)) != hipSuccess) break;
        if ((e = hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess) break;
        if ((e = hipMemcpyAsync(hcounts.data(), counts, size_t(nkeys) * sizeof(int), hipMemcpyDeviceToHost, s)) !=
            hipSuccess)
            break;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) break;
        if (hflag) break;
        if ((e = launch_iota(iota, M, s)) != hipSuccess) break;
        if ((e = sort_pairs(keys, keys_sorted, iota, p->perm, M, bits_for(nkeys), p->sort_temp, p->sort_temp_bytes,
                            s)) != hipSuccess)
            break;
        if ((e = launch_permute_points(p->om, p->perm, M, d, p->om_sorted, s)) != hipSuccess) break;
        if (p->use_wtab) {
            // the window table: allocated once for the plan's M (a re-bin
            // rewrites it in place)
            const size_t need = size_t(std::max<int64_t>(M, 1)) * size_t(table_stride(d, p->J));
            if (need > p->cap_wtab) {
                dfree(p->wtab);
                p->cap_wtab = 0;
                if ((e = dmalloc(&p->wtab, need)) != hipSuccess) break;
                p->cap_wtab = need;
            }
            if ((e = launch_weight_table(p->geom(), p->om_sorted, M, p->wtab, s)) != hipSuccess) break;
        }
        if ((e = hipStreamSynchronize(s)) != hipSuccess) break;
    } while (false);
    if (e != hipSuccess) return hip_fail(e, "binning the trajectory");
    if (hflag) return fail(NUFFT_ERR_NONFINITE, "trajectory has a NaN, infinite or out-of-range coordinate");

    // sub-bin offsets: sorted order is (tile, crossing code), stable in the caller's order
    std::vector<int> start(size_t(nkeys) + 1, 0);
    for (int64_t k = 0; k < nkeys; ++k) start[k + 1] = start[k] + hcounts[k];
    // gridding work items: per tile, the samples whose windows reach it, in chunks
    std::vector<GridItem> items;
    std::vector<HotTile> hot;
    std::vector<InterpItem> iitems;
    int64_t slots = 0;
    items.reserve(size_t(p->nbins));
    const int ichunk = 256 * kInterpSamplesPerThread;
    for (int64_t t = 0; t < p->nbins; ++t) {
        int tc[kMaxDim];
        int64_t rem = t;
        for (int a = d - 1; a >= 0; --a) {
            tc[a] = int(rem % p->nt[a]);
            rem /= p->nt[a];
        }
        int lo[kMaxNeighbors], hi[kMaxNeighbors];
        const int nseg = tile_segments(d, tc, p->nt, p->R, start.data(), lo, hi);
        int64_t S = 0;
        for (int q = 0; q < nseg; ++q) S += hi[q] - lo[q];
        const int nch = int(std::max<int64_t>(1, (S + p->chunk - 1) / p->chunk));
        const int slot = nch > 1 ? int(slots) : -1;
        for (int c = 0; c < nch; ++c) items.push_back(GridItem{int(t), c, nch, slot});
        if (nch > 1) {
            hot.push_back(HotTile{int(t), slot, nch, 0});
            slots += nch;
        }
    }
    // Gather work items: a crowded tile's own bin in chunks of `ichunk`; runs
    // of sparse tiles along the last axis (their samples are contiguous in the
    // sorted order) share one item of at most `ichunk` samples and
    // interp_merge tiles, which stages one region for all of them.
    {
        const int nt_last = p->nt[d - 1];
        int64_t t = 0;
        while (t < p->nbins) {
            const int b0 = start[size_t(t) << d], b1 = start[size_t(t + 1) << d];
            if (b1 - b0 >= ichunk) {
                for (int f = b0; f < b1; f += ichunk) iitems.push_back(InterpItem{int(t), f, std::min(ichunk, b1 - f), 1});
                ++t;
                continue;
            }
            if (b1 == b0) {
                ++t;
                continue;
            }
            int64_t u = t + 1;  // extend the run within the row while it fits
            while (u < p->nbins && u % nt_last != 0 && u - t < p->interp_merge &&
                   start[size_t(u + 1) << d] - b0 <= ichunk)
                ++u;
            const int e = start[size_t(u) << d];
            iitems.push_back(InterpItem{int(t), b0, e - b0, int(u - t)});
            t = u;
        }
    }
    // Longest items first: workgroups are dealt to the XCDs round-robin in
    // launch order, so the crowded tiles (all at the k-space centre, i.e. at
    // the two ends of the tile order) spread over the whole chip and the
    // light tiles fill in behind them.
    {
        std::vector<int64_t> cnt(items.size());
        std::vector<int> ord(items.size());
        for (size_t q = 0; q < items.size(); ++q) {
            const GridItem &gi = items[q];
            int tc[kMaxDim];
            int64_t rem = gi.tile;
            for (int a = d - 1; a >= 0; --a) {
                tc[a] = int(rem % p->nt[a]);
                rem /= p->nt[a];
            }
            int lo[kMaxNeighbors], hi[kMaxNeighbors];
            const int nseg = tile_segments(d, tc, p->nt, p->R, start.data(), lo, hi);
            int64_t S = 0;
            for (int k = 0; k < nseg; ++k) S += hi[k] - lo[k];
            cnt[q] = std::min<int64_t>(p->chunk, S - int64_t(gi.chunk) * p->chunk);
            ord[q] = int(q);
        }
        std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return cnt[x] > cnt[y]; });
        std::vector<GridItem> sorted(items.size());
        for (size_t q = 0; q < ord.size(); ++q) sorted[q] = items[ord[q]];
        items.swap(sorted);
        // (Measured: keeping gather items in tile order, dealt to the XCDs in
        // runs of neighbouring tiles, cuts the 3D gather's HBM reads by a
        // third through L2 hits on the halos but runs slower than longest
        // first, which balances the crowded centre over the chip.)
        std::stable_sort(iitems.begin(), iitems.end(),
                         [](const InterpItem &x, const InterpItem &y) { return x.count > y.count; });
    }
    std::vector<int2> split_of_tile(size_t(p->nbins), make_int2(0, 0));
    for (const HotTile &h : hot) split_of_tile[size_t(h.tile)] = make_int2(h.slot, h.nchunks);
    // The segments of every gridding item's tile, in the order tile_segments
    // lists them: (first sorted sample, offset of the segment in the item's
    // sample list), and (0, total) after the last, so a work item reads its
    // table in the same round trip as the item itself.
    constexpr int kSegRow = kMaxNeighbors + 1;
    std::vector<int2> item_segs(std::max<size_t>(items.size(), 1) * kSegRow, make_int2(0, 0));
    for (size_t q = 0; q < items.size(); ++q) {
        int tc[kMaxDim];
        int64_t rem = items[q].tile;
        for (int a = d - 1; a >= 0; --a) {
            tc[a] = int(rem % p->nt[a]);
            rem /= p->nt[a];
        }
        int lo[kMaxNeighbors], hi[kMaxNeighbors];
        const int nseg = tile_segments(d, tc, p->nt, p->R, start.data(), lo, hi);
        int pre = 0;
        for (int k = 0; k < nseg; ++k) {
            item_segs[q * kSegRow + size_t(k)] = make_int2(lo[k], pre);
            pre += hi[k] - lo[k];
        }
        item_segs[q * kSegRow + size_t(nseg)] = make_int2(0, pre);
    }
    HIP_TRY(upload_into(&p->sub_start, &p->cap_sub_start, start), "upload bin offsets");
    HIP_TRY(upload_into(&p->item_segs, &p->cap_item_segs, item_segs), "upload gridding segment tables");
    HIP_TRY(upload_into(&p->split_of_tile, &p->cap_split, split_of_tile), "upload split-tile index");
    HIP_TRY(upload_into(&p->items, &p->cap_items, items), "upload gridding work items");
    HIP_TRY(upload_into(&p->hot, &p->cap_hot, hot), "upload split tiles");
    p->n_items = int64_t(items.size());
    p->n_hot = int64_t(hot.size());
    p->n_slots = slots;
    p->n_iitems = 0;
    if (p->staged_interp) {
        HIP_TRY(upload_into(&p->iitems, &p->cap_iitems, iitems), "upload gather work items");
        p->n_iitems = int64_t(iitems.size());
    }
    return NUFFT_OK;
}

// Workspace for `grids` simultaneous K^d grids.
int ensure_workspace(nufft_plan_s *p, int grids) {
    if (grids <= p->cap_grids && p->n_slots <= p->cap_slots) return NUFFT_OK;
    const int g = std::max(grids, p->cap_grids);
    if (g > p->cap_grids) {
        dfree(p->grid);
        dfree(p->tmp);
        dfree(p->ysorted);
        p->cap_grids = 0;
        HIP_TRY(dmalloc(&p->grid, size_t(g) * p->grid_elems), "allocate grid workspace");
        HIP_TRY(dmalloc(&p->tmp, size_t(g) * std::max<int64_t>(p->tmp_elems, 1)), "allocate pass workspace");
        if (p->presort)
            HIP_TRY(dmalloc(&p->ysorted, size_t(g) * std::max<int64_t>(p->M, 1)), "allocate sorted samples");
    }
    dfree(p->partials);
    p->cap_slots = -1;
    HIP_TRY(dmalloc(&p->partials, size_t(g) * std::max<int64_t>(p->n_slots, 1) * p->tile_cells),
            "allocate partial tiles");
    p->cap_grids = g;
    p->cap_slots = p->n_slots;
    return NUFFT_OK;
}

// ---- stage sequences

// A stage sequence either launches its kernels or, given a collector, records
// each launch's arguments under a fixed stage slot (the multi-problem launch
// runs slot by slot, all problems' launches of one slot together).
enum StageKind { kStFirst, kStStrided, kStLast, kStInterp, kStGrid, kStReduce, kStPermute };
struct Emitted {
    int slot = 0;
    int kind = 0;
    FirstPassArgs first{};
    StridedPassArgs strided{};
    LastPassArgs last{};
    InterpArgs interp{};
    GridArgs grid{};
    ReduceArgs reduce{};
    PermuteJob permute{};
};
struct Collector {
    std::vector<Emitted> out;
    Emitted &add(int slot, int kind) {
        out.emplace_back();
        out.back().slot = slot;
        out.back().kind = kind;
        return out.back();
    }
};
// slots: forward pass p -> p, gather -> kMaxDim; adjoint permute -> 0, gridding
// -> 1, partial sums -> 2, inverse pass along axis a -> 3 + a
constexpr int kSlotInterp = kMaxDim;
constexpr int kSlotPermute = 0, kSlotGrid = 1, kSlotReduce = 2, kSlotInvPass = 3;

// G = F S (c x): x [B][N^d] -> out [B*C][K^d]; intermediates in the workspace.
// The FFT side of a transform: image N zero-padded onto grid K (or cropped
// back), per-axis scale tables (S, S^H), radix schedules, twiddles, coils and
// the two pass buffers.  The plan has one (N -> K with the deapodization);
// a Toeplitz operator has its own (N -> 2N, no scaling).
struct FftGeom {
    int d = 1;
    int64_t N[kMaxDim] = {1, 1, 1};
    int64_t K[kMaxDim] = {1, 1, 1};
    const RadixPlan *rp = nullptr;  // [d]
    float2 *const *tw = nullptr;    // [d]
    float *const *scale = nullptr;  // [d]
    float2 *const *phase = nullptr; // [d] min-max grid phase, or nullptr
    const float2 *coils = nullptr;  // [C][N^d] in coil mode, else nullptr
    int C = 1;
    float2 *grid = nullptr;
    float2 *tmp = nullptr;
    int fft_groups = 1024;
};

FftGeom plan_fft(const nufft_plan_s *p) {
    FftGeom f;
    f.d = p->d;
    for (int a = 0; a < p->d; ++a) {
        f.N[a] = p->N[a];
        f.K[a] = p->K[a];
    }
    f.rp = p->rp;
    f.tw = p->tw;
    f.scale = p->scale;
    f.phase = p->minmax ? p->phase : nullptr;
    f.coils = p->coil_mode ? p->coils : nullptr;
    f.C = p->coil_mode ? p->C : 1;
    f.grid = p->grid;
    f.tmp = p->tmp;
    f.fft_groups = p->fft_groups;
    return f;
}

// out = F S x: x [B][N^d] -> out [B*C][K^d] (times the coils in coil mode).
// With mult (Toeplitz product) the last forward pass's output is multiplied
// by it; only d = 1 does this here, d >= 2 fuses it into run_shfh.
int run_fs(nufft_plan_s *p, const FftGeom &f, const float2 *x, int B, float2 *out, hipStream_t s,
           const float2 *mult = nullptr, Collector *col = nullptr) {
    const int d = f.d;
    const int64_t grids = int64_t(B) * f.C;
    const float2 *cur = x;
    for (int pass = 0; pass < d; ++pass) {
        const int ax = d - 1 - pass;
        float2 *dst = (pass == d - 1) ? out : (((d - 1 - pass) % 2 == 0) ? f.grid : f.tmp);
        if (pass == 0) {
            FirstPassArgs a{};
            a.x = cur;
            a.out = dst;
            a.tw = f.tw[ax];
            a.rp = f.rp[ax];
            a.coils = f.coils;
            a.C = f.C;
            a.B = B;
            a.K = int(f.K[ax]);
            a.N = int(f.N[ax]);
            a.rows = 1;
            for (int b = 0; b < d - 1; ++b) a.rows *= f.N[b];
            a.d = d;
            a.target_groups = f.fft_groups;
            a.mult = (d == 1) ? mult : nullptr;
            a.phase = f.phase ? f.phase[ax] : nullptr;
            for (int b = 0; b < d; ++b) {
                a.Nax[b] = int(f.N[b]);
                a.scale[b] = f.scale[b];
            }
            if (col)
                col->add(pass, kStFirst).first = a;
            else
                HIP_TRY(timed(p, kFirstPass, s, [&] { return launch_first_pass(a, s); }), "forward first FFT pass");
        } else {
            StridedPassArgs a{};
            a.in = cur;
            a.out = dst;
            a.tw = f.tw[ax];
            a.rp = f.rp[ax];
            a.K = int(f.K[ax]);
            a.Lin = int(f.N[ax]);
            a.Lout = int(f.K[ax]);
            a.outer = 1;
            for (int b = 0; b < ax; ++b) a.outer *= f.N[b];
            a.inner = 1;
            for (int b = ax + 1; b < d; ++b) a.inner *= f.K[b];
            a.grids = grids;
            a.inverse = false;
            a.target_groups = f.fft_groups;
            a.phase = f.phase ? f.phase[ax] : nullptr;
            if (col)
                col->add(pass, kStStrided).strided = a;
            else
                HIP_TRY(timed(p, kStridedFwd, s, [&] { return launch_strided_pass(a, s); }),
                        "forward strided FFT pass");
        }
        cur = dst;
    }
    return NUFFT_OK;
}

// x = S^H F^H h (coil-combined): h [B*C][K^d] -> x [B][N^d].  With
// fused_partials, h's split tiles are still partial tiles (run_vh with
// reduce = false) and the first pass sums them.  With mult (Toeplitz
// product, d >= 2) the first pass multiplies its input by it.
int run_shfh(nufft_plan_s *p, const FftGeom &f, const float2 *h, int B, float2 *x, hipStream_t s,
             bool fused_partials = false, const float2 *mult = nullptr, Collector *col = nullptr) {
    const int d = f.d;
    const int64_t grids = int64_t(B) * f.C;
    const float2 *cur = h;
    for (int ax = 0; ax < d; ++ax) {
        if (ax == d - 1) {
            LastPassArgs a{};
            a.in = cur;
            a.x = x;
            a.tw = f.tw[ax];
            a.rp = f.rp[ax];
            a.coils = f.coils;
            a.C = f.C;
            a.B = B;
            a.K = int(f.K[ax]);
            a.N = int(f.N[ax]);
            a.rows = 1;
            for (int b = 0; b < d - 1; ++b) a.rows *= f.N[b];
            a.d = d;
            a.target_groups = f.fft_groups;
            a.phase = f.phase ? f.phase[ax] : nullptr;
            for (int b = 0; b < d; ++b) {
                a.Nax[b] = int(f.N[b]);
                a.scale[b] = f.scale[b];
            }
            if (col)
                col->add(kSlotInvPass + ax, kStLast).last = a;
            else
                HIP_TRY(timed(p, kLastPass, s, [&] { return launch_last_pass(a, s); }), "adjoint last FFT pass");
        } else {
            float2 *dst = (ax % 2 == 0) ? f.tmp : f.grid;
            StridedPassArgs a{};
            a.in = cur;
            a.out = dst;
            a.tw = f.tw[ax];
            a.rp = f.rp[ax];
            a.K = int(f.K[ax]);
            a.Lin = int(f.K[ax]);
            a.Lout = int(f.N[ax]);
            a.outer = 1;
            for (int b = 0; b < ax; ++b) a.outer *= f.N[b];
            a.inner = 1;
            for (int b = ax + 1; b < d; ++b) a.inner *= f.K[b];
            a.grids = grids;
            a.inverse = true;
            a.target_groups = f.fft_groups;
            a.phase = f.phase ? f.phase[ax] : nullptr;
            if (ax == 0) a.mult = mult;
            if (ax == 0 && fused_partials && p->n_hot > 0) {
                if (mult) return fail(NUFFT_ERR_UNSUPPORTED, "split tiles and a Toeplitz product in one pass");
                a.split_of_tile = p->split_of_tile;
                a.partials = p->partials;
                a.n_slots = p->n_slots;
                a.tile_cells = p->tile_cells;
                a.d = d;
                for (int b = 0; b < d; ++b) {
                    a.Kax[b] = int(p->K[b]);
                    a.T[b] = p->T[b];
                    a.nt[b] = p->nt[b];
                }
            }
            if (col)
                col->add(kSlotInvPass + ax, kStStrided).strided = a;
            else
                HIP_TRY(timed(p, kStridedInv, s, [&] { return launch_strided_pass(a, s); }),
                        "adjoint strided FFT pass");
            cur = dst;
        }
    }
    return NUFFT_OK;
}

int run_v(nufft_plan_s *p, const float2 *G, int grids, float2 *y, hipStream_t s, Collector *col = nullptr) {
    InterpArgs a{};
    a.geo = p->geom();
    a.om_sorted = p->om_sorted;
    a.perm = p->perm;
    a.M = p->M;
    a.G = G;
    a.grid_elems = p->grid_elems;
    a.grids = grids;
    a.y = y;
    a.items = p->staged_interp ? p->iitems : nullptr;
    a.n_items = p->n_iitems;
    a.merge = p->interp_merge;
    for (int ax = 0; ax < p->d; ++ax) {
        a.T[ax] = p->T[ax];
        a.nt[ax] = p->nt[ax];
    }
    if (col) {
        col->add(kSlotInterp, kStInterp).interp = a;
        return NUFFT_OK;
    }
    HIP_TRY(timed(p, kInterp, s, [&] { return launch_interp(a, s); }), "interpolation");
    return NUFFT_OK;
}

// reduce = false leaves split tiles as partial tiles for the first inverse FFT
// pass to sum (d >= 2 adjoint); stage_vh and 1D reduce here.
int run_vh(nufft_plan_s *p, const float2 *y, int grids, float2 *h, hipStream_t s, bool reduce = true,
           Collector *col = nullptr) {
    if (p->presort) {
        if (col)
            col->add(kSlotPermute, kStPermute).permute = PermuteJob{y, p->perm, p->M, grids, p->ysorted};
        else
            HIP_TRY(timed(p, kPermute, s,
                          [&] { return launch_permute_samples(y, p->perm, p->M, grids, p->ysorted, s); }),
                    "sort the samples");
    }
    GridArgs a{};
    a.geo = p->geom();
    a.om_sorted = p->om_sorted;
    a.perm = p->perm;
    a.sub_start = p->sub_start;
    a.M = p->M;
    for (int ax = 0; ax < p->d; ++ax) {
        a.T[ax] = p->T[ax];
        a.nt[ax] = p->nt[ax];
        a.R[ax] = p->R[ax];
    }
    a.tile_cells = p->tile_cells;
    a.seg_len = p->seg_len;
    a.segs = p->segs;
    a.group_lanes = p->group_lanes;
    a.stage_floats = p->stage_floats;
    a.chunk = p->chunk;
    a.items = p->items;
    a.n_items = p->n_items;
    a.y = p->presort ? p->ysorted : y;
    a.y_sorted = p->presort;
    a.grids = grids;
    a.h = h;
    a.n_kinds = segment_kinds(p->d, p->R, a.kinds);
    a.grid_elems = p->grid_elems;
    a.partials = p->partials;
    a.n_slots = p->n_slots;
    a.item_segs = p->item_segs;
    a.mfma = p->grid_mfma;
    a.rec_stride = p->rec_stride;
    a.blk = p->grid_blk;
    a.grid_waves = p->grid_waves;
    {
        int tsum = 0;
        for (int ax = 0; ax < p->d; ++ax) tsum += p->T[ax];
        a.grids_per_wg = p->grid_mfma ? grid_grids_per_wg(grids, p->tile_cells, tsum) : 1;
    }
    if (col)
        col->add(kSlotGrid, kStGrid).grid = a;
    else
        HIP_TRY(timed(p, kGrid, s, [&] { return launch_grid(a, s); }), "gridding");
    ReduceArgs r{};
    r.hot = p->hot;
    r.n_hot = p->n_hot;
    r.d = p->d;
    for (int ax = 0; ax < p->d; ++ax) {
        r.K[ax] = int(p->K[ax]);
        r.T[ax] = p->T[ax];
        r.nt[ax] = p->nt[ax];
    }
    r.tile_cells = p->tile_cells;
    r.partials = p->partials;
    r.n_slots = p->n_slots;
    r.h = h;
    r.grid_elems = p->grid_elems;
    r.grids = grids;
    if (p->n_hot > 0 && reduce) {
        if (col)
            col->add(kSlotReduce, kStReduce).reduce = r;
        else
            HIP_TRY(timed(p, kReduce, s, [&] { return launch_reduce_partials(r, s); }), "gridding partial sums");
    }
    return NUFFT_OK;
}

int begin_call(nufft_plan_t plan, void *stream) {
    int st = check_plan(plan);
    if (st) return st;
    HIP_TRY(hipSetDevice(plan->device), "select device");
    plan->last_stream = static_cast<hipStream_t>(stream);
    return NUFFT_OK;
}

}  // namespace

constexpr uint64_t kMultiMagic = 0x4e55464d554c5449ull;  // "NUFMULTI"
constexpr int kMultiCache = 4;  // pointer sets kept per direction

// One kernel launch of a multi-problem stage: the problems whose launches of
// one slot use the same kernel instance, with their job array and block
// table on the device.
struct MultiLaunch {
    int kind = 0;
    int threads = 0;
    bool inverse = false, split = false, staged = false;
    GridArgs proto{};  // gridding: the kernel instance
    int J = 0, d = 0;
    size_t lds = 0;
    void *jobs = nullptr;
    int4 *blocks = nullptr;
    int64_t nblocks = 0;
};

// Both directions' launches for one set of caller pointers, and their graph.
struct MultiCall {
    std::vector<const void *> in;
    std::vector<void *> out;
    std::vector<MultiLaunch> launches;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;  // recorded after each launch of exec
    bool launched = false;
    uint64_t last_use = 0;
};

struct nufft_multi_s {
    uint64_t magic = kMultiMagic;
    int device = 0;
    std::vector<nufft_plan_t> plans;
    std::vector<MultiCall> calls[2];  // [0] adjoint, [1] forward
    hipStream_t capture = nullptr;    // private stream the graphs are captured on
    uint64_t clock = 0;
};

namespace {

std::set<const void *> g_multi_registry;

int check_multi(nufft_multi_t m) {
    if (!m) return fail(NUFFT_ERR_BAD_PLAN, "multi-plan handle is NULL");
    std::lock_guard<std::mutex> lk(g_registry_mu);
    if (!g_multi_registry.count(m) || m->magic != kMultiMagic)
        return fail(NUFFT_ERR_BAD_PLAN, "multi-plan handle is not live");
    return NUFFT_OK;
}

// Frees a cached call.  Its last graph launch may still be running (calls
// return before the GPU is done): wait for it first, so no launch outlives the
// graph or the tables it reads.
void drop_call(MultiCall &mc) {
    if (mc.launched && mc.done) (void)hipEventSynchronize(mc.done);
    mc.launched = false;
    if (mc.exec) (void)hipGraphExecDestroy(mc.exec);
    if (mc.graph) (void)hipGraphDestroy(mc.graph);
    if (mc.done) (void)hipEventDestroy(mc.done);
    mc.exec = nullptr;
    mc.graph = nullptr;
    mc.done = nullptr;
    for (MultiLaunch &l : mc.launches) {
        if (l.jobs) (void)hipFree(l.jobs);
        dfree(l.blocks);
    }
    mc.launches.clear();
}

void free_multi(nufft_multi_s *m) {
    (void)hipSetDevice(m->device);
    for (auto &v : m->calls) {
        for (MultiCall &mc : v) drop_call(mc);
        v.clear();
    }
    if (m->capture) (void)hipStreamDestroy(m->capture);
    m->capture = nullptr;
}

template <class J>
hipError_t upload_jobs(const std::vector<J> &jobs, void **dev) {
    *dev = nullptr;
    hipError_t e = hipMalloc(dev, std::max<size_t>(jobs.size(), 1) * sizeof(J));
    if (e != hipSuccess || jobs.empty()) return e;
    return hipMemcpy(*dev, jobs.data(), jobs.size() * sizeof(J), hipMemcpyHostToDevice);
}

// Work blocks of one problem's launch of a stage: (job, x, y, z) per block.
// FFT stages run with the group's workgroup size `threads`.
void stage_blocks(const Emitted &em, int job, int threads, std::vector<int4> &out) {
    switch (em.kind) {
        case kStFirst: {
            const FftLaunch L = first_pass_launch(em.first, threads);
            for (int64_t b = 0; b < L.blocks; ++b) out.push_back(make_int4(job, int(b), 0, 0));
            break;
        }
        case kStStrided: {
            const FftLaunch L = strided_pass_launch(em.strided, threads);
            for (int64_t b = 0; b < L.blocks; ++b) out.push_back(make_int4(job, int(b), 0, 0));
            break;
        }
        case kStLast: {
            const FftLaunch L = last_pass_launch(em.last, threads);
            for (int64_t b = 0; b < L.blocks; ++b) out.push_back(make_int4(job, int(b), 0, 0));
            break;
        }
        case kStInterp: {
            const InterpArgs &a = em.interp;
            if (a.M == 0) break;
            const int64_t n = a.items ? a.n_items : (a.M + 255) / 256;
            for (int64_t b = 0; b < n; ++b) out.push_back(make_int4(job, int(b), 0, 0));
            break;
        }
        case kStGrid: {
            const GridArgs &a = em.grid;
            const int gp = a.mfma ? a.grids_per_wg : 1;
            for (int g = 0; g < (a.grids + gp - 1) / gp; ++g)
                for (int64_t b = 0; b < a.n_items; ++b) out.push_back(make_int4(job, int(b), g, 0));
            break;
        }
        case kStReduce: {
            const ReduceArgs &a = em.reduce;
            const int cbs = (a.tile_cells + kReduceCellsPerWg - 1) / kReduceCellsPerWg;
            for (int g = 0; g < a.grids; ++g)
                for (int cb = 0; cb < cbs; ++cb)
                    for (int64_t h = 0; h < a.n_hot; ++h) out.push_back(make_int4(job, int(h), cb, g));
            break;
        }
        case kStPermute: {
            const PermuteJob &a = em.permute;
            if (a.M == 0 || a.grids == 0) break;
            for (int64_t b = 0; b < (a.M + 255) / 256; ++b) out.push_back(make_int4(job, int(b), 0, 0));
            break;
        }
        default: break;
    }
}

// Key of the kernel instance a recorded launch uses (launches with equal keys
// in one slot share a multi-problem launch).  FFT passes share one
// workgroup size per slot (the largest any problem needs), so only the
// strided pass's direction and split-tile form separate them.
int64_t stage_key(const Emitted &em) {
    switch (em.kind) {
        case kStFirst: return 0;
        case kStStrided: {
            const bool split = em.strided.inverse && em.strided.split_of_tile != nullptr;
            return (em.strided.inverse ? 2 : 0) + (split ? 1 : 0);
        }
        case kStLast: return 0;
        case kStInterp: return em.interp.items ? 1 : 0;
        case kStGrid: return grid_variant(em.grid);
        default: return 0;
    }
}

// Builds, for caller pointers in/out, every stage launch of one direction over
// all problems, and captures them into a graph.
int build_call(nufft_multi_s *m, bool forward, const void *const *in, void *const *out, MultiCall &mc) {
    const size_t P = m->plans.size();
    std::vector<Collector> cols(P);
    for (size_t p = 0; p < P; ++p) {
        nufft_plan_s *pl = m->plans[p];
        const int C = pl->coil_mode ? pl->C : 1;
        int st;
        if (forward) {
            if ((st = run_fs(pl, plan_fft(pl), static_cast<const float2 *>(in[p]), 1, pl->grid, nullptr, nullptr,
                             &cols[p])))
                return st;
            if ((st = run_v(pl, pl->grid, C, static_cast<float2 *>(out[p]), nullptr, &cols[p]))) return st;
        } else {
            const bool fuse = pl->fuse_reduce;
            if ((st = run_vh(pl, static_cast<const float2 *>(in[p]), C, pl->grid, nullptr, !fuse, &cols[p])))
                return st;
            if ((st = run_shfh(pl, plan_fft(pl), pl->grid, 1, static_cast<float2 *>(out[p]), nullptr, fuse, nullptr,
                               &cols[p])))
                return st;
        }
    }
    for (int slot = 0; slot <= kSlotInvPass + kMaxDim; ++slot) {
        // the problems' launches of this slot, grouped by kernel instance
        std::vector<std::pair<int64_t, std::vector<const Emitted *>>> groups;
        for (size_t p = 0; p < P; ++p)
            for (const Emitted &em : cols[p].out) {
                if (em.slot != slot) continue;
                const int64_t key = stage_key(em) * 16 + em.kind;
                if (stage_key(em) < 0) return fail(NUFFT_ERR_UNSUPPORTED, "no multi-problem kernel for a stage");
                auto it = std::find_if(groups.begin(), groups.end(), [&](const auto &g) { return g.first == key; });
                if (it == groups.end()) {
                    groups.push_back({key, {}});
                    it = groups.end() - 1;
                }
                it->second.push_back(&em);
            }
        for (auto &grp : groups) {
            const std::vector<const Emitted *> &ems = grp.second;
            MultiLaunch L;
            L.kind = ems[0]->kind;
            // FFT passes: the largest workgroup size any problem of the group
            // takes on its own, given to all of them
            for (const Emitted *em : ems) {
                if (L.kind == kStFirst) L.threads = std::max(L.threads, first_pass_launch(em->first).threads);
                if (L.kind == kStStrided) L.threads = std::max(L.threads, strided_pass_launch(em->strided).threads);
                if (L.kind == kStLast) L.threads = std::max(L.threads, last_pass_launch(em->last).threads);
            }
            // blocks of every problem, dealt round-robin (each problem's own
            // launch order is longest work first, so the merged order is too,
            // roughly, and the heavy blocks spread over the XCDs)
            std::vector<std::vector<int4>> per(ems.size());
            for (size_t j = 0; j < ems.size(); ++j) stage_blocks(*ems[j], int(j), L.threads, per[j]);
            std::vector<int4> blocks;
            for (size_t r = 0;; ++r) {
                bool any = false;
                for (auto &v : per)
                    if (r < v.size()) {
                        blocks.push_back(v[r]);
                        any = true;
                    }
                if (!any) break;
            }
            if (blocks.empty()) continue;
            hipError_t e = hipSuccess;
            switch (L.kind) {
                case kStFirst: {
                    std::vector<FirstJob> jobs;
                    for (const Emitted *em : ems) {
                        const FftLaunch fl = first_pass_launch(em->first, L.threads);
                        jobs.push_back(FirstJob{em->first, fl.p0});
                        L.lds = std::max(L.lds, fl.lds);
                    }
                    e = upload_jobs(jobs, &L.jobs);
                    break;
                }
                case kStStrided: {
                    std::vector<StridedJob> jobs;
                    for (const Emitted *em : ems) {
                        const FftLaunch fl = strided_pass_launch(em->strided, L.threads);
                        jobs.push_back(StridedJob{em->strided, fl.p0, fl.p1});
                        L.lds = std::max(L.lds, fl.lds);
                        L.inverse = em->strided.inverse;
                        L.split = em->strided.inverse && em->strided.split_of_tile != nullptr;
                    }
                    e = upload_jobs(jobs, &L.jobs);
                    break;
                }
                case kStLast: {
                    std::vector<LastJob> jobs;
                    for (const Emitted *em : ems) {
                        const FftLaunch fl = last_pass_launch(em->last, L.threads);
                        jobs.push_back(LastJob{em->last, fl.p0, int(fl.p1)});
                        L.lds = std::max(L.lds, fl.lds);
                    }
                    e = upload_jobs(jobs, &L.jobs);
                    break;
                }
                case kStInterp: {
                    std::vector<InterpArgs> jobs;
                    for (const Emitted *em : ems) {
                        jobs.push_back(em->interp);
                        L.staged = em->interp.items != nullptr;
                        L.J = em->interp.geo.J;
                        L.d = em->interp.geo.d;
                        L.lds = std::max(L.lds, interp_lds(em->interp));
                    }
                    e = upload_jobs(jobs, &L.jobs);
                    break;
                }
                case kStGrid: {
                    std::vector<GridArgs> jobs;
                    for (const Emitted *em : ems) {
                        jobs.push_back(em->grid);
                        L.proto = em->grid;
                        L.lds = std::max(L.lds, grid_lds(em->grid));
                    }
                    e = upload_jobs(jobs, &L.jobs);
                    break;
                }
                case kStReduce: {
                    std::vector<ReduceArgs> jobs;
                    for (const Emitted *em : ems) jobs.push_back(em->reduce);
                    e = upload_jobs(jobs, &L.jobs);
                    break;
                }
                case kStPermute: {
                    std::vector<PermuteJob> jobs;
                    for (const Emitted *em : ems) jobs.push_back(em->permute);
                    e = upload_jobs(jobs, &L.jobs);
                    break;
                }
                default: break;
            }
            if (e == hipSuccess) e = upload(&L.blocks, blocks);
            L.nblocks = int64_t(blocks.size());
            mc.launches.push_back(L);
            if (e != hipSuccess) return hip_fail(e, "upload multi-problem tables");
        }
    }
    return NUFFT_OK;
}

hipError_t issue(const MultiLaunch &L, hipStream_t s) {
    switch (L.kind) {
        case kStFirst:
            return launch_first_pass_multi(static_cast<const FirstJob *>(L.jobs), L.blocks, L.nblocks, L.threads,
                                           L.lds, s);
        case kStStrided:
            return launch_strided_pass_multi(static_cast<const StridedJob *>(L.jobs), L.blocks, L.nblocks, L.threads,
                                             L.inverse, L.split, L.lds, s);
        case kStLast:
            return launch_last_pass_multi(static_cast<const LastJob *>(L.jobs), L.blocks, L.nblocks, L.threads, L.lds,
                                          s);
        case kStInterp:
            return launch_interp_multi(static_cast<const InterpArgs *>(L.jobs), L.blocks, L.nblocks, L.J, L.d,
                                       L.staged, L.lds, s);
        case kStGrid:
            return launch_grid_multi(static_cast<const GridArgs *>(L.jobs), L.blocks, L.nblocks, L.proto, L.lds, s);
        case kStReduce:
            return launch_reduce_partials_multi(static_cast<const ReduceArgs *>(L.jobs), L.blocks, L.nblocks, s);
        case kStPermute:
            return launch_permute_samples_multi(static_cast<const PermuteJob *>(L.jobs), L.blocks, L.nblocks, s);
        default: return hipErrorInvalidValue;
    }
}

// Run all P transforms of one direction on `user`: one launch per stage and
// kernel instance over every problem, captured into a graph the first time
// these pointers are seen (kept for kMultiCache pointer sets), then replayed.
int multi_run(nufft_multi_s *m, bool forward, const void *const *in, void *const *out, hipStream_t user) {
    const size_t P = m->plans.size();
    if (!in || !out) return fail(NUFFT_ERR_INVALID_ARG, "pointer arrays are NULL");
    for (size_t p = 0; p < P; ++p)
        if (!in[p] || !out[p]) return fail(NUFFT_ERR_INVALID_ARG, "pointer %zu is NULL", p);
    HIP_TRY(hipSetDevice(m->device), "select device");
    std::vector<MultiCall> &cache = m->calls[forward ? 1 : 0];
    MultiCall *mc = nullptr;
    for (MultiCall &c : cache) {
        bool hit = true;
        for (size_t p = 0; hit && p < P; ++p) hit = c.in[p] == in[p] && c.out[p] == out[p];
        if (hit) {
            mc = &c;
            break;
        }
    }
    if (!mc) {
        if (cache.size() >= size_t(kMultiCache)) {  // evict the least recently used pointer set
            auto lru = std::min_element(cache.begin(), cache.end(),
                                        [](const MultiCall &a, const MultiCall &b) { return a.last_use < b.last_use; });
            drop_call(*lru);
            cache.erase(lru);
        }
        cache.emplace_back();
        mc = &cache.back();
        mc->in.assign(in, in + P);
        mc->out.assign(out, out + P);
        int st = build_call(m, forward, in, out, *mc);
        if (st == NUFFT_OK) {
            hipError_t e = hipStreamBeginCapture(m->capture, hipStreamCaptureModeThreadLocal);
            for (size_t k = 0; e == hipSuccess && k < mc->launches.size(); ++k) e = issue(mc->launches[k], m->capture);
            hipGraph_t graph = nullptr;
            hipError_t e2 = hipStreamEndCapture(m->capture, &graph);
            mc->graph = graph;
            if (e == hipSuccess) e = e2;
            if (e == hipSuccess) e = hipGraphInstantiate(&mc->exec, graph, nullptr, nullptr, 0);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&mc->done, hipEventDisableTiming);
            if (e != hipSuccess) st = hip_fail(e, "capture the multi-problem launches");
        }
        if (st) {
            std::string msg = g_last_error;
            drop_call(*mc);
            cache.pop_back();
            g_last_error = msg;
            return st;
        }
    }
    mc->last_use = ++m->clock;
    HIP_TRY(hipGraphLaunch(mc->exec, user), "launch the multi-problem graph");
    HIP_TRY(hipEventRecord(mc->done, user), "record graph completion");
    mc->launched = true;
    return NUFFT_OK;
}

}  // namespace

constexpr uint64_t kToeplitzMagic = 0x4e5546544f45504cull;  // "NUFTOEPL"

struct nufft_toeplitz_s {
    uint64_t magic = kToeplitzMagic;
    nufft_plan_t plan = nullptr;
    int d = 1;
    int64_t N[kMaxDim] = {1, 1, 1};
    int64_t P[kMaxDim] = {1, 1, 1};  // 2N
    int64_t elems = 1;               // prod(2N)
    RadixPlan rp[kMaxDim];
    float2 *tw[kMaxDim] = {nullptr, nullptr, nullptr};
    float *ones[kMaxDim] = {nullptr, nullptr, nullptr};
    float *inv[kMaxDim] = {nullptr, nullptr, nullptr};  // 1 / (2 N_a)
    float2 *phat = nullptr;   // [prod(2N)]
    int cap = 0;              // grids the workspace holds
    float2 *grid = nullptr;   // pass buffers, [cap][prod(2N)] each
    float2 *tmp = nullptr;
    float2 *grid2 = nullptr;  // the spectrum between the forward and inverse passes
};

namespace {

std::set<const void *> g_toeplitz_registry;

int check_toeplitz(nufft_toeplitz_t t) {
    if (!t) return fail(NUFFT_ERR_BAD_PLAN, "Toeplitz handle is NULL");
    std::lock_guard<std::mutex> lk(g_registry_mu);
    if (!g_toeplitz_registry.count(t) || t->magic != kToeplitzMagic)
        return fail(NUFFT_ERR_BAD_PLAN, "Toeplitz handle is not live");
    return NUFFT_OK;
}

void destroy_toeplitz(nufft_toeplitz_s *t) {
    for (int a = 0; a < kMaxDim; ++a) {
        dfree(t->tw[a]);
        dfree(t->ones[a]);
        dfree(t->inv[a]);
    }
    dfree(t->phat);
    dfree(t->grid);
    dfree(t->tmp);
    dfree(t->grid2);
}

int ensure_toeplitz_workspace(nufft_toeplitz_s *t, int grids) {
    if (grids <= t->cap) return NUFFT_OK;
    dfree(t->grid);
    dfree(t->tmp);
    dfree(t->grid2);
    t->cap = 0;
    const size_t n = size_t(grids) * size_t(t->elems);
    HIP_TRY(dmalloc(&t->grid, n), "allocate Toeplitz workspace");
    HIP_TRY(dmalloc(&t->tmp, n), "allocate Toeplitz workspace");
    HIP_TRY(dmalloc(&t->grid2, n), "allocate Toeplitz workspace");
    t->cap = grids;
    return NUFFT_OK;
}

// psf = true: image = grid = 2N, scale 1/(2N_a) (the point-spread function's
// transform); false: image N on grid 2N, no scaling (the application).
FftGeom toeplitz_fft(const nufft_toeplitz_s *t, bool psf) {
    FftGeom f;
    f.d = t->d;
    for (int a = 0; a < t->d; ++a) {
        f.N[a] = psf ? t->P[a] : t->N[a];
        f.K[a] = t->P[a];
    }
    f.rp = t->rp;
    f.tw = t->tw;
    f.scale = psf ? t->inv : t->ones;
    f.grid = t->grid;
    f.tmp = t->tmp;
    f.fft_groups = t->plan->fft_groups;
    return f;
}

}  // namespace

extern "C" {

int nufft_multi_plan(int P, const nufft_problem_t *probs, void *stream, nufft_multi_t *out) {
    if (!out) return fail(NUFFT_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (P < 1 || P > 256 || !probs) return fail(NUFFT_ERR_INVALID_ARG, "P=%d must be in [1, 256]", P);
    for (int p = 1; p < P; ++p)
        if (probs[p].d != probs[0].d || probs[p].J != probs[0].J)
            return fail(NUFFT_ERR_UNSUPPORTED, "problem %d has a different d or J", p);
    nufft_multi_s *m = new (std::nothrow) nufft_multi_s();
    if (!m) return fail(NUFFT_ERR_OOM, "host allocation failed");
    auto bail = [&](int st) {
        std::string msg = g_last_error;
        free_multi(m);
        for (auto pl : m->plans) (void)nufft_destroy(pl);
        delete m;
        g_last_error = msg;
        return st;
    };
    (void)hipGetDevice(&m->device);
    for (int p = 0; p < P; ++p) {
        const nufft_problem_t &pr = probs[p];
        nufft_plan_t h = nullptr;
        int st = nufft_plan_ex(pr.d, pr.N, pr.K, pr.J, pr.M, pr.om, pr.opt, stream, &h);
        if (st) return bail(st);
        m->plans.push_back(h);
        if (pr.C > 0) {
            st = nufft_set_coils(h, pr.C, pr.coils);
            if (st) return bail(st);
        }
        // the multi-problem launches read each plan's workspace for its C grids
        st = ensure_workspace(h, pr.C > 0 ? pr.C : 1);
        if (st) return bail(st);
    }
    hipError_t e = hipStreamCreateWithFlags(&m->capture, hipStreamNonBlocking);
    if (e != hipSuccess) return bail(hip_fail(e, "create capture stream"));
    {
        std::lock_guard<std::mutex> lk(g_registry_mu);
        g_multi_registry.insert(m);
    }
    *out = m;
    return NUFFT_OK;
}

int nufft_multi_forward(nufft_multi_t m, const void *const *x_dev, void *const *y_dev, void *stream) {
    int st = check_multi(m);
    if (st) return st;
    return multi_run(m, true, x_dev, y_dev, static_cast<hipStream_t>(stream));
}

int nufft_multi_adjoint(nufft_multi_t m, const void *const *y_dev, void *const *x_dev, void *stream) {
    int st = check_multi(m);
    if (st) return st;
    return multi_run(m, false, y_dev, x_dev, static_cast<hipStream_t>(stream));
}

int nufft_multi_info(nufft_multi_t m, int64_t *launches_fwd, int64_t *launches_adj) {
    int st = check_multi(m);
    if (st) return st;
    for (int dir = 0; dir < 2; ++dir) {
        int64_t *dst = dir ? launches_fwd : launches_adj;
        if (!dst) continue;
        *dst = -1;
        const MultiCall *last = nullptr;
        for (const MultiCall &c : m->calls[dir])
            if (!last || c.last_use > last->last_use) last = &c;
        if (last) *dst = int64_t(last->launches.size());
    }
    return NUFFT_OK;
}

int nufft_multi_destroy(nufft_multi_t m) {
    int st = check_multi(m);
    if (st) return st;
    {
        std::lock_guard<std::mutex> lk(g_registry_mu);
        g_multi_registry.erase(m);
    }
    (void)hipSetDevice(m->device);
    (void)hipDeviceSynchronize();
    free_multi(m);  // graphs, tables and the capture stream first, the plans they read last
    for (auto pl : m->plans) (void)nufft_destroy(pl);
    m->plans.clear();
    m->magic = 0;
    delete m;
    return NUFFT_OK;
}

const char *nufft_status_string(int status) {
    switch (status) {
        case NUFFT_OK: return "success";
        case NUFFT_ERR_INVALID_ARG: return "invalid argument";
        case NUFFT_ERR_NO_DEVICE: return "no HIP device";
        case NUFFT_ERR_OOM: return "device out of memory";
        case NUFFT_ERR_HIP: return "HIP runtime error";
        case NUFFT_ERR_BAD_PLAN: return "bad plan handle";
        case NUFFT_ERR_NONFINITE: return "non-finite trajectory coordinate";
        case NUFFT_ERR_UNSUPPORTED: return "unsupported configuration";
        default: return "unknown status";
    }
}

const char *nufft_last_error(void) { return g_last_error.c_str(); }

int nufft_device_count(void) {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) return 0;
    return n;
}

int nufft_kernel_weights_host(int J, double sigma, int64_t n, const double *f, double *w, double *dw) {
    if (J < 2 || J > kMaxJ) return fail(NUFFT_ERR_INVALID_ARG, "J=%d outside [2, %d]", J, kMaxJ);
    if (!(sigma >= 1.0) || !(sigma < 1e6)) return fail(NUFFT_ERR_INVALID_ARG, "sigma must be >= 1");
    if (n < 0 || (n > 0 && (!f || !w))) return fail(NUFFT_ERR_INVALID_ARG, "bad arrays");
    AxisKernel k;
    if (!kb_fit(J, kb_beta(J, sigma), &k)) return fail(NUFFT_ERR_UNSUPPORTED, "kernel fit did not converge");
    float wf[kMaxJ], dwf[kMaxJ];
    for (int64_t i = 0; i < n; ++i) {
        kb_eval_fit(k, J, float(f[i]), wf, dwf);
        for (int j = 0; j < J; ++j) {
            w[i * J + j] = wf[j];
            if (dw) dw[i * J + j] = dwf[j];
        }
    }
    return NUFFT_OK;
}

int nufft_plan(int d, const int64_t *N, const int64_t *K, int J, int64_t M, const float *om_dev, void *stream,
               nufft_plan_t *out) {
    return nufft_plan_ex(d, N, K, J, M, om_dev, nullptr, stream, out);
}

int nufft_plan_ex(int d, const int64_t *N, const int64_t *K, int J, int64_t M, const float *om_dev,
                  const nufft_options_t *opt, void *stream, nufft_plan_t *out) {
    if (!out) return fail(NUFFT_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (d < 1 || d > kMaxDim) return fail(NUFFT_ERR_INVALID_ARG, "d=%d must be 1, 2 or 3", d);
    if (!N || !K) return fail(NUFFT_ERR_INVALID_ARG, "N or K is NULL");
    if (J < 2 || J > kMaxJ) return fail(NUFFT_ERR_INVALID_ARG, "J=%d outside [2, %d]", J, kMaxJ);
    if (M < 0 || M >= (int64_t(1) << 31)) return fail(NUFFT_ERR_INVALID_ARG, "M=%lld out of range", (long long)M);
    if (M > 0 && !om_dev) return fail(NUFFT_ERR_INVALID_ARG, "om is NULL with M > 0");
    int64_t img = 1, grd = 1;
    for (int a = 0; a < d; ++a) {
        if (N[a] < 2 || N[a] % 2) return fail(NUFFT_ERR_INVALID_ARG, "N[%d]=%lld must be even and >= 2", a, (long long)N[a]);
        if (K[a] < N[a] || K[a] % 2) return fail(NUFFT_ERR_INVALID_ARG, "K[%d]=%lld must be even and >= N", a, (long long)K[a]);
        if (K[a] > 4096) return fail(NUFFT_ERR_UNSUPPORTED, "K[%d]=%lld above 4096", a, (long long)K[a]);
        if (!smooth235(K[a])) return fail(NUFFT_ERR_UNSUPPORTED, "K[%d]=%lld has a prime factor above 5", a, (long long)K[a]);
        if (J > K[a]) return fail(NUFFT_ERR_INVALID_ARG, "J=%d exceeds K[%d]", J, a);
        img *= N[a];
        grd *= K[a];
    }
    if (grd >= (int64_t(1) << 31)) return fail(NUFFT_ERR_UNSUPPORTED, "grid of %lld cells too large", (long long)grd);
    int ndev = 0;
    hipError_t de = hipGetDeviceCount(&ndev);
    if (de != hipSuccess || ndev <= 0)
        return fail(NUFFT_ERR_NO_DEVICE, "no HIP device visible (hipGetDeviceCount: %s, count %d)", hipGetErrorString(de),
                    ndev);

    nufft_plan_s *p = new (std::nothrow) nufft_plan_s();
    if (!p) return fail(NUFFT_ERR_OOM, "host allocation failed");
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto bail = [&](int st) {
        std::string msg = g_last_error;
        free_plan(p);
        delete p;
        g_last_error = msg;
        return st;
    };
    if (hipGetDevice(&p->device) != hipSuccess) return bail(fail(NUFFT_ERR_HIP, "hipGetDevice failed"));
    p->d = d;
    p->J = J;
    p->M = M;
    p->img_elems = img;
    p->grid_elems = grd;
    for (int a = 0; a < d; ++a) {
        p->N[a] = N[a];
        p->K[a] = K[a];
    }
    // kernel, scaling and FFT constants per axis
    // tile edges: the last axis (one register row per lane in the gridding) at
    // most 32 cells, the leading axes at most 64 rows in all
    const int targets[3][3] = {{32, 1, 1}, {32, 16, 1}, {8, 8, 16}};
    const int need = J - 1;
    p->tile_cells = 1;
    p->nbins = 1;
    if (opt && opt->interp_merge < 0) return bail(fail(NUFFT_ERR_INVALID_ARG, "interp_merge negative"));
    if (opt && (opt->interpolator < 0 || opt->interpolator > 1))
        return bail(fail(NUFFT_ERR_INVALID_ARG, "interpolator takes 0 (Kaiser-Bessel) or 1 (min-max)"));
    p->minmax = opt && opt->interpolator == 1;
    if (opt && (opt->reserved[0] || opt->reserved[1]))
        return bail(fail(NUFFT_ERR_INVALID_ARG, "reserved option fields must be 0"));
    if (opt && (opt->fft_radix < 0 || opt->fft_radix > 3))
        return bail(fail(NUFFT_ERR_INVALID_ARG, "fft_radix takes 0, 1, 2 or 3"));
    if (opt && opt->grid_waves != 0 && opt->grid_waves != 1 && opt->grid_waves != 4)
        return bail(fail(NUFFT_ERR_INVALID_ARG, "grid_waves takes 0, 1 or 4"));
    p->grid_waves = (opt && opt->grid_waves == 1) ? 1 : 4;
    if (opt && (opt->weight_table < 0 || opt->weight_table > 1))
        return bail(fail(NUFFT_ERR_INVALID_ARG, "weight_table takes 0 or 1"));
    p->use_wtab = opt && opt->weight_table == 1;
    if (p->use_wtab && p->minmax)
        return bail(fail(NUFFT_ERR_UNSUPPORTED, "the window table holds Kaiser-Bessel weights only"));
    for (int a = 0; a < d; ++a) {
        const double beta = kb_beta(J, double(K[a]) / double(N[a]));
        if (p->minmax ? !minmax_fit(int(N[a]), int(K[a]), J, beta, &p->ker[a]) : !kb_fit(J, beta, &p->ker[a]))
            return bail(fail(NUFFT_ERR_UNSUPPORTED, "kernel polynomial fit did not converge"));
        if (!radix_plan(int(K[a]), &p->rp[a], opt ? opt->fft_radix : 0))
            return bail(fail(NUFFT_ERR_UNSUPPORTED, "no radix plan for K"));
        const int target = (opt && opt->tile[a] > 0) ? opt->tile[a] : targets[d - 1][a];
        p->T[a] = choose_tile(K[a], target, std::max(1, need));
        p->nt[a] = int(K[a] / p->T[a]);
        p->R[a] = p->nt[a] > 1 ? 2 : 1;
        p->tile_cells *= p->T[a];
        p->nbins *= p->nt[a];
        int st;
        hipError_t e;
        if ((e = upload(&p->scale[a], p->minmax ? minmax_scaling(int(N[a]), int(K[a]), J, beta)
                                                : kb_scaling(int(N[a]), int(K[a]), J, beta))) != hipSuccess ||
            (p->minmax && (e = upload(&p->phase[a], half_phase(int(K[a])))) != hipSuccess) ||
            (e = upload(&p->tw[a], twiddles(int(K[a])))) != hipSuccess ||
            (e = upload(&p->coef[a], coef_rows(p->ker[a].coef, J, p->ker[a].deg, coef_row_width(J), &p->nq[a]))) !=
                hipSuccess ||
            (e = upload(&p->dcoef[a], coef_rows(p->ker[a].dcoef, J, p->ker[a].deg_d, coef_row_width(J),
                                                &p->nq_d[a]))) != hipSuccess) {
            st = hip_fail(e, "upload plan constants");
            return bail(st);
        }
    }
    {
        // gridding: each lane accumulates LS cells of one tile row in registers;
        // the smallest LS in {4, 8, 16} that keeps the tile within one
        // wavefront (most lanes busy), else within the workgroup
        const int L = p->T[d - 1];
        const int rows = p->tile_cells / L;
        int ls = 0;
        for (int lim : {64, 256}) {
            for (int cand : {4, 8, 16})
                if (rows * ((L + cand - 1) / cand) <= lim) {
                    ls = cand;
                    break;
                }
            if (ls) break;
        }
        // 3D tiles of 16 cells on the last axis, 8 or 16 on the others and at
        // most 128 leading cells: the matrix cores by 4 x 4 blocks (default; grid_mfma = 3 asks for the
        // row-tile matrix-core kernel instead, 2 for the vector ALUs)
        if (opt && (opt->grid_mfma < 0 || opt->grid_mfma > 3))
            return bail(fail(NUFFT_ERR_INVALID_ARG, "grid_mfma takes 0, 1, 2 or 3"));
        const bool blk_ok = d == 3 && L == 16 && (p->T[0] == 8 || p->T[0] == 16) &&
                            (p->T[1] == 8 || p->T[1] == 16) && p->T[0] * p->T[1] <= 128;
        p->grid_blk = blk_ok && !(opt && (opt->grid_mfma == 2 || opt->grid_mfma == 3));
        if (p->grid_blk) ls = 16;
        if (!ls) return bail(fail(NUFFT_ERR_UNSUPPORTED, "no gridding tile shape for this K and J"));
        p->seg_len = ls;
        p->segs = (L + ls - 1) / ls;
        const int lanes = rows * p->segs;
        // a group size that divides the 256-thread workgroup (192 would leave
        // 64 threads without a staging area)
        p->group_lanes = lanes <= 64 ? 64 : lanes <= 128 ? 128 : 256;
        const int B = p->group_lanes;
        const int Lp = p->segs * ls;
        const int staged = B * Lp + 2 * (B + 1) + (d - 1) * (B + 1) + (d - 1) * J * (B + 1);
        p->stage_floats = std::max(staged, 2 * rows * Lp);
        p->stage_floats = (p->stage_floats + 3) & ~3;  // keep every group's rows 16-byte aligned
        if (!p->grid_blk && int64_t(256 / p->group_lanes) * p->stage_floats * int64_t(sizeof(float)) > kLdsBudget)
            return bail(fail(NUFFT_ERR_UNSUPPORTED, "gridding tile too large for LDS"));
        // matrix-core gridding by row tiles: 16 cells on the last axis and 16,
        // 32 or 64 rows (default where the tile allows it and the block kernel
        // does not apply)
        int tsum = 0;
        for (int a = 0; a < d; ++a) tsum += p->T[a];
        p->rec_stride = (2 + tsum) | 1;  // value + the tile's coordinates per axis, odd (no bank conflicts)
        const bool mfma_ok = d >= 2 && L == 16 && (rows == 16 || rows == 32 || rows == 64) &&
                             int64_t(4) * 64 * p->rec_stride * int64_t(sizeof(float)) <= kLdsBudget;
        if (opt && (opt->grid_mfma == 1 || opt->grid_mfma == 3) && !mfma_ok && !p->grid_blk)
            return bail(fail(NUFFT_ERR_UNSUPPORTED,
                             "matrix-core gridding needs T_last = 16, 16, 32 or 64 rows and sum(T) <= 61"));
        p->grid_mfma = !p->grid_blk && mfma_ok && !(opt && opt->grid_mfma == 2);
    }
    {
        const int64_t region = interp_region_elems(d, p->T, J, 1) * int64_t(sizeof(float2));
        p->staged_interp = region <= kLdsBudget && !(opt && opt->interp_direct);
        // Runs of sparse tiles per gather item: measured, longer items cost
        // the latency-bound 2D workload more than the staging they save, the
        // 3D one gains from pairs.  Cut to what fits the gather's LDS.
        const int want = (opt && opt->interp_merge > 0) ? opt->interp_merge : (d == 3 ? 2 : 1);
        p->interp_merge = 1;
        while (p->interp_merge < std::min(want, p->nt[d - 1]) &&
               interp_region_elems(d, p->T, J, p->interp_merge + 1) * int64_t(sizeof(float2)) <= kInterpLdsBudget)
            ++p->interp_merge;
    }
    if ((p->nbins << d) >= (int64_t(1) << 30)) return bail(fail(NUFFT_ERR_UNSUPPORTED, "too many bins"));
    p->chunk = d == 3 ? 1024 : 512;
    if (opt && opt->grid_chunk > 0) {
        if (opt->grid_chunk < 64) return bail(fail(NUFFT_ERR_INVALID_ARG, "grid_chunk below 64"));
        p->chunk = opt->grid_chunk;
    }
    if (opt && opt->fft_groups < 0) return bail(fail(NUFFT_ERR_INVALID_ARG, "fft_groups negative"));
    p->fft_groups = (opt && opt->fft_groups > 0) ? opt->fft_groups : 1024;
    if (opt && (opt->presort < 0 || opt->presort > 2 || opt->fuse_reduce < 0 || opt->fuse_reduce > 2))
        return bail(fail(NUFFT_ERR_INVALID_ARG, "presort and fuse_reduce take 0, 1 or 2"));
    // Defaults from measurement: in 3D the gridding's dependent loads through
    // the permutation cost more than one permute launch; in 2D they do not.
    p->presort = (opt && opt->presort) ? opt->presort == 1 : d == 3;
    // Default from measurement: fused in 2D (saves a launch on a latency-bound
    // problem), apart in 3D (the fused pass's extra registers cost occupancy).
    p->fuse_reduce = d >= 2 && ((opt && opt->fuse_reduce) ? opt->fuse_reduce == 1 : d == 2);
    // the fused pass divides column indices c < K_1 K_2 by K_2 with a 32-bit
    // high multiply, exact while K_1 K_2^2 < 2^32
    if (d == 3 && double(K[1]) * double(K[2]) * double(K[2]) >= 4294967296.0) p->fuse_reduce = false;
    // intermediate sizes of the FFT passes that land in the tmp buffer
    p->tmp_elems = 1;
    for (int pass = 0; pass < d - 1; ++pass) {
        const int ax = d - 1 - pass;
        if ((d - 1 - pass) % 2 != 0) {
            int64_t e = 1;
            for (int b = 0; b < d; ++b) e *= (b < ax) ? N[b] : K[b];
            p->tmp_elems = std::max(p->tmp_elems, e);
        }
    }
    for (int ax = 0; ax < d - 1; ++ax) {
        if (ax % 2 == 0) {
            int64_t e = 1;
            for (int b = 0; b < d; ++b) e *= (b <= ax) ? N[b] : K[b];
            p->tmp_elems = std::max(p->tmp_elems, e);
        }
    }
    {
        hipError_t e;
        if ((e = dmalloc(&p->om, size_t(std::max<int64_t>(M, 1)) * d)) != hipSuccess ||
            (e = dmalloc(&p->om_sorted, size_t(std::max<int64_t>(M, 1)) * d)) != hipSuccess ||
            (e = dmalloc(&p->perm, size_t(std::max<int64_t>(M, 1)))) != hipSuccess ||
            (e = dmalloc(&p->om_prev, size_t(std::max<int64_t>(M, 1)) * d)) != hipSuccess)
            return bail(hip_fail(e, "allocate trajectory"));
        // binning scratch: keys, sorted keys, identity, sub-bin counts, flag and
        // the radix sort's temporary storage, kept for every later re-bin
        const size_t m1 = size_t(std::max<int64_t>(M, 1));
        if ((e = dmalloc(&p->bkeys, m1)) != hipSuccess || (e = dmalloc(&p->bkeys_sorted, m1)) != hipSuccess ||
            (e = dmalloc(&p->biota, m1)) != hipSuccess ||
            (e = dmalloc(&p->bcounts, size_t(p->nbins << d))) != hipSuccess ||
            (e = dmalloc(&p->bflag, 1)) != hipSuccess ||
            (e = sort_pairs_temp_bytes(M, bits_for(p->nbins << d), &p->sort_temp_bytes)) != hipSuccess ||
            (e = hipMalloc(&p->sort_temp, std::max<size_t>(p->sort_temp_bytes, 1))) != hipSuccess)
            return bail(hip_fail(e, "allocate binning scratch"));
    }
    int st = bin_points(p, om_dev, s);
    if (st) return bail(st);
    st = ensure_workspace(p, 1);
    if (st) return bail(st);
    {
        std::lock_guard<std::mutex> lk(g_registry_mu);
        g_registry.insert(p);
    }
    *out = p;
    return NUFFT_OK;
}

int nufft_set_points(nufft_plan_t plan, const float *om_dev, void *stream) {
    int st = check_plan(plan);
    if (st) return st;
    const hipStream_t prev_stream = plan->last_stream;
    st = begin_call(plan, stream);
    if (st) return st;
    if (plan->M > 0 && !om_dev) return fail(NUFFT_ERR_INVALID_ARG, "om is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    // The tables below are rewritten in place: wait for the plan's previous
    // call (possibly on another stream) first.  Keep the previous trajectory
    // if the new one is rejected.
    if (prev_stream && prev_stream != s) HIP_TRY(hipStreamSynchronize(prev_stream), "wait for the previous call");
    const size_t bytes = size_t(plan->M) * plan->d * sizeof(float);
    if (plan->M > 0) HIP_TRY(hipMemcpyAsync(plan->om_prev, plan->om, bytes, hipMemcpyDeviceToDevice, s),
                             "backup trajectory");
    st = bin_points(plan, om_dev, s);
    if (st) {
        std::string msg = g_last_error;
        (void)bin_points(plan, plan->om_prev, s);
        g_last_error = msg;
        return st;
    }
    return ensure_workspace(plan, std::max(plan->cap_grids, 1));
}

int nufft_set_coils(nufft_plan_t plan, int C, const void *c_dev) {
    int st = check_plan(plan);
    if (st) return st;
    if (C < 0 || (C > 0 && !c_dev)) return fail(NUFFT_ERR_INVALID_ARG, "bad coil arguments");
    HIP_TRY(hipSetDevice(plan->device), "select device");
    HIP_TRY(hipDeviceSynchronize(), "synchronise before changing coils");
    dfree(plan->coils);
    if (C == 0) {
        plan->coil_mode = false;
        plan->C = 1;
        return NUFFT_OK;
    }
    HIP_TRY(dmalloc(&plan->coils, size_t(C) * plan->img_elems), "allocate coil maps");
    HIP_TRY(hipMemcpy(plan->coils, c_dev, size_t(C) * plan->img_elems * sizeof(float2), hipMemcpyDeviceToDevice),
            "copy coil maps");
    plan->coil_mode = true;
    plan->C = C;
    return ensure_workspace(plan, C);
}

int nufft_reserve(nufft_plan_t plan, int B) {
    int st = check_plan(plan);
    if (st) return st;
    if (B < 1) return fail(NUFFT_ERR_INVALID_ARG, "B must be >= 1");
    HIP_TRY(hipSetDevice(plan->device), "select device");
    const int C = plan->coil_mode ? plan->C : 1;
    return ensure_workspace(plan, B * C);
}

int nufft_forward_batched(nufft_plan_t plan, int B, const void *x_dev, void *y_dev, void *stream) {
    int st = begin_call(plan, stream);
    if (st) return st;
    if (B < 1) return fail(NUFFT_ERR_INVALID_ARG, "B must be >= 1");
    if (!x_dev || (!y_dev && plan->M > 0)) return fail(NUFFT_ERR_INVALID_ARG, "NULL data pointer");
    const int C = plan->coil_mode ? plan->C : 1;
    if ((st = ensure_workspace(plan, B * C))) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((st = run_fs(plan, plan_fft(plan), static_cast<const float2 *>(x_dev), B, plan->grid, s))) return st;
    return run_v(plan, plan->grid, B * C, static_cast<float2 *>(y_dev), s);
}

int nufft_adjoint_batched(nufft_plan_t plan, int B, const void *y_dev, void *x_dev, void *stream) {
    int st = begin_call(plan, stream);
    if (st) return st;
    if (B < 1) return fail(NUFFT_ERR_INVALID_ARG, "B must be >= 1");
    if (!x_dev || (!y_dev && plan->M > 0)) return fail(NUFFT_ERR_INVALID_ARG, "NULL data pointer");
    const int C = plan->coil_mode ? plan->C : 1;
    if ((st = ensure_workspace(plan, B * C))) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool fuse = plan->fuse_reduce;
    if ((st = run_vh(plan, static_cast<const float2 *>(y_dev), B * C, plan->grid, s, !fuse))) return st;
    return run_shfh(plan, plan_fft(plan), plan->grid, B, static_cast<float2 *>(x_dev), s, fuse);
}

int nufft_forward(nufft_plan_t plan, const void *x_dev, void *y_dev, void *stream) {
    return nufft_forward_batched(plan, 1, x_dev, y_dev, stream);
}

int nufft_adjoint(nufft_plan_t plan, const void *y_dev, void *x_dev, void *stream) {
    return nufft_adjoint_batched(plan, 1, y_dev, x_dev, stream);
}

int nufft_grad_points_batched(nufft_plan_t plan, int B, const void *x_dev, const void *gy_dev, float *gom_dev,
                              void *stream) {
    int st = begin_call(plan, stream);
    if (st) return st;
    if (plan->minmax) return fail(NUFFT_ERR_UNSUPPORTED, "trajectory gradients need the Kaiser-Bessel interpolator");
    if (B < 1) return fail(NUFFT_ERR_INVALID_ARG, "B must be >= 1");
    if (!x_dev || ((!gy_dev || !gom_dev) && plan->M > 0)) return fail(NUFFT_ERR_INVALID_ARG, "NULL data pointer");
    const int C = plan->coil_mode ? plan->C : 1;
    if ((st = ensure_workspace(plan, B * C))) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // F S (c_i x_b) for every image and coil: B * C grids in [b][i] order, the
    // order of gy's [B][C][M] rows, which the kernel sums over
    if ((st = run_fs(plan, plan_fft(plan), static_cast<const float2 *>(x_dev), B, plan->grid, s))) return st;
    GradArgs a{};
    a.geo = plan->geom();
    a.om_sorted = plan->om_sorted;
    a.perm = plan->perm;
    a.M = plan->M;
    a.G = plan->grid;
    a.grid_elems = plan->grid_elems;
    a.grids = B * C;
    a.gy = static_cast<const float2 *>(gy_dev);
    a.gom = gom_dev;
    HIP_TRY(timed(plan, kGrad, s, [&] { return launch_grad(a, s); }), "trajectory gradient");
    return NUFFT_OK;
}

int nufft_grad_points(nufft_plan_t plan, const void *x_dev, const void *gy_dev, float *gom_dev, void *stream) {
    return nufft_grad_points_batched(plan, 1, x_dev, gy_dev, gom_dev, stream);
}

int nufft_stage_fs(nufft_plan_t plan, const void *x_dev, void *G_dev, void *stream) {
    int st = begin_call(plan, stream);
    if (st) return st;
    if (!x_dev || !G_dev) return fail(NUFFT_ERR_INVALID_ARG, "NULL data pointer");
    if (plan->coil_mode) return fail(NUFFT_ERR_UNSUPPORTED, "stage calls take no coils");
    return run_fs(plan, plan_fft(plan), static_cast<const float2 *>(x_dev), 1, static_cast<float2 *>(G_dev),
                  static_cast<hipStream_t>(stream));
}

int nufft_stage_v(nufft_plan_t plan, const void *G_dev, void *y_dev, void *stream) {
    int st = begin_call(plan, stream);
    if (st) return st;
    if (!G_dev || (!y_dev && plan->M > 0)) return fail(NUFFT_ERR_INVALID_ARG, "NULL data pointer");
    return run_v(plan, static_cast<const float2 *>(G_dev), 1, static_cast<float2 *>(y_dev),
                 static_cast<hipStream_t>(stream));
}

int nufft_stage_vh(nufft_plan_t plan, const void *y_dev, void *h_dev, void *stream) {
    int st = begin_call(plan, stream);
    if (st) return st;
    if (!h_dev || (!y_dev && plan->M > 0)) return fail(NUFFT_ERR_INVALID_ARG, "NULL data pointer");
    return run_vh(plan, static_cast<const float2 *>(y_dev), 1, static_cast<float2 *>(h_dev),
                  static_cast<hipStream_t>(stream));
}

int nufft_stage_shfh(nufft_plan_t plan, const void *h_dev, void *x_dev, void *stream) {
    int st = begin_call(plan, stream);
    if (st) return st;
    if (!h_dev || !x_dev) return fail(NUFFT_ERR_INVALID_ARG, "NULL data pointer");
    if (plan->coil_mode) return fail(NUFFT_ERR_UNSUPPORTED, "stage calls take no coils");
    return run_shfh(plan, plan_fft(plan), static_cast<const float2 *>(h_dev), 1, static_cast<float2 *>(x_dev),
                    static_cast<hipStream_t>(stream));
}

int nufft_plan_info(nufft_plan_t plan, double *beta3, int *poly_degree, int *tile3, int64_t *n_bins,
                    int64_t *n_items, int64_t *workspace_bytes) {
    int st = check_plan(plan);
    if (st) return st;
    for (int a = 0; a < 3; ++a) {
        if (beta3) beta3[a] = a < plan->d ? plan->ker[a].beta : 0.0;
        if (tile3) tile3[a] = a < plan->d ? plan->T[a] : 1;
    }
    if (poly_degree) *poly_degree = plan->ker[0].deg;
    if (n_bins) *n_bins = plan->nbins;
    if (n_items) *n_items = plan->n_items;
    if (workspace_bytes)
        *workspace_bytes = int64_t(plan->cap_grids) *
                               (plan->grid_elems + plan->tmp_elems +
                                std::max<int64_t>(plan->n_slots, 1) * plan->tile_cells) *
                               int64_t(sizeof(float2)) +
                           int64_t(plan->cap_wtab) * int64_t(sizeof(float));
    return NUFFT_OK;
}

int nufft_timing_enable(nufft_plan_t plan, int enable) {
    int st = check_plan(plan);
    if (st) return st;
    HIP_TRY(hipSetDevice(plan->device), "select device");
    if (!plan->timing_recs.empty()) HIP_TRY(hipEventSynchronize(plan->timing_recs.back().stop), "drain timing events");
    recycle_timing(plan);
    plan->timing = enable != 0;
    return NUFFT_OK;
}

int nufft_timing_kernels(void) { return kNumKernels; }

int nufft_timing_read(nufft_plan_t plan, int kernel, const char **name, int64_t *launches, double *total_ms) {
    int st = check_plan(plan);
    if (st) return st;
    if (kernel < 0 || kernel >= kNumKernels) return fail(NUFFT_ERR_INVALID_ARG, "kernel index %d out of range", kernel);
    if (name) *name = kKernelNames[kernel];
    HIP_TRY(hipSetDevice(plan->device), "select device");
    int64_t n = 0;
    double ms = 0.0;
    for (auto &r : plan->timing_recs) {
        if (r.kernel != kernel) continue;
        HIP_TRY(hipEventSynchronize(r.stop), "wait for timing event");
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, r.start, r.stop), "read timing event");
        ms += t;
        ++n;
    }
    if (launches) *launches = n;
    if (total_ms) *total_ms = ms;
    return NUFFT_OK;
}

int nufft_destroy(nufft_plan_t plan) {
    int st = check_plan(plan);
    if (st) return st;
    {
        std::lock_guard<std::mutex> lk(g_registry_mu);
        g_registry.erase(plan);
    }
    (void)hipSetDevice(plan->device);
    if (plan->last_stream) (void)hipStreamSynchronize(plan->last_stream);
    (void)hipDeviceSynchronize();
    free_plan(plan);
    plan->magic = 0;
    delete plan;
    return NUFFT_OK;
}


// ------------------------------------------------------------ Toeplitz normal operator
// A^H W A x = crop( F^-1( P * F( pad(x) ) ) ) on the 2N grid, P the FFT of the
// point-spread function p[Delta] = sum_m w_m e^{+i omega_m . Delta},
// Delta in [-N, N)^d, divided by prod(2N): no interpolation per application.
int nufft_toeplitz_plan(nufft_plan_t plan, const float *w_dev, void *stream, nufft_toeplitz_t *out) {
    if (!out) return fail(NUFFT_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int st = begin_call(plan, stream);
    if (st) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int d = plan->d;
    int64_t N2[kMaxDim] = {1, 1, 1}, K2[kMaxDim] = {1, 1, 1};
    for (int a = 0; a < d; ++a) {
        N2[a] = 2 * plan->N[a];
        K2[a] = 2 * plan->K[a];
        if (N2[a] > 4096 || !smooth235(N2[a]))
            return fail(NUFFT_ERR_UNSUPPORTED, "Toeplitz grid 2N[%d]=%lld must be 2-3-5 smooth and <= 4096", a,
                        (long long)N2[a]);
    }
    auto t = std::make_unique<nufft_toeplitz_s>();
    t->plan = plan;
    t->d = d;
    t->elems = 1;
    for (int a = 0; a < d; ++a) {
        t->N[a] = plan->N[a];
        t->P[a] = N2[a];
        t->elems *= N2[a];
        if (!radix_plan(int(N2[a]), &t->rp[a])) return fail(NUFFT_ERR_UNSUPPORTED, "no radix plan for 2N");
        std::vector<float> ones(size_t(plan->N[a]), 1.0f);
        std::vector<float> inv(size_t(N2[a]), float(1.0 / double(N2[a])));
        hipError_t e;
        if ((e = upload(&t->tw[a], twiddles(int(N2[a])))) != hipSuccess ||
            (e = upload(&t->ones[a], ones)) != hipSuccess || (e = upload(&t->inv[a], inv)) != hipSuccess) {
            destroy_toeplitz(t.get());
            return hip_fail(e, "upload Toeplitz constants");
        }
    }
    // sample weights as complex values (1 when w_dev is NULL)
    const int64_t M = plan->M;
    std::vector<float2> wc(size_t(std::max<int64_t>(M, 1)), make_float2(1.0f, 0.0f));
    if (w_dev && M > 0) {
        std::vector<float> wh(static_cast<size_t>(M));
        hipError_t e = hipMemcpyAsync(wh.data(), w_dev, size_t(M) * sizeof(float), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            destroy_toeplitz(t.get());
            return hip_fail(e, "read sample weights");
        }
        for (int64_t m = 0; m < M; ++m) {
            if (!std::isfinite(wh[size_t(m)])) {
                destroy_toeplitz(t.get());
                return fail(NUFFT_ERR_NONFINITE, "weight %lld is not finite", (long long)m);
            }
            wc[size_t(m)] = make_float2(wh[size_t(m)], 0.0f);
        }
    }
    float2 *wdev = nullptr, *psf = nullptr;
    nufft_plan_t pp = nullptr;
    hipError_t e;
    if ((e = upload(&wdev, wc)) != hipSuccess || (e = dmalloc(&psf, size_t(t->elems))) != hipSuccess ||
        (e = dmalloc(&t->phat, size_t(t->elems))) != hipSuccess) {
        dfree(wdev);
        dfree(psf);
        destroy_toeplitz(t.get());
        return hip_fail(e, "allocate Toeplitz buffers");
    }
    // p = adjoint NUFFT of the weights with image 2N on grid 2K (same J)
    st = nufft_plan_ex(d, N2, K2, plan->J, M, plan->om, nullptr, stream, &pp);
    if (!st) st = nufft_adjoint(pp, wdev, psf, stream);
    if (!st) st = ensure_toeplitz_workspace(t.get(), 1);
    if (!st) {
        // P = F(p placed at Delta mod 2N) / prod(2N): the forward passes with
        // image = grid = 2N place the centred p circularly; the scale tables
        // carry 1 / (2N_a)
        FftGeom f = toeplitz_fft(t.get(), true);
        f.coils = nullptr;
        f.C = 1;
        st = run_fs(plan, f, psf, 1, t->phat, s);
    }
    if (!st) {
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = hip_fail(e, "Toeplitz point-spread function");
    }
    if (pp) (void)nufft_destroy(pp);
    dfree(wdev);
    dfree(psf);
    if (st) {
        destroy_toeplitz(t.get());
        return st;
    }
    {
        std::lock_guard<std::mutex> lk(g_registry_mu);
        g_toeplitz_registry.insert(t.get());
    }
    *out = t.release();
    return NUFFT_OK;
}

int nufft_toeplitz_apply(nufft_toeplitz_t t, int B, const void *x_dev, void *out_dev, void *stream) {
    int st = check_toeplitz(t);
    if (st) return st;
    nufft_plan_t plan = t->plan;
    if ((st = begin_call(plan, stream))) return fail(NUFFT_ERR_BAD_PLAN, "the operator's plan is gone");
    if (B < 1) return fail(NUFFT_ERR_INVALID_ARG, "B must be >= 1");
    if (!x_dev || !out_dev) return fail(NUFFT_ERR_INVALID_ARG, "NULL data pointer");
    const int C = plan->coil_mode ? plan->C : 1;
    if ((st = ensure_toeplitz_workspace(t, B * C))) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    FftGeom f = toeplitz_fft(t, false);
    f.coils = plan->coil_mode ? plan->coils : nullptr;
    f.C = C;
    // forward passes into the grid buffer (the product for d = 1 happens
    // there), inverse passes with the product fused into the first
    float2 *G = t->grid2;
    if ((st = run_fs(plan, f, static_cast<const float2 *>(x_dev), B, G, s, t->phat))) return st;
    return run_shfh(plan, f, G, B, static_cast<float2 *>(out_dev), s, false, t->d >= 2 ? t->phat : nullptr);
}

int nufft_toeplitz_destroy(nufft_toeplitz_t t) {
    int st = check_toeplitz(t);
    if (st) return st;
    {
        std::lock_guard<std::mutex> lk(g_registry_mu);
        g_toeplitz_registry.erase(t);
    }
    (void)hipDeviceSynchronize();
    destroy_toeplitz(t);
    t->magic = 0;
    delete t;
    return NUFFT_OK;
}

// ------------------------------------------------------------ density compensation
}  // extern "C"

namespace {

// `iters` density-compensation steps with the caller's buffers wc and u
// (complex [M] each); asynchronous on s.
int dc_iterate(nufft_plan_s *plan, int iters, float *w_dev, float2 *wc, float2 *u, hipStream_t s) {
    // u = V V^H w with the kernel normalised to peak 1: gridding of w / c onto
    // the oversampled grid, interpolation, and a division by c again
    double c = 1.0;
    for (int a = 0; a < plan->d; ++a) c *= kb_i0(plan->ker[a].beta);
    const float inv_c = float(1.0 / c);
    hipError_t e;
    if ((e = launch_real_to_complex(w_dev, wc, plan->M, inv_c, s)) != hipSuccess)
        return hip_fail(e, "weights to samples");
    for (int it = 0; it < iters; ++it) {
        int st;
        if ((st = run_vh(plan, wc, 1, plan->grid, s, true))) return st;
        if ((st = run_v(plan, plan->grid, 1, u, s))) return st;
        if ((e = launch_dc_update(w_dev, u, wc, plan->M, inv_c, s)) != hipSuccess)
            return hip_fail(e, "density update");
    }
    return NUFFT_OK;
}

int dc_check(nufft_plan_t plan, int iters, float *w_dev, void *stream) {
    int st = begin_call(plan, stream);
    if (st) return st;
    if (plan->minmax) return fail(NUFFT_ERR_UNSUPPORTED, "density compensation needs the Kaiser-Bessel interpolator");
    if (iters < 0) return fail(NUFFT_ERR_INVALID_ARG, "iters must be >= 0");
    if (plan->M > 0 && !w_dev) return fail(NUFFT_ERR_INVALID_ARG, "w is NULL");
    return NUFFT_OK;
}

}  // namespace

extern "C" {

int nufft_density_compensation(nufft_plan_t plan, int iters, float *w_dev, void *stream) {
    int st = dc_check(plan, iters, w_dev, stream);
    if (st) return st;
    if (plan->M == 0 || iters == 0) return NUFFT_OK;
    if ((st = ensure_workspace(plan, 1))) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    float2 *wc = nullptr, *u = nullptr;
    hipError_t e;
    if ((e = dmalloc(&wc, size_t(plan->M))) != hipSuccess || (e = dmalloc(&u, size_t(plan->M))) != hipSuccess) {
        dfree(wc);
        dfree(u);
        return hip_fail(e, "allocate density-compensation buffers");
    }
    st = dc_iterate(plan, iters, w_dev, wc, u, s);
    if ((e = hipStreamSynchronize(s)) != hipSuccess && !st) st = hip_fail(e, "density compensation");
    dfree(wc);
    dfree(u);
    return st;
}

int nufft_density_compensation_noalloc(nufft_plan_t plan, int iters, float *w_dev, void *stream) {
    int st = dc_check(plan, iters, w_dev, stream);
    if (st) return st;
    if (plan->M > kDcScratchMaxM)
        return fail(NUFFT_ERR_INVALID_ARG,
                    "M = %lld exceeds the %lld samples of the allocation-free density compensation's scratch",
                    static_cast<long long>(plan->M), static_cast<long long>(kDcScratchMaxM));
    if (plan->M == 0 || iters == 0) return NUFFT_OK;
    // the plan's own workspace (one grid, the partial tiles of the current
    // binning) must already exist: this call never allocates it
    if (plan->cap_grids < 1 || plan->n_slots > plan->cap_slots)
        return fail(NUFFT_ERR_INVALID_ARG, "the plan's workspace is not allocated: call nufft_reserve(plan, 1) first");
    float2 *wc = nullptr, *u = nullptr;
    HIP_TRY(dc_scratch(&wc, &u), "look up the device scratch");
    return dc_iterate(plan, iters, w_dev, wc, u, static_cast<hipStream_t>(stream));
}


// ------------------------------------------------------------ TV split-Bregman pieces
namespace {
int check_image(int d, const int64_t *N) {
    if (d < 1 || d > 3) return fail(NUFFT_ERR_INVALID_ARG, "d must be 1, 2 or 3");
    if (!N) return fail(NUFFT_ERR_INVALID_ARG, "N is NULL");
    for (int a = 0; a < d; ++a)
        if (N[a] < 1) return fail(NUFFT_ERR_INVALID_ARG, "N[%d] must be >= 1", a);
    return NUFFT_OK;
}
}  // namespace

int nufft_tv_shrink(int d, const int64_t *N, const void *x_dev, void *d_dev, void *b_dev, float t, void *stream) {
    int st = check_image(d, N);
    if (st) return st;
    if (!x_dev || !d_dev || !b_dev) return fail(NUFFT_ERR_INVALID_ARG, "NULL data pointer");
    if (!(t >= 0.f) || !std::isfinite(t)) return fail(NUFFT_ERR_INVALID_ARG, "threshold must be finite and >= 0");
    HIP_TRY(launch_tv_shrink(d, N, static_cast<const float2 *>(x_dev), static_cast<float2 *>(d_dev),
                             static_cast<float2 *>(b_dev), t, static_cast<hipStream_t>(stream)),
            "TV shrink");
    return NUFFT_OK;
}

int nufft_tv_rhs(int d, const int64_t *N, float mu, const void *ahy_dev, const void *df_dev, const void *bf_dev,
                 float lam, const void *d_dev, const void *b_dev, void *rhs_dev, void *stream) {
    int st = check_image(d, N);
    if (st) return st;
    if (!ahy_dev || !d_dev || !b_dev || !rhs_dev) return fail(NUFFT_ERR_INVALID_ARG, "NULL data pointer");
    if ((df_dev == nullptr) != (bf_dev == nullptr))
        return fail(NUFFT_ERR_INVALID_ARG, "df and bf are given together or not at all");
    HIP_TRY(launch_tv_rhs(d, N, mu, static_cast<const float2 *>(ahy_dev), static_cast<const float2 *>(df_dev),
                          static_cast<const float2 *>(bf_dev), lam, static_cast<const float2 *>(d_dev),
                          static_cast<const float2 *>(b_dev), static_cast<float2 *>(rhs_dev),
                          static_cast<hipStream_t>(stream)),
            "TV right-hand side");
    return NUFFT_OK;
}

int nufft_tv_normal(int d, const int64_t *N, float mu, const void *ahax_dev, float lam, const void *x_dev,
                    void *out_dev, void *stream) {
    int st = check_image(d, N);
    if (st) return st;
    if (!ahax_dev || !x_dev || !out_dev) return fail(NUFFT_ERR_INVALID_ARG, "NULL data pointer");
    HIP_TRY(launch_tv_normal(d, N, mu, static_cast<const float2 *>(ahax_dev), lam, static_cast<const float2 *>(x_dev),
                             static_cast<float2 *>(out_dev), static_cast<hipStream_t>(stream)),
            "TV normal operator");
    return NUFFT_OK;
}

int nufft_bregman_shrink(int64_t n, const void *r_dev, void *d_dev, void *b_dev, float t, void *stream) {
    if (n < 0) return fail(NUFFT_ERR_INVALID_ARG, "n must be >= 0");
    if (n > 0 && (!r_dev || !d_dev || !b_dev)) return fail(NUFFT_ERR_INVALID_ARG, "NULL data pointer");
    if (!(t >= 0.f) || !std::isfinite(t)) return fail(NUFFT_ERR_INVALID_ARG, "threshold must be finite and >= 0");
    HIP_TRY(launch_bregman_shrink(n, static_cast<const float2 *>(r_dev), static_cast<float2 *>(d_dev),
                                  static_cast<float2 *>(b_dev), t, static_cast<hipStream_t>(stream)),
            "Bregman shrink");
    return NUFFT_OK;
}
}  // extern "C"
