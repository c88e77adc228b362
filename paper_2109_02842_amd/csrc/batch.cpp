// Batched hybrid reconstruction: several scans of different geometry, length
// and image grid in one call.  Per-scan steps (plan tables, scan FFT, range
// compression, k_z IFFT) are launched per scan; the dominant back-projection
// of every scan that takes the pixel-per-lane kernel runs in ONE persistent
// launch per LDS row length over (scan, k_z block, tile) work items,
// heaviest scans first, in eight cost-balanced per-XCD queues with stealing.
// Everything runs in order on the caller's stream (each launch fills the
// GPU; overlapping different scans' steps on other streams was slower).  The
// call allocates nothing and does no host synchronisation, so a caller may
// capture it in a graph.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

#include "internal.hpp"

struct pl_hybrid_batch {
    // One persistent launch: the queued scans of one LDS row length.
    struct Queue {
        int kb = 0, rsc = 0, n_items = 0, grid = 0;
        size_t smem = 0, items_off = 0, bounds_off = 0;  // byte offsets in d_items
    };
    int device = -1;
    std::vector<const pl_geometry*> geoms;
    std::vector<pl::HybridPlan> plans;
    std::vector<size_t> ws_off;         // byte offset of each scan's workspace
    size_t counter_off = 0, total = 0;  // work-queue counters, workspace bytes
    std::vector<char> in_queue;         // scan takes part in a persistent launch
    std::vector<Queue> queues;
    void* d_desc = nullptr;             // device: per-scan descriptors
    void* d_items = nullptr;            // device: per queue, int4 work items then 9 bounds
    ~pl_hybrid_batch() {
        if (d_desc) (void)hipFree(d_desc);
        if (d_items) (void)hipFree(d_items);
    }
};

namespace {

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

}  // namespace

extern "C" {

int make_hybrid_batch(int32_t n, const pl_geometry* const* geoms, const pl_image_grid* grids,
                      const pl_hybrid_opts* opts, pl_hybrid_batch** out) {
    using namespace pl;
    clear_error();
    if (!out) return fail(PL_EINVAL, "make_hybrid_batch: null output");
    *out = nullptr;
    if (n < 1 || n > 4096) return fail(PL_EINVAL, "make_hybrid_batch: %d scans (1 .. 4096)", n);
    if (!geoms || !grids) return fail(PL_EINVAL, "make_hybrid_batch: null geometry or grid array");
    auto b = new pl_hybrid_batch();
    auto bail = [&](int rc) {
        delete b;
        return rc;
    };
    if (hipGetDevice(&b->device) != hipSuccess) return bail(fail(PL_EDEVICE, "make_hybrid_batch: no device"));
    b->geoms.assign(geoms, geoms + n);
    b->plans.resize(n);
    b->ws_off.resize(n);
    b->in_queue.assign(n, 0);
    size_t off = 0;
    for (int s = 0; s < n; ++s) {
        if (!geoms[s]) return bail(fail(PL_EINVAL, "make_hybrid_batch: scan %d has no geometry", s));
        int rc = make_plan(geoms[s], &grids[s], opts ? &opts[s] : nullptr, &b->plans[s]);
        if (rc) return bail(rc);
        b->ws_off[s] = off;
        off = align256(off + b->plans[s].total);
    }
    b->counter_off = off;  // eight counters per persistent launch (at most 8 launches)
    b->total = off + 256;

    // Scans in the persistent launches: pixel-per-lane plans sharing the k_z
    // block size of the first such scan, one launch per LDS row length (a
    // longer row would lower every workgroup's occupancy).
    int kb = 0;
    std::vector<int> rscs;
    for (int s = 0; s < n; ++s) {
        const HybridPlan& p = b->plans[s];
        if (!p.bp_gather) continue;
        if (!kb) kb = p.block;
        if (p.block != kb) continue;
        b->in_queue[s] = 1;
        if (std::find(rscs.begin(), rscs.end(), p.window_pad) == rscs.end()) rscs.push_back(p.window_pad);
    }
    if (rscs.size() > 8) return bail(fail(PL_EUNSUPPORTED, "make_hybrid_batch: more than 8 row lengths"));
    std::sort(rscs.begin(), rscs.end());
    std::vector<char> desc(gather_batch_desc_bytes() * n, 0);
    std::vector<int> all;  // every queue's items and bounds, back to back
    for (int rsc : rscs) {
        pl_hybrid_batch::Queue q;
        q.kb = kb;
        q.rsc = rsc;
        std::vector<int> order;
        for (int s = 0; s < n; ++s)
            if (b->in_queue[s] && b->plans[s].window_pad == rsc) order.push_back(s);
        // heaviest scans first (work per item ~ channels), scan order kept among equals
        std::stable_sort(order.begin(), order.end(),
                         [&](int i, int j) { return b->plans[i].n_ch > b->plans[j].n_ch; });
        // Eight per-XCD queues: every scan's (k_z block, tile) items, in
        // order, split into eight contiguous shares (all items of a scan
        // cost the same), and queue x holds share x of each scan in turn.
        // The XCDs then work through the scans together, each on a compact
        // range of one scan's range profiles, as separate launches would;
        // a queue spanning whole scans instead keeps up to eight scans'
        // profiles live at once (measured 10 % slower at C5).
        std::vector<std::vector<int>> per_xcd(8);
        for (int s : order) {
            const HybridPlan& p = b->plans[s];
            DeviceTables dt;
            int rc = geoms[s]->device_tables(&dt);
            if (rc) return bail(rc);
            rc = build_gather_batch_desc(p, b->ws_off[s], rsc, desc.data() + gather_batch_desc_bytes() * s);
            if (rc) return bail(rc);
            q.smem = std::max(q.smem, backproject_gather_lds_bytes(kb, rsc));
            const int n_tiles = p.tiles_x * p.tiles_y;
            const int n_scan_items = p.n_blocks * n_tiles;
            for (int i = 0; i < n_scan_items; ++i) {
                const int x = static_cast<int>((static_cast<long long>(i) * 8) / n_scan_items);
                const int blk = i / n_tiles;
                per_xcd[x].push_back(s);
                per_xcd[x].push_back(blk);
                per_xcd[x].push_back(i - blk * n_tiles);
                per_xcd[x].push_back(0);
            }
        }
        std::vector<int> items;
        std::vector<int> bounds(9, 0);
        for (int x = 0; x < 8; ++x) {
            items.insert(items.end(), per_xcd[x].begin(), per_xcd[x].end());
            bounds[x + 1] = static_cast<int>(items.size() / 4);
        }
        q.n_items = static_cast<int>(items.size() / 4);
        q.items_off = all.size() * sizeof(int);
        all.insert(all.end(), items.begin(), items.end());
        q.bounds_off = all.size() * sizeof(int);
        all.insert(all.end(), bounds.begin(), bounds.end());
        while (all.size() % 4) all.push_back(0);  // keep the next queue's items 16-byte aligned
        int rc = gather_batch_grid(kb, rsc, q.smem, &q.grid);
        if (rc) return bail(rc);
        b->queues.push_back(q);
    }
    if (!b->queues.empty() &&
        (hipMalloc(&b->d_desc, desc.size()) != hipSuccess || hipMalloc(&b->d_items, all.size() * sizeof(int)) != hipSuccess ||
         hipMemcpy(b->d_desc, desc.data(), desc.size(), hipMemcpyHostToDevice) != hipSuccess ||
         hipMemcpy(b->d_items, all.data(), all.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess))
        return bail(fail(PL_EDEVICE, "make_hybrid_batch: uploading the work queues failed"));
    *out = b;
    return PL_OK;
}

int destroy_hybrid_batch(pl_hybrid_batch* b) {
    pl::clear_error();
    delete b;
    return PL_OK;
}

int hybrid_batch_info(const pl_hybrid_batch* b, size_t* workspace_bytes, int32_t* queued_scans,
                      int32_t* work_items, int32_t* workgroups) {
    using namespace pl;
    clear_error();
    if (!b) return fail(PL_EINVAL, "hybrid_batch_info: null batch");
    if (workspace_bytes) *workspace_bytes = b->total;
    if (queued_scans) *queued_scans = static_cast<int32_t>(std::count(b->in_queue.begin(), b->in_queue.end(), 1));
    int items = 0, groups = 0;
    for (const auto& q : b->queues) {
        items += q.n_items;
        groups += q.grid;
    }
    if (work_items) *work_items = items;
    if (workgroups) *workgroups = groups;
    return PL_OK;
}

}  // extern "C"

namespace {

// Checks shared by the batch calls: the workspace and the device.
int check_batch_ws(const pl_hybrid_batch* b, void* ws, size_t ws_bytes, const char* what) {
    using namespace pl;
    if (!ws) return fail(PL_EWORKSPACE, "%s: null workspace", what);
    if ((reinterpret_cast<uintptr_t>(ws) & 255u) != 0) return fail(PL_EWORKSPACE, "%s: workspace must be 256-byte aligned", what);
    if (ws_bytes < b->total) return fail(PL_EWORKSPACE, "%s: workspace of %zu bytes, %zu needed", what, ws_bytes, b->total);
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != b->device)
        return fail(PL_EDEVICE, "%s: the batch was made on device %d", what, b->device);
    return PL_OK;
}

// The batch call; with `tables` false the workspace already holds every
// scan's plan tables (hybrid_batch_prepare).
int batch_impl(const pl_hybrid_batch* b, const float* const* echoes, float* const* images, void* ws, size_t ws_bytes,
               hipStream_t stream, bool tables, const char* what) {
    using namespace pl;
    clear_error();
    if (!b || !echoes || !images) return fail(PL_EINVAL, "%s: null argument", what);
    const int n = static_cast<int>(b->plans.size());
    for (int s = 0; s < n; ++s)
        if (!echoes[s] || !images[s]) return fail(PL_EINVAL, "%s: scan %d has a null buffer", what, s);
    int rc0 = check_batch_ws(b, ws, ws_bytes, what);
    if (rc0) return rc0;
    char* w = static_cast<char*>(ws);
    std::vector<DeviceTables> dts(n);
    int rc = PL_OK;
    for (int s = 0; s < n; ++s)
        if ((rc = b->geoms[s]->device_tables(&dts[s], stream))) return rc;

    // plan tables, scan FFT, range compression per scan, in order on the
    // caller's stream: each of these launches fills the GPU by itself, and
    // running several scans' steps at once on other streams made every
    // kernel slower and the whole front end longer than the same steps in
    // sequence (they contend for the CUs and evict each other's data)
    for (int s = 0; s < n; ++s) {
        const HybridPlan& p = b->plans[s];
        char* ws_s = w + b->ws_off[s];
        float2* spec = reinterpret_cast<float2*>(ws_s + p.off_spec);
        if (tables && (rc = launch_plan_tables(p, dts[s], ws_s, stream))) return rc;
        if ((rc = launch_scan_fft(b->geoms[s], reinterpret_cast<const float2*>(echoes[s]), spec, p.zfft,
                                  ws_s + p.off_zfft, stream)))
            return rc;
        if (p.bp_mfma)
            rc = launch_range_compress_mfma_split(p, spec, ws_s, reinterpret_cast<unsigned short*>(ws_s + p.off_q), stream);
        else if (p.precision == PL_PREC_FP32)
            rc = launch_range_compress_fp32(p, spec, ws_s, reinterpret_cast<float2*>(ws_s + p.off_q), stream);
        else
            rc = launch_range_compress_mfma(p, spec, ws_s, reinterpret_cast<float2*>(ws_s + p.off_q), stream);
        if (rc) return rc;
    }
    // back-projection: the persistent launch, then any scan outside it
    for (size_t k = 0; k < b->queues.size(); ++k) {
        const auto& q = b->queues[k];
        const char* base = static_cast<const char*>(b->d_items);
        if ((rc = launch_gather_batch(b->d_desc, base + q.items_off, reinterpret_cast<const int*>(base + q.bounds_off),
                                      reinterpret_cast<unsigned*>(w + b->counter_off) + 8 * k, w, q.kb, q.rsc, q.smem,
                                      q.grid, stream)))
            return rc;
    }
    for (int s = 0; s < n; ++s) {
        if (b->in_queue[s]) continue;
        const HybridPlan& p = b->plans[s];
        char* ws_s = w + b->ws_off[s];
        float2* G = reinterpret_cast<float2*>(ws_s + p.off_G);
        rc = p.bp_mfma ? launch_backproject_mfma(p, dts[s], reinterpret_cast<const unsigned short*>(ws_s + p.off_q),
                                                 ws_s, G, stream)
                       : launch_backproject(p, dts[s], reinterpret_cast<const float2*>(ws_s + p.off_q), ws_s, G, stream);
        if (rc) return rc;
    }
    // k_z inverse FFT per scan
    for (int s = 0; s < n; ++s) {
        const HybridPlan& p = b->plans[s];
        char* ws_s = w + b->ws_off[s];
        if ((rc = launch_kz_ifft(p, reinterpret_cast<const float2*>(ws_s + p.off_G), reinterpret_cast<float2*>(images[s]),
                                 ws_s + p.off_zfft, stream)))
            return rc;
    }
    return PL_OK;
}

}  // namespace

extern "C" {

int reconstruct_hybrid_batch(const pl_hybrid_batch* b, const float* const* echoes, float* const* images, void* ws,
                             size_t ws_bytes, hipStream_t stream) {
    return batch_impl(b, echoes, images, ws, ws_bytes, stream, true, "reconstruct_hybrid_batch");
}

int reconstruct_hybrid_batch_prepared(const pl_hybrid_batch* b, const float* const* echoes, float* const* images,
                                      void* ws, size_t ws_bytes, hipStream_t stream) {
    return batch_impl(b, echoes, images, ws, ws_bytes, stream, false, "reconstruct_hybrid_batch_prepared");
}

int hybrid_batch_prepare(const pl_hybrid_batch* b, void* ws, size_t ws_bytes, hipStream_t stream) {
    using namespace pl;
    clear_error();
    if (!b) return fail(PL_EINVAL, "hybrid_batch_prepare: null batch");
    int rc = check_batch_ws(b, ws, ws_bytes, "hybrid_batch_prepare");
    if (rc) return rc;
    char* w = static_cast<char*>(ws);
    for (size_t s = 0; s < b->plans.size(); ++s) {
        DeviceTables dt;
        if ((rc = b->geoms[s]->device_tables(&dt, stream))) return rc;
        if ((rc = launch_plan_tables(b->plans[s], dt, w + b->ws_off[s], stream))) return rc;
    }
    return PL_OK;
}

}  // extern "C"
