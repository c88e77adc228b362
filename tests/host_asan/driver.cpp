// Host-path exercise of the polyrecon C ABI for an AddressSanitizer build
// (host code instrumented, device code untouched).  Runs without a GPU:
// geometry construction and queries, hybrid plans over many option sets and
// workloads, workspace queries, argument and device errors, batch setup, and
// every destroy call; exits non-zero on an unexpected return code.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../include/polyrecon.h"

static int failures = 0;
#define EXPECT(cond)                                                                   \
    do {                                                                               \
        if (!(cond)) {                                                                 \
            std::fprintf(stderr, "%s:%d: expectation failed: %s (%s)\n", __FILE__, __LINE__, #cond, last_error()); \
            ++failures;                                                                \
        }                                                                              \
    } while (0)

static pl_geometry_desc mono(int chords, int elems, double R, int n_scan, int n_freq, double step) {
    pl_geometry_desc d{};
    d.mode = PL_MONO;
    d.n_chords = chords;
    d.radius_m = R;
    d.arc_center_rad = -M_PI / 2;
    d.n_elem = elems;
    d.spacing_m = 299792458.0 / (2 * 34e9);
    d.n_scan = n_scan;
    d.n_freq = n_freq;
    d.scan_step_m = step;
    d.scan_z0_m = -(n_scan - 1) * step / 2;
    d.f_start_hz = 26e9;
    d.f_stop_hz = 34e9;
    return d;
}

static pl_image_grid centred(int n, double extent) {
    const double dd = extent / n;
    return pl_image_grid{n, n, -extent / 2 + dd / 2, -extent / 2 + dd / 2, dd, dd};
}

int main() {
    std::vector<pl_geometry*> geoms;
    std::vector<pl_image_grid> grids;
    // C1, C2, C3-like, scans of every length class, and tiny ones
    pl_geometry_desc descs[8] = {mono(3, 16, 0.5, 24, 16, 0.005),  mono(5, 64, 0.6, 256, 64, 0.004),
                                 mono(4, 40, 0.6, 131, 48, 0.004), mono(3, 33, 0.6, 509, 77, 0.004),
                                 mono(2, 6, 0.4, 1, 8, 0.006),     mono(2, 6, 0.4, 4093, 8, 0.006),
                                 mono(2, 6, 0.4, 2304, 9, 0.006),  mono(6, 57, 0.6, 403, 112, 0.004)};
    pl_geometry_desc multi = mono(7, 32, 0.8, 512, 128, 0.003);
    multi.mode = PL_MULTI;
    multi.n_tx = 4;
    multi.spacing_m = 299792458.0 / 34e9;
    const double offs[3] = {-0.1, 0.0, 0.1};
    pl_geometry_desc multi3 = mono(3, 10, 0.5, 30, 12, 0.002);
    multi3.mode = PL_MULTI;
    multi3.n_tx = 3;
    multi3.spacing_m = 0.0088;
    multi3.tx_offsets_m = offs;
    std::vector<pl_geometry_desc> all(descs, descs + 8);
    all.push_back(multi);
    all.push_back(multi3);
    for (const auto& d : all) {
        pl_geometry* g = nullptr;
        EXPECT(make_geometry(&d, &g) == PL_OK && g);
        if (!g) continue;
        geoms.push_back(g);
        pl_geometry_info info{};
        EXPECT(geometry_info(g, &info, nullptr, nullptr, nullptr, nullptr, nullptr) == PL_OK);
        std::vector<double> tx(2 * info.n_channels), rx(2 * info.n_channels), z(info.n_scan), f(info.n_freq),
            ends(4 * info.n_chords);
        EXPECT(geometry_info(g, &info, tx.data(), rx.data(), z.data(), f.data(), ends.data()) == PL_OK);
        size_t fb = 0;
        EXPECT(fft_workspace_bytes(g, &fb) == PL_OK && fb > 0);
    }
    grids.push_back(centred(32, 0.30));
    grids.push_back(centred(200, 0.60));
    grids.push_back(centred(128, 0.60));
    grids.push_back(pl_image_grid{45, 37, -0.03, -0.02, 0.0015, 0.0015});
    grids.push_back(pl_image_grid{1, 1, 0.0, 0.0, 0.01, 0.01});
    grids.push_back(pl_image_grid{17, 5, -0.07, -0.05, 0.009, 0.022});

    // plans over option sets: every return code must be one the header names
    const int precisions[3] = {PL_PREC_FP32, PL_PREC_BF16, PL_PREC_FP16};
    const int mfma[4] = {-1, 0, 1, 2};
    const int tiles[3][2] = {{0, 0}, {16, 8}, {8, 8}};
    const int blocks[3] = {0, 64, 128};
    int planned = 0;
    for (pl_geometry* g : geoms)
        for (const auto& grid : grids)
            for (int p : precisions)
                for (int mb : mfma)
                    for (const auto& t : tiles)
                        for (int kb : blocks)
                            for (int ref = 0; ref < 2; ++ref)
                                for (int rm = 0; rm < 2; ++rm) {
                                    pl_hybrid_opts o{};
                                    o.precision = p;
                                    o.mfma_backprojection = mb;
                                    o.tile = t[0];
                                    o.tile_y = t[1];
                                    o.kz_block = kb;
                                    o.ref_mode = ref;
                                    o.range_method = rm;
                                    pl_hybrid_plan_info info{};
                                    std::vector<double> kref(4096 / 32);
                                    const int rc = hybrid_plan_info(g, &grid, &o, &info, kref.data());
                                    EXPECT(rc == PL_OK || rc == PL_EINVAL || rc == PL_EUNSUPPORTED);
                                    if (rc == PL_OK) {
                                        ++planned;
                                        EXPECT(info.n_blocks >= 1 && info.n_blocks <= 4096 / 32);
                                        EXPECT(info.scan_fft_len >= info.n_kz);
                                        size_t b = 0;
                                        EXPECT(hybrid_workspace_bytes(g, &grid, &o, &b) == PL_OK &&
                                               b == info.workspace_bytes);
                                    }
                                }
    EXPECT(planned > 1000);

    // argument errors before any device use
    float* fake = reinterpret_cast<float*>(static_cast<uintptr_t>(1) << 20);
    pl_hybrid_opts o{};
    size_t need = 0;
    EXPECT(hybrid_workspace_bytes(geoms[0], &grids[0], &o, &need) == PL_OK);
    EXPECT(reconstruct_hybrid(geoms[0], &grids[0], &o, nullptr, fake, fake, need, nullptr) == PL_EINVAL);
    EXPECT(reconstruct_hybrid(geoms[0], &grids[0], &o, fake, fake, nullptr, need, nullptr) == PL_EWORKSPACE);
    EXPECT(reconstruct_hybrid(geoms[0], &grids[0], &o, fake, fake, fake, need - 1, nullptr) == PL_EWORKSPACE);
    EXPECT(scan_fft(nullptr, fake, fake, fake, 1 << 20, nullptr) == PL_EINVAL);
    EXPECT(reconstruct_bp(geoms[0], &grids[0], 20, 10, fake, fake, fake, 1 << 30, nullptr) == PL_EINVAL);
    size_t bb = 0;
    EXPECT(bp_workspace_bytes(geoms[1], &grids[1], 4, &bb) == PL_OK && bb > 0);
    EXPECT(bp_workspace_bytes(geoms[1], &grids[1], 0, &bb) == PL_EINVAL);
    pl_geometry_desc bad = descs[0];
    bad.n_elem = 400;  // chord longer than the diameter
    pl_geometry* gbad = nullptr;
    EXPECT(make_geometry(&bad, &gbad) == PL_EGEOM && gbad == nullptr);
    bad = descs[0];
    bad.n_scan = 5000;
    EXPECT(make_geometry(&bad, &gbad) == PL_EINVAL);
    uint32_t warn = 0;
    EXPECT(check_sampling(geoms[0], &grids[0], &warn) == PL_OK);

    // batch setup: plans every scan; without a device the upload fails cleanly
    pl_hybrid_batch* batch = nullptr;
    std::vector<pl_image_grid> bgrids(geoms.size(), grids[2]);
    const int brc = make_hybrid_batch(static_cast<int32_t>(geoms.size()), geoms.data(), bgrids.data(), nullptr, &batch);
    EXPECT(brc == PL_OK || brc == PL_EDEVICE || brc == PL_EUNSUPPORTED);
    if (batch) {
        size_t wb = 0;
        int32_t q = 0, items = 0, wg = 0;
        EXPECT(hybrid_batch_info(batch, &wb, &q, &items, &wg) == PL_OK);
        EXPECT(destroy_hybrid_batch(batch) == PL_OK);
    }
    EXPECT(destroy_hybrid_batch(nullptr) == PL_OK);

    for (pl_geometry* g : geoms) EXPECT(destroy_geometry(g) == PL_OK);
    EXPECT(destroy_geometry(nullptr) == PL_OK);
    std::printf("host paths: %d plans, %d failures\n", planned, failures);
    return failures ? 1 : 0;
}
