// C-ABI entry points of the polyrecon library: argument checks, planning,
// and the launch sequence of each call.
#include <cmath>
#include <cstring>

#include "internal.hpp"

namespace pl {
namespace {

bool aligned256(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 255u) == 0; }

// stage: the single-stage entry points exchange complex64 range profiles,
// which only the VALU back-projection reads; they plan without the
// matrix-core back-projection.
int prepare(const pl_geometry* g, const pl_image_grid* grid, const pl_hybrid_opts* opts, void* ws, size_t ws_bytes,
            HybridPlan* p, DeviceTables* dt, const char* what, hipStream_t stream, bool stage = false,
            bool upload = true) {
    pl_hybrid_opts o{};
    if (opts) o = *opts;
    if (stage) {
        if (o.mfma_backprojection > 0)
            return fail(PL_EUNSUPPORTED, "%s: the MFMA back-projection runs only inside reconstruct_hybrid", what);
        o.mfma_backprojection = -1;
    }
    int rc = make_plan(g, grid, (opts || stage) ? &o : nullptr, p);
    if (rc) return rc;
    if (!ws) return fail(PL_EWORKSPACE, "%s: null workspace", what);
    if (!aligned256(ws)) return fail(PL_EWORKSPACE, "%s: workspace must be 256-byte aligned", what);
    if (ws_bytes < p->total)
        return fail(PL_EWORKSPACE, "%s: workspace of %zu bytes, %zu needed", what, ws_bytes, p->total);
    return g->device_tables(dt, stream, upload);
}

// The standalone transform calls: the tables of the length-n_scan transform
// written into the caller's workspace, checked for size and alignment.
int axis_tables(const pl_geometry* g, void* ws, size_t ws_bytes, hipStream_t stream, AxisFft* f, const char* what) {
    int rc = plan_axis_fft(g->n_scan, f);
    if (rc) return rc;
    if (!ws) return fail(PL_EWORKSPACE, "%s: null workspace", what);
    if (!aligned256(ws)) return fail(PL_EWORKSPACE, "%s: workspace must be 256-byte aligned", what);
    if (ws_bytes < f->bytes) return fail(PL_EWORKSPACE, "%s: workspace of %zu bytes, %zu needed", what, ws_bytes, f->bytes);
    return launch_axis_fft_tables(*f, static_cast<char*>(ws), stream);
}

}  // namespace
}  // namespace pl

extern "C" {

int hybrid_plan_info(const pl_geometry* g, const pl_image_grid* grid, const pl_hybrid_opts* opts,
                     pl_hybrid_plan_info* info, double* k_ref_host) {
    using namespace pl;
    clear_error();
    if (!info) return fail(PL_EINVAL, "hybrid_plan_info: null info");
    HybridPlan p;
    const int rc = make_plan(g, grid, opts, &p);
    if (rc) return rc;
    info->n_kz = p.n_z;
    info->n_l = p.n_l;
    info->n_fine = p.n_fine;
    info->kernel_width = p.W;
    info->n_blocks = p.n_blocks;
    info->block = p.block;
    info->window = p.window;
    info->tile_x = p.tile_x;
    info->tile_y = p.tile_y;
    info->bp_kernel = p.bp_mfma ? (p.bp_mfma_sp ? PL_BP_MFMA_SP : PL_BP_MFMA)
                                : (p.bp_gather ? PL_BP_PIXEL_LANES : PL_BP_KZ_LANES);
    info->waves = p.waves;
    info->du = p.du;
    info->beta = p.beta;
    info->workspace_bytes = p.total;
    info->range_method = p.range_method;
    info->dk_uniform = p.range_method == PL_RANGE_RESAMPLE ? p.dkl : 0.0;
    info->scan_fft_len = p.zfft.m;
    info->reserved_ = 0;
    if (k_ref_host) std::memcpy(k_ref_host, p.kref, sizeof(double) * p.n_blocks);  // n_blocks <= kMaxBlocks
    return PL_OK;
}

int hybrid_workspace_bytes(const pl_geometry* g, const pl_image_grid* grid, const pl_hybrid_opts* opts,
                           size_t* bytes) {
    using namespace pl;
    clear_error();
    if (!bytes) return fail(PL_EINVAL, "hybrid_workspace_bytes: null output");
    HybridPlan p;
    const int rc = make_plan(g, grid, opts, &p);
    if (rc) return rc;
    *bytes = p.total;
    return PL_OK;
}

int simulate_echo(const pl_geometry* g, int32_t n_scat, const double* xyz, const double* refl, float* echo,
                  hipStream_t stream) {
    using namespace pl;
    clear_error();
    if (!g || !echo) return fail(PL_EINVAL, "simulate_echo: null geometry or echo");
    if (n_scat < 0) return fail(PL_EINVAL, "simulate_echo: n_scat < 0");
    if (n_scat > 0 && (!xyz || !refl)) return fail(PL_EINVAL, "simulate_echo: null scatterer arrays");
    DeviceTables dt;
    int rc = g->device_tables(&dt, stream);
    if (rc) return rc;
    return launch_simulate(g, dt, n_scat, xyz, refl, reinterpret_cast<float2*>(echo), stream);
}

int fft_workspace_bytes(const pl_geometry* g, size_t* bytes) {
    using namespace pl;
    clear_error();
    if (!g || !bytes) return fail(PL_EINVAL, "fft_workspace_bytes: null pointer");
    AxisFft f;
    const int rc = plan_axis_fft(g->n_scan, &f);
    if (rc) return rc;
    *bytes = f.bytes;
    return PL_OK;
}

int scan_fft(const pl_geometry* g, const float* echo, float* spec, void* ws, size_t ws_bytes, hipStream_t stream) {
    using namespace pl;
    clear_error();
    if (!g || !echo || !spec) return fail(PL_EINVAL, "scan_fft: null pointer");
    AxisFft f;
    const int rc = axis_tables(g, ws, ws_bytes, stream, &f, "scan_fft");
    if (rc) return rc;
    return launch_scan_fft(g, reinterpret_cast<const float2*>(echo), reinterpret_cast<float2*>(spec), f,
                           static_cast<const char*>(ws), stream);
}

int range_compress(const pl_geometry* g, const pl_image_grid* grid, const pl_hybrid_opts* opts, const float* spec,
                   float* q, double* range_lo_host, void* ws, size_t ws_bytes, hipStream_t stream) {
    using namespace pl;
    clear_error();
    if (!spec || !q) return fail(PL_EINVAL, "range_compress: null pointer");
    HybridPlan p;
    DeviceTables dt;
    int rc = prepare(g, grid, opts, ws, ws_bytes, &p, &dt, "range_compress", stream, true);
    if (rc) return rc;
    char* w = static_cast<char*>(ws);
    if ((rc = launch_plan_tables(p, dt, w, stream))) return rc;
    rc = p.precision == PL_PREC_FP32
             ? launch_range_compress_fp32(p, reinterpret_cast<const float2*>(spec), w, reinterpret_cast<float2*>(q), stream)
             : launch_range_compress_mfma(p, reinterpret_cast<const float2*>(spec), w, reinterpret_cast<float2*>(q), stream);
    if (rc) return rc;
    if (range_lo_host) {
        if (hipMemcpyAsync(range_lo_host, w + p.off_llo, sizeof(double) * p.n_ch, hipMemcpyDeviceToHost, stream) !=
                hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess)
            return fail(PL_EDEVICE, "range_compress: copying range origins failed");
    }
    return PL_OK;
}

int backproject(const pl_geometry* g, const pl_image_grid* grid, const pl_hybrid_opts* opts, const float* q,
                float* spectrum, void* ws, size_t ws_bytes, hipStream_t stream) {
    using namespace pl;
    clear_error();
    if (!q || !spectrum) return fail(PL_EINVAL, "backproject: null pointer");
    HybridPlan p;
    DeviceTables dt;
    int rc = prepare(g, grid, opts, ws, ws_bytes, &p, &dt, "backproject", stream, true);
    if (rc) return rc;
    char* w = static_cast<char*>(ws);
    if ((rc = launch_plan_tables(p, dt, w, stream))) return rc;
    return launch_backproject(p, dt, reinterpret_cast<const float2*>(q), w, reinterpret_cast<float2*>(spectrum), stream);
}

int kz_ifft(const pl_geometry* g, const pl_image_grid* grid, const float* spectrum, float* image, void* ws,
            size_t ws_bytes, hipStream_t stream) {
    using namespace pl;
    clear_error();
    if (!g || !grid || !spectrum || !image) return fail(PL_EINVAL, "kz_ifft: null pointer");
    if (grid->nx < 1 || grid->ny < 1) return fail(PL_EINVAL, "kz_ifft: bad grid");
    HybridPlan p;
    p.n_z = g->n_scan;
    p.nx = grid->nx;
    p.ny = grid->ny;
    const int rc = axis_tables(g, ws, ws_bytes, stream, &p.zfft, "kz_ifft");
    if (rc) return rc;
    return launch_kz_ifft(p, reinterpret_cast<const float2*>(spectrum), reinterpret_cast<float2*>(image),
                          static_cast<const char*>(ws), stream);
}

}  // extern "C"

namespace pl {

// The hybrid reconstruction; tables = false skips the plan-table step (the
// caller prepared the workspace with hybrid_prepare for the same arguments).
int reconstruct_impl(const pl_geometry* g, const pl_image_grid* grid, const pl_hybrid_opts* opts, const float* echo,
                     float* image, void* ws, size_t ws_bytes, hipEvent_t* ev, hipStream_t stream, bool tables,
                     bool upload, const char* what) {
    clear_error();
    if (!echo || !image) return fail(PL_EINVAL, "%s: null echo or image", what);
    HybridPlan p;
    DeviceTables dt;
    int rc = prepare(g, grid, opts, ws, ws_bytes, &p, &dt, what, stream, false, upload);
    if (rc) return rc;
    auto mark = [&](int i) -> int {
        if (ev && ev[i] && hipEventRecord(ev[i], stream) != hipSuccess)
            return fail(PL_EDEVICE, "%s: hipEventRecord failed", what);
        return PL_OK;
    };
    char* w = static_cast<char*>(ws);
    float2* spec = reinterpret_cast<float2*>(w + p.off_spec);
    float2* q = reinterpret_cast<float2*>(w + p.off_q);
    float2* G = reinterpret_cast<float2*>(w + p.off_G);
    const char* ztab = w + p.off_zfft;
    if ((rc = mark(0)) || (tables && (rc = launch_plan_tables(p, dt, w, stream)))) return rc;
    if ((rc = mark(1)) || (rc = launch_scan_fft(g, reinterpret_cast<const float2*>(echo), spec, p.zfft, ztab, stream)))
        return rc;
    if ((rc = mark(2))) return rc;
    if (p.bp_mfma) {
        // split BF16 profiles in the same bytes as the complex64 ones
        unsigned short* qs = reinterpret_cast<unsigned short*>(w + p.off_q);
        if ((rc = launch_range_compress_mfma_split(p, spec, w, qs, stream))) return rc;
        if ((rc = mark(3)) || (rc = launch_backproject_mfma(p, dt, qs, w, G, stream))) return rc;
    } else {
        rc = p.precision == PL_PREC_FP32 ? launch_range_compress_fp32(p, spec, w, q, stream)
                                         : launch_range_compress_mfma(p, spec, w, q, stream);
        if (rc) return rc;
        if ((rc = mark(3)) || (rc = launch_backproject(p, dt, q, w, G, stream))) return rc;
    }
    if ((rc = mark(4)) || (rc = launch_kz_ifft(p, G, reinterpret_cast<float2*>(image), ztab, stream))) return rc;
    return mark(5);
}

}  // namespace pl

extern "C" {

int reconstruct_hybrid_events(const pl_geometry* g, const pl_image_grid* grid, const pl_hybrid_opts* opts,
                              const float* echo, float* image, void* ws, size_t ws_bytes, hipEvent_t* ev,
                              hipStream_t stream) {
    return pl::reconstruct_impl(g, grid, opts, echo, image, ws, ws_bytes, ev, stream, true, true,
                                "reconstruct_hybrid_events");
}

int reconstruct_hybrid(const pl_geometry* g, const pl_image_grid* grid, const pl_hybrid_opts* opts, const float* echo,
                       float* image, void* ws, size_t ws_bytes, hipStream_t stream) {
    return pl::reconstruct_impl(g, grid, opts, echo, image, ws, ws_bytes, nullptr, stream, true, true,
                                "reconstruct_hybrid");
}

int hybrid_prepare(const pl_geometry* g, const pl_image_grid* grid, const pl_hybrid_opts* opts, void* ws,
                   size_t ws_bytes, hipStream_t stream) {
    using namespace pl;
    clear_error();
    HybridPlan p;
    DeviceTables dt;
    int rc = prepare(g, grid, opts, ws, ws_bytes, &p, &dt, "hybrid_prepare", stream);
    if (rc) return rc;
    return launch_plan_tables(p, dt, static_cast<char*>(ws), stream);
}

int reconstruct_hybrid_prepared(const pl_geometry* g, const pl_image_grid* grid, const pl_hybrid_opts* opts,
                                const float* echo, float* image, void* ws, size_t ws_bytes, hipStream_t stream) {
    return pl::reconstruct_impl(g, grid, opts, echo, image, ws, ws_bytes, nullptr, stream, false, true,
                                "reconstruct_hybrid_prepared");
}

int adjoint_hybrid(const pl_geometry* g, const pl_image_grid* grid, const pl_hybrid_opts* opts, const float* image,
                   float* echo, void* ws, size_t ws_bytes, hipStream_t stream) {
    using namespace pl;
    clear_error();
    if (!image || !echo) return fail(PL_EINVAL, "adjoint_hybrid: null image or echo");
    HybridPlan p;
    DeviceTables dt;
    int rc = prepare(g, grid, opts, ws, ws_bytes, &p, &dt, "adjoint_hybrid", stream);
    if (rc) return rc;
    if (p.precision != PL_PREC_FP32 || !p.bp_gather)
        return fail(PL_EUNSUPPORTED, "adjoint_hybrid: needs the FP32 plan with the pixel-per-lane back-projection");
    if (p.range_method != PL_RANGE_NUFFT)
        return fail(PL_EUNSUPPORTED, "adjoint_hybrid: the adjoint is of the NUFFT range compression");
    char* w = static_cast<char*>(ws);
    float2* St = reinterpret_cast<float2*>(w + p.off_spec);
    float2* qt = reinterpret_cast<float2*>(w + p.off_q);
    float2* Gt = reinterpret_cast<float2*>(w + p.off_G);
    const char* ztab = w + p.off_zfft;
    if ((rc = launch_plan_tables(p, dt, w, stream))) return rc;
    if ((rc = launch_kz_fft_adjoint(p, reinterpret_cast<const float2*>(image), Gt, ztab, stream))) return rc;
    if ((rc = launch_backproject_adjoint(p, dt, Gt, w, qt, stream))) return rc;  // writes every element of q~
    if ((rc = launch_range_adjoint(p, qt, w, St, stream))) return rc;
    return launch_scan_fft_adjoint(g, St, reinterpret_cast<float2*>(echo), p.zfft, ztab, stream);
}

int bp_workspace_bytes(const pl_geometry* g, const pl_image_grid* grid, int32_t nz, size_t* bytes) {
    pl::clear_error();
    if (!g || !grid || !bytes) return pl::fail(PL_EINVAL, "bp_workspace_bytes: null pointer");
    if (grid->nx < 1 || grid->ny < 1 || nz < 1 || nz > g->n_scan)
        return pl::fail(PL_EINVAL, "bp_workspace_bytes: bad grid or plane count");
    *bytes = pl::bp_layout(g, grid, nz).bytes;
    return PL_OK;
}

int reconstruct_bp(const pl_geometry* g, const pl_image_grid* grid, int32_t iz0, int32_t nz, const float* echo,
                   float* image, void* ws, size_t ws_bytes, hipStream_t stream) {
    using namespace pl;
    clear_error();
    if (!g || !grid || !echo || !image) return fail(PL_EINVAL, "reconstruct_bp: null pointer");
    if (grid->nx < 1 || grid->ny < 1 || !(grid->dx > 0) || !(grid->dy > 0))
        return fail(PL_EINVAL, "reconstruct_bp: bad grid");
    if (iz0 < 0 || nz < 1 || iz0 + nz > g->n_scan)
        return fail(PL_EINVAL, "reconstruct_bp: planes [%d, %d) outside [0, %d)", iz0, iz0 + nz, g->n_scan);
    const size_t need = bp_layout(g, grid, nz).bytes;
    if (!ws || ws_bytes < need) return fail(PL_EWORKSPACE, "reconstruct_bp: workspace of %zu bytes, %zu needed", ws_bytes, need);
    if ((reinterpret_cast<uintptr_t>(ws) & 255u) != 0)
        return fail(PL_EWORKSPACE, "reconstruct_bp: workspace must be 256-byte aligned");
    DeviceTables dt;
    int rc = g->device_tables(&dt, stream);
    if (rc) return rc;
    return launch_bp(g, dt, grid, iz0, nz, reinterpret_cast<const float2*>(echo), static_cast<char*>(ws),
                     reinterpret_cast<float2*>(image), stream);
}

}  // extern "C"
