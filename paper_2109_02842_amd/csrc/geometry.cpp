// Polyline array geometry (Sec. II-A/B), error reporting and small host
// utilities of the polyrecon library.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "internal.hpp"

namespace pl {

static thread_local char g_last_error[512] = "";

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { g_last_error[0] = '\0'; }

int check_launch(const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(PL_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    return PL_OK;
}

bool factor_radices(int n, Radices* out) {
    Radices r;
    r.n = n;
    int m = n;
    const int order[5] = {8, 4, 2, 3, 5};
    for (int i = 0; i < 5; ++i) {
        while (m % order[i] == 0) {
            if (r.count >= kMaxRadices) return false;
            r.r[r.count++] = order[i];
            m /= order[i];
        }
    }
    if (m != 1 || n < 1) return false;
    *out = r;
    return true;
}

bool is_fft_friendly(int n) {
    Radices r;
    return factor_radices(n, &r);
}

int plan_axis_fft(int n, AxisFft* out) {
    if (n < 1 || n > kMaxScan) return fail(PL_EINVAL, "transform length %d outside [1, %d]", n, kMaxScan);
    AxisFft f;
    f.n = n;
    if (factor_radices(n, &f.rad)) {
        f.m = n;
    } else {
        // any smooth m >= 2n - 1 serves.  From n = 64 on, the smallest m =
        // 64 R (R 2,3,5-smooth, at most 32): the wavefront chirp-z kernel's
        // sizes.  Otherwise the workgroup kernel, each of whose radix stages
        // is one pass through LDS with a barrier: the m with the least m x
        // stages among those up to twice the smallest.
        int best = 0;
        long long best_cost = 0;
        Radices r;
        if (n >= 64)
            for (int rr = (2 * n - 1 + 63) / 64; rr <= 32 && !best; ++rr)
                if (is_fft_friendly(rr)) best = 64 * rr;
        const bool wave = best != 0;
        for (int m = 2 * n - 1; !wave && m <= std::min(kMaxChirpLen, 2 * (2 * n - 1)); ++m) {
            if (!factor_radices(m, &r)) continue;
            const long long cost = static_cast<long long>(m) * r.count;
            if (!best || cost < best_cost) {
                best = m;
                best_cost = cost;
            }
        }
        if (!best) return fail(PL_EUNSUPPORTED, "transform length %d needs a chirp-z length over %d", n, kMaxChirpLen);
        factor_radices(best, &f.rad);
        f.m = best;
        f.chirp = true;
    }
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = (off + bytes + 255) & ~static_cast<size_t>(255);
        return o;
    };
    f.off_tw = take(8ull * f.m);
    if (f.chirp) {
        f.off_chirp = take(8ull * f.n);
        f.off_pad = take(8ull * f.m);
        f.off_hat = take(8ull * f.m);
    }
    f.bytes = off;
    *out = f;
    return PL_OK;
}

}  // namespace pl

int pl_geometry::device_tables(pl::DeviceTables* out, hipStream_t stream, bool upload) const {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return pl::fail(PL_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    std::lock_guard<std::mutex> lock(mu);
    auto it = this->dev.find(dev);
    if (it != this->dev.end()) {
        *out = it->second;
        return PL_OK;
    }
    if (!upload)
        return pl::fail(PL_EINVAL, "the geometry's tables are not on device %d (geometry_upload first)", dev);
    pl::DeviceTables t;
    e = hipMalloc(&t.chan, chan.size() * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&t.k, k.size() * sizeof(double));
    if (e == hipSuccess)
        e = hipMemcpyAsync(t.chan, chan.data(), chan.size() * sizeof(double), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(t.k, k.data(), k.size() * sizeof(double), hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) {
        if (t.chan) (void)hipFree(t.chan);
        if (t.k) (void)hipFree(t.k);
        return pl::fail(PL_EDEVICE, "uploading geometry tables: %s", hipGetErrorString(e));
    }
    this->dev[dev] = t;
    *out = t;
    return PL_OK;
}

pl_geometry::~pl_geometry() {
    int cur = 0;
    const bool have = hipGetDevice(&cur) == hipSuccess;
    for (auto& kv : dev) {
        if (hipSetDevice(kv.first) != hipSuccess) continue;
        (void)hipFree(kv.second.chan);
        (void)hipFree(kv.second.k);
    }
    if (have) (void)hipSetDevice(cur);
}

extern "C" {

const char* last_error(void) { return pl::g_last_error; }

int make_geometry(const pl_geometry_desc* d, pl_geometry** out) {
    using namespace pl;
    clear_error();
    if (!d || !out) return fail(PL_EINVAL, "make_geometry: null pointer");
    if (d->mode != PL_MONO && d->mode != PL_MULTI) return fail(PL_EINVAL, "make_geometry: bad mode %d", d->mode);
    if (d->n_chords < 1 || d->n_elem < 1) return fail(PL_EINVAL, "make_geometry: n_chords and n_elem must be >= 1");
    if (!(d->radius_m > 0) || !(d->spacing_m > 0) || !std::isfinite(d->arc_center_rad))
        return fail(PL_EINVAL, "make_geometry: radius and spacing must be positive");
    if (d->n_scan < 1 || d->n_scan > kMaxScan) return fail(PL_EINVAL, "make_geometry: n_scan must be in [1, %d]", kMaxScan);
    if (d->n_freq < 1 || d->n_freq > kMaxFreq) return fail(PL_EINVAL, "make_geometry: n_freq must be in [1, %d]", kMaxFreq);
    if (!(d->scan_step_m > 0) || !std::isfinite(d->scan_z0_m)) return fail(PL_EINVAL, "make_geometry: scan step must be positive");
    if (!(d->f_start_hz > 0) || !(d->f_stop_hz >= d->f_start_hz) || (d->n_freq > 1 && !(d->f_stop_hz > d->f_start_hz)))
        return fail(PL_EINVAL, "make_geometry: need 0 < f_start < f_stop");
    const double L = d->n_elem * d->spacing_m;
    if (!(L < 2.0 * d->radius_m))
        return fail(PL_EGEOM, "make_geometry: chord length %.6g m is not below the diameter %.6g m", L, 2.0 * d->radius_m);

    std::vector<double> tx_off;
    if (d->mode == PL_MULTI) {
        if (d->n_tx < 1) return fail(PL_EINVAL, "make_geometry: multistatic arrays need n_tx >= 1");
        if (d->tx_offsets_m) {
            tx_off.assign(d->tx_offsets_m, d->tx_offsets_m + d->n_tx);
            for (double u : tx_off)
                if (!std::isfinite(u)) return fail(PL_EINVAL, "make_geometry: non-finite tx offset");
        } else if (d->n_tx == 4) {
            tx_off = {-L / 2, -L / 2 + d->spacing_m / 2, L / 2 - d->spacing_m / 2, L / 2};
        } else if (d->n_tx == 2) {
            tx_off = {-L / 2, L / 2};
        } else {
            return fail(PL_EINVAL, "make_geometry: default Tx placement needs n_tx = 2 or 4");
        }
    }

    pl_geometry* g = new (std::nothrow) pl_geometry();
    if (!g) return fail(PL_EINVAL, "make_geometry: out of host memory");
    g->mode = d->mode;
    g->n_chords = d->n_chords;
    g->n_elem = d->n_elem;
    g->n_tx = d->mode == PL_MULTI ? d->n_tx : 0;
    g->n_scan = d->n_scan;
    g->n_freq = d->n_freq;
    g->radius = d->radius_m;
    g->arc_center = d->arc_center_rad;
    g->spacing = d->spacing_m;
    g->scan_step = d->scan_step_m;
    g->scan_z0 = d->scan_z0_m;
    g->f_start = d->f_start_hz;
    g->f_stop = d->f_stop_hz;
    g->tx_off = tx_off;

    const double alpha = 2.0 * std::asin(L / (2.0 * d->radius_m));
    const int nc = d->n_chords, ne = d->n_elem;
    std::vector<double> elem(static_cast<size_t>(nc) * ne * 2), txe(static_cast<size_t>(nc) * tx_off.size() * 2);
    g->ends.resize(static_cast<size_t>(nc) * 4);
    for (int i = 0; i < nc; ++i) {
        const double phi = d->arc_center_rad + (i - (nc - 1) / 2.0) * alpha;
        const double ax = d->radius_m * std::cos(phi - alpha / 2), ay = d->radius_m * std::sin(phi - alpha / 2);
        const double bx = d->radius_m * std::cos(phi + alpha / 2), by = d->radius_m * std::sin(phi + alpha / 2);
        g->ends[4 * i + 0] = ax;
        g->ends[4 * i + 1] = ay;
        g->ends[4 * i + 2] = bx;
        g->ends[4 * i + 3] = by;
        const double mx = 0.5 * (ax + bx), my = 0.5 * (ay + by);
        const double len = std::hypot(bx - ax, by - ay);
        const double tx = (bx - ax) / len, ty = (by - ay) / len;
        for (int j = 0; j < ne; ++j) {
            const double u = (j + 0.5) * d->spacing_m - L / 2;
            elem[2 * (static_cast<size_t>(i) * ne + j)] = mx + u * tx;
            elem[2 * (static_cast<size_t>(i) * ne + j) + 1] = my + u * ty;
        }
        for (size_t j = 0; j < tx_off.size(); ++j) {
            txe[2 * (i * tx_off.size() + j)] = mx + tx_off[j] * tx;
            txe[2 * (i * tx_off.size() + j) + 1] = my + tx_off[j] * ty;
        }
    }
    if (d->mode == PL_MONO) {
        g->n_ch = nc * ne;
        g->tx = elem;
        g->rx = elem;
    } else {
        const int nt = static_cast<int>(tx_off.size());
        g->n_ch = nc * nt * ne;
        g->tx.resize(static_cast<size_t>(g->n_ch) * 2);
        g->rx.resize(static_cast<size_t>(g->n_ch) * 2);
        for (int i = 0; i < nc; ++i)
            for (int t = 0; t < nt; ++t)
                for (int r = 0; r < ne; ++r) {
                    const size_t c = (static_cast<size_t>(i) * nt + t) * ne + r;
                    g->tx[2 * c] = txe[2 * (static_cast<size_t>(i) * nt + t)];
                    g->tx[2 * c + 1] = txe[2 * (static_cast<size_t>(i) * nt + t) + 1];
                    g->rx[2 * c] = elem[2 * (static_cast<size_t>(i) * ne + r)];
                    g->rx[2 * c + 1] = elem[2 * (static_cast<size_t>(i) * ne + r) + 1];
                }
    }
    g->z.resize(d->n_scan);
    for (int m = 0; m < d->n_scan; ++m) g->z[m] = d->scan_z0_m + m * d->scan_step_m;
    g->f.resize(d->n_freq);
    g->k.resize(d->n_freq);
    const double df = d->n_freq > 1 ? (d->f_stop_hz - d->f_start_hz) / (d->n_freq - 1) : 0.0;
    for (int i = 0; i < d->n_freq; ++i) {
        g->f[i] = (i == d->n_freq - 1 && d->n_freq > 1) ? d->f_stop_hz : d->f_start_hz + i * df;
        g->k[i] = 2.0 * kPi * g->f[i] / kSpeedOfLight;
    }
    g->chan.resize(static_cast<size_t>(g->n_ch) * 4);
    for (int c = 0; c < g->n_ch; ++c) {
        g->chan[4 * c + 0] = g->tx[2 * c];
        g->chan[4 * c + 1] = g->tx[2 * c + 1];
        g->chan[4 * c + 2] = g->rx[2 * c];
        g->chan[4 * c + 3] = g->rx[2 * c + 1];
    }
    *out = g;
    return PL_OK;
}

int geometry_upload(const pl_geometry* g, hipStream_t stream) {
    pl::clear_error();
    if (!g) return pl::fail(PL_EINVAL, "geometry_upload: null geometry");
    pl::DeviceTables dt;
    return g->device_tables(&dt, stream, true);
}

int destroy_geometry(pl_geometry* g) {
    pl::clear_error();
    delete g;
    return PL_OK;
}

int geometry_info(const pl_geometry* g, pl_geometry_info* info, double* tx_xy, double* rx_xy,
                  double* z_scan, double* freq, double* chord_ends) {
    pl::clear_error();
    if (!g) return pl::fail(PL_EINVAL, "geometry_info: null geometry");
    if (info) {
        info->mode = g->mode;
        info->n_chords = g->n_chords;
        info->n_channels = g->n_ch;
        info->n_scan = g->n_scan;
        info->n_freq = g->n_freq;
        info->n_tx = g->n_tx;
        info->n_elem = g->n_elem;
        info->reserved = 0;
    }
    if (tx_xy) std::memcpy(tx_xy, g->tx.data(), g->tx.size() * sizeof(double));
    if (rx_xy) std::memcpy(rx_xy, g->rx.data(), g->rx.size() * sizeof(double));
    if (z_scan) std::memcpy(z_scan, g->z.data(), g->z.size() * sizeof(double));
    if (freq) std::memcpy(freq, g->f.data(), g->f.size() * sizeof(double));
    if (chord_ends) std::memcpy(chord_ends, g->ends.data(), g->ends.size() * sizeof(double));
    return PL_OK;
}

int check_sampling(const pl_geometry* g, const pl_image_grid* grid, uint32_t* warnings) {
    using namespace pl;
    clear_error();
    if (!g || !grid || !warnings) return fail(PL_EINVAL, "check_sampling: null pointer");
    if (grid->nx < 1 || grid->ny < 1 || !(grid->dx > 0) || !(grid->dy > 0))
        return fail(PL_EINVAL, "check_sampling: bad grid");
    uint32_t w = 0;
    const double lam_min = kSpeedOfLight / g->f_stop;
    const double cx = grid->x0 + 0.5 * (grid->nx - 1) * grid->dx;
    const double cy = grid->y0 + 0.5 * (grid->ny - 1) * grid->dy;
    const double D = std::hypot(grid->nx * grid->dx, grid->ny * grid->dy);
    // middle section: distance from its midpoint to the grid centre
    const int mid = g->n_chords / 2;
    double mx = 0.5 * (g->ends[4 * mid] + g->ends[4 * mid + 2]);
    double my = 0.5 * (g->ends[4 * mid + 1] + g->ends[4 * mid + 3]);
    if (g->n_chords % 2 == 0) {  // even count: the middle is the central joint
        mx = g->ends[4 * mid];
        my = g->ends[4 * mid + 1];
    }
    const double R0 = std::hypot(mx - cx, my - cy);
    const double LR = g->n_elem * g->spacing;
    double dmax = lam_min * std::sqrt((LR + D) * (LR + D) / 4 + R0 * R0) / (LR + D);  // (21)
    if (g->mode == PL_MONO) dmax *= 0.5;
    if (g->spacing > dmax * (1 + 1e-12)) w |= PL_WARN_ELEMENT_SPACING;
    const double half_scan = 0.5 * g->n_scan * g->scan_step;
    const double theta_z = 2.0 * std::atan(half_scan / R0);
    const double zmax = lam_min / (4.0 * std::sin(theta_z / 2));  // (22)
    if (g->scan_step > zmax * (1 + 1e-12)) w |= PL_WARN_SCAN_STEP;
    *warnings = w;
    return PL_OK;
}

}  // extern "C"
